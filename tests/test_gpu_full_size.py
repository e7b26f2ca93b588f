"""Full-size parity of the two largest workloads, through the C ABI.

The extended source (9 x 9 emitters x 1024^2 strata, 84.9M rays) and the 64-design batch (132M rays) are
compared pixel by pixel with the oracle's irradiance, computed here, and component by component with the
oracle's gradients, which tests/golden/make_gradients.py wrote from the oracle alone (its forward-mode gradient
of these workloads takes tens of minutes of host time).  Each stored gradient carries a hash of the inputs it
belongs to; a mismatch fails the test instead of comparing against a stale file.
"""
import os
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2302_12031_amd import ffrt
from paper_2302_12031_amd import workloads as W
from parity import MAX_MARGINAL, assert_gradient, assert_irradiance, flip_mask, gradient_errors

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
from make_gradients import input_hash, read  # noqa: E402

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _golden(name, wl):
    G = read(os.path.join(HERE, "golden", f"gradients_{name}.txt"))
    assert sorted(G) == list(range(len(wl.problems))), f"{name}: stored designs {sorted(G)[:5]}..."
    for d, (p, Pz, T) in enumerate(zip(wl.problems, wl.Pz, wl.targets)):
        rays, _, sha, g = G[d]
        assert rays == p.num_rays() and sha == input_hash(p, Pz, T), \
            f"{name} design {d}: stored gradient belongs to other inputs; rerun tests/golden/make_gradients.py {name}"
        assert g.size == Pz.size
    return G


def _run(plan, wl):
    Pz = plan.pack_cp(wl.Pz)
    T = plan.pack_img(wl.targets)
    st = plan.new_stats()
    irr = plan.forward(Pz, stats=st)
    loss, dLdI = plan.loss(irr, T)
    g = plan.adjoint(Pz, dLdI)
    torch.cuda.synchronize()
    return Pz, dict(irr=plan.unpack_img(irr.cpu().numpy()), loss=loss.cpu().numpy(),
                    g=plan.unpack_cp(g.cpu().numpy()), stats=plan.decode_stats(st))


def test_extended_source_full_size():
    """Irradiance per pixel, loss and gradient of the 84.9M-ray design.  The end-to-end gradient goes through
    the device's own single-precision image (its dL/dI); the adjoint alone is checked on the oracle's dL/dI
    (a vector-Jacobian product), which isolates it from the image's rounding."""
    wl = W.c4()
    p, Pz64, T64 = wl.problems[0], wl.Pz[0], wl.targets[0]
    G = _golden("c4", wl)
    _say(f"[full] c4: {wl.num_rays} rays (oracle forward ~20 s on 16 cores)")
    plan = ffrt.Plan(wl.problems)
    Pz, out = _run(plan, wl)
    I64, st64 = O.forward(p, Pz64)
    mask, n_flip, n_marg = flip_mask(plan, 0, Pz, p, Pz64, I64.shape, "c4")
    worst, rel = assert_irradiance(out["irr"][0], I64, mask, what="c4")
    s = out["stats"][0]
    assert s["n_traced"] == wl.num_rays
    assert st64["n_marginal"] <= MAX_MARGINAL * st64["n_rays"] + 5
    assert abs(float(s["flux_on_screen"]) - st64["flux_on_screen"]) <= 1e-4 * st64["flux_on_screen"]
    _, L_gold, _, g_gold = G[0]
    assert abs(out["loss"][0] - L_gold) <= 1e-4 * L_gold
    e_end, per_end, n_big = gradient_errors(out["g"][0], g_gold)
    assert e_end <= 1e-3, f"c4 end-to-end gradient error {e_end:.3g}"
    L64, dLdI64 = O.loss(I64, T64)
    assert abs(L64 - L_gold) <= 1e-12 * L_gold
    g_vjp = plan.unpack_cp(plan.adjoint(Pz, plan.pack_img([dLdI64])).cpu().numpy())[0]
    e_vjp = assert_gradient(g_vjp, g_gold, what="c4 adjoint on the oracle's dL/dI")
    _say(f"[full] c4: irr worst err/tol {worst:.3g}, bright rel {rel:.2e}, masked {int(mask.sum())}, "
         f"marginal {st64['n_marginal']} (flipped {n_flip}); gradient end-to-end {e_end:.2e} (per component "
         f"{per_end:.2e} over {n_big}), adjoint on oracle dL/dI {e_vjp:.2e}")


def test_all_64_designs_of_the_batch():
    """Every design of the 64-design batch (uneven nets and ray counts): irradiance per pixel, loss, and the
    gradient (end to end, and the adjoint on the oracle's dL/dI) against the oracle."""
    wl = W.c5()
    G = _golden("c5", wl)
    _say(f"[full] c5: {len(wl.problems)} designs, {wl.num_rays} rays")
    plan = ffrt.Plan(wl.problems)
    Pz, out = _run(plan, wl)
    dLdI64, worst_all, e_end_all, per_end_all = [], 0.0, 0.0, 0.0
    for d, (p, Pz64, T64) in enumerate(zip(wl.problems, wl.Pz, wl.targets)):
        I64, st64 = O.forward(p, Pz64)
        mask, _, _ = flip_mask(plan, d, Pz, p, Pz64, I64.shape, f"c5 design {d}")
        worst, _ = assert_irradiance(out["irr"][d], I64, mask, what=f"c5 design {d}", w_ray=1.0 / p.num_rays())
        assert out["stats"][d]["n_traced"] == p.num_rays()
        assert st64["n_marginal"] <= MAX_MARGINAL * st64["n_rays"] + 5
        _, L_gold, _, g_gold = G[d]
        assert abs(out["loss"][d] - L_gold) <= 1e-4 * L_gold, (d, out["loss"][d], L_gold)
        e_end, per_end, _ = gradient_errors(out["g"][d], g_gold)
        assert e_end <= 1e-3, f"c5 design {d}: end-to-end gradient error {e_end:.3g}"
        worst_all, e_end_all, per_end_all = max(worst_all, worst), max(e_end_all, e_end), max(per_end_all, per_end)
        dLdI64.append(O.loss(I64, T64)[1])
    g_vjp = plan.unpack_cp(plan.adjoint(Pz, plan.pack_img(dLdI64)).cpu().numpy())
    e_vjp = max(assert_gradient(g_vjp[d], G[d][3], what=f"c5 design {d} adjoint on the oracle's dL/dI")
                for d in range(len(wl.problems)))
    _say(f"[full] c5: irr worst err/tol {worst_all:.3g}; gradient end-to-end {e_end_all:.2e} (per component "
         f"{per_end_all:.2e}), adjoint on oracle dL/dI {e_vjp:.2e}")


def test_batch_of_64_designs_200_graph_steps():
    """200 optimisation steps of the 64-design batch replayed from a captured graph (20 steps per graph) equal
    the eager steps bit for bit, and every design's loss falls."""
    wl = W.c5()
    plans = [ffrt.Plan(wl.problems) for _ in range(2)]
    T = plans[0].pack_img(wl.targets)
    st_e, st_g = (pl.new_state(pl.pack_cp(wl.Pz)) for pl in plans)
    plans[0].step(st_e, T)
    loss1 = st_e["loss"].clone()
    plans[1].step(st_g, T)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plans[1].graph_capture(st_g, T, steps=20)
    torch.cuda.synchronize()
    for k in range(10):
        with torch.cuda.stream(s):
            plans[1].graph_launch()
        s.synchronize()
        for _ in range(20):
            plans[0].step(st_e, T)
        torch.cuda.synchronize()
        assert torch.equal(st_g["Pz"], st_e["Pz"]), f"after {20 * (k + 1) + 1} steps"
        assert torch.equal(st_g["loss"], st_e["loss"])
    assert int(st_g["t"][0]) == 201
    drop = (st_e["loss"] / loss1).cpu().numpy()
    assert (drop < 1.0).all(), np.where(drop >= 1.0)[0].tolist()
    _say(f"[full] c5 201 steps: loss ratio to step 1 median {np.median(drop):.3f}, max {drop.max():.3f}")
