"""GPU: lenses with both faces freeform (the entry face a second B-spline whose net follows the exit net),
through the C ABI, against the oracle: irradiance per pixel, the gradient over both nets, per-ray hits at full
size, the reduction to the plano-freeform lens, and optimisation steps."""
import sys
from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle as O
from paper_2302_12031_amd import ffrt
from paper_2302_12031_amd import workloads as W
from parity import MAX_MARGINAL, assert_gradient, assert_irradiance, flip_mask, gradient_errors

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(wl):
    plan = ffrt.Plan(wl.problems)
    Pz = plan.pack_cp(wl.Pz)
    T = plan.pack_img(wl.targets)
    st = plan.new_stats()
    irr = plan.forward(Pz, stats=st)
    loss, dLdI = plan.loss(irr, T)
    g = plan.adjoint(Pz, dLdI)
    torch.cuda.synchronize()
    return plan, dict(irr=plan.unpack_img(irr.cpu().numpy()), loss=loss.cpu().numpy(),
                      g=plan.unpack_cp(g.cpu().numpy()), stats=plan.decode_stats(st))


# (workload, per-pixel irradiance at this size and its relative tolerance, gradient compared)
CASES = {
    "c1": (lambda: W.with_entry_freeform(W.c1()), 1e-4, True),
    "c2": (lambda: W.with_entry_freeform(W.c2()), 1e-4, True),
    "c3": (lambda: W.with_entry_freeform(W.c3()), 1e-4, False),
    "c3s": (lambda: W.with_entry_freeform(W.c3(512)), None, True),
}


@pytest.mark.parametrize("name", list(CASES))
def test_two_face_forward_and_gradient_parity(name):
    make, irr_rel, grad = CASES[name]
    wl = make()
    _say(f"[two faces] {name}: {wl.name}, {wl.num_rays} rays")
    plan, out = _run(wl)
    p, Pz, T = wl.problems[0], wl.Pz[0], wl.targets[0]
    I64, st64 = O.forward(p, Pz)
    mask, _, _ = flip_mask(plan, 0, plan.pack_cp(wl.Pz), p, Pz, I64.shape, name)
    worst, rel, eg = float("nan"), float("nan"), float("nan")
    if irr_rel is not None:
        worst, rel = assert_irradiance(out["irr"][0], I64, mask, what=name, rel=irr_rel)
    s = out["stats"][0]
    assert s["n_traced"] == st64["n_rays"]
    assert st64["n_marginal"] <= MAX_MARGINAL * st64["n_rays"] + 5
    assert abs(int(s["n_hit"]) - st64["n_hit"]) <= st64["n_marginal"] + 2
    assert abs(float(s["flux_on_screen"]) - st64["flux_on_screen"]) <= 1e-4 * st64["flux_on_screen"]
    assert int(s["n_constraint_viol"]) == 0
    if grad:
        L64, g64, _, _ = O.grad(p, Pz, T)
        assert abs(out["loss"][0] - L64) <= 1e-4 * L64
        # global and per-component bars; rays at a kink of their derivative are re-traced in double precision
        # through both faces
        eg = assert_gradient(out["g"][0], g64, what=name)
        _, per, nbig = gradient_errors(out["g"][0], g64)
        _say(f"[two faces] {name}: per-component error {per:.3g} over {nbig} components")
        # both nets carry gradient, each within the tolerance of its own scale
        for f in range(2):
            assert np.abs(g64[f]).max() > 0
            assert np.abs(out["g"][0][f] - g64[f]).max() <= 2e-3 * np.abs(g64[f]).max(), f
    _say(f"[two faces] {name}: irr worst err/tol {worst:.3g}, bright rel {rel:.2e}, grad rel {eg:.2e}, "
         f"hits {int(s['n_hit'])}")


def test_flat_entry_net_matches_the_plano_freeform_lens():
    """An entry net at z_in reproduces the plano-freeform lens: per pixel, both plans' irradiance against the
    oracle's (which gives the two lenses the same image), and the exit-net gradient of the two-face plan against
    the plano plan's.  The two paths round differently (a plane hit against a root search on a flat net)."""
    for base in (W.c1(), W.c3()):
        two = W.with_entry_freeform(base, base=0.0, spread=0.0)
        plan_a, a = _run(base)
        plan_b, b = _run(two)
        I64, _ = O.forward(base.problems[0], base.Pz[0])
        for plan, wl, out, tag in ((plan_a, base, a, "plano"), (plan_b, two, b, "flat entry net")):
            mask, _, _ = flip_mask(plan, 0, plan.pack_cp(wl.Pz), wl.problems[0], wl.Pz[0], I64.shape, tag)
            assert_irradiance(out["irr"][0], I64, mask, what=f"{base.name} {tag}")
        # both plans re-trace their kink rays in double precision, but the flat entry net's root search and the
        # plane hit round differently: the global bar
        assert_gradient(b["g"][0][0], a["g"][0], what=base.name, per_component=False)


def test_two_face_per_ray_parity_full_size():
    wl = W.with_entry_freeform(W.c3())
    p, Pz = wl.problems[0], wl.Pz[0]
    plan = ffrt.Plan(wl.problems)
    ids = np.unique(np.random.default_rng(3).integers(0, wl.num_rays, 4096))
    gpu = plan.trace_rays(0, plan.pack_cp([Pz]), ids).cpu().numpy()
    ref = O.trace_rays(p, Pz, ids)
    clear = ref[:, 7] == 0
    assert (gpu[clear, 0] == ref[clear, 0]).sum() >= clear.sum() - 2
    hit = clear & (ref[:, 0] == O.HIT) & (gpu[:, 0] == O.HIT)
    scale = p.detector.z_screen * (1.0 + np.abs(ref[hit, 1:3]).max(1, keepdims=True) / p.detector.z_screen)
    dxy = np.abs(gpu[hit, 1:3] - ref[hit, 1:3]) / scale
    assert dxy.max() <= 2e-5, dxy.max()
    assert np.median(dxy) <= 5e-7, np.median(dxy)
    np.testing.assert_allclose(gpu[hit, 3], ref[hit, 3], rtol=2e-5)
    _say(f"[two faces per-ray] {hit.sum()} hits, landing err max {dxy.max():.2e}, median {np.median(dxy):.2e}")


def test_two_face_steps_reduce_the_loss_and_count_thin_spots():
    """Graph-captured Adam steps move both nets and lower the loss; a net pushed through the other is
    reported by the thickness counter."""
    wl = W.with_entry_freeform(W.c1())
    plan = ffrt.Plan(wl.problems)
    st = plan.new_state(plan.pack_cp(wl.Pz))
    T = plan.pack_img(wl.targets)
    P0 = st["Pz"].clone()
    plan.step(st, T, hp=ffrt.AdamHP(lr=1e-3))
    L0 = st["loss"].item()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.graph_capture(st, T, steps=50, hp=ffrt.AdamHP(lr=1e-3))
        plan.graph_launch(s)
    torch.cuda.synchronize()
    L1 = plan.loss(plan.forward(st["Pz"]), T)[0].item()
    _say(f"[two faces steps] loss {L0:.4e} -> {L1:.4e}")
    assert L1 < 0.9 * L0
    K = wl.problems[0].lens.n_u * wl.problems[0].lens.n_v
    moved = (st["Pz"] - P0).abs()
    assert moved[:K].max() > 0 and moved[K:].max() > 0
    bad = P0.clone()
    bad[K + 5] = bad[5] + 0.5                     # entry point above the exit point
    stt = plan.new_stats()
    plan.forward(bad, stats=stt)
    assert int(plan.decode_stats(stt)[0]["n_constraint_viol"]) == 1


def test_plan_with_every_retraced_group_matches_separate_plans():
    """One plan holding a design of every kernel group: plano collimated and point, two-face collimated and
    point, mesh collimated and point.  The groups whose kink rays go to the double-precision re-trace queue them
    in segments of their own, one after another; each design's image, loss and gradient must equal its own
    plan's, the image and gradient bit for bit (both are integer sums)."""
    base = [
        W.collimated_problem(160, 8, 48, jitter=1, seed=21, R=20.0, z=50.0),
        W.point_problem(192, 12, 64, seed=22),
    ]
    probs, Pz, Ts = [], [], []
    for k, p in enumerate(base):
        P = W.random_heights(p.lens.n_u, p.lens.n_v, 40 + k)
        T = W.target_mixture(p, 40 + k, 3, 3)
        two = W.with_entry_freeform(W.Workload("x", [p], [P], [T]))
        mesh = W.with_mesh(W.Workload("x", [p], [P], [T]), 2)
        for wl in (W.Workload("x", [p], [P], [T]), two, mesh):
            probs += wl.problems
            Pz += wl.Pz
            Ts += wl.targets
    plan = ffrt.Plan(probs)
    Pp, Tp = plan.pack_cp(Pz), plan.pack_img(Ts)
    irr = plan.forward(Pp)
    loss, dLdI = plan.loss(irr, Tp)
    g = plan.adjoint(Pp, dLdI)
    torch.cuda.synchronize()
    irr_all, g_all = plan.unpack_img(irr.cpu().numpy()), plan.unpack_cp(g.cpu().numpy())
    loss_all = loss.cpu().numpy()
    for d, p in enumerate(probs):
        one = ffrt.Plan([p])
        P1, T1 = one.pack_cp([Pz[d]]), one.pack_img([Ts[d]])
        i1 = one.forward(P1)
        l1, dl1 = one.loss(i1, T1)
        g1 = one.adjoint(P1, dl1)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(irr_all[d], one.unpack_img(i1.cpu().numpy())[0], err_msg=f"design {d}")
        np.testing.assert_allclose(loss_all[d], l1.cpu().numpy()[0], rtol=1e-6)
        np.testing.assert_array_equal(g_all[d], one.unpack_cp(g1.cpu().numpy())[0], err_msg=f"design {d}")
    _say(f"[two faces] a plan of {len(probs)} designs over every kernel group matches separate plans bit for bit")
