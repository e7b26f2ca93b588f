"""GPU: inside an optimisation step the adjoint takes the exit roots of point-source rays (exact root, flat
entry face) from the forward of the same step instead of searching again.  These tests check that such steps
agree with the separate forward / loss / adjoint calls, whose adjoint searches, and that the per-design root
slots of a batched plan line up (collimated designs interleaved with point and emitter-grid designs)."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2302_12031_amd import ffrt
from paper_2302_12031_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _step_vs_calls(wl):
    """dL/dP of one step against forward + loss + adjoint on the same P."""
    plan = ffrt.Plan(wl.problems)
    P0 = plan.pack_cp(wl.Pz)
    T = plan.pack_img(wl.targets)
    st = plan.new_state(P0.clone())
    plan.step(st, T)
    irr = plan.forward(P0)
    loss, dLdI = plan.loss(irr, T)
    g = plan.adjoint(P0, dLdI)
    torch.cuda.synchronize()
    return plan, st, loss, g


@pytest.mark.parametrize("name", ["c3", "c4"])
def test_step_with_reused_roots_matches_separate_calls(name):
    # the gradient comparison needs control-point sums over many rays, as in the parity tests' c4m case
    # (256^2 strata per emitter)
    wl = W.c3(512) if name == "c3" else W.c4(256, emitters=3)
    _say(f"[roots] {name}: {wl.num_rays} rays")
    plan, st, loss, g = _step_vs_calls(wl)
    torch.testing.assert_close(st["loss"], loss, rtol=1e-6, atol=0)
    gmax = g.abs().max().item()
    torch.testing.assert_close(st["dLdP"], g, rtol=1e-4, atol=1e-5 * gmax)
    # and the step's gradient against the FP64 oracle, to the parity tolerance
    p = wl.problems[0]
    _, g64, _, _ = O.grad(p, wl.Pz[0], wl.targets[0])
    gs = st["dLdP"].cpu().numpy().reshape(g64.shape)
    e = np.abs(gs - g64).max() / np.abs(g64).max()
    _say(f"[roots] {name}: step gradient vs FP64 oracle {e:.3g} of max |g|")
    assert e <= 1e-3


def test_graph_replay_with_reused_roots_matches_eager_steps():
    wl = W.c3(384)
    plan_e = ffrt.Plan(wl.problems)
    plan_g = ffrt.Plan(wl.problems)
    P0 = plan_e.pack_cp(wl.Pz)
    T = plan_e.pack_img(wl.targets)
    st_e = plan_e.new_state(P0.clone())
    st_g = plan_g.new_state(P0.clone())
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan_g.graph_capture(st_g, T, steps=3)
    torch.cuda.synchronize()
    for k in range(2):
        with torch.cuda.stream(s):
            plan_g.graph_launch()
        s.synchronize()
        for _ in range(3):
            plan_e.step(st_e, T)
        _ = torch.ones(1000, device="cuda").sum().item()  # unrelated eager work between replays
        torch.cuda.synchronize()
        torch.testing.assert_close(st_g["Pz"], st_e["Pz"], rtol=0, atol=2e-6)
        torch.testing.assert_close(st_g["loss"], st_e["loss"], rtol=1e-4, atol=0)
    _say(f"[roots] graph loss after 6 steps {st_g['loss'].item():.6e}")


def test_batched_plan_root_slots_match_separate_plans():
    probs = [
        W.collimated_problem(200, 8, 48, jitter=1, seed=5, R=20.0, z=50.0),
        W.point_problem(301, 12, 64, seed=6),
        W.collimated_problem(150, 10, 40, jitter=0, seed=7, R=20.0, z=50.0),
        W.point_problem(64, 9, 48, seed=8, emitters=3, emit_w=1.0),
        W.point_problem(257, 16, 80, seed=9),
    ]
    Pz = [W.random_heights(p.lens.n_u, p.lens.n_v, 30 + k) for k, p in enumerate(probs)]
    Ts = [W.target_mixture(p, 30 + k, 3, 3) for k, p in enumerate(probs)]
    plan = ffrt.Plan(probs)
    st = plan.new_state(plan.pack_cp(Pz))
    plan.step(st, plan.pack_img(Ts))
    torch.cuda.synchronize()
    g_all = st["dLdP"].cpu().numpy()
    loss_all = st["loss"].cpu().numpy()
    off = plan.cp_offsets
    for d, p in enumerate(probs):
        one = ffrt.Plan([p])
        s1 = one.new_state(one.pack_cp([Pz[d]]))
        one.step(s1, one.pack_img([Ts[d]]))
        torch.cuda.synchronize()
        g1 = s1["dLdP"].cpu().numpy()
        np.testing.assert_allclose(g_all[off[d]:off[d + 1]], g1, rtol=1e-4, atol=1e-5 * np.abs(g1).max())
        np.testing.assert_allclose(loss_all[d], s1["loss"].cpu().numpy()[0], rtol=1e-5)
    _say(f"[roots] batched plan of {len(probs)} designs matches separate plans")
