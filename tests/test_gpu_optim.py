"""GPU: optimisation step, HIP graph replay, autograd binding, finite differences and device-side
error counters, through the C ABI."""
import sys
from dataclasses import replace

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


def _setup(wl):
    plan = ffrt.Plan(wl.problems)
    st = plan.new_state(plan.pack_cp(wl.Pz))
    return plan, st, plan.pack_img(wl.targets)


def test_adam_matches_torch():
    wl = W.c1()
    plan, st, T = _setup(wl)
    p_ref = st["Pz"].clone().requires_grad_(True)
    opt = torch.optim.Adam([p_ref], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    g = torch.randn(plan.total_cp, device=plan.device)
    for k in range(5):
        gk = g * (k + 1)
        plan.adam(st["Pz"], gk, st["m"], st["v"], st["t"])
        p_ref.grad = gk.clone()
        opt.step()
        torch.cuda.synchronize()
        torch.testing.assert_close(st["Pz"], p_ref.detach(), rtol=1e-6, atol=1e-7)
    assert int(st["t"][0]) == 5


def test_step_equals_forward_loss_adjoint_adam():
    wl = W.c2(256)
    plan, st, T = _setup(wl)
    P0 = st["Pz"].clone()
    plan.step(st, T)
    # the same step from the individual calls
    irr = plan.forward(P0)
    loss, dLdI = plan.loss(irr, T)
    g = plan.adjoint(P0, dLdI)
    m = torch.zeros_like(P0); v = torch.zeros_like(P0); t = torch.zeros(1, dtype=torch.int32, device=P0.device)
    P1 = P0.clone()
    plan.adam(P1, g, m, v, t)
    torch.cuda.synchronize()
    # the gradient is summed in fixed point (order-independent), so the step reproduces its components
    # bit for bit
    assert torch.equal(st["loss"], loss)
    assert torch.equal(st["dLdP"], g)
    assert torch.equal(st["Pz"], P1)


def test_step_with_and_without_written_dLdI_agree():
    """The step forms dL/dI on the fly unless asked to write it; both paths give the same update."""
    wl = W.c3(512)
    plan_a = ffrt.Plan(wl.problems)
    plan_b = ffrt.Plan(wl.problems)
    P0 = plan_a.pack_cp(wl.Pz)
    st_a = plan_a.new_state(P0.clone())
    st_b = plan_b.new_state(P0.clone(), with_dLdI=True)
    T = plan_a.pack_img(wl.targets)
    for _ in range(3):
        plan_a.step(st_a, T)
        plan_b.step(st_b, T)
    torch.cuda.synchronize()
    assert torch.equal(st_a["loss"], st_b["loss"])
    assert torch.equal(st_a["dLdP"], st_b["dLdP"])
    assert torch.equal(st_a["Pz"], st_b["Pz"])
    _, G = plan_b.loss(st_b["irr"], T)
    torch.testing.assert_close(st_b["dLdI"], G, rtol=1e-6, atol=0)
    assert int(st_a["t"][0]) == int(st_b["t"][0]) == 3


@pytest.mark.parametrize("steps_per_graph", [1, 4])
def test_graph_replay_matches_eager_steps(steps_per_graph):
    wl = W.c2(512)
    plan_e, st_e, T = _setup(wl)
    plan_g, st_g, _ = _setup(wl)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan_g.graph_capture(st_g, T, steps=steps_per_graph)
    torch.cuda.synchronize()
    n_launch = 3
    for k in range(n_launch):
        with torch.cuda.stream(s):
            plan_g.graph_launch()
        s.synchronize()
        for _ in range(steps_per_graph):
            plan_e.step(st_e, T)
        _ = torch.ones(1000, device="cuda").sum().item()      # unrelated eager work between replays
        torch.cuda.synchronize()
        # images and gradients are summed in fixed point: replays reproduce the eager steps bit for bit
        assert torch.equal(st_g["Pz"], st_e["Pz"])
        assert torch.equal(st_g["loss"], st_e["loss"])
        assert int(st_g["t"][0]) == (k + 1) * steps_per_graph
    _say(f"[graph] loss after {n_launch * steps_per_graph} steps {st_g['loss'].item():.6e}")


def test_optimisation_decreases_loss():
    wl = W.c2(256)
    plan, st, T = _setup(wl)
    losses = []
    for _ in range(60):
        plan.step(st, T, hp=ffrt.AdamHP(lr=2e-3))
        losses.append(st["loss"].item())
    assert losses[-1] < 0.7 * losses[0], (losses[0], losses[-1])


def test_autograd_function_backward_is_the_adjoint():
    wl = W.c5(3, ray_scale=1 / 16)
    plan = ffrt.Plan(wl.problems)
    Pz = plan.pack_cp(wl.Pz).requires_grad_(True)
    T = plan.pack_img(wl.targets)
    loss = ffrt.TraceLoss.apply(Pz, T, plan)
    w = torch.tensor([1.0, 2.0, -0.5], device=Pz.device)
    (loss * w).sum().backward()
    irr = plan.forward(Pz.detach())
    _, dLdI = plan.loss(irr, T)
    g = plan.adjoint(Pz.detach(), dLdI)
    for d in range(3):
        a, b = plan.cp_offsets[d], plan.cp_offsets[d + 1]
        torch.testing.assert_close(Pz.grad[a:b], w[d] * g[a:b], rtol=1e-4, atol=1e-6 * g[a:b].abs().max().item())


def test_gradient_matches_oracle_central_fd_on_16_control_points():
    """Point source, C3 geometry: GPU adjoint vs FP64 central differences (h = 1e-4 mm) on 16 random CPs."""
    wl = W.c3(1024)
    p, Pz, T = wl.problems[0], wl.Pz[0], wl.targets[0]
    plan, st, Td = _setup(wl)
    irr = plan.forward(st["Pz"])
    loss, dLdI = plan.loss(irr, Td)
    g = plan.adjoint(st["Pz"], dLdI).cpu().numpy().reshape(Pz.shape)
    L64, g64, _, _ = O.grad(p, Pz, T)
    rng = W.rng(2, W.STREAM_FD)
    cps = rng.choice(Pz.size, 16, replace=False)
    _, st0 = O.forward(p, Pz)
    keys = ("n_hit", "n_side_wall", "n_tir", "n_off_screen")
    errs, flips = [], 0

    def fd_at(k, h):
        E = np.zeros(Pz.size); E[k] = h
        E = E.reshape(Pz.shape)
        Ip, sp = O.forward(p, Pz + E)
        Im, sm = O.forward(p, Pz - E)
        flipped = any(sp[c] != st0[c] or sm[c] != st0[c] for c in keys)
        return (O.loss(Ip, T)[0] - O.loss(Im, T)[0]) / (2 * h), flipped

    for k in cps:
        fd, flipped = fd_at(k, 1e-4)
        if flipped:
            # a ray changes its discrete state within +-h: the difference quotient is not the pathwise
            # derivative there; use a step 100x smaller instead
            flips += 1
            fd, _ = fd_at(k, 1e-6)
        errs.append(abs(fd - g.flat[k]) / np.abs(g64).max())
    _say(f"[fd] max |fd - adjoint| / max|g| = {max(errs):.3e} ({flips} of 16 CPs re-checked at h = 1e-6)")
    assert max(errs) <= 1e-3


def test_device_error_counters_and_noflux_skip():
    wl = W.c1()
    p = wl.problems[0]
    Pz = wl.Pz[0].copy()
    Pz[2, 3] = -0.5            # below the entry face z_in = 0 (sec. 2.1.2)
    Pz[4, 4] = np.nan
    plan = ffrt.Plan([p])
    stats = plan.new_stats()
    plan.forward(plan.pack_cp([Pz]), stats=stats)
    s = plan.decode_stats(stats)[0]
    assert s["n_constraint_viol"] == 2 and s["n_nan"] == 1
    # a screen that no ray reaches: loss is NaN, dL/dI zero and the Adam update is skipped
    far = replace(p, detector=replace(p.detector, R_x=0.01, R_y=0.01))
    plan2 = ffrt.Plan([far])
    st = plan2.new_state(plan2.pack_cp([wl.Pz[0]]))
    P0 = st["Pz"].clone()
    T = plan2.pack_img([np.ones(far.image_shape())])
    plan2.step(st, T)
    torch.cuda.synchronize()
    assert torch.isnan(st["loss"]).all()
    assert int(st["t"][0]) == 0
    torch.testing.assert_close(st["Pz"], P0, rtol=0, atol=0)
    s2 = plan2.decode_stats(st["stats"])[0]
    assert s2["n_hit"] == 0 and s2["n_off_screen"] == p.num_rays()


def test_kernel_timing_call():
    wl = W.c2(512)
    plan, st, T = _setup(wl)
    irr = plan.forward(st["Pz"])
    _, dLdI = plan.loss(irr, T)
    f, a = plan.time_kernels(st["Pz"], torch.empty_like(irr), dLdI, torch.empty_like(st["dLdP"]), reps=5)
    assert 0 < f < 1e3 and 0 < a < 1e3


def test_autotune_picks_a_valid_shape_and_keeps_parity():
    wl = W.c3(1024)
    plan, st, T = _setup(wl)
    irr = plan.forward(st["Pz"])
    _, dLdI = plan.loss(irr, T)
    f, a = plan.autotune(st["Pz"], irr, dLdI, st["dLdP"], reps=2)
    assert 0 <= f < len(ffrt.Plan.config_names(0)) and 0 <= a < len(ffrt.Plan.config_names(1))
    irr2 = plan.forward(st["Pz"])
    torch.testing.assert_close(irr2, irr, rtol=1e-5, atol=1e-6 * irr.max().item())


def test_trace_rays_edge_cases():
    wl = W.c1()
    plan = ffrt.Plan(wl.problems)
    Pz = plan.pack_cp(wl.Pz)
    assert plan.trace_rays(0, Pz, np.zeros(0, np.int64)).shape == (0, 8)
    n = wl.num_rays
    ids = np.array([0, n - 1, n // 2])
    out = plan.trace_rays(0, Pz, ids).cpu().numpy()
    ref = O.trace_rays(wl.problems[0], wl.Pz[0], ids)
    np.testing.assert_allclose(out[:, 1:3], ref[:, 1:3], atol=1e-4)
    with pytest.raises(ffrt.FfrtError):
        plan.trace_rays(3, Pz, ids)


def test_ragged_grids_and_ghost_pixels():
    """Sample grids that do not fill whole blocks, ghost pixels and the (5,3) and nu = 11 kernels."""
    cases = [
        W.collimated_problem(333, 11, 40, jitter=1, seed=9, R=15.0, z=30.0),
        replace(W.point_problem(301, 9, 48, seed=9, R=60.0), detector=replace(
            W.point_problem(301, 9, 48).detector, R_x=60.0, R_y=60.0, ghost=1)),
    ]
    p53 = W.collimated_problem(200, 10, 32, jitter=1, seed=4, R=15.0, z=30.0)
    cases.append(replace(p53, lens=replace(p53.lens, p=5, q=3)))
    p11 = W.collimated_problem(200, 10, 32, jitter=1, seed=4, R=15.0, z=30.0)
    cases.append(replace(p11, detector=replace(p11.detector, nu_x=11, nu_y=11)))
    from parity import assert_gradient, assert_irradiance, flip_mask
    for k, p in enumerate(cases):
        Pz = W.random_heights(p.lens.n_u, p.lens.n_v, 20 + k)
        T = W.target_mixture(p, 20 + k, 3, 3)
        plan = ffrt.Plan([p])
        Pd, Td = plan.pack_cp([Pz]), plan.pack_img([T])
        irr = plan.forward(Pd)
        _, dLdI = plan.loss(irr, Td)
        g = plan.adjoint(Pd, dLdI).cpu().numpy().reshape(Pz.shape)
        I = irr.cpu().numpy().reshape(p.image_shape())
        I64, _ = O.forward(p, Pz)
        mask, _, _ = flip_mask(plan, 0, Pd, p, Pz, I64.shape, f"case {k}")
        assert_irradiance(I, I64, mask, what=f"case {k}")
        L64, g64, _, _ = O.grad(p, Pz, T)
        assert_gradient(g, g64, what=f"case {k}")


@pytest.mark.parametrize("name", ["c2", "c3", "c5-subset"])
def test_gradient_is_reproducible_bit_for_bit(name):
    """The adjoint sums its contributions in 64-bit fixed point: repeated calls on the same inputs give the same
    dL/dP bit for bit, whatever order the workgroups' atomics arrive in."""
    if name == "c5-subset":
        full = W.c5()
        sel = [0, 1, 2, 3, 5, 8]
        wl = W.Workload("c5 subset", [full.problems[i] for i in sel], [full.Pz[i] for i in sel],
                        [full.targets[i] for i in sel])
    else:
        wl = {"c2": W.c2, "c3": W.c3}[name]()
    plan = ffrt.Plan(wl.problems)
    P = plan.pack_cp(wl.Pz)
    _, G = plan.loss(plan.forward(P), plan.pack_img(wl.targets))
    g1 = plan.adjoint(P, G)
    g2 = plan.adjoint(P, G)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)
    assert g1.abs().max().item() > 0


def test_lds_atomic_rate_microbenchmark():
    """ffrt_lds_atomic_rate: a positive chip-wide rate for both access patterns; the splat's pattern (shared
    banks and addresses) cannot beat distinct banks by more than timing noise."""
    peak = ffrt.lds_atomic_rate(0, reps=5)
    splat = ffrt.lds_atomic_rate(1, reps=5)
    _say(f"[lds] atomics/s: distinct banks {peak:.3e}, splat pattern {splat:.3e}")
    assert peak > 1e11 and splat > 1e10
    assert splat <= 1.1 * peak
    with pytest.raises(ffrt.FfrtError):
        ffrt.lds_atomic_rate(2)
