"""GPU: the control-point generators of sec. 2.4 (three control-net-sized tanh layers, dense or locally
connected, and the output correction), through the C ABI, against the oracle; their optimisation step and
graph replay; the zero-initialised generator against the no-network optimisation; the circular top-hat design
loop."""
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


def _dev(a, plan):
    return torch.tensor(np.ascontiguousarray(a).ravel(), dtype=torch.float32, device=plan.device)


ARCHS = [ffrt.MLP_DENSE, ffrt.MLP_SPARSE]


def _wshape(prob, arch):
    L = prob.lens
    K = L.n_u * L.n_v
    return (K, K) if arch == ffrt.MLP_DENSE else ((2 * L.p + 1) * (2 * L.q + 1), K)


def _params(prob, arch, seed, scale=0.5):
    K = prob.lens.n_u * prob.lens.n_v
    ws = _wshape(prob, arch)
    g = W.rng(seed, 20)
    return [g.normal(0, scale, K), g.normal(0, scale, K), g.normal(0, scale / np.sqrt(ws[0]), ws),
            g.normal(0, scale, K), g.normal(0, scale / np.sqrt(ws[0]), ws), g.normal(0, scale, K)]


def _oracle(prob, arch):
    L = prob.lens
    if arch == ffrt.MLP_DENSE:
        return O.mlp_forward, O.mlp_backward
    geo = (L.n_u, L.n_v, L.p, L.q)
    return (lambda prm, lo, span: O.sparse_mlp_forward(prm, lo, span, *geo),
            lambda prm, acts, span, g: O.sparse_mlp_backward(prm, acts, span, g, *geo))


def _batched_plan():
    """Designs of uneven control-net size (K = 16, 49, 256, 529, 1024), so the GEMV rows, the W^T chunks and
    the parameter offsets span several tiles and ragged tails."""
    probs = [W.collimated_problem(32, n, 16, seed=40 + n) for n in (4, 7, 16, 23, 32)]
    return probs, ffrt.Plan(probs)


@pytest.mark.parametrize("arch", ARCHS)
def test_mlp_forward_backward_match_oracle(arch):
    probs, plan = _batched_plan()
    prm = [_params(p, arch, 50 + d) for d, p in enumerate(probs)]
    lo = [W.rng(60 + d, 21).uniform(1.7, 1.9, p.cp_shape()) for d, p in enumerate(probs)]
    span = [W.rng(60 + d, 22).uniform(0.2, 0.6, p.cp_shape()) for d, p in enumerate(probs)]
    g = [W.rng(60 + d, 23).normal(size=p.cp_shape()) for d, p in enumerate(probs)]
    par = plan.pack_mlp(prm, arch)
    lo_d, sp_d, g_d = plan.pack_cp(lo), plan.pack_cp(span), plan.pack_cp(g)
    _say(f"[mlp arch {arch}] K = {[p.lens.n_u * p.lens.n_v for p in probs]}, {par.numel()} parameters")
    acts, P = plan.mlp_forward(par, lo_d, sp_d, arch=arch)
    grad = plan.mlp_backward(par, acts, sp_d, g_d, arch=arch)
    torch.cuda.synchronize()
    P_d = plan.unpack_cp(P.cpu().numpy())
    G_d = plan.unpack_mlp(grad.cpu().numpy(), arch)
    for d, p in enumerate(probs):
        K = p.lens.n_u * p.lens.n_v
        fwd, bwd = _oracle(p, arch)
        a_ref, P_ref = fwd(prm[d], lo[d].ravel(), span[d].ravel())
        np.testing.assert_allclose(P_d[d].ravel(), P_ref, rtol=0, atol=2e-6, err_msg=f"P d={d}")
        a = acts.cpu().numpy()[3 * plan.cp_offsets[d]:3 * plan.cp_offsets[d] + 3 * K].reshape(3, K)
        for k in range(3):
            np.testing.assert_allclose(a[k], a_ref[k], rtol=0, atol=2e-6, err_msg=f"acts {k} d={d}")
        ref = bwd(prm[d], a_ref, span[d].ravel(), g[d].ravel())
        for k, (gg, rr) in enumerate(zip(G_d[d], ref)):
            scale = max(np.abs(rr).max(), 1e-30)
            np.testing.assert_allclose(gg, rr, rtol=0, atol=1e-4 * scale, err_msg=f"grad {k} d={d}")


def _tophat_setup(init, arch):
    wl = W.tophat()
    p = wl.problems[0]
    lo, span = W.tophat_range(p)
    plan = ffrt.Plan(wl.problems)
    K = p.lens.n_u * p.lens.n_v
    shapes = [(K,), (K,), _wshape(p, arch), (K,), _wshape(p, arch), (K,)]
    if init == "zero":
        prm = [np.zeros(s) for s in shapes]
    elif init == "uniform":                 # the paper's small uniform initialisation U([-1e-4, 1e-4])
        g = W.rng(7, 24)
        prm = [g.uniform(-1e-4, 1e-4, s) for s in shapes]
    else:
        prm = _params(p, arch, 8, scale=0.3)
    return wl, p, plan, prm, lo, span


def _linear_hp(plan, st, T, lr):
    """Adam hyper-parameters with eps at the largest first gradient component, for comparisons of steps whose
    parameter gradients differ by rounding (~1e-7 relative): two chain rules (the generator's against the
    reparametrised one), or two runs of the dense generator's back-propagation, whose transposed products add
    float partial sums atomically.  With a tiny eps Adam maps a component near eps to an update anywhere in
    [0, lr], so such comparisons would see that noise, not the computation.  With this eps every update is
    close to linear in its gradient."""
    gP = plan.adjoint(st["Pz"], plan.loss(plan.forward(st["Pz"]), T)[1])
    g = plan.mlp_backward(st["params"], st["acts"], st["span"], gP, arch=st["arch"])
    torch.cuda.synchronize()
    return ffrt.AdamHP(lr=lr, eps=float(g.abs().max()))


def _adam_host(x, g, m, v, t, hp):
    m = hp.beta1 * m + (1 - hp.beta1) * g
    v = hp.beta2 * v + (1 - hp.beta2) * g * g
    step = hp.lr / (1 - hp.beta1 ** t)
    return x - step * m / (np.sqrt(v) / np.sqrt(1 - hp.beta2 ** t) + hp.eps), m, v


@pytest.mark.parametrize("arch", ARCHS)
def test_step_mlp_equals_its_components(arch):
    wl, p, plan, prm, lo, span = _tophat_setup("random", arch)
    T = plan.pack_img(wl.targets)
    par0, lo_d, sp_d = plan.pack_mlp([prm], arch), _dev(lo, plan), _dev(span, plan)
    hp = ffrt.AdamHP(lr=0.01)
    st = plan.new_mlp_state(par0.clone(), lo_d, sp_d, arch=arch)
    plan.step_mlp(st, T, hp=hp)
    # the same step from the individual calls
    acts, P = plan.mlp_forward(par0, lo_d, sp_d, arch=arch)
    irr = plan.forward(P)
    loss, G = plan.loss(irr, T)
    gP = plan.adjoint(P, G)
    gpar = plan.mlp_backward(par0, acts, sp_d, gP, arch=arch)
    torch.cuda.synchronize()
    x1, _, _ = _adam_host(par0.cpu().double().numpy(), gpar.cpu().double().numpy(), 0.0, 0.0, 1, hp)
    # the generator's forward pass has no atomics: the step's closing forward is bit-exact
    acts1, P1 = plan.mlp_forward(st["params"], lo_d, sp_d, arch=arch)
    torch.cuda.synchronize()
    assert torch.equal(st["loss"], loss)
    assert torch.equal(st["dLdP"], gP)          # fixed-point gradient sums: reproducible bit for bit
    np.testing.assert_allclose(st["params"].cpu().numpy(), x1, rtol=0, atol=2e-6)
    assert torch.equal(st["Pz"], P1) and torch.equal(st["acts"], acts1)
    assert int(st["t"][0]) == 1


@pytest.mark.parametrize("arch", ARCHS)
def test_graph_replay_of_mlp_steps_matches_eager(arch):
    wl, p, plan_g, prm, lo, span = _tophat_setup("random", arch)
    plan_e = ffrt.Plan(wl.problems)
    T = plan_g.pack_img(wl.targets)
    st_g = plan_g.new_mlp_state(plan_g.pack_mlp([prm], arch), _dev(lo, plan_g), _dev(span, plan_g), arch=arch)
    st_e = plan_e.new_mlp_state(plan_e.pack_mlp([prm], arch), _dev(lo, plan_e), _dev(span, plan_e), arch=arch)
    hp = _linear_hp(plan_e, st_e, T, lr=0.01)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan_g.graph_capture_mlp(st_g, T, steps=3, hp=hp)
    torch.cuda.synchronize()
    for k in range(2):
        with torch.cuda.stream(s):
            plan_g.graph_launch()
        s.synchronize()
        for _ in range(3):
            plan_e.step_mlp(st_e, T, hp=hp)
        _ = torch.ones(1000, device="cuda").sum().item()      # unrelated eager work between replays
        torch.cuda.synchronize()
        # dL/dP is reproducible bit for bit, but the dense generator's transposed products add their
        # partial sums with float atomics: a component whose terms nearly cancel carries up to ~1e-4 relative
        # rounding between runs, which Adam turns into ~lr 1e-4 parameter differences per step.  A replay
        # that skipped a step or read stale parameters would differ by ~lr.
        torch.testing.assert_close(st_g["params"], st_e["params"], rtol=0, atol=3e-5)
        torch.testing.assert_close(st_g["Pz"], st_e["Pz"], rtol=0, atol=3e-5)
        assert int(st_g["t"][0]) == 3 * (k + 1)


@pytest.mark.parametrize("arch", ARCHS)
def test_zero_initialised_generator_follows_the_no_network_optimisation(arch):
    """With every parameter zero only b3 is ever updated (the oracle pins this identity; sec. 3.2 states it
    for the sparse network), so the generator's control heights follow the no-network (reparametrised)
    optimisation started at theta = 0."""
    wl, p, plan, prm, lo, span = _tophat_setup("zero", arch)
    T = plan.pack_img(wl.targets)
    lo_d, sp_d = _dev(lo, plan), _dev(span, plan)
    st_m = plan.new_mlp_state(plan.pack_mlp([prm], arch), lo_d, sp_d, arch=arch)
    st_r = plan.new_reparam_state(torch.zeros(plan.total_cp, device=plan.device), lo_d, sp_d)
    hp = _linear_hp(plan, st_m, T, lr=0.03)
    for _ in range(20):
        plan.step_mlp(st_m, T, hp=hp)
        plan.step_reparam(st_r, T, hp=hp)
    torch.cuda.synchronize()
    w1, b1, W2, b2, W3, b3 = plan.unpack_mlp(st_m["params"], arch)[0]
    for a in (w1, b1, W2, b2, W3):
        assert not torch.any(a)
    # the two chain rules round differently (see _linear_hp)
    torch.testing.assert_close(b3, st_r["theta"], rtol=0, atol=3e-5)
    torch.testing.assert_close(st_m["Pz"], st_r["Pz"], rtol=0, atol=3e-5)


@pytest.mark.parametrize("arch", ARCHS)
def test_tophat_design_loop_with_a_generator(arch):
    """The network arms of the circular top-hat case with the paper's small uniform initialisation: the loss
    falls, every height stays inside its range, and the final loss agrees with the oracle's."""
    wl, p, plan, prm, lo, span = _tophat_setup("uniform", arch)
    T = plan.pack_img(wl.targets)
    st = plan.new_mlp_state(plan.pack_mlp([prm], arch), _dev(lo, plan), _dev(span, plan), arch=arch)
    hp = ffrt.AdamHP(lr=1e-3)
    losses = []
    for k in range(300):
        plan.step_mlp(st, T, hp=hp)
        if k % 50 == 0:
            losses.append(st["loss"].item())
    irr = plan.forward(st["Pz"])
    L_end = plan.loss(irr, T)[0].item()
    _say(f"[tophat arch {arch}] loss {losses} -> {L_end:.4e}")
    assert L_end < 0.35 * losses[0]
    P = st["Pz"].cpu().numpy().reshape(p.cp_shape())
    assert (P >= lo - 1e-6).all() and (P <= lo + span + 1e-6).all()
    L64 = O.loss(O.forward(p, P.astype(np.float64))[0], wl.targets[0])[0]
    assert abs(L_end - L64) <= 1e-3 * L64


def test_mlp_rejects_wrong_sizes():
    wl, p, plan, prm, lo, span = _tophat_setup("zero", ffrt.MLP_DENSE)
    with pytest.raises(ffrt.FfrtError):
        plan.mlp_forward(torch.zeros(10, device=plan.device), _dev(lo, plan), _dev(span, plan))
    with pytest.raises(ffrt.FfrtError):
        plan.pack_mlp([[np.zeros(3)] * 6])
    with pytest.raises(ffrt.FfrtError):
        plan.mlp_forward(plan.pack_mlp([prm]), _dev(lo, plan), _dev(span, plan), arch=2)
