"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics (no GPU).

Each test checks the oracle against something other than itself: a library routine (scipy B-splines,
torch Adam), a closed form (flat slab, paraxial focus, filter at a pixel centre, hand-computed loss),
an invariant the paper states (partition of unity, Greville linearity, flux conservation, the flat-lens
derivative sums of sec. 3.1), or brute-force finite differences on tiny inputs.
"""
import os
from dataclasses import replace

import numpy as np
import pytest
from scipy.interpolate import BSpline

import oracle as O
import surfaces as S
from paper_2302_12031_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------------------------------------
# B-spline basis and surface (sec. 2.1, 2.1.1)
# ------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("p,n", [(1, 4), (2, 5), (3, 8), (3, 16), (4, 9), (5, 8), (5, 32)])
def test_basis_matches_scipy(p, n):
    U = O.knots(p, n)
    us = np.concatenate([np.random.default_rng(p * 100 + n).uniform(0, 1, 200), U[p:n + 1], [1.0]])
    for u in us:
        ref = BSpline.design_matrix(np.array([u]), U, p).toarray()[0]
        np.testing.assert_allclose(O.basis_all(p, n, u, 0), ref, atol=1e-14)
        for der in (1, 2):
            if der > p or u >= 1.0:
                continue
            refd = np.array([BSpline(U, np.eye(n)[i], p)(u, nu=der) for i in range(n)])
            np.testing.assert_allclose(O.basis_all(p, n, u, der), refd, atol=1e-9 * max(1, np.abs(refd).max()))


@pytest.mark.parametrize("p,n", [(2, 6), (3, 8), (3, 13), (5, 9)])
def test_partition_of_unity_and_endpoints(p, n):
    for u in np.random.default_rng(1).uniform(0, 1, 2000):
        assert abs(O.basis_all(p, n, u, 0).sum() - 1.0) < 1e-14
        assert abs(O.basis_all(p, n, u, 1).sum()) < 1e-11
        assert abs(O.basis_all(p, n, u, 2).sum()) < 1e-9
        assert (O.basis_all(p, n, u, 0) >= -1e-16).all()
    b0, b1 = O.basis_all(p, n, 0.0), O.basis_all(p, n, 1.0)
    assert b0[0] == 1.0 and b0[1:].sum() == 0.0          # N_{0,p}(0) = 1
    assert b1[-1] == 1.0 and b1[:-1].sum() == 0.0         # N_{n1,p}(1) = 1


def test_knot_vector_clamped_equispaced():
    p, n = 3, 8
    U = O.knots(p, n)
    assert (U[:p + 1] == 0).all() and (U[-p - 1:] == 1).all()
    np.testing.assert_allclose(np.diff(U[p:n + 1]), 1.0 / (n - p), atol=1e-15)
    np.testing.assert_allclose(U, 1 - U[::-1], atol=1e-15)


def test_interior_span_is_cardinal_cubic():
    rows = np.loadtxt(os.path.join(GOLDEN, "cardinal_cubic_bspline.txt"))
    p, n = 3, 16
    h = 1.0 / (n - p)
    s = 8                          # an interior span: knots s-p+1 .. s+p all distinct
    for t, *vals in rows:
        u = (s - p + t) * h if t < 1 else (s - p + 1) * h - 1e-15
        b = O.basis_all(p, n, u)[s - p:s + 1]
        np.testing.assert_allclose(b, vals, atol=1e-12)


@pytest.mark.parametrize("p,n", [(2, 6), (3, 8), (5, 12)])
def test_greville_makes_x_linear(p, n):
    U = O.knots(p, n)
    g = np.array([U[i + 1:i + p + 1].mean() for i in range(n)])   # Greville abscissae
    r_x = 5.0
    for u in np.linspace(0, 1, 101):
        x = ((2 * g - 1) * r_x) @ O.basis_all(p, n, u)
        assert abs(x - (2 * u - 1) * r_x) < 1e-13


def _prob(n_u=8, n_v=8, **kw):
    p = W.collimated_problem(16, n_u, 16)
    return replace(p, lens=replace(p.lens, n_u=n_u, n_v=n_v, **kw))


def test_surface_matches_scipy_tensor_product():
    pr = _prob(9, 7)
    Pz = W.random_heights(9, 7, 5)
    U, V = O.knots(3, 9), O.knots(3, 7)
    for x, y in np.random.default_rng(2).uniform(-5, 5, (100, 2)):
        u, v = 0.5 * (x / 5 + 1), 0.5 * (y / 5 + 1)
        Bu = BSpline.design_matrix(np.array([u]), U, 3).toarray()[0]
        Bv = BSpline.design_matrix(np.array([v]), V, 3).toarray()[0]
        dBu = np.array([BSpline(U, np.eye(9)[i], 3)(u, nu=1) for i in range(9)])
        dBv = np.array([BSpline(V, np.eye(7)[i], 3)(v, nu=1) for i in range(7)])
        d2Bu = np.array([BSpline(U, np.eye(9)[i], 3)(u, nu=2) for i in range(9)])
        out = O.surface(pr, Pz, x, y)
        assert abs(out[0] - Bu @ Pz @ Bv) < 1e-13
        assert abs(out[1] - (dBu @ Pz @ Bv) / 10) < 1e-11          # d/dx = d/du / (2 r_x)
        assert abs(out[2] - (Bu @ Pz @ dBv) / 10) < 1e-11
        assert abs(out[3] - (d2Bu @ Pz @ Bv) / 100) < 1e-9
        assert abs(out[4] - (dBu @ Pz @ dBv) / 100) < 1e-10


def test_surface_corners_and_edges_interpolate_boundary_control_points():
    pr = _prob(8, 8)
    Pz = W.random_heights(8, 8, 3)
    assert abs(O.surface(pr, Pz, -5, -5)[0] - Pz[0, 0]) < 1e-14
    assert abs(O.surface(pr, Pz, 5, 5)[0] - Pz[-1, -1]) < 1e-14
    assert abs(O.surface(pr, Pz, -5, 5)[0] - Pz[0, -1]) < 1e-14
    V = O.knots(3, 8)
    for y in np.linspace(-5, 5, 11):
        v = 0.5 * (y / 5 + 1)
        Bv = BSpline.design_matrix(np.array([v]), V, 3).toarray()[0]
        assert abs(O.surface(pr, Pz, -5, y)[0] - Pz[0] @ Bv) < 1e-13


def test_convex_hull_bounds_per_span():
    # sec. 2.2.2: on a knot-span product the surface lies within the min/max of the CPs acting on it.
    pr = _prob(10, 10)
    Pz = W.random_heights(10, 10, 9)
    p = 3
    h = 1.0 / (10 - p)
    for x, y in np.random.default_rng(4).uniform(-5, 5, (500, 2)):
        u, v = 0.5 * (x / 5 + 1), 0.5 * (y / 5 + 1)
        su, sv = p + min(int(u / h), 10 - p - 1), p + min(int(v / h), 10 - p - 1)
        blk = Pz[su - p:su + 1, sv - p:sv + 1]
        z = O.surface(pr, Pz, x, y)[0]
        assert blk.min() - 1e-14 <= z <= blk.max() + 1e-14


# ------------------------------------------------------------------------------------------------
# Optics (sec. 2.2, 2.3)
# ------------------------------------------------------------------------------------------------
def test_snell_invariant_unit_length_and_tir_threshold():
    g = np.random.default_rng(7)
    n = 1.5
    for _ in range(500):
        d = g.normal(size=3); d[2] = abs(d[2]) + 0.2; d /= np.linalg.norm(d)
        m = g.normal(size=3) * 0.5; m[2] = 1.0; m /= np.linalg.norm(m)
        if d @ m <= 0:
            continue
        c = d @ m
        out = O.refract(d, m, n)
        sin_i = np.sqrt(max(0.0, 1 - c * c))
        if n * sin_i > 1:
            assert out is None                       # TIR beyond the critical angle
            continue
        assert out is not None
        assert abs(np.linalg.norm(out) - 1) < 1e-14
        # n (d - (d.m) m) = (d_t - (d_t.m) m): tangential momentum is conserved
        np.testing.assert_allclose(n * (d - c * m), out - (out @ m) * m, atol=1e-14)
        assert out @ m > 0
    # exactly at the critical angle sin = 1/n: grazing exit; slightly beyond: TIR
    th = np.arcsin(1 / n)
    for dth, tir in ((-1e-9, False), (1e-9, True)):
        d = np.array([np.sin(th + dth), 0, np.cos(th + dth)])
        assert (O.refract(d, np.array([0, 0, 1.0]), n) is None) == tir
    # normal incidence passes straight
    np.testing.assert_allclose(O.refract(np.array([0, 0, 1.0]), np.array([0, 0, 1.0]), n), [0, 0, 1])


def test_schlick_limits():
    assert abs(O.schlick(1.0, 1.5) - 0.04) < 1e-15      # R0 = ((n-1)/(n+1))^2
    assert abs(O.schlick(0.0, 1.5) - 1.0) < 1e-15
    # derivative in the angle vanishes at normal incidence: R(cos t) = R0 + O(t^10)
    assert abs(O.schlick(np.cos(1e-3), 1.5) - O.schlick(1.0, 1.5)) < 1e-16


def test_single_ray_filter_at_pixel_centre():
    pr = W.collimated_problem(16, 8, 16, R=8.0)              # w = 1 mm
    a = pr.detector.alpha
    img = O.splat_one(pr, 0.5, 0.5)                          # centre of pixel (8, 8)
    e = np.exp(-a * 1.5 ** 2)
    f = np.array([np.exp(-a) - e, 1 - e, np.exp(-a) - e])
    f /= f.sum()
    np.testing.assert_allclose(img[7:10, 7:10], np.outer(f, f), atol=1e-15)
    assert abs(img.sum() - 1.0) < 1e-15 and img[7:10, 7:10].sum() == img.sum()


def test_single_ray_filter_normalised_anywhere_and_edge():
    pr = W.collimated_problem(16, 8, 16, R=8.0)
    for X, Y in np.random.default_rng(3).uniform(-8, 8, (200, 2)):
        img = O.splat_one(pr, X, Y)
        assert abs(img.sum() - 1.0) < 1e-14
        assert (img >= 0).all() and np.count_nonzero(img) <= 9
    img = O.splat_one(pr, -7.5, 0.5)                         # landing in the first column: renormalised
    assert abs(img.sum() - 1) < 1e-14 and img[0].sum() > img[1].sum() > 0


def test_ghost_pixels_enlarge_grid():
    pr = W.collimated_problem(16, 8, 16, R=8.0)
    pg = replace(pr, detector=replace(pr.detector, ghost=1))
    assert O.image_size(pg) == (18, 18)
    a, b = O.splat_one(pr, 0.3, -1.2), O.splat_one(pg, 0.3, -1.2)
    np.testing.assert_allclose(a, b[1:-1, 1:-1], atol=1e-15)
    # at the edge the ghost column takes its share instead of renormalising onto the grid
    b = O.splat_one(pg, -7.9, 0.5)
    assert b[0].sum() > 0 and abs(b.sum() - 1) < 1e-14


def test_filter_continuous_across_window_shift():
    # the filter vanishes at the edge of its support, so a ray crossing a pixel boundary changes the image
    # continuously (the window moves by one pixel)
    pr = W.collimated_problem(16, 8, 16, R=8.0)
    a = O.splat_one(pr, 1.0 - 1e-12, 0.3)
    b = O.splat_one(pr, 1.0, 0.3)
    assert np.abs(a - b).max() < 1e-10


# ------------------------------------------------------------------------------------------------
# Whole-tracer closed forms
# ------------------------------------------------------------------------------------------------
def test_flux_conservation_all_sources():
    for wl in (W.c1(), W.c3(96), W.c4(24, 3)):
        p, Pz = wl.problems[0], wl.Pz[0]
        img, st = O.forward(p, Pz)
        assert st["n_rays"] == p.num_rays()
        assert abs(img.sum() - st["flux_on_screen"]) < 1e-12 * st["flux_on_screen"]
        assert st["n_hit"] + st["n_miss_entry"] + st["n_side_wall"] + st["n_tir"] + st["n_off_screen"] == st["n_rays"]


def test_flat_slab_collimated_closed_form():
    wl = W.c1()
    pr = wl.problems[0]
    Pz = np.full((8, 8), 2.0)
    ids = np.arange(0, pr.num_rays(), 37)
    out = O.trace_rays(pr, Pz, ids)
    S = O.samples(pr, ids)
    assert (out[:, 0] == O.HIT).all()
    np.testing.assert_allclose(out[:, 1], (2 * S[:, 0] - 1) * 5, atol=1e-12)      # lands at its start
    np.testing.assert_allclose(out[:, 2], (2 * S[:, 1] - 1) * 5, atol=1e-12)
    np.testing.assert_allclose(out[:, 3], (1 - 0.04) ** 2 / pr.num_rays(), rtol=1e-13)


@pytest.mark.parametrize("zf", [0.7, 2.0])
def test_flat_slab_point_source_closed_form(zf):
    wl = W.c3(64)
    pr = wl.problems[0]
    Pz = np.full((32, 32), zf)
    ids = np.arange(0, pr.num_rays(), 7)
    out = O.trace_rays(pr, Pz, ids)
    S = O.samples(pr, ids)
    th, a = S[:, 0], S[:, 1]
    cphi = 1 - (1 - np.cos(pr.source.half_angle)) * a
    phi = np.arccos(cphi)
    phit = np.arcsin(np.sin(phi) / 1.5)
    zs, zscr = pr.source.pos[2], pr.detector.z_screen
    rho = (0 - zs) * np.tan(phi) + zf * np.tan(phit) + (zscr - zf) * np.tan(phi)
    ok = out[:, 0] == O.HIT
    assert ok.mean() > 0.99
    np.testing.assert_allclose(out[ok, 1], rho[ok] * np.cos(th[ok]), atol=1e-11)
    np.testing.assert_allclose(out[ok, 2], rho[ok] * np.sin(th[ok]), atol=1e-11)
    R = np.array([O.schlick(c, 1.5) for c in cphi])
    np.testing.assert_allclose(out[ok, 3], (1 - R[ok]) ** 2 / pr.num_rays(), rtol=1e-12)
    np.testing.assert_allclose(out[ok, 6], zf / np.cos(phit[ok]), rtol=1e-12)       # path length in glass


def test_side_wall_closed_form():
    # flat slab, wide cone from just below the entry face: rays that would cross x = +-r inside the glass
    pr = W.point_problem(64, 8, 64, R=200.0, half_angle_deg=75.0)
    pr = replace(pr, source=replace(pr.source, pos=(0.0, 0.0, -1.0)))
    T = 2.0
    Pz = np.full((8, 8), T)
    ids = np.arange(pr.num_rays())
    out = O.trace_rays(pr, Pz, ids)
    S = O.samples(pr, ids)
    th, a = S[:, 0], S[:, 1]
    phi = np.arccos(1 - (1 - np.cos(pr.source.half_angle)) * a)
    phit = np.arcsin(np.sin(phi) / 1.5)
    p0 = np.tan(phi)[:, None] * np.stack([np.cos(th), np.sin(th)], 1)
    p1 = p0 + (T * np.tan(phit))[:, None] * np.stack([np.cos(th), np.sin(th)], 1)
    miss_entry = (np.abs(p0) > 5).any(1)
    side = ~miss_entry & (np.abs(p1) > 5).any(1)
    far = np.abs(np.abs(p1) - 5).min(1) > 1e-6
    assert (out[miss_entry, 0] == O.MISS_ENTRY).all()
    assert side.sum() > 10
    assert (out[side & far, 0] == O.SIDE_WALL).all()
    assert np.isin(out[~side & ~miss_entry & far, 0], [O.HIT, O.OFF_SCREEN]).all()


def test_spherical_cap_paraxial_focus():
    # Convex cap h = z_v - (R_c - sqrt(R_c^2 - r^2)) put on the B-spline by the Greville (Schoenberg)
    # quasi-interpolant.  Paraxial collimated rays must cross the axis at h(0,0) + 1/((n-1) kappa), kappa the
    # B-spline's own vertex curvature, which in turn is close to 1/R_c (plano-convex back focal length).
    n_cp, p = 24, 3
    U = O.knots(p, n_cp)
    g = np.array([U[i + 1:i + p + 1].mean() for i in range(n_cp)])
    Px = (2 * g - 1) * 5
    Rc, zv = 30.0, 3.0
    r2 = Px[:, None] ** 2 + Px[None, :] ** 2
    Pz = zv - (Rc - np.sqrt(Rc ** 2 - r2))
    pr = W.collimated_problem(2001, n_cp, 64, R=1000.0, z=200.0)
    pr = replace(pr, options=replace(pr.options, fresnel=0))
    s = O.surface(pr, Pz, 0.0, 0.0)
    kappa = -s[3]
    assert abs(s[1]) < 1e-14 and abs(s[4]) < 1e-13 and abs(s[3] - s[5]) < 1e-12
    assert abs(kappa * Rc - 1) < 2e-3
    f_back = 1 / ((1.5 - 1) * kappa)
    ids = np.array([1000 * 2001 + 1000 + k for k in (1, 2, 3)])     # rays at x = 0, y = 5k/2001 mm
    out = O.trace_rays(pr, Pz, ids)
    S = O.samples(pr, ids)
    for (st, X, Y, *_), (u, v, *_) in zip(out, S):
        y0 = (2 * v - 1) * 5
        h = O.surface(pr, Pz, 0.0, y0)[0]
        z_cross = h + y0 * (200.0 - h) / (y0 - Y)
        rel = (z_cross - s[0] - f_back) / f_back          # measured from the B-spline's own vertex
        assert abs(rel) < 10 * (y0 / f_back) ** 2 + 1e-9
        assert abs(X) < 1e-12


# ------------------------------------------------------------------------------------------------
# Sampling (sec. 2.2.1)
# ------------------------------------------------------------------------------------------------
def test_point_samples_uniform_in_solid_angle():
    pr = W.c3(128).problems[0]
    S = O.samples(pr, np.arange(pr.num_rays()))
    cphi = 1 - (1 - np.cos(pr.source.half_angle)) * S[:, 1]
    # E[cos phi] over a cone uniform in solid angle is (1 + cos phi_max) / 2
    assert abs(cphi.mean() - (1 + np.cos(pr.source.half_angle)) / 2) < 1e-4
    assert S[:, 0].min() >= 0 and S[:, 0].max() < 2 * np.pi
    # stratified: every (theta, a) stratum holds exactly one sample
    kt = np.floor(S[:, 0] / (2 * np.pi) * 128).astype(int)
    ka = np.floor(S[:, 1] * 128).astype(int)
    assert len(set(zip(kt, ka))) == 128 * 128


def test_rng_uniformity_and_streams():
    xs = np.array([O.rng(7, 2, i) for i in range(20000)], dtype=np.uint64)
    a = (xs >> np.uint64(40)).astype(np.float64) / 2 ** 24
    assert abs(a.mean() - 0.5) < 0.01 and abs(a.var() - 1 / 12) < 0.005
    assert len(set(xs.tolist())) == len(xs)
    assert O.rng(7, 2, 5) != O.rng(7, 3, 5) and O.rng(7, 2, 5) != O.rng(8, 2, 5)


def test_splitmix64_matches_the_published_outputs():
    """The counter-based generator against the reference implementation's outputs for seed 0."""
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")
    ref = [int(l, 16) for l in open(path) if l.strip() and not l.startswith("#")]
    assert [O.rng(0, 0, i) for i in range(len(ref))] == ref


@pytest.mark.parametrize("jitter", [0, 1])
def test_collimated_samples_one_per_cell(jitter):
    """Collimated samples (sec. 2.2.1): cell (k_u, k_v) of the N_u x N_v grid holds exactly one sample, at the
    cell centre ((k + 1/2) / N) without jitter, anywhere inside it with jitter, with 24-bit sub-cell offsets
    (so that single precision represents the sample exactly)."""
    pr = replace(W.c1().problems[0], source=replace(W.c1().problems[0].source, grid_u=24, grid_v=16, jitter=jitter,
                                                                                 seed=3))
    ids = np.arange(24 * 16)
    S = O.samples(pr, ids)
    ku, kv = ids // 16, ids % 16
    fu, fv = S[:, 0] * 24 - ku, S[:, 1] * 16 - kv
    if jitter:
        assert (fu >= 0).all() and (fu < 1).all() and (fv >= 0).all() and (fv < 1).all()
        for f in (fu, fv):
            np.testing.assert_array_equal(f * 2 ** 24, np.round(f * 2 ** 24))
            assert abs(f.mean() - 0.5) < 0.05 and len(set(f.tolist())) == len(f)
    else:
        np.testing.assert_array_equal(fu, 0.5)
        np.testing.assert_array_equal(fv, 0.5)
    assert (S[:, 0] * 24).astype(int).tolist() == ku.tolist() and (S[:, 1] * 16).astype(int).tolist() == kv.tolist()


def test_smallest_root_of_rays_that_cross_the_surface_twice():
    """The root problem of sec. 2.2.1 asks for the smallest positive root.  On the valley h = 2 + x^2 / 2 (an
    exact B-spline, checked first) rays from a wide cone cross the exit face, leave the glass and meet the
    rising wall again: f(t) = h(o + t d) - o_z - t d_z is a quadratic in t with two positive roots inside the
    aperture, known in closed form.  The oracle must return the smaller one (its scan for the first sign
    change), for every ray whose two roots are not within rounding of each other."""
    pr = S.valley_problem()
    Pz = S.valley_heights()
    xs = np.linspace(-5, 5, 23)
    for x in xs:
        for y in (-4.0, 0.3, 4.9):
            np.testing.assert_allclose(O.surface(pr, Pz, x, y)[0], 2.0 + 0.5 * x * x, rtol=0, atol=1e-12)
    ids = np.arange(pr.num_rays())
    o, d = _glass_rays(pr, ids)
    out = O.trace_rays(pr, Pz, ids)
    t1, t2 = S.valley_roots(o, d)
    ok = np.isfinite(t1)
    t_ap = S.aperture_exit(o, d)
    entered = out[:, 0] != O.MISS_ENTRY
    # both roots inside the aperture and further apart than the oracle's scan step (1/64 of a projected
    # knot span, at most ~0.07 here): the scan must stop at the first
    two = entered & ok & (t1 > 0) & (t2 < t_ap - 1e-6) & (t2 - t1 > 0.2)
    assert two.sum() >= 200, two.sum()
    assert (out[two, 0] != O.SIDE_WALL).all()
    np.testing.assert_allclose(out[two, 6], t1[two], rtol=0, atol=1e-9)
    # rays with a single crossing inside the aperture find it too
    one = entered & ok & (t1 > 0) & (t1 < t_ap - 1e-6) & (t2 > t_ap + 1e-6)
    assert one.sum() >= 200, one.sum()
    np.testing.assert_allclose(out[one, 6], t1[one], rtol=0, atol=1e-9)
    # and rays that stay below the surface until they leave the aperture go through the side wall
    none = entered & (~ok | (t1 > t_ap + 1e-6)) & (t_ap > 0)
    assert none.sum() >= 100 and (out[none, 0] == O.SIDE_WALL).all()


def test_grid_source_emitters_include_endpoints():
    pr = W.c4(8, 3).problems[0]
    per = 64
    S = O.samples(pr, np.arange(0, 9 * per, per))
    np.testing.assert_allclose(sorted(set(np.round(S[:, 2], 12))), [-0.5, 0.0, 0.5])
    np.testing.assert_allclose(sorted(set(np.round(S[:, 3], 12))), [-0.5, 0.0, 0.5])


# ------------------------------------------------------------------------------------------------
# Loss (sec. 2.5)
# ------------------------------------------------------------------------------------------------
def test_loss_hand_computed_2x2():
    L, g = O.loss(np.array([[1.0, 0.0], [0.0, 1.0]]), np.ones((2, 2)))
    # I_hat = diag(1/2), I_ref_hat = 1/4: D = +-1/4, ||D||_F = 1/2, L = (1/2)/sqrt(4)
    assert abs(L - 0.25) < 1e-16


def test_loss_invariances_and_gradient_fd():
    g = np.random.default_rng(0)
    I, T = g.uniform(0, 1, (6, 5)), g.uniform(0, 1, (6, 5))
    L, G = O.loss(I, T)
    assert abs(O.loss(3.7 * I, 0.2 * T)[0] - L) < 1e-15
    assert O.loss(2 * T, T)[0] < 1e-16
    h = 1e-6
    for idx in [(0, 0), (3, 2), (5, 4)]:
        E = np.zeros_like(I); E[idx] = h
        fd = (O.loss(I + E, T)[0] - O.loss(I - E, T)[0]) / (2 * h)
        assert abs(fd - G[idx]) < 1e-8 * max(1, abs(G).max())
    assert abs((G * I).sum()) < 1e-14           # scale invariance: dL/dI is orthogonal to I


def test_sum_of_squares_loss_hand_computed_2x2():
    """Loss kind 1, ||I_hat - T_hat||_F^2.  I = e_00, T = 1: I_hat = e_00, T_hat = 1/4, D = (3/4, -1/4, -1/4,
    -1/4), so L = 12/16 = 3/4; sum(D I_hat) = 3/4, s = 1, so dL/dI = 2 (D - 3/4) = (0, -2, -2, -2)."""
    I = np.array([[1.0, 0.0], [0.0, 0.0]])
    L, G = O.loss(I, np.ones((2, 2)), kind=1)
    assert L == 0.75
    np.testing.assert_array_equal(G, [[0.0, -2.0], [-2.0, -2.0]])
    # the RMS loss of the same pair: sqrt(3/4) / 2
    assert abs(O.loss(I, np.ones((2, 2)))[0] - np.sqrt(0.75) / 2) < 1e-16


def test_sum_of_squares_loss_invariances_and_gradient_fd():
    g = np.random.default_rng(3)
    I, T = g.uniform(0, 1, (7, 4)), g.uniform(0, 1, (7, 4))
    L, G = O.loss(I, T, kind=1)
    assert abs(O.loss(0.3 * I, 5.0 * T, kind=1)[0] - L) < 1e-15
    h = 1e-6
    for idx in [(0, 0), (4, 1), (6, 3)]:
        E = np.zeros_like(I); E[idx] = h
        fd = (O.loss(I + E, T, kind=1)[0] - O.loss(I - E, T, kind=1)[0]) / (2 * h)
        assert abs(fd - G[idx]) < 1e-8 * max(1, abs(G).max())
    assert abs((G * I).sum()) < 1e-14
    with pytest.raises(Exception):
        O.loss(I, T, kind=2)


# ------------------------------------------------------------------------------------------------
# Gradient (pathwise derivative) against brute-force finite differences on tiny inputs
# ------------------------------------------------------------------------------------------------
def _tiny(kind):
    if kind == "collimated":
        pr = W.collimated_problem(16, 5, 8, R=12.0, z=30.0)
    elif kind == "collimated_ghost":
        pr = W.collimated_problem(16, 6, 8, R=8.0, z=30.0)
        pr = replace(pr, detector=replace(pr.detector, ghost=1))
    elif kind == "point":
        pr = W.point_problem(16, 5, 8, R=40.0, z=40.0)
    elif kind == "grid":
        pr = W.point_problem(8, 5, 8, R=40.0, z=40.0, emitters=2, emit_w=1.0)
    else:
        pr = W.point_problem(16, 6, 8, R=40.0, z=40.0)
        pr = replace(pr, lens=replace(pr.lens, p=5, q=3), options=replace(pr.options, fresnel=0))
    n_u, n_v = pr.lens.n_u, pr.lens.n_v
    Pz = W.random_heights(n_u, n_v, 11, spread=0.3)
    T = W.target_mixture(pr, 11, 3, 3)
    return pr, Pz, T


@pytest.mark.parametrize("kind", ["collimated", "collimated_ghost", "point", "grid", "p5q3_nofresnel"])
def test_gradient_matches_central_fd(kind):
    pr, Pz, T = _tiny(kind)
    L, g, irr, G = O.grad(pr, Pz, T)
    ids = np.arange(pr.num_rays())
    base = O.trace_rays(pr, Pz, ids)[:, 0]
    h = 1e-6
    checked = 0
    for k in range(Pz.size):
        E = np.zeros(Pz.size); E[k] = h
        E = E.reshape(Pz.shape)
        sp = O.trace_rays(pr, Pz + E, ids)[:, 0]
        sm = O.trace_rays(pr, Pz - E, ids)[:, 0]
        if (sp != base).any() or (sm != base).any():
            continue      # a ray changes its discrete state within +-h: FD is not the pathwise derivative
        Lp = O.loss(O.forward(pr, Pz + E)[0], T)[0]
        Lm = O.loss(O.forward(pr, Pz - E)[0], T)[0]
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g.flat[k]) <= 1e-6 * np.abs(g).max() + 1e-7 * abs(fd), (k, fd, g.flat[k])
        checked += 1
    assert checked >= Pz.size // 2


def test_sum_of_squares_gradient_matches_central_fd():
    """The pathwise gradient of the sum-of-squares loss (option loss = 1) against central differences of that
    loss, on the tiny point-source problem."""
    pr, Pz, T = _tiny("point")
    pr = replace(pr, options=replace(pr.options, loss=1))
    L, g, irr, G = O.grad(pr, Pz, T)
    assert abs(L - O.loss(irr, T, kind=1)[0]) < 1e-15
    ids = np.arange(pr.num_rays())
    base = O.trace_rays(pr, Pz, ids)[:, 0]
    h = 1e-6
    checked = 0
    for k in range(Pz.size):
        E = np.zeros(Pz.size); E[k] = h
        E = E.reshape(Pz.shape)
        if (O.trace_rays(pr, Pz + E, ids)[:, 0] != base).any() or (O.trace_rays(pr, Pz - E, ids)[:, 0] != base).any():
            continue
        fd = (O.loss(O.forward(pr, Pz + E)[0], T, kind=1)[0] - O.loss(O.forward(pr, Pz - E)[0], T, kind=1)[0]) / (2 * h)
        assert abs(fd - g.flat[k]) <= 1e-6 * np.abs(g).max() + 1e-7 * abs(fd), (k, fd, g.flat[k])
        checked += 1
    assert checked >= Pz.size // 2


def test_image_jvp_matches_central_fd_and_locality():
    pr, Pz, T = _tiny("point")
    k = (1, 2)
    v = np.zeros_like(Pz); v[k] = 1.0
    dI = O.jvp(pr, Pz, v)
    h = 1e-6
    fd = (O.forward(pr, Pz + h * v)[0] - O.forward(pr, Pz - h * v)[0]) / (2 * h)
    np.testing.assert_allclose(dI, fd, atol=1e-6 * np.abs(dI).max())
    # locality: only rays hitting inside supp N_{1,p} x N_{2,q} contribute
    U, V = O.knots(3, 5), O.knots(3, 5)
    ids = np.arange(pr.num_rays())
    out = O.trace_rays(pr, Pz, ids)
    hit = out[:, 0] == O.HIT
    inside = (out[:, 4] >= U[k[0]]) & (out[:, 4] < U[k[0] + 4]) & (out[:, 5] >= V[k[1]]) & (out[:, 5] < V[k[1] + 4])
    touched = np.zeros_like(dI, dtype=bool)
    for X, Y in out[hit & inside][:, 1:3]:
        touched |= O.splat_one(pr, X, Y) > 0
    assert np.abs(dI[~touched]).max() == 0.0
    assert np.abs(dI[touched]).max() > 0.0


@pytest.mark.parametrize("p,q,nu", [(3, 3, 3), (3, 3, 11), (5, 3, 3)])
def test_flat_lens_derivative_sums_conserve_light(p, q, nu):
    # Sec. 3.1: for a flat lens under a collimated bundle, sum_ij dI_ij/dP is ~0 (light is conserved and
    # Schlick's slope vanishes at normal incidence).  The paper prints |sum| <= 1e-4 against a total of 93.
    rows = [l.split() for l in open(os.path.join(GOLDEN, "flat_lens_derivative_sums.txt")) if not l.startswith("#")]
    printed = {(int(r[0]), int(r[1]), int(r[2])): float(r[3]) for r in rows if len(r) == 4}
    total = float([r for r in rows if len(r) == 1][0][0])
    pr = W.collimated_problem(64, 10, 48, R=8.0, z=20.0)
    pr = replace(pr, lens=replace(pr.lens, p=p, q=q), detector=replace(pr.detector, nu_x=nu, nu_y=nu))
    Pz = np.full((10, 10), 2.0)
    v = np.zeros_like(Pz); v[4, 5] = 1.0
    img, st = O.forward(pr, Pz)
    assert st["n_hit"] == pr.num_rays()
    dI = O.jvp(pr, Pz, v)
    rel = abs(dI.sum()) / img.sum()
    assert rel < 1e-12
    assert rel <= abs(printed[(p, q, nu)]) / total + 1e-12
    assert np.abs(dI).max() > 1e-3 * img.max()     # the derivative itself is not trivially zero


# ------------------------------------------------------------------------------------------------
# Adam and determinism
# ------------------------------------------------------------------------------------------------
def test_adam_matches_torch():
    import torch
    g = np.random.default_rng(5)
    P = g.normal(size=50)
    m, v = np.zeros(50), np.zeros(50)
    tp = torch.tensor(P.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 8):
        grad = g.normal(size=50)
        O.adam(P, grad, m, v, t)
        tp.grad = torch.tensor(grad)
        opt.step()
        np.testing.assert_allclose(P, tp.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_threads_do_not_change_results():
    wl = W.c3(64)
    p, Pz, T = wl.problems[0], wl.Pz[0], wl.targets[0]
    a = O.forward(p, Pz, threads=1)[0]
    b = O.forward(p, Pz, threads=5)[0]
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-18)
    ga = O.grad(p, Pz, T, threads=1)[1]
    gb = O.grad(p, Pz, T, threads=3)[1]
    np.testing.assert_allclose(ga, gb, rtol=1e-11, atol=1e-18)


# ---------------------------------------------------------------------------------------------------
# Range reparametrisation (sec. 2.4.1) and control-point positions (sec. 2.1.1)
# ---------------------------------------------------------------------------------------------------
def test_reparam_limits_and_derivative():
    """P = lo + (tanh(theta) + 1) span / 2: the middle of the range at theta = 0, its ends as theta -> -+inf;
    the chain-rule factor against central differences."""
    lo, span = np.array([1.8, -0.3, 2.0]), np.array([0.4, 1.0, 0.0])
    np.testing.assert_allclose(O.reparam(np.zeros(3), lo, span), lo + span / 2, rtol=0, atol=1e-15)
    np.testing.assert_allclose(O.reparam(np.full(3, 40.0), lo, span), lo + span, rtol=0, atol=1e-15)
    np.testing.assert_allclose(O.reparam(np.full(3, -40.0), lo, span), lo, rtol=0, atol=1e-15)
    th = np.array([-1.3, 0.2, 0.9])
    g = np.array([0.7, -2.0, 5.0])
    h = 1e-6
    fd = g * (O.reparam(th + h, lo, span) - O.reparam(th - h, lo, span)) / (2 * h)
    np.testing.assert_allclose(O.reparam_grad(th, span, g), fd, rtol=1e-8, atol=1e-12)


def test_reparam_gradient_through_the_loss_matches_fd():
    """dL/dtheta = dL/dP * dP/dtheta through the traced loss, against central differences in theta."""
    from paper_2302_12031_amd import workloads as W
    p = W.collimated_problem(48, 6, 16, jitter=0, seed=3, R=8.0, z=30.0)
    lo, span = W.tophat_range(p)
    th = W.rng(3, 9).uniform(-0.5, 0.5, p.cp_shape())
    T = W.circular_tophat(p, 4.0)
    P = O.reparam(th, lo, span)
    L0, gP, _, _ = O.grad(p, P, T)
    gth = O.reparam_grad(th, span, gP)
    h = 1e-6
    for k in [(1, 1), (2, 3), (4, 2)]:
        E = np.zeros_like(th)
        E[k] = h
        Lp = O.loss(O.forward(p, O.reparam(th + E, lo, span))[0], T)[0]
        Lm = O.loss(O.forward(p, O.reparam(th - E, lo, span))[0], T)[0]
        assert abs((Lp - Lm) / (2 * h) - gth[k]) <= 1e-5 * np.abs(gth).max(), k


def test_control_xy_are_greville_positions():
    """The control points' x make X(u) = (2u - 1) r_x exactly: sum_i x_i N_i(u) = (2u - 1) r_x."""
    from paper_2302_12031_amd import workloads as W
    p = W.collimated_problem(32, 9, 16)
    x, y = O.control_xy(p)
    L = p.lens
    for u in np.linspace(0.0, 1.0, 13):
        Nu = O.basis_all(L.p, L.n_u, u)
        assert abs(Nu @ x[:, 0] - (2 * u - 1) * L.r_x) < 1e-13
        Nv = O.basis_all(L.q, L.n_v, u)
        assert abs(Nv @ y[0, :] - (2 * u - 1) * L.r_y) < 1e-13


# ------------------------------------------------------------------------------------------------
# Dense control-point generator (sec. 2.4): three fully connected tanh layers of control-net size
# ------------------------------------------------------------------------------------------------
def _mlp_params(K, seed, scale=0.6):
    g = np.random.default_rng(seed)
    return [g.normal(0, scale, K), g.normal(0, scale, K), g.normal(0, scale / np.sqrt(K), (K, K)),
            g.normal(0, scale, K), g.normal(0, scale / np.sqrt(K), (K, K)), g.normal(0, scale, K)]


def test_mlp_forward_matches_torch_linear_layers():
    """The forward pass equals torch.nn.Linear layers (weight [out, in], input 1) in float64, followed by
    the output correction."""
    import torch
    K = 7
    prm = _mlp_params(K, 1)
    lo, span = np.linspace(1.8, 2.1, K), np.linspace(0.2, 0.5, K)
    net = torch.nn.Sequential(torch.nn.Linear(1, K), torch.nn.Tanh(), torch.nn.Linear(K, K), torch.nn.Tanh(),
                              torch.nn.Linear(K, K), torch.nn.Tanh()).double()
    with torch.no_grad():
        net[0].weight.copy_(torch.tensor(prm[0])[:, None])
        net[0].bias.copy_(torch.tensor(prm[1]))
        net[2].weight.copy_(torch.tensor(prm[2]))
        net[2].bias.copy_(torch.tensor(prm[3]))
        net[4].weight.copy_(torch.tensor(prm[4]))
        net[4].bias.copy_(torch.tensor(prm[5]))
        y = net(torch.ones(1, 1, dtype=torch.float64))[0].numpy()
    (h1, h2, yo), P = O.mlp_forward(prm, lo, span)
    np.testing.assert_allclose(yo, y, rtol=0, atol=1e-15)
    np.testing.assert_allclose(P, lo + 0.5 * (y + 1.0) * span, rtol=0, atol=1e-15)


def test_mlp_backward_matches_central_fd():
    """Every parameter's gradient of J = c . P against central differences (fp64, h = 1e-6)."""
    K = 5
    prm = _mlp_params(K, 2)
    lo, span = np.full(K, 1.9), np.linspace(0.1, 0.6, K)
    c = np.random.default_rng(3).normal(size=K)
    acts, _ = O.mlp_forward(prm, lo, span)
    grads = O.mlp_backward(prm, acts, span, c)
    h = 1e-6
    for a, (p, g) in enumerate(zip(prm, grads)):
        assert g.shape == p.shape
        fd = np.zeros_like(p)
        for idx in np.ndindex(p.shape):
            q = [x.copy() for x in prm]
            q[a][idx] += h
            Jp = c @ O.mlp_forward(q, lo, span)[1]
            q[a][idx] -= 2 * h
            Jm = c @ O.mlp_forward(q, lo, span)[1]
            fd[idx] = (Jp - Jm) / (2 * h)
        np.testing.assert_allclose(g, fd, rtol=0, atol=1e-8 * max(1.0, np.abs(fd).max()), err_msg=str(a))


def test_mlp_hidden_unit_symmetries():
    """Relabelling the neurons of a hidden layer (with the weights that touch them) or flipping the sign of
    one (tanh is odd) leaves the output unchanged; negating every bias and w1 negates y."""
    K = 6
    prm = _mlp_params(K, 4)
    lo, span = np.zeros(K), np.ones(K)
    y0 = O.mlp_forward(prm, lo, span)[0][2]
    pi = np.random.default_rng(5).permutation(K)
    w1, b1, W2, b2, W3, b3 = prm
    y1 = O.mlp_forward([w1[pi], b1[pi], W2[:, pi], b2, W3, b3], lo, span)[0][2]
    y2 = O.mlp_forward([w1, b1, W2[pi, :], b2[pi], W3[:, pi], b3], lo, span)[0][2]
    s = np.ones(K)
    s[2] = -1.0
    y3 = O.mlp_forward([w1 * s, b1 * s, W2 * s[None, :], b2, W3, b3], lo, span)[0][2]
    y4 = O.mlp_forward([w1, b1, W2 * s[:, None], b2 * s, W3 * s[None, :], b3], lo, span)[0][2]
    for y in (y1, y2, y3, y4):
        np.testing.assert_allclose(y, y0, rtol=0, atol=1e-15)
    y5 = O.mlp_forward([-w1, -b1, W2, -b2, W3, -b3], lo, span)[0][2]
    np.testing.assert_allclose(y5, -y0, rtol=0, atol=1e-15)


def test_mlp_at_zero_is_the_no_network_case():
    """With every weight and the first two layers' biases zero, P = reparam(b3) and only b3 receives a
    gradient, equal to the no-network chain rule at theta = b3: the generator started at zero follows the
    no-network optimisation exactly."""
    K = 9
    b3 = np.random.default_rng(6).normal(0, 0.4, K)
    prm = [np.zeros(K), np.zeros(K), np.zeros((K, K)), np.zeros(K), np.zeros((K, K)), b3]
    lo, span = np.linspace(1.8, 2.0, K), np.linspace(0.3, 0.4, K)
    g = np.random.default_rng(7).normal(size=K)
    acts, P = O.mlp_forward(prm, lo, span)
    np.testing.assert_allclose(P, O.reparam(b3, lo, span), rtol=0, atol=1e-15)
    grads = O.mlp_backward(prm, acts, span, g)
    for a in range(5):
        assert not np.any(grads[a]), a
    np.testing.assert_allclose(grads[5], O.reparam_grad(b3, span, g), rtol=1e-14, atol=0)


def _sparse_params(n_u, n_v, p, q, seed, scale=0.5):
    g = np.random.default_rng(seed)
    K, C = n_u * n_v, (2 * p + 1) * (2 * q + 1)
    return [g.normal(0, scale, K), g.normal(0, scale, K), g.normal(0, scale / np.sqrt(C), (C, K)),
            g.normal(0, scale, K), g.normal(0, scale / np.sqrt(C), (C, K)), g.normal(0, scale, K)]


@pytest.mark.parametrize("n_u,n_v,p,q", [(5, 4, 1, 2), (6, 6, 3, 3)])
def test_sparse_layer_with_a_shared_kernel_is_a_convolution(n_u, n_v, p, q):
    """With one kernel shared by every neuron the sparse layer is torch's zero-padded (2p+1) x (2q+1)
    convolution (cross-correlation) of the layer input laid out on the control net."""
    import torch
    g = np.random.default_rng(8)
    ker = g.normal(size=(2 * p + 1, 2 * q + 1))
    x = g.normal(size=(n_u, n_v))
    Wc = np.repeat(ker.reshape(-1, 1), n_u * n_v, axis=1)
    z = O.sparse_matrix(Wc, n_u, n_v, p, q) @ x.ravel()
    ref = torch.nn.functional.conv2d(torch.tensor(x)[None, None], torch.tensor(ker)[None, None],
                                     padding=(p, q))[0, 0].numpy()
    np.testing.assert_allclose(z, ref.ravel(), rtol=0, atol=1e-13)


def test_sparse_mlp_backward_matches_central_fd():
    """Every stored parameter's gradient of J = c . P against central differences, zero for connections that
    leave the net."""
    n_u, n_v, p, q = 4, 5, 1, 2
    prm = _sparse_params(n_u, n_v, p, q, 9)
    K = n_u * n_v
    lo, span = np.full(K, 1.9), np.linspace(0.1, 0.6, K)
    c = np.random.default_rng(10).normal(size=K)
    acts, _ = O.sparse_mlp_forward(prm, lo, span, n_u, n_v, p, q)
    grads = O.sparse_mlp_backward(prm, acts, span, c, n_u, n_v, p, q)
    h = 1e-6
    for a, (pa, g) in enumerate(zip(prm, grads)):
        assert g.shape == pa.shape
        fd = np.zeros_like(pa)
        for idx in np.ndindex(pa.shape):
            qq = [x.copy() for x in prm]
            qq[a][idx] += h
            Jp = c @ O.sparse_mlp_forward(qq, lo, span, n_u, n_v, p, q)[1]
            qq[a][idx] -= 2 * h
            Jm = c @ O.sparse_mlp_forward(qq, lo, span, n_u, n_v, p, q)[1]
            fd[idx] = (Jp - Jm) / (2 * h)
        np.testing.assert_allclose(g, fd, rtol=0, atol=1e-8 * max(1.0, np.abs(fd).max()), err_msg=str(a))
    # the corner neuron (0, 0) has no input at a = 0 (row -1): those weights are inert
    assert grads[2][0:2 * q + 1, 0].tolist() == [0.0] * (2 * q + 1)


def test_sparse_mlp_at_zero_is_the_no_network_case():
    n_u, n_v, p, q = 5, 5, 3, 3
    K, C = 25, 49
    b3 = np.random.default_rng(11).normal(0, 0.4, K)
    prm = [np.zeros(K), np.zeros(K), np.zeros((C, K)), np.zeros(K), np.zeros((C, K)), b3]
    lo, span = np.full(K, 1.8), np.full(K, 0.4)
    g = np.random.default_rng(12).normal(size=K)
    acts, P = O.sparse_mlp_forward(prm, lo, span, n_u, n_v, p, q)
    np.testing.assert_allclose(P, O.reparam(b3, lo, span), rtol=0, atol=1e-15)
    grads = O.sparse_mlp_backward(prm, acts, span, g, n_u, n_v, p, q)
    for a in range(5):
        assert not np.any(grads[a]), a
    np.testing.assert_allclose(grads[5], O.reparam_grad(b3, span, g), rtol=1e-14, atol=0)


# ------------------------------------------------------------------------------------------------
# Triangle-mesh intersection (sec. 2.2.2): the paper's own intersector, as an option of the oracle
# ------------------------------------------------------------------------------------------------
def _mesh(p, m):
    return replace(p, options=replace(p.options, mesh_u=m, mesh_v=m))


def _glass_rays(p, ids):
    return S.glass_rays(p, ids)


def _mesh_triangles(p, Pz, m):
    """Every triangle of the mesh as three (x, y, z) corners on the surface: m x m rectangles per knot span
    product, each split along the diagonal from (u_k+1, v_l) to (u_k, v_l+1)."""
    L = p.lens
    U, V = O.knots(L.p, L.n_u), O.knots(L.q, L.n_v)
    us = np.unique(np.concatenate([np.linspace(U[i], U[i + 1], m + 1) for i in range(L.p, L.n_u)]))
    vs = np.unique(np.concatenate([np.linspace(V[j], V[j + 1], m + 1) for j in range(L.q, L.n_v)]))
    node = {}
    for a, u in enumerate(us):
        for b, v in enumerate(vs):
            x, y = (2 * u - 1) * L.r_x, (2 * v - 1) * L.r_y
            node[a, b] = np.array([x, y, O.surface(p, Pz, x, y)[0]])
    tris = []
    for a in range(len(us) - 1):
        for b in range(len(vs) - 1):
            tris.append((node[a, b], node[a + 1, b], node[a, b + 1]))
            tris.append((node[a + 1, b + 1], node[a, b + 1], node[a + 1, b]))
    return tris


def _moller_trumbore(o, d, tri):
    """Ray-triangle intersection (Moller & Trumbore 1997): t, or None."""
    v0, v1, v2 = tri
    e1, e2 = v1 - v0, v2 - v0
    pv = np.cross(d, e2)
    det = e1 @ pv
    if abs(det) < 1e-14:
        return None
    s = o - v0
    a = (s @ pv) / det
    qv = np.cross(s, e1)
    b = (d @ qv) / det
    if a < -1e-12 or b < -1e-12 or a + b > 1 + 1e-12:
        return None
    return (e2 @ qv) / det


def test_mesh_hit_is_the_first_triangle_hit_by_brute_force():
    """Point-source rays on a 3 x 3-span surface with 2 x 2 rectangles per span: the oracle's hit (box
    recursion, then the triangles of surviving spans) equals the smallest t over all 72 triangles found by
    Moller-Trumbore, and rays that meet none leave through the side wall."""
    p = _mesh(W.point_problem(12, 6, 16, seed=21, half_angle_deg=40.0), 2)
    Pz = W.random_heights(6, 6, 21, spread=0.4)
    tris = _mesh_triangles(p, Pz, 2)
    ids = np.arange(0, 144, 1)
    o, d = _glass_rays(p, ids)
    out = O.trace_rays(p, Pz, ids)
    n_hit = 0
    for r in range(len(ids)):
        if out[r, 0] == O.MISS_ENTRY:
            continue
        ts = [t for t in (_moller_trumbore(o[r], d[r], tr) for tr in tris) if t is not None and t >= 0]
        if not ts:
            assert out[r, 0] == O.SIDE_WALL, r
            continue
        n_hit += 1
        assert out[r, 0] != O.SIDE_WALL and out[r, 0] != O.MISS_ENTRY, r
        assert abs(out[r, 6] - min(ts)) <= 1e-9 * (1 + min(ts)), (r, out[r, 6], min(ts))
    assert n_hit > 100


def test_mesh_is_exact_on_a_plane():
    """Control heights a + b x_i + c y_j at the Greville positions make the surface a plane (sec. 2.1.1),
    which every triangle mesh represents exactly: mesh and exact hits agree for every ray."""
    p = W.point_problem(16, 8, 32, seed=22, half_angle_deg=35.0)
    x, y = O.control_xy(p)
    Pz = 2.0 + 0.03 * x - 0.02 * y
    ids = np.arange(256)
    ex = O.trace_rays(p, Pz, ids)
    for m in (1, 3):
        me = O.trace_rays(_mesh(p, m), Pz, ids)
        np.testing.assert_array_equal(me[:, 0], ex[:, 0])
        hit = ex[:, 0] == O.HIT
        np.testing.assert_allclose(me[hit, 1:7], ex[hit, 1:7], rtol=0, atol=1e-10)


def test_mesh_converges_quadratically_to_the_exact_hit():
    """Linear interpolation on triangles of size h errs by O(h^2): doubling the rectangles per span cuts
    the largest hit-height error about fourfold."""
    p = W.point_problem(16, 8, 32, seed=23, half_angle_deg=30.0)
    Pz = W.random_heights(8, 8, 23, spread=0.3)
    ids = np.arange(0, 256, 1)
    ex = O.trace_rays(p, Pz, ids)
    errs = []
    for m in (2, 4, 8, 16):
        me = O.trace_rays(_mesh(p, m), Pz, ids)
        ok = (ex[:, 0] == O.HIT) & (me[:, 0] == O.HIT)
        errs.append(np.abs(me[ok, 6] - ex[ok, 6]).max())
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(2.5 < r < 6.0 for r in ratios), (errs, ratios)


@pytest.mark.parametrize("kind", ["collimated", "point"])
def test_mesh_gradient_matches_central_fd(kind):
    """dL/dP of the mesh-mode trace (the hit moves with the corner heights of its triangle; the normal is
    the B-spline's) against central differences of the mesh-mode loss."""
    if kind == "collimated":
        p = _mesh(W.collimated_problem(48, 6, 16, jitter=1, seed=24, R=8.0, z=30.0), 3)
    else:
        p = _mesh(W.point_problem(40, 6, 16, seed=24, R=12.0, z=25.0, half_angle_deg=25.0), 3)
    Pz = W.random_heights(6, 6, 24, spread=0.15)
    T = W.rng(24, 3).uniform(0.5, 1.0, p.image_shape())
    L0, g, _, _ = O.grad(p, Pz, T)
    h = 1e-6
    for k in [(1, 2), (2, 3), (3, 3), (4, 1)]:
        E = np.zeros_like(Pz)
        E[k] = h
        Lp = O.loss(O.forward(p, Pz + E)[0], T)[0]
        Lm = O.loss(O.forward(p, Pz - E)[0], T)[0]
        assert abs((Lp - Lm) / (2 * h) - g[k]) <= 2e-5 * np.abs(g).max(), (k, (Lp - Lm) / (2 * h), g[k])


# ------------------------------------------------------------------------------------------------
# Box reconstruction (sec. 2.3, the simplest reconstruction): each ray's weight in its landing pixel
# ------------------------------------------------------------------------------------------------
def _box(p):
    return replace(p, detector=replace(p.detector, filter=1))


@pytest.mark.parametrize("kind", ["collimated", "point"])
def test_box_image_is_the_weighted_histogram_of_landings(kind):
    """The box image equals numpy's weighted 2-D histogram of the oracle's own ray landings over the pixel
    grid (a library routine), and it conserves the flux on the screen."""
    if kind == "collimated":
        p = _box(W.collimated_problem(64, 8, 32, jitter=1, seed=31))
    else:
        p = _box(W.point_problem(48, 8, 32, seed=31))
    Pz = W.random_heights(8, 8, 31)
    I, st = O.forward(p, Pz)
    R = O.trace_rays(p, Pz, np.arange(O.num_rays(p)))
    hit = R[:, 0] == O.HIT
    D = p.detector
    H, _, _ = np.histogram2d(R[hit, 1], R[hit, 2], bins=[D.n_x, D.n_y], range=[[-D.R_x, D.R_x], [-D.R_y, D.R_y]],
                             weights=R[hit, 3])
    np.testing.assert_allclose(I, H, rtol=1e-12, atol=1e-15)
    assert abs(I.sum() - st["flux_on_screen"]) <= 1e-12


def test_box_gradient_is_the_fresnel_part_only():
    """The box image does not move with the landing position: without Fresnel weights its pathwise gradient
    vanishes; with them it is the weights' derivative, checked against central differences of the image
    with every ray's pixel held fixed."""
    p0 = _box(W.collimated_problem(48, 6, 16, jitter=1, seed=32, R=8.0, z=30.0))
    Pz = W.random_heights(6, 6, 32, spread=0.15)
    T = W.rng(32, 3).uniform(0.5, 1.0, p0.image_shape())
    _, g, _, _ = O.grad(replace(p0, options=replace(p0.options, fresnel=0)), Pz, T)
    assert np.abs(g).max() == 0.0
    L, g, _, G = O.grad(p0, Pz, T)
    ids = np.arange(O.num_rays(p0))
    base = O.trace_rays(p0, Pz, ids)
    k, h = (2, 3), 1e-6
    E = np.zeros_like(Pz)
    E[k] = h
    Rp, Rm = O.trace_rays(p0, Pz + E, ids), O.trace_rays(p0, Pz - E, ids)
    ok = (base[:, 0] == O.HIT) & (Rp[:, 0] == O.HIT) & (Rm[:, 0] == O.HIT)
    D = p0.detector
    pix = (np.floor((base[ok, 1] + D.R_x) / (2 * D.R_x / D.n_x)).astype(int) * D.n_y +
           np.floor((base[ok, 2] + D.R_y) / (2 * D.R_y / D.n_y)).astype(int))
    fd = np.sum(G.ravel()[pix] * (Rp[ok, 3] - Rm[ok, 3]) / (2 * h))
    assert abs(fd - g[k]) <= 1e-6 * max(abs(fd), 1e-12) + 1e-12, (fd, g[k])


# ------------------------------------------------------------------------------------------------
# Both faces freeform (sec. 3.3 and the conclusion propose optimising the entry face too): the entry net
# follows the exit net in Pz
# ------------------------------------------------------------------------------------------------
def _two_faces(p):
    return replace(p, lens=replace(p.lens, entry_freeform=1))


@pytest.mark.parametrize("kind", ["collimated", "point"])
def test_flat_entry_net_reduces_to_the_plano_freeform_lens(kind):
    """An entry net with every height at z_in is the flat entry face: every ray is traced as by the
    plano-freeform lens, to rounding."""
    if kind == "collimated":
        p = W.collimated_problem(32, 8, 32, jitter=1, seed=41)
    else:
        p = W.point_problem(24, 8, 32, seed=41, half_angle_deg=35.0)
    Pz = W.random_heights(8, 8, 41)
    P2 = np.stack([Pz, np.full_like(Pz, p.lens.z_in)])
    ids = np.arange(O.num_rays(p))
    a = O.trace_rays(p, Pz, ids)
    b = O.trace_rays(_two_faces(p), P2, ids)
    np.testing.assert_array_equal(a[:, 0], b[:, 0])
    hit = a[:, 0] == O.HIT
    np.testing.assert_allclose(b[hit, 1:6], a[hit, 1:6], rtol=0, atol=1e-9)


def test_parallel_plate_keeps_every_direction():
    """Two parallel tilted planes make a plate: a ray leaves it in its incoming direction (textbook), so the
    segment from the exit point to the landing point is parallel to the source direction."""
    p = _two_faces(W.point_problem(16, 6, 32, seed=42, half_angle_deg=30.0, R=60.0, z=80.0))
    x, y = O.control_xy(p)
    entry = 0.5 + 0.04 * x - 0.03 * y
    P2 = np.stack([entry + 2.0, entry])
    ids = np.arange(O.num_rays(p))
    R = O.trace_rays(p, P2, ids)
    S = O.samples(p, ids)
    hit = R[:, 0] == O.HIT
    assert hit.sum() > 100
    ca = 1.0 - (1.0 - np.cos(p.source.half_angle)) * S[hit, 1]
    sa = np.sqrt(1.0 - ca ** 2)
    d0 = np.stack([np.cos(S[hit, 0]) * sa, np.sin(S[hit, 0]) * sa, ca], 1)
    L = p.lens
    qx, qy = (2 * R[hit, 4] - 1) * L.r_x, (2 * R[hit, 5] - 1) * L.r_y
    qz = np.array([O.surface(p, P2[0], a, b)[0] for a, b in zip(qx, qy)])
    seg = np.stack([R[hit, 1] - qx, R[hit, 2] - qy, p.detector.z_screen - qz], 1)
    seg /= np.linalg.norm(seg, axis=1, keepdims=True)
    np.testing.assert_allclose(seg, d0, rtol=0, atol=1e-9)


@pytest.mark.parametrize("kind", ["collimated", "point"])
def test_two_face_gradient_matches_central_fd(kind):
    """dL/dP over both nets (exit then entry) against central differences of the loss."""
    if kind == "collimated":
        p = _two_faces(W.collimated_problem(48, 6, 16, jitter=1, seed=43, R=8.0, z=30.0))
    else:
        p = _two_faces(W.point_problem(40, 6, 16, seed=43, R=12.0, z=25.0, half_angle_deg=25.0))
    g0 = W.rng(43, 5)
    P2 = np.stack([W.random_heights(6, 6, 43, spread=0.15) + 1.0, 0.2 + g0.uniform(-0.1, 0.1, (6, 6))])
    T = W.rng(43, 3).uniform(0.5, 1.0, p.image_shape())
    L0, g, _, _ = O.grad(p, P2, T)
    assert g.shape == P2.shape and np.abs(g[1]).max() > 0
    h = 1e-6
    for k in [(0, 1, 2), (0, 3, 3), (1, 2, 2), (1, 3, 4), (1, 4, 1)]:
        E = np.zeros_like(P2)
        E[k] = h
        Lp = O.loss(O.forward(p, P2 + E)[0], T)[0]
        Lm = O.loss(O.forward(p, P2 - E)[0], T)[0]
        assert abs((Lp - Lm) / (2 * h) - g[k]) <= 2e-5 * np.abs(g).max(), (k, (Lp - Lm) / (2 * h), g[k])
