"""Closed-form test surfaces shared by the oracle pins and the GPU tests."""
import numpy as np

import oracle as O
from paper_2302_12031_amd import workloads as W


def valley_heights(c0=2.0, kappa=0.5, n_u=8, n_v=4, p=3, r=5.0):
    """Control heights that make the degree-p B-spline exactly h(x, y) = c0 + kappa x^2: with X linear
    (X = (2u - 1) r), h is a quadratic g(u) = A + B u + C u^2 of u, reproduced by the control points given by its
    polar form at the knots: c_i = A + B s1_i / p + C s2_i / binom(p, 2), s1, s2 the first and second elementary
    symmetric functions of the knots u_{i+1} .. u_{i+p} (Marsden's identity)."""
    A, B, C = c0 + kappa * r * r, -4.0 * kappa * r * r, 4.0 * kappa * r * r
    U = O.knots(p, n_u)
    cps = []
    for i in range(n_u):
        k = U[i + 1:i + p + 1]
        s1 = k.sum()
        s2 = sum(k[a] * k[b] for a in range(p) for b in range(a + 1, p))
        cps.append(A + B * s1 / p + C * s2 / (p * (p - 1) / 2))
    return np.repeat(np.array(cps)[:, None], n_v, axis=1)


def valley_problem(strata=64, seed=4, det=32, R=200.0):
    """A point source off axis with a wide cone (70 degrees) under the valley: many rays cross the exit face,
    leave the glass and meet the rising wall again before the aperture edge."""
    return W.Problem(lens=W.Lens(n_u=8, n_v=4),
                     source=W.Source(kind=W.POINT, grid_u=strata, grid_v=strata, jitter=1, pos=(-4.0, 0.0, -1.0),
                                     half_angle=np.deg2rad(70.0), seed=seed),
                     detector=W.Detector(n_x=det, n_y=det, R_x=R, R_y=R, z_screen=40.0))


def valley_roots(o, d, c0=2.0, kappa=0.5):
    """Both roots t1 <= t2 of f(t) = c0 + kappa (o_x + t d_x)^2 - o_z - t d_z (NaN where none are real)."""
    a = kappa * d[:, 0] ** 2
    b = 2.0 * kappa * d[:, 0] * o[:, 0] - d[:, 2]
    c = c0 + kappa * o[:, 0] ** 2 - o[:, 2]
    disc = b * b - 4 * a * c
    ok = (disc > 0) & (a > 0)
    sq = np.sqrt(np.where(ok, disc, 0.0))
    with np.errstate(invalid="ignore", divide="ignore"):
        t1 = np.where(ok, (-b - sq) / (2 * a), np.nan)
        t2 = np.where(ok, (-b + sq) / (2 * a), np.nan)
    return t1, t2


def aperture_exit(o, d, r=5.0):
    """Ray parameter where o + t d leaves the prism over [-r, r]^2."""
    with np.errstate(divide="ignore", invalid="ignore"):
        tx = np.where(d[:, 0] > 0, (r - o[:, 0]) / d[:, 0], np.where(d[:, 0] < 0, (-r - o[:, 0]) / d[:, 0], np.inf))
        ty = np.where(d[:, 1] > 0, (r - o[:, 1]) / d[:, 1], np.where(d[:, 1] < 0, (-r - o[:, 1]) / d[:, 1], np.inf))
    return np.minimum(tx, ty)


def glass_rays(p, ids):
    """Origins on the entry face and directions inside the glass of point-source rays, rebuilt from the oracle's
    samples with the refraction pinned by the oracle tests (sec. 2.2.1)."""
    Sm = O.samples(p, ids)
    ca = 1.0 - (1.0 - np.cos(p.source.half_angle)) * Sm[:, 1]
    sa = np.sqrt(1.0 - ca ** 2)
    d0 = np.stack([np.cos(Sm[:, 0]) * sa, np.sin(Sm[:, 0]) * sa, ca], 1)
    t0 = (p.lens.z_in - p.source.pos[2]) / d0[:, 2]
    o = np.stack([Sm[:, 2] + t0 * d0[:, 0], Sm[:, 3] + t0 * d0[:, 1], np.full(len(ids), p.lens.z_in)], 1)
    d = np.array([O.refract(x, [0.0, 0.0, 1.0], 1.0 / p.lens.n_lens) for x in d0])
    return o, d
