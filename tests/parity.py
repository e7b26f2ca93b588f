"""Shared helpers of the GPU-vs-oracle parity tests (tolerances stated here)."""
import numpy as np

# Irradiance: |I_gpu - I_64| <= 1e-4 * max(I_64[px], 0.01 * max I_64, 4 w_ray) at every pixel outside the
# filter windows of rays whose status differs between the two (flip_mask).  The floor keeps the bound off pixels
# set by a handful of rays, whose relative error has no meaning.  On the dense workloads 1 % of the peak is the
# weight of 12 to 21 rays (w_ray = 1/N, the weight a ray starts with); on sparse designs of the 64-design batch
# it falls to a fifth of one ray, so the floor is also at least the weight of IRR_FLOOR_RAYS rays.
IRR_REL = 1e-4
IRR_FLOOR = 0.01
IRR_FLOOR_RAYS = 4
# Marginal rays (excluded through the mask) must stay rare: at most MAX_MARGINAL of all rays.
MAX_MARGINAL = 2e-5
# Gradient: ||g_gpu - g_64||_inf <= 1e-3 ||g_64||_inf, and |g_gpu - g_64| <= 1e-3 |g_64| on every component with
# |g_64| >= 0.01 ||g_64||_inf.
GRAD_REL = 1e-3
GRAD_FLOOR = 0.01


def irradiance_errors(I_gpu, I_64, mask=None, rel=IRR_REL, w_ray=0.0):
    tol = rel * np.maximum(I_64, max(IRR_FLOOR * I_64.max(), IRR_FLOOR_RAYS * w_ray))
    err = np.abs(I_gpu - I_64)
    ok = err <= tol
    if mask is not None:
        ok |= mask
    big = I_64 >= IRR_FLOOR * I_64.max()
    if mask is not None:
        big &= ~mask
    rel_big = (err[big] / I_64[big]).max() if big.any() else 0.0
    return ok, float((err / np.maximum(tol, 1e-300)).max()), float(rel_big)


def assert_irradiance(I_gpu, I_64, mask=None, max_masked_frac=0.02, what="", rel=IRR_REL, w_ray=0.0):
    ok, worst, rel_big = irradiance_errors(I_gpu, I_64, mask, rel, w_ray)
    n_mask = int(mask.sum()) if mask is not None else 0
    assert n_mask <= max_masked_frac * I_64.size + 9, f"{what}: {n_mask} masked pixels"
    bad = np.argwhere(~ok)
    assert ok.all(), (f"{what}: {len(bad)} pixels out of tolerance, first {bad[:5].tolist()}, "
                      f"worst err/tol {worst:.3g}, max rel on bright pixels {rel_big:.3g}")
    return worst, rel_big


# Rays whose discrete state (hit, entry miss, side wall, TIR, off screen) differs between the device and the
# oracle: at most MAX_FLIPPED of all rays, and the pixels of their filter windows are excluded.
MAX_FLIPPED = 1e-6


def _mark_windows(mask, prob, xy):
    d = prob.detector
    nx, ny = mask.shape
    wx, wy = 2.0 * d.R_x / d.n_x, 2.0 * d.R_y / d.n_y
    Rxe, Rye = d.R_x + 0.5 * (nx - d.n_x) * wx, d.R_y + 0.5 * (ny - d.n_y) * wy
    hx, hy = (d.nu_x - 1) // 2, (d.nu_y - 1) // 2
    for X, Y in xy:
        if not (np.isfinite(X) and np.isfinite(Y)):
            continue
        i = min(max(int(np.floor((X + Rxe) / wx)), 0), nx - 1)
        j = min(max(int(np.floor((Y + Rye) / wy)), 0), ny - 1)
        mask[max(i - hx, 0):i + hx + 1, max(j - hy, 0):j + hy + 1] = True


def flip_mask(plan, design, P_dev, prob, Pz64, shape, what=""):
    """The pixels to exclude from the per-pixel comparison: those in the filter windows of rays whose status
    differs between the device and the oracle.  Only the oracle's marginal rays (a decision within rounding
    distance) are candidates; each is traced on the device and, where the statuses differ, its window is
    marked at the oracle's landing (or where it would land on the other side) and at the device's."""
    import oracle as O
    ids, xy = O.marginal_rays(prob, Pz64)
    mask = np.zeros(shape, bool)
    if len(ids) == 0:
        return mask, 0, 0
    gpu = plan.trace_rays(design, P_dev, ids).cpu().numpy()
    ref = O.trace_rays(prob, Pz64, ids)
    flip = gpu[:, 0] != ref[:, 0]
    n_rays = prob.num_rays()
    assert flip.sum() <= MAX_FLIPPED * n_rays + 5, f"{what}: {int(flip.sum())} rays change status"
    _mark_windows(mask, prob, xy[flip])
    landed = flip & (gpu[:, 0] == 0)
    _mark_windows(mask, prob, gpu[landed, 1:3].astype(np.float64))
    return mask, int(flip.sum()), len(ids)


def gradient_errors(g_gpu, g_64):
    """(max |error| / max |g|, the largest per-component relative error over components >= 1 % of max |g|,
    the number of such components)."""
    g_gpu, g_64 = np.asarray(g_gpu, np.float64).ravel(), np.asarray(g_64, np.float64).ravel()
    m = np.abs(g_64).max()
    err = np.abs(g_gpu - g_64)
    big = np.abs(g_64) >= GRAD_FLOOR * m
    per = (err[big] / np.abs(g_64[big])).max() if big.any() else 0.0
    return float(err.max() / m), float(per), int(big.sum())


# The per-component check needs exact decisions at the kinks of a ray's derivative (pixel and screen edges,
# total internal reflection, triangle edges), which the double-precision re-trace of the flagged rays gives every
# kernel group.  per_component=False is for comparisons of two device paths that round differently (a plane hit
# against a root search on a flat net), where only the global bound applies.
def assert_gradient(g_gpu, g_64, rel=GRAD_REL, what="", per_component=True):
    e, per, n = gradient_errors(g_gpu, g_64)
    assert e <= rel, f"{what}: gradient error {e:.3g} of max |g| (tolerance {rel})"
    if per_component:
        g_gpu, g_64 = np.asarray(g_gpu, np.float64).ravel(), np.asarray(g_64, np.float64).ravel()
        big = np.abs(g_64) >= GRAD_FLOOR * np.abs(g_64).max()
        bad = np.where(big & (np.abs(g_gpu - g_64) > rel * np.abs(g_64)))[0]
        assert per <= rel, (f"{what}: {len(bad)} of {n} components >= {GRAD_FLOOR} max |g| off by more than {rel} "
                            f"relative (worst {per:.3g}; first {bad[:6].tolist()})")
    return e
