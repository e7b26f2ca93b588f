"""Shared helpers of the GPU-vs-oracle parity tests (tolerances stated here)."""
import numpy as np

# Irradiance: |I_gpu - I_64| <= 1e-4 * max(I_64[px], 0.01 * max I_64) at every pixel not touched by a
# marginal ray (a ray whose discrete state sits within rounding distance of flipping).
IRR_REL = 1e-4
IRR_FLOOR = 0.01
# Marginal rays (excluded through the mask) must stay rare: at most MAX_MARGINAL of all rays.
MAX_MARGINAL = 2e-5
# Gradient: ||g_gpu - g_64||_inf <= 1e-3 ||g_64||_inf, and |g_gpu - g_64| <= 1e-3 |g_64| on every component with
# |g_64| >= 0.01 ||g_64||_inf.
GRAD_REL = 1e-3
GRAD_FLOOR = 0.01


def irradiance_errors(I_gpu, I_64, mask=None, rel=IRR_REL):
    tol = rel * np.maximum(I_64, IRR_FLOOR * I_64.max())
    err = np.abs(I_gpu - I_64)
    ok = err <= tol
    if mask is not None:
        ok |= mask
    big = I_64 >= IRR_FLOOR * I_64.max()
    if mask is not None:
        big &= ~mask
    rel_big = (err[big] / I_64[big]).max() if big.any() else 0.0
    return ok, float((err / np.maximum(tol, 1e-300)).max()), float(rel_big)


def assert_irradiance(I_gpu, I_64, mask=None, max_masked_frac=0.05, what="", rel=IRR_REL):
    ok, worst, rel_big = irradiance_errors(I_gpu, I_64, mask, rel)
    n_mask = int(mask.sum()) if mask is not None else 0
    assert n_mask <= max_masked_frac * I_64.size + 9, f"{what}: {n_mask} masked pixels"
    bad = np.argwhere(~ok)
    assert ok.all(), (f"{what}: {len(bad)} pixels out of tolerance, first {bad[:5].tolist()}, "
                      f"worst err/tol {worst:.3g}, max rel on bright pixels {rel_big:.3g}")
    return worst, rel_big


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
# total internal reflection), which the double-precision re-trace gives the plano-freeform lens with the exact
# root.  The triangle-mesh and two-face kernels keep single-precision decisions there: for them the global
# bound is asserted and the per-component error reported.
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
