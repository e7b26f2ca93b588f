"""Problem descriptions and seeded synthetic inputs.

This module holds data only: the problem layout (lens, source, detector, options) and the seeded
generators of control-point heights and target images.  It contains none of the tracing arithmetic and is
shared by the HIP binding, the oracle-based tests and the benchmark.

Geometry common to every workload (the paper's plano-freeform lens, sec. 2.1): flat entry face z_in = 0,
aperture 10 mm x 10 mm (r_x = r_y = 5), refractive index 1.5, bicubic B-spline exit face whose control
heights are 2.0 mm + U[-0.2, 0.2] mm.  Reconstruction filter nu = 3, alpha = 1 per pixel^2, Schlick on.
Targets are Gaussian mixtures evaluated at pixel centres (the paper's target images are not available).
"""
from dataclasses import dataclass, field, replace
from typing import List, Tuple

import numpy as np

COLLIMATED, POINT, POINT_GRID = 0, 1, 2


@dataclass
class Lens:
    n_lens: float = 1.5
    r_x: float = 5.0
    r_y: float = 5.0
    z_in: float = 0.0
    delta_min: float = 0.0
    p: int = 3
    q: int = 3
    n_u: int = 8
    n_v: int = 8
    entry_freeform: int = 0   # 1: the entry face is a second B-spline; its net follows the exit net in Pz


@dataclass
class Source:
    kind: int = COLLIMATED
    grid_u: int = 256          # collimated: rays per axis; point: strata in theta
    grid_v: int = 256          # collimated: rays per axis; point: strata in a
    jitter: int = 0
    pos: Tuple[float, float, float] = (0.0, 0.0, -5.0)
    half_angle: float = 0.0
    emit_nx: int = 1
    emit_ny: int = 1
    emit_wx: float = 0.0
    emit_wy: float = 0.0
    seed: int = 0


@dataclass
class Detector:
    n_x: int = 64
    n_y: int = 64
    R_x: float = 20.0
    R_y: float = 20.0
    z_screen: float = 50.0
    alpha: float = 1.0
    nu_x: int = 3
    nu_y: int = 3
    ghost: int = 0
    filter: int = 0           # 0: Gaussian reconstruction filter, 1: box (the landing pixel's indicator)


@dataclass
class Options:
    fresnel: int = 1
    newton_max_iter: int = 8
    mesh_u: int = 0           # 0: exact intersection; >= 1: triangle mesh of sec. 2.2.2, rectangles per span
    mesh_v: int = 0
    loss: int = 0             # 0: the paper's RMS loss of the normalised images (sec. 2.5); 1: sum of squares


@dataclass
class Problem:
    lens: Lens = field(default_factory=Lens)
    source: Source = field(default_factory=Source)
    detector: Detector = field(default_factory=Detector)
    options: Options = field(default_factory=Options)

    def num_rays(self) -> int:
        s = self.source
        n = s.grid_u * s.grid_v
        if s.kind == POINT_GRID:
            n *= s.emit_nx * s.emit_ny
        return n

    def image_shape(self) -> Tuple[int, int]:
        d = self.detector
        if d.ghost:
            return d.n_x + d.nu_x - 1, d.n_y + d.nu_y - 1
        return d.n_x, d.n_y

    def cp_shape(self) -> Tuple[int, ...]:
        """Shape of the design's control heights: the exit net, or (exit, entry) with a freeform entry."""
        L = self.lens
        return (2, L.n_u, L.n_v) if L.entry_freeform else (L.n_u, L.n_v)


@dataclass
class Workload:
    name: str
    problems: List[Problem]
    Pz: List[np.ndarray]          # float64 [n_u, n_v] per design
    targets: List[np.ndarray]     # float64 [n_x, n_y] per design, sum 1

    @property
    def num_rays(self) -> int:
        return sum(p.num_rays() for p in self.problems)


# --------------------------------------------------------------------------------------------------
# Seeded generators (numpy PCG64 streams keyed by (seed, stream))
# --------------------------------------------------------------------------------------------------
STREAM_PZ, STREAM_TARGET, STREAM_FD, STREAM_BATCH = 0, 1, 3, 4


def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(stream)])


def single(a) -> np.ndarray:
    """The values rounded to single precision (returned as float64): the device path takes its inputs in
    single precision, so every generated input is representable there and both the device and the
    double-precision checks see exactly the same lens and target."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def random_heights(n_u: int, n_v: int, seed: int, base: float = 2.0, spread: float = 0.2) -> np.ndarray:
    return single(base + rng(seed, STREAM_PZ).uniform(-spread, spread, size=(n_u, n_v)))


def _pixel_centres(n: int, R: float) -> np.ndarray:
    w = 2.0 * R / n
    return (np.arange(n) + 0.5) * w - R


def gaussian_mixture(n_x, n_y, R_x, R_y, n_comp, g: np.random.Generator) -> np.ndarray:
    cx, cy = _pixel_centres(n_x, R_x)[:, None], _pixel_centres(n_y, R_y)[None, :]
    img = np.zeros((n_x, n_y))
    for _ in range(n_comp):
        mx, my = g.uniform(-0.5 * R_x, 0.5 * R_x), g.uniform(-0.5 * R_y, 0.5 * R_y)
        sx, sy = g.uniform(0.1 * R_x, 0.3 * R_x), g.uniform(0.1 * R_y, 0.3 * R_y)
        amp = g.uniform(0.5, 1.0)
        img += amp * np.exp(-0.5 * ((cx - mx) / sx) ** 2 - 0.5 * ((cy - my) / sy) ** 2)
    return img


def _blur(img: np.ndarray, sigma_px: float) -> np.ndarray:
    r = int(np.ceil(3 * sigma_px))
    k = np.exp(-0.5 * (np.arange(-r, r + 1) / sigma_px) ** 2)
    k /= k.sum()
    out = np.apply_along_axis(lambda a: np.convolve(a, k, mode="same"), 0, img)
    return np.apply_along_axis(lambda a: np.convolve(a, k, mode="same"), 1, out)


def target_mixture(prob: Problem, seed: int, n_min=3, n_max=3, rectangle=False) -> np.ndarray:
    g = rng(seed, STREAM_TARGET)
    nx, ny = prob.image_shape()
    d = prob.detector
    n_comp = int(g.integers(n_min, n_max + 1))
    img = gaussian_mixture(nx, ny, d.R_x, d.R_y, n_comp, g)
    if rectangle:
        cx, cy = _pixel_centres(nx, d.R_x)[:, None], _pixel_centres(ny, d.R_y)[None, :]
        xs = np.sort(g.uniform(-0.6 * d.R_x, 0.6 * d.R_x, 2))
        ys = np.sort(g.uniform(-0.6 * d.R_y, 0.6 * d.R_y, 2))
        img = img / img.max() + 0.5 * ((cx >= xs[0]) & (cx <= xs[1]) & (cy >= ys[0]) & (cy <= ys[1]))
        img = _blur(img, 1.0)
    return single(img / img.sum())


# --------------------------------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------------------------------
def collimated_problem(rays_side, cps_side, det_side, jitter=0, seed=0, R=20.0, z=50.0) -> Problem:
    return Problem(
        lens=Lens(n_u=cps_side, n_v=cps_side),
        source=Source(kind=COLLIMATED, grid_u=rays_side, grid_v=rays_side, jitter=jitter, seed=seed),
        detector=Detector(n_x=det_side, n_y=det_side, R_x=R, R_y=R, z_screen=z),
    )


def point_problem(strata_side, cps_side, det_side, seed=0, R=80.0, z=100.0, half_angle_deg=30.0,
                  emitters=1, emit_w=0.0, jitter=1) -> Problem:
    kind = POINT if emitters == 1 else POINT_GRID
    return Problem(
        lens=Lens(n_u=cps_side, n_v=cps_side),
        source=Source(kind=kind, grid_u=strata_side, grid_v=strata_side, jitter=jitter, pos=(0.0, 0.0, -5.0),
                      half_angle=np.deg2rad(half_angle_deg), emit_nx=emitters, emit_ny=emitters,
                      emit_wx=emit_w, emit_wy=emit_w, seed=seed),
        detector=Detector(n_x=det_side, n_y=det_side, R_x=R, R_y=R, z_screen=z),
    )


def c1() -> Workload:
    """Collimated 256x256 cell-centred rays, 8x8 control points, 64x64 detector at 50 mm, 3 Gaussians."""
    seed = 0
    p = collimated_problem(256, 8, 64, jitter=0, seed=seed)
    return Workload("collimated-256x256-cp8x8-det64", [p], [random_heights(8, 8, seed)],
                    [target_mixture(p, seed, 3, 3)])


def c2(rays_side=1024) -> Workload:
    """Collimated 1024x1024 jittered rays, 16x16 control points, 128x128 detector, 5-8 Gaussians plus a
    smoothed rectangle."""
    seed = 1
    p = collimated_problem(rays_side, 16, 128, jitter=1, seed=seed)
    return Workload(f"collimated-{rays_side}x{rays_side}-cp16x16-det128", [p], [random_heights(16, 16, seed)],
                    [target_mixture(p, seed, 5, 8, rectangle=True)])


def c3(strata_side=2048) -> Workload:
    """Point source 5 mm before the entry face, 30 degree cone, stratified strata_side^2 rays, 32x32
    control points, 256x256 detector at 100 mm."""
    seed = 2
    p = point_problem(strata_side, 32, 256, seed=seed)
    return Workload(f"point-{strata_side}x{strata_side}-cp32x32-det256", [p], [random_heights(32, 32, seed)],
                    [target_mixture(p, seed, 3, 8)])


def c4(strata_side=1024, emitters=9) -> Workload:
    """Extended 1 mm x 1 mm source as a 9x9 grid of point sources, strata_side^2 rays each, 32x32 control
    points, 256x256 detector at 100 mm."""
    seed = 3
    p = point_problem(strata_side, 32, 256, seed=seed, emitters=emitters, emit_w=1.0)
    return Workload(f"grid{emitters}x{emitters}-{strata_side}x{strata_side}-cp32x32-det256", [p],
                    [random_heights(32, 32, seed)], [target_mixture(p, seed, 3, 8)])


def c5(n_designs=64, ray_scale=1.0) -> Workload:
    """64 independent designs of uneven size: control grids from {8,16,24,32}^2, 2^U[18,23] rays each,
    detectors from 64^2 to 256^2, collimated or point sources with probability 1/2."""
    seed = 4
    g = rng(seed, STREAM_BATCH)
    probs, Pz, T = [], [], []
    for d in range(n_designs):
        cps = int(g.choice([8, 16, 24, 32]))
        n = 2.0 ** g.uniform(18, 23) * ray_scale
        side = max(8, int(round(np.sqrt(n))))
        det = int(g.choice(np.arange(64, 257, 32)))
        if g.uniform() < 0.5:
            p = collimated_problem(side, cps, det, jitter=1, seed=1000 + d)
        else:
            p = point_problem(side, cps, det, seed=1000 + d)
        probs.append(p)
        Pz.append(random_heights(cps, cps, 1000 + d))
        T.append(target_mixture(p, 1000 + d, 3, 8))
    return Workload(f"batch{n_designs}-uneven", probs, Pz, T)


def circular_tophat(prob: Problem, radius: float) -> np.ndarray:
    """Uniform disc of the given radius (mm) centred on the screen, sampled at pixel centres, sum 1."""
    nx, ny = prob.image_shape()
    d = prob.detector
    cx, cy = _pixel_centres(nx, d.R_x)[:, None], _pixel_centres(ny, d.R_y)[None, :]
    img = ((cx ** 2 + cy ** 2) <= radius ** 2).astype(np.float64)
    return single(img / img.sum())


def tophat(rays_side=512, cps_side=16, det_side=64) -> Workload:
    """Design case of sec. 3.2 without a network: a collimated bundle shaped into a circular top hat.  The
    lens starts flat (theta = 0 in the range reparametrisation of sec. 2.4.1, heights in [1.8, 2.2] mm); the
    screen (R = 8 mm at 30 mm) first shows the 10 x 10 mm square of the aperture, the target is a disc of
    radius 4 mm.  Ray count, control net and screen are synthetic (the paper's are in its supplement)."""
    p = collimated_problem(rays_side, cps_side, det_side, jitter=0, seed=5, R=8.0, z=30.0)
    lo, span = tophat_range(p)
    return Workload(f"tophat-{rays_side}x{rays_side}-cp{cps_side}x{cps_side}-det{det_side}", [p],
                    [lo + 0.5 * span], [circular_tophat(p, 4.0)])


def tophat_range(prob: Problem, z_min: float = 1.8, z_max: float = 2.2):
    """(lo, span) of the range reparametrisation, [n_u][n_v] each, no offset function."""
    shape = prob.cp_shape()
    return np.full(shape, z_min), np.full(shape, z_max - z_min)


WORKLOADS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5}


def with_rays(prob: Problem, side: int) -> Problem:
    """Same geometry with a different number of rays (or strata) per axis."""
    return replace(prob, source=replace(prob.source, grid_u=side, grid_v=side))


def with_mesh(wl: Workload, m: int) -> Workload:
    """The same workload traced on the triangle mesh of sec. 2.2.2 (m x m rectangles per knot span product)
    instead of the exact surface."""
    probs = [replace(p, options=replace(p.options, mesh_u=m, mesh_v=m)) for p in wl.problems]
    return Workload(f"{wl.name}-mesh{m}", probs, wl.Pz, wl.targets)


def with_entry_freeform(wl: Workload, seed: int = 11, base: float = 0.5, spread: float = 0.05) -> Workload:
    """The same workload with a freeform entry face: entry heights z_in + base +- spread (seeded), the exit
    net unchanged (the paper's proposal of optimising both faces).  The default spread gives entry slopes of
    at most ~0.3 on the 32 x 32 net, a gently curved face."""
    probs, Pz = [], []
    for d, (p, P) in enumerate(zip(wl.problems, wl.Pz)):
        probs.append(replace(p, lens=replace(p.lens, entry_freeform=1)))
        entry = single(p.lens.z_in + base + rng(seed + d, STREAM_PZ).uniform(-spread, spread, size=P.shape))
        Pz.append(np.stack([P, entry]))
    return Workload(f"{wl.name}-twofaces", probs, Pz, wl.targets)
