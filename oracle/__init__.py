"""FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import this
package.  It loads ``liboracle`` (built from ``ffrt_oracle.cpp`` by :func:`build`) and exposes numpy-level
wrappers.  It does not import the HIP package: a problem is any object with the attribute layout of
``Problem`` (lens / source / detector / options groups), read here by name.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ffrt_oracle.cpp")
_LIB = os.path.join(_HERE, "libffrt_oracle.so")

HIT, MISS_ENTRY, SIDE_WALL, TIR, OFF_SCREEN = 0, 1, 2, 3, 4


def build():
    """Compile the oracle with the host C++ compiler (no GPU code)."""
    # built beside the library and renamed over it, so a process that has the old one loaded keeps it intact
    tmp = _LIB + f".tmp{os.getpid()}"
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, _LIB)


class OrcProblem(ctypes.Structure):
    _fields_ = [
        ("n_lens", ctypes.c_double), ("r_x", ctypes.c_double), ("r_y", ctypes.c_double),
        ("z_in", ctypes.c_double), ("delta_min", ctypes.c_double),
        ("p", ctypes.c_int32), ("q", ctypes.c_int32), ("n_u", ctypes.c_int32), ("n_v", ctypes.c_int32),
        ("kind", ctypes.c_int32), ("grid_u", ctypes.c_int32), ("grid_v", ctypes.c_int32),
        ("jitter", ctypes.c_int32),
        ("pos_x", ctypes.c_double), ("pos_y", ctypes.c_double), ("pos_z", ctypes.c_double),
        ("half_angle", ctypes.c_double),
        ("emit_nx", ctypes.c_int32), ("emit_ny", ctypes.c_int32),
        ("emit_wx", ctypes.c_double), ("emit_wy", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("n_x", ctypes.c_int32), ("n_y", ctypes.c_int32),
        ("R_x", ctypes.c_double), ("R_y", ctypes.c_double), ("z_screen", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("nu_x", ctypes.c_int32), ("nu_y", ctypes.c_int32), ("ghost", ctypes.c_int32),
        ("fresnel", ctypes.c_int32), ("mesh_u", ctypes.c_int32), ("mesh_v", ctypes.c_int32),
        ("filter", ctypes.c_int32), ("entry_freeform", ctypes.c_int32), ("loss", ctypes.c_int32),
    ]


class OrcStats(ctypes.Structure):
    _fields_ = [("flux_on_screen", ctypes.c_double)] + [
        (n, ctypes.c_int64) for n in
        ("n_rays", "n_hit", "n_miss_entry", "n_side_wall", "n_tir", "n_off_screen", "n_marginal")
    ]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        dp, i64p = P(ctypes.c_double), P(ctypes.c_int64)
        pp = P(OrcProblem)
        sig = {
            "orc_num_rays": (ctypes.c_int64, [pp]),
            "orc_image_size": (None, [pp, P(ctypes.c_int32), P(ctypes.c_int32)]),
            "orc_knots": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, dp]),
            "orc_basis_all": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, dp]),
            "orc_surface": (ctypes.c_int, [pp, dp, ctypes.c_double, ctypes.c_double, dp]),
            "orc_samples": (ctypes.c_int, [pp, i64p, ctypes.c_int64, dp]),
            "orc_refract": (ctypes.c_int, [dp, dp, ctypes.c_double, dp]),
            "orc_schlick": (ctypes.c_double, [ctypes.c_double, ctypes.c_double]),
            "orc_splat_one": (ctypes.c_int, [pp, ctypes.c_double, ctypes.c_double, dp]),
            "orc_trace_rays": (ctypes.c_int, [pp, dp, i64p, ctypes.c_int64, dp]),
            "orc_forward": (ctypes.c_int, [pp, dp, dp, P(OrcStats), dp, ctypes.c_int32]),
            "orc_loss": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, dp, dp, dp, dp]),
            "orc_landing_gain": (ctypes.c_int, [pp, dp, i64p, ctypes.c_int64, dp]),
            "orc_marginal_rays": (ctypes.c_int, [pp, dp, ctypes.c_int64, i64p, dp, i64p, ctypes.c_int32]),
            "orc_loss_kind": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, dp, dp, dp, dp]),
            "orc_grad": (ctypes.c_int, [pp, dp, dp, dp, dp, dp, dp, ctypes.c_int32]),
            "orc_grad_split": (ctypes.c_int, [pp, dp, dp, ctypes.c_double, dp, dp, dp, ctypes.c_int32]),
            "orc_jvp": (ctypes.c_int, [pp, dp, dp, dp, ctypes.c_int32]),
            "orc_adam": (ctypes.c_int, [ctypes.c_int64, dp, dp, dp, dp, ctypes.c_int64, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double]),
            "orc_rng": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def to_struct(prob):
    """Convert a problem description (grouped attributes) to the oracle's flat struct."""
    L, S, D, O = prob.lens, prob.source, prob.detector, prob.options
    s = OrcProblem()
    s.n_lens, s.r_x, s.r_y, s.z_in, s.delta_min = L.n_lens, L.r_x, L.r_y, L.z_in, L.delta_min
    s.p, s.q, s.n_u, s.n_v = L.p, L.q, L.n_u, L.n_v
    s.kind, s.grid_u, s.grid_v, s.jitter = S.kind, S.grid_u, S.grid_v, S.jitter
    s.pos_x, s.pos_y, s.pos_z = S.pos
    s.half_angle = S.half_angle
    s.emit_nx, s.emit_ny, s.emit_wx, s.emit_wy = S.emit_nx, S.emit_ny, S.emit_wx, S.emit_wy
    s.seed = S.seed
    s.n_x, s.n_y, s.R_x, s.R_y = D.n_x, D.n_y, D.R_x, D.R_y
    s.z_screen, s.alpha, s.nu_x, s.nu_y, s.ghost = D.z_screen, D.alpha, D.nu_x, D.nu_y, D.ghost
    s.fresnel = O.fresnel
    s.mesh_u, s.mesh_v = getattr(O, "mesh_u", 0), getattr(O, "mesh_v", 0)
    s.filter = getattr(D, "filter", 0)
    s.entry_freeform = getattr(L, "entry_freeform", 0)
    s.loss = getattr(O, "loss", 0)
    return s


def num_rays(prob):
    s = to_struct(prob)
    n = lib().orc_num_rays(ctypes.byref(s))
    if n < 0:
        raise ValueError("invalid problem")
    return n


def image_size(prob):
    s = to_struct(prob)
    nx, ny = ctypes.c_int32(), ctypes.c_int32()
    lib().orc_image_size(ctypes.byref(s), ctypes.byref(nx), ctypes.byref(ny))
    return nx.value, ny.value


def knots(p, n):
    U = np.zeros(n + p + 1)
    assert lib().orc_knots(p, n, _dp(U)) == 0
    return U


def basis_all(p, n, u, der=0):
    out = np.zeros(n)
    assert lib().orc_basis_all(p, n, float(u), der, _dp(out)) == 0
    return out


def surface(prob, Pz, x, y):
    s = to_struct(prob)
    P = _f64(Pz).ravel()
    out = np.zeros(6)
    assert lib().orc_surface(ctypes.byref(s), _dp(P), float(x), float(y), _dp(out)) == 0
    return out


def samples(prob, ids):
    s = to_struct(prob)
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    out = np.zeros((len(ids), 4))
    assert lib().orc_samples(ctypes.byref(s), ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                             len(ids), _dp(out)) == 0
    return out


def refract(d, nrm, eta):
    d, nrm = _f64(d), _f64(nrm)
    out = np.zeros(3)
    tir = lib().orc_refract(_dp(d), _dp(nrm), float(eta), _dp(out))
    return None if tir else out


def schlick(c, n_lens):
    return lib().orc_schlick(float(c), float(n_lens))


def splat_one(prob, X, Y):
    s = to_struct(prob)
    nx, ny = image_size(prob)
    img = np.zeros((nx, ny))
    assert lib().orc_splat_one(ctypes.byref(s), float(X), float(Y), _dp(img)) == 0
    return img


def trace_rays(prob, Pz, ids):
    """Per-ray {status, X, Y, w, u, v, t, marginal} as an (n, 8) array."""
    s = to_struct(prob)
    P = _f64(Pz).ravel()
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    out = np.zeros((len(ids), 8))
    assert lib().orc_trace_rays(ctypes.byref(s), _dp(P), ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                len(ids), _dp(out)) == 0
    return out


def landing_gain(prob, Pz, ids):
    """Per-ray landing displacement (mm) per radian of rotation of the ray inside the glass (0: no landing)."""
    s = to_struct(prob)
    P = _f64(Pz).ravel()
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    out = np.zeros(len(ids))
    assert lib().orc_landing_gain(ctypes.byref(s), _dp(P), ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  len(ids), _dp(out)) == 0
    return out


def marginal_rays(prob, Pz, threads=0):
    """Ids of the rays whose discrete state is within rounding distance of flipping, and where each lands or
    would land on the other side of its decision ((n, 2), NaN where nowhere on the screen plane)."""
    s = to_struct(prob)
    P = _f64(Pz).ravel()
    n = ctypes.c_int64()
    i64 = ctypes.POINTER(ctypes.c_int64)
    assert lib().orc_marginal_rays(ctypes.byref(s), _dp(P), 0, None, None, ctypes.byref(n), threads) == 0
    ids = np.zeros(n.value, np.int64)
    xy = np.zeros((n.value, 2))
    assert lib().orc_marginal_rays(ctypes.byref(s), _dp(P), n.value, ids.ctypes.data_as(i64), _dp(xy),
                                   ctypes.byref(n), threads) == 0
    return ids, xy


def forward(prob, Pz, threads=0, with_mask=False):
    """Irradiance image (n_x, n_y), stats dict, and (optionally) the marginal-ray pixel mask."""
    s = to_struct(prob)
    P = _f64(Pz).ravel()
    nx, ny = image_size(prob)
    img = np.zeros((nx, ny))
    st = OrcStats()
    mask = np.zeros((nx, ny)) if with_mask else None
    rc = lib().orc_forward(ctypes.byref(s), _dp(P), _dp(img), ctypes.byref(st),
                           _dp(mask) if with_mask else None, threads)
    if rc:
        raise RuntimeError(f"orc_forward failed: {rc}")
    if with_mask:
        return img, st.as_dict(), mask.astype(bool)
    return img, st.as_dict()


def loss(irr, target, kind=0):
    """Loss of sec. 2.5 (kind 0, RMS) or its sum of squares (kind 1), and dL/dI."""
    irr, target = _f64(irr), _f64(target)
    nx, ny = irr.shape
    L = ctypes.c_double()
    g = np.zeros_like(irr)
    rc = lib().orc_loss_kind(kind, nx, ny, _dp(irr), _dp(target), ctypes.byref(L), _dp(g))
    if rc:
        raise RuntimeError(f"orc_loss failed: {rc}")
    return L.value, g


def grad(prob, Pz, target, threads=0):
    """(loss, dL/dP [n_u, n_v], irradiance, dL/dI)."""
    s = to_struct(prob)
    P = _f64(Pz)
    T = _f64(target)
    nx, ny = image_size(prob)
    g = np.zeros(P.shape)
    irr = np.zeros((nx, ny))
    G = np.zeros((nx, ny))
    L = ctypes.c_double()
    rc = lib().orc_grad(ctypes.byref(s), _dp(P), _dp(T), ctypes.byref(L), _dp(g), _dp(irr), _dp(G), threads)
    if rc:
        raise RuntimeError(f"orc_grad failed: {rc}")
    return L.value, g, irr, G


def grad_split(prob, Pz, target, k_min, threads=0):
    """(loss, dL/dP from well-conditioned rays, dL/dP from rays with |Snell discriminant| < k_min)."""
    s = to_struct(prob)
    P, T = _f64(Pz), _f64(target)
    g = np.zeros(P.shape)
    gi = np.zeros(P.shape)
    L = ctypes.c_double()
    rc = lib().orc_grad_split(ctypes.byref(s), _dp(P), _dp(T), float(k_min), ctypes.byref(L), _dp(g),
                              _dp(gi), threads)
    if rc:
        raise RuntimeError(f"orc_grad_split failed: {rc}")
    return L.value, g, gi


def jvp(prob, Pz, v, threads=0):
    s = to_struct(prob)
    P, V = _f64(Pz), _f64(v)
    nx, ny = image_size(prob)
    dI = np.zeros((nx, ny))
    assert lib().orc_jvp(ctypes.byref(s), _dp(P), _dp(V), _dp(dI), threads) == 0
    return dI


def adam(P, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place on float64 arrays (t = new step count)."""
    for a in (P, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    assert lib().orc_adam(P.size, _dp(P), _dp(g), _dp(m), _dp(v), t, lr, beta1, beta2, eps) == 0


def rng(seed, stream, index):
    return lib().orc_rng(seed, stream, index)


# ---------------------------------------------------------------------------------------------------
# Range reparametrisation of the control heights (sec. 2.4.1, eq. of the output correction): each control
# height is z_min (+ an offset f(P^x, P^y)) + (y + 1)(z_max - z_min) / 2 with y = tanh(theta).  Here lo holds
# z_min (+ f) and span = z_max - z_min, per control point.
# ---------------------------------------------------------------------------------------------------
def reparam(theta, lo, span):
    theta, lo, span = (np.asarray(a, dtype=np.float64) for a in (theta, lo, span))
    return lo + 0.5 * (np.tanh(theta) + 1.0) * span


def reparam_grad(theta, span, dLdP):
    """dL/dtheta from dL/dP: d tanh(theta)/d theta = 1 / cosh^2(theta)."""
    theta, span, dLdP = (np.asarray(a, dtype=np.float64) for a in (theta, span, dLdP))
    return dLdP * 0.5 * span / np.cosh(theta) ** 2


def control_xy(prob):
    """(x, y) of every control point, [n_u][n_v] each: the Greville abscissae u*_i = (u_{i+1} + ... +
    u_{i+p}) / p of the clamped knots (sec. 2.1.1, eq. of the nodal representation) mapped by
    X = (2u - 1) r_x, Y = (2v - 1) r_y."""
    L = prob.lens
    Uu, Uv = knots(L.p, L.n_u), knots(L.q, L.n_v)
    gu = np.array([Uu[i + 1:i + L.p + 1].mean() for i in range(L.n_u)])
    gv = np.array([Uv[j + 1:j + L.q + 1].mean() for j in range(L.n_v)])
    x = np.repeat(((2.0 * gu - 1.0) * L.r_x)[:, None], L.n_v, axis=1)
    y = np.repeat(((2.0 * gv - 1.0) * L.r_y)[None, :], L.n_u, axis=0)
    return x, y


# ---------------------------------------------------------------------------------------------------
# Dense control-point generator (sec. 2.4, the fully connected architecture): a multi-layer perceptron with
# the trivial input 1 and three fully connected tanh layers of the control-net size K = n_u n_v, whose output
# passes through the output correction above.  The parameters of one design are (w1, b1, W2, b2, W3, b3) with
# w1, b1, b2, b3 of length K and W2, W3 of shape K x K acting as z = W h + b (row i: inputs of neuron i).
# Control points are indexed row-major over the net, k = i n_v + j, as the control heights are.
# ---------------------------------------------------------------------------------------------------
def mlp_forward(params, lo, span):
    """Activations (h1, h2, y) and control heights P (length K) of one design's generator."""
    w1, b1, W2, b2, W3, b3 = (np.asarray(a, dtype=np.float64) for a in params)
    h1 = np.tanh(w1 * 1.0 + b1)          # the single input is the constant 1
    h2 = np.tanh(W2 @ h1 + b2)
    y = np.tanh(W3 @ h2 + b3)
    P = np.asarray(lo, np.float64) + 0.5 * (y + 1.0) * np.asarray(span, np.float64)
    return (h1, h2, y), P


def mlp_backward(params, acts, span, dLdP):
    """dL/d(w1, b1, W2, b2, W3, b3) from dL/dP by back-propagation through the output correction and the
    three layers (chain rule with d tanh(z)/dz = 1 - tanh(z)^2)."""
    w1, b1, W2, b2, W3, b3 = (np.asarray(a, dtype=np.float64) for a in params)
    h1, h2, y = acts
    dy = np.asarray(dLdP, np.float64) * 0.5 * np.asarray(span, np.float64)
    dz3 = dy * (1.0 - y * y)
    dW3, db3 = np.outer(dz3, h2), dz3
    dh2 = W3.T @ dz3
    dz2 = dh2 * (1.0 - h2 * h2)
    dW2, db2 = np.outer(dz2, h1), dz2
    dh1 = W2.T @ dz2
    dz1 = dh1 * (1.0 - h1 * h1)
    return dz1 * 1.0, dz1, dW2, db2, dW3, db3


# The sparse architecture of sec. 2.4: the two K x K layers connect control point (i, j) only to the control
# points (i + a - p, j + b - q), a in [0, 2p], b in [0, 2q], those whose basis functions share a knot span with
# its own (the connectivity of a (2p+1) x (2q+1) convolution), with a weight per connection W[c][k],
# c = a (2q + 1) + b, k = i n_v + j, and a bias per neuron.  Connections that leave the net do not exist.
def sparse_matrix(Wc, n_u, n_v, p, q):
    """The K x K matrix M with M[k, s] = W[c][k] for input s = connection c of neuron k, zero elsewhere."""
    Wc = np.asarray(Wc, np.float64)
    K = n_u * n_v
    M = np.zeros((K, K))
    for i in range(n_u):
        for j in range(n_v):
            for a in range(2 * p + 1):
                for b in range(2 * q + 1):
                    ii, jj = i + a - p, j + b - q
                    if 0 <= ii < n_u and 0 <= jj < n_v:
                        M[i * n_v + j, ii * n_v + jj] = Wc[a * (2 * q + 1) + b, i * n_v + j]
    return M


def sparse_mlp_forward(params, lo, span, n_u, n_v, p, q):
    """The sparse generator is the dense one with W2, W3 replaced by their K x K matrices."""
    w1, b1, W2, b2, W3, b3 = params
    return mlp_forward([w1, b1, sparse_matrix(W2, n_u, n_v, p, q), b2, sparse_matrix(W3, n_u, n_v, p, q), b3],
                       lo, span)


def sparse_mlp_backward(params, acts, span, dLdP, n_u, n_v, p, q):
    """Gradients of the sparse generator: the dense back-propagation through the K x K matrices, then the
    gradient of each stored connection weight read off its matrix entry (zero for connections that leave the
    net)."""
    w1, b1, W2, b2, W3, b3 = params
    dw1, db1, dM2, db2, dM3, db3 = mlp_backward(
        [w1, b1, sparse_matrix(W2, n_u, n_v, p, q), b2, sparse_matrix(W3, n_u, n_v, p, q), b3], acts, span, dLdP)
    C, K = (2 * p + 1) * (2 * q + 1), n_u * n_v
    dW2, dW3 = np.zeros((C, K)), np.zeros((C, K))
    for i in range(n_u):
        for j in range(n_v):
            for a in range(2 * p + 1):
                for b in range(2 * q + 1):
                    ii, jj = i + a - p, j + b - q
                    if 0 <= ii < n_u and 0 <= jj < n_v:
                        c, k, s = a * (2 * q + 1) + b, i * n_v + j, ii * n_v + jj
                        dW2[c, k], dW3[c, k] = dM2[k, s], dM3[k, s]
    return dw1, db1, dW2, db2, dW3, db3
