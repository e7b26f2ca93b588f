"""Python binding of libffrt (ctypes): argument marshalling only.

Every step of the tracing path runs in the HIP kernels of ``libffrt.so``; PyTorch supplies device memory
and the current stream.  Importing this module does not load the library; the first call does, and it
raises if the library has not been built (there is no CPU fallback).
"""
import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libffrt.so")


class FfrtError(RuntimeError):
    pass


# ------------------------------------------------------------------------------------------------
# ctypes mirrors of include/ffrt.h
# ------------------------------------------------------------------------------------------------
class CLens(ctypes.Structure):
    _fields_ = [("n_lens", ctypes.c_double), ("r_x", ctypes.c_double), ("r_y", ctypes.c_double),
                ("z_in", ctypes.c_double), ("delta_min", ctypes.c_double),
                ("p", ctypes.c_int32), ("q", ctypes.c_int32), ("n_u", ctypes.c_int32), ("n_v", ctypes.c_int32),
                ("entry_freeform", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class CSource(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("grid_u", ctypes.c_int32), ("grid_v", ctypes.c_int32),
                ("jitter", ctypes.c_int32), ("pos", ctypes.c_double * 3), ("half_angle", ctypes.c_double),
                ("emit_nx", ctypes.c_int32), ("emit_ny", ctypes.c_int32),
                ("emit_wx", ctypes.c_double), ("emit_wy", ctypes.c_double), ("seed", ctypes.c_uint64)]


class CDetector(ctypes.Structure):
    _fields_ = [("n_x", ctypes.c_int32), ("n_y", ctypes.c_int32), ("R_x", ctypes.c_double),
                ("R_y", ctypes.c_double), ("z_screen", ctypes.c_double), ("alpha", ctypes.c_double),
                ("nu_x", ctypes.c_int32), ("nu_y", ctypes.c_int32), ("ghost", ctypes.c_int32),
                ("filter", ctypes.c_int32)]


class COptions(ctypes.Structure):
    _fields_ = [("fresnel", ctypes.c_int32), ("newton_max_iter", ctypes.c_int32), ("mesh_u", ctypes.c_int32),
                ("mesh_v", ctypes.c_int32), ("loss", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class CProblem(ctypes.Structure):
    _fields_ = [("lens", CLens), ("src", CSource), ("det", CDetector), ("opt", COptions)]


class CAdam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


STATS_FIELDS = ["flux_on_screen", "n_traced", "n_hit", "n_miss_entry", "n_side_wall", "n_tir", "n_off_screen",
                "n_newton_fail", "n_fp64_refined", "n_nonmonotone", "n_search_steps", "n_constraint_viol", "n_nan"]
STATS_DTYPE = np.dtype([(STATS_FIELDS[0], np.float32)] + [(f, np.uint32) for f in STATS_FIELDS[1:]])
STATS_BYTES = STATS_DTYPE.itemsize

MLP_DENSE, MLP_SPARSE = 0, 1

HEADER_FUNCTIONS = [
    "ffrt_plan_create", "ffrt_plan_destroy", "ffrt_plan_workspace_size", "ffrt_plan_set_workspace",
    "ffrt_plan_layout", "ffrt_plan_num_designs", "ffrt_plan_num_rays", "ffrt_forward", "ffrt_loss",
    "ffrt_loss_f64",
    "ffrt_adjoint", "ffrt_adam", "ffrt_step", "ffrt_graph_capture", "ffrt_graph_launch",
    "ffrt_plan_time_kernels", "ffrt_num_configs",
    "ffrt_config_name", "ffrt_plan_set_config", "ffrt_plan_get_config", "ffrt_plan_autotune",
    "ffrt_trace_rays", "ffrt_rng", "ffrt_status_string", "ffrt_last_error",
    "ffrt_reparam_apply", "ffrt_reparam_grad", "ffrt_step_reparam", "ffrt_graph_capture_reparam",
    "ffrt_plan_control_xy", "ffrt_mlp_layout", "ffrt_mlp_forward", "ffrt_mlp_backward", "ffrt_step_mlp",
    "ffrt_graph_capture_mlp", "ffrt_plan_time_mlp", "ffrt_forward_static", "ffrt_lds_atomic_rate",
]

_lib = None


def lib():
    """Load libffrt.so (raises FfrtError when it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FfrtError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        P = ctypes.POINTER
        sig = {
            "ffrt_plan_create": [P(CProblem), i32, P(vp)],
            "ffrt_plan_destroy": [vp],
            "ffrt_plan_workspace_size": [vp, P(ctypes.c_size_t)],
            "ffrt_plan_set_workspace": [vp, vp, ctypes.c_size_t],
            "ffrt_plan_layout": [vp, P(i64), P(i64)],
            "ffrt_plan_num_designs": [vp, P(i32)],
            "ffrt_plan_num_rays": [vp, P(i64)],
            "ffrt_forward": [vp, vp, vp, vp, vp],
            "ffrt_forward_static": [vp, vp, vp, vp, vp],
            "ffrt_loss": [vp, vp, vp, vp, vp, vp],
            "ffrt_loss_f64": [vp, vp, vp, vp, vp],
            "ffrt_adjoint": [vp, vp, vp, vp, vp],
            "ffrt_adam": [vp, vp, vp, vp, vp, vp, P(CAdam), vp],
            "ffrt_step": [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, P(CAdam), vp],
            "ffrt_graph_capture": [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, P(CAdam), vp],
            "ffrt_graph_launch": [vp, vp],
            "ffrt_plan_time_kernels": [vp, vp, vp, vp, vp, i32, P(ctypes.c_float), P(ctypes.c_float), vp],
            "ffrt_num_configs": [i32, P(i32)],
            "ffrt_config_name": [i32, i32, ctypes.c_char_p, i32],
            "ffrt_plan_set_config": [vp, i32, i32],
            "ffrt_plan_get_config": [vp, i32, P(i32)],
            "ffrt_plan_autotune": [vp, vp, vp, vp, vp, i32, vp],
            "ffrt_trace_rays": [vp, i32, vp, vp, i64, vp, vp],
            "ffrt_rng": [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, i64, vp, vp],
            "ffrt_lds_atomic_rate": [i32, i32, P(ctypes.c_double), vp],
            "ffrt_reparam_apply": [vp, vp, vp, vp, vp, vp],
            "ffrt_reparam_grad": [vp, vp, vp, vp, vp, vp],
            "ffrt_step_reparam": [vp] + [vp] * 13 + [P(CAdam), vp],
            "ffrt_graph_capture_reparam": [vp, i32] + [vp] * 13 + [P(CAdam), vp],
            "ffrt_plan_control_xy": [vp, vp, vp],
            "ffrt_mlp_layout": [vp, i32, P(i64)],
            "ffrt_mlp_forward": [vp, i32, vp, vp, vp, vp, vp, vp],
            "ffrt_mlp_backward": [vp, i32, vp, vp, vp, vp, vp, vp],
            "ffrt_step_mlp": [vp, i32] + [vp] * 14 + [P(CAdam), vp],
            "ffrt_graph_capture_mlp": [vp, i32, i32] + [vp] * 14 + [P(CAdam), vp],
            "ffrt_plan_time_mlp": [vp, i32] + [vp] * 9 + [P(CAdam), i32] + [P(ctypes.c_float)] * 3 + [vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.ffrt_status_string.argtypes = [ctypes.c_int]
        L.ffrt_status_string.restype = ctypes.c_char_p
        L.ffrt_last_error.argtypes = []
        L.ffrt_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        L = lib()
        raise FfrtError(f"{what}: {L.ffrt_status_string(rc).decode()} ({L.ffrt_last_error().decode()})")


def to_cproblem(p):
    """Problem (workloads.Problem layout) -> CProblem."""
    c = CProblem()
    L, S, D, O = p.lens, p.source, p.detector, p.options
    c.lens = CLens(L.n_lens, L.r_x, L.r_y, L.z_in, L.delta_min, L.p, L.q, L.n_u, L.n_v, L.entry_freeform, 0)
    c.src = CSource(S.kind, S.grid_u, S.grid_v, S.jitter, (ctypes.c_double * 3)(*S.pos), S.half_angle,
                    S.emit_nx, S.emit_ny, S.emit_wx, S.emit_wy, S.seed)
    c.det = CDetector(D.n_x, D.n_y, D.R_x, D.R_y, D.z_screen, D.alpha, D.nu_x, D.nu_y, D.ghost, D.filter)
    c.opt = COptions(O.fresnel, O.newton_max_iter, O.mesh_u, O.mesh_v, getattr(O, "loss", 0), 0)
    return c


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


@dataclass
class AdamHP:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8

    def c(self):
        return CAdam(self.lr, self.beta1, self.beta2, self.eps)


def create_plan_handle(problems):
    """Validate problems and create a host-only plan handle (no GPU needed)."""
    arr = (CProblem * len(problems))(*[to_cproblem(p) for p in problems])
    h = ctypes.c_void_p()
    _check(lib().ffrt_plan_create(arr, len(problems), ctypes.byref(h)), "ffrt_plan_create")
    return h


class Plan:
    """A batch of designs traced together; owns its device workspace (a torch tensor)."""

    def __init__(self, problems, device="cuda"):
        self.problems = list(problems)
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        L = lib()
        self.h = create_plan_handle(self.problems)
        nbytes = ctypes.c_size_t()
        _check(L.ffrt_plan_workspace_size(self.h, ctypes.byref(nbytes)), "workspace_size")
        self.ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        _check(L.ffrt_plan_set_workspace(self.h, ctypes.c_void_p(aligned), nbytes.value), "set_workspace")
        self.n_designs = len(self.problems)
        cp = (ctypes.c_int64 * (self.n_designs + 1))()
        im = (ctypes.c_int64 * (self.n_designs + 1))()
        _check(L.ffrt_plan_layout(self.h, cp, im), "layout")
        self.cp_offsets = list(cp)
        self.img_offsets = list(im)
        n = ctypes.c_int64()
        _check(L.ffrt_plan_num_rays(self.h, ctypes.byref(n)), "num_rays")
        self.num_rays = n.value

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None and _lib is not None:
                _lib.ffrt_plan_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # ---- buffers -------------------------------------------------------------------------------
    @property
    def total_cp(self):
        return self.cp_offsets[-1]

    @property
    def total_img(self):
        return self.img_offsets[-1]

    def _f32(self, t, n, name):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.device != self.device or t.numel() != n:
            raise FfrtError(f"{name}: need a contiguous float32 tensor of {n} elements on {self.device}")
        return t

    def pack_cp(self, arrays):
        return torch.cat([torch.as_tensor(np.asarray(a, np.float32)).reshape(-1) for a in arrays]).to(self.device)

    def pack_img(self, arrays):
        return self.pack_cp(arrays)

    def unpack_cp(self, flat):
        out = []
        for d, p in enumerate(self.problems):
            a, b = self.cp_offsets[d], self.cp_offsets[d + 1]
            out.append(flat[a:b].reshape(p.cp_shape()))
        return out

    def unpack_img(self, flat):
        out = []
        for d, p in enumerate(self.problems):
            a, b = self.img_offsets[d], self.img_offsets[d + 1]
            out.append(flat[a:b].reshape(p.image_shape()))
        return out

    def new_stats(self):
        return torch.zeros(self.n_designs * STATS_BYTES, dtype=torch.uint8, device=self.device)

    @staticmethod
    def decode_stats(st):
        return np.frombuffer(st.cpu().numpy().tobytes(), dtype=STATS_DTYPE)

    # ---- the hot path -------------------------------------------------------------------------
    def forward(self, Pz, irr=None, stats=None, stream=None):
        self._f32(Pz, self.total_cp, "Pz")
        if irr is None:
            irr = torch.empty(self.total_img, dtype=torch.float32, device=self.device)
        self._f32(irr, self.total_img, "irr")
        _check(lib().ffrt_forward(self.h, _ptr(Pz), _ptr(irr), _ptr(stats), _stream(stream)), "ffrt_forward")
        return irr

    def forward_static(self, Pz, irr=None, stats=None, stream=None):
        """ffrt_forward_static: the forward in the library's static device array instead of the plan's
        workspace (for callers that cannot allocate; calls on one GPU must not overlap)."""
        self._f32(Pz, self.total_cp, "Pz")
        if irr is None:
            irr = torch.empty(self.total_img, dtype=torch.float32, device=self.device)
        self._f32(irr, self.total_img, "irr")
        _check(lib().ffrt_forward_static(self.h, _ptr(Pz), _ptr(irr), _ptr(stats), _stream(stream)),
               "ffrt_forward_static")
        return irr

    def loss(self, irr, target, loss=None, dLdI=None, stream=None):
        self._f32(irr, self.total_img, "irr")
        self._f32(target, self.total_img, "target")
        if loss is None:
            loss = torch.empty(self.n_designs, dtype=torch.float32, device=self.device)
        if dLdI is None:
            dLdI = torch.empty(self.total_img, dtype=torch.float32, device=self.device)
        _check(lib().ffrt_loss(self.h, _ptr(irr), _ptr(target), _ptr(loss), _ptr(dLdI), _stream(stream)),
               "ffrt_loss")
        return loss, dLdI

    def loss_f64(self, irr, target, loss=None, stream=None):
        """Loss values with double-precision reductions (for finite differences)."""
        self._f32(irr, self.total_img, "irr")
        self._f32(target, self.total_img, "target")
        if loss is None:
            loss = torch.empty(self.n_designs, dtype=torch.float64, device=self.device)
        _check(lib().ffrt_loss_f64(self.h, _ptr(irr), _ptr(target), _ptr(loss), _stream(stream)), "ffrt_loss_f64")
        return loss

    def adjoint(self, Pz, dLdI, dLdP=None, stream=None):
        self._f32(Pz, self.total_cp, "Pz")
        self._f32(dLdI, self.total_img, "dLdI")
        if dLdP is None:
            dLdP = torch.empty(self.total_cp, dtype=torch.float32, device=self.device)
        _check(lib().ffrt_adjoint(self.h, _ptr(Pz), _ptr(dLdI), _ptr(dLdP), _stream(stream)), "ffrt_adjoint")
        return dLdP

    def adam(self, Pz, g, m, v, t, hp=AdamHP(), stream=None):
        _check(lib().ffrt_adam(self.h, _ptr(Pz), _ptr(g), _ptr(m), _ptr(v), _ptr(t), ctypes.byref(hp.c()),
                               _stream(stream)), "ffrt_adam")

    def new_state(self, Pz, with_dLdI=False):
        """Buffers of an optimisation loop for control heights Pz (packed).  Without with_dLdI the step keeps
        dL/dI in the plan's workspace."""
        dev = self.device
        return dict(
            Pz=Pz, irr=torch.zeros(self.total_img, device=dev), loss=torch.zeros(self.n_designs, device=dev),
            dLdI=torch.zeros(self.total_img, device=dev) if with_dLdI else None,
            dLdP=torch.zeros(self.total_cp, device=dev),
            m=torch.zeros(self.total_cp, device=dev), v=torch.zeros(self.total_cp, device=dev),
            t=torch.zeros(self.n_designs, dtype=torch.int32, device=dev), stats=self.new_stats())

    def step(self, st, target, hp=AdamHP(), stream=None):
        _check(lib().ffrt_step(self.h, _ptr(st["Pz"]), _ptr(target), _ptr(st["irr"]), _ptr(st["loss"]),
                               _ptr(st.get("dLdI")), _ptr(st["dLdP"]), _ptr(st["m"]), _ptr(st["v"]), _ptr(st["t"]),
                               _ptr(st["stats"]), ctypes.byref(hp.c()), _stream(stream)), "ffrt_step")

    def graph_capture(self, st, target, steps=1, hp=AdamHP(), stream=None):
        _check(lib().ffrt_graph_capture(self.h, steps, _ptr(st["Pz"]), _ptr(target), _ptr(st["irr"]),
                                        _ptr(st["loss"]), _ptr(st.get("dLdI")), _ptr(st["dLdP"]), _ptr(st["m"]),
                                        _ptr(st["v"]), _ptr(st["t"]), _ptr(st["stats"]), ctypes.byref(hp.c()),
                                        _stream(stream)), "ffrt_graph_capture")

    # ---- range reparametrisation (sec. 2.4.1): P = lo + (tanh(theta) + 1) span / 2 ---------------------
    def control_xy(self):
        """Greville (x, y) of every control point, packed like Pz (float64 numpy arrays)."""
        x = np.zeros(self.total_cp)
        y = np.zeros(self.total_cp)
        _check(lib().ffrt_plan_control_xy(self.h, x.ctypes.data_as(ctypes.c_void_p),
                                          y.ctypes.data_as(ctypes.c_void_p)), "ffrt_plan_control_xy")
        return x, y

    def reparam_apply(self, theta, lo, span, Pz=None, stream=None):
        for a, n in ((theta, "theta"), (lo, "lo"), (span, "span")):
            self._f32(a, self.total_cp, n)
        if Pz is None:
            Pz = torch.empty(self.total_cp, dtype=torch.float32, device=self.device)
        _check(lib().ffrt_reparam_apply(self.h, _ptr(theta), _ptr(lo), _ptr(span), _ptr(Pz), _stream(stream)),
               "ffrt_reparam_apply")
        return Pz

    def reparam_grad(self, theta, span, dLdP, out=None, stream=None):
        for a, n in ((theta, "theta"), (span, "span"), (dLdP, "dLdP")):
            self._f32(a, self.total_cp, n)
        if out is None:
            out = torch.empty(self.total_cp, dtype=torch.float32, device=self.device)
        _check(lib().ffrt_reparam_grad(self.h, _ptr(theta), _ptr(span), _ptr(dLdP), _ptr(out), _stream(stream)),
               "ffrt_reparam_grad")
        return out

    def new_reparam_state(self, theta, lo, span, with_dLdI=False):
        """Optimisation state on theta; Pz is kept equal to P(theta) by the steps."""
        st = self.new_state(self.reparam_apply(theta, lo, span), with_dLdI)
        st.update(theta=theta, lo=lo, span=span)
        return st

    def step_reparam(self, st, target, hp=AdamHP(), stream=None):
        _check(lib().ffrt_step_reparam(self.h, _ptr(st["theta"]), _ptr(st["lo"]), _ptr(st["span"]), _ptr(st["Pz"]),
                                       _ptr(target), _ptr(st["irr"]), _ptr(st["loss"]), _ptr(st.get("dLdI")),
                                       _ptr(st["dLdP"]), _ptr(st["m"]), _ptr(st["v"]), _ptr(st["t"]),
                                       _ptr(st["stats"]), ctypes.byref(hp.c()), _stream(stream)), "ffrt_step_reparam")

    def graph_capture_reparam(self, st, target, steps=1, hp=AdamHP(), stream=None):
        _check(lib().ffrt_graph_capture_reparam(
            self.h, steps, _ptr(st["theta"]), _ptr(st["lo"]), _ptr(st["span"]), _ptr(st["Pz"]), _ptr(target),
            _ptr(st["irr"]), _ptr(st["loss"]), _ptr(st.get("dLdI")), _ptr(st["dLdP"]), _ptr(st["m"]), _ptr(st["v"]),
            _ptr(st["t"]), _ptr(st["stats"]), ctypes.byref(hp.c()), _stream(stream)), "ffrt_graph_capture_reparam")

    # ---- control-point generators (sec. 2.4): three K-wide tanh layers, then the output correction ------
    # arch: MLP_DENSE (fully connected K x K layers) or MLP_SPARSE (weights W[c][k] over the (2p+1) x (2q+1)
    # neighbourhood of each control point)
    def mlp_offsets(self, arch=0):
        """Offsets of each design's generator parameters in the packed parameter vector (n_designs + 1)."""
        off = (ctypes.c_int64 * (self.n_designs + 1))()
        _check(lib().ffrt_mlp_layout(self.h, arch, off), "ffrt_mlp_layout")
        return list(off)

    def _mlp_shapes(self, d, arch):
        p = self.problems[d].lens
        K = p.n_u * p.n_v
        Wshape = (K, K) if arch == MLP_DENSE else ((2 * p.p + 1) * (2 * p.q + 1), K)
        return [(K,), (K,), Wshape, (K,), Wshape, (K,)]

    def pack_mlp(self, per_design, arch=0):
        """Pack per-design (w1, b1, W2, b2, W3, b3) tuples into one float32 device vector."""
        parts = []
        for d, prm in enumerate(per_design):
            for a, shp in zip(prm, self._mlp_shapes(d, arch)):
                a = np.asarray(a, np.float32)
                if a.shape != shp:
                    raise FfrtError(f"design {d}: generator parameter of shape {a.shape}, expected {shp}")
                parts.append(torch.as_tensor(a).reshape(-1))
        return torch.cat(parts).to(self.device)

    def unpack_mlp(self, flat, arch=0):
        """Inverse of pack_mlp: per-design (w1, b1, W2, b2, W3, b3) views of a packed vector."""
        off, out = self.mlp_offsets(arch), []
        for d in range(self.n_designs):
            o, views = off[d], []
            for shp in self._mlp_shapes(d, arch):
                n = int(np.prod(shp))
                views.append(flat[o:o + n].reshape(shp))
                o += n
            out.append(tuple(views))
        return out

    def mlp_forward(self, params, lo, span, acts=None, Pz=None, arch=0, stream=None):
        self._f32(params, self.mlp_offsets(arch)[-1], "params")
        for a, n in ((lo, "lo"), (span, "span")):
            self._f32(a, self.total_cp, n)
        if acts is None:
            acts = torch.empty(3 * self.total_cp, dtype=torch.float32, device=self.device)
        if Pz is None:
            Pz = torch.empty(self.total_cp, dtype=torch.float32, device=self.device)
        self._f32(acts, 3 * self.total_cp, "acts")
        _check(lib().ffrt_mlp_forward(self.h, arch, _ptr(params), _ptr(lo), _ptr(span), _ptr(acts), _ptr(Pz),
                                      _stream(stream)), "ffrt_mlp_forward")
        return acts, Pz

    def mlp_backward(self, params, acts, span, dLdP, grad=None, arch=0, stream=None):
        n = self.mlp_offsets(arch)[-1]
        self._f32(params, n, "params")
        self._f32(acts, 3 * self.total_cp, "acts")
        for a, nm in ((span, "span"), (dLdP, "dLdP")):
            self._f32(a, self.total_cp, nm)
        if grad is None:
            grad = torch.empty(n, dtype=torch.float32, device=self.device)
        self._f32(grad, n, "grad")
        _check(lib().ffrt_mlp_backward(self.h, arch, _ptr(params), _ptr(acts), _ptr(span), _ptr(dLdP), _ptr(grad),
                                       _stream(stream)), "ffrt_mlp_backward")
        return grad

    def new_mlp_state(self, params, lo, span, arch=0, with_dLdI=False):
        """Optimisation state on the generator parameters; acts and Pz are kept equal to the forward pass of
        params by the steps."""
        acts, Pz = self.mlp_forward(params, lo, span, arch=arch)
        st = self.new_state(Pz, with_dLdI)
        st.update(params=params, lo=lo, span=span, acts=acts, m=torch.zeros_like(params),
                  v=torch.zeros_like(params), arch=arch)
        return st

    def step_mlp(self, st, target, hp=AdamHP(), stream=None):
        _check(lib().ffrt_step_mlp(self.h, st["arch"], _ptr(st["params"]), _ptr(st["m"]), _ptr(st["v"]), _ptr(st["t"]),
                                   _ptr(st["lo"]), _ptr(st["span"]), _ptr(st["acts"]), _ptr(st["Pz"]), _ptr(target),
                                   _ptr(st["irr"]), _ptr(st["loss"]), _ptr(st.get("dLdI")), _ptr(st["dLdP"]),
                                   _ptr(st["stats"]), ctypes.byref(hp.c()), _stream(stream)), "ffrt_step_mlp")

    def graph_capture_mlp(self, st, target, steps=1, hp=AdamHP(), stream=None):
        _check(lib().ffrt_graph_capture_mlp(
            self.h, st["arch"], steps, _ptr(st["params"]), _ptr(st["m"]), _ptr(st["v"]), _ptr(st["t"]), _ptr(st["lo"]),
            _ptr(st["span"]), _ptr(st["acts"]), _ptr(st["Pz"]), _ptr(target), _ptr(st["irr"]), _ptr(st["loss"]),
            _ptr(st.get("dLdI")), _ptr(st["dLdP"]), _ptr(st["stats"]), ctypes.byref(hp.c()), _stream(stream)),
            "ffrt_graph_capture_mlp")

    def time_mlp(self, st, dLdP, reps=20, hp=AdamHP(), stream=None):
        """Mean (forward, back-propagation, gradient + Adam) generator durations in ms (HIP events on the
        stream), on copies of the state's parameters and moments."""
        par, m, v = st["params"].clone(), st["m"].clone(), st["v"].clone()
        acts, Pz = torch.empty_like(st["acts"]), torch.empty_like(st["Pz"])
        f, b, u = ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
        _check(lib().ffrt_plan_time_mlp(self.h, st["arch"], _ptr(par), _ptr(m), _ptr(v), _ptr(st["t"]),
                                        _ptr(st["lo"]), _ptr(st["span"]), _ptr(acts), _ptr(Pz), _ptr(dLdP),
                                        ctypes.byref(hp.c()), reps, ctypes.byref(f), ctypes.byref(b),
                                        ctypes.byref(u), _stream(stream)), "ffrt_plan_time_mlp")
        return f.value, b.value, u.value

    def time_kernels(self, Pz, irr, dLdI, dLdP, reps=20, stream=None):
        """Mean (forward, adjoint) trace-kernel durations in ms (HIP events on the stream)."""
        f, a = ctypes.c_float(), ctypes.c_float()
        _check(lib().ffrt_plan_time_kernels(self.h, _ptr(Pz), _ptr(irr), _ptr(dLdI), _ptr(dLdP), reps,
                                            ctypes.byref(f), ctypes.byref(a), _stream(stream)), "time_kernels")
        return f.value, a.value

    def graph_launch(self, stream=None):
        _check(lib().ffrt_graph_launch(self.h, _stream(stream)), "ffrt_graph_launch")

    # ---- shapes -------------------------------------------------------------------------------
    @staticmethod
    def config_names(which):
        n = ctypes.c_int32()
        _check(lib().ffrt_num_configs(which, ctypes.byref(n)), "num_configs")
        names = []
        for i in range(n.value):
            buf = ctypes.create_string_buffer(128)
            _check(lib().ffrt_config_name(which, i, buf, 128), "config_name")
            names.append(buf.value.decode())
        return names

    def set_config(self, which, index):
        _check(lib().ffrt_plan_set_config(self.h, which, index), "set_config")

    def get_config(self, which):
        i = ctypes.c_int32()
        _check(lib().ffrt_plan_get_config(self.h, which, ctypes.byref(i)), "get_config")
        return i.value

    def autotune(self, Pz, irr, dLdI, dLdP, reps=3, stream=None):
        _check(lib().ffrt_plan_autotune(self.h, _ptr(Pz), _ptr(irr), _ptr(dLdI), _ptr(dLdP), reps,
                                        _stream(stream)), "autotune")
        return self.get_config(0), self.get_config(1)

    # ---- inspection ---------------------------------------------------------------------------
    def trace_rays(self, design, Pz, ids, stream=None):
        ids = torch.as_tensor(np.asarray(ids, np.int64)).to(self.device)
        out = torch.empty((ids.numel(), 8), dtype=torch.float32, device=self.device)
        _check(lib().ffrt_trace_rays(self.h, design, _ptr(Pz), _ptr(ids), ids.numel(), _ptr(out), _stream(stream)),
               "ffrt_trace_rays")
        return out


def rng(seed, stream_id, first, n, device="cuda"):
    """SplitMix64 outputs computed on the device, returned as numpy uint64."""
    out = torch.empty(n, dtype=torch.int64, device=device)
    _check(lib().ffrt_rng(seed, stream_id, first, n, _ptr(out), _stream()), "ffrt_rng")
    return out.cpu().numpy().view(np.uint64)


def lds_atomic_rate(pattern, reps=20, stream=None):
    """LDS atomic adds per second over the chip (pattern 0: distinct banks, 1: the forward's splat)."""
    r = ctypes.c_double()
    _check(lib().ffrt_lds_atomic_rate(pattern, reps, ctypes.byref(r), _stream(stream)), "ffrt_lds_atomic_rate")
    return r.value


class TraceLoss(torch.autograd.Function):
    """loss = L(P) per design (sec. 2.5); backward runs the adjoint kernel."""

    @staticmethod
    def forward(ctx, Pz, target, plan):
        irr = plan.forward(Pz)
        loss, dLdI = plan.loss(irr, target)
        ctx.plan = plan
        ctx.save_for_backward(Pz, dLdI)
        return loss

    @staticmethod
    def backward(ctx, gL):
        Pz, dLdI = ctx.saved_tensors
        plan = ctx.plan
        g = plan.adjoint(Pz.detach().contiguous(), dLdI)
        scale = torch.repeat_interleave(gL.to(torch.float32),
                                        torch.tensor([plan.cp_offsets[d + 1] - plan.cp_offsets[d]
                                                      for d in range(plan.n_designs)], device=gL.device))
        return g * scale, None, None
