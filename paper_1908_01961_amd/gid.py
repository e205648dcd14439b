"""ctypes binding of libgid (include/gid.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Device buffers are torch CUDA (ROCm) tensors; torch provides the
memory and the current stream.  The library must be built (paper_1908_01961_amd.build);
nothing here falls back to another implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_float, c_int32, c_size_t, c_uint32, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgid.so")

GID_OK = 0
STATUS = {0: "ok", 1: "invalid argument", 2: "out of memory", 3: "HIP runtime error",
          4: "non-finite value", 5: "call out of order", 6: "unsupported"}
REFINE = {"off": 0, "first": 1, "every": 2}
CR = {"chroma": 0, "literal": 1}
BSTEP = {"pixel": 0, "sum": 1}
KERNEL_KINDS = ("scan", "precompute", "gn_build", "pcg", "apply_bsum", "bsolve", "energy",
                "output")
TERMS = ("data", "cluster", "rsparsity", "rconsist", "mono", "isparsity", "smooth", "nonneg")
MAX_HALF = 128


class GidLambdas(ctypes.Structure):
    _fields_ = [(n, c_float) for n in ("data", "cluster", "r_sparsity", "p", "r_consistency",
                                         "monochrome", "i_sparsity", "smoothness", "non_neg", "ir", "cr")]


class GidParams(ctypes.Structure):
    _fields_ = [("struct_size", c_uint32), ("K", c_int32), ("lambda_", GidLambdas),
                ("eps_nonneg", c_float), ("eps_irls", c_float), ("retinex_k", c_float),
                ("chroma_gate", c_double), ("chroma_floor", c_double),
                ("gn_iters", c_int32), ("pcg_iters", c_int32), ("refine_mode", c_int32),
                ("temporal", c_int32), ("cr_mode", c_int32), ("record_energy", c_int32),
                ("use_graph", c_int32), ("bstep_scale", c_int32), ("spatial_pairs", c_int32),
                ("spatial_seed", ctypes.c_uint32)]


class GidFrameStats(ctypes.Structure):
    _fields_ = [("energy_final", c_double), ("energy_terms", c_double * 8),
                ("energy_half", c_double * MAX_HALF), ("pcg_rz_last", c_double * 64),
                ("n_half", c_int32), ("gn_done", c_int32), ("pcg_breakdowns", c_int32),
                ("bstep_rejected", c_int32), ("frame_index", c_int32), ("warm_start_learned", c_int32),
                ("energy_start_previous", c_double), ("energy_start_learned", c_double)]

    def to_dict(self) -> dict:
        return dict(energy_final=self.energy_final,
                    energy_terms=dict(zip(TERMS, list(self.energy_terms))),
                    energy_half=list(self.energy_half[: self.n_half]),
                    pcg_rz_last=list(self.pcg_rz_last[: self.gn_done]),
                    gn_done=self.gn_done, pcg_breakdowns=self.pcg_breakdowns,
                    bstep_rejected=self.bstep_rejected, frame_index=self.frame_index,
                    warm_start_learned=self.warm_start_learned,
                    energy_start_previous=self.energy_start_previous,
                    energy_start_learned=self.energy_start_learned)


_lib = None

#: (name, restype, argtypes) of every exported call of gid.h
SIGNATURES = [
    ("gid_default_params", c_int32, [c_int32, POINTER(GidParams)]),
    ("gid_create", c_int32, [POINTER(GidParams), c_int32, c_int32, c_void_p, POINTER(c_void_p)]),
    ("gid_destroy", c_int32, [c_void_p]),
    ("gid_set_base_colors", c_int32, [c_void_p, POINTER(c_double)]),
    ("gid_reset_clip", c_int32, [c_void_p]),
    ("gid_decompose_frame", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_double),
                                      POINTER(GidFrameStats)]),
    ("gid_synchronize", c_int32, [c_void_p]),
    ("gid_set_energy_target", c_int32, [c_void_p, c_double, c_int32]),
    ("gid_set_energy_check_from", c_int32, [c_void_p, c_int32]),
    ("gid_load_frame", c_int32, [c_void_p, c_void_p, c_void_p]),
    ("gid_set_state", c_int32, [c_void_p, c_void_p, POINTER(c_double)]),
    ("gid_set_prev_frame", c_int32, [c_void_p, c_void_p, c_void_p]),
    ("gid_get_state", c_int32, [c_void_p, c_void_p, POINTER(c_double)]),
    ("gid_eval_energy", c_int32, [c_void_p, POINTER(c_double), POINTER(c_double)]),
    ("gid_eval_rhs", c_int32, [c_void_p, c_void_p, c_void_p]),
    ("gid_apply_normal", c_int32, [c_void_p, c_void_p, c_void_p]),
    ("gid_layer_step", c_int32, [c_void_p, POINTER(c_double)]),
    ("gid_bstep_sums", c_int32, [c_void_p, POINTER(c_double), POINTER(c_double)]),
    ("gid_base_step", c_int32, [c_void_p, POINTER(c_int32)]),
    ("gid_set_profiling", c_int32, [c_void_p, c_int32]),
    ("gid_get_kernel_times", c_int32, [c_void_p, POINTER(c_double), POINTER(ctypes.c_int64)]),
    ("gid_batch_create", c_int32, [POINTER(c_void_p), c_int32, POINTER(c_void_p)]),
    ("gid_batch_destroy", c_int32, [c_void_p]),
    ("gid_batch_decompose", c_int32, [c_void_p, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p)]),
    ("gid_batch_synchronize", c_int32, [c_void_p, POINTER(c_double)]),
    ("gid_batch_last_error", ctypes.c_char_p, [c_void_p]),
    ("gid_autotune", c_int32, [c_void_p, ctypes.c_char_p, POINTER(c_int32)]),
    ("gid_set_workgroups", c_int32, [c_void_p, c_int32]),
    ("gid_get_workgroups", c_int32, [c_void_p]),
    ("gid_save_state", c_int32, [c_void_p, c_void_p, POINTER(c_size_t)]),
    ("gid_load_state", c_int32, [c_void_p, c_void_p, c_size_t]),
    ("gid_net_num_params", ctypes.c_int64, [c_int32]),
    ("gid_net_create", c_int32, [c_int32, c_int32, c_int32, c_void_p, POINTER(c_void_p)]),
    ("gid_net_destroy", c_int32, [c_void_p]),
    ("gid_net_set_params", c_int32, [c_void_p, POINTER(c_float), ctypes.c_int64]),
    ("gid_net_get_params", c_int32, [c_void_p, POINTER(c_float), ctypes.c_int64]),
    ("gid_net_forward", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_float)]),
    ("gid_net_gradients", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_float), c_float,
                                    POINTER(c_float), POINTER(c_double)]),
    ("gid_net_train_step", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_float), c_float, c_float,
                                     POINTER(c_double)]),
    ("gid_net_layer_forward", c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    ("gid_net_layer_wgrad", c_int32, [c_void_p, c_int32, c_void_p, c_void_p, POINTER(c_float), POINTER(c_float)]),
    ("gid_net_set_conv_workgroups", c_int32, [c_void_p, c_int32]),
    ("gid_net_last_error", ctypes.c_char_p, [c_void_p]),
    ("gid_set_warmstart", c_int32, [c_void_p, c_void_p]),
    ("gid_cluster_frame", c_int32, [c_void_p, c_int32, c_int32, c_int32, c_double, c_void_p, c_void_p,
                                    POINTER(c_double), POINTER(c_double), POINTER(c_int32)]),
    ("gid_cluster_frame_noalloc", c_int32, [c_void_p, c_int32, c_int32, c_int32, c_double, c_void_p, c_void_p,
                                            POINTER(c_double), POINTER(c_double), POINTER(c_int32)]),
    ("gid_resynthesize", c_int32, [c_void_p, c_int32, c_int32, c_int32, POINTER(c_double), c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_void_p]),
    ("gid_correct_region", c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p, POINTER(c_double),
                                     c_void_p, c_void_p, POINTER(c_double), POINTER(c_int32)]),
    ("gid_batch_set_launch", c_int32, [c_void_p, c_int32]),
    ("gid_batch_get_launch", c_int32, [c_void_p, POINTER(c_int32)]),
    ("gid_batch_autotune", c_int32, [c_void_p, POINTER(c_int32)]),
    ("gid_status_string", ctypes.c_char_p, [c_int32]),
    ("gid_last_error", ctypes.c_char_p, [c_void_p]),
]


def load_library(path: str = LIB_PATH):
    """Load libgid.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libgid.so is not built ({path}); run python -m paper_1908_01961_amd.build")
    # torch brings its own HIP runtime: loaded first, it is the one the library
    # binds to, so that torch's streams and allocations are valid in library calls
    # (loading the library first would bind it to a second runtime)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class GidError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def default_params(K: int, **overrides) -> GidParams:
    lib = load_library()
    p = GidParams()
    st = lib.gid_default_params(K, byref(p))
    if st != GID_OK:
        raise GidError(st, f"gid_default_params(K={K})")
    for k, v in overrides.items():
        if k == "refine_mode" and isinstance(v, str):
            v = REFINE[v]
        if k == "cr_mode" and isinstance(v, str):
            v = CR[v]
        if k == "bstep_scale" and isinstance(v, str):
            v = BSTEP[v]
        if k.startswith("lam_"):
            setattr(p.lambda_, k[4:], v)
        else:
            setattr(p, k, int(v) if isinstance(getattr(p, k), int) else v)
    return p


def _ptr(t, dtype, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {tuple(shape)}, got "
                         f"{t.dtype} {tuple(t.shape)}")
    return c_void_p(t.data_ptr())


def _dbl(arr, n):
    a = np.ascontiguousarray(np.asarray(arr, np.float64).reshape(-1))
    if a.size != n:
        raise ValueError(f"expected {n} values")
    return a, a.ctypes.data_as(POINTER(c_double))


def cluster_frame(frame, k_max: int = 10, merge_dist: float = 0.2, stream=None, noalloc: bool = False):
    """Base-colour initialisation of a clip from its first frame (Sec. 5.1):
    returns (ids uint8 tensor (H, W) on the frame's device, colours (k, 3) FP64,
    centres (k, 3) FP64).  noalloc uses the entry point with a fixed scratch array."""
    import torch
    lib = load_library()
    H, W = int(frame.shape[1]), int(frame.shape[2])
    f = _ptr(frame, torch.float32, (3, H, W), "frame")
    ids = torch.empty((H, W), dtype=torch.uint8, device=frame.device)
    cols = np.zeros(3 * k_max)
    cen = np.zeros(3 * k_max)
    k = c_int32(0)
    sp = c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
    fn = lib.gid_cluster_frame_noalloc if noalloc else lib.gid_cluster_frame
    st = fn(f, W, H, int(k_max), float(merge_dist), sp, c_void_p(ids.data_ptr()),
                               cols.ctypes.data_as(POINTER(c_double)), cen.ctypes.data_as(POINTER(c_double)),
                               byref(k))
    if st != GID_OK:
        raise GidError(st, "gid_cluster_frame")
    n = k.value
    return ids, cols[:3 * n].reshape(n, 3).copy(), cen[:3 * n].reshape(n, 3).copy()


def resynthesize(layers, b_new, gain=None, ids=None, refl_scale=None, out=None, stream=None):
    """Recombine layers ((K+4, H, W) float32 CUDA tensor, R first) with edited base
    colours b_new (K, 3), per-layer gains (K,) and a per-cluster reflectance scale
    (K, 3) applied through ids ((H, W) uint8 CUDA tensor); returns (3, H, W)."""
    import torch
    lib = load_library()
    n, H, W = (int(v) for v in layers.shape)
    K = n - 4
    lp = _ptr(layers, torch.float32, (n, H, W), "layers")
    out = torch.empty((3, H, W), dtype=torch.float32, device=layers.device) if out is None else out
    op = _ptr(out, torch.float32, (3, H, W), "out")
    b = np.ascontiguousarray(np.asarray(b_new, np.float64).reshape(-1))
    g = None if gain is None else np.ascontiguousarray(np.asarray(gain, np.float32).reshape(-1))
    sc = None if refl_scale is None else np.ascontiguousarray(np.asarray(refl_scale, np.float32).reshape(-1))
    ip = _ptr(ids, torch.uint8, (H, W), "ids") if ids is not None else None
    sp = c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
    st = lib.gid_resynthesize(lp, W, H, K, b.ctypes.data_as(POINTER(c_double)),
                              None if g is None else c_void_p(g.ctypes.data),
                              ip, None if sc is None else c_void_p(sc.ctypes.data), sp, op)
    if st != GID_OK:
        raise GidError(st, "gid_resynthesize")
    return out


def correct_region(params: "GidParams", frame, ids, region, colors, stream=None):
    """Misclustering correction (Sec. 5.2.2): returns (best colour index,
    sparsity per candidate (K,), corrected ids tensor)."""
    import torch
    lib = load_library()
    H, W = int(frame.shape[1]), int(frame.shape[2])
    K = params.K
    f = _ptr(frame, torch.float32, (3, H, W), "frame")
    i = _ptr(ids, torch.uint8, (H, W), "ids")
    r = _ptr(region, torch.uint8, (H, W), "region")
    out = torch.empty((H, W), dtype=torch.uint8, device=frame.device)
    cols = np.ascontiguousarray(np.asarray(colors, np.float64).reshape(-1))
    sp = np.zeros(K)
    best = c_int32(-1)
    stp = c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
    st = lib.gid_correct_region(byref(params), W, H, f, i, r, cols.ctypes.data_as(POINTER(c_double)), stp,
                                c_void_p(out.data_ptr()), sp.ctypes.data_as(POINTER(c_double)), byref(best))
    if st != GID_OK:
        raise GidError(st, "gid_correct_region")
    return best.value, sp, out


class Solver:
    """One libgid context: frames of width x height with K base colours."""

    def __init__(self, width: int, height: int, params: GidParams | int, stream=None):
        import torch
        self.lib = load_library()
        if isinstance(params, int):
            params = default_params(params)
        self.params = params
        self.W, self.H, self.K = int(width), int(height), int(params.K)
        self.n = self.K + 4
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        h = c_void_p()
        st = self.lib.gid_create(byref(params), self.W, self.H, c_void_p(stream.cuda_stream), byref(h))
        if st != GID_OK:
            raise GidError(st, f"gid_create({self.W}x{self.H}, K={self.K})")
        self.h = h
        self._stats = GidFrameStats()
        self._b = np.zeros(3 * self.K)

    def _check(self, st, what):
        if st != GID_OK:
            raise GidError(st, f"{what}: {self.lib.gid_last_error(self.h).decode()}")

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.gid_destroy(self.h)
            self.h = None

    def set_warmstart(self, net: "Net | None"):
        """Attach (or with None detach) a learned warm-start network."""
        self._check(self.lib.gid_set_warmstart(self.h, net.h if net is not None else None), "gid_set_warmstart")
        self._net = net

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- clip control
    def set_base_colors(self, b):
        a, p = _dbl(b, 3 * self.K)
        self._check(self.lib.gid_set_base_colors(self.h, p), "gid_set_base_colors")

    def reset_clip(self):
        self._check(self.lib.gid_reset_clip(self.h), "gid_reset_clip")

    # -- full frame
    def decompose_frame_async(self, frame, ids, layers=None):
        """Enqueue one frame; outputs are valid after synchronize()."""
        import torch
        f = _ptr(frame, torch.float32, (3, self.H, self.W), "frame")
        i = _ptr(ids, torch.uint8, (self.H, self.W), "ids") if ids is not None else None
        lp = _ptr(layers, torch.float32, (self.n, self.H, self.W), "layers") if layers is not None else None
        # a refused call leaves the pending frame's output buffer in place
        bout = np.zeros(3 * self.K)
        self._check(self.lib.gid_decompose_frame(self.h, f, i, lp, bout.ctypes.data_as(POINTER(c_double)),
                                                 byref(self._stats)), "gid_decompose_frame")
        self._b = bout

    def synchronize(self):
        self._check(self.lib.gid_synchronize(self.h), "gid_synchronize")
        return self._b.reshape(self.K, 3).copy(), self._stats.to_dict()

    def set_energy_target(self, target: float, max_gn: int = 0):
        """Stop each following frame once its energy is <= target (up to max_gn
        outer iterations); target <= 0 restores the fixed schedule."""
        self._check(self.lib.gid_set_energy_target(self.h, float(target), int(max_gn)), "gid_set_energy_target")

    def set_energy_check_from(self, first_gn: int):
        """Check the energy target only after outer iteration first_gn (1-based) and later."""
        self._check(self.lib.gid_set_energy_check_from(self.h, int(first_gn)), "gid_set_energy_check_from")

    def decompose_frame(self, frame, ids, layers=None):
        self.decompose_frame_async(frame, ids, layers)
        return self.synchronize()

    # -- single steps
    def load_frame(self, frame, ids):
        import torch
        f = _ptr(frame, torch.float32, (3, self.H, self.W), "frame")
        i = _ptr(ids, torch.uint8, (self.H, self.W), "ids")
        self._check(self.lib.gid_load_frame(self.h, f, i), "gid_load_frame")

    def set_state(self, u, b=None):
        import torch
        up = _ptr(u, torch.float32, (self.n, self.H, self.W), "u")
        if b is not None:
            arr, bp = _dbl(b, 3 * self.K)
        else:
            arr, bp = None, None
        self._check(self.lib.gid_set_state(self.h, up, bp), "gid_set_state")

    def set_prev_frame(self, frame_prev, r_prev):
        import torch
        f = _ptr(frame_prev, torch.float32, (3, self.H, self.W), "frame_prev")
        r = _ptr(r_prev, torch.float32, (3, self.H, self.W), "r_prev")
        self._check(self.lib.gid_set_prev_frame(self.h, f, r), "gid_set_prev_frame")

    def get_state(self):
        import torch
        u = torch.empty((self.n, self.H, self.W), dtype=torch.float32, device="cuda")
        b = np.zeros(3 * self.K)
        self._check(self.lib.gid_get_state(self.h, _ptr(u, torch.float32, u.shape, "u"),
                                           b.ctypes.data_as(POINTER(c_double))), "gid_get_state")
        return u, b.reshape(self.K, 3)

    def eval_energy(self):
        e = c_double()
        terms = (c_double * 8)()
        self._check(self.lib.gid_eval_energy(self.h, byref(e), terms), "gid_eval_energy")
        return e.value, dict(zip(TERMS, list(terms)))

    def eval_rhs(self):
        import torch
        g = torch.empty((self.n, self.H, self.W), dtype=torch.float32, device="cuda")
        d = torch.empty_like(g)
        self._check(self.lib.gid_eval_rhs(self.h, c_void_p(g.data_ptr()), c_void_p(d.data_ptr())), "gid_eval_rhs")
        return g, d

    def apply_normal(self, p):
        import torch
        pp = _ptr(p, torch.float32, (self.n, self.H, self.W), "p")
        q = torch.empty_like(p)
        self._check(self.lib.gid_apply_normal(self.h, pp, c_void_p(q.data_ptr())), "gid_apply_normal")
        return q

    def layer_step(self):
        rz = c_double()
        self._check(self.lib.gid_layer_step(self.h, byref(rz)), "gid_layer_step")
        return rz.value

    def bstep_sums(self):
        K = self.K
        A = np.zeros(3 * K * K)
        h = np.zeros(3 * K)
        self._check(self.lib.gid_bstep_sums(self.h, A.ctypes.data_as(POINTER(c_double)),
                                            h.ctypes.data_as(POINTER(c_double))), "gid_bstep_sums")
        return A.reshape(3, K, K), h.reshape(3, K)

    def base_step(self):
        ok = c_int32()
        self._check(self.lib.gid_base_step(self.h, byref(ok)), "gid_base_step")
        return bool(ok.value)

    # -- launch shape
    def autotune(self, cache_path: str | None = None) -> int:
        n = c_int32()
        path = cache_path.encode() if cache_path else None
        self._check(self.lib.gid_autotune(self.h, path, byref(n)), "gid_autotune")
        return n.value

    def set_workgroups(self, n: int):
        self._check(self.lib.gid_set_workgroups(self.h, int(n)), "gid_set_workgroups")

    @property
    def workgroups(self) -> int:
        return int(self.lib.gid_get_workgroups(self.h))

    # -- kernel timing
    def set_profiling(self, enable: bool):
        self._check(self.lib.gid_set_profiling(self.h, int(bool(enable))), "gid_set_profiling")

    def kernel_times(self) -> dict:
        nk = len(KERNEL_KINDS)
        ms = (c_double * nk)()
        n = (ctypes.c_int64 * nk)()
        self._check(self.lib.gid_get_kernel_times(self.h, ms, n), "gid_get_kernel_times")
        return {k: dict(ms=ms[i], launches=n[i]) for i, k in enumerate(KERNEL_KINDS)}

    # -- checkpoint
    def save_state(self) -> bytes:
        n = c_size_t()
        self._check(self.lib.gid_save_state(self.h, None, byref(n)), "gid_save_state")
        buf = ctypes.create_string_buffer(n.value)
        self._check(self.lib.gid_save_state(self.h, buf, byref(n)), "gid_save_state")
        return buf.raw[: n.value]

    def load_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(self.lib.gid_load_state(self.h, buf, len(blob)), "gid_load_state")


def _f32(arr, n, name):
    a = np.ascontiguousarray(np.asarray(arr, np.float32).reshape(-1))
    if a.size != n:
        raise ValueError(f"{name} must have {n} values, got {a.size}")
    return a, a.ctypes.data_as(POINTER(c_float))


class Net:
    """The learned warm-start network for frames of width x height with K base colours."""

    def __init__(self, K: int, width: int, height: int, stream=None):
        import torch
        self.lib = load_library()
        self.K, self.W, self.H = int(K), int(width), int(height)
        self.n = self.K + 4
        self.nparam = int(self.lib.gid_net_num_params(self.K))
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        h = c_void_p()
        st = self.lib.gid_net_create(self.K, self.W, self.H, c_void_p(stream.cuda_stream), byref(h))
        if st != GID_OK:
            raise GidError(st, f"gid_net_create(K={self.K}, {self.W}x{self.H})")
        self.h = h

    def _check(self, st, what):
        if st != GID_OK:
            raise GidError(st, f"{what}: {self.lib.gid_net_last_error(self.h).decode()}")

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.gid_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        a, p = _f32(flat, self.nparam, "params")
        self._check(self.lib.gid_net_set_params(self.h, p, self.nparam), "gid_net_set_params")

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.nparam, np.float32)
        self._check(self.lib.gid_net_get_params(self.h, out.ctypes.data_as(POINTER(c_float)), self.nparam),
                    "gid_net_get_params")
        return out

    def forward(self, frame, u_prev, u_out):
        import torch
        f = _ptr(frame, torch.float32, (3, self.H, self.W), "frame")
        u = _ptr(u_prev, torch.float32, (self.n, self.H, self.W), "u_prev")
        o = _ptr(u_out, torch.float32, (self.n, self.H, self.W), "u_out")
        db = np.zeros(3 * self.K, np.float32)
        self._check(self.lib.gid_net_forward(self.h, f, u, o, db.ctypes.data_as(POINTER(c_float))),
                    "gid_net_forward")
        return db

    def gradients(self, frame, u_prev, du_target, db_target, w_b: float = 1.0):
        import torch
        f = _ptr(frame, torch.float32, (3, self.H, self.W), "frame")
        u = _ptr(u_prev, torch.float32, (self.n, self.H, self.W), "u_prev")
        t = _ptr(du_target, torch.float32, (self.n, self.H, self.W), "du_target")
        tdb, tp = _f32(db_target, 3 * self.K, "db_target")
        g = np.zeros(self.nparam, np.float32)
        loss = c_double()
        self._check(self.lib.gid_net_gradients(self.h, f, u, t, tp, float(w_b), g.ctypes.data_as(POINTER(c_float)),
                                               byref(loss)), "gid_net_gradients")
        return g, loss.value

    def train_step(self, frame, u_prev, du_target, db_target, lr: float, w_b: float = 1.0, want_loss=True):
        import torch
        f = _ptr(frame, torch.float32, (3, self.H, self.W), "frame")
        u = _ptr(u_prev, torch.float32, (self.n, self.H, self.W), "u_prev")
        t = _ptr(du_target, torch.float32, (self.n, self.H, self.W), "du_target")
        tdb, tp = _f32(db_target, 3 * self.K, "db_target")
        loss = c_double()
        self._check(self.lib.gid_net_train_step(self.h, f, u, t, tp, float(w_b), float(lr),
                                                byref(loss) if want_loss else None), "gid_net_train_step")
        return loss.value if want_loss else None

    def layer_forward(self, layer: int, x_nhwc, out_nhwc):
        import torch
        x = _ptr(x_nhwc, torch.bfloat16, (self.H, self.W, 32), "x")
        o = _ptr(out_nhwc, torch.float32, (self.H, self.W, 32), "out")
        self._check(self.lib.gid_net_layer_forward(self.h, int(layer), x, o), "gid_net_layer_forward")

    def layer_wgrad(self, layer: int, x_nhwc, gy_nhwc, cin: int, cout: int):
        import torch
        x = _ptr(x_nhwc, torch.bfloat16, (self.H, self.W, 32), "x")
        gy = _ptr(gy_nhwc, torch.bfloat16, (self.H, self.W, 32), "gy")
        gw = np.zeros(cout * cin * 9, np.float32)
        gb = np.zeros(cout, np.float32)
        self._check(self.lib.gid_net_layer_wgrad(self.h, int(layer), x, gy, gw.ctypes.data_as(POINTER(c_float)),
                                                 gb.ctypes.data_as(POINTER(c_float))), "gid_net_layer_wgrad")
        return gw.reshape(cout, cin, 3, 3), gb

    def set_conv_workgroups(self, workgroups: int):
        """At most this many convolution workgroups (0: the resident grid)."""
        self._check(self.lib.gid_net_set_conv_workgroups(self.h, int(workgroups)), "gid_net_set_conv_workgroups")


BATCH_LAUNCH = {"one": 0, "per_k": 1}


class Batch:
    """Clips of uneven size solved together: by default one launch per kernel per
    step over all clips whatever their K, or one launch per K."""

    def __init__(self, solvers):
        self.lib = load_library()
        self.solvers = list(solvers)
        n = len(self.solvers)
        arr = (c_void_p * n)(*[s.h.value for s in self.solvers])
        h = c_void_p()
        st = self.lib.gid_batch_create(arr, n, byref(h))
        if st != GID_OK:
            raise GidError(st, "gid_batch_create")
        self.h = h
        self._e = np.zeros(n)

    def _check(self, st, what):
        if st != GID_OK:
            raise GidError(st, f"{what}: {self.lib.gid_batch_last_error(self.h).decode()}")

    def step_async(self, frames, ids, layers=None):
        """frames[i] / ids[i]: tensors for active clips, None for finished ones."""
        import torch
        n = len(self.solvers)
        fp = (c_void_p * n)()
        ip = (c_void_p * n)()
        lp = (c_void_p * n)()
        for i, s in enumerate(self.solvers):
            if frames[i] is None:
                continue
            fp[i] = _ptr(frames[i], torch.float32, (3, s.H, s.W), "frame").value
            ip[i] = _ptr(ids[i], torch.uint8, (s.H, s.W), "ids").value
            if layers is not None and layers[i] is not None:
                lp[i] = _ptr(layers[i], torch.float32, (s.n, s.H, s.W), "layers").value
        self._check(self.lib.gid_batch_decompose(self.h, fp, ip, lp), "gid_batch_decompose")

    def synchronize(self):
        self._check(self.lib.gid_batch_synchronize(self.h, self._e.ctypes.data_as(POINTER(c_double))),
                    "gid_batch_synchronize")
        return self._e.copy()

    def step(self, frames, ids, layers=None):
        self.step_async(frames, ids, layers)
        return self.synchronize()

    def set_launch(self, mode: str):
        """'one' (every kernel one launch over all clips) or 'per_k' (one launch per K)."""
        self._check(self.lib.gid_batch_set_launch(self.h, BATCH_LAUNCH[mode]), "gid_batch_set_launch")

    @property
    def launch(self) -> str:
        m = c_int32()
        self._check(self.lib.gid_batch_get_launch(self.h, byref(m)), "gid_batch_get_launch")
        return {v: k for k, v in BATCH_LAUNCH.items()}[m.value]

    def autotune(self) -> str:
        """Time both launch layouts on the clips' loaded frames and keep the faster."""
        m = c_int32()
        self._check(self.lib.gid_batch_autotune(self.h, byref(m)), "gid_batch_autotune")
        return {v: k for k, v in BATCH_LAUNCH.items()}[m.value]

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.gid_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
