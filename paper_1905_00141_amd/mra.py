"""Python binding of libmra.so: argument marshalling only.

Every step of the likelihood runs in the library's HIP kernels.  Inputs may be
NumPy arrays (host) or torch CUDA tensors (device, float64); PyTorch is used
only for device memory and streams.  If the library is missing the import of
this module fails: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmra.so")

MRA_OK, MRA_EINVAL, MRA_ENOTPD, MRA_ENOMEM, MRA_EDEVICE, MRA_EDOMAIN = 0, -1, -2, -3, -4, -5
MRA_EXP, MRA_MATERN, MRA_GAUSS = 0, 1, 2
MRA_DEVICE_PTRS = 1 << 0
MRA_ELIM_DUPLICATES = 1 << 1
MRA_ALLOW_ZERO_NUGGET = 1 << 2
MRA_FURTHER_APPROX = 1 << 3  # r knots at the finest level too (the further approximation; no kriging)
MRA_FOLD_GRAM = 1 << 4
MRA_FOLD_FACTOR = 1 << 5

EXPORTED = ["mra_build_tree", "mra_loglik", "mra_loglik_terms", "mra_loglik_levels", "mra_loglik_status",
            "mra_loglik_noalloc",
            "mra_predict", "mra_free_tree", "mra_last_error",
            "mra_tree_info", "mra_tree_arrays", "mra_profile_enable", "mra_profile_read",
            "mra_autotune", "mra_set_plan", "mra_set_tile_shapes", "mra_set_chunk_multiple", "mra_bench_mfma_f64",
            "mra_mlp_create", "mra_mlp_set_scaling", "mra_mlp_forward", "mra_mlp_loss_grad",
            "mra_mlp_train_step", "mra_mlp_get_params", "mra_mlp_free"]
MLP_WIDTH = 128
MLP_NPARAM = 50177


class MraInfo(C.Structure):
    _fields_ = [("n_in", C.c_int64), ("n_nan", C.c_int64), ("n_elim", C.c_int64), ("n_used", C.c_int64),
                ("J", C.c_int32), ("M", C.c_int32), ("r", C.c_int32), ("r_hat", C.c_int32), ("P", C.c_int32),
                ("n_regions", C.c_int64), ("n_leaves", C.c_int64), ("leaf_min", C.c_int64),
                ("leaf_max", C.c_int64), ("n_gram_regions", C.c_int64), ("n_dup", C.c_int64),
                ("leaf_hist", C.c_int64 * 16)]


class TuneResult(C.Structure):
    _fields_ = [("levels", C.c_int32), ("small_max", C.c_int32), ("fold_max", C.c_int64 * 16),
                ("ms_before", C.c_double), ("ms_after", C.c_double), ("trials", C.c_int32),
                ("tile", C.c_int32 * 16)]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("level", C.c_int32), ("launches", C.c_int64), ("ms", C.c_double),
                ("flops", C.c_double)]


class MraError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libmra error {code}: {msg}")
        self.code = code


def load_library(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: run `python -m paper_1905_00141_amd.build` first")
    L = C.CDLL(path)
    vp, pd, i64 = C.c_void_p, C.c_void_p, C.c_int64
    L.mra_build_tree.argtypes = [pd, pd, pd, i64, C.c_int, C.c_int, C.c_int, C.c_double, C.c_uint32, pd,
                                 C.POINTER(vp)]
    L.mra_build_tree.restype = C.c_int
    L.mra_loglik.argtypes = [vp, C.c_int, C.c_double, pd, i64, pd, vp]
    L.mra_loglik.restype = C.c_int
    L.mra_loglik_terms.argtypes = [vp, C.c_int, C.c_double, pd, i64, pd, pd, pd, vp]
    L.mra_loglik_terms.restype = C.c_int
    L.mra_loglik_levels.argtypes = [vp, C.c_int, C.c_double, pd, i64, pd, pd, vp]
    L.mra_loglik_levels.restype = C.c_int
    L.mra_loglik_noalloc.argtypes = [vp, C.c_int, C.c_double, pd, i64, pd, vp]
    L.mra_loglik_noalloc.restype = C.c_int
    L.mra_loglik_status.argtypes = [vp]
    L.mra_loglik_status.restype = C.c_int
    L.mra_predict.argtypes = [vp, C.c_int, C.c_double, pd, pd, pd, i64, pd, pd, vp]
    L.mra_predict.restype = C.c_int
    L.mra_free_tree.argtypes = [vp]
    L.mra_free_tree.restype = None
    L.mra_last_error.argtypes = []
    L.mra_last_error.restype = C.c_char_p
    L.mra_tree_info.argtypes = [vp, C.POINTER(MraInfo)]
    L.mra_tree_info.restype = C.c_int
    L.mra_tree_arrays.argtypes = [vp, pd, pd, pd, pd, pd]
    L.mra_tree_arrays.restype = C.c_int
    L.mra_profile_enable.argtypes = [C.c_int, C.c_char_p, C.c_int]
    L.mra_profile_enable.restype = C.c_int
    L.mra_profile_read.argtypes = [C.POINTER(KernelStat), C.c_int, C.POINTER(C.c_int)]
    L.mra_profile_read.restype = C.c_int
    L.mra_autotune.argtypes = [vp, C.c_int, C.c_double, pd, i64, C.POINTER(TuneResult)]
    L.mra_autotune.restype = C.c_int
    L.mra_set_plan.argtypes = [vp, vp, C.c_int]
    L.mra_set_plan.restype = C.c_int
    L.mra_set_tile_shapes.argtypes = [vp, vp]
    L.mra_set_tile_shapes.restype = C.c_int
    L.mra_set_chunk_multiple.argtypes = [vp, i64]
    L.mra_set_chunk_multiple.restype = C.c_int
    L.mra_bench_mfma_f64.argtypes = [i64, C.POINTER(C.c_double)]
    L.mra_bench_mfma_f64.restype = C.c_int
    f32 = C.c_float
    L.mra_mlp_create.argtypes = [vp, C.POINTER(vp)]
    L.mra_mlp_create.restype = C.c_int
    L.mra_mlp_set_scaling.argtypes = [vp, pd, pd, C.c_double, C.c_double]
    L.mra_mlp_set_scaling.restype = C.c_int
    L.mra_mlp_forward.argtypes = [vp, vp, i64, pd, vp]
    L.mra_mlp_forward.restype = C.c_int
    L.mra_mlp_loss_grad.argtypes = [vp, vp, pd, i64, vp, pd, vp]
    L.mra_mlp_loss_grad.restype = C.c_int
    L.mra_mlp_train_step.argtypes = [vp, vp, pd, i64, f32, f32, f32, f32, pd, vp]
    L.mra_mlp_train_step.restype = C.c_int
    L.mra_mlp_get_params.argtypes = [vp, vp]
    L.mra_mlp_get_params.restype = C.c_int
    L.mra_mlp_free.argtypes = [vp]
    L.mra_mlp_free.restype = None
    return L


# PyTorch (device memory and streams for the callers) carries its own HIP
# runtime.  Loading it before this library's runtime keeps the process working
# whichever of the two initialises the GPU first; with the opposite load order
# this library's runtime can find no device once PyTorch has initialised it.
try:
    import torch  # noqa: F401
except ImportError:  # the library itself does not need it
    pass

_lib = load_library()


def _check(rc):
    if rc != 0:
        raise MraError(rc, _lib.mra_last_error().decode())


def _ptr(a):
    """Address of a contiguous float64 NumPy array or torch tensor."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags.c_contiguous and a.dtype == np.float64
        return a.ctypes.data
    assert a.is_contiguous() and str(a.dtype) == "torch.float64"
    return a.data_ptr()


def _stream_ptr(stream):
    if stream is None:
        return None
    return int(getattr(stream, "cuda_stream", stream))


def profile_enable(on: bool = True, only_kernel: str | None = None, only_level: int = -1):
    """Bracket launches of mra_loglik with HIP events (all, or one kernel at one level)."""
    _check(_lib.mra_profile_enable(1 if on else 0, None if only_kernel is None else only_kernel.encode(),
                                   only_level))


def profile_read():
    """Per (kernel, level): launches, total ms, algorithmic flops since the last read."""
    cap = 256
    buf = (KernelStat * cap)()
    cnt = C.c_int()
    _check(_lib.mra_profile_read(buf, cap, C.byref(cnt)))
    return [dict(name=buf[i].name.decode(), level=buf[i].level, launches=buf[i].launches, ms=buf[i].ms,
                 flops=buf[i].flops) for i in range(min(cnt.value, cap))]


def mfma_peak_tflops(iters: int = 4096) -> float:
    """Measured FP64 matrix-core rate of the device (mra_bench_mfma_f64)."""
    v = C.c_double()
    _check(_lib.mra_bench_mfma_f64(int(iters), C.byref(v)))
    return v.value


def family_code(family: str):
    return {"exp": MRA_EXP, "matern": MRA_MATERN, "gauss": MRA_GAUSS}[family]


class Tree:
    """Handle on a library-built MRA partition (mra_build_tree)."""

    def __init__(self, x, y, z, J=4, r=16, M=3, offset=0.0, flags=0, domain=None):
        dev = not isinstance(x, np.ndarray)
        if not dev:
            x = np.ascontiguousarray(x, dtype=np.float64)
            y = np.ascontiguousarray(y, dtype=np.float64)
            z = np.ascontiguousarray(z, dtype=np.float64)
            n = len(x)
        else:
            n = x.numel()
            flags |= MRA_DEVICE_PTRS
        dom = None if domain is None else np.ascontiguousarray(domain, dtype=np.float64)
        h = C.c_void_p()
        _check(_lib.mra_build_tree(_ptr(x), _ptr(y), _ptr(z), n, J, r, M, float(offset), flags,
                                   None if dom is None else dom.ctypes.data, C.byref(h)))
        self._h = h
        info = MraInfo()
        _check(_lib.mra_tree_info(h, C.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in MraInfo._fields_}
        self.info["leaf_hist"] = list(info.leaf_hist)
        self.n_used = info.n_used
        self.M, self.J, self.r_hat, self.P = info.M, info.J, info.r_hat, info.P

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib.mra_free_tree(h)
            self._h = None

    def arrays(self):
        n, nl = self.info["n_used"], self.info["n_leaves"]
        x, y, z = np.empty(n), np.empty(n), np.empty(n)
        orig = np.empty(n, dtype=np.int64)
        off = np.empty(nl + 1, dtype=np.int64)
        _check(_lib.mra_tree_arrays(self._h, x.ctypes.data, y.ctypes.data, z.ctypes.data, orig.ctypes.data,
                                    off.ctypes.data))
        return dict(x=x, y=y, z=z, orig=orig, leaf_off=off)

    def loglik(self, theta, family="matern", nu=0.5, out=None, stream=None):
        """theta: (B, 3) NumPy array (host) or float64 CUDA tensor (device)."""
        if isinstance(theta, np.ndarray) or not hasattr(theta, "data_ptr"):
            th = np.ascontiguousarray(np.atleast_2d(theta), dtype=np.float64)
            B = th.shape[0]
            res = np.empty(B) if out is None else out
        else:
            th = theta
            B = th.shape[0]
            if out is None:
                import torch
                out = torch.empty(B, dtype=torch.float64, device=th.device)
            res = out
        _check(_lib.mra_loglik(self._h, family_code(family), float(nu), _ptr(th), B, _ptr(res),
                               _stream_ptr(stream)))
        return res

    def level_logdets(self, theta, family="matern", nu=0.5):
        """(loglik (B,), per-level log-determinant sums (B, M)); host arrays."""
        th = np.ascontiguousarray(np.atleast_2d(theta), dtype=np.float64)
        ll, lev = np.empty(th.shape[0]), np.empty((th.shape[0], self.M))
        _check(_lib.mra_loglik_levels(self._h, family_code(family), float(nu), th.ctypes.data, th.shape[0],
                                      ll.ctypes.data, lev.ctypes.data, None))
        return ll, lev

    def loglik_noalloc(self, theta, out, family="matern", nu=0.5, stream=None):
        """mra_loglik_noalloc: device theta (B, 3) and device out (B,), no allocation."""
        _check(_lib.mra_loglik_noalloc(self._h, family_code(family), float(nu), _ptr(theta), theta.shape[0],
                                       _ptr(out), _stream_ptr(stream)))
        return out

    def status(self):
        """Wait for the most recent evaluation and raise MraError if it failed
        (mra_loglik_status; for calls made with device pointers)."""
        _check(_lib.mra_loglik_status(self._h))

    def autotune(self, theta, family="matern", nu=0.5):
        """Time candidate execution plans on a host sample of theta and install the fastest."""
        th = np.ascontiguousarray(np.atleast_2d(theta), dtype=np.float64)
        r = TuneResult()
        _check(_lib.mra_autotune(self._h, family_code(family), float(nu), th.ctypes.data, th.shape[0], C.byref(r)))
        return dict(fold_max=[int(r.fold_max[i]) for i in range(r.levels - 1)], small_max=int(r.small_max),
                    tile=[int(r.tile[i]) for i in range(r.levels - 1)],
                    ms_before=r.ms_before, ms_after=r.ms_after, trials=int(r.trials))

    def set_chunk_multiple(self, multiple):
        """Round the theta per chunk down to a multiple of `multiple`: for
        theta in consecutive groups that share alpha and range."""
        _check(_lib.mra_set_chunk_multiple(self._h, int(multiple)))

    def set_tile_shapes(self, tile=None):
        """Schur-block tile shape per level 1 .. M-1 (-1 default, 0 64 x 64, 1 128 x 128)."""
        if tile is None:
            _check(_lib.mra_set_tile_shapes(self._h, None))
            return
        tl = np.ascontiguousarray(tile, dtype=np.int32)
        assert tl.shape == (self.info["M"] - 1,)
        _check(_lib.mra_set_tile_shapes(self._h, tl.ctypes.data))

    def set_plan(self, fold_max=None, small_max=64):
        """Install an execution plan (per-level fold thresholds, -1 = default rule)."""
        if fold_max is None:
            _check(_lib.mra_set_plan(self._h, None, int(small_max)))
            return
        fm = np.ascontiguousarray(fold_max, dtype=np.int64)
        assert fm.shape == (self.info["M"] - 1,)
        _check(_lib.mra_set_plan(self._h, fm.ctypes.data, int(small_max)))

    def loglik_terms(self, theta, family="matern", nu=0.5, stream=None):
        """(loglik, logdet, quad) per theta; host arrays or device tensors like loglik."""
        if isinstance(theta, np.ndarray) or not hasattr(theta, "data_ptr"):
            th = np.ascontiguousarray(np.atleast_2d(theta), dtype=np.float64)
            B = th.shape[0]
            ll, ld, q = np.empty(B), np.empty(B), np.empty(B)
        else:
            import torch
            th = theta
            B = th.shape[0]
            ll, ld, q = (torch.empty(B, dtype=torch.float64, device=th.device) for _ in range(3))
        _check(_lib.mra_loglik_terms(self._h, family_code(family), float(nu), _ptr(th), B, _ptr(ll), _ptr(ld),
                                     _ptr(q), _stream_ptr(stream)))
        return ll, ld, q

    def predict(self, theta, px, py, family="matern", nu=0.5, stream=None):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        dev = not isinstance(px, np.ndarray)
        if dev:
            import torch
            mean = torch.empty_like(px)
            var = torch.empty_like(px)
            th = torch.tensor(th, dtype=torch.float64, device=px.device)
        else:
            px = np.ascontiguousarray(px, dtype=np.float64)
            py = np.ascontiguousarray(py, dtype=np.float64)
            mean, var = np.empty(len(px)), np.empty(len(px))
        _check(_lib.mra_predict(self._h, family_code(family), float(nu), _ptr(th), _ptr(px), _ptr(py), len(px),
                                _ptr(mean), _ptr(var), _stream_ptr(stream)))
        return mean, var


def _ptr32(a):
    """Address of a contiguous float32 NumPy array or torch tensor."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags.c_contiguous and a.dtype == np.float32
        return a.ctypes.data
    assert a.is_contiguous() and str(a.dtype) == "torch.float32"
    return a.data_ptr()


class Mlp:
    """Handle on the library's FP32 surrogate network (include/mra_mlp.h).

    x: (B, 3) float32 (log sill, log range, log nugget); y: (B,) float64.
    NumPy arrays (host) or torch CUDA tensors (device), not mixed."""

    def __init__(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (MLP_NPARAM,):
            raise ValueError(f"params must hold {MLP_NPARAM} values")
        h = C.c_void_p()
        _check(_lib.mra_mlp_create(p.ctypes.data, C.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.mra_mlp_free(h)
            self._h = None

    def set_scaling(self, x_lo, x_hi, y_mean, y_std):
        lo = np.ascontiguousarray(x_lo, dtype=np.float64)
        hi = np.ascontiguousarray(x_hi, dtype=np.float64)
        _check(_lib.mra_mlp_set_scaling(self._h, lo.ctypes.data, hi.ctypes.data, float(y_mean), float(y_std)))

    def forward(self, x, out=None, stream=None):
        B = x.shape[0]
        if out is None:
            if isinstance(x, np.ndarray):
                out = np.empty(B)
            else:
                import torch
                out = torch.empty(B, dtype=torch.float64, device=x.device)
        _check(_lib.mra_mlp_forward(self._h, _ptr32(x), B, _ptr(out), _stream_ptr(stream)))
        return out

    def loss_grad(self, x, y, stream=None):
        B = x.shape[0]
        if isinstance(x, np.ndarray):
            g, loss = np.empty(MLP_NPARAM, dtype=np.float32), np.empty(1)
        else:
            import torch
            g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=x.device)
            loss = torch.empty(1, dtype=torch.float64, device=x.device)
        _check(_lib.mra_mlp_loss_grad(self._h, _ptr32(x), _ptr(y), B, _ptr32(g), _ptr(loss), _stream_ptr(stream)))
        return loss, g

    def train_step(self, x, y, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        B = x.shape[0]
        if isinstance(x, np.ndarray):
            loss = np.empty(1)
        else:
            import torch
            loss = torch.empty(1, dtype=torch.float64, device=x.device)
        _check(_lib.mra_mlp_train_step(self._h, _ptr32(x), _ptr(y), B, lr, beta1, beta2, eps, _ptr(loss),
                                       _stream_ptr(stream)))
        return loss

    def params(self):
        p = np.empty(MLP_NPARAM, dtype=np.float32)
        _check(_lib.mra_mlp_get_params(self._h, p.ctypes.data))
        return p
