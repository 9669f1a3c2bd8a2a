"""ctypes wrapper around the plain-C MRA oracle (``mra_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module; the product path never
does.  It shares no code with the HIP library.

The oracle follows the paper's definitions (Sec. 1.1, remainder covariances
and the predictive-process expansion; Sec. 1.2, partition and knots) and the
prior/posterior recursion derived from them.  See ``mra_oracle.c`` for the
formulas.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mra_oracle.c")
_LIB = os.path.join(_HERE, "libmra_oracle.so")

EXP, MATERN, GAUSS = 0, 1, 2
ELIM_DUPLICATES = 1 << 1
ALLOW_ZERO_NUGGET = 1 << 2
FURTHER_APPROX = 1 << 3  # r knots at the finest level too (the further approximation)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        d, i64, vp = C.c_double, C.c_int64, C.c_void_p
        pd = C.POINTER(C.c_double)
        L.oracle_mra_build_tree.argtypes = [pd, pd, pd, i64, C.c_int, C.c_int, C.c_int, d,
                                            C.c_uint32, pd, C.POINTER(vp)]
        L.oracle_mra_free_tree.argtypes = [vp]
        L.oracle_mra_free_tree.restype = None
        L.oracle_tree_dims.argtypes = [vp, C.POINTER(C.c_int64)]
        L.oracle_tree_arrays.argtypes = [vp, pd, pd, pd, C.POINTER(C.c_int64),
                                         C.POINTER(C.c_int64), pd]
        L.oracle_mra_loglik.argtypes = [vp, C.c_int, d, pd, i64, pd, pd]
        L.oracle_dense_sigma.argtypes = [vp, C.c_int, d, pd, pd]
        L.oracle_dense_loglik.argtypes = [vp, C.c_int, d, pd, pd]
        L.oracle_exact_loglik.argtypes = [vp, C.c_int, d, pd, pd]
        L.oracle_box_knots.argtypes = [d, d, d, d, C.c_int, d, pd, pd]
        L.oracle_grid_dims.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.oracle_last_error.restype = C.c_char_p
        if hasattr(L, "oracle_mra_predict"):
            L.oracle_mra_predict.argtypes = [vp, C.c_int, d, pd, pd, pd, i64, pd, pd]
            L.oracle_dense_predict.argtypes = [vp, C.c_int, d, pd, pd, pd, i64, pd, pd]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != 0:
        raise OracleError(rc, lib().oracle_last_error().decode())


def grid_dims(r: int):
    nx, ny = C.c_int(), C.c_int()
    _check(lib().oracle_grid_dims(r, C.byref(nx), C.byref(ny)))
    return nx.value, ny.value


def box_knots(box, r, offset):
    nx, ny = grid_dims(r)
    kx = np.empty(nx * ny)
    ky = np.empty(nx * ny)
    _check(lib().oracle_box_knots(float(box[0]), float(box[1]), float(box[2]), float(box[3]),
                                  r, float(offset), _p(kx), _p(ky)))
    return kx, ky


class Tree:
    """An oracle partition tree (Sec. 1.2)."""

    def __init__(self, x, y, z, J=4, r=16, M=3, offset=0.0, flags=0, domain=None):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        z = np.ascontiguousarray(z, dtype=np.float64)
        dom = None if domain is None else np.ascontiguousarray(domain, dtype=np.float64)
        h = C.c_void_p()
        _check(lib().oracle_mra_build_tree(_p(x), _p(y), _p(z), len(x), J, r, M, float(offset),
                                           flags, None if dom is None else _p(dom), C.byref(h)))
        self._h = h
        self.J, self.M, self.r = J, M, r
        dims = (C.c_int64 * 10)()
        lib().oracle_tree_dims(h, dims)
        (self.n_in, self.n_nan, self.n_elim, self.n_used, self.nreg, self.nleaf,
         self.rhat, self.nx, self.ny, self.n_dup) = [int(v) for v in dims]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.oracle_mra_free_tree(h)
            self._h = None

    def arrays(self):
        n = self.n_used
        x, y, z = np.empty(n), np.empty(n), np.empty(n)
        orig = np.empty(n, dtype=np.int64)
        off = np.empty(self.nleaf + 1, dtype=np.int64)
        box = np.empty((self.nreg, 4))
        lib().oracle_tree_arrays(self._h, _p(x), _p(y), _p(z),
                                 orig.ctypes.data_as(C.POINTER(C.c_int64)),
                                 off.ctypes.data_as(C.POINTER(C.c_int64)), _p(box))
        return dict(x=x, y=y, z=z, orig=orig, leaf_off=off, box=box)

    def loglik(self, theta, family=MATERN, nu=0.5, level_sums=False):
        th = np.ascontiguousarray(np.atleast_2d(theta), dtype=np.float64)
        B = th.shape[0]
        out = np.empty(B)
        ls = np.empty((B, self.M)) if level_sums else None
        _check(lib().oracle_mra_loglik(self._h, family, float(nu), _p(th), B, _p(out),
                                       None if ls is None else _p(ls)))
        return (out, ls) if level_sums else out

    def level_logdets(self, theta, family=MATERN, nu=0.5):
        """(B, M): per level, the sum of the regions' log-determinant terms."""
        th = np.ascontiguousarray(np.atleast_2d(theta), dtype=np.float64)
        out = np.empty((th.shape[0], self.M))
        L = lib()
        L.oracle_mra_level_logdets.argtypes = [C.c_void_p, C.c_int, C.c_double, C.POINTER(C.c_double), C.c_int64,
                                               C.POINTER(C.c_double)]
        _check(L.oracle_mra_level_logdets(self._h, family, float(nu), _p(th), th.shape[0], _p(out)))
        return out

    def dense_sigma(self, theta, family=MATERN, nu=0.5):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        S = np.empty((self.n_used, self.n_used))
        _check(lib().oracle_dense_sigma(self._h, family, float(nu), _p(th), _p(S)))
        return S

    def dense_loglik(self, theta, family=MATERN, nu=0.5):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        out = C.c_double()
        _check(lib().oracle_dense_loglik(self._h, family, float(nu), _p(th), C.byref(out)))
        return out.value

    def exact_loglik(self, theta, family=MATERN, nu=0.5):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        out = C.c_double()
        _check(lib().oracle_exact_loglik(self._h, family, float(nu), _p(th), C.byref(out)))
        return out.value

    def predict(self, theta, px, py, family=MATERN, nu=0.5, dense=False):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        px = np.ascontiguousarray(px, dtype=np.float64)
        py = np.ascontiguousarray(py, dtype=np.float64)
        mean, var = np.empty(len(px)), np.empty(len(px))
        f = lib().oracle_dense_predict if dense else lib().oracle_mra_predict
        _check(f(self._h, family, float(nu), _p(th), _p(px), _p(py), len(px), _p(mean), _p(var)))
        return mean, var


def subtree_du(tree: Tree, theta, level: int, k: int, family=MATERN, nu=0.5) -> float:
    """Sum of d + u over one subtree (bounded piece of an evaluation, for timing)."""
    L = lib()
    if not hasattr(L, "_subtree_typed"):
        L.oracle_mra_subtree.argtypes = [C.c_void_p, C.c_int, C.c_double, C.POINTER(C.c_double), C.c_int,
                                         C.c_int64, C.POINTER(C.c_double)]
        L._subtree_typed = True
    th = np.ascontiguousarray(theta, dtype=np.float64)
    out = C.c_double()
    _check(L.oracle_mra_subtree(tree._h, family, float(nu), _p(th), level, k, C.byref(out)))
    return out.value
