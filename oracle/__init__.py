"""Plain FP64 CPU oracle for Matrix Hit-and-Run (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding in ``paper_2104_07097_amd``) never touches it.

The C source ``mhar_ref.c`` is the oracle; this module builds it with gcc
(``-O2 -ffp-contract=off -fopenmp``, no fast-math) and wraps it with ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mhar_ref.c")
LIB = os.path.join(HERE, "libmhar_ref.so")

OK = 0
E_INVALID_ARG = -1
E_RANK_DEFICIENT = -3
E_NOT_INTERIOR = -4

CHAIN_UNBOUNDED = 1
CHAIN_DEGENERATE = 2
CHAIN_NONFINITE = 4
CHAIN_INFEASIBLE = 8

TAG_DIR = 0
TAG_THETA = 1
TAG_LOWRANK = 2
TAG_TRAIN = 4

_lib = None


def build(out: str = LIB, extra_flags: tuple = ()) -> str:
    """Compile the oracle into a shared library (always recompiles)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
           "-Wall", "-Wextra", *extra_flags, "-o", out, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def _bind(lib):
    d = ctypes.POINTER(ctypes.c_double)
    i32 = ctypes.POINTER(ctypes.c_int32)
    u32 = ctypes.POINTER(ctypes.c_uint32)
    i64, u64 = ctypes.c_int64, ctypes.c_uint64
    lib.mhar_ref_philox4x32_10.argtypes = [u32, u32, u32]
    lib.mhar_ref_philox4x32_10.restype = None
    lib.mhar_ref_uniform.argtypes = [u64, ctypes.c_uint32, u64, u64, ctypes.c_uint32, ctypes.c_int]
    lib.mhar_ref_uniform.restype = ctypes.c_double
    lib.mhar_ref_gauss.argtypes = [u64, ctypes.c_uint32, u64, u64, i64]
    lib.mhar_ref_gauss.restype = ctypes.c_double
    lib.mhar_ref_projection.argtypes = [i64, i64, d, d]
    lib.mhar_ref_projection.restype = ctypes.c_int
    lib.mhar_ref_check_interior.argtypes = [i64, i64, d, d, i64, d, d, i64, d]
    lib.mhar_ref_check_interior.restype = ctypes.c_int
    lib.mhar_ref_chord.argtypes = [i64, i64, d, d, d, d, d, d, i32]
    lib.mhar_ref_chord.restype = None
    lib.mhar_ref_direction.argtypes = [i64, d, i64, d, d, u64, u64, u64, d]
    lib.mhar_ref_direction.restype = None
    lib.mhar_ref_run.argtypes = [i64, i64, d, d, d, i64, d, d, i64, d, u64, u64, u64, i64,
                                 i32, i64, i64, d, ctypes.c_int]
    lib.mhar_ref_run.restype = ctypes.c_int
    lib.mhar_ref_precond_nll.argtypes = [i64, i64, d, d, i64, d, d, d, d]
    lib.mhar_ref_precond_nll.restype = ctypes.c_int
    lib.mhar_ref_precond_train_step.argtypes = [i64, i64, d, d, d, d, d, d, i64, d, i64,
                                                ctypes.c_double, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_double, d]
    lib.mhar_ref_precond_train_step.restype = ctypes.c_int
    lib.mhar_ref_adam.argtypes = [i64, d, d, d, d, i64, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double]
    lib.mhar_ref_adam.restype = None
    lib.mhar_ref_dikin_hessian.argtypes = [i64, i64, d, d, i64, d, d, d]
    lib.mhar_ref_dikin_hessian.restype = ctypes.c_int
    lib.mhar_ref_dikin_objective.argtypes = [i64, i64, d, d, d, d, d, d]
    lib.mhar_ref_dikin_objective.restype = ctypes.c_int
    lib.mhar_ref_dikin_train_step.argtypes = [i64, i64, d, d, i64, d, i64, d, d, d, ctypes.c_int,
                                              ctypes.c_double, ctypes.c_double, d]
    lib.mhar_ref_dikin_train_step.restype = ctypes.c_int
    return lib


def load(path: str | None = None, rebuild: bool = False):
    """Load (building first if needed) the oracle library."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None or rebuild:
        if rebuild or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = _bind(ctypes.CDLL(LIB))
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """Numpy-facing wrapper around one loaded copy of the oracle library."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load()

    def philox(self, ctr, key):
        c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
        k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
        out = (ctypes.c_uint32 * 4)()
        self.lib.mhar_ref_philox4x32_10(c, k, out)
        return [int(v) for v in out]

    def uniform(self, seed, tag, chain, step, block=0, which=0):
        return self.lib.mhar_ref_uniform(seed, tag, chain, step, block, which)

    def gauss(self, seed, tag, chain, step, j):
        return self.lib.mhar_ref_gauss(seed, tag, chain, step, j)

    def projection(self, n, A_eq):
        A_eq = _f64(A_eq)
        m_eq = 0 if A_eq is None else A_eq.shape[0]
        P = np.empty((n, n), dtype=np.float64)
        rc = self.lib.mhar_ref_projection(n, m_eq, _p(A_eq), _p(P))
        return rc, P

    def check_interior(self, A, b, X, A_eq=None, b_eq=None):
        A, b, X, A_eq, b_eq = map(_f64, (A, b, X, A_eq, b_eq))
        m, n = A.shape
        m_eq = 0 if A_eq is None else A_eq.shape[0]
        X = X.reshape(-1, n)
        return self.lib.mhar_ref_check_interior(n, m, _p(A), _p(b), m_eq, _p(A_eq), _p(b_eq),
                                                X.shape[0], _p(X))

    def chord(self, A, b, x, d):
        A, b, x, d = map(_f64, (A, b, x, d))
        m, n = A.shape
        lo = ctypes.c_double()
        hi = ctypes.c_double()
        fl = ctypes.c_int32()
        self.lib.mhar_ref_chord(n, m, _p(A), _p(b), _p(x), _p(d), ctypes.byref(lo),
                                ctypes.byref(hi), ctypes.byref(fl))
        return lo.value, hi.value, fl.value

    def direction(self, n, seed, chain, step, P=None, U=None, log_sigma=None):
        P, U, log_sigma = map(_f64, (P, U, log_sigma))
        r = 0 if U is None else U.shape[1]
        d = np.empty(n, dtype=np.float64)
        self.lib.mhar_ref_direction(n, _p(P), r, _p(U), _p(log_sigma), seed, chain, step, _p(d))
        return d

    def run(self, A, b, X0, steps, seed=0, P=None, chain_offset=0, step0=0, U=None,
            log_sigma=None, rec_stride=0, rec_chains=0, threads=0):
        """Advance the z chains in X0 (z x n) by `steps`; returns (X, status, rec)."""
        A, b, P, U, log_sigma = map(_f64, (A, b, P, U, log_sigma))
        m, n = A.shape
        X = np.array(X0, dtype=np.float64, copy=True).reshape(-1, n)
        z = X.shape[0]
        r = 0 if U is None else U.shape[1]
        status = np.zeros(z, dtype=np.int32)
        rec = None
        if rec_stride > 0:
            rec = np.zeros((steps // rec_stride, rec_chains, n), dtype=np.float64)
        rc = self.lib.mhar_ref_run(n, m, _p(A), _p(b), _p(P), r, _p(U), _p(log_sigma), z,
                                   _p(X), seed, chain_offset, step0, steps,
                                   status.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   rec_stride, rec_chains, _p(rec), threads)
        if rc != OK:
            raise RuntimeError(f"mhar_ref_run failed: {rc}")
        return X, status, rec

    def precond_nll(self, U, log_sigma, X):
        U, log_sigma, X = map(_f64, (U, log_sigma, X))
        n = log_sigma.shape[0]
        r = 0 if U is None else U.shape[1]
        X = X.reshape(-1, n)
        nll = ctypes.c_double()
        gU = np.zeros((n, max(r, 1)), dtype=np.float64)
        gl = np.zeros(n, dtype=np.float64)
        rc = self.lib.mhar_ref_precond_nll(n, r, _p(U), _p(log_sigma), X.shape[0], _p(X),
                                           ctypes.byref(nll), _p(gU), _p(gl))
        if rc != OK:
            raise RuntimeError(f"mhar_ref_precond_nll failed: {rc}")
        return nll.value, gU[:, :r], gl

    def precond_train_step(self, V, log_sigma, moments, X, t, lr, beta1=0.9, beta2=0.999,
                           eps=1e-8):
        """One scale-free Adam update; moments = (m1V, m2V, m1l, m2l).
        Returns (V, log_sigma, moments, U), all new arrays."""
        V, ls = (np.array(a, dtype=np.float64, copy=True) for a in (V, log_sigma))
        mom = [np.array(a, dtype=np.float64, copy=True) for a in moments]
        X = _f64(X).reshape(-1, ls.shape[0])
        n, r = V.shape
        U = np.empty_like(V)
        rc = self.lib.mhar_ref_precond_train_step(n, r, _p(V), _p(ls), *(_p(a) for a in mom),
                                                  X.shape[0], _p(X), t, lr, beta1, beta2, eps,
                                                  _p(U))
        if rc != OK:
            raise RuntimeError(f"mhar_ref_precond_train_step failed: {rc}")
        return V, ls, tuple(mom), U

    def adam(self, param, grad, m1, m2, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        param, grad, m1, m2 = (np.array(a, dtype=np.float64, copy=True) for a in
                               (param, grad, m1, m2))
        self.lib.mhar_ref_adam(param.size, _p(param), _p(grad), _p(m1), _p(m2), t, lr, beta1,
                               beta2, eps)
        return param, m1, m2

    def dikin_hessian(self, A, b, X):
        """(rc, xbar, H): the log-barrier Hessian at the mean of the states X."""
        A, b, X = map(_f64, (A, b, X))
        m, n = A.shape
        X = X.reshape(-1, n)
        xbar = np.empty(n)
        H = np.empty((n, n))
        rc = self.lib.mhar_ref_dikin_hessian(n, m, _p(A), _p(b), X.shape[0], _p(X), _p(xbar),
                                             _p(H))
        return rc, xbar, H

    def dikin_objective(self, U, log_sigma, H):
        """(K, grad_U, grad_log_sigma) of K = 1/2 tr(H Sigma) - 1/2 log det Sigma."""
        U, log_sigma, H = map(_f64, (U, log_sigma, H))
        n = log_sigma.shape[0]
        r = 0 if U is None else U.shape[1]
        K = ctypes.c_double()
        gU = np.zeros((n, max(r, 1)))
        gl = np.zeros(n)
        rc = self.lib.mhar_ref_dikin_objective(n, r, _p(U), _p(log_sigma), _p(H),
                                               ctypes.byref(K), _p(gU), _p(gl))
        if rc != OK:
            raise RuntimeError(f"mhar_ref_dikin_objective failed: {rc}")
        return K.value, gU[:, :r], gl

    def dikin_train_step(self, A, b, X, U, v, k_pow=8, eta=0.5, kappa=1.0):
        """One burn-in update towards the Dikin ellipsoid at mean(X), the
        diagonal scaled by kappa.  Returns (U, log_sigma, v, lam), all new arrays."""
        A, b, X = map(_f64, (A, b, X))
        m, n = A.shape
        X = X.reshape(-1, n)
        U = np.array(U, dtype=np.float64, copy=True)
        v = np.array(v, dtype=np.float64, copy=True)
        ls = np.empty(n)
        lam = ctypes.c_double()
        rc = self.lib.mhar_ref_dikin_train_step(n, m, _p(A), _p(b), X.shape[0], _p(X), U.shape[1],
                                                _p(U), _p(ls), _p(v), k_pow, eta, kappa,
                                                ctypes.byref(lam))
        if rc != OK:
            raise RuntimeError(f"mhar_ref_dikin_train_step failed: {rc}")
        return U, ls, v, lam.value
