"""Python binding of libmhar (include/mhar.h): argument marshalling only.

Every step of the sampler runs in the HIP library.  The functions named
``mhar_*`` mirror the C entry points one to one (plain integers and device
pointers); ``Problem`` and ``Chains`` are thin conveniences that take torch
tensors on a HIP device, allocate the device workspaces with torch and pass
the current torch stream.  There is no fallback: if the library is missing
and cannot be built, importing the binding fails.
"""
from __future__ import annotations

import ctypes
import os

from . import build as _build

OK = 0
E_INVALID_ARG = -1
E_SHAPE = -2
E_RANK_DEFICIENT = -3
E_NOT_INTERIOR = -4
E_WORKSPACE = -5
E_HIP = -6
E_UNSUPPORTED = -7
E_STATE = -8

FP64 = 0
FP32 = 1
BF16X3 = 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}

CHAIN_UNBOUNDED = 1
CHAIN_DEGENERATE = 2
CHAIN_NONFINITE = 4
CHAIN_INFEASIBLE = 8
FIT_FAILED = 32

FIT_STATES = 0
FIT_DIKIN = 1
FITS = {"states": FIT_STATES, "dikin": FIT_DIKIN}


class MharError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("recompute_every", ctypes.c_int32),
                ("steps_per_launch", ctypes.c_int32), ("path", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]


class Trace(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 4), ("ms", ctypes.c_double * 4)]


TRACE_KINDS = ("screen", "chords", "dirs", "recompute")


class Tune(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("ms_per_step", ctypes.c_double * 5)]


class Stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_uint64), ("chain_steps", ctypes.c_uint64),
                ("exact_rows", ctypes.c_uint64), ("recomputes", ctypes.c_uint64),
                ("kernel", ctypes.c_int32), ("split", ctypes.c_int32)]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_st = ctypes.c_int32

# name -> (restype, argtypes), exactly the declarations of include/mhar.h
SIGNATURES = {
    "mhar_version": (ctypes.c_int32, []),
    "mhar_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "mhar_last_error": (ctypes.c_char_p, []),
    "mhar_options_default": (_st, [ctypes.POINTER(Options)]),
    "mhar_problem_workspace_size": (_st, [_i64, _i64, _i64, ctypes.POINTER(Options),
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "mhar_problem_create": (_st, [_i64, _i64, _vp, _vp, _i64, _vp, _vp, ctypes.POINTER(Options),
                                  _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    "mhar_problem_get_projection": (_st, [_vp, _vp, _vp]),
    "mhar_problem_destroy": (_st, [_vp]),
    "mhar_chains_workspace_size": (_st, [_vp, _i64, ctypes.POINTER(ctypes.c_size_t)]),
    "mhar_chains_create": (_st, [_vp, _i64, _vp, _u64, _u64, _vp, ctypes.c_size_t, _vp,
                                 ctypes.POINTER(_vp)]),
    "mhar_step": (_st, [_vp, _i64, _vp]),
    "mhar_record": (_st, [_vp, _i64, _i64, _i64, _vp, _vp]),
    "mhar_get_state": (_st, [_vp, _vp, _vp, _vp]),
    "mhar_set_state": (_st, [_vp, _vp, _u64, _vp]),
    "mhar_get_step": (_st, [_vp, ctypes.POINTER(_u64)]),
    "mhar_sync": (_st, [_vp, _vp, ctypes.POINTER(ctypes.c_int32)]),
    "mhar_get_stats": (_st, [_vp, _vp, ctypes.POINTER(Stats)]),
    "mhar_chains_destroy": (_st, [_vp]),
    "mhar_precond_workspace_size": (_st, [_vp, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "mhar_precond_create": (_st, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_size_t, _vp]),
    "mhar_precond_set": (_st, [_vp, _vp, _vp, _vp]),
    "mhar_precond_get": (_st, [_vp, _vp, _vp, _vp]),
    "mhar_precond_loss": (_st, [_vp, _vp, _vp, _vp, _vp]),
    "mhar_precond_train": (_st, [_vp, _i64, ctypes.c_double, _vp]),
    "mhar_run_noalloc": (_st, [_i64, _i64, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _u64, _u64,
                               _u64, _i64, ctypes.POINTER(Options), _vp]),
    "mhar_checkpoint": (_st, [_vp, _vp, ctypes.POINTER(ctypes.c_size_t), _vp]),
    "mhar_restore": (_st, [_vp, _vp, ctypes.c_size_t, _vp]),
    "mhar_trace_enable": (_st, [_vp, ctypes.c_int32]),
    "mhar_trace_read": (_st, [_vp, _vp, ctypes.POINTER(Trace)]),
    "mhar_precond_set_complement": (_st, [_vp, ctypes.c_double]),
    "mhar_precond_freeze": (_st, [_vp]),
    "mhar_precond_destroy": (_st, [_vp]),
    "mhar_batch_workspace_size": (_st, [ctypes.c_int32, ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_size_t)]),
    "mhar_batch_create": (_st, [ctypes.c_int32, ctypes.POINTER(_vp), _vp, ctypes.c_size_t,
                                ctypes.POINTER(_vp)]),
    "mhar_batch_step": (_st, [_vp, _i64, _vp]),
    "mhar_batch_packed_workspace_size": (_st, [ctypes.c_int32, _vp, _vp, _vp, ctypes.POINTER(Options),
                                               ctypes.POINTER(ctypes.c_size_t)]),
    "mhar_batch_create_packed": (_st, [ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                       _u64, ctypes.POINTER(Options), _vp, ctypes.c_size_t, _vp,
                                       ctypes.POINTER(_vp)]),
    "mhar_batch_get_chains": (_st, [_vp, ctypes.c_int32, ctypes.POINTER(_vp)]),
    "mhar_chains_set_graph": (_st, [_vp, ctypes.c_int32]),
    "mhar_chains_autotune": (_st, [_vp, _i64, _vp, ctypes.POINTER(Tune)]),
    "mhar_batch_destroy": (_st, [_vp]),
}

_lib = None


def library_path() -> str:
    return _build.LIB


def load(path: str | None = None):
    """Load libmhar (building it first only if no built library exists)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or _build.LIB
    if not os.path.exists(p):
        _build.build(p)
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _check(code: int):
    if code != OK:
        lib = load()
        raise MharError(code, lib.mhar_last_error().decode() or lib.mhar_status_string(code).decode())


def _make_module_functions():
    # module-level functions with the C names (marshalling only)
    def make(name):
        def f(*args):
            return getattr(load(), name)(*args)
        f.__name__ = name
        f.__doc__ = f"Calls {name} of libmhar (see include/mhar.h)."
        return f
    return {name: make(name) for name in SIGNATURES}


globals().update(_make_module_functions())


PATHS = {"auto": 0, "general": 1, "resident": 2, "tiled": 3, "lane": 4}


def options(precision="fp32", recompute_every=50, steps_per_launch=0, path="auto") -> Options:
    o = Options()
    _check(load().mhar_options_default(ctypes.byref(o)))
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.recompute_every = int(recompute_every)
    o.steps_per_launch = int(steps_per_launch)
    o.path = PATHS[path] if isinstance(path, str) else int(path)
    return o


def _stream(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _workspace(torch, nbytes, device):
    buf = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off, int(nbytes)


class Problem:
    """{x : A x <= b, A_eq x = b_eq} set up on the device (mhar_problem_create)."""

    def __init__(self, A, b, A_eq=None, b_eq=None, precision="fp32", recompute_every=50,
                 steps_per_launch=0, path="auto"):
        import torch
        self.torch = torch
        lib = load()
        self.device = A.device
        A = A.to(torch.float64).contiguous()
        b = b.to(torch.float64).contiguous()
        m, n = A.shape
        m_eq = 0
        if A_eq is not None:
            A_eq = A_eq.to(device=self.device, dtype=torch.float64).contiguous()
            b_eq = b_eq.to(device=self.device, dtype=torch.float64).contiguous()
            m_eq = A_eq.shape[0]
        self.n, self.m, self.m_eq = n, m, m_eq
        self.opt = options(precision, recompute_every, steps_per_launch, path)
        sz = ctypes.c_size_t()
        _check(lib.mhar_problem_workspace_size(n, m, m_eq, ctypes.byref(self.opt), ctypes.byref(sz)))
        self._ws, ptr, nbytes = _workspace(torch, sz.value, self.device)
        h = ctypes.c_void_p()
        _check(lib.mhar_problem_create(n, m, A.data_ptr(), b.data_ptr(), m_eq,
                                       A_eq.data_ptr() if m_eq else None,
                                       b_eq.data_ptr() if m_eq else None, ctypes.byref(self.opt),
                                       ptr, nbytes, _stream(torch, self.device), ctypes.byref(h)))
        self.handle = h

    def projection(self):
        P = self.torch.empty((self.n, self.n), dtype=self.torch.float64, device=self.device)
        _check(load().mhar_problem_get_projection(self.handle, P.data_ptr(),
                                                   _stream(self.torch, self.device)))
        return P

    def close(self):
        if getattr(self, "handle", None):
            _check(load().mhar_problem_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_noalloc(A, b, X, steps, seed=0, chain_offset=0, step0=0, A_eq=None, b_eq=None,
                precision="fp64", recompute_every=50, path="auto"):
    """mhar_run_noalloc on torch device tensors: X (z x n FP64, contiguous) is
    advanced in place; returns the per-walk status bits (int32 tensor)."""
    import torch
    lib = load()
    m, n = A.shape
    m_eq = 0 if A_eq is None else A_eq.shape[0]
    st = torch.empty(X.shape[0], dtype=torch.int32, device=X.device)
    o = options(precision, recompute_every, 0, path)
    s = _stream(torch, X.device)
    _check(lib.mhar_run_noalloc(n, m, A.data_ptr(), b.data_ptr(), m_eq,
                                None if A_eq is None else A_eq.data_ptr(),
                                None if b_eq is None else b_eq.data_ptr(), X.shape[0], X.data_ptr(),
                                st.data_ptr(), int(seed), int(chain_offset), int(step0), int(steps),
                                ctypes.byref(o), s))
    return st


class Chains:
    """z walks on a Problem (mhar_chains_create and the per-step calls)."""

    def __init__(self, problem: Problem, X0, seed=0, chain_offset=0):
        torch = problem.torch
        self.torch = torch
        self.problem = problem
        lib = load()
        X0 = X0.to(device=problem.device, dtype=torch.float64).contiguous()
        self.z = X0.shape[0]
        sz = ctypes.c_size_t()
        _check(lib.mhar_chains_workspace_size(problem.handle, self.z, ctypes.byref(sz)))
        self._ws, ptr, nbytes = _workspace(torch, sz.value, problem.device)
        h = ctypes.c_void_p()
        _check(lib.mhar_chains_create(problem.handle, self.z, X0.data_ptr(), seed, chain_offset, ptr,
                                      nbytes, _stream(torch, problem.device), ctypes.byref(h)))
        self.handle = h

    @property
    def stream(self):
        return _stream(self.torch, self.problem.device)

    def step(self, steps: int):
        _check(load().mhar_step(self.handle, int(steps), self.stream))

    def set_graph(self, graph_steps: int):
        _check(load().mhar_chains_set_graph(self.handle, int(graph_steps)))

    def autotune(self, steps_per_trial: int = 20) -> dict:
        """Time every kernel path this handle can take and keep the fastest
        (mhar_chains_autotune); returns the path kept and ms per step by path."""
        t = Tune()
        _check(load().mhar_chains_autotune(self.handle, int(steps_per_trial), self.stream,
                                           ctypes.byref(t)))
        names = {v: k for k, v in PATHS.items()}
        return {"path": names[t.path],
                "ms_per_step": {names[i]: t.ms_per_step[i] for i in range(5) if t.ms_per_step[i] >= 0}}

    def record(self, steps: int, stride: int, chain_count: int):
        out = self.torch.empty((int(steps) // int(stride), int(chain_count), self.problem.n),
                               dtype=self.torch.float64, device=self.problem.device)
        _check(load().mhar_record(self.handle, int(steps), int(stride), int(chain_count),
                                  out.data_ptr(), self.stream))
        return out

    def state(self):
        X = self.torch.empty((self.z, self.problem.n), dtype=self.torch.float64,
                             device=self.problem.device)
        st = self.torch.empty(self.z, dtype=self.torch.int32, device=self.problem.device)
        _check(load().mhar_get_state(self.handle, X.data_ptr(), st.data_ptr(), self.stream))
        return X, st

    def set_state(self, X, step: int):
        X = X.to(device=self.problem.device, dtype=self.torch.float64).contiguous()
        _check(load().mhar_set_state(self.handle, X.data_ptr(), int(step), self.stream))
        self._keep = X

    def step_count(self) -> int:
        v = ctypes.c_uint64()
        _check(load().mhar_get_step(self.handle, ctypes.byref(v)))
        return v.value

    def sync(self) -> int:
        f = ctypes.c_int32()
        _check(load().mhar_sync(self.handle, self.stream, ctypes.byref(f)))
        return f.value

    def stats(self) -> dict:
        s = Stats()
        _check(load().mhar_get_stats(self.handle, self.stream, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def checkpoint(self) -> bytes:
        lib = load()
        sz = ctypes.c_size_t()
        _check(lib.mhar_checkpoint(self.handle, None, ctypes.byref(sz), self.stream))
        buf = ctypes.create_string_buffer(sz.value)
        _check(lib.mhar_checkpoint(self.handle, buf, ctypes.byref(sz), self.stream))
        return buf.raw[:sz.value]

    def restore(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(load().mhar_restore(self.handle, buf, len(blob), self.stream))

    def trace_enable(self, max_launches: int):
        _check(load().mhar_trace_enable(self.handle, int(max_launches)))

    def trace_read(self) -> dict:
        t = Trace()
        _check(load().mhar_trace_read(self.handle, self.stream, ctypes.byref(t)))
        return {k: {"launches": t.launches[i], "ms": t.ms[i]} for i, k in enumerate(TRACE_KINDS)}

    # ---- learned direction covariance ----
    def precond_create(self, rank: int, objective: str = "states"):
        lib = load()
        fit = FITS[objective]
        sz = ctypes.c_size_t()
        _check(lib.mhar_precond_workspace_size(self.handle, int(rank), fit, ctypes.byref(sz)))
        self._pc_ws, ptr, nbytes = _workspace(self.torch, sz.value, self.problem.device)
        _check(lib.mhar_precond_create(self.handle, int(rank), fit, ptr, nbytes, self.stream))
        self.rank = int(rank)
        self.objective = objective

    def precond_set(self, U, log_sigma):
        t = self.torch
        U = U.to(device=self.problem.device, dtype=t.float64).contiguous()
        ls = log_sigma.to(device=self.problem.device, dtype=t.float64).contiguous()
        _check(load().mhar_precond_set(self.handle, U.data_ptr(), ls.data_ptr(), self.stream))
        t.cuda.current_stream(self.problem.device).synchronize()

    def precond_get(self):
        t = self.torch
        U = t.empty((self.problem.n, self.rank), dtype=t.float64, device=self.problem.device)
        ls = t.empty(self.problem.n, dtype=t.float64, device=self.problem.device)
        _check(load().mhar_precond_get(self.handle, U.data_ptr(), ls.data_ptr(), self.stream))
        return U, ls

    def precond_loss(self):
        t = self.torch
        nll = t.empty(1, dtype=t.float64, device=self.problem.device)
        gU = t.empty((self.problem.n, self.rank), dtype=t.float64, device=self.problem.device)
        gl = t.empty(self.problem.n, dtype=t.float64, device=self.problem.device)
        _check(load().mhar_precond_loss(self.handle, nll.data_ptr(), gU.data_ptr(), gl.data_ptr(),
                                        self.stream))
        return nll, gU, gl

    def precond_train(self, steps: int, lr: float):
        _check(load().mhar_precond_train(self.handle, int(steps), float(lr), self.stream))

    def precond_set_complement(self, kappa: float):
        _check(load().mhar_precond_set_complement(self.handle, float(kappa)))

    def precond_freeze(self):
        _check(load().mhar_precond_freeze(self.handle))

    def precond_destroy(self):
        _check(load().mhar_precond_destroy(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            _check(load().mhar_chains_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several Chains (each on its own Problem, one precision) stepped together in
    one persistent launch (mhar_batch_create / mhar_batch_step)."""

    def __init__(self, chains_list):
        torch = chains_list[0].torch
        self.torch = torch
        self.chains = list(chains_list)
        lib = load()
        arr = (ctypes.c_void_p * len(self.chains))(*[c.handle.value for c in self.chains])
        sz = ctypes.c_size_t()
        _check(lib.mhar_batch_workspace_size(len(self.chains), arr, ctypes.byref(sz)))
        dev = self.chains[0].problem.device
        self._ws, ptr, nbytes = _workspace(torch, sz.value, dev)
        h = ctypes.c_void_p()
        _check(lib.mhar_batch_create(len(self.chains), arr, ptr, nbytes, ctypes.byref(h)))
        self.handle = h
        self.device = dev

    def step(self, steps: int):
        _check(load().mhar_batch_step(self.handle, int(steps), _stream(self.torch, self.device)))

    def close(self):
        if getattr(self, "handle", None):
            _check(load().mhar_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PackedBatch:
    """Polytopes given as packed device arrays with host offsets, stepped as
    one batch (mhar_batch_create_packed); the batch owns its handles."""

    def __init__(self, n, m, z, A_packed, A_offsets, b_packed, b_offsets, X0_packed, X0_offsets,
                 seed=0, precision="fp32", recompute_every=50, path="auto"):
        import torch
        self.torch = torch
        self.device = A_packed.device
        self.n, self.m, self.z = [int(v) for v in n], [int(v) for v in m], [int(v) for v in z]
        count = len(self.n)
        i64 = lambda v: (ctypes.c_int64 * count)(*[int(x) for x in v])
        self._arrays = [i64(self.n), i64(self.m), i64(self.z), i64(A_offsets), i64(b_offsets),
                        i64(X0_offsets)]
        cn, cm, cz, ao, bo, xo = [ctypes.cast(a, _vp) for a in self._arrays]
        self.opt = options(precision, recompute_every, 0, path)
        lib = load()
        sz = ctypes.c_size_t()
        _check(lib.mhar_batch_packed_workspace_size(count, cn, cm, cz, ctypes.byref(self.opt),
                                                    ctypes.byref(sz)))
        self._ws, ptr, nbytes = _workspace(torch, sz.value, self.device)
        h = ctypes.c_void_p()
        f64 = lambda t: t.to(device=self.device, dtype=torch.float64).contiguous()
        A_packed, b_packed, X0_packed = f64(A_packed), f64(b_packed), f64(X0_packed)
        _check(lib.mhar_batch_create_packed(count, cn, cm, cz, A_packed.data_ptr(), ao, b_packed.data_ptr(),
                                            bo, X0_packed.data_ptr(), xo, int(seed), ctypes.byref(self.opt),
                                            ptr, nbytes, _stream(torch, self.device), ctypes.byref(h)))
        self.handle = h

    @classmethod
    def from_lists(cls, As, bs, X0s, **kw):
        """Pack per-problem tensors (A_i m_i x n_i, b_i, X0_i z_i x n_i)."""
        import torch
        def pack(ts):
            flat = [t.reshape(-1) for t in ts]
            offs = [0]
            for t in flat[:-1]:
                offs.append(offs[-1] + t.numel())
            return torch.cat(flat), offs
        Ap, Ao = pack(As)
        bp, bo = pack(bs)
        Xp, Xo = pack(X0s)
        return cls([a.shape[1] for a in As], [a.shape[0] for a in As], [x.shape[0] for x in X0s],
                   Ap, Ao, bp, bo, Xp, Xo, **kw)

    def chains_handle(self, i: int):
        h = ctypes.c_void_p()
        _check(load().mhar_batch_get_chains(self.handle, int(i), ctypes.byref(h)))
        return h

    def step(self, steps: int):
        _check(load().mhar_batch_step(self.handle, int(steps), _stream(self.torch, self.device)))

    def state(self, i: int):
        X = self.torch.empty((self.z[i], self.n[i]), dtype=self.torch.float64, device=self.device)
        st = self.torch.empty(self.z[i], dtype=self.torch.int32, device=self.device)
        _check(load().mhar_get_state(self.chains_handle(i), X.data_ptr(), st.data_ptr(),
                                     _stream(self.torch, self.device)))
        return X, st

    def close(self):
        if getattr(self, "handle", None):
            _check(load().mhar_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
