"""Python binding of libmatexpre (the MatExPre hot path on one MI355X).

Argument marshalling only: every step of the computation runs in the HIP
library.  Functions carry the C-ABI names and take torch tensors (device
vectors), returning results or raising MxpError on a negative status.  The
library must have been built (paper_2506_03617_amd/build.py); importing this
module fails loudly if it is missing.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmatexpre.so")

MXP_OK = 0
MXP_NOT_CONVERGED = 1
MXP_ERR_INVALID_ARG = -1
MXP_ERR_OOM = -2
MXP_ERR_HIP = -3
MXP_ERR_BREAKDOWN = -4
MXP_ERR_NONFINITE = -5
MXP_ERR_UNSUPPORTED = -6

MXP_C64, MXP_C128, MXP_F32, MXP_F64 = 0, 1, 2, 3
MXP_PREC_FP64, MXP_PREC_MIXED = 0, 1
MXP_ABSORB_PML, MXP_ABSORB_CAP, MXP_ABSORB_ABC = 0, 1, 2
MXP_INNER_GMRES, MXP_INNER_FIXED_POINT, MXP_INNER_PSI2_GMRES, MXP_INNER_PSI2_FIXED_POINT = 0, 1, 2, 3


class MxpError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"status {status}: {message}")
        self.status = status


class mxp_grid_desc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("h", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("layer", (ctypes.c_int32 * 2) * 3),
        ("pml_C", ctypes.c_double),
        ("pml_power", ctypes.c_int32),
        ("c", ctypes.c_void_p),
        ("c_dtype", ctypes.c_int),
        ("c_const", ctypes.c_double),
        ("absorber", ctypes.c_int32),
        ("hard", (ctypes.c_int32 * 2) * 3),
    ]


class mxp_solve_opts(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double),
        ("shift", ctypes.c_double),
        ("fprtol", ctypes.c_double),
        ("rtol", ctypes.c_double),
        ("outer_restart", ctypes.c_int32),
        ("inner_restart", ctypes.c_int32),
        ("max_outer", ctypes.c_int32),
        ("max_inner", ctypes.c_int32),
        ("precision", ctypes.c_int),
        ("cheb_S", ctypes.c_int32),
        ("cheb_m", ctypes.c_int32),
        ("use_learned", ctypes.c_int32),
        ("stall_ratio", ctypes.c_double),
        ("use_graphs", ctypes.c_int32),
        ("inner_solver", ctypes.c_int32),
        ("fp64_below", ctypes.c_double),
        ("fp64_first", ctypes.c_int32),
    ]


class mxp_solve_stats(ctypes.Structure):
    _fields_ = [
        ("outer_its", ctypes.c_int32),
        ("inner_its_total", ctypes.c_int32),
        ("inner_mean", ctypes.c_double),
        ("inner_std", ctypes.c_double),
        ("stencil_steps", ctypes.c_int64),
        ("fn_actions", ctypes.c_int64),
        ("true_relres", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("restarts", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("learned_its", ctypes.c_int32),
        ("fallbacks", ctypes.c_int32),
        ("fp64_its", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class mxp_alloc_stats(ctypes.Structure):
    _fields_ = [
        ("allocs", ctypes.c_int64),
        ("frees", ctypes.c_int64),
        ("bytes_live", ctypes.c_int64),
        ("bytes_peak", ctypes.c_int64),
        ("late", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# device-memory hooks of mxp_context_create
MXP_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
MXP_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class mxp_schedule(ctypes.Structure):
    _fields_ = [
        ("S", ctypes.c_int32),
        ("m", ctypes.c_int32),
        ("m_psi", ctypes.c_int32),
        ("centre_re", ctypes.c_double),
        ("centre_im", ctypes.c_double),
        ("half_width", ctypes.c_double),
        ("box", ctypes.c_double * 4),
        ("trunc_bound", ctypes.c_double),
        ("similarity_cond", ctypes.c_double),
        ("amplification", ctypes.c_double),
        ("coef", ctypes.c_double * 1024),
        ("coef_psi", ctypes.c_double * 1024),
    ]

    def coefficients(self) -> np.ndarray:
        a = np.ctypeslib.as_array(self.coef)[: 2 * (self.m + 1)]
        return a[0::2] + 1j * a[1::2]

    def coefficients_psi(self) -> np.ndarray:
        a = np.ctypeslib.as_array(self.coef_psi)[: 2 * (self.m_psi + 1)]
        return a[0::2] + 1j * a[1::2]


# C-ABI symbols declared in include/matexpre.h
ABI_SYMBOLS = (
    "mxp_context_create", "mxp_context_destroy", "mxp_context_alloc_stats", "mxp_last_error", "mxp_version",
    "mxp_problem_create", "mxp_problem_destroy", "mxp_problem_size",
    "mxp_solve_opts_default", "mxp_design_schedule",
    "mxp_apply_A", "mxp_apply_exp", "mxp_apply_exp_noalloc", "mxp_apply_psi1", "mxp_apply_psi2", "mxp_apply_fn_krylov", "mxp_apply_precond", "mxp_solve",
    "mxp_set_tiles", "mxp_get_tiles", "mxp_solve_batch",
    "mxp_cnn_num_params", "mxp_cnn_create", "mxp_cnn_destroy", "mxp_cnn_get_params", "mxp_cnn_set_params",
    "mxp_cnn_get_grads", "mxp_cnn_get_activations", "mxp_cnn_forward", "mxp_cnn_backward", "mxp_cnn_train_step", "mxp_cnn_make_sample",
    "mxp_collect_pairs", "mxp_problem_set_learned", "mxp_cnn_save", "mxp_cnn_load", "mxp_solve_history",
)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2506_03617_amd/build.py`")
    # PyTorch ships its own HIP runtime under the same soname.  Loading torch
    # first makes the library bind to that one; loaded the other way round a
    # process holds two HIP/HSA runtimes and the second one finds no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    st = ctypes.c_int
    sig = {
        "mxp_context_create": (st, [ctypes.c_int, P, MXP_ALLOC_FN, MXP_FREE_FN, P, ctypes.POINTER(P)]),
        "mxp_context_alloc_stats": (st, [P, ctypes.POINTER(mxp_alloc_stats)]),
        "mxp_context_destroy": (None, [P]),
        "mxp_last_error": (ctypes.c_char_p, []),
        "mxp_version": (ctypes.c_char_p, []),
        "mxp_problem_create": (st, [P, ctypes.POINTER(mxp_grid_desc), ctypes.POINTER(P)]),
        "mxp_problem_destroy": (None, [P]),
        "mxp_problem_size": (ctypes.c_int64, [P]),
        "mxp_solve_opts_default": (st, [ctypes.POINTER(mxp_grid_desc), ctypes.POINTER(mxp_solve_opts)]),
        "mxp_design_schedule": (st, [ctypes.POINTER(mxp_grid_desc), ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, ctypes.POINTER(mxp_schedule)]),
        "mxp_apply_A": (st, [P, ctypes.c_double, ctypes.c_int, P, P]),
        "mxp_apply_exp": (st, [P, ctypes.c_double, ctypes.c_double, ctypes.c_int, P, P]),
        "mxp_apply_exp_noalloc": (st, [P, ctypes.c_double, ctypes.c_double, ctypes.c_int, P, P]),
        "mxp_apply_psi1": (st, [P, ctypes.c_double, ctypes.c_double, ctypes.c_int, P, P]),
        "mxp_apply_psi2": (st, [P, ctypes.c_double, ctypes.c_double, ctypes.c_int, P, P]),
        "mxp_apply_fn_krylov": (st, [P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int32, P, P, ctypes.POINTER(ctypes.c_int32)]),
        "mxp_apply_precond": (st, [P, ctypes.POINTER(mxp_solve_opts), ctypes.c_int, P, P,
                                   ctypes.POINTER(ctypes.c_int32)]),
        "mxp_solve": (st, [P, ctypes.POINTER(mxp_solve_opts), ctypes.c_int, P, P, ctypes.POINTER(mxp_solve_stats)]),
        "mxp_set_tiles": (st, [P, ctypes.c_int, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
        "mxp_get_tiles": (st, [P, ctypes.c_int, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
        "mxp_solve_batch": (st, [P, ctypes.c_int32, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(mxp_solve_opts),
                                 ctypes.c_int32, ctypes.POINTER(mxp_solve_stats)]),
        "mxp_cnn_num_params": (ctypes.c_int64, []),
        "mxp_cnn_create": (st, [P, ctypes.c_uint64, ctypes.POINTER(P)]),
        "mxp_cnn_destroy": (None, [P]),
        "mxp_cnn_get_params": (st, [P, P]),
        "mxp_cnn_set_params": (st, [P, P]),
        "mxp_cnn_get_grads": (st, [P, P]),
        "mxp_cnn_get_activations": (st, [P, ctypes.c_int32, ctypes.c_int64, P]),
        "mxp_cnn_save": (st, [P, ctypes.c_char_p]),
        "mxp_cnn_load": (st, [P, ctypes.c_char_p]),
        "mxp_cnn_forward": (st, [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P]),
        "mxp_cnn_backward": (st, [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P]),
        "mxp_cnn_train_step": (st, [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P,
                                    ctypes.c_float, ctypes.POINTER(ctypes.c_double)]),
        "mxp_cnn_make_sample": (st, [P, P, P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.c_double, ctypes.c_double, P, P]),
        "mxp_collect_pairs": (st, [P, ctypes.POINTER(mxp_solve_opts), P, P, ctypes.c_int32, P, P,
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(mxp_solve_stats)]),
        "mxp_problem_set_learned": (st, [P, P, ctypes.c_double]),
        "mxp_solve_history": (st, [P, ctypes.c_int32, P, P, ctypes.POINTER(ctypes.c_int32)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(status: int, allow_not_converged: bool = False) -> int:
    if status < 0 or (status == MXP_NOT_CONVERGED and not allow_not_converged):
        raise MxpError(status, lib.mxp_last_error().decode())
    return status


def mxp_version() -> str:
    return lib.mxp_version().decode()


def grid_desc(prob, c_host: Optional[np.ndarray] = None) -> mxp_grid_desc:
    """mxp_grid_desc from a workloads.Problem (c taken from prob.c as float64
    host array unless c_host is given).  The returned struct keeps a reference
    to the array it points at."""
    d = mxp_grid_desc()
    d.dim = prob.dim
    n = list(prob.n) + [1] * (3 - prob.dim)
    for a in range(3):
        d.n[a] = n[a]
    d.h = prob.h
    d.omega = prob.omega
    for a in range(3):
        L = prob.layer if a < prob.dim else 0
        d.layer[a][0] = L
        d.layer[a][1] = L
    d.pml_C = prob.pml_C
    d.pml_power = prob.pml_power
    d.absorber = {"pml": MXP_ABSORB_PML, "cap": MXP_ABSORB_CAP,
                  "abc": MXP_ABSORB_ABC}[getattr(prob, "absorber", "pml")]
    for a, side in getattr(prob, "hard_faces", ()):
        d.hard[a][side] = 1
    c = c_host if c_host is not None else prob.c
    if c is None:
        d.c = None
        d.c_dtype = MXP_F64
        d.c_const = prob.c_const
    else:
        arr = np.ascontiguousarray(c)
        if arr.dtype == np.float32:
            d.c_dtype = MXP_F32
        else:
            arr = np.ascontiguousarray(arr, dtype=np.float64)
            d.c_dtype = MXP_F64
        d._keep = arr
        d.c = arr.ctypes.data
        d.c_const = 0.0
    return d


def mxp_solve_opts_default(desc: mxp_grid_desc) -> mxp_solve_opts:
    o = mxp_solve_opts()
    _check(lib.mxp_solve_opts_default(ctypes.byref(desc), ctypes.byref(o)))
    return o


def mxp_design_schedule(desc: mxp_grid_desc, t: float, shift: float, precision: int) -> mxp_schedule:
    s = mxp_schedule()
    _check(lib.mxp_design_schedule(ctypes.byref(desc), t, shift, precision, ctypes.byref(s)))
    return s


def _ptr(tensor) -> int:
    return tensor.data_ptr()


def _dtype_of(tensor) -> int:
    import torch
    if tensor.dtype == torch.complex128:
        return MXP_C128
    if tensor.dtype == torch.complex64:
        return MXP_C64
    raise TypeError("vectors must be torch.complex64 or torch.complex128")


# Live handles, closed at interpreter exit before the HIP runtime goes away
# (problems first, then contexts).
_LIVE_PROBLEMS: "weakref.WeakSet" = weakref.WeakSet()
_LIVE_CONTEXTS: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _close_all():
    for obj in list(_LIVE_PROBLEMS):
        obj.close()
    for obj in list(_LIVE_CONTEXTS):
        obj.close()


class TorchAllocator:
    """mxp_context_create hooks backed by PyTorch's caching allocator: the
    library's workspaces come from the same pool as torch tensors, on the
    context's device and stream."""

    def __init__(self, device: int, stream):
        import torch
        self._torch = torch
        self.device = device
        self.stream = stream
        self.alloc = MXP_ALLOC_FN(self._alloc)
        self.free = MXP_FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        try:
            return self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
        except Exception:  # out of memory: the library reports MXP_ERR_OOM
            return None

    def _free(self, ptr, user):
        self._torch.cuda.caching_allocator_delete(ptr)


# Hooks stay alive for the whole process: problems and networks may outlive
# the Context object that made them.
_HOOKS = []


class Context:
    """mxp_context bound to a CUDA/HIP device and (by default) torch's current
    stream.  allocator: "torch" (default) takes the library's device memory
    from PyTorch's caching allocator, "hip" from hipMalloc, or pass an object
    with `alloc` / `free` attributes of types MXP_ALLOC_FN / MXP_FREE_FN."""

    def __init__(self, device: int = 0, stream=None, allocator="torch"):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        if allocator == "torch":
            allocator = TorchAllocator(device, stream)
        if allocator == "hip":
            self.allocator = None
            alloc, free = MXP_ALLOC_FN(), MXP_FREE_FN()
        else:
            self.allocator = allocator
            alloc, free = allocator.alloc, allocator.free
            _HOOKS.append(allocator)
        handle = ctypes.c_void_p()
        _check(lib.mxp_context_create(device, ctypes.c_void_p(stream.cuda_stream), alloc, free, None,
                                      ctypes.byref(handle)))
        self.handle = handle
        self.device = device
        _LIVE_CONTEXTS.add(self)

    def alloc_stats(self) -> dict:
        """Device allocations through this context (mxp_context_alloc_stats)."""
        out = mxp_alloc_stats()
        _check(lib.mxp_context_alloc_stats(self.handle, ctypes.byref(out)))
        return out.as_dict()

    def close(self):
        if self.handle:
            lib.mxp_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """mxp_problem for a workloads.Problem description."""

    def __init__(self, ctx: Context, prob):
        self.ctx = ctx
        self.desc = grid_desc(prob)
        self.spec = prob
        handle = ctypes.c_void_p()
        _check(lib.mxp_problem_create(ctx.handle, ctypes.byref(self.desc), ctypes.byref(handle)))
        self.handle = handle
        _LIVE_PROBLEMS.add(self)

    @property
    def size(self) -> int:
        return int(lib.mxp_problem_size(self.handle))

    def default_opts(self) -> mxp_solve_opts:
        return mxp_solve_opts_default(self.desc)

    def close(self):
        if self.handle:
            lib.mxp_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mxp_apply_A(prob: Problem, shift: float, x, y) -> None:
    _check(lib.mxp_apply_A(prob.handle, shift, _dtype_of(x), _ptr(x), _ptr(y)))


def mxp_apply_exp(prob: Problem, t: float, shift: float, x, y) -> None:
    _check(lib.mxp_apply_exp(prob.handle, t, shift, _dtype_of(x), _ptr(x), _ptr(y)))


def mxp_apply_exp_noalloc(prob: Problem, t: float, shift: float, x, y) -> None:
    """mxp_apply_exp that allocates no device memory (fixed 64 MiB scratch)."""
    _check(lib.mxp_apply_exp_noalloc(prob.handle, t, shift, _dtype_of(x), _ptr(x), _ptr(y)))


def mxp_apply_psi1(prob: Problem, t: float, shift: float, x, y) -> None:
    _check(lib.mxp_apply_psi1(prob.handle, t, shift, _dtype_of(x), _ptr(x), _ptr(y)))


def mxp_apply_psi2(prob: Problem, t: float, shift: float, x, y) -> None:
    _check(lib.mxp_apply_psi2(prob.handle, t, shift, _dtype_of(x), _ptr(x), _ptr(y)))


def mxp_apply_fn_krylov(prob: Problem, psi: bool, t: float, shift: float, tol: float, max_dim: int, x, y):
    """Arnoldi action (complex double).  Returns (status, basis size); status is
    MXP_OK or MXP_NOT_CONVERGED, other statuses raise."""
    import torch
    if x.dtype != torch.complex128 or y.dtype != torch.complex128:
        raise TypeError("mxp_apply_fn_krylov takes complex128 vectors")
    dim = ctypes.c_int32(0)
    st = lib.mxp_apply_fn_krylov(prob.handle, int(psi), t, shift, tol, max_dim, _ptr(x), _ptr(y), ctypes.byref(dim))
    return _check(st, allow_not_converged=True), dim.value


def _same_dtype(a, b) -> int:
    dt = _dtype_of(a)
    if _dtype_of(b) != dt:
        raise TypeError("both vectors must have the same dtype")
    return dt


def mxp_apply_precond(prob: Problem, opts: mxp_solve_opts, r, w) -> int:
    its = ctypes.c_int32(0)
    _check(lib.mxp_apply_precond(prob.handle, ctypes.byref(opts), _same_dtype(r, w), _ptr(r), _ptr(w),
                                 ctypes.byref(its)))
    return its.value


def mxp_solve(prob: Problem, opts: mxp_solve_opts, f, u) -> dict:
    st = mxp_solve_stats()
    status = _check(lib.mxp_solve(prob.handle, ctypes.byref(opts), _same_dtype(f, u), _ptr(f), _ptr(u),
                                  ctypes.byref(st)),
                    allow_not_converged=True)
    out = st.as_dict()
    out["status"] = status
    return out


def mxp_solve_batch(ctx: Context, problems, opts, f_list, u_list, max_resident: int = 0):
    """Batched solve: problems[q] with options opts[q]; f_list[q] / u_list[q]
    are complex128 device tensors holding nrhs_q right-hand sides / solutions
    back to back (shape (nrhs_q, size) or flat).  Returns (status, list of
    per-right-hand-side stats dicts, in order)."""
    nprob = len(problems)
    sizes = [p.size for p in problems]
    nrhs = [int(f.numel()) // n for f, n in zip(f_list, sizes)]
    for f, u, n, k in zip(f_list, u_list, sizes, nrhs):
        if f.numel() != k * n or u.numel() != k * n:
            raise ValueError("f and u must hold a whole number of right-hand sides")
        if _dtype_of(f) != MXP_C128 or _dtype_of(u) != MXP_C128:
            raise ValueError("batched solves take complex128 tensors")
    Parr = (ctypes.c_void_p * nprob)(*[p.handle.value for p in problems])
    Narr = (ctypes.c_int32 * nprob)(*nrhs)
    Farr = (ctypes.c_void_p * nprob)(*[_ptr(f) for f in f_list])
    Uarr = (ctypes.c_void_p * nprob)(*[_ptr(u) for u in u_list])
    Oarr = (mxp_solve_opts * nprob)(*opts)
    total = sum(nrhs)
    Sarr = (mxp_solve_stats * max(total, 1))()
    status = _check(lib.mxp_solve_batch(ctx.handle, nprob, Parr, Narr, Farr, Uarr, Oarr, max_resident, Sarr),
                    allow_not_converged=True)
    return status, [Sarr[k].as_dict() for k in range(total)]


class Network:
    """mxp_cnn: the learned stage's network on a context's device and stream."""

    def __init__(self, ctx: Context, seed: int = 0):
        self.ctx = ctx
        handle = ctypes.c_void_p()
        _check(lib.mxp_cnn_create(ctx.handle, seed, ctypes.byref(handle)))
        self.handle = handle
        _LIVE_PROBLEMS.add(self)

    @staticmethod
    def num_params() -> int:
        return int(lib.mxp_cnn_num_params())

    def get_params(self) -> np.ndarray:
        a = np.empty(self.num_params(), dtype=np.float32)
        _check(lib.mxp_cnn_get_params(self.handle, a.ctypes.data))
        return a

    def set_params(self, a) -> None:
        a = np.ascontiguousarray(a, dtype=np.float32)
        if a.size != self.num_params():
            raise ValueError("wrong parameter count")
        _check(lib.mxp_cnn_set_params(self.handle, a.ctypes.data))

    def get_grads(self) -> np.ndarray:
        a = np.empty(self.num_params(), dtype=np.float32)
        _check(lib.mxp_cnn_get_grads(self.handle, a.ctypes.data))
        return a

    def get_activations(self, layer: int, voxels: int) -> np.ndarray:
        """bf16 bits [voxels, 32] of hidden layer `layer` (1..5) from the last
        backward or training step."""
        a = np.empty((voxels, 32), dtype=np.uint16)
        _check(lib.mxp_cnn_get_activations(self.handle, layer, voxels, a.ctypes.data))
        return a

    def save(self, path) -> None:
        """Parameters and Adam state to a checkpoint file."""
        _check(lib.mxp_cnn_save(self.handle, os.fsencode(path)))

    def load(self, path) -> None:
        """Parameters and Adam state from a checkpoint file."""
        _check(lib.mxp_cnn_load(self.handle, os.fsencode(path)))

    def forward(self, shape, x, out) -> None:
        nb, nz, ny, nx = shape
        _check(lib.mxp_cnn_forward(self.handle, nb, nz, ny, nx, _ptr(x), _ptr(out)))

    def backward(self, shape, x, gout) -> None:
        nb, nz, ny, nx = shape
        _check(lib.mxp_cnn_backward(self.handle, nb, nz, ny, nx, _ptr(x), _ptr(gout)))

    def train_step(self, shape, x, target, lr: float) -> float:
        nb, nz, ny, nx = shape
        loss = ctypes.c_double()
        _check(lib.mxp_cnn_train_step(self.handle, nb, nz, ny, nx, _ptr(x), _ptr(target), lr, ctypes.byref(loss)))
        return loss.value

    def close(self):
        if self.handle:
            lib.mxp_cnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mxp_solve_history(prob: Problem):
    """Inner iterations and relative residual estimate of every outer
    iteration of the last single solve on `prob`."""
    n = ctypes.c_int32()
    _check(lib.mxp_solve_history(prob.handle, 0, None, None, ctypes.byref(n)))
    inner = np.zeros(n.value, dtype=np.int32)
    res = np.zeros(n.value, dtype=np.float64)
    if n.value:
        _check(lib.mxp_solve_history(prob.handle, n.value, inner.ctypes.data, res.ctypes.data, ctypes.byref(n)))
    return inner.tolist(), res.tolist()


def mxp_cnn_make_sample(prob: Problem, r, z, offset, crop, rscale: float, zscale: float, x, target) -> None:
    off = (ctypes.c_int32 * 3)(*offset)
    cr = (ctypes.c_int32 * 3)(*crop)
    _check(lib.mxp_cnn_make_sample(prob.handle, _ptr(r), _ptr(z), off, cr, rscale, zscale, _ptr(x), _ptr(target)))


def mxp_collect_pairs(prob: Problem, opts: mxp_solve_opts, f, u, r_out, z_out, max_pairs: int):
    """Solve while copying (v_j, M(v_j)) pairs into r_out / z_out (complex128
    device tensors of max_pairs * size values).  Returns (count, |r| list,
    |z| list, stats dict)."""
    rn = (ctypes.c_double * max(max_pairs, 1))()
    zn = (ctypes.c_double * max(max_pairs, 1))()
    cnt = ctypes.c_int32()
    st = mxp_solve_stats()
    status = _check(lib.mxp_collect_pairs(prob.handle, ctypes.byref(opts), _ptr(f), _ptr(u), max_pairs,
                                          _ptr(r_out), _ptr(z_out), rn, zn, ctypes.byref(cnt), ctypes.byref(st)),
                    allow_not_converged=True)
    out = st.as_dict()
    out["status"] = status
    return cnt.value, list(rn[:cnt.value]), list(zn[:cnt.value]), out


def mxp_problem_set_learned(prob: Problem, net, out_scale: float) -> None:
    _check(lib.mxp_problem_set_learned(prob.handle, net.handle if net is not None else None, out_scale))


def mxp_set_tiles(prob: Problem, precision: int, K: int, NX: int, Ly: int) -> None:
    _check(lib.mxp_set_tiles(prob.handle, precision, K, NX, Ly))


def mxp_get_tiles(prob: Problem, precision: int) -> dict:
    K, NX, Ly = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    us = ctypes.c_double()
    _check(lib.mxp_get_tiles(prob.handle, precision, ctypes.byref(K), ctypes.byref(NX), ctypes.byref(Ly),
                             ctypes.byref(us)))
    return {"K": K.value, "NX": NX.value, "Ly": Ly.value, "us_per_level": us.value}
