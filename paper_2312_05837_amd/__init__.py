"""Python binding of libising.so (include/ising.h): argument marshalling only.

Every function here has the name of the C entry point it calls.  Device
buffers are torch tensors on the GPU (torch supplies memory and the current
stream); all work runs in the library's HIP kernels.  Importing this package
fails loudly when the built library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Optional

# torch provides device memory and streams; import it first so that the HIP
# runtime it loads is the one this library binds to (a single runtime per process)
import torch  # noqa: E402,F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libising.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2312_05837_amd.build` "
                      "(or __graft_entry__.build()); there is no CPU fallback")
_lib = C.CDLL(LIB_PATH)

ISING_OK, ISING_EINVAL, ISING_ENOMEM, ISING_EDEVICE, ISING_EBUSY, ISING_ETIMEDOUT, ISING_ECANCELED, \
    ISING_ENOTSUP = range(8)
ISING_DENSE, ISING_CSR = 0, 1
ISING_I32, ISING_F32, ISING_F64 = 0, 1, 2
ISING_OPT_GD, ISING_OPT_ADAM = 0, 1
ISING_LOSS_VERTEX, ISING_LOSS_RELAXED = 0, 1
ISING_PREC_FP64, ISING_PREC_FP32, ISING_PREC_BF16X2, ISING_PREC_BF16, ISING_PREC_FP8 = 0, 1, 2, 3, 4
ISING_PREC_I8X3, ISING_PREC_I8X2 = 5, 6

STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "EBUSY", 5: "ETIMEDOUT",
                6: "ECANCELED", 7: "ENOTSUP"}


class IsingError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ising_problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("format", C.c_int32), ("value_type", C.c_int32), ("reserved0", C.c_int32),
                ("nnz", C.c_int64), ("J", C.c_void_p), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p), ("h", C.c_void_p)]


class ising_params(C.Structure):
    _fields_ = [("replicas", C.c_int32), ("steps", C.c_int32), ("optimizer", C.c_int32),
                ("precision", C.c_int32), ("lr", C.c_double), ("mu", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double), ("seed", C.c_uint64), ("prune", C.c_int32),
                ("loss", C.c_int32), ("conv_window", C.c_int32), ("reserved1", C.c_int32),
                ("conv_tol", C.c_double)]


class ising_stats(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_G", C.c_int32), ("rounds", C.c_int32), ("best_replica", C.c_int32),
                ("steps", C.c_int64), ("best_step", C.c_int32), ("converged", C.c_int32), ("eta", C.c_double),
                ("constant_C", C.c_double), ("t_upload_ms", C.c_double), ("t_prune_ms", C.c_double),
                ("t_ds_ms", C.c_double), ("t_finish_ms", C.c_double), ("t_total_ms", C.c_double),
                ("replica_spin_updates_per_s", C.c_double), ("t_ds_kernel_ms", C.c_double),
                ("mean_steps_run", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if not k.startswith("reserved")}


class ising_ds_state(C.Structure):
    _fields_ = [("theta", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p), ("s_best", C.c_void_p),
                ("e_best", C.c_void_p), ("best_step", C.c_void_p), ("energy_trace", C.c_void_p),
                ("loss_trace", C.c_void_p), ("conv_step", C.c_void_p), ("conv_state", C.c_void_p)]


class ising_serve_config(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_resident", C.c_int32), ("chunk_steps", C.c_int32),
                ("dense_streams", C.c_int32), ("no_graphs", C.c_int32)]


class ising_serve_info(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("admitted", C.c_uint64), ("completed", C.c_uint64),
                ("canceled", C.c_uint64), ("failed", C.c_uint64), ("chunks", C.c_uint64), ("launches", C.c_uint64),
                ("resident", C.c_int32), ("queued", C.c_int32), ("bytes_in_use", C.c_size_t),
                ("busy_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = C.c_void_p
_sigs = {
    "ising_create": (C.c_int, [C.c_int, C.POINTER(C.c_void_p)]),
    "ising_destroy": (C.c_int, [_P]),
    "ising_last_error": (C.c_char_p, [_P]),
    "ising_solve": (C.c_int, [_P, C.POINTER(ising_problem), C.POINTER(ising_params), _P, C.POINTER(C.c_double),
                              C.POINTER(C.c_int64), C.POINTER(ising_stats)]),
    "ising_solve_dev": (C.c_int, [_P, C.POINTER(ising_problem), C.POINTER(ising_params), _P, _P, _P,
                                  C.POINTER(ising_stats), _P]),
    "ising_last_kernel": (C.c_char_p, [_P]),
    "ising_energy": (C.c_int, [_P, C.POINTER(ising_problem), _P, C.c_int32, _P, _P]),
    "ising_energy_dev": (C.c_int, [_P, C.POINTER(ising_problem), _P, C.c_int32, _P, _P, _P]),
    "ising_energy_dev_noalloc": (C.c_int, [_P, C.POINTER(ising_problem), _P, C.c_int32, _P, _P, _P]),
    "ising_prune": (C.c_int, [_P, C.POINTER(ising_problem), C.POINTER(C.c_void_p)]),
    "ising_unprune": (C.c_int, [_P, _P, _P]),
    "ising_pruned_record": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "ising_pruned_copy": (C.c_int, [_P, _P, _P, _P, _P]),
    "ising_prune_dev": (C.c_int, [_P, C.POINTER(ising_problem), C.POINTER(C.c_void_p), _P]),
    "ising_pruned_free": (None, [_P]),
    "ising_pruned_info": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "ising_pruned_record_dev": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "ising_pruned_problem": (C.c_int, [_P, C.POINTER(ising_problem)]),
    "ising_pruned_copy_dev": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "ising_unprune_dev": (C.c_int, [_P, _P, _P, _P, _P]),
    "ising_ds_dev": (C.c_int, [_P, C.POINTER(ising_problem), C.POINTER(ising_params), _P, C.c_int32, C.c_int32,
                               C.POINTER(ising_ds_state), _P]),
    "ising_ds_max_n": (C.c_int32, [C.c_int32]),
    "ising_ds_dense_dev": (C.c_int, [_P, C.POINTER(ising_problem), C.POINTER(ising_params), _P, C.c_int32,
                                     C.c_int32, C.POINTER(ising_ds_state), _P]),
    "ising_select_dev": (C.c_int, [_P, _P, C.c_int32, _P, _P]),
    "ising_serve_start": (C.c_int, [_P, C.POINTER(ising_serve_config)]),
    "ising_serve_stop": (C.c_int, [_P]),
    "ising_submit": (C.c_int, [_P, C.POINTER(ising_problem), C.POINTER(ising_params), C.POINTER(C.c_uint64)]),
    "ising_wait": (C.c_int, [_P, C.c_uint64, C.c_int32, _P, C.POINTER(C.c_double), C.POINTER(ising_stats)]),
    "ising_cancel": (C.c_int, [_P, C.c_uint64]),
    "ising_serve_query": (C.c_int, [_P, C.POINTER(ising_serve_info)]),
    "ising_from_qubo": (C.c_int, [C.c_int32, _P, _P, _P, _P, C.POINTER(C.c_double)]),
    "ising_from_maxcut": (C.c_int, [C.c_int32, C.c_int64, _P, _P, _P, _P, _P, C.POINTER(C.c_int64),
                                    C.POINTER(C.c_double)]),
    "ising_from_nae3sat": (C.c_int, [C.c_int32, C.c_int64, _P, _P, _P, _P, C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int64)]),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def exported_symbols():
    return list(_sigs)


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------

def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _check(ctx, status):
    if status != ISING_OK:
        msg = _lib.ising_last_error(ctx).decode() if ctx else ""
        raise IsingError(status, msg)


def _vtype(dtype):
    import torch
    return {torch.int32: ISING_I32, torch.float32: ISING_F32, torch.float64: ISING_F64}[dtype]


def _dtype(vtype):
    import torch
    return {ISING_I32: torch.int32, ISING_F32: torch.float32, ISING_F64: torch.float64}[vtype]


@dataclass
class Problem:
    """An ising_problem plus the tensors that back it (kept alive here)."""
    n: int
    format: int
    value_type: int
    J: object = None
    row_ptr: object = None
    col: object = None
    val: object = None
    h: object = None
    nnz: int = 0
    keep: list = field(default_factory=list)

    def struct(self) -> ising_problem:
        return ising_problem(self.n, self.format, self.value_type, 0, self.nnz, _ptr(self.J), _ptr(self.row_ptr),
                             _ptr(self.col), _ptr(self.val), _ptr(self.h))


def dense_problem(J, h=None) -> Problem:
    """Problem from a dense (n, n) tensor J (int32/float32/float64) and optional h of the same dtype."""
    n = J.shape[0]
    return Problem(n, ISING_DENSE, _vtype(J.dtype), J=J.contiguous(), h=None if h is None else h.contiguous())


def csr_problem(row_ptr, col, val, h=None) -> Problem:
    n = row_ptr.shape[0] - 1
    return Problem(n, ISING_CSR, _vtype(val.dtype), row_ptr=row_ptr.contiguous(), col=col.contiguous(),
                   val=val.contiguous(), h=None if h is None else h.contiguous(), nnz=int(col.shape[0]))


def params(replicas=32, steps=100, optimizer="adam", precision="fp32", lr=6.0, mu=0.5, beta1=0.9,
           beta2=0.999, eps=1e-8, seed=0, prune=True, loss="vertex", conv_tol=0.0,
           conv_window=5) -> ising_params:
    opt = {"gd": ISING_OPT_GD, "adam": ISING_OPT_ADAM}[optimizer] if isinstance(optimizer, str) else optimizer
    prec = {"fp64": ISING_PREC_FP64, "fp32": ISING_PREC_FP32, "bf16x2": ISING_PREC_BF16X2,
            "bf16": ISING_PREC_BF16, "fp8": ISING_PREC_FP8, "i8x3": ISING_PREC_I8X3,
            "i8x2": ISING_PREC_I8X2}[precision] if isinstance(precision, str) \
        else precision
    lo = {"vertex": ISING_LOSS_VERTEX, "relaxed": ISING_LOSS_RELAXED}[loss] if isinstance(loss, str) else loss
    return ising_params(replicas, steps, opt, prec, lr, mu, beta1, beta2, eps, seed, 1 if prune else 0, lo,
                        conv_window, 0, conv_tol)


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def ising_create(device: int = 0):
    h = C.c_void_p()
    _check(None, _lib.ising_create(device, C.byref(h)))
    return h


def ising_destroy(ctx):
    _check(None, _lib.ising_destroy(ctx))


def ising_last_error(ctx) -> str:
    return _lib.ising_last_error(ctx).decode()


def ising_solve(ctx, problem_host: ising_problem, prm: ising_params):
    """Host-buffer solve.  problem_host points at host memory (numpy arrays kept alive by the caller)."""
    import numpy as np
    n = problem_host.n
    spins = np.zeros(n, dtype=np.int8)
    e = C.c_double()
    ei = C.c_int64()
    st = ising_stats()
    _check(ctx, _lib.ising_solve(ctx, C.byref(problem_host), C.byref(prm), spins.ctypes.data_as(C.c_void_p),
                                 C.byref(e), C.byref(ei), C.byref(st)))
    return spins, e.value, ei.value, st.as_dict()


def ising_solve_dev(ctx, problem: Problem, prm: ising_params, spins_out=None, energy_out=None,
                    energy_int_out=None, stream=None):
    import torch
    dev = torch.device("cuda")
    if spins_out is None:
        spins_out = torch.empty(problem.n, dtype=torch.int8, device=dev)
    if energy_out is None:
        energy_out = torch.empty(1, dtype=torch.float64, device=dev)
    if energy_int_out is None and problem.value_type == ISING_I32:
        energy_int_out = torch.empty(1, dtype=torch.int64, device=dev)
    st = ising_stats()
    ps = problem.struct()
    _check(ctx, _lib.ising_solve_dev(ctx, C.byref(ps), C.byref(prm), _ptr(spins_out), _ptr(energy_out),
                                     _ptr(energy_int_out), C.byref(st), _stream(stream)))
    return spins_out, energy_out, energy_int_out, st.as_dict()


def ising_last_kernel(ctx) -> str:
    return _lib.ising_last_kernel(ctx).decode()


def ising_energy(ctx, problem_host: ising_problem, spins):
    """Host-buffer energies of the rows of `spins` (numpy int8, (count, n) or (n,))."""
    import numpy as np
    S = np.ascontiguousarray(spins, dtype=np.int8)
    count = S.shape[0] if S.ndim == 2 else 1
    E = np.zeros(count, dtype=np.float64)
    Ei = np.zeros(count, dtype=np.int64) if problem_host.value_type == ISING_I32 else None
    _check(ctx, _lib.ising_energy(ctx, C.byref(problem_host), S.ctypes.data, count, E.ctypes.data,
                                  None if Ei is None else Ei.ctypes.data))
    return E, Ei


def ising_energy_dev_noalloc(ctx, problem: Problem, spins, E_out, E_int_out=None, stream=None):
    """ising_energy_dev with caller-provided outputs and the library's static scratch."""
    spins = spins.contiguous()
    count = spins.shape[0] if spins.dim() == 2 else 1
    ps = problem.struct()
    _check(ctx, _lib.ising_energy_dev_noalloc(ctx, C.byref(ps), _ptr(spins), count, _ptr(E_out), _ptr(E_int_out),
                                              _stream(stream)))
    return E_out, E_int_out


def ising_energy_dev(ctx, problem: Problem, spins, E_out=None, E_int_out=None, stream=None):
    import torch
    spins = spins.contiguous()
    count = spins.shape[0] if spins.dim() == 2 else 1
    if E_out is None:
        E_out = torch.empty(count, dtype=torch.float64, device=spins.device)
    if E_int_out is None and problem.value_type == ISING_I32:
        E_int_out = torch.empty(count, dtype=torch.int64, device=spins.device)
    ps = problem.struct()
    _check(ctx, _lib.ising_energy_dev(ctx, C.byref(ps), _ptr(spins), count, _ptr(E_out), _ptr(E_int_out),
                                      _stream(stream)))
    return E_out, E_int_out


class Pruned:
    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        if getattr(self, "handle", None):
            _lib.ising_pruned_free(self.handle)
            self.handle = None


def ising_prune(ctx, problem_host: ising_problem) -> Pruned:
    """Host-buffer pruning: problem_host points at host memory (kept alive by the caller)."""
    h = C.c_void_p()
    _check(ctx, _lib.ising_prune(ctx, C.byref(problem_host), C.byref(h)))
    return Pruned(h)


def ising_unprune(pr: Pruned, s_G):
    """Full host spin vector from host reduced spins (numpy int8)."""
    import numpy as np
    n = ising_pruned_info(pr)["n"]
    sG = np.ascontiguousarray(s_G, dtype=np.int8)
    out = np.zeros(n, dtype=np.int8)
    _check(None, _lib.ising_unprune(pr.handle, sG.ctypes.data if sG.size else None, out.ctypes.data))
    return out


def ising_pruned_record(pr: Pruned) -> dict:
    """The record and h_G as numpy arrays (host)."""
    import numpy as np
    info = ising_pruned_info(pr)
    n, nG = info["n"], info["n_G"]
    red = ising_pruned_problem(pr)
    hdt = {ISING_I32: np.int32, ISING_F32: np.float32, ISING_F64: np.float64}[red.value_type]
    out = dict(kind=np.zeros(n, np.int8), round_of=np.zeros(n, np.int32), fixed=np.zeros(n, np.int8),
               partner=np.zeros(n, np.int32), sigma=np.zeros(n, np.int8), G=np.zeros(max(nG, 1), np.int32),
               h_G=np.zeros(max(nG, 1), hdt))
    _check(None, _lib.ising_pruned_record(pr.handle, *(out[k].ctypes.data for k in
                                                       ("kind", "round_of", "fixed", "partner", "sigma", "G",
                                                        "h_G"))))
    out["G"] = out["G"][:nG]
    out["h_G"] = out["h_G"][:nG]
    return out


def ising_pruned_copy(pr: Pruned) -> dict:
    """The reduced problem as numpy arrays (host): J (dense) or row_ptr/col/val (CSR), and h."""
    import numpy as np
    red = ising_pruned_problem(pr)
    dt = {ISING_I32: np.int32, ISING_F32: np.float32, ISING_F64: np.float64}[red.value_type]
    nG = red.n
    h = np.zeros(max(nG, 1), dt)
    if red.format == ISING_DENSE:
        J = np.zeros((max(nG, 1), max(nG, 1)), dt)
        _check(None, _lib.ising_pruned_copy(pr.handle, J.ctypes.data, None, None, h.ctypes.data))
        return dict(J=J[:nG, :nG], h=h[:nG])
    rp = np.zeros(nG + 1, np.int32)
    col = np.zeros(max(red.nnz, 1), np.int32)
    val = np.zeros(max(red.nnz, 1), dt)
    _check(None, _lib.ising_pruned_copy(pr.handle, val.ctypes.data, rp.ctypes.data, col.ctypes.data, h.ctypes.data))
    return dict(row_ptr=rp, col=col[:red.nnz], val=val[:red.nnz], h=h[:nG])


def ising_prune_dev(ctx, problem: Problem, stream=None) -> Pruned:
    h = C.c_void_p()
    ps = problem.struct()
    _check(ctx, _lib.ising_prune_dev(ctx, C.byref(ps), C.byref(h), _stream(stream)))
    return Pruned(h)


def ising_pruned_free(pr: Pruned):
    if pr.handle:
        _lib.ising_pruned_free(pr.handle)
        pr.handle = None


def ising_pruned_info(pr: Pruned) -> dict:
    n, nG, rounds, nnz = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
    c = C.c_double()
    _check(None, _lib.ising_pruned_info(pr.handle, C.byref(n), C.byref(nG), C.byref(rounds), C.byref(nnz),
                                        C.byref(c)))
    return dict(n=n.value, n_G=nG.value, rounds=rounds.value, nnz_G=nnz.value, C=c.value)


def ising_pruned_problem(pr: Pruned) -> ising_problem:
    p = ising_problem()
    _check(None, _lib.ising_pruned_problem(pr.handle, C.byref(p)))
    return p


def ising_pruned_record_dev(ctx, pr: Pruned, stream=None) -> dict:
    import torch
    info = ising_pruned_info(pr)
    n, nG = info["n"], info["n_G"]
    red = ising_pruned_problem(pr)
    dev = torch.device("cuda")
    out = dict(kind=torch.empty(n, dtype=torch.int8, device=dev),
               round_of=torch.empty(n, dtype=torch.int32, device=dev),
               fixed=torch.empty(n, dtype=torch.int8, device=dev),
               partner=torch.empty(n, dtype=torch.int32, device=dev),
               sigma=torch.empty(n, dtype=torch.int8, device=dev),
               G=torch.empty(max(nG, 1), dtype=torch.int32, device=dev),
               h_G=torch.zeros(max(nG, 1), dtype=_dtype(red.value_type), device=dev))
    _check(ctx, _lib.ising_pruned_record_dev(ctx, pr.handle, _ptr(out["kind"]), _ptr(out["round_of"]),
                                             _ptr(out["fixed"]), _ptr(out["partner"]), _ptr(out["sigma"]),
                                             _ptr(out["G"]), _ptr(out["h_G"]), _stream(stream)))
    out["G"] = out["G"][:nG]
    out["h_G"] = out["h_G"][:nG]
    return out


def ising_pruned_copy_dev(ctx, pr: Pruned, stream=None) -> Problem:
    """The reduced problem copied into fresh tensors."""
    import torch
    red = ising_pruned_problem(pr)
    dev = torch.device("cuda")
    dt = _dtype(red.value_type)
    nG = red.n
    if red.format == ISING_DENSE:
        J = torch.zeros((nG, nG), dtype=dt, device=dev)
        h = torch.zeros(nG, dtype=dt, device=dev)
        _check(ctx, _lib.ising_pruned_copy_dev(ctx, pr.handle, _ptr(J), None, None, _ptr(h), _stream(stream)))
        return Problem(nG, ISING_DENSE, red.value_type, J=J, h=h)
    rp = torch.zeros(nG + 1, dtype=torch.int32, device=dev)
    col = torch.zeros(max(red.nnz, 1), dtype=torch.int32, device=dev)
    val = torch.zeros(max(red.nnz, 1), dtype=dt, device=dev)
    h = torch.zeros(max(nG, 1), dtype=dt, device=dev)
    _check(ctx, _lib.ising_pruned_copy_dev(ctx, pr.handle, _ptr(val), _ptr(rp), _ptr(col), _ptr(h),
                                           _stream(stream)))
    return Problem(nG, ISING_CSR, red.value_type, row_ptr=rp, col=col[:red.nnz], val=val[:red.nnz],
                   h=h[:nG], nnz=int(red.nnz))


def ising_unprune_dev(ctx, pr: Pruned, s_G, s_out=None, stream=None):
    import torch
    n = ising_pruned_info(pr)["n"]
    if s_out is None:
        s_out = torch.empty(n, dtype=torch.int8, device=torch.device("cuda"))
    _check(ctx, _lib.ising_unprune_dev(ctx, pr.handle, _ptr(s_G), _ptr(s_out), _stream(stream)))
    return s_out


def ising_ds_max_n(precision=ISING_PREC_FP32) -> int:
    return _lib.ising_ds_max_n(precision)


CONV_STATE_WIDTH = 9  # conv_window (at most 8) losses and L_1 per replica


def ds_state(n: int, replicas: int, precision="fp32", optimizer="adam", steps_trace: int = 0, conv: bool = False):
    """Allocate an ising_ds_state's tensors (dict) on the current device."""
    import torch
    dev = torch.device("cuda")
    dt = torch.float64 if precision in ("fp64", ISING_PREC_FP64) else torch.float32
    st = dict(theta=torch.zeros((replicas, n), dtype=dt, device=dev),
              m=torch.zeros((replicas, n), dtype=dt, device=dev),
              v=torch.zeros((replicas, n), dtype=dt, device=dev),
              s_best=torch.zeros((replicas, n), dtype=torch.int8, device=dev),
              e_best=torch.zeros(replicas, dtype=torch.float64, device=dev),
              best_step=torch.zeros(replicas, dtype=torch.int32, device=dev))
    if steps_trace:
        st["energy_trace"] = torch.zeros((steps_trace, replicas), dtype=torch.float64, device=dev)
        st["loss_trace"] = torch.zeros((steps_trace, replicas), dtype=torch.float64, device=dev)
    if conv:
        # the convergence test carried between calls: stop steps and the window of losses
        st["conv_step"] = torch.zeros(replicas, dtype=torch.int32, device=dev)
        st["conv_state"] = torch.zeros((replicas, CONV_STATE_WIDTH), dtype=dt, device=dev)
    return st


def ising_ds_dev(ctx, problem, prm: ising_params, state: dict, t0: int = 0, steps: Optional[int] = None,
                 uniform=None, stream=None):
    """Run domain selection steps t0+1..t0+steps on `state` (tensors from ds_state)."""
    ps = problem.struct() if isinstance(problem, Problem) else problem
    steps = prm.steps if steps is None else steps
    st = ising_ds_state(_ptr(state["theta"]), _ptr(state.get("m")), _ptr(state.get("v")), _ptr(state["s_best"]),
                        _ptr(state["e_best"]), _ptr(state["best_step"]), _ptr(state.get("energy_trace")),
                        _ptr(state.get("loss_trace")), _ptr(state.get("conv_step")), _ptr(state.get("conv_state")))
    _check(ctx, _lib.ising_ds_dev(ctx, C.byref(ps), C.byref(prm), _ptr(uniform), t0, steps, C.byref(st),
                                  _stream(stream)))
    return state


def ising_select_dev(ctx, e_best, best=None, stream=None):
    import torch
    if best is None:
        best = torch.empty(1, dtype=torch.int32, device=e_best.device)
    _check(ctx, _lib.ising_select_dev(ctx, _ptr(e_best), int(e_best.shape[0]), _ptr(best), _stream(stream)))
    return best


def ising_ds_dense_dev(ctx, problem, prm: ising_params, state: dict, t0: int = 0, steps: Optional[int] = None,
                       uniform=None, stream=None):
    """Matrix-core domain selection on a dense problem (state tensors from ds_state(..., "fp32"))."""
    ps = problem.struct() if isinstance(problem, Problem) else problem
    steps = prm.steps if steps is None else steps
    st = ising_ds_state(_ptr(state["theta"]), _ptr(state.get("m")), _ptr(state.get("v")), _ptr(state["s_best"]),
                        _ptr(state["e_best"]), _ptr(state["best_step"]), _ptr(state.get("energy_trace")),
                        _ptr(state.get("loss_trace")))
    _check(ctx, _lib.ising_ds_dense_dev(ctx, C.byref(ps), C.byref(prm), _ptr(uniform), t0, steps, C.byref(st),
                                        _stream(stream)))
    return state


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------

def host_problem(n, J=None, row_ptr=None, col=None, val=None, h=None):
    """ising_problem over host numpy arrays (int32 / float32 / float64 values).

    Returns (struct, keep): keep holds the arrays, which must outlive the call
    that reads the struct (ising_solve, ising_submit)."""
    import numpy as np
    vals = J if J is not None else val
    vt = {np.dtype(np.int32): ISING_I32, np.dtype(np.float32): ISING_F32,
          np.dtype(np.float64): ISING_F64}[np.asarray(vals).dtype]
    keep = []

    def ptr(a, dt=None):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data

    if J is not None:
        st = ising_problem(n, ISING_DENSE, vt, 0, 0, ptr(J), None, None, None, ptr(h, np.asarray(J).dtype))
    else:
        st = ising_problem(n, ISING_CSR, vt, 0, int(len(col)), None, ptr(row_ptr, np.int32), ptr(col, np.int32),
                           ptr(val), ptr(h, np.asarray(val).dtype))
    return st, keep


def ising_serve_start(ctx, hbm_budget_bytes=0, max_resident=0, chunk_steps=0, dense_streams=0, graphs=True):
    cfg = ising_serve_config(hbm_budget_bytes, max_resident, chunk_steps, dense_streams, 0 if graphs else 1)
    _check(ctx, _lib.ising_serve_start(ctx, C.byref(cfg)))


def ising_serve_stop(ctx):
    _check(ctx, _lib.ising_serve_stop(ctx))


def ising_submit(ctx, problem: ising_problem, prm: ising_params) -> int:
    t = C.c_uint64()
    _check(ctx, _lib.ising_submit(ctx, C.byref(problem), C.byref(prm), C.byref(t)))
    return t.value


def ising_wait(ctx, ticket: int, n: int, timeout_ms: int = -1):
    """(status, spins, energy, stats); status is an ISING_* code (the call does not raise)."""
    import numpy as np
    spins = np.zeros(n, dtype=np.int8)
    e = C.c_double()
    st = ising_stats()
    status = _lib.ising_wait(ctx, C.c_uint64(ticket), timeout_ms, spins.ctypes.data_as(C.c_void_p), C.byref(e),
                             C.byref(st))
    return status, spins, e.value, st.as_dict()


def ising_cancel(ctx, ticket: int):
    _check(ctx, _lib.ising_cancel(ctx, C.c_uint64(ticket)))


def ising_serve_query(ctx) -> dict:
    info = ising_serve_info()
    _check(ctx, _lib.ising_serve_query(ctx, C.byref(info)))
    return info.as_dict()


# ---- problem front-ends (host buffers) ----------------------------------------------------

def _host_check(status, what):
    if status != ISING_OK:
        raise IsingError(status, what)


def ising_from_qubo(Q, c=None):
    """(J, h, offset) with x^T Q x + c^T x = E(s) + offset, x = (1 + s) / 2."""
    import numpy as np
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    n = Q.shape[0]
    cc = None if c is None else np.ascontiguousarray(c, dtype=np.float64)
    J = np.zeros((n, n)); h = np.zeros(n); off = C.c_double()
    _host_check(_lib.ising_from_qubo(n, Q.ctypes.data, None if cc is None else cc.ctypes.data, J.ctypes.data,
                                     h.ctypes.data, C.byref(off)), "ising_from_qubo")
    return J, h, off.value


def ising_from_maxcut(n, edges, w=None):
    """CSR (row_ptr, col, val float64) of J = W and the total edge weight."""
    import numpy as np
    e = np.ascontiguousarray(np.asarray(edges).reshape(-1, 2), dtype=np.int32)
    m = e.shape[0]
    ww = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    nnz = C.c_int64(); W = C.c_double()
    args = (n, m, e.ctypes.data, None if ww is None else ww.ctypes.data)
    _host_check(_lib.ising_from_maxcut(*args, None, None, None, C.byref(nnz), C.byref(W)), "ising_from_maxcut")
    rp = np.zeros(n + 1, dtype=np.int32); col = np.zeros(nnz.value, dtype=np.int32)
    val = np.zeros(nnz.value, dtype=np.float64)
    _host_check(_lib.ising_from_maxcut(*args, rp.ctypes.data, col.ctypes.data, val.ctypes.data, C.byref(nnz),
                                       C.byref(W)), "ising_from_maxcut")
    return rp, col, val, W.value


def ising_from_nae3sat(n, clauses):
    """CSR (row_ptr, col, val int32) of the NAE-3SAT couplings and base: violated = (E + base) / 8."""
    import numpy as np
    cl = np.ascontiguousarray(np.asarray(clauses).reshape(-1, 3), dtype=np.int32)
    m = cl.shape[0]
    nnz = C.c_int64(); base = C.c_int64()
    _host_check(_lib.ising_from_nae3sat(n, m, cl.ctypes.data, None, None, None, C.byref(nnz), C.byref(base)),
                "ising_from_nae3sat")
    rp = np.zeros(n + 1, dtype=np.int32); col = np.zeros(nnz.value, dtype=np.int32)
    val = np.zeros(nnz.value, dtype=np.int32)
    _host_check(_lib.ising_from_nae3sat(n, m, cl.ctypes.data, rp.ctypes.data, col.ctypes.data, val.ctypes.data,
                                        C.byref(nnz), C.byref(base)), "ising_from_nae3sat")
    return rp, col, val, base.value
