"""Python binding of liblqcd, the MI355X staggered even/odd solver library.

Argument marshalling only: every operation runs in the library's HIP kernels.
(The one host-side computation is setup: the Remez exchange of ``rational``,
which produces the rational approximations' poles and residues.)
Tensors are torch tensors on the GPU (torch provides device memory and the
current stream).  The binding fails loudly when the library has not been
built; there is no CPU fallback.

Layouts follow ``include/lqcd.h``:
  natural links   complex128 [4][V][3][3]     natural fields complex128 [n][V][3]
  packed links    complex128/complex64 [2][4][NE][Vh]  (NE = 9, 6 or 7), or
                  [2][4][13][Vh/2] for LINKS12T (six complex planes and one
                  plane of reals, the U(1) angle, per [parity][mu] block)
  packed spinors  complex128/complex64 [n][3][Vh] (one parity)
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import torch

from .rational import RationalApprox, minimax, minimax_for_tol, spectral_bounds  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblqcd.so")

F64, F32 = 0, 1
LINKS18, LINKS12, LINKS12D, LINKS12T = 0, 1, 2, 3

OK = 0
ERR_INVALID_ARG = 1
ERR_UNSUPPORTED = 2
ERR_WORKSPACE = 3
ERR_HIP = 4
ERR_NOT_CONVERGED = 5
ERR_NUMERIC = 6


class LqcdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it first (python paper_1801_01473_amd/build.py "
        "or __graft_entry__.build()); there is no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)


class lqcd_geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("antiperiodic_t", ctypes.c_int32)]


class SolverParams(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
        ("inner_prec", ctypes.c_int32), ("inner_fmt", ctypes.c_int32),
        ("reliable_interval", ctypes.c_int32), ("use_graph", ctypes.c_int32),
        ("rhs_block", ctypes.c_int32), ("poll_interval", ctypes.c_int32),
        ("max_refine", ctypes.c_int32), ("shift_window", ctypes.c_int32),
        ("reliable_delta", ctypes.c_double),
        ("mixed_switch", ctypes.c_double), ("inner_tol_factor", ctypes.c_double),
    ]


class SolveStats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32), ("reliable_updates", ctypes.c_int32),
        ("refine_iters", ctypes.c_int32), ("converged", ctypes.c_int32),
        ("true_rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
        ("iters_fp64", ctypes.c_int32), ("shift_window", ctypes.c_int32),
        ("shift_updates_fp64", ctypes.c_int64), ("shift_updates_fp32", ctypes.c_int64),
        ("flush_shifts_fp64", ctypes.c_int64), ("flush_shifts_fp32", ctypes.c_int64),
        ("flush_slots_fp64", ctypes.c_int64), ("flush_slots_fp32", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_gp = ctypes.POINTER(lqcd_geom)
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
_dp = ctypes.POINTER(ctypes.c_double)
_pp = ctypes.POINTER(SolverParams)
_sp = ctypes.POINTER(SolveStats)

_SIGS = {
    "lqcd_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "lqcd_last_error": (ctypes.c_char_p, []),
    "lqcd_version": (ctypes.c_int, []),
    "lqcd_finalize": (ctypes.c_int, []),
    "lqcd_links_bytes": (ctypes.c_size_t, [_gp, ctypes.c_int, ctypes.c_int]),
    "lqcd_spinor_bytes": (ctypes.c_size_t, [_gp, ctypes.c_int]),
    "lqcd_pack_links": (ctypes.c_int, [_gp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp]),
    "lqcd_convert_links": (ctypes.c_int, [_gp, _vp, ctypes.c_int, ctypes.c_int, _vp,
                                          ctypes.c_int, ctypes.c_int, _vp]),
    "lqcd_unpack_links": (ctypes.c_int, [_gp, _vp, _vp, _vp]),
    "lqcd_pack_spinor": (ctypes.c_int, [_gp, ctypes.c_int, ctypes.c_int, _vp, _vp, _i32, _vp]),
    "lqcd_unpack_spinor": (ctypes.c_int, [_gp, ctypes.c_int, ctypes.c_int, _vp, _vp, _i32, _vp]),
    "lqcd_doe": (ctypes.c_int, [_gp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _i32, _vp]),
    "lqcd_deo": (ctypes.c_int, [_gp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _i32, _vp]),
    "lqcd_apply_A": (ctypes.c_int, [_gp, ctypes.c_int, ctypes.c_int, _vp, _dbl, _dbl, _vp, _vp,
                                    _vp, _i32, _vp]),
    "lqcd_solver_params_default": (None, [_pp]),
    "lqcd_solver_workspace_bytes": (ctypes.c_size_t, [_gp, _pp, _i32, _i32]),
    "lqcd_cg": (ctypes.c_int, [_gp, _pp, _vp, _vp, _dbl, _vp, _vp, _i32, _sp, _vp,
                               ctypes.c_size_t, _vp]),
    "lqcd_cg_multishift": (ctypes.c_int, [_gp, _pp, _vp, _vp, _i32, _dp, _vp, _vp, _i32, _sp,
                                          _vp, ctypes.c_size_t, _vp]),
    "lqcd_fermion_force": (ctypes.c_int, [_gp, _vp, _i32, _i32, _dp, _vp, _i32, _i32, _vp, _vp]),
    "lqcd_action_workspace_bytes": (ctypes.c_size_t, [_gp]),
    "lqcd_action": (ctypes.c_int, [_gp, _i32, _i32, _dbl, _dp, _vp, _vp, _dp, _vp,
                                   ctypes.c_size_t, _vp]),
    "lqcd_action_noalloc": (ctypes.c_int, [_gp, _i32, _i32, _dbl, _dp, _vp, _vp, _dp, _vp]),
    "lqcd_rational_combine": (ctypes.c_int, [_gp, _i32, _i32, _dbl, _dp, _vp, _vp, _vp, _vp]),
    "lqcd_apply_u1_phases": (ctypes.c_int, [_gp, _vp, _vp, _vp, _vp]),
    "lqcd_pack_links_u1": (ctypes.c_int, [_gp, _vp, _vp, ctypes.c_int, _vp, _vp]),
    "lqcd_stout_smear": (ctypes.c_int, [_gp, _vp, _dbl, _vp, _vp]),
    "lqcd_stout_workspace_bytes": (ctypes.c_size_t, [_gp]),
    "lqcd_stout_force": (ctypes.c_int, [_gp, _vp, _dbl, _vp, _i32, _vp, _vp, ctypes.c_size_t,
                                        _vp]),
    "lqcd_gauge_workspace_bytes": (ctypes.c_size_t, [_gp]),
    "lqcd_gauge_action": (ctypes.c_int, [_gp, _vp, _dbl, _dbl, _dp, _vp, ctypes.c_size_t, _vp]),
    "lqcd_gauge_force": (ctypes.c_int, [_gp, _vp, _dbl, _dbl, _i32, _vp, _vp]),
    "lqcd_gauge_force_staples_workspace_bytes": (ctypes.c_size_t, [_gp]),
    "lqcd_gauge_force_staples": (ctypes.c_int, [_gp, _vp, _dbl, _dbl, _i32, _vp, _vp,
                                                ctypes.c_size_t, _vp]),
    "lqcd_md_update_momenta": (ctypes.c_int, [_gp, _vp, _dbl, _vp, _vp]),
    "lqcd_md_update_links": (ctypes.c_int, [_gp, _vp, _dbl, _vp, _vp]),
    "lqcd_kinetic_energy": (ctypes.c_int, [_gp, _vp, _dp, _vp, ctypes.c_size_t, _vp]),
    "lqcd_stream_bandwidth": (ctypes.c_int, [ctypes.c_size_t, _i32, _dp, _dp]),
    "lqcd_kernel_timing_enable": (ctypes.c_int, [_i32]),
    "lqcd_kernel_timing_get": (ctypes.c_int, [_i32, ctypes.c_char_p, ctypes.c_size_t,
                                              ctypes.POINTER(ctypes.c_int64), _dp]),
}

EXPORTED = tuple(_SIGS)
_fns = {}


def _fn(name):
    f = _fns.get(name)
    if f is None:
        f = getattr(_lib, name)
        f.restype, f.argtypes = _SIGS[name]
        _fns[name] = f
    return f


def status_string(s: int) -> str:
    return _fn("lqcd_status_string")(s).decode()


def last_error() -> str:
    return _fn("lqcd_last_error")().decode()


def version() -> int:
    return int(_fn("lqcd_version")())


def finalize() -> None:
    _check(_fn("lqcd_finalize")())


def _check(status: int, allow=()):
    if status != OK and status not in allow:
        raise LqcdError(status, f"{status_string(status)}: {last_error()}")
    return status


def _stream():
    return _vp(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None):
    if t is None:
        return _vp(0)
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return _vp(t.data_ptr())


@dataclass(frozen=True)
class Geometry:
    L: tuple
    antiperiodic: bool = True

    @property
    def V(self) -> int:
        return self.L[0] * self.L[1] * self.L[2] * self.L[3]

    @property
    def Vh(self) -> int:
        return self.V // 2

    def c(self):
        g = lqcd_geom()
        for i in range(4):
            g.L[i] = int(self.L[i])
        g.antiperiodic_t = 1 if self.antiperiodic else 0
        return ctypes.byref(g)


def _cdtype(prec):
    return torch.complex128 if prec == F64 else torch.complex64


def _ne(fmt):
    return {LINKS18: 9, LINKS12: 6, LINKS12D: 7, LINKS12T: 13}[fmt]


def _links_shape(geom: Geometry, fmt):
    if fmt == LINKS12T:
        return (2, 4, 13, geom.Vh // 2)
    return (2, 4, _ne(fmt), geom.Vh)


def links_bytes(geom: Geometry, prec=F64, fmt=LINKS18) -> int:
    return int(_fn("lqcd_links_bytes")(geom.c(), prec, fmt))


def spinor_bytes(geom: Geometry, prec=F64) -> int:
    return int(_fn("lqcd_spinor_bytes")(geom.c(), prec))


def empty_links(geom: Geometry, prec=F64, fmt=LINKS18, device="cuda"):
    return torch.empty(_links_shape(geom, fmt), dtype=_cdtype(prec), device=device)


def empty_spinor(geom: Geometry, n=1, prec=F64, device="cuda"):
    return torch.empty((n, 3, geom.Vh), dtype=_cdtype(prec), device=device)


def _natural_links_arg(geom: Geometry, t, name):
    _tensor(t, name)
    if t.dtype != torch.complex128 or tuple(t.shape) != (4, geom.V, 3, 3):
        raise ValueError(f"{name} must be complex128 [4][{geom.V}][3][3], "
                         f"got {t.dtype} {tuple(t.shape)}")
    _finish(t, name)


def pack_links(geom: Geometry, U_nat: torch.Tensor, prec=F64, fmt=LINKS18, out=None):
    _natural_links_arg(geom, U_nat, "U_nat")
    if prec not in (F64, F32) or fmt not in (LINKS18, LINKS12, LINKS12D, LINKS12T):
        raise ValueError("unknown precision or link format")
    out = empty_links(geom, prec, fmt, U_nat.device) if out is None else out
    _links_arg(geom, out, "out", prec, fmt)
    _check(_fn("lqcd_pack_links")(geom.c(), _ptr(U_nat), prec, fmt, _ptr(out), _stream()))
    return out


def convert_links(geom: Geometry, src, src_prec, src_fmt, dst_prec, dst_fmt, out=None):
    _links_arg(geom, src, "src", src_prec, src_fmt)
    out = empty_links(geom, dst_prec, dst_fmt, src.device) if out is None else out
    _links_arg(geom, out, "out", dst_prec, dst_fmt)
    _check(_fn("lqcd_convert_links")(geom.c(), _ptr(src), src_prec, src_fmt, _ptr(out),
                                     dst_prec, dst_fmt, _stream()))
    return out


def unpack_links(geom: Geometry, U_packed, out=None):
    _u64_arg(geom, U_packed, "U_packed")
    out = torch.empty((4, geom.V, 3, 3), dtype=torch.complex128,
                      device=U_packed.device) if out is None else out
    _natural_links_arg(geom, out, "out")
    _check(_fn("lqcd_unpack_links")(geom.c(), _ptr(U_packed), _ptr(out), _stream()))
    return out


def pack_spinor(geom: Geometry, nat: torch.Tensor, parity: int, prec=F64, out=None):
    _tensor(nat, "nat")
    if nat.dtype != torch.complex128:
        raise ValueError("natural fields must be complex128")
    if nat.numel() == 0 or nat.numel() % (3 * geom.V):
        raise ValueError(f"natural fields must be [n][{geom.V}][3], got {tuple(nat.shape)}")
    nat = _finish(nat, "nat").reshape(-1, geom.V, 3)
    n = nat.shape[0]
    out = empty_spinor(geom, n, prec, nat.device) if out is None else out
    _spinor_arg(geom, out, prec, "out", n)
    _check(_fn("lqcd_pack_spinor")(geom.c(), parity, prec, _ptr(nat), _ptr(out), n, _stream()))
    return out


def unpack_spinor(geom: Geometry, packed: torch.Tensor, parity: int, out=None):
    _tensor(packed, "packed")
    prec = F64 if packed.dtype == torch.complex128 else F32
    n = _spinor_arg(geom, packed, prec, "packed")
    out = torch.empty((n, geom.V, 3), dtype=torch.complex128,
                      device=packed.device) if out is None else out
    _tensor(out, "out")
    if out.dtype != torch.complex128 or out.numel() != n * geom.V * 3:
        raise ValueError(f"out must be complex128 [{n}][{geom.V}][3]")
    _finish(out, "out")
    _check(_fn("lqcd_unpack_spinor")(geom.c(), parity, prec, _ptr(packed), _ptr(out), n,
                                     _stream()))
    return out


def _prec_of(t):
    return F64 if t.dtype == torch.complex128 else F32


def _fmt_of(U):
    return {9: LINKS18, 6: LINKS12, 7: LINKS12D, 13: LINKS12T}[int(U.shape[2])]


# ---------------------------------------------------------------- argument checks
# Every tensor handed to the library is checked here -- dtype, element count or
# shape, contiguity -- and then its device, before any call into it, so that a
# mismatch (say FP64 links with complex64 spinors) raises ValueError instead of
# letting a kernel read or write past a buffer.

def _tensor(t, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor, got {type(t).__name__}")
    return t


def _finish(t, name):
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _gpu(*ts):
    """Device check, after the dtype/size checks and before any allocation
    (_ptr repeats it for every pointer passed)."""
    for t in ts:
        if not t.is_cuda:
            raise ValueError("tensor must live on the GPU")


def _links_arg(geom: Geometry, U, name="U", prec=None, fmt=None):
    """Packed links [2][4][NE][Vh]; returns (prec, fmt)."""
    _tensor(U, name)
    if U.dtype not in (torch.complex128, torch.complex64):
        raise ValueError(f"{name} must be complex128 or complex64 packed links, got {U.dtype}")
    if U.dim() != 4 or tuple(U.shape[:2]) != (2, 4) or int(U.shape[2]) not in (9, 6, 7, 13) \
            or int(U.shape[3]) != (geom.Vh // 2 if int(U.shape[2]) == 13 else geom.Vh):
        raise ValueError(f"{name} must be packed links [2][4][9|6|7][{geom.Vh}] or "
                         f"[2][4][13][{geom.Vh // 2}], got {tuple(U.shape)}")
    p, f = _prec_of(U), _fmt_of(U)
    if prec is not None and p != prec:
        raise ValueError(f"{name} must be {_cdtype(prec)}, got {U.dtype}")
    if fmt is not None and f != fmt:
        raise ValueError(f"{name} must have {_ne(fmt)} elements per link, got {int(U.shape[2])}")
    _finish(U, name)
    return p, f


def _u64_arg(geom: Geometry, U, name="U64"):
    _links_arg(geom, U, name, F64, LINKS18)


def _spinor_arg(geom: Geometry, t, prec, name, n=None):
    """Packed single-parity spinors [n][3][Vh] of precision prec; returns n."""
    _tensor(t, name)
    if t.dtype != _cdtype(prec):
        raise ValueError(f"{name} must be {_cdtype(prec)} to match the links, got {t.dtype}")
    per = 3 * geom.Vh
    if t.numel() == 0 or t.numel() % per:
        raise ValueError(f"{name} must hold a whole number of packed spinors of 3 x {geom.Vh} "
                         f"entries, got {t.numel()} entries")
    if n is not None and t.numel() != n * per:
        raise ValueError(f"{name} must hold {n} packed spinors ({n * per} entries), "
                         f"got {t.numel()}")
    _finish(t, name)
    return t.numel() // per


def _real_links_out(geom: Geometry, t, name):
    """An FP64 18-real packed link-shaped output (forces, momenta)."""
    _links_arg(geom, t, name, F64, LINKS18)


def doe(geom: Geometry, U, psi_even, out=None):
    """D_oe: packed even spinors [n][3][Vh] -> packed odd spinors."""
    prec, _ = _links_arg(geom, U)
    n = _spinor_arg(geom, psi_even, prec, "psi_even")
    out = torch.empty_like(psi_even) if out is None else out
    _spinor_arg(geom, out, prec, "out", n)
    _check(_fn("lqcd_doe")(geom.c(), _prec_of(U), _fmt_of(U), _ptr(U), _ptr(psi_even),
                           _ptr(out), n, _stream()))
    return out


def deo(geom: Geometry, U, psi_odd, out=None):
    """D_eo: packed odd spinors -> packed even spinors."""
    prec, _ = _links_arg(geom, U)
    n = _spinor_arg(geom, psi_odd, prec, "psi_odd")
    out = torch.empty_like(psi_odd) if out is None else out
    _spinor_arg(geom, out, prec, "out", n)
    _check(_fn("lqcd_deo")(geom.c(), _prec_of(U), _fmt_of(U), _ptr(U), _ptr(psi_odd),
                           _ptr(out), n, _stream()))
    return out


def apply_A(geom: Geometry, U, mass, sigma, x_even, out=None, tmp=None):
    """((m^2 + sigma) - D_eo D_oe) x on packed even spinors."""
    prec, _ = _links_arg(geom, U)
    n = _spinor_arg(geom, x_even, prec, "x_even")
    out = torch.empty_like(x_even) if out is None else out
    tmp = torch.empty_like(x_even) if tmp is None else tmp
    _spinor_arg(geom, out, prec, "out", n)
    _spinor_arg(geom, tmp, prec, "tmp", n)
    _check(_fn("lqcd_apply_A")(geom.c(), _prec_of(U), _fmt_of(U), _ptr(U), float(mass),
                               float(sigma), _ptr(x_even), _ptr(out), _ptr(tmp), n, _stream()))
    return out


def solver_params(**kw) -> SolverParams:
    p = SolverParams()
    _fn("lqcd_solver_params_default")(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def solver_workspace_bytes(geom: Geometry, params: SolverParams, nshift: int, nrhs: int) -> int:
    return int(_fn("lqcd_solver_workspace_bytes")(geom.c(), ctypes.byref(params), nshift, nrhs))


_ws_cache = {}


def _workspace(nbytes: int, device) -> torch.Tensor:
    key = str(device)
    ws = _ws_cache.get(key)
    if ws is None or ws.numel() < nbytes:
        _ws_cache[key] = None
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = ws
    return ws


def release_workspace() -> None:
    _ws_cache.clear()


def cg(geom: Geometry, params: SolverParams, U64, b, x=None, sigma=0.0, Uinner=None,
       check=True):
    """CG on ((m^2 + sigma) - D_eo D_oe) x = b for packed FP64 even b [n][3][Vh].

    Returns (x, status, [stats per right-hand side]).  x holds the initial
    guess on entry when given.
    """
    _u64_arg(geom, U64)
    n = _spinor_arg(geom, b, F64, "b")
    x = torch.zeros_like(b) if x is None else x
    _spinor_arg(geom, x, F64, "x", n)
    if Uinner is not None:
        _links_arg(geom, Uinner, "Uinner", params.inner_prec, params.inner_fmt)
    _gpu(U64, b, x)
    ws_bytes = solver_workspace_bytes(geom, params, 1, n)
    ws = _workspace(ws_bytes, b.device)
    stats = (SolveStats * n)()
    st = _fn("lqcd_cg")(geom.c(), ctypes.byref(params), _ptr(U64), _ptr(Uinner), float(sigma),
                        _ptr(b), _ptr(x), n, stats, _ptr(ws), ws.numel(), _stream())
    if check:
        _check(st)
    return x, st, [s.as_dict() for s in stats]


def cg_multishift(geom: Geometry, params: SolverParams, U64, sigmas, b, x=None, Uinner=None,
                  check=True):
    """Multi-shift CG.  b: packed FP64 even [n][3][Vh]; returns x [n][nshift][3][Vh]."""
    _u64_arg(geom, U64)
    n = _spinor_arg(geom, b, F64, "b")
    sig = (ctypes.c_double * len(sigmas))(*[float(s) for s in sigmas])
    ns = len(sigmas)
    if x is None:
        x = torch.empty((n, ns, 3, geom.Vh), dtype=torch.complex128, device=b.device)
    _spinor_arg(geom, x, F64, "x", n * ns)
    if Uinner is not None:
        _links_arg(geom, Uinner, "Uinner", params.inner_prec, params.inner_fmt)
    _gpu(U64, b, x)
    ws_bytes = solver_workspace_bytes(geom, params, ns, n)
    ws = _workspace(ws_bytes, b.device)
    stats = (SolveStats * (n * ns))()
    st = _fn("lqcd_cg_multishift")(geom.c(), ctypes.byref(params), _ptr(U64), _ptr(Uinner), ns,
                                   sig, _ptr(b), _ptr(x), n, stats, _ptr(ws), ws.numel(),
                                   _stream())
    if check:
        _check(st)
    return x, st, [[stats[j * ns + i].as_dict() for i in range(ns)] for j in range(n)]


def fermion_force(geom: Geometry, U64, alpha, X, mode=0, out=None, accumulate=False):
    """Force from solutions X [npf][nshift][3][Vh] (packed FP64 even).

    mode 0: TA(U M) (su(3) force); mode 1: M^dag (raw gradient).  Output in the
    packed FP64 18-real link layout [2][4][9][Vh].
    """
    _u64_arg(geom, U64)
    nshift = len(alpha)
    if nshift < 1:
        raise ValueError("need at least one shift coefficient")
    nX = _spinor_arg(geom, X, F64, "X")
    if nX % nshift:
        raise ValueError(f"X must hold npf x {nshift} even vectors, got {nX}")
    npf = nX // nshift
    al = (ctypes.c_double * nshift)(*[float(a) for a in alpha])
    out = empty_links(geom, F64, LINKS18, X.device) if out is None else out
    _real_links_out(geom, out, "out")
    _check(_fn("lqcd_fermion_force")(geom.c(), _ptr(U64), npf, nshift, al, _ptr(X), int(mode),
                                     1 if accumulate else 0, _ptr(out), _stream()))
    return out


def action(geom: Geometry, alpha0, alpha, phi, X) -> float:
    nshift = len(alpha)
    npf = _spinor_arg(geom, phi, F64, "phi")
    _spinor_arg(geom, X, F64, "X", npf * nshift)
    _gpu(phi, X)
    al = (ctypes.c_double * nshift)(*[float(a) for a in alpha])
    nbytes = int(_fn("lqcd_action_workspace_bytes")(geom.c()))
    ws = _workspace(nbytes, phi.device)
    S = ctypes.c_double(0.0)
    _check(_fn("lqcd_action")(geom.c(), npf, nshift, float(alpha0), al, _ptr(phi), _ptr(X),
                              ctypes.byref(S), _ptr(ws), ws.numel(), _stream()))
    return float(S.value)


def action_noalloc(geom: Geometry, alpha0, alpha, phi, X) -> float:
    """``action`` through the entry point that allocates nothing (its partial
    sums live in the library's fixed device array; concurrent calls on one
    device race)."""
    nshift = len(alpha)
    npf = _spinor_arg(geom, phi, F64, "phi")
    _spinor_arg(geom, X, F64, "X", npf * nshift)
    _gpu(phi, X)
    al = (ctypes.c_double * nshift)(*[float(a) for a in alpha])
    S = ctypes.c_double(0.0)
    _check(_fn("lqcd_action_noalloc")(geom.c(), npf, nshift, float(alpha0), al, _ptr(phi),
                                      _ptr(X), ctypes.byref(S), _stream()))
    return float(S.value)


def rational_combine(geom: Geometry, alpha0, alpha, b, X, out=None):
    """y_j = alpha0 b_j + sum_i alpha_i X_ji on the GPU (packed FP64 even
    vectors; b [n][3][Vh], X [n][nshift][3][Vh]); out may be b."""
    nshift = len(alpha)
    n = _spinor_arg(geom, b, F64, "b")
    _spinor_arg(geom, X, F64, "X", n * nshift)
    out = torch.empty_like(b) if out is None else out
    _spinor_arg(geom, out, F64, "out", n)
    al = (ctypes.c_double * nshift)(*[float(a) for a in alpha])
    _check(_fn("lqcd_rational_combine")(geom.c(), n, nshift, float(alpha0), al, _ptr(b),
                                        _ptr(X), _ptr(out), _stream()))
    return out


def rational_apply(geom: Geometry, params: SolverParams, U64, approx, b, Uinner=None):
    """r(A) b for a rational function in partial fractions (a RationalApprox or
    anything with alpha0, alpha, sigma): one multi-shift solve at the poles,
    then the combination.  Returns (y, per-(rhs, shift) solve stats)."""
    X, _, stats = cg_multishift(geom, params, U64, approx.sigma, b, Uinner=Uinner)
    y = rational_combine(geom, approx.alpha0, approx.alpha, b, X)
    return y, stats


def pseudofermion_heatbath(geom: Geometry, params: SolverParams, U64, approx_eighth, xi,
                           Uinner=None):
    """RHMC pseudofermion heatbath (Sec. 2): phi = r(A) xi with r ~ x^(1/8) and
    xi complex Gaussian noise of density exp(-|xi|^2) (drawn by the caller).
    Then phi^dag A^(-1/4) phi = |xi|^2 up to the approximation errors, so phi
    has the density exp(-phi^dag A^(-1/4) phi) of the pseudofermion action.
    Returns (phi, stats)."""
    if approx_eighth.power != 0.125:
        raise ValueError("the heatbath needs the x^(1/8) approximation")
    return rational_apply(geom, params, U64, approx_eighth, xi, Uinner)


def rational_action(geom: Geometry, params: SolverParams, U64, approx_quarter, phi,
                    Uinner=None):
    """S = sum_j phi_j^dag r(A) phi_j with r ~ x^(-1/4) (Eq. (1) fermion term in
    rational form), FP64, for the accept/reject step.  Returns (S, X, stats);
    X [n][nshift][3][Vh] serves the force as well."""
    X, _, stats = cg_multishift(geom, params, U64, approx_quarter.sigma, phi, Uinner=Uinner)
    S = action(geom, approx_quarter.alpha0, approx_quarter.alpha, phi, X)
    return S, X, stats


def metropolis_accept(h_old: float, h_new: float, u: float) -> bool:
    """Accept/reject step of (R)HMC: accept with probability
    min(1, exp(-(h_new - h_old))), for u uniform in [0, 1) drawn by the caller;
    the energies are FP64 (the paper runs this test in double precision)."""
    if not (0.0 <= u < 1.0):
        raise ValueError("u must be in [0, 1)")
    dh = float(h_new) - float(h_old)
    if not math.isfinite(dh):
        return False
    return dh <= 0.0 or u < math.exp(-dh)


def apply_u1_phases(geom: Geometry, U64, theta, out=None):
    """Links u_mu(x) U_mu(x), u = exp(i theta_mu(x)), theta real [4][V] (natural
    order, FP64, on the device); packed FP64 18-real in and out.  Use 18-real
    formats for every precision with phased links (they are not SU(3))."""
    _u64_arg(geom, U64)
    _tensor(theta, "theta")
    if theta.dtype != torch.float64 or tuple(theta.shape) != (4, geom.V):
        raise ValueError("theta must be float64 [4][V]")
    theta = theta.contiguous()
    out = torch.empty_like(U64) if out is None else out
    _u64_arg(geom, out, "out")
    _check(_fn("lqcd_apply_u1_phases")(geom.c(), _ptr(U64), _ptr(theta), _ptr(out), _stream()))
    return out


def pack_links_u1(geom: Geometry, U64, theta, prec=F32, out=None):
    """LINKS12T links of one flavour: rows 0-1 of the SU(3) links U64 (packed
    FP64 18-real) and the angles theta (float64 [4][V], natural order, on the
    device), stored in precision prec; the operator recomputes exp(i theta)."""
    _u64_arg(geom, U64)
    _tensor(theta, "theta")
    if theta.dtype != torch.float64 or tuple(theta.shape) != (4, geom.V):
        raise ValueError("theta must be float64 [4][V]")
    theta = theta.contiguous()
    out = empty_links(geom, prec, LINKS12T, U64.device) if out is None else out
    _links_arg(geom, out, "out", prec, LINKS12T)
    _gpu(theta)
    _check(_fn("lqcd_pack_links_u1")(geom.c(), _ptr(U64), _ptr(theta), int(prec), _ptr(out),
                                     _stream()))
    return out


def stout_smear(geom: Geometry, U64, rho: float, levels: int = 1):
    """[U^(0), U^(1), ..., U^(levels)]: repeated stout smearing (packed FP64
    18-real); U^(0) is U64 itself."""
    _u64_arg(geom, U64)
    out = [U64]
    for _ in range(levels):
        nxt = torch.empty_like(U64)
        _check(_fn("lqcd_stout_smear")(geom.c(), _ptr(out[-1]), float(rho), _ptr(nxt), _stream()))
        out.append(nxt)
    return out


def stout_force(geom: Geometry, chain, rho: float, G_top, mode: int = 0):
    """Carry a raw gradient G_top (M^dag with respect to the most smeared
    links chain[-1], e.g. fermion_force(..., mode=1)) down the smearing chain
    [U^(0), ..., U^(k)] of stout_smear; returns TA(U^(0) M) (mode 0) or the raw
    gradient M^dag with respect to U^(0) (mode 1)."""
    for k, Uk in enumerate(chain):
        _u64_arg(geom, Uk, f"chain[{k}]")
    _real_links_out(geom, G_top, "G_top")
    _gpu(G_top, *chain)
    nbytes = int(_fn("lqcd_stout_workspace_bytes")(geom.c()))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=G_top.device)
    G = G_top
    for j in range(len(chain) - 2, -1, -1):
        out = torch.empty_like(G_top)
        _check(_fn("lqcd_stout_force")(geom.c(), _ptr(chain[j]), float(rho), _ptr(G),
                                       mode if j == 0 else 1, _ptr(out), _ptr(ws), ws.numel(),
                                       _stream()))
        G = out
    return G


SYMANZIK_C1 = -1.0 / 12.0


def gauge_action(geom: Geometry, U64, beta: float, c1: float = SYMANZIK_C1) -> float:
    """Tree-level Symanzik gauge action S_g (c1 = 0: Wilson) of packed FP64
    18-real links."""
    _u64_arg(geom, U64)
    _gpu(U64)
    ws = _workspace(int(_fn("lqcd_gauge_workspace_bytes")(geom.c())), U64.device)
    S = ctypes.c_double(0.0)
    _check(_fn("lqcd_gauge_action")(geom.c(), _ptr(U64), float(beta), float(c1), ctypes.byref(S),
                                    _ptr(ws), ws.numel(), _stream()))
    return float(S.value)


def gauge_force(geom: Geometry, U64, beta: float, c1: float = SYMANZIK_C1, out=None,
                accumulate=False, method: str = "staples"):
    """F = TA(U M) of S_g, packed like the links; accumulate adds into out.
    method "staples": through stored plaquette-staple fields (workspace);
    "direct": every staple of every link multiplied out in place."""
    _u64_arg(geom, U64)
    out = empty_links(geom, F64, LINKS18, U64.device) if out is None else out
    _real_links_out(geom, out, "out")
    if method == "direct":
        _check(_fn("lqcd_gauge_force")(geom.c(), _ptr(U64), float(beta), float(c1),
                                       1 if accumulate else 0, _ptr(out), _stream()))
    elif method == "staples":
        nbytes = int(_fn("lqcd_gauge_force_staples_workspace_bytes")(geom.c()))
        ws = _workspace(nbytes, U64.device)
        _check(_fn("lqcd_gauge_force_staples")(geom.c(), _ptr(U64), float(beta), float(c1),
                                               1 if accumulate else 0, _ptr(out), _ptr(ws),
                                               ws.numel(), _stream()))
    else:
        raise ValueError(f"unknown gauge force method {method!r}")
    return out


def md_update_momenta(geom: Geometry, H, F, eps: float):
    """H <- H - i eps F in place."""
    _real_links_out(geom, H, "H")
    _real_links_out(geom, F, "F")
    _check(_fn("lqcd_md_update_momenta")(geom.c(), _ptr(F), float(eps), _ptr(H), _stream()))
    return H


def md_update_links(geom: Geometry, U64, H, eps: float):
    """U <- exp(i eps H) U in place (re-orthonormalised to SU(3))."""
    _u64_arg(geom, U64)
    _real_links_out(geom, H, "H")
    _check(_fn("lqcd_md_update_links")(geom.c(), _ptr(H), float(eps), _ptr(U64), _stream()))
    return U64


def kinetic_energy(geom: Geometry, H) -> float:
    """H^2 / 2 = half the sum over links of Tr H^2."""
    _real_links_out(geom, H, "H")
    _gpu(H)
    ws = _workspace(int(_fn("lqcd_gauge_workspace_bytes")(geom.c())), H.device)
    K = ctypes.c_double(0.0)
    _check(_fn("lqcd_kinetic_energy")(geom.c(), _ptr(H), ctypes.byref(K), _ptr(ws), ws.numel(),
                                      _stream()))
    return float(K.value)


OMELYAN_LAMBDA = 0.1931833275037836


def md_integrate(geom: Geometry, U64, H, tau: float, nsteps: int, force,
                 integrator: str = "omelyan", lam: float = OMELYAN_LAMBDA):
    """Integrate U' = i H U, H' = -i F(U) from 0 to tau in nsteps steps, in
    place (Sec. 4.3, Alg. 2: force, new momenta, new configuration).  force(U64, F)
    writes the total force into F.  "leapfrog": kick eps/2, (drift eps,
    kick eps) ..., last kick eps/2; "omelyan": the second-order minimum-norm
    scheme kick lam eps, drift eps/2, kick (1 - 2 lam) eps, drift eps/2,
    kick lam eps, adjacent kicks of consecutive steps merged.  Returns the
    number of force evaluations."""
    if nsteps < 1 or not math.isfinite(tau):
        raise ValueError("need nsteps >= 1 and a finite tau")
    eps = float(tau) / nsteps
    F = empty_links(geom, F64, LINKS18, U64.device)
    nforce = 0

    def kick(c):
        nonlocal nforce
        force(U64, F)
        nforce += 1
        md_update_momenta(geom, H, F, c * eps)

    def drift(c):
        md_update_links(geom, U64, H, c * eps)

    if integrator == "leapfrog":
        kick(0.5)
        for n in range(nsteps):
            drift(1.0)
            kick(1.0 if n < nsteps - 1 else 0.5)
    elif integrator == "omelyan":
        kick(lam)
        for n in range(nsteps):
            drift(0.5)
            kick(1.0 - 2.0 * lam)
            drift(0.5)
            kick(2.0 * lam if n < nsteps - 1 else lam)
    else:
        raise ValueError(f"unknown integrator {integrator!r}")
    return nforce


def md_integrate_nested(geom: Geometry, U64, H, tau: float, steps, forces,
                        lam: float = OMELYAN_LAMBDA):
    """Multi-step (nested time-scale) integration: level 0 takes steps[0]
    Omelyan steps over tau with forces[0]; every drift of level k is a full
    integration of level k + 1 (steps[k + 1] steps) over that time; the
    innermost drift is the link update.  Typical use: the fermion force
    (expensive, smooth) outside, the gauge force inside.  Each level is the
    second-order minimum-norm scheme of md_integrate, so the composition is
    reversible and second order.  Returns the force evaluations per level."""
    if len(steps) != len(forces) or not steps or min(steps) < 1:
        raise ValueError("need one step count >= 1 per force")
    F = empty_links(geom, F64, LINKS18, U64.device)
    counts = [0] * len(steps)

    def kick(k, dt):
        forces[k](U64, F)
        counts[k] += 1
        md_update_momenta(geom, H, F, dt)

    def drift(k, t):
        if k == len(steps) - 1:
            md_update_links(geom, U64, H, t)
        else:
            level(k + 1, t)

    def level(k, T):
        n = steps[k]
        eps = T / n
        kick(k, lam * eps)
        for i in range(n):
            drift(k, 0.5 * eps)
            kick(k, (1.0 - 2.0 * lam) * eps)
            drift(k, 0.5 * eps)
            kick(k, (2.0 * lam if i < n - 1 else lam) * eps)

    level(0, float(tau))
    return counts


def rhmc_trajectory(geom: Geometry, params: SolverParams, U64, beta: float, approx_eighth,
                    approx_quarter, xi, H, u: float, tau: float = 1.0, nsteps: int = 10,
                    c1: float = SYMANZIK_C1, integrator: str = "omelyan",
                    gauge_substeps: int = 1, stout_rho: float = 0.0, stout_levels: int = 0):
    """One RHMC trajectory (Sec. 2, Sec. 4.3) for one staggered field with the
    pseudofermion action phi^dag A^(-1/4) phi (Eq. (1)):
      heatbath phi = r_{1/8}(A) xi; H_0 = H^2/2 + S_g + S_f;
      MD over tau with the gauge + fermion force (the fermion force from a
      multi-shift solve at the poles of r_{-1/4} at the current links);
      H_1; accept with probability min(1, exp(-(H_1 - H_0))) for the caller's
      uniform u, else restore the links.
    U64 (packed FP64 18-real) and H (packed momenta, Hermitian traceless) are
    updated in place; xi [n][3][Vh] packed even FP64 noise of density
    exp(-|xi|^2).  gauge_substeps > 1: multi-step integration, the fermion
    force on the nsteps outer steps and the gauge force on gauge_substeps
    inner steps per outer drift (Omelyan at both levels).  stout_levels > 0:
    the Dirac operator uses the stout-smeared links U^(k) (rho = stout_rho),
    the gauge action the unsmeared ones, and the fermion force is carried back
    through the smearing levels (Sec. 2).  Returns a dict with the energies,
    dH, accepted and counts."""
    U0 = U64.clone()
    q = approx_quarter

    def dirac_links(U):
        return stout_smear(geom, U, stout_rho, stout_levels) if stout_levels > 0 else [U]

    phi, _ = pseudofermion_heatbath(geom, params, dirac_links(U64)[-1], approx_eighth, xi)

    def energy():
        S_f, _, st = rational_action(geom, params, dirac_links(U64)[-1], q, phi)
        return kinetic_energy(geom, H), gauge_action(geom, U64, beta, c1), S_f

    def fermion_only(U, F):
        chain = dirac_links(U)
        X, _, _ = cg_multishift(geom, params, chain[-1], q.sigma, phi)
        if stout_levels > 0:
            G = fermion_force(geom, chain[-1], q.alpha, X, mode=1)
            F.copy_(stout_force(geom, chain, stout_rho, G, mode=0))
        else:
            fermion_force(geom, U, q.alpha, X, mode=0, out=F)
        del X

    def force(U, F):
        fermion_only(U, F)
        gauge_force(geom, U, beta, c1, out=F, accumulate=True)

    e0 = energy()
    if gauge_substeps > 1:
        nforce = md_integrate_nested(
            geom, U64, H, tau, [nsteps, gauge_substeps],
            [fermion_only, lambda U, F: gauge_force(geom, U, beta, c1, out=F)])[0]
    else:
        nforce = md_integrate(geom, U64, H, tau, nsteps, force, integrator)
    e1 = energy()
    h0, h1 = sum(e0), sum(e1)
    acc = metropolis_accept(h0, h1, u)
    if not acc:
        U64.copy_(U0)
    return dict(H0=h0, H1=h1, dH=h1 - h0, accepted=acc, force_evaluations=nforce,
                kinetic=(e0[0], e1[0]), gauge=(e0[1], e1[1]), fermion=(e0[2], e1[2]))


def stream_bandwidth(nbytes: int = 1 << 30, reps: int = 20):
    """(copy GB/s, triad GB/s) of the current device."""
    c = ctypes.c_double(0.0)
    t = ctypes.c_double(0.0)
    _check(_fn("lqcd_stream_bandwidth")(int(nbytes), int(reps), ctypes.byref(c), ctypes.byref(t)))
    return float(c.value), float(t.value)


def kernel_timing(enable: bool | None = None):
    """Enable/disable the solvers' per-kernel event timing, or (enable=None)
    return {class: (launches, total_ms)} accumulated so far."""
    if enable is not None:
        _check(_fn("lqcd_kernel_timing_enable")(1 if enable else 0))
        return None
    out = {}
    buf = ctypes.create_string_buffer(128)
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    i = 0
    while _fn("lqcd_kernel_timing_get")(i, buf, 128, ctypes.byref(n), ctypes.byref(ms)) == OK:
        out[buf.value.decode()] = (int(n.value), float(ms.value))
        i += 1
    return out


class FermionAction(torch.autograd.Function):
    """S_f(U) = sum_j [alpha0 |phi_j|^2 + sum_i alpha_i <phi_j, (A[U] + sigma_i)^-1 phi_j>].

    Forward: multi-shift CG for all shifts and pseudofermions, then the FP64
    action.  Backward: the adjoint force kernel in raw mode, whose output M^dag
    is torch's gradient for complex inputs (dS/dRe U + i dS/dIm U).

    U_nat: complex128 [4][V][3][3] on the GPU; phi: packed FP64 even [npf][3][Vh].
    """

    @staticmethod
    def forward(ctx, U_nat, phi, geom, alpha0, alpha, sigma, params):
        U64 = pack_links(geom, U_nat.detach().contiguous())
        X, _, _ = cg_multishift(geom, params, U64, sigma, phi)
        S = action(geom, alpha0, alpha, phi, X)
        ctx.save_for_backward(X)
        ctx.geom, ctx.alpha, ctx.U64 = geom, list(alpha), U64
        return torch.tensor(S, dtype=torch.float64, device=U_nat.device)

    @staticmethod
    def backward(ctx, grad_out):
        (X,) = ctx.saved_tensors
        G = fermion_force(ctx.geom, ctx.U64, ctx.alpha, X, mode=1)
        G_nat = unpack_links(ctx.geom, G)
        return grad_out * G_nat, None, None, None, None, None, None
