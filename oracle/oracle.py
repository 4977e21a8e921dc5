"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Wraps ``liboracle_fmgsr.so`` (built from ``fmgsr_oracle.c``) with numpy
arrays.  Nothing here does arithmetic of the method: every number comes from
the C oracle.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None

_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_ptr = ctypes.POINTER(ctypes.c_double)


class Options(ctypes.Structure):
    """Mirror of ``orc_options`` (see fmgsr_oracle.c)."""
    _fields_ = [("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32),
                ("nsr", ctypes.c_int32), ("rhs_restrict", ctypes.c_int32),
                ("tau_mode", ctypes.c_int32), ("smoother", ctypes.c_int32),
                ("tau_assembled", ctypes.c_int32), ("block_all", ctypes.c_int32)]


def options(nu1=2, nu2=1, nsr=1, rhs_restrict="fw", tau="split", smoother="rb",
            tau_assembled=False, block_all=0):
    return Options(nu1, nu2, nsr, {"fw": 0, "avg": 1}[rhs_restrict],
                   {"split": 0, "literal": 1}[tau], {"rb": 0, "lex": 1}[smoother],
                   int(bool(tau_assembled)), int(block_all))


class RxOptions(ctypes.Structure):
    """Mirror of ``orc_rx_options`` (see fmgsr_oracle_reaction.c)."""
    _fields_ = [("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32),
                ("nsr", ctypes.c_int32), ("tau_mode", ctypes.c_int32),
                ("tau_assembled", ctypes.c_int32)]


RX_KINDS = {"poisson": 0, "cubic": 1, "linear": 2}


def rx_options(nu1=2, nu2=1, nsr=1, tau="split", tau_assembled=False):
    return RxOptions(nu1, nu2, nsr, {"split": 0, "literal": 1}[tau], int(bool(tau_assembled)))


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.orc_apply_L.argtypes = [_ptr, _i64, _dbl, _dbl, _ptr]
        L.orc_restrict_avg.argtypes = [_ptr, _i64, _ptr]
        L.orc_restrict_fw.argtypes = [_ptr, _i64, _ptr]
        L.orc_prolong_linear.argtypes = [_ptr, _i64, _ptr]
        L.orc_interp_fmg.argtypes = [_ptr, _i64, _dbl, _dbl, _ptr]
        L.orc_rb_sweep.argtypes = [_ptr, _ptr, _i64, _i64, _i64, _dbl, _dbl]
        L.orc_lex_sweep.argtypes = [_ptr, _ptr, _i64, _i64, _i64, ctypes.c_int, _dbl, _dbl]
        L.orc_kaczmarz.argtypes = [_ptr, _i64, _i64, _i64, _ptr]
        L.orc_coarse_solve.argtypes = [_ptr, _i64, _dbl, _dbl, _ptr]
        L.orc_coarse_solve.restype = ctypes.c_int
        L.orc_smooth_blocks.argtypes = [_ptr, _ptr, _i64, _i64, _i64, ctypes.c_int,
                                        ctypes.c_int, _ptr, _dbl, _dbl, _ptr, ctypes.c_int]
        L.orc_smooth_blocks.restype = ctypes.c_int
        L.orc_fmgsr_solve_ex.argtypes = [_ptr, _dbl, _dbl, _i64, ctypes.c_int, _i64, _i64,
                                         ctypes.POINTER(Options), _ptr, ctypes.c_int]
        L.orc_fmgsr_solve_ex.restype = ctypes.c_int
        L.orc_fmgsr_solve_keep.argtypes = [_ptr, _dbl, _dbl, _i64, ctypes.c_int, _i64, _i64,
                                           ctypes.POINTER(Options), _ptr, _ptr]
        L.orc_fmgsr_solve_keep.restype = ctypes.c_int
        L.orc_fmgsr_decompress.argtypes = [_ptr, _ptr, _dbl, _dbl, _i64, _i64, _i64,
                                           ctypes.POINTER(Options), _i64, _i64, _ptr]
        L.orc_fmgsr_decompress.restype = ctypes.c_int
        L.orc_fas_vcycle.argtypes = [_ptr, _ptr, _dbl, _dbl, _i64, ctypes.c_int,
                                     ctypes.POINTER(Options)]
        L.orc_fas_vcycle.restype = ctypes.c_int
        _ci = ctypes.c_int
        L.orc_rx_apply.argtypes = [_ci, _ptr, _ptr, _i64, _dbl, _dbl, _ptr]
        L.orc_rx_ngs_sweep.argtypes = [_ci, _ptr, _ptr, _ptr, _i64, _i64, _i64, _dbl, _dbl]
        L.orc_rx_newton.argtypes = [_ci, _ptr, _ptr, _i64, _dbl, _dbl, _ptr, _ci, _dbl,
                                    ctypes.POINTER(_ci)]
        L.orc_rx_newton.restype = _ci
        L.orc_rx_fmgsr_solve_ex.argtypes = [_ci, _ptr, _ptr, _dbl, _dbl, _i64, _ci, _i64, _i64,
                                            ctypes.POINTER(RxOptions), _ptr, _ci]
        L.orc_rx_fmgsr_solve_ex.restype = _ci
        L.orc_rx_fmgsr_solve_keep.argtypes = [_ci, _ptr, _ptr, _dbl, _dbl, _i64, _ci, _i64, _i64,
                                              ctypes.POINTER(RxOptions), _ptr, _ptr]
        L.orc_rx_fmgsr_solve_keep.restype = _ci
        L.orc_rx_fas_vcycle.argtypes = [_ci, _ptr, _ptr, _ptr, _dbl, _dbl, _i64, _ci,
                                        ctypes.POINTER(RxOptions)]
        L.orc_rx_fas_vcycle.restype = _ci
        L.orc_rx_adjoint_direct.argtypes = [_ptr, _ptr, _ptr, _i64, _ptr, _ptr]
        L.orc_rx_adjoint_direct.restype = _ci
        L.orc_rx_fmgsr_adjoint.argtypes = [_ptr, _ptr, _ptr, _i64, _ci, _i64, _i64,
                                           ctypes.POINTER(RxOptions), _ptr, _ptr]
        L.orc_rx_fmgsr_adjoint.restype = _ci
        _LIB = L
    return _LIB


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_ptr)


def apply_L(u, gL=0.0, gR=0.0):
    u, pu = _c(u)
    out = np.empty_like(u)
    lib().orc_apply_L(pu, u.size, gL, gR, out.ctypes.data_as(_ptr))
    return out


def restrict_avg(u):
    u, pu = _c(u)
    out = np.empty(u.size // 2)
    lib().orc_restrict_avg(pu, u.size, out.ctypes.data_as(_ptr))
    return out


def restrict_fw(r):
    r, pr = _c(r)
    out = np.empty(r.size // 2)
    lib().orc_restrict_fw(pr, r.size, out.ctypes.data_as(_ptr))
    return out


def prolong_linear(e):
    e, pe = _c(e)
    out = np.empty(2 * e.size)
    lib().orc_prolong_linear(pe, e.size, out.ctypes.data_as(_ptr))
    return out


def interp_fmg(c, gL=0.0, gR=0.0):
    c, pc = _c(c)
    out = np.empty(2 * c.size)
    lib().orc_interp_fmg(pc, c.size, gL, gR, out.ctypes.data_as(_ptr))
    return out


def rb_sweep(u, F, lo=None, hi=None, gL=0.0, gR=0.0):
    u = np.array(u, dtype=np.float64, copy=True)
    F, pF = _c(F)
    n = u.size
    lib().orc_rb_sweep(u.ctypes.data_as(_ptr), pF, n, 0 if lo is None else lo,
                       n if hi is None else hi, gL, gR)
    return u


def lex_sweep(u, F, lo=None, hi=None, backward=False, gL=0.0, gR=0.0):
    u = np.array(u, dtype=np.float64, copy=True)
    F, pF = _c(F)
    n = u.size
    lib().orc_lex_sweep(u.ctypes.data_as(_ptr), pF, n, 0 if lo is None else lo,
                        n if hi is None else hi, int(backward), gL, gR)
    return u


def kaczmarz(u, c, lo=None, hi=None):
    u = np.array(u, dtype=np.float64, copy=True)
    c, pc = _c(c)
    n = u.size
    lib().orc_kaczmarz(u.ctypes.data_as(_ptr), n, 0 if lo is None else lo,
                       n if hi is None else hi, pc)
    return u


def coarse_solve(F, gL=0.0, gR=0.0):
    F, pF = _c(F)
    out = np.empty_like(F)
    st = lib().orc_coarse_solve(pF, F.size, gL, gR, out.ctypes.data_as(_ptr))
    if st != 0:
        raise RuntimeError(f"orc_coarse_solve failed: {st}")
    return out


def smooth_blocks(v, F, S, b, nu, smoother="rb", kaczmarz_c=None, gL=0.0, gR=0.0, order=0):
    v, pv = _c(v)
    F, pF = _c(F)
    out = np.empty_like(v)
    if kaczmarz_c is not None:
        kc, pk = _c(kaczmarz_c)
    else:
        kc, pk = None, None
    st = lib().orc_smooth_blocks(pv, pF, v.size, S, b, nu, {"rb": 0, "lex": 1}[smoother],
                                 pk, gL, gR, out.ctypes.data_as(_ptr), order)
    if st != 0:
        raise RuntimeError(f"orc_smooth_blocks failed: {st}")
    return out


def fmgsr_solve(f, gL=0.0, gR=0.0, levels=None, segments=1, buffer=0, order=0, **opt):
    """One FMG-FAS(-SR) iteration.  ``opt`` are the keywords of ``options``."""
    f, pf = _c(f)
    n = f.size
    if levels is None:
        levels = int(np.log2(n)) + 1
    o = options(**opt)
    out = np.empty_like(f)
    st = lib().orc_fmgsr_solve_ex(pf, gL, gR, n, levels, segments, buffer,
                                  ctypes.byref(o), out.ctypes.data_as(_ptr), order)
    if st != 0:
        raise ValueError(f"orc_fmgsr_solve failed with status {st}")
    return out


def fmgsr_solve_keep(f, gL=0.0, gR=0.0, levels=None, segments=1, buffer=0, **opt):
    """One FMG-FAS(-SR) iteration returning (u, c): the finest level and the
    level-(M-1) solution of the final V-cycle (the PDE-compressed form)."""
    f, pf = _c(f)
    n = f.size
    if levels is None:
        levels = int(np.log2(n)) + 1
    o = options(**opt)
    out = np.empty_like(f)
    c = np.empty(n // 2)
    st = lib().orc_fmgsr_solve_keep(pf, gL, gR, n, levels, segments, buffer, ctypes.byref(o),
                                    out.ctypes.data_as(_ptr), c.ctypes.data_as(_ptr))
    if st != 0:
        raise ValueError(f"orc_fmgsr_solve_keep failed with status {st}")
    return out, c


def fmgsr_decompress(c, f, lo, hi, gL=0.0, gR=0.0, segments=1, buffer=0, **opt):
    """Fine solution on [lo, hi) expanded from the level-(M-1) solution c."""
    c, pc = _c(c)
    f, pf = _c(f)
    o = options(**opt)
    out = np.empty(max(hi - lo, 0))
    st = lib().orc_fmgsr_decompress(pc, pf, gL, gR, f.size, segments, buffer, ctypes.byref(o),
                                    lo, hi, out.ctypes.data_as(_ptr))
    if st != 0:
        raise ValueError(f"orc_fmgsr_decompress failed with status {st}")
    return out


def fas_vcycle(u, f, gL=0.0, gR=0.0, levels=None, **opt):
    """One FAS V-cycle (Fig. 1) from iterate u; returns the new iterate."""
    u = np.array(u, dtype=np.float64, copy=True)
    f, pf = _c(f)
    n = f.size
    if levels is None:
        levels = int(np.log2(n)) + 1
    o = options(**opt)
    st = lib().orc_fas_vcycle(u.ctypes.data_as(_ptr), pf, gL, gR, n, levels, ctypes.byref(o))
    if st != 0:
        raise ValueError(f"orc_fas_vcycle failed with status {st}")
    return u


# ---------------------------------------------------------------------------
# Reaction operators (fmgsr_oracle_reaction.c)
# ---------------------------------------------------------------------------

def _coef(kind, a, n):
    if a is None:
        if RX_KINDS[kind] != 0:
            raise ValueError("the reaction kinds need a coefficient")
        a = np.zeros(n)
    return _c(a)


def rx_apply(kind, a, u, gL=0.0, gR=0.0):
    """N(u) = L u + R(u) (R13)."""
    u, pu = _c(u)
    a, pa = _coef(kind, a, u.size)
    out = np.empty_like(u)
    lib().orc_rx_apply(RX_KINDS[kind], pa, pu, u.size, gL, gR, out.ctypes.data_as(_ptr))
    return out


def rx_ngs_sweep(kind, a, u, F, lo=None, hi=None, gL=0.0, gR=0.0):
    u = np.array(u, dtype=np.float64, copy=True)
    F, pF = _c(F)
    a, pa = _coef(kind, a, u.size)
    n = u.size
    lib().orc_rx_ngs_sweep(RX_KINDS[kind], pa, u.ctypes.data_as(_ptr), pF, n,
                           0 if lo is None else lo, n if hi is None else hi, gL, gR)
    return u


def rx_newton(kind, a, F, gL=0.0, gR=0.0, u0=None, max_it=30, rtol=1e-14):
    """Newton's method with exact tridiagonal steps (R17); returns (u, steps)."""
    F, pF = _c(F)
    a, pa = _coef(kind, a, F.size)
    u = np.zeros_like(F) if u0 is None else np.array(u0, dtype=np.float64, copy=True)
    it = ctypes.c_int(0)
    st = lib().orc_rx_newton(RX_KINDS[kind], pa, pF, F.size, gL, gR, u.ctypes.data_as(_ptr),
                             max_it, rtol, ctypes.byref(it))
    if st != 0:
        raise RuntimeError(f"orc_rx_newton failed: {st}")
    return u, it.value


def rx_fmgsr_solve(kind, f, a=None, gL=0.0, gR=0.0, levels=None, segments=1, buffer=0,
                   order=0, **opt):
    """One FMG-FAS(-SR) iteration for the reaction operators (R13-R17)."""
    f, pf = _c(f)
    n = f.size
    a, pa = _coef(kind, a, n)
    if levels is None:
        levels = int(np.log2(n)) + 1
    o = rx_options(**opt)
    out = np.empty_like(f)
    st = lib().orc_rx_fmgsr_solve_ex(RX_KINDS[kind], pf, pa, gL, gR, n, levels, segments, buffer,
                                     ctypes.byref(o), out.ctypes.data_as(_ptr), order)
    if st != 0:
        raise ValueError(f"orc_rx_fmgsr_solve failed with status {st}")
    return out


def rx_fmgsr_solve_keep(kind, f, a=None, gL=0.0, gR=0.0, levels=None, segments=1, buffer=0,
                        **opt):
    """rx_fmgsr_solve, also returning the level-(M-1) solution the iteration
    ends with (Sec. 2.4): (u, coarse)."""
    f, pf = _c(f)
    n = f.size
    a, pa = _coef(kind, a, n)
    if levels is None:
        levels = int(np.log2(n)) + 1
    o = rx_options(**opt)
    out = np.empty_like(f)
    coarse = np.empty(n // 2, dtype=np.float64)
    st = lib().orc_rx_fmgsr_solve_keep(RX_KINDS[kind], pf, pa, gL, gR, n, levels, segments,
                                       buffer, ctypes.byref(o), out.ctypes.data_as(_ptr),
                                       coarse.ctypes.data_as(_ptr))
    if st != 0:
        raise ValueError(f"orc_rx_fmgsr_solve_keep failed with status {st}")
    return out, coarse


def rx_fas_vcycle(kind, u, f, a=None, gL=0.0, gR=0.0, levels=None, **opt):
    u = np.array(u, dtype=np.float64, copy=True)
    f, pf = _c(f)
    n = f.size
    a, pa = _coef(kind, a, n)
    if levels is None:
        levels = int(np.log2(n)) + 1
    o = rx_options(**opt)
    st = lib().orc_rx_fas_vcycle(RX_KINDS[kind], u.ctypes.data_as(_ptr), pf, pa, gL, gR, n,
                                 levels, ctypes.byref(o))
    if st != 0:
        raise ValueError(f"orc_rx_fas_vcycle failed with status {st}")
    return u


def rx_adjoint_direct(kappa, u, dJdu):
    """(grad_f, grad_kappa) from the exact adjoint solve (R18)."""
    kappa, pk = _c(kappa)
    u, pu = _c(u)
    dJdu, pd = _c(dJdu)
    gf, gk = np.empty_like(u), np.empty_like(u)
    st = lib().orc_rx_adjoint_direct(pk, pu, pd, u.size, gf.ctypes.data_as(_ptr),
                                     gk.ctypes.data_as(_ptr))
    if st != 0:
        raise RuntimeError(f"orc_rx_adjoint_direct failed: {st}")
    return gf, gk


def rx_fmgsr_adjoint(kappa, u, dJdu, levels=None, segments=1, buffer=0, **opt):
    """(grad_f, grad_kappa) with lambda from one FMG-FAS-SR iteration (R18)."""
    kappa, pk = _c(kappa)
    u, pu = _c(u)
    dJdu, pd = _c(dJdu)
    n = u.size
    if levels is None:
        levels = int(np.log2(n)) + 1
    o = rx_options(**opt)
    gf, gk = np.empty_like(u), np.empty_like(u)
    st = lib().orc_rx_fmgsr_adjoint(pk, pu, pd, n, levels, segments, buffer, ctypes.byref(o),
                                    gf.ctypes.data_as(_ptr), gk.ctypes.data_as(_ptr))
    if st != 0:
        raise ValueError(f"orc_rx_fmgsr_adjoint failed with status {st}")
    return gf, gk
