"""Python binding of the gfx950 FMG-FAS-SR library (``libfmgsr.so``).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch provides device memory and the current stream.  There is
no fallback: if the library is missing or no GPU is present the calls raise.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmgsr.so")

FMGSR_OK, FMGSR_EINVAL, FMGSR_ENOMEM, FMGSR_EDEVICE, FMGSR_ENOTSUP = 0, -1, -2, -3, -4
FMGSR_ENONFINITE = -5
TAU_MODES = {"split": 0, "literal": 1}
RHS_RESTRICTIONS = {"fw": 0, "avg": 1}
OPS = {"poisson": 0, "cubic": 1, "linear": 2}
PRECISIONS = {"fp64": 0, "fp32relax": 1}

_lib = None


class Options(ctypes.Structure):
    """Mirror of ``fmgsr_options`` (include/fmgsr.h)."""
    _fields_ = [("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32),
                ("sr_levels", ctypes.c_int32), ("tau_mode", ctypes.c_int32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("functionals", ctypes.c_void_p), ("coarse_out", ctypes.c_void_p),
                ("rhs_restriction", ctypes.c_int32), ("check_finite", ctypes.c_int32)]


class Operator(ctypes.Structure):
    """Mirror of ``fmgsr_operator``."""
    _fields_ = [("kind", ctypes.c_int32), ("kappa", ctypes.c_void_p)]


class BatchShape(ctypes.Structure):
    """Mirror of ``fmgsr_batch_shape``."""
    _fields_ = [("threads", ctypes.c_int32), ("run", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("halo", ctypes.c_int32), ("lds_bytes", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("group", ctypes.c_int32),
                ("stalled", ctypes.c_int32)]


class KernelStat(ctypes.Structure):
    """Mirror of ``fmgsr_kernel_stat``."""
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("algo_bytes", ctypes.c_double)]


class FmgsrError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {lib().fmgsr_status_string(status).decode()}")


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no non-HIP fallback)")
        L = ctypes.CDLL(LIB_PATH)
        L.fmgsr_default_options.argtypes = [ctypes.POINTER(Options)]
        L.fmgsr_default_options.restype = None
        L.fmgsr_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(Options)]
        L.fmgsr_workspace_bytes.restype = ctypes.c_size_t
        L.fmgsr_workspace_bytes_for.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                                ctypes.c_int32, ctypes.POINTER(Options)]
        L.fmgsr_workspace_bytes_for.restype = ctypes.c_size_t
        L.fmgsr_launch_lds_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                             ctypes.c_int32, ctypes.POINTER(Options)]
        L.fmgsr_launch_lds_bytes.restype = ctypes.c_size_t
        L.fmgsr_solve.argtypes = [ctypes.POINTER(Operator), ctypes.c_void_p, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_int32, ctypes.POINTER(Options), ctypes.c_void_p,
                                  ctypes.c_void_p]
        L.fmgsr_solve.restype = ctypes.c_int
        L.fmgsr_solve_noalloc.argtypes = L.fmgsr_solve.argtypes
        L.fmgsr_solve_noalloc.restype = ctypes.c_int
        L.fmgsr_decompress.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int32, ctypes.POINTER(Options), ctypes.c_int64,
                                       ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
        L.fmgsr_decompress.restype = ctypes.c_int
        L.fmgsr_status_string.argtypes = [ctypes.c_int32]
        L.fmgsr_status_string.restype = ctypes.c_char_p
        L.fmgsr_profile_enable.argtypes = [ctypes.c_char_p]
        L.fmgsr_profile_enable.restype = ctypes.c_int
        L.fmgsr_profile_collect.argtypes = [ctypes.POINTER(KernelStat), ctypes.c_int32]
        L.fmgsr_profile_collect.restype = ctypes.c_int32
        L.fmgsr_version.argtypes = []
        L.fmgsr_version.restype = ctypes.c_char_p
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.fmgsr_batch_create.argtypes = [i32, vp, vp, vp, vp, i32, vp, i32,
                                         ctypes.POINTER(Options), ctypes.POINTER(vp)]
        L.fmgsr_batch_solve.argtypes = [vp, vp, vp, vp, vp]
        L.fmgsr_batch_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.fmgsr_batch_solve_keep.argtypes = [vp, vp, vp, vp, vp, vp]
        L.fmgsr_batch_adjoint_compressed.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.fmgsr_batch_autotune.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double)]
        L.fmgsr_batch_query.argtypes = [vp, ctypes.POINTER(BatchShape), vp]
        L.fmgsr_batch_destroy.argtypes = [vp]
        L.fmgsr_solve_batched.argtypes = [i32, vp, vp, vp, vp, i32, ctypes.POINTER(Operator), vp,
                                          vp, ctypes.POINTER(Options), vp, vp]
        L.fmgsr_adjoint.argtypes = [ctypes.POINTER(Operator), vp, ctypes.c_double,
                                    ctypes.c_double, i64, i32, i64, i32, ctypes.POINTER(Options),
                                    vp, vp, vp, vp, vp]
        for name in ("fmgsr_batch_create", "fmgsr_batch_solve", "fmgsr_batch_adjoint",
                     "fmgsr_batch_solve_keep", "fmgsr_batch_adjoint_compressed",
                     "fmgsr_batch_autotune", "fmgsr_batch_query", "fmgsr_batch_destroy",
                     "fmgsr_solve_batched", "fmgsr_adjoint"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def make_options(nu=(2, 1), sr_levels=1, tau="split", workspace=None, precision="fp64",
                 rhs_restrict="fw", check_finite=False):
    o = Options()
    lib().fmgsr_default_options(ctypes.byref(o))
    o.nu1, o.nu2 = int(nu[0]), int(nu[1])
    o.sr_levels = int(sr_levels)
    o.tau_mode = TAU_MODES[tau]
    o.precision = PRECISIONS[precision]
    o.rhs_restriction = RHS_RESTRICTIONS[rhs_restrict]
    o.check_finite = int(bool(check_finite))
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    return o


def workspace_bytes(n, levels, nu=(2, 1), sr_levels=1, tau="split", segments=None, buffer=None,
                    functionals=False, coarse_out=False, rhs_restrict="fw"):
    """Workspace bytes for any segments, or (segments and buffer given) for
    exactly these segments and buffer."""
    o = make_options(nu, sr_levels, tau, rhs_restrict=rhs_restrict)
    if functionals:
        o.functionals = ctypes.c_void_p(1)  # only its presence matters for the size
    if coarse_out:
        o.coarse_out = ctypes.c_void_p(1)
    if segments is None:
        return int(lib().fmgsr_workspace_bytes(int(n), int(levels), ctypes.byref(o)))
    return int(lib().fmgsr_workspace_bytes_for(int(n), int(levels), int(segments), int(buffer),
                                               ctypes.byref(o)))


def launch_lds_bytes(n, levels, segments, buffer, nu=(2, 1), sr_levels=1, tau="split"):
    """Largest dynamic LDS one workgroup of this solve requests."""
    o = make_options(nu, sr_levels, tau)
    return int(lib().fmgsr_launch_lds_bytes(int(n), int(levels), int(segments), int(buffer),
                                            ctypes.byref(o)))


def alloc_workspace(n, levels, device, **kw):
    nbytes = workspace_bytes(n, levels, **kw)
    if nbytes == 0:
        raise FmgsrError(FMGSR_EINVAL, "fmgsr_workspace_bytes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _check_vec(t, name, numel=None, at_least=None, device=None):
    """Reject anything the C ABI could not use safely: the library sees raw
    pointers only, so a short array or a float32 one would be read and
    written past its end on the device.  numel: exact element count;
    at_least: minimum count (packed batch arrays); device: must match."""
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous() and t.dim() == 1):
        raise ValueError(f"{name} must be a contiguous 1-D float64 tensor on the GPU")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    if at_least is not None and t.numel() < at_least:
        raise ValueError(f"{name} has {t.numel()} elements, the packed extent is {at_least}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")


def _check_workspace(ws, device):
    if not (isinstance(ws, torch.Tensor) and ws.is_cuda and ws.is_contiguous()
            and ws.device == device):
        raise ValueError("workspace must be a contiguous GPU tensor on the solve's device")


def solve(f, g=(0.0, 0.0), levels=None, segments=1, buffer=0, nu=(2, 1), sr_levels=1,
          tau="split", out=None, workspace=None, stream=None, op="poisson", kappa=None,
          precision="fp64", functionals=None, write_u=True, coarse_out=None, rhs_restrict="fw",
          check_finite=False):
    """One FMG-FAS-SR iteration for -u'' (+ reaction) = f on [0,1] (see
    include/fmgsr.h).

    f: contiguous float64 tensor on the GPU.  Returns u (same shape), or None
    with ``write_u=False``.  The call is asynchronous on ``stream`` (default:
    torch's current stream); the reaction operators (``op`` = "cubic" or
    "linear" with ``kappa``) run synchronously as a batch of one.
    coarse_out: float64 tensor of n/2 cells that receives the level-(M-1)
    solution (the PDE-compressed form ``decompress`` expands).
    rhs_restrict: "fw" (full weighting) or "avg" (two-cell average, literal
    tau only).  check_finite: refuse a non-finite f or result with
    FMGSR_ENONFINITE (synchronises the stream).
    """
    return _solve("fmgsr_solve", f, g, levels, segments, buffer, nu, sr_levels, tau, out,
                  workspace, stream, op, kappa, precision, functionals, write_u, coarse_out,
                  rhs_restrict, check_finite)


def solve_noalloc(f, g=(0.0, 0.0), levels=None, segments=1, buffer=0, nu=(2, 1), sr_levels=1,
                  tau="split", out=None, stream=None, precision="fp64", functionals=None,
                  write_u=True, rhs_restrict="fw", check_finite=False):
    """``solve`` through ``fmgsr_solve_noalloc``: the library's static device
    scratch serves as workspace, so the call allocates nothing on the device
    (``out`` must then be given by callers that cannot allocate either).
    Poisson operator only; calls that overlap on one GPU race."""
    return _solve("fmgsr_solve_noalloc", f, g, levels, segments, buffer, nu, sr_levels, tau, out,
                  None, stream, "poisson", None, precision, functionals, write_u, None,
                  rhs_restrict, check_finite)


def _solve(entry, f, g, levels, segments, buffer, nu, sr_levels, tau, out, workspace, stream, op,
           kappa, precision, functionals, write_u, coarse_out, rhs_restrict, check_finite):
    _check_vec(f, "f")
    n = f.numel()
    if op not in OPS:
        raise ValueError(f"unknown operator {op!r}")
    if (op == "poisson") != (kappa is None):
        raise ValueError("kappa is required for the reaction operators and refused for poisson")
    if kappa is not None:
        _check_vec(kappa, "kappa", numel=n, device=f.device)
    if levels is None:
        levels = n.bit_length()  # n a power of two -> N0 = 1
    if not write_u:
        if functionals is None and coarse_out is None:
            raise ValueError("write_u=False needs a functionals or a coarse_out tensor")
        out = None
    elif out is None:
        out = torch.empty_like(f)
    else:
        _check_vec(out, "out", numel=n, device=f.device)
    if functionals is not None:
        _check_vec(functionals, "functionals", at_least=2, device=f.device)
    if coarse_out is not None:
        _check_vec(coarse_out, "coarse_out", numel=n // 2, device=f.device)
    if workspace is not None:
        _check_workspace(workspace, f.device)
    if stream is None:
        stream = torch.cuda.current_stream(f.device)
    o = make_options(nu, sr_levels, tau, workspace, precision, rhs_restrict, check_finite)
    if functionals is not None:
        o.functionals = functionals.data_ptr()
    if coarse_out is not None:
        o.coarse_out = coarse_out.data_ptr()
    op = Operator(OPS[op], kappa.data_ptr() if kappa is not None else None)
    st = getattr(lib(), entry)(ctypes.byref(op), f.data_ptr(), float(g[0]), float(g[1]), n,
                               int(levels), int(segments), int(buffer), ctypes.byref(o),
                               out.data_ptr() if out is not None else None,
                               ctypes.c_void_p(stream.cuda_stream))
    if st != FMGSR_OK:
        raise FmgsrError(st, entry)
    return out


def decompress(coarse, f, lo=0, hi=None, g=(0.0, 0.0), segments=1, buffer=0, nu=(2, 1),
               precision="fp64", out=None, stream=None):
    """Finest-level solution on cells [lo, hi) expanded from the level-(M-1)
    solution ``coarse`` (``solve(..., coarse_out=...)``) and f by the SR up
    pass of the covering segments (fmgsr_decompress).  Returns a tensor of
    hi - lo cells; asynchronous on ``stream``."""
    _check_vec(f, "f")
    n = f.numel()
    _check_vec(coarse, "coarse", numel=n // 2, device=f.device)
    hi = n if hi is None else int(hi)
    lo = int(lo)
    if not 0 <= lo <= hi <= n:
        raise ValueError(f"range [{lo}, {hi}) is not inside [0, {n}]")
    if out is None:
        out = torch.empty(hi - lo, dtype=torch.float64, device=f.device)
    else:
        _check_vec(out, "out", numel=hi - lo, device=f.device)
    if hi == lo:
        return out
    o = make_options(nu, 1, "split", None, precision)
    s = (stream or torch.cuda.current_stream(f.device)).cuda_stream
    st = lib().fmgsr_decompress(coarse.data_ptr(), f.data_ptr(), float(g[0]), float(g[1]), n,
                                int(segments), int(buffer), ctypes.byref(o), lo, hi,
                                out.data_ptr(), ctypes.c_void_p(s))
    if st != FMGSR_OK:
        raise FmgsrError(st, "fmgsr_decompress")
    return out


class Batch:
    """A batched-solve plan (``fmgsr_batch_create``): many independent
    problems of uneven size solved in one persistent launch.

    sizes, levels: per-problem fine cells and grids; segments: per-problem SR
    segment counts or None (library choice); g: [batch, 2] Dirichlet values
    or None.  Packed device arrays put problem j at ``offsets[j]``."""

    def __init__(self, sizes, levels, buffer=8, segments=None, g=None, op="cubic", nu=(2, 1),
                 precision="fp64", offsets=None):
        import numpy as np
        self.batch = len(sizes)
        self.sizes = np.ascontiguousarray(sizes, dtype=np.int64)
        self.levels = np.ascontiguousarray(levels, dtype=np.int32)
        self.offsets = (np.concatenate([[0], np.cumsum(self.sizes)[:-1]]).astype(np.int64)
                        if offsets is None else np.ascontiguousarray(offsets, dtype=np.int64))
        self.total = int((self.offsets + self.sizes).max())
        # the kept level-(M-1) solutions: problem j at offsets[j] // 2, n_j / 2 values
        multi = self.levels > 1
        self.coarse_total = (int((self.offsets[multi] // 2 + self.sizes[multi] // 2).max())
                             if multi.any() else 0)
        self.op = op
        seg = None if segments is None else np.ascontiguousarray(segments, dtype=np.int64)
        gh = None if g is None else np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
        o = make_options(nu, 1, "split", None, precision)
        h = ctypes.c_void_p()
        ptr = lambda a: None if a is None else a.ctypes.data
        st = lib().fmgsr_batch_create(self.batch, ptr(self.sizes), ptr(self.offsets),
                                      ptr(self.levels), ptr(seg), int(buffer), ptr(gh), OPS[op],
                                      ctypes.byref(o), ctypes.byref(h))
        if st != FMGSR_OK:
            raise FmgsrError(st, "fmgsr_batch_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.fmgsr_batch_destroy(h)
            self._h = None

    def _stream(self, stream, dev):
        return (stream or torch.cuda.current_stream(dev)).cuda_stream

    def _coef(self, kappa, dev):
        if self.op == "poisson":
            if kappa is not None:
                raise ValueError("a poisson plan takes no kappa")
            return None
        _check_vec(kappa, "kappa", at_least=self.total, device=dev)
        return kappa

    def solve(self, f, kappa=None, out=None, stream=None):
        _check_vec(f, "f", at_least=self.total)
        kappa = self._coef(kappa, f.device)
        if out is None:
            out = torch.empty_like(f)
        else:
            _check_vec(out, "out", at_least=self.total, device=f.device)
        st = lib().fmgsr_batch_solve(self._h, f.data_ptr(),
                                     kappa.data_ptr() if kappa is not None else None,
                                     out.data_ptr(), self._stream(stream, f.device))
        if st != FMGSR_OK:
            raise FmgsrError(st, "fmgsr_batch_solve")
        return out

    def solve_keep(self, f, kappa=None, coarse=None, out=None, write_u=True, stream=None):
        """(u or None, coarse): the iteration keeping every problem's
        level-(M-1) solution (fmgsr_batch_solve_keep); write_u=False skips
        the finest level (compression only)."""
        _check_vec(f, "f", at_least=self.total)
        kappa = self._coef(kappa, f.device)
        if coarse is None:
            coarse = torch.empty(max(self.coarse_total, 1), dtype=torch.float64, device=f.device)
        else:
            _check_vec(coarse, "coarse", at_least=max(self.coarse_total, 1), device=f.device)
        if write_u:
            if out is None:
                out = torch.empty_like(f)
            else:
                _check_vec(out, "out", at_least=self.total, device=f.device)
        else:
            out = None
        st = lib().fmgsr_batch_solve_keep(self._h, f.data_ptr(),
                                          kappa.data_ptr() if kappa is not None else None,
                                          out.data_ptr() if out is not None else None,
                                          coarse.data_ptr(), self._stream(stream, f.device))
        if st != FMGSR_OK:
            raise FmgsrError(st, "fmgsr_batch_solve_keep")
        return out, coarse

    def adjoint_compressed(self, kappa, f_fwd, coarse_fwd, dJdu, grad_f=None, grad_kappa=None,
                           stream=None):
        """(grad_f, grad_kappa) like ``adjoint``, u_fwd rebuilt from the
        forward's rhs and kept level (fmgsr_batch_adjoint_compressed)."""
        if self.op != "cubic":
            raise ValueError("the adjoint needs a plan made for the cubic operator")
        _check_vec(dJdu, "dJdu", at_least=self.total)
        dev = dJdu.device
        _check_vec(kappa, "kappa", at_least=self.total, device=dev)
        _check_vec(f_fwd, "f_fwd", at_least=self.total, device=dev)
        _check_vec(coarse_fwd, "coarse_fwd", at_least=max(self.coarse_total, 1), device=dev)
        if grad_f is None:
            grad_f = torch.empty_like(dJdu)
        else:
            _check_vec(grad_f, "grad_f", at_least=self.total, device=dev)
        if grad_kappa is None:
            grad_kappa = torch.empty_like(dJdu)
        else:
            _check_vec(grad_kappa, "grad_kappa", at_least=self.total, device=dev)
        st = lib().fmgsr_batch_adjoint_compressed(
            self._h, kappa.data_ptr(), f_fwd.data_ptr(), coarse_fwd.data_ptr(), dJdu.data_ptr(),
            grad_f.data_ptr(), grad_kappa.data_ptr(), self._stream(stream, dev))
        if st != FMGSR_OK:
            raise FmgsrError(st, "fmgsr_batch_adjoint_compressed")
        return grad_f, grad_kappa

    def adjoint(self, kappa, u_fwd, dJdu, grad_f=None, grad_kappa=None, stream=None):
        """(grad_f, grad_kappa) of J with dJ/du = dJdu (fmgsr_batch_adjoint)."""
        if self.op != "cubic":
            raise ValueError("the adjoint needs a plan made for the cubic operator")
        _check_vec(dJdu, "dJdu", at_least=self.total)
        dev = dJdu.device
        _check_vec(kappa, "kappa", at_least=self.total, device=dev)
        _check_vec(u_fwd, "u_fwd", at_least=self.total, device=dev)
        if grad_f is None:
            grad_f = torch.empty_like(dJdu)
        else:
            _check_vec(grad_f, "grad_f", at_least=self.total, device=dev)
        if grad_kappa is None:
            grad_kappa = torch.empty_like(dJdu)
        else:
            _check_vec(grad_kappa, "grad_kappa", at_least=self.total, device=dev)
        st = lib().fmgsr_batch_adjoint(self._h, kappa.data_ptr(), u_fwd.data_ptr(),
                                       dJdu.data_ptr(), grad_f.data_ptr(), grad_kappa.data_ptr(),
                                       self._stream(stream, dJdu.device))
        if st != FMGSR_OK:
            raise FmgsrError(st, "fmgsr_batch_adjoint")
        return grad_f, grad_kappa

    def autotune(self, f, kappa=None, scratch=None, stream=None):
        _check_vec(f, "f", at_least=self.total)
        kappa = self._coef(kappa, f.device)
        if scratch is None:
            scratch = torch.empty_like(f)
        else:
            _check_vec(scratch, "scratch", at_least=self.total, device=f.device)
        ms = ctypes.c_double(0.0)
        st = lib().fmgsr_batch_autotune(self._h, f.data_ptr(),
                                        kappa.data_ptr() if kappa is not None else None,
                                        scratch.data_ptr(), self._stream(stream, f.device),
                                        ctypes.byref(ms))
        if st != FMGSR_OK:
            raise FmgsrError(st, "fmgsr_batch_autotune")
        return ms.value

    def query(self):
        import numpy as np
        sh = BatchShape()
        segs = np.zeros(self.batch, dtype=np.int64)
        st = lib().fmgsr_batch_query(self._h, ctypes.byref(sh), segs.ctypes.data)
        if st != FMGSR_OK:
            raise FmgsrError(st, "fmgsr_batch_query")
        return {"threads": sh.threads, "run": sh.run, "grid": sh.grid, "halo": sh.halo,
                "lds_bytes": sh.lds_bytes, "workspace_bytes": sh.workspace_bytes,
                "group": sh.group, "stalled": sh.stalled, "segments": segs}


def adjoint(f, kappa, dJdu, g=(0.0, 0.0), levels=None, segments=0, buffer=8, nu=(2, 1),
            u_fwd=None, precision="fp64", stream=None):
    """(grad_f, grad_kappa) for one cubic problem (fmgsr_adjoint; synchronous)."""
    _check_vec(f, "f")
    n = f.numel()
    for t, nm in ((kappa, "kappa"), (dJdu, "dJdu")):
        _check_vec(t, nm, numel=n, device=f.device)
    if u_fwd is not None:
        _check_vec(u_fwd, "u_fwd", numel=n, device=f.device)
    if levels is None:
        levels = n.bit_length()
    gf, gk = torch.empty_like(f), torch.empty_like(f)
    o = make_options(nu, 1, "split", None, precision)
    op = Operator(OPS["cubic"], kappa.data_ptr())
    s = (stream or torch.cuda.current_stream(f.device)).cuda_stream
    st = lib().fmgsr_adjoint(ctypes.byref(op), f.data_ptr(), float(g[0]), float(g[1]), n,
                             int(levels), int(segments), int(buffer), ctypes.byref(o),
                             u_fwd.data_ptr() if u_fwd is not None else None, dJdu.data_ptr(),
                             gf.data_ptr(), gk.data_ptr(), s)
    if st != FMGSR_OK:
        raise FmgsrError(st, "fmgsr_adjoint")
    return gf, gk


class CubicSolve(torch.autograd.Function):
    """u = FMG-FAS-SR solution of -u'' + kappa u^3 = f for every problem of a
    batch plan, differentiable in f and kappa: the backward pass runs the
    library's adjoint, i.e. the gradient of the discrete solution map, with
    lambda from one FMG-SR iteration.

        u = CubicSolve.apply(f, kappa, plan)           # keeps the coarse level
        u = CubicSolve.apply(f, kappa, plan, "u")      # keeps u

    keep="coarse" (default, Sec. 2.4): the forward keeps its level-(M-1)
    solution (n/2 values) and the backward rebuilds u_fwd from it and f
    (fmgsr_batch_adjoint_compressed; more arithmetic, less memory).
    keep="u": u itself is saved (fmgsr_batch_adjoint).  Both give the same
    gradients bit for bit."""

    @staticmethod
    def forward(ctx, f, kappa, plan, keep="coarse"):
        if keep not in ("coarse", "u"):
            raise ValueError("keep is 'coarse' or 'u'")
        ctx.plan = plan
        ctx.keep = keep
        if keep == "coarse":
            u, coarse = plan.solve_keep(f.detach(), kappa.detach())
            ctx.save_for_backward(kappa, f, coarse)
        else:
            u = plan.solve(f.detach(), kappa.detach())
            ctx.save_for_backward(kappa, u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        if ctx.keep == "coarse":
            kappa, f, coarse = ctx.saved_tensors
            gf, gk = ctx.plan.adjoint_compressed(kappa.detach(), f.detach(), coarse,
                                                 grad_u.contiguous())
        else:
            kappa, u = ctx.saved_tensors
            gf, gk = ctx.plan.adjoint(kappa, u, grad_u.contiguous())
        return gf, gk, None, None


def profile_enable(kernel_filter=None):
    """Bracket every library kernel launch (matching ``kernel_filter``) with
    HIP events on its stream until ``profile_collect``."""
    st = lib().fmgsr_profile_enable(kernel_filter.encode() if kernel_filter else None)
    if st != FMGSR_OK:
        raise FmgsrError(st, "fmgsr_profile_enable")


def profile_collect():
    """Return {kernel: {"launches", "total_ms", "algo_bytes"}} and stop recording."""
    buf = (KernelStat * 64)()
    k = lib().fmgsr_profile_collect(buf, 64)
    if k < 0:
        raise FmgsrError(k, "fmgsr_profile_collect")
    return {buf[i].name.decode(): {"launches": buf[i].launches, "total_ms": buf[i].total_ms,
                                   "algo_bytes": buf[i].algo_bytes} for i in range(min(k, 64))}


def version():
    return lib().fmgsr_version().decode()
