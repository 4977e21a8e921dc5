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
TAU_MODES = {"split": 0, "literal": 1}

_lib = None


class Options(ctypes.Structure):
    """Mirror of ``fmgsr_options`` (include/fmgsr.h)."""
    _fields_ = [("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32),
                ("sr_levels", ctypes.c_int32), ("tau_mode", ctypes.c_int32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


class Operator(ctypes.Structure):
    """Mirror of ``fmgsr_operator``."""
    _fields_ = [("kind", ctypes.c_int32), ("kappa", ctypes.c_void_p)]


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
        L.fmgsr_solve.argtypes = [ctypes.POINTER(Operator), ctypes.c_void_p, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_int32, ctypes.POINTER(Options), ctypes.c_void_p,
                                  ctypes.c_void_p]
        L.fmgsr_solve.restype = ctypes.c_int
        L.fmgsr_status_string.argtypes = [ctypes.c_int32]
        L.fmgsr_status_string.restype = ctypes.c_char_p
        L.fmgsr_profile_enable.argtypes = [ctypes.c_char_p]
        L.fmgsr_profile_enable.restype = ctypes.c_int
        L.fmgsr_profile_collect.argtypes = [ctypes.POINTER(KernelStat), ctypes.c_int32]
        L.fmgsr_profile_collect.restype = ctypes.c_int32
        L.fmgsr_version.argtypes = []
        L.fmgsr_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def make_options(nu=(2, 1), sr_levels=1, tau="split", workspace=None):
    o = Options()
    lib().fmgsr_default_options(ctypes.byref(o))
    o.nu1, o.nu2 = int(nu[0]), int(nu[1])
    o.sr_levels = int(sr_levels)
    o.tau_mode = TAU_MODES[tau]
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    return o


def workspace_bytes(n, levels, nu=(2, 1), sr_levels=1, tau="split"):
    o = make_options(nu, sr_levels, tau)
    return int(lib().fmgsr_workspace_bytes(int(n), int(levels), ctypes.byref(o)))


def alloc_workspace(n, levels, device, **kw):
    nbytes = workspace_bytes(n, levels, **kw)
    if nbytes == 0:
        raise FmgsrError(FMGSR_EINVAL, "fmgsr_workspace_bytes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def solve(f, g=(0.0, 0.0), levels=None, segments=1, buffer=0, nu=(2, 1), sr_levels=1,
          tau="split", out=None, workspace=None, stream=None):
    """One FMG-FAS-SR iteration for -u'' = f on [0,1] (see include/fmgsr.h).

    f: contiguous float64 tensor on the GPU.  Returns u (same shape).  The
    call is asynchronous on ``stream`` (default: torch's current stream).
    """
    if not (isinstance(f, torch.Tensor) and f.is_cuda and f.dtype == torch.float64
            and f.is_contiguous() and f.dim() == 1):
        raise ValueError("f must be a contiguous 1-D float64 tensor on the GPU")
    n = f.numel()
    if levels is None:
        levels = n.bit_length()  # n a power of two -> N0 = 1
    if out is None:
        out = torch.empty_like(f)
    elif not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
              and out.numel() == n):
        raise ValueError("out must be a contiguous float64 GPU tensor of f's size")
    if stream is None:
        stream = torch.cuda.current_stream(f.device)
    o = make_options(nu, sr_levels, tau, workspace)
    op = Operator(0, None)
    st = lib().fmgsr_solve(ctypes.byref(op), f.data_ptr(), float(g[0]), float(g[1]), n,
                           int(levels), int(segments), int(buffer), ctypes.byref(o),
                           out.data_ptr(), ctypes.c_void_p(stream.cuda_stream))
    if st != FMGSR_OK:
        raise FmgsrError(st, "fmgsr_solve")
    return out


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
