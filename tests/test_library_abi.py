"""CPU-side checks of the HIP library: it loads, exports every function
include/fmgsr.h declares, and validates arguments on the host (before any
GPU work is enqueued)."""
import ctypes
import os
import re

import pytest

from paper_1207_6720_amd import fmgsr as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fmgsr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fmgsr_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert "fmgsr_solve" in names and "fmgsr_workspace_bytes" in names
    L = ctypes.CDLL(F.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_status_strings():
    assert "gfx950" in F.version()
    for st in (0, -1, -2, -3, -4, 7):
        assert F.lib().fmgsr_status_string(st)


def _solve_raw(n, levels, segs, buf, **kw):
    o = F.make_options(**kw)
    return F.lib().fmgsr_solve(None, None, 0.0, 0.0, n, levels, segs, buf, ctypes.byref(o),
                               None, None)


@pytest.mark.parametrize("args,kw", [
    ((1000, 11, 4, 4), {}),               # n not divisible by 2^(levels-1)
    ((1024, 11, 3, 4), {}),               # segments do not divide n
    ((1024, 11, 1024, 4), {}),            # odd segment core (s = 1)
    ((1 << 20, 21, 1, 8), {}),            # segment window exceeds one workgroup
    ((1024, 0, 4, 4), {}),                # no levels
    ((1024, 41, 4, 4), {}),               # too many levels
    ((4096, 2, 4, 4), {}),                # coarsest grid of 2048 cells
    ((1024, 11, 4, -1), {}),              # negative buffer
    ((1024, 11, 4, 4), {"nu": (17, 1)}),  # too many sweeps
    ((1024, 11, 4, 4), {}),               # valid sizes, NULL device pointers
    ((1, 1, 1, 0), {"sr_levels": 1}),     # SR level needs a coarser level
    ((1024, 11, 4, 4), {"sr_levels": 11}),  # more SR levels than coarser grids
    ((1024, 11, 256, 4), {"sr_levels": 3}),  # core 4 -> 2 -> 1: odd on the third SR level
    ((1024, 11, 4, 4), {"sr_levels": 2}),  # valid multi-level SR, NULL device pointers
])
def test_invalid_arguments_rejected_on_host(args, kw):
    assert _solve_raw(*args, **kw) == F.FMGSR_EINVAL


def test_unsupported_requests():
    # per-patch literal tau exists for the finest SR level only
    assert _solve_raw(1024, 11, 4, 4, sr_levels=2, tau="literal") == F.FMGSR_ENOTSUP
    assert _solve_raw(1024, 11, 4, 4, tau="literal", precision="fp32relax") == F.FMGSR_ENOTSUP
    o = F.make_options()
    for kind, expect in ((1, F.FMGSR_EINVAL), (2, F.FMGSR_EINVAL), (7, F.FMGSR_EINVAL)):
        op = F.Operator(kind, None)  # reaction kinds need a device kappa
        assert F.lib().fmgsr_solve(ctypes.byref(op), None, 0.0, 0.0, 1024, 11, 4, 4,
                                   ctypes.byref(o), None, None) == expect


def _create(sizes, levels, segs=None, buffer=8, op=1, **kw):
    import numpy as np
    n = np.asarray(sizes, dtype=np.int64)
    L = np.asarray(levels, dtype=np.int32)
    s = None if segs is None else np.asarray(segs, dtype=np.int64)
    o = F.make_options(**kw)
    h = ctypes.c_void_p()
    st = F.lib().fmgsr_batch_create(len(n), n.ctypes.data, None, L.ctypes.data,
                                    None if s is None else s.ctypes.data, buffer, None, op,
                                    ctypes.byref(o), ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("sizes,levels,segs,buffer,kw", [
    ([1000], [5], None, 8, {}),             # n not divisible by 2^(levels-1)
    ([512 * 8], [4], None, 8, {}),          # coarsest grid of 512 cells (> 256)
    ([4096], [0], None, 8, {}),             # no levels
    ([4096], [13], [3], 8, {}),             # segments do not divide n
    ([4096], [13], [4096], 8, {}),          # odd segment core
    ([4096], [13], None, 65, {}),           # buffer too wide
    ([4096], [13], None, -1, {}),           # negative buffer
    ([4096], [13], None, 8, {"nu": (17, 1)}),
    ([0], [1], None, 8, {}),                # empty problem
])
def test_batch_create_rejects_invalid_problems(sizes, levels, segs, buffer, kw):
    st, h = _create(sizes, levels, segs, buffer, **kw)
    assert st == F.FMGSR_EINVAL and not h.value


def test_batch_create_unsupported_options():
    assert _create([4096], [13], tau="literal")[0] == F.FMGSR_ENOTSUP
    assert _create([4096], [13], sr_levels=0)[0] == F.FMGSR_ENOTSUP
    assert F.lib().fmgsr_batch_solve(None, None, None, None, None) == F.FMGSR_EINVAL
    assert F.lib().fmgsr_batch_destroy(None) == F.FMGSR_EINVAL


def test_workspace_sizes():
    n = 1 << 20
    hier = (n - 1) * 8
    split = F.workspace_bytes(n, 21)
    assert split >= 3 * hier + (n // 2) * 8
    assert F.workspace_bytes(n, 21, tau="literal") >= split + hier
    assert F.workspace_bytes(n, 21, sr_levels=0) >= 3 * hier + n * 8
    assert F.workspace_bytes(1000, 11) == 0


def test_exact_workspace_for_segments():
    """With one SR level, split tau and a buffer covering both sweep cones the
    SR passes run inside the vertical kernels and the restricted fine
    iterate (n/2 doubles) is not stored, with or without functionals;
    otherwise the exact size is the bound."""
    n, L, S = 1 << 20, 21, 256
    bound = F.workspace_bytes(n, L)
    assert F.workspace_bytes(n, L, segments=S, buffer=8) == bound - (n // 2) * 8
    assert F.workspace_bytes(n, L, segments=S, buffer=3, nu=(2, 1)) == bound - (n // 2) * 8
    # the functionals are then summed per vertical tile, not in Uh
    assert F.workspace_bytes(n, L, segments=S, buffer=8, functionals=True) == bound - (n // 2) * 8
    for kw in (dict(buffer=2), dict(buffer=2, functionals=True), dict(buffer=3, nu=(2, 2))):
        assert F.workspace_bytes(n, L, segments=S, **kw) == bound, kw
    lit = F.workspace_bytes(n, L, tau="literal")
    assert F.workspace_bytes(n, L, segments=S, buffer=8, tau="literal") == lit
    assert F.workspace_bytes(n, L, segments=3, buffer=8) == 0      # invalid segments
    # plain FMG-FAS with split tau rebuilds the finest pre-smoothed iterate
    # inside its top up kernel (n doubles less) when both top kernels walk two
    # or more levels; literal tau, one-level up kernels (nu2 = 16) and a finest
    # level right above the coarse core store it
    assert (F.workspace_bytes(n, L, segments=1, buffer=0, sr_levels=0)
            == F.workspace_bytes(n, L, sr_levels=0) - n * 8)
    for kw in (dict(tau="literal"), dict(nu=(2, 16))):
        assert (F.workspace_bytes(n, L, segments=1, buffer=0, sr_levels=0, **kw)
                == F.workspace_bytes(n, L, sr_levels=0, **kw)), kw
    n2, L2 = 1 << 11, 12
    assert (F.workspace_bytes(n2, L2, segments=1, buffer=0, sr_levels=0)
            == F.workspace_bytes(n2, L2, sr_levels=0))


def test_two_sr_levels_store_neither_finest_level():
    """With two or more SR levels, level M-1 keeps no U or V array: the
    workspace shrinks by V^{M-1} (n/2 cells) and by U^{M-1} less the n/4 cells
    that hold I^ of level M-1; more SR levels store the same."""
    for n, levels in ((1 << 20, 21), (5 << 16, 17), (1 << 28, 29)):
        one = F.workspace_bytes(n, levels, sr_levels=1)
        two = F.workspace_bytes(n, levels, sr_levels=2)
        three = F.workspace_bytes(n, levels, sr_levels=3)
        saved = (n // 2 + n // 2 - n // 4) * 8
        assert abs((one - two) - saved) <= 3 * 256, (n, one - two, saved)
        assert three == two


def test_binding_rejects_host_and_float32_arrays():
    """The binding checks every tensor before any library call: the C ABI
    sees raw pointers only, so a host array or a float32 coefficient would be
    read as device FP64 data of the wrong extent."""
    import torch
    f64 = torch.zeros(64, dtype=torch.float64)
    f32 = torch.zeros(64, dtype=torch.float32)
    with pytest.raises(ValueError):
        F.solve(f64, levels=7)                              # host memory
    with pytest.raises(ValueError):
        F.solve(f32, levels=7)                              # float32
    with pytest.raises(ValueError):
        F.adjoint(f64, f64, f64, levels=7)                  # host memory
    with pytest.raises(ValueError):
        F._check_vec(torch.zeros(2, 32, dtype=torch.float64), "f")  # not 1-D
    with pytest.raises(ValueError):
        F._check_vec(torch.zeros(64, dtype=torch.float64)[::2], "f")  # not contiguous


def test_launch_lds_fits_the_grant_for_every_geometry():
    """Every kernel with dynamic LDS is granted the device's per-workgroup
    LDS (MI355X: 160 KiB) less its own static LDS (a few hundred bytes at
    most); a solve checks each request against its kernel's grant before
    enqueuing.  The coarse core's request is its level stack: iterates and
    right-hand sides of levels 0..C, the correction buffer of level C-1, 8
    N0 doubles of cyclic reduction and the sweeps' second buffer (level C);
    the segment kernels take 13 doubles per thread."""
    grant = 160 * 1024 - 1024
    # N0 = 1: core levels up to 2048 cells (C = 11)
    ntot, esz = 4095, 1024
    assert F.launch_lds_bytes(1 << 28, 29, 1 << 16, 8) == (2 * ntot + esz + 8 + 2048) * 8
    # the largest coarsest grid (N0 = 1024): the core takes levels 0 and 1
    # when a level lies above them (the finest level is never in the core)
    assert F.launch_lds_bytes(4096, 3, 1, 0, sr_levels=0) == (2 * 3072 + 1024 + 8 * 1024 + 2048) * 8
    assert F.launch_lds_bytes(2048, 2, 1, 0, sr_levels=0) == (2 * 1024 + 8 * 1024 + 1024) * 8
    # widest segment window: 1024 threads of 8 cells
    s = 8160  # + 2 x 10 pad cells: 1023 runs of 8
    assert F.launch_lds_bytes(8 * s, 9, 8, 8) == max(1024 * 13 * 8,
                                                     F.launch_lds_bytes(8 * s, 9, 1, 0, sr_levels=0))
    worst = 0
    for n0 in (1, 3, 5, 63, 64, 65, 255, 511, 1000, 1024):
        for extra in range(0, 14):
            n = n0 << extra
            for sr, segs, buf in ((0, 1, 0), (1, 1, 8), (2, 1, 8)):
                if sr > extra:
                    continue
                worst = max(worst, F.launch_lds_bytes(n, extra + 1, segs, buf, sr_levels=sr))
    assert 0 < worst <= grant
    assert F.launch_lds_bytes(1000, 11, 4, 4) == 0      # invalid sizes


def test_option_validation_on_host():
    """check_finite takes 0 or 1, the rhs restriction FULLWEIGHT or AVERAGE,
    and the average restriction needs literal tau (split tau rests on
    L_H I^ = I L_h, which only full weighting satisfies): an invalid
    combination has no workspace size and is refused before anything runs."""
    n, L = 1 << 12, 13
    assert F.lib().fmgsr_status_string(F.FMGSR_ENONFINITE).decode().startswith("FMGSR_ENONFINITE")
    o = F.make_options(check_finite=True)
    assert F.lib().fmgsr_workspace_bytes(n, L, ctypes.byref(o)) > 0
    o.check_finite = 2
    assert F.lib().fmgsr_workspace_bytes(n, L, ctypes.byref(o)) == 0
    assert F.workspace_bytes(n, L, tau="literal", rhs_restrict="avg") > 0
    assert F.workspace_bytes(n, L, tau="split", rhs_restrict="avg") == 0
    o = F.make_options()
    o.rhs_restriction = 2
    assert F.lib().fmgsr_workspace_bytes(n, L, ctypes.byref(o)) == 0
    # the kept coarse solution needs exactly one SR level
    assert F.workspace_bytes(n, L, coarse_out=True) > 0
    assert F.workspace_bytes(n, L, sr_levels=2, coarse_out=True) == 0
    assert F.workspace_bytes(n, L, sr_levels=0, coarse_out=True) == 0
    # the batched engine supports none of these options
    import numpy as np
    sizes, levels = np.array([4096], dtype=np.int64), np.array([13], dtype=np.int32)
    for kw in ({"check_finite": True}, {"tau": "literal", "rhs_restrict": "avg"}):
        o = F.make_options(**kw)
        h = ctypes.c_void_p()
        st = F.lib().fmgsr_batch_create(1, sizes.ctypes.data, None, levels.ctypes.data, None, 8,
                                        None, 1, ctypes.byref(o), ctypes.byref(h))
        assert st == F.FMGSR_ENOTSUP and not h.value
