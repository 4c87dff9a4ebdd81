"""The C-ABI library loads on the CPU, exports every symbol the header
declares, and rejects invalid host arguments before touching a device."""
import ctypes
import subprocess

import numpy as np
import pytest

from paper_1309_0100_amd import fredec as F


@pytest.fixture(scope="module")
def lib():
    return F.load()


def test_exports_every_declared_symbol(lib):
    names = F.header_functions()
    assert len(names) >= 10
    out = subprocess.run(["nm", "-D", "--defined-only", F.LIB_PATH], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(lib, n)


def test_strerror_and_version(lib):
    assert lib.fredec_version() >= 100
    for code in range(0, -9, -1):
        assert lib.fredec_strerror(code)
    assert b"unknown" in lib.fredec_strerror(-99)


def _p(a):
    return a.ctypes.data


def _scan_ws(lib, soff, boff, Fs, prec=0):
    soff = np.asarray(soff, np.int64)
    boff = np.asarray(boff, np.int64)
    Fs = np.asarray(Fs, np.int64)
    n = ctypes.c_size_t()
    rc = lib.fredec_scan_workspace(soff.size - 1, _p(soff), _p(boff), _p(Fs), prec, ctypes.byref(n))
    return rc, n.value


def test_scan_workspace_validation(lib):
    rc, n = _scan_ws(lib, [0, 100], [0, 2], [1000])
    assert rc == F.OK and n > 0
    assert _scan_ws(lib, [0, 100, 150], [0, 2, 2], [1000, 10])[0] == F.OK
    assert _scan_ws(lib, [0, 10], [0, 2], [1000])[0] == F.EDOF          # N - 3m - 4 = 0
    assert _scan_ws(lib, [0, 100], [0, 25], [1000])[0] == F.ENOTSUP     # m > FREDEC_MAX_BASE
    assert _scan_ws(lib, [0, 100], [0, 0], [0])[0] == F.EINVAL          # F <= 0
    assert _scan_ws(lib, [0, 0], [0, 0], [10])[0] == F.EINVAL           # N <= 0
    assert _scan_ws(lib, [0, 100], [0, 0], [10], prec=7)[0] == F.EINVAL
    # the workspace grows with F (tiles), N (records) and m (columns)
    assert _scan_ws(lib, [0, 100], [0, 0], [10 ** 6])[1] > _scan_ws(lib, [0, 100], [0, 0], [10])[1]
    assert _scan_ws(lib, [0, 1000], [0, 3], [10])[1] > _scan_ws(lib, [0, 1000], [0, 0], [10])[1]


def test_scan_rejects_host_errors_without_device(lib):
    N, Fg = 100, 500
    soff = np.array([0, N], np.int64)
    boff = np.array([0, 1], np.int64)
    base = np.array([0.1])
    df = np.array([1e-3])
    Fs = np.array([Fg], np.int64)
    rc, need = _scan_ws(lib, soff, boff, Fs)
    dummy = ctypes.c_void_p(16)   # never dereferenced: every call below fails a host check

    def call(ctx=None, soff=soff, boff=boff, base=base, df=df, Fs=Fs, prec=0, ws=dummy, wsb=need, z=dummy):
        return lib.fredec_scan(ctx, None, soff.size - 1, dummy, dummy, dummy, _p(soff),
                               _p(base) if base is not None else None, _p(boff), _p(df), _p(Fs), prec,
                               ws, wsb, z, None, None, None)

    assert call() == F.EINVAL                                   # valid arguments, null context
    assert call(wsb=need - 1) == F.ENOMEM
    assert call(ws=None) == F.ENOMEM
    assert call(z=None) == F.EINVAL
    assert call(base=None) == F.EINVAL
    assert call(df=np.array([np.nan])) == F.EINVAL
    assert call(df=np.array([0.0])) == F.EINVAL
    assert call(base=np.array([np.inf])) == F.EINVAL
    assert call(soff=np.array([0, 6], np.int64)) == F.EDOF
    assert call(prec=3) == F.EINVAL


def test_scan_at_and_normalize_validation(lib):
    d = ctypes.c_void_p(16)
    n = ctypes.c_size_t()
    assert lib.fredec_scan_at_workspace(100, 2, ctypes.byref(n)) == F.OK and n.value > 0
    assert lib.fredec_scan_at_workspace(100, 30, ctypes.byref(n)) == F.ENOTSUP
    assert lib.fredec_scan_at(None, None, d, d, d, 100, None, 0, 1e-3, d, 10, d, n.value, d, None) == F.EINVAL
    assert lib.fredec_scan_at(None, None, d, d, d, 6, None, 1, 1e-3, d, 10, d, n.value, d, None) == F.EINVAL
    base = np.array([0.1])
    assert lib.fredec_scan_at(None, None, d, d, d, 6, _p(base), 1, 1e-3, d, 10, d, n.value, d, None) == F.EDOF
    assert lib.fredec_scan_at(None, None, d, d, d, 100, _p(base), 1, 0.0, d, 10, d, n.value, d, None) == F.EINVAL
    assert lib.fredec_scan_at(None, None, d, d, d, 100, _p(base), 1, 1e-3, d, 1 << 31, d, n.value, d, None) == F.EINVAL
    assert lib.fredec_normalize_workspace(0, ctypes.byref(n)) == F.EINVAL
    soff = np.array([0, 0], np.int64)
    assert lib.fredec_normalize(None, None, 1, _p(soff), d, d, d, d, 1 << 20, d, d, d, None, None) == F.EINVAL


def test_create_without_gpu_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.fredec_create(ctypes.byref(h), 0) == F.EDEVICE


def test_zcrit_host_entry_point_matches_oracle(lib):
    import oracle as O
    zc = F.zcrit(1234.5, 8, 0.05)
    for d in range(1, 9):
        assert abs(zc[d] - O.zcrit(d, 1234.5, 0.05)) <= 1e-12 * zc[d]
    A = np.linspace(0.5, 2.0, 9)
    zc2 = F.zcrit(50.0, 8, 0.1, A)
    for d in range(1, 9):
        assert abs(zc2[d] - O.zcrit(d, 50.0, 0.1, A[d])) <= 1e-12 * zc2[d]
    with pytest.raises(F.FredecError):
        F.zcrit(-1.0, 3, 0.05)
    with pytest.raises(F.FredecError):
        F.zcrit(10.0, 3, 1.5)


def test_selection_entry_points_validate_host_arguments(lib):
    d = ctypes.c_void_p(16)
    n = ctypes.c_size_t()
    assert lib.fredec_cascade_workspace(30, ctypes.byref(n)) == F.ENOTSUP
    assert lib.fredec_cascade_workspace(10, ctypes.byref(n)) == F.OK and n.value >= 1024
    zc = np.zeros(11)
    assert lib.fredec_cascade(None, None, d, 10, 100, _p(zc), d, n.value, d, d, None) == F.EINVAL
    assert lib.fredec_cascade(None, None, d, 10, 100, _p(zc), d, 10, d, d, None) == F.ENOMEM
    zc[3] = np.nan
    assert lib.fredec_cascade(None, None, d, 10, 100, _p(zc), d, n.value, d, d, None) == F.EINVAL
    assert lib.fredec_phase1_workspace(100, 1000, 5, 0, ctypes.byref(n)) == F.OK
    out = np.zeros(16)
    i32 = [ctypes.c_int32() for _ in range(4)]
    W = ctypes.c_double()
    args = lambda fap0, fap1: (None, None, d, d, d, 100, 1e-3, 1000, fap0, fap1, 1.0, 0, 5, 0, d, n.value, _p(out),
                               _p(out), ctypes.byref(i32[0]), _p(out), ctypes.byref(i32[1]), ctypes.byref(i32[2]),
                               ctypes.byref(i32[3]), ctypes.byref(W))
    assert lib.fredec_phase1(*args(0.2, 0.1)) == F.EINVAL        # FAP_1 >= FAP_0 violated
    assert lib.fredec_phase1(*args(0.05, 0.1)) == F.EINVAL       # valid, null context
    masks = np.array([1, 3], np.uint64)
    assert lib.fredec_tuples_workspace(100, 2, _p(masks), 2, 0, ctypes.byref(n)) == F.OK
    assert lib.fredec_tuples_workspace(100, 30, None, 3, 0, ctypes.byref(n)) == F.ENOTSUP
    assert lib.fredec_tuples_workspace(100, 3, None, 5, 0, ctypes.byref(n)) == F.EINVAL   # need 2^3 - 1
    assert lib.fredec_tuples_workspace(10, 3, None, 7, 0, ctypes.byref(n)) == F.EDOF
    toff = np.array([0, 2, 2], np.int64)
    assert lib.fredec_grad_workspace(100, _p(toff), 2, ctypes.byref(n)) == F.EINVAL       # empty tuple


def test_plan_entry_points_validate_host_arguments(lib):
    """The prepared-call entry points run the same host checks as the plain
    calls, return no plan on failure, and refuse a missing context or plan."""
    N, Fg = 100, 500
    soff = np.array([0, N], np.int64)
    boff = np.array([0, 1], np.int64)
    base = np.array([0.1])
    df = np.array([1e-3])
    Fs = np.array([Fg], np.int64)
    rc, need = _scan_ws(lib, soff, boff, Fs)
    d = ctypes.c_void_p(16)   # never dereferenced: every call below fails a host check
    plan = ctypes.c_void_p(12345)

    def scan_plan(soff=soff, base=base, df=df, prec=0, wsb=need, out=True):
        plan.value = 12345
        return lib.fredec_scan_plan(None, None, soff.size - 1, _p(soff), _p(base) if base is not None else None,
                                    _p(boff), _p(df), _p(Fs), prec, d, wsb, ctypes.byref(plan) if out else None)

    assert scan_plan() == F.EINVAL and plan.value is None       # valid arguments, null context
    assert scan_plan(wsb=need - 1) == F.ENOMEM and plan.value is None
    assert scan_plan(base=None) == F.EINVAL
    assert scan_plan(df=np.array([np.inf])) == F.EINVAL
    assert scan_plan(soff=np.array([0, 6], np.int64)) == F.EDOF
    assert scan_plan(prec=2) == F.EINVAL
    assert scan_plan(out=False) == F.EINVAL
    assert lib.fredec_plan_scan(None, None, None, d, d, d, d, None, None, None) == F.EINVAL

    pool = np.array([0.1, 0.2, 0.3])
    n = ctypes.c_size_t()
    assert lib.fredec_tuples_workspace(200, 3, None, 7, 2, ctypes.byref(n)) == F.OK
    assert lib.fredec_tuples_plan(None, None, 200, _p(pool), 3, None, 7, 2, 0, d, n.value,
                                  ctypes.byref(plan)) == F.EINVAL and plan.value is None
    assert lib.fredec_tuples_plan(None, None, 200, _p(pool), 3, None, 7, 2, 0, d, n.value - 1,
                                  ctypes.byref(plan)) == F.ENOMEM
    assert lib.fredec_tuples_plan(None, None, 200, _p(pool), 3, None, 6, 2, 0, d, n.value,
                                  ctypes.byref(plan)) == F.EINVAL           # n_tuples != 2^n - 1 without masks
    assert lib.fredec_tuples_plan(None, None, 9, _p(pool), 3, None, 7, 2, 0, d, 1 << 30,
                                  ctypes.byref(plan)) == F.EDOF
    assert lib.fredec_plan_tuples(None, None, None, d, d, d, None, None, None, None, None) == F.EINVAL

    toff = np.array([0, 2, 3], np.int64)
    assert lib.fredec_grad_workspace(200, _p(toff), 2, ctypes.byref(n)) == F.OK
    assert lib.fredec_ascent_plan(None, None, 200, _p(toff), 2, 20, 0.1, 0, d, n.value,
                                  ctypes.byref(plan)) == F.EINVAL and plan.value is None
    assert lib.fredec_ascent_plan(None, None, 200, _p(toff), 2, 20, 0.0, 0, d, n.value,
                                  ctypes.byref(plan)) == F.EINVAL           # clamp must be > 0
    assert lib.fredec_ascent_plan(None, None, 200, _p(toff), 2, 20, 0.1, 0, d, n.value - 1,
                                  ctypes.byref(plan)) == F.ENOMEM
    bad = np.array([0, 2, 2], np.int64)
    assert lib.fredec_ascent_plan(None, None, 200, _p(bad), 2, 20, 0.1, 0, d, n.value,
                                  ctypes.byref(plan)) == F.EINVAL           # empty tuple
    assert lib.fredec_plan_ascent(None, None, None, d, d, d, d, None, None, None) == F.EINVAL
    lib.fredec_plan_destroy(None)


def test_scan_static_rejects_host_errors_without_device(lib):
    """fredec_scan_static checks its host arguments and the static scratch
    limit before it needs a context or a device."""
    dummy = ctypes.c_void_p(16)   # never dereferenced: every call below fails a host check
    base = np.array([0.1] * 25)

    def call(N=100, m=1, df=1e-3, Fg=500, prec=0, z=dummy):
        return lib.fredec_scan_static(None, None, dummy, dummy, dummy, N, _p(base) if m else None, m, df, Fg, prec,
                                      z, None, None, None)

    assert call() == F.EINVAL                     # valid arguments, null context
    assert call(z=None) == F.EINVAL
    assert call(N=0) == F.EINVAL
    assert call(Fg=0) == F.EINVAL
    assert call(prec=5) == F.EINVAL
    assert call(df=0.0) == F.EINVAL
    assert call(N=10, m=2) == F.EDOF              # N - 3m - 4 = 0
    assert call(m=25) == F.ENOTSUP                # m > FREDEC_MAX_BASE
    # float32 re-scoring lists for F = 4e6 exceed FREDEC_STATIC_SCRATCH_BYTES
    assert call(N=10_000, m=12, Fg=4_000_000, prec=1) == F.ENOTSUP
    # the same scan in float64 fits
    assert call(N=10_000, m=12, Fg=4_000_000, prec=0) == F.EINVAL
    assert _scan_ws(lib, [0, 10_000], [0, 12], [4_000_000], prec=1)[1] > F.STATIC_SCRATCH_BYTES
    assert _scan_ws(lib, [0, 10_000], [0, 12], [4_000_000], prec=0)[1] <= F.STATIC_SCRATCH_BYTES
