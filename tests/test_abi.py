"""C-ABI library: loads, exports every declared symbol, validates arguments.
CPU only: nothing here launches a kernel."""
import ctypes
import os
import re

import pytest

import paper_2412_01852_amd as rs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    inc = os.path.join(ROOT, "include")
    for fn in sorted(os.listdir(inc)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(inc, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        text = re.sub(r"#[^\n]*", "", text)
        for m in re.finditer(r"\b([a-z_][a-z0-9_]*)\s*\(", text):
            name = m.group(1)
            prefix = text[max(0, m.start() - 80): m.start()]
            if name.startswith("rotseq_") and not re.search(r"typedef[^;]*$", prefix):
                names.append(name)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(rs.library_path())
    names = declared_functions()
    assert "rotseq_d" in names and "rotseq_s" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


def test_version_and_strerror():
    assert rs.version() >= 100
    assert rs.strerror(0) == "success"
    assert "invalid argument" in rs.strerror(-4)
    for code in range(1, 6):
        assert rs.strerror(code) != "unknown error code"


@pytest.mark.parametrize("args,expect", [
    ((4, 5, 6, 1, 4, 1, 4, 1, 4), 0),
    ((-1, 5, 6, 1, 4, 1, 4, 1, 4), -1),
    ((4, -5, 6, 1, 4, 1, 4, 1, 4), -2),
    ((4, 5, -6, 1, 4, 1, 4, 1, 4), -3),
    ((4, 5, 6, None, 4, 1, 4, 1, 4), -4),
    ((4, 5, 6, 1, 3, 1, 4, 1, 4), -5),
    ((4, 5, 6, 1, 4, None, 4, 1, 4), -6),
    ((4, 5, 6, 1, 4, 1, 3, 1, 4), -7),
    ((4, 5, 6, 1, 4, 1, 4, None, 4), -8),
    ((4, 5, 6, 1, 4, 1, 4, 1, 3), -9),
    # quick-return shapes accept NULL pointers but still check leading dims
    ((0, 5, 6, None, 1, None, 4, None, 4), 0),
    ((4, 1, 6, None, 4, None, 1, None, 1), 0),
    ((4, 5, 0, None, 4, None, 4, None, 4), 0),
    ((0, 0, 0, None, 0, None, 0, None, 0), -5),
    ((0, 0, 0, None, 1, None, 1, None, 0), -9),
    ((3, 1, 2, None, 3, None, 0, None, 1), -7),
])
def test_check_args(args, expect):
    assert rs.check_args(*args) == expect


def test_workspace_bytes():
    assert rs.workspace_bytes("float64", 0, 5, 6) == 0
    assert rs.workspace_bytes("float64", 5, 1, 6) == 0
    assert rs.workspace_bytes("float64", 5, 5, 0) == 0
    a = rs.workspace_bytes("float64", 64, 100, 16)
    b = rs.workspace_bytes("float32", 64, 100, 16)
    assert a > b > 0
    assert a % 256 == 0
    # bands of 16: 12 passes over (n + 15 padded to 21) steps of 16 pairs
    big = rs.workspace_bytes("float64", 10240, 10240, 192)
    assert big >= 12 * 10255 * 16 * 16
    assert rs.workspace_bytes("float64", 64, 100, 16, {"band": 3}) == 0
    assert rs.workspace_bytes("float64", 64, 100, 16, {"arith": 9}) == 0


def _problem(m, n, k, A, lda=None, ldc=None, lds=None, C=0x2000000, S=0x3000000):
    n1 = max(1, n - 1)
    return rs.Problem(m, n, k, A, lda if lda is not None else max(1, m),
                      C, ldc if ldc is not None else n1, S, lds if lds is not None else n1)


def _create(probs, count=None):
    lib = rs._lib._load()
    arr = (rs.Problem * max(1, len(probs)))(*probs)
    h = ctypes.c_void_p()
    n = len(probs) if count is None else count
    return lib.rotseq_batch_create_d(n, arr if probs else None, None, ctypes.byref(h))


@pytest.mark.parametrize("opts", [{"inverse": 1}, {"left": 1}, {"kernel": 1}, {"band": 5},
                                  {"arith": 9}])
def test_batch_refuses_unsupported_options(opts):
    """Batches support the forward right application with the chain kernel
    only; the refusal comes before any device call."""
    lib = rs._lib._load()
    base = 0x10000000
    probs = [_problem(8, 10, 4, base + i * 0x100000) for i in range(3)]
    arr = (rs.Problem * 3)(*probs)
    h = ctypes.c_void_p()
    assert lib.rotseq_batch_create_d(3, arr, rs._lib._opts(opts), ctypes.byref(h)) == 4


def test_batch_rejects_bad_count_and_null_array():
    assert _create([], count=-1) == -1
    assert _create([], count=3) == -2


@pytest.mark.parametrize("field,value,argpos", [
    ("m", -1, 1), ("n", -2, 2), ("k", -1, 3), ("A", None, 4), ("lda", 3, 5),
    ("C", None, 6), ("ldc", 5, 7), ("S", None, 8), ("lds", 2, 9)])
def test_batch_names_entry_and_argument(field, value, argpos):
    """Entry 2 (0-based) invalid -> -(1000*3 + argpos); nothing is launched."""
    base = 0x10000000
    probs = [_problem(8, 10, 4, base + i * 0x100000) for i in range(4)]
    p = probs[2]
    setattr(p, field, value)
    probs[2] = p
    assert _create(probs) == -(1000 * 3 + argpos)


def test_batch_detects_overlapping_matrices():
    base = 0x10000000
    probs = [_problem(8, 10, 4, base), _problem(8, 10, 4, base + 0x100000),
             _problem(8, 10, 4, base + 8 * 8 * 9)]  # starts inside entry 0's last column
    assert _create(probs) == -(1000 * 3 + 4)


def test_batch_null_handles_are_rejected():
    lib = rs._lib._load()
    assert lib.rotseq_batch_update_d(None, 0, None) == -1
    assert lib.rotseq_batch_update_s(None, 0, None) == -1
    assert lib.rotseq_batch_execute(None, None) == -1
    assert lib.rotseq_batch_tune(None, None, 3) == -1
    assert lib.rotseq_batch_info_get(None, None) == -1
    assert lib.rotseq_batch_status(None, None, 0) == -1
    assert lib.rotseq_batch_destroy(None) == 0


def test_wait_hook_argument_check_and_reset():
    """rotseq_test_set_waits refuses a negative limit and restores the
    defaults with (0, 0); host-only (it sets values later launches read)."""
    lib = rs._lib._load()
    assert lib.rotseq_test_set_waits(-1, 0) == -1
    assert lib.rotseq_test_set_waits(1, 1) == 0
    assert lib.rotseq_test_set_waits(0, 0) == 0


def test_server_argument_checks_without_device():
    lib = rs._lib._load()
    assert lib.rotseq_server_create(None, None) == -2
    cfg = rs.ServerConfig(0, -1)
    h = ctypes.c_void_p()
    assert lib.rotseq_server_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
    mid = ctypes.c_int64()
    assert lib.rotseq_server_open(None, 4, 4, None, 4, ctypes.byref(mid)) == -1
    assert lib.rotseq_server_submit(None, 1, 4, None, 3, None, 3, ctypes.byref(mid)) == -1
    assert lib.rotseq_server_wait(None, 1, 0, None) == -1
    assert lib.rotseq_server_read(None, 1, None, 1) == -1
    assert lib.rotseq_server_close(None, 1) == -1
    assert lib.rotseq_server_stats_get(None, None) == -1
    assert lib.rotseq_server_destroy(None) == 0


def test_new_error_codes_have_descriptions():
    for code in range(6, 10):
        assert rs.strerror(code) != rs.strerror(999)


def test_options_struct_layout():
    """rotseq_opts is eight int32 fields: arith, kernel, band, waves, publish,
    inverse, left, shape."""
    assert ctypes.sizeof(rs.Options) == 32
    assert rs.Options.inverse.offset == 20
    assert rs.Options.left.offset == 24


def _ex(fn, m, n, k, A, lda, C, ldc, S, lds, opts=None):
    lib = rs._lib._load()
    o = rs._lib._opts(opts)
    return getattr(lib, fn)(m, n, k, A, lda, C, ldc, S, lds, None, o, None, 0)


@pytest.mark.parametrize("fn", ["rotseq_ex_d", "rotseq_refl_ex_d", "rotseq_refl_ex_s"])
def test_left_argument_checks_without_device(fn):
    """With left application C/S (or TAU/NU) have m-1 rows and the work
    condition is n > 0, m > 1; all checked before any device call."""
    L = {"left": 1}
    assert _ex(fn, 6, 3, 2, 1, 6, 1, 2, 1, 5, L) == -7   # ldc = n-1 is too small for left
    assert _ex(fn, 6, 3, 2, 1, 6, 1, 5, 1, 4, L) == -9
    assert _ex(fn, 6, 3, 2, 1, 5, 1, 5, 1, 5, L) == -5   # lda >= m still
    assert _ex(fn, 6, 3, 2, None, 6, 1, 5, 1, 5, L) == -4
    assert _ex(fn, 6, 0, 2, None, 6, None, 5, None, 5, L) == 0  # n == 0: quick return
    assert _ex(fn, 1, 7, 2, None, 1, None, 1, None, 1, L) == 0  # m == 1: quick return
    # the same shape without `left` checks C against n-1
    assert _ex(fn, 6, 3, 2, 1, 6, 1, 1, 1, 2) == -7


def test_reflectors_arithmetic():
    """Reflectors run in the lifting form, or with ROTSEQ_ARITH_EXACT as written
    (forward order only); the FMA form, and the inverse order or chain options
    with the exact form, are refused before anything touches the device."""
    assert _ex("rotseq_refl_ex_d", 64, 10, 3, 1, 64, 1, 9, 1, 9, {"arith": rs.ARITH_FMA}) == 4
    for extra in ({"inverse": 1}, {"band": 4}, {"waves": 2}, {"kernel": rs.KERNEL_CHAIN}):
        assert _ex("rotseq_refl_ex_d", 64, 10, 3, 1, 64, 1, 9, 1, 9,
                   dict(extra, arith=rs.ARITH_EXACT)) == 4


def test_left_workspace_adds_packed_copy():
    """Left application sweeps the transposed n x m copy packed into the
    workspace after the plan's own buffers."""
    m, n, k = 300, 70, 16
    left = rs.workspace_bytes("float64", m, n, k, {"left": 1})
    right_t = rs.workspace_bytes("float64", n, m, k)
    assert left >= right_t + m * n * 8
    assert left - (right_t + m * n * 8) < 256
    assert rs.workspace_bytes("float64", 1, 70, 16, {"left": 1}) == 0
    assert rs.workspace_bytes("float64", 300, 0, 16, {"left": 1}) == 0
    assert rs.workspace_bytes("float64", 300, 1, 16, {"left": 1}) > 0


def _r3(fn, m, n, k, A, lda, T, ldt, N1, ld1, N2, ld2, ws=None, wsb=0):
    lib = ctypes.CDLL(rs.library_path())
    f = getattr(lib, fn)
    f.restype = ctypes.c_int
    i64, vp = ctypes.c_int64, ctypes.c_void_p
    f.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp, vp, ctypes.c_size_t]
    return f(m, n, k, A, lda, T, ldt, N1, ld1, N2, ld2, None, ws, wsb)


@pytest.mark.parametrize("fn", ["rotseq_refl3_d", "rotseq_refl3_s"])
def test_refl3_argument_checks_without_device(fn):
    """Arguments are checked in order (-i for argument i) before anything
    touches the device; TAU/NU1/NU2 need n-2 rows; quick returns accept NULL."""
    ok = (6, 10, 3, 1, 6, 1, 8, 1, 8, 1, 8)
    for pos, bad in [(0, -1), (1, -1), (2, -1), (3, None), (4, 5), (5, None), (6, 7), (7, None),
                     (8, 7), (9, None), (10, 7)]:
        args = list(ok)
        args[pos] = bad
        assert _r3(fn, *args) == -(pos + 1), (pos, bad)
    assert _r3(fn, 0, 10, 3, None, 1, None, 8, None, 8, None, 8) == 0
    assert _r3(fn, 6, 2, 3, None, 6, None, 1, None, 1, None, 1) == 0
    assert _r3(fn, 6, 10, 0, None, 6, None, 8, None, 8, None, 8) == 0
    # a caller workspace that is too small or misaligned is refused before any launch
    assert _r3(fn, *ok, ws=256, wsb=16) == 3
    assert _r3(fn, *ok, ws=0x1001, wsb=1 << 30) == 3


def test_refl3_workspace_bytes():
    """Records of (nu1, nu2, -tau, -tau nu1, -tau nu2) for bands of 8 (FP64)
    or 4 (FP32) sequences over the padded wavefront steps; zero for
    quick-return shapes and unknown dtypes."""
    lib = ctypes.CDLL(rs.library_path())
    f = lib.rotseq_refl3_workspace_bytes
    f.restype = ctypes.c_size_t
    f.argtypes = [ctypes.c_char, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
    d = f(b"d", 10240, 10240, 192)
    assert d >= 192 * 10240 * 5 * 8 and d < 192 * (10240 + 64) * 5 * 8 + 256
    f32 = f(b"s", 10240, 10240, 192)
    assert f32 >= 192 * 10240 * 5 * 4 and f32 < 192 * (10240 + 64) * 5 * 4 + 256
    assert f(b"d", 0, 100, 8) == 0 and f(b"d", 5, 2, 8) == 0 and f(b"d", 5, 100, 0) == 0
    assert f(b"x", 5, 100, 8) == 0


def test_refl3_ex_workspace_bytes():
    """Left application adds the packed copy; other options are refused."""
    base = rs.refl3_workspace_bytes("float64", 300, 200, 24)
    assert rs.refl3_workspace_bytes("float64", 300, 200, 24, {"inverse": 1}) == base
    left = rs.refl3_workspace_bytes("float64", 300, 200, 24, {"left": 1})
    right_t = rs.refl3_workspace_bytes("float64", 200, 300, 24)
    assert left >= right_t + 300 * 200 * 8
    assert rs.refl3_workspace_bytes("float64", 2, 200, 24, {"left": 1}) == 0
    assert rs.refl3_workspace_bytes("float64", 300, 200, 24, {"band": 4}) == 0
