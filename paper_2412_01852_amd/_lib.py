"""ctypes binding of librotseq's C ABI (argument marshalling only).

Matrices are torch tensors on the HIP device in column-major layout: a
logical m x n matrix is a 2-D tensor of shape (m, n) with strides (1, ld),
ld >= m (``device_colmajor`` makes one).  Every computation runs in the HIP
kernels of librotseq.so; there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librotseq.so")

ARITH_AUTO, ARITH_EXACT, ARITH_FMA, ARITH_LIFT = 0, 1, 2, 3
KERNEL_AUTO, KERNEL_MULTIPASS, KERNEL_CHAIN, KERNEL_MFMA = 0, 1, 2, 3

_lib = None


class RotseqError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        msg = f"librotseq error {code}: {strerror(code)}"
        super().__init__(f"{what}: {msg}" if what else msg)


class Options(ctypes.Structure):
    _fields_ = [("arith", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("band", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("publish", ctypes.c_int32), ("inverse", ctypes.c_int32),
                ("left", ctypes.c_int32), ("shape", ctypes.c_int32)]


class Profile(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_int64), ("prep_ms", ctypes.c_double),
                ("sweep_ms", ctypes.c_double), ("sweep_ms_min", ctypes.c_double),
                ("sweep_ms_max", ctypes.c_double)]


class Problem(ctypes.Structure):
    """rotseq_problem_d / rotseq_problem_s (same layout: pointers are void*)."""
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64),
                ("S", ctypes.c_void_p), ("lds", ctypes.c_int64)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("band", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("workgroups", ctypes.c_int64),
                ("waves_total", ctypes.c_int64), ("flops", ctypes.c_double),
                ("bytes", ctypes.c_double), ("device_bytes", ctypes.c_size_t)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_batch", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 5)]


class SweepInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("submit_us", ctypes.c_double), ("start_us", ctypes.c_double),
                ("end_us", ctypes.c_double)]


class LaunchInfo(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("band", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("workgroups", ctypes.c_int32), ("bands_per_wave", ctypes.c_int32),
                ("rows_per_wave", ctypes.c_int32), ("segments", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("workspace_bytes", ctypes.c_uint64)]


def launch_describe(dtype, m, n, k, lda=None, opts=None):
    """rotseq_launch_describe: the launch a call of this shape would make on
    the current device (dict of rotseq_launch_info)."""
    ch = {"float64": b"d", "double": b"d", "d": b"d", "float32": b"s", "float": b"s", "s": b"s"}[
        str(dtype).replace("torch.", "")]
    out = LaunchInfo()
    rc = _load().rotseq_launch_describe(ch, m, n, k, lda if lda is not None else max(1, m), _opts(opts),
                                        ctypes.byref(out))
    if rc != 0:
        raise RotseqError(rc, "launch_describe")
    return {f: getattr(out, f) for f, _ in LaunchInfo._fields_ if f != "reserved"}


class CeilingResult(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("valu_flops", ctypes.c_double),
                ("mfma_flops", ctypes.c_double), ("clock_mhz", ctypes.c_double)]


def fp64_ceiling(mode, waves=16, iters=1 << 16):
    """rotseq_fp64_ceiling: FP64 issue rates of the device (mode 1 vector FMA,
    2 vector FMA with a DPP-broadcast operand, 3 matrix FMA, 4 both at once);
    returns a dict with ms, valu_flops, mfma_flops, clock_mhz."""
    out = CeilingResult()
    rc = _load().rotseq_fp64_ceiling(int(mode), int(waves), int(iters), ctypes.byref(out))
    if rc != 0:
        raise RotseqError(rc, "fp64_ceiling")
    return {f: getattr(out, f) for f, _ in CeilingResult._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [("sweeps_done", ctypes.c_int64), ("sweeps_failed", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("matrices_resident", ctypes.c_int64),
                ("matrices_pending", ctypes.c_int64), ("resident_bytes", ctypes.c_uint64),
                ("peak_resident_bytes", ctypes.c_uint64), ("flops", ctypes.c_double),
                ("busy_s", ctypes.c_double), ("gflops", ctypes.c_double),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("mean_batch", ctypes.c_double)]


def profile_enable(on=True):
    _load().rotseq_profile_enable(1 if on else 0)


def profile_read(reset=False):
    """Totals of the event-timed kernels since the last reset (waits for them)."""
    out = Profile()
    rc = _load().rotseq_profile_read(ctypes.byref(out), 1 if reset else 0)
    if rc != 0:
        raise RotseqError(rc, "profile_read")
    return {f: getattr(out, f) for f, _ in Profile._fields_}


def device_status(reset=False):
    """Sticky device error bits (synchronizes the device); 0 means clean."""
    return _load().rotseq_device_status(1 if reset else 0)


STATUS_NOT_ORTHOGONAL = 1 << 16


def test_set_waits(spin_limit=0, unreachable=False):
    """rotseq_test_set_waits: bounded waits between workgroups give up after
    ``spin_limit`` polls (0 = default); with ``unreachable`` every such wait
    gives up (a test hook for the error paths)."""
    rc = _load().rotseq_test_set_waits(int(spin_limit), 1 if unreachable else 0)
    if rc != 0:
        raise RotseqError(rc, "test_set_waits")


def library_path():
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with "
                           "`python -m paper_2412_01852_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    i64, vp, i32 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
    base = [i64, i64, i64, vp, i64, vp, i64, vp, i64, vp]
    for name in ("rotseq_d", "rotseq_s", "rotseq_noalloc_d"):
        f = getattr(lib, name)
        f.restype, f.argtypes = i32, base
    for name in ("rotseq_ex_d", "rotseq_ex_s", "rotseq_refl_ex_d", "rotseq_refl_ex_s"):
        f = getattr(lib, name)
        f.restype, f.argtypes = i32, base + [ctypes.POINTER(Options), vp, ctypes.c_size_t]
    for name in ("rotseq_refl3_d", "rotseq_refl3_s"):
        f = getattr(lib, name)
        f.restype, f.argtypes = i32, [i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp, vp,
                                      ctypes.c_size_t]
    for name in ("rotseq_refl3_ex_d", "rotseq_refl3_ex_s"):
        f = getattr(lib, name)
        f.restype, f.argtypes = i32, [i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp,
                                      ctypes.POINTER(Options), vp, ctypes.c_size_t]
    lib.rotseq_refl3_workspace_bytes.restype = ctypes.c_size_t
    lib.rotseq_refl3_workspace_bytes.argtypes = [ctypes.c_char, i64, i64, i64]
    lib.rotseq_refl3_ex_workspace_bytes.restype = ctypes.c_size_t
    lib.rotseq_refl3_ex_workspace_bytes.argtypes = [ctypes.c_char, i64, i64, i64, ctypes.POINTER(Options)]
    lib.rotseq_workspace_bytes.restype = ctypes.c_size_t
    lib.rotseq_workspace_bytes.argtypes = [ctypes.c_char, i64, i64, i64, ctypes.POINTER(Options)]
    lib.rotseq_check_args.restype = i32
    lib.rotseq_check_args.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64]
    lib.rotseq_strerror.restype = ctypes.c_char_p
    lib.rotseq_strerror.argtypes = [i32]
    lib.rotseq_version.restype = i32
    lib.rotseq_version.argtypes = []
    lib.rotseq_device_status.restype = i32
    lib.rotseq_device_status.argtypes = [i32]
    lib.rotseq_launch_describe.restype = i32
    lib.rotseq_launch_describe.argtypes = [ctypes.c_char, i64, i64, i64, i64, ctypes.POINTER(Options),
                                           ctypes.POINTER(LaunchInfo)]
    lib.rotseq_fp64_ceiling.restype = i32
    lib.rotseq_fp64_ceiling.argtypes = [ctypes.c_int32, ctypes.c_int32, i64, ctypes.POINTER(CeilingResult)]
    lib.rotseq_test_set_waits.restype = i32
    lib.rotseq_test_set_waits.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.rotseq_profile_enable.restype = i32
    lib.rotseq_profile_enable.argtypes = [i32]
    lib.rotseq_profile_read.restype = i32
    lib.rotseq_profile_read.argtypes = [ctypes.POINTER(Profile), i32]
    pp = ctypes.POINTER(Problem)
    for name in ("rotseq_batched_d", "rotseq_batched_s"):
        f = getattr(lib, name)
        f.restype, f.argtypes = i32, [ctypes.c_int32, pp, vp]
    for name in ("rotseq_batch_create_d", "rotseq_batch_create_s"):
        f = getattr(lib, name)
        f.restype, f.argtypes = i32, [ctypes.c_int32, pp, ctypes.POINTER(Options),
                                      ctypes.POINTER(ctypes.c_void_p)]
    lib.rotseq_batch_execute.restype, lib.rotseq_batch_execute.argtypes = i32, [vp, vp]
    for name in ("rotseq_batch_update_d", "rotseq_batch_update_s"):
        f = getattr(lib, name)
        f.restype, f.argtypes = i32, [vp, ctypes.c_int32, pp]
    lib.rotseq_batch_tune.restype, lib.rotseq_batch_tune.argtypes = i32, [vp, vp, ctypes.c_int32]
    lib.rotseq_batch_status.restype = i32
    lib.rotseq_batch_status.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), i32]
    lib.rotseq_batch_info_get.restype = i32
    lib.rotseq_batch_info_get.argtypes = [vp, ctypes.POINTER(BatchInfo)]
    lib.rotseq_batch_destroy.restype, lib.rotseq_batch_destroy.argtypes = i32, [vp]
    pv = ctypes.POINTER(ctypes.c_void_p)
    lib.rotseq_server_create.restype = i32
    lib.rotseq_server_create.argtypes = [ctypes.POINTER(ServerConfig), pv]
    lib.rotseq_server_open.restype = i32
    lib.rotseq_server_open.argtypes = [vp, i64, i64, vp, i64, ctypes.POINTER(i64)]
    lib.rotseq_server_submit.restype = i32
    lib.rotseq_server_submit.argtypes = [vp, i64, i64, vp, i64, vp, i64, ctypes.POINTER(i64)]
    lib.rotseq_server_wait.restype = i32
    lib.rotseq_server_wait.argtypes = [vp, i64, i64, ctypes.POINTER(SweepInfo)]
    lib.rotseq_server_read.restype = i32
    lib.rotseq_server_read.argtypes = [vp, i64, vp, i64]
    lib.rotseq_server_close.restype, lib.rotseq_server_close.argtypes = i32, [vp, i64]
    lib.rotseq_server_stats_get.restype = i32
    lib.rotseq_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.rotseq_server_destroy.restype, lib.rotseq_server_destroy.argtypes = i32, [vp]
    _lib = lib
    return lib


def strerror(code):
    return _load().rotseq_strerror(int(code)).decode()


def version():
    return _load().rotseq_version()


def check_args(m, n, k, A, lda, C, ldc, S, lds):
    """Host-only argument check (pointers are ints or None)."""
    return _load().rotseq_check_args(m, n, k, A, lda, C, ldc, S, lds)


def _opts(opts):
    if opts is None:
        return None
    if isinstance(opts, Options):
        return ctypes.byref(opts)
    o = Options()
    for key, val in dict(opts).items():
        setattr(o, key, int(val))
    return ctypes.byref(o)


def workspace_bytes(dtype, m, n, k, opts=None):
    ch = {"float64": b"d", "double": b"d", "d": b"d", "float32": b"s", "float": b"s", "s": b"s"}[
        str(dtype).replace("torch.", "")]
    return _load().rotseq_workspace_bytes(ch, m, n, k, _opts(opts))


def _ld(t, name):
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    rows, cols = t.shape
    if rows and cols and t.stride(0) != 1:
        raise ValueError(f"{name} must be column-major (stride(0) == 1)")
    if cols <= 1 or rows == 0:
        return max(1, rows)
    return t.stride(1)


def _is_left(opts):
    if opts is None:
        return False
    if isinstance(opts, Options):
        return bool(opts.left)
    return bool(dict(opts).get("left", 0))


def rotseq(A, C, S, *, opts=None, workspace=None, stream=None):
    """A <- A * G(0,0) ... G(n-2,k-1) in place on the GPU (Algorithms 1-2).

    A: (m, n) float64/float32 column-major device tensor; C, S: (n-1, k) of the
    same dtype ((m-1, k) with ``opts["left"]``, rotations mixing rows).
    ``opts`` is an Options or a dict of its fields; ``workspace`` an optional
    uint8 device tensor; ``stream`` a torch stream (default: the current
    one).  Returns A.
    """
    return _call(False, A, C, S, opts, workspace, stream)


def rotseq_noalloc(A, C, S, *, stream=None):
    """rotseq_noalloc_d: as rotseq for float64 tensors, with the workspace in
    the library's fixed device array (nothing is allocated).  Returns A."""
    import torch
    if A.dtype != torch.float64 or C.dtype != A.dtype or S.dtype != A.dtype:
        raise TypeError("rotseq_noalloc takes float64 A, C and S")
    m, n = A.shape
    k = C.shape[1]
    if C.shape != S.shape or C.shape[0] != max(n - 1, 0):
        raise ValueError(f"coefficient arrays must be ({max(n - 1, 0)}, k); got {tuple(C.shape)}, {tuple(S.shape)}")
    for t, nm in ((A, "A"), (C, "C"), (S, "S")):
        if t.numel() and not t.is_cuda:
            raise ValueError(f"{nm} must be a device tensor")
    st = stream if stream is not None else torch.cuda.current_stream(A.device)
    ptr = lambda t: t.data_ptr() if t.numel() else None  # noqa: E731
    rc = _load().rotseq_noalloc_d(m, n, k, ptr(A), _ld(A, "A"), ptr(C), _ld(C, "C"), ptr(S),
                                  _ld(S, "S"), ctypes.c_void_p(st.cuda_stream))
    if rc != 0:
        raise RotseqError(rc, "rotseq_noalloc")
    return A


def reflseq(A, TAU, NU, *, opts=None, workspace=None, stream=None):
    """A <- A * H(0,0) ... H(n-2,k-1) for 2x2 reflectors H = I - tau v v^T,
    v = e_j + nu e_{j+1} (rotseq_refl_ex_*); arguments as for rotseq with
    TAU, NU in place of C, S."""
    return _call(True, A, TAU, NU, opts, workspace, stream)


def refl3seq(A, TAU, NU1, NU2, *, opts=None, workspace=None, stream=None):
    """A <- A * H(0,0) ... H(n-3,k-1) for 3x3 reflectors H = I - tau v v^T,
    v = e_j + nu1 e_{j+1} + nu2 e_{j+2} (rotseq_refl3_*).  A: (m, n)
    float64/float32 column-major device tensor; TAU, NU1, NU2: (n-2, k) of
    the same dtype ((m-2, k) with ``opts["left"]``).  ``opts`` may ask for
    ``inverse`` and ``left`` (rotseq_refl3_ex_*).  Returns A."""
    import torch
    if A.dtype not in (torch.float64, torch.float32):
        raise TypeError("A must be float64 or float32")
    if any(t.dtype != A.dtype for t in (TAU, NU1, NU2)):
        raise TypeError("A and the coefficient arrays must share a dtype")
    m, n = A.shape
    k = TAU.shape[1]
    r = m if _is_left(opts) else n
    if TAU.shape != NU1.shape or TAU.shape != NU2.shape or TAU.shape[0] != max(r - 2, 0):
        raise ValueError(f"coefficient arrays must be ({max(r - 2, 0)}, k); got "
                         f"{tuple(TAU.shape)}, {tuple(NU1.shape)}, {tuple(NU2.shape)}")
    for t, nm in ((A, "A"), (TAU, "TAU"), (NU1, "NU1"), (NU2, "NU2")):
        if t.numel() and not t.is_cuda:
            raise ValueError(f"{nm} must be a device tensor")
    st = stream if stream is not None else torch.cuda.current_stream(A.device)
    ptr = lambda t: t.data_ptr() if t.numel() else None  # noqa: E731
    lib = _load()
    wptr = workspace.data_ptr() if workspace is not None else None
    wbytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    args = (m, n, k, ptr(A), _ld(A, "A"), ptr(TAU), _ld(TAU, "TAU"), ptr(NU1), _ld(NU1, "NU1"),
            ptr(NU2), _ld(NU2, "NU2"), ctypes.c_void_p(st.cuda_stream))
    if opts is None:
        fn = lib.rotseq_refl3_d if A.dtype == torch.float64 else lib.rotseq_refl3_s
        rc = fn(*args, wptr, wbytes)
    else:
        fn = lib.rotseq_refl3_ex_d if A.dtype == torch.float64 else lib.rotseq_refl3_ex_s
        rc = fn(*args, _opts(opts), wptr, wbytes)
    if rc != 0:
        raise RotseqError(rc, "refl3seq")
    return A


def refl3_workspace_bytes(dtype, m, n, k, opts=None):
    ch = {"float64": b"d", "double": b"d", "d": b"d", "float32": b"s", "float": b"s", "s": b"s"}[
        str(dtype).replace("torch.", "")]
    if opts is None:
        return _load().rotseq_refl3_workspace_bytes(ch, m, n, k)
    return _load().rotseq_refl3_ex_workspace_bytes(ch, m, n, k, _opts(opts))


def _call(refl, A, C, S, opts, workspace, stream):
    import torch
    if A.dtype not in (torch.float64, torch.float32):
        raise TypeError("A must be float64 or float32")
    if C.dtype != A.dtype or S.dtype != A.dtype:
        raise TypeError("A and the coefficient arrays must share a dtype")
    m, n = A.shape
    k = C.shape[1]
    r = m if _is_left(opts) else n
    if C.shape != S.shape or C.shape[0] != max(r - 1, 0):
        raise ValueError(f"coefficient arrays must be ({max(r - 1, 0)}, k); got {tuple(C.shape)}, {tuple(S.shape)}")
    for t, nm in ((A, "A"), (C, "C"), (S, "S")):
        if t.numel() and not t.is_cuda:
            raise ValueError(f"{nm} must be a device tensor")
    lda, ldc, lds = _ld(A, "A"), _ld(C, "C"), _ld(S, "S")
    st = stream if stream is not None else torch.cuda.current_stream(A.device)
    handle = ctypes.c_void_p(st.cuda_stream)
    ptr = lambda t: t.data_ptr() if t.numel() else None  # noqa: E731
    lib = _load()
    dbl = A.dtype == torch.float64
    if opts is None and workspace is None and not refl:
        fn = lib.rotseq_d if dbl else lib.rotseq_s
        rc = fn(m, n, k, ptr(A), lda, ptr(C), ldc, ptr(S), lds, handle)
    else:
        if refl:
            fn = lib.rotseq_refl_ex_d if dbl else lib.rotseq_refl_ex_s
        else:
            fn = lib.rotseq_ex_d if dbl else lib.rotseq_ex_s
        wptr = workspace.data_ptr() if workspace is not None else None
        wbytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
        rc = fn(m, n, k, ptr(A), lda, ptr(C), ldc, ptr(S), lds, handle, _opts(opts), wptr, wbytes)
    if rc != 0:
        raise RotseqError(rc, "reflseq" if refl else "rotseq")
    return A


def device_colmajor(view, device="cuda", dtype=None):
    """Copy a column-major numpy view (with its padded buffer) to the device.

    Returns an (m, n) tensor with strides (1, ld) over a device buffer holding
    the whole ld x n host buffer, padding included.
    """
    import numpy as np
    import torch
    buf = view.base if view.base is not None else view
    buf = np.asfortranarray(buf)
    ld, cols = buf.shape
    t = torch.from_numpy(np.ascontiguousarray(buf.T))  # (cols, ld), row j = column j
    if dtype is not None:
        t = t.to(dtype)
    t = t.to(device)
    return t.t()[: view.shape[0], : view.shape[1]]


def host_colmajor(t):
    """Device column-major (m, n) tensor -> numpy float64 (m, n) array."""
    return t.detach().to("cpu", dtype=__import__("torch").float64).numpy()


def _problems(items):
    """(A, C, S) device tensor triples -> (ctypes Problem array, is_double)."""
    import torch
    arr = (Problem * max(len(items), 1))()
    dbl = None
    for i, (A, C, S) in enumerate(items):
        if A.dtype not in (torch.float64, torch.float32) or C.dtype != A.dtype or S.dtype != A.dtype:
            raise TypeError(f"problem {i}: A, C, S must share a float64/float32 dtype")
        if dbl is None:
            dbl = A.dtype == torch.float64
        elif dbl != (A.dtype == torch.float64):
            raise TypeError("all problems of a batch must share a dtype")
        m, n = A.shape
        ptr = lambda t: t.data_ptr() if t.numel() else None  # noqa: E731
        arr[i] = Problem(m, n, C.shape[1], ptr(A), _ld(A, "A"), ptr(C), _ld(C, "C"),
                         ptr(S), _ld(S, "S"))
    return arr, bool(dbl) if dbl is not None else True


def _stream(stream, device=None):
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(st.cuda_stream)


def batched(items, stream=None):
    """One-shot batch: A_i <- A_i * prod G for every (A_i, C_i, S_i); blocks."""
    arr, dbl = _problems(items)
    lib = _load()
    fn = lib.rotseq_batched_d if dbl else lib.rotseq_batched_s
    rc = fn(len(items), arr, _stream(stream))
    if rc != 0:
        raise RotseqError(rc, "batched")


class Batch:
    """A batch plan (rotseq_batch_*): create once, execute many times.

    ``execute`` only launches kernels (no allocation, no synchronization), so
    it can be captured into a CUDA/HIP graph.  The tensors must stay alive
    while the plan exists.
    """

    def __init__(self, items, opts=None):
        arr, dbl = _problems(items)
        self._keep = list(items)
        self._handle = ctypes.c_void_p()
        lib = _load()
        fn = lib.rotseq_batch_create_d if dbl else lib.rotseq_batch_create_s
        rc = fn(len(items), arr, _opts(opts), ctypes.byref(self._handle))
        if rc != 0:
            raise RotseqError(rc, "batch_create")

    def execute(self, stream=None):
        rc = _load().rotseq_batch_execute(self._handle, _stream(stream))
        if rc != 0:
            raise RotseqError(rc, "batch_execute")

    def update(self, items):
        """Point the plan at other tensors of the same shapes, in the same
        order (rotseq_batch_update_*); synchronizes the device."""
        arr, dbl = _problems(items)
        lib = _load()
        fn = lib.rotseq_batch_update_d if dbl else lib.rotseq_batch_update_s
        rc = fn(self._handle, len(items), arr)
        if rc != 0:
            raise RotseqError(rc, "batch_update")
        self._keep = list(items)

    def tune(self, reps=3, stream=None):
        rc = _load().rotseq_batch_tune(self._handle, _stream(stream), int(reps))
        if rc != 0:
            raise RotseqError(rc, "batch_tune")

    def status(self, reset=False):
        """(return code, per-entry ROTSEQ_E_* codes in creation order) of
        rotseq_batch_status; synchronizes the device."""
        words = (ctypes.c_int32 * max(len(self._keep), 1))()
        rc = _load().rotseq_batch_status(self._handle, words, 1 if reset else 0)
        if rc not in (0, 5):
            raise RotseqError(rc, "batch_status")
        return rc, [int(words[i]) for i in range(len(self._keep))]

    def info(self):
        out = BatchInfo()
        rc = _load().rotseq_batch_info_get(self._handle, ctypes.byref(out))
        if rc != 0:
            raise RotseqError(rc, "batch_info")
        return {f: getattr(out, f) for f, _ in BatchInfo._fields_ if f != "reserved"}

    def close(self):
        if self._handle:
            _load().rotseq_batch_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _host_f64(a, name):
    """A host float64 column-major array (a copy if needed) and its ld."""
    import numpy as np
    a = np.asarray(a)
    if a.ndim != 2:
        raise ValueError(f"{name} must be 2-D")
    if a.dtype != np.float64 or not (a.flags.f_contiguous or a.shape[1] <= 1):
        a = np.asfortranarray(a, dtype=np.float64)
    ld = a.strides[1] // 8 if a.shape[1] > 1 else max(1, a.shape[0])
    return a, max(1, ld)


class Server:
    """rotseq_server_*: resident FP64 matrices, sweeps batched by a worker."""

    def __init__(self, budget_bytes=0, max_batch=0):
        cfg = ServerConfig(int(budget_bytes), int(max_batch))
        self._h = ctypes.c_void_p()
        rc = _load().rotseq_server_create(ctypes.byref(cfg), ctypes.byref(self._h))
        if rc != 0:
            raise RotseqError(rc, "server_create")

    def open(self, A):
        a, ld = _host_f64(A, "A")
        mid = ctypes.c_int64()
        rc = _load().rotseq_server_open(self._h, a.shape[0], a.shape[1], a.ctypes.data if a.size else None,
                                        ld, ctypes.byref(mid))
        if rc != 0:
            raise RotseqError(rc, "server_open")
        return mid.value

    def submit(self, mid, C, S):
        c, ldc = _host_f64(C, "C")
        s_, lds = _host_f64(S, "S")
        t = ctypes.c_int64()
        rc = _load().rotseq_server_submit(self._h, mid, c.shape[1], c.ctypes.data if c.size else None,
                                          ldc, s_.ctypes.data if s_.size else None, lds,
                                          ctypes.byref(t))
        if rc != 0:
            raise RotseqError(rc, "server_submit")
        return t.value

    def wait(self, ticket, timeout_us=-1):
        """Returns (status, info dict)."""
        info = SweepInfo()
        rc = _load().rotseq_server_wait(self._h, ticket, int(timeout_us), ctypes.byref(info))
        return rc, {f: getattr(info, f) for f, _ in SweepInfo._fields_ if f != "reserved"}

    def read(self, mid, m, n):
        import numpy as np
        out = np.zeros((m, n), dtype=np.float64, order="F")
        rc = _load().rotseq_server_read(self._h, mid, out.ctypes.data if out.size else None, max(1, m))
        if rc != 0:
            raise RotseqError(rc, "server_read")
        return out

    def close(self, mid):
        rc = _load().rotseq_server_close(self._h, mid)
        if rc != 0:
            raise RotseqError(rc, "server_close")

    def stats(self):
        st = ServerStats()
        rc = _load().rotseq_server_stats_get(self._h, ctypes.byref(st))
        if rc != 0:
            raise RotseqError(rc, "server_stats")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def destroy(self):
        if self._h:
            rc = _load().rotseq_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            if rc != 0:
                raise RotseqError(rc, "server_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()
