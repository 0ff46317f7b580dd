"""CPU oracle for applying sequences of plane rotations (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does.

Arrays follow the column-major convention of the C source: a logical
``m x n`` matrix is a numpy array of shape ``(m, n)`` whose element (i, j)
lives at ``base[i + j*ld]``, i.e. Fortran order with leading dimension ``ld``
(``arr.strides == (8, 8*ld)``).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load(path=None):
    global _lib
    if path is not None:
        lib = ctypes.CDLL(path)
    else:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
    i64, dp = ctypes.c_int64, ctypes.c_void_p
    for name in ("oracle_rotseq_d", "oracle_rotseq_inverse_d", "oracle_rotseq_left_d",
                 "oracle_rotseq_left_inverse_d", "oracle_reflseq_d", "oracle_reflseq_inverse_d",
                 "oracle_reflseq_left_d"):
        f = getattr(lib, name)
        f.restype = None
        f.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64]
    for name in ("oracle_refl3seq_d", "oracle_refl3seq_inverse_d"):
        f = getattr(lib, name)
        f.restype = None
        f.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64, dp, i64]
    f = lib.oracle_refl3seq_left_d
    f.restype = None
    f.argtypes = [i64, i64, i64, ctypes.c_int, dp, i64, dp, i64, dp, i64, dp, i64]
    f = lib.oracle_rotseq_threads_d
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int, i64, i64, i64, dp, i64, dp, i64, dp, i64]
    if path is None:
        _lib = lib
    return lib


def _ld(arr, name):
    """Leading dimension of a column-major float64 view; validates layout."""
    if arr.dtype != np.float64:
        raise TypeError(f"{name} must be float64 (got {arr.dtype})")
    if arr.ndim != 2:
        raise ValueError(f"{name} must be 2-D")
    rows, cols = arr.shape
    if rows == 0 or cols == 0:
        return max(1, rows)
    if arr.strides[0] != 8:
        raise ValueError(f"{name} must be column-major (unit row stride)")
    if cols == 1:
        return max(1, rows)
    ld = arr.strides[1] // 8
    if ld < rows:
        raise ValueError(f"{name}: leading dimension {ld} < rows {rows}")
    return ld


def _ptr(arr):
    return arr.ctypes.data if arr.size else None


def _args(A, C, S, left):
    m, n = A.shape
    nm1, k = C.shape
    if S.shape != C.shape:
        raise ValueError("C and S must have the same shape")
    r = m if left else n  # length of the dimension the sequences mix
    if r >= 1 and nm1 != max(r - 1, 0):
        raise ValueError(f"C has {nm1} rows, expected {r - 1}")
    args = (m, n, k, _ptr(A), _ld(A, "A"), _ptr(C), _ld(C, "C"), _ptr(S), _ld(S, "S"))
    return args, (m == 0 or n == 0 or r <= 1 or k == 0)


def rotseq(A, C, S, *, lib=None, inverse=False, threads=None, left=False):
    """Apply Algorithm 2 in place to the column-major float64 view ``A``.

    ``A`` is m x n, ``C`` and ``S`` are (n-1) x k.  With ``inverse=True`` the
    inverse sequence is applied instead (reverse order, transposed rotations).
    ``threads`` > 1 splits the rows across host threads (bitwise identical).
    With ``left=True`` the rotations mix adjacent rows instead of columns
    (C and S are (m-1) x k): A <- Q^T A, or Q A with ``inverse=True``.
    Returns ``A``.
    """
    lib = lib or _load()
    args, quick = _args(A, C, S, left)
    if quick:
        return A
    if left:
        (lib.oracle_rotseq_left_inverse_d if inverse else lib.oracle_rotseq_left_d)(*args)
    elif inverse:
        lib.oracle_rotseq_inverse_d(*args)
    elif threads and threads > 1:
        if lib.oracle_rotseq_threads_d(int(threads), *args) < 0:
            raise RuntimeError("oracle thread start failed")
    else:
        lib.oracle_rotseq_d(*args)
    return A


def reflseq(A, TAU, NU, *, lib=None, inverse=False, left=False):
    """Apply a sequence of 2x2 reflectors in place to the column-major view ``A``.

    Reflector (j, p) is H = I - tau v v^T with v = e_j + nu e_{j+1},
    tau = TAU[j, p], nu = NU[j, p]; per pair w = x + nu*y, x -= tau*w,
    y -= (tau*nu)*w.  Right application (columns j, j+1; TAU and NU are
    (n-1) x k) in the order of Algorithm 2, or with ``inverse=True`` the same
    reflectors in reverse order; ``left=True`` mixes rows j, j+1 instead
    (TAU and NU are (m-1) x k).  Returns ``A``.
    """
    lib = lib or _load()
    if inverse and left:
        raise ValueError("the oracle has no left inverse reflector sequence")
    args, quick = _args(A, TAU, NU, left)
    if quick:
        return A
    if left:
        lib.oracle_reflseq_left_d(*args)
    elif inverse:
        lib.oracle_reflseq_inverse_d(*args)
    else:
        lib.oracle_reflseq_d(*args)
    return A


def refl3seq(A, TAU, NU1, NU2, *, inverse=False, left=False, lib=None):
    """Apply a sequence of 3x3 reflectors in place: reflector (j, p) is
    I - tau v v^T with v = e_j + nu1 e_{j+1} + nu2 e_{j+2} acting on
    columns j..j+2 (rows with ``left``); TAU, NU1, NU2 are (n-2) x k
    ((m-2) x k with ``left``).  Forward: A H(0,0) ... H(n-3,k-1);
    ``inverse``: A H(n-3,k-1) ... H(0,0); ``left``: H(m-3,k-1) ... H(0,0) A,
    and with ``inverse`` H(0,0) ... H(m-3,k-1) A.  Returns ``A``."""
    lib = lib or _load()
    m, n = A.shape
    nm2, k = TAU.shape
    r = m if left else n
    if NU1.shape != TAU.shape or NU2.shape != TAU.shape:
        raise ValueError("TAU, NU1 and NU2 must have the same shape")
    if r >= 2 and nm2 != max(r - 2, 0):
        raise ValueError(f"TAU has {nm2} rows, expected {r - 2}")
    if (n == 0 if left else m == 0) or r <= 2 or k == 0:
        return A
    args = (_ptr(A), _ld(A, "A"), _ptr(TAU), _ld(TAU, "TAU"),
            _ptr(NU1), _ld(NU1, "NU1"), _ptr(NU2), _ld(NU2, "NU2"))
    if left:
        lib.oracle_refl3seq_left_d(m, n, k, 1 if inverse else 0, *args)
    elif inverse:
        lib.oracle_refl3seq_inverse_d(m, n, k, *args)
    else:
        lib.oracle_refl3seq_d(m, n, k, *args)
    return A


def colmajor(arr, ld=None, fill=np.nan):
    """Copy a 2-D array into a fresh column-major float64 buffer.

    With ``ld`` > rows the padding rows of the buffer are set to ``fill`` so a
    test can check that nothing outside the logical matrix is touched.
    Returns the logical (rows x cols) view; ``view.base`` holds the buffer.
    """
    arr = np.asarray(arr, dtype=np.float64)
    rows, cols = arr.shape
    ld = max(1, rows) if ld is None else ld
    buf = np.full((ld, max(cols, 1)), fill, dtype=np.float64, order="F")
    buf[:rows, :cols] = arr
    return buf[:rows, :cols]
