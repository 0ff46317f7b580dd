"""Helpers shared by the GPU parity tests (marshalling and error measures)."""
import sys

import numpy as np

import oracle
import paper_2412_01852_amd as rs


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(view, dtype):
    import torch
    return rs.device_colmajor(view, "cuda", {"f64": torch.float64, "f32": torch.float32}[dtype])


def padding_bits(t):
    """Bit patterns of the padding rows of a device column-major tensor's buffer."""
    import torch
    ld = t.stride(1) if t.shape[1] > 1 else t.shape[0]
    full = torch.as_strided(t, (ld, t.shape[1]), (1, ld)) if t.numel() else t
    pad = full[t.shape[0]:, :].detach().cpu().contiguous()
    return pad.view(torch.int64 if t.dtype == torch.float64 else torch.int32).numpy().copy()


def widened(view, dtype):
    """Host float64 copy of what the device sees for `view` in `dtype`."""
    a = np.asarray(view)
    return a.astype(np.float32).astype(np.float64) if dtype == "f32" else a.astype(np.float64)


def oracle_rows(A, C, S, rows, dtype):
    """Oracle result for a subset of rows (rows are independent)."""
    sub = oracle.colmajor(widened(A, dtype)[rows])
    oracle.rotseq(sub, oracle.colmajor(widened(C, dtype)), oracle.colmajor(widened(S, dtype)))
    return np.asarray(sub)


def relerr(got, ref, a0):
    den = np.linalg.norm(a0)
    return float(np.linalg.norm(got - ref) / (den if den else 1.0))


TOL = {"f64": 1e-13, "f32": 5e-6}
