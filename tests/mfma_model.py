"""CPU models of the matrix-instruction sweep (test infrastructure).

1. The window decomposition.  A band of 8 sequences p0..p0+7 applies, at
   wavefront step t, the rotations (t-q, p0+q) for q = 0..7 (Section 1.1).
   Window w holds steps 8w..8w+7; they touch the 16 columns 8w-7..8w+8, so
   the window is one 16 x 16 orthogonal matrix Q(band, w) applied to those
   columns (the accumulate-then-multiply idea of Section 8).  After window
   w, columns 8w-7..8w ("block w") are final for the band and columns
   8w+1..8w+8 stay in flight.  Window -1 is the identity: it only moves the
   band's first input block into flight.  `window_q` builds Q with plain
   rotations; `band_model` applies the windows to a matrix; their result
   must match the oracle up to rounding.

2. The schedule.  In wave-local super-step sp, band i runs window
   sp-1-2i, on band i-1's block finished one super-step earlier.
   `schedule_events` lists, for one workgroup of W waves of
   NB bands each, the super-step at which every (wave, band, window) runs,
   every ring slot is written and read, and every block is published to
   the next workgroup, with the same formulas as the kernel; the tests
   check that every input is produced strictly earlier and never
   overwritten before it is read.
"""
import math

import numpy as np

KB = 8   # sequences per band and steps per window
KW = 16  # window width


def nwin_of(n):
    """Windows per band: the steps 0..n+6 of a band in windows of 8."""
    return (n + KB - 1 + KB - 1) // KB


def window_q(C, S, n, k, band, w):
    """Q(band, w): the 16 x 16 product of the window's rotations, as the
    right factor of the 16 window columns (column u <-> 8w-7+u)."""
    Q = np.eye(KW)
    if w < 0:
        return Q
    for tau in range(KB):
        t = KB * w + tau
        for q in range(KB):
            j, p = t - q, KB * band + q
            if not (0 <= j <= n - 2 and p < k):
                continue
            c, s = C[j, p], S[j, p]
            u = j - (KB * w - (KB - 1))
            x, y = Q[:, u].copy(), Q[:, u + 1].copy()
            Q[:, u] = c * x + s * y
            Q[:, u + 1] = -s * x + c * y
    return Q


def block_cols(v):
    """Columns of block v (the finished columns of window v)."""
    return np.arange(KB * v - (KB - 1), KB * v + 1)


def band_model(X, C, S, band):
    """One band applied window by window: X (m x n) -> result (new array)."""
    m, n = X.shape
    k = C.shape[1]
    nw = nwin_of(n)

    def get(cols):
        out = np.zeros((m, len(cols)))
        ok = (cols >= 0) & (cols < n)
        out[:, ok] = X[:, cols[ok]]
        return out

    Y = np.zeros_like(X)
    inflight = np.zeros((m, KB))
    for w in range(-1, nw):
        Xw = np.concatenate([inflight, get(block_cols(w + 1))], axis=1)
        Z = Xw @ window_q(C, S, n, k, band, w)
        if w >= 0:
            cols = block_cols(w)
            ok = (cols >= 0) & (cols < n)
            Y[:, cols[ok]] = Z[:, :KB][:, ok]
        inflight = Z[:, KB:]
    return Y


def sweep_model(A, C, S):
    """All bands in order: A * G(0,0) ... G(n-2,k-1) through the windows."""
    X = np.array(A, dtype=np.float64)
    k = C.shape[1]
    for band in range(math.ceil(k / KB)):
        X = band_model(X, C, S, band)
    return X


def qsw_layout(Q):
    """The 64 x 4 matrix-operand layout of Q^T read by the kernel: lane l,
    slab s holds Q[4s + l//16, l%16]."""
    out = np.zeros((64, 4))
    for lane in range(64):
        for s in range(4):
            out[lane, s] = Q[4 * s + lane // 16, lane % 16]
    return out


# ------------------------------------------------------------------ schedule


def wave_stride(nb_wave):
    """Super-steps between the starts of neighbouring waves: 2 nb_wave
    rounded up to the unroll of 4 (the last band finishes block v at
    wave-local super-step v + 2 nb_wave - 1)."""
    return 4 * ((2 * nb_wave + 3) // 4)


PUB_LAG = 1      # super-steps between storing a block and publishing it
FLAG_MARGIN = 3  # super-steps between publishing and a poll sure to see it


def seg_delay(waves, nb_wave):
    """Extra super-steps of each later segment (a multiple of 4): its first
    wave loads block v+3 at its super-step v on the strength of the flag
    poll it issued one super-step earlier; the previous segment's last wave
    stored block v+3 at off_{W-1} + 2 NB - 1 + v + 3 and published it
    PUB_LAG super-steps later, and a poll FLAG_MARGIN super-steps after that
    sees it."""
    need = wave_stride(nb_wave) * (waves - 1) + 2 * nb_wave + 3 + PUB_LAG + FLAG_MARGIN
    return 4 * ((need + 3) // 4)


def schedule_events(waves, nb_wave, nwin, seg=0):
    """Events of one workgroup (segment `seg`) in absolute super-steps:
    ('mfma', wave, band, window, step), ('ring_w', wave, block, slot, step),
    ('ring_r', wave, block, slot, step), ('out', wave, block, step),
    ('in', wave, block, step)."""
    pre = 4 + seg * seg_delay(waves, nb_wave)
    stride = wave_stride(nb_wave)
    ev = []
    for j in range(waves):
        off = pre + j * stride
        for i in range(nb_wave):
            for w in range(-1, nwin):
                ev.append(("mfma", j, i, w, off + 1 + 2 * i + w))
        for v in range(0, nwin + 1):  # input blocks 0..nwin
            if j == 0:
                ev.append(("in", j, v, off + v))
            else:
                ev.append(("ring_r", j, v, v % 4, off + v))
        for w in range(0, nwin + 1):  # output blocks 0..nwin of the last band
            if j == waves - 1:
                ev.append(("out", j, w, off + 2 * nb_wave - 1 + w))
            else:
                ev.append(("ring_w", j, w, w % 4, off + 2 * nb_wave - 1 + w))
    return ev


def total_steps(waves, nb_wave, nwin, seg=0):
    """Super-steps a workgroup runs (a multiple of 4, barriers included)."""
    pre = 4 + seg * seg_delay(waves, nb_wave)
    t = pre + (waves - 1) * wave_stride(nb_wave) + 2 * nb_wave - 1 + nwin + 1
    return 4 * ((t + 3) // 4)
