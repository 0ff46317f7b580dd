"""CPU models of the matrix-instruction sweep (test infrastructure).

1. The window decomposition.  A band of 8 sequences p0..p0+7 applies, at
   wavefront step t, the rotations (t-q, p0+q) for q = 0..7 (Section 1.1).
   Window w holds steps 8w+7..8w+14; they touch the 16 columns
   8w..8w+15, so the window is one 16 x 16 orthogonal matrix Q(band, w)
   applied to those columns (the accumulate-then-multiply idea of Section
   8).  After window w, columns 8w..8w+7 ("block w") are final for the band
   and columns 8w+8..8w+15 stay in flight; window w's new columns are block
   w+1.  Window -1 (steps -1..6) starts the band on block 0.  Blocks never
   straddle column 0, so a block's columns are a fixed offset from its
   first column.  `window_q` builds Q with plain rotations; `band_model`
   applies the windows to a matrix; their result must match the oracle up
   to rounding.

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
    """Windows 0..nwin-1 per band (after window -1): block nwin-1 holds
    column n-1, and window nwin-1 ends at step 8 nwin + 6 >= n + 5, the
    band's last step."""
    return (n + KB - 1) // KB


def window_q(C, S, n, k, band, w):
    """Q(band, w): the 16 x 16 product of the window's rotations, as the
    right factor of the 16 window columns (column u <-> 8w-7+u)."""
    Q = np.eye(KW)
    for tau in range(KB):
        t = KB * w + KB - 1 + tau
        for q in range(KB):
            j, p = t - q, KB * band + q
            if not (0 <= j <= n - 2 and p < k):
                continue
            c, s = C[j, p], S[j, p]
            u = j - KB * w
            x, y = Q[:, u].copy(), Q[:, u + 1].copy()
            Q[:, u] = c * x + s * y
            Q[:, u + 1] = -s * x + c * y
    return Q


def block_cols(v):
    """Columns of block v (the finished columns of window v)."""
    return np.arange(KB * v, KB * v + KB)


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

WAVES = 4        # waves per workgroup
POLL_LAG = 4     # super-steps between a flag poll and the use of its value
PUB_WAIT = 2     # super-steps between storing a block and the wait covering it
FLAG_MARGIN = 2  # super-steps between publishing and a poll sure to see it


def wave_stride(nb_wave):
    """Super-steps between the starts of neighbouring waves: 2 nb_wave
    rounded up to the unroll of 4 (the last band finishes block v at
    wave-local super-step v + 2 nb_wave - 1)."""
    return 4 * ((2 * nb_wave + 3) // 4)


def pub_offset(nb_wave):
    """Block v of the last wave is finished at its super-step v + 2NB - 1,
    stored to A by all waves one super-step later, covered by every wave's
    wait PUB_WAIT super-steps after that, and published in the next."""
    return 2 * nb_wave + PUB_WAIT + 1


def seg_delay(nb_wave):
    """Extra super-steps of each later segment (a multiple of 4): its waves
    load block v at super-step v-3 (relative to the segment's start) on the
    strength of a flag poll issued POLL_LAG super-steps earlier, which must
    come FLAG_MARGIN super-steps after the previous segment published v."""
    need = wave_stride(nb_wave) * (WAVES - 1) + pub_offset(nb_wave) + 3 + POLL_LAG + FLAG_MARGIN
    return 4 * ((need + 3) // 4)


def total_steps(nb_wave, nwin, seg=0):
    """Super-steps a workgroup runs (a multiple of 4): up to the stores of
    block nwin-1 of its last wave."""
    pre = 4 + seg * seg_delay(nb_wave)
    t = pre + (WAVES - 1) * wave_stride(nb_wave) + 2 * nb_wave + nwin
    return 4 * ((t + 3) // 4)


def schedule_events(nb_wave, nwin, seg=0, active=WAVES):
    """Events of one workgroup (segment `seg`, `active` waves with bands) in
    absolute super-steps:
      ('mfma', wave, band, window, t)     band runs window
      ('ring_w', wave, block, slot, t)    last band's block into the ring
      ('ring_r', wave, block, slot, t)    first band reads the previous ring
      ('load', block, t)                  all waves load parts of a block
      ('stage_w', block, slot, t)         ... and write them to the stage
      ('stage_r', block, slot, t)         first wave's first band reads it
      ('store', block, slot, t)           all waves store parts of the last
                                          active wave's block
      ('publish', block, t)               flag = block + 1"""
    pre = 4 + seg * seg_delay(nb_wave)
    stride = wave_stride(nb_wave)
    off = [pre + j * stride for j in range(WAVES)]
    out = active - 1
    ev = []
    for j in range(WAVES):
        for i in range(nb_wave):
            for w in range(-1, nwin):
                ev.append(("mfma", j, i, w, off[j] + 1 + 2 * i + w))
        for v in range(0, nwin + 1):
            ev.append(("ring_w", j, v, v % 4, off[j] + v + 2 * nb_wave - 1))
            if j > 0:
                ev.append(("ring_r", j, v, v % 4, off[j] + v))
    for v in range(0, nwin + 1):
        ev.append(("load", v, pre + v - 3))
        ev.append(("stage_w", v, v % 4, pre + v - 1))
        ev.append(("stage_r", v, v % 4, pre + v))
    for v in range(0, nwin):
        ev.append(("store", v, v % 4, off[out] + v + 2 * nb_wave))
        ev.append(("publish", v, off[out] + v + pub_offset(nb_wave)))
    return ev
