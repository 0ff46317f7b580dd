"""CPU model of the GPU sweep's schedule and coefficient preparation.

It replays, with numpy over the rows of a tile, exactly the order in which
the multipass kernel applies rotations: bands of K sequences, wavefront step
t applying rotations (t - q, p0 + q) for q = 0..K-1, a register ring of
K + 1 + D columns, identity padding of the startup/shutdown triangles and
virtual zero columns.  With the Algorithm 1 formula it must reproduce the
oracle bitwise (the reordering only respects dependencies).  It also models
the lifting form's sign bookkeeping (prep_negmask / prep_parity / prep_coef
/ prep_sign) so that logic is checked on the CPU.
"""
import numpy as np

PREFETCH = 4


def plan(n, k, band=0):
    if band == 0:
        band = 1
        while band < 16 and band < k:
            band *= 2
    unroll = band + 1 + PREFETCH
    npass = -(-k // band)
    steps = -(-(n + band - 1) // unroll) * unroll
    return band, npass, steps, unroll


def pair_rotation(kind, cv, sv):
    """(c, s, flip): the rotation part of a pair and whether it then negates
    its right column.  kind "rotate": (C, S) = (c, s).  "reflect": (C, S) =
    (tau, nu) of H = I - tau v v^T, v = (1, nu), which for an orthogonal H is
    the rotation (1 - tau, -tau nu) followed by negating the right column
    (nothing for tau = 0).  "reflect_rev": the same reflector on the
    column-reversed matrix, the rotation (tau - 1, -tau nu) then the flip
    (still the identity for tau = 0)."""
    if kind == "rotate":
        return cv, sv, False
    flip = cv != 0.0
    c = 1.0 - cv
    if kind == "reflect_rev" and flip:  # tau = 0 is the identity either way
        c = -c
    return c, -(cv * sv), flip


def prep(C, S, band, npass, steps, arith, kind="rotate"):
    """Coefficient records coef[pass, t, q] = (a, b) and final column signs.

    negL/negR[pass, j] bit q: pair (j, pass*band + q) negates its left/right
    column (both for a rotation with c < 0; a reflector's flip toggles the
    right one)."""
    n1, k = C.shape
    n = n1 + 1
    negL = np.zeros((npass, n1), dtype=np.int64)
    negR = np.zeros((npass, n1), dtype=np.int64)
    for pss in range(npass):
        for q in range(band):
            p = pss * band + q
            if p >= k:
                continue
            for j in range(n1):
                c, _, flip = pair_rotation(kind, C[j, p], S[j, p])
                neg = 1 if c < 0 else 0
                negL[pss, j] |= neg << q
                negR[pss, j] |= (neg ^ int(flip)) << q
    pc = lambda v: bin(int(v)).count("1") & 1  # noqa: E731
    parL = np.zeros((npass + 1, n1), dtype=np.int64)
    parR = np.zeros((npass + 1, n1), dtype=np.int64)
    for pss in range(npass):
        for j in range(n1):
            parL[pss + 1, j] = parL[pss, j] ^ pc(negL[pss, j])
            parR[pss + 1, j] = parR[pss, j] ^ pc(negR[pss, j])
    sign = np.ones(n)
    for c in range(n):
        f = (int(parR[npass, c - 1]) if c > 0 else 0) ^ (int(parL[npass, c]) if c + 1 < n else 0)
        sign[c] = -1.0 if f else 1.0
    coef = np.zeros((npass, steps, band, 2))
    low = lambda q: (1 << q) - 1  # noqa: E731
    for pss in range(npass):
        for t in range(steps):
            for q in range(band):
                j, p = t - q, pss * band + q
                if 0 <= j < n1 and p < k:
                    c, s, _ = pair_rotation(kind, C[j, p], S[j, p])
                    if arith == "lift":
                        # sign(j) before (j, p): (j-1, p' <= p) as right column,
                        # (j, p' < p) as left column; sign(j+1): (j, p' < p) as
                        # right column, (j+1, p' < p) as left column.
                        sj = int(parL[pss, j]) ^ pc(negL[pss, j] & low(q))
                        if j > 0:
                            sj ^= int(parR[pss, j - 1]) ^ pc(negR[pss, j - 1] & low(q + 1))
                        sj1 = int(parR[pss, j]) ^ pc(negR[pss, j] & low(q))
                        if j + 1 < n1:
                            sj1 ^= int(parL[pss, j + 1]) ^ pc(negL[pss, j + 1] & low(q))
                        tau = sj ^ sj1
                        sd = -s if tau else s
                        if not (c < 0):
                            a, b = sd / (1.0 + c), -sd
                        else:
                            a, b = -sd / (1.0 - c), sd
                        coef[pss, t, q] = (a, b)
                    else:
                        coef[pss, t, q] = (c, s)
                else:
                    coef[pss, t, q] = (0.0, 0.0) if arith == "lift" else (1.0, 0.0)
    return coef, sign


def rotate(x, y, a, b, arith):
    if arith == "exact":
        return a * x + b * y, -b * x + a * y
    # lifting form, unfused in this model
    x = x + a * y
    y = y + b * x
    x = x + a * y
    return x, y


def sweep(A, C, S, band=0, arith="exact", kind="rotate"):
    """Apply the rotations (or, with kind "reflect"/"reflect_rev", the
    reflectors (C, S) = (tau, nu)) to the (m, n) float64 array A in kernel
    order."""
    m, n = A.shape
    k = C.shape[1]
    if m == 0 or n <= 1 or k == 0:
        return A
    K, npass, steps, R = plan(n, k, band)
    coef, sign = prep(C, S, K, npass, steps, arith, kind)
    D = PREFETCH
    col = lambda c: A[:, c].copy() if 0 <= c < n else np.zeros(m)  # noqa: E731
    for pss in range(npass):
        ring = [np.zeros(m) for _ in range(R)]
        for c in range(D + 1):
            ring[c % R] = col(c)
        for t in range(steps):
            ring[(t + D + 1) % R] = col(t + D + 1)
            for q in range(K):
                xi, yi = (t - q) % R, (t - q + 1) % R
                a, b = coef[pss, t, q]
                ring[xi], ring[yi] = rotate(ring[xi], ring[yi], a, b, arith)
            c = t - K + 1
            v = ring[c % R]
            if arith == "lift" and pss == npass - 1 and 0 <= c < n:
                v = v * sign[c]
            if 0 <= c < n:
                A[:, c] = v
    return A
