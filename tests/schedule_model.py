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


def prep(C, S, band, npass, steps, arith):
    """Coefficient records coef[pass, t, q] = (a, b) and final column signs."""
    n1, k = C.shape
    n = n1 + 1
    neg = np.zeros((npass, n1), dtype=np.uint64)
    for pss in range(npass):
        for q in range(band):
            p = pss * band + q
            if p < k:
                neg[pss] |= (C[:, p] < 0).astype(np.uint64) << np.uint64(q)
    par = np.zeros((npass + 1, n1), dtype=np.uint8)
    acc = np.zeros(n1, dtype=np.uint8)
    popc = np.vectorize(lambda v: bin(int(v)).count("1") & 1, otypes=[np.uint8])
    for pss in range(npass):
        par[pss] = acc
        acc = acc ^ popc(neg[pss]) if n1 else acc
    par[npass] = acc
    tot = par[npass]
    sign = np.ones(n)
    for c in range(n):
        f = (int(tot[c - 1]) if c > 0 else 0) ^ (int(tot[c]) if c + 1 < n else 0)
        sign[c] = -1.0 if f else 1.0
    coef = np.zeros((npass, steps, band, 2))
    low = lambda q: (1 << q) - 1  # noqa: E731
    for pss in range(npass):
        for t in range(steps):
            for q in range(band):
                j, p = t - q, pss * band + q
                if 0 <= j < n1 and p < k:
                    c, s = C[j, p], S[j, p]
                    if arith == "lift":
                        tau = 0
                        if j > 0:
                            tau ^= int(par[pss, j - 1]) ^ (bin(int(neg[pss, j - 1]) & low(q + 1)).count("1") & 1)
                        if j + 1 < n1:
                            tau ^= int(par[pss, j + 1]) ^ (bin(int(neg[pss, j + 1]) & low(q)).count("1") & 1)
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


def sweep(A, C, S, band=0, arith="exact"):
    """Apply the rotations to the (m, n) float64 array A in kernel order."""
    m, n = A.shape
    k = C.shape[1]
    if m == 0 or n <= 1 or k == 0:
        return A
    K, npass, steps, R = plan(n, k, band)
    coef, sign = prep(C, S, K, npass, steps, arith)
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
