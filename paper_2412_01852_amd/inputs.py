"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module only draws random numbers and lays them out; it contains none of
the rotation arithmetic.  The paper measures on synthetic matrices (random
square matrices with k = 180 sequences, Section "Experiments"); the shapes
below restate the workloads this library is measured on:

* A: i.i.d. standard normal entries, stored column-major (A[i + j*lda]).
* theta: i.i.d. uniform on [0, 2*pi), stored column-major as (n-1) x k,
  drawn after A from the same generator; C = cos(theta), S = sin(theta).
* FP32 inputs are round-to-nearest casts of the same FP64 draws.

Generators are numpy PCG64 seeded per problem; batches of problems use
independent streams from ``SeedSequence(seed).spawn(count)``.

Reflector sequences (the paper's 2x2 reflector variant) and rotations that
mix rows get their own generators with the same conventions.
"""
from dataclasses import dataclass
import math

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclass
class Problem:
    m: int
    n: int
    k: int
    A: np.ndarray  # (m, n) column-major view, float64
    C: np.ndarray  # (n-1, k) column-major view, float64
    S: np.ndarray  # (n-1, k) column-major view, float64

    @property
    def flops(self):
        """Counted work: 6 flops per (rotation, row), 6 m (n-1) k."""
        return 6 * self.m * max(self.n - 1, 0) * self.k


def _colmajor_buffer(rows, cols, ld, fill):
    ld = max(1, rows if ld is None else ld)
    if ld < rows:
        raise ValueError("leading dimension smaller than the row count")
    buf = np.full((ld, max(cols, 1)), fill, dtype=np.float64, order="F")
    return buf, buf[:rows, :cols]


def make_problem(m, n, k, seed=0, *, lda=None, ldc=None, lds=None,
                 pad_fill=np.nan, rng=None):
    """One problem of the given shape; padding rows of each buffer hold ``pad_fill``."""
    rng = rng if rng is not None else np.random.Generator(np.random.PCG64(seed))
    _, A = _colmajor_buffer(m, n, lda, pad_fill)
    A[...] = rng.standard_normal(m * n).reshape(n, m).T
    nm1 = max(n - 1, 0)
    theta = rng.uniform(0.0, TWO_PI, nm1 * k).reshape(k, nm1).T
    _, C = _colmajor_buffer(nm1, k, ldc, pad_fill)
    _, S = _colmajor_buffer(nm1, k, lds, pad_fill)
    C[...] = np.cos(theta)
    S[...] = np.sin(theta)
    return Problem(m, n, k, A, C, S)


def make_left_problem(m, n, k, seed=0, *, lda=None, ldc=None, lds=None, pad_fill=np.nan):
    """Problem for rotations that mix rows: A is m x n, C and S are (m-1) x k
    (same distributions as make_problem; ``Problem.C`` keeps the (m-1) rows)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    _, A = _colmajor_buffer(m, n, lda, pad_fill)
    A[...] = rng.standard_normal(m * n).reshape(n, m).T
    mm1 = max(m - 1, 0)
    theta = rng.uniform(0.0, TWO_PI, mm1 * k).reshape(k, mm1).T
    _, C = _colmajor_buffer(mm1, k, ldc, pad_fill)
    _, S = _colmajor_buffer(mm1, k, lds, pad_fill)
    C[...] = np.cos(theta)
    S[...] = np.sin(theta)
    return Problem(m, n, k, A, C, S)


def make_reflectors(r, k, rng, *, ld_tau=None, ld_nu=None, identity_frac=0.05,
                    pad_fill=np.nan):
    """(r x k) reflector parameters (tau, nu) of orthogonal 2x2 reflectors
    I - tau v v^T, v = (1, nu): nu = tan(phi) with phi uniform on
    (-pi/2, pi/2), tau = 2 / (1 + nu^2) (so every angle of the reflecting
    line is equally likely), and a fraction ``identity_frac`` of tau = 0
    (identity) entries as an annihilation of an already-zero entry gives."""
    phi = rng.uniform(-0.5 * math.pi, 0.5 * math.pi, r * k).reshape(k, r).T
    ident = rng.uniform(0.0, 1.0, r * k).reshape(k, r).T < identity_frac
    _, TAU = _colmajor_buffer(r, k, ld_tau, pad_fill)
    _, NU = _colmajor_buffer(r, k, ld_nu, pad_fill)
    NU[...] = np.tan(phi)
    TAU[...] = np.where(ident, 0.0, 2.0 / (1.0 + NU * NU))
    return TAU, NU


def make_refl_problem(m, n, k, seed=0, *, left=False, lda=None, ldc=None, lds=None,
                      pad_fill=np.nan):
    """Reflector problem: A i.i.d. normal (m x n); ``Problem.C`` holds tau and
    ``Problem.S`` holds nu, (n-1) x k, or (m-1) x k with ``left``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    _, A = _colmajor_buffer(m, n, lda, pad_fill)
    A[...] = rng.standard_normal(m * n).reshape(n, m).T
    r = max((m if left else n) - 1, 0)
    TAU, NU = make_reflectors(r, k, rng, ld_tau=ldc, ld_nu=lds, pad_fill=pad_fill)
    return Problem(m, n, k, A, TAU, NU)


@dataclass
class Refl3Problem:
    m: int
    n: int
    k: int
    A: np.ndarray    # (m, n) column-major view, float64
    TAU: np.ndarray  # (n-2, k) column-major views, float64
    NU1: np.ndarray
    NU2: np.ndarray

    @property
    def flops(self):
        """Counted work: 10 flops per (reflector, row), 10 m (n-2) k
        (w = x + nu1 y + nu2 z: 4; x, y, z updates: 2 each)."""
        return 10 * self.m * max(self.n - 2, 0) * self.k


def make_reflectors3(r, k, rng, *, lds=(None, None, None), identity_frac=0.05, pad_fill=np.nan):
    """(r x k) parameters (tau, nu1, nu2) of orthogonal 3x3 reflectors
    I - tau v v^T, v = (1, nu1, nu2): the unit normal u of the reflecting
    plane is uniform on the sphere and v = u / u_0, so tau = 2 u_0^2; a
    fraction ``identity_frac`` is tau = 0 (identity), as for windows that
    are already reduced.  ``lds`` are the three leading dimensions."""
    u = rng.standard_normal(3 * r * k).reshape(3, k, r).transpose(0, 2, 1)
    u = u / np.linalg.norm(u, axis=0)
    ident = rng.uniform(0.0, 1.0, r * k).reshape(k, r).T < identity_frac
    TAU, NU1, NU2 = (_colmajor_buffer(r, k, ld, pad_fill)[1] for ld in lds)
    NU1[...] = u[1] / u[0]
    NU2[...] = u[2] / u[0]
    TAU[...] = np.where(ident, 0.0, 2.0 / (1.0 + NU1 * NU1 + NU2 * NU2))
    return TAU, NU1, NU2


def make_refl3_problem(m, n, k, seed=0, *, lda=None, lds=(None, None, None), pad_fill=np.nan):
    """3x3 reflector problem: A i.i.d. normal (m x n), (n-2) x k reflectors."""
    rng = np.random.Generator(np.random.PCG64(seed))
    _, A = _colmajor_buffer(m, n, lda, pad_fill)
    A[...] = rng.standard_normal(m * n).reshape(n, m).T
    TAU, NU1, NU2 = make_reflectors3(max(n - 2, 0), k, rng, lds=lds, pad_fill=pad_fill)
    return Refl3Problem(m, n, k, A, TAU, NU1, NU2)


def make_cs(n, k, rng):
    """Fresh rotation coefficients (n-1) x k, contiguous column-major."""
    nm1 = max(n - 1, 0)
    theta = rng.uniform(0.0, TWO_PI, nm1 * k).reshape(k, nm1).T
    return np.asfortranarray(np.cos(theta)), np.asfortranarray(np.sin(theta))


def log_uniform_int(rng, lo, hi, size=None):
    """round(exp(U[ln lo, ln hi])) clipped to [lo, hi]."""
    v = np.exp(rng.uniform(math.log(lo), math.log(hi), size))
    return np.clip(np.rint(v), lo, hi).astype(np.int64)


def batched_shapes(count=512, seed=4, n_lo=64, n_hi=2048, ks=(8, 16, 32, 64)):
    """Shapes of the uneven batch: n log-uniform, m = n, k uniform over ``ks``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = log_uniform_int(rng, n_lo, n_hi, count)
    kk = rng.choice(np.asarray(ks), count)
    return [(int(n), int(n), int(k)) for n, k in zip(ns, kk)]


def batched_problems(count=512, seed=4, **kw):
    """The uneven batch: one independent PCG64 stream per problem."""
    shapes = batched_shapes(count, seed, **kw)
    children = np.random.SeedSequence(seed).spawn(count)
    out = []
    for (m, n, k), ss in zip(shapes, children):
        out.append(make_problem(m, n, k, rng=np.random.Generator(np.random.PCG64(ss))))
    return out


def served_requests(count, seed=5, n_lo=128, n_hi=4096, sweeps=20,
                    ks=(16, 32, 64, 128), rate_per_s=1000.0):
    """Served stream: Poisson arrivals, resident matrices, 20 sweeps each.

    k is drawn once per request; every sweep draws fresh angles.  Returns a
    list of dicts with arrival time (s), shape, k and the per-request seed
    sequence from which the matrix and the sweeps' coefficients are drawn.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_per_s, count)
    ns = log_uniform_int(rng, n_lo, n_hi, count)
    kk = rng.choice(np.asarray(ks), count)
    children = np.random.SeedSequence(seed).spawn(count)
    t = np.cumsum(gaps)
    return [dict(arrival=float(t[i]), m=int(ns[i]), n=int(ns[i]), k=int(kk[i]),
                 sweeps=sweeps, seed=children[i]) for i in range(count)]


def request_matrix(req):
    """The resident matrix of a served request, and a generator for its sweeps."""
    rng = np.random.Generator(np.random.PCG64(req["seed"]))
    m, n = req["m"], req["n"]
    A = np.asfortranarray(rng.standard_normal(m * n).reshape(n, m).T)
    return A, rng
