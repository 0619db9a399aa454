"""Seeded synthetic pencils (A, B) shaped like the paper's workloads.

This module holds only input generation; it contains none of the reduction's
arithmetic, so both the HIP path's tests/benchmarks and the CPU oracle draw
their inputs from here.

Generators (numpy ``default_rng`` = PCG64, FP64, column-major output; A is
always drawn before B's source):

* ``random_pencil``: Test Suite 1 of Sec. 4 -- A with iid N(0,1) entries, B
  the triangular factor of the QR factorisation of an iid N(0,1) matrix (a
  fairly well-conditioned B with no infinite eigenvalues).
* ``illcond_pencil``: A iid N(0,1); B upper triangular with iid N(0,1)
  strictly-upper entries and diagonal magnitudes log-uniform in [1e-8, 1]
  with random signs.  Back substitution with such a B grows without bound
  (it overflows FP64 beyond n ~ 128), so it stresses the overflow-safe
  solves behind the opposite reflectors.
* ``batch_sizes`` / ``batch_pencil``: many independent small pencils with
  orders uniform in [32, 512] (HT reduction inside deflation windows, Sec. 1),
  pencil i seeded by ``SeedSequence(seed).spawn(count)[i]``.
* ``zero_column_pencil``: random_pencil with some columns of B set to
  zero (input of the zero-column preprocessing of Sec. 3.5).
* ``saddle_pencil``: Test Suite 4 of Sec. 4 -- A = [X Y; Y^T 0],
  B = diag(I, 0) with X symmetric positive definite of order 3n/4.  Here X =
  G G^T / m + I with Gaussian G and Y Gaussian (the paper states only
  "random SPD" and "random full-rank").

Named workloads (``workload(name)``):
  "n256"  : random_pencil(256, seed=0)
  "n4096" : random_pencil(4096, seed=1)
  "n16384": illcond_pencil(16384, seed=2)
  "batch" : 2048 pencils, sizes from batch_sizes(2048, seed=4)
"""
import numpy as np


def _layout(M, order):
    return np.asfortranarray(M) if order == "F" else np.ascontiguousarray(M)


def random_pencil(n, seed, order="F"):
    """``order`` only picks the memory layout of the returned arrays ("F":
    column-major, "C": row-major, which skips a large transposing copy);
    the matrices are the same."""
    rng = np.random.default_rng(seed)
    A = _layout(rng.standard_normal((n, n)), order)
    G = rng.standard_normal((n, n))
    if n == 0:
        return A, _layout(G, order)
    R = np.linalg.qr(G, mode="r")
    B = _layout(np.triu(R), order)
    return A, B


def illcond_pencil(n, seed, order="F"):
    rng = np.random.default_rng(seed)
    A = _layout(rng.standard_normal((n, n)), order)
    B = rng.standard_normal((n, n))
    B = np.triu(B, 1)
    mags = 10.0 ** rng.uniform(-8.0, 0.0, size=n)
    signs = np.where(rng.integers(0, 2, size=n) == 0, -1.0, 1.0)
    B[np.arange(n), np.arange(n)] = signs * mags
    return A, _layout(B, order)


def saddle_pencil(n, seed):
    rng = np.random.default_rng(seed)
    m = (3 * n) // 4
    G = rng.standard_normal((m, m))
    X = G @ G.T / max(m, 1) + np.eye(m)
    Y = rng.standard_normal((m, n - m))
    A = np.zeros((n, n))
    A[:m, :m] = X
    A[:m, m:] = Y
    A[m:, :m] = Y.T
    B = np.zeros((n, n))
    B[np.arange(m), np.arange(m)] = 1.0
    return np.asfortranarray(A), np.asfortranarray(B)


def zero_column_pencil(n, ell, seed):
    """random_pencil(n, seed) with `ell` of B's columns (chosen uniformly,
    drawn after A and B's source) set to zero: ell infinite eigenvalues and a
    rank n - ell triangular B, the input of the zero-column preprocessing of
    Sec. 3.5 with a nonsingular B22 afterwards."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    G = rng.standard_normal((n, n))
    B = np.triu(np.linalg.qr(G, mode="r")) if n else G
    cols = rng.choice(n, size=ell, replace=False) if ell else []
    B[:, cols] = 0.0
    return np.asfortranarray(A), np.asfortranarray(B)


def batch_sizes(count, seed, lo=32, hi=512):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=count)


def batch_pencil(i, n, count, seed):
    child = np.random.SeedSequence(seed).spawn(count)[i]
    return random_pencil(int(n), child)


def batch_pencils(count, seed, lo=32, hi=512):
    """List of (A, B) for the batched workload (pencil i from child seed i)."""
    sizes = batch_sizes(count, seed, lo, hi)
    children = np.random.SeedSequence(seed).spawn(count)
    return [random_pencil(int(n), children[i]) for i, n in enumerate(sizes)]


WORKLOADS = {
    "n256": ("random", 256, 0),
    "n4096": ("random", 4096, 1),
    "n16384": ("illcond", 16384, 2),
}


def workload(name, n=None, order="F"):
    kind, n0, seed = WORKLOADS[name]
    n = n0 if n is None else n
    if kind == "random":
        return random_pencil(n, seed, order)
    return illcond_pencil(n, seed, order)
