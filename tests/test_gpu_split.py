"""GPU checks of the precision form (split-precision WY updates).

1. ht_wy_gemm on operands whose digit slices represent them exactly (and
   whose dropped slice pairs are zero): the emulated product must equal the
   exact product bit for bit.  This pins the MFMA lane layouts, the level
   weights, the per-chunk exponents, all four transposition kernels and
   ragged tile / chunk tails, for the BF16 and the FP8 digit formats, on
   grids of one tile, of several row tiles and of several column tiles.
2. Random FP64 operands: the error stays within the bound of the splitting,
   (ns + 5) 2^{-b ns} 2^{e_row + e_col} per contraction index, and it
   shrinks as slices are added.
3. ht_reduce with split WY updates: the FP64 invariants (orthogonality <=
   1e-13 n, backward errors <= 1e-14 n) and parity with the oracle at 1e-10,
   the same bars as the native form; with few slices the backward error
   grows, which shows the split products are really in the path.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import checks
from paper_1710_08538_amd import htred, inputs

pytestmark = pytest.mark.gpu
TOL = 1e-10
BITS = {htred.HT_PREC_SPLIT_BF16: 7, htred.HT_PREC_SPLIT_FP8: 4}
U = 2.0 ** -53


def dev(M):
    return htred.to_device_colmajor(M)


def stored(M, trans):
    """The array handed to the product for op(X) = M."""
    return np.asfortranarray(M.T if trans else M)


def run_gemm(opA, opB, ta, tb, prec, ns, C0=None, alpha=1.0, beta=0.0):
    print("ht_wy_gemm prec=%d ns=%d ta=%d tb=%d m,k,n=%s" % (prec, ns, ta, tb,
          (opA.shape[0], opA.shape[1], opB.shape[1])), flush=True)
    C = dev(C0) if C0 is not None else None
    out = htred.wy_gemm(dev(stored(opA, ta)), dev(stored(opB, tb)), C=C, transA=ta, transB=tb,
                        alpha=alpha, beta=beta if C0 is not None else 0.0, prec=prec,
                        n_slices=ns)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def exact_operands(prec, m, k, n, seed):
    """op(A): one-digit integers times per-row powers of two; op(B): integers
    of three digits times per-column powers of two.  With ns >= 3 every slice
    pair that is kept is exact and every dropped pair is zero, and the FP64
    product of such operands is exact too."""
    b = BITS[prec]
    rng = np.random.default_rng(seed)
    A = rng.integers(-(2 ** b - 1), 2 ** b, size=(m, k)).astype(np.float64)
    B = rng.integers(-(2 ** (3 * b) - 1), 2 ** (3 * b), size=(k, n)).astype(np.float64)
    A *= np.exp2(rng.integers(-30, 30, size=(m, 1)))
    B *= np.exp2(rng.integers(-30, 30, size=(1, n)))
    A[rng.random((m, k)) < 0.1] = 0.0  # zero entries and an all-zero row
    A[min(3, m - 1), :] = 0.0
    return A, B


@pytest.mark.parametrize("prec", [htred.HT_PREC_SPLIT_BF16, htred.HT_PREC_SPLIT_FP8])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
@pytest.mark.parametrize("m,k,n", [(64, 32, 64), (130, 77, 45), (1, 1, 1), (200, 300, 129),
                                   (40, 96, 300), (64, 256, 256)])
def test_split_gemm_exact_on_representable_operands(prec, ta, tb, m, k, n):
    A, B = exact_operands(prec, m, k, n, seed=m * 7 + k + n)
    got = run_gemm(A, B, ta, tb, prec, 3)
    np.testing.assert_array_equal(got, A @ B)


@pytest.mark.parametrize("prec", [htred.HT_PREC_SPLIT_BF16, htred.HT_PREC_SPLIT_FP8])
def test_split_gemm_alpha_beta(prec):
    A, B = exact_operands(prec, 70, 40, 33, seed=5)
    C0 = np.random.default_rng(6).integers(-1000, 1000, size=(70, 33)).astype(np.float64)
    got = run_gemm(A, B, False, False, prec, 3, C0=C0, alpha=-2.0, beta=0.5)
    np.testing.assert_array_equal(got, -2.0 * (A @ B) + 0.5 * C0)


def split_bound(A, B, prec, ns):
    b = BITS[prec]
    k = A.shape[1]
    rowmax = np.abs(A).max(axis=1, keepdims=True)
    colmax = np.abs(B).max(axis=0, keepdims=True)
    # per index: dropped slice pairs < (ns + 2.1) 2^{-b ns}, remainders
    # < 2^{1 - b ns}; exponents 2^e <= 2 max, for rows and for columns
    return (4.0 * k * (ns + 5) * 2.0 ** (-b * ns) * rowmax * colmax
            + 4.0 * k * U * (np.abs(A) @ np.abs(B)))


@pytest.mark.parametrize("prec,slices", [(htred.HT_PREC_SPLIT_BF16, (2, 4, 7, 8)),
                                         (htred.HT_PREC_SPLIT_FP8, (3, 7, 13, 14))])
def test_split_gemm_error_bound(prec, slices):
    rng = np.random.default_rng(11)
    m, k, n = 150, 256, 100
    A = rng.standard_normal((m, k)) * np.exp2(rng.integers(-20, 20, size=(m, 1)))
    B = rng.standard_normal((k, n)) * np.exp2(rng.integers(-20, 20, size=(1, n)))
    ref = A @ B  # FP64; its own error is inside the bound's u term
    errs = []
    for ns in slices:
        got = run_gemm(A, B, True, False, prec, ns)
        err = np.abs(got - ref)
        assert (err <= split_bound(A, B, prec, ns)).all(), (ns, float(err.max()))
        errs.append(float((err / (np.abs(A) @ np.abs(B))).max()))
    # more slices, smaller error (down to the FP64 level)
    assert errs[0] > 1e3 * errs[-1], errs
    assert errs[-1] < 1e-13, errs


def test_fp64_path_of_wy_gemm():
    rng = np.random.default_rng(3)
    A, B = rng.standard_normal((90, 70)), rng.standard_normal((70, 50))
    got = run_gemm(A, B, False, False, htred.HT_PREC_FP64, 0)
    np.testing.assert_allclose(got, A @ B, rtol=0, atol=1e-12)


@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
@pytest.mark.parametrize("m,k,n", [(1, 1, 1), (64, 16, 64), (130, 77, 45), (200, 300, 129),
                                   (17, 1000, 33), (300, 5, 260), (65, 0, 63)])
def test_fp64_wy_gemm_exact(ta, tb, m, k, n):
    """The FP64 matrix-core product on operands whose products and sums are
    exact in FP64 (small integers times powers of two): every entry equals
    the exact result, for the four transposition variants, ragged tiles and
    chunks, and an empty contraction (C = beta C)."""
    rng = np.random.default_rng(m * 7 + k * 3 + n)
    A = rng.integers(-7, 8, size=(m, k)).astype(np.float64) * np.exp2(rng.integers(-20, 20, (m, 1)))
    B = rng.integers(-2 ** 20, 2 ** 20, size=(k, n)).astype(np.float64) * \
        np.exp2(rng.integers(-20, 20, (1, n)))
    C0 = rng.integers(-2 ** 20, 2 ** 20, size=(m, n)).astype(np.float64)
    got = run_gemm(A, B, ta, tb, htred.HT_PREC_FP64, 0)
    assert np.array_equal(got, A @ B)
    got = run_gemm(A, B, ta, tb, htred.HT_PREC_FP64, 0, C0=C0, alpha=-2.0, beta=0.5)
    assert np.array_equal(got, -2.0 * (A @ B) + 0.5 * C0)


def run_reduce(A0, B0, **kw):
    print("ht_reduce n=%d %s" % (A0.shape[0], kw), flush=True)
    A, B = dev(A0), dev(B0)
    Q, Z, st = htred.reduce(A, B, stats=True, **kw)
    torch.cuda.synchronize()
    return (A.cpu().numpy(), B.cpu().numpy(), Q.cpu().numpy(), Z.cpu().numpy()), st


@pytest.mark.parametrize("prec,n,nb", [(htred.HT_PREC_SPLIT_BF16, 700, 64),
                                       (htred.HT_PREC_SPLIT_BF16, 1000, 128),
                                       (htred.HT_PREC_SPLIT_FP8, 700, 64)])
def test_reduce_split_matches_fp64_bars(prec, n, nb):
    A0, B0 = inputs.random_pencil(n, seed=n + 17)
    got, st = run_reduce(A0, B0, nb=nb, prec=prec)
    inv = checks.invariants(A0, B0, *got)
    assert checks.invariants_ok(inv, n), str(inv)
    assert st["absorptions"] >= 2
    d = checks.compare(oracle.ms_ht(A0, B0), got, A0, B0)
    for key in ("max_H", "max_T", "max_Q", "max_Z"):
        assert d[key] <= TOL, (key, d)


def test_reduce_split_illconditioned():
    A0, B0 = inputs.illcond_pencil(600, seed=23)
    got, st = run_reduce(A0, B0, nb=64, prec=htred.HT_PREC_SPLIT_BF16)
    assert all(np.isfinite(M).all() for M in got)
    inv = checks.invariants(A0, B0, *got)
    assert checks.invariants_ok(inv, 600), str(inv)


def test_reduce_few_slices_degrades_backward_error():
    """Three BF16 slices keep about 21 bits: the backward error rises far
    above the FP64 level, so the split products are the ones in use."""
    n = 500
    A0, B0 = inputs.random_pencil(n, seed=31)
    got64, _ = run_reduce(A0, B0, nb=64)
    got3, _ = run_reduce(A0, B0, nb=64, prec=htred.HT_PREC_SPLIT_BF16, n_slices=3)
    inv64 = checks.invariants(A0, B0, *got64)
    inv3 = checks.invariants(A0, B0, *got3)
    assert inv3["bwd_A"] > 1e3 * inv64["bwd_A"], (inv3, inv64)
    assert inv3["bwd_A"] < 1e-3, inv3
