"""GPU parity of the accelerated absorption with l >= 3 blocks (Sec. 3.5:
accelerated reduction of V2 and U2, block triangular reduction of B, block
back substitution) through ht_reduce with ht_options.ell, against the CPU
oracle.

Hessenberg-triangular reduction with Q e1 = Z e1 = e1 is unique up to signs
(implicit-Q theorem), so the l-block scheme must reach the same sign-
normalised H, T, Q, Z as Algorithm 2 and the basic scheme; the tolerances
are those of the basic scheme's parity tests."""
import numpy as np
import pytest

import oracle
from oracle import checks
from paper_1710_08538_amd import inputs

from test_gpu_reduce import TOL, assert_invariants, assert_parity, run_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,nb,ell", [(5, 1, 3), (12, 2, 3), (40, 8, 3), (70, 8, 4), (100, 16, 3),
                                      (131, 32, 3), (200, 64, 3), (257, 32, 4), (300, 32, 5),
                                      (301, 64, 3)])
def test_ell_parity_with_basic_ht(n, nb, ell):
    A0, B0 = inputs.random_pencil(n, seed=4000 + n)
    got, st = run_gpu(A0, B0, nb=nb, ell=ell)
    assert_invariants(A0, B0, got)
    assert_parity(oracle.basic_ht(A0, B0)[:4], got, A0, B0)
    assert st["columns"] == max(n - 2, 0)
    assert st["scaled_solves"] == 0


def test_ell_forced_refinement_failures():
    """Panels cut after one reflector pair (k = 1 absorptions): windows of
    (l-1) nb + 1 rows and one-reflector restoring steps (the refinement
    failure case of Sec. 3.5)."""
    n = 70
    A0, B0 = inputs.random_pencil(n, seed=5)
    got, st = run_gpu(A0, B0, nb=16, ell=3, max_ir=0, ir_tol_factor=0.0)
    assert st["ir_failures"] > 0
    assert n - 2 - 2 <= st["absorptions"] <= n - 2
    assert_invariants(A0, B0, got)
    assert_parity(oracle.basic_ht(A0, B0)[:4], got, A0, B0)


def test_ell_partial_refinement_failures():
    n = 150
    A0, B0 = inputs.random_pencil(n, seed=6)
    got, st = run_gpu(A0, B0, nb=32, ell=3, max_ir=2, ir_tol_factor=0.05)
    assert_invariants(A0, B0, got)
    assert_parity(oracle.basic_ht(A0, B0)[:4], got, A0, B0)


def test_ell_n1000_matches_oracle_and_basic_scheme():
    n = 1000
    A0, B0 = inputs.random_pencil(n, seed=7)
    got3, st3 = run_gpu(A0, B0, nb=64, ell=3)
    print(st3, flush=True)
    assert_invariants(A0, B0, got3)
    ref = oracle.fast_ht(A0, B0)[:4]
    assert_parity(ref, got3, A0, B0)
    got2, st2 = run_gpu(A0, B0, nb=64)
    d = checks.compare(got2, got3, A0, B0)
    assert max(d[k] for k in ("max_H", "max_T", "max_Q", "max_Z")) <= TOL, d
    assert st3["columns"] == st2["columns"] == n - 2


def test_ell_with_split_precision_products():
    """The l-block scheme with its window products in the BF16 precision form
    meets the FP64 bars (the products go through the same WY-update path)."""
    from paper_1710_08538_amd import htred
    n = 300
    A0, B0 = inputs.random_pencil(n, seed=n + 17)
    got, st = run_gpu(A0, B0, nb=32, ell=3, prec=htred.HT_PREC_SPLIT_BF16)
    assert_invariants(A0, B0, got)
    assert_parity(oracle.ms_ht(A0, B0), got, A0, B0)


def test_ell_after_zero_column_preprocessing():
    """ht_preprocess, then the l-block reduction from column ilo."""
    from oracle import preprocess
    from paper_1710_08538_amd import htred
    from test_gpu_front import _bars_ok, _dev, _host, _residuals
    n, ell0, nb = 300, 20, 32
    A0, B0 = inputs.zero_column_pencil(n, ell0, seed=n)
    print("ht_preprocess + ht_reduce(ilo, ell=3) n=%d" % n, flush=True)
    A, B = _dev(A0), _dev(B0)
    Q, Z, ilo = htred.preprocess(A, B, nb=nb)
    assert ilo == ell0
    htred.reduce(A, B, Q, Z, nb=nb, ilo=ilo, ell=3, qmode=htred.HT_QZ_ACCUMULATE,
                 zmode=htred.HT_QZ_ACCUMULATE)
    got = _host(A, B, Q, Z)
    assert not np.any(np.tril(got[0], -2)) and not np.any(np.tril(got[1], -1))
    r = _residuals(A0, B0, *got)
    assert _bars_ok(r, n), r
    ref = preprocess.preprocessed_ht(A0, B0)
    d = checks.compare_ilo(ref[:4], got, A0, B0, ell0)
    for key in ("max_H", "max_T", "max_Q", "max_Z"):
        assert d[key] <= TOL, (key, d)
