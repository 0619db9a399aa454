"""GPU parity of the steps around the reduction, through the C ABI:
ht_triangularize_b (the QR front end of the QZ algorithm, Sec. 1) and
ht_preprocess + ht_reduce with ilo (the zero-column preprocessing of
Sec. 3.5), against the CPU reference in oracle/preprocess.py.

QR factors are unique up to the signs of R's rows, and the preprocessed HT
reduction up to the signs fixed by checks.sign_normalise_ilo; entries are
compared after those normalisations at 1e-10 relative to ||A||_F, ||B||_F,
sqrt(n), as for ht_reduce.  Pencils whose T keeps exact zeros on its
trailing diagonal (the saddle-point pencils of Test Suite 4) have no unique
reduction; they are checked by the invariants."""
import numpy as np
import pytest
import torch

from oracle import checks, preprocess
from paper_1710_08538_amd import htred, inputs

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _dev(M):
    return htred.to_device_colmajor(M)


def _host(*Ms):
    torch.cuda.synchronize()
    return tuple(M.cpu().numpy() for M in Ms)


def _residuals(A0, B0, H, T, Q, Z):
    n = A0.shape[0]
    I = np.eye(n)
    return {"bwd_A": np.linalg.norm(Q @ H @ Z.T - A0) / np.linalg.norm(A0),
            "bwd_B": np.linalg.norm(Q @ T @ Z.T - B0) / max(np.linalg.norm(B0), 1e-300),
            "orth_Q": np.linalg.norm(Q.T @ Q - I), "orth_Z": np.linalg.norm(Z.T @ Z - I)}


def _bars_ok(r, n):
    n = max(n, 1)
    return (r["bwd_A"] <= 1e-14 * n and r["bwd_B"] <= 1e-14 * n and r["orth_Q"] <= 1e-13 * n
            and r["orth_Z"] <= 1e-13 * n)


@pytest.mark.parametrize("n,nb", [(1, 64), (2, 64), (50, 64), (130, 64), (131, 32), (300, 128),
                                  (700, 64), (1000, 128)])
def test_triangularize_b_matches_oracle(n, nb):
    rng = np.random.default_rng(n + nb)
    A0, B0 = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    print("ht_triangularize_b n=%d nb=%d" % (n, nb), flush=True)
    A, B = _dev(A0), _dev(B0)
    Q = htred.triangularize_b(A, B, nb=nb)
    A1, R, Q0 = _host(A, B, Q)
    assert not np.any(np.tril(R, -1))
    rA, rR, rQ = preprocess.triangularize_b(A0, B0)
    dg, dr = np.sign(np.diag(R)), np.sign(np.diag(rR))
    nA, nB = np.linalg.norm(A0), np.linalg.norm(B0)
    assert np.abs(dg[:, None] * R - dr[:, None] * rR).max() <= TOL * nB
    assert np.abs(dg[:, None] * A1 - dr[:, None] * rA).max() <= TOL * nA
    assert np.abs(Q0 * dg[None, :] - rQ * dr[None, :]).max() <= TOL * np.sqrt(n)
    assert np.linalg.norm(Q0 @ R - B0) <= 1e-14 * n * nB
    assert np.linalg.norm(Q0 @ A1 - A0) <= 1e-14 * n * nA
    assert np.linalg.norm(Q0.T @ Q0 - np.eye(n)) <= 1e-13 * n


def test_triangularize_b_accumulates_and_feeds_the_reduction():
    """QZ step 1 then the HT reduction with accumulated Q: the whole chain
    (A, general B) -> (H, T) meets the bars, and equals the oracle's chain
    (numpy QR, then O-fast) after sign normalisation."""
    import oracle
    n, nb = 300, 64
    rng = np.random.default_rng(5)
    A0, B0 = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    print("ht_triangularize_b + ht_reduce n=%d" % n, flush=True)
    A, B = _dev(A0), _dev(B0)
    Q = htred.triangularize_b(A, B, nb=nb)
    Z = htred.colmajor_empty(n)
    htred.reduce(A, B, Q, Z, nb=nb, qmode=htred.HT_QZ_ACCUMULATE)
    got = _host(A, B, Q, Z)
    r = _residuals(A0, B0, *got)
    assert _bars_ok(r, n), r
    assert not np.any(np.tril(got[0], -2)) and not np.any(np.tril(got[1], -1))
    rA, rR, rQ = preprocess.triangularize_b(A0, B0)
    H, T, Qh, Zh, _ = oracle.fast_ht(rA, rR)
    # the front end's Q0 fixes Q e1 up to sign: normalise through T(0,0) (Z e1 = e1)
    ref = (H, T, rQ @ Qh, Zh)
    d = checks.compare_ilo(ref, got, A0, B0, 0)
    for key in ("max_H", "max_T", "max_Q", "max_Z"):
        assert d[key] <= TOL, (key, d)


def _diag_pencil(n, ell, seed):
    """A ~ N(0,1); B diagonal with ell exact zeros (at random places) and
    the other entries uniform in [0.5, 2] with random signs."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    d = rng.uniform(0.5, 2.0, n) * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    d[rng.choice(n, size=ell, replace=False)] = 0.0
    return np.asfortranarray(A), np.asfortranarray(np.diag(d))


@pytest.mark.parametrize("kind,n,ell,nb", [("tri", 40, 5, 16), ("tri", 300, 20, 64),
                                           ("tri", 700, 130, 64), ("diag", 257, 40, 32),
                                           ("tri", 1000, 300, 128)])
def test_preprocess_then_reduce_matches_oracle(kind, n, ell, nb):
    A0, B0 = (inputs.zero_column_pencil(n, ell, seed=n) if kind == "tri"
              else _diag_pencil(n, ell, seed=n))
    print("ht_preprocess + ht_reduce(ilo) %s n=%d l=%d nb=%d" % (kind, n, ell, nb), flush=True)
    A, B = _dev(A0), _dev(B0)
    Q, Z, ilo = htred.preprocess(A, B, nb=nb)
    assert ilo == ell
    htred.reduce(A, B, Q, Z, nb=nb, ilo=ilo, qmode=htred.HT_QZ_ACCUMULATE,
                 zmode=htred.HT_QZ_ACCUMULATE)
    got = _host(A, B, Q, Z)
    H, T = got[0], got[1]
    assert not np.any(np.tril(H, -2)) and not np.any(np.tril(T, -1)) and not np.any(T[:, :ell])
    r = _residuals(A0, B0, *got)
    assert _bars_ok(r, n), r
    ref = preprocess.preprocessed_ht(A0, B0)
    assert ref[4] == ell
    d = checks.compare_ilo(ref[:4], got, A0, B0, ell)
    for key in ("max_H", "max_T", "max_Q", "max_Z"):
        assert d[key] <= TOL, (key, d)


def test_preprocess_without_zero_columns_is_a_no_op():
    n = 64
    A0, B0 = inputs.random_pencil(n, seed=8)
    A, B = _dev(A0), _dev(B0)
    Q, Z, ilo = htred.preprocess(A, B, nb=32)
    got = _host(A, B, Q, Z)
    assert ilo == 0
    assert np.array_equal(got[0], A0) and np.array_equal(got[1], np.triu(B0))
    assert np.array_equal(got[2], np.eye(n)) and np.array_equal(got[3], np.eye(n))


@pytest.mark.parametrize("n,nb", [(64, 16), (400, 64)])
def test_saddle_pencils_preprocessed(n, nb):
    """Test Suite 4's saddle-point pencils (B = diag(I, 0), l = n/4):
    preprocessing then the reduction meet the invariants; T's first l
    columns are zero."""
    A0, B0 = inputs.saddle_pencil(n, seed=n)
    print("ht_preprocess saddle n=%d" % n, flush=True)
    A, B = _dev(A0), _dev(B0)
    Q, Z, ilo = htred.preprocess(A, B, nb=nb)
    assert ilo == n - (3 * n) // 4
    Q, Z, st = htred.reduce(A, B, Q, Z, nb=nb, ilo=ilo, qmode=htred.HT_QZ_ACCUMULATE,
                            zmode=htred.HT_QZ_ACCUMULATE, stats=True)
    got = _host(A, B, Q, Z)
    assert not np.any(np.tril(got[0], -2)) and not np.any(np.tril(got[1], -1))
    assert not np.any(got[1][:, :ilo])
    r = _residuals(A0, B0, *got)
    assert _bars_ok(r, n), r
    assert st["columns"] == n - 2 - ilo
