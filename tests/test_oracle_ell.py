"""Pins of the l-block absorption geometry (Sec. 3.5, accelerated reduction of
V2 and U2, block triangular reduction of B, block back substitution) in
oracle/ell_blocks.py, against what the mathematics fixes: orthogonality,
the reduced forms of V2 and U2, B's block upper triangular form, the number
of reflectors of the restoring transforms, and the solution of B x = c."""
import numpy as np
import pytest

from oracle import ell_blocks as eb


def block_upper(m, s, rng):
    bounds = eb.block_bounds(m, s)
    B = np.triu(rng.standard_normal((m, m)))
    for a, e in zip(bounds[:-1], bounds[1:]):
        B[a:e, a:e] = rng.standard_normal((e - a, e - a)) + 4 * np.eye(e - a)
    return B, bounds


def reflector_count(G):
    """Rank of G - I: a product of c reflectors differs from I by rank <= c."""
    sv = np.linalg.svd(G - np.eye(G.shape[0]), compute_uv=False)
    return int((sv > 1e-10).sum())


@pytest.mark.parametrize("m,s", [(1, 4), (4, 4), (5, 4), (8, 4), (23, 4), (24, 8), (130, 64)])
def test_block_bounds_cover_and_align_at_the_bottom(m, s):
    b = eb.block_bounds(m, s)
    assert b[0] == 0 and b[-1] == m
    sizes = np.diff(b)
    assert (sizes > 0).all()
    assert (sizes[1:] == s).all() and 0 < sizes[0] <= s


@pytest.mark.parametrize("r,c", [(4, 2), (8, 4), (6, 1), (16, 8), (5, 5)])
def test_clear_leading_columns(r, c):
    """2nb x 3nb construction (l = 3, k = nb) and its (2nb + k) variant: C G
    has zero first c columns, G is orthogonal and consists of c reflectors."""
    rng = np.random.default_rng(r * 10 + c)
    C = rng.standard_normal((r, r + c))
    G = eb.clear_leading_columns(C, c)
    assert np.abs(G.T @ G - np.eye(r + c)).max() < 1e-14
    assert np.abs((C @ G)[:, :c]).max() < 1e-13 * np.abs(C).max()
    assert reflector_count(G) == c


@pytest.mark.parametrize("z,c", [(4, 2), (8, 4), (6, 1), (16, 8), (3, 5)])
def test_clear_trailing_rows(z, c):
    rng = np.random.default_rng(z * 10 + c + 1)
    C = rng.standard_normal((z + c, z))
    G = eb.clear_trailing_rows(C, c)
    assert np.abs(G.T @ G - np.eye(z + c)).max() < 1e-14
    assert np.abs((G.T @ C)[z:, :]).max() < 1e-13 * np.abs(C).max()
    assert reflector_count(G) == c


CASES = [(20, 4, 2), (23, 4, 2), (23, 4, 1), (9, 4, 2), (4, 4, 2), (41, 8, 4), (13, 6, 3),
         (64, 16, 8), (70, 16, 5)]


@pytest.mark.parametrize("m,s,k", CASES)
def test_right_pass(m, s, k):
    rng = np.random.default_rng(m * 100 + s * 10 + k)
    B, bounds = block_upper(m, s, rng)
    V2 = rng.standard_normal((m, k))
    B1, V, Z, nrefl = eb.right_pass(B, V2, k, s)
    scale = np.abs(B).max()
    assert np.abs(Z.T @ Z - np.eye(m)).max() < 1e-13
    assert np.abs(B @ Z - B1).max() < 1e-13 * scale  # only rounding-level entries zeroed
    assert eb.below_blocks_max(B1, bounds) == 0.0
    # V2 -> [0; L1]: the windows' transforms alone, applied to V2
    assert np.array_equal(V[:m - k], np.zeros((m - k, k)))
    assert np.array_equal(np.triu(V[m - k:], 1), np.zeros((k, k)))
    assert abs(np.linalg.norm(V) - np.linalg.norm(V2)) < 1e-12 * np.linalg.norm(V2)
    # one restoring transform of carry reflectors per block below the top one
    carries = [cr for _, _, cr in eb.right_windows(bounds, k)]
    assert nrefl == sum(carries)
    assert all(cr == k for cr in carries[2:])


@pytest.mark.parametrize("m,s,k", CASES)
def test_left_pass(m, s, k):
    rng = np.random.default_rng(m * 100 + s * 10 + k + 7)
    B, bounds = block_upper(m, s, rng)
    U2 = rng.standard_normal((m, k))
    B1, U, Q, nrefl = eb.left_pass(B, U2, k, s)
    scale = np.abs(B).max()
    assert np.abs(Q.T @ Q - np.eye(m)).max() < 1e-13
    assert np.abs(Q.T @ B - B1).max() < 1e-13 * scale
    assert eb.below_blocks_max(B1, bounds) == 0.0
    assert np.array_equal(U[k:], np.zeros((m - k, k)))
    assert np.array_equal(np.tril(U[:k], -1), np.zeros((k, k)))
    assert abs(np.linalg.norm(U) - np.linalg.norm(U2)) < 1e-12 * np.linalg.norm(U2)
    assert nrefl == k * (len(bounds) - 2)


def test_window_count_falls_by_about_l_minus_one():
    """Sec. 3.5: about (n - nb) / ((l - 1) nb) transformations instead of
    (n - nb) / nb."""
    m, nb = 1024, 32
    for ell in (2, 3, 4, 5):
        wins = eb.right_windows(eb.block_bounds(m, (ell - 1) * nb), nb)
        assert len(wins) == -(-m // ((ell - 1) * nb))


@pytest.mark.parametrize("m,s", [(1, 4), (7, 4), (23, 4), (64, 16), (100, 32)])
def test_block_solve(m, s):
    rng = np.random.default_rng(m + s)
    B, bounds = block_upper(m, s, rng)
    c = rng.standard_normal(m)
    x = eb.block_solve(B, bounds, c)
    assert np.abs(x - np.linalg.solve(B, c)).max() < 1e-12 * max(1.0, np.abs(x).max())


def test_block_solve_pivots():
    """A diagonal block with a zero leading entry needs the row interchange."""
    B = np.array([[0.0, 1.0, 2.0], [1.0, 0.0, 3.0], [0.0, 0.0, 5.0]])
    x = eb.block_solve(B, [0, 2, 3], np.array([1.0, 2.0, 5.0]))
    assert np.allclose(x, [-1.0, -1.0, 1.0], rtol=0, atol=1e-15)


# Planted mistakes: each plausible slip in the geometry must fail a pin above.

def _pins_right(m=41, s=8, k=4):
    test_right_pass(m, s, k)


def _pins_left(m=41, s=8, k=4):
    test_left_pass(m, s, k)


def test_planted_windows_without_carry_fail(monkeypatch):
    """V2 windows that cover only their own block (no rows carried from the
    window above) leave V2 unreduced."""
    def no_carry(bounds, k):
        return [(a, e, 0) for a, e in zip(bounds[:-1], bounds[1:])]
    monkeypatch.setattr(eb, "right_windows", no_carry)
    with pytest.raises(AssertionError):
        _pins_right()


def test_planted_lq_of_the_wrong_rows_fails(monkeypatch):
    """Reducing the last instead of the first k rows of the RQ factor does
    not clear the fill."""
    def wrong_rows(C, c):
        import scipy.linalg
        _, Q = scipy.linalg.rq(C)
        Q2, _ = np.linalg.qr(Q[-c:, :].T, mode="complete")
        return Q2
    monkeypatch.setattr(eb, "clear_leading_columns", wrong_rows)
    with pytest.raises(AssertionError):
        _pins_right()


def test_planted_ql_replaced_by_qr_fails(monkeypatch):
    """A QR instead of a QL decomposition of the factor's last k columns does
    not clear the k rows below a block."""
    def qr_instead(C, c):
        w, z = C.shape
        Q, _ = np.linalg.qr(C, mode="complete")
        Q3, _ = np.linalg.qr(Q[:, z:], mode="complete")
        return Q3
    monkeypatch.setattr(eb, "clear_trailing_rows", qr_instead)
    with pytest.raises(AssertionError):
        _pins_left()


def test_planted_bounds_aligned_at_the_top_fail(monkeypatch):
    """Blocks aligned at the top (remainder at the bottom) break the U2
    windows' alignment with the tops of the diagonal blocks of a B built
    with bottom-aligned blocks."""
    true_bounds = eb.block_bounds

    def top_aligned(m, s):
        if m <= s:
            return [0, m]
        return list(range(0, m, s)) + [m]
    rng = np.random.default_rng(3)
    m, s, k = 41, 8, 4
    B, bounds = block_upper(m, s, rng)  # bottom-aligned blocks
    monkeypatch.setattr(eb, "block_bounds", top_aligned)
    B1, _, _, _ = eb.left_pass(B, rng.standard_normal((m, k)), k, s)
    assert true_bounds(m, s) != top_aligned(m, s)
    assert eb.below_blocks_max(B1, bounds) > 1e-3
