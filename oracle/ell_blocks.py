"""Block geometry of the accelerated absorption with l >= 3 blocks (Sec. 3.5,
"Accelerated reduction of V2 and U2"), on dense numpy matrices (test
infrastructure only; nothing here is called by the library).

The trailing m x m part of B is kept block upper triangular with diagonal
blocks of size s = (l - 1) nb aligned at the bottom: [0, p), [p, p + s), ...,
[m - s, m), with 0 < p <= s (a single block [0, m) when m <= s).  One
absorption of k <= nb reflectors then does:

* right side: a QL chain on V2 from the top, one window per diagonal block
  covering the block and the k rows carried from the window above (s + k
  rows, the first window the top block alone), each window's transform
  applied to B from the right; then, from the bottom block up, the RQ
  decomposition of the block's rows over the window's columns and an LQ
  decomposition of the first k rows of its orthogonal factor give k
  reflectors that clear the fill left of the block (the 2nb x 3nb
  construction of Sec. 3.5 for l = 3, k = nb; 2nb x (2nb + k) after a
  refinement failure);
* left side: a QR chain on U2 from the bottom, windows aligned with the tops
  of the diagonal blocks (the bottom block alone first, then each block with
  the k rows carried from below), applied to B from the left; then, from the
  top block down, the QR decomposition of the block's columns over its rows
  and the k rows below it, and a QL decomposition of the last k columns of
  the orthogonal factor, give k reflectors that clear those k rows.

Every function states the passage it follows.  numpy.linalg.qr and
scipy.linalg.rq are the library primitives (complete factors).
"""
import numpy as np
import scipy.linalg


def block_bounds(m, s):
    """Diagonal block boundaries [b_0, b_1, ..., m] of the trailing m x m part,
    aligned at the bottom with stride s (the top block holds the remainder)."""
    if m <= 0:
        return [0]
    if m <= s:
        return [0, m]
    p = m % s or s
    return [0] + list(range(p, m + 1, s))


def below_blocks_max(B, bounds):
    """Largest |entry| of B below its diagonal blocks (0.0 when B is block
    upper triangular with these bounds)."""
    mx = 0.0
    for a, e in zip(bounds[:-1], bounds[1:]):
        if e < B.shape[0]:
            mx = max(mx, float(np.abs(B[e:, a:e]).max(initial=0.0)))
    return mx


def _exchange(n):
    return np.eye(n)[::-1]


def ql(X):
    """Complete QL decomposition X = Q [0; L] (X w x k, w >= k), through the
    QR decomposition of the row- and column-reversed matrix."""
    w, k = X.shape
    Jw, Jk = _exchange(w), _exchange(k)
    Qr, Rr = np.linalg.qr(Jw @ X @ Jk, mode="complete")
    return Jw @ Qr @ Jw, Jw @ Rr @ Jk


def clear_leading_columns(C, c):
    """Right-side block reduction of Sec. 3.5: for C (r x (r + c)), the RQ
    decomposition C = R Q, then the LQ decomposition of the first c rows of Q,
    E1^T Q = [D 0] Qt.  Returns Qt^T (orthogonal, (r+c) x (r+c), a product of c
    reflectors) with (C Qt^T)[:, :c] = 0."""
    r, w = C.shape
    assert w == r + c
    _, Q = scipy.linalg.rq(C)
    M = Q[:c, :]
    # LQ of M through the QR decomposition of M^T: M^T = Q2 R2, M Q2 = R2^T
    Q2, _ = np.linalg.qr(M.T, mode="complete")
    return Q2


def clear_trailing_rows(C, c):
    """Left-side block reduction of Sec. 3.5: for C ((z + c) x z), the QR
    decomposition C = Q [R; 0], then the QL decomposition of the last c
    columns of Q, Q E_last = Q3 [0; L].  Returns Q3 (orthogonal, a product of
    c reflectors) with (Q3^T C)[z:, :] = 0."""
    w, z = C.shape
    assert w == z + c
    Q, _ = np.linalg.qr(C, mode="complete")
    Q3, _ = ql(Q[:, z:])
    return Q3


def right_windows(bounds, k):
    """(start, end, carry) of the QL windows on V2, top to bottom: window t
    covers diagonal block t and the `carry` rows left above it by the window
    before (k, or the whole top block when it has at most k rows)."""
    wins = []
    carry = 0
    for a, e in zip(bounds[:-1], bounds[1:]):
        start = a - carry
        wins.append((start, e, carry))
        carry = min(k, e - start)
    return wins


def left_windows(bounds, k):
    """(start, end, carry) of the QR windows on U2, bottom to top: window t
    covers diagonal block t and the k rows (`carry`) left at the top of the
    window below it."""
    wins = []
    carry = 0
    for a, e in reversed(list(zip(bounds[:-1], bounds[1:]))):
        end = e + carry
        wins.append((a, end, carry))
        carry = min(k, end - a)
    return wins


def right_pass(B, V2, k, s):
    """Right absorption of Sec. 3.5 on the trailing part: reduce V2 (m x k) to
    [0; L1] by the QL windows, apply each window's transform to B from the
    right, then restore B's block upper triangular form from the bottom up.
    Returns (B', V2', Z) with B' = B Z up to the entries set to exact zeros,
    and the number of reflectors of the restoring transforms."""
    B = np.array(B, dtype=np.float64)
    V2 = np.array(V2, dtype=np.float64)
    m = B.shape[0]
    bounds = block_bounds(m, s)
    Z = np.eye(m)
    wins = right_windows(bounds, k)
    for a, e, _ in wins:
        if e - a <= k and a == 0 and e < m:
            continue  # a top block of at most k rows is carried whole
        Qw, Lw = ql(V2[a:e, :])
        V2[a:e, :] = Lw
        B[:, a:e] = B[:, a:e] @ Qw
        Z[:, a:e] = Z[:, a:e] @ Qw
    nrefl = 0
    for (a, e, carry), (ba, be) in reversed(list(zip(wins, zip(bounds[:-1], bounds[1:])))):
        if carry == 0:
            continue
        G = clear_leading_columns(B[ba:be, a:e], carry)
        B[:, a:e] = B[:, a:e] @ G
        Z[:, a:e] = Z[:, a:e] @ G
        B[ba:be, a:ba] = 0.0
        nrefl += carry
    return B, V2, Z, nrefl


def left_pass(B, U2, k, s):
    """Left absorption of Sec. 3.5 on the trailing part: reduce U2 (m x k) to
    [R1; 0] by the QR windows from the bottom, apply each window's transform
    to B from the left, then restore B's block upper triangular form from
    the top down.  Returns (B', U2', Q, nrefl) with B' = Q^T B up to the
    entries set to exact zeros."""
    B = np.array(B, dtype=np.float64)
    U2 = np.array(U2, dtype=np.float64)
    m = B.shape[0]
    bounds = block_bounds(m, s)
    Q = np.eye(m)
    for a, e, _ in left_windows(bounds, k):
        Qw, Rw = np.linalg.qr(U2[a:e, :], mode="complete")
        U2[a:e, :] = Rw
        B[a:e, :] = Qw.T @ B[a:e, :]
        Q[:, a:e] = Q[:, a:e] @ Qw
    nrefl = 0
    for a, e in zip(bounds[:-1], bounds[1:]):
        if e >= m:
            break
        c = min(k, m - e)
        G = clear_trailing_rows(B[a:e + c, a:e], c)
        B[a:e + c, :] = G.T @ B[a:e + c, :]
        Q[:, a:e + c] = Q[:, a:e + c] @ G
        B[e:e + c, a:e] = 0.0
        nrefl += c
    return B, U2, Q, nrefl


def block_solve(B, bounds, c):
    """Block back substitution of Sec. 3.5 (impact on Algorithm 1): x with
    B x = c for block upper triangular B, from the bottom block up, each
    diagonal block solved through its LU decomposition with partial
    pivoting."""
    x = np.zeros(B.shape[0])
    for a, e in reversed(list(zip(bounds[:-1], bounds[1:]))):
        P, L, U = scipy.linalg.lu(B[a:e, a:e])
        rhs = c[a:e] - B[a:e, e:] @ x[e:]
        y = scipy.linalg.solve_triangular(L, P.T @ rhs, lower=True, unit_diagonal=True)
        x[a:e] = scipy.linalg.solve_triangular(U, y, lower=False)
    return x
