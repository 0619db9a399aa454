"""CPU reference of the steps around the HT reduction (test infrastructure).

* ``triangularize_b``: the first step of the QZ algorithm (Sec. 1): B is
  brought to upper triangular form by an orthogonal transformation from the
  left, B = Q0 R, which is applied to A as well (A <- Q0^T A).  numpy's
  Householder QR is the library primitive.
* ``preprocess``: the zero-column preprocessing of Sec. 3.5 (Preprocessing):
  when B has l > 1 zero columns, a permutation Z0 moves them to the front
  (Q0 = Z0 when B is diagonal, so that B stays diagonal, else Q0 = I); the
  QR factorisation of the first l columns of A0 = Q0^T A Z0 gives Q1 with
  A1 = (Q0 Q1)^T A Z0 = [A11 A12; 0 A22] (A11 upper triangular) and
  B1 = (Q0 Q1)^T B Z0 = [0 B12; 0 B22].  The leading l x l part is then in
  generalised Schur form and only (A22, B22) remains to be reduced; B22 is
  made triangular again first (``triangularize_b`` on the trailing pencil),
  since the HT reduction starts from a triangular B.
* ``preprocessed_ht``: preprocessing followed by the O(n^3) oracle (O-fast)
  on the trailing pencil, assembled into the reduction of the whole pencil:
  H = Q^T A Z upper Hessenberg, T = Q^T B Z upper triangular, with the
  first l columns of T zero.

Only ``tests/`` may use this module.  It shares no code with the HIP path.
"""
import numpy as np

from .core import fast_ht


def triangularize_b(A, B):
    """QZ step 1: returns (Q0^T A, R, Q0) with B = Q0 R, R upper triangular."""
    Q0, R = np.linalg.qr(np.asarray(B, dtype=np.float64), mode="complete")
    return Q0.T @ A, np.triu(R), Q0


def zero_columns(B):
    """Indices of the columns of B that are exactly zero."""
    return [j for j in range(B.shape[1]) if not np.any(B[:, j])]


def preprocess(A, B):
    """Returns (A1, B1, Q, Z, l): A1 = Q^T A Z, B1 = Q^T B Z with the first l
    columns of B1 zero, A1(:, :l) upper triangular (exact zeros below), and
    B1(l:, l:) upper triangular.  With fewer than two zero columns nothing is
    done (l = 0, Q = Z = I), as the paper preprocesses only l > 1."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    n = A.shape[0]
    zc = zero_columns(B)
    ell = len(zc)
    eye = np.eye(n)
    if ell <= 1:
        return A.copy(), np.triu(B), eye.copy(), eye.copy(), 0
    rest = [j for j in range(n) if j not in set(zc)]
    perm = zc + rest
    Z0 = eye[:, perm]
    diagonal = not np.any(B - np.diag(np.diag(B)))
    Q0 = Z0 if diagonal else eye
    A0 = Q0.T @ A @ Z0
    B0 = Q0.T @ B @ Z0
    Q1, _ = np.linalg.qr(A0[:, :ell], mode="complete")
    A1 = Q1.T @ A0
    B1 = Q1.T @ B0
    A1[:, :ell] = np.triu(A1[:, :ell])  # below A11: rounding noise of the QR
    B1[:, :ell] = 0.0                   # Q1^T applied to zero columns
    A22, R2, Q2 = triangularize_b(A1[ell:, ell:], B1[ell:, ell:])
    A1[ell:, ell:] = A22
    B1[ell:, ell:] = R2
    Q = Q0 @ Q1
    Q[:, ell:] = Q[:, ell:] @ Q2
    return A1, B1, Q, Z0.copy(), ell


def preprocessed_ht(A, B, threads=0):
    """Preprocessing, then O-fast on the trailing pencil; returns
    (H, T, Q, Z, l) for the whole pencil."""
    A1, B1, Q, Z, ell = preprocess(A, B)
    if A1.shape[0] - ell <= 0:
        return A1, B1, Q, Z, ell
    H22, T22, Q22, Z22, _ = fast_ht(A1[ell:, ell:], B1[ell:, ell:], threads=threads)
    H, T = A1.copy(), B1.copy()
    H[:ell, ell:] = A1[:ell, ell:] @ Z22
    T[:ell, ell:] = B1[:ell, ell:] @ Z22
    H[ell:, ell:] = H22
    T[ell:, ell:] = T22
    Q[:, ell:] = Q[:, ell:] @ Q22
    Z[:, ell:] = Z[:, ell:] @ Z22
    return H, T, Q, Z, ell
