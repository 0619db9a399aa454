"""Comparison helpers for HT reductions (test infrastructure only).

An HT reduction H = Q^T A Z, T = Q^T B Z with Q e1 = e1 is unique up to
H' = D_Q H D_Z, T' = D_Q T D_Z (D_Q, D_Z diagonal with entries +-1) when B is
nonsingular and H T^{-1} is unreduced: Q spans the Krylov sequence of
A B^{-1} started at e1 (implicit-Q theorem) and Z follows from the RQ
factorisation of Q^T B.  ``sign_normalise`` fixes D_Q, D_Z so that
diag(T') >= 0 and subdiag(H') >= 0; two correct reductions then agree
entry by entry up to rounding.

The invariants are those the paper checks (structure and the residuals
||H - Q^T A Z||, ||T - Q^T B Z||, Sec. 4) and the bounds of Theorem A.1 and
its corollary (backward error O(u)||A||_F, orthogonality O(u)).

Functions accept numpy arrays or torch tensors (dense products run on the
arrays' device); they never modify their inputs.
"""
import numpy as np


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _fro(X):
    if _is_torch(X):
        import torch
        return float(torch.linalg.norm(X))
    return float(np.linalg.norm(X))


def _sgn(x):
    return 1.0 if x >= 0 else -1.0


def sign_vectors(H, T, upto=None):
    """d_q (length c+1) and d_z (length c+1) of the normalisation, c = upto.

    d_q[0] = +1; d_z[i] = d_q[i] sgn(T_ii); d_q[i+1] = d_z[i] sgn(H_{i+1,i}),
    sgn(0) = +1.  With upto = c only the first c columns of H are used.
    """
    n = H.shape[0]
    if upto is None:
        upto = n - 1
    c = max(0, min(upto, n - 1))
    Hd = np.asarray(H[1:c + 1, :c].diagonal().cpu() if _is_torch(H) else np.diag(H[1:c + 1, :c]))
    Td = np.asarray(T[:c + 1, :c + 1].diagonal().cpu() if _is_torch(T) else np.diag(T[:c + 1, :c + 1]))
    dq = np.ones(c + 1)
    dz = np.ones(c + 1)
    for i in range(c + 1):
        dz[i] = dq[i] * _sgn(Td[i])
        if i < c:
            dq[i + 1] = dz[i] * _sgn(Hd[i])
    return dq, dz


def sign_normalise(H, T, Q, Z, upto=None):
    """Return (H', T', Q', Z') restricted to the columns that are final after
    `upto` reduced columns: H[:, :c], T[:, :c+1], Q[:, :c+1], Z[:, :c+1]
    (the full matrices when upto is None).  Rows of H' and T' are limited to
    0..c for the partial case (all of them are final there)."""
    n = H.shape[0]
    full = upto is None or upto >= n - 1
    dq, dz = sign_vectors(H, T, upto)
    c = len(dq) - 1
    if _is_torch(H):
        import torch
        dqt = torch.as_tensor(dq, dtype=H.dtype, device=H.device)
        dzt = torch.as_tensor(dz, dtype=H.dtype, device=H.device)
    else:
        dqt, dzt = dq, dz
    if full:
        Hn = dqt[:, None] * H * dzt[None, :]
        Tn = dqt[:, None] * T * dzt[None, :]
        return Hn, Tn, Q * dqt[None, :], Z * dzt[None, :]
    Hn = dqt[:c + 1, None] * H[:c + 1, :c] * dzt[None, :c]
    Tn = dqt[:c + 1, None] * T[:c + 1, :c + 1] * dzt[None, :c + 1]
    return Hn, Tn, Q[:, :c + 1] * dqt[None, :], Z[:, :c + 1] * dzt[None, :]


def compare(ref, got, A0, B0, upto=None):
    """Sign-normalised entrywise comparison of two reductions.

    ref, got: tuples (H, T, Q, Z).  Returns a dict of
    max|dH|/||A||_F, max|dT|/||B||_F, max|dQ|/sqrt(n), max|dZ|/sqrt(n) and
    the Frobenius counterparts.
    """
    n = A0.shape[0]
    r = sign_normalise(*ref, upto=upto)
    g = sign_normalise(*got, upto=upto)
    nA, nB, sq = _fro(A0), _fro(B0), float(np.sqrt(max(n, 1)))
    out = {}
    for name, a, b, scale in (("H", r[0], g[0], nA), ("T", r[1], g[1], nB),
                              ("Q", r[2], g[2], sq), ("Z", r[3], g[3], sq)):
        d = a - b
        if _is_torch(d):
            mx = float(d.abs().max()) if d.numel() else 0.0
        else:
            mx = float(np.abs(d).max()) if d.size else 0.0
        out["max_" + name] = mx / max(scale, 1e-300)
        out["fro_" + name] = _fro(d) / max(scale, 1e-300)
    return out


def sign_normalise_ilo(H, T, Q, Z, ell):
    """Sign normalisation of a reduction whose first `ell` columns were
    fixed by the zero-column preprocessing (Z's first ell columns are
    permutation columns, so d_z = +1 there; Q's come from a QR
    factorisation, fixed by diag(H) >= 0 there).  Column ell starts the
    trailing reduction: d_z = +1 (Z e_ell is a permutation column too) and
    d_q from T(ell, ell) >= 0; from there on the rule of sign_vectors.
    Numpy arrays only; returns (H', T', Q', Z')."""
    n = H.shape[0]
    dq = np.ones(n)
    dz = np.ones(n)
    for i in range(min(ell, n)):
        dq[i] = _sgn(H[i, i])
    if ell < n:
        dq[ell] = _sgn(T[ell, ell])
        for i in range(ell, n):
            dz[i] = dq[i] * _sgn(T[i, i])
            if i + 1 < n:
                dq[i + 1] = dz[i] * _sgn(H[i + 1, i])
    return dq[:, None] * H * dz[None, :], dq[:, None] * T * dz[None, :], Q * dq[None, :], \
        Z * dz[None, :]


def compare_ilo(ref, got, A0, B0, ell):
    """compare() for reductions that start after `ell` preprocessed columns
    (sign_normalise_ilo instead of sign_normalise)."""
    n = A0.shape[0]
    r = sign_normalise_ilo(*ref, ell)
    g = sign_normalise_ilo(*got, ell)
    nA, nB, sq = _fro(A0), _fro(B0), float(np.sqrt(max(n, 1)))
    out = {}
    for name, a, b, scale in (("H", r[0], g[0], nA), ("T", r[1], g[1], nB),
                              ("Q", r[2], g[2], sq), ("Z", r[3], g[3], sq)):
        d = a - b
        out["max_" + name] = (float(np.abs(d).max()) if d.size else 0.0) / max(scale, 1e-300)
        out["fro_" + name] = _fro(d) / max(scale, 1e-300)
    return out


def structure_violations(H, T):
    """Number of nonzero entries below H's subdiagonal and below T's diagonal
    (both must be exact zeros)."""
    if _is_torch(H):
        import torch
        return int((torch.tril(H, -2) != 0).sum()), int((torch.tril(T, -1) != 0).sum())
    return int(np.count_nonzero(np.tril(H, -2))), int(np.count_nonzero(np.tril(T, -1)))


def invariants(A0, B0, H, T, Q, Z):
    """Structure, orthogonality and backward errors of a reduction.

    Returns dict with keys zeros_H, zeros_T (violation counts), orth_Q, orth_Z
    (||X^T X - I||_F), bwd_A (||Q H Z^T - A||_F / ||A||_F), bwd_B, and the
    first-row/column exactness of Q and Z (Q e1 = e1, Z e1 = e1).
    """
    n = A0.shape[0]
    zH, zT = structure_violations(H, T)
    if _is_torch(H):
        import torch
        I = torch.eye(n, dtype=H.dtype, device=H.device)
        e1_Q = bool((Q[:, 0] == I[:, 0]).all() and (Q[0, :] == I[0, :]).all()) if n else True
        e1_Z = bool((Z[:, 0] == I[:, 0]).all() and (Z[0, :] == I[0, :]).all()) if n else True
    else:
        I = np.eye(n)
        e1_Q = bool(np.array_equal(Q[:, 0], I[:, 0]) and np.array_equal(Q[0, :], I[0, :])) if n else True
        e1_Z = bool(np.array_equal(Z[:, 0], I[:, 0]) and np.array_equal(Z[0, :], I[0, :])) if n else True
    nA, nB = _fro(A0), _fro(B0)
    return {
        "zeros_H": zH,
        "zeros_T": zT,
        "orth_Q": _fro(Q.T @ Q - I),
        "orth_Z": _fro(Z.T @ Z - I),
        "bwd_A": _fro(Q @ H @ Z.T - A0) / max(nA, 1e-300),
        "bwd_B": _fro(Q @ T @ Z.T - B0) / max(nB, 1e-300),
        "e1_Q": e1_Q,
        "e1_Z": e1_Z,
    }


def invariants_ok(inv, n):
    """The acceptance thresholds: exact zeros, ||X^T X - I||_F <= 1e-13 n,
    backward errors <= 1e-14 n (Theorem A.1 with a concrete constant)."""
    n = max(n, 1)
    return (inv["zeros_H"] == 0 and inv["zeros_T"] == 0
            and inv["orth_Q"] <= 1e-13 * n and inv["orth_Z"] <= 1e-13 * n
            and inv["bwd_A"] <= 1e-14 * n and inv["bwd_B"] <= 1e-14 * n
            and inv["e1_Q"] and inv["e1_Z"])


def krylov_reference(A, B):
    """HT reduction straight from its characterisation, for tiny n only.

    Q is the orthonormal basis of the Krylov sequence e1, M e1, M^2 e1, ...
    of M = A B^{-1} (so Q^T M Q is Hessenberg and Q e1 = e1), Z comes from
    the RQ factorisation Q^T B = T Z^T, and H = Q^T A Z.  The Krylov matrix
    is badly conditioned, so this is meaningful only for n <= ~6.
    """
    import scipy.linalg as sl
    n = A.shape[0]
    M = A @ np.linalg.inv(B)
    K = np.zeros((n, n))
    v = np.zeros(n)
    v[0] = 1.0
    for i in range(n):
        K[:, i] = v
        v = M @ v
    Q, _ = np.linalg.qr(K)
    T, Zt = sl.rq(Q.T @ B)
    Z = Zt.T
    H = Q.T @ A @ Z
    return H, T, Q, Z
