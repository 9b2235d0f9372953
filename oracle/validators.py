"""Independent checks used to pin the oracle (test infrastructure only).

Each routine here reaches a quantity the oracle also computes by a different
route, so that a mistake in the oracle's rank step or pseudoinverse assembly
shows up as a mismatch.
"""
from __future__ import annotations

import numpy as np


def penrose_residuals(A: np.ndarray, X: np.ndarray):
    """Relative residuals of the four Penrose conditions that define X = A^+:
    A X A = A, X A X = X, (A X)^T = A X, (X A)^T = X A."""
    AX = A @ X
    XA = X @ A
    na, nx = np.linalg.norm(A), np.linalg.norm(X)
    return (
        float(np.linalg.norm(AX @ A - A) / na),
        float(np.linalg.norm(XA @ X - X) / nx),
        float(np.linalg.norm(AX.T - AX) / np.linalg.norm(AX)),
        float(np.linalg.norm(XA.T - XA) / np.linalg.norm(XA)),
    )


def dedup_closed_form(H: np.ndarray, T: np.ndarray, groups: np.ndarray) -> np.ndarray:
    """Minimum-norm least-squares solution when H = H_u E, where H_u holds the
    distinct columns and E (n_u x L) is the 0/1 membership matrix
    (E[g, j] = 1 iff column j is a copy of distinct column g).

    With D = diag(multiplicities), H = (H_u D^{1/2}) (D^{-1/2} E) and the rows
    of D^{-1/2} E are orthonormal, so H^+ = E^T D^{-1/2} (H_u D^{1/2})^+.  The
    inner pseudoinverse is taken by an SVD of the N x n_u matrix (no Gram is
    formed), which is accurate to ~cond * eps rather than cond^2 * eps.
    """
    groups = np.asarray(groups)
    n_u = int(groups.max()) + 1
    first = np.full(n_u, -1)
    for j, g in enumerate(groups):
        if first[g] < 0:
            first[g] = j
    Hu = H[:, first]
    mult = np.bincount(groups, minlength=n_u).astype(np.float64)
    sq = np.sqrt(mult)
    U, s, Vt = np.linalg.svd(Hu * sq[None, :], full_matrices=False)
    cut = s[0] * max(Hu.shape) * 2.0 ** -52
    r = int(np.count_nonzero(s > cut))
    inner = Vt[:r].T @ ((U[:, :r].T @ T) / s[:r, None])      # (Hu D^1/2)^+ T
    return (inner / sq[:, None])[groups]


def prescribed_svd_matrix(rng: np.random.Generator, N: int, L: int, svals: np.ndarray):
    """H = U diag(svals) V^T with random orthonormal U (N x k), V (L x k);
    returns (H, H^+) with H^+ = V diag(1/s for s > 0) U^T exactly known."""
    k = svals.size
    U, _ = np.linalg.qr(rng.standard_normal((N, k)))
    V, _ = np.linalg.qr(rng.standard_normal((L, k)))
    H = (U * svals[None, :]) @ V.T
    inv = np.where(svals > 0, 1.0 / np.where(svals > 0, svals, 1.0), 0.0)
    Hp = (V * inv[None, :]) @ U.T
    return H, Hp
