"""FP64 CPU oracle for the rank-based pseudoinverse ELM training path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls this module:
it is imported only by the tests, by the smoke check and by the CPU-baseline
leg of the benchmark.  It shares no code with the HIP path; the only common
dependency is the seeded input generator module, which holds none of the
method's arithmetic.

Everything here is plain NumPy/SciPy in float64, written for a reader to check
against Ragala & Kumar, "Rank Based Pseudoinverse Computation in Extreme
Learning Machine for large Datasets" (arXiv 2011.02436):

* hidden layer            Section 2.1, eq. (1) and eq. (4); step 2 of the
                          RBP-ELM algorithm; sigmoid activation (Section 4)
* least-squares problem   eq. (3); beta = H^+ Y, eq. (5)
* normal equations        eq. (8), N >= L; the N < L form H^T (H H^T)^-1
                          stated just before eq. (8)
* permutation and rank    Section 3, eq. (6) and steps 3-4 of the algorithm
* beta split              eq. (7); step 9 of the algorithm

Readings (the paper leaves these open; each is listed in the design notes):

* The permutation P and rank r come from a greedy diagonally pivoted Cholesky
  of the Gram H^T H (H H^T when N < L; largest remaining Schur diagonal
  first, lowest original index on exact ties), stopped when the largest
  remaining diagonal is <= tau = 16 (n + K) 2^-53 max_j M_jj, n the order of
  the Gram and K the number of products summed into each entry.  (The LAPACK
  xPSTRF default n 2^-53 max M_jj sits below the Gram's own rounding when
  K > n: on H H^T with N < L and fewer distinct nodes than samples it accepted
  noise pivots on 11 of 40 random draws; see default_tau.)
* With H P = [H1 H2] and r = rank(H), H2 = H1 K for K = R11^-1 R12, so
  H = F G with F = H1 (full column rank) and G = [I K] P^T (full row rank),
  and H^+ = G^T (G G^T)^-1 (F^T F)^-1 F^T with F^T F = R11^T R11 and
  G G^T = I + K K^T.  The block formulas of eqs. (19)-(23) need H1 and H2 to
  be linearly independent of each other, which fails exactly when r < L, so
  this full-rank-factorisation form is the one taken for the rank-deficient
  case; it gives the same beta as eq. (8) whenever H has full column rank.
* Two FP64 iterative-refinement steps beta += H^+ (T - H beta) are applied,
  which removes rounding error amplified by forming the Gram.

Parity pins (tests/test_oracle.py): the SVD pseudoinverse (definition of the
Moore-Penrose inverse), the four Penrose conditions, the structural rank of
duplicated nodes, the closed form for duplicated columns, closed forms for
W = 0, matrices with prescribed singular values, LAPACK dpstrf rank and pivot
order at a given threshold, the rank of a generically rank-deficient H H^T
against its SVD, and scipy's logistic function.
"""
from __future__ import annotations

import math
import time
from typing import Dict, Optional

import numpy as np
from scipy.linalg import solve_triangular, cho_factor, cho_solve

EPS53 = 2.0 ** -53  # unit roundoff of IEEE binary64 (LAPACK's DLAMCH('E'))


# ----------------------------------------------------------------------------
# Hidden layer: H[i, j] = g(w_j . x_i + b_j), g = logistic sigmoid.
# Section 2.1, eq. (1) (the per-sample model) and eq. (4) (the N x L matrix,
# samples as rows); the activation is the sigmoid named in Section 4.
# ----------------------------------------------------------------------------
def sigmoid(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(-z))


def hidden(X: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """N x L hidden-layer matrix, float64."""
    X = np.asarray(X, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return sigmoid(X @ W + b[None, :])


# ----------------------------------------------------------------------------
# Gram and right-hand side of the normal equations, eq. (8):
# beta = (H^T H)^-1 H^T Y.  For N < L the text before eq. (8) gives
# H^+ = H^T (H H^T)^-1, whose Gram is H H^T.
# ----------------------------------------------------------------------------
def gram(H: np.ndarray, T: Optional[np.ndarray] = None):
    M = H.T @ H
    Z = None if T is None else H.T @ T
    return M, Z


def gram_streamed(X, W, b, T, chunk_rows: int = 16384):
    """H^T H and H^T T accumulated over row chunks of H (the same sums as
    `gram`, only grouped by rows so that H never has to be held whole)."""
    L = W.shape[1]
    M = np.zeros((L, L))
    Z = np.zeros((L, T.shape[1]))
    for s in range(0, X.shape[0], chunk_rows):
        Hc = hidden(X[s:s + chunk_rows], W, b)
        M += Hc.T @ Hc
        Z += Hc.T @ T[s:s + chunk_rows]
    return M, Z


# ----------------------------------------------------------------------------
# Permutation P and rank r (Section 3, eq. (6); algorithm steps 3-4):
# greedy diagonally pivoted Cholesky  P^T M P ~= R^T R,  R = [R11 R12], r x L.
# ----------------------------------------------------------------------------
def default_tau(M: np.ndarray, K: Optional[int] = None) -> float:
    """Stopping threshold of the rank step (the paper leaves it open):
    tau = 16 (n + K) 2^-53 max_j M_jj, n the order of M and K the number of
    products summed into each entry (samples for H^T H, nodes for H H^T; n
    when not given).  Every entry of a Gram of the positive sigmoid matrix
    carries up to K u of its size in rounding, so a direction that is
    dependent in exact arithmetic keeps a Schur diagonal of about K u max M_jj
    (measured: 1.1 K u on H H^T with N < L); LAPACK's default n u sits below
    that when K > n and then accepts noise pivots."""
    n = M.shape[0]
    if K is None:
        K = n
    return 16.0 * (n + K) * EPS53 * (float(np.max(np.diag(M))) if n else 0.0)


def pivoted_cholesky(M: np.ndarray, tau: Optional[float] = None, K: Optional[int] = None):
    """Rank-revealing Cholesky with complete (diagonal) pivoting.

    Returns (R, piv, r): R is r x L upper trapezoidal in pivoted order, piv
    the original column index at each pivoted position, r the rank.  At step k
    the pivot is the remaining column with the largest Schur-complement
    diagonal (lowest original index on an exact tie); the factorisation stops
    when that diagonal is <= tau (default_tau(M, K) when tau is None).
    """
    M = np.asarray(M, dtype=np.float64)
    L = M.shape[0]
    A = M.copy()
    piv = np.arange(L)
    d = np.diag(A).copy()
    R = np.zeros((L, L))
    if tau is None:
        tau = default_tau(M, K)
    r = L
    for k in range(L):
        rest = d[k:]
        best = rest.max()
        if not best > tau:
            r = k
            break
        ties = k + np.flatnonzero(rest == best)
        j = int(ties[np.argmin(piv[ties])])
        if j != k:
            piv[[k, j]] = piv[[j, k]]
            d[[k, j]] = d[[j, k]]
            A[[k, j], :] = A[[j, k], :]
            A[:, [k, j]] = A[:, [j, k]]
            R[:k, [k, j]] = R[:k, [j, k]]
        rkk = math.sqrt(d[k])
        R[k, k] = rkk
        if k + 1 < L:
            R[k, k + 1:] = (A[k, k + 1:] - R[:k, k] @ R[:k, k + 1:]) / rkk
            d[k + 1:] -= R[k, k + 1:] ** 2
    return R[:r].copy(), piv, r


# ----------------------------------------------------------------------------
# Full-rank factorisation H P = H1 [I K] and its pseudoinverse.
# ----------------------------------------------------------------------------
class Factor:
    """Result of the rank step for one Gram (H^T H, or H H^T when N < L)."""

    def __init__(self, R: np.ndarray, piv: np.ndarray, r: int, transposed: bool):
        self.piv = piv
        self.r = r
        self.transposed = transposed
        self.R11 = R[:, :r]
        self.R12 = R[:, r:]
        # K = R11^-1 R12, so that the dependent block is H2 = H1 K
        self.K = solve_triangular(self.R11, self.R12) if r > 0 else np.zeros((0, R.shape[1]))
        # G G^T = I + K K^T (r x r), factored once
        S = np.eye(r) + self.K @ self.K.T
        self.S_chol = cho_factor(S) if r > 0 else None

    def _gram_f_solve(self, Y):
        """(F^T F)^-1 Y = (R11^T R11)^-1 Y."""
        return solve_triangular(self.R11, solve_triangular(self.R11, Y, trans="T"))

    def _gram_g_solve(self, Y):
        """(G G^T)^-1 Y = (I + K K^T)^-1 Y."""
        return cho_solve(self.S_chol, Y)


def rank_factor(H: np.ndarray, tau: Optional[float] = None, M: Optional[np.ndarray] = None) -> Factor:
    """Rank step on H: pivoted Cholesky of H^T H when N >= L, of H H^T when
    N < L (the two branches stated before eq. (8))."""
    N, L = H.shape
    transposed = N < L
    if M is None:
        M = H @ H.T if transposed else H.T @ H
    R, piv, r = pivoted_cholesky(M, tau, K=L if transposed else N)
    return Factor(R, piv, r, transposed)


def apply_pinv(F: Factor, H: Optional[np.ndarray], rhs: np.ndarray, Z: Optional[np.ndarray] = None):
    """beta = H^+ rhs through the factorisation.

    N >= L (F built from H^T H):  H = F G with F = H1, G = [I K] P^T,
      H^+ rhs = G^T (G G^T)^-1 (R11^T R11)^-1 H1^T rhs,  H1^T rhs = (H^T rhs)[piv[:r]].
      `Z` may pass H^T rhs directly.
    N < L (F built from H H^T): H^T = F' G' with F' = H[piv[:r], :]^T,
      H^+ rhs = F' (R11^T R11)^-1 (I + K K^T)^-1 (rhs[piv[:r]] + K rhs[piv[r:]]).
    """
    r, piv = F.r, F.piv
    if not F.transposed:
        if Z is None:
            Z = H.T @ rhs
        L, m = Z.shape
        beta = np.zeros((L, m))
        if r == 0:
            return beta
        y = F._gram_f_solve(Z[piv[:r]])
        u = F._gram_g_solve(y)
        beta_perm = np.vstack([u, F.K.T @ u])          # eq. (7) block order
        beta[piv] = beta_perm
        return beta
    N, L = H.shape
    m = rhs.shape[1]
    if r == 0:
        return np.zeros((L, m))
    w = rhs[piv[:r]] + F.K @ rhs[piv[r:]]
    u = F._gram_g_solve(w)
    y = F._gram_f_solve(u)
    return H[piv[:r], :].T @ y


def solve(H: np.ndarray, T: np.ndarray, refine_steps: int = 2, tau: Optional[float] = None):
    """beta = H^+ T (eq. 5) by the rank-based route, plus FP64 refinement.
    Returns (beta, factor)."""
    H = np.asarray(H, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    F = rank_factor(H, tau)
    beta = apply_pinv(F, H, T)
    for _ in range(refine_steps):
        beta = beta + apply_pinv(F, H, T - H @ beta)
    return beta, F


def train(X, W, b, T, refine_steps: int = 2, tau: Optional[float] = None,
          chunk_rows: Optional[int] = None, timings: Optional[Dict[str, float]] = None):
    """Whole ELM training (algorithm steps 1-9 after the random weights are
    drawn): H, rank step, beta.  With `chunk_rows` the N >= L Gram and the
    refinement residuals are accumulated over row chunks (H recomputed per
    chunk), for problems whose H does not fit in host memory.

    Returns (beta, rank).  `timings`, if given, receives wall seconds split
    into 'rows' (work proportional to N: hidden layer, Gram, refinement
    residuals) and 'factor' (work independent of N: rank step and solves).
    """
    t = timings if timings is not None else {}
    t.setdefault("rows", 0.0)
    t.setdefault("factor", 0.0)
    N, L = X.shape[0], W.shape[1]
    if chunk_rows is None or N < L:
        t0 = time.perf_counter()
        H = hidden(X, W, b)
        transposed = N < L
        M = H @ H.T if transposed else H.T @ H
        Z = None if transposed else H.T @ T
        t1 = time.perf_counter()
        F = rank_factor(H, tau, M=M)
        beta = apply_pinv(F, H, T, Z=Z)
        t2 = time.perf_counter()
        t["rows"] += t1 - t0
        t["factor"] += t2 - t1
        for _ in range(refine_steps):
            t0 = time.perf_counter()
            E = T - H @ beta
            g = None if transposed else H.T @ E
            t1 = time.perf_counter()
            beta = beta + apply_pinv(F, H, E, Z=g)
            t["rows"] += t1 - t0
            t["factor"] += time.perf_counter() - t1
        return beta, F.r
    t0 = time.perf_counter()
    M, Z = gram_streamed(X, W, b, T, chunk_rows)
    t1 = time.perf_counter()
    F = rank_factor(ShapeOnly(N, L), tau, M=M)
    beta = apply_pinv(F, None, None, Z=Z)
    t2 = time.perf_counter()
    t["rows"] += t1 - t0
    t["factor"] += t2 - t1
    for _ in range(refine_steps):
        t0 = time.perf_counter()
        g = ne_gradient_streamed(X, W, b, T, beta, chunk_rows)
        t1 = time.perf_counter()
        beta = beta + apply_pinv(F, None, None, Z=g)
        t["rows"] += t1 - t0
        t["factor"] += time.perf_counter() - t1
    return beta, F.r


class ShapeOnly:
    """Stand-in carrying only the shape of H (streamed N >= L route)."""

    def __init__(self, N, L):
        self.shape = (N, L)


def ne_gradient_streamed(X, W, b, T, beta, chunk_rows: int = 16384):
    """H^T (T - H beta) accumulated over row chunks."""
    g = np.zeros_like(beta)
    for s in range(0, X.shape[0], chunk_rows):
        Hc = hidden(X[s:s + chunk_rows], W, b)
        g += Hc.T @ (T[s:s + chunk_rows] - Hc @ beta)
    return g


# ----------------------------------------------------------------------------
# The definition itself: Moore-Penrose pseudoinverse by SVD (eq. 5; the paper
# names SVD as the accurate reference method in Section 1).
# ----------------------------------------------------------------------------
def svd_rank_cutoff(s: np.ndarray, shape) -> float:
    return (s[0] if s.size else 0.0) * max(shape) * 2.0 ** -52


def pinv_svd(H: np.ndarray, rcond: Optional[float] = None):
    """(H^+, r) from the thin SVD H = U S V^T: H^+ = V S^+ U^T, keeping the
    singular values above s_max * max(N, L) * 2^-52 (or rcond * s_max)."""
    H = np.asarray(H, dtype=np.float64)
    U, s, Vt = np.linalg.svd(H, full_matrices=False)
    cut = svd_rank_cutoff(s, H.shape) if rcond is None else rcond * (s[0] if s.size else 0.0)
    r = int(np.count_nonzero(s > cut))
    Hp = (Vt[:r].T / s[:r]) @ U[:, :r].T
    return Hp, r


def solve_svd(H: np.ndarray, T: np.ndarray, rcond: Optional[float] = None):
    """beta = H^+ T with H^+ from the SVD, applied without forming H^+."""
    H = np.asarray(H, dtype=np.float64)
    U, s, Vt = np.linalg.svd(H, full_matrices=False)
    cut = svd_rank_cutoff(s, H.shape) if rcond is None else rcond * (s[0] if s.size else 0.0)
    r = int(np.count_nonzero(s > cut))
    beta = Vt[:r].T @ ((U[:, :r].T @ T) / s[:r, None])
    return beta, r


# ----------------------------------------------------------------------------
# Prediction (step 3 of the three-step ELM) and the metrics used beside it.
# ----------------------------------------------------------------------------
def predict(X, W, b, beta):
    """Y = H beta and the arg-max label of each row (lowest index on ties)."""
    Y = hidden(X, W, b) @ beta
    return Y, np.argmax(Y, axis=1)


def training_accuracy(X, W, b, beta, labels) -> float:
    """Share of training samples whose arg-max output is their class (Table 2)."""
    _, lab = predict(X, W, b, beta)
    return float(np.mean(lab == labels))


def ne_residual(H, T, beta) -> float:
    """||H^T (T - H beta)||_F / ||H^T T||_F in float64."""
    num = np.linalg.norm(H.T @ (T - H @ beta))
    den = np.linalg.norm(H.T @ T)
    return float(num / den) if den > 0 else float(num)


def ne_residual_streamed(X, W, b, T, beta, chunk_rows: int = 16384) -> float:
    g = ne_gradient_streamed(X, W, b, T, beta, chunk_rows)
    z = np.zeros_like(beta)
    for s in range(0, X.shape[0], chunk_rows):
        z += hidden(X[s:s + chunk_rows], W, b).T @ T[s:s + chunk_rows]
    den = np.linalg.norm(z)
    return float(np.linalg.norm(g) / den) if den > 0 else float(np.linalg.norm(g))


def rel_err(a, ref) -> float:
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(np.asarray(a) - ref) / den) if den > 0 else float(np.linalg.norm(a))
