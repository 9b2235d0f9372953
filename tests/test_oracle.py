"""Pins for the FP64 oracle (CPU only).

Every check reaches the oracle's result by a route that is not the oracle's
own: the SVD definition of the pseudoinverse, the Penrose conditions, closed
forms, LAPACK, scipy's logistic function, hand-derived values, and the
paper's own block formulas on a full-column-rank case.  A few tests plant a
mistake in a copy of the oracle and show that the pins catch it.
"""
import math
import os

import numpy as np
import pytest
from scipy.linalg import lapack
from scipy.special import expit

import elm_workloads as wl
import oracle as O
from oracle import validators as V

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# hidden layer (eq. 1 / eq. 4, sigmoid)
# --------------------------------------------------------------------------
def test_sigmoid_matches_scipy_expit_and_special_values():
    z = np.concatenate([np.linspace(-50, 50, 2001), [-800.0, -40.0, 0.0, 40.0, 800.0]])
    # within 2 ulp of scipy's logistic function over the whole range
    assert np.all(np.abs(O.sigmoid(z) - expit(z)) <= 2 * np.spacing(expit(z)))
    assert O.sigmoid(np.array([0.0]))[0] == 0.5
    assert abs(O.sigmoid(np.array([math.log(3.0)]))[0] - 0.75) <= 1e-16
    # symmetry g(-z) = 1 - g(z)
    zz = np.linspace(-20, 20, 101)
    assert np.max(np.abs(O.sigmoid(-zz) - (1 - O.sigmoid(zz)))) <= 2 * np.spacing(1.0)


def test_hidden_closed_forms():
    rng = np.random.default_rng(0)
    N, d, L = 7, 5, 6
    W = rng.uniform(-1, 1, (d, L))
    b = rng.uniform(0, 1, L)
    # W = 0: every row equals g(b)
    H = O.hidden(rng.standard_normal((N, d)), np.zeros((d, L)), b)
    assert np.all(np.abs(H - expit(b)[None, :]) <= 2 * np.spacing(1.0))
    # unit-vector samples pick one row of W: H[i, j] = g(W[i, j] + b[j])
    H = O.hidden(np.eye(d), W, b)
    assert np.all(np.abs(H - expit(W + b[None, :])) <= 2 * np.spacing(1.0))
    # a shape check: samples are rows, hidden nodes are columns
    assert O.hidden(rng.standard_normal((N, d)), W, b).shape == (N, L)


# --------------------------------------------------------------------------
# rank step (eq. 6, algorithm steps 3-4)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L,k", [(40, 40), (60, 23), (120, 97)])
def test_pivoted_cholesky_matches_lapack_dpstrf(L, k):
    rng = np.random.default_rng(L)
    B = rng.standard_normal((L + 10, k)) @ rng.standard_normal((k, L))   # rank k
    M = B.T @ B
    tau = O.default_tau(M)
    R, piv, r = O.pivoted_cholesky(M, tau)
    # dpstrf's tol is an absolute threshold on the remaining diagonal
    c, p, rk, info = lapack.dpstrf(M, lower=0, tol=tau)
    assert r == k == rk
    assert np.array_equal(piv[:r], p[:r] - 1)
    assert np.max(np.abs(R[:, :r] - np.triu(c)[:r, :r])) <= 1e-10 * np.max(np.abs(R))
    # the factor reproduces the permuted Gram
    Mp = M[np.ix_(piv, piv)]
    assert np.max(np.abs(R.T @ R - Mp)) <= 1e-12 * np.max(np.abs(M))


def test_rank_threshold_on_generically_rank_deficient_h_ht():
    # N < L with fewer distinct nodes (385) than samples (399): H H^T is
    # rank-deficient without any duplicated rows, so its rejected Schur
    # diagonals are rounding noise of the Gram (about K u max diag, K = L
    # products per entry) rather than exact zeros.  The threshold must sit
    # above that noise: the rank equals the SVD's and the structural rank,
    # and the solution satisfies the normal equations.
    p = wl.random_problem(seed=138, N=399, d=32, L=443, m=3, n_dup=58)
    H = O.hidden(p.X, p.W, p.b)
    M = H @ H.T
    s = np.linalg.svd(H, compute_uv=False)
    F = O.rank_factor(H)
    assert F.transposed
    assert F.r == p.structural_rank == 385 == int(np.sum(s > 1e-10 * s[0]))
    beta, _ = O.solve(H, p.T)
    assert O.ne_residual(H, p.T, beta) <= 1e-10
    assert O.rel_err(beta, np.linalg.pinv(H, rcond=1e-10) @ p.T) <= 1e-8
    # LAPACK's default n u max diag lies below the noise here and keeps a
    # noise pivot (why the threshold scales with K as well)
    _, _, r_lapack = O.pivoted_cholesky(M, tau=H.shape[0] * 2.0 ** -53 * M.diagonal().max())
    assert r_lapack > 385


def test_pivot_tie_break_lowest_original_index():
    # all diagonals equal and orthogonal columns: every step is a tie
    M = np.diag([3.0, 3.0, 3.0, 3.0])
    _, piv, r = O.pivoted_cholesky(M)
    assert r == 4 and list(piv) == [0, 1, 2, 3]
    # duplicated column 2 == column 0 (bitwise) and a larger column 3
    H = np.array([[1.0, 0.0, 1.0, 2.0], [0.0, 1.0, 0.0, 0.0], [1.0, 1.0, 1.0, 0.0]])
    _, piv, r = O.pivoted_cholesky(H.T @ H)
    assert r == 3 and piv[0] == 3


def test_structural_rank_of_duplicated_nodes():
    p = wl.tiny_fp64()
    H = O.hidden(p.X, p.W, p.b)
    F = O.rank_factor(H)
    assert F.r == p.structural_rank == 160
    assert O.solve_svd(H, p.T)[1] == 160
    # each rejected column is a bitwise copy of an accepted one
    acc = set(p.groups[F.piv[:F.r]])
    assert len(acc) == 160 and set(p.groups[F.piv[F.r:]]) <= acc


def test_K_is_selection_matrix_for_duplicates():
    p = wl.tiny_fp64()
    F = O.rank_factor(O.hidden(p.X, p.W, p.b))
    assert np.max(np.abs(F.K - np.round(F.K))) <= 1e-12
    assert np.array_equal(np.round(F.K).sum(axis=0), np.ones(F.K.shape[1]))


# --------------------------------------------------------------------------
# beta = H^+ T (eq. 5) against the SVD definition and the Penrose conditions
# --------------------------------------------------------------------------
def test_tiny_config_matches_svd_and_dedup_closed_form():
    p = wl.tiny_fp64()
    H = O.hidden(p.X, p.W, p.b)
    beta, F = O.solve(H, p.T)
    ref, rs = O.solve_svd(H, p.T)
    assert F.r == rs == 160
    assert O.rel_err(beta, ref) <= 1e-11
    assert O.rel_err(beta, V.dedup_closed_form(H, p.T, p.groups)) <= 1e-11
    # exact copies get exactly shared weight: beta is constant within a group
    for g in np.unique(p.groups):
        cols = np.flatnonzero(p.groups == g)
        assert np.max(np.abs(beta[cols] - beta[cols[0]])) <= 1e-12 * np.max(np.abs(beta))


@pytest.mark.parametrize("N,L,n_dup", [(300, 80, 0), (300, 80, 17), (60, 140, 0), (60, 140, 30), (97, 97, 9)])
def test_random_shapes_match_svd(N, L, n_dup):
    p = wl.random_problem(seed=N * 1000 + L + n_dup, N=N, d=16, L=L, m=3, n_dup=n_dup)
    H = O.hidden(p.X, p.W, p.b)
    beta, F = O.solve(H, p.T)
    ref, rs = O.solve_svd(H, p.T)
    assert F.r == rs
    assert F.transposed == (N < L)
    assert O.rel_err(beta, ref) <= 1e-10


def test_penrose_conditions_on_explicit_pinv():
    for (N, L, nd) in [(200, 50, 10), (40, 90, 0), (40, 90, 20)]:
        p = wl.random_problem(seed=N + L + nd, N=N, d=16, L=L, m=2, n_dup=nd)
        H = O.hidden(p.X, p.W, p.b)
        F = O.rank_factor(H)
        Hp = O.apply_pinv(F, H, np.eye(N))          # H^+ applied to I_N
        res = V.penrose_residuals(H, Hp)
        assert max(res) <= 1e-9, res


def test_prescribed_singular_values_exact_pinv():
    rng = np.random.default_rng(11)
    N, L = 120, 40
    s = np.concatenate([np.linspace(3.0, 0.5, 25), np.zeros(15)])
    H, Hp_exact = V.prescribed_svd_matrix(rng, N, L, np.concatenate([s, np.zeros(0)]))
    T = rng.standard_normal((N, 3))
    beta, F = O.solve(H, T)
    assert F.r == 25
    assert O.rel_err(beta, Hp_exact @ T) <= 1e-12


def test_golden_hand_derived_pinv():
    txt = open(os.path.join(GOLDEN, "dup_column_pinv.txt")).read().split("\n")
    rows = [ln for ln in txt if ln and not ln.startswith("#")]
    i = rows.index("H")
    j = rows.index("HPINV_TIMES_6")
    k = rows.index("RANK")
    H = np.array([[float(v) for v in ln.split()] for ln in rows[i + 1:j]])
    Hp6 = np.array([[float(v) for v in ln.split()] for ln in rows[j + 1:k]])
    rank = int(rows[k + 1])
    F = O.rank_factor(H)
    assert F.r == rank
    Hp = O.apply_pinv(F, H, np.eye(H.shape[0]))
    assert np.max(np.abs(6.0 * Hp - Hp6)) <= 1e-13


def test_zero_matrix_rank_zero_beta_zero():
    H = np.zeros((10, 4))
    beta, F = O.solve(H, np.ones((10, 2)))
    assert F.r == 0 and np.all(beta == 0)
    H = np.zeros((3, 8))
    beta, F = O.solve(H, np.ones((3, 2)))
    assert F.r == 0 and np.all(beta == 0) and beta.shape == (8, 2)


def test_w_zero_closed_forms():
    rng = np.random.default_rng(5)
    N, d, L, m = 50, 3, 12, 4
    X = rng.standard_normal((N, d))
    T = rng.standard_normal((N, m))
    b = rng.uniform(0, 1, L)
    H = O.hidden(X, np.zeros((d, L)), b)          # H = 1 g(b)^T, rank 1
    # columns are exact multiples (not bitwise copies) of one another, so the
    # Gram's rounding noise (~N eps) sits above the L eps default threshold;
    # any threshold inside the gap [noise, smallest true pivot] gives rank 1
    tau = 1e-10 * np.max(np.sum(H * H, axis=0))
    beta, F = O.solve(H, T, tau=tau)
    s = expit(b)
    assert F.r == 1
    assert O.rel_err(beta, np.outer(s, T.mean(axis=0)) / (s @ s)) <= 1e-13
    H0 = O.hidden(X, np.zeros((d, L)), np.zeros(L))   # H = 0.5 everywhere
    beta0, F0 = O.solve(H0, T, tau=tau)
    assert F0.r == 1
    assert O.rel_err(beta0, np.broadcast_to(2.0 * T.mean(axis=0) / L, (L, m))) <= 1e-14


def test_minimum_norm_differs_from_basic_solution():
    # dropping the (G G^T)^-1 step gives a least-squares solution that is not
    # the minimum-norm one: it must differ from H^+ T on a rank-deficient H
    p = wl.tiny_fp64()
    H = O.hidden(p.X, p.W, p.b)
    F = O.rank_factor(H)
    Z = H.T @ p.T
    y = F._gram_f_solve(Z[F.piv[:F.r]])
    basic = np.zeros_like(Z)
    basic[F.piv[:F.r]] = y
    beta = O.apply_pinv(F, H, p.T)
    assert O.ne_residual(H, p.T, basic) <= 1e-9             # still a LS solution
    assert O.rel_err(basic, beta) >= 0.1
    assert np.linalg.norm(beta) < np.linalg.norm(basic)


def test_paper_block_formulas_equal_oracle_on_full_column_rank():
    """eqs. (19)-(23) with the transpose on H1 restored: for a full-column-rank
    H split into any [H1 H2], the block-elimination result equals H^+ Y."""
    p = wl.random_problem(seed=21, N=150, d=5, L=30, m=3)
    H = O.hidden(p.X, p.W, p.b)
    Y = p.T
    for r in (10, 22):
        H1, H2 = H[:, :r], H[:, r:]
        A = H2.T @ H2                                   # eq. (20)
        B = np.linalg.solve(A, H2.T @ Y)                # eq. (21)
        C = np.eye(H.shape[0]) - H2 @ np.linalg.solve(A, H2.T)   # eq. (22)
        D = H1.T @ C @ H1                               # eq. (23)
        b1 = np.linalg.solve(D, H1.T @ (Y - H2 @ B))    # eq. (19), top
        b2 = B - np.linalg.solve(A, H2.T @ H1 @ b1)     # eq. (19), bottom
        beta_block = np.vstack([b1, b2])                # eq. (7)
        beta, F = O.solve(H, Y)
        assert F.r == 30
        assert O.rel_err(beta_block, beta) <= 1e-9


def test_refinement_reduces_normal_equation_residual():
    p = wl.random_problem(seed=3, N=800, d=8, L=120, m=3, n_dup=12)
    H = O.hidden(p.X, p.W, p.b)
    b0, _ = O.solve(H, p.T, refine_steps=0)
    b2, _ = O.solve(H, p.T, refine_steps=2)
    ref, _ = O.solve_svd(H, p.T)
    assert O.rel_err(b2, ref) <= O.rel_err(b0, ref) + 1e-15
    assert O.ne_residual(H, p.T, b2) <= 1e-13


def test_streamed_train_equals_in_memory_train():
    p = wl.tiny_fp64()
    b1, r1 = O.train(p.X, p.W, p.b, p.T)
    b2, r2 = O.train(p.X, p.W, p.b, p.T, chunk_rows=300)
    assert r1 == r2 == 160
    assert O.rel_err(b2, b1) <= 1e-12
    H = O.hidden(p.X, p.W, p.b)
    assert abs(O.ne_residual_streamed(p.X, p.W, p.b, p.T, b2, 300) - O.ne_residual(H, p.T, b2)) <= 1e-15


def test_predict_labels_hand_checked():
    # tiny hand case: H = g(0) = 0.5 everywhere, beta columns give outputs
    X = np.zeros((3, 2))
    W = np.zeros((2, 2))
    b = np.zeros(2)
    beta = np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 2.0]])   # outputs [1, 1, 1]: tie
    Y, lab = O.predict(X, W, b, beta)
    assert np.array_equal(Y, np.ones((3, 3)))
    assert list(lab) == [0, 0, 0]                         # lowest index on ties
    beta2 = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 1.0]])   # outputs [0, 0, 1]
    assert list(O.predict(X, W, b, beta2)[1]) == [2, 2, 2]


# --------------------------------------------------------------------------
# planted mistakes: a wrong oracle must fail the pins above
# --------------------------------------------------------------------------
def _planted_apply(kind):
    def apply(F, H, rhs, Z=None):
        if Z is None:
            Z = H.T @ rhs
        L, m = Z.shape
        y = F._gram_f_solve(Z[F.piv[:F.r]])
        u = F._gram_g_solve(y)
        if kind == "no_K_term":
            bp = np.vstack([u, np.zeros((L - F.r, m))])
        elif kind == "transposed_K":
            Kt = np.zeros((L - F.r, F.r))
            Kt[:min(L - F.r, F.r), :min(L - F.r, F.r)] = F.K[:min(L - F.r, F.r), :min(L - F.r, F.r)]
            bp = np.vstack([u, Kt @ u])
        elif kind == "unpermuted":
            return np.vstack([u, F.K.T @ u])
        beta = np.zeros((L, m))
        beta[F.piv] = bp
        return beta
    return apply


@pytest.mark.parametrize("kind", ["no_K_term", "transposed_K", "unpermuted"])
def test_planted_mistakes_are_caught(kind):
    p = wl.tiny_fp64()
    H = O.hidden(p.X, p.W, p.b)
    F = O.rank_factor(H)
    wrong = _planted_apply(kind)(F, H, p.T)
    ref, _ = O.solve_svd(H, p.T)
    assert O.rel_err(wrong, ref) > 1e-3


def test_planted_wrong_tau_changes_rank():
    # a threshold far above the pivot gap (rule misread as relative 1e-2)
    # drops genuine directions; the structural-rank pin catches it
    p = wl.tiny_fp64()
    H = O.hidden(p.X, p.W, p.b)
    M = H.T @ H
    _, _, r = O.pivoted_cholesky(M, tau=1e-2 * np.max(np.diag(M)))
    assert r != p.structural_rank


def test_greedy_pivots_bounded_by_inverse_diagonal():
    """The certified full-rank path rests on two facts about the greedy
    diagonally pivoted Cholesky (Section 3's rank step): its pivots never
    increase, and its last pivot is the Schur complement of the last index
    with respect to all others, 1 / (M^-1)_jj; so every pivot is at least
    1 / max_j (M^-1)_jj."""
    for seed, (N, d, L) in enumerate([(400, 8, 60), (900, 32, 120), (300, 4, 40)]):
        p = wl.random_problem(700 + seed, N, d, L, 2)
        H = O.hidden(p.X, p.W, p.b)
        M = H.T @ H
        R, piv, r = O.pivoted_cholesky(M, tau=0.0)
        assert r == L
        pivots = np.diag(R) ** 2
        assert np.all(np.diff(pivots) <= 1e-12 * pivots[0])
        Minv = np.linalg.inv(M)
        assert abs(pivots[-1] * Minv[piv[-1], piv[-1]] - 1.0) <= 1e-6
        lam = 1.0 / Minv.diagonal().max()
        assert pivots.min() >= lam * (1 - 1e-6)
