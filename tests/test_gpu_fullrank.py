"""GPU: the certified full-rank path of the rank step (unpivoted blocked
Cholesky, certificate lambda = 1 / max_j (M^-1)_jj), against the FP64 CPU
oracle's greedy pivoted Cholesky.  The order threshold is lowered so that
small problems take the path.  Covered: ragged last blocks (300 = 2 x 128 +
44, 1000 = 7 x 128 + 104, single rows at 129 and 1153), one block (128),
look-ahead updates on a second stream (1300, 1153), the
N < L route, duplicated nodes (bitwise-equal Gram rows: set aside, the
distinct nodes certified; the greedy rule with the path off), duplicated
samples on the N < L route,
dependent columns with no repeated value (the unpivoted factorisation stops
and the greedy rule runs), distinct columns with equal norms (certified), a
threshold the certificate cannot clear (the greedy rule runs, full rank) and
the default order threshold on both sides."""
import numpy as np
import pytest
import torch

import elm_workloads as wl
import oracle as O

from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -53


@pytest.fixture(scope="module")
def elm():
    from paper_2011_02436_amd import elm as mod
    return mod


@pytest.fixture
def low_threshold(elm):
    old = elm.set_option("full_rank_min_order", 1)
    yield
    elm.set_option("full_rank_min_order", old)


def _dev(p):
    return to_dev(p.X), to_dev(p.W), to_dev(p.b), to_dev(p.T)


def _reference(p):
    H = O.hidden(p.X, p.W, p.b)
    M = H.T @ H if p.N >= p.L else H @ H.T
    K = p.N if p.N >= p.L else p.L
    R, piv, r = O.pivoted_cholesky(M, K=K)
    beta, F = O.solve(H, p.T)
    assert F.r == r
    lam = 1.0 / np.linalg.inv(M).diagonal().max() if r == M.shape[0] else 0.0
    s = np.linalg.svd(H[:, F.piv[:r]] if p.N >= p.L else H[F.piv[:r], :], compute_uv=False)
    return beta, r, R[r - 1, r - 1] ** 2, lam, (s[0] / s[-1]) ** 2


# 1300 = three groups of 512 block rows: the second stream's look-ahead
# update (rows beyond the next group) runs once.  Single-row last blocks
# (129 = 128 + 1, 1153 = 9 x 128 + 1) and exactly one block (128) exercise the
# diagonal-block kernel's padding (its inverse's identity rows).
FULL = [(6000, 64, 300, 50), (8000, 128, 1000, 52), (4000, 16, 300, 53), (500, 64, 1200, 55),
        (9000, 128, 1300, 56), (3000, 32, 129, 57), (9000, 128, 1153, 58), (2000, 32, 128, 59)]


@pytest.mark.parametrize("shape", FULL, ids=[f"N{s[0]}_L{s[2]}" for s in FULL])
@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_certified_full_rank_matches_oracle(elm, low_threshold, shape, precision):
    N, d, L, seed = shape
    p = wl.random_problem(seed, N, d, L, 3)
    beta_ref, r, last_greedy, lam, k2 = _reference(p)
    res = elm.train(*_dev(p), precision=precision, ir_tol=1e-12 if precision == "fp64" else 1e-10)
    fi = res.info["factor"]
    print(f"N={N} L={L} {precision}: certified {fi['certified_full_rank']} rank {res.rank} (oracle {r}); "
          f"lambda {fi['last_pivot']:.6e} (oracle 1/max(M^-1)_jj {lam:.6e}, last greedy pivot "
          f"{last_greedy:.6e}); tau {fi['tau']:.3e}")
    assert fi["certified_full_rank"] and fi["reliable"]
    assert res.rank == r == min(N, L)
    assert fi["first_rejected"] == -np.inf
    # the certificate is the exact leave-one-out bound, below the greedy rule's last pivot
    if precision == "fp64":
        assert abs(fi["last_pivot"] - lam) <= 1e-8 * lam
    else:  # the BF16 Gram's own bound: within the Gram's rounding of the FP64 one
        assert abs(fi["last_pivot"] - lam) <= 0.05 * lam
    assert fi["last_pivot"] <= last_greedy * (1 + 1e-8) or precision != "fp64"
    assert fi["last_pivot"] >= 64 * fi["tau"]
    err = O.rel_err(res.beta.cpu().numpy(), beta_ref)
    tol = 1e-10 if precision == "fp64" else 1e-6
    print(f"beta err {err:.2e} (bar {tol:.0e}; kappa^2 eps {k2 * EPS:.1e})")
    assert err <= tol, (err, tol)


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_duplicated_nodes_set_aside_then_certified(elm, low_threshold, precision):
    # equal columns give bitwise-equal Gram rows: the copies are set aside,
    # the distinct nodes certified (mode 2), with the oracle's rank, last
    # greedy pivot and beta; the order is the distinct nodes, then the copies
    p = wl.random_problem(54, 3000, 64, 700, 3, n_dup=70)
    beta_ref, r, last, _, k2 = _reference(p)
    res = elm.train(*_dev(p), precision=precision, ir_tol=1e-12)
    fi = res.info["factor"]
    assert fi["certified_full_rank"] == 2
    assert res.rank == r == p.structural_rank == 630
    assert fi["first_rejected"] == 0.0
    if precision == "fp64":
        assert abs(fi["last_pivot"] - last) <= 1e-8 * last
    piv = res.factor.pivots()
    assert sorted(piv.tolist()) == list(range(p.L))
    keep, rest = piv[:r], piv[r:]
    assert np.all(np.diff(keep) > 0) and np.all(np.diff(rest) > 0)
    assert len(set(p.groups[keep])) == r                   # one node per group
    assert set(p.groups[rest]) <= set(p.groups[keep])      # the rest are copies
    err = O.rel_err(res.beta.cpu().numpy(), beta_ref)
    bar = 1e-10 if precision == "fp64" else 1e-6
    print(f"{precision}: beta err {err:.2e} (bar {bar:.0e}; kappa^2 eps {k2 * EPS:.1e})")
    assert err <= bar


def test_duplicated_nodes_greedy_rule_when_disabled(elm):
    # the same problem with the certified path off: the greedy rule, the same
    # rank and beta
    old = elm.set_option("full_rank_min_order", 0)
    try:
        p = wl.random_problem(54, 3000, 64, 700, 3, n_dup=70)
        beta_ref, r, _, _, _ = _reference(p)
        res = elm.train(*_dev(p), precision="fp64", ir_tol=1e-12)
        assert res.info["factor"]["certified_full_rank"] == 0
        assert res.rank == r == 630
        assert O.rel_err(res.beta.cpu().numpy(), beta_ref) <= 1e-10
    finally:
        elm.set_option("full_rank_min_order", old)


def test_threshold_above_certificate_falls_back_to_greedy(elm, low_threshold):
    # tau_rel = 1e-3: 64 tau is above lambda (~2e-2 of the largest diagonal),
    # so nothing is certified; the greedy rule still keeps every position
    p = wl.random_problem(50, 6000, 64, 300, 3)
    res = elm.train(*_dev(p), precision="fp64", ir_tol=1e-12, tau_rel=1e-3)
    fi = res.info["factor"]
    H = O.hidden(p.X, p.W, p.b)
    _, _, r = O.pivoted_cholesky(H.T @ H, tau=fi["tau"])
    assert not fi["certified_full_rank"]
    assert res.rank == r == 300


def test_default_threshold_keeps_small_grams_on_the_greedy_path(elm):
    assert elm.get_option("full_rank_min_order") == 64
    p = wl.random_problem(50, 6000, 64, 48, 3)
    res = elm.train(*_dev(p), precision="fp64", ir_tol=1e-12)
    assert not res.info["factor"]["certified_full_rank"]
    assert res.rank == 48


def test_default_threshold_certifies_full_rank_grams(elm):
    p = wl.random_problem(50, 6000, 64, 300, 3)
    beta_ref, r, _, lam, _ = _reference(p)
    res = elm.train(*_dev(p), precision="fp64", ir_tol=1e-12)
    fi = res.info["factor"]
    assert fi["certified_full_rank"]
    assert res.rank == r == 300
    assert abs(fi["last_pivot"] - lam) <= 1e-8 * lam
    assert O.rel_err(res.beta.cpu().numpy(), beta_ref) <= 1e-10


def test_dependent_columns_without_repeats_stop_the_certificate(elm):
    # columns that are mixtures of two others (no repeated Gram diagonal
    # value): the unpivoted factorisation meets a pivot below its bound, stops,
    # and the greedy rule finds the oracle's rank
    rng = np.random.default_rng(61)
    p = wl.random_problem(61, 3000, 64, 700, 3)
    H = O.hidden(p.X, p.W, p.b)
    dep = rng.choice(np.arange(100, 700), size=35, replace=False)
    src = np.setdiff1d(np.arange(700), dep)
    for j in dep:
        a, b_ = rng.choice(src, size=2, replace=False)
        w = rng.uniform(0.2, 0.8)
        H[:, j] = w * H[:, a] + (1.0 - w) * H[:, b_]
    M = H.T @ H
    assert np.unique(M.diagonal()).size == 700
    _, _, r = O.pivoted_cholesky(M, K=3000)
    assert r == 665
    f = elm.elm_rank_factor(torch.from_numpy(H).to("cuda:0"))
    fi = f.info()
    assert not fi["certified_full_rank"]
    assert f.rank == r


def test_equal_norms_without_duplicates_are_certified(elm):
    # two pairs of distinct columns with bitwise-equal norms (integer entries:
    # every sum is exact, so reversing a column keeps its norm): equal Gram
    # diagonal values alone do not send a Gram to the greedy rule
    rng = np.random.default_rng(62)
    H = rng.integers(-8, 9, size=(2000, 300)).astype(np.float64)
    H[:, 1] = H[::-1, 0]
    H[:, 7] = H[::-1, 3]
    M = H.T @ H
    assert M[1, 1] == M[0, 0] and M[7, 7] == M[3, 3] and M[0, 1] != M[0, 0]
    f = elm.elm_rank_factor(torch.from_numpy(H).to("cuda:0"))
    assert f.info()["certified_full_rank"]
    assert f.rank == np.linalg.matrix_rank(H) == 300


def test_duplicated_samples_on_the_transposed_route(elm):
    # N < L (the Gram H H^T): 60 of 600 samples repeat others, so 60 rows of
    # H and of the Gram repeat: set aside, the 540 distinct samples certified,
    # with the oracle's rank and beta
    rng = np.random.default_rng(63)
    p = wl.random_problem(63, 600, 32, 900, 3)
    X = p.X.copy()
    rows = rng.choice(600, size=60, replace=False)
    X[rows] = X[rng.choice(np.setdiff1d(np.arange(600), rows), size=60)]
    H = O.hidden(X, p.W, p.b)
    beta_ref, F = O.solve(H, p.T)
    assert F.r == len(np.unique(X, axis=0)) == 540
    res = elm.train(to_dev(X), to_dev(p.W), to_dev(p.b), to_dev(p.T), precision="fp64", ir_tol=1e-12)
    fi = res.info["factor"]
    assert fi["transposed"] and fi["certified_full_rank"] == 2
    assert res.rank == 540
    err = O.rel_err(res.beta.cpu().numpy(), beta_ref)
    print(f"beta err {err:.2e} (bar 1e-10)")
    assert err <= 1e-10
