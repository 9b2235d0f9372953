"""GPU: the paper's own block form of the solve (Section 3, eqs. 19-23,
elm_block_solve) against the FP64 oracle.

For a hidden matrix of full column rank the block elimination reaches the
unique least-squares solution beta = H^+ T (eq. 5), so every split point and
every column order must give the oracle's beta (rank-based route, FP64) to the
FP64 bar, 1e-10 relative.  The CPU suite pins that reading of eqs. 19-23 (the
transpose on H1 restored) on the oracle itself.  Cases: splits at 1, in the
middle, at L - 1 and at L (H2 empty); both factorisations of A and D (one
workgroup up to order 128, the blocked Cholesky above); a permuted column
order; the Gram passed in or formed by the call; the digits-like workload at
full size (N=60000, d=784, L=2000) against its stored oracle result; and a
rank-deficient H, where A or D is singular and the call must say so.
"""
import os

import numpy as np
import pytest
import torch

import elm_workloads as wl
import oracle as O

from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def elm():
    from paper_2011_02436_amd import elm as mod
    return mod


def _hidden(elm, p):
    X, W, b = to_dev(p.X), to_dev(p.W), to_dev(p.b)
    H = torch.empty((p.N, p.L), dtype=torch.float64, device=X.device)
    elm.elm_hidden(X, W, b, H=H)
    return H


@pytest.mark.parametrize("N,d,L,m,splits", [
    (3000, 16, 300, 3, (1, 100, 299, 300)),
    (2000, 12, 129, 2, (128, 1)),
    (5000, 20, 257, 5, (100, 200, 129)),
])
def test_block_solve_matches_oracle(elm, N, d, L, m, splits):
    p = wl.random_problem(seed=N + L, N=N, d=d, L=L, m=m)
    Hh = O.hidden(p.X, p.W, p.b)
    ref, F = O.solve(Hh, p.T)
    assert F.r == L                      # full column rank
    H = _hidden(elm, p)
    T = to_dev(p.T)
    M = elm.elm_gram(H, "sample")
    for split in splits:
        for gram_in in (True, False):
            beta = elm.elm_block_solve(H, T, split, M=M if gram_in else None)
            err = O.rel_err(beta.cpu().numpy(), ref)
            print(f"N={N} L={L} split {split} (A {L - split}, D {split}), Gram passed {gram_in}: "
                  f"err vs oracle {err:.2e} (bar 1e-10)")
            assert err <= 1e-10


def test_block_solve_permuted_columns(elm):
    # H P = [H1 H2] for a random order P: beta comes back in original order
    p = wl.random_problem(seed=41, N=4000, d=10, L=240, m=4)
    ref, F = O.solve(O.hidden(p.X, p.W, p.b), p.T)
    assert F.r == p.L
    H = _hidden(elm, p)
    perm = np.random.default_rng(5).permutation(p.L).astype(np.int32)
    piv = torch.from_numpy(perm).to(H.device)
    for split in (60, 180):
        beta = elm.elm_block_solve(H, to_dev(p.T), split, piv=piv)
        err = O.rel_err(beta.cpu().numpy(), ref)
        print(f"permuted order, split {split}: err {err:.2e}")
        assert err <= 1e-10


def test_block_solve_full_size_digits(elm):
    """N=60000, d=784 (80% zeros), L=2000, m=10, full rank: the block form at
    three split points against the oracle's stored beta (kappa_r ~ 204, so
    kappa_r^2 eps ~ 5e-12 leaves the 1e-10 bar meaningful)."""
    p = wl.digits_like()
    with np.load(os.path.join(GOLDEN, "fullsize_digits_like.npz")) as z:
        ref, rank = z["beta"], int(z["rank"])
    assert rank == p.L
    H = _hidden(elm, p)
    T = to_dev(p.T)
    M = elm.elm_gram(H, "sample")
    for split in (500, 1000, 1999):
        beta = elm.elm_block_solve(H, T, split, M=M)
        err = O.rel_err(beta.cpu().numpy(), ref)
        print(f"digits_like full size, split {split}: err vs oracle {err:.2e} (bar 1e-10)")
        assert err <= 1e-10


def test_block_solve_rejects_rank_deficient(elm):
    # duplicated nodes: H2 repeats a column of H1 (D singular) or of itself
    # (A singular); the block form has no solution and the call says so
    p = wl.random_problem(seed=8, N=1500, d=8, L=100, m=2, n_dup=10)
    H = _hidden(elm, p)
    with pytest.raises(elm.ElmError) as ei:
        elm.elm_block_solve(H, to_dev(p.T), 50)
    assert ei.value.status == 5    # ELM_ERR_NOT_PSD
