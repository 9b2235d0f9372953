"""GPU: the training without a stored H (elm_train_streamed), against the
FP64 oracle.

The streamed form forms the hidden matrix chunk by chunk, sums the chunks'
Grams and H^T T in chunk order, and forms each chunk again for every
refinement residual; it must reach the oracle's rank exactly and beta within
the form's bar (1e-10 FP64, 1e-6 for the low-precision Grams with FP64
refinement).  Cases: a ragged last chunk, chunks shorter than L, one chunk, a
target width past the hidden layer's fused H^T T (m = 17), duplicated nodes
(rank-deficient), and the regression workload at full size (N=500000,
L=10000) in the BF16 form against its stored oracle result.
"""
import os

import numpy as np
import pytest
import torch

import elm_workloads as wl
import oracle as O
from oracle import validators as V

from gpu_helpers import check_fp64_beta, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def elm():
    from paper_2011_02436_amd import elm as mod
    return mod


def _dev(p):
    return to_dev(p.X), to_dev(p.W), to_dev(p.b), to_dev(p.T)


@pytest.mark.parametrize("N,d,L,m,n_dup,chunk", [
    (30011, 16, 600, 3, 60, 7000),     # ragged last chunk (2011 rows)
    (5000, 24, 700, 2, 0, 512),        # chunks shorter than L
    (8000, 20, 300, 17, 30, 8000),     # one chunk; H^T T by the column pass
])
@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_streamed_matches_oracle(elm, N, d, L, m, n_dup, chunk, precision):
    p = wl.random_problem(seed=N + L + m, N=N, d=d, L=L, m=m, n_dup=n_dup)
    H = O.hidden(p.X, p.W, p.b)
    ref, F = O.solve(H, p.T)
    res = elm.train_streamed(*_dev(p), precision=precision, chunk_rows=chunk, ir_tol=1e-10)
    got = res.beta.cpu().numpy()
    print(f"streamed {precision} N={N} L={L} m={m} chunk {chunk}: rank {res.rank} (oracle {F.r}), "
          f"gram {res.info['gram_dtype']}, NE {res.info['ne_residual']:.1e}, corrections {res.info['iterations']}")
    assert res.rank == F.r == p.structural_rank
    assert res.info["ne_residual"] <= 1e-10
    if res.info["gram_dtype"] == "fp64":
        sv = np.linalg.svd(H[:, F.piv[:F.r]], compute_uv=False)
        check_fp64_beta(f"streamed {precision}", got, ref, V.dedup_closed_form(H, p.T, p.groups),
                        sv[0] / sv[-1])
    else:
        err = O.rel_err(got, ref)
        print(f"  beta err vs oracle {err:.2e} (bar 1e-6)")
        assert err <= 1e-6


def test_streamed_full_size_precision_form(elm):
    """N=500000, d=128, L=10000, m=4 in the BF16 form with 65536-row chunks:
    H (40 GB in FP64) is never stored; beta against the oracle's stored one."""
    p = wl.smooth_regression()
    with np.load(os.path.join(GOLDEN, "fullsize_smooth_regression.npz")) as z:
        ref, rank = z["beta"], int(z["rank"])
    torch.cuda.reset_peak_memory_stats()
    res = elm.train_streamed(*_dev(p), precision="bf16", chunk_rows=65536, ir_tol=1e-10)
    torch.cuda.synchronize()
    err = O.rel_err(res.beta.cpu().numpy(), ref)
    print(f"streamed C4 bf16: rank {res.rank} (oracle {rank}), gram {res.info['gram_dtype']}, "
          f"NE {res.info['ne_residual']:.1e}, corrections {res.info['iterations']}, beta err {err:.2e} (bar 1e-6)")
    assert res.rank == rank == 10000
    assert res.info["gram_dtype"] == "bf16"
    assert res.info["ne_residual"] <= 1e-10
    assert err <= 1e-6
