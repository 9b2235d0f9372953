"""GPU: the autotuners' table (elm_tune_table_*) and the batch autotuner
(elm_autotune_batch).

The table changes tile schedules only: a batch trained after tuning must
still equal the single trainings bit for bit (both take the tuned panel
width and Gram splits) and match the FP64 oracle (rank exactly, beta within
the form's bar).  The table round-trips through its text file, and
malformed rows are refused.
"""
import os

import numpy as np
import pytest
import torch

import elm_workloads as wl
import oracle as O

from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def elm():
    from paper_2011_02436_amd import elm as mod
    return mod


@pytest.fixture(autouse=True)
def greedy_singles(elm):
    """The batch takes the greedy rank rule at every order; the single
    trainings compared with it bit for bit take that rule too."""
    old = elm.set_option("full_rank_min_order", 0)
    yield
    elm.set_option("full_rank_min_order", old)


@pytest.fixture()
def clean_table(elm):
    saved = elm.tune_table()
    elm.tune_table_set([])
    yield
    elm.tune_table_set(saved)


def _dev(p):
    return to_dev(p.X), to_dev(p.W), to_dev(p.b), to_dev(p.T)


def test_table_round_trip(elm, clean_table, tmp_path):
    rows = [{"kind": "panel", "dtype": "any", "n_log2": -1, "k_log2": -1, "value": 128},
            {"kind": "gram_splits", "dtype": "bf16", "n_log2": 14, "k_log2": 19, "value": 24},
            {"kind": "gram_chunks", "dtype": "fp64", "n_log2": 10, "k_log2": 13, "value": 5}]
    elm.tune_table_set(rows)
    assert elm.tune_table() == rows
    path = str(tmp_path / "tune.txt")
    elm.tune_table_save(path)
    elm.tune_table_set([])
    assert elm.tune_table() == []
    elm.tune_table_load(path)
    assert elm.tune_table() == rows
    with pytest.raises(elm.ElmError):
        elm.tune_table_set([{"kind": "panel", "dtype": "any", "n_log2": -1, "k_log2": -1, "value": 48}])
    bad = tmp_path / "bad.txt"
    bad.write_text("3 -1 -1 -1 64\n1 2 14\n")
    with pytest.raises(elm.ElmError):
        elm.tune_table_load(str(bad))
    assert elm.tune_table() == rows   # a refused file leaves the table as it was


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_autotuned_batch_matches_single_and_oracle(elm, clean_table, precision):
    shapes = [(3000, 700, 70), (2500, 530, 53), (1500, 300, 30), (4000, 1100, 110), (800, 1000, 100)]
    probs = [wl.random_problem(90 + i, N, 16, L, 3, n_dup=k) for i, (N, L, k) in enumerate(shapes)]
    dev = [_dev(p) for p in probs]
    before, after = elm.autotune_batch(dev, precision=precision, ir_tol=1e-12)
    table = elm.tune_table()
    print(f"{precision}: batch {before:.2f} ms -> {after:.2f} ms, table {table}")
    assert after <= before
    betas, infos, stats = elm.train_batched(dev, precision=precision, ir_tol=1e-12, check=False)
    for e, (p, (X, W, b, T)) in enumerate(zip(probs, dev)):
        one = elm.train(X, W, b, T, precision=precision, ir_tol=1e-12, check_convergence=False)
        assert torch.equal(one.beta, betas[e]), e
        ref, F = O.solve(O.hidden(p.X, p.W, p.b), p.T)
        err = O.rel_err(betas[e].cpu().numpy(), ref)
        print(f"  [{e}] N={p.N} L={p.L}: rank {infos[e]['rank']} (oracle {F.r}), err {err:.2e}")
        assert infos[e]["rank"] == F.r
        assert err <= (1e-10 if precision == "fp64" else 1e-6)


@pytest.mark.parametrize("dt", ["fp32", "fp64"])
def test_autotuned_wide_gram_chunks(elm, clean_table, dt):
    # the FP32 / FP64 Gram's K chunks: the tuned Gram is still the Gram (FP64
    # of the rounded input within the accumulation bound), symmetric, with
    # bitwise-equal rows for equal columns
    N, L = 60000, 700
    rng = np.random.default_rng(31)
    H64 = rng.uniform(0, 1, (N, L))
    H64[:, 9] = H64[:, 4]
    if dt == "fp64":
        H, layout = to_dev(H64), "sample"
    else:
        H, layout = to_dev(H64.T.copy()).to(torch.float32), "node"
    chunks, ms = elm.autotune_gram(H, layout=layout)
    rows = elm.tune_table()
    print(f"{dt}: {chunks} chunks, {ms:.3f} ms, table {rows}")
    assert any(r["kind"] == "gram_chunks" and r["value"] == chunks for r in rows)
    M = elm.elm_gram(H, layout).cpu().numpy()
    Hr = H64 if dt == "fp64" else H.double().cpu().numpy().T
    ref = Hr.T @ Hr
    assert np.array_equal(M, M.T)
    tol = 1e-12 if dt == "fp64" else 4 * np.sqrt(N) * 2.0 ** -24
    assert np.max(np.abs(M - ref)) <= tol * np.max(np.abs(ref))
    assert np.array_equal(M[9], M[4])
