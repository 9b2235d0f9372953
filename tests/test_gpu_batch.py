"""GPU: batched independent trainings (elm_train_batched) against the FP64
CPU oracle, on a small draw of the hidden-size-sweep workload (ragged N and
L, 10% duplicated nodes, some problems with N < L)."""
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


@pytest.fixture(autouse=True)
def greedy_singles(elm):
    """The batch takes the greedy rank rule at every order; the single
    trainings compared with it bit for bit take that rule too."""
    old = elm.set_option("full_rank_min_order", 0)
    yield
    elm.set_option("full_rank_min_order", old)


@pytest.fixture(scope="module")
def batch():
    probs = wl.batch_sweep(seed=21, count=12, L_range=(24, 400), N_range=(200, 3000))
    refs = []
    for p in probs:
        H = O.hidden(p.X, p.W, p.b)
        beta, F = O.solve(H, p.T)
        # rounding-order differences in a normal-equation solve scale with
        # kappa^2 of the independent columns
        s = np.linalg.svd(H[:, F.piv[:F.r]] if p.N >= p.L else H[F.piv[:F.r], :], compute_uv=False)
        refs.append((beta, F.r, (s[0] / s[-1]) ** 2))
    return probs, refs


@pytest.fixture(scope="module")
def mixed():
    """Orders on both sides of the one-workgroup limit (512) in one group:
    several panels (1100), a ragged last panel (530), the N < L route with
    n = N = 700, and a small problem."""
    shapes = [(3000, 1100, 110), (700, 1200, 120), (2500, 530, 53), (1500, 300, 30)]
    probs = [wl.random_problem(40 + i, N, 16, L, 3, n_dup=k) for i, (N, L, k) in enumerate(shapes)]
    refs = []
    for p in probs:
        H = O.hidden(p.X, p.W, p.b)
        beta, F = O.solve(H, p.T)
        s = np.linalg.svd(H[:, F.piv[:F.r]] if p.N >= p.L else H[F.piv[:F.r], :], compute_uv=False)
        refs.append((beta, F.r, (s[0] / s[-1]) ** 2))
    return probs, refs


def _dev(p):
    return to_dev(p.X), to_dev(p.W), to_dev(p.b), to_dev(p.T)


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_batched_matches_oracle(elm, batch, precision):
    probs, refs = batch
    assert any(p.N < p.L for p in probs) and any(p.N >= p.L for p in probs)
    dev = [_dev(p) for p in probs]
    betas, infos, stats = elm.train_batched(dev, precision=precision, ir_tol=1e-12)
    assert stats == [0] * len(probs)
    for e, (p, (ref, r, k2)) in enumerate(zip(probs, refs)):
        err = O.rel_err(betas[e].cpu().numpy(), ref)
        info = infos[e]
        want_dt = "fp64" if (precision == "fp64" or p.N < p.L) else precision
        tol = 1e-10 if precision == "fp64" else 1e-6
        print(f"[{e}] N={p.N} L={p.L} rank {info['rank']} (oracle {r}) {info['gram_dtype']} "
              f"its {info['iterations']} ne {info['ne_residual']:.1e} err {err:.2e} tol {tol:.1e} "
              f"(kappa^2 eps {k2 * EPS:.1e})")
        assert info["rank"] == r == p.structural_rank
        assert info["gram_dtype"] == want_dt and info["escalations"] == 0
        assert info["transposed"] == (p.N < p.L)
        assert info["ne_residual"] <= 1e-12
        assert err <= tol


def test_batched_equals_single_trainings(elm, batch):
    probs, _ = batch
    dev = [_dev(p) for p in probs[:5]]
    betas, infos, _ = elm.train_batched(dev, precision="fp64", ir_tol=1e-12)
    for e, (X, W, b, T) in enumerate(dev):
        one = elm.train(X, W, b, T, precision="fp64", ir_tol=1e-12)
        # same kernels, same order of operations on every stream
        assert torch.equal(one.beta, betas[e])
        assert one.rank == infos[e]["rank"]


def test_batched_rejects_malformed_problem_before_running(elm, batch):
    probs, _ = batch
    dev = [_dev(p) for p in probs[:3]]
    X, W, b, T = dev[1]
    dev[1] = (X, W, b, T[:, :0])  # m = 0
    with pytest.raises((elm.ElmError, ValueError)):
        elm.train_batched(dev)
    empty_betas, empty_infos, empty_stats = elm.train_batched([])
    assert empty_betas == [] and empty_infos == [] and empty_stats == []


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_batched_mixed_orders_match_oracle(elm, mixed, precision):
    probs, refs = mixed
    dev = [_dev(p) for p in probs]
    betas, infos, stats = elm.train_batched(dev, precision=precision, ir_tol=1e-12)
    assert stats == [0] * len(probs)
    for e, (p, (ref, r, k2)) in enumerate(zip(probs, refs)):
        err = O.rel_err(betas[e].cpu().numpy(), ref)
        info = infos[e]
        tol = 1e-10 if precision == "fp64" else 1e-6
        print(f"[{e}] N={p.N} L={p.L} rank {info['rank']} (oracle {r}) {info['gram_dtype']} "
              f"its {info['iterations']} ne {info['ne_residual']:.1e} err {err:.2e} tol {tol:.1e} "
              f"(kappa^2 eps {k2 * EPS:.1e})")
        assert info["rank"] == r == p.structural_rank
        assert info["transposed"] == (p.N < p.L)
        assert info["ne_residual"] <= 1e-12
        assert err <= tol


def test_batched_mixed_orders_equal_single_trainings(elm, mixed):
    probs, _ = mixed
    dev = [_dev(p) for p in probs]
    betas, infos, _ = elm.train_batched(dev, precision="fp64", ir_tol=1e-12)
    for e, (X, W, b, T) in enumerate(dev):
        one = elm.train(X, W, b, T, precision="fp64", ir_tol=1e-12)
        assert torch.equal(one.beta, betas[e])
        assert one.rank == infos[e]["rank"]
        assert one.info["factor"] == infos[e]["factor"]


def test_batched_escalation_matches_single_training(elm, batch):
    # a problem whose BF16 rank decision lies within the Gram's noise (the
    # single-training escalation case) among ordinary ones: it is trained
    # again from a higher-precision Gram, the others are not
    probs, _ = batch
    hard = wl.random_problem(seed=11, N=4000, d=2, L=120, m=2)
    dev = [_dev(probs[0]), _dev(hard), _dev(probs[1])]
    betas, infos, stats = elm.train_batched(dev, precision="bf16", ir_tol=1e-10, ir_max_iter=8,
                                            check=False)
    X, W, b, T = dev[1]
    one = elm.train(X, W, b, T, precision="bf16", ir_tol=1e-10, ir_max_iter=8, check_convergence=False)
    print(f"batched escalation: {infos[1]['gram_dtype']} after {infos[1]['escalations']} "
          f"(guard {infos[1]['guard']}); single {one.info['gram_dtype']} after {one.info['escalations']}")
    assert infos[1]["escalations"] == one.info["escalations"] == 2
    assert infos[1]["guard"] == one.info["guard"] == 1
    assert infos[1]["gram_dtype"] == "fp64" and infos[1]["rank"] == one.rank
    assert torch.equal(betas[1], one.beta)
    assert infos[0]["escalations"] == 0 and infos[2]["escalations"] == 0
    assert stats[0] == 0 and stats[2] == 0


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_batched_replays_are_identical(elm, mixed, precision):
    # the shared pivot-step launches and the whole refinement of a batch are
    # captured once as HIP graphs and replayed by later calls with the same
    # shape: every replay, with other work and synchronisations between them,
    # gives the first call's results, which equal the single trainings'
    probs, refs = mixed
    dev = [_dev(p) for p in probs]
    first, infos0, st0 = elm.train_batched(dev, precision=precision, ir_tol=1e-12, check=False)
    rep0 = elm.batch_report()
    print(f"{precision} first call: {rep0}")
    for rep in range(3):
        X, W, b, T = dev[0]
        elm.train(X, W, b, T, precision="bf16", ir_tol=1e-10)  # unrelated eager work
        torch.cuda.synchronize()
        again, infos, st = elm.train_batched(dev, precision=precision, ir_tol=1e-12, check=False)
        report = elm.batch_report()
        assert report["graph_captures"] == 0 and report["graph_launches"] >= 1, report
        # one group: four host synchronisations with the batch stream
        # (thresholds, ranks, the factors' flags, the refinement's final state)
        assert report["groups"] == 1 and report["batch_stream_syncs"] == 4, report
        assert st == st0
        for e in range(len(probs)):
            assert torch.equal(again[e], first[e]), (rep, e)
            assert infos[e]["rank"] == infos0[e]["rank"] == refs[e][1]
            assert infos[e]["ne_history"] == infos0[e]["ne_history"], (rep, e)
    for e, (X, W, b, T) in enumerate(dev):
        one = elm.train(X, W, b, T, precision=precision, ir_tol=1e-12, check_convergence=False)
        assert torch.equal(one.beta, first[e]), e


def _solve_fields(info):
    return (info["rank"], info["iterations"], info["ne_residual"], info["transposed"])


def test_batched_bf16_equals_single_trainings(elm, batch):
    # BF16 Grams need different numbers of corrections per problem, so the
    # problems leave the shared refinement loop at different iterations
    probs, _ = batch
    dev = [_dev(p) for p in probs[:8]]
    betas, infos, stats = elm.train_batched(dev, precision="bf16", ir_tol=1e-12)
    assert stats == [0] * len(dev)
    its = set()
    for e, (X, W, b, T) in enumerate(dev):
        one = elm.train(X, W, b, T, precision="bf16", ir_tol=1e-12)
        assert torch.equal(one.beta, betas[e]), e
        assert _solve_fields(one.info) == _solve_fields(infos[e]), e
        assert one.info["ne_history"] == infos[e]["ne_history"], e
        if probs[e].N >= probs[e].L:
            its.add(infos[e]["iterations"])
    print(f"iterations per problem: {sorted(its)}")
    assert len(its) > 1


@pytest.mark.parametrize("ir_max_iter", [0, 1])
def test_batched_iteration_cap_equals_single_trainings(elm, batch, ir_max_iter):
    # ir_tol = 0 is never reached: every problem stops at the cap (or when a
    # correction makes no progress) with NO_CONVERGENCE, beta the last iterate
    probs, _ = batch
    dev = [_dev(p) for p in probs[:6]]
    betas, infos, stats = elm.train_batched(dev, precision="fp64", ir_tol=0.0, ir_max_iter=ir_max_iter,
                                            check=False)
    for e, (X, W, b, T) in enumerate(dev):
        one = elm.train(X, W, b, T, precision="fp64", ir_tol=0.0, ir_max_iter=ir_max_iter,
                        check_convergence=False)
        assert torch.equal(one.beta, betas[e]), e
        assert _solve_fields(one.info) == _solve_fields(infos[e]), e
        if ir_max_iter == 0:
            assert stats[e] == 0 and infos[e]["ne_residual"] == -1.0
        else:
            assert stats[e] == elm.ELM_ERR_NO_CONVERGENCE and infos[e]["iterations"] <= 1


@pytest.fixture(scope="module")
def tails():
    """Shapes the other fixtures miss: Grams of G above order 128 (the shared
    two-block steps up to order 256, the per-problem blocked Cholesky above
    it, then the shared inverse) in the Woodbury form (n - r < r) and the
    direct form (n - r >= r), full rank (no K), m > 8 (trained per problem
    beside the shared launches) and N < L, in one batch."""
    specs = [(3000, 700, 200, 3), (2500, 600, 350, 3), (2000, 300, 0, 3), (1500, 200, 20, 12),
             (400, 900, 90, 3), (3000, 1400, 300, 3)]
    probs = [wl.random_problem(60 + i, N, 16, L, m, n_dup=k) for i, (N, L, k, m) in enumerate(specs)]
    refs = []
    for p in probs:
        H = O.hidden(p.X, p.W, p.b)
        beta, F = O.solve(H, p.T)
        s = np.linalg.svd(H[:, F.piv[:F.r]] if p.N >= p.L else H[F.piv[:F.r], :], compute_uv=False)
        refs.append((beta, F.r, (s[0] / s[-1]) ** 2))
    return probs, refs


@pytest.mark.parametrize("precision", ["fp64", "bf16", "fp32"])
def test_batched_tail_shapes_match_oracle_and_single(elm, tails, precision):
    probs, refs = tails
    dev = [_dev(p) for p in probs]
    betas, infos, stats = elm.train_batched(dev, precision=precision, ir_tol=1e-12)
    assert stats == [0] * len(probs)
    for e, (p, (ref, r, k2)) in enumerate(zip(probs, refs)):
        info = infos[e]
        err = O.rel_err(betas[e].cpu().numpy(), ref)
        tol = 1e-10 if precision == "fp64" else 1e-6
        n = min(p.N, p.L)
        print(f"[{e}] N={p.N} L={p.L} m={p.m} rank {info['rank']} (oracle {r}), n - r = {n - r}, "
              f"{info['gram_dtype']} its {info['iterations']} err {err:.2e} tol {tol:.1e} "
              f"(kappa^2 eps {k2 * EPS:.1e})")
        assert info["rank"] == r == p.structural_rank
        assert info["ne_residual"] <= 1e-12
        assert err <= tol
        X, W, b, T = dev[e]
        one = elm.train(X, W, b, T, precision=precision, ir_tol=1e-12)
        assert torch.equal(one.beta, betas[e]), e
        assert one.info["iterations"] == info["iterations"]
    # the shapes reach the branches they are meant for
    r = [info["rank"] for info in infos]
    assert 700 - r[0] > 128 and 700 - r[0] < r[0]
    assert 600 - r[1] > 128 and 600 - r[1] >= r[1]
    assert r[2] == 300
    assert 1400 - r[5] > 256 and 1400 - r[5] < r[5]


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_batched_wide_targets_match_oracle_and_single(elm, precision):
    # 16 < m <= 64 (trained per problem on the worker streams beside the
    # shared launches of the m <= 8 problems)
    specs = [(2600, 230, 23, 17), (1800, 300, 30, 40), (2200, 150, 0, 64), (2000, 260, 26, 5)]
    probs = [wl.random_problem(80 + i, N, 20, L, m, n_dup=k) for i, (N, L, k, m) in enumerate(specs)]
    dev = [_dev(p) for p in probs]
    betas, infos, stats = elm.train_batched(dev, precision=precision, ir_tol=1e-12)
    assert stats == [0] * len(probs)
    tol = 1e-10 if precision == "fp64" else 1e-6
    for e, p in enumerate(probs):
        ref, F = O.solve(O.hidden(p.X, p.W, p.b), p.T)
        err = O.rel_err(betas[e].cpu().numpy(), ref)
        print(f"[{e}] N={p.N} L={p.L} m={p.m} rank {infos[e]['rank']} (oracle {F.r}) "
              f"{infos[e]['gram_dtype']} err {err:.2e} (bar {tol:.0e})")
        assert infos[e]["rank"] == F.r == p.structural_rank
        assert err <= tol
        X, W, b, T = dev[e]
        one = elm.train(X, W, b, T, precision=precision, ir_tol=1e-12)
        assert torch.equal(one.beta, betas[e]), e


def test_batched_agrees_with_a_certified_single_training(elm):
    # with the default order threshold a single training certifies these
    # full-rank problems; the batch takes the greedy rule: the same rank, beta
    # equal to rounding
    elm.set_option("full_rank_min_order", 64)
    probs = [wl.random_problem(70 + i, N, 16, L, 3) for i, (N, L) in enumerate([(3000, 300), (600, 900), (2000, 150)])]
    dev = [_dev(p) for p in probs]
    betas, infos, _ = elm.train_batched(dev, precision="fp64", ir_tol=1e-12)
    for e, (X, W, b, T) in enumerate(dev):
        one = elm.train(X, W, b, T, precision="fp64", ir_tol=1e-12)
        assert one.info["factor"]["certified_full_rank"]
        assert not infos[e]["factor"]["certified_full_rank"]
        assert one.rank == infos[e]["rank"] == min(probs[e].N, probs[e].L)
        err = O.rel_err(betas[e].cpu().numpy(), one.beta.cpu().numpy())
        # two correct normal-equation solvers differ by up to kappa^2 eps
        s = np.linalg.svd(O.hidden(probs[e].X, probs[e].W, probs[e].b), compute_uv=False)
        bar = max(1e-10, (s[0] / s[-1]) ** 2 * EPS)
        print(f"[{e}] N={probs[e].N} L={probs[e].L}: batch vs certified single {err:.1e} (bar {bar:.1e})")
        assert err <= bar
