"""GPU: the one-call training entry (elm_train) and the rank-decision
diagnostics (elm_factor_get_info), against the FP64 CPU oracle.

The precision policy is checked on a case where a 16-bit Gram cannot resolve
the rank: with d = 2 inputs the FP64 Schur diagonals fall to ~1e-14 of the
largest while the BF16 rounding noise is ~1e-6, so the BF16 (and FP32) rank
decisions are flagged and the training moves up to the FP64 Gram.
"""

import numpy as np
import pytest
import torch

import elm_workloads as wl
import oracle as O
from oracle import validators as V

from gpu_helpers import check_fp64_beta, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def elm():
    from paper_2011_02436_amd import elm as mod
    return mod


def _dev(p):
    return to_dev(p.X), to_dev(p.W), to_dev(p.b), to_dev(p.T)


def test_factor_info_fp64_matches_oracle(elm):
    p = wl.tiny_fp64()
    X, W, b, _ = _dev(p)
    H = torch.empty((p.N, p.L), dtype=torch.float64, device=X.device)
    elm.elm_hidden(X, W, b, H=H)
    f = elm.elm_rank_factor(H, "sample")
    info = f.info()
    Href = O.hidden(p.X, p.W, p.b)
    M, _ = O.gram(Href)
    R, piv, r = O.pivoted_cholesky(M)
    mx = M.diagonal().max()
    print(f"factor info fp64: {info}")
    assert info["rank"] == r == p.structural_rank
    assert info["gram_dtype"] == "fp64" and info["reliable"]
    assert abs(info["max_diag"] - mx) <= 1e-13 * mx
    assert abs(info["last_pivot"] - R[r - 1, r - 1] ** 2) <= 1e-9 * mx
    assert abs(info["tau"] - O.default_tau(M, K=p.N)) <= 1e-13 * O.default_tau(M, K=p.N)
    # duplicated columns leave Schur diagonals at rounding level
    assert info["first_rejected"] <= info["tau"]
    assert abs(info["first_rejected"]) <= 1e3 * info["n"] * 2.0 ** -53 * mx


@pytest.mark.parametrize("lp", ["bf16", "fp16", "fp32"])
def test_factor_info_lowprec_tiny_is_reliable(elm, lp):
    p = wl.tiny_fp64()
    X, W, b, _ = _dev(p)
    H = torch.empty((p.N, p.L), dtype=torch.float64, device=X.device)
    dt = {"bf16": torch.bfloat16, "fp16": torch.float16, "fp32": torch.float32}[lp]
    Hlp = torch.empty((p.L, p.N), dtype=dt, device=X.device)
    elm.elm_hidden(X, W, b, H=H, Hlp=Hlp)
    info = elm.elm_rank_factor(Hlp, "node").info()
    ref = elm.elm_rank_factor(H, "sample").info()
    print(f"factor info {lp}: {info}")
    assert info["rank"] == ref["rank"] == p.structural_rank
    assert info["gram_dtype"] == lp and info["reliable"]
    u = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11, "fp32": 2.0 ** -24}[lp]
    assert info["noise_floor"] >= u * u / 3 * info["max_diag"]
    assert info["last_pivot"] >= 2 * info["noise_floor"]
    # the smallest pivot moves by about the rounding noise, not more
    assert abs(info["last_pivot"] - ref["last_pivot"]) <= 0.2 * ref["last_pivot"]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("bf16", 1e-6), ("fp16", 1e-6),
                                           ("fp32", 1e-6)])
def test_train_entry_matches_oracle(elm, precision, tol):
    p = wl.tiny_fp64()
    X, W, b, T = _dev(p)
    res = elm.train(X, W, b, T, precision=precision, ir_tol=1e-12)
    ref, _ = O.solve(O.hidden(p.X, p.W, p.b), p.T)
    err = O.rel_err(res.beta.cpu().numpy(), ref)
    print(f"elm_train {precision}: rank {res.rank} err {err:.2e} info {res.info['ne_history']}")
    assert res.rank == p.structural_rank
    assert res.info["gram_dtype"] == precision
    assert res.info["escalations"] == 0 and res.info["guard"] == 0
    assert res.info["ne_residual"] <= 1e-12
    assert err <= tol
    assert res.factor is not None and res.factor.info()["rank"] == res.rank


def test_train_escalates_when_rank_is_within_noise(elm):
    p = wl.random_problem(seed=11, N=4000, d=2, L=120, m=2)
    X, W, b, T = _dev(p)
    # the same refinement budget for both (the defaults differ by precision)
    r64 = elm.train(X, W, b, T, precision="fp64", ir_tol=1e-10, ir_max_iter=8, check_convergence=False)
    res = elm.train(X, W, b, T, precision="bf16", ir_tol=1e-10, ir_max_iter=8, check_convergence=False)
    print(f"escalation: fp64 rank {r64.rank}; bf16 request -> {res.info['gram_dtype']} after "
          f"{res.info['escalations']} steps (guard {res.info['guard']}), rank {res.rank}, "
          f"factor {res.info['factor']}")
    assert res.info["escalations"] == 2 and res.info["guard"] == 1
    assert res.info["gram_dtype"] == "fp64"
    assert res.rank == r64.rank < p.L
    # same FP64 Gram, same kernels: the same beta.  (Here the FP64 pivots
    # decay smoothly to the threshold -- the last kept one is ~1e-11 of the
    # largest, six orders below the BF16 noise floor -- so the comparison is
    # with the library's own FP64 form, not with the oracle, whose rounding
    # order may keep one column more or less.)
    err = O.rel_err(res.beta.cpu().numpy(), r64.beta.cpu().numpy())
    assert err <= 1e-12
    assert res.info["factor"]["last_pivot"] <= 1e-8 * res.info["factor"]["max_diag"]


def test_train_escalation_matches_oracle_and_closed_form(elm):
    # d = 3 inputs, 16 nodes of which 2 are copies: the FP64 pivots fall to
    # 2.0e-6 of the largest (kept; the FP64 threshold is ~1e-11) and the copies'
    # Schur diagonals to ~1e-16 (rejected), a clean gap for the FP64 rank.  The
    # last kept pivot lies within the BF16 and FP32 Grams' rounding noise
    # (about 1e-5 and 2e-6 of the largest diagonal), so both are flagged and
    # the training ends on the FP64 Gram; r and beta must then be the
    # oracle's, and beta the duplicated-column closed form's.
    # kappa_r is ~3200 here (kappa_r^2 eps 1.2e-9), so with uncorrelated
    # targets beta's rounding sensitivity would exceed the 1e-10 bar for any
    # FP64 solver.  The targets are a linear function of H plus 1e-3 noise
    # instead: the least-squares residual is then small and the sensitivity is
    # kappa eps + kappa^2 eps ||r|| / (||H|| ||beta||) ~ 5e-13.  The solve from
    # the FP64 factor alone still carries a forward error of about
    # kappa_r^2 eps (the Gram's rounding) while its normal-equation residual is
    # already at its floor, so, as the oracle does, two refinement corrections
    # are always applied (ir_tol = 0: the loop runs to ir_max_iter and reports
    # that it did not reach 0).
    p = wl.random_problem(seed=109, N=4000, d=3, L=16, m=2, n_dup=2)
    H = O.hidden(p.X, p.W, p.b)
    rng = np.random.default_rng(1109)
    T_h = H @ rng.standard_normal((p.L, p.m)) + 1e-3 * rng.standard_normal((p.N, p.m))
    X, W, b, _ = _dev(p)
    T = to_dev(T_h)
    ref, F = O.solve(H, T_h)
    closed = V.dedup_closed_form(H, T_h, p.groups)
    s = np.linalg.svd(H[:, F.piv[:F.r]], compute_uv=False)
    kappa = s[0] / s[-1]
    resid = np.linalg.norm(T_h - H @ closed) / (s[0] * np.linalg.norm(closed))
    sens = kappa * 2.0 ** -53 + kappa ** 2 * 2.0 ** -53 * resid
    res = elm.train(X, W, b, T, precision="bf16", ir_tol=0.0, ir_max_iter=2, check_convergence=False)
    fi = res.info["factor"]
    err = O.rel_err(res.beta.cpu().numpy(), ref)
    err_c = O.rel_err(res.beta.cpu().numpy(), closed)
    print(f"escalation: residuals {res.info['ne_history']}, corrections kept {res.info['iterations']}")
    print(f"escalation: {res.info['gram_dtype']} after {res.info['escalations']} (guard {res.info['guard']}), "
          f"rank {res.rank} (oracle {F.r}), last pivot {fi['last_pivot'] / fi['max_diag']:.2e} of max, "
          f"err vs oracle {err:.2e}, vs closed form {err_c:.2e} (bar 1e-10; kappa_r {kappa:.0f}, "
          f"sensitivity {sens:.1e}; oracle vs closed form {O.rel_err(ref, closed):.1e})")
    assert res.info["escalations"] == 2 and res.info["guard"] == 1
    assert res.info["gram_dtype"] == "fp64" and fi["reliable"]
    assert res.rank == F.r == p.structural_rank == 14
    assert res.info["iterations"] == 2
    assert err <= 1e-10
    assert err_c <= 1e-10


@pytest.mark.parametrize("m", [17, 40, 64])
@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_train_wide_targets_match_oracle(elm, m, precision):
    # 16 < m <= 64: the widest residual / H^T e / output kernels and the
    # widest thin products of the solves
    p = wl.random_problem(seed=90 + m, N=2600, d=20, L=230, m=m, n_dup=23)
    X, W, b, T = _dev(p)
    ref, F = O.solve(O.hidden(p.X, p.W, p.b), p.T)
    res = elm.train(X, W, b, T, precision=precision, ir_tol=1e-12)
    err = O.rel_err(res.beta.cpu().numpy(), ref)
    tol = 1e-10 if precision == "fp64" else 1e-6
    print(f"m={m} {precision}: rank {res.rank} (oracle {F.r}) err {err:.2e} (bar {tol:.0e}) "
          f"its {res.info['iterations']} ne {res.info['ne_residual']:.1e}")
    assert res.rank == F.r == p.structural_rank
    assert res.info["ne_residual"] <= 1e-12
    assert err <= tol
    # predict through the stored H and through X, W, b for the same beta
    Hd = torch.empty((p.N, p.L), dtype=torch.float64, device=X.device)
    elm.elm_hidden(X, W, b, H=Hd)
    Y1, lab1 = elm.elm_predict_hidden(Hd, res.beta)
    Y2, lab2 = elm.elm_predict(X, W, b, res.beta)
    want = O.hidden(p.X, p.W, p.b) @ res.beta.cpu().numpy()
    assert O.rel_err(Y1.cpu().numpy(), want) <= 1e-12
    assert O.rel_err(Y2.cpu().numpy(), want) <= 1e-12
    srt = np.sort(want, axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 1e-9 * np.abs(want).max()
    assert np.array_equal(lab1.cpu().numpy()[clear], np.argmax(want, axis=1)[clear])
    assert np.array_equal(lab2.cpu().numpy()[clear], np.argmax(want, axis=1)[clear])


def test_train_lowprec_with_n_below_l_uses_fp64(elm):
    p = wl.random_problem(seed=12, N=300, d=16, L=500, m=3)
    X, W, b, T = _dev(p)
    res = elm.train(X, W, b, T, precision="bf16", ir_tol=1e-10)
    ref, _ = O.solve(O.hidden(p.X, p.W, p.b), p.T)
    assert res.info["gram_dtype"] == "fp64" and res.info["transposed"]
    assert res.rank == 300
    err = O.rel_err(res.beta.cpu().numpy(), ref)
    print(f"N < L, bf16 request: fp64 route, err {err:.2e} (bar 1e-10)")
    assert err <= 1e-10


def test_train_rejects_bad_arguments(elm):
    p = wl.tiny_fp64()
    X, W, b, T = _dev(p)
    with pytest.raises(TypeError):
        elm.train(X.float(), W, b, T)
    with pytest.raises(ValueError):
        elm.train(X, W, b, T, precision="int8")
    bad = torch.empty((p.N, p.L), dtype=torch.bfloat16, device=X.device)  # wrong shape for Hlp
    with pytest.raises(ValueError):
        elm.train(X, W, b, T, precision="bf16", Hlp=bad)
    with pytest.raises(elm.ElmError):
        elm.train(X, W, b, T, ir_tol=2.0)


@pytest.mark.parametrize("m", [1, 8, 12])
def test_train_target_widths(elm, m):
    # m <= 8 forms H^T T inside the hidden-layer kernel; wider targets take
    # the separate streaming pass
    p = wl.random_problem(seed=30 + m, N=3001, d=24, L=257, m=m, n_dup=17)
    X, W, b, T = _dev(p)
    ref, _ = O.solve(O.hidden(p.X, p.W, p.b), p.T)
    for precision, tol in (("fp64", 1e-10), ("bf16", 1e-6)):
        res = elm.train(X, W, b, T, precision=precision, ir_tol=1e-12)
        err = O.rel_err(res.beta.cpu().numpy(), ref)
        print(f"m={m} {precision}: rank {res.rank} err {err:.2e} its {res.info['iterations']}")
        assert res.rank == p.structural_rank
        assert err <= tol


@pytest.mark.parametrize("precision,its", [("fp64", None), ("bf16", None), ("fp64", 0)])
def test_train_outputs_are_h_beta(elm, precision, its):
    # Y and labels come from the last refinement pass (a separate pass when
    # there is no refinement); they must be H beta for the returned beta
    p = wl.random_problem(seed=41, N=2500, d=16, L=300, m=5, n_dup=30)
    X, W, b, T = _dev(p)
    res = elm.train(X, W, b, T, precision=precision, ir_tol=1e-12, ir_max_iter=its, outputs=True)
    H = O.hidden(p.X, p.W, p.b)
    want = H @ res.beta.cpu().numpy()
    got = res.Y.cpu().numpy()
    assert O.rel_err(got, want) <= 1e-13
    lab = res.labels.cpu().numpy()
    # arg-max with the lowest index on ties; rows whose top two outputs are
    # within rounding of each other may take either
    top2 = np.sort(want, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > 1e-12 * np.abs(want).max()
    assert np.array_equal(lab[clear], np.argmax(want, axis=1)[clear])
    assert np.all((lab >= 0) & (lab < p.m))
    acc = float(np.mean(lab == p.labels))
    ref_acc = O.training_accuracy(p.X, p.W, p.b, res.beta.cpu().numpy(), p.labels)
    assert abs(acc - ref_acc) <= 2.0 / p.N


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_train_generically_rank_deficient_n_below_l(elm, precision):
    # N < L with fewer distinct nodes than samples: H H^T is singular without
    # duplicated rows, so its rejected pivots are rounding noise of the Gram;
    # the default threshold must reject them (the oracle pins the same case
    # against the SVD).  kappa_r is ~8300 here (kappa_r^2 eps 7.6e-9): the
    # oracle itself is 3.3e-10 from the SVD and closed-form solutions, so beta
    # is held to the conditioning rule (closed form within kappa_r^2 eps).
    p = wl.random_problem(seed=138, N=399, d=32, L=443, m=3, n_dup=58)
    X, W, b, T = _dev(p)
    H = O.hidden(p.X, p.W, p.b)
    ref, F = O.solve(H, p.T)
    closed = V.dedup_closed_form(H, p.T, p.groups)
    sv = np.linalg.svd(H, compute_uv=False)
    res = elm.train(X, W, b, T, precision=precision, ir_tol=1e-12)
    print(f"{precision}: rank {res.rank} (oracle {F.r}) ne {res.info['ne_residual']:.1e}, "
          f"corrections {res.info['iterations']}")
    assert res.rank == F.r == 385
    assert res.info["transposed"] and res.info["gram_dtype"] == "fp64"
    assert res.info["ne_residual"] <= 1e-12
    check_fp64_beta(f"N < L {precision}", res.beta.cpu().numpy(), ref, closed, sv[0] / sv[F.r - 1])
