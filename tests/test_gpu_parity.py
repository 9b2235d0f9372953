"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars: rank exact; beta within 1e-10 relative on the FP64 path and 1e-6 on
the mixed-precision path (after FP64 refinement); low-precision copies of H
bit-exact with round-to-nearest-even of the device's own FP64 H.
"""
import numpy as np
import pytest
import torch

import elm_workloads as wl
import oracle as O
from oracle import validators as V

from gpu_helpers import bf16_rne, fp16_rne, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def elm():
    from paper_2011_02436_amd import elm as mod
    return mod


def _dev_problem(p):
    return to_dev(p.X), to_dev(p.W), to_dev(p.b), to_dev(p.T)


# ----------------------------------------------------------------------------
# hidden layer
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("N,d,L", [(2000, 20, 200), (77, 5, 13), (1000, 54, 130), (129, 128, 65)])
def test_hidden_fp64_matches_oracle(elm, N, d, L):
    p = wl.random_problem(seed=N + d + L, N=N, d=d, L=L, m=2)
    X, W, b, _ = _dev_problem(p)
    H = torch.empty((N, L), dtype=torch.float64, device=X.device)
    elm.elm_hidden(X, W, b, H=H)
    ref = O.hidden(p.X, p.W, p.b)
    got = H.cpu().numpy()
    # The kernel and NumPy may sum the d products of z = x.w + b in different
    # orders: |dz| <= 2 (d + 1) u (sum_k |x_k w_k| + |b|) for both sums
    # together, which moves sigma(z) by sigma (1 - sigma) |dz|; exp and the
    # division add a few roundings of sigma on each side (8 u covers them).
    u = 2.0 ** -53
    dz = 2 * (d + 1) * u * (np.abs(p.X) @ np.abs(p.W) + np.abs(p.b)[None, :])
    bound = ref * ((1.0 - ref) * dz + 8 * u)
    ratio = np.max(np.abs(got - ref) / bound)
    ulps = np.max(np.abs(got - ref) / np.spacing(ref))
    print(f"hidden fp64 N={N} d={d} L={L}: worst |diff| / bound {ratio:.3f}, {ulps:.1f} ulp")
    assert ratio <= 1.0


@pytest.mark.parametrize("lp", ["bf16", "fp16", "fp32"])
def test_hidden_lowprec_copy_is_rne_of_fp64(elm, lp):
    p = wl.random_problem(seed=5, N=1000, d=20, L=96, m=2)
    X, W, b, _ = _dev_problem(p)
    H = torch.empty((p.N, p.L), dtype=torch.float64, device=X.device)
    dt = {"bf16": torch.bfloat16, "fp16": torch.float16, "fp32": torch.float32}[lp]
    Hlp = torch.empty((p.L, p.N), dtype=dt, device=X.device)
    elm.elm_hidden(X, W, b, H=H, Hlp=Hlp)
    h64 = H.cpu().numpy()
    got = Hlp.float().cpu().numpy().astype(np.float64).T
    if lp == "bf16":
        want = bf16_rne(h64)
    elif lp == "fp16":
        want = fp16_rne(h64)
    else:
        want = h64.astype(np.float32).astype(np.float64)
    assert np.array_equal(got, want)


def test_hidden_fp32_inputs(elm):
    p = wl.random_problem(seed=9, N=300, d=30, L=70, m=2)
    X, W, b = (to_dev(a, torch.float32) for a in (p.X, p.W, p.b))
    H = torch.empty((p.N, p.L), dtype=torch.float32, device=X.device)
    elm.elm_hidden(X, W, b, H=H)
    ref = O.hidden(p.X.astype(np.float32), p.W.astype(np.float32), p.b.astype(np.float32))
    assert np.max(np.abs(H.cpu().numpy() - ref)) <= 2e-6


# ----------------------------------------------------------------------------
# end-to-end FP64 path
# ----------------------------------------------------------------------------
def test_tiny_config_fp64_end_to_end(elm):
    p = wl.tiny_fp64()
    X, W, b, T = _dev_problem(p)
    res = elm.train(X, W, b, T, precision="fp64")
    beta = res.beta.cpu().numpy()
    ref, F = O.solve(O.hidden(p.X, p.W, p.b), p.T)
    err = O.rel_err(beta, ref)
    print(f"tiny fp64: rank {res.rank} vs {F.r}; beta err {err:.2e}; info {res.info}")
    assert res.rank == F.r == 160
    assert err <= 1e-10
    # the pivot order is a permutation whose first r entries are one per distinct node
    piv = res.factor.pivots()
    assert sorted(piv.tolist()) == list(range(p.L))
    assert len(set(p.groups[piv[:res.rank]])) == 160


@pytest.mark.parametrize("N,d,L,m,n_dup", [
    (500, 16, 120, 3, 0), (500, 16, 120, 3, 23), (333, 16, 257, 5, 40),
    (90, 16, 140, 3, 0), (90, 16, 140, 3, 25), (150, 16, 150, 2, 10), (1, 3, 4, 1, 0), (5, 3, 1, 2, 0)])
def test_random_shapes_fp64(elm, N, d, L, m, n_dup):
    p = wl.random_problem(seed=7 * N + L + n_dup, N=N, d=d, L=L, m=m, n_dup=n_dup)
    X, W, b, T = _dev_problem(p)
    res = elm.train(X, W, b, T, precision="fp64", ir_max_iter=2, check_convergence=False)
    H = O.hidden(p.X, p.W, p.b)
    ref, rs = O.solve_svd(H, p.T)
    _, F = O.solve(H, p.T)
    err = O.rel_err(res.beta.cpu().numpy(), ref)
    print(f"N={N} L={L} dup={n_dup}: rank {res.rank} oracle {F.r} svd {rs}; err {err:.2e}")
    assert res.rank == F.r
    assert err <= 1e-10


def test_gram_rows_of_duplicates_are_bitwise_equal(elm):
    # the pivoted Cholesky can only zero a duplicated node if its Gram row is
    # bitwise equal to the original's; check on the end result: K is a 0/1
    # selection matrix and beta is constant within each group of copies
    p = wl.tiny_fp64()
    X, W, b, T = _dev_problem(p)
    res = elm.train(X, W, b, T, precision="fp64", ir_max_iter=0)
    beta = res.beta.cpu().numpy()
    for g in np.unique(p.groups):
        cols = np.flatnonzero(p.groups == g)
        assert np.max(np.abs(beta[cols] - beta[cols[0]])) <= 1e-12 * np.max(np.abs(beta))


def test_repeat_runs_bitwise_identical(elm):
    p = wl.random_problem(seed=3, N=700, d=16, L=150, m=3, n_dup=15)
    X, W, b, T = _dev_problem(p)
    a = elm.train(X, W, b, T, precision="fp64").beta.cpu().numpy()
    c = elm.train(X, W, b, T, precision="fp64").beta.cpu().numpy()
    assert np.array_equal(a, c)


# ----------------------------------------------------------------------------
# mixed precision: low-precision Gram, FP64 rank decision and refinement
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("lp", ["bf16", "fp16", "fp32"])
def test_mixed_precision_tiny_config(elm, lp):
    p = wl.tiny_fp64()
    X, W, b, T = _dev_problem(p)
    res = elm.train(X, W, b, T, precision=lp, ir_tol=1e-10)
    ref, F = O.solve(O.hidden(p.X, p.W, p.b), p.T)
    err = O.rel_err(res.beta.cpu().numpy(), ref)
    print(f"tiny {lp}: rank {res.rank}, err {err:.2e}, info {res.info}")
    assert res.rank == F.r
    assert err <= 1e-6
    assert res.info["ne_residual"] <= 1e-10


def test_mixed_precision_full_rank(elm):
    p = wl.random_problem(seed=12, N=6000, d=32, L=300, m=4)
    X, W, b, T = _dev_problem(p)
    res = elm.train(X, W, b, T, precision="bf16", ir_tol=1e-10)
    ref, F = O.solve(O.hidden(p.X, p.W, p.b), p.T)
    err = O.rel_err(res.beta.cpu().numpy(), ref)
    print(f"bf16 full rank: rank {res.rank}, err {err:.2e}, its {res.info['iterations']}")
    assert res.rank == F.r == 300
    assert err <= 1e-6


# ----------------------------------------------------------------------------
# predict
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_predict_matches_oracle(elm, dtype):
    p = wl.random_problem(seed=4, N=513, d=12, L=77, m=6)
    rng = np.random.default_rng(0)
    beta = rng.standard_normal((p.L, p.m))
    X, W, b = (to_dev(a, dtype) for a in (p.X, p.W, p.b))
    Y, lab = elm.elm_predict(X, W, b, to_dev(beta))
    Yref, labref = O.predict(p.X, p.W, p.b, beta)
    tol = 1e-12 if dtype == torch.float64 else 1e-4
    assert np.max(np.abs(Y.cpu().numpy() - Yref)) <= tol * np.max(np.abs(Yref))
    # labels agree wherever the top two outputs are separated
    srt = np.sort(Yref, axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 1e-6 * np.max(np.abs(Yref))
    assert np.array_equal(lab.cpu().numpy()[clear], labref[clear])


# ----------------------------------------------------------------------------
# ABI validation with a live handle
# ----------------------------------------------------------------------------
def test_abi_rejects_bad_arguments(elm):
    import ctypes
    h = elm.handle()
    lib = elm._lib
    vp = ctypes.c_void_p
    X = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
    # ldx < d
    assert lib.elm_hidden(h.ptr, 10, 3, 4, vp(X.data_ptr()), 2, vp(X.data_ptr()), 4, vp(X.data_ptr()),
                          0, vp(X.data_ptr()), 4, vp(), 0, 2) == 2
    # no output
    assert lib.elm_hidden(h.ptr, 10, 3, 4, vp(X.data_ptr()), 3, vp(X.data_ptr()), 4, vp(X.data_ptr()),
                          0, vp(), 0, vp(), 0, 2) == 1
    # N = 0
    assert lib.elm_hidden(h.ptr, 0, 3, 4, vp(X.data_ptr()), 3, vp(X.data_ptr()), 4, vp(X.data_ptr()),
                          0, vp(X.data_ptr()), 4, vp(), 0, 2) == 1
    f = vp()
    r = ctypes.c_int64()
    # tau_rel >= 1
    assert lib.elm_rank_factor(h.ptr, 10, 3, vp(X.data_ptr()), 3, 0, 0, ctypes.c_double(1.0),
                               ctypes.byref(f), ctypes.byref(r)) == 1
    # bf16 sample-major is unsupported
    assert lib.elm_rank_factor(h.ptr, 10, 3, vp(X.data_ptr()), 3, 2, 0, ctypes.c_double(0.0),
                               ctypes.byref(f), ctypes.byref(r)) == 7


def test_zero_hidden_matrix_gives_rank_zero(elm):
    H = torch.zeros((20, 6), dtype=torch.float64, device="cuda")
    f = elm.elm_rank_factor(H, "sample")
    assert f.rank == 0
    T = torch.ones((20, 2), dtype=torch.float64, device="cuda")
    beta, info = elm.elm_pinv_solve(f, T, H, ir_max_iter=0)
    assert torch.all(beta == 0)


def test_dedup_closed_form_mixture_shape(elm):
    # rank-deficient mid-size case against the duplicated-column closed form
    p = wl.mixture_rankdef(N=8000, L=600)
    X, W, b, T = _dev_problem(p)
    res = elm.train(X, W, b, T, precision="fp64")
    H = O.hidden(p.X, p.W, p.b)
    ref = V.dedup_closed_form(H, p.T, p.groups)
    err = O.rel_err(res.beta.cpu().numpy(), ref)
    print(f"mixture N=8000 L=600: rank {res.rank} (structural {p.structural_rank}), err {err:.2e}")
    assert res.rank == p.structural_rank == 540
    assert err <= 1e-10


# ----------------------------------------------------------------------------
# Gram kernels on their own (multi-tile, split-K, ragged edges)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("N,L", [(2000, 200), (20011, 600), (5000, 257), (70000, 530), (900, 1200)])
def test_gram_fp64_matches_numpy(elm, N, L):
    rng = np.random.default_rng(N + L)
    Hn = rng.uniform(0, 1, (N, L))
    H = to_dev(Hn)
    M = elm.elm_gram(H, "sample").cpu().numpy()
    ref = Hn.T @ Hn if N >= L else Hn @ Hn.T
    assert np.array_equal(M, M.T)
    assert np.max(np.abs(M - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("lp", ["bf16", "fp16", "fp32"])
@pytest.mark.parametrize("N,L", [(2000, 200), (20011, 600), (70000, 530), (6001, 777)])
def test_gram_lowprec_matches_fp64_of_rounded_input(elm, lp, N, L):
    rng = np.random.default_rng(N * 3 + L)
    H64 = rng.uniform(0, 1, (N, L))
    H64[:, 5] = H64[:, 3]                      # a duplicated column
    dt = {"bf16": torch.bfloat16, "fp16": torch.float16, "fp32": torch.float32}[lp]
    Hn = to_dev(H64.T.copy()).to(dt)           # node-major copy
    Hr = Hn.double().cpu().numpy()             # the values the kernel sees
    M = elm.elm_gram(Hn, "node").cpu().numpy()
    ref = Hr @ Hr.T
    assert np.array_equal(M, M.T)
    # FP32 accumulation within each split-K chunk, FP64 across chunks
    assert np.max(np.abs(M - ref)) <= 2e-6 * np.max(np.abs(ref))
    # bitwise-equal input columns give bitwise-equal Gram rows
    assert np.array_equal(M[5], M[3])


@pytest.mark.parametrize("lp", ["bf16", "fp16"])
def test_gram_16bit_same_for_every_leading_dimension(elm, lp):
    """The node-major 16-bit Gram takes 64-sample stages of whole 128-byte
    lines when rows start on 64-element boundaries, stages that straddle lines
    when the leading dimension is only a multiple of 8, and 32-sample register
    steps otherwise; every path multiplies the same 16-sample steps in the same
    order, so the three layouts of the same values give bitwise-equal Grams
    (N = 20000: the last split ends in half a stage; L = 600: a ragged last
    tile)."""
    N, L = 20000, 600
    rng = np.random.default_rng(77)
    dt = {"bf16": torch.bfloat16, "fp16": torch.float16}[lp]
    vals = to_dev(rng.uniform(0, 1, (L, N))).to(dt)
    Ms = []
    for ld in (-(-N // 64) * 64, N, N + 3):
        assert (ld % 64 == 0) or ld == N or ld % 8 != 0
        Hn = torch.empty((L, ld), dtype=dt, device=vals.device)[:, :N]
        Hn.copy_(vals)
        Ms.append(elm.elm_gram(Hn, "node").cpu().numpy())
    ref = vals.double().cpu().numpy()
    ref = ref @ ref.T
    assert np.max(np.abs(Ms[0] - ref)) <= 2e-6 * np.max(np.abs(ref))
    assert np.array_equal(Ms[0], Ms[1])
    assert np.array_equal(Ms[0], Ms[2])


def test_predict_hidden_matches_numpy(elm):
    rng = np.random.default_rng(2)
    H = rng.uniform(0, 1, (1000, 130))
    beta = rng.standard_normal((130, 7))
    Y, lab = elm.elm_predict_hidden(to_dev(H), to_dev(beta))
    ref = H @ beta
    assert np.max(np.abs(Y.cpu().numpy() - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert np.array_equal(lab.cpu().numpy(), np.argmax(ref, axis=1))


def test_autotuned_gram_splits(elm):
    # the autotuner picks among the default rule's split count and its 1/2,
    # 3/4, 3/2 and 2 multiples; the tuned Gram is still the Gram (FP32 partial
    # sums, FP64 across them) of the rounded input, symmetric, with bitwise
    # equal rows for equal columns
    N, L = 300000, 2304  # 45 x 46 / 2 = 1035 tiles of 256: the many-tiles rule
    rng = np.random.default_rng(77)
    H64 = rng.uniform(0, 1, (N, L))
    H64[:, 7] = H64[:, 2]
    Hn = to_dev(H64.T.copy()).to(torch.bfloat16)
    splits, ms = elm.autotune_gram(Hn)
    assert 1 <= splits <= 48 and ms > 0
    Hr = Hn.double().cpu().numpy()
    M = elm.elm_gram(Hn, "node").cpu().numpy()
    ref = Hr @ Hr.T
    assert np.array_equal(M, M.T)
    # FP32 sums over the kc = N / splits samples of a work item (rounding
    # errors grow like sqrt(kc) 2^-24 of the sum), FP64 across items
    kc = -(-N // splits)
    assert np.max(np.abs(M - ref)) <= 4 * np.sqrt(kc) * 2.0 ** -24 * np.max(np.abs(ref))
    assert np.array_equal(M[7], M[2])
    # repeat calls with the tuned schedule are bitwise identical
    assert np.array_equal(elm.elm_gram(Hn, "node").cpu().numpy(), M)
