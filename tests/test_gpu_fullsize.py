"""GPU: the training path at the workloads' full sizes, in the configuration
the benchmark times, against the FP64 oracle's stored results and through
properties that hold at any size.

The expected ranks and beta come from tests/golden/make_fullsize.py, which
runs only the FP64 CPU oracle (minutes per workload, too long for test
time) and stores r, beta and kappa_r for each; rank must be equal and beta
within 1e-10 (FP64 form) or 1e-6 (low-precision Gram + FP64 refinement)
relative, each error printed beside its bar and kappa_r^2 2^-53 (the
scale of rounding differences two correct FP64 normal-equation solvers may
show).  Besides:

* rank: the structural rank of the planted node duplication;
* beta solves the least-squares problem: the relative normal-equation
  residual ||H^T (T - H beta)|| / ||H^T T||, recomputed here with plain torch
  FP64 products (not the library's kernels), is <= 1e-10 at the benchmark's
  own stopping tolerance (and the library's own report agrees);
* beta is the minimum-norm solution: the null space of H is spanned by the
  differences of duplicated columns, so beta is orthogonal to it exactly when
  it is equal across each group of duplicates;
* sampled entries of H and of the training-set outputs H beta against FP64
  NumPy evaluations of their definitions, and the BF16 copy against the
  round-to-nearest-even of H.
"""
import math
import os

import numpy as np
import pytest
import torch

import elm_workloads as wl
import oracle as O

from gpu_helpers import bf16_rne, to_dev

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    """Stored oracle results of one full-size workload (plain float64/int64
    arrays; loaded without pickles)."""
    with np.load(os.path.join(GOLDEN, f"fullsize_{name}.npz")) as z:
        return {k: z[k] for k in z.files}


def check_against_golden(tag, beta, rank, g, tol):
    err = O.rel_err(beta, g["beta"])
    k2e = float(g["kappa"]) ** 2 * EPS
    line = f"{tag}: rank {rank} (oracle {int(g['rank'])}), beta err vs oracle {err:.2e} (bar {tol:.0e}; " \
           f"kappa_r {float(g['kappa']):.0f}, kappa_r^2 eps {k2e:.1e})"
    if "beta_check" in g:
        line += f", vs independent check {O.rel_err(beta, g['beta_check']):.2e}"
    print(line)
    assert rank == int(g["rank"])
    assert err <= tol


@pytest.fixture(scope="module")
def elm():
    from paper_2011_02436_amd import elm as mod
    return mod


def _ne_residual_torch(H64, T, beta, chunk=65536):
    """||H^T (T - H beta)||_F / ||H^T T||_F with torch FP64 products, row chunks."""
    g = torch.zeros((H64.shape[1], T.shape[1]), dtype=torch.float64, device=H64.device)
    z = torch.zeros_like(g)
    for s in range(0, H64.shape[0], chunk):
        Hc = H64[s:s + chunk]
        Tc = T[s:s + chunk]
        e = Tc - Hc @ beta
        g += Hc.T @ e
        z += Hc.T @ Tc
    return float(torch.linalg.norm(g) / torch.linalg.norm(z))


def _sampled_h(p, H64, rng, count=64):
    """Sampled H entries, their FP64 NumPy values and a bound on the
    difference: the two d-term dot products may round in different orders
    (|dz| <= (d + 1) u sum |x_k w_k| + |b| ... ), which moves sigma(z) by
    (1 - sigma) |dz| relative, plus a few roundings in exp and the division."""
    u = 2.0 ** -53
    rows = rng.integers(0, p.N, size=count)
    cols = rng.integers(0, p.L, size=count)
    prods = p.X[rows] * p.W[:, cols].T
    z = prods.sum(axis=1) + p.b[cols]
    ref = 1.0 / (1.0 + np.exp(-z))
    dz = 2 * (p.d + 1) * u * (np.abs(prods).sum(axis=1) + np.abs(p.b[cols]))
    bound = ref * ((1.0 - ref) * dz + 8 * u)
    got = H64[torch.from_numpy(rows).to(H64.device), torch.from_numpy(cols).to(H64.device)].cpu().numpy()
    return rows, cols, got, ref, bound


def _group_spread(beta, groups):
    """Largest deviation of beta within a group of duplicated columns."""
    worst = 0.0
    order = np.argsort(groups, kind="stable")
    g_sorted = groups[order]
    starts = np.flatnonzero(np.r_[True, g_sorted[1:] != g_sorted[:-1]])
    ends = np.r_[starts[1:], len(order)]
    for s, e in zip(starts, ends):
        if e - s > 1:
            blk = beta[order[s:e]]
            worst = max(worst, float(np.abs(blk - blk.mean(axis=0)).max()))
    return worst


def test_full_size_precision_form(elm):
    """N=500000, d=128, L=10000, m=4; BF16 Gram, FP64 rank decision and
    refinement to 1e-10, training-set outputs: the benchmark's step."""
    p = wl.smooth_regression()
    X, W, b, T = to_dev(p.X), to_dev(p.W), to_dev(p.b), to_dev(p.T)
    H64 = torch.empty((p.N, p.L), dtype=torch.float64, device=X.device)
    Hlp = torch.empty((p.L, p.N), dtype=torch.bfloat16, device=X.device)
    res = elm.train(X, W, b, T, precision="bf16", ir_tol=1e-10, H64=H64, Hlp=Hlp, outputs=True)
    torch.cuda.synchronize()
    fi = res.info["factor"]
    ne = _ne_residual_torch(H64, T, res.beta)
    print(f"C4: rank {res.rank}, gram {res.info['gram_dtype']}, certified {fi['certified_full_rank']}, "
          f"library NE {res.info['ne_residual']:.3e}, torch NE {ne:.3e}, its {res.info['iterations']}")
    assert res.rank == p.structural_rank == 10000
    check_against_golden("C4 bf16", res.beta.cpu().numpy(), res.rank, golden("smooth_regression"), 1e-6)
    assert res.info["gram_dtype"] == "bf16" and res.info["escalations"] == 0
    assert fi["reliable"]
    assert res.info["ne_residual"] <= 1e-10
    assert ne <= 1e-10
    # two FP64 evaluations of a residual this small differ in their rounding
    assert abs(ne - res.info["ne_residual"]) <= 0.5 * res.info["ne_residual"] + 1e-12
    rng = np.random.default_rng(123)
    rows, cols, got, ref, bound = _sampled_h(p, H64, rng)
    assert np.all(np.abs(got - ref) <= bound)
    lp = Hlp[torch.from_numpy(cols).to(X.device), torch.from_numpy(rows).to(X.device)].double().cpu().numpy()
    assert np.array_equal(lp, bf16_rne(got))
    beta = res.beta.cpu().numpy()
    ridx = rng.integers(0, p.N, size=16)
    for i in ridx:
        h = H64[int(i)].cpu().numpy()
        want = np.array([math.fsum(h * beta[:, k]) for k in range(p.m)])
        assert np.max(np.abs(res.Y[int(i)].cpu().numpy() - want)) <= 1e-12 * max(1.0, np.abs(want).max())


def test_full_size_precision_form_fp16(elm):
    """The same workload in the FP16 form (FP16 Gram of the library's own
    node-major copy, FP64 rank decision and refinement to 1e-10): rank and beta
    against the oracle's stored result, within the mixed-path bar."""
    p = wl.smooth_regression()
    X, W, b, T = to_dev(p.X), to_dev(p.W), to_dev(p.b), to_dev(p.T)
    res = elm.train(X, W, b, T, precision="fp16", ir_tol=1e-10)
    torch.cuda.synchronize()
    print(f"C4 fp16: rank {res.rank}, gram {res.info['gram_dtype']}, NE {res.info['ne_residual']:.3e}, "
          f"corrections {res.info['iterations']}")
    assert res.rank == p.structural_rank == 10000
    assert res.info["gram_dtype"] == "fp16" and res.info["escalations"] == 0
    assert res.info["ne_residual"] <= 1e-10
    check_against_golden("C4 fp16", res.beta.cpu().numpy(), res.rank, golden("smooth_regression"), 1e-6)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_size_rank_deficient_mixture(elm, precision):
    """N=100000, d=54, L=5000 with 500 duplicated nodes (rank 4500), 7 classes."""
    p = wl.mixture_rankdef()
    X, W, b, T = to_dev(p.X), to_dev(p.W), to_dev(p.b), to_dev(p.T)
    H64 = torch.empty((p.N, p.L), dtype=torch.float64, device=X.device)
    res = elm.train(X, W, b, T, precision=precision, ir_tol=1e-10, H64=H64)
    torch.cuda.synchronize()
    ne = _ne_residual_torch(H64, T, res.beta)
    beta = res.beta.cpu().numpy()
    spread = _group_spread(beta, p.groups) / np.abs(beta).max()
    print(f"C3 {precision}: rank {res.rank} (structural {p.structural_rank}), gram {res.info['gram_dtype']}, "
          f"NE {ne:.3e}, duplicate spread {spread:.2e}, its {res.info['iterations']}")
    assert res.rank == p.structural_rank == 4500
    check_against_golden(f"C3 {precision}", beta, res.rank, golden("mixture_rankdef"),
                         1e-10 if precision == "fp64" else 1e-6)
    # the 500 copies set aside, the 4500 distinct nodes certified
    assert res.info["factor"]["certified_full_rank"] == 2
    assert ne <= 1e-10
    assert spread <= 1e-9
    rng = np.random.default_rng(7)
    _, _, got, ref, bound = _sampled_h(p, H64, rng)
    assert np.all(np.abs(got - ref) <= bound)


def test_full_size_rank_deficient_mixture_greedy_rule(elm):
    """C3 (FP64 form) with the certified path off: the greedy pivoted Cholesky
    (256-wide panels) at order 5000, against the oracle's stored beta."""
    p = wl.mixture_rankdef()
    X, W, b, T = to_dev(p.X), to_dev(p.W), to_dev(p.b), to_dev(p.T)
    old = elm.set_option("full_rank_min_order", 0)
    try:
        res = elm.train(X, W, b, T, precision="fp64", ir_tol=1e-10)
    finally:
        elm.set_option("full_rank_min_order", old)
    assert res.info["factor"]["certified_full_rank"] == 0
    assert res.rank == p.structural_rank == 4500
    check_against_golden("C3 fp64 greedy", res.beta.cpu().numpy(), res.rank, golden("mixture_rankdef"), 1e-10)


def test_full_size_digits_fp32_form(elm):
    """N=60000, d=784 (80% zeros), L=2000, 10 classes; FP32 Gram + refinement."""
    p = wl.digits_like()
    X, W, b, T = to_dev(p.X), to_dev(p.W), to_dev(p.b), to_dev(p.T)
    H64 = torch.empty((p.N, p.L), dtype=torch.float64, device=X.device)
    res = elm.train(X, W, b, T, precision="fp32", ir_tol=1e-10, H64=H64, outputs=True)
    torch.cuda.synchronize()
    ne = _ne_residual_torch(H64, T, res.beta)
    acc = float((res.labels.cpu().numpy() == p.labels).mean())
    print(f"C2 fp32: rank {res.rank}, NE {ne:.3e}, its {res.info['iterations']}, training accuracy {acc:.4f}")
    assert res.rank == p.structural_rank == 2000
    check_against_golden("C2 fp32", res.beta.cpu().numpy(), res.rank, golden("digits_like"), 1e-6)
    assert res.info["gram_dtype"] == "fp32"
    assert ne <= 1e-10
    # labels are the arg-max of the returned outputs (lowest index on ties)
    Y = res.Y.cpu().numpy()
    assert np.array_equal(res.labels.cpu().numpy(), np.argmax(Y, axis=1))


def test_full_size_fp64_form_regression(elm):
    """N=500000, d=128, L=10000, m=4 in the plain FP64 form (FP64 Gram), the
    form the benchmark times beside the precision form."""
    p = wl.smooth_regression()
    X, W, b, T = to_dev(p.X), to_dev(p.W), to_dev(p.b), to_dev(p.T)
    H64 = torch.empty((p.N, p.L), dtype=torch.float64, device=X.device)
    res = elm.train(X, W, b, T, precision="fp64", ir_tol=1e-10, H64=H64)
    torch.cuda.synchronize()
    print(f"C4 fp64: NE {res.info['ne_residual']:.2e}, its {res.info['iterations']}")
    assert res.info["gram_dtype"] == "fp64" and res.info["ne_residual"] <= 1e-10
    check_against_golden("C4 fp64", res.beta.cpu().numpy(), res.rank, golden("smooth_regression"), 1e-10)


@pytest.mark.parametrize("precision", ["bf16", "fp32", "fp64"])
def test_full_size_batch_sweep(elm, precision):
    """The 256-ELM hidden-size sweep (N log-U[1000, 50000], L log-U[64, 2048],
    d=32, m=5, 10% duplicated nodes) in one elm_train_batched call, as the
    benchmark runs it (refinement to NE residual 1e-10): every ELM's rank
    exactly, and beta against the oracle's within the form's bar.

    Conditioning-limited ELMs (kappa_r^2 2^-53 above the bar: 19 of the 256,
    the near-square ones, kappa_r up to ~1e5) are where two correct FP64
    normal-equation solvers may differ by more than the bar (the oracle itself
    is up to 1e-8 from the closed form there).  Each one outside the bar is
    printed with kappa_r and its distance to the duplicated-column closed form
    (accurate to about kappa_r eps), beside the oracle's own distance, and must
    lie within kappa_r^2 2^-53 of the closed form: the first-order rounding
    bound of a normal-equation solve, with no constant factor."""
    probs = wl.batch_sweep()
    g = golden("batch_sweep")
    dev = [tuple(to_dev(a) for a in (q.X, q.W, q.b, q.T)) for q in probs]
    betas, infos, stats = elm.train_batched(dev, precision=precision, ir_tol=1e-10, check=False)
    torch.cuda.synchronize()
    tol = 1e-10 if precision == "fp64" else 1e-6
    off = g["offsets"]
    lim_off = {}
    pos = 0
    for e in g["limited"]:
        n_e = int(off[e + 1] - off[e])
        lim_off[int(e)] = (pos, pos + n_e)
        pos += n_e
    worst = (0.0, -1)
    bad, limited_out = [], []
    for e, q in enumerate(probs):
        ref = g["beta"][off[e]:off[e + 1]]
        got = betas[e].cpu().numpy()
        err = O.rel_err(got, ref)
        kappa = float(g["kappa"][e])
        k2e = kappa * kappa * EPS
        ok = infos[e]["rank"] == int(g["rank"][e]) and stats[e] == 0
        if err > tol and k2e > tol and e in lim_off:
            a, b_ = lim_off[e]
            err_c = O.rel_err(got, g["beta_check_limited"][a:b_])
            limited_out.append((e, q.N, q.L, kappa, k2e, err, err_c, float(g["check_err"][e])))
            ok = ok and err_c <= k2e
        else:
            ok = ok and err <= tol
            if err > worst[0]:
                worst = (err, e)
        if not ok:
            bad.append((e, q.N, q.L, infos[e]["rank"], int(g["rank"][e]), err, kappa, stats[e],
                        infos[e]["gram_dtype"], infos[e]["iterations"]))
    e = worst[1]
    print(f"C5 {precision}: worst beta err {worst[0]:.2e} (bar {tol:.0e}) at ELM {e} (N={probs[e].N}, "
          f"L={probs[e].L}, kappa_r {float(g['kappa'][e]):.0f}, kappa_r^2 eps "
          f"{float(g['kappa'][e]) ** 2 * EPS:.1e}); gram dtypes {sorted(set(i['gram_dtype'] for i in infos))}")
    for (e_, N_, L_, kap, k2e, err, err_c, err_o) in limited_out:
        print(f"  conditioning-limited ELM {e_} (N={N_}, L={L_}): kappa_r {kap:.0f}, kappa_r^2 eps {k2e:.1e}; "
              f"vs oracle {err:.1e}; vs closed form: library {err_c:.1e}, oracle {err_o:.1e}")
    for b_ in bad:
        print("  outside the bar:", b_)
    assert not bad
