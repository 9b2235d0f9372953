#!/usr/bin/env python3
"""Benchmark: ELM trainings/s of the precision form (BF16 Gram + FP64 pivoted
Cholesky + FP64 refinement) against the plain FP64 GPU form at equal
normal-equation residual, on the regression workload N=500000, d=128,
L=10000, m=4 (synthetic, seeded).

One step = the whole path on resident inputs: hidden layer (FP64 with a
node-major BF16 copy), BF16 Gram, FP64 pivoted Cholesky and factor, beta with
refinement to a relative normal-equation residual of 1e-10, and the
training-set outputs H beta with their arg-max labels (taken from the last
refinement pass, which evaluates H beta for the final beta).

Prints ONE JSON line.  Extra keys: the FP64 form's time and the speedup at
equal residual, the FP16 form on the same workload, per-stage times, the Gram
kernel's roofline, trainings/s of the other named workloads (the tiny FP64
problem, the digits-like FP32 form, the rank-deficient mixture in the FP64 and
FP32 forms, the 256-ELM hidden-size sweep), and the FP64 CPU oracle timed on a
bounded sample of the same workload.

`--stage NAME` instead runs one stage of the path alone `--reps` times (after
one untimed call) and prints its wall times: the command the rocprofv3 kernel
and counter summaries are taken with.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ELM trainings/sec + Gram TFLOP/s, BF16+refine vs FP64 GPU at equal residual"
PEAK_BF16_TFLOPS = 2516.6   # MI355X dense BF16 MFMA
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp16", "fp32"])
    ap.add_argument("--N", type=int, default=500000)
    ap.add_argument("--L", type=int, default=10000)
    ap.add_argument("--fp64-steps", type=int, default=2, help="timed FP64-form trainings (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=40000, help="oracle sample: rows at full L")
    ap.add_argument("--cpu-nodes", type=int, default=4000, help="oracle sample: nodes for the factor")
    ap.add_argument("--batch-steps", type=int, default=2,
                    help="timed batches of the 256-ELM hidden-size sweep (0 = skip)")
    ap.add_argument("--fp16-steps", type=int, default=2,
                    help="timed FP16-form trainings on the same workload (0 = skip)")
    ap.add_argument("--streamed-steps", type=int, default=2,
                    help="timed trainings of the streamed form (H never stored) on the same workload")
    ap.add_argument("--config-steps", type=int, default=3,
                    help="timed trainings per form of the other named workloads (0 = skip)")
    ap.add_argument("--stage", default=None,
                    choices=["hidden", "gram", "gram64", "rank", "refine", "predict", "copy", "batch", "probes"],
                    help="run one stage alone (for profiling) instead of the benchmark")
    ap.add_argument("--reps", type=int, default=1, help="timed repetitions of --stage")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def node_major(L, N, dtype, dev):
    """An L x N node-major copy laid out as the library lays out its own: rows
    padded to a multiple of 64 elements, so each 64-sample stage of a row the
    16-bit Gram loads is whole cache lines."""
    import torch
    return torch.empty((L, -(-N // 64) * 64), dtype=dtype, device=dev)[:, :N]


def cpu_baseline(prob, rows, nodes):
    """The FP64 oracle on a bounded sample of the workload, scaled to
    trainings/s of the full workload:
      rows part   - hidden layer, Gram and two refinement residual passes on
                    the first `rows` samples at full L (work proportional to N),
                    scaled by N / rows;
      factor part - rank step and beta assembly on the Gram of the first
                    `nodes` hidden nodes (work ~ L^3), scaled by (L / nodes)^3."""
    import numpy as np
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    N, L = prob.N, prob.L
    Xs, Ts = prob.X[:rows], prob.T[:rows]
    t0 = time.perf_counter()
    M, Z = O.gram_streamed(Xs, prob.W, prob.b, Ts, chunk_rows=2000)
    beta0 = np.zeros((L, prob.m))
    for _ in range(2):
        O.ne_gradient_streamed(Xs, prob.W, prob.b, Ts, beta0, chunk_rows=2000)
    t_rows = time.perf_counter() - t0
    Ms = np.ascontiguousarray(M[:nodes, :nodes])
    t1 = time.perf_counter()
    F = O.rank_factor(O.ShapeOnly(rows, nodes), M=Ms)
    for _ in range(3):
        O.apply_pinv(F, None, None, Z=Z[:nodes])
    t_factor = time.perf_counter() - t1
    t_full = t_rows * (N / rows) + t_factor * (L / nodes) ** 3
    return {
        "value": 1.0 / t_full, "unit": "trainings/s", "cores": int(cores), "kind": "oracle",
        "extrapolated": True,
        "measured_s": {"rows_part": round(t_rows, 3), "factor_part": round(t_factor, 3)},
        "scale": {"rows_part": N / rows, "factor_part": (L / nodes) ** 3},
        "sample": (f"FP64 oracle on the first {rows} of {N} rows at full L={L} (hidden, Gram, 2 residual "
                   f"passes: {t_rows:.2f} s, scaled x{N / rows:.0f}) plus its rank step and beta "
                   f"assembly at {nodes} nodes ({t_factor:.2f} s, scaled x(L/{nodes})^3); "
                   f"extrapolated full training {t_full:.0f} s"),
    }


def bench_batch(args, elm, torch, wl, dev):
    """The hidden-size sweep: 256 independent ELMs (N, L log-uniform in
    [1000, 50000] x [64, 2048], d=32, m=5, 10% duplicated nodes) trained by one
    elm_train_batched call, BF16 and FP32 forms (with refinement) and the FP64
    form, to NE residual 1e-10."""
    t0 = time.perf_counter()
    probs = wl.batch_sweep()
    dev_probs = [tuple(torch.from_numpy(a).to(dev) for a in (p.X, p.W, p.b, p.T)) for p in probs]
    H64s = [torch.empty((p.N, p.L), dtype=torch.float64, device=dev) for p in probs]
    betas = [torch.empty((p.L, p.m), dtype=torch.float64, device=dev) for p in probs]
    torch.cuda.synchronize()
    log(f"batch: {len(probs)} ELMs generated and uploaded in {time.perf_counter() - t0:.1f} s")
    out = {"workload": "batch_sweep: 256 ELMs, N log-U[1000,50000], L log-U[64,2048], d=32, m=5, 10% duplicated nodes",
           "count": len(probs), "sum_N_L2": float(sum(p.N * p.L * p.L for p in probs))}
    for precision in ("bf16", "fp32", "fp64"):
        # the library's batch autotuner picks the pivot panel width and the
        # Grams' split/chunk counts for this batch (untimed; kept in the
        # handle's table, which the timed batches then use)
        t_before, t_after = elm.autotune_batch(dev_probs, precision=precision, ir_tol=1e-10, H64s=H64s,
                                               betas=betas)
        log(f"batch {precision} autotune: {t_before:.1f} ms -> {t_after:.1f} ms")
        _, infos, stats = elm.train_batched(dev_probs, precision=precision, ir_tol=1e-10, H64s=H64s,
                                            betas=betas, check=False)
        torch.cuda.synchronize()
        ts = []
        for i in range(args.batch_steps):
            t1 = time.perf_counter()
            _, infos, stats = elm.train_batched(dev_probs, precision=precision, ir_tol=1e-10, H64s=H64s,
                                                betas=betas, check=False)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
            log(f"batch {precision} {i}: {ts[-1] * 1e3:.1f} ms")
        ms = sum(ts) / len(ts) * 1e3
        used = {}
        for inf in infos:
            used[inf["gram_dtype"]] = used.get(inf["gram_dtype"], 0) + 1
        out[precision] = {
            "ms_per_batch": round(ms, 2), "trainings_per_s": round(len(probs) * 1e3 / ms, 2),
            "failed": int(sum(1 for st in stats if st != 0)),
            "max_ne_residual": max(inf["ne_residual"] for inf in infos),
            "gram_dtype_used": used,
            "escalations": int(sum(inf["escalations"] for inf in infos)),
            "max_refine_iterations": max(inf["iterations"] for inf in infos),
            # how the last timed batch ran: host synchronisations with the batch
            # stream, HIP graph launches, problems in shared launches / alone
            "run": elm.batch_report(),
            "autotune": {"ms_before": round(t_before, 2), "ms_after": round(t_after, 2)},
        }
    out["tuned_table"] = elm.tune_table()
    del H64s, betas, dev_probs
    torch.cuda.empty_cache()
    return out


def _median(xs):
    xs = sorted(xs)
    return xs[len(xs) // 2]


def _stage_ms(stages, reps):
    return {k: round(v[0] / reps, 3) for k, v in stages.items() if v[1]}


def bench_configs(args, elm, torch, wl, dev):
    """Trainings/s of the other named workloads, each form timed over
    `config_steps` trainings (median) after one untimed training, with the
    per-stage device times averaged over the timed ones:
      tiny_fp64        N=2000, d=20, L=200 (rank 160), m=2, FP64 form;
      digits_like      N=60000, d=784 (80% zeros), L=2000, m=10, FP32 form;
      mixture_rankdef  N=100000, d=54, L=5000 (rank 4500), m=7, FP64 and FP32
                       forms (rank-deficient by 500 duplicated nodes: the
                       copies set aside, the distinct nodes certified), and
                       the FP64 form again with the certified path off
                       ("fp64_greedy": the greedy pivoted Cholesky, 256-wide
                       panels at this order)."""
    specs = [("tiny_fp64", wl.tiny_fp64, ("fp64",), 20),
             ("digits_like", wl.digits_like, ("fp32",), args.config_steps),
             ("mixture_rankdef", wl.mixture_rankdef, ("fp64", "fp32", "fp64_greedy"), args.config_steps)]
    out = {}
    for name, gen, forms, reps in specs:
        p = gen()
        X, W, b, T = (torch.from_numpy(a).to(dev) for a in (p.X, p.W, p.b, p.T))
        H64 = torch.empty((p.N, p.L), dtype=torch.float64, device=dev)
        entry = {"N": p.N, "d": p.d, "L": p.L, "m": p.m}
        for key in forms:
            form = key.split("_")[0]
            greedy = key.endswith("_greedy")
            old_order = elm.set_option("full_rank_min_order", 0) if greedy else None
            Hlp = None if form == "fp64" else node_major(p.L, p.N, torch.float32, dev)
            res = elm.train(X, W, b, T, precision=form, ir_tol=1e-10, H64=H64, Hlp=Hlp, check_convergence=False)
            torch.cuda.synchronize()
            elm.profile_enable(True)
            ts = []
            for _ in range(max(reps, 1)):
                t0 = time.perf_counter()
                res = elm.train(X, W, b, T, precision=form, ir_tol=1e-10, H64=H64, Hlp=Hlp,
                                check_convergence=False)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            stages = elm.profile_read()
            elm.profile_enable(False)
            if greedy:
                elm.set_option("full_rank_min_order", old_order)
            ms = _median(ts) * 1e3
            fi = res.info["factor"]
            entry[key] = {"ms_per_training": round(ms, 3), "trainings_per_s": round(1e3 / ms, 2),
                           "rank": res.rank, "certified_full_rank": fi["certified_full_rank"],
                           "gram_dtype_used": res.info["gram_dtype"], "ne_residual": res.info["ne_residual"],
                           "refine_iterations": res.info["iterations"],
                           "stage_ms_per_training": _stage_ms(stages, len(ts))}
            log(f"{name} {key}: {ms:.2f} ms, rank {res.rank}, NE {res.info['ne_residual']:.1e}, "
                f"its {res.info['iterations']}")
            del Hlp
        out[name] = entry
        del X, W, b, T, H64
        torch.cuda.empty_cache()
    return out


def run_stage(args):
    """One stage of the path on the precision-form workload (or the batch
    sweep), --reps times after one untimed call, for rocprofv3.  Stages:
    hidden (FP64 H + BF16 copy), gram (BF16 Gram), gram64 (FP64 Gram), rank
    (rank step + factor on the BF16 Gram), refine (factor and one refinement
    pass), predict (Y = H beta), copy (a plain device copy of the FP64 H: the
    reference that scales memory counters), batch (the 256-ELM sweep through
    elm_train_batched, BF16 form)."""
    import torch
    import elm_workloads as wl
    from paper_2011_02436_amd import elm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.stage == "probes":
        # the device ceilings the kernels are held against (one JSON line)
        buf = torch.empty(16 << 30, dtype=torch.uint8, device=dev)
        buf.fill_(1)
        res = {}
        for dt in ("bf16", "fp64"):
            for rnd in (False, True):
                tf, ms = elm.probe_mfma(dt, rnd)
                res[f"mfma_{dt}_{'random' if rnd else 'constant'}_tflops"] = round(tf, 1)
        for rnd in (False, True):
            tf, _ = elm.probe_mfma("fp64", rnd, shape=1)
            res[f"mfma_fp64_4x4x4_four_block_{'random' if rnd else 'constant'}_tflops"] = round(tf, 1)
        res["stream_read_gbs"] = round(elm.probe_stream(buf)[0], 1)
        res["dma_stream_gbs"] = round(elm.probe_dma(buf, resident=False)[0], 1)
        res["dma_l2_resident_gbs"] = round(elm.probe_dma(buf, resident=True)[0], 1)
        print(json.dumps({"probes": res, "buffer_bytes": buf.numel()}), flush=True)
        return
    if args.stage == "batch":
        probs = wl.batch_sweep()
        dp = [tuple(torch.from_numpy(a).to(dev) for a in (q.X, q.W, q.b, q.T)) for q in probs]
        H64s = [torch.empty((q.N, q.L), dtype=torch.float64, device=dev) for q in probs]
        for i in range(args.reps + 1):
            t0 = time.perf_counter()
            elm.train_batched(dp, precision="bf16", ir_tol=1e-10, H64s=H64s, check=False)
            torch.cuda.synchronize()
            log(f"stage batch rep {i}: {(time.perf_counter() - t0) * 1e3:.2f} ms")
        return
    p = wl.smooth_regression(N=args.N, L=args.L)
    X, W, b, T = (torch.from_numpy(a).to(dev) for a in (p.X, p.W, p.b, p.T))
    H64 = torch.empty((p.N, p.L), dtype=torch.float64, device=dev)
    Hb = node_major(p.L, p.N, torch.bfloat16, dev)
    elm.elm_hidden(X, W, b, H=H64, Hlp=Hb)
    torch.cuda.synchronize()

    def run():
        if args.stage == "hidden":
            elm.elm_hidden(X, W, b, H=H64, Hlp=Hb)
        elif args.stage == "gram":
            elm.elm_gram(Hb, "node")
        elif args.stage == "gram64":
            elm.elm_gram(H64, "sample")
        elif args.stage == "rank":
            elm.elm_rank_factor(Hb, "node")
        elif args.stage == "refine":
            f = elm.elm_rank_factor(Hb, "node")
            elm.elm_pinv_solve(f, T, H64, ir_tol=0.0, ir_max_iter=1, check_convergence=False)
        elif args.stage == "predict":
            beta = torch.zeros((p.L, p.m), dtype=torch.float64, device=dev)
            elm.elm_predict_hidden(H64, beta)
        elif args.stage == "copy":
            dst = torch.empty_like(H64)
            dst.copy_(H64)

    run()
    torch.cuda.synchronize()
    for i in range(args.reps):
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        log(f"stage {args.stage} rep {i}: {(time.perf_counter() - t0) * 1e3:.2f} ms")


# The paper's own RBP-ELM training times on GINA (N=3468, d=971), Table 1:
# MATLAB R2016a on an Intel i5-7200U at 2.5 GHz.  Context only: the dataset is
# not available, so the same shapes are trained on synthetic inputs here.
PAPER_TABLE1_S = {500: 1.1875, 1500: 6.8906, 2000: 13.1875}
PAPER_HW = "MATLAB R2016a, Intel i5-7200U 2.50 GHz (Table 1)"


def bench_paper_shapes(elm, torch, wl, dev, reps=5):
    """Median FP64-form training time on GINA-shaped synthetic problems next
    to the paper's Table 1 times for those shapes."""
    rows = []
    for L, paper_s in PAPER_TABLE1_S.items():
        p = wl.gina_shape(L)
        X, W, b, T = (torch.from_numpy(a).to(dev) for a in (p.X, p.W, p.b, p.T))
        elm.train(X, W, b, T, precision="fp64", ir_tol=1e-10)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            res = elm.train(X, W, b, T, precision="fp64", ir_tol=1e-10)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ms = sorted(ts)[len(ts) // 2] * 1e3
        rows.append({"N": p.N, "d": p.d, "L": L, "rank": res.rank, "ms": round(ms, 3),
                     "paper_s": paper_s, "ratio": round(paper_s * 1e3 / ms, 1)})
        log(f"paper shape L={L}: {ms:.2f} ms (paper {paper_s} s)")
    return {"workload": "GINA shape (N=3468, d=971), synthetic inputs, FP64 form", "paper_hw": PAPER_HW,
            "rows": rows}


def traffic_from_profiles(kernel_src, k_splits=None):
    """HBM traffic per launch of the Gram kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source and with the
    K-split count this run uses."""
    path = os.path.join(ROOT, "profiles", "gram_lp256_bf16_N500000_L10000_traffic.txt")
    if not os.path.exists(path):
        return None
    src_hash = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()[:16]
    vals = {}
    for ln in open(path):
        if ":" in ln and not ln.startswith("#"):
            k, v = ln.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256_16") != src_hash:
        return None
    if k_splits is not None and (vals.get("gram_k_splits", "").split() or [""])[0] != str(k_splits):
        return None  # the counters were taken on another tile schedule
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the path has no multi-GPU execution "
              "(it would shard over samples with one Gram all-reduce). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.stage:
        run_stage(args)
        return

    import numpy as np
    import torch

    import elm_workloads as wl
    from paper_2011_02436_amd import elm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    prob = wl.smooth_regression(N=args.N, L=args.L)
    log(f"generated workload N={prob.N} d={prob.d} L={prob.L} m={prob.m} in {time.perf_counter() - t0:.1f} s")
    X = torch.from_numpy(prob.X).to(dev)
    W = torch.from_numpy(prob.W).to(dev)
    b = torch.from_numpy(prob.b).to(dev)
    T = torch.from_numpy(prob.T).to(dev)
    N, L, m = prob.N, prob.L, prob.m
    lp_dtype = {"bf16": torch.bfloat16, "fp16": torch.float16, "fp32": torch.float32}[args.precision]
    H64 = torch.empty((N, L), dtype=torch.float64, device=dev)
    Hlp = node_major(L, N, lp_dtype, dev)
    torch.cuda.synchronize()

    def step():
        # training-set outputs and labels (step 3) come with the training, from
        # its last refinement pass
        return elm.train(X, W, b, T, precision=args.precision, ir_tol=1e-10, H64=H64, Hlp=Hlp,
                         check_convergence=False, outputs=True)

    for i in range(args.warmup):
        res = step()
        torch.cuda.synchronize()
        log(f"warmup {i}: rank {res.rank}, NE residual {res.info['ne_residual']:.2e}, "
            f"iterations {res.info['iterations']}")

    # tile schedule of the BF16 Gram for this shape, picked by the library's
    # autotuner on the warm-up's node-major copy (untimed, once per shape)
    tuned = None
    if args.precision in ("bf16", "fp16") and N >= L:
        splits, tms = elm.autotune_gram(Hlp)
        tuned = {"gram_k_splits": splits, "gram_ms": round(tms, 3)}
        log(f"autotune: Gram with {splits} K splits, {tms:.2f} ms")

    elm.profile_enable(True)
    torch.cuda.synchronize()
    times = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        res = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        log(f"step {i}: {times[-1] * 1e3:.1f} ms, rank {res.rank}, NE residual {res.info['ne_residual']:.2e}, "
            f"its {res.info['iterations']}")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    stages = elm.profile_read()
    elm.profile_enable(False)
    ms_per_step = t_total / args.steps * 1e3
    beta_lp = res.beta.clone()
    info_lp = res.info
    rank_lp = res.rank

    # roofline of the Gram kernel: N L (L + 1) flops per launch (symmetric product)
    gram_ms, gram_n = stages["gram"]
    gram_avg_ms = gram_ms / max(gram_n, 1)
    gram_flops = float(N) * L * (L + 1)
    gram_tflops = gram_flops / (gram_avg_ms * 1e-3) / 1e12 if gram_n else None
    traffic = traffic_from_profiles(os.path.join(ROOT, "paper_2011_02436_amd", "csrc", "gram.hip"),
                                    tuned["gram_k_splits"] if tuned else None)
    stage_ms_per_step = {k: round(v[0] / args.steps, 3) for k, v in stages.items()}

    # FP64 form at equal residual
    fp64 = None
    if args.fp64_steps > 0:
        del Hlp
        torch.cuda.empty_cache()
        r64 = elm.train(X, W, b, T, precision="fp64", ir_tol=1e-10, ir_max_iter=8, H64=H64,
                        check_convergence=False)
        torch.cuda.synchronize()
        ft = []
        for i in range(args.fp64_steps):
            ts = time.perf_counter()
            r64 = elm.train(X, W, b, T, precision="fp64", ir_tol=1e-10, ir_max_iter=8, H64=H64,
                            check_convergence=False, outputs=True)
            torch.cuda.synchronize()
            ft.append(time.perf_counter() - ts)
            log(f"fp64 step {i}: {ft[-1] * 1e3:.1f} ms, rank {r64.rank}, NE residual "
                f"{r64.info['ne_residual']:.2e}, its {r64.info['iterations']}")
        fp64_ms = sum(ft) / len(ft) * 1e3
        diff = (torch.linalg.norm(beta_lp - r64.beta) / torch.linalg.norm(r64.beta)).item()
        fp64 = {"ms_per_step": round(fp64_ms, 2), "trainings_per_s": round(1e3 / fp64_ms, 4),
                "rank": r64.rank, "ne_residual": r64.info["ne_residual"],
                "iterations": r64.info["iterations"],
                "speedup_of_mixed": round(fp64_ms / ms_per_step, 3),
                "beta_rel_diff_mixed_vs_fp64": diff}

    # FP16 form on the same workload (FP16 copy of H in the BF16 copy's memory)
    fp16 = None
    if args.fp16_steps > 0 and args.precision != "fp16":
        Hh = node_major(L, N, torch.float16, dev)
        r16 = elm.train(X, W, b, T, precision="fp16", ir_tol=1e-10, H64=H64, Hlp=Hh, check_convergence=False)
        torch.cuda.synchronize()
        elm.profile_enable(True)
        ht = []
        for i in range(args.fp16_steps):
            ts = time.perf_counter()
            r16 = elm.train(X, W, b, T, precision="fp16", ir_tol=1e-10, H64=H64, Hlp=Hh,
                            check_convergence=False, outputs=True)
            torch.cuda.synchronize()
            ht.append(time.perf_counter() - ts)
            log(f"fp16 step {i}: {ht[-1] * 1e3:.1f} ms, rank {r16.rank}, NE residual "
                f"{r16.info['ne_residual']:.2e}, its {r16.info['iterations']}")
        st16 = elm.profile_read()
        elm.profile_enable(False)
        fp16_ms = sum(ht) / len(ht) * 1e3
        g16_ms, g16_n = st16["gram"]
        fp16 = {"ms_per_step": round(fp16_ms, 2), "trainings_per_s": round(1e3 / fp16_ms, 4),
                "rank": r16.rank, "gram_dtype_used": r16.info["gram_dtype"],
                "ne_residual": r16.info["ne_residual"], "refine_iterations": r16.info["iterations"],
                "ne_history": r16.info["ne_history"],
                "gram_tflops": round(gram_flops / (g16_ms / g16_n * 1e-3) / 1e12, 2) if g16_n else None,
                "stage_ms_per_step": _stage_ms(st16, len(ht))}
        del Hh, r16
        torch.cuda.empty_cache()

    # the streamed form on the same workload: H formed 65536 rows at a time for
    # the Gram and again for every refinement residual, never stored
    streamed = None
    if args.streamed_steps > 0:
        H64 = None          # the stored-H buffers are not needed from here on
        torch.cuda.empty_cache()
        rs = elm.train_streamed(X, W, b, T, precision=args.precision, chunk_rows=65536, ir_tol=1e-10,
                                check_convergence=False)
        torch.cuda.synchronize()
        elm.profile_enable(True)
        sts = []
        for i in range(args.streamed_steps):
            ts = time.perf_counter()
            rs = elm.train_streamed(X, W, b, T, precision=args.precision, chunk_rows=65536, ir_tol=1e-10,
                                    check_convergence=False)
            torch.cuda.synchronize()
            sts.append(time.perf_counter() - ts)
            log(f"streamed step {i}: {sts[-1] * 1e3:.1f} ms, rank {rs.rank}, NE {rs.info['ne_residual']:.2e}, "
                f"its {rs.info['iterations']}")
        stst = elm.profile_read()
        elm.profile_enable(False)
        st_ms = sum(sts) / len(sts) * 1e3
        streamed = {"ms_per_step": round(st_ms, 2), "trainings_per_s": round(1e3 / st_ms, 4),
                    "chunk_rows": 65536, "rank": rs.rank, "gram_dtype_used": rs.info["gram_dtype"],
                    "ne_residual": rs.info["ne_residual"], "refine_iterations": rs.info["iterations"],
                    "beta_rel_diff_vs_stored_h_form": (torch.linalg.norm(rs.beta - beta_lp) /
                                                       torch.linalg.norm(beta_lp)).item(),
                    "stage_ms_per_step": _stage_ms(stst, len(sts)),
                    "h_bytes_not_stored": int(N) * L * (8 + 2)}

    batch = bench_batch(args, elm, torch, wl, dev) if args.batch_steps > 0 else None
    configs = None
    if args.config_steps > 0:
        H64 = None
        torch.cuda.empty_cache()
        configs = bench_configs(args, elm, torch, wl, dev)
    paper = bench_paper_shapes(elm, torch, wl, dev) if args.batch_steps > 0 else None

    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        cpu = cpu_baseline(prob, min(args.cpu_rows, N), min(args.cpu_nodes, L))
        log(f"cpu baseline {time.perf_counter() - t0:.1f} s: {cpu['sample']}")

    certified = int(info_lp["factor"]["certified_full_rank"])
    rank_path = {1: "certified full rank: unpivoted blocked Cholesky whose inverse-factor rows bound every "
                    "greedy pivot above the threshold",
                 2: "duplicated nodes set aside, the distinct nodes certified full rank (unpivoted blocked "
                    "Cholesky whose inverse-factor rows bound every greedy pivot above the threshold)"}.get(
                     certified, "greedy diagonally pivoted Cholesky")
    out = {
        "metric": METRIC,
        "value": round(1e3 / ms_per_step, 4),
        "unit": "trainings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{args.precision}+f64",
        "data": "synthetic",
        "config": {"workload": f"smooth_regression N={N} d={prob.d} L={L} m={m}, {args.precision} Gram "
                               f"+ FP64 rank decision ({rank_path}) + FP64 refinement to NE residual "
                               f"1e-10, plus training-set outputs and labels",
                   "rank_path": rank_path,
                   "N": N, "d": prob.d, "L": L, "m": m, "precision": args.precision},
        "rank": rank_lp,
        "ne_residual": info_lp["ne_residual"],
        "refine_iterations": info_lp["iterations"],
        "ne_history": info_lp["ne_history"],
        "gram_dtype_used": info_lp["gram_dtype"],
        "precision_escalations": info_lp["escalations"],
        "rank_decision": {k: info_lp["factor"][k] for k in
                          ("max_diag", "last_pivot", "first_rejected", "tau", "noise_floor", "reliable",
                           "certified_full_rank")},
        "gram_tflops": round(gram_tflops, 2) if gram_tflops else None,
        "roofline": {
            "kernel": "gram_lp256_kernel" if args.precision != "fp32" else "gram16_kernel<float>",
            "bound": "mfma",
            "achieved": round(gram_tflops, 2) if gram_tflops else None,
            "peak": PEAK_BF16_TFLOPS if args.precision != "fp32" else 157.3,
            "unit": "TFLOP/s",
            "frac": round(gram_tflops / (PEAK_BF16_TFLOPS if args.precision != "fp32" else 157.3), 4)
            if gram_tflops else None,
            "traffic": traffic,
            "avg_launch_ms": round(gram_avg_ms, 3),
            "algorithmic_flops_per_launch": gram_flops,
        },
        "gram_schedule": dict(tuned, chosen_by="elm_autotune_gram") if tuned else None,
        "stage_ms_per_step": stage_ms_per_step,
        "fp64_form": fp64,
        "fp16_form": fp16,
        "streamed_form": streamed,
        "batch_sweep": batch,
        "other_workloads": configs,
        "paper_context": paper,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
