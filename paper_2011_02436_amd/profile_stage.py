"""Run one stage of the training path on the precision-form workload, for
profiling a single kernel under rocprofv3 (kernel trace or counters).

    python -m paper_2011_02436_amd.profile_stage --stage gram [--N 500000 --L 10000]

Stages: hidden (FP64 H + BF16 copy), gram (BF16 Gram), gram64 (FP64 Gram),
rank (pivoted Cholesky + factor), refine (factor and one refinement pass),
predict (Y = H beta), copy (a plain device copy of the FP64 H, the
reference for scaling memory counters), batch (the 256-ELM hidden-size sweep
through elm_train_batched, BF16 form).  Each stage runs --reps times after
one untimed call.
"""
import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stage", required=True,
                    choices=["hidden", "gram", "gram64", "rank", "refine", "predict", "copy", "batch"])
    ap.add_argument("--N", type=int, default=500000)
    ap.add_argument("--L", type=int, default=10000)
    ap.add_argument("--reps", type=int, default=1)
    args = ap.parse_args()

    import torch
    import elm_workloads as wl
    from paper_2011_02436_amd import elm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.stage == "batch":
        probs = wl.batch_sweep()
        dp = [tuple(torch.from_numpy(a).to(dev) for a in (q.X, q.W, q.b, q.T)) for q in probs]
        H64s = [torch.empty((q.N, q.L), dtype=torch.float64, device=dev) for q in probs]
        for i in range(args.reps + 1):
            t0 = time.perf_counter()
            elm.train_batched(dp, precision="bf16", ir_tol=1e-10, H64s=H64s, check=False)
            torch.cuda.synchronize()
            print(f"[profile_stage] batch rep {i}: {(time.perf_counter() - t0) * 1e3:.2f} ms", flush=True)
        return
    p = wl.smooth_regression(N=args.N, L=args.L)
    X, W, b, T = (torch.from_numpy(a).to(dev) for a in (p.X, p.W, p.b, p.T))
    H64 = torch.empty((p.N, p.L), dtype=torch.float64, device=dev)
    Hb = torch.empty((p.L, p.N), dtype=torch.bfloat16, device=dev)
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
        print(f"[profile_stage] {args.stage} rep {i}: {(time.perf_counter() - t0) * 1e3:.2f} ms", flush=True)


if __name__ == "__main__":
    main()
