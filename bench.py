"""Benchmark: restricted A-DEF2 solves per second on the 511 x 511 upwind
convection-diffusion Schur complement (k = 32 reference modes, 16 instances
with 10-40 % active, rel. residual 1e-10).

One step = restrict + coarse setup + solve for all 16 instances.
  headline : all 16 instances in one batched launch sequence (precision per
             --precision, default mixed: FP32 operator and panels, FP64
             vectors, FP64 residual replacement)
  plain    : FP64 A-DEF2, one instance at a time
Prints one JSON line (see the contract in the repository README / DESIGN).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=511)
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--precision", choices=["mixed", "fp32", "fp64"], default="mixed")
    ap.add_argument("--inner-rtol", type=float, default=1e-2)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=200,
                    help="oracle iterations timed for the CPU baseline sample")
    return ap.parse_args()


def cpu_baseline(w, S_spec, iters_ref: float, n_iter: int):
    """Time the FP64 oracle on a bounded sample of instance 0: restriction,
    coarse setup and n_iter A-DEF2 iterations; scale to solves/s with the
    iteration count the GPU FP64 path needed (mean over the batch)."""
    import oracle
    from threadpoolctl import threadpool_limits
    inst = w.instances[0]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        I, _, nI = oracle.compact(inst.mask)
        S_II, d_I = oracle.restricted_operator(S_spec, I)
        Zo, kept = oracle.restricted_basis(w.Z, I)
        cs, fb = oracle.coarse_setup(S_II, Zo)
        t1 = time.perf_counter()
        oracle.adef2(S_II, inst.b[I], cs, 1e-30, maxit=n_iter)
        t2 = time.perf_counter()
    t_setup = t1 - t0
    t_it = (t2 - t1) / n_iter
    per_solve = t_setup + iters_ref * t_it
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"instance 0 (n_I={nI}): restriction + QR + coarse setup ({t_setup:.2f} s) and "
                       f"{n_iter} FP64 A-DEF2 iterations ({t_it * 1e3:.2f} ms/iteration), scaled to "
                       f"{iters_ref:.0f} iterations per solve (GPU FP64 mean)"),
            "seconds_per_solve": per_solve}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU runs are not "
                                   "part of this build (instances shard across GPUs with no "
                                   "communication, see DESIGN.md)"}))
        sys.exit(2)
    import torch

    import gen
    from paper_2606_17971_amd import binding as lib

    torch.cuda.set_device(0)
    t = time.time()
    w = gen.c2_workload(n=args.n, k=args.k, B=args.batch)
    op = w.op
    print(f"[bench] workload {w.name} generated in {time.time() - t:.1f}s", file=sys.stderr, flush=True)
    masks = torch.as_tensor(np.stack([i.mask for i in w.instances]), device="cuda")
    bs = torch.as_tensor(np.stack([i.b for i in w.instances]), device="cuda")
    B = args.batch
    prec = {"mixed": lib.MIXED_REFINE, "fp32": lib.FP32_REFINE, "fp64": lib.FP64}[args.precision]

    head = lib.Solver(precision=prec, inner_rtol=args.inner_rtol)
    head.set_reference_factored(op.A, op.alpha, op.shift, w.Z)

    def head_step():
        return head.solve_batched(masks, bs, args.tol)

    for _ in range(args.warmup):
        out = head_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        out = head_step()
        print(f"[bench] headline step {s} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_head = (time.perf_counter() - t0) / args.steps
    head_iters = np.asarray(out["iters"])
    head_rel = np.asarray(out["relres_true"])
    X_head = out["x"].clone()

    plain = None
    if not args.no_plain:
        ps = lib.Solver(precision=lib.FP64)
        ps.set_reference_factored(op.A, op.alpha, op.shift, w.Z)

        def plain_step():
            res = []
            for m in range(B):
                ps.restrict(masks[m])
                res.append(ps.solve(bs[m], args.tol))
            return res

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = plain_step()
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        p_iters = np.array([r.iters for r in res])
        X_plain = torch.stack([r.x for r in res])
        num = torch.linalg.norm(X_head - X_plain, dim=1)
        den = torch.linalg.norm(X_plain, dim=1)
        e_rel = (num / den).cpu().numpy()
        plain = {"solves_per_s": B / t_plain, "ms_per_step": t_plain * 1e3,
                 "iters_mean": float(p_iters.mean()), "iters_max": int(p_iters.max()),
                 "relres_true_max": float(max(r.relres_true for r in res)),
                 "headline_vs_plain_e_rel_max": float(e_rel.max())}
        print(f"[bench] plain step done ({t_plain:.2f}s)", file=sys.stderr, flush=True)

    # roofline: one instrumented headline step, HIP events around every launch
    prof = lib.Solver(precision=prec, inner_rtol=args.inner_rtol, profile=1)
    prof.set_reference_factored(op.A, op.alpha, op.shift, w.Z)
    prof.solve_batched(masks, bs, args.tol)
    st = prof.stats()
    dom = max(st, key=lambda k: st[k]["ms"])
    d = st[dom]
    achieved = d["alg_bytes"] / (d["ms"] * 1e-3) / 1e9 if d["ms"] > 0 else 0.0
    kernels = {k: {"launches": v["launches"], "avg_us": v["ms"] / v["launches"] * 1e3,
                   "alg_GBps": v["alg_bytes"] / (v["ms"] * 1e-3) / 1e9}
               for k, v in st.items() if v["launches"] and v["ms"] > 0}
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                "avg_us": round(d["ms"] / d["launches"] * 1e3, 2), "kernels": kernels}

    cpu = None
    if not args.no_cpu_baseline:
        ref_iters = plain["iters_mean"] if plain else float(head_iters.mean())
        spec = ("factored", op.A, op.alpha, op.shift)
        cpu = cpu_baseline(w, spec, ref_iters, args.cpu_iters)

    value = B / t_head
    line = {
        "metric": "solves/s + HBM GB/s at 511^2 grid; batched+learned vs plain at rel err <=1e-8",
        "value": round(value, 4), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_head * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {lib.MIXED_REFINE: "f32 operator/panels + f64 vectors",
                  lib.FP32_REFINE: "f32 + f64 refinement", lib.FP64: "f64"}[prec],
        "data": "synthetic",
        "config": {"workload": f"cd2d_upwind_{args.n}x{args.n}_k{args.k}_B{B}", "grid": args.n,
                   "N": op.N, "k": args.k, "instances": B, "tol": args.tol,
                   "mode": "batched", "precision": args.precision,
                   "operator": "S = alpha A^T A + shift I (A: 5-point upwind, factored)"},
        "iters": {"mean": float(head_iters.mean()), "min": int(head_iters.min()),
                  "max": int(head_iters.max())},
        "relres_true_max": float(head_rel.max()),
        "plain": plain,
        "speedup_vs_plain": (round(value / plain["solves_per_s"], 3) if plain else None),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
