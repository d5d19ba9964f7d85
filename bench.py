"""Benchmark: restricted A-DEF2 solves per second on the 511 x 511 upwind
convection-diffusion Schur complement (k = 32 reference modes, 16 instances
with 10-40 % active, rel. residual 1e-10).

One step = MLP inference + basis enrichment + restrict + coarse setup +
solve for all 16 instances.
  headline : all 16 instances in one batched launch sequence with the
             learned enrichment (8 vectors from the problem parameters) and
             precision per --precision (default mixed: FP32 operator and
             panels, FP64 vectors, FP64 residual replacement)
  batched  : the same without enrichment (reference modes only)
  plain    : FP64 A-DEF2, one instance at a time
Before timing, the enrichment is fitted once: GPU solves of --train family
members (snapshots), their POD on the GPU, and --train-steps Adam steps of
the MLP on the GPU.
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
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--force-learned", action="store_true",
                    help="apply the enrichment even when its gain test fails")
    ap.add_argument("--no-batched-compare", action="store_true")
    ap.add_argument("--train", type=int, default=40, help="snapshot solves for the enrichment")
    ap.add_argument("--pod", type=int, default=32, help="POD modes the MLP combines")
    ap.add_argument("--train-steps", type=int, default=400)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--snap-tol", type=float, default=1e-8)
    ap.add_argument("--rpt", type=int, default=0, choices=[0, 1, 2],
                    help="rows per thread of the iteration kernels (0 = tuned)")
    ap.add_argument("--w-mode", type=int, default=0, choices=[0, 1, 2, 3, 4],
                    help="1 = read W, 2 = W-free tile-major, 3 = W-free per instance, "
                         "4 = tile-major boundary form, 0 = tuned")
    ap.add_argument("--w-boundary", type=int, default=2, choices=[0, 1, 2],
                    help="boundary form of W for eigen reference modes: 0 off, 1 on, "
                         "2 when every reference mode is an eigenvector")
    ap.add_argument("--counter-run", action="store_true",
                    help="short run for rocprofv3 counter passes: one headline solve capped at "
                         "--counter-maxit iterations, then a 256 MiB device copy of known size; "
                         "prints no benchmark line")
    ap.add_argument("--counter-maxit", type=int, default=192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pod-merge", action="store_true",
                    help="skip the POD safe-merge comparator arm (reported, never the headline)")
    ap.add_argument("--pod-merge-p", type=int, default=8, help="POD candidates of the comparator arm")
    ap.add_argument("--tau-safe", type=float, default=1e4)
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


def fit_enrichment(solver, args, lib):
    """Fit the learned enrichment of solver on GPU data: snapshot solves of
    args.train family members (parameter seed 700, disjoint from the timed
    instances), POD of the snapshots, MLP training.  Returns a summary."""
    import torch

    import gen
    t0 = time.perf_counter()
    th = gen.c2_thetas(args.train, 700)
    insts = [gen.c2_family_instance(args.n, t) for t in th]
    m_tr = torch.as_tensor(np.stack([i.mask for i in insts]), device="cuda")
    b_tr = torch.as_tensor(np.stack([i.b for i in insts]), device="cuda")
    th_tr = torch.as_tensor(th.astype(np.float32), device="cuda")
    t1 = time.perf_counter()
    snap = solver.solve_batched(m_tr, b_tr, args.snap_tol)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"[bench] {args.train} snapshot solves in {t2 - t1:.1f}s", file=sys.stderr, flush=True)
    X = snap["x"]
    Phi, sig = solver.pod(X.T, args.pod)
    if not sig[0] > 0:
        raise RuntimeError("snapshot solves returned zero solutions; cannot fit the enrichment")
    solver.learned_set_params(gen.mlp_params(1))
    solver.learned_prepare(m_tr, b_tr, X, th_tr)
    hist = solver.learned_train(args.train_steps, lr=args.lr)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    print(f"[bench] POD + {args.train_steps} training steps in {t3 - t2:.1f}s "
          f"(loss {hist[0]:.4f} -> {hist[-1]:.4f})", file=sys.stderr, flush=True)
    # gain test: batched solves of 16 training members (tolerance of the
    # timed solves) with and without the enrichment; it is kept only if it
    # saves time (enrichment adds 8 columns to every panel pass)
    sel = slice(0, min(16, args.train))

    def timed_solve(theta, tol):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        o = solver.solve_batched(m_tr[sel], b_tr[sel], tol, theta=theta)
        torch.cuda.synchronize()
        return time.perf_counter() - ta, o

    timed_solve(None, 1e-6)                # kernel variants are tuned on the first solve
    timed_solve(th_tr[sel], 1e-6)
    t_plain, o_plain = timed_solve(None, args.tol)
    t_lrn, o_lrn = timed_solve(th_tr[sel], args.tol)
    keep = t_lrn < 0.98 * t_plain
    print(f"[bench] gain test on 16 training members: plain basis {t_plain:.2f}s, learned {t_lrn:.2f}s "
          f"-> enrichment {'kept' if keep else 'not used'}", file=sys.stderr, flush=True)
    return {"snapshots": args.train, "snapshot_tol": args.snap_tol, "pod_modes": args.pod,
            "sigma_ratio_last": float(sig[-1] / sig[0]), "train_steps": args.train_steps,
            "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
            "snapshot_s": round(t2 - t1, 2), "fit_s": round(t3 - t2, 2),
            "inputs_s": round(t1 - t0, 2),
            "gain_test": {"instances": 16, "plain_s": round(t_plain, 3), "learned_s": round(t_lrn, 3),
                          "plain_iters_mean": float(np.mean(o_plain["iters"])),
                          "learned_iters_mean": float(np.mean(o_lrn["iters"])),
                          "learned_used": int(np.sum(o_lrn["learned"])), "kept": bool(keep)}}, Phi


def pod_merge_arm(args, lib, op, Z, Phi, masks, bs, prec, tune, t_head, head_iters):
    """The paper's non-learned enrichment as a comparator: the first p POD
    modes of the same snapshots appended after the reference modes and
    merged per instance by the conditioning rule (tau_safe), solving the
    timed instances on a solver of its own."""
    import torch
    s = lib.Solver(precision=prec, inner_rtol=args.inner_rtol, **tune)
    s.set_reference_factored(op.A, op.alpha, op.shift, Z)
    s.set_pod_modes(Phi[:, :args.pod_merge_p])
    s.pod_enrich(args.pod_merge_p, args.tau_safe)
    s.solve_batched(masks, bs, 1e-6)                 # kernel variants are tuned on the first solve
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    o = s.solve_batched(masks, bs, args.tol)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    s.close()
    it = np.asarray(o["iters"])
    B = masks.shape[0]
    print(f"[bench] POD safe-merge arm: {t:.2f}s ({B / t:.3f} solves/s), iterations {it.mean():.0f} "
          f"vs {head_iters.mean():.0f}", file=sys.stderr, flush=True)
    return {"candidates": args.pod_merge_p, "tau_safe": args.tau_safe, "solves_per_s": round(B / t, 4),
            "vs_headline": round(t_head / t, 3), "iters_mean": float(it.mean()),
            "headline_iters_mean": float(head_iters.mean()),
            "cond_E_max": float(np.max(o["cond_E"])),
            "relres_true_max": float(np.asarray(o["relres_true"]).max())}


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary in
    profiles/, or None when there is none for it or the kernel sources changed
    since the counters were taken."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in ("dev_common.h", "dev_kernels.h"):
        with open(os.path.join(ROOT, "paper_2606_17971_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    sha = h.hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.md"))):
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith(("#", "|", "`")):
                key, _, val = line.partition(":")
                kv[key.strip()] = val.strip()
        if kv.get("kernel") == kernel and kv.get("kernel-source-sha256") == sha:
            return {"traffic": float(kv["traffic-bytes-per-launch"]),
                    "traffic_alg_bytes": float(kv["alg-bytes-per-launch"]),
                    "traffic_source": os.path.relpath(path, ROOT)}
    return None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; a batch of instances would "
                                   "shard across GPUs with no communication, which is not "
                                   "implemented"}))
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

    tune = dict(rows_per_thread=args.rpt, w_mode=args.w_mode, w_boundary=args.w_boundary)
    head = lib.Solver(precision=prec, inner_rtol=args.inner_rtol, **tune)
    head.set_reference_factored(op.A, op.alpha, op.shift, w.Z)
    thetas = torch.as_tensor(np.stack([i.theta for i in w.instances]).astype(np.float32), device="cuda")
    learned, Phi = (None, None) if args.no_learned else fit_enrichment(head, args, lib)
    # the enrichment is applied only when its gain test passed
    apply_learned = learned is not None and (args.force_learned or learned["gain_test"]["kept"])
    if args.counter_run:
        head.set_opts(maxit=args.counter_maxit)
    use_theta = thetas if apply_learned else None

    def head_step():
        return head.solve_batched(masks, bs, args.tol, theta=use_theta)

    if args.counter_run:
        out = head_step()
        torch.cuda.synchronize()
        src = torch.empty(32 << 20, dtype=torch.float64, device="cuda").uniform_()
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"counter_run": True, "iters": np.asarray(out["iters"]).tolist(),
                          "variant": list(head.variant()[:2]), "copy_bytes_each_way": src.numel() * 8}))
        return
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
    v_rpt, v_wm, v_ms = head.variant()
    head_rel = np.asarray(out["relres_true"])
    X_head = out["x"].clone()

    batched = None
    if apply_learned and not args.no_batched_compare:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ob = head.solve_batched(masks, bs, args.tol)
        torch.cuda.synchronize()
        t_b = time.perf_counter() - t0
        bi = np.asarray(ob["iters"])
        batched = {"solves_per_s": B / t_b, "ms_per_step": t_b * 1e3, "iters_mean": float(bi.mean()),
                   "iters_max": int(bi.max()), "relres_true_max": float(np.asarray(ob["relres_true"]).max()),
                   "iters_per_instance": bi.tolist(),
                   "cond_E_max": float(np.max(ob["cond_E"]))}
        print(f"[bench] batched (reference modes only) done ({t_b:.2f}s)", file=sys.stderr, flush=True)

    pod_arm = None
    if Phi is not None and not args.no_pod_merge:
        try:
            pod_arm = pod_merge_arm(args, lib, op, w.Z, Phi, masks, bs, prec, tune, t_head, head_iters)
        except Exception as e:            # reported, never fatal for the headline
            pod_arm = {"error": str(e)}

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
    prof = lib.Solver(precision=prec, inner_rtol=args.inner_rtol, profile=1,
                      rows_per_thread=v_rpt, w_mode=v_wm, w_boundary=args.w_boundary)
    prof.set_reference_factored(op.A, op.alpha, op.shift, w.Z)
    if apply_learned:
        prof.set_pod_modes(Phi)
        prof.learned_set_params(head.learned_get_params())
    prof.solve_batched(masks, bs, args.tol, theta=use_theta)
    st = prof.stats()
    dom = max(st, key=lambda k: st[k]["ms"])
    d = st[dom]
    achieved = d["alg_bytes"] / (d["ms"] * 1e-3) / 1e9 if d["ms"] > 0 else 0.0
    kernels = {k: {"launches": v["launches"], "avg_us": v["ms"] / v["launches"] * 1e3,
                   "alg_GBps": v["alg_bytes"] / (v["ms"] * 1e-3) / 1e9}
               for k, v in st.items() if v["launches"] and v["ms"] > 0}
    kp = ((args.k + (8 if apply_learned else 0)) + 7) // 8 * 8
    vt, mt = {lib.MIXED_REFINE: ("double", "float"), lib.FP32_REFINE: ("float", "float"),
              lib.FP64: ("double", "double")}[prec]
    if dom in ("update_tm", "pupdate_tm"):
        inst = f"k_{dom}<{mt}, {kp}>"
    elif dom == "update":
        inst = f"k_{dom}<{vt}, {mt}, {kp}, {v_rpt}, {'true' if args.w_boundary else 'false'}>"
    else:
        inst = f"k_{dom}<{vt}, {mt}, {kp}, {v_rpt}>"
    tr = measured_traffic(inst)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr["traffic"] if tr else None,
                "kernel": dom, "instantiation": inst,
                "alg_bytes_per_launch": round(d["alg_bytes"] / d["launches"]),
                "avg_us": round(d["ms"] / d["launches"] * 1e3, 2), "kernels": kernels}
    if tr:
        roofline["traffic_alg_bytes_same_launches"] = tr["traffic_alg_bytes"]
        roofline["traffic_source"] = tr["traffic_source"]

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
        "dtype": {lib.MIXED_REFINE: "f32+f64", lib.FP32_REFINE: "f32+f64", lib.FP64: "f64"}[prec],
        "dtype_detail": {lib.MIXED_REFINE: "FP32 operator and Z/W panels, FP64 vectors and residuals",
                         lib.FP32_REFINE: "FP32 operator, panels and vectors, FP64 refinement",
                         lib.FP64: "FP64 throughout"}[prec],
        "data": "synthetic",
        "config": {"workload": f"cd2d_upwind_{args.n}x{args.n}_k{args.k}_B{B}", "grid": args.n,
                   "N": op.N, "k": args.k, "instances": B, "tol": args.tol,
                   "mode": "batched+learned" if learned is not None else "batched",
                   "learned_applied": bool(apply_learned),
                   "precision": args.precision,
                   "operator": "S = alpha A^T A + shift I (A: 5-point upwind, factored)"},
        "iters": {"mean": float(head_iters.mean()), "min": int(head_iters.min()),
                  "max": int(head_iters.max())},
        "variant": {"rows_per_thread": v_rpt, "w_mode": v_wm, "tuned": args.rpt == 0 or args.w_mode == 0,
                    "trial_ms": [round(float(t), 3) for t in v_ms]},
        "learned_used": (int(np.asarray(out["learned"]).sum()) if apply_learned else 0),
        "cond_E": {"min": float(np.min(out["cond_E"])), "max": float(np.max(out["cond_E"]))},
        "iters_per_instance": np.asarray(out["iters"]).tolist(),
        "learned_fit": learned,
        "batched_reference_modes": batched,
        "pod_merge": pod_arm,
        "relres_true_max": float(head_rel.max()),
        "plain": plain,
        "speedup_vs_plain": (round(value / plain["solves_per_s"], 3) if plain else None),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
