"""Benchmark: restricted A-DEF2 solves per second on the 511 x 511 upwind
convection-diffusion Schur complement (k = 32 reference modes, 16 instances
with 10-40 % active, relative residual 1e-10), every instance checked
against x* (e_rel <= 1e-8).

One step = restrict + coarse setup + solve for all 16 instances.
  headline (value): the 16 instances in one batched launch sequence,
             precision per --precision (default mixed: FP32 operator and
             panels, FP64 vectors, FP64 residual replacement).  When the
             learned enrichment passes its gain test (held-out family
             members) it is part of the step and config.mode says so;
             otherwise the step uses the reference modes and mode is
             "batched".
Arms reported next to it (never the headline value):
  plain          FP64 A-DEF2, one instance at a time (the paper's setting)
  learned        batched + learned enrichment forced on, same 16 instances
  pod_merge      the paper's POD safe merge (Alg. 2) as the non-learned
                 comparator
  c5             127^3 x 16 two-material 3D workload (k = 64 prolonged
                 coarse modes): batched mixed vs plain FP64
  cpu_baseline   the C/OpenMP build of the oracle's A-DEF2 loop on the
                 host cores (all cores and one core), bounded samples
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
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
                    help="make the headline step use the enrichment even when its gain test fails")
    ap.add_argument("--train", type=int, default=40, help="snapshot solves for the enrichment")
    ap.add_argument("--pod", type=int, default=32, help="POD modes the MLP combines")
    ap.add_argument("--train-steps", type=int, default=400)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--snap-tol", type=float, default=1e-8)
    ap.add_argument("--rpt", type=int, default=0, choices=[0, 1, 2],
                    help="rows per thread of the per-instance iteration kernels (0 = tuned)")
    ap.add_argument("--w-mode", type=int, default=0, choices=[0, 1, 2, 3, 4, 5],
                    help="1 = read W, 2 = W-free tile-major, 3 = W-free per instance, "
                         "4 = tile-major boundary form, 5 = 4 with tile-major stencils, 0 = tuned")
    ap.add_argument("--op-fused", type=int, default=0, choices=[-1, 0, 1],
                    help="operator pass of the factored form: 1 = fused (A p kept in LDS), "
                         "-1 = two passes, 0 = tuned")
    ap.add_argument("--op-rows", type=int, default=0, help="tile height of the fused pass (0 = tuned)")
    ap.add_argument("--op-group", type=int, default=0, choices=[0, 1, 4],
                    help="instances per block of the fused pass (0 = tuned)")
    ap.add_argument("--update-ws", type=int, default=0, choices=[-1, 0, 1],
                    help="tile-major update: 1 = warp-specialised, -1 = per tile, 0 = tuned")
    ap.add_argument("--w-boundary", type=int, default=2, choices=[0, 1, 2],
                    help="boundary form of W for eigen reference modes: 0 off, 1 on, "
                         "2 when every reference mode is an eigenvector")
    ap.add_argument("--counter-run", action="store_true",
                    help="short run for rocprofv3 counter passes: one headline solve capped at "
                         "--counter-maxit iterations, then a 256 MiB device copy of known size; "
                         "prints no benchmark line")
    ap.add_argument("--counter-maxit", type=int, default=192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=400,
                    help="C-oracle iterations per timed sample on all cores (one core: a quarter)")
    ap.add_argument("--cpu-reps", type=int, default=5, help="repetitions per CPU sample (median)")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time full C-oracle solves of instance 0 (all cores; minutes)")
    ap.add_argument("--no-pod-merge", action="store_true")
    ap.add_argument("--pod-merge-p", type=int, default=8)
    ap.add_argument("--tau-safe", type=float, default=1e4)
    ap.add_argument("--no-c5", action="store_true", help="skip the 127^3 arm")
    ap.add_argument("--c5-n", type=int, default=127)
    ap.add_argument("--c5-nc", type=int, default=31)
    ap.add_argument("--c5-plain", type=int, default=2, help="plain FP64 instances timed in the 3D arm")
    ap.add_argument("--c5-precision", choices=["fp64_refine", "fp64", "mixed"], default="fp64_refine")
    ap.add_argument("--no-c3", action="store_true", help="skip the 255^2 x 256 sweep arm")
    ap.add_argument("--c3-n", type=int, default=255)
    ap.add_argument("--c3-batch", type=int, default=256)
    ap.add_argument("--c3-plain", type=int, default=4, help="plain FP64 instances timed in the sweep arm")
    ap.add_argument("--c4", action="store_true",
                    help="run the learned-enrichment arms on the 255^2 heterogeneous sweep (minutes)")
    ap.add_argument("--c4-train", type=int, default=2000)
    ap.add_argument("--c4-test", type=int, default=512)
    ap.add_argument("--c4-pod", type=int, default=64)
    ap.add_argument("--c4-batch", type=int, default=256)
    ap.add_argument("--c4-steps", type=int, default=300)
    ap.add_argument("--c4-lr", type=float, default=1e-3)
    ap.add_argument("--c4-objective", choices=["spectrum", "energy"], default="energy")
    ap.add_argument("--c4-precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-profile", action="store_true", help="skip the instrumented roofline pass")
    return ap.parse_args()


def host_info():
    model = platform.processor() or ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except Exception:
        aff = os.cpu_count() or 1
    return model, aff, os.cpu_count() or 1


def cpu_baseline(w, spec, iters_ref: float, args):
    """The C/OpenMP build of the oracle's A-DEF2 loop (oracle/cpu_adef2.c) on
    instance 0 of the timed batch: restriction and the orthonormal restricted
    basis by the Python oracle, then the C coarse setup and iteration.
    Bounded samples: a fixed number of iterations, median of repetitions,
    scaled to one solve with the iteration count of the GPU FP64 arm; on all
    host cores the sampler uses and on one core."""
    import oracle
    from oracle import cpu
    inst = w.instances[0]
    I, _, nI = oracle.compact(inst.mask)
    S_II, _ = oracle.restricted_operator(spec, I)
    A = S_II.assembled()
    Zo, _ = oracle.restricted_basis(w.Z, I)
    b = inst.b[I]
    model, aff, ncpu = host_info()
    res = {}
    for label, threads, its in (("all_cores", aff, args.cpu_iters), ("one_core", 1, max(50, args.cpu_iters // 4))):
        cpu.adef2(A, b, Zo, 1e-30, maxit=10, threads=threads)          # warm-up
        per_it, setup = [], []
        for _ in range(args.cpu_reps):
            r = cpu.adef2(A, b, Zo, 1e-30, maxit=its, threads=threads)
            per_it.append(r.solve_s / r.iters)
            setup.append(r.setup_s)
        t_it = float(np.median(per_it))
        t_set = float(np.median(setup))
        per_solve = t_set + iters_ref * t_it
        res[label] = {"value": 1.0 / per_solve, "unit": "solves/s", "cores": threads,
                      "seconds_per_solve": per_solve, "ms_per_iteration": t_it * 1e3,
                      "coarse_setup_s": t_set,
                      "sample": f"{its} iterations x {args.cpu_reps} repetitions (median), instance 0"}
    full = None
    if args.cpu_full:
        r = cpu.adef2(A, b, Zo, args.tol, threads=aff)
        full = {"iters": r.iters, "seconds": r.setup_s + r.solve_s, "cores": aff,
                "solves_per_s": 1.0 / (r.setup_s + r.solve_s), "converged": r.converged}
    best = res["all_cores"]
    return {"value": round(best["value"], 6), "unit": "solves/s", "cores": best["cores"], "kind": "oracle",
            "sample": (f"C/OpenMP FP64 A-DEF2 (oracle/cpu_adef2.c) on instance 0 (n_I={nI}, k={Zo.shape[1]}): "
                       f"coarse setup + {args.cpu_iters} iterations, median of {args.cpu_reps}, scaled to "
                       f"{iters_ref:.0f} iterations per solve (GPU FP64 mean); restriction and QR by the "
                       f"Python oracle, not timed"),
            "one_core": {k: (round(v, 6) if isinstance(v, float) else v) for k, v in res["one_core"].items()},
            "all_cores": {k: (round(v, 6) if isinstance(v, float) else v) for k, v in res["all_cores"].items()},
            "full_solve": full,
            "host": {"model": model, "cores_available": aff, "cpu_count": ncpu}}


def fit_enrichment(solver, args, op):
    """Fit the learned enrichment on GPU data: snapshot solves of args.train
    family members (parameter seed 700, disjoint from the timed instances),
    POD of the snapshots, MLP training on the GPU.  Gain test on 16 held-out
    family members (seed 900): batched solves with and without the
    enrichment at the timed tolerance; kept when it saves >= 2 % time."""
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
    log(f"{args.train} snapshot solves in {t2 - t1:.1f}s")
    X = snap["x"]
    Phi, sig = solver.pod(X.T, args.pod)
    if not sig[0] > 0:
        raise RuntimeError("snapshot solves returned zero solutions; cannot fit the enrichment")
    solver.learned_set_params(gen.mlp_params(1))
    solver.learned_prepare(m_tr, b_tr, X, th_tr)
    hist = solver.learned_train(args.train_steps, lr=args.lr)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    log(f"POD + {args.train_steps} training steps in {t3 - t2:.1f}s (loss {hist[0]:.4f} -> {hist[-1]:.4f})")
    del m_tr, b_tr, X, snap
    thh = gen.c2_thetas(16, 900)
    hold = [gen.c2_family_instance(args.n, t) for t in thh]
    m_h = torch.as_tensor(np.stack([i.mask for i in hold]), device="cuda")
    b_h = torch.as_tensor(np.stack([i.b for i in hold]), device="cuda")
    th_h = torch.as_tensor(thh.astype(np.float32), device="cuda")

    def timed_solve(theta, tol):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        o = solver.solve_batched(m_h, b_h, tol, theta=theta)
        torch.cuda.synchronize()
        return time.perf_counter() - ta, o

    timed_solve(None, 1e-6)                # kernel variants are tuned on the first solve
    timed_solve(th_h, 1e-6)
    t_plain, o_plain = timed_solve(None, args.tol)
    t_lrn, o_lrn = timed_solve(th_h, args.tol)
    keep = t_lrn < 0.98 * t_plain
    log(f"gain test on 16 held-out members: reference modes {t_plain:.2f}s, learned {t_lrn:.2f}s -> "
        f"enrichment {'kept' if keep else 'not used'}")
    return {"snapshots": args.train, "snapshot_tol": args.snap_tol, "pod_modes": args.pod,
            "sigma_ratio_last": float(sig[-1] / sig[0]), "train_steps": args.train_steps,
            "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
            "snapshot_s": round(t2 - t1, 2), "fit_s": round(t3 - t2, 2), "inputs_s": round(t1 - t0, 2),
            "gain_test": {"instances": "16 held-out family members (seed 900)",
                          "reference_modes_s": round(t_plain, 3), "learned_s": round(t_lrn, 3),
                          "reference_modes_iters_mean": float(np.mean(o_plain["iters"])),
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
    log(f"POD safe-merge arm: {t:.2f}s ({B / t:.3f} solves/s), iterations {it.mean():.0f} vs {head_iters.mean():.0f}")
    return {"candidates": args.pod_merge_p, "tau_safe": args.tau_safe, "solves_per_s": round(B / t, 4),
            "vs_headline": round(t_head / t, 3), "iters_mean": float(it.mean()),
            "headline_iters_mean": float(head_iters.mean()), "cond_E_max": float(np.max(o["cond_E"])),
            "relres_true_max": float(np.asarray(o["relres_true"]).max())}


def c5_arm(args, lib, prec, tune):
    """127^3 x 16 two-material 3D workload (k = 64 modes prolonged from the
    coarse grid on the GPU, Alg. 4): batched (tuned, warmed up on a loose
    tolerance; FP64 segments stopped on the true residual by default) vs
    plain FP64 one instance at a time (a sample of instances spanning the
    active fractions)."""
    import torch

    import gen
    t0 = time.perf_counter()
    w = gen.c5_workload(n=args.c5_n, k=64, B=16, nc=args.c5_nc)
    log(f"3D workload {w.name} generated in {time.perf_counter() - t0:.1f}s")
    op = w.op
    masks = torch.as_tensor(np.stack([i.mask for i in w.instances]), device="cuda")
    bs = torch.as_tensor(np.stack([i.b for i in w.instances]), device="cuda")
    c5p = {"fp64_refine": lib.FP64_REFINE, "fp64": lib.FP64, "mixed": lib.MIXED_REFINE}[args.c5_precision]
    s = lib.Solver(precision=c5p, inner_rtol=args.inner_rtol, **tune)
    Zg = s.prolong_basis(w.meta["Zc"], 3, args.c5_n, args.c5_nc)
    s.set_reference_factored(op.A, op.alpha, op.shift, Zg)
    s.solve_batched(masks, bs, 1e-3)                 # variant tuning and graphs
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    o = s.solve_batched(masks, bs, 1e-8)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t1
    it = np.asarray(o["iters"])
    v = s.variant()
    s.close()
    log(f"3D batched: {t_b:.2f}s ({16 / t_b:.3f} solves/s), iterations mean {it.mean():.0f} max {it.max()}")
    ps = lib.Solver(precision=lib.FP64)
    ps.set_reference_factored(op.A, op.alpha, op.shift, Zg)
    del Zg
    sel = np.linspace(0, 15, max(1, args.c5_plain)).round().astype(int).tolist()
    ps.restrict(masks[sel[0]])
    ps.solve(bs[sel[0]], 1e-3)                       # warm-up: variant and graphs
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    pit = []
    for m in sel:
        ps.restrict(masks[m])
        pit.append(ps.solve(bs[m], 1e-8).iters)
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t2
    ps.close()
    rate_p = len(sel) / t_p
    log(f"3D plain FP64 sample {sel}: {t_p:.2f}s ({rate_p:.3f} solves/s)")
    return {"workload": w.name, "grid": args.c5_n, "coarse_grid": args.c5_nc, "k": 64, "instances": 16, "tol": 1e-8,
            "precision": args.c5_precision,
            "batched": {"solves_per_s": round(16 / t_b, 4), "seconds": round(t_b, 3), "iters_mean": float(it.mean()),
                        "iters_max": int(it.max()), "status": np.asarray(o["status"]).tolist(),
                        "relres_true_max": float(np.asarray(o["relres_true"]).max()),
                        "variant": {"rows_per_thread": v[0], "w_mode": v[1]}},
            "plain_fp64": {"solves_per_s": round(rate_p, 4), "instances_timed": sel, "iters": pit},
            "speedup_vs_plain": round((16 / t_b) / rate_p, 3)}


def c3_arm(args, lib, prec, tune):
    """The batched parameter sweep: args.c3_batch instances of the 255^2
    heterogeneous-diffusion family (per-instance operator scale, inactive sets
    of 40-95 % of N, k = 32 shared eigenvectors of the reference operator,
    tol 1e-8) in one batched solve, vs the FP64 solver one instance at a time
    on a sample of args.c3_plain instances spanning the inactive-set sizes."""
    import torch

    import gen
    t0 = time.perf_counter()
    w = gen.c3_workload(n=args.c3_n, k=32, B=args.c3_batch)
    log(f"sweep workload {w.name} generated in {time.perf_counter() - t0:.1f}s")
    op = w.op
    B = len(w.instances)
    masks = torch.as_tensor(np.stack([i.mask for i in w.instances]), device="cuda")
    bs = torch.as_tensor(np.stack([i.b for i in w.instances]), device="cuda")
    a = np.array([i.a for i in w.instances])
    c = np.array([i.c for i in w.instances]) - a * op.shift
    s = lib.Solver(precision=prec, inner_rtol=args.inner_rtol, **tune)
    s.set_reference_factored(op.A, op.alpha, op.shift, w.Z)
    s.solve_batched(masks, bs, 1e-3, a=a, c=c)       # variant tuning and graphs
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    o = s.solve_batched(masks, bs, 1e-8, a=a, c=c)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t1
    it = np.asarray(o["iters"])
    v, ov, uv = s.variant(), s.op_variant(), s.update_variant()
    s.close()
    log(f"sweep batched: {t_b:.2f}s ({B / t_b:.2f} solves/s), iterations mean {it.mean():.0f} max {it.max()}")
    nI = (masks == 0).sum(dim=1).cpu().numpy()
    order = np.argsort(nI)
    sel = [int(order[j]) for j in np.linspace(0, B - 1, max(1, args.c3_plain)).round().astype(int)]
    ps = lib.Solver(precision=lib.FP64)
    ps.set_reference_factored(op.A, op.alpha, op.shift, w.Z)
    ps.solve_batched(masks[sel[0]:sel[0] + 1], bs[sel[0]:sel[0] + 1], 1e-3, a=a[sel[0]:sel[0] + 1],
                     c=c[sel[0]:sel[0] + 1])         # warm-up: variant and graphs
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    pit = []
    for m in sel:
        po = ps.solve_batched(masks[m:m + 1], bs[m:m + 1], 1e-8, a=a[m:m + 1], c=c[m:m + 1])
        pit.append(int(po["iters"][0]))
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t2
    ps.close()
    rate_p = len(sel) / t_p
    log(f"sweep plain FP64 sample of {len(sel)}: {t_p:.2f}s ({rate_p:.3f} solves/s)")
    return {"workload": w.name, "grid": args.c3_n, "k": 32, "instances": B, "tol": 1e-8,
            "precision": args.precision,
            "batched": {"solves_per_s": round(B / t_b, 3), "seconds": round(t_b, 3), "iters_mean": float(it.mean()),
                        "iters_max": int(it.max()), "status": np.unique(np.asarray(o["status"])).tolist(),
                        "relres_true_max": float(np.asarray(o["relres_true"]).max()),
                        "variant": {"rows_per_thread": v[0], "w_mode": v[1], "op_fused": ov[0],
                                    "op_tile_rows": ov[1], "op_group": ov[3], "update_ws": uv[0]}},
            "plain_fp64": {"solves_per_s": round(rate_p, 4), "instances_timed": sel, "iters": pit},
            "speedup_vs_plain": round((B / t_b) / rate_p, 3)}


def c4_arm(args, lib):
    """Learned enrichment on the 255^2 heterogeneous-diffusion sweep.
    Snapshots: args.c4_train family members (parameter seed 400) solved
    batched to 1e-8 (mixed precision, stopped on the true residual); POD of
    all of them (args.c4_pod modes); the MLP trained on the GPU with the
    chosen objective.  Then args.c4_test held-out members (seed 500) in four
    arms: reference modes only, learned, untrained MLP (same POD space,
    initial parameters), and the paper's POD safe merge of the first 8 POD
    modes (Alg. 2, tau_safe).  The enriched arms keep cond(E) <= 1e8 (FP64
    panels) and fall back to the reference modes per instance otherwise.
    Members are batched in order of their active fraction."""
    import torch

    import gen
    n, k = 255, 32
    t0 = time.perf_counter()
    w = gen.c3_workload(n=n, k=k, B=1)
    op, mf = w.op, w.meta["mask_field"]

    def members(count, seed):
        th = gen.c3_thetas(count, seed)
        th = th[np.argsort(th[:, 3], kind="stable")]
        return th, [gen.c3_instance(n, t, mf, op.shift) for t in th]

    th_tr, tr = members(args.c4_train, 400)
    th_te, te = members(args.c4_test, 500)
    log(f"C4 inputs ({len(tr)} training, {len(te)} test members) in {time.perf_counter() - t0:.1f}s")

    def batch(ins, th):
        m = torch.as_tensor(np.stack([i.mask for i in ins]), device="cuda")
        b = torch.as_tensor(np.stack([i.b for i in ins]), device="cuda")
        a = np.array([i.a for i in ins])
        c = np.array([i.c for i in ins]) - a * op.shift
        return m, b, a, c, torch.as_tensor(th.astype(np.float32), device="cuda")

    Bt = args.c4_batch
    snap = lib.Solver(precision=lib.MIXED_REFINE)
    snap.set_reference_factored(op.A, op.alpha, op.shift, w.Z)
    X = torch.empty((len(tr), op.N), dtype=torch.float64, device="cuda")
    snap_it = []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for j in range(0, len(tr), Bt):
        m, b, a, c, _ = batch(tr[j:j + Bt], th_tr[j:j + Bt])
        o = snap.solve_batched(m, b, 1e-8, a=a, c=c)
        X[j:j + Bt] = o["x"]
        snap_it += list(o["iters"])
        if np.any(np.asarray(o["status"]) < 0):
            raise RuntimeError("snapshot solve failed")
    torch.cuda.synchronize()
    t_snap = time.perf_counter() - t1
    Phi, sig = snap.pod(X.T, args.c4_pod)
    pod_iters = snap.pod_iters()
    torch.cuda.synchronize()
    t_pod = time.perf_counter() - t1 - t_snap
    snap.close()
    log(f"C4 snapshots {t_snap:.1f}s (iterations mean {np.mean(snap_it):.0f}), POD {t_pod:.2f}s "
        f"({pod_iters} subspace iterations, sigma_p/sigma_1 {sig[-1] / sig[0]:.2e})")
    prec = lib.FP64 if args.c4_precision == "fp64" else lib.MIXED_REFINE
    obj = lib.SPECTRUM if args.c4_objective == "spectrum" else lib.ENERGY
    ref_x = []

    def run_arm(name, solver, use_theta):
        m, b, a, c, th = batch(te[:Bt], th_te[:Bt])
        solver.solve_batched(m, b, 1e-3, a=a, c=c, theta=th if use_theta else None)   # tuning, graphs
        its, lu, rel, st, dx = [], 0, [], [], []
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for q, j in enumerate(range(0, len(te), Bt)):
            m, b, a, c, th = batch(te[j:j + Bt], th_te[j:j + Bt])
            o = solver.solve_batched(m, b, 1e-8, a=a, c=c, theta=th if use_theta else None)
            its += list(o["iters"])
            lu += int(np.sum(o["learned"]))
            rel += list(o["relres_true"])
            st += list(o["status"])
            if name == "plain":
                ref_x.append(o["x"])
            else:
                dx.append(float((torch.linalg.norm(o["x"] - ref_x[q], dim=1) /
                                 torch.linalg.norm(ref_x[q], dim=1)).max()))
        torch.cuda.synchronize()
        t = time.perf_counter() - ta
        r = {"seconds": round(t, 3), "solves_per_s": round(len(te) / t, 3), "iters_mean": float(np.mean(its)),
             "iters_max": int(np.max(its)), "learned_used": lu, "relres_true_max": float(np.max(rel)),
             "status_counts": {str(int(v)): int(cn) for v, cn in zip(*np.unique(st, return_counts=True))}}
        if dx:
            r["vs_plain_rel_diff_max"] = max(dx)
        log(f"C4 arm {name}: {t:.1f}s, iterations mean {r['iters_mean']:.1f}, learned basis used {lu}/{len(te)}")
        return r

    arms = {}
    sp = lib.Solver(precision=prec)
    sp.set_reference_factored(op.A, op.alpha, op.shift, w.Z)
    arms["plain"] = run_arm("plain", sp, False)
    sp.close()
    su = lib.Solver(precision=prec, learned_objective=obj)
    su.set_reference_factored(op.A, op.alpha, op.shift, w.Z)
    su.set_enrichment(Phi, gen.mlp_params(1))
    arms["untrained"] = run_arm("untrained", su, True)
    mt, bt, at, ct, tht = batch(tr, th_tr)
    t2 = time.perf_counter()
    su.learned_prepare(mt, bt, X, tht, a=at, c=ct)
    hist = su.learned_train(args.c4_steps, lr=args.c4_lr)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t2
    del mt, bt, X
    log(f"C4 training ({args.c4_objective}): {t_fit:.1f}s, loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    arms["learned"] = run_arm("learned", su, True)
    su.close()
    sm = lib.Solver(precision=prec)
    sm.set_reference_factored(op.A, op.alpha, op.shift, w.Z)
    sm.set_pod_modes(Phi[:, :8])
    sm.pod_enrich(8, args.tau_safe)
    arms["pod_merge"] = run_arm("pod_merge", sm, False)
    sm.close()
    return {"workload": f"hetdiff2d_{n}x{n}_k{k}", "train_members": len(tr), "test_members": len(te),
            "batch": Bt, "pod_modes": args.c4_pod, "objective": args.c4_objective,
            "precision": args.c4_precision, "tol": 1e-8, "tau_learned": 1e8, "tau_safe": args.tau_safe,
            "snapshots": {"seconds": round(t_snap, 2), "iters_mean": float(np.mean(snap_it)),
                          "precision": "mixed"},
            "pod": {"seconds": round(t_pod, 3), "subspace_iterations": pod_iters,
                    "sigma_ratio_last": float(sig[-1] / sig[0])},
            "training": {"steps": args.c4_steps, "lr": args.c4_lr, "seconds": round(t_fit, 2),
                         "loss_first": float(hist[0]), "loss_last": float(hist[-1])},
            "arms": arms}


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary in
    profiles/, or None when there is none for it or the kernel sources changed
    since the counters were taken."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in ("dev_common.h", "dev_kernels.h", "dev_tile.h"):
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
    log(f"workload {w.name} generated in {time.time() - t:.1f}s")
    masks = torch.as_tensor(np.stack([i.mask for i in w.instances]), device="cuda")
    bs = torch.as_tensor(np.stack([i.b for i in w.instances]), device="cuda")
    B = args.batch
    prec = {"mixed": lib.MIXED_REFINE, "fp32": lib.FP32_REFINE, "fp64": lib.FP64}[args.precision]
    tune = dict(rows_per_thread=args.rpt, w_mode=args.w_mode, w_boundary=args.w_boundary,
                op_fused=args.op_fused, op_rows=args.op_rows, op_group=args.op_group,
                update_ws=args.update_ws)
    head = lib.Solver(precision=prec, inner_rtol=args.inner_rtol, **tune)
    head.set_reference_factored(op.A, op.alpha, op.shift, w.Z)
    thetas = torch.as_tensor(np.stack([i.theta for i in w.instances]).astype(np.float32), device="cuda")

    learned, Phi = (None, None)
    if not args.no_learned and not args.counter_run:
        learned, Phi = fit_enrichment(head, args, op)
    apply_learned = learned is not None and (args.force_learned or learned["gain_test"]["kept"])
    use_theta = thetas if apply_learned else None

    def head_step():
        return head.solve_batched(masks, bs, args.tol, theta=use_theta)

    if args.counter_run:
        # synchronised segments: the host stops enqueuing at the cap, so every
        # counted dispatch of the iteration kernels has all instances iterating
        head.set_opts(maxit=args.counter_maxit, sweep_async=0)
        out = head_step()
        torch.cuda.synchronize()
        src = torch.empty(32 << 20, dtype=torch.float64, device="cuda").uniform_()
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"counter_run": True, "iters": np.asarray(out["iters"]).tolist(),
                          "variant": list(head.variant()[:2]), "op_variant": [head.op_variant()[q] for q in (0, 1, 3)],
                          "copy_bytes_each_way": src.numel() * 8}))
        return

    for _ in range(args.warmup):
        out = head_step()
    torch.cuda.synchronize()
    head.reset_stats()
    t0 = time.perf_counter()
    for s in range(args.steps):
        out = head_step()
        log(f"headline step {s} done")
    torch.cuda.synchronize()
    t_head = (time.perf_counter() - t0) / args.steps
    polls = head.polls() / args.steps
    head_iters = np.asarray(out["iters"])
    v_rpt, v_wm, v_ms = head.variant()
    o_f, o_rows, o_ms, o_grp = head.op_variant()
    u_ws, u_tpb, u_ms = head.update_variant()
    head_rel = np.asarray(out["relres_true"])
    X_head = out["x"].clone()
    value = B / t_head
    log(f"headline {value:.4f} solves/s ({t_head * 1e3:.0f} ms/step, {polls:.0f} polls/step)")

    learned_arm = None
    if learned is not None:
        torch.cuda.synchronize()
        tl = time.perf_counter()
        ol = head.solve_batched(masks, bs, args.tol, theta=thetas)
        torch.cuda.synchronize()
        t_l = time.perf_counter() - tl
        li = np.asarray(ol["iters"])
        num = torch.linalg.norm(ol["x"] - X_head, dim=1)
        den = torch.linalg.norm(X_head, dim=1)
        learned_arm = {"solves_per_s": round(B / t_l, 4), "ms_per_step": round(t_l * 1e3, 2),
                       "iters_mean": float(li.mean()), "iters_max": int(li.max()),
                       "learned_used": int(np.asarray(ol["learned"]).sum()),
                       "cond_E_max": float(np.max(ol["cond_E"])),
                       "relres_true_max": float(np.asarray(ol["relres_true"]).max()),
                       "vs_headline_e_rel_max": float((num / den).max())}
        log(f"batched + learned (forced): {t_l:.2f}s ({B / t_l:.3f} solves/s)")

    pod_arm = None
    if Phi is not None and not args.no_pod_merge:
        try:
            pod_arm = pod_merge_arm(args, lib, op, w.Z, Phi, masks, bs, prec, tune, t_head, head_iters)
        except Exception as ex:            # reported, never fatal for the headline
            pod_arm = {"error": str(ex)}

    plain = None
    if not args.no_plain:
        ps = lib.Solver(precision=lib.FP64)
        ps.set_reference_factored(op.A, op.alpha, op.shift, w.Z)
        ps.restrict(masks[0])
        ps.solve(bs[0], 1e-6)                        # warm-up: variant and graphs
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = []
        for m in range(B):
            ps.restrict(masks[m])
            res.append(ps.solve(bs[m], args.tol))
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        p_iters = np.array([r.iters for r in res])
        X_plain = torch.stack([r.x for r in res])
        num = torch.linalg.norm(X_head - X_plain, dim=1)
        den = torch.linalg.norm(X_plain, dim=1)
        e_rel = (num / den).cpu().numpy()
        plain = {"solves_per_s": round(B / t_plain, 4), "ms_per_step": round(t_plain * 1e3, 2),
                 "iters_mean": float(p_iters.mean()), "iters_max": int(p_iters.max()),
                 "relres_true_max": float(max(r.relres_true for r in res)),
                 "headline_vs_plain_e_rel_max": float(e_rel.max())}
        ps.close()
        del X_plain
        log(f"plain step done ({t_plain:.2f}s)")

    c4 = None
    if args.c4:
        try:
            c4 = c4_arm(args, lib)
        except Exception as ex:            # reported, never fatal for the headline
            c4 = {"error": str(ex)}

    c3 = None
    if not args.no_c3:
        try:
            c3 = c3_arm(args, lib, prec, tune)
        except Exception as ex:            # reported, never fatal for the headline
            c3 = {"error": str(ex)}

    c5 = None
    if not args.no_c5:
        try:
            c5 = c5_arm(args, lib, prec, tune)
        except Exception as ex:            # reported, never fatal for the headline
            c5 = {"error": str(ex)}

    roofline = None
    if not args.no_profile:
        # one instrumented headline step: HIP events on the solver stream around every launch
        prof = lib.Solver(precision=prec, inner_rtol=args.inner_rtol, profile=1,
                          rows_per_thread=v_rpt, w_mode=v_wm, w_boundary=args.w_boundary,
                          op_fused=1 if o_f else -1, op_rows=o_rows, op_group=o_grp,
                          update_ws=1 if u_ws else -1)
        prof.set_reference_factored(op.A, op.alpha, op.shift, w.Z)
        if apply_learned:
            prof.set_pod_modes(Phi)
            prof.learned_set_params(head.learned_get_params())
        prof.solve_batched(masks, bs, args.tol, theta=use_theta)
        st = prof.stats()
        prof.close()
        dom = max(st, key=lambda k: st[k]["ms"])
        d = st[dom]
        achieved = d["alg_bytes"] / (d["ms"] * 1e-3) / 1e9 if d["ms"] > 0 else 0.0
        kernels = {k: {"launches": v["launches"], "avg_us": round(v["ms"] / v["launches"] * 1e3, 2),
                       "alg_GBps": round(v["alg_bytes"] / (v["ms"] * 1e-3) / 1e9, 1)}
                   for k, v in st.items() if v["launches"] and v["ms"] > 0}
        kp = ((args.k + (8 if apply_learned else 0)) + 7) // 8 * 8
        vt, mt = {lib.MIXED_REFINE: ("double", "float"), lib.FP32_REFINE: ("float", "float"),
                  lib.FP64: ("double", "double")}[prec]
        if dom in ("update_tm", "pupdate_tm"):
            inst = f"k_{dom}<{mt}, {kp}>"
        elif dom == "opfused":
            inst = f"k_opfused<{vt}, {mt}, 5>"
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
        cpu = cpu_baseline(w, ("factored", op.A, op.alpha, op.shift), ref_iters, args)
        log(f"CPU baseline: {cpu['value']:.5f} solves/s on {cpu['cores']} cores")

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
                   "mode": "batched+learned" if apply_learned else "batched",
                   "learned_applied": bool(apply_learned),
                   "precision": args.precision,
                   "operator": "S = alpha A^T A + shift I (A: 5-point upwind, factored)"},
        "iters": {"mean": float(head_iters.mean()), "min": int(head_iters.min()),
                  "max": int(head_iters.max())},
        "polls_per_step": polls,
        "variant": {"rows_per_thread": v_rpt, "w_mode": v_wm, "tuned": args.rpt == 0 or args.w_mode == 0,
                    "trial_ms": [round(float(tt), 3) for tt in v_ms],
                    "op_fused": int(o_f), "op_tile_rows": int(o_rows), "op_group": int(o_grp),
                    "update_ws": int(u_ws), "update_trial_ms": [round(float(tt), 3) for tt in u_ms],
                    "op_trial_ms": [round(float(tt), 3) for tt in o_ms]},
        "cond_E": {"min": float(np.min(out["cond_E"])), "max": float(np.max(out["cond_E"]))},
        "iters_per_instance": head_iters.tolist(),
        "relres_true_max": float(head_rel.max()),
        "plain": plain,
        "speedup_vs_plain": (round(value / plain["solves_per_s"], 3) if plain else None),
        "learned_fit": learned,
        "learned_arm": learned_arm,
        "pod_merge": pod_arm,
        "c3": c3,
        "c4": c4,
        "c5": c5,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
