"""GPU parity on the other workloads: the 255^2 heterogeneous-diffusion sweep
at its full size (256 instances, per-instance operator scale, tol 1e-8), a 3D
two-material case, and the mixed-precision mode on small batches.

Full-size checks compare sampled instances with x* from the oracle (banded
Cholesky with double-double refinement), compare iteration counts with the
oracle's FP64 A-DEF2 on two of them, and check the true residual of every
instance.  Bar (FP64 and mixed): e_rel <=
max(1e-8, 2 e_rel of the oracle's FP64 A-DEF2 at the same tolerance)."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[case] {msg}", flush=True)


def _factored(op, a=1.0, c=None):
    return ("factored", op.A, a * op.alpha, op.shift if c is None else c)


def _xstar(S, mask, b):
    I, _, _ = oracle.compact(mask)
    S_II, _ = oracle.restricted_operator(S, I)
    return I, S_II, oracle.exact_solution(S_II, b[I])


@pytest.fixture(scope="module")
def c3full():
    return gen.c3_workload(n=255, k=32, B=256)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_c3_full_batch_sampled(lib, c3full, prec):
    w = c3full
    op = w.op
    B = len(w.instances)
    case(f"c3 255^2 B={B} k=32 tol 1e-8 {prec}")
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    a = np.array([i.a for i in w.instances])
    c = np.array([i.c for i in w.instances]) - a * op.shift
    s = lib.Solver(precision=lib.MIXED_REFINE if prec == "mixed" else lib.FP64)
    s.set_reference_factored(op.A, op.alpha, op.shift, w.Z)
    out = s.solve_batched(masks, bs, 1e-8, a=a, c=c)
    X = out["x"].cpu().numpy()
    st = np.asarray(out["status"])
    print(f"   iters mean {np.mean(out['iters']):.0f} max {np.max(out['iters'])}; "
          f"statuses {np.unique(st, return_counts=True)}", flush=True)
    assert np.all(st == 0)
    rel = np.asarray(out["relres_true"])
    print(f"   true relative residual max {rel.max():.2e}", flush=True)
    # mixed: the FP64 residual b - S x decides the stop, so it meets tol.
    # FP64: as in the paper, the recurrence residual decides; rounding in the
    # components of the largest eigenvalues makes the FP64 iterate's true
    # residual drift above the recurrence one (cond(S_II) up to ~1e9 here)
    # while e_rel, dominated by the smooth components, stays ~1e-11.  The
    # oracle's own FP64 A-DEF2 drifts the same way: compared on the sampled
    # instances below; e_rel against x* is the accuracy bar.
    assert np.all(rel <= (2e-8 if prec == "mixed" else 1e-5))
    nI = (masks == 0).sum(axis=1)
    np.testing.assert_array_equal(out["n_inactive"], nI)
    assert np.all(X[masks == 1] == 0.0)
    # sampled instances: smallest and largest inactive set, and four more
    order = np.argsort(nI)
    sample = [int(order[0]), int(order[-1])] + [int(order[j]) for j in (51, 102, 153, 204)]
    for j, m in enumerate(sample):
        inst = w.instances[m]
        S = _factored(op, inst.a, inst.c)
        I, _, xs = _xstar(S, inst.mask, inst.b)
        e = oracle.rel_err(X[m, I], xs)
        print(f"   m={m} n_I={nI[m]} e_rel={e:.2e} iters {out['iters'][m]}", flush=True)
        # the oracle's own FP64 A-DEF2 reaches 2e-11..7e-11 here, so the bar is 1e-8
        assert e <= 1e-8, (m, e)
        if prec == "fp64" and j in (0, 2):      # iteration parity on two of them (CPU time)
            ref = oracle.solve_instance(S, w.Z, inst.mask, inst.b, 1e-8)
            print(f"      oracle iters {ref.iters}; true relres GPU {rel[m]:.2e} oracle {ref.relres_true:.2e}",
                  flush=True)
            assert abs(int(out["iters"][m]) - ref.iters) <= max(2, ref.iters // 100)
            # the same drift of the true residual as the oracle's FP64 loop
            assert rel[m] <= 10 * ref.relres_true + 1e-9


@pytest.mark.parametrize("prec,op_fused", [("mixed", 0), ("fp64", 0), ("fp64", 1), ("mixed", 1)])
def test_3d_two_material(lib, prec, op_fused):
    """3D 7-point operator at 23^3.  op_fused = 1 forces the fused operator
    pass with the run-time diagonal loop (7 diagonals; the 529-row reach of a
    grid plane still fits in LDS at this size)."""
    w = gen.c5_workload(n=23, k=16, B=3)
    op = w.op
    case(f"3d n=23 k=16 B=3 {prec} op_fused={op_fused}")
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    s = lib.Solver(precision=lib.MIXED_REFINE if prec == "mixed" else lib.FP64, op_fused=op_fused)
    s.set_reference_factored(op.A, op.alpha, op.shift, w.Z)
    out = s.solve_batched(masks, bs, 1e-10)
    X = out["x"].cpu().numpy()
    S = _factored(op)
    for m, inst in enumerate(w.instances):
        I, _, xs = _xstar(S, inst.mask, inst.b)
        ref = oracle.solve_instance(S, w.Z, inst.mask, inst.b, 1e-10)
        e = oracle.rel_err(X[m, I], xs)
        print(f"   m={m} e_rel={e:.2e} iters {out['iters'][m]} oracle {ref.iters}", flush=True)
        assert out["status"][m] == 0
        assert e <= max(1e-8, 2 * oracle.rel_err(ref.x[I], xs)), (m, e)
        if prec == "fp64":
            assert abs(int(out["iters"][m]) - ref.iters) <= 2
    if op_fused == 1:
        assert s.op_variant()[0] == 1 and s.op_variant()[3] == 1


@pytest.mark.parametrize("form", ["assembled", "factored"])
def test_mixed_batched_small(lib, form):
    w = gen.c2_workload(n=95, k=16, B=4)
    op = w.op
    case(f"mixed batched cd2d n=95 B=4 {form}")
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    s = lib.Solver(precision=lib.MIXED_REFINE)
    if form == "factored":
        s.set_reference_factored(op.A, op.alpha, op.shift, w.Z)
        S = _factored(op)
    else:
        s.set_reference(op.S(), w.Z)
        S = op.S()
    out = s.solve_batched(masks, bs, 1e-10)
    X = out["x"].cpu().numpy()
    for m, inst in enumerate(w.instances):
        I, _, xs = _xstar(S, inst.mask, inst.b)
        ref = oracle.solve_instance(S, w.Z, inst.mask, inst.b, 1e-10)
        e = oracle.rel_err(X[m, I], xs)
        assert out["status"][m] == 0
        assert out["relres_true"][m] <= 1e-10
        assert e <= max(1e-8, 2 * oracle.rel_err(ref.x[I], xs)), (m, e)
        # FP32 segments with FP64 residual replacement stay close to FP64 counts
        assert int(out["iters"][m]) <= 1.5 * ref.iters + 50
