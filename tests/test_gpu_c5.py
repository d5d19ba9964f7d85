"""GPU parity on the 3D two-material workload (conjugate-heat-transfer-like
diffusion, kappa in {1, 1000}, S = K^2 / h^3 + 1e-2 h^3 I, k = 64 reference
modes built by the paper's coarse-grid route: eigenvectors of the coarse
operator, prolonged linearly and orthonormalised (Sec. "Coarse-grid
eigenmode prolongation", Alg. 4), 15-35 % active, tol 1e-8).

Two routes to the exact solution (both stated per test):
  * 31^3 (coarse grid 15^3): x* of each restricted system by a direct
    factorisation with double-double refinement (oracle route O9(i)); the
    GPU's e_rel must be within max(1e-8, 2 e_rel of the oracle's own FP64
    A-DEF2), and FP64 iteration counts within 2 of the oracle's.
  * 127^3 x 16 (coarse grid 31^3, the benchmark workload): a direct solve of
    1.3-1.7 M unknowns of the squared 3D operator is beyond the test budget,
    so the bar there is the true residual ||b_I - S_II x_I|| / ||b_I||
    evaluated in double-double on the CPU for sampled instances (every
    instance's FP64 residual is also checked), plus the structure checks
    (active entries exactly 0, inactive counts).  That size runs FP64
    segments restarted from the true residual (FP64_REFINE), which stops on
    b - S x.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import gen
import oracle
from oracle import basis as OB

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[case] {msg}", flush=True)


def _spec(op):
    return ("factored", op.A, op.alpha, op.shift)


@pytest.fixture(scope="module")
def c5small():
    w = gen.c5_workload(n=31, k=64, B=4, nc=15)
    Zo, kept = OB.coarse_basis(w.meta["Zc"], 31, 15, 3)
    spec = _spec(w.op)

    def xstar(inst):
        I, _, _ = oracle.compact(inst.mask)
        F, _ = oracle.restricted_operator(spec, I)
        return I, oracle.exact_solution(F, inst.b[I])

    with ThreadPoolExecutor(4) as ex:
        xs = list(ex.map(xstar, w.instances))
    return w, Zo, xs


PRECS = {"fp64": "FP64", "mixed": "MIXED_REFINE", "fp64_refine": "FP64_REFINE"}


@pytest.mark.parametrize("prec", ["fp64", "mixed", "fp64_refine"])
def test_c5_small_against_xstar(lib, c5small, prec):
    w, Zo, xs = c5small
    op = w.op
    case(f"3d two-material 31^3 k=64 (prolonged from 15^3) B=4 {prec}; route: direct x*")
    s = lib.Solver(precision=getattr(lib, PRECS[prec]))
    Zg = s.prolong_basis(w.meta["Zc"], 3, 31, 15)
    assert Zg.shape[1] == Zo.shape[1]
    # the GPU's prolonged basis spans the oracle's (Alg. 4 on both sides)
    Zgn = Zg.cpu().numpy()
    assert np.linalg.norm(Zgn - Zo @ (Zo.T @ Zgn)) <= 1e-10 * np.sqrt(Zo.shape[1])
    s.set_reference_factored(op.A, op.alpha, op.shift, Zg)
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    out = s.solve_batched(masks, bs, 1e-8)
    X = out["x"].cpu().numpy()
    spec = _spec(op)
    for m, inst in enumerate(w.instances):
        I, x_star = xs[m]
        ref = oracle.solve_instance(spec, Zo, inst.mask, inst.b, 1e-8)
        e = oracle.rel_err(X[m, I], x_star)
        e_or = oracle.rel_err(ref.x[I], x_star)
        print(f"   m={m} n_I={len(I)} e_rel={e:.2e} (oracle {e_or:.2e}) iters {out['iters'][m]} "
              f"oracle {ref.iters} status {out['status'][m]}", flush=True)
        assert out["status"][m] == 0
        assert e <= max(1e-8, 2 * e_or), (m, e)
        if prec == "fp64":
            assert abs(int(out["iters"][m]) - ref.iters) <= 2
        elif prec == "fp64_refine":
            # FP64 segments restarted from the true residual: the stop is
            # decided by b - S x, a few restarts cost a few iterations
            assert out["relres_true"][m] <= 1e-8
            assert int(out["iters"][m]) <= 1.5 * ref.iters + 50
        else:
            assert out["relres_true"][m] <= 1e-8
            # FP32 values of K with 1:1000 coefficient jumps: u32 cond(K) is
            # ~1e-1, so the FP32 segments resolve the smooth error slowly and
            # the FP64 residual replacements carry the accuracy (measured:
            # about 3x the FP64 iterations); bounded, not matched
            assert int(out["iters"][m]) <= 4 * ref.iters + 100
        assert np.all(X[m, inst.mask == 1] == 0.0)


def test_c5_full_size_batched(lib):
    """127^3 x 16, k = 64, FP64 segments with residual replacement (the
    benchmark's 3D arm).  With the 1:1000 jumps the FP32 operator values
    slow the mixed-precision segments down (see the 31^3 test), and plain
    FP64, which stops on the recurrence residual, leaves a true residual of
    ~1e-6 at this size (cond(S_II) ~ 1e13): FP64_REFINE stops on b - S x."""
    w = gen.c5_workload(n=127, k=64, B=16, nc=31)
    op = w.op
    case("3d two-material 127^3 k=64 (prolonged from 31^3) B=16 fp64_refine; route: double-double residual")
    s = lib.Solver(precision=lib.FP64_REFINE)
    Zg = s.prolong_basis(w.meta["Zc"], 3, 127, 31)
    print(f"   prolonged basis: {Zg.shape[1]} columns", flush=True)
    assert Zg.shape[1] >= 60
    s.set_reference_factored(op.A, op.alpha, op.shift, Zg)
    del Zg
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    out = s.solve_batched(masks, bs, 1e-8)
    st = np.asarray(out["status"])
    it = np.asarray(out["iters"])
    print(f"   iterations mean {it.mean():.0f} min {it.min()} max {it.max()}; statuses "
          f"{np.unique(st, return_counts=True)}; variant {s.variant()[:2]}", flush=True)
    assert np.all(st == 0)
    print(f"   FP64 true residual max {np.max(out['relres_true']):.2e}", flush=True)
    assert np.all(np.asarray(out["relres_true"]) <= 1e-8)
    nI = (masks == 0).sum(axis=1)
    np.testing.assert_array_equal(out["n_inactive"], nI)
    X = out["x"].cpu().numpy()
    assert np.all(X[masks == 1] == 0.0)
    spec = _spec(op)

    def dd_rel(m):
        inst = w.instances[m]
        I, _, _ = oracle.compact(inst.mask)
        F, _ = oracle.restricted_operator(spec, I)
        r = oracle.dd_residual(F, X[m, I], inst.b[I])
        return np.linalg.norm(r) / np.linalg.norm(inst.b[I])

    with ThreadPoolExecutor(2) as ex:
        rel = list(ex.map(dd_rel, (0, 15)))
    for m, r in zip((0, 15), rel):
        print(f"   m={m} double-double relative residual {r:.2e}", flush=True)
        # the stop is b - S x <= 1e-8 ||b|| evaluated in FP64; the
        # double-double value differs by the FP64 evaluation error only
        assert r <= 2e-8
