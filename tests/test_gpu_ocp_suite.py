"""The 2D optimal-control suite (2d_asym, 2d_sym, 2d_nonsep) end to end on the
GPU: the primal active-set loop, then cold Jacobi-PCG (k = 0) and raw
reference-eigenmode deflation (r = 40 sine modes, the exact eigenvectors of
M) on each final inactive-set system.

100^2: against the oracle on 6 instances per problem (active sets bit-exact,
outer counts equal, cold and r = 16 iteration counts within 1 %; with only
16 modes at this size deflation can cost iterations on 2d_asym and 2d_sym,
1249 vs 1071 in the oracle, so no ordering is asserted).
300^2, 30 instances: against the numbers the paper prints
(tests/golden/ocp_2d_suite.txt): mean cold iterations within 2 % (measured:
equal to the unit) and the r = 40 iteration reduction within 10 points.
The deflated counts are a loose pin: they depend on the A-DEF2 loop form,
where this library follows the cited A-DEF2 recurrence rather than the
loop as printed in Alg. 1, and on the order of modes inside degenerate
eigenvalue groups; measured reductions are 3-7 points below the printed
ones while the cold counts agree exactly."""
import os

import numpy as np
import pytest

import gen
from oracle.active_set import active_set, coupled_rhs
from oracle.solver import compact, jacobi_pcg, restricted_operator, solve_instance

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(__file__)
TOL = 1e-10


def case(msg):
    print(f"[case] {msg}", flush=True)


def printed():
    rows = {}
    with open(os.path.join(HERE, "golden", "ocp_2d_suite.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            rows[t[0]] = dict(cold300=int(t[3]), cold500=int(t[5]), red40=float(t[10]))
    return rows


def _rhs(w, masks):
    spec = ("factored", w.op.A, w.op.alpha, w.op.shift)
    return np.stack([coupled_rhs(spec, w.y_d[m], w.psi[m], masks[m]) for m in range(masks.shape[0])])


def _run(lib, w, k, n):
    """Active-set loop with k sine modes, then cold and deflated solves of the final systems."""
    Z = gen.sine_modes_2d(n, k)[0]
    s = lib.Solver(precision=lib.FP64)
    s.set_reference_factored(w.op.A, w.op.alpha, w.op.shift, Z)
    out = s.active_set_batched(w.y_d, w.psi, tau=w.tau, tol=TOL, max_outer=20)
    masks = out["masks"].cpu().numpy()
    b = _rhs(w, masks)
    defl = s.solve_batched(masks, b, TOL)
    s.close()
    c = lib.Solver(precision=lib.FP64)
    c.set_reference_factored(w.op.A, w.op.alpha, w.op.shift, None)
    cold = c.solve_batched(masks, b, TOL)
    c.close()
    return out, masks, cold, defl


@pytest.mark.parametrize("name", gen.OCP_2D)
def test_suite_100_against_oracle(lib, name):
    n, B = 100, 6
    case(f"{name} {n}^2 x {B}: active set, cold (k=0) and r=16 solves vs oracle")
    w = gen.ocp_2d(name, n=n, B=B)
    out, masks, cold, defl = _run(lib, w, 16, n)
    spec = ("factored", w.op.A, w.op.alpha, w.op.shift)
    Z = gen.sine_modes_2d(n, 16)[0]
    for m in range(B):
        y_ref, a_ref, k_ref, conv = active_set(spec, w.y_d[m], w.psi[m], tau=w.tau)
        I, _, _ = compact(a_ref)
        S_II, _ = restricted_operator(spec, I)
        b_ref = coupled_rhs(spec, w.y_d[m], w.psi[m], a_ref)
        it_ref = jacobi_pcg(S_II, b_ref[I], TOL).iters
        it_defl = solve_instance(spec, Z, a_ref, b_ref, TOL).iters
        print(f"   m={m} outer={out['outer'][m]} (oracle {k_ref}) |A|={int(masks[m].sum())} "
              f"(oracle {int(a_ref.sum())}) cold={cold['iters'][m]} (oracle {it_ref}) "
              f"r16={defl['iters'][m]} (oracle {it_defl}) status={out['status'][m]}/{cold['status'][m]}/{defl['status'][m]}",
              flush=True)
        assert out["status"][m] == 0 and cold["status"][m] == 0 and defl["status"][m] == 0
        assert out["outer"][m] == k_ref
        assert np.array_equal(masks[m], a_ref)
        assert abs(int(cold["iters"][m]) - it_ref) <= max(2, 0.01 * it_ref)
        assert abs(int(defl["iters"][m]) - it_defl) <= max(2, 0.01 * it_defl)


@pytest.mark.parametrize("name", gen.OCP_2D)
def test_suite_300_replicates_printed_counts(lib, name):
    n, B = 300, 30
    ref = printed()[name]
    case(f"{name} {n}^2 x {B}: cold and r=40 iteration counts vs the printed tables")
    w = gen.ocp_2d(name, n=n, B=B)
    out, masks, cold, defl = _run(lib, w, 40, n)
    assert np.all(out["status"] == 0) and np.all(cold["status"] == 0)
    assert np.all(defl["status"] == 0)
    assert np.all((out["outer"] >= 2) & (out["outer"] <= 4))
    mc = float(np.mean(cold["iters"]))
    md = float(np.mean(defl["iters"]))
    red = 100.0 * (1.0 - md / mc)
    red_inst = 100.0 * float(np.mean(1.0 - defl["iters"] / cold["iters"]))
    frac = masks.mean(axis=1)
    print(f"   outer {sorted(set(out['outer'].tolist()))}, active {frac.mean():.3f} "
          f"[{frac.min():.3f}, {frac.max():.3f}]", flush=True)
    print(f"   cold mean {mc:.1f} (printed {ref['cold300']}), r=40 mean {md:.1f}, reduction "
          f"{red:.1f} % (per-instance mean {red_inst:.1f} %; printed {ref['red40']:.0f} %)", flush=True)
    assert abs(mc - ref["cold300"]) <= 0.02 * ref["cold300"]
    assert abs(red - ref["red40"]) <= 10.0


@pytest.mark.parametrize("name", gen.OCP_2D)
def test_suite_500_cold_counts(lib, name):
    """The paper's largest 2D grid: mean cold Jacobi-PCG iterations over 30
    instances on the final inactive sets, within 2 % of the printed counts.
    The iteration cap is the paper's 1e5 (App. "CG stopping criterion"); on
    2d_nonsep the instance with the smallest active set reaches it, and the
    printed mean is matched (to 0.01 %) only with that capped count in it,
    so a cold solve may end at the cap, with exactly 1e5 iterations."""
    n, B = 500, 30
    ref = printed()[name]
    case(f"{name} {n}^2 x {B}: cold iteration counts vs the printed table")
    w = gen.ocp_2d(name, n=n, B=B)
    s = lib.Solver(precision=lib.FP64)
    s.set_reference_factored(w.op.A, w.op.alpha, w.op.shift, gen.sine_modes_2d(n, 40)[0])
    out = s.active_set_batched(w.y_d, w.psi, tau=w.tau, tol=TOL, max_outer=20)
    s.close()
    masks = out["masks"].cpu().numpy()
    b = _rhs(w, masks)
    c = lib.Solver(precision=lib.FP64)
    c.set_reference_factored(w.op.A, w.op.alpha, w.op.shift, None)
    cold = c.solve_batched(masks, b, TOL)
    c.close()
    mc = float(np.mean(cold["iters"]))
    frac = masks.mean(axis=1)
    print(f"   outer {sorted(set(out['outer'].tolist()))}, active {frac.mean():.3f} "
          f"[{frac.min():.3f}, {frac.max():.3f}], cold mean {mc:.1f} (printed {ref['cold500']})", flush=True)
    assert np.all(out["status"] == 0)
    capped = cold["status"] == lib.W_MAXIT
    assert np.all((cold["status"] == 0) | capped)
    assert np.all(cold["iters"][capped] == 100000)
    assert abs(mc - ref["cold500"]) <= 0.02 * ref["cold500"]
