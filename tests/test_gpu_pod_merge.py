"""Online POD enrichment with the conditioning-based safe merge (Alg. 2) on
the GPU against the oracle.

Causal use on the 2d_nonsep sweep at 100^2 (16 instances in parameter
order): the archive holds the oracle's full-state solutions of the first 8
instances, its first 6 POD modes (oracle, mean-centred SVD) are handed to
the library as candidates after 16 sine modes, and the next 8 instances are
solved.  Three tau_safe values: 1e4 (the paper's default; every first
candidate already doubles cond(E) here, so nothing is merged), 1.85e4 (the
merge stops after 0-6 candidates depending on the instance; every trial
cond is at least 1 % away from it) and 1e5 (all merged).  Bars: cond(E) to
1e-6 relative (it differs by more than 1 % between prefixes, so this also
checks which candidates were kept), FP64 iteration counts within 1 %, a
true relative residual within 2 x tol (the stopping rule, App. "CG stopping
criterion"), and a distance to the exact restricted solution within
max(1e-8, 2 x the oracle's own at the same tolerance): here the oracle's
A-DEF2 itself ends 1.1e-8 from it, residual 1e-10 times the conditioning."""
import numpy as np
import pytest

import gen
import oracle
from oracle.active_set import active_set, coupled_rhs
from oracle.learned import pod_modes
from oracle.solver import compact, restricted_operator

pytestmark = pytest.mark.gpu

N_GRID, K, P, TOL = 100, 16, 6, 1e-10


def case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def podcase():
    w = gen.ocp_2d("2d_nonsep", n=N_GRID, B=16)
    spec = ("factored", w.op.A, w.op.alpha, w.op.shift)
    ys, acts = [], []
    for m in range(16):
        y, act, _, _ = active_set(spec, w.y_d[m], w.psi[m], tau=w.tau)
        ys.append(y)
        acts.append(act)
    Phi, _ = pod_modes(np.column_stack(ys[:8]), P)
    sel = list(range(8, 16))
    masks = np.stack([acts[m] for m in sel])
    bs = np.stack([coupled_rhs(spec, w.y_d[m], w.psi[m], acts[m]) for m in sel])
    xs = []
    for j in range(len(sel)):
        I, _, _ = compact(masks[j])
        S_II, _ = restricted_operator(spec, I)
        xs.append((I, oracle.exact_solution(S_II, bs[j][I])))
    return w, spec, gen.sine_modes_2d(N_GRID, K)[0], Phi, masks, bs, xs


@pytest.mark.parametrize("tau_safe", [1e4, 1.85e4, 1e5])
def test_pod_safe_merge_matches_oracle(lib, podcase, tau_safe):
    w, spec, Z, Phi, masks, bs, xs = podcase
    case(f"POD safe merge 2d_nonsep {N_GRID}^2, k={K} + {P} candidates, tau_safe={tau_safe:g}")
    s = lib.Solver(precision=lib.FP64)
    s.set_reference_factored(w.op.A, w.op.alpha, w.op.shift, Z)
    s.set_pod_modes(Phi)
    s.pod_enrich(P, tau_safe)
    out = s.solve_batched(masks, bs, TOL)
    X = out["x"].cpu().numpy()
    for j in range(masks.shape[0]):
        ref = oracle.solve_instance(spec, Z, masks[j], bs[j], TOL, Phi=Phi, tau_safe=tau_safe)
        I, x_ex = xs[j]
        e = oracle.rel_err(X[j, I], x_ex)
        e_ref = oracle.rel_err(ref.x[I], x_ex)
        print(f"   j={j} iters={out['iters'][j]} (oracle {ref.iters}) cond={out['cond_E'][j]:.6e} "
              f"(oracle {ref.cond_E:.6e}, k={ref.k_eff}) status={out['status'][j]} e_rel={e:.2e} "
              f"(oracle {e_ref:.2e}) relres={out['relres_true'][j]:.2e}",
              flush=True)
        assert out["status"][j] == 0 and ref.status == 0
        assert abs(out["cond_E"][j] / ref.cond_E - 1.0) <= 1e-6
        assert abs(int(out["iters"][j]) - ref.iters) <= max(2, 0.01 * ref.iters)
        assert out["relres_true"][j] <= 2 * TOL
        assert e <= max(1e-8, 2 * e_ref)
    s.close()


def test_pod_enrich_zero_restores_reference_modes(lib, podcase):
    w, spec, Z, Phi, masks, bs, _ = podcase
    case("pod_enrich(0) after an enrichment gives the plain reference-mode results")
    outs = []
    for enrich in (False, True):
        s = lib.Solver(precision=lib.FP64, rows_per_thread=1, w_mode=1, op_fused=-1)
        s.set_reference_factored(w.op.A, w.op.alpha, w.op.shift, Z)
        if enrich:
            s.set_pod_modes(Phi)
            s.pod_enrich(P, 1e5)
            s.solve_batched(masks, bs, TOL)
            s.pod_enrich(0)
        outs.append(s.solve_batched(masks, bs, TOL))
        s.close()
    assert np.array_equal(outs[0]["iters"], outs[1]["iters"])
    assert bool((outs[0]["x"] == outs[1]["x"]).all().item())
    with pytest.raises(lib.Adef2Error):
        s = lib.Solver(precision=lib.FP64)
        s.set_reference_factored(w.op.A, w.op.alpha, w.op.shift, Z)
        s.pod_enrich(P, 1e4)        # no POD modes held yet
