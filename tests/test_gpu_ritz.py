"""Rayleigh-Ritz reselection (Sec. "Ritz re-selection") on the GPU against
the oracle: a pool of the 40 lowest sine modes restricted to the final
active sets of the 2d_sym problem at 100^2, 20 Ritz vectors kept.  Bars:
cond(E) (the ratio of the kept Ritz values) to 1e-6 relative, FP64
iteration counts within 1 % of the oracle's, every solve within 1e-8 of the
exact restricted solution; with ritz_keep >= the pool the results are
bitwise those of the default path."""
import numpy as np
import pytest

import gen
import oracle
from oracle.active_set import active_set, coupled_rhs
from oracle.solver import compact, restricted_basis, restricted_operator, ritz_reselect

pytestmark = pytest.mark.gpu

N_GRID, POOL, KEEP, TOL = 100, 40, 20, 1e-10


def case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ritz_case():
    w = gen.ocp_2d("2d_sym", n=N_GRID, B=4)
    spec = ("factored", w.op.A, w.op.alpha, w.op.shift)
    Z = gen.sine_modes_2d(N_GRID, POOL)[0]
    masks, bs, refs = [], [], []
    for m in range(4):
        _, act, _, _ = active_set(spec, w.y_d[m], w.psi[m], tau=w.tau)
        b = coupled_rhs(spec, w.y_d[m], w.psi[m], act)
        I, _, _ = compact(act)
        S_II, _ = restricted_operator(spec, I)
        _, mu = ritz_reselect(S_II, restricted_basis(Z, I)[0], KEEP)
        ref = oracle.solve_instance(spec, Z, act, b, TOL, ritz_keep=KEEP)
        xs = oracle.exact_solution(S_II, b[I])
        masks.append(act)
        bs.append(b)
        refs.append((I, mu[-1] / mu[0], ref.iters, xs))
    return w, Z, np.stack(masks), np.stack(bs), refs


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_ritz_reselection_matches_oracle(lib, ritz_case, prec):
    w, Z, masks, bs, refs = ritz_case
    case(f"Ritz reselection 2d_sym {N_GRID}^2 pool {POOL} keep {KEEP} {prec}")
    p = lib.FP64 if prec == "fp64" else lib.MIXED_REFINE
    s = lib.Solver(precision=p, ritz_keep=KEEP)
    s.set_reference_factored(w.op.A, w.op.alpha, w.op.shift, Z)
    out = s.solve_batched(masks, bs, TOL)
    X = out["x"].cpu().numpy()
    for m, (I, cond_ref, it_ref, xs) in enumerate(refs):
        e = oracle.rel_err(X[m, I], xs)
        print(f"   m={m} iters={out['iters'][m]} (oracle {it_ref}) cond={out['cond_E'][m]:.6e} "
              f"(oracle {cond_ref:.6e}) status={out['status'][m]} e_rel={e:.2e}", flush=True)
        assert out["status"][m] == 0
        assert abs(out["cond_E"][m] / cond_ref - 1.0) <= 1e-6
        if prec == "fp64":
            assert abs(int(out["iters"][m]) - it_ref) <= max(2, 0.01 * it_ref)
        assert e <= 1e-8
    s.close()


def test_ritz_keep_at_pool_size_is_default_path(lib, ritz_case):
    w, Z, masks, bs, _ = ritz_case
    case("ritz_keep >= pool reproduces the default path bitwise")
    outs = []
    for keep in (0, POOL):
        s = lib.Solver(precision=lib.FP64, ritz_keep=keep, rows_per_thread=1, w_mode=1, op_fused=-1)
        s.set_reference_factored(w.op.A, w.op.alpha, w.op.shift, Z)
        outs.append(s.solve_batched(masks, bs, TOL))
        s.close()
    assert np.array_equal(outs[0]["iters"], outs[1]["iters"])
    assert torch_equal(outs[0]["x"], outs[1]["x"])


def torch_equal(a, b):
    return bool((a == b).all().item())
