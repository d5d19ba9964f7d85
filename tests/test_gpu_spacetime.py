"""Space-time extension on the GPU against the oracle: the all-at-once
implicit-Euler system M_st = alpha F^T F + I (F's time coupling is one more
diagonal of the factored operator, so t = F v, F^T t is the forward-backward
sweep with every time step in parallel) with the Kronecker deflation basis
I_nt (x) Z_s (eq. kron_basis; 6 sine modes x 10 steps = 60 columns).

2D, n = 15, n_t = 10 (2250 unknowns), two rotations.  Bars: the primal
active-set loop gives the oracle's outer counts and bit-equal active sets,
y within 1e-8 of the oracle's exact-solve loop; the deflated solves of the
final systems take the oracle's iteration counts within 1 % with the
Kronecker basis and with the constant-in-time lift 1_nt (x) Z_s, and (as
the paper reports) the lift removes far fewer iterations than the
Kronecker basis."""
import numpy as np
import pytest

import gen
import oracle
from oracle.active_set import active_set, coupled_rhs

pytestmark = pytest.mark.gpu

N_GRID, N_T, R, TOL = 15, 10, 6, 1e-10


def case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def st():
    w = gen.spacetime_2d(n=N_GRID, n_t=N_T, B=2)
    spec = ("factored", w.op.A, w.op.alpha, w.op.shift)
    Zs = gen.sine_modes_2d(N_GRID, R)[0]
    ref = [active_set(spec, w.y_d[m], w.psi[m], tau=w.tau) for m in range(2)]
    return w, spec, Zs, ref


def test_spacetime_active_set_kron_matches_oracle(lib, st):
    w, spec, Zs, ref = st
    case(f"space-time 2D n={N_GRID} n_t={N_T}: active-set loop with the Kronecker basis")
    Zst = gen.kron_basis(Zs, N_T)
    s = lib.Solver(precision=lib.FP64)
    s.set_reference_factored(w.op.A, w.op.alpha, w.op.shift, Zst)
    out = s.active_set_batched(w.y_d, w.psi, tau=w.tau, tol=TOL)
    Y = out["y"].cpu().numpy()
    M = out["masks"].cpu().numpy()
    for m, (y_ref, a_ref, k_ref, conv) in enumerate(ref):
        e = oracle.rel_err(Y[m], y_ref)
        print(f"   m={m} outer={out['outer'][m]} (oracle {k_ref}) active={M[m].mean():.3f} "
              f"inner iters={out['inner_iters'][m]} e_rel={e:.2e}", flush=True)
        assert conv and out["status"][m] == 0
        assert out["outer"][m] == k_ref
        assert np.array_equal(M[m], a_ref)
        assert e <= 1e-8
    s.close()


def test_spacetime_kron_vs_constant_lift(lib, st):
    w, spec, Zs, ref = st
    case("space-time deflated solves: Kronecker basis vs constant-in-time lift")
    masks = np.stack([r[1] for r in ref])
    bs = np.stack([coupled_rhs(spec, w.y_d[m], w.psi[m], masks[m]) for m in range(2)])
    its = {}
    for name, Z in (("kron", gen.kron_basis(Zs, N_T)), ("const", gen.const_time_basis(Zs, N_T))):
        s = lib.Solver(precision=lib.FP64)
        s.set_reference_factored(w.op.A, w.op.alpha, w.op.shift, Z)
        out = s.solve_batched(masks, bs, TOL)
        s.close()
        its[name] = out["iters"]
        for m in range(2):
            r = oracle.solve_instance(spec, Z, masks[m], bs[m], TOL)
            print(f"   {name} m={m} iters={out['iters'][m]} (oracle {r.iters}) status={out['status'][m]}",
                  flush=True)
            assert out["status"][m] == 0
            assert abs(int(out["iters"][m]) - r.iters) <= max(2, 0.01 * r.iters)
    assert np.all(its["kron"] * 1.5 < its["const"])
