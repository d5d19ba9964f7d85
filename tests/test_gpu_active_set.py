"""Primal active-set outer loop on the GPU against the FP64 oracle.

Workload: the 2d_sym optimal-control family at n = 63 (4 amplitudes of the
desired state, bound at the 80 % quantile of the unconstrained state), 16
reference sine modes, inner CG tolerance 1e-10.  The oracle solves every
inner system exactly; the oracle's own A-DEF2 at the same tolerance lands
within 7e-10 of it, hence the 1e-8 bar on y.  Every inactive point of the
oracle's solution lies at least 1e-3 below the bound, far outside the inner
solve's error, so the active sets must agree exactly, and so must the outer
iteration counts."""
import numpy as np
import pytest

import gen
import oracle
from oracle.active_set import active_set

pytestmark = pytest.mark.gpu

N_GRID, K, TAU, TOL = 63, 16, 1e-10, 1e-10


def case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ocp():
    w = gen.ocp_2d_sym(n=N_GRID, B=4)
    Z = gen.sine_modes_2d(N_GRID, K)[0]
    spec = ("factored", w.op.A, w.op.alpha, w.op.shift)
    ref = [active_set(spec, w.y_d[m], w.psi[m], tau=TAU) for m in range(w.y_d.shape[0])]
    return w, Z, ref


def _solver(lib, w, Z, prec, form):
    s = lib.Solver(precision=prec)
    if form == "factored":
        s.set_reference_factored(w.op.A, w.op.alpha, w.op.shift, Z)
    else:
        s.set_reference(w.op.S(), Z)
    return s


@pytest.mark.parametrize("form", ["factored", "assembled"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_active_set_matches_oracle(lib, ocp, prec, form):
    w, Z, ref = ocp
    case(f"active set 2d_sym n={N_GRID} B=4 {prec} {form}")
    s = _solver(lib, w, Z, lib.FP64 if prec == "fp64" else lib.MIXED_REFINE, form)
    out = s.active_set_batched(w.y_d, w.psi, tau=TAU, tol=TOL, max_outer=20)
    Y = out["y"].cpu().numpy()
    M = out["masks"].cpu().numpy()
    for m, (y_ref, a_ref, k_ref, conv) in enumerate(ref):
        e = oracle.rel_err(Y[m], y_ref)
        print(f"   m={m} outer={out['outer'][m]} (oracle {k_ref}) |A|={int(M[m].sum())} "
              f"(oracle {int(a_ref.sum())}) inner iters={out['inner_iters'][m]} "
              f"status={out['status'][m]} e_rel={e:.3e}", flush=True)
        assert conv
        assert out["status"][m] in ((0,) if prec == "fp64" else (0, 3))
        assert out["outer"][m] == k_ref
        assert np.array_equal(M[m], a_ref)
        act = M[m] == 1
        assert np.all(Y[m, act] == w.psi[m, act])
        assert np.all(Y[m, ~act] <= w.psi[m, ~act] - TAU)
        assert e <= 1e-8
    s.close()


def test_active_set_outer_cap_and_arguments(lib, ocp):
    w, Z, ref = ocp
    case("active set: max_outer = 1 reports W_MAXIT; invalid tau is rejected")
    s = _solver(lib, w, Z, lib.FP64, "factored")
    out = s.active_set_batched(w.y_d, w.psi, tau=TAU, tol=TOL, max_outer=1)
    assert all(r[2] > 1 for r in ref)
    assert np.all(out["outer"] == 1)
    assert np.all(out["status"] == lib.W_MAXIT)
    # the first step is the unconstrained solve (empty active set)
    spec = ("factored", w.op.A, w.op.alpha, w.op.shift)
    for m in range(w.y_d.shape[0]):
        y_unc = active_set(spec, w.y_d[m], np.full(w.op.N, 1e30), tau=TAU)[0]
        assert oracle.rel_err(out["y"][m].cpu().numpy(), y_unc) <= 1e-8
    with pytest.raises(lib.Adef2Error):
        s.active_set_batched(w.y_d, w.psi, tau=-1.0)
    s.close()


def test_active_set_unconstrained_closed_form(lib):
    """psi far above the state: one outer step, empty active set, and y equal
    to the discrete closed form a / (1 + alpha' mu^2) sin(pi x1) sin(pi x2)."""
    n = 63
    w = gen.ocp_2d_sym(n=n, B=3)
    case("active set with an inactive bound: closed form, FP64 and FP32_REFINE")
    h = 1.0 / (n + 1)
    mu = 8.0 * np.sin(np.pi * h / 2.0) ** 2
    base = w.y_d[0] / w.params[0]
    for prec in (lib.FP64, lib.FP32_REFINE):
        s = lib.Solver(precision=prec)
        s.set_reference_factored(w.op.A, w.op.alpha, w.op.shift, gen.sine_modes_2d(n, K)[0])
        out = s.active_set_batched(w.y_d, np.full_like(w.psi, 10.0), tau=TAU, tol=TOL)
        Y = out["y"].cpu().numpy()
        assert np.all(out["outer"] == 1) and not out["masks"].cpu().numpy().any()
        for m, a in enumerate(w.params):
            ref = a / (1.0 + w.op.alpha * mu * mu) * base
            e = oracle.rel_err(Y[m], ref)
            print(f"   prec={prec} a={a:.3f} e_rel={e:.2e} status={out['status'][m]}", flush=True)
            assert e <= 1e-8
        s.close()


def test_active_set_single_instance_fp32_refine(lib, ocp):
    w, Z, ref = ocp
    case("active set, one instance, FP32_REFINE")
    s = _solver(lib, w, Z, lib.FP32_REFINE, "factored")
    out = s.active_set_batched(w.y_d[2:3], w.psi[2:3], tau=TAU, tol=TOL)
    y_ref, a_ref, k_ref, _ = ref[2]
    assert out["outer"][0] == k_ref
    assert np.array_equal(out["masks"].cpu().numpy()[0], a_ref)
    assert oracle.rel_err(out["y"].cpu().numpy()[0], y_ref) <= 1e-8
    s.close()
