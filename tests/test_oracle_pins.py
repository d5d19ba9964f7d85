"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these tests retypes an oracle formula: each one checks the oracle
against a closed form, an invariant, a special case that reduces to a textbook
or library routine, exact rational arithmetic, or brute force on tiny inputs.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import gen
import oracle
from oracle import solver as oa


def _tiny(n=15, k=8, active=0.2, seed=0):
    w = gen.c1_workload(n=n, k=k, seeds=(seed,), active=active)
    return w, w.op.S(), w.instances[0]


def _restricted(S, Z, mask):
    I, g2l, nI = oracle.compact(mask)
    S_II, d_I = oracle.restrict(S, I)
    return I, g2l, nI, S_II, d_I


# ---------------------------------------------------------------------------
# compaction and restriction
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_compaction_properties(seed):
    rng = np.random.default_rng(seed)
    mask = (rng.uniform(size=1000) < 0.3).astype(np.uint8)
    I, g2l, nI = oracle.compact(mask)
    assert nI == int((mask == 0).sum())
    assert np.all(np.diff(I) > 0)                       # strictly ascending
    assert np.all(mask[I] == 0)
    assert np.all(g2l[I] == np.arange(nI))
    assert np.all(g2l[mask == 1] == -1)


def test_compaction_edge_cases():
    for mask in [np.zeros(7, np.uint8), np.ones(7, np.uint8), np.zeros(0, np.uint8)]:
        I, g2l, nI = oracle.compact(mask)
        assert nI == int((mask == 0).sum()) and len(I) == nI


def test_restriction_equals_scatter_matvec_gather():
    w, S, inst = _tiny()
    I, _, nI, S_II, d_I = _restricted(S, w.Z, inst.mask)
    x = np.random.default_rng(1).standard_normal(nI)
    full = np.zeros(S.shape[0])
    full[I] = x
    np.testing.assert_allclose(S_II @ x, (S @ full)[I], rtol=0, atol=1e-15 * abs(S).max() * 13)
    np.testing.assert_array_equal(d_I, S.diagonal()[I])
    assert abs(S_II - S_II.T).max() == 0.0


def test_cauchy_interlacing():
    """lambda_j(S) <= mu_j(S_II) <= lambda_{j+N-n_I}(S)  (Sec. spectral coherence)."""
    w, S, inst = _tiny(n=11, active=0.3)
    I, _, nI, S_II, _ = _restricted(S, w.Z, inst.mask)
    lam = np.linalg.eigvalsh(S.toarray())
    mu = np.linalg.eigvalsh(S_II.toarray())
    N = S.shape[0]
    tol = 1e-12 * lam[-1]
    assert np.all(lam[:nI] <= mu + tol)
    assert np.all(mu <= lam[N - nI:] + tol)


def test_min_eigenvalue_bounded_by_shift():
    """lambda_min(S) >= c for S = a B + c I with B PSD (paper: lambda_min(M) >= 1)."""
    for w in (gen.c1_workload(n=9, k=0), ):
        S = w.op.S().toarray()
        assert np.linalg.eigvalsh(S)[0] >= w.op.shift * (1 - 1e-10)
    op, _ = gen.c2_operator(n=9)
    assert np.linalg.eigvalsh(op.S().toarray())[0] >= op.shift * (1 - 1e-8)


# ---------------------------------------------------------------------------
# restricted basis (QR) and coarse space
# ---------------------------------------------------------------------------
def test_restricted_basis_orthonormal_same_span():
    w, S, inst = _tiny(n=15, k=10)
    I, *_ = _restricted(S, w.Z, inst.mask)
    Q, kept = oracle.restricted_basis(w.Z, I)
    assert Q.shape[1] == 10 and list(kept) == list(range(10))
    np.testing.assert_allclose(Q.T @ Q, np.eye(10), atol=1e-13)
    ZI = w.Z[I, :]
    # same span: the orthogonal projector onto span(Z_I) fixes Q
    Pz = ZI @ np.linalg.solve(ZI.T @ ZI, ZI.T)
    np.testing.assert_allclose(Pz @ Q, Q, atol=1e-12)


def test_restricted_basis_drops_dependent_and_zero_columns():
    w, S, inst = _tiny(n=15, k=6)
    I, *_ = _restricted(S, w.Z, inst.mask)
    Z = np.column_stack([w.Z[:, :3], w.Z[:, 1], np.zeros(w.Z.shape[0]), w.Z[:, 3:]])
    Q, kept = oracle.restricted_basis(Z, I)
    assert list(kept) == [0, 1, 2, 5, 6, 7]
    assert Q.shape[1] == 6
    np.testing.assert_allclose(Q.T @ Q, np.eye(6), atol=1e-13)


def test_projector_is_M_orthogonal():
    """P^2 = P and M P = P^T M  (eq. proj; P is an M_II-orthogonal projector)."""
    w, S, inst = _tiny(n=11, k=6)
    I, _, nI, S_II, _ = _restricted(S, w.Z, inst.mask)
    Zo, _ = oracle.restricted_basis(w.Z, I)
    cs, fb = oracle.coarse_setup(S_II, Zo)
    assert not fb
    P = np.column_stack([oa.apply_projector(cs, e) for e in np.eye(nI)])
    M = S_II.toarray()
    scale = np.abs(M).max()
    np.testing.assert_allclose(P @ P, P, atol=1e-10)
    np.testing.assert_allclose(M @ P, P.T @ M, atol=1e-10 * scale)
    np.testing.assert_allclose(P @ Zo, 0.0, atol=1e-10)


def test_condition_number_of_exact_eigenbasis():
    """With Z = eigenvectors of M_II, E = diag(lambda): cond = lambda_max/lambda_min."""
    w, S, inst = _tiny(n=9, k=0)
    mask = np.zeros(S.shape[0], np.uint8)
    lam, V = np.linalg.eigh(S.toarray())
    cs, fb = oracle.coarse_setup(S, V[:, :5])
    assert not fb
    np.testing.assert_allclose(cs.E, np.diag(lam[:5]), atol=1e-12 * lam[4])
    assert abs(cs.cond / (lam[4] / lam[0]) - 1) < 1e-10
    cs, fb = oracle.coarse_setup(S, V[:, :5], tau_cond=0.5 * lam[4] / lam[0])
    assert fb


# ---------------------------------------------------------------------------
# A-DEF2 loop
# ---------------------------------------------------------------------------
def test_k0_is_textbook_jacobi_pcg_scipy():
    w, S, inst = _tiny(n=31, k=0)
    I, _, nI, S_II, d_I = _restricted(S, w.Z, inst.mask)
    b = inst.b[I]
    res = oracle.jacobi_pcg(S_II, b, 1e-8)
    count = [0]
    xs, info = spla.cg(S_II, b, rtol=1e-8, atol=0.0, maxiter=100000,
                       M=sp.diags(1.0 / d_I), callback=lambda xk: count.__setitem__(0, count[0] + 1))
    assert info == 0
    assert abs(res.iters - count[0]) <= 1
    assert oracle.rel_err(res.x, xs) < 1e-6
    assert np.linalg.norm(b - S_II @ res.x) <= 1.01e-8 * np.linalg.norm(b) * 10


def test_finite_termination_unpreconditioned():
    """No preconditioner, b a combination of m eigenvectors of M_II outside
    span(Z): CG terminates after exactly m steps (Krylov space of dim m)."""
    w, S, inst = _tiny(n=9, k=0)
    M = S.toarray()
    lam, V = np.linalg.eigh(M)
    Z = V[:, :3]
    cs, _ = oracle.coarse_setup(S, Z)
    m = 4
    b = V[:, [3, 6, 10, 20]] @ np.array([1.0, 2.0, -1.0, 0.5])
    res = oracle.adef2(S, b, cs, 1e-10, d_inv=np.ones(S.shape[0]))
    assert res.iters == m
    x_exact = V[:, [3, 6, 10, 20]] @ (np.array([1.0, 2.0, -1.0, 0.5]) / lam[[3, 6, 10, 20]])
    assert oracle.rel_err(res.x, x_exact) < 1e-9


def test_rhs_in_coarse_space_needs_no_iteration():
    w, S, inst = _tiny(n=15, k=8)
    I, _, nI, S_II, _ = _restricted(S, w.Z, inst.mask)
    Zo, _ = oracle.restricted_basis(w.Z, I)
    cs, _ = oracle.coarse_setup(S_II, Zo)
    c = np.arange(1, 9, dtype=float)
    b = S_II @ (Zo @ c)
    res = oracle.adef2(S_II, b, cs, 1e-10)
    assert res.iters == 0
    assert oracle.rel_err(res.x, Zo @ c) < 1e-12


def test_full_rank_coarse_space_is_exact():
    """k = n_I: the coarse correction alone solves the system (0 iterations)."""
    N = 25
    w, S, inst = _tiny(n=5, k=0)
    mask = np.zeros(N, np.uint8)
    mask[[0, 7, 12, 18, 24]] = 1
    I, _, nI, S_II, _ = _restricted(S, None, mask)
    Z = np.random.default_rng(3).standard_normal((N, nI))
    Zo, kept = oracle.restricted_basis(Z, I)
    assert len(kept) == nI
    cs, _ = oracle.coarse_setup(S_II, Zo)
    b = np.random.default_rng(4).standard_normal(nI)
    res = oracle.adef2(S_II, b, cs, 1e-12)
    assert res.iters == 0
    assert oracle.rel_err(res.x, np.linalg.solve(S_II.toarray(), b)) < 1e-10


def _run_recorded(n=15, k=8, tol=1e-12, seed=0, maxit=1500):
    w, S, inst = _tiny(n=n, k=k, seed=seed)
    I, _, nI, S_II, _ = _restricted(S, w.Z, inst.mask)
    Zo, _ = oracle.restricted_basis(w.Z, I)
    cs, _ = oracle.coarse_setup(S_II, Zo)
    b = inst.b[I]
    res = oracle.adef2(S_II, b, cs, tol, maxit=maxit, record=True)
    xs = oracle.exact_solution(S_II, b)
    return S_II, b, Zo, res, xs


def _invariant_violations(S_II, b, Zo, res, xs):
    """Which A-DEF2 pins fail for a recorded run (used by the mutation test)."""
    bad = []
    bn = np.linalg.norm(b)
    # recurrence residual equals the true residual (unprojected, App. stopping)
    for x, r in res.history:
        if np.linalg.norm(r - (b - S_II @ x)) > 1e-9 * bn:
            bad.append("residual_drift")
            break
    # Z^T r_k = 0 relative to ||b||
    if max(np.linalg.norm(Zo.T @ r) for _, r in res.history) > 1e-11 * bn:
        bad.append("ZTr")
    # energy norm of the error is non-increasing
    en = [float(np.sqrt(max((x - xs) @ (S_II @ (x - xs)), 0.0))) for x, _ in res.history]
    if any(en[i + 1] > en[i] * (1 + 1e-8) + 1e-14 * en[0] for i in range(len(en) - 1)):
        bad.append("energy")
    if not res.converged or oracle.rel_err(res.x, xs) > 1e-8:
        bad.append("accuracy")
    return bad


@pytest.mark.parametrize("seed", [0, 1])
def test_adef2_invariants(seed):
    S_II, b, Zo, res, xs = _run_recorded(seed=seed)
    assert res.converged and res.iters > 5
    assert _invariant_violations(S_II, b, Zo, res, xs) == []


def test_deflation_reduces_iterations_c1():
    w = gen.c1_workload(n=63, k=16)
    S = w.op.S()
    inst = w.instances[0]
    rd = oracle.solve_instance(S, w.Z, inst.mask, inst.b, 1e-8)
    rp = oracle.solve_instance(S, w.Z[:, :0], inst.mask, inst.b, 1e-8)
    assert rd.status == 0 and rp.status == 0
    assert rd.iters < rp.iters
    assert rd.relres_true < 1.5e-8 and rp.relres_true < 1.5e-8


def test_fallback_is_plain_pcg():
    w = gen.c1_workload(n=31, k=8)
    S = w.op.S()
    inst = w.instances[0]
    rf = oracle.solve_instance(S, w.Z, inst.mask, inst.b, 1e-8, tau_cond=1.0)
    rp = oracle.solve_instance(S, w.Z[:, :0], inst.mask, inst.b, 1e-8)
    assert rf.status == oracle.STATUS_FALLBACK and rf.k_eff == 0
    assert rf.iters == rp.iters
    np.testing.assert_array_equal(rf.x, rp.x)


def test_maxit_status():
    w = gen.c1_workload(n=31, k=8)
    inst = w.instances[0]
    r = oracle.solve_instance(w.op.S(), w.Z, inst.mask, inst.b, 1e-12, maxit=3)
    assert r.status == oracle.STATUS_MAXIT and r.iters == 3


def test_two_dimensional_symmetric_closed_form():
    """The paper's 2d_sym case (golden fixture): y_d = a sin(pi x) sin(pi y) is an
    eigenvector of M = alpha L^2 + I, so y* = y_d / lambda_11 and deflation with
    the sine modes needs no iteration; lambda_11 -> 1 + 4 pi^4 alpha as h -> 0."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "2d_sym.txt")
    vals = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            key, *rest = line.split()
            vals[key] = rest
    alpha = float(vals["alpha"][0])
    lam_cont = 1 + 4 * math.pi ** 4 * alpha
    prev = None
    for n in (15, 31, 63):
        h = 1.0 / (n + 1)
        L = gen.laplacian_2d(n) / (h * h)
        M = sp.csr_matrix(alpha * (L @ L) + sp.identity(n * n))
        Z, pairs, _ = gen.sine_modes_2d(n, 3)
        assert pairs[0] == (1, 1)
        mu1 = 4 / h ** 2 * math.sin(math.pi / (2 * (n + 1))) ** 2
        lam11 = alpha * (2 * mu1) ** 2 + 1
        for a in map(float, vals["a_values"]):
            yd = a * Z[:, 0] * (n + 1) / 2.0          # a sin(pi x) sin(pi y) on the nodes
            cs, fb = oracle.coarse_setup(M, Z)
            # the exact x = y_d / lambda_11 leaves a rounding residual ~ u ||M|| ||x||
            res = oracle.adef2(M, yd, cs, 1e-8)
            assert res.iters == 0
            assert oracle.rel_err(res.x, yd / lam11) < 1e-11
            # unpreconditioned CG: an eigenvector rhs converges in one step
            res0 = oracle.jacobi_pcg(M, yd, 1e-8, d_inv=np.ones(n * n))
            assert res0.iters == 1
        err = abs(lam11 - lam_cont)
        if prev is not None:
            assert err < prev / 3.5                   # O(h^2) convergence to the printed value
        prev = err
    assert prev / lam_cont < 2e-3


# ---------------------------------------------------------------------------
# exact solution machinery
# ---------------------------------------------------------------------------
def test_two_sum_two_prod_exact():
    rng = np.random.default_rng(0)
    a = rng.standard_normal(200) * 10.0 ** rng.integers(-8, 8, 200)
    b = rng.standard_normal(200) * 10.0 ** rng.integers(-8, 8, 200)
    s, e = oa.two_sum(a, b)
    p, f = oa.two_prod(a, b)
    for i in range(200):
        assert Fraction(s[i]) + Fraction(e[i]) == Fraction(a[i]) + Fraction(b[i])
        assert Fraction(p[i]) + Fraction(f[i]) == Fraction(a[i]) * Fraction(b[i])


def test_dd_residual_against_exact_rationals():
    rng = np.random.default_rng(1)
    A = sp.random(12, 12, density=0.5, random_state=2, format="csr") + sp.identity(12)
    x = rng.standard_normal(12)
    b = A @ x + 1e-12 * rng.standard_normal(12)
    r = oracle.dd_residual(A, x, b)
    Ad = A.toarray()
    for i in range(12):
        exact = Fraction(b[i]) - sum(Fraction(Ad[i, j]) * Fraction(x[j]) for j in range(12))
        assert abs(Fraction(r[i]) - exact) <= abs(exact) * Fraction(2.3e-16) + Fraction(1e-300)


def _fraction_solve(A, b):
    n = len(b)
    M = [[Fraction(A[i, j]) for j in range(n)] + [Fraction(b[i])] for i in range(n)]
    for c in range(n):
        piv = M[c][c]
        for r_ in range(c + 1, n):
            f = M[r_][c] / piv
            for j in range(c, n + 1):
                M[r_][j] -= f * M[c][j]
    x = [Fraction(0)] * n
    for i in reversed(range(n)):
        x[i] = (M[i][n] - sum(M[i][j] * x[j] for j in range(i + 1, n))) / M[i][i]
    return x


@pytest.mark.parametrize("dense_limit,method", [(4000, "auto"), (2, "banded"), (2, "auto")])
def test_exact_solution_matches_rational_solve(dense_limit, method):
    """An ill-conditioned SPD system (cond ~ 1e9) solved to ~1 ulp forward error."""
    w = gen.c1_workload(n=3, k=0)
    A = w.op.S()
    Q, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((9, 9)))
    Ad = (Q * np.logspace(0, 9, 9)) @ Q.T
    Ad = 0.5 * (Ad + Ad.T)
    A = sp.csr_matrix(Ad)
    b = np.random.default_rng(6).standard_normal(9)
    x = oracle.exact_solution(A, b, dense_limit=dense_limit, method=method)
    xe = np.array([float(v) for v in _fraction_solve(Ad, b)])
    assert np.linalg.norm(x - xe) <= 4e-16 * np.linalg.norm(xe)


def test_exact_solution_routes_agree_on_a_restricted_system():
    """Dense Cholesky, banded Cholesky and sparse LU, each followed by
    double-double refinement, give the same x* of a factored restricted
    system (cond ~ 1e7) to a few ulps: the refinement, not the factorisation,
    sets the accuracy."""
    w = gen.c2_workload(n=47, k=0, B=1)
    op = w.op
    inst = w.instances[0]
    I, _, _ = oracle.compact(inst.mask)
    F, _ = oracle.restrict_factored(op.A, op.alpha, op.shift, I)
    b = inst.b[I]
    xd = oracle.exact_solution(F, b, method="dense")
    xb = oracle.exact_solution(F, b, method="banded")
    xs = oracle.exact_solution(F, b, method="splu")
    assert np.linalg.norm(xb - xd) <= 1e-14 * np.linalg.norm(xd)
    assert np.linalg.norm(xs - xd) <= 1e-14 * np.linalg.norm(xd)


# ---------------------------------------------------------------------------
# mutation check: plausible oracle mistakes are caught by the pins above
# ---------------------------------------------------------------------------
def _mut_no_projection(cs, v):          # Alg. 1 exactly as printed: p built from K r
    return v


def _mut_sign(cs, v):
    return v if cs.k == 0 else v + cs.Z @ cs.solve(cs.W.T @ v)


def _mut_transposed_operand(cs, v):     # Z^T v where W^T v belongs
    return v if cs.k == 0 else v - cs.Z @ cs.solve(cs.Z.T @ v)


@pytest.mark.parametrize("mutant", [_mut_no_projection, _mut_sign, _mut_transposed_operand])
def test_planted_mistakes_are_detected(monkeypatch, mutant):
    monkeypatch.setattr(oa, "apply_projector", mutant)
    S_II, b, Zo, res, xs = _run_recorded(tol=1e-12)
    assert _invariant_violations(S_II, b, Zo, res, xs) != []


def test_planted_coarse_correction_mistake_is_detected(monkeypatch):
    monkeypatch.setattr(oa, "coarse_coefficients", lambda cs, r: np.zeros(0) if cs.k == 0
                        else -cs.solve(cs.Z.T @ r))
    S_II, b, Zo, res, xs = _run_recorded(tol=1e-12)
    assert _invariant_violations(S_II, b, Zo, res, xs) != []


# ---------------------------------------------------------------------------
# factored operator M = alpha A^T A + shift I (eq. schur)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("maker", ["c1", "c2", "c3"])
def test_factored_restriction_equals_assembled_submatrix(maker):
    """(A^T A)[I, I] = A[:, I]^T A[:, I]: the factored restricted operator agrees
    with the submatrix of the assembled full-domain operator."""
    if maker == "c1":
        op = gen.c1_workload(n=15, k=0).op
    elif maker == "c2":
        op, _ = gen.c2_operator(n=15)
    else:
        op, _ = gen.c3_operator(n=15)
    mask = gen.mask_top_fraction(gen.sinusoid_field(15, 4), 0.3)
    I, _, nI = oracle.compact(mask)
    S_II, d_I = oracle.restrict(op.S(), I)
    F, dF = oracle.restrict_factored(op.A, op.alpha, op.shift, I)
    x = np.random.default_rng(2).standard_normal(nI)
    np.testing.assert_allclose(F @ x, S_II @ x, rtol=0, atol=1e-12 * abs(S_II).max() * np.abs(x).max() * 20)
    np.testing.assert_allclose(dF, d_I, rtol=1e-13)
    np.testing.assert_allclose(F.toarray(), S_II.toarray(), rtol=0, atol=1e-12 * abs(S_II).max())


def test_factored_dd_residual_against_exact_rationals():
    rng = np.random.default_rng(8)
    A = sp.random(10, 10, density=0.4, random_state=9, format="csr") + sp.identity(10)
    I = np.array([0, 2, 3, 5, 6, 9])
    F = oa.FactoredOp(A, 0.37, 1.25e-3, I)
    x = rng.standard_normal(len(I))
    b = F @ x + 1e-13 * rng.standard_normal(len(I))
    r = oracle.dd_residual(F, x, b)
    AI = A.toarray()[:, I]
    fa, fs = Fraction(0.37), Fraction(1.25e-3)
    for i in range(len(I)):
        acc = Fraction(0)
        for j in range(len(I)):
            mij = sum(Fraction(AI[l, i]) * Fraction(AI[l, j]) for l in range(10))
            acc += mij * Fraction(x[j])
        exact = Fraction(b[i]) - fa * acc - fs * Fraction(x[i])
        assert abs(Fraction(r[i]) - exact) <= abs(exact) * Fraction(1e-15) + Fraction(1e-300)


def test_factored_exact_solution_is_the_factored_operators():
    """x* of the factored operator has a residual, evaluated in exact rational
    arithmetic, at the level of one rounding of x (not of cond(M) u)."""
    w = gen.c2_workload(n=7, k=0, B=1)
    op = w.op
    inst = w.instances[0]
    I, _, nI = oracle.compact(inst.mask)
    F, _ = oracle.restrict_factored(op.A, op.alpha, op.shift, I)
    b = inst.b[I]
    x = oracle.exact_solution(F, b)
    AI = op.A.toarray()[:, I]
    fa, fs = Fraction(op.alpha), Fraction(op.shift)
    xf = [Fraction(v) for v in x]
    t = [sum(Fraction(AI[l, j]) * xf[j] for j in range(nI) if AI[l, j] != 0) for l in range(AI.shape[0])]
    res = []
    for i in range(nI):
        u = sum(Fraction(AI[l, i]) * t[l] for l in range(AI.shape[0]) if AI[l, i] != 0)
        res.append(float(Fraction(b[i]) - fa * u - fs * xf[i]))
    Mx = np.abs(F.toarray()) @ np.abs(x)
    assert np.all(np.abs(res) <= 8 * 2.2e-16 * Mx)


# ---------------------------------------------------------------------------
# primal active-set outer loop
# ---------------------------------------------------------------------------
def _sym_unconstrained(w):
    n = w.op.n
    h = 1.0 / (n + 1)
    x1, x2 = gen._coords(n, 2)
    mu = 8.0 * np.sin(np.pi * h / 2.0) ** 2
    return np.sin(np.pi * x1) * np.sin(np.pi * x2) / (1.0 + w.op.alpha * mu * mu)


def test_active_set_unconstrained_closed_form():
    """psi above the unconstrained solution: one outer step, empty active set,
    y = M^-1 y_d, which for y_d = a sin sin is a / (1 + alpha mu^2) sin sin."""
    from oracle.active_set import active_set
    w = gen.ocp_2d_sym(n=31, B=3)
    spec = ("factored", w.op.A, w.op.alpha, w.op.shift)
    base = _sym_unconstrained(w)
    for m in range(3):
        y, act, k, conv = active_set(spec, w.y_d[m], np.full(w.op.N, 10.0))
        assert conv and k == 1 and act.sum() == 0
        np.testing.assert_allclose(y, w.params[m] * base, rtol=1e-12, atol=1e-15)


def test_active_set_fixed_point_and_iterations():
    """At return: y_A = psi_A, y_I solves M_II y_I = (y_d)_I - M_IA psi_A, the
    active set equals {y > psi - tau}, and the loop took 2-4 outer steps (the
    paper's range for its benchmark families)."""
    from oracle.active_set import active_set, apply_full
    w = gen.ocp_2d_sym(n=31, B=3)
    spec = ("factored", w.op.A, w.op.alpha, w.op.shift)
    for m in range(3):
        y, act, k, conv = active_set(spec, w.y_d[m], w.psi[m])
        assert conv and 2 <= k <= 4, k
        A = act != 0
        np.testing.assert_array_equal(y[A], w.psi[m][A])
        r = w.y_d[m] - apply_full(spec, y)
        assert np.linalg.norm(r[~A]) <= 1e-10 * np.linalg.norm(w.y_d[m][~A])
        np.testing.assert_array_equal((y > w.psi[m] - 1e-10).astype(np.uint8), act)
        # the constraint holds up to tau on the inactive set after convergence
        assert np.all(y[~A] <= w.psi[m][~A] - 1e-10 + 1e-12)


# ---------------------------------------------------------------------------
# Ritz reselection (Sec. "Ritz re-selection")
# ---------------------------------------------------------------------------
def _sym_op(n):
    w = gen.ocp_2d_sym(n=n, B=1)
    return w.op, ("factored", w.op.A, w.op.alpha, w.op.shift)


def test_ritz_recovers_lowest_modes_closed_form():
    """Empty active set: M_II = M, whose eigenvectors are the sine modes with
    eigenvalues 1 + alpha' (s_i + s_j)^2.  A pool of the 16 lowest modes mixed
    by a random rotation must give back the 4 lowest (a gap follows the 4th:
    (1,1), (1,2), (2,1), (2,2), then (1,3)) with their closed-form values."""
    from oracle.solver import restricted_basis, restricted_operator, ritz_reselect
    n = 31
    op, spec = _sym_op(n)
    Z, pairs, _ = gen.sine_modes_2d(n, 16)
    Qr, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((16, 16)))
    I = np.arange(op.N)
    S_II, _ = restricted_operator(spec, I)
    Zo, _ = restricted_basis(Z @ Qr, I)
    Zs, mu = ritz_reselect(S_II, Zo, 4)
    h = 1.0 / (n + 1)
    s = lambda q: 4.0 * np.sin(q * np.pi * h / 2.0) ** 2
    lam = sorted(1.0 + op.alpha * (s(i) + s(j)) ** 2 for i, j in pairs)[:4]
    assert np.allclose(mu, lam, rtol=1e-12)
    low = Z[:, :4]
    assert np.linalg.norm(Zs - low @ (low.T @ Zs)) <= 1e-10
    assert np.allclose(Zs.T @ Zs, np.eye(4), atol=1e-12)


def test_ritz_values_interlace_and_diagonalise():
    """With a real active set the kept Ritz values bound the lowest eigenvalues
    of M_II from above (Courant-Fischer), the kept basis is orthonormal and
    diagonalises the projected operator, and r >= pool returns the pool."""
    from oracle.solver import compact, restricted_basis, restricted_operator, ritz_reselect
    n = 15
    op, spec = _sym_op(n)
    rng = np.random.default_rng(9)
    mask = (rng.random(op.N) < 0.25).astype(np.uint8)
    I, _, _ = compact(mask)
    S_II, _ = restricted_operator(spec, I)
    Z = gen.sine_modes_2d(n, 12)[0]
    Zo, _ = restricted_basis(Z, I)
    Zs, mu = ritz_reselect(S_II, Zo, 5)
    ev = np.linalg.eigvalsh(S_II.toarray())
    assert np.all(mu >= ev[:5] * (1 - 1e-12))
    assert np.all(np.diff(mu) >= 0)
    F = Zs.T @ (S_II @ Zs)
    assert np.allclose(F, np.diag(mu), atol=1e-9 * mu[-1])
    assert np.allclose(Zs.T @ Zs, np.eye(5), atol=1e-12)
    same, none = ritz_reselect(S_II, Zo, Zo.shape[1])
    assert none is None and same is Zo
    # a smaller pool never gives smaller Ritz values (the pool spans less)
    _, mu8 = ritz_reselect(S_II, restricted_basis(Z[:, :8], I)[0], 5)
    assert np.all(mu8 >= mu * (1 - 1e-12))


# ---------------------------------------------------------------------------
# safe merge of POD candidates (Alg. 2)
# ---------------------------------------------------------------------------
def test_safe_merge_skip_and_break_rules():
    """Diagonal M with unit-vector candidates, so every cond is known:
    Phi_eig = [e0] (eigenvalue 1); candidates e1 (2), a vector inside
    span(e0, e1) (dependent: skipped, merge continues), e2 (1e5: cond 1e5 >
    tau_safe = 1e4, merge stops), e3 (3: never reached)."""
    from oracle.solver import safe_merge
    n = 8
    d = np.array([1.0, 2.0, 1e5, 3.0, 5.0, 6.0, 7.0, 8.0])
    M = sp.diags(d).tocsr()
    e = np.eye(n)
    Phi_eig = e[:, :1]
    dep = (e[:, 0] + e[:, 1]) / np.sqrt(2.0)
    Phi_pod = np.column_stack([e[:, 1], dep, e[:, 2], e[:, 3]])
    Z = safe_merge(M, Phi_eig, Phi_pod, tau_safe=1e4)
    assert Z.shape == (n, 2)
    assert np.allclose(np.abs(Z), e[:, :2])
    # without the conditioning stop the later candidates are taken
    Z2 = safe_merge(M, Phi_eig, Phi_pod, tau_safe=1e6)
    assert Z2.shape == (n, 4)
    assert np.allclose(Z2.T @ Z2, np.eye(4), atol=1e-14)
    assert np.allclose(np.abs(Z2[:, 3]), e[:, 3])


def test_safe_merge_spans_union_and_keeps_eigen_prefix():
    from oracle.solver import compact, restricted_basis, restricted_operator, safe_merge
    n = 15
    op, spec = _sym_op(n)
    rng = np.random.default_rng(3)
    mask = (rng.random(op.N) < 0.2).astype(np.uint8)
    I, _, _ = compact(mask)
    S_II, _ = restricted_operator(spec, I)
    Phi_eig = restricted_basis(gen.sine_modes_2d(n, 6)[0], I)[0]
    Phi_pod = restricted_basis(rng.standard_normal((op.N, 4)), I)[0]
    Z = safe_merge(S_II, Phi_eig, Phi_pod, tau_safe=np.inf)
    assert Z.shape[1] == 10
    assert np.array_equal(Z[:, :6], Phi_eig)
    assert np.allclose(Z.T @ Z, np.eye(10), atol=1e-12)
    U = np.column_stack([Phi_eig, Phi_pod])
    assert np.linalg.norm(U - Z @ (Z.T @ U)) <= 1e-10


# ---------------------------------------------------------------------------
# coarse-grid prolongation (Alg. 4)
# ---------------------------------------------------------------------------
def test_prolongation_1d_hat_functions():
    """Column j of P1D is the coarse hat function sampled at the fine nodes;
    for n = 2 n_c + 1 it copies coarse values and averages at midpoints."""
    from oracle.basis import prolongation_1d
    n, nc = 20, 7
    P = prolongation_1d(n, nc).toarray()
    x = np.arange(1, n + 1) / (n + 1)
    X = np.arange(1, nc + 1) / (nc + 1)
    H = 1.0 / (nc + 1)
    hat = np.maximum(0.0, 1.0 - np.abs(x[:, None] - X[None, :]) / H)
    assert np.allclose(P, hat, atol=1e-14)
    P2 = prolongation_1d(2 * nc + 1, nc).toarray()
    for j in range(nc):
        assert P2[2 * j + 1, j] == 1.0
    assert np.allclose(P2[0], 0.5 * np.eye(nc)[0])
    assert np.allclose(P2[2], 0.5 * (np.eye(nc)[0] + np.eye(nc)[1]))


def test_prolongation_kron_order_and_accuracy():
    """2D: P applied to a separable coarse field is the outer product of the
    1D interpolants (x fastest); prolonged coarse sine modes are within the
    linear-interpolation error bound of the fine sine modes."""
    from oracle.basis import coarse_basis, prolongation, prolongation_1d
    n, nc = 63, 31
    P1 = prolongation_1d(n, nc)
    g = np.random.default_rng(2).standard_normal(nc)
    hh = np.random.default_rng(3).standard_normal(nc)
    field = np.outer(hh, g).ravel()                     # [y][x], x fastest
    out = prolongation(n, nc, 2) @ field
    assert np.allclose(out, np.outer(P1 @ hh, P1 @ g).ravel(), atol=1e-13)
    Zc = gen.sine_modes_2d(nc, 3)[0]
    Q, keep = coarse_basis(Zc, n, nc, 2)
    assert keep.size == 3 and np.allclose(Q.T @ Q, np.eye(3), atol=1e-13)
    Zf = gen.sine_modes_2d(n, 3)[0]
    # interpolation error of sin(q pi x) on a grid of width H: (H q pi)^2 / 8
    H = 1.0 / (nc + 1)
    bound = 2 * (H * 2 * np.pi) ** 2 / 8
    assert np.linalg.norm(Zf - Q @ (Q.T @ Zf), 2) <= bound


def test_coarse_basis_drops_dependent_column():
    from oracle.basis import coarse_basis
    nc, n = 9, 19
    Zc = gen.sine_modes_2d(nc, 4)[0]
    Zc = np.column_stack([Zc[:, :2], Zc[:, 0] + 2 * Zc[:, 1], Zc[:, 2:]])
    Q, keep = coarse_basis(Zc, n, nc, 2)
    assert list(keep) == [0, 1, 3, 4]
    assert np.allclose(Q.T @ Q, np.eye(4), atol=1e-13)


def test_reference_eigs_closed_form():
    """2d_sym operator: eigenvalues 1 + alpha' (s_i + s_j)^2 with the sine
    modes as eigenvectors (Sec. "Analytical eigenmodes on tensor-product
    grids")."""
    from oracle.basis import reference_eigs
    n = 15
    op, spec = _sym_op(n)
    lam, U = reference_eigs(spec, 6)
    Z, pairs, _ = gen.sine_modes_2d(n, 6)
    h = 1.0 / (n + 1)
    s = lambda q: 4.0 * np.sin(q * np.pi * h / 2.0) ** 2
    ref = np.array(sorted(1.0 + op.alpha * (s(i) + s(j)) ** 2 for i, j in pairs))
    assert np.allclose(lam, ref, rtol=1e-12)
    assert np.linalg.norm(Z - U @ (U.T @ Z)) <= 1e-10


# ---------------------------------------------------------------------------
# space-time extension (App. "Space-time extension", eq. kron_basis)
# ---------------------------------------------------------------------------
def test_spacetime_forward_is_implicit_euler_and_blocks_match():
    """F y = u for y marched by implicit Euler from y^0 = 0; M_st = alpha
    F^T F + I has the block structure of the paper's figure: diagonal
    blocks alpha (D^T D + B^T B) + I except the last (alpha D^T D + I),
    off-diagonal blocks -alpha D^T B / -alpha B^T D, zero beyond."""
    import scipy.sparse.linalg as spla
    n, n_t, T, alpha = 6, 5, 1.0, 1e-3
    h = 1.0 / (n + 1)
    L = gen.laplacian_2d(n) / (h * h)
    F = gen.spacetime_forward(L, n_t, T)
    Ns, dt = n * n, T / n_t
    u = np.random.default_rng(4).standard_normal(Ns * n_t)
    D = (sp.identity(Ns) / dt + L).tocsc()
    y = np.zeros(Ns * n_t)
    prev = np.zeros(Ns)
    for k in range(n_t):
        prev = spla.spsolve(D, u[k * Ns:(k + 1) * Ns] + prev / dt)
        y[k * Ns:(k + 1) * Ns] = prev
    assert np.linalg.norm(F @ y - u) <= 1e-10 * np.linalg.norm(u)
    M = (alpha * (F.T @ F) + sp.identity(Ns * n_t)).toarray()
    Dd = D.toarray()
    Bb = np.eye(Ns) / dt
    blk = lambda i, j: M[i * Ns:(i + 1) * Ns, j * Ns:(j + 1) * Ns]
    for i in range(n_t):
        diag = alpha * (Dd.T @ Dd + (Bb.T @ Bb if i < n_t - 1 else 0)) + np.eye(Ns)
        assert np.allclose(blk(i, i), diag, rtol=1e-12, atol=1e-12 * np.abs(diag).max())
        if i + 1 < n_t:
            assert np.allclose(blk(i, i + 1), -alpha * Dd.T @ Bb, atol=1e-9)
            assert np.allclose(blk(i + 1, i), -alpha * Bb.T @ Dd, atol=1e-9)
        for j in range(i + 2, n_t):
            assert not blk(i, j).any() and not blk(j, i).any()


def test_kron_basis_structure():
    n, n_t, r = 5, 4, 3
    Zs = gen.sine_modes_2d(n, r)[0]
    Zst = gen.kron_basis(Zs, n_t)
    assert Zst.shape == (n * n * n_t, r * n_t)
    assert np.allclose(Zst.T @ Zst, np.eye(r * n_t), atol=1e-14)
    # column k r + j is mode j at time step k only
    Ns = n * n
    assert np.array_equal(Zst[2 * Ns:3 * Ns, 2 * r + 1], Zs[:, 1])
    assert not Zst[:2 * Ns, 2 * r + 1].any() and not Zst[3 * Ns:, 2 * r + 1].any()
    C = gen.const_time_basis(Zs, n_t)
    assert np.allclose(C, Zst @ np.kron(np.ones((n_t, 1)), np.eye(r)))
