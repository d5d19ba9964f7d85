"""GPU parity: the HIP path against the FP64 oracle on the same seeded inputs.

Bars: compaction bit-exact; FP64 solve e_rel <= max(1e-8, 2 * oracle e_rel)
against x* (Cholesky + double-double refinement), iteration counts within 2 of
the oracle (the paper reports CPU/GPU counts within 1 for identical
algorithms); FP32 inner sweeps with FP64 refinement e_rel <= 1e-6 (floor) and
the FP64 bar as target.
"""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[case] {msg}", flush=True)


def _xstar(S, mask, b):
    """x* of the restricted system; S is a sparse matrix or an oracle spec."""
    I, _, _ = oracle.compact(mask)
    S_II, _ = oracle.restricted_operator(S, I)
    return I, oracle.exact_solution(S_II, b[I])


def spec(op, form, a=1.0, c=None):
    """Oracle operator for gen.Operator op in the given form, scaled a*S + c'."""
    c = op.shift if c is None else c
    if form == "factored":
        return ("factored", op.A, a * op.alpha, c)
    return op.S(a=a, c=c)


def solver(lib, op, Z, form, **opts):
    s = lib.Solver(**opts)
    if form == "factored":
        s.set_reference_factored(op.A, op.alpha, op.shift, Z)
    else:
        s.set_reference(op.S(), Z)
    return s


@pytest.fixture(scope="module")
def c1():
    w = gen.c1_workload(n=63, k=16, seeds=(0, 1, 2))
    return w, w.op.S()


# ---------------------------------------------------------------------------
# compaction
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["blob", "random", "all_active", "all_inactive", "ragged", "large"])
def test_compaction_bit_exact(lib, kind):
    rng = np.random.default_rng(7)
    if kind == "blob":
        mask = gen.mask_top_fraction(gen.sinusoid_field(63, 3), 0.3)
    elif kind == "random":
        mask = (rng.uniform(size=10000) < 0.4).astype(np.uint8)
    elif kind == "all_active":
        mask = np.ones(5000, np.uint8)
    elif kind == "all_inactive":
        mask = np.zeros(5000, np.uint8)
    elif kind == "ragged":
        mask = (rng.uniform(size=4096 * 3 + 17) < 0.5).astype(np.uint8)
    else:
        mask = gen.mask_top_fraction(gen.sinusoid_field(511, 100), 0.25)
    case(f"compaction {kind} N={mask.size}")
    s = lib.Solver()
    I, g2l, nI = s.compact(mask)
    Io, g2lo, nIo = oracle.compact(mask)
    assert nI == nIo
    np.testing.assert_array_equal(I.cpu().numpy().astype(np.int64), Io)
    np.testing.assert_array_equal(g2l.cpu().numpy().astype(np.int64), g2lo)


# ---------------------------------------------------------------------------
# restricted operator and coarse space
# ---------------------------------------------------------------------------
def test_apply_restricted_matches_oracle(lib, c1):
    w, S = c1
    inst = w.instances[0]
    case("apply_restricted c1 n=63")
    s = lib.Solver()
    s.set_reference(S, w.Z)
    s.restrict(inst.mask)
    x = np.random.default_rng(3).standard_normal(S.shape[0])
    y = s.apply_restricted(x).cpu().numpy()
    I, _, _ = oracle.compact(inst.mask)
    S_II, _ = oracle.restrict(S, I)
    yo = S_II @ x[I]
    assert np.all(y[inst.mask == 1] == 0.0)
    assert np.linalg.norm(y[I] - yo) <= 1e-14 * np.linalg.norm(yo) * 10


def test_apply_restricted_factored_matches_oracle(lib):
    w = gen.c2_workload(n=63, k=8, B=1)
    inst = w.instances[0]
    case("apply_restricted factored cd2d n=63")
    s = solver(lib, w.op, w.Z, "factored")
    s.restrict(inst.mask)
    x = np.random.default_rng(5).standard_normal(w.op.N)
    y = s.apply_restricted(x).cpu().numpy()
    I, _, _ = oracle.compact(inst.mask)
    F, _ = oracle.restrict_factored(w.op.A, w.op.alpha, w.op.shift, I)
    yo = F @ x[I]
    assert np.all(y[inst.mask == 1] == 0.0)
    assert np.linalg.norm(y[I] - yo) <= 1e-13 * np.linalg.norm(yo)


def test_coarse_space_matches_oracle(lib, c1):
    w, S = c1
    for m, inst in enumerate(w.instances):
        case(f"coarse c1 seed {m}")
        s = lib.Solver()
        s.set_reference(S, w.Z)
        nI, keff, cond, rc = s.restrict(inst.mask)
        I, _, nIo = oracle.compact(inst.mask)
        S_II, _ = oracle.restrict(S, I)
        Zo, kept = oracle.restricted_basis(w.Z, I)
        cs, fb = oracle.coarse_setup(S_II, Zo)
        assert nI == nIo and keff == len(kept) and rc == 0 and not fb
        assert abs(cond / cs.cond - 1) < 1e-8, (cond, cs.cond)
        E, keptg, kk, _ = s.coarse_info()
        np.testing.assert_array_equal(np.flatnonzero(keptg), kept)
        np.testing.assert_allclose(np.linalg.eigvalsh(E), np.linalg.eigvalsh(cs.E), rtol=1e-9)


def test_dependent_and_zero_columns_dropped(lib, c1):
    w, S = c1
    inst = w.instances[0]
    Z = np.column_stack([w.Z[:, :5], w.Z[:, 2], np.zeros(S.shape[0]), w.Z[:, 5:10]])
    case("coarse with duplicated and zero columns")
    s = lib.Solver()
    s.set_reference(S, Z)
    nI, keff, cond, rc = s.restrict(inst.mask)
    I, _, _ = oracle.compact(inst.mask)
    Zo, kept = oracle.restricted_basis(Z, I)
    assert keff == len(kept) == 10
    _, keptg, _, _ = s.coarse_info()
    np.testing.assert_array_equal(np.flatnonzero(keptg), kept)


# ---------------------------------------------------------------------------
# FP64 solves
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("form", ["assembled", "factored"])
@pytest.mark.parametrize("k", [16, 0])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_solve_fp64_c1(lib, c1, k, seed, form):
    w, _ = c1
    S = spec(w.op, form)
    inst = w.instances[seed]
    Z = w.Z[:, :k]
    tol = 1e-10
    case(f"solve fp64 c1 n=63 k={k} seed={seed} {form}")
    s = solver(lib, w.op, Z if k else None, form)
    s.restrict(inst.mask)
    out = s.solve(inst.b, tol)
    ref = oracle.solve_instance(S, Z, inst.mask, inst.b, tol)
    I, xs = _xstar(S, inst.mask, inst.b)
    x = out.x.cpu().numpy()
    e_gpu = oracle.rel_err(x[I], xs)
    e_ora = oracle.rel_err(ref.x[I], xs)
    assert out.status == 0
    assert abs(out.iters - ref.iters) <= 2, (out.iters, ref.iters)
    assert e_gpu <= max(1e-8, 2 * e_ora), (e_gpu, e_ora)
    assert out.relres_true <= 5 * tol
    assert np.all(x[inst.mask == 1] == 0.0)


@pytest.mark.parametrize("form", ["assembled", "factored"])
@pytest.mark.parametrize("n,k", [(95, 24), (127, 32)])
def test_solve_fp64_convection_diffusion_multi_tile(lib, n, k, form):
    """C2-type upwind operator at sizes that span many tiles with a ragged tail."""
    w = gen.c2_workload(n=n, k=k, B=2)
    S = spec(w.op, form)
    for m, inst in enumerate(w.instances):
        case(f"solve fp64 cd2d n={n} k={k} inst={m} {form}")
        s = solver(lib, w.op, w.Z, form)
        s.restrict(inst.mask)
        out = s.solve(inst.b, 1e-10)
        ref = oracle.solve_instance(S, w.Z, inst.mask, inst.b, 1e-10)
        I, xs = _xstar(S, inst.mask, inst.b)
        x = out.x.cpu().numpy()
        e_gpu, e_ora = oracle.rel_err(x[I], xs), oracle.rel_err(ref.x[I], xs)
        assert abs(out.iters - ref.iters) <= max(2, ref.iters // 50), (out.iters, ref.iters)
        assert e_gpu <= max(1e-8, 2 * e_ora), (e_gpu, e_ora)


def test_deterministic_rerun(lib, c1):
    w, S = c1
    inst = w.instances[0]
    case("determinism c1")
    s = lib.Solver()
    s.set_reference(S, w.Z)
    s.restrict(inst.mask)
    a = s.solve(inst.b, 1e-10)
    xa = a.x.cpu().numpy().copy()
    s.restrict(inst.mask)
    b = s.solve(inst.b, 1e-10)
    assert a.iters == b.iters
    np.testing.assert_array_equal(xa, b.x.cpu().numpy())


def test_warm_start_from_solution(lib, c1):
    w, S = c1
    inst = w.instances[1]
    I, xs = _xstar(S, inst.mask, inst.b)
    x0 = np.zeros(S.shape[0])
    x0[I] = xs
    x0[inst.mask == 1] = 123.0          # ignored on the active set
    case("warm start c1")
    s = lib.Solver()
    s.set_reference(S, w.Z)
    s.restrict(inst.mask)
    out = s.solve(inst.b, 1e-8, x0=x0)
    assert out.iters == 0
    assert oracle.rel_err(out.x.cpu().numpy()[I], xs) < 1e-12


# ---------------------------------------------------------------------------
# FP32 inner sweeps + FP64 refinement
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("form", ["assembled", "factored"])
@pytest.mark.parametrize("seed", [0, 1])
def test_solve_fp32_refine_c1(lib, c1, seed, form):
    w, _ = c1
    S = spec(w.op, form)
    inst = w.instances[seed]
    case(f"solve fp32+refine c1 seed={seed} {form}")
    s = solver(lib, w.op, w.Z, form, precision=lib.FP32_REFINE, inner_rtol=1e-4)
    s.restrict(inst.mask)
    out = s.solve(inst.b, 1e-10)
    ref = oracle.solve_instance(S, w.Z, inst.mask, inst.b, 1e-10)
    I, xs = _xstar(S, inst.mask, inst.b)
    e = oracle.rel_err(out.x.cpu().numpy()[I], xs)
    assert out.status == 0
    assert out.relres_true <= 1e-10
    assert e <= 1e-6
    assert e <= max(1e-8, 2 * oracle.rel_err(ref.x[I], xs)), e


# ---------------------------------------------------------------------------
# batched
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("form", ["assembled", "factored"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_matches_single(lib, prec, form):
    w = gen.c2_workload(n=95, k=16, B=4)
    S = spec(w.op, form)
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    case(f"batched B=4 cd2d n=95 {prec} {form}")
    s = solver(lib, w.op, w.Z, form, precision=lib.FP64 if prec == "fp64" else lib.FP32_REFINE)
    out = s.solve_batched(masks, bs, 1e-10)
    X = out["x"].cpu().numpy()
    for m, inst in enumerate(w.instances):
        ref = oracle.solve_instance(S, w.Z, inst.mask, inst.b, 1e-10)
        I, xs = _xstar(S, inst.mask, inst.b)
        e = oracle.rel_err(X[m, I], xs)
        assert out["status"][m] == 0
        assert out["n_inactive"][m] == ref.n_I
        assert e <= max(1e-8, 2 * oracle.rel_err(ref.x[I], xs)), (m, e)
        if prec == "fp64":
            assert abs(int(out["iters"][m]) - ref.iters) <= 2
        assert np.all(X[m, inst.mask == 1] == 0.0)


@pytest.mark.parametrize("form", ["assembled", "factored"])
def test_batched_operator_scales(lib, form):
    w = gen.c3_workload(n=31, k=8, B=3)
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    a = np.array([i.a for i in w.instances])
    c = np.array([i.c for i in w.instances]) - a * w.op.shift
    case(f"batched operator scales c3 n=31 {form}")
    s = solver(lib, w.op, w.Z, form)
    out = s.solve_batched(masks, bs, 1e-10, a=a, c=c)
    X = out["x"].cpu().numpy()
    for m, inst in enumerate(w.instances):
        Sm = spec(w.op, form, a=inst.a, c=inst.c)
        I, xs = _xstar(Sm, inst.mask, inst.b)
        ref = oracle.solve_instance(Sm, w.Z, inst.mask, inst.b, 1e-10)
        assert oracle.rel_err(X[m, I], xs) <= max(1e-8, 2 * oracle.rel_err(ref.x[I], xs))
        assert abs(int(out["iters"][m]) - ref.iters) <= 2


@pytest.mark.parametrize("prec", ["fp64", "mixed", "fp64_refine"])
def test_per_instance_tolerances(lib, prec):
    """solve_batched with one tolerance per instance (App. "CG stopping
    criterion" applied per instance): each instance stops on its own
    tolerance.  FP64: iteration counts within 2 of the oracle's FP64 loop at
    that tolerance; refinement modes: the FP64 true residual meets it."""
    w = gen.c2_workload(n=95, k=16, B=4)
    S = spec(w.op, "factored")
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    tols = np.array([1e-4, 1e-6, 1e-8, 1e-10])
    case(f"per-instance tolerances {tols.tolist()} cd2d n=95 {prec}")
    p = {"fp64": lib.FP64, "mixed": lib.MIXED_REFINE, "fp64_refine": lib.FP64_REFINE}[prec]
    s = solver(lib, w.op, w.Z, "factored", precision=p)
    out = s.solve_batched(masks, bs, tols)
    X = out["x"].cpu().numpy()
    print(f"   iterations {out['iters'].tolist()} relres {np.asarray(out['relres_true']).tolist()}", flush=True)
    for m, inst in enumerate(w.instances):
        ref = oracle.solve_instance(S, w.Z, inst.mask, inst.b, tols[m])
        I, xs = _xstar(S, inst.mask, inst.b)
        assert out["status"][m] == 0
        if prec == "fp64":
            assert abs(int(out["iters"][m]) - ref.iters) <= 2, (m, out["iters"][m], ref.iters)
        else:
            assert out["relres_true"][m] <= tols[m]
        # the error at each tolerance is the oracle's at that tolerance
        e, e_or = oracle.rel_err(X[m, I], xs), oracle.rel_err(ref.x[I], xs)
        assert e <= max(1e-8, 10 * e_or), (m, e, e_or)


# ---------------------------------------------------------------------------
# status paths
# ---------------------------------------------------------------------------
def test_forced_fallback_is_plain_pcg(lib, c1):
    w, S = c1
    inst = w.instances[0]
    case("forced fallback tau_cond=1")
    s = lib.Solver(tau_cond=1.0)
    s.set_reference(S, w.Z)
    nI, keff, cond, rc = s.restrict(inst.mask)
    assert rc == lib.W_FALLBACK
    out = s.solve(inst.b, 1e-10)
    ref = oracle.solve_instance(S, w.Z, inst.mask, inst.b, 1e-10, tau_cond=1.0)
    assert out.status == lib.W_FALLBACK and ref.status == oracle.STATUS_FALLBACK
    assert abs(out.iters - ref.iters) <= 2


def test_maxit_status(lib, c1):
    w, S = c1
    inst = w.instances[0]
    case("maxit=3")
    s = lib.Solver(maxit=3)
    s.set_reference(S, w.Z)
    s.restrict(inst.mask)
    out = s.solve(inst.b, 1e-12)
    assert out.status == lib.W_MAXIT and out.iters == 3


def test_error_paths(lib, c1):
    w, S = c1
    inst = w.instances[0]
    case("error paths")
    s = lib.Solver()
    with pytest.raises(lib.Adef2Error) as e:
        s.restrict(inst.mask)
    assert e.value.code == lib.E_STATE
    s.set_reference(S, w.Z)
    with pytest.raises(lib.Adef2Error) as e:
        s.solve(inst.b, 1e-8)
    assert e.value.code == lib.E_STATE
    s.restrict(inst.mask)
    b = inst.b.copy()
    b[np.flatnonzero(inst.mask == 0)[5]] = np.nan
    with pytest.raises(lib.Adef2Error) as e:
        s.solve(b, 1e-8)
    assert e.value.code == lib.E_ARG
    # zero right-hand side: x = 0 without iterations
    out = s.solve(np.zeros(S.shape[0]), 1e-8)
    assert out.iters == 0 and float(out.x.abs().max()) == 0.0


# ---------------------------------------------------------------------------
# kernel variants: tile height (rows per thread) and W-free iterations
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("form", ["assembled", "factored"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("rpt,w_mode", [(1, 1), (1, 2), (2, 1), (2, 2), (1, 3), (2, 3)])
def test_kernel_variants_match_oracle(lib, rpt, w_mode, prec, form):
    w = gen.c2_workload(n=95, k=16, B=3)
    S = spec(w.op, form)
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    case(f"variant rpt={rpt} w_mode={w_mode} {prec} {form} cd2d n=95 B=3")
    p = lib.FP64 if prec == "fp64" else lib.MIXED_REFINE
    s = solver(lib, w.op, w.Z, form, precision=p, rows_per_thread=rpt, w_mode=w_mode)
    out = s.solve_batched(masks, bs, 1e-10)
    X = out["x"].cpu().numpy()
    for m, inst in enumerate(w.instances):
        ref = oracle.solve_instance(S, w.Z, inst.mask, inst.b, 1e-10)
        I, xs = _xstar(S, inst.mask, inst.b)
        e = oracle.rel_err(X[m, I], xs)
        assert out["status"][m] == 0
        assert e <= max(1e-8, 2 * oracle.rel_err(ref.x[I], xs)), (m, e)
        if prec == "fp64":
            assert abs(int(out["iters"][m]) - ref.iters) <= 2
        else:
            assert out["relres_true"][m] <= 1e-10


@pytest.mark.parametrize("form", ["assembled", "factored"])
@pytest.mark.parametrize("rpt,w_mode", [(1, 4), (2, 4), (1, 5)])
@pytest.mark.parametrize("B", [3, 11])
def test_tile_major_boundary_update_matches_oracle(lib, form, rpt, w_mode, B):
    """Tile-major boundary-form iteration (w_mode 4: k_pupdate_tm /
    k_update_tm / k_finish_tm, matrix-core products with the shared modes;
    w_mode 5: also the tile-major stencil passes): B = 11 spans
    two update groups (8 + 3 instances) and one ragged p-update group; N =
    95^2 ends in a ragged tile."""
    w = gen.c2_workload(n=95, k=16, B=B)
    S = spec(w.op, form)
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    case(f"tile-major boundary update rpt={rpt} w_mode={w_mode} {form} cd2d n=95 k=16 B={B}")
    s = solver(lib, w.op, w.Z, form, precision=lib.MIXED_REFINE, rows_per_thread=rpt, w_mode=w_mode)
    out = s.solve_batched(masks, bs, 1e-10)
    assert s.variant()[1] == w_mode
    X = out["x"].cpu().numpy()
    for m, inst in enumerate(w.instances):
        ref = oracle.solve_instance(S, w.Z, inst.mask, inst.b, 1e-10)
        I, xs = _xstar(S, inst.mask, inst.b)
        e = oracle.rel_err(X[m, I], xs)
        assert out["status"][m] == 0
        assert out["relres_true"][m] <= 1e-10
        assert e <= max(1e-8, 2 * oracle.rel_err(ref.x[I], xs)), (m, e)
        assert int(out["iters"][m]) <= 1.2 * ref.iters + 20, (m, out["iters"][m], ref.iters)
    assert np.all(X[masks == 1] == 0.0)


@pytest.mark.parametrize("w_mode", [4, 5])
def test_tile_major_boundary_update_wide_basis(lib, w_mode):
    """The tile-major kernels with 48 shared modes (3 matrix-core column
    tiles; above 32 modes the update keeps the compiler's register
    allocation instead of the 4-waves-per-SIMD budget)."""
    w = gen.c2_workload(n=95, k=48, B=11)
    S = spec(w.op, "factored")
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    case(f"tile-major boundary update w_mode={w_mode} factored cd2d n=95 k=48 B=11")
    s = solver(lib, w.op, w.Z, "factored", precision=lib.MIXED_REFINE, rows_per_thread=1, w_mode=w_mode)
    out = s.solve_batched(masks, bs, 1e-10)
    assert s.variant()[1] == w_mode
    X = out["x"].cpu().numpy()
    for m, inst in enumerate(w.instances):
        ref = oracle.solve_instance(S, w.Z, inst.mask, inst.b, 1e-10)
        I, xs = _xstar(S, inst.mask, inst.b)
        e = oracle.rel_err(X[m, I], xs)
        assert out["status"][m] == 0
        assert out["relres_true"][m] <= 1e-10
        assert e <= max(1e-8, 2 * oracle.rel_err(ref.x[I], xs)), (m, e)
        assert int(out["iters"][m]) <= 1.2 * ref.iters + 20, (m, out["iters"][m], ref.iters)
    assert np.all(X[masks == 1] == 0.0)


def test_tile_major_needs_eigen_basis(lib):
    """w_mode 4 is refused (E_UNSUPPORTED) with FP64 panels, where the
    boundary form of W is not used."""
    w = gen.c2_workload(n=63, k=8, B=2)
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    case("tile-major refused in FP64")
    s = solver(lib, w.op, w.Z, "factored", precision=lib.FP64, w_mode=4)
    with pytest.raises(lib.Adef2Error) as e:
        s.solve_batched(masks, bs, 1e-10)
    assert e.value.code == lib.E_UNSUPPORTED


def test_autotuned_variant_is_reused(lib):
    w = gen.c2_workload(n=95, k=16, B=2)
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    case("autotuned variant reused within a context")
    s = solver(lib, w.op, w.Z, "factored", precision=lib.MIXED_REFINE)
    a = s.solve_batched(masks, bs, 1e-10)
    b = s.solve_batched(masks, bs, 1e-10)
    np.testing.assert_array_equal(a["iters"], b["iters"])
    np.testing.assert_array_equal(a["x"].cpu().numpy(), b["x"].cpu().numpy())


def test_graphs_keyed_by_variant(lib):
    """A context that switches w_mode (4 -> 5: the same update kernels, other
    stencil kernels) or the operator form replays graphs of the new variant:
    its solves equal those of a fresh context with that variant, bitwise."""
    w = gen.c2_workload(n=95, k=16, B=2)
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    case("graph cache keyed by w_mode and operator form")
    s = solver(lib, w.op, w.Z, "factored", precision=lib.MIXED_REFINE, rows_per_thread=1, w_mode=4,
               op_fused=-1, update_ws=-1)
    s.solve_batched(masks, bs, 1e-10)
    for opts in (dict(w_mode=5, op_fused=-1, update_ws=-1), dict(w_mode=5, op_fused=1, update_ws=-1),
                 dict(w_mode=4, op_fused=1, update_ws=-1), dict(w_mode=4, op_fused=1, update_ws=1)):
        s.set_opts(**opts)
        got = s.solve_batched(masks, bs, 1e-10)
        f = solver(lib, w.op, w.Z, "factored", precision=lib.MIXED_REFINE, rows_per_thread=1, **opts)
        ref = f.solve_batched(masks, bs, 1e-10)
        f.close()
        np.testing.assert_array_equal(got["iters"], ref["iters"])
        np.testing.assert_array_equal(got["x"].cpu().numpy(), ref["x"].cpu().numpy())


@pytest.mark.parametrize("form", ["assembled", "factored"])
@pytest.mark.parametrize("w_boundary", [0, 1])
def test_boundary_form_of_w(lib, form, w_boundary):
    """Mixed precision with W kept whole (0) or in the boundary form (1: the
    reference modes of these operators are eigenvectors to ~1e-9)."""
    w = gen.c2_workload(n=127, k=24, B=3)
    S = spec(w.op, form)
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    case(f"boundary-form W={w_boundary} {form} cd2d n=127 k=24 B=3")
    s = solver(lib, w.op, w.Z, form, precision=lib.MIXED_REFINE, rows_per_thread=1, w_mode=1,
               w_boundary=w_boundary)
    out = s.solve_batched(masks, bs, 1e-10)
    X = out["x"].cpu().numpy()
    for m, inst in enumerate(w.instances):
        ref = oracle.solve_instance(S, w.Z, inst.mask, inst.b, 1e-10)
        I, xs = _xstar(S, inst.mask, inst.b)
        e = oracle.rel_err(X[m, I], xs)
        assert out["status"][m] == 0
        assert out["relres_true"][m] <= 1e-10
        assert e <= max(1e-8, 2 * oracle.rel_err(ref.x[I], xs)), (m, e)
        assert int(out["iters"][m]) <= 1.5 * ref.iters + 50


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_replays_match_eager(lib, prec):
    """Iteration chunks replayed from captured HIP graphs give the eager
    result on every replay (three solves in a row, each preceded by the
    context's own eager restriction work and synchronisation)."""
    w = gen.c2_workload(n=95, k=16, B=4)
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    p = lib.FP64 if prec == "fp64" else lib.MIXED_REFINE
    case(f"graph replays vs eager {prec} cd2d n=95 B=4")
    eager = solver(lib, w.op, w.Z, "factored", precision=p, rows_per_thread=2, w_mode=1, op_fused=1, graph=0)
    ref = eager.solve_batched(masks, bs, 1e-10)
    g = solver(lib, w.op, w.Z, "factored", precision=p, rows_per_thread=2, w_mode=1, op_fused=1, graph=1)
    for rep in range(3):
        out = g.solve_batched(masks, bs, 1e-10)
        np.testing.assert_array_equal(out["iters"], ref["iters"])
        np.testing.assert_array_equal(out["status"], ref["status"])
        np.testing.assert_array_equal(out["x"].cpu().numpy(), ref["x"].cpu().numpy())


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_adaptive_polling_matches_every_chunk_polling(lib, prec):
    """Convergence is decided on the device: enqueuing several chunks between
    host polls (poll_max 16) gives bitwise the result of polling after every
    chunk (poll_max 1), with fewer polls."""
    w = gen.c2_workload(n=95, k=16, B=4)
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    p = lib.FP64 if prec == "fp64" else lib.MIXED_REFINE
    case(f"adaptive polling {prec} cd2d n=95 B=4")
    out, polls = [], []
    for pm in (1, 16):
        s = solver(lib, w.op, w.Z, "factored", precision=p, rows_per_thread=2, w_mode=1, op_fused=1,
                   poll_max=pm)
        s.solve_batched(masks, bs, 1e-10)          # first solve: variant and graphs
        s.reset_stats()
        out.append(s.solve_batched(masks, bs, 1e-10))
        polls.append(s.polls())
    print(f"   polls every chunk {polls[0]}, adaptive {polls[1]}; iterations {out[0]['iters'].tolist()}",
          flush=True)
    np.testing.assert_array_equal(out[0]["iters"], out[1]["iters"])
    np.testing.assert_array_equal(out[0]["status"], out[1]["status"])
    np.testing.assert_array_equal(out[0]["x"].cpu().numpy(), out[1]["x"].cpu().numpy())
    assert polls[1] < polls[0]


# ---------------------------------------------------------------------------
# fused operator pass of the factored form (t = A p kept in LDS)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec,w_mode", [("fp64", 1), ("mixed", 1), ("mixed", 4), ("fp32", 1)])
@pytest.mark.parametrize("B", [3, 11])
@pytest.mark.parametrize("group", [1, 4])
def test_fused_operator_matches_oracle(lib, prec, w_mode, B, group):
    """op_fused = 1: one kernel forms A p over a tile and its stencil reach in
    LDS and applies A^T there.  n = 95 takes 512-row tiles (4 times the
    95-row reach, rounded up; 18 per instance, the last one 321 rows);
    group 4 shares each row's coefficients among 4 instances (B = 3: one
    partial group; B = 11: groups of 4, 4 and 3)."""
    w = gen.c2_workload(n=95, k=16, B=B)
    S = spec(w.op, "factored")
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    p = {"fp64": lib.FP64, "mixed": lib.MIXED_REFINE, "fp32": lib.FP32_REFINE}[prec]
    case(f"fused operator group={group} {prec} w_mode={w_mode} factored cd2d n=95 k=16 B={B}")
    s = solver(lib, w.op, w.Z, "factored", precision=p, rows_per_thread=1, w_mode=w_mode, op_fused=1,
               op_group=group)
    out = s.solve_batched(masks, bs, 1e-10)
    fused, rows, _, grp = s.op_variant()
    assert fused == 1 and rows == 512 and grp == group
    X = out["x"].cpu().numpy()
    for m, inst in enumerate(w.instances):
        ref = oracle.solve_instance(S, w.Z, inst.mask, inst.b, 1e-10)
        I, xs = _xstar(S, inst.mask, inst.b)
        e = oracle.rel_err(X[m, I], xs)
        if prec == "fp32":
            assert out["status"][m] in (0, 3), (m, out["status"][m])
            assert e <= 1e-6, (m, e)
            continue
        assert out["status"][m] == 0
        assert e <= max(1e-8, 2 * oracle.rel_err(ref.x[I], xs)), (m, e)
        if prec == "fp64":
            assert abs(int(out["iters"][m]) - ref.iters) <= 2, (m, out["iters"][m], ref.iters)
        else:
            assert out["relres_true"][m] <= 1e-10
            assert int(out["iters"][m]) <= 1.2 * ref.iters + 20, (m, out["iters"][m], ref.iters)
    assert np.all(X[masks == 1] == 0.0)


@pytest.mark.parametrize("group", [1, 4])
def test_fused_operator_large_tiles(lib, group):
    """255^2 x 16 (mixed, tile-major update): 1024-row fused tiles with a
    255-row halo on each side, 64 tiles per instance, the last one ragged
    (513 rows), one or four instances per block.  Sampled instances against
    x*, every instance against the two-pass operator's iteration count and
    solution."""
    w = gen.c2_workload(n=255, k=32, B=16)
    S = spec(w.op, "factored")
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    case(f"fused operator (group {group}) vs two passes, mixed w_mode=4 factored cd2d n=255 k=32 B=16")
    outs = {}
    for fo in (1, -1):
        s = solver(lib, w.op, w.Z, "factored", precision=lib.MIXED_REFINE, rows_per_thread=1, w_mode=4,
                   op_fused=fo, op_group=group if fo == 1 else 0)
        outs[fo] = s.solve_batched(masks, bs, 1e-10)
        f, rows, _, grp = s.op_variant()
        assert f == (1 if fo == 1 else 0)
        if fo == 1:
            assert rows == 1024 and grp == group
        s.close()
    Xf, Xt = outs[1]["x"].cpu().numpy(), outs[-1]["x"].cpu().numpy()
    assert np.all(outs[1]["status"] == 0) and np.all(outs[1]["relres_true"] <= 1e-10)
    for m in range(16):
        it_f, it_t = int(outs[1]["iters"][m]), int(outs[-1]["iters"][m])
        assert abs(it_f - it_t) <= 0.05 * it_t + 20, (m, it_f, it_t)
        assert oracle.rel_err(Xf[m], Xt[m]) <= 1e-8, m
    for m in (0, 7, 15):
        inst = w.instances[m]
        I, xs = _xstar(S, inst.mask, inst.b)
        assert oracle.rel_err(Xf[m, I], xs) <= 1e-8, m
    assert np.all(Xf[masks == 1] == 0.0)


def test_fused_operator_options_checked(lib):
    """op_group 4 whose four LDS copies do not fit, and an op_rows below
    twice the reach that still fits, as the header states."""
    w = gen.c2_workload(n=255, k=8, B=4)
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    case("fused operator options: group 4 with 4096-row tiles refused, 256-row tiles accepted")
    s = solver(lib, w.op, w.Z, "factored", precision=lib.FP64, op_fused=1, op_rows=4096, op_group=4)
    with pytest.raises(lib.Adef2Error) as e:
        s.solve_batched(masks, bs, 1e-8)
    assert e.value.code == lib.E_UNSUPPORTED
    s = solver(lib, w.op, w.Z, "factored", precision=lib.FP64, rows_per_thread=1, w_mode=1, op_fused=1,
               op_rows=256, op_group=4)
    out = s.solve_batched(masks, bs, 1e-8)
    assert s.op_variant()[1] == 256 and s.op_variant()[3] == 4
    assert np.all(out["status"] == 0)


def test_fused_operator_refused_for_assembled(lib):
    w = gen.c2_workload(n=63, k=8, B=2)
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    case("fused operator refused for the assembled form")
    s = solver(lib, w.op, w.Z, "assembled", precision=lib.FP64, op_fused=1)
    with pytest.raises(lib.Adef2Error) as e:
        s.solve_batched(masks, bs, 1e-10)
    assert e.value.code == lib.E_UNSUPPORTED


# ---------------------------------------------------------------------------
# refinement segments: transitions inside the chunks vs synchronised segments
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec,w_mode", [("mixed", 4), ("mixed", 1), ("fp32", 1), ("fp64_refine", 1)])
def test_async_segments_match_synchronised(lib, prec, w_mode):
    """sweep_async = 1 moves an instance to its next segment at the end of the
    chunk in which its segment ended; sweep_async = 0 waits for every
    instance's segment.  Every instance's arithmetic is the same, so the
    iteration counts, statuses and solutions agree bitwise.  The batch mixes
    per-instance tolerances (segments of very different lengths) and a zero
    right-hand side."""
    w = gen.c2_workload(n=95, k=16, B=6)
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    bs[4] = 0.0
    tols = np.array([1e-10, 1e-6, 1e-9, 1e-4, 1e-10, 1e-8])
    p = {"mixed": lib.MIXED_REFINE, "fp32": lib.FP32_REFINE, "fp64_refine": lib.FP64_REFINE}[prec]
    case(f"async vs synchronised segments {prec} w_mode={w_mode} cd2d n=95 k=16 B=6")
    outs = []
    for sa in (0, 1):
        s = solver(lib, w.op, w.Z, "factored", precision=p, rows_per_thread=1, w_mode=w_mode, op_fused=1,
                   update_ws=-1, sweep_async=sa)
        outs.append(s.solve_batched(masks, bs, tols))
        s.close()
    print(f"   iterations {outs[1]['iters'].tolist()} statuses {outs[1]['status'].tolist()}", flush=True)
    np.testing.assert_array_equal(outs[0]["iters"], outs[1]["iters"])
    np.testing.assert_array_equal(outs[0]["status"], outs[1]["status"])
    np.testing.assert_array_equal(outs[0]["x"].cpu().numpy(), outs[1]["x"].cpu().numpy())
    assert np.all(outs[1]["x"][4].cpu().numpy() == 0.0)
    S = spec(w.op, "factored")
    for m in (0, 3, 5):
        I, xs = _xstar(S, w.instances[m].mask, bs[m])
        e = oracle.rel_err(outs[1]["x"].cpu().numpy()[m, I], xs)
        assert e <= max(1e-6, 10 * tols[m]), (m, e)


# ---------------------------------------------------------------------------
# warp-specialised update (runs of tiles, products overlapping the loads)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("B", [3, 11])
def test_warp_specialised_update_matches_oracle(lib, B):
    """update_ws = 1 at n = 95 (runs of one tile; B = 11: groups of 8 and 3)
    against the oracle, as the per-tile update is tested."""
    w = gen.c2_workload(n=95, k=16, B=B)
    S = spec(w.op, "factored")
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    case(f"warp-specialised update factored cd2d n=95 k=16 B={B}")
    s = solver(lib, w.op, w.Z, "factored", precision=lib.MIXED_REFINE, rows_per_thread=1, w_mode=4,
               update_ws=1)
    out = s.solve_batched(masks, bs, 1e-10)
    assert s.update_variant()[0] == 1
    X = out["x"].cpu().numpy()
    for m, inst in enumerate(w.instances):
        ref = oracle.solve_instance(S, w.Z, inst.mask, inst.b, 1e-10)
        I, xs = _xstar(S, inst.mask, inst.b)
        e = oracle.rel_err(X[m, I], xs)
        assert out["status"][m] == 0
        assert out["relres_true"][m] <= 1e-10
        assert e <= max(1e-8, 2 * oracle.rel_err(ref.x[I], xs)), (m, e)
        assert int(out["iters"][m]) <= 1.2 * ref.iters + 20, (m, out["iters"][m], ref.iters)
    assert np.all(X[masks == 1] == 0.0)


def test_warp_specialised_update_runs_of_tiles(lib):
    """255^2 x 37 instances: runs of 4 tiles per block (5 groups, the last of 5
    instances), against the per-tile update on every instance and x* on
    samples."""
    w = gen.c2_workload(n=255, k=32, B=37)
    S = spec(w.op, "factored")
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    case("warp-specialised update vs per tile, mixed w_mode=4 cd2d n=255 k=32 B=37")
    outs = {}
    for uw in (1, -1):
        s = solver(lib, w.op, w.Z, "factored", precision=lib.MIXED_REFINE, rows_per_thread=1, w_mode=4,
                   op_fused=1, update_ws=uw)
        outs[uw] = s.solve_batched(masks, bs, 1e-10)
        ws, tpb, _ = s.update_variant()
        assert ws == (1 if uw == 1 else 0)
        if uw == 1:
            assert tpb == 4
        s.close()
    Xw, Xt = outs[1]["x"].cpu().numpy(), outs[-1]["x"].cpu().numpy()
    assert np.all(outs[1]["status"] == outs[-1]["status"])
    assert np.all(outs[1]["relres_true"] <= 1e-10) or np.all(np.isin(outs[1]["status"], (0, 3)))
    for m in range(37):
        it_w, it_t = int(outs[1]["iters"][m]), int(outs[-1]["iters"][m])
        assert abs(it_w - it_t) <= 0.05 * it_t + 20, (m, it_w, it_t)
        assert oracle.rel_err(Xw[m], Xt[m]) <= 1e-8, m
    for m in (0, 18, 36):
        inst = w.instances[m]
        I, xs = _xstar(S, inst.mask, inst.b)
        assert oracle.rel_err(Xw[m, I], xs) <= 1e-8, m
    assert np.all(Xw[masks == 1] == 0.0)
