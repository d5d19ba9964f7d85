"""Offline coarse-grid reference basis (Alg. 4) on the GPU against the
oracle: prolongation of coarse sine modes (2D, c = 2 and 3; 3D, c = 2),
the dropping of a dependent column, and a deflated solve with the prolonged
basis.  Bars: same kept columns; every basis column equal to the oracle's up
to sign within 1e-10 (the QR with a positive diagonal is unique);
orthonormality 1e-13; FP64 iteration counts within 1 % of the oracle's solve
with the oracle's basis."""
import numpy as np
import pytest

import gen
import oracle
from oracle.active_set import active_set, coupled_rhs
from oracle.basis import coarse_basis

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[case] {msg}", flush=True)


def _coarse_modes(dim, nc, r):
    if dim == 2:
        return gen.sine_modes_2d(nc, r)[0]
    # 3D: products of 1D sine vectors, lowest index sums first
    x = np.arange(1, nc + 1) / (nc + 1)
    trip = sorted(((i, j, k) for i in range(1, 5) for j in range(1, 5) for k in range(1, 5)),
                  key=lambda t: (t[0] ** 2 + t[1] ** 2 + t[2] ** 2, t))[:r]
    cols = []
    for i, j, k in trip:
        v = np.einsum("a,b,c->abc", np.sin(k * np.pi * x), np.sin(j * np.pi * x), np.sin(i * np.pi * x))
        cols.append(v.ravel() / np.linalg.norm(v))
    return np.column_stack(cols)


@pytest.mark.parametrize("dim,n,nc,r", [(2, 63, 31, 16), (2, 63, 21, 16), (3, 23, 11, 8)])
def test_prolonged_basis_matches_oracle(lib, dim, n, nc, r):
    case(f"prolong basis dim={dim} n={n} nc={nc} r={r}")
    Zc = _coarse_modes(dim, nc, r)
    s = lib.Solver(precision=lib.FP64)
    Zg = s.prolong_basis(Zc, dim, n, nc).cpu().numpy()
    Zo, keep = coarse_basis(Zc, n, nc, dim)
    print(f"   kept {Zg.shape[1]} (oracle {keep.size})", flush=True)
    assert Zg.shape == Zo.shape
    assert np.abs(Zg.T @ Zg - np.eye(Zg.shape[1])).max() <= 1e-13
    d = np.abs(np.sum(Zg * Zo, axis=0))
    assert np.abs(d - 1.0).max() <= 1e-10
    assert np.linalg.norm(Zg - Zo * np.sign(np.sum(Zg * Zo, axis=0)), axis=0).max() <= 1e-10
    s.close()


def test_prolong_drops_dependent_column(lib):
    case("prolong basis drops a dependent coarse column")
    nc, n = 15, 31
    Zc = gen.sine_modes_2d(nc, 4)[0]
    Zc = np.column_stack([Zc[:, :2], Zc[:, 0] - 3 * Zc[:, 1], Zc[:, 2:]])
    s = lib.Solver(precision=lib.FP64)
    Zg = s.prolong_basis(Zc, 2, n, nc).cpu().numpy()
    Zo, keep = coarse_basis(Zc, n, nc, 2)
    assert list(keep) == [0, 1, 3, 4] and Zg.shape[1] == 4
    assert np.linalg.norm(Zg - Zo @ (Zo.T @ Zg)) <= 1e-10
    with pytest.raises(lib.Adef2Error):
        s.prolong_basis(Zc, 2, 10, 15)          # coarse grid finer than the fine grid
    s.close()


def test_solve_with_prolonged_basis(lib):
    n, nc, r = 63, 31, 16
    case(f"2d_sym {n}^2 solved with {r} modes prolonged from {nc}^2")
    w = gen.ocp_2d("2d_sym", n=n, B=3)
    spec = ("factored", w.op.A, w.op.alpha, w.op.shift)
    Zc = gen.sine_modes_2d(nc, r)[0]
    Zo, _ = coarse_basis(Zc, n, nc, 2)
    masks, bs, refs = [], [], []
    for m in range(3):
        _, act, _, _ = active_set(spec, w.y_d[m], w.psi[m], tau=w.tau)
        b = coupled_rhs(spec, w.y_d[m], w.psi[m], act)
        masks.append(act)
        bs.append(b)
        refs.append(oracle.solve_instance(spec, Zo, act, b, 1e-10))
    s = lib.Solver(precision=lib.FP64)
    Zg = s.prolong_basis(Zc, 2, n, nc).cpu().numpy()
    s.set_reference_factored(w.op.A, w.op.alpha, w.op.shift, Zg)
    out = s.solve_batched(np.stack(masks), np.stack(bs), 1e-10)
    for m in range(3):
        print(f"   m={m} iters={out['iters'][m]} (oracle {refs[m].iters}) status={out['status'][m]}",
              flush=True)
        assert out["status"][m] == 0
        assert abs(int(out["iters"][m]) - refs[m].iters) <= max(2, 0.01 * refs[m].iters)
    s.close()


def test_coarse_pipeline_on_convection_diffusion(lib):
    """The offline builders end to end on the GPU for the upwind
    convection-diffusion operator: the 40 smallest eigenpairs on the 127^2
    grid (block inverse iteration, relative residual 1e-6), the lowest 32
    prolonged to 255^2 (c = 2), then deflated FP64 solves of four family
    instances against the same solves with the fine-grid modes (shift-invert
    Lanczos in the input generator) and without deflation.  The prolonged
    basis must deflate nearly as well as the fine modes (at most 1.5x their
    iterations) and far better than none."""
    nc, n, k = 127, 255, 32
    case(f"coarse {nc}^2 eigensolve -> prolong to {n}^2 -> deflated solves")
    opc, _ = gen.c2_operator(nc)
    s = lib.Solver(precision=lib.FP64)
    s.set_reference_factored(opc.A, opc.alpha, opc.shift, None)
    X0 = np.random.default_rng(21).standard_normal((opc.N, 40))
    eig = s.reference_eigs(X0, max_iter=200, tol=1e-6, inner_tol=1e-10)
    print(f"   coarse eigensolve: {eig['iters']} steps, status {eig['status']}, "
          f"resid max {eig['resid'][:k].max():.1e}", flush=True)
    assert eig["status"] == 0
    Zc = eig["Z"][:, :k].cpu().numpy()
    Zf = s.prolong_basis(Zc, 2, n, nc).cpu().numpy()
    s.close()
    assert Zf.shape[1] == k
    w = gen.c2_workload(n=n, k=k, B=4)
    op = w.op
    masks = np.stack([i.mask for i in w.instances])
    bs = np.stack([i.b for i in w.instances])
    its = {}
    for name, Z in (("prolonged", Zf), ("fine", w.Z), ("cold", None)):
        t = lib.Solver(precision=lib.FP64)
        t.set_reference_factored(op.A, op.alpha, op.shift, Z)
        out = t.solve_batched(masks, bs, 1e-10)
        t.close()
        assert np.all(out["status"] == 0)
        its[name] = np.asarray(out["iters"])
        print(f"   {name:9s} iterations {its[name].tolist()}", flush=True)
    assert np.all(its["prolonged"] <= 1.5 * its["fine"])
    assert np.all(its["prolonged"] < 0.8 * its["cold"])
