"""Pins of the learned-enrichment oracle (loss, gradient, POD, MLP, Adam)."""
import numpy as np
import scipy.sparse as sp
import pytest
import torch

import gen
import oracle
from oracle import learned as L


@pytest.fixture(scope="module")
def sample():
    w = gen.c1_workload(n=15, k=6, seeds=(1,))
    S = w.op.S()
    inst = w.instances[0]
    I, _, nI = oracle.compact(inst.mask)
    S_II, _ = oracle.restrict(S, I)
    b = inst.b[I]
    xs = oracle.exact_solution(S_II, b)
    rng = np.random.default_rng(0)
    Phi = np.linalg.qr(rng.standard_normal((S.shape[0], 10)))[0]
    return S_II, w.Z[I, :], Phi[I, :], b, xs


def test_pod_matches_method_of_snapshots():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((200, 12)) @ np.diag(np.logspace(0, -3, 12)) @ rng.standard_normal((12, 30))
    Phi, s = L.pod_modes(X, 6)
    Xc = X - X.mean(axis=1, keepdims=True)
    lam, V = np.linalg.eigh(Xc.T @ Xc)
    lam, V = lam[::-1][:6], V[:, ::-1][:, :6]
    np.testing.assert_allclose(s, np.sqrt(lam), rtol=1e-9)
    U2 = Xc @ V / np.sqrt(lam)
    np.testing.assert_allclose(np.abs(Phi.T @ U2), np.eye(6), atol=1e-8)


def test_pod_recovers_a_prescribed_spectrum():
    """Closed form: the centred snapshot matrix is U diag(sigma) V^T, so the
    POD returns sigma and +-U (mean removal must be exact: V^T 1 = 0)."""
    sigma = 5.0 * 0.9 ** np.arange(40)
    X, U = gen.pod_snapshots(300, 120, sigma, seed=4)
    Phi, s = L.pod_modes(X, 20)
    np.testing.assert_allclose(s, sigma[:20], rtol=1e-10)
    np.testing.assert_allclose(np.abs(np.sum(Phi * U[:, :20], axis=0)), np.ones(20), atol=1e-9)
    # sign convention: the largest-magnitude entry of every mode is positive
    assert np.all(Phi[np.argmax(np.abs(Phi), axis=0), np.arange(20)] > 0)


def test_loss_equals_energy_left_by_the_coarse_correction(sample):
    S_II, ZI, PI, b, xs = sample
    d = L.loss_data(S_II, ZI, PI, b, xs)
    C = np.random.default_rng(1).standard_normal((8, PI.shape[1]))
    U = np.column_stack([ZI, PI @ C.T])
    assert abs(L.loss(C, d) - L.coarse_energy_left(S_II, U, b, xs)) < 1e-9
    assert abs((1 - d.e0 / d.bx) - L.coarse_energy_left(S_II, ZI, b, xs)) < 1e-10


def test_loss_range_invariance_and_exact_capture(sample):
    S_II, ZI, PI, b, xs = sample
    d = L.loss_data(S_II, ZI, PI, b, xs)
    rng = np.random.default_rng(2)
    C = rng.standard_normal((8, PI.shape[1]))
    G = rng.standard_normal((8, 8)) + 3 * np.eye(8)
    l0 = L.loss(C, d)
    assert 0.0 <= l0 <= 1.0 - d.e0 / d.bx + 1e-12
    assert abs(L.loss(G @ C, d) - l0) < 1e-9
    # a basis vector equal to x* leaves no energy
    P2 = np.column_stack([xs, PI[:, 1:]])
    d2 = L.loss_data(S_II, ZI, P2, b, xs)
    e1 = np.zeros((1, P2.shape[1]))
    e1[0, 0] = 1.0
    assert abs(L.loss(e1, d2)) < 1e-9


@pytest.mark.parametrize("eps", [0.0, 1e-6])
def test_loss_gradient_central_differences(sample, eps):
    S_II, ZI, PI, b, xs = sample
    d = L.loss_data(S_II, ZI, PI, b, xs)
    C = np.random.default_rng(4).standard_normal((8, PI.shape[1]))
    G = L.loss_grad(C, d, eps)
    Gfd = np.zeros_like(C)
    h = 1e-6
    for i in range(C.shape[0]):
        for j in range(C.shape[1]):
            Cp, Cm = C.copy(), C.copy()
            Cp[i, j] += h
            Cm[i, j] -= h
            Gfd[i, j] = (L.loss(Cp, d, eps) - L.loss(Cm, d, eps)) / (2 * h)
    assert np.linalg.norm(G - Gfd) <= 1e-6 * np.linalg.norm(G)


# ---------------------------------------------------------------------------
# deflated-spectrum objective
# ---------------------------------------------------------------------------
def test_spectral_data_closed_form_on_sine_modes():
    """Laplacian (diagonal 4) with exact sine eigenmodes: the candidates are
    already S-orthogonal to the reference modes, so H = diag(lambda) of the
    candidate modes and N = 4 I; the best 8-dimensional enrichment reaches
    the 8 smallest of those eigenvalues over 4 (Ky Fan)."""
    import scipy.linalg as sla
    n, k, p = 15, 6, 14
    S = gen.laplacian_2d(n)
    Zall, _, lam = gen.sine_modes_2d(n, k + p)
    Z, Phi = Zall[:, :k], Zall[:, k:]
    d = L.spectral_data(S, Z, Phi)
    np.testing.assert_allclose(d.H, np.diag(lam[k:]), atol=1e-12)
    np.testing.assert_allclose(d.N, 4.0 * np.eye(p), atol=1e-12)
    w, V = sla.eigh(d.H, d.N)
    C = V[:, :8].T
    np.testing.assert_allclose(np.exp(L.spectral_loss(C, d)), np.sort(lam[k:])[:8].sum() / 4.0, rtol=1e-12)


def test_deflated_candidates_are_s_orthogonal_and_span_the_same_space():
    rng = np.random.default_rng(5)
    n = 120
    T = gen._second_diff(n) + sp.diags(rng.uniform(0.1, 1.0, n))
    Z = rng.standard_normal((n, 5))
    Phi = rng.standard_normal((n, 7))
    P = L.deflated_candidates(T, Z, Phi)
    assert np.abs(Z.T @ (T @ P)).max() <= 1e-10 * np.abs(Z.T @ (T @ Phi)).max()
    B1 = np.linalg.qr(np.column_stack([Z, P]))[0]
    B2 = np.linalg.qr(np.column_stack([Z, Phi]))[0]
    np.testing.assert_allclose(np.linalg.svd(B1.T @ B2, compute_uv=False), np.ones(12), atol=1e-10)
    # H, N are the S- and D-weighted Grams of P~
    d = L.spectral_data(T, Z, Phi)
    np.testing.assert_allclose(d.H, P.T @ (T @ P), rtol=1e-12, atol=1e-12 * np.abs(d.H).max())
    np.testing.assert_allclose(d.N, P.T @ (T.diagonal()[:, None] * P), rtol=1e-12,
                               atol=1e-12 * np.abs(d.N).max())


def _spec_sample(seed=6):
    rng = np.random.default_rng(seed)
    p = 12
    A = rng.standard_normal((p, p))
    H = A @ A.T + 0.1 * np.eye(p)
    B = rng.standard_normal((p, p))
    N = B @ B.T + 0.5 * np.eye(p)
    return L.SpecData(H, N), rng.standard_normal((8, p))


def test_spectral_loss_invariance_and_lower_bound():
    import scipy.linalg as sla
    d, C = _spec_sample()
    A = np.random.default_rng(7).standard_normal((8, 8)) + 3.0 * np.eye(8)
    # a change of basis of the 8 vectors leaves their span, hence R, unchanged
    assert abs(L.spectral_loss(A @ C, d) - L.spectral_loss(C, d)) <= 1e-11
    w, V = sla.eigh(d.H, d.N)
    best = np.log(w[:8].sum())
    assert abs(L.spectral_loss(V[:, :8].T, d) - best) <= 1e-12
    rng = np.random.default_rng(8)
    for _ in range(20):
        assert L.spectral_loss(rng.standard_normal((8, 12)), d) >= best - 1e-12


@pytest.mark.parametrize("eps", [1e-6])
def test_spectral_grad_central_differences(eps):
    d, C = _spec_sample(9)
    G = L.spectral_grad(C, d)
    num = np.zeros_like(C)
    for i in range(C.shape[0]):
        for j in range(C.shape[1]):
            E = np.zeros_like(C)
            E[i, j] = eps
            num[i, j] = (L.spectral_loss(C + E, d) - L.spectral_loss(C - E, d)) / (2 * eps)
    np.testing.assert_allclose(G, num, rtol=1e-6, atol=1e-8 * np.abs(G).max())


def test_mlp_backward_central_differences():
    params = L.mlp_init(5)
    for k in params:
        params[k] = L.bf16_round(params[k]) if k.startswith("W") else params[k]
    theta = np.random.default_rng(6).uniform(size=(3, 4))
    dout = np.random.default_rng(7).standard_normal((3, 512))
    out, cache = L.mlp_forward(params, theta)
    g = L.mlp_backward(cache, dout)
    # finite differences on the FP64 function of the (already bf16) weights
    f = lambda P: float(np.sum(L.mlp_forward(P, theta)[0] * dout))  # noqa: E731
    rng = np.random.default_rng(8)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        for _ in range(4):
            idx = tuple(rng.integers(0, n) for n in params[k].shape)
            P1 = {kk: v.astype(np.float64) for kk, v in params.items()}
            P2 = {kk: v.astype(np.float64) for kk, v in params.items()}
            h = 1e-3
            P1[k][idx] += h
            P2[k][idx] -= h
            fd = (_fwd64(P1, theta, dout) - _fwd64(P2, theta, dout)) / (2 * h)
            assert abs(fd - g[k][idx]) <= 1e-6 * max(1.0, abs(fd))


def _fwd64(P, theta, dout):
    a1 = theta @ P["W1"].T + P["b1"]
    h1 = L.gelu(a1)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = L.gelu(a2)
    return float(np.sum((h2 @ P["W3"].T + P["b3"]) * dout))


def test_mlp_forward_matches_torch():
    params = L.mlp_init(9)
    theta = np.random.default_rng(10).uniform(size=(5, 4))
    out, _ = L.mlp_forward(params, theta)
    x = torch.tensor(theta, dtype=torch.float64)
    for l in (1, 2, 3):
        Wt = torch.tensor(params[f"W{l}"]).to(torch.bfloat16).to(torch.float64)
        x = x @ Wt.T + torch.tensor(params[f"b{l}"], dtype=torch.float64)
        if l < 3:
            x = torch.nn.functional.gelu(x)
    np.testing.assert_allclose(out, x.numpy(), rtol=1e-12, atol=1e-12)


def test_bf16_round_matches_torch():
    a = np.random.default_rng(11).standard_normal(10000).astype(np.float32) * 10.0 ** np.random.default_rng(12).integers(-5, 5, 10000)
    ref = torch.tensor(a).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(L.bf16_round(a), ref)


def test_adam_matches_torch():
    params = {"W": np.random.default_rng(13).standard_normal((4, 3)).astype(np.float32)}
    tp = torch.nn.Parameter(torch.tensor(params["W"].astype(np.float64)))
    opt = torch.optim.Adam([tp], lr=1e-2)
    state = {}
    for it in range(5):
        g = np.random.default_rng(20 + it).standard_normal((4, 3))
        L.adam_step(params, {"W": g}, state, lr=1e-2)
        tp.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(params["W"], tp.detach().numpy(), rtol=2e-6, atol=1e-6)
