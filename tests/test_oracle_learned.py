"""Pins of the learned-enrichment oracle (loss, gradient, POD, MLP, Adam)."""
import numpy as np
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
