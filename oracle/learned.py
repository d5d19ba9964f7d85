"""FP64 oracle of the learned coarse-space enrichment (test infrastructure only).

The paper enriches the restricted reference modes with POD modes of earlier
solutions (Sec. "Online POD enrichment": mean-centred snapshot matrix, its
SVD) merged under a conditioning guard (Alg. 2, Sec. "Conditioning-based safe
merge").  The learned variant built here replaces the fixed choice of POD
modes by 8 combinations V = Phi C^T of the first p POD modes, with C (8 x p)
produced from the problem parameters theta by a small MLP.  The paper has no
learned component; the objective below is a reading of ours: the fraction of the solution's energy norm that the A-DEF2 coarse
correction with the basis [Z_I, V_I] leaves unresolved.

Only the tests and the smoke check use this module.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "pod_modes", "LossData", "loss_data", "loss", "loss_grad", "coarse_energy_left",
    "SpecData", "deflated_candidates", "spectral_data", "spectral_loss", "spectral_grad",
    "bf16_round", "gelu", "gelu_grad", "mlp_init", "mlp_forward", "mlp_backward",
    "adam_step", "DIMS",
]

DIMS = (4, 128, 128, 512)      # theta -> h1 -> h2 -> C (8 x 64)


# ---------------------------------------------------------------------------
# POD (Sec. "Online POD enrichment")
# ---------------------------------------------------------------------------
def pod_modes(X: np.ndarray, p: int):
    """First p POD modes of the snapshot columns of X (N x M).

    Snapshots are mean-centred (S = [y_j - mean]) and the left singular
    vectors of the centred matrix, ordered by decreasing singular value, are
    returned with the singular values.  Signs: largest-magnitude entry > 0.
    """
    Xc = X - X.mean(axis=1, keepdims=True)
    U, s, _ = np.linalg.svd(Xc, full_matrices=False)
    U = U[:, :p].copy()
    for j in range(U.shape[1]):
        if U[np.argmax(np.abs(U[:, j])), j] < 0:
            U[:, j] = -U[:, j]
    return U, s[:p]


# ---------------------------------------------------------------------------
# energy-capture loss of a learned enrichment
# ---------------------------------------------------------------------------
class LossData:
    """Per-sample quantities of the loss: H (p x p), g (p), e0 = b_Z^T G_ZZ^-1 b_Z,
    bx = b^T x*."""

    def __init__(self, H, g, e0, bx):
        self.H, self.g, self.e0, self.bx = H, g, e0, bx


def loss_data(S_II, Z_I: np.ndarray, Phi_I: np.ndarray, b: np.ndarray, xstar: np.ndarray) -> LossData:
    """H = G_PP - G_PZ G_ZZ^-1 G_ZP and g = b_P - G_PZ G_ZZ^-1 b_Z, with
    G_XY = X^T M_II Y on the restricted (not re-orthonormalised) columns."""
    SZ = np.asarray(S_II @ Z_I)
    SP = np.asarray(S_II @ Phi_I)
    Gzz = Z_I.T @ SZ
    Gzp = Z_I.T @ SP
    Gpp = Phi_I.T @ SP
    bz = Z_I.T @ b
    bp = Phi_I.T @ b
    Gzz = 0.5 * (Gzz + Gzz.T)
    A = np.linalg.solve(Gzz, np.column_stack([Gzp, bz]))
    H = Gpp - Gzp.T @ A[:, :-1]
    H = 0.5 * (H + H.T)
    g = bp - Gzp.T @ A[:, -1]
    e0 = float(bz @ A[:, -1])
    return LossData(H, g, e0, float(b @ xstar))


def loss(C: np.ndarray, d: LossData, eps: float = 0.0) -> float:
    """L(C) = 1 - (e0 + s^T (C H C^T + eps I)^-1 s) / b^T x*,  s = C g."""
    s = C @ d.g
    T = C @ d.H @ C.T + eps * np.eye(C.shape[0])
    return 1.0 - (d.e0 + float(s @ np.linalg.solve(T, s))) / d.bx


def loss_grad(C: np.ndarray, d: LossData, eps: float = 0.0) -> np.ndarray:
    """dL/dC = -(2 u g^T - 2 u u^T C H) / b^T x*,  u = T^-1 s."""
    s = C @ d.g
    T = C @ d.H @ C.T + eps * np.eye(C.shape[0])
    u = np.linalg.solve(T, s)
    return -(2.0 * np.outer(u, d.g) - 2.0 * np.outer(u, u) @ C @ d.H) / d.bx


# ---------------------------------------------------------------------------
# deflated-spectrum loss of a learned enrichment (a reading of ours, like the
# energy loss): CG's iteration count is governed by the spectrum of the
# Jacobi-preconditioned operator left after deflation, so the enrichment
# should hold its slowest modes.  With V = P~ C^T (P~: the candidates made
# S_II-orthogonal to the reference modes), the sum of the Ritz values of
# D^-1 S_II on span(V) is R(C) = tr((C N C^T)^-1 C H C^T),
# H = P~^T S_II P~, N = P~^T D P~, D = diag(S_II); the loss is log R.
# ---------------------------------------------------------------------------
class SpecData:
    """Per-sample H = P~^T S_II P~ and N = P~^T D P~ (p x p)."""

    def __init__(self, H, N):
        self.H, self.N = H, N


def deflated_candidates(S_II, Z_I: np.ndarray, Phi_I: np.ndarray) -> np.ndarray:
    """P~ = Phi_I - Z_I (Z_I^T S_II Z_I)^-1 Z_I^T S_II Phi_I: the candidates
    with their S_II-projection onto span(Z_I) removed (A-DEF2's coarse space
    is S_II-orthogonal to what the iteration sees)."""
    SZ = np.asarray(S_II @ Z_I)
    Gzz = Z_I.T @ SZ
    Gzz = 0.5 * (Gzz + Gzz.T)
    return Phi_I - Z_I @ np.linalg.solve(Gzz, SZ.T @ Phi_I)


def spectral_data(S_II, Z_I: np.ndarray, Phi_I: np.ndarray) -> SpecData:
    """H and N of the deflated-spectrum loss, from P~ written out."""
    P = deflated_candidates(S_II, Z_I, Phi_I)
    d = np.asarray(S_II.diagonal()).ravel()
    H = P.T @ np.asarray(S_II @ P)
    N = P.T @ (d[:, None] * P)
    return SpecData(0.5 * (H + H.T), 0.5 * (N + N.T))


def spectral_loss(C: np.ndarray, d: SpecData) -> float:
    """L(C) = log tr((C N C^T)^-1 C H C^T)."""
    T = C @ d.H @ C.T
    U = C @ d.N @ C.T
    return float(np.log(np.trace(np.linalg.solve(U, T))))


def spectral_grad(C: np.ndarray, d: SpecData) -> np.ndarray:
    """dL/dC = 2 (U^-1 C H - U^-1 T U^-1 C N) / R, T = C H C^T, U = C N C^T,
    R = tr(U^-1 T)."""
    T = C @ d.H @ C.T
    U = C @ d.N @ C.T
    X = np.linalg.inv(U)
    R = float(np.trace(X @ T))
    return 2.0 * (X @ C @ d.H - X @ T @ X @ C @ d.N) / R


def coarse_energy_left(S_II, U: np.ndarray, b: np.ndarray, xstar: np.ndarray) -> float:
    """||x* - x_c||_M^2 / ||x*||_M^2 for the coarse correction
    x_c = U (U^T M U)^-1 U^T b  (Sec. A-DEF2: Q b, the deflated initial guess)."""
    SU = np.asarray(S_II @ U)
    xc = U @ np.linalg.solve(U.T @ SU, U.T @ b)
    e = xstar - xc
    return float(e @ np.asarray(S_II @ e)) / float(xstar @ np.asarray(S_II @ xstar))


# ---------------------------------------------------------------------------
# MLP theta -> C (4 -> 128 -> 128 -> 512, exact erf GELU)
# ---------------------------------------------------------------------------
def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest bfloat16 (ties to even), kept as FP32."""
    f = np.asarray(a, dtype=np.float32).copy()
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def gelu(x):
    return 0.5 * x * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0))) + \
        x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def mlp_init(seed: int = 0, dims=DIMS):
    """He-uniform weights (FP32 master copies), zero biases."""
    rng = np.random.default_rng(seed)
    params = {}
    for l in range(3):
        fan_in = dims[l]
        lim = math.sqrt(6.0 / fan_in) * (0.1 if l == 2 else 1.0)
        params[f"W{l + 1}"] = rng.uniform(-lim, lim, size=(dims[l + 1], dims[l])).astype(np.float32)
        params[f"b{l + 1}"] = np.zeros(dims[l + 1], dtype=np.float32)
    return params


def mlp_forward(params, theta: np.ndarray):
    """theta (B x 4) -> out (B x 512), in FP64 with BF16-rounded weights.

    Returns (out, cache)."""
    W = [bf16_round(params[f"W{l}"]).astype(np.float64) for l in (1, 2, 3)]
    b = [params[f"b{l}"].astype(np.float64) for l in (1, 2, 3)]
    x0 = np.asarray(theta, dtype=np.float64)
    a1 = x0 @ W[0].T + b[0]
    h1 = gelu(a1)
    a2 = h1 @ W[1].T + b[1]
    h2 = gelu(a2)
    out = h2 @ W[2].T + b[2]
    return out, (x0, a1, h1, a2, h2, W)


def mlp_backward(cache, dout: np.ndarray):
    """Gradients of sum(out * dout) w.r.t. W1..W3, b1..b3 (FP64)."""
    x0, a1, h1, a2, h2, W = cache
    g = {}
    g["W3"] = dout.T @ h2
    g["b3"] = dout.sum(axis=0)
    dh2 = dout @ W[2]
    da2 = dh2 * gelu_grad(a2)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ W[1]
    da1 = dh1 * gelu_grad(a1)
    g["W1"] = da1.T @ x0
    g["b1"] = da1.sum(axis=0)
    return g


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) of the FP32 master parameters."""
    t = state.get("t", 0) + 1
    state["t"] = t
    for k in params:
        m = state.setdefault("m" + k, np.zeros_like(params[k], dtype=np.float64))
        v = state.setdefault("v" + k, np.zeros_like(params[k], dtype=np.float64))
        m[:] = b1 * m + (1 - b1) * grads[k]
        v[:] = b2 * v + (1 - b2) * grads[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        params[k] = (params[k] - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)
    return params
