"""Seeded synthetic inputs for the restricted Schur-complement solves.

This module builds *inputs* only: grids, the full-domain SPD operator S as a
CSR matrix, the offline reference modes Z, active-set masks, right-hand sides
and the problem parameters of each instance.  It contains none of the solver's
arithmetic (no restriction, no coarse space, no Krylov iteration); both the
GPU library and the CPU oracle consume the arrays produced here.

Every workload is synthetic and follows the shapes of the paper's benchmark
families (unit square / cube, homogeneous Dirichlet conditions imposed by
keeping only interior nodes, h = 1/(n+1), lexicographic ordering with x
fastest; finite-difference discretisation, Appendix "Finite difference
discretization").  The Schur complement is the mass-weighted analogue of
M = alpha A^T A + I (Sec. "Reduced inactive set system", eq. schur) that the
paper allows for finite-element-style scalings:

    S = a * K^T M_L^{-1} K + c * M_L,   M_L = h^d I (lumped mass),

with K the (FE-scaled) state operator; a and c per workload.

Where the paper leaves a detail open, the reading taken is stated next to
the generator that uses it.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = [
    "Operator", "Instance", "Workload",
    "laplacian_2d", "upwind_2d", "diffusion_2d", "diffusion_3d",
    "sinusoid_field", "gaussian_field_2d", "inclusion_field_3d",
    "mask_top_fraction", "gaussian_bump", "sine_modes_2d",
    "c1_workload", "c2_workload", "c2_family_instance", "c2_thetas", "mlp_params",
    "OCPWorkload", "ocp_2d_sym", "c3_workload", "c5_workload",
    "cache_dir",
]


# ----------------------------------------------------------------------------
# containers
# ----------------------------------------------------------------------------
@dataclass
class Operator:
    """Full-domain operator family  S(a, c) = a * B + c * I  on an n^d grid.

    ``B = alpha A^T A`` is the squared-stencil part, ``A`` the (FE-scaled) state
    operator and ``shift`` the default identity coefficient, i.e. the paper's
    M = alpha A^T A + I in its mass-weighted form; ``S`` is the default member
    (a = 1), assembled as CSR in FP64.
    """
    n: int
    dim: int
    B: sp.csr_matrix | None      # None: assembled on first use as alpha A^T A
    shift: float
    name: str
    A: sp.csr_matrix | None = None
    alpha: float = 1.0

    @property
    def N(self) -> int:
        return self.n ** self.dim

    @property
    def h(self) -> float:
        return 1.0 / (self.n + 1)

    def S(self, a: float = 1.0, c: float | None = None) -> sp.csr_matrix:
        c = self.shift if c is None else c
        if self.B is None:
            self.B = canonical_csr(self.alpha * (self.A.T @ self.A))
        M = (a * self.B + c * sp.identity(self.N, format="csr")).tocsr()
        return canonical_csr(M)


@dataclass
class Instance:
    mask: np.ndarray          # uint8[N], 1 = active, 0 = inactive
    b: np.ndarray             # f64[N], global order (b[A] ignored by the solver)
    a: float = 1.0            # operator scale: S = a*B + c*I
    c: float | None = None
    theta: np.ndarray | None = None   # problem parameters (learned enrichment)


@dataclass
class Workload:
    name: str
    op: Operator
    Z: np.ndarray             # f64[N, k], column-major (Fortran order)
    instances: list[Instance]
    tol: float
    meta: dict = field(default_factory=dict)


def canonical_csr(M) -> sp.csr_matrix:
    """CSR with sorted column indices, int64 row pointers, int32 columns."""
    M = sp.csr_matrix(M)
    M.sum_duplicates()
    M.sort_indices()
    M.eliminate_zeros()
    out = sp.csr_matrix((M.data.astype(np.float64), M.indices.astype(np.int32),
                         M.indptr), shape=M.shape)
    # scipy narrows index arrays on construction; pin the documented widths
    out.indptr = np.ascontiguousarray(M.indptr, dtype=np.int64)
    out.indices = np.ascontiguousarray(M.indices, dtype=np.int32)
    out.has_sorted_indices = True
    return out


# ----------------------------------------------------------------------------
# grids and stencils (Appendix "Finite difference discretization")
# ----------------------------------------------------------------------------
def _second_diff(n: int) -> sp.csr_matrix:
    e = np.ones(n)
    return sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1], format="csr")


def laplacian_2d(n: int) -> sp.csr_matrix:
    """Unscaled 5-point stencil (4, -1) on the n x n interior grid.

    Equals h^2 times the FD Laplacian of eq. (fd_lap); in 2D this is also the
    stiffness scaling of bilinear finite elements, so M_L = h^2 I pairs with it.
    """
    T = _second_diff(n)
    I = sp.identity(n, format="csr")
    return (sp.kron(I, T) + sp.kron(T, I)).tocsr()


def upwind_2d(n: int, beta) -> sp.csr_matrix:
    """First-order upwind convection  h * (beta . grad_h y), FE-scaled (x h^2).

    For beta_x > 0 the x-difference is (y_i - y_{i-1}) / h, for beta_x < 0 it is
    (y_{i+1} - y_i) / h; likewise in y.  Rows of boundary nodes drop the
    neighbour outside the grid (homogeneous Dirichlet).
    """
    h = 1.0 / (n + 1)
    e = np.ones(n)
    I = sp.identity(n, format="csr")
    bx, by = float(beta[0]), float(beta[1])

    def one_sided(b):
        if b >= 0:
            return b * sp.diags([-e[:-1], e], [-1, 0], format="csr")
        return -b * sp.diags([e, -e[:-1]], [0, 1], format="csr")

    Cx = sp.kron(I, one_sided(bx))
    Cy = sp.kron(one_sided(by), I)
    return (h * (Cx + Cy)).tocsr()


def _harmonic(a, b):
    return 2.0 * a * b / (a + b)


def diffusion_2d(kappa: np.ndarray) -> sp.csr_matrix:
    """-div(kappa grad y) with harmonic face averages (eq. harmonic), unscaled.

    ``kappa`` is an n x n nodal field indexed [iy, ix].  Faces to the Dirichlet
    boundary use the node's own kappa.
    """
    n = kappa.shape[0]
    N = n * n
    idx = np.arange(N).reshape(n, n)
    rows, cols, vals = [], [], []
    diag = np.zeros((n, n))
    # x faces
    kx = _harmonic(kappa[:, :-1], kappa[:, 1:])
    diag[:, :-1] += kx
    diag[:, 1:] += kx
    rows += [idx[:, :-1].ravel(), idx[:, 1:].ravel()]
    cols += [idx[:, 1:].ravel(), idx[:, :-1].ravel()]
    vals += [-kx.ravel(), -kx.ravel()]
    # y faces
    ky = _harmonic(kappa[:-1, :], kappa[1:, :])
    diag[:-1, :] += ky
    diag[1:, :] += ky
    rows += [idx[:-1, :].ravel(), idx[1:, :].ravel()]
    cols += [idx[1:, :].ravel(), idx[:-1, :].ravel()]
    vals += [-ky.ravel(), -ky.ravel()]
    # boundary faces
    diag[:, 0] += kappa[:, 0]
    diag[:, -1] += kappa[:, -1]
    diag[0, :] += kappa[0, :]
    diag[-1, :] += kappa[-1, :]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return K.tocsr()


def diffusion_3d(kappa: np.ndarray) -> sp.csr_matrix:
    """h * (7-point flux form of -div(kappa grad y)), harmonic faces, 3D.

    ``kappa`` is an n^3 nodal field indexed [iz, iy, ix].  The factor h is the
    finite-element stiffness scaling in 3D (h^{d-2}).
    """
    n = kappa.shape[0]
    h = 1.0 / (n + 1)
    N = n ** 3
    idx = np.arange(N).reshape(n, n, n)
    rows, cols, vals = [], [], []
    diag = np.zeros((n, n, n))
    for ax in range(3):
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[ax] = slice(None, -1)
        sl_hi[ax] = slice(1, None)
        kf = _harmonic(kappa[tuple(sl_lo)], kappa[tuple(sl_hi)])
        diag[tuple(sl_lo)] += kf
        diag[tuple(sl_hi)] += kf
        rows += [idx[tuple(sl_lo)].ravel(), idx[tuple(sl_hi)].ravel()]
        cols += [idx[tuple(sl_hi)].ravel(), idx[tuple(sl_lo)].ravel()]
        vals += [-kf.ravel(), -kf.ravel()]
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[ax] = 0
        last[ax] = -1
        diag[tuple(first)] += kappa[tuple(first)]
        diag[tuple(last)] += kappa[tuple(last)]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    K = sp.coo_matrix((h * np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return K.tocsr()


# ----------------------------------------------------------------------------
# seeded fields, masks and right-hand sides
# ----------------------------------------------------------------------------
def _coords(n: int, dim: int):
    h = 1.0 / (n + 1)
    x = h * np.arange(1, n + 1)
    if dim == 2:
        Y, X = np.meshgrid(x, x, indexing="ij")
        return X.ravel(), Y.ravel()
    Zc, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return X.ravel(), Y.ravel(), Zc.ravel()


def sinusoid_field(n: int, seed: int, dim: int = 2, terms: int = 6,
                   phase_shift: float = 0.0) -> np.ndarray:
    """Sum of ``terms`` cosines with integer frequencies in 1..4 and U[0,2pi) phases."""
    rng = np.random.default_rng(seed)
    xs = _coords(n, dim)
    f = np.zeros(n ** dim)
    for _ in range(terms):
        freq = rng.integers(1, 5, size=dim)
        phi = rng.uniform(0.0, 2.0 * np.pi)
        arg = sum(2.0 * np.pi * freq[d] * xs[d] for d in range(dim))
        f += np.cos(arg + phi + phase_shift)
    return f


def gaussian_field_2d(n: int, seed: int, ell: float = 0.1) -> np.ndarray:
    """Unit-variance Gaussian random field with squared-exponential covariance.

    White noise on a 2x padded periodic grid is smoothed by a Gaussian kernel of
    standard deviation ell / sqrt(2) via FFT, cropped and rescaled to unit
    sample variance.  Returned as an n x n array [iy, ix].
    """
    rng = np.random.default_rng(seed)
    m = 2 * (n + 1)
    h = 1.0 / (n + 1)
    w = rng.standard_normal((m, m))
    k = np.fft.fftfreq(m, d=h) * 2.0 * np.pi
    KY, KX = np.meshgrid(k, k, indexing="ij")
    s = ell / math.sqrt(2.0)
    filt = np.exp(-0.5 * s * s * (KX ** 2 + KY ** 2))
    g = np.real(np.fft.ifft2(np.fft.fft2(w) * filt))[:n, :n]
    g = (g - g.mean()) / g.std()
    return g


def inclusion_field_3d(n: int, seed: int, kappa_in: float = 1000.0, radius: float = 0.08,
                       volume: float = 0.15) -> np.ndarray:
    """Background 1 with spherical inclusions of ``kappa_in`` until ``volume`` is reached."""
    rng = np.random.default_rng(seed)
    X, Y, Zc = (a.reshape(n, n, n) for a in _coords(n, 3))
    kap = np.ones((n, n, n))
    inside = np.zeros((n, n, n), dtype=bool)
    while inside.mean() < volume:
        c = rng.uniform(0.0, 1.0, size=3)
        inside |= (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Zc - c[2]) ** 2 <= radius ** 2
    kap[inside] = kappa_in
    return kap


def mask_top_fraction(field_values: np.ndarray, rho: float) -> np.ndarray:
    """Active where the field is among the floor(rho*N) largest values.

    Ties are broken by index (lower index first among equal values), so exactly
    floor(rho*N) nodes are active.
    """
    N = field_values.size
    n_act = int(math.floor(rho * N))
    order = np.lexsort((np.arange(N), -field_values))
    mask = np.zeros(N, dtype=np.uint8)
    mask[order[:n_act]] = 1
    return mask


def gaussian_bump(n: int, centre, width: float = 0.05, dim: int = 2) -> np.ndarray:
    """h^d * exp(-|x - c|^2 / (2 width^2)) on the interior nodes (lumped-mass rhs)."""
    h = 1.0 / (n + 1)
    xs = _coords(n, dim)
    r2 = sum((xs[d] - centre[d]) ** 2 for d in range(dim))
    return (h ** dim) * np.exp(-r2 / (2.0 * width * width))


# ----------------------------------------------------------------------------
# reference modes (offline input; the paper's Sec. "Analytical eigenmodes")
# ----------------------------------------------------------------------------
def sine_modes_2d(n: int, k: int):
    """The k lowest discrete sine modes of a squared 2D Laplacian-based operator.

    phi_{ij}[a, b] = (2/(n+1)) sin(i pi a/(n+1)) sin(j pi b/(n+1)), a, b = 1..n,
    ordered by sigma_i + sigma_j with sigma_q = 4 sin^2(q pi / (2(n+1))), ties
    broken lexicographically by (i, j).  Column (i, j) varies with x through i.
    Returns (Z [N x k] Fortran-ordered, [(i, j)] pairs, sigma sums).
    """
    q = np.arange(1, n + 1)
    sig = 4.0 * np.sin(q * np.pi / (2.0 * (n + 1))) ** 2
    # candidates: only small i + j can be among the k lowest
    m = min(n, k + 1)
    cand = [(sig[i - 1] + sig[j - 1], i, j) for i in range(1, m + 1) for j in range(1, m + 1)]
    cand.sort()
    chosen = cand[:k]
    a = np.arange(1, n + 1)
    Z = np.empty((n * n, k), order="F")
    for col, (_, i, j) in enumerate(chosen):
        sx = math.sqrt(2.0 / (n + 1)) * np.sin(i * np.pi * a / (n + 1))
        sy = math.sqrt(2.0 / (n + 1)) * np.sin(j * np.pi * a / (n + 1))
        Z[:, col] = np.outer(sy, sx).ravel()
    return Z, [(i, j) for _, i, j in chosen], np.array([s for s, _, _ in chosen])


def cache_dir() -> str:
    d = os.environ.get("ADEF2_CACHE", os.path.join(os.path.dirname(os.path.dirname(
        os.path.abspath(__file__))), "_cache"))
    os.makedirs(d, exist_ok=True)
    return d


def _cached(name: str, fn):
    path = os.path.join(cache_dir(), name + ".npy")
    if os.path.exists(path):
        return np.load(path)
    arr = fn()
    tmp = path + ".tmp.npy"
    np.save(tmp, arr)
    os.replace(tmp, path)
    return arr


def _low_right_singular(K: sp.spmatrix, k: int, seed: int = 0) -> np.ndarray:
    """k lowest eigenvectors of K^T K by shift-invert Lanczos (ARPACK) on (K^T K)^{-1}.

    (K^T K)^{-1} v is applied as K^{-1} K^{-T} v with one sparse LU of K, so the
    squared operator is never factorised.  This is the paper's offline
    eigensolver (shift-invert Lanczos, Sec. "Core idea"); S = a K^T K / h^2 + c I
    shares these eigenvectors for every a > 0 and c.
    """
    N = K.shape[0]
    lu = spla.splu(sp.csc_matrix(K))
    A = spla.LinearOperator((N, N), dtype=np.float64,
                            matvec=lambda v: lu.solve(lu.solve(np.asarray(v).ravel(), trans="T")))
    v0 = np.random.default_rng(seed).standard_normal(N)
    w, V = spla.eigsh(A, k=k, which="LM", tol=1e-13, v0=v0)
    order = np.argsort(-w)           # largest 1/lambda first = smallest lambda first
    V = V[:, order]
    # deterministic sign: largest-magnitude entry positive
    for j in range(k):
        if V[np.argmax(np.abs(V[:, j])), j] < 0:
            V[:, j] = -V[:, j]
    return np.asfortranarray(V)


def _low_symmetric(K: sp.spmatrix, k: int, seed: int = 0) -> np.ndarray:
    """k lowest eigenvectors of a symmetric K by shift-invert Lanczos (sigma = 0)."""
    N = K.shape[0]
    v0 = np.random.default_rng(seed).standard_normal(N)
    w, V = spla.eigsh(sp.csc_matrix(K), k=k, sigma=0.0, which="LM", tol=1e-13, v0=v0)
    order = np.argsort(w)
    V = V[:, order]
    for j in range(k):
        if V[np.argmax(np.abs(V[:, j])), j] < 0:
            V[:, j] = -V[:, j]
    return np.asfortranarray(V)


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
def c1_workload(n: int = 63, k: int = 16, seeds=(0,), active: float = 0.2) -> Workload:
    """Plain method, single instance: constant-coefficient 2D Laplacian-based S.

    S = 1e-2 K M_L^{-1} K + M_L with K the unscaled 5-point stencil, M_L = h^2 I;
    Z = k closed-form sine modes; mask = top ``active`` fraction of a seeded
    sinusoid field; b ~ N(0, 1) from the same seed.
    """
    h = 1.0 / (n + 1)
    K = canonical_csr(laplacian_2d(n))
    B = canonical_csr(1e-2 * (K @ K) / (h * h))
    op = Operator(n=n, dim=2, B=B, shift=h * h, name=f"lap2d_sq_{n}", A=K, alpha=1e-2 / (h * h))
    Z, pairs, sig = sine_modes_2d(n, k) if k > 0 else (np.zeros((n * n, 0), order="F"), [], np.zeros(0))
    insts = []
    for s in seeds:
        mask = mask_top_fraction(sinusoid_field(n, s), active)
        b = np.random.default_rng(s).standard_normal(n * n)
        insts.append(Instance(mask=mask, b=b))
    return Workload(name=f"c1_lap2d_n{n}_k{k}", op=op, Z=Z, instances=insts, tol=1e-8,
                    meta={"pairs": pairs, "sigma_sum": sig})


def c2_operator(n: int = 511, theta: float = math.pi / 6, peclet: float = 50.0):
    h = 1.0 / (n + 1)
    beta = peclet * np.array([math.cos(theta), math.sin(theta)])
    K = canonical_csr(laplacian_2d(n) + upwind_2d(n, beta))
    B = canonical_csr((K.T @ K) / (h * h))
    op = Operator(n=n, dim=2, B=B, shift=1e-2 * h * h, name=f"cd2d_upwind_{n}", A=K,
                  alpha=1.0 / (h * h))
    return op, K


def c2_family_instance(n: int, theta, field_seed: int = 100) -> Instance:
    """One member of the 4-parameter convection-diffusion family.

    theta in [0, 1]^4: active fraction 0.10 + 0.30 theta0 (top quantile of one
    fixed sinusoid field, seed 100, shifted in phase by 2 pi theta3), source
    centre (0.2 + 0.6 theta1, 0.2 + 0.6 theta2), Gaussian bump of width 0.05.
    """
    t = np.asarray(theta, dtype=np.float64)
    rho = 0.10 + 0.30 * t[0]
    f = sinusoid_field(n, field_seed, phase_shift=2.0 * np.pi * t[3])
    mask = mask_top_fraction(f, rho)
    b = gaussian_bump(n, (0.2 + 0.6 * t[1], 0.2 + 0.6 * t[2]))
    return Instance(mask=mask, b=b, theta=t.copy())


def c2_thetas(count: int, seed: int, spread_rho: bool = False) -> np.ndarray:
    th = np.random.default_rng(seed).uniform(0.0, 1.0, size=(count, 4))
    if spread_rho:
        th[:, 0] = np.arange(count) / max(count - 1, 1)
    return th


def c2_workload(n: int = 511, k: int = 32, B: int = 16, theta: float = math.pi / 6,
                peclet: float = 50.0, seed0: int = 200) -> Workload:
    """2D convection-diffusion, upwind K, S = K^T M_L^{-1} K + 1e-2 M_L.

    B instances of the 4-parameter family (c2_family_instance) with active
    fractions spread evenly over 10-40 % (theta0 = m/(B-1)) and the other
    parameters ~ U[0,1] (seed 200).  Z = k lowest eigenvectors of S.
    """
    op, K = c2_operator(n, theta, peclet)
    Z = _cached(f"c2_Z_n{n}_k{k}_t{theta:.6f}_pe{peclet:g}",
                lambda: _low_right_singular(K, k)) if k > 0 else np.zeros((op.N, 0), order="F")
    Z = np.asfortranarray(Z)
    insts = [c2_family_instance(n, th) for th in c2_thetas(B, seed0, spread_rho=True)]
    return Workload(name=f"c2_cd2d_n{n}_k{k}_B{B}", op=op, Z=Z, instances=insts, tol=1e-10,
                    meta={"theta": theta, "peclet": peclet})


# ---------------------------------------------------------------------------
# State-constrained optimal control, the 2D Laplacian suite (App. "2D
# Laplacian problems"): M = alpha L^T L + I with L = -Laplacian (5-point FD,
# Dirichlet, h = 1/(n+1)) = K / h^2 in terms of the (4, -1) stencil K, so
# M = (alpha / h^4) K^T K + I, alpha = 1e-3.  Desired states:
#   2d_asym   : sum of 4 Gaussians (sigma 0.1) at radius sqrt(0.08) about
#               (0.5, 0.5), angles 5 pi/4 + (k-1) pi/2 + theta, theta in [0, pi/2]
#   2d_sym    : a sin(pi x1) sin(pi x2), a in [0.8, 1.2]
#   2d_nonsep : a sin(2 pi x1 x2),      a in [0.8, 1.2]
# The bound psi is constant: the (1 - active) quantile of the unconstrained
# state M^-1 y_d at the mid parameter (App. "Mesh sizes and active-set
# details", percentile protocol).  The grid sine modes diagonalise K, hence
# M, so M^-1 y_d is computed exactly by an orthonormal 2D DST-I: eigenvalue
# 1 + alpha ((s_i + s_j) / h^2)^2, s_q = 4 sin^2(q pi h / 2).  Parameters are
# uniformly spaced over their range (the paper uses 30 instances).
# ---------------------------------------------------------------------------
@dataclass
class OCPWorkload:
    name: str
    op: "Operator"
    y_d: np.ndarray           # [B][N]
    psi: np.ndarray           # [B][N]
    params: np.ndarray        # [B]
    tau: float = 1e-10


OCP_2D = ("2d_asym", "2d_sym", "2d_nonsep")
OCP_RANGES = {"2d_asym": (0.0, math.pi / 2), "2d_sym": (0.8, 1.2), "2d_nonsep": (0.8, 1.2)}


def ocp_desired_state(name: str, n: int, p: float) -> np.ndarray:
    x1, x2 = _coords(n, 2)
    if name == "2d_sym":
        return p * np.sin(np.pi * x1) * np.sin(np.pi * x2)
    if name == "2d_nonsep":
        return p * np.sin(2.0 * np.pi * x1 * x2)
    if name == "2d_asym":
        r, sig = math.sqrt(0.08), 0.1
        out = np.zeros_like(x1)
        for k in range(4):
            ang = 5.0 * math.pi / 4.0 + k * math.pi / 2.0 + p
            c1, c2 = 0.5 + r * math.cos(ang), 0.5 + r * math.sin(ang)
            out += np.exp(-((x1 - c1) ** 2 + (x2 - c2) ** 2) / (2.0 * sig * sig))
        return out
    raise ValueError(name)


def ocp_unconstrained(n: int, y_d: np.ndarray, alpha: float = 1e-3) -> np.ndarray:
    """M^-1 y_d for M = (alpha / h^4) K^T K + I on the n x n grid (exact, DST-I)."""
    from scipy.fft import dstn, idstn
    h = 1.0 / (n + 1)
    s = 4.0 * np.sin(np.arange(1, n + 1) * np.pi * h / 2.0) ** 2
    lam = 1.0 + alpha * ((s[:, None] + s[None, :]) / h ** 2) ** 2
    c = dstn(y_d.reshape(n, n), type=1, norm="ortho")
    return idstn(c / lam, type=1, norm="ortho").ravel()


def ocp_2d(name: str, n: int = 127, B: int = 4, alpha: float = 1e-3, active: float = 0.2) -> OCPWorkload:
    h = 1.0 / (n + 1)
    K = canonical_csr(laplacian_2d(n))
    N = n * n
    op = Operator(n=n, dim=2, B=canonical_csr((alpha / h ** 4) * (K.T @ K)), shift=1.0,
                  name=f"ocp{name.replace('_', '')}_n{n}", A=K, alpha=alpha / h ** 4)
    lo, hi = OCP_RANGES[name]
    y_unc_mid = ocp_unconstrained(n, ocp_desired_state(name, n, 0.5 * (lo + hi)), alpha)
    psi_val = float(np.quantile(y_unc_mid, 1.0 - active))
    params = np.linspace(lo, hi, B) if B > 1 else np.array([0.5 * (lo + hi)])
    y_d = np.stack([ocp_desired_state(name, n, p) for p in params])
    psi = np.full((B, N), psi_val)
    return OCPWorkload(name=f"ocp_{name}_n{n}_B{B}", op=op, y_d=y_d, psi=psi, params=params)


def ocp_2d_sym(n: int = 127, B: int = 4, alpha: float = 1e-3, active: float = 0.2) -> OCPWorkload:
    return ocp_2d("2d_sym", n, B, alpha, active)


# ---------------------------------------------------------------------------
# 3D Laplacian optimal control, 3d_obstacle (App. "3D Laplacian problems"):
# y_d = 3 sum_k exp(-|x - s_k(theta)|^2 / (2 * 0.12^2)), the four sources
# (0.3,0.3,0.5), (0.3,0.7,0.5), (0.7,0.3,0.5), (0.7,0.7,0.5) rotated about
# the x3-axis through (0.5, 0.5) by theta in [0, pi/2]; M = alpha L^T L + I,
# L = 7-point -Laplacian.  The bound is the (1 - active) quantile of the
# unconstrained state at the mid angle (the 2D percentile protocol; the
# paper bisects psi loosely for its 3D suite), computed exactly by a 3D DST.
# ---------------------------------------------------------------------------
def laplacian_3d(n: int) -> sp.csr_matrix:
    """Unscaled 7-point stencil (6, -1) on the n^3 interior grid, x fastest."""
    T = _second_diff(n)
    I = sp.identity(n, format="csr")
    return canonical_csr(sp.kron(sp.kron(I, I), T) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(T, I), I))


def sine_modes_3d(n: int, k: int):
    """The k lowest grid sine modes of the 3D Laplacian (orthonormal), ordered
    by s_i + s_j + s_l with ties broken lexicographically by (i, j, l);
    i is the x index.  Returns (Z [N x k], [(i, j, l)])."""
    h = 1.0 / (n + 1)
    s = lambda q: 4.0 * math.sin(q * math.pi * h / 2.0) ** 2
    qmax = min(n, int(math.ceil(k ** (1.0 / 3.0))) + 3)
    trip = sorted(((i, j, l) for i in range(1, qmax + 1) for j in range(1, qmax + 1) for l in range(1, qmax + 1)),
                  key=lambda t: (s(t[0]) + s(t[1]) + s(t[2]), t))[:k]
    x = np.arange(1, n + 1) * h
    c = math.sqrt(2.0 / (n + 1)) ** 3
    cols = [c * np.einsum("a,b,c->abc", np.sin(l * math.pi * x), np.sin(j * math.pi * x),
                          np.sin(i * math.pi * x)).ravel() for i, j, l in trip]
    return np.asfortranarray(np.column_stack(cols)), trip


def ocp_unconstrained_3d(n: int, y_d: np.ndarray, alpha: float = 1e-3) -> np.ndarray:
    from scipy.fft import dstn, idstn
    h = 1.0 / (n + 1)
    s = 4.0 * np.sin(np.arange(1, n + 1) * np.pi * h / 2.0) ** 2
    lam = 1.0 + alpha * ((s[:, None, None] + s[None, :, None] + s[None, None, :]) / h ** 2) ** 2
    c = dstn(y_d.reshape(n, n, n), type=1, norm="ortho")
    return idstn(c / lam, type=1, norm="ortho").ravel()


def ocp_3d_obstacle(n: int = 20, B: int = 4, alpha: float = 1e-3, active: float = 0.2) -> OCPWorkload:
    h = 1.0 / (n + 1)
    K = laplacian_3d(n)
    op = Operator(n=n, dim=3, B=canonical_csr((alpha / h ** 4) * (K.T @ K)), shift=1.0,
                  name=f"ocp3dobst_n{n}", A=K, alpha=alpha / h ** 4)
    x1, x2, x3 = _coords(n, 3)
    base = ((0.3, 0.3, 0.5), (0.3, 0.7, 0.5), (0.7, 0.3, 0.5), (0.7, 0.7, 0.5))

    def y_d(theta):
        out = np.zeros_like(x1)
        ct, st = math.cos(theta), math.sin(theta)
        for bx, by, bz in base:
            cx = 0.5 + ct * (bx - 0.5) - st * (by - 0.5)
            cy = 0.5 + st * (bx - 0.5) + ct * (by - 0.5)
            out += np.exp(-((x1 - cx) ** 2 + (x2 - cy) ** 2 + (x3 - bz) ** 2) / (2.0 * 0.12 ** 2))
        return 3.0 * out

    psi_val = float(np.quantile(ocp_unconstrained_3d(n, y_d(math.pi / 4), alpha), 1.0 - active))
    params = np.linspace(0.0, math.pi / 2, B) if B > 1 else np.array([math.pi / 4])
    return OCPWorkload(name=f"ocp_3d_obstacle_n{n}_B{B}", op=op, y_d=np.stack([y_d(t) for t in params]),
                       psi=np.full((B, n ** 3), psi_val), params=params)


# ---------------------------------------------------------------------------
# Space-time extension (App. "Space-time extension"): implicit Euler in all
# at once form.  F is block lower bidiagonal with diagonal blocks
# D = I/dt + L and subdiagonal blocks -I/dt (y^0 = 0), M_st = alpha F^T F + I
# is block tridiagonal; unknowns ordered time-major (step n holds entries
# n N_s .. (n+1) N_s - 1).  The desired state follows the paper's space-time
# recipe in 2D: a temporal ramp (1 - exp(-t/0.2)) times four Gaussians
# (sigma 0.12) rotating with theta about the centre as in 2d_asym, t_n = n dt,
# T = 1.  The bound is fixed at 0.7 max y_unc at the mid parameter (the
# space-time protocol; not target-calibrated), y_unc by a sparse direct solve.
# ---------------------------------------------------------------------------
def spacetime_forward(L: sp.spmatrix, n_t: int, T: float = 1.0) -> sp.csr_matrix:
    dt = T / n_t
    Ns = L.shape[0]
    I = sp.identity(Ns, format="csr")
    sub = sp.diags([np.ones(n_t - 1)], [-1], shape=(n_t, n_t))
    F = sp.kron(sp.identity(n_t), I / dt + L) - sp.kron(sub, I / dt)
    return canonical_csr(F)


def kron_basis(Z_s: np.ndarray, n_t: int) -> np.ndarray:
    """Z_st = I_nt (x) Z_s (eq. kron_basis), dense N_s n_t x r n_t."""
    return np.kron(np.eye(n_t), Z_s)


def const_time_basis(Z_s: np.ndarray, n_t: int) -> np.ndarray:
    """The constant-in-time lift 1_nt (x) Z_s."""
    return np.kron(np.ones((n_t, 1)), Z_s)


def spacetime_2d(n: int = 15, n_t: int = 10, B: int = 2, alpha: float = 1e-3, T: float = 1.0) -> OCPWorkload:
    h = 1.0 / (n + 1)
    L = canonical_csr(laplacian_2d(n) / (h * h))
    F = spacetime_forward(L, n_t, T)
    Ns = n * n
    N = Ns * n_t
    op = Operator(n=n, dim=2, B=canonical_csr(alpha * (F.T @ F)), shift=1.0, name=f"st2d_n{n}_t{n_t}",
                  A=F, alpha=alpha)
    dt = T / n_t
    x1, x2 = _coords(n, 2)
    r, sig = math.sqrt(0.08), 0.12

    def y_d(theta):
        g = np.zeros(Ns)
        for k in range(4):
            ang = 5.0 * math.pi / 4.0 + k * math.pi / 2.0 + theta
            c1, c2 = 0.5 + r * math.cos(ang), 0.5 + r * math.sin(ang)
            g += np.exp(-((x1 - c1) ** 2 + (x2 - c2) ** 2) / (2.0 * sig * sig))
        ramp = 1.0 - np.exp(-dt * np.arange(1, n_t + 1) / 0.2)
        return np.kron(ramp, g)

    M = (alpha * (F.T @ F) + sp.identity(N)).tocsc()
    y_unc = spla.spsolve(M, y_d(math.pi / 4))
    psi_val = 0.7 * float(np.max(y_unc))
    # the four Gaussians repeat under a rotation by pi/2: sample [0, pi/2)
    params = np.linspace(0.0, math.pi / 2, B, endpoint=False) if B > 1 else np.array([math.pi / 4])
    return OCPWorkload(name=f"st2d_n{n}_t{n_t}_B{B}", op=op, y_d=np.stack([y_d(t) for t in params]),
                       psi=np.full((B, N), psi_val), params=params)


MLP_DIMS = (4, 128, 128, 512)


def mlp_params(seed: int = 0) -> np.ndarray:
    """Seeded initial parameters of the theta -> C network, packed FP32:
    W1 (128x4), b1, W2 (128x128), b2, W3 (512x128), b3, weights row-major
    [out][in].  He-uniform weights (last layer scaled by 0.1), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(3):
        lim = math.sqrt(6.0 / MLP_DIMS[l]) * (0.1 if l == 2 else 1.0)
        W = rng.uniform(-lim, lim, size=(MLP_DIMS[l + 1], MLP_DIMS[l])).astype(np.float32)
        parts += [W.ravel(), np.zeros(MLP_DIMS[l + 1], dtype=np.float32)]
    return np.concatenate(parts)


def pod_snapshots(N: int, M: int, sigma, seed: int = 0):
    """Snapshot columns with a prescribed centred spectrum:
    X = mu 1^T + U diag(sigma) V^T with U (N x r) and V (M x r) orthonormal
    and V^T 1 = 0, so the mean-centred matrix is exactly U diag(sigma) V^T
    (its singular values are sigma, its left singular vectors U).
    Returns X (N x M, column-major) and U."""
    rng = np.random.default_rng(seed)
    sigma = np.asarray(sigma, dtype=np.float64)
    r = len(sigma)
    U = np.linalg.qr(rng.standard_normal((N, r)))[0]
    G = rng.standard_normal((M, r))
    G -= G.mean(axis=0, keepdims=True)
    V = np.linalg.qr(G)[0]
    mu = rng.standard_normal(N)
    X = np.asfortranarray(mu[:, None] + (U * sigma) @ V.T)
    return X, U


def c3_operator(n: int = 255, seed: int = 300):
    h = 1.0 / (n + 1)
    G = gaussian_field_2d(n, seed)
    KG = canonical_csr(diffusion_2d(np.exp(G)))
    B = canonical_csr(1e-2 * (KG @ KG) / (h * h))
    op = Operator(n=n, dim=2, B=B, shift=h * h, name=f"hetdiff2d_{n}", A=KG, alpha=1e-2 / (h * h))
    return op, KG


def c3_thetas(count: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(count, 4))


def c3_instance(n: int, theta, mask_field: np.ndarray, shift: float) -> Instance:
    mu, cx, cy, t = (float(v) for v in theta)
    rho = 0.05 + 0.55 * t
    mask = mask_top_fraction(mask_field, rho)
    b = gaussian_bump(n, (0.2 + 0.6 * cx, 0.2 + 0.6 * cy))
    return Instance(mask=mask, b=b, a=(1.0 + mu) ** 2, c=shift, theta=np.asarray(theta, dtype=np.float64))


def c3_workload(n: int = 255, k: int = 32, B: int = 256, theta_seed: int = 310,
                field_seed: int = 301, op_seed: int = 300) -> Workload:
    """Heterogeneous-diffusion sweep: S_mu = (1+mu)^2 * 1e-2 K_G M_L^{-1} K_G + M_L.

    K_G: diffusion with kappa = exp(G), G a unit-variance squared-exponential
    field (correlation length 0.1, seed 300), harmonic faces.  Its eigenvectors
    (shift-invert Lanczos on K_G) are the eigenvectors of every S_mu.
    theta = (mu, cx, cy, t) ~ U[0,1]^4; active fraction 0.05 + 0.55 t as the
    top quantile of one fixed sinusoid field (nested sets); Gaussian-bump rhs.
    """
    op, KG = c3_operator(n, op_seed)
    Z = _cached(f"c3_Z_n{n}_k{k}_s{op_seed}", lambda: _low_symmetric(KG, k)) if k > 0 \
        else np.zeros((op.N, 0), order="F")
    Z = np.asfortranarray(Z)
    mf = sinusoid_field(n, field_seed)
    thetas = c3_thetas(B, theta_seed)
    insts = [c3_instance(n, th, mf, op.shift) for th in thetas]
    return Workload(name=f"c3_hetdiff2d_n{n}_k{k}_B{B}", op=op, Z=Z, instances=insts, tol=1e-8,
                    meta={"mask_field": mf})


def c5_operator(n: int = 127, seed: int = 600):
    """K = h (7-point flux form) with kappa in {1, 1000}; S = K^2 / h^3 + 1e-2 h^3 I.
    S is assembled only when asked for (50 M entries at 127^3); the solver
    applies it in the factored form."""
    h = 1.0 / (n + 1)
    kap = inclusion_field_3d(n, seed)
    K = canonical_csr(diffusion_3d(kap))
    op = Operator(n=n, dim=3, B=None, shift=1e-2 * h ** 3, name=f"cht3d_{n}", A=K, alpha=1.0 / h ** 3)
    return op, K


def c5_workload(n: int = 127, k: int = 64, B: int = 16, seed0: int = 700, nc: int | None = None) -> Workload:
    """3D two-material diffusion (1:1000 inclusions, 15% volume), S = K M_L^{-1} K + 1e-2 M_L.

    Reference modes: with ``nc`` None, the k lowest eigenvectors of K itself
    (they are S's; small grids).  With ``nc`` given (a coarse grid with
    n + 1 = c (nc + 1), the paper's offline route for large grids, Sec.
    "Coarse-grid eigenmode prolongation"), ``Z`` is None and ``meta`` holds
    the k lowest eigenvectors ``Zc`` of the coarse operator K_c (the same
    inclusion field on the nc^3 grid): the solver side prolongs and
    orthonormalises them (Alg. 4)."""
    op, K = c5_operator(n)
    meta = {}
    if nc is not None:
        if (n + 1) % (nc + 1) != 0:
            raise ValueError("coarse grid must satisfy n + 1 = c (nc + 1)")
        _, Kc = c5_operator(nc)
        Zc = _cached(f"c5_Z_n{nc}_k{k}", lambda: _low_symmetric(Kc, k))
        meta = {"Zc": np.asfortranarray(Zc), "nc": nc}
        Z = None
    else:
        Z = _cached(f"c5_Z_n{n}_k{k}", lambda: _low_symmetric(K, k)) if k > 0 \
            else np.zeros((op.N, 0), order="F")
        Z = np.asfortranarray(Z)
    insts = []
    for m in range(B):
        rho = 0.15 + 0.20 * m / max(B - 1, 1)
        mask = mask_top_fraction(sinusoid_field(n, seed0 + m, dim=3), rho)
        cen = np.random.default_rng(seed0 + 100 + m).uniform(0.2, 0.8, size=3)
        b = gaussian_bump(n, cen, dim=3)
        insts.append(Instance(mask=mask, b=b))
    return Workload(name=f"c5_cht3d_n{n}_k{k}_B{B}", op=op, Z=Z, instances=insts, tol=1e-8, meta=meta)
