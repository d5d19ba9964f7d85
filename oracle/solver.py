"""FP64 CPU oracle for restricted-system A-DEF2 deflated Jacobi-PCG.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference that the
GPU library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it; the HIP path shares no
code with it.

Each function follows a passage of the paper (arXiv 2606.17971, "Online
Spectral Deflation for State Constrained Optimal Control Problems"):

* inactive set, restricted system ........ Sec. 2 "Reduced inactive set system",
                                           eq. (reduced)
* submatrix restriction .................. App. "Matrix assembly and active set
                                           restriction"
* restricted reference basis + QR ........ Sec. "Core idea: reference eigenmode
                                           basis" (simple restriction)
* Ritz reselection from a pool .......... Sec. "Ritz re-selection"
* POD candidates, safe merge ............. Sec. "Online POD enrichment",
                                           Sec. "Conditioning-based safe
                                           merge", Alg. 2
* coarse Gram E, fallback ................ Sec. "Online deflated solve (A-DEF2)",
                                           Alg. 3 (online workflow), Remark
                                           tau_cond; App. "GPU implementation"
                                           (Cholesky of E, reused per solve)
* A-DEF2 loop ............................ Alg. 1 with the reading below
* stopping rule .......................... App. "CG stopping criterion",
                                           eq. (cg_stop)
* exact solution for parity .............. eq. (accuracy_rel_err): the direct
                                           solution of eq. (reduced)

Reading of Alg. 1: as printed, the loop advances x along
the *unprojected* preconditioned residual while the step length uses the
projected operator, so x drifts inside range(Z) and the unprojected residual
used by the stopping test stops decreasing.  The oracle uses the A-DEF2
recurrence of the works the algorithm cites (Tang et al. 2009; Gaul et al.
2014): CG preconditioned by  P K + Q  with P = I - Z E^{-1} Z^T M_II
(eq. proj) and Q = Z E^{-1} Z^T (eq. coarse), started from the deflated
initial guess.  The search direction is built from y = P K r + Q r.  In exact
arithmetic Z^T r = 0, so Q r vanishes and y = P K r; the Q r term is kept
because it removes the rounding drift of Z^T r, which the projected
iteration cannot reduce otherwise (it is the additive coarse term that makes
A-DEF2 robust to inexact coarse solves).  The recurrence residual is the
unprojected residual b - M_II x, one residual serves both the recurrence and
the stopping test, as the appendix on stopping describes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = [
    "compact", "restrict", "restricted_basis", "ritz_reselect", "safe_merge", "CoarseSpace",
    "coarse_setup",
    "apply_projector", "adef2", "jacobi_pcg", "SolveResult", "solve_instance",
    "two_sum", "two_prod", "dd_residual", "exact_solution", "rel_err",
    "FactoredOp", "restrict_factored", "restricted_operator",
    "STATUS_OK", "STATUS_FALLBACK", "STATUS_MAXIT",
]

STATUS_OK = 0
STATUS_FALLBACK = 1
STATUS_MAXIT = 2


# ---------------------------------------------------------------------------
# inactive set and restriction (eq. reduced; App. matrix assembly)
# ---------------------------------------------------------------------------
def compact(mask: np.ndarray):
    """Inactive index set of a 0/1 active mask.

    Returns (I, g2l, n_I): I lists the indices with mask == 0 in ascending
    order; g2l[i] is the position of i in I, or -1 for active nodes.
    """
    mask = np.asarray(mask)
    N = mask.size
    I = []
    g2l = np.full(N, -1, dtype=np.int64)
    for i in range(N):
        if mask[i] == 0:
            g2l[i] = len(I)
            I.append(i)
    return np.asarray(I, dtype=np.int64), g2l, len(I)


def restrict(S: sp.spmatrix, I: np.ndarray):
    """M_II = S[I, I] by submatrix indexing, and its diagonal d_I."""
    S = sp.csr_matrix(S)
    S_II = S[I, :][:, I].tocsr()
    d_I = S.diagonal()[I].copy()
    return S_II, d_I


class FactoredOp:
    """M_II = alpha A[:, I]^T A[:, I] + shift I, the restriction of the paper's
    M = alpha A^T A + I (eq. schur, mass-weighted) to the inactive set.

    (A^T A)[I, I] = A[:, I]^T A[:, I] because every row of A contributes; the
    product is applied as two sparse matrix-vector products and never formed,
    except by ``assembled()`` (used only to factorise a preconditioner).
    """

    def __init__(self, A, alpha: float, shift: float, I):
        self.A_I = sp.csr_matrix(A)[:, I].tocsr()
        self.alpha = float(alpha)
        self.shift = float(shift)
        n = len(I)
        self.shape = (n, n)
        self.T = self

    def __matmul__(self, x):
        x = np.asarray(x)
        return self.alpha * (self.A_I.T @ (self.A_I @ x)) + self.shift * x

    def diagonal(self):
        col2 = np.asarray(self.A_I.multiply(self.A_I).sum(axis=0)).ravel()
        return self.alpha * col2 + self.shift

    def assembled(self) -> sp.csr_matrix:
        M = self.alpha * (self.A_I.T @ self.A_I) + self.shift * sp.identity(self.shape[0])
        return sp.csr_matrix(M)

    def toarray(self):
        return self.assembled().toarray()


def restrict_factored(A, alpha: float, shift: float, I):
    """M_II of M = alpha A^T A + shift I, and its diagonal."""
    op = FactoredOp(A, alpha, shift, I)
    return op, op.diagonal()


def restricted_operator(spec, I):
    """M_II for an operator given either as an assembled sparse matrix or as
    ("factored", A, alpha, shift)."""
    if isinstance(spec, tuple) and spec and spec[0] == "factored":
        return restrict_factored(spec[1], spec[2], spec[3], I)
    return restrict(spec, I)


def restricted_basis(Z: np.ndarray, I: np.ndarray, drop_rel: float = 1e-6):
    """Simple restriction Z|_I followed by QR orthonormalisation.

    Householder QR of Z[I, :] (no pivoting).  Column j is dropped when the
    part of it orthogonal to the earlier columns, |R_jj|, is at most
    ``drop_rel`` times the norm of the restricted column itself (a column
    numerically inside the span of its predecessors, or identically zero).
    Returns the orthonormal basis (n_I x k') and the kept column indices.
    """
    ZI = np.asarray(Z)[I, :]
    k = ZI.shape[1]
    if k == 0 or ZI.shape[0] == 0:
        return np.zeros((ZI.shape[0], 0)), np.zeros(0, dtype=np.int64)
    Q, R = np.linalg.qr(ZI, mode="reduced")
    norms = np.linalg.norm(ZI, axis=0)
    keep = [j for j in range(k) if norms[j] > 0 and abs(R[j, j]) > drop_rel * norms[j]]
    if len(keep) < k:
        # re-orthonormalise the kept columns only, so the span excludes the
        # dropped directions exactly
        Q, R = np.linalg.qr(ZI[:, keep], mode="reduced")
    return Q, np.asarray(keep, dtype=np.int64)


def ritz_reselect(S_II, Zo: np.ndarray, r: int):
    """Sec. "Ritz re-selection": the orthonormal restricted pool Zo
    (n_I x r_pool) defines the projected eigenproblem
    Zo^T M_II Zo c_j = mu_j c_j; the r eigenvectors with the smallest Ritz
    values give the basis Zo [c_1 .. c_r].  Returns (basis, Ritz values of
    the kept vectors); r <= 0 or r >= r_pool returns the pool unchanged."""
    if r <= 0 or r >= Zo.shape[1]:
        return Zo, None
    F = Zo.T @ np.asarray(S_II @ Zo)
    F = 0.5 * (F + F.T)
    mu, C = np.linalg.eigh(F)            # ascending
    return Zo @ C[:, :r], mu[:r]


def safe_merge(S_II, Phi_eig: np.ndarray, Phi_pod: np.ndarray, tau_safe: float = 1e4,
               tau_dep: float = 1e-10) -> np.ndarray:
    """Alg. 2: start from the orthonormal eigenmode basis; take the POD
    candidates in order, orthogonalise each against the current basis (two
    passes of Gram-Schmidt), skip it when what remains is shorter than
    tau_dep, otherwise normalise it and accept the trial basis unless
    cond(Z_trial^T M_II Z_trial) exceeds tau_safe, which ends the merge."""
    Z = np.asarray(Phi_eig, dtype=np.float64)
    for j in range(Phi_pod.shape[1]):
        z = np.array(Phi_pod[:, j], dtype=np.float64)
        for _ in range(2):
            z = z - Z @ (Z.T @ z)
        nz = float(np.linalg.norm(z))
        if nz < tau_dep:
            continue
        trial = np.column_stack([Z, z / nz])
        Et = trial.T @ np.asarray(S_II @ trial)
        ev = np.linalg.eigvalsh(0.5 * (Et + Et.T))
        if not (ev[0] > 0 and ev[-1] / ev[0] <= tau_safe):
            break
        Z = trial
    return Z


# ---------------------------------------------------------------------------
# coarse space (Sec. A-DEF2: E, Q, P; App. GPU implementation: Cholesky)
# ---------------------------------------------------------------------------
@dataclass
class CoarseSpace:
    Z: np.ndarray                  # n_I x k orthonormal basis
    W: np.ndarray                  # M_II Z
    E: np.ndarray                  # Z^T M_II Z, symmetrised
    cond: float                    # 2-norm condition number of E (inf on failure)
    chol: tuple | None             # Cholesky factor of E, or None
    kept: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int64))

    @property
    def k(self) -> int:
        return self.Z.shape[1]

    def solve(self, g: np.ndarray) -> np.ndarray:
        """E^{-1} g by the two triangular solves with the Cholesky factor."""
        return sla.cho_solve(self.chol, g)


def coarse_setup(S_II: sp.spmatrix, Zo: np.ndarray, tau_cond: float = 1e10):
    """E = Z^T M_II Z, its condition number and Cholesky factor.

    Returns (space, fallback): fallback is True when cond(E) > tau_cond or the
    Cholesky factorisation fails (Alg. 3, Remark tau_cond); the instance is
    then solved by plain Jacobi-PCG.
    """
    k = Zo.shape[1]
    if k == 0:
        e = np.zeros((0, 0))
        return CoarseSpace(Zo, Zo.copy(), e, 1.0, None), False
    W = np.asarray(S_II @ Zo)
    E = Zo.T @ W
    E = 0.5 * (E + E.T)
    ev = np.linalg.eigvalsh(E)
    cond = float(ev[-1] / ev[0]) if ev[0] > 0 else math.inf
    try:
        chol = sla.cho_factor(E, lower=True)
    except np.linalg.LinAlgError:
        chol = None
    fallback = chol is None or not (cond <= tau_cond)
    return CoarseSpace(Zo, W, E, cond, chol), fallback


def apply_projector(cs: CoarseSpace, v: np.ndarray) -> np.ndarray:
    """P v = v - Z E^{-1} Z^T M_II v = v - Z E^{-1} (W^T v)  (eq. proj)."""
    if cs.k == 0:
        return v
    return v - cs.Z @ cs.solve(cs.W.T @ v)


def coarse_coefficients(cs: CoarseSpace, r: np.ndarray) -> np.ndarray:
    """E^{-1} Z^T r, the coordinates of the coarse correction Q r = Z E^{-1} Z^T r
    (eq. coarse)."""
    if cs.k == 0:
        return np.zeros(0)
    return cs.solve(cs.Z.T @ r)


def preconditioned_residual(cs: CoarseSpace, z: np.ndarray, r: np.ndarray) -> np.ndarray:
    """y = P K r + Q r with z = K r: the A-DEF2 preconditioner (P^T_D M^-1 + Q
    in the notation of Tang et al. 2009) applied to r."""
    if cs.k == 0:
        return z
    return apply_projector(cs, z) + cs.Z @ coarse_coefficients(cs, r)


# ---------------------------------------------------------------------------
# A-DEF2 deflated PCG (Alg. 1, projected reading)
# ---------------------------------------------------------------------------
@dataclass
class LoopResult:
    x: np.ndarray
    iters: int
    converged: bool
    history: list = field(default_factory=list)


def adef2(S_II, b, cs: CoarseSpace, tol: float, maxit: int = 100000, x0=None,
          d_inv=None, record: bool = False) -> LoopResult:
    """A-DEF2 deflated preconditioned CG on M_II x = b.

    Steps (Alg. 1 with the A-DEF2 preconditioner, see module docstring):
      c0  = E^{-1} Z^T (b - M x0)
      x   = x0 + Z c0                             deflated initial guess
      r   = (b - M x0) - W c0                     unprojected residual b - M x
      z   = K r,  y = P z + Q r,  p = y           K = diag(M_II)^{-1}
      rho = r.y
      while ||r|| > tol ||b|| and it < maxit:     eq. (cg_stop), max 1e5
          w = M p;  alpha = rho / p.w
          x += alpha p;  r -= alpha w
          z = K r;  y = P z + Q r;  rho' = r.y
          p = y + (rho'/rho) p;  rho = rho'
    ``d_inv`` defaults to the Jacobi preconditioner; pass ones for none.
    With ``record`` the iterates and residuals are kept (tiny problems only).

    The residual after the coarse correction is formed from r0 and W = M Z
    rather than recomputed as b - M x: both equal b - M x in exact arithmetic,
    but a recomputed residual carries a rounding component of size
    u ||M|| ||x|| inside range(Z) that the projected iteration never reduces
    (Z^T M p = W^T P y = 0), so the unprojected residual would stall there.
    """
    n = b.shape[0]
    if d_inv is None:
        d_inv = 1.0 / S_II.diagonal()
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - S_II @ x
    c0 = coarse_coefficients(cs, r)
    if cs.k > 0:
        x = x + cs.Z @ c0                     # x = x0 + Q (b - M x0)
        r = r - cs.W @ c0                     # = b - M x, with Z^T r = 0 to coarse rounding
    bnorm = float(np.linalg.norm(b))
    hist = []
    if record:
        hist.append((x.copy(), r.copy()))
    if bnorm == 0.0:
        return LoopResult(np.zeros(n), 0, True, hist)
    z = d_inv * r
    y = preconditioned_residual(cs, z, r)
    rho = float(r @ y)
    p = y
    it = 0
    while float(np.linalg.norm(r)) > tol * bnorm and it < maxit:
        w = S_II @ p
        alpha = rho / float(p @ w)
        x = x + alpha * p
        r = r - alpha * w
        z = d_inv * r
        y = preconditioned_residual(cs, z, r)
        rho_new = float(r @ y)
        p = y + (rho_new / rho) * p
        rho = rho_new
        it += 1
        if record:
            hist.append((x.copy(), r.copy()))
    converged = float(np.linalg.norm(r)) <= tol * bnorm
    return LoopResult(x, it, converged, hist)


def jacobi_pcg(S_II, b, tol: float, maxit: int = 100000, x0=None, d_inv=None,
               record: bool = False) -> LoopResult:
    """Cold Jacobi-PCG: the A-DEF2 loop with an empty coarse space (Alg. 3 fallback)."""
    empty = CoarseSpace(np.zeros((b.shape[0], 0)), np.zeros((b.shape[0], 0)),
                        np.zeros((0, 0)), 1.0, None)
    return adef2(S_II, b, empty, tol, maxit, x0, d_inv, record)


# ---------------------------------------------------------------------------
# one instance end to end (Alg. 3, steps restrict .. reconstruct)
# ---------------------------------------------------------------------------
@dataclass
class SolveResult:
    x: np.ndarray                  # global length N, zero on the active set
    iters: int
    relres_true: float
    cond_E: float
    status: int
    n_I: int
    k_eff: int


def solve_instance(S, Z, mask, b, tol: float, tau_cond: float = 1e10,
                   maxit: int = 100000, x0=None, precond: str = "jacobi",
                   ritz_keep: int = 0, Phi=None, tau_safe: float = 1e4,
                   tau_dep: float = 1e-10) -> SolveResult:
    """Restrict, build the coarse space, solve and scatter one instance.

    S is an assembled sparse matrix or ("factored", A, alpha, shift).  b and x
    are global (length N); b on the active set is ignored and x there is
    returned as zero.  ``x0`` (global) is an optional warm start.
    ``ritz_keep`` > 0 reselects that many Ritz vectors from the restricted
    pool (Sec. "Ritz re-selection").  ``Phi`` (N x p POD modes) enriches the
    restricted eigenmodes by the safe merge (Alg. 2) before the coarse setup.
    """
    I, _, n_I = compact(mask)
    S_II, d_I = restricted_operator(S, I)
    b_I = np.asarray(b, dtype=np.float64)[I]
    Zo, kept = restricted_basis(Z, I)
    if Phi is not None and Phi.shape[1] > 0:
        Zo = safe_merge(S_II, Zo, restricted_basis(Phi, I)[0], tau_safe, tau_dep)
    Zo, _ = ritz_reselect(S_II, Zo, ritz_keep)
    cs, fallback = coarse_setup(S_II, Zo, tau_cond)
    cs.kept = kept
    status = STATUS_OK
    cond = cs.cond if cs.k > 0 else 1.0
    if fallback:
        status = STATUS_FALLBACK
        cs = CoarseSpace(np.zeros((n_I, 0)), np.zeros((n_I, 0)), np.zeros((0, 0)), 1.0, None)
    d_inv = 1.0 / d_I if precond == "jacobi" else np.ones(n_I)
    x0_I = None if x0 is None else np.asarray(x0, dtype=np.float64)[I]
    res = adef2(S_II, b_I, cs, tol, maxit, x0_I, d_inv)
    if not res.converged and status == STATUS_OK:
        status = STATUS_MAXIT
    x = np.zeros(np.asarray(mask).size)
    x[I] = res.x
    bn = float(np.linalg.norm(b_I))
    rel = float(np.linalg.norm(b_I - S_II @ res.x)) / bn if bn > 0 else 0.0
    return SolveResult(x, res.iters, rel, cond, status, n_I, cs.k)


# ---------------------------------------------------------------------------
# exact solution for parity (eq. accuracy_rel_err uses a direct solve)
# ---------------------------------------------------------------------------
def two_sum(a, b):
    """Knuth's error-free sum: a + b = s + e exactly."""
    s = a + b
    bb = s - a
    e = (a - (s - bb)) + (b - bb)
    return s, e


_SPLIT = 134217729.0  # 2^27 + 1


def _split(a):
    c = _SPLIT * a
    hi = c - (c - a)
    return hi, a - hi


def two_prod(a, b):
    """Dekker's error-free product: a * b = p + e exactly (no FMA needed)."""
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def _dd_add(hi, lo, p, e):
    """(hi, lo) + (p, e) in double-double."""
    s1, e1 = two_sum(hi, p)
    e1 = e1 + (lo + e)
    return two_sum(s1, e1)


def dd_matvec(A: sp.spmatrix, x_hi: np.ndarray, x_lo=None, acc=None):
    """acc + A (x_hi + x_lo) in double-double; returns (hi, lo)."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    hi = np.zeros(n) if acc is None else np.array(acc[0], dtype=np.float64)
    lo = np.zeros(n) if acc is None else np.array(acc[1], dtype=np.float64)
    counts = np.diff(A.indptr)
    rows = np.repeat(np.arange(n), counts)
    slot = np.arange(A.nnz) - np.repeat(A.indptr[:-1], counts)
    for s in range(int(counts.max()) if n and A.nnz else 0):
        sel = slot == s
        rr = rows[sel]
        a = A.data[sel]
        p, e = two_prod(a, x_hi[A.indices[sel]])
        if x_lo is not None:
            e = e + a * x_lo[A.indices[sel]]
        hi[rr], lo[rr] = _dd_add(hi[rr], lo[rr], p, e)
    return hi, lo


def dd_residual(A, x: np.ndarray, b: np.ndarray) -> np.ndarray:
    """b - A x accumulated in double-double, rounded once to FP64.

    A is a sparse matrix or a FactoredOp (then b - alpha A_I^T (A_I x) - shift x
    with every product and sum in double-double)."""
    x = np.asarray(x, dtype=np.float64)
    if isinstance(A, FactoredOp):
        t_hi, t_lo = dd_matvec(A.A_I, x)
        u_hi, u_lo = dd_matvec(sp.csr_matrix(A.A_I.T), t_hi, t_lo)
        p, e = two_prod(np.full_like(u_hi, A.alpha), u_hi)
        e = e + A.alpha * u_lo
        q, f = two_prod(np.full_like(x, A.shift), x)
        hi, lo = _dd_add(np.array(b, dtype=np.float64), np.zeros_like(x), -p, -e)
        hi, lo = _dd_add(hi, lo, -q, -f)
        return hi + lo
    neg_hi, neg_lo = dd_matvec(-sp.csr_matrix(A), x, acc=(np.array(b, dtype=np.float64),
                                                         np.zeros(len(b))))
    return neg_hi + neg_lo


def exact_solution(A: sp.spmatrix, b: np.ndarray, max_refine: int = 20,
                   dense_limit: int = 4000, method: str = "auto") -> np.ndarray:
    """x* = A^{-1} b for SPD A, to about FP64 unit roundoff in the forward error.

    A direct factorisation (dense Cholesky for small systems; for larger
    ones the sparse LU of SuperLU in a minimum-degree ordering, or, with
    method="banded", banded Cholesky in the given ordering), then iterative
    refinement whose residuals are accumulated in double-double (Carson &
    Higham 2018: with residuals in extra precision the limiting forward error
    is of the order of the working precision when cond(A) u < 1).  The
    factorisation only has to be stable enough for the refinement to
    contract, so every method reaches the same x* (eq. accuracy_rel_err uses
    the direct solution as the reference).
    """
    Ares = A
    A = A.assembled() if isinstance(A, FactoredOp) else sp.csr_matrix(A)
    n = A.shape[0]
    if n == 0:
        return np.zeros(0)
    if method == "dense" or (method == "auto" and n <= dense_limit):
        fac = sla.cho_factor(A.toarray(), lower=True)
        solve = lambda r: sla.cho_solve(fac, r)  # noqa: E731
    elif method == "banded":
        # banded Cholesky in the given ordering (lower band storage)
        coo = A.tocoo()
        bw = int(np.max(np.abs(coo.row - coo.col)))
        ab = np.zeros((bw + 1, n))
        low = coo.row >= coo.col
        ab[(coo.row - coo.col)[low], coo.col[low]] = coo.data[low]
        cb = sla.cholesky_banded(ab, lower=True)
        solve = lambda r: sla.cho_solve_banded((cb, True), r)  # noqa: E731
    else:
        lu = spla.splu(sp.csc_matrix(A), permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                       options=dict(SymmetricMode=True))
        solve = lu.solve
    x = solve(b)
    for _ in range(max_refine):
        d = solve(dd_residual(Ares, x, b))
        x = x + d
        if np.linalg.norm(d) <= 1e-16 * np.linalg.norm(x):
            break
    return x


def rel_err(x, x_ref) -> float:
    """e_rel = ||x - x_ref|| / ||x_ref||  (eq. accuracy_rel_err)."""
    den = float(np.linalg.norm(x_ref))
    return float(np.linalg.norm(np.asarray(x) - np.asarray(x_ref))) / den if den > 0 else 0.0
