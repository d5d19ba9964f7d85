"""FP64 oracle of the offline coarse-grid reference basis (test
infrastructure only; only the tests use this module).

Sec. "Coarse-grid eigenmode prolongation", eq. (prolong) and Alg. 4: coarse
eigenmodes are carried to the fine grid by linear interpolation (the
Kronecker product of the 1D operator over the dimensions), then
orthonormalised by an economy QR, dropping columns whose |R_jj| is below the
singular-value tolerance.

Readings: the 1D operator evaluates, at fine node i (position (i+1)/(n+1)),
the piecewise-linear interpolant of the coarse values at positions
(j+1)/(n_c+1) with zero Dirichlet values at 0 and 1 (for c = 2 and
n = 2 n_c + 1 this is the standard multigrid interpolation).  The drop
test is relative, |R_jj| <= tau_sv ||column j|| (the paper gives no value;
default 1e-10), and the returned basis is an orthonormal basis of the span
of the kept columns (a QR of the kept columns), as for the restricted
modes.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = ["prolongation_1d", "prolongation", "coarse_basis", "reference_eigs"]


def prolongation_1d(n: int, nc: int) -> sp.csr_matrix:
    """n x nc linear interpolation, zero boundary values."""
    rows, cols, vals = [], [], []
    for i in range(n):
        t = (i + 1) / (n + 1) * (nc + 1)      # coarse coordinate; nodes at 1..nc
        j = int(np.floor(t))
        w = t - j
        for node, wt in ((j, 1.0 - w), (j + 1, w)):
            if 1 <= node <= nc and wt != 0.0:
                rows.append(i)
                cols.append(node - 1)
                vals.append(wt)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))


def prolongation(n: int, nc: int, dim: int) -> sp.csr_matrix:
    """P = P1D (x) ... (x) P1D for the lexicographic layout with x fastest."""
    P1 = prolongation_1d(n, nc)
    P = P1
    for _ in range(dim - 1):
        P = sp.kron(P1, P, format="csr")
    return P


def coarse_basis(Zc: np.ndarray, n: int, nc: int, dim: int, tau_sv: float = 1e-10):
    """Prolongate the coarse modes (columns of Zc, nc^dim x r) and
    orthonormalise; returns (basis n^dim x r', kept column indices)."""
    Pt = np.asarray(prolongation(n, nc, dim) @ Zc)
    Q, R = np.linalg.qr(Pt, mode="reduced")
    norms = np.linalg.norm(Pt, axis=0)
    keep = [j for j in range(Pt.shape[1]) if norms[j] > 0 and abs(R[j, j]) > tau_sv * norms[j]]
    if len(keep) < Pt.shape[1]:
        Q, _ = np.linalg.qr(Pt[:, keep], mode="reduced")
    return Q, np.asarray(keep, dtype=np.int64)


def reference_eigs(spec, r: int):
    """The r smallest eigenpairs of the full reference operator by its plain
    definition (dense symmetric eigensolver; small grids only).  spec is an
    assembled matrix or ("factored", A, alpha, shift)."""
    if isinstance(spec, tuple) and spec and spec[0] == "factored":
        _, A, alpha, shift = spec
        S = (alpha * (A.T @ A) + shift * sp.identity(A.shape[0])).toarray()
    else:
        S = spec.toarray()
    lam, U = np.linalg.eigh(0.5 * (S + S.T))
    return lam[:r], U[:, :r]
