"""FP64 oracle of the primal active-set outer loop (test infrastructure only).

The appendix algorithm on active-set identification: start from y = 0 and an
empty active set; at every outer step fix y on the active set to the bound
psi, solve the restricted system M_II y_I = (y_d)_I - M_IA psi_A (eq.
reduced), and predict the next active set as {i : y_i > psi_i - tau}; stop
when the prediction repeats the current set.  The inner solve here is the
exact solution (Cholesky with double-double refinement) or, on request,
the oracle's A-DEF2.

Only the tests use this module.
"""
from __future__ import annotations

import numpy as np

from .solver import compact, exact_solution, restricted_operator, solve_instance

__all__ = ["apply_full", "coupled_rhs", "active_set"]


def apply_full(spec, v: np.ndarray) -> np.ndarray:
    """M v on the full domain for an assembled matrix or ("factored", A, alpha, shift)."""
    if isinstance(spec, tuple) and spec and spec[0] == "factored":
        _, A, alpha, shift = spec
        return alpha * (A.T @ (A @ v)) + shift * v
    return spec @ v


def coupled_rhs(spec, y_d: np.ndarray, psi: np.ndarray, active: np.ndarray) -> np.ndarray:
    """(y_d)_I - M_IA psi_A as a global vector (entries on the active set are
    not part of the system and are returned as 0)."""
    psi_A = np.where(active != 0, psi, 0.0)
    b = y_d - apply_full(spec, psi_A)
    return np.where(active != 0, 0.0, b)


def active_set(spec, y_d: np.ndarray, psi: np.ndarray, tau: float = 1e-10, max_outer: int = 20,
               inner: str = "exact", Z=None, tol: float = 1e-12):
    """Returns (y, active mask, outer iterations, converged)."""
    N = y_d.shape[0]
    active = np.zeros(N, dtype=np.uint8)
    y = np.zeros(N)
    for k in range(max_outer):
        I, _, _ = compact(active)
        b = coupled_rhs(spec, y_d, psi, active)
        y = np.where(active != 0, psi, 0.0)
        if I.size:
            if inner == "exact":
                S_II, _ = restricted_operator(spec, I)
                y[I] = exact_solution(S_II, b[I])
            else:
                y[I] = solve_instance(spec, Z, active, b, tol).x[I]
        new = (y > psi - tau).astype(np.uint8)
        if np.array_equal(new, active):
            return y, active, k + 1, True
        active = new
    return y, active, max_outer, False
