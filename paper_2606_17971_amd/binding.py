"""Python binding of libadef2 (argument marshalling only).

Every numerical step runs in the HIP library; this module moves arrays to the
GPU with torch, passes raw device pointers through the C ABI declared in
include/adef2.h, and converts results back.  There is no fallback: importing
this module fails when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadef2.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      f"`python -m paper_2606_17971_amd.build` (hipcc, gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

OK, E_ARG, E_STATE, E_HIP, E_NOMEM, E_NOT_SPD, E_UNSUPPORTED, E_NOCONV = 0, -1, -2, -3, -4, -5, -6, -7
W_FALLBACK, W_MAXIT, W_STAGNATED = 1, 2, 3
FP64, FP32_REFINE, MIXED_REFINE, FP64_REFINE = 0, 1, 2, 3
JACOBI, NONE = 0, 1
ENERGY, SPECTRUM = 0, 1   # learned_objective
MAX_K = 64


class Opts(ctypes.Structure):
    _fields_ = [
        ("tau_cond", ctypes.c_double),
        ("drop_rel", ctypes.c_double),
        ("maxit", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("precond", ctypes.c_int32),
        ("inner_rtol", ctypes.c_double),
        ("max_sweeps", ctypes.c_int32),
        ("segment_maxit", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("rows_per_thread", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("w_mode", ctypes.c_int32),
        ("w_boundary", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("ritz_keep", ctypes.c_int32),
        ("tau_safe", ctypes.c_double),
        ("tau_dep", ctypes.c_double),
        ("poll_max", ctypes.c_int32),
        ("learned_objective", ctypes.c_int32),
        ("op_fused", ctypes.c_int32),
        ("op_rows", ctypes.c_int32),
        ("op_group", ctypes.c_int32),
        ("sweep_async", ctypes.c_int32),
        ("update_ws", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_kernels", ctypes.c_int32),
        ("name", ctypes.c_char_p * 24),
        ("launches", ctypes.c_int64 * 24),
        ("total_ms", ctypes.c_double * 24),
        ("alg_bytes", ctypes.c_double * 24),
        ("polls", ctypes.c_int64),
        ("pod_iters", ctypes.c_int64),
    ]


_P = ctypes.c_void_p
_i32, _i64, _f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_Pi32, _Pi64, _Pf64 = (ctypes.POINTER(t) for t in (_i32, _i64, _f64))

_sig = {
    "adef2_default_opts": (None, [ctypes.POINTER(Opts)]),
    "adef2_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(Opts), _P]),
    "adef2_destroy": (ctypes.c_int, [_P]),
    "adef2_set_opts": (ctypes.c_int, [_P, ctypes.POINTER(Opts)]),
    "adef2_set_reference": (ctypes.c_int, [_P, _i64, _P, _P, _P, _i64, _i32, _P]),
    "adef2_set_reference_factored": (ctypes.c_int, [_P, _i64, _P, _P, _P, _i64, _f64, _f64, _i32, _P]),
    "adef2_set_operator_scale": (ctypes.c_int, [_P, _f64, _f64]),
    "adef2_compact": (ctypes.c_int, [_P, _P, _i64, _P, _P, _Pi64]),
    "adef2_restrict": (ctypes.c_int, [_P, _P, _Pi64, _Pi32, _Pf64]),
    "adef2_compact_noalloc": (ctypes.c_int, [_P, _P, _i64, _P, _P, _P, _Pi64]),
    "adef2_solve": (ctypes.c_int, [_P, _P, _P, _f64, _P, _Pi32, _Pf64, _Pf64]),
    "adef2_solve_batched": (ctypes.c_int, [_P, _i32, _P, _P, _P, _P, _P, _f64, _P, _P, _P, _P, _P, _P, _P,
                                           _P]),
    "adef2_pod": (ctypes.c_int, [_P, _i32, _P, _i32, _P, _P]),
    "adef2_set_pod_modes": (ctypes.c_int, [_P, _i32, _P]),
    "adef2_learned_set_params": (ctypes.c_int, [_P, _P, _f64]),
    "adef2_learned_get_params": (ctypes.c_int, [_P, _P]),
    "adef2_learned_prepare": (ctypes.c_int, [_P, _i32, _P, _P, _P, _P, _P, _P]),
    "adef2_learned_loss_grad": (ctypes.c_int, [_P, _P, _P]),
    "adef2_learned_train": (ctypes.c_int, [_P, _i32, ctypes.c_float, _P]),
    "adef2_learned_forward": (ctypes.c_int, [_P, _i32, _P, _P]),
    "adef2_apply_restricted": (ctypes.c_int, [_P, _P, _P]),
    "adef2_coarse_info": (ctypes.c_int, [_P, _P, _P, _Pi32, _Pf64]),
    "adef2_variant": (ctypes.c_int, [_P, _Pi32, _Pi32, _P]),
    "adef2_operator_variant": (ctypes.c_int, [_P, _Pi32, _Pi32, _Pi32, _P]),
    "adef2_update_variant": (ctypes.c_int, [_P, _Pi32, _Pi32, _P]),
    "adef2_active_set_batched": (ctypes.c_int, [_P, _i32, _P, _P, _f64, _f64, _i32, _P, _P, _P, _P, _P]),
    "adef2_pod_enrich": (ctypes.c_int, [_P, _i32, _f64]),
    "adef2_set_enrichment": (ctypes.c_int, [_P, _i32, _P, _P, _i32, _f64]),
    "adef2_prolong_basis": (ctypes.c_int, [_P, _i32, _i64, _i64, _i32, _P, _f64, _P, _Pi32]),
    "adef2_reference_eigs": (ctypes.c_int, [_P, _i32, _P, _i32, _f64, _f64, _P, _P, _P, _Pi32]),
    "adef2_get_stats": (ctypes.c_int, [_P, ctypes.POINTER(Stats)]),
    "adef2_reset_stats": (ctypes.c_int, [_P]),
    "adef2_last_error": (ctypes.c_char_p, [_P]),
}
EXPORTS = tuple(_sig)
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class Adef2Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"adef2 error {code}: {msg}")
        self.code = code


def default_opts(**kw) -> Opts:
    o = Opts()
    _lib.adef2_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _dev(x, dtype) -> torch.Tensor:
    """Contiguous device tensor of the given dtype (copies host data)."""
    if isinstance(x, torch.Tensor):
        t = x.to(device="cuda", dtype=dtype)
    else:
        t = torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")
    return t.contiguous()


def _colmajor(Z) -> torch.Tensor:
    """Column-major FP64 device copy of an N x k array (numpy or torch)."""
    if isinstance(Z, torch.Tensor):
        return Z.to(device="cuda", dtype=torch.float64).T.contiguous().reshape(-1)
    return _dev(np.asfortranarray(Z, dtype=np.float64).ravel(order="F"), torch.float64)


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


@dataclass
class SolveOut:
    x: torch.Tensor
    iters: int
    relres_true: float
    cond_E: float
    status: int


class Solver:
    """One library context bound to the current torch stream."""

    def __init__(self, stream: torch.cuda.Stream | None = None, **opts):
        if not torch.cuda.is_available():
            raise RuntimeError("adef2 needs a GPU (HIP device)")
        self.stream = stream or torch.cuda.current_stream()
        self._ctx = _P()
        self.opts = default_opts(**opts)
        rc = _lib.adef2_create(ctypes.byref(self._ctx), ctypes.byref(self.opts),
                               _P(self.stream.cuda_stream))
        if rc != OK:
            raise Adef2Error(rc, _lib.adef2_last_error(None).decode())
        self._keep = []
        self.n = 0
        self.k = 0

    def close(self):
        if self._ctx:
            _lib.adef2_destroy(self._ctx)
            self._ctx = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, allow=(OK, W_FALLBACK, W_MAXIT, W_STAGNATED)) -> int:
        if rc not in allow:
            raise Adef2Error(rc, _lib.adef2_last_error(self._ctx).decode())
        return rc

    def set_opts(self, **kw):
        for k, v in kw.items():
            setattr(self.opts, k, v)
        self._check(_lib.adef2_set_opts(self._ctx, ctypes.byref(self.opts)))

    # --- reference -------------------------------------------------------
    def set_reference(self, S, Z=None):
        """S: scipy CSR (symmetric positive definite); Z: N x k array or None."""
        n = S.shape[0]
        rp = _dev(np.asarray(S.indptr, dtype=np.int64), torch.int64)
        ci = _dev(np.asarray(S.indices, dtype=np.int32), torch.int32)
        va = _dev(np.asarray(S.data, dtype=np.float64), torch.float64)
        k = 0 if Z is None else int(Z.shape[1])
        Zt = _colmajor(Z) if k > 0 else None
        rc = _lib.adef2_set_reference(self._ctx, n, _ptr(rp), _ptr(ci), _ptr(va), int(S.nnz), k,
                                      _ptr(Zt))
        self._check(rc, allow=(OK,))
        self.n, self.k = n, k

    def set_reference_factored(self, A, alpha: float, shift: float, Z=None):
        """S = alpha A^T A + shift I with A a scipy CSR matrix; Z: N x k or None."""
        n = A.shape[0]
        rp = _dev(np.asarray(A.indptr, dtype=np.int64), torch.int64)
        ci = _dev(np.asarray(A.indices, dtype=np.int32), torch.int32)
        va = _dev(np.asarray(A.data, dtype=np.float64), torch.float64)
        k = 0 if Z is None else int(Z.shape[1])
        Zt = _colmajor(Z) if k > 0 else None
        rc = _lib.adef2_set_reference_factored(self._ctx, n, _ptr(rp), _ptr(ci), _ptr(va),
                                               int(A.nnz), float(alpha), float(shift), k, _ptr(Zt))
        self._check(rc, allow=(OK,))
        self.n, self.k = n, k

    def set_operator(self, op, Z=None, factored: bool = True):
        """Reference operator from a gen.Operator (factored form when it has one)."""
        if factored and getattr(op, "A", None) is not None:
            self.set_reference_factored(op.A, op.alpha, op.shift, Z)
        else:
            self.set_reference(op.S(), Z)

    def set_operator_scale(self, a: float, c: float):
        self._check(_lib.adef2_set_operator_scale(self._ctx, float(a), float(c)), allow=(OK,))

    # --- compaction / restriction ----------------------------------------
    def compact(self, mask):
        m = _dev(mask, torch.uint8)
        n = m.numel()
        I = torch.empty(n, dtype=torch.int32, device="cuda")
        g2l = torch.empty(n, dtype=torch.int32, device="cuda")
        nI = _i64(0)
        self._check(_lib.adef2_compact(self._ctx, _ptr(m), n, _ptr(I), _ptr(g2l), ctypes.byref(nI)),
                    allow=(OK,))
        return I[: nI.value], g2l, nI.value

    def compact_noalloc(self, mask):
        """adef2_compact_noalloc: (I, g2l, n_inactive, device count tensor)."""
        m = _dev(mask, torch.uint8)
        n = m.numel()
        I = torch.empty(n, dtype=torch.int32, device="cuda")
        g2l = torch.empty(n, dtype=torch.int32, device="cuda")
        cnt = torch.empty(1, dtype=torch.int64, device="cuda")
        nI = _i64(0)
        self._check(_lib.adef2_compact_noalloc(self._ctx, _ptr(m), n, _ptr(I), _ptr(g2l), _ptr(cnt),
                                               ctypes.byref(nI)), allow=(OK,))
        return I[: nI.value], g2l, nI.value, cnt

    def restrict(self, mask):
        m = _dev(mask, torch.uint8)
        nI, ke, cond = _i64(0), _i32(0), _f64(0.0)
        rc = _lib.adef2_restrict(self._ctx, _ptr(m), ctypes.byref(nI), ctypes.byref(ke),
                                 ctypes.byref(cond))
        self._check(rc, allow=(OK, W_FALLBACK))
        return nI.value, ke.value, cond.value, rc

    # --- solves ------------------------------------------------------------
    def solve(self, b, tol: float, x0=None) -> SolveOut:
        bt = _dev(b, torch.float64)
        x0t = None if x0 is None else _dev(x0, torch.float64)
        x = torch.empty(self.n, dtype=torch.float64, device="cuda")
        it, rel, cond = _i32(0), _f64(0.0), _f64(0.0)
        rc = _lib.adef2_solve(self._ctx, _ptr(bt), _ptr(x0t), float(tol), _ptr(x), ctypes.byref(it),
                              ctypes.byref(rel), ctypes.byref(cond))
        self._check(rc)
        return SolveOut(x, it.value, rel.value, cond.value, rc)

    def solve_batched(self, masks, b, tol, a=None, c=None, theta=None):
        """tol: one relative tolerance, or one per instance."""
        M = _dev(masks, torch.uint8)
        Bt = _dev(b, torch.float64)
        Th = None if theta is None else _dev(theta, torch.float32)
        B = M.shape[0]
        x = torch.empty((B, self.n), dtype=torch.float64, device="cuda")
        a_h = None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        c_h = None if c is None else np.ascontiguousarray(c, dtype=np.float64)
        iters = np.zeros(B, np.int32)
        status = np.zeros(B, np.int32)
        rel = np.zeros(B, np.float64)
        cond = np.zeros(B, np.float64)
        nI = np.zeros(B, np.int64)
        lrn = np.zeros(B, np.int32)
        tol_a = np.asarray(tol, dtype=np.float64)
        tol_each = np.ascontiguousarray(np.broadcast_to(tol_a, (B,))) if tol_a.ndim else None
        tol0 = float(tol_a.ravel()[0]) if tol_a.ndim else float(tol_a)
        hp = lambda arr: None if arr is None else arr.ctypes.data  # noqa: E731
        rc = _lib.adef2_solve_batched(self._ctx, B, _ptr(M), _ptr(Bt), hp(a_h), hp(c_h), _ptr(Th),
                                      tol0, hp(tol_each), _ptr(x), hp(iters), hp(status), hp(rel),
                                      hp(cond), hp(nI), hp(lrn))
        self._check(rc)
        return dict(x=x, iters=iters, status=status, relres_true=rel, cond_E=cond, n_inactive=nI,
                    learned=lrn, rc=rc)

    # --- learned enrichment ----------------------------------------------------
    NPARAM = 83200

    def pod(self, X, p: int):
        """POD modes of the snapshot columns of X (N x M)."""
        Xt = _dev(np.asfortranarray(X).ravel(order="F") if not isinstance(X, torch.Tensor)
                  else X.T.contiguous().reshape(-1), torch.float64)
        M = int(X.shape[1])
        Phi = torch.empty(self.n * p, dtype=torch.float64, device="cuda")
        sig = np.zeros(p)
        self._check(_lib.adef2_pod(self._ctx, M, _ptr(Xt), p, _ptr(Phi), sig.ctypes.data), allow=(OK,))
        return Phi.reshape(p, self.n).T, sig

    def set_pod_modes(self, Phi):
        Pt = _dev(np.asfortranarray(Phi).ravel(order="F") if not isinstance(Phi, torch.Tensor)
                  else Phi.T.contiguous().reshape(-1), torch.float64)
        self._check(_lib.adef2_set_pod_modes(self._ctx, int(Phi.shape[1]), _ptr(Pt)), allow=(OK,))

    def set_enrichment(self, Phi, params=None, n_vec: int = 8, tau_learned: float = 1e8):
        """POD modes Phi (N x p) and, optionally, the MLP parameters in one call."""
        Pt = _dev(np.asfortranarray(Phi).ravel(order="F") if not isinstance(Phi, torch.Tensor)
                  else Phi.T.contiguous().reshape(-1), torch.float64)
        pp = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        if pp is not None:
            assert pp.size == self.NPARAM
        self._check(_lib.adef2_set_enrichment(self._ctx, int(Phi.shape[1]), _ptr(Pt),
                                              None if pp is None else pp.ctypes.data, int(n_vec),
                                              float(tau_learned)), allow=(OK,))

    def learned_set_params(self, params: np.ndarray, tau_learned: float = 1e8):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == self.NPARAM
        self._check(_lib.adef2_learned_set_params(self._ctx, p.ctypes.data, float(tau_learned)),
                    allow=(OK,))

    def learned_get_params(self) -> np.ndarray:
        p = np.zeros(self.NPARAM, np.float32)
        self._check(_lib.adef2_learned_get_params(self._ctx, p.ctypes.data), allow=(OK,))
        return p

    def learned_prepare(self, masks, b, xsol, theta, a=None, c=None):
        M = _dev(masks, torch.uint8)
        Bt = _dev(b, torch.float64)
        Xt = _dev(xsol, torch.float64)
        Th = _dev(theta, torch.float32)
        a_h = None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        c_h = None if c is None else np.ascontiguousarray(c, dtype=np.float64)
        hp = lambda arr: None if arr is None else arr.ctypes.data  # noqa: E731
        self._check(_lib.adef2_learned_prepare(self._ctx, int(M.shape[0]), _ptr(M), _ptr(Bt), _ptr(Xt),
                                               _ptr(Th), hp(a_h), hp(c_h)), allow=(OK,))
        self._mtr = int(M.shape[0])

    def learned_loss_grad(self):
        loss = np.zeros(self._mtr)
        grad = np.zeros(self.NPARAM, np.float32)
        self._check(_lib.adef2_learned_loss_grad(self._ctx, loss.ctypes.data, grad.ctypes.data),
                    allow=(OK,))
        return loss, grad

    def learned_train(self, steps: int, lr: float = 1e-3):
        hist = np.zeros(steps)
        self._check(_lib.adef2_learned_train(self._ctx, int(steps), float(lr), hist.ctypes.data),
                    allow=(OK,))
        return hist

    def learned_forward(self, theta):
        Th = _dev(theta, torch.float32)
        out = torch.empty((Th.shape[0], 512), dtype=torch.float32, device="cuda")
        self._check(_lib.adef2_learned_forward(self._ctx, int(Th.shape[0]), _ptr(Th), _ptr(out)),
                    allow=(OK,))
        return out

    def apply_restricted(self, x) -> torch.Tensor:
        xt = _dev(x, torch.float64)
        y = torch.empty_like(xt)
        self._check(_lib.adef2_apply_restricted(self._ctx, _ptr(xt), _ptr(y)), allow=(OK,))
        return y

    def active_set_batched(self, y_d, psi, tau: float = 1e-10, tol: float = 1e-10, max_outer: int = 20):
        """Primal active-set loop for B instances (y_d, psi: B x N)."""
        Yd = _dev(y_d, torch.float64)
        Ps = _dev(psi, torch.float64)
        B = int(Yd.shape[0])
        y = torch.empty_like(Yd)
        masks = torch.empty(Yd.shape, dtype=torch.uint8, device="cuda")
        outer = np.zeros(B, np.int32)
        inner = np.zeros(B, np.int32)
        status = np.zeros(B, np.int32)
        rc = _lib.adef2_active_set_batched(self._ctx, B, _ptr(Yd), _ptr(Ps), float(tau), float(tol),
                                           int(max_outer), _ptr(y), _ptr(masks), outer.ctypes.data,
                                           inner.ctypes.data, status.ctypes.data)
        self._check(rc)
        return dict(y=y, masks=masks, outer=outer, inner_iters=inner, status=status)

    def pod_enrich(self, p: int, tau_safe: float = 1e4):
        """Append the first p held POD modes as safe-merge candidates (p = 0: none)."""
        self._check(_lib.adef2_pod_enrich(self._ctx, int(p), float(tau_safe)), allow=(OK,))

    def prolong_basis(self, Zc, dim: int, n: int, nc: int, tau_sv: float = 1e-10):
        """Coarse modes Zc (nc^dim x r) -> orthonormal fine-grid basis (n^dim x r')."""
        r = int(Zc.shape[1])
        Zt = _colmajor(Zc)
        Nf = n ** dim
        out = torch.empty(Nf * r, dtype=torch.float64, device="cuda")
        ro = _i32(0)
        self._check(_lib.adef2_prolong_basis(self._ctx, int(dim), int(n), int(nc), r, _ptr(Zt), float(tau_sv),
                                             _ptr(out), ctypes.byref(ro)), allow=(OK,))
        return out.reshape(r, Nf).T[:, :ro.value]

    def reference_eigs(self, X0, max_iter: int = 100, tol: float = 1e-8, inner_tol: float = 1e-12):
        """Smallest eigenpairs of the reference operator from the start block X0 (n x r)."""
        r = int(X0.shape[1])
        Xt = _dev(np.asfortranarray(X0, dtype=np.float64).ravel(order="F"), torch.float64)
        Z = torch.empty(self.n * r, dtype=torch.float64, device="cuda")
        lam = np.zeros(r)
        res = np.zeros(r)
        it = _i32(0)
        rc = _lib.adef2_reference_eigs(self._ctx, r, _ptr(Xt), int(max_iter), float(tol), float(inner_tol),
                                       _ptr(Z), lam.ctypes.data, res.ctypes.data, ctypes.byref(it))
        self._check(rc, allow=(OK, W_MAXIT))
        return dict(Z=Z.reshape(r, self.n).T, lam=lam, resid=res, iters=it.value, status=rc)

    def variant(self):
        """(rows_per_thread, w_mode, trial ms) of the last solve."""
        r, wm = _i32(0), _i32(0)
        ms = np.zeros(10, np.float32)
        self._check(_lib.adef2_variant(self._ctx, ctypes.byref(r), ctypes.byref(wm), ms.ctypes.data),
                    allow=(OK,))
        return r.value, wm.value, ms

    def update_variant(self):
        """(warp-specialised, tiles per block, trial ms [per tile, warp-
        specialised]) of the last solve's update kernel."""
        ws, tpb = _i32(0), _i32(0)
        ms = np.zeros(2, np.float32)
        self._check(_lib.adef2_update_variant(self._ctx, ctypes.byref(ws), ctypes.byref(tpb), ms.ctypes.data),
                    allow=(OK,))
        return ws.value, tpb.value, ms

    def op_variant(self):
        """(fused, tile rows, trial ms [two passes, fused at 2 / 4 / 8 x the
        stencil reach with one instance per block, the same with four],
        instances per block) of the last solve."""
        f, rows, grp = _i32(0), _i32(0), _i32(0)
        ms = np.zeros(7, np.float32)
        self._check(_lib.adef2_operator_variant(self._ctx, ctypes.byref(f), ctypes.byref(rows),
                                                ctypes.byref(grp), ms.ctypes.data), allow=(OK,))
        return f.value, rows.value, ms, grp.value

    def coarse_info(self):
        k = max(self.k, 1)
        E = np.zeros(k * k)
        kept = np.zeros(k, np.int32)
        ke, cond = _i32(0), _f64(0.0)
        self._check(_lib.adef2_coarse_info(self._ctx, E.ctypes.data, kept.ctypes.data,
                                           ctypes.byref(ke), ctypes.byref(cond)), allow=(OK,))
        kk = ke.value
        Em = E.reshape(k, k, order="F")[:kk, :kk] if self.k else np.zeros((0, 0))
        return Em, kept[: self.k], kk, cond.value

    def stats(self) -> dict:
        s = Stats()
        self._check(_lib.adef2_get_stats(self._ctx, ctypes.byref(s)), allow=(OK,))
        return {s.name[i].decode(): dict(launches=s.launches[i], ms=s.total_ms[i],
                                         alg_bytes=s.alg_bytes[i]) for i in range(s.n_kernels)}

    def pod_iters(self) -> int:
        """Subspace iterations of the last pod() (0: direct eigensolver)."""
        s = Stats()
        self._check(_lib.adef2_get_stats(self._ctx, ctypes.byref(s)), allow=(OK,))
        return int(s.pod_iters)

    def polls(self) -> int:
        """Host polls of the device convergence state since the last reset."""
        s = Stats()
        self._check(_lib.adef2_get_stats(self._ctx, ctypes.byref(s)), allow=(OK,))
        return int(s.polls)

    def reset_stats(self):
        self._check(_lib.adef2_reset_stats(self._ctx), allow=(OK,))


def status_name(code: int) -> str:
    return {OK: "ok", E_ARG: "e_arg", E_STATE: "e_state", E_HIP: "e_hip", E_NOMEM: "e_nomem",
            E_NOT_SPD: "e_not_spd", E_UNSUPPORTED: "e_unsupported", E_NOCONV: "e_noconv",
            W_FALLBACK: "w_fallback",
            W_MAXIT: "w_maxit", W_STAGNATED: "w_stagnated"}.get(code, str(code))


__all__ = ["Solver", "Opts", "default_opts", "Adef2Error", "EXPORTS", "LIB_PATH", "status_name"]
