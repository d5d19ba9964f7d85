"""Argument checks of the entry points around the hot path: each bad call
returns an error code (raised by the binding) before any kernel runs, and
the context stays usable."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


def test_bad_arguments_are_rejected(lib):
    print("[case] argument errors of active_set / pod_enrich / prolong / eigs", flush=True)
    w = gen.ocp_2d_sym(n=15, B=2)
    Z = gen.sine_modes_2d(15, 4)[0]
    s = lib.Solver(precision=lib.FP64)
    with pytest.raises(lib.Adef2Error):                 # before set_reference
        s.active_set_batched(w.y_d, w.psi)
    with pytest.raises(lib.Adef2Error):
        s.pod_enrich(2)
    with pytest.raises(lib.Adef2Error):
        s.reference_eigs(np.ones((w.op.N, 2)))
    s.set_reference_factored(w.op.A, w.op.alpha, w.op.shift, Z)
    with pytest.raises(lib.Adef2Error):
        s.active_set_batched(w.y_d, w.psi, max_outer=0)
    with pytest.raises(lib.Adef2Error):
        s.active_set_batched(w.y_d, w.psi, tol=0.0)
    with pytest.raises(lib.Adef2Error):
        s.pod_enrich(-1)
    with pytest.raises(lib.Adef2Error):
        s.pod_enrich(61)                                # k + p > 64
    with pytest.raises(lib.Adef2Error):
        s.reference_eigs(np.ones((w.op.N, 65)))
    with pytest.raises(lib.Adef2Error):
        s.reference_eigs(np.ones((w.op.N, 2)), max_iter=0)
    with pytest.raises(lib.Adef2Error):
        s.prolong_basis(np.ones((49, 2)), dim=4, n=15, nc=7)
    with pytest.raises(lib.Adef2Error):
        s.prolong_basis(np.ones((49, 2)), dim=2, n=15, nc=7, tau_sv=-1.0)
    with pytest.raises(lib.Adef2Error):
        lib.Solver(precision=lib.FP64, ritz_keep=-1)
    # still usable
    out = s.active_set_batched(w.y_d, w.psi)
    assert np.all(out["status"] == 0)
    s.close()
