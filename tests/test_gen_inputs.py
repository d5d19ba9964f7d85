"""Checks of the synthetic inputs: operators, reference modes, masks."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import gen


def test_sine_modes_are_eigenvectors_and_lowest():
    n, k = 9, 12
    w = gen.c1_workload(n=n, k=k)
    S = w.op.S().toarray()
    Z = w.Z
    np.testing.assert_allclose(Z.T @ Z, np.eye(k), atol=1e-13)
    h = 1.0 / (n + 1)
    lam = 1e-2 * w.meta["sigma_sum"] ** 2 / h ** 2 + h * h
    for j in range(k):
        r = S @ Z[:, j] - lam[j] * Z[:, j]
        assert np.linalg.norm(r) <= 1e-13 * np.abs(S).max()
    ev = np.linalg.eigvalsh(S)
    np.testing.assert_allclose(np.sort(lam), ev[:k], rtol=1e-11)


def test_sine_mode_tie_break_is_lexicographic():
    _, pairs, sig = gen.sine_modes_2d(63, 17)
    # the 16th/17th modes are the degenerate pair (1,5)/(5,1): keep (1,5) first
    assert pairs[15] == (1, 5) and pairs[16] == (5, 1)
    assert sig[15] == sig[16]


def test_c2_reference_modes_small_grid():
    w = gen.c2_workload(n=31, k=6, B=2)
    S = w.op.S()
    Z = w.Z
    np.testing.assert_allclose(Z.T @ Z, np.eye(6), atol=1e-10)
    ev = np.linalg.eigvalsh(S.toarray())
    rq = np.array([Z[:, j] @ (S @ Z[:, j]) for j in range(6)])
    np.testing.assert_allclose(rq, ev[:6], rtol=1e-8)
    assert abs(S - S.T).max() <= 1e-12 * abs(S).max()


def test_c3_operator_family_shares_eigenvectors():
    op, KG = gen.c3_operator(n=15)
    Z = gen._low_symmetric(KG, 4)
    for a in (1.0, 2.5):
        S = op.S(a=a)
        for j in range(4):
            v = S @ Z[:, j]
            lam = Z[:, j] @ v
            assert np.linalg.norm(v - lam * Z[:, j]) <= 1e-9 * abs(lam)


@pytest.mark.parametrize("rho", [0.0, 0.1, 0.37, 1.0])
def test_mask_exact_fraction(rho):
    f = gen.sinusoid_field(20, 3)
    m = gen.mask_top_fraction(f, rho)
    assert m.dtype == np.uint8 and int(m.sum()) == math.floor(rho * 400)
    if 0 < rho < 1:
        assert f[m == 1].min() >= f[m == 0].max()


def test_c3_masks_nested():
    f = gen.sinusoid_field(15, 301)
    m1 = gen.mask_top_fraction(f, 0.2)
    m2 = gen.mask_top_fraction(f, 0.5)
    assert np.all(m2[m1 == 1] == 1)


def test_csr_canonical():
    w = gen.c1_workload(n=7, k=0)
    S = w.op.S()
    assert S.indptr.dtype == np.int64 and S.indices.dtype == np.int32
    for i in range(S.shape[0]):
        cols = S.indices[S.indptr[i]:S.indptr[i + 1]]
        assert np.all(np.diff(cols) > 0)


def test_mlp_params_match_oracle_init_layout():
    from oracle import learned as OL
    for seed in (0, 5):
        prm = OL.mlp_init(seed)
        flat = np.concatenate([prm["W1"].ravel(), prm["b1"], prm["W2"].ravel(), prm["b2"],
                               prm["W3"].ravel(), prm["b3"]])
        np.testing.assert_array_equal(gen.mlp_params(seed), flat)
        assert flat.size == 83200


def test_c2_family_members():
    n = 31
    th = gen.c2_thetas(5, 3, spread_rho=True)
    assert np.allclose(th[:, 0], np.linspace(0, 1, 5))
    for t in th:
        inst = gen.c2_family_instance(n, t)
        assert inst.mask.sum() == int(np.floor((0.10 + 0.30 * t[0]) * n * n))
        assert np.argmax(inst.b) == np.argmax(gen.gaussian_bump(n, (0.2 + 0.6 * t[1], 0.2 + 0.6 * t[2])))
    # phase 0 and phase 1 (a full period) give the same mask
    a = gen.c2_family_instance(n, [0.5, 0.5, 0.5, 0.0]).mask
    b = gen.c2_family_instance(n, [0.5, 0.5, 0.5, 1.0]).mask
    assert (a != b).sum() <= 2
