"""The no-allocation compaction (adef2_compact_noalloc, static scratch)
against adef2_compact and the oracle: two calls in a row on one context,
the second with a smaller mask; bit-exact."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


def test_compact_noalloc_matches_compact(lib):
    big = gen.c2_workload(n=511, k=0, B=1).instances[0].mask
    small = gen.c1_workload(n=63, k=0).instances[0].mask
    s = lib.Solver()
    for mask in (big, small):
        print(f"[case] compact_noalloc n={mask.size}", flush=True)
        I_r, g_r, n_r = s.compact(mask)
        I_n, g_n, n_n, cnt = s.compact_noalloc(mask)
        assert n_n == n_r and int(cnt.item()) == n_r
        np.testing.assert_array_equal(I_n.cpu().numpy(), I_r.cpu().numpy())
        np.testing.assert_array_equal(g_n.cpu().numpy(), g_r.cpu().numpy())
        I_o, g_o, n_o = oracle.compact(mask)
        assert n_n == n_o
        np.testing.assert_array_equal(I_n.cpu().numpy(), I_o)
        np.testing.assert_array_equal(g_n.cpu().numpy(), g_o)
    # empty mask and the size limit
    I_n, g_n, n_n, cnt = s.compact_noalloc(np.zeros(0, np.uint8))
    assert n_n == 0 and int(cnt.item()) == 0
