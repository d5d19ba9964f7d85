"""The C/OpenMP build of the oracle's A-DEF2 loop (the CPU baseline) against
the Python oracle: same iterations (up to one, from the order of OpenMP
reductions) and the same solution, with and without deflation, on one and
several threads."""
import numpy as np
import pytest

import gen
import oracle
from oracle import cpu


@pytest.mark.parametrize("k", [16, 0])
@pytest.mark.parametrize("threads", [1, 4])
def test_c_oracle_matches_python_oracle(k, threads):
    w = gen.c1_workload(n=63, k=k)
    S = w.op.S()
    inst = w.instances[0]
    I, _, _ = oracle.compact(inst.mask)
    S_II, _ = oracle.restricted_operator(S, I)
    Zo, _ = oracle.restricted_basis(w.Z, I)
    ref = oracle.solve_instance(S, w.Z, inst.mask, inst.b, 1e-10)
    r = cpu.adef2(S_II, inst.b[I], Zo, 1e-10, threads=threads)
    assert r.converged and not r.fallback
    assert abs(r.iters - ref.iters) <= 1
    assert oracle.rel_err(r.x, ref.x[I]) <= 1e-10


def test_c_oracle_factored_operator_and_zero_rhs():
    w = gen.c2_workload(n=31, k=8, B=1)
    op = w.op
    inst = w.instances[0]
    spec = ("factored", op.A, op.alpha, op.shift)
    I, _, _ = oracle.compact(inst.mask)
    F, _ = oracle.restricted_operator(spec, I)
    Zo, _ = oracle.restricted_basis(w.Z, I)
    ref = oracle.solve_instance(spec, w.Z, inst.mask, inst.b, 1e-10)
    r = cpu.adef2(F, inst.b[I], Zo, 1e-10, threads=2)
    assert abs(r.iters - ref.iters) <= 1
    assert oracle.rel_err(r.x, ref.x[I]) <= 1e-9
    z = cpu.adef2(F, np.zeros(len(I)), Zo, 1e-10)
    assert z.iters == 0 and np.all(z.x == 0.0)
