"""The allocation-free set-up entry point (ugkwp_set_material_noalloc) against
ugkwp_set_material, through the C ABI: two calls in a row on one GPU (the
second on a smaller mesh, so the shared static staging array holds the first
call's longer contents), each compared with the allocating call on a context
of the same problem, and the runs that follow compared with each other and
with the oracle."""
import ctypes as C
import sys

import numpy as np
import pytest

import oracle
from paper_2312_16981_amd import ugkwp
from paper_2312_16981_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t)) if a is not None else None


def abi_set_material(fn, ctx, prob):
    cv, T0, Tr0 = _f64(prob.cv), _f64(prob.T0), _f64(prob.Tr0)
    pin = np.ascontiguousarray(prob.pinned, dtype=np.uint8)
    return getattr(ugkwp.load(), fn)(ctx.h, _ptr(cv), _ptr(T0), _ptr(Tr0), _ptr(pin, C.c_uint8))


def check_pair(prob, nsteps):
    say(f"[noalloc] {prob.name} ncell={prob.ncell} G={prob.G}")
    a = ugkwp.from_problem(prob)
    b = ugkwp.from_problem(prob)
    # start both from another state, then set the problem's material through each call
    hot = prob.with_(T0=np.full(prob.ncell, 0.3), Tr0=np.full(prob.ncell, 0.25))
    for c in (a, b):
        c.set_material(hot.cv, hot.T0, hot.Tr0, hot.pinned)
        c.step(2)
    assert abi_set_material("ugkwp_set_material", a, prob) == 0
    assert abi_set_material("ugkwp_set_material_noalloc", b, prob) == 0, ugkwp.load().ugkwp_last_error(b.h)
    for x, y in zip(a.get_fields(), b.get_fields()):
        assert np.array_equal(x, y)
    assert a.get_counters() == b.get_counters() == (0, 0) and b.pool_size() == 0
    a.step(nsteps)
    b.step(nsteps)
    for x, y in zip(a.get_fields(), b.get_fields()):
        assert np.max(np.abs(x - y)) <= 1e-12 * max(np.max(np.abs(y)), 1e-300)
    assert a.get_counters() == b.get_counters() and a.pool_size() == b.pool_size()
    sim = oracle.Sim(prob)
    sim.step(nsteps)
    rho, T, _ = b.get_fields()
    ro, To, _ = sim.fields()
    assert np.max(np.abs(rho - ro)) <= 1e-10 * np.max(np.abs(ro))
    assert np.max(np.abs(T - To)) <= 1e-10 * np.max(To)


def test_noalloc_set_material_matches_allocating_call():
    check_pair(W.c5_lognormal(n=48, G=6, w_ref=2e-4, pool_cap=1 << 21, dt=2e-2), 4)
    check_pair(W.c1_marshak_like(), 6)


def test_noalloc_set_material_rejects_a_batch():
    probs = [W.c1_marshak_like().with_(seed=k) for k in range(2)]
    ctx = ugkwp.from_batch(probs)
    rc = abi_set_material("ugkwp_set_material_noalloc", ctx, probs[0])
    assert rc == ugkwp.EINVAL
