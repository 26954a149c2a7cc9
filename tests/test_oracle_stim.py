"""Pins of the oracle's stimulated-emission opacity factor (Sec. 3.3's
gamma0 (1 - e^{-h nu/kT}) / (h nu)^3): sigma(nu, T) = kappa nu^-p (1 - e^{-nu/T}),
a group's opacity Simpson's mean of that over the group (the rule the base
method uses for nu^-p), the particles at T^n, and the source iteration's
coefficients from its iterate T^k (Algorithm 2)."""
import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from paper_2312_16981_amd import workloads as W
from test_oracle_physics import phi_ref, zero_d_problem


def simpson_stim(e, T):
    nm = 0.5 * (e[:-1] + e[1:])

    def f(nu):
        return nu ** -3.0 * (1.0 - np.exp(-nu / T))
    return (f(e[:-1]) + 4 * f(nm) + f(e[1:])) / 6.0


def test_zero_d_step_solves_backward_euler_with_the_factor_at_the_new_temperature():
    dt = 0.02
    p = zero_d_problem(dt, T0=0.8, Tr=0.2).with_(opacity_stim=1)
    s = oracle.Sim(p)
    rho_n, T_n, _ = s.fields()
    s.step(1)
    rho, T, _ = s.fields()
    e = p.nu_edges

    def parts(Tn1):
        sig = p.kappa[0] * simpson_stim(e, Tn1)
        ph = np.array([phi_ref(Tn1, e[g], e[g + 1]) for g in range(3)])
        return sig, sig * dt, ph

    def f(Tn1):
        sig, lam, ph = parts(Tn1)
        r = (rho_n[0] + lam * ph) / (1 + lam)
        return 0.7 * (Tn1 - T_n[0]) - np.sum(dt * sig * (r - ph))
    Tref = brentq(f, 1e-3, 2.0, xtol=1e-16, rtol=1e-15)
    sig, lam, ph = parts(Tref)
    assert T[0] == pytest.approx(Tref, rel=1e-12)
    np.testing.assert_allclose(rho[0], (rho_n[0] + lam * ph) / (1 + lam), rtol=1e-11)
    # the factor matters at this temperature (else the pin would not see it)
    assert np.min(simpson_stim(e, Tref) / simpson_stim(e, 1e-9)) < 0.5


def cold(stim, **kw):
    """Every nu / T above 37 throughout: 1 - e^{-nu/T} rounds to 1."""
    p = dict(dt=1e-3, steps=0, w_ref=1e-27, pool_cap=1 << 20, name="cold", numin=0.5, numax=10.0,
             T0=1e-3, Tb=0.012, opacity_stim=stim)
    p.update(kw)
    return W.slab(40, 6, lambda x: np.full_like(x, 2.0), **p)


def test_cold_medium_is_the_base_method_bit_for_bit():
    a, b = oracle.Sim(cold(0)), oracle.Sim(cold(1))
    for sim in (a, b):
        sim.step(6)
    assert a.pool()["x"].size > 100
    for u, v in zip(a.fields(), b.fields()):
        assert np.array_equal(u, v)
    for k in ("x", "nu", "w"):
        assert np.array_equal(a.pool()[k], b.pool()[k])


def hot(stim, **kw):
    p = dict(dt=2e-3, steps=0, w_ref=2e-5, pool_cap=1 << 20, name="hot", T0=0.5, Tb=1.0,
             opacity_stim=stim)
    p.update(kw)
    return W.slab(50, 8, lambda x: np.full_like(x, 5.0), **p)


def test_hot_medium_is_thinner_and_conserves_energy():
    a, b = oracle.Sim(hot(0)), oracle.Sim(hot(1))
    for n in range(8):
        a.step(1)
        b.step(1)
        d = b.diag()
        assert abs(d["residual"]) <= 1e-12 * abs(d["e_end"]), n
    # (1 - e^{-nu/T}) < 1 lowers sigma: more particles survive their flights
    assert b.pool()["x"].size > a.pool()["x"].size


def test_equilibrium_between_mirrors_stays_put():
    p = zero_d_problem(0.05, T0=0.4, Tr=0.4).with_(opacity_stim=1, T_power=0.5, w_ref=1e30)
    s = oracle.Sim(p)
    rho0, T0, _ = s.fields()
    s.step(5)
    rho, T, _ = s.fields()
    np.testing.assert_allclose(T, T0, rtol=1e-14)
    np.testing.assert_allclose(rho, rho0, rtol=1e-14)


def test_recording_refuses_the_factor_and_bad_values_are_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.Sim(hot(1)).record(True)
    with pytest.raises(Exception):
        oracle.Sim(hot(2))
