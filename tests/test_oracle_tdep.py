"""Pins of the oracle's temperature-dependent opacity sigma(nu, T) = kappa nu^-p T^-q
(Sec. 3.1 takes sigma0 / (nu^3 sqrt(T)), q = 1/2): the particles and the wave
split of a step see T^n, and the source iteration recomputes sigma, lambda and
the face coefficients from its iterate in every sweep (Algorithm 2), so that a
converged step solves the backward-Euler system with sigma(T^{n+1})."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.optimize import brentq

import oracle
from paper_2312_16981_amd import workloads as W
from test_oracle_physics import phi_ref, simpson_sigma, zero_d_problem

Q = 0.5


def test_zero_d_step_solves_backward_euler_with_sigma_at_the_new_temperature():
    dt = 0.02
    p = zero_d_problem(dt).with_(T_power=Q)
    s = oracle.Sim(p)
    rho_n, T_n, _ = s.fields()
    s.step(1)
    rho, T, _ = s.fields()
    e = p.nu_edges
    S = simpson_sigma(e)

    def parts(Tn1):
        sig = p.kappa[0] * Tn1 ** -Q * S
        lam = sig * dt
        ph = np.array([phi_ref(Tn1, e[g], e[g + 1]) for g in range(3)])
        return sig, lam, ph

    def f(Tn1):
        sig, lam, ph = parts(Tn1)
        r = (rho_n[0] + lam * ph) / (1 + lam)
        return 0.7 * (Tn1 - T_n[0]) - np.sum(dt * sig * (r - ph))
    Tref = brentq(f, 1e-3, 2.0, xtol=1e-16, rtol=1e-15)
    sig, lam, ph = parts(Tref)
    rref = (rho_n[0] + lam * ph) / (1 + lam)
    assert T[0] == pytest.approx(Tref, rel=1e-12)
    np.testing.assert_allclose(rho[0], rref, rtol=1e-12)
    # and the opacity did change over the step (else the pin would not see q)
    assert abs(T[0] / T_n[0] - 1) > 1e-2


def test_zero_d_first_order_convergence_to_ode():
    e = np.array([0.05, 0.3, 1.0, 5.0])
    kap = np.array([3.0, 0.5, 20.0])
    S = simpson_sigma(e)
    cv, t_end = 0.7, 0.2

    def rhs(t, y):
        r, T = y[:3], y[3]
        sig = kap * T ** -Q * S
        ph = np.array([phi_ref(T, e[g], e[g + 1]) for g in range(3)])
        return np.concatenate([sig * (ph - r), [np.sum(sig * (r - ph)) / cv]])
    r0 = np.array([phi_ref(0.1, e[g], e[g + 1]) for g in range(3)])
    sol = solve_ivp(rhs, (0, t_end), np.concatenate([r0, [0.5]]), method="Radau", rtol=1e-12, atol=1e-14)
    Tode = sol.y[3, -1]
    errs = []
    for nstep in (10, 20, 40, 80):
        s = oracle.Sim(zero_d_problem(t_end / nstep).with_(T_power=Q))
        s.step(nstep)
        errs.append(abs(s.fields()[1][0] - Tode))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 1.0) < 0.1), orders


def marshak_like(q=Q, nx=60, G=8, **kw):
    p = dict(dt=2e-3, steps=0, w_ref=2e-5, pool_cap=1 << 20, name="marshak_like", T_power=q)
    p.update(kw)
    return W.slab(nx, G, lambda x: np.full_like(x, 0.3), **p)


def test_energy_conservation_and_equilibrium():
    s = oracle.Sim(marshak_like())
    for n in range(15):
        s.step(1)
        d = s.diag()
        assert abs(d["residual"]) <= 1e-12 * abs(d["e_end"]), n
    # uniform equilibrium between mirrors stays put, whatever sigma(T)
    p = zero_d_problem(0.05, T0=0.4, Tr=0.4).with_(T_power=Q, w_ref=1e30)
    s = oracle.Sim(p)
    rho0, T0, _ = s.fields()
    s.step(5)
    rho, T, _ = s.fields()
    np.testing.assert_allclose(T, T0, rtol=1e-14)
    np.testing.assert_allclose(rho, rho0, rtol=1e-14)


def test_particles_see_the_step_temperature():
    """q = 0 is the base method bit for bit; with q > 0 the cold cells are
    thicker (sigma grows as T^-q), so fewer particles survive the first steps."""
    a = oracle.Sim(marshak_like(q=0.0))
    b = oracle.Sim(marshak_like(q=0.0, T_power=0.0))
    c = oracle.Sim(marshak_like())
    for sim in (a, b, c):
        sim.step(6)
    for u, v in zip(a.fields(), b.fields()):
        assert np.array_equal(u, v)
    assert c.pool()["x"].size < a.pool()["x"].size


def test_recording_refuses_temperature_dependent_opacity():
    with pytest.raises(oracle.OracleError):
        oracle.Sim(marshak_like()).record(True)
