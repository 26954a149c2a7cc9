"""Pins of the oracle's linearized source iteration: each sweep takes the new
temperature's emission as phi^k + phi'(T^k) (T^{k+1} - T^k) and solves every
cell's energy balance for T^{k+1} (a local Newton step). Its fixed point is the
literal iteration's (Eq. macroSysFinal, Appendix B); it also converges where
the literal one cannot, when Sum_g dt sigma_g phi'_g / (eps^2 C_v (1 + lambda_g))
exceeds 1 (stiff material coupling)."""
import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from paper_2312_16981_amd import workloads as W
from test_oracle_physics import phi_ref, simpson_sigma, zero_d_problem

LIN = 8


def stiff(lin, dt=0.5, cv=1e-3):
    p = zero_d_problem(dt, kap=(200.0, 50.0, 400.0), T0=0.5, Tr=0.1, cv=cv)
    return p.with_(flags=p.flags | (LIN if lin else 0), si_max_iters=200)


def test_stiff_zero_d_step_converges_to_the_backward_euler_root():
    p = stiff(True)
    s = oracle.Sim(p)
    rho_n, T_n, _ = s.fields()
    s.step(1)
    rho, T, _ = s.fields()
    e, dt, cv = p.nu_edges, p.dt, p.cv[0]
    sig = p.kappa[0] * simpson_sigma(e)
    lam = sig * dt

    def ph(Tn1):
        return np.array([phi_ref(Tn1, e[g], e[g + 1]) for g in range(3)])

    def f(Tn1):
        r = (rho_n[0] + lam * ph(Tn1)) / (1 + lam)
        return cv * (Tn1 - T_n[0]) - np.sum(dt * sig * (r - ph(Tn1)))
    Tref = brentq(f, 1e-3, 2.0, xtol=1e-16, rtol=1e-15)
    assert T[0] == pytest.approx(Tref, rel=1e-12)
    np.testing.assert_allclose(rho[0], (rho_n[0] + lam * ph(Tref)) / (1 + lam), rtol=1e-11)
    # the case is stiff: the literal iteration's contraction factor is far above 1
    h = 1e-6 * Tref
    dph = (ph(Tref + h) - ph(Tref - h)) / (2 * h)
    J = np.sum(dt * sig * dph / (cv * (1 + lam)))
    assert J > 10
    assert s.diag()["sweeps"] <= 12          # a Newton step per sweep


def test_literal_iteration_fails_on_the_stiff_case():
    with pytest.raises(oracle.OracleError):
        oracle.Sim(stiff(False)).step(1)


def test_same_fixed_point_as_the_literal_iteration():
    """From one state, one step of each variant ends on the same fields (both
    converged to 1e-13), on a slab with a temperature-dependent opacity and on a
    2-D medium with pinned cells."""
    probs = [W.slab(60, 8, lambda x: np.full_like(x, 0.3), dt=2e-3, steps=0, w_ref=2e-5,
                    pool_cap=1 << 20, name="slab_q", T_power=0.5),
             W.c3_lattice(n=16, G=4, w_ref=1e-3, pool_cap=1 << 20)]
    for p in probs:
        warm = oracle.Sim(p)
        warm.step(5)
        st = warm.state()
        out = []
        for lin in (False, True):
            s = oracle.Sim(p.with_(flags=p.flags | (LIN if lin else 0)))
            s.restore(st)
            s.step(1)
            out.append((s.fields(), s.diag()))
        (fa, da), (fb, db) = out
        np.testing.assert_allclose(fb[1], fa[1], rtol=1e-11)
        np.testing.assert_allclose(fb[0], fa[0], rtol=1e-10, atol=1e-12 * np.abs(fa[0]).max())
        assert np.array_equal(fb[2], fa[2])  # the particles do not see the iteration
        assert db["sweeps"] <= da["sweeps"]


def test_energy_conservation():
    p = stiff(True, dt=0.05, cv=0.01).with_(bc=[W.BC_PLANCK, W.BC_VACUUM, 0, 0])
    s = oracle.Sim(p)
    for n in range(10):
        s.step(1)
        d = s.diag()
        assert abs(d["residual"]) <= 1e-12 * abs(d["e_end"]), n


def test_adjoint_of_a_linearized_run_matches_the_literal_one():
    """The adjoint differentiates the fixed point, which both iterations share:
    recording a run made with the linearized sweep gives the literal run's
    gradient (to the iterations' tolerance)."""
    p = W.c5_lognormal(n=10, G=4, w_ref=2e-4, pool_cap=1 << 20, dt=2e-3)
    V = (p.x1 - p.x0) / p.nx * (p.y1 - p.y0) / p.ny
    grads = []
    for fl in (0, LIN):
        s = oracle.Sim(p.with_(flags=fl))
        s.record(True)
        s.step(6)
        grads.append(s.adjoint(V * p.cv))
    ga, gb = grads
    assert np.abs(ga).max() > 0
    np.testing.assert_allclose(gb, ga, rtol=1e-8, atol=1e-10 * np.abs(ga).max())
