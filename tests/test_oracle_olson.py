"""Pins of the oracle's material models of the Olson problems (Sec. 3.4-3.5):
Olson's temperature-dependent heat capacity (Eq. cvolson), a volumetric
radiation source Q(x) switched off at a given time, and a tabulated
opacity sigma(nu, T) per material.  Each is checked against something the
oracle does not compute itself: the Saha-type identity that alpha solves and
a finite difference of it, the bracket of Eq. cvolson as the derivative of
(T + chi)(1 + alpha), an independent implicit 0-D solve, closed forms of a
transparent box, energy ledgers, and a table built from the power law, whose
log-log interpolation is exact, reproducing the analytic opacity run."""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.optimize import brentq

import oracle
from paper_2312_16981_amd import workloads as W
from test_oracle_physics import phi_ref, simpson_sigma, zero_d_problem


# ---------------------------------------------------------------- Olson's heat capacity
def _alpha_paper(T, chi):
    """alpha and dalpha/dT as printed, in the form e^{-chi/T} (sqrt(1 + 4 e^{chi/T}) - 1)/2
    (fine for chi/T below a few hundred)."""
    E = np.exp(chi / T)
    r = np.sqrt(1.0 + 4.0 * E)
    a = 0.5 / E * (r - 1.0)
    return a, chi / T ** 2 * (a - 1.0 / r)


@pytest.mark.parametrize("chi", [0.1, 0.3, 1e-3])
def test_alpha_solves_saha_identity_and_its_derivative(chi):
    """alpha^2 = e^{-chi/T} (1 - alpha) (alpha is the root in (0, 1) of that quadratic),
    and the returned derivative agrees with a Richardson central difference."""
    for T in np.geomspace(1e-3, 50.0, 37):
        a, da = oracle.olson_alpha(T, chi)
        assert 0.0 <= a < 1.0
        E = np.exp(-chi / T)
        assert abs(a * a - E * (1.0 - a)) <= 4e-15 * max(a * a, E * (1 - a), 1e-300) + 1e-300
        h = 1e-3 * T / max(1.0, chi / T)
        d1 = (oracle.olson_alpha(T + h, chi)[0] - oracle.olson_alpha(T - h, chi)[0]) / (2 * h)
        d2 = (oracle.olson_alpha(T + h / 2, chi)[0] - oracle.olson_alpha(T - h / 2, chi)[0]) / h
        dr = (4 * d2 - d1) / 3
        assert abs(da - dr) <= 1e-8 * abs(da) + 2e-15 * a / h, (T, da, dr)   # + rounding of the difference
        if chi / T < 300:
            ap, dap = _alpha_paper(T, chi)
            assert a == pytest.approx(ap, rel=1e-12, abs=1e-300)
            assert da == pytest.approx(dap, rel=1e-9, abs=1e-280)
    # limits: fully ionised when hot, neutral when cold
    assert oracle.olson_alpha(1e6, chi)[0] == pytest.approx((np.sqrt(5) - 1) / 2, rel=1e-6)
    assert oracle.olson_alpha(chi / 800.0, chi)[0] < 1e-170


def _olson_sim(nx=4, H=(0.1, 0.5, 0.0, 0.1), chi=(0.1, 0.3, 0.0, 0.1), cv=0.7):
    p = W.slab(nx, 3, lambda x: np.ones_like(x), dt=1e-2, steps=0, w_ref=1e-3)
    return p.with_(cv=np.full(nx, cv), olson_H=np.asarray(H, float), olson_chi=np.asarray(chi, float))


def test_heat_capacity_is_the_derivative_of_the_ionisation_energy():
    """The bracket of Eq. cvolson is d/dT [(T + chi)(1 + alpha)]: C_v(T) / H against a
    central difference of that product; cells with H = 0 keep their C_v."""
    p = _olson_sim()
    s = oracle.Sim(p)

    def u(T, chi):
        return (T + chi) * (1.0 + oracle.olson_alpha(T, chi)[0])
    for i, (H, chi) in enumerate(zip(p.olson_H, p.olson_chi)):
        for T in (0.01, 0.05, 0.1, 0.37, 2.0):
            cv = s.heat_capacity(i, T)
            if H == 0.0:
                assert cv == 0.7
                continue
            h = 1e-4 * T
            d1 = (u(T + h, chi) - u(T - h, chi)) / (2 * h)
            d2 = (u(T + h / 2, chi) - u(T - h / 2, chi)) / h
            assert cv / H == pytest.approx((4 * d2 - d1) / 3, rel=1e-8)


def test_material_energy_integrates_the_heat_capacity():
    """U(T2) - U(T1) equals the integral of C_v by adaptive quadrature, U(T) -> 0 as
    T -> 0, and constant-C_v cells have U = C_v T."""
    p = _olson_sim()
    s = oracle.Sim(p)
    for i in range(4):
        assert s.material_energy(i, 1e-9) <= 1e-8 * max(p.olson_H[i], 0.7)
        for T1, T2 in [(0.005, 0.02), (0.02, 0.3), (0.3, 2.0), (0.05, 0.051)]:
            ref, err = quad(lambda t: s.heat_capacity(i, t), T1, T2, epsabs=0, epsrel=1e-13, limit=200)
            got = s.material_energy(i, T2) - s.material_energy(i, T1)
            assert got == pytest.approx(ref, rel=1e-11), (i, T1, T2)
        if p.olson_H[i] == 0.0:
            assert s.material_energy(i, 0.37) == 0.7 * 0.37


def test_bad_heat_capacity_input_is_refused():
    with pytest.raises(oracle.OracleError):
        oracle.Sim(_olson_sim(H=(0.1, -1.0, 0.0, 0.1)))
    with pytest.raises(oracle.OracleError):
        oracle.Sim(_olson_sim(chi=(0.1, np.nan, 0.0, 0.1)))


def _u_olson(T, H, chi):
    """H [T (1 + alpha) + chi alpha] with alpha in the printed form."""
    al, _ = _alpha_paper(T, chi)
    return H * (T * (1.0 + al) + chi * al)


@pytest.mark.parametrize("linearized,T0,Tr,c,eps", [(False, 0.3, 0.6, 1.0, 1.0), (True, 0.3, 0.6, 1.0, 1.0),
                                                    (False, 0.01, 0.3, 1.0, 1.0), (True, 0.01, 0.3, 1.0, 1.0),
                                                    (False, 0.05, 0.3, 2.0, 0.5), (True, 0.05, 0.3, 2.0, 0.5)])
def test_zero_d_step_solves_implicit_equation_with_olson_heat_capacity(linearized, T0, Tr, c, eps):
    """One cell between mirrors: a converged step solves U(T') - U(T^n) =
    dt sum_g sigma_g (rho'_g - phi_g(T')), rho' = (rho^n + lambda phi(T'))/(1 + lambda),
    with U = H [T (1 + alpha) + chi alpha] of Eq. cvolson's heat capacity (independent
    root find), from a warm and from Olson's cold start."""
    dt, H, chi = 0.02, 0.1, 0.1
    p = zero_d_problem(dt, T0=T0, Tr=Tr).with_(olson_H=np.array([H]), olson_chi=np.array([chi]), c=c, eps=eps,
                                               flags=W.FLAG_SI_LINEARIZED if linearized else 0)
    s = oracle.Sim(p)
    rho_n, T_n, _ = s.fields()
    s.step(1)
    rho, T, _ = s.fields()
    e = p.nu_edges
    sig = p.kappa[0] * simpson_sigma(e)
    lam = c * sig * dt / eps ** 2

    def f(Tn1):
        ph = np.array([phi_ref(Tn1, e[g], e[g + 1], c=c) for g in range(3)])
        r = (rho_n[0] + lam * ph) / (1 + lam)
        return _u_olson(Tn1, H, chi) - _u_olson(T_n[0], H, chi) - np.sum(dt / eps ** 2 * sig * (r - ph))
    Tref = brentq(f, 1e-3, 2.0, xtol=1e-16, rtol=1e-15)
    ph = np.array([phi_ref(Tref, e[g], e[g + 1], c=c) for g in range(3)])
    assert T[0] == pytest.approx(Tref, rel=1e-11)
    np.testing.assert_allclose(rho[0], (rho_n[0] + lam * ph) / (1 + lam), rtol=1e-11)
    # a constant C_v = H lands elsewhere: the test sees the ionisation terms
    s2 = oracle.Sim(p.with_(olson_H=None, olson_chi=None, cv=np.array([H])))
    s2.step(1)
    assert abs(s2.fields()[1][0] - Tref) > 1e-4 * Tref


@pytest.mark.parametrize("flags", [W.FLAG_SLOPES, W.FLAG_SLOPES | W.FLAG_SI_LINEARIZED])
def test_olson_heat_capacity_conserves_the_discrete_energy(flags):
    """The ledger with the material energy U(T) closes to rounding in a 1-D slab with
    particles, slopes, a cold start against a hot wall and a mixed Olson /
    constant-C_v medium."""
    nx = 40
    H = np.where(np.arange(nx) < 25, 0.1, 0.5)
    chi = np.where(np.arange(nx) < 25, 0.1, 0.3)
    p = W.slab(nx, 6, lambda x: np.where(x < 0.6, 2.0, 30.0), dt=5e-3, steps=0, w_ref=2e-4, T0=0.01,
               Tb=1.0, pool_cap=1 << 20, flags=flags)
    p = p.with_(olson_H=H, olson_chi=chi)
    s = oracle.Sim(p)
    for _ in range(10):
        s.step(1)
        d = s.diag()
        assert abs(d["residual"]) <= 1e-12 * d["e_end"], d
    assert d["n_births"] > 0


# ---------------------------------------------------------------- volumetric source
def _box(q, t_off, nx=8, kap=0.0, dt=0.05):
    p = W.slab(nx, 3, lambda x: np.full_like(x, kap), dt=dt, steps=0, w_ref=1e-3, T0=0.2, pool_cap=1 << 20)
    return p.with_(bc=[W.BC_REFLECT, W.BC_REFLECT, 0, 0], nu_power=0.0, source=q, source_t_off=t_off)


def test_source_fills_a_transparent_box_until_switched_off():
    """sigma = 0 between mirrors: no exchange and no loss, so the radiation in every
    group grows by dt V sum_i q_i per step for the steps that start before t_off
    (here steps 0, 1 and 2 of a step size 0.05 with t_off = 0.125), then stays."""
    nx, dt = 8, 0.05
    rng = np.random.default_rng(3)
    q = rng.uniform(0.0, 2.0, (nx, 3))
    q[:, 1] = 0.0
    p = _box(q, 0.125, nx=nx, dt=dt)
    s = oracle.Sim(p)
    rho0, T0, _ = s.fields()
    V = 1.0 / nx
    for n in range(1, 7):
        s.step(1)
        rho, T, _ = s.fields()
        grown = min(n, 3) * dt * q.sum(0) * V
        np.testing.assert_allclose(rho.sum(0) * V, rho0.sum(0) * V + grown, rtol=1e-13, atol=0)
        np.testing.assert_array_equal(T, T0)
        d = s.diag()
        assert d["injection"] == pytest.approx(dt * q.sum() * V / p.c if n <= 3 else 0.0, rel=1e-14, abs=0)
        assert abs(d["residual"]) <= 1e-13 * d["e_end"]


def test_planckian_source_rate_in_a_transparent_box():
    """Q(x) = B(nu, Ts) f(x) on the transport equation's right side adds (c/eps^2)
    f_i phi_g(Ts) to rho per unit time: sigma = 0 between mirrors with c = 2 and
    eps = 0.5, the group totals grow by that rate and the ledger counts it as
    energy dt V q / c."""
    nx, dt, c, eps, Ts = 8, 0.05, 2.0, 0.5, 0.7
    f = np.linspace(1.0, 0.1, nx)
    p = _box(None, 10.0, nx=nx, dt=dt).with_(c=c, eps=eps, source=None, source_shape=f, source_T=Ts)
    s = oracle.Sim(p)
    rho0, _, _ = s.fields()
    V = 1.0 / nx
    e = p.nu_edges
    spec = np.array([phi_ref(Ts, e[g], e[g + 1], c=c) for g in range(3)])
    s.step(2)
    rho, _, _ = s.fields()
    rate = c / eps ** 2 * np.sum(f) * V * spec
    np.testing.assert_allclose(rho.sum(0) * V, rho0.sum(0) * V + 2 * dt * rate, rtol=1e-13)
    assert s.diag()["injection"] == pytest.approx(dt * rate.sum() / c, rel=1e-13)
    assert abs(s.diag()["residual"]) <= 1e-13 * s.diag()["e_end"]


def test_source_heats_a_zero_d_cell_as_the_implicit_equation_says():
    """One cell between mirrors with a source q: rho' = (rho^n + dt q + lambda phi(T'))/(1 + lambda)
    and C_v (T' - T^n) = dt sum_g sigma_g (rho'_g - phi_g(T')) (independent root find)."""
    dt = 0.02
    q = np.array([[0.3, 2.0, 0.05]])
    p = zero_d_problem(dt).with_(source=q, source_t_off=1.0)
    s = oracle.Sim(p)
    rho_n, T_n, _ = s.fields()
    s.step(1)
    rho, T, _ = s.fields()
    e = p.nu_edges
    sig = p.kappa[0] * simpson_sigma(e)
    lam = sig * dt

    def r_of(Tn1):
        ph = np.array([phi_ref(Tn1, e[g], e[g + 1]) for g in range(3)])
        return (rho_n[0] + dt * q[0] + lam * ph) / (1 + lam), ph

    def f(Tn1):
        r, ph = r_of(Tn1)
        return 0.7 * (Tn1 - T_n[0]) - np.sum(dt * sig * (r - ph))
    Tref = brentq(f, 1e-3, 2.0, xtol=1e-16, rtol=1e-15)
    assert T[0] == pytest.approx(Tref, rel=1e-12)
    np.testing.assert_allclose(rho[0], r_of(Tref)[0], rtol=1e-12)


@pytest.mark.parametrize("flags", [0, W.FLAG_SLOPES | W.FLAG_WAVE_ITER, W.FLAG_SI_LINEARIZED])
def test_source_energy_ledger(flags):
    """A source peaked at the left wall (the shape of Sec. 3.4's e^{-693 x^3}) in a slab
    with mirrors: every step's energy change equals the injected dt V q / c, the source
    stops at t_off, and nothing else enters."""
    nx, G = 40, 5
    xc = (np.arange(nx) + 0.5) / nx
    q = np.exp(-693.0 * (0.3 * xc) ** 3)[:, None] * np.linspace(1.0, 0.2, G)[None, :]
    p = W.slab(nx, G, lambda x: np.full_like(x, 3.0), dt=4e-3, steps=0, w_ref=2e-4, T0=0.01,
               pool_cap=1 << 20, flags=flags)
    p = p.with_(bc=[W.BC_REFLECT, W.BC_REFLECT, 0, 0], source=q, source_t_off=0.02)
    s = oracle.Sim(p)
    inj = 0.0
    for n in range(8):
        s.step(1)
        d = s.diag()
        assert abs(d["residual"]) <= 1e-12 * d["e_end"], d
        assert d["inflow_wave"] == 0.0 and d["inflow_eq"] == 0.0
        inj += d["injection"]
    assert inj == pytest.approx(5 * p.dt * q.sum() / nx / p.c, rel=1e-13)


def test_bad_source_is_refused():
    q = np.ones((8, 3))
    q[2, 1] = -1.0
    with pytest.raises(oracle.OracleError):
        oracle.Sim(_box(q, 1.0))
    with pytest.raises(oracle.OracleError):
        oracle.Sim(_box(np.ones((8, 3)), -1.0))


# ---------------------------------------------------------------- tabulated opacity
def _power_law_table(kmat, p, q, nu_nodes, T_nodes):
    return np.array([[[k * nu ** -p * T ** -q for nu in nu_nodes] for T in T_nodes] for k in kmat])


def test_table_interpolation_is_log_log_bilinear_and_clamped():
    nu_nodes = np.array([0.01, 0.1, 1.0, 10.0])
    T_nodes = np.array([1e-3, 1e-2, 1.0])
    rng = np.random.default_rng(2)
    sig = 10 ** rng.uniform(-2, 4, (2, 3, 4))
    p = W.slab(4, 3, lambda x: np.ones_like(x), dt=1e-3, steps=0, w_ref=1e-3)
    p = p.with_(opacity_table={"mat": np.array([0, 1, 1, 0]), "nu": nu_nodes, "T": T_nodes, "sigma": sig})
    s = oracle.Sim(p)
    for m in range(2):
        for j, T in enumerate(T_nodes):
            for i, nu in enumerate(nu_nodes):
                assert s.table_sigma(m, nu, T) == pytest.approx(sig[m, j, i], rel=1e-14)
        # midpoint in log-log: geometric mean of the four corners
        nu_m, T_m = np.sqrt(0.1 * 1.0), np.sqrt(1e-2 * 1.0)
        gm = (sig[m, 1, 1] * sig[m, 1, 2] * sig[m, 2, 1] * sig[m, 2, 2]) ** 0.25
        assert s.table_sigma(m, nu_m, T_m) == pytest.approx(gm, rel=1e-13)
        # clamped beyond the ends
        assert s.table_sigma(m, 1e-5, 1e-6) == pytest.approx(sig[m, 0, 0], rel=1e-14)
        assert s.table_sigma(m, 1e3, 50.0) == pytest.approx(sig[m, 2, 3], rel=1e-14)
        # along one axis at a node of the other: linear in ln sigma
        t = 0.3
        nu_t = np.exp((1 - t) * np.log(0.01) + t * np.log(0.1))
        ref = np.exp((1 - t) * np.log(sig[m, 2, 0]) + t * np.log(sig[m, 2, 1]))
        assert s.table_sigma(m, nu_t, 1.0) == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("group_sigma", [False, True])
def test_power_law_table_reproduces_the_analytic_opacity_run(group_sigma):
    """kappa_m nu^-3 T^-1/2 is exactly linear in (ln nu, ln T), so a table of it over a
    range that covers every frequency and temperature gives the same run as the
    analytic opacity, particles included, to rounding."""
    nx, G = 30, 6
    mat = (np.arange(nx) >= 18).astype(np.int32)
    kmat = np.array([2.0, 40.0])
    flags = W.FLAG_SLOPES | (W.FLAG_GROUP_SIGMA if group_sigma else 0)
    p = W.slab(nx, G, lambda x: np.ones_like(x), dt=4e-3, steps=0, w_ref=2e-4, T0=0.01,
               pool_cap=1 << 20, T_power=0.5, flags=flags, numin=0.01, numax=10.0)
    p = p.with_(kappa=np.repeat(kmat[mat][:, None], G, axis=1).copy())
    nu_nodes = np.geomspace(0.005, 20.0, 7)
    T_nodes = np.geomspace(1e-4, 5.0, 5)
    tab = {"mat": mat, "nu": nu_nodes, "T": T_nodes, "sigma": _power_law_table(kmat, 3.0, 0.5, nu_nodes, T_nodes)}
    a = oracle.Sim(p)
    b = oracle.Sim(p.with_(opacity_table=tab))
    for n in range(8):
        a.step(1)
        b.step(1)
    ra, Ta, pa = a.fields()
    rb, Tb, pb = b.fields()
    np.testing.assert_allclose(Tb, Ta, rtol=1e-12)
    np.testing.assert_allclose(rb, ra, rtol=1e-11, atol=1e-12 * np.max(ra))
    assert a.diag()["n_births"] == b.diag()["n_births"]
    assert a.diag()["n_crossings"] == b.diag()["n_crossings"]
    assert abs(b.diag()["residual"]) <= 1e-12 * b.diag()["e_end"]


def test_table_turns_on_the_temperature_dependent_iteration():
    """A table whose sigma falls with T: the source iteration re-evaluates sigma at
    its iterate, so the step equals the one of the analytic T^-1 opacity (0-D cell,
    independent root find with sigma(T'))."""
    dt = 0.05
    e = np.array([0.05, 0.3, 1.0, 5.0])
    nu_nodes = np.geomspace(0.01, 10.0, 5)
    T_nodes = np.geomspace(1e-3, 10.0, 4)
    p = zero_d_problem(dt, kap=(1.0, 1.0, 1.0), T0=0.2, Tr=0.6)
    p = p.with_(opacity_table={"mat": np.array([0]), "nu": nu_nodes, "T": T_nodes,
                               "sigma": _power_law_table([4.0], 0.0, 1.0, nu_nodes, T_nodes)},
                si_max_iters=2000)
    s = oracle.Sim(p)
    rho_n, T_n, _ = s.fields()
    s.step(1)
    rho, T, _ = s.fields()

    def f(Tn1):
        sig = np.full(3, 4.0 / Tn1)
        lam = sig * dt
        ph = np.array([phi_ref(Tn1, e[g], e[g + 1]) for g in range(3)])
        r = (rho_n[0] + lam * ph) / (1 + lam)
        return 0.7 * (Tn1 - T_n[0]) - np.sum(dt * sig * (r - ph))
    Tref = brentq(f, 1e-3, 2.0, xtol=1e-16, rtol=1e-15)
    assert T[0] == pytest.approx(Tref, rel=1e-11)


def test_record_refuses_the_olson_models():
    for kw in ({"olson_H": np.full(4, 0.1), "olson_chi": np.full(4, 0.1)},
               {"source": np.ones((4, 3))}):
        p = W.slab(4, 3, lambda x: np.ones_like(x), dt=1e-3, steps=0, w_ref=1e-3).with_(**kw)
        s = oracle.Sim(p)
        with pytest.raises(oracle.OracleError):
            s.record(True)


# ---------------------------------------------------------------- Olson 1-D workload
def test_olson_1d_first_steps_conserve_and_heat_from_the_source():
    """The Olson foam problem (tabulated opacity, Olson's heat capacity, the Planckian
    source B(0.5) e^{-693 x^3}, mirrors): each step closes its energy ledger, the energy
    grows by exactly the injected source, and the heat stays near x = 0."""
    p = W.olson1d()
    s = oracle.Sim(p)
    E0 = None
    inj = 0.0
    for n in range(6):
        s.step(1)
        d = s.diag()
        E0 = d["e_start"] if E0 is None else E0
        inj += d["injection"]
        assert abs(d["residual"]) <= 1e-12 * d["e_end"], d
    T = s.fields()[1]
    assert T[0] > 0.012 and T[-1] == pytest.approx(0.01, rel=1e-6)
    assert np.all(np.diff(T[1:40]) <= 1e-12)         # falling away from the source
    # injection: (c/eps^2) f_i phi_g(0.5) summed over cells and groups, times dt V / c
    e = p.nu_edges
    spec = sum(phi_ref(0.5, e[g], e[g + 1]) for g in range(p.G))
    V = (p.x1 - p.x0) / p.nx
    assert inj == pytest.approx(6 * p.dt * V * spec * np.sum(p.source_shape), rel=1e-12)


def test_literal_and_linearized_iterations_reach_the_same_step():
    """Both iterations converge to the one fixed point of the step's implicit system."""
    a = oracle.Sim(W.olson1d(flags=0))
    b = oracle.Sim(W.olson1d())
    for n in range(3):
        a.step(1)
        b.step(1)
    ra, Ta, _ = a.fields()
    rb, Tb, _ = b.fields()
    np.testing.assert_allclose(Ta, Tb, rtol=1e-11)
    np.testing.assert_allclose(ra, rb, rtol=1e-10, atol=1e-12 * np.max(ra))
