"""Pins of the oracle's numerical collision time in thin-thick-joint cells
(Sec. 3.2, second case): tau_num = eps^2/(c sigma) + C |T^l - T^r|/(T^l + T^r) dt
replaces tau in the sampling fraction e^{-dt/tau} of the cells that share a face
across which the group opacity jumps by a factor >= jump."""
import numpy as np
import pytest

import oracle
from paper_2312_16981_amd import workloads as W


def thick_thin(C=1e5, jump=10.0, nx=60, G=6):
    """Thick-to-thin slab: kappa = 1000 for x <= 0.3 at T = 0.5, kappa = 10 beyond
    at T = 1e-3 (radiation and material in equilibrium), Planckian wall at T = 1,
    so that the joint cells see a temperature jump from the start."""
    p = W.slab(nx, G, lambda x: np.where(x <= 0.3, 1000.0, 10.0), dt=2e-3, steps=0,
               w_ref=2e-5, pool_cap=1 << 20, tau_num_C=C, tau_num_jump=jump,
               name="thick_thin")
    xc = (np.arange(nx) + 0.5) / nx
    T0 = np.where(xc <= 0.3, 0.5, 1e-3)
    return p.with_(T0=T0.copy(), Tr0=T0.copy())


def simpson(edges, p=3.0):
    nl, nh = edges[:-1], edges[1:]
    nm = 0.5 * (nl + nh)
    return (nl ** -p + 4 * nm ** -p + nh ** -p) / 6.0


def expected_fraction(p, T):
    """e^{-dt/tau_num} per (cell, group), written from the definition: the
    physical tau = eps^2/(c sigma), and in a joint cell tau + C delta dt with
    delta the largest relative temperature jump over its joint faces."""
    sig = p.kappa * simpson(p.nu_edges)[None, :]
    tau = np.where(sig > 0, p.eps ** 2 / (p.c * np.where(sig > 0, sig, 1.0)), np.inf)
    frac = np.exp(-p.dt / tau)
    for i in range(p.nx):
        for g in range(p.G):
            deltas = []
            for j in (i - 1, i + 1):
                if 0 <= j < p.nx:
                    hi, lo = max(sig[i, g], sig[j, g]), min(sig[i, g], sig[j, g])
                    if hi > 0 and hi >= p.tau_num_jump * lo:
                        deltas.append(abs(T[i] - T[j]) / (T[i] + T[j]))
            if deltas:
                tnum = tau[i, g] + p.tau_num_C * max(deltas) * p.dt
                frac[i, g] = np.exp(-p.dt / tnum)
    return frac


def test_sampling_fraction_follows_tau_num():
    """After a few steps (so that T varies), the energy sampled into particles in
    every (cell, group) equals e^{-dt/tau_num} rho^h V, with rho^h = rho^n - rho^p."""
    p = thick_thin()
    sim = oracle.Sim(p)
    sim.step(8)
    rho, T, rhop = sim.fields()
    frac = expected_fraction(p, T)
    joint = ~np.isclose(frac, np.exp(-p.dt * p.c * p.kappa * simpson(p.nu_edges)[None, :] / p.eps ** 2),
                        rtol=0, atol=0)
    assert joint.any(), "no cell took tau_num"
    sim.step(1)
    t = sim.tallies()
    V = (p.x1 - p.x0) / p.nx
    E = frac * (rho - rhop) * V
    nb, wnew = t["nbirth"], t["wnew"]
    s = nb >= 1
    assert s[joint].sum() > 0
    np.testing.assert_allclose(nb[s] * wnew[s], E[s], rtol=1e-13, atol=0)
    q = E / (p.w_ref * V)
    assert np.all(np.where(s, True, q < 1.0))


def test_joint_cells_sample_more_and_energy_is_conserved():
    base = thick_thin(C=0.0)
    num = thick_thin()
    a, b = oracle.Sim(base), oracle.Sim(num)
    for n in range(12):
        a.step(1)
        b.step(1)
        d = b.diag()
        assert abs(d["residual"]) <= 1e-12 * abs(d["e_end"]), n
    assert b.tallies()["nbirth"].sum() > a.tallies()["nbirth"].sum()


def test_without_joint_faces_the_step_is_unchanged():
    """tau_num only acts where the opacity jumps: with a jump threshold above
    every ratio, the run is the base method bit for bit."""
    a = oracle.Sim(thick_thin(C=0.0))
    b = oracle.Sim(thick_thin(C=1e5, jump=1e9))
    a.step(6)
    b.step(6)
    for u, v in zip(a.fields(), b.fields()):
        assert np.array_equal(u, v)
    assert np.array_equal(a.tallies()["nbirth"], b.tallies()["nbirth"])


def test_recording_refuses_tau_num():
    sim = oracle.Sim(thick_thin())
    with pytest.raises(oracle.OracleError):
        sim.record(True)


def test_static_source_uses_the_joint_cells_wave_coefficient():
    """Q of every interior cell from its definition (Sec. 2.2 and Remark 3):
    rho^n + (dt/V)(F_in - F_out) + w^{fr,p}/V with the wave flux
    c/(4 eps)(A_l rho^h_l - A_r rho^h_r) through each face, A = C4(s) -
    e^{-dt/tau_num} in a sampled cell (e^{-s} outside the joint cells) and
    C4(s) in an unsampled one, and w^{fr,p} from the gross particle crossings."""
    p = thick_thin()
    sim = oracle.Sim(p)
    sim.step(5)
    rho, T, rhop = sim.fields()
    frac = expected_fraction(p, T)
    sim.step(1)
    t = sim.tallies()
    sig = p.kappa * simpson(p.nu_edges)[None, :]
    s = p.c * sig * p.dt / p.eps ** 2
    c4 = -np.expm1(-s) / s
    A = np.where(t["nbirth"] >= 1, c4 - frac, c4)
    rh = rho - rhop
    V = (p.x1 - p.x0) / p.nx
    cq = p.c / (4 * p.eps)
    fx = t["fx"]                                   # [face][G][+x, -x]
    checked = 0
    for i in range(1, p.nx - 1):
        F_left = cq * (A[i - 1] * rh[i - 1] - A[i] * rh[i])
        F_right = cq * (A[i] * rh[i] - A[i + 1] * rh[i + 1])
        w_in = fx[i, :, 0] + fx[i + 1, :, 1]
        w_out = fx[i, :, 1] + fx[i + 1, :, 0]
        Q = rho[i] + p.dt / V * (F_left - F_right) + (w_in - w_out) / V
        np.testing.assert_allclose(t["Q"][i], Q, rtol=1e-12, atol=1e-12 * np.max(np.abs(t["Q"])))
        checked += 1
    joint = ~np.isclose(frac, np.exp(-s), rtol=0, atol=0)
    assert checked == p.nx - 2 and (joint & (t["nbirth"] >= 1)).any()
