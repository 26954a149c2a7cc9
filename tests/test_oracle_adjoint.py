"""Pins of the oracle's adjoint of the frozen-tally macroscopic map.

The adjoint differentiates the map that holds the particle-phase results of a
recorded run fixed (net particle flux, survivor density, sampled flags) and
lets everything else follow the opacity.  It is pinned against:
  - 40-digit derivatives (mpmath) of the closed-form flux coefficients it uses;
  - central finite differences of the frozen replay, along random directions
    and entry by entry;
  - the replay itself, which must reproduce the recorded forward run;
  - with no particles (nothing frozen), central finite differences of the
    unmodified forward step from t = 0.
"""
import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2312_16981_amd import workloads as W

mp.mp.dps = 40


def cell_volume(p):
    return (p.x1 - p.x0) / p.nx * ((p.y1 - p.y0) / p.ny if p.dim == 2 else 1.0)


def energy(p, T):
    """Material energy J = sum_i V C_v T_i."""
    return float(np.sum(cell_volume(p) * p.cv * T))


CASES = {
    # 2-D, log-normal opacity, Planckian left wall, particles in thin cells
    "lognormal": (lambda: W.c5_lognormal(n=10, G=4, w_ref=2e-4, pool_cap=1 << 20, dt=2e-3), 6),
    # 1-D, Planckian left wall, reflective right wall
    "slab_reflect": (lambda: W.c1_marshak_like(w_ref=2e-5).with_(bc=[W.BC_PLANCK, W.BC_REFLECT, 0, 0]), 8),
    # 2-D lattice: opacity jumps of 100x, pinned source cells, vacuum walls
    "lattice_pinned": (lambda: W.c3_lattice(n=14, G=3, w_ref=1e-3, pool_cap=1 << 20, dt=2e-2), 4),
    # 1-D stiff material coupling (C_v = 0.01, kappa = 50): the literal sweep and the
    # unpreconditioned transposed sweep both diverge; run with the linearized sweep
    "stiff_slab": (lambda: _stiff_slab(), 3),
}


def _stiff_slab(**kw):
    nx = 40
    p = dict(dt=0.02, steps=0, w_ref=2e-5, pool_cap=1 << 20, flags=W.FLAG_SI_LINEARIZED)
    p.update(kw)
    q = W.slab(nx, 6, lambda x: np.full_like(x, 50.0), **p)
    return q.with_(cv=np.full(nx, 0.01), T0=np.full(nx, 0.05), Tr0=np.full(nx, 0.05))


def recorded(name):
    make, nsteps = CASES[name]
    p = make()
    sim = oracle.Sim(p)
    sim.record(True)
    sim.step(nsteps)
    return p, sim


# ------------------------------------------------------------ coefficient derivatives

def _c4(s):
    return (1 - mp.exp(-s)) / s


def _w(s):
    return _c4(s) - mp.exp(-s)


def _c2dt(s):
    return (2 * _c4(s) - 1 - mp.exp(-s)) / s


@pytest.mark.parametrize("fn,ref", [(oracle.coef_c4_ds, _c4), (oracle.coef_w_ds, _w),
                                    (oracle.coef_c2_over_dt_ds, _c2dt)])
def test_coefficient_derivatives_match_mpmath(fn, ref):
    grid = [1e-14, 1e-9, 1e-5, 1e-3, 0.05, 0.3, 0.9999, 1.0, 1.0001, 1.7, 1.9999, 2.0, 2.0001,
            2.5, 3.7, 8.0, 40.0, 700.0, 1e5, 1e9]
    for s in grid:
        d = mp.diff(ref, mp.mpf(s))
        got = fn(s)
        # relative to the size of the terms (~1/s^2 for large s): d(C2/dt)/ds has a
        # root near s = 2.6, where no relative bound holds
        assert abs(got - float(d)) <= 1e-14 * max(abs(float(d)), 0.05 / (1 + s * s)), (fn.__name__, s)


def test_coefficient_derivative_limits():
    """s -> 0: dC4/ds -> -1/2, dW/ds -> 1/2, d(C2/dt)/ds -> -1/6 (term by term)."""
    assert oracle.coef_c4_ds(0.0) == -0.5
    assert oracle.coef_w_ds(0.0) == 0.5
    assert abs(oracle.coef_c2_over_dt_ds(0.0) + 1.0 / 6.0) < 1e-17


# ------------------------------------------------------------ replay and adjoint

@pytest.mark.parametrize("name", sorted(CASES))
def test_replay_reproduces_recorded_run(name):
    p, sim = recorded(name)
    T = sim.fields()[1]
    Tr = sim.replay_frozen(p.kappa)
    assert np.max(np.abs(Tr - T)) <= 1e-12 * np.max(T)


@pytest.mark.parametrize("name", sorted(CASES))
def test_adjoint_directional_derivative(name):
    p, sim = recorded(name)
    grad = sim.adjoint(cell_volume(p) * p.cv)
    assert grad.shape == p.kappa.shape and np.all(np.isfinite(grad))
    rng = np.random.default_rng(11)
    h = 1e-4
    for _ in range(2):
        v = rng.standard_normal(p.kappa.shape)
        fd = (energy(p, sim.replay_frozen(p.kappa * (1 + h * v)))
              - energy(p, sim.replay_frozen(p.kappa * (1 - h * v)))) / (2 * h)
        ad = float(np.sum(grad * p.kappa * v))
        assert abs(fd - ad) <= 1e-7 * abs(ad), (fd, ad)


@pytest.mark.parametrize("name", sorted(CASES))
def test_adjoint_entries(name):
    """Entry by entry: the 6 largest |dJ/dlog kappa| and 6 random entries."""
    p, sim = recorded(name)
    grad = sim.adjoint(cell_volume(p) * p.cv)
    g_log = (grad * p.kappa).reshape(-1)
    scale = np.max(np.abs(g_log))
    rng = np.random.default_rng(5)
    idx = list(np.argsort(-np.abs(g_log))[:6]) + list(rng.choice(g_log.size, 6, replace=False))
    h = 1e-4
    for j in idx:
        e = np.zeros(g_log.size)
        e[j] = 1.0
        e = e.reshape(p.kappa.shape)
        fd = (energy(p, sim.replay_frozen(p.kappa * (1 + h * e)))
              - energy(p, sim.replay_frozen(p.kappa * (1 - h * e)))) / (2 * h)
        assert abs(fd - g_log[j]) <= 1e-6 * scale + 1e-6 * abs(g_log[j]), (j, fd, g_log[j])


def test_adjoint_without_particles_matches_forward_fd():
    """No particles: the frozen map is the whole step, so the adjoint is the
    derivative of the unmodified forward run from t = 0."""
    p = W.c1_marshak_like(w_ref=1e300).with_(bc=[W.BC_PLANCK, W.BC_VACUUM, 0, 0])
    p = p.with_(kappa=p.kappa * np.linspace(0.2, 3.0, p.nx)[:, None])
    nsteps = 8
    sim = oracle.Sim(p)
    sim.record(True)
    sim.step(nsteps)
    grad = sim.adjoint(cell_volume(p) * p.cv)

    def J(kappa):
        s = oracle.Sim(p.with_(kappa=kappa))
        s.step(nsteps)
        return energy(p, s.fields()[1])

    rng = np.random.default_rng(3)
    v = rng.standard_normal(p.kappa.shape)
    h = 1e-4
    fd = (J(p.kappa * (1 + h * v)) - J(p.kappa * (1 - h * v))) / (2 * h)
    ad = float(np.sum(grad * p.kappa * v))
    assert abs(fd - ad) <= 1e-7 * abs(ad), (fd, ad)


def test_stiff_adjoint_without_particles_matches_forward_fd():
    """Stiff coupling (the local contraction factor of the literal sweep is far
    above 1 at the fixed point): the forward run needs the linearized sweep and
    the transposed iteration its preconditioned form.  With no particles the
    adjoint is the derivative of the unmodified forward run from t = 0."""
    p = _stiff_slab(w_ref=1e300)
    p = p.with_(kappa=p.kappa * np.linspace(0.5, 2.0, p.nx)[:, None])
    nsteps = 4
    sim = oracle.Sim(p)
    sim.record(True)
    sim.step(nsteps)
    T = sim.fields()[1]
    e = p.nu_edges
    sig = p.kappa[0] * (e[:-1] ** -3 + 4 * (0.5 * (e[:-1] + e[1:])) ** -3 + e[1:] ** -3) / 6.0
    lam = p.c * sig * p.dt / p.eps ** 2
    dphi = np.array([oracle.dphi_group(T[0], e[g], e[g + 1]) for g in range(p.G)])
    d = p.dt / (p.eps ** 2 * p.cv[0]) * np.sum(sig * dphi / (1 + lam))
    assert d > 5.0                            # the unpreconditioned iterations diverge
    grad = sim.adjoint(cell_volume(p) * p.cv)

    def J(kappa):
        s = oracle.Sim(p.with_(kappa=kappa))
        s.step(nsteps)
        return energy(p, s.fields()[1])

    rng = np.random.default_rng(4)
    for _ in range(2):
        v = rng.standard_normal(p.kappa.shape)
        h = 1e-4
        fd = (J(p.kappa * (1 + h * v)) - J(p.kappa * (1 - h * v))) / (2 * h)
        ad = float(np.sum(grad * p.kappa * v))
        assert abs(fd - ad) <= 1e-7 * abs(ad), (fd, ad)


def test_adjoint_is_linear_in_the_objective():
    p, sim = recorded("lattice_pinned")
    rng = np.random.default_rng(8)
    a = rng.standard_normal(p.ncell)
    b = rng.standard_normal(p.ncell)
    ga, gb, gab = sim.adjoint(a), sim.adjoint(b), sim.adjoint(2.0 * a - 3.0 * b)
    np.testing.assert_allclose(gab, 2.0 * ga - 3.0 * gb, rtol=1e-9, atol=1e-12 * np.max(np.abs(gab)))


def test_pinned_cells_only_objective():
    """An objective on pinned cells alone has zero gradient: their temperature never moves."""
    p, sim = recorded("lattice_pinned")
    d = np.where(p.pinned == 1, 1.0, 0.0)
    assert np.all(sim.adjoint(d) == 0.0)


def test_adjoint_full_lognormal_shape_entries():
    """The adjoint workload's shape (128 x 128 cells x 16 groups, log-normal
    opacity, Planckian wall) over its first 2 steps.  After two steps only a
    thin layer of cells near the wall carries gradient, so the entries checked
    are the 8 largest of dJ/dlog kappa, 24 drawn among those above 1e-3 of the
    largest, and 8 drawn among the rest.  Each is compared with a central
    difference of the frozen replay (the particle results held fixed: common
    random numbers) at a relative step h = 1e-3, whose truncation and rounding
    errors both stay below 1e-7 of the gradient's scale on this case."""
    p = W.c5_lognormal()
    sim = oracle.Sim(p)
    sim.record(True)
    sim.step(2)
    grad = sim.adjoint(cell_volume(p) * p.cv)
    g_log = (grad * p.kappa).reshape(-1)
    scale = np.max(np.abs(g_log))
    rng = np.random.default_rng(64)
    order = np.argsort(-np.abs(g_log))
    big = np.flatnonzero(np.abs(g_log) >= 1e-3 * scale)
    small = np.flatnonzero(np.abs(g_log) < 1e-3 * scale)
    assert big.size > 500
    picks = np.concatenate([order[:8],
                            rng.choice(np.setdiff1d(big, order[:8]), 24, replace=False),
                            rng.choice(small, 8, replace=False)])
    h = 1e-3
    for j in picks:
        e = np.zeros(g_log.size)
        e[j] = 1.0
        e = e.reshape(p.kappa.shape)
        fd = (energy(p, sim.replay_frozen(p.kappa * (1 + h * e)))
              - energy(p, sim.replay_frozen(p.kappa * (1 - h * e)))) / (2 * h)
        assert abs(fd - g_log[j]) <= 1e-7 * scale + 1e-5 * abs(g_log[j]), (j, fd, g_log[j])
