"""GPU vs FP64 oracle for the material models of Olson's problems (Sec. 3.4-3.5):
Olson's heat capacity in energy form, the volumetric source (a rate per
(cell, group) or the Planckian B(nu, Ts) f(x)) with its switch-off time, and a
tabulated opacity sigma(nu, T) per material (the per-particle flights through
the cell rows, and the group opacity of the sweeps and of the sampling), in
1-D, 2-D and batches.  Same bar as the other parity tests: integers bit-exact,
every field, tally and particle within 1e-10 of its array's max-norm, equal
sweep counts."""
import numpy as np
import pytest

import oracle
from paper_2312_16981_amd import ugkwp
from paper_2312_16981_amd import workloads as W
from test_gpu_parity import compare_pool, compare_state, run_pair, say

pytestmark = pytest.mark.gpu
LIN, SL, WI, GS = W.FLAG_SI_LINEARIZED, W.FLAG_SLOPES, W.FLAG_WAVE_ITER, W.FLAG_GROUP_SIGMA


def _olson_slab(flags, nx=60, G=6):
    H = np.where(np.arange(nx) < 35, 0.1, 0.5)
    chi = np.where(np.arange(nx) < 35, 0.1, 0.3)
    p = W.slab(nx, G, lambda x: np.where(x < 0.6, 2.0, 30.0), dt=5e-3, steps=0, w_ref=2e-4, T0=0.01,
               pool_cap=1 << 20, flags=flags, name=f"olson_cv_slab_f{flags}")
    return p.with_(olson_H=H, olson_chi=chi)


@pytest.mark.parametrize("flags", [0, LIN, SL | LIN, SL | WI])
def test_olson_heat_capacity_slab(flags):
    run_pair(_olson_slab(flags), 8, every=4)


@pytest.mark.parametrize("flags", [0, WI | SL])
def test_rate_source_switching_off(flags):
    nx, G = 50, 5
    xc = (np.arange(nx) + 0.5) / nx
    q = np.exp(-693.0 * (0.3 * xc) ** 3)[:, None] * np.linspace(1.0, 0.2, G)[None, :]
    p = W.slab(nx, G, lambda x: np.full_like(x, 3.0), dt=4e-3, steps=0, w_ref=2e-4, T0=0.01,
               pool_cap=1 << 20, flags=flags, name=f"source_slab_f{flags}")
    p = p.with_(bc=[W.BC_REFLECT, W.BC_REFLECT, 0, 0], source=q, source_t_off=0.02)
    ctx, sim = run_pair(p, 9, every=3)
    assert ctx.get_diag()["injection"] == 0.0 and sim.diag()["injection"] == 0.0   # switched off by step 5


@pytest.mark.parametrize("flags", [LIN, 0, LIN | SL, LIN | GS])
def test_olson_1d(flags):
    """The Olson foam problem: tabulated opacity (per-particle flights through the
    cell rows, or group opacities), Olson's heat capacity, Planckian source.  (The
    wave flux from the iterate, UGKWP_FLAG_WAVE_ITER, does not converge here at
    dt = dx / c, on either side.)"""
    p = W.olson1d(flags=flags)
    run_pair(p.with_(name=f"olson1d_f{flags}"), 12, every=4)


def test_olson_1d_whole_run_in_one_call():
    """The whole run to c t = 4 (107 steps; the source switches off at c t = 2) in one
    call, compared with the oracle at the end."""
    p = W.olson1d()
    ctx = ugkwp.from_problem(p)
    sim = oracle.Sim(p)
    say(f"[olson] olson1d, {p.steps} steps in one call")
    ctx.step(p.steps)
    sim.step(p.steps)
    compare_state(ctx, sim, p, what=f"olson1d step {p.steps}")
    compare_pool(ctx, sim, 1)
    assert ctx.get_diag()["injection"] == 0.0          # c t = 4 > 2: the source is off


@pytest.mark.parametrize("flags", [LIN, LIN | SL])
def test_olson_2d_small(flags):
    p = W.olson2d(n=40, G=8, flags=flags)
    run_pair(p.with_(name=f"olson2d_40_f{flags}"), 6, every=3)


def test_olson_2d_full_mesh_first_steps():
    """The 285 x 285, 24-group mesh of Sec. 3.5, 3 steps in one call."""
    p = W.olson2d()
    ctx = ugkwp.from_problem(p)
    sim = oracle.Sim(p)
    say("[olson] olson2d 285x285, 3 steps in one call")
    ctx.step(3)
    sim.step(3)
    compare_state(ctx, sim, p, what="olson2d step 3")
    assert ctx.get_diag()["sweeps_max"] == sim.diag()["sweeps"]


def test_batch_of_olson_instances():
    probs = []
    for k, (nx, H) in enumerate([(40, 0.1), (96, 0.3), (17, 0.05)]):
        p = W.olson1d(nx=nx, G=6, seed=900 + k, pool_cap=1 << 18, dt=0.04)
        probs.append(p.with_(olson_H=np.full(nx, H), name=f"olson_b{k}"))
    say("[olson] batch of", len(probs))
    ctx = ugkwp.from_batch(probs)
    sims = [oracle.Sim(q) for q in probs]
    for n in range(10):
        ctx.step(1)
        for s in sims:
            s.step(1)
    for k, (q, s) in enumerate(zip(probs, sims)):
        compare_state(ctx, s, q, inst=k, what=f"olson batch instance {k}")


def test_power_law_table_matches_the_analytic_opacity_on_the_gpu():
    """A table of kappa nu^-3 T^-1/2 reproduces the analytic opacity's GPU run."""
    nx, G = 40, 6
    p = W.slab(nx, G, lambda x: np.where(x < 0.5, 2.0, 40.0), dt=4e-3, steps=0, w_ref=2e-4, T0=0.01,
               pool_cap=1 << 20, T_power=0.5, numin=0.01, numax=10.0)
    nu_n, T_n = np.geomspace(0.005, 20.0, 7), np.geomspace(1e-4, 5.0, 5)
    mat = (np.arange(nx) >= nx // 2).astype(np.int32)
    sig = np.array([[[k * nu ** -3 * T ** -0.5 for nu in nu_n] for T in T_n] for k in (2.0, 40.0)])
    a = ugkwp.from_problem(p)
    b = ugkwp.from_problem(p.with_(opacity_table={"mat": mat, "nu": nu_n, "T": T_n, "sigma": sig}))
    a.step(6)
    b.step(6)
    ra, Ta, _ = a.get_fields(0)
    rb, Tb, _ = b.get_fields(0)
    assert np.max(np.abs(Ta - Tb)) <= 1e-11 * np.max(Ta)
    assert np.max(np.abs(ra - rb)) <= 1e-10 * np.max(ra)
    assert a.get_diag()["n_births"] == b.get_diag()["n_births"]


def test_recording_and_bad_input_refused():
    p = W.olson1d(nx=16, G=4)
    ctx = ugkwp.from_problem(p)
    with pytest.raises(ugkwp.UGKWPError):
        ctx.record(3)
    with pytest.raises(ugkwp.UGKWPError):
        ctx.set_heat_capacity(np.full(16, -1.0), np.zeros(16))
    with pytest.raises(ugkwp.UGKWPError):
        ctx.set_source(np.full(16 * 4, np.nan), 1.0)
    t = p.opacity_table
    with pytest.raises(ugkwp.UGKWPError):
        ctx.set_opacity_table(np.full(16, 3), t["nu"], t["T"], t["sigma"])
    with pytest.raises(ugkwp.UGKWPError):
        ctx.set_opacity_table(t["mat"], t["nu"][::-1], t["T"], t["sigma"])
    # the context still runs the problem it was given
    sim = oracle.Sim(p)
    ctx.step(3)
    sim.step(3)
    compare_state(ctx, sim, p, what="after refused calls")


@pytest.mark.parametrize("which", ["olson1d", "slab_all_flags"])
def test_checkpoint_restart_with_the_later_variants(which):
    """A saved state restored into a fresh context continues like the oracle's
    uninterrupted run: with Olson's models across the source's switch-off (steps
    0-39 saved, 40-79 restored), and with every second-order flag."""
    from test_gpu_parity import TOL, relerr
    if which == "olson1d":
        p, n = W.olson1d(), 40
    else:
        p, n = W.c1_marshak_like().with_(flags=SL | WI | W.FLAG_BOUNDARY_PARTICLES, name="slab_all_flags"), 12
    say(f"[checkpoint] {p.name} steps {n} + {n}")
    a = ugkwp.from_problem(p)
    a.step(n)
    buf = a.get_state()
    b = ugkwp.from_problem(p)
    b.set_state(buf)
    b.step(n)
    sim = oracle.Sim(p)
    sim.step(2 * n)
    compare_state(b, sim, p, what=f"{p.name} restored")
    compare_pool(b, sim, p.dim)
    a.step(n)
    ra, ta, _ = a.get_fields()
    rb, tb, _ = b.get_fields()
    assert relerr(rb, ra) <= TOL and relerr(tb, ta) <= TOL


def test_autotune_with_tabulated_flights():
    """The push's launch-shape autotuner on the table's flights (and its restore of
    the tallies and counters it touched): the run goes on like the oracle's."""
    p = W.olson2d(n=40, G=8).with_(name="olson2d_40_autotune")
    ctx = ugkwp.from_problem(p)
    sim = oracle.Sim(p)
    ctx.step(4)
    sim.step(4)
    res = ctx.autotune()
    assert res["threads"] in (256, 512) and res["candidates"] >= 6
    ctx.step(3)
    sim.step(3)
    compare_state(ctx, sim, p, what="olson2d after autotune")
    compare_pool(ctx, sim, 2)
