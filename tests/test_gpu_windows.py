"""GPU vs FP64 oracle over the windows the benchmark measures, in the launch
configuration it times: one library call of many steps (steps enqueued ahead
of the host), the push launch shape picked by the autotuner, phase timing
switched on.  Same bar as the other parity tests: integers bit-exact,
floating point within 1e-10 of each array's max-norm.

Where the oracle cannot run the whole window from t = 0 (the 2-D lattice at
~6e7 particles, steps 480-499: about 40 minutes of oracle time), both sides
start from a seeded synthetic state of that size instead and take the
window's launch configuration from there."""
import sys

import numpy as np
import pytest

import oracle
from paper_2312_16981_amd import ugkwp
from paper_2312_16981_amd import workloads as W
from test_gpu_parity import compare_pool, compare_state, relerr, TOL

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_slab_benchmark_window_from_t0():
    """The 2000-cell x 64-group two-material slab, run as the benchmark runs it:
    500 steps in one call, the autotuner, 5 warm-up steps, the 20 timed steps in
    one call (steps 505-524), then 20 steps with every phase timed; the oracle
    runs the same 545 steps from t = 0.  The particle pushes of the timed steps
    (entering particles plus births, summed over the call) are compared with the
    oracle's per-step counts."""
    p = W.c2_two_material()
    ctx = ugkwp.from_problem(p)
    sim = oracle.Sim(p)
    say("[window] slab: 500 steps in one call")
    ctx.step(500)
    sim.step(500)
    compare_state(ctx, sim, p, what="slab step 500")
    tuned = ctx.autotune()
    say(f"[window] slab: autotuned {tuned}")
    ctx.step(5)
    sim.step(5)
    ctx.get_totals(reset=True)
    say("[window] slab: 20 timed steps in one call")
    ctx.step(20)
    pushes = 0
    for _ in range(20):
        sim.step(1)
        d = sim.diag()
        pushes += d["n_alive_in"] + d["n_births"]
    tot = ctx.get_totals()
    assert tot["steps"] == 20 and tot["n_pushed"] == pushes, (tot["n_pushed"], pushes)
    compare_state(ctx, sim, p, what="slab step 525")
    compare_pool(ctx, sim, 1)
    assert sim.diag()["n_alive_out"] > 2_000_000
    ctx.set_phase_times(True)
    say("[window] slab: 20 phase-timed steps in one call")
    ctx.step(20)
    sim.step(20)
    compare_state(ctx, sim, p, what="slab step 545")
    compare_pool(ctx, sim, 1)
    dg, do = ctx.get_diag(), sim.diag()
    assert dg["n_alive_out"] == do["n_alive_out"] and dg["sweeps_max"] == do["sweeps"]
    assert abs(dg["residual"]) <= 1e-12 * abs(dg["e_end"])


def test_lattice_full_size_across_a_pool_sort():
    """The 256^2 x 32 lattice from t = 0 for 20 steps (the 2-D pool sort runs
    every 16 steps): 4 steps, the autotuner, then 16 steps in one call."""
    p = W.c3_lattice()
    ctx = ugkwp.from_problem(p)
    sim = oracle.Sim(p)
    say("[window] lattice: 4 steps")
    ctx.step(4)
    sim.step(4)
    say(f"[window] lattice: autotuned {ctx.autotune()}")
    say("[window] lattice: 16 steps in one call")
    ctx.step(16)
    sim.step(16)
    compare_state(ctx, sim, p, what="lattice step 20")
    compare_pool(ctx, sim, 2)


def test_lattice_full_size_at_the_window_particle_count():
    """The lattice at the particle count of its timed window (6e7 particles,
    256^2 x 32): a seeded synthetic mid-run state (hot material around the
    pinned source, particles in the thin squares, see workloads) is given to
    both sides; the GPU then runs as the benchmark does (the autotuner on that
    pool, then 4 steps in one call) and every field, tally and particle is
    compared with the oracle's 4 steps from the same state."""
    p = W.c3_lattice()
    st = W.lattice_mid_run_state(p, 60_000_000)
    q = p.with_(T0=st["T0"], Tr0=st["Tr0"])
    say("[window] lattice: synthetic mid-run state of 6e7 particles to the GPU")
    ctx = ugkwp.from_problem(q)
    ctx.set_pool(st["pool"], st["births"], st["rhop"])
    say(f"[window] lattice: autotuned {ctx.autotune()}")
    say("[window] lattice: 4 steps in one call")
    ctx.get_totals(reset=True)
    ctx.step(4)
    sim = oracle.Sim(q)
    sim.set_pool(st["pool"], st["births"], st["rhop"])
    del st
    pushes = 0
    for _ in range(4):
        sim.step(1)
        d = sim.diag()
        pushes += d["n_alive_in"] + d["n_births"]
    tot = ctx.get_totals()
    assert tot["n_pushed"] == pushes > 200_000_000
    compare_state(ctx, sim, q, what="lattice mid-run state + 4 steps")
    compare_pool(ctx, sim, 2)
    dg, do = ctx.get_diag(), sim.diag()
    assert dg["n_alive_out"] == do["n_alive_out"] and dg["sweeps_max"] == do["sweeps"]
    assert abs(dg["residual"]) <= 1e-12 * abs(dg["e_end"])


def test_graph_replay_batch_matches_oracle():
    """HIP-graph replay of a batched context of uneven slabs against
    independent oracle runs of every instance."""
    probs = []
    rng = np.random.default_rng(31)
    for k, (nx, G) in enumerate([(37, 5), (130, 16), (64, 33), (9, 3)]):
        kl, kr = 10 ** rng.uniform(-2, 3, 2)
        xj = rng.uniform(0.2, 0.8)
        probs.append(W.slab(nx, G, lambda x, kl=kl, kr=kr, xj=xj: np.where(x < xj, kl, kr), dt=1e-3,
                            steps=0, w_ref=3e-5, seed=300 + k, pool_cap=1 << 18, name=f"gb{k}"))
    say("[window] graph replay of a batch of", len(probs))
    ctx = ugkwp.from_batch(probs, extra_flags=ugkwp.FLAG_GRAPH)
    sims = [oracle.Sim(q) for q in probs]
    for n in range(40):
        ctx.step(1)
        for s in sims:
            s.step(1)
        if n % 13 == 12 or n == 39:
            for k, (q, s) in enumerate(zip(probs, sims)):
                compare_state(ctx, s, q, inst=k, what=f"graph batch instance {k} step {n}")


def test_adjoint_full_workload_against_oracle():
    """The adjoint workload as stated: 128^2 x 16 log-normal medium, 100
    recorded steps from t = 0 in one call, then the adjoint of the material
    energy, against the oracle's adjoint of its own 100-step run."""
    p = W.c5_lognormal()
    V = (p.x1 - p.x0) / p.nx * (p.y1 - p.y0) / p.ny
    ctx = ugkwp.from_problem(p)
    say("[window] adjoint: 100 recorded steps")
    ctx.record(100)
    ctx.step(100)
    g = ctx.adjoint(V * p.cv).reshape(p.ncell, p.G)
    sim = oracle.Sim(p)
    sim.record(True)
    sim.step(100)
    o = sim.adjoint(V * p.cv)
    assert np.abs(o).max() > 0
    e = relerr(g, o)
    say(f"[window] adjoint: max-norm relative error {e:.2e}")
    assert e <= TOL


@pytest.mark.parametrize("which", ["slab_all_flags", "olson1d"])
def test_graph_replay_of_the_later_variants_matches_oracle(which):
    """HIP-graph replays with the second-order wave part, the iterate's wave flux and
    boundary particles, and with Olson's models (tabulated opacity, heat capacity, a
    source that switches off inside the run), against the oracle."""
    if which == "slab_all_flags":
        p = W.c1_marshak_like().with_(flags=W.FLAG_SLOPES | W.FLAG_WAVE_ITER | W.FLAG_BOUNDARY_PARTICLES,
                                      name="slab100_graph_all_flags")
        n = 24
    else:
        p = W.olson1d().with_(name="olson1d_graph")
        n = 60                                   # the source switches off at step 54 (c t = 2)
    say(f"[graph] {p.name}, {n} steps")
    ctx = ugkwp.from_problem(p, extra_flags=ugkwp.FLAG_GRAPH)
    sim = oracle.Sim(p)
    for k in range(n):
        ctx.step(1)
        sim.step(1)
        if (k + 1) % 12 == 0:
            compare_state(ctx, sim, p, what=f"{p.name} step {k}")
    compare_pool(ctx, sim, p.dim)
