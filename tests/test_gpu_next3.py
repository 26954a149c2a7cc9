"""GPU vs FP64 oracle for the second-order and implicit variants of the wave
part: MINMOD slopes (UGKWP_FLAG_SLOPES), the wave flux from each
source-iteration iterate (UGKWP_FLAG_WAVE_ITER) and Planckian boundary-source
particles (UGKWP_FLAG_BOUNDARY_PARTICLES), alone and together, in 1-D, 2-D and
batches.  Same bar as the other parity tests: integers bit-exact, every field,
tally and particle within 1e-10 of its array's max-norm."""
import numpy as np
import pytest

import oracle
from paper_2312_16981_amd import ugkwp
from paper_2312_16981_amd import workloads as W
from test_gpu_parity import compare_state, run_pair, say

pytestmark = pytest.mark.gpu
SL, WI, BP = W.FLAG_SLOPES, W.FLAG_WAVE_ITER, W.FLAG_BOUNDARY_PARTICLES


def _slab(**kw):
    return W.c1_marshak_like(**kw)


def _lognormal(**kw):
    p = dict(w_ref=2e-4, pool_cap=1 << 21, dt=2e-2)
    p.update(kw)
    return W.c5_lognormal(n=20, G=5, **p)


def _two_walls_2d(**kw):
    p = _lognormal(**kw)
    return p.with_(bc=[W.BC_PLANCK, W.BC_REFLECT, W.BC_PLANCK, W.BC_VACUUM], bcT=[1.0, 0.0, 0.7, 0.0])


@pytest.mark.parametrize("flags", [SL, WI, BP, SL | WI, SL | BP, SL | WI | BP])
def test_slab(flags):
    run_pair(_slab().with_(flags=flags, name=f"slab100_g10_f{flags}"), 12, every=4)


@pytest.mark.parametrize("flags", [SL, WI, BP, SL | WI | BP])
def test_lognormal_2d(flags):
    run_pair(_lognormal().with_(flags=flags, name=f"lognormal20_g5_f{flags}"), 6, every=3)


def test_two_planckian_walls_2d():
    run_pair(_two_walls_2d().with_(flags=SL | BP, name="two_walls_2d"), 6, every=3)


def test_with_linearized_iteration_and_temperature_dependent_opacity():
    p = W.slab(60, 8, lambda x: np.full_like(x, 20.0), dt=5e-3, steps=0, w_ref=2e-5, pool_cap=1 << 21,
               T_power=0.5, name="tdep_slab")
    p = p.with_(cv=np.full(60, 0.05))
    run_pair(p.with_(flags=W.FLAG_SI_LINEARIZED | SL | WI | BP), 8, every=4)


def test_with_joint_cells_numerical_collision_time():
    p = W.thick_thin_joint(nx=60, G=8, w_ref=4e-5, pool_cap=1 << 21)
    run_pair(p.with_(flags=SL | BP, name="thick_thin_slopes"), 10, every=5)


def test_lattice_with_pinned_cells():
    p = W.c3_lattice(n=24, G=5, dt=2e-2, w_ref=1e-5, pool_cap=1 << 21)
    run_pair(p.with_(flags=SL | WI, name="lattice24_slopes_iter"), 5)


def test_batch_of_uneven_instances():
    probs = []
    rng = np.random.default_rng(41)
    for k, (nx, G) in enumerate([(37, 5), (90, 16), (12, 3)]):
        kl, kr = 10 ** rng.uniform(-2, 3, 2)
        xj = rng.uniform(0.2, 0.8)
        probs.append(W.slab(nx, G, lambda x, kl=kl, kr=kr, xj=xj: np.where(x < xj, kl, kr), dt=1e-3, steps=0,
                            w_ref=3e-5, seed=700 + k, pool_cap=1 << 18, flags=SL | WI | BP, name=f"b3_{k}"))
    say("[next3] batch of", len(probs))
    ctx = ugkwp.from_batch(probs)
    sims = [oracle.Sim(q) for q in probs]
    for n in range(8):
        ctx.step(1)
        for s in sims:
            s.step(1)
    for k, (q, s) in enumerate(zip(probs, sims)):
        compare_state(ctx, s, q, inst=k, what=f"batch instance {k}")


def test_full_size_slab_with_slopes_and_boundary_particles():
    """The 2000 x 64 two-material slab with every variant on, 30 steps in one call."""
    p = W.c2_two_material().with_(flags=SL | WI | BP)
    ctx = ugkwp.from_problem(p)
    sim = oracle.Sim(p)
    say("[next3] full slab, 30 steps in one call")
    ctx.step(30)
    sim.step(30)
    compare_state(ctx, sim, p, what="slab2000 step 30")
    dg = ctx.get_diag()
    assert dg["inflow_particles"] > 0 and abs(dg["residual"]) <= 1e-12 * abs(dg["e_end"])


def test_recording_refused():
    for fl in (SL, WI, BP):
        ctx = ugkwp.from_problem(_slab().with_(flags=fl))
        with pytest.raises(ugkwp.UGKWPError):
            ctx.record(3)
