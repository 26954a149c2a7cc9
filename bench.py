"""Throughput benchmark of the UGKWP hot path on one MI355X.

Workload: the two-material slab (2000 cells x 64 log-spaced groups on
[0.01, 10], kappa = 0.01 | 1000 jump at x = 0.5, dt = 1e-4, Planckian left
wall at T = 1), advanced from t = 0 through a fixed 500-step spin-up that
fills the particle pool (set-up, untimed), then `--warmup` untimed steps,
then `--steps` timed steps.  A step is one full time step of the method
(sampling, particle push, wave flux, source iteration) over the whole mesh.

Prints one JSON line: particle-pushes/s over the timed steps (whole step,
inputs resident in HBM), cell-group source-iteration updates/s, the push
kernel's roofline against MI355X HBM bandwidth (8 TB/s) measured with HIP
events on the stream the kernel runs on, and the FP64 CPU oracle's rate on a
bounded sample of the same workload as a CPU baseline.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PUSH_BYTES_READ = 48       # x, mu, nu, w, id (8 B each) + cell word, group (4 B each)
PUSH_BYTES_WRITE = 12      # new position and cell word of a survivor (updated in place)
PUSH_BYTES_DEAD = 4        # empty-slot mark of a particle absorbed or gone
SPINUP = 500


def cpu_baseline(prob, budget_s=15.0):
    """The oracle as it stands, single thread, on the first steps of the same run."""
    import oracle
    sim = oracle.Sim(prob)
    pushes = 0
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and steps < prob.steps:
        sim.step(1)
        pushes += sim.diag()["n_alive_in"] + sim.diag()["n_births"]
        steps += 1
    dt = time.perf_counter() - t0
    return {"value": pushes / dt, "unit": "particle-pushes/s", "cores": 1, "kind": "oracle",
            "sample": f"steps 0-{steps - 1} of the same slab run from t=0 ({pushes} pushes, "
                      f"{dt:.1f} s, single thread)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--sort-interval", type=int, default=0,
                    help="steps between counting sorts of the pool (0 = library default)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2312_16981_amd import ugkwp
    from paper_2312_16981_amd import workloads as W

    torch.cuda.set_device(0)
    prob = W.c2_two_material()
    stream = torch.cuda.current_stream()
    ctx = ugkwp.from_problem(prob, stream=stream.cuda_stream, sort_interval=args.sort_interval)
    ncg = prob.ncell * prob.G

    ctx.step(SPINUP)
    for _ in range(args.warmup):
        ctx.step(1)
    torch.cuda.synchronize()

    pushes = 0
    survivors = 0
    sweeps = 0
    ms_push = 0.0
    ms_si = 0.0
    ms_sort = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.step(1)
        d = ctx.get_diag()
        pushes += d["n_pushed"]
        survivors += d["n_alive_out"]
        sweeps += d["sweeps_max"]
        ms_push += d["ms_push"]
        ms_si += d["ms_si"]
        ms_sort += d["ms_sort"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    value = pushes / elapsed
    algo_bytes = (PUSH_BYTES_READ * pushes + PUSH_BYTES_WRITE * survivors
                  + PUSH_BYTES_DEAD * (pushes - survivors))
    achieved = algo_bytes / (ms_push * 1e-3) / 1e9
    out = {
        "metric": "particle-pushes/s (whole UGKWP step, FP64, parity 1e-10 vs oracle)",
        "value": value,
        "unit": "particle-pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / max(args.steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"two-material slab {prob.nx} cells x {prob.G} groups, dt=1e-4, "
                               f"kappa 0.01|1000 jump at x=0.5, steps {SPINUP + args.warmup}-"
                               f"{SPINUP + args.warmup + args.steps - 1} of the run from t=0",
                   "particles_per_step": pushes / max(args.steps, 1),
                   "parallelism": "single GPU"},
        "cell_group_updates_per_s": ncg * sweeps / elapsed,
        "cell_group_updates_per_s_si_only": ncg * sweeps / (ms_si * 1e-3) if ms_si > 0 else None,
        "push_kernel_pushes_per_s": pushes / (ms_push * 1e-3),
        "sweeps_per_step": sweeps / max(args.steps, 1),
        "ms_per_step_phases": {"push": ms_push / max(args.steps, 1), "si": ms_si / max(args.steps, 1),
                               "sort": ms_sort / max(args.steps, 1)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_push<1>", "algorithmic_bytes_per_push":
                     f"{PUSH_BYTES_READ} read + {PUSH_BYTES_WRITE} per survivor + "
                     f"{PUSH_BYTES_DEAD} per absorbed/escaped particle"},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
