"""Throughput benchmark of the UGKWP hot path on one MI355X.

Workloads (--workload):
  lattice  (default) 2-D block lattice 256 x 256 cells x 32 groups on [0,7]^2
           with a pinned central source, dt = 1e-3, 500 steps: the timed steps
           are the last of the 500 (steps 480-499 with --steps 20 --warmup 5),
           where the pool holds ~6e7 particles
  slab     two-material slab: 2000 cells x 64 log-spaced groups on
           [0.01, 10], kappa = 0.01 | 1000 jump at x = 0.5, dt = 1e-4,
           Planckian left wall at T = 1
  batch    512 independent slabs of 64..4096 cells and 16/32/64 groups in one
           context (one launch per kernel per step); --per-instance steps the
           same instances in 512 separate contexts instead
  adjoint  2-D 128 x 128 cells x 16 groups, log-normal opacity, dt = 1e-3:
           --steps recorded steps from t = 0 (default 100), then the adjoint
           of the frozen-tally macroscopic map (dJ/dkappa of the material energy)

Each run advances from t = 0 through a fixed spin-up (set-up, untimed) that
fills the particle pool, then `--warmup` untimed steps, then `--steps` timed
steps.  A step is one full time step of the method (sampling, particle push,
wave flux, source iteration) over every instance.

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
PUSH_BYTES_READ = 44       # x, mu, nu, w, id and group word (8 B each) + cell word (4 B)
PUSH_BYTES_WRITE = 12      # new position and cell word of a survivor (updated in place)
PUSH_BYTES_DEAD = 4        # empty-slot mark of a particle absorbed or gone
SPINUP = {"slab": 500, "lattice": 300, "batch": 100, "adjoint": 0, "thickthin": 200, "marshak": 100, "larsen": 100,
          "olson1d": 0, "olson2d": 0}
ADJ_SWEEP_BYTES = 40       # rbar, sigma, phi' and two face coefficients per (cell, group) update (lambda is formed from sigma)
SI_SWEEP_BYTES = 64        # Q, lambda, sigma, phi^k, rho^k, one face D read; rho^{k+1}, phi^{k+1} written

# HBM bytes per push of k_push measured with rocprofv3 FETCH_SIZE / WRITE_SIZE,
# each scaled by its reading for a plain 1 GiB copy (FETCH_SIZE x 2.0, WRITE_SIZE
# x 1.0), over the windows of the profiles under profiles/.  They hold only for
# the push kernel sources they were taken with (SHA-256 prefix below); any change
# to those sources makes bench.py report the traffic as unknown.
PUSH_SOURCES = ("kernels.hip", "device_math.hpp", "device_common.hpp", "common.hpp")
PUSH_TRAFFIC = {
    "slab": {"sources": "130a38c77fd81f1c", "read_per_push": 45.04, "write_per_push": 12.89},
    "lattice": {"sources": "130a38c77fd81f1c", "read_per_push": 62.23, "write_per_push": 21.64},
}


def push_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in PUSH_SOURCES:
        with open(os.path.join(ROOT, "paper_2312_16981_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]
BYTES_2D = (60, 20, 4)     # 2-D: x, y, ox, oy, nu, w, id and group word + cell word; writes x, y, cell word


def cpu_info():
    """Host CPU model, logical CPUs and the CPUs this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count(), len(os.sched_getaffinity(0))


class pinned_to_one_cpu:
    """Run the enclosed block on one CPU (the first this process may use): the
    oracle is single-threaded, and the pinning keeps the scheduler from moving it."""

    def __enter__(self):
        self.old = os.sched_getaffinity(0)
        self.cpu = min(self.old)
        os.sched_setaffinity(0, {self.cpu})
        return self

    def __exit__(self, *exc):
        os.sched_setaffinity(0, self.old)


def cpu_baseline_window(prob, n_particles, budget_s=15.0):
    """The oracle as it stands, single thread pinned to one CPU, on the
    lattice at the timed window's particle count: from the seeded synthetic
    mid-run state with the window's pool size (workloads.lattice_mid_run_state),
    steps until the budget is spent (at least one)."""
    import oracle
    from paper_2312_16981_amd import workloads as W
    st = W.lattice_mid_run_state(prob, int(n_particles))
    q = prob.with_(T0=st["T0"], Tr0=st["Tr0"])
    sim = oracle.Sim(q)
    sim.set_pool(st["pool"], st["births"], st["rhop"])
    del st
    pushes = steps = cgu = 0
    ncg = prob.ncell * prob.G
    with pinned_to_one_cpu() as pin:
        t0 = time.perf_counter()
        while steps == 0 or time.perf_counter() - t0 < budget_s:
            sim.step(1)
            d = sim.diag()
            pushes += d["n_alive_in"] + d["n_births"]
            cgu += ncg * d["sweeps"]
            steps += 1
        dt = time.perf_counter() - t0
    model, ncpu, _ = cpu_info()
    return {"value": pushes / dt, "unit": "particle-pushes/s", "cores": 1, "kind": "oracle",
            "cell_group_updates_per_s": cgu / dt,
            "sample": f"{steps} steps of the 256x256x32 lattice from a seeded synthetic state holding the "
                      f"timed window's {int(n_particles)} particles ({pushes} pushes, {dt:.1f} s)",
            "cpu_model": model, "host_logical_cpus": ncpu, "pinned_cpu": pin.cpu}


def cpu_baseline(probs, budget_s=15.0):
    """The oracle as it stands, single thread pinned to one CPU, on the first
    steps of the same run (for a batch: the instances in turn, each from t = 0)."""
    import oracle
    pin = pinned_to_one_cpu().__enter__()
    pushes = 0
    steps = 0
    cgu = 0
    t0 = time.perf_counter()
    sims = []
    done = False
    for prob in probs:
        sim = oracle.Sim(prob)
        sims.append(sim)
        for _ in range(prob.steps):
            sim.step(1)
            d = sim.diag()
            pushes += d["n_alive_in"] + d["n_births"]
            cgu += prob.ncell * prob.G * d["sweeps"]
            steps += 1
            if time.perf_counter() - t0 >= budget_s:
                done = True
                break
        if done:
            break
    dt = time.perf_counter() - t0
    pin.__exit__()
    what = (f"steps 0-{steps - 1} of the same run from t=0" if len(probs) == 1 else
            f"{steps} instance-steps of the first {len(sims)} instances from t=0")
    model, ncpu, _ = cpu_info()
    return {"value": pushes / dt, "unit": "particle-pushes/s", "cores": 1, "kind": "oracle",
            "cell_group_updates_per_s": cgu / dt,
            "sample": f"{what} ({pushes} pushes, {dt:.1f} s, single thread)",
            "cpu_model": model, "host_logical_cpus": ncpu, "pinned_cpu": pin.cpu}


def cpu_baseline_adjoint(prob, budget_s=15.0):
    """The oracle's adjoint as it stands, single thread: a forward run recorded
    from t = 0 for as many steps as fit in half the budget, then its adjoint."""
    import oracle
    sim = oracle.Sim(prob)
    sim.record(True)
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < 0.5 * budget_s and steps < prob.steps:
        sim.step(1)
        steps += 1
    V = cell_volume(prob)
    t1 = time.perf_counter()
    sim.adjoint(V * prob.cv)
    dt = time.perf_counter() - t1
    upd = sim.adjoint_updates()
    return {"value": upd / dt, "unit": "cell-group updates/s", "cores": 1, "kind": "oracle",
            "sample": f"adjoint of steps 0-{steps - 1} of the same run ({upd} cell-group updates of the "
                      f"transposed iteration, {dt:.1f} s, single thread)"}


def cell_volume(p):
    return (p.x1 - p.x0) / p.nx * ((p.y1 - p.y0) / p.ny if p.dim == 2 else 1.0)


def run_adjoint(args, stream):
    """Record --steps steps from t = 0, then time the adjoint (after one untimed
    warm-up of both on a short run)."""
    import numpy as np
    import torch
    from paper_2312_16981_amd import ugkwp
    from paper_2312_16981_amd import workloads as W
    prob = W.c5_lognormal()
    nsteps = args.steps
    ctx = ugkwp.from_problem(prob, stream=stream.cuda_stream)
    dJdT = cell_volume(prob) * np.asarray(prob.cv)
    ctx.record(max(args.warmup, 1))
    ctx.step(max(args.warmup, 1))
    ctx.adjoint(dJdT)
    ctx.set_material(prob.cv, prob.T0, prob.Tr0, prob.pinned)      # back to t = 0
    ctx.record(nsteps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(nsteps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    ctx.adjoint(dJdT)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    st = ctx.last_adjoint
    cgu = st["cell_group_updates"]
    ms_sw = st["ms_sweeps"]
    achieved = ADJ_SWEEP_BYTES * cgu / (ms_sw * 1e-3) / 1e9
    out = {
        "metric": "cell-group updates/s (adjoint of the frozen-tally macroscopic map, FP64, parity 1e-10 vs oracle)",
        "value": cgu / t_adj,
        "unit": "cell-group updates/s",
        "n_gpus": 1,
        "steps": nsteps,
        "warmup": args.warmup,
        "ms_per_step": t_adj * 1e3 / nsteps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2-D log-normal opacity {prob.nx}x{prob.ny} cells x {prob.G} groups, dt=1e-3, "
                               f"adjoint of steps 0-{nsteps - 1} (dJ/dkappa of the material energy)",
                   "cell_groups": prob.ncell * prob.G, "parallelism": "single GPU"},
        "forward_ms_per_step_recording": t_fwd * 1e3 / nsteps,
        "adjoint_ms": t_adj * 1e3,
        "adjoint_gpu_ms": st["ms"],
        "adjoint_sweeps_per_step": cgu / (prob.ncell * prob.G) / nsteps,
        "sweep_ms": ms_sw,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_adj_sweep",
                     "algorithmic_bytes_per_update": ADJ_SWEEP_BYTES},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_adjoint(prob, args.cpu_budget)
    print(json.dumps(out), flush=True)


def summarize_trace(csv_path, steps, push_kernel="k_push"):
    """Text summary of a rocprofv3 kernel trace of this benchmark restricted to
    the timed steps: the window runs from the push dispatch that begins the
    timed steps to the one that begins the phase-timed steps after them
    (min(steps, 50) of them, the last pushes of the run).  Prints per-kernel
    calls, total and average duration in that window."""
    import csv
    rows = list(csv.DictReader(open(csv_path)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    pushes = [r for r in rows if push_kernel in r["Kernel_Name"]]
    nph = min(steps, 50)
    if len(pushes) < steps + nph:
        raise SystemExit(f"trace holds {len(pushes)} push dispatches, fewer than {steps} + {nph} steps")
    t0 = int(pushes[-steps - nph]["Start_Timestamp"])
    t1 = int(pushes[-nph]["Start_Timestamp"])
    stats = {}
    for r in rows:
        if int(r["Start_Timestamp"]) < t0 or int(r["Start_Timestamp"]) >= t1:
            continue
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        e = stats.setdefault(r["Kernel_Name"], [0, 0, 0, 1 << 62])
        e[0] += 1
        e[1] += d
        e[2] = max(e[2], d)
        e[3] = min(e[3], d)
    total = sum(v[1] for v in stats.values())
    lines = [f"timed window: {steps} steps before the last {nph} ({len(pushes)} push dispatches in the trace)",
             f"{'kernel':70s} {'calls':>6s} {'total_us':>10s} {'avg_us':>9s} {'min_us':>8s} {'max_us':>8s} {'pct':>6s}"]
    for name, (n, tot, mx, mn) in sorted(stats.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"{name[:70]:70s} {n:6d} {tot / 1e3:10.1f} {tot / n / 1e3:9.2f} {mn / 1e3:8.2f} "
                     f"{mx / 1e3:8.2f} {100.0 * tot / total:6.2f}")
    return "\n".join(lines)


def summarize_counters(csv_path, steps, kernel="k_push"):
    """Per-dispatch average of each counter in a rocprofv3 --pmc CSV over the
    dispatches of the kernel whose name contains `kernel` in the timed steps
    (the `steps` before the min(steps, 50) phase-timed ones at the end, as in
    summarize_trace; the last `steps` if the run is shorter), and over the
    largest dispatches of every other kernel (for a copy-probe run)."""
    import csv
    rows = list(csv.DictReader(open(csv_path)))
    by = {}
    for r in rows:
        key = (r["Kernel_Name"], r["Counter_Name"])
        by.setdefault(key, []).append((int(r.get("Dispatch_Id", r.get("Correlation_Id", 0))),
                                       float(r["Counter_Value"]), int(r.get("Grid_Size", 0))))
    lines = [f"{'kernel':60s} {'counter':12s} {'dispatches':>10s} {'avg_KiB':>14s} {'grid':>10s}"]
    for (name, ctr), v in sorted(by.items()):
        v.sort()
        if kernel in name:
            nph = min(steps, 50)
            sel = v[-steps - nph:-nph] if len(v) >= steps + nph else v[-steps:]
        else:
            gmax = max(g for _, _, g in v)
            sel = [t for t in v if t[2] == gmax]
        avg = sum(t[1] for t in sel) / len(sel)
        lines.append(f"{name[:60]:60s} {ctr:12s} {len(sel):10d} {avg:14.1f} {sel[-1][2]:10d}")
    return "\n".join(lines)


def batched_vs_per_instance(probs, stream, spin, nsteps=20, sort_interval=0):
    """The batch's instances as one batched context and as one context each,
    both fresh from t = 0 and stepped to `spin`, then `nsteps` steps timed on
    each (same work: the same seeds give the same particles)."""
    import torch
    from paper_2312_16981_amd import ugkwp
    out = {}
    for mode in ("batched", "per_instance"):
        if mode == "batched":
            ctxs = [ugkwp.from_batch(probs, stream=stream.cuda_stream, pool_capacity=1 << 26,
                                     sort_interval=sort_interval)]
        else:
            ctxs = [ugkwp.from_problem(p, stream=stream.cuda_stream, sort_interval=sort_interval) for p in probs]
        for c in ctxs:
            c.step(spin)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in ctxs:
            c.step(nsteps)
        torch.cuda.synchronize()
        out[mode] = (time.perf_counter() - t0) * 1e3 / nsteps
        del ctxs
    return {"steps": f"{spin}-{spin + nsteps - 1} of fresh runs from t=0",
            "batched_ms_per_step": out["batched"], "per_instance_ms_per_step": out["per_instance"],
            "speedup": out["per_instance"] / out["batched"]}


def copy_probe(mib=1024, reps=5):
    """A plain elementwise copy (dst = -src, float64) of `mib` MiB read and
    `mib` MiB written, repeated: the known-size reference for HBM byte counters,
    and the copy rate this GPU reaches (read + written bytes over the mean time
    of the repetitions after the first, by events on torch's stream)."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps - 1):
        torch.neg(src, out=dst)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / max(1, reps - 1)
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "reps": reps,
                      "copy_ms": ms, "copy_GBps": 2 * n * 8 / ms / 1e6}), flush=True)


def workload_name(wl, probs, spin, args):
    first, last = spin + args.warmup, spin + args.warmup + args.steps - 1
    if wl == "slab":
        p = probs[0]
        return (f"two-material slab {p.nx} cells x {p.G} groups, dt=1e-4, kappa 0.01|1000 jump at "
                f"x=0.5, steps {first}-{last} of the run from t=0")
    if wl == "marshak":
        p = probs[0]
        return (f"homogeneous Marshak wave {p.nx} cells x {p.G} groups on [0,5], sigma = 10/(nu^3 sqrt(T)), "
                f"C_v = 0.1, reflective right wall, dt=dx/c, steps {first}-{last} of the run from t=0")
    if wl == "larsen":
        p = probs[0]
        return (f"Larsen three-region slab {p.nx} cells x {p.G} groups on [0,4], sigma = gamma0 (1 - e^(-nu/T))/nu^3, "
                f"gamma0 1|1000|1, C_v = 0.05109/a (paper units scaled to c = a = 1), tau_num C = 1e3, dt=dx/c, "
                f"steps {first}-{last} of the run from t=0")
    if wl == "thickthin":
        p = probs[0]
        return (f"thick-to-thin slab {p.nx} cells x {p.G} groups on [0,1.5], kappa 1000|10 jump at x=0.5, "
                f"dt=dx/c, numerical collision time of the joint cells C=1e5, steps {first}-{last} of the run "
                f"from t=0")
    if wl in ("olson1d", "olson2d"):
        p = probs[0]
        return (f"Olson {p.dim}-D foam problem {p.nx}x{p.ny} cells x {p.G} groups (tabulated foam"
                f"{' and aluminium' if p.dim == 2 else ''} opacity, Olson heat capacity, Planckian source), "
                f"dt=dx/c, linearized source iteration, steps {first}-{last} of the run from t=0")
    if wl == "lattice":
        p = probs[0]
        return (f"2-D lattice {p.nx}x{p.ny} cells x {p.G} groups, dt=1e-3, kappa 100|1 squares, "
                f"pinned source, steps {first}-{last} of the run from t=0")
    return (f"{len(probs)} independent slabs (64-4096 cells, 16/32/64 groups, kappa jump), dt=1e-4, "
            f"steps {first}-{last} of the run from t=0")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--summarize-trace", metavar="KERNEL_TRACE_CSV",
                    help="print the kernel summary of a rocprofv3 trace of this benchmark over the "
                         "last --steps steps, and exit")
    ap.add_argument("--summarize-counters", metavar="COUNTER_CSV",
                    help="print per-dispatch counter averages of a rocprofv3 --pmc CSV of this "
                         "benchmark over the last --steps push dispatches, and exit")
    ap.add_argument("--copy-probe", type=int, metavar="MIB", default=0,
                    help="run a plain device copy of MIB MiB (HBM counter reference) and exit")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=-1,
                    help="timed steps (default 20 on the lattice, 400 on the other forward workloads; "
                         "for the adjoint workload the recorded steps, 100)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--workload", choices=("lattice", "slab", "batch", "adjoint", "thickthin", "marshak", "larsen",
                                           "olson1d", "olson2d"),
                    default="lattice")
    ap.add_argument("--per-instance", action="store_true",
                    help="batch workload: one context per instance instead of one batched context")
    ap.add_argument("--no-compare", action="store_true",
                    help="batch workload: leave out the batched-vs-per-instance comparison (for kernel traces "
                         "of the batched run alone)")
    ap.add_argument("--spinup", type=int, default=-1, help="untimed steps from t=0 (default per workload)")
    ap.add_argument("--sort-interval", type=int, default=0,
                    help="steps between counting sorts of the pool (0 = library default)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default push launch shape instead of tuning it after the spin-up")
    ap.add_argument("--si-linearized", action="store_true",
                    help="linearized source iteration (a local Newton step per sweep; same fixed point)")
    ap.add_argument("--graph", action="store_true",
                    help="replay the launches before the push and the source-iteration sweeps from "
                         "captured HIP graphs")
    args = ap.parse_args()
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace, args.steps))
        return
    if args.summarize_counters:
        print(summarize_counters(args.summarize_counters, args.steps))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        copy_probe(args.copy_probe)
        return

    import torch
    from paper_2312_16981_amd import ugkwp
    from paper_2312_16981_amd import workloads as W

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    wl = args.workload
    if args.steps < 0:
        # the Olson problems: their whole runs (c t = 4 in 1-D, 3 in 2-D) after the warm-up
        args.steps = {"adjoint": 100, "lattice": 20, "olson1d": 102, "olson2d": 220}.get(wl, 400)
    if wl == "adjoint":
        run_adjoint(args, stream)
        return
    if wl == "slab":
        probs = [W.c2_two_material()]
    elif wl == "lattice":
        probs = [W.c3_lattice()]
    elif wl == "thickthin":
        probs = [W.thick_thin_joint()]
    elif wl == "marshak":
        probs = [W.marshak()]
    elif wl == "larsen":
        probs = [W.larsen()]
    elif wl == "olson1d":
        probs = [W.olson1d()]
    elif wl == "olson2d":
        probs = [W.olson2d()]
    else:
        probs = W.c4_batch()
    if args.si_linearized:
        probs = [p.with_(flags=p.flags | W.FLAG_SI_LINEARIZED) for p in probs]
    ncg = sum(p.ncell * p.G for p in probs)
    if args.spinup >= 0:
        spin = args.spinup
    elif wl == "lattice":
        # the timed steps end where the workload's 500-step run ends
        spin = max(0, probs[0].steps - args.warmup - args.steps)
    else:
        spin = SPINUP[wl]
    xf = ugkwp.FLAG_GRAPH if args.graph else 0
    if wl == "batch" and args.per_instance:
        ctxs = [ugkwp.from_problem(p, stream=stream.cuda_stream, sort_interval=args.sort_interval, extra_flags=xf)
                for p in probs]
    elif wl == "batch":
        ctxs = [ugkwp.from_batch(probs, stream=stream.cuda_stream, pool_capacity=1 << 26,
                                 sort_interval=args.sort_interval, extra_flags=xf)]
    else:
        ctxs = [ugkwp.from_problem(probs[0], stream=stream.cuda_stream, sort_interval=args.sort_interval,
                                   extra_flags=xf)]

    for c in ctxs:
        c.step(spin)
    tuned = None
    # (the Olson runs start without particles: nothing to tune on)
    if not args.no_autotune and not wl.startswith("olson"):
        tuned = [c.autotune() for c in ctxs]
    # time the push of every timed step where a push lasts a millisecond (2-D);
    # in 1-D one step in 4 (each event pair adds a few microseconds to a step)
    for c in ctxs:
        c.set_push_timing(1 if probs[0].dim == 2 else 4)
    for c in ctxs:
        c.step(args.warmup)
        c.get_totals(reset=True)
    torch.cuda.synchronize()

    # the timed steps: one library call per context (steps run back to back inside it)
    t0 = time.perf_counter()
    for c in ctxs:
        c.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tots = [c.get_totals() for c in ctxs]
    pushes = sum(t["n_pushed"] for t in tots)
    survivors = sum(t["n_survived"] for t in tots)
    sweeps = sum(t["sweeps_sum"] for t in tots)
    # the push is timed with a HIP event pair on one step in 8 of the timed steps
    # (each event costs a few microseconds of GPU time); its rates use those steps
    ms_push = sum(t["ms_push"] for t in tots)
    n_timed = sum(t["push_timed"] for t in tots)
    pushes_t = sum(t["n_pushed_timed"] for t in tots)
    surv_t = sum(t["n_survived_timed"] for t in tots)
    # phase breakdown: a further stretch of steps with every phase timed (each
    # phase event costs a few microseconds, so the timed steps above time the push only)
    nph = min(args.steps, 50)
    for c in ctxs:
        c.set_phase_times(True)
        c.get_totals(reset=True)
        c.step(nph)
    ptot = [c.get_totals() for c in ctxs]
    ph = {k: sum(t[k] for t in ptot) / max(nph, 1) for k in ("ms_sample", "ms_push", "ms_macro", "ms_si", "ms_sort")}
    # cell-group updates: every instance's cell-groups times its own sweep count
    cgu = sum(t["cg_updates"] for t in tots)
    ph_cgu = sum(t["cg_updates"] for t in ptot)
    ms_si_ph = sum(t["ms_si"] for t in ptot)

    value = pushes / elapsed
    br, bw, bd = (PUSH_BYTES_READ, PUSH_BYTES_WRITE, PUSH_BYTES_DEAD) if probs[0].dim == 1 else BYTES_2D
    algo_bytes = br * pushes_t + bw * surv_t + bd * (pushes_t - surv_t)
    achieved = algo_bytes / (ms_push * 1e-3) / 1e9
    traffic = None
    tr = PUSH_TRAFFIC.get(wl)
    if tr and not args.per_instance and tr["sources"] == push_sources_digest():
        traffic = (tr["read_per_push"] + tr["write_per_push"]) * pushes_t / max(n_timed, 1)
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
        "config": {"workload": workload_name(wl, probs, spin, args),
                   "particles_per_step": pushes / max(args.steps, 1),
                   "cell_groups": ncg,
                   "parallelism": "single GPU" + (", per-instance contexts" if args.per_instance else ""),
                   "launch": "HIP graph replays" if args.graph else "kernels launched directly",
                   "source_iteration": ("linearized (Newton step per sweep)" if probs[0].flags & W.FLAG_SI_LINEARIZED
                                        else "literal"),
                   "push_shape": ("default (occupancy-filled grid of 256-thread blocks, 4 particles per thread)"
                                  if tuned is None else
                                  f"autotuned: {tuned[0]['blocks']} blocks of {tuned[0]['threads']} threads, "
                                  f"{tuned[0]['ppt']} particles per thread "
                                  f"({tuned[0]['us_best']:.1f} vs {tuned[0]['us_default']:.1f} us default)"
                                  + (f", per context ({len(tuned)})" if len(tuned) > 1 else ""))},
        "cell_group_updates_per_s": cgu / elapsed,
        "cell_group_updates_per_s_si_only": ph_cgu / (ms_si_ph * 1e-3) if ms_si_ph > 0 else None,
        "push_kernel_pushes_per_s": pushes_t / (ms_push * 1e-3),
        "push_kernel_avg_us": ms_push * 1e3 / max(n_timed, 1),
        "push_timed_steps": n_timed,
        "sweeps_per_step": sweeps / max(args.steps, 1) / len(probs),
        "ms_per_step_phases": {"sample": ph["ms_sample"], "push": ph["ms_push"], "macro": ph["ms_macro"],
                               "si": ph["ms_si"], "sort": ph["ms_sort"],
                               "from": f"{nph} further steps with every phase timed"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (measured bytes per push x pushes per launch)",
                     "algorithmic_bytes_per_launch": algo_bytes / max(n_timed, 1),
                     "kernel": f"k_push<{probs[0].dim}>", "algorithmic_bytes_per_push":
                     f"{br} read + {bw} per survivor + {bd} per absorbed/escaped particle"},
    }
    if ms_si_ph > 0:
        # the source-iteration phase as a second roofline object (every sweep and decide
        # launch between two events, from the phase-timed steps)
        si_ach = SI_SWEEP_BYTES * ph_cgu / (ms_si_ph * 1e-3) / 1e9
        out["roofline_si"] = {"bound": "hbm", "achieved": si_ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": si_ach / HBM_PEAK_GBS, "kernel": "k_si_sweep (the source-iteration phase)",
                              "algorithmic_bytes_per_update": SI_SWEEP_BYTES,
                              "from": f"{nph} further steps with every phase timed"}
    if wl == "batch" and ms_si_ph > 0:
        # the source iteration dominates the batched step: its phase (every sweep and
        # decide launch between two events) is the roofline kernel, the push is kept
        si_ach = SI_SWEEP_BYTES * ph_cgu / (ms_si_ph * 1e-3) / 1e9
        out["roofline_push"] = out["roofline"]
        out["roofline"] = {"bound": "hbm", "achieved": si_ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": si_ach / HBM_PEAK_GBS, "traffic": None,
                           "kernel": "k_si_sweep (the source-iteration phase: sweeps and decides)",
                           "algorithmic_bytes_per_update": SI_SWEEP_BYTES,
                           "from": f"{nph} further steps with every phase timed"}
    if wl == "batch" and not args.per_instance and not args.no_compare:
        del ctxs
        out["batched_vs_per_instance"] = batched_vs_per_instance(probs, stream, spin, 20, args.sort_interval)
    if not args.no_cpu_baseline:
        if wl == "lattice":
            out["cpu_baseline"] = cpu_baseline_window(probs[0], pushes / max(args.steps, 1), args.cpu_budget)
        else:
            out["cpu_baseline"] = cpu_baseline(probs, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
