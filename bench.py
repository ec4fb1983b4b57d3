"""Throughput of the PIC-MCC particle step on one MI355X.

Workload (default): the large single discharge -- 6 cm gap, 4096 cells, O2 at
100 Pa / 300 K, 400 V at 13.56 MHz, dt = T_rf/8000, 2^25 macro particles
(charge-neutral split 40 % e, 10 % O-, 50 % O2+), FP32 particle state, 24-bit
fixed-point charge, FP64 field solve.  A step is one pass of the whole hot
path: field solve, fused gather/push/absorb/null-collision MCC/deposit of every
species, partner reactions, births, and every 10th step the cell sort followed
by the intra-species Coulomb collisions.  Before the W warm-up steps the
discharge gets a warm start of --warm-start-cycles rf cycles (default 1:
8000 steps, whose first ~1000 are the autotuner's trials of launch shapes and
grids); default W = 2000 and K = 40000 (5 rf cycles timed).

Prints one JSON line.  ``value`` is particle pushes per second over the timed
steps (inputs resident in HBM, wall clock between two stream synchronisations).
``roofline`` prices the fused particle kernel (gather, push, absorption,
null-collision MCC, deposit) against HBM with the algorithmic bytes of a
particle step: the whole particle state read and written, read cell 4 + off 4
+ v 12 + id 8, write cell 4 + off 4 + v 12 = 48 B in FP32 (80 B in FP64), times
the particles pushed per launch, divided by the kernel's average duration from
HIP events recorded on the library's stream around every 8th launch of the
timed steps (``--time-every``: the two event records add a gap of a few
microseconds to each step they bracket, so timing every launch would slow the
measured step; one fused-kernel launch per step).  The kernel
itself never touches vy and vz of the ~95 % of particles that do not collide
(the field is along x); ``achieved_touched``/``frac_touched`` count only the
32 B (FP32; 48 B in FP64) it must move for every particle.  ``traffic`` is the
kernel's HBM bytes per launch from rocprofv3 counters (profiles/, taken in a
separate run of the same kernel sources; null when the sources changed since),
and ``frac_traffic`` the fraction of peak those bytes reach.  ``host`` names the
CPU model and core counts; the CPU baseline's all-cores leg uses every core
available to the process.

Other modes: ``--workload sweep`` (many discharges advanced together),
``--workload serve`` (the serving loop over a request stream),
``--workload ablation`` (the metastable pair C = 0 / C = 1/6 on the production
discharge); ``--coulomb-inter`` adds the unlike-species Coulomb pass to a
single-discharge run and reports its longest collision chains; ``--dsmc``
replaces the null-collision MCC of every push by the paper's per-cell
collision list every sort_every steps (the push kernel then moves and deposits
only, and the roofline prices it with the same bytes).
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_STEP = {"fp32": 48, "fp64": 80}      # whole particle state read and written
BYTES_TOUCHED = {"fp32": 32, "fp64": 48}       # cell, off, vx read and written, id read
TRAFFIC_FILES = {"fp32": os.path.join(ROOT, "profiles", "traffic_k_push.json"),
                 "fp64": os.path.join(ROOT, "profiles", "traffic_k_push_fp64.json")}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_0705_0495_amd", "csrc", f)
                  for f in ("pic_kernels.hpp", "pic_list.hpp", "pic.hip")]


def kernel_source_sha():
    """Hash of the HIP sources' code (comments and blank lines left out):
    counter files name the code they were taken from."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        text = open(f, encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in text.splitlines()]
        h.update("\n".join(ln for ln in lines if ln.strip()).encode())
    return h.hexdigest()[:16]


def host_info():
    """CPU model and core counts of the host the benchmark runs on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "cores_available": len(os.sched_getaffinity(0))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--workload", default="large", choices=["small", "prod", "large", "sweep", "serve", "ablation"])
    ap.add_argument("--cycles", type=int, default=20, help="ablation: rf cycles per run")
    ap.add_argument("--requests", type=int, default=32, help="serve: requests in the stream")
    ap.add_argument("--rate", type=float, default=4.0, help="serve: Poisson arrivals per second (0: all at once)")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="serve: device memory for particle stores")
    ap.add_argument("--max-cycles", type=int, default=400, help="serve: rf cycles per request at most")
    ap.add_argument("--stream", default="served", choices=["served", "sweep"], help="serve: request distribution")
    ap.add_argument("--discharges", type=int, default=64, help="sweep: number of discharges")
    ap.add_argument("--eager", action="store_true", help="sweep: no graph replay")
    ap.add_argument("--sequential", action="store_true", help="sweep: also time the discharges one after another")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the occupancy-derived push grid")
    ap.add_argument("--dsmc", action="store_true",
                    help="collisions (4)-(19) as the per-cell list of Sec. II every sort_every steps")
    ap.add_argument("--coulomb-inter", action="store_true",
                    help="large/prod/small: unlike-species Coulomb collisions as well (off in the paper's runs)")
    ap.add_argument("--cpu-steps", type=int, default=800)
    ap.add_argument("--cpu-scale", type=float, default=1.0 / 32)
    ap.add_argument("--cpu-cores", type=int, default=0,
                    help="all-cores baseline: oracle instances (0: every core available to the process)")
    ap.add_argument("--warm-start-cycles", type=float, default=1.0,
                    help="large/prod/small: rf cycles run before the warm-up (the discharge's warm start)")
    ap.add_argument("--time-every", type=int, default=8,
                    help="HIP events around every n-th launch of the fused kernel in the timed steps")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the discharge is not sharded "
              "across GPUs.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "sweep":
        return sweep_main(args)
    if args.workload == "serve":
        return serve_main(args)
    if args.workload == "ablation":
        return ablation_main(args)
    from paper_0705_0495_amd import Discharge
    from pic_inputs import build_tables, workload

    wl = workload(args.workload)
    if args.coulomb_inter:
        wl = dataclasses.replace(wl, coulomb_inter=True)
    if args.dsmc:
        wl = dataclasses.replace(wl, dsmc=True)
    sig, thr, loss = build_tables()
    t0 = time.time()
    cap = [4 * n + (1 << 20) for n in wl.n_init]
    d = Discharge(wl, sig, thr, loss, precision=args.precision, capacity=cap)
    print(f"[bench] created {args.workload} ({sum(wl.n_init)} particles) in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    # warm start (the configuration times whole rf cycles of a running
    # discharge, not the initial load): warm_start_cycles rf cycles, whose
    # first steps are the autotuner's trials of launch shapes and grids
    # (real steps; results depend on neither)
    warm = int(round(args.warm_start_cycles * wl.steps_per_period))
    grid = None
    done = 0
    if not args.no_autotune and warm >= 1000:
        grid = d.autotune(100)
        done = d.moments()["step"]
        shape = d.launch_shape()
        print(f"[bench] autotuned push kernel: {shape[0]} threads x {shape[1]} particles per thread, "
              f"{grid} workgroups ({done} trial steps)", file=sys.stderr, flush=True)
    chunk = 500
    target = warm + args.warmup
    while done < target:
        k = min(chunk, target - done)
        tw = time.perf_counter()
        d.step(k)
        d.sync()
        done += k
        m = d.moments()
        print(f"[bench] {'warm start' if done <= warm else 'warmup'} {done}/{target}: "
              f"{(time.perf_counter() - tw) * 1e3 / k:.3f} ms/step, alive {m['alive']}", file=sys.stderr, flush=True)
    m0 = d.moments()
    d.timing(True, every=args.time_every)
    d.sync()
    t0 = time.perf_counter()
    done = 0
    report = 4000
    while done < args.steps:
        k = min(report, args.steps - done)
        d.step(k)
        done += k
        if done < args.steps:
            d.sync()
            print(f"[bench] timed {done}/{args.steps}", file=sys.stderr, flush=True)
    d.sync()
    elapsed = time.perf_counter() - t0
    push_ms, launches = d.kernel_time()
    d.timing(False)
    m1 = d.moments()
    psteps = m1["particle_steps"] - m0["particle_steps"]
    value = psteps / elapsed
    print(f"[bench] timed {args.steps} steps in {elapsed:.2f}s, {psteps} particle pushes, "
          f"alive {m1['alive']}", file=sys.stderr, flush=True)

    bpp = BYTES_PER_STEP[args.precision]
    # one launch of the fused kernel per step; `launches` of them timed
    avg_launch_s = (push_ms / 1e3) / max(launches, 1)
    per_launch = psteps / args.steps
    bytes_per_launch = bpp * per_launch
    achieved = bytes_per_launch / avg_launch_s / 1e9
    # HBM bytes per launch measured by counters (FETCH_SIZE + WRITE_SIZE of
    # the same kernel in two rocprofv3 --pmc runs, calibrated against a copy
    # of known size; profiles/), per push, scaled to this run's pushes per
    # launch.  Not measured in this run: taken from the file, and only if the
    # file names the kernel sources this library was built from.
    traffic = None
    traffic_note = None
    tfile = TRAFFIC_FILES.get(args.precision)
    if tfile and os.path.exists(tfile):
        try:
            t = json.load(open(tfile))
            if t.get("workload") != args.workload or t.get("precision") != args.precision:
                traffic_note = "no counter file for this workload"
            elif args.dsmc:
                # the counters were taken with the null-collision MCC in the push
                traffic_note = "no counter file for the push kernel of the per-cell list"
            elif t.get("source_sha") != kernel_source_sha():
                traffic_note = "counters in profiles/ predate the current kernel sources"
            else:
                traffic = round(t["bytes_per_push"] * per_launch)
                traffic_note = f"from {os.path.relpath(tfile, ROOT)} ({t['bytes_per_push']} B per push)"
        except (OSError, ValueError, KeyError):
            traffic = None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_push", "avg_launch_ms": round(avg_launch_s * 1e3, 4), "timed_launches": launches,
                "bytes_per_push": bpp, "traffic_source": traffic_note}
    if traffic:
        roofline["achieved_traffic"] = round(traffic / avg_launch_s / 1e9, 1)
        roofline["frac_traffic"] = round(traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4)
    touched = BYTES_TOUCHED[args.precision] * per_launch / avg_launch_s / 1e9
    roofline["achieved_touched"] = round(touched, 1)
    roofline["frac_touched"] = round(touched / HBM_PEAK_GBS, 4)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        swl = wl.scaled(args.cpu_scale)
        o = O.Oracle(swl, sig, thr, loss, precision=args.precision)
        _, _, ms0 = o.counters()
        c0 = time.perf_counter()
        o.step(args.cpu_steps)
        ce = time.perf_counter() - c0
        _, _, ms1 = o.counters()
        cpu = {"value": round((ms1["psteps"] - ms0["psteps"]) / ce, 1), "unit": "particle-steps/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{args.workload} discharge with every population scaled by {args.cpu_scale:g} "
                         f"({sum(swl.n_init)} particles), {args.cpu_steps} steps from the initial load, "
                         f"single-threaded C oracle ({args.precision})"}
        o.close()
        # all host cores: independent copies of the same sample, one per core,
        # stepped in threads (the oracle is C behind ctypes, which releases
        # the GIL); created one after another, stepped together
        import threading
        avail = len(os.sched_getaffinity(0))
        ncores = max(1, min(avail, args.cpu_cores) if args.cpu_cores > 0 else avail)
        steps_mc = max(1, args.cpu_steps // 2)
        inst = [O.Oracle(swl, sig, thr, loss, precision=args.precision) for _ in range(ncores)]
        p0 = [i.counters()[2]["psteps"] for i in inst]
        th = [threading.Thread(target=i.step, args=(steps_mc,)) for i in inst]
        c0 = time.perf_counter()
        for t_ in th:
            t_.start()
        for t_ in th:
            t_.join()
        ce = time.perf_counter() - c0
        ptot = sum(i.counters()[2]["psteps"] - q for i, q in zip(inst, p0))
        for i in inst:
            i.close()
        cpu["all_cores"] = {"value": round(ptot / ce, 1), "unit": "particle-steps/s", "cores": ncores,
                            "kind": "oracle",
                            "sample": f"{ncores} copies of the same sample stepped {steps_mc} steps at once, "
                                      "one thread each"}
        print(f"[bench] oracle on {ncores} cores: {ptot / ce:.4g} particle-steps/s", file=sys.stderr, flush=True)

    out = {
        "metric": "particle-steps/s (gather+push+MCC+deposit)",
        "value": round(value, 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl.gap_m * 100:g} cm, {wl.n_cells} cells, {wl.pressure_Pa:g} Pa, "
                               f"{wl.voltage_V:g} V, {wl.frequency_Hz / 1e6:g} MHz, dt=T/{wl.steps_per_period}, "
                               f"{sum(wl.n_init)} macro particles {tuple(wl.n_init)}",
                   "ion_subcycle": wl.ion_subcycle, "sort_every": wl.sort_every,
                   "coulomb_every": wl.coulomb_every, "coulomb_inter": bool(wl.coulomb_inter),
                   "collisions": "per-cell list every sort_every steps (Sec. II)" if wl.dsmc
                   else "null-collision MCC every push",
                   "precision": args.precision, "push_grid": grid,
                   "push_shape": list(d.launch_shape()[:2])},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "host": host_info(),
    }
    print(json.dumps(out), flush=True)
    if wl.coulomb_inter:
        inter_chains(d, wl)
    d.close()


def inter_chains(d, wl):
    """Unlike-species Coulomb pass: the particle of the less numerous species
    of a pair collides ceil(N_max / N_min) times in a row.  Prints, from the
    final cell populations, the longest of these sequential chains per pair."""
    import numpy as np
    cnt = [np.bincount(d.particles(s)[1], minlength=wl.n_cells) for s in range(3)]
    for q, (a, b) in enumerate([(0, 1), (0, 2), (1, 2)]):
        na, nb = cnt[a], cnt[b]
        both = (na > 0) & (nb > 0)
        chain = np.where(both, -(-np.maximum(na, nb) // np.maximum(np.minimum(na, nb), 1)), 0)
        i = int(np.argmax(chain))
        print(f"[bench] unlike pair {('e,O-', 'e,O2+', 'O-,O2+')[q]}: longest chain {int(chain.max())} links in cell {i} "
              f"({int(na[i])} and {int(nb[i])} particles), {int((chain > 100).sum())} cells above 100 links, "
              f"median {np.median(chain[both]) if both.any() else 0:.0f}", file=sys.stderr, flush=True)


def ablation_main(args):
    """The metastable ablation pair (Sec. IV): the production discharge run
    with C = 0 (no associative detachment) and with C = 1/6, from the same
    seeded load, for --cycles rf cycles each.  Reports the cycle-averaged
    macro-particle counts of the last cycle and the aggregate throughput."""
    import numpy as np
    from paper_0705_0495_amd import Discharge
    from pic_inputs import build_tables, workload
    sig, thr, loss = build_tables()
    base = workload("prod")
    n = base.n_cells
    vol = np.full(n + 1, base.area_m2 * base.gap_m / n)
    vol[[0, -1]] *= 0.5
    runs, psteps, elapsed = {}, 0, 0.0
    for C in (0.0, 1.0 / 6.0):
        wl = dataclasses.replace(base, metastable_frac=C)
        d = Discharge(wl, sig, thr, loss, precision=args.precision, capacity=[4 * x + (1 << 20) for x in wl.n_init])
        d.set_graphs(True)
        d.sync()
        t0 = time.perf_counter()
        for k in range(args.cycles):
            d.step(wl.steps_per_period)
            d.sync()
            print(f"[bench] C={C:.4g} cycle {k + 1}/{args.cycles}", file=sys.stderr, flush=True)
        elapsed += time.perf_counter() - t0
        m = d.moments()
        psteps += m["particle_steps"]
        dens = np.asarray(m["density"])
        runs[f"C={C:.4g}"] = {
            "e": round(float((dens[0] * vol).sum() / wl.weight)),
            "O-": round(float((dens[1] * vol).sum() / wl.weight)),
            "O2+": round(float((dens[2] * vol).sum() / wl.weight)),
            "associative_detachments": int(m["events"][16]),
        }
        print(f"[bench] C={C:.4g}: {runs[f'C={C:.4g}']}", file=sys.stderr, flush=True)
        d.close()
    value = psteps / elapsed
    out = {
        "metric": "particle-steps/s (gather+push+MCC+deposit)",
        "value": round(value, 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": 2 * args.cycles * base.steps_per_period,
        "warmup": 0,
        "ms_per_step": round(elapsed * 1e3 / (2 * args.cycles * base.steps_per_period), 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"ablation: prod discharge ({base.gap_m * 100:g} cm, {n} cells, "
                               f"{base.pressure_Pa:g} Pa, {base.voltage_V:g} V) with C = 0 and C = 1/6, "
                               f"{args.cycles} rf cycles each from the same seeded load",
                   "precision": args.precision},
        "ablation": {"cycles": args.cycles, "last_cycle_mean_macro_particles": runs},
    }
    print(json.dumps(out), flush=True)


def sweep_main(args):
    """Batched discharges (independent voltages, pressures, gaps, grids and
    loads, seeded), advanced together with pic_step_batch: each on its own
    stream, with graph replay unless --eager.  ``value`` is the aggregate
    particle pushes per second of all discharges over the timed steps."""
    from paper_0705_0495_amd import Discharge, step_batch
    from pic_inputs import build_tables, sweep
    wls = sweep(args.discharges)
    sig, thr, loss = build_tables()
    t0 = time.time()
    ds = []
    for w in wls:
        d = Discharge(w, sig, thr, loss, precision=args.precision, capacity=[4 * n + (1 << 20) for n in w.n_init])
        d.set_graphs(not args.eager)
        ds.append(d)
    ntot = sum(sum(w.n_init) for w in wls)
    print(f"[bench] created {len(ds)} discharges ({ntot} particles) in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)

    def run(k, label):
        done = 0
        while done < k:
            c = min(500, k - done)
            step_batch(ds, c)
            for d in ds:
                d.sync()
            done += c
            print(f"[bench] {label} {done}/{k}", file=sys.stderr, flush=True)

    shape = None
    if not args.no_autotune and args.warmup >= 600:
        # part of the warm-up: batched steps on each tile shape and two push
        # grids (real steps; results do not depend on them), the fastest kept
        from paper_0705_0495_amd import autotune_batch
        shape = autotune_batch(ds, 100)
        print(f"[bench] autotuned batched push: {shape[0]} x {shape[1]}, {shape[2]} workgroups", file=sys.stderr,
              flush=True)
        run(args.warmup - 600, "warmup")
    else:
        run(args.warmup, "warmup")
    p0 = sum(d.moments()["particle_steps"] for d in ds)
    for d in ds:
        d.sync()
    t1 = time.perf_counter()
    run(args.steps, "timed")
    elapsed = time.perf_counter() - t1
    p1 = sum(d.moments()["particle_steps"] for d in ds)
    value = (p1 - p0) / elapsed
    seq = None
    if args.sequential:
        ks = max(1, args.steps // 4)
        q0 = sum(d.moments()["particle_steps"] for d in ds)
        t2 = time.perf_counter()
        for d in ds:
            d.step(ks)
            d.sync()
        es = time.perf_counter() - t2
        q1 = sum(d.moments()["particle_steps"] for d in ds)
        seq = round((q1 - q0) / es, 1)
        print(f"[bench] sequential {ks} steps each: {seq:.4g} particle-steps/s", file=sys.stderr, flush=True)
    bpp = BYTES_PER_STEP[args.precision]
    achieved = bpp * value / 1e9
    out = {
        "metric": "particle-steps/s (gather+push+MCC+deposit)",
        "value": round(value, 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"sweep: {len(ds)} discharges, U~U[50,400] V, p~logU[5,100] Pa, L~U[2,6] cm, "
                               f"N_c in {{256,512,1024,2048}}, N~logU[1e5,4e6] ({ntot} particles in all), "
                               "dt=T/4000, sort and Coulomb every 10 steps",
                   "graphs": not args.eager, "precision": args.precision,
                   "push_shape": list(shape) if shape else None},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "whole step of all discharges (48 B per push over the wall clock)"},
        "sequential_value": seq,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    for d in ds:
        d.close()


def serve_main(args):
    """The serving loop on a finite stream of requests (Poisson arrivals at
    --rate per second), each run to its steady-state detector (the rf-cycle
    averaged ion count changes by less than 1 % against 50 cycles earlier,
    twice in a row) or --max-cycles rf cycles, under a device-memory budget,
    admitted at launch-period boundaries.  Requests: --stream served (default;
    small discharges that reach steady state in about a hundred rf cycles) or
    sweep (the batched sweep's distribution, which does not reach it within
    any cap that fits here).  ``value`` is the aggregate particle pushes per
    second over the whole stream; the line also gives p50/p99 time from
    arrival to steady state (over the requests that reached it) and to
    retirement."""
    import numpy as np
    from paper_0705_0495_amd.serve import Request, Server
    from pic_inputs import build_tables, served_stream, sweep
    wls = served_stream(args.requests) if args.stream == "served" else sweep(args.requests, seed=705049600)
    rng = np.random.default_rng(705049601)
    gaps = rng.exponential(1.0 / args.rate, size=len(wls)) if args.rate > 0 else np.zeros(len(wls))
    tables = build_tables()
    s = Server(tables, int(args.budget_gb * 2**30), precision=args.precision)
    t0 = time.perf_counter()
    t = t0
    for i, w in enumerate(wls):
        t += float(gaps[i])
        s.submit(Request(i, w, max_cycles=args.max_cycles, arrival=t))
    while s.queue or s.active:
        if not s.active and s.queue and s.queue[0].arrival > time.perf_counter():
            time.sleep(min(1.0, s.queue[0].arrival - time.perf_counter()))
            continue
        done = s.step_quantum()
        for r in done:
            print(f"[bench] request {r.rid} {'steady' if r.steady else 'capped'} after {r.cycles} cycles, "
                  f"{r.t_done - r.t_arrival:.2f}s from arrival", file=sys.stderr, flush=True)
    elapsed = time.perf_counter() - t0
    lat = s.latency()
    pushes = sum(r.pushes for r in s.results)  # the library's count, read at retirement
    out = {
        "metric": "particle-steps/s (gather+push+MCC+deposit)",
        "value": round(pushes / elapsed, 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": None,
        "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"serve: {len(wls)} requests ({args.stream} stream), Poisson arrivals at "
                               f"{args.rate:g}/s, run to steady state or {args.max_cycles} rf cycles, "
                               f"{args.budget_gb:g} GiB budget, admission at launch-period boundaries",
                   "precision": args.precision},
        "latency_s": {"p50": round(lat["p50_s"], 3), "p99": round(lat["p99_s"], 3)},
        "time_to_steady_state_s": {"p50": round(lat["ss_p50_s"], 3), "p99": round(lat["ss_p99_s"], 3)},
        "served": lat["served"], "steady": lat["steady"], "wall_s": round(elapsed, 2),
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
