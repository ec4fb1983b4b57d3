"""Cycle-averaged moments of a named discharge computed by the CPU oracle.

For each of three seeds the oracle is run for `cycles` rf cycles and the
moments of the cycles after the first `skip` are averaged: densities of e,
O- and O2+ at the nodes, the potential, the electron energy histogram at
x = L/2 (normalised), and collision events per cycle and channel.  Only the
oracle is called; the result is written to
``<workload>_<precision>_moments.npz`` next to this file.

    python tests/golden/moments.py small            # 20 cycles, average 11-20
    python tests/golden/moments.py small_list       # the same on the per-cell collision list
    python tests/golden/moments.py prod --cycles 3 --skip 1
"""
from __future__ import annotations

import argparse
import dataclasses
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

SEED_OFFSETS = (0, 100, 200)


def seeded(name, k):
    from pic_inputs import workload
    wl = workload(name)
    return dataclasses.replace(wl, seed=wl.seed + SEED_OFFSETS[k])


def node_volumes(wl):
    N = wl.n_cells
    vol = np.full(N + 1, wl.area_m2 * wl.gap_m / N)
    vol[0] *= 0.5
    vol[-1] *= 0.5
    return vol


def averages(cycle_fn, cycles, skip):
    """Average the per-cycle moments returned by cycle_fn() over cycles skip+1..cycles."""
    acc = None
    for k in range(cycles):
        m = cycle_fn()
        if k < skip:
            continue
        acc = m if acc is None else {key: acc[key] + m[key] for key in acc}
    return {key: v / (cycles - skip) for key, v in acc.items()}


def oracle_run(args):
    name, k, precision, cycles, skip = args
    from oracle.oracle import Oracle
    from pic_inputs import build_tables
    wl = seeded(name, k)
    o = Oracle(wl, *build_tables(), precision=precision)
    M = wl.steps_per_period
    vol = node_volumes(wl)
    last = np.zeros(19)

    def cycle():
        nonlocal last
        o.step(M)
        Q, phi, eedf, _ = o.cycle_sums()
        ev, _, _ = o.counters()
        d = {"density": wl.weight * (Q / 16777216.0) / vol / M, "phi": phi / M,
             "eedf": eedf / max(1, eedf.sum()), "events": ev - last}
        last = ev.astype(float)
        return d

    out = averages(cycle, cycles, skip)
    o.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["small", "small_list", "prod"])
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--cycles", type=int, default=20)
    ap.add_argument("--skip", type=int, default=10)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    out = a.out or os.path.join(HERE, f"{a.workload}_{a.precision}_moments.npz")
    jobs = [(a.workload, k, a.precision, a.cycles, a.skip) for k in range(len(SEED_OFFSETS))]
    with ProcessPoolExecutor(len(jobs)) as ex:
        res = list(ex.map(oracle_run, jobs))
    np.savez(out, seed_offsets=np.array(SEED_OFFSETS), cycles=a.cycles, skip=a.skip,
             **{k: np.stack([r[k] for r in res]) for k in res[0]})
    print("wrote", out)


if __name__ == "__main__":
    main()
