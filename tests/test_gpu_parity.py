"""GPU (HIP, gfx950) against the CPU oracle, step by step.

Both sides draw the same Philox streams and follow the same operation order,
so particle ids, cells, counts, collision events and the integer node charge
must agree exactly; positions and velocities must agree to 1e-5 relative in
FP32 (the bar of the method's precision statement) and 1e-12 in FP64.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from pic_inputs import build_tables, workload
from tests.oracle_helpers import PARTNER_BOOST

pytestmark = pytest.mark.gpu

TOL = {"fp32": (1e-5, 1e-6), "fp64": (1e-12, 1e-12)}


def _gpu():
    from paper_0705_0495_amd import Discharge
    return Discharge


def _by_id(t):
    ids, cell, off, v = t
    a = np.argsort(ids, kind="stable")
    return ids[a], cell[a], off[a], v[a]


def compare(g, o, prec, label, sample_mod=None):
    rtol, otol = TOL[prec]
    for s in range(3):
        gi, gc, go, gv = _by_id(g.particles(s))
        oi, oc, oo, ov = _by_id(o.particles(s))
        assert len(gi) == len(oi), f"{label} species {s}: {len(gi)} vs {len(oi)} particles"
        if len(gi) == 0:
            continue
        if sample_mod:
            kg, ko = gi % sample_mod == 0, oi % sample_mod == 0
            gi, gc, go, gv = gi[kg], gc[kg], go[kg], gv[kg]
            oi, oc, oo, ov = oi[ko], oc[ko], oo[ko], ov[ko]
        assert np.array_equal(gi, oi), f"{label} species {s}: ids differ"
        bad = np.nonzero(gc != oc)[0]
        assert len(bad) == 0, f"{label} species {s}: {len(bad)} cells differ, first id {gi[bad[0]]}"
        assert np.allclose(go, oo, rtol=0, atol=otol), f"{label} species {s}: positions"
        scale = np.maximum(np.abs(ov), np.abs(ov).max(axis=0, keepdims=True) * 1e-3)
        err = np.abs(gv - ov) / np.maximum(scale, 1e-30)
        assert err.max() <= rtol, f"{label} species {s}: velocity rel err {err.max()}"
    m = g.moments()
    ev, ab, misc = o.counters()
    assert np.array_equal(m["events"], ev), f"{label}: events {m['events']} vs {ev}"
    assert np.array_equal(m["absorbed"], ab), f"{label}: absorbed {m['absorbed']} vs {ab}"
    assert m["step"] == misc["step"] and m["next_id"] == misc["next_id"] and m["births"] == misc["births"]
    assert m["particle_steps"] == misc["psteps"]
    assert np.array_equal(g.charge(), o.charge()), f"{label}: node charge differs"


def ragged_small(**kw):
    return dataclasses.replace(workload("small"), n_init=(5003, 1001, 4999), **kw)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_creation_matches_oracle(prec):
    wl = ragged_small()
    sig, thr, loss = build_tables()
    g = _gpu()(wl, sig, thr, loss, precision=prec)
    o = O.Oracle(wl, sig, thr, loss, precision=prec)
    compare(g, o, prec, "creation")
    gphi, gE = g.field()
    ophi, oE = o.field()
    assert np.array_equal(gphi, ophi)
    assert np.array_equal(gE, oE)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("boost", [1.0, PARTNER_BOOST])
def test_steps_match_oracle(prec, boost):
    wl = ragged_small()
    sig, thr, loss = build_tables(partner_boost=boost)
    g = _gpu()(wl, sig, thr, loss, precision=prec)
    o = O.Oracle(wl, sig, thr, loss, precision=prec)
    done = 0
    for target in (1, 2, 5, 11, 30, 80, 200):
        g.step(target - done)
        o.step(target - done)
        done = target
        g.sync()
        compare(g, o, prec, f"step {done}")
        gphi, gE = g.field()
        ophi, oE = o.field()
        assert np.array_equal(gphi, ophi), f"step {done}: potential differs"
    if boost > 1:
        ev, _, misc = o.counters()
        assert ev[12] + ev[13] + ev[17] > 0 and misc["requests"] > 0


def test_subcycled_ions_match_oracle():
    wl = ragged_small(ion_subcycle=3, sort_every=6, coulomb_every=6)
    sig, thr, loss = build_tables(partner_boost=PARTNER_BOOST)
    g = _gpu()(wl, sig, thr, loss, precision="fp32")
    o = O.Oracle(wl, sig, thr, loss, precision="fp32")
    for k in range(4):
        g.step(25)
        o.step(25)
        compare(g, o, "fp32", f"subcycled step {25 * (k + 1)}")


def test_one_rf_cycle_diagnostics_match_oracle():
    wl = workload("small")
    sig, thr, loss = build_tables()
    g = _gpu()(wl, sig, thr, loss, precision="fp32")
    o = O.Oracle(wl, sig, thr, loss, precision="fp32")
    g.step(wl.steps_per_period)
    o.step(wl.steps_per_period)
    compare(g, o, "fp32", "one cycle")
    m = g.moments()
    Q, phi, eedf, fneg = o.cycle_sums()
    assert m["cycles"] == 1
    assert np.array_equal(m["eedf"], eedf)
    assert np.array_equal(m["fneg"], fneg)
    dx = wl.gap_m / wl.n_cells
    vol = np.full(wl.n_cells + 1, wl.area_m2 * dx)
    vol[0] *= 0.5
    vol[-1] *= 0.5
    dens = wl.weight * (Q / 16777216.0) / vol / wl.steps_per_period
    assert np.allclose(m["density"], dens, rtol=1e-14, atol=0)
    assert np.array_equal(m["phi"], phi / wl.steps_per_period)


def test_rf_cycle_closing_between_sorts_matches_oracle():
    """Sort every 7 steps, so that the rf cycle (1000 steps) closes in a step
    without a sort, where the node charge of the step is formed outside the
    end-of-step kernel; partner reactions boosted so that they change the
    charge around it.  One cycle and three steps."""
    wl = dataclasses.replace(workload("small"), sort_every=7, coulomb_every=7)
    sig, thr, loss = build_tables(partner_boost=PARTNER_BOOST)
    g = _gpu()(wl, sig, thr, loss, precision="fp32")
    o = O.Oracle(wl, sig, thr, loss, precision="fp32")
    n = wl.steps_per_period + 3
    g.step(n)
    o.step(n)
    compare(g, o, "fp32", "one cycle and 3 steps, sort every 7")
    m = g.moments()
    Q, phi, eedf, fneg = o.cycle_sums()
    assert m["cycles"] == 1
    assert np.array_equal(m["eedf"], eedf)
    assert np.array_equal(m["fneg"], fneg)
    dx = wl.gap_m / wl.n_cells
    vol = np.full(wl.n_cells + 1, wl.area_m2 * dx)
    vol[0] *= 0.5
    vol[-1] *= 0.5
    dens = wl.weight * (Q / 16777216.0) / vol / wl.steps_per_period
    assert np.allclose(m["density"], dens, rtol=1e-14, atol=0)
    assert np.array_equal(m["phi"], phi / wl.steps_per_period)
    ev = o.counters()[0]
    assert ev[12] > 0 or ev[13] > 0 or ev[17] > 0, ev


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_results_independent_of_launch_shape(prec):
    """Tile shapes (threads per workgroup x particles per thread) and
    persistent grids of the push kernel change no result."""
    wl = ragged_small()
    sig, thr, loss = build_tables(partner_boost=PARTNER_BOOST)
    ref = None
    for shape, grid in (((256, 4), 0), ((256, 4), 1), ((256, 4), 7), ((256, 4), 61), ((512, 4), 0), ((512, 4), 3),
                        ((256, 8), 0), ((256, 8), 5)):
        g = _gpu()(wl, sig, thr, loss, precision=prec)
        g.set_shape(*shape)
        if grid:
            g.set_grid(grid)
        assert g.launch_shape()[:2] == shape
        g.step(60)
        out = [_by_id(g.particles(s)) for s in range(3)]
        ev = g.moments()["events"]
        if ref is None:
            ref = (out, ev)
            continue
        for s in range(3):
            for a, b in zip(out[s], ref[0][s]):
                assert np.array_equal(a, b)
        assert np.array_equal(ev, ref[1])
        g.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_production_size_matches_oracle(prec):
    """The 4.5M-particle production discharge in the launch configuration the
    benchmark uses: 101 steps, through the ion sub-cycles (every 10 steps) and
    the first sort and Coulomb pass (step 100), every particle compared."""
    wl = workload("prod")
    sig, thr, loss = build_tables()
    g = _gpu()(wl, sig, thr, loss, precision=prec)
    o = O.Oracle(wl, sig, thr, loss, precision=prec)
    done = 0
    for target in (1, 11, 101):
        g.step(target - done)
        o.step(target - done)
        done = target
        compare(g, o, prec, f"prod {prec} step {target}")
    g.close()
    o.close()


def test_large_size_matches_oracle():
    """The 2^25-particle discharge of the benchmark: 20 steps, through two
    sorts and Coulomb passes (steps 10 and 20); step 1 on every 997th
    particle, steps 11 and 20 on every particle, counters and charge in full."""
    wl = workload("large")
    sig, thr, loss = build_tables()
    g = _gpu()(wl, sig, thr, loss, precision="fp32")
    o = O.Oracle(wl, sig, thr, loss, precision="fp32")
    g.step(1)
    o.step(1)
    compare(g, o, "fp32", "large step 1", sample_mod=997)
    done = 1
    for target in (11, 20):
        g.step(target - done)
        o.step(target - done)
        done = target
        compare(g, o, "fp32", f"large step {target}")
    assert np.array_equal(g.charge(), o.charge())
    g.close()
    o.close()


@pytest.mark.parametrize("prec,n_cells", [("fp32", 4608), ("fp64", 2304)])
def test_global_field_push_matches_oracle(prec, n_cells):
    """Grids above what the push stages in LDS (4099 cells in FP32, 2049 in
    FP64, as the FP64 large discharge): the push gathers the node field from
    global memory.  35 steps through three sorts and Coulomb passes, partner
    reactions boosted."""
    wl = dataclasses.replace(workload("small").scaled(6.0, name="small-x6"), n_cells=n_cells)
    sig, thr, loss = build_tables(partner_boost=PARTNER_BOOST)
    g = _gpu()(wl, sig, thr, loss, precision=prec)
    o = O.Oracle(wl, sig, thr, loss, precision=prec)
    done = 0
    for target in (1, 10, 11, 35):
        g.step(target - done)
        o.step(target - done)
        done = target
        compare(g, o, prec, f"{n_cells} cells step {target}")
        assert np.array_equal(g.field()[1], o.field()[1])
    assert np.array_equal(g.charge(), o.charge())
    g.close()
    o.close()


def test_large_run_is_reproducible():
    """The 2^25-particle discharge over 2000 steps (200 sorts and Coulomb
    passes), twice: in one call on the default grid, and in chunks of 100 steps
    on a smaller persistent grid.  Every result is a deterministic function of
    the input (integer deposits, id-keyed random numbers), so the two runs must
    agree bit for bit whatever order the workgroups ran in; a workgroup whose
    waves disagreed on a shared value (the deposit window's base cell, read
    while another wave was already storing the tile) broke this within a few
    hundred steps."""
    import hashlib
    wl = workload("large")
    sig, thr, loss = build_tables()
    cap = [4 * n + (1 << 20) for n in wl.n_init]
    prints = []
    for grid, chunk in ((0, 2000), (509, 100)):
        g = _gpu()(wl, sig, thr, loss, precision="fp32", capacity=cap)
        if grid:
            g.set_grid(grid)
        for _ in range(2000 // chunk):
            g.step(chunk)
            g.sync()
        m = g.moments()
        h = hashlib.sha1()
        for s in range(3):
            for a in _by_id(g.particles(s)):
                h.update(np.ascontiguousarray(a).tobytes())
        prints.append((g.charge(), g.field()[1], m["events"], m["absorbed"], m["next_id"], h.hexdigest()))
        g.close()
    a, b = prints
    assert np.array_equal(a[0], b[0]), "node charge differs"
    assert np.array_equal(a[1], b[1]), "field differs"
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3]) and a[4] == b[4], "counters differ"
    assert a[5] == b[5], "particles differ"


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("lnl", [10.0, 1e4])
def test_coulomb_matches_oracle(prec, lnl):
    """Intra-species Coulomb collisions with every sort (every 5 steps):
    ln Lambda = 10 gives small angles only, 1e4 also large angles and the
    isotropic branch; ragged counts give triangles in odd cells."""
    wl = ragged_small(sort_every=5, coulomb_every=5, coulomb_log=lnl)
    sig, thr, loss = build_tables(partner_boost=PARTNER_BOOST)
    g = _gpu()(wl, sig, thr, loss, precision=prec)
    o = O.Oracle(wl, sig, thr, loss, precision=prec)
    done = 0
    for target in (5, 10, 25, 60):
        g.step(target - done)
        o.step(target - done)
        done = target
        compare(g, o, prec, f"coulomb step {done}")


def test_coulomb_dense_cells_match_oracle():
    """Thousands of particles of a species per cell: many pairing buckets and
    several positions per thread."""
    wl = dataclasses.replace(workload("small"), n_cells=16, n_init=(40001, 20001, 39999), sort_every=2,
                             coulomb_every=2)
    sig, thr, loss = build_tables()
    g = _gpu()(wl, sig, thr, loss, precision="fp32")
    o = O.Oracle(wl, sig, thr, loss, precision="fp32")
    for k in range(3):
        g.step(2)
        o.step(2)
        compare(g, o, "fp32", f"dense coulomb step {2 * (k + 1)}")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_coulomb_big_cells_match_oracle(prec):
    """About 10000 particles of a species per cell, more than the cells whose
    velocities are staged in LDS (8192 in FP32, 4096 in FP64): these take the
    path that orders in LDS and collides in global memory."""
    wl = dataclasses.replace(workload("small"), n_cells=8, n_init=(80001, 1001, 79999), sort_every=2,
                             coulomb_every=2)
    sig, thr, loss = build_tables()
    g = _gpu()(wl, sig, thr, loss, precision=prec)
    o = O.Oracle(wl, sig, thr, loss, precision=prec)
    for k in range(2):
        g.step(2)
        o.step(2)
        compare(g, o, prec, f"big-cell coulomb step {2 * (k + 1)}")


def test_coulomb_cell_overflow_is_reported():
    """More than 16384 particles of one species in a cell: the Coulomb pass
    reports PIC_EOVERFLOW instead of pairing a part of the cell."""
    from paper_0705_0495_amd.binding import PicError
    wl = dataclasses.replace(workload("small"), n_cells=4, n_init=(80000, 0, 80000), sort_every=1,
                             coulomb_every=1)
    sig, thr, loss = build_tables()
    g = _gpu()(wl, sig, thr, loss, precision="fp32")
    g.step(1)
    with pytest.raises(PicError) as e:
        g.sync()
    assert e.value.code == -5


def test_large_size_coulomb_matches_oracle():
    """The 2^25-particle discharge with the cell sort and the Coulomb pass in
    its first step; every particle compared (a few thousand particles per
    species and cell, so equal pairing hashes occur and are ordered by id)."""
    wl = dataclasses.replace(workload("large"), sort_every=1, coulomb_every=1)
    sig, thr, loss = build_tables()
    g = _gpu()(wl, sig, thr, loss, precision="fp32")
    o = O.Oracle(wl, sig, thr, loss, precision="fp32")
    g.step(1)
    o.step(1)
    compare(g, o, "fp32", "large coulomb step 1")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("lnl", [10.0, 1e4])
def test_inter_species_coulomb_matches_oracle(prec, lnl):
    """Unlike-species Coulomb collisions after the like-species pass, with
    every sort: cells where either species of a pair is the more numerous,
    ties, and cells where one species is absent; ln Lambda = 1e4 also takes
    the isotropic branch."""
    wl = ragged_small(sort_every=5, coulomb_every=5, coulomb_log=lnl, coulomb_inter=True)
    sig, thr, loss = build_tables(partner_boost=PARTNER_BOOST)
    g = _gpu()(wl, sig, thr, loss, precision=prec)
    o = O.Oracle(wl, sig, thr, loss, precision=prec)
    done = 0
    for target in (5, 10, 25):
        g.step(target - done)
        o.step(target - done)
        done = target
        compare(g, o, prec, f"inter coulomb step {done}")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_inter_species_coulomb_long_chains_match_oracle(prec):
    """Few O- among thousands of electrons and ions per cell: every O-
    collides about a hundred times in a row, and a species above 1024 per
    cell gives a workgroup thread several partners' chains."""
    wl = dataclasses.replace(workload("small"), n_cells=8, n_init=(30001, 301, 20001), sort_every=2,
                             coulomb_every=2, coulomb_inter=True)
    sig, thr, loss = build_tables()
    g = _gpu()(wl, sig, thr, loss, precision=prec)
    o = O.Oracle(wl, sig, thr, loss, precision=prec)
    for k in range(2):
        g.step(2)
        o.step(2)
        compare(g, o, prec, f"inter coulomb chains step {2 * (k + 1)}")


def test_inter_species_coulomb_off_leaves_like_pass_alone():
    """The switch off gives exactly the like-species results; on, the state
    differs (the unlike pairs did collide)."""
    base = ragged_small(sort_every=5, coulomb_every=5)
    sig, thr, loss = build_tables()
    off = _gpu()(base, sig, thr, loss, precision="fp32")
    on = _gpu()(dataclasses.replace(base, coulomb_inter=True), sig, thr, loss, precision="fp32")
    o = O.Oracle(base, sig, thr, loss, precision="fp32")
    for d in (off, on):
        d.step(10)
    o.step(10)
    compare(off, o, "fp32", "inter off step 10")
    assert not np.array_equal(_by_id(off.particles(0))[3], _by_id(on.particles(0))[3])


def test_large_size_inter_species_coulomb_matches_oracle():
    """The 2^25-particle discharge with the sort and both Coulomb passes in its
    first step; every particle compared."""
    wl = dataclasses.replace(workload("large"), sort_every=1, coulomb_every=1, coulomb_inter=True)
    sig, thr, loss = build_tables()
    g = _gpu()(wl, sig, thr, loss, precision="fp32")
    o = O.Oracle(wl, sig, thr, loss, precision="fp32")
    g.step(1)
    o.step(1)
    compare(g, o, "fp32", "large inter coulomb step 1")


def test_inter_species_coulomb_batch_matches_alone():
    """A batch mixing discharges with the unlike-species pass on and off (one
    launch per kernel) ends exactly as each stepped alone."""
    from paper_0705_0495_amd import step_batch
    sig, thr, loss = build_tables()
    base = ragged_small(sort_every=5, coulomb_every=5)
    wls = [dataclasses.replace(base, coulomb_inter=True, name="inter"),
           dataclasses.replace(base, name="like"),
           dataclasses.replace(base, n_cells=24, coulomb_inter=True, name="inter24")]
    batch = [_gpu()(w, sig, thr, loss, precision="fp32") for w in wls]
    step_batch(batch, 20)
    for g in batch:
        g.sync()
    for w, g in zip(wls, batch):
        alone = _gpu()(w, sig, thr, loss, precision="fp32")
        alone.step(20)
        alone.sync()
        _same_state(_state(alone), _state(g), w.name)
        alone.close()
        g.close()


def test_metastable_ablation_matches_oracle():
    """The ablation pair of the metastable fraction: C = 0 closes associative
    detachment (no events on either side), C = 1/6 (the default, tested
    throughout) keeps it; both discharges match the oracle."""
    for C in (0.0, 1.0 / 6.0):
        wl = ragged_small(metastable_frac=C, pressure_Pa=100.0)
        sig, thr, loss = build_tables()
        g = _gpu()(wl, sig, thr, loss, precision="fp32")
        o = O.Oracle(wl, sig, thr, loss, precision="fp32")
        done = 0
        for target in (5, 30):
            g.step(target - done)
            o.step(target - done)
            done = target
            compare(g, o, "fp32", f"C={C:g} step {done}")
        ad = g.moments()["events"][16]
        assert (ad == 0) if C == 0.0 else (ad > 0), (C, ad)
        g.close()


def test_births_above_lds_key_capacity_match_oracle():
    """More than 8192 births in one step (hot electrons, ionisation only,
    scaled up): birth ranks fall back from LDS keys to global memory."""
    from tests.oracle_helpers import tables_only
    wl = dataclasses.replace(workload("small"), n_init=(100000, 1000, 100000), T_init_eV=(30.0, 0.026, 0.026))
    sig, thr, loss = tables_only([11])
    o0 = O.Oracle(wl, sig, thr, loss, precision="fp32")
    pm = o0.constants()["pmax_e"]
    o0.close()
    sig = sig * (0.3 / pm)
    g = _gpu()(wl, sig, thr, loss, precision="fp32")
    o = O.Oracle(wl, sig, thr, loss, precision="fp32")
    g.step(1)
    o.step(1)
    _, _, misc = o.counters()
    assert misc["births"] > 8192, misc["births"]
    compare(g, o, "fp32", "many births step 1")
    g.step(2)
    o.step(2)
    compare(g, o, "fp32", "many births step 3")


def _state(g):
    out = [_by_id(g.particles(s)) for s in range(3)]
    m = g.moments()
    return out, g.charge(), g.field(), m["events"], m["absorbed"], m["next_id"], m["particle_steps"]


def _same_state(a, b, label):
    for s in range(3):
        for x, y in zip(a[0][s], b[0][s]):
            assert np.array_equal(x, y), f"{label}: species {s} differs"
    assert np.array_equal(a[1], b[1]), f"{label}: charge differs"
    assert np.array_equal(a[2][0], b[2][0]) and np.array_equal(a[2][1], b[2][1]), f"{label}: field differs"
    assert np.array_equal(a[3], b[3]) and np.array_equal(a[4], b[4]), f"{label}: counters differ"
    assert a[5] == b[5] and a[6] == b[6], f"{label}: ids or pushes differ"


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_graph_replay_matches_eager(prec, inter=False):
    """Captured step sequences (20 steps: sort and Coulomb every 10, twice)
    replayed several times, with eager steps and synchronisation in between,
    give the eager run's state after every chunk; partner reactions boosted so
    that the end-of-step kernel takes both of its paths."""
    wl = ragged_small(sort_every=10, coulomb_every=10, coulomb_inter=inter)
    sig, thr, loss = build_tables(partner_boost=PARTNER_BOOST)
    ge = _gpu()(wl, sig, thr, loss, precision=prec)
    gg = _gpu()(wl, sig, thr, loss, precision=prec)
    gg.set_graphs(True)
    done = 0
    for k in (20, 20, 13, 27, 40, 5, 60):
        # one discharge at a time: this compares replay with eager stepping,
        # not two discharges sharing the GPU
        ge.step(k)
        ge.sync()
        gg.step(k)
        gg.sync()
        done += k
        _same_state(_state(ge), _state(gg), f"after {done} steps")
    ge.close()
    gg.close()


@pytest.mark.parametrize("mode,prec", [("batched", "fp32"), ("batched", "fp64"), ("round_robin", "fp32")])
def test_batch_matches_alone(mode, prec):
    """Discharges of the batched sweep, scaled down, advanced together end
    exactly as each stepped alone: with one launch per kernel for all of them
    (same periods), and round robin on their own streams with graph replay
    (one discharge with another sort period makes the batch mixed)."""
    from paper_0705_0495_amd import step_batch
    from pic_inputs import sweep
    wls = [w.scaled(0.05, name=w.name) for w in sweep(64)[:5]]
    # dense cells: above the small Coulomb class (listed for the largest
    # class) and above the largest (the big-cell path)
    wls += [dataclasses.replace(workload("small"), n_cells=8).scaled(2.0, name="dense8"),
            dataclasses.replace(workload("small"), n_cells=4).scaled(4.0, name="dense4")]
    if mode == "round_robin":
        wls[2] = dataclasses.replace(wls[2], sort_every=5, coulomb_every=5)
    sig, thr, loss = build_tables()
    batch = [_gpu()(w, sig, thr, loss, precision=prec) for w in wls]
    for g in batch:
        g.set_graphs(True)
    step_batch(batch, 45)
    step_batch(batch, 35)
    for g in batch:
        g.sync()
    for w, g in zip(wls, batch):
        alone = _gpu()(w, sig, thr, loss, precision=prec)
        alone.step(80)
        alone.sync()
        _same_state(_state(alone), _state(g), w.name)
        alone.close()
        g.close()


def test_round_robin_large_coulomb_matches_alone():
    """Two 2^25-particle discharges with Coulomb collisions (every 10 and
    every 20 steps, so the batch is mixed and runs round robin on two
    streams), 199 steps in one call: with Coulomb collisions on, the call
    chains the two contexts' periods so that their kernels never overlap, and
    each ends exactly as stepped alone.  (Run concurrently, such pairs have
    diverged from their lone runs.)"""
    from paper_0705_0495_amd import step_batch
    base = workload("large")
    wls = [base, dataclasses.replace(base, coulomb_every=20, seed=base.seed + 1)]
    sig, thr, loss = build_tables()
    pair = [_gpu()(w, sig, thr, loss, precision="fp32") for w in wls]
    step_batch(pair, 199)
    got = []
    for g in pair:
        g.sync()
        got.append(_state(g))
        g.close()
    for w, st in zip(wls, got):
        alone = _gpu()(w, sig, thr, loss, precision="fp32")
        alone.step(199)
        alone.sync()
        _same_state(_state(alone), st, w.name)
        alone.close()


def test_served_discharges_match_alone():
    """The serving loop with room for two discharges at a time: the third is
    admitted when the first retires and then advances in the same batched
    launches as the second, four thousand steps apart (same phase of the
    step sequence).  Every served discharge ends exactly as stepped alone."""
    from paper_0705_0495_amd.serve import Request, Server, bytes_needed
    from pic_inputs import sweep
    wls = [w.scaled(0.01, name=w.name) for w in sweep(64)[:3]]
    tables = build_tables()
    budget = 2 * max(bytes_needed(w, "fp32") for w in wls)
    reqs = [Request(i, w, max_cycles=c, tol=0.0) for i, (w, c) in enumerate(zip(wls, (1, 3, 2)))]
    served = {}

    class Keep:
        """Discharge that records its final state before the server closes it."""

        def __init__(self, wl, *t, **kw):
            self.g = _gpu()(wl, *t, **kw)
            self.wl = wl

        def __getattr__(self, k):
            return getattr(self.g, k)

        def close(self):
            served[self.wl.name] = _state(self.g)
            self.g.close()

    from paper_0705_0495_amd import step_batch
    s = Server(tables, budget, backend=Keep, step_batch=lambda ds, n: step_batch([d.g for d in ds], n))
    for r in reqs:
        s.submit(r)
    res = s.run()
    assert sorted((r.rid, r.cycles) for r in res) == [(0, 1), (1, 3), (2, 2)]
    for w, c in zip(wls, (1, 3, 2)):
        alone = _gpu()(w, *tables, precision="fp32", capacity=[4 * n + (1 << 20) for n in w.n_init])
        alone.step(c * w.steps_per_period)
        alone.sync()
        _same_state(_state(alone), served[w.name], w.name)
        alone.close()


def test_batch_autotune_and_shapes_change_no_result():
    """The batch autotuner's trials are ordinary batched steps; a batch on each
    tile shape, with graph replay of whole periods, ends as each discharge
    stepped alone."""
    from paper_0705_0495_amd import autotune_batch, step_batch
    from pic_inputs import sweep
    wls = [w.scaled(0.02, name=w.name) for w in sweep(64)[:3]]
    sig, thr, loss = build_tables()
    batch = [_gpu()(w, sig, thr, loss, precision="fp32") for w in wls]
    t, p, g = autotune_batch(batch, 20)
    assert (t, p) in ((256, 4), (512, 4), (256, 8)) and g > 0
    done = 6 * 20
    for d in batch:
        d.set_graphs(True)
    step_batch(batch, 40)
    done += 40
    for w, d in zip(wls, batch):
        alone = _gpu()(w, sig, thr, loss, precision="fp32")
        alone.set_shape(256, 8)
        alone.step(done)
        alone.sync()
        _same_state(_state(alone), _state(d), w.name)
        alone.close()
        d.close()


def test_autotune_changes_no_result():
    """The grid autotuner's trial steps are ordinary steps: afterwards the
    discharge equals a twin stepped the same number of times on the default
    grid, and so does the next stretch on the chosen grid."""
    wl = ragged_small()
    sig, thr, loss = build_tables(partner_boost=PARTNER_BOOST)
    a = _gpu()(wl, sig, thr, loss, precision="fp32")
    b = _gpu()(wl, sig, thr, loss, precision="fp32")
    g = a.autotune(10)
    assert g > 0
    b.step(a.moments()["step"])
    _same_state(_state(a), _state(b), "after tuning")
    a.step(25)
    b.step(25)
    _same_state(_state(a), _state(b), "after 25 more steps")
    a.close()
    b.close()


def test_graph_replay_with_unlike_pass_matches_eager():
    """The same with the unlike-species Coulomb pass in the captured sequence
    (its workgroups exchange ranks and velocities through global memory
    between their phases)."""
    test_graph_replay_matches_eager("fp32", inter=True)

