"""The per-cell collision list of Sec. II (pic_gas::dsmc) on the GPU against
the oracle: the same Philox streams and operation order on both sides, so ids,
cells, counts, events and the integer node charge agree exactly and positions
and velocities to 1e-5 relative (FP32) or 1e-12 (FP64)."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from pic_inputs import build_tables, workload
from tests.oracle_helpers import PARTNER_BOOST
from tests.test_gpu_parity import _gpu, _same_state, _state, compare, ragged_small

pytestmark = pytest.mark.gpu

# the null-collision tests' partner boost: on the small discharge the list's
# partner types then collide a few dozen times in 200 steps, their bounds
# N_t(c) tau W max(sigma g) / (A dx) staying below one
LIST_BOOST = PARTNER_BOOST


def list_small(**kw):
    return ragged_small(dsmc=True, **kw)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("boost", [1.0, LIST_BOOST])
def test_list_steps_match_oracle(prec, boost):
    """Ragged populations (5003, 1001, 4999), passes every 10 steps, Coulomb
    after each; compared before, at and after passes."""
    wl = list_small()
    sig, thr, loss = build_tables(partner_boost=boost)
    g = _gpu()(wl, sig, thr, loss, precision=prec)
    o = O.Oracle(wl, sig, thr, loss, precision=prec)
    done = 0
    for target in (1, 9, 10, 11, 20, 50, 100, 200):
        g.step(target - done)
        o.step(target - done)
        done = target
        g.sync()
        compare(g, o, prec, f"list step {done}")
        gphi, gE = g.field()
        ophi, oE = o.field()
        assert np.array_equal(gphi, ophi), f"list step {done}: potential differs"
    ev, _, misc = o.counters()
    assert ev[0] > 0 and ev[10] > 0 and ev[11] > 0
    if boost > 1:
        assert ev[12] > 0 and ev[13] > 0 and ev[17] > 0, ev


def test_list_subcycled_ions_match_oracle():
    wl = list_small(ion_subcycle=5, sort_every=10, coulomb_every=20)
    sig, thr, loss = build_tables(partner_boost=LIST_BOOST)
    g = _gpu()(wl, sig, thr, loss, precision="fp32")
    o = O.Oracle(wl, sig, thr, loss, precision="fp32")
    for k in range(4):
        g.step(35)
        o.step(35)
        compare(g, o, "fp32", f"list subcycled step {35 * (k + 1)}")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_list_larger_discharge_matches_oracle(prec):
    """Eight times the small discharge (about 160k particles, many workgroups
    per kernel), three passes."""
    wl = dataclasses.replace(workload("small"), dsmc=True).scaled(8.0)
    sig, thr, loss = build_tables(partner_boost=LIST_BOOST)
    g = _gpu()(wl, sig, thr, loss, precision=prec)
    o = O.Oracle(wl, sig, thr, loss, precision=prec)
    done = 0
    for target in (10, 30):
        g.step(target - done)
        o.step(target - done)
        done = target
        g.sync()
        compare(g, o, prec, f"list x8 step {target}")


def test_list_large_size_matches_oracle():
    """The 2^25-particle discharge of the benchmark on the list (bench.py
    --dsmc): 20 steps, two passes each followed by Coulomb; step 1 on every
    997th particle, steps 10 (the first pass) and 20 on every particle,
    counters and charge in full."""
    wl = dataclasses.replace(workload("large"), dsmc=True)
    sig, thr, loss = build_tables()
    g = _gpu()(wl, sig, thr, loss, precision="fp32")
    o = O.Oracle(wl, sig, thr, loss, precision="fp32")
    g.step(1)
    o.step(1)
    compare(g, o, "fp32", "large list step 1", sample_mod=997)
    done = 1
    for target in (10, 20):
        g.step(target - done)
        o.step(target - done)
        done = target
        compare(g, o, "fp32", f"large list step {target}")
    ev = o.counters()[0]
    assert ev[0] > 0 and ev[11] > 0
    g.close()
    o.close()


def test_list_graph_replay_matches_eager():
    """Whole periods (two passes with their re-sorts) captured and replayed,
    eager steps in between: the eager run's state after every chunk."""
    wl = list_small(sort_every=10, coulomb_every=10)
    sig, thr, loss = build_tables(partner_boost=LIST_BOOST)
    ge = _gpu()(wl, sig, thr, loss, precision="fp32")
    gg = _gpu()(wl, sig, thr, loss, precision="fp32")
    gg.set_graphs(True)
    done = 0
    for k in (20, 20, 13, 27, 40, 60):
        ge.step(k)
        ge.sync()
        gg.step(k)
        gg.sync()
        done += k
        _same_state(_state(ge), _state(gg), f"list graphs after {done} steps")
    ge.close()
    gg.close()


def test_list_discharge_in_a_batch_steps_alone():
    """pic_step_batch does not batch a discharge on the list: each ends as
    if stepped alone."""
    from paper_0705_0495_amd import step_batch
    sig, thr, loss = build_tables(partner_boost=LIST_BOOST)
    wls = [list_small(), ragged_small(seed=705049777)]
    batch = [_gpu()(w, sig, thr, loss, precision="fp32") for w in wls]
    step_batch(batch, 40)
    for g in batch:
        g.sync()
    for w, g in zip(wls, batch):
        alone = _gpu()(w, sig, thr, loss, precision="fp32")
        alone.step(40)
        alone.sync()
        _same_state(_state(alone), _state(g), f"{'list' if w.dsmc else 'null'} in a batch")


def test_list_with_unlike_coulomb_matches_oracle():
    """The list followed by both Coulomb passes (like and unlike species)
    after its sort."""
    wl = list_small(coulomb_inter=True)
    sig, thr, loss = build_tables(partner_boost=LIST_BOOST)
    g = _gpu()(wl, sig, thr, loss, precision="fp32")
    o = O.Oracle(wl, sig, thr, loss, precision="fp32")
    done = 0
    for target in (10, 30, 60):
        g.step(target - done)
        o.step(target - done)
        done = target
        g.sync()
        compare(g, o, "fp32", f"list + unlike Coulomb step {done}")


def test_allocation_free_batch_refuses_list_discharges():
    """pic_step_batch_static batches only what pic_step_batch would: a
    discharge on the list is refused (an argument error that leaves it
    usable)."""
    from paper_0705_0495_amd import PicError, step_batch_static
    sig, thr, loss = build_tables()
    a = _gpu()(list_small(), sig, thr, loss, precision="fp32")
    b = _gpu()(ragged_small(dsmc=True, seed=705049778), sig, thr, loss, precision="fp32")
    with pytest.raises(PicError):
        step_batch_static([a, b], 20)
    a.step(20)
    a.sync()
    o = O.Oracle(list_small(), sig, thr, loss, precision="fp32")
    o.step(20)
    compare(a, o, "fp32", "list after a refused static batch")


def test_list_bounds_are_rejected_or_raised():
    from paper_0705_0495_amd import PicError
    sig, thr, loss = build_tables()
    # a gas type whose tau n max(sigma g) exceeds one: rejected at creation
    big = sig.copy()
    big[0] *= 200.0
    with pytest.raises(PicError):
        _gpu()(list_small(), big, thr, loss, precision="fp32")
    # a partner type above one in a cell with test particles: guard at the pass
    hot = build_tables(partner_boost=PARTNER_BOOST * 20)
    g = _gpu()(list_small(), *hot, precision="fp32")
    o = O.Oracle(list_small(), *hot, precision="fp32")
    g.step(10)
    with pytest.raises(PicError):
        g.sync()
    with pytest.raises(RuntimeError):
        o.step(10)
