"""The batched step that allocates nothing (pic_step_batch_static, tables in a
fixed device array) against the batched step with tables allocated for the
leading context (pic_step_batch): identical results, on two calls in a row,
the second with fewer discharges, and the limits reported as errors."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

from pic_inputs import build_tables, sweep

pytestmark = pytest.mark.gpu


def _by_id(t):
    ids, cell, off, v = t
    a = np.argsort(ids, kind="stable")
    return ids[a], cell[a], off[a], v[a]


def _state(g):
    parts = [_by_id(g.particles(s)) for s in range(3)]
    m = g.moments()
    return parts, g.charge(), g.field(), m["events"], m["absorbed"], m["next_id"], m["particle_steps"]


def _same(a, b, label):
    for s in range(3):
        for x, y in zip(a[0][s], b[0][s]):
            assert np.array_equal(x, y), f"{label}: species {s} differs"
    assert np.array_equal(a[1], b[1]), f"{label}: charge differs"
    assert np.array_equal(a[2][0], b[2][0]) and np.array_equal(a[2][1], b[2][1]), f"{label}: field differs"
    assert np.array_equal(a[3], b[3]) and np.array_equal(a[4], b[4]), f"{label}: counters differ"
    assert a[5] == b[5] and a[6] == b[6], f"{label}: ids or pushes differ"


def test_static_batch_matches_batch():
    from paper_0705_0495_amd import Discharge, PicError, step_batch, step_batch_static
    wls = [w.scaled(0.02, name=w.name) for w in sweep(64)[:4]]
    tables = build_tables()
    a = [Discharge(w, *tables, precision="fp32") for w in wls]
    b = [Discharge(w, *tables, precision="fp32") for w in wls]
    print(f"static batch: {[sum(w.n_init) for w in wls]} particles, 30 steps", flush=True)
    step_batch_static(a, 30)
    step_batch(b, 30)
    for w, x, y in zip(wls, a, b):
        _same(_state(x), _state(y), f"{w.name} after the first call")
    print("static batch: the first two again, 25 steps", flush=True)
    step_batch_static(a[:2], 25)
    step_batch(b[:2], 25)
    for w, x, y in zip(wls[:2], a[:2], b[:2]):
        _same(_state(x), _state(y), f"{w.name} after the second call")
    for w, x, y in zip(wls[2:], a[2:], b[2:]):
        _same(_state(x), _state(y), f"{w.name} (not in the second call)")
    # limits: too many discharges, or discharges that do not share a phase
    with pytest.raises(PicError):
        step_batch_static([a[0]] * 65, 1)
    with pytest.raises(PicError):
        step_batch_static([a[0], a[2]], 1)
    # argument errors leave the discharges usable
    step_batch_static(a[:2], 5)
    step_batch(b[:2], 5)
    for w, x, y in zip(wls[:2], a[:2], b[:2]):
        _same(_state(x), _state(y), f"{w.name} after the rejected calls")
    for d in a + b:
        d.close()
