"""Degenerate and extreme discharges on the GPU against the oracle, for both
collision schemes: no particles at all, a single electron, ions without
electrons, and the largest grid the library takes (8192 cells, where the
field solve runs nine nodes per thread and the push gathers the node field
from global memory)."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from pic_inputs import build_tables, workload
from tests.oracle_helpers import PARTNER_BOOST
from tests.test_gpu_parity import _gpu, compare

pytestmark = pytest.mark.gpu

CASES = {
    "empty": dict(n_init=(0, 0, 0)),
    "one_electron": dict(n_init=(1, 0, 0)),
    "ions_only": dict(n_init=(0, 300, 300)),
    "max_cells": dict(n_cells=8192, n_init=(20000, 4000, 20000)),
}


@pytest.mark.parametrize("dsmc", [False, True])
@pytest.mark.parametrize("case,prec", [("empty", "fp32"), ("one_electron", "fp32"), ("ions_only", "fp32"),
                                       ("max_cells", "fp32"), ("max_cells", "fp64")])
def test_edge_discharges_match_oracle(case, prec, dsmc):
    wl = dataclasses.replace(workload("small"), dsmc=dsmc, **CASES[case])
    # on 8192 cells the list's partner bound (W / (A dx)) would exceed one with the boost
    boost = 1.0 if (dsmc and case == "max_cells") else PARTNER_BOOST
    sig, thr, loss = build_tables(partner_boost=boost)
    g = _gpu()(wl, sig, thr, loss, precision=prec)
    o = O.Oracle(wl, sig, thr, loss, precision=prec)
    done = 0
    for target in (1, 10, 25):
        g.step(target - done)
        o.step(target - done)
        done = target
        g.sync()
        compare(g, o, prec, f"{case} {'list' if dsmc else 'null'} step {done}")
        gphi, gE = g.field()
        ophi, oE = o.field()
        assert np.array_equal(gphi, ophi) and np.array_equal(gE, oE), f"{case} step {done}: field differs"
    g.close()
    o.close()
