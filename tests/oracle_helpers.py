"""Shared helpers for the oracle pin tests and the GPU parity tests."""
from __future__ import annotations

import dataclasses

import numpy as np

from pic_inputs import build_tables, workload
from pic_inputs.configs import Workload

QE = 1.602176634e-19
KB = 1.380649e-23
ME = 9.1093837015e-31
AMU = 1.66053906660e-27
MO2 = 31.998 * AMU
MASS = (ME, 15.999 * AMU + ME, MO2 - ME)

# The partner reactions (13), (14), (19) are rare with the stand-in cross
# sections.  Tests of pairing, claims and the partner path of the step's end
# scale those three channels by this factor: on the small discharge
# (W = 2210, 10k particles) the partner slots then take about a quarter of the
# electrons' null-collision bound, about 75 requests and 0.7 accepted partner
# events per step.
PARTNER_BOOST = 1.0e5


def quiet(wl: Workload, **kw) -> Workload:
    """A workload with (almost) no self field and no Coulomb collisions:
    tiny weight, no drive."""
    base = dict(weight=1e-30, voltage_V=0.0, coulomb_every=0)
    base.update(kw)
    return dataclasses.replace(wl.resolved(), **base)


def zero_tables():
    sig, thr, loss = build_tables()
    return np.zeros_like(sig), thr, loss


def tables_only(channels, partner_boost=1.0):
    """The stand-in tables with every channel not listed set to zero."""
    sig, thr, loss = build_tables(partner_boost=partner_boost)
    keep = np.zeros(sig.shape[0], bool)
    keep[list(channels)] = True
    sig[~keep] = 0.0
    return sig, thr, loss


def small(**kw):
    return dataclasses.replace(workload("small"), **kw)
