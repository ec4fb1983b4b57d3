"""Pins of the oracle's per-cell collision list (Sec. II, Eq. (1); switch
``dsmc``): every sort_every steps the particles of each cell go through the
collision types (4)-(19) of Table I in order, each with P = n_j sigma_j u tau,
tau = sort_every dt; products take part in the later types; the partner
populations of a type are those at its start.

The pins use cross sections sigma_j = K_j / g(E) (g the relative speed at
relative energy E for the channel's reduced mass), so that sigma_j u = K_j and
every decision of a type has the same probability; the expected counts are
then closed forms of the populations."""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import pytest

from oracle import oracle as O
from pic_inputs import build_tables, energy_grid
from tests.oracle_helpers import KB, MASS, MO2, PARTNER_BOOST, QE, small

MU_GAS = [m * MO2 / (m + MO2) for m in MASS]
PAIR = {12: (0, 2), 13: (0, 1), 17: (1, 2)}


def mu_of(j):
    if j in PAIR:
        s, t = PAIR[j]
        return MASS[s] * MASS[t] / (MASS[s] + MASS[t])
    s = 0 if j <= 11 else (1 if j <= 16 else 2)
    return MU_GAS[s]


def const_rate_tables(K: dict):
    """sigma_j = K_j / g(E) for the listed channels (threshold and loss 0), all
    other channels closed."""
    sig, thr, loss = build_tables()
    sig[:] = 0.0
    E = energy_grid()
    for j, k in K.items():
        sig[j] = k / np.sqrt(2.0 * E * QE / mu_of(j))
        thr[j] = 0.0
        loss[j] = 0.0
    return sig, thr, loss


def quiet_list(**kw):
    base = dict(weight=1e-30, voltage_V=0.0, coulomb_every=0, dsmc=True, sort_every=10, ion_subcycle=1)
    base.update(kw)
    return small(**base)


def tau_of(wl):
    return wl.sort_every / (wl.frequency_Hz * wl.steps_per_period)


def n_gas(wl):
    return wl.pressure_Pa / (KB * wl.T_gas_K)


def within(count, n, p, k=4.5):
    """count against a binomial(n, p) mean, k standard deviations."""
    mean = n * p
    sd = math.sqrt(max(n * p * (1.0 - p), 1.0))
    return abs(count - mean) <= k * sd, (count, mean, sd)


# ----------------------------------------------------------------------------
# gas types: probability n sigma u tau with tau = sort_every dt
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_gas_types_are_independent_decisions_with_list_tau(prec):
    """Electrons only; elastic (4) with P = 0.7 and the vibrational type (7)
    (four levels, one decision) with P = 0.6 in total.  The two types decide
    one after the other, so their counts are binomial over the electrons with
    these probabilities although they add up to more than one; the levels of
    (7) share its events in proportion to K."""
    wl = quiet_list(n_init=(20_000, 0, 0), T_init_eV=(3.0, 0.026, 0.026))
    f = n_gas(wl) * tau_of(wl)
    P4, P7 = 0.7, 0.6
    lev = np.array([1.0, 2.0, 3.0, 4.0]) / 10.0
    K = {0: P4 / f}
    for q in range(4):
        K[1 + q] = P7 * lev[q] / f
    o = O.Oracle(wl, *const_rate_tables(K), precision=prec, field_off=True)
    o.step(wl.sort_every - 1)
    assert not o.counters()[0].any()              # no collision during the free flights
    o.step(1)
    ev, ab, misc = o.counters()
    n = o.alive(0)                                # elastic and zero-loss excitation keep every electron
    ok, info = within(ev[0], n, P4)
    assert ok, info
    ok, info = within(ev[1:5].sum(), n, P7)
    assert ok, info
    for q in range(4):
        ok, info = within(ev[1 + q], n, P7 * lev[q])
        assert ok, (q, info)
    assert not ev[5:].any()
    # with tau = dt (the null-collision step) the counts would be ten times lower
    assert ev[0] > 5 * n * P4 / wl.sort_every


def test_gas_type_rate_follows_the_table_with_reduced_mass():
    """The stand-in elastic table (4) and a nearly cold gas: each electron's
    probability is n sigma(E) g tau with E = mu g^2 / 2 (mu the e-O2 reduced
    mass) and g its own speed."""
    T_gas = 1.0
    wl0 = quiet_list(n_init=(20_000, 0, 0), T_init_eV=(5.0, 0.026, 0.026), T_gas_K=T_gas)
    # the gas density of 10 Pa at 300 K, held at 1 K
    wl = dataclasses.replace(wl0, pressure_Pa=10.0 * T_gas / 300.0)
    sig, thr, loss = build_tables()
    keep = np.zeros(sig.shape[0], bool)
    keep[0] = True
    sig[~keep] = 0.0
    # scale the table so that the largest probability stays below one
    tau = tau_of(wl)
    E = energy_grid()
    g = np.sqrt(2.0 * E * QE / MU_GAS[0])
    scale = 0.5 / (n_gas(wl) * tau * float(np.max(sig[0] * g)))
    sig[0] *= scale
    o = O.Oracle(wl, sig, thr, loss, precision="fp64", field_off=True)
    o.step(wl.sort_every - 1)
    _, _, _, v = o.particles(0)
    o.step(1)
    ev = o.counters()[0]
    sp = np.sqrt((v ** 2).sum(axis=1))
    Ei = 0.5 * MU_GAS[0] * sp ** 2 / QE
    P = n_gas(wl) * tau * np.interp(Ei, E, sig[0]) * sp
    mean = float(P.sum())
    sd = math.sqrt(float((P * (1 - P)).sum()))
    assert mean > 2000
    assert abs(ev[0] - mean) < 4.5 * sd, (ev[0], mean, sd)


# ----------------------------------------------------------------------------
# products take part in the later types of the same pass
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_products_take_part_in_later_types(prec):
    """Electrons only; attachment (15) with P = 0.5 makes O-, associative
    detachment (17) with P = 0.4 acts on them in the same pass.  Under a
    scheme that placed the products only after the pass, (17) would not
    occur before the second pass."""
    wl = quiet_list(n_init=(20_000, 0, 0), T_init_eV=(3.0, 0.026, 0.026))
    f = n_gas(wl) * tau_of(wl)
    P15, P17 = 0.5, 0.4
    K = {10: P15 / f, 16: P17 / (wl.metastable_frac * f)}
    o = O.Oracle(wl, *const_rate_tables(K), precision=prec, field_off=True)
    o.step(wl.sort_every - 1)
    n0 = o.alive(0)
    ab0 = o.counters()[1].sum(axis=0)
    o.step(1)
    ev, ab, misc = o.counters()
    # electrons at the pass: those left after the last free flight
    n0 = n0 - int(ab.sum(axis=0)[0] - ab0[0])
    ok, info = within(ev[10], n0, P15)
    assert ok, info
    ok, info = within(ev[16], int(ev[10]), P17)
    assert ok, info
    assert ev[16] > 0.3 * ev[10]
    assert o.alive(0) == n0 - ev[10] + ev[16]
    assert o.alive(1) == ev[10] - ev[16]
    assert misc["births"] == ev[10] + ev[16]


# ----------------------------------------------------------------------------
# partner types: populations at the start of each type, one partner per test
# particle, smallest id wins a contested partner
# ----------------------------------------------------------------------------
def _cell_load(n_cells, cells, per, speeds, seed=7):
    """Particles at rest in x (v_x = 0), moving along y: per[s] of species s
    in each listed cell."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in range(3):
        k = per[s] * len(cells)
        vs = np.zeros((k, 3))
        vs[:, 1] = speeds[s] * rng.uniform(0.5, 1.5, k)
        parts.append((np.repeat(np.asarray(cells, np.int32), per[s]), rng.uniform(0.05, 0.95, k), vs))
    return parts


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_partner_types_use_the_populations_at_their_start(prec):
    """32 cells with 300 e, 150 O- and 40 O2+ each, nobody moving along x.
    (13) e + O2+: each electron accepts with P = N_p kappa13 and takes one
    O2+ of its cell at random, so an O2+ survives with (1 - kappa13)^300.
    (14) O- + O2+ then sees the survivors only: each is taken with
    1 - (1 - kappa14)^150.  Closed forms of both counts."""
    n_cells = 64
    cells = list(range(16, 48))
    Ne, Nn, Np = 300, 150, 40
    k13, k14 = 1.0 / 300.0, 1.0 / 150.0
    wl = quiet_list(n_cells=n_cells, n_init=(Ne * 32, Nn * 32, Np * 32), weight=1.0)
    dx = wl.gap_m / wl.n_cells
    KPl = tau_of(wl) * wl.weight / (wl.area_m2 * dx)
    o = O.Oracle(wl, *const_rate_tables({12: k13 / KPl, 17: k14 / KPl}), precision=prec, field_off=True)
    o.load(_cell_load(n_cells, cells, (Ne, Nn, Np), (1e5, 2e3, 0.0)))
    o.step(wl.sort_every)
    ev, ab, misc = o.counters()
    assert not ab.any()
    n_p = Np * len(cells)
    s13 = (1.0 - k13) ** Ne
    ok, info = within(ev[12], n_p, 1.0 - s13)
    assert ok, info
    ok, info = within(ev[17], n_p, s13 * (1.0 - (1.0 - k14) ** Nn))
    assert ok, info
    assert o.alive(2) == n_p - ev[12] - ev[17]
    assert o.alive(0) == Ne * len(cells) - ev[12]
    assert o.alive(1) == Nn * len(cells) - ev[17]
    assert misc["accepted"] == ev[12] + ev[17]
    assert misc["requests"] >= misc["accepted"]


def test_impact_detachment_takes_o_minus_born_in_the_same_pass():
    """Attachment (15) with P = 0.5 on 300 electrons per cell, then impact
    detachment (19) with the O- of the cell, all of which were born in this
    pass: none of (19) is possible without the products of (15)."""
    n_cells = 64
    cells = list(range(16, 48))
    Ne = 300
    wl = quiet_list(n_cells=n_cells, n_init=(Ne * 32, 0, 0), weight=1.0)
    dx = wl.gap_m / wl.n_cells
    KPl = tau_of(wl) * wl.weight / (wl.area_m2 * dx)
    f = n_gas(wl) * tau_of(wl)
    k19 = 1.0 / 400.0
    o = O.Oracle(wl, *const_rate_tables({10: 0.5 / f, 13: k19 / KPl}), precision="fp64", field_off=True)
    load = _cell_load(n_cells, cells, (Ne, 0, 0), (1e5, 0.0, 0.0))
    o.load(load)
    o.step(wl.sort_every)
    ev, ab, misc = o.counters()
    assert ev[10] > 4000 and ev[13] > 0
    # X electrons of a cell survive (15) (binomial(300, 1/2)); its 300 - X O- are
    # each taken by one of them with 1 - (1 - k19)^X
    from scipy.stats import binom
    X = np.arange(Ne + 1)
    pmf = binom.pmf(X, Ne, 0.5)
    per_cell = float(np.sum(pmf * (Ne - X) * (1.0 - (1.0 - k19) ** X)))
    mean = per_cell * len(cells)
    ok, info = within(ev[13], int(ev[10]), mean / float(ev[10]))
    assert ok, info
    assert o.alive(1) == ev[10] - ev[13]
    assert o.alive(0) == Ne * len(cells) - ev[10] + ev[13]


# ----------------------------------------------------------------------------
# guards, conservation, balance
# ----------------------------------------------------------------------------
def test_list_bounds_are_checked():
    wl = quiet_list(n_init=(2000, 0, 0))
    f = n_gas(wl) * tau_of(wl)
    with pytest.raises(RuntimeError):
        O.Oracle(wl, *const_rate_tables({0: 1.2 / f}), precision="fp64", field_off=True)
    with pytest.raises(RuntimeError):
        O.Oracle(dataclasses.replace(wl, ion_subcycle=3), *const_rate_tables({0: 0.5 / f}), precision="fp64")
    # partner bound above one in a cell with test particles: guard at the pass
    n_cells = 64
    wlp = quiet_list(n_cells=n_cells, n_init=(32 * 10, 0, 32 * 40), weight=1.0)
    dx = wlp.gap_m / n_cells
    KPl = tau_of(wlp) * wlp.weight / (wlp.area_m2 * dx)
    o = O.Oracle(wlp, *const_rate_tables({12: (1.0 / 30.0) / KPl}), precision="fp64", field_off=True)
    o.load(_cell_load(n_cells, list(range(16, 48)), (10, 0, 40), (1e5, 0.0, 0.0)))
    with pytest.raises(RuntimeError):
        o.step(wlp.sort_every)


def _list_small(**kw):
    return dataclasses.replace(small(**kw), dsmc=True)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_count_balance_every_pass(prec):
    sig, thr, loss = build_tables(partner_boost=PARTNER_BOOST)
    wl = _list_small()
    o = O.Oracle(wl, sig, thr, loss, precision=prec)
    prev_ev, prev_ab, _ = o.counters()
    prev_n = [o.alive(s) for s in range(3)]
    for _ in range(15):
        o.step(wl.sort_every)
        ev, ab, _ = o.counters()
        d = ev - prev_ev
        da = (ab - prev_ab).sum(axis=0)
        n = [o.alive(s) for s in range(3)]
        assert n[0] - prev_n[0] == d[11] + d[15] + d[16] + d[13] - d[10] - d[12] - da[0]
        assert n[1] - prev_n[1] == d[10] - d[17] - d[15] - d[16] - d[13] - da[1]
        assert n[2] - prev_n[2] == d[11] - d[12] - d[17] - da[2]
        prev_ev, prev_ab, prev_n = ev, ab, n
    ev, ab, misc = o.counters()
    assert ev[12] > 0 and ev[13] > 0 and ev[17] > 0, ev
    ids = np.concatenate([o.particles(s)[0] for s in range(3)])
    assert len(np.unique(ids)) == len(ids)
    assert misc["next_id"] == sum(wl.n_init) + misc["births"]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 3e-5)])
def test_per_event_conservation_in_the_list(prec, tol):
    sig, thr, loss = build_tables(partner_boost=PARTNER_BOOST)
    o = O.Oracle(_list_small(), sig, thr, loss, precision=prec)
    o.log_enable(400_000)
    o.step(200)
    log = o.log()
    assert len(log) > 1000
    chans = set()
    for e in log:
        j = int(e[0])
        chans.add(j)
        if j in (10, 12, 17):
            continue
        if j in (15, 16):
            assert e[11] == pytest.approx((0.1 if j == 15 else 1.0) * e[12], rel=1e-5 if prec == "fp32" else 1e-12)
            continue
        pb, pa = e[4:7], e[7:10]
        assert np.max(np.abs(pa - pb)) <= tol * np.max(np.abs(pb)) + 1e-40
        dE = e[2] - e[3] - e[10] * QE
        assert abs(dE) <= 4 * tol * e[2] + 1e-30, (j, dE, e[2])
    assert {0, 1, 6, 11, 13, 14, 18} <= chans


def test_list_and_null_collision_schemes_agree_statistically():
    """Both schemes realise Eq. (1); over 400 steps of the small discharge the
    gas-channel event counts agree within their Poisson spread."""
    sig, thr, loss = build_tables()
    a = O.Oracle(small(), sig, thr, loss, precision="fp32")
    b = O.Oracle(_list_small(), sig, thr, loss, precision="fp32")
    a.step(400)
    b.step(400)
    ea, eb = a.counters()[0], b.counters()[0]
    for j in (0, 5, 6, 7, 11, 14, 18):
        m = 0.5 * (ea[j] + eb[j])
        assert m > 50
        assert abs(int(ea[j]) - int(eb[j])) < 5.0 * math.sqrt(2.0 * m) + 0.05 * m, (j, ea[j], eb[j])
