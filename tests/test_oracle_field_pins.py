"""Pins of the oracle's charge assignment, field gather and ion sub-cycling
(CPU only).

Linear weighting is the paper's rule for both directions, force interpolation
and charge assignment (Sec. II, item (i)).  The checks here fix it with
things other than the oracle's own formulas: the electron plasma oscillation
of a cold, neutral plasma (a closed form that needs the deposit and the
gather together), the exact field of a uniform charge read back through the
push, and the first moment of a single particle's charge.  Initial loads are
placed with the oracle's test hook (quiet starts).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import pytest
from scipy.optimize import curve_fit

from oracle import oracle as O
from tests.oracle_helpers import MASS, ME, QE, quiet, small, zero_tables

EPS0 = 8.8541878128e-12


def _place(x, dx, n_cells):
    """(cell, off) of positions x in [0, L)."""
    c = np.floor(x / dx).astype(np.int64)
    off = x / dx - c
    # rounding at a cell edge: keep off in [0, 1)
    up = off >= 1.0
    c[up] += 1
    off[up] = 0.0
    assert np.all((c >= 0) & (c < n_cells)) and np.all((off >= 0) & (off < 1))
    return c.astype(np.int32), off


def _empty():
    return (np.zeros(0, np.int32), np.zeros(0), np.zeros((0, 3)))


@pytest.mark.parametrize("wdt", [1.0, 0.3])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_langmuir_oscillation_frequency(prec, wdt):
    """A cold neutral plasma whose electrons are displaced by
    xi0 sin(2 pi x / L) oscillates at the plasma frequency: the displacement
    vanishes at both electrodes and integrates to zero, so with both
    electrodes at 0 V the field at every sheet is e n0 xi / eps0 (density
    perturbation ~ cos(2 pi x / L), potential ~ cos(2 pi x / L) - 1).  The
    leapfrog turns omega_pe into (2/dt) asin(omega_pe dt / 2).  k dx = pi / 64,
    so the grid's own corrections (linear weighting both ways, 3-point
    Poisson, centred field) are ~3e-4.  Swapping the two weights of the
    charge assignment would turn the restoring field into an anti-restoring
    one."""
    N = 128
    ppc = 32
    ne = N * ppc
    wl0 = small(n_cells=N, n_init=(ne, 0, ne), T_init_eV=(0.0, 0.0, 0.0), voltage_V=0.0,
                pressure_Pa=0.0, coulomb_every=0)
    L = wl0.gap_m
    dx = L / N
    dt = 1.0 / (wl0.frequency_Hz * wl0.steps_per_period)
    wpe = wdt / dt
    n0 = wpe ** 2 * EPS0 * ME / QE ** 2
    W = n0 * wl0.area_m2 * L / ne
    wl = dataclasses.replace(wl0, weight=W)
    sig, thr, loss = zero_tables()
    o = O.Oracle(wl, sig, thr, loss, precision=prec)
    x0 = (np.arange(ne) + 0.5) * (L / ne)
    xi0 = 0.2 * dx
    ce, oe = _place(x0 + xi0 * np.sin(2 * np.pi * x0 / L), dx, N)
    ci, oi = _place(x0, dx, N)
    o.load([(ce, oe, np.zeros((ne, 3))), _empty(), (ci, oi, np.zeros((ne, 3)))])
    steps = 400 if wdt < 0.5 else 120
    phi_mid = []
    for _ in range(steps):
        o.step(1)
        phi_mid.append(o.field()[0][N // 2])
    y = np.array(phi_mid)
    n = np.arange(1, steps + 1, dtype=float)
    expect = 2.0 * math.asin(wdt / 2.0)              # radians per step

    def model(t, a, b, w, c):
        return a * np.cos(w * t) + b * np.sin(w * t) + c

    p, _ = curve_fit(model, n, y, p0=(y[0], 0.0, expect * 1.01, 0.0))
    assert abs(p[2] / expect - 1) < 1e-3, (p[2], expect, wdt)
    # and not the frequency without the leapfrog's correction (where it is resolvable)
    if wdt >= 1.0:
        assert abs(p[2] / wdt - 1) > 0.03
    # the oscillation keeps its amplitude (no numerical heating or damping of the mode)
    amp = math.hypot(p[0], p[1])
    assert np.max(np.abs(y - p[3])) < 1.05 * amp
    o.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 2e-5)])
def test_gather_reads_linear_field_exactly(prec, tol):
    """A uniform ion charge between the electrodes (quiet start, a power of
    two per cell, so every interior node holds the same charge and the
    boundary nodes half of it) gives the field U/L - rho (L/2 - x)/eps0, exact
    at the nodes and linear between them; linear interpolation must return
    it at every particle position.  The field a particle felt is read back
    from the leapfrog's initial half step v(-dt/2) = -(q/m) E(x) dt/2 of a
    particle at rest.  The few test electrons add a charge of relative size
    n_e / n_i to the field (the tolerance covers it)."""
    N, ppc = 16, 4096
    ni = N * ppc
    ne = 24
    U = 37.0
    wl0 = quiet(small(n_cells=N, n_init=(ne, 0, ni), T_init_eV=(0.0, 0.0, 0.0), pressure_Pa=0.0),
                voltage_V=U)
    L = wl0.gap_m
    dx = L / N
    W = 1e6
    wl = dataclasses.replace(wl0, weight=W)
    sig, thr, loss = zero_tables()
    o = O.Oracle(wl, sig, thr, loss, precision=prec, drive_dc=True)
    ci = np.repeat(np.arange(N), ppc).astype(np.int32)
    oi = np.tile((np.arange(ppc) + 0.5) / ppc, N)
    rs = np.random.default_rng(3)
    xe = rs.uniform(0.02 * L, 0.98 * L, ne)
    ce, oe = _place(xe, dx, N)
    o.load([(ce, oe, np.zeros((ne, 3))), _empty(), (ci, oi, np.zeros((ni, 3)))])
    dt = 1.0 / (wl.frequency_Hz * wl.steps_per_period)
    ids, c, f, v = o.particles(0)
    x = (c + f) * dx
    E_read = v[:, 0] * 2.0 * ME / (QE * dt)           # q = -e: v = +e E dt / (2 m)
    rho = QE * W * ppc / (wl.area_m2 * dx)
    E_exact = U / L - rho / EPS0 * (L / 2 - x)
    scale = np.max(np.abs(E_exact))
    assert np.max(np.abs(E_read - E_exact)) < max(tol, 3.0 * ne / ni) * scale
    # swapped weights would be off by up to rho dx / eps0 (1 / 8 of the scale here)
    assert rho * dx / EPS0 > 0.1 * scale
    o.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_single_particle_charge_assignment(prec):
    """Linear weighting of one particle: its charge 2^24 splits between the
    two nodes of its cell, and the first moment of the node charge is the
    particle's position (to the 2^-24 resolution of the fixed point)."""
    N = 8
    wl = quiet(small(n_cells=N, n_init=(1, 0, 0)))
    sig, thr, loss = zero_tables()
    dt = np.float32 if prec == "fp32" else np.float64
    for cell, off in [(0, 0.0), (3, 0.25), (5, 0.7), (7, 1 - 2.0**-20), (2, 0.123456789)]:
        o = O.Oracle(wl, sig, thr, loss, precision=prec)
        o.load([(np.array([cell], np.int32), np.array([off]), np.zeros((1, 3))), _empty(), _empty()])
        Q = o.charge()[0]
        assert Q.sum() == 2**24
        assert np.count_nonzero(Q) <= 2 and Q.min() >= 0
        assert set(np.nonzero(Q)[0]) <= {cell, cell + 1}
        centroid = (np.arange(N + 1) * Q).sum() / 2**24
        assert abs(centroid - (cell + float(dt(off)))) <= 2.0**-24
        o.close()


@pytest.mark.parametrize("nsub", [3, 10])
def test_subcycled_ions_move_every_nsub_steps(nsub):
    """With ion sub-cycling the ions are moved at the steps n with
    n mod n_sub = 0, each time by v n_sub dt (free flight, no field); the
    electrons every step by v dt."""
    wl = quiet(small(n_init=(2000, 1000, 2000), T_init_eV=(3.0, 1.0, 1.0), ion_subcycle=nsub,
                     sort_every=nsub, pressure_Pa=0.0))
    sig, thr, loss = zero_tables()
    o = O.Oracle(wl, sig, thr, loss, precision="fp64")
    dx = wl.gap_m / wl.n_cells
    dt = 1.0 / (wl.frequency_Hz * wl.steps_per_period)
    start = [o.particles(s) for s in range(3)]
    for steps in (1, nsub - 1, nsub, nsub + 1, 4 * nsub + 2):
        o.step(steps - o.counters()[2]["step"])
        for s in range(3):
            pushes = steps if s == 0 else -(-steps // nsub)     # ceil(steps / nsub)
            tau = dt if s == 0 else nsub * dt
            ids0, c0, f0, v0 = start[s]
            ids1, c1, f1, v1 = o.particles(s)
            pos = {int(k): i for i, k in enumerate(ids0)}
            idx = np.array([pos[int(k)] for k in ids1])
            ref = (c0[idx] + f0[idx]) * dx + v0[idx, 0] * pushes * tau
            assert np.max(np.abs((c1 + f1) * dx - ref)) < 1e-9 * dx, (s, steps)
    o.close()
