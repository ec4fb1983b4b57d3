"""Pins of the CPU oracle against things other than itself.

Each test checks the oracle against a closed form, an invariant, a special
case that reduces to a library routine, or a statement of the paper.  All run
on the CPU (no GPU).
"""
from __future__ import annotations

import dataclasses
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy.linalg import solve_banded

from oracle import oracle as O
from pic_inputs import build_tables, energy_grid
from pic_inputs import xsec as X
from tests.oracle_helpers import (KB, MASS, ME, MO2, PARTNER_BOOST, QE, quiet, small, tables_only,
                                  zero_tables)

HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------------------------
# random numbers
# ----------------------------------------------------------------------------
@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc (rocRAND headers) not available")
def test_philox_matches_rocrand(tmp_path):
    """Philox4x32-10 block function equals rocRAND's (library routine)."""
    exe = tmp_path / "ref"
    subprocess.check_call(["hipcc", "-O1", "-o", str(exe), os.path.join(HERE, "philox_rocrand_ref.cpp")])
    rs = np.random.default_rng(12345)
    cases = [([0, 0, 0, 0], [0, 0]), ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2)]
    for _ in range(200):
        cases.append((list(rs.integers(0, 2**32, 4)), list(rs.integers(0, 2**32, 2))))
    inp = "\n".join(" ".join("%x" % v for v in c + k) for c, k in cases) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for (c, k), line in zip(cases, out):
        ref = [int(x, 16) for x in line.split()]
        assert O.philox([int(v) for v in c], [int(v) for v in k]) == ref


# ----------------------------------------------------------------------------
# cross-section tables and their interpolation
# ----------------------------------------------------------------------------
def test_grid_is_binade_grid():
    E = energy_grid()
    assert E[0] == 2.0**-14 and E[-1] == 2.0**14 and len(E) == 897
    assert np.all(np.diff(E) > 0)
    # 32 equal steps per binade
    for b in range(28):
        seg = E[32 * b: 32 * b + 33]
        assert np.allclose(np.diff(seg), seg[0] / 32.0, rtol=0, atol=0)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_interpolation_nodes_and_ends(prec):
    sig, thr, loss = build_tables()
    o = O.Oracle(quiet(small(n_init=(10, 10, 10))), sig, thr, loss, precision=prec)
    E = energy_grid()
    dt = np.float32 if prec == "fp32" else np.float64
    for j in (0, 11, 14, 16, 17, 18):
        for k in (0, 1, 100, 480, 895, 896):
            assert o.sigma(j, E[k]) == float(dt(sig[j, k]))
        # clamped below the first node and above the last one
        assert o.sigma(j, 1e-6) == float(dt(sig[j, 0]))
        assert o.sigma(j, 1e6) == float(dt(sig[j, -1]))
        # linear in E inside a segment
        for k in (3, 300, 700):
            Em = 0.5 * (E[k] + E[k + 1])
            assert o.sigma(j, Em) == pytest.approx(0.5 * (sig[j, k] + sig[j, k + 1]), rel=2e-6)


@pytest.mark.parametrize("E", [0.01, 0.026, 0.1, 1.0, 10.0, 100.0])
def test_interpolated_closed_forms(E):
    """Eq. (4), (8), (9) of the paper, evaluated directly, against the oracle's
    interpolated table (interpolation error of a convex 1/E^a on a grid of
    32 points per binade is < 2e-4)."""
    sig, thr, loss = build_tables()
    o = O.Oracle(quiet(small(n_init=(10, 10, 10))), sig, thr, loss, precision="fp64")
    okada = (3 * math.pi * (0.5 * 3.77e-24 / E) ** (2.0 / 3.0) + 1.2e-15) * 1e-4
    lz = 0.8 * (1 + 2.85 / E) * 1e-14 * 1e-4
    ad = 5.96e-16 / math.sqrt(E) * 1e-4
    assert o.sigma(14, E) == pytest.approx(okada, rel=2e-4)
    assert o.sigma(17, E) == pytest.approx(lz, rel=2e-4)
    assert o.sigma(16, E) == pytest.approx(ad, rel=2e-4)


def test_paper_thresholds_respected():
    sig, thr, loss = build_tables()
    E = energy_grid()
    assert np.all(sig[6, E < 6.4] == 0) and sig[6, E > 6.5].min() > 0      # (9) 6.4 eV
    assert np.all(sig[7, E < 8.6] == 0)                                     # (10) 8.6 eV
    assert np.all(sig[15, E < 1.3] == 0)                                    # (16) ~1.3 eV
    assert np.all(sig[10, E < 4.0] == 0)                                    # (15) zero below 4 eV
    # associative detachment dominates direct detachment below about 6 eV
    lo = (E > 1.4) & (E < 5.5)
    assert np.all(sig[16, lo] > sig[15, lo])
    hi = E > 7.0
    assert np.all(sig[16, hi] < sig[15, hi])
    # charge exchange: half the momentum-transfer value outside [0.251, 8.5] eV
    out = (E < 0.251) | (E > 8.5)
    assert np.allclose(sig[18, out], 0.5 * X._sigma_momentum_o2p(E[out]))


# ----------------------------------------------------------------------------
# field solve
# ----------------------------------------------------------------------------
def test_poisson_matches_banded_solver():
    rs = np.random.default_rng(7)
    N, dx, cphi, cE, U0 = 200, 1e-4, 3.7e-9, 2.2e-6, 123.4
    q = rs.integers(-2**40, 2**40, N + 1)
    phi, E = O.solve_field(q, dx, cphi, cE, U0)
    ab = np.zeros((3, N - 1))
    ab[0, 1:] = -1.0
    ab[1, :] = 2.0
    ab[2, :-1] = -1.0
    rhs = cphi * q[1:N].astype(float)
    rhs[0] += U0
    ref = solve_banded((1, 1), ab, rhs)
    scale = np.abs(ref).max()
    assert np.max(np.abs(phi[1:N] - ref)) < 1e-11 * scale
    assert phi[0] == U0 and phi[N] == 0.0
    assert np.allclose(E[1:N], (phi[0:N - 1] - phi[2:N + 1]) / (2 * dx), rtol=1e-14, atol=0)


def test_poisson_uniform_charge_is_exact_parabola():
    """The 3-point scheme is exact for a quadratic potential; the half-cell
    Gauss boundary field equals U/L - rho L/(2 eps0) exactly."""
    N, dx, U0 = 128, 3.125e-4, 50.0
    A, W = 5.5e-7, 1234.5
    EPS0 = 8.8541878128e-12
    cphi = ((dx * QE) * W) / ((EPS0 * 16777216.0) * A)
    cE = (QE * W) / ((EPS0 * 16777216.0) * A)
    qv = 3 * 2**24
    q = np.full(N + 1, qv, np.int64)
    q[0] = q[N] = qv // 2
    phi, E = O.solve_field(q, dx, cphi, cE, U0)
    i = np.arange(N + 1)
    exact = U0 * (1 - i / N) + cphi * qv * i * (N - i) / 2.0
    assert np.max(np.abs(phi - exact)) < 1e-13 * np.abs(exact).max()
    rho = QE * W * qv / (16777216.0 * A * dx)
    L = N * dx
    assert E[0] == pytest.approx(U0 / L - rho * L / (2 * EPS0), rel=1e-12)
    assert E[N] == pytest.approx(U0 / L + rho * L / (2 * EPS0), rel=1e-12)
    x = i * dx
    assert np.allclose(E[1:N], (U0 / L - rho / EPS0 * (L / 2 - x))[1:N], rtol=1e-11, atol=1e-9)


@pytest.mark.parametrize("mode", [1, 3, 10])
def test_poisson_sine_mode(mode):
    N, dx, cphi = 64, 1e-3, 1e-9
    i = np.arange(N + 1)
    Qa = 2**55
    q = np.rint(Qa * np.sin(np.pi * mode * i / N)).astype(np.int64)
    phi, _ = O.solve_field(q, dx, cphi, 0.0, 0.0)
    # discrete eigenfunction: phi = cphi q / (4 sin^2(pi m / 2N))
    ref = cphi * q / (4 * np.sin(np.pi * mode / (2 * N)) ** 2)
    assert np.max(np.abs(phi - ref)) < 1e-12 * np.abs(ref).max()


# ----------------------------------------------------------------------------
# push and deposit
# ----------------------------------------------------------------------------
def _x(cell, off, dx):
    return (cell + off) * dx


def test_free_flight_fp64():
    wl = quiet(small(n_init=(2000, 500, 2000)))
    sig, thr, loss = zero_tables()
    o = O.Oracle(wl, sig, thr, loss, precision="fp64")
    dx = wl.gap_m / wl.n_cells
    dt = 1.0 / (wl.frequency_Hz * wl.steps_per_period)
    start = [o.particles(s) for s in range(3)]
    nst = 40
    o.step(nst)
    for s in range(3):
        ids0, c0, f0, v0 = start[s]
        ids1, c1, f1, v1 = o.particles(s)
        pos = {int(k): i for i, k in enumerate(ids0)}
        idx = np.array([pos[int(k)] for k in ids1])
        x0 = _x(c0[idx], f0[idx], dx)
        x1 = _x(c1, f1, dx)
        ref = x0 + v0[idx, 0] * nst * dt
        assert np.max(np.abs(x1 - ref)) < 1e-9 * dx
        assert np.array_equal(v1, v0[idx])
        # everything that left crossed an electrode in straight flight
        gone = np.setdiff1d(ids0, ids1)
        if len(gone):
            g = np.array([pos[int(k)] for k in gone])
            xf = _x(c0[g], f0[g], dx) + v0[g, 0] * nst * dt
            assert np.all((xf < 1e-9 * dx) | (xf >= wl.gap_m - 1e-9 * dx))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 2e-3)])
def test_uniform_field_orbit(prec, tol):
    """With a constant field the leapfrog is exact: x_n = x0 + v0 t + a t^2/2."""
    U = 2.0
    wl = quiet(small(n_init=(3000, 0, 3000)), voltage_V=U)
    sig, thr, loss = zero_tables()
    o = O.Oracle(wl, sig, thr, loss, precision=prec, drive_dc=True)
    dx = wl.gap_m / wl.n_cells
    dt = 1.0 / (wl.frequency_Hz * wl.steps_per_period)
    Efield = U / wl.gap_m
    start = [o.particles(s) for s in range(3)]
    nst = 30
    o.step(nst)
    for s, q in ((0, -QE), (2, QE)):
        a = q * Efield / MASS[s]
        ids0, c0, f0, v0 = start[s]
        ids1, c1, f1, v1 = o.particles(s)
        pos = {int(k): i for i, k in enumerate(ids0)}
        idx = np.array([pos[int(k)] for k in ids1])
        # stored velocity at t=0 is v(-dt/2)
        vstart = v0[idx, 0] + a * dt / 2
        t = nst * dt
        ref = _x(c0[idx], f0[idx], dx) + vstart * t + 0.5 * a * t * t
        assert np.max(np.abs(_x(c1, f1, dx) - ref)) < tol * dx
        assert np.allclose(v1[:, 0], vstart + a * (nst - 0.5) * dt, rtol=1e-5 if prec == "fp32" else 1e-12,
                           atol=1e-3 if prec == "fp32" else 1e-9)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_deposit_total_is_exact(prec):
    sig, thr, loss = build_tables()
    o = O.Oracle(small(), sig, thr, loss, precision=prec)
    for _ in range(3):
        o.step(37)
        Q = o.charge()
        for s in range(3):
            assert Q[s].sum() == o.alive(s) * 2**24
            assert Q[s].min() >= 0


# ----------------------------------------------------------------------------
# null-collision rates against Maxwellian integrals of the tables
# ----------------------------------------------------------------------------
def _maxwell_rate(sig_row, thr_eV, mu, kT_eV):
    """<sigma(E) g> for a relative energy distributed as a Maxwellian with
    temperature kT_eV, sigma = the piecewise-linear table (closed below thr)."""
    E = energy_grid()
    xg, wg = np.polynomial.legendre.leggauss(16)
    total = 0.0
    def f(e):  # E * exp(-E/kT) weight of <sigma g> after the change of variables
        return e * np.exp(-e / kT_eV)
    # below the first node sigma is constant
    a, b = 0.0, E[0]
    ee = 0.5 * (b - a) * xg + 0.5 * (b + a)
    total += np.sum(wg * 0.5 * (b - a) * np.where(ee >= thr_eV, sig_row[0], 0.0) * f(ee))
    for k in range(len(E) - 1):
        a, b = E[k], E[k + 1]
        if a > 60 * kT_eV:
            break
        ee = 0.5 * (b - a) * xg + 0.5 * (b + a)
        s = sig_row[k] + (sig_row[k + 1] - sig_row[k]) * (ee - a) / (b - a)
        s = np.where(ee >= thr_eV, s, 0.0)
        total += np.sum(wg * 0.5 * (b - a) * s * f(ee))
    # <sigma g> = sqrt(8 e / (pi mu)) (kT)^{-3/2} int sigma E exp(-E/kT) dE   (E, kT in eV)
    return math.sqrt(8.0 * QE / (math.pi * mu)) * kT_eV ** -1.5 * total


@pytest.mark.parametrize("T_eV", [3.0, 10.0])
def test_electron_channel_rates_fp64(T_eV):
    """Fresh Maxwellian load, no field, one step: the events of every gas
    channel are binomial with mean N tau n_gas <sigma_j g>, Eq. (1), where the
    average is over the relative energy, itself Maxwellian with
    kT_eff = mu (kT_e/m_e + kT_g/M)."""
    ne = 300_000
    wl = quiet(small(n_init=(ne, 0, 0), T_init_eV=(T_eV, 0.026, 0.026)), weight=1e-30)
    sig, thr, loss = tables_only(range(12))
    # scale the weak channels up so that every channel is tested with >= ~100 events
    for j, f in ((1, 30), (2, 30), (3, 30), (4, 30), (5, 20), (8, 200), (9, 400), (10, 150), (11, 4)):
        sig[j] *= f
    o = O.Oracle(wl, sig, thr, loss, precision="fp64")
    assert o.constants()["pmax_e"] < 1.0
    o.step(1)
    ev, ab, misc = o.counters()
    n_mcc = misc["psteps"] - ab[:, 0].sum()
    dt = 1.0 / (wl.frequency_Hz * wl.steps_per_period)
    ngas = wl.pressure_Pa / (KB * wl.T_gas_K)
    mu = ME * MO2 / (ME + MO2)
    kT = mu * (wl.T_init_eV[0] * QE / ME + KB * wl.T_gas_K / MO2) / QE
    checked = 0
    for j in range(12):
        lam = n_mcc * dt * ngas * _maxwell_rate(sig[j], thr[j], mu, kT)
        if lam < 30:
            assert ev[j] < lam + 6 * math.sqrt(lam) + 6
            continue
        assert abs(ev[j] - lam) < 4.5 * math.sqrt(lam), (j, ev[j], lam)
        checked += 1
    assert checked >= (8 if T_eV < 5 else 10)


@pytest.mark.parametrize("C", [0.0, 1.0 / 6.0, 1.0 / 3.0])
@pytest.mark.parametrize("T_eV", [0.026, 1.0])
def test_associative_detachment_rate_is_distribution_free(T_eV, C):
    """sigma_ad g = const (the paper's K_ad ~ const): the AD rate per O- is
    C n_O2 K_ad for any O- distribution, K_ad = 5.96e-20 m^2 sqrt(2e/mu);
    linear in the metastable fraction C, and none at all for C = 0 (the
    ablation pair C = 0 / C = 1/6 of Sec. IV)."""
    nn = 100_000
    wl = quiet(small(n_init=(0, nn, 0), pressure_Pa=100.0, steps_per_period=100,
                     T_init_eV=(3.0, T_eV, 0.026), metastable_frac=C), weight=1e-30)
    sig, thr, loss = tables_only([16])
    o = O.Oracle(wl, sig, thr, loss, precision="fp64")
    mu = MASS[1] * MO2 / (MASS[1] + MO2)
    K = 5.96e-20 * math.sqrt(2 * QE / mu)
    assert K == pytest.approx(2.535e-16, rel=1e-3)
    dt = 1.0 / (wl.frequency_Hz * wl.steps_per_period)
    ngas = wl.pressure_Pa / (KB * wl.T_gas_K)
    p = dt * wl.metastable_frac * ngas * K
    lam = 0.0
    prev_ab = np.zeros((2, 3), np.int64)
    for _ in range(6):
        n_before = o.alive(1)
        o.step(1)
        ev, ab, misc = o.counters()
        lam += (n_before - (ab - prev_ab)[:, 1].sum()) * p
        prev_ab = ab
    if C == 0.0:
        assert ev[16] == 0
    else:
        assert abs(ev[16] - lam) < 4.5 * math.sqrt(lam), (ev[16], lam)
    assert o.alive(1) == nn - ev[16] - ab[:, 1].sum()
    assert o.alive(0) == ev[16] - ab[:, 0].sum()


def test_maxwell_molecule_relaxation():
    """Isotropic elastic scattering with a constant collision frequency
    (sigma = a / sqrt(E)) relaxes <E> - 3/2 kT_gas by (1 - kappa nu tau) per
    step, kappa = 2 m M / (m + M)^2."""
    nn = 60_000
    wl = quiet(small(n_init=(0, nn, 0), T_init_eV=(3.0, 1.0, 0.026)), weight=1e-30)
    sig, thr, loss = build_tables()
    E = energy_grid()
    mu = MASS[1] * MO2 / (MASS[1] + MO2)
    dt = 1.0 / (wl.frequency_Hz * wl.steps_per_period)
    ngas = wl.pressure_Pa / (KB * wl.T_gas_K)
    nu_tau = 0.02
    a = nu_tau / (dt * ngas * math.sqrt(2 * QE / mu))
    sig[:] = 0.0
    sig[14] = a / np.sqrt(E)
    o = O.Oracle(wl, sig, thr, loss, precision="fp64")
    kappa = 2 * MASS[1] * MO2 / (MASS[1] + MO2) ** 2
    assert kappa == pytest.approx(0.44445, rel=1e-4)
    e_gas = 1.5 * KB * wl.T_gas_K / QE

    def mean_E():
        v = o.particles(1)[3]
        return 0.5 * MASS[1] * np.mean(np.sum(v * v, axis=1)) / QE

    e0 = mean_E()
    for n in (60, 120, 240):
        o.step(n - o.counters()[2]["step"])
        pred = e_gas + (1 - kappa * nu_tau) ** n * (e0 - e_gas)
        assert mean_E() == pytest.approx(pred, rel=0.02), n


# ----------------------------------------------------------------------------
# conservation and balance
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_count_balance_every_step(prec):
    sig, thr, loss = build_tables(partner_boost=PARTNER_BOOST)
    o = O.Oracle(small(), sig, thr, loss, precision=prec)
    prev_ev, prev_ab, _ = o.counters()
    prev_n = [o.alive(s) for s in range(3)]
    for _ in range(150):
        o.step(1)
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
    assert misc["requests"] > misc["accepted"] > 0


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 3e-5)])
def test_per_event_conservation(prec, tol):
    sig, thr, loss = build_tables(partner_boost=PARTNER_BOOST)
    o = O.Oracle(small(), sig, thr, loss, precision=prec)
    o.log_enable(400_000)
    o.step(200)
    log = o.log()
    assert len(log) > 1000
    chans = set()
    for e in log:
        j = int(e[0])
        chans.add(j)
        if j in (10,):
            continue
        if j in (15, 16):
            # (16): ejected electron gets 1/10 of the primary energy; (17): E_rel
            assert e[11] == pytest.approx((0.1 if j == 15 else 1.0) * e[12], rel=1e-5 if prec == "fp32" else 1e-12)
            continue
        pb, pa = e[4:7], e[7:10]
        assert np.max(np.abs(pa - pb)) <= tol * np.max(np.abs(pb)) + 1e-40
        dE = e[2] - e[3] - e[10] * QE
        assert abs(dE) <= 4 * tol * e[2] + 1e-30, (j, dE, e[2])
    assert {0, 1, 6, 11, 13, 14, 18} <= chans


def test_births_get_consecutive_canonical_ids():
    sig, thr, loss = build_tables(partner_boost=PARTNER_BOOST)
    o = O.Oracle(small(), sig, thr, loss, precision="fp32")
    n0 = sum(small().n_init)
    o.step(100)
    ids = np.concatenate([o.particles(s)[0] for s in range(3)])
    ev, ab, misc = o.counters()
    assert len(np.unique(ids)) == len(ids)
    assert misc["next_id"] == n0 + misc["births"]
    assert ids.max() < misc["next_id"]


def test_fp32_and_fp64_agree_statistically():
    """The two precisions follow the same random streams; after one rf cycle
    their macroscopic state differs only at the level of statistical noise."""
    sig, thr, loss = build_tables()
    res = []
    for prec in ("fp32", "fp64"):
        o = O.Oracle(small(), sig, thr, loss, precision=prec)
        o.step(1000)
        res.append(([o.alive(s) for s in range(3)], o.cycle_sums()[0]))
    for s in range(3):
        assert res[0][0][s] == pytest.approx(res[1][0][s], rel=0.03)
    q32, q64 = res[0][1].astype(float), res[1][1].astype(float)
    assert np.abs(q32 - q64).sum() / q64.sum() < 0.05


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_sampler_elementary_functions_against_numpy(prec):
    """sin/cos(2 pi u) and ln(u) of the samplers (series with fixed term
    counts) against numpy in double, on the uniforms the generator produces
    and on the quadrant edges."""
    rng = np.random.default_rng(7)
    w = rng.integers(0, 2**32, 200000, dtype=np.uint64)
    if prec == "fp32":
        u = ((w >> 9).astype(np.float64) + 0.5) * 2.0**-23
        edges = np.array([0.5, 1, 2, 1023, 1024, 2047, 2048, 4095, 4096, 6143, 6144, 8191]) * 2.0**-13
        u = np.concatenate([u, edges, [2.0**-24, 1 - 2.0**-24]])
        tol_trig, tol_log = 3e-7, 3e-7
    else:
        u = (w.astype(np.float64) + 0.5) * 2.0**-32
        u = np.concatenate([u, [0.125, 0.25, 0.375, 0.5, 0.625, 0.75, 0.875, 2.0**-33, 1 - 2.0**-33]])
        # numpy's own argument 2*pi*u is rounded: about 4 ulp of 2 pi
        tol_trig, tol_log = 1.5e-15, 6e-16
    sn, cs, lg = O.math(u, prec)
    assert np.max(np.abs(sn - np.sin(2 * np.pi * u))) < tol_trig
    assert np.max(np.abs(cs - np.cos(2 * np.pi * u))) < tol_trig
    assert np.max(np.abs(lg - np.log(u)) / np.maximum(1.0, np.abs(np.log(u)))) < tol_log
    # exact values where the quadrant reduction lands on a node
    s0, c0, l1 = O.math(np.array([0.25, 0.5, 0.75]), prec)
    assert np.allclose(s0, [1, 0, -1], atol=tol_trig) and np.allclose(c0, [0, -1, 0], atol=tol_trig)


# ----------------------------------------------------------------------------
# partner reactions (13), (19), (14): Eq. (1) with the real density
# n_t = W N_t(c) / (A dx) of the partner species in the test particle's cell
# ----------------------------------------------------------------------------
PAIRS = {12: (0, 2), 13: (0, 1), 17: (1, 2)}   # channel: (test species, partner species)


@pytest.mark.parametrize("ramp", [False, True])
@pytest.mark.parametrize("j", [12, 13, 17])
def test_partner_rates_follow_eq1_with_weight(j, ramp):
    """One step of Maxwellian loads of the test and partner species, the
    self field switched off so that a realistic weight W ~ 1e10 can be used,
    no gas.  The partner channel's cross section is a / sqrt(E) (sigma g = K
    constant, above the channel's threshold), or that times min(1, E/E1),
    which makes the thinning by sigma(g) g / M_j reject a good share.
    Accepted requests per test particle are Poisson with mean
    tau W N_t(c) / (A dx) <sigma_j g>; a partner taken by several accepted
    requests goes to one of them, which removes (A_c^2 + A_c)/(2 n_c) of the
    A_c accepted requests of a cell with n_c partners on average."""
    s, t = PAIRS[j]
    n = [0, 0, 0]
    n[s], n[t] = 100_000, 40_000
    T = (3.0, 0.8, 0.3)
    base = small(n_init=tuple(n), T_init_eV=T, n_cells=4, pressure_Pa=0.0, voltage_V=0.0,
                 coulomb_every=0)
    sig, thr, loss = build_tables()
    sig[:] = 0.0
    E = energy_grid()
    mu = MASS[s] * MASS[t] / (MASS[s] + MASS[t])
    kT = mu * (T[s] / MASS[s] + T[t] / MASS[t])       # eV: relative energy is Maxwellian at kT
    a = 1e-19
    sig[j] = a / np.sqrt(E)
    if ramp:
        sig[j] *= np.minimum(1.0, E / kT)
    sig[j, E < thr[j]] = 0.0
    K = a * math.sqrt(2 * QE / mu)
    kmean = _maxwell_rate(sig[j], thr[j], mu, kT)
    if not ramp:
        from scipy.special import gammaincc
        assert kmean == pytest.approx(K * gammaincc(1.5, thr[j] / kT), rel=1e-6)
    dt = 1.0 / (base.frequency_Hz * base.steps_per_period)
    dx = base.gap_m / base.n_cells
    # free flight of the test particles for one step: their cells when they collide
    probe = O.Oracle(dataclasses.replace(base, weight=1.0), sig, thr, loss, precision="fp64", field_off=True)
    ids_s, c_s, f_s, v_s = probe.particles(s)
    _, c_t, _, _ = probe.particles(t)
    probe.close()
    x1 = (c_s + f_s) * dx + v_s[:, 0] * dt
    c1 = np.floor(x1 / dx).astype(np.int64)
    c1 = c1[(c1 >= 0) & (c1 < base.n_cells)]
    n_t = np.bincount(c_t, minlength=base.n_cells).astype(float)
    n_s = np.bincount(c1, minlength=base.n_cells).astype(float)
    # W for about 1000 accepted requests
    W = 1000.0 * base.area_m2 * dx / (dt * kmean * float(np.sum(n_s * n_t)))
    wl = dataclasses.replace(base, weight=W)
    o = O.Oracle(wl, sig, thr, loss, precision="fp64", field_off=True)
    assert o.constants()["pmax_e" if s == 0 else "pmax_n"] < 0.1
    o.step(1)
    ev, ab, misc = o.counters()
    lam_c = n_s * n_t * dt * W * kmean / (base.area_m2 * dx)
    lam = float(np.sum(lam_c - (lam_c ** 2 + lam_c) / (2.0 * n_t)))
    assert 800 < lam < 1100
    assert abs(ev[j] - lam) < 4.5 * math.sqrt(lam), (j, ramp, ev[j], lam)
    others = [k for k in range(19) if k != j]
    assert not ev[others].any()
    # without the weight in the partner density the rate would be W times lower
    assert W > 1e8


# ----------------------------------------------------------------------------
# ion channels: direct detachment (16) and charge exchange (6) against
# Maxwellian integrals of the tables, Eq. (1) and (3)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("sp,chans,T_eV", [(1, (14, 15), 3.0), (1, (14, 15), 8.0), (2, (18,), 0.026),
                                           (2, (18,), 1.0)])
def test_ion_channel_rates_fp64(sp, chans, T_eV):
    """Fresh Maxwellian ion load, no field, one step: events of O- elastic (5),
    direct detachment (16) and O2+ charge exchange (6) (its half momentum
    transfer value and the bridge of Eq. (3)) are binomial with mean
    N tau n_gas <sigma_j g>, the average over the relative energy, Maxwellian
    with kT_eff = mu (kT_s/m_s + kT_g/M)."""
    n = [0, 0, 0]
    n[sp] = 300_000
    T = [3.0, 0.026, 0.026]
    T[sp] = T_eV
    wl = quiet(small(n_init=tuple(n), T_init_eV=tuple(T), pressure_Pa=100.0), weight=1e-30)
    sig, thr, loss = tables_only(chans)
    dt = 1.0 / (wl.frequency_Hz * wl.steps_per_period)
    ngas = wl.pressure_Pa / (KB * wl.T_gas_K)
    mu = MASS[sp] * MO2 / (MASS[sp] + MO2)
    kT = mu * (T_eV * QE / MASS[sp] + KB * wl.T_gas_K / MO2) / QE
    # scale a channel up where its rate would give fewer than ~300 events
    for j in chans:
        lam = n[sp] * dt * ngas * _maxwell_rate(sig[j], thr[j], mu, kT)
        if lam < 300:
            sig[j] *= math.ceil(300 / lam)
    o = O.Oracle(wl, sig, thr, loss, precision="fp64")
    assert o.constants()["pmax_n" if sp == 1 else "pmax_p"] < 1.0
    o.step(1)
    ev, ab, misc = o.counters()
    n_mcc = misc["psteps"] - ab[:, sp].sum()
    checked = 0
    for j in chans:
        lam = n_mcc * dt * ngas * _maxwell_rate(sig[j], thr[j], mu, kT)
        if lam < 30:
            assert ev[j] < lam + 6 * math.sqrt(lam) + 6, (j, ev[j], lam)
            continue
        assert abs(ev[j] - lam) < 4.5 * math.sqrt(lam), (j, ev[j], lam)
        checked += 1
    assert checked == len(chans)
    assert not ev[[k for k in range(19) if k not in chans]].any()
