"""Cross-section tables for the 19-reaction oxygen set (Table I of the paper).

Grid.  Every channel is tabulated on the same energy grid

    E_k = 2**(-14 + k // 32) * (1 + (k % 32) / 32)  eV,   k = 0 .. 896,

i.e. 32 points per binade from 2**-14 eV (6.1e-5 eV) to 2**14 eV (16384 eV).
Both implementations interpolate linearly in E between neighbouring nodes; the
grid is chosen so that the node index and the interpolation weight follow
exactly from the bit pattern of an IEEE energy value.  Below the first node the
first value is used, above the last node the last value (the paper extrapolates
measured data as a constant beyond the largest tabulated energy, Sec. III).

Data.  Only four channels have closed forms in the paper:
  (5)  O- + O2 elastic, polarisation model, Eq. (4), n = 3, C = 3.77e-24,
       sigma_0 = 1.2e-15 cm^2;
  (14) O- + O2+ neutralisation, Landau-Zener fit, Eq. (8);
  (17) O- + O2(a) associative detachment, Langevin model, Eq. (9);
  (13) dissociative recombination = B * sigma_0(E) with B = 3, Eq. (6), but
       sigma_0 (the non-resonant cross section) is not printed.
All other channels are measured data the paper shows only as figures.  Those
figures are not available, so this module uses *synthetic stand-ins*: smooth
shapes of realistic order of magnitude with the thresholds the paper states
(6.4 eV and 8.6 eV dissociation, ~1.3 eV direct detachment, attachment zero
below ~4 eV) and textbook values elsewhere.  They are not any dataset's values.

Thresholds and energy losses.  ``threshold_eV[j]`` is the energy below which a
channel is closed; ``loss_eV[j]`` is the excitation energy dE of the inelastic
binary collision, Eq. (5).  Values not given in the paper (vibrational quanta,
Rydberg, metastable, ionisation and O- detachment energies) are builder
choices and are listed as such in the design notes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

N_POINTS = 897          # 28 binades x 32 + closing node at 2**14 eV
E_MIN_EXP = -14
CM2 = 1.0e-4            # cm^2 -> m^2

# species indices used throughout: 0 = electron, 1 = O-, 2 = O2+, -1 = O2 gas
E, NEG, POS, GAS = 0, 1, 2, -1


@dataclass(frozen=True)
class Channel:
    index: int
    reaction: int        # number in Table I
    name: str
    test: int            # species of the test particle
    target: int          # GAS or a simulated species (partner channel)
    threshold_eV: float
    loss_eV: float


CHANNELS = (
    Channel(0, 4, "e+O2 elastic", E, GAS, 0.0, 0.0),
    Channel(1, 7, "e+O2 vib v=1", E, GAS, 0.193, 0.193),
    Channel(2, 7, "e+O2 vib v=2", E, GAS, 0.386, 0.386),
    Channel(3, 7, "e+O2 vib v=3", E, GAS, 0.579, 0.579),
    Channel(4, 7, "e+O2 vib v=4", E, GAS, 0.772, 0.772),
    Channel(5, 8, "e+O2 Rydberg", E, GAS, 9.97, 9.97),
    Channel(6, 9, "e+O2 dissociation 6.4 eV", E, GAS, 6.4, 6.4),
    Channel(7, 10, "e+O2 dissociation 8.6 eV", E, GAS, 8.6, 8.6),
    Channel(8, 11, "e+O2 a1Delta_g", E, GAS, 0.977, 0.977),
    Channel(9, 12, "e+O2 b1Sigma_g", E, GAS, 1.627, 1.627),
    Channel(10, 15, "e+O2 dissociative attachment", E, GAS, 4.2, 0.0),
    Channel(11, 18, "e+O2 impact ionisation", E, GAS, 12.06, 12.06),
    Channel(12, 13, "e+O2+ dissociative recombination", E, POS, 0.0, 0.0),
    Channel(13, 19, "e+O- impact detachment", E, NEG, 1.46, 1.46),
    Channel(14, 5, "O-+O2 elastic", NEG, GAS, 0.0, 0.0),
    Channel(15, 16, "O-+O2 direct detachment", NEG, GAS, 1.3, 0.0),
    Channel(16, 17, "O-+O2(a) associative detachment", NEG, GAS, 0.0, 0.0),
    Channel(17, 14, "O-+O2+ neutralisation", NEG, POS, 0.0, 0.0),
    Channel(18, 6, "O2+ + O2 charge exchange", POS, GAS, 0.0, 0.0),
)
N_CHANNELS = len(CHANNELS)


def energy_grid() -> np.ndarray:
    """Node energies E_k in eV (exact binary fractions)."""
    k = np.arange(N_POINTS)
    e = E_MIN_EXP + k // 32
    m = k % 32
    return np.ldexp(1.0 + m / 32.0, e)


# --- closed forms printed in the paper ------------------------------------

def sigma_okada(E):
    """Eq. (4): [n pi/(n-2) ((n-2)/2 * C/E)^(2/n) + sigma_0] cm^2, n = 3."""
    n, C, s0 = 3.0, 3.77e-24, 1.2e-15
    return (n * math.pi / (n - 2.0) * ((n - 2.0) / 2.0 * C / E) ** (2.0 / n) + s0) * CM2


def sigma_neutralisation(E):
    """Eq. (8): 0.8 (1 + 2.85/E[eV]) 1e-14 cm^2."""
    return 0.8 * (1.0 + 2.85 / E) * 1.0e-14 * CM2


def sigma_assoc_detachment(E):
    """Eq. (9): 5.96e-16 / sqrt(E[eV]) cm^2."""
    return 5.96e-16 / np.sqrt(E) * CM2


# --- synthetic stand-ins (documented shapes, not datasets) -----------------

def _rise_fall(E, thr, e_pk, s_pk):
    """0 below thr, linear rise to s_pk at e_pk, then s_pk * e_pk / E."""
    E = np.asarray(E, dtype=float)
    out = np.where(E < e_pk, s_pk * (E - thr) / (e_pk - thr), s_pk * e_pk / E)
    return np.where(E < thr, 0.0, out)


def _triangle(E, thr, e_pk, e_end, s_pk):
    E = np.asarray(E, dtype=float)
    up = s_pk * (E - thr) / (e_pk - thr)
    down = s_pk * (e_end - E) / (e_end - e_pk)
    out = np.where(E < e_pk, up, down)
    return np.where((E < thr) | (E > e_end), 0.0, out)


def _sigma_e_elastic(E):
    E = np.asarray(E, dtype=float)
    x = E / 20.0
    return 3.5e-20 * (1.0 + 1.5 * x / (1.0 + x * x)) / (1.0 + E / 200.0)


def _sigma_dr0(E):
    """Stand-in for the non-resonant recombination cross section sigma_0(E)."""
    return 2.0e-20 / np.asarray(E, dtype=float)


def _sigma_direct_detachment(E):
    E = np.asarray(E, dtype=float)
    r = np.clip(1.0 - 1.3 / E, 0.0, None)
    return np.where(E < 1.3, 0.0, 3.5e-20 * r ** 1.5)


def _sigma_momentum_o2p(E):
    return 4.0e-19 * (1.0 + 0.5 / np.sqrt(np.asarray(E, dtype=float)))


def _sigma_charge_exchange(E):
    """Eq. (3) construction: 1/2 sigma_m below 0.251 eV and above 8.5 eV,
    linear in E in between."""
    E = np.asarray(E, dtype=float)
    lo, hi = 0.251, 8.5
    half = 0.5 * _sigma_momentum_o2p(E)
    s_lo, s_hi = 0.5 * _sigma_momentum_o2p(lo), 0.5 * _sigma_momentum_o2p(hi)
    mid = s_lo + (s_hi - s_lo) * (E - lo) / (hi - lo)
    return np.where((E > lo) & (E < hi), mid, half)


def build_tables(dr_scale_B: float = 3.0, partner_boost: float = 1.0):
    """Return (sigma [N_CHANNELS, N_POINTS] in m^2, threshold_eV, loss_eV).

    ``partner_boost`` multiplies the three partner channels (13), (14), (19);
    tests use it to exercise pairing and claims at small particle numbers.
    """
    Ek = energy_grid()
    sig = np.zeros((N_CHANNELS, N_POINTS))
    sig[0] = _sigma_e_elastic(Ek)
    for v in range(1, 5):
        thr = 0.193 * v
        sig[v] = _rise_fall(Ek, thr, thr + 0.6, 1.2e-21 / v)
    sig[5] = _rise_fall(Ek, 9.97, 20.0, 5.0e-22)
    sig[6] = _rise_fall(Ek, 6.4, 15.0, 8.0e-21)
    sig[7] = _rise_fall(Ek, 8.6, 20.0, 6.0e-21)
    sig[8] = _rise_fall(Ek, 0.977, 2.5, 1.0e-22)
    sig[9] = _rise_fall(Ek, 1.627, 4.0, 2.0e-23)
    sig[10] = _triangle(Ek, 4.2, 6.5, 10.0, 1.4e-22)
    sig[11] = _rise_fall(Ek, 12.06, 110.0, 2.7e-20)
    sig[12] = dr_scale_B * _sigma_dr0(Ek)
    sig[13] = _rise_fall(Ek, 1.46, 20.0, 5.0e-20)
    sig[14] = np.array([sigma_okada(e) for e in Ek])
    sig[15] = _sigma_direct_detachment(Ek)
    sig[16] = sigma_assoc_detachment(Ek)
    sig[17] = np.array([sigma_neutralisation(e) for e in Ek])
    sig[18] = _sigma_charge_exchange(Ek)
    thr = np.array([c.threshold_eV for c in CHANNELS])
    loss = np.array([c.loss_eV for c in CHANNELS])
    # a channel is closed at every node strictly below its threshold
    for c in CHANNELS:
        sig[c.index, Ek < c.threshold_eV] = 0.0
    if partner_boost != 1.0:
        for j in (12, 13, 17):
            sig[j] *= partner_boost
    return np.ascontiguousarray(sig), thr, loss
