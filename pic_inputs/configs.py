"""Discharge workloads (synthetic, seeded).

The physical set-up follows Sec. II of the paper: a planar 1d3v gap of width L,
one electrode driven by U(t) = U_rf sin(2 pi f t), the other grounded, both
perfectly absorbing, O2 reservoir at pressure p and temperature T.

Normalisation (Sec. II): the lateral area is A = lambda_De^2 of a reference
electron system (n_res, T_res).  The paper quotes n_res ~ 1e8-1e9 cm^-3 and
k T_res ~ 10 eV; we take n_res = 1e9 cm^-3 and T_res = 10 eV, and give every
species the same macro weight W = n_res * A * L / N_e(0), so that the initial
electron load represents n_res.

The three named workloads are the single-discharge cases used for parity and
measurement:
  small  -- 4 cm, 128 cells, 10 Pa, 100 V, dt = T_rf/1000, 10k e + 2k O- + 10k O2+
  prod   -- 4 cm, 1024 cells, 50 Pa, 200 V, dt = T_rf/4000, ions sub-cycled x10,
            2M e + 0.5M O- + 2M O2+
  large  -- 6 cm, 4096 cells, 100 Pa, 400 V, dt = T_rf/8000,
            2^25 macro-particles, charge-neutral split 40 % e, 10 % O-, 50 % O2+
All use 13.56 MHz, a uniform initial load with Maxwellian velocities
(electrons 3 eV, ions 0.026 eV), C = 1/6 for associative detachment, and
intra-species Coulomb collisions (ln Lambda = 10) at every cell sort.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

EPS0 = 8.8541878128e-12
QE = 1.602176634e-19

N_RES = 1.0e15          # m^-3  (1e9 cm^-3)
T_RES_EV = 10.0


def debye_area(n_res=N_RES, t_res_ev=T_RES_EV):
    """A = lambda_De^2 = eps0 k T_res / (e^2 n_res)."""
    return EPS0 * t_res_ev / (QE * n_res)


@dataclass(frozen=True)
class Workload:
    name: str
    gap_m: float
    n_cells: int
    pressure_Pa: float
    voltage_V: float
    frequency_Hz: float
    steps_per_period: int
    ion_subcycle: int
    n_init: tuple            # (electrons, O-, O2+)
    T_init_eV: tuple = (3.0, 0.026, 0.026)
    T_gas_K: float = 300.0
    metastable_frac: float = 1.0 / 6.0
    sort_every: int = 10
    coulomb_every: int = 0       # intra-species Coulomb collisions every n2 steps (0: off)
    coulomb_log: float = 10.0
    coulomb_inter: bool = False  # inter-species Coulomb collisions as well
    dsmc: bool = False           # collisions (4)-(19) as the per-cell list of Sec. II every sort_every steps
    seed: int = 705049500
    area_m2: float = field(default_factory=debye_area)
    weight: float = 0.0      # 0 -> n_res * A * L / N_e(0)

    def resolved(self) -> "Workload":
        w = self.weight
        if w == 0.0:
            w = N_RES * self.area_m2 * self.gap_m / float(self.n_init[0])
        return replace(self, weight=w)

    def scaled(self, factor: float, name: str | None = None) -> "Workload":
        """Same discharge with every initial population scaled by ``factor``;
        the weight is rescaled so the represented densities stay the same."""
        base = self.resolved()
        n = tuple(max(1, int(round(x * factor))) for x in base.n_init)
        w = base.weight * base.n_init[0] / n[0]
        return replace(base, n_init=n, weight=w, name=name or f"{base.name}/x{factor:g}")


WORKLOADS = {
    "small": Workload("small", 0.04, 128, 10.0, 100.0, 13.56e6, 1000, 1,
                      (10_000, 2_000, 10_000), sort_every=10, coulomb_every=10, seed=705049501),
    "prod": Workload("prod", 0.04, 1024, 50.0, 200.0, 13.56e6, 4000, 10,
                     (2_000_000, 500_000, 2_000_000), sort_every=100, coulomb_every=100, seed=705049502),
    # 2^25 particles split so that the load is charge neutral (O2+ = e + O-):
    # 40 % e, 10 % O-, 50 % O2+.  Assigning the 50 % to electrons instead leaves
    # 20 % of the negative charge uncompensated (~3 kV of space-charge potential
    # at t = 0), which at 100 Pa starts an ionisation avalanche that multiplies
    # the electron count about tenfold within the first rf cycle.
    "large": Workload("large", 0.06, 4096, 100.0, 400.0, 13.56e6, 8000, 1,
                      (13_421_773, 3_355_443, 16_777_216), sort_every=10, coulomb_every=10,
                      seed=705049503),
    # the small discharge with the collisions (4)-(19) as the per-cell list
    # every 10 steps
    "small_list": Workload("small_list", 0.04, 128, 10.0, 100.0, 13.56e6, 1000, 1,
                           (10_000, 2_000, 10_000), sort_every=10, coulomb_every=10, seed=705049501,
                           dsmc=True),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name].resolved()


def sweep(count: int = 64, seed: int = 705049504) -> list:
    """The batched parameter sweep: independent discharges with
    U ~ U[50, 400] V, p ~ logU[5, 100] Pa, L ~ U[2, 6] cm,
    N_c in {256, 512, 1024, 2048}, N ~ logU[1e5, 4e6] macro particles,
    dt = T_rf / 4000, 13.56 MHz, sort and Coulomb every 10 steps.  Each
    population is split charge neutrally as in the large discharge (40 % e,
    10 % O-, 50 % O2+) and the weight makes the initial electron density
    n_res.  Seeded: the same call gives the same discharges."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        U = float(rng.uniform(50.0, 400.0))
        p = float(np.exp(rng.uniform(np.log(5.0), np.log(100.0))))
        L = float(rng.uniform(0.02, 0.06))
        nc = int(rng.choice([256, 512, 1024, 2048]))
        n = float(np.exp(rng.uniform(np.log(1e5), np.log(4e6))))
        ne, nn = int(round(0.4 * n)), int(round(0.1 * n))
        wl = Workload(f"sweep{i}", L, nc, p, U, 13.56e6, 4000, 1, (ne, nn, ne + nn),
                      sort_every=10, coulomb_every=10, seed=seed + 1 + i)
        out.append(wl.resolved())
    return out


def served_stream(count: int = 32, seed: int = 705049700) -> list:
    """Requests of the served stream: small discharges that reach the
    periodic steady state within about a hundred rf cycles -- 4 cm, 128
    cells, 13.56 MHz, dt = T_rf/1000, the small discharge's load (10k e, 2k
    O-, 10k O2+), with U ~ U[300, 400] V and p ~ U[15, 25] Pa, sort and
    Coulomb every 10 steps.  (The batched sweep's discharges need of the order
    of 10^3 rf cycles of 4000 steps each, minutes to hours per request, so a
    stream of them cannot be run to steady state here.)  Seeded."""
    import numpy as np
    rng = np.random.default_rng(seed)
    base = WORKLOADS["small"]
    out = []
    for i in range(count):
        U = float(rng.uniform(300.0, 400.0))
        p = float(rng.uniform(15.0, 25.0))
        out.append(replace(base, name=f"served{i}", voltage_V=U, pressure_Pa=p, seed=seed + 1 + i).resolved())
    return out
