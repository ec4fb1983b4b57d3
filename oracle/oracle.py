"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module.  The product library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pic_oracle.c")
LIBS = {"fp32": os.path.join(HERE, "liboracle32.so"), "fp64": os.path.join(HERE, "liboracle64.so")}
CFLAGS = ["-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wno-unused-function"]

NCH, NPT = 19, 897


def build(verbose: bool = False) -> None:
    """Compile both precisions of the oracle with gcc."""
    for prec, out in LIBS.items():
        cmd = ["gcc", *CFLAGS, SRC, "-o", out, "-lm"]
        if prec == "fp64":
            cmd.insert(1, "-DORACLE_FP64")
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)


class Params(C.Structure):
    _fields_ = [
        ("gap_m", C.c_double), ("n_cells", C.c_int32), ("area_m2", C.c_double), ("weight", C.c_double),
        ("steps_per_period", C.c_int32), ("ion_subcycle", C.c_int32), ("sort_every", C.c_int32),
        ("drive_dc", C.c_int32), ("n_init", C.c_int64 * 3), ("T_init_eV", C.c_double * 3),
        ("seed", C.c_uint64), ("voltage_V", C.c_double), ("frequency_Hz", C.c_double),
        ("pressure_Pa", C.c_double), ("T_gas_K", C.c_double), ("metastable_frac", C.c_double),
        ("eedf_bins", C.c_int32), ("eedf_emax_eV", C.c_double), ("fneg_xbins", C.c_int32),
        ("fneg_ebins", C.c_int32), ("fneg_emax_eV", C.c_double), ("coulomb_every", C.c_int32),
        ("coulomb_log", C.c_double), ("coulomb_inter", C.c_int32), ("field_off", C.c_int32),
        ("dsmc", C.c_int32),
    ]


_loaded = {}


def lib(prec: str = "fp32"):
    if prec in _loaded:
        return _loaded[prec]
    path = LIBS[prec]
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
        build()
    L = C.CDLL(path)
    P = C.POINTER
    L.or_create.restype = C.c_void_p
    L.or_create.argtypes = [P(Params), P(C.c_double), P(C.c_double), P(C.c_double), P(C.c_int)]
    L.or_destroy.argtypes = [C.c_void_p]
    L.or_step.argtypes = [C.c_void_p, C.c_int64]
    L.or_alive.restype = C.c_int64
    L.or_alive.argtypes = [C.c_void_p, C.c_int]
    L.or_particles.restype = C.c_int64
    L.or_particles.argtypes = [C.c_void_p, C.c_int, C.c_int64, P(C.c_uint64), P(C.c_int32), P(C.c_double),
                               P(C.c_double)]
    L.or_field.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
    L.or_charge.argtypes = [C.c_void_p, P(C.c_int64)]
    L.or_counters.argtypes = [C.c_void_p, P(C.c_int64), P(C.c_int64), P(C.c_int64)]
    L.or_cycle_sums.argtypes = [C.c_void_p, P(C.c_int64), P(C.c_double), P(C.c_int64), P(C.c_int64)]
    L.or_constants.argtypes = [C.c_void_p, P(C.c_double)]
    L.or_philox.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
    L.or_sigma.restype = C.c_double
    L.or_sigma.argtypes = [C.c_void_p, C.c_int, C.c_double]
    L.or_solve_field.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double, P(C.c_int64),
                                 P(C.c_double), P(C.c_double)]
    L.or_log_enable.argtypes = [C.c_void_p, C.c_int64]
    L.or_scale_velocities.argtypes = [C.c_void_p, C.c_int, P(C.c_double)]
    L.or_math.argtypes = [P(C.c_double), C.c_int64, P(C.c_double), P(C.c_double), P(C.c_double)]
    L.or_load.restype = C.c_int
    L.or_load.argtypes = [C.c_void_p, P(C.c_int64), P(C.c_int32), P(C.c_double), P(C.c_double)]
    L.or_log_read.restype = C.c_int64
    L.or_log_read.argtypes = [C.c_void_p, P(C.c_double), C.c_int64]
    _loaded[prec] = L
    return L


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def philox(ctr, key, prec="fp32"):
    L = lib(prec)
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    L.or_philox(c, k, o)
    return list(o)


def math(u, prec="fp32"):
    """The sampler's sin(2 pi u), cos(2 pi u) and ln(u) of the oracle."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    sn, cs, lg = np.zeros_like(u), np.zeros_like(u), np.zeros_like(u)
    lib(prec).or_math(_ptr(u, C.c_double), len(u), _ptr(sn, C.c_double), _ptr(cs, C.c_double), _ptr(lg, C.c_double))
    return sn, cs, lg


def solve_field(q, dx, cphi, cE, U0, prec="fp64"):
    q = np.ascontiguousarray(q, dtype=np.int64)
    N = len(q) - 1
    phi = np.zeros(N + 1)
    E = np.zeros(N + 1)
    lib(prec).or_solve_field(N, dx, cphi, cE, U0, _ptr(q, C.c_int64), _ptr(phi, C.c_double), _ptr(E, C.c_double))
    return phi, E


class Oracle:
    """One discharge advanced by the CPU oracle."""

    def __init__(self, wl, sigma, threshold, loss, precision="fp32", drive_dc=False,
                 eedf_bins=128, eedf_emax_eV=64.0, fneg_xbins=32, fneg_ebins=64, fneg_emax_eV=8.0,
                 coulomb_every=None, field_off=False):
        self.L = lib(precision)
        self.wl = wl
        p = Params()
        p.gap_m = wl.gap_m
        p.n_cells = wl.n_cells
        p.area_m2 = wl.area_m2
        p.weight = wl.weight
        p.steps_per_period = wl.steps_per_period
        p.ion_subcycle = wl.ion_subcycle
        p.sort_every = wl.sort_every
        p.drive_dc = 1 if drive_dc else 0
        for s in range(3):
            p.n_init[s] = int(wl.n_init[s])
            p.T_init_eV[s] = float(wl.T_init_eV[s])
        p.seed = wl.seed
        p.voltage_V = wl.voltage_V
        p.frequency_Hz = wl.frequency_Hz
        p.pressure_Pa = wl.pressure_Pa
        p.T_gas_K = wl.T_gas_K
        p.metastable_frac = wl.metastable_frac
        p.eedf_bins = eedf_bins
        p.eedf_emax_eV = eedf_emax_eV
        p.fneg_xbins = fneg_xbins
        p.fneg_ebins = fneg_ebins
        p.fneg_emax_eV = fneg_emax_eV
        p.coulomb_every = wl.coulomb_every if coulomb_every is None else coulomb_every
        p.coulomb_log = wl.coulomb_log
        p.coulomb_inter = 1 if getattr(wl, "coulomb_inter", False) else 0
        p.field_off = 1 if field_off else 0
        p.dsmc = 1 if getattr(wl, "dsmc", False) else 0
        self.params = p
        self.eedf_bins = eedf_bins
        self.nf = fneg_xbins * fneg_ebins
        sig = np.ascontiguousarray(sigma, dtype=np.float64)
        thr = np.ascontiguousarray(threshold, dtype=np.float64)
        los = np.ascontiguousarray(loss, dtype=np.float64)
        err = C.c_int(0)
        self.h = self.L.or_create(C.byref(p), _ptr(sig, C.c_double), _ptr(thr, C.c_double), _ptr(los, C.c_double),
                                  C.byref(err))
        if not self.h:
            raise RuntimeError(f"or_create failed: {err.value}")
        self.N = wl.n_cells

    def close(self):
        if self.h:
            self.L.or_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        rc = self.L.or_step(self.h, n)
        if rc != 0:
            raise RuntimeError(f"or_step failed: {rc}")

    def alive(self, sp):
        return self.L.or_alive(self.h, sp)

    def particles(self, sp):
        n = self.alive(sp)
        ids = np.zeros(n, np.uint64)
        cell = np.zeros(n, np.int32)
        off = np.zeros(n)
        v = np.zeros((n, 3))
        self.L.or_particles(self.h, sp, n, _ptr(ids, C.c_uint64), _ptr(cell, C.c_int32), _ptr(off, C.c_double),
                            _ptr(v, C.c_double))
        return ids, cell, off, v

    def field(self):
        phi = np.zeros(self.N + 1)
        E = np.zeros(self.N + 1)
        self.L.or_field(self.h, _ptr(phi, C.c_double), _ptr(E, C.c_double))
        return phi, E

    def charge(self):
        Q = np.zeros((3, self.N + 1), np.int64)
        self.L.or_charge(self.h, _ptr(Q, C.c_int64))
        return Q

    def counters(self):
        ev = np.zeros(19, np.int64)
        ab = np.zeros((2, 3), np.int64)
        misc = np.zeros(8, np.int64)
        self.L.or_counters(self.h, _ptr(ev, C.c_int64), _ptr(ab, C.c_int64), _ptr(misc, C.c_int64))
        keys = ["psteps", "births", "next_id", "step", "cycles", "tophits", "requests", "accepted"]
        return ev, ab, dict(zip(keys, (int(x) for x in misc)))

    def cycle_sums(self):
        Q = np.zeros((3, self.N + 1), np.int64)
        phi = np.zeros(self.N + 1)
        eedf = np.zeros(self.eedf_bins + 1, np.int64)
        fneg = np.zeros(self.nf, np.int64)
        self.L.or_cycle_sums(self.h, _ptr(Q, C.c_int64), _ptr(phi, C.c_double), _ptr(eedf, C.c_int64),
                             _ptr(fneg, C.c_int64))
        return Q, phi, eedf, fneg

    def constants(self):
        o = np.zeros(16)
        self.L.or_constants(self.h, _ptr(o, C.c_double))
        keys = ["pmax_e", "pmax_n", "pmax_p", "Mgas_e", "Mgas_n", "Mgas_p", "Mad", "M13", "M19", "M14",
                "dx", "dt", "ngas", "cphi", "cE", "segmax_p"]
        return dict(zip(keys, o))

    def sigma(self, chan, E):
        return self.L.or_sigma(self.h, chan, E)

    def scale_velocities(self, sp, f):
        a = np.ascontiguousarray(f, dtype=np.float64)
        self.L.or_scale_velocities(self.h, sp, _ptr(a, C.c_double))

    def load(self, parts):
        """Replace the initial load (test hook, before the first step): parts is
        a list of three (cell, off, v) arrays, species e, O-, O2+."""
        n = np.array([len(p[0]) for p in parts], np.int64)
        cell = np.ascontiguousarray(np.concatenate([p[0] for p in parts]), dtype=np.int32)
        off = np.ascontiguousarray(np.concatenate([p[1] for p in parts]), dtype=np.float64)
        v = np.ascontiguousarray(np.concatenate([np.reshape(p[2], (-1, 3)) for p in parts]), dtype=np.float64)
        rc = self.L.or_load(self.h, _ptr(n, C.c_int64), _ptr(cell, C.c_int32), _ptr(off, C.c_double),
                            _ptr(v, C.c_double))
        if rc != 0:
            raise RuntimeError(f"or_load failed: {rc}")

    def log_enable(self, cap):
        self.L.or_log_enable(self.h, cap)

    def log(self, cap=1 << 20):
        out = np.zeros((cap, 16))
        n = self.L.or_log_read(self.h, _ptr(out, C.c_double), cap)
        return out[: min(n, cap)]
