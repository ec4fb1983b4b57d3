"""ctypes binding of libpic.so (the C ABI declared in include/pic.h).

Argument marshalling only: every step of the particle path runs in the HIP
kernels of the library.  The binding raises if the library is missing; there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_FP32, PIC_FP64 = 0, 1
NCHAN, NPOINTS = 19, 897
ERRORS = {-1: "PIC_EINVAL", -2: "PIC_ENOMEM", -3: "PIC_EDEVICE", -4: "PIC_EGUARD", -5: "PIC_EOVERFLOW"}


class PicError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Geometry(C.Structure):
    _fields_ = [
        ("gap_m", C.c_double), ("n_cells", C.c_int32), ("area_m2", C.c_double), ("weight", C.c_double),
        ("steps_per_period", C.c_int32), ("ion_subcycle", C.c_int32), ("sort_every", C.c_int32),
        ("drive_dc", C.c_int32), ("n_init", C.c_int64 * 3), ("T_init_eV", C.c_double * 3), ("seed", C.c_uint64),
        ("precision", C.c_int32), ("capacity", C.c_int64 * 3), ("eedf_bins", C.c_int32),
        ("eedf_emax_eV", C.c_double), ("fneg_xbins", C.c_int32), ("fneg_ebins", C.c_int32),
        ("fneg_emax_eV", C.c_double), ("coulomb_every", C.c_int32),
    ]


class Gas(C.Structure):
    _fields_ = [
        ("T_gas_K", C.c_double), ("metastable_frac", C.c_double), ("sigma_m2", C.POINTER(C.c_double)),
        ("threshold_eV", C.POINTER(C.c_double)), ("loss_eV", C.POINTER(C.c_double)),
        ("coulomb_log", C.c_double), ("coulomb_inter", C.c_int32), ("dsmc", C.c_int32),
    ]


class Moments(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("cycles", C.c_int64), ("alive", C.c_int64 * 3), ("events", C.c_int64 * NCHAN),
        ("absorbed", (C.c_int64 * 3) * 2), ("particle_steps", C.c_int64), ("births", C.c_int64),
        ("next_id", C.c_int64), ("density_m3", C.POINTER(C.c_double)), ("phi_V", C.POINTER(C.c_double)),
        ("eedf", C.POINTER(C.c_int64)), ("fneg", C.POINTER(C.c_int64)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("PIC_LIBRARY", LIB_PATH)  # another build of the same C ABI
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    L = C.CDLL(path)
    P = C.POINTER
    L.pic_create.argtypes = [P(Geometry), P(Gas), C.c_double, C.c_double, C.c_double, P(C.c_void_p)]
    L.pic_set_stream.argtypes = [C.c_void_p, C.c_void_p]
    L.pic_step.argtypes = [C.c_void_p, C.c_int64]
    L.pic_sync.argtypes = [C.c_void_p]
    L.pic_moments.argtypes = [C.c_void_p, P(Moments)]
    L.pic_particles.argtypes = [C.c_void_p, C.c_int, C.c_int64, P(C.c_uint64), P(C.c_int32), P(C.c_double),
                                P(C.c_double), P(C.c_int64)]
    L.pic_field.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
    L.pic_charge.argtypes = [C.c_void_p, P(C.c_int64)]
    L.pic_timing.argtypes = [C.c_void_p, C.c_int]
    L.pic_kernel_time.argtypes = [C.c_void_p, P(C.c_double), P(C.c_int64)]
    L.pic_set_grid.argtypes = [C.c_void_p, C.c_int32]
    L.pic_set_graphs.argtypes = [C.c_void_p, C.c_int]
    L.pic_autotune.argtypes = [C.c_void_p, C.c_int64, P(C.c_int32)]
    L.pic_step_batch.argtypes = [P(C.c_void_p), C.c_int, C.c_int64]
    L.pic_step_batch_static.argtypes = [P(C.c_void_p), C.c_int, C.c_int64]
    L.pic_set_shape.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
    L.pic_launch_shape.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_int32), P(C.c_int32)]
    L.pic_autotune_batch.argtypes = [P(C.c_void_p), C.c_int, C.c_int64, P(C.c_int32), P(C.c_int32),
                                     P(C.c_int32)]
    L.pic_destroy.argtypes = [C.c_void_p]
    L.pic_last_error.argtypes = [C.c_void_p]
    L.pic_last_error.restype = C.c_char_p
    _lib = L
    return L


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class Discharge:
    """One rf discharge whose particle state lives in device memory."""

    def __init__(self, wl, sigma, threshold, loss, precision="fp32", drive_dc=False, capacity=None,
                 eedf_bins=128, eedf_emax_eV=64.0, fneg_xbins=32, fneg_ebins=64, fneg_emax_eV=8.0, stream=None):
        self.L = lib()
        g = Geometry()
        g.gap_m = wl.gap_m
        g.n_cells = wl.n_cells
        g.area_m2 = wl.area_m2
        g.weight = wl.weight
        g.steps_per_period = wl.steps_per_period
        g.ion_subcycle = wl.ion_subcycle
        g.sort_every = wl.sort_every
        g.drive_dc = 1 if drive_dc else 0
        for s in range(3):
            g.n_init[s] = int(wl.n_init[s])
            g.T_init_eV[s] = float(wl.T_init_eV[s])
            g.capacity[s] = int(capacity[s]) if capacity is not None else 0
        g.seed = wl.seed
        g.precision = PIC_FP64 if precision == "fp64" else PIC_FP32
        g.eedf_bins = eedf_bins
        g.eedf_emax_eV = eedf_emax_eV
        g.fneg_xbins = fneg_xbins
        g.fneg_ebins = fneg_ebins
        g.fneg_emax_eV = fneg_emax_eV
        g.coulomb_every = getattr(wl, "coulomb_every", 0)
        self._sig = np.ascontiguousarray(sigma, dtype=np.float64)
        self._thr = np.ascontiguousarray(threshold, dtype=np.float64)
        self._loss = np.ascontiguousarray(loss, dtype=np.float64)
        gas = Gas()
        gas.T_gas_K = wl.T_gas_K
        gas.metastable_frac = wl.metastable_frac
        gas.sigma_m2 = _p(self._sig, C.c_double)
        gas.threshold_eV = _p(self._thr, C.c_double)
        gas.loss_eV = _p(self._loss, C.c_double)
        gas.coulomb_log = getattr(wl, "coulomb_log", 0.0)
        gas.coulomb_inter = int(bool(getattr(wl, "coulomb_inter", False)))
        gas.dsmc = int(bool(getattr(wl, "dsmc", False)))
        self.h = C.c_void_p()
        rc = self.L.pic_create(C.byref(g), C.byref(gas), wl.voltage_V, wl.frequency_Hz, wl.pressure_Pa,
                               C.byref(self.h))
        if rc != 0:
            raise PicError(rc, "pic_create")
        self.wl = wl
        self.N = wl.n_cells
        self.eedf_bins = eedf_bins
        self.nf = fneg_xbins * fneg_ebins
        if stream is not None:
            self._check(self.L.pic_set_stream(self.h, C.c_void_p(stream)))

    def _check(self, rc):
        if rc != 0:
            msg = self.L.pic_last_error(self.h)
            raise PicError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            self.L.pic_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        self._check(self.L.pic_step(self.h, n))

    def sync(self):
        self._check(self.L.pic_sync(self.h))

    def particles(self, sp):
        n = C.c_int64(0)
        self._check(self.L.pic_particles(self.h, sp, 0, None, None, None, None, C.byref(n)))
        cap = n.value
        ids = np.zeros(cap, np.uint64)
        cell = np.zeros(cap, np.int32)
        off = np.zeros(cap)
        v = np.zeros((cap, 3))
        self._check(self.L.pic_particles(self.h, sp, cap, _p(ids, C.c_uint64), _p(cell, C.c_int32),
                                         _p(off, C.c_double), _p(v, C.c_double), C.byref(n)))
        return ids, cell, off, v

    def field(self):
        phi = np.zeros(self.N + 1)
        E = np.zeros(self.N + 1)
        self._check(self.L.pic_field(self.h, _p(phi, C.c_double), _p(E, C.c_double)))
        return phi, E

    def charge(self):
        Q = np.zeros((3, self.N + 1), np.int64)
        self._check(self.L.pic_charge(self.h, _p(Q, C.c_int64)))
        return Q

    def moments(self):
        m = Moments()
        dens = np.zeros((3, self.N + 1))
        phi = np.zeros(self.N + 1)
        eedf = np.zeros(self.eedf_bins + 1, np.int64)
        fneg = np.zeros(max(self.nf, 1), np.int64)
        m.density_m3 = _p(dens, C.c_double)
        m.phi_V = _p(phi, C.c_double)
        m.eedf = _p(eedf, C.c_int64)
        m.fneg = _p(fneg, C.c_int64)
        self._check(self.L.pic_moments(self.h, C.byref(m)))
        return dict(step=m.step, cycles=m.cycles, alive=list(m.alive), events=np.array(m.events[:]),
                    absorbed=np.array([list(r) for r in m.absorbed]), particle_steps=m.particle_steps,
                    births=m.births, next_id=m.next_id, density=dens, phi=phi, eedf=eedf, fneg=fneg[: self.nf])

    def set_grid(self, workgroups):
        self._check(self.L.pic_set_grid(self.h, workgroups))

    def set_graphs(self, enable=True):
        self._check(self.L.pic_set_graphs(self.h, 1 if enable else 0))

    def autotune(self, steps_per_trial=200):
        """Pick the fastest persistent grid of the push kernel by timing a few
        (6 x steps_per_trial real steps); returns its workgroup count."""
        g = C.c_int32(0)
        self._check(self.L.pic_autotune(self.h, steps_per_trial, C.byref(g)))
        return g.value

    def set_shape(self, threads_per_workgroup, particles_per_thread):
        """Tile shape of the fused particle kernel (256x4, 512x4 or 256x8)."""
        self._check(self.L.pic_set_shape(self.h, threads_per_workgroup, particles_per_thread))

    def launch_shape(self):
        """(threads per workgroup, particles per thread, persistent workgroups) of the push."""
        t, p, g = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        self._check(self.L.pic_launch_shape(self.h, C.byref(t), C.byref(p), C.byref(g)))
        return t.value, p.value, g.value

    def timing(self, enable=True, every=1):
        """HIP events around every `every`-th launch of the fused kernel."""
        self._check(self.L.pic_timing(self.h, int(every) if enable else 0))

    def kernel_time(self):
        ms = C.c_double(0)
        n = C.c_int64(0)
        self._check(self.L.pic_kernel_time(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value


def step_batch(discharges, n_steps):
    """Advance independent discharges together (pic_step_batch): each on its
    own stream, their work interleaved so that they run concurrently."""
    if not discharges:
        return
    L = discharges[0].L
    arr = (C.c_void_p * len(discharges))(*[d.h for d in discharges])
    rc = L.pic_step_batch(arr, len(discharges), n_steps)
    if rc != 0:
        for d in discharges:
            msg = L.pic_last_error(d.h)
            if msg:
                raise PicError(rc, msg.decode())
        raise PicError(rc, "")


def step_batch_static(discharges, n_steps):
    """Batched steps without library allocations (pic_step_batch_static): the
    batch's tables live in a fixed device array; at most PIC_BATCH_STATIC_MAX
    (64) discharges of the same precision, periods and phase."""
    if not discharges:
        return
    L = discharges[0].L
    arr = (C.c_void_p * len(discharges))(*[d.h for d in discharges])
    rc = L.pic_step_batch_static(arr, len(discharges), n_steps)
    if rc != 0:
        msg = L.pic_last_error(discharges[0].h)
        raise PicError(rc, msg.decode() if msg else "")


def autotune_batch(discharges, steps_per_trial=50):
    """Time the batched launches of pic_step_batch on every tile shape and two
    push grids (real steps of every discharge) and keep the fastest for
    batches led by discharges[0]; returns (threads, particles per thread,
    workgroups)."""
    L = discharges[0].L
    arr = (C.c_void_p * len(discharges))(*[d.h for d in discharges])
    t, p, g = C.c_int32(0), C.c_int32(0), C.c_int32(0)
    rc = L.pic_autotune_batch(arr, len(discharges), steps_per_trial, C.byref(t), C.byref(p), C.byref(g))
    if rc != 0:
        msg = L.pic_last_error(discharges[0].h)
        raise PicError(rc, msg.decode() if msg else "")
    return t.value, p.value, g.value
