"""Oracle for the EM-shower step loop -- TEST INFRASTRUCTURE ONLY.

A plain, slow CPU definition of what the device library computes:

* ``oracle.tables``   -- FP64 physics tables from closed-form cross sections
                         and a Gauss-Legendre range quadrature (numpy);
* ``oracle/transport.c`` -- history-based transport in plain C (one event at a
                         time, LIFO stack of secondaries), Philox4x64-10 random
                         numbers keyed by (event, track key, step).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product package never does; it has
its own table builder and transport kernels and shares no code with this one.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from . import tables

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "transport.c")

GAMMA, ELECTRON, POSITRON = 0, 1, 2
P_COMPTON, P_PHOTO, P_PAIR, P_MOLLER, P_BHABHA, P_BREMS = range(6)
OUT_INTERACT, OUT_LOSS, OUT_BOUNDARY, OUT_ESCAPE, OUT_STOP, OUT_GUARD, OUT_NO_INTERACT = range(7)
F_NONE, F_ZLO, F_ZHI, F_XLO, F_XHI, F_YLO, F_YHI = range(7)

TRACK_DTYPE = np.dtype([
    ("event", "<u8"), ("key", "<u8"), ("type", "<i4"), ("slab", "<i4"),
    ("step", "<u4"), ("alive", "<i4"), ("T", "<f8"), ("nl", "<f8"),
    ("r", "<f8", (3,)), ("u", "<f8", (3,)),
], align=True)
assert TRACK_DTYPE.itemsize == 96

MAX_SEC = 4
RESULT_DTYPE = np.dtype([
    ("outcome", "<i4"), ("process", "<i4"), ("face", "<i4"), ("dep_slab", "<i4"),
    ("step_len", "<f8"), ("edep", "<f8"), ("escaped", "<f8"),
    ("n_pair", "<i4"), ("n_annih", "<i4"), ("n_sec", "<i4"), ("reject_capped", "<i4"),
    ("drew_u0", "<i4"), ("n_draws", "<i4"),
    ("sec", TRACK_DTYPE, (MAX_SEC,)),
], align=True)
assert RESULT_DTYPE.itemsize == 448

MARGIN_DTYPE = np.dtype([("margin", "<f8"), ("kind", "<i4"), ("n_notes", "<i4")], align=True)
assert MARGIN_DTYPE.itemsize == 16
# decision kinds of a margin (see note() in transport.c)
MARGIN_KINDS = ["none", "cut at step start", "process threshold", "loss vs interaction limit",
                "final range", "geometry vs physics limit", "face tie", "direction sign", "chord beyond plane",
                "chord face tie", "chord at start", "near face (d_int)", "boundary search acceptance (d_int)",
                "last substep", "cut after loss", "process selection", "rejection test", "sampling branch",
                "secondary cut", "rotation pole branch"]
TRACE_DTYPE = np.dtype([("pre", TRACK_DTYPE), ("post", TRACK_DTYPE), ("res", RESULT_DTYPE), ("m", MARGIN_DTYPE)],
                       align=True)
assert TRACE_DTYPE.itemsize == 96 + 96 + 448 + 16

LEDGER_DTYPE = np.dtype([
    ("escaped", "<f8"), ("n_pair", "<u8"), ("n_annih", "<u8"), ("steps", "<u8"),
    ("n_sec", "<u8", (3,)), ("n_guard", "<u8"), ("n_reject_cap", "<u8"),
], align=True)
assert LEDGER_DTYPE.itemsize == 72


class _Problem(C.Structure):
    _fields_ = [
        ("n_slabs", C.c_int32), ("n_materials", C.c_int32),
        ("z_planes", C.c_void_p), ("slab_material", C.c_void_p),
        ("half_width", C.c_double), ("B", C.c_double * 3),
        ("tables", C.c_void_p), ("ecut", C.c_double), ("seed", C.c_uint64),
        ("no_discrete", C.c_int32), ("msc", C.c_int32), ("x0_cm", C.c_void_p),
    ]


def build(force: bool = True) -> str:
    """Compile transport.c with gcc (plain IEEE FP64: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                        "-ffp-contract=off", "-Wall", "-Wno-unused-function", "-o", tmp, SRC,
                        "-lm", "-lpthread"], check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=True)
        L = C.CDLL(LIB_PATH)
        L.orc_step.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_void_p]
        L.orc_step.restype = None
        L.orc_interact.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_int, C.POINTER(C.c_int), C.c_void_p]
        L.orc_interact.restype = None
        L.orc_run_events.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32,
                                     C.c_void_p, C.c_void_p, C.c_int]
        L.orc_run_events.restype = C.c_uint64
        L.orc_philox4x64.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_philox4x64.restype = None
        L.orc_rk4.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_rk4.restype = None
        L.orc_propagate_field.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_double, C.POINTER(C.c_int),
                                          C.POINTER(C.c_int)]
        L.orc_propagate_field.restype = C.c_double
        L.orc_lookup.argtypes = [C.c_void_p, C.c_double]
        L.orc_lookup.restype = C.c_double
        L.orc_inverse_range.argtypes = [C.c_void_p, C.c_double]
        L.orc_inverse_range.restype = C.c_double
        L.orc_xs.argtypes = [C.POINTER(_Problem), C.c_int, C.c_int, C.c_double]
        L.orc_xs.restype = C.c_double
        L.orc_msc_theta0.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_msc_theta0.restype = C.c_double
        L.orc_msc_deflect.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_int, C.c_double, C.c_double]
        L.orc_msc_deflect.restype = None
        L.orc_step_margin.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_step_margin.restype = None
        L.orc_trace_event.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64]
        L.orc_trace_event.restype = C.c_uint64
        _lib = L
    return _lib


class Problem:
    """Geometry + materials + cut + seed, with the oracle's own FP64 tables."""

    def __init__(self, z_planes, slab_material, half_width, B, materials, ecut, seed,
                 no_discrete=False, table_blob=None, msc=False):
        self.z_planes = np.ascontiguousarray(z_planes, dtype=np.float64)
        self.slab_material = np.ascontiguousarray(slab_material, dtype=np.int32)
        self.materials = [m if isinstance(m, tables.Material) else tables.Material(*m) for m in materials]
        self.ecut = float(ecut)
        self.tables = (np.ascontiguousarray(table_blob, dtype=np.float64) if table_blob is not None
                       else tables.build_tables(self.materials, self.ecut))
        self.n_slabs = len(self.slab_material)
        s = _Problem()
        s.n_slabs = self.n_slabs
        s.n_materials = len(self.materials)
        s.z_planes = self.z_planes.ctypes.data
        s.slab_material = self.slab_material.ctypes.data
        s.half_width = float(half_width)
        for i in range(3):
            s.B[i] = float(B[i])
        s.tables = self.tables.ctypes.data
        s.ecut = self.ecut
        s.seed = int(seed)
        s.no_discrete = int(bool(no_discrete))
        self.x0_cm = np.array([m.X0_cm for m in self.materials], dtype=np.float64)
        s.msc = int(bool(msc))
        s.x0_cm = self.x0_cm.ctypes.data
        self._s = s

    # -- single step ----------------------------------------------------------
    def step(self, track):
        """Take one step of each track in `track` (array of TRACK_DTYPE, updated
        in place).  Returns the RESULT_DTYPE records."""
        tr = np.atleast_1d(track)
        assert tr.dtype == TRACK_DTYPE and tr.flags.c_contiguous
        res = np.zeros(len(tr), dtype=RESULT_DTYPE)
        L = lib()
        for i in range(len(tr)):
            L.orc_step(C.byref(self._s), tr[i:i + 1].ctypes.data, res[i:i + 1].ctypes.data)
        return res

    def step_margins(self, track):
        """As step(), and also the smallest decision margin of each step
        (MARGIN_DTYPE records: margin, kind index into MARGIN_KINDS)."""
        tr = np.atleast_1d(track)
        assert tr.dtype == TRACK_DTYPE and tr.flags.c_contiguous
        res = np.zeros(len(tr), dtype=RESULT_DTYPE)
        m = np.zeros(len(tr), dtype=MARGIN_DTYPE)
        L = lib()
        for i in range(len(tr)):
            L.orc_step_margin(C.byref(self._s), tr[i:i + 1].ctypes.data, res[i:i + 1].ctypes.data,
                              m[i:i + 1].ctypes.data)
        return res, m

    def trace_event(self, prims):
        """Every step of one event's history (the primaries `prims`, one
        event, TRACK_DTYPE), in history order: TRACE_DTYPE records."""
        p = np.ascontiguousarray(prims, dtype=TRACK_DTYPE)
        L = lib()
        cap = 1 << 14
        while True:
            out = np.zeros(cap, dtype=TRACE_DTYPE)
            n = L.orc_trace_event(C.byref(self._s), p.ctypes.data, len(p), out.ctypes.data, cap)
            if n <= cap:
                return out[:n]
            cap = int(n)

    def interact(self, track, process, j0=1):
        tr = np.atleast_1d(track)
        res = np.zeros(len(tr), dtype=RESULT_DTYPE)
        L = lib()
        for i in range(len(tr)):
            j = C.c_int(j0)
            L.orc_interact(C.byref(self._s), tr[i:i + 1].ctypes.data, int(process), C.byref(j),
                           res[i:i + 1].ctypes.data)
        return res

    def propagate_field(self, track, s_phys):
        tr = np.atleast_1d(track)
        face = C.c_int(0)
        nsub = C.c_int(0)
        s = lib().orc_propagate_field(C.byref(self._s), tr.ctypes.data, float(s_phys), C.byref(face), C.byref(nsub))
        return s, face.value, nsub.value

    def xs(self, mat, proc, T):
        return lib().orc_xs(C.byref(self._s), int(mat), int(proc), float(T))

    def msc_deflect(self, track, mat, T_pre, s):
        """Apply the multiple-scattering deflection of a step of length s to
        each track (direction updated in place)."""
        tr = np.atleast_1d(track)
        assert tr.dtype == TRACK_DTYPE and tr.flags.c_contiguous
        L = lib()
        for i in range(len(tr)):
            L.orc_msc_deflect(C.byref(self._s), tr[i:i + 1].ctypes.data, int(mat), float(T_pre), float(s))


    # -- whole events -----------------------------------------------------------
    def run_events(self, prims, rows, n_rows, n_threads=1):
        """History-based transport of all primaries.  Returns (edep[n_rows, n_slabs],
        ledger[n_rows], total steps)."""
        prims = np.ascontiguousarray(prims, dtype=TRACK_DTYPE)
        rows = np.ascontiguousarray(rows, dtype=np.uint32)
        edep = np.zeros((n_rows, self.n_slabs))
        led = np.zeros(n_rows, dtype=LEDGER_DTYPE)
        steps = lib().orc_run_events(C.byref(self._s), prims.ctypes.data, rows.ctypes.data, len(prims),
                                     int(n_rows), edep.ctypes.data, led.ctypes.data, int(n_threads))
        return edep, led, int(steps)


def philox4x64(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def rk4(r, u, h, kf, B):
    r = np.ascontiguousarray(r, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    r1 = np.zeros(3)
    u1 = np.zeros(3)
    lib().orc_rk4(r.ctypes.data, u.ctypes.data, float(h), float(kf), B.ctypes.data, r1.ctypes.data, u1.ctypes.data)
    return r1, u1


def lookup(v, T):
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().orc_lookup(v.ctypes.data, float(T))


def inverse_range(R, r):
    R = np.ascontiguousarray(R, dtype=np.float64)
    return lib().orc_inverse_range(R.ctypes.data, float(r))


def tracks_from_primaries(prims, seed_rows=None):
    """Convert input primaries (workloads.PRIM_DTYPE) to oracle tracks; returns (tracks, rows)."""
    t = np.zeros(len(prims), dtype=TRACK_DTYPE)
    t["event"] = prims["event"]
    t["key"] = prims["key"]
    t["type"] = prims["type"]
    t["slab"] = prims["slab"]
    t["alive"] = 1
    t["T"] = prims["T"]
    t["nl"] = -1.0
    t["r"] = prims["r"]
    t["u"] = prims["u"]
    rows = np.asarray(prims["event"], dtype=np.uint32) if seed_rows is None else np.asarray(seed_rows, np.uint32)
    return t, rows


def problem_for(workload, **kw):
    st = workload.stack
    return Problem(st.z_planes, st.slab_material, st.half_width, st.B, st.materials, workload.ecut,
                   workload.seed, **kw)


def msc_theta0(T, s, X0):
    """Highland width of the projected scattering angle [rad] (0 for s = 0)."""
    return lib().orc_msc_theta0(float(T), float(s), float(X0))
