"""Thin Python binding of libemstep.so (the C ABI in include/emstep.h).

Argument marshalling only: every step of the transport runs in the library's
HIP kernels.  PyTorch provides the device workspace (one uint8 tensor) and the
HIP stream.  There is no fallback: if the library is missing this module
raises at import time.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
# torch must be loaded before the library: its bundled HIP runtime carries the
# same SONAME as the system one, so the library then binds to that single
# runtime (the one that owns the workspace tensor and the stream)
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libemstep.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2503_17608_amd/build.py (hipcc, gfx950)")

_lib = C.CDLL(LIB_PATH)

ABI_VERSION = 8
FP64, MIXED = 0, 1
SORT_NONE, SORT_PARTITION, SORT_RADIX, SORT_QUEUE = 0, 1, 2, 3
SORT_POLICIES = {"none": SORT_NONE, "partition": SORT_PARTITION, "radix": SORT_RADIX, "queue": SORT_QUEUE}
GAMMA, ELECTRON, POSITRON = 0, 1, 2
TABLE_NODES, TABLES_PER_MATERIAL = 181, 8

OK, ERR_INVALID_ARG, ERR_STATE, ERR_CAPACITY, ERR_DEVICE, ERR_NUMERIC, ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6


class Options(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("precision", C.c_int32),
        ("n_slots", C.c_uint64), ("n_initializers", C.c_uint64), ("n_primaries", C.c_uint64),
        ("max_events", C.c_uint32), ("max_slabs", C.c_uint32), ("max_materials", C.c_uint32),
        ("sort_policy", C.c_int32), ("init_partition", C.c_int32), ("max_substeps", C.c_int32),
        ("seed", C.c_uint64), ("block_size", C.c_int32), ("graph_iterations", C.c_int32),
        ("lds_tables", C.c_int32), ("streams", C.c_int32), ("msc", C.c_int32), ("deterministic", C.c_int32),
    ]


class Material(C.Structure):
    _fields_ = [("Z", C.c_double), ("A", C.c_double), ("density", C.c_double), ("I_eV", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("sort_policy", C.c_int32), ("tail_threshold", C.c_uint32), ("block", C.c_int32 * 16),
                ("drain_threshold", C.c_uint32), ("drain_steps", C.c_uint32), ("reuse_parent_slot", C.c_uint32),
                ("fuse_interactions", C.c_uint32), ("phase_sort", C.c_uint32 * 2), ("fuse_along", C.c_uint32)]


class Counters(C.Structure):
    _fields_ = [("iterations", C.c_uint64), ("alive", C.c_uint64), ("queued", C.c_uint64),
                ("pending_primaries", C.c_uint64), ("steps", C.c_uint64), ("overflow", C.c_uint32),
                ("completed", C.c_uint32), ("work", C.c_uint64 * 24)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "work"}
        d["work"] = {name: int(self.work[i]) for i, name in WORK_INDEX.items()}
        return d


WORK_INDEX = {0: "reused_slots", 1: "init", 2: "pre_step", 4: "along_neutral", 5: "along_charged", 6: "along_field",
              7: "compton", 8: "photoelectric", 9: "pair", 10: "moller", 11: "bhabha", 12: "bremsstrahlung",
              13: "annihilation", 14: "field_paused", 15: "field_substeps", 16: "drain"}


PRIMARY_DTYPE = np.dtype([
    ("event", "<u8"), ("key", "<u8"), ("type", "<i4"), ("slab", "<i4"),
    ("T", "<f8"), ("r", "<f8", (3,)), ("u", "<f8", (3,)),
], align=True)
TRACK_DTYPE = np.dtype([
    ("key", "<u8"), ("row", "<u4"), ("step", "<u4"), ("type", "<i4"), ("slab", "<i4"),
    ("T", "<f8"), ("nl", "<f8"), ("r", "<f8", (3,)), ("u", "<f8", (3,)),
], align=True)
LEDGER_DTYPE = np.dtype([
    ("escaped", "<f8"), ("n_pair", "<u8"), ("n_annih", "<u8"), ("steps", "<u8"),
    ("n_sec", "<u8", (3,)), ("n_guard", "<u8"), ("n_reject_cap", "<u8"),
], align=True)
assert PRIMARY_DTYPE.itemsize == 80 and TRACK_DTYPE.itemsize == 88 and LEDGER_DTYPE.itemsize == 72

_P = C.c_void_p
_sigs = {
    "ems_abi_version": (C.c_uint32, []),
    "ems_last_error": (C.c_char_p, []),
    "ems_query_workspace": (C.c_int, [C.POINTER(Options), C.POINTER(C.c_uint64)]),
    "ems_create": (C.c_int, [C.POINTER(Options), _P, C.c_uint64, _P, C.POINTER(_P)]),
    "ems_destroy": (None, [_P]),
    "ems_load_materials": (C.c_int, [_P, _P, C.c_uint32]),
    "ems_load_geometry": (C.c_int, [_P, _P, _P, C.c_uint32, C.c_double, _P]),
    "ems_build_tables": (C.c_int, [_P, C.c_double]),
    "ems_load_tables": (C.c_int, [_P, _P, C.c_uint32, C.c_double]),
    "ems_read_tables": (C.c_int, [_P, _P, C.c_uint64]),
    "ems_push_primaries": (C.c_int, [_P, _P, C.c_uint64]),
    "ems_step": (C.c_int, [_P, C.c_uint32, C.POINTER(Counters)]),
    "ems_run": (C.c_int, [_P, C.c_uint64, C.POINTER(Counters)]),
    "ems_read_counters": (C.c_int, [_P, C.POINTER(Counters)]),
    "ems_poll_completed": (C.c_int, [_P, _P, C.c_uint32, C.POINTER(C.c_uint32)]),
    "ems_last_counters": (C.c_int, [_P, C.POINTER(Counters)]),
    "ems_read_edep": (C.c_int, [_P, C.c_uint64, _P, C.c_uint32, _P]),
    "ems_read_all_tallies": (C.c_int, [_P, _P, _P, _P]),
    "ems_release_event": (C.c_int, [_P, C.c_uint64]),
    "ems_release_events": (C.c_int, [_P, _P, C.c_uint64]),
    "ems_debug_register_event": (C.c_int, [_P, C.c_uint64, C.POINTER(C.c_uint32)]),
    "ems_debug_inject": (C.c_int, [_P, _P, C.c_uint64]),
    "ems_debug_iterate": (C.c_int, [_P, C.c_uint32, C.c_int32]),
    "ems_debug_read_tracks": (C.c_int, [_P, _P, C.c_uint64]),
    "ems_debug_read_secondaries": (C.c_int, [_P, _P, C.c_uint64, C.POINTER(C.c_uint64)]),
    "ems_debug_sort": (C.c_int, [_P, _P, C.c_uint64, C.c_int32, _P]),
    "ems_sort_keys_noalloc": (C.c_int, [_P, _P, C.c_uint64, C.c_int32, _P]),
    "ems_set_tuning": (C.c_int, [_P, C.POINTER(Tuning)]),
    "ems_get_tuning": (C.c_int, [_P, C.POINTER(Tuning)]),
    "ems_profile_enable": (C.c_int, [_P, C.c_int32]),
    "ems_profile_read": (C.c_int, [_P, _P, _P, _P, C.c_uint32, C.POINTER(C.c_uint32)]),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class EmsError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what} failed ({status}): {_lib.ems_last_error().decode()}")


def _check(status, what):
    if status != OK:
        raise EmsError(status, what)


def _ptr(a: np.ndarray):
    return C.c_void_p(a.ctypes.data)


def exported_symbols():
    return list(_sigs)


class Session:
    """One library context: slots, buffers and tallies resident on `device`."""

    def __init__(self, n_slots, precision="f64", n_initializers=None, n_primaries=None, max_events=1024,
                 max_slabs=128, max_materials=4, sort_policy="none", init_partition=False, max_substeps=10,
                 seed=1, block_size=0, graph_iterations=0, lds_tables=1, streams=4, device="cuda:0",
                 stream=None, msc=False, deterministic=False):
        o = Options()
        o.abi_version = ABI_VERSION
        o.precision = MIXED if precision in ("mixed", "f32", MIXED) else FP64
        o.n_slots = int(n_slots)
        o.n_initializers = int(n_initializers if n_initializers else 16 * n_slots)
        o.n_primaries = int(n_primaries if n_primaries else max(1 << 16, n_slots))
        o.max_events = int(max_events)
        o.max_slabs = int(max_slabs)
        o.max_materials = int(max_materials)
        o.sort_policy = SORT_POLICIES[sort_policy] if isinstance(sort_policy, str) else int(sort_policy)
        o.init_partition = int(bool(init_partition))
        o.max_substeps = int(max_substeps)
        o.seed = int(seed)
        o.block_size = int(block_size)
        o.graph_iterations = int(graph_iterations)
        o.lds_tables = int(lds_tables)
        o.streams = int(streams)
        o.msc = int(bool(msc))
        o.deterministic = int(bool(deterministic))
        self.options = o
        nbytes = C.c_uint64(0)
        _check(_lib.ems_query_workspace(C.byref(o), C.byref(nbytes)), "ems_query_workspace")
        self.device = torch.device(device)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        if stream is not None:
            self.stream = stream
        elif graph_iterations > 0:
            # graph capture needs a stream other than the null stream
            self.stream = torch.cuda.Stream(self.device)
        else:
            self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(_lib.ems_create(C.byref(o), C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                               C.c_void_p(self.stream.cuda_stream), C.byref(h)), "ems_create")
        self._h = h
        self.n_slabs = 0

    def close(self):
        if getattr(self, "_h", None):
            _lib.ems_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- loading ------------------------------------------------------------------
    def load(self, z_planes, slab_material, half_width, B, materials, ecut, tables=None):
        mats = (Material * len(materials))(*[Material(*m) for m in materials])
        _check(_lib.ems_load_materials(self._h, C.cast(mats, C.c_void_p), len(materials)), "ems_load_materials")
        z = np.ascontiguousarray(z_planes, dtype=np.float64)
        sm = np.ascontiguousarray(slab_material, dtype=np.int32)
        b = np.ascontiguousarray(B, dtype=np.float64)
        _check(_lib.ems_load_geometry(self._h, _ptr(z), _ptr(sm), len(sm), float(half_width), _ptr(b)),
               "ems_load_geometry")
        self.n_slabs = len(sm)
        self.n_materials = len(materials)
        if tables is None:
            _check(_lib.ems_build_tables(self._h, float(ecut)), "ems_build_tables")
        else:
            t = np.ascontiguousarray(tables, dtype=np.float64)
            _check(_lib.ems_load_tables(self._h, _ptr(t), len(materials), float(ecut)), "ems_load_tables")

    def read_tables(self):
        out = np.zeros((self.n_materials, TABLES_PER_MATERIAL, TABLE_NODES))
        _check(_lib.ems_read_tables(self._h, _ptr(out), out.size), "ems_read_tables")
        return out

    # -- primaries and stepping -----------------------------------------------------
    def push(self, primaries):
        p = np.ascontiguousarray(primaries)
        if p.dtype != PRIMARY_DTYPE:
            q = np.zeros(len(p), dtype=PRIMARY_DTYPE)
            for f in PRIMARY_DTYPE.names:
                q[f] = p[f]
            p = q
        _check(_lib.ems_push_primaries(self._h, _ptr(p), len(p)), "ems_push_primaries")

    def step(self, iterations=1, read=True):
        c = Counters()
        _check(_lib.ems_step(self._h, int(iterations), C.byref(c) if read else None), "ems_step")
        return c.as_dict() if read else None

    def run(self, max_iterations=1_000_000):
        c = Counters()
        _check(_lib.ems_run(self._h, int(max_iterations), C.byref(c)), "ems_run")
        return c.as_dict()

    def counters(self):
        c = Counters()
        _check(_lib.ems_read_counters(self._h, C.byref(c)), "ems_read_counters")
        return c.as_dict()

    def last_counters(self):
        """Counters of the snapshot the last synchronizing call read (no device work)."""
        c = Counters()
        _check(_lib.ems_last_counters(self._h, C.byref(c)), "ems_last_counters")
        return c.as_dict()

    # -- results ----------------------------------------------------------------------
    def read_edep(self, event):
        e = np.zeros(self.n_slabs)
        led = np.zeros(1, dtype=LEDGER_DTYPE)
        _check(_lib.ems_read_edep(self._h, int(event), _ptr(e), self.n_slabs, _ptr(led)), "ems_read_edep")
        return e, led[0]

    def read_all(self):
        n = self.options.max_events
        e = np.zeros((n, self.n_slabs))
        led = np.zeros(n, dtype=LEDGER_DTYPE)
        ev = np.zeros(n, dtype=np.uint64)
        _check(_lib.ems_read_all_tallies(self._h, _ptr(e), _ptr(led), _ptr(ev)), "ems_read_all_tallies")
        return e, led, ev

    def tallies_by_event(self, events):
        """edep[len(events), n_slabs] and ledgers ordered like `events`."""
        e, led, ev = self.read_all()
        row = {int(x): i for i, x in enumerate(ev) if x != np.uint64(2 ** 64 - 1)}
        idx = np.array([row[int(x)] for x in events])
        return e[idx], led[idx]

    def release(self, event):
        """Release one event id, or an array of them (one clearing kernel)."""
        if np.ndim(event) == 0:
            _check(_lib.ems_release_event(self._h, int(event)), "ems_release_event")
        else:
            ev = np.ascontiguousarray(event, dtype=np.uint64)
            _check(_lib.ems_release_events(self._h, _ptr(ev), len(ev)), "ems_release_events")

    def poll_completed(self, cap=4096):
        ev = np.zeros(cap, dtype=np.uint64)
        n = C.c_uint32(0)
        _check(_lib.ems_poll_completed(self._h, _ptr(ev), cap, C.byref(n)), "ems_poll_completed")
        return ev[: n.value]

    def launch(self, iterations):
        """Enqueue step iterations without waiting (graph batches when configured)."""
        _check(_lib.ems_step(self._h, int(iterations), None), "ems_step")

    # -- test hooks ---------------------------------------------------------------------
    def register_event(self, event):
        r = C.c_uint32(0)
        _check(_lib.ems_debug_register_event(self._h, int(event), C.byref(r)), "ems_debug_register_event")
        return r.value

    def inject(self, tracks):
        t = np.ascontiguousarray(tracks, dtype=TRACK_DTYPE)
        _check(_lib.ems_debug_inject(self._h, _ptr(t), len(t)), "ems_debug_inject")

    def iterate(self, iterations=1, no_init=False):
        _check(_lib.ems_debug_iterate(self._h, int(iterations), int(bool(no_init))), "ems_debug_iterate")

    def read_tracks(self, n):
        t = np.zeros(n, dtype=TRACK_DTYPE)
        _check(_lib.ems_debug_read_tracks(self._h, _ptr(t), n), "ems_debug_read_tracks")
        return t

    def read_secondaries(self, cap=None):
        n = C.c_uint64(0)
        _check(_lib.ems_debug_read_secondaries(self._h, None, 0, C.byref(n)), "ems_debug_read_secondaries")
        m = n.value if cap is None else min(cap, n.value)
        t = np.zeros(m, dtype=TRACK_DTYPE)
        if m:
            _check(_lib.ems_debug_read_secondaries(self._h, _ptr(t), m, C.byref(n)), "ems_debug_read_secondaries")
        return t

    def sort(self, keys, policy="partition"):
        k = np.ascontiguousarray(keys, dtype=np.uint8)
        perm = np.zeros(len(k), dtype=np.uint32)
        _check(_lib.ems_debug_sort(self._h, _ptr(k), len(k), SORT_POLICIES[policy], _ptr(perm)), "ems_debug_sort")
        return perm

    def sort_device(self, keys, perm, policy="partition"):
        """Allocation-free sort of device keys (torch uint8 tensor) into the
        device permutation `perm` (torch int32/uint32 tensor of the same
        length), enqueued on the session's stream."""
        assert keys.is_cuda and perm.is_cuda and keys.dtype == torch.uint8 and perm.element_size() == 4
        assert keys.is_contiguous() and perm.is_contiguous() and perm.numel() >= keys.numel()
        _check(_lib.ems_sort_keys_noalloc(self._h, C.c_void_p(keys.data_ptr()), keys.numel(),
                                          SORT_POLICIES[policy], C.c_void_p(perm.data_ptr())),
               "ems_sort_keys_noalloc")

    def tuning(self):
        t = Tuning()
        _check(_lib.ems_get_tuning(self._h, C.byref(t)), "ems_get_tuning")
        return {"sort_policy": t.sort_policy, "tail_threshold": t.tail_threshold,
                "drain_threshold": t.drain_threshold, "drain_steps": t.drain_steps,
                "reuse_parent_slot": bool(t.reuse_parent_slot), "fuse_interactions": bool(t.fuse_interactions),
                "phase_sort": (int(t.phase_sort[0]), int(t.phase_sort[1])), "fuse_along": bool(t.fuse_along),
                "block": {KERNEL_ROLES[i]: t.block[i] for i in range(len(KERNEL_ROLES)) if t.block[i]}}

    def set_tuning(self, sort_policy=None, tail_threshold=None, block=None, drain_threshold=None, drain_steps=None,
                   reuse_parent_slot=None, fuse_interactions=None, phase_sort=None, fuse_along=None):
        """Change knobs that affect speed only; block maps kernel role names to
        block sizes; phase_sort is a pair of 32-bit masks over occupancy
        buckets floor(log2 live tracks): bit b of mask p set = sort point p
        reorders in iterations of bucket b."""
        cur = Tuning()
        _check(_lib.ems_get_tuning(self._h, C.byref(cur)), "ems_get_tuning")
        if sort_policy is not None:
            cur.sort_policy = SORT_POLICIES[sort_policy] if isinstance(sort_policy, str) else int(sort_policy)
        if tail_threshold is not None:
            cur.tail_threshold = int(tail_threshold)
        if drain_threshold is not None:
            cur.drain_threshold = int(drain_threshold)
        if drain_steps is not None:
            cur.drain_steps = int(drain_steps)
        if reuse_parent_slot is not None:
            cur.reuse_parent_slot = 1 if reuse_parent_slot else 0
        if fuse_interactions is not None:
            cur.fuse_interactions = 1 if fuse_interactions else 0
        if fuse_along is not None:
            cur.fuse_along = 1 if fuse_along else 0
        if block is not None:
            for name, b in block.items():
                cur.block[KERNEL_ROLES.index(name)] = int(b)
        if phase_sort is not None:
            cur.phase_sort[0] = int(phase_sort[0]) & 0xFFFFFFFF
            cur.phase_sort[1] = int(phase_sort[1]) & 0xFFFFFFFF
        _check(_lib.ems_set_tuning(self._h, C.byref(cur)), "ems_set_tuning")

    def profile(self, mask):
        _check(_lib.ems_profile_enable(self._h, int(mask)), "ems_profile_enable")

    def profile_read(self):
        names = (C.c_char_p * 32)()
        ms = np.zeros(32)
        n_l = np.zeros(32, dtype=np.uint64)
        n = C.c_uint32(0)
        _check(_lib.ems_profile_read(self._h, C.cast(names, C.c_void_p), _ptr(ms), _ptr(n_l), 32, C.byref(n)),
               "ems_profile_read")
        return {names[i].decode(): (float(ms[i]), int(n_l[i])) for i in range(n.value)}


KERNEL_ROLES = ["vacancies", "init", "pre_step", "sort", "along_neutral", "along_charged", "along_field",
                "compton", "photoelectric", "pair", "moller", "bhabha", "bremsstrahlung", "drain", "interactions",
                "annihilation"]


def role_mask(*names):
    m = 0
    for n in names:
        m |= 1 << KERNEL_ROLES.index(n)
    return m
