"""Seeded synthetic inputs for the EM-shower step loop.

This module only generates inputs -- materials, the slab stack, primaries with
their random-number keys -- and holds none of the transport arithmetic.  Both
the device library (through its Python binding) and the oracle receive exactly
the same arrays from here.

The paper's benchmark problems (TestEM3, CMS and ATLAS geometries with 16
events of 1300 x 10 GeV electrons; "Performance results") need detector
geometry files and Geant4.  A lead / liquid-argon sampling-calorimeter slab
stack stands in for them; the workloads below are named by what they are.

Primary keys and sampled quantities come from numpy's Philox4x64-10 in the
primary-generation domain (counter word 3 = 2): primary i of event e uses
counter (i, 0, b, 2) under key (seed, e); block 0 gives the track key, the
species, the energy and the polar cosine; block 1 gives the azimuth.  The
number of primaries of event e is word 0 of counter (2^64-1, 0, 0, 2).
numpy's generator increments its counter before the first block, so the
generator is started at counter - 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA, ELECTRON, POSITRON = 0, 1, 2

# (Z, A [g/mol], density [g/cm^3], mean excitation energy I [eV])
LEAD = (82.0, 207.2, 11.35, 823.0)
LIQUID_ARGON = (18.0, 39.948, 1.396, 188.0)

PRIM_DTYPE = np.dtype([
    ("event", "<u8"), ("key", "<u8"), ("type", "<i4"), ("slab", "<i4"),
    ("T", "<f8"), ("r", "<f8", (3,)), ("u", "<f8", (3,)),
], align=True)
assert PRIM_DTYPE.itemsize == 80

U64 = (1 << 64) - 1


def philox_block(seed: int, event: int, c0: int, c1: int, c2: int, c3: int) -> np.ndarray:
    """Philox4x64-10 block at counter (c0..c3), key (seed, event), via numpy."""
    ctr = (c0 | (c1 << 64) | (c2 << 128) | (c3 << 192)) - 1
    ctr &= (1 << 256) - 1
    words = [(ctr >> (64 * i)) & U64 for i in range(4)]
    g = np.random.Philox(key=np.array([seed & U64, event & U64], dtype=np.uint64),
                         counter=np.array(words, dtype=np.uint64))
    return g.random_raw(4)


def unit(w) -> float:
    return ((int(w) >> 12) + 0.5) * 2.0 ** -52


@dataclass
class Stack:
    """Slab stack: z planes (n_slabs + 1), material index per slab, lateral half width."""
    z_planes: np.ndarray
    slab_material: np.ndarray
    half_width: float
    B: tuple = (0.0, 0.0, 0.0)
    materials: list = field(default_factory=lambda: [LEAD, LIQUID_ARGON])

    @property
    def n_slabs(self) -> int:
        return len(self.slab_material)


def sampling_stack(n_layers: int, width_cm: float, B_tesla=(0.0, 0.0, 0.0),
                   pb_cm: float = 0.2, lar_cm: float = 0.5) -> Stack:
    """n_layers of (Pb pb_cm, LAr lar_cm): 2 n_layers slabs starting at z = 0."""
    th = []
    mats = []
    for _ in range(n_layers):
        th += [pb_cm, lar_cm]
        mats += [0, 1]
    z = np.zeros(len(th) + 1)
    for i, t in enumerate(th):
        z[i + 1] = z[i] + t
    return Stack(z, np.array(mats, dtype=np.int32), 0.5 * width_cm, tuple(float(b) for b in B_tesla))


@dataclass
class Workload:
    name: str
    stack: Stack
    ecut: float
    seed: int
    n_events: int
    primaries: np.ndarray          # PRIM_DTYPE, event = row index
    n_slots: int
    precision: str = "f64"


def make_primaries(seed: int, n_events: int, per_event, species, e_range, cone_deg: float = 0.0,
                   first_event: int = 0) -> np.ndarray:
    """Primaries at r = 0 on the front face (slab 0).

    per_event: int (fixed count) or (lo, hi) for lo + floor((hi-lo+1) U).
    species:   int (fixed) or 'mixed' for floor(3 U).
    e_range:   float (fixed kinetic energy) or (lo, hi) log-uniform.
    cone_deg:  0 for +z, else uniform in solid angle within the cone.
    """
    out = []
    for e in range(first_event, first_event + n_events):
        if isinstance(per_event, tuple):
            lo, hi = per_event
            w = philox_block(seed, e, U64, 0, 0, 2)[0]
            n = lo + min(int(math.floor(unit(w) * (hi - lo + 1))), hi - lo)
        else:
            n = int(per_event)
        for i in range(n):
            w = philox_block(seed, e, i, 0, 0, 2)
            if species == "mixed":
                typ = min(int(math.floor(3.0 * unit(w[1]))), 2)
            else:
                typ = int(species)
            if isinstance(e_range, tuple):
                lo, hi = e_range
                T = lo * (hi / lo) ** unit(w[2])
            else:
                T = float(e_range)
            if cone_deg > 0.0:
                cmin = math.cos(math.radians(cone_deg))
                cost = 1.0 - unit(w[3]) * (1.0 - cmin)
                phi = 2.0 * math.pi * unit(philox_block(seed, e, i, 0, 1, 2)[0])
                sint = math.sqrt(max(0.0, 1.0 - cost * cost))
                u = (sint * math.cos(phi), sint * math.sin(phi), cost)
            else:
                u = (0.0, 0.0, 1.0)
            out.append((e, int(w[0]), typ, 0, T, (0.0, 0.0, 0.0), u))
    return np.array(out, dtype=PRIM_DTYPE)


def small_electron_showers(n_events: int = 1000, seed: int = 1) -> Workload:
    """1000 e- at 10 MeV, 20-layer Pb/LAr stack 10x10 cm, no field, 1 MeV cut, FP64, 4096 slots."""
    st = sampling_stack(20, 10.0)
    return Workload("pb_lar20_e10MeV_cut1MeV", st, 1.0, seed, n_events,
                    make_primaries(seed, n_events, 1, ELECTRON, 10.0), 4096)


def electron_showers_1gev_field(n_events: int = 10000, seed: int = 1, n_slots: int = 1 << 20) -> Workload:
    """1e4 e- at 1 GeV, 50-layer Pb/LAr stack 40x40 cm, 1 T along x, 0.1 MeV cut, FP64, 2^20 slots."""
    st = sampling_stack(50, 40.0, (1.0, 0.0, 0.0))
    return Workload("pb_lar50_e1GeV_B1T_cut0.1MeV", st, 0.1, seed, n_events,
                    make_primaries(seed, n_events, 1, ELECTRON, 1000.0), n_slots)


def mixed_cone_showers(n_events: int = 10000, seed: int = 1, n_slots: int = 1 << 20) -> Workload:
    """1e4 primaries, 1/3 each gamma/e-/e+, log-uniform 100 MeV-10 GeV, 5 degree cone; stack as above."""
    st = sampling_stack(50, 40.0, (1.0, 0.0, 0.0))
    return Workload("pb_lar50_mixed_0.1-10GeV_cone5_B1T", st, 0.1, seed, n_events,
                    make_primaries(seed, n_events, 1, "mixed", (100.0, 10000.0), cone_deg=5.0), n_slots,
                    precision="mixed")


def batched_mixed_events(n_events: int = 64, seed: int = 1, n_slots: int = 1 << 22) -> Workload:
    """64 events of 1-500 mixed primaries, log-uniform 10 MeV-100 GeV, +z; stack as above."""
    st = sampling_stack(50, 40.0, (1.0, 0.0, 0.0))
    return Workload("pb_lar50_64ev_1-500mixed_0.01-100GeV_B1T", st, 0.1, seed, n_events,
                    make_primaries(seed, n_events, (1, 500), "mixed", (10.0, 100000.0)), n_slots)


def lhc_like_events(n_events: int = 16, seed: int = 1, n_slots: int = 1 << 21, per_event: int = 1300,
                    energy_mev: float = 10000.0) -> Workload:
    """16 events of 1300 e- at 10 GeV each (the event size of the paper's benchmark problems: the energy
    an LHC collision deposits), +z; 50-layer stack, 1 T, 0.1 MeV cut, FP64."""
    st = sampling_stack(50, 40.0, (1.0, 0.0, 0.0))
    return Workload(f"pb_lar50_{n_events}ev_{per_event}e{energy_mev / 1000:g}GeV_B1T", st, 0.1, seed, n_events,
                    make_primaries(seed, n_events, per_event, ELECTRON, energy_mev), n_slots)


def poisson_arrival_times(seed: int, rate_hz: float, n: int) -> np.ndarray:
    """Arrival times of n events at Poisson rate: key (seed, 2^64-1), counter (k, 0, 0, 3)."""
    t = 0.0
    out = np.empty(n)
    for k in range(n):
        w = philox_block(seed, U64, k, 0, 0, 3)[0]
        t += -math.log(unit(w)) / rate_hz
        out[k] = t
    return out


def serving_events(n_events: int = 1000, seed: int = 1, per_event=(1, 200), e_range=(10.0, 100000.0),
                   first_event: int = 0) -> Workload:
    """Events of 1-200 mixed primaries, log-uniform 10 MeV-100 GeV, +z; 50-layer stack, 1 T; for Poisson
    arrivals (see poisson_arrival_times)."""
    st = sampling_stack(50, 40.0, (1.0, 0.0, 0.0))
    return Workload("pb_lar50_serving_1-200mixed_0.01-100GeV_B1T", st, 0.1, seed, n_events,
                    make_primaries(seed, n_events, per_event, "mixed", e_range, first_event=first_event),
                    1 << 23, precision="mixed")
