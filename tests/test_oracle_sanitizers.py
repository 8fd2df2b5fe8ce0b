"""The oracle under the CPU sanitizers.

oracle/transport.c is compiled with gcc into a standalone driver
(tests/sanitize/oracle_driver.c) twice: with AddressSanitizer and
UndefinedBehaviorSanitizer, and with ThreadSanitizer (the oracle runs events
on a pthread pool).  Each build transports real showers (1 GeV electrons in
the 1 T stack; 10 MeV electrons without field, with multiple scattering) on
four threads and takes single steps of random states (on planes, near walls,
set and unset interaction lengths).  The run must end cleanly with no
sanitizer report, and its results must be bit-identical to the oracle
library that the other tests load: the sanitizers observe, they do not
change the arithmetic (no FMA contraction, no fast-math, SSE2 doubles).
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_helpers import random_states

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "sanitize", "oracle_driver.c")

SANITIZERS = {
    "address,undefined": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
    "thread": ["-fsanitize=thread"],
}


def _build(tmp_path, name):
    exe = str(tmp_path / ("oracle_" + name.replace(",", "_")))
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fno-fast-math", "-ffp-contract=off",
           *SANITIZERS[name], "-o", exe, DRIVER, "-lm", "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def _write_input(path, pb, prims, rows, n_rows, states, msc, threads):
    s = pb._s
    with open(path, "wb") as f:
        f.write(np.array([pb.n_slabs, len(pb.materials), int(msc), threads], dtype=np.int32).tobytes())
        f.write(np.array([s.half_width, s.B[0], s.B[1], s.B[2], pb.ecut], dtype=np.float64).tobytes())
        f.write(np.array([s.seed, len(prims), len(states)], dtype=np.uint64).tobytes())
        f.write(np.array([n_rows, 0], dtype=np.uint32).tobytes())
        f.write(pb.z_planes.tobytes())
        f.write(pb.slab_material.tobytes())
        f.write(pb.tables.tobytes())
        f.write(pb.x0_cm.tobytes())
        f.write(np.ascontiguousarray(prims, dtype=oracle.TRACK_DTYPE).tobytes())
        f.write(np.ascontiguousarray(rows, dtype=np.uint32).tobytes())
        f.write(np.ascontiguousarray(states, dtype=oracle.TRACK_DTYPE).tobytes())


def _read_output(path, n_rows, n_slabs, n_states):
    b = open(path, "rb").read()
    o = 0
    steps = int(np.frombuffer(b, np.uint64, 1, o)[0]); o += 8
    edep = np.frombuffer(b, np.float64, n_rows * n_slabs, o).reshape(n_rows, n_slabs); o += 8 * n_rows * n_slabs
    led = np.frombuffer(b, oracle.LEDGER_DTYPE, n_rows, o); o += oracle.LEDGER_DTYPE.itemsize * n_rows
    st = np.frombuffer(b, oracle.TRACK_DTYPE, n_states, o); o += oracle.TRACK_DTYPE.itemsize * n_states
    res = np.frombuffer(b, oracle.RESULT_DTYPE, n_states, o); o += oracle.RESULT_DTYPE.itemsize * n_states
    assert o == len(b)
    return steps, edep, led, st, res


CASES = {
    "field_1GeV": lambda: (workloads.electron_showers_1gev_field(4), False),
    "nofield_10MeV_msc": lambda: (workloads.small_electron_showers(40), True),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("san", sorted(SANITIZERS))
def test_oracle_clean_and_identical_under_sanitizers(tmp_path, san, case):
    w, msc = CASES[case]()
    pb = oracle.problem_for(w, msc=msc)
    prims, rows = oracle.tracks_from_primaries(w.primaries)
    states = random_states(w, 3000, np.random.default_rng(5))
    exe = _build(tmp_path, san)
    inp, out = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write_input(inp, pb, prims, rows, w.n_events, states, msc, threads=4)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24",
               TSAN_OPTIONS="halt_on_error=1:exitcode=25")
    r = subprocess.run([exe, inp, out], capture_output=True, text=True, env=env, timeout=600)
    report = r.stderr[-4000:]
    assert r.returncode == 0, report
    for marker in ("AddressSanitizer", "runtime error", "ThreadSanitizer", "LeakSanitizer"):
        assert marker not in r.stderr, report
    steps, edep, led, st_after, res = _read_output(out, w.n_events, pb.n_slabs, len(states))
    e_ref, l_ref, steps_ref = pb.run_events(prims, rows, w.n_events, 4)
    assert steps == steps_ref
    assert np.array_equal(edep, e_ref)
    assert np.array_equal(led, l_ref)
    ref_states = states.copy()
    ref_res = pb.step(ref_states)
    assert np.array_equal(st_after, ref_states)
    assert np.array_equal(res["outcome"], ref_res["outcome"])
    assert np.array_equal(res["edep"], ref_res["edep"])
    assert np.array_equal(res["sec"], ref_res["sec"])
