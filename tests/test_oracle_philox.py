"""Pins of the oracle's Philox4x32-10 (the counter-based generator that draws
every random start and every tie decision; Salmon et al., SC'11) against
values that do not come from this repository:

* the published known-answer vectors (fixture ``golden/philox4x32_10_kat.txt``);
* the engine of rocRAND's source header, compiled here into a small host
  program (``native/rocrand_philox_ref.cpp``) and run on 10^5 random
  (counter, key) pairs plus the all-zero and all-ones inputs.

The oracle itself includes nothing from rocRAND; only this test does.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
KAT = os.path.join(HERE, "golden", "philox4x32_10_kat.txt")
REF_SRC = os.path.join(HERE, "native", "rocrand_philox_ref.cpp")
ROCRAND_HDR = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"


def kat_vectors():
    rows = []
    with open(KAT) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(x, 16) for x in line.split()]
            assert len(v) == 10
            rows.append((np.array(v[0:4], np.uint32), np.array(v[4:6], np.uint32), np.array(v[6:10], np.uint32)))
    return rows


def test_philox_known_answer_vectors():
    rows = kat_vectors()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = oracle.philox(ctr, key)
        assert np.array_equal(got, want), (ctr, key, got, want)


def test_philox_stream_matches_single_calls():
    """The stream helper used by other pins is the same function on consecutive counters."""
    out = oracle.philox_stream((7 << 32) | 5, 0xFFFFFFF0, 3, 2, 1, 40)
    for i in range(40):
        c = np.array([(0xFFFFFFF0 + i) & 0xFFFFFFFF, 3, 2, 1], np.uint32)
        assert np.array_equal(out[i], oracle.philox(c, np.array([5, 7], np.uint32)))


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    cc = _hipcc()
    if cc is None or not os.path.exists(ROCRAND_HDR):
        pytest.skip("hipcc or the rocRAND source header is not available")
    exe = str(tmp_path_factory.mktemp("rocrand") / "philox_ref")
    subprocess.check_call([cc, "-O2", "--offload-arch=gfx950", "-I/opt/rocm/include", REF_SRC, "-o", exe])

    def run(inputs):
        d = tmp_path_factory.mktemp("io")
        fi, fo = str(d / "in.bin"), str(d / "out.bin")
        np.ascontiguousarray(inputs, np.uint32).tofile(fi)
        subprocess.check_call([exe, fi, fo])
        return np.fromfile(fo, dtype=np.uint32).reshape(-1, 4)

    return run


def test_rocrand_engine_reproduces_known_answers(rocrand_ref):
    rows = kat_vectors()
    inp = np.stack([np.concatenate([c, k]) for c, k, _ in rows])
    out = rocrand_ref(inp)
    for (c, k, want), got in zip(rows, out):
        assert np.array_equal(got, want)


def test_philox_matches_rocrand_on_random_inputs(rocrand_ref):
    rng = np.random.default_rng(20240611)
    n = 100_000
    inp = rng.integers(0, 2**32, size=(n, 6), dtype=np.uint64).astype(np.uint32)
    # the counter forms the library uses: (spin, sweep or 0xFFFFFFFF, instance, restart)
    inp[: n // 4, 1] = 0xFFFFFFFF
    inp[n // 4: n // 2, 0] &= 0xFFFFF
    inp = np.concatenate([inp, np.zeros((1, 6), np.uint32), np.full((1, 6), 0xFFFFFFFF, np.uint32)])
    ref = rocrand_ref(inp)
    lib = oracle._load()
    got = np.zeros((inp.shape[0], 4), np.uint32)
    c = np.zeros(4, np.uint32)
    k = np.zeros(2, np.uint32)
    o = np.zeros(4, np.uint32)
    pc, pk, po = oracle._p(c), oracle._p(k), oracle._p(o)
    for i in range(inp.shape[0]):
        c[:] = inp[i, :4]
        k[:] = inp[i, 4:]
        lib.oracle_philox4x32_10(pc, pk, po)
        got[i] = o
    bad = np.nonzero(np.any(got != ref, axis=1))[0]
    assert bad.size == 0, f"{bad.size} mismatches, first at input {inp[bad[0]]}"
