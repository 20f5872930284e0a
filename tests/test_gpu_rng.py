"""The device Philox4x32-10 (word 0, the word every start and tie decision
reads) against the published known-answer vectors and against the oracle on
random counters in the forms the library uses."""
import numpy as np
import pytest

import oracle
import paper_0912_3912_amd as sg
from test_oracle_philox import kat_vectors

pytestmark = pytest.mark.gpu


def _word0(ctr, seed, gpu):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(ctr, np.uint32).view(np.int32)).to(gpu)
    return sg.philox_word0(t, seed).cpu().numpy().view(np.uint32)


def test_device_philox_known_answers(gpu):
    for ctr, key, want in kat_vectors():
        seed = int(key[0]) | (int(key[1]) << 32)
        got = _word0(ctr[None, :], seed, gpu)
        assert int(got[0]) == int(want[0]), (ctr, key, hex(int(got[0])), hex(int(want[0])))


def test_device_philox_matches_oracle(gpu):
    rng = np.random.default_rng(5)
    for seed in (0, 7, (3 << 32) | 11, 0xFFFFFFFFFFFFFFFF):
        ctr = rng.integers(0, 2**32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
        ctr[:1024, 1] = 0xFFFFFFFF         # start counters
        ctr[1024:2048, 0] &= 0xFFFF        # small spin indices
        got = _word0(ctr, seed, gpu)
        key = np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint32)
        want = np.array([oracle.philox(c, key)[0] for c in ctr], np.uint32)
        assert np.array_equal(got, want)


def test_device_philox_empty(gpu):
    import torch
    t = torch.zeros((0, 4), dtype=torch.int32, device=gpu)
    assert sg.philox_word0(t, 1).numel() == 0
