"""pic_philox_noalloc (no device allocation, fixed device staging) against
pic_philox on the same counters: bit-identical words, on two calls in a row,
the second smaller; sizes beyond the staging capacity are rejected."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_philox_noalloc_matches_philox(gpu_lib):
    print("\n[gpu-case] pic_philox_noalloc vs pic_philox", flush=True)
    rng = np.random.default_rng(77)
    key = np.array([0x01234567, 0x89ABCDEF], dtype=np.uint32)
    for n in (65536, 1000):
        ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
        a = gpu_lib.pic_philox_noalloc(ctr, key)
        b = gpu_lib.pic_philox(ctr, key)
        assert np.array_equal(a, b), n
        assert a.any()


def test_philox_noalloc_rejects_oversize(gpu_lib):
    print("\n[gpu-case] pic_philox_noalloc oversize", flush=True)
    ctr = np.zeros((65537, 4), dtype=np.uint32)
    with pytest.raises(gpu_lib.PicError) as e:
        gpu_lib.pic_philox_noalloc(ctr, np.zeros(2, dtype=np.uint32))
    assert "exceeds the staging capacity" in str(e.value)
