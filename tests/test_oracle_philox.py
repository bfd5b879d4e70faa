"""Pins of the oracle's generic Philox to numpy's independent Philox4x64-10
(same round structure and key schedule); 4x32 output statistics."""

import numpy as np
import pytest

from oracle import philox as ph


@pytest.mark.parametrize("key,ctr", [((1, 2), (5, 0, 0, 0)), ((0, 0), (0, 0, 0, 0)),
                                     ((0xDEADBEEF12345678, 0x0123456789ABCDEF),
                                      (2 ** 64 - 2, 7, 2 ** 63 + 11, 99))])
def test_philox4x64_matches_numpy(key, ctr):
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
    ref = bg.random_raw(8)
    # numpy increments the 256-bit counter before each block
    c1 = list(ctr)
    out = []
    for _ in range(2):
        carry = 1
        for i in range(4):
            v = c1[i] + carry
            c1[i] = v % 2 ** 64
            carry = v // 2 ** 64
        out += [int(w) for w in ph.philox4(c1, key, ph.PHILOX_4x64)]
    assert out == [int(r) for r in ref]


def test_philox4x32_vectorised_equals_scalar_and_is_uniform():
    ids = np.arange(200000, dtype=np.uint64) * 7919 + 13
    w = ph.draw32(12345, ids, 17, ph.PURPOSE_IONIZE)
    for j in (0, 1, 77, 199999):
        s = ph.philox4([int(ids[j]) & 0xFFFFFFFF, int(ids[j]) >> 32, 17, ph.PURPOSE_IONIZE],
                       [12345, 0], ph.PHILOX_4x32)
        assert [int(x) for x in s] == [int(w[i][j]) for i in range(4)]
    # chi^2 uniformity of the top 8 bits of every word (255 dof, 5-sigma band)
    for i in range(4):
        h = np.bincount((w[i] >> np.uint64(24)).astype(np.int64), minlength=256)
        e = len(ids) / 256
        chi2 = np.sum((h - e) ** 2 / e)
        assert abs(chi2 - 255) < 5 * np.sqrt(2 * 255)
    # different purposes / steps give unrelated streams
    w2 = ph.draw32(12345, ids, 18, ph.PURPOSE_IONIZE)
    assert np.mean(w[0] == w2[0]) < 1e-3
