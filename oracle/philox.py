"""Philox counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11), written generically over the word width.

TEST INFRASTRUCTURE (part of the oracle).  One generic implementation serves
both widths: Philox4x64-10 is pinned against numpy's independent Philox bit
generator (tests/test_oracle_philox.py), which fixes the round structure (the
multiply-high/low pairs, the xor with the key and the word permutation) and the
key schedule; Philox4x32-10, the width the method draws from, is the same code
with the 32-bit constants published in the same paper.

Counter layout used by the method (one block of four 32-bit words per draw):
counter = (id_lo, id_hi, step, purpose), key = (seed_lo, seed_hi).
"""

import numpy as np

_M32 = np.uint64(0xFFFFFFFF)

# Multipliers and Weyl key increments from the Philox paper.
PHILOX_4x32 = dict(W=32, M0=0xD2511F53, M1=0xCD9E8D57, K0=0x9E3779B9, K1=0xBB67AE85)
PHILOX_4x64 = dict(W=64, M0=0xD2E7470EE14C6C93, M1=0xCA5A826395121157,
                   K0=0x9E3779B97F4A7C15, K1=0xBB67AE8584CAA73B)

# Purposes of the method's draws (fourth counter word).
PURPOSE_POS = 1      # initial neutral offsets
PURPOSE_VEL = 2      # thermal velocity of a neutral (handed to its children)
PURPOSE_IONIZE = 3   # ionization decision
PURPOSE_STRESS_E = 4  # pre-ionized stress variant: electron velocity
PURPOSE_STRESS_P = 5  # pre-ionized stress variant: positive-carrier velocity
PURPOSE_TRACK = 6     # trajectory sampling: whether a particle's track is recorded


def _mulhilo(a, b, W):
    """Full product of two W-bit words -> (hi, lo), numpy uint64 arrays."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    if W == 32:
        p = a * b
        return p >> np.uint64(32), p & _M32
    a0, a1 = a & _M32, a >> np.uint64(32)
    b0, b1 = b & _M32, b >> np.uint64(32)
    with np.errstate(over="ignore"):
        p00 = a0 * b0
        p01 = a0 * b1
        p10 = a1 * b0
        p11 = a1 * b1
        mid = (p00 >> np.uint64(32)) + (p01 & _M32) + (p10 & _M32)
        lo = (p00 & _M32) | ((mid & _M32) << np.uint64(32))
        hi = p11 + (p01 >> np.uint64(32)) + (p10 >> np.uint64(32)) + (mid >> np.uint64(32))
    return hi, lo


def philox4(counter, key, params, rounds=10):
    """Philox-4xW-R block function.

    counter: sequence of 4 arrays (or ints) of W-bit words; key: 2 words.
    Returns a list of 4 uint64 arrays holding the W-bit output words.
    """
    W = params["W"]
    mask = np.uint64((1 << W) - 1)
    x = [np.asarray(c, dtype=np.uint64) & mask for c in counter]
    k0 = np.asarray(key[0], dtype=np.uint64) & mask
    k1 = np.asarray(key[1], dtype=np.uint64) & mask
    M0, M1 = np.uint64(params["M0"]), np.uint64(params["M1"])
    K0, K1 = np.uint64(params["K0"]), np.uint64(params["K1"])
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r > 0:
                k0 = (k0 + K0) & mask
                k1 = (k1 + K1) & mask
            hi0, lo0 = _mulhilo(M0, x[0], W)
            hi1, lo1 = _mulhilo(M1, x[2], W)
            x = [(hi1 ^ x[1] ^ k0) & mask, lo1 & mask, (hi0 ^ x[3] ^ k1) & mask, lo0 & mask]
    return x


def draw32(seed, pid, step, purpose):
    """Four 32-bit words for particle ids ``pid`` (array) at ``step``/``purpose``."""
    pid = np.asarray(pid, dtype=np.uint64)
    seed = int(seed)
    ctr = [pid & _M32, pid >> np.uint64(32),
           np.full(pid.shape, step, dtype=np.uint64),
           np.full(pid.shape, purpose, dtype=np.uint64)]
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    return philox4(ctr, key, PHILOX_4x32)
