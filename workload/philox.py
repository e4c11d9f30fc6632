"""Counter-based random numbers shared by the synthetic workload generator.

Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11): a 128-bit counter and a 64-bit key are mapped through ten
rounds of two 32x32->64 multiplies, xors with the key and a Weyl key schedule.
Any element of a synthetic tensor can be regenerated alone from
(seed, field, stream, index), which is what lets a CPU checker rebuild a few
pairs of a workload that only the GPU holds whole.

Normals are Irwin-Hall sums of the four 32-bit outputs of one counter:
    z = ((u0 + u1 + u2 + u3) - 2**33) * 2**-32 * sqrt(3)
The integer sum and the power-of-two scaling are exact; the two multiplies
(by sqrt(3), then by the tensor scale) are single IEEE roundings, so the same
bits come out of this file and of the HIP generator.  The distribution has
unit variance and bounded support |z| <= 2*sqrt(3).

This module holds no arithmetic of the DLPNO method.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)
SQRT3 = float(np.sqrt(np.float64(3.0)))
TWO_M32 = 2.0 ** -32
KEY_HI_SALT = 0x5EED0DF1


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on vectors of 32-bit counter words (any integer dtype).

    Returns four uint64 arrays holding 32-bit values."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    c0, c1, c2, c3 = c0.copy(), c1.copy(), c2.copy(), c3.copy()
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for r in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
        if r < 9:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
    return c0, c1, c2, c3


def key_of(seed):
    seed = int(seed)
    return seed & 0xFFFFFFFF, (KEY_HI_SALT ^ (seed >> 32)) & 0xFFFFFFFF


def normals(seed, field, stream, index):
    """Irwin-Hall(4) unit normals for counters (index_lo, index_hi, stream, field)."""
    index = np.asarray(index, dtype=np.uint64)
    k0, k1 = key_of(seed)
    u0, u1, u2, u3 = philox4x32_10(index & MASK32, index >> np.uint64(32),
                                   np.asarray(stream, dtype=np.uint64), field, k0, k1)
    s = (u0 + u1 + u2 + u3).astype(np.int64) - (1 << 33)
    return (s.astype(np.float64) * TWO_M32) * SQRT3


def uniforms(seed, field, stream, index):
    """Uniforms in [0, 1) from the first 32-bit word: u0 * 2**-32."""
    index = np.asarray(index, dtype=np.uint64)
    k0, k1 = key_of(seed)
    u0, _, _, _ = philox4x32_10(index & MASK32, index >> np.uint64(32),
                                np.asarray(stream, dtype=np.uint64), field, k0, k1)
    return u0.astype(np.float64) * TWO_M32
