"""Philox4x32-10 counter-based generator, written from its published definition
(J. Salmon, M. Moraes, R. Dror, D. Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11, Sec. 4: the Philox-4x32 S-box with two 32x32->64 multiplies
per round, Weyl key schedule, 10 rounds).

The paper being implemented does not specify its random numbers.  The reading
adopted for the whole method is a stateless stream:

    key     = (seed & 0xffffffff, seed >> 32)
    counter = (c0, c1, c2, c3), 32-bit words
    u       = (x + 0.5) * 2**-32  in float64, x one 32-bit output word

so u lies strictly inside (0, 1).  The counter layout used by the sampler and
the MH step lives in those modules.

Test infrastructure only (see the package docstring).
Pinned by tests/test_oracle_philox.py against rocRAND's Philox4x32-10 engine
compiled and run on the host (an independent implementation).
"""
import numpy as np

# Round multipliers and Weyl key increments of Philox4x32 (Salmon et al., Table 2
# and Sec. 4.2).
_MUL0 = np.uint64(0xD2511F53)
_MUL1 = np.uint64(0xCD9E8D57)
_WEYL0 = np.uint64(0x9E3779B9)
_WEYL1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_SHIFT = np.uint64(32)


def philox4x32_10(counter, key):
    """Apply the 10-round Philox4x32 bijection.

    counter: integer array [..., 4] (values < 2**32)
    key:     integer array [..., 2] (values < 2**32), broadcast against counter
    returns: uint64 array [..., 4] holding the four 32-bit output words
    """
    ctr = np.asarray(counter, dtype=np.uint64) & _MASK
    k = np.asarray(key, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = ctr[..., 0], ctr[..., 1], ctr[..., 2], ctr[..., 3]
    k0, k1 = k[..., 0], k[..., 1]
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + _WEYL0) & _MASK
            k1 = (k1 + _WEYL1) & _MASK
        p0 = _MUL0 * c0            # full 64-bit product of two 32-bit words
        p1 = _MUL1 * c2
        hi0, lo0 = p0 >> _SHIFT, p0 & _MASK
        hi1, lo1 = p1 >> _SHIFT, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=-1)


def seed_key(seed):
    """Split a 64-bit seed into the two 32-bit key words."""
    seed = int(seed)
    return np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)


def to_uniform(x):
    """Map a 32-bit word to (x + 1/2) / 2**32, strictly inside (0, 1)."""
    return (np.asarray(x, dtype=np.float64) + 0.5) * (2.0 ** -32)
