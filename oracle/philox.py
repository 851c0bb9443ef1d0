"""Philox4x64-10 counter-based generator, written from its published definition.

TEST INFRASTRUCTURE ONLY: this package is the FP64 CPU oracle.  Only the tests,
the smoke check and the CPU-baseline leg of the benchmark may import it.

Definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11, section 4 and table 2): the 256-bit counter (c0, c1, c2, c3)
and the 128-bit key (k0, k1) go through ten rounds.  One round replaces the
counter by

    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))

where hi/lo are the upper/lower 64-bit halves of the 128-bit product; between
rounds the key is bumped by the Weyl constants (W0, W1) modulo 2**64.

Pinned by tests against numpy's own Philox4x64-10 bit generator.
"""

MASK64 = (1 << 64) - 1

# multipliers and Weyl key increments of Philox4x64 (SC'11, table 2)
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15   # golden ratio
PHILOX_W1 = 0xBB67AE8584CAA73B   # sqrt(3) - 1


def philox4x64(counter, key, rounds=10):
    """Return the four 64-bit outputs of Philox4x64-`rounds` for one counter.

    counter: 4 ints in [0, 2**64); key: 2 ints in [0, 2**64).
    """
    c0, c1, c2, c3 = (int(c) & MASK64 for c in counter)
    k0, k1 = (int(k) & MASK64 for k in key)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return (c0, c1, c2, c3)


def u01(x):
    """Map a 64-bit word to a double in [0, 1) from its top 53 bits."""
    return float(int(x) >> 11) * (2.0 ** -53)
