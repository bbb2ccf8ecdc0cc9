"""Philox4x32-10 counter-based generator and the Gaussian sketch matrices.

The paper draws a Gaussian random matrix inside each randomized factorization
(Alg. 1 and Alg. 3, "Draw a Gaussian random matrix").  To let an independent
implementation reproduce exactly the same draws, the sketch matrix Omega_j of
slice j is keyed by a counter instead of a stateful stream:

  * generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
    numbers: as easy as 1, 2, 3", SC'11), written here from that definition;
  * key   = (seed mod 2^32, seed div 2^32);
  * counter = (g, slice, call, stream) where element e of Omega_j (column-major,
    e = i + n2*c) lives in group g = e // 4, lane e % 4;
  * uniforms u = (x + 1/2) * 2^-32 from each 32-bit word (never 0 or 1);
  * Box-Muller on word pairs: (x0, x1) -> r cos(t), r sin(t) and (x2, x3) ->
    r' cos(t'), r' sin(t'), r = sqrt(-2 ln u_a), t = 2 pi u_b.

Pins: the Philox known-answer vectors (tests/golden/philox4x32_10_kat.txt) and
the normality / independence statistics in the oracle tests.
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_TWO_PI = 6.283185307179586


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds on arrays of 32-bit counters (as uint64 holders).

    One round: the products M0*c0 and M1*c2 are split in high and low halves;
    the new counter is (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0).  The key is
    bumped by the Weyl constants between rounds.
    """
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & _MASK for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def uniforms_from_words(x):
    """Map 32-bit words to doubles in (0, 1): (x + 1/2) / 2^32 (exact in FP64)."""
    return (np.asarray(x, dtype=np.float64) + 0.5) * (1.0 / 4294967296.0)


def gaussian_block(n_elems, slice_id, call_id, stream_id, seed):
    """The first n_elems N(0,1) draws of one (slice, call, stream) key, in FP64."""
    n_groups = (n_elems + 3) // 4
    g = np.arange(n_groups, dtype=np.uint64)
    seed = int(seed)
    w = philox4x32_10(g, np.uint64(slice_id), np.uint64(call_id), np.uint64(stream_id),
                      np.uint64(seed & 0xFFFFFFFF), np.uint64((seed >> 32) & 0xFFFFFFFF))
    u = [uniforms_from_words(x) for x in w]
    r01 = np.sqrt(-2.0 * np.log(u[0]))
    r23 = np.sqrt(-2.0 * np.log(u[2]))
    t01 = _TWO_PI * u[1]
    t23 = _TWO_PI * u[3]
    z = np.empty((n_groups, 4), dtype=np.float64)
    z[:, 0] = r01 * np.cos(t01)
    z[:, 1] = r01 * np.sin(t01)
    z[:, 2] = r23 * np.cos(t23)
    z[:, 3] = r23 * np.sin(t23)
    return z.reshape(-1)[:n_elems]


def omega(n2, l, slice_id, call_id=0, stream_id=0, seed=0):
    """Omega_j in R^{n2 x l}, column-major element order e = i + n2*c."""
    z = gaussian_block(n2 * l, slice_id, call_id, stream_id, seed)
    return z.reshape((n2, l), order="F")
