"""Counter-based random stream of the oracle.

The paper draws its random numbers with gsl (Sec. 5.1) and fixes no stream.
The reading taken here is a counter-based stream so that every path of every
knot is reproducible independently of scheduling: Philox4x32-10 (Salmon,
Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11),

    key     = (seed mod 2^32, seed div 2^32)
    counter = (draw j, path p, knot k, instance i)

One call yields four 32-bit words r0..r3.  Each word becomes a uniform in
(0, 1) and two uniforms become two standard normals by the Box-Muller
transform; draw j therefore feeds the two Brownian increments of Euler steps
2j (from r0, r1) and 2j+1 (from r2, r3).

All arithmetic is NumPy: uint64 for the 32x32->64 bit products, float64 for
the uniforms and normals.
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)
_SHIFT = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds on arrays of counters.

    c0..c3: integer arrays (broadcastable) holding 32-bit counter words.
    k0, k1: Python ints, the two 32-bit key words.
    Returns four uint64 arrays holding the 32-bit output words.

    Round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 (full 64-bit products),
    new counter = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); between rounds the
    key is bumped by the Weyl constants (W0, W1) modulo 2^32.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK
    c2 = np.asarray(c2, dtype=np.uint64) & _MASK
    c3 = np.asarray(c3, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    key0 = int(k0) & 0xFFFFFFFF
    key1 = int(k1) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd > 0:
            key0 = (key0 + _W0) & 0xFFFFFFFF
            key1 = (key1 + _W1) & 0xFFFFFFFF
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _SHIFT, p0 & _MASK
        hi1, lo1 = p1 >> _SHIFT, p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(key0), lo1,
                          hi0 ^ c3 ^ np.uint64(key1), lo0)
    return c0, c1, c2, c3


def seed_key(seed):
    """Split a 64-bit seed into the two Philox key words (low word first)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def uniform_fp64(r):
    """Map a 32-bit word r to the open interval (0, 1): u = (r + 1/2) 2^-32.

    Exact in float64; never 0 or 1, so log(u) is finite.
    """
    return (np.asarray(r, dtype=np.float64) + 0.5) * 2.0 ** -32


def box_muller(u0, u1):
    """Two independent N(0,1) samples from two uniforms:
    rho = sqrt(-2 ln u0), theta = 2 pi u1, returns (rho cos theta, rho sin theta)."""
    rho = np.sqrt(-2.0 * np.log(u0))
    theta = 2.0 * np.pi * u1
    return rho * np.cos(theta), rho * np.sin(theta)


def normals_for_draw(j, path, knot, instance, seed):
    """Brownian normals of Euler steps 2j and 2j+1 for the given paths.

    Returns ((xi_x, xi_y) of step 2j, (xi_x, xi_y) of step 2j+1), each an array
    shaped like ``path``.  ``j``, ``knot`` and ``instance`` broadcast.
    """
    k0, k1 = seed_key(seed)
    r0, r1, r2, r3 = philox4x32_10(j, path, knot, instance, k0, k1)
    a = box_muller(uniform_fp64(r0), uniform_fp64(r1))
    b = box_muller(uniform_fp64(r2), uniform_fp64(r3))
    return a, b
