"""Philox4x64-10 counter-based generator (oracle side).

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.

Written from the published definition of the Philox family (Salmon, Moraes,
Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11, Sec. 5 and
Table 2): a 4-word, 64-bit-lane counter is pushed through 10 rounds of
  (x0, x1, x2, x3) -> (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1, lo(M0*x0))
with the 2-word key bumped by the Weyl increments (W0, W1) between rounds.

The paper under study only says that the Hubbard-Stratonovich field is sampled
by Monte Carlo; it fixes no generator.  A counter-based generator makes every
uniform a pure function of (seed, grid, chain, sweep, slice), so the GPU path
and this oracle consume the same stream without sharing code.

Stream layout used by the whole method (see ``uniform``):
  key     = (seed + chain, grid_id)
  counter = (slice l, sweep, 0, stream)     stream 0: acceptance, 1: initial field
  u       = (x0 >> 11) * 2**-53              (53-bit uniform in [0, 1))

Pinned against ``numpy.random.Philox`` (an independent implementation of the
same published generator) in tests/test_oracle_philox.py.
"""
import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1
ROUNDS = 10


def philox4x64_scalar(ctr, key, rounds=ROUNDS):
    """Reference Philox4x64 on Python integers: ctr = 4 ints, key = 2 ints."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in ctr)
    k0, k1 = (int(k) & MASK64 for k in key)
    for r in range(rounds):
        if r:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo64(a, b):
    """Full 64x64 -> 128-bit product of uint64 arrays, via 32-bit halves."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _LO32, a >> _S32
    b_lo, b_hi = b & _LO32, b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _LO32) + (hl & _LO32)
    lo = (ll & _LO32) | ((mid & _LO32) << _S32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1, rounds=ROUNDS):
    """Vectorised Philox4x64 over broadcastable uint64 arrays."""
    with np.errstate(over="ignore"):
        x0 = np.asarray(c0, dtype=np.uint64)
        x1 = np.asarray(c1, dtype=np.uint64)
        x2 = np.asarray(c2, dtype=np.uint64)
        x3 = np.asarray(c3, dtype=np.uint64)
        k0 = np.asarray(k0, dtype=np.uint64)
        k1 = np.asarray(k1, dtype=np.uint64)
        m0, m1 = np.uint64(M0), np.uint64(M1)
        w0, w1 = np.uint64(W0), np.uint64(W1)
        for r in range(rounds):
            if r:
                k0 = k0 + w0
                k1 = k1 + w1
            hi0, lo0 = _mulhilo64(m0, x0)
            hi1, lo1 = _mulhilo64(m1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


STREAM_ACCEPT = 0
STREAM_INIT = 1


def uniform(seed, chain, grid_id, sweep, sl, stream):
    """53-bit uniforms in [0, 1) for the method's stream layout (broadcasts)."""
    with np.errstate(over="ignore"):
        k0 = np.uint64(seed) + np.asarray(chain, dtype=np.uint64)
    x0, _, _, _ = philox4x64(sl, sweep, 0, stream, k0, grid_id)
    return (x0 >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def sweep_uniforms(seed, chain, grid_id, sweep, L):
    """Acceptance uniforms for slices 0..L-1 of one sweep."""
    return uniform(seed, chain, grid_id, sweep, np.arange(L, dtype=np.uint64), STREAM_ACCEPT)


def initial_field(seed, chain, grid_id, L):
    """Initial auxiliary field: s_l = +1 if u < 1/2 else -1 (stream 1, sweep 0)."""
    u = uniform(seed, chain, grid_id, 0, np.arange(L, dtype=np.uint64), STREAM_INIT)
    return np.where(u < 0.5, 1, -1).astype(np.int8)
