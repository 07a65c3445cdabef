"""Counter-based noise selection (oracle side).

The forecast's model noise V (Sec. 3.1.2: a zero-mean Gaussian vector with
covariance Sigma_v per member) is read from a bank of precomputed periodic
noise screens.  Which screen, shift and orientation each member uses at each
frame is drawn by Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11), implemented here from its published
definition: ten rounds of two 32x32->64-bit multiplies with multipliers
0xD2511F53 and 0xCD9E8D57, the output words permuted and xored with the key,
and the key bumped by the Weyl constants 0x9E3779B9 and 0xBB67AE85 between
rounds.

Selection rule for (seed, instance, frame, member), 64-bit seed split into the
key (low word, high word), counter (frame, member, instance, 0):
  r0..r3 = Philox4x32-10(counter, key)
  screen = r0 mod n_screens,  oy = r1 mod S,  ox = r2 mod S,  o = r3 mod 8
  node (i, j): (u, v) = (i, j), swapped when o & 1, u negated when o & 2,
  v negated when o & 4; value = bank[screen, (oy + u) mod S, (ox + v) mod S].
S must be a power of two and at least N + 1.
"""
from __future__ import annotations

import numpy as np

_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block.  ctr: 4 ints, key: 2 ints -> 4 ints."""
    c0, c1, c2, c3 = (int(x) & _MASK for x in ctr)
    k0, k1 = (int(x) & _MASK for x in key)
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> 32, p0 & _MASK
        hi1, lo1 = p1 >> 32, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def member_draw(seed: int, instance: int, frame: int, member: int, n_screens: int,
                side: int):
    """(screen, oy, ox, orientation) for one member at one frame."""
    key = (seed & _MASK, (seed >> 32) & _MASK)
    r = philox4x32_10((frame, member, instance, 0), key)
    return r[0] % n_screens, r[1] % side, r[2] % side, r[3] % 8


def bank_noise(bank: np.ndarray, node_coords: np.ndarray, m: int, seed: int,
               instance: int, frame: int) -> np.ndarray:
    """V (n, m) for one frame: column j is member j's draw from the bank."""
    bank = np.asarray(bank)
    n_screens, side = bank.shape[0], bank.shape[1]
    i = node_coords[:, 0].astype(np.int64)
    j = node_coords[:, 1].astype(np.int64)
    V = np.empty((len(i), m), dtype=np.float64)
    for mem in range(m):
        s, oy, ox, o = member_draw(seed, instance, frame, mem, n_screens, side)
        u, v = (j, i) if o & 1 else (i, j)
        if o & 2:
            u = -u
        if o & 4:
            v = -v
        V[:, mem] = bank[s, (oy + u) % side, (ox + v) % side]
    return V
