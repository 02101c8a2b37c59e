"""Philox-4x32-10 counter-based generator and Box-Muller normals (oracle).

Philox-4x32 as published by Salmon, Moraes, Dror & Shaw (2011), "Parallel
random numbers: as easy as 1, 2, 3" (SC'11): a 4-word counter and 2-word
key; each of 10 rounds multiplies counter words 0 and 2 by the constants
0xD2511F53 and 0xCD9E8D57, splits the 64-bit products into high and low
halves, and recombines
    (hi(M1 c2) ^ c1 ^ k0,  lo(M1 c2),  hi(M0 c0) ^ c3 ^ k1,  lo(M0 c0));
between rounds the key is bumped by the Weyl constants 0x9E3779B9 and
0xBB67AE85 (mod 2^32).

HMC momenta (Sec. 4.2, App. B: p ~ N(0, M)) are drawn from this stream so
that a chain's trajectory is reproducible from (seed, trajectory index)
alone.  Normal variates use the Box-Muller transform (Box & Muller 1958):
u = (x + 1/2) 2^-32 for a 32-bit word x; r = sqrt(-2 ln u1);
z = (r cos 2 pi u2, r sin 2 pi u2).
"""
from __future__ import annotations

import math
from typing import Sequence, Tuple

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> Tuple[int, int, int, int]:
    c = [int(x) & MASK for x in ctr]
    k0, k1 = int(key[0]) & MASK, int(key[1]) & MASK
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & MASK, p1 & MASK,
             ((p0 >> 32) ^ c[3] ^ k1) & MASK, p0 & MASK]
    return c[0], c[1], c[2], c[3]


def unit_open(x: int) -> float:
    """(x + 1/2) / 2^32, strictly inside (0, 1)."""
    return (x + 0.5) * 2.0 ** -32


def normals(n: int, seed: int, stream: int, traj: int, purpose: int = 0) -> np.ndarray:
    """n standard normals; block k uses counter (k, traj, stream, purpose), key
    (seed lo, seed hi).  Purpose 0 draws HMC momenta; purpose 5 draws the probe
    vectors of the Hutchinson mass-matrix estimate (``traj`` = probe index)."""
    key = (seed & MASK, (seed >> 32) & MASK)
    out = np.empty(4 * ((n + 3) // 4))
    for k in range(len(out) // 4):
        x = philox4x32_10((k, traj, stream, purpose), key)
        for h in range(2):
            u1, u2 = unit_open(x[2 * h]), unit_open(x[2 * h + 1])
            r = math.sqrt(-2.0 * math.log(u1))
            out[4 * k + 2 * h] = r * math.cos(2.0 * math.pi * u2)
            out[4 * k + 2 * h + 1] = r * math.sin(2.0 * math.pi * u2)
    return out[:n]


def accept_uniform(seed: int, stream: int, traj: int) -> float:
    """The Metropolis uniform of one trajectory: word 0 of counter (0xFFFFFFFF, traj, stream, 1)."""
    key = (seed & MASK, (seed >> 32) & MASK)
    x = philox4x32_10((MASK, traj, stream, 1), key)
    return unit_open(x[0])
