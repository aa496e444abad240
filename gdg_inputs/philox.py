"""Philox4x32-10 counter-based generator and the seeded shot sampler.

Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3" (SC'11): a 4x32-bit counter and a 2x32-bit key,
ten rounds of two 32x32->64 multiplies with the key bumped by the Weyl
constants between rounds.

Shot sampling (input generation, shared by every consumer of the shots):
column c of shot s fires iff word (c mod 4) of
philox(counter=(c div 4, s, stream, 0xC0DE), key=(seed_lo, seed_hi)) is below
the column's uint32 threshold floor(p_c * 2^32). Integer comparisons only, so a
device implementation reproduces the same shots bit for bit.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
SAMPLE_TAG = 0xC0DE


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10. All inputs broadcastable uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint32)
    c1 = np.asarray(c1, dtype=np.uint32)
    c2 = np.asarray(c2, dtype=np.uint32)
    c3 = np.asarray(c3, dtype=np.uint32)
    k0 = np.asarray(k0, dtype=np.uint32)
    k1 = np.asarray(k1, dtype=np.uint32)
    c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(c0, c1, c2, c3, k0, k1)
    c0 = c0.copy(); c1 = c1.copy(); c2 = c2.copy(); c3 = c3.copy()
    k0 = k0.copy(); k1 = k1.copy()
    with np.errstate(over="ignore"):
        return _rounds(c0, c1, c2, c3, k0, k1)


def _rounds(c0, c1, c2, c3, k0, k1):
    for r in range(10):
        p0 = c0.astype(np.uint64) * M0
        p1 = c2.astype(np.uint64) * M1
        hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
        lo0 = (p0 & MASK).astype(np.uint32)
        hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
        lo1 = (p1 & MASK).astype(np.uint32)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        if r < 9:
            k0 = k0 + W0
            k1 = k1 + W1
    return c0, c1, c2, c3


def sample_errors(thresholds: np.ndarray, n_shots: int, seed: int, stream: int = 0,
                  shot0: int = 0) -> np.ndarray:
    """Fault vectors e[shot, column] (uint8 0/1) for shots shot0..shot0+n_shots-1."""
    thr = np.asarray(thresholds, dtype=np.uint32)
    n = thr.size
    ngroups = (n + 3) // 4
    k0 = np.uint32(seed & 0xFFFFFFFF)
    k1 = np.uint32((seed >> 32) & 0xFFFFFFFF)
    shots = (np.arange(n_shots, dtype=np.uint64) + np.uint64(shot0)).astype(np.uint32)
    grp = np.arange(ngroups, dtype=np.uint32)
    out = np.zeros((n_shots, ngroups * 4), dtype=np.uint8)
    chunk = max(1, (1 << 22) // max(ngroups, 1))
    for s0 in range(0, n_shots, chunk):
        sh = shots[s0:s0 + chunk][:, None]
        r = philox4x32_10(grp[None, :], sh, np.uint32(stream), np.uint32(SAMPLE_TAG),
                          k0, k1)
        u = np.stack(r, axis=-1).reshape(sh.shape[0], ngroups * 4)
        out[s0:s0 + chunk] = u < np.concatenate([thr, np.zeros(ngroups * 4 - n,
                                                                 np.uint32)])[None, :]
    return out[:, :n]


def syndromes(dem, errors: np.ndarray):
    """Detector values H_circ e and observables L e (mod 2) for fault vectors."""
    e = np.asarray(errors, dtype=np.uint8)
    n_shots = e.shape[0]
    det = np.zeros((n_shots, dem.n_rows), dtype=np.uint8)
    obs = np.zeros((n_shots, dem.n_obs), dtype=np.uint8)
    shots, cols = np.nonzero(e)
    for s, c in zip(shots.tolist(), cols.tolist()):
        det[s, dem.col_rows(c)] ^= 1
        ob = dem.col_obs(c)
        if ob.size:
            obs[s, ob] ^= 1
    return det, obs
