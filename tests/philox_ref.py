"""Independent Philox4x32-10 in Python, used only to pin the C reference.

Written from the published definition (Salmon et al., "Parallel random
numbers: as easy as 1, 2, 3", SC'11): a 4-word counter and 2-word key; each
of the ten rounds forms the 64-bit products of counter words 0 and 2 with two
fixed multipliers, then the new counter is
  (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0)),
and the key is bumped by the two Weyl constants between rounds.

Two forms: ``philox_int`` on Python integers (one call) and ``philox_np`` on
numpy uint64 arrays (many calls at once).
"""
import numpy as np

MULT = (0xD2511F53, 0xCD9E8D57)
WEYL = (0x9E3779B9, 0xBB67AE85)
MASK32 = 0xFFFFFFFF


def philox_int(ctr, key, rounds=10):
    c = [int(w) & MASK32 for w in ctr]
    k = [int(w) & MASK32 for w in key]
    for r in range(rounds):
        if r:
            k = [(k[0] + WEYL[0]) & MASK32, (k[1] + WEYL[1]) & MASK32]
        prod_a = MULT[0] * c[0]
        prod_b = MULT[1] * c[2]
        c = [((prod_b >> 32) ^ c[1] ^ k[0]) & MASK32, prod_b & MASK32,
             ((prod_a >> 32) ^ c[3] ^ k[1]) & MASK32, prod_a & MASK32]
    return c


def philox_np(c0, c1, c2, c3, k0, k1, rounds=10):
    """Vectorised form; all arguments broadcastable uint64 arrays holding 32-bit words."""
    m = np.uint64(MASK32)
    s32 = np.uint64(32)
    c0, c1, c2, c3 = (np.asarray(a, dtype=np.uint64) & m for a in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & m
    k1 = np.asarray(k1, dtype=np.uint64) & m
    for r in range(rounds):
        if r:
            k0 = (k0 + np.uint64(WEYL[0])) & m
            k1 = (k1 + np.uint64(WEYL[1])) & m
        pa = np.uint64(MULT[0]) * c0
        pb = np.uint64(MULT[1]) * c2
        c0, c1, c2, c3 = ((pb >> s32) ^ c1 ^ k0, pb & m, (pa >> s32) ^ c3 ^ k1, pa & m)
    return c0, c1, c2, c3


def uniform_pairs(seed, scenario_id, first, count, slot, attempt=0):
    """(count, 2) uniforms: counter (i, slot | attempt<<8, lo(id), hi(id)), key = seed,
    64-bit words (w1:w0), (w3:w2) mapped to ((w >> 12) + 0.5) * 2**-52."""
    i = np.arange(first, first + count, dtype=np.uint64)
    o0, o1, o2, o3 = philox_np(i, np.uint64(slot | (attempt << 8)),
                               np.uint64(scenario_id & MASK32),
                               np.uint64((scenario_id >> 32) & MASK32),
                               np.uint64(seed & MASK32), np.uint64((seed >> 32) & MASK32))
    w0 = (o1 << np.uint64(32)) | o0
    w1 = (o3 << np.uint64(32)) | o2
    u0 = ((w0 >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0 ** -52
    u1 = ((w1 >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0 ** -52
    return np.stack([u0, u1], axis=1)
