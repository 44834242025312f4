"""Oracle-side decoding/encoding of the limb storage format (TEST INFRASTRUCTURE ONLY).

Storage of an array of N numbers at p = 32*L bits (structure of arrays):
  limbs: uint32[L, N]   plane k holds 32-bit limb k of every mantissa, k = 0 least significant
  hdr:   int32[N]       (e << 1) | s ; a zero has e = -2^30 (hdr = INT32_MIN or INT32_MIN + 1)

This is an independent reader/writer of that layout for the oracle; it shares no code with the
GPU path or with the input generators.
"""
import numpy as np

from .mpnum import MP

ZERO_E = -(1 << 30)


def decode(limbs, hdr, p):
    limbs = np.asarray(limbs, dtype=np.uint32)
    hdr = np.asarray(hdr, dtype=np.int32)
    nlimb = p // 32
    assert limbs.shape[0] == nlimb and limbs.shape[1] == hdr.shape[0]
    out = []
    cols = limbs.T.astype(object)
    for i in range(hdr.shape[0]):
        h = int(hdr[i])
        s = h & 1
        e = h >> 1
        if e == ZERO_E:
            out.append(MP(s, 0, 0, p))
            continue
        m = 0
        row = cols[i]
        for k in range(nlimb - 1, -1, -1):
            m = (m << 32) | int(row[k])
        out.append(MP(s, m, e, p))
    return out


def encode(values, p):
    nlimb = p // 32
    n = len(values)
    limbs = np.zeros((nlimb, n), dtype=np.uint32)
    hdr = np.zeros(n, dtype=np.int32)
    mask = (1 << 32) - 1
    for i, v in enumerate(values):
        if v.m == 0:
            hdr[i] = (ZERO_E << 1) | v.s
            continue
        hdr[i] = (v.e << 1) | v.s
        m = v.m
        for k in range(nlimb):
            limbs[k, i] = m & mask
            m >>= 32
    return limbs, hdr
