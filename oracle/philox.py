"""Philox4x32-10 counter-based generator, plain Python integers.

TEST INFRASTRUCTURE ONLY.  This module belongs to the oracle: only the tests,
the smoke check and the CPU-baseline leg of the benchmark may import it.

The SMC sampler draws momenta (Alg. smc_ChEES, "sample momentum"), Metropolis
uniforms (eq. mh_ratio_rn) and the resampling uniform (Sec. III) at random.
The parity tests usually inject those numbers; when they are not injected,
both the device library and this oracle draw them from the same published
counter-based generator, Philox4x32 with 10 rounds (Salmon, Moraes, Dror and
Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011).  This file is
written from that definition and shares nothing with the device code.

Stream layout (a convention of this project, mirrored by the library):
counter = (block, particle, iteration, stream id), key = (seed low 32 bits,
seed high 32 bits).  Each 32-bit word x maps to the open-interval uniform
(x + 1/2) / 2^32, which is exact in binary64.  Normals come from the
Box--Muller transform on a pair of such uniforms.
"""

import math

MASK32 = 0xFFFFFFFF
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85

STREAM_INIT = 1      # initial draw theta_0 ~ q0
STREAM_MOMENTUM = 2  # momenta of each trajectory
STREAM_MH = 3        # Metropolis-Hastings uniforms
STREAM_RESAMPLE = 4  # resampling uniform(s)
STREAM_FLOW = 5      # initial weights of the flow preconditioner
STREAM_JITTER = 6    # uniform jitter draws (uniform and offset-equidistant schemes)
STREAM_SHUFFLE = 7   # round functions of the equidistant schemes' shuffle


def philox4x32_10(counter, key):
    """One Philox4x32-10 block: 4 counter words, 2 key words -> 4 words."""
    c0, c1, c2, c3 = (int(v) & MASK32 for v in counter)
    k0, k1 = (int(v) & MASK32 for v in key)
    for _ in range(10):
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK32
        hi1, lo1 = p1 >> 32, p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK32, lo1, (hi0 ^ c3 ^ k1) & MASK32, lo0
        k0 = (k0 + PHILOX_W0) & MASK32
        k1 = (k1 + PHILOX_W1) & MASK32
    return (c0, c1, c2, c3)


def seed_key(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & MASK32, seed >> 32)


def u01(word):
    """Open-interval uniform from one 32-bit word: (x + 1/2) / 2^32."""
    return (float(word) + 0.5) / 4294967296.0


def normals(seed, particle, iteration, stream, count):
    """`count` standard normals for one particle, via Box--Muller pairs.

    Block b supplies words (w0, w1, w2, w3); normals 4b, 4b+1 come from the
    pair (w0, w1) and normals 4b+2, 4b+3 from (w2, w3):
        r = sqrt(-2 log u_a),  n_even = r cos(2 pi u_b),  n_odd = r sin(2 pi u_b).
    """
    key = seed_key(seed)
    out = []
    block = 0
    while len(out) < count:
        w = philox4x32_10((block, particle, iteration, stream), key)
        for a, b in ((w[0], w[1]), (w[2], w[3])):
            r = math.sqrt(-2.0 * math.log(u01(a)))
            t = 2.0 * math.pi * u01(b)
            out.append(r * math.cos(t))
            out.append(r * math.sin(t))
        block += 1
    return out[:count]


def uniform(seed, particle, iteration, stream):
    """One open-interval uniform: word 0 of block 0."""
    w = philox4x32_10((0, particle, iteration, stream), seed_key(seed))
    return u01(w[0])


# ---------------------------------------------------------------------------
# Vectorised form (numpy uint64), same definition, used for whole populations.
# ---------------------------------------------------------------------------
import numpy as _np


def philox4x32_10_np(c0, c1, c2, c3, key):
    """Philox4x32-10 over arrays of counters (each a uint64 array < 2^32)."""
    m = _np.uint64(MASK32)
    c0, c1, c2, c3 = (_np.asarray(v, dtype=_np.uint64) & m for v in (c0, c1, c2, c3))
    k0, k1 = (_np.uint64(int(v) & MASK32) for v in key)
    M0, M1 = _np.uint64(PHILOX_M0), _np.uint64(PHILOX_M1)
    W0, W1 = _np.uint64(PHILOX_W0), _np.uint64(PHILOX_W1)
    s32 = _np.uint64(32)
    for _ in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> s32, p0 & m
        hi1, lo1 = p1 >> s32, p1 & m
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & m, lo1, (hi0 ^ c3 ^ k1) & m, lo0
        k0 = (k0 + W0) & m
        k1 = (k1 + W1) & m
    return c0, c1, c2, c3


def u01_np(words):
    return (words.astype(_np.float64) + 0.5) / 4294967296.0


def normals_np(seed, num_particles, iteration, stream, count):
    """(num_particles, count) standard normals; row j equals normals(seed, j, ...)."""
    nblk = (count + 3) // 4
    blk, part = _np.meshgrid(_np.arange(nblk, dtype=_np.uint64),
                             _np.arange(num_particles, dtype=_np.uint64))
    it = _np.full_like(blk, iteration)
    st = _np.full_like(blk, stream)
    w0, w1, w2, w3 = philox4x32_10_np(blk, part, it, st, seed_key(seed))
    out = _np.empty((num_particles, nblk, 4))
    for (a, b), col in (((w0, w1), 0), ((w2, w3), 2)):
        r = _np.sqrt(-2.0 * _np.log(u01_np(a)))
        t = 2.0 * _np.pi * u01_np(b)
        out[:, :, col] = r * _np.cos(t)
        out[:, :, col + 1] = r * _np.sin(t)
    return out.reshape(num_particles, nblk * 4)[:, :count]


def uniforms_np(seed, num_particles, iteration, stream):
    """(num_particles,) uniforms; entry j equals uniform(seed, j, ...)."""
    part = _np.arange(num_particles, dtype=_np.uint64)
    z = _np.zeros_like(part)
    w0, _, _, _ = philox4x32_10_np(z, part, z + _np.uint64(iteration), z + _np.uint64(stream),
                                   seed_key(seed))
    return u01_np(w0)
