"""Counter-based Gaussian sampling noise (the paper only asks for N(0, Sigma)).

Philox4x32 with 10 rounds as published by Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11): each round takes
the two 32x32->64 products of counter words 0 and 2 with the two round
multipliers, mixes their high halves with the other two counter words and
the key, and the key is advanced by the two Weyl increments between
rounds.  Uniforms are turned into normals with the Box-Muller transform
(Box & Muller, 1958).

Counter layout used by this build: key = (seed_lo, seed_hi XOR problem_id),
counter = (sample k, step t, instance m, iteration).  Words x0..x3 give
u1 = (x0 + 1) 2^-32, u2 = x1 2^-32 -> normals (n0, n1), and likewise
(x2, x3) -> (n2, n3); they perturb (thrust, omega_x, omega_y, omega_z).

Parity note: the paper fixes no generator, so this bit stream is pinned
only by statistical checks of its output and by bitwise agreement with
the independent GPU implementation.
"""
import numpy as np

MASK = np.uint64(0xFFFFFFFF)
MUL0, MUL1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
WEYL0, WEYL1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)


def philox4x32_10(ctr, key):
    """ctr: 4 arrays of uint32 values; key: 2 uint32 values -> 4 uint32 arrays."""
    c = [np.asarray(w, np.uint64) & MASK for w in ctr]
    c = np.broadcast_arrays(*c)
    c = [np.array(w) for w in c]
    k0, k1 = np.uint64(key[0]) & MASK, np.uint64(key[1]) & MASK
    for r in range(10):
        if r:
            k0 = (k0 + WEYL0) & MASK
            k1 = (k1 + WEYL1) & MASK
        p0 = MUL0 * c[0]
        p1 = MUL1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return [w.astype(np.uint32) for w in c]


def philox_key(seed, problem_id):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, ((seed >> 32) ^ int(problem_id)) & 0xFFFFFFFF)


def raw_words(seed, problem_id, M, K, N, iteration=0):
    """uint32 words (4, M, K, N) for every (instance, sample, step)."""
    m, k, t = np.meshgrid(np.arange(M), np.arange(K), np.arange(N), indexing="ij")
    ctr = (k, t, m, np.full_like(k, iteration))
    return np.stack(philox4x32_10(ctr, philox_key(seed, problem_id)))


def box_muller(a, b):
    """Two uint32 words -> two standard normals (float64)."""
    u1 = (a.astype(np.float64) + 1.0) * 2.0 ** -32
    u2 = b.astype(np.float64) * 2.0 ** -32
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2.0 * np.pi * u2), r * np.sin(2.0 * np.pi * u2)


def normals(seed, problem_id, M, K, N, iteration=0):
    """Standard normals (M, K, N, 4) in channel order (F, wx, wy, wz)."""
    w = raw_words(seed, problem_id, M, K, N, iteration)
    n0, n1 = box_muller(w[0], w[1])
    n2, n3 = box_muller(w[2], w[3])
    return np.stack([n0, n1, n2, n3], -1)
