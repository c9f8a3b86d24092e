"""Counter-based normal noise (test infrastructure only).

The method consumes independent standard normals: W^(r) and W^(w) for the
Brownian slip (Sections 3.1 and 3.3) and W, W~ for the EM-RFD step
(Section 4.4).  When a caller does not pass them, the device library draws
them itself from a counter-based generator; this module re-implements that
generator from its published definitions so that the draws can be checked
bit for bit and handed to the oracle:

  Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11): a 4 x 32-bit counter and a 2 x 32-bit key; ten
  rounds, each taking the high and low halves of two 32 x 32 -> 64-bit
  products with the multipliers 0xD2511F53 and 0xCD9E8D57 and mixing them
  with the other two words and the key; the key is advanced by the Weyl
  constants 0x9E3779B9 and 0xBB67AE85 between rounds.

  Box-Muller (Box and Muller, 1958): two uniforms u1 in (0, 1], u2 in
  [0, 1) give r = sqrt(-2 ln u1), z0 = r cos(2 pi u2), z1 = r sin(2 pi u2).

Stream layout (shared with the library): element i of stream `stream` at
draw `counter`, for the 64-bit `seed`:
  counter words (i >> 1, stream, counter low 32 bits, counter high 32 bits),
  key words (seed low 32 bits, seed high 32 bits);
  Philox output (x0, x1, x2, x3);
  u1 = ((x0 << 32 | x1) >> 11 + 1) 2^-53,  u2 = ((x2 << 32 | x3) >> 11) 2^-53;
  element 2j is z0 and element 2j + 1 is z1 of the pair j.
Streams: 0 = W^(r) (2N), 1 = W_grid (2 M^2), 2 = W~ (3n).
"""
import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF

STREAM_W_R, STREAM_W_GRID, STREAM_W_TILDE = 0, 1, 2


def philox4x32_10(ctr, key):
    """ctr: (4, n) uint64 arrays of 32-bit words; key: (2,) or (2, n).
    Returns the (4, n) output words as uint64 holding 32-bit values."""
    x = [np.asarray(c, dtype=np.uint64) & MASK for c in ctr]
    k0 = np.asarray(key[0], dtype=np.uint64) & MASK
    k1 = np.asarray(key[1], dtype=np.uint64) & MASK
    for r in range(10):
        p0 = np.uint64(M0) * x[0]          # exact: both factors < 2^32
        p1 = np.uint64(M1) * x[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        x = [hi1 ^ x[1] ^ k0, lo1, hi0 ^ x[3] ^ k1, lo0]
        if r < 9:
            k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
            k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
    return np.stack(x)


def raw_words(seed, stream, counter, n_pairs):
    """Philox output words (4, n_pairs) of pairs j = 0 .. n_pairs - 1."""
    j = np.arange(n_pairs, dtype=np.uint64)
    c = [j, np.full_like(j, stream), np.full_like(j, counter & MASK), np.full_like(j, (counter >> 32) & MASK)]
    return philox4x32_10(c, (seed & MASK, (seed >> 32) & MASK))


def normals(seed, stream, counter, n):
    """n standard normals of the given stream and draw (FP64)."""
    x = raw_words(seed, stream, counter, (n + 1) // 2)
    a = ((x[0] << np.uint64(32)) | x[1]) >> np.uint64(11)
    b = ((x[2] << np.uint64(32)) | x[3]) >> np.uint64(11)
    u1 = (a.astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = b.astype(np.float64) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * len(a))
    z[0::2] = r * np.cos(2.0 * np.pi * u2)
    z[1::2] = r * np.sin(2.0 * np.pi * u2)
    return z[:n]
