"""Build step: write the Sobol direction-number table the library embeds.

The table V[dim][bit] (uint32, 32 bits per dimension, Joe–Kuo direction
numbers, dimension 0 = van der Corput) is taken from SciPy's Sobol engine,
an implementation independent of this project, and checked against points
that engine generates: with x_j(n) the XOR of V_j[b] over the set bits b of
gray(n) = n ^ (n >> 1), the first 2^12 points must match bit for bit.

Output: a little-endian binary file of dims * 32 uint32 values.
"""
import sys

import numpy as np


def direction_table():
    import scipy.stats.qmc as qmc
    d = qmc.Sobol.MAXDIM
    eng = qmc.Sobol(d=d, scramble=False, bits=32)
    V = np.ascontiguousarray(eng._sv, dtype=np.uint32)   # [dims][32]
    if V.shape != (d, 32):
        raise RuntimeError(f"unexpected direction table shape {V.shape}")
    # self-check on 64 dimensions and 4096 points against generated points
    chk = qmc.Sobol(d=64, scramble=False, bits=32)
    pts = np.rint(chk.random(4096) * 2.0 ** 32).astype(np.uint64).astype(np.uint32)
    n = np.arange(4096, dtype=np.uint64)
    g = n ^ (n >> np.uint64(1))
    x = np.zeros((4096, 64), dtype=np.uint32)
    for b in range(12):
        sel = ((g >> np.uint64(b)) & np.uint64(1)).astype(bool)
        x[sel] ^= V[:64, b]
    if not np.array_equal(x, pts):
        raise RuntimeError("direction table does not reproduce the engine's points")
    return V


def main(out_path):
    V = direction_table()
    V.astype("<u4").tofile(out_path)
    return V.shape[0]


if __name__ == "__main__":
    print(main(sys.argv[1]))
