"""Write threshold_blocks.txt: 8x8 blocks whose directional contrast v
(Algorithm 1) is exactly one of the values where Eq. (13) changes its
result (2^10 - 1, 2^10, 2^16 - 1, 2^16, 2^17 - 1, 2^17).

The blocks are inputs for the GPU parity tests; v is evaluated by the
oracle only.  s_d is a quadratic form in the centred samples, so for a few
chosen pixel positions its coefficients are read off the oracle's
direction costs of unit blocks and their pairwise sums, and many deviation
vectors are then scored at once; every hit is re-checked by a direct oracle
call before it is written.

    python tests/golden/make_threshold_blocks.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle  # noqa: E402

TARGETS = [1023, 1024, 65535, 65536, 131071, 131072]
OUT = os.path.join(HERE, "threshold_blocks.txt")


def costs(dev):
    return oracle.direction_costs((128 + dev).astype(np.uint16), 8).astype(np.int64)


def contrast(dev):
    c = costs(dev)
    best = 0
    for d in range(1, 8):
        if c[d] > c[best]:
            best = d
    return int(c[best] - c[(best + 4) & 7])


def main():
    rng = np.random.default_rng(1602)
    found = {}
    tries = 0
    while len(found) < len(TARGETS):
        tries += 1
        assert tries < 20000, "search did not converge"
        npx = 2 if tries % 3 else 3
        pos = set()
        while len(pos) < npx:
            pos.add(tuple(int(v) for v in rng.integers(0, 8, 2)))
        pos = sorted(pos)
        unit = []
        for p in pos:
            e = np.zeros((8, 8), np.int64)
            e[p] = 1
            unit.append(e)
        diag = [costs(e) for e in unit]
        cross = {(a, b): costs(unit[a] + unit[b]) - diag[a] - diag[b]
                 for a in range(npx) for b in range(a + 1, npx)}
        lim = 40 if tries % 2 else 127
        x = rng.integers(-lim, lim + 1, size=(200000, npx))
        s = np.zeros((x.shape[0], 8), np.int64)
        for a in range(npx):
            s += diag[a][None, :] * (x[:, a] ** 2)[:, None]
        for (a, b), c in cross.items():
            s += c[None, :] * (x[:, a] * x[:, b])[:, None]
        best = np.argmax(s, axis=1)  # first maximum: the lowest direction
        r = np.arange(len(s))
        v = s[r, best] - s[r, (best + 4) & 7]
        for t in TARGETS:
            if t in found:
                continue
            idx = np.nonzero(v == t)[0]
            if idx.size:
                k = int(idx[0])
                blk = np.zeros((8, 8), np.int64)
                for a, p in enumerate(pos):
                    blk[p] += x[k, a]
                assert contrast(blk) == t
                found[t] = [(p[0], p[1], int(x[k, a])) for a, p in enumerate(pos)]
    with open(OUT, "w") as f:
        f.write("# Written by make_threshold_blocks.py (oracle only).\n"
                "# v, then row,col,deviation of each pixel that differs from 128 in an\n"
                "# 8-bit 8x8 block (all other pixels are 128).\n")
        for t in TARGETS:
            f.write(f"{t} " + " ".join(f"{i},{j},{d}" for i, j, d in found[t]) + "\n")
    print(OUT)


if __name__ == "__main__":
    main()
