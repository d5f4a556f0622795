"""Test helpers: marshal the oracle's dense SOCP into the library's compact
cone layout and back (selection of structurally non-zero blocks; no method
arithmetic)."""
import numpy as np

from oracle import linearize


def cone_blocks(s, j):
    """(first block time, number of blocks) of cone j in the compact layout."""
    if s.kind[j] == linearize.KIND_STATE:
        return 0, int(s.time[j]) + 1
    return int(s.time[j]), 1


def compact_socp(s):
    nx, nu, T = s.nx, s.nu, s.T
    bh, bv = [], []
    for j in range(s.ng):
        k0, nb = cone_blocks(s, j)
        bh.append(np.concatenate([[0.0], s.bhat[j, k0 * nx:(k0 + nb) * nx]]))
        bj = s.bmat[j].reshape(T, nu)
        blocks = np.zeros((nb, nu))
        for m in range(nb):
            k = k0 + m
            if k < T:
                blocks[m] = bj[k]
        bv.append(blocks.ravel())
    return dict(A=s.A, B=s.B, xhat=s.xhat, uhat=s.uhat, g0=s.g0, w=s.w,
                bhat=np.concatenate(bh), bvec=np.concatenate(bv))


def entry_offsets(s):
    off = [0]
    for j in range(s.ng):
        _, nb = cone_blocks(s, j)
        off.append(off[-1] + 1 + nb * s.nx)
    return np.array(off)


def expand_entries(s, x):
    """Compact per-entry vector -> dense (ng, 1 + nz) rows (zeros outside the support)."""
    off = entry_offsets(s)
    D = np.zeros((s.ng, 1 + s.nz))
    for j in range(s.ng):
        k0, nb = cone_blocks(s, j)
        seg = x[off[j]:off[j + 1]]
        D[j, 0] = seg[0]
        D[j, 1 + k0 * s.nx:1 + (k0 + nb) * s.nx] = seg[1:]
    return D


def compress_rows(s, D):
    """Dense (ng, 1 + nz) rows -> compact per-entry vector."""
    out = []
    for j in range(s.ng):
        k0, nb = cone_blocks(s, j)
        out.append(np.concatenate([[D[j, 0]], D[j, 1 + k0 * s.nx:1 + (k0 + nb) * s.nx]]))
    return np.concatenate(out)


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))
