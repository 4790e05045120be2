"""Oracle neighbour list (Sec. 2.1, "Preprocessing Modules").

Definition followed: an edge i -> j exists when i != j, both atoms carry the
same batch (molecule) index, and their distance is strictly lower than the
cutoff.  Graphs are directed, so each pair appears as i -> j and j -> i.
With an orthorhombic periodic box the minimum-image convention is used and
the integer image shift n (in box vectors) is recorded so that the edge
vector is v_ij = x_j + n * L - x_i.

The predicate is evaluated exactly as follows so that any implementation can
reproduce the same pair set bit for bit: coordinates are float32 values
widened to float64; d0 = x_j - x_i; n = -rint(d0 / L) (round half to even);
d = d0 + n * L; d2 = (dx*dx + dy*dy) + dz*dz, each operation rounded to
float64 with no fused multiply-add; the pair is kept iff
d2 < r * r with r the float32 cutoff widened to float64.

The minimum-image convention is only unambiguous when every box side is at
least twice the cutoff; smaller boxes are rejected.
"""
import numpy as np


def _check(pos, box, r_list):
    if pos.dtype != np.float32:
        raise TypeError("positions must be float32 (the values both sides see)")
    if box is not None:
        L = np.asarray(box, dtype=np.float32).astype(np.float64)
        rl = np.float64(np.float32(r_list))
        if np.any(L < 2.0 * rl):
            raise ValueError("box side below twice the list cutoff")


def _min_image(d0, L):
    n = -np.rint(d0 / L)
    return d0 + n * L, n


def neighbor_rows(pos, mol, box, r_list, rows, block=64):
    """Directed edges (i, j, n) for the centres in ``rows`` (ascending i,
    then ascending j).  Each row costs O(N)."""
    _check(pos, box, r_list)
    x = pos.astype(np.float64)
    N = x.shape[0]
    mol = np.zeros(N, dtype=np.int64) if mol is None else np.asarray(mol)
    rl = np.float64(np.float32(r_list))
    r2 = rl * rl
    L = None if box is None else np.asarray(box, dtype=np.float32).astype(np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    I, J, S = [], [], []
    for b0 in range(0, len(rows), block):
        r = rows[b0:b0 + block]
        d0 = x[None, :, :] - x[r, None, :]                 # [B, N, 3]
        if L is None:
            d, n = d0, np.zeros_like(d0)
        else:
            d, n = _min_image(d0, L)
        d2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        keep = (d2 < r2) & (mol[None, :] == mol[r, None])
        keep[np.arange(len(r)), r] = False
        bi, bj = np.nonzero(keep)                          # row-major: sorted by (row, j)
        I.append(r[bi])
        J.append(bj)
        S.append(n[bi, bj].astype(np.int64))
    if not I:
        return (np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros((0, 3), np.int64))
    return np.concatenate(I), np.concatenate(J), np.concatenate(S)


def neighbor_list(pos, mol, box, r_list):
    """All directed edges, sorted by (i, j)."""
    return neighbor_rows(pos, mol, box, r_list, np.arange(pos.shape[0]))


def brute_force_pairs(pos, mol, box, r_list, max_image=3):
    """Pure-Python enumeration over every periodic image |n_k| <= max_image
    (plain double arithmetic, same operation order as the predicate).  For
    tiny inputs only; used to pin ``neighbor_list``."""
    _check(pos, box, r_list)
    N = pos.shape[0]
    rl = float(np.float32(r_list))
    r2 = rl * rl
    Ls = None if box is None else [float(np.float32(b)) for b in box]
    imgs = [(0, 0, 0)] if Ls is None else [
        (a, b, c) for a in range(-max_image, max_image + 1)
        for b in range(-max_image, max_image + 1) for c in range(-max_image, max_image + 1)]
    out = []
    for i in range(N):
        for j in range(N):
            if i == j or (mol is not None and mol[i] != mol[j]):
                continue
            for n in imgs:
                d = []
                for k in range(3):
                    dk = float(pos[j, k]) - float(pos[i, k])
                    if Ls is not None:
                        dk = dk + float(n[k]) * Ls[k]
                    d.append(dk)
                d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
                if d2 < r2:
                    out.append((i, j, n))
    out.sort()
    return out
