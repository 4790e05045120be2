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


def _cell_index(x, lo, cs, nc):
    """Integer cell of each coordinate along one axis (clamped to the grid)."""
    return np.clip(np.floor((x - lo) / cs).astype(np.int64), 0, nc - 1)


def _cells_per_axis(L, side):
    """Most cells of at least ``side`` that fit along a box side (>= 2)."""
    return max(2, int(np.floor(L / side)))


def neighbor_list_cells(pos, mol, box, r_list, rows_per_chunk=4096):
    """All directed edges, sorted by (i, j), found by binning the atoms into
    cells no smaller than the cutoff (the paper names cell lists as the way
    past its O(N^2) search, Sec. 2.1).  Only the candidates are found
    differently: every candidate pair goes through the same exact predicate
    as ``neighbor_rows``, so the edge set is the same.

    Cells: with a box, coordinates are wrapped into [0, L) and each axis is
    cut into nc = floor(L / (r_list (1 + 1e-9))) >= 2 equal cells, so a cell
    side exceeds the cutoff; two atoms closer than the cutoff under the
    minimum image then sit in the same or adjacent cells (modulo nc), and the
    27-cell stencil (duplicates removed when nc < 3) holds every partner.
    Without a box the cells cover the bounding box of the atoms."""
    _check(pos, box, r_list)
    x = pos.astype(np.float64)
    N = x.shape[0]
    if N == 0:
        z = np.zeros(0, np.int64)
        return z, z, np.zeros((0, 3), np.int64)
    mol = np.zeros(N, dtype=np.int64) if mol is None else np.asarray(mol, dtype=np.int64)
    rl = np.float64(np.float32(r_list))
    r2 = rl * rl
    L = None if box is None else np.asarray(box, dtype=np.float32).astype(np.float64)
    margin = 1.0 + 1e-9
    cell = np.zeros((N, 3), dtype=np.int64)
    nc = np.zeros(3, dtype=np.int64)
    for k in range(3):
        if L is None:
            lo, ext = x[:, k].min(), x[:, k].max() - x[:, k].min()
            nc[k] = max(1, int(np.floor(ext / (rl * margin))))
            cs = max(ext / nc[k], rl * margin)
            cell[:, k] = _cell_index(x[:, k], lo, cs, nc[k])
        else:
            nc[k] = _cells_per_axis(L[k], rl * margin)
            w = np.mod(x[:, k], L[k])
            cell[:, k] = _cell_index(w, 0.0, L[k] / nc[k], nc[k])
    flat = (cell[:, 0] * nc[1] + cell[:, 1]) * nc[2] + cell[:, 2]
    order = np.argsort(flat, kind="stable")
    n_cells = int(nc[0] * nc[1] * nc[2])
    start = np.searchsorted(flat[order], np.arange(n_cells), side="left")
    end = np.searchsorted(flat[order], np.arange(n_cells), side="right")
    # stencil offsets per axis, without duplicates (nc < 3 wraps onto itself)
    offs = []
    for k in range(3):
        if L is None:
            offs.append(np.array([-1, 0, 1]))
        else:
            offs.append(np.unique(np.mod(np.array([-1, 0, 1]), nc[k])))
    I, J, S = [], [], []
    for b0 in range(0, N, rows_per_chunk):
        ri = np.arange(b0, min(N, b0 + rows_per_chunk))
        ci = cell[ri]
        cand_i, cand_j = [], []
        for ox in offs[0]:
            for oy in offs[1]:
                for oz in offs[2]:
                    cc = ci + np.array([ox, oy, oz])
                    if L is None:
                        ok = np.all((cc >= 0) & (cc < nc), axis=1)
                    else:
                        cc = np.mod(cc, nc)
                        ok = np.ones(len(ri), dtype=bool)
                    f = (cc[:, 0] * nc[1] + cc[:, 1]) * nc[2] + cc[:, 2]
                    f = np.where(ok, f, 0)
                    cnt = np.where(ok, end[f] - start[f], 0)
                    rep_i = np.repeat(ri, cnt)
                    first = np.repeat(start[f], cnt)
                    k_in = np.arange(len(rep_i)) - np.repeat(np.cumsum(cnt) - cnt, cnt)
                    cand_i.append(rep_i)
                    cand_j.append(order[first + k_in])
        ci_, cj_ = np.concatenate(cand_i), np.concatenate(cand_j)
        d0 = x[cj_] - x[ci_]
        if L is None:
            d, n = d0, np.zeros_like(d0)
        else:
            d, n = _min_image(d0, L)
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        keep = (d2 < r2) & (mol[ci_] == mol[cj_]) & (ci_ != cj_)
        I.append(ci_[keep])
        J.append(cj_[keep])
        S.append(n[keep].astype(np.int64))
    I, J, S = np.concatenate(I), np.concatenate(J), np.concatenate(S)
    srt = np.lexsort((J, I))
    return I[srt], J[srt], S[srt]
