"""Seeded geometries for the five benchmark workloads and adversarial cases.

The paper benchmarks ANI-2x on periodic water boxes (648 atoms to 500K atoms)
and a solvated protein of about 20K atoms (Sec. 5, "Performance benchmarks").
No structure files ship with it, so every workload here is synthetic:

* water cluster: 24 rigid waters, O placed uniformly at random in a 12 A cube
  by random sequential addition with O-O >= 2.7 A, random orientations;
* water box: rigid waters at 1.0 g/cm^3 on a simple-cubic lattice of
  ceil(n^(1/3))^3 sites (n sites chosen at random), random orientations,
  wrapped into the periodic cube;
* organic box: 23,000 atoms of a fixed H/C/O/N/S/F/Cl mix at 0.1 atoms/A^3,
  random sequential addition with minimum-image distance >= 0.9 A;
* serving molecules: chain-grown bonded-like clusters of 8-150 atoms
  (log-uniform sizes), bond lengths U(0.95, 1.6) A from a parent drawn among
  the last four atoms, non-bonded distance >= 1.5 A;
* adversarial neighbour-list cases (atoms on cell faces, at x = L, negative
  coordinates, pairs exactly at the list cutoff, duplicated molecules in
  different batch slots).

Water: O-H 0.9572 A, H-O-H 104.52 degrees.  Atom order per water: O, H, H.
"""
from dataclasses import dataclass
import math

import numpy as np

from .params import MASSES, SPECIES_INDEX

H, C, N, O, F, S, CL = (SPECIES_INDEX[s] for s in ("H", "C", "N", "O", "F", "S", "Cl"))
WATER_MOLAR_MASS = 18.01528          # g/mol
AVOGADRO_PER_A3 = 0.602214076        # N_A * 1e-24 (g/cm^3 -> amu/A^3 factor)
ORGANIC_MIX = ((H, 0.50), (C, 0.25), (O, 0.12), (N, 0.08), (S, 0.03), (F, 0.01), (CL, 0.01))


@dataclass
class Workload:
    name: str
    pos: np.ndarray        # float32 [N, 3], Angstrom
    species: np.ndarray    # int32 [N]
    mol: np.ndarray        # int32 [N], non-decreasing molecule id
    n_mol: int
    box: np.ndarray        # float32 [3] (orthorhombic) or None (open)

    @property
    def n_atoms(self):
        return int(self.pos.shape[0])

    @property
    def masses(self):
        return MASSES[self.species].astype(np.float32)


def random_rotations(rng, n):
    """Uniform random rotation matrices from normalised Gaussian quaternions."""
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _water_local():
    r, th = 0.9572, math.radians(104.52)
    return np.array([[0.0, 0.0, 0.0],
                     [r * math.sin(th / 2), 0.0, r * math.cos(th / 2)],
                     [-r * math.sin(th / 2), 0.0, r * math.cos(th / 2)]])


def _place_waters(rng, centres):
    n = len(centres)
    R = random_rotations(rng, n)
    local = _water_local()
    xyz = centres[:, None, :] + np.einsum("nij,aj->nai", R, local)
    return xyz.reshape(-1, 3)


def _wrap32(x, L):
    """Wrap float64 coordinates into [0, L) and return float32 values that are
    guaranteed to lie in [0, L) after rounding."""
    L64 = np.asarray(L, dtype=np.float64)
    y = np.mod(x, L64)
    y32 = y.astype(np.float32)
    L32 = np.asarray(L, dtype=np.float32)
    y32 = np.where(y32 >= L32, np.float32(0.0), y32)
    return y32.astype(np.float32)


def water_box_side(n_mol, density_gcc=1.0):
    vol = n_mol * WATER_MOLAR_MASS / (AVOGADRO_PER_A3 * density_gcc)
    return vol ** (1.0 / 3.0)


def water_cluster(n_mol=24, side=12.0, min_oo=2.7, seed=1001):
    rng = np.random.default_rng(seed)
    centres = []
    while len(centres) < n_mol:
        c = rng.uniform(0.0, side, size=3)
        if all(np.linalg.norm(c - o) >= min_oo for o in centres):
            centres.append(c)
    xyz = _place_waters(rng, np.array(centres))
    species = np.tile(np.array([O, H, H], dtype=np.int32), n_mol)
    return Workload("water_cluster_%d" % (3 * n_mol), xyz.astype(np.float32), species,
                    np.zeros(3 * n_mol, dtype=np.int32), 1, None)


def water_box(n_mol=1500, density_gcc=1.0, seed=1002, side=None):
    rng = np.random.default_rng(seed)
    L = water_box_side(n_mol, density_gcc) if side is None else float(side)
    m = int(math.ceil(n_mol ** (1.0 / 3.0) - 1e-9))
    a = L / m
    sites = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1)
    sites = (sites.reshape(-1, 3) + 0.5) * a
    chosen = rng.choice(len(sites), size=n_mol, replace=False)
    chosen.sort()
    xyz = _place_waters(rng, sites[chosen])
    box = np.array([L, L, L], dtype=np.float32)
    pos = _wrap32(xyz, box.astype(np.float64))
    species = np.tile(np.array([O, H, H], dtype=np.int32), n_mol)
    return Workload("water_box_%d" % (3 * n_mol), pos, species,
                    np.zeros(3 * n_mol, dtype=np.int32), 1, box)


def _mix_counts(n, mix=ORGANIC_MIX):
    counts = [int(round(n * f)) for _, f in mix]
    counts[0] += n - sum(counts)
    return counts


def organic_box(n=23000, density=0.1, min_dist=0.9, seed=1003):
    rng = np.random.default_rng(seed)
    L = (n / density) ** (1.0 / 3.0)
    box = np.array([L, L, L], dtype=np.float32)
    L32 = box.astype(np.float64)
    ncell = max(1, int(L / min_dist))
    cs = L / ncell
    grid = {}
    pts = np.empty((n, 3))
    k = 0
    md2 = min_dist * min_dist
    while k < n:
        p = rng.uniform(0.0, L, size=3)
        p = np.asarray(_wrap32(p, L32), dtype=np.float64)
        c = (p / cs).astype(int) % ncell
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    key = ((c[0] + dx) % ncell, (c[1] + dy) % ncell, (c[2] + dz) % ncell)
                    for q in grid.get(key, ()):
                        d = pts[q] - p
                        d -= L32 * np.round(d / L32)
                        if d @ d < md2:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            pts[k] = p
            grid.setdefault((c[0], c[1], c[2]), []).append(k)
            k += 1
    species = np.concatenate([np.full(cnt, s, dtype=np.int32)
                              for (s, _), cnt in zip(ORGANIC_MIX, _mix_counts(n))])
    rng.shuffle(species)
    return Workload("organic_box_%d" % n, pts.astype(np.float32), species.astype(np.int32),
                    np.zeros(n, dtype=np.int32), 1, box)


def serving_molecule(rng, n=None, lo=8, hi=150):
    """One bonded-like molecule grown atom by atom (open boundaries)."""
    if n is None:
        n = int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi + 1)))))
        n = min(max(n, lo), hi)
    probs = np.array([f for _, f in ORGANIC_MIX])
    species = rng.choice(np.array([s for s, _ in ORGANIC_MIX], dtype=np.int32), size=n, p=probs)
    pts = np.zeros((n, 3))
    k = 1
    while k < n:
        placed = False
        for _attempt in range(200):
            parent = k - 1 - int(rng.integers(0, min(4, k)))
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            cand = pts[parent] + rng.uniform(0.95, 1.6) * d
            d2 = np.sum((pts[:k] - cand) ** 2, axis=1)
            d2[parent] = np.inf
            if np.all(d2 >= 1.5 * 1.5):
                pts[k] = cand
                k += 1
                placed = True
                break
        if not placed:      # crowded tail: restart the growth from scratch
            k = 1
    pos = pts
    pos -= pos.mean(axis=0)
    return pos.astype(np.float32), species.astype(np.int32)


def serving_stream(n_requests=20000, rate=2000.0, seed=1004):
    """Poisson arrivals of single-molecule requests: (arrival_s, species, pos)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    reqs = []
    for k in range(n_requests):
        pos, sp = serving_molecule(rng)
        reqs.append((float(t[k]), sp, pos))
    return reqs


def batch_molecules(mols, name="batch"):
    """Concatenate (pos, species) molecules into one open-boundary Workload."""
    pos = np.concatenate([m[0] for m in mols]).astype(np.float32)
    species = np.concatenate([m[1] for m in mols]).astype(np.int32)
    mol = np.concatenate([np.full(len(m[1]), k, dtype=np.int32) for k, m in enumerate(mols)])
    return Workload(name, pos, species, mol, len(mols), None)


def workload(cfg, **kw):
    """Workload for benchmark configuration 1, 2, 3, 4 (a batch of serving
    molecules) or 5."""
    if cfg == 1:
        return water_cluster(seed=1001, **kw)
    if cfg == 2:
        return water_box(1500, seed=1002, **kw)
    if cfg == 3:
        return organic_box(23000, seed=1003, **kw)
    if cfg == 4:
        rng = np.random.default_rng(1004)
        n_mol = kw.pop("n_mol", 64)
        return batch_molecules([serving_molecule(rng) for _ in range(n_mol)], "serving_batch")
    if cfg == 5:
        return water_box(33333, seed=1005, **kw)
    raise ValueError("unknown configuration %r" % (cfg,))


def small_water_box(n_mol=64, seed=7, side=None):
    """A periodic water box small enough for the oracle's O(N^2) paths; the
    side defaults to the 1.0 g/cm^3 value but is at least 2 * 5.6 A."""
    L = water_box_side(n_mol) if side is None else side
    return water_box(n_mol, seed=seed, side=max(L, 11.3))


def adversarial_cases(r_list=5.1):
    """Small inputs that stress the neighbour predicate and the cell binning."""
    cases = []
    f = np.float32
    # pair exactly at the cutoff (excluded: strict less-than), and just inside
    rl = f(r_list)
    inside = np.nextafter(rl, f(0))
    pos = np.array([[0, 0, 0], [rl, 0, 0], [0, inside, 0], [0, 0, -inside]], dtype=f)
    cases.append(Workload("exact_cutoff_open", pos, np.array([0, 1, 3, 3], np.int32),
                          np.zeros(4, np.int32), 1, None))
    # periodic: atoms on cell faces, at 0, at L-ulp, negative and beyond-L coordinates
    L = f(12.0)
    box = np.array([L, L, L], dtype=f)
    pts = [[0, 0, 0], [np.nextafter(L, f(0)), 0, 0], [L / 2, L / 2, L / 2],
           [-0.5, 11.9, 3.0], [12.4, -0.1, 6.0], [5.1, 0, 0], [6.0, 6.0, 0.0],
           [11.0, 11.0, 11.0], [1.0, 1.0, 1.0], [6.0, 0.0, 6.0], [-11.5, 23.0, 0.5]]
    pos = np.array(pts, dtype=f)
    cases.append(Workload("faces_periodic", pos, (np.arange(len(pts)) % 7).astype(np.int32),
                          np.zeros(len(pts), np.int32), 1, box))
    # pairs exactly r_list apart across the periodic boundary
    pos = np.array([[0.25, 1, 1], [0.25 + 12.0 - float(rl), 1, 1], [3, 3, 3]], dtype=f)
    cases.append(Workload("exact_cutoff_periodic", pos, np.array([3, 0, 0], np.int32),
                          np.zeros(3, np.int32), 1, box))
    # identical molecules in different batch slots must not see each other
    rng = np.random.default_rng(5)
    m = rng.uniform(0, 3, size=(6, 3)).astype(f)
    pos = np.concatenate([m, m, m + f(0.01)])
    sp = np.tile(np.array([0, 1, 3, 3, 0, 6], np.int32), 3)
    mol = np.repeat(np.arange(3, dtype=np.int32), 6)
    cases.append(Workload("coincident_molecules", pos, sp, mol, 3, None))
    # box exactly 2 * r_list wide in one dimension (smallest legal), 2 cells
    L2 = f(2 * float(rl) + 0.5)
    box2 = np.array([L2, f(20.0), f(20.0)], dtype=f)
    pos = rng.uniform(0, 1, size=(40, 3)).astype(f) * box2
    cases.append(Workload("thin_box", pos.astype(f), (np.arange(40) % 7).astype(np.int32),
                          np.zeros(40, np.int32), 1, box2))
    # three cells along every dimension (the row builder's stencil-shift
    # path): atoms on faces, at L - ulp, outside the box (the blocks then
    # take the minimum image pair by pair)
    L3 = f(16.0)
    box3 = np.array([L3, L3, L3], dtype=f)
    pts = [[0, 0, 0], [np.nextafter(L3, f(0)), 0, 0], [L3 / 2, L3 / 2, L3 / 2],
           [-0.5, 15.9, 4.0], [16.4, -0.1, 8.0], [5.1, 0, 0], [8.0, 8.0, 0.0],
           [15.0, 15.0, 15.0], [1.0, 1.0, 1.0], [8.0, 0.0, 8.0], [-15.5, 31.0, 0.5],
           [16.0 / 3, 16.0 / 3, 32.0 / 3], [32.0 / 3, 0.01, 15.99]]
    pos = np.array(pts, dtype=f)
    cases.append(Workload("faces_periodic_3cells", pos, (np.arange(len(pts)) % 7).astype(np.int32),
                          np.zeros(len(pts), np.int32), 1, box3))
    # every atom inside the box, three cells per dimension: pairs across the
    # periodic boundary at r_list and one or two ulp either side of it (their
    # float32 distance falls in the band the exact predicate decides)
    pts = []
    for k, base in enumerate([0.25, 0.75, 1.5]):
        xb = f(f(base) + L3 - rl)
        for step in (-2, -1, 0, 1, 2):
            v = xb
            for _ in range(abs(step)):
                v = np.nextafter(v, f(np.inf) if step > 0 else f(-np.inf))
            a = [base, 2.0 + 3 * k + 0.3 * (step + 2), 7.0]
            b = [float(v), a[1], a[2]]
            pts += [a, b] if k != 1 else [[a[1], a[0], a[2]], [b[1], b[0], b[2]]]
    pts += [[3.0, 12.0, 12.5], [13.0, 4.0, 2.0], [9.5, 9.5, 9.5]]
    pos = np.array(pts, dtype=f)
    cases.append(Workload("boundary_cutoff_3cells", pos, (np.arange(len(pts)) % 7).astype(np.int32),
                          np.zeros(len(pts), np.int32), 1, box3))
    # single atom, and a molecule of one atom beside a molecule of two
    cases.append(Workload("single_atom", np.zeros((1, 3), f), np.zeros(1, np.int32),
                          np.zeros(1, np.int32), 1, None))
    pos = np.array([[0, 0, 0], [0.5, 0, 0], [1.0, 0, 0]], dtype=f)
    cases.append(Workload("lonely_molecule", pos, np.array([6, 1, 0], np.int32),
                          np.array([0, 1, 1], np.int32), 2, None))
    return cases
