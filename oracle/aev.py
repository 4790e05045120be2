"""Oracle atomic environment vector (ANI form), float64.

Definitions followed:

* edge geometry v_ij = x_j + n L - x_i and r_ij = |v_ij| (Sec. 2.1, processing
  modules recompute distances from coordinates so they can be differentiated);
* cosine switching function fc(r; Rc) = 0.5 cos(pi r / Rc) + 0.5 for r < Rc,
  0 beyond (Sec. 2.1, the cosine function used by ANI);
* radial part: Gaussian shells exp(-eta_R (r - R_k)^2) (Sec. 2.2, "Chemical
  and Radial Encodings"), summed over neighbours j of species s:
      G[i, s, k] = sum_j p_R exp(-eta_R (r_ij - R_k)^2) fc(r_ij; Rc_R);
* angular part: the ANI angular basis (0.5 + 0.5 cos(theta_ijk - theta_z))^zeta
  (App. A, angular resources), times a Gaussian of the mean distance, summed
  over unordered pairs {j, k} of neighbours within Rc_A, binned by the
  unordered species pair (s, t):
      G[i, p(s,t), a, z] = sum_{j<k} 2 ((1 + cos(theta' - theta_z)) / 2)^zeta
                           exp(-eta_A ((r_ij + r_ik)/2 - R_a)^2)
                           fc(r_ij; Rc_A) fc(r_ik; Rc_A)
  with theta' = arccos(0.95 cos theta_ijk); cos(theta' - theta_z) is expanded
  as u cos(theta_z) + sqrt(1 - u^2) sin(theta_z), u = 0.95 cos theta_ijk.

Layout of the 1008 features: radial column 16 s + k (7 x 16 = 112), then
angular column 112 + 32 p + 8 a + z with p the upper-triangular index of the
species pair (28 pairs x 4 x 8 = 896).  Species order H, C, N, O, F, S, Cl.
"""
import numpy as np


def f64(x):
    """Model parameters are float32 numbers; the oracle evaluates with their
    exact float64 widening."""
    return np.asarray(np.asarray(x, dtype=np.float32), dtype=np.float64)


class AEVLayout:
    def __init__(self, spec):
        self.ns = spec.n_species
        self.nr = spec.n_shf_r
        self.na = spec.n_shf_a
        self.nz = spec.n_shf_z
        self.radial_dim = self.ns * self.nr
        self.dim = self.radial_dim + self.ns * (self.ns + 1) // 2 * self.na * self.nz

    def pair_index(self, s, t):
        """Upper-triangular index of the unordered species pair (s, t)."""
        s, t = np.minimum(s, t), np.maximum(s, t)
        return s * self.ns - (s * (s - 1)) // 2 + (t - s)

    def radial_col(self, s, k):
        return self.nr * s + k

    def angular_col(self, p, a, z):
        return self.radial_dim + self.na * self.nz * p + self.nz * a + z


def switch(r, rc):
    rc = f64(rc)
    return np.where(r < rc, 0.5 * np.cos(np.pi * r / rc) + 0.5, 0.0)


def switch_deriv(r, rc):
    rc = f64(rc)
    return np.where(r < rc, -0.5 * np.pi / rc * np.sin(np.pi * r / rc), 0.0)


def pair_geometry(pos, box, nl):
    """Edge vectors and lengths in float64 for the edge list (i, j, n)."""
    i, j, n = nl
    x = pos.astype(np.float64)
    v = x[j] - x[i]
    if box is not None:
        v = v + n.astype(np.float64) * f64(box)
    r = np.sqrt(np.sum(v * v, axis=1))
    return v, r


def angular_triplets(i, r, rc_a):
    """Unordered pairs of edges {e1, e2} (e1 < e2) sharing the centre i and
    both shorter than rc_a.  Edges are sorted by centre.  Returns (e1, e2)."""
    ang = np.nonzero(r < f64(rc_a))[0]
    if len(ang) == 0:
        z = np.zeros(0, np.int64)
        return z, z
    ci = i[ang]
    starts = np.r_[0, np.nonzero(np.diff(ci))[0] + 1]
    counts = np.diff(np.r_[starts, len(ang)])
    local = np.arange(len(ang)) - np.repeat(starts, counts)       # position in its group
    m = np.repeat(counts, counts)
    partners = m - 1 - local                                      # later edges in the group
    e1 = np.repeat(np.arange(len(ang)), partners)
    blk = np.repeat(np.cumsum(partners) - partners, partners)
    e2 = e1 + 1 + (np.arange(len(e1)) - blk)
    return ang[e1], ang[e2]


def angular_factors(v1, r1, v2, r2, spec):
    """Per-triplet factors: F1 [T, nz], F2 [T, na], fc1 fc2, plus the pieces
    the derivative needs."""
    cs = f64(spec.cos_scale)
    zeta = f64(spec.zeta)
    thz = f64(spec.shf_z)
    ra = f64(spec.shf_a)
    eta = f64(spec.eta_a)
    dot = np.sum(v1 * v2, axis=1)
    den = np.maximum(r1 * r2, 1e-10)
    c = np.clip(dot / den, -1.0, 1.0)
    u = cs * c
    sq = np.sqrt(1.0 - u * u)
    w = u[:, None] * np.cos(thz)[None, :] + sq[:, None] * np.sin(thz)[None, :]
    base = 0.5 * (1.0 + w)
    F1 = np.where(base > 0.0, np.power(np.maximum(base, 0.0), zeta), 0.0)
    rbar = 0.5 * (r1 + r2)
    F2 = np.exp(-eta * (rbar[:, None] - ra[None, :]) ** 2)
    return dict(dot=dot, den=den, c=c, u=u, sq=sq, w=w, base=base, F1=F1, rbar=rbar, F2=F2)


def aev(pos, species, box, nl, spec, centers=None, chunk=1 << 18, geometry=None, n_atoms=None):
    """AEV rows (float64) for all atoms, or for the atoms listed in
    ``centers`` (the edge list must then contain at least their rows).
    ``geometry`` = (v, r) float64 edge vectors and lengths overrides the
    ones computed from ``pos`` (used for finite differences)."""
    lay = AEVLayout(spec)
    N = pos.shape[0] if n_atoms is None else n_atoms
    i, j, n = nl
    v, r = pair_geometry(pos, box, nl) if geometry is None else geometry
    if centers is not None:
        centers = np.asarray(centers, dtype=np.int64)
        rowpos = np.full(N, -1, dtype=np.int64)
        rowpos[centers] = np.arange(len(centers))
        sel = rowpos[i] >= 0
        i, j, n, v, r = i[sel], j[sel], n[sel], v[sel], r[sel]
        out_i = rowpos[i]
        n_out = len(centers)
    else:
        out_i = i
        n_out = N
    Z = np.asarray(species, dtype=np.int64)

    # radial
    pr = f64(spec.radial_prefactor)
    fcr = switch(r, spec.rc_r)
    rk = f64(spec.shf_r)
    radial = pr * np.exp(-f64(spec.eta_r) * (r[:, None] - rk[None, :]) ** 2) * fcr[:, None]
    col = (out_i * lay.dim)[:, None] + lay.radial_col(Z[j], 0)[:, None] + np.arange(lay.nr)[None, :]
    flat = np.bincount(col.ravel(), weights=radial.ravel(), minlength=n_out * lay.dim)

    # angular
    e1, e2 = angular_triplets(i, r, spec.rc_a)
    fca = switch(r, spec.rc_a)
    az = (lay.nz * np.arange(lay.na)[:, None] + np.arange(lay.nz)[None, :]).ravel()   # 8a + z
    for t0 in range(0, len(e1), chunk):
        a1, a2 = e1[t0:t0 + chunk], e2[t0:t0 + chunk]
        fac = angular_factors(v[a1], r[a1], v[a2], r[a2], spec)
        w2 = 2.0 * fca[a1] * fca[a2]
        term = w2[:, None, None] * fac["F2"][:, :, None] * fac["F1"][:, None, :]   # [T, a, z]
        p = lay.pair_index(Z[j[a1]], Z[j[a2]])
        col = (out_i[a1] * lay.dim + lay.angular_col(p, 0, 0))[:, None] + az[None, :]
        flat += np.bincount(col.ravel(), weights=term.reshape(len(a1), -1).ravel(),
                            minlength=n_out * lay.dim)
    return flat.reshape(n_out, lay.dim)
