"""Oracle energies and forces (Sec. 2.4: per-structure sum of atomic
energies; forces are minus the gradient of the total energy).

Chain rule, written out:
    g_i = dE_i/dAEV_i                                 (MLP adjoint, mlp.py)
    G_ij = dE_i/dv_ij                                 (edge gradient, 3-vector)
  radial, for each edge i->j with r = |v_ij| < Rc_R:
    dE_i/dr += sum_k g_i[16 Z_j + k] p_R e_k (-2 eta_R (r - R_k) fc(r) + fc'(r)),
    e_k = exp(-eta_R (r - R_k)^2),  G_ij += (dE_i/dr) v_ij / r
  angular, for each unordered pair {j, k} of edges shorter than Rc_A, with
  T_az = 2 F1_z(c) F2_a(rbar) fc(r_ij) fc(r_ik) and coefficients
  g_az = g_i[112 + 32 p(Z_j, Z_k) + 8 a + z]:
    dE/dc    = sum_az g_az 2 F2_a fc_j fc_k dF1_z/dc,
    dE/drbar = sum_az g_az 2 F1_z fc_j fc_k dF2_a/drbar,
    dE/dfc_j = sum_az g_az 2 F1_z F2_a fc_k,
    G_ij += dE/dc dc/dv_ij + (dE/drbar / 2 + dE/dfc_j fc'(r_ij)) v_ij / r_ij
  (and symmetrically for k), with
    dc/dv_ij = v_ik / (r_ij r_ik) - c v_ij / r_ij^2,
    dF1_z/dc = 0.95 (zeta/2) ((1 + w_z)/2)^(zeta-1) (cos th_z - u sin th_z / sqrt(1-u^2)),
    dF2_a/drbar = -2 eta_A (rbar - R_a) F2_a.
  An edge of zero length (coincident atoms) has no direction; its gradient
  is taken as zero (1/r is replaced by 0 there).
  Forces, since v_ij = x_j + n L - x_i:
    F_a = -dE/dx_a = sum_{a->j} G_aj - sum_{i->a} G_ia.
  Virial (the stress-tensor output of Sec. 5.1), per structure and per atom:
    W = - sum over edges i->j of v_ij (outer) G_ij,
  which is sum_a x_a (outer) F_a for an open structure; a homogeneous strain
  v -> (1 + eps) v of every edge vector changes E by -tr(W^T eps) to first
  order.
"""
import numpy as np

from .aev import AEVLayout, aev as aev_fn, angular_factors, angular_triplets, f64, pair_geometry, \
    switch, switch_deriv
from .mlp import mlp_energies_per_net, mlp_energy_and_grad
from .neighbors import neighbor_list, neighbor_list_cells


def edge_gradients(pos, species, box, nl, spec, g, centers=None, chunk=1 << 18, geometry=None,
                   n_atoms=None):
    """G [P, 3] = dE_i / dv_ij for every edge of the list whose centre is in
    ``centers`` (all edges if None).  ``g`` holds dE/dAEV rows indexed like
    ``centers`` (or by atom if None)."""
    lay = AEVLayout(spec)
    N = pos.shape[0] if n_atoms is None else n_atoms
    i, j, n = nl
    if centers is not None:
        rowpos = np.full(N, -1, dtype=np.int64)
        rowpos[np.asarray(centers)] = np.arange(len(centers))
        gi = rowpos[i]
    else:
        gi = i
    valid = gi >= 0
    v, r = pair_geometry(pos, box, nl) if geometry is None else geometry
    Z = np.asarray(species, dtype=np.int64)
    G = np.zeros((len(i), 3))
    # an edge of zero length has no direction: its gradient is taken as zero
    rinv = np.where(r > 0, 1.0 / np.where(r > 0, r, 1.0), 0.0)

    # radial
    rc = f64(spec.rc_r)
    eta = f64(spec.eta_r)
    rk = f64(spec.shf_r)
    pr = f64(spec.radial_prefactor)
    sel = np.nonzero(valid & (r < rc))[0]
    rr = r[sel][:, None]
    e = np.exp(-eta * (rr - rk[None, :]) ** 2)
    dterm = pr * e * (-2.0 * eta * (rr - rk[None, :]) * switch(rr, rc) + switch_deriv(rr, rc))
    cols = lay.radial_col(Z[j[sel]], 0)[:, None] + np.arange(lay.nr)[None, :]
    coef = g[gi[sel][:, None], cols]
    dEdr = np.sum(coef * dterm, axis=1)
    G[sel] += (dEdr * rinv[sel])[:, None] * v[sel]

    # angular
    e1, e2 = angular_triplets(i, r, spec.rc_a)
    keep = valid[e1]
    e1, e2 = e1[keep], e2[keep]
    rca = f64(spec.rc_a)
    fca = switch(r, rca)
    dfca = switch_deriv(r, rca)
    thz = f64(spec.shf_z)
    ra = f64(spec.shf_a)
    eta_a = f64(spec.eta_a)
    zeta = f64(spec.zeta)
    cs = f64(spec.cos_scale)
    for t0 in range(0, len(e1), chunk):
        a1, a2 = e1[t0:t0 + chunk], e2[t0:t0 + chunk]
        f = angular_factors(v[a1], r[a1], v[a2], r[a2], spec)
        p = lay.pair_index(Z[j[a1]], Z[j[a2]])
        base_col = lay.angular_col(p, 0, 0)
        cols = base_col[:, None] + np.arange(lay.na * lay.nz)[None, :]
        gaz = g[gi[a1][:, None], cols].reshape(len(a1), lay.na, lay.nz)
        F1, F2 = f["F1"], f["F2"]                                         # [T,z], [T,a]
        base = f["base"]
        dF1dw = np.where(base > 0, 0.5 * zeta * np.power(np.maximum(base, 1e-300), zeta - 1.0), 0.0)
        dwdu = np.cos(thz)[None, :] - (f["u"] / f["sq"])[:, None] * np.sin(thz)[None, :]
        dF1dc = dF1dw * dwdu * cs                                          # [T,z]
        dF2 = -2.0 * eta_a * (f["rbar"][:, None] - ra[None, :]) * F2       # [T,a]
        fj, fk = fca[a1], fca[a2]
        dEdc = 2.0 * fj * fk * np.einsum("taz,ta,tz->t", gaz, F2, dF1dc)
        dEdrbar = 2.0 * fj * fk * np.einsum("taz,ta,tz->t", gaz, dF2, F1)
        S = np.einsum("taz,ta,tz->t", gaz, F2, F1)
        dEdfj = 2.0 * fk * S
        dEdfk = 2.0 * fj * S
        r1, r2 = r[a1], r[a2]
        v1, v2 = v[a1], v[a2]
        c = f["c"]
        den = f["den"]
        i1, i2 = rinv[a1], rinv[a2]
        dc1 = v2 / den[:, None] - (c * i1 * i1)[:, None] * v1
        dc2 = v1 / den[:, None] - (c * i2 * i2)[:, None] * v2
        s1 = 0.5 * dEdrbar + dEdfj * dfca[a1]
        s2 = 0.5 * dEdrbar + dEdfk * dfca[a2]
        G1 = dEdc[:, None] * dc1 + (s1 * i1)[:, None] * v1
        G2 = dEdc[:, None] * dc2 + (s2 * i2)[:, None] * v2
        for k in range(3):
            G[:, k] += np.bincount(a1, weights=G1[:, k], minlength=len(i))
            G[:, k] += np.bincount(a2, weights=G2[:, k], minlength=len(i))
    return G


def forces_from_edges(N, nl, G):
    i, j, _ = nl
    F = np.zeros((N, 3))
    for k in range(3):
        F[:, k] = np.bincount(i, weights=G[:, k], minlength=N) - np.bincount(j, weights=G[:, k], minlength=N)
    return F


def virial_from_edges(nl, v, G, mol=None, n_mol=1, n_atoms=None):
    """(W_mol [n_mol,3,3], W_atom [N,3,3]): W = -sum_edges v_ij (outer) G_ij,
    per structure (edges summed in ascending centre order) and per centre."""
    i = nl[0]
    N = (int(i.max()) + 1 if len(i) else 0) if n_atoms is None else n_atoms
    outer = -v[:, :, None] * G[:, None, :]                      # [P,3,3]
    W_atom = np.zeros((N, 3, 3))
    for a in range(3):
        for b in range(3):
            W_atom[:, a, b] = np.bincount(i, weights=outer[:, a, b], minlength=N)
    mol = np.zeros(N, dtype=np.int64) if mol is None else np.asarray(mol)
    W_mol = np.zeros((n_mol, 3, 3))
    for a in range(N):
        W_mol[mol[a]] += W_atom[a]
    return W_mol, W_atom


def energy_forces(pos, species, mol, n_mol, box, spec, r_list=None, precision="fp64",
                  nl=None, need_forces=True, need_virial=False, need_nets=False, rng=None):
    """Full evaluation.  Returns dict with E_mol [n_mol], E_atom [N],
    F [N,3] (if requested), aev [N,D], g [N,D], nl.  precision: "fp64",
    "bf16" (the BF16 form's emulation) or "mca" (Monte Carlo arithmetic at
    its rounding points, drawing from rng)."""
    if r_list is None:
        r_list = spec.rc_r
    N = pos.shape[0]
    if nl is None:
        # the O(N^2) scan of the definition for small systems, the cell-binned
        # search (pinned to the same edge set) beyond
        search = neighbor_list if N <= 4096 else neighbor_list_cells
        nl = search(pos, mol, box, r_list)
    A = aev_fn(pos, species, box, nl, spec)
    E_atom, g = mlp_energy_and_grad(A, species, spec, precision, need_grad=need_forces, rng=rng)
    mol = np.zeros(N, dtype=np.int64) if mol is None else np.asarray(mol)
    E_mol = np.zeros(n_mol)
    for a in range(N):                                  # ascending atom index
        E_mol[mol[a]] += E_atom[a]
    out = dict(E_mol=E_mol, E_atom=E_atom, aev=A, g=g, nl=nl)
    if need_nets:
        # every network's structure energies (ascending atom order)
        E_net = mlp_energies_per_net(A, species, spec, precision)
        E_mol_net = np.zeros((E_net.shape[0], n_mol))
        for a in range(N):
            E_mol_net[:, mol[a]] += E_net[:, a]
        out["E_mol_net"] = E_mol_net
    if need_forces or need_virial:
        G = edge_gradients(pos, species, box, nl, spec, g)
        out["G"] = G
        out["F"] = forces_from_edges(N, nl, G)
    if need_virial:
        v, _ = pair_geometry(pos, box, nl)
        out["W_mol"], out["W_atom"] = virial_from_edges(nl, v, out["G"], mol, n_mol, N)
    return out


def _geometry64(x, box, nl):
    i, j, n = nl
    v = x[j] - x[i]
    if box is not None:
        v = v + n.astype(np.float64) * f64(box)
    return v, np.sqrt(np.sum(v * v, axis=1))


def total_energy(pos64, species, box, spec, nl, precision="fp64"):
    """Total energy for float64 positions and a fixed edge list (for finite
    differences; the list must cover every pair that can come within Rc_R)."""
    x = np.asarray(pos64, dtype=np.float64)
    A = aev_fn(None, species, box, nl, spec, geometry=_geometry64(x, box, nl), n_atoms=x.shape[0])
    E_atom, _ = mlp_energy_and_grad(A, species, spec, precision, need_grad=False)
    return float(np.sum(E_atom))


def energy_forces_f64(pos64, species, box, spec, nl, precision="fp64"):
    """(total energy, forces [N,3]) for float64 positions and a fixed edge
    list (the list must cover every pair that can come within Rc_R)."""
    x = np.asarray(pos64, dtype=np.float64)
    geo = _geometry64(x, box, nl)
    A = aev_fn(None, species, box, nl, spec, geometry=geo, n_atoms=x.shape[0])
    E_atom, g = mlp_energy_and_grad(A, species, spec, precision)
    G = edge_gradients(None, species, box, nl, spec, g, geometry=geo, n_atoms=x.shape[0])
    return float(np.sum(E_atom)), forces_from_edges(x.shape[0], nl, G)
