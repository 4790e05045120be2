"""Helpers shared by the GPU parity tests (inputs, oracle calls, tolerances)."""
import numpy as np
import torch

import oracle
import synthetic

# Tolerances of the FP32 path against the FP64 oracle.
E_ATOM_REL = 1e-5      # per-atom energy, relative to max(|E_i|, rms E)
F_MAX_ABS = 1e-4       # eV/A, max over atoms and components
E_MOL_REL = 1e-5       # structure energy, relative to its network part (net_scale; self energies are exact)

# The BF16 form against the FP64 oracle: bounds from the bfloat16 unit
# roundoff (oracle.bf16_energy_sigma: first-order spread of each energy when
# every rounding point errs independently by up to u = 2^-8; forces: each
# atom's spread under the oracle re-run in Monte Carlo arithmetic at the same
# points).  Force errors are heavy-tailed across atoms (an atom's spread
# follows the size of its neighbours' gradients), so the force gate is per
# atom.
BF16_K_SIGMA = 6.0     # energies: |dE| <= 6 sigma (+ the FP32 allowance)
BF16_K_FORCE = 8.0     # forces: |dF_a| <= 8 x atom a's spread (+ F_MAX_ABS)


def dev():
    return torch.device("cuda", 0)


def to_dev(w):
    d = dev()
    pos = torch.from_numpy(np.ascontiguousarray(w.pos)).to(d)
    sp = torch.from_numpy(np.ascontiguousarray(w.species.astype(np.int32))).to(d)
    mol = torch.from_numpy(np.ascontiguousarray(w.mol.astype(np.int32))).to(d) if w.n_mol > 1 else None
    return pos, sp, mol


def pairset(i, j, n):
    return set(zip(np.asarray(i).tolist(), np.asarray(j).tolist(), map(tuple, np.asarray(n).tolist())))


def energy_error(E, E_ref):
    """max_i |E_i - E_ref_i| / max(|E_ref_i|, rms(E_ref))."""
    E = np.asarray(E, dtype=np.float64)
    rms = np.sqrt(np.mean(E_ref ** 2)) if len(E_ref) else 1.0
    return float(np.max(np.abs(E - E_ref) / np.maximum(np.abs(E_ref), rms))) if len(E_ref) else 0.0


def bf16_flip_error(x, ref, scale):
    """Per-row error of the BF16 form against the oracle's bf16 emulation, as
    (median, max) of max_row|x - ref| / scale.

    Both sides round the same values to bfloat16, but the GPU accumulates in
    float32 and the oracle exactly; where the two pre-rounding values straddle
    a bfloat16 rounding boundary the rounded inputs differ by one bf16 ulp
    (2^-8 relative).  Such flips touch a minority of atoms (about one atom in
    ten for these widths), so the median row must sit at float32 accumulation
    error while the maximum is bounded by the effect of a few flips."""
    d = np.abs(np.asarray(x, np.float64) - ref)
    if d.ndim > 1:
        d = d.reshape(len(d), -1).max(1)
    d = d / scale
    return (float(np.median(d)), float(d.max())) if len(d) else (0.0, 0.0)


def organic(n, seed=31, density=0.1):
    return synthetic.organic_box(n=n, density=density, seed=seed)


def oracle_ef(w, spec, r_list=None, precision="fp64"):
    return oracle.energy_forces(w.pos, w.species, w.mol if w.n_mol > 1 else None, w.n_mol, w.box, spec,
                                r_list=r_list, precision=precision)


def net_scale(E_atom, species, spec, mol=None, n_mol=1):
    """Per structure: the size of the network's part of its energy (the
    self energies are added exactly), max(sum_i |E_i - e_s|, n_m x rms_j
    |E_j - e_s|).  The floor plays the part max(|E_i|, rms E) plays for one
    atom: a structure whose network energies happen to sum near zero (a lone
    atom, say) is still measured on the scale of its atoms' energies."""
    se = np.asarray(spec.self_energy, dtype=np.float64)[np.asarray(species, dtype=np.int64)]
    mol = np.zeros(len(E_atom), dtype=np.int64) if mol is None else np.asarray(mol, dtype=np.int64)
    net = np.abs(np.asarray(E_atom, dtype=np.float64) - se)
    out = np.zeros(n_mol)
    np.add.at(out, mol, net)
    count = np.bincount(mol, minlength=n_mol)
    rms = float(np.sqrt(np.mean(net ** 2))) if len(net) else 0.0
    return np.maximum(out, count * rms)


def e_mol_error(e_mol, ref, w, spec):
    """max over structures of |dE_mol| / net_scale (the network part of the
    structure energy)."""
    sc = net_scale(ref["E_atom"], w.species, spec, w.mol if w.n_mol > 1 else None, w.n_mol)
    return float(np.max(np.abs(np.asarray(e_mol, np.float64) - ref["E_mol"]) / np.maximum(sc, 1e-30)))


def bf16_energy_gate(e_atom, e_mol, ref, w, spec):
    """The BF16 form's energies against the FP64 oracle, in units of the
    first-order bfloat16 spread (plus the FP32 form's own allowance).
    Returns (max per-atom ratio, structure ratio); both must be <= 1."""
    mol = w.mol if w.n_mol > 1 else None
    sa, sm = oracle.bf16_energy_sigma(ref["aev"], w.species, spec, mol, w.n_mol)
    Er = ref["E_atom"]
    rms = np.sqrt(np.mean(Er ** 2))
    allow_a = E_ATOM_REL * np.maximum(np.abs(Er), rms)
    ra = np.abs(np.asarray(e_atom, np.float64) - Er) / (BF16_K_SIGMA * sa + allow_a)
    sc = net_scale(Er, w.species, spec, mol, w.n_mol)
    rm = np.abs(np.asarray(e_mol, np.float64) - ref["E_mol"]) / (BF16_K_SIGMA * sm + E_MOL_REL * sc)
    return float(ra.max()), float(rm.max())


def bf16_force_sigma(pos, species, box, spec, ref, atoms=None, runs=8, seed=0):
    """Per-atom spread of the BF16 form's forces [len(atoms)] (every atom if
    None): the oracle's dE/dAEV re-run ``runs`` times in Monte Carlo
    arithmetic at the form's rounding points (relative errors uniform in
    [-u, u], u = 2^-8, whose variance exceeds that of round-to-nearest), each
    pushed through the float64 edge-gradient chain of the same list and
    geometry; sigma_a is the rms over runs and the three components of
    F_mca - F_fp64.  Only the centres whose edges touch the requested atoms
    are evaluated (an atom's force holds its own edges and those pointing at
    it)."""
    from oracle.aev import pair_geometry
    from oracle.forces import edge_gradients, forces_from_edges
    from oracle.mlp import mlp_energy_and_grad
    N = len(species)
    i, j, _ = ref["nl"]
    atoms = np.arange(N) if atoms is None else np.asarray(atoms)
    want = np.zeros(N, dtype=bool)
    want[atoms] = True
    centres = np.nonzero(want | np.bincount(i[want[j]], minlength=N).astype(bool))[0]
    geo = pair_geometry(pos, box, ref["nl"])
    sp = np.asarray(species)
    rng = np.random.default_rng(seed)
    acc = np.zeros(len(atoms))
    for _ in range(runs):
        _, g = mlp_energy_and_grad(ref["aev"][centres], sp[centres], spec, "mca", rng=rng)
        G = edge_gradients(pos, species, box, ref["nl"], spec, g, centers=centres, geometry=geo)
        F = forces_from_edges(N, ref["nl"], G)
        acc += np.sum((F[atoms] - ref["F"][atoms]) ** 2, axis=1)
    return np.sqrt(acc / (3.0 * runs))


def bf16_force_gate(F, F_ref, sigma):
    """(max ratio, rms ratio): every component |dF_a| against 8 sigma_a +
    1e-4 eV/A (sigma_a from bf16_force_sigma, per atom), the rms over all
    components against 2 x the rms of sigma + 1e-5; both must be <= 1."""
    d = np.abs(np.asarray(F, np.float64) - F_ref)
    sigma = np.asarray(sigma, np.float64)
    return (float(np.max(d / (BF16_K_FORCE * sigma[:, None] + F_MAX_ABS))),
            float(np.sqrt(np.mean(d ** 2)) / (2.0 * np.sqrt(np.mean(sigma ** 2)) + 1e-5)))
