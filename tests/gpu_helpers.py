"""Helpers shared by the GPU parity tests (inputs, oracle calls, tolerances)."""
import numpy as np
import torch

import oracle
import synthetic

# Tolerances of the FP32 path against the FP64 oracle.
E_ATOM_REL = 1e-5      # per-atom energy, relative to max(|E_i|, rms E)
F_MAX_ABS = 1e-4       # eV/A, max over atoms and components


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


def organic(n, seed=31, density=0.1):
    return synthetic.organic_box(n=n, density=density, seed=seed)


def oracle_ef(w, spec, r_list=None, precision="fp64"):
    return oracle.energy_forces(w.pos, w.species, w.mol if w.n_mol > 1 else None, w.n_mol, w.box, spec,
                                r_list=r_list, precision=precision)
