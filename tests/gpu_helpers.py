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
