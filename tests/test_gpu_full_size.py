"""Parity at the benchmark's full sizes, through the calls the benchmark
times: the 23,000-atom organic-like box (nnp_energy_forces on a list built
once), checked on every atom against one full oracle evaluation, and the
99,999-atom water box (the MD engine: fixed-stride rows, skin 0.5 A, rebuilds
by the Verlet-list bound and every 20 steps, checked after a run that crosses
a rebuild), checked on sampled atoms, in the FP32 and BF16-MLP forms.

For the 99,999-atom box the oracle evaluates each sampled atom a on the
sub-system of all atoms within 2 Rc_R (+ 0.2 A) of it, kept with their own
coordinates in the same periodic box.  The atoms whose energies depend on
the position of a are those within Rc_R of it, and their environments lie
inside that sub-system, so the sub-system's E_a and F_a are those of the
whole box.  The sample holds, for every species, the first and last atom of
its segment of the species-grouped rows and the atoms on either side of the
first network-tile boundaries, plus random atoms: 160 in all.

The BF16 form is gated against the FP64 oracle by the bfloat16 error model
(energies: 6 sigma of oracle.bf16_energy_sigma; forces: 8 x each atom's
spread under the oracle re-run in Monte Carlo arithmetic at the form's
rounding points)."""
import numpy as np
import pytest
import torch

import oracle
import synthetic
import paper_2405_01491_amd as nnp
from paper_2405_01491_amd import md as nmd
from tests.gpu_helpers import (BF16_K_SIGMA, E_ATOM_REL, E_MOL_REL, F_MAX_ABS, bf16_energy_gate, bf16_force_gate,
                               bf16_force_sigma, dev, e_mol_error, energy_error, to_dev)

pytestmark = pytest.mark.gpu

N_SAMPLE = 160
TILE = 32          # rows per network tile at these sizes


def sample_atoms(species, n, seed):
    """First and last atom of each species' segment, the atoms around the
    first tile boundaries of each segment, then random atoms."""
    pick = set()
    for s in np.unique(species):
        idx = np.nonzero(species == s)[0]                      # the segment, in grouped-row order
        for q in (0, TILE - 1, TILE, 2 * TILE - 1, 2 * TILE, len(idx) - 1):
            if 0 <= q < len(idx):
                pick.add(int(idx[q]))
    rng = np.random.default_rng(seed)
    while len(pick) < n:
        pick.add(int(rng.integers(0, len(species))))
    return np.array(sorted(pick))


def _sub_system(pos, box, a, rc):
    d = pos.astype(np.float64) - pos[a].astype(np.float64)
    L = np.asarray(box, dtype=np.float64)
    d -= L * np.round(d / L)
    idx = np.nonzero(np.sum(d * d, axis=1) < (2.0 * rc + 0.2) ** 2)[0]
    return idx, int(np.searchsorted(idx, a))


def _oracle_atoms(pos, species, box, spec, atoms, bf16):
    """FP64 E_a and F_a for each sampled atom and, for the BF16 form, the
    first-order BF16 sigma of E_a and the Monte Carlo spread of F_a."""
    E, S, SF = np.zeros(len(atoms)), np.zeros(len(atoms)), np.zeros(len(atoms))
    F = np.zeros((len(atoms), 3))
    for q, a in enumerate(atoms):
        idx, k = _sub_system(pos, box, a, spec.rc_r)
        out = oracle.energy_forces(pos[idx], species[idx], None, 1, box, spec, r_list=spec.rc_r)
        E[q], F[q] = out["E_atom"][k], out["F"][k]
        if bf16:
            S[q] = oracle.bf16_energy_sigma(out["aev"], species[idx], spec)[0][k]
            SF[q] = bf16_force_sigma(pos[idx], species[idx], box, spec, out, atoms=[k], seed=q)[0]
    return E, F, S, SF


def _check_sampled(name, precision, E, F, pos, species, box, spec, atoms):
    E_ref, F_ref, sig, sig_f = _oracle_atoms(pos, species, box, spec, atoms, precision == "bf16")
    rms = np.sqrt(np.mean(E_ref ** 2))
    ee = float(np.max(np.abs(E - E_ref) / np.maximum(np.abs(E_ref), rms)))
    fe = float(np.abs(F - F_ref).max())
    msg = "%s %s, %d sampled atoms vs fp64 oracle: E_atom err %.3g, F max err %.3g eV/A" % (
        name, precision, len(atoms), ee, fe)
    if precision == "fp32":
        print(msg)
        assert ee < E_ATOM_REL and fe < F_MAX_ABS
        return
    ra = np.abs(E - E_ref) / (BF16_K_SIGMA * sig + E_ATOM_REL * np.maximum(np.abs(E_ref), rms))
    rf, rr = bf16_force_gate(F, F_ref, sig_f)
    print(msg + "; bound ratios E_atom %.3f, F max %.3f, F rms %.3f (rms Monte Carlo spread %.3g eV/A)"
          % (ra.max(), rf, rr, float(np.sqrt(np.mean(sig_f ** 2)))))
    assert ra.max() <= 1.0 and rf <= 1.0 and rr <= 1.0


@pytest.fixture(scope="module")
def organic_ref(spec_bias):
    w = synthetic.workload(3)
    return w, oracle.energy_forces(w.pos, w.species, None, 1, w.box, spec_bias)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_organic_box_23000_every_atom(spec_bias, organic_ref, precision):
    w, ref = organic_ref
    model = nnp.Model(spec_bias, precision)
    pos, sp, _ = to_dev(w)
    nl = nnp.nnp_neighbors(model, pos, None, 1, w.box, spec_bias.rc_r)
    e_mol, e_atom, F = nnp.nnp_energy_forces(model, pos, sp, None, 1, w.box, nl, e_atom=True)
    torch.cuda.synchronize()
    nnp.nnp_check(model)
    e_mol, e_atom, F = e_mol.cpu().numpy(), e_atom.cpu().numpy(), F.cpu().numpy()
    ee = energy_error(e_atom, ref["E_atom"])
    em = e_mol_error(e_mol, ref, w, spec_bias)
    fe = float(np.abs(F - ref["F"]).max())
    msg = "organic_box_23000 %s, all atoms vs fp64 oracle: E_atom err %.3g, E_mol err %.3g, F max err %.3g" % (
        precision, ee, em, fe)
    if precision == "fp32":
        print(msg)
        assert ee < E_ATOM_REL and em < E_MOL_REL and fe < F_MAX_ABS
    else:
        ra, rm = bf16_energy_gate(e_atom, e_mol, ref, w, spec_bias)
        sig = bf16_force_sigma(w.pos, w.species, w.box, spec_bias, ref, runs=6)
        rf, rr = bf16_force_gate(F, ref["F"], sig)
        print(msg + "; bound ratios E_atom %.3f, E_mol %.3f, F max %.3f, F rms %.3f" % (ra, rm, rf, rr))
        assert ra <= 1.0 and rm <= 1.0 and rf <= 1.0 and rr <= 1.0
    # the structure energy is the float64 sum of the atomic energies
    assert abs(float(e_mol[0]) - float(e_atom.astype(np.float64).sum())) < 1e-9 * max(1.0, abs(float(e_mol[0])))


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_water_box_99999_engine_sampled(spec_bias, precision):
    w = synthetic.workload(5)
    model = nnp.Model(spec_bias, precision)
    pos, sp, _ = to_dev(w)
    masses = synthetic.MASSES[w.species]
    v0 = torch.from_numpy(nmd.maxwell_boltzmann(masses, 300.0, seed=2024)).to(dev())
    eng = nmd.MDEngine(model, pos, v0, sp, masses, w.box, dt=0.5, integrator="nve", skin=0.5, rebuild_every=20)
    eng.run(25)
    x, _, F, e_pot = eng.state()
    torch.cuda.synchronize()
    info = eng.info()
    assert info["steps"] == 25 and info["rebuilds"] >= 2
    x_np = x.cpu().numpy()
    atoms = sample_atoms(w.species, N_SAMPLE, 99)
    # per-atom energies at the engine's positions through the plain call
    nl = nnp.nnp_neighbors(model, x, None, 1, w.box, spec_bias.rc_r)
    e_mol, e_atom, F_plain = nnp.nnp_energy_forces(model, x, sp, None, 1, w.box, nl, e_atom=True)
    torch.cuda.synchronize()
    nnp.nnp_check(model)
    _check_sampled("water_box_99999 engine", precision, e_atom.cpu().numpy()[atoms], F.cpu().numpy()[atoms], x_np,
                   w.species, w.box, spec_bias, atoms)
    # the engine's energy and forces agree with the plain call on every atom
    assert abs(float(e_pot[0]) - float(e_mol[0])) < 1e-9 * max(1.0, abs(float(e_mol[0])))
    assert torch.max(torch.abs(F - F_plain)).item() < 1e-5
