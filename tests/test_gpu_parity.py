"""AEV, species networks, energies and forces on the GPU vs the FP64 oracle.

Tolerances: per-atom energy 1e-5 relative (to max(|E_i|, rms E)), forces
1e-4 eV/A max abs for the FP32 form; AEV features and dE/dAEV within the
float32 arithmetic bounds stated in each test."""
import numpy as np
import pytest
import torch

import oracle
import synthetic
import paper_2405_01491_amd as nnp
from tests.gpu_helpers import E_ATOM_REL, F_MAX_ABS, dev, energy_error, oracle_ef, organic, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def model(spec_bias):
    return nnp.Model(spec_bias, "fp32")


def _workloads():
    return {
        "cluster72": lambda: synthetic.workload(1),
        "water_box_192": lambda: synthetic.geometry.small_water_box(64),
        "organic_3000": lambda: organic(3000),
        "serving_batch": lambda: synthetic.workload(4, n_mol=24),
    }


@pytest.mark.parametrize("name", list(_workloads()))
def test_aev_parity(model, spec_bias, name):
    w = _workloads()[name]()
    pos, sp, mol = to_dev(w)
    nl = nnp.nnp_neighbors(model, pos, mol, w.n_mol, w.box, 5.1)
    A = nnp.nnp_aev(model, pos, sp, w.box, nl).cpu().numpy().astype(np.float64)
    nnp.nnp_check(model)
    ref = oracle.aev(w.pos, w.species, w.box, oracle.neighbor_list(w.pos, w.mol if w.n_mol > 1 else None,
                                                                   w.box, 5.1), spec_bias)
    D = spec_bias.aev_dim
    assert np.all(A[:, D:] == 0.0)
    err = np.abs(A[:, :D] - ref) / (1.0 + np.abs(ref))
    print("%s: max AEV err %.3g (max |AEV| %.3g)" % (name, err.max(), np.abs(ref).max()))
    assert err.max() < 2e-5


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_mlp_parity(spec_bias, precision):
    m = nnp.Model(spec_bias, precision)
    w = organic(2000)
    ref_aev = oracle.aev(w.pos, w.species, w.box, oracle.neighbor_list(w.pos, None, w.box, 5.1), spec_bias)
    A = np.zeros((w.n_atoms, m.aev_stride), np.float32)
    A[:, :spec_bias.aev_dim] = ref_aev
    e, g = nnp.nnp_mlp(m, torch.from_numpy(w.species).to(dev()), torch.from_numpy(A).to(dev()))
    e = e.cpu().numpy().astype(np.float64)
    g = g.cpu().numpy().astype(np.float64)
    assert np.all(g[:, spec_bias.aev_dim:] == 0.0)
    # reference on the float32-rounded features the GPU received
    oprec = "bf16" if precision == "bf16" else "fp64"
    E_ref, g_ref = oracle.mlp_energy_and_grad(A[:, :spec_bias.aev_dim].astype(np.float64), w.species, spec_bias,
                                              oprec)
    ee = energy_error(e, E_ref)
    gscale = np.max(np.abs(g_ref))
    ge = np.max(np.abs(g[:, :spec_bias.aev_dim] - g_ref)) / gscale
    print("mlp %s: E err %.3g, dE/dAEV err %.3g (scale %.3g)" % (precision, ee, ge, gscale))
    if precision == "fp32":
        assert ee < E_ATOM_REL and ge < 1e-5
    else:
        # same bf16 rounding points as the oracle's emulation; float32 accumulation
        assert ee < 2e-4 and ge < 2e-3
        E64, _ = oracle.mlp_energy_and_grad(A[:, :spec_bias.aev_dim].astype(np.float64), w.species, spec_bias)
        print("mlp bf16 vs fp64 oracle: E err %.3g" % energy_error(e, E64))


@pytest.mark.parametrize("name", list(_workloads()) + ["water_4500"])
def test_energy_forces_parity(model, spec_bias, name):
    w = synthetic.workload(2) if name == "water_4500" else _workloads()[name]()
    pos, sp, mol = to_dev(w)
    r_list = 5.6 if w.box is not None else 5.1
    nl = nnp.nnp_neighbors(model, pos, mol, w.n_mol, w.box, r_list)
    e_mol, e_atom, F = nnp.nnp_energy_forces(model, pos, sp, mol, w.n_mol, w.box, nl, e_atom=True)
    torch.cuda.synchronize()
    nnp.nnp_check(model)
    ref = oracle_ef(w, spec_bias, r_list=r_list)
    ee = energy_error(e_atom.cpu().numpy(), ref["E_atom"])
    em = np.max(np.abs(e_mol.cpu().numpy() - ref["E_mol"]) / np.maximum(1.0, np.abs(ref["E_mol"])))
    fe = np.max(np.abs(F.cpu().numpy() - ref["F"]))
    print("%s: E_atom err %.3g, E_mol err %.3g, F max err %.3g eV/A (max |F| %.3g)"
          % (name, ee, em, fe, np.abs(ref["F"]).max()))
    assert ee < E_ATOM_REL
    assert em < 1e-5
    assert fe < F_MAX_ABS


def test_bf16_form_error_table(spec_bias):
    m = nnp.Model(spec_bias, "bf16")
    w = organic(3000)
    pos, sp, mol = to_dev(w)
    nl = nnp.nnp_neighbors(m, pos, None, 1, w.box, 5.1)
    e_mol, e_atom, F = nnp.nnp_energy_forces(m, pos, sp, None, 1, w.box, nl, e_atom=True)
    ref = oracle_ef(w, spec_bias)
    emu = oracle_ef(w, spec_bias, precision="bf16")
    e_atom = e_atom.cpu().numpy()
    F = F.cpu().numpy()
    print("bf16 vs fp64: E_atom %.3g F max %.3g; vs bf16-emulated: E_atom %.3g F max %.3g"
          % (energy_error(e_atom, ref["E_atom"]), np.abs(F - ref["F"]).max(),
             energy_error(e_atom, emu["E_atom"]), np.abs(F - emu["F"]).max()))
    assert energy_error(e_atom, emu["E_atom"]) < 2e-4
    assert np.abs(F - emu["F"]).max() < 2e-2


def test_autograd_matches_forces(model, spec_bias):
    w = synthetic.workload(4, n_mol=6)
    pos, sp, mol = to_dev(w)
    x = pos.clone().requires_grad_(True)
    E = nnp.energy(model, x, sp, mol, w.n_mol, None)
    wts = torch.arange(1, w.n_mol + 1, dtype=torch.float64, device=dev())
    (E * wts).sum().backward()
    ref = oracle_ef(w, spec_bias)
    want = -ref["F"] * np.arange(1, w.n_mol + 1)[w.mol][:, None]
    assert np.max(np.abs(x.grad.cpu().numpy() - want)) < 1e-4 * w.n_mol


def test_deterministic_and_batch_invariant(model):
    rng = np.random.default_rng(77)
    mols = [synthetic.serving_molecule(rng) for _ in range(12)]
    wb = synthetic.geometry.batch_molecules(mols)
    pos, sp, mol = to_dev(wb)
    nl = nnp.nnp_neighbors(model, pos, mol, wb.n_mol, None, 5.1)
    e1, a1, f1 = [t.clone() for t in nnp.nnp_energy_forces(model, pos, sp, mol, wb.n_mol, None, nl, e_atom=True)]
    e2, a2, f2 = nnp.nnp_energy_forces(model, pos, sp, mol, wb.n_mol, None, nl, e_atom=True)
    assert torch.equal(e1, e2) and torch.equal(a1, a2) and torch.equal(f1, f2)
    off = 0
    for k, (p, s) in enumerate(mols):
        pk = torch.from_numpy(p).to(dev())
        sk = torch.from_numpy(s).to(dev())
        nlk = nnp.nnp_neighbors(model, pk, None, 1, None, 5.1)
        ek, ak, fk = nnp.nnp_energy_forces(model, pk, sk, None, 1, None, nlk, e_atom=True)
        n = len(s)
        assert torch.equal(ek[0], e1[k]), k
        assert torch.equal(ak, a1[off:off + n]), k
        assert torch.equal(fk, f1[off:off + n]), k
        off += n


def test_species_out_of_range_flagged(model):
    w = synthetic.workload(1)
    pos, sp, _ = to_dev(w)
    bad = sp.clone()
    bad[3] = 9
    nl = nnp.nnp_neighbors(model, pos, None, 1, None, 5.1)
    nnp.nnp_energy_forces(model, pos, bad, None, 1, None, nl)
    with pytest.raises(nnp.NNPError):
        nnp.nnp_check(model)
    nnp.nnp_energy_forces(model, pos, sp, None, 1, None, nl)
    nnp.nnp_check(model)
