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
from tests.gpu_helpers import (E_ATOM_REL, E_MOL_REL, F_MAX_ABS, bf16_energy_gate, bf16_flip_error, bf16_force_gate,
                               bf16_force_sigma, dev, e_mol_error, energy_error, oracle_ef, organic, to_dev)

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


@pytest.mark.parametrize("path", ["fused", "per_layer"])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_mlp_parity(spec_bias, precision, path):
    m = nnp.Model(spec_bias, precision)
    assert m.fused_mlp
    m.set_fused_mlp(path == "fused")
    assert m.fused_mlp == (path == "fused")
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
    print("mlp %s %s: E err %.3g, dE/dAEV err %.3g (scale %.3g)" % (precision, path, ee, ge, gscale))
    if precision == "fp32":
        assert ee < E_ATOM_REL and ge < 1e-5
    else:
        # same bf16 rounding points as the oracle's emulation; float32 accumulation
        net = E_ref - np.asarray(spec_bias.self_energy)[w.species]
        rms = np.sqrt(np.mean(net ** 2))
        emed, emax = bf16_flip_error(e, E_ref, rms)
        gmed, gmax = bf16_flip_error(g[:, :spec_bias.aev_dim], g_ref, gscale)
        print("mlp bf16 %s vs emulation (median, max): E/rms %.3g %.3g, dE/dAEV %.3g %.3g"
              % (path, emed, emax, gmed, gmax))
        assert emed < 2e-6 and emax < 1e-2 and gmed < 2e-6 and gmax < 1e-2
        assert ee < 2e-4 and ge < 1e-2
        # against the exact network on the same features: within the bfloat16 error model
        A64 = A[:, :spec_bias.aev_dim].astype(np.float64)
        E64, _ = oracle.mlp_energy_and_grad(A64, w.species, spec_bias)
        sa, _ = oracle.bf16_energy_sigma(A64, w.species, spec_bias)
        z = np.abs(e - E64) / sa
        print("mlp bf16 vs fp64 oracle: E err %.3g, |dE| / sigma max %.3g rms %.3g"
              % (energy_error(e, E64), z.max(), np.sqrt(np.mean(z ** 2))))
        assert z.max() < 6.0


def test_fused_and_per_layer_paths_agree(spec_bias):
    w = organic(2000)
    pos, sp, _ = to_dev(w)
    for precision in ("fp32", "bf16"):
        m = nnp.Model(spec_bias, precision)
        nl = nnp.nnp_neighbors(m, pos, None, 1, w.box, 5.1)
        m.set_fused_mlp(True)
        e1, a1, f1 = [t.clone() for t in nnp.nnp_energy_forces(m, pos, sp, None, 1, w.box, nl, e_atom=True)]
        m.set_fused_mlp(False)
        e2, a2, f2 = nnp.nnp_energy_forces(m, pos, sp, None, 1, w.box, nl, e_atom=True)
        da = (a1 - a2).abs().max().item()
        df = (f1 - f2).abs().max().item()
        print("%s fused vs per-layer: max |dE_atom| %.3g, max |dF| %.3g" % (precision, da, df))
        # atomic energies include self energies (up to 460 eV): compare in units of their float32 ulp
        tol_e = (4 if precision == "fp32" else 64) * 1.2e-7 * max(1.0, a2.abs().max().item())
        tol_f = 1e-5 if precision == "fp32" else 5e-3
        assert da < tol_e and df < tol_f


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
    em = e_mol_error(e_mol.cpu().numpy(), ref, w, spec_bias)
    fe = np.max(np.abs(F.cpu().numpy() - ref["F"]))
    print("%s: E_atom err %.3g, E_mol err %.3g (of sum |E_i - e_s|), F max err %.3g eV/A (max |F| %.3g)"
          % (name, ee, em, fe, np.abs(ref["F"]).max()))
    assert ee < E_ATOM_REL
    assert em < E_MOL_REL
    assert fe < F_MAX_ABS


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_generic_widths_mlp_only(precision):
    """Per-layer GEMM path on given features (isolates the networks from AEV rounding)."""
    import synthetic.weights as sw
    spec = synthetic.ani2x_like_spec(weight_seed=99, bias_scale=0.05)
    spec.widths = (1008, 128, 64, 96, 1)
    spec.weights = sw.glorot_weights(7, spec.widths, 99, 0.05)
    m = nnp.Model(spec, precision)
    assert not m.fused_mlp
    w = organic(1500)
    ref_aev = oracle.aev(w.pos, w.species, w.box, oracle.neighbor_list(w.pos, None, w.box, 5.1), spec)
    A = np.zeros((w.n_atoms, m.aev_stride), np.float32)
    A[:, :spec.aev_dim] = ref_aev
    e, g = nnp.nnp_mlp(m, torch.from_numpy(w.species).to(dev()), torch.from_numpy(A).to(dev()))
    E_ref, g_ref = oracle.mlp_energy_and_grad(A[:, :spec.aev_dim].astype(np.float64), w.species, spec,
                                              "bf16" if precision == "bf16" else "fp64")
    rms = np.sqrt(np.mean(E_ref ** 2))
    emed, emax = bf16_flip_error(e.cpu().numpy(), E_ref, rms)
    gmed, gmax = bf16_flip_error(g.cpu().numpy()[:, :spec.aev_dim], g_ref, np.abs(g_ref).max())
    print("generic widths mlp-only %s (median, max): E/rms %.3g %.3g, dE/dAEV %.3g %.3g"
          % (precision, emed, emax, gmed, gmax))
    if precision == "fp32":
        assert emax < 1e-5 and gmax < 1e-5
    else:
        assert emed < 2e-6 and emax < 1e-2 and gmed < 2e-6 and gmax < 1e-2


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_generic_widths_parity(precision):
    """Widths other than 1008-256-192-160-1 run the per-layer GEMM path."""
    import synthetic.weights as sw
    spec = synthetic.ani2x_like_spec(weight_seed=99, bias_scale=0.05)
    spec.widths = (1008, 128, 64, 96, 1)
    spec.weights = sw.glorot_weights(7, spec.widths, 99, 0.05)
    m = nnp.Model(spec, precision)
    w = organic(1500)
    pos, sp, _ = to_dev(w)
    nl = nnp.nnp_neighbors(m, pos, None, 1, w.box, 5.1)
    e_mol, e_atom, F = nnp.nnp_energy_forces(m, pos, sp, None, 1, w.box, nl, e_atom=True)
    ref = oracle_ef(w, spec, precision="bf16" if precision == "bf16" else "fp64")
    ee = energy_error(e_atom.cpu().numpy(), ref["E_atom"])
    ea = np.abs(e_atom.cpu().numpy() - ref["E_atom"]).max()
    fe = np.abs(F.cpu().numpy() - ref["F"]).max()
    rms = np.sqrt(np.mean(ref["E_atom"] ** 2))
    print("generic widths %s: E_atom err %.3g (abs %.3g eV, rms E %.3g eV), F err %.3g"
          % (precision, ee, ea, rms, fe))
    if precision == "fp32":
        assert ee < E_ATOM_REL and fe < F_MAX_ABS
    else:
        emed, emax = bf16_flip_error(e_atom.cpu().numpy(), ref["E_atom"], rms)
        print("generic widths bf16 vs emulation (median, max): E/rms %.3g %.3g" % (emed, emax))
        assert emed < 1e-5 and emax < 1e-2 and fe < 2e-2


@pytest.mark.parametrize("path", ["fused", "per_layer"])
@pytest.mark.parametrize("name", ["organic_3000", "water_box_192", "serving_batch"])
def test_bf16_form_within_error_model(spec_bias, path, name):
    """The BF16-MLP form against the FP64 oracle, gated by bounds derived
    from the bfloat16 unit roundoff: every atomic energy within 6 sigma of
    the first-order error model (plus the FP32 allowance), every structure
    energy within 6 sigma of its own (the weight roundings are shared by all
    atoms of a species), every force component within 8 x its atom's spread
    under the oracle re-run in Monte Carlo arithmetic.  Against the oracle's emulation of the same
    rounding points it agrees to float32 accumulation for the median atom."""
    m = nnp.Model(spec_bias, "bf16")
    m.set_fused_mlp(path == "fused")
    w = {"organic_3000": lambda: organic(3000), "water_box_192": lambda: synthetic.geometry.small_water_box(64),
         "serving_batch": lambda: synthetic.workload(4, n_mol=24)}[name]()
    pos, sp, mol = to_dev(w)
    nl = nnp.nnp_neighbors(m, pos, mol, w.n_mol, w.box, 5.1)
    e_mol, e_atom, F = nnp.nnp_energy_forces(m, pos, sp, mol, w.n_mol, w.box, nl, e_atom=True)
    ref = oracle_ef(w, spec_bias)
    emu = oracle.energy_forces(w.pos, w.species, w.mol if w.n_mol > 1 else None, w.n_mol, w.box, spec_bias,
                               nl=ref["nl"], precision="bf16")
    e_mol, e_atom, F = e_mol.cpu().numpy(), e_atom.cpu().numpy(), F.cpu().numpy()
    ra, rm = bf16_energy_gate(e_atom, e_mol, ref, w, spec_bias)
    sig = bf16_force_sigma(w.pos, w.species, w.box, spec_bias, ref)
    spread = float(np.sqrt(np.mean(sig ** 2)))
    rf, rr = bf16_force_gate(F, ref["F"], sig)
    print("bf16 %s %s vs fp64: E_atom %.3g, E_mol %.3g, F max %.3g rms %.3g (MC spread %.3g); bound ratios: "
          "E_atom %.3f E_mol %.3f F max %.3f F rms %.3f; vs emulation: E_atom %.3g F max %.3g"
          % (path, name, energy_error(e_atom, ref["E_atom"]), e_mol_error(e_mol, ref, w, spec_bias),
             np.abs(F - ref["F"]).max(), np.sqrt(np.mean((F - ref["F"]) ** 2)), spread, ra, rm, rf, rr,
             energy_error(e_atom, emu["E_atom"]), np.abs(F - emu["F"]).max()))
    assert ra <= 1.0 and rm <= 1.0 and rf <= 1.0 and rr <= 1.0
    rms = np.sqrt(np.mean((emu["E_atom"] - np.asarray(spec_bias.self_energy)[w.species]) ** 2))
    emed, _ = bf16_flip_error(e_atom, emu["E_atom"], rms)
    assert emed < 2e-6


def test_autograd_matches_finite_differences(model, spec_bias):
    """NNPEnergy's gradient (the hand-written adjoint through autograd)
    against central differences of the energy the same GPU path computes
    (forces are minus the energy gradient, Sec. 2.4).  Richardson
    extrapolation of steps h and h/2 removes the h^2 term; what is left is
    the float32 energy noise divided by h."""
    w = synthetic.workload(4, n_mol=3)
    pos, sp, mol = to_dev(w)
    x = pos.clone().requires_grad_(True)
    E = nnp.energy(model, x, sp, mol, w.n_mol, None)
    E.sum().backward()
    grad = x.grad.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(8)
    picks = [(int(a), int(k)) for a, k in zip(rng.choice(w.n_atoms, 12, replace=False), rng.integers(0, 3, 12))]
    x0 = w.pos.astype(np.float64)

    def e_at(a, k, h):
        y = x0.copy()
        y[a, k] += h
        yt = torch.from_numpy(y.astype(np.float32)).to(dev())
        hh = float(np.float32(y[a, k]) - np.float32(x0[a, k]))     # the step the float32 input really takes
        with torch.no_grad():
            return float(nnp.energy(model, yt, sp, mol, w.n_mol, None).sum()), hh

    errs = []
    for a, k in picks:
        fd = []
        for h in (2e-2, 1e-2):
            ep, hp = e_at(a, k, h)
            em, hm = e_at(a, k, -h)
            fd.append((ep - em) / (hp - hm))
        rich = (4.0 * fd[1] - fd[0]) / 3.0
        errs.append(abs(rich - grad[a, k]))
    scale = np.abs(grad).max()
    print("autograd vs central differences: max |diff| %.3g eV/A (max |dE/dx| %.3g)" % (max(errs), scale))
    assert max(errs) < 2e-3 + 1e-3 * scale


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


@pytest.mark.parametrize("case", ["organic_box", "batch"])
def test_virial_parity(spec_bias, case):
    if case == "organic_box":
        w = organic(2000)
    else:
        w = synthetic.workload(4, n_mol=12)
    m = nnp.Model(spec_bias, "fp32")
    pos, sp, mol = to_dev(w)
    nl = nnp.nnp_neighbors(m, pos, mol, w.n_mol, w.box, 5.1)
    out = {}
    nnp.nnp_energy_forces(m, pos, sp, mol, w.n_mol, w.box, nl, out=out, virial=True, atom_virial=True)
    ref = oracle.energy_forces(w.pos, w.species, w.mol if w.n_mol > 1 else None, w.n_mol, w.box, spec_bias,
                               need_virial=True)
    Wm = out["virial"].cpu().numpy()
    Wa = out["atom_virial"].cpu().numpy()
    sa = np.abs(ref["W_atom"]).max()
    ea = np.abs(Wa - ref["W_atom"]).max() / sa
    em = np.abs(Wm - ref["W_mol"]).max() / max(np.abs(ref["W_mol"]).max(), sa)
    print("virial %s: per-atom max err %.3g, per-structure %.3g (of scale %.3g eV)" % (case, ea, em, sa))
    assert ea < 2e-5 and em < 2e-5
    # the forces of the virial call are those of the plain call
    _, _, F = nnp.nnp_energy_forces(m, pos, sp, mol, w.n_mol, w.box, nl)
    assert torch.equal(F, out["forces"])


@pytest.mark.parametrize("case", ["organic_box", "batch"])
def test_ensemble_parity(case):
    """Ensemble of eight networks on one AEV: mean energies and forces and
    every network's structure energies against the oracle (FP32)."""
    spec = synthetic.ani2x_like_ensemble(n_nets=8, weight_seed=4242, bias_scale=0.05,
                                         self_energy=np.array([-0.6, -38.0, -54.7, -75.1, -99.8, -398.1, -460.1]))
    w = organic(1500) if case == "organic_box" else synthetic.workload(4, n_mol=10)
    m = nnp.Model(spec, "fp32")
    assert m.n_nets == 8 and m.fused_mlp
    pos, sp, mol = to_dev(w)
    nl = nnp.nnp_neighbors(m, pos, mol, w.n_mol, w.box, 5.1)
    e_mol, e_net, e_atom, F = nnp.nnp_energy_forces_ensemble(m, pos, sp, mol, w.n_mol, w.box, nl, e_atom=True)
    ref = oracle.energy_forces(w.pos, w.species, w.mol if w.n_mol > 1 else None, w.n_mol, w.box, spec,
                               need_nets=True)
    ee = energy_error(e_atom.cpu().numpy(), ref["E_atom"])
    fe = np.abs(F.cpu().numpy() - ref["F"]).max()
    ne = np.abs(e_net.cpu().numpy() - ref["E_mol_net"]).max() / np.abs(ref["E_mol_net"]).max()
    me = np.abs(e_mol.cpu().numpy() - ref["E_mol"]).max() / np.abs(ref["E_mol"]).max()
    print("ensemble %s: E_atom err %.3g, E_mol rel %.3g, per-net E_mol rel %.3g, F max %.3g"
          % (case, ee, me, ne, fe))
    assert ee < E_ATOM_REL and me < 1e-5 and ne < 1e-5 and fe < F_MAX_ABS
    # the plain entry point gives the same mean energies and forces
    e2, _, F2 = nnp.nnp_energy_forces(m, pos, sp, mol, w.n_mol, w.box, nl)
    assert torch.equal(e2, e_mol) and torch.equal(F2, F)


def test_ensemble_bf16_matches_emulation():
    spec = synthetic.ani2x_like_ensemble(n_nets=4, weight_seed=99, bias_scale=0.05)
    w = organic(1200)
    m = nnp.Model(spec, "bf16")
    pos, sp, _ = to_dev(w)
    nl = nnp.nnp_neighbors(m, pos, None, 1, w.box, 5.1)
    _, e_atom, F = nnp.nnp_energy_forces(m, pos, sp, None, 1, w.box, nl, e_atom=True)
    emu = oracle.energy_forces(w.pos, w.species, None, 1, w.box, spec, precision="bf16")
    rms = np.sqrt(np.mean(emu["E_atom"] ** 2))
    emed, emax = bf16_flip_error(e_atom.cpu().numpy(), emu["E_atom"], rms)
    fe = np.abs(F.cpu().numpy() - emu["F"]).max()
    print("ensemble bf16 vs emulation (median, max): E/rms %.3g %.3g, F max %.3g" % (emed, emax, fe))
    assert emed < 1e-5 and emax < 1e-2 and fe < 2e-2


def test_isolated_atoms_and_sparse_features(model, spec_bias):
    """Atoms without neighbours (every feature zero) beside molecules of
    several species: the networks see only the feature blocks some atom of a
    tile can have non-zero, and the result equals the oracle's dense one."""
    mols = synthetic.workload(4, n_mol=6)
    pos = [mols.pos]
    sp = [mols.species]
    far = np.array([60.0, 60.0, 60.0], dtype=np.float32)
    for k in range(20):   # lone atoms 12 A apart, one of each species in turn
        pos.append((far + np.float32(12.0) * np.array([k % 4, (k // 4) % 4, k // 16], np.float32))[None, :])
        sp.append(np.array([k % spec_bias.n_species], np.int32))
    P = np.concatenate(pos).astype(np.float32)
    S = np.concatenate(sp).astype(np.int32)
    # the molecules keep their own ids; each lone atom is a structure of its own
    M = np.concatenate([mols.mol, mols.n_mol + np.arange(20)]).astype(np.int32)
    w = synthetic.geometry.Workload("molecules_and_lone_atoms", P, S, M, mols.n_mol + 20, None)
    x, s_, m_ = to_dev(w)
    nl = nnp.nnp_neighbors(model, x, m_, w.n_mol, None, 5.1)
    e_mol, e_atom, F = nnp.nnp_energy_forces(model, x, s_, m_, w.n_mol, None, nl, e_atom=True)
    torch.cuda.synchronize()
    nnp.nnp_check(model)
    ref = oracle_ef(w, spec_bias, r_list=5.1)
    ee = energy_error(e_atom.cpu().numpy(), ref["E_atom"])
    fe = np.max(np.abs(F.cpu().numpy() - ref["F"]))
    em = e_mol_error(e_mol.cpu().numpy(), ref, w, spec_bias)
    print("isolated + molecules: E_atom err %.3g, E_mol err %.3g, F max err %.3g" % (ee, em, fe))
    assert ee < E_ATOM_REL and em < E_MOL_REL and fe < F_MAX_ABS


def test_angular_neighbour_limit(model, spec_bias):
    """A compact cluster, every atom within 3.4 A of a central one: 25 to 92
    angular neighbours per atom (the limit is NNP_MAX_ANGULAR = 96), 4,186
    angular pairs for the centre, bins of one species and of two, so the
    kernels' pair enumeration runs over pair counts up to the limit."""
    rng = np.random.default_rng(41)
    n = 93
    pts = [np.zeros(3)]
    while len(pts) < n:   # uniform in the ball, at least 0.7 A apart
        p = rng.uniform(-3.4, 3.4, 3)
        if np.linalg.norm(p) <= 3.4 and min(np.linalg.norm(p - q) for q in pts) >= 0.7:
            pts.append(p)
    P = (np.array(pts) + 20.0).astype(np.float32)
    S = rng.integers(0, 4, size=n).astype(np.int32)
    d = np.linalg.norm(P[:, None] - P[None], axis=2)
    assert ((d < 3.5) & (d > 0)).sum(axis=1).max() == 92
    w = synthetic.geometry.Workload("angular_limit_cluster", P, S, np.zeros(n, np.int32), 1, None)
    x, s_, _ = to_dev(w)
    nl = nnp.nnp_neighbors(model, x, None, 1, None, 5.1)
    e_mol, e_atom, F = nnp.nnp_energy_forces(model, x, s_, None, 1, None, nl, e_atom=True)
    torch.cuda.synchronize()
    nnp.nnp_check(model)
    ref = oracle_ef(w, spec_bias, r_list=5.1)
    ee = energy_error(e_atom.cpu().numpy(), ref["E_atom"])
    fe = np.max(np.abs(F.cpu().numpy() - ref["F"]))
    print("angular limit cluster: E_atom err %.3g, F max err %.3g eV/A (max |F| %.3g)" % (ee, fe, np.abs(ref["F"]).max()))
    assert ee < E_ATOM_REL and fe < F_MAX_ABS
