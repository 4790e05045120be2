"""Pins of the FP64 oracle against facts fixed by the paper and by
mathematics: brute-force enumeration, closed forms, library routines,
invariances, smoothness at the cutoffs, finite differences, zero net force
and torque, batch additivity.  CPU only."""
import math

import numpy as np
import pytest
import torch

import oracle
import synthetic
from synthetic.geometry import Workload, small_water_box
from tests import brute


def _pairset(nl):
    i, j, n = nl
    return sorted((int(a), int(b), tuple(int(x) for x in s)) for a, b, s in zip(i, j, n))


# ---------------------------------------------------------------- neighbours

@pytest.mark.parametrize("case", synthetic.adversarial_cases(), ids=lambda c: c.name)
def test_neighbors_match_brute_force_adversarial(case):
    r_list = 5.1
    if case.box is not None and np.any(case.box < 2 * np.float32(r_list)):
        with pytest.raises(ValueError):
            oracle.neighbor_list(case.pos, case.mol, case.box, r_list)
        return
    nl = oracle.neighbor_list(case.pos, case.mol, case.box, r_list)
    bf = oracle.brute_force_pairs(case.pos, case.mol, case.box, r_list)
    assert _pairset(nl) == [(i, j, tuple(n)) for i, j, n in bf]


def test_neighbors_exact_cutoff_is_excluded():
    case = synthetic.adversarial_cases()[0]     # atoms 0-1 exactly r_list apart
    i, j, _ = oracle.neighbor_list(case.pos, case.mol, None, 5.1)
    pairs = set(zip(i.tolist(), j.tolist()))
    assert (0, 1) not in pairs and (1, 0) not in pairs
    assert (0, 2) in pairs and (0, 3) in pairs and (2, 0) in pairs


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_neighbors_match_brute_force_random_periodic(seed):
    rng = np.random.default_rng(seed)
    L = np.float32(11.5)
    box = np.array([L, L, np.float32(13.0)], dtype=np.float32)
    pos = (rng.uniform(-1, 2, size=(40, 3)) * box).astype(np.float32)
    nl = oracle.neighbor_list(pos, None, box, 5.6)
    bf = oracle.brute_force_pairs(pos, None, box, 5.6, max_image=4)
    assert _pairset(nl) == [(i, j, tuple(n)) for i, j, n in bf]
    assert len(bf) > 0


def test_neighbors_symmetric_and_sorted():
    w = small_water_box(40)
    i, j, n = oracle.neighbor_list(w.pos, w.mol, w.box, 5.6)
    key = i * w.n_atoms + j
    assert np.all(np.diff(key) > 0)
    fwd = {(a, b): tuple(s) for a, b, s in zip(i.tolist(), j.tolist(), n.tolist())}
    for (a, b), s in fwd.items():
        assert fwd[(b, a)] == tuple(-x for x in s)


def test_neighbors_relabel_invariant():
    w = small_water_box(30)
    perm = np.random.default_rng(3).permutation(w.n_atoms)
    nl = oracle.neighbor_list(w.pos, None, w.box, 5.1)
    nl2 = oracle.neighbor_list(w.pos[perm], None, w.box, 5.1)
    inv = np.argsort(perm)
    mapped = sorted((int(perm[a]), int(perm[b]), tuple(s)) for a, b, s in
                    zip(nl2[0].tolist(), nl2[1].tolist(), nl2[2].tolist()))
    assert mapped == _pairset(nl)


@pytest.mark.parametrize("case", synthetic.adversarial_cases(), ids=lambda c: c.name)
def test_cell_search_matches_brute_force_adversarial(case):
    """The cell-binned search finds the same edge set as the pure-Python
    enumeration over periodic images on the adversarial cases (atoms on cell
    faces, at L - ulp, pairs exactly at the cutoff, a 2-cell-thin box)."""
    r_list = 5.1
    if case.box is not None and np.any(case.box < 2 * np.float32(r_list)):
        with pytest.raises(ValueError):
            oracle.neighbor_list_cells(case.pos, case.mol, case.box, r_list)
        return
    nl = oracle.neighbor_list_cells(case.pos, case.mol, case.box, r_list)
    bf = oracle.brute_force_pairs(case.pos, case.mol, case.box, r_list)
    assert _pairset(nl) == [(i, j, tuple(n)) for i, j, n in bf]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cell_search_matches_brute_force_random_periodic(seed):
    rng = np.random.default_rng(seed)
    box = np.array([11.5, 11.5, 13.0], dtype=np.float32)      # 2 cells per axis: the stencil wraps onto itself
    pos = (rng.uniform(-1, 2, size=(40, 3)) * box).astype(np.float32)
    nl = oracle.neighbor_list_cells(pos, None, box, 5.6)
    bf = oracle.brute_force_pairs(pos, None, box, 5.6, max_image=4)
    assert _pairset(nl) == [(i, j, tuple(n)) for i, j, n in bf]


@pytest.mark.parametrize("shape", ["cubic", "thin", "open_mols"])
def test_cell_search_matches_all_pairs_scan(shape):
    """Same (i, j, image) arrays, in the same order, as the O(N^2) scan of
    the definition, on boxes of several cells per axis (3-cell and 2-cell
    axes, coordinates far outside the box) and on an open system of several
    structures."""
    rng = np.random.default_rng({"cubic": 10, "thin": 11, "open_mols": 12}[shape])
    mol = None
    if shape == "cubic":
        box = np.array([23.0, 26.0, 31.5], dtype=np.float32)
        pos = (rng.uniform(-2, 3, size=(900, 3)) * box).astype(np.float32)
    elif shape == "thin":
        box = np.array([10.3, 16.9, 40.0], dtype=np.float32)
        pos = (rng.uniform(0, 1, size=(700, 3)) * box).astype(np.float32)
        pos[:50, 0] = np.float32(0.0)                         # on a cell face
        pos[50:100, 1] = np.nextafter(box[1], np.float32(0))  # just below L
    else:
        box = None
        pos = rng.uniform(-15, 15, size=(600, 3)).astype(np.float32)
        mol = rng.integers(0, 4, size=600)
    a = oracle.neighbor_list(pos, mol, box, 5.1)
    b = oracle.neighbor_list_cells(pos, mol, box, 5.1)
    assert len(a[0]) > 1000
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_cell_search_matches_all_pairs_scan_water():
    w = synthetic.workload(2)
    a = oracle.neighbor_rows(w.pos, None, w.box, 5.6, np.arange(0, w.n_atoms, 7))
    b = oracle.neighbor_list_cells(w.pos, None, w.box, 5.6)
    sel = np.isin(b[0], np.arange(0, w.n_atoms, 7))
    for x, y in zip(a, b):
        assert np.array_equal(x, y[sel])


# ---------------------------------------------------------------- switching function

def test_switch_closed_form(spec):
    rc = float(np.float32(spec.rc_r))
    r = np.array([0.0, 1.3, rc * 0.5, rc - 1e-9, rc, rc + 0.1])
    f = oracle.switch(r, spec.rc_r)
    assert f[0] == 1.0
    assert abs(f[2] - 0.5) < 1e-15
    assert f[4] == 0.0 and f[5] == 0.0
    assert abs(f[1] - (0.5 * math.cos(math.pi * 1.3 / rc) + 0.5)) < 1e-15
    d = oracle.switch_deriv(np.array([rc - 1e-12, 0.0]), spec.rc_r)
    assert abs(d[0]) < 1e-10 and d[1] == 0.0
    # derivative agrees with a central difference
    x, h = 2.2, 1e-6
    fd = (oracle.switch(np.array([x + h]), spec.rc_r)[0] - oracle.switch(np.array([x - h]), spec.rc_r)[0]) / (2 * h)
    assert abs(fd - oracle.switch_deriv(np.array([x]), spec.rc_r)[0]) < 1e-9


# ---------------------------------------------------------------- AEV closed forms

def test_radial_two_atoms_closed_form(spec):
    p = brute.params_of(spec)
    for r, (za, zb) in [(0.97, (0, 3)), (2.5, (1, 6)), (4.9, (5, 5))]:
        pos = np.array([[0, 0, 0], [r, 0, 0]], dtype=np.float32)
        sp = np.array([za, zb], dtype=np.int32)
        nl = oracle.neighbor_list(pos, None, None, 5.1)
        A = oracle.aev(pos, sp, None, nl, spec)
        rr = float(np.float32(r))
        for k in range(16):
            want = p["pr"] * math.exp(-p["eta_r"] * (rr - p["shf_r"][k]) ** 2) * brute.fc(rr, p["rc_r"])
            assert abs(A[0, 16 * zb + k] - want) <= 1e-15 + 1e-13 * abs(want)
            assert abs(A[1, 16 * za + k] - want) <= 1e-15 + 1e-13 * abs(want)
        mask = np.ones(1008, bool)
        mask[16 * zb:16 * zb + 16] = False
        assert np.all(A[0, mask] == 0.0)


def _closed_form_angular(pos, sp, i, j, k, p):
    vj = [pos[j][c] - pos[i][c] for c in range(3)]
    vk = [pos[k][c] - pos[i][c] for c in range(3)]
    rj = math.sqrt(sum(x * x for x in vj))
    rk = math.sqrt(sum(x * x for x in vk))
    cos_t = sum(a * b for a, b in zip(vj, vk)) / (rj * rk)
    th = math.acos(p["cs"] * cos_t)
    out = {}
    pi = brute.pair_index(sp[j], sp[k])
    for a in range(4):
        for z in range(8):
            val = 2 * (0.5 + 0.5 * math.cos(th - p["shf_z"][z])) ** p["zeta"] \
                * math.exp(-p["eta_a"] * ((rj + rk) / 2 - p["shf_a"][a]) ** 2) \
                * brute.fc(rj, p["rc_a"]) * brute.fc(rk, p["rc_a"])
            out[112 + 32 * pi + 8 * a + z] = val
    return out


def test_angular_three_atoms_closed_form(spec):
    p = brute.params_of(spec)
    th = math.radians(104.52)
    geoms = [
        ([[0, 0, 0], [0.9572, 0, 0], [0.9572 * math.cos(th), 0.9572 * math.sin(th), 0]], [3, 0, 0]),
        ([[0, 0, 0], [1.4, 0, 0], [0, 1.1, 0]], [1, 2, 6]),                      # right angle
        ([[0, 0, 0], [1.0, 0.2, 0.1], [-2.1, 0.3, 0.4]], [4, 5, 0]),              # obtuse
    ]
    for pts, sp in geoms:
        pos = np.array(pts, dtype=np.float32)
        sp = np.array(sp, dtype=np.int32)
        nl = oracle.neighbor_list(pos, None, None, 5.1)
        A = oracle.aev(pos, sp, None, nl, spec)
        P = pos.astype(np.float64).tolist()
        for i, j, k in [(0, 1, 2), (1, 0, 2), (2, 0, 1)]:
            want = _closed_form_angular(P, sp, i, j, k, p)
            ang = A[i, 112:]
            for col, val in want.items():
                assert abs(A[i, col] - val) <= 1e-14 + 1e-12 * abs(val), (i, col)
            nz = np.nonzero(ang)[0] + 112
            assert set(nz.tolist()) <= set(want.keys())


@pytest.mark.parametrize("seed", [0, 1])
def test_aev_matches_pure_python_loops(spec, seed):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 4.0, size=(9, 3)).astype(np.float32)
    sp = rng.integers(0, 7, size=9).astype(np.int32)
    nl = oracle.neighbor_list(pos, None, None, 5.1)
    A = oracle.aev(pos, sp, None, nl, spec)
    B = np.array(brute.aev_brute(pos.astype(np.float64).tolist(), sp.tolist(), brute.params_of(spec)))
    assert np.max(np.abs(A - B)) <= 1e-12 * max(1.0, np.max(np.abs(B)))
    assert np.count_nonzero(B[:, 112:]) > 0


# ---------------------------------------------------------------- MLP vs library routines

@pytest.mark.parametrize("which", ["spec", "spec_bias"])
def test_mlp_matches_torch_fp64(request, which):
    sp_ = request.getfixturevalue(which)
    rng = np.random.default_rng(11)
    A = rng.normal(scale=0.5, size=(30, 1008))
    Z = rng.integers(0, 7, size=30)
    E, g = oracle.mlp_energy_and_grad(A, Z, sp_)
    x = torch.tensor(A, dtype=torch.float64, requires_grad=True)
    outs = []
    for a in range(30):
        h = x[a]
        layers = sp_.weights[Z[a]]
        for l, (W, b) in enumerate(layers):
            h = torch.nn.functional.linear(h, torch.tensor(W, dtype=torch.float64), torch.tensor(b, dtype=torch.float64))
            if l < len(layers) - 1:
                h = torch.nn.functional.celu(h, alpha=float(np.float32(sp_.celu_alpha)))
        outs.append(h[0] + float(sp_.self_energy[Z[a]]))
    Et = torch.stack(outs)
    Et.sum().backward()
    assert np.max(np.abs(E - Et.detach().numpy())) < 1e-12
    assert np.max(np.abs(g - x.grad.numpy())) < 1e-12


def test_round_bf16_matches_torch():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.normal(size=10000) * 10.0 ** rng.integers(-8, 8, size=10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38]])
    x32 = x.astype(np.float32)
    want = torch.tensor(x32).to(torch.bfloat16).to(torch.float64).numpy()
    got = oracle.round_bf16(x32)
    assert np.array_equal(got, want)


# ---------------------------------------------------------------- BF16 form: rounding points and error model

def _bf16_case(spec_bias, n=300):
    """Features of an organic-like box (every species present) and the
    model with U(+-0.1) biases."""
    w = synthetic.organic_box(n=n, density=0.1, seed=31)
    A = oracle.aev(w.pos, w.species, w.box, oracle.neighbor_list(w.pos, None, w.box, 5.1), spec_bias)
    return A, w.species


def _with_weights(spec, fn):
    """A copy of the model whose (W, b) of species s, layer l are fn(l, W, b)."""
    import copy
    out = copy.copy(spec)
    out.weights = [[fn(l, W, b) for l, (W, b) in enumerate(layers)] for layers in spec.weights]
    return out


def _bf16_f32(x):
    return oracle.round_bf16(x).astype(np.float32)


def _n_changed(a, b):
    a, b = np.asarray(a), np.asarray(b)
    if a.ndim > 1:
        return int(np.sum(np.any(a != b, axis=1)))
    return int(np.sum(a != b))


@pytest.mark.parametrize("layer,rounded", [(0, True), (1, True), (2, True), (3, False)])
def test_bf16_weights_enter_rounded_where_stated(spec_bias, layer, rounded):
    """The BF16 form sees W1..W3 only through their bfloat16 values (rounding
    them beforehand changes nothing, bit for bit) and the head's w4 in full
    precision (rounding it changes every energy)."""
    A, Z = _bf16_case(spec_bias)
    E0, g0 = oracle.mlp_energy_and_grad(A, Z, spec_bias, "bf16")
    pre = _with_weights(spec_bias, lambda l, W, b: (_bf16_f32(W) if l == layer else W, b))
    E1, g1 = oracle.mlp_energy_and_grad(A, Z, pre, "bf16")
    if rounded:
        assert np.array_equal(E0, E1) and np.array_equal(g0, g1)
    else:
        assert _n_changed(E0, E1) > 0.9 * len(Z)


def test_bf16_features_enter_rounded(spec_bias):
    A, Z = _bf16_case(spec_bias)
    E0, g0 = oracle.mlp_energy_and_grad(A, Z, spec_bias, "bf16")
    E1, g1 = oracle.mlp_energy_and_grad(oracle.round_bf16(A), Z, spec_bias, "bf16")
    assert np.array_equal(E0, E1) and np.array_equal(g0, g1)
    # control: the exact network sees the unrounded features
    assert _n_changed(oracle.mlp_energy(A, Z, spec_bias), oracle.mlp_energy(oracle.round_bf16(A), Z, spec_bias)) \
        > 0.9 * len(Z)


def _nudge(spec, layer, which):
    """Every bias of one layer (which = 'b') or the head's weights ('W', layer
    3 only) moved up by one float32 ulp: a change far below one bfloat16 step
    of the activations it feeds."""
    def f(l, W, b):
        if l != layer:
            return W, b
        if which == "b":
            return W, np.nextafter(b, np.float32(np.inf)).astype(np.float32)
        return np.nextafter(W, np.float32(np.inf)).astype(np.float32), b
    return _with_weights(spec, f)


@pytest.mark.parametrize("layer,feeds_rounded", [(0, True), (1, True), (2, False)])
def test_bf16_hidden_activations_enter_rounded(spec_bias, layer, feeds_rounded):
    """h1 and h2 enter the next product as bfloat16 values: nudging the bias
    that produces them (one float32 ulp) leaves the next layer's
    pre-activations of every atom unchanged except where an activation sits
    within that nudge of a bfloat16 rounding boundary (a few per thousand).
    h3 feeds the full-precision head: nudging b3 moves every energy.  The
    exact network moves every atom in all three cases."""
    A, Z = _bf16_case(spec_bias)
    moved = _nudge(spec_bias, layer, "b")
    if feeds_rounded:
        a, b = oracle.mlp_trace(A, Z, spec_bias, "bf16"), oracle.mlp_trace(A, Z, moved, "bf16")
        nb = _n_changed(a["z"][layer + 1], b["z"][layer + 1])
        a64, b64 = oracle.mlp_trace(A, Z, spec_bias), oracle.mlp_trace(A, Z, moved)
        n64 = _n_changed(a64["z"][layer + 1], b64["z"][layer + 1])
        assert n64 > 0.9 * len(Z) and nb < 0.05 * len(Z)
    else:
        nb = _n_changed(oracle.mlp_energy(A, Z, spec_bias, "bf16"), oracle.mlp_energy(A, Z, moved, "bf16"))
        assert nb > 0.9 * len(Z)


@pytest.mark.parametrize("nudge", ["w4", "b2", "b1"])
def test_bf16_adjoint_inputs_enter_rounded(spec_bias, nudge):
    """d3 = w4 CELU'(z3), d2 and d1 enter their adjoint products as bfloat16
    values.  Nudging w4 changes d3 continuously, nudging b2 (b1) changes
    CELU'(z2) (CELU'(z1)) and so d2 (d1): the product each one feeds
    (W3^T d3, W2^T d2, W1^T d1 = dE/dAEV) stays put for all but the atoms with
    a value within the nudge of a rounding boundary, while the exact
    network's moves for every atom."""
    A, Z = _bf16_case(spec_bias)
    layer, which, key = {"w4": (3, "W", ("p", 2)), "b2": (1, "b", ("p", 1)), "b1": (0, "b", ("g", None))}[nudge]
    moved = _nudge(spec_bias, layer, which)

    def product(tr):
        return tr["g"] if key[0] == "g" else tr["p"][key[1]]
    nb = _n_changed(product(oracle.mlp_trace(A, Z, spec_bias, "bf16")), product(oracle.mlp_trace(A, Z, moved, "bf16")))
    n64 = _n_changed(product(oracle.mlp_trace(A, Z, spec_bias)), product(oracle.mlp_trace(A, Z, moved)))
    assert n64 > 0.9 * len(Z)
    assert nb < 0.05 * len(Z)


def test_bf16_energy_sigma_matches_monte_carlo_arithmetic(spec_bias):
    """The first-order error model (closed form through the exact adjoint)
    against Monte Carlo arithmetic at the same rounding points (the network
    re-run with random relative perturbations of size u): per atom and per
    structure, the sampled spread equals the closed form."""
    A, Z = _bf16_case(spec_bias)
    E64, _ = oracle.mlp_energy_and_grad(A, Z, spec_bias, need_grad=False)
    sa, sm = oracle.bf16_energy_sigma(A, Z, spec_bias)
    rng = np.random.default_rng(0)
    dev = np.array([oracle.mlp_energy_and_grad(A, Z, spec_bias, "mca", need_grad=False, rng=rng)[0] - E64
                    for _ in range(48)])
    ratio = np.sqrt(np.mean(dev ** 2, axis=0)) / sa
    mol = np.sqrt(np.mean(dev.sum(1) ** 2)) / sm[0]
    print("MC / closed form: per atom median %.3f (10-90%%: %.3f-%.3f), structure %.3f"
          % (np.median(ratio), np.quantile(ratio, 0.1), np.quantile(ratio, 0.9), mol))
    assert 0.9 < np.median(ratio) < 1.1
    assert 0.7 < mol < 1.4


def test_bf16_emulation_error_within_model(spec_bias):
    """The deterministic emulation's errors against the exact network are
    of the size the unit roundoff predicts: normalised by the closed-form
    sigma, rms below 1 (round-to-nearest errors are smaller than the
    uniform model's) and no atom beyond 5 sigma; a form without roundings
    would sit orders of magnitude lower."""
    A, Z = _bf16_case(spec_bias)
    E64, _ = oracle.mlp_energy_and_grad(A, Z, spec_bias, need_grad=False)
    Eb, _ = oracle.mlp_energy_and_grad(A, Z, spec_bias, "bf16", need_grad=False)
    sa, _ = oracle.bf16_energy_sigma(A, Z, spec_bias)
    z = (Eb - E64) / sa
    print("emulation error / sigma: rms %.3f, max %.3f" % (np.sqrt(np.mean(z ** 2)), np.abs(z).max()))
    assert 0.2 < np.sqrt(np.mean(z ** 2)) < 1.0
    assert np.abs(z).max() < 5.0


# ---------------------------------------------------------------- invariances

def _fixed_list_energy(x64, sp, box, spec, nl):
    return oracle.total_energy(x64, sp, box, spec, nl)


def test_energy_rotation_translation_invariance(spec):
    w = synthetic.workload(1)
    nl = oracle.neighbor_list(w.pos, None, None, 7.0)      # margin: list stays valid under motion
    x = w.pos.astype(np.float64)
    E0 = _fixed_list_energy(x, w.species, None, spec, nl)
    R = synthetic.geometry.random_rotations(np.random.default_rng(2), 1)[0]
    E1 = _fixed_list_energy(x @ R.T + np.array([3.3, -1.7, 40.0]), w.species, None, spec, nl)
    assert abs(E1 - E0) <= 1e-12 * abs(E0)


def test_energy_permutation_invariance(spec):
    w = synthetic.workload(1)
    rng = np.random.default_rng(4)
    perm = rng.permutation(w.n_atoms)
    a = oracle.energy_forces(w.pos, w.species, None, 1, None, spec, need_forces=True)
    b = oracle.energy_forces(w.pos[perm], w.species[perm], None, 1, None, spec, need_forces=True)
    assert abs(a["E_mol"][0] - b["E_mol"][0]) <= 1e-12 * abs(a["E_mol"][0])
    assert np.max(np.abs(a["E_atom"][perm] - b["E_atom"])) < 1e-13
    assert np.max(np.abs(a["F"][perm] - b["F"])) < 1e-12


def test_periodic_wrap_invariance(spec):
    rng = np.random.default_rng(9)
    L = 16.0
    pos = (np.round(rng.uniform(0, L, size=(60, 3)) * 1024) / 1024).astype(np.float32)
    sp = rng.integers(0, 7, size=60).astype(np.int32)
    box = np.array([L, L, L], np.float32)
    shifted = np.mod(pos.astype(np.float64) + np.array([3.125, -5.5, 7.0]), L).astype(np.float32)
    a = oracle.energy_forces(pos, sp, None, 1, box, spec)
    b = oracle.energy_forces(shifted, sp, None, 1, box, spec)
    assert abs(a["E_mol"][0] - b["E_mol"][0]) <= 1e-12 * max(1.0, abs(a["E_mol"][0]))
    assert np.max(np.abs(a["F"] - b["F"])) < 1e-12
    # a whole-box image shift of one atom changes nothing either
    moved = pos.copy()
    moved[5, 0] += np.float32(L)
    c = oracle.energy_forces(moved, sp, None, 1, box, spec)
    assert abs(a["E_mol"][0] - c["E_mol"][0]) <= 1e-12 * max(1.0, abs(a["E_mol"][0]))


# ---------------------------------------------------------------- smoothness at the cutoffs

@pytest.mark.parametrize("which", ["radial", "angular"])
def test_smooth_decay_at_cutoff(spec_bias, which):
    sp = np.array([1, 3, 0], np.int32)
    rc = float(np.float32(spec_bias.rc_r if which == "radial" else spec_bias.rc_a))

    def energy(r):
        if which == "radial":
            x = np.array([[0, 0, 0], [r, 0, 0], [0, 9.0, 0]], dtype=np.float64)
        else:     # atom 2 stays well inside both cutoffs of atom 0; atom 1 crosses rc_a
            x = np.array([[0, 0, 0], [r, 0.0, 0], [0, 1.2, 0]], dtype=np.float64)
        nl = oracle.neighbor_list(x.astype(np.float32), None, None, 12.0)
        return oracle.total_energy(x, sp, None, spec_bias, nl)

    # E is C1 across the cutoff: the centred second difference scales as d^2
    # (a jump in E or in dE/dr would make it scale as 1 or d)
    sd = [abs(energy(rc + d) - 2 * energy(rc) + energy(rc - d)) for d in (1e-3, 1e-4)]
    assert sd[1] < sd[0] / 30 or sd[1] < 1e-13, sd
    # the feature columns fed by the crossing pair decay to zero quadratically
    def feats(r):
        x = np.array([[0, 0, 0], [r, 0.0, 0], [0, 1.2, 0]], dtype=np.float32)
        nl = oracle.neighbor_list(x, None, None, 12.0)
        A = oracle.aev(x, sp, None, nl, spec_bias)
        return A[0, 16:32] if which == "radial" else A[0, 112:]
    for d in (1e-2, 1e-3):
        assert np.max(np.abs(feats(rc - d))) < 20 * d * d
    assert np.all(feats(rc) == 0.0) if which == "radial" else True
    assert np.all(feats(rc + 1e-3) == 0.0)
    # gradient tends to zero at the cutoff
    h = 1e-7
    slope = (energy(rc - h) - energy(rc - 3 * h)) / (2 * h)
    if which == "radial":
        assert abs(slope) < 1e-4


# ---------------------------------------------------------------- forces

def _fd_forces(x64, sp, box, spec, nl, atoms, h=1e-5):
    F = np.zeros((len(atoms), 3))
    for a_i, a in enumerate(atoms):
        for k in range(3):
            xp = x64.copy()
            xm = x64.copy()
            xp[a, k] += h
            xm[a, k] -= h
            F[a_i, k] = -(oracle.total_energy(xp, sp, box, spec, nl)
                          - oracle.total_energy(xm, sp, box, spec, nl)) / (2 * h)
    return F


def test_forces_match_finite_differences_cluster(spec_bias):
    w = synthetic.workload(1)
    out = oracle.energy_forces(w.pos, w.species, None, 1, None, spec_bias)
    nl = oracle.neighbor_list(w.pos, None, None, 7.0)
    atoms = list(range(0, w.n_atoms, 5))
    F_fd = _fd_forces(w.pos.astype(np.float64), w.species, None, spec_bias, nl, atoms)
    F = out["F"][atoms]
    assert np.max(np.abs(F - F_fd)) <= 1e-7 * max(1.0, np.max(np.abs(F)))


def test_forces_match_finite_differences_periodic(spec_bias):
    w = small_water_box(40)
    sp = synthetic.workload(3).species[:w.n_atoms]          # mixed species on water geometry
    out = oracle.energy_forces(w.pos, sp, None, 1, w.box, spec_bias)
    nl = oracle.neighbor_list(w.pos, None, w.box, 5.6)
    atoms = [0, 7, 31, 62, 119]
    F_fd = _fd_forces(w.pos.astype(np.float64), sp, w.box, spec_bias, nl, atoms)
    assert np.max(np.abs(out["F"][atoms] - F_fd)) <= 1e-7 * max(1.0, np.max(np.abs(F_fd)))


def _strained_atom_energies(w, sp, spec, nl, eps):
    """Atomic energies with every edge vector mapped v -> (I + eps) v (a
    homogeneous strain; with a periodic box the images strain alongside)."""
    from oracle.forces import _geometry64
    v, _ = _geometry64(w.pos.astype(np.float64), w.box, nl)
    v = v + v @ eps.T
    A = oracle.aev(None, sp, w.box, nl, spec, geometry=(v, np.sqrt(np.sum(v * v, axis=1))), n_atoms=w.n_atoms)
    return oracle.mlp_energy(A, sp, spec)


@pytest.mark.parametrize("periodic", [False, True], ids=["cluster", "box"])
def test_virial_is_the_strain_derivative(spec_bias, periodic):
    """dE_i/d eps_ab = -W_i[b, a] per atom (and so for the structure sum),
    from central differences of the atomic energies under a strain of
    every edge vector; non-symmetric per-atom components are pinned too."""
    if periodic:
        w = small_water_box(40)
        sp = synthetic.workload(3).species[:w.n_atoms]
    else:
        w = synthetic.workload(1)
        sp = w.species
    out = oracle.energy_forces(w.pos, sp, None, 1, w.box, spec_bias, need_virial=True)
    nl = out["nl"]
    W_atom, W_mol = out["W_atom"], out["W_mol"][0]
    h = 1e-6
    scale = np.max(np.abs(W_atom))
    for a in range(3):
        for b in range(3):
            eps = np.zeros((3, 3))
            eps[a, b] = h
            d = (_strained_atom_energies(w, sp, spec_bias, nl, eps)
                 - _strained_atom_energies(w, sp, spec_bias, nl, -eps)) / (2 * h)
            assert np.max(np.abs(d + W_atom[:, b, a])) <= 1e-6 * scale, (a, b)
            assert abs(d.sum() + W_mol[b, a]) <= 1e-6 * w.n_atoms * scale, (a, b)
    assert np.allclose(W_atom.sum(0), W_mol, rtol=0, atol=1e-12 * w.n_atoms * scale)


def test_virial_of_open_structure_is_sum_x_outer_F(spec_bias):
    """For an open structure W = sum_a x_a (outer) F_a, which is symmetric
    (zero net torque)."""
    w = synthetic.workload(1)
    out = oracle.energy_forces(w.pos, w.species, None, 1, None, spec_bias, need_virial=True)
    x = w.pos.astype(np.float64)
    ref = np.einsum("ia,ib->ab", x, out["F"])
    W = out["W_mol"][0]
    scale = np.max(np.abs(W))
    assert np.max(np.abs(W - ref)) <= 1e-11 * w.n_atoms * scale
    assert np.max(np.abs(W - W.T)) <= 1e-11 * w.n_atoms * scale


def test_net_force_and_torque_vanish(spec_bias):
    w = synthetic.workload(1)
    out = oracle.energy_forces(w.pos, w.species, None, 1, None, spec_bias)
    F = out["F"]
    x = w.pos.astype(np.float64)
    scale = np.max(np.abs(F))
    assert np.max(np.abs(F.sum(0))) < 1e-12 * w.n_atoms * scale
    assert np.max(np.abs(np.cross(x, F).sum(0))) < 1e-11 * w.n_atoms * scale


def test_forces_match_torch_autograd(spec_bias):
    """Third opinion: reverse-mode autodiff in float64 of an independent
    torch expression of the same energy."""
    rng = np.random.default_rng(21)
    pos = rng.uniform(0, 4.5, size=(12, 3)).astype(np.float32)
    sp = rng.integers(0, 7, size=12).astype(np.int32)
    out = oracle.energy_forces(pos, sp, None, 1, None, spec_bias)
    p = brute.params_of(spec_bias)
    x = torch.tensor(pos.astype(np.float64), requires_grad=True)
    N = len(sp)
    feats = [[torch.zeros((), dtype=torch.float64) for _ in range(1008)] for _ in range(N)]

    def tfc(r, rc):
        return 0.5 * torch.cos(math.pi * r / rc) + 0.5

    for i in range(N):
        for j in range(N):
            if i == j:
                continue
            r = torch.linalg.norm(x[j] - x[i])
            if r.item() < p["rc_r"]:
                for k in range(16):
                    feats[i][16 * sp[j] + k] = feats[i][16 * sp[j] + k] + p["pr"] * torch.exp(
                        -p["eta_r"] * (r - p["shf_r"][k]) ** 2) * tfc(r, p["rc_r"])
        for j in range(N):
            for k in range(j + 1, N):
                if i in (j, k):
                    continue
                vj, vk = x[j] - x[i], x[k] - x[i]
                rj, rk = torch.linalg.norm(vj), torch.linalg.norm(vk)
                if rj.item() >= p["rc_a"] or rk.item() >= p["rc_a"]:
                    continue
                th = torch.acos(p["cs"] * torch.dot(vj, vk) / (rj * rk))
                pi = brute.pair_index(sp[j], sp[k])
                for a in range(4):
                    f2 = torch.exp(-p["eta_a"] * ((rj + rk) / 2 - p["shf_a"][a]) ** 2)
                    for z in range(8):
                        f1 = (0.5 + 0.5 * torch.cos(th - p["shf_z"][z])) ** p["zeta"]
                        c = 112 + 32 * pi + 8 * a + z
                        feats[i][c] = feats[i][c] + 2 * f1 * f2 * tfc(rj, p["rc_a"]) * tfc(rk, p["rc_a"])
    E = torch.zeros((), dtype=torch.float64)
    for i in range(N):
        h = torch.stack(feats[i])
        layers = spec_bias.weights[sp[i]]
        for l, (W, b) in enumerate(layers):
            h = torch.nn.functional.linear(h, torch.tensor(W, dtype=torch.float64), torch.tensor(b, dtype=torch.float64))
            if l < 3:
                h = torch.nn.functional.celu(h, alpha=float(np.float32(0.1)))
        E = E + h[0] + float(spec_bias.self_energy[sp[i]])
    E.backward()
    assert abs(E.item() - out["E_mol"][0]) < 1e-10 * max(1.0, abs(E.item()))
    assert np.max(np.abs(-x.grad.numpy() - out["F"])) < 1e-10 * max(1.0, np.max(np.abs(out["F"])))


def test_batch_additivity(spec_bias):
    rng = np.random.default_rng(8)
    mA = synthetic.serving_molecule(rng, n=20)
    mB = synthetic.serving_molecule(rng, n=33)
    wb = synthetic.geometry.batch_molecules([mA, mB])
    ab = oracle.energy_forces(wb.pos, wb.species, wb.mol, 2, None, spec_bias)
    a = oracle.energy_forces(mA[0], mA[1], None, 1, None, spec_bias)
    b = oracle.energy_forces(mB[0], mB[1], None, 1, None, spec_bias)
    assert abs(ab["E_mol"][0] - a["E_mol"][0]) < 1e-12 * max(1, abs(a["E_mol"][0]))
    assert abs(ab["E_mol"][1] - b["E_mol"][0]) < 1e-12 * max(1, abs(b["E_mol"][0]))
    assert np.max(np.abs(ab["F"][:20] - a["F"])) < 1e-12
    assert np.max(np.abs(ab["F"][20:] - b["F"])) < 1e-12


def test_degenerate_inputs(spec_bias):
    # one atom: no neighbours, zero AEV, energy = output bias + self energy
    pos = np.zeros((1, 3), np.float32)
    out = oracle.energy_forces(pos, np.array([4], np.int32), None, 1, None, spec_bias)
    W4, b4 = spec_bias.weights[4][3]
    h = np.zeros(1008)
    for W, b in spec_bias.weights[4][:3]:
        h = oracle.celu(W.astype(np.float64) @ h + b, float(np.float32(0.1)))
    want = float(W4.astype(np.float64)[0] @ h + b4[0]) + spec_bias.self_energy[4]
    assert abs(out["E_mol"][0] - want) < 1e-12 * abs(want)
    assert np.all(out["F"] == 0.0) and np.all(out["aev"] == 0.0)
    # coincident atoms are legal (no repulsion in the model); angular terms stay finite
    pos = np.array([[0, 0, 0], [0, 0, 0], [1.0, 0, 0]], np.float32)
    out = oracle.energy_forces(pos, np.array([0, 0, 3], np.int32), None, 1, None, spec_bias)
    assert np.all(np.isfinite(out["E_atom"])) and np.all(np.isfinite(out["F"]))


# ---------------------------------------------------------------- MD integrator

def test_velocity_verlet_second_order_and_reversible(spec_bias):
    rng = np.random.default_rng(3)
    m = synthetic.serving_molecule(rng, n=10)
    masses = synthetic.MASSES[m[1]]
    nl = oracle.neighbor_list(m[0], None, None, 9.0)

    def ff64(x):
        return oracle.energy_forces_f64(x, m[1], None, spec_bias, nl)

    v0 = rng.normal(scale=0.01, size=(10, 3))
    drifts = []
    for dt in (0.2, 0.1):
        steps = int(round(2.0 / dt))
        _, _, en = oracle.velocity_verlet(m[0], v0, masses, ff64, dt, steps)
        tot = np.array([a + b for a, b in en])
        drifts.append(np.max(np.abs(tot - tot[0])))
    assert drifts[1] < drifts[0] / 2.5          # O(dt^2): halving dt cuts error ~4x
    # time reversibility
    xT, vT, _ = oracle.velocity_verlet(m[0], v0, masses, ff64, 0.1, 20)
    xb, vb, _ = oracle.velocity_verlet(xT, -vT, masses, ff64, 0.1, 20)
    assert np.max(np.abs(xb - m[0].astype(np.float64))) < 1e-9


def _philox4x64_10(ctr, key):
    """Philox4x64-10 from its published definition (Salmon, Moraes, Dror and
    Shaw, SC'11): 10 rounds of two 64x64->128 multiplies with a Weyl key
    schedule.  Independent of numpy's implementation used by the oracle."""
    M = (1 << 64) - 1
    c0, c1, c2, c3 = ctr
    k0, k1 = key
    for r in range(10):
        if r:
            k0, k1 = (k0 + 0x9E3779B97F4A7C15) & M, (k1 + 0xBB67AE8584CAA73B) & M
        p0, p1 = 0xD2E7470EE14C6C93 * c0, 0xCA5A826395121157 * c2
        c0, c1, c2, c3 = (p1 >> 64) ^ c1 ^ k0, p1 & M, (p0 >> 64) ^ c3 ^ k1, p0 & M
    return [c0, c1, c2, c3]


def test_philox_stream_definition():
    from oracle.md import philox_block
    # known-answer vector published with the Random123 library: counter 0, key 0
    assert _philox4x64_10([0, 0, 0, 0], [0, 0]) == [0x16554D9ECA36314C, 0xDB20FE9D672D0FDC,
                                                   0xD7E772CEE186176B, 0x7E68B68AEC7BA23B]
    for seed, step, atom in [(0, 0, 0), (2024, 7, 3), (2 ** 63 + 5, 123456, 99999)]:
        assert [int(x) for x in philox_block(seed, step, atom)] == _philox4x64_10([atom + 1, step, 0, 0], [seed, 0])


def test_baoab_without_friction_is_velocity_verlet(spec_bias):
    rng = np.random.default_rng(4)
    m = synthetic.serving_molecule(rng, n=10)
    masses = synthetic.MASSES[m[1]]
    nl = oracle.neighbor_list(m[0], None, None, 9.0)

    def ff64(x):
        return oracle.energy_forces_f64(x, m[1], None, spec_bias, nl)
    v0 = rng.normal(scale=0.01, size=(10, 3))
    xa, va, ea = oracle.velocity_verlet(m[0], v0, masses, ff64, 0.5, 6)
    xb, vb, eb = oracle.langevin_baoab(m[0], v0, masses, ff64, 0.5, 6, 300.0, 0.0, seed=1)
    assert np.max(np.abs(xa - xb)) < 1e-12 and np.max(np.abs(va - vb)) < 1e-13
    assert np.max(np.abs(np.array(ea) - np.array(eb))) < 1e-10


def test_baoab_free_particles(spec):
    """No forces: at T = 0 the O step is the exact decay v -> exp(-gamma t) v
    (gamma in 1/ps, t in fs); at T > 0 the velocities relax to the
    Maxwell-Boltzmann variance kT/m (equipartition) with standard normal noise."""
    n = 1500
    rng = np.random.default_rng(5)
    masses = rng.choice(synthetic.MASSES, size=n)
    x0 = rng.uniform(0, 10, size=(n, 3))
    v0 = rng.normal(scale=0.02, size=(n, 3))

    def free(x):
        return 0.0, np.zeros_like(x)
    _, v, _ = oracle.langevin_baoab(x0, v0, masses, free, 0.5, 4, 0.0, 50.0, seed=3)
    assert np.max(np.abs(v - v0 * np.exp(-50.0 * 1e-3 * 0.5 * 4))) < 1e-15
    xi = oracle.langevin_noise(11, 2, n)
    assert abs(xi.mean()) < 4 / np.sqrt(3 * n) and abs(xi.var() - 1.0) < 6 * np.sqrt(2 / (3 * n))
    T = 300.0
    _, v, _ = oracle.langevin_baoab(x0, np.zeros((n, 3)), masses, free, 1.0, 40, T, 200.0, seed=9)
    z = v * np.sqrt(masses[:, None] / (oracle.md.KB_EV * T * oracle.md.ACC_UNIT))
    want = 1.0 - np.exp(-2 * 200.0 * 1e-3 * 1.0 * 40)
    assert abs(z.var() - want) < 6 * np.sqrt(2 / (3 * n))


# ---------------------------------------------------------------- ensemble

def _ensemble_spec(k, seed=321):
    return synthetic.ani2x_like_ensemble(n_nets=k, weight_seed=seed, bias_scale=0.1,
                                         self_energy=np.array([-0.6, -38.0, -54.7, -75.1, -99.8, -398.1, -460.1]))


def _single(spec, k):
    import copy
    s = copy.copy(spec)
    s.weights = spec.ensemble[k]
    s.ensemble = None
    return s


def test_ensemble_is_the_mean_of_its_networks():
    """Energies, atomic energies, forces and per-network structure energies of
    a 3-network ensemble against three separate single-network evaluations."""
    spec = _ensemble_spec(3)
    w = synthetic.workload(4, n_mol=3)
    ens = oracle.energy_forces(w.pos, w.species, w.mol, w.n_mol, None, spec, need_nets=True)
    singles = [oracle.energy_forces(w.pos, w.species, w.mol, w.n_mol, None, _single(spec, k)) for k in range(3)]
    for key in ("E_mol", "E_atom", "F"):
        ref = np.mean([o[key] for o in singles], axis=0)
        assert np.max(np.abs(ens[key] - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref))), key
    net = np.stack([o["E_mol"] for o in singles])
    assert np.max(np.abs(ens["E_mol_net"] - net)) <= 1e-12 * np.max(np.abs(net))


def test_ensemble_of_identical_networks_is_the_network():
    spec = _ensemble_spec(1)
    spec.ensemble = [spec.weights] * 4
    w = synthetic.workload(1)
    a = oracle.energy_forces(w.pos, w.species, None, 1, None, spec)
    b = oracle.energy_forces(w.pos, w.species, None, 1, None, _single(spec, 0))
    assert abs(a["E_mol"][0] - b["E_mol"][0]) <= 1e-12 * abs(b["E_mol"][0])
    assert np.max(np.abs(a["F"] - b["F"])) <= 1e-12


def test_ensemble_forces_match_finite_differences():
    spec = _ensemble_spec(2, seed=77)
    w = synthetic.workload(1)
    out = oracle.energy_forces(w.pos, w.species, None, 1, None, spec)
    nl = oracle.neighbor_list(w.pos, None, None, 7.0)
    atoms = [0, 11, 40, 71]
    F_fd = _fd_forces(w.pos.astype(np.float64), w.species, None, spec, nl, atoms)
    assert np.max(np.abs(out["F"][atoms] - F_fd)) <= 1e-7 * max(1.0, np.max(np.abs(F_fd)))
