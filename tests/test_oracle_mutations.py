"""Plant plausible mistakes in the oracle (a flipped sign, a dropped term, a
transposed index, a non-strict cutoff) and check that at least one pin
catches each of them.  CPU only; the oracle is restored after each case."""
import importlib

import numpy as np

import oracle

oaev = importlib.import_module("oracle.aev")
oforces = importlib.import_module("oracle.forces")
omlp = importlib.import_module("oracle.mlp")
onb = importlib.import_module("oracle.neighbors")
from tests import test_oracle_pins as pins


def _fails(fn, *args):
    try:
        fn(*args)
    except (AssertionError, ValueError, IndexError):
        return True
    return False


def test_mutant_switch_sign(monkeypatch, spec):
    monkeypatch.setattr(oaev, "switch", lambda r, rc: np.where(r < oaev.f64(rc), 0.5 * np.cos(np.pi * r / oaev.f64(rc)) - 0.5, 0.0))
    assert _fails(pins.test_radial_two_atoms_closed_form, spec)


def test_mutant_angle_expansion_sign(monkeypatch, spec):
    orig = oaev.angular_factors

    def bad(v1, r1, v2, r2, sp):
        f = orig(v1, r1, v2, r2, sp)
        thz = oaev.f64(sp.shf_z)
        w = f["u"][:, None] * np.cos(thz)[None, :] - f["sq"][:, None] * np.sin(thz)[None, :]
        f["F1"] = np.power(np.maximum(0.5 * (1 + w), 0), oaev.f64(sp.zeta))
        return f
    monkeypatch.setattr(oaev, "angular_factors", bad)
    assert _fails(pins.test_angular_three_atoms_closed_form, spec)


def test_mutant_species_pair_unordered(monkeypatch, spec):
    # forgetting to order (s, t) before taking the triangular index
    monkeypatch.setattr(oaev.AEVLayout, "pair_index",
                        lambda self, s, t: np.abs(s * self.ns - (s * (s - 1)) // 2 + (t - s)))
    assert _fails(pins.test_aev_matches_pure_python_loops, spec, 0)


def test_mutant_angular_terms_transposed(monkeypatch, spec):
    # F1 indexed by the radial shell and F2 by the angle section
    orig = oaev.angular_factors

    def bad(v1, r1, v2, r2, sp):
        f = orig(v1, r1, v2, r2, sp)
        f["F1"] = f["F1"][:, ::-1].copy()
        return f
    monkeypatch.setattr(oaev, "angular_factors", bad)
    assert _fails(pins.test_aev_matches_pure_python_loops, spec, 0)


def test_mutant_missing_celu_derivative(monkeypatch, spec_bias):
    monkeypatch.setattr(omlp, "celu_deriv", lambda x, a: np.ones_like(x))

    class Req:
        def getfixturevalue(self, _):
            return spec_bias
    assert _fails(pins.test_mlp_matches_torch_fp64, Req(), "spec_bias")


def test_mutant_dropped_angle_gradient(monkeypatch, spec_bias):
    orig = np.einsum

    def einsum_drop(sig, *ops):
        out = orig(sig, *ops)
        if sig == "taz,ta,tz->t" and ops[2] is not None and ops[1] is not None:
            einsum_drop.calls += 1
            if einsum_drop.calls % 3 == 1:      # the dE/dc contraction
                return out * 0.0
        return out
    einsum_drop.calls = 0
    monkeypatch.setattr(oforces.np, "einsum", einsum_drop)
    assert _fails(pins.test_forces_match_finite_differences_cluster, spec_bias)


def test_mutant_radial_gradient_sign(monkeypatch, spec_bias):
    orig = oaev.switch_deriv
    monkeypatch.setattr(oforces, "switch_deriv", lambda r, rc: -orig(r, rc))
    assert _fails(pins.test_forces_match_finite_differences_cluster, spec_bias)


def test_mutant_non_strict_cutoff(monkeypatch):
    orig = onb.neighbor_rows

    def loose(pos, mol, box, r_list, rows, block=64):
        return orig(pos, mol, box, float(np.nextafter(np.float32(r_list), np.float32(10))), rows, block)
    monkeypatch.setattr(onb, "neighbor_rows", loose)
    monkeypatch.setattr(oracle, "neighbor_list", lambda pos, mol, box, r: loose(pos, mol, box, r, np.arange(pos.shape[0])))
    assert _fails(pins.test_neighbors_exact_cutoff_is_excluded)


def test_mutant_wrong_image_rounding(monkeypatch):
    monkeypatch.setattr(onb, "_min_image", lambda d0, L: (d0 - np.floor(d0 / L) * L, -np.floor(d0 / L)))
    case = [c for c in __import__("synthetic").adversarial_cases() if c.name == "faces_periodic"][0]
    assert _fails(pins.test_neighbors_match_brute_force_adversarial, case)


def test_mutant_virial_attributed_to_neighbour(monkeypatch, spec_bias):
    # each edge's term booked on atom j instead of its centre i (the structure sum is unchanged);
    # a transposed outer product would be no mistake: each W_i is symmetric, since E_i is
    # invariant under a rotation of its edge vectors
    orig = oforces.virial_from_edges

    def bad(nl, v, G, mol=None, n_mol=1, n_atoms=None):
        return orig((nl[1], nl[0], nl[2]), v, G, mol, n_mol, n_atoms)
    monkeypatch.setattr(oforces, "virial_from_edges", bad)
    assert _fails(pins.test_virial_is_the_strain_derivative, spec_bias, True)


def test_mutant_virial_sign(monkeypatch, spec_bias):
    orig = oforces.virial_from_edges

    def bad(nl, v, G, mol=None, n_mol=1, n_atoms=None):
        return orig(nl, -v, G, mol, n_mol, n_atoms)
    monkeypatch.setattr(oforces, "virial_from_edges", bad)
    assert _fails(pins.test_virial_of_open_structure_is_sum_x_outer_F, spec_bias)


def test_mutant_ensemble_self_energy_per_network(monkeypatch):
    # the self energy kept in every network's energy and added again after the mean
    orig = omlp._single_net

    def bad(aev, species, spec, precision, need_grad, weights, with_self=True, rng=None, trace=None):
        return orig(aev, species, spec, precision, need_grad, weights, with_self=True, rng=rng, trace=trace)
    monkeypatch.setattr(omlp, "_single_net", bad)
    assert _fails(pins.test_ensemble_is_the_mean_of_its_networks)


def test_mutant_cells_smaller_than_cutoff(monkeypatch):
    # cells cut finer than the cutoff: the 27-cell stencil misses partners
    monkeypatch.setattr(onb, "_cells_per_axis", lambda L, side: max(2, int(np.ceil(1.6 * L / side))))
    assert _fails(pins.test_cell_search_matches_all_pairs_scan, "cubic")


def test_mutant_cell_index_rounded(monkeypatch):
    # binning by rounding instead of flooring puts atoms one cell off
    monkeypatch.setattr(onb, "_cell_index",
                        lambda x, lo, cs, nc: np.clip(np.rint((x - lo) / cs).astype(np.int64), 0, nc - 1))
    assert _fails(pins.test_cell_search_matches_all_pairs_scan, "cubic")


# ---------------------------------------------------------------- BF16 form: rounding points

def _fails_any(fn, cases):
    return any(_fails(fn, *c) for c in cases)


def test_mutant_bf16_head_weights_rounded(monkeypatch, spec_bias):
    monkeypatch.setattr(omlp, "BF16_WEIGHTS", (True, True, True, True))
    assert _fails(pins.test_bf16_weights_enter_rounded_where_stated, spec_bias, 3, False)


def test_mutant_bf16_w2_unrounded(monkeypatch, spec_bias):
    monkeypatch.setattr(omlp, "BF16_WEIGHTS", (True, False, True, False))
    assert _fails(pins.test_bf16_weights_enter_rounded_where_stated, spec_bias, 1, True)


def test_mutant_bf16_features_unrounded(monkeypatch, spec_bias):
    monkeypatch.setattr(omlp, "BF16_INPUTS", (False, True, True))
    assert _fails(pins.test_bf16_features_enter_rounded, spec_bias)


def test_mutant_bf16_h1_unrounded(monkeypatch, spec_bias):
    monkeypatch.setattr(omlp, "BF16_INPUTS", (True, False, True))
    assert _fails(pins.test_bf16_hidden_activations_enter_rounded, spec_bias, 0, True)


def test_mutant_bf16_h2_unrounded(monkeypatch, spec_bias):
    monkeypatch.setattr(omlp, "BF16_INPUTS", (True, True, False))
    assert _fails(pins.test_bf16_hidden_activations_enter_rounded, spec_bias, 1, True)


def test_mutant_bf16_d3_unrounded(monkeypatch, spec_bias):
    monkeypatch.setattr(omlp, "BF16_ADJOINT", (False, True, True))
    assert _fails(pins.test_bf16_adjoint_inputs_enter_rounded, spec_bias, "w4")


def test_mutant_bf16_d2_unrounded(monkeypatch, spec_bias):
    monkeypatch.setattr(omlp, "BF16_ADJOINT", (True, False, True))
    assert _fails(pins.test_bf16_adjoint_inputs_enter_rounded, spec_bias, "b2")


def test_mutant_bf16_d1_unrounded(monkeypatch, spec_bias):
    monkeypatch.setattr(omlp, "BF16_ADJOINT", (True, True, False))
    assert _fails(pins.test_bf16_adjoint_inputs_enter_rounded, spec_bias, "b1")


def test_mutant_bf16_sigma_drops_input_term(monkeypatch, spec_bias):
    # the closed-form spread without the input roundings (weights only)
    monkeypatch.setattr(omlp, "BF16_INPUTS", (False, False, False))
    orig = omlp._single_net

    def single(aev, species, spec, precision, need_grad, weights, with_self=True, rng=None, trace=None):
        with monkeypatch.context() as m:
            m.setattr(omlp, "BF16_INPUTS", (True, True, True))
            return orig(aev, species, spec, precision, need_grad, weights, with_self, rng, trace)
    monkeypatch.setattr(omlp, "_single_net", single)
    assert _fails(pins.test_bf16_energy_sigma_matches_monte_carlo_arithmetic, spec_bias)

