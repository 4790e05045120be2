"""FP64 CPU oracle for the AEV neural-network potential (energy and forces).

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import or call anything here; the GPU
product path never does, and the oracle imports nothing from the product.

It is a plain, slow, obviously correct evaluation of the definition, in
float64 with numpy:

* neighbours: directed pairs of atoms of the same structure whose distance
  is strictly lower than the cutoff, with minimum-image shifts for an
  orthorhombic periodic box (Sec. 2.1, "Preprocessing Modules");
* geometry and the cosine switching function (Sec. 2.1, processing modules);
* the ANI atomic environment vector: Gaussian radial shells (Sec. 2.2,
  "Chemical and Radial Encodings") and the ANI angular basis
  (0.5 + 0.5 cos(theta - theta_n))^zeta (App. A, angular resources), as
  defined by the ANI reference the paper cites for its ANI_AEV module;
* one species-specialised MLP per chemical species (Sec. 2.2, "Neural
  Networks"), atomic energies summed per structure (Sec. 2.4, ANI flow);
* forces as minus the gradient of the total energy (Sec. 2.4), evaluated by
  an explicit chain rule through MLP, AEV and pair geometry.

Pins (in the tests marked "not gpu"): brute-force enumeration on tiny inputs,
closed forms for two- and three-atom systems, invariances, smooth decay at
the cutoffs, finite differences of the energy, zero net force and torque,
batch additivity.  The absolute values of the published ANI-2x model are
parity unpinned: its trained weights are not available, so random weights
are used.
"""
from .neighbors import neighbor_list, neighbor_list_cells, neighbor_rows, brute_force_pairs
from .aev import switch, switch_deriv, aev, AEVLayout
from .mlp import celu, celu_deriv, mlp_energy, mlp_energy_and_grad, round_bf16, bf16_energy_sigma, mlp_trace
from .forces import energy_forces, edge_gradients, forces_from_edges, total_energy, energy_forces_f64
from .md import velocity_verlet, langevin_baoab, langevin_noise

__all__ = [
    "neighbor_list", "neighbor_list_cells", "neighbor_rows", "brute_force_pairs",
    "switch", "switch_deriv", "aev", "AEVLayout",
    "celu", "celu_deriv", "mlp_energy", "mlp_energy_and_grad", "round_bf16", "bf16_energy_sigma", "mlp_trace",
    "energy_forces", "edge_gradients", "forces_from_edges", "total_energy", "energy_forces_f64",
    "velocity_verlet", "langevin_baoab", "langevin_noise",
]
