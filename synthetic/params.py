"""Model hyper-parameters of the ANI-2x-shaped potential (numbers only).

The AEV hyper-parameters follow the ANI-2x model the paper benchmarks (Sec. 5,
"Performance benchmarks"; AEV of Smith, Isayev and Roitberg 2017):
radial cutoff 5.1 A with 16 Gaussian shells (eta 19.7), angular cutoff 3.5 A
with 4 radial shells (eta 12.5) times 8 angle sections (zeta 14.1), over 7
species.  Shell grids are the evenly spaced ANI-2x grids; they are passed to
both implementations as parameters.
"""
from dataclasses import dataclass, field
import math

import numpy as np

SPECIES = ("H", "C", "N", "O", "F", "S", "Cl")
SPECIES_INDEX = {s: i for i, s in enumerate(SPECIES)}
# amu, indexed like SPECIES
MASSES = np.array([1.008, 12.011, 14.007, 15.999, 18.998, 32.06, 35.45])


@dataclass
class ModelSpec:
    n_species: int
    rc_r: float
    eta_r: float
    shf_r: np.ndarray          # [n_shf_r]
    rc_a: float
    eta_a: float
    zeta: float
    shf_a: np.ndarray          # [n_shf_a]
    shf_z: np.ndarray          # [n_shf_z]  angle sections theta_z
    radial_prefactor: float
    cos_scale: float
    widths: tuple              # (aev_dim, h1, h2, h3, 1)
    celu_alpha: float
    weights: list = field(default_factory=list)   # [species][layer] -> (W [out,in] f32, b [out] f32)
    self_energy: np.ndarray = None                 # [n_species] f64
    ensemble: list = None                          # [net] -> weights as above (net 0 is `weights`)

    @property
    def n_shf_r(self):
        return len(self.shf_r)

    @property
    def n_shf_a(self):
        return len(self.shf_a)

    @property
    def n_shf_z(self):
        return len(self.shf_z)

    @property
    def n_pairs_species(self):
        return self.n_species * (self.n_species + 1) // 2

    @property
    def radial_dim(self):
        return self.n_species * self.n_shf_r

    @property
    def angular_dim(self):
        return self.n_pairs_species * self.n_shf_a * self.n_shf_z

    @property
    def aev_dim(self):
        return self.radial_dim + self.angular_dim


def ani2x_like_spec(weight_seed=123456, bias_scale=0.0, self_energy=None):
    """The 7-species, 1008-feature, 1008-256-192-160-1 CELU(0.1) model with
    Glorot-uniform weights drawn from ``weight_seed``."""
    from .weights import glorot_weights
    shf_r = np.array([0.8 + 0.26875 * k for k in range(16)], dtype=np.float32)
    shf_a = np.array([0.8 + 0.3375 * a for a in range(4)], dtype=np.float32)
    shf_z = np.array([(2 * z + 1) * math.pi / 16 for z in range(8)], dtype=np.float32)
    widths = (1008, 256, 192, 160, 1)
    spec = ModelSpec(
        n_species=7, rc_r=5.1, eta_r=19.7, shf_r=shf_r,
        rc_a=3.5, eta_a=12.5, zeta=14.1, shf_a=shf_a, shf_z=shf_z,
        radial_prefactor=0.25, cos_scale=0.95,
        widths=widths, celu_alpha=0.1,
    )
    assert spec.aev_dim == widths[0]
    spec.weights = glorot_weights(7, widths, weight_seed, bias_scale)
    spec.self_energy = (np.zeros(7) if self_energy is None
                        else np.asarray(self_energy, dtype=np.float64))
    return spec


def ani2x_like_ensemble(n_nets=8, weight_seed=123456, bias_scale=0.0, self_energy=None):
    """An ensemble of n_nets networks of the same shape on one AEV (ANI-2x
    has eight).  Network k draws its weights from seed weight_seed + k, so
    network 0 is the single network of ani2x_like_spec(weight_seed)."""
    from .weights import glorot_weights
    spec = ani2x_like_spec(weight_seed, bias_scale, self_energy)
    spec.ensemble = [spec.weights] + [glorot_weights(spec.n_species, spec.widths, weight_seed + k, bias_scale)
                                      for k in range(1, n_nets)]
    return spec
