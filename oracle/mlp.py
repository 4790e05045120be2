"""Oracle species-specialised MLP (Sec. 2.2, "Neural Networks": fully
species-dependent network parameters; Sec. 2.4: ChemicalNet maps each atom's
AEV to its atomic energy).

For an atom of species s with feature vector a:
    z1 = W1_s a + b1_s,  h1 = CELU(z1)          (1008 -> 256)
    z2 = W2_s h1 + b2_s, h2 = CELU(z2)          (256 -> 192)
    z3 = W3_s h2 + b3_s, h3 = CELU(z3)          (192 -> 160)
    E  = w4_s . h3 + b4_s + e_s                 (160 -> 1)
with CELU(x) = max(0, x) + min(0, alpha (exp(x / alpha) - 1)).

The gradient dE/da used for the forces runs the same chain backwards:
    d3 = w4 * CELU'(z3), d2 = (W3^T d3) * CELU'(z2), d1 = (W2^T d2) * CELU'(z1),
    dE/da = W1^T d1,  with CELU'(x) = 1 for x > 0 and exp(x / alpha) otherwise.

Precision "bf16" evaluates the reduced-precision form: every input of the
three matrix products of the forward pass (the AEV and h1, h2) and of the
three of the backward pass (d3, d2, d1), and the weight matrices W1..W3, are
rounded to bfloat16 (round to nearest even, through float32), and products
are accumulated exactly (float64).  The last layer (a dot product), the
activations and their derivatives stay in full precision.

An ensemble (ANI-2x has eight networks; Sec. 5.5 evaluates the first one)
gives every atom the mean of its networks' energies, E_i = (1/K) sum_k E_i^k
(+ the self energy once), and dE/da is the mean of the networks' gradients.
"""
import numpy as np


def celu(x, alpha):
    return np.where(x > 0, x, alpha * np.expm1(np.minimum(x, 0.0) / alpha))


def celu_deriv(x, alpha):
    return np.where(x > 0, 1.0, np.exp(np.minimum(x, 0.0) / alpha))


def round_bf16(x):
    """Round to the nearest bfloat16 (ties to even), via float32; returns
    float64 values."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _layers(spec, s, precision, weights=None):
    out = []
    for l, (W, b) in enumerate((spec.weights if weights is None else weights)[s]):
        W = np.asarray(W, dtype=np.float32).astype(np.float64)
        b = np.asarray(b, dtype=np.float32).astype(np.float64)
        if precision == "bf16" and l < len(spec.weights[s]) - 1:
            W = round_bf16(W)
        out.append((W, b))
    return out


def networks(spec):
    """Every network's weights: the ensemble, or the single network."""
    return spec.ensemble if getattr(spec, "ensemble", None) else [spec.weights]


def mlp_energy_and_grad(aev, species, spec, precision="fp64", need_grad=True):
    """Atomic energies E [N] and, if requested, dE/daev [N, D] (float64); the
    ensemble mean for an ensemble spec."""
    nets = networks(spec)
    if len(nets) == 1:
        return _single_net(aev, species, spec, precision, need_grad, nets[0])
    se = np.zeros(spec.n_species) if spec.self_energy is None else np.asarray(spec.self_energy, np.float64)
    E = np.zeros(len(species))
    g = np.zeros(aev.shape) if need_grad else None
    for w in nets:
        Ek, gk = _single_net(aev, species, spec, precision, need_grad, w, with_self=False)
        E += Ek
        if need_grad:
            g += gk
    E /= len(nets)
    E += se[np.asarray(species, dtype=np.int64)]
    if need_grad:
        g /= len(nets)
    return E, g


def mlp_energies_per_net(aev, species, spec, precision="fp64"):
    """[K, N]: every network's atomic energies, self energy included."""
    return np.stack([_single_net(aev, species, spec, precision, False, w)[0] for w in networks(spec)])


def _single_net(aev, species, spec, precision, need_grad, weights, with_self=True):
    if precision not in ("fp64", "bf16"):
        raise ValueError(precision)
    q = round_bf16 if precision == "bf16" else (lambda x: x)
    alpha = float(np.float32(spec.celu_alpha))
    N, D = aev.shape
    E = np.zeros(N)
    g = np.zeros((N, D)) if need_grad else None
    se = np.zeros(spec.n_species) if spec.self_energy is None or not with_self else spec.self_energy
    for s in range(spec.n_species):
        rows = np.nonzero(np.asarray(species) == s)[0]
        if len(rows) == 0:
            continue
        L = _layers(spec, s, precision, weights)
        h = aev[rows]
        zs = []
        for W, b in L[:-1]:
            z = q(h) @ W.T + b
            zs.append(z)
            h = celu(z, alpha)
        w4, b4 = L[-1]
        E[rows] = (h @ w4.T)[:, 0] + b4[0] + se[s]
        if need_grad:
            d = w4[0][None, :] * celu_deriv(zs[-1], alpha)
            for l in range(len(L) - 2, 0, -1):
                d = (q(d) @ L[l][0]) * celu_deriv(zs[l - 1], alpha)
            g[rows] = q(d) @ L[0][0]
    return E, g


def mlp_energy(aev, species, spec, precision="fp64"):
    return mlp_energy_and_grad(aev, species, spec, precision, need_grad=False)[0]
