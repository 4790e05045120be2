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
are accumulated exactly (float64).  The last layer (a dot product, not a
matrix product), the activations and their derivatives stay in full
precision.  The rounding points are listed in BF16_WEIGHTS, BF16_INPUTS and
BF16_ADJOINT.

Precision "mca" is Monte Carlo arithmetic (Parker, 1997) at bfloat16's unit
roundoff u = 2^-8: at every one of those rounding points each value x
becomes x (1 + u r) with r uniform in [-1, 1], drawn from the generator
passed in.  Repeated runs sample the spread the bfloat16 roundings cause,
without depending on where the rounding boundaries fall.

bf16_energy_sigma gives the same spread to first order in closed form: the
standard deviation of the BF16 form's atomic and structure energies when
each rounding point contributes an independent relative error of variance
u^2 / 3, propagated by the exact adjoint of the float64 network.

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


# Rounding points of the BF16 form, in layer order: the weight matrices W1..W3
# and not the head's w4; the inputs of the three forward products (AEV, h1,
# h2); the inputs of the three adjoint products (d3 into W3^T, d2 into W2^T,
# d1 into W1^T).
BF16_WEIGHTS = (True, True, True, False)
BF16_INPUTS = (True, True, True)
BF16_ADJOINT = (True, True, True)

U_BF16 = 2.0 ** -8          # unit roundoff of bfloat16 (8 significant bits)


def _rounder(precision, rng):
    if precision == "bf16":
        return round_bf16
    if precision == "mca":
        if rng is None:
            raise ValueError("Monte Carlo arithmetic needs a random generator")
        return lambda x: np.asarray(x, np.float64) * (1.0 + U_BF16 * rng.uniform(-1.0, 1.0, size=np.shape(x)))
    return lambda x: x


def _layers(spec, s, precision, weights=None, rng=None):
    q = _rounder(precision, rng)
    out = []
    for l, (W, b) in enumerate((spec.weights if weights is None else weights)[s]):
        W = np.asarray(W, dtype=np.float32).astype(np.float64)
        b = np.asarray(b, dtype=np.float32).astype(np.float64)
        if precision != "fp64" and BF16_WEIGHTS[l]:
            W = q(W)
        out.append((W, b))
    return out


def networks(spec):
    """Every network's weights: the ensemble, or the single network."""
    return spec.ensemble if getattr(spec, "ensemble", None) else [spec.weights]


def mlp_energy_and_grad(aev, species, spec, precision="fp64", need_grad=True, rng=None):
    """Atomic energies E [N] and, if requested, dE/daev [N, D] (float64); the
    ensemble mean for an ensemble spec."""
    nets = networks(spec)
    if len(nets) == 1:
        return _single_net(aev, species, spec, precision, need_grad, nets[0], rng=rng)
    se = np.zeros(spec.n_species) if spec.self_energy is None else np.asarray(spec.self_energy, np.float64)
    E = np.zeros(len(species))
    g = np.zeros(aev.shape) if need_grad else None
    for w in nets:
        Ek, gk = _single_net(aev, species, spec, precision, need_grad, w, with_self=False, rng=rng)
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


def _single_net(aev, species, spec, precision, need_grad, weights, with_self=True, rng=None, trace=None):
    if precision not in ("fp64", "bf16", "mca"):
        raise ValueError(precision)
    q = _rounder(precision, rng)
    qi = [q if precision != "fp64" and BF16_INPUTS[l] else (lambda x: x) for l in range(3)]
    qd = [q if precision != "fp64" and BF16_ADJOINT[l] else (lambda x: x) for l in range(3)]
    alpha = float(np.float32(spec.celu_alpha))
    N, D = aev.shape
    E = np.zeros(N)
    g = np.zeros((N, D)) if need_grad else None
    se = np.zeros(spec.n_species) if spec.self_energy is None or not with_self else spec.self_energy
    for s in range(spec.n_species):
        rows = np.nonzero(np.asarray(species) == s)[0]
        if len(rows) == 0:
            continue
        L = _layers(spec, s, precision, weights, rng)
        h = aev[rows]
        zs = []
        for l, (W, b) in enumerate(L[:-1]):
            z = qi[min(l, 2)](h) @ W.T + b
            zs.append(z)
            h = celu(z, alpha)
        w4, b4 = L[-1]
        E[rows] = (h @ w4.T)[:, 0] + b4[0] + se[s]
        if trace is not None:
            for l, z in enumerate(zs):
                trace.setdefault("z", {}).setdefault(l, np.zeros((N, z.shape[1])))[rows] = z
        if need_grad:
            # the adjoint products, from the last layer down: input d_{l+1}
            # enters W_{l+1}^T (BF16_ADJOINT is ordered d3, d2, d1)
            d = w4[0][None, :] * celu_deriv(zs[-1], alpha)
            for l in range(len(L) - 2, 0, -1):
                p = qd[min(len(L) - 2 - l, 2)](d) @ L[l][0]
                if trace is not None:
                    trace.setdefault("p", {}).setdefault(l, np.zeros((N, p.shape[1])))[rows] = p
                d = p * celu_deriv(zs[l - 1], alpha)
            g[rows] = qd[min(len(L) - 2, 2)](d) @ L[0][0]
    return E, g


def mlp_trace(aev, species, spec, precision="fp64"):
    """Intermediate products of the single network, in atom order: z[l] the
    pre-activations of layers 1..3 (l = 0, 1, 2) and p[l] = W_{l+1}^T d_{l+1}
    the adjoint products before the CELU' factor (p[2] from d3, p[1] from d2),
    plus E and dE/daev."""
    tr = {}
    E, g = _single_net(aev, species, spec, precision, True, networks(spec)[0], trace=tr)
    tr["E"], tr["g"] = E, g
    return tr


def bf16_energy_sigma(aev, species, spec, mol=None, n_mol=1, u=U_BF16):
    """First-order standard deviation of the BF16 form's energies: per atom
    [N] and per structure [n_mol] (single network).

    To first order the BF16 energy of atom i differs from the exact one by
        sum_l sum_j D_l[i,j] sum_k W_l[j,k] X_l[i,k] (e^W_l[j,k] + e^X_l[i,k]),
    with X_l the input of product l (the AEV, h1, h2), D_l[i,j] = dE_i/dz_l[i,j]
    the exact adjoint, and e the relative rounding errors at the points the
    form rounds (BF16_WEIGHTS, BF16_INPUTS).  Taking every e independent with
    mean 0 and variance u^2 / 3 (uniform in [-u, u]):
        var E_i = u^2/3 sum_l [ sum_jk (D W X)^2 + sum_k X[i,k]^2 (sum_j D[i,j] W[j,k])^2 ],
    and for a structure, whose atoms of one species share the same weight
    errors,
        var E_m = u^2/3 sum_l [ sum_jk W[j,k]^2 (sum_{i in m} D[i,j] X[i,k])^2
                                + sum_{i in m} sum_k X[i,k]^2 (sum_j D[i,j] W[j,k])^2 ].
    The adjoint-side roundings do not touch the energy."""
    alpha = float(np.float32(spec.celu_alpha))
    species = np.asarray(species, dtype=np.int64)
    N = len(species)
    mol = np.zeros(N, dtype=np.int64) if mol is None else np.asarray(mol, dtype=np.int64)
    v_atom = np.zeros(N)
    v_mol = np.zeros(n_mol)
    c = u * u / 3.0
    for s in range(spec.n_species):
        rows = np.nonzero(species == s)[0]
        if len(rows) == 0:
            continue
        L = _layers(spec, s, "fp64")
        xs, zs = [], []
        h = aev[rows]
        for W, b in L[:-1]:
            xs.append(h)
            z = h @ W.T + b
            zs.append(z)
            h = celu(z, alpha)
        # exact adjoints dE/dz_l
        ds = [None] * (len(L) - 1)
        d = L[-1][0][0][None, :] * celu_deriv(zs[-1], alpha)
        ds[-1] = d
        for l in range(len(L) - 2, 0, -1):
            d = (d @ L[l][0]) * celu_deriv(zs[l - 1], alpha)
            ds[l - 1] = d
        ms = mol[rows]
        for l, (W, _b) in enumerate(L[:-1]):
            X, Dl = xs[l], ds[l]
            w_on = BF16_WEIGHTS[l]
            x_on = BF16_INPUTS[min(l, 2)]
            DW = Dl @ W                                          # [n, in]
            if w_on:
                v_atom[rows] += c * np.sum((Dl ** 2) @ (W ** 2) * X ** 2, axis=1)
            if x_on:
                tx = c * np.sum(X ** 2 * DW ** 2, axis=1)
                v_atom[rows] += tx
                np.add.at(v_mol, ms, tx)
            if w_on:
                for m in np.unique(ms):
                    sel = ms == m
                    M = Dl[sel].T @ X[sel]                       # [out, in]: sum_i D[i,j] X[i,k]
                    v_mol[m] += c * np.sum(W ** 2 * M ** 2)
    return np.sqrt(v_atom), np.sqrt(v_mol)


def mlp_energy(aev, species, spec, precision="fp64"):
    return mlp_energy_and_grad(aev, species, spec, precision, need_grad=False)[0]
