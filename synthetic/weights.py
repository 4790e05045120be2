"""Random network weights (Glorot-uniform), drawn once on the host.

Drawn from numpy's PCG64 generator in a fixed order: species, then layer,
then W (row-major [out][in]) followed by b.  The seed plays the role of the
paper's model-initialisation key (Sec. 2.4, "Building a FeNNix model").
Weights are float32 values; both implementations receive the same numbers.
"""
import numpy as np


def glorot_weights(n_species, widths, seed, bias_scale=0.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _s in range(n_species):
        layers = []
        for l in range(len(widths) - 1):
            fan_in, fan_out = widths[l], widths[l + 1]
            lim = np.sqrt(6.0 / (fan_in + fan_out))
            W = rng.uniform(-lim, lim, size=(fan_out, fan_in)).astype(np.float32)
            if bias_scale > 0:
                b = rng.uniform(-bias_scale, bias_scale, size=fan_out).astype(np.float32)
            else:
                b = np.zeros(fan_out, dtype=np.float32)
            layers.append((W, b))
        out.append(layers)
    return out
