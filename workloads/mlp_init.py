"""Seeded initial parameters of the boundary-closure MLP (an input to both
the oracle and the library: neither side draws random numbers itself).

He-uniform weights, W ~ U(-sqrt(6 / fan_in), sqrt(6 / fan_in)), zero biases,
drawn from NumPy's PCG64(seed); flat layout W1, b1, W2, b2, W3, b3 with W
row-major (out x in).
"""
import numpy as np

SIZES = (78, 128, 128, 75)


def init_params(seed=0, sizes=SIZES):
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for i in range(len(sizes) - 1):
        n_in, n_out = sizes[i], sizes[i + 1]
        bound = np.sqrt(6.0 / n_in)
        parts.append(rng.uniform(-bound, bound, size=n_out * n_in))
        parts.append(np.zeros(n_out))
    return np.concatenate(parts)
