"""Counter-free seeded streams used by the synthetic workloads.

The systematic-resampling offset ``u`` is drawn on the host from a SplitMix64
stream (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) and handed to both the oracle and the GPU library as
an input, so neither side draws it.
"""

import numpy as np

_MASK = (1 << 64) - 1


def _splitmix64_next(state):
    state = (state + 0x9E3779B97F4A7C15) & _MASK
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    z = z ^ (z >> 31)
    return state, z


def splitmix64_uniforms(seed, count):
    """Return ``count`` doubles in [0, 1) as ``(x >> 11) * 2**-53``."""
    state = int(seed) & _MASK
    out = np.empty(int(count), dtype=np.float64)
    for k in range(int(count)):
        state, z = _splitmix64_next(state)
        out[k] = (z >> 11) * (1.0 / 9007199254740992.0)
    return out
