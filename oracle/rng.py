"""Oracle: SplitMix64 counter-based noise for the initial state.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) advances its state by the
golden-ratio increment 0x9E3779B97F4A7C15 and emits the state through two
xor-shift-multiply rounds and a final xor-shift.  Here one output step is
applied to a counter, so that the oracle and the library draw the same
numbers without sharing code:

    ctr = planet * 2^40 + col * 2^20 + lev
    u   = (mix64(seed XOR ctr) >> 11) * 2^-53          in [0, 1)
    eps = amp * (2 u - 1)                               in [-amp, amp)
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64(x):
    """One SplitMix64 output step for state(s) x (uint64, wrapping)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed, ctr):
    """u in [0, 1) from the top 53 bits of mix64(seed ^ ctr)."""
    z = mix64(np.uint64(seed) ^ np.asarray(ctr, dtype=np.uint64))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def column_noise(seed, n_col, n_lev, amp, planet=0):
    """eps[col, lev] uniform in [-amp, amp)."""
    col = np.arange(n_col, dtype=np.uint64)[:, None]
    lev = np.arange(n_lev, dtype=np.uint64)[None, :]
    ctr = (np.uint64(planet) << np.uint64(40)) + (col << np.uint64(20)) + lev
    return amp * (2.0 * uniform01(seed, ctr) - 1.0)
