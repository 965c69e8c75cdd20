"""thor_field_stats_noalloc (the allocation-free entry point, partial sums in
a library-owned device array) against thor_field_stats (caller scratch)
through the C ABI: two calls in a row, the second with a smaller input, of
the statistics of arrays and of differences of arrays."""
import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _fields(n_arrays, n_col, n_lev, seed):
    import torch
    g = torch.Generator(device="cuda:0").manual_seed(seed)
    shape = (n_arrays, 5, n_col, n_lev)
    C = (torch.randn(shape, device="cuda:0", generator=g) * 3.0 + 1.5).float()
    F = (C + 0.1 * torch.randn(shape, device="cuda:0", generator=g)).float()
    return C, F


def test_noalloc_field_stats_equal_the_scratch_version():
    from paper_1607_05535_amd import thor
    # 30 arrays of 642 columns x 32 levels need three groups of the 1 MiB
    # scratch (12 arrays each); then 5 arrays of 162 columns x 16 levels
    for n_arrays, n_col, n_lev, seed in ((30, 642, 32, 1), (5, 162, 16, 2)):
        C, F = _fields(n_arrays, n_col, n_lev, seed)
        stride = 5 * n_col * n_lev
        for Fn in (None, F):
            ref = thor.thor_field_stats(C, Fn, n_arrays, stride, n_col, n_lev)
            got = thor.thor_field_stats_noalloc(C, Fn, n_arrays, stride, n_col, n_lev)
            rel = np.abs(got - ref).max() / np.abs(ref).max()
            say(f"[noalloc] {n_arrays} x {n_col} x {n_lev} diff={Fn is not None}: "
                f"max rel {rel:.2e}, bitwise {np.array_equal(got, ref)}")
            assert rel < 1e-14, rel
    with pytest.raises(thor.ThorError):
        thor.thor_field_stats_noalloc(C, None, n_arrays, stride, n_col, 3)   # 3 does not divide 256
