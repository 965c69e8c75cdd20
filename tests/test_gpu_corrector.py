"""Learned corrector pipeline: restriction, bounded application and the gain
of a trained network over the plain coarse step, judged by the restricted
fine run (small grids)."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_lev", [32, 13])
def test_restriction_of_a_uniform_rest_state(n_lev):
    """Every fine column of a resting isothermal state is the same column:
    the restriction reproduces it on the coarse grid, whatever was there
    (also with a level count whose state rows are padded)."""
    import torch
    from paper_1607_05535_amd import thor
    fw, cw = workloads.corrector_pair(4, 2, n_lev=n_lev, dt_coarse=2400.0)
    fw.noise_amp = 0.0
    cw.T0 = 900.0                       # a different state to overwrite
    fg, cg = thor.Grid(4), thor.Grid(2)
    fine = thor.State(fg, *thor.structs_from_workload(fw))
    coarse = thor.State(cg, *thor.structs_from_workload(cw))
    ref = {k: fine.field(k)[0][0] for k in ("T", "p", "rho", "rhotheta")}
    thor.Restriction(fg, cg)(fine, coarse)
    torch.cuda.synchronize()
    for k, v in ref.items():
        got = coarse.field(k)[0]
        assert np.abs(got / v[None, :] - 1).max() < 1e-12, k
    for k in ("u", "v", "w"):
        assert np.abs(coarse.field(k)[0]).max() < 1e-12


def test_fp32_fields_equal_the_diagnostics_with_padded_rows():
    """thor_state_fields32 (the network's input fields, [5][col][lev]) at 13
    levels (state rows of 16) against the FP64 diagnostics after two steps."""
    import torch
    from paper_1607_05535_amd import thor
    from tests.gpu_util import lib_state, small_earth
    w = small_earth(glevel=3, n_lev=13, n_large=2, noise=1.0)
    st = lib_state(w)
    st.step(2, w.n_acoustic)
    out = torch.empty((5, st.n_col, st.n_lev), dtype=torch.float32, device="cuda:0")
    thor.thor_state_fields32(st, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for i, k in enumerate(("T", "u", "v", "w", "p")):
        ref = st.field(k)[0]
        scale = max(np.abs(ref).max(), 1e-30)
        assert np.abs(got[i] - ref).max() <= 2e-7 * scale, k


def _pipeline():
    from paper_1607_05535_amd import learned
    fw, cw = workloads.corrector_pair(4, 3, dt_coarse=4800.0)
    return learned.Pipeline(fw, cw, ratio=4)


def test_bound_zero_keeps_the_plain_coarse_state():
    from paper_1607_05535_amd import thor, learned
    P = _pipeline()
    C, F = P.make_pairs([7], spinup=4, pairs_per_seed=2)
    norm = P.norm(C, F)
    net = thor.MLP(learned.widths_for(P.L), P.N, seed=1)
    corr = thor.Corrector(P.work, net, norm, bound=0.0)
    before = P.work.export()[0]
    assert corr.apply() == 0
    assert np.array_equal(P.work.export()[0], before)


def test_non_finite_output_keeps_the_plain_coarse_state():
    """A network whose u output at one level is NaN for every column (its
    output bias set to NaN, T and p finite) corrects no column, even with a
    bound that would accept every finite output; with that bias finite the
    same network corrects columns."""
    from paper_1607_05535_amd import thor, learned
    P = _pipeline()
    C, F = P.make_pairs([7], spinup=4, pairs_per_seed=2)
    norm = P.norm(C, F)
    widths = learned.widths_for(P.L)
    net = thor.MLP(widths, P.N, seed=1)
    params = net.get_params()
    u3 = params.size - widths[-1] + (1 * P.L + 3)   # last bias: outputs [field][level], u is field 1
    before = P.work.export()[0]
    params[u3] = np.nan
    net.set_params(params)
    corr = thor.Corrector(P.work, net, norm, bound=1e30)
    assert corr.apply() == 0
    assert np.array_equal(P.work.export()[0], before)
    params[u3] = 0.0
    net.set_params(params)
    corr = thor.Corrector(P.work, net, norm, bound=1e30)
    assert corr.apply() > 0


def test_trained_corrector_beats_plain_coarse_step():
    P = _pipeline()
    say("[corrector] g4 fine / g3 coarse, L32")
    C, F = P.make_pairs([11, 12, 13, 14], spinup=20, pairs_per_seed=24, log=say)
    norm = P.norm(C, F)
    net, corr, losses = P.train(C, F, norm, steps=600, batch=1024, lr=2e-3, seed=3, log=say)
    assert losses[-1][1] < 0.5 * losses[0][1]
    res = P.evaluate(corr, [99], spinup=20, pairs_per_seed=8)
    say(f"           held-out {res}")
    assert res["columns_corrected_fraction"] > 0.5
    for k in ("T", "p"):
        assert res[k]["rms_corrected"] < res[k]["rms_plain"], k


def test_corrector_rejects_a_network_of_the_wrong_shape():
    """A network whose widths or batch capacity do not fit the state is an
    argument error, before anything runs."""
    from paper_1607_05535_amd import thor, learned
    P = _pipeline()
    norm = np.ones(20 * P.L, dtype=np.float32)
    for widths, max_batch in ((learned.widths_for(P.L)[:-1] + [32], P.N),      # wrong output width
                              ([64] + learned.widths_for(P.L)[1:], P.N),        # wrong input width
                              (learned.widths_for(P.L), P.N - 1)):               # batch too small
        net = thor.MLP(widths, max_batch, seed=1)
        with pytest.raises(thor.ThorError) as e:
            thor.Corrector(P.work, net, norm)
        assert e.value.code == thor.THOR_EINVAL


def test_corrector_at_its_own_configuration():
    """The learned form at the g7 -> g5 configuration (gas giant, L32, one
    Earth day of fine spin-up per trajectory), small: 2 training seeds x 30
    pairs, 400 Adam steps, judged on a held-out seed's 30 pairs.  The
    corrected coarse step is closer to the restricted fine run than the plain
    one in T, p, w and u, and corrected coarse steps are faster than the
    fine steps they stand in for."""
    from paper_1607_05535_amd import train_corrector
    rep = train_corrector.run(7, 5, seeds=3, pairs=30, spinup=576, steps=400, batch=4096, lr=1e-3)
    ho = rep["held_out"]
    say(f"[corrector] g7 -> g5: gains " + ", ".join(f"{k} {ho[k]['gain']:.2f}" for k in ("T", "u", "v", "w", "p"))
        + f"; speed-up {rep['speedup_vs_fine']:.1f}")
    # measured: T 5.0, u 1.77, v 1.17, w 12.6, p 7.8; 41x faster than the fine run
    assert ho["columns_corrected_fraction"] > 0.5
    for k, bar in (("T", 1.5), ("p", 1.5), ("w", 1.5), ("u", 1.2)):
        assert ho[k]["gain"] > bar, (k, ho[k])
    assert rep["speedup_vs_fine"] > 4.0
