"""BF16-MFMA corrector network kernels against the FP64 reference MLP:
forward outputs, loss and gradients within BF16 tolerance, and training."""
import numpy as np
import pytest

from oracle import mlp as omlp
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

WIDTHS = [1120, 256, 256, 256, 160]


def _net(B, seed=3):
    import torch
    from paper_1607_05535_amd import thor
    net = thor.MLP(WIDTHS, B, seed=seed)
    rs = np.random.default_rng(seed)
    x32 = rs.normal(size=(B, WIDTHS[0])).astype(np.float32)
    x = torch.from_numpy(x32).to("cuda:0").to(torch.bfloat16)
    xr = x.float().cpu().numpy().astype(np.float64)   # what the kernels see
    t32 = (0.5 * rs.normal(size=(B, WIDTHS[-1]))).astype(np.float32)
    t = torch.from_numpy(t32).to("cuda:0")
    return net, x, xr, t, t32.astype(np.float64)


def _ref_params(net):
    return [(W.astype(np.float64), b.astype(np.float64)) for W, b in net.unpack(net.get_params())]


def test_forward_matches_reference():
    import torch
    B = 100    # ragged against the 64-row GEMM tiles and the 48-row fused tiles
    say(f"[mlp] forward widths={WIDTHS} B={B}")
    net, x, xr, t, tr = _net(B)
    y = torch.empty(B, WIDTHS[-1], dtype=torch.float32, device="cuda:0")
    net.forward(x, y)
    got = y.cpu().numpy().astype(np.float64)
    ref, _ = omlp.forward(_ref_params(net), xr)
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say(f"      forward rel err {rel:.3e}")
    assert rel < 2e-2


@pytest.mark.parametrize("B", [1, 100, 10242])
def test_fused_inference_equals_layer_by_layer(B):
    """The fused 4-layer inference kernel (one workgroup per 48-row tile,
    inputs and hidden activations in LDS, weights in fragment order) against
    the layer-by-layer GEMMs: the same products in the same order, so the
    same outputs, at a single row, a ragged tile and the g5 corrector's
    10242 columns."""
    import torch
    net, x, xr, t, tr = _net(B, seed=7)
    y1 = torch.empty(B, WIDTHS[-1], dtype=torch.float32, device="cuda:0")
    y2 = torch.empty_like(y1)
    net.set_fused(False)
    net.forward(x, y1)
    net.set_fused(True)
    net.forward(x, y2)
    net.set_fused(False)
    a, b = y1.cpu().numpy(), y2.cpu().numpy()
    say(f"[mlp] fused vs layered B={B}: max |diff| {np.abs(a - b).max():.3e}, bitwise {np.array_equal(a, b)}")
    assert np.abs(a - b).max() <= 1e-6 * np.abs(a).max()


def test_gradients_match_reference():
    B = 128
    net, x, xr, t, tr = _net(B, seed=5)
    loss, g = net.loss_grad(x, t)
    params = _ref_params(net)
    ref_loss = omlp.loss(params, xr, tr)
    assert abs(loss / ref_loss - 1) < 2e-2
    ref = omlp.backward(params, xr, tr)
    got = net.unpack(g.astype(np.float64))
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(got, ref)):
        for name, a, r in (("W", gW, rW), ("b", gb, rb)):
            rel = np.linalg.norm(a - r) / np.linalg.norm(r)
            cos = float(np.sum(a * r) / (np.linalg.norm(a) * np.linalg.norm(r)))
            say(f"      layer {li} d{name}: rel {rel:.3e} cos {cos:.6f}")
            assert rel < 2e-2 and cos > 0.999, (li, name, rel, cos)


def test_training_reduces_loss():
    B = 256
    net, x, xr, t, tr = _net(B, seed=7)
    l0, _ = net.loss_grad(x, t, want_grad=False)
    for _ in range(200):
        net.train_step(x, t, 1e-3)
    l1, _ = net.loss_grad(x, t, want_grad=False)
    say(f"      loss {l0:.4f} -> {l1:.4f}")
    assert l1 < 0.1 * l0


def test_argument_errors():
    from paper_1607_05535_amd import thor
    net, x, xr, t, tr = _net(64)
    with pytest.raises(thor.ThorError):
        net.loss_grad(x[:40], t[:40])          # batch not a multiple of 32
    with pytest.raises(thor.ThorError):
        thor.MLP([100, 64], 32)                # width not a multiple of 32


def test_split_batch_gradients_match_reference_and_repeat_bitwise():
    """A batch of 2048 rows reduces the weight gradients over 8 chunks and
    the bias gradients over 32: still the reference gradients, and the same
    bits on a second call (fixed summation order)."""
    import torch
    B = 2048
    net, x, xr, t, tr = _net(B, seed=9)
    loss, g = net.loss_grad(x, t)
    loss2, g2 = net.loss_grad(x, t)
    assert loss == loss2 and np.array_equal(g, g2)
    params = _ref_params(net)
    ref = omlp.backward(params, xr, tr)
    got = net.unpack(g.astype(np.float64))
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(got, ref)):
        for name, a, r in (("W", gW, rW), ("b", gb, rb)):
            rel = np.linalg.norm(a - r) / np.linalg.norm(r)
            cos = float(np.sum(a * r) / (np.linalg.norm(a) * np.linalg.norm(r)))
            assert rel < 2e-2 and cos > 0.999, (li, name, rel, cos)
    # the inference path (no stored pre-activations) gives the same outputs
    y = torch.empty(B, WIDTHS[-1], dtype=torch.float32, device="cuda:0")
    net.forward(x, y)
    d = y.cpu().numpy().astype(np.float64) - tr
    assert abs(np.mean(d * d) / loss - 1) < 1e-6
