"""Warm-start network on the GPU (bf16 matrix-core products, fp32
accumulation) against the FP64 reference network: forward outputs,
gradients (cosine >= 0.999, relative norm error <= 2e-2, the tolerance of
bf16 operands), one Adam step, and a short training run."""
import numpy as np
import pytest

from oracle import mlp as ref

pytestmark = pytest.mark.gpu

WIDTHS = [4, 256, 256, 256, 1280]


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, (n, 4))
    t = 0.1 * np.sin(x @ rng.standard_normal((4, 1280)))
    return x, t


@pytest.mark.parametrize("widths,batch", [(WIDTHS, 512), ([4, 40, 33, 70], 37), ([3, 64, 5], 4096)])
def test_forward_and_gradients_match_reference(widths, batch):
    from paper_2503_20605_amd import MLP
    p = ref.init_params(widths, 7)
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, (batch, widths[0]))
    t = 0.1 * rng.standard_normal((batch, widths[-1]))
    m = MLP(widths, batch)
    m.set_params(p)
    y = m.forward(x).cpu().numpy()
    yo, _ = ref.forward(p, widths, x)
    ey = np.max(np.abs(y - yo)) / np.max(np.abs(yo))
    loss, g = m.gradients(x, t)
    lo, go = ref.loss_and_grad(p, widths, x, t)
    cos = float(np.dot(g, go) / (np.linalg.norm(g) * np.linalg.norm(go)))
    rel = float(np.linalg.norm(g - go) / np.linalg.norm(go))
    print(f"[mlp] widths={widths} batch={batch} forward rel {ey:.2e} loss {loss:.6g}/{lo:.6g} "
          f"grad cos {cos:.6f} rel {rel:.3e}", flush=True)
    assert ey <= 3e-2
    assert abs(loss - lo) <= 2e-2 * lo
    assert cos >= 0.999 and rel <= 2e-2


def test_training_reduces_loss():
    from paper_2503_20605_amd import MLP
    x, t = _data(1024, 3)
    m = MLP(WIDTHS, 1024)
    m.set_params(ref.init_params(WIDTHS, 7))
    l0 = m.train_step(x, t, 1e-3)
    for _ in range(200):
        l = m.train_step(x, t, 1e-3)
    print(f"[mlp] loss {l0:.4e} -> {l:.4e}", flush=True)
    assert l < 0.2 * l0
    # the trained weights still agree with the reference network
    p = m.get_params().astype(np.float64)
    y = m.forward(x).cpu().numpy()
    yo, _ = ref.forward(p, WIDTHS, x)
    assert np.max(np.abs(y - yo)) <= 3e-2 * np.max(np.abs(yo))
