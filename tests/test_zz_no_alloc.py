"""The allocation-free forward pass of the warm-start network
(iblb_mlp_forward_noalloc, static device scratch) against the workspace
forward pass (iblb_mlp_forward) through the C ABI: the same kernels on the
same inputs, so the outputs must agree bit for bit, on two calls in a row
(the second with fewer rows, so stale scratch from the first would show),
and a batch whose scratch exceeds the static array is refused."""
import numpy as np
import pytest

from oracle import mlp as ref

pytestmark = pytest.mark.gpu

WIDTHS = [4, 256, 256, 256, 1280]


def test_noalloc_forward_matches_workspace_forward_twice():
    import torch
    from paper_2503_20605_amd import MLP, IblbError
    m = MLP(WIDTHS, 1024)
    m.set_params(ref.init_params(WIDTHS, 7))
    rng = np.random.default_rng(3)
    for batch in (1000, 333):
        print(f"[noalloc] batch {batch}", flush=True)
        x = m._dev(rng.uniform(-1, 1, (batch, WIDTHS[0])))
        want = m.forward(x).cpu().numpy()
        y = torch.full((batch, WIDTHS[-1]), float("nan"), dtype=torch.float32, device=m.device)
        m.forward_noalloc(x, y)
        m.stream.synchronize()
        got = y.cpu().numpy()
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, want), float(np.max(np.abs(got - want)))
    # a row of this network takes 2 * 4 + 4 * 256 + 2 * 2 * 256 = 2056 bytes
    # of scratch, so 8 MiB hold 4080 rows: 5000 rows are refused before
    # anything is launched
    x = m._dev(rng.uniform(-1, 1, (5000, WIDTHS[0])))
    y = torch.empty((5000, WIDTHS[-1]), dtype=torch.float32, device=m.device)
    with pytest.raises(IblbError) as e:
        m.forward_noalloc(x, y)
    assert e.value.code == -1
    m.close()
