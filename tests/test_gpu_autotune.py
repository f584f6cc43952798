"""The lattice-kernel autotuner through the C ABI: its choice rule (the
lowest-numbered variant within 2% of the fastest coupled step), the steps
it takes, its cache file, and that the run it leaves behind still matches
the oracle."""
import math

import numpy as np
import pytest

import workloads as wl
from helpers import gpu_solver

pytestmark = pytest.mark.gpu


def test_choice_rule_steps_and_cache(tmp_path):
    W = wl.droplet_2d_small()
    s = gpu_solver([W.params], [W.nodes])
    print("[autotune] 2D 128x64, 8 steps per timing", flush=True)
    v, ms = s.autotune(steps=8)
    assert 0 <= v < 32 and len(ms) == 32
    assert all(m > 0.0 and math.isfinite(m) for m in ms)
    best = min(ms)
    assert ms[v] <= 1.02 * best
    assert all(m > 1.02 * best for m in ms[:v])
    # every variant runs the given steps twice
    assert s.diagnostics(0)["step"] == 32 * 2 * 8
    cache = tmp_path / "tune.txt"
    v1, ms1 = s.autotune(steps=8, cache_path=str(cache))
    assert all(m > 0.0 for m in ms1)
    n1 = s.diagnostics(0)["step"]
    assert n1 == 2 * 32 * 2 * 8
    v2, ms2 = s.autotune(steps=8, cache_path=str(cache))
    assert v2 == v1 and all(m == -1.0 for m in ms2)
    assert s.diagnostics(0)["step"] == n1          # a cache hit runs no step
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1 and lines[0].endswith(f"|{v1}")
    assert s.diagnostics(0)["status"] == 0


def test_tuned_run_matches_the_oracle():
    """The steps the autotuner takes are ordinary steps of the run: 32 x 2 x 4
    tuning steps plus 56 more give the oracle's 400-step state."""
    import oracle as o
    W = wl.droplet_2d_small(steps=400)
    s = gpu_solver([W.params], [W.nodes])
    print("[autotune] 2D 128x64, 256 tuning steps + 144", flush=True)
    s.autotune(steps=4)
    s.step(400 - 32 * 2 * 4)
    q, _, _ = s.read_nodes(0)
    ref = o.run(W.params, W.nodes, 400)
    qo = ref["q"].T if ref["q"].shape[0] == 2 else ref["q"]
    assert np.max(np.abs(q - qo)) < 1e-5
