"""Host-side bookkeeping of the benchmark script: lattice-kernel names per
variant, the source hash that keys the stored HBM-traffic readings, the
lookup of those readings, and the single-GPU guard.  No GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

CSRC = os.path.join(ROOT, "paper_2503_20605_amd", "csrc")


def _sources():
    def rd(name):
        with open(os.path.join(CSRC, name), "rb") as f:
            return f.read()
    return rd("lattice.hpp"), rd("kernels.hpp"), rd("iblb.hip")


def test_kernel_names_of_the_32_variants():
    """Variants v and v + 16 launch the same kernel form (only the host's
    block order differs); the 16 forms are distinct."""
    names = [bench.lb_kernel_name(3, 0, v) for v in range(32)]
    assert names[:16] == names[16:]
    assert len(set(names[:16])) == 16
    assert bench.lb_kernel_name(3, 0, 25) == "k_lb<3, 0, 256, 1, 1, 0, 1>"
    assert bench.lb_kernel_name(2, 1, 5, one=0) == "k_lb<2, 1, 64, 1, 0, 0, 0>"
    assert bench.lb_kernel_name(3, 0, 29, vis=1) == "k_lb<3, 0, 0, 1, 0, 1, 0>"
    assert [bench.LB_ORDER[v // 16] for v in (0, 15, 16, 31)] == ["xcd-runs", "xcd-runs", "storage", "storage"]


def test_source_hash_ignores_comments_and_layout_but_not_code():
    lat, ker, host = _sources()
    h = bench.lb_source_hash(lat, ker, host)
    assert h == bench.lb_source_hash()
    commented = ker.replace(b"namespace iblb {", b"namespace iblb {  // a remark\n\n", 1)
    assert bench.lb_source_hash(lat, commented, host) == h
    # a change in the lattice kernel's code, in the plane pad or in the
    # tile order changes the hash
    assert bench.lb_source_hash(lat, ker.replace(b"ppl = D.ppl", b"ppl = D.ppl + 0", 1), host) != h
    assert bench.lb_source_hash(lat, ker, host.replace(b"#define IBLB_PLANE_PAD 64", b"#define IBLB_PLANE_PAD 32", 1)) != h
    assert bench.lb_source_hash(lat, ker, host.replace(b"order_of(c->variant) == 0", b"order_of(c->variant) != 0", 1)) != h


def test_traffic_lookup_follows_the_stored_readings():
    with open(bench.TRAFFIC_FILE) as f:
        text = f.read()
    rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    assert rec["readings"]
    r = rec["readings"][0]
    got = bench.measured_traffic(r["kernel"], r["workload"], r["block_order"])
    if rec["source_hash"] == bench.lb_source_hash():
        assert got == round(r["fetch_bytes"] + r["write_bytes"])
    else:  # readings of an older kernel are not reported
        assert got is None
    assert bench.measured_traffic("k_lb<no such kernel>", r["workload"], r["block_order"]) is None
    other = "storage" if r["block_order"] == "xcd-runs" else "xcd-runs"
    match = [x for x in rec["readings"] if x["kernel"] == r["kernel"] and x["workload"] == r["workload"]
             and x["block_order"] == other]
    if not match:
        assert bench.measured_traffic(r["kernel"], r["workload"], other) is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "exactly one GPU" in json.loads(p.stdout.strip().splitlines()[-1])["error"]


@pytest.mark.parametrize("dim,storage,want", [(2, 0, 72), (2, 1, 36), (3, 0, 152), (3, 2, 76)])
def test_algorithmic_bytes_per_cell(dim, storage, want):
    assert bench.bytes_per_cell(dim, storage) == want
