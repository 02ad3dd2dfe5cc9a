"""Host logic of bench.py that decides what the benchmark line reports:
the HBM traffic figure comes from the committed counter summary only while
the kernel sources are the ones the counters were taken with."""
import json
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _summary(config):
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{config}_f_grad.txt")
    with open(path) as fh:
        return [json.loads(line[5:]) for line in fh if line.startswith("JSON ")][0]


@pytest.mark.parametrize("config", ["c2", "c5"])
def test_traffic_is_the_dispatch_weighted_mean_of_the_summary(config, monkeypatch):
    rec = _summary(config)
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: rec["source_sha256"])
    ks = [v for n, v in rec["kernels"].items() if n.startswith("inla::tile_product_kernel<")]
    assert ks, "the summary lists the product kernel"
    want = sum(v["hbm_bytes_per_dispatch"] * v["dispatches"] for v in ks) / sum(v["dispatches"] for v in ks)
    got = bench.hbm_traffic(config, "inla::tile_product_kernel")
    assert got == pytest.approx(want, rel=1e-12)
    # a kernel the summary does not list has no figure
    assert bench.hbm_traffic(config, "inla::no_such_kernel") is None


def test_traffic_is_null_once_the_kernel_sources_change(monkeypatch):
    rec = _summary("c2")
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: "0" * 64)
    assert rec["source_sha256"] != "0" * 64
    assert bench.hbm_traffic("c2", "inla::tile_product_kernel") is None
    # and a workload without a summary has none either
    assert bench.hbm_traffic("no_such_workload", "inla::tile_product_kernel") is None

