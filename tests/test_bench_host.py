"""Host logic of bench.py (no GPU): launch-form names are unique and
round-trip through --form, the kernels a step runs per form, the committed
traffic summaries are found for the profiled forms while the kernel sources
are unchanged (with or without a graph), and more than one GPU is refused
with a message."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_form_names_unique(bench):
    forms = bench.headline_forms()
    names = [bench.form_name(f) for f in forms]
    assert len(set(names)) == len(names)
    assert "per_step_4waves_ordered_graph" in names


def test_step_kernels(bench):
    assert bench.step_kernels({"mode": "fused"}, ("mlp",)) == ["k_run_fused"]
    assert bench.step_kernels({"mode": "step", "waves": 4, "order": 1}, ("repair",)) == \
        ["k_order", "k_step_mw<4>", "k_step_rest"]
    assert bench.step_kernels({"mode": "step", "waves": 4, "order": 1, "cut": 40, "mid": 16}, ("mlp",)) == \
        ["k_order", "k_step_mw<4>", "k_step_mw<2>", "k_step", "k_step_rest", "k_build_listed"]


def test_traffic_found_for_profiled_forms(bench):
    d = json.load(open(os.path.join(ROOT, "profiles", "step_multi2048_traffic.json")))
    if d["source_sha256_16"] != bench.source_hash():
        pytest.skip("kernel sources changed since the profile: traffic is reported as null")
    for name in d["forms"]:
        form = next(f for f in bench.headline_forms() if bench.form_name(f) == name)
        t = bench.measured_traffic(form, "multi2048")
        assert t == d["forms"][name]["traffic_bytes_per_step"]
        # the same kernels without a graph
        assert bench.measured_traffic(dict(form, graph=False), "multi2048") == t
    assert bench.measured_traffic({"mode": "fused", "graph": False}, "multi2048") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)
