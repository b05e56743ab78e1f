"""bench.py on the smallest workload (uniform 32^3, 393,216 rays), run as a
child process on the GPU: its one JSON line carries every field of the
benchmark line, the roofline object and the CPU baseline, with consistent
values.  A guard on the line's shape, not a measurement."""

import json
import os
import subprocess
import sys

import pytest

from gpu_common import require_gpu

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def line():
    require_gpu()
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "0", "--steps", "2",
                        "--warmup", "1", "--copy-gb", "0.25", "--cpu-stride", "64", "--no-grid-tree"],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert p.returncode == 0, p.stderr[-2000:]
    out = [x for x in p.stdout.splitlines() if x.strip()]
    assert len(out) == 1, p.stdout
    return json.loads(out[0])


def test_benchmark_fields(line):
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in line, k
    assert line["n_gpus"] == 1 and line["steps"] == 2 and line["warmup"] == 1
    assert line["higher_is_better"] is True and line["vs_baseline"] is None
    assert line["data"] == "synthetic"
    c = line["config"]
    assert c["workload"] == "uniform32_iid_nside1" and c["rays"] == 32768 * 12
    assert c["ray_leaf_steps"] == 8062760
    # value is the forward's steps over the pass time
    assert line["value"] == pytest.approx(c["ray_leaf_steps"] / (line["ms_per_step"] / 1e3), rel=2e-3)


def test_roofline_object(line):
    for key in ("roofline", "forward_roofline", "adjoint_roofline"):
        r = line[key]
        assert r["bound"] == "alu" and r["unit"] == "T VALU lane-ops/s"
        assert r["peak"] > 0
        for k in ("achieved", "frac", "traffic"):
            assert k in r
        if r["achieved"] is not None:
            assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], rel=1e-2)
            assert 0.0 < r["frac"] < 1.0
            assert r["traffic"] > 0
        alg = r["algorithmic"]
        assert alg["bytes"] == alg["bytes_per_step"] * line["config"]["ray_leaf_steps"] \
            + alg["bytes_per_ray"] * line["config"]["rays"]
    ceil = line["ceilings"]
    assert 0 < ceil["copy"]["gbs"] < 8000 and 0 < ceil["read"]["gbs"] < 8000


def test_cpu_baseline_object(line):
    cb = line["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] == 1 and cb["value"] > 0
    assert cb["unit"] == line["unit"]
    assert "every 64th source" in cb["sample"]
    assert cb["all_cores"]["cores"] >= 1 and cb["all_cores"]["value"] > 0
