"""Host-side arithmetic of bench.py: the roofline object built from a
kernel time, a stored counter profile and the measured ceilings, the lookup
of stored profiles by source hash, and the one-GPU guard.  No GPU needed."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

CEIL = {"copy": {"gbs": 5000.0}, "read": {"gbs": 6000.0},
        "valu": {"fp32_fma": {"lane_ops_per_s": 40e12}}}
PROF = {"hbm_bytes_per_launch": 2.0e9, "fetch_bytes": 1.5e9, "write_bytes": 0.5e9,
        "l2_hit_rate": 0.9, "valu_instr_per_launch": 1.0e9}


def test_roofline_from_profile_and_ceilings():
    # 100 ms, 6.4e9 steps (1e8 wavefront-steps), 1e6 rays
    r = bench.roofline_of("k_forward_f32k", 100.0, 6.4e9, 1e6, PROF, CEIL)
    assert r["bound"] == "alu" and r["unit"] == "T VALU lane-ops/s"
    # 1e9 wavefront instructions x 64 lanes / 0.1 s = 6.4e11 lane-ops/s
    assert r["achieved"] == pytest.approx(0.64)
    assert r["peak"] == pytest.approx(40.0)
    assert r["frac"] == pytest.approx(0.64 / 40.0, rel=1e-3)
    assert r["valu_instr_per_wavefront_step"] == pytest.approx(10.0)
    assert r["traffic"] == 2.0e9
    # 2 GB in 0.1 s = 20 GB/s, against 8 TB/s and the 5 TB/s copy
    assert r["hbm"]["counter_gbs"] == pytest.approx(20.0)
    assert r["hbm"]["frac_of_peak"] == pytest.approx(20.0 / 8000.0, abs=1e-4)
    assert r["hbm"]["frac_of_achievable_copy"] == pytest.approx(20.0 / 5000.0, abs=1e-4)
    # algorithmic: 13 B per step and 32 B per ray for the FP32-Kahan forward
    alg = r["algorithmic"]
    assert (alg["bytes_per_step"], alg["bytes_per_ray"]) == (13, 32)
    assert alg["bytes"] == pytest.approx(6.4e9 * 13 + 1e6 * 32)
    assert alg["gbs"] == pytest.approx((6.4e9 * 13 + 1e6 * 32) / 0.1 / 1e9, abs=0.05)


def test_per_unit_bytes_of_every_kernel():
    assert bench.BYTES_PER_STEP == {"k_forward_f32k": 13, "k_forward_f64": 17, "k_backward": 21,
                                    "k_forward_adjoint": 34}
    # the fused pass moves what the two kernels move, with one source read
    assert bench.BYTES_PER_STEP["k_forward_adjoint"] == (bench.BYTES_PER_STEP["k_forward_f32k"]
                                                         + bench.BYTES_PER_STEP["k_backward"])
    r = bench.roofline_of("k_shielding_f32", 50.0, 1e9, 1e6, None, CEIL, 25, 5.5)
    assert r["algorithmic"]["bytes"] == pytest.approx(25e9 + 5.5e6)


def test_roofline_without_profile_leaves_measured_fields_null():
    r = bench.roofline_of("k_forward_adjoint", 10.0, 1e9, 1e6, None, CEIL)
    assert r["achieved"] is None and r["frac"] is None and r["traffic"] is None
    assert "hbm" not in r and "no committed profile" in r["note"]
    r = bench.roofline_of("k_forward_adjoint", 10.0, 1e9, 1e6, PROF, None)
    assert r["peak"] is None and r["frac"] is None and r["achieved"] is not None


def test_stored_counters_require_the_current_sources(tmp_path, monkeypatch):
    prof = dict(PROF, source_hash="abc")
    (tmp_path / "profiles").mkdir()
    with open(tmp_path / "profiles" / "traffic.json", "w") as fh:
        json.dump({"wl": {"k_forward_f32k": prof}}, fh)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.stored_counters("k_forward_f32k", "wl", "abc") == prof
    assert bench.stored_counters("k_forward_f32k", "wl", "abd") is None
    assert bench.stored_counters("k_backward", "wl", "abc") is None
    assert bench.stored_counters("k_forward_f32k", "other", "abc") is None


def test_committed_profiles_match_their_recorded_hashes():
    # every committed entry names the sources it was taken on, and its HBM
    # bytes are the scaled fetched plus written bytes (each rounded apart)
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        rec = json.load(fh)
    assert "calibration" in rec and rec["calibration"]["fetch_factor"] > 0
    for wl, kernels in rec.items():
        if wl == "calibration":
            continue
        for k, e in kernels.items():
            assert len(e["source_hash"]) == 16
            assert abs(e["hbm_bytes_per_launch"] - e["fetch_bytes"] - e["write_bytes"]) <= 2
            assert 0.0 <= e["l2_hit_rate"] <= 1.0


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU only" in p.stderr and p.stdout == ""


def test_source_hash_ignores_comments_but_not_code(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_2605_09882_amd", "csrc")
    dst = tmp_path / "paper_2605_09882_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in ("rt_ray.h", "rt_walk.hip", "rt_octree.cpp"):
        with open(os.path.join(src, f)) as fh:
            (dst / f).write_text(fh.read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    walk = (dst / "rt_walk.hip").read_text()
    (dst / "rt_walk.hip").write_text("// a new comment\n/* and a\n block */" + walk.replace("\n", "\n\n", 3))
    assert bench.kernel_source_hash() == h0
    (dst / "rt_walk.hip").write_text(walk.replace("kFlushEvery = 16", "kFlushEvery = 17"))
    assert bench.kernel_source_hash() != h0
