"""Benchmark of the reverse ray walk on one MI355X.

Workload (default): the paper-scale cloud -- a 512^3 lognormal field with a
k^-4 spectrum and sigma_ln(rho) = 2, coarsened to a leaf-only octree by the
density + uniformity rule (about 39M leaves), rays from all 512^3 cell
centres in the 12 HEALPix directions (nside = 1), about 1.6e9 rays.

One step = one pass of the whole hot path over that batch: the HEALPix
direction table, the FP32-Kahan forward walk (N and A = exp(-kappa N)), and
the adjoint walk of L = sum w A (w ~ U(0,1) per ray) scattering dL/drho onto
the leaves, both in the one kernel of rt_columns_with_adjoint (each
wavefront walks its rays for N and A, then walks them again to scatter).
The value is ray-leaf steps per second of that pass: the leaf visits of the
forward walk (the adjoint re-walks the same ones) divided by the time of the
pass.  The same pass as two calls (rt_columns, then rt_columns_backward, the
path of the autograd function) is timed after it; the FP64 walk over the
same rays, and the
several-fields walk (n_H and three lines: per-source escape probabilities
and A_V,eff), and the construction of the contribution grid from the 512^3
grid on the device, are timed after the pass and reported beside it.

Prints one JSON line.  --gpus N > 1 is refused: the library runs on one GPU.
"""

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue rate from the chip's unit counts and clock: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz (one wave64 instruction per SIMD every 4 cycles).  The
# FP32 FMA probe issues faster than this, so the roofline's peak is the
# probe's rate measured in the same run; this figure is reported beside it.
VALU_NOMINAL_LANE_OPS = 256 * 4 * 16 * 2.4e9
CPU_SAMPLE_STRIDE = 2048
# Algorithmic bytes of the method per ray-leaf step: the leaf record (Morton
# key 8 B, level 1 B, value 4 B FP32 or 8 B FP64); the adjoint re-reads the
# record and adds into the gradient of the leaf, counted as the 4 B read and
# 4 B write of an FP32 gradient (the FP64 gradient kept here moves 8 + 8 B).
# Per ray: the source (24 B), the outputs, and the adjoint's loss weight.
BYTES_PER_STEP = {"k_forward_f32k": 13, "k_forward_f64": 17, "k_backward": 21,
                  "k_forward_adjoint": 34}
BYTES_PER_RAY = {"k_forward_f32k": 32, "k_forward_f64": 40, "k_backward": 32,
                 "k_forward_adjoint": 36}
# several-fields walk: n_H and three lines (key 8 + level 1 + 4 or 8 per field
# per step)
SHIELD_LINES = 3


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", type=int, default=4, help="workload index (0..4)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-stride", type=int, default=CPU_SAMPLE_STRIDE,
                   help="the CPU baseline walks every n-th source with all directions")
    p.add_argument("--no-fp64", action="store_true")
    p.add_argument("--no-shielding", action="store_true")
    p.add_argument("--no-grid-tree", action="store_true")
    p.add_argument("--copy-gb", type=float, default=4.0,
                   help="size of the stream probes' buffers (GB) that measure achievable bandwidth")
    p.add_argument("--ceilings-only", action="store_true",
                   help="run only the bandwidth and VALU probes and print their JSON")
    return p.parse_args()


_COMMENT = re.compile(r"//[^\n]*|/\*.*?\*/", re.S)


def kernel_source_hash(kernel_file="rt_walk.hip"):
    """Hash of the sources that fix what a kernel executes: the device walk,
    the kernel's own source with its launch shape, and the octree's search
    structures.  Comments and whitespace are left out (none of these files
    holds a comment marker inside a string), so a stored profile stays valid
    until the code itself changes."""
    h = hashlib.sha256()
    for f in ("rt_ray.h", kernel_file, "rt_octree.cpp"):
        with open(os.path.join(ROOT, "paper_2605_09882_amd", "csrc", f)) as fh:
            code = _COMMENT.sub(" ", fh.read())
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()[:16]


def stored_counters(kernel, workload, src_hash):
    """The committed rocprofv3 counter summary of this kernel and workload
    (HBM bytes per launch from FETCH_SIZE + WRITE_SIZE, scaled against a
    copy of known size; L2 hit rate; VALU instructions per launch), if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    e = rec.get(workload, {}).get(kernel)
    if not e or e.get("source_hash") != src_hash:
        return None
    return e


def _best_ms(torch, fn, reps=5):
    """Shortest of reps timed calls of fn, by HIP events on torch's current
    stream (the stream the library's calls are queued on)."""
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        s.record()
        fn()
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e)
        best = ms if best is None else min(best, ms)
    return best


def ceilings(torch, dev, gb):
    """The two ceilings of the roofline, measured by the library's probes on
    this GPU: achievable HBM bandwidth (a hand-written 16-byte stream copy
    and a read-only stream over gb GB buffers) and the VALU issue rate of
    FP64 fma, int32 xor-add and FP32 fma chains of known length."""
    from paper_2605_09882_amd import _abi

    stream = torch.cuda.current_stream(dev).cuda_stream
    g = _abi.rt_calib_stream_granule()
    nbytes = max(1, int(gb * 1e9) // g) * g
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    sink = torch.empty(nbytes // g, dtype=torch.int32, device=dev)
    ms_copy = _best_ms(torch, lambda: _abi.rt_calib_copy(a.data_ptr(), b.data_ptr(), nbytes, stream))
    if not torch.equal(a, b):
        raise RuntimeError("stream copy probe produced a wrong copy")
    ms_read = _best_ms(torch, lambda: _abi.rt_calib_read(a.data_ptr(), nbytes, sink.data_ptr(), stream))
    del a, b, sink
    out = {"copy": {"bytes_per_launch": 2 * nbytes, "ms": round(ms_copy, 4),
                    "gbs": round(2 * nbytes / (ms_copy / 1e3) / 1e9, 1)},
           "read": {"bytes_per_launch": nbytes, "ms": round(ms_read, 4),
                    "gbs": round(nbytes / (ms_read / 1e3) / 1e9, 1)}}
    props = torch.cuda.get_device_properties(dev)
    cus = props.multi_processor_count
    # 16 wavefronts per SIMD (4 SIMDs per CU) hide the chains' latency
    n_threads = cus * 4 * 16 * 64
    iters = 20000
    valu = {}
    res = torch.empty(n_threads, dtype=torch.int32, device=dev)
    for kind, name, per_iter in ((0, "fp64_fma", 8), (1, "int32_xad", 9), (2, "fp32_fma", 8)):
        ms = _best_ms(torch, lambda: _abi.rt_calib_valu(kind, n_threads, iters, res.data_ptr(), stream), 3)
        instr = n_threads // 64 * iters * per_iter
        valu[name] = {"wave_instr_per_launch": instr, "ms": round(ms, 4),
                      "wave_instr_per_s": instr / (ms / 1e3),
                      "lane_ops_per_s": 64 * instr / (ms / 1e3)}
    del res
    out["valu"] = valu
    out["compute_units"] = cus
    return out


def roofline_of(kname, kms, steps, rays, prof, ceil, bytes_per_step=None, bytes_per_ray=None):
    """Roofline of one kernel launch of kms milliseconds over `steps`
    ray-leaf steps and `rays` rays.

    The walks are bound by vector-instruction issue, not by HBM: their
    leaf records are served from the caches (the counters show a small
    fraction of the HBM peak while the VALU issue rate is near its ceiling).
    So `achieved` is the kernel's VALU issue rate: the wavefront instructions
    one launch issues (SQ_INSTS_VALU, from the committed profile of this
    kernel and workload, valid while the kernel sources are unchanged) times
    64 lanes, over the launch duration measured here; `peak` is the issue
    rate of the FP32 FMA probe measured in this run.  HBM is reported beside
    it from counter bytes (FETCH_SIZE + WRITE_SIZE, calibrated), against the
    8 TB/s peak and against the stream probes' achievable rates; the
    method's algorithmic bytes are reported as such, without a fraction of
    the HBM peak (the caches serve most of them)."""
    sec = kms / 1e3
    probe = ceil["valu"]["fp32_fma"]["lane_ops_per_s"] if ceil else None
    r = {"bound": "alu", "achieved": None, "peak": round(probe / 1e12, 3) if probe else None,
         "unit": "T VALU lane-ops/s", "frac": None,
         "traffic": prof["hbm_bytes_per_launch"] if prof else None,
         "kernel": kname, "kernel_ms": round(kms, 3),
         "peak_source": "rt_calib_valu FP32 FMA chains, measured in this run",
         "peak_nominal": round(VALU_NOMINAL_LANE_OPS / 1e12, 3),
         "peak_nominal_source": "256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz"}
    if prof:
        instr = prof["valu_instr_per_launch"]
        lane_ops = 64 * instr / sec
        r["achieved"] = round(lane_ops / 1e12, 3)
        if probe:
            r["frac"] = round(lane_ops / probe, 4)
        r["valu_instr_per_launch"] = instr
        r["valu_instr_per_wavefront_step"] = round(instr / (steps / 64), 2)
        gbs = prof["hbm_bytes_per_launch"] / sec / 1e9
        r["hbm"] = {"counter_gbs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                    "fetch_bytes": prof["fetch_bytes"], "write_bytes": prof["write_bytes"],
                    "l2_hit_rate": prof["l2_hit_rate"]}
        if ceil:
            r["hbm"]["achievable_copy_gbs"] = ceil["copy"]["gbs"]
            r["hbm"]["achievable_read_gbs"] = ceil["read"]["gbs"]
            r["hbm"]["frac_of_achievable_copy"] = round(gbs / ceil["copy"]["gbs"], 4)
    else:
        r["note"] = "no committed profile of the current kernel sources: VALU and counter fields null"
    bps = BYTES_PER_STEP.get(kname, bytes_per_step)
    bpr = BYTES_PER_RAY.get(kname, bytes_per_ray)
    if bps is not None:
        alg = steps * bps + rays * bpr
        r["algorithmic"] = {"bytes_per_step": bps, "bytes_per_ray": bpr, "bytes": alg,
                            "gbs": round(alg / sec / 1e9, 1),
                            "note": "compulsory leaf-record bytes of the method, mostly served "
                                    "from the caches; not a fraction of the HBM peak"}
    return r


def cpu_baseline(w, dirs_host, stride):
    """The oracle on every stride-th source with all directions:
    single-threaded (the reported value), and split over all available
    cores."""
    import numpy as np

    import oracle

    src = w.sources[::stride]
    t0 = time.perf_counter()
    out = oracle.columns(w.tree, src, dirs_host, w.kappa, rho32=w.tree.rho.astype(np.float32))
    dt = time.perf_counter() - t0
    steps = int(out["steps"].sum())
    # the same sample split over every core this process may use
    host = host_cpu()
    nc = max(1, int(host["cores_available"] or 1))
    t1 = time.perf_counter()
    oracle.columns(w.tree, src, dirs_host, w.kappa, rho32=w.tree.rho.astype(np.float32), threads=nc)
    dt_all = time.perf_counter() - t1
    return {"value": steps / dt, "unit": "ray-leaf steps/s", "cores": 1, "kind": "oracle",
            "all_cores": {"value": steps / dt_all, "cores": nc},
            "sample": f"every {stride}th source ({src.shape[0]} sources x "
                      f"{dirs_host.shape[0]} dirs = {src.shape[0] * dirs_host.shape[0]} rays, "
                      f"{steps} leaf steps, {dt:.1f} s, FP64 + FP32-Kahan columns)",
            "host": host}


def host_cpu():
    """CPU model and the number of cores this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count()
    return {"cpu": model, "cores_available": n}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "design is described but not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2605_09882_amd as rt
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    ceil = ceilings(torch, dev, args.copy_gb) if args.copy_gb > 0 else None
    if ceil:
        v = ceil["valu"]
        log(f"stream copy {ceil['copy']['gbs']:.0f} GB/s, read {ceil['read']['gbs']:.0f} GB/s; VALU "
            + ", ".join(f"{k} {x['wave_instr_per_s']:.3e} wave-instr/s" for k, x in v.items()))
    if args.ceilings_only:
        print(json.dumps({"ceilings": ceil}), flush=True)
        return

    t0 = time.time()
    w = W.make_workload(args.workload)
    log(f"workload {w.name}: {w.tree.n} leaves, {w.sources.shape[0]} sources, nside {w.nside}, "
        f"generated in {time.time() - t0:.1f} s")

    tree = rt.Octree(w.tree.keys, w.tree.levels, w.tree.depth, dev)
    src = torch.as_tensor(w.sources).to(dev)
    rho32 = torch.as_tensor(w.tree.rho.astype(np.float32)).to(dev)
    rho64 = torch.as_tensor(w.tree.rho).to(dev)
    S = src.shape[0]
    Dn = rt.healpix_npix(w.nside)
    gen = torch.Generator(device=dev)
    gen.manual_seed(3000 + w.index)
    wgt = torch.rand((Dn, S), generator=gen, device=dev, dtype=torch.float32).t()
    grad = torch.zeros(w.tree.n, dtype=torch.float64, device=dev)
    kappa = w.kappa

    dirs_host = rt.healpix_dirs(w.nside)
    dirs = torch.as_tensor(dirs_host).to(dev)
    steps_t, _, _ = rt.columns_trace(tree, src, dirs)
    total_steps = int(steps_t.to(torch.int64).sum())
    if int(steps_t.min()) < 1:
        raise RuntimeError("a ray of the workload was rejected")
    del steps_t
    rays = S * Dn
    log(f"{rays} rays, {total_steps} ray-leaf steps ({total_steps / rays:.1f} per ray)")
    src_hash = kernel_source_hash()

    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def one_step(marks=None):
        d = torch.as_tensor(rt.healpix_dirs(w.nside)).to(dev, non_blocking=False)
        grad.zero_()
        if marks:
            marks[0].record()
        N, A, _ = rt.columns_with_adjoint(tree, rho32, src, d, kappa, wA=wgt, grad=grad)
        if marks:
            marks[1].record()
        return N, A

    def separate_step(marks):
        d = torch.as_tensor(rt.healpix_dirs(w.nside)).to(dev, non_blocking=False)
        marks[0].record()
        N, A = rt.columns(tree, rho32, src, d, kappa)
        marks[1].record()
        grad.zero_()
        marks[2].record()
        rt.columns_backward(tree, src, d, kappa, gA=wgt, A=A, grad=grad)
        marks[3].record()
        return N, A

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()

    marks = [[ev() for _ in range(2)] for _ in range(args.steps)]
    start, stop = ev(), ev()
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record()
    for k in range(args.steps):
        one_step(marks[k])
    stop.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    t_gpu = start.elapsed_time(stop) / 1e3
    t_total = max(t_wall, t_gpu)
    ms_step = 1e3 * t_total / args.steps
    fused_ms = float(np.mean([m[0].elapsed_time(m[1]) for m in marks]))
    value = total_steps * args.steps / t_total
    log(f"step {ms_step:.1f} ms: forward and adjoint in one kernel {fused_ms:.1f} ms")

    # the same pass as two calls (the autograd function's path)
    separate_step([ev() for _ in range(4)])
    torch.cuda.synchronize()
    smarks = [[ev() for _ in range(4)] for _ in range(args.steps)]
    for k in range(args.steps):
        separate_step(smarks[k])
    torch.cuda.synchronize()
    fwd_ms = float(np.mean([m[0].elapsed_time(m[1]) for m in smarks]))
    bwd_ms = float(np.mean([m[2].elapsed_time(m[3]) for m in smarks]))
    sep_ms = float(np.mean([m[0].elapsed_time(m[3]) for m in smarks]))
    log(f"separate calls {sep_ms:.1f} ms: forward {fwd_ms:.1f} ms, adjoint {bwd_ms:.1f} ms")

    # FP64 walk of the same rays, for comparison
    fp64 = None
    if not args.no_fp64:
        rt.columns(tree, rho64, src, dirs, kappa)
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record()
        for _ in range(args.steps):
            N64, _ = rt.columns(tree, rho64, src, dirs, kappa)
        b.record()
        torch.cuda.synchronize()
        ms64 = a.elapsed_time(b) / args.steps
        fp64 = {"ms": round(ms64, 3), "steps_per_s": total_steps / (ms64 / 1e3),
                "roofline": roofline_of("k_forward_f64", ms64, total_steps, rays,
                                        stored_counters("k_forward_f64", w.name, src_hash), ceil)}
        del N64
        log(f"FP64 walk {ms64:.1f} ms")

    # several fields per leaf (n_H and three lines) over the same rays:
    # per-source escape probabilities and A_V,eff from one walk per ray, with
    # the fields stored in FP32 (rt_shielding_f32) and in FP64 (rt_shielding)
    shield = None
    if not args.no_shielding:
        inp = W.line_inputs(w.tree, w.sources, SHIELD_LINES, 6000 + w.index)
        T = torch.as_tensor(inp["temp"]).to(dev)
        nf = 1 + SHIELD_LINES
        # per source: the point 24 B, T 8 B, A_V,eff 8 B, one beta per line;
        # counted per ray here (the sources over their directions)
        per_ray = (24 + 8 + 8 * nf) / Dn
        shield = {"fields": nf}
        for name, dtype, fbytes in (("f32_fields", np.float32, 4), ("f64_fields", np.float64, 8)):
            F = torch.as_tensor(inp["fields"].astype(dtype)).to(dev)

            def shield_call():
                return rt.shielding(tree, F, src, dirs, inp["length"], temp=T, vturb=inp["vturb"],
                                    line_A=inp["line_A"], line_nu=inp["line_nu"])

            shield_call()
            torch.cuda.synchronize()
            a, b = ev(), ev()
            a.record()
            for _ in range(args.steps):
                res = shield_call()
            b.record()
            torch.cuda.synchronize()
            ms_sh = a.elapsed_time(b) / args.steps
            kname = f"k_shielding_{name[:3]}"
            prof_sh = stored_counters(kname, w.name, kernel_source_hash("rt_fields.hip"))
            shield[name] = {
                "ms": round(ms_sh, 3), "steps_per_s": total_steps / (ms_sh / 1e3),
                "field_steps_per_s": nf * total_steps / (ms_sh / 1e3),
                "vs_fp64_walk": round(ms_sh / fp64["ms"], 3) if fp64 else None,
                "av_eff_median": float(res["av_eff"].median()),
                "roofline": roofline_of(kname, ms_sh, total_steps, rays, prof_sh, ceil,
                                        9 + fbytes * nf, per_ray)}
            del F, res
            log(f"several-fields walk ({nf} fields, {name}) {ms_sh:.1f} ms")
        del T

    # the contribution grid rebuilt on the device from the workload's 512^3
    # grid (the same field and rule as the host generator)
    build = None
    if not args.no_grid_tree and "density_floor" in w.info:
        n_side = 1 << w.tree.depth
        field = W.lognormal(W.gaussian_random_field(n_side, -4.0, 1000 + w.index), 2.0)
        grid = torch.as_tensor(W.octree.grid_to_morton(field)).to(dev)
        del field
        floor = w.info["density_floor"]
        keys, _, _ = rt.grid_tree(grid, w.tree.depth, floor)
        same = bool(torch.equal(keys, torch.as_tensor(w.tree.keys.view(np.int64)).to(dev)))
        del keys
        times = []
        for _ in range(max(args.steps, 3)):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            keys, _, _ = rt.grid_tree(grid, w.tree.depth, floor)
            times.append(time.perf_counter() - t1)
            del keys
        ms_b = 1e3 * min(times)
        # and the octree handle staged from the device arrays (checks + top table)
        keys, levels, _ = rt.grid_tree(grid, w.tree.depth, floor)
        t_oct = []
        for _ in range(3):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            tree_dev = rt.Octree.from_device(keys, levels, w.tree.depth)
            torch.cuda.synchronize()
            t_oct.append(time.perf_counter() - t1)
            del tree_dev
        del keys, levels
        cells = grid.numel()
        build = {"cells": cells, "leaves": w.tree.n, "ms": round(ms_b, 3),
                 "cells_per_s": cells / (ms_b / 1e3), "same_tree_as_host": same,
                 "octree_from_device_ms": round(1e3 * min(t_oct), 3),
                 "timing": "wall clock per call, including the leaf-count read-back"}
        del grid
        log(f"grid tree on the device: {cells} cells -> {w.tree.n} leaves in {ms_b:.2f} ms "
            f"(same as the host tree: {same}); octree handle from the device arrays in "
            f"{build['octree_from_device_ms']:.2f} ms")

    # roofline of the pass's kernel (see roofline_of)
    kname, kms = "k_forward_adjoint", fused_ms
    roofline = roofline_of(kname, kms, total_steps, rays, stored_counters(kname, w.name, src_hash),
                           ceil)
    adjoint_roofline = roofline_of("k_backward", bwd_ms, total_steps, rays,
                                   stored_counters("k_backward", w.name, src_hash), ceil)
    forward_roofline = roofline_of("k_forward_f32k", fwd_ms, total_steps, rays,
                                   stored_counters("k_forward_f32k", w.name, src_hash), ceil)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, dirs_host, max(1, args.cpu_stride))
        log(f"cpu baseline {cpu['value']:.3e} steps/s ({cpu['sample']})")

    line = {
        "metric": "ray-leaf steps/sec (FP32-Kahan forward + adjoint pass; FP64 walk beside it)",
        "pass": "forward and adjoint in one kernel (rt_columns_with_adjoint)",
        "value": value,
        "unit": "ray-leaf steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (Kahan) accumulation, f64 traversal",
        "data": "synthetic",
        "config": {"workload": w.name, "leaves": w.tree.n, "sources": S, "directions": Dn,
                   "rays": rays, "ray_leaf_steps": total_steps, "kappa": kappa,
                   "parallelism": "single GPU"},
        "fused_kernel_ms": round(fused_ms, 3),
        "separate_calls": {"ms": round(sep_ms, 3), "steps_per_s": total_steps / (sep_ms / 1e3),
                           "note": "rt_columns then rt_columns_backward (the autograd path)"},
        "forward_ms": round(fwd_ms, 3),
        "adjoint_ms": round(bwd_ms, 3),
        "fp32k_forward_steps_per_s": total_steps / (fwd_ms / 1e3),
        "adjoint_steps_per_s": total_steps / (bwd_ms / 1e3),
        "fp64_walk": fp64,
        "shielding": shield,
        "grid_tree": build,
        "roofline": roofline,
        "forward_roofline": forward_roofline,
        "adjoint_roofline": adjoint_roofline,
        "ceilings": ceil,
        "cpu_baseline": cpu,
        "kernel_source_hash": src_hash,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
