"""Throughput of the fused D3Q19 step + kinetic sensor on one MI355X.

Default workload: the 128^3 D3Q19 lid-driven cavity in float32 (lid 0.05,
Re 1000, halfway bounce-back walls), with the sensor, its 8^3 block maxima
and the refine/coarsen flags evaluated at every step.  A "step" is one
launch of the fused kernel over the whole grid.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W]
                  [--workload cavity128|cavity256|channel256|refined256|predictor|cavity64_2d|conv_sweep]
                  [--storage f32|f32s|f64|f16s|bf16s|f16sr|bf16sr] [--lattice 19|27]
                  [--smagorinsky C] [--no-cpu-baseline] [--no-copy-calibration]

MLUPS = cells * K / t / 1e6 over K back-to-back steps (HIP events on the
library's stream).  The roofline entry prices the dominant kernel at its
algorithmic traffic, one read and one write of every population per cell
update (2 * q * bytes per value), against the 8 TB/s HBM3E peak.  Its
duration is the timed region's mean step period; with the in-place scheme
two kernels alternate (gather-scatter and local), and single launches
bracketed by events (per_kernel_us_single_launch, which also time the event
packets) split that period between them (per_kernel_us); "kernel" names the
slower one, whose figure is "achieved".  A 1 GiB device copy of random data
is timed for comparison (copy_calibration, frac_of_copy).
"traffic" is the measured HBM bytes per launch of that kernel from the
committed rocprofv3 counter summary, when it was taken on the current kernel
source.  The 128^3 in-place state (152 MiB) can stay in the 256 MB Infinity
Cache (roofline.cache_resident); the default workload therefore also times
the same step + sensor on the 256^3 cavity in float32 (ping-pong, 2.55 GB
moved per step, beyond that cache), reported as roofline_cache_proof.  The
CPU baseline is the FP64 oracle timed on the host on a short run of the same
workload.

--workload refined256: the two-level patch hierarchy.  A 256^3 D3Q19
cavity (Re 1000) runs 1000 coarse steps, up to 400 cubic patches with fine
edges from {16, 24, 32, 48} are placed on the blocks its sensor flags
(seeded), and K coarse steps (2K fine steps, graph-replayed) are timed.
The value counts lattice updates of both levels; the roofline entry prices
the fine step (all patches, one persistent launch) at one read and one write
of every population of every fine cell, its duration timed in production
order after the timed region (lbm_hierarchy_profile: HIP events between the
launches of 4 coarse steps; the coarse step, ghost fill and the second fine
step, which also restricts to the coarse level, are listed beside it under
per_kernel_us).

--workload cavity64_2d: the 64^2 D2Q9 float64 cavity (Re 100, 2000 steps,
sensor every 100), whose steps are bound by launch latency: timed with up to
5 sensor-free steps per launch (lbm_set_multistep, the default for such
grids) and with one launch per step, launched from the host and replayed in
runs of 98 steps from HIP graphs (lbm_use_graphs).

--workload predictor: K training iterations (forward, backward, Adam) of
the flag predictor on a seeded batch of 8 block grids of 16^3; the roofline
entry prices one 16 -> 16 channel convolution at its algorithmic flops
against the dense BF16 matrix-core peak.  The batch stays on the device and
one iteration is replayed from a HIP graph (eager_iterations_per_s gives the
same loop launched kernel by kernel).

--workload conv_sweep: the predictor's 16 -> 16 convolution (forward and
weight gradient) on 8, 32, 128 and 512 block grids of 16^3, each timed over
20 graph-replayed launches; one JSON line with a row per batch.
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _workload(name, storage):
    import lbm_inputs
    if name == "cavity128":
        return lbm_inputs.cavity3d(n=128, storage=storage)
    if name == "cavity256":
        return lbm_inputs.cavity3d(n=256, storage=storage)
    if name == "channel256":
        return lbm_inputs.channel3d(n=256, storage=storage)
    raise SystemExit(f"unknown workload {name}")


def _traffic_from_profile(kernel_tag, source="step_kernel.hpp"):
    """HBM bytes per launch measured by rocprofv3 (FETCH_SIZE + WRITE_SIZE,
    scaled by a copy-kernel calibration), read from the committed summary if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_tag}.txt")
    if not os.path.exists(path):
        return None
    src = os.path.join(ROOT, "paper_1507_06767_amd", "csrc", source)
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != digest:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_env():
    """GPU, HIP and torch versions and host CPU of this run."""
    import torch
    cpu = ""
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    p = torch.cuda.get_device_properties(0)
    rocm = None
    try:
        with open("/opt/rocm/.info/version") as fh:
            rocm = fh.read().strip()
    except OSError:
        pass
    clock = None
    try:   # peak engine clock of device 0: hipDeviceGetAttribute(hipDeviceAttributeClockRate = 5), kHz
        hip = ctypes.CDLL("libamdhip64.so")
        khz = ctypes.c_int(0)
        if hip.hipDeviceGetAttribute(ctypes.byref(khz), 5, 0) == 0:
            clock = khz.value // 1000
    except OSError:
        pass
    return {"gpu": p.name, "gcn_arch": getattr(p, "gcnArchName", ""), "cus": p.multi_processor_count,
            "gpu_clock_mhz": clock, "rocm": rocm, "hip": torch.version.hip, "torch": torch.__version__,
            "cpu": cpu, "cpu_count": os.cpu_count()}


def copy_calibration(nbytes=1 << 30, reps=20):
    """Device-to-device copy bandwidth of torch's copy kernel on nbytes
    (read + write counted), the practical ceiling of a streaming kernel; also
    the reference whose rocprofv3 FETCH_SIZE / WRITE_SIZE scale the counters."""
    import torch
    # random values: lines of zeros (and likely other uniform patterns) move
    # faster through the memory system than real data
    g = torch.Generator(device="cuda:0").manual_seed(5)
    src = torch.rand(nbytes // 4, dtype=torch.float32, device="cuda:0", generator=g)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) / 1e3 / reps
    del src, dst
    return {"bytes_per_copy": nbytes, "gbs": round(2 * nbytes / sec / 1e9, 1), "us": round(sec * 1e6, 2)}


def cpu_baseline(w, tau, sample_steps, smagorinsky=0.0):
    """The FP64 oracle on the same workload, all host threads, a short run;
    also one thread on a shorter run.  Returns the JSON entry and the oracle's
    last sensor result of the timed run, (step, block maxima, flags), or None
    when that run has no sensor step."""
    import oracle
    G = oracle.Grid(q=w.q, n=w.n, bc=w.bc, wall_u=w.wall_u, tau=tau, force=w.force,
                    theta_refine=w.theta_refine, theta_coarsen=w.theta_coarsen, smagorinsky=smagorinsky)
    S = G.equilibrium_state()
    S, _ = G.run(S, 0, 1, 1)                   # first touch of the work arrays
    threads = oracle.threads()
    t0 = time.perf_counter()
    S, hist = G.run(S, 1, sample_steps, w.sensor_every)
    dt = time.perf_counter() - t0
    one_steps = max(1, sample_steps // 20)
    prev = oracle.set_threads(1)
    t1 = time.perf_counter()
    S, _ = G.run(S, 1 + sample_steps, one_steps, w.sensor_every)
    dt1 = time.perf_counter() - t1
    oracle.set_threads(prev)
    entry = {"value": round(w.cells * sample_steps / dt / 1e6, 3), "unit": "MLUPS", "cores": threads,
             "kind": "oracle",
             "sample": f"{sample_steps} steps of the same {w.n[0]}x{w.n[1]}x{w.n[2]} workload in FP64, "
                       f"sensor every step, {dt:.1f} s",
             "one_core": {"value": round(w.cells * one_steps / dt1 / 1e6, 3), "unit": "MLUPS",
                          "sample": f"{one_steps} steps, {dt1:.1f} s"}}
    return entry, (hist[-1] if hist else None)


def flag_agreement(lbm, torch, desc, every, ref, theta, eps=2e-4):
    """The GPU path from rest to the oracle's sensor step `ref[0]` on the same
    workload: its refine/keep/coarsen flags against the FP64 oracle's, block
    by block.  Blocks whose oracle maximum lies within `eps` (relative) of a
    threshold may round either way in float32 and are counted apart."""
    k, bm_ref, fl_ref = ref
    blk = lbm.Blocks(desc, device="cuda:0")
    blk.step_n(k, every)
    bm, fl, kk, _ = blk.sensor_flags()
    blk.close()
    assert kk == k
    near = np.zeros(bm_ref.shape, dtype=bool)
    for t in theta:
        near |= np.abs(bm_ref - t) <= eps * t
    differ = fl != fl_ref
    return {"step": int(k), "blocks": int(fl.size), "equal": int((~differ).sum()),
            "frac": round(float((~differ).mean()), 6), "differ_near_threshold": int((differ & near).sum()),
            "differ_elsewhere": int((differ & ~near).sum()),
            "max_block_rel_err": float((np.abs(bm - bm_ref) / np.maximum(bm_ref, theta[0])).max()),
            "oracle": "FP64, same initial state and steps"}


def cache_proof_leg(lbm, torch, steps, warmup, every=1):
    """The same step + sensor on the 256^3 cavity, float32, ping-pong: its two
    1.19 GiB buffers cannot stay in the 256 MB Infinity Cache, so every step
    streams the state from and to HBM.  Timed like the main leg (HIP events
    around `steps` back-to-back steps on the library's stream); one kernel
    runs per step, so the mean step period is its duration."""
    import lbm_inputs
    w = lbm_inputs.cavity3d(n=256, storage="f32")
    st, tau = lbm.lbm_tau_from_reynolds(w.lid_speed, w.n_across, w.reynolds)
    desc = lbm.make_desc(19, w.n, w.bc, tau, storage=lbm.LBM_F32, wall_u=w.wall_u,
                         theta_refine=w.theta_refine, theta_coarsen=w.theta_coarsen)
    blk = lbm.Blocks(desc, device="cuda:0")
    stream = blk.stream
    blk.step_n(warmup, every)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    blk.step_n(steps, every)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    bm, fl, k, nonfinite = blk.sensor_flags()
    sch = blk.scheme()
    blk.close()
    step_s = ms / 1e3 / steps
    algo = 2 * 19 * 4 * w.cells
    achieved = algo / step_s / 1e9
    tag = "cavity256_f32_pingpong"
    return {"workload": w.name, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": _traffic_from_profile(tag), "kernel": "pingpong",
            "algorithmic_bytes_per_launch": algo, "per_kernel_us": {"pingpong": round(step_s * 1e6, 2)},
            "mlups": round(w.cells / step_s / 1e6, 1), "steps": steps, "warmup": warmup,
            "sensor_every": every, "scheme": sch, "last_sensor_step": k, "nonfinite": bool(nonfinite),
            "working_set_bytes": algo}


def run_refined(args, lbm, torch):
    """The two-level hierarchy over the 256^3 cavity; returns the JSON dict."""
    import lbm_inputs
    storage = {"f32": lbm.LBM_F32, "f32s": lbm.LBM_F32_SHIFTED, "f64": lbm.LBM_F64,
               "f16s": lbm.LBM_F16_SHIFTED, "bf16s": lbm.LBM_BF16_SHIFTED,
               "f16sr": lbm.LBM_F16_SHIFTED_SR, "bf16sr": lbm.LBM_BF16_SHIFTED_SR}[args.storage]
    sr = storage in (lbm.LBM_F16_SHIFTED_SR, lbm.LBM_BF16_SHIFTED_SR)
    w = lbm_inputs.cavity3d(n=256, storage=args.storage)
    st, tau = lbm.lbm_tau_from_reynolds(w.lid_speed, w.n_across, w.reynolds)
    desc = lbm.make_desc(19, w.n, w.bc, tau, storage=storage, wall_u=w.wall_u,
                         streaming=lbm.LBM_STREAMING_PINGPONG)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    blk = lbm.Blocks(desc, device="cuda:0", stream=stream)
    blk.step_n(1000, 1000)
    bm, fl, _, _ = blk.sensor_flags()
    boxes = lbm_inputs.place_patches(fl == 1, 8, w.n, count=400, seed=7)
    # stochastic rounding keys on the step index: launched step by step
    H = lbm.Hierarchy(blk, boxes, use_graph=not sr)
    tx, wg, fine_us = H.autotune(5)
    H.step_n(args.warmup, 0)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    H.step_n(args.steps, 0)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    # per-kernel durations in production order and data (4 coarse steps
    # launched one by one, HIP events between the launches)
    prof = H.profile(4)
    fine_us_tuned = fine_us
    fine_us = prof["fine"]        # the first fine step (the second also restricts)
    H.step_n(2, 2)
    fbm, ffl, _ = H.sensor()
    rho, u = blk.macros()
    info = H.info()
    coarse_cells, fine_cells = w.cells, info["fine_cells"]
    updates = (coarse_cells + 2 * fine_cells) * args.steps
    elem = 8 if storage == lbm.LBM_F64 else (2 if storage >= lbm.LBM_F16_SHIFTED else 4)
    fine_bytes = 2 * 19 * elem * fine_cells
    achieved = fine_bytes / (fine_us * 1e-6) / 1e9
    uniform_fine_updates = 2 * 8 * coarse_cells            # a uniform 512^3 grid, 2 steps per coarse step
    result = {
        "metric": "MLUPS (both levels) of the two-level patch hierarchy over the 256^3 cavity",
        "value": round(updates / (ms * 1e-3) / 1e6, 1),
        "unit": "MLUPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.storage, "data": "synthetic",
        "config": {"workload": "refined cavity3d_d3q19_256^3 + fine patches", "patches": len(boxes),
                   "patch_edges_fine": sorted({2 * (hi[0] - lo[0]) for lo, hi in boxes}),
                   "fine_cells": fine_cells, "coarse_cells": coarse_cells, "n_eff": info["n_eff"],
                   "uniform_fine_equivalent_cells": 8 * coarse_cells, "tau_coarse": tau,
                   "tau_fine": info["tau_fine"], "fine_tile_max": [tx, 8, 8], "fine_workgroups": wg,
                   "work_vs_uniform_fine": round((coarse_cells + 2 * fine_cells) / uniform_fine_updates, 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": ("patch_band_step" if tx == 48 else f"patch_step (W = {tx})")
                               + " (the fine step over all patches, one persistent launch)",
                     "algorithmic_bytes_per_launch": fine_bytes,
                     "per_kernel_us": {"patch_step": round(prof["fine"], 2), "patch_ghosts": round(prof["ghosts"], 2),
                                       "patch_step_with_restriction": round(prof["fine_restrict"], 2),
                                       "coarse_step": round(prof["coarse"], 2)},
                     "patch_step_us_autotune": round(fine_us_tuned, 2)},
        "fine_refine_blocks": int((ffl == 1).sum()),
        "nonfinite": bool(not np.isfinite(rho).all()),
    }
    result["roofline"]["traffic"] = _traffic_from_profile(f"refined256_{args.storage}_patch_step", "patch_kernels.hpp")
    H.close()
    blk.close()
    if not args.no_copy_calibration:
        cal = copy_calibration()
        result["copy_calibration"] = cal
        result["roofline"]["frac_of_copy"] = round(achieved / cal["gbs"], 4)
    return result


def run_cavity2d(args, lbm, torch):
    """The 64^2 D2Q9 float64 cavity (Re 100, sensor every 100 steps):
    launch-bound.  Timed with up to 5 sensor-free steps per launch (the
    temporal-blocking kernel, the default for such grids) and with one launch
    per step, each launched from the host and replayed in runs of 98 steps
    from HIP graphs; returns the JSON dict."""
    import lbm_inputs
    w = lbm_inputs.cavity2d()
    st, tau = lbm.lbm_tau_from_reynolds(w.lid_speed, w.n_across, w.reynolds)
    torch.cuda.set_device(0)
    out = {}
    for multi, chunk in ((5, 0), (5, 98), (0, 0), (0, 98)):
        desc = lbm.make_desc(9, w.n, w.bc, tau, storage=lbm.LBM_F64, wall_u=w.wall_u)
        stream = torch.cuda.Stream()
        blk = lbm.Blocks(desc, device="cuda:0", stream=stream)
        blk.set_multistep(multi)
        blk.use_graphs(chunk)
        blk.step_n(args.warmup, w.sensor_every)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        blk.step_n(w.steps, w.sensor_every)
        b.record(stream)
        torch.cuda.synchronize()
        out[multi, chunk] = a.elapsed_time(b) / w.steps * 1e3
        blk.close()
    us = out[5, 98]
    return {
        "metric": "us per step of the 64^2 D2Q9 FP64 cavity (step + sensor every 100 steps)",
        "value": round(w.cells / (us * 1e-6) / 1e6, 1), "unit": "MLUPS",
        "n_gpus": 1, "steps": w.steps, "warmup": args.warmup, "ms_per_step": round(us / 1e3, 6),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "lattice": "D2Q9", "extent": list(w.n), "tau": tau,
                   "sensor_every": w.sensor_every},
        "us_per_step": {"multistep5_graph_chunk_98": round(out[5, 98], 3),
                        "multistep5_launched": round(out[5, 0], 3),
                        "one_step_per_launch_graph_chunk_98": round(out[0, 98], 3),
                        "one_step_per_launch_launched": round(out[0, 0], 3)},
        "roofline": {"bound": "launch", "achieved": None, "peak": None, "unit": None, "frac": None,
                     "traffic": None,
                     "kernel": "step_multi<9, double, ...> (5 steps of 4096 cells per launch: latency bound)"},
    }


def run_predictor(args, lbm, torch):
    """Training iterations of the flag predictor as configured (4 input
    channels: the block means of rho - rho0 and u; 4 convolutions 4 -> 16 ->
    16 -> 16 -> 1) on a seeded synthetic batch of 8 block grids of 16^3;
    returns the JSON dict."""
    import lbm_inputs
    from paper_1507_06767_amd import cnn
    from paper_1507_06767_amd.predictor import FlagPredictor
    torch.cuda.set_device(0)
    shape = (8, 16, 16, 16)
    nv = int(np.prod(shape))
    x = (2.0 * lbm_inputs.uniform(11, nv * 4) - 1.0).reshape(shape + (4,))
    t = (2.0 * lbm_inputs.uniform(12, nv) - 1.0).reshape(shape)
    net = FlagPredictor(channels=(4, 16, 16, 16, 1), residual=False, seed=0)
    # the batch stays on the device; one iteration (12 launches) is captured
    # into a HIP graph and replayed
    net.load_batch(x, t)
    for _ in range(args.warmup):
        net.train_step(shape, 1e-3)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(args.steps):
        net.train_step(shape, 1e-3)
    b.record()
    torch.cuda.synchronize()
    ms_eager = a.elapsed_time(b)
    graph = net.capture_train_step(shape, 1e-3)
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.record()
    for _ in range(args.steps):
        graph.replay()
    b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = a.elapsed_time(b)
    net.replayed(args.steps + 1)
    # one 16 -> 16 forward convolution: 50 launches captured into a graph and
    # replayed back to back (launching them one by one from the host would
    # time the host, not the kernel)
    L = net.layers[1]
    B = net._buffers(shape)
    reps = 50
    conv_graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(conv_graph):
        for _ in range(reps):
            assert cnn.lbm_cnn_conv3d_forward(B["acts"][0], *shape, L.ci, L.packed, L.co, L.b, 1, None,
                                              B["acts"][1]) == 0
    conv_graph.replay()
    torch.cuda.synchronize()
    a.record()
    conv_graph.replay()
    b.record()
    torch.cuda.synchronize()
    conv_us = a.elapsed_time(b) / reps * 1e3
    flops = 2.0 * nv * L.co * 27 * L.ci
    achieved = flops / (conv_us * 1e-6) / 1e12
    return {
        "metric": "training iterations per second of the flag predictor (4 conv3d layers, BF16 MFMA)",
        "value": round(args.steps / (ms * 1e-3), 1), "unit": "iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16 (fp32 accumulate)",
        "data": "synthetic", "wall_s": round(wall, 3),
        "eager_iterations_per_s": round(args.steps / (ms_eager * 1e-3), 1),
        "config": {"workload": "flag predictor 4-16-16-16-1, batch 8 x 16^3 blocks", "voxels": nv,
                   "launch": "HIP graph of one iteration, replayed"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": round(achieved / 2500.0, 6), "traffic": None,
                     "kernel": "conv3d_forward 16->16 (mean of 50 graph-replayed launches)",
                     "flops_per_launch": flops,
                     "per_kernel_us": {"conv3d_forward_16x16": round(conv_us, 2)}},
    }


def run_conv_sweep(args, lbm, torch):
    """Batch sweep of the predictor's 16 -> 16 convolution: forward and
    weight gradient on 8, 32, 128 and 512 block grids of 16^3 (random
    activations), each timed over 20 launches captured into a HIP graph;
    returns the JSON dict."""
    import lbm_inputs
    from paper_1507_06767_amd import cnn
    from paper_1507_06767_amd.predictor import FlagPredictor
    torch.cuda.set_device(0)
    rows = []
    for nb in (8, 32, 128, 512):
        shape = (nb, 16, 16, 16)
        nv = int(np.prod(shape))
        net = FlagPredictor(channels=(16, 16, 16, 16, 1), seed=0)
        B = net._buffers(shape)
        L = net.layers[1]
        x, y = B["acts"][0], B["acts"][1]
        x.copy_(torch.from_numpy((2.0 * lbm_inputs.uniform(13, x.numel()) - 1.0).astype(np.float32)))
        reps = 20
        timing = {}
        for name, call in (("forward", lambda: cnn.lbm_cnn_conv3d_forward(x, *shape, L.ci, L.packed, L.co, L.b, 1,
                                                                            None, y)),
                           ("wgrad", lambda: cnn.lbm_cnn_conv3d_wgrad(x, y, *shape, L.ci, L.co, B["work"], L.gw,
                                                                        L.gb))):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                for _ in range(reps):
                    assert call() == 0
            g.replay()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            g.replay()
            b.record()
            torch.cuda.synchronize()
            timing[name] = a.elapsed_time(b) / reps * 1e3
        flops = 2.0 * nv * 16 * 27 * 16
        rows.append({"batch": nb, "voxels": nv, "forward_us": round(timing["forward"], 2),
                     "forward_tflops": round(flops / timing["forward"] / 1e6, 1),
                     "wgrad_us": round(timing["wgrad"], 2),
                     "wgrad_tflops": round(flops / timing["wgrad"] / 1e6, 1)})
        del net, B
        torch.cuda.empty_cache()
    return {"metric": "16 -> 16 conv3d forward and weight-gradient time per batch (BF16 MFMA)",
            "unit": "us", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
            "config": {"workload": "predictor convolution batch sweep, block grids of 16^3"},
            "peak_tflops": 2500.0, "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="cavity128")
    ap.add_argument("--storage", default="f32", choices=["f32", "f32s", "f64", "f16s", "bf16s", "f16sr", "bf16sr"])
    ap.add_argument("--lattice", type=int, default=19, choices=[19, 27])
    ap.add_argument("--smagorinsky", type=float, default=0.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=100)
    ap.add_argument("--kernel-samples", type=int, default=200,
                    help="single launches timed one by one for the per-kernel durations")
    ap.add_argument("--no-copy-calibration", action="store_true",
                    help="skip timing a 1 GiB device copy (reported as copy_calibration)")
    ap.add_argument("--no-cache-proof", action="store_true",
                    help="skip the 256^3 leg of the default workload (roofline_cache_proof)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the domain would shard into z-slabs; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1507_06767_amd as lbm

    if args.workload in ("refined256", "predictor", "cavity64_2d", "conv_sweep"):
        run = {"refined256": run_refined, "predictor": run_predictor, "cavity64_2d": run_cavity2d,
               "conv_sweep": run_conv_sweep}[args.workload]
        print(json.dumps(run(args, lbm, torch)), flush=True)
        return

    storage = {"f32": lbm.LBM_F32, "f32s": lbm.LBM_F32_SHIFTED, "f64": lbm.LBM_F64,
               "f16s": lbm.LBM_F16_SHIFTED, "bf16s": lbm.LBM_BF16_SHIFTED,
               "f16sr": lbm.LBM_F16_SHIFTED_SR, "bf16sr": lbm.LBM_BF16_SHIFTED_SR}[args.storage]
    w = _workload(args.workload, args.storage)
    if args.lattice != w.q:
        import dataclasses
        w = dataclasses.replace(w, q=args.lattice, name=w.name.replace("d3q19", f"d3q{args.lattice}"))
    if w.reynolds is not None:
        st, tau = lbm.lbm_tau_from_reynolds(w.lid_speed, w.n_across, w.reynolds)
        assert st == 0
    else:
        tau = w.tau
    desc = lbm.make_desc(w.q, w.n, w.bc, tau, storage=storage, wall_u=w.wall_u, force=w.force,
                         theta_refine=w.theta_refine, theta_coarsen=w.theta_coarsen,
                         smagorinsky=args.smagorinsky)
    torch.cuda.set_device(0)
    blk = lbm.Blocks(desc, device="cuda:0")
    stream = blk.stream
    every = w.sensor_every

    blk.step_n(args.warmup, every)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    start.record(stream)
    blk.step_n(args.steps, every)
    end.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = start.elapsed_time(end)
    bm, fl, k, nonfinite = blk.sensor_flags()

    # Per-kernel durations: single launches bracketed by events on the same
    # stream.  The in-place scheme alternates a gather-scatter and a local
    # launch; both move the same algorithmic bytes.
    per = {"gather_scatter": [], "local": [], "pingpong": []}
    evs = []
    for _ in range(args.kernel_samples):
        sch = blk.scheme()
        kind = ("gather_scatter" if sch["next_is_gather"] else "local") if sch["inplace"] else "pingpong"
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        blk.step_n(1, every)
        b.record(stream)
        evs.append((kind, a, b))
    torch.cuda.synchronize()
    for kind, a, b in evs:
        per[kind].append(a.elapsed_time(b) / 1e3)
    per_raw = {kind: sum(v) / len(v) for kind, v in per.items() if v}
    # A single launch between two events also times the event packets
    # (about 2 us).  The timed region runs the kernels back to back, so its
    # mean step period is the level; the bracketed launches give only the
    # split between the two in-place kernels, which alternate one per step.
    step_s = ms / 1e3 / args.steps
    if len(per_raw) == 2:
        tot = sum(per_raw.values())
        per = {kind: 2 * step_s * t / tot for kind, t in per_raw.items()}
    else:
        per = {kind: step_s for kind in per_raw}
    dominant = max(per, key=per.get)

    elem = 8 if storage == lbm.LBM_F64 else (2 if storage >= lbm.LBM_F16_SHIFTED else 4)
    bytes_per_update = 2 * w.q * elem
    sec = ms / 1e3
    mlups = w.cells * args.steps / sec / 1e6
    per_launch_s = per[dominant]
    achieved = bytes_per_update * w.cells / per_launch_s / 1e9
    tag = f"{args.workload}_{args.storage}_{dominant}"
    traffic = _traffic_from_profile(tag)

    result = {
        "metric": "MLUPS and % HBM roofline for D3Q19 step+sensor; flag agreement vs FP64 oracle",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": f"D{2 if w.q == 9 else 3}Q{w.q}",
                   "extent": list(w.n), "tau": tau, "sensor": "L2 ratio, 8^3 block max + flags",
                   "sensor_every": every, "theta_refine": w.theta_refine,
                   "smagorinsky": args.smagorinsky},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": dominant,
                     "algorithmic_bytes_per_launch": bytes_per_update * w.cells,
                     "per_kernel_us": {kd: round(t * 1e6, 2) for kd, t in per.items()},
                     "per_kernel_us_single_launch": {kd: round(t * 1e6, 2) for kd, t in per_raw.items()},
                     "step_avg_achieved": round(bytes_per_update * w.cells / (sec / args.steps) / 1e9, 1),
                     "scheme": blk.scheme()},
        "last_sensor_step": k,
        "refine_blocks": int((fl == 1).sum()),
        "nonfinite": bool(nonfinite),
        "wall_s": round(t_wall, 3),
        "env": host_env(),
    }
    blk.close()
    # The in-place 128^3 float32 state (152 MiB) can stay in the 256 MB
    # Infinity Cache, so the figure above is not an HBM-only one; the 256^3
    # leg below is.
    state_bytes = (1 if result["roofline"]["scheme"]["inplace"] else 2) * w.q * elem * w.cells
    result["roofline"]["state_bytes"] = state_bytes
    result["roofline"]["cache_resident"] = state_bytes <= (256 << 20)
    if (args.workload == "cavity128" and args.storage == "f32" and w.q == 19 and args.smagorinsky == 0.0
            and not args.no_cache_proof):
        result["roofline_cache_proof"] = cache_proof_leg(lbm, torch, args.steps, args.warmup)
    if not args.no_copy_calibration:
        cal = copy_calibration()
        result["copy_calibration"] = cal
        result["roofline"]["frac_of_copy"] = round(achieved / cal["gbs"], 4)
        if "roofline_cache_proof" in result:
            cp = result["roofline_cache_proof"]
            cp["frac_of_copy"] = round(cp["achieved"] / cal["gbs"], 4)
    if not args.no_cpu_baseline:
        result["cpu_baseline"], ref = cpu_baseline(w, tau, args.cpu_sample_steps, args.smagorinsky)
        if ref is not None:
            result["flag_agreement"] = flag_agreement(lbm, torch, desc, every, ref,
                                                      (w.theta_refine, w.theta_coarsen))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
