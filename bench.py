#!/usr/bin/env python3
"""Throughput of the matrix-free SPGM projector on one MI355X.

A step is one SPGM iteration (Sec. IV, Eq. 5 with the minibatch gradient of Eq. 6): sort the
minibatch, forward-project it, form the residual, back-project, take the gradient step and
the complex soft threshold -- every kernel of the hot path, on one minibatch of synthetic
measurements resident in HBM.

Reported value: projector Gentries/s = B * N * steps / t / 1e9 (entries of A_B formed per
gradient evaluation A_B^H (A_B s - y_B)), plus SPGM iterations/s, the relative error of the
GPU iterate against the FP64 oracle after the first iterations of the same solve, the
roofline of the dominant kernel (timed live with HIP events on the library's stream), and
the oracle's own rate on the host cores.

Usage: python bench.py [--gpus 1] [--steps 100] [--warmup 10] [--workload c2]
       --workload c2     (default) the largest single-GPU configuration: 48 Tx + 48 Rx, 100
                         frequencies, 128x128x64 voxels, B = 16384
       --workload c1     mid-size: 32 Tx + 32 Rx, 64 frequencies, 64x64x32 voxels, B = 4096
       --workload c3     ragged batch of 96 scenes
       --workload c4grad forward + backward of a 10-iteration unrolled SPGM (learnable steps)
       --workload calib  measured issue rates of FMA, sin, cos and the entry body (roofline inputs)
       --workload c1k32  32 scenes of the c1 geometry through the shared-geometry batched path
       --workload c1s    c1 geometry with structured (16 f x 16 Tx x 16 Rx) minibatches
       --workload c1tv   c1 with the magnitude-TV prox (10 dual iterations per step) on a blocky scene
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2509_00774_amd import workloads as W  # noqa: E402

# VALU ceiling in FP32 FMA slots: the chip's 157.3 TFLOP/s FP32 vector peak is 78.64e12 lane-FMAs/s,
# 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz (measured on gfx950: plain v_fma_f32 issue at 25-32 lanes per
# SIMD and clock, `--workload calib`).  Transcendentals (v_sin_f32, v_cos_f32) issue at a quarter of
# that rate (measured 8 lanes per SIMD and clock), i.e. 4 slots each.  One entry of A applied to a
# vector needs at least 13 slots: the phase FMA (1), sin and cos (4 + 4) and the 4 FMAs of the complex
# multiply-add.
VALU_SLOTS_PER_S = 256 * 4 * 32 * 2.4e9
TRANS_SLOTS = 4
SLOTS_PER_ENTRY = 5 + 2 * TRANS_SLOTS
SLOT_UNIT = "T FP32 lane-slots/s (FMA = 1, sin/cos = 4)"
STEP_SIZES = os.path.join(ROOT, "tests", "golden", "step_sizes.json")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")
SOURCES = [os.path.join(ROOT, "paper_2509_00774_amd", "csrc", name)
           for name in ("spgm.hip", "spgm_mm.inc", "spgm_sf.inc", "spgm_reg.inc")] + [
    os.path.join(ROOT, "include", "spgm.h"), os.path.join(ROOT, "paper_2509_00774_amd", "build.py")]
# Total-variation prox: algorithmic bytes per voxel and dual iteration (read b, r, w; write w, r
# as three float32 components each).
TV_BYTES_PER_VOXEL = 4 + 4 * 12
HBM_PEAK = 8.0e12


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def source_sha():
    """Fingerprint of every source of libspgm.so and of its build flags (counter records are void
    once any changes)."""
    h = hashlib.sha256()
    for path in SOURCES:
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def mm_shape_key(shape):
    """Key of a batched launch shape (spgm_plan_batched_shape's first six values)."""
    return "shape" + "x".join(str(int(v)) for v in shape[:6])


def stored_traffic(kernel, workload, shape=None):
    """HBM bytes per launch from the committed counter runs (per launch shape: row splits and
    waves per work-group for the tile kernels, a mm_shape_key string for the batched kernels),
    if the kernel source is unchanged."""
    if not os.path.exists(TRAFFIC):
        return None
    data = json.load(open(TRAFFIC))
    if shape is None:
        suffix = ""
    elif isinstance(shape, str):
        suffix = "/" + shape
    else:
        suffix = "/splits%d/waves%d" % tuple(shape)
    key = "%s/%s" % (kernel, workload) + suffix
    rec = data.get(key)
    if not rec or rec.get("source_sha") != source_sha():
        return None
    return rec.get("bytes_per_launch")


def timed_solve(args, torch, plan, timed_rows, y, s, eta, alpha):
    """Time len(timed_rows) SPGM iterations from s = 0 (graph replay unless --eager); returns the
    wall time and the HIP-event totals of the two tile kernels."""
    if not args.eager:
        # The timed region replays the captured graph; the capture (and one replay) happens
        # before it.  Kernel durations for the roofline come from an eager pass of the same
        # launches right after, timed with HIP events on the library's stream.
        plan.spgm_solve_graph(timed_rows, y, s, eta, alpha)
        s.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.spgm_solve_graph(timed_rows, y, s, eta, alpha)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.zero_()
        plan.spgm_plan_timing(True)
        plan.spgm_plan_timing_read()
        plan.spgm_solve(timed_rows, y, s, eta, alpha)
        fwd_ms, fwd_n, adj_ms, adj_n = plan.spgm_plan_timing_read()
        plan.spgm_plan_timing(False)
    else:
        plan.spgm_plan_timing(True)
        plan.spgm_plan_timing_read()  # reset counters
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.spgm_solve(timed_rows, y, s, eta, alpha)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        fwd_ms, fwd_n, adj_ms, adj_n = plan.spgm_plan_timing_read()
        plan.spgm_plan_timing(False)
    return t1 - t0, fwd_ms, fwd_n, adj_ms, adj_n


def entry_ceiling(binding):
    """Measured entry-body rate of the chip (the algorithmic minimum instruction sequence per entry,
    latency hidden), best of three probe launches; entries/s."""
    return max(binding.calibrate(3, 4096)[0] for _ in range(3))


def alu_roofline(entries, fwd_ms, fwd_n, adj_ms, adj_n, shapes, wl, phase, ceiling=None):
    """Roofline record of the slower tile kernel: VALU issue slots per launch (entries x the
    9-slot minimum per entry) over its average HIP-event duration, against the issue ceiling.
    shapes: ((forward splits, waves), (adjoint splits, waves)) of the timed launches."""
    fwd_avg = fwd_ms / max(fwd_n, 1) * 1e-3
    adj_avg = adj_ms / max(adj_n, 1) * 1e-3
    kname, kavg = ("k_fwd_tile", fwd_avg) if fwd_avg >= adj_avg else ("k_adj_tile", adj_avg)
    achieved = entries * SLOTS_PER_ENTRY / kavg / 1e12
    peak = VALU_SLOTS_PER_S / 1e12
    kshape = shapes[0 if kname == "k_fwd_tile" else 1]
    traffic = stored_traffic(kname, wl, kshape) if phase == "comp32" else None
    return {"bound": "alu", "kernel": kname, "achieved": round(achieved, 3), "peak": round(peak, 3),
            "unit": SLOT_UNIT, "frac": round(achieved / peak, 4), "traffic": traffic,
            "entries_per_launch": int(entries), "slots_per_entry": SLOTS_PER_ENTRY,
            "avg_launch_ms": round(kavg * 1e3, 5),
            "fwd_tile_ms": round(fwd_avg * 1e3, 5), "adj_tile_ms": round(adj_avg * 1e3, 5),
            "fwd_gentries_per_s": round(entries / fwd_avg / 1e9, 1),
            "adj_gentries_per_s": round(entries / adj_avg / 1e9, 1),
            "measured_entry_ceiling_gentries_per_s": None if ceiling is None else round(ceiling / 1e9, 1),
            "frac_of_measured_ceiling": None if ceiling is None else round(entries / kavg / ceiling, 4)}


PHASE_DESC = {"comp32": "compensated fp32 (fp64 per-tile reference)", "f64": "fp64 distance and phase",
              "naive32": "naive fp32"}


def phase_mode_of(binding, name):
    return {"comp32": binding.PHASE_COMP32, "f64": binding.PHASE_F64, "naive32": binding.PHASE_NAIVE32}[name]


def bench_large(args, torch, binding, dev):
    """The largest single-GPU configuration (48 Tx + 48 Rx, 100 frequencies, 128x128x64 voxels,
    B = 16384): graph-replayed SPGM steps on the patches scene.  The oracle checks, at full size,
    a forward of a dense random vector on a seeded 5 % of the minibatch rows and the first SPGM
    step from s = 0 on a seeded 5 % of the voxels (that step needs only A_B^H y_B), and its time
    on those samples is the CPU baseline."""
    wl = "c2"
    cfg = W.CONFIGS[wl]
    geom = W.config_geometry(wl)
    M, N = W.dims(geom)
    B = cfg["B"]
    K, Wm = args.steps, args.warmup
    sj = json.load(open(STEP_SIZES))[wl]
    eta = float(np.float32(sj["eta"]))
    alpha = float(np.float32(sj["lambda"] * eta))
    log("workload %s: T=%d R=%d F=%d M=%d N=%d B=%d; drawing %d minibatches" % (
        wl, cfg["T"], cfg["R"], cfg["F"], M, N, B, 1 + Wm + K))
    rows = W.config_rows(wl, K=1 + Wm + K)
    s_true, idx = W.config_scene(wl)
    plan = binding.Plan(geom, phase_mode=phase_mode_of(binding, args.phase))
    splits = None if args.no_tune else plan.spgm_plan_autotune(B)
    if splits:
        log("autotuned row splits: forward %d, adjoint %d" % splits)
    # Measurements: forward projection of the seeded scene in minibatch-sized row chunks, plus
    # seeded noise at the workload's SNR.
    s_true_d = torch.from_numpy(s_true.astype(np.complex64)).to(dev)
    y0 = torch.empty(M, dtype=torch.complex64, device=dev)
    for c0 in range(0, M, B):
        c1 = min(M, c0 + B)
        plan.spgm_forward(torch.arange(c0, c1, dtype=torch.int32, device=dev), s_true_d, out=y0[c0:c1])
    y0_host = y0.cpu().numpy().astype(np.complex128)
    y = torch.from_numpy(W.add_noise(y0_host, cfg["snr_db"], seed=cfg["seed"] + 2).astype(np.complex64)).to(dev)
    rows_d = torch.from_numpy(rows).to(dev)
    del s_true_d
    # Parity samples, before the timed solve: a forward of a dense random vector on minibatch 0,
    # and the first step from zero on minibatch 0.
    rows0 = rows[0]
    s_rand = W.random_complex(N, seed=cfg["seed"] + 20).astype(np.complex64)
    y_rand = plan.spgm_forward(rows_d[0].contiguous(), torch.from_numpy(s_rand).to(dev)).cpu().numpy()
    s1 = torch.zeros(N, dtype=torch.complex64, device=dev)
    plan.spgm_solve(rows_d[:1].contiguous(), y, s1, eta, alpha)
    s1_host = s1.cpu().numpy()
    del s1
    s = torch.zeros(N, dtype=torch.complex64, device=dev)
    log("warmup %d steps" % Wm)
    if Wm > 0:
        plan.spgm_solve(rows_d[1:1 + Wm].contiguous(), y, s, eta, alpha)
    s.zero_()
    timed_rows = rows_d[1 + Wm:1 + Wm + K].contiguous()
    dt, fwd_ms, fwd_n, adj_ms, adj_n = timed_solve(args, torch, plan, timed_rows, y, s, eta, alpha)
    assert plan.spgm_plan_status() == 0
    s_fin = s.cpu().numpy().astype(np.complex128)
    nmse_truth_db = float(10.0 * np.log10(np.sum(np.abs(s_fin - s_true) ** 2) / np.sum(np.abs(s_true) ** 2)))
    log("timed %d steps in %.4f s (%.4f ms/step); forward tile %.4f ms avg over %d, adjoint tile %.4f ms avg over %d" % (
        K, dt, 1e3 * dt / K, fwd_ms / max(fwd_n, 1), fwd_n, adj_ms / max(adj_n, 1), adj_n))
    entries = float(B) * N
    shapes = plan.spgm_plan_launch_shape(B)
    roofline = alu_roofline(entries, fwd_ms, fwd_n, adj_ms, adj_n, shapes, wl, args.phase, entry_ceiling(binding))

    cpu = None
    par = {}
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.Oracle(geom)
        js = W.voxel_sample(B, 0.05, seed=cfg["seed"] + 21)
        vs = W.voxel_sample(N, 0.05, seed=cfg["seed"] + 22)
        ms = W.voxel_sample(M, 0.01, seed=cfg["seed"] + 23)
        log("oracle: measurements (all %d rows of the %d-voxel scene)" % (M, idx.size))
        y0_orc = orc.forward_sparse(np.arange(M), idx, s_true[idx])
        y_orc = W.add_noise(y0_orc, cfg["snr_db"], seed=cfg["seed"] + 2)
        par["rel_l2_scene_forward_1pct_rows"] = oracle.rel_l2(y0_host[ms], y0_orc[ms])
        log("oracle: forward on %d rows x %d voxels, first step on %d voxels x %d rows, %d threads" % (
            js.size, N, vs.size, B, oracle.num_threads()))
        c0 = time.perf_counter()
        y_ref = orc.forward(rows0[js], s_rand.astype(np.complex128))
        c1 = time.perf_counter()
        g_ref = orc.adjoint_voxels(rows0, y_orc[rows0], vs)
        c2 = time.perf_counter()
        s1_ref = oracle.prox_l1((eta / B) * g_ref, alpha)
        par["rel_l2_forward_5pct_rows"] = oracle.rel_l2(y_rand[js], y_ref)
        par["rel_l2_first_step_5pct_voxels"] = oracle.rel_l2(s1_host[vs], s1_ref)
        par["first_step_nonzeros_in_sample"] = int(np.count_nonzero(s1_ref))
        n_ent = float(js.size) * N + float(B) * vs.size
        cpu = {"value": round(n_ent / (c2 - c0) / 1e9, 4), "unit": "Gentries/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "one step's entries on a seeded 5%% sample: forward of %d of the %d minibatch rows over all "
                         "%d voxels (%.1f s) and the adjoint of the minibatch on %d voxels (%.1f s), FP64" % (
                             js.size, B, N, c1 - c0, vs.size, c2 - c1)}
        log("oracle parity: %s" % json.dumps(par))
    out = {
        "metric": "projector Gentries/s (A_B s + A_B^H r) and SPGM iters/s at fixed NMSE vs oracle",
        "value": round(entries * K / dt / 1e9, 2),
        "unit": "Gentries/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": round(1e3 * dt / K, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c2: %d Tx + %d Rx, %d frequencies, %dx%dx%d voxels, B=%d rows per minibatch, "
                               "points plus three planar patches" % (cfg["T"], cfg["R"], cfg["F"], *cfg["grid"], B),
                   "M": M, "N": N, "B": B, "hip_graph": not args.eager,
                   "launch_shape": {"forward": {"splits": shapes[0][0], "waves": shapes[0][1]},
                                    "adjoint": {"splits": shapes[1][0], "waves": shapes[1][1]},
                                    "autotuned": splits is not None},
                   "phase": PHASE_DESC[args.phase]},
        "spgm_iters_per_s": round(K / dt, 2),
        "rel_l2_vs_oracle": None if not par else float("%.3e" % max(
            par["rel_l2_forward_5pct_rows"], par["rel_l2_first_step_5pct_voxels"])),
        "parity_samples": {k: (float("%.3e" % v) if isinstance(v, float) else v) for k, v in par.items()},
        "nmse_db_vs_truth_after_steps": round(nmse_truth_db, 2),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    plan.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2",
                    choices=["c2", "c0", "c1", "c4", "c3", "c1k32", "c1s", "c1tv", "c4grad", "calib"],
                    help="c2 (default) is the largest single-GPU configuration; c3 is the ragged batch of 96 "
                         "scenes advanced together")
    ap.add_argument("--cpu-iters", type=int, default=5, help="iterations of the oracle timed on the host")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the row-split autotuner")
    ap.add_argument("--eager", action="store_true",
                    help="time the solve as individual launches instead of a captured HIP graph")
    ap.add_argument("--phase", default="comp32", choices=["comp32", "f64", "naive32"],
                    help="phase precision variant of the projector")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first launch one plain copy-like kernel (torch.neg) that reads and writes this many "
                         "bytes, as a known-size reference for the HBM byte counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the projector runs on a single MI355X; "
              "runs over several GPUs are not supported.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2509_00774_amd import binding

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.copy_bytes > 0:
        a = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        log("copy reference: %d bytes read, %d bytes written" % (a.numel() * 4, b.numel() * 4))
        del a, b
    wl = args.workload
    if wl == "c2":
        return bench_large(args, torch, binding, dev)
    if wl == "c3":
        return bench_ragged(args, torch, binding, dev)
    if wl == "c4grad":
        return bench_unrolled(args, torch, binding, dev)
    if wl == "calib":
        return bench_calibrate(args, binding)
    if wl == "c1k32":
        return bench_batched(args, torch, binding, dev)
    if wl == "c1s":
        return bench_structured(args, torch, binding, dev)
    if wl == "c1tv":
        return bench_tv(args, torch, binding, dev)
    cfg = W.CONFIGS[wl]
    geom = W.config_geometry(wl)
    M, N = W.dims(geom)
    B = cfg["B"]
    K, Wm = args.steps, args.warmup
    steps_json = json.load(open(STEP_SIZES))[wl]
    eta = float(np.float32(steps_json["eta"]))
    alpha = float(np.float32(steps_json["lambda"] * eta))

    log("workload %s: T=%d R=%d F=%d M=%d N=%d B=%d; drawing %d minibatches" % (
        wl, cfg["T"], cfg["R"], cfg["F"], M, N, B, Wm + K))
    rows = W.config_rows(wl, K=max(Wm + K, args.cpu_iters))
    s_true, idx = W.config_scene(wl)

    plan = binding.Plan(geom, phase_mode=phase_mode_of(binding, args.phase))
    splits = None if args.no_tune else plan.spgm_plan_autotune(B)
    if splits:
        log("autotuned row splits: forward %d, adjoint %d" % splits)
    # Synthetic measurements: forward projection of the seeded scene by the library itself,
    # plus seeded noise at the workload's SNR.
    all_rows = torch.arange(M, dtype=torch.int32, device=dev)
    y0 = plan.spgm_forward(all_rows, torch.from_numpy(s_true.astype(np.complex64)).to(dev))
    y_host = W.add_noise(y0.cpu().numpy().astype(np.complex128), cfg["snr_db"], seed=cfg["seed"] + 2)
    y = torch.from_numpy(y_host.astype(np.complex64)).to(dev)
    rows_d = torch.from_numpy(rows).to(dev)
    s = torch.zeros(N, dtype=torch.complex64, device=dev)
    torch.cuda.synchronize()

    # Parity sample: the first iterations of the solve from zero, kept for the oracle check.
    n_par = args.cpu_iters
    s_par = torch.zeros(N, dtype=torch.complex64, device=dev)
    plan.spgm_solve(rows_d[:n_par].contiguous(), y, s_par, eta, alpha)
    s_par_host = s_par.cpu().numpy()

    log("warmup %d steps" % Wm)
    if Wm > 0:
        plan.spgm_solve(rows_d[:Wm].contiguous(), y, s, eta, alpha)
    timed_rows = rows_d[Wm:Wm + K].contiguous()
    dt, fwd_ms, fwd_n, adj_ms, adj_n = timed_solve(args, torch, plan, timed_rows, y, s, eta, alpha)
    assert plan.spgm_plan_status() == 0
    # reconstruction quality of the K-step solve from zero (both branches leave it in s)
    s_fin = s.cpu().numpy().astype(np.complex128)
    nmse_truth_db = float(10.0 * np.log10(np.sum(np.abs(s_fin - s_true) ** 2) / np.sum(np.abs(s_true) ** 2)))
    log("timed %d steps in %.4f s (%.4f ms/step); forward tile %.4f ms avg over %d, adjoint tile %.4f ms avg over %d" % (
        K, dt, 1e3 * dt / K, fwd_ms / max(fwd_n, 1), fwd_n, adj_ms / max(adj_n, 1), adj_n))

    entries = float(B) * N
    value = entries * K / dt / 1e9
    shapes = plan.spgm_plan_launch_shape(B)
    roofline = alu_roofline(entries, fwd_ms, fwd_n, adj_ms, adj_n, shapes, wl, args.phase, entry_ceiling(binding))

    cpu = None
    rel_vs_oracle = None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.Oracle(geom)
        log("oracle: measurements for the parity sample")
        y0_orc = orc.forward_sparse(np.arange(M), idx, s_true[idx])
        y_orc = W.add_noise(y0_orc, cfg["snr_db"], seed=cfg["seed"] + 2)
        log("oracle: timing %d SPGM iterations on %d threads" % (n_par, oracle.num_threads()))
        c0 = time.perf_counter()
        s_orc = orc.solve(rows[:n_par], y_orc, np.zeros(N), eta, alpha)
        c1 = time.perf_counter()
        cpu = {"value": round(entries * n_par / (c1 - c0) / 1e9, 4), "unit": "Gentries/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "%d SPGM iterations of the same workload (B=%d rows x N=%d voxels each), FP64, %.1f s" % (
                   n_par, B, N, c1 - c0)}
        rel_vs_oracle = oracle.rel_l2(s_par_host, s_orc)
        log("oracle: %.1f s, GPU iterate %d rel_l2 vs oracle %.3e" % (c1 - c0, n_par, rel_vs_oracle))

    out = {
        "metric": "projector Gentries/s (A_B s + A_B^H r) and SPGM iters/s at fixed NMSE vs oracle",
        "value": round(value, 2),
        "unit": "Gentries/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": round(1e3 * dt / K, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %d Tx + %d Rx, %d frequencies, %dx%dx%d voxels, B=%d rows per minibatch" % (
            wl, cfg["T"], cfg["R"], cfg["F"], *cfg["grid"], B),
            "M": M, "N": N, "B": B, "hip_graph": not args.eager,
            "launch_shape": {"forward": {"splits": shapes[0][0], "waves": shapes[0][1]},
                             "adjoint": {"splits": shapes[1][0], "waves": shapes[1][1]},
                             "autotuned": splits is not None},
            "phase": PHASE_DESC[args.phase]},
        "spgm_iters_per_s": round(K / dt, 2),
        "rel_l2_vs_oracle": None if rel_vs_oracle is None else float("%.3e" % rel_vs_oracle),
        "rel_l2_vs_oracle_after_iters": n_par,
        "nmse_db_vs_truth_after_steps": round(nmse_truth_db, 2),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    plan.close()


def bench_unrolled(args, torch, binding, dev):
    """Differentiable unrolled SPGM (16 Tx + 16 Rx, 32 frequencies, 32x32x16 voxels, B = 2048,
    K = 10 iterations with learnable per-iteration step sizes and thresholds): forward plus
    backward of the unroll (MSE loss to the true scene), against 10 plain iterations of the
    float32 solve.  Entries formed per forward + backward: 2 K B N in the forward, 4 K B N in
    the backward (segment recompute with the kept gradient, then A^H A zbar)."""
    from paper_2509_00774_amd.autograd import unrolled_spgm
    cfg = W.CONFIGS["c4"]
    geom = W.config_geometry("c4")
    M, N = W.dims(geom)
    B, K = cfg["B"], cfg["K"]
    reps, Wm = args.steps, args.warmup
    sj = json.load(open(STEP_SIZES))["c4"]
    eta = (sj["eta"] * (1.0 + 0.05 * np.arange(K))).astype(np.float32).astype(np.float64)
    tau = (sj["lambda"] * eta).astype(np.float32).astype(np.float64)
    s_true, idx = W.config_scene("c4")
    rows = W.config_rows("c4", K=K)
    plan = binding.Plan(geom)
    splits = None if args.no_tune else plan.spgm_plan_autotune(B)
    y0 = plan.spgm_forward(torch.arange(M, dtype=torch.int32, device=dev),
                           torch.from_numpy(s_true.astype(np.complex64)).to(dev))
    y = torch.from_numpy(W.add_noise(y0.cpu().numpy().astype(np.complex128), cfg["snr_db"],
                                     seed=cfg["seed"] + 2).astype(np.complex64)).to(dev)
    rows_d = torch.from_numpy(rows).to(dev)
    st = torch.from_numpy(s_true.astype(np.complex64)).to(dev)

    def fwd_bwd():
        s0 = torch.zeros(N, dtype=torch.complex64, device=dev, requires_grad=True)
        e = torch.tensor(eta, dtype=torch.float64, device=dev, requires_grad=True)
        t = torch.tensor(tau, dtype=torch.float64, device=dev, requires_grad=True)
        out = unrolled_spgm(plan, rows_d, y, s0, e, t)
        loss = torch.mean(torch.abs(out - st) ** 2)
        loss.backward()
        return out, s0.grad, e.grad, t.grad

    for _ in range(Wm):
        fwd_bwd()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res = fwd_bwd()
    torch.cuda.synchronize()
    t_fb = (time.perf_counter() - t0) / reps
    s = torch.zeros(N, dtype=torch.complex64, device=dev)
    plan.spgm_solve(rows_d, y, s, float(eta[0]), float(tau[0]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.spgm_solve(rows_d, y, s, float(eta[0]), float(tau[0]))
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / reps
    entries = 6.0 * K * B * N
    log("unrolled forward + backward: %.3f ms; 10 plain iterations: %.3f ms" % (1e3 * t_fb, 1e3 * t_plain))
    out, gs0, geta, gtau = (r.detach() for r in res)
    cpu = None
    par = {}
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.Oracle(geom)
        y_h = y.cpu().numpy().astype(np.complex128)
        log("oracle: unrolled forward and chain rule in FP64 on %d threads" % oracle.num_threads())
        c0 = time.perf_counter()
        it = oracle.unrolled_forward(orc, rows, y_h, np.zeros(N), eta, tau)
        sbar = 2.0 * (it[-1] - s_true.astype(np.complex64).astype(np.complex128)) / N
        s0bar, eta_bar, tau_bar = oracle.unrolled_vjp(orc, rows, y_h, it, eta, tau, sbar)
        c1 = time.perf_counter()
        par = {"s_K": oracle.rel_l2(out.cpu().numpy(), it[-1]), "d_s0": oracle.rel_l2(gs0.cpu().numpy(), s0bar),
               "d_eta": oracle.rel_l2(geta.cpu().numpy(), eta_bar), "d_tau": oracle.rel_l2(gtau.cpu().numpy(), tau_bar)}
        cpu = {"value": round(entries / (c1 - c0) / 1e9, 4), "unit": "Gentries/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "one forward + backward of the same 10-iteration unroll (FP64 iterates and chain rule), "
                         "%.1f s" % (c1 - c0)}
        log("oracle: %.1f s; parity %s" % (c1 - c0, json.dumps(par)))
    achieved = entries * SLOTS_PER_ENTRY / t_fb / 1e12
    peak = VALU_SLOTS_PER_S / 1e12
    out_line = {
        "metric": "unrolled SPGM forward + backward Gentries/s (6 K B N entries per pass) against K plain iterations",
        "value": round(entries / t_fb / 1e9, 2), "unit": "Gentries/s", "n_gpus": 1, "steps": reps, "warmup": Wm,
        "ms_per_step": round(1e3 * t_fb, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c4grad: 16 Tx + 16 Rx, 32 frequencies, 32x32x16 voxels, B=2048, 10 unrolled iterations "
                               "with learnable eta_k, tau_k, MSE loss, sqrt(K) checkpoints",
                   "M": M, "N": N, "B": B, "K": K,
                   "row_splits": None if splits is None else {"forward": splits[0], "adjoint": splits[1]}},
        "ms_plain_k_iterations": round(1e3 * t_plain, 4),
        "fwd_bwd_over_plain": round(t_fb / t_plain, 3),
        "rel_l2_vs_oracle": None if not par else float("%.3e" % max(par.values())),
        "parity": {k: float("%.3e" % v) for k, v in par.items()},
        "roofline": {"bound": "alu", "kernel": "whole forward + backward", "achieved": round(achieved, 3),
                     "peak": round(peak, 3), "unit": SLOT_UNIT, "frac": round(achieved / peak, 4),
                     "traffic": None, "entries_per_pass": int(entries), "slots_per_entry": SLOTS_PER_ENTRY},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out_line), flush=True)
    plan.close()


def bench_calibrate(args, binding):
    """Issue rates behind the VALU roofline: v_fma_f32, v_sin_f32, v_cos_f32 and the entry body
    (phase FMA, sin, cos, four FMAs), each the best of five launches of the library's probe."""
    names = ["fma", "sin", "cos", "entry_body"]
    rates = {}
    for kind, name in enumerate(names):
        best = max(binding.calibrate(kind, 4096)[0] for _ in range(5))
        rates[name] = best
        log("%s: %.3f T chain steps/s" % (name, best / 1e12))
    fma = rates["fma"]
    out = {"metric": "VALU issue rates (T lane-ops/s)", "value": round(rates["entry_body"] / 1e12, 4),
           "unit": "T entry bodies/s", "n_gpus": 1, "steps": 5, "warmup": 1, "higher_is_better": True,
           "config": {"workload": "calib: 8 work-groups of 256 threads per compute unit, 8 independent chains per lane"},
           "rates_T_per_s": {k: round(v / 1e12, 3) for k, v in rates.items()},
           "fma_peak_T_per_s": round(VALU_SLOTS_PER_S / 1e12, 3),
           "fma_fraction_of_peak": round(fma / VALU_SLOTS_PER_S, 4),
           "sin_fraction_of_quarter_rate": round(rates["sin"] * TRANS_SLOTS / VALU_SLOTS_PER_S, 4),
           "cos_fraction_of_quarter_rate": round(rates["cos"] * TRANS_SLOTS / VALU_SLOTS_PER_S, 4),
           "entry_body_fraction_of_peak": round(rates["entry_body"] * SLOTS_PER_ENTRY / VALU_SLOTS_PER_S, 4)}
    print(json.dumps(out), flush=True)


def bench_ragged(args, torch, binding, dev):
    """96 independent scenes (ragged arrays, bands and grids) advanced together, one launch per
    phase per iteration, the whole solve captured in one HIP graph.  Step sizes and l1 weights
    per scene come from the oracle-written table (5 % of each scene's lambda_max).  The oracle
    checks the first iteration of every scene on a seeded 1 % voxel sample and the first two
    iterations of the scenes with the smallest grids in full; its time on that work is the CPU
    baseline."""
    scenes = W.ragged_scenes()
    K, Wm = args.steps, args.warmup
    steps = json.load(open(STEP_SIZES))["c3"]["scenes"]
    log("ragged batch: %d scenes, sum B*N = %.3e entries per operator per iteration" % (
        len(scenes), sum(sc["B"] * sc["N"] for sc in scenes)))
    batch = binding.Batch([sc["geom"] for sc in scenes])
    ys, rows, etas, alphas, s_true, y_hosts = [], [], [], [], [], []
    for i, sc in enumerate(scenes):
        st, idx = W.random_scene(sc["N"], sc["density"], seed=sc["seed"] + 1)
        plan = batch.plans[i]
        y0 = plan.spgm_forward(torch.arange(sc["M"], dtype=torch.int32, device=dev),
                               torch.from_numpy(st.astype(np.complex64)).to(dev))
        y = W.add_noise(y0.cpu().numpy().astype(np.complex128), sc["snr_db"], seed=sc["seed"] + 2)
        ys.append(torch.from_numpy(y.astype(np.complex64)).to(dev))
        rows.append(torch.from_numpy(W.draw_rows(sc["M"], sc["B"], max(K, Wm, 2), seed=sc["seed"] + 3)).to(dev))
        eta = float(np.float32(steps[i]["eta"]))
        etas.append(eta)
        alphas.append(float(np.float32(steps[i]["lambda"] * eta)))
        s_true.append(st)
    rps = None if args.no_tune else batch.autotune([sc["B"] for sc in scenes])
    if rps:
        log("ragged batch: %d rows per work item (autotuned)" % rps)
    ss = [torch.zeros(sc["N"], dtype=torch.complex64, device=dev) for sc in scenes]
    # parity sample: the first two iterations of every scene from zero
    s_par1 = [torch.zeros(sc["N"], dtype=torch.complex64, device=dev) for sc in scenes]
    batch.solve([r[:1].contiguous() for r in rows], ys, s_par1, etas, alphas, use_graph=True)
    s_par2 = [torch.zeros(sc["N"], dtype=torch.complex64, device=dev) for sc in scenes]
    batch.solve([r[:2].contiguous() for r in rows], ys, s_par2, etas, alphas, use_graph=True)
    torch.cuda.synchronize()
    s_par1 = [t.cpu().numpy() for t in s_par1]
    s_par2 = [t.cpu().numpy() for t in s_par2]
    if Wm:
        batch.solve([r[:Wm].contiguous() for r in rows], ys, ss, etas, alphas, use_graph=True)
    timed = [r[:K].contiguous() for r in rows]
    for s in ss:
        s.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.solve(timed, ys, ss, etas, alphas, use_graph=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert batch.status() == 0
    dt = t1 - t0
    entries = float(sum(sc["B"] * sc["N"] for sc in scenes))
    value = entries * K / dt / 1e9
    log("timed %d iterations of %d scenes in %.3f s (%.3f ms per iteration)" % (K, len(scenes), dt, 1e3 * dt / K))
    nmse_db = [float(10 * np.log10(np.sum(np.abs(ss[i].cpu().numpy() - s_true[i]) ** 2) / np.sum(np.abs(s_true[i]) ** 2)))
               for i in range(len(scenes))]
    errs1, errs2 = {}, {}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        rows_h = [r[:2].cpu().numpy() for r in rows]
        t_work, n_ent = 0.0, 0.0
        log("oracle: measurements of the %d scenes" % len(scenes))
        for i, sc in enumerate(scenes):
            orc = oracle.Oracle(sc["geom"])
            st, idx = W.random_scene(sc["N"], sc["density"], seed=sc["seed"] + 1)
            y_orc = W.add_noise(orc.forward_sparse(np.arange(sc["M"]), idx, st[idx]), sc["snr_db"], seed=sc["seed"] + 2)
            vs = W.voxel_sample(sc["N"], 0.01, seed=sc["seed"] + 42)
            r0 = rows_h[i][0]
            c0 = time.perf_counter()
            ref1 = oracle.prox_l1((etas[i] / sc["B"]) * orc.adjoint_voxels(r0, y_orc[r0], vs), alphas[i])
            t_work += time.perf_counter() - c0
            n_ent += float(sc["B"]) * vs.size
            errs1[i] = oracle.rel_l2(s_par1[i][vs], ref1)
            if sc["N"] <= 2048:
                c0 = time.perf_counter()
                ref2 = orc.solve(rows_h[i], y_orc, np.zeros(sc["N"]), etas[i], alphas[i])
                t_work += time.perf_counter() - c0
                n_ent += 4.0 * sc["B"] * sc["N"]
                errs2[i] = oracle.rel_l2(s_par2[i], ref2)
        cpu = {"value": round(n_ent / t_work / 1e9, 4), "unit": "Gentries/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "first iteration of all %d scenes on 1%% voxel samples plus two full iterations of the %d "
                         "smallest scenes, FP64, %.1f s" % (len(scenes), len(errs2), t_work)}
        log("oracle parity: iteration 1 (96 scenes, 1%% voxels) worst rel_l2 %.3e; iteration 2 (%d scenes) worst %.3e"
            % (max(errs1.values()), len(errs2), max(errs2.values())))
    achieved = 2 * entries * SLOTS_PER_ENTRY * K / dt / 1e12
    peak = VALU_SLOTS_PER_S / 1e12
    out = {
        "metric": "projector Gentries/s (A_B s + A_B^H r) and SPGM iters/s at fixed NMSE vs oracle",
        "value": round(value, 2), "unit": "Gentries/s", "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": round(1e3 * dt / K, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c3: ragged batch of %d scenes (T, R in 8..32, F in 16..64, grids 16x16x8..64x64x32, "
                               "B = ceil(M/4)), l1 weight 5%% of each scene's lambda_max, one launch per phase, "
                               "whole solve in one HIP graph" % len(scenes),
                   "scenes": len(scenes), "sum_BN": int(entries),
                   "launch_shape": {"rows_per_work_item": rps or 1024, "autotuned": rps is not None}},
        "spgm_iters_per_s": round(K / dt, 2),
        "rel_l2_vs_oracle": None if not errs1 else float("%.3e" % max(list(errs1.values()) + list(errs2.values()))),
        "rel_l2_vs_oracle_iter1_1pct_voxels_per_scene": {str(i): float("%.3e" % e) for i, e in errs1.items()},
        "rel_l2_vs_oracle_iter2_small_scenes": {str(i): float("%.3e" % e) for i, e in errs2.items()},
        "nmse_db_vs_truth_after_steps_per_scene": {str(i): round(v, 2) for i, v in enumerate(nmse_db)},
        "roofline": {"bound": "alu", "kernel": "whole iteration (both tile phases)", "achieved": round(achieved, 3),
                     "peak": round(peak, 3), "unit": SLOT_UNIT, "frac": round(achieved / peak, 4),
                     "traffic": None, "entries_per_launch": int(entries), "slots_per_entry": SLOTS_PER_ENTRY},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    batch.close()


# Dense bfloat16 MFMA peak of MI355X (matrix cores, no sparsity).
MFMA_BF16_PEAK = 2.5e15
# VALU slots per entry in the batched kernels: phase FMA, sin and cos (4 slots each), the two
# amplitude multiplies and one packed conversion to 16 bits; the products move to the MFMA.
MM_SLOTS_PER_ENTRY = 1 + 2 * TRANS_SLOTS + 3


def bench_batched(args, torch, binding, dev):
    """Shared-geometry batch: 32 scenes of the c1 geometry advanced together by the batched
    SPGM step (entries formed once per minibatch and applied to all 32 right-hand sides as a
    bfloat16 complex GEMM on the matrix cores).  Also solves every scene with the float32
    projector for the same iterations and reports both reconstruction errors (matched NMSE)."""
    cfg = W.CONFIGS["c1"]
    geom = W.config_geometry("c1")
    M, N = W.dims(geom)
    B = cfg["B"]
    Kr = 32
    steps, Wm = args.steps, args.warmup
    prec = binding.MM_BF16
    sj = json.load(open(STEP_SIZES))["c1"]
    eta = float(np.float32(sj["eta"]))
    alpha = float(np.float32(sj["lambda"] * eta))
    log("batched c1 x %d scenes: M=%d N=%d B=%d; drawing %d minibatches" % (Kr, M, N, B, Wm + steps))
    plan = binding.Plan(geom)
    shape = plan.spgm_plan_batched_shape(B) if args.no_tune else plan.spgm_plan_autotune_batched(B, prec)
    log("batched launch shape%s: forward %d row tiles per wave, %d bricks per work-group, %d waves over %d z slices; "
        "adjoint %d splits, %d staged rows" % ((" (autotuned)" if not args.no_tune else "",) + tuple(shape[:6])))
    all_rows = torch.arange(M, dtype=torch.int32, device=dev)
    S_true = np.zeros((N, Kr), dtype=np.complex64)
    Y = np.zeros((M, Kr), dtype=np.complex64)
    for k in range(Kr):
        st, _ = W.random_scene(N, cfg["density"], seed=5000 + k)
        S_true[:, k] = st
        y0 = plan.spgm_forward(all_rows, torch.from_numpy(st.astype(np.complex64)).to(dev))
        Y[:, k] = W.add_noise(y0.cpu().numpy().astype(np.complex128), cfg["snr_db"], seed=6000 + k)
    Yd = torch.from_numpy(Y).to(dev)
    rows = W.draw_rows(M, B, Wm + steps, seed=cfg["seed"] + 3)
    rows_d = torch.from_numpy(rows).to(dev)
    S = torch.zeros(N, Kr, dtype=torch.complex64, device=dev)
    if Wm:
        plan.spgm_solve_batched(rows_d[:Wm].contiguous(), Yd, S, eta, alpha, precision=prec)
    S.zero_()
    timed = rows_d[Wm:Wm + steps].contiguous()
    plan.spgm_plan_timing(True)
    plan.spgm_plan_timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.spgm_solve_batched(timed, Yd, S, eta, alpha, precision=prec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fwd_ms, fwd_n, adj_ms, adj_n = plan.spgm_plan_timing_read()
    plan.spgm_plan_timing(False)
    assert plan.spgm_plan_status() == 0
    dt = t1 - t0
    fwd_avg, adj_avg = fwd_ms / max(fwd_n, 1) * 1e-3, adj_ms / max(adj_n, 1) * 1e-3
    entries = float(B) * N
    log("timed %d batched iterations in %.3f s (%.3f ms each); batched forward %.4f ms, adjoint %.4f ms" % (
        steps, dt, 1e3 * dt / steps, 1e3 * fwd_avg, 1e3 * adj_avg))
    # Matched reconstruction error: the float32 projector on each scene, same rows and steps.
    S_b = S.cpu().numpy().astype(np.complex128)
    nmse_b, nmse_f = [], []
    t_f = 0.0
    for k in range(Kr):
        s32 = torch.zeros(N, dtype=torch.complex64, device=dev)
        yk = Yd[:, k].contiguous()
        torch.cuda.synchronize()
        a = time.perf_counter()
        plan.spgm_solve(timed, yk, s32, eta, alpha)
        torch.cuda.synchronize()
        t_f += time.perf_counter() - a
        st = S_true[:, k].astype(np.complex128)
        den = np.sum(np.abs(st) ** 2)
        nmse_b.append(10 * np.log10(np.sum(np.abs(S_b[:, k] - st) ** 2) / den))
        nmse_f.append(10 * np.log10(np.sum(np.abs(s32.cpu().numpy() - st) ** 2) / den))
    dnmse = float(np.max(np.abs(np.array(nmse_b) - np.array(nmse_f))))
    log("NMSE vs truth after %d iterations: batched bf16 mean %.3f dB, float32 mean %.3f dB, worst gap %.4f dB; "
        "float32 solves of the %d scenes one by one: %.3f s" % (steps, np.mean(nmse_b), np.mean(nmse_f), dnmse, Kr, t_f))
    flops = 8.0 * entries * Kr  # real flops of one batched operator
    fwd_name = "k_mm_fwd_rows" if shape[6] else "k_mm_fwd"  # entries in A-operand order or via LDS
    kname, kavg = (fwd_name, fwd_avg) if fwd_avg >= adj_avg else ("k_mm_adj", adj_avg)
    achieved = flops / kavg
    cpu = None
    rel = None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.Oracle(geom)
        y1 = Y[:, 0].astype(np.complex128)
        s_par = torch.zeros(N, 1, dtype=torch.complex64, device=dev)
        plan.spgm_solve_batched(rows_d[:1].contiguous(), Yd[:, :1].contiguous(), s_par, eta, alpha, precision=prec)
        log("oracle: one SPGM iteration of scene 0 on %d threads" % oracle.num_threads())
        c0 = time.perf_counter()
        ref = orc.solve(rows[:1], y1, np.zeros(N), eta, alpha)
        c1 = time.perf_counter()
        rel = oracle.rel_l2(s_par.cpu().numpy()[:, 0], ref)
        cpu = {"value": round(entries / (c1 - c0) / 1e9, 4), "unit": "G entry-RHS products/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "1 SPGM iteration of 1 of the 32 scenes (B=%d x N=%d), FP64, %.1f s" % (B, N, c1 - c0)}
        log("oracle: %.1f s; batched bf16 iterate after 1 iteration rel_l2 vs oracle %.3e" % (c1 - c0, rel))
    out = {
        "metric": "batched projector G entry-RHS products/s (K x B x N per operator, forward + adjoint) at matched NMSE",
        "value": round(entries * Kr * steps / dt / 1e9, 1),
        "unit": "G entry-RHS/s",
        "n_gpus": 1, "steps": steps, "warmup": Wm, "ms_per_step": round(1e3 * dt / steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "c1 geometry (32 Tx + 32 Rx, 64 frequencies, 64x64x32 voxels, B=4096) with K=32 "
                               "scenes sharing the minibatch; batched SPGM step, bfloat16 operands, float32 accumulation",
                   "M": M, "N": N, "B": B, "K": Kr,
                   "launch_shape": {"fwd_row_tiles_per_wave": shape[0], "fwd_bricks_per_wg": shape[1],
                                    "fwd_waves": shape[2], "fwd_z_slices": shape[3], "adj_splits": shape[4],
                                    "adj_staged_rows": shape[5], "autotuned": not args.no_tune}},
        "spgm_iters_per_s": round(steps / dt, 2),
        "scene_iters_per_s": round(Kr * steps / dt, 1),
        "float32_scene_iters_per_s": round(Kr * steps / t_f, 1),
        "nmse_db_batched_mean": round(float(np.mean(nmse_b)), 4),
        "nmse_db_float32_mean": round(float(np.mean(nmse_f)), 4),
        "nmse_db_worst_gap": round(dnmse, 4),
        "rel_l2_vs_oracle_after_1_iter": None if rel is None else float("%.3e" % rel),
        "roofline": {"bound": "mfma", "kernel": kname, "achieved": round(achieved / 1e12, 2),
                     "peak": MFMA_BF16_PEAK / 1e12, "unit": "TFLOP/s", "frac": round(achieved / MFMA_BF16_PEAK, 4),
                     "traffic": stored_traffic(kname, "c1k32", mm_shape_key(shape)), "flops_per_launch": flops,
                     "avg_launch_ms": round(kavg * 1e3, 5),
                     "fwd_mm_ms": round(fwd_avg * 1e3, 5), "adj_mm_ms": round(adj_avg * 1e3, 5),
                     "fwd_gentries_per_s": round(entries / fwd_avg / 1e9, 1),
                     "adj_gentries_per_s": round(entries / adj_avg / 1e9, 1),
                     "alu_view": {"achieved": round(entries * MM_SLOTS_PER_ENTRY / kavg / 1e12, 3),
                                  "peak": round(VALU_SLOTS_PER_S / 1e12, 3), "unit": SLOT_UNIT,
                                  "frac": round(entries * MM_SLOTS_PER_ENTRY / kavg / VALU_SLOTS_PER_S, 4),
                                  "slots_per_entry": MM_SLOTS_PER_ENTRY}},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    plan.close()


def bench_structured(args, torch, binding, dev):
    """c1 geometry with structured minibatches (16 frequencies x 16 Tx x 16 Rx = 4096 rows, the
    c1 minibatch size): the separable factorisation of Eq. 2 with float32 GEMMs on the matrix
    cores.  Reported in the same unit as the pair kernels (B N entries applied per gradient)."""
    cfg = W.CONFIGS["c1"]
    geom = W.config_geometry("c1")
    M, N = W.dims(geom)
    nf, nt, nr = 16, 16, 16
    B = nf * nt * nr
    K, Wm = args.steps, args.warmup
    sj = json.load(open(STEP_SIZES))["c1"]
    eta = float(np.float32(sj["eta"]))
    alpha = float(np.float32(sj["lambda"] * eta))
    log("structured c1: (%d f, %d Tx, %d Rx) = %d rows, N=%d; drawing %d minibatches" % (nf, nt, nr, B, N, Wm + K))
    fs, ts, rs = W.draw_structured_subsets(cfg["T"], cfg["R"], cfg["F"], nf, nt, nr, max(Wm + K, args.cpu_iters),
                                           seed=cfg["seed"] + 7)
    s_true, idx = W.config_scene("c1")
    plan = binding.Plan(geom)
    items = (plan.spgm_plan_structured_shape(nf, nt, nr) if args.no_tune
             else plan.spgm_plan_autotune_structured(nf, nt, nr))
    log("structured kernels: %d items per thread%s" % (items, "" if args.no_tune else " (autotuned)"))
    all_rows = torch.arange(M, dtype=torch.int32, device=dev)
    y0 = plan.spgm_forward(all_rows, torch.from_numpy(s_true.astype(np.complex64)).to(dev))
    y_host = W.add_noise(y0.cpu().numpy().astype(np.complex128), cfg["snr_db"], seed=cfg["seed"] + 2)
    y = torch.from_numpy(y_host.astype(np.complex64)).to(dev)
    fs_d, ts_d, rs_d = (torch.from_numpy(x).to(dev) for x in (fs, ts, rs))
    n_par = args.cpu_iters
    s_par = torch.zeros(N, dtype=torch.complex64, device=dev)
    plan.spgm_solve_structured(fs_d[:n_par].contiguous(), ts_d[:n_par].contiguous(), rs_d[:n_par].contiguous(), y,
                               s_par, eta, alpha)
    s_par_host = s_par.cpu().numpy()
    s = torch.zeros(N, dtype=torch.complex64, device=dev)
    if Wm:
        plan.spgm_solve_structured(fs_d[:Wm].contiguous(), ts_d[:Wm].contiguous(), rs_d[:Wm].contiguous(), y, s,
                                   eta, alpha)
    s.zero_()
    sl = slice(Wm, Wm + K)
    tf, tt, tr = fs_d[sl].contiguous(), ts_d[sl].contiguous(), rs_d[sl].contiguous()
    plan.spgm_plan_timing(True)
    plan.spgm_plan_timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.spgm_solve_structured(tf, tt, tr, y, s, eta, alpha)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fwd_ms, fwd_n, adj_ms, adj_n = plan.spgm_plan_timing_read()
    plan.spgm_plan_timing(False)
    assert plan.spgm_plan_status() == 0
    dt = t1 - t0
    fwd_avg, adj_avg = fwd_ms / max(fwd_n, 1) * 1e-3, adj_ms / max(adj_n, 1) * 1e-3
    entries = float(B) * N
    log("timed %d structured iterations in %.4f s (%.4f ms each); forward %.4f ms, adjoint %.4f ms" % (
        K, dt, 1e3 * dt / K, 1e3 * fwd_avg, 1e3 * adj_avg))
    # Roofline of the dominant kernel: float32 matrix-core flops of its per-frequency GEMMs.
    flops = 8.0 * entries
    kname, kavg = ("k_sf_fwd", fwd_avg) if fwd_avg >= adj_avg else ("k_sf_adj", adj_avg)
    achieved = flops / kavg
    cpu = None
    rel = None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.Oracle(geom)
        y_orc = W.add_noise(orc.forward_sparse(np.arange(M), idx, s_true[idx]), cfg["snr_db"], seed=cfg["seed"] + 2)
        rows = np.stack([W.structured_rows(cfg["T"], cfg["R"], fs[k], ts[k], rs[k]) for k in range(n_par)])
        log("oracle: %d SPGM iterations on the product rows, %d threads" % (n_par, oracle.num_threads()))
        c0 = time.perf_counter()
        ref = orc.solve(rows, y_orc, np.zeros(N), eta, alpha)
        c1 = time.perf_counter()
        rel = oracle.rel_l2(s_par_host, ref)
        cpu = {"value": round(entries * n_par / (c1 - c0) / 1e9, 4), "unit": "Gentries/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "%d SPGM iterations on the same structured minibatches (B=%d rows x N=%d voxels), FP64, %.1f s"
                         % (n_par, B, N, c1 - c0)}
        log("oracle: %.1f s, GPU iterate %d rel_l2 vs oracle %.3e" % (c1 - c0, n_par, rel))
    out = {
        "metric": "projector Gentries/s (A_B s + A_B^H r) and SPGM iters/s at fixed NMSE vs oracle",
        "value": round(entries * K / dt / 1e9, 2), "unit": "Gentries/s", "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": round(1e3 * dt / K, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c1 geometry (32 Tx + 32 Rx, 64 frequencies, 64x64x32 voxels) with structured "
                               "minibatches of 16 frequencies x 16 Tx x 16 Rx (B=4096); separable factorisation, "
                               "float32 GEMMs on the matrix cores", "M": M, "N": N, "B": B,
                   "structured": [nf, nt, nr],
                   "launch_shape": {"items_per_thread": items, "autotuned": not args.no_tune}},
        "spgm_iters_per_s": round(K / dt, 2),
        "rel_l2_vs_oracle": None if rel is None else float("%.3e" % rel),
        "rel_l2_vs_oracle_after_iters": n_par,
        "roofline": {"bound": "mfma", "kernel": kname, "achieved": round(achieved / 1e12, 3),
                     "peak": 157.3, "unit": "TFLOP/s (float32 matrix cores)", "frac": round(achieved / 157.3e12, 4),
                     "traffic": stored_traffic(kname, "c1s", "items%d" % items), "flops_per_launch": flops,
                     "avg_launch_ms": round(kavg * 1e3, 5),
                     "sf_fwd_ms": round(fwd_avg * 1e3, 5), "sf_adj_ms": round(adj_avg * 1e3, 5),
                     "factors_per_launch": nf * (nt + nr) * N},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    plan.close()


def bench_tv(args, torch, binding, dev):
    """c1 geometry and minibatches with the magnitude-TV prox in place of the soft threshold
    (10 dual iterations per step) on a blocky random-phase scene.  The step is the same
    gradient evaluation followed by the TV prox; the TV dual iteration is timed on its own."""
    cfg = W.CONFIGS["c1"]
    geom = W.config_geometry("c1")
    M, N = W.dims(geom)
    B = cfg["B"]
    K, Wm = args.steps, args.warmup
    tv_iters = 10
    sj = json.load(open(STEP_SIZES))["c1"]
    eta = float(np.float32(sj["eta"]))
    rows = W.config_rows("c1", K=max(Wm + K, args.cpu_iters))
    s_true = W.blocky_field(cfg["grid"], n_boxes=6, noise=0.0, seed=cfg["seed"] + 11)
    plan = binding.Plan(geom)
    splits = None if args.no_tune else plan.spgm_plan_autotune(B)
    all_rows = torch.arange(M, dtype=torch.int32, device=dev)
    y0 = plan.spgm_forward(all_rows, torch.from_numpy(s_true.astype(np.complex64)).to(dev))
    y_host = W.add_noise(y0.cpu().numpy().astype(np.complex128), cfg["snr_db"], seed=cfg["seed"] + 12)
    y = torch.from_numpy(y_host.astype(np.complex64)).to(dev)
    # TV weight: the stored l1 weight of the c1 workload (from the oracle), times the step size
    alpha = float(np.float32(sj["lambda"] * eta))
    rows_d = torch.from_numpy(rows).to(dev)
    n_par = args.cpu_iters
    s_par = torch.zeros(N, dtype=torch.complex64, device=dev)
    plan.spgm_solve_reg(rows_d[:n_par].contiguous(), y, s_par, eta, alpha, binding.REG_TV_MAGNITUDE,
                        tv_iters=tv_iters)
    s_par_host = s_par.cpu().numpy()
    s = torch.zeros(N, dtype=torch.complex64, device=dev)
    if Wm:
        plan.spgm_solve_reg(rows_d[:Wm].contiguous(), y, s, eta, alpha, binding.REG_TV_MAGNITUDE, tv_iters=tv_iters)
    s.zero_()
    timed = rows_d[Wm:Wm + K].contiguous()
    plan.spgm_plan_timing(True)
    plan.spgm_plan_timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.spgm_solve_reg(timed, y, s, eta, alpha, binding.REG_TV_MAGNITUDE, tv_iters=tv_iters)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fwd_ms, fwd_n, adj_ms, adj_n = plan.spgm_plan_timing_read()
    plan.spgm_plan_timing(False)
    assert plan.spgm_plan_status() == 0
    dt = t1 - t0
    # TV dual iteration: slope of the prox time between 8 and 208 dual iterations, HIP events on
    # the stream the prox is launched on (includes the gaps between back-to-back launches).
    v = s.clone()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    stream = torch.cuda.current_stream()
    plan.spgm_prox(v, alpha, binding.REG_TV_MAGNITUDE, tv_iters=208)
    ev[0].record(stream)
    plan.spgm_prox(v, alpha, binding.REG_TV_MAGNITUDE, tv_iters=8)
    ev[1].record(stream)
    ev[2].record(stream)
    plan.spgm_prox(v, alpha, binding.REG_TV_MAGNITUDE, tv_iters=208)
    ev[3].record(stream)
    torch.cuda.synchronize()
    tv_iter_s = (ev[2].elapsed_time(ev[3]) - ev[0].elapsed_time(ev[1])) * 1e-3 / 200.0
    tv_bytes = float(TV_BYTES_PER_VOXEL) * N
    fwd_avg, adj_avg = fwd_ms / max(fwd_n, 1) * 1e-3, adj_ms / max(adj_n, 1) * 1e-3
    entries = float(B) * N
    kname, kavg = ("k_fwd_tile", fwd_avg) if fwd_avg >= adj_avg else ("k_adj_tile", adj_avg)
    achieved = entries * SLOTS_PER_ENTRY / kavg / 1e12
    peak = VALU_SLOTS_PER_S / 1e12
    log("timed %d TV-regularised iterations in %.4f s (%.4f ms each); forward %.4f ms, adjoint %.4f ms, "
        "TV dual iteration %.2f us" % (K, dt, 1e3 * dt / K, 1e3 * fwd_avg, 1e3 * adj_avg, 1e6 * tv_iter_s))
    cpu = None
    rel = None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.Oracle(geom)
        y_orc = W.add_noise(orc.forward(np.arange(M), s_true), cfg["snr_db"], seed=cfg["seed"] + 12)
        log("oracle: %d TV-regularised SPGM iterations, %d threads" % (n_par, oracle.num_threads()))
        c0 = time.perf_counter()
        ref = np.zeros(N, dtype=np.complex128)
        for k in range(n_par):
            ref = orc.step_reg(rows[k], y_orc, ref, eta, alpha, 2, tv_iters=tv_iters)
        c1 = time.perf_counter()
        rel = oracle.rel_l2(s_par_host, ref)
        cpu = {"value": round(entries * n_par / (c1 - c0) / 1e9, 4), "unit": "Gentries/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "%d TV-regularised SPGM iterations of the same workload (B=%d rows x N=%d voxels, "
                         "%d dual iterations per prox), FP64, %.1f s" % (n_par, B, N, tv_iters, c1 - c0)}
        log("oracle: %.1f s, GPU iterate %d rel_l2 vs oracle %.3e" % (c1 - c0, n_par, rel))
    out = {
        "metric": "projector Gentries/s (A_B s + A_B^H r) and SPGM iters/s at fixed NMSE vs oracle",
        "value": round(entries * K / dt / 1e9, 2), "unit": "Gentries/s", "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": round(1e3 * dt / K, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c1 (32 Tx + 32 Rx, 64 frequencies, 64x64x32 voxels, B=4096) with the magnitude-TV "
                               "prox, %d dual iterations per step, blocky random-phase scene" % tv_iters,
                   "M": M, "N": N, "B": B, "tv_iters": tv_iters, "hip_graph": False,
                   "row_splits": None if splits is None else {"forward": splits[0], "adjoint": splits[1]}},
        "spgm_iters_per_s": round(K / dt, 2),
        "rel_l2_vs_oracle": None if rel is None else float("%.3e" % rel),
        "rel_l2_vs_oracle_after_iters": n_par,
        "roofline": {"bound": "alu", "kernel": kname, "achieved": round(achieved, 3), "peak": round(peak, 3),
                     "unit": SLOT_UNIT, "frac": round(achieved / peak, 4),
                     "traffic": stored_traffic(kname, "c1tv",
                                               plan.spgm_plan_launch_shape(B)[0 if kname == "k_fwd_tile" else 1]),
                     "entries_per_launch": int(entries), "slots_per_entry": SLOTS_PER_ENTRY,
                     "avg_launch_ms": round(kavg * 1e3, 5), "fwd_tile_ms": round(fwd_avg * 1e3, 5),
                     "adj_tile_ms": round(adj_avg * 1e3, 5)},
        "tv_dual_iteration": {"bound": "hbm", "kernel": "k_tv_iter<false>", "us": round(tv_iter_s * 1e6, 3),
                              "bytes": tv_bytes, "achieved": round(tv_bytes / tv_iter_s / 1e9, 1),
                              "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": round(tv_bytes / tv_iter_s / HBM_PEAK, 4),
                              "share_of_step": round(tv_iters * tv_iter_s / (dt / K), 4)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
