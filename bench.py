#!/usr/bin/env python3
"""Benchmark of the deform-and-query path on one MI355X.

Step (the timed unit of ``value``): one training step of the path on the
8192-ray workload -- march through the 128^3 occupancy grid, 24-init Broyden
deform, hash encode, MLP, composite, L2 loss, and every backward pass
(composite, MLP, encode, implicit-function-theorem deform), all in the
library's HIP kernels, FP32.  The sample count stays in device memory and
each step is one HIP graph replay.  value = posed samples (kept by the
occupancy skip) per second over the K timed steps, inputs resident in HBM.

Extra keys of the one JSON line:
  stages_ms, stage_roofline
                GPU time of each stage (its calls captured in a graph of
                their own and replayed back to back, HIP events on the
                stream) and each stage's algorithmic work against its bound
  roofline      the dominant stage against its roofline, with the HBM
                traffic of its kernels from rocprofv3 counters
  host_count_eager_ms_per_step
                the same step with a host round trip for the sample count
  mixed_training_step
                FP16 table + BF16 MLP training step
  frame_540     ms per 540x540 frame: FP32 multi-init vs FP16 table + BF16
                MLP + learned root initialiser, and their pixel errors
  learned_init  the initialiser on held-out poses: steps, fallback rate,
                root error, deform time vs multi-init
  tiny_forward_f32, empty_space_skipping, hash_stress_2e23
                the tiny forward, skipping on/off (the synthetic analogue of
                Tab. 3) and a 2^23-entry hash table
  batched_render
                16 poses at mixed resolutions in one HIP graph (autotuned
                stream schedule)
  cpu_baseline  the FP64 oracle timed on the host cores

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-frame] [--no-mixed] [--init-poses P]
                       [--copy-calibration] [--pmc-summary FETCH_DIR WRITE_DIR]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_VEC_TFLOPS = 157.3
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0

# Algorithmic work per unit, counted from the method (not from the kernels'
# actual traffic); the per-stage table of the JSON line uses these.
# deform, pre-blended form: per init, the start point B_i^-1 x' (18), the
# residual and Jacobian at it (8 corners of A_c x_h and their interpolation,
# the trilinear derivatives: ~470) and the 3x3 inverse (~45), ~564 in all;
# per Broyden step, the step -H g (18), the residual at the new point (~230)
# and the rank-one update of H (~78), ~326
DEFORM_FLOP_PER_INIT = 564.0
DEFORM_FLOP_PER_STEP = 326.0
HASH_GATHER_BYTES = {4: 16 * 8 * 2 * 4, 2: 16 * 8 * 2 * 2}  # 16 levels x 8 corners x 2 features
FEAT_BYTES = {4: 16 * 2 * 4, 2: 16 * 2 * 2}
# table gradient: read-modify-write of the 256 touched FP32 entries, dL/dfeat
# and x read; position gradient: the table gather, dL/dfeat and x read, the
# gradient written
HASH_BWD_BYTES = 2 * 16 * 8 * 2 * 4 + 16 * 2 * 4 + 12
HASH_BWD_X_BYTES = 16 * 8 * 2 * 4 + 16 * 2 * 4 + 12 + 12
IFT_BYTES_PER_SAMPLE = 2 * 8 * 12 * 4 + 24 + 12 + 8 * 24 * 4  # moment RMW + x, v, u + skinning rows
MLP_FWD_FLOP = 12800.0
MLP_BWD_FLOP = 25600.0 + 12800.0  # backward plus the recomputed forward
MARCH_BYTES_PER_SAMPLE, MARCH_BYTES_PER_RAY = 20, 56
RENDER_FWD_BYTES_PER_SAMPLE, RENDER_BWD_BYTES_PER_SAMPLE, RENDER_BYTES_PER_RAY = 16, 32, 40

# kernels of each stage (names as rocprofv3 reports them)
STAGE_KERNELS = {
    "march": ["march_count", "march_scan", "march_fill"],
    "deform": ["blend_kernel", "solve_kernel", "guided_kernel", "fallback_kernel", "rootinit_kernel"],
    "hash_fwd": ["encode_kernel"],
    "mlp_fwd": ["mlp_fwd_f32", "mlp_fwd_bf16"],
    "render_fwd": ["render_fwd"],
    "loss+render_bwd": ["l2_loss_kernel", "render_bwd"],
    "mlp_bwd": ["mlp_bwd_f32", "mlp_bwd_bf16", "reduce_partials"],
    "hash_bwd_table": ["bin_count_kernel", "bin_hist_scan_kernel", "bin_plan_kernel", "bin_scatter_kernel",
                       "bin_clear_split_kernel", "bin_accum_kernel"],
    "hash_bwd_x": ["xgrad_level_kernel", "xgrad_sum_kernel"],
    "deform_bwd": ["ift_v_kernel", "ift_q_kernel", "ift_contract_kernel", "ift_b_kernel"],
}
PMC_SUMMARY = os.path.join(ROOT, "profiles", "training_step_f32_hbm_traffic.md")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(w, budget_s=10.0, single_core_budget_s=8.0):
    """The FP64 oracle's training step on the same workload, repeated until
    about budget_s seconds of host time have passed (at least once), on all
    the host's cores; then on one core.  Posed samples/s over those runs."""
    import oracle
    oracle.lib()

    def run(budget):
        runs, samples = 0, 0
        t0 = time.perf_counter()
        while True:
            ref = oracle.train_step(w)
            samples += ref["march"]["xs"].shape[0]
            runs += 1
            dt = time.perf_counter() - t0
            if dt >= budget or dt * (runs + 1) / runs > 3 * budget:
                return samples, runs, dt

    cores = oracle.num_threads()
    samples, runs, dt = run(budget_s)
    oracle.set_num_threads(1)
    s1, r1, d1 = run(single_core_budget_s)
    oracle.set_num_threads(cores)
    return {"value": samples / dt, "unit": "posed samples/s", "cores": cores, "kind": "oracle",
            "sample": f"the full training step ({w.R} rays, {samples // runs} posed samples), forward + every "
                      f"backward, {runs} run(s) in {dt:.1f} s",
            "single_core": {"value": s1 / d1, "runs": r1, "seconds": round(d1, 1)},
            "host_cpu": _cpu_model()}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def source_digest():
    """Digest of the library's kernel sources; counter figures taken from
    other sources are stale."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2212_10550_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_traffic(stage, kernels=None):
    """HBM bytes per launch of a stage's kernels from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, each divided by the factor a plain
    copy kernel of known size reads), or None when the summary is missing or
    the kernel sources changed since the counters were taken."""
    try:
        with open(PMC_SUMMARY) as f:
            txt = f.read()
        blob = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("source_digest") != source_digest():
        return None
    per = blob["kernels"]
    tot, seen = 0.0, False
    for name, rec in per.items():
        if any(k in name for k in (kernels or STAGE_KERNELS.get(stage, []))):
            tot += rec["fetch_kib"] * 1024 / blob["copy_factor_fetch"] + rec["write_kib"] * 1024 / blob["copy_factor_write"]
            seen = True
    return tot if seen else None


def stage_rooflines(stage_ms, S, R, steps_total, nb, es, mlp_bf16, backward=True, fallback_steps=None):
    """One roofline entry per stage: algorithmic work / stage time against
    the bound the stage's work sits on."""
    out = {}

    def put(name, bound, work, unit_work):
        if name not in stage_ms or stage_ms[name] <= 0:
            return
        t = stage_ms[name] * 1e-3
        if bound == "hbm":
            ach, peak, unit = work / t / 1e9, PEAK_HBM_GBS, "GB/s"
        elif bound == "mfma":
            peak = PEAK_BF16_MFMA_TFLOPS if mlp_bf16 else PEAK_FP32_MFMA_TFLOPS
            ach, unit = work / t / 1e12, "TFLOP/s"
        else:
            ach, peak, unit = work / t / 1e12, PEAK_FP32_VEC_TFLOPS, "TFLOP/s"
        out[name] = {"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
                     "ms": stage_ms[name], "work_per_launch": work, "work_unit": unit_work}

    put("march", "hbm", MARCH_BYTES_PER_SAMPLE * S + MARCH_BYTES_PER_RAY * R, "bytes")
    if steps_total is not None:
        put("deform", "alu", DEFORM_FLOP_PER_INIT * nb * S + DEFORM_FLOP_PER_STEP * steps_total, "flop")
    put("hash_fwd", "hbm", (HASH_GATHER_BYTES[es] + 12 + FEAT_BYTES[2 if mlp_bf16 else 4]) * S, "bytes")
    put("mlp_fwd", "mfma", MLP_FWD_FLOP * S, "flop")
    put("render_fwd", "hbm", RENDER_FWD_BYTES_PER_SAMPLE * S + RENDER_BYTES_PER_RAY * R, "bytes")
    if backward:
        put("loss+render_bwd", "hbm", RENDER_BWD_BYTES_PER_SAMPLE * S + 2 * RENDER_BYTES_PER_RAY * R, "bytes")
        put("mlp_bwd", "mfma", MLP_BWD_FLOP * S, "flop")
        put("hash_bwd_table", "hbm", HASH_BWD_BYTES * S, "bytes")
        put("hash_bwd_x", "hbm", HASH_BWD_X_BYTES * S, "bytes")
        put("deform_bwd", "hbm", IFT_BYTES_PER_SAMPLE * S, "bytes")
    return out


def roofline(stage_ms, solve_ms, S, R, steps_total, nb):
    """The contract's roofline object for the dominant kernel of the FP32
    training step: the multi-init solve (`solve_kernel`), its algorithmic
    flops (every init's start, residual, Jacobian and inverse, every
    Broyden step the kernel reports) over its own average duration (the
    deform stage's graph replay less that of the blend alone, HIP events on
    the launch stream)."""
    table = stage_rooflines(stage_ms, S, R, steps_total, nb, 4, False)
    work = DEFORM_FLOP_PER_INIT * nb * S + DEFORM_FLOP_PER_STEP * steps_total
    ach = work / (solve_ms * 1e-3) / 1e12
    r = {"kernel": "solve_kernel", "stage": "deform", "bound": "alu", "achieved": ach,
         "peak": PEAK_FP32_VEC_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_FP32_VEC_TFLOPS,
         "traffic": pmc_traffic("deform", kernels=["solve_kernel"]),
         "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-kernel scaled)",
         "work_per_launch": work, "work_unit": "flop", "ms_per_launch": solve_ms,
         "work_count": f"{DEFORM_FLOP_PER_INIT:.0f} flop per init x {nb} inits x {S} samples + "
                       f"{DEFORM_FLOP_PER_STEP:.0f} flop per Broyden step x {steps_total} steps"}
    return r, table


def time_graph(torch, fn, n=10, reps=20):
    """GPU ms per call of fn: `reps` calls captured back to back in one HIP
    graph, the graph replayed n times between two HIP events on the current
    stream (the per-launch gap of a graph replay is then paid once per reps
    calls, not per call)."""
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(n):
        g.replay()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / (n * reps)


def deform_kernel_ms(torch, K, p):
    """(blend, solve) ms per call of the FP32 multi-init deform: the call
    with no samples (the blend alone) and the full call, each repeated in one
    graph; the solve is the difference."""
    w = p.w
    call = lambda S: K.snarf_deform(p.xs, S, p.cap, p.B, p.W, w.skin_aabb, w.hash_aabb, w.max_iter, w.tol_stop,
                                    w.tol_valid, p.xc, p.bone, None, None, p.ws_deform,
                                    S_dev=None if S == 0 else p.n_samples)
    blend = time_graph(torch, lambda: call(0))
    full = time_graph(torch, lambda: call(p.cap))
    return blend, full - blend


def time_forward(p, n, torch, stages=False):
    """ms per forward over n runs after warm-up (HIP-graph replays for a
    device-count pipeline); with stages, also the GPU ms of each stage
    (replayed on its own, Pipeline.stage_times).  Returns (ms, S, stage_ms)."""
    for _ in range(2):
        p.forward()
    torch.cuda.synchronize()
    stage_ms = p.stage_times(n, backward=False) if stages else None
    run = p.forward
    if p.device_count:
        p.capture_forward()
        run = p.replay
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / n
    return ms, p.read_count(), stage_ms


def time_train(p, steps, warmup, torch, stages=False):
    """Training steps: optional GPU ms of each stage (Pipeline.stage_times),
    then `steps` timed HIP-graph replays of the whole step (device-count
    pipeline).  Returns (seconds for the timed steps, S per step, stage_ms)."""
    for _ in range(warmup):
        p.train_step()
    torch.cuda.synchronize()
    stage_ms = p.stage_times(steps) if stages else None
    p.capture_train_step()
    for _ in range(warmup):
        p.train_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        p.train_step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, p.read_count(), stage_ms


def fit_initialiser(args, torch):
    """The learned root initialiser, fitted once on the solver's own roots
    (an input of the path, like the hash table's values)."""
    from paper_2212_10550_amd import rootinit
    t0 = time.perf_counter()
    data = rootinit.make_dataset(range(1000, 1000 + args.init_poses), 4096, device="cuda:0")
    params = rootinit.fit(data, epochs=args.init_epochs)
    del data
    torch.cuda.synchronize()
    return params, f"{args.init_poses} poses x 4096 points, {args.init_epochs} epochs, {time.perf_counter() - t0:.1f} s"


def frame_leg(args, params, fit_note, torch, np, K, synth, Pipeline, out, checks):
    wf = synth.full_frame()
    # FP32 multi-init reference frame
    p32 = Pipeline(wf, device="cuda:0", device_count=True)
    ms32, S, st32 = time_forward(p32, 5, torch, stages=True)
    c32 = p32.color.double().cpu().numpy()
    steps32 = int(p32.steps[:S].to(torch.int64).sum().item())
    del p32
    # FP16 table + BF16 MLP with the 24-init solve (the frame configuration
    # as specified)
    pm24 = Pipeline(wf, device="cuda:0", table_dtype=torch.float16, mlp_dtype=K.BF16, device_count=True)
    ms24, S24, st24 = time_forward(pm24, 5, torch, stages=True)
    c24 = pm24.color.double().cpu().numpy()
    steps24 = int(pm24.steps[:S24].to(torch.int64).sum().item())
    del pm24
    d24 = np.abs(c24 - c32)
    # FP16 table + BF16 MLP + learned initialiser
    pmx = Pipeline(wf, device="cuda:0", table_dtype=torch.float16, mlp_dtype=K.BF16, rootinit_params=params,
                   device_count=True)
    msmx, Smx, stmx = time_forward(pmx, 5, torch, stages=True)
    cmx = pmx.color.double().cpu().numpy()
    stepsmx = int(pmx.steps[:Smx].to(torch.int64).sum().item())
    fb = int(pmx.guided.n_fallback.item())
    used = int(pmx.n_used.to(torch.int64).sum().item())
    keys = ("color", "opacity", "n_used", "T_final")
    staged_out = {k: getattr(pmx, k).clone() for k in keys}
    del pmx
    # the same frame through the persistent kernel (one pose of a batch):
    # the same arithmetic, rays evaluated front to back up to termination
    from paper_2212_10550_amd.batch import BatchRenderer
    br = BatchRenderer([wf], params)
    tune_p = br.autotune((), n=5, persistent=((16, 256, 4, 3), (8, 256, 4, 3), (12, 256, 4, 3), (32, 256, 4, 2)))
    msp = br.time_ms(10)
    br.render()
    torch.cuda.synchronize()
    pp = br.poses[0]
    persistent = {"ms_per_frame": msp, "fps": 1e3 / msp, "schedule": br.schedule, "autotune_ms": tune_p,
                  "samples_evaluated": int(pp.n_evaluated.item()), "fallback_samples": int(pp.n_fallback.item()),
                  "outputs_bit_equal_staged": all(torch.equal(getattr(pp, k), staged_out[k]) for k in keys)}
    del br, staged_out
    dmx = np.abs(cmx - c32)
    out["frame_540"] = {
        "workload": "540x540 rays, 128^3 occupancy (~10%), <=128 samples/ray, early termination at T < 1e-4, "
                    "24-bone pose, hash T=2^19",
        "posed_samples": S, "samples_after_termination": used,
        "f32_multi_init": {"ms_per_frame": ms32, "fps": 1e3 / ms32, "broyden_steps": steps32,
                           "stages_ms": {k: round(v, 4) for k, v in st32.items()},
                           "stage_roofline": stage_rooflines(st32, S, wf.R, steps32, 24, 4, False, backward=False)},
        "f16_bf16_multi_init": {"ms_per_frame": ms24, "fps": 1e3 / ms24, "broyden_steps": steps24,
                                "stages_ms": {k: round(v, 4) for k, v in st24.items()},
                                "stage_roofline": stage_rooflines(st24, S24, wf.R, steps24, 24, 2, True,
                                                                  backward=False),
                                "pixel_diff_vs_f32_multi_init": {"mean": float(d24.mean()), "max": float(d24.max())}},
        "f16_bf16_learned_init": {"ms_per_frame": msmx, "fps": 1e3 / msmx, "broyden_steps": stepsmx,
                                  "stages_ms": {k: round(v, 4) for k, v in stmx.items()},
                                  "stage_roofline": stage_rooflines(stmx, Smx, wf.R, None, 24, 2, True,
                                                                    backward=False),
                                  "fallback_samples": fb,
                                  "pixel_diff_vs_f32_multi_init": {"mean": float(dmx.mean()),
                                                                   "max": float(dmx.max())},
                                  "persistent_kernel": persistent},
        "speedup_learned_mixed_vs_f32_multi": ms32 / msmx,
        "speedup_persistent_mixed_vs_f32_multi": ms32 / msp,
        "initialiser_fit": fit_note,
        "paper_context": "the paper renders its avatars at ~15 FPS at 540x540 and reconstructs one in about 60 s, on "
                         "one RTX 3090 (Sec. 4.2, Tab. 3; context only, different workload and hardware)",
    }
    checks["frame"] = (wf, c32, cmx, c24)


def extra_legs(args, params, torch, np, K, synth, Pipeline, out):
    """Tiny FP32 forward; empty-space skipping on/off (the synthetic analogue
    of Tab. 3); hash encode at T = 2^23 (FP16 table, 512 MiB)."""
    # tiny forward: 1024 rays x 64 samples, no occupancy grid, FP32
    wt = synth.tiny_forward()
    pt = Pipeline(wt, device="cuda:0", device_count=True)
    ms, S, _ = time_forward(pt, 20, torch)
    out["tiny_forward_f32"] = {"workload": "1024 front-face rays x 64 samples, 32^3x24 skinning grid, hash 2^14 FP32",
                               "ms": ms, "posed_samples": S, "samples_per_s": S / (ms * 1e-3)}
    del pt
    # empty-space skipping off: every cell occupied (Sec. 3.3, Tab. 3)
    w = synth.train_step()
    wd = synth.train_step()
    wd.occ = np.ones_like(w.occ)
    res = {}
    for tag, wl in (("with_skipping", w), ("without_skipping", wd)):
        pd = Pipeline(wl, device="cuda:0", device_count=True)
        dt, Sd, _ = time_train(pd, 5, 2, torch)
        res[tag] = {"ms_per_step": dt * 1e3 / 5, "posed_samples": Sd}
        del pd
    wf = synth.full_frame()
    wfd = synth.full_frame()
    wfd.occ = np.ones_like(wf.occ)
    for tag, wl in (("frame_with_skipping", wf), ("frame_without_skipping", wfd)):
        pf = Pipeline(wl, device="cuda:0", table_dtype=torch.float16, mlp_dtype=K.BF16, rootinit_params=params,
                      device_count=True)
        msf, Sf, _ = time_forward(pf, 3, torch)
        res[tag] = {"ms_per_frame": msf, "posed_samples": Sf, "dtype": "f16/bf16, learned init"}
        del pf
    res["training_speedup"] = res["without_skipping"]["ms_per_step"] / res["with_skipping"]["ms_per_step"]
    res["render_speedup"] = res["frame_without_skipping"]["ms_per_frame"] / res["frame_with_skipping"]["ms_per_frame"]
    res["paper_context"] = "Tab. 3 on RTX 3090: training 3m10s -> 1m47s, rendering ~1 -> ~15 FPS with skipping"
    out["empty_space_skipping"] = res
    # hash grid at T = 2^23 entries per level (FP16, 512 MiB): gathers reach HBM
    S = 1 << 20
    x = torch.rand(3, S, device="cuda:0")
    table = (torch.rand(16, 1 << 23, 2, device="cuda:0") - 0.5).half()
    feat = torch.empty(16 * S * 2, dtype=torch.bfloat16, device="cuda:0")
    gt = torch.empty(16, 1 << 23, 2, device="cuda:0")
    gf = torch.randn(16 * S * 2, device="cuda:0")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for _ in range(2):
        ev[0].record()
        for _ in range(5):
            K.hashgrid_encode(x, None, S, S, table, 16.0, 1.38, (0, 0, 0, 1, 1, 1), feat)
        ev[1].record()
        for _ in range(2):
            K.hashgrid_encode_bwd(gf, x, None, S, S, table, 16.0, 1.38, (0, 0, 0, 1, 1, 1), gt, None, K.OVERWRITE)
        ev[2].record()
    torch.cuda.synchronize()
    fwd_ms = ev[0].elapsed_time(ev[1]) / 5
    bwd_ms = ev[1].elapsed_time(ev[2]) / 2
    fwd_bytes = (16 * 8 * 2 * 2 + 12 + 16 * 2 * 2) * S
    out["hash_stress_2e23"] = {"points": S, "table": "16 x 2^23 x 2 FP16 (512 MiB)", "fwd_ms": fwd_ms,
                               "fwd_algorithmic_GBs": fwd_bytes / (fwd_ms * 1e-3) / 1e9,
                               "fwd_frac_of_hbm_peak": fwd_bytes / (fwd_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                               "bwd_table_ms_incl_zero_fill": bwd_ms}
    del table, gt


def occgrid_leg(torch, np, K, synth, out):
    """Per-pose inference occupancy grid (Sec. 3.3) for the 540^2 frame's
    pose: G = 64 (the paper's lattice) and 128 (the grid the march reads),
    FP32 with the 24-init solve and FP16 table / BF16 MLP; the paper calls
    its cost negligible next to rendering a frame."""
    wf = synth.full_frame()
    dev = "cuda:0"
    B = torch.as_tensor(wf.B, device=dev)
    W = torch.as_tensor(wf.W, device=dev)
    t32 = torch.as_tensor(wf.table, device=dev)
    t16 = t32.half()
    prm = torch.as_tensor(wf.mlp, device=dev)
    Dz, Dy, Dx, nb = wf.W.shape
    L, T, F = t32.shape
    res = {"workload": "540^2 frame pose; lattice of cell centres over the unit box; density threshold 10 "
                       "(the frame's density bias puts valid roots near 55), dilation 1 cell"}
    for G in (64, 128):
        for tag, table, md in (("f32", t32, K.F32), ("f16_bf16", t16, K.BF16)):
            bits = torch.empty(K.occ_words(G), dtype=torch.int32, device=dev)
            ws = torch.empty(K.occgrid_build_workspace_size(G, L, F, md, Dx, Dy, Dz), dtype=torch.uint8, device=dev)

            def run():
                K.occgrid_build(G, wf.occ_aabb, B, W, wf.skin_aabb, wf.hash_aabb, wf.max_iter, wf.tol_stop,
                                wf.tol_valid, table, wf.base_res, wf.growth, prm, md, 10.0, 1, bits, None, ws)

            run()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(5):
                run()
            b.record()
            torch.cuda.synchronize()
            occ = int(sum(bin(v & 0xFFFFFFFF).count("1") for v in bits.cpu().tolist()))
            entry = {"ms": a.elapsed_time(b) / 5, "lattice_points": G ** 3, "occupied_fraction": occ / G ** 3}
            if tag == "f32":
                # training stage: one moving-average update of the shared grid
                # from one jittered point per cell (the jitter drawn on the host)
                jit = torch.as_tensor(np.random.default_rng(G).random((3, G ** 3), dtype=np.float32) * 0.999,
                                      device=dev)
                vals = torch.zeros(G ** 3, device=dev)

                def upd():
                    K.occgrid_update(G, wf.occ_aabb, jit, B, W, wf.skin_aabb, wf.hash_aabb, wf.max_iter, wf.tol_stop,
                                     wf.tol_valid, table, wf.base_res, wf.growth, prm, md, 0.95, 10.0, 1, vals, bits,
                                     ws)

                upd()
                a.record()
                for _ in range(5):
                    upd()
                b.record()
                torch.cuda.synchronize()
                entry["training_update_ms"] = a.elapsed_time(b) / 5
                # density regulariser over the same number of points
                sig = torch.rand(G ** 3, device=dev) * 5.0
                loss = torch.empty(1, device=dev)
                gs = torch.empty(G ** 3, device=dev)
                pts = torch.rand(3, G ** 3, device=dev)
                rws = torch.empty(K.density_reg_workspace_size(G ** 3), dtype=torch.uint8, device=dev)
                K.density_reg(pts, sig, G ** 3, G ** 3, bits, G, wf.occ_aabb, 0.1, loss, gs, rws)
                a.record()
                for _ in range(5):
                    K.density_reg(pts, sig, G ** 3, G ** 3, bits, G, wf.occ_aabb, 0.1, loss, gs, rws)
                b.record()
                torch.cuda.synchronize()
                entry["density_reg_ms"] = a.elapsed_time(b) / 5
                del jit, vals, sig, gs, pts
            res[f"G{G}_{tag}"] = entry
            del ws, bits
    out["occupancy_grid_build"] = res


def training_loop_leg(torch, np, K, synth, out):
    """The training loop (`train.Trainer`): one captured graph per step with
    the loss of Sec. 3.4, every backward and Adam on the table and the MLP;
    the shared occupancy grid's update (Sec. 3.3) timed on its own and
    amortised over k = 16 steps; and a fit of a teacher field's renders."""
    from paper_2212_10550_amd.pipeline import Pipeline
    from paper_2212_10550_amd.train import Trainer
    res = {"workload": "training step (8192 rays of a 540x540 camera, 128^3 occupancy) + Adam (table 16 x 2^19 x 2, "
                       "MLP 6532) per step; occupancy-grid update of a random eighth of the 128^3 cells every k = 16 steps"}
    for tag, kw in (("f32", {}), ("f16_bf16", dict(table_dtype=torch.float16, mlp_dtype=K.BF16))):
        w = synth.train_step()
        tr = Trainer(w, occ_every=16, **kw)
        tr.capture()
        for _ in range(5):
            tr.graph.replay()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        n = 50
        a.record()
        for _ in range(n):
            tr.graph.replay()
        b.record()
        torch.cuda.synchronize()
        step_ms = a.elapsed_time(b) / n
        a.record()
        for _ in range(3):
            tr.occupancy_update()
        b.record()
        torch.cuda.synchronize()
        upd_ms = a.elapsed_time(b) / 3
        res[tag] = {"ms_per_step_with_adam": step_ms, "occupancy_update_ms": upd_ms,
                    "ms_per_step_amortised": step_ms + upd_ms / 16}
        del tr
    # a student fitting a teacher's renders (FP32, no occupancy updates)
    w = synth.train_step()
    teacher = synth.train_step()
    teacher.table = synth.make_hash_table(w.L, 1 << w.log2T, 2, seed=9, scale=0.1).astype(np.float32)
    teacher.mlp = synth.make_mlp(seed=12).astype(np.float32)
    pt = Pipeline(teacher, device="cuda:0")
    pt.forward()
    torch.cuda.synchronize()
    w.target = pt.color.float().cpu().numpy()
    tr = Trainer(w, alpha_gt=pt.opacity.clone(), occ_every=0)
    tr.capture()
    l0 = tr.loss_value()
    t0 = time.perf_counter()
    for _ in range(100):
        tr.step()
    torch.cuda.synchronize()
    res["fit_teacher_100_steps"] = {"loss_start": l0, "loss_end": tr.loss_value(),
                                    "wall_s": time.perf_counter() - t0}
    out["training_loop"] = res


def multiroot_leg(torch, np, K, synth, out):
    """Multi-root aggregation (largest density over every distinct valid
    root) against the lowest-residual root on a folded pose's 540^2 frame
    (FP32, 24 inits, host counts for both)."""
    from paper_2212_10550_amd.multiroot import MaxDensityRenderer
    from paper_2212_10550_amd.pipeline import Pipeline
    w = synth.folded_frame()
    res = {"workload": "540x540 rays of a folded pose (one leg bone turned 120 degrees, skinning softmax "
                       "temperature 100), 128^3 occupancy (~10 %), <=128 samples/ray, FP32, 24-init Broyden"}

    def timed(fn, n=3):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(n):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    p = Pipeline(w, device="cuda:0")
    res["lowest_residual_ms"] = timed(p.forward)
    c0 = p.color.clone()
    del p
    mr = MaxDensityRenderer(w, K_roots=4)
    res["max_density_ms"] = timed(mr.forward)
    nr = mr.n_roots().to(torch.int64)
    res["posed_samples"] = int(mr.S)
    res["samples_with_two_or_more_roots"] = int((nr >= 2).sum().item())
    res["pixel_change_vs_lowest_residual"] = {"mean": float((mr.p.color - c0).abs().mean().item()),
                                              "max": float((mr.p.color - c0).abs().max().item())}
    out["multi_root_aggregation"] = res


def batch_leg(args, params, poses, gen_s, torch, np, synth, out, checks):
    """16 poses of one avatar (occupancy 5-25 %, 270^2 / 540^2 / 1080^2) in
    one HIP graph, FP16 table, BF16 MLP, learned root initialiser with
    multi-init fallback.  The autotuner times the persistent kernel under
    several tile shapes and the staged kernels on 1, 2 and 4 streams, and
    keeps the fastest; the other execution then renders the same batch and
    every pose's outputs are compared bit for bit.  samples_per_s counts the
    posed samples (what the staged kernels evaluate); the persistent kernel
    skips the groups after each ray's termination."""
    from paper_2212_10550_amd.batch import BatchRenderer
    br = BatchRenderer(poses, params)
    tune = br.autotune((1, 2, 4), n=3)
    ms = br.time_ms(5)
    S = br.total_samples
    keys = ("color", "opacity", "n_used", "T_final")
    br.render()
    torch.cuda.synchronize()
    got = [{k: getattr(p, k).clone() for k in keys} for p in br.poses]
    fb = [int(p.n_fallback.item()) for p in br.poses]
    chosen_persistent = br.persistent is not None
    evaluated = sum(int(p.n_evaluated.item()) for p in br.poses) if chosen_persistent else S
    colors = {k: br.poses[k].color.double().cpu().numpy() for k in (0, 4, 2)}
    # the other execution on the same batch
    if br.persistent is not None:
        br.set_streams(2)
        other = "staged kernels, 2 streams"
    else:
        br.set_persistent()
        other = "persistent kernel, default tile shape"
    for p in br.poses:
        for k in keys:
            getattr(p, k).fill_(-1)
    br.render()
    torch.cuda.synchronize()
    same = all(torch.equal(getattr(p, k), g[k]) for p, g in zip(br.poses, got) for k in keys)
    fb_other = [int(p.n_fallback.item()) for p in br.poses]
    if br.persistent is not None:
        evaluated = sum(int(p.n_evaluated.item()) for p in br.poses)
    used = sum(int(p.n_used.sum().item()) for p in br.poses)
    del got
    out["batched_render"] = {
        "workload": "16 poses (seeds 3000-3015), occupancy 5 % + 20 % k/15, resolution 270^2/540^2/1080^2 by k mod 3, "
                    "<=128 samples/ray, termination at T < 1e-4; f16 table, bf16 MLP, learned init + fallback",
        "rays": int(sum(p.R for p in br.poses)), "posed_samples": int(S),
        "ms_per_batch": ms, "samples_per_s": S / (ms * 1e-3), "frames_per_s": 16 / (ms * 1e-3),
        "execution": "one HIP graph replay per batch, the autotuner's fastest schedule",
        "schedule": br_schedule(tune), "autotune_ms": tune,
        "samples_used_by_compositing": used,
        "samples_evaluated_persistent": evaluated,
        "fallback_samples": int(sum(fb)),
        "outputs_equal_other_execution": {"other": other, "pixels_bit_equal": bool(same),
                                           "fallback_samples_other": int(sum(fb_other))},
        "input_generation_s": gen_s,
    }
    checks["batch"] = (poses, colors)
    del br


def br_schedule(tune):
    return min(tune, key=tune.get)


def learned_init_leg(params, torch, np, K, synth, out, n_poses=64):
    """Held-out poses: guided solve (learned start, multi-init fallback) vs
    the 24-init solve on the same points.  Statistics come from one eager
    pass; the time from one HIP graph per method holding every pose's call
    (each pose is 4096 points, far too few to hide launch gaps eagerly)."""
    from paper_2212_10550_amd import rootinit
    test = rootinit.make_dataset(range(2000, 2000 + n_poses), 4096, device="cuda:0")
    w = synth.train_step()
    W_t = torch.as_tensor(w.W, device="cuda:0")
    Dz, Dy, Dx, nb = w.W.shape
    e = lambda *shape, dt=torch.float32: torch.empty(*shape, dtype=dt, device="cuda:0")
    poses = []
    for p in range(n_poses):
        xp = test["xp"][test["pose_index"] == p].T.contiguous()
        S = xp.shape[1]
        poses.append(dict(xp=xp, S=S, B=test["B"][p].contiguous(), pose=test["pose"][p].contiguous(),
                          xg=e(3, S), bg=e(S, dt=torch.int16), sg=e(S, dt=torch.int16),
                          xm=e(3, S), bm=e(S, dt=torch.int16), sm=e(S, dt=torch.int16)))
    gd = rootinit.GuidedDeform(params, w, max(q["S"] for q in poses), device="cuda:0")
    ws = e(K.deform_workspace_size(Dx, Dy, Dz), dt=torch.uint8)

    def guided(q):
        gd.run(q["xp"], q["S"], q["S"], q["pose"], q["B"], W_t, q["xg"], q["bg"], None, q["sg"])

    def multi(q):
        K.snarf_deform(q["xp"], q["S"], q["S"], q["B"], W_t, w.skin_aabb, w.hash_aabb, w.max_iter, w.tol_stop,
                       w.tol_valid, q["xm"], q["bm"], None, q["sm"], ws)

    n = fb = steps_g = steps_m = 0
    errs = []
    for q in poses:
        guided(q)
        multi(q)
        torch.cuda.synchronize()
        fb += int(gd.n_fallback.item())
        ok = (q["bg"] >= 0) & (q["bm"] >= 0)
        errs.append((q["xg"] - q["xm"]).norm(dim=0)[ok].cpu().numpy())
        n += q["S"]
        steps_g += int(q["sg"].to(torch.int64).sum().item())
        steps_m += int(q["sm"].to(torch.int64).sum().item())

    def graph_ms(fn, reps=5, plist=None):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for q in (poses if plist is None else plist):
                fn(q)
        g.replay()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            g.replay()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    ms_g, ms_m = graph_ms(guided), graph_ms(multi)

    # the same calls spread over four streams inside the graph (per-stream
    # buffers), so that concurrent poses hide each other's latency
    n_str = 4
    streams = [torch.cuda.Stream() for _ in range(n_str)]
    gds = [rootinit.GuidedDeform(params, w, max(q["S"] for q in poses), device="cuda:0") for _ in range(n_str)]
    wss = [e(K.deform_workspace_size(Dx, Dy, Dz), dt=torch.uint8) for _ in range(n_str)]

    def spread(fn):
        def run():
            main = torch.cuda.current_stream()
            for st in streams:
                st.wait_stream(main)
            for k, q in enumerate(poses):
                with torch.cuda.stream(streams[k % n_str]):
                    fn(q, k % n_str)
            for st in streams:
                main.wait_stream(st)
        return run

    def guided_s(q, j):
        gds[j].run(q["xp"], q["S"], q["S"], q["pose"], q["B"], W_t, q["xg"], q["bg"], None, q["sg"])

    def multi_s(q, j):
        K.snarf_deform(q["xp"], q["S"], q["S"], q["B"], W_t, w.skin_aabb, w.hash_aabb, w.max_iter, w.tol_stop,
                       w.tol_valid, q["xm"], q["bm"], None, q["sm"], wss[j])

    def graph_ms_run(run, reps=5):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            run()
        g.replay()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            g.replay()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    ms_g4, ms_m4 = graph_ms_run(spread(guided_s)), graph_ms_run(spread(multi_s))

    # 16 held-out poses at 65,536 points each, where the per-pose fixed
    # costs no longer dominate (a frame has ~10^6 samples)
    n_big = 16
    big = rootinit.make_dataset(range(2000, 2000 + n_big), 65536, device="cuda:0")
    bposes = []
    for p in range(n_big):
        xp = big["xp"][big["pose_index"] == p].T.contiguous()
        S = xp.shape[1]
        bposes.append(dict(xp=xp, S=S, B=big["B"][p].contiguous(), pose=big["pose"][p].contiguous(),
                           xg=e(3, S), bg=e(S, dt=torch.int16), sg=e(S, dt=torch.int16),
                           xm=e(3, S), bm=e(S, dt=torch.int16), sm=e(S, dt=torch.int16)))
    del big
    gdb = rootinit.GuidedDeform(params, w, max(q["S"] for q in bposes), device="cuda:0")

    def guided_b(q):
        gdb.run(q["xp"], q["S"], q["S"], q["pose"], q["B"], W_t, q["xg"], q["bg"], None, q["sg"])

    fb_big = 0
    for q in bposes:
        guided_b(q)
        torch.cuda.synchronize()
        fb_big += int(gdb.n_fallback.item())
    n_b = sum(q["S"] for q in bposes)
    ms_gb, ms_mb = graph_ms(guided_b, plist=bposes), graph_ms(multi, plist=bposes)
    err = np.concatenate(errs)
    out["learned_init"] = {
        "held_out": f"{n_poses} poses (seeds 2000-{2000 + n_poses - 1}) x 4096 posed points = {n} samples",
        "fallback_rate": fb / n,
        "broyden_steps_per_sample": {"learned": steps_g / n, "multi_init_24": steps_m / n},
        "root_err_vs_multi_init": {"mean": float(err.mean()), "max": float(err.max())},
        "deform_ms_all_poses": {"learned_bf16_guided": ms_g, "multi_init_24": ms_m},
        "deform_samples_per_s": {"learned_bf16_guided": n / ms_g * 1e3, "multi_init_24": n / ms_m * 1e3},
        "deform_ms_all_poses_4_streams": {"learned_bf16_guided": ms_g4, "multi_init_24": ms_m4},
        "large": {"held_out": f"{n_big} poses (seeds 2000-{2000 + n_big - 1}) x 65536 posed points = {n_b} samples",
                  "fallback_rate": fb_big / max(n_b, 1),
                  "deform_ms_all_poses": {"learned_bf16_guided": ms_gb, "multi_init_24": ms_mb},
                  "speedup": ms_mb / ms_gb},
        "timing": "one HIP graph per method with every pose's call in order (4_streams: the same calls spread "
                  "over four streams inside the graph); each call includes the per-pose blend of the skinning grid "
                  "with the bone transforms (the same work in both methods)",
    }


def mixed_leg(args, params, w, S0, steps_total, nb, loss32, gp32, torch, np, K, Pipeline, out, checks):
    """The training step with the FP16 table and the BF16 MLP (forward and
    backward), FP32 compositing and implicit-function-theorem backward, and
    the learned root initialiser with the 24-init fallback (params None:
    the 24-init solve)."""
    pm = Pipeline(w, device="cuda:0", table_dtype=torch.float16, mlp_dtype=K.BF16, device_count=True,
                  rootinit_params=params)
    dt, Sm, stm = time_train(pm, args.steps, args.warmup, torch, stages=True)
    gpm = pm.grad_params.double().cpu().numpy()
    steps_m = int(pm.steps[:Sm].to(torch.int64).sum().item())
    res = {
        "dtype": "f16 table, bf16 MLP (MFMA, f32 accumulate), f32 deform, compositing and IFT",
        "root_finding": "learned initialiser + one Broyden solve, 24-init fallback" if params is not None
        else "24-init Broyden",
        "value": Sm * args.steps / dt, "unit": "posed samples/s", "ms_per_step": dt * 1e3 / args.steps,
        "stages_ms": {k: round(v, 4) for k, v in stm.items()},
        "stage_roofline": stage_rooflines(stm, S0, w.R, None if params is not None else steps_total, nb, 2, True),
        "broyden_steps_per_step": steps_m,
        "loss_rel_diff_vs_f32": abs(float(pm.loss.item()) - loss32) / abs(loss32),
        "mlp_grad_rel_l2_diff_vs_f32": float(np.linalg.norm(gpm - gp32) / np.linalg.norm(gp32))}
    if params is not None:
        res["fallback_samples"] = int(pm.guided.n_fallback.item())
        res["fallback_rate"] = res["fallback_samples"] / max(Sm, 1)
    out["mixed_training_step"] = res
    checks["mixed"] = (w, float(pm.loss.item()), pm.color.double().cpu().numpy(), gpm)
    del pm


def oracle_checks(checks, out, np, synth):
    """The GPU results of the legs against the FP64 oracle (run on the host
    beside the CPU baseline): pixel errors of the frames and of one batched
    pose per resolution, and the mixed-precision training step's pixel,
    loss and MLP-gradient errors."""
    import oracle
    if "frame" in checks:
        wf, c32, cmx, c24 = checks["frame"]
        sub = np.arange(0, wf.R, 97)
        ref = oracle.forward(synth.ray_subset(wf, sub))["color"]
        e32, emx, e24 = np.abs(c32[sub] - ref), np.abs(cmx[sub] - ref), np.abs(c24[sub] - ref)
        fr = out["frame_540"]
        fr["oracle_rays_compared"] = int(len(sub))
        fr["f32_multi_init"]["pixel_err_vs_oracle"] = {"mean": float(e32.mean()), "max": float(e32.max())}
        fr["f16_bf16_multi_init"]["pixel_err_vs_oracle"] = {
            "mean": float(e24.mean()), "p99.9": float(np.quantile(e24, 0.999)), "max": float(e24.max())}
        fr["f16_bf16_learned_init"]["pixel_err_vs_oracle"] = {
            "mean": float(emx.mean()), "p99.9": float(np.quantile(emx, 0.999)), "max": float(emx.max())}
    if "batch" in checks:
        poses, colors = checks["batch"]
        errs = {}
        for k, got in colors.items():
            w = poses[k]
            idx = np.arange(0, w.R, 1009)
            e = np.abs(got[idx] - oracle.forward(synth.ray_subset(w, idx))["color"])
            errs[f"pose{k}_{int(round(w.R ** 0.5))}sq"] = {"rays": int(len(idx)), "mean": float(e.mean()),
                                                           "max": float(e.max())}
        out["batched_render"]["pixel_err_vs_oracle"] = errs
    if "mixed" in checks:
        w, loss, color, gp = checks["mixed"]
        ref = oracle.train_step(w)  # FP32 master table and MLP, FP64 arithmetic, the oracle's own roots
        e = np.abs(color - ref["color"])
        gref = np.asarray(ref["grad_params"])
        out["mixed_training_step"]["error_vs_fp64_oracle"] = {
            "reference": "the oracle's own training step (its roots, FP32 master values, FP64 arithmetic)",
            "pixel": {"mean": float(e.mean()), "p99.9": float(np.quantile(e, 0.999)), "max": float(e.max())},
            "loss_rel": abs(loss - ref["loss"]) / abs(ref["loss"]),
            "grad_params_norm_rel": float(np.linalg.norm(gp - gref) / np.linalg.norm(gref))}


def reap_children():
    """Wait for (then end) any child process this run started, so that none
    outlives the bench; reports what it found."""
    try:
        import psutil
    except ImportError:
        return []
    kids = psutil.Process().children(recursive=True)
    found = [(k.pid, k.name()) for k in kids]
    for k in kids:
        try:
            k.terminate()
        except psutil.Error:
            pass
    psutil.wait_procs(kids, timeout=5)
    return found


def short_kernel_name(name):
    name = name.strip().strip('"')
    if name.startswith("void "):
        name = name[5:]
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(", 1)[0]


def pmc_summary(fetch_dir, write_dir):
    """Per-kernel FETCH_SIZE / WRITE_SIZE (KiB per dispatch) from two
    rocprofv3 --pmc runs, and the copy-kernel factors; printed as the JSON
    block the profile summary holds."""
    import csv
    import glob

    def load(d, counter):
        per = {}
        for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(fn) as f:
                for row in csv.DictReader(f):
                    if row.get("Counter_Name") != counter:
                        continue
                    key = (fn, row["Dispatch_Id"])
                    name = short_kernel_name(row["Kernel_Name"])
                    v = per.setdefault(key, [name, 0.0])
                    v[1] += float(row["Counter_Value"])
        agg = {}
        for name, v in per.values():
            a = agg.setdefault(name, [0, 0.0])
            a[0] += 1
            a[1] += v
        return {k: (n, tot / n) for k, (n, tot) in agg.items()}

    fe, wr = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    copy = [k for k in fe if "MulFunctor" in k]
    if not copy:
        raise SystemExit("no copy-calibration kernel in the counter runs")
    nbytes = COPY_CAL_FLOATS * 4
    out = {"source_digest": source_digest(),
           "copy_kernel": copy[0], "copy_bytes_each_way": nbytes,
           "copy_factor_fetch": fe[copy[0]][1] * 1024 / nbytes, "copy_factor_write": wr[copy[0]][1] * 1024 / nbytes,
           "kernels": {}}
    for k in sorted(fe):
        if k in copy:
            continue
        out["kernels"][k] = {"dispatches": fe[k][0], "fetch_kib": round(fe[k][1], 1),
                             "write_kib": round(wr.get(k, (0, 0.0))[1], 1)}
    print(json.dumps(out, indent=1))


def counter_table(dirs, kernels=None):
    """Per-kernel mean of every counter found in rocprofv3 --pmc output
    folders (one folder per pass), as a markdown table; kernels: optional
    name filters."""
    import csv
    import glob
    per = {}
    names = set()
    for d in dirs:
        for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(fn) as f:
                for row in csv.DictReader(f):
                    k = short_kernel_name(row["Kernel_Name"])
                    if kernels and not any(q in k for q in kernels):
                        continue
                    c = row["Counter_Name"]
                    names.add(c)
                    key = (fn, row["Dispatch_Id"], c)
                    per.setdefault(k, {}).setdefault(key, 0.0)
                    per[k][key] += float(row["Counter_Value"])
    cols = sorted(names)
    means = {}
    lines = ["## Every counter, per kernel (means over dispatches)", "",
             "| kernel | " + " | ".join(cols) + " |", "|---" * (len(cols) + 1) + "|"]
    for k in sorted(per):
        vals = []
        for c in cols:
            v = [val for (fn, did, cc), val in per[k].items() if cc == c]
            if v:
                means[(k, c)] = sum(v) / len(v)
            vals.append(f"{means[(k, c)]:.4g}" if v else "")
        lines.append(f"| {k} | " + " | ".join(vals) + " |")
    print("\n".join(derived_counters(sorted(per), means) + [""] + lines))


def derived_counters(kernels, means):
    """Derived per-kernel figures from counter means (MI355X: 256 CUs in 8
    XCDs, 4 SIMDs per CU).  GRBM_GUI_ACTIVE is the sum of the 8 XCDs'
    busy-cycle counts (their ratio to a kernel's timed duration at 2.4 GHz
    is 8), so a dispatch lasts GRBM_GUI_ACTIVE / 8 cycles; the texture
    address (TA) and data (TD) units are one per CU, MFMA busy cycles are
    counted per SIMD."""
    def m(k, c):
        return means.get((k, c))

    def ratio(a, b, scale=1.0):
        return None if a is None or not b else a / (b * scale)

    out = ["## Derived per kernel", "",
           "| kernel | cycles per dispatch | TA busy | TD busy | TA cycles per vector-memory read | L1 hit rate | "
           "L2 hit rate | MFMA busy | vector-memory reads per wave | VALU per wave |",
           "|---|---|---|---|---|---|---|---|---|---|"]
    for k in kernels:
        g = m(k, "GRBM_GUI_ACTIVE")
        cyc = g / 8 if g else None
        hit, miss = m(k, "TCC_HIT_sum"), m(k, "TCC_MISS_sum")
        acc, req = m(k, "TCP_TOTAL_CACHE_ACCESSES_sum"), m(k, "TCP_TCC_READ_REQ_sum")
        waves = m(k, "SQ_WAVES")
        row = [cyc, ratio(m(k, "TA_TA_BUSY_sum"), cyc, 256), ratio(m(k, "TD_TD_BUSY_sum"), cyc, 256),
               ratio(m(k, "TA_TA_BUSY_sum"), m(k, "SQ_INSTS_VMEM_RD")),
               None if not acc or req is None else 1.0 - req / acc,
               None if hit is None or miss is None or hit + miss == 0 else hit / (hit + miss),
               ratio(m(k, "SQ_VALU_MFMA_BUSY_CYCLES"), cyc, 1024),
               ratio(m(k, "SQ_INSTS_VMEM_RD"), waves), ratio(m(k, "SQ_INSTS_VALU"), waves)]
        fmt = ["{:.4g}", "{:.2f}", "{:.2f}", "{:.1f}", "{:.3f}", "{:.3f}", "{:.3f}", "{:.1f}", "{:.0f}"]
        out.append(f"| {k} | " + " | ".join("" if v is None else f.format(v) for v, f in zip(row, fmt)) + " |")
    return out


def kernel_stats(trace_dir, replay_of=None):
    """Markdown summary of a rocprofv3 --kernel-trace --stats folder: every
    kernel's calls and durations (from its kernel_stats.csv) and, with
    replay_of, the kernels of one launch sequence that starts with a kernel
    of that name (one graph replay of a step or frame) with grid, start and
    duration, from its kernel_trace.csv."""
    import csv
    import glob
    out = []
    if replay_of:
        for fn in glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True):
            with open(fn) as f:
                rows = [(short_kernel_name(r["Kernel_Name"]), int(r["Grid_Size_X"]) if "Grid_Size_X" in r else
                         int(r.get("Grid_Size", 0)), int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
                        for r in csv.DictReader(f)]
            rows.sort(key=lambda t: t[2])
            starts = [i for i, r in enumerate(rows) if r[0].startswith(replay_of)] + [len(rows)]
            seqs = [rows[a:b] for a, b in zip(starts[:-1], starts[1:])]
            if not seqs:
                continue
            # the sequences with the most distinct kernels (whole steps or
            # frames), and of those the one with the shortest span (a graph
            # replay rather than an eagerly launched one)
            most = max(len({k for k, *_ in q}) for q in seqs)
            full = [q for q in seqs if len({k for k, *_ in q}) == most]
            seq = min(full, key=lambda q: max(e for *_, e in q) - q[0][2])
            # cut at the first idle gap over 50 us (the launches that follow
            # belong to other work)
            for j in range(1, len(seq)):
                if seq[j][2] - max(e for *_, e in seq[:j]) > 50_000:
                    seq = seq[:j]
                    break
            t0 = seq[0][2]
            out += [f"## One launch sequence starting with {replay_of} (the tightest of the {len(full)} with every "
                    "kernel)", "", "| kernel | grid (work-items) | start us | duration us |", "|---|---|---|---|"]
            tot = 0.0
            for name, grid, st, en in seq:
                tot += (en - st) / 1e3
                out.append(f"| {name} | {grid} | {(st - t0) / 1e3:.1f} | {(en - st) / 1e3:.1f} |")
            span = (max(e for _, _, _, e in seq) - t0) / 1e3
            out += ["", f"Kernel time {tot:.1f} us over a {span:.1f} us span from the first kernel's start to the "
                    "last one's end.", ""]
            break
    for fn in glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True):
        with open(fn) as f:
            rows = list(csv.DictReader(f))
        out += ["## All kernels of the run", "", "| kernel | calls | avg us | min us | max us | % of GPU time |",
                "|---|---|---|---|---|---|"]
        for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
            out.append(f"| {short_kernel_name(r['Name'])[:70]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                       f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
        break
    print("\n".join(out))


COPY_CAL_FLOATS = 256 << 20  # 1 GiB read and written (4x the 256 MB Infinity Cache)


def copy_calibration(torch):
    """A plain elementwise copy of known size (read 1 GiB, write 1 GiB),
    for scaling the HBM byte counters."""
    src = torch.empty(COPY_CAL_FLOATS, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-frame", action="store_true")
    ap.add_argument("--init-poses", type=int, default=256)
    ap.add_argument("--init-epochs", type=int, default=20)
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP16/BF16 training-step leg")
    ap.add_argument("--only", default=None,
                    help="comma-separated subset of the frame-side legs to run (frame, init, occgrid, loop, multiroot, "
                         "extra, batch), e.g. for a profiler run; the training step always runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain copy kernel of known size (for scaling rocprofv3 byte counters)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc output folders (no GPU needed) and exit")
    ap.add_argument("--counter-table", nargs="+", metavar="PMC_DIR",
                    help="per-kernel mean of every counter in rocprofv3 --pmc folders (no GPU needed), then exit")
    ap.add_argument("--kernels", default=None, help="with --counter-table: comma-separated kernel-name filters")
    ap.add_argument("--kernel-stats", metavar="TRACE_DIR",
                    help="summarise a rocprofv3 --kernel-trace --stats folder (no GPU needed), then exit")
    ap.add_argument("--replay-of", default=None,
                    help="with --kernel-stats: list one launch sequence starting with this kernel name")
    args = ap.parse_args()
    if args.kernel_stats:
        kernel_stats(args.kernel_stats, args.replay_of)
        return
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.counter_table:
        counter_table(args.counter_table, args.kernels.split(",") if args.kernels else None)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this path runs on one GPU; rays, samples and poses are independent, so "
                                   "more GPUs would each take a share, but multi-GPU runs are not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np

    from paper_2212_10550_amd import synth

    # the batched render's occupancy grids are built in a process pool, which
    # forks before this process has loaded anything that touches the GPU
    poses, gen_s = None, 0.0
    if not args.no_frame and (args.only is None or "batch" in args.only.split(",")):
        log("building the 16 batched-render poses")
        t0 = time.perf_counter()
        poses = synth.batch_poses(16, workers=min(16, os.cpu_count() or 1))
        gen_s = time.perf_counter() - t0

    import torch

    from paper_2212_10550_amd import lib as K
    from paper_2212_10550_amd.pipeline import Pipeline

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    log("building inputs")
    w = synth.train_step()
    # host-count path (one host round trip per step for the sample count),
    # reported beside the timed path for context
    ph = Pipeline(w, device="cuda:0")
    log("warmup")
    for _ in range(args.warmup):
        ph.train_step()
    torch.cuda.synchronize()
    S0 = ph.S
    steps_total = int(ph.steps[:S0].to(torch.int64).sum().item())
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ph.train_step()
    torch.cuda.synchronize()
    host_count_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    loss32 = float(ph.loss.item())
    gp32 = ph.grad_params.double().cpu().numpy()
    del ph
    # timed path: device-resident counts, the step replayed as one HIP graph
    log(f"S={S0}; timing {args.steps} steps")
    p = Pipeline(w, device="cuda:0", device_count=True)
    dt, S1, stage_ms = time_train(p, args.steps, args.warmup, torch, stages=True)
    if S1 != S0:
        raise RuntimeError(f"sample count differs between paths: {S1} vs {S0}")
    ms_step = dt * 1e3 / args.steps
    value = S0 * args.steps / dt
    nb = w.B.shape[0]
    out = {
        "metric": "posed samples/s (deform+encode+MLP+composite, fwd+bwd); ms per 540² frame",
        "value": value, "unit": "posed samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded 24-bone skeleton, pose, skinning grid, occupancy, camera rays, hash table, MLP)",
        "config": {"workload": "training step: 8192 rays of a 540x540 camera, <=128 samples/ray, 128^3 occupancy "
                               "(~15%), skinning grid 64x64x32x24, hash 16 levels x 2^19 x 2 FP32, MLP 32-64-64-4, "
                               "24-init Broyden (<=10 steps), L2 loss, every backward pass incl. the IFT",
                   "rays": w.R, "posed_samples_per_step": S0, "broyden_steps_per_step": steps_total},
        "execution": "device-resident sample counts; each step one HIP graph replay",
        "host_count_eager_ms_per_step": host_count_ms,
        "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()},
    }
    blend, solve = deform_kernel_ms(torch, K, p)
    out["deform_kernels_ms"] = {"blend_kernel": round(blend, 4), "solve_kernel": round(solve, 4),
                                "timing": "20 calls captured back to back in one graph, replayed 10 times"}
    out["roofline"], out["stage_roofline"] = roofline(stage_ms, solve, S0, w.R, steps_total, nb)
    if abs(float(p.loss.item()) - loss32) > 1e-6 * abs(loss32):
        raise RuntimeError("graph-replayed step and host-count step disagree on the loss")
    del p
    checks = {}
    params = None
    if not args.no_frame:
        log("fitting the root initialiser on solver roots")
        params, fit_note = fit_initialiser(args, torch)
    # the same step with FP16 hash features, the BF16 MLP and the learned
    # initialiser (the 24-init solve when it is not fitted)
    if not args.no_mixed:
        log("FP16/BF16 training step")
        mixed_leg(args, params, w, S0, steps_total, nb, loss32, gp32, torch, np, K, Pipeline, out, checks)
    if args.copy_calibration:
        copy_calibration(torch)
    if not args.no_frame:
        legs = set(args.only.split(",")) if args.only else None
        run = lambda name: legs is None or name in legs
        if run("frame"):
            log("540x540 frame")
            frame_leg(args, params, fit_note, torch, np, K, synth, Pipeline, out, checks)
        if run("init"):
            log("learned initialiser on held-out poses")
            learned_init_leg(params, torch, np, K, synth, out)
        if run("occgrid"):
            log("occupancy grid construction")
            occgrid_leg(torch, np, K, synth, out)
        if run("loop"):
            log("training loop with Adam and occupancy updates")
            training_loop_leg(torch, np, K, synth, out)
        if run("multiroot"):
            log("multi-root aggregation on a folded pose")
            multiroot_leg(torch, np, K, synth, out)
        if run("extra"):
            log("tiny forward, skipping on/off, hash stress")
            extra_legs(args, params, torch, np, K, synth, Pipeline, out)
        if run("batch") and poses is not None:
            log("batched render of 16 poses")
            batch_leg(args, params, poses, gen_s, torch, np, synth, out, checks)
    if not args.no_cpu_baseline:
        log("oracle on the host")
        out["cpu_baseline"] = cpu_baseline(w)
        log("GPU results against the oracle")
        oracle_checks(checks, out, np, synth)
    left = reap_children()
    if left:
        log(f"child processes ended at exit: {left}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
