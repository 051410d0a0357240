#!/usr/bin/env python3
"""Benchmark of the deform-and-query path on one MI355X.

Step (the timed unit of ``value``): one training step of the path on the
8192-ray workload -- march through the 128^3 occupancy grid, 24-init Broyden
deform, hash encode, MLP, composite, L2 loss, and every backward pass
(composite, MLP, encode, implicit-function-theorem deform), all in the
library's HIP kernels, FP32.  value = posed samples (kept by the occupancy
skip) per second over the K timed steps, inputs resident in HBM.

Extra keys of the one JSON line:
  stages_ms     per-stage time of the step (HIP events on the launch stream)
  roofline      the dominant stage's kernel against its roofline
  frame_540     ms per 540x540 frame: FP32 multi-init vs FP16 table + BF16
                MLP + learned root initialiser, and their pixel errors
  learned_init  the initialiser on held-out poses: steps, fallback rate,
                root error, deform time vs multi-init
  cpu_baseline  the FP64 oracle timed on the host cores

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-frame] [--init-poses P]
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

# Algorithmic work per unit (counted from the kernels)
DEFORM_FLOP_PER_INIT = 670.0   # start point, Jacobian, inverse
DEFORM_FLOP_PER_STEP = 380.0   # one Broyden step (residual 290 + update 90)
HASH_FWD_BYTES = 16 * 8 * 2 * 4 + 12 + 16 * 2 * 4       # FP32 gathers + x + features
HASH_BWD_BYTES = 2 * 16 * 8 * 2 * 4 + 12 + 16 * 2 * 4   # read-modify-write of the touched entries
IFT_BYTES_PER_SAMPLE = 2 * 8 * 12 * 4 + 24 + 12 + 8 * 24 * 4  # moment RMW + x, v, u + skinning rows
MLP_BWD_FLOP = 25600.0 + 12800.0  # backward plus the recomputed forward


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(w, budget_s=10.0):
    """The FP64 oracle's training step on the same workload, repeated until
    about budget_s seconds of host time have passed (at least once), on the
    host's cores; posed samples/s over those runs."""
    import oracle
    oracle.lib()
    runs, samples = 0, 0
    t0 = time.perf_counter()
    while True:
        ref = oracle.train_step(w)
        samples += ref["march"]["xs"].shape[0]
        runs += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s or dt * (runs + 1) / runs > 3 * budget_s:
            break
    return {"value": samples / dt, "unit": "posed samples/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"the full training step ({w.R} rays, {samples // runs} posed samples), forward + every "
                      f"backward, {runs} run(s) in {dt:.1f} s"}


def roofline(stage_ms, S, steps_total, nb):
    dom = max(stage_ms, key=stage_ms.get)
    t = stage_ms[dom] * 1e-3
    if dom == "deform":
        work = DEFORM_FLOP_PER_INIT * nb * S + DEFORM_FLOP_PER_STEP * steps_total
        ach = work / t / 1e12
        return {"kernel": "snarf_deform (solve_kernel + blend_kernel)", "bound": "alu", "achieved": ach,
                "peak": PEAK_FP32_VEC_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_FP32_VEC_TFLOPS,
                "traffic": None, "work_per_launch": work, "work_unit": "flop"}
    if dom == "mlp_bwd":
        work = MLP_BWD_FLOP * S
        ach = work / t / 1e12
        return {"kernel": "mlp_bwd_f32", "bound": "mfma", "achieved": ach, "peak": PEAK_FP32_MFMA_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / PEAK_FP32_MFMA_TFLOPS, "traffic": None, "work_per_launch": work,
                "work_unit": "flop"}
    per = {"hash_bwd": HASH_BWD_BYTES, "hash_fwd": HASH_FWD_BYTES, "deform_bwd": IFT_BYTES_PER_SAMPLE}.get(dom)
    kern = {"hash_bwd": "table_grad_kernel + encode_bwd_kernel", "hash_fwd": "encode_kernel",
            "deform_bwd": "ift_v/ift_q/ift_contract kernels"}.get(dom, dom)
    if per is None:
        return {"kernel": dom, "bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": None,
                "traffic": None}
    work = per * S
    ach = work / t / 1e9
    return {"kernel": kern, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": ach / PEAK_HBM_GBS, "traffic": None, "work_per_launch": work, "work_unit": "bytes"}


def time_forward(p, n, torch):
    for _ in range(2):
        p.forward()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        S = p.forward()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / n, S


def frame_leg(args, torch, np, K, synth, Pipeline, out):
    import oracle
    from paper_2212_10550_amd import rootinit
    wf = synth.full_frame()
    log("fitting the root initialiser on solver roots")
    t0 = time.perf_counter()
    data = rootinit.make_dataset(range(1000, 1000 + args.init_poses), 4096, device="cuda:0")
    params = rootinit.fit(data, epochs=args.init_epochs)
    fit_s = time.perf_counter() - t0
    del data
    # FP32 multi-init reference frame
    p32 = Pipeline(wf, device="cuda:0")
    ms32, S = time_forward(p32, 5, torch)
    c32 = p32.color.double().cpu().numpy()
    steps32 = int(p32.steps[:S].to(torch.int64).sum().item())
    del p32
    # FP16 table + BF16 MLP + learned initialiser
    pmx = Pipeline(wf, device="cuda:0", table_dtype=torch.float16, mlp_dtype=K.BF16, rootinit_params=params)
    msmx, Smx = time_forward(pmx, 5, torch)
    cmx = pmx.color.double().cpu().numpy()
    stepsmx = int(pmx.steps[:Smx].to(torch.int64).sum().item())
    fb = int(pmx.guided.n_fallback.item())
    used = int(pmx.n_used.to(torch.int64).sum().item())
    del pmx
    # pixel error on a seeded subset of rays against the FP64 oracle
    sub = np.arange(0, wf.R, 97)
    ref = oracle.forward(synth.ray_subset(wf, sub))["color"]
    e32 = np.abs(c32[sub] - ref)
    emx = np.abs(cmx[sub] - ref)
    dmx = np.abs(cmx - c32)
    out["frame_540"] = {
        "workload": "540x540 rays, 128^3 occupancy (~10%), <=128 samples/ray, early termination at T < 1e-4, "
                    "24-bone pose, hash T=2^19",
        "posed_samples": S, "samples_after_termination": used,
        "f32_multi_init": {"ms_per_frame": ms32, "fps": 1e3 / ms32, "broyden_steps": steps32,
                           "pixel_err_vs_oracle": {"mean": float(e32.mean()), "max": float(e32.max())}},
        "f16_bf16_learned_init": {"ms_per_frame": msmx, "fps": 1e3 / msmx, "broyden_steps": stepsmx,
                                  "fallback_samples": fb,
                                  "pixel_err_vs_oracle": {"mean": float(emx.mean()),
                                                          "p99.9": float(np.quantile(emx, 0.999)),
                                                          "max": float(emx.max())},
                                  "pixel_diff_vs_f32_multi_init": {"mean": float(dmx.mean()),
                                                                   "max": float(dmx.max())}},
        "speedup_learned_mixed_vs_f32_multi": ms32 / msmx,
        "oracle_rays_compared": int(len(sub)),
        "initialiser_fit": f"{args.init_poses} poses x 4096 points, {args.init_epochs} epochs, {fit_s:.1f} s",
        "paper_context": "15 FPS at 540x540 on one RTX 3090 (Sec. 4.2, Tab. 3)",
    }
    return params


def extra_legs(args, params, torch, np, K, synth, Pipeline, out):
    """Tiny FP32 forward; empty-space skipping on/off (the synthetic analogue
    of Tab. 3); hash encode at T = 2^23 (FP16 table, 512 MiB)."""
    # tiny forward: 1024 rays x 64 samples, no occupancy grid, FP32
    wt = synth.tiny_forward()
    pt = Pipeline(wt, device="cuda:0")
    ms, S = time_forward(pt, 20, torch)
    out["tiny_forward_f32"] = {"workload": "1024 front-face rays x 64 samples, 32^3x24 skinning grid, hash 2^14 FP32",
                               "ms": ms, "posed_samples": S, "samples_per_s": S / (ms * 1e-3)}
    del pt
    # empty-space skipping off: every cell occupied (Sec. 3.3, Tab. 3)
    w = synth.train_step()
    wd = synth.train_step()
    wd.occ = np.ones_like(w.occ)
    res = {}
    for tag, wl in (("with_skipping", w), ("without_skipping", wd)):
        pd = Pipeline(wl, device="cuda:0")
        for _ in range(2):
            pd.train_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            Sd = pd.train_step()
        torch.cuda.synchronize()
        res[tag] = {"ms_per_step": (time.perf_counter() - t0) * 1e3 / 5, "posed_samples": Sd}
        del pd
    wf = synth.full_frame()
    wfd = synth.full_frame()
    wfd.occ = np.ones_like(wf.occ)
    for tag, wl in (("frame_with_skipping", wf), ("frame_without_skipping", wfd)):
        pf = Pipeline(wl, device="cuda:0", table_dtype=torch.float16, mlp_dtype=K.BF16, rootinit_params=params)
        msf, Sf = time_forward(pf, 3, torch)
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


def learned_init_leg(params, torch, np, K, synth, out):
    """Held-out poses: guided solve vs 24-init solve on the same points."""
    from paper_2212_10550_amd import rootinit
    test = rootinit.make_dataset(range(2000, 2016), 4096, device="cuda:0")
    w = synth.train_step()
    W_t = torch.as_tensor(w.W, device="cuda:0")
    Dz, Dy, Dx, nb = w.W.shape
    tot = dict(n=0, fb=0, steps_g=0, steps_m=0, t_g=0.0, t_m=0.0, err=[])
    for p in range(16):
        sel = test["pose_index"] == p
        xp = test["xp"][sel].T.contiguous()
        S = xp.shape[1]
        B = test["B"][p].contiguous()
        gd = rootinit.GuidedDeform(params, w, S, device="cuda:0")
        xg = torch.empty(3, S, device="cuda:0")
        bg = torch.empty(S, dtype=torch.int16, device="cuda:0")
        sg = torch.empty(S, dtype=torch.int16, device="cuda:0")
        xm = torch.empty(3, S, device="cuda:0")
        bm = torch.empty(S, dtype=torch.int16, device="cuda:0")
        sm = torch.empty(S, dtype=torch.int16, device="cuda:0")
        ws = torch.empty(K.deform_workspace_size(Dx, Dy, Dz), dtype=torch.uint8, device="cuda:0")
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        for rep in range(2):
            ev[0].record()
            gd.run(xp, S, S, test["pose"][p].contiguous(), B, W_t, xg, bg, None, sg)
            ev[1].record()
            K.snarf_deform(xp, S, S, B, W_t, w.skin_aabb, w.hash_aabb, w.max_iter, w.tol_stop, w.tol_valid, xm, bm,
                           None, sm, ws)
            ev[2].record()
        torch.cuda.synchronize()
        ok = (bg >= 0) & (bm >= 0)
        tot["err"].append((xg - xm).norm(dim=0)[ok].cpu().numpy())
        tot["n"] += S
        tot["fb"] += int(gd.n_fallback.item())
        tot["steps_g"] += int(sg.to(torch.int64).sum().item())
        tot["steps_m"] += int(sm.to(torch.int64).sum().item())
        tot["t_g"] += ev[0].elapsed_time(ev[1])
        tot["t_m"] += ev[1].elapsed_time(ev[2])
    err = np.concatenate(tot["err"])
    out["learned_init"] = {
        "held_out": f"16 poses (seeds 2000-2015) x 4096 posed points = {tot['n']} samples",
        "fallback_rate": tot["fb"] / tot["n"],
        "broyden_steps_per_sample": {"learned": tot["steps_g"] / tot["n"], "multi_init_24": tot["steps_m"] / tot["n"]},
        "root_err_vs_multi_init": {"mean": float(err.mean()), "max": float(err.max())},
        "deform_ms": {"learned_bf16_guided": tot["t_g"], "multi_init_24": tot["t_m"]},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-frame", action="store_true")
    ap.add_argument("--init-poses", type=int, default=256)
    ap.add_argument("--init-epochs", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this path runs on one GPU; multi-GPU runs are not part of this build "
                                   "(see the sharding notes in DESIGN.md)", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2212_10550_amd import lib as K
    from paper_2212_10550_amd import synth
    from paper_2212_10550_amd.pipeline import Pipeline, StageTimer

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    log("building inputs")
    w = synth.train_step()
    p = Pipeline(w, device="cuda:0")
    log("warmup")
    for _ in range(args.warmup):
        p.train_step()
    torch.cuda.synchronize()
    S0 = p.S
    steps_total = int(p.steps[:S0].to(torch.int64).sum().item())
    log(f"S={S0}; timing {args.steps} steps")
    timer = StageTimer()
    p.timer = timer
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    samples = 0
    for _ in range(args.steps):
        samples += p.train_step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    p.timer = None
    ms_step = (t1 - t0) * 1e3 / args.steps
    stage_ms = {k: v / args.steps for k, v in timer.totals_ms().items()}
    value = samples / (t1 - t0)
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
        "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "roofline": roofline(stage_ms, S0, steps_total, nb),
        "hash_fwd_algorithmic_GBs": HASH_FWD_BYTES * S0 / (stage_ms["hash_fwd"] * 1e-3) / 1e9,
    }
    loss32 = float(p.loss.item())
    gp32 = p.grad_params.double().cpu().numpy()
    del p
    # the same step with FP16 hash features and the BF16 MLP (forward and backward)
    pm = Pipeline(w, device="cuda:0", table_dtype=torch.float16, mlp_dtype=K.BF16)
    for _ in range(args.warmup):
        pm.train_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sm = 0
    for _ in range(args.steps):
        sm += pm.train_step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gpm = pm.grad_params.double().cpu().numpy()
    out["mixed_training_step"] = {
        "dtype": "f16 table, bf16 MLP (MFMA, f32 accumulate), f32 deform and compositing",
        "value": sm / (t1 - t0), "unit": "posed samples/s", "ms_per_step": (t1 - t0) * 1e3 / args.steps,
        "loss_rel_diff_vs_f32": abs(float(pm.loss.item()) - loss32) / abs(loss32),
        "mlp_grad_rel_l2_diff_vs_f32": float(np.linalg.norm(gpm - gp32) / np.linalg.norm(gp32))}
    del pm
    if not args.no_frame:
        log("540x540 frame")
        params = frame_leg(args, torch, np, K, synth, Pipeline, out)
        log("learned initialiser on held-out poses")
        learned_init_leg(params, torch, np, K, synth, out)
        log("tiny forward, skipping on/off, hash stress")
        extra_legs(args, params, torch, np, K, synth, Pipeline, out)
    if not args.no_cpu_baseline:
        log("oracle on the host")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
