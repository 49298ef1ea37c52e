#!/usr/bin/env python3
"""Throughput of the Elfpie iteration on one MI355X.

Workload: the paper-shaped single field of view -- FP32, 512 x 512 high-resolution
spectrum, 15 x 15 LEDs (K = 225), 128 x 128 low-resolution images, Zernike-aberrated
pupil, LED position jitter, vignetting, Poisson / Gaussian / salt-and-pepper noise --
built from seeded synthetic inputs.  One step = one full iteration (all LEDs, object
branch, spectrum and pupil updates, loss).  The measured stack is simulated on the
GPU with the library's own forward model from the seeded ground truth; the CPU
baseline leg re-simulates it with the oracle.

Prints one JSON line (see the keys below).  Only one GPU is used: --gpus above 1 is
refused.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LED sub-image updates/sec (K×iters/s) at K=225, 128² low-res; % HBM roofline"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2209_14671_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def byte_model(K, S, B, A, elem=4):
    """Algorithmic HBM bytes: per-LED branch and whole iteration, for reals of `elem`
    bytes (complex 2 elem; the Eq. 19 second moment is 8 bytes in both precisions).
    FP32: per LED 24 S + 4 B (window of psi on the support, image, C and D) plus P once;
    per iteration 40 S + 4 B per LED (C and D re-read) plus 112 A (object transforms,
    Hessian, update)."""
    c, r = 2 * elem, elem
    led_kernel = K * (3 * c * S + r * B) + c * S
    iteration = K * (5 * c * S + r * B) + (11 * c + 16 + 2 * r) * A
    return led_kernel, iteration


WORKLOADS = {
    1: ("f64", "config 1, FP64: 128x128 high-res, 5x5 LEDs (K=25), 32x32 low-res, circular pupil, noise-free"),
    2: ("f32", "single FOV, FP32: 512x512 high-res, 15x15 LEDs (K=225), 128x128 low-res, "
               "Zernike pupil, noise + salt-and-pepper + vignetting + LED jitter"),
    3: ("f32", "64 independent FOV tiles, FP32: low-res 64/96/128/192/256 (high-res 4x), K 49/121/169/225 "
               "(centred LED sub-grids), circular pupil, noise-free; one graph replay per iteration of all tiles"),
    4: ("f32", "FP32: 256x256 high-res, 11x11 LEDs (K=121), 64x64 low-res, circular pupil, noise-free"),
    5: ("f32", "FP32: 1024x1024 high-res, 15x15 LEDs (K=225), 256x256 low-res, circular pupil, noise-free"),
}
LED_KERNEL = {1: "k_led<double,32>", 2: "k_led<float,128>", 3: "whole batch iteration", 4: "k_led<float,64>",
              5: "k_big_rows_inv + k_big_cols + k_big_rows_fwd (256^2 tile through HBM)"}


def measured_traffic(src_hash):
    """HBM traffic of the per-LED kernel from the committed rocprofv3 counter summary,
    valid only while the kernel sources still hash to the value recorded there."""
    path = os.path.join(ROOT, "profiles", "k_led_config2_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != src_hash:
        return None
    return d.get("traffic_bytes_per_launch")


def copy_bandwidth(dev, mib, reps=3):
    """Read + write GB/s of a plain device-to-device copy of `mib` MiB (larger than the
    256 MB last-level cache at the default size), HIP-event timed on the current stream."""
    import torch
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    gbs = 2 * (n * 4) * reps / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del src, dst
    return round(gbs, 1)


def autograd_bench(args, dev):
    """Forward + backward of the differentiable loss (FP32, 256^2, K=121, 64^2): the
    backward recomputing the per-LED fields against one reading fields the forward kept."""
    import torch

    import synth
    import paper_2209_14671_amd as E
    case = synth.config_case(4)
    o = case.optics
    meas = simulated_stack(case, dev)
    plan = E.Plan(E.problem_from_optics(o, case.led_k, precision=E.F32, flags=E.PUPIL_SUPPORT), device=dev)
    st = plan.init_state(meas)
    res = {}
    for store in (False, True):
        def once():
            psi = st.psi.clone().requires_grad_(True)
            P = st.P.clone().requires_grad_(True)
            E.elfpie_loss(psi, P, plan, meas, store_fields=store).backward()
        for _ in range(args.warmup):
            once()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(args.steps):
            once()
        ev1.record()
        torch.cuda.synchronize()
        res["stored" if store else "recompute"] = ev0.elapsed_time(ev1) / args.steps
    K, B = plan.K, plan.n_lo ** 2
    print(json.dumps({
        "metric": "forward + backward of the Elfpie loss (autograd), recomputed vs stored per-LED fields",
        "unit": "ms", "higher_is_better": False, "steps": args.steps, "warmup": args.warmup, "dtype": "f32",
        "data": "synthetic", "config": {"workload": "differentiable loss, FP32: 256x256 high-res, 11x11 LEDs "
                                                    "(K=121), 64x64 low-res", "K": K, "n_lo": plan.n_lo,
                                        "n_hi": plan.n_hi},
        "ms_recompute": round(res["recompute"], 4), "ms_stored": round(res["stored"], 4),
        "stored_fields_bytes": K * B * 8}), flush=True)


def simulated_stack(case, dev):
    """The measured stack of a synthetic case, simulated with the library's forward model
    at the true (jittered) LED positions, then degraded on the host."""
    import torch

    import synth
    import paper_2209_14671_amd as E
    o = case.optics
    sim = E.Plan(E.problem_from_optics(o, case.led_k_true, precision=E.F32), device=dev)
    psi_true = sim.spectrum_from_object(torch.from_numpy(case.obj).to(torch.complex64).to(dev))
    clean = sim.forward(psi_true, torch.from_numpy(case.pupil).to(torch.complex64).to(dev), intens=True)["intens"]
    meas = synth.degrade(clean.cpu().numpy().astype(np.float64), case.degradation, case.noise_seed)
    sim.close()
    return torch.from_numpy(meas).to(torch.float32).to(dev)


def optimizer_bench(args, dev):
    """Sec. 6.2 / Fig. 13 on synthetic data: the loss after 0, 10, 20, 50 and 100 iterations
    of Eq. 19 and of NAdam, AdaBelief and SGD on the same stack, with the time per
    iteration.  Steps: lr 1e-2 for the moment methods (the same parameters); SGD, whose
    step has the units of the gradient, at three sizes.  A diverged loss is null."""
    import torch

    import synth
    import paper_2209_14671_amd as E
    case = synth.config_case(2)
    meas = simulated_stack(case, dev)
    flags = E.LEARN_PUPIL | E.PUPIL_SUPPORT | E.PUPIL_FILTER
    rows = {}
    for name, opt, lr in (("eq19", E.OPT_ELFPIE, 1e-2), ("nadam", E.OPT_NADAM, 1e-2),
                          ("adabelief", E.OPT_ADABELIEF, 1e-2), ("sgd_1e-4", E.OPT_SGD, 1e-4),
                          ("sgd_1e-3", E.OPT_SGD, 1e-3), ("sgd_1e-2", E.OPT_SGD, 1e-2)):
        plan = E.Plan(E.problem_from_optics(case.optics, case.led_k, precision=E.F32, flags=flags, optimizer=opt,
                                            lr=lr), device=dev)
        st = plan.init_state(meas)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        h = plan.run(st, meas, 100)
        ev1.record()
        torch.cuda.synchronize()
        L = h[:, 3].cpu().numpy()
        pick = {str(i): L[i] for i in (0, 10, 20, 50)} | {"100": L[-1]}
        rows[name] = {"lr": lr, "us_per_iter": round(ev0.elapsed_time(ev1) * 10.0, 2),
                      "loss": {k: (float(v) if np.isfinite(v) else None) for k, v in pick.items()}}
        log(f"{name}: loss {L[0]:.4e} -> {L[-1]:.4e}")
        plan.close()
    print(json.dumps({"metric": "loss after n iterations per update rule (Sec. 6.2 comparison)", "data": "synthetic",
                      "dtype": "f32", "config": {"workload": "single FOV, FP32: 512x512 high-res, 15x15 LEDs (K=225), "
                                                             "128x128 low-res, degraded stack"},
                      "optimizers": rows}), flush=True)


SWEEP_NOISES = ("gaussian", "snp", "poisson")
# Table 1's dark-field noise levels (%), by noise type, then c in (0.25, 0.5, 0.75), then level.
TABLE1_NL = {
    "gaussian": ((20.49, 99.18, 800.10, 7669.71), (31.02, 102.59, 796.48, 7662.03), (41.98, 107.06, 793.00, 7656.55)),
    "snp": ((989.06, 9583.58, 47757.62, 95453.10), (971.87, 9648.64, 47799.04, 95697.25),
            (972.56, 9543.86, 47771.76, 95571.99)),
    "poisson": ((36.37, 66.13, 81.07, 94.23), (41.78, 67.58, 80.57, 92.12), (49.39, 70.74, 81.67, 91.36)),
}


def sweep_bench(args, dev, iters=100):
    """Sec. 4.2's simulation study on synthetic stacks of the paper's shape (512^2 / K=225 /
    128^2, FP32, pupil learning on), every case reconstructed together in ONE batch (one
    graph replay per iteration of all of them): LED shift d in {0, 0.5, 2} mm (simulation
    only), illumination strength c in {0.25, 0.5, 0.75} and Table 1's four levels of
    Gaussian, salt-and-pepper and Poisson noise (Eq. 20), `reps` seeds per cell (an object
    and an LED shift per seed, shared by the cells).  Per cell: the dark-field noise level
    (Eq. 21) beside Table 1's, and the LSNR (Eq. 22) of abs(O) and angle(O) after `iters`
    iterations, averaged over seeds.  Also the batch's time per iteration."""
    import torch

    import synth
    import paper_2209_14671_amd as E
    from paper_2209_14671_amd import metrics
    optics = synth.Optics(n_lo=128, upsample=4, led_grid=15)
    flags = E.LEARN_PUPIL | E.PUPIL_SUPPORT | E.PUPIL_FILTER
    cells, tiles, k_total = [], [], 0
    for rep in range(args.reps):
        for di, d in enumerate((0.0, 0.5, 2.0)):
            base = synth.make_case(optics, [6, rep], jitter_mm=d)
            sim = E.Plan(E.problem_from_optics(optics, base.led_k_true, precision=E.F32), device=dev)
            psi_true = sim.spectrum_from_object(torch.from_numpy(base.obj).to(torch.complex64).to(dev))
            clean = sim.forward(psi_true, torch.from_numpy(base.pupil).to(torch.complex64).to(dev),
                                intens=True)["intens"].cpu().numpy().astype(np.float64)
            sim.close()
            dark = metrics.dark_field(base.led_k_true, optics.n_lo, optics.dx_lo_um, optics.wavelength_um, optics.na)
            for ci, c in enumerate((0.25, 0.5, 0.75)):
                for ni, noise in enumerate(SWEEP_NOISES):
                    for lv in range(4):
                        deg = synth.sweep_degradation(noise, lv, c)
                        noisy = synth.degrade(clean, deg, np.random.SeedSequence([6, rep, di, ci, ni, lv]), dark=dark)
                        meas = torch.from_numpy(noisy).to(torch.float32).to(dev)
                        plan = E.Plan(E.problem_from_optics(optics, base.led_k, precision=E.F32, flags=flags),
                                      device=dev)
                        tiles.append((plan, plan.init_state(meas), meas))
                        k_total += plan.K
                        cells.append({"rep": rep, "d_mm": d, "c": c, "noise": noise, "level": lv + 1, "obj": base.obj,
                                      "nl": metrics.noise_level(clean, noisy, dark)})
            log(f"seed {rep}, d = {d} mm: {len(tiles)} stacks built")
    batch = E.Batch(tiles, n_branches=4)  # a fixed branch count: the tuning is switched off
    branches = batch.n_branches
    log(f"{len(tiles)} tiles in one batch, {branches} branches")
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    batch.run(iters, history=False)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    for cell, (plan, st, _) in zip(cells, tiles):
        O = plan.object_from_spectrum(st.psi).cpu().numpy().astype(np.complex128)
        cell["la"] = metrics.lsnr(np.abs(O), np.abs(cell["obj"]))
        cell["lp"] = metrics.lsnr(np.angle(O), np.angle(cell["obj"]))
    batch.close()
    for plan, _, _ in tiles:
        plan.close()
    rows = []
    for d in (0.0, 0.5, 2.0):
        for ci, c in enumerate((0.25, 0.5, 0.75)):
            for noise in SWEEP_NOISES:
                for lv in range(1, 5):
                    sel = [x for x in cells if x["d_mm"] == d and x["c"] == c and x["noise"] == noise
                           and x["level"] == lv]
                    la = float(np.mean([x["la"] for x in sel]))
                    lp = float(np.mean([x["lp"] for x in sel]))
                    rows.append({"d_mm": d, "c": c, "noise": noise, "level": lv,
                                 "NL_pct": round(float(np.mean([x["nl"] for x in sel])), 2),
                                 "NL_pct_table1": TABLE1_NL[noise][ci][lv - 1],
                                 "lsnr_amp_db": round(la, 2), "lsnr_phase_db": round(lp, 2),
                                 "lsnr_mean_db": round((la + lp) / 2, 2)})
                    if lv in (1, 4):
                        log(f"d={d} c={c} {noise} Lv{lv}: NL {rows[-1]['NL_pct']} % (Table 1: "
                            f"{rows[-1]['NL_pct_table1']} %), LSNR amp {la:.2f} dB, phase {lp:.2f} dB")
    print(json.dumps({"metric": "reconstruction LSNR (Eq. 22) over the Sec. 4.2 grid with Table 1's noise levels",
                      "unit": "dB", "iterations": iters, "reps": args.reps, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "512x512 high-res, 15x15 LEDs (K=225), 128x128 low-res, circular "
                                             "pupil; every case in one batch", "tiles": len(tiles),
                                 "branches": branches},
                      "batch_ms_per_iter": round(ms / iters, 4),
                      "led_updates_per_s": round(k_total * iters / (ms / 1e3), 1),
                      "rows": rows}), flush=True)


def precision_bench(args, dev):
    """1024^2 high-res / K = 225 / 256^2 low-res, FP32: the plain form (FFT row and column
    transforms) against ELFPIE_F32_MFMA_BF16X3 (the row transforms as split-BF16 DFT-matrix
    products on the matrix cores), same stack and initial state: microseconds per iteration
    over `steps` timed iterations after `warmup`, and the isolated per-LED branch.  Their
    errors against the FP64 oracle after 100 iterations come from
    tests/test_gpu_precision_study.py (the oracle is not run here)."""
    import torch

    import synth
    import paper_2209_14671_amd as E
    case = synth.config_case(5)
    o = case.optics
    meas = simulated_stack(case, dev)
    flags = E.LEARN_PUPIL | E.PUPIL_SUPPORT | E.PUPIL_FILTER
    forms = {}
    for name, prec in (("fft_f32", E.F32), ("mfma_bf16x3", E.F32_MFMA_BF16X3)):
        plan = E.Plan(E.problem_from_optics(o, case.led_k, precision=prec, flags=flags), device=dev)
        st = plan.init_state(meas)
        hist = torch.empty((max(args.warmup, args.steps, 1), 4), dtype=torch.float64, device=dev)
        if args.warmup:
            plan.run(st, meas, args.warmup, history=hist)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        h = plan.run(st, meas, args.steps, history=hist)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / max(args.steps, 1)
        stages = plan.stage_timing(st, meas, max(args.stage_reps // 5, 3))
        L = h[:, 3].cpu().numpy()
        forms[name] = {"us_per_iter": round(ms * 1e3, 2), "value": round(plan.K / (ms * 1e-3), 1),
                       "led_branch_us": round(stages["led"] * 1e3, 2), "loss_first": float(L[0]),
                       "loss_last": float(L[-1])}
        log(f"{name}: {ms * 1e3:.1f} us/iteration, LED branch {stages['led'] * 1e3:.1f} us")
        plan.close()
    print(json.dumps({"metric": "LED sub-image updates/sec (K x iters/s): FFT form vs split-BF16 MFMA row transforms",
                      "unit": "LED-updates/s", "steps": args.steps, "warmup": args.warmup, "dtype": "f32",
                      "data": "synthetic", "config": {"workload": WORKLOADS[5][1], "K": 225, "n_lo": 256, "n_hi": 1024},
                      "forms": forms, "source_hash": kernel_source_hash()}), flush=True)


def batch_bench(args, dev):
    """Config 3: 64 independent tiles in one batch (four parallel graph branches), `steps`
    replays timed; value = sum of K over tiles x steps / seconds."""
    import torch

    import synth
    import paper_2209_14671_amd as E
    cases = synth.config3_tiles(64)
    flags = E.LEARN_PUPIL | E.PUPIL_SUPPORT | E.PUPIL_FILTER
    log(f"building {len(cases)} tiles")
    tiles, bytes_it, k_total = [], 0, 0
    for case in cases:
        o = case.optics
        meas = simulated_stack(case, dev)
        plan = E.Plan(E.problem_from_optics(o, case.led_k, precision=E.F32, flags=flags), device=dev)
        tiles.append((plan, plan.init_state(meas), meas))
        bytes_it += byte_model(plan.K, plan.S, plan.n_lo ** 2, plan.n_hi ** 2)[1]
        k_total += plan.K
    batch = E.Batch(tiles, n_branches=4)  # a fixed branch count: the tuning is switched off
    log(f"branches {batch.n_branches}")
    if args.warmup:
        batch.run(args.warmup, history=False)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    hist = batch.run(args.steps)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    ms_step = ms / max(args.steps, 1)
    if not all(bool(torch.isfinite(h).all()) for h in hist):
        raise RuntimeError("non-finite loss during the timed run")
    value = k_total * args.steps / (ms / 1e3)
    gbs = bytes_it / (ms_step * 1e-3) / 1e9
    log(f"{ms_step * 1e3:.1f} us per batch iteration, {value:.0f} LED-updates/s")
    out = {"metric": "LED sub-image updates/sec (sum K x iters/s over tiles); % HBM roofline",
           "value": round(value, 1), "unit": "LED-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": WORKLOADS[3][1], "tiles": len(tiles), "K_total": k_total,
                      "branches": batch.n_branches},
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": LED_KERNEL[3],
                        "algorithmic_bytes": bytes_it},
           "source_hash": kernel_source_hash()}
    if not args.no_cpu_baseline:
        log("CPU baseline (oracle, bounded sample)")
        out["cpu_baseline"] = cpu_baseline_tiles(cases, flags)
    batch.close()
    print(json.dumps(out), flush=True)


def cpu_baseline_tiles(cases, flags, budget_s=10.0):
    """The oracle on the tiles in order, one iteration each, until the budget is spent;
    the rate counts the iteration time only (simulation and set-up excluded)."""
    import oracle as orc
    n_led, done, step_wall, step_cpu = 0, 0, 0.0, 0.0
    t0 = time.perf_counter()
    for case in cases:
        if time.perf_counter() - t0 > budget_s:
            break
        o = case.optics
        sim = orc.problem_from_optics(o, case.led_k_true)
        meas = orc.intensities(orc.spectrum_from_object(case.obj), case.pupil, sim)
        prob = orc.problem_from_optics(o, case.led_k, flags=flags)
        st = orc.init_state(meas, prob)
        w0, c0 = time.perf_counter(), time.process_time()
        orc.step(st, meas, prob)
        step_wall += time.perf_counter() - w0
        step_cpu += time.process_time() - c0
        n_led += prob.K
        done += 1
    model, avail = host_cpu()
    return {"value": n_led / step_wall, "unit": "LED-updates/s", "cores": max(1, round(step_cpu / step_wall)),
            "kind": "oracle", "host_cpu": model, "cores_available": avail,
            "sample": f"one oracle iteration on each of the first {done} tiles (NumPy FP64), {step_wall:.1f} s"}


def host_cpu():
    """Model name of the host CPU and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(case, flags, budget_s=12.0, max_iter=100000):
    """The FP64 oracle (unchanged) on the same workload for a bounded number of iterations."""
    import oracle as orc
    import synth
    o = case.optics
    sim = orc.problem_from_optics(o, case.led_k_true)
    clean = orc.intensities(orc.spectrum_from_object(case.obj), case.pupil, sim)
    meas = synth.degrade(clean, case.degradation, case.noise_seed)
    prob = orc.problem_from_optics(o, case.led_k, flags=flags)
    st = orc.init_state(meas, prob)
    n = 0
    c0 = time.process_time()
    t0 = time.perf_counter()
    while n < max_iter and (time.perf_counter() - t0) < budget_s:
        st, _ = orc.step(st, meas, prob)
        n += 1
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    K = prob.K
    model, avail = host_cpu()
    return {"value": K * n / wall, "unit": "LED-updates/s", "cores": max(1, round(cpu / wall)),
            "kind": "oracle", "host_cpu": model, "cores_available": avail,
            "sample": f"{n} oracle iterations of the same workload (NumPy FP64), {wall:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stage-reps", type=int, default=50)
    ap.add_argument("--reps", type=int, default=1,
                    help="sweep: seeds per cell of the grid (108 cells, one 512^2 / K=225 stack each)")
    ap.add_argument("--copy-mib", type=int, default=1024,
                    help="size of the plain device copy timed after the run (0: skip); the same copy "
                         "calibrates the FETCH_SIZE / WRITE_SIZE counters in counter runs")
    ap.add_argument("--config", type=int, choices=sorted(WORKLOADS), default=2,
                    help="workload of the iteration line: 2 is the headline (512^2 / K=225 / 128^2, FP32); "
                         "1, 4 and 5 give the absolute numbers of the other single-FOV shapes")
    ap.add_argument("--workload", choices=["iteration", "autograd", "optimizers", "sweep", "precision"],
                    default="iteration",
                    help="iteration: the throughput line (default); autograd: forward + backward of the "
                         "differentiable loss at 256^2 / K=121 / 64^2, recomputed against stored fields; "
                         "optimizers: loss curves of Eq. 19 and the Sec. 6.2 alternatives on the "
                         "512^2 / K=225 / 128^2 stack; sweep: reconstruction quality (LSNR, Eq. 22) over LED "
                         "shift, uneven illumination and Table 1's noise levels (the Tables 2-4 grid) on "
                         "synthetic stacks, all reconstructed in one batch; "
                         "precision: the FFT form against the split-BF16 matrix-core row transforms at "
                         "1024^2 / K=225 / 256^2")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    import paper_2209_14671_amd as E

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "autograd":
        autograd_bench(args, dev)
        return
    if args.workload == "optimizers":
        optimizer_bench(args, dev)
        return
    if args.workload == "sweep":
        sweep_bench(args, dev)
        return
    if args.workload == "precision":
        precision_bench(args, dev)
        return
    if args.config == 3:
        batch_bench(args, dev)
        return
    case = synth.config_case(args.config)
    o = case.optics
    flags = E.LEARN_PUPIL | E.PUPIL_SUPPORT | E.PUPIL_FILTER
    dtype, workload = WORKLOADS[args.config]
    prec = E.F64 if dtype == "f64" else E.F32
    cdt, rdt = (torch.complex128, torch.float64) if dtype == "f64" else (torch.complex64, torch.float32)

    # simulate the measured stack on the GPU (library forward model, true LED positions)
    log("simulating the measured stack")
    sim = E.Plan(E.problem_from_optics(o, case.led_k_true, precision=prec), device=dev)
    obj = torch.from_numpy(case.obj).to(cdt).to(dev)
    psi_true = sim.spectrum_from_object(obj)
    p_true = torch.from_numpy(case.pupil).to(cdt).to(dev)
    clean = sim.forward(psi_true, p_true, intens=True)["intens"].cpu().numpy().astype(np.float64)
    meas_np = synth.degrade(clean, case.degradation, case.noise_seed)
    meas = torch.from_numpy(meas_np).to(rdt).to(dev)
    sim.close()

    plan = E.Plan(E.problem_from_optics(o, case.led_k, precision=prec, flags=flags), device=dev)
    K, S, B, A = plan.K, plan.S, plan.n_lo ** 2, plan.n_hi ** 2
    st = plan.init_state(meas)
    stream = torch.cuda.current_stream()

    # the plain-copy calibration first: it also brings the GPU out of idle before the
    # warm-up iterations
    copy = copy_bandwidth(dev, args.copy_mib) if args.copy_mib else None
    # one history buffer for the warm-up and the timed run: the run graphs are keyed on its
    # address, so the warm-up captures them and the timed run only replays
    hist_buf = torch.empty((max(args.warmup, args.steps, 1), 4), dtype=torch.float64, device=dev)
    # per-kernel timing (HIP events around back-to-back launches on this stream; the state is
    # read, not changed), then the warm-up iterations right before the timed ones
    log("per-stage timing")
    stages = plan.stage_timing(st, meas, args.stage_reps)
    log(f"warmup {args.warmup} iterations")
    if args.warmup:
        plan.run(st, meas, args.warmup, history=hist_buf)
    torch.cuda.synchronize()
    cap0 = plan.stats()["captures"]

    log(f"timing {args.steps} iterations")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    hist = plan.run(st, meas, args.steps, history=hist_buf)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    captures_timed = plan.stats()["captures"] - cap0
    ms = ev0.elapsed_time(ev1)
    ms_step = ms / max(args.steps, 1)
    value = K * args.steps / (ms / 1e3)
    h = hist.cpu().numpy()
    if not np.all(np.isfinite(h)):
        raise RuntimeError("non-finite loss during the timed run")
    log(f"{ms_step * 1e3:.1f} us/iteration, loss {h[0, 3]:.4e} -> {h[-1, 3]:.4e} (wall {wall:.3f} s)")

    led_bytes, it_bytes = byte_model(K, S, B, A, 8 if dtype == "f64" else 4)
    fused = bool(stages.get("object_in_led_launch"))
    if fused:  # the object branch's column pass rides in the launch: T1 read, T2 written
        led_bytes += 2 * (2 * (8 if dtype == "f64" else 4)) * A
    led_s = stages["led"] * 1e-3
    src_hash = kernel_source_hash()
    traffic = measured_traffic(src_hash) if args.config == 2 else None
    roof = {"bound": "hbm", "achieved": round(led_bytes / led_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(led_bytes / led_s / 1e9 / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": LED_KERNEL[args.config] + (" with object-branch blocks" if fused else ""),
            "algorithmic_bytes": led_bytes,
            "avg_launch_ms": round(stages["led"], 4)}
    if copy is not None:
        roof["copy_GBs"] = copy
    it_gbs = it_bytes / (ms_step * 1e-3) / 1e9

    out = {
        "metric": METRIC if args.config == 2 else "LED sub-image updates/sec (K x iters/s); % HBM roofline",
        "value": round(value, 1), "unit": "LED-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": workload,
                   "K": K, "n_lo": plan.n_lo, "n_hi": plan.n_hi, "support_px": S, "learn_pupil": True},
        "roofline": roof,
        "iteration_roofline": {"algorithmic_bytes": it_bytes, "achieved_GBs": round(it_gbs, 1),
                               "frac": round(it_gbs / HBM_PEAK_GBS, 4)},
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "graph_captures_in_timed_run": captures_timed,
        "source_hash": src_hash,
    }
    if not args.no_cpu_baseline:
        log("CPU baseline (oracle, bounded sample)")
        out["cpu_baseline"] = cpu_baseline(case, flags)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
