"""Benchmark of the SOC Monte Carlo hot path on one MI355X.

Workload: 128^3 regular grid, lognormal density (Gaussian random field with
P(k) ~ k^-3, sigma_ln = 1, mean face-to-face tau_V = 5), synthetic dust on
64 log-spaced frequencies 0.1-3000 um, isotropic synthetic external field
and two 10^4 K blackbody point sources, 10^6 packages per frequency.

Iteration 1 simulates the constant sources (background 5e5 + 2 x 2.5e5
packages per frequency) once and keeps their absorbed energy.  Every later
iteration -- one benchmark step -- re-simulates the dust emission at the
current temperatures (10^6 luminosity-weighted packages per frequency, all
64 frequencies in one persistent launch) on top of the kept absorption and
solves the temperatures.
Steps are the iterations of the plain method "iterate T to 1% change".

Time to 1% temperature convergence (the paper's two statistics of
Sect. 3.3, taken against a reference field): T_ref is the mean temperature
of the timed iterations.  Two more runs with the same seed, and so the
same constant-source pass, are then timed from their constant pass to the
first iteration within 1% of T_ref over all cells and over the hottest 5%:
the plain method, and the learned start, whose U-Net is trained in this
run on clouds the plain method solves here (its data and training seconds
are reported beside it).

Prints one JSON line (rank 0, N = 1 only).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_STEP = 12.0   # 4 B density gather + 8 B FP64 absorbed update per cell step
# regular-grid instantiation of the persistent MC kernel that runs every
# frequency of a pass in one launch
MC_KERNEL = "soc::mc_multi_kernel<false, false>"
# HBM traffic of the MC kernel measured with rocprofv3 counters (FETCH_SIZE,
# WRITE_SIZE, scaled by a 1 GiB copy); used only while the kernel sources
# and compile flags still hash to the value recorded with it.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mc_kernel_lognormal128_traffic.md")
MC_SOURCES = ("mc.hip", "soc_device.h", "soc_kernels.h")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def mc_source_hash():
    """SHA-256 of the MC kernel's sources and the library's compile flags."""
    import hashlib
    from __graft_entry__ import HIP_FLAGS
    h = hashlib.sha256()
    for name in MC_SOURCES:
        with open(os.path.join(ROOT, "paper_1812_06632_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    h.update(" ".join(HIP_FLAGS).encode())
    return h.hexdigest()


def recorded_counters():
    """(HBM bytes per MC launch, memory-side atomic transactions per cell
    step) from the committed counter summary; None for each value that is
    absent, and for both when the summary was taken on other kernel
    sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None, None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("mc_source_sha256") != mc_source_hash():
        return None, None

    def num(key):
        try:
            return float(vals[key])
        except (KeyError, ValueError):
            return None
    return num("hbm_bytes_per_launch"), num("atomic_transactions_per_cell_step")


def device_ceilings(soc, ctx, torch, ncells):
    """Measured ceilings of the MC kernel's memory operations at the grid's
    size: random FP64 atomic adds and a 1 GiB streaming copy (the copy is
    also the scale reference of the HBM byte counters)."""
    a = torch.zeros(ncells, dtype=torch.float64, device="cuda")
    blocks, threads, per = 4096, 256, 64
    soc.ubench(ctx, 0, a, None, ncells, per, 0, blocks, threads)
    ms = min(soc.ubench(ctx, 0, a, None, ncells, per, 0, blocks, threads) for _ in range(3))
    atomics = blocks * threads * per / (ms * 1e-3)
    nbytes = 1 << 30
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    soc.ubench(ctx, 2, src, dst, nbytes, 1, 0, 8192, 256)
    ms = min(soc.ubench(ctx, 2, src, dst, nbytes, 1, 0, 8192, 256) for _ in range(3))
    copy_gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    del a, src, dst
    return atomics, copy_gbs


def ceilings(soc, torch, ncells):
    """Every micro-benchmark mode at the benchmark grid's size."""
    ctx = soc.Context(0)
    blocks, threads, per = 4096, 256, 64
    a = torch.zeros(8 * ncells, dtype=torch.float64, device="cuda")
    names = {0: "FP64, random, one shared array", 1: "FP64, random, one private copy per XCD (hardware XCC id)",
             2: "FP64, wave-coalesced 64-double blocks", 3: "FP64, random in a 4096-double LDS array",
             4: "FP32, random, one shared array", 5: "uint64, random, one shared array",
             6: "uint32, random, one shared array"}
    for n_el in sorted({ncells, 1 << 15}, reverse=True):
        for mode, label in names.items():
            a.zero_()
            soc.ubench(ctx, 0, a, None, n_el, per, mode, blocks, threads)
            ms = min(soc.ubench(ctx, 0, a, None, n_el, per, mode, blocks, threads) for _ in range(3))
            print(json.dumps({"kind": "atomic_add", "mode": mode, "pattern": label, "array_elems": n_el,
                              "ms": ms, "per_s": blocks * threads * per / (ms * 1e-3)}), flush=True)
    w = torch.randint(0, 2**31 - 1, (ncells,), dtype=torch.int32, device="cuda")
    out = torch.zeros(4, dtype=torch.int32, device="cuda")
    for nb in (4096, 16384):
        soc.ubench(ctx, 1, w, out, ncells, per, 0, nb, threads)
        ms = min(soc.ubench(ctx, 1, w, out, ncells, per, 0, nb, threads) for _ in range(3))
        print(json.dumps({"kind": "dependent_gather_4B", "array_words": ncells, "blocks": nb, "ms": ms,
                          "per_s": nb * threads * per / (ms * 1e-3)}), flush=True)
    _, copy_gbs = device_ceilings(soc, ctx, torch, ncells)
    print(json.dumps({"kind": "copy", "bytes": 1 << 30, "GBs_read_plus_write": copy_gbs}), flush=True)
    ctx.close()


BF16_MFMA_PEAK_TFLOPS = 2500.0   # dense BF16 matrix-core peak of MI355X


def batch_bench(args, soc, torch, W):
    """Many independent clouds in one persistent launch: lognormal models of
    16^3-96^3 cells, 32 frequencies, 1e5-1e6 background packages per
    (model, frequency) pair.  One pass = zero every absorbed array, the
    batched launch over all pairs, the temperature update of every model;
    it is captured once in a HIP graph and replayed (the iteration word
    advances on every replay).  Reports packages/s and cell steps/s over
    the timed replays."""
    from paper_1812_06632_amd import autotune as AT
    t0 = time.time()
    grids, (nu, w, sabs, ssca, g, I), pk = W.batch_clouds(args.batch_models, args.batch_freqs)
    log(f"batch workload: {len(grids)} models, {sum(gr.ncells for gr in grids)} cells, "
        f"{int(pk.sum())} packages per pass ({time.time() - t0:.1f}s)")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx = soc.Context(0, stream=s)
        G = [soc.grid_from_workload(ctx, gr) for gr in grids]
        table = soc.temp_table_build(ctx, nu, w, sabs, 2.0, 3000.0, 1024)
        A = [torch.zeros(gr.ncells, dtype=torch.float64, device="cuda") for gr in grids]
        T = [torch.zeros(gr.ncells, dtype=torch.float32, device="cuda") for gr in grids]

        def pair_list(models, freqs):
            return [dict(grid=m, freq=(float(nu[k]), float(w[k]), float(sabs[k]), float(ssca[k]), float(g[k])),
                         freq_index=k, I_bg=float(I[k]), n_bg=int(pk[m, k]), absorbed=A[m])
                    for m in models for k in freqs]

        # ---- launch schedule: the autotuner on every 8th model at every 8th
        # frequency (1/64 of the work, the same mix of sizes), timed with HIP
        # events around the batched launch
        tuned = None
        lds_default = ctx.get_option("batch_lds_cells")
        if not args.no_tune:
            cal = pair_list(range(0, len(grids), 8), range(0, len(nu), 8))
            default = {k: ctx.get_option(k) for k in ("block", "blocks_per_cu", "refill_min", "chunk")}
            default.update(tile_packages=args.tile, batch_lds_cells=lds_default)
            cal_batches = {}

            def run(cfg):
                kb = (cfg["tile_packages"], cfg["batch_lds_cells"])
                if kb not in cal_batches:
                    ctx.set_option("batch_lds_cells", cfg["batch_lds_cells"])
                    cal_batches[kb] = soc.Batch(ctx, G, cal, seed=1, tile_packages=cfg["tile_packages"])
                cal_batches[kb].run(iteration=0)

            # two families: small grids tallied in LDS by whole-pair workgroups
            # (fixed 512-lane launch shape), or every pair tiled
            spaces = [{"tile_packages": AT.BATCH_TILES, "refill_min": (1, 16), "chunk": (256, 1024),
                       "batch_lds_cells": (lds_default,)},
                      {"tile_packages": AT.BATCH_TILES, "block": (128, 256), "blocks_per_cu": (2, 4, 8),
                       "refill_min": (1, 16), "batch_lds_cells": (0,)}]
            measure = AT.event_timer(ctx, run)
            t0 = time.time()
            results = []
            for i, space in enumerate(spaces):
                tuner = AT.Autotuner()
                key = f"batch:{i}"
                cfg = tuner.tune(key, measure, space=space, repeats=2)
                results.append((tuner.cache[key]["seconds"], cfg, len(tuner.cache[key]["tried"])))
            t_default = min(measure(default) for _ in range(2))
            for bb in cal_batches.values():
                bb.close()
            best_s, tuned, n_cand = min(results, key=lambda r: r[0])
            n_cand = sum(r[2] for r in results)
            for k in ("block", "blocks_per_cu", "refill_min", "chunk"):
                ctx.set_option(k, default[k])
            AT.apply(ctx, tuned)
            ctx.set_option("batch_lds_cells", tuned["batch_lds_cells"])
            log(f"autotuned schedule {tuned} in {time.time() - t0:.1f}s: calibration launch {best_s * 1e3:.2f} ms "
                f"(default schedule {t_default * 1e3:.2f} ms)")
        pairs = pair_list(range(len(grids)), range(len(nu)))

        def full_pass(cfg, reps):
            """Build the whole batch under schedule cfg, capture one pass in a
            graph and time reps replays: (s per pass, packages, cell steps,
            tiles, packages per pass)."""
            AT.apply(ctx, cfg)
            ctx.set_option("batch_lds_cells", cfg["batch_lds_cells"])
            bb = soc.Batch(ctx, G, pairs, seed=1, tile_packages=cfg["tile_packages"])
            nt, npk = bb.info()
            bb.run(iteration=0)
            torch.cuda.synchronize()
            soc.graph_begin(ctx)
            for a in A:
                a.zero_()
            bb.run(iteration=soc.ITER_ADVANCE)
            for m in range(len(grids)):
                soc.update_temperature(ctx, G[m], table, A[m], T[m])
            gr = soc.graph_end(ctx)
            for _ in range(max(args.warmup, 1)):
                gr.launch()
            torch.cuda.synchronize()
            before = ctx.read_stats()
            t1 = time.time()
            for _ in range(reps):
                gr.launch()
            torch.cuda.synchronize()
            el_ = time.time() - t1
            after = ctx.read_stats()
            gr.close()
            bb.close()
            return (el_ / reps, after["packages"] - before["packages"], after["cell_steps"] - before["cell_steps"],
                    nt, npk)

        # the calibration sample is 1/64 of the pass; the tuned schedule is
        # kept only if it also beats the default on two replays of the
        # whole pass
        default_cfg = {k: ctx.get_option(k) for k in ("block", "blocks_per_cu", "refill_min", "chunk")}
        default_cfg.update(tile_packages=args.tile, batch_lds_cells=lds_default)
        full_check = None
        chosen = default_cfg
        if tuned:
            tuned_cfg = dict(default_cfg, **tuned)
            t_tuned_full = full_pass(tuned_cfg, 2)[0]
            t_default_full = full_pass(default_cfg, 2)[0]
            full_check = {"tuned_s": t_tuned_full, "default_s": t_default_full}
            chosen = tuned_cfg if t_tuned_full <= t_default_full else default_cfg
            log(f"whole pass: tuned {t_tuned_full:.3f}s, default {t_default_full:.3f}s")
        per_pass, pk_done, st_done, n_tiles, n_pk = full_pass(chosen, args.steps)
        el = per_pass * args.steps
    line = {"kind": "batch", "models": len(grids), "pairs": len(pairs), "tiles": n_tiles,
            "cells": int(sum(gr.ncells for gr in grids)), "packages_per_pass": n_pk, "passes": args.steps,
            "ms_per_pass": per_pass * 1e3, "packages_per_s": pk_done / el, "cell_steps_per_s": st_done / el,
            "tile_packages": chosen["tile_packages"], "graph": True,
            "schedule": {k: ctx.get_option(k) for k in ("block", "blocks_per_cu", "refill_min", "chunk",
                                                       "scatter_min", "inner_steps", "batch_lds_cells")},
            "autotuned": tuned is not None, "schedule_kept": "tuned" if chosen is not default_cfg else "default",
            "whole_pass_check": full_check,
            "calibration": ({"workload": "every 8th model at every 8th frequency (1/64 of the pass)",
                             "best_s": best_s, "default_schedule_s": t_default, "candidates": n_cand}
                            if tuned else None)}
    print(json.dumps(line), flush=True)
    ctx.close()


def unet_step(args, soc, torch):
    """Forward, backward and Adam of the U-Net at its production shape,
    timed with events on the library's stream; flops are the real
    (unpadded) multiply-adds x 2, backward counted as twice the forward."""
    ctx = soc.Context(0)
    n, S = args.unet_batch, 64
    net = soc.UNet(ctx, 2, 2, 32, 4, n, (S, S, S), seed=1)
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn((n, S, S, S, 2), device="cuda", generator=g)
    t = torch.randn((n, S, S, S, 2), device="cuda", generator=g)
    y = net.forward(x)
    _, dy = net.mse(y, t, loss=False)
    net.backward(dy)
    net.adam()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    R = max(args.steps, 1) * 3
    stream = ctx.stream
    ev[0].record(stream)
    for _ in range(R):
        net.forward(x, y)
    ev[1].record(stream)
    for _ in range(R):
        net.backward(dy)
    ev[2].record(stream)
    for _ in range(R):
        net.adam()
    ev[3].record(stream)
    torch.cuda.synchronize()
    tf, tb, ta = (ev[i].elapsed_time(ev[i + 1]) / R for i in range(3))
    f = net.flops(n)
    line = {"kind": "unet_step", "shape": f"{n} x {S}^3", "base": 32, "levels": 4, "params": net.param_count,
            "gflop_forward": f / 1e9, "ms_forward": tf, "ms_backward": tb, "ms_adam": ta,
            "ms_step": tf + tb + ta, "tflops_forward": f / tf / 1e9, "tflops_backward": 2 * f / tb / 1e9,
            "tflops_step": 3 * f / (tf + tb + ta) / 1e9,
            "frac_of_bf16_peak_step": 3 * f / (tf + tb + ta) / 1e9 / BF16_MFMA_PEAK_TFLOPS}
    print(json.dumps(line), flush=True)
    net.close()
    ctx.close()


def surrogate_gain(args, soc, torch, W):
    """The learned start on a thick cloud (sigma_ln --target-sigma, mean
    tau_V --target-tau, --target-n^3 cells, the benchmark's frequencies and
    sources, --target-packages per frequency and iteration).

    Training: --train-clouds random 64^3 clouds of the training family
    solved by the plain method here (plus --val-clouds held out); the
    two-output U-Net is trained on them, and, for a learning curve, on
    subsets of them (--curve), each scored on the held-out clouds.

    Target runs, each timed from its constant pass to the first iteration
    within 1% of T_ref (mean |T - T_ref| / T_ref over all cells with dust
    and over the hottest 5%); T_ref is the mean of --ref-avg plain
    iterations after --ref-burn, with the same seed and hence the same
    constant-source pass, their dust emission drawn from iteration indices
    beyond --max-iter:
      plain        plain iterations from the constant-source temperatures;
      mode_A       plain iterations from the network's temperatures;
      mode_B       reference-field iterations (Sect. 2.1.2, running mean of
                   whole-emission estimates) seeded with the network's
                   temperatures and absorbed energies, the prediction
                   counted as one iteration's packages;
      reference    the same reference-field iterations without the network;
      control      plain iterations from T1 times the training set's mean
                   ratio T / T1 (no learning: what a global correction
                   gives).
    Every run also reports where the plain stopping rule (change between
    iterations below 1%) fires and its error there: the plain method as
    the judge of the prediction."""
    from paper_1812_06632_amd.driver import PlainSolver, ReferenceFieldSolver
    from paper_1812_06632_amd.surrogate import Surrogate, make_dataset, Y_SCALE
    ctx = soc.Context(0)
    S = 64
    t0 = time.time()
    X, Y = make_dataset(ctx, args.train_clouds + args.val_clouds, seed=11, n=64, S=S, K=32,
                        packages=args.train_packages, log=log)
    t_data = time.time() - t0
    ntr = args.train_clouds
    Xv, Yv = X[ntr:], Y[ntr:]
    mean_ratio = float(Y[:ntr, ..., 0].mean().item()) * Y_SCALE   # training-set mean log10(T / T1)

    def val_loss(sur):
        """Mean squared error per output channel on the held-out clouds."""
        se = torch.zeros(Y.shape[-1], dtype=torch.float64, device="cuda")
        for i in range(0, Xv.shape[0], 4):
            y = sur.net.forward(Xv[i:i + 4].contiguous())
            se += ((y - Yv[i:i + 4]) ** 2).double().sum(dim=(0, 1, 2, 3))
        return (se / (Yv.numel() / Yv.shape[-1])).tolist()

    curve = []
    for n_sub in sorted({int(v) for v in args.curve.split(",") if v} | {ntr}):
        if n_sub > ntr:
            continue
        sur = Surrogate(ctx, S=S, base=32, levels=4, batch=4, seed=3)
        t0 = time.time()
        losses = sur.fit(X[:n_sub], Y[:n_sub], steps=args.train_steps, lr=5e-4,
                         log=log if n_sub == ntr else None)
        torch.cuda.synchronize()
        t_train = time.time() - t0
        vl = val_loss(sur) if Xv.shape[0] else None
        curve.append({"clouds": n_sub, "train_s": t_train, "final_loss": losses[-1][1] if losses else None,
                      "val_mse_T": vl[0] if vl else None, "val_mse_A": vl[1] if vl else None})
        log(f"learning curve: {n_sub} clouds, val mse {vl}")
        if n_sub == ntr:
            net = sur
        else:
            sur.close()
    del X, Y, Xv, Yv

    n = args.target_n
    P = W.lognormal_problem(n=n, K=args.freqs, sigma_ln=args.target_sigma, tau_v_mean=args.target_tau,
                            packages_per_freq=args.target_packages)
    rho = P.grid.density().reshape(n, n, n).astype(np.float64)
    tau_max = float(max((rho.sum(axis=a)).max() for a in range(3)) * W.SIGMA_V * P.grid.root_cell_cm)
    del rho
    ref = PlainSolver(ctx, P, seed=1)
    torch.cuda.synchronize()
    t0 = time.time()
    ref.constant_pass()
    acc = torch.zeros(P.grid.ncells, dtype=torch.float64, device="cuda")
    # the averaged iterations draw from iteration streams past the timed
    # runs' last one, so that no timed iterate shares its dust-emission
    # random numbers with T_ref (only the constant-source pass is shared)
    shift = max(0, args.max_iter - args.ref_burn)
    for it in range(2, args.ref_burn + args.ref_avg + 2):
        if it > args.ref_burn + 1:
            ref.dust_iteration(it + shift)
            acc += ref.T
        else:
            ref.dust_iteration(it)
    T_ref = (acc / args.ref_avg).float()
    t_ref = time.time() - t0
    dense = torch.from_numpy(P.grid.density()).cuda() > 0
    crit = RefCriterion(torch, T_ref, dense)
    del ref, acc
    log(f"{n}^3 reference ({args.ref_burn} + {args.ref_avg} iterations, {t_ref:.1f}s): <T> "
        f"{crit.Tr.mean().item():.3f} K, hottest 5% {crit.Tr[crit.hot].mean().item():.3f} K")

    def mode_a(s_):
        return s_.set_temperature(net.predict_T(s_, s_.T))

    def mode_b(s_):
        y = net.predict(s_, s_.T)
        T0 = net.predict_T(s_, s_.T, y=y)
        A0 = net.predict_A(s_, s_.A_const, y)
        return s_.seed_prediction(T0, A0, s_.n_packages(2))

    def control(s_):
        return s_.set_temperature(torch.clamp(s_.T * (10.0 ** mean_ratio), max=P.T_max) * (s_.T > 0))

    runs = {}
    for label, make, start in (("plain", lambda: PlainSolver(ctx, P, seed=1), None),
                               ("mode_A", lambda: PlainSolver(ctx, P, seed=1), mode_a),
                               ("mode_B", lambda: ReferenceFieldSolver(ctx, P, seed=1, mode="average"), mode_b),
                               ("reference", lambda: ReferenceFieldSolver(ctx, P, seed=1, mode="average"), None),
                               ("control", lambda: PlainSolver(ctx, P, seed=1), control)):
        solver = make()
        t_hit, n_hit, stop, hist = timed_to_criterion(torch, solver, crit, start=start, max_iter=args.max_iter,
                                                      run_on=True)
        at_stop = next((h for h in hist if h[0] == stop), None)
        levels = {}
        for lev in (0.05, 0.03, 0.02, 0.015, 0.01):
            h = next((h for h in hist if h[2] < lev and h[3] < lev), None)
            levels[f"{lev:g}"] = [h[0], round(h[1], 3)] if h else None
        runs[label] = {"s_to_1pct": t_hit, "iterations_to_1pct": n_hit,
                       "iteration_and_s_within": levels,
                       "stopping_rule_iteration": stop,
                       "err_at_stopping_rule": [at_stop[2], at_stop[3]] if at_stop else None,
                       "by_iteration": [[h[0], round(h[1], 3), round(h[2], 5), round(h[3], 5)] for h in hist]}
        log(f"{label}: within 1% of T_ref at iteration {n_hit} ({t_hit}s); stopping rule at {stop}; {hist}")
        del solver
    line = {"kind": "surrogate_gain",
            "workload": f"lognormal {n}^3, sigma_ln {args.target_sigma}, mean tau_V {args.target_tau} "
                        f"(largest face-to-face tau_V {tau_max:.0f}), two 1e6 L_sun sources, {args.freqs} "
                        f"frequencies, {args.target_packages} packages per frequency and iteration "
                        f"({args.target_packages * args.freqs:.3g} per iteration)",
            "T_ref": {"burn_in": args.ref_burn, "averaged": args.ref_avg, "seconds": t_ref,
                      "mean_T": crit.Tr.mean().item(), "hot5_mean_T": crit.Tr[crit.hot].mean().item()},
            "training": {"clouds": ntr, "held_out": args.val_clouds, "cells": "64^3", "frequencies": 32,
                         "packages_per_frequency": args.train_packages, "steps": args.train_steps, "batch": 4,
                         "data_s": t_data, "params": net.net.param_count, "learning_curve": curve,
                         "control_mean_log10_T_over_T1": mean_ratio},
            "runs": runs,
            "speedup_mode_A": (runs["plain"]["s_to_1pct"] / runs["mode_A"]["s_to_1pct"]
                               if runs["plain"]["s_to_1pct"] and runs["mode_A"]["s_to_1pct"] else None),
            "speedup_mode_B": (runs["plain"]["s_to_1pct"] / runs["mode_B"]["s_to_1pct"]
                               if runs["plain"]["s_to_1pct"] and runs["mode_B"]["s_to_1pct"] else None)}
    print(json.dumps(line), flush=True)
    net.close()
    ctx.close()


def reference_gain(args, soc, torch, W):
    """Plain versus reference-field iteration (Sect. 2.1.2, 3.6) on two
    clouds -- the benchmark cloud (sigma_ln 1, mean tau_V 5) and an
    optically thick one where dust self-heating takes several iterations
    (sigma_ln --target-sigma, tau_V --target-tau) -- with the benchmark's
    frequencies, sources and package count.  Six runs of --ref-iters
    iterations each: plain and the two readings of the reference field
    (correction packages; running mean of whole-emission estimates) with a
    constant package count, and the same three with a count growing
    geometrically from 1/--ref-factor of it.  Each is timed and compared with a long plain reference (mean of
    8 iterations after 12): the first iteration within 1% of it (over all
    cells and over the hottest 5%), the iteration the stopping rule fires,
    and the rms temperature difference between two runs with independent
    dust-emission seeds at the end (the paper's noise measure)."""
    from paper_1812_06632_amd.driver import PlainSolver, ReferenceFieldSolver, geometric_schedule
    ctx = soc.Context(0)
    I = args.ref_iters
    sched = geometric_schedule(args.packages, args.ref_factor, I)

    def cloud(label, sigma, tau):
        P = W.lognormal_problem(n=args.n, K=args.freqs, sigma_ln=sigma, tau_v_mean=tau,
                                packages_per_freq=args.packages)
        ref = PlainSolver(ctx, P, seed=7)
        ref.constant_pass()
        burn, avg = 12, 8
        acc = torch.zeros_like(ref.T, dtype=torch.float64)
        for it in range(2, burn + avg + 2):
            ref.dust_iteration(it)
            if it > burn + 1:
                acc += ref.T.double()
        T_ref = acc / avg
        del ref
        dense = torch.from_numpy(P.grid.density()).cuda() > 0
        Tr = T_ref[dense]
        hot = Tr >= torch.quantile(Tr.float(), 0.95).double()
        log(f"{label}: reference <T> {Tr.mean().item():.3f} K, hottest 5% {Tr[hot].mean().item():.3f} K")

        def err(T):
            r = (T.double()[dense] - Tr).abs() / Tr
            return r.mean().item(), r[hot].mean().item()

        out = {}
        runs = [("plain", None, None), ("correction", "correction", None), ("average", "average", None),
                ("plain_growing", None, sched), ("correction_growing", "correction", sched),
                ("average_growing", "average", sched)]
        for name, mode, pk in runs:
            finals = []
            for seed in (1, 2):
                if mode:
                    S = ReferenceFieldSolver(ctx, P, seed=seed, packages=pk, mode=mode)
                else:
                    S = PlainSolver(ctx, P, seed=seed, packages=pk)
                errs = {}
                ctx.read_stats(reset=True)
                hist, at = S.run(max_iter=I, until_stop=False,
                                 on_iter=(lambda it, T: errs.__setitem__(it, err(T))) if seed == 1 else None)
                st = ctx.read_stats(reset=True)
                finals.append(S.T.double()[dense].clone())
                if seed == 1:
                    ref1 = next((it for it in sorted(errs) if errs[it][0] < 0.01 and errs[it][1] < 0.01), None)
                    wall = hist[-1][1]
                    rec = {"iterations": I, "wall_s": wall, "stopping_rule_at": at,
                           "wall_s_to_stopping_rule": hist[at - 1][1] if at else None,
                           "iterations_to_1pct_of_ref": ref1,
                           "wall_s_to_1pct_of_ref": hist[ref1 - 1][1] if ref1 else None,
                           "err_final": [round(v, 5) for v in errs[I]],
                           "err_by_iteration": {int(k): [round(v[0], 5), round(v[1], 5)] for k, v in errs.items()},
                           "dust_packages_per_freq": [S.n_packages(it) for it in range(2, I + 1)],
                           "packages_per_s": st["packages"] / wall}
                del S
            d = finals[0] / finals[1] - 1.0
            rec["rms_between_seeds"] = [math.sqrt((d * d).mean().item()), math.sqrt((d[hot] ** 2).mean().item())]
            out[name] = rec
            log(f"{label} {name}: {I} iterations {rec['wall_s']:.2f}s, within 1% of the reference from iteration "
                f"{rec['iterations_to_1pct_of_ref']}, stopping rule at {rec['stopping_rule_at']}, final error "
                f"{rec['err_final']}, rms between seeds {rec['rms_between_seeds'][0]:.4f} "
                f"(hottest 5% {rec['rms_between_seeds'][1]:.4f})")
        return {"cloud": label, "sigma_ln": sigma, "tau_V": tau, "reference_mean_T": Tr.mean().item(),
                "reference_hot5_mean_T": Tr[hot].mean().item(), "runs": out}

    clouds = [cloud("benchmark cloud", 1.0, 5.0), cloud("thick cloud", args.target_sigma, args.target_tau)]
    line = {"kind": "reference_field", "cells": f"{args.n}^3", "frequencies": args.freqs,
            "packages_per_freq": args.packages, "iterations": I, "growing_from": args.packages / args.ref_factor,
            "clouds": clouds}
    print(json.dumps(line), flush=True)
    ctx.close()


def ali_gain(args, soc, torch, W):
    """Plain versus diagonal-ALI iteration (Sect. 2.1.2, 4.1) on the paper's
    ALI test setup: a lognormal cloud shrunk to a (--ali-box pc)^3 box with
    mean tau_V --ali-tau and one central --ali-lsun L_sun source, so that
    dust near the source is hot and its emission is absorbed nearby.  The
    same density field (made at 128^3) is block-averaged to 32^3, 64^3 and
    128^3: coarser cells are optically thicker, where ALI should help most.
    At each resolution, both iterations run --ali-iters iterations against a
    long reference run (mean of the last 8 of --ali-ref-iters ALI
    iterations; the two iterations share their fixed point, and in thick
    clouds the plain one is still far from it after 40): the first
    iteration whose mean and hottest-5% mean temperatures are within 1% of
    the reference's (the paper's |<dT>| measure), the wall time to it, and
    the cost per iteration."""
    import dataclasses

    from paper_1812_06632_amd.driver import PlainSolver
    ctx = soc.Context(0)
    base = W.lognormal_problem(n=128, K=args.freqs, sigma_ln=1.0, tau_v_mean=args.ali_tau, box_pc=args.ali_box,
                               L_star_lsun=args.ali_lsun, ps_frac=((0.5, 0.5, 0.5),), packages_per_freq=args.packages)
    rho128 = base.grid.density().reshape(128, 128, 128).astype(np.float64)
    out = []
    for n in (32, 64, 128):
        f = 128 // n
        rho = rho128.reshape(n, f, n, f, n, f).mean(axis=(1, 3, 5))
        ps = base.ps_pos / f
        for p in ps:
            rho[int(p[2]), int(p[1]), int(p[0])] = 0.0   # the source sits in an empty cell
        P = dataclasses.replace(base, grid=W.regular_grid(rho.astype(np.float32), base.grid.root_cell_cm * f),
                                ps_pos=ps)
        ref = PlainSolver(ctx, P, seed=7, ali=True)
        ref.constant_pass()
        avg = 8
        burn = args.ali_ref_iters - avg
        m_ref = h_ref = 0.0
        for it in range(2, burn + avg + 2):
            s = ref.dust_iteration(it)
            if it > burn + 1:
                m_ref += s["mean_T"] / avg
                h_ref += s["hot5_mean_T"] / avg
        del ref
        log(f"{n}^3: reference <T> {m_ref:.3f} K, hottest 5% {h_ref:.3f} K")
        runs = {}
        for ali in (False, True):
            S = PlainSolver(ctx, P, seed=1, ali=ali)
            hist, at = S.run(max_iter=args.ali_iters, until_stop=False)
            dm = [abs(h[2]["mean_T"] / m_ref - 1) for h in hist]
            dh = [abs(h[2]["hot5_mean_T"] / h_ref - 1) for h in hist]
            within = next((h[0] for h, a, b in zip(hist, dm, dh) if a < 0.01 and b < 0.01), None)
            reach = {f"iterations_to_{int(x * 100)}pct": next((h[0] for h, a, b in zip(hist, dm, dh)
                                                                 if a < x and b < x), None) for x in (0.1, 0.05)}
            per_it = (hist[-1][1] - hist[0][1]) / (len(hist) - 1)
            runs["ali" if ali else "plain"] = {
                "iterations_to_1pct": within, "wall_s_to_1pct": hist[within - 1][1] if within else None,
                "stopping_rule_at": at, "s_per_dust_iteration": per_it, **reach,
                "rel_dmean_by_iteration": [round(x, 5) for x in dm], "rel_dhot5_by_iteration": [round(x, 5) for x in dh]}
            log(f"{n}^3 {'ALI' if ali else 'plain'}: within 1% of the reference at iteration {within}, "
                f"stopping rule at {at}, {per_it:.3f} s per dust iteration")
            del S
        rec = {"cells": f"{n}^3", "reference_mean_T": m_ref, "reference_hot5_mean_T": h_ref, "runs": runs,
               "ali_overhead": runs["ali"]["s_per_dust_iteration"] / runs["plain"]["s_per_dust_iteration"] - 1.0}
        if runs["ali"]["wall_s_to_1pct"] and runs["plain"]["wall_s_to_1pct"]:
            rec["speedup_to_1pct"] = runs["plain"]["wall_s_to_1pct"] / runs["ali"]["wall_s_to_1pct"]
        out.append(rec)
    line = {"kind": "ali", "workload": f"lognormal sigma_ln 1, mean tau_V {args.ali_tau}, {args.ali_box} pc box, one "
                                      f"{args.ali_lsun:g} L_sun source at the centre, {args.freqs} frequencies, "
                                      f"{args.packages} packages/frequency", "resolutions": out}
    print(json.dumps(line), flush=True)
    ctx.close()


def octree_bench(args, soc, torch, W):
    """The octree workload: 64^3 root cells with three refinement levels
    where the density exceeds 4x the mean (4.68 M leaves), a lognormal cloud
    with a central dense core (tau_V 100 from the centre to the edge), a
    10^4 K source of 10^6 L_sun inside the core and the external field, 128
    frequencies, 10^7 packages per frequency (half from the field, half
    from the source).  The persistent kernel's launch schedule is tuned by
    the autotuner on one-launch calibration passes (every 8th frequency at
    10^6 packages); the whole 128-frequency pass is then timed with the
    default and with the tuned schedule, and the faster of the two runs the
    one-launch form.  CPU
    baseline: the oracle on a sample of the same packages."""
    from paper_1812_06632_amd import autotune

    t0 = time.time()
    G = W.octree_lognormal(n_root=64, nlevels=4)
    nu, w = W.frequency_grid(128)
    sabs, ssca, gg = W.dust_model(nu)
    log(f"octree: {G.ncells} cells, {int((G.words.view(np.int32) >= 0).sum())} leaves ({time.time() - t0:.1f}s)")
    ctx = soc.Context(0)
    g = soc.grid_from_workload(ctx, G)
    A = torch.zeros(G.ncells, dtype=torch.float64, device="cuda")
    pos = [[32.1, 31.9, 32.05]]
    freqs = [(float(nu[k]), float(w[k]), float(sabs[k]), float(ssca[k]), float(gg[k])) for k in range(len(nu))]
    I = W.isrf(nu)
    Lnu = W.blackbody_Lnu(nu, 1e6 * W.L_SUN, 1e4)
    n_half = 5_000_000

    def one(k, n):
        soc.simulate_frequency(ctx, g, freqs[k], A, I_bg=float(I[k]), ps_pos=pos, ps_Lnu=[float(Lnu[k])], n_bg=n,
                               n_ps_pk=n, seed=1, iteration=1, freq_index=k)

    src = [dict(I_bg=float(I[k]), ps_pos=pos, ps_Lnu=[float(Lnu[k])], n_bg=n_half, n_ps_pk=n_half)
           for k in range(len(nu))]

    def full_pass(multi=False):
        A.zero_()
        ctx.read_stats(reset=True)
        torch.cuda.synchronize()
        t = time.time()
        if multi:
            soc.simulate_frequencies(ctx, g, freqs, A, src, range(len(nu)), seed=1, iteration=1)   # one launch
        else:
            for k in range(len(nu)):
                one(k, n_half)
        torch.cuda.synchronize()
        el = time.time() - t
        st = ctx.read_stats(reset=True)
        return el, st

    # calibration: the one-launch form at every 8th frequency, 10^6 packages
    # each (one launch of 16 frequencies, so its tail weighs as in the pass)
    ks = [int(np.argmin(np.abs(np.log(2.99792458e14 / nu / l)))) for l in (0.55, 100.0)]
    tau_cell = float(sabs[ks[0]] + ssca[ks[0]]) * float(np.median(G.density()[G.density() > 0])) * G.root_cell_cm
    key = autotune.class_key("octree", G.ncells, tau_cell, "bg+ps")
    sub = list(range(0, len(nu), 8))
    src_cal = [dict(src[k], n_bg=500_000, n_ps_pk=500_000) for k in sub]

    def calibrate(cfg):
        soc.simulate_frequencies(ctx, g, [freqs[k] for k in sub], A, src_cal, sub, seed=1, iteration=1)

    measure = autotune.event_timer(ctx, calibrate)
    defaults = {n: ctx.get_option(n) for n in autotune.DEFAULT_SPACE}
    t0 = time.time()
    best = autotune.Autotuner().tune(key, measure)
    log(f"octree: autotuned {best} in {time.time() - t0:.1f}s (default {defaults})")
    autotune.apply(ctx, defaults)
    one(ks[0], n_half)   # warm-up
    t_def, st_def = full_pass()
    autotune.apply(ctx, best)
    t_tuned, st = full_pass()
    # keep whichever schedule is faster on the whole pass for the
    # one-launch form
    if t_def < t_tuned:
        best, t_tuned, st = defaults, t_def, st_def
        autotune.apply(ctx, best)
    t_multi, _ = full_pass(multi=True)
    ctx.set_option("multi_spread", 0)   # one launch, each frequency drained by all waves in turn
    t_multi_seq, _ = full_pass(multi=True)
    ctx.set_option("multi_spread", 1)
    log(f"octree: 128 frequencies x 10^7 packages: default schedule {t_def:.2f}s, kept {best} {t_tuned:.2f}s, "
        f"one launch {t_multi:.2f}s (frequencies in turn: {t_multi_seq:.2f}s)")
    cons = (st["e_absorbed"] + st["e_escaped"]) / st["e_emitted"] - 1.0
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import orc
        ncpu = host_cpu()[0]
        t1 = time.time()
        n_pk = n_st = 0
        for k in ks:
            _, so, _ = orc.simulate_frequency(G, freqs[k], I_bg=float(I[k]), ps_pos=pos, ps_Lnu=[float(Lnu[k])],
                                              n_bg=4_000_000, n_ps_pk=4_000_000, seed=1, iteration=1, freq_index=k,
                                              nthreads=ncpu)
            n_pk += so["packages"]
            n_st += so["cell_steps"]
        tc = time.time() - t1
        cpu = {"value": n_pk / tc, "unit": "packages/s", "cores": ncpu, "kind": "oracle",
               "cell_steps_per_s": n_st / tc,
               "sample": f"8 x 10^6 packages at each of frequencies {ks} of the same octree and sources "
                         f"(FP64 C oracle, OpenMP)"}
        log(f"oracle: {n_pk} packages in {tc:.2f}s")
    line = {"kind": "octree", "workload": "octree 64^3 root + 3 levels (4.68 M leaves), central core tau_V 100, "
                                          "10^4 K source of 10^6 L_sun + external field, 128 frequencies, "
                                          "10^7 packages/frequency",
            "packages": st["packages"], "cell_steps": st["cell_steps"], "s_per_pass": min(t_multi, t_tuned),
            "form": "one launch" if t_multi <= t_tuned else "one launch per frequency",
            "s_per_pass_one_launch": t_multi, "s_per_pass_one_launch_frequencies_in_turn": t_multi_seq,
            "s_per_pass_per_frequency_launches": t_tuned,
            "packages_per_s": st["packages"] / min(t_multi, t_tuned),
            "cell_steps_per_s": st["cell_steps"] / min(t_multi, t_tuned),
            "s_per_pass_default_schedule": t_def, "schedule": best, "energy_conservation": cons,
            "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)
    ctx.close()


def scatter_bench(args, soc, torch, W):
    """Scattered-light image (forced first scattering, peel-off of every
    scattering, Sect. 2.1.1) of the benchmark cloud at 0.55 um, seen along
    +z: external field and the two point sources, --packages packages.  The
    work is dominated by the rays from every scattering to the boundary; a
    ray step is one dependent 4-byte density gather, so the bound is the
    measured dependent-gather rate.  CPU baseline: the oracle on a sample."""
    P = W.lognormal_problem(n=args.n, K=args.freqs, packages_per_freq=args.packages)
    lam = 2.99792458e14 / P.nu
    k = int(np.argmin(np.abs(np.log(lam / 0.55))))
    f = (float(P.nu[k]), float(P.w[k]), float(P.sigma_abs[k]), float(P.sigma_sca[k]), float(P.g[k]))
    ctx = soc.Context(0)
    g = soc.grid_from_workload(ctx, P.grid)
    kw = dict(axis=2, forced=True, I_bg=float(P.I_bg[k]), ps_pos=P.ps_pos, ps_Lnu=P.ps_Lnu[:, k], n_bg=P.n_bg,
              n_ps_pk=P.n_ps_pk, iteration=1, freq_index=k)
    img = torch.zeros(soc.scatter_image_shape(g, 2), dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        soc.scatter_map(ctx, g, f, img, seed=99, stats=True, **kw)
    tot = {"packages": 0, "cell_steps": 0, "scatterings": 0, "ray_steps": 0}
    torch.cuda.synchronize()
    t0 = time.time()
    for i in range(args.steps):
        st = soc.scatter_map(ctx, g, f, img, seed=i + 1, stats=True, **kw)
        for key in tot:
            tot[key] += st[key]
    torch.cuda.synchronize()
    el = time.time() - t0
    w = torch.randint(0, 2**31 - 1, (P.grid.ncells,), dtype=torch.int32, device="cuda")
    out = torch.zeros(4, dtype=torch.int32, device="cuda")
    soc.ubench(ctx, 1, w, out, P.grid.ncells, 64, 0, 16384, 256)
    gather = 16384 * 256 * 64 / (min(soc.ubench(ctx, 1, w, out, P.grid.ncells, 64, 0, 16384, 256)
                                     for _ in range(3)) * 1e-3)
    steps_per_s = (tot["cell_steps"] + tot["ray_steps"]) / el
    log(f"scattered light: {args.steps} images in {el:.3f}s, {tot['packages'] / el:.3e} packages/s, "
        f"{tot['scatterings'] / el:.3e} peel-offs/s, {steps_per_s:.3e} steps/s (ray steps "
        f"{tot['ray_steps'] / max(tot['cell_steps'] + tot['ray_steps'], 1):.2f} of all), gather ceiling {gather:.3e}/s")
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import orc
        n_s = 20 * args.packages   # about 10 s on 16 host threads
        kw_s = dict(kw)
        kw_s["n_bg"], kw_s["n_ps_pk"] = n_s // 2, n_s // 4
        nthreads = host_cpu()[0]
        t1 = time.time()
        _, so = orc.scatter_map(P.grid, f, seed=5, nthreads=nthreads, **kw_s)
        el_c = time.time() - t1
        cpu = {"value": so["packages"] / el_c, "unit": "packages/s", "cores": nthreads, "kind": "oracle",
               "sample": f"{so['packages']} packages of the same image (FP64 C oracle, OpenMP)"}
        log(f"oracle: {so['packages']} packages in {el_c:.2f}s")
    line = {"kind": "scatter_map", "workload": f"lognormal {args.n}^3, 0.55 um, external field + 2 point sources, "
                                               f"{args.packages} packages, forced first scattering, peel-off towards +z",
            "steps": args.steps, "ms_per_image": el / args.steps * 1e3, "packages_per_s": tot["packages"] / el,
            "peel_offs_per_s": tot["scatterings"] / el, "steps_per_s": steps_per_s,
            "ray_step_fraction": tot["ray_steps"] / max(tot["cell_steps"] + tot["ray_steps"], 1),
            "roofline": {"bound": "dependent 4-byte gathers (measured)", "achieved": steps_per_s, "peak": gather,
                         "unit": "steps/s", "frac": steps_per_s / gather,
                         "hbm_GBs_algorithmic": 4.0 * steps_per_s / 1e9},
            "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)
    ctx.close()


def shg_bench(args, soc, torch, W):
    """Stochastically heated grains (Sect. 2.1.1, Appendix A) on the
    benchmark cloud: one Monte Carlo pass of the constant sources at each of
    the --freqs frequencies into its own absorbed-energy array (the grain
    model's cross sections), then the temperature distributions of
    --shg-sizes grain sizes on --shg-bins enthalpy bins and the emission of
    every cell at every frequency.  The paper's laptop GPU needed 0.5 ms per
    cell for 25 sizes and 128 frequencies (App. A).  CPU baseline: the
    oracle on a sample of cells."""
    import dataclasses

    P0 = W.lognormal_problem(n=args.n, K=args.freqs, packages_per_freq=args.packages)
    G = W.grain_model(P0.nu, P0.w, n_size=args.shg_sizes, n_enthalpy=args.shg_bins)
    P = dataclasses.replace(P0, sigma_abs=G.sigma_per_H, emit_sigma_abs=G.sigma_per_H)
    ctx = soc.Context(0)
    g = soc.grid_from_workload(ctx, P.grid)
    nc = P.grid.ncells
    from paper_1812_06632_amd.driver import absorbed_spectra
    torch.cuda.synchronize()
    t0 = time.time()
    A = absorbed_spectra(ctx, g, P, seed=1, iteration=1)
    torch.cuda.synchronize()
    t_mc = time.time() - t0
    log(f"SHG: {P.K} Monte Carlo passes {t_mc:.3f}s")
    model = soc.ShgModel(ctx, G)
    E = torch.zeros_like(A)
    t0 = time.time()
    soc.shg_solve(ctx, g, model, A, E)       # warm-up
    torch.cuda.synchronize()
    log(f"SHG: first solve {time.time() - t0:.3f}s")
    t0 = time.time()
    for _ in range(args.steps):
        soc.shg_solve(ctx, g, model, A, E)
    torch.cuda.synchronize()
    t_shg = (time.time() - t0) / args.steps
    leaves = int((P.grid.density() > 0).sum())
    flops_cell_size = 2.0 * args.shg_bins * P.K + 2.0 * args.shg_bins * args.shg_bins   # emission sum + substitution
    rate = leaves / t_shg
    log(f"SHG: {P.K} MC passes {t_mc:.3f}s; solve {t_shg * 1e3:.2f} ms for {leaves} cells x {args.shg_sizes} sizes "
        f"x {args.shg_bins} bins = {rate:.3e} cells/s")
    emitted = float((E * torch.from_numpy(P.w).cuda()[:, None]).sum())
    absorbed = float(A.sum())
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import shg_oracle as O
        Ah = A[:, :: max(1, nc // 4096)].cpu().numpy()
        rho = P.grid.density()[:: max(1, nc // 4096)].astype(np.float64)
        V = P.grid.root_cell_cm ** 3
        n_s = 0
        t1 = time.time()
        for c in range(Ah.shape[1]):
            if rho[c] > 0:
                O.solve_cell(G, Ah[:, c], rho[c] * V)
                n_s += 1
            if time.time() - t1 > 10.0:
                break
        el = time.time() - t1
        cpu = {"value": n_s / el, "unit": "cells/s", "cores": 1, "kind": "oracle",
               "sample": f"{n_s} cells of the same cloud (FP64 numpy oracle, one thread)"}
        log(f"oracle: {n_s} cells in {el:.2f}s")
    line = {"kind": "shg", "workload": f"lognormal {args.n}^3 benchmark cloud, {P.K} frequencies, constant sources "
                                       f"({args.packages} packages/frequency), {args.shg_sizes} grain sizes, "
                                       f"{args.shg_bins} enthalpy bins", "cells": leaves,
            "mc_s": t_mc, "solve_ms": t_shg * 1e3, "cells_per_s": rate,
            "paper_laptop_cells_per_s_25_sizes_128_freq": 2000.0,
            "emitted_over_absorbed": emitted / absorbed,
            "roofline": {"bound": "alu (fp64)", "achieved": rate * args.shg_sizes * flops_cell_size / 1e12,
                         "peak": 78.6, "unit": "TFLOP/s",
                         "frac": rate * args.shg_sizes * flops_cell_size / 1e12 / 78.6,
                         "flops_per_cell_and_size": flops_cell_size},
            "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)
    model.close()
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--freqs", type=int, default=64)
    ap.add_argument("--packages", type=int, default=1_000_000)
    ap.add_argument("--max-iter", type=int, default=12, help="iterations at most of each learned-start run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-converge", action="store_true",
                    help="skip the time-to-1%% runs (plain and learned start)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned start in the time-to-1%% runs")
    ap.add_argument("--no-sub-records", action="store_true",
                    help="skip the one-pass octree and batch records of the default line")
    ap.add_argument("--lt-clouds", type=int, default=96, help="training clouds of the in-run learned start")
    ap.add_argument("--lt-packages", type=int, default=100_000, help="their packages per frequency")
    ap.add_argument("--lt-steps", type=int, default=1500, help="training steps of the in-run learned start")
    ap.add_argument("--ceilings", action="store_true",
                    help="only run the device micro-benchmarks (one JSON line each) and exit")
    ap.add_argument("--surrogate", action="store_true",
                    help="only run the learned-start gain test (one JSON line) and exit")
    ap.add_argument("--unet", action="store_true",
                    help="only time the U-Net training step (64^3, base 32, 4 levels; one JSON line) and exit")
    ap.add_argument("--unet-batch", type=int, default=4)
    ap.add_argument("--batch", action="store_true",
                    help="only time the batched many-cloud workload as a replayed HIP graph (one JSON line) and exit")
    ap.add_argument("--batch-models", type=int, default=256)
    ap.add_argument("--batch-freqs", type=int, default=32)
    ap.add_argument("--tile", type=int, default=16384, help="tile size when the batch schedule is not tuned")
    ap.add_argument("--no-tune", action="store_true", help="batch: default schedule, no autotuning")
    ap.add_argument("--train-clouds", type=int, default=2000)
    ap.add_argument("--val-clouds", type=int, default=48)
    ap.add_argument("--train-packages", type=int, default=100_000)
    ap.add_argument("--curve", default="250,500,1000", help="training-set sizes of the learning curve")
    ap.add_argument("--target-n", type=int, default=256)
    ap.add_argument("--target-sigma", type=float, default=1.5)
    ap.add_argument("--target-tau", type=float, default=50.0)
    ap.add_argument("--target-packages", type=int, default=1_562_500)
    ap.add_argument("--ref-burn", type=int, default=12)
    ap.add_argument("--ref-avg", type=int, default=8)
    ap.add_argument("--train-steps", type=int, default=5000)
    ap.add_argument("--reference", action="store_true",
                    help="plain versus reference-field iteration, constant and growing package counts")
    ap.add_argument("--ref-iters", type=int, default=10)
    ap.add_argument("--ref-factor", type=float, default=16.0)
    ap.add_argument("--ali", action="store_true", help="plain versus diagonal-ALI iteration at three resolutions")
    ap.add_argument("--scatter", action="store_true", help="scattered-light image by forced scattering and peel-off")
    ap.add_argument("--shg", action="store_true", help="stochastically heated grains on the benchmark cloud")
    ap.add_argument("--octree", action="store_true", help="the octree workload with an autotuned launch schedule")
    ap.add_argument("--shg-sizes", type=int, default=25)
    ap.add_argument("--shg-bins", type=int, default=128)
    ap.add_argument("--ali-iters", type=int, default=20)
    ap.add_argument("--ali-ref-iters", type=int, default=60)
    ap.add_argument("--ali-tau", type=float, default=500.0)
    ap.add_argument("--ali-box", type=float, default=0.05)
    ap.add_argument("--ali-lsun", type=float, default=1.0e5)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (several GPUs would each take a "
              "range of package ids and sum their absorbed energy with one all-reduce per iteration).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1812_06632_amd import soc, workloads as W

    if args.ceilings:
        ceilings(soc, torch, args.n ** 3)
        return
    if args.surrogate:
        surrogate_gain(args, soc, torch, W)
        return
    if args.unet:
        unet_step(args, soc, torch)
        return
    if args.batch:
        batch_bench(args, soc, torch, W)
        return
    if args.reference:
        reference_gain(args, soc, torch, W)
        return
    if args.ali:
        ali_gain(args, soc, torch, W)
        return
    if args.scatter:
        scatter_bench(args, soc, torch, W)
        return
    if args.shg:
        shg_bench(args, soc, torch, W)
        return
    if args.octree:
        octree_bench(args, soc, torch, W)
        return

    headline(args, soc, torch, W)


def host_cpu():
    """(threads the oracle may use, nproc, CPU model): the threads are the
    OpenMP setting if one is made, else every CPU this process may run on."""
    nproc = os.cpu_count() or 1
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = nproc
    omp = os.environ.get("OMP_NUM_THREADS")
    threads = int(omp) if omp and omp.isdigit() and int(omp) > 0 else allowed
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return threads, nproc, allowed, model


class RefCriterion:
    """The paper's two convergence statistics (Sect. 3.3) taken against a
    reference field: mean |T - T_ref| / T_ref over the cells with dust and
    over the hottest 5% of them (by T_ref)."""

    def __init__(self, torch, T_ref, dense):
        self.torch = torch
        self.dense = dense
        self.Tr = T_ref.double()[dense]
        srt = torch.sort(self.Tr)[0]
        self.hot = self.Tr >= srt[int(0.95 * (srt.numel() - 1))]

    def __call__(self, T):
        r = (T.double().reshape(-1)[self.dense] - self.Tr).abs() / self.Tr
        return r.mean().item(), r[self.hot].mean().item()


def timed_to_criterion(torch, S, crit, start=None, max_iter=8, tol=0.01, run_on=False):
    """Wall clock of one run of the solver from its constant pass until the
    end of the first iteration whose temperatures are within tol of the
    reference field on both statistics.  start(S), if given, runs after the
    constant pass and sets the state the dust iterations start from.  The
    criterion is evaluated outside the clock.  With run_on the run goes on
    to max_iter (and to the plain stopping rule) after meeting it.  Returns
    (seconds or None, iterations or None, stopping-rule iteration or None,
    [(iteration, seconds, err_all, err_hot5, <T>, hot5 <T>)])."""
    from paper_1812_06632_amd.driver import converged
    torch.cuda.synchronize()
    t0 = time.time()
    paused = 0.0
    st = S.constant_pass()
    if start is not None:
        st = start(S)
    torch.cuda.synchronize()
    hist = []
    it = 1
    hit = None
    stop = None
    prev = None
    while True:
        t_it = time.time() - t0 - paused
        tp = time.time()
        e = crit(S.T)
        paused += time.time() - tp
        hist.append((it, t_it, e[0], e[1], st["mean_T"], st["hot5_mean_T"]))
        if hit is None and e[0] < tol and e[1] < tol:
            hit = (t_it, it)
        if stop is None and prev is not None and converged(prev, st, tol):
            stop = it
        if (hit is not None and not run_on) or it >= max_iter or (run_on and hit and stop):
            return (hit[0] if hit else None), (hit[1] if hit else None), stop, hist
        prev = st
        it += 1
        st = S.dust_iteration(it)
        torch.cuda.synchronize()


def octree_record(soc, torch, W):
    """One 128-frequency pass of the octree workload (as `--octree`, 10^7
    packages per frequency) in one launch with the library's default
    schedule: packages/s and cell steps/s."""
    t0 = time.time()
    G = W.octree_lognormal(n_root=64, nlevels=4)
    nu, w = W.frequency_grid(128)
    sabs, ssca, gg = W.dust_model(nu)
    t_build = time.time() - t0
    ctx = soc.Context(0)
    g = soc.grid_from_workload(ctx, G)
    A = torch.zeros(G.ncells, dtype=torch.float64, device="cuda")
    pos = [[32.1, 31.9, 32.05]]
    I = W.isrf(nu)
    Lnu = W.blackbody_Lnu(nu, 1e6 * W.L_SUN, 1e4)
    freqs = [(float(nu[k]), float(w[k]), float(sabs[k]), float(ssca[k]), float(gg[k])) for k in range(len(nu))]

    src = [dict(I_bg=float(I[k]), ps_pos=pos, ps_Lnu=[float(Lnu[k])], n_bg=5_000_000, n_ps_pk=5_000_000)
           for k in range(len(nu))]
    soc.simulate_frequency(ctx, g, freqs[len(nu) // 2], A, I_bg=float(I[len(nu) // 2]), ps_pos=pos,
                           ps_Lnu=[float(Lnu[len(nu) // 2])], n_bg=500_000, n_ps_pk=500_000, seed=1, iteration=1,
                           freq_index=len(nu) // 2)   # warm-up
    A.zero_()
    ctx.read_stats(reset=True)
    torch.cuda.synchronize()
    t0 = time.time()
    soc.simulate_frequencies(ctx, g, freqs, A, src, range(len(nu)), seed=1, iteration=1)   # one launch
    torch.cuda.synchronize()
    el = time.time() - t0
    st = ctx.read_stats(reset=True)
    ctx.close()
    log(f"octree pass: {el:.2f}s, {st['packages'] / el:.3e} packages/s (host build {t_build:.1f}s)")
    return {"workload": "octree 64^3 root + 3 levels (4.68 M leaves), central core tau_V 100, 10^4 K source of "
                        "10^6 L_sun + external field, 128 frequencies, 10^7 packages/frequency, one launch, "
                        "default schedule",
            "s_per_pass": el, "packages_per_s": st["packages"] / el, "cell_steps_per_s": st["cell_steps"] / el,
            "energy_conservation": (st["e_absorbed"] + st["e_escaped"]) / st["e_emitted"] - 1.0}


def batch_record(soc, torch, W):
    """One pass of the batched workload (as `--batch`: 256 clouds of 16^3-96^3
    cells, 32 frequencies, one persistent launch, replayed HIP graph) with
    the default schedule: packages/s and cell steps/s."""
    grids, (nu, w, sabs, ssca, g, I), pk = W.batch_clouds(256, 32)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx = soc.Context(0, stream=s)
        G = [soc.grid_from_workload(ctx, gr) for gr in grids]
        table = soc.temp_table_build(ctx, nu, w, sabs, 2.0, 3000.0, 1024)
        A = [torch.zeros(gr.ncells, dtype=torch.float64, device="cuda") for gr in grids]
        T = [torch.zeros(gr.ncells, dtype=torch.float32, device="cuda") for gr in grids]
        pairs = [dict(grid=m, freq=(float(nu[k]), float(w[k]), float(sabs[k]), float(ssca[k]), float(g[k])),
                      freq_index=k, I_bg=float(I[k]), n_bg=int(pk[m, k]), absorbed=A[m])
                 for m in range(len(grids)) for k in range(len(nu))]
        b = soc.Batch(ctx, G, pairs, seed=1, tile_packages=16384)
        b.run(iteration=0)
        torch.cuda.synchronize()
        soc.graph_begin(ctx)
        for a in A:
            a.zero_()
        b.run(iteration=soc.ITER_ADVANCE)
        for m in range(len(grids)):
            soc.update_temperature(ctx, G[m], table, A[m], T[m])
        graph = soc.graph_end(ctx)
        graph.launch()
        torch.cuda.synchronize()
        before = ctx.read_stats()
        t0 = time.time()
        graph.launch()
        torch.cuda.synchronize()
        el = time.time() - t0
        after = ctx.read_stats()
    graph.close()
    b.close()
    ctx.close()
    n_pk = after["packages"] - before["packages"]
    log(f"batch pass: {el:.2f}s, {n_pk / el:.3e} packages/s")
    return {"workload": "256 lognormal clouds of 16^3-96^3 cells, 32 frequencies, 1e5-1e6 packages per pair, one "
                        "persistent launch + temperature updates in a replayed HIP graph, default schedule",
            "s_per_pass": el, "packages_per_s": n_pk / el,
            "cell_steps_per_s": (after["cell_steps"] - before["cell_steps"]) / el}


def headline(args, soc, torch, W):
    """The benchmark workload: dust-iteration throughput, the time to 1%
    temperature convergence of the plain method and of the learned start,
    the roofline of the MC kernel and the oracle on the host."""
    from paper_1812_06632_amd.driver import PlainSolver, converged

    t_setup = time.time()
    P = W.lognormal_problem(n=args.n, K=args.freqs, packages_per_freq=args.packages)
    K = P.K
    ctx = soc.Context(0)
    ctx.set_option("timing", 1)
    S = PlainSolver(ctx, P, seed=1)
    nc = P.grid.ncells
    freqs = S.freqs
    log(f"setup {time.time() - t_setup:.1f}s: {args.n}^3 cells, {K} frequencies, {args.packages} packages/freq")

    # ---- iteration 1: constant sources
    torch.cuda.synchronize()
    t0 = time.time()
    tst = S.constant_pass()
    torch.cuda.synchronize()
    t_const = time.time() - t0
    st_const = ctx.read_stats(reset=True)
    ctx.mc_timing(reset=True)
    log(f"iteration 1 (constant sources): {t_const:.3f}s, <T> {tst['mean_T']:.2f} K, hot5 {tst['hot5_mean_T']:.2f} K")
    history = [(1, tst)]

    it = 2
    for _ in range(args.warmup):
        s = S.dust_iteration(it)
        history.append((it, s))
        log(f"warmup iteration {it}: <T> {s['mean_T']:.3f} K hot5 {s['hot5_mean_T']:.3f} K")
        it += 1
    ctx.read_stats(reset=True)
    ctx.mc_timing(reset=True)
    T_sum = torch.zeros(nc, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(args.steps):
        s = S.dust_iteration(it)
        T_sum += S.T   # the reference field: mean of the timed iterations (one small add per step)
        history.append((it, s))
        log(f"timed iteration {it}: <T> {s['mean_T']:.3f} K hot5 {s['hot5_mean_T']:.3f} K")
        it += 1
    torch.cuda.synchronize()
    elapsed = time.time() - t0
    st = ctx.read_stats(reset=True)
    mc_ms, mc_launches = ctx.mc_timing(reset=True)
    ctx.set_option("timing", 0)
    pk_per_s = st["packages"] / elapsed
    steps_per_s = st["cell_steps"] / elapsed
    avg_launch_s = mc_ms / 1e3 / max(mc_launches, 1)
    steps_per_launch = st["cell_steps"] / max(mc_launches, 1)
    achieved = BYTES_PER_STEP * steps_per_launch / avg_launch_s / 1e9
    log(f"timed: {elapsed:.3f}s for {args.steps} iterations, {pk_per_s:.3e} packages/s, {steps_per_s:.3e} "
        f"cell-steps/s, MC kernel avg {avg_launch_s * 1e3:.3f} ms/launch")
    atomic_ceiling, copy_gbs = device_ceilings(soc, ctx, torch, nc)
    log(f"ceilings: random FP64 atomics {atomic_ceiling:.3e}/s over {nc} doubles, copy {copy_gbs:.0f} GB/s")

    # ---- the stopping rule of the plain method (change between iterations)
    stop_iter = None
    for i in range(1, len(history)):
        if converged(history[i - 1][1], history[i][1]):
            stop_iter = history[i][0]
            break
    T = S.T

    # ---- time to 1% of the reference field, plain and learned start
    conv = None
    if not args.no_converge:
        T_ref = (T_sum / max(args.steps, 1)).float()
        dense = torch.from_numpy(P.grid.density()).cuda() > 0
        crit = RefCriterion(torch, T_ref, dense)
        conv = {"criterion": "mean |T - T_ref| / T_ref < 1% over all cells with dust and over the hottest 5% "
                             "of them (by T_ref)",
                "T_ref": f"mean temperature of the {args.steps} timed iterations of the plain run (iterations "
                         f"{2 + args.warmup}-{1 + args.warmup + args.steps}), same seed and constant-source "
                         f"pass as the timed runs",
                "T_ref_mean_K": float(crit.Tr.mean().item()), "T_ref_hot5_mean_K": float(crit.Tr[crit.hot].mean().item())}
        Sp = PlainSolver(ctx, P, seed=1)
        t_plain, n_plain, _, h_plain = timed_to_criterion(torch, Sp, crit)
        log(f"plain: within 1% of T_ref at iteration {n_plain} after {t_plain}s  {h_plain}")
        conv.update({"plain_s": t_plain, "plain_iterations": n_plain,
                     "plain_err_by_iteration": [[h[0], round(h[1], 4), round(h[2], 5), round(h[3], 5)]
                                                for h in h_plain]})
        if not args.no_learned:
            from paper_1812_06632_amd.surrogate import Surrogate, make_dataset
            t0 = time.time()
            X, Y = make_dataset(ctx, args.lt_clouds, seed=11, n=64, S=64, K=32, packages=args.lt_packages, log=log)
            t_data = time.time() - t0
            sur = Surrogate(ctx, S=64, base=32, levels=4, batch=4, seed=3)
            t0 = time.time()
            losses = sur.fit(X, Y, steps=args.lt_steps, lr=5e-4, log=log)
            torch.cuda.synchronize()
            t_train = time.time() - t0
            del X, Y
            Ss = PlainSolver(ctx, P, seed=1)
            t_sur, n_sur, _, h_sur = timed_to_criterion(torch, Ss, crit,
                                                        start=lambda s_: s_.set_temperature(sur.predict_T(s_, s_.T)))
            log(f"learned start: within 1% of T_ref at iteration {n_sur} after {t_sur}s  {h_sur}")
            conv.update({"surrogate_s": t_sur, "surrogate_iterations": n_sur,
                         "surrogate_err_by_iteration": [[h[0], round(h[1], 4), round(h[2], 5), round(h[3], 5)]
                                                        for h in h_sur],
                         "speedup": (t_plain / t_sur) if (t_plain and t_sur) else None,
                         "training": {"clouds": args.lt_clouds, "cells": "64^3", "frequencies": 32,
                                      "packages_per_frequency": args.lt_packages, "steps": args.lt_steps,
                                      "batch": 4, "network": "U-Net 4 levels, base 32, BF16 MFMA, trained in this run",
                                      "data_s": t_data, "train_s": t_train,
                                      "final_loss": losses[-1][1] if losses else None,
                                      "params": sur.net.param_count}})
            sur.close()

    # ---- CPU baseline: the oracle on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import orc
        threads, nproc, allowed, model = host_cpu()
        Th = T.cpu().numpy()
        sample_f = [i * K // 5 for i in range(1, 5)]   # about 10-15 s of oracle work
        npk = 10_000_000
        t0 = time.time()
        tot_pk = tot_st = 0
        for k in sample_f:
            _, so, _ = orc.simulate_frequency(P.grid, freqs[k], T=Th, n_dust=npk, dust_mode=1, seed=1,
                                              iteration=it, freq_index=k, nthreads=threads)
            tot_pk += so["packages"]
            tot_st += so["cell_steps"]
            log(f"cpu oracle: frequency {k} done ({time.time() - t0:.1f}s)")
        tcpu = time.time() - t0
        cpu = {"value": tot_pk / tcpu, "unit": "packages/s", "cores": threads, "kind": "oracle",
               "cell_steps_per_s": tot_st / tcpu, "nproc": nproc, "cpus_allowed": allowed, "cpu_model": model,
               "sample": f"dust emission, {npk} weighted packages at each of frequencies {sample_f} of the "
                         f"same {args.n}^3 workload and temperatures (FP64 C oracle, OpenMP, {threads} threads)"}

    subs = None
    if not args.no_sub_records:
        subs = {"octree": octree_record(soc, torch, W), "batch": batch_record(soc, torch, W)}

    traffic, tx_per_step = recorded_counters()
    out = {
        "metric": "photon packages/s",
        "value": pk_per_s,
        "unit": "packages/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"lognormal {args.n}^3 regular grid, sigma_ln 1, mean tau_V 5, {K} frequencies "
                               f"0.1-3000 um, external field + 2 point sources, {args.packages} packages/frequency, "
                               f"dust re-emission iterations (luminosity-weighted)",
                   "packages_per_step": K * P.n_dust, "cells": nc},
        "cell_steps_per_s": steps_per_s,
        "const_sources_packages_per_s": st_const["packages"] / t_const,
        "time_to_1pct_T_s": conv["plain_s"] if conv else None,
        "time_to_1pct_T_surrogate_s": conv.get("surrogate_s") if conv else None,
        "time_to_1pct": conv,
        "stopping_rule_iteration": stop_iter,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": MC_KERNEL, "avg_launch_ms": avg_launch_s * 1e3,
                     "cell_steps_per_launch": steps_per_launch, "bytes_per_cell_step": BYTES_PER_STEP,
                     "binding": "memory-side FP64 atomic transactions (one per deposit, except that the deposits "
                                "of one atomic instruction in one 64-byte line merge), not HBM bytes",
                     "atomic_ceiling_per_s": atomic_ceiling,
                     "atomic_transactions_per_cell_step": tx_per_step,
                     "atomic_frac": (steps_per_launch / avg_launch_s * tx_per_step / atomic_ceiling
                                     if tx_per_step else None),
                     "cell_steps_per_s_over_atomic_ceiling": steps_per_launch / avg_launch_s / atomic_ceiling,
                     "copy_GBs": copy_gbs},
        "cpu_baseline": cpu,
        "other_workloads": subs,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
