#!/usr/bin/env python3
"""Benchmark of one blocked-linear-method step on one MI355X.

Workload (FP64): N_V = 4,096 parameters in 8 blocks of 512, N_s = 1,000,000
samples in 65,536-sample chunks (15 full + a 16,960 tail), low-rank synthetic
derivative ratios (rank 32), N_K = 5 kept directions per block, N_O = 1
previous-update direction, shifts {1e-4, 1e-3, 1e-2} solved together.

A step is: begin_step (previous direction) -> build over all chunks ->
block solves -> projection over all chunks -> stage two.  The sample chunks
are generated on the device before timing and stay resident in HBM.  The
previous direction is the update of one untimed step without history on the
same data (shift 1e-3).

Prints one JSON line.  Value: build FLOP (the algorithmic count
2 N_s sum_b [d_b^2 + d_b (d_b + 1)/2], d_b = 1 + M_b + N_O (N_B - 1)) per
second of whole step time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "block H/S build TFLOP/s + BLM step ms; mixed vs FP64 at ≤1e-6 rel energy err"
PEAK_FP64 = 78.6      # TFLOP/s, MI355X dense FP64 (matrix and vector)

# HBM bytes of one FP64 block-build launch on this workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by what the same
# counter reads for a plain 2 GiB copy (FETCH x2, WRITE x1).  Valid only for
# the kernel source they were taken on: reported as null once the source of
# the sample-streaming kernels has changed.
GRAM_TRAFFIC = {
    "source_sha256": "efb1445a42c5dedbd4054a361353706c5d16088e674403c757e64cff90ba5875",
    "fetch_scale": 1.99996, "write_scale": 1.0,
    # slice groups per tile -> (FETCH_SIZE, WRITE_SIZE) KiB per launch
    "by_groups": {1: (105566351.0, 27200.0), 2: (230332281.0, 54400.0), 3: (229755819.0, 81600.0),
                  4: (233044943.0, 108800.0), 6: (231931632.0, 163200.0), 8: (232274965.0, 217600.0),
                  12: (231207027.0, 326400.0), 15: (230408402.0, 408000.0)},
}


def gram_source_digest():
    """SHA-256 of the Gram-tile section of the FP64 kernel source (from its
    section header to the projection's): the counters below were taken on
    that code, and are reported only while it is unchanged."""
    import hashlib
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1702_01481_amd", "csrc",
                       "blm_kernels.hip")
    try:
        text = open(src).read()
        a = text.index("// Gram tiles")
        b = text.index("// projection onto per-block directions")
    except (OSError, ValueError):
        return None
    return hashlib.sha256(text[a:b].encode()).hexdigest()


def gram_traffic_bytes(groups):
    """HBM bytes of one FP64 block-build launch with this many slice groups,
    from the rocprofv3 counters taken on the same Gram-tile source; None if
    the source has changed or the counters do not cover that launch shape."""
    t = GRAM_TRAFFIC
    if gram_source_digest() != t["source_sha256"] or groups not in t["by_groups"]:
        return None
    fetch, write = t["by_groups"][groups]
    return 1024.0 * (fetch * t["fetch_scale"] + write * t["write_scale"])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_flops(offsets, n_old, n_samples) -> float:
    nb = len(offsets) - 1
    tot = 0.0
    for b in range(nb):
        d = 1 + (offsets[b + 1] - offsets[b]) + n_old * (nb - 1)
        tot += d * d + d * (d + 1) / 2
    return 2.0 * n_samples * tot


def cpu_baseline(O0, e0, EL0, w, offsets, old, n_keep, shifts):
    """The oracle as it stands on the host cores: block estimates of one
    65,536-sample chunk, then the 24 block solves of those estimates."""
    from threadpoolctl import threadpool_info

    from oracle import blm_oracle as orc
    O = O0.cpu().numpy()
    e = e0.cpu().numpy()
    EL = EL0.cpu().numpy()
    n = O.shape[0]
    t0 = time.perf_counter()
    D = orc.previous_directions(old, np.asarray(offsets))
    probs, _ = orc.block_problems([(O, e, EL, None)], np.asarray(offsets), D)
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    for delta in shifts:
        for p in probs:
            orc.solve_block(p, delta, n_keep)
    t_solve = time.perf_counter() - t0
    fl = build_flops(offsets, 1 if old is not None else 0, n)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {
        "value": fl / t_build / 1e12,
        "unit": "TFLOP/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"block estimates of the first {n}-sample chunk at full N_V ({t_build:.2f} s), "
                   f"plus all {len(shifts) * len(probs)} block solves ({t_solve:.2f} s); "
                   f"host nproc={os.cpu_count()}"),
        "build_s": t_build,
        "solve_s": t_solve,
    }


def mixed_step(args, prec, w, chunks, old, offsets, shifts, n_samples, en64, upd64, ms64, build64, fl_build):
    """The same step with the sample contractions in mixed precision (BF16
    split pieces, or FP8 codes with BF16 residuals); the reduced-precision
    copies are made from the resident FP64 samples before timing."""
    import torch

    from paper_1702_01481_amd import blm
    if prec == "fp8":
        split = [(blm.Fp8Samples(O), blm.Fp8Samples(e), EL) for O, e, EL in chunks]
    else:
        pieces = 3 if prec == "bf16x3" else 2
        split = [(blm.SplitSamples(O, pieces), blm.SplitSamples(e, pieces), EL) for O, e, EL in chunks]
    torch.cuda.synchronize()
    log(f"packed {prec} storage")
    ctx = blm.BLM(w.n_params, offsets, w.n_keep, w.n_old, shifts, n_samples, precision=prec)
    ctx.set_timing(True)
    groups = None
    if not args.no_autotune:
        ctx.begin_step(old)
        groups = ctx.autotune(split)
        log(f"{prec} build: {groups} slice groups per tile")

    def step():
        ctx.begin_step(old)
        ctx.build(split)
        ctx.solve()
        ctx.project(split)
        return ctx.stage2()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    phase = {k: [] for k in blm.TIMING_NAMES}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        upd, en, _, _ = step()
        for k, v in ctx.timings().items():
            phase[k].append(v)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    ctx.close()
    del split
    torch.cuda.empty_cache()
    pm = {k: float(np.mean(v)) for k, v in phase.items()}
    build_ms = pm["theta_proj"] + pm["block_gram"] + pm["block_reduce"] + max(pm["block_strips"], 0.0)
    u64 = upd64.double().cpu().numpy()
    um = upd.double().cpu().numpy()
    cos = [float(u64[i] @ um[i] / (np.linalg.norm(u64[i]) * np.linalg.norm(um[i]))) for i in range(len(shifts))]
    rel = [float(abs(en[i] - en64[i]) / abs(en64[i])) for i in range(len(shifts))]
    log(f"{prec} step {ms:.1f} ms, energy rel err {rel}")
    return {
        "precision": prec,
        "ms_per_step": round(ms, 3),
        "build_ms": round(build_ms, 3),
        "build_tflops": round(fl_build / (build_ms * 1e-3) / 1e12, 4),
        "gram_ms": round(pm["block_gram"], 3),
        "gram_algorithmic_tflops": round(fl_build / (pm["block_gram"] * 1e-3) / 1e12, 4),
        "build_slice_groups": groups,
        "phase_ms": {k: round(v, 3) for k, v in pm.items()},
        "energy_rel_err_vs_fp64": rel,
        "update_cosine_vs_fp64": cos,
        "step_speedup_vs_fp64": round(ms64 / ms, 3),
        "build_speedup_vs_fp64": round(build64 / build_ms, 3),
        "meets_1e-6": bool(max(rel) <= 1e-6),
    }


def streamed_target(args):
    """The 30,000-parameter workload (40 uneven blocks, N_O = 0, delta = 1e-3)
    at its full 4,000,000 samples, whose samples (1.9 TB as FP64) do not fit
    in HBM: each 65,536-sample chunk is made on the device, handed to an FP64,
    a BF16 x3 and an FP8 context in turn (the mixed storage packed from it
    first) and dropped; the second pass makes the same chunks again.  Only
    the library calls are timed, with events on the shared stream: the
    generator and the producer-side packing are not part of the step."""
    import torch

    from paper_1702_01481_amd import blm, synth
    w = synth.workload("uneven")
    n_samples = args.streamed_samples or w.n_samples
    offsets, shifts = w.block_offsets, list(w.shifts)
    gen = synth.SampleGenerator(w.n_params, w.rank, w.seed, sigma_E=w.sigma_E, device="cuda")
    sizes, left = [], n_samples
    while left > 0:
        sizes.append(min(w.chunk, left))
        left -= sizes[-1]
    precs = ("fp64", "bf16x3", "fp8")
    ctxs = {p: blm.BLM(w.n_params, offsets, w.n_keep, w.n_old, shifts, w.chunk, precision=p) for p in precs}
    ms = {p: {"build": 0.0, "solve": 0.0, "project": 0.0, "stage2": 0.0} for p in precs}
    st = torch.cuda.current_stream()
    pending = []

    def timed(p, phase, fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        r = fn()
        b.record(st)
        pending.append((p, phase, a, b))
        return r

    def settle():
        torch.cuda.synchronize()
        for p, phase, a, b in pending:
            ms[p][phase] += a.elapsed_time(b)
        pending.clear()
        for c in ctxs.values():
            c.drop_chunk_refs()

    def stored(p, O, e, EL):
        if p == "fp64":
            return (O, e, EL)
        if p == "bf16x3":
            return (blm.SplitSamples(O, 3), blm.SplitSamples(e, 3), EL)
        return (blm.Fp8Samples(O), blm.Fp8Samples(e), EL)

    t_start = time.perf_counter()
    t_gen = 0.0
    for c in ctxs.values():
        c.begin_step()
    groups = {}
    if not args.no_autotune:
        # launch shape of each context's build, timed on the first chunk
        O, e, EL = gen.chunk(0, sizes[0])
        for p in precs:
            groups[p] = ctxs[p].autotune([stored(p, O, e, EL)])
            torch.cuda.synchronize()
            ctxs[p].drop_chunk_refs()
        del O, e, EL
        log(f"streamed: slice groups per tile {groups}")
    out = {}
    for pas in (1, 2):
        for i, n in enumerate(sizes):
            t0 = time.perf_counter()
            O, e, EL = gen.chunk(i, n)
            torch.cuda.synchronize()
            t_gen += time.perf_counter() - t0
            for p in precs:
                ch = [stored(p, O, e, EL)]
                if pas == 1:
                    timed(p, "build", lambda: ctxs[p].build(ch))
                else:
                    timed(p, "project", lambda: ctxs[p].project(ch))
                del ch
            del O, e, EL
            settle()
            log(f"streamed pass {pas}: chunk {i + 1}/{len(sizes)}")
        for p in precs:
            t0 = time.perf_counter()
            if pas == 1:
                ctxs[p].solve()
            else:
                out[p] = ctxs[p].stage2()
            torch.cuda.synchronize()
            ms[p]["solve" if pas == 1 else "stage2"] += 1e3 * (time.perf_counter() - t0)
            log(f"streamed pass {pas}: {p} {'block solves' if pas == 1 else 'stage two'} done")
    fl = build_flops(offsets, w.n_old, n_samples)
    res = {"workload": w.name if n_samples == w.n_samples else f"uneven_30000x{n_samples}",
           "n_params": w.n_params, "n_blocks": w.n_blocks, "n_samples": n_samples, "chunk": w.chunk,
           "n_keep": w.n_keep, "n_old": w.n_old, "shifts": shifts, "data": "synthetic, made on the device per chunk",
           "build_flops": fl, "precisions": {}}
    u64, e64 = out["fp64"][0].double().cpu().numpy(), out["fp64"][1]
    mats64 = [ctxs["fp64"].block_matrices(b, 0) for b in range(w.n_blocks)]
    step64 = sum(ms["fp64"].values())
    for p in precs:
        step = sum(ms[p].values())
        upd, en = out[p][0].double().cpu().numpy(), out[p][1]
        r = {"step_ms": round(step, 1), "phase_ms": {k: round(v, 1) for k, v in ms[p].items()},
             "build_slice_groups": groups.get(p),
             "build_tflops": round(fl / (ms[p]["build"] * 1e-3) / 1e12, 2), "energy": [float(x) for x in en]}
        if p != "fp64":
            worst = 0.0
            for b in range(w.n_blocks):
                H, S = ctxs[p].block_matrices(b, 0)
                H6, S6 = mats64[b]
                worst = max(worst, np.linalg.norm(S - S6) / np.linalg.norm(S6),
                            np.linalg.norm(H - H6) / np.linalg.norm(H6))
            r["block_matrix_rel_err_vs_fp64"] = worst
            r["energy_rel_err_vs_fp64"] = [float(abs(en[i] - e64[i]) / abs(e64[i])) for i in range(len(shifts))]
            r["update_cosine_vs_fp64"] = [float(u64[i] @ upd[i] / (np.linalg.norm(u64[i]) * np.linalg.norm(upd[i])))
                                          for i in range(len(shifts))]
            r["step_speedup_vs_fp64"] = round(step64 / step, 3)
            r["build_speedup_vs_fp64"] = round(ms["fp64"]["build"] / ms[p]["build"], 3)
        res["precisions"][p] = r
    res["generator_s"] = round(t_gen, 1)
    res["wall_s"] = round(time.perf_counter() - t_start, 1)
    for c in ctxs.values():
        c.close()
    print(json.dumps(res))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--samples", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the heuristic slice-group count of the build instead of timing the candidates")
    ap.add_argument("--mixed", default="bf16x3,fp8",
                    help="comma-separated mixed precisions (bf16x3, bf16x2, fp8) also run on the same "
                         "samples, or none")
    ap.add_argument("--streamed", action="store_true",
                    help="instead: one step of the 30,000-parameter, 4M-sample workload in FP64, BF16x3 "
                         "and FP8, its chunks made on the device as they are needed")
    ap.add_argument("--streamed-samples", type=int, default=0,
                    help="with --streamed: fewer samples than the workload's 4,000,000")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device-to-device copy three times (the reference "
                         "for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = 1 << 28                       # 2 GiB of float64
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 8 * n, "launches": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; sharding the samples over "
                                   "several GPUs is designed but not built", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_1702_01481_amd import blm, synth

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    if args.streamed:
        return streamed_target(args)
    w = synth.workload("fp64")
    n_samples = args.samples
    offsets = w.block_offsets
    shifts = list(w.shifts)
    dev = torch.device("cuda")
    gen = synth.SampleGenerator(w.n_params, w.rank, w.seed, sigma_E=w.sigma_E, device=dev)
    sizes = []
    left = n_samples
    while left > 0:
        sizes.append(min(w.chunk, left))
        left -= sizes[-1]
    chunks = []
    for i, n in enumerate(sizes):
        O, e, EL = gen.chunk(i, n)
        chunks.append((O, e, EL))
    del gen
    torch.cuda.synchronize()
    log(f"generated {len(chunks)} chunks, {n_samples} samples x {w.n_params} params in HBM")

    ctx = blm.BLM(w.n_params, offsets, w.n_keep, w.n_old, shifts, n_samples)
    ctx.set_timing(True)

    def step(old):
        ctx.begin_step(old)
        ctx.build(chunks)
        ctx.solve()
        ctx.project(chunks)
        return ctx.stage2()

    # previous direction: one step without history (zero rows are dropped)
    t1 = time.perf_counter()
    upd, en0, _, _ = step(torch.zeros(w.n_old, w.n_params, dtype=torch.float64, device=dev))
    old = upd[1:2].clone().contiguous()
    log(f"history step done in {time.perf_counter() - t1:.3f} s: {ctx.timings()}")
    groups = None
    if not args.no_autotune:
        ctx.begin_step(old)
        groups = ctx.autotune(chunks)
        log(f"fp64 build: {groups} slice groups per tile")
    for _ in range(args.warmup):
        step(old)
    torch.cuda.synchronize()
    log("warmup done")

    phase = {k: [] for k in blm.TIMING_NAMES}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        upd, en, al, fl = step(old)
        for k, v in ctx.timings().items():
            phase[k].append(v)
        log(f"step {len(phase['block_gram'])} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1e3 * elapsed / args.steps

    # the same steps with the build replayed from one recorded HIP graph
    ctx.capture_build(chunks)

    def step_graph():
        ctx.begin_step(old)
        ctx.replay_build()
        ctx.solve()
        ctx.project(chunks)
        return ctx.stage2()

    step_graph()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, en_g, _, _ = step_graph()
    torch.cuda.synchronize()
    ms_graph = 1e3 * (time.perf_counter() - t0) / args.steps
    graph_build = {"ms_per_step": round(ms_graph, 3),
                   "energy_equal_to_eager": bool(np.array_equal(np.asarray(en_g), np.asarray(en)))}
    log(f"replayed-build steps: {ms_graph:.1f} ms, {graph_build}")

    st = ctx.solver_stats()
    eig_phase_names = ("cholesky", "congruence", "hessenberg", "qr", "select", "inverse_iter",
                       "back_transform", "orthonormalise")
    eig_phases = {k: round(float(st[:, 4 + i].max()) / 1e5, 3) for i, k in enumerate(eig_phase_names)}
    eig_phases["qr_sweeps_max"] = int(st[:, 3].max())
    fl_build = build_flops(offsets, w.n_old, n_samples)
    gram_ms = float(np.mean(phase["block_gram"]))
    build_ms = float(np.mean([a + b + c for a, b, c in zip(phase["theta_proj"], phase["block_gram"],
                                                          phase["block_reduce"])]))
    achieved = fl_build / (gram_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": round(fl_build / (ms_step * 1e-3) / 1e12, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_params": w.n_params, "n_blocks": w.n_blocks,
                   "n_samples": n_samples, "chunk": w.chunk, "rank": w.rank, "n_keep": w.n_keep,
                   "n_old": w.n_old, "shifts": shifts, "precision": "fp64"},
        "build_tflops": round(fl_build / (build_ms * 1e-3) / 1e12, 4),
        "build_ms": round(build_ms, 3),
        "build_slice_groups": groups,
        "phase_ms": {k: round(float(np.mean(v)), 3) for k, v in phase.items()},
        "block_eig_phase_ms_max": eig_phases,
        "graph_build": graph_build,
        "energy": [float(x) for x in en],
        "flags": [int(x) for x in fl],
        "roofline": {"bound": "mfma", "achieved": round(achieved, 4), "peak": PEAK_FP64,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64, 4),
                     "traffic": gram_traffic_bytes(groups),
                     "kernel": "gram_kernel (block H/S build, FP64 MFMA 16x16x4)",
                     "flops_per_launch": fl_build},
    }
    if args.mixed != "none":
        out["mixed"] = []
        for prec in args.mixed.split(","):
            if prec not in ("bf16x3", "bf16x2", "fp8"):
                raise SystemExit(f"unknown mixed precision {prec}")
            out["mixed"].append(mixed_step(args, prec, w, chunks, old, offsets, shifts, n_samples, en, upd,
                                           ms_step, build_ms, fl_build))
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on one chunk")
        O0, e0, EL0 = chunks[0]
        cb = cpu_baseline(O0, e0, EL0, None, offsets, old.cpu().numpy(), w.n_keep, shifts)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
