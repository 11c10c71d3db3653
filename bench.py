"""Benchmark of the near-field hot path on one MI355X.

One step = abacus_nf_build_cells + abacus_nf_forces over one batch of the
workload (all of binning, sort, cell offsets, layout, work list, pairwise
kernel and finalize), inputs already resident in HBM.  Prints one JSON line.

Default: the late-time workload (N=2^27, K=256, half of the particles in 1% of
the cells), spline softening, compensated FP32 sums (the largest single-GPU
configuration of the metric), with its median / p99 fractional error on 10^5
sampled sinks against the FP64 oracle.  The same line carries, under
"variants", the plain FP32 sums and the Plummer kernel on the same workload and
the 64 batched boxes as one HIP-graph replay in both summation modes (a few
steps each, errors on smaller samples).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "near-field interactions/s + particle updates/s, 1 GPU, median frac err ≤1e-5"
FP32_PEAK_TFLOPS = 157.3          # MI355X FP32 vector peak (256 CUs x 2.4 GHz x 64 lanes x 2 FMA x 2 packed)
FLOPS_PER_PAIR = {0: 26, 1: 20}   # the paper's convention: op = 1, rsqrt = 2 (spline 26; Plummer 20)
FLOP_CONVENTION = ("Sec. 4.3 convention: every operation 1, rsqrt 2, per evaluated pair: 26 (spline: polynomial, "
                   "compare and select counted for every pair), 20 (Plummer)")
MODES = {"fp32": 0, "comp32": 1, "fp64": 2}
KINDS = {"spline": 0, "plummer": 1}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


HEADER_MARK = b"// (The definitions above are all the force kernel takes from this header.)"


def kernel_source_digest() -> str:
    """Digest of the force kernel's sources: its file and the part of the shared header it uses (the work
    items, queues and tile geometry, up to the marker line), so a counter summary is valid only for these
    sources."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2110_11398_amd", "csrc")
    h.update(open(os.path.join(csrc, "forces.hip"), "rb").read())
    header = open(os.path.join(csrc, "nf_internal.h"), "rb").read()
    h.update(header.split(HEADER_MARK)[0])
    return h.hexdigest()[:16]


def counter_summary(what: str, workload: str, kind: str, mode: str, tuning: dict):
    """A committed counter summary of the force kernel (profiles/<what>_forces_<workload>_<kind>_<mode>.json),
    if it was taken on these kernel sources with this kernel variant (otherwise None)."""
    path = os.path.join(ROOT, "profiles", f"{what}_forces_{workload}_{kind}_{mode}.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except ValueError:
        return None
    if d.get("source_digest") != kernel_source_digest():
        return None
    for k in ("sinks_per_lane", "unroll", "chunk", "occupancy", "max_lanes"):
        if d.get("tuning", {}).get(k) != tuning.get(k):
            return None
    return d


def traffic_from_profile(workload: str, kind: str, mode: str, tuning: dict):
    """HBM bytes per force-kernel launch from a committed FETCH_SIZE / WRITE_SIZE summary (or None)."""
    d = counter_summary("traffic", workload, kind, mode, tuning)
    return d.get("bytes_per_launch") if d else None


def executed_flops_from_profile(workload: str, kind: str, mode: str, tuning: dict):
    """FP32 operations the hardware executed per pair (SQ_INSTS_VALU_FLOPS_FP32 + _TRANS) from a committed
    counter summary (or None)."""
    d = counter_summary("valu", workload, kind, mode, tuning)
    return d.get("executed_flops_per_pair") if d else None


def oracle_sample(boxes, kind, target_s, threads, m_fixed=0):
    """Time the FP64 oracle on a bounded sample of sinks (about target_s seconds, or m_fixed sinks in all).

    One box: sinks drawn from it. Several boxes: the sample is spread over up to 8 boxes (the first ones, equal
    shares), each evaluated with its own softening and mass. Returns the baseline record and a list of
    (global index of the sampled sinks, FP64 reference accelerations)."""
    import oracle
    from workloads.gen import sample_sinks
    use = boxes[:min(8, len(boxes))]
    offs = np.cumsum([0] + [b.n for b in boxes])

    def run(m_total):
        share = max(1, m_total // len(use))
        parts, pairs = [], 0
        for k, b in enumerate(use):
            sk = sample_sinks(b.n, min(share, b.n), 99 + k)
            ref, pr = oracle.forces(b.pos, b.box, b.K, 2, b.eps, kind, b.gm, sinks=sk, threads=threads,
                                    return_pairs=True)
            parts.append((sk + offs[k], ref))
            pairs += pr
        return parts, pairs, sum(len(sk) for sk, _ in parts)

    n_use = sum(b.n for b in use)
    m = m_fixed if m_fixed > 0 else 256 * len(use)
    while True:
        # grow the sample (at most 20x per round) until it takes about target_s: the oracle's per-call
        # binning of all particles of a box makes the first, small samples look more expensive per sink
        t0 = time.perf_counter()
        parts, pairs, got = run(m)
        dt = time.perf_counter() - t0
        if m_fixed > 0 or dt >= target_s / 2 or got >= n_use or m >= n_use:
            break
        m = int(min(n_use, m * min(20.0, max(2.0, target_s / max(dt, 1e-3)))))
    where = "box 0" if len(use) == 1 else f"boxes 0-{len(use) - 1} (equal shares, seeds 99+box)"
    base = {"value": pairs / dt, "unit": "interactions/s", "cores": threads, "kind": "oracle",
            "sample": f"{got} sinks drawn without replacement (seed 99) of {where}; {pairs} FP64 pairs in {dt:.2f} s"}
    # the same oracle on one core, on a tenth of the sample of box 0 (a reference point for the thread scaling)
    b = boxes[0]
    m1 = max(16, min(b.n, got // 10))
    s1 = sample_sinks(b.n, m1, 99)
    t0 = time.perf_counter()
    _, p1 = oracle.forces(b.pos, b.box, b.K, 2, b.eps, kind, b.gm, sinks=s1, threads=1, return_pairs=True)
    d1 = time.perf_counter() - t0
    base["single_core"] = {"value": p1 / d1, "unit": "interactions/s", "cores": 1,
                           "sample": f"{m1} sinks of box 0 (seed 99); {p1} FP64 pairs in {d1:.2f} s"}
    base.update(host_description())
    return base, parts


def cpu_model() -> str:
    """The host CPU as /proc/cpuinfo names it: model name, vendor, family / model / stepping."""
    fields = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                k, v = (x.strip() for x in line.split(":", 1))
                if k in ("model name", "vendor_id", "cpu family", "model", "stepping") and k not in fields:
                    fields[k] = v
            if not line.strip() and fields:
                break
    except OSError:
        pass
    if not fields:
        return ""
    return (f"{fields.get('model name', '')} ({fields.get('vendor_id', '')}, family {fields.get('cpu family', '?')} "
            f"model {fields.get('model', '?')} stepping {fields.get('stepping', '?')})")


def oracle_threads() -> int:
    """Threads for the oracle: the host CPU share this process is given (OMP_NUM_THREADS when set, as on a
    GPU machine where each GPU owns a share of the host), else every CPU it may run on."""
    visible = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    try:
        share = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        share = 0
    return max(1, min(visible, share) if share > 0 else visible)


def host_description() -> dict:
    return {"cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "cpus_available": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def frac_errors(acc_all, parts):
    """Median and 99th percentile of |a - a_ref| / |a_ref| over the sampled sinks of all sampled boxes."""
    fes = []
    for idx, ref in parts:
        a = acc_all[idx].astype(np.float64)
        na = np.linalg.norm(ref, axis=1)
        fes.append(np.linalg.norm(a - ref, axis=1)[na > 0] / na[na > 0])
    fe = np.concatenate(fes)
    return float(np.median(fe)), float(np.percentile(fe, 99)), int(sum(len(i) for i, _ in parts))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="late", choices=["tiny", "clustered", "precision", "batched", "late"])
    ap.add_argument("--kind", default="spline", help="spline, plummer, or a comma list")
    ap.add_argument("--mode", default="comp32", help="fp32, comp32, fp64, or a comma list")
    ap.add_argument("--err-sinks", type=int, default=100000,
                    help="size of the oracle sample for the errors and the CPU baseline (0: sized to about "
                         "--cpu-seconds)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants", default="auto", choices=["auto", "on", "off"],
                    help="also run, and nest in the same line, plain FP32 sums and the Plummer kernel on the same "
                         "workload and the batched boxes as one HIP-graph replay (auto: with the default workload, "
                         "kind and mode)")
    ap.add_argument("--variant-steps", type=int, default=3)
    ap.add_argument("--variant-err-sinks", type=int, default=30000)
    ap.add_argument("--f64-out", action="store_true",
                    help="also report the errors of the FP64 output (abacus_nf_forces_f64) on the oracle sample")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2110_11398_amd", "tuning_cache.json"),
                    help="autotuner cache (JSON); the tuning for this device/kind/mode/size class is looked up "
                         "there and searched (then recorded) if missing")
    ap.add_argument("--no-tune", action="store_true", help="use the library's default tuning")
    ap.add_argument("--graph", action="store_true",
                    help="capture one step (build_cells + forces) in a HIP graph and time its replays")
    ap.add_argument("--tuning", default="", help="comma list k=v of abacus_nf_tuning fields")
    ap.add_argument("--density", action="store_true",
                    help="also compute the fused kernel density estimate (b = 0.4 x mean spacing per box)")
    ap.add_argument("--stage", default="forces", choices=["forces", "multipoles", "taylor", "kdk"],
                    help="forces: the near-field step (default); multipoles: cell multipoles of the layout; "
                         "taylor: far field of synthetic per-cell Taylor series co-added to the accelerations; "
                         "kdk: leapfrog steps (half kick, drift, rebuild, near-field forces, half kick)")
    ap.add_argument("--order", type=int, default=8, help="series order for --stage multipoles / taylor")
    ap.add_argument("--merge", action="store_true",
                    help="--stage kdk: gather positions, velocities and accelerations into cell order after each "
                         "step (the merge step of the paper's pipeline)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (a known-size kernel that "
                         "calibrates the HBM byte counters of a profiler run)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU decomposition is "
              "a design note, not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2110_11398_amd as nf
    from workloads import gen

    gen.set_verbose(True)
    t0 = time.perf_counter()
    w = gen.workload(args.workload)
    log(f"generated {args.workload}: N={w.n_total} boxes={len(w.boxes)} in {time.perf_counter() - t0:.1f} s")
    pos = torch.from_numpy(w.concat_positions()).cuda()
    acc = torch.empty((w.n_total, 3), dtype=torch.float32, device="cuda")
    if args.copy_calibration_mb > 0:
        nbytes = args.copy_calibration_mb << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nbytes} bytes read, {nbytes} bytes written")
        del src, dst
    boxes = [(b.n, b.box, b.K) for b in w.boxes]
    eps = [b.eps for b in w.boxes]
    gm = [b.gm for b in w.boxes]
    if args.stage == "multipoles":
        print(json.dumps(run_multipoles(args, nf, torch, w, pos, boxes)), flush=True)
        return
    if args.stage == "taylor":
        print(json.dumps(run_taylor(args, nf, torch, gen, w, pos, boxes, acc)), flush=True)
        return
    if args.stage == "kdk":
        print(json.dumps(run_kdk(args, nf, torch, w, pos, boxes, eps, gm, acc)), flush=True)
        return
    variants = args.variants == "on" or (args.variants == "auto" and args.workload == "late" and
                                         args.kind == "spline" and args.mode == "comp32" and not args.density
                                         and not args.graph and not args.tuning)
    threads = oracle_threads()
    samples = {}

    def errors_of(line, kind, m_fixed, with_baseline):
        """Median / p99 fractional error of acc on the oracle sample of this kind (timed once per kind)."""
        if kind not in samples:
            samples[kind] = oracle_sample(w.boxes, kind, args.cpu_seconds, threads, m_fixed)
        base, parts = samples[kind]
        if with_baseline:
            line["cpu_baseline"] = dict(base)
            # full step on the oracle, extrapolated from its measured rate (not run)
            line["cpu_baseline"]["extrapolated_full_step_s"] = line["config"]["interactions_per_step"] / base["value"]
        med, p99, ns = frac_errors(acc.cpu().numpy(), parts)
        line["median_frac_err"], line["p99_frac_err"], line["err_sample_sinks"] = med, p99, ns
        return parts

    lines = []
    for kname in args.kind.split(","):
        for mname in args.mode.split(","):
            line = run_one(args, nf, torch, w, pos, boxes, eps, gm, acc, KINDS[kname], MODES[mname], kname, mname,
                           args.steps, args.warmup, args.graph)
            if not args.no_cpu_baseline:
                parts = errors_of(line, KINDS[kname], args.err_sinks, True)
                if args.f64_out:
                    # the same forces with FP64 output (no final FP32 rounding), an untimed extra call with the
                    # timed call's tuning (the same tiles, so the same summation order)
                    cells = nf.build_cells(pos, boxes, 2)
                    cells.set_tuning(**{k: int(v) for k, v in line["config"]["tuning"].items()})
                    a64 = cells.forces_f64(eps, gm, KINDS[kname], MODES[mname])
                    med, p99, _ = frac_errors(a64.cpu().numpy(), parts)
                    line["median_frac_err_f64_out"], line["p99_frac_err_f64_out"] = med, p99
                    cells.free()
            lines.append(line)
    if variants:
        head = lines[0]
        out = {}
        # the same workload: plain FP32 sums (errors on the spline sample), and the Plummer kernel
        for kname, mname in (("spline", "fp32"), ("plummer", "comp32")):
            v = run_one(args, nf, torch, w, pos, boxes, eps, gm, acc, KINDS[kname], MODES[mname], kname, mname,
                        args.variant_steps, 1, False)
            if not args.no_cpu_baseline:
                errors_of(v, KINDS[kname], args.variant_err_sinks, False)
            out[f"{args.workload}/{kname}/{mname}"] = compact(v)
        del pos
        torch.cuda.empty_cache()
        # the batched boxes, build + forces captured once in a HIP graph and replayed
        wb = gen.workload("batched")
        log(f"generated batched: N={wb.n_total} boxes={len(wb.boxes)}")
        pb = torch.from_numpy(wb.concat_positions()).cuda()
        ab = torch.empty((wb.n_total, 3), dtype=torch.float32, device="cuda")
        bb = [(b.n, b.box, b.K) for b in wb.boxes]
        eb, gb = [b.eps for b in wb.boxes], [b.gm for b in wb.boxes]
        _, bparts = oracle_sample(wb.boxes, KINDS["spline"], args.cpu_seconds, threads,
                                  args.variant_err_sinks) if not args.no_cpu_baseline else (None, None)
        for mname in ("comp32", "fp32"):
            v = run_one(args, nf, torch, wb, pb, bb, eb, gb, ab, KINDS["spline"], MODES[mname], "spline", mname,
                        args.variant_steps, 1, True)
            if bparts is not None:
                med, p99, ns = frac_errors(ab.cpu().numpy(), bparts)
                v["median_frac_err"], v["p99_frac_err"], v["err_sample_sinks"] = med, p99, ns
            out[f"batched-graph/spline/{mname}"] = compact(v)
        head["variants"] = out
    for line in lines:
        print(json.dumps(line), flush=True)


def compact(line):
    """The fields of a variant kept in the headline's JSON line."""
    keep = ("value", "unit", "ms_per_step", "steps", "particle_updates_per_s", "median_frac_err", "p99_frac_err",
            "err_sample_sinks")
    out = {k: line[k] for k in keep if k in line}
    out["config"] = {k: line["config"][k] for k in ("workload", "n", "boxes", "kind", "mode", "interactions_per_step",
                                                    "tuning", "hip_graph")}
    out["stages_ms"] = line["stages_ms"]
    out["roofline"] = {k: line["roofline"][k] for k in ("achieved", "frac", "frac_executed", "kernel_ms")
                       if k in line["roofline"]}
    return out


def run_one(args, nf, torch, w, pos, boxes, eps, gm, acc, kind, mode, kname, mname, steps, warmup, use_graph):
    cells = nf.build_cells(pos, boxes, 2)
    rho = torch.empty(w.n_total, dtype=torch.float32, device="cuda") if args.density else None
    bk = [0.4 * b.box / b.n ** (1.0 / 3.0) if b.n else b.box / b.K for b in w.boxes]

    def step_forces():
        if rho is not None:
            cells.forces_density(eps, gm, bk, kind, mode, acc, rho)
        else:
            cells.forces(eps, gm, kind, mode, acc)
    if args.tuning:
        cells.set_tuning(**{k: int(v) for k, v in (kv.split("=") for kv in args.tuning.split(","))})
    elif not args.no_tune:
        t0 = time.perf_counter()
        if rho is not None:
            t = cells.autotune_density(eps, gm, bk, kind, mode, acc, rho, reps=2, cache_path=args.tune_cache)
        else:
            t = cells.autotune(eps, gm, kind, mode, acc, reps=2, cache_path=args.tune_cache)
        log(f"tuning ({time.perf_counter() - t0:.1f} s): {t.as_dict()}")
    step_forces()
    nf.sync()
    interactions = cells.interactions()
    log(f"interactions per step: {interactions:.6e}")

    for _ in range(warmup):
        nf.build_cells(pos, boxes, 2, cells=cells)
        step_forces()
    nf.sync()

    graph = None
    if use_graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            nf.build_cells(pos, boxes, 2, cells=cells)
            step_forces()
        graph.replay()
        torch.cuda.synchronize()
        nf.sync()
    # HIP events around each stage, on the stream the kernels run on (eager steps); graph replays are
    # timed as a whole and their stage split comes from the same steps run eagerly afterwards
    cells.set_timing(graph is None)
    stage_ms = np.zeros(4)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        if graph is not None:
            graph.replay()
        else:
            nf.build_cells(pos, boxes, 2, cells=cells)
            step_forces()
            stage_ms += np.array(cells.last_times())
    e1.record()
    torch.cuda.synchronize()
    nf.sync()
    ms_step = e0.elapsed_time(e1) / steps
    stage_ms /= steps
    if graph is not None:
        cells.set_timing(True)
        stage_ms = np.zeros(4)
        for _ in range(steps):
            nf.build_cells(pos, boxes, 2, cells=cells)
            step_forces()
            stage_ms += np.array(cells.last_times())
        stage_ms /= steps
        nf.sync()
        del graph
    cells.set_timing(False)
    log(f"[{w.name} {kname}/{mname}] ms/step {ms_step:.3f}; stages ms build={stage_ms[0]:.3f} "
        f"worklist={stage_ms[1]:.3f} kernel={stage_ms[2]:.3f} finalize={stage_ms[3]:.3f}")

    step_s = ms_step / 1e3
    kern_s = stage_ms[2] / 1e3
    tuning = cells.get_tuning().as_dict()
    achieved = FLOPS_PER_PAIR[kind] * interactions / kern_s / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_PEAK_TFLOPS,
                "traffic": traffic_from_profile(w.name, kname, mname, tuning),
                "kernel": "k_forces", "kernel_ms": stage_ms[2],
                "flops_per_launch": FLOPS_PER_PAIR[kind] * interactions,
                "flop_convention": FLOP_CONVENTION,
                "pairs_per_s_kernel": interactions / kern_s}
    executed = executed_flops_from_profile(w.name, kname, mname, tuning)
    if executed is not None:
        # the same launch counted by the hardware's FLOP counters (the Newtonian fast path skips the softening
        # polynomial, so fewer operations execute than the convention credits)
        roofline["executed_flops_per_pair"] = executed
        roofline["frac_executed"] = executed * interactions / kern_s / 1e12 / FP32_PEAK_TFLOPS
    out = {"metric": METRIC, "value": interactions / step_s, "unit": "interactions/s", "n_gpus": 1,
           "steps": steps, "warmup": warmup, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{w.name}: {w.description}", "n": w.n_total, "boxes": len(w.boxes),
                      "K": [b.K for b in w.boxes][:4], "kind": kname, "mode": mname,
                      "interactions_per_step": interactions, "tuning": tuning, "hip_graph": bool(use_graph),
                      "density": bool(args.density)},
           "particle_updates_per_s": w.n_total / step_s,
           "particle_updates_per_s_forces_only": w.n_total / ((stage_ms[1] + stage_ms[2] + stage_ms[3]) / 1e3),
           "stages_ms": {"build_cells": stage_ms[0], "work_list": stage_ms[1], "forces_kernel": stage_ms[2],
                         "finalize": stage_ms[3]},
           "roofline": roofline}
    cells.free()
    return out


def _time_calls(args, torch, nf, fn):
    """Mean milliseconds per call of fn over args.steps calls after args.warmup, with events on the
    current stream (the stream the library launches on)."""
    for _ in range(max(1, args.warmup)):
        fn()
    nf.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    nf.sync()
    return e0.elapsed_time(e1) / args.steps


def _roofline(nbytes, flops, ms, kernel):
    """The binding roof of a kernel that both streams HBM and does FP64 vector arithmetic: the one whose
    fraction of its peak is higher (HBM 8 TB/s, FP64 vector 78.6 TFLOP/s)."""
    gbs = nbytes / (ms / 1e3) / 1e9
    tfs = flops / (ms / 1e3) / 1e12
    hbm = {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0}
    alu = {"bound": "alu", "achieved": tfs, "peak": 78.6, "unit": "TFLOP/s", "frac": tfs / 78.6}
    r = dict(hbm if hbm["frac"] >= alu["frac"] else alu)
    other = alu if r["bound"] == "hbm" else hbm
    r.update({"traffic": None, "kernel": kernel, "kernel_ms": ms, "bytes_per_launch": nbytes,
              "flops_per_launch": flops, "other_roof": other})
    return r


def taylor_flops_per_particle(p: int) -> int:
    """FP64 flops the series evaluation does per particle (an FMA counts 2): powers of v and w, one Horner
    pass (value and derivative, 2 FMAs per step) per column (b, k), then per column the product v^b w^k
    (1), its FMA into d/du (2) and, where b > 0 or k > 0, the scaled-power product and FMA into d/dv or
    d/dw (4 each); finally the three scaled subtractions (2 each)."""
    f = 2 * p
    for b in range(p + 1):
        for k in range(p + 1 - b):
            top = p - b - k
            f += 4 * top + 3 + (4 if b > 0 else 0) + (4 if k > 0 else 0)
    return f + 6


def run_taylor(args, nf, torch, gen, w, pos, boxes, acc):
    """Far field of synthetic per-cell Taylor series of order p at every particle, co-added to acc."""
    cells = nf.build_cells(pos, boxes, 2)
    n, nc = cells.size()
    p = args.order
    ncomp = (p + 1) * (p + 2) * (p + 3) // 6
    T = torch.from_numpy(gen.taylor_coefficients(nc, p, seed=41, amp=1e-3)).cuda()
    acc.zero_()
    ms_input_order = _time_calls(args, torch, nf, lambda: cells.taylor_forces(p, T, acc))
    # the paper keeps particles cell by cell (the merge step): the same evaluation on arrays in cell order
    cells.reorder([pos, acc])
    ms = _time_calls(args, torch, nf, lambda: cells.taylor_forces(p, T, acc))
    occupied = sum(int((np.bincount(_cells_of(b), minlength=b.K ** 3) > 0).sum()) for b in w.boxes)
    # positions and permutation read, accelerations read and written, coefficients of occupied cells read
    nbytes = 16 * n + 4 * n + 24 * n + 4 * (nc + 1) + 8 * ncomp * occupied
    flops = taylor_flops_per_particle(p) * n
    cells.free()
    return {"metric": "far-field Taylor evaluation: particles/s", "value": n / (ms / 1e3), "unit": "particles/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{args.workload}: {w.description}", "n": n, "cells": nc,
                       "occupied_cells": occupied, "order": p, "components": ncomp,
                       "particle_order": "cell order (after abacus_nf_reorder)"},
            "ms_input_order": ms_input_order, "particles_per_s_input_order": n / (ms_input_order / 1e3),
            "roofline": _roofline(nbytes, flops, ms, "k_taylor")}


def run_kdk(args, nf, torch, w, pos, boxes, eps, gm, acc):
    """Leapfrog steps of the near field: each step is half kick, drift, rebuild of the cells, forces, half
    kick.  The step size comes once from the cell criterion (eta = 0.25) on seeded velocities; the kick and
    drift kernels are also timed alone (each streams 36 bytes per particle)."""
    kind, mode = KINDS[args.kind.split(",")[0]], MODES[args.mode.split(",")[0]]
    cells = nf.build_cells(pos, boxes, 2)
    if not args.no_tune:
        cells.autotune(eps, gm, kind, mode, cache_path=args.tune_cache)
    n = w.n_total
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    vel = 1e-3 * torch.randn((n, 3), generator=g, device="cuda", dtype=torch.float32)
    cells.forces(eps, gm, kind, mode, out=acc)
    dt = cells.timestep(vel, acc, 0.25)
    pairs = cells.interactions()
    def step():
        cells.kdk_step(dt, eps, gm, pos, vel, acc, kind, mode)
        if args.merge:
            cells.reorder([pos, vel, acc])

    ms = _time_calls(args, torch, nf, step)
    # the step-size criterion on the state after the steps: from the gathered accelerations, and from the
    # per-cell maxima the last force pass recorded (each call blocks for its n_boxes results)
    ts_ms = _time_calls(args, torch, nf, lambda: cells.timestep(vel, acc, 0.25))
    ts_fused_ms = _time_calls(args, torch, nf, lambda: cells.timestep(vel, None, 0.25))
    probe = torch.empty_like(vel)
    kick_ms = _time_calls(args, torch, nf, lambda: cells.kick(dt, acc, probe))
    drift_ms = _time_calls(args, torch, nf, lambda: cells.drift([0.0] * len(boxes), probe, pos))
    stream_bytes = 36 * n
    line = {"metric": "leapfrog steps: particle updates/s (near field)", "value": n / (ms / 1e3),
            "unit": "particle updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"{args.workload}: {w.description}", "n": n, "boxes": len(boxes),
                       "kind": args.kind.split(",")[0], "mode": args.mode.split(",")[0], "dt": dt,
                       "merge_each_step": bool(args.merge),
                       "interactions_per_step_at_start": pairs, "tuning": cells.get_tuning().as_dict()},
            "interactions_per_s_at_start": pairs / (ms / 1e3),
            "timestep_call_ms": {"gathered_acc": ts_ms, "force_pass_maxima": ts_fused_ms},
            "kick": {"ms": kick_ms, "GB/s": stream_bytes / (kick_ms / 1e3) / 1e9,
                     "frac_hbm": stream_bytes / (kick_ms / 1e3) / 1e9 / 8000.0},
            "drift": {"ms": drift_ms, "GB/s": stream_bytes / (drift_ms / 1e3) / 1e9,
                      "frac_hbm": stream_bytes / (drift_ms / 1e3) / 1e9 / 8000.0}}
    cells.free()
    return line


def _cells_of(b):
    """Cell index of every particle of a box (floor of the position in cell widths, clamped)."""
    t = np.minimum(np.floor(b.pos.astype(np.float64) * (b.K / b.box)).astype(np.int64), b.K - 1)
    return (t[:, 0] * b.K + t[:, 1]) * b.K + t[:, 2]


def run_multipoles(args, nf, torch, w, pos, boxes):
    """Cell multipoles of order p from the built layout."""
    cells = nf.build_cells(pos, boxes, 2)
    n, nc = cells.size()
    p = args.order
    ncomp = (p + 1) * (p + 2) * (p + 3) // 6
    mass = [b.gm for b in w.boxes]
    out = torch.empty((nc, ncomp), dtype=torch.float64, device="cuda")
    ms = _time_calls(args, torch, nf, lambda: cells.multipoles(p, mass, out))
    nbytes = 16 * n + 4 * (nc + 1) + 8 * ncomp * nc   # spos read once, cell offsets, moments written once
    # per particle: 3p powers, then per component two products and an add
    flops = (3 * p + 3 * ncomp) * n
    cells.free()
    return {"metric": "cell multipoles: particles/s", "value": n / (ms / 1e3), "unit": "particles/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{args.workload}: {w.description}", "n": n, "cells": nc, "order": p,
                       "components": ncomp},
            "roofline": _roofline(nbytes, flops, ms,
                                  "abacus_nf_multipoles call (k_set_mass, k_multipoles, k_mp_combine)")}


if __name__ == "__main__":
    main()
