"""Benchmark of the pixel -> command hot path on one MI355X.

A step is one frame through every stage: calibration + slopes for every
sensor, the split-K control-matrix MVM, the in-order accumulation +
integrator (and the POLC product when the workload has it).  Frames are
resident in HBM before the timed region and run through the persistent frame
loop in batches of `--bank` frames per launch; ``value`` is frames per second.

Also reported on the same JSON line:
  latency_us   serving-path latency of the persistent loop (last chunk
               submitted from host memory -> commands seen on the host), frames
               paced at 500 Hz with the chunks spread over a 1.5 ms readout;
               this figure includes PCIe;
  roofline     the frame-loop kernel's algorithmic bytes per launch / its
               average launch duration, from HIP events on its stream;
  mvm          the standalone split-K MVM kernel (warm and after a cache flush);
  variants     the same step with BF16 and FP8 matrix storage, and the
               per-launch (non-persistent) path;
  cpu_baseline the CPU oracle on a bounded sample of the same frames.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("frame latency p50/p99 µs + RMS jitter; CM MVM HBM GB/s vs peak, "
          "FP32 vs BF16")
HBM_PEAK_GBS = 8000.0
ELEM = {"f32": 4, "bf16": 2, "fp8": 1}

WORKLOAD_TEXT = {
    "scao_sh_74": "ELT SCAO Shack-Hartmann: 74x74 subapertures (3972 valid, 28% obstruction), "
                  "10x10 px, 740x740 uint16 frame in 16 row chunks, 5318 actuators, "
                  "5318 x 7944 control matrix, gain 0.4, leak 0.01",
    "scao_pyr_92": "ELT SCAO pyramid: four 92x92 pupils (6144 valid px) on a 240x240 uint16 "
                   "frame in 16 row chunks, 5318 x 12288 control matrix",
    "ltao_68": "LTAO: 6 LGS SH 68x68 @10 px + 1 NGS 8x8 @16 px, 5330 x 40368 control "
               "matrix, implicit POLC (5330 x 5330 FP32)",
    "mcao_74": "MCAO: 6 LGS SH 74x74 @10 px + 3 NGS 2x2 @16 px, 6318 x 47688 control "
               "matrix, implicit POLC (6318 x 6318 FP32)",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("rtc_device.h", "rtc_internal.h", "rtc_kernels.hip", "rtc_persist.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1903_01852_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, dtype: str):
    """HBM bytes per MVM launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "mvm_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except ValueError:
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    ent = d.get("entries", {}).get(f"{workload}:{dtype}")
    return None if ent is None else ent.get("hbm_bytes_per_launch")


def build_inputs(workload: str, bank: int):
    import synth
    wl = synth.get_workload(workload)
    inst = wl.instances[0]
    frames, cals = [], []
    for w in range(len(inst.wfs)):
        fr, cal = synth.sensor_inputs(wl, 0, w, n=bank)
        frames.append(fr)
        cals.append(cal)
    R = synth.control_matrix(wl, 0)
    M = None
    if inst.polc:
        import numpy as np
        na = inst.n_act
        M = synth.gaussian_matrix(na, na, 0.5 / np.sqrt(na), synth.seed_for(wl.index, 0, 99, 5),
                                  np.float32)
    return wl, inst, frames, cals, R, M


def alg_bytes_per_frame(inst, info, dtype):
    """Bytes the method must move per frame: matrix (+ FP8 scales), POLC matrix,
    processed pixels (2 B) and their calibration (dark, flat, bg: 12 B), slopes,
    commands read and written."""
    px = 0
    for w in inst.wfs:
        px += w.n_units * (w.px * w.px if w.kind == "sh" else 4)
    b = inst.n_act * info["n_slopes"] * ELEM[dtype] + (4 * inst.n_act if dtype == "fp8" else 0)
    if inst.polc:
        b += 4 * inst.n_act * inst.n_act
    return b + 14 * px + 4 * info["n_slopes"] + 8 * inst.n_act


def make_engine(rtc, inst, dtype, cals, R, M, mode="persistent"):
    eng = rtc.Engine([(inst, dtype)], ring_depth=4, mode=mode)
    eng.load_matrices(0, R, M=M)
    for w, cal in enumerate(cals):
        eng.load_calibration(0, w, cal.dark, cal.flat, cal.bg, cal.thr, cal.ref)
    return eng


def run_steps(eng, dframes, bank, n, stream):
    done = 0
    while done < n:
        k = min(bank, n - done)
        eng.process_frames(0, dframes, k, stream=stream)
        done += k


def throughput(torch, eng, dframes, bank, steps, warmup):
    """Wall time of `steps` frames, and the average duration of one launch
    (`bank` frames) from HIP events recorded on the launch stream."""
    st = torch.cuda.current_stream()
    run_steps(eng, dframes, bank, warmup, st)
    torch.cuda.synchronize()
    n_launch = (steps + bank - 1) // bank
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n_launch)]
    t0 = time.perf_counter()
    done = 0
    for a, b in ev:
        k = min(bank, steps - done)
        a.record(st)
        eng.process_frames(0, dframes, k, stream=st)
        b.record(st)
        done += k
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    full = [a.elapsed_time(b) / 1e3 for a, b in ev[:steps // bank]]
    return dt, (sum(full) / len(full) if full else None)


def mvm_timing(torch, eng, n_iter=200, cold=False):
    """Average MVM kernel duration (s) from HIP events on the launch stream.

    warm: n_iter back-to-back launches between two events.  cold: before each
    launch a 1 GiB buffer is read (not written, so no dirty lines are left to
    write back) to evict the matrix from L2 and the Infinity Cache, and each
    launch is bracketed by its own events."""
    st = torch.cuda.current_stream()
    if not cold:
        eng.run_mvm(0, 10, stream=st)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        eng.run_mvm(0, n_iter, stream=st)
        b.record(st)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3 / n_iter
    flush = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    sink = torch.empty((), dtype=torch.float32, device="cuda")
    tot = 0.0
    n = max(10, n_iter // 10)
    for _ in range(n):
        torch.sum(flush, dim=0, out=sink)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        eng.run_mvm(0, 1, stream=st)
        b.record(st)
        torch.cuda.synchronize()
        tot += a.elapsed_time(b) / 1e3
    del flush
    return tot / n


def serving_latency(rtc, eng, inst, frames, n_frames, warmup=100, period_s=2e-3,
                    readout_s=1.5e-3):
    """Paced serving loop from host memory; returns latencies in microseconds."""
    import numpy as np
    nw = len(inst.wfs)
    chunks = []        # (wfs, chunk, r0, r1) in readout order, sensors read in parallel
    n_ch = max(w.n_chunks for w in inst.wfs)
    for c in range(n_ch):
        for w in range(nw):
            if c < inst.wfs[w].n_chunks:
                r0, r1 = eng.chunk_rows(0, w, c)
                chunks.append((w, c, r0, r1))
    gap = readout_s / max(1, n_ch)
    lat = []
    bank = frames[0].shape[0]
    t_next = time.perf_counter()
    for f in range(n_frames + warmup):
        t_frame = t_next
        for idx, (w, c, r0, r1) in enumerate(chunks):
            t_c = t_frame + (c + 1) * gap
            while time.perf_counter() < t_c:
                pass
            eng.submit_chunk(0, w, f, c, frames[w][f % bank][r0:r1])
        _, info = eng.wait_commands(0, f, timeout_s=5.0)
        if f >= warmup:
            lat.append((info["t_ready_ns"] - info["t_last_chunk_ns"]) / 1e3)
        t_next = t_frame + period_s
    lat = np.asarray(lat)
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
            "mean": float(lat.mean()), "rms_jitter": float(lat.std()),
            "max": float(lat.max()), "frames": int(lat.size),
            "pacing": f"{1 / period_s:.0f} Hz, chunks spread over {readout_s * 1e3:.1f} ms",
            "includes": "host memcpy into the pinned ring, PCIe copy, last chunk's slopes and "
                        "K-block MVM, integrator, copy of the commands to pinned host memory"}


def cpu_baseline(inst, frames, cals, R, M, budget_s=12.0):
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    Rm = np.asarray(R, np.float64)
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.run(inst, [f[n % f.shape[0]:n % f.shape[0] + 1] for f in frames], cals, Rm, 1,
                   M=None if M is None else M.astype(np.float64))
        n += 1
        if time.perf_counter() - t0 > budget_s and n >= 3:
            break
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "frames/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n} frames of the same workload through the FP64 numpy oracle "
                      f"(binary32 calibration, FP64 slopes/MVM/integrator), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--workload", default="scao_sh_74")
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--variants", default="bf16,fp8")
    ap.add_argument("--bank", type=int, default=64)
    ap.add_argument("--latency-frames", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--quick", action="store_true", help="throughput only (for profiling)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy 5 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the "
              "controller's hot path runs on a single MI355X", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1903_01852_amd import rtc
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    rtc.lib()

    log(f"bench: building inputs for {args.workload} (bank {args.bank})")
    wl, inst, frames, cals, R, M = build_inputs(args.workload, args.bank)
    dframes = [torch.from_numpy(f).cuda() for f in frames]

    def one(dtype, full, mode="persistent"):
        eng = make_engine(rtc, inst, dtype, cals, R, M, mode=mode)
        info = eng.infos[0]
        dt, launch_s = throughput(torch, eng, dframes, args.bank, args.steps, args.warmup)
        res = {"frames_per_s": args.steps / dt, "ms_per_step": dt * 1e3 / args.steps,
               "alg_bytes_per_frame": alg_bytes_per_frame(inst, info, dtype)}
        if launch_s is not None:
            res["launch_us"] = launch_s * 1e6
            res["frames_per_launch"] = args.bank
            res["loop_gbs"] = res["alg_bytes_per_frame"] * args.bank / launch_s / 1e9
        if full:
            warm = mvm_timing(torch, eng)
            cold = mvm_timing(torch, eng, cold=True)
            alg = (inst.n_act * info["n_slopes"] * ELEM[dtype] + 4 * info["n_slopes"]
                   + 4 * inst.n_act)
            res.update({"mvm_us_warm": warm * 1e6, "mvm_us_cold": cold * 1e6,
                        "alg_bytes": alg, "cm_bytes_stored": info["cm_bytes"],
                        "gbs_warm": alg / warm / 1e9, "gbs_cold": alg / cold / 1e9})
        log(f"bench: {dtype}: {res}")
        return eng, res

    if args.copy_probe:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copy probe: 5 x {src.numel() * 4} bytes read and written")
        del src, dst

    eng, main_res = one(args.dtype, True)
    variants = {}
    if not args.quick:
        for dt_name in [v for v in args.variants.split(",") if v and v != args.dtype]:
            e2, r2 = one(dt_name, True)
            e2.close()
            variants[dt_name] = r2
        e3, r3 = one(args.dtype, False, mode="stream")
        e3.close()
        variants[f"{args.dtype}_per_launch_path"] = r3

    latency = None
    if not args.quick and not args.no_latency:
        log("bench: serving latency")
        eng.set_state(0, None, None, 0)
        latency = serving_latency(rtc, eng, inst, frames, args.latency_frames)
        log(f"bench: latency {latency}")
    eng.close()

    cpu = None
    if not args.quick and not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        cpu = cpu_baseline(inst, frames, cals, R, M)

    achieved = main_res["loop_gbs"]
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args.workload, args.dtype),
            "kernel": "k_frame_loop",
            "avg_launch_us": round(main_res["launch_us"], 3),
            "frames_per_launch": args.bank,
            "algorithmic_bytes_per_launch": main_res["alg_bytes_per_frame"] * args.bank}
    mvm = {"kernel": f"k_mvm<{args.dtype}>", "alg_bytes": main_res["alg_bytes"],
           "warm_us": round(main_res["mvm_us_warm"], 3), "warm_gbs": round(main_res["gbs_warm"], 1),
           "cold_us": round(main_res["mvm_us_cold"], 3), "cold_gbs": round(main_res["gbs_cold"], 1),
           "cold_frac": round(main_res["gbs_cold"] / HBM_PEAK_GBS, 4)}
    out = {
        "metric": METRIC, "value": round(main_res["frames_per_s"], 1), "unit": "frames/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
        "data": "synthetic (seeded SH spots / pyramid images with the paper's shapes, "
                "Gaussian control matrix)",
        "config": {"workload": args.workload, "description": WORKLOAD_TEXT.get(args.workload),
                   "frames_in_bank": args.bank, "cm_storage": args.dtype},
        "roofline": roof,
        "mvm": mvm,
        "latency_us": latency,
        "variants": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv)
                         for kk, vv in v.items()} for k, v in variants.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
