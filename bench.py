"""Benchmark of the pixel -> command hot path on one MI355X.

Headline (BASELINE metric: frame latency p50/p99 us + RMS jitter, the MVM's
HBM GB/s against peak, FP32 vs BF16): the LTAO serving configuration, the
largest that runs on one GPU -- an LTAO instance (6 LGS Shack-Hartmann
sensors of 68x68 subapertures at 10 px and one 8x8 NGS at 16 px, 5330
actuators, 5330 x 40368 control matrix, implicit POLC, gain and leak switched
mid-run through the API) running beside the 74x74 SCAO instance of uneven
size in one persistent frame loop, FP32 control matrices.

A step is a batch of `--frames-per-step` frames (default 50) of that
configuration served at the paper's 500 Hz: every sensor's pixels arrive as
16 row chunks spread over a 1.5 ms readout from host memory, each frame goes
through every stage (calibration, slopes, the split-K MVM, reduction,
integrator, POLC product), and the commands are published to host memory.
The chunks are submitted and the commands collected by the library's own
pacer threads (rtc_pacer_run, pinned to cores), so the figures hold no
interpreter pause.  W warm-up steps are served first, then exactly K timed
steps between two device synchronisations.

  value          latency p50 (us) of the LTAO instance: its last chunk handed
                 to the library -> its commands seen in host memory (PCIe both
                 ways included); p99, RMS jitter, max and the device part beside
                 it, and the same for the SCAO instance
  roofline       the split-K MVM kernel on that configuration's LTAO matrix
                 (861 MB FP32, beyond the 256 MB Infinity Cache), each launch
                 after a 1 GiB read-only cache flush: algorithmic bytes per
                 launch / its average duration from HIP events on its stream
  cpu_baseline   the CPU oracle on the same workload (both instances per frame),
                 per-frame time at all host threads and at one thread
Extras (skipped with --quick): BF16 and FP8 storage of the same
configuration, MCAO serving, the MVM on every matrix beyond the cache, the
74x74 SCAO configuration (per-launch throughput, cache-resident MVM),
telemetry, matrix swap, zero-copy hand-off, the sensor-size scan and the
pyramid normalisations.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("frame latency p50/p99 µs + RMS jitter; CM MVM HBM GB/s vs peak, "
          "FP32 vs BF16")
HBM_PEAK_GBS = 8000.0
MVM_RUN = 16               # per-launch path: k_mvm_next launches per event pair
ELEM = {"f32": 4, "bf16": 2, "fp8": 1}
PERIOD_S = 2e-3            # 500 Hz (the paper's MCAO / LTAO frame rate)
READOUT_S = 1.5e-3

WORKLOAD_TEXT = {
    "scao_sh_74": "ELT SCAO Shack-Hartmann: 74x74 subapertures (3972 valid, 28% obstruction), "
                  "10x10 px, 740x740 uint16 frame in 16 row chunks, 5318 actuators, "
                  "5318 x 7944 control matrix, gain 0.4, leak 0.01",
    "scao_pyr_92": "ELT SCAO pyramid: four 92x92 pupils (6144 valid px) on a 240x240 uint16 "
                   "frame in 16 row chunks, 5318 x 12288 control matrix",
    "ltao_68": "LTAO: 6 LGS SH 68x68 @10 px (680x680 frames) + 1 NGS 8x8 @16 px, 16 row "
               "chunks per LGS, 5330 actuators, 5330 x 40368 control matrix, implicit POLC "
               "(5330 x 5330 FP32), gain/leak 0.4/0.01 switched to 0.3/0.02 mid-run; beside it "
               "in the same persistent launch the 74x74 SCAO SH instance (5318 x 7944)",
    "mcao_74": "MCAO: 6 LGS SH 74x74 @10 px + 3 NGS 2x2 @16 px, 6318 x 47688 control "
               "matrix, implicit POLC (6318 x 6318 FP32)",
    "mcao_80": "MCAO at the paper's 80x80 LGS size: 6 LGS SH 80x80 @10 px + 3 NGS 2x2, "
               "6318 x 55416 control matrix, implicit POLC",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources each measured kernel is built from; a counter summary applies only
# while they are unchanged.
KERNEL_SOURCES = {"k_mvm": ("rtc_device.h", "rtc_internal.h", "rtc_kernels.hip"),
                  "k_mvm_next": ("rtc_device.h", "rtc_internal.h", "rtc_kernels.hip"),
                  "k_frame_loop": ("rtc_device.h", "rtc_internal.h", "rtc_persist.hip")}


def kernel_source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, "paper_1903_01852_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, dtype: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (profiles/kernel_traffic.json), if it was taken on the kernel's
    current sources; else None."""
    p = os.path.join(ROOT, "profiles", "kernel_traffic.json")
    name = kernel.split("<")[0]
    if not os.path.exists(p) or name not in KERNEL_SOURCES:
        return None
    try:
        d = json.load(open(p))
    except ValueError:
        return None
    ent = d.get("entries", {}).get(f"{workload}:{dtype}:{name}")
    if ent is None or ent.get("source_sha256_16") != kernel_source_hash(name):
        return None
    return ent.get("hbm_bytes_per_launch")


def polc_matrix_for(wl, i):
    """POLC matrix of instance i: a stand-in for R.D with its statistics (the FP64
    product costs TFLOPs on the host at these sizes)."""
    import numpy as np
    import synth
    inst = wl.instances[i]
    if not inst.polc:
        return None
    na = inst.n_act
    return synth.gaussian_matrix(na, na, 0.5 / np.sqrt(na), synth.seed_for(wl.index, i, 99, 5),
                                 np.float32)


def build_inputs(name: str, bank: int):
    """Per instance: R, M (or None), per-sensor frame banks, calibrations."""
    import synth
    wl = synth.get_workload(name)
    out = []
    for i, inst in enumerate(wl.instances):
        frames, cals = [], []
        for w in range(len(inst.wfs)):
            fr, cal = synth.sensor_inputs(wl, i, w, n=bank)
            frames.append(fr)
            cals.append(cal)
        out.append({"R": synth.control_matrix(wl, i), "M": polc_matrix_for(wl, i),
                    "frames": frames, "cals": cals})
    return wl, out


def load_engine(rtc, wl, data, dtype, mode, only=None):
    idx = list(range(len(wl.instances))) if only is None else [only]
    eng = rtc.Engine([(wl.instances[i], dtype) for i in idx], ring_depth=4, mode=mode)
    for k, i in enumerate(idx):
        eng.load_matrices(k, data[i]["R"], M=data[i]["M"])
        for w, cal in enumerate(data[i]["cals"]):
            eng.load_calibration(k, w, cal.dark, cal.flat, cal.bg, cal.thr, cal.ref)
    return eng


def _pct(v):
    import numpy as np
    v = np.asarray(v, dtype=np.float64)
    v = v[~np.isnan(v)]
    if v.size == 0:
        return None
    return {"p50": float(np.percentile(v, 50)), "p99": float(np.percentile(v, 99)),
            "mean": float(v.mean()), "rms_jitter": float(v.std()), "max": float(v.max()),
            "frames": int(v.size)}


STEADY_LATE_US = 5.0


def latency_stats(samples):
    """Statistics of one stream's pacer samples: host latency (last chunk handed
    over -> commands seen), the device part, the latency from the last chunk
    that completes a column block, the paper's b)-style steady subset (frames
    whose first and last chunks the pacer handed over within STEADY_LATE_US of
    its usual lateness, the median: the last chunks of all sensors fall due
    together and are copied in one after another), and the pacer's own
    lateness."""
    import numpy as np
    # a frame whose commands were out before its last chunk was handed over
    # (its last rows hold no pixel it needs) has latency 0 from the last pixel
    host = np.maximum(samples["host_us"], 0.0)
    dev = np.where(samples["dev_us"] >= 0, samples["dev_us"], np.nan)
    steady = ((samples["late_us"] <= np.median(samples["late_us"]) + STEADY_LATE_US)
              & (samples["start_late_us"] <= np.median(samples["start_late_us"]) + STEADY_LATE_US))
    r = _pct(host)
    r["device"] = _pct(dev)
    r["from_completing_chunk"] = _pct(samples["complete_us"])
    r["published_before_last_chunk"] = int(((samples["dev_us"] < 0)
                                            | (samples["host_us"] < 0)).sum())
    r["steady_subset"] = _pct(host[steady])
    r["pacer_late_us"] = {"last_chunk": _pct(samples["late_us"]),
                          "first_chunk": _pct(samples["start_late_us"])}
    return r


def rnd(d):
    if isinstance(d, dict):
        return {k: rnd(v) for k, v in d.items()}
    if isinstance(d, float):
        return round(d, 3)
    return d


def serve(eng, data, n_frames, warmup, first=0, switch=None, zero_copy=False, insts=None):
    """Paced serving run of every instance (or `insts`) through the library's
    pacer; returns per instance the latency statistics."""
    insts = list(range(len(data))) if insts is None else insts
    streams = [(k, data[i]["frames"]) for k, i in enumerate(insts)]
    s = eng.pace(streams, n_frames + warmup, warmup=warmup, period_s=PERIOD_S,
                 readout_s=READOUT_S, first_frame=first, zero_copy=zero_copy, switch=switch)
    return [latency_stats(s[k]) for k in range(len(insts))]


# Milestones of a served frame from the frame loop's timeline record (event,
# and whether the first or the last wavefront to reach it matters), in
# microseconds after the sentinel saw the frame's last chunk.
TIMELINE = (("last ingest starts", "ingest_start", "last"),
            ("last ingest done", "ingest", "last"),
            ("last slopes start", "cen_start", "last"),
            ("last slopes counted", "centroids", "last"),
            ("last block's first MVM task", "last_block", "first"),
            ("first tile's partials complete", "tile_ready", "first"),
            ("last tile's partials complete", "tile_ready", "last"),
            ("last join answered", "joined", "last"),
            ("last sum formed", "summed", "last"),
            ("last commands written", "cmds", "last"))


def timeline(torch, rtc, name, dtype, n_rec=150, warmup=50):
    """Where a served frame's latency goes: the paced serving run with the
    library's per-wavefront timeline record, per instance the median over
    frames of each milestone (device clock, 100 MHz)."""
    import numpy as np
    wl, data = build_inputs(name, 16)
    eng = load_engine(rtc, wl, data, dtype, "persistent")
    eng.trace_enable(n_rec + warmup)
    s = eng.pace([(k, d["frames"]) for k, d in enumerate(data)], n_rec + warmup,
                 warmup=warmup, period_s=PERIOD_S, readout_s=READOUT_S)
    tr = eng.trace_read().astype(np.int64)       # (frames, waves, events)
    eng.close()
    ev = {e: i for i, e in enumerate(rtc.TRACE_EVENTS)}
    out = {}
    for k, inst in enumerate(wl.instances):
        per = {m[0]: [] for m in TIMELINE}
        per["published"] = []
        for i in range(n_rec):
            t_seen, t_pub = int(s[k][i]["dev_ticks_start"]), int(s[k][i]["dev_ticks_cmd"])
            if t_seen == 0:
                continue
            rec = tr[warmup + i]
            # an instance's wavefronts run from its sentinel (which records
            # nothing) to the next instance's sentinel
            sentinels = np.flatnonzero(rec[:, ev["frame_start"]] == 0)
            w0 = sentinels[k] if k < len(sentinels) else 0
            w1 = sentinels[k + 1] if k + 1 < len(sentinels) else rec.shape[0]
            mine = rec[w0:w1]
            mine = mine[mine[:, ev["frame_start"]] > 0]
            for label, e, which in TIMELINE:
                v = mine[:, ev[e]]
                v = v[v > 0]
                if v.size:
                    per[label].append(((v.min() if which == "first" else v.max()) - t_seen) / 100.0)
            per["published"].append((t_pub - t_seen) / 100.0)
        out[inst.name] = {lab: round(float(np.median(v)), 2) for lab, v in per.items() if v}
        out[inst.name]["host_p50"] = round(float(np.median(s[k]["host_us"])), 2)
    return out


def mvm_timing(torch, eng, n_iter=200, cold=False, inst=0):
    """Average MVM kernel duration (s) from HIP events on the launch stream.

    warm: n_iter back-to-back launches between two events.  cold: before each
    launch a 1 GiB buffer is read (not written, so no dirty lines are left to
    write back) to evict the matrix from L2 and the Infinity Cache, and each
    launch is bracketed by its own events."""
    st = torch.cuda.current_stream()
    if not cold:
        eng.run_mvm(inst, 10, stream=st)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        eng.run_mvm(inst, n_iter, stream=st)
        b.record(st)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3 / n_iter, n_iter
    flush = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    sink = torch.empty((), dtype=torch.float32, device="cuda")
    tot = 0.0
    n = max(10, n_iter // 10)
    for _ in range(n):
        torch.sum(flush, dim=0, out=sink)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        eng.run_mvm(inst, 1, stream=st)
        b.record(st)
        torch.cuda.synchronize()
        tot += a.elapsed_time(b) / 1e3
    del flush
    return tot / n, n


def mvm_alg_bytes(inst, n_slopes, dtype):
    """Bytes the MVM must move: the matrix (+ FP8 row scales), slopes read,
    partial-free result read and written (command vector)."""
    return (inst.n_act * n_slopes * ELEM[dtype] + 4 * n_slopes + 8 * inst.n_act
            + (4 * inst.n_act if dtype == "fp8" else 0))


def box_reference(torch, reps=10):
    """HBM reference of this particular box: a plain 512 MiB device-to-device
    copy (read + write bytes per second, median of `reps`)."""
    src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream()
    for _ in range(3):
        dst.copy_(src)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        dst.copy_(src)
        b.record(st)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b) / 1e3)
    ts.sort()
    t = ts[len(ts) // 2]
    nbytes = 2 * src.numel() * 4
    del src, dst
    return {"copy_gbs": round(nbytes / t / 1e9, 1), "bytes": nbytes,
            "what": "median of 10 device-to-device copies of 512 MiB (read + write)"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(wl, data, budget_s=12.0):
    """The CPU oracle on the same workload: every instance's frame per step,
    FP64 matrices (binary32 calibration), timed per frame at all host threads
    and at one thread (threadpoolctl limits numpy's BLAS)."""
    import numpy as np
    import oracle
    from threadpoolctl import threadpool_info, threadpool_limits
    mats = [(np.asarray(d["R"], np.float64), None if d["M"] is None else d["M"].astype(np.float64))
            for d in data]

    def run(limit):
        times = []
        t_end = time.perf_counter() + budget_s
        f = 0
        with threadpool_limits(limits=limit):
            used = max([x.get("num_threads", 1) for x in threadpool_info()] + [1])
            while time.perf_counter() < t_end or len(times) < 3:
                t0 = time.perf_counter()
                for i, inst in enumerate(wl.instances):
                    fr = data[i]["frames"]
                    oracle.run(inst, [b[f % b.shape[0]:f % b.shape[0] + 1] for b in fr],
                               data[i]["cals"], mats[i][0], 1, M=mats[i][1])
                times.append((time.perf_counter() - t0) * 1e6)
                f += 1
        t = np.asarray(times)
        return {"median_us": float(np.median(t)), "p99_us": float(np.percentile(t, 99)),
                "frames": int(t.size), "threads": int(used)}
    allc = run(None)
    one = run(1)
    return {"value": allc["median_us"], "unit": "us", "cores": allc["threads"], "kind": "oracle",
            "sample": f"{allc['frames']} frames of the same workload (LTAO and SCAO instances, "
                      f"one frame each per step) through the FP64 numpy oracle (binary32 "
                      f"calibration), per-frame median over ~{budget_s:.0f} s; no pacing",
            "p99": allc["p99_us"], "one_thread": one, "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count()}


# matrices larger than the 256 MB Infinity Cache: their MVM rate is an HBM rate
LARGE_MVM = (("ltao_68", "f32"), ("ltao_68", "bf16"), ("ltao_68", "fp8"), ("mcao_74", "bf16"),
             ("mcao_74", "fp8"), ("mcao_80", "bf16"), ("mcao_80", "fp8"))


def mvm_large(torch, rtc, log, cache):
    """The standalone MVM on the LTAO and MCAO matrices, warm (back to back) and
    after a 1 GiB read-only cache flush."""
    import synth
    res = {}
    for name, dtype in LARGE_MVM:
        wl = synth.get_workload(name)
        inst = wl.instances[0]
        if name not in cache:
            cache.clear()
            cache[name] = (synth.control_matrix(wl, 0), polc_matrix_for(wl, 0))
        R, M = cache[name]
        eng = rtc.Engine([(inst, dtype)], mode="stream")
        eng.load_matrices(0, R, M=M)
        info = eng.infos[0]
        warm, _ = mvm_timing(torch, eng, n_iter=100)
        cold, _ = mvm_timing(torch, eng, n_iter=100, cold=True)
        eng.close()
        alg = mvm_alg_bytes(inst, info["n_slopes"], dtype)
        r = {"n_act": inst.n_act, "n_slopes": info["n_slopes"], "alg_bytes": alg,
             "warm_us": warm * 1e6, "warm_gbs": alg / warm / 1e9,
             "cold_us": cold * 1e6, "cold_gbs": alg / cold / 1e9,
             "cold_frac": alg / cold / 1e9 / HBM_PEAK_GBS,
             "traffic": measured_traffic(name, dtype, "k_mvm")}
        res[f"{name}:{dtype}"] = rnd(r)
        log(f"bench: mvm {name} {dtype}: {alg / 1e6:.0f} MB, warm {warm * 1e6:.1f} us "
            f"({r['warm_gbs']:.0f} GB/s), cold {cold * 1e6:.1f} us ({r['cold_gbs']:.0f} GB/s, "
            f"{r['cold_frac']:.3f} of peak)")
    return res


def batch_throughput(torch, eng, frames, n, warmup, inst=0, timed_launches=False):
    """Frames/s of the batch path over device-resident frames, and (per-launch
    path) the average k_mvm_next launch from the library's HIP events."""
    st = torch.cuda.current_stream()
    bank = frames[0].shape[0]
    def run(k):
        done = 0
        while done < k:
            m = min(bank, k - done)
            eng.process_frames(inst, frames, m, stream=st)
            done += m
    run(warmup)
    torch.cuda.synchronize()
    if timed_launches:
        eng.mvm_timing(inst, n, MVM_RUN)
    t0 = time.perf_counter()
    run(n)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = {"frames_per_s": n / dt}
    if timed_launches:
        k, tot = eng.mvm_timing_read(inst)
        eng.mvm_timing(inst, 0, 1)
        if k:
            r["k_mvm_next_us"] = tot / k * 1e6     # mvm_timing_read returns seconds
            r["k_mvm_next_launches_timed"] = k
    return r


def scao_extras(torch, rtc, log):
    """The 74x74 SCAO configuration: per-launch batch throughput and the MVM
    warm / cold.  Its matrices (169 / 85 / 42 MB) fit the 256 MB Infinity
    Cache, so the warm MVM rates are cache rates, not HBM rates (inferred from
    timing: warm above the box's copy rate, cold well below)."""
    wl, data = build_inputs("scao_sh_74", 64)
    inst = wl.instances[0]
    dfr = [torch.from_numpy(f).cuda() for f in data[0]["frames"]]
    res = {"infinity_cache_resident": True,
           "what": "matrix fits the 256 MB Infinity Cache: warm figures are cache rates"}
    for dtype in ("f32", "bf16", "fp8"):
        eng = load_engine(rtc, wl, data, dtype, "stream")
        info = eng.infos[0]
        r = batch_throughput(torch, eng, dfr, 2000, 200, timed_launches=True)
        warm, _ = mvm_timing(torch, eng)
        cold, _ = mvm_timing(torch, eng, cold=True)
        alg = mvm_alg_bytes(inst, info["n_slopes"], dtype)
        r.update({"mvm_alg_bytes": alg, "mvm_warm_us": warm * 1e6,
                  "mvm_warm_gbs_cache": alg / warm / 1e9, "mvm_cold_us": cold * 1e6,
                  "mvm_cold_gbs": alg / cold / 1e9})
        eng.close()
        eng = load_engine(rtc, wl, data, dtype, "persistent")
        r["frame_loop_batch"] = batch_throughput(torch, eng, dfr, 2000, 200)
        eng.set_state(0, None, None, 0)        # serving restarts at frame 0
        lat = serve(eng, data, 1000, 100)[0]
        eng.set_state(0, None, None, 0)
        r["serving_latency_us"] = lat
        r["serving_latency_zero_copy_us"] = serve(eng, data, 1000, 100, zero_copy=True)[0]
        eng.close()
        res[dtype] = rnd(r)
        log(f"bench: scao_sh_74 {dtype}: {r['frames_per_s']:.0f} frames/s per-launch, "
            f"k_mvm_next {r.get('k_mvm_next_us', 0):.1f} us, serving p50 {lat['p50']:.1f} "
            f"p99 {lat['p99']:.1f} us")
    return res


def telemetry_and_swap(torch, rtc, log):
    """SCAO FP32 serving with telemetry of every frame drained by a host thread,
    and with a second control matrix staged by another thread while frames run
    and swapped in at a frame boundary."""
    import numpy as np
    import synth
    wl, data = build_inputs("scao_sh_74", 64)
    inst = wl.instances[0]
    res = {}
    eng = load_engine(rtc, wl, data, "f32", "persistent")
    eng.telemetry_enable(0, 1, 256)
    got, stop = [0, 0], threading.Event()

    def drain():
        while not stop.is_set():
            try:
                _, _, _, ti = eng.telemetry_next(0, timeout_s=0.05)
            except Exception:
                continue
            got[0] += 1
            got[1] += ti["lost"]
    th = threading.Thread(target=drain)
    th.start()
    lat = serve(eng, data, 1000, 100)[0]
    time.sleep(0.1)
    stop.set()
    th.join()
    eng.telemetry_enable(0, 1, 0)
    lat["telemetry"] = {"decimation": 1, "slots": 256, "records_read": got[0],
                        "records_lost": got[1]}
    res["telemetry_every_frame"] = rnd(lat)
    log(f"bench: scao f32 with telemetry: p50 {lat['p50']:.1f} p99 {lat['p99']:.1f} us")
    # matrix swap: staging starts 0.2 s into the run, the swap follows at once
    eng.set_state(0, None, None, 0)
    R2 = synth.gaussian_matrix(inst.n_act, inst.n_slopes, 1.0 / np.sqrt(inst.n_slopes),
                               synth.seed_for(wl.index, 0, 77, 1), np.float32)
    sw = {}

    def stage():
        time.sleep(0.3)
        sw["t0"] = time.perf_counter()
        eng.stage_matrices(0, R2)
        sw["t1"] = time.perf_counter()
        sw["f_eff"] = eng.swap_matrices(0)
    t_run = time.perf_counter()
    th = threading.Thread(target=stage)
    th.start()
    s = eng.pace([(0, data[0]["frames"])], 1100, warmup=0, period_s=PERIOD_S,
                 readout_s=READOUT_S)[0]
    th.join()
    eng.close()
    fa = s["frame"].astype(np.int64)
    fs = int((sw["t0"] - t_run) / PERIOD_S)
    fe = sw["f_eff"]
    r = {"stage_s": sw["t1"] - sw["t0"], "stage_frame_approx": fs, "f_eff": fe}
    for k, m in {"before_stage": (fa >= 100) & (fa < fs), "during_stage": (fa >= fs) & (fa < fe),
                 "first_20_after_swap": (fa >= fe) & (fa < fe + 20), "after_swap": fa >= fe}.items():
        if m.any():
            r[k] = {"host": _pct(s["host_us"][m]),
                    "device": _pct(np.where(s["dev_us"][m] >= 0, s["dev_us"][m], np.nan))}
    res["matrix_swap"] = rnd(r)
    log(f"bench: matrix swap: staged in {r['stage_s']:.3f} s, effective frame {fe}")
    return res


def serving_suite(torch, rtc, log, frames_n):
    """MCAO serving (74x74 and the paper's 80x80 LGS), BF16 and FP8."""
    res = {}
    for name in ("mcao_74", "mcao_80"):
        wl, data = build_inputs(name, 16)
        for dtype in ("bf16", "fp8"):
            eng = load_engine(rtc, wl, data, dtype, "persistent")
            lat = serve(eng, data, frames_n, 100)[0]
            eng.close()
            res[f"{name}:{dtype}"] = rnd(lat)
            log(f"bench: serving {name} {dtype}: p50 {lat['p50']:.1f} p99 {lat['p99']:.1f} "
                f"jitter {lat['rms_jitter']:.2f} us (device p50 {lat['device']['p50']:.1f})")
        del data
    return res


def wfs_sweep(torch, rtc, n_frames, log):
    """Serving latency against sensor size at a constant frame size (the paper's
    scaling study): Shack-Hartmann 74..110 subapertures across on 800x800 frames
    (10, 10, 8, 8, 7 px per subaperture) and pyramid 80..120 pupil pixels across
    on 240x240 frames, each with a 5318-actuator FP32 control matrix.  For the
    small pyramid pupils the frame's last chunks hold no pupil pixel, so the
    commands are out before they arrive: latency is also reported from the last
    chunk that completes a column block."""
    import synth
    res = {}
    points = [("sh", n, synth.ShWfs(nsub=n, px=min(10, 800 // n), obs=0.28, frame_h=800,
                                    frame_w=800, origin=((800 - n * min(10, 800 // n)) // 2,) * 2))
              for n in (74, 80, 90, 100, 110)]
    for p in (80, 90, 100, 110, 120):
        o0, o1 = (120 - p) // 2, 120 + (120 - p) // 2
        points.append(("pyr", p, synth.PyrWfs(pupil_px=p, quad_origins=((o0, o0), (o1, o0),
                                                                        (o0, o1), (o1, o1)))))
    for i, (kind, n, wfs) in enumerate(points):
        inst = synth.Instance(f"sweep_{kind}{n}", (wfs,), 5318, ("f32",))
        wl = synth.Workload(200 + i, inst.name, (inst,), n_frames=n_frames, bank=16)
        synth.workloads.WORKLOADS[wl.name] = wl
        try:
            fr, cal = synth.sensor_inputs(wl, 0, 0, n=16)
            R = synth.control_matrix(wl, 0)
        finally:
            del synth.workloads.WORKLOADS[wl.name]
        data = [{"R": R, "M": None, "frames": [fr], "cals": [cal]}]
        eng = load_engine(rtc, wl, data, "f32", "persistent")
        r = serve(eng, data, n_frames, 100)[0]
        eng.close()
        key = f"{kind}_{n}x{n}"
        res[key] = {"n_slopes": inst.n_slopes, "n_act": inst.n_act,
                    "px_per_subap": getattr(wfs, "px", None), **rnd(r)}
        log(f"bench: sweep {key}: {inst.n_slopes} slopes, p50 {r['p50']:.1f} p99 {r['p99']:.1f} "
            f"us, from the completing chunk p50 {r['from_completing_chunk']['p50']:.1f} us")
    return res


def pyramid_norms(torch, rtc, steps, log):
    """Per-launch batch frames/s of the 92-pixel pyramid (5318 x 12288 FP32
    matrix) with local and with global normalisation."""
    import dataclasses
    import synth
    res = {}
    base = synth.get_workload("scao_pyr_92")
    for norm in ("local", "global"):
        wfs = dataclasses.replace(base.instances[0].wfs[0], norm=norm)
        inst = dataclasses.replace(base.instances[0], wfs=(wfs,))
        wl = dataclasses.replace(base, name=f"scao_pyr_92_{norm}", instances=(inst,))
        synth.workloads.WORKLOADS[wl.name] = wl
        try:
            fr, cal = synth.sensor_inputs(wl, 0, 0, n=16)
            R = synth.control_matrix(wl, 0)
        finally:
            del synth.workloads.WORKLOADS[wl.name]
        data = [{"R": R, "M": None, "frames": [fr], "cals": [cal]}]
        eng = load_engine(rtc, wl, data, "f32", "stream")
        r = batch_throughput(torch, eng, [torch.from_numpy(fr).cuda()], steps, 64)
        eng.close()
        res[norm] = {"frames_per_s": round(r["frames_per_s"], 1), "n_slopes": inst.n_slopes}
        log(f"bench: pyramid 92 px {norm} normalisation: {r['frames_per_s']:.0f} frames/s")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--frames-per-step", type=int, default=50)
    ap.add_argument("--dtype", default="f32", choices=("f32", "bf16", "fp8"))
    ap.add_argument("--quick", action="store_true",
                    help="the headline, its roofline and the CPU baseline only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extra-frames", type=int, default=1000,
                    help="frames per serving extra")
    ap.add_argument("--mvm-large-only", action="store_true",
                    help="only the standalone MVM on the matrices beyond the cache (profiling)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the roofline's cold MVM launches (hardware-counter runs)")
    ap.add_argument("--frame-loop-only", action="store_true",
                    help="only the frame loop's batch form on the 74x74 SCAO FP32 case, 4 "
                         "launches of 64 device-resident frames after one warm-up launch "
                         "(hardware-counter runs)")
    ap.add_argument("--timeline", metavar="WORKLOAD",
                    help="only the serving timeline of WORKLOAD (with --dtype): where a "
                         "frame's latency goes, from the loop's per-wavefront record")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy 5 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: the "
              "controller's hot path runs on a single MI355X", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1903_01852_amd import rtc
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    rtc.lib()

    if args.copy_probe:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copy probe: 5 x {src.numel() * 4} bytes read and written")
        del src, dst

    ref = box_reference(torch)
    log(f"bench: box reference {ref}")
    if args.mvm_large_only:
        print(json.dumps({"box_reference": ref, "mvm_large": mvm_large(torch, rtc, log, {})}),
              flush=True)
        return

    if args.timeline:
        print(json.dumps({"timeline": {"workload": args.timeline, "dtype": args.dtype,
                                       "us_after_last_chunk_seen": timeline(
                                           torch, rtc, args.timeline, args.dtype)}}),
              flush=True)
        return

    if args.frame_loop_only:
        wl_s, data_s = build_inputs("scao_sh_74", 64)
        inst_s = wl_s.instances[0]
        eng = load_engine(rtc, wl_s, data_s, "f32", "persistent")
        dfr = [torch.from_numpy(f).cuda() for f in data_s[0]["frames"]]
        r = batch_throughput(torch, eng, dfr, 256, 64)
        n_s = eng.infos[0]["n_slopes"]
        eng.close()
        # per frame: the matrix and command bytes of the MVM, and 2 B of raw pixel
        # plus 12 B of calibration per processed pixel
        px = (n_s // 2) * inst_s.wfs[0].px ** 2
        alg = mvm_alg_bytes(inst_s, n_s, "f32") + 14 * px
        print(json.dumps({"frame_loop_only": {"frames_per_s": round(r["frames_per_s"], 1),
                                              "frames_per_launch": 64,
                                              "alg_bytes_per_frame": alg}}), flush=True)
        return

    # ---------------------------------------------------------------- headline
    name = "ltao_68"
    log(f"bench: building inputs for {name}")
    wl, data = build_inputs(name, 64)
    ltao = wl.instances[0]
    fps = args.frames_per_step
    if args.roofline_only:
        eng = load_engine(rtc, wl, data, args.dtype, "stream", only=0)
        cold, n_cold = mvm_timing(torch, eng, n_iter=200, cold=True)
        alg = mvm_alg_bytes(ltao, eng.infos[0]["n_slopes"], args.dtype)
        eng.close()
        print(json.dumps({"roofline_only": {"avg_launch_us": round(cold * 1e6, 3),
                                            "launches": n_cold, "alg_bytes": alg,
                                            "gbs": round(alg / cold / 1e9, 1)}}), flush=True)
        return
    eng = load_engine(rtc, wl, data, args.dtype, "persistent")
    infos = eng.infos
    sw_run = args.steps * fps // 2
    switch = (0, sw_run, ltao.switch[1], ltao.switch[2])
    log(f"bench: {args.warmup} warm-up steps of {fps} frames")
    serve(eng, data, args.warmup * fps, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = eng.pace([(k, d["frames"]) for k, d in enumerate(data)], args.steps * fps, warmup=0,
                 period_s=PERIOD_S, readout_s=READOUT_S, first_frame=args.warmup * fps,
                 switch=switch)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lat = {inst.name: latency_stats(s[k]) for k, inst in enumerate(wl.instances)}
    eng.close()
    head = lat[ltao.name]
    log(f"bench: {name} {args.dtype}: LTAO p50 {head['p50']:.1f} p99 {head['p99']:.1f} "
        f"jitter {head['rms_jitter']:.2f} us (device p50 {head['device']['p50']:.1f}); "
        f"SCAO p50 {lat['scao_sh']['p50']:.1f} us; {dt:.2f} s")

    # ---------------------------------------------------------------- roofline
    # the LTAO matrix alone, cold: every launch after a 1 GiB cache flush
    eng = load_engine(rtc, wl, data, args.dtype, "stream", only=0)
    n_slopes = eng.infos[0]["n_slopes"]
    cold, n_cold = mvm_timing(torch, eng, n_iter=200, cold=True)
    extras = {}
    if not args.quick:
        # back-to-back launches and the per-launch batch path (inputs resident
        # in HBM): extras, outside the launches the roofline averages
        warm, _ = mvm_timing(torch, eng, n_iter=100)
        thr = batch_throughput(torch, eng,
                               [torch.from_numpy(f).cuda() for f in data[0]["frames"]], 256, 32)
        extras["ltao_mvm_warm_back_to_back_us"] = round(warm * 1e6, 3)
        extras["ltao_batch_throughput"] = rnd({**thr, "what": "LTAO instance alone, per-launch "
                                               "batch path over device-resident frames"})
    eng.close()
    alg = mvm_alg_bytes(ltao, n_slopes, args.dtype)
    roof = {"bound": "hbm", "achieved": round(alg / cold / 1e9, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(alg / cold / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(name, args.dtype, "k_mvm"),
            "kernel": f"k_mvm<{args.dtype}>",
            "what": f"split-K MVM on the LTAO matrix {ltao.n_act} x {n_slopes} "
                    f"({alg / 1e6:.0f} MB, beyond the 256 MB Infinity Cache), each launch after "
                    "a 1 GiB read-only cache flush",
            "avg_launch_us": round(cold * 1e6, 3), "launches_timed": n_cold,
            "algorithmic_bytes_per_launch": alg}
    log(f"bench: roofline {roof}")

    if not args.quick:
        for dt2 in [d for d in ("f32", "bf16", "fp8") if d != args.dtype]:
            eng = load_engine(rtc, wl, data, dt2, "persistent")
            l2 = serve(eng, data, args.extra_frames, 100,
                       switch=(0, args.extra_frames // 2 + 100, ltao.switch[1], ltao.switch[2]))
            eng.close()
            extras[f"{name}:{dt2}"] = {inst.name: rnd(l2[k]) for k, inst in enumerate(wl.instances)}
            log(f"bench: {name} {dt2}: LTAO p50 {l2[0]['p50']:.1f} p99 {l2[0]['p99']:.1f} us")
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        cpu = rnd(cpu_baseline(wl, data))
        log(f"bench: cpu {cpu}")
    del data
    if not args.quick:
        extras["mvm_beyond_infinity_cache"] = mvm_large(torch, rtc, log, {})
        extras["serving_mcao_us"] = serving_suite(torch, rtc, log, args.extra_frames)
        extras["scao_sh_74"] = scao_extras(torch, rtc, log)
        extras["scao_sh_74_f32_serving_features"] = telemetry_and_swap(torch, rtc, log)
        extras["latency_sweep_us"] = wfs_sweep(torch, rtc, 500, log)
        extras["pyramid_normalisation"] = pyramid_norms(torch, rtc, 2000, log)

    out = {
        "metric": METRIC, "value": round(head["p50"], 3), "unit": "us",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3 / args.steps, 4), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
        "data": "synthetic (seeded SH spots with photon and read noise, Gaussian control and "
                "POLC matrices; shapes of the paper's LTAO and SCAO systems)",
        "config": {"workload": name, "description": WORKLOAD_TEXT[name],
                   "instances_in_launch": [inst.name for inst in wl.instances],
                   "frames_per_step": fps, "frame_rate_hz": 1 / PERIOD_S,
                   "readout_ms": READOUT_S * 1e3, "cm_storage": args.dtype,
                   "gain_leak_switch_at_timed_frame": sw_run,
                   "path": "persistent frame loop, pixels from pinned host memory"},
        "latency_us": {k: rnd(v) for k, v in lat.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
        "box_reference": ref,
        "extras": extras or None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
