"""Benchmark of the pixel -> command hot path on one MI355X.

A step is one frame through every stage: calibration + slopes for every
sensor, the split-K control-matrix MVM, the in-order accumulation +
integrator (and the POLC product when the workload has it).  Frames are
resident in HBM before the timed region.  ``value`` is frames per second of
the batch path named by ``--path``:
  stream      per-launch kernels on one stream: frame f's split-K MVM (whose
              last wavefront per row tile runs the integrator) in one grid with
              frame f + 1's calibration + slopes (into the other slope buffer);
              the default, and the faster batch form;
  persistent  the persistent frame loop, ``--bank`` frames per launch.

Also reported on the same JSON line:
  roofline     the dominant kernel of the chosen path (k_mvm_next: frame f's MVM
               with frame f + 1's slopes in one grid; or k_frame_loop):
               algorithmic bytes per launch / its average duration, from HIP
               events recorded on its own stream over the timed region (one
               pair per run of 16 consecutive k_mvm_next launches, or per
               frame-loop launch); ``traffic`` from the committed rocprofv3
               counter summary when it was taken on the current kernel source;
  paths        frames/s and kernel GB/s of both batch forms for every storage
               type (FP32, BF16, FP8);
  latency_us   serving latency of the persistent loop per storage type (last
               chunk submitted from host memory -> commands seen on the host),
               frames paced at 500 Hz with the chunks spread over a 1.5 ms
               readout; p50 / p99 / RMS jitter; includes PCIe; ``zero_copy``
               the same with the chunks written in place into the lent ring
               slot (latency from the commit);
               ``telemetry_every_frame``: the same with slopes, counts and
               commands of every frame streamed to a host reader thread;
               ``matrix_swap``: a second control matrix staged by another thread
               while frames run and swapped in at a frame boundary, latency per
               phase;
  latency_suite_us  the same for the MCAO, LTAO + SCAO and 80x80 MCAO serving
               cases (one persistent launch each);
  latency_sweep_us  serving latency against sensor size at constant frame size;
  mvm          the standalone MVM kernel per storage type, warm (back to back)
               and after a 1 GiB read-only flush of the caches;
  mvm_beyond_infinity_cache  the same on the matrices larger than the cache;
  pyramid_normalisation  per-launch frames/s of the 92-pixel pyramid with local
               and with global normalisation;
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
MVM_RUN = 16               # per-launch path: k_mvm_next launches per event pair
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


def mvm_next_alg_bytes(inst, info, dtype):
    """Bytes of one k_mvm_next launch: frame f's MVM (matrix, slopes read,
    commands read and written) and frame f + 1's slopes (pixels, calibration,
    slopes written): a frame's bytes less the POLC product, a launch of its own."""
    b = alg_bytes_per_frame(inst, info, dtype)
    return b - (4 * inst.n_act * inst.n_act if inst.polc else 0)


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


def throughput(torch, eng, dframes, bank, steps, warmup, path):
    """Wall time of `steps` frames and the average duration of the path's
    dominant kernel: per launch of `bank` frames of the frame loop (HIP events
    around each process_frames call on its stream), or per k_mvm_next launch of
    the per-launch path (HIP events the library records around runs of
    MVM_RUN consecutive launches)."""
    st = torch.cuda.current_stream()
    run_steps(eng, dframes, bank, warmup, st)
    torch.cuda.synchronize()
    n_launch = (steps + bank - 1) // bank
    ev = []
    if path == "persistent":
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(n_launch)]
    else:
        eng.mvm_timing(0, steps, MVM_RUN)
    t0 = time.perf_counter()
    done = 0
    for i in range(n_launch):
        k = min(bank, steps - done)
        if ev:
            ev[i][0].record(st)
        eng.process_frames(0, dframes, k, stream=st)
        if ev:
            ev[i][1].record(st)
        done += k
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if ev:
        full = [a.elapsed_time(b) / 1e3 for a, b in ev[:steps // bank]]
        return dt, (sum(full) / len(full) if full else None), len(full), bank
    n, tot = eng.mvm_timing_read(0)
    eng.mvm_timing(0, 0, 1)
    return dt, (tot / n if n else None), n, 1


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


def _pct(v):
    import numpy as np
    v = np.asarray(v, dtype=np.float64)
    v = v[~np.isnan(v)]
    return {"p50": float(np.percentile(v, 50)), "p99": float(np.percentile(v, 99)),
            "mean": float(v.mean()), "rms_jitter": float(v.std()), "max": float(v.max())}


def serving_latency(eng, streams, n_frames, warmup=100, period_s=2e-3, readout_s=1.5e-3,
                    switch=None, zero_copy=False, swap=None, telemetry=None):
    """Paced serving loop from host memory for one or more instances of one
    engine, every sensor read out in parallel: chunk c of each sensor of an
    instance with n chunks is delivered (c + 1) * readout / n after the frame
    start.  streams: [(instance index, per-sensor frame banks)].  switch:
    (instance index, frame, gain, leak) applied through the API before that
    frame.  Returns per instance: host latency (last chunk submitted -> commands
    seen on the host) and the device part (the loop's own clock from the
    sentinel seeing the last chunk to the commands being published).
    zero_copy: chunks written in place into the lent ring slot (rtc_acquire_chunk,
    rtc_commit_chunk) instead of copied in by rtc_submit_pixel_chunk.
    swap: (instance index, frame, R, M): a second matrix set staged by another
    host thread from that frame on (rtc_stage_matrices, while frames run) and
    swapped in (rtc_swap_matrices) at the first frame start after the staging
    returned; adds per-phase latency statistics of that instance.
    telemetry: (decimation, slots): every instance streams slopes, counts and
    commands into its telemetry ring, drained by a reader thread per instance
    (rtc_telemetry_next) while frames run."""
    import threading
    plan = []
    for idx, banks in streams:
        info = eng.infos[idx]
        nw = info["n_wfs"]
        n_ch = [eng.n_chunks(idx, w) for w in range(nw)]
        for w in range(nw):
            for c in range(n_ch[w]):
                r0, r1 = eng.chunk_rows(idx, w, c)
                plan.append(((c + 1) * readout_s / n_ch[w], idx, w, c, r0, r1))
    plan.sort(key=lambda x: (x[0], x[1], x[2]))
    host = {idx: [] for idx, _ in streams}
    dev = {idx: [] for idx, _ in streams}
    fno = []
    banks = dict(streams)
    sw = {}
    readers, tel_stop, tel_got = [], threading.Event(), {}
    if telemetry is not None:
        for idx, _ in streams:
            eng.telemetry_enable(idx, telemetry[0], telemetry[1])
            tel_got[idx] = [0, 0]

            def drain_tel(idx=idx):
                while not tel_stop.is_set():
                    try:
                        _, _, _, ti = eng.telemetry_next(idx, timeout_s=0.05)
                    except Exception:
                        continue
                    tel_got[idx][0] += 1
                    tel_got[idx][1] += ti["lost"]
            th_t = threading.Thread(target=drain_tel)
            th_t.start()
            readers.append(th_t)
    t_next = time.perf_counter()
    for f in range(n_frames + warmup):
        if switch is not None and f == switch[1]:
            eng.set_params(switch[0], switch[2], switch[3])
        if swap is not None and f == swap[1]:
            def stage():
                t0 = time.perf_counter()
                eng.stage_matrices(swap[0], swap[2], M=swap[3])
                sw["stage_s"] = time.perf_counter() - t0
            th = threading.Thread(target=stage)
            th.start()
        if swap is not None and f > swap[1] and "f_eff" not in sw and not th.is_alive():
            th.join()
            sw["f_eff"] = eng.swap_matrices(swap[0])
        t_frame = t_next
        for t_c, idx, w, c, r0, r1 in plan:
            while time.perf_counter() < t_frame + t_c:
                pass
            bank = banks[idx][w]
            if zero_copy:
                eng.acquire_chunk(idx, w, f, c)[...] = bank[f % bank.shape[0]][r0:r1]
                eng.commit_chunk(idx, w, f, c)
            else:
                eng.submit_chunk(idx, w, f, c, bank[f % bank.shape[0]][r0:r1])
        for idx, _ in streams:
            _, info = eng.wait_commands(idx, f, timeout_s=5.0)
            if f >= warmup:
                host[idx].append((info["t_ready_ns"] - info["t_last_chunk_ns"]) / 1e3)
                # a frame published before its last chunk arrived (its last rows
                # hold no pixel it needs) counts as 0
                dev[idx].append(max(0, info["dev_ticks_cmd"] - info["dev_ticks_start"]) * 0.01
                                if info["dev_ticks_start"] else float("nan"))
        if f >= warmup:
            fno.append(f)
        t_next = t_frame + period_s
    if swap is not None and "f_eff" not in sw:
        th.join()
        raise RuntimeError("the staged matrices were not swapped in before the last frame")
    if telemetry is not None:
        time.sleep(0.1)
        tel_stop.set()
        for th_t in readers:
            th_t.join()
        for idx, _ in streams:
            eng.telemetry_enable(idx, 1, 0)
    out = {}
    for idx, _ in streams:
        r = _pct(host[idx])
        r["frames"] = len(host[idx])
        r["device"] = _pct(dev[idx])
        if telemetry is not None:
            r["telemetry"] = {"decimation": telemetry[0], "slots": telemetry[1],
                              "records_read": tel_got[idx][0], "records_lost": tel_got[idx][1]}
        if swap is not None and swap[0] == idx:
            import numpy as np
            fa, h, d = np.asarray(fno), np.asarray(host[idx]), np.asarray(dev[idx])
            fe = sw["f_eff"]
            phases = {"before_stage": fa < swap[1],
                      "during_stage": (fa >= swap[1]) & (fa < fe),
                      "first_20_after_swap": (fa >= fe) & (fa < fe + 20),
                      "after_swap": fa >= fe}
            r["swap"] = {"stage_s": sw["stage_s"], "stage_frame": swap[1], "f_eff": fe}
            for k, m in phases.items():
                if m.any():
                    r["swap"][k] = {"frames": int(m.sum()), "host": _pct(h[m]),
                                    "device": _pct(d[m])}
        out[idx] = r
    return out


SERVING_NOTE = {"pacing": "500 Hz frames, every sensor's chunks spread over a 1.5 ms readout",
                "host": "last chunk submitted (host memcpy into the pinned ring, doorbell) -> "
                        "commands seen in the pinned mailbox by the host",
                "device": "device clock (100 MHz): the loop's sentinel seeing the frame's last "
                          "chunk -> the last tile's commands published"}


def latency_suite(torch, rtc, dtypes, n_frames, log):
    """ELT-scale serving cases in one persistent launch each: MCAO (6 LGS SH 74x74 + 3 NGS
    2x2, POLC) and LTAO (6 LGS SH 68x68 + 1 NGS 8x8, POLC, gain and leak switched
    mid-run) running beside the SCAO SH 74x74 instance of uneven size."""
    import numpy as np
    import synth
    res = {}
    for name in ("mcao_74", "ltao_68", "mcao_80"):
        wl = synth.get_workload(name)
        mats, banks = [], []
        for i, inst in enumerate(wl.instances):
            R = synth.control_matrix(wl, i)
            M = None
            if inst.polc:
                na = inst.n_act
                M = synth.gaussian_matrix(na, na, 0.5 / np.sqrt(na),
                                          synth.seed_for(wl.index, i, 99, 5), np.float32)
            fr, cal = [], []
            for w in range(len(inst.wfs)):
                f_w, c_w = synth.sensor_inputs(wl, i, w, n=16)
                fr.append(f_w)
                cal.append(c_w)
            mats.append((R, M, cal))
            banks.append(fr)
        # the paper-size MCAO's FP32 matrix (1.4 GB) is not one of its storage choices
        for dtype in [d for d in dtypes if name != "mcao_80" or d != "f32"]:
            log(f"bench: serving {name} {dtype}")
            eng = rtc.Engine([(inst, dtype) for inst in wl.instances], ring_depth=4,
                             mode="persistent")
            for i, (R, M, cal) in enumerate(mats):
                eng.load_matrices(i, R, M=M)
                for w, c in enumerate(cal):
                    eng.load_calibration(i, w, c.dark, c.flat, c.bg, c.thr, c.ref)
            switch = None
            sw_inst = [i for i, inst in enumerate(wl.instances) if inst.switch is not None]
            if sw_inst:
                i = sw_inst[0]
                switch = (i, n_frames // 2 + 100, wl.instances[i].switch[1],
                          wl.instances[i].switch[2])
            lat = serving_latency(eng, [(i, banks[i]) for i in range(len(wl.instances))],
                                  n_frames, switch=switch)
            if name == "mcao_74" and dtype == dtypes[0]:
                # the same with slopes, counts and commands of every frame streamed
                eng.set_state(0, None, None, 0)
                tel = serving_latency(eng, [(0, banks[0])], n_frames, telemetry=(1, 256))[0]
                res[f"{name}:{wl.instances[0].name}:{dtype}:telemetry_every_frame"] = {
                    k: (round(v, 3) if isinstance(v, float) else v) for k, v in tel.items()}
                log(f"bench: {name} {dtype} with telemetry: p50 {tel['p50']:.1f} "
                    f"p99 {tel['p99']:.1f} us")
            eng.close()
            for i, inst in enumerate(wl.instances):
                key = f"{name}:{inst.name}:{dtype}"
                r = lat[i]
                r.update({"n_act": inst.n_act, "n_wfs": len(inst.wfs), "polc": inst.polc,
                          "instances_in_launch": len(wl.instances)})
                if switch is not None and switch[0] == i:
                    r["gain_leak_switch_at_frame"] = switch[1] - 100
                res[key] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items()}
                log(f"bench: {key}: p50 {r['p50']:.1f} p99 {r['p99']:.1f} "
                    f"jitter {r['rms_jitter']:.2f} us (device p50 {r['device']['p50']:.1f})")
        del mats, banks
    return res


def wfs_sweep(torch, rtc, n_frames, log):
    """Serving latency against sensor size at a constant frame size (the paper's
    scaling study): Shack-Hartmann 74..110 subapertures across on 800x800 frames
    (10, 10, 8, 8, 7 px per subaperture) and pyramid 80..120 pupil pixels across
    on 240x240 frames, each with a 5318-actuator FP32 control matrix."""
    import numpy as np
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
        eng = rtc.Engine([(inst, "f32")], ring_depth=4, mode="persistent")
        eng.load_matrices(0, R)
        eng.load_calibration(0, 0, cal.dark, cal.flat, cal.bg, cal.thr, cal.ref)
        r = serving_latency(eng, [(0, [fr])], n_frames)[0]
        eng.close()
        key = f"{kind}_{n}x{n}"
        res[key] = {"n_slopes": inst.n_slopes, "n_act": inst.n_act,
                    "px_per_subap": getattr(wfs, "px", None),
                    **{k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items()}}
        log(f"bench: sweep {key}: {inst.n_slopes} slopes, p50 {r['p50']:.1f} p99 {r['p99']:.1f} "
            f"jitter {r['rms_jitter']:.2f} us (device p50 {r['device']['p50']:.1f})")
    return res


def pyramid_norms(torch, rtc, steps, log):
    """Per-launch batch frames/s of the 92-pixel pyramid (5318 x 12288 FP32
    matrix) with local and with global normalisation (the latter adds the
    pupil-sum kernel before each frame's slopes)."""
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
        eng = rtc.Engine([(inst, "f32")], mode="stream")
        eng.load_matrices(0, R)
        eng.load_calibration(0, 0, cal.dark, cal.flat, cal.bg, cal.thr, cal.ref)
        d = [torch.from_numpy(fr).cuda()]
        st = torch.cuda.current_stream()
        run_steps(eng, d, 16, 64, st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_steps(eng, d, 16, steps, st)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        eng.close()
        res[norm] = {"frames_per_s": round(steps / dt, 1), "n_slopes": inst.n_slopes}
        log(f"bench: pyramid 92 px {norm} normalisation: {steps / dt:.0f} frames/s")
    return res


# matrices larger than the 256 MB Infinity Cache: their MVM rate is an HBM rate
LARGE_MVM = (("mcao_74", "bf16"), ("mcao_74", "fp8"), ("ltao_68", "f32"), ("ltao_68", "bf16"),
             ("mcao_80", "bf16"), ("mcao_80", "fp8"))


def mvm_large(torch, rtc, log):
    """The standalone MVM on the MCAO and LTAO matrices (each beyond the Infinity
    Cache), warm (back to back) and after a 1 GiB read-only cache flush."""
    import numpy as np
    import synth
    res = {}
    done = {}
    for name, dtype in LARGE_MVM:
        wl = synth.get_workload(name)
        inst = wl.instances[0]
        if name not in done:
            done.clear()
            done[name] = synth.control_matrix(wl, 0)
        R = done[name]
        na = inst.n_act
        M = (synth.gaussian_matrix(na, na, 0.5 / np.sqrt(na), synth.seed_for(wl.index, 0, 99, 5),
                                   np.float32) if inst.polc else None)
        eng = rtc.Engine([(inst, dtype)], mode="stream")
        eng.load_matrices(0, R, M=M)
        info = eng.infos[0]
        warm = mvm_timing(torch, eng, n_iter=100)
        cold = mvm_timing(torch, eng, n_iter=100, cold=True)
        eng.close()
        alg = (na * info["n_slopes"] * ELEM[dtype] + 4 * info["n_slopes"] + 4 * na
               + (4 * na if dtype == "fp8" else 0))
        r = {"n_act": na, "n_slopes": info["n_slopes"], "alg_bytes": alg,
             "warm_us": warm * 1e6, "warm_gbs": alg / warm / 1e9, "warm_frac": alg / warm / 1e9 / HBM_PEAK_GBS,
             "cold_us": cold * 1e6, "cold_gbs": alg / cold / 1e9, "cold_frac": alg / cold / 1e9 / HBM_PEAK_GBS,
             # HBM bytes of one warm launch from the committed counter summary
             "traffic": measured_traffic(name, dtype, "k_mvm")}
        res[f"{name}:{dtype}"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
        log(f"bench: mvm {name} {dtype}: {alg / 1e6:.0f} MB, warm {warm * 1e6:.1f} us "
            f"({r['warm_gbs']:.0f} GB/s), cold {cold * 1e6:.1f} us ({r['cold_gbs']:.0f} GB/s)")
    return res


def box_reference(torch, reps=10):
    """HBM reference of this particular box: a plain 512 MiB device-to-device
    copy (read + write bytes per second, median of `reps`).  MI355X boxes in one
    pool have shown different sustained bandwidths for the same code, so every
    kernel figure is reported beside this one."""
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
    ap.add_argument("--path", default="stream", choices=("stream", "persistent"))
    ap.add_argument("--variants", default="bf16,fp8")
    ap.add_argument("--bank", type=int, default=64)
    ap.add_argument("--latency-frames", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--no-latency-suite", action="store_true",
                    help="skip the MCAO / LTAO+SCAO serving cases")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the serving-latency sweep over sensor sizes")
    ap.add_argument("--sweep-frames", type=int, default=500)
    ap.add_argument("--no-mvm-large", action="store_true",
                    help="skip the standalone MVM on the MCAO / LTAO matrices")
    ap.add_argument("--mvm-large-only", action="store_true",
                    help="only the standalone MVM on the MCAO / LTAO matrices (for profiling)")
    ap.add_argument("--quick", action="store_true",
                    help="the chosen path and storage type only (for profiling)")
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

    if args.copy_probe:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copy probe: 5 x {src.numel() * 4} bytes read and written")
        del src, dst

    def mvm_alg_bytes(info, dtype):
        return (inst.n_act * info["n_slopes"] * ELEM[dtype] + 4 * info["n_slopes"]
                + 4 * inst.n_act + (4 * inst.n_act if dtype == "fp8" else 0))

    def run_path(eng, dtype, path):
        info = eng.infos[0]
        dt, kern_s, n_timed, per = throughput(torch, eng, dframes, args.bank, args.steps,
                                              args.warmup, path)
        per_frame = alg_bytes_per_frame(inst, info, dtype)
        res = {"frames_per_s": args.steps / dt, "ms_per_step": dt * 1e3 / args.steps,
               "alg_bytes_per_frame": per_frame}
        if kern_s:
            kb = (per_frame * per if path == "persistent"
                  else mvm_next_alg_bytes(inst, info, dtype))
            res.update({"kernel": ("k_frame_loop" if path == "persistent"
                                   else f"k_mvm_next<{dtype}>"),
                        "kernel_us": kern_s * 1e6, "kernel_launches_timed": n_timed,
                        "kernel_alg_bytes": kb, "kernel_gbs": kb / kern_s / 1e9})
        log(f"bench: {dtype} {path}: {res}")
        return res

    def mvm_standalone(eng, dtype):
        info = eng.infos[0]
        warm = mvm_timing(torch, eng)
        cold = mvm_timing(torch, eng, cold=True)
        alg = mvm_alg_bytes(info, dtype)
        return {"alg_bytes": alg, "cm_bytes_stored": info["cm_bytes"],
                "warm_us": warm * 1e6, "warm_gbs": alg / warm / 1e9,
                "cold_us": cold * 1e6, "cold_gbs": alg / cold / 1e9}

    ref = box_reference(torch)
    log(f"bench: box reference {ref}")
    if args.mvm_large_only:
        print(json.dumps({"box_reference": ref, "mvm_large": mvm_large(torch, rtc, log)}), flush=True)
        return

    dtypes = [args.dtype] + ([] if args.quick else
                             [v for v in args.variants.split(",") if v and v != args.dtype])
    paths = {"stream": {}, "persistent": {}}
    mvm = {}
    latency = {}
    for dtype in dtypes:
        for path in ("stream", "persistent"):
            if args.quick and path != args.path:
                continue
            eng = make_engine(rtc, inst, dtype, cals, R, M, mode=path)
            paths[path][dtype] = run_path(eng, dtype, path)
            if path == "stream":
                mvm[dtype] = mvm_standalone(eng, dtype)
                log(f"bench: {dtype} mvm: {mvm[dtype]}")
            elif not args.quick and not args.no_latency:
                eng.set_state(0, None, None, 0)
                latency[dtype] = serving_latency(eng, [(0, frames)], args.latency_frames)[0]
                eng.set_state(0, None, None, 0)
                latency[dtype]["zero_copy"] = serving_latency(
                    eng, [(0, frames)], args.latency_frames, zero_copy=True)[0]
                if dtype == args.dtype:
                    # slopes, counts and commands of every frame streamed to the host
                    eng.set_state(0, None, None, 0)
                    latency[dtype]["telemetry_every_frame"] = serving_latency(
                        eng, [(0, frames)], args.latency_frames, telemetry=(1, 256))[0]
                    # a second control matrix staged and swapped in while frames run
                    import numpy as np
                    import synth
                    eng.set_state(0, None, None, 0)
                    R2 = synth.gaussian_matrix(inst.n_act, R.shape[1], 1.0 / np.sqrt(R.shape[1]),
                                               synth.seed_for(wl.index, 0, 77, 1), np.float32)
                    M2 = None if M is None else synth.gaussian_matrix(
                        inst.n_act, inst.n_act, 0.5 / np.sqrt(inst.n_act),
                        synth.seed_for(wl.index, 0, 77, 2), np.float32)
                    latency[dtype]["matrix_swap"] = serving_latency(
                        eng, [(0, frames)], args.latency_frames,
                        swap=(0, 100 + args.latency_frames // 5, R2, M2))[0]["swap"]
                log(f"bench: {dtype} latency: {latency[dtype]}")
            eng.close()

    large = None
    if not args.quick and not args.no_mvm_large:
        large = mvm_large(torch, rtc, log)

    suite = None
    if not args.quick and not args.no_latency and not args.no_latency_suite:
        suite = latency_suite(torch, rtc, dtypes, args.latency_frames, log)

    sweep = None
    if not args.quick and not args.no_latency and not args.no_sweep:
        sweep = wfs_sweep(torch, rtc, args.sweep_frames, log)
    pyr_norm = None if args.quick else pyramid_norms(torch, rtc, 2000, log)

    cpu = None
    if not args.quick and not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        cpu = cpu_baseline(inst, frames, cals, R, M)

    main_res = paths[args.path][args.dtype]
    achieved = main_res["kernel_gbs"]
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args.workload, args.dtype, main_res["kernel"]),
            "kernel": main_res["kernel"],
            "avg_launch_us": round(main_res["kernel_us"], 3),
            "launches_timed": main_res["kernel_launches_timed"],
            "algorithmic_bytes_per_launch": main_res["kernel_alg_bytes"]}

    def rnd(d):
        return {k: (round(v, 3) if isinstance(v, float) else rnd(v) if isinstance(v, dict)
                    else v) for k, v in d.items()}

    out = {
        "metric": METRIC, "value": round(main_res["frames_per_s"], 1), "unit": "frames/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
        "data": "synthetic (seeded SH spots / pyramid images with the paper's shapes, "
                "Gaussian control matrix)",
        "config": {"workload": args.workload, "description": WORKLOAD_TEXT.get(args.workload),
                   "path": {"stream": "per-launch kernels",
                            "persistent": "persistent frame loop"}[args.path],
                   "frames_in_bank": args.bank, "cm_storage": args.dtype},
        "roofline": roof,
        "box_reference": ref,
        "latency_us": ({k: rnd(v) for k, v in latency.items()} | {"what": SERVING_NOTE}
                       if latency else None),
        "latency_suite_us": ({**suite, "what": SERVING_NOTE} if suite else None),
        "paths": {p: {k: rnd(v) for k, v in d.items()} for p, d in paths.items() if d},
        "mvm": {k: rnd(v) for k, v in mvm.items()},
        "mvm_beyond_infinity_cache": large,
        "latency_sweep_us": ({**sweep, "what": SERVING_NOTE} if sweep else None),
        "pyramid_normalisation": pyr_norm,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
