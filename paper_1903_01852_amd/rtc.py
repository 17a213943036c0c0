"""Python binding of ``librtc.so`` (argument marshalling only).

Every step of the pixel -> command path runs in the library's gfx950
kernels; this module converts arguments and checks status codes.  torch is
imported first so that the library binds to the same HIP runtime as torch.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library links against)

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librtc.so")

RTC_OK = 0
STATUS = {0: "RTC_OK", -1: "RTC_E_INVAL", -2: "RTC_E_NOMEM", -3: "RTC_E_DEVICE",
          -4: "RTC_E_TIMEOUT", -5: "RTC_E_STATE", -6: "RTC_E_RING_FULL",
          -7: "RTC_E_FRAME_DROPPED", -8: "RTC_E_SCRATCH"}
WFS_KIND = {"sh": 0, "pyr": 1}
CM_DTYPE = {"f32": 0, "bf16": 1, "fp8": 2}
CM_ELEM = {"f32": 4, "bf16": 2, "fp8": 1}
THR_MODE = {"subtract": 0, "zero": 1, "none": 2}
MODE = {"stream": 0, "persistent": 1}
PYR_NORM = {"local": 0, "global": 1}
MAX_WFS = 16

EXPORTS = ("rtc_create", "rtc_destroy", "rtc_strerror", "rtc_get_info", "rtc_chunk_rows",
           "rtc_load_matrices", "rtc_load_calibration", "rtc_set_params", "rtc_get_state",
           "rtc_set_state", "rtc_submit_pixel_chunk", "rtc_wait_commands",
           "rtc_process_frames", "rtc_read_slopes", "rtc_read_matrix", "rtc_run_mvm",
           "rtc_mvm_timing", "rtc_mvm_timing_read", "rtc_trace_enable", "rtc_trace_read",
           "rtc_acquire_chunk", "rtc_commit_chunk", "rtc_stage_matrices",
           "rtc_swap_matrices", "rtc_telemetry_enable", "rtc_telemetry_next",
           "rtc_process_frames_noalloc", "rtc_pacer_run")
TRACE_EVENTS = ("frame_start", "gate", "centroids", "mvm_first", "mvm_last", "ingest",
                "accum", "frame_end", "cen_start", "last_block", "tile_ready", "cmds",
                "ingest_start", "summed", "joined")


class RtcError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}")


class WfsDescC(C.Structure):
    _fields_ = [("kind", C.c_int32), ("frame_h", C.c_int32), ("frame_w", C.c_int32),
                ("n_chunks", C.c_int32), ("thr_mode", C.c_int32),
                ("nsub", C.c_int32), ("px", C.c_int32), ("origin_row", C.c_int32),
                ("origin_col", C.c_int32), ("subap_valid", C.POINTER(C.c_uint8)),
                ("pupil_px", C.c_int32), ("quad_row", C.c_int32 * 4),
                ("quad_col", C.c_int32 * 4), ("pupil_valid", C.POINTER(C.c_uint8)),
                ("pyr_norm", C.c_int32)]


class InstanceDescC(C.Structure):
    _fields_ = [("n_wfs", C.c_int32), ("wfs", C.POINTER(WfsDescC)), ("n_act", C.c_int32),
                ("cm_dtype", C.c_int32), ("polc", C.c_int32), ("gain", C.c_float),
                ("leak", C.c_float)]


class CreateDescC(C.Structure):
    _fields_ = [("device", C.c_int32), ("n_inst", C.c_int32),
                ("inst", C.POINTER(InstanceDescC)), ("ring_depth", C.c_int32),
                ("mode", C.c_int32)]


class FrameInfoC(C.Structure):
    _fields_ = [("frame", C.c_uint64), ("t_last_chunk_ns", C.c_int64),
                ("t_ready_ns", C.c_int64), ("dev_ticks_start", C.c_uint64),
                ("dev_ticks_cmd", C.c_uint64), ("drops", C.c_uint32), ("reserved", C.c_uint32)]


class PacerStreamC(C.Structure):
    _fields_ = [("inst", C.c_int32), ("n_bank", C.c_int32), ("banks", C.POINTER(C.c_void_p)),
                ("cmds", C.c_void_p)]


class PacerDescC(C.Structure):
    _fields_ = [("period_s", C.c_double), ("readout_s", C.c_double), ("n_frames", C.c_int32),
                ("warmup", C.c_int32), ("first_frame", C.c_uint64), ("zero_copy", C.c_int32),
                ("switch_stream", C.c_int32), ("switch_frame", C.c_int32),
                ("switch_gain", C.c_float), ("switch_leak", C.c_float), ("pin", C.c_int32),
                ("timeout_s", C.c_double)]


class PacerSampleC(C.Structure):
    _fields_ = [("frame", C.c_uint64), ("host_us", C.c_double), ("dev_us", C.c_double),
                ("complete_us", C.c_double), ("late_us", C.c_double),
                ("start_late_us", C.c_double), ("dev_ticks_start", C.c_uint64),
                ("dev_ticks_cmd", C.c_uint64)]


class TelemetryInfoC(C.Structure):
    _fields_ = [("frame", C.c_uint64), ("dropped", C.c_uint32), ("lost", C.c_uint32)]


class InstanceInfoC(C.Structure):
    _fields_ = [("n_wfs", C.c_int32), ("n_units", C.c_int32), ("n_slopes", C.c_int32),
                ("n_act", C.c_int32), ("n_kblocks", C.c_int32), ("mask_words", C.c_int32),
                ("cm_bytes", C.c_int64), ("cm_bytes_logical", C.c_int64),
                ("polc_bytes", C.c_int64)]


_lib = None


def lib() -> C.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                               "`python -m paper_1903_01852_amd.build`")
        L = C.CDLL(_LIB_PATH)
        vp, i32, u64, i64 = C.c_void_p, C.c_int32, C.c_uint64, C.c_int64
        L.rtc_create.argtypes = [C.POINTER(CreateDescC), C.POINTER(vp)]
        L.rtc_destroy.argtypes = [vp]
        L.rtc_strerror.argtypes = [C.c_int]
        L.rtc_strerror.restype = C.c_char_p
        L.rtc_get_info.argtypes = [vp, i32, C.POINTER(InstanceInfoC)]
        L.rtc_chunk_rows.argtypes = [vp, i32, i32, i32, C.POINTER(i32), C.POINTER(i32)]
        L.rtc_load_matrices.argtypes = [vp, i32, vp, vp, vp]
        L.rtc_stage_matrices.argtypes = [vp, i32, vp, vp, vp]
        L.rtc_telemetry_enable.argtypes = [vp, i32, i32, i32]
        L.rtc_telemetry_next.argtypes = [vp, i32, vp, vp, vp, vp, i64,
                                         C.POINTER(TelemetryInfoC)]
        L.rtc_swap_matrices.argtypes = [vp, i32, C.POINTER(u64)]
        L.rtc_load_calibration.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp]
        L.rtc_set_params.argtypes = [vp, i32, C.c_float, C.c_float, C.POINTER(u64)]
        L.rtc_get_state.argtypes = [vp, i32, vp, vp, C.POINTER(u64)]
        L.rtc_set_state.argtypes = [vp, i32, vp, vp, u64]
        L.rtc_submit_pixel_chunk.argtypes = [vp, i32, i32, u64, i32, vp]
        L.rtc_wait_commands.argtypes = [vp, i32, u64, vp, i64, C.POINTER(FrameInfoC)]
        L.rtc_acquire_chunk.argtypes = [vp, i32, i32, u64, i32, C.POINTER(C.c_void_p),
                                        C.POINTER(i32)]
        L.rtc_commit_chunk.argtypes = [vp, i32, i32, u64, i32]
        L.rtc_process_frames.argtypes = [vp, i32, C.POINTER(vp), C.POINTER(i64), i32, vp, vp,
                                         vp, vp]
        L.rtc_process_frames_noalloc.argtypes = [vp, i32, C.POINTER(vp), C.POINTER(i64), i32,
                                                 vp, vp, vp, vp]
        L.rtc_read_slopes.argtypes = [vp, i32, vp, vp, vp]
        L.rtc_read_matrix.argtypes = [vp, i32, vp, vp]
        L.rtc_run_mvm.argtypes = [vp, i32, i32, vp]
        L.rtc_mvm_timing.argtypes = [vp, i32, i32, i32]
        L.rtc_mvm_timing_read.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(C.c_double)]
        L.rtc_pacer_run.argtypes = [vp, C.POINTER(PacerDescC), i32, C.POINTER(PacerStreamC),
                                    C.POINTER(PacerSampleC), C.POINTER(i32)]
        L.rtc_trace_enable.argtypes = [vp, i32]
        L.rtc_trace_read.argtypes = [vp, vp, i64, C.POINTER(i32), C.POINTER(i32)]
        for name in EXPORTS:
            if name != "rtc_strerror":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _ok(status: int, where: str) -> None:
    if status != RTC_OK:
        raise RtcError(status, where)


def _ptr(a) -> C.c_void_p | None:
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return C.c_void_p(a.data_ptr())
    return C.c_void_p(a.ctypes.data)


def _stream_ptr(stream) -> C.c_void_p | None:
    if stream is None:
        return None
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def wfs_to_c(w, keep: list) -> WfsDescC:
    """Sensor description from an object with the synth sensor attributes."""
    d = WfsDescC()
    d.kind = WFS_KIND[w.kind]
    d.frame_h, d.frame_w = int(w.frame_h), int(w.frame_w)
    d.n_chunks = int(w.n_chunks)
    d.thr_mode = THR_MODE[w.thr_mode]
    valid = np.ascontiguousarray(np.asarray(w.valid, np.uint8))
    keep.append(valid)
    vptr = valid.ctypes.data_as(C.POINTER(C.c_uint8))
    if w.kind == "sh":
        d.nsub, d.px = int(w.nsub), int(w.px)
        d.origin_row, d.origin_col = (int(v) for v in w.origin)
        d.subap_valid = vptr
    else:
        d.pupil_px = int(w.pupil_px)
        for q, (r, c) in enumerate(w.quad_origins):
            d.quad_row[q], d.quad_col[q] = int(r), int(c)
        d.pupil_valid = vptr
        d.pyr_norm = PYR_NORM[getattr(w, "norm", "local")]
    return d


class Engine:
    """One engine: device buffers, pixel rings and command state of its instances.

    ``instances`` is a list of (instance, cm_dtype) pairs; an instance has the
    attributes ``wfs`` (sensors), ``n_act``, ``polc``, ``gain`` and ``leak``.
    """

    def __init__(self, instances, device: int = 0, ring_depth: int = 4, mode: str = "stream"):
        L = lib()
        self._keep = []
        insts = (InstanceDescC * len(instances))()
        self.specs = []
        for i, (inst, dtype) in enumerate(instances):
            ws = (WfsDescC * len(inst.wfs))()
            for j, w in enumerate(inst.wfs):
                ws[j] = wfs_to_c(w, self._keep)
            self._keep.append(ws)
            insts[i].n_wfs = len(inst.wfs)
            insts[i].wfs = ws
            insts[i].n_act = int(inst.n_act)
            insts[i].cm_dtype = CM_DTYPE[dtype]
            insts[i].polc = int(bool(inst.polc))
            insts[i].gain = float(inst.gain)
            insts[i].leak = float(inst.leak)
            self.specs.append((inst, dtype))
        desc = CreateDescC(device=device, n_inst=len(instances), inst=insts,
                           ring_depth=ring_depth, mode=MODE[mode])
        h = C.c_void_p()
        _ok(L.rtc_create(C.byref(desc), C.byref(h)), "rtc_create")
        self._h = h
        self._keep = []
        self.infos = [self.info(i) for i in range(len(instances))]

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            lib().rtc_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- queries
    def info(self, inst: int = 0) -> dict:
        s = InstanceInfoC()
        _ok(lib().rtc_get_info(self._h, inst, C.byref(s)), "rtc_get_info")
        return {k: getattr(s, k) for k, _ in InstanceInfoC._fields_}

    def n_chunks(self, inst: int, wfs: int) -> int:
        """Row chunks per frame of sensor wfs, as configured."""
        return int(self.specs[inst][0].wfs[wfs].n_chunks)

    def chunk_rows(self, inst: int, wfs: int, chunk: int):
        a, b = C.c_int32(), C.c_int32()
        _ok(lib().rtc_chunk_rows(self._h, inst, wfs, chunk, C.byref(a), C.byref(b)),
            "rtc_chunk_rows")
        return a.value, b.value

    # -- configuration
    def load_matrices(self, inst: int, R, D=None, M=None):
        R = np.ascontiguousarray(R, np.float32)
        D = None if D is None else np.ascontiguousarray(D, np.float64)
        M = None if M is None else np.ascontiguousarray(M, np.float32)
        _ok(lib().rtc_load_matrices(self._h, inst, _ptr(R), _ptr(D), _ptr(M)),
            "rtc_load_matrices")

    def stage_matrices(self, inst: int, R, D=None, M=None):
        R = np.ascontiguousarray(R, np.float32)
        D = None if D is None else np.ascontiguousarray(D, np.float64)
        M = None if M is None else np.ascontiguousarray(M, np.float32)
        _ok(lib().rtc_stage_matrices(self._h, inst, _ptr(R), _ptr(D), _ptr(M)),
            "rtc_stage_matrices")

    def swap_matrices(self, inst: int) -> int:
        f = C.c_uint64()
        _ok(lib().rtc_swap_matrices(self._h, inst, C.byref(f)), "rtc_swap_matrices")
        return f.value

    def telemetry_enable(self, inst: int, decimation: int, n_slots: int):
        _ok(lib().rtc_telemetry_enable(self._h, inst, decimation, n_slots),
            "rtc_telemetry_enable")

    def telemetry_next(self, inst: int = 0, timeout_s: float = 5.0, masks: bool = False):
        """Next telemetry record: (slopes, counts, cmds, info dict), and with
        masks=True the thresholded-pixel masks (uint64 words) as a fifth item."""
        info = self.infos[inst]
        s = np.empty(info["n_slopes"], np.float32)
        c = np.empty(info["n_units"], np.int32)
        a = np.empty(info["n_act"], np.float32)
        m = np.empty(info["mask_words"], np.uint64) if masks else None
        ti = TelemetryInfoC()
        _ok(lib().rtc_telemetry_next(self._h, inst, _ptr(s), _ptr(c), _ptr(a), _ptr(m),
                                     int(timeout_s * 1e9), C.byref(ti)), "rtc_telemetry_next")
        d = {"frame": ti.frame, "dropped": ti.dropped, "lost": ti.lost}
        return (s, c, a, d, m) if masks else (s, c, a, d)

    def load_calibration(self, inst: int, wfs: int, dark=None, flat=None, bg=None, thr=None,
                         ref=None):
        arrs = [None if a is None else np.ascontiguousarray(a, np.float32)
                for a in (dark, flat, bg, thr, ref)]
        _ok(lib().rtc_load_calibration(self._h, inst, wfs, *[_ptr(a) for a in arrs]),
            "rtc_load_calibration")

    def set_params(self, inst: int, gain: float, leak: float) -> int:
        f = C.c_uint64()
        _ok(lib().rtc_set_params(self._h, inst, gain, leak, C.byref(f)), "rtc_set_params")
        return f.value

    def get_state(self, inst: int = 0):
        n = self.infos[inst]["n_act"]
        a, p = np.empty(n, np.float32), np.empty(n, np.float32)
        f = C.c_uint64()
        _ok(lib().rtc_get_state(self._h, inst, _ptr(a), _ptr(p), C.byref(f)), "rtc_get_state")
        return a, p, f.value

    def set_state(self, inst: int, a=None, p=None, next_frame: int = 0):
        a = None if a is None else np.ascontiguousarray(a, np.float32)
        p = None if p is None else np.ascontiguousarray(p, np.float32)
        _ok(lib().rtc_set_state(self._h, inst, _ptr(a), _ptr(p), next_frame), "rtc_set_state")

    # -- serving
    def submit_chunk(self, inst: int, wfs: int, frame: int, chunk: int, rows: np.ndarray):
        rows = np.ascontiguousarray(rows, np.uint16)
        _ok(lib().rtc_submit_pixel_chunk(self._h, inst, wfs, frame, chunk, _ptr(rows)),
            "rtc_submit_pixel_chunk")

    def submit_status(self, inst: int, wfs: int, frame: int, chunk: int, rows: np.ndarray) -> int:
        rows = np.ascontiguousarray(rows, np.uint16)
        return lib().rtc_submit_pixel_chunk(self._h, inst, wfs, frame, chunk, _ptr(rows))

    def acquire_chunk(self, inst: int, wfs: int, frame: int, chunk: int) -> np.ndarray:
        """Zero-copy submit, first half: a (rows, frame_w) uint16 view of the pinned
        ring slot the chunk goes to.  Fill it, then call commit_chunk."""
        p, pitch = C.c_void_p(), C.c_int32()
        _ok(lib().rtc_acquire_chunk(self._h, inst, wfs, frame, chunk, C.byref(p),
                                    C.byref(pitch)), "rtc_acquire_chunk")
        r0, r1 = self.chunk_rows(inst, wfs, chunk)
        w = int(self.specs[inst][0].wfs[wfs].frame_w)
        n = (r1 - r0 - 1) * pitch.value + w if r1 > r0 else 0
        buf = np.ctypeslib.as_array(C.cast(p, C.POINTER(C.c_uint16)), shape=(max(n, 1),))
        return np.lib.stride_tricks.as_strided(buf, shape=(r1 - r0, w),
                                               strides=(pitch.value * 2, 2))

    def commit_chunk(self, inst: int, wfs: int, frame: int, chunk: int):
        _ok(lib().rtc_commit_chunk(self._h, inst, wfs, frame, chunk), "rtc_commit_chunk")

    def commit_status(self, inst: int, wfs: int, frame: int, chunk: int) -> int:
        return lib().rtc_commit_chunk(self._h, inst, wfs, frame, chunk)

    def wait_commands(self, inst: int, frame: int, timeout_s: float = 5.0):
        n = self.infos[inst]["n_act"]
        out = np.empty(n, np.float32)
        fi = FrameInfoC()
        _ok(lib().rtc_wait_commands(self._h, inst, frame, _ptr(out), int(timeout_s * 1e9),
                                    C.byref(fi)), "rtc_wait_commands")
        return out, {k: getattr(fi, k) for k, _ in FrameInfoC._fields_}

    def wait_status(self, inst: int, frame: int, timeout_s: float = 0.0) -> int:
        n = self.infos[inst]["n_act"]
        out = np.empty(n, np.float32)
        return lib().rtc_wait_commands(self._h, inst, frame, _ptr(out), int(timeout_s * 1e9),
                                       None)

    # -- batch over device-resident frames
    def process_frames(self, inst: int, frames, n_frames: int, cmds=None, slopes=None,
                       counts=None, stream=None, noalloc: bool = False):
        """frames: one uint16 CUDA tensor (n, H, W) per sensor.  noalloc: the
        allocation-free entry point (rtc_process_frames_noalloc)."""
        nw = len(frames)
        ptrs = (C.c_void_p * nw)(*[f.data_ptr() for f in frames])
        strides = (C.c_int64 * nw)(*[f.shape[-1] * f.shape[-2] for f in frames])
        for f in frames:
            if f.dtype != torch.uint16 or not f.is_cuda or not f.is_contiguous():
                raise ValueError("frames must be contiguous uint16 device tensors")
            if f.shape[0] < n_frames:
                raise ValueError("not enough frames")
        fn = lib().rtc_process_frames_noalloc if noalloc else lib().rtc_process_frames
        _ok(fn(self._h, inst, ptrs, strides, n_frames, _ptr(cmds), _ptr(slopes), _ptr(counts),
               _stream_ptr(stream)),
            "rtc_process_frames_noalloc" if noalloc else "rtc_process_frames")

    def pace(self, streams, n_frames: int, warmup: int = 0, period_s: float = 2e-3,
             readout_s: float = 1.5e-3, first_frame: int = 0, zero_copy: bool = False,
             switch=None, pin: bool = True, timeout_s: float = 5.0, cmds: bool = False):
        """Paced serving run in the library's own threads (rtc_pacer_run).
        streams: [(instance, [bank per sensor: uint16 numpy (B, H, W)])];
        switch: (stream index, run index, gain, leak) or None.  Returns a
        structured numpy array (n_streams, n_frames - warmup) with fields
        frame, host_us, dev_us (negative: published before the last chunk),
        complete_us (from the last chunk that completes a column block), late_us,
        start_late_us.  cmds=True: also every recorded frame's commands, one
        (n_frames - warmup, n_act) float32 array per stream (returned second)."""
        keep = []
        n_rec = n_frames - warmup
        cmd_out = []
        cs = (PacerStreamC * len(streams))()
        for k, (inst, banks) in enumerate(streams):
            arr = [np.ascontiguousarray(b, dtype=np.uint16) for b in banks]
            keep.append(arr)
            ptrs = (C.c_void_p * len(arr))(*[a.ctypes.data for a in arr])
            keep.append(ptrs)
            cs[k].inst = inst
            cs[k].n_bank = min(a.shape[0] for a in arr)
            cs[k].banks = ptrs
            if cmds:
                buf = np.zeros((n_rec, self.infos[inst]["n_act"]), np.float32)
                cmd_out.append(buf)
                cs[k].cmds = buf.ctypes.data
        d = PacerDescC(period_s=period_s, readout_s=readout_s, n_frames=n_frames, warmup=warmup,
                       first_frame=first_frame, zero_copy=int(zero_copy),
                       switch_stream=-1 if switch is None else switch[0],
                       switch_frame=-1 if switch is None else switch[1],
                       switch_gain=0.0 if switch is None else switch[2],
                       switch_leak=0.0 if switch is None else switch[3],
                       pin=int(pin), timeout_s=timeout_s)
        out = (PacerSampleC * (len(streams) * n_rec))()
        failed = C.c_int32(-1)
        st = lib().rtc_pacer_run(self._h, C.byref(d), len(streams), cs, out, C.byref(failed))
        if st != RTC_OK:
            raise RtcError(st, f"rtc_pacer_run (frame index {failed.value})")
        dt = np.dtype([("frame", np.uint64), ("host_us", np.float64), ("dev_us", np.float64),
                       ("complete_us", np.float64), ("late_us", np.float64),
                       ("start_late_us", np.float64), ("dev_ticks_start", np.uint64),
                       ("dev_ticks_cmd", np.uint64)])
        samples = np.frombuffer(bytes(out), dtype=dt).reshape(len(streams), n_rec).copy()
        return (samples, cmd_out) if cmds else samples

    def run_mvm(self, inst: int, n_iter: int, stream=None):
        _ok(lib().rtc_run_mvm(self._h, inst, n_iter, _stream_ptr(stream)), "rtc_run_mvm")

    def mvm_timing(self, inst: int, capacity: int, every: int = 1):
        """Time the MVM launch of every `every`-th later per-launch frame, up to
        `capacity` launches, with HIP events on its stream (0 turns it off)."""
        _ok(lib().rtc_mvm_timing(self._h, inst, capacity, every), "rtc_mvm_timing")

    def mvm_timing_read(self, inst: int = 0):
        """(number of timed MVM launches, their total duration in seconds); clears."""
        n, ms = C.c_int32(0), C.c_double(0.0)
        _ok(lib().rtc_mvm_timing_read(self._h, inst, C.byref(n), C.byref(ms)),
            "rtc_mvm_timing_read")
        return n.value, ms.value / 1e3

    def trace_enable(self, n_frames: int):
        """Record the frame loop's per-wavefront timeline for the first n_frames
        frames of each later launch (0 turns it off)."""
        _ok(lib().rtc_trace_enable(self._h, n_frames), "rtc_trace_enable")

    def trace_read(self) -> np.ndarray:
        """The last launch's record as (frames, waves, len(TRACE_EVENTS)) uint64."""
        nw, nf = C.c_int32(0), C.c_int32(0)
        _ok(lib().rtc_trace_read(self._h, None, 0, C.byref(nw), C.byref(nf)), "rtc_trace_read")
        out = np.zeros((nf.value, nw.value, len(TRACE_EVENTS)), np.uint64)
        if out.size:
            _ok(lib().rtc_trace_read(self._h, _ptr(out), out.size, None, None), "rtc_trace_read")
        return out

    def read_slopes(self, inst: int = 0):
        info = self.infos[inst]
        s = np.empty(info["n_slopes"], np.float32)
        c = np.empty(info["n_units"], np.int32)
        m = np.empty(info["mask_words"], np.uint64)
        _ok(lib().rtc_read_slopes(self._h, inst, _ptr(s), _ptr(c), _ptr(m)), "rtc_read_slopes")
        return s, c, m

    def read_matrix(self, inst: int = 0):
        info = self.infos[inst]
        dtype = self.specs[inst][1]
        npd = {"f32": np.float32, "bf16": np.uint16, "fp8": np.uint8}[dtype]
        codes = np.empty((info["n_act"], info["n_slopes"]), npd)
        scales = np.empty(info["n_act"], np.float32)
        _ok(lib().rtc_read_matrix(self._h, inst, _ptr(codes), _ptr(scales)), "rtc_read_matrix")
        return codes, scales
