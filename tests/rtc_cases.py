"""Shared helpers of the GPU parity tests: build inputs, run the library, compare.

Inputs come from ``synth`` only; expected values from ``oracle`` only.
"""
from __future__ import annotations

import sys

import numpy as np

import oracle
import synth

TOL = {"f32": 1e-5, "bf16": 1e-2, "fp8": 3e-2}   # per-frame relative L2 of the commands
DEQ_TOL = 1e-5                                    # against the dequantised-matrix oracle
SLOPE_TOL_SH = 1e-4                               # px, FP32 centre of gravity
SLOPE_TOL_PYR = 1e-5                              # normalised units


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


class Case:
    """Frames, calibration and matrices of one instance of a workload."""

    def __init__(self, wl_name: str, inst_index: int = 0, n_frames: int = 8,
                 polc_m: str = "direct"):
        self.wl = synth.get_workload(wl_name)
        self.inst = self.wl.instances[inst_index]
        self.n = n_frames
        self.frames, self.cals = [], []
        for w in range(len(self.inst.wfs)):
            fr, cal = synth.sensor_inputs(self.wl, inst_index, w, n=n_frames)
            self.frames.append(fr)
            self.cals.append(cal)
        self.R = synth.control_matrix(self.wl, inst_index)
        self.D = None
        self.M = None
        if self.inst.polc:
            if polc_m == "direct":
                # a stand-in for R.D with the same statistics, given directly as M
                na = self.inst.n_act
                self.M = synth.gaussian_matrix(na, na, 0.5 / np.sqrt(na),
                                               synth.seed_for(self.wl.index, inst_index, 99, 5),
                                               np.float32)
            else:
                self.D = synth.interaction_matrix(self.wl, inst_index)

    def oracle_M(self):
        """The oracle's POLC matrix (the FP64 product R.D is formed once)."""
        if self.M is not None:
            return self.M.astype(np.float64)
        if self.D is not None:
            if getattr(self, "_M_rd", None) is None:
                self._M_rd = oracle.polc_matrix(self.R, self.D)
            return self._M_rd
        return None

    def load(self, eng, idx: int = 0):
        eng.load_matrices(idx, self.R, D=self.D, M=self.M)
        for w, cal in enumerate(self.cals):
            eng.load_calibration(idx, w, cal.dark, cal.flat, cal.bg, cal.thr, cal.ref)

    def run_oracle(self, dtype: str = "f32", dequantized: bool = False, n: int | None = None,
                   keep_masks: bool = False):
        return oracle.run(self.inst, self.frames, self.cals, self.R, self.n if n is None else n,
                          cm_dtype=dtype, M=self.oracle_M(), dequantized=dequantized,
                          keep_masks=keep_masks)


def mid_case(polc: bool, n_frames: int = 30, polc_m: str = "from_D", index: int = 92) -> Case:
    """A mid-size instance: one 24x24 Shack-Hartmann sensor (10 px, 240x240
    frame in 6 chunks), 700 actuators."""
    wfs = synth.ShWfs(nsub=24, px=10, obs=0.28, frame_h=240, frame_w=240, n_chunks=6)
    inst = synth.Instance(f"mid{index}", (wfs,), 700, ("f32",), polc=polc, gain=0.4, leak=0.01)
    wl = synth.Workload(index, f"mid{index}", (inst,), n_frames=n_frames, bank=n_frames)
    synth.workloads.WORKLOADS[wl.name] = wl
    try:
        return Case(wl.name, n_frames=n_frames, polc_m=polc_m)
    finally:
        del synth.workloads.WORKLOADS[wl.name]


def run_batch(eng, idx: int, case: Case, n: int | None = None, first: int = 0):
    """Device-resident batch through rtc_process_frames of bank frames
    [first, first + n); returns numpy arrays."""
    import torch
    n = case.n - first if n is None else n
    info = eng.infos[idx]
    dfr = [torch.from_numpy(np.ascontiguousarray(f[first:first + n])).cuda()
           for f in case.frames]
    cmds = torch.zeros((n, info["n_act"]), dtype=torch.float32, device="cuda")
    slopes = torch.zeros((n, info["n_slopes"]), dtype=torch.float32, device="cuda")
    counts = torch.zeros((n, info["n_units"]), dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream()
    eng.process_frames(idx, dfr, n, cmds=cmds, slopes=slopes, counts=counts, stream=st)
    torch.cuda.synchronize()
    return (cmds.cpu().numpy().astype(np.float64), slopes.cpu().numpy().astype(np.float64),
            counts.cpu().numpy())


def run_stream(eng, idx: int, case: Case, n: int | None = None, first_frame: int = 0):
    """Serving path: every chunk of every sensor submitted from host memory."""
    n = case.n if n is None else n
    out = []
    infos = []
    for f in range(n):
        frame_no = first_frame + f
        for w, bank in enumerate(case.frames):
            img = bank[frame_no % bank.shape[0]]
            for c in range(case.inst.wfs[w].n_chunks):
                r0, r1 = eng.chunk_rows(idx, w, c)
                eng.submit_chunk(idx, w, frame_no, c, img[r0:r1])
        cmds, info = eng.wait_commands(idx, frame_no, timeout_s=10.0)
        out.append(cmds.astype(np.float64))
        infos.append(info)
    return np.stack(out), infos


def rel_l2(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    return np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)


def mask_bits(ref_masks, inst) -> np.ndarray:
    """Oracle masks of one frame packed like rtc_read_slopes: per unit, raster
    bits in 64-bit words (SH), one word with bits I1..I4 (pyramid)."""
    words = []
    for w, m in zip(inst.wfs, ref_masks):
        if w.kind == "sh":
            npx = w.px * w.px
            flat = m.reshape(m.shape[0], npx)
            nw = (npx + 63) // 64
            pad = np.zeros((flat.shape[0], nw * 64), bool)
            pad[:, :npx] = flat
            bits = pad.reshape(-1, nw, 64).astype(np.uint64) << np.arange(64, dtype=np.uint64)
            words.append(np.bitwise_or.reduce(bits, axis=2).reshape(-1))
        else:
            bits = m.astype(np.uint64) << np.arange(4, dtype=np.uint64)
            words.append(np.bitwise_or.reduce(bits, axis=1))
    return np.concatenate(words)
