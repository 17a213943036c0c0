// Host side of the persistent frame loop (RTC_MODE_PERSISTENT).
//
// Serving: the host copies each chunk into a pinned ring slot and rings the
// sensor's doorbell; the resident kernel centroids, multiplies and integrates
// on its own and publishes the commands into a pinned mailbox.  Batch: the
// same kernel runs a finite run of device-resident frames.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "rtc_engine.h"
#include "rtc_seq.h"

using namespace rtc;

namespace {

constexpr uint64_t kIdleTicks = 10ull * 100000000ull;    // 10 s of the 100 MHz device clock
constexpr uint64_t kDepTicks = 2ull * 100000000ull;      // 2 s for any internal dependency
constexpr int64_t kStopTimeoutNs = 5000000000LL;
constexpr int64_t kStampWaitNs = 2000000LL;     // last-chunk stamp after an early publication

uint64_t db_word(uint64_t q, uint64_t chunks) { return (q << kDbShift) | chunks; }

volatile uint64_t *vol(uint64_t *p) { return reinterpret_cast<volatile uint64_t *>(p); }

void store_release(uint64_t *p, uint64_t v) {
    std::atomic_thread_fence(std::memory_order_release);
    *vol(p) = v;
}

uint64_t load_acquire(uint64_t *p) {
    const uint64_t v = *vol(p);
    std::atomic_thread_fence(std::memory_order_acquire);
    return v;
}

// Fill the device-side descriptor of an instance (fields common to both uses).
PersistInst describe(rtc_engine *e, Instance *I) {
    PersistInstState &P = I->ps;
    PersistInst d{};
    d.sh = I->d_sh;
    d.py = I->d_py;
    d.n_sh = I->n_sh;
    d.n_pyr = I->n_pyr;
    d.kbs = I->d_kb;
    d.kbw = P.kbw;
    d.segs = I->d_seg;
    d.seg_ends = I->d_seg_ends;
    d.tail_ends = I->d_tail_ends;
    d.n_head = I->n_head_seg;
    d.steps = nullptr;
    d.n_kb = (int)I->kb.size();
    d.n_cen_all = P.n_cen_all;
    d.n_ing_all = P.n_ing_all;
    d.ing_cnt = P.ing_cnt;
    d.n_seg = (int)I->seg.size();
    d.n_steps = (int)I->steps.size();
    d.n_wfs = (int)I->wfs.size();
    d.wp = P.wp;
    d.sh_dark = I->d_sh_dark;
    d.sh_flat = I->d_sh_flat;
    d.sh_bg = I->d_sh_bg;
    d.sh_thr = I->d_sh_thr;
    d.py_dark = I->d_py_dark;
    d.py_flat = I->d_py_flat;
    d.py_bg = I->d_py_bg;
    d.py_thr = I->d_py_thr;
    d.ref = I->d_ref;
    for (int k = 0; k < 2; ++k) {
        d.cm[k] = I->d_cm_s[k];
        d.scale[k] = I->d.cm_dtype == RTC_CM_FP8 ? I->d_scale_s[k] : nullptr;
        d.M[k] = I->d_M_s[k];
    }
    d.dtype = I->d.cm_dtype;
    d.n_act = I->n_act;
    d.n_tiles = I->n_tiles;
    d.stream_nt = I->stream_nt ? 1 : 0;
    d.polc = I->d.polc;
    d.kbm = I->d_kbm;
    d.segm = I->d_segm;
    d.segm_ends = I->d_segm_ends;
    d.n_kbm = (int)I->kbm.size();
    d.n_segm = (int)I->segm.size();
    d.s_pad[0] = I->d_spad;
    d.y_part[0] = I->d_ypart;
    d.p_part[0] = I->d_ppart;
    for (int k = 1; k < kDepth; ++k) {
        d.s_pad[k] = P.spad_x[k - 1];
        d.y_part[k] = P.ypart_x[k - 1];
        d.p_part[k] = P.ppart_x[k - 1];
    }
    d.p = I->d_p;
    d.a = I->d_a;
    d.a_stride = I->a_len;
    d.cen_fan = P.cen_fan;
    d.tile_fan = P.tile_fan;
    d.pol_fan = P.pol_fan;
    d.tile_cnt = P.tile_cnt;
    d.head_cnt = P.head_cnt;
    d.pre = P.pre;
    d.join = P.join;
    d.pol_cnt = P.pol_cnt;
    d.p_done = P.p_done;
    d.tile_pub = P.tile_pub;
    d.pol_seg = P.pol_seg;
    d.db_mirror = P.db_mirror;
    d.drop_mirror = P.drop_mirror;
    d.ring_depth = e->ring_depth;
    d.doorbell = P.doorbell;
    d.drop_host = P.drop_host;
    d.params = P.params;
    d.param_mirror = P.param_mirror;
    if (P.tel_slots > 0) {
        d.tel_ring = P.tel_ring;
        d.tel_host = P.tel_host;
        d.tel_flags = P.tel_flags;
        d.tel_rec = P.tel_rec;
        d.tel_mask_off = P.tel_mask_off;
        d.tel_dshift = P.tel_dshift;
        d.tel_smask = P.tel_slots - 1;
    }
    d.mail = I->h_mail;
    d.cmd_seq = P.cmd_seq;
    d.tile_host = P.tile_host;
    d.pol_seq = P.pol_seq;
    d.tel = P.tel;
    d.n_slopes = I->n_slopes;
    d.n_units = I->n_units;
    return d;
}

// Device steps array lives in the kbw allocation's tail (see persist_alloc).
Step *steps_dev(Instance *I) {
    return reinterpret_cast<Step *>(I->ps.kbw + I->ps.kbw_h.size());
}

// Serving: descriptors of every instance through a synchronous copy (the
// loop is launched rarely).  Batch: one descriptor through a pinned staging
// slot and a copy ordered on the launch stream, so back-to-back batches on a
// stream never overwrite a descriptor a running kernel still reads.
rtc_status upload_and_launch(rtc_engine *e, const std::vector<Instance *> &insts,
                             std::vector<PersistInst> &descs, hipStream_t st, bool batch,
                             int n_blocks) {
    PersistEngine &pe = e->pe;
    // every launch counts from its first frame
    for (size_t i = 0; i < insts.size(); ++i) {
        const PersistInstState &P = insts[i]->ps;
        launch_seed_counters(st, P.ctr, P.n_ctr, (size_t)(P.join - P.ctr), insts[i]->n_tiles,
                             (int)(descs[i].q_begin % kDepth), insts[i]->d.polc);
    }
    PersistInst *dev = pe.d_inst;
    if (!batch) {
        HIP_TRY(hipMemcpy(pe.d_inst, descs.data(), descs.size() * sizeof(PersistInst),
                          hipMemcpyHostToDevice));
    } else {
        const int k = pe.batch_slot;
        pe.batch_slot ^= 1;
        HIP_TRY(hipEventSynchronize(pe.batch_copied[k]));   // slot k's last copy has run
        *pe.h_batch[k] = descs[0];
        HIP_TRY(hipMemcpyAsync(pe.d_batch[k], pe.h_batch[k], sizeof(PersistInst),
                               hipMemcpyHostToDevice, st));
        HIP_TRY(hipEventRecord(pe.batch_copied[k], st));
        dev = pe.d_batch[k];
    }
    *reinterpret_cast<volatile uint32_t *>(pe.stop_host) = 0;
    *reinterpret_cast<volatile uint32_t *>(pe.status) = 0;
    HIP_TRY(hipMemsetAsync(pe.stop_dev, 0, sizeof(uint32_t), st));
    PersistArgs A{};
    A.inst = dev;
    A.n_inst = (int)descs.size();
    A.stop_host = pe.stop_host;
    A.stop_dev = pe.stop_dev;
    A.status = pe.status;
    A.dep_watchdog = kDepTicks;
    A.idle_watchdog = kIdleTicks;
    A.n_waves = n_blocks * 4;
    if (pe.trace != nullptr) {
        pe.trace_waves = A.n_waves;
        A.trace = pe.trace;
        A.trace_frames = pe.trace_frames;
        HIP_TRY(hipMemsetAsync(pe.trace, 0,
                               (size_t)pe.trace_frames * A.n_waves * RTC_TRACE_EVENTS * 8, st));
    }
    launch_frame_loop(st, n_blocks, A, !batch);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
        std::fprintf(stderr, "rtc: frame loop launch failed: %s\n", hipGetErrorString(err));
        return fail(e, RTC_E_DEVICE);
    }
    return RTC_OK;
}

// Before a run starting at sequence q0 the state a_{q0-1} must sit in buffer
// (q0 - 1) & 1; between runs it lives in buffer 0.
rtc_status stage_state_in(Instance *I, uint64_t q0, hipStream_t st) {
    if (((q0 - 1) & 1) == 1)
        HIP_TRY(hipMemcpyAsync(I->d_a + I->a_len, I->d_a, (size_t)I->a_len * 4,
                               hipMemcpyDeviceToDevice, st));
    return RTC_OK;
}
rtc_status stage_state_out(Instance *I, uint64_t q_last, hipStream_t st) {
    if ((q_last & 1) == 1)
        HIP_TRY(hipMemcpyAsync(I->d_a, I->d_a + I->a_len, (size_t)I->a_len * 4,
                               hipMemcpyDeviceToDevice, st));
    return RTC_OK;
}

rtc_status launch_serving(rtc_engine *e) {
    PersistEngine &pe = e->pe;
    HIP_TRY(hipDeviceSynchronize());      // no batch work may still run on the state
    const int W = pe.n_blocks * 4;
    const int n = (int)e->inst.size();
    // workers in proportion to the bytes each instance streams per frame
    std::vector<double> wt(n);
    double tot = 0;
    for (int i = 0; i < n; ++i) {
        wt[i] = (double)e->inst[i]->cm_bytes + (double)e->inst[i]->m_bytes;
        tot += wt[i];
    }
    if (W < n * 66) return RTC_E_INVAL;
    std::vector<PersistInst> descs;
    int w = 0;
    for (int i = 0; i < n; ++i) {
        Instance *I = e->inst[i];
        if (!I->loaded) return RTC_E_STATE;
        int share = i == n - 1 ? W - w : (int)std::floor(wt[i] / tot * (W - n * 66)) + 66;
        PersistInst d = describe(e, I);
        d.steps = steps_dev(I);
        d.serving = 1;
        for (size_t s = 0; s < I->wfs.size(); ++s) {
            const WfsState &S = I->wfs[s];
            d.src[s] = S.d_ring;
            d.src_stride[s] = (int64_t)S.slot16;
            d.src_pitch[s] = S.pitch16;
            d.ring_host[s] = S.h_stage;
            d.ring_bytes[s] = (uint64_t)S.ring_elems * 2;
        }
        d.q_begin = load_acquire(I->ps.cmd_seq);   // first frame not yet published
        d.q_end = ~0ull;
        d.w0 = w;
        d.w1 = w + share;
        I->ps.w0 = d.w0;
        I->ps.w1 = d.w1;
        w += share;
        TRY(stage_state_in(I, d.q_begin, pe.stream));
        descs.push_back(d);
    }
    TRY(upload_and_launch(e, e->inst, descs, pe.stream, false, pe.n_blocks));
    pe.running = true;
    pe.serving = true;
    return RTC_OK;
}

bool stream_done(hipStream_t st) { return hipStreamQuery(st) == hipSuccess; }

}  // namespace

// Device buffers of the frame loop, for every instance of the engine.
rtc_status persist_alloc(rtc_engine *e) {
    PersistEngine &pe = e->pe;
    HIP_TRY(hipStreamCreateWithFlags(&pe.stream, hipStreamNonBlocking));
    TRY(host_pinned(e, &pe.stop_host, 1));
    TRY(host_pinned(e, &pe.status, 1));
    TRY(dev_alloc(e, &pe.stop_dev, 1));
    TRY(dev_alloc(e, &pe.d_inst, e->inst.size()));
    for (int k = 0; k < 2; ++k) {
        TRY(dev_alloc(e, &pe.d_batch[k], 1));
        TRY(host_pinned(e, &pe.h_batch[k], 1));
        HIP_TRY(hipEventCreateWithFlags(&pe.batch_copied[k], hipEventDisableTiming));
    }
    int dev_cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, e->device));
    // the grid must be entirely resident: a serving loop runs indefinitely and
    // leaves room on every CU for whatever else shares the device; a batch
    // launch is finite and takes the whole occupancy
    const int occ_serve = frame_loop_max_blocks_per_cu(true);
    const int occ_batch = frame_loop_max_blocks_per_cu(false);
    if (occ_serve < 1 || occ_batch < 1) return RTC_E_DEVICE;
    pe.n_blocks = dev_cus * std::min(2, occ_serve);
    pe.n_blocks_batch = dev_cus * occ_batch;
    for (Instance *I : e->inst) {
        PersistInstState &P = I->ps;
        const size_t nkb = I->kb.size(), nt = (size_t)I->n_tiles;
        for (int k = 0; k < kDepth - 1; ++k) {
            TRY(dev_alloc(e, &P.spad_x[k], I->spad_len));
            TRY(dev_alloc(e, &P.ypart_x[k], I->seg.size() * (size_t)I->n_act));
            TRY(dev_alloc(e, &P.ppart_x[k],
                          std::max<size_t>(I->segm.size(), 1) * (size_t)I->n_act));
        }
        // counters, each in a slot of its own; arrival counters kDepth times:
        // fan-in barriers cen [D][nkb], tile [D], pol [D]; tile_cnt, join and
        // pol_cnt [D][nt]; p_done and tile_pub [nt] once; ing_cnt [D][n_steps]
        // then its done flags [D][n_steps]; pol_seg [D][n_segm]; head_cnt [D][nt]
        const size_t fan = kFanSlots, D = kDepth, nst = I->steps.size(), nsm = I->segm.size();
        const size_t n_slots =
            D * nkb * fan + 2 * D * fan + 4 * D * nt + 2 * nt + 2 * D * nst + D * nsm;
        P.n_ctr = n_slots * kCtrSlot;
        TRY(dev_alloc(e, &P.ctr, P.n_ctr));
        P.cen_fan = P.ctr;
        P.tile_fan = P.cen_fan + D * nkb * fan * kCtrSlot;
        P.pol_fan = P.tile_fan + D * fan * kCtrSlot;
        P.tile_cnt = P.pol_fan + D * fan * kCtrSlot;
        P.join = P.tile_cnt + D * nt * kCtrSlot;
        P.pol_cnt = P.join + D * nt * kCtrSlot;
        P.p_done = P.pol_cnt + D * nt * kCtrSlot;
        P.tile_pub = P.p_done + nt * kCtrSlot;
        P.ing_cnt = P.tile_pub + nt * kCtrSlot;
        P.pol_seg = P.ing_cnt + 2 * D * nst * kCtrSlot;
        P.head_cnt = P.pol_seg + D * nsm * kCtrSlot;
        TRY(dev_alloc(e, &P.pre, (size_t)kDepth * I->n_act));
        // serving ingest: each readout step's rows as 16-byte units of a ring
        // slot, in pieces, numbered in readout order; the buffer accesses take
        // 32-bit byte offsets
        for (const WfsState &S : I->wfs)
            if (S.ring_elems * 2 >= (size_t)1 << 31) return RTC_E_INVAL;
        int ing = 0;
        for (Step &st : I->steps) {
            const WfsState &S = I->wfs[st.wfs];
            st.u0 = S.row0[st.chunk] * S.pitch16 / 8;
            st.n16 = (S.row0[st.chunk + 1] - S.row0[st.chunk]) * S.pitch16 / 8;
            st.ing0 = ing;
            st.ing_n = (st.n16 + kIngestUnits - 1) / kIngestUnits;
            ing += st.ing_n;
        }
        P.n_ing_all = ing;
        TRY(dev_alloc(e, &P.db_mirror, I->wfs.size()));
        TRY(dev_alloc(e, &P.drop_mirror, e->ring_depth));
        TRY(dev_alloc(e, &P.param_mirror, 1));
        TRY(dev_alloc(e, &P.wp, RTC_MAX_WFS));
        HIP_TRY(hipMemcpy(P.wp, I->params.w, sizeof(I->params.w), hipMemcpyHostToDevice));
        TRY(host_pinned(e, &P.doorbell, I->wfs.size()));
        TRY(host_pinned(e, &P.drop_host, e->ring_depth));
        TRY(host_pinned(e, &P.params, 1));
        TRY(host_pinned(e, &P.cmd_seq, 1));
        TRY(host_pinned(e, &P.tile_host, (size_t)I->n_tiles));
        TRY(host_pinned(e, &P.pol_seq, 1));
        TRY(host_pinned(e, &P.tel, e->ring_depth));
        P.slot_frame.assign(e->ring_depth, ~0ull);
        P.slot_t_last.assign(e->ring_depth, 0);
        P.slot_tlc0.assign(e->ring_depth, 0);
        P.slot_tpub0.assign(e->ring_depth, 0);
        P.slot_dropped.assign(e->ring_depth, 0);
        // work of each column block; task 0 of each list goes to the worker
        // after the previous list's last task so that the load spreads evenly
        int cen_base = 0, mvm_base = 0;
        for (size_t b = 0; b < nkb; ++b) {
            const KBlock &K = I->kb[b];
            const WfsState &S = I->wfs[K.wfs];
            KbWork W{};
            W.kind = S.d.kind;
            W.wfs = K.wfs;
            const int ub = K.k0 / 2 - S.u0, ue = (K.k0 + K.k) / 2 - S.u0;
            W.cu0 = S.kind0 + ub;
            W.cu1 = S.kind0 + ue;
            W.n_cen = S.d.kind == RTC_WFS_SH ? ue - ub : (ue - ub + kWave - 1) / kWave;
            W.cen_base = cen_base;
            W.seg0 = I->kb_seg0[b];
            W.nseg = I->kb_nseg[b];
            W.mvm_base = mvm_base;
            cen_base += W.n_cen;
            mvm_base += W.nseg * I->n_tiles;
            P.kbw_h.push_back(W);
        }
        P.n_cen_all = cen_base;
        // one allocation: KbWork table followed by the readout steps
        const size_t bytes = P.kbw_h.size() * sizeof(KbWork) + I->steps.size() * sizeof(Step);
        uint8_t *buf = nullptr;
        TRY(dev_alloc(e, &buf, bytes));
        P.kbw = reinterpret_cast<KbWork *>(buf);
        HIP_TRY(hipMemcpy(P.kbw, P.kbw_h.data(), P.kbw_h.size() * sizeof(KbWork),
                          hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(steps_dev(I), I->steps.data(), I->steps.size() * sizeof(Step),
                          hipMemcpyHostToDevice));
        for (const Segment &sg : I->seg)
            if (sg.nv > kMaxSegVectors) return RTC_E_INVAL;
        for (const Segment &sg : I->segm)
            if (sg.nv > kMaxSegVectors) return RTC_E_INVAL;
        TRY(persist_params(e, I));
    }
    return RTC_OK;
}

// Stop the frame loop (if running) and wait for every wavefront to exit.
rtc_status persist_stop(rtc_engine *e) {
    PersistEngine &pe = e->pe;
    if (!pe.running) return RTC_OK;
    *reinterpret_cast<volatile uint32_t *>(pe.stop_host) = 1;
    const int64_t t0 = now_ns();
    while (!stream_done(pe.stream)) {
        if (now_ns() - t0 > kStopTimeoutNs) {
            std::fprintf(stderr, "rtc: frame loop did not stop\n");
            return fail(e, RTC_E_DEVICE);
        }
        std::this_thread::yield();
    }
    if (pe.serving) {
        for (Instance *I : e->inst) {
            const uint64_t pub = load_acquire(I->ps.cmd_seq);
            if (pub > 0) TRY(stage_state_out(I, pub - 1, pe.stream));
        }
        HIP_TRY(hipStreamSynchronize(pe.stream));
    }
    pe.running = false;
    pe.serving = false;
    if (*reinterpret_cast<volatile uint32_t *>(pe.status) != PERSIST_OK) {
        std::fprintf(stderr, "rtc: frame loop ended on a watchdog\n");
        return fail(e, RTC_E_DEVICE);
    }
    return RTC_OK;
}

// Stop the serving loop once every started frame is published and its POLC
// term is formed, so that counters and state stay consistent for a restart.
rtc_status persist_quiesce(rtc_engine *e) {
    PersistEngine &pe = e->pe;
    if (!pe.running) return RTC_OK;
    if (pe.serving) {
        const int64_t t0 = now_ns();
        for (Instance *I : e->inst) {
            if (I->cur_started) return RTC_E_STATE;   // a frame is half delivered
            PersistInstState &P = I->ps;
            while (load_acquire(P.cmd_seq) < P.seq ||
                   (I->d.polc && load_acquire(P.pol_seq) < P.seq)) {
                if (stream_done(pe.stream) || now_ns() - t0 > kStopTimeoutNs)
                    return fail(e, RTC_E_DEVICE);
                std::this_thread::yield();
            }
        }
    }
    return persist_stop(e);
}

rtc_status persist_trace(rtc_engine *e, int n_frames) {
    PersistEngine &pe = e->pe;
    if (pe.trace != nullptr) {
        HIP_TRY(hipFree(pe.trace));
        pe.trace = nullptr;
    }
    pe.trace_frames = 0;
    pe.trace_waves = 0;
    if (n_frames == 0) return RTC_OK;
    const size_t bytes =
        (size_t)n_frames * std::max(pe.n_blocks, pe.n_blocks_batch) * 4 * RTC_TRACE_EVENTS * 8;
    if (hipMalloc(&pe.trace, bytes) != hipSuccess) {
        pe.trace = nullptr;
        return RTC_E_NOMEM;
    }
    HIP_TRY(hipMemset(pe.trace, 0, bytes));
    pe.trace_frames = n_frames;
    return RTC_OK;
}

void persist_free(rtc_engine *e) {
    PersistEngine &pe = e->pe;
    for (Instance *I : e->inst) persist_telemetry_free(I);
    if (pe.trace) (void)hipFree(pe.trace);
    for (int k = 0; k < 2; ++k)
        if (pe.batch_copied[k]) (void)hipEventDestroy(pe.batch_copied[k]);
    if (pe.stream) (void)hipStreamDestroy(pe.stream);
}

// Zero every frame-loop sequence (the loop must be stopped); each launch
// resets its own counters.
void persist_reset(Instance *I) {
    PersistInstState &P = I->ps;
    (void)hipMemset(P.db_mirror, 0, I->wfs.size() * sizeof(uint64_t));
    (void)hipMemset(P.drop_mirror, 0, P.slot_frame.size() * sizeof(uint64_t));
    for (size_t w = 0; w < I->wfs.size(); ++w) *vol(P.doorbell + w) = 0;
    for (size_t k = 0; k < P.slot_frame.size(); ++k) *vol(P.drop_host + k) = 0;
    *vol(P.cmd_seq) = 0;
    *vol(P.pol_seq) = 0;
    for (int t = 0; t < I->n_tiles; ++t) *vol(P.tile_host + t) = 0;
    P.seq = 0;
    P.q_cur = 0;
    std::fill(P.slot_frame.begin(), P.slot_frame.end(), ~0ull);
    std::fill(P.slot_dropped.begin(), P.slot_dropped.end(), 0);
    (void)persist_params(nullptr, I);
    // a pending swap is cancelled (its matrices stay staged)
    if (I->m_pending) {
        I->m_pending = false;
        I->m_staged = true;
    }
    persist_mswap(I, ~0ull >> 2, 1 - I->m_active);   // every frame on the active slot
    P.mq_last = 0;
    // frames count from 0 again: no part flag may still name one of them
    P.tel_next = 0;
    if (P.tel_slots > 0) {
        std::memset(P.tel_flags, 0, (size_t)P.tel_slots * kTelMaxTasks * 8);
        std::fill(P.tel_frame.begin(), P.tel_frame.end(), ~0ull);
        std::fill(P.tel_dropped.begin(), P.tel_dropped.end(), 0);
    }
}

void persist_telemetry_free(Instance *I) {
    PersistInstState &P = I->ps;
    if (P.tel_ring) (void)hipFree(P.tel_ring);
    if (P.tel_host) (void)hipHostFree(P.tel_host);
    if (P.tel_flags) (void)hipHostFree(P.tel_flags);
    P.tel_ring = nullptr;
    P.tel_host = nullptr;
    P.tel_flags = nullptr;
    P.tel_slots = 0;
}

int tel_tasks(const Instance *I) {
    return (I->ps.tel_rec / 4 + kTelUnits - 1) / kTelUnits;
}

// Telemetry ring of 2^k slots recording every 2^j-th frame (n_slots 0: off).
// Records are formed in device memory (the slope and command stores stay at
// HBM speed) and copied to the pinned host ring with 16-byte stores, off the
// frame's latency path.
rtc_status persist_telemetry(rtc_engine *e, Instance *I, int decimation, int n_slots) {
    PersistInstState &P = I->ps;
    HIP_TRY(hipDeviceSynchronize());
    persist_telemetry_free(I);
    if (n_slots == 0) return RTC_OK;
    // slopes, counts, commands, then the masks on a 16-byte boundary
    P.tel_mask_off = (I->n_slopes + I->n_units + I->n_act + 3) & ~3;
    P.tel_rec = (P.tel_mask_off + 2 * I->mask_words + 3) & ~3;
    if (tel_tasks(I) > kTelMaxTasks) return RTC_E_INVAL;
    const size_t ring_bytes = (size_t)P.tel_rec * 4 * n_slots;
    const size_t flag_bytes = (size_t)n_slots * kTelMaxTasks * 8;
    if (hipMalloc(&P.tel_ring, ring_bytes) != hipSuccess) {
        P.tel_ring = nullptr;
        return RTC_E_NOMEM;
    }
    if (hipHostMalloc(&P.tel_host, ring_bytes, hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc(&P.tel_flags, flag_bytes, hipHostMallocCoherent) != hipSuccess) {
        persist_telemetry_free(I);
        return RTC_E_NOMEM;
    }
    HIP_TRY(hipMemset(P.tel_ring, 0, ring_bytes));
    std::memset(P.tel_host, 0, ring_bytes);
    std::memset(P.tel_flags, 0, flag_bytes);
    int sh = 0;
    while ((1 << sh) < decimation) ++sh;
    P.tel_dshift = sh;
    P.tel_slots = n_slots;
    P.tel_frame.assign((size_t)n_slots, ~0ull);
    P.tel_dropped.assign((size_t)n_slots, 0);
    // the first record read is the next frame to start
    P.tel_next = ((P.seq + (uint64_t)decimation - 1) >> sh) << sh;
    (void)e;
    return RTC_OK;
}

// The next telemetry record, in frame order: waits for its frame to be
// published; records overwritten before they were read are skipped (counted).
rtc_status persist_telemetry_next(rtc_engine *e, Instance *I, float *slopes, int32_t *counts,
                                  float *cmds, uint64_t *masks, int64_t timeout_ns,
                                  rtc_telemetry_info *info) {
    PersistInstState &P = I->ps;
    const int64_t t0 = now_ns();
    uint32_t lost = 0;
    for (;;) {
        uint64_t q;
        size_t k;
        uint64_t span;
        {
            std::lock_guard<std::mutex> lk(I->mu);
            if (P.tel_slots == 0) return RTC_E_STATE;
            const uint64_t d = 1ull << P.tel_dshift;
            span = d * (uint64_t)P.tel_slots;
            // a record is overwritten once the frame span later has started
            if (P.seq > P.tel_next + span) {
                const uint64_t first = ((P.seq - span + d - 1) >> P.tel_dshift) << P.tel_dshift;
                lost += (uint32_t)((first - P.tel_next) >> P.tel_dshift);
                P.tel_next = first;
            }
            q = P.tel_next;
            k = (size_t)((q >> P.tel_dshift) & (uint64_t)(P.tel_slots - 1));
        }
        // every part of the record copied for frame q (a part already holding
        // a later frame's copy: the record was overwritten, skip ahead)
        uint64_t *flags = P.tel_flags + k * kTelMaxTasks;
        const int nt = tel_tasks(I);
        bool overwritten = false;
        for (int j = 0; j < nt && !overwritten;) {
            const uint64_t fv = load_acquire(flags + j);
            if (fv == q + 1) {
                ++j;
                continue;
            }
            overwritten = fv > q + 1;
            if (now_ns() - t0 > timeout_ns) return RTC_E_TIMEOUT;
            if (e->pe.running && stream_done(e->pe.stream) &&
                *reinterpret_cast<volatile uint32_t *>(e->pe.status) != PERSIST_OK)
                return fail(e, RTC_E_DEVICE);
            std::this_thread::yield();
        }
        if (overwritten) continue;
        const float *rec = P.tel_host + k * (size_t)P.tel_rec;
        if (slopes) std::memcpy(slopes, rec, (size_t)I->n_slopes * 4);
        if (counts) std::memcpy(counts, rec + I->n_slopes, (size_t)I->n_units * 4);
        if (cmds) std::memcpy(cmds, rec + I->n_slopes + I->n_units, (size_t)I->n_act * 4);
        if (masks) std::memcpy(masks, rec + P.tel_mask_off, (size_t)I->mask_words * 8);
        std::lock_guard<std::mutex> lk(I->mu);
        if (P.seq > q + span) continue;     // overwritten while copied: skip ahead
        if (info) {
            info->frame = P.tel_frame[k];
            info->dropped = P.tel_dropped[k];
            info->lost = lost;
        }
        P.tel_next = q + (1ull << P.tel_dshift);
        return RTC_OK;
    }
}

// Matrix slot switch word: frames from sequence number q_switch on use `slot`,
// earlier ones the other slot.
void persist_mswap(Instance *I, uint64_t q_switch, int slot) {
    PersistInstState &P = I->ps;
    P.mword = (q_switch << 1) | (uint64_t)slot;
    if (q_switch < (~0ull >> 2)) P.mq_last = q_switch;
    store_release(&P.params->mword, P.mword);
}

// Waits until no frame streams the inactive matrix slot: every frame before
// the last swap published and, with POLC, its POLC product formed.
rtc_status persist_wait_matrix_free(rtc_engine *e, Instance *I) {
    PersistEngine &pe = e->pe;
    if (!(pe.running && pe.serving)) {
        HIP_TRY(hipDeviceSynchronize());
        return RTC_OK;
    }
    PersistInstState &P = I->ps;
    const int64_t t0 = now_ns();
    while (load_acquire(P.cmd_seq) < P.mq_last ||
           (I->d.polc && load_acquire(P.pol_seq) < P.mq_last)) {
        if (now_ns() - t0 > kStopTimeoutNs) return RTC_E_TIMEOUT;
        std::this_thread::yield();
    }
    return RTC_OK;
}

// Coefficients of both parameter slots into the pinned block, switching at
// the first frame that has not started.
rtc_status persist_params(rtc_engine *e, Instance *I) {
    (void)e;
    PersistInstState &P = I->ps;
    const int staged = 1 - I->active;
    ParamBlock pb{};
    for (int s = 0; s < 2; ++s) {
        const double gd = I->gain[s], ld = I->leak[s];
        pb.g[s] = (float)gd;
        pb.c1[s] = I->d.polc ? (float)(1.0 - ld - gd) : (float)(1.0 - ld);
    }
    const uint64_t q_switch = I->pending ? (I->cur_started ? P.q_cur + 1 : P.seq) : ~0ull >> 2;
    volatile ParamBlock *h = P.params;
    for (int s = 0; s < 2; ++s) {
        h->c1[s] = pb.c1[s];
        h->g[s] = pb.g[s];
    }
    P.param_word = (q_switch << 1) | (uint64_t)staged;
    store_release(&P.params->word, P.param_word);
    return RTC_OK;
}

namespace {

// Opens chunk `chunk` of sensor w of frame `frame`: starts the frame when it is
// a new one (delivering an incomplete predecessor as dropped) and launches the
// loop when it is not running.
rtc_status begin_chunk(rtc_engine *e, Instance *I, int w, uint64_t frame, int chunk) {
    PersistInstState &P = I->ps;
    PersistEngine &pe = e->pe;
    WfsState &S = I->wfs[w];
    if (pe.running && !pe.serving) return RTC_E_STATE;
    if (S.acquired >= 0) return RTC_E_INVAL;     // a lent chunk is not committed yet
    if (I->cur_frame != ~0ull && frame < I->cur_frame) return RTC_E_FRAME_DROPPED;
    if (frame < I->next_frame) return RTC_E_FRAME_DROPPED;
    if (I->cur_frame == ~0ull || frame > I->cur_frame) {
        const uint64_t pub = load_acquire(P.cmd_seq);
        const uint64_t q = P.seq;
        if (q - pub >= (uint64_t)e->ring_depth) return RTC_E_RING_FULL;
        if (I->cur_frame != ~0ull && I->cur_started) {
            // the frame in progress never completed: deliver it as dropped (the
            // loop skips its integrator update) so the loop can move on
            const uint64_t qd = P.q_cur;
            P.slot_dropped[qd % P.slot_dropped.size()] = 1;
            if (P.tel_slots > 0 && (qd & ((1ull << P.tel_dshift) - 1)) == 0)
                P.tel_dropped[(qd >> P.tel_dshift) & (uint64_t)(P.tel_slots - 1)] = 1;
            I->drops++;
            store_release(P.drop_host + qd % P.slot_dropped.size(), qd + 1);
            for (size_t s = 0; s < I->wfs.size(); ++s)
                if (I->wfs[s].next_chunk < I->wfs[s].d.n_chunks)
                    store_release(P.doorbell + s, db_word(qd, I->wfs[s].d.n_chunks));
        }
        if (I->pending && frame >= I->f_switch) settle_params(I, frame);
        settle_matrices(I, frame);
        P.q_cur = q;
        P.seq = q + 1;
        if (P.tel_slots > 0 && (q & ((1ull << P.tel_dshift) - 1)) == 0) {
            const size_t k = (size_t)((q >> P.tel_dshift) & (uint64_t)(P.tel_slots - 1));
            P.tel_frame[k] = frame;
            P.tel_dropped[k] = 0;
        }
        const size_t slot = q % P.slot_frame.size();
        P.slot_frame[slot] = frame;
        P.slot_dropped[slot] = 0;
        P.slot_t_last[slot] = 0;
        P.slot_tlc0[slot] = reinterpret_cast<volatile FrameTel *>(P.tel + slot)->ticks_last_chunk;
        P.slot_tpub0[slot] = reinterpret_cast<volatile FrameTel *>(P.tel + slot)->ticks_publish;
        I->cur_frame = frame;
        I->cur_started = false;
        for (auto &W : I->wfs) W.next_chunk = 0;
        if (pe.running && stream_done(pe.stream)) {
            // the loop left on its own: after an idle period (fine) or a watchdog
            pe.running = false;
            pe.serving = false;
            if (*reinterpret_cast<volatile uint32_t *>(pe.status) != PERSIST_OK)
                return fail(e, RTC_E_DEVICE);
        }
        if (!pe.running) TRY(launch_serving(e));
    }
    if (chunk != S.next_chunk) return RTC_E_INVAL;
    return RTC_OK;
}

// The ring slot row where chunk rows start (rows at the ring's 16-byte pitch).
uint16_t *chunk_dst(rtc_engine *e, Instance *I, int w, int chunk) {
    const WfsState &S = I->wfs[w];
    return S.h_stage + (size_t)(I->ps.q_cur % (uint64_t)e->ring_depth) * S.slot16 +
           (size_t)S.row0[chunk] * S.pitch16;
}

// Hands the chunk's rows in the ring to the loop (its doorbell).
void end_chunk(Instance *I, int w, uint64_t frame, int chunk, int64_t t_in) {
    PersistInstState &P = I->ps;
    WfsState &S = I->wfs[w];
    const uint64_t q = P.q_cur;
    store_release(P.doorbell + w, db_word(q, (uint64_t)chunk + 1));
    S.next_chunk++;
    I->cur_started = true;
    bool all = true;
    for (auto &W : I->wfs) all = all && W.next_chunk == W.d.n_chunks;
    if (all) {
        P.slot_t_last[q % P.slot_t_last.size()] = t_in;
        I->next_frame = frame + 1;
        I->cur_frame = ~0ull;
        I->cur_started = false;
    }
}

}  // namespace

rtc_status persist_submit(rtc_engine *e, Instance *I, int w, uint64_t frame, int chunk,
                          const uint16_t *rows, int64_t t_in) {
    TRY(begin_chunk(e, I, w, frame, chunk));
    const WfsState &S = I->wfs[w];
    uint16_t *dst = chunk_dst(e, I, w, chunk);
    for (int r = 0; r < S.row0[chunk + 1] - S.row0[chunk]; ++r)
        std::memcpy(dst + (size_t)r * S.pitch16, rows + (size_t)r * S.d.frame_w,
                    (size_t)S.d.frame_w * 2);
    end_chunk(I, w, frame, chunk, t_in);
    return RTC_OK;
}

rtc_status persist_acquire(rtc_engine *e, Instance *I, int w, uint64_t frame, int chunk,
                           uint16_t **rows, int32_t *pitch) {
    TRY(begin_chunk(e, I, w, frame, chunk));
    WfsState &S = I->wfs[w];
    S.acquired = chunk;
    S.acq_frame = frame;
    *rows = chunk_dst(e, I, w, chunk);
    *pitch = S.pitch16;
    return RTC_OK;
}

rtc_status persist_commit(rtc_engine *e, Instance *I, int w, uint64_t frame, int chunk,
                          int64_t t_in) {
    (void)e;
    WfsState &S = I->wfs[w];
    if (S.acquired != chunk || S.acq_frame != frame) return RTC_E_INVAL;
    S.acquired = -1;
    if (I->cur_frame != frame) return RTC_E_FRAME_DROPPED;   // superseded meanwhile
    end_chunk(I, w, frame, chunk, t_in);
    return RTC_OK;
}

rtc_status persist_wait(rtc_engine *e, Instance *I, uint64_t frame, float *cmds,
                        int64_t timeout_ns, rtc_frame_info *info) {
    PersistInstState &P = I->ps;
    const int64_t t0 = now_ns();
    const size_t depth = P.slot_frame.size();
    uint64_t q = ~0ull;
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(I->mu);
            for (uint64_t k = 0; k < depth && P.seq > k; ++k) {
                const uint64_t qq = P.seq - 1 - k;
                if (P.slot_frame[qq % depth] == frame) {
                    q = qq;
                    break;
                }
            }
            if (q == ~0ull && frame < I->next_frame && I->cur_frame != frame)
                return RTC_E_FRAME_DROPPED;    // too old, or never started
        }
        if (q != ~0ull) break;
        if (now_ns() - t0 > timeout_ns) return RTC_E_TIMEOUT;
        std::this_thread::yield();
    }
    const size_t slot = q % depth;
    // every tile flags its commands once they are in the mailbox (a tile's
    // frames are integrated in order, so its flag only grows): the frame is
    // ready when every flag has reached it, or when the publication count has
    // (the loop counts the tiles on the device before it publishes)
    const int nt = I->n_tiles;
    int tk = 0;      // tiles before tk are known ready
    for (;;) {
        tk = tiles_ready_from([&](int t) { return load_acquire(P.tile_host + t); }, nt, q, tk);
        if (tk == nt || load_acquire(P.cmd_seq) >= q + 1) break;
        if (now_ns() - t0 > timeout_ns) return RTC_E_TIMEOUT;
        if (e->pe.running && stream_done(e->pe.stream)) return fail(e, RTC_E_DEVICE);
    }
    const int64_t t_ready = now_ns();
    {
        std::lock_guard<std::mutex> lk(I->mu);
        if (P.slot_frame[slot] != frame) return RTC_E_FRAME_DROPPED;   // slot reused
        if (P.slot_dropped[slot]) return RTC_E_FRAME_DROPPED;
    }
    std::memcpy(cmds, I->h_mail + slot * (size_t)I->n_act, (size_t)I->n_act * 4);
    // The loop rewrites this mailbox slot for frame q + depth, which a
    // producer thread may start once frame q is published.  As in a seqlock,
    // the copy is whole only if that frame had not been started when the copy
    // ended (the loop writes a frame's commands after its chunks arrive, which
    // is after the host started it).
    std::atomic_thread_fence(std::memory_order_acquire);
    {
        std::lock_guard<std::mutex> lk(I->mu);
        if (!mailbox_copy_whole(P.seq, q, depth) || P.slot_frame[slot] != frame)
            return RTC_E_FRAME_DROPPED;
    }
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->frame = frame;
        info->t_last_chunk_ns = P.slot_t_last[slot];
        info->t_ready_ns = t_ready;
        volatile FrameTel *tel = P.tel + slot;
        // a frame whose last chunks carry no pixel it needs is published before
        // the loop sees those chunks arrive: wait briefly for that stamp (0 if
        // it does not come)
        uint64_t start = tel->ticks_last_chunk;
        if (P.slot_t_last[slot] != 0) {
            while (start == P.slot_tlc0[slot] && now_ns() - t_ready < kStampWaitNs) {
                std::this_thread::yield();
                start = tel->ticks_last_chunk;
            }
        }
        info->dev_ticks_start = start == P.slot_tlc0[slot] ? 0 : start;
        // the tiles' flags can reach the host before the loop has counted the
        // tiles and stamped the publication: wait briefly for that stamp
        uint64_t pub = tel->ticks_publish;
        while (pub == P.slot_tpub0[slot] && now_ns() - t_ready < kStampWaitNs) {
            std::this_thread::yield();
            pub = tel->ticks_publish;
        }
        info->dev_ticks_cmd = pub;
        info->drops = I->drops;
    }
    return RTC_OK;
}

rtc_status persist_batch(rtc_engine *e, Instance *I, const uint16_t *const *frames,
                         const int64_t *frame_stride, int32_t n_frames, float *cmds,
                         float *slopes, int32_t *counts, hipStream_t st) {
    PersistEngine &pe = e->pe;
    if (n_frames == 0) return RTC_OK;
    if (pe.running) TRY(persist_quiesce(e));
    PersistInstState &P = I->ps;
    PersistInst d = describe(e, I);
    d.steps = steps_dev(I);
    d.serving = 0;
    for (size_t s = 0; s < I->wfs.size(); ++s) {
        d.src[s] = frames[s];
        d.src_stride[s] = frame_stride[s];
        d.src_pitch[s] = I->wfs[s].d.frame_w;
    }
    d.q_begin = P.seq;
    d.q_end = P.seq + (uint64_t)n_frames;
    // coefficients: slot 0 = active parameters, slot 1 = staged ones from the
    // first frame at or after the pending switch
    const int a = I->active;
    for (int s = 0; s < 2; ++s) {
        const int src = s == 0 ? a : 1 - a;
        const double gd = I->gain[src], ld = I->leak[src];
        d.coef.g[s] = (float)gd;
        d.coef.c1[s] = I->d.polc ? (float)(1.0 - ld - gd) : (float)(1.0 - ld);
    }
    d.coef.q_switch = ~0ull;
    const uint64_t f0 = I->next_frame;
    if (I->pending) {
        const uint64_t fs = std::max(I->f_switch, f0);
        if (fs < f0 + (uint64_t)n_frames) {
            d.coef.q_switch = d.q_begin + (fs - f0);
            settle_params(I, fs);
        }
    }
    // matrices: the active slot, then the staged one from a pending swap's
    // frame on, if that frame is in the batch
    d.coef.mslot[0] = I->m_active;
    d.coef.mslot[1] = 1 - I->m_active;
    d.coef.q_mswitch = ~0ull;
    if (I->m_pending) {
        const uint64_t fs = std::max(I->m_switch, f0);
        if (fs < f0 + (uint64_t)n_frames) {
            d.coef.q_mswitch = d.q_begin + (fs - f0);
            settle_matrices(I, fs);
        }
    }
    d.cmds_out = cmds;
    d.slopes_out = slopes;
    d.counts_out = counts;
    d.w0 = 0;
    d.w1 = pe.n_blocks_batch * 4;
    // this instance alone; the other descriptors must not claim workers
    std::vector<PersistInst> descs(1, d);
    TRY(stage_state_in(I, d.q_begin, st));
    TRY(upload_and_launch(e, {I}, descs, st, true, pe.n_blocks_batch));
    TRY(stage_state_out(I, d.q_end - 1, st));
    P.seq = d.q_end;
    I->next_frame += (uint64_t)n_frames;
    return RTC_OK;
}
