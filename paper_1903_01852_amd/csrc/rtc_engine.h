// Engine state shared by the host runtime sources (private header).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <ctime>
#include <mutex>
#include <vector>

#include "rtc.h"
#include "rtc_internal.h"

using rtc::FrameTel;
using rtc::KBlock;
using rtc::KbWork;
using rtc::ParamBlock;
using rtc::PersistInst;
using rtc::PyrUnit;
using rtc::Segment;
using rtc::ShUnit;
using rtc::Step;
using rtc::WfsParamSet;

struct DevBuf {
    void *p = nullptr;
    size_t n = 0;
};

struct WfsState {
    rtc_wfs_desc d{};
    std::vector<uint8_t> valid;
    int u0 = 0, u1 = 0;            // unit range in the instance
    int kind0 = 0;                 // first index in the SH or pyramid unit list
    std::vector<int> row0;         // chunk row starts, n_chunks + 1 entries
    std::vector<int> kb_of_chunk;  // column block produced by each chunk, or -1
    std::vector<int> unit_ready;   // last frame row each unit needs (per unit)
    // serving
    int next_chunk = 0;
    uint16_t *d_ring = nullptr;    // ring_depth frames on the device
    uint16_t *h_stage = nullptr;   // pinned staging ring (ring_depth frames)
    size_t ring_elems = 0;         // uint16 in each ring
    int pitch16 = 0;               // persistent serving: row pitch (uint16), rows padded to 16 B
    int acquired = -1;             // chunk lent by rtc_acquire_chunk, not yet committed
    uint64_t acq_frame = 0;
    size_t slot16 = 0;             // persistent serving: uint16 per ring slot
};

struct FrameSlot {
    uint64_t frame = ~0ull;
    bool complete = false;         // work enqueued
    bool dropped = false;
    hipEvent_t done = nullptr;
    int64_t t_last_chunk = 0;
};

// Persistent frame loop: per-instance buffers and bookkeeping.
struct PersistInstState {
    // device
    // copies 1 .. kDepth - 1 of the slope and partial buffers (copy 0 is the
    // per-launch path's)
    float *spad_x[rtc::kDepth - 1] = {}, *ypart_x[rtc::kDepth - 1] = {},
          *ppart_x[rtc::kDepth - 1] = {};
    uint64_t *ctr = nullptr;       // every frame-loop counter, zeroed on reset
    size_t n_ctr = 0;
    uint64_t *cen_fan = nullptr, *tile_fan = nullptr, *pol_fan = nullptr;
    uint64_t *tile_cnt = nullptr, *join = nullptr, *pol_cnt = nullptr, *p_done = nullptr;
    uint64_t *tile_pub = nullptr, *pol_seg = nullptr, *head_cnt = nullptr;
    uint64_t *tile_host = nullptr; // pinned [n_tiles]: q + 1 of a tile's last commands in the mailbox
    float *pre = nullptr;          // [kDepth][n_act] prefixes of the reconstruction sum
    int n_cen_all = 0;             // centroid tasks of a frame
    int n_ing_all = 0;             // ingest pieces of a frame (serving)
    uint64_t *ing_cnt = nullptr;   // [kDepth][n_steps] ingest counters
    uint64_t *db_mirror = nullptr, *drop_mirror = nullptr;
    ParamBlock *param_mirror = nullptr;
    KbWork *kbw = nullptr;
    rtc::WfsParam *wp = nullptr;
    // pinned host
    uint64_t *doorbell = nullptr;  // per sensor: (q << 20) | chunks
    uint64_t *drop_host = nullptr; // per slot: q + 1 of a dropped frame
    ParamBlock *params = nullptr;
    uint64_t *cmd_seq = nullptr;   // q + 1 of the last published frame
    uint64_t *pol_seq = nullptr;   // q + 1 of the last frame whose POLC term is done
    FrameTel *tel = nullptr;       // per mailbox slot
    // host
    std::vector<KbWork> kbw_h;
    uint64_t seq = 0;              // sequence number of the next frame to start
    uint64_t q_cur = 0;            // sequence number of the frame in progress
    std::vector<uint64_t> slot_frame;   // frame id of the frame in each slot
    std::vector<int64_t> slot_t_last;   // host clock at its last chunk
    std::vector<uint64_t> slot_tlc0;    // the slot's last-chunk stamp before the frame (stale)
    std::vector<uint64_t> slot_tpub0;   // the slot's publication stamp before the frame (stale)
    std::vector<uint8_t> slot_dropped;
    uint64_t param_word = 0;       // (q_switch << 1) | staged slot, as last written
    uint64_t mword = 0;            // (q_mswitch << 1) | slot, as last written
    uint64_t mq_last = 0;          // frames before this sequence number may use the inactive matrix slot
    // telemetry: the serving loop forms records in a device ring and copies
    // each into the pinned host ring once its frame is published
    float *tel_ring = nullptr;     // device, [slots][rec]: slopes, counts, commands
    float *tel_host = nullptr;     // pinned, the same layout
    uint64_t *tel_flags = nullptr; // pinned, [slots][kTelMaxTasks]: q + 1 per copied part
    int tel_rec = 0;               // 4-byte words per record (a multiple of 4)
    int tel_mask_off = 0;          // word offset of the masks in a record
    int tel_dshift = 0;            // decimation 2^tel_dshift
    int tel_slots = 0;             // 0: telemetry off
    uint64_t tel_next = 0;         // sequence number of the next record to read
    std::vector<uint64_t> tel_frame;    // frame number of each slot's record
    std::vector<uint8_t> tel_dropped;   // the record's frame was dropped
    int w0 = 0, w1 = 0;            // worker range of the running loop
};

struct Instance {
    rtc_instance_desc d{};
    std::vector<hipEvent_t> mvm_ev;    // MVM timer: event pairs (rtc_mvm_timing)
    std::vector<int32_t> mvm_ev_len;   // launches each recorded pair brackets
    size_t mvm_ev_used = 0;            // pairs recorded
    int mvm_ev_every = 1;              // launches per pair
    int mvm_run = 0;                   // launches in the open pair
    bool mvm_open = false;             // a pair's first event is recorded
    std::vector<WfsState> wfs;
    int n_units = 0, n_slopes = 0, n_act = 0, n_sh = 0, n_pyr = 0;
    int mask_words = 0;
    std::vector<ShUnit> sh;
    std::vector<PyrUnit> py;
    std::vector<KBlock> kb;        // reconstruction column blocks, in readout order
    std::vector<Step> steps;       // (sensor, chunk) pairs in readout order
    std::vector<KBlock> kbm;       // POLC column blocks
    std::vector<Segment> seg, segm;            // segments: reconstruction, POLC
    std::vector<int> kb_seg0, kb_nseg;         // segments of each column block
    std::vector<uint32_t> seg_ends, segm_ends; // bit j: segment j ends its block (recon / POLC)
    int n_head_seg = 0;                        // segments before the reconstruction sum's tail
    std::vector<uint32_t> tail_ends;           // seg_ends of the tail's segments, from bit 0
    int spad_len = 0;
    int64_t cm_bytes = 0, m_bytes = 0;
    bool stream_nt = false;        // non-temporal matrix loads (the engine's matrices exceed the cache)
    WfsParamSet params{};
    rtc::WfsList pyr_global{};     // pyramid sensors with global normalisation
    // device
    ShUnit *d_sh = nullptr;
    PyrUnit *d_py = nullptr;
    KBlock *d_kb = nullptr, *d_kbm = nullptr;
    Segment *d_seg = nullptr, *d_segm = nullptr;
    rtc::SegRun *d_run = nullptr, *d_runm = nullptr;   // the segments, block fields folded in
    uint32_t *d_seg_ends = nullptr, *d_segm_ends = nullptr, *d_tail_ends = nullptr;
    float *d_sh_dark = nullptr, *d_sh_flat = nullptr, *d_sh_bg = nullptr, *d_sh_thr = nullptr;
    float *d_py_dark = nullptr, *d_py_flat = nullptr, *d_py_bg = nullptr, *d_py_thr = nullptr;
    float *d_ref = nullptr;
    float *d_pyr_sum = nullptr;    // per sensor: the frame's pupil sum (global normalisation)
    float *d_spad = nullptr, *d_sout = nullptr;
    float *d_spad2 = nullptr;      // per-launch batch: slopes of the next frame
    int32_t *d_counts = nullptr;
    uint64_t *d_masks = nullptr;
    // matrices, two slots: frames use slot m_active; a staged matrix set in
    // the other slot becomes active at frame m_switch (rtc_swap_matrices)
    uint8_t *d_cm_s[2] = {nullptr, nullptr};
    float *d_scale_s[2] = {nullptr, nullptr};
    uint8_t *d_M_s[2] = {nullptr, nullptr};
    int m_active = 0;
    bool m_staged = false;         // the inactive slot holds matrices not yet swapped in
    bool m_pending = false;        // a swap takes effect at frame m_switch
    uint64_t m_switch = 0;
    int frame_mslot = 0;           // slot of the frame in progress (per-launch serving)
    float *d_ypart = nullptr, *d_ppart = nullptr;
    float *d_a = nullptr;          // command state, padded to the POLC block size
    float *d_p = nullptr;          // POLC term for the next frame, M a
    float *d_yscratch = nullptr;   // destination of the timing-only MVM
    uint32_t *d_count = nullptr;   // per-tile arrival counters: reconstruction
    uint32_t *d_count_m = nullptr; //                            POLC
    uint32_t *d_count_t = nullptr; //                            timing MVM
    int n_tiles = 0;
    int a_len = 0;
    float frame_c1 = 0, frame_g = 0;   // coefficients of the frame in progress (serving)
    bool loaded = false;
    // parameters: two slots, the staged one becomes active at frame f_switch
    float gain[2] = {0, 0}, leak[2] = {0, 0};
    int active = 0;
    bool pending = false;
    uint64_t f_switch = 0;
    uint64_t next_frame = 0;       // next frame the batch path processes
    // Frames started since the last matrix load or state reset (the frame loop
    // counts the same in its q): the parity of a frame's index in this
    // sequence picks its streaming direction.
    uint64_t seq = 0;
    uint64_t frame_seq = 0;        // index of the frame in progress (per-launch serving)
    uint32_t drops = 0;
    // serving
    uint64_t cur_frame = ~0ull;
    bool cur_started = false;
    std::vector<FrameSlot> slots;
    float *h_mail = nullptr;       // pinned, ring_depth x n_act
    PersistInstState ps;
    std::mutex mu;
};

struct PersistEngine {
    hipStream_t stream = nullptr;  // the frame loop's own stream
    bool running = false;
    bool serving = false;
    int n_blocks = 0;              // grid of the serving loop (room left on each CU)
    int n_blocks_batch = 0;        // grid of a batch launch (full occupancy)
    uint32_t *stop_host = nullptr; // pinned
    uint32_t *status = nullptr;    // pinned
    uint32_t *stop_dev = nullptr;  // device
    PersistInst *d_inst = nullptr; // device descriptors of the serving loop
    PersistInst *d_batch[2] = {nullptr, nullptr};   // device descriptor per batch launch
    PersistInst *h_batch[2] = {nullptr, nullptr};   // pinned staging of those
    hipEvent_t batch_copied[2] = {nullptr, nullptr};
    int batch_slot = 0;
    uint64_t *trace = nullptr;     // device timeline record (rtc_trace_enable)
    int trace_frames = 0;
    int trace_waves = 0;           // grid of the launch the record holds
};

struct rtc_engine {
    int device = 0;
    int ring_depth = 2;
    int mode = RTC_MODE_STREAM;
    hipStream_t stream = nullptr;
    hipStream_t up_stream = nullptr;   // matrix uploads beside running frames
    uint8_t *h_up = nullptr;           // pinned staging of those uploads (2 halves)
    hipEvent_t up_done[2] = {nullptr, nullptr};
    std::vector<Instance *> inst;
    std::vector<DevBuf> allocs;
    std::vector<void *> pinned;
    std::atomic<int> sticky{RTC_OK};
    PersistEngine pe;
    uint8_t *scratch = nullptr;        // this device's copy of the library's static scratch
};

#define HIP_TRY(expr)                                                                \
    do {                                                                             \
        hipError_t _e = (expr);                                                      \
        if (_e != hipSuccess) {                                                      \
            std::fprintf(stderr, "rtc: %s failed: %s (%s:%d)\n", #expr,              \
                         hipGetErrorString(_e), __FILE__, __LINE__);                 \
            return RTC_E_DEVICE;                                                     \
        }                                                                            \
    } while (0)

template <class T>
inline rtc_status dev_alloc(rtc_engine *e, T **p, size_t count) {
    void *q = nullptr;
    const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    if (hipMalloc(&q, bytes) != hipSuccess) return RTC_E_NOMEM;
    if (hipMemset(q, 0, bytes) != hipSuccess) return RTC_E_DEVICE;
    e->allocs.push_back({q, bytes});
    *p = static_cast<T *>(q);
    return RTC_OK;
}

template <class T>
inline rtc_status host_pinned(rtc_engine *e, T **p, size_t count) {
    void *q = nullptr;
    const size_t bytes = std::max<size_t>(count * sizeof(T), 64);
    // coherent (fine-grained) host memory: device reads and writes bypass its caches
    if (hipHostMalloc(&q, bytes, hipHostMallocCoherent) != hipSuccess) return RTC_E_NOMEM;
    std::memset(q, 0, bytes);
    e->pinned.push_back(q);
    *p = static_cast<T *>(q);
    return RTC_OK;
}

inline rtc_status fail(rtc_engine *e, rtc_status s) {
    if (s == RTC_E_DEVICE && e) e->sticky.store(RTC_E_DEVICE);
    return s;
}

#define TRY(expr)                                                                    \
    do {                                                                             \
        rtc_status _s = (expr);                                                      \
        if (_s != RTC_OK) return fail(e, _s);                                        \
    } while (0)


inline int64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}
// Matrix uploads go through two pinned staging halves of this size.
constexpr size_t kUploadHalf = 32u << 20;
inline int elem_size(int dt) { return dt == RTC_CM_F32 ? 4 : dt == RTC_CM_BF16 ? 2 : 1; }
inline int elems_per_vec(int dt) { return 16 / elem_size(dt); }

// rtc_engine.cpp
void coeffs(const Instance *I, uint64_t f, float *c1, float *g);
void settle_params(Instance *I, uint64_t f);
int mat_slot(const Instance *I, uint64_t f);
void settle_matrices(Instance *I, uint64_t f);
rtc_status check(rtc_engine *e, int32_t inst, Instance **out);

// rtc_serve.cpp (persistent frame loop)
rtc_status persist_alloc(rtc_engine *e);
rtc_status persist_stop(rtc_engine *e);
void persist_reset(Instance *I);
rtc_status persist_submit(rtc_engine *e, Instance *I, int w, uint64_t frame, int chunk,
                          const uint16_t *rows, int64_t t_in);
rtc_status persist_wait(rtc_engine *e, Instance *I, uint64_t frame, float *cmds,
                        int64_t timeout_ns, rtc_frame_info *info);
rtc_status persist_batch(rtc_engine *e, Instance *I, const uint16_t *const *frames,
                         const int64_t *frame_stride, int32_t n_frames, float *cmds,
                         float *slopes, int32_t *counts, hipStream_t st);
rtc_status persist_params(rtc_engine *e, Instance *I);
void persist_mswap(Instance *I, uint64_t q_switch, int slot);
void persist_telemetry_free(Instance *I);
rtc_status persist_telemetry(rtc_engine *e, Instance *I, int decimation, int n_slots);
rtc_status persist_telemetry_next(rtc_engine *e, Instance *I, float *slopes, int32_t *counts,
                                  float *cmds, uint64_t *masks, int64_t timeout_ns,
                                  rtc_telemetry_info *info);
rtc_status persist_wait_matrix_free(rtc_engine *e, Instance *I);
rtc_status persist_quiesce(rtc_engine *e);
rtc_status persist_acquire(rtc_engine *e, Instance *I, int w, uint64_t frame, int chunk,
                           uint16_t **rows, int32_t *pitch);
rtc_status persist_commit(rtc_engine *e, Instance *I, int w, uint64_t frame, int chunk,
                          int64_t t_in);
// Timeline record of the frame loop: frames per launch (0 = off).
constexpr int kMaxTraceFrames = 4096;
rtc_status persist_trace(rtc_engine *e, int n_frames);
void persist_free(rtc_engine *e);
