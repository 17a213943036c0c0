// Internal layouts shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rtc.h"

namespace rtc {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kTileRows = 64;      // matrix rows per MVM tile: one row per lane
constexpr int kPolcBlock = 512;    // command elements per POLC column block
constexpr int kMaxSegVectors = 128; // longest MVM segment (16-byte vectors per row; its slopes sit in LDS)
constexpr int kMinLastSegVectors = 16;  // shortest segment of a sensor's last column block
constexpr int kEndWordsPerLane = 4; // block-end mask words each lane holds in a reduction
constexpr int kMaxSegments = kEndWordsPerLane * kWave * 32;   // segments of one matrix
constexpr int kMaxShPx = 16;       // largest SH subaperture side (pixels)
constexpr int kMaxShPasses = (kMaxShPx * kMaxShPx + kWave - 1) / kWave;

// Per-sensor constants the kernels need.
struct WfsParam {
    int32_t kind;          // RTC_WFS_*
    int32_t W, H;          // frame size
    int32_t p;             // SH: pixels per subaperture side
    int32_t thr_mode;      // RTC_THR_*
    int32_t mask_words;    // SH: ceil(p*p/64)
    float half;            // SH: (p - 1) / 2
    int32_t norm;          // pyramid: RTC_PYR_NORM_*
    int32_t qrow[4], qcol[4];
    int32_t pu0, pn;       // pyramid: the sensor's units [pu0, pu0 + pn) of the unit list
};

struct WfsParamSet {
    WfsParam w[RTC_MAX_WFS];
};

struct FrameSet {
    const uint16_t *f[RTC_MAX_WFS];
};

// A list of sensors (indices into the instance's sensors).
struct WfsList {
    int32_t w[RTC_MAX_WFS];
    int32_t n;
};

// One Shack-Hartmann subaperture (32 bytes).
struct ShUnit {
    int32_t row0, col0;    // first pixel in the frame
    int32_t wfs;           // sensor index within the instance
    int32_t unit;          // unit index within the instance (slope pair index)
    int32_t pad;           // index of its x slope in the padded slope vector
    int32_t cal;           // offset of its p*p calibration values
    int32_t mask;          // first mask word
    int32_t r;
};

// One pyramid pupil pixel (32 bytes).
struct PyrUnit {
    int32_t i, j;          // row, column inside the pupil image
    int32_t wfs, unit, pad;
    int32_t mask;
    int32_t r0, r1;
};

// One column block of a matrix: the columns whose slopes one (sensor, chunk)
// produces.  The block is stored tile by tile: tile t holds rows
// [64t, 64t + nr) and, for vector v and row l, the 16 bytes of columns
// [v*E, v*E + E) of row 64t + l at byte offset (v * nr + l) * 16.
struct KBlock {
    int64_t base;          // byte offset of tile 0 in the matrix buffer
    int32_t kv;            // 16-byte vectors per row (columns padded to kv*E)
    int32_t spad;          // offset of its first column in the padded vector
    int32_t k0;            // first column in the logical matrix
    int32_t k;             // logical columns
    int32_t wfs, chunk;
};

// One (sensor, chunk) of the readout order and the column block it completes
// (-1 when the chunk completes no unit).
struct Step {
    int32_t wfs, chunk, kb;
    // serving ingest: the chunk's rows of a ring slot are 16-byte units
    // [u0, u0 + n16) (rows are padded to 16 bytes), copied host -> device in
    // pieces of kIngestUnits; its pieces are [ing0, ing0 + ing_n) of the
    // frame's piece list
    int32_t u0, n16, ing0, ing_n, r;
};
constexpr int kIngestUnits = 512;                 // 16-byte units per ingest piece (8 KiB)

// A segment is the part of one column block that one wavefront streams for a
// tile: vectors [v0, v0 + nv) of block kb (each block is cut into nearly
// equal segments of at most kMaxSegVectors).  Each segment owns one partial
// (its index in the global segment order).  Every path (per-launch MVM, the
// frame loop's batch and serving tasks) streams the same segments and adds
// the same partials in the same order.
struct Segment {
    int32_t kb, v0, nv, r;
};
// A segment with its column block's fields folded in, for the per-launch MVM:
// one record read per segment instead of a segment then its block.
struct SegRun {
    int64_t base;          // the block's byte offset of tile 0
    int32_t kv;            // the block's 16-byte vectors per row
    int32_t xoff;          // offset of the segment's first slope in the padded vector
    int32_t v0, nv;        // the segment's vectors within the block
    int32_t r0, r1;
};

// Per-tile arrival counters of the per-launch MVM sit 256 bytes apart:
// agent-scope atomics on one cache line serialise (~10^4 arrivals per MVM on
// a handful of lines cost 25-45 us), on distinct lines they run in parallel.
constexpr int kCountStride = 64;   // uint32 per counter

// Work done by the last wavefront to finish a row tile of an MVM.
enum { EPI_NONE = 0, EPI_INTEGRATE = 1, EPI_REDUCE = 2 };
struct MvmEpilogue {
    int32_t mode;          // EPI_*
    int32_t n_parts;       // segment partials per row (all launches of the frame)
    int32_t rev;           // 1: each segment streamed last vector first (odd frames)
    int32_t r0;
    const uint32_t *seg_ends;  // bit j: segment j ends its column block
    uint32_t *count;       // per-tile arrival counters (tile t at count[t * kCountStride]),
                           // zero between frames
    const float *p;        // INTEGRATE: POLC term (nullable)
    const float *scale;    // INTEGRATE: FP8 row scales (nullable)
    float *a;              // INTEGRATE: command state, updated in place
    float *out;            // INTEGRATE: copy of the new commands (nullable)
    float *y;              // REDUCE: destination
    float c1, g;           // INTEGRATE: a = c1 a + g (y + p)
};

// ---------------------------------------------------------------------------
// Persistent frame loop (rtc_persist.hip).

// Work of one column block in the frame loop: its centroid tasks (one per SH
// unit, one per 64 pyramid units) and its MVM tasks (segment x tile).  Task j
// of a block goes to worker (base + j) mod n_workers.
struct KbWork {
    int32_t kind;          // RTC_WFS_*
    int32_t wfs;
    int32_t cu0, cu1;      // unit range in the SH or pyramid list
    int32_t n_cen;         // centroid tasks
    int32_t cen_base;
    int32_t seg0, nseg;    // the block's segments
    int32_t mvm_base;
    int32_t r0, r1, r2;
};

// Frame coefficients a = c1 a + g (y + p): slot A for frames < q_switch,
// slot B from q_switch on.  Matrices: slot mslot[0] for frames < q_mswitch,
// mslot[1] from q_mswitch on.
struct Coef {
    float c1[2], g[2];
    uint64_t q_switch;
    uint64_t q_mswitch;
    int32_t mslot[2];
};

// Host-visible parameter block of a serving instance (pinned).  The host
// writes the staged slot's values, then `word` = (q_switch << 1) | staged.
// `mword` = (q_mswitch << 1) | s: frames from q_mswitch on use matrix slot s,
// earlier frames slot 1 - s.
struct ParamBlock {
    float c1[2], g[2];
    uint64_t word;
    uint64_t mword;
};

struct FrameTel {
    uint64_t ticks_last_chunk;     // device clock when the frame's last chunk was seen
    uint64_t ticks_publish;        // device clock when its commands were published
};

// Frames of one frame-loop instance in flight at once: slopes, partials and
// arrival counters exist kDepth times, frame q using copy q % kDepth.
constexpr int kDepth = 3;

struct PersistInst {
    // tables
    const ShUnit *sh;
    const PyrUnit *py;
    int32_t n_sh, n_pyr;
    const KBlock *kbs;
    const KbWork *kbw;
    const Segment *segs;
    const uint32_t *seg_ends;      // bit j: segment j ends its column block
    const uint32_t *tail_ends;     // the same for the sum's tail, segment n_head at bit 0
    int32_t n_head, r9;            // segments before the sum's tail (their prefix is formed apart)
    const Step *steps;
    int32_t n_kb, n_seg, n_steps, n_wfs;
    int32_t n_cen_all, r5;         // centroid tasks of a frame (every block)
    const WfsParam *wp;
    // calibration
    const float *sh_dark, *sh_flat, *sh_bg, *sh_thr;
    const float *py_dark, *py_flat, *py_bg, *py_thr;
    const float *ref;
    // reconstruction matrix, two slots (a staged matrix becomes active at a
    // frame boundary)
    const uint8_t *cm[2];
    const float *scale[2];         // FP8 row scales or null
    int32_t dtype, n_act, n_tiles, polc;
    int32_t stream_nt, r7;         // the engine's matrices exceed the Infinity Cache
    // POLC
    const uint8_t *M[2];           // slot s pairs with cm[s]
    const KBlock *kbm;
    const Segment *segm;
    const uint32_t *segm_ends;
    int32_t n_kbm, n_segm;
    // state and scratch
    float *s_pad[kDepth];          // frame q uses buffer q % kDepth
    float *y_part[kDepth];
    float *p_part[kDepth];
    float *p;
    float *a;                      // two command buffers of a_stride floats (frame parity)
    int32_t a_stride, r4;
    // counters, one kCtrSlot-sized slot each; [kDepth]: by q % kDepth
    uint64_t *cen_fan;             // [kDepth][n_kb] fan-in: centroid tasks of a block
    uint64_t *tile_fan;            // [kDepth] fan-in: tiles whose commands are out
    uint64_t *pol_fan;             // [kDepth] fan-in: tiles whose POLC term is formed
    uint64_t *tile_cnt;            // [kDepth][n_tiles] tail partials (and the prefix) of a tile formed
    uint64_t *head_cnt;            // [kDepth][n_tiles] head partials of a tile formed
    float *pre;                    // [kDepth][n_act] the sum's prefix over the head blocks
    uint64_t *join;                // [kDepth][n_tiles] accumulation joins
    uint64_t *pol_cnt;             // [kDepth][n_tiles] POLC partials of a tile
    uint64_t *p_done;              // [n_tiles] q + 1 of the last POLC term reduced
    uint64_t *tile_pub;            // [n_tiles] q + 1 of the last commands written
    uint64_t *pol_seg;             // [kDepth][n_segm] POLC tasks of a segment done reading a_q
    uint64_t *db_mirror;           // device copy of the doorbells, per sensor
    uint64_t *drop_mirror;         // per mailbox slot: q + 1 of a dropped frame
    // frame source
    int32_t serving;
    int32_t ring_depth;
    const uint16_t *src[RTC_MAX_WFS];      // serving: device ring; batch: device frames
    int64_t src_stride[RTC_MAX_WFS];       // uint16 per frame (ring slot)
    int32_t src_pitch[RTC_MAX_WFS];        // uint16 per row
    const uint16_t *ring_host[RTC_MAX_WFS];  // serving: the pinned ring the host fills
    uint64_t ring_bytes[RTC_MAX_WFS];      // size of each pinned ring
    uint64_t *ing_cnt;                     // [kDepth][n_steps] ingest pieces copied
    int32_t n_ing_all, r6;                 // ingest pieces of a frame
    const uint64_t *doorbell;              // pinned, per sensor: (q << 20) | chunks
    const uint64_t *drop_host;             // pinned, per slot: q + 1 of a dropped frame
    const ParamBlock *params;              // serving (pinned)
    ParamBlock *param_mirror;              // serving (device)
    Coef coef;                             // batch
    // telemetry (serving): frames q with q % 2^tel_dshift == 0 write their
    // slopes, counts and commands into device ring slot (q >> tel_dshift) &
    // tel_smask, one record of tel_rec words (a multiple of 4): slopes, then
    // counts, then commands, then from word tel_mask_off the thresholded-pixel
    // masks (mask_words uint64); once the frame is published, workers copy the
    // record into the same slot of the pinned host ring, task j setting
    // tel_flags[slot][j] = q + 1 after its part
    float *tel_ring;                       // null: off
    float *tel_host;
    uint64_t *tel_flags;                   // pinned, [slots][kTelMaxTasks]
    int32_t tel_rec;
    int32_t tel_mask_off, r8;              // word offset of the masks (uint64, 16-byte aligned)
    int32_t tel_dshift, tel_smask;
    // outputs
    float *mail;                           // pinned, ring_depth x n_act (serving)
    uint64_t *cmd_seq;                     // pinned: q + 1 of the last published frame
    uint64_t *tile_host;                   // pinned, per tile: q + 1 of the last frame whose
                                           // commands of the tile are in the mailbox
    uint64_t *pol_seq;                     // pinned: q + 1 of the last frame whose POLC term is done
    FrameTel *tel;                         // pinned, per slot
    float *cmds_out;                       // batch, n_frames x n_act (nullable)
    float *slopes_out;                     // batch, n_frames x n_slopes (nullable)
    int32_t *counts_out;                   // batch (nullable)
    int32_t n_slopes, n_units;
    // frames and workers
    uint64_t q_begin, q_end;               // sequence numbers processed by this launch
    int32_t w0, w1;                        // worker range (a serving instance's first is its sentinel)
    int32_t r3;
};

struct PersistArgs {
    const PersistInst *inst;               // device array
    int32_t n_inst;
    int32_t r0;
    const uint32_t *stop_host;             // pinned: nonzero asks the loop to exit
    uint32_t *stop_dev;                    // device mirror of the stop request
    uint32_t *status;                      // pinned: nonzero after a watchdog expiry
    uint64_t dep_watchdog;                 // device-clock ticks a dependency wait may take
    uint64_t idle_watchdog;                // device-clock ticks a doorbell wait may take
    uint64_t *trace;                       // timeline record or null
    int32_t trace_frames;                  // frames recorded per launch
    int32_t n_waves;                       // wavefronts in the grid
};

enum { PERSIST_OK = 0, PERSIST_WATCHDOG = 1 };
// Telemetry copy: 16-byte units per task, and the most tasks a record takes
// (records up to 2 MiB).
constexpr int kTelUnits = 1024;
constexpr int kTelMaxTasks = 128;
constexpr uint64_t kDbChunkMask = (1ull << 20) - 1;
constexpr int kDbShift = 20;
// Frame-loop counters sit 256 bytes apart: agent-scope atomics on one cache
// line serialise (~12 ns each), on distinct lines they proceed in parallel.
constexpr int kCtrSlot = 32;                      // uint64 per counter slot
// A fan-in barrier of n tasks: task j counts on stripe j % kFanStripes, the
// arrival completing a stripe's quota counts on the top slot, and waiters
// poll only the top slot.
constexpr int kFanStripes = 32;
constexpr int kFanSlots = kFanStripes + 2;        // stripes, the top, the done flag

// serving: the indefinitely running form (2 waves per SIMD, so up to 256
// VGPRs a lane); otherwise the batch form (4 waves per SIMD)
void launch_frame_loop(hipStream_t st, int n_blocks, const PersistArgs &args, bool serving);
void launch_seed_counters(hipStream_t st, uint64_t *ctr, size_t n, size_t join_off, int n_tiles,
                          int par, int polc);
int frame_loop_max_blocks_per_cu(bool serving);

// Launchers (defined in rtc_kernels.hip).
void launch_sh_centroid(hipStream_t st, const ShUnit *units, int u0, int u1,
                        const FrameSet &frames, const WfsParamSet &params,
                        const float *dark, const float *flat, const float *bg,
                        const float *thr, const float *ref, float *s_pad, float *s_out,
                        int32_t *counts, uint64_t *masks);
void launch_pyr_slopes(hipStream_t st, const PyrUnit *units, int u0, int u1, int n_pyr,
                       const FrameSet &frames, const WfsParamSet &params,
                       const float *dark4, const float *flat4, const float *bg4,
                       const float *thr, const float *ref, float *s_pad, float *s_out,
                       int32_t *counts, uint64_t *masks, const float *gsum);
// Per sensor of `wfs` (pyramids with global normalisation), the frame's
// intensity sum over the pupil into gsum[sensor].
void launch_pyr_sum(hipStream_t st, const PyrUnit *units, int n_pyr, const FrameSet &frames,
                    const WfsParamSet &params, const float *dark4, const float *flat4,
                    const float *bg4, const float *thr, const WfsList &wfs, float *gsum);
// stream_nt: stream the matrix with non-temporal loads (matrices larger than
// the Infinity Cache); otherwise ordinary loads keep a smaller matrix resident.
constexpr int64_t kCacheResidentBytes = 192ll << 20;
// Segments [s0, s0 + n_segs) of a matrix times x_pad into their partials
// (y_part[segment][row]); the epilogue runs when a tile's partials are
// complete (E.n_parts segments over all launches of the frame).
void launch_mvm(hipStream_t st, int dtype, bool stream_nt, const void *cm, const SegRun *runs,
                int s0, int n_segs, int n_rows, const float *x_pad, float *y_part,
                const MvmEpilogue &epi);
// Slopes of the next frame, formed by extra workgroups of the current frame's
// MVM launch (every SH unit, then every pyramid unit of the instance).
struct NextSlopes {
    const ShUnit *sh;
    const PyrUnit *py;
    int32_t n_sh, n_pyr;
    FrameSet frames;
    const float *sh_dark, *sh_flat, *sh_bg, *sh_thr;
    const float *py_dark, *py_flat, *py_bg, *py_thr;
    const float *ref;
    float *s_pad, *s_out;
    int32_t *counts;
    uint64_t *masks;
    const float *py_gsum;          // pyramid sensors with global normalisation: frame sums
};
// launch_mvm (reading x_pad) plus, in the same grid, the slopes of the next
// frame into next.s_pad (a different buffer than x_pad).
void launch_mvm_next(hipStream_t st, int dtype, bool stream_nt, const void *cm,
                     const SegRun *runs, int n_segs, int n_rows, const float *x_pad,
                     float *y_part, const MvmEpilogue &epi, const NextSlopes &next,
                     const WfsParamSet &params);
// Static scratch of rtc_process_frames_noalloc (rtc_kernels.hip): its size,
// the device address of the current device's copy (call with the device
// current), and a fill kernel for its counters.
constexpr size_t kScratchBytes = 16ull << 20;
hipError_t scratch_address(void **ptr);
void launch_fill_u32(hipStream_t st, uint32_t *p, size_t n, uint32_t v);
void launch_dgemm_rd(hipStream_t st, const float *R, const double *D, double *M, int n_act,
                     int n_s);

}  // namespace rtc
