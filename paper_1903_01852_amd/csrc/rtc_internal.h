// Internal layouts shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rtc.h"

namespace rtc {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kTileRows = 64;      // matrix rows per MVM tile: one row per lane
constexpr int kPolcBlock = 512;    // command elements per POLC column block
constexpr int kPieceVectors = 128; // target length of an MVM piece (16-byte vectors per row)
constexpr int kMinMvmWaves = 1536; // at least this many wavefronts per full MVM (6 per CU)
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
    int32_t pad0;
    int32_t qrow[4], qcol[4];
};

struct WfsParamSet {
    WfsParam w[RTC_MAX_WFS];
};

struct FrameSet {
    const uint16_t *f[RTC_MAX_WFS];
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

// A segment is the part of one column block that one wavefront streams for a
// tile: vectors [v0, v0 + nv) of block kb.  Each segment owns one partial
// (its index in the global segment order).  The column range of every tile is
// cut into pieces of nearly equal length so that wavefronts finish together;
// a piece is a run of consecutive segments.  The serving path launches the
// same segments chunk by chunk, so both paths add the same partials in the
// same order.
struct Segment {
    int32_t kb, v0, nv, r;
};
struct Piece {
    int32_t seg0, nseg;
};

// Work done by the last wavefront to finish a row tile of an MVM.
enum { EPI_NONE = 0, EPI_INTEGRATE = 1, EPI_REDUCE = 2 };
struct MvmEpilogue {
    int32_t mode;          // EPI_*
    int32_t n_parts;       // column-block partials per row (all launches of the frame)
    uint32_t *count;       // per-tile arrival counters, zero between frames
    const float *p;        // INTEGRATE: POLC term (nullable)
    const float *scale;    // INTEGRATE: FP8 row scales (nullable)
    float *a;              // INTEGRATE: command state, updated in place
    float *out;            // INTEGRATE: copy of the new commands (nullable)
    float *y;              // REDUCE: destination
    float c1, g;           // INTEGRATE: a = c1 a + g (y + p)
};

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
                       int32_t *counts, uint64_t *masks);
void launch_mvm(hipStream_t st, int dtype, const void *cm, const KBlock *kbs,
                const Segment *segs, const Piece *pieces, int p0, int n_pieces, int n_rows,
                const float *x_pad, float *y_part, const MvmEpilogue &epi);
void launch_dgemm_rd(hipStream_t st, const float *R, const double *D, double *M, int n_act,
                     int n_s);

}  // namespace rtc
