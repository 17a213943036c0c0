// Internal layouts shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rtc.h"

namespace rtc {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kTileRows = 64;      // matrix rows per MVM tile: one row per lane
constexpr int kPolcBlock = 512;    // command elements per POLC column block

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
void launch_mvm(hipStream_t st, int dtype, const void *cm, const KBlock *kbs, int kb0, int n_kb,
                int n_rows, const float *x_pad, float *y_part);
void launch_integrate(hipStream_t st, const float *y_part, int n_kb, const float *p_part,
                      int n_pkb, int n_rows, const float *scale, float *a, float *a_pad,
                      float *out, float c1, float g);
void launch_dgemm_rd(hipStream_t st, const float *R, const double *D, double *M, int n_act,
                     int n_s);

}  // namespace rtc
