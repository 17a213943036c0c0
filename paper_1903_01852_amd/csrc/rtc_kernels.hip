// gfx950 kernels of the pixel -> command path.
//
//  k_sh_centroid   calibration + threshold + centre of gravity, one wavefront
//                  per Shack-Hartmann subaperture (section 2.2)
//  k_pyr_slopes    calibration + normalised quadrant differences, one lane per
//                  pyramid pupil pixel (section 2.2)
//  k_mvm<DT>       split-K control-matrix x slope product, one wavefront per
//                  (column block, 64-row tile), one matrix row per lane,
//                  FP32 / BF16 / FP8-e4m3 storage, FP32 accumulation
//                  (section 2.3; the product is memory-bandwidth bound)
//                  The last wavefront to finish a 64-row tile sums the tile's
//                  partials in fixed block order and applies the FP8 row scale,
//                  the implicit POLC term and the leaky integrator
//                  (sections 1.1, 3.4), or forms the POLC term itself.
//  k_dgemm_rd      one-off FP64 product M = R.D for implicit POLC
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rtc_internal.h"

namespace rtc {

// Binary32 calibration, one rounding per operation: contraction into a fused
// multiply-add would change the thresholded-pixel masks.
__device__ __forceinline__ float calibrate_px(float raw, float dark, float flat, float bg) {
#pragma clang fp contract(off)
    const float t = raw - dark;
    const float u = t * flat;
    return u - bg;
}

__device__ __forceinline__ float threshold_px(float c, float thr, int mode, bool &m) {
#pragma clang fp contract(off)
    if (mode == RTC_THR_NONE) {
        m = true;
        return c;
    }
    m = c > thr;
    if (!m) return 0.0f;
    return mode == RTC_THR_SUBTRACT ? c - thr : c;
}

// Sum over the 64 lanes in a fixed order: DPP within each row of 16 lanes
// (pair swap, quad swap, half-row mirror, row mirror), then the four row
// sums in row order.  The result is uniform.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp<0xB1>(v);    // quad_perm(1,0,3,2)
    v += dpp<0x4E>(v);    // quad_perm(2,3,0,1)
    v += dpp<0x141>(v);   // row_half_mirror
    v += dpp<0x140>(v);   // row_mirror
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return ((r0 + r1) + r2) + r3;
}

// ---------------------------------------------------------------------------
// Shack-Hartmann: 4 wavefronts per workgroup, one subaperture per wavefront.
// Lane l handles pixels l, l+64, ... of the subaperture (raster order), so the
// ballot of pass j is mask word j of the subaperture.
__global__ __launch_bounds__(256) void k_sh_centroid(
    const ShUnit *__restrict__ units, int u0, int u1, FrameSet frames, WfsParamSet params,
    const float *__restrict__ dark, const float *__restrict__ flat,
    const float *__restrict__ bg, const float *__restrict__ thr,
    const float *__restrict__ ref, float *__restrict__ s_pad, float *__restrict__ s_out,
    int32_t *__restrict__ counts, uint64_t *__restrict__ masks) {
    const int lane = threadIdx.x & (kWave - 1);
    const int u = u0 + __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (u >= u1) return;
    const ShUnit d = units[u];
    const WfsParam &P = params.w[d.wfs];
    const uint16_t *__restrict__ fr = frames.f[d.wfs];
    const int p = P.p;
    const int npx = p * p;
    const float T = thr[u];
    const int mode = P.thr_mode;
    // every pixel and calibration load of the subaperture is issued before
    // any is used (at most kMaxShPasses per lane)
    uint32_t raw[kMaxShPasses];
    float dk[kMaxShPasses], fl[kMaxShPasses], bgv[kMaxShPasses];
#pragma unroll
    for (int j = 0; j < kMaxShPasses; ++j) {
        const int i = j * kWave + lane;
        raw[j] = 0;
        dk[j] = 0.0f;
        fl[j] = 0.0f;
        bgv[j] = 0.0f;
        if (i < npx) {
            const int r = i / p;
            const int c = i - r * p;
            raw[j] = fr[(size_t)(d.row0 + r) * P.W + (d.col0 + c)];
            dk[j] = dark[d.cal + i];
            fl[j] = flat[d.cal + i];
            bgv[j] = bg[d.cal + i];
        }
    }
    float sw = 0.0f, sx = 0.0f, sy = 0.0f;
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < kMaxShPasses; ++j) {
        const int i = j * kWave + lane;
        bool m = false;
        if (i < npx) {
            const int r = i / p;
            const int c = i - r * p;
            const float cv = calibrate_px((float)raw[j], dk[j], fl[j], bgv[j]);
            const float w = threshold_px(cv, T, mode, m);
            const float x = (float)c - P.half;
            const float y = (float)r - P.half;
            sw += w;
            sx = fmaf(w, x, sx);
            sy = fmaf(w, y, sy);
        }
        const uint64_t bal = __ballot(m);
        cnt += __popcll(bal);
        if (masks != nullptr && lane == 0 && j * kWave < npx) masks[d.mask + j] = bal;
    }
    sw = wave_sum(sw);
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    if (lane == 0) {
        float ox = 0.0f, oy = 0.0f;
        if (sw > 0.0f) {
            ox = sx / sw - ref[2 * d.unit];
            oy = sy / sw - ref[2 * d.unit + 1];
        }
        s_out[2 * d.unit] = ox;
        s_out[2 * d.unit + 1] = oy;
        s_pad[d.pad] = ox;
        s_pad[d.pad + 1] = oy;
        counts[d.unit] = cnt;
    }
}

// ---------------------------------------------------------------------------
// Pyramid: one lane per pupil pixel.  Calibration arrays are [quadrant][unit]
// so that lanes read consecutive addresses.
__global__ __launch_bounds__(256) void k_pyr_slopes(
    const PyrUnit *__restrict__ units, int u0, int u1, int n_pyr, FrameSet frames,
    WfsParamSet params, const float *__restrict__ dark4, const float *__restrict__ flat4,
    const float *__restrict__ bg4, const float *__restrict__ thr,
    const float *__restrict__ ref, float *__restrict__ s_pad, float *__restrict__ s_out,
    int32_t *__restrict__ counts, uint64_t *__restrict__ masks) {
    const int k = u0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= u1) return;
    const PyrUnit d = units[k];
    const WfsParam &P = params.w[d.wfs];
    const uint16_t *__restrict__ fr = frames.f[d.wfs];
    const float T = thr[k];
    float I[4];
    uint64_t bits = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float raw = (float)fr[(size_t)(P.qrow[q] + d.i) * P.W + (P.qcol[q] + d.j)];
        const float cv = calibrate_px(raw, dark4[q * n_pyr + k], flat4[q * n_pyr + k],
                                      bg4[q * n_pyr + k]);
        bool m;
        I[q] = threshold_px(cv, T, P.thr_mode, m);
        bits |= (uint64_t)m << q;
    }
    const float S = (I[0] + I[1]) + (I[2] + I[3]);
    float sx = 0.0f, sy = 0.0f;
    if (S > 0.0f) {
        sx = ((I[0] + I[1]) - (I[2] + I[3])) / S - ref[2 * d.unit];
        sy = ((I[0] + I[2]) - (I[1] + I[3])) / S - ref[2 * d.unit + 1];
    }
    s_out[2 * d.unit] = sx;
    s_out[2 * d.unit + 1] = sy;
    s_pad[d.pad] = sx;
    s_pad[d.pad + 1] = sy;
    counts[d.unit] = __popcll(bits);
    if (masks != nullptr) masks[d.mask] = bits;
}

// ---------------------------------------------------------------------------
// Split-K MVM.  Each 16-byte vector of a tile holds E consecutive columns of
// one row, so lane l streams row 64t + l while the 64 lanes of a load cover
// 1 KiB of contiguous memory.  The slope values of a vector are the same for
// every lane, so they come through the scalar unit.
template <int DT> struct Elem;
template <> struct Elem<RTC_CM_F32> { static constexpr int E = 4; };
template <> struct Elem<RTC_CM_BF16> { static constexpr int E = 8; };
template <> struct Elem<RTC_CM_FP8> { static constexpr int E = 16; };

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// Accumulates the E products of one 16-byte vector.
template <int DT>
__device__ __forceinline__ void dot16(const uint4 q, const float4 *__restrict__ xs, int v,
                                      float &a0, float &a1) {
    if constexpr (DT == RTC_CM_F32) {
        const float4 s = xs[v];
        a0 = fmaf(__uint_as_float(q.x), s.x, a0);
        a1 = fmaf(__uint_as_float(q.y), s.y, a1);
        a0 = fmaf(__uint_as_float(q.z), s.z, a0);
        a1 = fmaf(__uint_as_float(q.w), s.w, a1);
    } else if constexpr (DT == RTC_CM_BF16) {
        const float4 s0 = xs[2 * v];
        const float4 s1 = xs[2 * v + 1];
        a0 = fmaf(bf16_lo(q.x), s0.x, a0);
        a1 = fmaf(bf16_hi(q.x), s0.y, a1);
        a0 = fmaf(bf16_lo(q.y), s0.z, a0);
        a1 = fmaf(bf16_hi(q.y), s0.w, a1);
        a0 = fmaf(bf16_lo(q.z), s1.x, a0);
        a1 = fmaf(bf16_hi(q.z), s1.y, a1);
        a0 = fmaf(bf16_lo(q.w), s1.z, a0);
        a1 = fmaf(bf16_hi(q.w), s1.w, a1);
    } else {
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const float4 s = xs[4 * v + h];
            const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[h], false);
            const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[h], true);
            a0 = fmaf(lo[0], s.x, a0);
            a1 = fmaf(lo[1], s.y, a1);
            a0 = fmaf(hi[0], s.z, a0);
            a1 = fmaf(hi[1], s.w, a1);
        }
    }
}

// Sum of the n column-block partials of row r, in increasing block order.
// The partials were written by wavefronts on any XCD; agent-scope atomic loads
// read them past this XCD's (non-coherent) L2.
__device__ __forceinline__ float load_part(const float *part, size_t i) {
    return __hip_atomic_load(part + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float sum_parts(const float *__restrict__ part, int n, int n_rows,
                                          int r) {
    float y = 0.0f;
    int j = 0;
    for (; j + 8 <= n; j += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = load_part(part, (size_t)(j + u) * n_rows + r);
#pragma unroll
        for (int u = 0; u < 8; ++u) y += v[u];
    }
    for (; j < n; ++j) y += load_part(part, (size_t)j * n_rows + r);
    return y;
}

// Epilogue run by the last wavefront to finish a 64-row tile (every column
// block of the tile has then written its partial):
//   EPI_INTEGRATE: a = c1 a + g (scale * sum partials + p)   (commands)
//   EPI_REDUCE:    y = sum partials                          (POLC term p)
__device__ __forceinline__ void tile_epilogue(const MvmEpilogue &E, const float *__restrict__ part,
                                              int n_rows, int t, int lane, int nr) {
    const int r = t * kTileRows + lane;
    if (lane >= nr) return;
    float y = sum_parts(part, E.n_parts, n_rows, r);
    if (E.mode == EPI_REDUCE) {
        E.y[r] = y;
        return;
    }
    if (E.scale != nullptr) y *= E.scale[r];
    if (E.p != nullptr) y += E.p[r];
    const float an = fmaf(E.c1, E.a[r], E.g * y);
    E.a[r] = an;
    if (E.out != nullptr) E.out[r] = an;
}

// Streams vectors [0, nv) of one segment for this lane's row, U vectors (U
// loads in flight) per batch; the slope values of a batch are contiguous, so
// they arrive in a few wide scalar loads issued beside the vector loads.  The
// last, partial batch guards each load instead.
template <int DT, int U>
__device__ __forceinline__ float stream_segment(const uint4 *__restrict__ p, int nr,
                                                const float4 *__restrict__ xs, int nv) {
    float a0 = 0.0f, a1 = 0.0f;
    int v = 0;
    for (; v + U <= nv; v += U) {
        uint4 q[U];
#pragma unroll
        for (int u = 0; u < U; ++u) q[u] = p[(v + u) * nr];
#pragma unroll
        for (int u = 0; u < U; ++u) dot16<DT>(q[u], xs, v + u, a0, a1);
    }
    if (v < nv) {
        uint4 q[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (v + u < nv) q[u] = p[(v + u) * nr];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (v + u < nv) dot16<DT>(q[u], xs, v + u, a0, a1);
    }
    return a0 + a1;
}

template <int DT, int U>
__global__ __launch_bounds__(256) void k_mvm(const uint8_t *__restrict__ cm,
                                             const KBlock *__restrict__ kbs,
                                             const Segment *__restrict__ segs,
                                             const Piece *__restrict__ pieces, int p0,
                                             int n_pieces, int n_tiles, int n_rows,
                                             const float *__restrict__ x,
                                             float *__restrict__ y_part, MvmEpilogue E) {
    constexpr int kE = Elem<DT>::E;
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (wv >= n_pieces * n_tiles) return;
    const int pi = wv / n_tiles;
    const int t = wv - pi * n_tiles;
    const Piece P = pieces[p0 + pi];
    const int nr = min(kTileRows, n_rows - t * kTileRows);
    for (int sgi = 0; sgi < P.nseg; ++sgi) {
        const int sg = P.seg0 + sgi;
        const Segment S = segs[sg];
        const KBlock K = kbs[S.kb];
        if (lane < nr) {
            const uint4 *__restrict__ p =
                reinterpret_cast<const uint4 *>(cm + K.base + (int64_t)t * kTileRows * K.kv * 16) +
                (int64_t)S.v0 * nr + lane;
            const float4 *__restrict__ xs =
                reinterpret_cast<const float4 *>(x + K.spad + (int64_t)S.v0 * kE);
            const float part = stream_segment<DT, U>(p, nr, xs, S.nv);
            // agent-scope atomic store: written through to the memory side,
            // where every XCD's agent-scope loads see it
            __hip_atomic_store(y_part + (size_t)sg * n_rows + t * kTileRows + lane, part,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (E.mode == EPI_NONE) return;
    // Count this tile's partials only once their stores have completed
    // (vmcnt drained); the wavefront bringing the count to E.n_parts runs the
    // epilogue.
    // Whole-L2 release/acquire fences are avoided on purpose: every datum
    // handed between wavefronts goes through agent-scope atomics.
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    uint32_t old = 0;
    if (lane == 0)
        old = __hip_atomic_fetch_add(&E.count[t], (uint32_t)P.nseg, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
    old = __shfl(old, 0, kWave);
    if (old + (uint32_t)P.nseg != (uint32_t)E.n_parts) return;
    if (lane == 0) __hip_atomic_store(&E.count[t], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    tile_epilogue(E, y_part, n_rows, t, lane, nr);
}

// ---------------------------------------------------------------------------
// M = R.D in FP64 (R widened exactly from FP32).  64x64 output tile per
// workgroup, 4x4 per thread, k in steps of 16 through LDS; every M element is
// accumulated in increasing k order.
__global__ __launch_bounds__(256) void k_dgemm_rd(const float *__restrict__ R,
                                                  const double *__restrict__ D,
                                                  double *__restrict__ M, int n, int ns) {
    __shared__ double As[16][64 + 1];
    __shared__ double Bs[16][64 + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int row0 = blockIdx.y * 64, col0 = blockIdx.x * 64;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < ns; k0 += 16) {
        for (int idx = threadIdx.x; idx < 16 * 64; idx += 256) {
            const int kk = idx & 15, rr = idx >> 4;      // A: rows x k
            const int gr = row0 + rr, gk = k0 + kk;
            As[kk][rr] = (gr < n && gk < ns) ? (double)R[(size_t)gr * ns + gk] : 0.0;
            const int cc = idx & 63, kb = idx >> 6;      // B: k x cols
            const int gc = col0 + cc, gk2 = k0 + kb;
            Bs[kb][cc] = (gc < n && gk2 < ns) ? D[(size_t)gk2 * n + gc] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = row0 + ty * 4 + i, c = col0 + tx * 4 + j;
            if (r < n && c < n) M[(size_t)r * n + c] = acc[i][j];
        }
}

// ---------------------------------------------------------------------------
// Host launchers.
void launch_sh_centroid(hipStream_t st, const ShUnit *units, int u0, int u1,
                        const FrameSet &frames, const WfsParamSet &params, const float *dark,
                        const float *flat, const float *bg, const float *thr, const float *ref,
                        float *s_pad, float *s_out, int32_t *counts, uint64_t *masks) {
    const int n = u1 - u0;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_sh_centroid, dim3((n + 3) / 4), dim3(256), 0, st, units, u0, u1,
                       frames, params, dark, flat, bg, thr, ref, s_pad, s_out, counts, masks);
}

void launch_pyr_slopes(hipStream_t st, const PyrUnit *units, int u0, int u1, int n_pyr,
                       const FrameSet &frames, const WfsParamSet &params, const float *dark4,
                       const float *flat4, const float *bg4, const float *thr,
                       const float *ref, float *s_pad, float *s_out, int32_t *counts,
                       uint64_t *masks) {
    const int n = u1 - u0;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_pyr_slopes, dim3((n + 255) / 256), dim3(256), 0, st, units, u0, u1,
                       n_pyr, frames, params, dark4, flat4, bg4, thr, ref, s_pad, s_out,
                       counts, masks);
}

void launch_mvm(hipStream_t st, int dtype, const void *cm, const KBlock *kbs,
                const Segment *segs, const Piece *pieces, int p0, int n_pieces, int n_rows,
                const float *x_pad, float *y_part, const MvmEpilogue &epi) {
    if (n_pieces <= 0 || n_rows <= 0) return;
    const int n_tiles = (n_rows + kTileRows - 1) / kTileRows;
    const int waves = n_pieces * n_tiles;
    const dim3 grid((waves + 3) / 4), block(256);
    const uint8_t *c = static_cast<const uint8_t *>(cm);
    switch (dtype) {
    case RTC_CM_F32:
        hipLaunchKernelGGL((k_mvm<RTC_CM_F32, 16>), grid, block, 0, st, c, kbs, segs, pieces, p0,
                           n_pieces, n_tiles, n_rows, x_pad, y_part, epi);
        break;
    case RTC_CM_BF16:
        hipLaunchKernelGGL((k_mvm<RTC_CM_BF16, 16>), grid, block, 0, st, c, kbs, segs, pieces, p0,
                           n_pieces, n_tiles, n_rows, x_pad, y_part, epi);
        break;
    default:
        hipLaunchKernelGGL((k_mvm<RTC_CM_FP8, 16>), grid, block, 0, st, c, kbs, segs, pieces, p0,
                           n_pieces, n_tiles, n_rows, x_pad, y_part, epi);
        break;
    }
}

void launch_dgemm_rd(hipStream_t st, const float *R, const double *D, double *M, int n_act,
                     int n_s) {
    const dim3 grid((n_act + 63) / 64, (n_act + 63) / 64);
    hipLaunchKernelGGL(k_dgemm_rd, grid, dim3(256), 0, st, R, D, M, n_act, n_s);
}

}  // namespace rtc
