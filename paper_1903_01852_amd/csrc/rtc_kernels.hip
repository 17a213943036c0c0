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
//  k_mvm_next<DT>  k_mvm of frame f with, in extra workgroups of the same
//                  grid, the slopes of frame f + 1 (batch of device-resident
//                  frames: the slopes' latency hides under the MVM's stream)
//  k_dgemm_rd      one-off FP64 product M = R.D for implicit POLC
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rtc_device.h"

namespace rtc {

// ---------------------------------------------------------------------------
// Shack-Hartmann: 4 wavefronts per workgroup, one subaperture per wavefront.
__global__ __launch_bounds__(256) void k_sh_centroid(
    const ShUnit *__restrict__ units, int u0, int u1, FrameSet frames, WfsParamSet params,
    const float *__restrict__ dark, const float *__restrict__ flat,
    const float *__restrict__ bg, const float *__restrict__ thr,
    const float *__restrict__ ref, SlopeOut o) {
    const int lane = threadIdx.x & (kWave - 1);
    const int u = u0 + __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (u >= u1) return;
    const ShUnit d = units[u];
    sh_unit<STORE_PLAIN>(d, thr[u], frames.f[d.wfs], params.w[d.wfs], dark, flat, bg, ref, o,
                         lane);
}

// ---------------------------------------------------------------------------
// Pyramid: one lane per pupil pixel.
__global__ __launch_bounds__(256) void k_pyr_slopes(
    const PyrUnit *__restrict__ units, int u0, int u1, int n_pyr, FrameSet frames,
    WfsParamSet params, const float *__restrict__ dark4, const float *__restrict__ flat4,
    const float *__restrict__ bg4, const float *__restrict__ thr,
    const float *__restrict__ ref, SlopeOut o, const float *__restrict__ gsum) {
    const int k = u0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= u1) return;
    const PyrUnit d = units[k];
    const WfsParam &P = params.w[d.wfs];
    pyr_unit<STORE_PLAIN>(d, k, n_pyr, thr[k], frames.f[d.wfs], P, dark4, flat4, bg4, ref, o,
                          P.norm == RTC_PYR_NORM_GLOBAL ? gsum[d.wfs] : 0.0f);
}

// Global normalisation: the frame's intensity sum over the pupil of pyramid
// sensor wfs[blockIdx.x] (every valid pixel, its four images).  Thread t adds
// the sensor's units t, t + 256, ... in order, then a fixed halving tree in LDS
// adds the 256 partial sums: the same value on every run and path.
__global__ __launch_bounds__(256) void k_pyr_sum(const PyrUnit *__restrict__ units, int n_pyr,
                                                 FrameSet frames, WfsParamSet params,
                                                 const float *__restrict__ dark4,
                                                 const float *__restrict__ flat4,
                                                 const float *__restrict__ bg4,
                                                 const float *__restrict__ thr, WfsList wfs,
                                                 float *__restrict__ gsum) {
    __shared__ float part[256];
    const int w = wfs.w[blockIdx.x];
    const WfsParam &P = params.w[w];
    float acc = 0.0f;
    // unrolled so that several units' loads are in flight; the additions stay
    // in unit order
#pragma unroll 4
    for (int j = (int)threadIdx.x; j < P.pn; j += 256) {
        const int k = P.pu0 + j;
        const PyrUnit d = units[k];
        float I[4];
        (void)pyr_intensities(d, k, n_pyr, thr[k], frames.f[w], P, dark4, flat4, bg4, I);
        acc += (I[0] + I[1]) + (I[2] + I[3]);
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) gsum[w] = part[0];
}

// Epilogue run by the last wavefront to finish a 64-row tile (every column
// block of the tile has then written its partial):
//   EPI_INTEGRATE: a = c1 a + g (scale * sum partials + p)   (commands)
//   EPI_REDUCE:    y = sum partials                          (POLC term p)
// The sum is taken block by block in block order, each block's segments in
// order, exactly as the persistent frame loop accumulates it.
__device__ __forceinline__ void tile_epilogue(const MvmEpilogue &E, const float *__restrict__ part,
                                              int n_rows, int t, int lane, int nr) {
    const int r = t * kTileRows + lane;
    if (lane >= nr) return;
    const int2 *kb_segs = E.kb_segs;
    float y = sum_in_blocks<32>(part, E.n_parts, E.n_kb, n_rows, r, [&](int b) {
        const int2 sb = kb_segs[b];
        return sb.x + sb.y;
    });
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

// One wavefront of the split-K MVM: piece wv / n_tiles of tile wv % n_tiles.
template <int DT, int U, bool NT>
__device__ __forceinline__ void mvm_wave(int wv, int lane, const uint8_t *__restrict__ cm,
                                         const SegRun *__restrict__ runs,
                                         const Piece *__restrict__ pieces, int p0, int n_pieces,
                                         int n_tiles, int n_rows, const float *__restrict__ x,
                                         float *__restrict__ y_part, const MvmEpilogue &E) {
    if (wv >= n_pieces * n_tiles) return;
    const int pi = wv / n_tiles;
    const int t = wv - pi * n_tiles;
    const Piece P = pieces[p0 + pi];
    const int nr = min(kTileRows, n_rows - t * kTileRows);
    // odd frames run the piece backwards, segments and vectors alike
    const int rev = __builtin_amdgcn_readfirstlane(E.rev);
    for (int sgi = 0; sgi < P.nseg; ++sgi) {
        const int sg = P.seg0 + (rev ? P.nseg - 1 - sgi : sgi);
        const SegRun S = runs[sg];
        if (lane < nr) {
            const uint4 *__restrict__ p =
                reinterpret_cast<const uint4 *>(cm + S.base + (int64_t)t * kTileRows * S.kv * 16) +
                (int64_t)S.v0 * nr + lane;
            const float4 *__restrict__ xs = reinterpret_cast<const float4 *>(x + S.xoff);
            const float part = rev ? stream_segment<DT, U, const float4 *, NT, true>(p, nr, xs, S.nv)
                                   : stream_segment<DT, U, const float4 *, NT>(p, nr, xs, S.nv);
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

template <int DT, int U, bool NT>
__global__ __launch_bounds__(256) void k_mvm(const uint8_t *__restrict__ cm,
                                             const SegRun *__restrict__ runs,
                                             const Piece *__restrict__ pieces, int p0,
                                             int n_pieces, int n_tiles, int n_rows,
                                             const float *__restrict__ x,
                                             float *__restrict__ y_part, MvmEpilogue E) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    mvm_wave<DT, U, NT>(wv, lane, cm, runs, pieces, p0, n_pieces, n_tiles, n_rows, x, y_part, E);
}

// The MVM's workgroups come first, so they are dispatched first and stream
// from the start; the slope workgroups fill the remaining wavefront slots.
template <int DT, int U, bool NT>
__global__ __launch_bounds__(256) void k_mvm_next(const uint8_t *__restrict__ cm,
                                                  const SegRun *__restrict__ runs,
                                                  const Piece *__restrict__ pieces, int n_pieces,
                                                  int n_tiles, int n_rows,
                                                  const float *__restrict__ x,
                                                  float *__restrict__ y_part, MvmEpilogue E,
                                                  int mvm_blocks, NextSlopes N,
                                                  WfsParamSet params) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int blk = __builtin_amdgcn_readfirstlane(blockIdx.x);
    if (blk < mvm_blocks) {
        mvm_wave<DT, U, NT>(blk * 4 + wave, lane, cm, runs, pieces, 0, n_pieces, n_tiles, n_rows,
                            x, y_part, E);
        return;
    }
    const SlopeOut o{N.s_pad, N.s_out, N.counts, N.masks};
    const int b = blk - mvm_blocks;
    const int sh_blocks = (N.n_sh + 3) / 4;
    if (b < sh_blocks) {
        const int u = b * 4 + wave;
        if (u >= N.n_sh) return;
        const ShUnit d = N.sh[u];
        sh_unit<STORE_PLAIN>(d, N.sh_thr[u], N.frames.f[d.wfs], params.w[d.wfs], N.sh_dark,
                             N.sh_flat, N.sh_bg, N.ref, o, lane);
    } else {
        const int k = (b - sh_blocks) * 256 + (int)threadIdx.x;
        if (k >= N.n_pyr) return;
        const PyrUnit d = N.py[k];
        const WfsParam &P = params.w[d.wfs];
        pyr_unit<STORE_PLAIN>(d, k, N.n_pyr, N.py_thr[k], N.frames.f[d.wfs], P, N.py_dark,
                              N.py_flat, N.py_bg, N.ref, o,
                              P.norm == RTC_PYR_NORM_GLOBAL ? N.py_gsum[d.wfs] : 0.0f);
    }
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
    const SlopeOut o{s_pad, s_out, counts, masks};
    hipLaunchKernelGGL(k_sh_centroid, dim3((n + 3) / 4), dim3(256), 0, st, units, u0, u1,
                       frames, params, dark, flat, bg, thr, ref, o);
}

void launch_pyr_slopes(hipStream_t st, const PyrUnit *units, int u0, int u1, int n_pyr,
                       const FrameSet &frames, const WfsParamSet &params, const float *dark4,
                       const float *flat4, const float *bg4, const float *thr,
                       const float *ref, float *s_pad, float *s_out, int32_t *counts,
                       uint64_t *masks, const float *gsum) {
    const int n = u1 - u0;
    if (n <= 0) return;
    const SlopeOut o{s_pad, s_out, counts, masks};
    hipLaunchKernelGGL(k_pyr_slopes, dim3((n + 255) / 256), dim3(256), 0, st, units, u0, u1,
                       n_pyr, frames, params, dark4, flat4, bg4, thr, ref, o, gsum);
}

void launch_pyr_sum(hipStream_t st, const PyrUnit *units, int n_pyr, const FrameSet &frames,
                    const WfsParamSet &params, const float *dark4, const float *flat4,
                    const float *bg4, const float *thr, const WfsList &wfs, float *gsum) {
    if (wfs.n <= 0) return;
    hipLaunchKernelGGL(k_pyr_sum, dim3(wfs.n), dim3(256), 0, st, units, n_pyr, frames, params,
                       dark4, flat4, bg4, thr, wfs, gsum);
}

// Vectors per batch: 16 for FP32; 8 for BF16 and FP8, whose batch of slope
// values (8 or 16 per vector, read through the scalar unit) would not fit the
// scalar registers at 16 (measured: FP8 on a 302 MB matrix 87 -> 78 us cold).
template <bool NT>
void launch_mvm_t(hipStream_t st, int dtype, const uint8_t *c, const SegRun *runs,
                  const Piece *pieces, int p0, int n_pieces, int n_tiles, int n_rows,
                  const float *x_pad, float *y_part, const MvmEpilogue &epi) {
    const dim3 grid((n_pieces * n_tiles + 3) / 4), block(256);
    switch (dtype) {
    case RTC_CM_F32:
        hipLaunchKernelGGL((k_mvm<RTC_CM_F32, 16, NT>), grid, block, 0, st, c, runs, pieces, p0,
                           n_pieces, n_tiles, n_rows, x_pad, y_part, epi);
        break;
    case RTC_CM_BF16:
        hipLaunchKernelGGL((k_mvm<RTC_CM_BF16, 8, NT>), grid, block, 0, st, c, runs, pieces, p0,
                           n_pieces, n_tiles, n_rows, x_pad, y_part, epi);
        break;
    default:
        hipLaunchKernelGGL((k_mvm<RTC_CM_FP8, 8, NT>), grid, block, 0, st, c, runs, pieces, p0,
                           n_pieces, n_tiles, n_rows, x_pad, y_part, epi);
        break;
    }
}

void launch_mvm(hipStream_t st, int dtype, bool stream_nt, const void *cm, const SegRun *runs,
                const Piece *pieces, int p0, int n_pieces, int n_rows, const float *x_pad,
                float *y_part, const MvmEpilogue &epi) {
    if (n_pieces <= 0 || n_rows <= 0) return;
    const int n_tiles = (n_rows + kTileRows - 1) / kTileRows;
    const uint8_t *c = static_cast<const uint8_t *>(cm);
    if (stream_nt)
        launch_mvm_t<true>(st, dtype, c, runs, pieces, p0, n_pieces, n_tiles, n_rows, x_pad, y_part,
                           epi);
    else
        launch_mvm_t<false>(st, dtype, c, runs, pieces, p0, n_pieces, n_tiles, n_rows, x_pad,
                            y_part, epi);
}

template <bool NT>
void launch_mvm_next_t(hipStream_t st, int dtype, const uint8_t *c, const SegRun *runs,
                       const Piece *pieces, int n_pieces, int n_tiles,
                       int n_rows, const float *x_pad, float *y_part, const MvmEpilogue &epi,
                       const NextSlopes &next, const WfsParamSet &params) {
    const int mvm_blocks = (n_pieces * n_tiles + 3) / 4;
    const dim3 grid(mvm_blocks + (next.n_sh + 3) / 4 + (next.n_pyr + 255) / 256), block(256);
    switch (dtype) {
    case RTC_CM_F32:
        hipLaunchKernelGGL((k_mvm_next<RTC_CM_F32, 16, NT>), grid, block, 0, st, c, runs,
                           pieces, n_pieces, n_tiles, n_rows, x_pad, y_part, epi, mvm_blocks,
                           next, params);
        break;
    case RTC_CM_BF16:
        hipLaunchKernelGGL((k_mvm_next<RTC_CM_BF16, 8, NT>), grid, block, 0, st, c, runs,
                           pieces, n_pieces, n_tiles, n_rows, x_pad, y_part, epi, mvm_blocks,
                           next, params);
        break;
    default:
        hipLaunchKernelGGL((k_mvm_next<RTC_CM_FP8, 8, NT>), grid, block, 0, st, c, runs,
                           pieces, n_pieces, n_tiles, n_rows, x_pad, y_part, epi, mvm_blocks,
                           next, params);
        break;
    }
}

void launch_mvm_next(hipStream_t st, int dtype, bool stream_nt, const void *cm,
                     const SegRun *runs, const Piece *pieces, int n_pieces, int n_rows,
                     const float *x_pad, float *y_part, const MvmEpilogue &epi,
                     const NextSlopes &next, const WfsParamSet &params) {
    if (n_pieces <= 0 || n_rows <= 0) return;
    const int n_tiles = (n_rows + kTileRows - 1) / kTileRows;
    const uint8_t *c = static_cast<const uint8_t *>(cm);
    if (stream_nt)
        launch_mvm_next_t<true>(st, dtype, c, runs, pieces, n_pieces, n_tiles, n_rows, x_pad,
                                y_part, epi, next, params);
    else
        launch_mvm_next_t<false>(st, dtype, c, runs, pieces, n_pieces, n_tiles, n_rows, x_pad,
                                 y_part, epi, next, params);
}

void launch_dgemm_rd(hipStream_t st, const float *R, const double *D, double *M, int n_act,
                     int n_s) {
    const dim3 grid((n_act + 63) / 64, (n_act + 63) / 64);
    hipLaunchKernelGGL(k_dgemm_rd, grid, dim3(256), 0, st, R, D, M, n_act, n_s);
}

}  // namespace rtc
