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

#include <algorithm>

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
    // every lane loads its words of the block-end mask (the test reads them
    // across lanes); lanes past a short tile read row 0's partials
    const SegEnds ends = load_seg_ends(E.seg_ends, E.n_parts, lane);
    const int r = t * kTileRows + (lane < nr ? lane : 0);
    // the integrator's operands load beside the first partials
    const bool integ = E.mode == EPI_INTEGRATE;
    float sc = 1.0f, pp = 0.0f, ap = 0.0f;
    float y = sum_partials<64>(part, E.n_parts, n_rows, r, ends, [&] {
        if (integ) {
            if (E.scale != nullptr) sc = E.scale[r];
            if (E.p != nullptr) pp = E.p[r];
            ap = E.a[r];
        }
        return true;
    });
    if (lane >= nr) return;
    if (!integ) {
        E.y[r] = y;
        return;
    }
    if (E.scale != nullptr) y *= sc;
    if (E.p != nullptr) y += pp;
    const float an = fmaf(E.c1, ap, E.g * y);
    E.a[r] = an;
    if (E.out != nullptr) E.out[r] = an;
}

// The split-K MVM.  A workgroup streams one segment (part of one column
// block) for four consecutive 64-row tiles, one tile per wavefront, one row
// per lane; the segment's slope values are staged once in LDS and read by
// every lane as broadcasts, and each wavefront streams its tile's part with
// seg_stream (double-buffered batches of U 16-byte vectors).  Odd frames
// (REV) visit the vectors last to first; the accumulation order is the frame
// loop's, so the partials equal its own bit for bit.
//
// The segment's slopes are staged by the whole workgroup (zero past its last
// vector, one zero batch beyond), with this wavefront's first matrix batch
// issued before the copy's wait, so that the two round trips overlap.
template <int DT, int U, bool NT, bool REV>
__device__ __forceinline__ float seg_partial_buf(const SegStream<U, NT> &ss, const float *x,
                                                 int nx, int n4, bool live, RTC_LDS float *lds) {
    constexpr int EL = Elem<DT>::E;
    constexpr int kStage = (((kMaxSegVectors + U - 1) / U + 1) * U * EL / 4 + 255) / 256;
    lds4_t sv[kStage];
    const lds4_t *__restrict__ xs4 = reinterpret_cast<const lds4_t *>(x);
#pragma unroll
    for (int j = 0; j < kStage; ++j) {
        const int i = j * 256 + (int)threadIdx.x;
        sv[j] = xs4[4 * i < nx ? i : 0];
    }
    vec16_t qa[U];
    ss.load(qa, REV ? ss.nb - 1 : 0);
#pragma unroll
    for (int j = 0; j < kStage; ++j) {
        const int i = j * 256 + (int)threadIdx.x;
        if (i < n4) ((RTC_LDS lds4_t *)lds)[i] = 4 * i < nx ? sv[j] : lds4_t{0.0f, 0.0f, 0.0f, 0.0f};
    }
    // LDS writes complete, then the barrier (no fence: it would also wait for
    // the matrix loads in flight)
    __builtin_amdgcn_s_waitcnt(0xC07F);       // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    if (!live) return 0.0f;
    const RTC_LDS lds4_t *xl = (const RTC_LDS lds4_t *)lds;
    return seg_stream<DT, U, NT, REV>(ss, qa, xl);
}

template <int DT, int U, bool NT>
__device__ __forceinline__ void mvm_group(int g, int wave, int lane, const uint8_t *__restrict__ cm,
                                          const SegRun *__restrict__ runs, int s0, int n_tiles,
                                          int n_rows, const float *__restrict__ x,
                                          float *__restrict__ y_part, const MvmEpilogue &E,
                                          RTC_LDS float *lds) {
    constexpr int EL = Elem<DT>::E;
    const int tgroups = (n_tiles + 3) / 4;
    const int si = g / tgroups;
    const int t = (g - si * tgroups) * 4 + wave;
    const int sg = s0 + si;
    const SegRun S = runs[sg];
    const int nb = (S.nv + U - 1) / U;
    const int n4 = (nb + 1) * U * EL / 4;      // padded slope float4s
    const int nx = S.nv * EL;                  // real slope values
    // the segment's part of tile t: nv vectors of nr rows, 16 bytes each (a
    // wavefront past the last tile gets an empty range: its loads read zeros)
    const bool live = t < n_tiles;
    const int tt = live ? t : n_tiles - 1;
    const int nr = min(kTileRows, n_rows - tt * kTileRows);
    SegStream<U, NT> ss;
    ss.rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(cm + S.base + ((int64_t)tt * kTileRows * S.kv + (int64_t)S.v0 * nr) * 16),
        (short)0, live ? S.nv * nr * 16 : 0, 0x00020000);
    ss.nb = nb;
    ss.voff = lane * 16;                      // this lane's row within a vector
    ss.vstride = nr * 16;                     // bytes between consecutive vectors
    const bool rev = __builtin_amdgcn_readfirstlane(E.rev) != 0;
    const float *xs = x + S.xoff;
    const float part = rev ? seg_partial_buf<DT, U, NT, true>(ss, xs, nx, n4, live, lds)
                           : seg_partial_buf<DT, U, NT, false>(ss, xs, nx, n4, live, lds);
    if (!live) return;
    if (lane < nr)
        __hip_atomic_store(y_part + (size_t)sg * n_rows + t * kTileRows + lane, part,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
        old = __hip_atomic_fetch_add(&E.count[t * kCountStride], 1u, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
    old = __shfl(old, 0, kWave);
    if (old + 1u != (uint32_t)E.n_parts) return;
    if (lane == 0)
        __hip_atomic_store(&E.count[t * kCountStride], 0u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    tile_epilogue(E, y_part, n_rows, t, lane, nr);
}

// Segments [s0, s0 + n) of the matrix, grid = n x ceil(n_tiles / 4).
template <int DT, int U, bool NT>
__global__ __launch_bounds__(256) void k_mvm(const uint8_t *__restrict__ cm,
                                             const SegRun *__restrict__ runs, int s0,
                                             int n_tiles, int n_rows,
                                             const float *__restrict__ x,
                                             float *__restrict__ y_part, MvmEpilogue E) {
    extern __shared__ __attribute__((aligned(16))) float lds_dyn[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    mvm_group<DT, U, NT>(__builtin_amdgcn_readfirstlane(blockIdx.x), wave, lane, cm, runs, s0,
                         n_tiles, n_rows, x, y_part, E, (RTC_LDS float *)lds_dyn);
}

// The MVM's workgroups come first, so they are dispatched first and stream
// from the start; the slope workgroups fill the remaining wavefront slots.
template <int DT, int U, bool NT>
__global__ __launch_bounds__(256) void k_mvm_next(const uint8_t *__restrict__ cm,
                                                  const SegRun *__restrict__ runs,
                                                  int n_tiles, int n_rows,
                                                  const float *__restrict__ x,
                                                  float *__restrict__ y_part, MvmEpilogue E,
                                                  int mvm_blocks, NextSlopes N,
                                                  WfsParamSet params) {
    extern __shared__ __attribute__((aligned(16))) float lds_dyn[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int blk = __builtin_amdgcn_readfirstlane(blockIdx.x);
    if (blk < mvm_blocks) {
        mvm_group<DT, U, NT>(blk, wave, lane, cm, runs, 0, n_tiles, n_rows, x, y_part, E,
                             (RTC_LDS float *)lds_dyn);
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
// Static scratch of the allocation-free batch entry point: MVM partials and
// per-tile arrival counters.  Every device the library runs on holds its own
// copy for the life of the process; host code takes its address from
// scratch_address (the name itself is a host-side stand-in, not a device
// address).
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// Fill n uint32 with v (counters that must start at zero; a kernel rather
// than a memset, so that the work can be captured in a graph).
__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *__restrict__ p, size_t n, uint32_t v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Host launchers.

hipError_t scratch_address(void **ptr) {
    return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

void launch_fill_u32(hipStream_t st, uint32_t *p, size_t n, uint32_t v) {
    if (n == 0) return;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, st, p, n, v);
}
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

// Vectors per batch (double-buffered, so twice as many 16-byte loads per lane
// in flight): 8 for every storage type.
constexpr int kMvmBatch = 8;

// LDS of an MVM workgroup: its segment's slope values, padded to whole batches
// plus one batch of zeros.
size_t mvm_lds_bytes(int dtype) {
    const int E = dtype == RTC_CM_F32 ? 4 : dtype == RTC_CM_BF16 ? 8 : 16;
    return (size_t)(((kMaxSegVectors + kMvmBatch - 1) / kMvmBatch + 1) * kMvmBatch) * E * 4;
}

template <bool NT>
void launch_mvm_t(hipStream_t st, int dtype, const uint8_t *c, const SegRun *runs, int s0,
                  int n_segs, int n_tiles, int n_rows, const float *x_pad, float *y_part,
                  const MvmEpilogue &epi) {
    const dim3 grid(n_segs * ((n_tiles + 3) / 4)), block(256);
    const size_t lds = mvm_lds_bytes(dtype);
    switch (dtype) {
    case RTC_CM_F32:
        hipLaunchKernelGGL((k_mvm<RTC_CM_F32, kMvmBatch, NT>), grid, block, lds, st, c, runs, s0,
                           n_tiles, n_rows, x_pad, y_part, epi);
        break;
    case RTC_CM_BF16:
        hipLaunchKernelGGL((k_mvm<RTC_CM_BF16, kMvmBatch, NT>), grid, block, lds, st, c, runs, s0,
                           n_tiles, n_rows, x_pad, y_part, epi);
        break;
    default:
        hipLaunchKernelGGL((k_mvm<RTC_CM_FP8, kMvmBatch, NT>), grid, block, lds, st, c, runs, s0,
                           n_tiles, n_rows, x_pad, y_part, epi);
        break;
    }
}

void launch_mvm(hipStream_t st, int dtype, bool stream_nt, const void *cm, const SegRun *runs,
                int s0, int n_segs, int n_rows, const float *x_pad, float *y_part,
                const MvmEpilogue &epi) {
    if (n_segs <= 0 || n_rows <= 0) return;
    const int n_tiles = (n_rows + kTileRows - 1) / kTileRows;
    const uint8_t *c = static_cast<const uint8_t *>(cm);
    if (stream_nt)
        launch_mvm_t<true>(st, dtype, c, runs, s0, n_segs, n_tiles, n_rows, x_pad, y_part, epi);
    else
        launch_mvm_t<false>(st, dtype, c, runs, s0, n_segs, n_tiles, n_rows, x_pad, y_part, epi);
}

template <bool NT>
void launch_mvm_next_t(hipStream_t st, int dtype, const uint8_t *c, const SegRun *runs,
                       int n_segs, int n_tiles, int n_rows, const float *x_pad, float *y_part,
                       const MvmEpilogue &epi, const NextSlopes &next,
                       const WfsParamSet &params) {
    const int mvm_blocks = n_segs * ((n_tiles + 3) / 4);
    const dim3 grid(mvm_blocks + (next.n_sh + 3) / 4 + (next.n_pyr + 255) / 256), block(256);
    const size_t lds = mvm_lds_bytes(dtype);
    switch (dtype) {
    case RTC_CM_F32:
        hipLaunchKernelGGL((k_mvm_next<RTC_CM_F32, kMvmBatch, NT>), grid, block, lds, st, c,
                           runs, n_tiles, n_rows, x_pad, y_part, epi, mvm_blocks, next, params);
        break;
    case RTC_CM_BF16:
        hipLaunchKernelGGL((k_mvm_next<RTC_CM_BF16, kMvmBatch, NT>), grid, block, lds, st, c,
                           runs, n_tiles, n_rows, x_pad, y_part, epi, mvm_blocks, next, params);
        break;
    default:
        hipLaunchKernelGGL((k_mvm_next<RTC_CM_FP8, kMvmBatch, NT>), grid, block, lds, st, c,
                           runs, n_tiles, n_rows, x_pad, y_part, epi, mvm_blocks, next, params);
        break;
    }
}

void launch_mvm_next(hipStream_t st, int dtype, bool stream_nt, const void *cm,
                     const SegRun *runs, int n_segs, int n_rows, const float *x_pad,
                     float *y_part, const MvmEpilogue &epi, const NextSlopes &next,
                     const WfsParamSet &params) {
    if (n_segs <= 0 || n_rows <= 0) return;
    const int n_tiles = (n_rows + kTileRows - 1) / kTileRows;
    const uint8_t *c = static_cast<const uint8_t *>(cm);
    if (stream_nt)
        launch_mvm_next_t<true>(st, dtype, c, runs, n_segs, n_tiles, n_rows, x_pad, y_part, epi,
                                next, params);
    else
        launch_mvm_next_t<false>(st, dtype, c, runs, n_segs, n_tiles, n_rows, x_pad, y_part,
                                 epi, next, params);
}

void launch_dgemm_rd(hipStream_t st, const float *R, const double *D, double *M, int n_act,
                     int n_s) {
    const dim3 grid((n_act + 63) / 64, (n_act + 63) / 64);
    hipLaunchKernelGGL(k_dgemm_rd, grid, dim3(256), 0, st, R, D, M, n_act, n_s);
}

}  // namespace rtc
