// Device building blocks shared by the per-launch kernels and the persistent
// frame loop.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rtc_internal.h"

namespace rtc {

// Global-memory view of a pointer.  Pointers that reach a kernel through a
// table in device memory (rather than as kernel arguments) are generic to the
// compiler, which then emits flat instructions; flat loads count against the
// LDS counter too, so every wait for an LDS read would also drain the matrix
// stream.  Device and pinned host buffers are all global memory.
#define RTC_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ RTC_GLOBAL T *gbl(T *p) {
    return (RTC_GLOBAL T *)p;
}
template <class T>
__device__ __forceinline__ const RTC_GLOBAL T *gbl(const T *p) {
    return (const RTC_GLOBAL T *)p;
}

// Read-only data (tables, descriptors written before the launch) in the
// constant address space: uniform loads become scalar loads, and the compiler
// may keep them across stores and atomics, which cannot alias them.
#define RTC_CONST __attribute__((address_space(4)))

// LDS, named explicitly where a pointer travels through calls the compiler
// may not inline (it would otherwise fall back to flat instructions).
#define RTC_LDS __attribute__((address_space(3)))
typedef float lds4_t __attribute__((ext_vector_type(4)));

// One entry of a read-only table, copied out a dword at a time (a struct
// cannot be copy-constructed from another address space).
template <class T>
__device__ __forceinline__ T ldc(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "table entries are dword multiples");
    const RTC_CONST uint32_t *w = (const RTC_CONST uint32_t *)p;
    uint32_t t[sizeof(T) / 4];
#pragma unroll
    for (size_t i = 0; i < sizeof(T) / 4; ++i) t[i] = w[i];
    T r;
    __builtin_memcpy(&r, t, sizeof(T));
    return r;
}
// The same for an entry each lane picks for itself (global address space).
template <class T>
__device__ __forceinline__ T ldg(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "table entries are dword multiples");
    const RTC_GLOBAL uint32_t *w = (const RTC_GLOBAL uint32_t *)p;
    uint32_t t[sizeof(T) / 4];
#pragma unroll
    for (size_t i = 0; i < sizeof(T) / 4; ++i) t[i] = w[i];
    T r;
    __builtin_memcpy(&r, t, sizeof(T));
    return r;
}

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
// Store policies for slope values: STORE_PLAIN when consumers run in later
// kernels, STORE_AGENT when wavefronts of the same kernel on other XCDs read
// them (agent-scope atomic store, written through the non-coherent L2).
enum { STORE_PLAIN = 0, STORE_AGENT = 1 };
template <int SP>
__device__ __forceinline__ void put(float *p, float v) {
    if constexpr (SP == STORE_AGENT)
        __hip_atomic_store(gbl(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *gbl(p) = v;
}

// Load policies for pixels: LOAD_PLAIN for frames in device memory written
// before the kernel started; LOAD_AGENT for the device ring that wavefronts of
// the same kernel refill while it runs (agent-scope 32-bit loads read past the
// XCD's non-coherent L2, which could otherwise return a ring slot's previous
// frame; the aligned word may include the neighbouring pixel, so rings carry
// slack after the last slot).
enum { LOAD_PLAIN = 0, LOAD_AGENT = 1 };
template <int LP>
__device__ __forceinline__ uint32_t load_px(const uint16_t *p) {
    if constexpr (LP == LOAD_AGENT) {
        const uintptr_t a = reinterpret_cast<uintptr_t>(p);
        const uint32_t *w = reinterpret_cast<const uint32_t *>(a & ~(uintptr_t)3);
        const uint32_t v = __hip_atomic_load(gbl(w), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return (a & 2) ? (v >> 16) : (v & 0xFFFFu);
    } else {
        return *gbl(p);
    }
}

struct SlopeOut {
    float *s_pad;          // padded slope vector read by the MVM
    float *s_out;          // compact slopes (nullable)
    int32_t *counts;       // thresholded pixels per unit (nullable)
    uint64_t *masks;       // thresholded-pixel masks (nullable)
    int32_t out_agent;     // s_out and counts are read while the kernel runs
};

// Compact outputs: read after the kernel, or (out_agent) copied out while it
// runs, so written through the XCD's L2 to the memory side.
template <class T>
__device__ __forceinline__ void put_out(const SlopeOut &o, T *p, T v) {
    if (o.out_agent)
        __hip_atomic_store(gbl(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *gbl(p) = v;
}

// Shack-Hartmann unit: one wavefront.  Lane l handles pixels l, l+64, ... of
// the subaperture (raster order), so the ballot of pass j is mask word j.
// Every pixel and calibration load is issued before any is used.
template <int SP, int LP = LOAD_PLAIN>
__device__ __forceinline__ void sh_unit(const ShUnit &d, float T, const uint16_t *__restrict__ fr,
                                        const WfsParam &P, const float *__restrict__ dark,
                                        const float *__restrict__ flat,
                                        const float *__restrict__ bg,
                                        const float *__restrict__ ref, const SlopeOut &o,
                                        int lane) {
    const int p = P.p;
    const int npx = p * p;
    const int mode = P.thr_mode;
    // every load is issued at once, without a condition (lanes past the
    // unit's pixels read its last pixel and drop it), so the unit costs one
    // round trip to memory; the reference slopes come with them
    uint32_t raw[kMaxShPasses];
    float dk[kMaxShPasses], fl[kMaxShPasses], bgv[kMaxShPasses];
#pragma unroll
    for (int j = 0; j < kMaxShPasses; ++j) {
        const int i = min(j * kWave + lane, npx - 1);
        const int r = i / p;
        const int c = i - r * p;
        raw[j] = load_px<LP>(fr + (size_t)(d.row0 + r) * P.W + (d.col0 + c));
        dk[j] = gbl(dark)[d.cal + i];
        fl[j] = gbl(flat)[d.cal + i];
        bgv[j] = gbl(bg)[d.cal + i];
    }
    const float rx = gbl(ref)[2 * d.unit], ry = gbl(ref)[2 * d.unit + 1];
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
        if (o.masks != nullptr && lane == 0 && j * kWave < npx) put_out(o, o.masks + d.mask + j, bal);
    }
    sw = wave_sum(sw);
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    if (lane == 0) {
        float ox = 0.0f, oy = 0.0f;
        if (sw > 0.0f) {
            ox = sx / sw - rx;
            oy = sy / sw - ry;
        }
        put<SP>(o.s_pad + d.pad, ox);
        put<SP>(o.s_pad + d.pad + 1, oy);
        if (o.s_out != nullptr) {
            put_out(o, o.s_out + 2 * d.unit, ox);
            put_out(o, o.s_out + 2 * d.unit + 1, oy);
        }
        if (o.counts != nullptr) put_out(o, o.counts + d.unit, (int32_t)cnt);
    }
}

// Pyramid unit: one lane.  Calibration arrays are [quadrant][unit] so that
// lanes read consecutive addresses.
// Calibrated, thresholded intensities of pupil pixel k in the four images
// (bit q of the return value: the pixel of image q is in the mask).
template <int LP = LOAD_PLAIN>
__device__ __forceinline__ uint64_t pyr_intensities(const PyrUnit &d, int k, int n_pyr, float T,
                                                    const uint16_t *__restrict__ fr,
                                                    const WfsParam &P,
                                                    const float *__restrict__ dark4,
                                                    const float *__restrict__ flat4,
                                                    const float *__restrict__ bg4, float (&I)[4]) {
    // every load first, so the unit costs one round trip to memory
    uint32_t raw[4];
    float dk[4], fl[4], bgv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        raw[q] = load_px<LP>(fr + (size_t)(P.qrow[q] + d.i) * P.W + (P.qcol[q] + d.j));
        dk[q] = gbl(dark4)[q * n_pyr + k];
        fl[q] = gbl(flat4)[q * n_pyr + k];
        bgv[q] = gbl(bg4)[q * n_pyr + k];
    }
    uint64_t bits = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float cv = calibrate_px((float)raw[q], dk[q], fl[q], bgv[q]);
        bool m;
        I[q] = threshold_px(cv, T, P.thr_mode, m);
        bits |= (uint64_t)m << q;
    }
    return bits;
}

// The frame's intensity sum over the pupil of pyramid sensor P by one
// wavefront, in exactly the order of k_pyr_sum's 256 threads: lane l holds the
// running sums of threads l, l + 64, l + 128, l + 192 (units t, t + 256, ... in
// order), then the same halving tree, its first two levels in registers and
// the rest across lanes.  Every lane returns the sum.
template <int LP = LOAD_PLAIN>
__device__ __forceinline__ float pyr_pupil_sum_wave(const PyrUnit *__restrict__ units, int n_pyr,
                                                    const float *__restrict__ thr,
                                                    const uint16_t *__restrict__ fr,
                                                    const WfsParam &P,
                                                    const float *__restrict__ dark4,
                                                    const float *__restrict__ flat4,
                                                    const float *__restrict__ bg4, int lane) {
    float a[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int j0 = 0; j0 < P.pn; j0 += 256) {
#pragma unroll 1
        for (int c = 0; c < 4; ++c) {
            const int j = j0 + c * kWave + lane;
            if (j < P.pn) {
                const int k = P.pu0 + j;
                const PyrUnit d = ldg(units + k);
                float I[4];
                (void)pyr_intensities<LP>(d, k, n_pyr, gbl(thr)[k], fr, P, dark4, flat4, bg4, I);
                a[c] += (I[0] + I[1]) + (I[2] + I[3]);
            }
        }
    }
    a[0] += a[2];
    a[1] += a[3];
    a[0] += a[1];
#pragma unroll
    for (int h = 32; h > 0; h >>= 1) a[0] += __shfl_down(a[0], h, kWave);
    return __shfl(a[0], 0, kWave);
}

// gS: the frame's intensity sum over the pupil (sensors with global
// normalisation; unused otherwise).
template <int SP, int LP = LOAD_PLAIN>
__device__ __forceinline__ void pyr_unit(const PyrUnit &d, int k, int n_pyr, float T,
                                         const uint16_t *__restrict__ fr, const WfsParam &P,
                                         const float *__restrict__ dark4,
                                         const float *__restrict__ flat4,
                                         const float *__restrict__ bg4,
                                         const float *__restrict__ ref, const SlopeOut &o,
                                         float gS) {
    const float rx = gbl(ref)[2 * d.unit], ry = gbl(ref)[2 * d.unit + 1];
    float I[4];
    const uint64_t bits = pyr_intensities<LP>(d, k, n_pyr, T, fr, P, dark4, flat4, bg4, I);
    const float S = P.norm == RTC_PYR_NORM_GLOBAL ? gS : (I[0] + I[1]) + (I[2] + I[3]);
    float sx = 0.0f, sy = 0.0f;
    if (S > 0.0f) {
        sx = ((I[0] + I[1]) - (I[2] + I[3])) / S - rx;
        sy = ((I[0] + I[2]) - (I[1] + I[3])) / S - ry;
    }
    put<SP>(o.s_pad + d.pad, sx);
    put<SP>(o.s_pad + d.pad + 1, sy);
    if (o.s_out != nullptr) {
        put_out(o, o.s_out + 2 * d.unit, sx);
        put_out(o, o.s_out + 2 * d.unit + 1, sy);
    }
    if (o.counts != nullptr) put_out(o, o.counts + d.unit, (int32_t)__popcll(bits));
    if (o.masks != nullptr) put_out(o, o.masks + d.mask, bits);
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

// One 16-byte matrix vector as a native vector (copyable from any address space).
typedef uint32_t vec16_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// Accumulates the E products of one 16-byte vector; xs points at the slope
// values as float4 (global memory) or lds4_t (LDS).
template <int DT, class XS>
__device__ __forceinline__ void dot16(const vec16_t q, XS xs, int v, float &a0, float &a1) {
    if constexpr (DT == RTC_CM_F32) {
        const auto s = xs[v];
        a0 = fmaf(__uint_as_float(q.x), s.x, a0);
        a1 = fmaf(__uint_as_float(q.y), s.y, a1);
        a0 = fmaf(__uint_as_float(q.z), s.z, a0);
        a1 = fmaf(__uint_as_float(q.w), s.w, a1);
    } else if constexpr (DT == RTC_CM_BF16) {
        const auto s0 = xs[2 * v];
        const auto s1 = xs[2 * v + 1];
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
            const auto s = xs[4 * v + h];
            const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[h], false);
            const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[h], true);
            a0 = fmaf(lo[0], s.x, a0);
            a1 = fmaf(lo[1], s.y, a1);
            a0 = fmaf(hi[0], s.z, a0);
            a1 = fmaf(hi[1], s.w, a1);
        }
    }
}

// Streams vectors [0, nv) of one segment for this lane's row, U vectors (U
// loads in flight) per batch; the slope values of a batch are contiguous, so
// they arrive in a few wide scalar loads issued beside the vector loads.  The
// last, partial batch guards each load instead.  NT: non-temporal loads, for
// matrices larger than the Infinity Cache (a matrix that fits stays resident
// from frame to frame with ordinary loads).
//
// REV streams the vectors from the last to the first (the partial batch
// first), accumulating in that order.  Frames alternate the direction: the
// vectors a wavefront read last in one frame are still in L2 when the next
// frame starts there.
template <int DT, int U, class XS, bool NT = false, bool REV = false>
__device__ __forceinline__ float stream_segment(const uint4 *__restrict__ pg, int nr, XS xs,
                                                int nv) {
    const RTC_GLOBAL vec16_t *__restrict__ p = (const RTC_GLOBAL vec16_t *)pg;
    float a0 = 0.0f, a1 = 0.0f;
    if constexpr (REV) {
        int v = nv - nv % U;
        if (v < nv) {
            vec16_t q[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (v + u < nv)
                    q[u] = NT ? __builtin_nontemporal_load(p + (v + u) * nr) : p[(v + u) * nr];
#pragma unroll
            for (int u = U - 1; u >= 0; --u)
                if (v + u < nv) dot16<DT>(q[u], xs, v + u, a0, a1);
        }
        while (v > 0) {
            v -= U;
            vec16_t q[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                q[u] = NT ? __builtin_nontemporal_load(p + (v + u) * nr) : p[(v + u) * nr];
#pragma unroll
            for (int u = U - 1; u >= 0; --u) dot16<DT>(q[u], xs, v + u, a0, a1);
        }
        return a0 + a1;
    }
    int v = 0;
    for (; v + U <= nv; v += U) {
        vec16_t q[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            q[u] = NT ? __builtin_nontemporal_load(p + (v + u) * nr) : p[(v + u) * nr];
#pragma unroll
        for (int u = 0; u < U; ++u) dot16<DT>(q[u], xs, v + u, a0, a1);
    }
    if (v < nv) {
        vec16_t q[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (v + u < nv)
                q[u] = NT ? __builtin_nontemporal_load(p + (v + u) * nr) : p[(v + u) * nr];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (v + u < nv) dot16<DT>(q[u], xs, v + u, a0, a1);
    }
    return a0 + a1;
}

// stream_segment with the direction chosen at run time (one copy of the loop):
// pass vector j is vector j (forward) or nv - 1 - j (backward), so the
// accumulation order equals stream_segment's or its REV form's.
template <int DT, int U, class XS>
__device__ __forceinline__ float stream_segment_dir(const uint4 *__restrict__ pg, int nr, XS xs,
                                                    int nv, bool rev) {
    const RTC_GLOBAL vec16_t *__restrict__ p = (const RTC_GLOBAL vec16_t *)pg;
    const int s = rev ? -1 : 1;
    const int c0 = rev ? nv - 1 : 0;
    float a0 = 0.0f, a1 = 0.0f;
    int j = 0;
    for (; j + U <= nv; j += U) {
        const int c = c0 + s * j;
        vec16_t q[U];
#pragma unroll
        for (int u = 0; u < U; ++u) q[u] = p[(c + s * u) * nr];
#pragma unroll
        for (int u = 0; u < U; ++u) dot16<DT>(q[u], xs, c + s * u, a0, a1);
    }
    if (j < nv) {
        const int c = c0 + s * j;
        vec16_t q[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j + u < nv) q[u] = p[(c + s * u) * nr];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j + u < nv) dot16<DT>(q[u], xs, c + s * u, a0, a1);
    }
    return a0 + a1;
}

// ---------------------------------------------------------------------------
// Double-buffered segment stream (per-launch MVM and frame loop).  The
// segment's part of a tile is one buffer resource (nv vectors of nr rows, 16
// bytes each); lane l reads row l of each vector (1 KiB contiguous per
// wavefront load).  Offsets are scalar, and a vector past the segment's end
// reads as zeros without a memory access, so every batch issues exactly U
// loads and the compiler's memory-counter waits stay exact instead of
// draining the stream.
constexpr int kBufNT = 2;      // buffer-load cache policy: non-temporal

// Batches are taken in pairs, so that no loop exit sits between a batch's
// loads and their use (the compiler would otherwise sink the prefetch past
// it).  An odd batch count ends with one batch past the end: its loads return
// zeros without touching memory and its slopes in LDS are zeros, so it adds
// exact zeros after every real product.
template <int U, bool NT>
struct SegStream {
    __amdgpu_buffer_rsrc_t rs;
    int nb, voff, vstride;
    __device__ __forceinline__ int bmap(int b) const { return (b < 0 || b >= nb) ? nb : b; }
    __device__ __forceinline__ void load(vec16_t (&q)[U], int b) const {
        const int o = bmap(b) * U * vstride;
#pragma unroll
        for (int u = 0; u < U; ++u)
            q[u] = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, o + u * vstride,
                                                         NT ? kBufNT : 0);
    }
};

// The double-buffered stream of one segment's vectors against its slopes in
// LDS (xl: padded to whole batches plus one zero batch), the first batch
// already loaded into qa.  Returns this lane's partial.
template <int DT, int U, bool NT, bool REV>
__device__ __forceinline__ float seg_stream(const SegStream<U, NT> &ss, vec16_t (&qa)[U],
                                            const RTC_LDS lds4_t *xl) {
    constexpr int step = REV ? -1 : 1;
    int b = REV ? ss.nb - 1 : 0;
    vec16_t qb[U];
    float a0 = 0.0f, a1 = 0.0f;
    auto compute = [&](const vec16_t (&q)[U], int bb) {
        const int v0 = ss.bmap(bb) * U;
        if constexpr (!REV) {
#pragma unroll
            for (int u = 0; u < U; ++u) dot16<DT>(q[u], xl, v0 + u, a0, a1);
        } else {
#pragma unroll
            for (int u = U - 1; u >= 0; --u) dot16<DT>(q[u], xl, v0 + u, a0, a1);
        }
    };
    // the scheduler barriers keep each batch's loads ahead of the previous
    // batch's products (left to itself, the scheduler sinks them to save
    // registers, which drains the stream at every batch)
    for (int i = 0; i < (ss.nb + 1) / 2; ++i) {
        ss.load(qb, b + step);
        __builtin_amdgcn_sched_barrier(0);
        compute(qa, b);
        __builtin_amdgcn_sched_barrier(0);
        ss.load(qa, b + 2 * step);
        __builtin_amdgcn_sched_barrier(0);
        compute(qb, b + step);
        __builtin_amdgcn_sched_barrier(0);
        b += 2 * step;
    }
    return a0 + a1;
}

// The partials were written by wavefronts on any XCD; agent-scope atomic loads
// read them past this XCD's (non-coherent) L2.
__device__ __forceinline__ float load_agent(const float *p) {
    return __hip_atomic_load(gbl(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block ends of a segment list as a bitmask: bit j of word j / 32 is set when
// segment j is the last of its column block.  A wavefront holds the mask in
// registers, lane l holding words l, l + 64, ... (kEndWordsPerLane of them:
// up to kMaxSegments segments, checked when an instance is built), so that a
// reduction tests block ends without a dependent memory access per block.
struct SegEnds {
    uint32_t w[kEndWordsPerLane];
};
__device__ __forceinline__ SegEnds load_seg_ends(const uint32_t *ends, int n, int lane) {
    SegEnds m;
    const int nw = (n + 31) >> 5;
#pragma unroll
    for (int k = 0; k < kEndWordsPerLane; ++k) {
        const int i = k * kWave + lane;
        m.w[k] = i < nw ? gbl(ends)[i] : 0u;
    }
    return m;
}
// Mask word wi (uniform): segments 32 wi .. 32 wi + 31.
__device__ __forceinline__ uint32_t seg_end_word(const SegEnds &m, int wi) {
    const int k = wi >> 6;
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < kEndWordsPerLane; ++i)
        if (i == k) v = (uint32_t)__builtin_amdgcn_readlane((int)m.w[i], wi & 63);
    return v;
}

// Sum of one row over a tile's column blocks, in block order, each block's
// segment partials in order: y = ((B_0 + B_1) + B_2) + ..., B_k = ((0 + p_a)
// + p_b) + ... for part[j * n_rows + r], j in [0, n), block ends from the mask.
// The partials were stored by wavefronts on any XCD: agent-coherent buffer
// loads (cache policy sc1) read them past this XCD's L2.  BATCH (a multiple of
// 32) loads are issued back to back with no condition (an index past the
// last partial reads zero from the buffer's range check), so one round trip
// to memory covers a batch.  The first batch is peeled: after its loads are
// issued, after_first() issues whatever else the caller needs from memory
// (those round trips then overlap) and returns false to abandon the sum
// (the result is then 0).  With use_y0, the fold continues from the state y0
// (read after after_first()) that earlier blocks, ending at a block end, left:
// the sum of those blocks.  r must be below n_rows.
constexpr int kBufAgent = 16;
template <int BATCH, class After>
__device__ __forceinline__ float sum_partials(const float *part, int n, int n_rows, int r,
                                              const SegEnds &ends, After &&after_first,
                                              bool use_y0 = false, const float &y0 = 0.0f) {
    static_assert(BATCH % 32 == 0, "batches cover whole mask words");
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)part, (short)0, n * n_rows * (int)sizeof(float), 0x00020000);
    float y = 0.0f, blk = 0.0f;
    bool first = true;
    float v[BATCH];
    auto load = [&](int s0) {
#pragma unroll
        for (int u = 0; u < BATCH; ++u)
            v[u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                rs, ((s0 + u) * n_rows + r) * 4, 0, kBufAgent));
    };
    auto fold = [&](int s0) {
#pragma unroll
        for (int h = 0; h < BATCH / 32; ++h) {
            const uint32_t w = seg_end_word(ends, (s0 >> 5) + h);
#pragma unroll
            for (int u = 0; u < 32; ++u) {
                const int j = s0 + 32 * h + u;
                if (j < n) {
                    blk += v[32 * h + u];
                    if ((w >> u) & 1u) {
                        y = first ? blk : y + blk;
                        first = false;
                        blk = 0.0f;
                    }
                }
            }
        }
    };
    load(0);
    if (!after_first()) return 0.0f;
    if (use_y0) {
        y = y0;
        first = false;
    }
    fold(0);
    for (int s0 = BATCH; s0 < n; s0 += BATCH) {
        load(s0);
        fold(s0);
    }
    return y;
}

}  // namespace rtc
