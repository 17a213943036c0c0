// Persistent frame loop: one resident grid runs the whole pixel -> command
// path frame after frame.
//
// Every wavefront is a worker.  A frame is a fixed sequence of readout steps
// (sensor, chunk); each step's column block carries centroid tasks and MVM
// tasks (segment x 64-row tile), spread round-robin over the instance's
// workers.  Every worker walks the same sequence, so each wait below is for
// work that comes earlier in every worker's order and is done by a resident
// wavefront: the loop cannot deadlock as long as the whole grid is resident,
// which the host guarantees by sizing the grid from the occupancy query.
//
// Frames are numbered by a sequence q.  Counters are monotonic 64-bit values,
// reset by each launch.  Up to kDepth frames are in flight (slopes, partials
// and arrival counters exist kDepth times, frame q using copy q % kDepth); a
// worker starts frame q only once frame q - kDepth has published every tile
// (the frame gate), so the frames sharing a counter or a buffer never
// overlap, and the target for frame q is ((q - first) / kDepth + 1) x (work
// per frame).  Everything one wavefront hands
// to another goes through agent-scope atomics (written through past the XCD's
// non-coherent L2), with the writer draining its stores before it counts
// them.  Counters live 256 bytes apart, and counts with many contributors go
// through striped fan-in barriers, since same-line atomics serialise.
//
// Serving instances read pixels straight from the pinned host ring; a
// sentinel wavefront per instance mirrors the host doorbells into device
// memory.  Commands go to a pinned host mailbox with system-scope stores,
// followed by the frame's sequence number (the paper's latency ends when the
// DM command is ready, section 3.1).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "rtc_device.h"

namespace rtc {

namespace {

// The instance descriptor is written before the launch and never changes
// while the loop runs, so it is read as constant memory: scalar loads that hit
// the scalar cache.  It is also volatile: the compiler then reloads a field
// where it is used instead of keeping every field it ever needs live in
// registers across the whole loop (which spills), and a reload after a store
// or an atomic stays a cheap scalar load rather than a trip to memory.  The
// kernel arguments are constant memory too.
using InstRef = volatile const RTC_CONST PersistInst &;
using ArgsRef = const RTC_CONST PersistArgs &;

// Every buffer the loop touches is global memory (device or pinned host), so
// each access goes through gbl(): see rtc_device.h.
__device__ __forceinline__ uint64_t ld_agent64(const uint64_t *p) {
    return __hip_atomic_load(gbl(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent64(uint64_t *p, uint64_t v) {
    __hip_atomic_store(gbl(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t add_agent64(uint64_t *p, uint64_t v) {
    return __hip_atomic_fetch_add(gbl(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_sys64(const uint64_t *p) {
    return __hip_atomic_load(gbl(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void st_agent(float *p, float v) {
    __hip_atomic_store(gbl(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_sys(float *p, float v) {
    __hip_atomic_store(gbl(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
// Wait until every store this wavefront issued has completed.
__device__ __forceinline__ void drain() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
__device__ __forceinline__ bool stopping(ArgsRef A) {
    return __hip_atomic_load(gbl(A.stop_dev), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}
__device__ __forceinline__ void watchdog_expired(ArgsRef A) {
    __hip_atomic_store(gbl(A.status), (uint32_t)PERSIST_WATCHDOG, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(gbl(A.stop_dev), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Spin until *ctr >= target.  False when the loop must exit (stop request or
// watchdog expiry); the stop flag and the clock are checked every 32 polls.
__device__ __forceinline__ bool wait_geq(const uint64_t *ctr, uint64_t target, ArgsRef A,
                         uint64_t limit) {
    if (ld_agent64(ctr) >= target) return true;
    const uint64_t t0 = wall_clock64();
    for (uint32_t it = 1;; ++it) {
        __builtin_amdgcn_s_sleep(1);
        if (ld_agent64(ctr) >= target) return true;
        if ((it & 31) == 0) {
            if (stopping(A)) return false;
            if (wall_clock64() - t0 > limit) {
                watchdog_expired(A);
                return false;
            }
        }
    }
}

__device__ __forceinline__ bool db_reached(uint64_t db, uint64_t q, uint64_t chunks) {
    const uint64_t dq = db >> kDbShift;
    return dq > q || (dq == q && (db & kDbChunkMask) >= chunks);
}

// Spin of a worker with nothing else to do until ok(*p) holds, checking for a
// stop request every kSpinPolls loads (false then).  The pointer and the test
// are set before the spin, so a poll costs one round trip to memory, where a
// pass of the worker's main loop (which re-reads its tables to find the next
// piece of work) costs several; and the worker does not leave the spin, so
// whatever it prepared before it (a matrix batch in flight) is still in hand
// when the word changes.
constexpr int kSpinPolls = 64;
template <class Ok>
__device__ __forceinline__ bool spin_until(const uint64_t *p, Ok ok, ArgsRef A) {
    for (;;) {
        for (int k = 0; k < kSpinPolls; ++k) {
            __builtin_amdgcn_s_sleep(1);
            if (ok(ld_agent64(p))) return true;
        }
        if (stopping(A)) return false;
    }
}


// Timeline record (rtc_trace_enable): this wavefront's events of one frame.
struct Trace {
    uint64_t *rec = nullptr;        // null when not recorded
    __device__ __forceinline__ void stamp(int ev, int lane) const {
        if (rec != nullptr && lane == 0) gbl(rec)[ev] = wall_clock64();
    }
};

// Arrivals counted on a parity counter after frame q: the launch resets the
// counters, so frames q, q - 2, ... down to the launch's first frame.
__device__ __forceinline__ uint64_t par_target(InstRef I, uint64_t q, uint64_t per_frame) {
    return ((q - I.q_begin) / kDepth + 1) * per_frame;
}
// Copy of the slope/partial buffers and arrival counters frame q uses.
__device__ __forceinline__ int dslot(uint64_t q) {
    return (int)(q % kDepth);
}

// Counter i of an array of counter slots.
__device__ __forceinline__ uint64_t *slot(uint64_t *base, size_t i) {
    return base + i * kCtrSlot;
}

// Fan-in barrier `key` (of n_keys) used by frame q: kFanStripes stripe slots,
// the top slot, then the done flag.
__device__ __forceinline__ uint64_t *fan_grp(uint64_t *base, uint64_t q, int n_keys, int key) {
    return slot(base, ((size_t)dslot(q) * n_keys + key) * kFanSlots);
}
__device__ __forceinline__ uint64_t *fan_top(uint64_t *grp) {
    return slot(grp, kFanStripes);
}
// Waiters poll a word that no arrival updates: loads of a counter that atomics
// are updating at the same time delay those atomics (measured: the last of 32
// stripe arrivals at the top took 3 us with some 300 wavefronts polling it,
// where atomics on one word alone serialise at about 13 ns each).  The arrival
// that completes the barrier stores q + 1 here once its atomic has returned.
__device__ __forceinline__ uint64_t *fan_flag(uint64_t *grp) {
    return slot(grp, kFanStripes + 1);
}
__device__ __forceinline__ bool fan_done(uint64_t *grp, uint64_t q) {
    return ld_agent64(fan_flag(grp)) >= q + 1;
}
// Top count once frame q has passed a barrier of n tasks.
__device__ __forceinline__ uint64_t fan_target(InstRef I, uint64_t q, int n) {
    return par_target(I, q, (uint64_t)min(n, kFanStripes));
}
// Count this wavefront's tasks of frame q on a barrier of n tasks: lane
// s < kFanStripes holds in cnt how many of its tasks j have j % kFanStripes
// == s (a stripe's quota is the number of such j below n).  The wavefront's
// stores must be drained.  True, on every lane, for the arrival that
// completes the barrier.
__device__ __forceinline__ bool fan_arrive(InstRef I, uint64_t *grp, uint64_t q, int n, uint32_t cnt, int lane) {
    bool done = false;
    if (cnt != 0) {
        const uint64_t quota = (uint64_t)((n - lane + kFanStripes - 1) / kFanStripes);
        const uint64_t old = add_agent64(slot(grp, lane), cnt);
        if (old + cnt == par_target(I, q, quota)) {
            done = add_agent64(fan_top(grp), 1) + 1 == fan_target(I, q, n);
            if (done) st_agent64(fan_flag(grp), q + 1);
        }
    }
    return __any(done);
}
// The lane holding task j's stripe count.
__device__ __forceinline__ bool stripe_lane(int j, int lane) {
    return lane == (int)((unsigned)j % kFanStripes);
}

// Tiles of frame q whose commands are out: one counter (a frame has at most a
// few hundred tiles, and they arrive over microseconds), so the last tile
// publishes after a single atomic.
__device__ __forceinline__ uint64_t *tiles_out(InstRef I, uint64_t q) {
    return fan_top(fan_grp(I.tile_fan, q, 1, 0));
}
__device__ __forceinline__ uint64_t tiles_target(InstRef I, uint64_t q) {
    return par_target(I, q, (uint64_t)I.n_tiles);
}
// Raised by the last tile of frame q: waiters poll it, not the count.
__device__ __forceinline__ uint64_t *tiles_flag(InstRef I, uint64_t q) {
    return fan_flag(fan_grp(I.tile_fan, q, 1, 0));
}

// First task index of this worker among n tasks whose task 0 goes to `base`.
__device__ __forceinline__ int first_task(int rank, int nw, int base) {
    int j = (rank - base) % nw;
    return j < 0 ? j + nw : j;
}
// Round-robin start of frame q's tasks of one kind (n_all per frame): frame q
// continues where frame q - 1 ended, so the workers holding one task more than
// the others change from frame to frame.
__device__ __forceinline__ int rot(uint64_t q, int n_all, int nw) {
    return (int)(((q % (uint64_t)nw) * (uint64_t)n_all) % (uint64_t)nw);
}

__device__ __forceinline__ const uint16_t *frame_src(InstRef I, int w, uint64_t q) {
    if (I.serving) return I.src[w] + (int64_t)(q % (uint64_t)I.ring_depth) * I.src_stride[w];
    return I.src[w] + (int64_t)(q - I.q_begin) * I.src_stride[w];
}

// Commands of frame q live in buffer q & 1: frame q reads buffer (q - 1) & 1
// while the POLC product of frame q - 1 may still be reading it.
__device__ __forceinline__ float *a_buf(InstRef I, uint64_t q) {
    return I.a + (q & 1) * (uint64_t)I.a_stride;
}

__device__ __forceinline__ int vec_elems(int dtype) {
    return dtype == RTC_CM_F32 ? 4 : dtype == RTC_CM_BF16 ? 8 : 16;
}

// MVM task of the loop: segment S of column block K on tile t for this
// wavefront, with the double-buffered stream of the per-launch MVM
// (seg_stream, batches of kLoopBatch vectors).  The segment's slopes, written
// by other wavefronts of this kernel during the frame, are staged in this
// wavefront's LDS slice with agent-scope 16-byte buffer loads (a value past
// the segment reads as zero, which pads the slice to whole batches plus a
// zero batch); the first matrix batch is issued before the copy's wait so the
// two round trips overlap.  rev streams the vectors last to first.
constexpr int kLoopBatch = 8;
constexpr int kLoopLdsFloats = ((kMaxSegVectors + kLoopBatch - 1) / kLoopBatch + 1) * kLoopBatch * 16;
template <int DT, bool REV>
__device__ __forceinline__ float loop_task(const uint8_t *cm, const KBlock &K, const Segment &S,
                                           int t, int nr, int lane, const float *xs,
                                           RTC_LDS float *lds) {
    constexpr int EL = Elem<DT>::E, U = kLoopBatch;
    constexpr int kPer = (kLoopLdsFloats / 4 + kWave - 1) / kWave;
    const int nb = (S.nv + U - 1) / U;
    const int n4 = (nb + 1) * U * EL / 4;
    const __amdgpu_buffer_rsrc_t rx =
        __builtin_amdgcn_make_buffer_rsrc((void *)xs, (short)0, S.nv * EL * 4, 0x00020000);
    lds4_t sv[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = j * kWave + lane;
        const vec16_t w = __builtin_amdgcn_raw_buffer_load_b128(rx, i * 16, 0, kBufAgent);
        sv[j] = lds4_t{__uint_as_float(w.x), __uint_as_float(w.y), __uint_as_float(w.z),
                       __uint_as_float(w.w)};
    }
    SegStream<U, false> ss;
    ss.rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(cm + K.base + ((int64_t)t * kTileRows * K.kv + (int64_t)S.v0 * nr) * 16),
        (short)0, S.nv * nr * 16, 0x00020000);
    ss.nb = nb;
    ss.voff = lane * 16;
    ss.vstride = nr * 16;
    vec16_t qa[U];
    ss.load(qa, REV ? nb - 1 : 0);
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = j * kWave + lane;
        if (i < n4) ((RTC_LDS lds4_t *)lds)[i] = sv[j];
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);       // lgkmcnt(0): this wavefront's LDS writes done
    __builtin_amdgcn_wave_barrier();
    return seg_stream<DT, U, false, REV>(ss, qa, (const RTC_LDS lds4_t *)lds);
}

// Partial of segment S on tile t for this lane's row (rows past the tile read
// as zero rows and are not stored): storage type at run time, direction by
// frame parity (odd frames backwards, as the per-launch kernels).
__device__ __forceinline__ float seg_partial(InstRef I, int ms, uint64_t q, const KBlock &K,
                                             const Segment &S, int t, int nr, int lane,
                                             const float *xs, RTC_LDS float *lds) {
    const uint8_t *cm = I.cm[ms];   // read from the descriptor at use: no registers held
    const bool rev = (q & 1) != 0;
    switch (I.dtype) {
    case RTC_CM_F32:
        return rev ? loop_task<RTC_CM_F32, true>(cm, K, S, t, nr, lane, xs, lds)
                   : loop_task<RTC_CM_F32, false>(cm, K, S, t, nr, lane, xs, lds);
    case RTC_CM_BF16:
        return rev ? loop_task<RTC_CM_BF16, true>(cm, K, S, t, nr, lane, xs, lds)
                   : loop_task<RTC_CM_BF16, false>(cm, K, S, t, nr, lane, xs, lds);
    default:
        return rev ? loop_task<RTC_CM_FP8, true>(cm, K, S, t, nr, lane, xs, lds)
                   : loop_task<RTC_CM_FP8, false>(cm, K, S, t, nr, lane, xs, lds);
    }
}

// Matrix slot of frame q: its reconstruction matrix and FP8 scales, and the
// POLC matrix applied to its commands (forming frame q + 1's POLC term).
// Serving reads the device mirror of
// the host's switch word, which the sentinel refreshes before it mirrors any
// doorbell that follows a swap.
__device__ __forceinline__ int mat_slot(InstRef I, uint64_t q) {
    if (I.serving) {
        const ParamBlock *pb = I.param_mirror;
        const uint64_t w = ld_agent64(&pb->mword);
        const int s = (int)(w & 1);
        return q >= (w >> 1) ? s : 1 - s;
    }
    return q >= I.coef.q_mswitch ? I.coef.mslot[1] : I.coef.mslot[0];
}

// A serving worker's MVM task that may wait for its block's slopes: the first
// matrix batch is in flight before the wait (its matrix slot read then is
// right unless a swap settles during the wait: the slot is read again after
// it and the batch reissued if it changed), so the wait ends into the slope
// copy alone.  ok is false, with nothing computed, when ready() is; ms is the
// frame's matrix slot.
template <int DT, bool REV, class Ready>
__device__ __forceinline__ float loop_task_early(InstRef I, uint64_t q, const KBlock &K,
                                                 const Segment &S, int t, int nr, int lane,
                                                 const float *xs, RTC_LDS float *lds, Ready ready,
                                                 bool &ok, int &ms) {
    constexpr int EL = Elem<DT>::E, U = kLoopBatch;
    constexpr int kPer = (kLoopLdsFloats / 4 + kWave - 1) / kWave;
    const int nb = (S.nv + U - 1) / U;
    const int n4 = (nb + 1) * U * EL / 4;
    const int64_t off = K.base + ((int64_t)t * kTileRows * K.kv + (int64_t)S.v0 * nr) * 16;
    const int ms0 = mat_slot(I, q);
    SegStream<U, false> ss;
    ss.rs = __builtin_amdgcn_make_buffer_rsrc((void *)(I.cm[ms0] + off), (short)0,
                                              S.nv * nr * 16, 0x00020000);
    ss.nb = nb;
    ss.voff = lane * 16;
    ss.vstride = nr * 16;
    vec16_t qa[U];
    ss.load(qa, REV ? nb - 1 : 0);
    if (!ready()) {
        ok = false;
        return 0.0f;
    }
    ms = mat_slot(I, q);
    const __amdgpu_buffer_rsrc_t rx =
        __builtin_amdgcn_make_buffer_rsrc((void *)xs, (short)0, S.nv * EL * 4, 0x00020000);
    lds4_t sv[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = j * kWave + lane;
        const vec16_t w = __builtin_amdgcn_raw_buffer_load_b128(rx, i * 16, 0, kBufAgent);
        sv[j] = lds4_t{__uint_as_float(w.x), __uint_as_float(w.y), __uint_as_float(w.z),
                       __uint_as_float(w.w)};
    }
    if (ms != ms0) {   // a matrix swap took effect with this frame
        ss.rs = __builtin_amdgcn_make_buffer_rsrc((void *)(I.cm[ms] + off), (short)0,
                                                  S.nv * nr * 16, 0x00020000);
        ss.load(qa, REV ? nb - 1 : 0);
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = j * kWave + lane;
        if (i < n4) ((RTC_LDS lds4_t *)lds)[i] = sv[j];
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);       // lgkmcnt(0): this wavefront's LDS writes done
    __builtin_amdgcn_wave_barrier();
    return seg_stream<DT, U, false, REV>(ss, qa, (const RTC_LDS lds4_t *)lds);
}
template <class Ready>
__device__ __forceinline__ float seg_partial_early(InstRef I, uint64_t q, const KBlock &K,
                                                   const Segment &S, int t, int nr, int lane,
                                                   const float *xs, RTC_LDS float *lds,
                                                   Ready ready, bool &ok, int &ms) {
    const bool rev = (q & 1) != 0;
    switch (I.dtype) {
    case RTC_CM_F32:
        return rev ? loop_task_early<RTC_CM_F32, true>(I, q, K, S, t, nr, lane, xs, lds, ready, ok, ms)
                   : loop_task_early<RTC_CM_F32, false>(I, q, K, S, t, nr, lane, xs, lds, ready, ok, ms);
    case RTC_CM_BF16:
        return rev ? loop_task_early<RTC_CM_BF16, true>(I, q, K, S, t, nr, lane, xs, lds, ready, ok, ms)
                   : loop_task_early<RTC_CM_BF16, false>(I, q, K, S, t, nr, lane, xs, lds, ready, ok, ms);
    default:
        return rev ? loop_task_early<RTC_CM_FP8, true>(I, q, K, S, t, nr, lane, xs, lds, ready, ok, ms)
                   : loop_task_early<RTC_CM_FP8, false>(I, q, K, S, t, nr, lane, xs, lds, ready, ok, ms);
    }
}

// Telemetry: frame q is recorded when q is a multiple of the decimation, in
// ring slot (q / decimation) mod slots (both powers of two).
__device__ __forceinline__ bool tel_frame(InstRef I, uint64_t q) {
    return I.tel_ring != nullptr && (q & ((1ull << I.tel_dshift) - 1)) == 0;
}
// The record of frame q (slopes first).
__device__ __forceinline__ float *tel_rec(InstRef I, uint64_t q) {
    return I.tel_ring + ((q >> I.tel_dshift) & (uint64_t)I.tel_smask) * (uint64_t)I.tel_rec;
}

// Frame coefficients for frame q of a batch launch (serving reads them from
// the device mirror of the parameter block, with the row's other operands).
__device__ __forceinline__ void frame_coef(InstRef I, uint64_t q, float &c1, float &g) {
    const int s = q >= I.coef.q_switch ? 1 : 0;
    c1 = I.coef.c1[s];
    g = I.coef.g[s];
}

// ---------------------------------------------------------------------------
// Sentinel of a serving instance: mirror the host doorbells, parameters and
// drop marks into device memory, stamp each frame's last chunk, relay a stop
// request.
__device__ __forceinline__ void sentinel(InstRef I, ArgsRef A, int lane) {
    const int nw = I.n_wfs;
    int nch = 0;          // lane w: chunks per frame of sensor w
    for (int st = 0; st < I.n_steps; ++st) {
        const Step S = ldc(I.steps + st);
        if (S.wfs == lane) nch = max(nch, S.chunk + 1);
    }
    uint64_t last = ~0ull;
    uint64_t last_word = ~0ull, last_mword = ~0ull;
    uint64_t last_drop = ~0ull;
    uint64_t seen_q = I.q_begin;   // next frame whose last chunk has not been stamped
    uint64_t t_change = wall_clock64();
    // One poll of the host words, the doorbells first: parameters are read
    // after the doorbells and mirrored before them, so a doorbell seen here
    // was rung after any parameter change it follows; drop marks likewise (the
    // host writes a frame's mark before the doorbells that complete it).
    uint64_t db_n = 0, word_n = 0, mword_n = 0, dm_n = 0;
    const auto poll = [&] {
        if (lane < nw) db_n = ld_sys64(I.doorbell + lane);
        word_n = ld_sys64(&I.params->word);
        mword_n = ld_sys64(&I.params->mword);
        if (lane < I.ring_depth) dm_n = ld_sys64(I.drop_host + lane);
    };
    poll();
    for (uint32_t it = 0;; ++it) {
        // the next poll is in flight while this one is processed: a read
        // across PCIe takes about a microsecond, and two in flight halve the
        // time from a doorbell's store to its being seen
        const uint64_t db = db_n, word = word_n, mword = mword_n, dm = dm_n;
        poll();
        // mirror stores of this pass that a doorbell mirrored after them must
        // follow (the wait for them also waits for the poll in flight, so it
        // is taken only when there are any)
        bool mirrored = false;
        if (word != last_word || mword != last_mword) {
            if (lane < 2) {
                const float c1 = __hip_atomic_load(gbl(&I.params->c1[lane]), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_SYSTEM);
                const float g = __hip_atomic_load(gbl(&I.params->g[lane]), __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(gbl(&I.param_mirror->c1[lane]), c1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(gbl(&I.param_mirror->g[lane]), g, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            drain();
            if (lane == 0) {
                st_agent64(&I.param_mirror->word, word);
                st_agent64(&I.param_mirror->mword, mword);
            }
            last_word = word;
            last_mword = mword;
            mirrored = true;
        }
        const bool drop_changed = lane < I.ring_depth && dm != last_drop;
        if (drop_changed) {
            st_agent64(I.drop_mirror + lane, dm);
            last_drop = dm;
        }
        mirrored = mirrored || __any(drop_changed);
        const bool changed = lane < nw && db != last;
        if (__any(changed)) {
            if (mirrored) drain();
            if (changed) st_agent64(I.db_mirror + lane, db);
            last = db;
            t_change = wall_clock64();
        }
        // stamp frame seen_q once every sensor has delivered all its chunks
        const bool ok = lane >= nw || db_reached(db, seen_q, (uint64_t)nch);
        if (__all(ok)) {
            if (lane == 0) {
                FrameTel *tel = I.tel + (seen_q % (uint64_t)I.ring_depth);
                __hip_atomic_store(gbl(&tel->ticks_last_chunk), wall_clock64(), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
            }
            ++seen_q;
        }
        if ((it & 15) == 0) {
            const uint32_t stop = __hip_atomic_load(gbl(A.stop_host), __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_SYSTEM);
            // A serving loop idle for longer than the idle limit ends the kernel
            // (the host relaunches it on demand), but only between frames: no
            // chunk of the next frame delivered, every delivered frame
            // published and its POLC term formed.
            bool quiet = wall_clock64() - t_change > A.idle_watchdog;
            if (quiet) {
                const bool none = lane >= nw || !db_reached(db, seen_q, 1);
                const uint64_t na = (uint64_t)min(I.n_tiles, kFanStripes);
                uint64_t pub = 0, pol = 0;
                for (int k = 0; k < kDepth; ++k) {
                    pub += ld_agent64(tiles_out(I, k));
                    pol += ld_agent64(fan_top(fan_grp(I.pol_fan, k, 1, 0)));
                }
                const uint64_t nf = seen_q - I.q_begin;   // counters start at the launch
                quiet = __all(none) && pub == nf * (uint64_t)I.n_tiles &&
                        (!I.polc || pol == nf * na);
            }
            if (stop != 0 || quiet) {
                __hip_atomic_store(gbl(A.stop_dev), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
            // a frame left half delivered for much longer still ends the loop,
            // as an error, so that no wavefront outlives an abandoned engine
            if (wall_clock64() - t_change > 6 * A.idle_watchdog) {
                watchdog_expired(A);
                return;
            }
            if (stopping(A)) return;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// ---------------------------------------------------------------------------
// Accumulation as a join.  A tile's commands for frame q need (E) its
// reconstruction sum, (A) the tile's commands of frame q - 1 (the integrator
// reads them, and frames must be integrated in order) and, with POLC, (P) its
// POLC term.  Each party adds one to the tile's join counter; the party that
// completes the count does the work, so nobody waits, and then arrives as the
// (A) party of the next frame.  Join counters exist kDepth times like the
// arrival counters; the launch pre-counts the (A) and (P) parts of its first
// frame.
//
// The sum is over the column blocks in readout order, each block's segment
// partials in order: y = ((B_0 + B_1) + B_2) + ... with B_k = ((0 + p_0) + p_1)
// + ...  Batch has every partial at once, so the wavefront completing a tile's
// partials is its (E) party and sums them in one pass.  Serving gets blocks
// over the readout: the last partial of block k on a tile forms B_k at once
// (blocks in parallel, whatever their order of arrival), and the wavefront
// completing the tile's block sums is its (E) party and adds them in order.
__device__ __forceinline__ uint64_t join_need(InstRef I) {
    return I.polc ? 3 : 2;
}
__device__ __forceinline__ uint64_t *join_ctr(InstRef I, uint64_t q, int t) {
    return slot(I.join, (size_t)dslot(q) * I.n_tiles + t);
}
// True when this wavefront's arrival completes the join of (q, t).
__device__ __forceinline__ bool join(InstRef I, uint64_t q, int t, int lane) {
    uint64_t old = 0;
    if (lane == 0) old = add_agent64(join_ctr(I, q, t), 1);
    old = __shfl(old, 0, kWave);
    return (old + 1) % join_need(I) == 0;
}

// Operands of row r's commands for frame q other than its reconstruction sum.
// The frame's coefficients, FP8 row scale and drop mark are settled before
// any wavefront starts the frame, so they may be loaded early (beside the
// sum); the previous commands and the POLC term come from the join's other
// parties and are loaded only once the join is complete.  Every load of a
// group is issued before any of its values is used, so a group costs one
// round trip to memory.
struct RowOps {
    float c1, g, scale, p, aprev;
    bool dropped;
    uint64_t a_free;   // POLC: tasks of frame q - 2 done reading the tile's columns
};
struct RowRaw {
    uint64_t word, mword, drop, a_free;
    float c1s[2], gs[2], scs[2];
};
// With POLC, the tile's commands of frame q overwrite those of frame q - 2,
// which the POLC tasks of frame q - 2 on the tile's columns (one segment: a
// POLC block is one segment and a whole number of tiles) may still read.
static_assert(kPolcBlock / 4 <= kMaxSegVectors && kPolcBlock % kTileRows == 0,
              "a tile's columns lie in one POLC segment");
__device__ __forceinline__ uint64_t *a_free_ctr(InstRef I, uint64_t q, int t) {
    return slot(I.pol_seg, (size_t)dslot(q) * I.n_segm + t * kTileRows / kPolcBlock);
}
__device__ __forceinline__ void row_ops_issue(InstRef I, uint64_t q, int r, RowRaw &w) {
    // descriptor fields first (scalar loads), then the vector loads
    const bool serving = I.serving != 0, polc = I.polc != 0, fp8 = I.dtype == RTC_CM_FP8;
    const ParamBlock *pb = I.param_mirror;
    const uint64_t *dm = I.drop_mirror + (q % (uint64_t)I.ring_depth);
    const float *sc0 = I.scale[0], *sc1 = I.scale[1];
    w = RowRaw{};
    w.a_free = ~0ull;
    if (polc && q >= I.q_begin + 2) w.a_free = ld_agent64(a_free_ctr(I, q - 2, r / kTileRows));
    if (serving) {
        w.word = ld_agent64(&pb->word);
        w.mword = ld_agent64(&pb->mword);
        for (int k = 0; k < 2; ++k) {
            w.c1s[k] = __hip_atomic_load(gbl(&pb->c1[k]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            w.gs[k] = __hip_atomic_load(gbl(&pb->g[k]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        w.drop = ld_agent64(dm);
    }
    if (fp8) {
        w.scs[0] = gbl(sc0)[r];
        w.scs[1] = gbl(sc1)[r];
    }
}
// Ties the loaded values to this point of the program: the compiler would
// otherwise move cheap uses (a comparison) up to the loads, and the wait for
// them ahead of the group's later memory operations.
__device__ __forceinline__ void pin_raw(RowRaw &w) {
    asm volatile("" : "+v"(w.word), "+v"(w.mword), "+v"(w.drop), "+v"(w.a_free));
    asm volatile("" : "+v"(w.c1s[0]), "+v"(w.c1s[1]), "+v"(w.gs[0]), "+v"(w.gs[1]),
                 "+v"(w.scs[0]), "+v"(w.scs[1]));
}
// The early operands from their loaded values (the word of a parameter or
// matrix switch: frames from q_switch = word >> 1 on use slot word & 1).
__device__ __forceinline__ void row_ops_early(InstRef I, uint64_t q, const RowRaw &w, RowOps &o) {
    o.a_free = w.a_free;
    o.scale = 1.0f;
    if (I.serving) {
        // the device mirror of the parameter block: the sentinel refreshes it
        // before it mirrors any doorbell that follows a host change, and this
        // frame's doorbells have been seen (so both slots may be read with the
        // word rather than after it)
        const int s = q >= (w.word >> 1) ? (int)(w.word & 1) : 1 - (int)(w.word & 1);
        o.c1 = s ? w.c1s[1] : w.c1s[0];
        o.g = s ? w.gs[1] : w.gs[0];
        o.dropped = w.drop == q + 1;
        const int ms = q >= (w.mword >> 1) ? (int)(w.mword & 1) : 1 - (int)(w.mword & 1);
        if (I.dtype == RTC_CM_FP8) o.scale = ms ? w.scs[1] : w.scs[0];
    } else {
        frame_coef(I, q, o.c1, o.g);
        o.dropped = false;
        if (I.dtype == RTC_CM_FP8) o.scale = mat_slot(I, q) ? w.scs[1] : w.scs[0];
    }
}
__device__ __forceinline__ void row_ops_joined(InstRef I, uint64_t q, int r, RowOps &o) {
    o.p = I.polc ? load_agent(I.p + r) : 0.0f;
    o.aprev = load_agent(a_buf(I, q ^ 1) + r);   // buffer of frame q - 1
}

// Commands of tile t for frame q from the reconstruction sum y of row r: the
// FP8 row scale, the POLC term and the leaky integrator (a dropped serving
// frame keeps the previous commands), then publication.
__device__ __forceinline__ void tile_commands(InstRef I, ArgsRef A, uint64_t q, int t, int r,
                                              bool row, float y, const RowOps &o, int lane,
                                              const Trace &tr) {
    if (o.a_free != ~0ull && o.a_free < par_target(I, q - 2, (uint64_t)I.n_tiles) &&
        !wait_geq(a_free_ctr(I, q - 2, t), par_target(I, q - 2, (uint64_t)I.n_tiles), A,
                  A.dep_watchdog))
        return;
    if (row) {
        if (I.dtype == RTC_CM_FP8) y *= o.scale;
        if (I.polc) y += o.p;
        const float an = o.dropped ? o.aprev : fmaf(o.c1, o.aprev, o.g * y);
        st_agent(a_buf(I, q) + r, an);
        if (I.serving) {
            st_sys(I.mail + (size_t)(q % (uint64_t)I.ring_depth) * I.n_act + r, an);
            if (tel_frame(I, q)) st_agent(tel_rec(I, q) + I.n_slopes + I.n_units + r, an);
        }
        else if (I.cmds_out != nullptr)
            gbl(I.cmds_out)[(size_t)(q - I.q_begin) * I.n_act + r] = an;
    }
    drain();
    tr.stamp(RTC_TRACE_CMDS, lane);
    if (lane == 0 && I.serving)   // the tile's commands are in the mailbox
        __hip_atomic_store(gbl(I.tile_host + t), q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (lane == 0) st_agent64(slot(I.tile_pub, t), q + 1);
    if (lane == 0 && add_agent64(tiles_out(I, q), 1) + 1 == tiles_target(I, q)) {
        st_agent64(tiles_flag(I, q), q + 1);
        if (I.serving) {
            FrameTel *tel = I.tel + (q % (uint64_t)I.ring_depth);
            __hip_atomic_store(gbl(&tel->ticks_publish), wall_clock64(), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(gbl(I.cmd_seq), q + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// The tile's reconstruction sum for row r: its segment partials of the frame,
// block by block in readout order, the block ends from the mask (every lane
// holds its words; r of lanes past a short tile is clamped).  The head blocks'
// part is the prefix formed once they were complete (fold_head); the tail's
// partials continue the fold from it.  The row's other operands are loaded
// with the first partials.
constexpr int kSumBatch = 32;
__device__ __forceinline__ const float *tail_part(InstRef I, uint64_t q) {
    return I.y_part[dslot(q)] + (size_t)I.n_head * I.n_act;
}
__device__ __forceinline__ const float *pre_of(InstRef I, uint64_t q, int r) {
    return I.pre + (size_t)dslot(q) * I.n_act + r;
}
// Tail partials and the prefix of a tile's count (the prefix is one arrival).
__device__ __forceinline__ uint64_t tile_need(InstRef I) {
    return (uint64_t)(I.n_seg - I.n_head + (I.n_head > 0 ? 1 : 0));
}
__device__ __forceinline__ float tile_sum(InstRef I, uint64_t q, int r, const SegEnds &ends,
                                          RowOps &o) {
    const bool has_pre = I.n_head > 0;
    float pre = 0.0f;
    return sum_partials<kSumBatch>(tail_part(I, q), I.n_seg - I.n_head, I.n_act, r, ends, [&] {
        RowRaw w;
        row_ops_issue(I, q, r, w);
        if (has_pre) pre = load_agent(pre_of(I, q, r));
        row_ops_joined(I, q, r, o);
        pin_raw(w);
        row_ops_early(I, q, w, o);
        return true;
    }, has_pre, pre);
}

// The head's part of tile t's sum for frame q, once all its partials are
// stored: the fold's state after the head blocks, for the tail to continue.
__device__ __forceinline__ void fold_head(InstRef I, uint64_t q, int t, int lane) {
    const int nr = min(kTileRows, I.n_act - t * kTileRows);
    const int rc = t * kTileRows + (lane < nr ? lane : 0);
    const SegEnds ends = load_seg_ends(I.seg_ends, I.n_head, lane);
    const float y = sum_partials<kSumBatch>(I.y_part[dslot(q)], I.n_head, I.n_act, rc, ends,
                                            [] { return true; });
    if (lane < nr) st_agent(I.pre + (size_t)dslot(q) * I.n_act + rc, y);
    drain();
}

// Commands of tile t for frame q from its sum y, then of every following frame
// whose join this completes.  Returns the number of frames done.
__device__ __forceinline__ int finish_chain(InstRef I, ArgsRef A, uint64_t q, int t, int lane,
                                            const Trace &tr, float y, const RowOps &o0,
                                            const SegEnds &ends) {
    const int nr = min(kTileRows, I.n_act - t * kTileRows);
    const int r = t * kTileRows + lane;
    const int rc = t * kTileRows + (lane < nr ? lane : 0);
    tile_commands(I, A, q, t, r, lane < nr, y, o0, lane, tr);
    for (int done = 1;; ++done) {
        ++q;
        if (q >= I.q_end || !join(I, q, t, lane)) return done;
        RowOps o;
        y = tile_sum(I, q, rc, ends, o);
        tile_commands(I, A, q, t, r, lane < nr, y, o, lane, tr);
    }
}

// The accumulation a completed join starts, stamped into the frame's record.
__device__ __forceinline__ void accumulate(InstRef I, ArgsRef A, uint64_t q, int t, int lane,
                                           Trace &tr) {
    const int nr = min(kTileRows, I.n_act - t * kTileRows);
    const int rc = t * kTileRows + (lane < nr ? lane : 0);
    const SegEnds ends = load_seg_ends(I.tail_ends, I.n_seg - I.n_head, lane);
    RowOps o;
    const float y = tile_sum(I, q, rc, ends, o);
    (void)finish_chain(I, A, q, t, lane, tr, y, o, ends);
    tr.stamp(RTC_TRACE_ACCUM, lane);
}

// The (E) party of (q, t), whose partials are all stored (its arrival saw
// every partial's count): the first batch of the sum and the early row
// operands are issued with the join's atomic, so those round trips overlap;
// the sum is abandoned when the join is not complete (its last party does
// the work), else the operands the other parties wrote follow.
__device__ __forceinline__ void tile_ready(InstRef I, ArgsRef A, uint64_t q, int t, int lane,
                                           Trace &tr) {
    const int nr = min(kTileRows, I.n_act - t * kTileRows);
    const int rc = t * kTileRows + (lane < nr ? lane : 0);
    const SegEnds ends = load_seg_ends(I.tail_ends, I.n_seg - I.n_head, lane);
    const bool has_pre = I.n_head > 0;
    float pre = 0.0f;
    RowOps o;
    bool joined = false;
    const float y = sum_partials<kSumBatch>(tail_part(I, q), I.n_seg - I.n_head, I.n_act, rc, ends, [&] {
        RowRaw w;
        row_ops_issue(I, q, rc, w);
        if (has_pre) pre = load_agent(pre_of(I, q, rc));
        joined = join(I, q, t, lane);   // waits for the group
        tr.stamp(RTC_TRACE_JOINED, lane);
        pin_raw(w);
        if (!joined) return false;
        row_ops_joined(I, q, rc, o);
        row_ops_early(I, q, w, o);
        return true;
    }, has_pre, pre);
    if (!joined) return;
    tr.stamp(RTC_TRACE_SUMMED, lane);
    (void)finish_chain(I, A, q, t, lane, tr, y, o, ends);
    tr.stamp(RTC_TRACE_ACCUM, lane);
}

// Spin until tiles [t0, t1] (fewer than kWave of them) and tile tr have
// written their commands of frame q: lane i < kWave - 1 polls tile t0 + i,
// the last lane tile tr, so the pollers of a frame's POLC tasks spread over
// the tiles' flags instead of one counter that the tiles' own arrivals update.
static_assert(kMaxSegVectors * 4 / kTileRows + 1 < kWave, "a POLC segment spans few tiles");
__device__ __forceinline__ bool wait_tiles(InstRef I, ArgsRef A, uint64_t q, int t0, int t1,
                                           int tr, int lane) {
    const int t = lane == kWave - 1 ? tr : t0 + lane;
    bool ok = (lane < kWave - 1 && t > t1) || ld_agent64(slot(I.tile_pub, t)) >= q + 1;
    if (__all(ok)) return true;
    const uint64_t c0 = wall_clock64();
    for (uint32_t it = 1;; ++it) {
        __builtin_amdgcn_s_sleep(2);
        ok = ok || ld_agent64(slot(I.tile_pub, t)) >= q + 1;
        if (__all(ok)) return true;
        if ((it & 31) == 0) {
            if (stopping(A)) return false;
            if (wall_clock64() - c0 > A.dep_watchdog) {
                watchdog_expired(A);
                return false;
            }
        }
    }
}

// POLC term of frame q + 1: p = M a_q, partials per POLC segment, reduced by
// the wavefront completing a tile.
__device__ __forceinline__ bool polc_tasks(InstRef I, ArgsRef A, uint64_t q, int rank,
                           int nw, int lane, RTC_LDS float *lds, Trace &tr) {
    const int n_tasks = I.n_segm * I.n_tiles;
    int j = first_task(rank, nw, rot(q, n_tasks, nw));
    if (j >= n_tasks) return true;
    const float *aq = a_buf(I, q);
    float *part = I.p_part[dslot(q)];
    for (; j < n_tasks; j += nw) {
        const int sg = j / I.n_tiles;
        const int t = j - sg * I.n_tiles;
        const Segment S = ldc(I.segm + sg);
        const KBlock K = ldc(I.kbm + S.kb);
        const int nr = min(kTileRows, I.n_act - t * kTileRows);
        // the segment's commands of frame q (its tiles published), and tile
        // t's own: its commands of frame q have read p, which this task's
        // reduction may overwrite with the next frame's term
        const int c0 = K.k0 + S.v0 * 4;
        if (!wait_tiles(I, A, q, c0 / kTileRows, (min(c0 + S.nv * 4, I.n_act) - 1) / kTileRows, t,
                        lane))
            return false;
        // the POLC matrix of frame q's slot (the product completes frame q),
        // read once frame q has published commands: a worker with no task of
        // the frame may reach this before the frame's chunks, and a matrix
        // swap, have arrived
        const int ms = mat_slot(I, q);
        const float v = loop_task<RTC_CM_F32, false>(I.M[ms], K, S, t, nr, lane,
                                                     aq + K.spad + S.v0 * 4, lds);
        // p_part copy of frame q is free once frame q - kDepth's term of the tile
        // is reduced
        if (q >= I.q_begin + kDepth &&
            !wait_geq(slot(I.p_done, t), q - kDepth + 1, A, A.dep_watchdog))
            return false;
        if (lane < nr) st_agent(part + (size_t)sg * I.n_act + t * kTileRows + lane, v);
        drain();
        uint64_t old = 0;
        if (lane == 0) {
            add_agent64(slot(I.pol_seg, (size_t)dslot(q) * I.n_segm + sg), 1);   // a_q read
            old = add_agent64(slot(I.pol_cnt, (size_t)dslot(q) * I.n_tiles + t), 1);
        }
        old = __shfl(old, 0, kWave);
        if (old + 1 != par_target(I, q, (uint64_t)I.n_segm)) continue;
        const SegEnds ends = load_seg_ends(I.segm_ends, I.n_segm, lane);
        const int r = t * kTileRows + (lane < nr ? lane : 0);
        const float y = sum_partials<kSumBatch>(part, I.n_segm, I.n_act, r, ends, [] { return true; });
        if (lane < nr) st_agent(I.p + r, y);
        drain();
        if (lane == 0) st_agent64(slot(I.p_done, t), q + 1);
        const bool all = fan_arrive(I, fan_grp(I.pol_fan, q, 1, 0), q, I.n_tiles,
                                    stripe_lane(t, lane) ? 1u : 0u, lane);
        if (all && I.serving && lane == 0)
            __hip_atomic_store(gbl(I.pol_seq), q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        // (P) party of frame q + 1 on this tile
        if (q + 1 < I.q_end && join(I, q + 1, t, lane)) accumulate(I, A, q + 1, t, lane, tr);
    }
    return true;
}

// This worker's first task of each kind in frame q, as an index into the
// frame's whole list of that kind (every block; blocks hold consecutive
// ranges in readout order).  Its later tasks follow nw apart, so a worker walks
// its tasks with one running index and no division.
struct FrameTasks {
    int cen, mvm;
};
__device__ __forceinline__ FrameTasks frame_tasks(InstRef I, uint64_t q, int rank, int nw) {
    FrameTasks f;
    f.cen = first_task(rank, nw, rot(q, I.n_cen_all, nw));
    f.mvm = first_task(rank, nw, rot(q, I.n_seg * I.n_tiles, nw));
    return f;
}

// Centroid tasks of this worker in column block W of frame q: the running
// index j (into the frame's task list) advances past the block.  Lane s
// accumulates in cnt this worker's tasks on stripe s, counting tasks by their
// frame index (global_idx: one barrier for the frame) or their block index.
// ready() is asked, once the sensor's parameters and the first Shack-Hartmann
// task's descriptor are in registers, whether the block's pixels have arrived
// (a serving worker may wait for them there); false returns false with no task
// done.
template <class Ready>
__device__ __forceinline__ bool centroid_tasks(InstRef I, uint64_t q, const KbWork &W, int nw,
                                               int lane, const SlopeOut &so, bool global_idx,
                                               int &j, uint32_t &cnt, Ready ready) {
    const int end = W.cen_base + W.n_cen;
    if (j >= end) return true;
    const uint16_t *fr = frame_src(I, W.wfs, q);
    WfsParam P = ldc(I.wp + W.wfs);
    P.W = I.src_pitch[W.wfs];            // row pitch of the frame source
    const int j0 = j;
    ShUnit d0{};
    float thr0 = 0.0f;
    if (W.kind == RTC_WFS_SH) {
        const int u = W.cu0 + (j0 - W.cen_base);
        d0 = ldc(I.sh + u);
        thr0 = gbl(I.sh_thr)[u];
    }
    // the scalar reads above complete before the wait (the pixel addresses
    // depend on them anyway): a worker that waited then finds them in hand
    // rather than in a cache its neighbours have since refilled
    asm volatile("" ::"s"(fr), "s"(P.p), "s"(P.W), "s"(P.thr_mode), "s"(P.half), "s"(d0.row0),
                 "s"(d0.col0), "s"(d0.cal), "s"(d0.pad));
    if (!ready()) return false;
    // global normalisation: the sensor's one block waits for its whole frame,
    // and each wavefront forms the pupil sum itself (no cross-wavefront
    // dependency), in the per-launch path's order
    float gS = 0.0f;
    if (W.kind == RTC_WFS_PYR && P.norm == RTC_PYR_NORM_GLOBAL) {
        if (I.serving)
            gS = pyr_pupil_sum_wave<LOAD_AGENT>(I.py, I.n_pyr, I.py_thr, fr, P, I.py_dark,
                                                I.py_flat, I.py_bg, lane);
        else
            gS = pyr_pupil_sum_wave<LOAD_PLAIN>(I.py, I.n_pyr, I.py_thr, fr, P, I.py_dark,
                                                I.py_flat, I.py_bg, lane);
    }
    for (; j < end; j += nw) {
        const int jc = j - W.cen_base;
        if (stripe_lane(global_idx ? j : jc, lane)) ++cnt;
        if (W.kind == RTC_WFS_SH) {
            const int u = W.cu0 + jc;
            const bool first = j == j0;
            const ShUnit d = first ? d0 : ldc(I.sh + u);
            const float thr = first ? thr0 : gbl(I.sh_thr)[u];
            if (I.serving)
                sh_unit<STORE_AGENT, LOAD_AGENT>(d, thr, fr, P, I.sh_dark, I.sh_flat, I.sh_bg,
                                                  I.ref, so, lane);
            else
                sh_unit<STORE_AGENT, LOAD_PLAIN>(d, thr, fr, P, I.sh_dark, I.sh_flat, I.sh_bg,
                                                 I.ref, so, lane);
        } else {
            const int k = W.cu0 + jc * kWave + lane;
            if (k < W.cu1) {
                const PyrUnit d = ldg(I.py + k);
                if (I.serving)
                    pyr_unit<STORE_AGENT, LOAD_AGENT>(d, k, I.n_pyr, gbl(I.py_thr)[k], fr, P,
                                                       I.py_dark, I.py_flat, I.py_bg, I.ref, so,
                                                       gS);
                else
                    pyr_unit<STORE_AGENT, LOAD_PLAIN>(d, k, I.n_pyr, gbl(I.py_thr)[k], fr, P,
                                                      I.py_dark, I.py_flat, I.py_bg, I.ref, so,
                                                      gS);
            }
        }
    }
    return true;
}

// MVM tasks (segment x tile) of this worker in column block kb of frame q.
// Each task counts on its tile's counter; the arrival completing the tile's
// partials of the frame (every segment of every block) is the tile's (E)
// party.  ready() is asked, once the block's and the first task's segment
// descriptors are in registers (EARLY: and the first task's first matrix
// batch is in flight), whether the block's slopes are complete (a serving
// worker may wait for them there); false returns false with no task done.
// The matrix slot is settled only after it: the swap word of a frame that has
// not yet arrived may be stale.
template <bool EARLY, class Ready>
__device__ __forceinline__ bool mvm_tasks(InstRef I, ArgsRef A, uint64_t q, const KbWork &W, int kb,
                                          int nw, int lane, RTC_LDS float *lds, int &m, Trace &tr,
                                          int budget, Ready ready) {
    const int n_tiles = I.n_tiles;
    const int end = W.mvm_base + W.nseg * n_tiles;
    if (m >= end) return true;
    const KBlock K = ldc(I.kbs + kb);
    const int m0 = m;
    const int sg0 = W.seg0 + (m0 - W.mvm_base) / n_tiles;
    const Segment S0 = ldc(I.segs + sg0);
    asm volatile("" ::"s"(K.base), "s"(K.kv), "s"(K.spad), "s"(S0.v0), "s"(S0.nv));
    const auto rdy = [&] {
        if (!ready()) return false;
        if (tr.rec != nullptr && lane == 0 && gbl(tr.rec)[RTC_TRACE_MVM_FIRST] == 0)
            gbl(tr.rec)[RTC_TRACE_MVM_FIRST] = wall_clock64();
        return true;
    };
    const float *spad = I.s_pad[dslot(q)];
    const int E = vec_elems(I.dtype);
    int ms = 0;
    float v0 = 0.0f;                     // EARLY: the first task's partial
    if constexpr (EARLY) {
        const int t0 = (m0 - W.mvm_base) - (sg0 - W.seg0) * n_tiles;
        const int nr0 = min(kTileRows, I.n_act - t0 * kTileRows);
        bool ok = true;
        v0 = seg_partial_early(I, q, K, S0, t0, nr0, lane, spad + K.spad + S0.v0 * E, lds, rdy,
                               ok, ms);
        if (!ok) return false;
    } else {
        if (!rdy()) return false;
        ms = mat_slot(I, q);
    }
    for (; m < end && budget > 0; m += nw, --budget) {
        const int jm = m - W.mvm_base;
        const int sl = jm / n_tiles;
        const int t = jm - sl * n_tiles;
        const int sg = W.seg0 + sl;
        const Segment Sg = m == m0 ? S0 : ldc(I.segs + sg);
        const int nr = min(kTileRows, I.n_act - t * kTileRows);
        const float v = (EARLY && m == m0)
                            ? v0
                            : seg_partial(I, ms, q, K, Sg, t, nr, lane, spad + K.spad + Sg.v0 * E, lds);
        if (lane < nr) st_agent(I.y_part[dslot(q)] + (size_t)sg * I.n_act + t * kTileRows + lane, v);
        drain();
        uint64_t old = 0;
        if (sg < I.n_head) {
            // a head partial: the arrival completing the tile's head folds it
            if (lane == 0) old = add_agent64(slot(I.head_cnt, (size_t)dslot(q) * n_tiles + t), 1);
            old = __shfl(old, 0, kWave);
            if (old + 1 != par_target(I, q, (uint64_t)I.n_head)) continue;
            fold_head(I, q, t, lane);
        }
        if (lane == 0) old = add_agent64(slot(I.tile_cnt, (size_t)dslot(q) * n_tiles + t), 1);
        old = __shfl(old, 0, kWave);
        if (old + 1 != par_target(I, q, tile_need(I))) continue;
        // (E) party: the tile's reconstruction sum is ready
        tr.stamp(RTC_TRACE_TILE_READY, lane);
        tile_ready(I, A, q, t, lane, tr);
    }
    tr.stamp(RTC_TRACE_MVM_LAST, lane);
    return true;
}

// This wavefront's timeline record of frame q, if recorded.
__device__ __forceinline__ Trace trace_of(InstRef I, ArgsRef A, uint64_t q, int wid) {
    Trace tr;
    if (A.trace != nullptr && q - I.q_begin < (uint64_t)A.trace_frames)
        tr.rec = A.trace + ((q - I.q_begin) * (uint64_t)A.n_waves + (uint64_t)wid) *
                               RTC_TRACE_EVENTS;
    return tr;
}
__device__ __forceinline__ void trace_end(Trace &tr, int lane) {
    tr.stamp(RTC_TRACE_FRAME_END, lane);
}

// Frame gate: frame q reuses the buffers and counters of frame q - kDepth.
__device__ __forceinline__ bool gate(InstRef I, ArgsRef A, uint64_t q) {
    return q < I.q_begin + kDepth ||
           wait_geq(tiles_flag(I, q), q - kDepth + 1, A, A.dep_watchdog);
}

// Serving ingest: copy this worker's pieces of readout step `st` (frame q)
// from the pinned host ring into the device ring, then count them.  Loads are
// 16-byte system-coherent buffer loads (the host refills ring slots while the
// loop runs, and per-pixel loads across PCIe are limited by the request rate,
// not the bytes); stores are 16-byte agent-coherent, so wavefronts on any XCD
// read the new frame.  Buffer accesses are range-checked against each ring.
constexpr int kIngestPerLane = kIngestUnits / kWave;
static_assert(kIngestPerLane * kWave == kIngestUnits, "a piece is whole loads of the wavefront");
static_assert(kTelUnits % (4 * kWave) == 0, "a telemetry task is whole rounds of four loads");
// Ingest count of readout step st of frame q, and its done flag.
__device__ __forceinline__ uint64_t *ing_ctr(InstRef I, uint64_t q, int st) {
    return slot(I.ing_cnt, (size_t)dslot(q) * I.n_steps + st);
}
__device__ __forceinline__ uint64_t *ing_flag(InstRef I, uint64_t q, int st) {
    return slot(I.ing_cnt, ((size_t)kDepth + dslot(q)) * I.n_steps + st);
}
__device__ __forceinline__ void ingest_tasks(InstRef I, uint64_t q, const Step &S, int st, int nw, int lane,
                             int &j) {
    const int end = S.ing0 + S.ing_n;
    if (j >= end) return;
    const int w = S.wfs;
    // both buffers span exactly the step's units of this frame's ring slot:
    // every access is issued without a condition (no branch, so the loads stay
    // in flight together and each store waits for its own load only), and the
    // range check drops a last piece's units past the step
    const uint64_t off =
        ((q % (uint64_t)I.ring_depth) * (uint64_t)I.src_stride[w] / 8 + (uint64_t)S.u0) * 16;
    const int nbytes = S.n16 * 16;
    __amdgpu_buffer_rsrc_t hsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)((const uint8_t *)I.ring_host[w] + off), (short)0, nbytes, 0x00020000);
    __amdgpu_buffer_rsrc_t ddst = __builtin_amdgcn_make_buffer_rsrc(
        (void *)((const uint8_t *)I.src[w] + off), (short)0, nbytes, 0x00020000);
    constexpr int kSys = 1 | 16, kAgent = 16;   // cache policy: sc0 sc1, sc1
    uint64_t cnt = 0;
    for (; j < end; j += nw, ++cnt) {
        const int u0 = (j - S.ing0) * kIngestUnits;
        vec16_t v[kIngestPerLane];
#pragma unroll
        for (int k = 0; k < kIngestPerLane; ++k)
            v[k] = __builtin_amdgcn_raw_buffer_load_b128(hsrc, (u0 + k * kWave + lane) * 16, 0, kSys);
#pragma unroll
        for (int k = 0; k < kIngestPerLane; ++k)
            __builtin_amdgcn_raw_buffer_store_b128(v[k], ddst, (u0 + k * kWave + lane) * 16, 0, kAgent);
    }
    drain();
    // the arrival completing the step's count raises its flag (the slope
    // workers poll the flag, not the counter)
    if (lane == 0 &&
        add_agent64(ing_ctr(I, q, st), cnt) + cnt == par_target(I, q, (uint64_t)S.ing_n))
        st_agent64(ing_flag(I, q, st), q + 1);
}

// Telemetry copy of recorded frame q: once the frame is published, task j
// copies 16-byte units [j kTelUnits, (j + 1) kTelUnits) of its record from the
// device ring to the pinned host ring (agent-coherent loads, system-coherent
// stores), then sets its flag.  Off the frame's latency path.
__device__ __forceinline__ bool tel_copy_tasks(InstRef I, ArgsRef A, uint64_t q, int rank, int nw, int lane) {
    const int n16 = I.tel_rec / 4;
    const int n_tasks = (n16 + kTelUnits - 1) / kTelUnits;
    int j = first_task(rank, nw, rot(q, n_tasks, nw));
    if (j >= n_tasks) return true;
    if (!wait_geq(tiles_flag(I, q), q + 1, A, A.dep_watchdog))
        return false;
    const uint64_t ts = (q >> I.tel_dshift) & (uint64_t)I.tel_smask;
    const int bytes = n16 * 16;
    __amdgpu_buffer_rsrc_t src = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(I.tel_ring + ts * (uint64_t)I.tel_rec), (short)0, bytes, 0x00020000);
    __amdgpu_buffer_rsrc_t dst = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(I.tel_host + ts * (uint64_t)I.tel_rec), (short)0, bytes, 0x00020000);
    constexpr int kSys = 1 | 16, kAgent = 16;   // cache policy: sc0 sc1, sc1
    for (; j < n_tasks; j += nw) {
        const int u1 = min(n16, (j + 1) * kTelUnits);
        // a unit past u1 lies past the record (tasks cover whole multiples of
        // 4 kWave units), so the buffers' range checks drop it
        for (int u0 = j * kTelUnits; u0 < u1; u0 += 4 * kWave) {
            vec16_t v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                v[k] = __builtin_amdgcn_raw_buffer_load_b128(src, (u0 + k * kWave + lane) * 16, 0,
                                                             kAgent);
#pragma unroll
            for (int k = 0; k < 4; ++k)
                __builtin_amdgcn_raw_buffer_store_b128(v[k], dst, (u0 + k * kWave + lane) * 16, 0,
                                                       kSys);
        }
        drain();
        if (lane == 0)
            __hip_atomic_store(gbl(I.tel_flags + ts * kTelMaxTasks + j), q + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
    }
    return true;
}

// Serving worker: a small scheduler over the frame's readout steps with one
// cursor per kind of work, in priority order.  Ingest: copy its pieces of
// every chunk whose doorbell has rung.  Slopes: form its slopes of every step
// whose chunks (this one and all before it, as a unit's rows may span two
// chunks) are in device memory; they feed the blocks' barriers, which every
// worker's MVM tasks wait for.  MVM: run one task of the oldest block whose
// barrier has completed, then look again.  It never blocks on a barrier while
// earlier-stage work is available, so no worker holds up a block that others
// wait on, and the steps of a frame (about a hundred for six laser guide
// stars) pipeline instead of queueing behind each other.
// Serving worker roles: which kinds of work a worker takes, and its rank
// among the workers of each kind (its tasks of a kind are every n-th of the
// frame's, starting at its rank).
struct Roles {
    bool ing, cen, mvm;
    int ing_rank, ing_n, cen_rank, cen_n, mvm_rank, mvm_n;
};
constexpr int kSplitMinWorkers = 1024;   // smaller instances keep one group
constexpr int kIngestWorkers = 32;       // ingest-only workers of a split instance
constexpr int kSlopeShare = 4;           // 1 / kSlopeShare of the rest take the slopes
// The slopes of column block kb of frame q are all stored; a worker with only
// products to form (spin) waits for them in a bounded spin.
__device__ __forceinline__ bool block_ready(InstRef I, ArgsRef A, uint64_t q, const KbWork &W,
                                            int kb, bool spin) {
    uint64_t *grp = fan_grp(I.cen_fan, q, I.n_kb, kb);
    if (W.n_cen == 0 || fan_done(grp, q)) return true;   // (no arrival without slope tasks)
    return spin && spin_until(fan_flag(grp), [&](uint64_t v) { return v >= q + 1; }, A);
}

__device__ __forceinline__ void serving_worker(InstRef I, ArgsRef A, int wid, int rank, int nw, int lane,
                               RTC_LDS float *lds) {
    // With many workers, three groups: a few take only the ingest, a quarter of
    // the rest the slopes, the others the products.  No ingest or slope worker
    // is then inside a longer task when a chunk's pixels land, so the frame's
    // last chunk is copied and its slopes start as soon as their turn comes.
    // A smaller instance keeps one group (its last block's products need
    // every worker).  POLC and telemetry copies (after publication) go to
    // every worker.
    Roles ro;
    if (nw < kSplitMinWorkers) {
        ro = Roles{true, true, true, rank, nw, rank, nw, rank, nw};
    } else {
        const int ni = kIngestWorkers, nc = (nw - ni) / kSlopeShare;
        if (rank < ni)
            ro = Roles{true, false, false, rank, ni, 0, 1, 0, 1};
        else if (rank < ni + nc)   // with no ingest-only workers, the slope group ingests
            ro = Roles{ni == 0, true, false, rank - ni, nc, rank - ni, nc, 0, 1};
        else
            ro = Roles{false, false, true, 0, 1, 0, 1, rank - ni - nc, nw - ni - nc};
    }
    // a worker of a single kind waits for its next piece of work in a spin
    const bool ingest_only = ro.ing && !ro.cen && !ro.mvm;
    const bool slopes_only = ro.cen && !ro.ing && !ro.mvm;
    const bool mvm_only = ro.mvm && !ro.ing && !ro.cen;
    for (uint64_t q = I.q_begin; q < I.q_end; ++q) {
        if (stopping(A)) return;
        Trace tr = trace_of(I, A, q, wid);
        tr.stamp(RTC_TRACE_FRAME_START, lane);
        if (!gate(I, A, q)) return;
        tr.stamp(RTC_TRACE_GATE, lane);
        SlopeOut so{I.s_pad[dslot(q)], nullptr, nullptr, nullptr, 1};
        if (tel_frame(I, q)) {
            so.s_out = tel_rec(I, q);
            so.counts = reinterpret_cast<int32_t *>(so.s_out + I.n_slopes);
            so.masks = reinterpret_cast<uint64_t *>(so.s_out + I.tel_mask_off);
        }
        FrameTasks ft;
        ft.cen = first_task(ro.cen_rank, ro.cen_n, rot(q, I.n_cen_all, ro.cen_n));
        ft.mvm = first_task(ro.mvm_rank, ro.mvm_n, rot(q, I.n_seg * I.n_tiles, ro.mvm_n));
        int ing = first_task(ro.ing_rank, ro.ing_n, rot(q, I.n_ing_all, ro.ing_n));
        const int n_steps = I.n_steps, n_tiles = I.n_tiles;
        // next step to ingest, known ingested, slopes, MVM (a group skips the others')
        int is = ro.ing ? 0 : n_steps, ic = 0, cs = ro.cen ? 0 : n_steps,
            ms = ro.mvm ? 0 : n_steps;
        uint32_t idle = 0;
        bool last_seen = false;   // an MVM task of the frame's last block started
        while (is < n_steps || cs < n_steps || ms < n_steps) {
            bool progressed = false;
            // ingest of every delivered chunk
            while (is < n_steps) {
                const Step S = ldc(I.steps + is);
                if (ing < S.ing0 + S.ing_n) {
                    const uint64_t *db = I.db_mirror + S.wfs;
                    const uint64_t want = (uint64_t)S.chunk + 1;
                    if (!db_reached(ld_agent64(db), q, want) &&
                        !(ingest_only &&
                          spin_until(db, [&](uint64_t v) { return db_reached(v, q, want); }, A)))
                        break;
                    tr.stamp(RTC_TRACE_INGEST_START, lane);
                    ingest_tasks(I, q, S, is, ro.ing_n, lane, ing);
                    tr.stamp(RTC_TRACE_INGEST, lane);
                    progressed = true;
                }
                ++is;
            }
            // slopes of every step whose chunks are all in device memory
            while (cs < n_steps) {
                const Step S = ldc(I.steps + cs);
                if (S.kb < 0) {
                    ++cs;
                    continue;
                }
                const KbWork W = ldc(I.kbw + S.kb);
                if (ft.cen < W.cen_base + W.n_cen) {
                    // every step up to this one copied into device memory
                    const auto ingested = [&] {
                        while (ic <= cs) {
                            // (a step with no pixel units has nothing to count)
                            const uint64_t *flag = ing_flag(I, q, ic);
                            if (ldc(I.steps + ic).ing_n > 0 && ld_agent64(flag) < q + 1 &&
                                !(slopes_only &&
                                  spin_until(flag, [&](uint64_t v) { return v >= q + 1; }, A)))
                                return false;
                            ++ic;
                        }
                        tr.stamp(RTC_TRACE_CEN_START, lane);
                        return true;
                    };
                    uint32_t cnt = 0;
                    if (!centroid_tasks(I, q, W, ro.cen_n, lane, so, false, ft.cen, cnt, ingested))
                        break;
                    drain();
                    (void)fan_arrive(I, fan_grp(I.cen_fan, q, I.n_kb, S.kb), q, W.n_cen, cnt,
                                     lane);
                    tr.stamp(RTC_TRACE_CENTROIDS, lane);
                    progressed = true;
                }
                ++cs;
            }
            // one MVM task of the oldest block with this worker's tasks left
            while (ms < n_steps) {
                const Step S = ldc(I.steps + ms);
                if (S.kb < 0) {
                    ++ms;
                    continue;
                }
                const KbWork W = ldc(I.kbw + S.kb);
                const int end = W.mvm_base + W.nseg * n_tiles;
                if (ft.mvm >= end) {
                    ++ms;
                    continue;
                }
                const auto slopes_in = [&] {
                    if (!block_ready(I, A, q, W, S.kb, mvm_only)) return false;
                    if (S.kb == I.n_kb - 1 && !last_seen) {
                        tr.stamp(RTC_TRACE_LAST_BLOCK, lane);
                        last_seen = true;
                    }
                    return true;
                };
                // a worker with only products to form issues its task's first
                // matrix batch before it waits (the others ask first, so that a
                // block that is not ready costs them no matrix traffic)
                if (mvm_only ? mvm_tasks<true>(I, A, q, W, S.kb, ro.mvm_n, lane, lds, ft.mvm, tr,
                                               1, slopes_in)
                             : mvm_tasks<false>(I, A, q, W, S.kb, ro.mvm_n, lane, lds, ft.mvm,
                                                tr, 1, slopes_in)) {
                    if (ft.mvm >= end) ++ms;
                    progressed = true;
                }
                break;
            }
            if (progressed) {
                idle = 0;
            } else {
                __builtin_amdgcn_s_sleep(1);
                if ((++idle & 31) == 0 && stopping(A)) return;
            }
        }
        if (I.polc && !polc_tasks(I, A, q, rank, nw, lane, lds, tr)) return;
        if (tel_frame(I, q) && !tel_copy_tasks(I, A, q, rank, nw, lane)) return;
        trace_end(tr, lane);
    }
}

// Batch: this worker's centroid tasks of frame q (every block; one barrier
// for the frame).  False when the loop must exit.
__device__ __forceinline__ bool batch_centroids(InstRef I, ArgsRef A, uint64_t q, int rank, int nw, int lane,
                                Trace &tr) {
    tr.stamp(RTC_TRACE_FRAME_START, lane);
    if (!gate(I, A, q)) return false;
    tr.stamp(RTC_TRACE_GATE, lane);
    const int64_t qo = (int64_t)(q - I.q_begin);
    const SlopeOut so{I.s_pad[dslot(q)], I.slopes_out ? I.slopes_out + qo * I.n_slopes : nullptr,
                      I.counts_out ? I.counts_out + qo * I.n_units : nullptr, nullptr};
    uint32_t cnt = 0;
    int j = frame_tasks(I, q, rank, nw).cen;
    const int n_kb = I.n_kb, n_all = I.n_cen_all;
    for (int kb = 0; kb < n_kb && j < n_all; ++kb)
        (void)centroid_tasks(I, q, ldc(I.kbw + kb), nw, lane, so, true, j, cnt,
                             [] { return true; });
    drain();
    (void)fan_arrive(I, fan_grp(I.cen_fan, q, I.n_kb, 0), q, I.n_cen_all, cnt, lane);
    tr.stamp(RTC_TRACE_CENTROIDS, lane);
    return true;
}

// Batch worker: every pixel is already in device memory, so the loop is
// software-pipelined over frames.  Iteration q forms the slopes of frame
// q + 1, multiplies frame q (whose slopes were finished one iteration
// earlier) and forms the POLC term of frame q from a_{q-1}.  The gate of frame
// q + 1 is frame q + 1 - kDepth, multiplied kDepth - 1 iterations earlier, so
// workers may drift apart by about an iteration without waiting (slopes two
// frames ahead would gate on the frame multiplied just before, which measured
// slower).  Every wait of iteration q is on work each worker did in an earlier
// iteration, so the loop cannot deadlock.
__device__ __forceinline__ void batch_worker(InstRef I, ArgsRef A, int wid, int rank, int nw, int lane,
                             RTC_LDS float *lds) {
    constexpr int kAhead = 1;
    const uint64_t q0 = I.q_begin, q1 = I.q_end;
    for (uint64_t c = q0; c < q0 + kAhead && c < q1; ++c) {
        Trace tc = trace_of(I, A, c, wid);
        if (!batch_centroids(I, A, c, rank, nw, lane, tc)) return;
    }
    Trace tp;
    for (uint64_t q = q0; q < q1; ++q) {
        if (stopping(A)) return;
        Trace tr = trace_of(I, A, q, wid);
        if (q + kAhead < q1) {
            Trace tn = trace_of(I, A, q + kAhead, wid);
            if (!batch_centroids(I, A, q + kAhead, rank, nw, lane, tn)) return;
        }
        if (!wait_geq(fan_flag(fan_grp(I.cen_fan, q, I.n_kb, 0)), q + 1, A,
                      A.dep_watchdog))
            return;
        int m = frame_tasks(I, q, rank, nw).mvm;
        const int n_kb = I.n_kb, n_all = I.n_seg * I.n_tiles;
        for (int kb = 0; kb < n_kb && m < n_all; ++kb)
            (void)mvm_tasks<false>(I, A, q, ldc(I.kbw + kb), kb, nw, lane, lds, m, tr, 1 << 30,
                                   [] { return true; });
        if (I.polc && q > q0 && !polc_tasks(I, A, q - 1, rank, nw, lane, lds, tr)) return;
        trace_end(tr, lane);
    }
    if (I.polc && !polc_tasks(I, A, q1 - 1, rank, nw, lane, lds, tp)) return;
}

}  // namespace

// The kernel arguments open the kernel-argument segment; each wavefront finds
// its instance by its index in the grid.
#define RTC_FRAME_LOOP_BODY(SERVING)                                                     \
    (void)args;                                                                          \
    ArgsRef A = *(const RTC_CONST PersistArgs *)__builtin_amdgcn_kernarg_segment_ptr();  \
    __shared__ __attribute__((aligned(16))) float lds_all[4][kLoopLdsFloats];            \
    const int lane = threadIdx.x & (kWave - 1);                                          \
    const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6)); \
    RTC_LDS float *lds = (RTC_LDS float *)lds_all[threadIdx.x >> 6];                     \
    for (int i = 0; i < A.n_inst; ++i) {                                                 \
        InstRef I = ((volatile const RTC_CONST PersistInst *)A.inst)[i];                 \
        if (wid < I.w0 || wid >= I.w1) continue;                                         \
        if (SERVING) {                                                                   \
            if (wid == I.w0)                                                             \
                sentinel(I, A, lane);                                                    \
            else                                                                         \
                serving_worker(I, A, wid, wid - I.w0 - 1, I.w1 - I.w0 - 1, lane, lds);   \
        } else {                                                                         \
            batch_worker(I, A, wid, wid - I.w0, I.w1 - I.w0, lane, lds);                 \
        }                                                                                \
        return;                                                                          \
    }

// Serving form: it runs until stopped beside whatever else the device runs,
// at two workgroups per CU, so a lane may hold up to 256 VGPRs.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void
k_frame_loop_serve(PersistArgs args) {
    RTC_FRAME_LOOP_BODY(true)
}

// Batch form: a finite launch over frames already in device memory, at the
// whole occupancy (three workgroups per CU: the most that fit without
// spilling).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void
k_frame_loop_batch(PersistArgs args) {
    RTC_FRAME_LOOP_BODY(false)
}
#undef RTC_FRAME_LOOP_BODY

// Counters of one instance at the start of a launch: zero, except the joins
// of the first frame (copy par), which find their (A) part, and with POLC
// their (P) part, already counted.
__global__ void k_seed_counters(uint64_t *ctr, size_t n, size_t join_off, int n_tiles, int par,
                                int polc) {
    const size_t join_end = join_off + (size_t)kDepth * n_tiles * kCtrSlot;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        uint64_t v = 0;
        if (i >= join_off && i < join_end && (i - join_off) % kCtrSlot == 0 &&
            (int)((i - join_off) / kCtrSlot / n_tiles) == par)
            v = polc ? 2 : 1;
        gbl(ctr)[i] = v;
    }
}

void launch_seed_counters(hipStream_t st, uint64_t *ctr, size_t n, size_t join_off, int n_tiles,
                          int par, int polc) {
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_seed_counters, dim3(blocks), dim3(256), 0, st, ctr, n, join_off, n_tiles,
                       par, polc);
}

void launch_frame_loop(hipStream_t st, int n_blocks, const PersistArgs &args, bool serving) {
    if (serving)
        hipLaunchKernelGGL(k_frame_loop_serve, dim3(n_blocks), dim3(256), 0, st, args);
    else
        hipLaunchKernelGGL(k_frame_loop_batch, dim3(n_blocks), dim3(256), 0, st, args);
}

int frame_loop_max_blocks_per_cu(bool serving) {
    int n = 0;
    const hipError_t err =
        serving ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_frame_loop_serve, 256, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_frame_loop_batch, 256, 0);
    return err == hipSuccess ? n : 0;
}

}  // namespace rtc
