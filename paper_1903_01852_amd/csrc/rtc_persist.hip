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
// never reset.  A worker may reach frame q + 1 while frame q is still in
// flight (slopes, partials and commands are double-buffered by frame parity),
// so every arrival counter exists twice, indexed by q & 1; frame q + 2 cannot
// start a block before frame q has finished it, so the frames sharing a
// counter never overlap, and the target for frame q is (q / 2 + 1) x (work
// per frame).  Everything one wavefront hands to another goes through
// agent-scope atomics (written through past the XCD's non-coherent L2), with
// the writer draining its stores before it counts them.
//
// Serving instances read pixels straight from the pinned host ring; a
// sentinel wavefront per instance mirrors the host doorbells into device
// memory.  Commands go to a pinned host mailbox with system-scope stores,
// followed by the frame's sequence number (the paper's latency ends when the
// DM command is ready, section 3.1).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rtc_device.h"

namespace rtc {

namespace {

__device__ __forceinline__ uint64_t ld_agent64(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent64(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t add_agent64(uint64_t *p, uint64_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_sys64(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void st_agent(float *p, float v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_sys(float *p, float v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
// Wait until every store this wavefront issued has completed.
__device__ __forceinline__ void drain() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
__device__ __forceinline__ bool stopping(const PersistArgs &A) {
    return __hip_atomic_load(A.stop_dev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}
__device__ void watchdog_expired(const PersistArgs &A) {
    __hip_atomic_store(A.status, (uint32_t)PERSIST_WATCHDOG, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(A.stop_dev, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Spin until *ctr >= target.  False when the loop must exit (stop request or
// watchdog expiry); the stop flag and the clock are checked every 32 polls.
__device__ bool wait_geq(const uint64_t *ctr, uint64_t target, const PersistArgs &A,
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

__device__ __forceinline__ uint64_t db_pack(uint64_t q, uint64_t chunks) {
    return (q << kDbShift) | chunks;
}
__device__ __forceinline__ bool db_reached(uint64_t db, uint64_t q, uint64_t chunks) {
    const uint64_t dq = db >> kDbShift;
    return dq > q || (dq == q && (db & kDbChunkMask) >= chunks);
}

// Wait for chunk `chunk` of frame q of sensor w (serving instances).  Only a
// stop request ends this wait: the sentinel turns a long idle period into one.
__device__ bool wait_chunk(const PersistInst &I, const PersistArgs &A, int w, uint64_t q,
                           int chunk) {
    const uint64_t *m = I.db_mirror + w;
    if (db_reached(ld_agent64(m), q, chunk + 1)) return true;
    for (uint32_t it = 1;; ++it) {
        __builtin_amdgcn_s_sleep(1);
        if (db_reached(ld_agent64(m), q, chunk + 1)) return true;
        if ((it & 31) == 0 && stopping(A)) return false;
    }
}

// Stage n floats written by other wavefronts of this kernel into this
// wavefront's LDS slice (two floats per agent-scope atomic load).
__device__ __forceinline__ void stage_lds(float *lds, const float *src, int n, int lane) {
    const uint64_t *s2 = reinterpret_cast<const uint64_t *>(src);
    uint64_t *d2 = reinterpret_cast<uint64_t *>(lds);
    const int n2 = (n + 1) >> 1;
    constexpr int kPer = (kMaxSegVectors * 16 / 2 + kWave - 1) / kWave;   // worst case (FP8)
    uint64_t v[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = j * kWave + lane;
        v[j] = i < n2 ? __hip_atomic_load(s2 + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = j * kWave + lane;
        if (i < n2) d2[i] = v[j];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void lds_done() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Arrivals counted on a parity counter after frame q (frames q, q - 2, ...).
__device__ __forceinline__ uint64_t par_target(uint64_t q, uint64_t per_frame) {
    return (q / 2 + 1) * per_frame;
}

// First task index of this worker among n tasks whose task 0 goes to `base`.
__device__ __forceinline__ int first_task(int rank, int nw, int base) {
    int j = (rank - base) % nw;
    return j < 0 ? j + nw : j;
}

__device__ __forceinline__ const uint16_t *frame_src(const PersistInst &I, int w, uint64_t q) {
    if (I.serving) return I.src[w] + (int64_t)(q % (uint64_t)I.ring_depth) * I.src_stride[w];
    return I.src[w] + (int64_t)(q - I.q_begin) * I.src_stride[w];
}

// Commands of frame q live in buffer q & 1: frame q reads buffer (q - 1) & 1
// while the POLC product of frame q - 1 may still be reading it.
__device__ __forceinline__ float *a_buf(const PersistInst &I, uint64_t q) {
    return I.a + (q & 1) * (uint64_t)I.a_stride;
}

__device__ __forceinline__ int vec_elems(int dtype) {
    return dtype == RTC_CM_F32 ? 4 : dtype == RTC_CM_BF16 ? 8 : 16;
}

// Vectors in flight per lane.  Slope values come from LDS into VGPRs here, so
// the batch is smaller than in the per-launch kernel (scalar slope loads);
// 16 resident wavefronts per CU keep ~32 MB of matrix loads in flight.
template <int DT> struct LoopBatch { static constexpr int U = 8; };
template <> struct LoopBatch<RTC_CM_FP8> { static constexpr int U = 4; };

template <int DT>
__device__ __forceinline__ float mvm_partial(const PersistInst &I, const uint8_t *cm,
                                             const KBlock &K, const Segment &S, int t, int nr,
                                             int lane, const float *lds) {
    if (lane >= nr) return 0.0f;
    const uint4 *p = reinterpret_cast<const uint4 *>(cm + K.base + (int64_t)t * kTileRows * K.kv * 16) +
                     (int64_t)S.v0 * nr + lane;
    return stream_segment<DT, LoopBatch<DT>::U>(p, nr, reinterpret_cast<const float4 *>(lds), S.nv);
}

__device__ __forceinline__ float seg_partial(const PersistInst &I, const KBlock &K,
                                             const Segment &S, int t, int nr, int lane,
                                             const float *lds) {
    switch (I.dtype) {
    case RTC_CM_F32: return mvm_partial<RTC_CM_F32>(I, I.cm, K, S, t, nr, lane, lds);
    case RTC_CM_BF16: return mvm_partial<RTC_CM_BF16>(I, I.cm, K, S, t, nr, lane, lds);
    default: return mvm_partial<RTC_CM_FP8>(I, I.cm, K, S, t, nr, lane, lds);
    }
}

// Frame coefficients for frame q.
__device__ __forceinline__ void frame_coef(const PersistInst &I, uint64_t q, float &c1, float &g) {
    if (I.serving) {
        // device mirror, refreshed by the sentinel before it mirrors any
        // doorbell that follows a host parameter change
        const ParamBlock *pb = I.param_mirror;
        const uint64_t word = ld_agent64(&pb->word);
        const uint64_t qs = word >> 1;
        const int staged = (int)(word & 1);
        const int s = q >= qs ? staged : 1 - staged;
        c1 = __hip_atomic_load(&pb->c1[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        g = __hip_atomic_load(&pb->g[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        const int s = q >= I.coef.q_switch ? 1 : 0;
        c1 = I.coef.c1[s];
        g = I.coef.g[s];
    }
}

// ---------------------------------------------------------------------------
// Sentinel of a serving instance: mirror the host doorbells, parameters and
// drop marks into device memory, stamp each frame's last chunk, relay a stop
// request.
__device__ void sentinel(const PersistInst &I, const PersistArgs &A, int lane) {
    const int nw = I.n_wfs;
    int nch = 0;          // lane w: chunks per frame of sensor w
    for (int st = 0; st < I.n_steps; ++st)
        if (I.steps[st].wfs == lane) nch = max(nch, I.steps[st].chunk + 1);
    uint64_t last = ~0ull;
    uint64_t last_word = ~0ull;
    uint64_t last_drop = ~0ull;
    uint64_t seen_q = I.q_begin;   // next frame whose last chunk has not been stamped
    uint64_t t_change = wall_clock64();
    for (uint32_t it = 0;; ++it) {
        uint64_t db = 0;
        if (lane < nw) db = ld_sys64(I.doorbell + lane);
        // parameters are read after the doorbells and mirrored before them:
        // a doorbell seen here was rung after any parameter change it follows
        const uint64_t word = ld_sys64(&I.params->word);
        if (word != last_word) {
            if (lane < 2) {
                const float c1 = __hip_atomic_load(&I.params->c1[lane], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_SYSTEM);
                const float g = __hip_atomic_load(&I.params->g[lane], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&I.param_mirror->c1[lane], c1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&I.param_mirror->g[lane], g, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            drain();
            if (lane == 0) st_agent64(&I.param_mirror->word, word);
            last_word = word;
        }
        // drop marks likewise: the host writes a frame's mark before the
        // doorbells that complete it
        uint64_t dm = 0;
        if (lane < I.ring_depth) dm = ld_sys64(I.drop_host + lane);
        if (lane < I.ring_depth && dm != last_drop) {
            st_agent64(I.drop_mirror + lane, dm);
            last_drop = dm;
        }
        const bool changed = lane < nw && db != last;
        if (__any(changed)) {
            drain();
            if (changed) st_agent64(I.db_mirror + lane, db);
            last = db;
            t_change = wall_clock64();
        }
        // stamp frame seen_q once every sensor has delivered all its chunks
        const bool ok = lane >= nw || db_reached(db, seen_q, (uint64_t)nch);
        if (__all(ok)) {
            if (lane == 0) {
                FrameTel *tel = I.tel + (seen_q % (uint64_t)I.ring_depth);
                __hip_atomic_store(&tel->ticks_last_chunk, wall_clock64(), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
            }
            ++seen_q;
        }
        if ((it & 15) == 0) {
            const uint32_t stop = __hip_atomic_load(A.stop_host, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_SYSTEM);
            // A serving loop idle for longer than the idle limit ends the kernel
            // (the host relaunches it on demand), but only between frames: no
            // chunk of the next frame delivered, every delivered frame
            // published and its POLC term formed.
            bool quiet = wall_clock64() - t_change > A.idle_watchdog;
            if (quiet) {
                const bool none = lane >= nw || !db_reached(db, seen_q, 1);
                const uint64_t pub = ld_agent64(I.tiles_done) + ld_agent64(I.tiles_done + 1);
                const uint64_t pol = ld_agent64(I.pol_tiles);
                quiet = __all(none) && pub == seen_q * (uint64_t)I.n_tiles &&
                        (!I.polc || pol == seen_q * (uint64_t)I.n_tiles);
            }
            if (stop != 0 || quiet) {
                __hip_atomic_store(A.stop_dev, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
// Block accumulation as a join.  Accumulating block kb of frame q on tile t
// needs (E) every partial of the block on the tile, (A) the previous block
// accumulated (block n_kb - 1 of frame q - 1 for kb = 0) and, for the last
// block with POLC, (P) the POLC term of the tile.  Each party adds one to the
// block's join counter; the party that completes the count does the work, so
// nobody ever waits, and then joins the next block as its (A) party.  Join
// counters are doubled by frame parity like the arrival counters; the first
// frame after a reset finds its (A) and (P) parts pre-counted by the host.
__device__ __forceinline__ uint64_t join_need(const PersistInst &I, int kb) {
    return (I.polc && kb == I.n_kb - 1) ? 3 : 2;
}
__device__ __forceinline__ uint64_t *join_ctr(const PersistInst &I, uint64_t q, int kb, int t) {
    return I.join + ((size_t)(q & 1) * I.n_kb + kb) * I.n_tiles + t;
}
// True when this wavefront's arrival completes the join of (q, kb, t).
__device__ __forceinline__ bool join(const PersistInst &I, uint64_t q, int kb, int t, int lane) {
    uint64_t old = 0;
    if (lane == 0) old = add_agent64(join_ctr(I, q, kb, t), 1);
    old = __shfl(old, 0, kWave);
    return (old + 1) % join_need(I, kb) == 0;
}

// Accumulate block kb of frame q into tile t, then every following block
// whose join this completes.  Blocks are added in readout order, each block's
// segments in order: the same arithmetic as the per-launch epilogue.  The
// last block applies the FP8 row scale, the POLC term and the leaky
// integrator, and publishes the tile's commands.
__device__ void run_chain(const PersistInst &I, uint64_t q, int kb, int t, int lane) {
    const uint64_t nkb = (uint64_t)I.n_kb;
    const int nr = min(kTileRows, I.n_act - t * kTileRows);
    const int r = t * kTileRows + lane;
    for (;;) {
        const bool last_block = kb == I.n_kb - 1;
        if (lane < nr) {
            const int2 sb = I.kb_segs[kb];
            float y = kb == 0 ? 0.0f : load_agent(I.y_acc + r);
            y += sum_parts(I.y_part[q & 1], sb.x, sb.y, I.n_act, r);
            if (!last_block) {
                st_agent(I.y_acc + r, y);
            } else {
                float c1, g;
                frame_coef(I, q, c1, g);
                if (I.scale != nullptr) y *= I.scale[r];
                if (I.polc) y += load_agent(I.p + r);
                const float aprev = load_agent(a_buf(I, q ^ 1) + r);   // buffer of frame q - 1
                bool dropped = false;
                if (I.serving)
                    dropped = ld_agent64(I.drop_mirror + (q % (uint64_t)I.ring_depth)) == q + 1;
                const float an = dropped ? aprev : fmaf(c1, aprev, g * y);
                st_agent(a_buf(I, q) + r, an);
                if (I.serving)
                    st_sys(I.mail + (size_t)(q % (uint64_t)I.ring_depth) * I.n_act + r, an);
                else if (I.cmds_out != nullptr)
                    I.cmds_out[(size_t)(q - I.q_begin) * I.n_act + r] = an;
            }
        }
        drain();
        if (lane == 0) st_agent64(I.acc_done + t, q * nkb + (uint64_t)kb + 1);
        if (last_block) {
            uint64_t old = 0;
            if (lane == 0) old = add_agent64(I.tiles_done + (q & 1), 1);
            old = __shfl(old, 0, kWave);
            if (old + 1 == par_target(q, (uint64_t)I.n_tiles) && I.serving && lane == 0) {
                FrameTel *tel = I.tel + (q % (uint64_t)I.ring_depth);
                __hip_atomic_store(&tel->ticks_publish, wall_clock64(), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(I.cmd_seq, q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            ++q;
            kb = 0;
        } else {
            ++kb;
        }
        if (!join(I, q, kb, t, lane)) return;
    }
}

// POLC term of frame q + 1: p = M a_q, partials per POLC segment, reduced by
// the wavefront completing a tile.
__device__ bool polc_tasks(const PersistInst &I, const PersistArgs &A, uint64_t q, int rank,
                           int nw, int lane, float *lds) {
    const int n_tasks = I.n_segm * I.n_tiles;
    int j = first_task(rank, nw, 0);
    if (j >= n_tasks) return true;
    if (!wait_geq(I.tiles_done + (q & 1), par_target(q, (uint64_t)I.n_tiles), A, A.dep_watchdog))
        return false;
    const float *aq = a_buf(I, q);
    float *part = I.p_part[q & 1];
    for (; j < n_tasks; j += nw) {
        const int sg = j / I.n_tiles;
        const int t = j - sg * I.n_tiles;
        const Segment S = I.segm[sg];
        const KBlock K = I.kbm[S.kb];
        stage_lds(lds, aq + K.spad + S.v0 * 4, S.nv * 4, lane);
        if (q >= 2 && !wait_geq(I.p_done + t, q - 1, A, A.dep_watchdog)) return false;
        const int nr = min(kTileRows, I.n_act - t * kTileRows);
        const float v = mvm_partial<RTC_CM_F32>(I, I.M, K, S, t, nr, lane, lds);
        if (lane < nr) st_agent(part + (size_t)sg * I.n_act + t * kTileRows + lane, v);
        lds_done();
        drain();
        uint64_t old = 0;
        if (lane == 0) old = add_agent64(I.pol_cnt + (q & 1) * I.n_tiles + t, 1);
        old = __shfl(old, 0, kWave);
        if (old + 1 != par_target(q, (uint64_t)I.n_segm)) continue;
        const int r = t * kTileRows + lane;
        if (lane < nr) {
            float y = 0.0f;
            for (int b = 0; b < I.n_kbm; ++b) {
                const int2 sb = I.kbm_segs[b];
                y += sum_parts(part, sb.x, sb.y, I.n_act, r);
            }
            st_agent(I.p + r, y);
        }
        drain();
        if (lane == 0) st_agent64(I.p_done + t, q + 1);
        uint64_t pt = 0;
        if (lane == 0) pt = add_agent64(I.pol_tiles, 1);
        pt = __shfl(pt, 0, kWave);
        if (I.serving && lane == 0 && pt + 1 == (q + 1) * (uint64_t)I.n_tiles)
            __hip_atomic_store(I.pol_seq, q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        // (P) party of frame q + 1's last block on this tile
        if (join(I, q + 1, I.n_kb - 1, t, lane)) run_chain(I, q + 1, I.n_kb - 1, t, lane);
    }
    return true;
}

// One worker of one instance.
__device__ void worker(const PersistInst &I, const PersistArgs &A, int rank, int nw, int lane,
                       float *lds) {
    const uint64_t ntl = (uint64_t)I.n_tiles;
    for (uint64_t q = I.q_begin; q < I.q_end; ++q) {
        if (stopping(A)) return;
        float *spad = I.s_pad[q & 1];
        const int E = vec_elems(I.dtype);
        const int64_t qo = (int64_t)(q - I.q_begin);
        const SlopeOut so{spad,
                          I.slopes_out ? I.slopes_out + qo * I.n_slopes : nullptr,
                          I.counts_out ? I.counts_out + qo * I.n_units : nullptr, nullptr};
        for (int st = 0; st < I.n_steps; ++st) {
            const Step S = I.steps[st];
            if (S.kb < 0) continue;
            const KbWork W = I.kbw[S.kb];
            const uint64_t n_mvm = (uint64_t)W.nseg * ntl;
            int jc = first_task(rank, nw, W.cen_base);
            int jm = first_task(rank, nw, W.mvm_base);
            const bool any_cen = jc < W.n_cen;
            const bool any_mvm = (uint64_t)jm < n_mvm;
            if (!any_cen && !any_mvm) continue;
            if (I.serving && !wait_chunk(I, A, S.wfs, q, S.chunk)) return;
            // centroid tasks
            if (any_cen) {
                // slopes buffer q & 1 is free once frame q - 2 has finished this block
                if (q >= 2 && !wait_geq(I.mvm_done + (q & 1) * I.n_kb + S.kb, (q / 2) * n_mvm, A,
                                        A.dep_watchdog))
                    return;
                const uint16_t *fr = frame_src(I, W.wfs, q);
                const WfsParam &P = I.wp[W.wfs];
                int n_done = 0;
                for (; jc < W.n_cen; jc += nw, ++n_done) {
                    if (W.kind == RTC_WFS_SH) {
                        const int u = W.cu0 + jc;
                        const ShUnit d = I.sh[u];
                        if (I.serving)
                            sh_unit<STORE_AGENT, LOAD_SYSTEM>(d, I.sh_thr[u], fr, P, I.sh_dark,
                                                              I.sh_flat, I.sh_bg, I.ref, so, lane);
                        else
                            sh_unit<STORE_AGENT, LOAD_PLAIN>(d, I.sh_thr[u], fr, P, I.sh_dark,
                                                             I.sh_flat, I.sh_bg, I.ref, so, lane);
                    } else {
                        const int k = W.cu0 + jc * kWave + lane;
                        if (k < W.cu1) {
                            const PyrUnit d = I.py[k];
                            if (I.serving)
                                pyr_unit<STORE_AGENT, LOAD_SYSTEM>(d, k, I.n_pyr, I.py_thr[k], fr,
                                                                   P, I.py_dark, I.py_flat,
                                                                   I.py_bg, I.ref, so);
                            else
                                pyr_unit<STORE_AGENT, LOAD_PLAIN>(d, k, I.n_pyr, I.py_thr[k], fr,
                                                                  P, I.py_dark, I.py_flat, I.py_bg,
                                                                  I.ref, so);
                        }
                    }
                }
                drain();
                if (lane == 0) add_agent64(I.cen_done + (q & 1) * I.n_kb + S.kb, (uint64_t)n_done);
            }
            // MVM tasks of this block
            if (any_mvm) {
                if (!wait_geq(I.cen_done + (q & 1) * I.n_kb + S.kb, par_target(q, (uint64_t)W.n_cen),
                              A, A.dep_watchdog))
                    return;
                const KBlock K = I.kbs[S.kb];
                int staged = -1;
                uint64_t n_done = 0;
                for (; (uint64_t)jm < n_mvm; jm += nw, ++n_done) {
                    const int sl = jm / I.n_tiles;
                    const int t = jm - sl * I.n_tiles;
                    const int sg = W.seg0 + sl;
                    const Segment Sg = I.segs[sg];
                    if (staged != sg) {
                        if (staged >= 0) lds_done();
                        stage_lds(lds, spad + K.spad + Sg.v0 * E, Sg.nv * E, lane);
                        staged = sg;
                    }
                    if (q >= 2 &&
                        !wait_geq(I.acc_done + t, (q - 2) * (uint64_t)I.n_kb + (uint64_t)S.kb + 1, A,
                                  A.dep_watchdog))
                        return;
                    const int nr = min(kTileRows, I.n_act - t * kTileRows);
                    const float v = seg_partial(I, K, Sg, t, nr, lane, lds);
                    if (lane < nr)
                        st_agent(I.y_part[q & 1] + (size_t)sg * I.n_act + t * kTileRows + lane, v);
                    drain();
                    uint64_t old = 0;
                    if (lane == 0)
                        old = add_agent64(
                            I.kbt_cnt + ((size_t)(q & 1) * I.n_kb + S.kb) * I.n_tiles + t, 1);
                    old = __shfl(old, 0, kWave);
                    // (E) party: the block's last partial on this tile
                    if (old + 1 == par_target(q, (uint64_t)W.nseg) && join(I, q, S.kb, t, lane))
                        run_chain(I, q, S.kb, t, lane);
                }
                lds_done();
                if (lane == 0) add_agent64(I.mvm_done + (q & 1) * I.n_kb + S.kb, n_done);
            }
        }
        if (I.polc && !polc_tasks(I, A, q, rank, nw, lane, lds)) return;
    }
}

}  // namespace

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_frame_loop(PersistArgs A) {
    __shared__ __attribute__((aligned(16))) float lds_all[4][kMaxSegVectors * 16];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    float *lds = lds_all[threadIdx.x >> 6];
    for (int i = 0; i < A.n_inst; ++i) {
        const PersistInst &I = A.inst[i];
        if (wid < I.w0 || wid >= I.w1) continue;
        if (I.serving) {
            if (wid == I.w0) {
                sentinel(I, A, lane);
                return;
            }
            worker(I, A, wid - I.w0 - 1, I.w1 - I.w0 - 1, lane, lds);
        } else {
            worker(I, A, wid - I.w0, I.w1 - I.w0, lane, lds);
        }
        return;
    }
}

void launch_frame_loop(hipStream_t st, int n_blocks, const PersistArgs &args) {
    hipLaunchKernelGGL(k_frame_loop, dim3(n_blocks), dim3(256), 0, st, args);
}

int frame_loop_max_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_frame_loop, 256, 0) != hipSuccess)
        return 0;
    return n;
}

}  // namespace rtc
