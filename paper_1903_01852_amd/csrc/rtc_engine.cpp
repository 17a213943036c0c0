// Host runtime and C ABI of the real-time-controller hot path.
//
// Owns every device and pinned buffer of an engine, builds the unit and
// column-block tables from the sensor geometry, encodes and re-tiles the
// control matrix, and drives the gfx950 kernels either per chunk (stream
// mode) or over device-resident frame batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "rtc.h"
#include "rtc_engine.h"
#include "rtc_internal.h"

using namespace rtc;



// ---------------------------------------------------------------- encoders
uint16_t bf16_rne(float f) {
    uint32_t b;
    std::memcpy(&b, &f, 4);
    const uint32_t lsb = (b >> 16) & 1u;
    return (uint16_t)((b + 0x7FFFu + lsb) >> 16);
}

// OCP e4m3fn, round to nearest with ties to even, for |f| <= 448.
uint8_t fp8_rne(float f) {
    uint32_t b;
    std::memcpy(&b, &f, 4);
    const uint8_t sign = (uint8_t)((b >> 24) & 0x80u);
    const uint32_t mag = b & 0x7FFFFFFFu;
    float a;
    std::memcpy(&a, &mag, 4);
    uint32_t code;
    if (a < 0.015625f) {                       // below 2^-6: subnormal binade, quantum 2^-9
        code = (uint32_t)std::nearbyint(a * 512.0f);   // exact scaling, ties to even
    } else {
        const int e = (int)(mag >> 23) - 127;  // -6 .. 8
        const uint32_t m23 = mag & 0x7FFFFFu;
        const uint32_t m3 = (m23 + 0x7FFFFu + ((m23 >> 20) & 1u)) >> 20;   // may carry to 8
        code = (uint32_t)((e + 7) << 3) + m3;
    }
    return (uint8_t)(sign | code);
}

int chunk_row(int H, int n, int c) { return (int)(((int64_t)c * H) / n); }

rtc_status validate_wfs(const rtc_wfs_desc &w) {
    if (w.frame_h <= 0 || w.frame_w <= 0 || w.n_chunks <= 0 || w.n_chunks > w.frame_h)
        return RTC_E_INVAL;
    if (w.thr_mode < RTC_THR_SUBTRACT || w.thr_mode > RTC_THR_NONE) return RTC_E_INVAL;
    if (w.kind == RTC_WFS_SH) {
        if (w.nsub <= 0 || w.px <= 0 || w.px > kMaxShPx || !w.subap_valid) return RTC_E_INVAL;
        if (w.origin_row < 0 || w.origin_col < 0) return RTC_E_INVAL;
        if (w.origin_row + (int64_t)w.nsub * w.px > w.frame_h) return RTC_E_INVAL;
        if (w.origin_col + (int64_t)w.nsub * w.px > w.frame_w) return RTC_E_INVAL;
    } else if (w.kind == RTC_WFS_PYR) {
        if (w.pupil_px <= 0 || !w.pupil_valid) return RTC_E_INVAL;
        if (w.pyr_norm != RTC_PYR_NORM_LOCAL && w.pyr_norm != RTC_PYR_NORM_GLOBAL)
            return RTC_E_INVAL;
        for (int q = 0; q < 4; ++q) {
            if (w.quad_row[q] < 0 || w.quad_col[q] < 0) return RTC_E_INVAL;
            if (w.quad_row[q] + w.pupil_px > w.frame_h) return RTC_E_INVAL;
            if (w.quad_col[q] + w.pupil_px > w.frame_w) return RTC_E_INVAL;
        }
    } else {
        return RTC_E_INVAL;
    }
    return RTC_OK;
}

// Segments of a matrix: each column block cut into nearly equal parts of at
// most max_seg vectors (and at least n_min[b] parts, when given), in block
// order.  A segment is one wavefront's work on
// one 64-row tile (per-launch MVM and frame loop alike) and owns one partial.
void build_segments(const std::vector<KBlock> &kbs, int max_seg, std::vector<Segment> &seg,
                    const std::vector<int> *n_min) {
    for (size_t b = 0; b < kbs.size(); ++b) {
        const int kv = kbs[b].kv;
        int n = (kv + max_seg - 1) / max_seg;
        if (n_min != nullptr) n = std::max(n, std::min((*n_min)[b], kv));
        for (int i = 0; i < n; ++i) {
            const int a = (int)((int64_t)kv * i / n), z = (int)((int64_t)kv * (i + 1) / n);
            seg.push_back(Segment{(int32_t)b, a, z - a, 0});
        }
    }
}

// Bit j set when segment j is the last of its column block.
std::vector<uint32_t> segment_ends(const std::vector<Segment> &seg) {
    std::vector<uint32_t> m((seg.size() + 31) / 32 + 1, 0u);
    for (size_t j = 0; j < seg.size(); ++j)
        if (j + 1 == seg.size() || seg[j + 1].kb != seg[j].kb) m[j / 32] |= 1u << (j % 32);
    return m;
}

// Longest segment of the reconstruction MVM by storage type (vectors).
int segment_vectors(int dtype) {
    (void)dtype;
    return kMaxSegVectors;
}

// Segments with their block's fields folded in (E slope values per vector).
std::vector<SegRun> seg_runs(const std::vector<KBlock> &kbs, const std::vector<Segment> &seg,
                             int E) {
    std::vector<SegRun> run;
    run.reserve(seg.size());
    for (const Segment &S : seg) {
        const KBlock &K = kbs[S.kb];
        run.push_back(SegRun{K.base, K.kv, K.spad + S.v0 * E, S.v0, S.nv, 0, 0});
    }
    return run;
}

// Geometry -> units, chunk readiness, column blocks, padded slope layout.
rtc_status build_instance(rtc_engine *e, Instance *I) {
    const int E = elems_per_vec(I->d.cm_dtype);
    int unit = 0, mask = 0;
    for (int w = 0; w < (int)I->wfs.size(); ++w) {
        WfsState &S = I->wfs[w];
        const rtc_wfs_desc &d = S.d;
        S.u0 = unit;
        WfsParam &P = I->params.w[w];
        P.kind = d.kind;
        P.W = d.frame_w;
        P.H = d.frame_h;
        P.thr_mode = d.thr_mode;
        S.row0.resize(d.n_chunks + 1);
        for (int c = 0; c <= d.n_chunks; ++c) S.row0[c] = chunk_row(d.frame_h, d.n_chunks, c);
        if (d.kind == RTC_WFS_SH) {
            P.p = d.px;
            P.half = 0.5f * (float)(d.px - 1);
            P.mask_words = (d.px * d.px + 63) / 64;
            S.kind0 = (int)I->sh.size();
            for (int i = 0; i < d.nsub; ++i)
                for (int j = 0; j < d.nsub; ++j) {
                    if (!S.valid[(size_t)i * d.nsub + j]) continue;
                    ShUnit u{};
                    u.row0 = d.origin_row + i * d.px;
                    u.col0 = d.origin_col + j * d.px;
                    u.wfs = w;
                    u.unit = unit++;
                    u.mask = mask;
                    mask += P.mask_words;
                    I->sh.push_back(u);
                    S.unit_ready.push_back(u.row0 + d.px - 1);
                }
        } else {
            P.p = 0;
            P.mask_words = 1;
            for (int q = 0; q < 4; ++q) {
                P.qrow[q] = d.quad_row[q];
                P.qcol[q] = d.quad_col[q];
            }
            int qmax = 0;
            for (int q = 0; q < 4; ++q) qmax = std::max(qmax, d.quad_row[q]);
            // globally normalised slopes all complete with the frame's last row
            const bool global = d.pyr_norm == RTC_PYR_NORM_GLOBAL;
            P.norm = d.pyr_norm;
            if (global) I->pyr_global.w[I->pyr_global.n++] = w;
            S.kind0 = (int)I->py.size();
            for (int i = 0; i < d.pupil_px; ++i)
                for (int j = 0; j < d.pupil_px; ++j) {
                    if (!S.valid[(size_t)i * d.pupil_px + j]) continue;
                    PyrUnit u{};
                    u.i = i;
                    u.j = j;
                    u.wfs = w;
                    u.unit = unit++;
                    u.mask = mask;
                    mask += 1;
                    I->py.push_back(u);
                    S.unit_ready.push_back(global ? d.frame_h - 1 : qmax + i);
                }
            P.pu0 = S.kind0;
            P.pn = (int)I->py.size() - S.kind0;
        }
        S.u1 = unit;
        if (S.u1 == S.u0) return RTC_E_INVAL;    // a sensor without units
    }
    I->n_units = unit;
    I->n_slopes = 2 * unit;
    I->mask_words = mask;
    I->n_sh = (int)I->sh.size();
    I->n_pyr = (int)I->py.size();
    // calibration offsets of SH units: p*p values each, in unit order
    {
        int off = 0;
        for (auto &u : I->sh) {
            u.cal = off;
            off += I->params.w[u.wfs].p * I->params.w[u.wfs].p;
        }
    }
    // column blocks: units become ready in raster order, so each chunk
    // completes a contiguous unit range of its sensor.  Blocks are numbered in
    // readout order, the order in which every path accumulates them: sensors
    // are read out in parallel over the same frame time, so chunk c of a sensor
    // cut into n chunks arrives at (c + 1) / n of the readout; steps are sorted
    // by that fraction, then by sensor.
    int spad = 0;
    int64_t base = 0;
    const int n_tiles = (I->n_act + kTileRows - 1) / kTileRows;
    std::vector<std::vector<std::pair<int, int>>> ranges(I->wfs.size());
    int max_chunks = 0;
    for (int w = 0; w < (int)I->wfs.size(); ++w) {
        WfsState &S = I->wfs[w];
        S.kb_of_chunk.assign(S.d.n_chunks, -1);
        max_chunks = std::max(max_chunks, S.d.n_chunks);
        int next = 0;     // next unit (relative) not yet assigned
        const int nu = S.u1 - S.u0;
        for (int c = 0; c < S.d.n_chunks; ++c) {
            const int last_row = S.row0[c + 1] - 1;
            int end = next;
            while (end < nu && S.unit_ready[end] <= last_row) ++end;
            ranges[w].push_back({next, end});
            next = end;
        }
        if (next != nu) return RTC_E_INVAL;
    }
    std::vector<std::pair<int, int>> order;      // (sensor, chunk) in readout order
    for (int w = 0; w < (int)I->wfs.size(); ++w)
        for (int c = 0; c < I->wfs[w].d.n_chunks; ++c) order.push_back({w, c});
    std::stable_sort(order.begin(), order.end(), [&](const std::pair<int, int> &a,
                                                     const std::pair<int, int> &b) {
        const int64_t fa = (int64_t)(a.second + 1) * I->wfs[b.first].d.n_chunks;
        const int64_t fb = (int64_t)(b.second + 1) * I->wfs[a.first].d.n_chunks;
        return fa != fb ? fa < fb : a.first < b.first;
    });
    (void)max_chunks;
    for (const auto &wc : order) {
        {
            const int w = wc.first, c = wc.second;
            WfsState &S = I->wfs[w];
            const int next = ranges[w][c].first, end = ranges[w][c].second;
            I->steps.push_back(Step{w, c, end > next ? (int)I->kb.size() : -1, 0, 0, 0, 0, 0});
            if (end == next) continue;
            KBlock K{};
            K.k0 = 2 * (S.u0 + next);
            K.k = 2 * (end - next);
            K.kv = (K.k + E - 1) / E;
            K.spad = spad;
            K.base = base;
            K.wfs = w;
            K.chunk = c;
            // map units to padded slope indices
            for (int u = next; u < end; ++u) {
                const int pad = spad + 2 * (u - next);
                if (S.d.kind == RTC_WFS_SH)
                    I->sh[S.kind0 + u].pad = pad;
                else
                    I->py[S.kind0 + u].pad = pad;
            }
            S.kb_of_chunk[c] = (int)I->kb.size();
            I->kb.push_back(K);
            spad += ((K.kv * E + 15) / 16) * 16;    // 64-byte aligned block starts
            base += (int64_t)n_tiles * kTileRows * K.kv * 16;
        }
    }
    // the last tile of each block holds fewer rows; trim the allocation to the
    // real end of the last block
    {
        const int last_nr = I->n_act - (n_tiles - 1) * kTileRows;
        const KBlock &L = I->kb.back();
        I->cm_bytes = L.base + (int64_t)(n_tiles - 1) * kTileRows * L.kv * 16 +
                      (int64_t)last_nr * L.kv * 16;
    }
    I->spad_len = spad;
    // The last block of each sensor is multiplied after the frame's last chunk,
    // on the latency path, while the earlier blocks had the readout to run:
    // those last blocks are cut into more segments, so that their tasks
    // (segments x tiles) cover the device's wavefronts (two workgroups of four
    // per CU), down to kMinLastSegVectors vectors a segment.
    std::vector<int> n_min(I->kb.size(), 1);
    std::vector<int> last(I->wfs.size(), -1);
    {
        for (size_t b = 0; b < I->kb.size(); ++b) last[I->kb[b].wfs] = (int)b;
        int n_last = 0;
        for (int b : last) n_last += b >= 0 ? 1 : 0;
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, e->device) !=
                hipSuccess ||
            cus < 1)
            return RTC_E_DEVICE;
        const int want = (8 * cus + n_last * n_tiles - 1) / std::max(1, n_last * n_tiles);
        for (int b : last)
            if (b >= 0)
                n_min[b] = std::min(want, (I->kb[b].kv + kMinLastSegVectors - 1) /
                                              kMinLastSegVectors);
    }
    build_segments(I->kb, std::min(segment_vectors(I->d.cm_dtype), kMaxSegVectors), I->seg,
                   &n_min);
    I->kb_seg0.assign(I->kb.size(), 0);
    I->kb_nseg.assign(I->kb.size(), 0);
    for (size_t i = 0; i < I->seg.size(); ++i) {
        const int b = I->seg[i].kb;
        if (I->kb_nseg[b] == 0) I->kb_seg0[b] = (int)i;
        I->kb_nseg[b]++;
    }
    if (I->seg.size() > (size_t)kMaxSegments) return RTC_E_INVAL;
    I->seg_ends = segment_ends(I->seg);
    // Head and tail of the reconstruction sum (frame loop): the tail runs from
    // the earliest of the sensors' last blocks to the end, the head is every
    // block before it.  During serving the head's blocks are complete long
    // before the frame's last chunk, so their part of the sum (the fold's
    // state after them) is formed off the latency path.
    {
        int tail_kb = (int)I->kb.size() - 1;
        for (int b : last)
            if (b >= 0) tail_kb = std::min(tail_kb, b);
        I->n_head_seg = I->kb_seg0[tail_kb];
        I->tail_ends =
            segment_ends(std::vector<Segment>(I->seg.begin() + I->n_head_seg, I->seg.end()));
    }
    // POLC column blocks of kPolcBlock commands, F32
    if (I->d.polc) {
        const int nb = (I->n_act + kPolcBlock - 1) / kPolcBlock;
        int64_t mb = 0;
        for (int b = 0; b < nb; ++b) {
            KBlock K{};
            K.k0 = b * kPolcBlock;
            K.k = std::min(kPolcBlock, I->n_act - K.k0);
            K.kv = (K.k + 3) / 4;
            K.spad = K.k0;
            K.base = mb;
            mb += (int64_t)n_tiles * kTileRows * K.kv * 16;
            I->kbm.push_back(K);
        }
        const int last_nr = I->n_act - (n_tiles - 1) * kTileRows;
        const KBlock &L = I->kbm.back();
        I->m_bytes = L.base + (int64_t)(n_tiles - 1) * kTileRows * L.kv * 16 +
                     (int64_t)last_nr * L.kv * 16;
        I->a_len = nb * kPolcBlock;
        build_segments(I->kbm, kMaxSegVectors, I->segm, nullptr);
        if (I->segm.size() > (size_t)kMaxSegments) return RTC_E_INVAL;
        I->segm_ends = segment_ends(I->segm);
    } else {
        I->a_len = I->n_act;
    }
    return RTC_OK;
}

rtc_status alloc_instance(rtc_engine *e, Instance *I) {
    const size_t nkb = I->kb.size();
    TRY(dev_alloc(e, &I->d_sh, std::max<size_t>(I->sh.size(), 1)));
    TRY(dev_alloc(e, &I->d_py, std::max<size_t>(I->py.size(), 1)));
    TRY(dev_alloc(e, &I->d_kb, nkb));
    TRY(dev_alloc(e, &I->d_kbm, std::max<size_t>(I->kbm.size(), 1)));
    TRY(dev_alloc(e, &I->d_seg, I->seg.size()));
    TRY(dev_alloc(e, &I->d_seg_ends, I->seg_ends.size()));
    TRY(dev_alloc(e, &I->d_tail_ends, I->tail_ends.size()));
    TRY(dev_alloc(e, &I->d_segm_ends, std::max<size_t>(I->segm_ends.size(), 1)));
    TRY(dev_alloc(e, &I->d_segm, std::max<size_t>(I->segm.size(), 1)));
    TRY(dev_alloc(e, &I->d_run, I->seg.size()));
    TRY(dev_alloc(e, &I->d_runm, std::max<size_t>(I->segm.size(), 1)));
    size_t sh_px = 0;
    for (auto &u : I->sh) sh_px += (size_t)I->params.w[u.wfs].p * I->params.w[u.wfs].p;
    TRY(dev_alloc(e, &I->d_sh_dark, sh_px));
    TRY(dev_alloc(e, &I->d_sh_flat, sh_px));
    TRY(dev_alloc(e, &I->d_sh_bg, sh_px));
    TRY(dev_alloc(e, &I->d_sh_thr, I->sh.size()));
    TRY(dev_alloc(e, &I->d_py_dark, 4 * I->py.size()));
    TRY(dev_alloc(e, &I->d_py_flat, 4 * I->py.size()));
    TRY(dev_alloc(e, &I->d_py_bg, 4 * I->py.size()));
    TRY(dev_alloc(e, &I->d_py_thr, I->py.size()));
    TRY(dev_alloc(e, &I->d_ref, I->n_slopes));
    TRY(dev_alloc(e, &I->d_pyr_sum, RTC_MAX_WFS));
    TRY(dev_alloc(e, &I->d_spad, I->spad_len));
    TRY(dev_alloc(e, &I->d_spad2, I->spad_len));
    TRY(dev_alloc(e, &I->d_sout, I->n_slopes));
    TRY(dev_alloc(e, &I->d_counts, I->n_units));
    TRY(dev_alloc(e, &I->d_masks, I->mask_words));
    // two slots of every matrix: frames stream one while a staged set waits
    // in the other (rtc_stage_matrices / rtc_swap_matrices)
    for (int s = 0; s < 2; ++s) {
        TRY(dev_alloc(e, &I->d_cm_s[s], (size_t)I->cm_bytes));
        TRY(dev_alloc(e, &I->d_scale_s[s], I->n_act));
        if (I->d.polc) TRY(dev_alloc(e, &I->d_M_s[s], (size_t)I->m_bytes));
    }
    if (I->d.polc) TRY(dev_alloc(e, &I->d_ppart, I->segm.size() * (size_t)I->n_act));
    TRY(dev_alloc(e, &I->d_ypart, I->seg.size() * (size_t)I->n_act));
    TRY(dev_alloc(e, &I->d_a, 2 * (size_t)I->a_len));   // buffer 1: frame-loop parity
    TRY(dev_alloc(e, &I->d_p, I->n_act));
    TRY(dev_alloc(e, &I->d_yscratch, I->n_act));
    I->n_tiles = (I->n_act + kTileRows - 1) / kTileRows;
    TRY(dev_alloc(e, &I->d_count, (size_t)I->n_tiles * kCountStride));
    TRY(dev_alloc(e, &I->d_count_m, (size_t)I->n_tiles * kCountStride));
    TRY(dev_alloc(e, &I->d_count_t, (size_t)I->n_tiles * kCountStride));
    HIP_TRY(hipMemcpy(I->d_sh, I->sh.data(), I->sh.size() * sizeof(ShUnit), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(I->d_py, I->py.data(), I->py.size() * sizeof(PyrUnit), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(I->d_kb, I->kb.data(), nkb * sizeof(KBlock), hipMemcpyHostToDevice));
    if (!I->kbm.empty())
        HIP_TRY(hipMemcpy(I->d_kbm, I->kbm.data(), I->kbm.size() * sizeof(KBlock),
                          hipMemcpyHostToDevice));
    auto up = [](void *dst, const void *src, size_t bytes) {
        return bytes ? hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
    };
    HIP_TRY(up(I->d_seg, I->seg.data(), I->seg.size() * sizeof(Segment)));
    HIP_TRY(up(I->d_seg_ends, I->seg_ends.data(), I->seg_ends.size() * 4));
    HIP_TRY(up(I->d_tail_ends, I->tail_ends.data(), I->tail_ends.size() * 4));
    HIP_TRY(up(I->d_segm_ends, I->segm_ends.data(), I->segm_ends.size() * 4));
    HIP_TRY(up(I->d_segm, I->segm.data(), I->segm.size() * sizeof(Segment)));
    const std::vector<SegRun> run = seg_runs(I->kb, I->seg, elems_per_vec(I->d.cm_dtype));
    const std::vector<SegRun> runm = seg_runs(I->kbm, I->segm, elems_per_vec(RTC_CM_F32));
    HIP_TRY(up(I->d_run, run.data(), run.size() * sizeof(SegRun)));
    HIP_TRY(up(I->d_runm, runm.data(), runm.size() * sizeof(SegRun)));
    // default calibration: dark 0, flat 1, bg 0, threshold 0, reference 0
    std::vector<float> ones(std::max(sh_px, 4 * I->py.size()), 1.0f);
    HIP_TRY(hipMemcpy(I->d_sh_flat, ones.data(), sh_px * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(I->d_py_flat, ones.data(), 4 * I->py.size() * 4, hipMemcpyHostToDevice));
    std::vector<float> one_scale(I->n_act, 1.0f);
    for (int s = 0; s < 2; ++s)
        HIP_TRY(hipMemcpy(I->d_scale_s[s], one_scale.data(), I->n_act * 4, hipMemcpyHostToDevice));
    // serving buffers
    for (auto &S : I->wfs) {
        // the persistent serving loop pads rows to 16 bytes so that every chunk
        // is a whole number of 16-byte units; the per-launch path packs rows
        S.pitch16 = (S.d.frame_w + 7) & ~7;
        S.slot16 = (size_t)S.d.frame_h * S.pitch16;
        S.ring_elems = S.slot16 * e->ring_depth + 8;   // + slack for word loads
        TRY(dev_alloc(e, &S.d_ring, S.ring_elems));
        TRY(host_pinned(e, &S.h_stage, S.ring_elems));
    }
    TRY(host_pinned(e, &I->h_mail, (size_t)e->ring_depth * I->n_act));
    I->slots.resize(e->ring_depth);
    for (auto &sl : I->slots) HIP_TRY(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
    return RTC_OK;
}

float active_gain(const Instance *I, uint64_t f) {
    const int s = (I->pending && f >= I->f_switch) ? 1 - I->active : I->active;
    return I->gain[s];
}
float active_leak(const Instance *I, uint64_t f) {
    const int s = (I->pending && f >= I->f_switch) ? 1 - I->active : I->active;
    return I->leak[s];
}
// Retire the staged slot once frame f uses it.
void settle_params(Instance *I, uint64_t f) {
    if (I->pending && f >= I->f_switch) {
        I->active = 1 - I->active;
        I->pending = false;
    }
}

// Matrix slot of frame f: its reconstruction matrix and FP8 scales, and the
// POLC matrix applied to its commands (forming frame f + 1's POLC term).
int mat_slot(const Instance *I, uint64_t f) {
    return (I->m_pending && f >= I->m_switch) ? 1 - I->m_active : I->m_active;
}
void settle_matrices(Instance *I, uint64_t f) {
    if (I->m_pending && f >= I->m_switch) {
        I->m_active = 1 - I->m_active;
        I->m_pending = false;
        I->m_staged = false;
    }
}

// Coefficients of a_f = c1 a_{f-1} + g (y + p).
void coeffs(const Instance *I, uint64_t f, float *c1, float *g) {
    const double gd = active_gain(I, f), ld = active_leak(I, f);
    *g = (float)gd;
    *c1 = I->d.polc ? (float)(1.0 - ld - gd) : (float)(1.0 - ld);
}

void enqueue_centroid(Instance *I, hipStream_t st, const FrameSet &fs, int w, int u_begin,
                      int u_end) {
    WfsState &S = I->wfs[w];
    if (S.d.kind == RTC_WFS_SH) {
        const int a = S.kind0 + (u_begin - S.u0), b = S.kind0 + (u_end - S.u0);
        launch_sh_centroid(st, I->d_sh, a, b, fs, I->params, I->d_sh_dark, I->d_sh_flat,
                           I->d_sh_bg, I->d_sh_thr, I->d_ref, I->d_spad, I->d_sout,
                           I->d_counts, I->d_masks);
    } else {
        const int a = S.kind0 + (u_begin - S.u0), b = S.kind0 + (u_end - S.u0);
        if (S.d.pyr_norm == RTC_PYR_NORM_GLOBAL) {
            WfsList one{};
            one.w[0] = w;
            one.n = 1;
            launch_pyr_sum(st, I->d_py, I->n_pyr, fs, I->params, I->d_py_dark, I->d_py_flat,
                           I->d_py_bg, I->d_py_thr, one, I->d_pyr_sum);
        }
        launch_pyr_slopes(st, I->d_py, a, b, I->n_pyr, fs, I->params, I->d_py_dark,
                          I->d_py_flat, I->d_py_bg, I->d_py_thr, I->d_ref, I->d_spad,
                          I->d_sout, I->d_counts, I->d_masks, I->d_pyr_sum);
    }
}

// Epilogue of the reconstruction MVM: integrate the commands of the frame at
// index seq of the sequence (matrix slot ms: its FP8 row scales).  Odd indices
// stream each segment backwards.
// Partials and per-tile arrival counters the per-launch MVMs of a frame use:
// the engine's own buffers, or the library's static scratch
// (rtc_process_frames_noalloc).
struct MvmScratch {
    float *ypart;          // reconstruction partials [segment][row]
    uint32_t *count;       // reconstruction tile counters
    float *ppart;          // POLC partials
    uint32_t *count_m;     // POLC tile counters
};
MvmScratch engine_scratch(Instance *I) { return {I->d_ypart, I->d_count, I->d_ppart, I->d_count_m}; }

MvmEpilogue integrate_epi(Instance *I, int ms, uint64_t seq, float c1, float g, float *out,
                          uint32_t *count) {
    MvmEpilogue E{};
    E.mode = EPI_INTEGRATE;
    E.rev = (int32_t)(seq & 1);
    E.n_parts = (int)I->seg.size();
    E.seg_ends = I->d_seg_ends;
    E.count = count;
    E.p = I->d.polc ? I->d_p : nullptr;
    E.scale = I->d.cm_dtype == RTC_CM_FP8 ? I->d_scale_s[ms] : nullptr;
    E.a = I->d_a;
    E.out = out;
    E.c1 = c1;
    E.g = g;
    return E;
}

// POLC term for the next frame: p = M a (section 3.4: formed after the
// command is ready, off the latency path of the next frame), with the POLC
// matrix of slot ms (the slot of the frame whose commands a holds).
void enqueue_polc(Instance *I, hipStream_t st, int ms, float *ppart, uint32_t *count_m) {
    if (!I->d.polc) return;
    MvmEpilogue E{};
    E.mode = EPI_REDUCE;
    E.n_parts = (int)I->segm.size();
    E.seg_ends = I->d_segm_ends;
    E.count = count_m;
    E.y = I->d_p;
    launch_mvm(st, RTC_CM_F32, I->stream_nt, I->d_M_s[ms], I->d_runm, 0, (int)I->segm.size(),
               I->n_act, I->d_a, ppart, E);
}

rtc_status check(rtc_engine *e, int32_t inst, Instance **out) {
    if (!e) return RTC_E_INVAL;
    if (e->sticky.load() != RTC_OK) return (rtc_status)e->sticky.load();
    if (inst < 0 || inst >= (int)e->inst.size()) return RTC_E_INVAL;
    *out = e->inst[inst];
    return RTC_OK;
}

rtc_status last_error(rtc_engine *e) {
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) {
        std::fprintf(stderr, "rtc: kernel launch failed: %s\n", hipGetErrorString(err));
        return fail(e, RTC_E_DEVICE);
    }
    return RTC_OK;
}

// Encode R (n_act x n_s, FP32, row-major) into the tiled storage layout.
void encode_matrix(const Instance *I, const float *R, int dt, const std::vector<float> &scale,
                   std::vector<uint8_t> &out, const std::vector<KBlock> &blocks, int n_cols,
                   int64_t bytes) {
    out.assign((size_t)bytes, 0);
    const int es = elem_size(dt), E = 16 / es;
    const int n_rows = I->n_act;
    const int n_tiles = (n_rows + kTileRows - 1) / kTileRows;
    const int nthreads = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (int th = 0; th < nthreads; ++th) {
        pool.emplace_back([&, th]() {
            for (int t = th; t < n_tiles; t += nthreads) {
                const int nr = std::min(kTileRows, n_rows - t * kTileRows);
                for (const KBlock &K : blocks) {
                    uint8_t *blk = out.data() + K.base + (int64_t)t * kTileRows * K.kv * 16;
                    for (int l = 0; l < nr; ++l) {
                        const int r = t * kTileRows + l;
                        const float *row = R + (size_t)r * n_cols;
                        for (int v = 0; v < K.kv; ++v) {
                            uint8_t *dst = blk + ((size_t)v * nr + l) * 16;
                            for (int el = 0; el < E; ++el) {
                                const int c = v * E + el;
                                if (c >= K.k) break;
                                const float x = row[K.k0 + c];
                                if (dt == RTC_CM_F32) {
                                    std::memcpy(dst + 4 * el, &x, 4);
                                } else if (dt == RTC_CM_BF16) {
                                    const uint16_t h = bf16_rne(x);
                                    std::memcpy(dst + 2 * el, &h, 2);
                                } else {
                                    float q = x / scale[r];
                                    q = std::min(448.0f, std::max(-448.0f, q));
                                    dst[el] = fp8_rne(q);
                                }
                            }
                        }
                    }
                }
            }
        });
    }
    for (auto &t : pool) t.join();
}


// Waits for a HIP event, at most kUploadTimeoutNs.
constexpr int64_t kUploadTimeoutNs = 30'000'000'000LL;
rtc_status wait_event(rtc_engine *e, hipEvent_t ev) {
    const int64_t t0 = now_ns();
    for (;;) {
        const hipError_t q = hipEventQuery(ev);
        if (q == hipSuccess) return RTC_OK;
        if (q != hipErrorNotReady) return fail(e, RTC_E_DEVICE);
        if (now_ns() - t0 > kUploadTimeoutNs) {
            std::fprintf(stderr, "rtc: matrix upload did not complete\n");
            return fail(e, RTC_E_DEVICE);
        }
        std::this_thread::yield();
    }
}

// Copies n bytes from host memory to device memory through the two pinned
// staging halves on the upload stream (DMA beside any frames in flight);
// returns once the copy has landed.
rtc_status upload(rtc_engine *e, void *dst, const void *src, size_t n) {
    uint8_t *d = static_cast<uint8_t *>(dst);
    const uint8_t *h = static_cast<const uint8_t *>(src);
    size_t i = 0;
    for (size_t off = 0; off < n; off += kUploadHalf, ++i) {
        const int k = (int)(i & 1);
        TRY(wait_event(e, e->up_done[k]));
        const size_t m = std::min(kUploadHalf, n - off);
        std::memcpy(e->h_up + k * kUploadHalf, h + off, m);
        HIP_TRY(hipMemcpyAsync(d + off, e->h_up + k * kUploadHalf, m, hipMemcpyHostToDevice,
                               e->up_stream));
        HIP_TRY(hipEventRecord(e->up_done[k], e->up_stream));
    }
    TRY(wait_event(e, e->up_done[0]));
    TRY(wait_event(e, e->up_done[1]));
    return RTC_OK;
}

// Encodes R (and M, or M = R.D formed once in FP64 on the device) into matrix
// slot `slot`.
rtc_status put_matrices(rtc_engine *e, Instance *I, int slot, const float *R, const double *D,
                        const float *M) {
    const int na = I->n_act, ns = I->n_slopes;
    const int dt = I->d.cm_dtype;
    std::vector<float> scale(na, 1.0f);
    if (dt == RTC_CM_FP8) {
        for (int r = 0; r < na; ++r) {
            float amax = 0.0f;
            const float *row = R + (size_t)r * ns;
            for (int c = 0; c < ns; ++c) amax = std::max(amax, std::fabs(row[c]));
            if (!std::isfinite(amax)) return RTC_E_INVAL;
            scale[r] = amax > 0.0f ? amax / 448.0f : 1.0f;
        }
    }
    std::vector<uint8_t> enc;
    encode_matrix(I, R, dt, scale, enc, I->kb, ns, I->cm_bytes);
    TRY(upload(e, I->d_cm_s[slot], enc.data(), enc.size()));
    TRY(upload(e, I->d_scale_s[slot], scale.data(), (size_t)na * 4));
    enc.clear();
    enc.shrink_to_fit();
    if (I->d.polc) {
        std::vector<float> Mf((size_t)na * na);
        if (M) {
            std::memcpy(Mf.data(), M, Mf.size() * 4);
        } else {
            // M = R.D in FP64 on the device, rounded once to FP32; the
            // temporaries are freed on every return path
            struct DevTmp {
                void *p = nullptr;
                ~DevTmp() {
                    if (p) (void)hipFree(p);
                }
            } tR, tD, tM;
            HIP_TRY(hipMalloc(&tR.p, (size_t)na * ns * 4));
            HIP_TRY(hipMalloc(&tD.p, (size_t)ns * na * 8));
            HIP_TRY(hipMalloc(&tM.p, (size_t)na * na * 8));
            float *dR = static_cast<float *>(tR.p);
            double *dD = static_cast<double *>(tD.p), *dM = static_cast<double *>(tM.p);
            HIP_TRY(hipMemcpy(dR, R, (size_t)na * ns * 4, hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(dD, D, (size_t)ns * na * 8, hipMemcpyHostToDevice));
            launch_dgemm_rd(e->stream, dR, dD, dM, na, ns);
            TRY(last_error(e));
            HIP_TRY(hipStreamSynchronize(e->stream));
            std::vector<double> Md((size_t)na * na);
            HIP_TRY(hipMemcpy(Md.data(), dM, Md.size() * 8, hipMemcpyDeviceToHost));
            for (size_t i = 0; i < Md.size(); ++i) Mf[i] = (float)Md[i];
        }
        std::vector<float> one(na, 1.0f);
        encode_matrix(I, Mf.data(), RTC_CM_F32, one, enc, I->kbm, na, I->m_bytes);
        TRY(upload(e, I->d_M_s[slot], enc.data(), enc.size()));
    }
    return RTC_OK;
}

// Per-launch batch of device-resident frames (stream mode) with the given MVM
// scratch.  The caller holds I->mu and has checked the arguments.
rtc_status process_frames_stream(rtc_engine *e, Instance *I, const uint16_t *const *frames,
                                 const int64_t *frame_stride, int32_t n_frames, float *cmds,
                                 float *slopes, int32_t *counts, hipStream_t st,
                                 const MvmScratch &sc) {
    // Frame f's MVM runs in one grid with the slopes of frame f + 1 (into the
    // other slope buffer), so only frame 0's slopes are a launch of their own.
    auto frame_set = [&](int f) {
        FrameSet fs{};
        for (size_t w = 0; w < I->wfs.size(); ++w) fs.f[w] = frames[w] + (int64_t)f * frame_stride[w];
        return fs;
    };
    auto copy_out = [&](int f) -> rtc_status {
        if (slopes)
            HIP_TRY(hipMemcpyAsync(slopes + (size_t)f * I->n_slopes, I->d_sout, I->n_slopes * 4,
                                   hipMemcpyDeviceToDevice, st));
        if (counts)
            HIP_TRY(hipMemcpyAsync(counts + (size_t)f * I->n_units, I->d_counts, I->n_units * 4,
                                   hipMemcpyDeviceToDevice, st));
        return RTC_OK;
    };
    float *spad[2] = {I->d_spad, I->d_spad2};
    if (n_frames > 0) {
        const FrameSet fs = frame_set(0);
        if (I->n_sh > 0)
            launch_sh_centroid(st, I->d_sh, 0, I->n_sh, fs, I->params, I->d_sh_dark,
                               I->d_sh_flat, I->d_sh_bg, I->d_sh_thr, I->d_ref, spad[0],
                               I->d_sout, I->d_counts, I->d_masks);
        if (I->n_pyr > 0) {
            launch_pyr_sum(st, I->d_py, I->n_pyr, fs, I->params, I->d_py_dark, I->d_py_flat,
                           I->d_py_bg, I->d_py_thr, I->pyr_global, I->d_pyr_sum);
            launch_pyr_slopes(st, I->d_py, 0, I->n_pyr, I->n_pyr, fs, I->params, I->d_py_dark,
                              I->d_py_flat, I->d_py_bg, I->d_py_thr, I->d_ref, spad[0],
                              I->d_sout, I->d_counts, I->d_masks, I->d_pyr_sum);
        }
        TRY(copy_out(0));
    }
    for (int f = 0; f < n_frames; ++f) {
        float *x = spad[f & 1];
        float c1, g;
        coeffs(I, I->next_frame, &c1, &g);
        settle_params(I, I->next_frame);
        const int ms = mat_slot(I, I->next_frame);
        settle_matrices(I, I->next_frame);
        const MvmEpilogue E =
            integrate_epi(I, ms, I->seq++, c1, g, cmds ? cmds + (size_t)f * I->n_act : nullptr,
                          sc.count);
        if (f + 1 < n_frames) {
            NextSlopes N{};
            N.sh = I->d_sh;
            N.py = I->d_py;
            N.n_sh = I->n_sh;
            N.n_pyr = I->n_pyr;
            N.frames = frame_set(f + 1);
            N.sh_dark = I->d_sh_dark;
            N.sh_flat = I->d_sh_flat;
            N.sh_bg = I->d_sh_bg;
            N.sh_thr = I->d_sh_thr;
            N.py_dark = I->d_py_dark;
            N.py_flat = I->d_py_flat;
            N.py_bg = I->d_py_bg;
            N.py_thr = I->d_py_thr;
            N.py_gsum = I->d_pyr_sum;
            // frame f + 1's pupil sums before the grid that forms its slopes
            launch_pyr_sum(st, I->d_py, I->n_pyr, N.frames, I->params, I->d_py_dark,
                           I->d_py_flat, I->d_py_bg, I->d_py_thr, I->pyr_global, I->d_pyr_sum);
            N.ref = I->d_ref;
            N.s_pad = spad[(f + 1) & 1];
            N.s_out = I->d_sout;
            N.counts = I->d_counts;
            N.masks = I->d_masks;
            // the timer brackets runs of these launches (all alike): one event
            // pair per run of mvm_ev_every, or up to the batch's last of them
            if (!I->mvm_open && 2 * (I->mvm_ev_used + 1) <= I->mvm_ev.size()) {
                HIP_TRY(hipEventRecord(I->mvm_ev[2 * I->mvm_ev_used], st));
                I->mvm_open = true;
                I->mvm_run = 0;
            }
            launch_mvm_next(st, I->d.cm_dtype, I->stream_nt, I->d_cm_s[ms], I->d_run,
                            (int)I->seg.size(), I->n_act, x, sc.ypart, E, N, I->params);
            if (I->mvm_open && (++I->mvm_run == I->mvm_ev_every || f + 2 >= n_frames)) {
                HIP_TRY(hipEventRecord(I->mvm_ev[2 * I->mvm_ev_used + 1], st));
                I->mvm_ev_len[I->mvm_ev_used++] = I->mvm_run;
                I->mvm_open = false;
            }
        } else {
            launch_mvm(st, I->d.cm_dtype, I->stream_nt, I->d_cm_s[ms], I->d_run, 0,
                       (int)I->seg.size(), I->n_act, x, sc.ypart, E);
        }
        enqueue_polc(I, st, ms, sc.ppart, sc.count_m);
        if (f + 1 < n_frames) TRY(copy_out(f + 1));
        I->next_frame++;
    }
    return last_error(e);
}


// =========================================================================
extern "C" {

const char *rtc_strerror(rtc_status s) {
    switch (s) {
    case RTC_OK: return "ok";
    case RTC_E_INVAL: return "invalid argument";
    case RTC_E_NOMEM: return "out of memory";
    case RTC_E_DEVICE: return "device error";
    case RTC_E_TIMEOUT: return "timeout";
    case RTC_E_STATE: return "invalid state";
    case RTC_E_RING_FULL: return "pixel ring full";
    case RTC_E_FRAME_DROPPED: return "frame dropped";
    case RTC_E_SCRATCH: return "work exceeds the static scratch";
    }
    return "unknown status";
}

rtc_status rtc_create(const rtc_create_desc *desc, rtc_engine **out) {
    if (!desc || !out) return RTC_E_INVAL;
    *out = nullptr;
    if (desc->n_inst < 1 || desc->n_inst > RTC_MAX_INST || !desc->inst) return RTC_E_INVAL;
    if (desc->ring_depth < 2 || desc->ring_depth > 64) return RTC_E_INVAL;
    if (desc->mode != RTC_MODE_STREAM && desc->mode != RTC_MODE_PERSISTENT) return RTC_E_INVAL;
    for (int i = 0; i < desc->n_inst; ++i) {
        const rtc_instance_desc &d = desc->inst[i];
        if (d.n_wfs < 1 || d.n_wfs > RTC_MAX_WFS || !d.wfs || d.n_act < 1) return RTC_E_INVAL;
        if (d.cm_dtype < RTC_CM_F32 || d.cm_dtype > RTC_CM_FP8) return RTC_E_INVAL;
        if (!std::isfinite(d.gain) || !std::isfinite(d.leak)) return RTC_E_INVAL;
        for (int w = 0; w < d.n_wfs; ++w)
            if (validate_wfs(d.wfs[w]) != RTC_OK) return RTC_E_INVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || desc->device < 0 || desc->device >= ndev)
        return RTC_E_DEVICE;
    rtc_engine *e = new (std::nothrow) rtc_engine();
    if (!e) return RTC_E_NOMEM;
    e->device = desc->device;
    e->ring_depth = desc->ring_depth;
    e->mode = desc->mode;
    auto bail = [&](rtc_status s) {
        rtc_destroy(e);
        return s;
    };
    if (hipSetDevice(e->device) != hipSuccess) return bail(RTC_E_DEVICE);
    // the device address of the static scratch (rtc_process_frames_noalloc),
    // taken with the engine's device current: each device has its own copy
    {
        void *sp = nullptr;
        const hipError_t se = scratch_address(&sp);
        if (se != hipSuccess || sp == nullptr) {
            std::fprintf(stderr, "rtc: static scratch address: %s\n", hipGetErrorString(se));
            return bail(RTC_E_DEVICE);
        }
        e->scratch = static_cast<uint8_t *>(sp);
    }
    if (hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking) != hipSuccess)
        return bail(RTC_E_DEVICE);
    if (hipStreamCreateWithFlags(&e->up_stream, hipStreamNonBlocking) != hipSuccess)
        return bail(RTC_E_DEVICE);
    for (int k = 0; k < 2; ++k)
        if (hipEventCreateWithFlags(&e->up_done[k], hipEventDisableTiming) != hipSuccess)
            return bail(RTC_E_DEVICE);
    {
        void *q = nullptr;
        if (hipHostMalloc(&q, 2 * kUploadHalf, hipHostMallocDefault) != hipSuccess)
            return bail(RTC_E_NOMEM);
        e->pinned.push_back(q);
        e->h_up = static_cast<uint8_t *>(q);
    }
    for (int i = 0; i < desc->n_inst; ++i) {
        Instance *I = new (std::nothrow) Instance();
        if (!I) return bail(RTC_E_NOMEM);
        e->inst.push_back(I);
        I->d = desc->inst[i];
        I->d.wfs = nullptr;
        I->n_act = I->d.n_act;
        I->gain[0] = I->gain[1] = I->d.gain;
        I->leak[0] = I->leak[1] = I->d.leak;
        I->wfs.resize(I->d.n_wfs);
        for (int w = 0; w < I->d.n_wfs; ++w) {
            WfsState &S = I->wfs[w];
            S.d = desc->inst[i].wfs[w];
            if (S.d.kind == RTC_WFS_SH) {
                S.valid.assign(S.d.subap_valid, S.d.subap_valid + (size_t)S.d.nsub * S.d.nsub);
                S.d.subap_valid = nullptr;
            } else {
                S.valid.assign(S.d.pupil_valid,
                               S.d.pupil_valid + (size_t)S.d.pupil_px * S.d.pupil_px);
                S.d.pupil_valid = nullptr;
            }
        }
        rtc_status s = build_instance(e, I);
        if (s != RTC_OK) return bail(s);
        s = alloc_instance(e, I);
        if (s != RTC_OK) return bail(s);
    }
    // every instance streams its matrices each frame and they share the
    // Infinity Cache: beyond its size, stream them with non-temporal loads
    int64_t per_frame = 0;
    for (const Instance *I : e->inst) per_frame += I->cm_bytes + I->m_bytes;
    for (Instance *I : e->inst) I->stream_nt = per_frame > kCacheResidentBytes;
    if (e->mode == RTC_MODE_PERSISTENT) {
        rtc_status s = persist_alloc(e);
        if (s != RTC_OK) return bail(s);
    }
    *out = e;
    return RTC_OK;
}

rtc_status rtc_destroy(rtc_engine *e) {
    if (!e) return RTC_E_INVAL;
    (void)hipSetDevice(e->device);
    if (e->mode == RTC_MODE_PERSISTENT) {
        (void)persist_stop(e);
        persist_free(e);
    }
    if (e->stream) (void)hipStreamSynchronize(e->stream);
    for (Instance *I : e->inst) {
        for (auto &sl : I->slots)
            if (sl.done) (void)hipEventDestroy(sl.done);
        if (!I->mvm_ev.empty()) (void)hipDeviceSynchronize();   // timer events on user streams
        for (hipEvent_t ev : I->mvm_ev) (void)hipEventDestroy(ev);
        delete I;
    }
    if (e->up_stream) (void)hipStreamSynchronize(e->up_stream);
    for (auto &b : e->allocs) (void)hipFree(b.p);
    for (void *p : e->pinned) (void)hipHostFree(p);
    for (hipEvent_t ev : e->up_done)
        if (ev) (void)hipEventDestroy(ev);
    if (e->up_stream) (void)hipStreamDestroy(e->up_stream);
    if (e->stream) (void)hipStreamDestroy(e->stream);
    delete e;
    return RTC_OK;
}

rtc_status rtc_get_info(rtc_engine *e, int32_t inst, rtc_instance_info *info) {
    Instance *I;
    TRY(check(e, inst, &I));
    if (!info) return RTC_E_INVAL;
    info->n_wfs = (int)I->wfs.size();
    info->n_units = I->n_units;
    info->n_slopes = I->n_slopes;
    info->n_act = I->n_act;
    info->n_kblocks = (int)I->kb.size();
    info->mask_words = I->mask_words;
    info->cm_bytes = I->cm_bytes;
    info->cm_bytes_logical = (int64_t)I->n_act * I->n_slopes * elem_size(I->d.cm_dtype) +
                             (I->d.cm_dtype == RTC_CM_FP8 ? 4LL * I->n_act : 0);
    info->polc_bytes = I->m_bytes;
    return RTC_OK;
}

rtc_status rtc_chunk_rows(rtc_engine *e, int32_t inst, int32_t wfs, int32_t chunk,
                          int32_t *row_begin, int32_t *row_end) {
    Instance *I;
    TRY(check(e, inst, &I));
    if (wfs < 0 || wfs >= (int)I->wfs.size()) return RTC_E_INVAL;
    const WfsState &S = I->wfs[wfs];
    if (chunk < 0 || chunk >= S.d.n_chunks || !row_begin || !row_end) return RTC_E_INVAL;
    *row_begin = S.row0[chunk];
    *row_end = S.row0[chunk + 1];
    return RTC_OK;
}

rtc_status rtc_load_matrices(rtc_engine *e, int32_t inst, const float *R, const double *D,
                             const float *M) {
    Instance *I;
    TRY(check(e, inst, &I));
    if (!R) return RTC_E_INVAL;
    if (I->d.polc && !D && !M) return RTC_E_INVAL;
    HIP_TRY(hipSetDevice(e->device));
    if (e->mode == RTC_MODE_PERSISTENT) TRY(persist_quiesce(e));
    HIP_TRY(hipDeviceSynchronize());
    // any staged or pending swap is dropped; the matrices go to the active slot
    I->m_staged = false;
    I->m_pending = false;
    TRY(put_matrices(e, I, I->m_active, R, D, M));
    const int na = I->n_act;
    HIP_TRY(hipMemset(I->d_p, 0, (size_t)na * 4));
    HIP_TRY(hipMemset(I->d_count, 0, (size_t)I->n_tiles * kCountStride * 4));
    HIP_TRY(hipMemset(I->d_a, 0, (size_t)I->a_len * 4));
    HIP_TRY(hipMemset(I->d_spad, 0, (size_t)I->spad_len * 4));
    HIP_TRY(hipMemset(I->d_spad2, 0, (size_t)I->spad_len * 4));
    I->next_frame = 0;
    I->seq = 0;
    I->cur_frame = ~0ull;
    I->cur_started = false;
    if (e->mode == RTC_MODE_PERSISTENT) persist_reset(I);
    I->loaded = true;
    return RTC_OK;
}

rtc_status rtc_stage_matrices(rtc_engine *e, int32_t inst, const float *R, const double *D,
                              const float *M) {
    Instance *I;
    TRY(check(e, inst, &I));
    if (!R) return RTC_E_INVAL;
    if (I->d.polc && !D && !M) return RTC_E_INVAL;
    HIP_TRY(hipSetDevice(e->device));
    int slot;
    {
        std::lock_guard<std::mutex> lk(I->mu);
        if (!I->loaded || I->m_pending) return RTC_E_STATE;
        slot = 1 - I->m_active;
        I->m_staged = false;
    }
    const bool serving = e->mode == RTC_MODE_PERSISTENT && e->pe.running && e->pe.serving;
    // the FP64 product M = R.D allocates and synchronises the device
    if (I->d.polc && !M && serving) return RTC_E_STATE;
    // frames still streaming the inactive slot (those before the last swap)
    // must be done before it is overwritten
    if (e->mode == RTC_MODE_PERSISTENT)
        TRY(persist_wait_matrix_free(e, I));
    else
        HIP_TRY(hipDeviceSynchronize());
    TRY(put_matrices(e, I, slot, R, M ? nullptr : D, M));
    std::lock_guard<std::mutex> lk(I->mu);
    I->m_staged = true;
    return RTC_OK;
}

rtc_status rtc_swap_matrices(rtc_engine *e, int32_t inst, uint64_t *f_eff_out) {
    Instance *I;
    TRY(check(e, inst, &I));
    std::lock_guard<std::mutex> lk(I->mu);
    if (!I->m_staged || I->m_pending) return RTC_E_STATE;
    uint64_t f = I->next_frame;
    if (I->cur_frame != ~0ull && I->cur_started) f = std::max(f, I->cur_frame + 1);
    I->m_switch = f;
    I->m_pending = true;
    if (f_eff_out) *f_eff_out = f;
    if (e->mode == RTC_MODE_PERSISTENT) {
        PersistInstState &P = I->ps;
        persist_mswap(I, I->cur_started ? P.q_cur + 1 : P.seq, 1 - I->m_active);
    }
    return RTC_OK;
}

rtc_status rtc_telemetry_enable(rtc_engine *e, int32_t inst, int32_t decimation,
                                int32_t n_slots) {
    Instance *I;
    TRY(check(e, inst, &I));
    auto pow2 = [](int32_t v) { return v > 0 && (v & (v - 1)) == 0; };
    if (!pow2(decimation) || decimation > 65536 || n_slots < 0 || n_slots > 65536 ||
        (n_slots > 0 && !pow2(n_slots)))
        return RTC_E_INVAL;
    if (e->mode != RTC_MODE_PERSISTENT) return RTC_E_STATE;
    HIP_TRY(hipSetDevice(e->device));
    TRY(persist_quiesce(e));
    std::lock_guard<std::mutex> lk(I->mu);
    return persist_telemetry(e, I, decimation, n_slots);
}

rtc_status rtc_telemetry_next(rtc_engine *e, int32_t inst, float *slopes, int32_t *counts,
                              float *cmds, uint64_t *masks, int64_t timeout_ns,
                              rtc_telemetry_info *info) {
    Instance *I;
    TRY(check(e, inst, &I));
    if (e->mode != RTC_MODE_PERSISTENT) return RTC_E_STATE;
    return persist_telemetry_next(e, I, slopes, counts, cmds, masks, timeout_ns, info);
}

rtc_status rtc_load_calibration(rtc_engine *e, int32_t inst, int32_t wfs, const float *dark,
                                const float *flat, const float *bg, const float *thr,
                                const float *ref) {
    Instance *I;
    TRY(check(e, inst, &I));
    if (wfs < 0 || wfs >= (int)I->wfs.size()) return RTC_E_INVAL;
    HIP_TRY(hipSetDevice(e->device));
    if (e->mode == RTC_MODE_PERSISTENT) TRY(persist_quiesce(e));
    HIP_TRY(hipDeviceSynchronize());
    WfsState &S = I->wfs[wfs];
    const int W = S.d.frame_w;
    auto pick = [](const float *m, size_t idx, float dflt) { return m ? m[idx] : dflt; };
    if (S.d.kind == RTC_WFS_SH) {
        const int p = S.d.px;
        const int n = S.u1 - S.u0;
        std::vector<float> dk((size_t)n * p * p), fl(dk.size()), bgv(dk.size()), th(n);
        for (int k = 0; k < n; ++k) {
            const ShUnit &u = I->sh[S.kind0 + k];
            for (int i = 0; i < p * p; ++i) {
                const size_t idx = (size_t)(u.row0 + i / p) * W + (u.col0 + i % p);
                dk[(size_t)k * p * p + i] = pick(dark, idx, 0.0f);
                fl[(size_t)k * p * p + i] = pick(flat, idx, 1.0f);
                bgv[(size_t)k * p * p + i] = pick(bg, idx, 0.0f);
            }
            th[k] = pick(thr, k, 0.0f);
        }
        const size_t off = I->sh[S.kind0].cal;
        HIP_TRY(hipMemcpy(I->d_sh_dark + off, dk.data(), dk.size() * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(I->d_sh_flat + off, fl.data(), fl.size() * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(I->d_sh_bg + off, bgv.data(), bgv.size() * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(I->d_sh_thr + S.kind0, th.data(), th.size() * 4, hipMemcpyHostToDevice));
    } else {
        const int n = S.u1 - S.u0;
        const int np = I->n_pyr;
        std::vector<float> dk(4 * (size_t)np), fl(dk.size()), bgv(dk.size());
        HIP_TRY(hipMemcpy(dk.data(), I->d_py_dark, dk.size() * 4, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(fl.data(), I->d_py_flat, fl.size() * 4, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(bgv.data(), I->d_py_bg, bgv.size() * 4, hipMemcpyDeviceToHost));
        std::vector<float> th(n, pick(thr, 0, 0.0f));
        for (int k = 0; k < n; ++k) {
            const PyrUnit &u = I->py[S.kind0 + k];
            for (int q = 0; q < 4; ++q) {
                const size_t idx = (size_t)(S.d.quad_row[q] + u.i) * W + (S.d.quad_col[q] + u.j);
                dk[(size_t)q * np + S.kind0 + k] = pick(dark, idx, 0.0f);
                fl[(size_t)q * np + S.kind0 + k] = pick(flat, idx, 1.0f);
                bgv[(size_t)q * np + S.kind0 + k] = pick(bg, idx, 0.0f);
            }
        }
        HIP_TRY(hipMemcpy(I->d_py_dark, dk.data(), dk.size() * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(I->d_py_flat, fl.data(), fl.size() * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(I->d_py_bg, bgv.data(), bgv.size() * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(I->d_py_thr + S.kind0, th.data(), th.size() * 4, hipMemcpyHostToDevice));
    }
    std::vector<float> rf(2 * (size_t)(S.u1 - S.u0));
    for (size_t i = 0; i < rf.size(); ++i) rf[i] = pick(ref, i, 0.0f);
    HIP_TRY(hipMemcpy(I->d_ref + 2 * S.u0, rf.data(), rf.size() * 4, hipMemcpyHostToDevice));
    return RTC_OK;
}

rtc_status rtc_set_params(rtc_engine *e, int32_t inst, float gain, float leak,
                          uint64_t *f_eff_out) {
    Instance *I;
    TRY(check(e, inst, &I));
    if (!std::isfinite(gain) || !std::isfinite(leak)) return RTC_E_INVAL;
    std::lock_guard<std::mutex> lk(I->mu);
    // a still-pending change is replaced; the staged slot is the inactive one
    const int s = 1 - I->active;
    I->gain[s] = gain;
    I->leak[s] = leak;
    uint64_t f = I->next_frame;
    if (I->cur_frame != ~0ull && I->cur_started) f = std::max(f, I->cur_frame + 1);
    I->f_switch = f;
    I->pending = true;
    if (f_eff_out) *f_eff_out = f;
    if (e->mode == RTC_MODE_PERSISTENT) TRY(persist_params(e, I));
    return RTC_OK;
}

rtc_status rtc_get_state(rtc_engine *e, int32_t inst, float *a, float *p, uint64_t *next_frame) {
    Instance *I;
    TRY(check(e, inst, &I));
    HIP_TRY(hipSetDevice(e->device));
    if (e->mode == RTC_MODE_PERSISTENT) TRY(persist_quiesce(e));
    HIP_TRY(hipDeviceSynchronize());
    if (a) HIP_TRY(hipMemcpy(a, I->d_a, I->n_act * 4, hipMemcpyDeviceToHost));
    if (p) HIP_TRY(hipMemcpy(p, I->d_p, I->n_act * 4, hipMemcpyDeviceToHost));
    if (next_frame) *next_frame = I->next_frame;
    return RTC_OK;
}

rtc_status rtc_set_state(rtc_engine *e, int32_t inst, const float *a, const float *p,
                         uint64_t next_frame) {
    Instance *I;
    TRY(check(e, inst, &I));
    HIP_TRY(hipSetDevice(e->device));
    if (e->mode == RTC_MODE_PERSISTENT) TRY(persist_quiesce(e));
    HIP_TRY(hipDeviceSynchronize());
    std::lock_guard<std::mutex> lk(I->mu);
    if (e->mode == RTC_MODE_PERSISTENT) persist_reset(I);
    HIP_TRY(hipMemset(I->d_a, 0, (size_t)I->a_len * 4));
    if (a) HIP_TRY(hipMemcpy(I->d_a, a, I->n_act * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(I->d_p, 0, (size_t)I->n_act * 4));
    if (p && I->d.polc) HIP_TRY(hipMemcpy(I->d_p, p, I->n_act * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(I->d_count, 0, (size_t)I->n_tiles * kCountStride * 4));
    I->next_frame = next_frame;
    I->seq = 0;
    I->cur_frame = ~0ull;
    I->cur_started = false;
    for (auto &sl : I->slots) {
        sl.frame = ~0ull;
        sl.complete = false;
        sl.dropped = false;
    }
    for (auto &W : I->wfs) {
        W.next_chunk = 0;
        W.acquired = -1;
    }
    return RTC_OK;
}

rtc_status rtc_process_frames(rtc_engine *e, int32_t inst, const uint16_t *const *frames,
                              const int64_t *frame_stride, int32_t n_frames, float *cmds,
                              float *slopes, int32_t *counts, void *stream) {
    Instance *I;
    TRY(check(e, inst, &I));
    if (!I->loaded) return RTC_E_STATE;
    if (!frames || !frame_stride || n_frames < 0) return RTC_E_INVAL;
    for (size_t w = 0; w < I->wfs.size(); ++w) {
        if (!frames[w]) return RTC_E_INVAL;
        if (n_frames > 1 && frame_stride[w] < (int64_t)I->wfs[w].d.frame_h * I->wfs[w].d.frame_w)
            return RTC_E_INVAL;
    }
    HIP_TRY(hipSetDevice(e->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(I->mu);
    if (e->mode == RTC_MODE_PERSISTENT) {
        if (I->cur_started) return RTC_E_STATE;
        TRY(persist_batch(e, I, frames, frame_stride, n_frames, cmds, slopes, counts, st));
        return last_error(e);
    }
    return process_frames_stream(e, I, frames, frame_stride, n_frames, cmds, slopes, counts, st,
                                 engine_scratch(I));
}

rtc_status rtc_process_frames_noalloc(rtc_engine *e, int32_t inst, const uint16_t *const *frames,
                                      const int64_t *frame_stride, int32_t n_frames,
                                      float *cmds, float *slopes, int32_t *counts,
                                      void *stream) {
    Instance *I;
    TRY(check(e, inst, &I));
    if (!I->loaded) return RTC_E_STATE;
    if (e->mode != RTC_MODE_STREAM) return RTC_E_STATE;
    if (!frames || !frame_stride || n_frames < 0) return RTC_E_INVAL;
    for (size_t w = 0; w < I->wfs.size(); ++w) {
        if (!frames[w]) return RTC_E_INVAL;
        if (n_frames > 1 && frame_stride[w] < (int64_t)I->wfs[w].d.frame_h * I->wfs[w].d.frame_w)
            return RTC_E_INVAL;
    }
    // carve the static scratch: partials, then counters, each 256-byte aligned
    auto up256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t n_cnt = (size_t)I->n_tiles * kCountStride;
    const size_t b_ypart = up256(I->seg.size() * (size_t)I->n_act * 4);
    const size_t b_ppart = I->d.polc ? up256(I->segm.size() * (size_t)I->n_act * 4) : 0;
    const size_t b_cnt = up256(n_cnt * 4);
    if (b_ypart + b_ppart + 2 * b_cnt > kScratchBytes) return RTC_E_SCRATCH;
    MvmScratch sc;
    sc.ypart = reinterpret_cast<float *>(e->scratch);
    sc.ppart = I->d.polc ? reinterpret_cast<float *>(e->scratch + b_ypart) : nullptr;
    sc.count = reinterpret_cast<uint32_t *>(e->scratch + b_ypart + b_ppart);
    sc.count_m = reinterpret_cast<uint32_t *>(e->scratch + b_ypart + b_ppart + b_cnt);
    HIP_TRY(hipSetDevice(e->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(I->mu);
    // the array keeps the last call's contents (an earlier call may also have
    // stopped half way): the counters start from zero, by a kernel
    launch_fill_u32(st, sc.count, 2 * b_cnt / 4, 0u);
    return process_frames_stream(e, I, frames, frame_stride, n_frames, cmds, slopes, counts, st,
                                 sc);
}

rtc_status rtc_run_mvm(rtc_engine *e, int32_t inst, int32_t n_iter, void *stream) {
    Instance *I;
    TRY(check(e, inst, &I));
    if (!I->loaded) return RTC_E_STATE;
    if (n_iter < 0) return RTC_E_INVAL;
    HIP_TRY(hipSetDevice(e->device));
    if (e->mode == RTC_MODE_PERSISTENT) TRY(persist_quiesce(e));
    hipStream_t st = static_cast<hipStream_t>(stream);
    MvmEpilogue E{};
    E.mode = EPI_REDUCE;
    E.n_parts = (int)I->seg.size();
    E.seg_ends = I->d_seg_ends;
    E.count = I->d_count_t;
    E.y = I->d_yscratch;
    std::lock_guard<std::mutex> lk(I->mu);
    for (int i = 0; i < n_iter; ++i)
        launch_mvm(st, I->d.cm_dtype, I->stream_nt, I->d_cm_s[I->m_active], I->d_run, 0,
                   (int)I->seg.size(), I->n_act, I->d_spad, I->d_ypart, E);
    return last_error(e);
}

rtc_status rtc_mvm_timing(rtc_engine *e, int32_t inst, int32_t capacity, int32_t every) {
    Instance *I;
    TRY(check(e, inst, &I));
    if (e->mode != RTC_MODE_STREAM) return RTC_E_STATE;
    if (capacity < 0 || capacity > (1 << 20) || every < 1) return RTC_E_INVAL;
    HIP_TRY(hipSetDevice(e->device));
    std::lock_guard<std::mutex> lk(I->mu);
    HIP_TRY(hipDeviceSynchronize());     // no recorded event may still be pending
    for (hipEvent_t ev : I->mvm_ev) HIP_TRY(hipEventDestroy(ev));
    I->mvm_ev.clear();
    I->mvm_ev_len.assign((size_t)capacity, 0);
    I->mvm_ev_used = 0;
    I->mvm_ev_every = every;
    I->mvm_open = false;
    for (int32_t k = 0; k < 2 * capacity; ++k) {
        hipEvent_t ev;
        HIP_TRY(hipEventCreate(&ev));
        I->mvm_ev.push_back(ev);
    }
    return RTC_OK;
}

rtc_status rtc_mvm_timing_read(rtc_engine *e, int32_t inst, int32_t *n, double *total_ms) {
    Instance *I;
    TRY(check(e, inst, &I));
    if (e->mode != RTC_MODE_STREAM) return RTC_E_STATE;
    HIP_TRY(hipSetDevice(e->device));
    std::lock_guard<std::mutex> lk(I->mu);
    double tot = 0.0;
    int32_t launches = 0;
    if (I->mvm_ev_used > 0) HIP_TRY(hipEventSynchronize(I->mvm_ev[2 * I->mvm_ev_used - 1]));
    for (size_t k = 0; k < I->mvm_ev_used; ++k) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, I->mvm_ev[2 * k], I->mvm_ev[2 * k + 1]));
        tot += ms;
        launches += I->mvm_ev_len[k];
    }
    if (n) *n = launches;
    if (total_ms) *total_ms = tot;
    I->mvm_ev_used = 0;
    return RTC_OK;
}

rtc_status rtc_trace_enable(rtc_engine *e, int32_t n_frames) {
    if (e == nullptr) return RTC_E_INVAL;
    if (e->mode != RTC_MODE_PERSISTENT || e->pe.running) return RTC_E_STATE;
    if (n_frames < 0 || n_frames > kMaxTraceFrames) return RTC_E_INVAL;
    HIP_TRY(hipSetDevice(e->device));
    HIP_TRY(hipDeviceSynchronize());     // no batch launch may still write the record
    return persist_trace(e, n_frames);
}

rtc_status rtc_trace_read(rtc_engine *e, uint64_t *out, int64_t capacity, int32_t *n_waves,
                          int32_t *n_frames) {
    if (e == nullptr) return RTC_E_INVAL;
    if (e->mode != RTC_MODE_PERSISTENT) return RTC_E_STATE;
    const int waves = e->pe.trace_waves;
    const int64_t n = (int64_t)e->pe.trace_frames * waves * RTC_TRACE_EVENTS;
    if (n_waves) *n_waves = waves;
    if (n_frames) *n_frames = e->pe.trace_frames;
    if (out == nullptr || n == 0) return RTC_OK;
    if (capacity < n) return RTC_E_INVAL;
    HIP_TRY(hipSetDevice(e->device));
    TRY(persist_quiesce(e));             // a serving loop never ends on its own soon
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(out, e->pe.trace, (size_t)n * 8, hipMemcpyDeviceToHost));
    return RTC_OK;
}

rtc_status rtc_read_slopes(rtc_engine *e, int32_t inst, float *slopes, int32_t *counts,
                           uint64_t *masks) {
    Instance *I;
    TRY(check(e, inst, &I));
    if (e->mode == RTC_MODE_PERSISTENT) return RTC_E_STATE;
    HIP_TRY(hipSetDevice(e->device));
    HIP_TRY(hipDeviceSynchronize());
    if (slopes) HIP_TRY(hipMemcpy(slopes, I->d_sout, I->n_slopes * 4, hipMemcpyDeviceToHost));
    if (counts) HIP_TRY(hipMemcpy(counts, I->d_counts, I->n_units * 4, hipMemcpyDeviceToHost));
    if (masks)
        HIP_TRY(hipMemcpy(masks, I->d_masks, (size_t)I->mask_words * 8, hipMemcpyDeviceToHost));
    return RTC_OK;
}

rtc_status rtc_read_matrix(rtc_engine *e, int32_t inst, void *codes, float *scales) {
    Instance *I;
    TRY(check(e, inst, &I));
    if (!I->loaded) return RTC_E_STATE;
    HIP_TRY(hipSetDevice(e->device));
    HIP_TRY(hipStreamSynchronize(e->stream));
    if (codes) {
        std::vector<uint8_t> enc((size_t)I->cm_bytes);
        HIP_TRY(hipMemcpy(enc.data(), I->d_cm_s[I->m_active], enc.size(), hipMemcpyDeviceToHost));
        const int es = elem_size(I->d.cm_dtype), E = 16 / es;
        const int ns = I->n_slopes;
        uint8_t *dst = static_cast<uint8_t *>(codes);
        const int n_tiles = (I->n_act + kTileRows - 1) / kTileRows;
        for (int t = 0; t < n_tiles; ++t) {
            const int nr = std::min(kTileRows, I->n_act - t * kTileRows);
            for (const KBlock &K : I->kb) {
                const uint8_t *blk = enc.data() + K.base + (int64_t)t * kTileRows * K.kv * 16;
                for (int l = 0; l < nr; ++l) {
                    const int r = t * kTileRows + l;
                    for (int c = 0; c < K.k; ++c) {
                        const int v = c / E, el = c % E;
                        std::memcpy(dst + ((size_t)r * ns + K.k0 + c) * es,
                                    blk + ((size_t)v * nr + l) * 16 + el * es, es);
                    }
                }
            }
        }
    }
    if (scales)
        HIP_TRY(hipMemcpy(scales, I->d_scale_s[I->m_active], I->n_act * 4, hipMemcpyDeviceToHost));
    return RTC_OK;
}

// ------------------------------------------------------------- serving (stream mode)
rtc_status rtc_acquire_chunk(rtc_engine *e, int32_t inst, int32_t wfs, uint64_t frame,
                             int32_t chunk, uint16_t **rows, int32_t *pitch) {
    Instance *I;
    TRY(check(e, inst, &I));
    if (e->mode != RTC_MODE_PERSISTENT || !I->loaded) return RTC_E_STATE;
    if (wfs < 0 || wfs >= (int)I->wfs.size() || !rows || !pitch) return RTC_E_INVAL;
    if (chunk < 0 || chunk >= I->wfs[wfs].d.n_chunks) return RTC_E_INVAL;
    std::lock_guard<std::mutex> lk(I->mu);
    return persist_acquire(e, I, wfs, frame, chunk, rows, pitch);
}

rtc_status rtc_commit_chunk(rtc_engine *e, int32_t inst, int32_t wfs, uint64_t frame,
                            int32_t chunk) {
    const int64_t t_in = now_ns();
    Instance *I;
    TRY(check(e, inst, &I));
    if (e->mode != RTC_MODE_PERSISTENT || !I->loaded) return RTC_E_STATE;
    if (wfs < 0 || wfs >= (int)I->wfs.size()) return RTC_E_INVAL;
    std::lock_guard<std::mutex> lk(I->mu);
    return persist_commit(e, I, wfs, frame, chunk, t_in);
}

rtc_status rtc_submit_pixel_chunk(rtc_engine *e, int32_t inst, int32_t wfs, uint64_t frame,
                                  int32_t chunk, const uint16_t *rows) {
    const int64_t t_in = now_ns();
    Instance *I;
    TRY(check(e, inst, &I));
    if (!I->loaded) return RTC_E_STATE;
    if (wfs < 0 || wfs >= (int)I->wfs.size() || !rows) return RTC_E_INVAL;
    WfsState &S = I->wfs[wfs];
    if (chunk < 0 || chunk >= S.d.n_chunks) return RTC_E_INVAL;
    std::lock_guard<std::mutex> lk(I->mu);
    if (e->mode == RTC_MODE_PERSISTENT) return persist_submit(e, I, wfs, frame, chunk, rows, t_in);
    if (I->cur_frame != ~0ull && frame < I->cur_frame) return RTC_E_FRAME_DROPPED;
    if (frame < I->next_frame) return RTC_E_FRAME_DROPPED;
    if (I->cur_frame == ~0ull || frame > I->cur_frame) {
        if (I->cur_frame != ~0ull && I->cur_started) {
            // the frame in progress never completed: drop it
            FrameSlot &old = I->slots[I->cur_frame % I->slots.size()];
            old.dropped = true;
            I->drops++;
            // its column blocks left partial arrival counts behind
            HIP_TRY(hipMemsetAsync(I->d_count, 0, (size_t)I->n_tiles * kCountStride * 4, e->stream));
        }
        FrameSlot &sl = I->slots[frame % I->slots.size()];
        if (sl.frame != ~0ull) {
            if (sl.complete) {
                const hipError_t q = hipEventQuery(sl.done);
                if (q == hipErrorNotReady) return RTC_E_RING_FULL;
                if (q != hipSuccess) return fail(e, RTC_E_DEVICE);
            } else {
                // an abandoned frame may still have copies in flight from this slot
                HIP_TRY(hipStreamSynchronize(e->stream));
            }
        }
        I->cur_frame = frame;
        I->cur_started = false;
        for (auto &W : I->wfs) W.next_chunk = 0;
        coeffs(I, frame, &I->frame_c1, &I->frame_g);
        I->frame_mslot = mat_slot(I, frame);
        I->frame_seq = I->seq++;
        sl.frame = frame;
        sl.complete = false;
        sl.dropped = false;
    }
    if (chunk != S.next_chunk) return RTC_E_INVAL;
    I->cur_started = true;
    HIP_TRY(hipSetDevice(e->device));
    const int slot = (int)(frame % (uint64_t)e->ring_depth);
    const size_t fpx = (size_t)S.d.frame_h * S.d.frame_w;
    const int r0 = S.row0[chunk], r1 = S.row0[chunk + 1];
    const size_t off = (size_t)slot * fpx + (size_t)r0 * S.d.frame_w;
    const size_t n = (size_t)(r1 - r0) * S.d.frame_w;
    std::memcpy(S.h_stage + off, rows, n * 2);
    HIP_TRY(hipMemcpyAsync(S.d_ring + off, S.h_stage + off, n * 2, hipMemcpyHostToDevice,
                           e->stream));
    const int kb = S.kb_of_chunk[chunk];
    if (kb >= 0) {
        const KBlock &K = I->kb[kb];
        FrameSet fs{};
        for (size_t w = 0; w < I->wfs.size(); ++w)
            fs.f[w] = I->wfs[w].d_ring + (size_t)slot * I->wfs[w].d.frame_h * I->wfs[w].d.frame_w;
        const int ub = K.k0 / 2, ue = (K.k0 + K.k) / 2;
        enqueue_centroid(I, e->stream, fs, wfs, ub, ue);
        launch_mvm(e->stream, I->d.cm_dtype, I->stream_nt, I->d_cm_s[I->frame_mslot], I->d_run,
                   I->kb_seg0[kb], I->kb_nseg[kb], I->n_act, I->d_spad, I->d_ypart,
                   integrate_epi(I, I->frame_mslot, I->frame_seq, I->frame_c1, I->frame_g,
                                 nullptr, I->d_count));
    }
    S.next_chunk++;
    bool all = true;
    for (auto &W : I->wfs) all = all && W.next_chunk == W.d.n_chunks;
    if (all) {
        FrameSlot &sl = I->slots[frame % I->slots.size()];
        float *mail = I->h_mail + (size_t)slot * I->n_act;
        settle_params(I, frame);
        settle_matrices(I, frame);
        HIP_TRY(hipMemcpyAsync(mail, I->d_a, I->n_act * 4, hipMemcpyDeviceToHost, e->stream));
        HIP_TRY(hipEventRecord(sl.done, e->stream));
        enqueue_polc(I, e->stream, I->frame_mslot, I->d_ppart, I->d_count_m);
        sl.t_last_chunk = t_in;
        sl.complete = true;
        I->next_frame = frame + 1;
        I->cur_started = false;
        I->cur_frame = ~0ull;
    }
    return last_error(e);
}

rtc_status rtc_wait_commands(rtc_engine *e, int32_t inst, uint64_t frame, float *cmds,
                             int64_t timeout_ns, rtc_frame_info *info) {
    Instance *I;
    TRY(check(e, inst, &I));
    if (!cmds) return RTC_E_INVAL;
    if (e->mode == RTC_MODE_PERSISTENT) return persist_wait(e, I, frame, cmds, timeout_ns, info);
    const int64_t t0 = now_ns();
    FrameSlot *sl = &I->slots[frame % I->slots.size()];
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(I->mu);
            if (sl->frame == frame && sl->dropped) return RTC_E_FRAME_DROPPED;
            if (sl->frame == frame && sl->complete) break;
            if (sl->frame != ~0ull && sl->frame > frame) return RTC_E_FRAME_DROPPED;
        }
        if (now_ns() - t0 > timeout_ns) return RTC_E_TIMEOUT;
        std::this_thread::yield();
    }
    for (;;) {
        const hipError_t q = hipEventQuery(sl->done);
        if (q == hipSuccess) break;
        if (q != hipErrorNotReady) return fail(e, RTC_E_DEVICE);
        if (now_ns() - t0 > timeout_ns) return RTC_E_TIMEOUT;
    }
    const int64_t t_ready = now_ns();
    const int slot = (int)(frame % (uint64_t)e->ring_depth);
    std::memcpy(cmds, I->h_mail + (size_t)slot * I->n_act, I->n_act * 4);
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->frame = frame;
        info->t_last_chunk_ns = sl->t_last_chunk;
        info->t_ready_ns = t_ready;
        info->drops = I->drops;
    }
    return RTC_OK;
}

}  // extern "C"
