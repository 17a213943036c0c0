// Paced camera-stream driver (rtc_pacer.h): a producer thread that submits
// chunks on a busy-waited schedule and one waiter thread per instance, pinned
// to cores, so that serving latency is measured without the caller's own
// scheduling in it.
#include <pthread.h>
#include <sched.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "rtc.h"
#include "rtc_engine.h"
#include "rtc_pacer.h"

namespace {

int64_t mono_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

// The k-th CPU this process may run on (-1 if there are fewer).
int allowed_cpu(int k) {
    cpu_set_t set;
    CPU_ZERO(&set);
    if (sched_getaffinity(0, sizeof(set), &set) != 0) return -1;
    for (int c = 0, seen = 0; c < CPU_SETSIZE; ++c)
        if (CPU_ISSET(c, &set) && seen++ == k) return c;
    return -1;
}

void pin_to(int cpu) {
    if (cpu < 0) return;
    cpu_set_t set;
    CPU_ZERO(&set);
    CPU_SET(cpu, &set);
    (void)pthread_setaffinity_np(pthread_self(), sizeof(set), &set);
}

struct Chunk {
    int64_t at_ns;       // offset from the frame start
    int stream, wfs, chunk, row0, row1;
    bool completes;      // the chunk completes a column block (some slope needs its rows)
};

}  // namespace

extern "C" rtc_status rtc_pacer_run(rtc_engine *e, const rtc_pacer_desc *d, int32_t n_streams,
                                    const rtc_pacer_stream *streams, rtc_pacer_sample *out,
                                    int32_t *failed_frame) {
    if (!e || !d || !streams || !out || n_streams < 1) return RTC_E_INVAL;
    if (d->n_frames < 1 || d->warmup < 0 || d->warmup >= d->n_frames || d->period_s <= 0 ||
        d->readout_s < 0 || d->timeout_s <= 0)
        return RTC_E_INVAL;
    if (e->mode != RTC_MODE_PERSISTENT) return RTC_E_STATE;
    if (failed_frame) *failed_frame = -1;
    // the readout plan of one frame, every sensor in parallel
    std::vector<Chunk> plan;
    std::vector<int32_t> n_act(n_streams);
    for (int s = 0; s < n_streams; ++s) {
        const rtc_pacer_stream &S = streams[s];
        if (S.inst < 0 || S.inst >= (int)e->inst.size() || S.n_bank < 1 || !S.banks)
            return RTC_E_INVAL;
        const Instance *I = e->inst[S.inst];
        if (!I->loaded) return RTC_E_STATE;
        n_act[s] = I->n_act;
        for (int w = 0; w < (int)I->wfs.size(); ++w) {
            if (!S.banks[w]) return RTC_E_INVAL;
            const int n = I->wfs[w].d.n_chunks;
            for (int c = 0; c < n; ++c)
                plan.push_back(Chunk{(int64_t)std::llround(1e9 * d->readout_s * (c + 1) / n), s, w,
                                     c, I->wfs[w].row0[c], I->wfs[w].row0[c + 1],
                                     I->wfs[w].kb_of_chunk[c] >= 0});
        }
    }
    std::stable_sort(plan.begin(), plan.end(), [](const Chunk &a, const Chunk &b) {
        return a.at_ns != b.at_ns ? a.at_ns < b.at_ns
                                  : (a.stream != b.stream ? a.stream < b.stream : a.wfs < b.wfs);
    });
    const int n_rec = d->n_frames - d->warmup;
    const int64_t period = (int64_t)std::llround(1e9 * d->period_s);
    // per stream and frame: lateness of the first and the last chunk
    std::vector<double> late_first((size_t)n_streams * d->n_frames, 0.0),
        late_last((size_t)n_streams * d->n_frames, 0.0);
    // per stream and frame: host clock of the last block-completing chunk's
    // hand-over and of the commands being seen
    std::vector<int64_t> t_complete((size_t)n_streams * d->n_frames, 0),
        t_last((size_t)n_streams * d->n_frames, 0),
        t_ready((size_t)n_streams * d->n_frames, 0);
    std::atomic<int> status{RTC_OK};
    std::atomic<int> failed{-1};
    auto fail_at = [&](rtc_status st, int f) {
        int ok = RTC_OK;
        if (status.compare_exchange_strong(ok, (int)st)) failed.store(f);
    };
    const int64_t t0 = mono_ns() + 2000000;   // 2 ms to start the threads
    std::thread producer([&]() {
        if (d->pin) pin_to(allowed_cpu(0));
        std::vector<int> first_of(n_streams);
        for (int f = 0; f < d->n_frames && status.load() == RTC_OK; ++f) {
            const uint64_t frame = d->first_frame + (uint64_t)f;
            if (d->switch_stream >= 0 && d->switch_stream < n_streams && f == d->switch_frame) {
                const rtc_status st = rtc_set_params(e, streams[d->switch_stream].inst,
                                                     d->switch_gain, d->switch_leak, nullptr);
                if (st != RTC_OK) {
                    fail_at(st, f);
                    break;
                }
            }
            const int64_t tf = t0 + (int64_t)f * period;
            std::fill(first_of.begin(), first_of.end(), 1);
            for (const Chunk &C : plan) {
                const int64_t due = tf + C.at_ns;
                int64_t now;
                while ((now = mono_ns()) < due) {
                }
                const rtc_pacer_stream &S = streams[C.stream];
                const Instance *I = e->inst[S.inst];
                const size_t k = (size_t)C.stream * d->n_frames + f;
                // the hand-over starts now (the library stamps its entry alike)
                const int64_t t_in = mono_ns();
                t_last[k] = t_in;
                if (C.completes) t_complete[k] = t_in;
                const rtc_wfs_desc &wd = I->wfs[C.wfs].d;
                const uint16_t *img = S.banks[C.wfs] + (size_t)(f % S.n_bank) * wd.frame_h * wd.frame_w;
                const uint16_t *rows = img + (size_t)C.row0 * wd.frame_w;
                rtc_status st;
                if (d->zero_copy) {
                    uint16_t *dst = nullptr;
                    int32_t pitch = 0;
                    st = rtc_acquire_chunk(e, S.inst, C.wfs, frame, C.chunk, &dst, &pitch);
                    if (st == RTC_OK) {
                        for (int r = 0; r < C.row1 - C.row0; ++r)
                            std::memcpy(dst + (size_t)r * pitch, rows + (size_t)r * wd.frame_w,
                                        (size_t)wd.frame_w * 2);
                        st = rtc_commit_chunk(e, S.inst, C.wfs, frame, C.chunk);
                    }
                } else {
                    st = rtc_submit_pixel_chunk(e, S.inst, C.wfs, frame, C.chunk, rows);
                }
                if (st != RTC_OK) {
                    fail_at(st, f);
                    break;
                }
                const double late = (double)(now - due) * 1e-3;
                if (first_of[C.stream]) {
                    late_first[k] = late;
                    first_of[C.stream] = 0;
                }
                late_last[k] = late;
            }
        }
    });
    std::vector<std::thread> waiters;
    for (int s = 0; s < n_streams; ++s) {
        waiters.emplace_back([&, s]() {
            if (d->pin) pin_to(allowed_cpu(1 + s));
            std::vector<float> cmds(n_act[s]);
            for (int f = 0; f < d->n_frames; ++f) {
                rtc_frame_info info;
                float *dst = (streams[s].cmds != nullptr && f >= d->warmup)
                                 ? streams[s].cmds + (size_t)(f - d->warmup) * n_act[s]
                                 : cmds.data();
                const rtc_status st =
                    rtc_wait_commands(e, streams[s].inst, d->first_frame + (uint64_t)f, dst,
                                      (int64_t)(1e9 * d->timeout_s), &info);
                if (status.load() != RTC_OK) return;
                if (st != RTC_OK) {
                    fail_at(st, f);
                    return;
                }
                if (f < d->warmup) continue;
                rtc_pacer_sample &o = out[(size_t)s * n_rec + (f - d->warmup)];
                o.frame = info.frame;
                t_ready[(size_t)s * d->n_frames + f] = info.t_ready_ns;
                o.dev_ticks_start = info.dev_ticks_start;
                o.dev_ticks_cmd = info.dev_ticks_cmd;
                o.dev_us = info.dev_ticks_start
                               ? ((double)info.dev_ticks_cmd - (double)info.dev_ticks_start) * 0.01
                               : -1.0;
            }
        });
    }
    producer.join();
    for (auto &t : waiters) t.join();
    // the pacer's lateness, once both sides are done with the frames
    for (int s = 0; s < n_streams; ++s)
        for (int i = 0; i < n_rec; ++i) {
            const size_t k = (size_t)s * d->n_frames + d->warmup + i;
            out[(size_t)s * n_rec + i].late_us = late_last[k];
            out[(size_t)s * n_rec + i].complete_us = (double)(t_ready[k] - t_complete[k]) * 1e-3;
            // negative when the commands were out before the last chunk was
            // handed over (its rows hold no pixel the frame needs)
            out[(size_t)s * n_rec + i].host_us = (double)(t_ready[k] - t_last[k]) * 1e-3;
            out[(size_t)s * n_rec + i].start_late_us = late_first[k];
        }
    if (failed_frame) *failed_frame = failed.load();
    return (rtc_status)status.load();
}
