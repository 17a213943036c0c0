/*
 * rtc_pacer.h - paced camera-stream driver for measuring serving latency.
 *
 * The paper measures latency from the arrival of a frame's last pixel to the
 * DM command being ready, with a camera simulator that streams each camera's
 * frame as packets spread over its readout (section 2.1: inter-packet and
 * inter-frame delays set independently; its own frame-time jitter is reported
 * beside the controller's, about 5 us RMS in steady periods).  This driver
 * plays that role for a serving engine (RTC_MODE_PERSISTENT): one producer
 * thread submits every sensor's chunks on a busy-waited monotonic-clock
 * schedule (all sensors read out in parallel, chunk c of a sensor cut into n
 * chunks delivered (c + 1) / n of the readout after the frame start), and
 * one waiter thread per instance collects the commands; both are pinned to
 * cores of the calling process, so no interpreter or scheduler pause of the
 * caller enters the figures.  The pacer's own lateness is recorded per frame.
 */
#ifndef RTC_PACER_H
#define RTC_PACER_H

#include "rtc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t inst;                    /* instance index in the engine */
    int32_t n_bank;                  /* frames in each sensor's bank */
    const uint16_t *const *banks;    /* host, one per sensor of the instance: n_bank frames of
                                        frame_h x frame_w uint16, frame f uses bank frame f % n_bank */
    float *cmds;                     /* host, nullable: the commands of every recorded frame,
                                        (n_frames - warmup) x n_act FP32 */
} rtc_pacer_stream;

typedef struct {
    double period_s;                 /* frame period (500 Hz: 2e-3) */
    double readout_s;                /* readout time over which each sensor's chunks are spread */
    int32_t n_frames;                /* frames to run, warm-up included */
    int32_t warmup;                  /* leading frames not recorded */
    uint64_t first_frame;            /* frame number of the first frame */
    int32_t zero_copy;               /* 1: rtc_acquire_chunk / rtc_commit_chunk, 0: submit */
    int32_t switch_stream;           /* stream whose gain and leak change (-1: none) */
    int32_t switch_frame;            /* run index (warm-up included) before which they change */
    float switch_gain, switch_leak;
    int32_t pin;                     /* 1: pin the producer and waiters to distinct cores */
    double timeout_s;                /* per-frame wait limit */
} rtc_pacer_desc;

typedef struct {
    uint64_t frame;                  /* frame number */
    double host_us;                  /* last chunk handed to the library -> commands seen
                                        (negative when they were seen first: the frame's
                                        last chunks hold no pixel it needs) */
    double dev_us;                   /* device clock: last chunk seen -> commands published;
                                        negative when published before the last chunk arrived
                                        (its last rows hold no pixel the frame needs) */
    double complete_us;              /* the last chunk that completes a column block (holds
                                        rows some slope needs) handed over -> commands seen;
                                        equals host_us unless the frame's last chunks hold
                                        no pixel the frame needs */
    double late_us;                  /* the frame's last chunk handed over this late against
                                        its schedule (the pacer's own jitter) */
    double start_late_us;            /* the frame's first chunk this late against its schedule */
    uint64_t dev_ticks_start;        /* device clock (100 MHz) of the last chunk seen, 0 if not */
    uint64_t dev_ticks_cmd;          /* device clock of the commands' publication */
} rtc_pacer_sample;

/* Runs d->n_frames paced frames through every stream and writes, for each
 * stream s and recorded frame i, out[s * (n_frames - warmup) + i].  Blocks
 * until done.  Errors: RTC_E_INVAL on bad arguments, RTC_E_STATE unless the
 * engine is persistent with its matrices loaded; any status a submit or wait
 * call returns ends the run with that status (the frame's index is in
 * *failed_frame, nullable). */
rtc_status rtc_pacer_run(rtc_engine *e, const rtc_pacer_desc *d, int32_t n_streams,
                         const rtc_pacer_stream *streams, rtc_pacer_sample *out,
                         int32_t *failed_frame);

#ifdef __cplusplus
}
#endif
#endif /* RTC_PACER_H */
