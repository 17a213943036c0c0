/*
 * rtc.h - C ABI of the MI355X adaptive-optics real-time-controller hot path.
 *
 * The library turns wavefront-sensor pixels into deformable-mirror commands,
 * one frame at a time, following the four per-sensor stages of the paper
 * (Jenkins, Basden & Myers, "A many-core CPU prototype of an MCAO and LTAO RTC
 * for ELT-scale instruments", section 1.1 figure of the AO-loop processes):
 *
 *   calibration  -> slopes (Shack-Hartmann centre of gravity, section 2.2, or
 *                   pyramid normalised quadrant differences, section 2.2)
 *                -> reconstruction (one dense control-matrix x slope MVM,
 *                   section 2.3), summed over every sensor of an instance
 *                   (section 3, partial commands summed on the master)
 *                -> DM command (leaky integrator, plus the implicit
 *                   pseudo-open-loop term M a_{f-1}, section 3.4).
 *
 * Pixels arrive as row chunks of a camera readout (section 2.2: slopes can be
 * computed as soon as the rows they need have arrived), so the matrix product
 * of a chunk's slopes overlaps the readout of later chunks.
 *
 * Conventions for every call:
 *  - Every pointer argument is owned by the caller and is only read (or
 *    written) during the call, unless stated otherwise.  "host" pointers are
 *    ordinary CPU memory; "device" pointers are HIP device memory of the
 *    engine's GPU.
 *  - Calls return an rtc_status; nothing throws across the ABI.  A device
 *    error is sticky: once RTC_E_DEVICE is returned, every later call on the
 *    engine returns it, except rtc_destroy.
 *  - Arrays are row-major and densely packed.
 *  - Results are deterministic: the same frames from the same state give the
 *    same commands bit for bit on every path (batch or serving, per-launch or
 *    persistent engine).  The FP32 accumulation order of the matrix product
 *    alternates with the parity of a frame's index among the frames started
 *    since the last rtc_load_matrices or rtc_set_state (not its frame number),
 *    so one frame processed at an even and at an odd index differs by FP32
 *    rounding only.
 */
#ifndef RTC_H
#define RTC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rtc_engine rtc_engine;

typedef enum {
    RTC_OK = 0,
    RTC_E_INVAL = -1,          /* bad argument, size or ordering */
    RTC_E_NOMEM = -2,          /* host or device allocation failed */
    RTC_E_DEVICE = -3,         /* HIP runtime or kernel error (sticky) */
    RTC_E_TIMEOUT = -4,        /* wait expired before the frame completed */
    RTC_E_STATE = -5,          /* call not valid in the current state */
    RTC_E_RING_FULL = -6,      /* pixel ring has no free slot */
    RTC_E_FRAME_DROPPED = -7,  /* the frame was superseded before completing */
    RTC_E_SCRATCH = -8         /* the work exceeds the library's static scratch */
} rtc_status;

enum { RTC_WFS_SH = 0, RTC_WFS_PYR = 1 };
/* Control-matrix storage: FP32, BF16 (round to nearest even) or OCP FP8
 * e4m3fn with one FP32 scale per matrix row (scale_r = max_j |R_rj| / 448).
 * Accumulation is FP32 in every case. */
enum { RTC_CM_F32 = 0, RTC_CM_BF16 = 1, RTC_CM_FP8 = 2 };
/* Threshold after calibration, c = ((raw - dark) * flat) - bg in binary32:
 * SUBTRACT: w = c > T ? c - T : 0;  ZERO: w = c > T ? c : 0;  NONE: w = c. */
enum { RTC_THR_SUBTRACT = 0, RTC_THR_ZERO = 1, RTC_THR_NONE = 2 };
/* Pyramid normalisation: LOCAL divides each pupil pixel's differences by its
 * own four-image sum (section 2.2: four pixels per slope, so slopes follow the
 * rows as they arrive); GLOBAL by one sum over every valid pupil pixel of the
 * frame (formed in one fixed order, so every path gives the same value), so
 * the sensor's slopes wait for its whole frame and form one column block. */
enum { RTC_PYR_NORM_LOCAL = 0, RTC_PYR_NORM_GLOBAL = 1 };
/* STREAM: each chunk submission enqueues its own kernels on the engine stream.
 * PERSISTENT: one resident kernel polls the pinned pixel ring and runs the
 * whole frame loop on the device. */
enum { RTC_MODE_STREAM = 0, RTC_MODE_PERSISTENT = 1 };

#define RTC_MAX_WFS 16
#define RTC_MAX_INST 8

typedef struct {
    int32_t kind;                 /* RTC_WFS_SH or RTC_WFS_PYR */
    int32_t frame_h, frame_w;     /* uint16 pixels */
    int32_t n_chunks;             /* chunk c holds rows [c*H/n, (c+1)*H/n) (floor) */
    int32_t thr_mode;             /* RTC_THR_* */
    /* Shack-Hartmann: nsub x nsub subapertures of px x px pixels (px <= 16)
     * whose first pixel is at (origin_row, origin_col). */
    int32_t nsub, px, origin_row, origin_col;
    const uint8_t *subap_valid;   /* host, nsub*nsub flags, raster order */
    /* Pyramid: four pupil images of pupil_px x pupil_px pixels, image q at
     * (quad_row[q], quad_col[q]); q = 0..3 are I1..I4 of
     * Sx = (I1 + I2 - I3 - I4) / S, Sy = (I1 + I3 - I2 - I4) / S. */
    int32_t pupil_px;
    int32_t quad_row[4], quad_col[4];
    const uint8_t *pupil_valid;   /* host, pupil_px*pupil_px flags */
    int32_t pyr_norm;             /* RTC_PYR_NORM_* */
} rtc_wfs_desc;

typedef struct {
    int32_t n_wfs;                /* 1..RTC_MAX_WFS */
    const rtc_wfs_desc *wfs;      /* host, n_wfs entries */
    int32_t n_act;                /* command length */
    int32_t cm_dtype;             /* RTC_CM_* */
    int32_t polc;                 /* 1: implicit pseudo-open-loop term on */
    float gain, leak;
} rtc_instance_desc;

typedef struct {
    int32_t device;               /* HIP device ordinal */
    int32_t n_inst;               /* 1..RTC_MAX_INST */
    const rtc_instance_desc *inst;
    int32_t ring_depth;           /* frames buffered per sensor (>= 2) */
    int32_t mode;                 /* RTC_MODE_* */
} rtc_create_desc;

typedef struct {
    uint64_t frame;               /* frame number the commands belong to */
    int64_t t_last_chunk_ns;      /* host CLOCK_MONOTONIC at the last chunk's submission
                                     (0 if the commands were published and collected
                                     before the frame's last chunk was submitted) */
    int64_t t_ready_ns;           /* host CLOCK_MONOTONIC when the commands were seen */
    uint64_t dev_ticks_start;     /* device 100 MHz clock: last chunk seen (persistent
                                     mode; 0 if not seen: a frame whose last chunks
                                     hold no pixel it needs can be published first,
                                     dev_ticks_cmd < dev_ticks_start then) */
    uint64_t dev_ticks_cmd;       /* device 100 MHz clock: commands published */
    uint32_t drops;               /* frames dropped on this instance so far */
    uint32_t reserved;
} rtc_frame_info;

typedef struct {
    int32_t n_wfs;
    int32_t n_units;              /* subapertures (SH) plus pupil pixels (pyramid) */
    int32_t n_slopes;             /* 2 * n_units */
    int32_t n_act;
    int32_t n_kblocks;            /* (sensor, chunk) column blocks of the matrix */
    int32_t mask_words;           /* uint64 mask words over all units (rtc_read_slopes) */
    int64_t cm_bytes;             /* bytes of the stored matrix, padding included */
    int64_t cm_bytes_logical;     /* n_act * n_slopes * element size (+ scales) */
    int64_t polc_bytes;           /* bytes of the stored POLC matrix (0 if off) */
} rtc_instance_info;

/* Engine lifetime.  rtc_create sets up one or more controller instances on
 * one GPU, each with its own sensors, command vector and control matrix: the
 * paper's SCAO, MCAO (6 LGS + 3 NGS, 3 DMs) and LTAO (6 LGS + 1 NGS, 1 DM)
 * systems (section 3, table comparing SCAO, MCAO and LTAO), where the partial
 * commands of every sensor of an instance are summed into one command vector
 * (section 3, the master node).  Copies the descriptors; subap/pupil maps
 * are read during the call only.  Allocates every device and pinned host
 * buffer the frame loop uses; nothing is allocated afterwards while frames
 * run.  RTC_E_INVAL on a malformed descriptor (sizes, a sensor outside its
 * frame, a sensor without valid units), RTC_E_DEVICE when the device is
 * missing, RTC_E_NOMEM when an allocation fails; *out is NULL on error.
 * rtc_destroy stops the loop and frees everything (NULL: RTC_E_INVAL). */
rtc_status rtc_create(const rtc_create_desc *desc, rtc_engine **out);
rtc_status rtc_destroy(rtc_engine *e);
const char *rtc_strerror(rtc_status s);
rtc_status rtc_get_info(rtc_engine *e, int32_t inst, rtc_instance_info *info);
/* Row range [row_begin, row_end) of chunk `chunk` of sensor `wfs`. */
rtc_status rtc_chunk_rows(rtc_engine *e, int32_t inst, int32_t wfs, int32_t chunk,
                          int32_t *row_begin, int32_t *row_end);

/* Control matrix R (host, n_act x n_slopes, FP32, slopes ordered sensor by
 * sensor, units in raster order, (x, y) interleaved): reconstruction is one
 * dense matrix-vector product per frame (section 2.3, the 5318 x 9232 MVM;
 * section 3.4 for the POLC matrix M, applied to the summed command).  The library encodes R
 * in the instance's storage type and re-tiles it on the device.  With POLC
 * on, give either D (host, n_slopes x n_act, FP64), and M = R.D is formed
 * once in FP64 on the device from the FP32 R, or M itself (host, n_act x
 * n_act, FP32).  M is stored in FP32.  Resets the command state.  Blocks
 * until the matrices are resident (stops a running serving loop first).
 * RTC_E_INVAL without R, or with POLC on and neither D nor M; non-finite
 * values in R give RTC_E_INVAL for FP8 storage (its row scales). */
rtc_status rtc_load_matrices(rtc_engine *e, int32_t inst, const float *R,
                             const double *D, const float *M);

/* Control-matrix swap without stopping the loop (the paper's reconstructor
 * change, section 3.2, without the blocking swap of the CPU prototype and
 * without the latency spike it reports).  Every instance holds two slots of
 * its matrices (R in the storage type, FP8 row scales, POLC M); frames use the
 * active slot.
 *
 * rtc_stage_matrices encodes R, and M or D exactly as rtc_load_matrices does,
 * into the inactive slot while frames keep running: the upload is a DMA copy
 * through pinned staging memory owned by the engine, on a stream of its own.
 * It first waits until no frame still uses the inactive slot (frames before
 * the previous swap), and returns once the staged matrices are resident.
 * Errors: RTC_E_STATE before rtc_load_matrices, while a swap is pending, and
 * when D (not M) is given while the persistent serving loop runs (the FP64
 * product allocates and synchronises the device); RTC_E_TIMEOUT if frames
 * before the previous swap are not published within 5 s (e.g. a frame left
 * half delivered); the command state is unchanged.
 *
 * rtc_swap_matrices makes the staged slot active from frame *f_eff_out, the
 * first frame whose processing has not started (the rule of rtc_set_params);
 * no frame is blocked and the command state carries over.  Frame f uses one
 * slot for its reconstruction matrix and FP8 scales and for the POLC product
 * on its commands, so the POLC term of frame f_eff is still formed with the
 * previous M: p_f = M_(slot of f - 1) a_(f - 1).  RTC_E_STATE if nothing is
 * staged or a swap is already pending.  One caller at a time per instance. */
rtc_status rtc_stage_matrices(rtc_engine *e, int32_t inst, const float *R,
                              const double *D, const float *M);
rtc_status rtc_swap_matrices(rtc_engine *e, int32_t inst, uint64_t *f_eff_out);

/* Detector calibration of one sensor, the first per-sensor stage of the
 * pipeline (section 2.3 names pixel calibration among the stages timed; the
 * order dark -> flat -> background -> threshold is this library's reading).
 * Host FP32 arrays, each nullable:
 * dark, flat, bg: frame_h x frame_w (defaults 0, 1, 0); thr: one value per
 * subaperture (SH) or one value (pyramid) (default 0); ref: reference slopes,
 * 2 per unit (default 0). */
rtc_status rtc_load_calibration(rtc_engine *e, int32_t inst, int32_t wfs,
                                const float *dark, const float *flat, const float *bg,
                                const float *thr, const float *ref);

/* Stage new gain and leak in the inactive parameter slot (section 3.2: double
 * buffered parameters).  They take effect from frame *f_eff_out, the first
 * frame whose processing has not started; no frame is blocked. */
rtc_status rtc_set_params(rtc_engine *e, int32_t inst, float gain, float leak,
                          uint64_t *f_eff_out);

/* Command state of the integrator: a (n_act), the commands of the last
 * frame, and the POLC term p = M a for the next frame (n_act; section 3.4:
 * formed for the next frame once the command is ready), host FP32, and the
 * number of the next frame.  rtc_set_state with NULL pointers zeroes them and
 * restarts the frame sequence (the accumulation direction restarts at even).
 * Both stop a running serving loop between frames (RTC_E_STATE while a frame
 * is half delivered) and synchronise the device. */
rtc_status rtc_get_state(rtc_engine *e, int32_t inst, float *a, float *p, uint64_t *next_frame);
rtc_status rtc_set_state(rtc_engine *e, int32_t inst, const float *a, const float *p,
                         uint64_t next_frame);

/* Serving path.  Pixels arrive from each camera as a stream of row chunks
 * tagged with a frame number (section 2.1, the UDP camera stream; section 3:
 * the frame number stamped by the camera matches commands to frames), and
 * slopes are formed as soon as the rows they need have arrived (section 2.2,
 * pipelining of SH and pyramid sensors).  Submit chunk `chunk` of frame
 * `frame` of sensor `wfs` (host rows: the chunk's rows, frame_w uint16 each;
 * copied during the call).  Chunks of one frame
 * and sensor must come in increasing order (else RTC_E_INVAL).  A frame
 * number below the frame in progress gives RTC_E_FRAME_DROPPED; starting a
 * newer frame before the current one completed drops the current one.  The
 * frame's commands are produced once every chunk of every sensor of the
 * instance has been submitted. */
rtc_status rtc_submit_pixel_chunk(rtc_engine *e, int32_t inst, int32_t wfs, uint64_t frame,
                                  int32_t chunk, const uint16_t *rows);
/* Zero-copy form of rtc_submit_pixel_chunk (persistent mode only, else
 * RTC_E_STATE): rtc_acquire_chunk opens the chunk under the same frame and
 * order rules and lends the caller the pinned host ring slot that the loop
 * reads it from: *rows points at the chunk's first row, *pitch receives the
 * row pitch in uint16 (frame_w rounded up to 8).  The caller writes the
 * chunk's rows there, frame_w values per row, then calls rtc_commit_chunk
 * with the same (wfs, frame, chunk), which hands the rows to the loop; the
 * frame's arrival time is taken at commit.  One chunk per sensor may be lent
 * at a time (acquiring another before the commit gives RTC_E_INVAL; so does a
 * commit that names another chunk).  A commit after a newer frame of the
 * instance was started meanwhile gives RTC_E_FRAME_DROPPED.  The pointer is
 * owned by the library and valid until the commit. */
rtc_status rtc_acquire_chunk(rtc_engine *e, int32_t inst, int32_t wfs, uint64_t frame,
                             int32_t chunk, uint16_t **rows, int32_t *pitch);
rtc_status rtc_commit_chunk(rtc_engine *e, int32_t inst, int32_t wfs, uint64_t frame,
                            int32_t chunk);
/* Wait up to timeout_ns for the commands of `frame` and copy them to cmds
 * (host, n_act FP32).  info (nullable) receives the frame's timestamps: the
 * paper's latency runs from the arrival of the last pixel to the DM command
 * being ready (section 3, lab test setup; section 3.1).  RTC_E_TIMEOUT when
 * the commands are not out in time, RTC_E_FRAME_DROPPED when the frame was
 * superseded, never started, or its mailbox slot was reused by a later frame
 * while it was copied (a slow reader on a separate thread). */
rtc_status rtc_wait_commands(rtc_engine *e, int32_t inst, uint64_t frame, float *cmds,
                             int64_t timeout_ns, rtc_frame_info *info);

/* Telemetry stream (the paper's circular telemetry buffers of slopes and DM
 * commands, streamed while the loop runs; section on streaming telemetry).
 * Persistent mode only (RTC_E_STATE otherwise).  rtc_telemetry_enable makes
 * every `decimation`-th frame started on the instance (frames counted from
 * the last rtc_load_matrices or rtc_set_state) write its slopes, its counts
 * of thresholded pixels, its commands and its thresholded-pixel masks into a
 * ring of n_slots records in
 * pinned host memory owned by the engine; decimation and n_slots are powers
 * of two up to 65536, n_slots 0 turns telemetry off.  It stops the serving
 * loop between frames (RTC_E_STATE while a frame is half delivered) and
 * discards the previous ring.  The first record is the next frame to start.
 *
 * rtc_telemetry_next copies the next record in frame order (host arrays,
 * each nullable: slopes n_slopes FP32 as rtc_read_slopes orders them, counts
 * n_units int32, cmds n_act FP32, masks mask_words uint64 laid out as
 * rtc_read_slopes lays them out: the thresholded-pixel masks of the frame,
 * the paper's pixel telemetry in one bit per pixel) once its frame is published, waiting at
 * most timeout_ns (RTC_E_TIMEOUT).  A record is overwritten when the frame
 * decimation * n_slots later starts; records overwritten before being read
 * are skipped and counted in info->lost.  A dropped frame's record has
 * info->dropped = 1, its slopes and counts are partial and its commands are
 * the previous frame's.  One reader per instance. */
typedef struct {
    uint64_t frame;               /* frame number of the record */
    uint32_t dropped;             /* 1: the frame was dropped */
    uint32_t lost;                /* records skipped (overwritten) before this one */
} rtc_telemetry_info;
rtc_status rtc_telemetry_enable(rtc_engine *e, int32_t inst, int32_t decimation,
                                int32_t n_slots);
rtc_status rtc_telemetry_next(rtc_engine *e, int32_t inst, float *slopes, int32_t *counts,
                              float *cmds, uint64_t *masks, int64_t timeout_ns,
                              rtc_telemetry_info *info);

/* Batch path over device-resident frames: runs n_frames consecutive frames
 * through the whole hot path, in order, updating the command state exactly as
 * the serving path would.  frames[w] (device) points at n_frames frames of
 * sensor w spaced frame_stride[w] uint16 apart.  Outputs (device, nullable):
 * cmds n_frames x n_act, slopes n_frames x n_slopes, counts n_frames x n_units.
 * Work is enqueued on `stream` (a hipStream_t; NULL is the device's null
 * stream) and the call returns without waiting. */
rtc_status rtc_process_frames(rtc_engine *e, int32_t inst, const uint16_t *const *frames,
                              const int64_t *frame_stride, int32_t n_frames,
                              float *cmds, float *slopes, int32_t *counts, void *stream);

/* rtc_process_frames for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and command-state update as
 * rtc_process_frames in RTC_MODE_STREAM (bit for bit: the same kernels in the
 * same order), but the matrix products' partial sums and per-tile arrival
 * counters live in a static device array of the library (16 MiB, one copy
 * per device, held until the process ends) instead of the engine's buffers;
 * the call allocates nothing and clears the counters with a kernel, not a
 * memset.  Every call on one device shares that device's array: calls that
 * overlap on one device (two streams, two engines or two threads) race, so
 * order them.  Errors: RTC_E_STATE in RTC_MODE_PERSISTENT or before
 * rtc_load_matrices; RTC_E_SCRATCH when the instance's partials and counters
 * (n_segments x n_act + POLC segments x n_act floats, plus 2 x 256 B per
 * 64-row tile) exceed the array; otherwise as rtc_process_frames. */
rtc_status rtc_process_frames_noalloc(rtc_engine *e, int32_t inst,
                                      const uint16_t *const *frames,
                                      const int64_t *frame_stride, int32_t n_frames,
                                      float *cmds, float *slopes, int32_t *counts,
                                      void *stream);

/* Slopes, per-unit counts of thresholded pixels and the thresholded-pixel
 * masks of the most recent frame (host, each nullable).  masks: mask_words
 * uint64; unit u's pixels, raster order within the subaperture, are bits of
 * consecutive words starting at a 64-bit boundary; a pyramid unit has one
 * word whose bits 0..3 are I1..I4.  Synchronises the engine stream. */
rtc_status rtc_read_slopes(rtc_engine *e, int32_t inst, float *slopes, int32_t *counts,
                           uint64_t *masks);
/* Stored control matrix of the active slot in logical order (host): codes
 * n_act x n_slopes of 4, 2 or 1 bytes per element, and for FP8 the n_act row
 * scales. */
rtc_status rtc_read_matrix(rtc_engine *e, int32_t inst, void *codes, float *scales);

/* Timing aid: enqueue the reconstruction MVM alone (every column block, on
 * the current slopes) n_iter times on `stream` (hipStream_t, NULL = null
 * stream).  Changes no command state. */
rtc_status rtc_run_mvm(rtc_engine *e, int32_t inst, int32_t n_iter, void *stream);

/* MVM kernel timer (RTC_MODE_STREAM diagnostics).  With capacity > 0, later
 * rtc_process_frames frames that have a successor in their batch (their
 * reconstruction MVM launch also forms the successor's slopes) are timed in
 * runs of `every` consecutive launches: one pair of HIP events on the batch's
 * stream brackets each run (a run also ends at the batch's last such frame),
 * up to capacity pairs, so the two queue packets a pair adds are spread over
 * the run.  A run includes what its frames enqueue between the launches (the
 * POLC product, output copies).  capacity 0 turns the timer off.
 * rtc_mvm_timing_read synchronises on the last recorded pair, returns the
 * number of timed launches and the sum of the runs' durations (ms) and clears
 * the record.  RTC_E_STATE in persistent mode. */
rtc_status rtc_mvm_timing(rtc_engine *e, int32_t inst, int32_t capacity, int32_t every);
rtc_status rtc_mvm_timing_read(rtc_engine *e, int32_t inst, int32_t *n, double *total_ms);

/* Frame-loop timeline (RTC_MODE_PERSISTENT diagnostics).  With n_frames > 0,
 * every wavefront of every later frame-loop launch records RTC_TRACE_EVENTS
 * device-clock values (wall clock, 100 MHz) for each of the first n_frames
 * frames of that launch, overwriting the previous launch's record; 0 turns the
 * record off (its cost is then one test per frame).  Synchronises the engine;
 * the loop must not be running (RTC_E_STATE otherwise). */
#define RTC_TRACE_EVENTS 15
enum {
    RTC_TRACE_FRAME_START = 0,   /* the wavefront reached the frame */
    RTC_TRACE_GATE = 1,          /* frame q - 2 published: the frame may start */
    RTC_TRACE_CENTROIDS = 2,     /* its last centroid tasks of the frame done and counted */
    RTC_TRACE_MVM_FIRST = 3,     /* its first MVM task starts (slopes ready) */
    RTC_TRACE_MVM_LAST = 4,      /* its last MVM task (and accumulation) done */
    RTC_TRACE_INGEST = 5,        /* serving: its last ingest pieces copied and counted */
    RTC_TRACE_ACCUM = 6,         /* its last tile accumulation done (commands counted) */
    RTC_TRACE_FRAME_END = 7,     /* POLC tasks done, leaving the frame */
    RTC_TRACE_CEN_START = 8,     /* its last centroid tasks start (their pixels are in) */
    RTC_TRACE_LAST_BLOCK = 9,    /* its first MVM task of the frame's last block starts */
    RTC_TRACE_TILE_READY = 10,   /* it completed a tile's partials (the sum starts) */
    RTC_TRACE_CMDS = 11,         /* its last tile's commands written (before counting) */
    RTC_TRACE_INGEST_START = 12, /* serving: its last ingest pieces start (doorbell seen) */
    RTC_TRACE_SUMMED = 13,       /* its last tile sum (and command operands) in registers */
    RTC_TRACE_JOINED = 14        /* its last join atomic returned (first partials loaded) */
};
rtc_status rtc_trace_enable(rtc_engine *e, int32_t n_frames);
/* Copies the record of the last launch into out (host): value
 * [(frame * n_waves + wave) * RTC_TRACE_EVENTS + event], frame relative to
 * the launch's first, wave = global wavefront index (a serving instance's
 * sentinel included, left zero).  Zero marks an event that did not happen.
 * capacity counts uint64 values; n_waves and n_frames (nullable) receive the
 * record's shape.  Stops a running serving loop (as rtc_get_state does) and
 * synchronises the device. */
rtc_status rtc_trace_read(rtc_engine *e, uint64_t *out, int64_t capacity, int32_t *n_waves,
                          int32_t *n_frames);

#ifdef __cplusplus
}
#endif
#endif /* RTC_H */
