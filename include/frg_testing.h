/*
 * frg_testing.h -- test double of the serving loop and a trace-replay harness for measuring it
 * (part of the same library as frg.h).
 *
 * For callers that test request scheduling without a GPU (admission against the HBM budget,
 * arrival order, cancellation, time-outs, latency accounting).  A fake session runs no device
 * work and computes nothing: a fused launch of requests totalling N integrand nodes completes
 * base_us + ns_per_node * N / 1000 microseconds after it starts, and the requests' host output
 * buffers are left untouched.  Every other frg_session_* call behaves as for a real session.
 */
#ifndef FRG_TESTING_H
#define FRG_TESTING_H

#include "frg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* cfg->hbm_budget_bytes must be >= 4096 (there is no context to take a default from).
 * FRG_E_INVAL on a bad config or negative timings. */
frg_status frg_session_open_fake(const frg_session_config *cfg, double ns_per_node,
                                 double base_us, frg_session **out);

/* Fake sessions only: the next n launches fail as a device error would (their tickets end with
 * FRG_E_DEVICE and their memory is released).  FRG_E_INVAL for a real session or n < 0. */
frg_status frg_session_fake_fail_launches(frg_session *s, int n);

/* ---- open-loop trace replay (serving measurements) ----------------------------------------- */

/* One kind of request of a trace (for instance one stage of one time-stepper). */
typedef struct {
    frg_integral_desc desc;  /* as submitted to a session; the plain path runs it in float64 */
    int n_ext;
    const double *ext;       /* host inputs (NULL for the LPA families) */
    const double *m2;        /* host [n_ext] */
    int table_id;            /* session-resident dressing table, or -1 (Z == 1) */
    const double *Z_dev;     /* the same table in device memory for the plain path, or NULL */
    int nZ;
    double x_min, x_max;
    const double *expect;    /* host [n_ext] or NULL: each completed result is compared with it
                                bit for bit (the plain path compares float64 kinds only) */
} frg_replay_kind;

typedef struct {
    double t_us;  /* arrival time from the start of the replay, ascending */
    int kind;
} frg_replay_arrival;

typedef struct {
    double latency_us;  /* arrival -> result in a host buffer */
    int status;         /* frg_status of the request */
    int mismatch;       /* 1 if the result differed from kind.expect */
} frg_replay_result;

/* Replay `n_arr` arrivals open-loop (each at its time, whatever is still running) and record
 * every request's latency.  mode 0: submitted to session s, completions taken by n_waiters
 * threads blocked in frg_session_wait.  mode 1: the plain per-batch path on ctx -- first in,
 * first out on one stream, each request's inputs copied to the device, one
 * frg_integrate_batch in float64, the result copied back.  *wall_us = first arrival to last
 * completion.  Host timing only; the caller keeps the inputs and tables alive. */
frg_status frg_serving_replay(frg_context *ctx, frg_session *s, int mode, int n_kinds,
                              const frg_replay_kind *kinds, int n_arr,
                              const frg_replay_arrival *arr, int n_waiters,
                              frg_replay_result *res, double *wall_us);

/* ---- FLOP-count probe ------------------------------------------------------------------------ */

/* One kernel dispatch (blocks x 64 lanes, each `iters` evaluations on a varying argument) of the
 * float64 sequence `seq` the integrand loops use -- 0: none (the bare loop, to subtract), 1: the
 * table logarithm, 2: expm1(-y) by Cody-Waite reduction, 3: exp(-y) by the same reduction, 4: the
 * reciprocal seed with one Newton step -- writing one sum per lane to out[blocks * 64] (device).
 * A profiler's FP64 FLOP counter for the dispatch, less that of seq 0, divided by
 * blocks * 64 * iters, is the sequence's FLOP count per call.  Synchronises `stream`. */
frg_status frg_flop_probe(int seq, int blocks, int iters, double *out, hipStream_t stream);

/* ---- float32 accuracy probe ------------------------------------------------------------------ */

/* Largest error, over every float32 input of its range, of one elementary operation of the
 * float32 precision form, into *max_err (host): which = 0: absolute error of the hardware log2
 * (v_log_f32) on [1/2, 1); 1: relative error of the float32 expm1(-y) on normal y <= 2^21;
 * 2: relative error of the hardware reciprocal (v_rcp_f32) on [2^-100, 2^100); 3: relative
 * error of the hardware 2^x (v_exp_f32) on [-126, 0).  References: the float64 log2, expm1 and
 * exp2 of the HIP math library.  Synchronises `stream`. */
frg_status frg_math_probe(int which, double *max_err, hipStream_t stream);

/* The constants the float32 form's error bound uses: out[0] = u = 2^-24, out[1..4] = the bounds
 * on the four errors frg_math_probe measures (same order). */
void frg_fp32_error_constants(double out[5]);

#ifdef __cplusplus
}
#endif
#endif /* FRG_TESTING_H */
