/*
 * frg_testing.h -- test double of the serving loop (part of the same library as frg.h).
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

#ifdef __cplusplus
}
#endif
#endif /* FRG_TESTING_H */
