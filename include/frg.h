/*
 * frg.h -- C ABI of the MI355X (gfx950) batched loop-integral library for functional
 * renormalisation group flows.
 *
 * What the library computes follows Sattler & Pawlowski, "DiFfRG: A Discretisation Framework
 * for functional Renormalisation Group flows" (arXiv 2412.13043):
 *   - a flow right-hand side is a set of loop-momentum integrals, one per external point, whose
 *     integrands carry the regulator insertion k dR_k/dk (Sec. 2.1, generalised flow equation and
 *     the tower of n-point flows; t = log(Lambda/k), k d/dk = -d/dt);
 *   - each integral is evaluated by a "Quadrature" integrator, a tensor-product quadrature that
 *     treats all vacuum dimensions alike, over |q| and the loop angles; in d = 4 the angle
 *     variables are cos1 and (for two angles beyond it) phi (Sec. 5.3 "Momentum integrations",
 *     App. F "Kernel definitions");
 *   - an integration kernel is described by its type, number of angles, dimension d and compute
 *     type ctype in {double, float} (App. F), and receives constants, per-point variables and
 *     tabulated functions interpolated on logarithmic coordinates (App. F "Parameter
 *     definitions", FunctionTex1D);
 *   - the model's right-hand side fills one residual entry per integral call (App. G listing;
 *     Sec. 5.2 dt_variables), batched here over all external points of a flow.
 * The quadrature family is Gauss-Legendre: radial nodes on [0, q_max k], x = cos1 on [-1, 1]
 * with the d = 4 measure factor sqrt(1 - x^2), phi on [0, pi] with measure sin(phi).
 *
 * Conventions for every call:
 *   - Every entry point returns frg_status; nothing throws across the ABI.  On any error the
 *     output buffers are left unspecified and frg_last_error() (thread-local) names the cause.
 *   - Argument and shape errors are reported synchronously with FRG_E_INVAL before anything is
 *     enqueued.  HIP runtime failures are FRG_E_DEVICE.
 *   - "device" pointers are HIP device memory (for example torch CUDA/HIP tensors); the caller
 *     owns them and keeps them alive until the stream reaches the work (for sessions: until the
 *     ticket completes).  "host" pointers are ordinary host memory.
 *   - Work is enqueued on the caller's stream (NULL = the default stream) and is asynchronous
 *     unless stated otherwise; results are visible after the stream is synchronised.
 *   - All arrays are float64, structure-of-arrays, contiguous.
 *   - The library owns its quadrature-rule cache, scratch, tile lists, autotune cache and the
 *     session-resident dressing tables.
 */
#ifndef FRG_H
#define FRG_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct frg_context frg_context; /* device, rule cache, scratch pools, autotune cache */
typedef struct frg_session frg_session; /* serving loop over one context */

typedef enum {
    FRG_OK = 0,
    FRG_E_INVAL = 1,       /* bad argument, descriptor or shape; nothing was enqueued */
    FRG_E_NOMEM = 2,       /* allocation failed or request exceeds the HBM budget */
    FRG_E_DEVICE = 3,      /* HIP runtime error; see frg_last_error() */
    FRG_E_NOTREADY = 4,    /* ticket not finished (poll) */
    FRG_E_TIMEOUT = 5,     /* wait timed out */
    FRG_E_CANCELLED = 6,   /* ticket was cancelled */
    FRG_E_UNSUPPORTED = 7  /* valid but not implemented combination */
} frg_status;

typedef enum {
    FRG_FP64 = 0,       /* integrand and all sums in float64 */
    FRG_FP32_KAHAN = 1  /* float32 integrand, compensated float32 inner sums, float64 outer sums;
                           propagators near the pole evaluated in float64 (see near_pole_tau) */
} frg_precision;

typedef enum {
    FRG_FAMILY_LPA = 1,         /* radial only, any d >= 1 (local potential approximation) */
    FRG_FAMILY_TWO_POINT = 2,   /* d = 4, one angle (cos1) */
    FRG_FAMILY_THREE_POINT = 3, /* d = 4, cos1 and phi (third angle trivial: factor 2 pi) */
    FRG_FAMILY_LPA_T = 4,       /* finite temperature, d = 3 + 1: Matsubara sum x radial */
    FRG_FAMILY_TWO_POINT_T = 5, /* finite temperature, d = 3 + 1: Matsubara sum x radial x cos1 */
    FRG_FAMILY_THREE_POINT_T = 6 /* finite temperature, d = 3 + 1: Matsubara sum x radial x cos1 x
                                    phi */
} frg_family;

typedef enum {
    FRG_REG_EXPONENTIAL = 0,  /* R = l2/(exp(l2/k^2) - 1) */
    FRG_REG_POLY_EXP = 1,     /* R = k^2 exp(-sum_{i=1}^{N} y^i/i), y = l2/k^2: the shape s_N of
                                 Sec. 3.1 (the paper's default regulator, N = 8) */
    FRG_REG_FLAT = 2          /* R = (k^2 - l2) Theta(k^2 - l2) (Litim), k dR/dk = 2 k^2 Theta */
} frg_regulator;

typedef enum {
    FRG_BOSONIC = 0,   /* Matsubara frequencies w_n = 2 pi n T */
    FRG_FERMIONIC = 1  /* w_n = 2 pi (n + 1/2) T */
} frg_statistics;

/*
 * Integral descriptor ("integration kernel" in the paper's App. F terms).
 *
 *   family 1:  I_e = Omega_d/(2pi)^d sum_a w_a q_a^(d-1) Rdot(q_a^2)/(q_a^2 + R(q_a^2) + m2_e)^2
 *   family 2:  I_e = 4pi/(2pi)^4 sum_ab w_a w_b sqrt(1-x_b^2) q_a^3 Rdot(q_a^2) G(q_a^2)^2
 *                    G(q_a^2 + p_e^2 + 2 q_a p_e x_b)
 *   family 3:  I_e = 2pi/(2pi)^4 sum_abc w_a w_b w_c sqrt(1-x_b^2) sin(phi_c) q_a^3 Rdot G(q_a^2)^2
 *                    G(l1^2) G(l2^2),   l1 = q + p1, l2 = q - p2,
 *                    p1 = p e1, p2 = p (cos(alpha) e1 + sin(alpha) e2):
 *                    l1^2 = q^2 + p^2 + 2 q p x,
 *                    l2^2 = q^2 + p^2 - 2 q p (x cos(alpha) + sqrt(1-x^2) cos(phi) sin(alpha))
 * with the regulator R(l2) (by default the exponential one, R = l2/(exp(l2/k^2) - 1), whose
 * scale derivative is Rdot = k dR/dk = 2 k^2 y^2 e^y/(e^y - 1)^2, y = l2/k^2; see frg_regulator:
 * polynomial-exponential Rdot = 2 k^2 exp(-S_N(y)) (1 + sum_{i=1}^{N} y^i), flat
 * Rdot = 2 k^2 Theta(k^2 - l2)) and the propagator G(l2) = 1/(Z(l2) l2 + R(l2) + m2).
 * With the flat regulator the integrand has a kink at |q| = k; a radial node within rounding
 * of it may fall on either side.  Radial GL(n_q) on [0, q_max*k]; x GL(n_x) on [-1, 1];
 * phi GL(n_phi) on [0, pi].  Momenta squared below zero from rounding are clamped to 0.
 *
 * Finite temperature (Sec. 5.3 "Momentum integrations": the "Quadratureq0"/"Quadraturex0"
 * integrator types, which treat the imaginary-time direction as a Matsubara sum; Sec. 3.1: a
 * regulator acting on the spatial momentum only).  d must be 4 (three spatial dimensions and the
 * frequency).  T sum_{n in Z} f(w_n) is evaluated with the frequency rule sum_j c_j f(w_j):
 *   - every Matsubara frequency with |w_n| <= Lambda, weight T, where Lambda = freq_max
 *     ("q0": a fixed frequency domain) or freq_max * k ("x0", freq_scaled = 1: the domain scales
 *     with k);
 *   - n_tail > 0: the omitted frequencies as the integral (1/2pi) int_{|w| >= Omega} f dw, with
 *     Omega = (largest explicit |w|) + pi T, by GL(n_tail) in t on [0, 1] after w = +-Omega/t on
 *     each side (error of the midpoint boundary: O(T^2 f'(Omega)));
 *   - the frequencies are sorted ascending; radial node a and frequency j form the radial index
 *     a n_f + j of the sums (contributions are added in that order).
 *   family 4:  I_e = sum_j c_j 4pi/(2pi)^3 sum_a w_a q_a^2 Rdot(q_a^2) G_j(q_a)^2,
 *                    G_j(q) = 1/(w_j^2 + q^2 + R(q^2) + m2_e)
 *   family 5:  I_e = sum_j c_j 2pi/(2pi)^3 sum_ab w_a w_b q_a^2 Rdot(q_a^2) G_j(q_a)^2 H_j(l),
 *                    G_j(q) = 1/(w_j^2 + Z(q^2) q^2 + R(q^2) + m2_e),
 *                    H_j(l) = 1/((w_j + p0_e)^2 + Z(l^2) l^2 + R(l^2) + m2_e),
 *                    l^2 = q_a^2 + p_e^2 + 2 q_a p_e x_b (spatial; Z and R act on spatial momenta)
 *   family 6:  I_e = sum_j c_j 2/(2pi)^3 sum_abc w_a w_b w_c q_a^2 Rdot(q_a^2) G_j(q_a)^2
 *                    H1_j(l1) H2_j(l2),
 *                    H1_j(l) = 1/((w_j + p01_e)^2 + Z(l^2) l^2 + R(l^2) + m2_e), H2_j with p02_e,
 *                    l1^2 = q^2 + p^2 + 2 q p x, l2^2 = q^2 + p^2 - 2 q p (x cos(alpha) +
 *                    sqrt(1-x^2) cos(phi) sin(alpha)) (spatial, as in family 3 with p1 = p e1,
 *                    p2 = p (cos(alpha) e1 + sin(alpha) e2));
 *              in three spatial dimensions the cos1 weight is dx alone (no sqrt(1-x^2)) and the
 *              phi weight dphi alone (no sin(phi)); the azimuth runs over [0, 2pi) and the
 *              integrand is even in it, so phi GL(n_phi) on [0, pi] carries a factor 2
 * p0_e is the external frequency: a bosonic 2 pi m T, or for a fermion the paper's
 * p0f = pi T exp(-k/(pi T)) (App. "Derivation of the four-Fermi system").
 * Complex external frequencies (complex_freq = 1, families 5 and 6): an inner leg's external
 * frequency is p0 + i p0i, as for the paper's external fermion legs at chemical potential mu,
 * whose imaginary-time component is p0f - i mu (same appendix): H continues analytically,
 * H_j(l) = 1/((w_j + p0 + i p0i)^2 + Z(l^2) l^2 + R(l^2) + m2_e) (the radial leg keeps its real
 * w_j), and I_e is complex.  The ext array appends the imaginary parts (family 5: p, p0, p0i;
 * family 6: p, alpha, p01, p02, p01i, p02i) and out holds 2 n_ext values, Re I_e at e and
 * Im I_e at n_ext + e.  Float64 only, without dout_dm2 and dout_dz (FRG_E_UNSUPPORTED), not
 * for flows (frg_flow_rhs, steppers: FRG_E_UNSUPPORTED); a continued pole
 * (w_j + p0 + i p0i)^2 = -(Z l^2 + R + m2) on a node gives inf or nan.
 * Limits: at least one explicit frequency (fermionic: Lambda >= pi T); n_tail <= FRG_MAX_NODES;
 * n_f = explicit + 2 n_tail <= FRG_MAX_NODES; n_q n_f <= FRG_MAX_FT_NODES.
 */
typedef struct {
    int family;            /* frg_family */
    int d;                 /* 1..8 for LPA; must be 4 for families 2 to 6 */
    int n_q;               /* radial nodes, 1..FRG_MAX_NODES */
    int n_x;               /* cos1 nodes (families 2, 3, 5, 6), 1..FRG_MAX_NODES; ignored for LPA */
    int n_phi;             /* phi nodes (families 3, 6), 1..FRG_MAX_NODES; ignored otherwise */
    int precision;         /* frg_precision */
    double q_max;          /* radial upper limit in units of k, > 0 */
    double k;              /* RG scale, > 0 */
    double near_pole_tau;  /* FP32 form only: a propagator whose denominator D satisfies
                              D < tau (|Z l2 + R| + |m2|) is evaluated in float64; 0 = never */
    /* families 4, 5 and 6 only (ignored otherwise; zero them) */
    double T;              /* temperature (same units as k), > 0 */
    double freq_max;       /* explicit frequencies |w| <= freq_max (or freq_max * k), > 0 */
    int statistics;        /* frg_statistics */
    int n_tail;            /* GL nodes per side for the omitted frequencies; 0 = none */
    int freq_scaled;       /* 0: Lambda = freq_max ("q0"); 1: Lambda = freq_max * k ("x0") */
    /* every family */
    int regulator;         /* frg_regulator (0, the exponential one, when zeroed); every
                              regulator in both precisions */
    int reg_order;         /* N of FRG_REG_POLY_EXP, 1..16; 0 = 8 */
    int complex_freq;      /* families 5 and 6: 1 = complex external frequencies of the inner
                              legs (see below), 0 = real; must be 0 for the other families */
} frg_integral_desc;

#define FRG_MAX_NODES 1024
#define FRG_MAX_FT_NODES 65536
#define FRG_MAX_TABLE 4096

/* Dressing Z tabulated on n points log-uniform in |l| over [x_min, x_max] (device pointer),
 * linear in log|l| between points, constant outside.  values == NULL means Z == 1.
 * Ignored by families 1 and 4 (Z == 1 there). */
typedef struct {
    const double *values;
    int n;                 /* 2..FRG_MAX_TABLE */
    double x_min, x_max;   /* 0 < x_min < x_max */
} frg_log_table;

/* One batch of n_ext external points sharing one descriptor and one dressing table. */
typedef struct {
    int n_ext;             /* >= 0; 0 is a valid no-op */
    const double *ext;     /* device. families 1, 4: unused (may be NULL); family 2: p[n_ext];
                              family 3: p[n_ext] followed by alpha[n_ext] (2 n_ext values);
                              family 5: p[n_ext] followed by p0[n_ext] (2 n_ext values);
                              family 6: p, alpha, p01 and p02, each [n_ext] (4 n_ext values:
                              the spatial momenta as in family 3, the external frequencies of
                              the two inner legs); with complex_freq the imaginary parts
                              follow (families 5 and 6: 3 and 6 n_ext values) */
    const double *m2;      /* device [n_ext] per-point m^2, or NULL to use m2_scalar */
    double m2_scalar;
    frg_log_table Z;
    double *out;           /* device [n_ext]: I_e ([2 n_ext], Re then Im, with complex_freq) */
    double *err_out;       /* device [n_ext] or NULL: stated relative error bound per result of
                              the FP32 form (0 for FP64): with u = 2^-24, kappa the largest
                              amplification (|Z l2 + R| + |m2|)/D among that point's float32
                              propagators and nG the float32 propagators per integrand term
                              (two-point 1, three-point 2), (6 + 2 nG) u + nG (eE + er) +
                              nG kappa K, where eE, er are the measured errors of the float32
                              exponential and reciprocal and K the per-kappa error of one
                              propagator, set by the regulator, the dressing table's largest
                              relative step and its smallest entry (assumed positive); LPA
                              (7 + 10 kappa) u + 2 er */
    double *dout_dm2;      /* device [n_ext] or NULL: dI_e/dm2_e, the derivative of each result in
                              its point's mass, evaluated in the same pass by forward-mode
                              differentiation through every propagator (dG/dm2 = -G^2; the
                              Jacobian entries of implicit steppers, Sec. 5.2 and the "AD" option
                              of App. F); float64 only (FRG_E_UNSUPPORTED otherwise); taken by
                              frg_integrate_batch, frg_integrate_multi and sessions (there a
                              host buffer, returned with out) */
    double *dout_dz;       /* device [n_ext * Z.n] or NULL: dI_e/dZ_i, row-major (entry i of point
                              e at e * Z.n + i), the derivatives of each result in the entries of
                              its dressing table (the forward-mode derivatives of the "AD" option
                              of App. F for a flow of the dressing; Sec. 5.2 jacobian_variables).
                              Z enters through the linear interpolation of every propagator's
                              dressing, so dG(v)/dZ_i = -G(v)^2 v w_i(v) with w_i(v) the
                              interpolation weight of entry i at v; entries no node reaches are
                              exactly 0.  The vertex families 2, 3, 5 and 6 (at finite
                              temperature the dressing multiplies the spatial momentum) in
                              float64 with a dressing table only (FRG_E_UNSUPPORTED for the
                              LPA families, complex frequencies and the float32 form,
                              FRG_E_INVAL without a table), frg_integrate_batch,
                              frg_integrate_multi and sessions (there a host buffer, returned
                              with out; a resident table counts as the table); the caller
                              owns the buffer.  Computed by a second kernel after the
                              integrals on the same stream.  Each point's parts are rounded to
                              units of 2^-62 of its largest part and added as integers, so
                              the values are the same bits for any launch shape or order, and
                              where every term has one sign each entry errs by at most its
                              number of parts x 2^-62 of its row's largest entry */
} frg_batch;

/* ---- threshold functions of the flat regulator -------------------------------------------- */

/* out[i] = l_n^d(w[i]) = (2/d) (n + [n == 0]) / (1 + w[i])^(n + 1) for i < count: the threshold
 * functions of the flat regulator R = (k^2 - q^2) Theta(k^2 - q^2) (Sec. 5, the convenience
 * functions for standard setups), i.e. the closed form of the LPA loop integral with it,
 * I(m^2) = Omega_d/(2 pi)^d k^(d-2) l_1^d(m^2/k^2) (family 1 with FRG_REG_FLAT integrates the
 * same function by quadrature; the two agree to rounding when q_max = 1), with
 * dI/dm^2 = -Omega_d/(2 pi)^d k^(d-4) l_2^d and, in general, dl_n/dw = -(n + [n == 0]) l_{n+1}.
 * w and out: device arrays of count doubles, caller-owned; asynchronous on `stream` (no context
 * needed).  1 <= d <= 16, 0 <= n <= 16, count >= 0 (0: no-op), else FRG_E_INVAL; w <= -1 is no
 * error (the pole gives inf or a sign flip, as the formula does). */
frg_status frg_litim_threshold(int d, int n, const double *w, double *out, int count,
                               hipStream_t stream);

/* ---- context ------------------------------------------------------------------------------- */

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the library's own device
 * allocations for sessions (0 = 90% of free memory).  *out receives the handle. */
frg_status frg_context_create(int device, size_t hbm_budget_bytes, frg_context **out);
/* Waits for the context's work, frees everything it owns. NULL is a no-op. */
frg_status frg_context_destroy(frg_context *ctx);
/* Message of the last failing call on this thread ("" if none). Valid until the next call. */
const char *frg_last_error(void);

/* ---- batched integration ------------------------------------------------------------------- */

/* Evaluate I_e for all points of one batch (paper Sec. 5.3: the integrator's get(k, args...),
 * batched over external points).  One kernel launch on `stream`. */
frg_status frg_integrate_batch(frg_context *ctx, const frg_integral_desc *desc,
                               const frg_batch *batch, hipStream_t stream);

/* Evaluate n batches with independent descriptors (any mix of families, node counts and
 * precisions) in one fused persistent launch: the work is cut into tiles, ordered largest
 * first, and consumed by a grid sized to the device.  Each result is bitwise identical to the
 * same batch submitted alone through frg_integrate_batch with the same descriptor. */
frg_status frg_integrate_multi(frg_context *ctx, int n, const frg_integral_desc *descs,
                               const frg_batch *batches, hipStream_t stream);

/* Static scratch of frg_integrate_batch_noalloc, per device (bytes). */
#define FRG_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)

/* For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  The same computation, arguments, errors and results
 * (bit for bit) as frg_integrate_batch, but no device memory is allocated or freed by the call:
 * the scratch it needs -- the descriptor's quadrature rules if the context has not cached them
 * yet (an earlier frg_integrate_batch with the same rule parameters caches them), the radial
 * contributions of radially chunked requests and the float32 form's amplification slots -- lives
 * in one static device array of FRG_NOALLOC_SCRATCH_BYTES per device, held until the process
 * ends.  A request needing more returns FRG_E_NOMEM (nothing enqueued).  The array is shared by
 * every call on the device and keeps the last call's contents (the call clears what must start
 * at zero): calls whose work may overlap on one device -- different streams, or host threads
 * without ordering between them -- race on it and must not be issued. */
frg_status frg_integrate_batch_noalloc(frg_context *ctx, const frg_integral_desc *desc,
                                       const frg_batch *batch, hipStream_t stream);

/* Pick the tile shape (lanes per external point over radial nodes and over cos1 nodes; radial
 * chunks per external tile) of frg_integrate_batch and
 * frg_flow_rhs for this descriptor and batch size by timing the candidate shapes on the given
 * batch (its out buffer is overwritten with the integrals), and keep the fastest in the context.
 * If the environment variable FRG_AUTOTUNE_CACHE names a file, tuned shapes are loaded from it
 * when the context is created and appended to it here, one line per shape:
 * "family precision n_q n_x n_phi n_ext target lq_log2 chunks lx_log2" (target = 16 x CUs);
 * if FRG_AUTOTUNE_LOG names a file, every candidate's time is appended to it
 * ("family precision n_q n_x n_phi n_ext lq_log2 chunks lx_log2 us").
 * Finite-temperature descriptors are keyed as their vacuum counterparts with n_q n_f radial
 * nodes (family 4 as 1, family 5 as 2) and share their tuned shapes.
 * Results do not depend on the shape, only speed does.  Synchronises `stream`.
 * *best_us (optional) receives the best time per launch. */
frg_status frg_autotune(frg_context *ctx, const frg_integral_desc *desc, const frg_batch *batch,
                        hipStream_t stream, int reps, double *best_us);

/* ---- flow right-hand side ------------------------------------------------------------------- */

/*
 * State of a flow whose right-hand side is assembled from one family of loop integrals.
 *   family 1 (LPA of the O(N) model, paper Sec. 3.1 in its flux form):
 *       state = u_i = U'(rho_i) on the grid rho_i (n_ext >= 3, strictly increasing);
 *       m_s^2 = u + 2 rho u', m_p^2 = u (both floored at m2_floor), u', u'' from the quadratic
 *       through three neighbouring grid points (one-sided at the ends), and
 *       du_i/dt = 1/2 [ I(m_s^2) (3 u' + 2 rho u'') + (n_comp - 1) I(m_p^2) u' ]
 *       with t = log(Lambda/k) (Sec. 2.1).  Needs 2 n_ext integrals per call.
 *   family 4: the same at finite temperature (the paper's finite-temperature O(N) example,
 *       Sec. 3.1), I the family-4 integral.
 *   families 2, 3, 5 and 6 (vertex expansion): state = m2_e per external point (floored at
 *       m2_floor), grid = the batch's ext array, and dstate_e/dt = coef * I_e.
 */
typedef struct {
    int family;
    int n_ext;
    const double *state;   /* device [n_ext] */
    const double *grid;    /* device: families 1, 4 rho[n_ext]; 2 p[n_ext]; 3 p, alpha and
                              5 p, p0 [2 n_ext]; 6 p, alpha, p01, p02 [4 n_ext] */
    frg_log_table Z;       /* families 2, 3, 5, 6 */
    int n_comp;            /* families 1, 4: N of O(N) (>= 1) */
    double m2_floor;       /* mass floor (-0.9 k^2 in the LPA workload) */
    double coef;           /* families 2, 3, 5, 6: dstate/dt = coef * I */
} frg_flow_state;

/* dstate_dt (device [n_ext]) = RHS(state) for one flow (see frg_flow_state).  The whole chain
 * state -> masses -> integrals -> assembly runs on the device.  The first call for a shape
 * builds a plan (work buffers, tile shape, kernel arguments) that later calls with the same
 * shape, pointers and stream reuse; pointer or shape changes build a new plan.  By default the
 * plan's kernels are launched directly on `stream`.  If the environment variable FRG_FLOW_GRAPH
 * is "1" when the context is created, the plan is captured once as a HIP graph and every call
 * replays it instead (on this platform a graph replay costs about 20 us more than direct
 * launches of a one- to three-kernel plan, so direct launch is the default). */
frg_status frg_flow_rhs(frg_context *ctx, const frg_integral_desc *desc,
                        const frg_flow_state *state, double *dstate_dt, hipStream_t stream);

/* ---- adaptive flow stepper ------------------------------------------------------------------ */

/*
 * Integrates a flow dstate/dt = RHS(state; k(t)) in RG time t = log(Lambda/k) (Sec. 2.1), with
 * k(t) = Lambda exp(-t) and Lambda = desc->k, by the explicit embedded Runge-Kutta pair of
 * Dormand and Prince, order 5(4), with first-same-as-last stages (the RK45 class of explicit
 * steppers of Sec. 5.2 "Time-stepping", favoured there for vertex expansions).  RHS is the
 * right-hand side of frg_flow_rhs for the same descriptor and flow state, re-evaluated at the
 * stage's k (rules, prefactors, dressing coordinates and, at finite temperature, the frequency
 * rule follow k; the dressing table and grid stay as given; the mass floor keeps its ratio to
 * k^2: m2_floor (k/Lambda)^2).
 *
 * Step control: err = sqrt(mean_i (e_i / (atol + rtol max(|y_i|, |ynew_i|)))^2) with e the
 * difference of the fifth- and fourth-order solutions; a step with err <= 1 is accepted; the
 * next step is h min(fac_max, max(0.2, 0.9 err^(-1/5))), fac_max = 5 (1 right after a
 * rejection), clipped to [h_min, h_max] and to the end of the interval.  fixed_step = 1 takes
 * steps of h0 (the last one shortened to end at t_end) without control.  method = 2 is the
 * Runge-Kutta-Fehlberg 7(8) pair instead (the RK78 class of the same section; E. Fehlberg,
 * NASA TR R-287, 1968): 13 right-hand sides per attempted step (a rejected step keeps its
 * first), the eighth-order solution kept, e = the difference of the eighth- and seventh-order
 * solutions (41/840 h (k_1 + k_11 - k_12 - k_13) up to sign), the same norm and rule with
 * exponent -1/8.
 *
 * Everything per step runs on `stream` on the device -- the stage vectors (seven; Fehlberg 13),
 * their right-hand sides, the stage combinations and the error norm -- except the accept/reject
 * decision, for which the host reads one float64 per step.  The state (flow_state.state) is
 * updated in place on the device; the stepper owns its stage buffers (allocated at creation).
 */
typedef struct {
    double rtol, atol;        /* > 0 */
    double h0;                /* first step (or the fixed step), > 0 */
    double h_min, h_max;      /* 0 < h_min <= h_max */
    int max_steps;            /* attempted steps per frg_stepper_advance call, >= 1 */
    int fixed_step;           /* 1: steps of exactly h0, no error control */
    int method;               /* 0: Dormand-Prince 5(4) as above; 2: Fehlberg 7(8) as above;
                                 3: Adams-Bashforth-Moulton 4 PECE with a variable step:
                                 Milne's estimate (19/270)(y_c - y_p) of the corrector's error
                                 in the norm above, err <= 1 accepts, next step h min(fmax,
                                 max(0.2, 0.9 err^(-1/5))) in [h_min, h_max] with fmax = 1.5 (1
                                 after a rejection; increases below 10 % not taken); whenever
                                 the step changes the right-hand-side history is moved onto the
                                 new spacing by the cubic through its four points; the first
                                 three steps are RK4 steps of h0; fixed_step not used;
                                 1: Adams-Bashforth-Moulton 4
                                 in PECE mode (predict with AB4, evaluate, correct with AM4,
                                 evaluate; Sec. 5.2 names the ABM class) with steps of exactly
                                 h0 and no error control (fixed_step, rtol and atol are not
                                 used, but still checked); the
                                 first three steps, and a last step shortened to end at t_end
                                 (after which the history restarts), are classical RK4 steps */
} frg_stepper_config;

typedef struct {
    double t;                 /* RG time reached */
    double h;                 /* next step size */
    double last_err;          /* error norm of the last attempted step (0 with fixed_step) */
    uint64_t accepted, rejected, rhs_evals;  /* totals since creation */
} frg_stepper_stats;

typedef struct frg_stepper frg_stepper;

/* The stepper starts at t = 0 (k = desc->k).  desc, state and cfg are copied; the device
 * buffers state->state (evolved in place), state->grid and state->Z.values must stay valid for
 * the stepper's lifetime.  Families as frg_flow_rhs. */
frg_status frg_stepper_create(frg_context *ctx, const frg_integral_desc *desc,
                              const frg_flow_state *state, const frg_stepper_config *cfg,
                              frg_stepper **out);
/* Advance to t_end (>= the current t) or until max_steps attempts; synchronises `stream` once
 * per step.  FRG_E_TIMEOUT if max_steps ran out first (the state is valid at stats->t),
 * FRG_E_INVAL if the step size fell below h_min or the error norm is not finite (the state is
 * the last accepted one). */
frg_status frg_stepper_advance(frg_stepper *st, double t_end, hipStream_t stream,
                               frg_stepper_stats *stats);
frg_status frg_stepper_destroy(frg_stepper *st);

/* ---- serving -------------------------------------------------------------------------------- */

typedef struct {
    int max_inflight;          /* launches in flight at once (>= 1) */
    size_t hbm_budget_bytes;   /* device bytes the session may hold for admitted requests;
                                  0 = the context budget */
    int poll_us;               /* while launches are in flight the scheduler checks them every
                                  poll_us microseconds, spinning (0 = 2); idle, it sleeps until
                                  a submission */
    int watchdog_ms;           /* a launch outstanding longer than this fails its tickets */
} frg_session_config;

typedef struct {
    double p50_us, p99_us;     /* submit -> result visible on the host, completed requests
                                  (from a histogram of 0.5 % wide logarithmic bins: the upper
                                  edge of the bin holding the percentile) */
    double gnodes_per_s;       /* integrand evaluations / busy wall time */
    uint64_t admitted, queued, rejected, completed, failed, cancelled;
    uint64_t nodes;            /* integrand evaluations completed */
    uint64_t launches;         /* fused launches issued */
    uint64_t tickets_held;     /* tickets the session still keeps (not yet reported, or still
                                  referenced by a running launch) */
    /* means over completed requests of the phases of their last launch: submit -> launch
       formed, formed -> enqueued on the device, enqueued -> completion seen, completion seen
       -> results in the client's buffers */
    double mean_queue_us, mean_launch_us, mean_device_us, mean_finish_us;
} frg_stats;

/* Pinned host staging of one launch slot of a session (bytes); a request whose inputs and
 * outputs need more than this minus the slot's launch tables (about 3 MiB) is rejected with
 * FRG_E_NOMEM at submit. */
#define FRG_SESSION_STAGING_BYTES ((size_t)32 << 20)

/* Requests submitted to a session hold HOST pointers (ext, m2, out, err_out, dout_dm2); the session
 * stages them into device memory it owns, admitted against the HBM budget, evaluates them in
 * fused launches that new arrivals join while earlier launches run (continuous batching), and
 * copies results back before the ticket completes.  A launch holds a bounded amount of work
 * (about 2e8 integrand nodes); a larger request is evaluated in parts of whole external tiles
 * over several launches (each result is still bitwise that of frg_integrate_batch).  Requests
 * are admitted in arrival order, except that requests that fit the budget may go ahead of one
 * that does not fit yet, a bounded number of times.  Pinned host staging (max_inflight x
 * FRG_SESSION_STAGING_BYTES) and the launch tables are allocated when the session opens.
 * A ticket is forgotten once frg_session_wait or frg_session_poll has reported its end (FRG_OK
 * or its failure status): later calls with it return FRG_E_INVAL. */
frg_status frg_session_open(frg_context *ctx, const frg_session_config *cfg, frg_session **out);
/* Copy a dressing table (host values) into device memory for the session's lifetime.
 * A request whose batch.Z.values is NULL and whose table_id >= 0 uses the resident table. */
frg_status frg_session_register_table(frg_session *s, const double *Z_host, int n, double x_min,
                                      double x_max, int *table_id);
/* Queue one request; returns immediately with a ticket.  FRG_E_NOMEM if the request alone
 * exceeds the session budget or a slot's host staging; FRG_E_INVAL on a bad descriptor or
 * batch. */
frg_status frg_session_submit(frg_session *s, const frg_integral_desc *desc,
                              const frg_batch *batch_host, int table_id, uint64_t *ticket);
/* *done = 1 when the ticket's results are in the host output buffers.  A ticket that failed
 * returns its failure status: FRG_E_TIMEOUT if the watchdog gave up on its launch, FRG_E_DEVICE
 * on a HIP error, FRG_E_CANCELLED if cancelled. */
frg_status frg_session_poll(frg_session *s, uint64_t ticket, int *done);
/* Block until the ticket completes (FRG_OK), fails, is cancelled, or timeout_ms passes
 * (FRG_E_TIMEOUT; timeout_ms < 0 waits forever). */
frg_status frg_session_wait(frg_session *s, uint64_t ticket, int timeout_ms);
/* Cancel a ticket that has not been launched yet (FRG_E_NOTREADY if already running). */
frg_status frg_session_cancel(frg_session *s, uint64_t ticket);
frg_status frg_session_stats(frg_session *s, frg_stats *out);
/* Drain in-flight work, fail queued tickets with FRG_E_CANCELLED, free the session. */
frg_status frg_session_close(frg_session *s);

#ifdef __cplusplus
}
#endif
#endif /* FRG_H */
