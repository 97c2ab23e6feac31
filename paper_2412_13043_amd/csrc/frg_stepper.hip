// Adaptive explicit stepper for flows dstate/dt = RHS(state; k(t)) in RG time t = log(Lambda/k),
// k(t) = Lambda exp(-t) (Sec. 2.1): the embedded Runge-Kutta pair of Dormand and Prince,
// order 5(4), with first-same-as-last stages, and the Runge-Kutta-Fehlberg 7(8) pair (the RK45
// and RK78 classes of explicit steppers named in Sec. 5.2, "Time-stepping"), and the fixed-step
// Adams-Bashforth-Moulton 4.  The stages, right-hand sides and the error norm run on the
// device; the host reads one float64 per step to accept or reject it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "frg_runtime.hpp"

namespace frg {
namespace {

// Dormand & Prince (1980), RK5(4)7FM: nodes c_s, stage coefficients a_sj, and e_j = b_j - bhat_j
// (fifth- minus fourth-order weights).  The fifth-order weights b are the last stage's row, so
// the last stage evaluates the right-hand side at the new solution, which is the next step's
// first stage when the step is accepted.
constexpr double kC[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};
constexpr double kA[7][6] = {
    {0.0, 0.0, 0.0, 0.0, 0.0, 0.0},
    {1.0 / 5.0, 0.0, 0.0, 0.0, 0.0, 0.0},
    {3.0 / 40.0, 9.0 / 40.0, 0.0, 0.0, 0.0, 0.0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0.0, 0.0, 0.0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0.0, 0.0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0.0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0}};
constexpr double kE[7] = {71.0 / 57600.0,      0.0,           -71.0 / 16695.0, 71.0 / 1920.0,
                          -17253.0 / 339200.0, 22.0 / 525.0, -1.0 / 40.0};

// E. Fehlberg (1968), the 13-stage Runge-Kutta 7(8) formulas: nodes, stage coefficients, the
// eighth-order weights (the solution kept) and e_j = b8_j - b7_j, nonzero on stages 1, 11, 12
// and 13 (the error estimate 41/840 h (k_1 + k_11 - k_12 - k_13), up to sign).
constexpr double kC78[13] = {0.0,       2.0 / 27.0, 1.0 / 9.0, 1.0 / 6.0, 5.0 / 12.0,
                             1.0 / 2.0, 5.0 / 6.0,  1.0 / 6.0, 2.0 / 3.0, 1.0 / 3.0,
                             1.0,       0.0,        1.0};
constexpr double kA78[13][12] = {
    {},
    {2.0 / 27.0},
    {1.0 / 36.0, 1.0 / 12.0},
    {1.0 / 24.0, 0.0, 1.0 / 8.0},
    {5.0 / 12.0, 0.0, -25.0 / 16.0, 25.0 / 16.0},
    {1.0 / 20.0, 0.0, 0.0, 1.0 / 4.0, 1.0 / 5.0},
    {-25.0 / 108.0, 0.0, 0.0, 125.0 / 108.0, -65.0 / 27.0, 125.0 / 54.0},
    {31.0 / 300.0, 0.0, 0.0, 0.0, 61.0 / 225.0, -2.0 / 9.0, 13.0 / 900.0},
    {2.0, 0.0, 0.0, -53.0 / 6.0, 704.0 / 45.0, -107.0 / 9.0, 67.0 / 90.0, 3.0},
    {-91.0 / 108.0, 0.0, 0.0, 23.0 / 108.0, -976.0 / 135.0, 311.0 / 54.0, -19.0 / 60.0,
     17.0 / 6.0, -1.0 / 12.0},
    {2383.0 / 4100.0, 0.0, 0.0, -341.0 / 164.0, 4496.0 / 1025.0, -301.0 / 82.0,
     2133.0 / 4100.0, 45.0 / 82.0, 45.0 / 164.0, 18.0 / 41.0},
    {3.0 / 205.0, 0.0, 0.0, 0.0, 0.0, -6.0 / 41.0, -3.0 / 205.0, -3.0 / 41.0, 3.0 / 41.0,
     6.0 / 41.0},
    {-1777.0 / 4100.0, 0.0, 0.0, -341.0 / 164.0, 4496.0 / 1025.0, -289.0 / 82.0,
     2193.0 / 4100.0, 51.0 / 82.0, 33.0 / 164.0, 12.0 / 41.0, 0.0, 1.0}};
constexpr double kB78[13] = {0.0,         0.0,          0.0,          0.0,         0.0,
                             34.0 / 105.0, 9.0 / 35.0,  9.0 / 35.0,   9.0 / 280.0, 9.0 / 280.0,
                             0.0,         41.0 / 840.0, 41.0 / 840.0};
constexpr double kE78[13] = {-41.0 / 840.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0,
                             -41.0 / 840.0, 41.0 / 840.0, 41.0 / 840.0};

constexpr int kMaxStages = 13;

// A linear combination sum_j c_j K_j of up to 13 stage vectors.
struct Combo {
    const double *K[kMaxStages];
    double c[kMaxStages];
    int nk;
};

// out = y + h sum_j c_j K_j (the stage terms in order j = 0, 1, ...).
// (y NULL: out = h sum_j c_j K_j.)
__global__ void __launch_bounds__(256) rk_combine_kernel(int n, const double *__restrict__ y,
                                                         double h, Combo k,
                                                         double *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < k.nk; ++j) s = fma(k.c[j], k.K[j][i], s);
    out[i] = y ? fma(h, s, y[i]) : h * s;
}

// One workgroup: err2 = sum_i (h sum_j e_j K_j[i] / (atol + rtol max(|y_i|, |yn_i|)))^2, each
// thread over a fixed stride, then a fixed tree in LDS (the same bits on every run).
__global__ void __launch_bounds__(256) rk_error_kernel(int n, const double *__restrict__ y,
                                                       const double *__restrict__ yn, double h,
                                                       Combo e, double rtol, double atol,
                                                       double *__restrict__ err2) {
    __shared__ double part[256];
    const int t = (int)threadIdx.x;
    double acc = 0.0;
    for (int i = t; i < n; i += 256) {
        double s = 0.0;
        for (int j = 0; j < e.nk; ++j) s = fma(e.c[j], e.K[j][i], s);
        const double sc = atol + rtol * fmax(fabs(y[i]), fabs(yn[i]));
        const double r = h * s / sc;
        acc = fma(r, r, acc);
    }
    part[t] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) part[t] += part[t + w];
        __syncthreads();
    }
    if (t == 0) err2[0] = part[0];
}

}  // namespace
}  // namespace frg

using namespace frg;

struct frg_stepper {
    frg_context *ctx = nullptr;
    frg_integral_desc desc{};  // k = Lambda (t = 0)
    frg_flow_state state{};
    frg_stepper_config cfg{};
    TileShape shape;
    bool lpa = false;
    int n = 0;
    DeviceBuffer stages;    // K_0..K_12, the stage input and the new solution: 15 n doubles
    DeviceBuffer contrib;   // radially chunked right-hand sides
    DeviceBuffer counters;  // float32 amplification slots (zero at rest)
    DeviceBuffer ftrule;    // finite temperature: the frequency rule at the stage's k
    DeviceBuffer err_dev;
    double *err_host = nullptr;
    double *K[kMaxStages] = {};
    double *ytmp = nullptr, *ynew = nullptr;
    // Adams-Bashforth-Moulton: f_n, f_{n-1}, f_{n-2}, f_{n-3} (in K[0..3], rotated) and how many
    // of them are valid
    double *F[4] = {};
    int hist = 0;
    double t = 0.0, h = 0.0, last_err = 0.0;  // h: the next step (variable ABM: the history's)
    bool fsal = false;     // K[0] holds RHS(t, state) (after a rejected step too)
    bool rejected_last = false;
    uint64_t accepted = 0, rejected = 0, evals = 0;
    ~frg_stepper() {
        if (err_host) (void)hipHostFree(err_host);
    }
};

namespace {

// RHS at RG time ts of the stage vector y into out, on stream s (caller holds ctx->mu).
frg_status stepper_rhs(frg_stepper *S, double ts, const double *y, double *out, hipStream_t s) {
    frg_integral_desc d = S->desc;
    const double scale = std::exp(-ts);  // k / Lambda
    d.k = S->desc.k * scale;
    // the mass floor keeps its ratio to k^2 (the propagator's pole moves with k^2)
    const double floor = S->state.m2_floor * scale * scale;
    frg_batch b;
    std::memset(&b, 0, sizeof b);
    b.n_ext = S->lpa ? 2 * S->n : S->n;
    b.ext = S->lpa ? nullptr : S->state.grid;
    b.m2 = y;
    b.Z = S->state.Z;
    b.out = out;
    RadialRule own;
    const RadialRule *rp = nullptr;
    frg_status st;
    if (is_ft(d.family)) {
        if ((st = ft_rule_into(S->ctx, d, S->ftrule.ptr, S->ftrule.bytes, &own, s)) != FRG_OK)
            return st;
        rp = &own;
    }
    ReqDev r;
    if (S->lpa)
        st = make_request(S->ctx, d, b, S->shape, 1, 0.0, 1.0, &r, rp);
    else
        st = make_request(S->ctx, d, b, S->shape, 2, floor, S->state.coef, &r, rp);
    if (st != FRG_OK) return st;
    r.contrib_base = 0;
    r.ctr_base = 0;
    if (S->lpa) {
        FRG_HIP_CHECK(launch_lpa_rhs(r, S->n, S->state.n_comp, S->state.grid, y, floor, out, s));
    } else {
        FRG_HIP_CHECK(launch_batch(&r, nullptr, tile_count(r), lds_bytes_for(r),
                                   (double *)S->contrib.ptr, (unsigned *)S->counters.ptr, s));
        FRG_HIP_CHECK(launch_finalize(r, (const double *)S->contrib.ptr,
                                      (unsigned *)S->counters.ptr, s));
    }
    ++S->evals;
    return FRG_OK;
}

hipError_t combine(int n, const double *y, double h, const double *const *K, const double *c,
                   int nk, double *out, hipStream_t s) {
    Combo k;
    std::memset(&k, 0, sizeof k);
    for (int j = 0; j < nk; ++j) {
        k.K[j] = K[j];
        k.c[j] = c[j];
    }
    k.nk = nk;
    hipLaunchKernelGGL(rk_combine_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, y, h, k, out);
    return hipGetLastError();
}

// Adams-Bashforth (order 4) predictor and Adams-Moulton (order 4) corrector weights over the
// history f_n, f_{n-1}, ... (the corrector's first weight is that of f at the predicted point),
// and the classical RK4 stage nodes and weights of the start.
constexpr double kAB4[4] = {55.0 / 24.0, -59.0 / 24.0, 37.0 / 24.0, -9.0 / 24.0};
constexpr double kAM4[4] = {9.0 / 24.0, 19.0 / 24.0, -5.0 / 24.0, 1.0 / 24.0};
constexpr double kRK4B[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};

// One classical RK4 step of size h from (t, y) with k1 = F[0] into ynew (stages in K[4..6]).
frg_status rk4_step(frg_stepper *S, double h, const double *y, hipStream_t s) {
    const int n = S->n;
    const double half = 0.5, one = 1.0;
    double *k[4] = {S->F[0], S->K[4], S->K[5], S->K[6]};
    frg_status st;
    for (int j = 1; j < 4; ++j) {
        const double *prev[1] = {k[j - 1]};
        FRG_HIP_CHECK(combine(n, y, h, prev, j < 3 ? &half : &one, 1, S->ytmp, s));
        if ((st = stepper_rhs(S, S->t + (j < 3 ? 0.5 : 1.0) * h, S->ytmp, k[j], s)) != FRG_OK)
            return st;
    }
    FRG_HIP_CHECK(combine(n, y, h, (const double *const *)k, kRK4B, 4, S->ynew, s));
    return FRG_OK;
}

// Fixed-step Adams-Bashforth-Moulton 4 in PECE mode (steps of h0; RK4 start and shortened
// last step, after which the history restarts).
frg_status abm_advance(frg_stepper *S, double t_end, hipStream_t s, int *attempts_out) {
    const frg_stepper_config &c = S->cfg;
    const int n = S->n;
    double *y = const_cast<double *>(S->state.state);
    int attempts = 0;
    frg_status st;
    while (S->t < t_end) {
        if (attempts >= c.max_steps) {
            set_error("max_steps (%d) attempted before t_end", c.max_steps);
            *attempts_out = attempts;
            return FRG_E_TIMEOUT;
        }
        ++attempts;
        double h = c.h0;
        const bool last = S->t + h >= t_end * (1.0 - 1e-14) - 1e-300;
        if (last) h = t_end - S->t;
        const bool shortened = last && h < c.h0 * (1.0 - 1e-9);
        std::lock_guard<std::mutex> lk(S->ctx->mu);
        if (S->hist == 0) {
            if ((st = stepper_rhs(S, S->t, y, S->F[0], s)) != FRG_OK) return st;
            S->hist = 1;
        }
        if (shortened || S->hist < 4) {
            if ((st = rk4_step(S, h, y, s)) != FRG_OK) return st;
        } else {
            FRG_HIP_CHECK(combine(n, y, h, (const double *const *)S->F, kAB4, 4, S->ytmp, s));
            if ((st = stepper_rhs(S, S->t + h, S->ytmp, S->K[4], s)) != FRG_OK) return st;
            const double *corr[4] = {S->K[4], S->F[0], S->F[1], S->F[2]};
            FRG_HIP_CHECK(combine(n, y, h, corr, kAM4, 4, S->ynew, s));
        }
        FRG_HIP_CHECK(hipMemcpyAsync(y, S->ynew, (size_t)n * sizeof(double),
                                     hipMemcpyDeviceToDevice, s));
        S->t = last ? t_end : S->t + h;
        if (shortened) {
            S->hist = 0;  // the history was taken at step h0
        } else {
            double *oldest = S->F[3];
            for (int j = 3; j > 0; --j) S->F[j] = S->F[j - 1];
            S->F[0] = oldest;
        }
        if ((st = stepper_rhs(S, S->t, y, S->F[0], s)) != FRG_OK) return st;
        S->hist = std::min(S->hist + 1, 4);
        ++S->accepted;
    }
    *attempts_out = attempts;
    return FRG_OK;
}

// The history f_n, f_{n-1}, f_{n-2}, f_{n-3} (spacing h) moved to spacing ratio h: the cubic
// through the four points at s = j ratio old steps back (Lagrange), into the spare stage
// buffers, which then become the history.
frg_status respace(frg_stepper *S, double ratio, hipStream_t s) {
    double *spare[3] = {S->K[4], S->K[5], S->K[6]};
    for (int j = 1; j < 4; ++j) {
        const double x = j * ratio;
        double w[4];
        for (int i = 0; i < 4; ++i) {
            w[i] = 1.0;
            for (int m = 0; m < 4; ++m)
                if (m != i) w[i] *= (x - m) / (double)(i - m);
        }
        FRG_HIP_CHECK(combine(S->n, nullptr, 1.0, (const double *const *)S->F, w, 4,
                              spare[j - 1], s));
    }
    for (int j = 1; j < 4; ++j) {
        double *old = S->F[j];
        S->F[j] = spare[j - 1];
        // the freed buffer takes the spare's place among K[4..6]
        S->K[3 + j] = old;
    }
    return FRG_OK;
}

// Adams-Bashforth-Moulton 4 PECE with a variable step: Milne's estimate (19/270)(y_c - y_p) of
// the corrector's local error in the norm of the Runge-Kutta pairs, err <= 1 accepts; next step
// h min(fmax, max(0.2, 0.9 err^(-1/5))) in [h_min, h_max], fmax = 1.5 (1 after a rejection), no
// increase below 10 %; the history re-spaced by its cubic whenever the step changes; RK4 steps
// of h0 build the first history.
frg_status abm_var_advance(frg_stepper *S, double t_end, hipStream_t s, int *attempts_out) {
    const frg_stepper_config &c = S->cfg;
    const int n = S->n;
    double *y = const_cast<double *>(S->state.state);
    int attempts = 0;
    frg_status st;
    const double milne[2] = {19.0 / 270.0, -19.0 / 270.0};
    while (S->t < t_end) {
        if (attempts >= c.max_steps) {
            set_error("max_steps (%d) attempted before t_end", c.max_steps);
            *attempts_out = attempts;
            return FRG_E_TIMEOUT;
        }
        ++attempts;
        double h = S->h;
        const bool last = S->t + h >= t_end * (1.0 - 1e-14) - 1e-300;
        if (last) h = t_end - S->t;
        std::unique_lock<std::mutex> lk(S->ctx->mu);
        if (S->hist == 0) {
            if ((st = stepper_rhs(S, S->t, y, S->F[0], s)) != FRG_OK) return st;
            S->hist = 1;
        }
        if (S->hist < 4) {
            // start: RK4 (a shortened last one restarts the history from its end point)
            if ((st = rk4_step(S, h, y, s)) != FRG_OK) return st;
            FRG_HIP_CHECK(hipMemcpyAsync(y, S->ynew, (size_t)n * sizeof(double),
                                         hipMemcpyDeviceToDevice, s));
            S->t = last ? t_end : S->t + h;
            const bool keep = h == S->h;
            double *oldest = S->F[3];
            for (int j = 3; j > 0; --j) S->F[j] = S->F[j - 1];
            S->F[0] = oldest;
            if ((st = stepper_rhs(S, S->t, y, S->F[0], s)) != FRG_OK) return st;
            S->hist = keep ? std::min(S->hist + 1, 4) : 1;
            ++S->accepted;
            continue;
        }
        if (h != S->h && (st = respace(S, h / S->h, s)) != FRG_OK) return st;
        FRG_HIP_CHECK(combine(n, y, h, (const double *const *)S->F, kAB4, 4, S->ytmp, s));
        if ((st = stepper_rhs(S, S->t + h, S->ytmp, S->K[7], s)) != FRG_OK) return st;
        const double *corr[4] = {S->K[7], S->F[0], S->F[1], S->F[2]};
        FRG_HIP_CHECK(combine(n, y, h, corr, kAM4, 4, S->ynew, s));
        Combo e;
        std::memset(&e, 0, sizeof e);
        e.K[0] = S->ynew;
        e.K[1] = S->ytmp;
        e.c[0] = milne[0];
        e.c[1] = milne[1];
        e.nk = 2;
        hipLaunchKernelGGL(rk_error_kernel, dim3(1), dim3(256), 0, s, n, y, S->ynew, 1.0, e,
                           c.rtol, c.atol, (double *)S->err_dev.ptr);
        FRG_HIP_CHECK(hipGetLastError());
        FRG_HIP_CHECK(hipMemcpyAsync(S->err_host, S->err_dev.ptr, sizeof(double),
                                     hipMemcpyDeviceToHost, s));
        FRG_HIP_CHECK(hipStreamSynchronize(s));
        const double err = std::sqrt(*S->err_host / (double)n);
        if (!std::isfinite(err)) {
            set_error("error norm is not finite at t = %g (h = %g)", S->t, h);
            return FRG_E_INVAL;
        }
        S->last_err = err;
        if (err <= 1.0) {
            FRG_HIP_CHECK(hipMemcpyAsync(y, S->ynew, (size_t)n * sizeof(double),
                                         hipMemcpyDeviceToDevice, s));
            S->t = last ? t_end : S->t + h;
            double *oldest = S->F[3];
            for (int j = 3; j > 0; --j) S->F[j] = S->F[j - 1];
            S->F[0] = oldest;
            if ((st = stepper_rhs(S, S->t, y, S->F[0], s)) != FRG_OK) return st;
            ++S->accepted;
            double fac = err > 0.0 ? 0.9 * std::pow(err, -0.2) : 1.5;
            fac = std::min(S->rejected_last ? 1.0 : 1.5, std::max(0.2, fac));
            if (fac >= 1.0 && fac < 1.1) fac = 1.0;
            const double hn = std::min(std::max(h * fac, c.h_min), c.h_max);
            S->h = h;  // the history's spacing
            if (hn != h && (st = respace(S, hn / h, s)) != FRG_OK) return st;
            S->h = hn;
            S->rejected_last = false;
        } else {
            ++S->rejected;
            S->rejected_last = true;
            if (h <= c.h_min) {
                set_error("step size at h_min = %g rejected at t = %g (err = %g)", c.h_min, S->t,
                          err);
                *attempts_out = attempts;
                return FRG_E_INVAL;
            }
            const double fac = std::min(1.0, std::max(0.2, 0.9 * std::pow(err, -0.2)));
            const double hn = std::min(std::max(h * fac, c.h_min), c.h_max);
            if ((st = respace(S, hn / h, s)) != FRG_OK) return st;
            S->h = hn;
        }
    }
    *attempts_out = attempts;
    return FRG_OK;
}

}  // namespace

extern "C" {

frg_status frg_stepper_create(frg_context *ctx, const frg_integral_desc *desc,
                              const frg_flow_state *state, const frg_stepper_config *cfg,
                              frg_stepper **out) {
    clear_error();
    if (!ctx || !desc || !state || !cfg || !out) {
        set_error("null argument to frg_stepper_create");
        return FRG_E_INVAL;
    }
    const frg_stepper_config &c = *cfg;
    if (!(c.rtol > 0.0) || !(c.atol > 0.0) || !(c.h0 > 0.0) || !(c.h_min > 0.0) ||
        !(c.h_max >= c.h_min) || !std::isfinite(c.h_max) || !std::isfinite(c.rtol) ||
        !std::isfinite(c.atol) || !std::isfinite(c.h0) || c.max_steps < 1 ||
        (c.fixed_step != 0 && c.fixed_step != 1) || c.method < 0 || c.method > 3) {
        set_error("stepper config needs rtol, atol, h0 > 0, 0 < h_min <= h_max (finite), "
                  "max_steps >= 1, fixed_step 0 or 1, method 0 to 3");
        return FRG_E_INVAL;
    }
    if (state->family != desc->family) {
        set_error("flow state family %d does not match descriptor family %d", state->family,
                  desc->family);
        return FRG_E_INVAL;
    }
    if (desc->complex_freq) {
        set_error("complex external frequencies give complex integrals: no flow to integrate");
        return FRG_E_UNSUPPORTED;
    }
    const bool lpa = is_lpa(desc->family);
    const int n = state->n_ext;
    if (!state->state || !state->grid || n < (lpa ? 3 : 1)) {
        set_error("flow state needs state and grid pointers and n_ext >= %d", lpa ? 3 : 1);
        return FRG_E_INVAL;
    }
    if (lpa && state->n_comp < 1) {
        set_error("n_comp must be >= 1");
        return FRG_E_INVAL;
    }
    if (!std::isfinite(state->m2_floor) || !std::isfinite(state->coef)) {
        set_error("m2_floor and coef must be finite");
        return FRG_E_INVAL;
    }
    frg_batch b;
    std::memset(&b, 0, sizeof b);
    b.n_ext = lpa ? 2 * n : n;
    b.ext = lpa ? nullptr : state->grid;
    b.m2 = state->state;
    b.Z = state->Z;
    b.out = const_cast<double *>(state->state);  // the state is evolved in place
    frg_status st = validate(desc, &b, true);
    if (st != FRG_OK) return st;

    auto S = std::make_unique<frg_stepper>();
    S->ctx = ctx;
    S->desc = *desc;
    S->state = *state;
    S->cfg = c;
    S->lpa = lpa;
    S->n = n;
    S->h = std::min(std::max(c.h0, c.h_min), c.h_max);
    std::lock_guard<std::mutex> lk(ctx->mu);
    FRG_HIP_CHECK(hipSetDevice(ctx->device));
    S->shape = choose_shape(ctx, *desc, b.n_ext, 16 * ctx->num_cus);
    // work buffers sized at t = 0: at finite temperature with a k-scaled frequency domain the
    // number of frequencies only falls as k does
    ReqDev r;
    if ((st = make_request(ctx, *desc, b, S->shape, lpa ? 1 : 2, state->m2_floor, state->coef,
                           &r)) != FRG_OK)
        return st;
    FRG_HIP_CHECK(S->stages.alloc((size_t)(kMaxStages + 2) * n * sizeof(double)));
    double *base = (double *)S->stages.ptr;
    for (int j = 0; j < kMaxStages; ++j) S->K[j] = base + (size_t)j * n;
    for (int j = 0; j < 4; ++j) S->F[j] = S->K[j];
    S->ytmp = base + (size_t)kMaxStages * n;
    S->ynew = base + (size_t)(kMaxStages + 1) * n;
    FRG_HIP_CHECK(S->contrib.alloc(std::max<size_t>(contrib_doubles(r), 1) * sizeof(double)));
    const size_t nc = std::max<size_t>(counter_count(r), 1);
    FRG_HIP_CHECK(S->counters.alloc(nc * sizeof(unsigned)));
    FRG_HIP_CHECK(launch_fill_zero_u32((unsigned *)S->counters.ptr, nc, ctx->aux));
    if (is_ft(desc->family)) {
        FreqRule f;
        if ((st = freq_rule(*desc, &f)) != FRG_OK) return st;
        FRG_HIP_CHECK(S->ftrule.alloc(ft_rule_bytes(desc->n_q, f.n_f)));
    }
    FRG_HIP_CHECK(S->err_dev.alloc(sizeof(double)));
    FRG_HIP_CHECK(hipHostMalloc((void **)&S->err_host, sizeof(double), hipHostMallocDefault));
    FRG_HIP_CHECK(hipStreamSynchronize(ctx->aux));
    *out = S.release();
    return FRG_OK;
}

frg_status frg_stepper_advance(frg_stepper *S, double t_end, hipStream_t s,
                               frg_stepper_stats *stats) {
    clear_error();
    if (!S) {
        set_error("stepper is NULL");
        return FRG_E_INVAL;
    }
    if (!std::isfinite(t_end) || t_end < S->t) {
        set_error("t_end must be finite and >= the current t = %g", S->t);
        return FRG_E_INVAL;
    }
    const frg_stepper_config &c = S->cfg;
    const int n = S->n;
    double *y = const_cast<double *>(S->state.state);
    frg_status res = FRG_OK;
    int attempts = 0;
    {
        std::lock_guard<std::mutex> lk(S->ctx->mu);
        FRG_HIP_CHECK(hipSetDevice(S->ctx->device));
    }
    if (c.method == 1) res = abm_advance(S, t_end, s, &attempts);
    if (c.method == 3) res = abm_var_advance(S, t_end, s, &attempts);
    // the embedded pairs: Dormand-Prince 5(4) (first same as last) or Fehlberg 7(8)
    const bool f78 = c.method == 2;
    const int ns = f78 ? 13 : 7;
    const double *cn = f78 ? kC78 : kC;
    const double *er = f78 ? kE78 : kE;
    const double expo = f78 ? -0.125 : -0.2;  // -1/(lower order + 1)
    while ((c.method == 0 || c.method == 2) && S->t < t_end) {
        if (attempts >= c.max_steps) {
            set_error("max_steps (%d) attempted before t_end", c.max_steps);
            res = FRG_E_TIMEOUT;
            break;
        }
        ++attempts;
        double h = c.fixed_step ? c.h0 : S->h;
        const bool last = S->t + h >= t_end * (1.0 - 1e-14) - 1e-300;
        if (last) h = t_end - S->t;
        frg_status st = FRG_OK;
        {
            std::lock_guard<std::mutex> lk(S->ctx->mu);
            if (!S->fsal) {
                if ((st = stepper_rhs(S, S->t, y, S->K[0], s)) != FRG_OK) return st;
                S->fsal = true;
            }
            for (int st_i = 1; st_i < ns; ++st_i) {
                // Dormand-Prince: the last stage's input is the new solution
                double *in = (!f78 && st_i == 6) ? S->ynew : S->ytmp;
                const double *a = f78 ? kA78[st_i] : kA[st_i];
                FRG_HIP_CHECK(combine(n, y, h, (const double *const *)S->K, a, st_i, in, s));
                if ((st = stepper_rhs(S, S->t + cn[st_i] * h, in, S->K[st_i], s)) != FRG_OK)
                    return st;
            }
            if (f78)
                FRG_HIP_CHECK(combine(n, y, h, (const double *const *)S->K, kB78, 13, S->ynew, s));
        }
        double err = 0.0;
        if (!c.fixed_step) {
            Combo e;
            std::memset(&e, 0, sizeof e);
            for (int j = 0; j < ns; ++j) {
                if (er[j] == 0.0) continue;
                e.K[e.nk] = S->K[j];
                e.c[e.nk] = er[j];
                ++e.nk;
            }
            hipLaunchKernelGGL(rk_error_kernel, dim3(1), dim3(256), 0, s, n, y, S->ynew, h, e,
                               c.rtol, c.atol, (double *)S->err_dev.ptr);
            FRG_HIP_CHECK(hipGetLastError());
            FRG_HIP_CHECK(hipMemcpyAsync(S->err_host, S->err_dev.ptr, sizeof(double),
                                         hipMemcpyDeviceToHost, s));
            FRG_HIP_CHECK(hipStreamSynchronize(s));
            err = std::sqrt(*S->err_host / (double)n);
            if (!std::isfinite(err)) {
                set_error("error norm is not finite at t = %g (h = %g)", S->t, h);
                return FRG_E_INVAL;
            }
        }
        S->last_err = err;
        if (c.fixed_step || err <= 1.0) {
            FRG_HIP_CHECK(hipMemcpyAsync(y, S->ynew, (size_t)n * sizeof(double),
                                         hipMemcpyDeviceToDevice, s));
            if (f78)
                S->fsal = false;  // no stage sits at the new solution
            else
                std::swap(S->K[0], S->K[6]);  // the last stage is RHS(t + h, ynew)
            S->t = last ? t_end : S->t + h;
            ++S->accepted;
            if (c.fixed_step) continue;
            const double fac = err > 0.0 ? 0.9 * std::pow(err, expo) : 5.0;
            const double fac_max = S->rejected_last ? 1.0 : 5.0;
            S->h = std::min(std::max(h * std::min(fac_max, std::max(0.2, fac)), c.h_min), c.h_max);
            S->rejected_last = false;
        } else {
            ++S->rejected;
            S->rejected_last = true;
            if (h <= c.h_min) {
                set_error("step size at h_min = %g rejected at t = %g (err = %g)", c.h_min, S->t,
                          err);
                res = FRG_E_INVAL;
                break;
            }
            const double fac = 0.9 * std::pow(err, expo);
            S->h = std::min(std::max(h * std::min(1.0, std::max(0.2, fac)), c.h_min), c.h_max);
        }
    }
    // the last state copy is queued on s: the state is final when the call returns
    FRG_HIP_CHECK(hipStreamSynchronize(s));
    if (stats) {
        stats->t = S->t;
        stats->h = S->h;
        stats->last_err = S->last_err;
        stats->accepted = S->accepted;
        stats->rejected = S->rejected;
        stats->rhs_evals = S->evals;
    }
    return res;
}

frg_status frg_stepper_destroy(frg_stepper *S) {
    clear_error();
    if (!S) return FRG_OK;
    (void)hipSetDevice(S->ctx->device);
    (void)hipDeviceSynchronize();
    delete S;
    return FRG_OK;
}

}  // extern "C"
