// HIP kernels for gfx950 (CDNA4): quadrature rules, the per-tile loop-integral bodies of the
// three integrand families in float64 and in the float32 precision form, the fused multi-request
// consumer, and the fused LPA right-hand side.
//
// Work decomposition.  A workgroup is one 64-lane wavefront.  A tile is (request, external tile,
// radial chunk).  For the LPA family one lane owns one external point and the whole radial sum.
// For the vertex families the lanes of a point share its radial nodes (and, three-point, its
// cos1 nodes); each (point, radial node) contribution is a fixed sequence of operations, and the
// point's result adds the contributions in radial order -- within the wavefront by cross-lane
// pulls when the tile holds every radial node, else through a [n_q][n_ext] scratch block that a
// finalize kernel sums in radial order.  Each result therefore depends only on its own request, never on the
// tiling, batch composition or launch shape.
//
// All device code is built with -ffp-contract=off: every fused multiply-add is written out with
// fma(), so the operation sequence (and so the rounding) is fixed by the source.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "frg_internal.hpp"
#include "frg_math.hpp"

namespace frg {

// --------------------------------------------------------------------------------------------
// Quadrature rules
// --------------------------------------------------------------------------------------------
// Gauss-Legendre roots written as x = cos(theta): Newton's method in theta on P_n(cos theta),
// with P_n and P_n' from the three-term recurrence and the derivative recurrence
// P'_{j+1} = P'_{j-1} + (2j+1) P_j.  Working in theta keeps 1 +- x = 2 cos^2(theta/2),
// 2 sin^2(theta/2) and sqrt(1 - x^2) = sin(theta) accurate at the ends of the interval.
__device__ static void legendre_pd(int n, double x, double &p, double &dp) {
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    for (int j = 1; j < n; ++j) {
        double p2 = ((2.0 * j + 1.0) * x * p1 - (double)j * p0) / (double)(j + 1);
        double d2 = d0 + (2.0 * j + 1.0) * p1;
        p0 = p1;
        p1 = p2;
        d0 = d1;
        d1 = d2;
    }
    p = p1;
    dp = d1;
}

// i-th root in increasing theta (decreasing x); returns theta and the [-1, 1] weight.
__device__ static void gl_root(int n, int i, double &theta, double &w) {
    const double pi = 3.141592653589793238462643383279502884;
    double t = pi * (4.0 * i + 3.0) / (4.0 * n + 2.0);
    double p = 0.0, dp = 1.0;
    for (int it = 0; it < 30; ++it) {
        legendre_pd(n, cos(t), p, dp);
        // d/dtheta P_n(cos theta) = -sin(theta) P_n'(cos theta)
        double step = p / (sin(t) * dp);
        t += step;
        if (fabs(step) < 1e-15 * t) {
            legendre_pd(n, cos(t), p, dp);
            t += p / (sin(t) * dp);
            break;
        }
    }
    legendre_pd(n, cos(t), p, dp);
    double s = sin(t);
    theta = t;
    w = 2.0 / (s * s * dp * dp);
}

// e = exp(-y) and E = expm1(-y) for y >= 0, both to full relative precision (the regulator
// derivative at the radial nodes multiplies e directly, so e must stay accurate when tiny).
__device__ __forceinline__ void exp_pair64(double y, double &e, double &E) {
    if (y < 0.69314718055994530942) {
        E = expm1(-y);
        e = 1.0 + E;
    } else {
        e = exp(-y);
        E = e - 1.0;
    }
}

// Propagator variant: E = expm1(-y) to full relative precision and e = 1 + E.  e is accurate to
// 1e-16 absolute, which is all the propagator needs: where e is tiny its term l2 e is below
// 1e-16 of the denominator.
__device__ __forceinline__ void exp_pair64_prop(double y, double &e, double &E) {
    E = expm1(-y);
    e = 1.0 + E;
}

__global__ void __launch_bounds__(64) rules_kernel(
    int n_q, double q_max, int d, int n_x, int n_phi, double *q, double *W, double *R, float *qf,
    float *Wf, float *Rf, double *x, double *xw, double *xs, float *xf, float *xwf, float *xsf,
    double *fc, double *fw, float *fcf, float *fwf, int plain, int reg, int reg_n) {
    const double pi = 3.141592653589793238462643383279502884;
    int which = blockIdx.y;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (which == 0 && i < n_q) {
        double th, w;
        gl_root(n_q, i, th, w);
        double c = cos(0.5 * th);
        double qh = q_max * c * c;  // (q_max/2)(1 + cos theta)
        double wh = 0.5 * q_max * w;
        double y = qh * qh;          // k = 1
        double Rh, Rd;
        if (reg == 1) {
            // R = exp(-S_N(y)), k dR/dk = 2 exp(-S_N(y)) (1 + y S_N'(y)), y S_N' = sum_i y^i
            double sn = 1.0 / reg_n, pn = 1.0;
            for (int j = reg_n - 1; j >= 1; --j) {
                sn = fma(sn, y, 1.0 / j);
                pn = fma(pn, y, 1.0);
            }
            const double e = exp(-fmin(sn * y, 1000.0));
            Rh = e;
            Rd = 2.0 * e * fma(pn, y, 1.0);
        } else if (reg == 2) {
            // flat: R = 1 - y, k dR/dk = 2 below y = 1; both 0 from y = 1 on
            Rh = y < 1.0 ? 1.0 - y : 0.0;
            Rd = y < 1.0 ? 2.0 : 0.0;
        } else if (y > 0.0) {
            double e, E;
            exp_pair64(y, e, E);
            Rh = y * e / (-E);
            Rd = 2.0 * y * y * e / (E * E);
        } else {
            Rh = 1.0;
            Rd = 2.0;
        }
        double qp = 1.0;
        for (int j = 0; j < d - 1; ++j) qp *= qh;
        int slot = n_q - 1 - i;  // ascending q
        q[slot] = qh;
        W[slot] = wh * qp * Rd;
        R[slot] = Rh;
        qf[slot] = (float)qh;
        Wf[slot] = (float)(wh * qp * Rd);
        Rf[slot] = (float)Rh;
    } else if (which == 1 && i < n_x) {
        double th, w;
        gl_root(n_x, i, th, w);
        double xv = cos(th), sv = sin(th);
        int slot = n_x - 1 - i;  // ascending x
        // d = 4: dx sqrt(1 - x^2) from the second polar angle; d = 3 (kPlainCos1): dx alone
        const double wx = (plain & kPlainCos1) ? w : w * sv;
        x[slot] = xv;
        xs[slot] = sv;
        xw[slot] = wx;
        xf[slot] = (float)xv;
        xsf[slot] = (float)sv;
        xwf[slot] = (float)wx;
    } else if (which == 2 && i < n_phi) {
        double th, w;
        gl_root(n_phi, i, th, w);
        double c = cos(0.5 * th);
        double ph = pi * c * c;  // (pi/2)(1 + cos theta), ascending in slot order
        double wp = 0.5 * pi * w;
        int slot = n_phi - 1 - i;
        double sp, cp;
        sincos(ph, &sp, &cp);
        // d = 4: dphi sin(phi) from the third polar angle; d = 3 (kPlainPhi): the azimuth, dphi
        const double wf = (plain & kPlainPhi) ? wp : wp * sp;
        fc[slot] = cp;
        fw[slot] = wf;
        fcf[slot] = (float)cp;
        fwf[slot] = (float)wf;
    }
}

hipError_t launch_rules(int n_q, double q_max, int d, int n_x, int n_phi, double *q, double *W,
                        double *R, float *qf, float *Wf, float *Rf, double *x, double *xw,
                        double *xs, float *xf, float *xwf, float *xsf, double *fc, double *fw,
                        float *fcf, float *fwf, hipStream_t s, int plain, int reg, int reg_n) {
    int nmax = n_q > n_x ? n_q : n_x;
    nmax = nmax > n_phi ? nmax : n_phi;
    dim3 grid((nmax + 63) / 64, 3);
    hipLaunchKernelGGL(rules_kernel, grid, dim3(64), 0, s, n_q, q_max, d, n_x, n_phi, q, W, R,
                       qf, Wf, Rf, x, xw, xs, xf, xwf, xsf, fc, fw, fcf, fwf, plain, reg, reg_n);
    return hipGetLastError();
}

// Finite-temperature radial rule: entry i = a n_f + j of radial node a and frequency j (the
// frequencies of one radial node adjacent, so that a wavefront's lanes share one spatial node
// and whole wavefronts take the far-field path together).
__global__ void __launch_bounds__(64) ft_rule_kernel(
    int n_q, int n_f, int n_tail, int n_lo, double eta, double T, double Omega, double k,
    const double *bq, const double *bW, const double *bR, double *q, double *W, double *R,
    float *qf, float *Wf, float *Rf, double *w0) {
    const double pi = 3.141592653589793238462643383279502884;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n_q * n_f) return;
    const int a = (int)(i / n_f);
    const int j = (int)(i - (long long)a * n_f);
    double w, c;
    if (j < n_tail || j >= n_f - n_tail) {
        // tail node: t_s (ascending) = GL root on [0, 1]; negative side first (w = -Omega/t,
        // ascending in w for ascending t), positive side mirrored (w = Omega/t, descending t)
        const int s = j < n_tail ? j : n_f - 1 - j;
        double th, gw;
        gl_root(n_tail, n_tail - 1 - s, th, gw);  // root index n-1-s is the s-th smallest
        const double ch = cos(0.5 * th);
        const double t = ch * ch;
        w = (j < n_tail ? -Omega : Omega) / t;
        c = Omega * (0.5 * gw) / (t * t) / (2.0 * pi);
    } else {
        w = 2.0 * pi * T * ((double)(n_lo + (j - n_tail)) + eta);
        c = T;
    }
    const double wh = w / k;
    const double Ri = fma(wh, wh, bR[a]);
    const double Wi = bW[a] * (c / k);
    q[i] = bq[a];
    R[i] = Ri;
    W[i] = Wi;
    qf[i] = (float)bq[a];
    Rf[i] = (float)Ri;
    Wf[i] = (float)Wi;
    w0[i] = w;
}

__global__ void __launch_bounds__(256) rule_sum_kernel(const double *q, const double *R,
                                                      double *A, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) A[i] = fma(q[i], q[i], R[i]);
}

hipError_t launch_rule_sum(const double *q, const double *R, double *A, long long n,
                           hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(rule_sum_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, q, R,
                       A, n);
    return hipGetLastError();
}

hipError_t launch_ft_rule(int n_q, int n_f, int n_tail, int n_lo, double eta, double T,
                          double Omega, double k, const RadialRule &base, double *q, double *W,
                          double *R, float *qf, float *Wf, float *Rf, double *w0, hipStream_t s) {
    const long long n = (long long)n_q * n_f;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(ft_rule_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, n_q, n_f,
                       n_tail, n_lo, eta, T, Omega, k, base.q, base.W, base.R, q, W, R, qf, Wf, Rf,
                       w0);
    return hipGetLastError();
}

// --------------------------------------------------------------------------------------------
// Float64 integrand pieces
// --------------------------------------------------------------------------------------------
// Smallest momentum squared fed to the propagator.  l2 <= 0 only arises from rounding; with
// l2 = 1e-300 the propagator equals its l2 = 0 limit 1/(k^2 + m2) to within 1e-300 relative, the
// dressing clamps to its first entry, and no 0/0 occurs in the single-division form below.
// A leg along the cos1 angle needs no clamp: Gauss-Legendre nodes are interior,
// |x| <= 1 - 2.3e-6 for n <= 1024, and l2 = q^2 + p^2 + 2qpx >= (1 - |x|)(q^2 + p^2), far above
// the few ulp of q^2 + p^2 that its evaluation can err by.  The three-point leg through phi can
// come arbitrarily close to zero (alpha on a node angle, phi near 0) and keeps the clamp.
#define FRG_L2_TINY 1e-300

// Quadrature rules stay constant while an integrand kernel runs.  Reading them through the
// constant address space lets the compiler use scalar loads for the wave-uniform rule entries
// (batched and issued ahead of use) instead of a vector memory round trip per inner-loop step,
// which it must otherwise assume the kernel's own stores may alias.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *kc(const T *p) {
    return (const __attribute__((address_space(4))) T *)p;
}

// Occupancy targets (waves per SIMD) of the integrand kernels; they bound the VGPR budget.  The
// two-point kernels fit 5 waves; the three-point kernels and the general fused kernel (every
// family and precision) are held to 4, where they keep their working set in registers.
#ifndef FRG_WAVES_PER_EU_BATCH
#define FRG_WAVES_PER_EU_BATCH 5
#endif
#ifndef FRG_WAVES_PER_EU_MULTI
#define FRG_WAVES_PER_EU_MULTI 4
// mass-derivative instances carry a second set of accumulators
#define FRG_WAVES_PER_EU_DER 4
#define FRG_WAVES_PER_EU_DER3 3
#endif
// Propagators evaluated together per inner-loop step (instruction-level parallelism).
#ifndef FRG_ILP
#define FRG_ILP 2
#endif

// Tables staged in LDS for one request: the logarithm table, then the dressing as n + 1 entries
// (Z_0, 0), (Z_0, Z_1 - Z_0), ..., (Z_{n-2}, Z_{n-1} - Z_{n-2}), (Z_{n-1}, 0) addressed by
// s + 1, s = (log|l| - log x_min)/Delta: the constant first and last entries absorb every s
// outside [0, n-1], so one integer clamp of the cell index replaces clamping s (the float32 form
// reads the same pairs and rounds them to float32 at use).
struct Smem {
    double2 *logt;
    double2 *Z64;
    float *f32c;  // float32 form: [0] K, [1] the fallback's weight (see fp32_constants)
};

// Cell index and fraction of the padded dressing table for coordinate sp = s + 1.
__device__ __forceinline__ void zcell64(double sp, int nZ, int &i, double &f) {
    // v_cvt_u32_f64 saturates (negative and NaN to 0), so only the upper clamp is left; the
    // padded end entries make the fraction irrelevant wherever a clamp applies
    unsigned u;
    asm("v_cvt_u32_f64 %0, %1" : "=v"(u) : "v"(sp));
    i = (int)min(u, (unsigned)nZ);
    f = __builtin_amdgcn_fract(sp);
}

// Dressing Z(l2) (l2 > 0): s + 1 = za*log(l2) + zb1.
__device__ __forceinline__ double dressing64(const Smem &sm, int nZ, double za, double zb1,
                                             double l2) {
    int i;
    double f;
    zcell64(fma(fm::log_tab(l2, sm.logt), za, zb1), nZ, i, f);
    const double2 z = sm.Z64[i];
    return fma(f, z.y, z.x);
}

// G(l2) = 1/(Z l2 + R(l2) + m2) with R = l2 e/(-E), e = exp(-y), E = expm1(-y), y = l2/k^2,
// written with one reciprocal: G = (-E)/((-E)(Z l2 + m2) + l2 e), and l2 e = l2 + l2 E.
// l2 e carries an absolute error of ~1e-16 l2 where e is tiny, which is below 1e-16 of the
// denominator.  l2 > 0.
__device__ __forceinline__ double prop64(double l2, double z, double m2, double inv_k2) {
    const double E = fm::expm1_neg(l2 * inv_k2);
    const double den = fma(-E, fma(z, l2, m2), fma(l2, E, l2));
    return -E * fm::rcp_nr(den);
}

// W propagators at once, G[w] = G(l2[w]) with the tabulated dressing, ordered by phase so that the
// LDS gathers of all W points are in flight while the regulator (which does not depend on the
// dressing) is evaluated, and the W dependency chains interleave.
// Far field: for y = l2/k^2 >= FRG_FAR_Y, fm::expm1_neg(y) is exactly -1 (2^n < 2^-55 in its
// reconstruction), so l2 e = l2 + l2 E = 0 and the propagator below is exactly 1/(Z l2 + m2) --
// the same bits without evaluating the exponential.  A wavefront takes that path only when all
// its active lanes are in the far field (a uniform branch).  Used where whole wavefronts often
// are: two-point tiles group a few neighbouring radial nodes of neighbouring momenta, and fused
// three-point launches take tiles of 8 points (one |p|, neighbouring angles) x 8 neighbouring
// radial nodes, whose lanes are all in the far field at about half the steps of the workload
// (a wavefront over all radial nodes of one point is, at a quarter of them, and pays more for
// the vote than it saves).
#define FRG_FAR_Y 38.0

// 1/i, i = 1..16: coefficients of the polynomial-exponential regulator's exponent
__constant__ double kRegInv[17] = {0.0,       1.0,        1.0 / 2.0,  1.0 / 3.0,  1.0 / 4.0,
                                   1.0 / 5.0, 1.0 / 6.0,  1.0 / 7.0,  1.0 / 8.0,  1.0 / 9.0,
                                   1.0 / 10.0, 1.0 / 11.0, 1.0 / 12.0, 1.0 / 13.0, 1.0 / 14.0,
                                   1.0 / 15.0, 1.0 / 16.0};

// S_N(y) = sum_{i=1}^{N} y^i / i (Horner), 1 <= N <= 16; the paper's N = 8 as a fixed chain
// (the order is uniform across the wavefront, so the branch is too).
__device__ __forceinline__ double poly_s(double y, int n) {
    if (n == 8) {
        double acc = fma(0.125, y, 1.0 / 7.0);
        acc = fma(acc, y, 1.0 / 6.0);
        acc = fma(acc, y, 0.2);
        acc = fma(acc, y, 0.25);
        acc = fma(acc, y, 1.0 / 3.0);
        acc = fma(acc, y, 0.5);
        acc = fma(acc, y, 1.0);
        return acc * y;
    }
    double acc = kc(kRegInv)[n];
    for (int i = n - 1; i >= 1; --i) acc = fma(acc, y, kc(kRegInv)[i]);
    return acc * y;
}

// S_N(y) in float32 (the float32 form): the same Horner chain with the coefficients 1/i rounded
// to float32; y >= 0, so every term is positive and the result carries at most (2N + 1) u.
__device__ __forceinline__ float poly_s_f(float y, int n) {
    if (n == 8) {
        float acc = fmaf(0.125f, y, 1.0f / 7.0f);
        acc = fmaf(acc, y, 1.0f / 6.0f);
        acc = fmaf(acc, y, 0.2f);
        acc = fmaf(acc, y, 0.25f);
        acc = fmaf(acc, y, 1.0f / 3.0f);
        acc = fmaf(acc, y, 0.5f);
        acc = fmaf(acc, y, 1.0f);
        return acc * y;
    }
    float acc = (float)kc(kRegInv)[n];
    for (int i = n - 1; i >= 1; --i) acc = fmaf(acc, y, (float)kc(kRegInv)[i]);
    return acc * y;
}

// Regulators (REG): 0 exponential, R = l2/(e^y - 1); 1 polynomial-exponential
// R = k^2 exp(-S_N(y)); 2 flat, R = (k^2 - l2) Theta(k^2 - l2); y = l2/k^2.  For REG 1 and 2
// the callers pass l2 and m2 in units of k^2 (inv_k2 = 1) and G is 1/(Z y + R/k^2 + m2/k^2);
// far_y is the y beyond which R/k^2 is exactly 0 in float64 (REG 1), reg_n the order N.
template <int W, bool FAR = false, int REG = 0>
__device__ __forceinline__ void propagators64(const double (&l2)[W], double (&G)[W],
                                              const Smem &sm, int nZ, double za, double zb1,
                                              double m2, double inv_k2, double far_y = FRG_FAR_Y,
                                              int reg_n = 8) {
    // flat regulator: no transcendental to skip
    constexpr bool kFar = FAR && REG != 2;
    const double fy = REG == 0 ? FRG_FAR_Y : far_y;
    bool far = kFar;
#pragma unroll
    for (int w = 0; w < W; ++w) far = far && (l2[w] * inv_k2 >= fy);
    if (kFar && __all(far)) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const double zv = dressing64(sm, nZ, za, zb1, l2[w]);
            G[w] = fm::rcp_nr(fma(zv, l2[w], m2));
        }
        return;
    }
    double2 t[W];
#pragma unroll
    for (int w = 0; w < W; ++w) t[w] = sm.logt[(__double2hiint(l2[w]) >> 12) & 0xff];
    // REG 0: E = expm1(-y); REG 1, 2: E = R/k^2
    double E[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        if (REG == 0)
            E[w] = fm::expm1_neg(l2[w] * inv_k2);
        else if (REG == 1)
            E[w] = fm::exp_neg(fmin(poly_s(l2[w], reg_n), 1000.0));
        else
            E[w] = fmax(1.0 - l2[w], 0.0);
    }
    int iz[W];
    double fz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const double f = __builtin_amdgcn_frexp_mant(l2[w]);
        const int k = __builtin_amdgcn_frexp_exp(l2[w]);
        const double r = fma(f, t[w].x, -1.0);
        double p = fma(r, -0.25, 0.3333333333333333);
        p = fma(r, p, -0.5);
        p = fma(r, p, 1.0);
        p = r * p;
        const double ln = fma((double)k, fm::LN2_HI, t[w].y + p);
        zcell64(fma(ln, za, zb1), nZ, iz[w], fz[w]);
    }
    double2 z[W];
#pragma unroll
    for (int w = 0; w < W; ++w) z[w] = sm.Z64[iz[w]];
    if (REG != 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const double zv = fma(fz[w], z[w].y, z[w].x);
            G[w] = fm::rcp_nr(fma(zv, l2[w], m2) + E[w]);
        }
        return;
    }
    double le[W];
#pragma unroll
    for (int w = 0; w < W; ++w) le[w] = fma(l2[w], E[w], l2[w]);
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const double zv = fma(fz[w], z[w].y, z[w].x);
        const double den = fma(-E[w], fma(zv, l2[w], m2), le[w]);
        G[w] = -E[w] * fm::rcp_nr(den);
    }
}

__device__ __forceinline__ double lane_m2(const ReqDev &r, int e) {
    if (r.m2_mode == 0) return r.m2s;
    double v = r.m2[e];
    if (r.m2_mode == 2) v = fmax(v, r.m2_floor);
    return v;
}

// Radial prologue for (external point, radial node a): W^_a G(q^2)^2 and the angle coefficients
// c0 = q^2 + p^2, c1 = 2 q p.
struct RadialTerm {
    double wg, c0, c1, g;  // g = G(q^2) itself (for the mass derivative)
};

// A contribution and (DER) its derivative in the point's m2.
struct Dual {
    double v, d;
};

__device__ __forceinline__ RadialTerm radial64(const ReqDev &r, const Smem &sm, int a, double p,
                                               double m2) {
    RadialTerm t;
    const double q = r.k * kc(r.rad.q)[a];
    const double q2 = q * q;
    const double zq = dressing64(sm, r.nZ, r.za, r.zb + 1.0, fmax(q2, FRG_L2_TINY));
    const double A = fma(zq, q2, r.k2 * kc(r.rad.R)[a]);
    const double G = fm::rcp_nr(A + m2);
    t.wg = kc(r.rad.W)[a] * (G * G);
    t.c0 = fma(p, p, q2);
    t.c1 = 2.0 * q * p;
    t.g = G;
    return t;
}

// Contribution of (e, a) to the two-point integral (without the global prefactor).  m2 enters
// the radial leg, m2x the inner leg: equal in vacuum; at finite temperature the inner leg's mass
// term carries the shifted frequency, m2x = m2 + (w_j + p0)^2 (the radial leg's w_j^2 is folded
// into the rule's R).
// d/dm2 of W G(q^2)^2 G(l^2) = W G(q^2)^2 (-2 G(q^2) G(l^2) - G(l^2)^2): the inner sums of G^
// and G^2 (units of k^2) give both.
__device__ __forceinline__ Dual two_point_pair(const RadialTerm &t, double inner, double inner2,
                                               double inv_k2) {
    Dual out;
    out.v = t.wg * (inner * inv_k2);
    out.d = t.wg * (-2.0 * t.g * (inner * inv_k2) - inner2 * (inv_k2 * inv_k2));
    return out;
}

template <int REG, bool DER>
__device__ __forceinline__ Dual contrib_two64(const ReqDev &r, const Smem &sm, int a, double p,
                                              double m2, double m2x, double inv_k2) {
    // inner loop in units of k^2: y = l2/k^2 with G(l2) = G^(y)/k^2, G^ = 1/(Z y + R/k^2 + m2/k^2)
    const RadialTerm t = radial64(r, sm, a, p, m2);
    const double c0 = t.c0 * inv_k2, c1 = t.c1 * inv_k2, m2h = m2x * inv_k2;
    const int nx = r.n_x, nZ = r.nZ;
    const double za = r.za, zb1 = r.zbk + 1.0;
    double inner = 0.0, inner2 = 0.0;
    int b = 0;
    for (; b + FRG_ILP <= nx; b += FRG_ILP) {
        double l2[FRG_ILP], G[FRG_ILP];
#pragma unroll
        for (int w = 0; w < FRG_ILP; ++w) l2[w] = fma(c1, kc(r.ang.x)[b + w], c0);
        propagators64<FRG_ILP, true, REG>(l2, G, sm, nZ, za, zb1, m2h, 1.0, r.far_y, r.reg_n);
#pragma unroll
        for (int w = 0; w < FRG_ILP; ++w) {
            inner = fma(kc(r.ang.xw)[b + w], G[w], inner);
            if (DER) inner2 = fma(kc(r.ang.xw)[b + w], G[w] * G[w], inner2);
        }
    }
    for (; b < nx; ++b) {
        double l2[1] = {fma(c1, kc(r.ang.x)[b], c0)}, G[1];
        propagators64<1, true, REG>(l2, G, sm, nZ, za, zb1, m2h, 1.0, r.far_y, r.reg_n);
        inner = fma(kc(r.ang.xw)[b], G[0], inner);
        if (DER) inner2 = fma(kc(r.ang.xw)[b], G[0] * G[0], inner2);
    }
    if (DER) return two_point_pair(t, inner, inner2, inv_k2);
    return Dual{t.wg * (inner * inv_k2), 0.0};
}

// Contribution of (e, a) to the three-point integral.  l1 does not depend on phi, so G(l1^2) is
// evaluated once per (a, b); l2^2 = (c0 - c1 x cos a) - c1 sqrt(1-x^2) sin a cos phi.
// One cos1 node b of the three-point contribution (units of k^2): t = xw_b G^(l1^2) and the phi
// sum inner = sum_c w_c G^(l2^2); m2h1 and m2h2 are the mass terms of the two legs (equal in
// vacuum; at finite temperature each carries its leg's shifted frequency squared).
template <int REG, bool DER>
__device__ __forceinline__ void xterm64(const ReqDev &r, const Smem &sm, int b, double c0,
                                        double c1, double ca, double sa, double m2h1,
                                        double m2h2, double &t, double &inner, double &g1b,
                                        double &inner2) {
    const int nphi = r.n_phi, nZ = r.nZ;
    const double za = r.za, zb1 = r.zbk + 1.0;
    const double xb = kc(r.ang.x)[b];
    double l1[1] = {fma(c1, xb, c0)}, g1[1];
    propagators64<1, true, REG>(l1, g1, sm, nZ, za, zb1, m2h1, 1.0, r.far_y, r.reg_n);
    const double A2 = fma(-c1, xb * ca, c0);
    const double B2 = -c1 * (kc(r.ang.xs)[b] * sa);
    double acc = 0.0, acc2 = 0.0;
    int c = 0;
    for (; c + FRG_ILP <= nphi; c += FRG_ILP) {
        double l2[FRG_ILP], G[FRG_ILP];
#pragma unroll
        for (int w = 0; w < FRG_ILP; ++w)
            l2[w] = fmax(fma(B2, kc(r.phi.c)[c + w], A2), FRG_L2_TINY);
        propagators64<FRG_ILP, true, REG>(l2, G, sm, nZ, za, zb1, m2h2, 1.0, r.far_y, r.reg_n);
#pragma unroll
        for (int w = 0; w < FRG_ILP; ++w) {
            acc = fma(kc(r.phi.w)[c + w], G[w], acc);
            if (DER) acc2 = fma(kc(r.phi.w)[c + w], G[w] * G[w], acc2);
        }
    }
    for (; c < nphi; ++c) {
        double l2[1] = {fmax(fma(B2, kc(r.phi.c)[c], A2), FRG_L2_TINY)}, G[1];
        propagators64<1, false, REG>(l2, G, sm, nZ, za, zb1, m2h2, 1.0, r.far_y, r.reg_n);
        acc = fma(kc(r.phi.w)[c], G[0], acc);
        if (DER) acc2 = fma(kc(r.phi.w)[c], G[0] * G[0], acc2);
    }
    t = kc(r.ang.xw)[b] * g1[0];
    inner = acc;
    g1b = g1[0];
    inner2 = acc2;
}

// --------------------------------------------------------------------------------------------
// Float32 precision form
// --------------------------------------------------------------------------------------------
// float32 integrand; the sum over the innermost angle is compensated (Kahan) in float32 over
// blocks of FRG_ILP nodes; the per-(e, a) contribution is widened to float64 before the radial
// weight, and every sum across radial nodes is float64.  A propagator whose float32 denominator
// is small against its parts (D < tau (|Z l2 + R| + |m2|), i.e. near the pole m2 -> -(Z l2 + R))
// is re-evaluated in float64.
struct Kahan32 {
    float s, c;
    __device__ __forceinline__ void add(float v) {
        float y = v - c;
        float t = s + y;
        c = (t - s) - y;
        s = t;
    }
};

// Per-point constants of the float32 form; like the float64 loops it works in units of k^2
// (y = l2/k^2, m2/k^2, G^ = k^2 G).
struct Par32 {
    int nZ;
    float m2f, am2f;  // m2/k^2 and its magnitude
    float tau;        // near-pole threshold
    float kfb;        // weight of a float64 fallback's amplification (see fp32_constants)
    int reg_n;        // order N of the polynomial-exponential regulator
    float fary;       // its far field: y beyond which R/k^2 < e^-24
    double za2, zb1;  // s + 1 = za2 log2(y) + zb1
    double m2;        // the float64 fallback's mass
};

// Dressing cell and fraction at a float32 y.  y = m 2^e exactly (frexp, m in [1/2, 1)), so
// log2 y = e + log2 m with the hardware v_log_f32 on the mantissa only, whose absolute error
// there is at most kErrLog2f; e + log2 m and s + 1 = za2 log2 y + zb1 are formed in float64.
// The coordinate's error is then za2 kErrLog2f (plus float64 rounding), against about
// 2^-24 (n_Z + |zb1|) had s + 1 been rounded to float32 at its magnitude.
__device__ __forceinline__ void zcell32(float y, const Par32 &P, int &i, float &f) {
    const float m = __builtin_amdgcn_frexp_mantf(y);
    const int e = __builtin_amdgcn_frexp_expf(y);
    double fd;
    zcell64(fma((double)__builtin_amdgcn_logf(m) + (double)e, P.za2, P.zb1), P.nZ, i, fd);
    f = (float)fd;
}

// Near-pole node of the float32 form: the propagator in float64 at the float32 y, with the
// float64 dressing entries at the float32 form's cell and fraction, and its amplification
// kappa = (|Z y + R| + |m2|)/D.  Its float64 arithmetic adds nothing measurable, but y was
// rounded to float32 and the coordinate carries za2 kErrLog2f plus the fraction's rounding, and
// kappa amplifies both like every other perturbation: kappa enters kmax scaled by their share
// kfb of the float32 nodes' per-kappa error K, so that kappa K of the bound covers them.
// REG 0: G = (-E)/((-E)(Z y + m2) + y e); REG 1, 2: G = 1/(Z y + m2 + R/k^2).
template <int REG = 0>
__device__ __forceinline__ float prop_fallback(const Par32 &P, float y, double2 zz, float fz,
                                               float &kmax) {
    const double l2 = (double)y;
    const double z = fma((double)fz, zz.y, zz.x);
    float kap, g;
    if (REG == 0) {
        const double E = fm::expm1_neg(l2);
        const double le = fma(l2, E, l2);
        const double rd = fm::rcp_nr(fma(-E, fma(z, l2, P.m2), le));
        kap = (float)(fabs(fma(-E, fma(z, l2, fabs(P.m2)), le) * rd) * (double)P.kfb);
        g = (float)(-E * rd);
    } else {
        const double R = REG == 1 ? fm::exp_neg(fmin(poly_s(l2, P.reg_n), 1000.0))
                                  : fmax(1.0 - l2, 0.0);
        const double rd = fm::rcp_nr(fma(z, l2, P.m2) + R);
        kap = (float)(fabs((fma(z, l2, fabs(P.m2)) + R) * rd) * (double)P.kfb);
        g = (float)rd;
    }
    kmax = __uint_as_float(max(__float_as_uint(kmax), __float_as_uint(kap)));
    return g;
}

// W float32 propagators; kmax tracks the largest amplification (|Z l2 + R| + |m2|)/D of the
// float32 evaluations.
// Far field of the float32 form: fm::expm1_neg_f(y) is exactly -1 for y >= 17, so E = -1,
// l2 e = 0 and both the denominator and its parts lose the exponential exactly (see FRG_FAR_Y).
#define FRG_FAR_Y32 18.0f

template <int W, bool FAR = false, int REG = 0>
__device__ __forceinline__ void propagators32(const float (&l2)[W], float (&G)[W], float &kmax,
                                              const Smem &sm, const Par32 &P) {
    if (REG != 0) {
        // polynomial-exponential (R/k^2 = e^-S_N(y)) and flat (R/k^2 = max(1 - y, 0))
        // regulators: D = Z y + m2 + R/k^2, G = 1/D.  Far field of the polynomial-exponential
        // one (a wave-uniform branch): where every lane has y >= fary, R/k^2 < e^-24 is
        // dropped (the bound's constant K carries it).
        int iz[W];
        float fz[W], E[W];
#pragma unroll
        for (int w = 0; w < W; ++w) zcell32(l2[w], P, iz[w], fz[w]);
        double2 z[W];
#pragma unroll
        for (int w = 0; w < W; ++w) z[w] = sm.Z64[iz[w]];
        bool far = FAR && REG == 1;
#pragma unroll
        for (int w = 0; w < W; ++w) far = far && (l2[w] >= P.fary);
        if (FAR && REG == 1 && __all(far)) {
#pragma unroll
            for (int w = 0; w < W; ++w) E[w] = 0.0f;
        } else {
#pragma unroll
            for (int w = 0; w < W; ++w)
                E[w] = REG == 1 ? fm::exp_neg_f(poly_s_f(l2[w], P.reg_n))
                                : fmaxf(1.0f - l2[w], 0.0f);
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const float zv = fmaf(fz[w], (float)z[w].y, (float)z[w].x);
            const float den = fmaf(zv, l2[w], P.m2f) + E[w];
            const float parts = fmaf(zv, l2[w], P.am2f) + E[w];
            if (den < P.tau * parts) {
                G[w] = prop_fallback<REG>(P, l2[w], z[w], fz[w], kmax);
            } else {
                const float rd = __builtin_amdgcn_rcpf(den);
                G[w] = rd;
                kmax = __uint_as_float(max(__float_as_uint(kmax), __float_as_uint(parts * rd)));
            }
        }
        return;
    }
    bool far = FAR;
#pragma unroll
    for (int w = 0; w < W; ++w) far = far && (l2[w] >= FRG_FAR_Y32);
    if (FAR && __all(far)) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
            int iz;
            float fz;
            zcell32(l2[w], P, iz, fz);
            const double2 zz = sm.Z64[iz];
            const float zv = fmaf(fz, (float)zz.y, (float)zz.x);
            const float den = fmaf(zv, l2[w], P.m2f);
            const float parts = fmaf(zv, l2[w], P.am2f);
            if (den < P.tau * parts) {
                G[w] = prop_fallback(P, l2[w], zz, fz, kmax);
            } else {
                const float rd = __builtin_amdgcn_rcpf(den);
                G[w] = rd;
                kmax = __uint_as_float(max(__float_as_uint(kmax), __float_as_uint(parts * rd)));
            }
        }
        return;
    }
    int iz[W];
    float fz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) zcell32(l2[w], P, iz[w], fz[w]);
    double2 z[W];  // float64 entries, rounded to float32 where the float32 node uses them
#pragma unroll
    for (int w = 0; w < W; ++w) z[w] = sm.Z64[iz[w]];
    float E[W];
#pragma unroll
    for (int w = 0; w < W; ++w) E[w] = fm::expm1_neg_f(l2[w]);
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const float zv = fmaf(fz[w], (float)z[w].y, (float)z[w].x);
        const float le = fmaf(l2[w], E[w], l2[w]);
        const float den = fmaf(-E[w], fmaf(zv, l2[w], P.m2f), le);
        const float parts = fmaf(-E[w], fmaf(zv, l2[w], P.am2f), le);
        if (den < P.tau * parts) {
            G[w] = prop_fallback(P, l2[w], z[w], fz[w], kmax);
        } else {
            const float rd = __builtin_amdgcn_rcpf(den);
            G[w] = -E[w] * rd;
            // both non-negative: the larger float is the larger bit pattern
            kmax = __uint_as_float(max(__float_as_uint(kmax), __float_as_uint(parts * rd)));
        }
    }
}

__device__ __forceinline__ Par32 par32(const ReqDev &r, const Smem &sm, double m2,
                                       double inv_k2) {
    Par32 P;
    P.nZ = r.nZ;
    P.m2 = m2 * inv_k2;
    P.m2f = (float)P.m2;
    P.am2f = fabsf(P.m2f);
    P.tau = (float)r.tau;
    P.kfb = sm.f32c[1];
    P.reg_n = r.reg_n;
    P.fary = r.far_y32;
    P.za2 = r.za * 0.69314718055994530942;
    P.zb1 = r.zbk + 1.0;
    return P;
}

template <int REG>
__device__ __forceinline__ double contrib_two32(const ReqDev &r, const Smem &sm, int a, double p,
                                                double m2, double m2x, double inv_k2,
                                                float &kmax) {
    const RadialTerm t = radial64(r, sm, a, p, m2);
    const Par32 P = par32(r, sm, m2x, inv_k2);
    const double c0 = t.c0 * inv_k2, c1 = t.c1 * inv_k2;  // y = l2/k^2 > 0 (see FRG_L2_TINY)
    Kahan32 acc{0.0f, 0.0f};
    const int nx = r.n_x;
    int b = 0;
    for (; b + FRG_ILP <= nx; b += FRG_ILP) {
        float l2[FRG_ILP], G[FRG_ILP];
#pragma unroll
        for (int w = 0; w < FRG_ILP; ++w)
            l2[w] = (float)fma(c1, kc(r.ang.x)[b + w], c0);
        propagators32<FRG_ILP, true, REG>(l2, G, kmax, sm, P);
        float blk = 0.0f;
#pragma unroll
        for (int w = 0; w < FRG_ILP; ++w) blk = fmaf(kc(r.ang.xwf)[b + w], G[w], blk);
        acc.add(blk);
    }
    for (; b < nx; ++b) {
        float l2[1] = {(float)fma(c1, kc(r.ang.x)[b], c0)}, G[1];
        propagators32<1, true, REG>(l2, G, kmax, sm, P);
        acc.add(kc(r.ang.xwf)[b] * G[0]);
    }
    return t.wg * (((double)acc.s - (double)acc.c) * inv_k2);
}

// Two-point contribution with the cos1 nodes shared by lx adjacent lanes (lx = 1: one lane takes
// them all).  In rounds of lx consecutive nodes each lane evaluates one propagator; the round's
// first lane pulls them across lanes and accumulates them in cos1 order exactly as the one-lane
// loops do (float64: one fused multiply-add per node; float32: the same FRG_ILP-node blocks and
// compensated additions), so the bits do not depend on lx.  Called by all lanes of a wavefront
// together when lx > 1; act marks the lanes with a point and radial node to evaluate.
template <int PREC, int REG, bool DER>
__device__ __forceinline__ Dual contrib_two(const ReqDev &r, const Smem &sm, int a, double p,
                                            double m2, double m2x, double inv_k2, float &kmax,
                                            bool act, int sx, int lx) {
    if (lx == 1) {
        if (!act) return Dual{0.0, 0.0};
        if (PREC == 0) return contrib_two64<REG, DER>(r, sm, a, p, m2, m2x, inv_k2);
        return Dual{contrib_two32<REG>(r, sm, a, p, m2, m2x, inv_k2, kmax), 0.0};
    }
    RadialTerm t{0.0, 0.0, 0.0, 0.0};
    double c0 = 0.0, c1 = 0.0;
    Par32 P;
    if (act) {
        t = radial64(r, sm, a, p, m2);
        c0 = t.c0 * inv_k2;
        c1 = t.c1 * inv_k2;
        if (PREC == 1) P = par32(r, sm, m2x, inv_k2);
    }
    const double m2h = m2x * inv_k2, za = r.za, zb1 = r.zbk + 1.0;
    const int nx = r.n_x, nZ = r.nZ;
    const int xbase = (int)threadIdx.x & ~(lx - 1);
    const int nblk = nx - nx % FRG_ILP;  // nodes the float32 loop covers in whole blocks
    double inner = 0.0, inner2 = 0.0;
    Kahan32 acc{0.0f, 0.0f};
    float blk = 0.0f;
    for (int j0 = 0; j0 < nx; j0 += lx) {
        const int b = j0 + sx;
        double g = 0.0;
        float gf = 0.0f;
        if (act && b < nx) {
            if (PREC == 0) {
                double l2[1] = {fma(c1, kc(r.ang.x)[b], c0)}, G[1];
                propagators64<1, true, REG>(l2, G, sm, nZ, za, zb1, m2h, 1.0, r.far_y, r.reg_n);
                g = G[0];
            } else {
                float l2[1] = {(float)fma(c1, kc(r.ang.x)[b], c0)}, G[1];
                propagators32<1, true, REG>(l2, G, kmax, sm, P);
                gf = G[0];
            }
        }
        const int nk = min(lx, nx - j0);
        for (int k = 0; k < nk; ++k) {
            const int bk = j0 + k;
            if (PREC == 0) {
                const double gk = __shfl(g, xbase + k);
                inner = fma(kc(r.ang.xw)[bk], gk, inner);
                if (DER) inner2 = fma(kc(r.ang.xw)[bk], gk * gk, inner2);
            } else {
                const float gk = __shfl(gf, xbase + k);
                if (bk < nblk) {
                    const int w = bk % FRG_ILP;
                    blk = fmaf(kc(r.ang.xwf)[bk], gk, w == 0 ? 0.0f : blk);
                    if (w == FRG_ILP - 1) acc.add(blk);
                } else {
                    acc.add(kc(r.ang.xwf)[bk] * gk);
                }
            }
        }
    }
    if (PREC == 0) {
        if (DER) return two_point_pair(t, inner, inner2, inv_k2);
        return Dual{t.wg * (inner * inv_k2), 0.0};
    }
    return Dual{t.wg * (((double)acc.s - (double)acc.c) * inv_k2), 0.0};
}

template <int REG>
// P1 carries the first leg's mass, P the second's (the same in vacuum).
__device__ __forceinline__ void xterm32(const ReqDev &r, const Smem &sm, const Par32 &P1,
                                        const Par32 &P, int b, double c0, double c1, double ca,
                                        double sa, float &kmax, double &t, double &inner) {
    const int nphi = r.n_phi;
    const double xb = kc(r.ang.x)[b];
    float l1[1] = {(float)fma(c1, xb, c0)}, g1[1];
    propagators32<1, false, REG>(l1, g1, kmax, sm, P1);
    const double A2 = fma(-c1, xb * ca, c0);
    const double B2 = -c1 * (kc(r.ang.xs)[b] * sa);
    Kahan32 acc{0.0f, 0.0f};
    int c = 0;
    for (; c + FRG_ILP <= nphi; c += FRG_ILP) {
        float l2[FRG_ILP], G[FRG_ILP];
#pragma unroll
        for (int w = 0; w < FRG_ILP; ++w)
            l2[w] = (float)fmax(fma(B2, kc(r.phi.c)[c + w], A2), 1e-30);
        propagators32<FRG_ILP, false, REG>(l2, G, kmax, sm, P);
        float blk = 0.0f;
#pragma unroll
        for (int w = 0; w < FRG_ILP; ++w) blk = fmaf(kc(r.phi.wf)[c + w], G[w], blk);
        acc.add(blk);
    }
    for (; c < nphi; ++c) {
        float l2[1] = {(float)fmax(fma(B2, kc(r.phi.c)[c], A2), 1e-30)}, G[1];
        propagators32<1, false, REG>(l2, G, kmax, sm, P);
        acc.add(kc(r.phi.wf)[c] * G[0]);
    }
    inner = (double)acc.s - (double)acc.c;
    t = (double)kc(r.ang.xw)[b] * (double)g1[0];
}

// Contribution of (e, a) to the three-point integral (without the global prefactor), the cos1
// nodes shared by lx adjacent lanes (lx = 1: one lane takes them all).  In rounds of lx
// consecutive nodes each lane evaluates one; the round's first lane pulls the (t, inner) pairs
// across lanes and folds them into mid in cos1 order, so mid is the same sequence of fused
// multiply-adds for every lx.  All lanes of a wavefront call this together when lx > 1 (the
// cross-lane pulls need them); act marks the lanes with a point and radial node to evaluate.
// DER: d/dm2 of G(q^2)^2 G1 G2 = -2 G(q^2)^3 G1 G2 - G(q^2)^2 (G1^2 G2 + G1 G2^2); per cos1 node
// the phi sums of G2 and G2^2 and G1 itself give midA = sum xw G1^2 sum G2 and
// midB = sum xw G1 sum G2^2 next to mid = sum xw G1 sum G2 (units of k^2).
// m2 enters the radial leg, m2x1 and m2x2 the legs l1 and l2 (all equal in vacuum; at finite
// temperature m2x_i = m2 + (w_j + p0i)^2, the radial leg's w_j^2 folded into the rule's R).
template <int PREC, int REG, bool DER>
__device__ __forceinline__ Dual contrib_three(const ReqDev &r, const Smem &sm, int a, double p,
                                              double ca, double sa, double m2, double m2x1,
                                              double m2x2, double inv_k2, float &kmax, bool act,
                                              int sx, int lx) {
    RadialTerm t{0.0, 0.0, 0.0, 0.0};
    double c0 = 0.0, c1 = 0.0;
    Par32 P, P1;
    if (act) {
        t = radial64(r, sm, a, p, m2);
        c0 = t.c0 * inv_k2;
        c1 = t.c1 * inv_k2;
        if (PREC == 1) {
            P1 = par32(r, sm, m2x1, inv_k2);
            P = par32(r, sm, m2x2, inv_k2);
        }
    }
    const double m2h1 = m2x1 * inv_k2, m2h2 = m2x2 * inv_k2;
    const int nx = r.n_x;
    const int xbase = (int)threadIdx.x & ~(lx - 1);
    double mid = 0.0, midA = 0.0, midB = 0.0;
    for (int j0 = 0; j0 < nx; j0 += lx) {
        const int b = j0 + sx;
        double tb = 0.0, ib = 0.0, gb = 0.0, i2b = 0.0;
        if (act && b < nx) {
            if (PREC == 0)
                xterm64<REG, DER>(r, sm, b, c0, c1, ca, sa, m2h1, m2h2, tb, ib, gb, i2b);
            else
                xterm32<REG>(r, sm, P1, P, b, c0, c1, ca, sa, kmax, tb, ib);
        }
        if (lx == 1) {
            mid = fma(tb, ib, mid);
            if (DER) {
                midA = fma(tb * gb, ib, midA);
                midB = fma(tb, i2b, midB);
            }
        } else {
            const int nk = min(lx, nx - j0);
            for (int k = 0; k < nk; ++k) {
                const double tk = __shfl(tb, xbase + k), ik = __shfl(ib, xbase + k);
                mid = fma(tk, ik, mid);
                if (DER) {
                    midA = fma(tk * __shfl(gb, xbase + k), ik, midA);
                    midB = fma(tk, __shfl(i2b, xbase + k), midB);
                }
            }
        }
    }
    const double i4 = inv_k2 * inv_k2;
    if (!DER) return Dual{t.wg * (mid * i4), 0.0};
    return Dual{t.wg * (mid * i4),
                t.wg * (-2.0 * t.g * (mid * i4) - (midA + midB) * (i4 * inv_k2))};
}

// --------------------------------------------------------------------------------------------
// Complex external frequencies (finite temperature, internal families 7 and 8)
// --------------------------------------------------------------------------------------------
// An inner leg whose external frequency is p0 + i p0i (the paper's external fermion legs at
// chemical potential carry p0f - i mu) has the mass term (w_j + p0 + i p0i)^2 + m2 =
// m2r + i mi with m2r = m2 + (w_j + p0)^2 - p0i^2 and mi = 2 (w_j + p0) p0i, and its
// propagator is the complex G = 1/(D + i mi) = (D - i mi)/(D^2 + mi^2), D = Z y + R/k^2 + m2r
// (units of k^2).  The exponential regulator's form D = den/(-E) (den as in propagators64)
// gives G = (-E)(den + i E mi)/(den^2 + E^2 mi^2); den and E are scaled by 2^-e(E) first (E =
// m_E 2^e(E), exact), so that neither square underflows as y -> 0, where both vanish like y.
// One reciprocal per node, as for a real propagator.
template <int W, bool FAR, int REG>
__device__ __forceinline__ void propagators64c(const double (&l2)[W], double (&Gr)[W],
                                               double (&Gi)[W], const Smem &sm, int nZ,
                                               double za, double zb1, double m2, double mi,
                                               double far_y, int reg_n) {
    constexpr bool kFar = FAR && REG != 2;
    const double fy = REG == 0 ? FRG_FAR_Y : far_y;
    bool far = kFar;
#pragma unroll
    for (int w = 0; w < W; ++w) far = far && (l2[w] >= fy);
    if (kFar && __all(far)) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const double D = fma(dressing64(sm, nZ, za, zb1, l2[w]), l2[w], m2);
            const double inv = fm::rcp_nr(fma(D, D, mi * mi));
            Gr[w] = D * inv;
            Gi[w] = -mi * inv;
        }
        return;
    }
    double2 t[W];
#pragma unroll
    for (int w = 0; w < W; ++w) t[w] = sm.logt[(__double2hiint(l2[w]) >> 12) & 0xff];
    double E[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        if (REG == 0)
            E[w] = fm::expm1_neg(l2[w]);
        else if (REG == 1)
            E[w] = fm::exp_neg(fmin(poly_s(l2[w], reg_n), 1000.0));
        else
            E[w] = fmax(1.0 - l2[w], 0.0);
    }
    int iz[W];
    double fz[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const double f = __builtin_amdgcn_frexp_mant(l2[w]);
        const int k = __builtin_amdgcn_frexp_exp(l2[w]);
        const double r = fma(f, t[w].x, -1.0);
        double p = fma(r, -0.25, 0.3333333333333333);
        p = fma(r, p, -0.5);
        p = fma(r, p, 1.0);
        p = r * p;
        const double ln = fma((double)k, fm::LN2_HI, t[w].y + p);
        zcell64(fma(ln, za, zb1), nZ, iz[w], fz[w]);
    }
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const double2 z = sm.Z64[iz[w]];
        const double zv = fma(fz[w], z.y, z.x);
        if (REG != 0) {
            const double D = fma(zv, l2[w], m2) + E[w];
            const double inv = fm::rcp_nr(fma(D, D, mi * mi));
            Gr[w] = D * inv;
            Gi[w] = -mi * inv;
        } else {
            const double den = fma(-E[w], fma(zv, l2[w], m2), fma(l2[w], E[w], l2[w]));
            const double mE = __builtin_amdgcn_frexp_mant(E[w]);  // E = mE 2^eE, mE < 0
            const int eE = __builtin_amdgcn_frexp_exp(E[w]);
            const double ds = __builtin_amdgcn_ldexp(den, -eE);
            const double em = mE * mi;
            const double inv = fm::rcp_nr(fma(ds, ds, em * em));
            Gr[w] = -mE * ds * inv;
            Gi[w] = -mE * em * inv;
        }
    }
}

// Two-point contribution of (e, a) with a complex inner-leg mass m2r + i mi (units of k^2
// after the scaling below): Dual{Re, Im}.  Lanes share cos1 nodes as in contrib_two.
template <int REG>
__device__ __forceinline__ Dual contrib_two_c(const ReqDev &r, const Smem &sm, int a, double p,
                                              double m2, double m2r, double mi, double inv_k2,
                                              bool act, int sx, int lx) {
    RadialTerm t{0.0, 0.0, 0.0, 0.0};
    double c0 = 0.0, c1 = 0.0;
    if (act) {
        t = radial64(r, sm, a, p, m2);
        c0 = t.c0 * inv_k2;
        c1 = t.c1 * inv_k2;
    }
    const double m2h = m2r * inv_k2, mih = mi * inv_k2, za = r.za, zb1 = r.zbk + 1.0;
    const int nx = r.n_x, nZ = r.nZ;
    double ir = 0.0, ii = 0.0;
    if (lx == 1) {
        if (!act) return Dual{0.0, 0.0};
        int b = 0;
        for (; b + FRG_ILP <= nx; b += FRG_ILP) {
            double l2[FRG_ILP], gr[FRG_ILP], gi[FRG_ILP];
#pragma unroll
            for (int w = 0; w < FRG_ILP; ++w) l2[w] = fma(c1, kc(r.ang.x)[b + w], c0);
            propagators64c<FRG_ILP, true, REG>(l2, gr, gi, sm, nZ, za, zb1, m2h, mih, r.far_y,
                                               r.reg_n);
#pragma unroll
            for (int w = 0; w < FRG_ILP; ++w) {
                ir = fma(kc(r.ang.xw)[b + w], gr[w], ir);
                ii = fma(kc(r.ang.xw)[b + w], gi[w], ii);
            }
        }
        for (; b < nx; ++b) {
            double l2[1] = {fma(c1, kc(r.ang.x)[b], c0)}, gr[1], gi[1];
            propagators64c<1, true, REG>(l2, gr, gi, sm, nZ, za, zb1, m2h, mih, r.far_y,
                                         r.reg_n);
            ir = fma(kc(r.ang.xw)[b], gr[0], ir);
            ii = fma(kc(r.ang.xw)[b], gi[0], ii);
        }
    } else {
        const int xbase = (int)threadIdx.x & ~(lx - 1);
        for (int j0 = 0; j0 < nx; j0 += lx) {
            const int b = j0 + sx;
            double gr = 0.0, gi = 0.0;
            if (act && b < nx) {
                double l2[1] = {fma(c1, kc(r.ang.x)[b], c0)}, Gr[1], Gi[1];
                propagators64c<1, true, REG>(l2, Gr, Gi, sm, nZ, za, zb1, m2h, mih, r.far_y,
                                             r.reg_n);
                gr = Gr[0];
                gi = Gi[0];
            }
            const int nk = min(lx, nx - j0);
            for (int k = 0; k < nk; ++k) {
                ir = fma(kc(r.ang.xw)[j0 + k], __shfl(gr, xbase + k), ir);
                ii = fma(kc(r.ang.xw)[j0 + k], __shfl(gi, xbase + k), ii);
            }
        }
    }
    return Dual{t.wg * (ir * inv_k2), t.wg * (ii * inv_k2)};
}

// One cos1 node b of the three-point contribution with complex leg masses (m1r + i m1i on l1,
// m2r + i m2i on l2; units of k^2): t = xw_b G(l1^2) and the phi sum inner = sum_c w_c G(l2^2),
// both complex.
template <int REG>
__device__ __forceinline__ void xterm64c(const ReqDev &r, const Smem &sm, int b, double c0,
                                         double c1, double ca, double sa, double m1r,
                                         double m1i, double m2r, double m2i, double &tr,
                                         double &ti, double &inr, double &ini) {
    const int nphi = r.n_phi, nZ = r.nZ;
    const double za = r.za, zb1 = r.zbk + 1.0;
    const double xb = kc(r.ang.x)[b];
    double l1[1] = {fma(c1, xb, c0)}, g1r[1], g1i[1];
    propagators64c<1, true, REG>(l1, g1r, g1i, sm, nZ, za, zb1, m1r, m1i, r.far_y, r.reg_n);
    const double A2 = fma(-c1, xb * ca, c0);
    const double B2 = -c1 * (kc(r.ang.xs)[b] * sa);
    double ar = 0.0, ai = 0.0;
    int c = 0;
    for (; c + FRG_ILP <= nphi; c += FRG_ILP) {
        double l2[FRG_ILP], gr[FRG_ILP], gi[FRG_ILP];
#pragma unroll
        for (int w = 0; w < FRG_ILP; ++w)
            l2[w] = fmax(fma(B2, kc(r.phi.c)[c + w], A2), FRG_L2_TINY);
        propagators64c<FRG_ILP, true, REG>(l2, gr, gi, sm, nZ, za, zb1, m2r, m2i, r.far_y,
                                           r.reg_n);
#pragma unroll
        for (int w = 0; w < FRG_ILP; ++w) {
            ar = fma(kc(r.phi.w)[c + w], gr[w], ar);
            ai = fma(kc(r.phi.w)[c + w], gi[w], ai);
        }
    }
    for (; c < nphi; ++c) {
        double l2[1] = {fmax(fma(B2, kc(r.phi.c)[c], A2), FRG_L2_TINY)}, gr[1], gi[1];
        propagators64c<1, false, REG>(l2, gr, gi, sm, nZ, za, zb1, m2r, m2i, r.far_y, r.reg_n);
        ar = fma(kc(r.phi.w)[c], gr[0], ar);
        ai = fma(kc(r.phi.w)[c], gi[0], ai);
    }
    tr = kc(r.ang.xw)[b] * g1r[0];
    ti = kc(r.ang.xw)[b] * g1i[0];
    inr = ar;
    ini = ai;
}

// Three-point contribution of (e, a) with complex leg masses: Dual{Re, Im} of
// W G(q^2)^2 sum_b t_b inner_b.
template <int REG>
__device__ __forceinline__ Dual contrib_three_c(const ReqDev &r, const Smem &sm, int a, double p,
                                                double ca, double sa, double m2, double m1r,
                                                double m1i, double m2r, double m2i,
                                                double inv_k2, bool act, int sx, int lx) {
    RadialTerm t{0.0, 0.0, 0.0, 0.0};
    double c0 = 0.0, c1 = 0.0;
    if (act) {
        t = radial64(r, sm, a, p, m2);
        c0 = t.c0 * inv_k2;
        c1 = t.c1 * inv_k2;
    }
    const double h1r = m1r * inv_k2, h1i = m1i * inv_k2, h2r = m2r * inv_k2, h2i = m2i * inv_k2;
    const int nx = r.n_x;
    const int xbase = (int)threadIdx.x & ~(lx - 1);
    double mr = 0.0, mi = 0.0;
    for (int j0 = 0; j0 < nx; j0 += lx) {
        const int b = j0 + sx;
        double tr = 0.0, ti = 0.0, ir = 0.0, ii = 0.0;
        if (act && b < nx) xterm64c<REG>(r, sm, b, c0, c1, ca, sa, h1r, h1i, h2r, h2i, tr, ti, ir, ii);
        if (lx == 1) {
            mr = fma(tr, ir, fma(-ti, ii, mr));
            mi = fma(tr, ii, fma(ti, ir, mi));
        } else {
            const int nk = min(lx, nx - j0);
            for (int k = 0; k < nk; ++k) {
                const double tkr = __shfl(tr, xbase + k), tki = __shfl(ti, xbase + k);
                const double ikr = __shfl(ir, xbase + k), iki = __shfl(ii, xbase + k);
                mr = fma(tkr, ikr, fma(-tki, iki, mr));
                mi = fma(tkr, iki, fma(tki, ikr, mi));
            }
        }
    }
    const double i4 = inv_k2 * inv_k2;
    return Dual{t.wg * (mr * i4), t.wg * (mi * i4)};
}

// float32 form's stated relative error bound per result.  u = 2^-24 (float32 unit roundoff);
// kappa = the largest amplification (|Z y + R| + |m2|)/D among the point's float32 propagators
// (the fallback's enter scaled, see prop_fallback); nG = float32 propagators per integrand term
// (two-point 1, three-point 2); eE, er = largest relative errors of fm::expm1_neg_f and of the
// v_rcp_f32 reciprocal (kErrExpm1f, kErrRcpf, exhaustively measured); K = fp32_constants().
//   err = (6 + 2 nG) u + nG (eE + er) + nG kappa K
// Per float32 propagator G~ = fl((-E~) rcp(D~)), D~ = fl((-E~) fl(Z~ y~ + m~) + fl(y~ + y~ E~)):
//  - not amplified: eE (numerator), er, the product's rounding and D~'s last rounding: 2u + eE + er;
//  - amplified by kappa (each an absolute error of D relative to its parts (-E)(Z y + |m2|) + y e):
//    the rounding of y (below), m2 (u), the inner and the le roundings (2u), E~ in (-E)(Z y + m2)
//    (eE), E~ in le = y (1 + E) (y |E| eE against parts >= y min(1, Z): eE / min(1, Zmin)), and
//    Z~: float32 entries and fraction and the fma (2u + 1.5 u L) plus the coordinate's error
//    (L za2 kErrLog2f);
//  - the rounding of y itself (|dy/y| <= u) moves G by kappa u |y dN/dy| / (|Z y + R| + |m2|) with
//    N = Z y + R + m2: y Z' / Z <= za L, and |y R'| = R (y/(1 - e^-y) - 1) <= 1.32 R for y <= 2
//    and <= 0.724 <= (0.362 / Zmin)(Z y + R) beyond: u_y = u (1 + za L + max(1.32, 0.37/Zmin)).
// Per term: the float32 weight (u), the FRG_ILP-node block sum (2u) and the compensated sum of
// blocks (2u) -- two-point 6u + 2u + eE + er = (6 + 2) u + ...; three-point: the phi sum's 5u and
// two propagators, 10u + 2 (eE + er).  Every integrand term is positive, so the bound of a term
// bounds the integral.  First order in u; kappa is the computed one.
__device__ __forceinline__ double fp32_bound(float kmax, float K, const ReqDev &r) {
    const double nG = (r.family == 3 || r.family == 6) ? 2.0 : 1.0;
    return (6.0 + 2.0 * nG) * kU32 + nG * (kErrExpm1f + kErrRcpf) + nG * (double)kmax * (double)K;
}

// K = per-kappa relative error of one float32 propagator and the share of it that a float64
// fallback keeps (see prop_fallback), from the table's largest step L = max|Z_{i+1} - Z_i| /
// min|Z_i| (per coordinate unit), Zmin = min|Z_i| and the request's coordinate scale za (per
// unit of ln y); both stored rounded up.  Per regulator (each item an absolute error of D
// relative to its parts, as in fp32_bound):
//  exponential: see fp32_bound.
//  polynomial-exponential, D = Z y + m2 + E, E = e^-S, S = S_N(y): in the far field (y >= fary,
//    S >= 24) E is dropped, e^-24 = 3.8e-11 against parts >= Zmin fary; else E carries
//    E (S eS + eX) with
//    eS = (2N + 1) u + 1.5 u the exponent's error (Horner of positive terms, the product with
//    log2(e)) and eX = kErrExp2f, and S E / parts <= cS = max(1, 0.59/Zmin): where S <= 1,
//    S E / parts <= S E / E = S <= 1; S > 1 needs y > 1 - 1/e for every N, and there
//    S E <= 1/e while parts >= Z y; the rounding of y moves E by u |y E'| = u E sum y^i
//    <= u N S E;
//  flat, E = max(1 - y, 0): E's rounding u, and the rounding of y moves E by u y <= u Z y/Zmin.
// Common to all: m2 rounded (u), the inner fma (u), the float32 dressing (2u + 1.5 u L), its
// coordinate (L za2 kErrLog2f) and the rounding of y through Z (u (1 + za L)).
__device__ __forceinline__ void fp32_constants(const ReqDev &r, float mx, float mn, float *c) {
    const double L = mn > 0.0f ? (double)mx / (double)mn : 1.0e300;
    const double zlo = fmin(1.0, (double)mn);
    const double us = L * (r.za * 0.69314718055994530942 * kErrLog2f + 1.0e-12);  // coordinate
    double uy, K;
    if (r.reg == 1) {
        const double cs = fmax(1.0, 0.59 / zlo), n = (double)r.reg_n;
        uy = kU32 * (1.0 + r.za * L + n * cs);
        K = uy + us + kU32 * (4.0 + 1.5 * L) + cs * (2.0 * n + 2.5) * kU32 + kErrExp2f +
            3.8e-11 / (zlo * (double)r.far_y32);  // the far field's dropped e^-S_N < e^-24
    } else if (r.reg == 2) {
        uy = kU32 * (1.0 + r.za * L + 1.0 / zlo);
        K = uy + us + kU32 * (5.0 + 1.5 * L);
    } else {
        uy = kU32 * (1.0 + r.za * L + fmax(1.32, 0.37 / zlo));
        K = uy + us + kU32 * (5.0 + 1.5 * L) + kErrExpm1f * (1.0 + 1.0 / zlo);
    }
    c[0] = K < 1.0e30 ? (float)(K * (1.0 + 1.0 / 1048576.0)) : 3.0e38f;
    // the fallback: the rounding of y, the coordinate and the fraction's rounding (u/2 of a step)
    c[1] = (float)((uy + us + 0.5 * kU32 * L) / K * (1.0 + 1.0 / 1048576.0));
}

// --------------------------------------------------------------------------------------------
// Tile bodies
// --------------------------------------------------------------------------------------------
// The logarithm table is the same for every request of a context: a persistent workgroup stages
// it once.  Loads are issued together before the LDS stores (no round trip per entry).
__device__ __forceinline__ void stage_log(Smem &sm, const double2 *logt) {
    static_assert(kLogTable == 4 * kWave, "log table staged in four wavefront passes");
    const int i = (int)threadIdx.x;
    const double2 v0 = logt[i], v1 = logt[i + kWave], v2 = logt[i + 2 * kWave],
                  v3 = logt[i + 3 * kWave];
    sm.logt[i] = v0;
    sm.logt[i + kWave] = v1;
    sm.logt[i + 2 * kWave] = v2;
    sm.logt[i + 3 * kWave] = v3;
}

// Padded dressing of one request: entry j (0..n) is (Z_{j-1}, Z_j - Z_{j-1}) with constant end
// entries; for the float32 form also the bound's constants from the table's largest step
// max|Z_{i+1} - Z_i| and smallest entry min|Z_i| (one wavefront per workgroup).
template <int PREC>  // the kernel's precision: 0, 1, or -1 (the request's, at run time)
__device__ __forceinline__ void stage_dressing(const ReqDev &r, Smem &sm) {
    constexpr int U = 2;  // entries per lane whose loads are in flight together
    const int n = r.nZ;
    const bool f32 = PREC == 1 || (PREC < 0 && r.precision == 1);
    float mx = 0.0f, mn = 3.0e38f;
    for (int j0 = (int)threadIdx.x; j0 <= n; j0 += U * kWave) {
        double lo[U], hi[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = min(j0 + u * kWave, n);
            lo[u] = r.Z[max(j - 1, 0)];
            hi[u] = r.Z[min(j, n - 1)];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = j0 + u * kWave;
            if (j > n) break;
            const double dz = (j == 0 || j == n) ? 0.0 : hi[u] - lo[u];
            sm.Z64[j] = make_double2(lo[u], dz);
            if (f32) {
                if (j >= 1) mn = fminf(mn, (float)fabs(lo[u]));
                if (j >= 1 && j < n) mx = fmaxf(mx, (float)fabs(dz));
            }
        }
    }
    if (f32) {
        for (int o = kWave / 2; o > 0; o >>= 1) {
            mx = fmaxf(mx, __shfl_xor(mx, o));
            mn = fminf(mn, __shfl_xor(mn, o));
        }
        if (threadIdx.x == 0) fp32_constants(r, mx, mn, sm.f32c);
    }
}

// Radial sum of one point's contributions in radial order, with 8 loads in flight per wait.
// The point's contributions added in radial order; kInFlight loads are issued before their
// additions (the finalize runs one thread per point, few wavefronts: load latency bound).
__device__ __forceinline__ double radial_sum(const double *blk, int n_q, long long stride, int e) {
    constexpr int kInFlight = 32;
    double s = 0.0;
    int a = 0;
    for (; a + kInFlight <= n_q; a += kInFlight) {
        double v[kInFlight];
#pragma unroll
        for (int j = 0; j < kInFlight; ++j) v[j] = blk[(long long)(a + j) * stride + e];
#pragma unroll
        for (int j = 0; j < kInFlight; ++j) s += v[j];
    }
    for (; a < n_q; ++a) s += blk[(long long)a * stride + e];
    return s;
}

__device__ __forceinline__ void bind_smem(Smem &sm, double2 *lds, int nZ, float *f32c) {
    sm.logt = lds;
    sm.Z64 = lds + kLogTable;
    sm.f32c = f32c;
}

// LPA: one lane per external point, the whole radial sum in one lane, no scratch.
// One LPA integral pref * sum_a W_a / (A_a + m2)^2 with A_a = k^2 (q^_a^2 + R^_a).  The float32
// form states (7 + 10 kappa) u + 2 er in err (u = 2^-24, er = kErrRcpf, kappa = the largest
// (A + |m2|)/(A + m2) of its float32 terms): A from float32 q^, R^ and k^2 carries 5u, so
// t = A + m2 carries 5 kappa u + u and g^2 = rcp(t)^2 twice that and 2 er; the weight, the
// two products and the compensated sum add 5u.  Near-pole terms (float64 from the float64
// nodes) carry only their rounding to float32.
// With r.dout (float64) also dI/dm2 = pref sum_a W_a (-2 G_a^3) into *dv.
template <int PREC>
__device__ __forceinline__ double lpa_integral(const ReqDev &r, double m2, double &err,
                                               double *dv = nullptr) {
    const int nq = r.n_q;
    if (PREC == 0) {
        // in units of k^2: G^ = 1/(A_a + m2/k^2) = k^2 G with A_a = q^2 + R per rule entry (one
        // add per node), the k^-4 of G^2 (k^-6 of G^3) applied once at the end
        const double ik2 = 1.0 / r.k2, m2h = m2 * ik2;
        double acc = 0.0;
        if (dv) {
            double dacc = 0.0;
            for (int a = 0; a < nq; ++a) {
                const double g = fm::rcp_nr(kc(r.rad.A)[a] + m2h);
                acc = fma(kc(r.rad.W)[a], g * g, acc);
                dacc = fma(kc(r.rad.W)[a], g * g * g, dacc);
            }
            *dv = r.pref * (-2.0 * (dacc * (ik2 * ik2 * ik2)));
        } else {
            // blocks of 8 radial nodes: the 8 reciprocals are independent and overlap, then
            // enter the sum in radial order (the same additions as one node at a time)
            constexpr int U = 8;
            int a = 0;
            for (; a + U <= nq; a += U) {
                double g2[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const double g = fm::rcp_nr(kc(r.rad.A)[a + u] + m2h);
                    g2[u] = g * g;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) acc = fma(kc(r.rad.W)[a + u], g2[u], acc);
            }
            for (; a < nq; ++a) {
                const double g = fm::rcp_nr(kc(r.rad.A)[a] + m2h);
                acc = fma(kc(r.rad.W)[a], g * g, acc);
            }
        }
        err = 0.0;
        return r.pref * (acc * (ik2 * ik2));
    }
    // float32 terms, compensated float32 sum; near-pole denominators in float64
    const float k2f = (float)r.k2, m2f = (float)m2, tau = (float)r.tau;
    Kahan32 acc{0.0f, 0.0f};
    float kmax = 1.0f;
    for (int a = 0; a < nq; ++a) {
        const float qh = kc(r.rad.qf)[a];
        const float A = k2f * fmaf(qh, qh, kc(r.rad.Rf)[a]);
        const float t = A + m2f;
        float g;
        if (t < tau * (A + fabsf(m2f))) {
            const double qd = kc(r.rad.q)[a];
            g = (float)fm::rcp_nr(fma(r.k2, fma(qd, qd, kc(r.rad.R)[a]), m2));
        } else {
            g = __builtin_amdgcn_rcpf(t);
            kmax = fmaxf(kmax, (A + fabsf(m2f)) * g);
        }
        acc.add(kc(r.rad.Wf)[a] * (g * g));
    }
    err = (7.0 + 10.0 * (double)kmax) * kU32 + 2.0 * kErrRcpf;
    return r.pref * ((double)acc.s - (double)acc.c);
}

template <int PREC>
__device__ __forceinline__ void tile_lpa(const ReqDev &r, int et) {
    const int e = et * kWave + (int)threadIdx.x;
    if (e >= r.n_ext) return;
    double err, dv = 0.0;
    const double v = lpa_integral<PREC>(r, lane_m2(r, e), err, r.dout ? &dv : nullptr);
    r.out[e] = v;
    if (r.dout) r.dout[e] = dv;
    if (r.err) r.err[e] = err;
}

// Value of v in lane l (l the same for every lane of the wavefront).
__device__ __forceinline__ double readlane64(double v, int l) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Vertex families (FAM 2 two-point, 3 three-point, 5 and 6 two- and three-point at finite
// temperature, 7 and 8 the same with complex external frequencies): lanes = (external point,
// radial sub-lane, cos1 sub-lane); the point's contributions are added in radial order inside
// the wavefront, or (radially chunked requests) stored for the finalize kernel.
template <int FAM, int PREC, int REG, bool DER>
__device__ __forceinline__ void tile_vertex(const ReqDev &r, const Smem &sm, int et, int chunk,
                                            double *__restrict__ contrib,
                                            unsigned *__restrict__ counters) {
    // lanes per point = lq (radial) x lx (cos1); lane = (point, sq, sx)
    const int lxl = r.lx_log2;
    const int lpl = r.lq_log2 + lxl;
    const int lq = 1 << r.lq_log2, lx = 1 << lxl;
    const int le = kWave >> lpl;
    const int lane = (int)threadIdx.x;
    const int el = lane >> lpl;
    const int sub = lane & ((1 << lpl) - 1);
    const int sq = sub >> lxl, sx = sub & (lx - 1);
    const int e = et * le + el;
    const bool valid = e < r.n_ext;
    const int a0 = (int)(((long long)r.n_q * chunk) / r.chunks);
    const int a1 = (int)(((long long)r.n_q * (chunk + 1)) / r.chunks);
    const double inv_k2 = 1.0 / r.k2;
    double *blk = contrib + r.contrib_base;
    // chunked tiles, float32 form: per-point slots of the largest amplification (zero at rest,
    // reset by the finalize kernel), then one slot for the dressing table's relative step
    unsigned *kslot = counters + r.ctr_base;
    float kmax = 1.0f;
    double p = 0.0, m2 = 0.0, ca = 1.0, sa = 0.0, p0 = 0.0, p02 = 0.0, p0i = 0.0, p02i = 0.0;
    if (valid) {
        p = r.ext[e];
        m2 = lane_m2(r, e);
        if (FAM == 3 || FAM == 6 || FAM == 8) sincos(r.ext[r.n_ext + e], &sa, &ca);
        if (FAM == 5 || FAM == 7) p0 = r.ext[r.n_ext + e];
        if (FAM == 7) p0i = r.ext[2 * r.n_ext + e];
        if (FAM == 6 || FAM == 8) {
            p0 = r.ext[2 * r.n_ext + e];
            p02 = r.ext[3 * r.n_ext + e];
        }
        if (FAM == 8) {
            p0i = r.ext[4 * r.n_ext + e];
            p02i = r.ext[5 * r.n_ext + e];
        }
    }
    // contribution of radial node a (valid in the point's sx == 0 lanes); every lane of the
    // wavefront calls it together, lanes without work pass act = false
    auto node = [&](int a, bool act) -> Dual {
        if (FAM == 3)
            return contrib_three<PREC, REG, DER>(r, sm, act ? a : 0, p, ca, sa, m2, m2, m2, inv_k2,
                                                 kmax, act, sx, lx);
        if (FAM == 6) {
            // radial index a = (spatial node, frequency j): the legs' frequencies w_j + p01 and
            // w_j + p02
            const int ai = act ? a : 0;
            const double w1 = kc(r.rad.w0)[ai] + p0, w2 = kc(r.rad.w0)[ai] + p02;
            return contrib_three<PREC, REG, DER>(r, sm, ai, p, ca, sa, m2, fma(w1, w1, m2),
                                                 fma(w2, w2, m2), inv_k2, kmax, act, sx, lx);
        }
        if (FAM == 7) {
            // complex leg frequency w_j + p0 + i p0i: Dual{Re, Im} (the imaginary part takes
            // the derivative's slot)
            const int ai = act ? a : 0;
            const double wl = kc(r.rad.w0)[ai] + p0;
            return contrib_two_c<REG>(r, sm, ai, p, m2, fma(wl, wl, fma(-p0i, p0i, m2)),
                                      2.0 * wl * p0i, inv_k2, act, sx, lx);
        }
        if (FAM == 8) {
            const int ai = act ? a : 0;
            const double w1 = kc(r.rad.w0)[ai] + p0, w2 = kc(r.rad.w0)[ai] + p02;
            return contrib_three_c<REG>(r, sm, ai, p, ca, sa, m2, fma(w1, w1, fma(-p0i, p0i, m2)),
                                        2.0 * w1 * p0i, fma(w2, w2, fma(-p02i, p02i, m2)),
                                        2.0 * w2 * p02i, inv_k2, act, sx, lx);
        }
        if (FAM == 5) {
            // radial index a = (frequency j, spatial node): the inner leg's frequency w_j + p0
            const int ai = act ? a : 0;
            const double wl = kc(r.rad.w0)[ai] + p0;
            return contrib_two<PREC, REG, DER>(r, sm, ai, p, m2, fma(wl, wl, m2), inv_k2, kmax,
                                               act, sx, lx);
        }
        return contrib_two<PREC, REG, DER>(r, sm, act ? a : 0, p, m2, m2, inv_k2, kmax, act, sx,
                                           lx);
    };
    if (r.chunks == 1) {
        // The wavefront holds every radial node of its points.  The lq radial sub-lanes of a
        // point take rounds of lq consecutive radial nodes; after each round the point's first
        // lane pulls the round's values across lanes and adds them in radial order -- the same
        // sequence of additions as the radial sum of chunked tiles (identical bits), with no
        // scratch stores, no barrier and no device-scope fence (an L2 writeback and invalidate
        // on a multi-XCD part).
        const int base = lane & ~((1 << lpl) - 1);
        double sum = 0.0, dsum = 0.0;
        for (int r0 = 0; r0 < r.n_q; r0 += lq) {
            const int a = r0 + sq;
            const Dual v = node(a, valid && a < r.n_q);
            const int nk = min(lq, r.n_q - r0);
            if (lpl == 6) {
                // one point per wavefront: the source lanes are the same for every lane, so the
                // values are broadcast with scalar reads instead of LDS permutes (same additions)
                for (int k = 0; k < nk; ++k) {
                    sum += readlane64(v.v, k * lx);
                    if (DER) dsum += readlane64(v.d, k * lx);
                }
            } else {
                for (int k = 0; k < nk; ++k) {
                    sum += __shfl(v.v, base + k * lx);
                    if (DER) dsum += __shfl(v.d, base + k * lx);
                }
            }
        }
        if (PREC == 1) {
            for (int o = 1; o < (1 << lpl); o <<= 1) kmax = fmaxf(kmax, __shfl_xor(kmax, o));
        }
        if (valid && sub == 0) {
            r.out[e] = r.pref * sum;
            if (DER && r.dout) r.dout[e] = r.pref * dsum;
            if (r.err) r.err[e] = (PREC == 1) ? fp32_bound(kmax, sm.f32c[0], r) : 0.0;
        }
        return;
    }
    // DER: the derivative contributions follow the values as a second [n_q][n_ext] block
    const long long dblk = (long long)r.n_q * r.n_ext;
    for (int r0 = a0; r0 < a1; r0 += lq) {
        const int a = r0 + sq;
        const bool act = valid && a < a1;
        const Dual v = node(a, act);
        if (act && sx == 0) {
            blk[(long long)a * r.n_ext + e] = v.v;
            if (DER && r.dout) blk[dblk + (long long)a * r.n_ext + e] = v.d;
        }
    }
    // the finalize kernel (a later launch on the same stream) adds the chunks in radial order
    if (PREC == 1) {
        if (valid) atomicMax(&kslot[e], __float_as_uint(kmax));
        if (lane == 0) kslot[r.n_ext] = __float_as_uint(sm.f32c[0]);  // same value from every tile
    }
}

// Radially chunked requests: one thread per external point adds the [n_q][n_ext] contributions
// in radial order (the same additions as the in-wavefront sum of single-chunk tiles) and states
// the float32 bound from the amplification slots, which it returns to zero.
__device__ __forceinline__ void finalize_point(const ReqDev &r, int e, const double *contrib,
                                               unsigned *counters) {
    const double s = radial_sum(contrib + r.contrib_base, r.n_q, r.n_ext, e);
    r.out[e] = r.pref * s;
    if (r.dout) {
        const double *d = contrib + r.contrib_base + (long long)r.n_q * r.n_ext;
        r.dout[e] = r.pref * radial_sum(d, r.n_q, r.n_ext, e);
    }
    if (r.precision == 1) {
        unsigned *kslot = counters + r.ctr_base;
        if (r.err)
            r.err[e] = fp32_bound(__uint_as_float(kslot[e]), __uint_as_float(kslot[r.n_ext]), r);
        kslot[e] = 0u;
    } else if (r.err) {
        r.err[e] = 0.0;
    }
}

__global__ void __launch_bounds__(64) finalize_kernel(ReqDev r, const double *contrib,
                                                     unsigned *counters) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= r.n_ext) return;
    finalize_point(r, e, contrib, counters);
}

// The radially chunked requests of a fused launch, after it: workgroup b sums the 64 points from
// 64 fin[b].et of request fin[b].req.
__global__ void __launch_bounds__(64) multi_finalize_kernel(const ReqDev *__restrict__ reqs,
                                                           const TileDev *__restrict__ fin,
                                                           const double *contrib,
                                                           unsigned *counters) {
    const TileDev f = fin[blockIdx.x];
    const ReqDev &r = reqs[f.req];
    const int e = f.et * kWave + (int)threadIdx.x;
    if (e >= r.n_ext) return;
    finalize_point(r, e, contrib, counters);
}

hipError_t launch_multi_finalize(const ReqDev *reqs_dev, const TileDev *fin_dev, int n_fin,
                                 const double *contrib, unsigned *counters, hipStream_t s) {
    if (n_fin <= 0) return hipSuccess;
    hipLaunchKernelGGL(multi_finalize_kernel, dim3(n_fin), dim3(kWave), 0, s, reqs_dev, fin_dev,
                       contrib, counters);
    return hipGetLastError();
}

// One request: tile = blockIdx.x -> (external tile, chunk).
template <int FAM, int PREC, int REG, bool DER>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(
    DER ? ((FAM == 3 || FAM == 6 || FAM == 8) ? FRG_WAVES_PER_EU_DER3 : FRG_WAVES_PER_EU_DER)
        : ((FAM == 3 || FAM == 6 || PREC != 0) ? FRG_WAVES_PER_EU_MULTI
                                                : FRG_WAVES_PER_EU_BATCH))))
batch_kernel(ReqDev r, double *contrib, unsigned *counters) {
    extern __shared__ double2 lds_dyn[];
    if (FAM == 1) {
        tile_lpa<PREC>(r, blockIdx.x);
        return;
    }
    __shared__ float f32c[2];
    Smem sm;
    bind_smem(sm, lds_dyn, r.nZ, f32c);
    const int et = blockIdx.x / r.chunks;
    const int chunk = blockIdx.x - et * r.chunks;
    stage_log(sm, r.logt);
    stage_dressing<PREC>(r, sm);
    __syncthreads();
    tile_vertex<FAM, PREC, REG, DER>(r, sm, et, chunk, contrib, counters);
}

typedef void (*batch_fn)(ReqDev, double *, unsigned *);

// Kernel instance for (family, precision, regulator, mass derivative); the float32 form exists
// without derivative only, and the LPA kernel reads its regulator from the radial rule and its
// derivative flag from the request.
template <int F, bool D>
static batch_fn batch_for_reg(int reg) {
    if (reg == 1) return batch_kernel<F, 0, 1, D>;
    if (reg == 2) return batch_kernel<F, 0, 2, D>;
    return batch_kernel<F, 0, 0, D>;
}

template <int F>
static batch_fn batch_for_family(int prec, int reg, bool der) {
    if (prec == 1)
        return reg == 1 ? batch_kernel<F, 1, 1, false>
                        : (reg == 2 ? batch_kernel<F, 1, 2, false> : batch_kernel<F, 1, 0, false>);
    return der ? batch_for_reg<F, true>(reg) : batch_for_reg<F, false>(reg);
}

static batch_fn batch_variant(int fam, int prec, int reg, bool der) {
    if (fam == 1) return prec == 0 ? batch_kernel<1, 0, 0, false> : batch_kernel<1, 1, 0, false>;
    if (fam == 2) return batch_for_family<2>(prec, reg, der);
    if (fam == 5) return batch_for_family<5>(prec, reg, der);
    if (fam == 6) return batch_for_family<6>(prec, reg, der);
    // complex frequencies: the imaginary part rides in the derivative's slot
    if (fam == 7) return batch_for_reg<7, true>(reg);
    if (fam == 8) return batch_for_reg<8, true>(reg);
    return batch_for_family<3>(prec, reg, der);
}

hipError_t launch_batch(const ReqDev *req_host, const ReqDev *req_dev_ptr, int n_tiles,
                        int lds_bytes, double *contrib, unsigned *counters, hipStream_t s) {
    (void)req_dev_ptr;
    const ReqDev &r = *req_host;
    if (n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_variant(r.family, r.precision, r.reg, r.dout != nullptr),
                       dim3(n_tiles), dim3(kWave), lds_bytes, s, r, contrib, counters);
    return hipGetLastError();
}

// Many requests in one launch.  A grid sized to the device takes the first tiles (ordered
// largest first by the host) by workgroup index and pulls the rest from a global counter until
// the list is empty.  A fill kernel ahead of every launch clears the counter (relaunches and
// graph replays need no memset), so no workgroup has to order its exit against the others with
// a device-scope fence.
// FAM = PREC = REG = -1 is the general kernel (any mix of families, precisions and
// regulators); a launch whose requests all share one family, precision and regulator uses the
// instance specialised for them, which carries only that path and so needs fewer registers
// (more resident waves).
template <int FAM, int PREC, int REG, bool DER>
__device__ __forceinline__ void vertex_tile(const ReqDev &r, Smem &sm, const TileDev &td,
                                            double *contrib, unsigned *counters) {
    tile_vertex<FAM, PREC, REG, DER>(r, sm, td.et, td.chunk, contrib, counters);
}

template <int F, bool D>
__device__ __forceinline__ void vertex_tile_reg(const ReqDev &r, Smem &sm, const TileDev &td,
                                                double *contrib, unsigned *counters) {
    if (r.reg == 1)
        vertex_tile<F, 0, 1, D>(r, sm, td, contrib, counters);
    else if (r.reg == 2)
        vertex_tile<F, 0, 2, D>(r, sm, td, contrib, counters);
    else
        vertex_tile<F, 0, 0, D>(r, sm, td, contrib, counters);
}

// The general kernel comes in two instances: without mass derivatives, and (D) for launches
// with at least one request that asks for them; there a request without dout runs the same
// derivative-carrying code (identical values) and skips the derivative stores.
template <int F, bool D>
__device__ __forceinline__ void vertex_tile_any(const ReqDev &r, Smem &sm, const TileDev &td,
                                                double *contrib, unsigned *counters) {
    if (r.precision == 1) {
        if (r.reg == 1)
            vertex_tile<F, 1, 1, false>(r, sm, td, contrib, counters);
        else if (r.reg == 2)
            vertex_tile<F, 1, 2, false>(r, sm, td, contrib, counters);
        else
            vertex_tile<F, 1, 0, false>(r, sm, td, contrib, counters);
    } else {
        vertex_tile_reg<F, D>(r, sm, td, contrib, counters);
    }
}

template <int FAM, int PREC, int REG, bool DER>
__device__ __forceinline__ void multi_tile(const ReqDev &r, Smem &sm, const TileDev &td,
                                           double *contrib, unsigned *counters) {
    if (FAM > 0) {
        vertex_tile<(FAM > 0 ? FAM : 2), (PREC > 0 ? PREC : 0), (REG > 0 ? REG : 0), DER>(
            r, sm, td, contrib, counters);
        return;
    }
    if (r.family == 2)
        vertex_tile_any<2, DER>(r, sm, td, contrib, counters);
    else if (r.family == 5)
        vertex_tile_any<5, DER>(r, sm, td, contrib, counters);
    else if (r.family == 6)
        vertex_tile_any<6, DER>(r, sm, td, contrib, counters);
    else if (r.family == 3)
        vertex_tile_any<3, DER>(r, sm, td, contrib, counters);
    else if constexpr (DER) {
        // complex frequencies (their requests carry dout, so only this instance sees them)
        if (r.family == 7)
            vertex_tile_reg<7, true>(r, sm, td, contrib, counters);
        else
            vertex_tile_reg<8, true>(r, sm, td, contrib, counters);
    }
}

// Occupancy target of a fused-kernel instance: the three-point families and the general kernel
// carry more state than the two-point families, the mass derivative a second set of
// accumulators, and the polynomial-exponential regulator's exponent a few more registers.  The
// float32 form of the two-point families holds 4 (at 5 it spills), that of the
// finite-temperature three-point family (two legs' float32 constants) 3.
constexpr int multi_waves(int fam, int prec, int reg, bool der) {
    return der ? ((fam < 0 || fam == 3 || fam == 6 || fam == 8) ? FRG_WAVES_PER_EU_DER3
                                                                : FRG_WAVES_PER_EU_DER)
               : ((fam < 0 || fam == 3 || fam == 6)
                      ? ((reg == 1 || (fam == 6 && prec != 0)) ? FRG_WAVES_PER_EU_DER3
                                                               : FRG_WAVES_PER_EU_MULTI)
                      : ((reg == 1 || prec != 0) ? FRG_WAVES_PER_EU_MULTI
                                                 : FRG_WAVES_PER_EU_BATCH));
}

template <int FAM, int PREC, int REG, bool DER>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(multi_waves(FAM, PREC, REG, DER))))
multi_kernel(const ReqDev *__restrict__ reqs, const TileDev *__restrict__ tiles, int n_tiles,
             double *contrib, unsigned *counters, unsigned *work) {
    extern __shared__ double2 lds_dyn[];
    __shared__ int tile_s;
    __shared__ float f32c[2];
    Smem sm;
    int staged = -1;
    bool log_staged = false;
    for (int round = 0;; ++round) {
        // The first round is static (tile = workgroup index): thousands of workgroups starting
        // together would otherwise queue on one atomic.  Later tiles come from the counter.
        int t;
        if (round == 0) {
            t = (int)blockIdx.x;
        } else {
            if ((int)gridDim.x >= n_tiles) break;
            if (threadIdx.x == 0) tile_s = (int)gridDim.x + (int)atomicAdd(&work[0], 1u);
            __syncthreads();
            t = tile_s;
            __syncthreads();
        }
        if (t >= n_tiles) break;
        const TileDev td = tiles[t];
        const ReqDev &r = reqs[td.req];
        if (FAM == 1 || (FAM < 0 && r.family == 1)) {
            if ((PREC >= 0 ? PREC : r.precision) == 0)
                tile_lpa<0>(r, td.et);
            else
                tile_lpa<1>(r, td.et);
            continue;
        }
        if (FAM != 1) {
            bind_smem(sm, lds_dyn, r.nZ, f32c);
            if (staged != td.req) {
                // every request of a launch shares the context's logarithm table
                if (!log_staged) stage_log(sm, r.logt);
                log_staged = true;
                stage_dressing<PREC>(r, sm);
                __syncthreads();
                staged = td.req;
            }
            multi_tile<FAM, PREC, REG, DER>(r, sm, td, contrib, counters);
            __syncthreads();
        }
    }
}

typedef void (*multi_fn)(const ReqDev *, const TileDev *, int, double *, unsigned *, unsigned *);

template <int F, bool D>
static multi_fn multi_for_reg(int reg) {
    if (reg == 1) return multi_kernel<F, 0, 1, D>;
    if (reg == 2) return multi_kernel<F, 0, 2, D>;
    return multi_kernel<F, 0, 0, D>;
}

template <int F>
static multi_fn multi_for_family(int prec, int reg, int der) {
    if (prec == 1)
        return reg == 1 ? multi_kernel<F, 1, 1, false>
                        : (reg == 2 ? multi_kernel<F, 1, 2, false> : multi_kernel<F, 1, 0, false>);
    return der ? multi_for_reg<F, true>(reg) : multi_for_reg<F, false>(reg);
}

// (fam, prec, reg) shared by every request of the launch, or -1 (mixed: the general kernel);
// der = 1 if any request asks for the mass derivative.
static multi_fn multi_variant(int fam, int prec, int reg, int der) {
    if (fam < 0 || prec < 0 || reg < 0)
        return der ? multi_kernel<-1, -1, -1, true> : multi_kernel<-1, -1, -1, false>;
    if (fam == 1) return prec == 0 ? multi_kernel<1, 0, 0, false> : multi_kernel<1, 1, 0, false>;
    if (fam == 2) return multi_for_family<2>(prec, reg, der);
    if (fam == 3) return multi_for_family<3>(prec, reg, der);
    if (fam == 5) return multi_for_family<5>(prec, reg, der);
    if (fam == 6) return multi_for_family<6>(prec, reg, der);
    if (fam == 7) return multi_for_reg<7, true>(reg);
    if (fam == 8) return multi_for_reg<8, true>(reg);
    return der ? multi_kernel<-1, -1, -1, true> : multi_kernel<-1, -1, -1, false>;
}

// Workgroups of the fused kernel resident per CU with `lds_bytes` of dynamic LDS (sizes the
// persistent grid).
int multi_blocks_per_cu(int fam, int prec, int reg, int der, int lds_bytes) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, multi_variant(fam, prec, reg, der), kWave,
                                                     lds_bytes) != hipSuccess ||
        n < 1)
        n = 4;
    return n;
}

// Persistent grid: at most the workgroups the CUs hold at once, and no more than the tile list
// needs in whole rounds -- with R = ceil(tiles / resident) rounds, ceil(tiles / R) workgroups
// share the tiles evenly instead of leaving a last round mostly idle.
int multi_grid(int n_tiles, int fam, int prec, int reg, int der, int lds_bytes, int num_cus) {
    const int resident =
        std::max(1, multi_blocks_per_cu(fam, prec, reg, der, lds_bytes) * num_cus);
    if (n_tiles <= resident) return std::max(n_tiles, 1);
    const int rounds = (n_tiles + resident - 1) / resident;
    return (n_tiles + rounds - 1) / rounds;
}

hipError_t launch_multi(const ReqDev *reqs_dev, int fam, int prec, int reg, int der,
                        const TileDev *tiles_dev, int n_tiles, int grid, int lds_bytes,
                        double *contrib, unsigned *counters, unsigned *work_ctr, hipStream_t s,
                        bool clear_work) {
    if (n_tiles <= 0) return hipSuccess;
    if (clear_work) {
        const hipError_t e = launch_fill_zero_u32(work_ctr, 2, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(multi_variant(fam, prec, reg, der), dim3(grid), dim3(kWave), lds_bytes, s,
                       reqs_dev, tiles_dev, n_tiles, contrib, counters, work_ctr);
    return hipGetLastError();
}

// --------------------------------------------------------------------------------------------
// Derivatives of the vertex integrals in the dressing-table entries
// --------------------------------------------------------------------------------------------
// The integral depends on entry Z_j only through the dressing's linear interpolation at each
// propagator argument v: dG(v)/dZ_j = -G(v)^2 v w_j(v), with w_j(v) the interpolation weight of
// entry j at v.  By the product rule over the legs,
//   two-point:   dI_e/dZ_j = pref sum_a W_a [ -2 G(q_a^2)^3 q_a^2 w_j(q_a^2) sum_b xw_b G(l2_ab)
//                                           - G(q_a^2)^2 sum_b xw_b G(l2_ab)^2 l2_ab w_j(l2_ab) ]
//   three-point: the radial leg (weight 2), the first inner leg G(l1_ab) and the second
//                G(l2_abc), each with the other propagators as factors.
// At finite temperature (FAM 5) a runs over the (spatial node, frequency) radial index; the
// dressing multiplies the spatial momentum of both legs and the inner leg's mass term carries
// the frequency, m2 + (w_a + p0)^2, as in the integral.
// The sums are organised in rows: a radial node (FAM 2, 5) with its cos1 nodes, or a (radial,
// cos1) pair (FAM 3) with its phi nodes.  Along a row the innermost propagator's argument grows
// (ascending x with p taken as |p|; ascending phi with sin(alpha) taken as |sin(alpha)|), so its
// cells are non-decreasing and the row falls into runs of equal cell.  One workgroup takes one
// point; each lane takes whole rows and adds each run's parts for the cell's lower and upper
// entry in float64, in row order.  Across lanes the parts are added exactly, as 64-bit integers
// in units of 2^-S of the point's sum: a first pass over the rows finds the largest part P
// (2^(E-1) <= P < 2^E) and sets S = 61 - E; the second pass rounds each part to the nearest unit
// (at most 2^-62 P) and adds it, split into its multiple of 2^32 units and the rest, to two
// integer accumulators per entry in LDS.  Integer addition is associative, so the result is the
// same bits for any assignment of rows to lanes and any order of the atomics; each entry errs by
// at most (its parts) x 2^-62 P, and where every term has one sign (G > 0 throughout) the row's
// largest entry is at least P, so the error relative to it stays below 2^-62 per part (about
// 1e-14 for the 10^5 parts of a three-point point).

// One float64 propagator (the arithmetic of propagators64<1, false, REG>, in units of k^2) with
// its padded cell and fraction.
template <int REG>
__device__ __forceinline__ double prop_cell64(double l2, const Smem &sm, int nZ, double za,
                                              double zb1, double m2, int reg_n, int &iz,
                                              double &fz) {
    const double2 t = sm.logt[(__double2hiint(l2) >> 12) & 0xff];
    double E;
    if (REG == 0)
        E = fm::expm1_neg(l2);
    else if (REG == 1)
        E = fm::exp_neg(fmin(poly_s(l2, reg_n), 1000.0));
    else
        E = fmax(1.0 - l2, 0.0);
    const double f = __builtin_amdgcn_frexp_mant(l2);
    const int k = __builtin_amdgcn_frexp_exp(l2);
    const double r = fma(f, t.x, -1.0);
    double p = fma(r, -0.25, 0.3333333333333333);
    p = fma(r, p, -0.5);
    p = fma(r, p, 1.0);
    p = r * p;
    const double ln = fma((double)k, fm::LN2_HI, t.y + p);
    zcell64(fma(ln, za, zb1), nZ, iz, fz);
    const double2 z = sm.Z64[iz];
    const double zv = fma(fz, z.y, z.x);
    if (REG != 0) return fm::rcp_nr(fma(zv, l2, m2) + E);
    const double den = fma(-E, fma(zv, l2, m2), fma(l2, E, l2));
    return -E * fm::rcp_nr(den);
}

// Padded cell index and fraction of the dressing coordinate s + 1 = za log(v) + zb1.
__device__ __forceinline__ void dz_cell(const Smem &sm, int nZ, double za, double zb1, double v,
                                        int &iz, double &f) {
    zcell64(fma(fm::log_tab(v, sm.logt), za, zb1), nZ, iz, f);
}

constexpr int kDzMaxWaves = 16;  // wavefronts per workgroup (one point)

// LDS of a workgroup: the logarithm and dressing tables, then the integer accumulators
size_t dz_lds_bytes(int nZ) {
    return (size_t)(kLogTable + nZ + 1) * sizeof(double2) +
           (size_t)nZ * 2 * sizeof(unsigned long long);
}

// Parts of one row, handed to part(entry, value): the runs of the innermost leg (lower and upper
// entry of each run's cell), then the row's single-cell terms -- the radial leg and (FAM 3, 6)
// the first inner leg.  Values in the units of the point's sum before the prefactor.  p0 and p02
// are the inner legs' external frequencies (FAM 5: p0; FAM 6: p01 and p02).
template <int FAM, int REG, typename Part>
__device__ __forceinline__ void dz_row(const ReqDev &r, const Smem &sm, long long row, double p,
                                       double ca, double sa, double p0, double p02, double m2,
                                       double inv_k2, Part &&part) {
    constexpr bool kThree = FAM == 3 || FAM == 6;
    const int nZ = r.nZ;
    const double zb1 = r.zbk + 1.0;
    const int a = kThree ? (int)(row / r.n_x) : (int)row;
    const RadialTerm t = radial64(r, sm, a, p, m2);
    const double q = r.k * kc(r.rad.q)[a];
    const double q2 = q * q;
    const double c0 = t.c0 * inv_k2, c1 = t.c1 * inv_k2;
    const double uf = kThree ? inv_k2 * inv_k2 : inv_k2;  // units of the inner sums
    double rw, A, B, mh, g1 = 0.0, l1 = 0.0, f1 = 0.0, xw = 0.0;
    int i1 = 0;
    if (kThree) {
        const int b = (int)(row - (long long)a * r.n_x);
        const double xb = kc(r.ang.x)[b];
        double mh1 = m2 * inv_k2;
        mh = mh1;
        if (FAM == 6) {
            // radial index a = (spatial node, frequency j): the legs carry w_j + p01, w_j + p02
            const double w1 = kc(r.rad.w0)[a] + p0, w2 = kc(r.rad.w0)[a] + p02;
            mh1 = fma(w1, w1, m2) * inv_k2;
            mh = fma(w2, w2, m2) * inv_k2;
        }
        l1 = fma(c1, xb, c0);
        g1 = prop_cell64<REG>(l1, sm, nZ, r.za, zb1, mh1, r.reg_n, i1, f1);
        xw = kc(r.ang.xw)[b];
        rw = t.wg * (xw * g1);
        A = fma(-c1, xb * ca, c0);
        B = -c1 * (kc(r.ang.xs)[b] * sa);
    } else {
        double m2x = m2;
        if (FAM == 5) {
            const double wl = kc(r.rad.w0)[a] + p0;
            m2x = fma(wl, wl, m2);
        }
        rw = t.wg;
        A = c0;
        B = c1;
        mh = m2x * inv_k2;
    }
    // cell iz (padded): entry iz - 1 takes (1 - f) v, entry iz takes f v; at the clamped ends
    // one entry takes all of v
    auto single = [&](int iz, double f, double v) {
        if (iz == 0) {
            part(0, v);
        } else if (iz == nZ) {
            part(nZ - 1, v);
        } else {
            part(iz - 1, (1.0 - f) * v);
            part(iz, f * v);
        }
    };
    const int n_in = kThree ? r.n_phi : r.n_x;
    double inner = 0.0, lo = 0.0, hi = 0.0;
    int cur = -1, prev = 0;
    for (int c = 0; c < n_in; ++c) {
        const double u = kThree ? kc(r.phi.c)[c] : kc(r.ang.x)[c];
        const double w = kThree ? kc(r.phi.w)[c] : kc(r.ang.xw)[c];
        double l2 = fma(B, u, A);
        if (kThree) l2 = fmax(l2, FRG_L2_TINY);
        int iz;
        double f;
        const double G = prop_cell64<REG>(l2, sm, nZ, r.za, zb1, mh, r.reg_n, iz, f);
        inner += w * G;
        const double v = -rw * (w * (G * G)) * (l2 * uf);
        // a node within rounding of a cell boundary that reads one cell below its predecessor
        // is taken at the boundary (the same weights up to that rounding)
        if (iz < prev) {
            iz = prev;
            f = 0.0;
        } else {
            prev = iz;
        }
        if (iz != cur) {
            if (cur > 0) part(cur - 1, lo);
            if (cur >= 0 && cur < nZ) part(cur, hi);
            cur = iz;
            lo = 0.0;
            hi = 0.0;
        }
        if (iz == 0)
            hi += v;
        else if (iz == nZ)
            lo += v;
        else {
            lo = fma(1.0 - f, v, lo);
            hi = fma(f, v, hi);
        }
    }
    if (cur > 0) part(cur - 1, lo);
    if (cur >= 0 && cur < nZ) part(cur, hi);
    // radial leg -2 W G(q^2)^3 q^2 [xw G^(l1)] I (FAM 3, 6 per (a, b), I = sum_c w_c G^(l2));
    // FAM 3, 6 first inner leg -W G(q^2)^2 xw G^(l1)^2 l1 I
    int iq;
    double fq;
    dz_cell(sm, nZ, r.za, r.zb + 1.0, fmax(q2, FRG_L2_TINY), iq, fq);
    single(iq, fq, -2.0 * t.g * q2 * rw * (inner * uf));
    if (kThree) single(i1, f1, -t.wg * (xw * (g1 * g1)) * l1 * (inner * uf));
}

// Workgroup b takes point e = e0 + b; its row is jac[(e - e0) * nZ ...].
template <int FAM, int REG>
__global__ void __launch_bounds__(64 * kDzMaxWaves) dz_kernel(ReqDev r, double *__restrict__ jac,
                                                             int e0) {
    extern __shared__ double2 lds_dyn[];
    __shared__ float f32c[2];
    __shared__ double wmax[kDzMaxWaves];
    Smem sm;
    const int nZ = r.nZ, e = e0 + (int)blockIdx.x;
    const int lane = (int)threadIdx.x & (kWave - 1), wv = (int)threadIdx.x / kWave;
    const int nw = (int)blockDim.x / kWave, nt = (int)blockDim.x;
    const long long n_rows = (FAM == 3 || FAM == 6) ? (long long)r.n_q * r.n_x : r.n_q;
    bind_smem(sm, lds_dyn, nZ, f32c);
    unsigned long long *acc_hi = (unsigned long long *)(lds_dyn + kLogTable + nZ + 1);
    unsigned long long *acc_lo = acc_hi + nZ;
    if (wv == 0) {
        stage_log(sm, r.logt);
        stage_dressing<0>(r, sm);
    }
    for (int j = (int)threadIdx.x; j < 2 * nZ; j += nt) acc_hi[j] = 0ull;
    __syncthreads();
    const double p = fabs(r.ext[e]);
    double ca = 1.0, sa = 0.0, p0 = 0.0, p02 = 0.0;
    if (FAM == 3 || FAM == 6) {
        sincos(r.ext[r.n_ext + e], &sa, &ca);
        sa = fabs(sa);
    }
    if (FAM == 5) p0 = r.ext[r.n_ext + e];
    if (FAM == 6) {
        p0 = r.ext[2 * r.n_ext + e];
        p02 = r.ext[3 * r.n_ext + e];
    }
    const double m2 = lane_m2(r, e);
    const double inv_k2 = 1.0 / r.k2;
    // pass 1: the largest part (a NaN part makes P NaN)
    double mx = 0.0;
    for (long long row = threadIdx.x; row < n_rows; row += nt)
        dz_row<FAM, REG>(r, sm, row, p, ca, sa, p0, p02, m2, inv_k2, [&](int, double v) {
            const double av = fabs(v);
            mx = (av > mx || av != av) ? av : mx;
        });
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const double y = __shfl_xor(mx, o);
        mx = (y > mx || y != y) ? y : mx;
    }
    if (lane == 0) wmax[wv] = mx;
    __syncthreads();
    double P = 0.0;
    for (int w = 0; w < nw; ++w) P = (wmax[w] > P || wmax[w] != wmax[w]) ? wmax[w] : P;
    const bool exact = P > 0.0 && P <= 1.0e300;  // finite and nonzero
    // units of 2^-S, S = 61 - E: |part| 2^S < 2^61, so its multiple of 2^32 units fits an int
    const int Eexp = exact ? __builtin_amdgcn_frexp_exp(P) : 0;
    const double scale = ldexp(1.0, 61 - Eexp);
    if (exact) {
        // pass 2: the parts, exactly
        for (long long row = threadIdx.x; row < n_rows; row += nt)
            dz_row<FAM, REG>(r, sm, row, p, ca, sa, p0, p02, m2, inv_k2, [&](int j, double v) {
                if (v == 0.0) return;
                const double x = v * scale;
                const double h = floor(x * 0x1p-32);
                const double l = rint(fma(-h, 0x1p32, x));  // in [0, 2^32]
                atomicAdd(&acc_hi[j], (unsigned long long)(long long)(int)h);
                atomicAdd(&acc_lo[j], (unsigned long long)l);
            });
    }
    __syncthreads();
    for (int j = (int)threadIdx.x; j < nZ; j += nt) {
        // no part at all: zero; a non-finite part: that value in every entry of the point
        const double v =
            exact ? ldexp(fma((double)(long long)acc_hi[j], 0x1p32, (double)acc_lo[j]), Eexp - 61)
                  : (P == 0.0 ? 0.0 : P);
        jac[(long long)(e - e0) * nZ + j] = r.pref * v;
    }
}

template <int FAM>
static void (*dz_for_reg(int reg))(ReqDev, double *, int) {
    return reg == 1 ? dz_kernel<FAM, 1> : (reg == 2 ? dz_kernel<FAM, 2> : dz_kernel<FAM, 0>);
}

hipError_t launch_dz(const ReqDev &r, double *jac, hipStream_t s) {
    return launch_dz_points(r, jac, 0, r.n_ext, s);
}

hipError_t launch_dz_points(const ReqDev &r, double *jac, int e0, int n_pts, hipStream_t s) {
    if (n_pts <= 0) return hipSuccess;
    if (e0 < 0 || e0 + n_pts > r.n_ext) return hipErrorInvalidValue;
    const bool three = r.family == 3 || r.family == 6;
    if ((r.family != 2 && r.family != 5 && !three) || r.precision != 0 || r.nZ < 2 ||
        r.n_x < 1 || (three && r.n_phi < 1))
        return hipErrorInvalidValue;
    void (*fn)(ReqDev, double *, int) = r.family == 3   ? dz_for_reg<3>(r.reg)
                                   : r.family == 6 ? dz_for_reg<6>(r.reg)
                                   : r.family == 5 ? dz_for_reg<5>(r.reg)
                                                   : dz_for_reg<2>(r.reg);
    // one workgroup per point, a row or more per lane; fewer wavefronts per workgroup when there
    // are points enough to fill the chip (the result does not depend on the choice)
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return hipGetLastError();
    const long long n_rows = three ? (long long)r.n_q * r.n_x : r.n_q;
    int waves = (int)std::min<long long>(kDzMaxWaves, (n_rows + kWave - 1) / kWave);
    while (waves > 4 && (long long)n_pts * waves > 16LL * cus) waves /= 2;
    waves = std::max(1, waves);
    hipLaunchKernelGGL(fn, dim3(n_pts), dim3(kWave * waves), dz_lds_bytes(r.nZ), s, r, jac, e0);
    return hipGetLastError();
}

// Logarithm table for fm::log_tab: (2 c_j, ln(1/c_j) - ln 2), c_j = 1/(1 + (j + 1/2)/256) rounded
// to double (2 c_j is exact), ln(1/c_j) - ln 2 to a few ulp of a number below 1 in magnitude.
__global__ void __launch_bounds__(256) log_table_kernel(double2 *out) {
    const int j = threadIdx.x;
    if (j >= kLogTable) return;
    const double c = 1.0 / (1.0 + (j + 0.5) / 256.0);
    out[j] = make_double2(2.0 * c, -log(c) - 0.69314718055994530942);
}

hipError_t launch_log_table(double2 *out, hipStream_t s) {
    hipLaunchKernelGGL(log_table_kernel, dim3(1), dim3(kLogTable), 0, s, out);
    return hipGetLastError();
}

// --------------------------------------------------------------------------------------------
// LPA flow state and assembly
// --------------------------------------------------------------------------------------------
// u', u'' at grid point i from the quadratic through three neighbouring points (Newton divided
// differences; the stencil is shifted inwards at the two ends).
// The whole LPA right-hand side in one launch, one thread per grid point: u' and u'' from the
// quadratic through three neighbouring grid points (one-sided at the ends), the sigma and pi
// masses floored at m2_floor, their two integrals (the same operations as the LPA tile) and the
// flux-form assembly du/dt = 1/2 [I(m_s^2) (3u' + 2 rho u'') + (N - 1) I(m_p^2) u'].
template <int PREC>
__global__ void __launch_bounds__(64) lpa_rhs_kernel(ReqDev r, int n, int n_comp,
                                                     const double *__restrict__ rho,
                                                     const double *__restrict__ u,
                                                     double m2_floor, double *dudt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = i == 0 ? 1 : (i == n - 1 ? n - 2 : i);
    const double x0 = rho[c - 1], x1 = rho[c], x2 = rho[c + 1];
    const double f0 = u[c - 1], f1 = u[c], f2 = u[c + 1];
    const double d01 = (f1 - f0) / (x1 - x0);
    const double d12 = (f2 - f1) / (x2 - x1);
    const double d012 = (d12 - d01) / (x2 - x0);
    const double xi = rho[i];
    const double up = d01 + d012 * ((xi - x0) + (xi - x1));
    const double upp = 2.0 * d012;
    const double ms = u[i] + 2.0 * xi * up;
    const double mp = u[i];
    const double fs = 3.0 * up + 2.0 * xi * upp;
    const double fp = up;
    double es, ep;
    const double Is = lpa_integral<PREC>(r, fmax(ms, m2_floor), es);
    const double Ip = lpa_integral<PREC>(r, fmax(mp, m2_floor), ep);
    dudt[i] = 0.5 * (Is * fs + (double)(n_comp - 1) * Ip * fp);
}

hipError_t launch_finalize(const ReqDev &r, const double *contrib, unsigned *counters,
                           hipStream_t s) {
    if (r.family == 1 || r.chunks <= 1 || r.n_ext == 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3((r.n_ext + 63) / 64), dim3(64), 0, s, r, contrib,
                       counters);
    return hipGetLastError();
}

hipError_t launch_lpa_rhs(const ReqDev &r, int n, int n_comp, const double *rho, const double *u,
                          double m2_floor, double *dudt, hipStream_t s) {
    if (r.precision == 0)
        hipLaunchKernelGGL(lpa_rhs_kernel<0>, dim3((n + 63) / 64), dim3(64), 0, s, r, n, n_comp,
                           rho, u, m2_floor, dudt);
    else
        hipLaunchKernelGGL(lpa_rhs_kernel<1>, dim3((n + 63) / 64), dim3(64), 0, s, r, n, n_comp,
                           rho, u, m2_floor, dudt);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) fill_zero_u32_kernel(unsigned *p, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

hipError_t launch_fill_zero_u32(unsigned *p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_zero_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       p, n);
    return hipGetLastError();
}

}  // namespace frg
