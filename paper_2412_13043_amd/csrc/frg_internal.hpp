// Internal structures shared by the host runtime and the HIP kernels.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace frg {

constexpr int kWave = 64;          // CDNA wavefront width; one workgroup = one wavefront
constexpr int kMaxRule = 1024;     // FRG_MAX_NODES
constexpr int kMaxTable = 4096;    // FRG_MAX_TABLE

// Quadrature rules computed on the device once and cached by the context.
//  radial (k = 1): q^_a, W^_a = w^_a q^_a^(d-1) Rdot^(q^_a^2), R^_a = R(q^_a^2) for the request's
//                  regulator
//  cos1:           x_b, xw_b = w_b sqrt(1 - x_b^2), xs_b = sqrt(1 - x_b^2)      (+ float copies)
//                  (d = 3 spatial measure: xw_b = w_b)
//  phi:            fc_c = cos(phi_c), fw_c = w_c sin(phi_c)                      (+ float copies)
// Finite temperature: one radial rule over the index i = a n_f + j of radial node a and frequency
// j (d = 3 spatial weights), with the frequency folded in: q^_i = q^_a, R^_i = R^_a + (w_j/k)^2,
// W^_i = W^_a c_j / k, and w0_i = w_j (null for vacuum rules).
struct RadialRule {
    const double *q, *W, *R;
    const float *qf, *Wf, *Rf;
    const double *w0;
    const double *A;  // q^2 + R per entry (the LPA denominator in units of k^2, less m2/k^2)
};
struct AngleRule {
    const double *x, *xw, *xs;
    const float *xf, *xwf, *xsf;
};
struct PhiRule {
    const double *c, *w;
    const float *cf, *wf;
};

// One request ("batch" of external points under one descriptor), as the kernels see it.
// Kernel families beyond the public ones: the finite-temperature two- and three-point families
// (5, 6) with complex external frequencies of the inner legs; their requests carry the
// imaginary part of each result where the others carry dI/dm2 (dout).
constexpr int kFamTwoPointComplex = 7;
constexpr int kFamThreePointComplex = 8;

struct ReqDev {
    int family, d, n_q, n_x, n_phi, precision;  // family: public family or kFam*Complex
    int n_ext;
    int lq_log2;      // lanes per external point over radial nodes: 1 << lq_log2 (vertex families)
    int lx_log2;      // ... times lanes over cos1 nodes: 1 << lx_log2 (vertex families; LPA 0)
    int chunks;       // radial chunks per external tile
    int ext_tiles;    // ceil(n_ext / (64 >> (lq_log2 + lx_log2)))
    int nZ;           // 0 => Z == 1
    int m2_mode;      // 0 scalar, 1 array, 2 array floored at m2_floor (flow states)
    int reg;          // regulator: 0 exponential, 1 polynomial-exponential, 2 flat
    int reg_n;        // order N of the polynomial-exponential regulator
    double far_y;     // y = l2/k^2 beyond which R is exactly 0 in float64 (regulator 1)
    float far_y32;    // y beyond which R/k^2 < e^-24 (regulator 1, float32 form)
    long long ctr_base;      // first counter of this request in the counter array
    long long contrib_base;  // first double of this request's [n_q][n_ext] contribution block
    double k, k2;
    double pref;      // final multiplier: Omega-factor * k^(d+2) (and flow coef, if any)
    double m2s;       // scalar m2
    double m2_floor;
    double za, zb;    // dressing coordinate s = za * log(l2) + zb
    double zbk;       // the same coordinate from y = l2/k^2: s = za * log(y) + zbk
    double tau;       // near-pole threshold (FP32 form)
    RadialRule rad;
    AngleRule ang;
    PhiRule phi;
    const double2 *logt;  // 256-entry table of the float64 logarithm (c_j, ln(1/c_j))
    const double *ext;    // family 2: p; family 3: p then alpha
    const double *m2;
    const double *Z;
    double *out;
    double *err;
    double *dout;         // dI/dm2 per point (complex families: Im I per point), or null
};

// A unit of work: external tile `et` of request `req`, radial chunk `chunk`.
struct TileDev {
    int req;
    int et;
    int chunk;
    int pad;
};

// Angular rules of three spatial dimensions (finite temperature), by the `plain` flags of
// launch_rules: the cos1 weight without sqrt(1 - x^2), the phi weight without sin(phi).
constexpr int kPlainCos1 = 1;
constexpr int kPlainPhi = 2;

// Kernel entry points (defined in frg_kernels.hip).
hipError_t launch_rules(int n_q, double q_max, int d, int n_x, int n_phi, double *q, double *W,
                        double *R, float *qf, float *Wf, float *Rf, double *x, double *xw,
                        double *xs, float *xf, float *xwf, float *xsf, double *fc, double *fw,
                        float *fcf, float *fwf, hipStream_t s, int plain = 0, int reg = 0,
                        int reg_n = 8);
// Finite-temperature radial rule (see RadialRule) from a d = 3 vacuum rule `base` of n_q nodes:
// n_f frequencies, the first and last n_tail of them the tail nodes +-Omega/t (t GL on [0, 1],
// weight Omega w_t/(2 pi t^2)), the rest 2 pi T (n + eta) for n = n_lo, n_lo + 1, ... (weight T).
// A[i] = fma(q[i], q[i], R[i]) for i < n (a radial rule's per-entry q^2 + R).
hipError_t launch_rule_sum(const double *q, const double *R, double *A, long long n,
                           hipStream_t s);
hipError_t launch_ft_rule(int n_q, int n_f, int n_tail, int n_lo, double eta, double T,
                          double Omega, double k, const RadialRule &base, double *q, double *W,
                          double *R, float *qf, float *Wf, float *Rf, double *w0, hipStream_t s);
hipError_t launch_batch(const ReqDev *req_dev_host, const ReqDev *req_dev_ptr, int n_tiles,
                        int lds_bytes, double *contrib, unsigned *counters, hipStream_t s);
// fam/prec: the family and precision shared by every request of the launch, or -1 (mixed).
// clear_work = false: the caller has already zeroed the two tile counters in work_ctr (for
// instance with the copy that uploads the tile list).
hipError_t launch_multi(const ReqDev *reqs_dev, int fam, int prec, int reg, int der,
                        const TileDev *tiles_dev, int n_tiles, int grid, int lds_bytes,
                        double *contrib, unsigned *counters, unsigned *work_ctr, hipStream_t s,
                        bool clear_work = true);
hipError_t launch_fill_zero_u32(unsigned *p, size_t n, hipStream_t s);
// Vertex families (2, 3, 5, 6), float64: jac[e * r.nZ + i] = dI_e/dZ_i for every point of r
// (one workgroup per point over every entry; r needs a dressing table).
hipError_t launch_dz(const ReqDev &r, double *jac, hipStream_t s);
// The same for points [e0, e0 + n_pts) only, their rows from jac on (row e - e0).
hipError_t launch_dz_points(const ReqDev &r, double *jac, int e0, int n_pts, hipStream_t s);
// radially chunked requests: radial sums after the integrand launch (no-op otherwise)
hipError_t launch_finalize(const ReqDev &r, const double *contrib, unsigned *counters,
                           hipStream_t s);
// After a fused launch: the radial sums of its chunked requests, one workgroup per (request,
// block of 64 points) entry of fin (req, et = block).
hipError_t launch_multi_finalize(const ReqDev *reqs_dev, const TileDev *fin_dev, int n_fin,
                                 const double *contrib, unsigned *counters, hipStream_t s);
hipError_t launch_lpa_rhs(const ReqDev &r, int n, int n_comp, const double *rho, const double *u,
                          double m2_floor, double *dudt, hipStream_t s);
hipError_t launch_log_table(double2 *out, hipStream_t s);
int multi_blocks_per_cu(int fam, int prec, int reg, int der, int lds_bytes);
int multi_grid(int n_tiles, int fam, int prec, int reg, int der, int lds_bytes, int num_cus);
constexpr int kLogTable = 256;

// Float32 form's error constants (relative unless stated): u = 2^-24; the largest absolute error
// of v_log_f32 (log2) on [1/2, 1), the largest relative errors of fm::expm1_neg_f on y >= 0, of
// v_rcp_f32 on normal arguments and of v_exp_f32 (2^x) on [-126, 0), each rounded up from an
// exhaustive measurement over every float32 input of its range (frg_math_probe on gfx950:
// 0.9973 u, 1.4798 u, 1.5348 u, 1.4234 u).
constexpr double kU32 = 5.9604644775390625e-8;
constexpr double kErrLog2f = 1.0 * kU32;
constexpr double kErrExpm1f = 1.5 * kU32;
constexpr double kErrRcpf = 1.6 * kU32;
constexpr double kErrExp2f = 1.5 * kU32;

}  // namespace frg
