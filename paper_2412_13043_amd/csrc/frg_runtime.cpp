// Host runtime of the loop-integral library: context, device-built quadrature-rule cache,
// argument validation, tile planning, per-stream scratch, and the C-ABI entry points for batched
// integration and flow right-hand sides.
#include "frg_runtime.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

namespace frg {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

frg_status freq_rule(const frg_integral_desc &d, FreqRule *out) {
    if (!finite_pos(d.T) || !finite_pos(d.freq_max) || !finite_pos(d.k)) {
        set_error("finite temperature needs T, freq_max and k finite and > 0");
        return FRG_E_INVAL;
    }
    if (d.statistics != FRG_BOSONIC && d.statistics != FRG_FERMIONIC) {
        set_error("statistics must be FRG_BOSONIC or FRG_FERMIONIC, got %d", d.statistics);
        return FRG_E_INVAL;
    }
    if (d.n_tail < 0 || d.n_tail > FRG_MAX_NODES) {
        set_error("n_tail must be in [0, %d], got %d", FRG_MAX_NODES, d.n_tail);
        return FRG_E_INVAL;
    }
    const double pi = 3.141592653589793238462643383279502884;
    FreqRule f;
    f.T = d.T;
    f.lambda = d.freq_scaled ? d.freq_max * d.k : d.freq_max;
    f.eta = d.statistics == FRG_FERMIONIC ? 0.5 : 0.0;
    // largest n >= 0 with 2 pi T (n + eta) <= Lambda
    const double nh = std::floor(f.lambda / (2.0 * pi * d.T) - f.eta);
    if (!(nh >= 0.0)) {
        set_error("no Matsubara frequency inside |w| <= %g at T = %g", f.lambda, d.T);
        return FRG_E_INVAL;
    }
    if (nh > (double)FRG_MAX_NODES) {
        set_error("more than %d Matsubara frequencies inside |w| <= %g at T = %g", FRG_MAX_NODES,
                  f.lambda, d.T);
        return FRG_E_INVAL;
    }
    const int n_hi = (int)nh;
    f.n_lo = d.statistics == FRG_FERMIONIC ? -n_hi - 1 : -n_hi;
    f.n_exp = n_hi - f.n_lo + 1;
    f.n_tail = d.n_tail;
    f.n_f = f.n_exp + 2 * d.n_tail;
    f.Omega = 2.0 * pi * d.T * ((double)n_hi + f.eta) + pi * d.T;
    if (f.n_f > FRG_MAX_NODES) {
        set_error("frequency rule has %d nodes (limit %d)", f.n_f, FRG_MAX_NODES);
        return FRG_E_INVAL;
    }
    *out = f;
    return FRG_OK;
}

int reg_order(const frg_integral_desc &d) {
    return d.regulator == FRG_REG_POLY_EXP ? (d.reg_order > 0 ? d.reg_order : 8) : 0;
}

// Smallest y (to a relative 1e-12) with S_N(y) = sum_{i=1}^{N} y^i/i >= s_far; with s_far = 760
// exp(-S_N) is exactly 0 in float64 beyond it (the smallest subnormal is exp(-744.4)), so the
// polynomial-exponential regulator vanishes exactly there.
double poly_exp_far_y(int n, double s_far) {
    auto S = [n](double y) {
        double acc = 1.0 / n;
        for (int i = n - 1; i >= 1; --i) acc = acc * y + 1.0 / i;
        return acc * y;
    };
    double lo = 0.0, hi = 1e4;
    for (int it = 0; it < 200 && hi - lo > 1e-12 * hi; ++it) {
        const double mid = 0.5 * (lo + hi);
        (S(mid) >= s_far ? hi : lo) = mid;
    }
    return hi;
}

frg_integral_desc plan_desc(const frg_integral_desc &d) {
    frg_integral_desc p = d;
    if (!is_ft(d.family)) return p;
    FreqRule f;
    if (freq_rule(d, &f) != FRG_OK) return p;
    p.family = d.family == FRG_FAMILY_LPA_T
                   ? FRG_FAMILY_LPA
                   : (d.family == FRG_FAMILY_THREE_POINT_T ? FRG_FAMILY_THREE_POINT
                                                           : FRG_FAMILY_TWO_POINT);
    p.n_q = d.n_q * f.n_f;
    return p;
}

double nodes_per_point(const frg_integral_desc &d) {
    const frg_integral_desc p = plan_desc(d);
    return (double)p.n_q * (is_vertex(p.family) ? p.n_x : 1) *
           (p.family == FRG_FAMILY_THREE_POINT ? p.n_phi : 1);
}

frg_status validate(const frg_integral_desc *d, const frg_batch *b, bool device_ptrs) {
    if (!d || !b) {
        set_error("null descriptor or batch");
        return FRG_E_INVAL;
    }
    if (d->family < 1 || d->family > 6) {
        set_error("family must be 1 (LPA), 2 (two-point), 3 (three-point), 4 (LPA at finite "
                  "temperature), 5 (two-point at finite temperature) or 6 (three-point at finite "
                  "temperature), got %d", d->family);
        return FRG_E_INVAL;
    }
    if (d->precision != FRG_FP64 && d->precision != FRG_FP32_KAHAN) {
        set_error("precision must be FRG_FP64 or FRG_FP32_KAHAN, got %d", d->precision);
        return FRG_E_INVAL;
    }
    if (d->regulator < FRG_REG_EXPONENTIAL || d->regulator > FRG_REG_FLAT) {
        set_error("regulator must be 0 (exponential), 1 (polynomial-exponential) or 2 (flat), "
                  "got %d", d->regulator);
        return FRG_E_INVAL;
    }
    if (d->reg_order < 0 || d->reg_order > 16) {
        set_error("reg_order must be in [0, 16] (0 = 8), got %d", d->reg_order);
        return FRG_E_INVAL;
    }
    if (d->family == FRG_FAMILY_LPA) {
        if (d->d < 1 || d->d > 8) {
            set_error("LPA family needs 1 <= d <= 8, got %d", d->d);
            return FRG_E_INVAL;
        }
    } else if (d->d != 4) {
        set_error("vertex families are implemented for d = 4 only, got d = %d", d->d);
        return FRG_E_UNSUPPORTED;
    }
    if (d->n_q < 1 || d->n_q > FRG_MAX_NODES) {
        set_error("n_q must be in [1, %d], got %d", FRG_MAX_NODES, d->n_q);
        return FRG_E_INVAL;
    }
    if (is_vertex(d->family) && (d->n_x < 1 || d->n_x > FRG_MAX_NODES)) {
        set_error("n_x must be in [1, %d], got %d", FRG_MAX_NODES, d->n_x);
        return FRG_E_INVAL;
    }
    if (has_phi(d->family) && (d->n_phi < 1 || d->n_phi > FRG_MAX_NODES)) {
        set_error("n_phi must be in [1, %d], got %d", FRG_MAX_NODES, d->n_phi);
        return FRG_E_INVAL;
    }
    if (!finite_pos(d->q_max) || !finite_pos(d->k)) {
        set_error("q_max and k must be finite and > 0");
        return FRG_E_INVAL;
    }
    if (!std::isfinite(d->near_pole_tau) || d->near_pole_tau < 0.0 || d->near_pole_tau >= 1.0) {
        set_error("near_pole_tau must be in [0, 1)");
        return FRG_E_INVAL;
    }
    if (is_ft(d->family)) {
        FreqRule f;
        const frg_status fs = freq_rule(*d, &f);
        if (fs != FRG_OK) return fs;
        if ((long long)d->n_q * f.n_f > FRG_MAX_FT_NODES) {
            set_error("n_q * n_frequencies = %lld exceeds %d", (long long)d->n_q * f.n_f,
                      FRG_MAX_FT_NODES);
            return FRG_E_INVAL;
        }
    }
    if (b->n_ext < 0 || b->n_ext > (1 << 24)) {
        set_error("n_ext must be in [0, 2^24], got %d", b->n_ext);
        return FRG_E_INVAL;
    }
    if (b->dout_dm2 && d->precision != FRG_FP64) {
        set_error("dout_dm2 (the mass derivative) is implemented in float64 only");
        return FRG_E_UNSUPPORTED;
    }
    if (d->complex_freq != 0 && d->complex_freq != 1) {
        set_error("complex_freq must be 0 or 1, got %d", d->complex_freq);
        return FRG_E_INVAL;
    }
    if (d->complex_freq) {
        if (d->family != FRG_FAMILY_TWO_POINT_T && d->family != FRG_FAMILY_THREE_POINT_T) {
            set_error("complex external frequencies apply to families 5 and 6 only");
            return FRG_E_INVAL;
        }
        if (d->precision != FRG_FP64 || b->dout_dm2 || b->dout_dz) {
            set_error("complex external frequencies are implemented in float64 without "
                      "dout_dm2 and dout_dz");
            return FRG_E_UNSUPPORTED;
        }
    }
    if (b->dout_dz) {
        if (!is_vertex(d->family) || d->precision != FRG_FP64) {
            set_error("dout_dz (derivatives in the dressing-table entries) is implemented for "
                      "the vertex families (2, 3, 5, 6) in float64 only");
            return FRG_E_UNSUPPORTED;
        }
        if (!b->Z.values) {
            set_error("dout_dz needs a dressing table (Z.values is NULL)");
            return FRG_E_INVAL;
        }
    }
    if (b->n_ext == 0) return FRG_OK;
    if (!b->out) {
        set_error("out is NULL");
        return FRG_E_INVAL;
    }
    if (is_vertex(d->family) && !b->ext) {
        set_error("ext is NULL for a vertex family");
        return FRG_E_INVAL;
    }
    if (!b->m2 && !std::isfinite(b->m2_scalar)) {
        set_error("m2_scalar is not finite");
        return FRG_E_INVAL;
    }
    if (is_vertex(d->family) && b->Z.values) {
        if (b->Z.n < 2 || b->Z.n > FRG_MAX_TABLE) {
            set_error("dressing table size must be in [2, %d], got %d", FRG_MAX_TABLE, b->Z.n);
            return FRG_E_INVAL;
        }
        if (!finite_pos(b->Z.x_min) || !finite_pos(b->Z.x_max) || !(b->Z.x_max > b->Z.x_min)) {
            set_error("dressing grid needs 0 < x_min < x_max");
            return FRG_E_INVAL;
        }
    }
    if ((double)plan_desc(*d).n_q * (double)b->n_ext > 2.0e9) {
        set_error("n_q * n_ext too large for one batch");
        return FRG_E_INVAL;
    }
    if (device_ptrs) {
        // every pointer the kernels dereference must be device-accessible memory
        const void *ptrs[6] = {b->ext, b->m2, b->out, b->err_out, b->dout_dm2, b->dout_dz};
        for (const void *p : ptrs) {
            if (!p) continue;
            hipPointerAttribute_t attr;
            if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
                (void)hipGetLastError();
                set_error("pointer %p is not HIP device memory", p);
                return FRG_E_INVAL;
            }
            if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) {
                set_error("pointer %p is not HIP device memory", p);
                return FRG_E_INVAL;
            }
        }
        if (is_vertex(d->family) && b->Z.values) {
            hipPointerAttribute_t attr;
            if (hipPointerGetAttributes(&attr, b->Z.values) != hipSuccess ||
                (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)) {
                (void)hipGetLastError();
                set_error("dressing table is not HIP device memory");
                return FRG_E_INVAL;
            }
        }
    }
    return FRG_OK;
}

// ---------------------------------------------------------------------------------------------
// Rule cache
// ---------------------------------------------------------------------------------------------
// Radial rule layout: q, W, R (float64), qf, Wf, Rf (float32; finite temperature: w0 before
// them), then A = q^2 + R (float64, 8-byte aligned after the floats).
static size_t radial_rule_bytes(int n);
static double *after_floats(float *end) {
    return (double *)(((uintptr_t)end + 7) & ~(uintptr_t)7);
}

static frg_status get_radial(frg_context *ctx, int n, double q_max, int d, int reg, int reg_n,
                             RadialRule *out) {
    auto key = std::make_tuple(n, q_max, d, reg, reg_n);
    auto it = ctx->radial.find(key);
    if (it == ctx->radial.end()) {
        auto e = std::make_unique<RadialEntry>();
        FRG_HIP_CHECK(e->buf.alloc(radial_rule_bytes(n)));
        double *q = (double *)e->buf.ptr, *W = q + n, *R = W + n;
        float *qf = (float *)(R + n), *Wf = qf + n, *Rf = Wf + n;
        double *A = after_floats(Rf + n);
        FRG_HIP_CHECK(launch_rules(n, q_max, d, 0, 0, q, W, R, qf, Wf, Rf, nullptr, nullptr,
                                   nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                   nullptr, ctx->aux, false, reg, reg_n));
        FRG_HIP_CHECK(launch_rule_sum(q, R, A, n, ctx->aux));
        FRG_HIP_CHECK(hipStreamSynchronize(ctx->aux));
        e->rule = RadialRule{q, W, R, qf, Wf, Rf, nullptr, A};
        it = ctx->radial.emplace(key, std::move(e)).first;
    }
    *out = it->second->rule;
    return FRG_OK;
}

static frg_status get_cos1(frg_context *ctx, int n, AngleRule *out, bool plain = false) {
    const int key = n + (plain ? (1 << 20) : 0);
    auto it = ctx->cos1.find(key);
    if (it == ctx->cos1.end()) {
        auto e = std::make_unique<AngleEntry>();
        FRG_HIP_CHECK(e->buf.alloc((size_t)n * (3 * sizeof(double) + 3 * sizeof(float)) + 64));
        double *x = (double *)e->buf.ptr, *xw = x + n, *xs = xw + n;
        float *xf = (float *)(xs + n), *xwf = xf + n, *xsf = xwf + n;
        FRG_HIP_CHECK(launch_rules(0, 1.0, 1, n, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                                   nullptr, x, xw, xs, xf, xwf, xsf, nullptr, nullptr, nullptr,
                                   nullptr, ctx->aux, plain ? kPlainCos1 : 0));
        FRG_HIP_CHECK(hipStreamSynchronize(ctx->aux));
        e->rule = AngleRule{x, xw, xs, xf, xwf, xsf};
        it = ctx->cos1.emplace(key, std::move(e)).first;
    }
    *out = it->second->rule;
    return FRG_OK;
}

size_t ft_rule_bytes(int n_q, int n_f) {
    return (size_t)n_q * (size_t)n_f * (5 * sizeof(double) + 3 * sizeof(float)) + 64;
}

frg_status ft_rule_into(frg_context *ctx, const frg_integral_desc &d, void *buf, size_t bytes,
                        RadialRule *out, hipStream_t s, const RadialRule *base_rule) {
    FreqRule f;
    frg_status st = freq_rule(d, &f);
    if (st != FRG_OK) return st;
    if (ft_rule_bytes(d.n_q, f.n_f) > bytes) {
        set_error("finite-temperature rule buffer too small");
        return FRG_E_INVAL;
    }
    RadialRule base;
    if (base_rule)
        base = *base_rule;
    else if ((st = get_radial(ctx, d.n_q, d.q_max, 3, d.regulator, reg_order(d), &base)) !=
             FRG_OK)
        return st;
    const size_t n = (size_t)d.n_q * (size_t)f.n_f;
    double *q = (double *)buf, *W = q + n, *R = W + n, *w0 = R + n;
    float *qf = (float *)(w0 + n), *Wf = qf + n, *Rf = Wf + n;
    double *A = after_floats(Rf + n);
    FRG_HIP_CHECK(launch_ft_rule(d.n_q, f.n_f, f.n_tail, f.n_lo, f.eta, f.T, f.Omega, d.k, base, q,
                                 W, R, qf, Wf, Rf, w0, s));
    FRG_HIP_CHECK(launch_rule_sum(q, R, A, (long long)n, s));
    *out = RadialRule{q, W, R, qf, Wf, Rf, w0, A};
    return FRG_OK;
}

// Finite-temperature radial rule: the frequency rule folded into a d = 3 radial rule, cached.
static frg_status get_ft_radial(frg_context *ctx, const frg_integral_desc &d, const FreqRule &f,
                                RadialRule *out) {
    auto key = std::make_tuple(d.n_q, d.q_max, d.k, d.T, f.lambda, d.statistics, d.n_tail,
                               d.regulator * 32 + reg_order(d));
    auto it = ctx->ft_radial.find(key);
    if (it == ctx->ft_radial.end()) {
        auto e = std::make_unique<RadialEntry>();
        const size_t bytes = ft_rule_bytes(d.n_q, f.n_f);
        FRG_HIP_CHECK(e->buf.alloc(bytes));
        frg_status st = ft_rule_into(ctx, d, e->buf.ptr, bytes, &e->rule, ctx->aux);
        if (st != FRG_OK) return st;
        FRG_HIP_CHECK(hipStreamSynchronize(ctx->aux));
        it = ctx->ft_radial.emplace(key, std::move(e)).first;
    }
    *out = it->second->rule;
    return FRG_OK;
}

static frg_status get_phi(frg_context *ctx, int n, PhiRule *out, bool plain = false) {
    const int key = n + (plain ? (1 << 20) : 0);
    auto it = ctx->phi.find(key);
    if (it == ctx->phi.end()) {
        auto e = std::make_unique<PhiEntry>();
        FRG_HIP_CHECK(e->buf.alloc((size_t)n * (2 * sizeof(double) + 2 * sizeof(float)) + 64));
        double *c = (double *)e->buf.ptr, *w = c + n;
        float *cf = (float *)(w + n), *wf = cf + n;
        FRG_HIP_CHECK(launch_rules(0, 1.0, 1, 0, n, nullptr, nullptr, nullptr, nullptr, nullptr,
                                   nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, c,
                                   w, cf, wf, ctx->aux, plain ? kPlainPhi : 0));
        FRG_HIP_CHECK(hipStreamSynchronize(ctx->aux));
        e->rule = PhiRule{c, w, cf, wf};
        it = ctx->phi.emplace(key, std::move(e)).first;
    }
    *out = it->second->rule;
    return FRG_OK;
}

static size_t radial_rule_bytes(int n) {
    return (size_t)n * (4 * sizeof(double) + 3 * sizeof(float)) + 64;
}
static size_t cos1_rule_bytes(int n) {
    return (size_t)n * (3 * sizeof(double) + 3 * sizeof(float)) + 64;
}
static size_t phi_rule_bytes(int n) {
    return (size_t)n * (2 * sizeof(double) + 2 * sizeof(float)) + 64;
}
static size_t up256(size_t v) { return (v + 255) & ~(size_t)255; }

bool cached_rules(frg_context *ctx, const frg_integral_desc &d, RadialRule *rad, AngleRule *ang,
                  PhiRule *phi) {
    if (is_ft(d.family)) {
        FreqRule f;
        if (freq_rule(d, &f) != FRG_OK) return false;
        auto it = ctx->ft_radial.find(std::make_tuple(d.n_q, d.q_max, d.k, d.T, f.lambda,
                                                      d.statistics, d.n_tail,
                                                      d.regulator * 32 + reg_order(d)));
        if (it == ctx->ft_radial.end()) return false;
        *rad = it->second->rule;
    } else {
        auto it = ctx->radial.find(std::make_tuple(d.n_q, d.q_max, d.d, d.regulator,
                                                   reg_order(d)));
        if (it == ctx->radial.end()) return false;
        *rad = it->second->rule;
    }
    if (is_vertex(d.family)) {
        auto it = ctx->cos1.find(d.n_x + (is_ft(d.family) ? (1 << 20) : 0));
        if (it == ctx->cos1.end()) return false;
        *ang = it->second->rule;
    }
    if (has_phi(d.family)) {
        auto it = ctx->phi.find(d.n_phi + (is_ft(d.family) ? (1 << 20) : 0));
        if (it == ctx->phi.end()) return false;
        *phi = it->second->rule;
    }
    return true;
}

size_t rules_bytes(const frg_integral_desc &d) {
    size_t b = up256(radial_rule_bytes(d.n_q));  // vacuum rule (finite temperature: its d = 3 base)
    if (is_ft(d.family)) {
        FreqRule f;
        if (freq_rule(d, &f) != FRG_OK) return 0;
        b += up256(ft_rule_bytes(d.n_q, f.n_f));
    }
    if (is_vertex(d.family)) b += up256(cos1_rule_bytes(d.n_x));
    if (has_phi(d.family)) b += up256(phi_rule_bytes(d.n_phi));
    return b;
}

frg_status rules_into(frg_context *ctx, const frg_integral_desc &d, void *buf, size_t bytes,
                      RadialRule *rad, AngleRule *ang, PhiRule *phi, hipStream_t s) {
    if (rules_bytes(d) == 0 || rules_bytes(d) > bytes) {
        set_error("quadrature-rule buffer too small");
        return FRG_E_INVAL;
    }
    char *p = (char *)buf;
    // the same kernels, arguments and layouts as the context's cache, so the same bits
    const int n = d.n_q;
    const int rd = is_ft(d.family) ? 3 : d.d;
    double *q = (double *)p, *W = q + n, *R = W + n;
    float *qf = (float *)(R + n), *Wf = qf + n, *Rf = Wf + n;
    double *A = after_floats(Rf + n);
    FRG_HIP_CHECK(launch_rules(n, d.q_max, rd, 0, 0, q, W, R, qf, Wf, Rf, nullptr, nullptr,
                               nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                               nullptr, s, false, d.regulator, reg_order(d)));
    FRG_HIP_CHECK(launch_rule_sum(q, R, A, n, s));
    RadialRule base{q, W, R, qf, Wf, Rf, nullptr, A};
    p += up256(radial_rule_bytes(n));
    if (is_ft(d.family)) {
        FreqRule f;
        frg_status st = freq_rule(d, &f);
        if (st != FRG_OK) return st;
        const size_t fb = ft_rule_bytes(d.n_q, f.n_f);
        if ((st = ft_rule_into(ctx, d, p, fb, rad, s, &base)) != FRG_OK) return st;
        p += up256(fb);
    } else {
        *rad = base;
    }
    if (is_vertex(d.family)) {
        const int m = d.n_x;
        double *x = (double *)p, *xw = x + m, *xs = xw + m;
        float *xf = (float *)(xs + m), *xwf = xf + m, *xsf = xwf + m;
        FRG_HIP_CHECK(launch_rules(0, 1.0, 1, m, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                                   nullptr, x, xw, xs, xf, xwf, xsf, nullptr, nullptr, nullptr,
                                   nullptr, s, is_ft(d.family) ? kPlainCos1 : 0));
        *ang = AngleRule{x, xw, xs, xf, xwf, xsf};
        p += up256(cos1_rule_bytes(m));
    }
    if (has_phi(d.family)) {
        const int m = d.n_phi;
        double *c = (double *)p, *w = c + m;
        float *cf = (float *)(w + m), *wf = cf + m;
        FRG_HIP_CHECK(launch_rules(0, 1.0, 1, 0, m, nullptr, nullptr, nullptr, nullptr, nullptr,
                                   nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                   c, w, cf, wf, s, is_ft(d.family) ? kPlainPhi : 0));
        *phi = PhiRule{c, w, cf, wf};
    }
    return FRG_OK;
}

// ---------------------------------------------------------------------------------------------
// Planning
// ---------------------------------------------------------------------------------------------
static int ilog2(int v) {
    int r = 0;
    while ((1 << (r + 1)) <= v) ++r;
    return r;
}

// Tile shape of a vertex request launched alone, by a cost estimate over every shape: lanes per
// point over radial nodes (lq) and cos1 nodes (lx), points per wavefront (le = 64 / (lq lx))
// and radial chunks (c).  A wavefront runs its lanes in lockstep, so its time is the longest
// lane's work W = ceil(ceil(n_q / c) / lq) ceil(n_x / lx) n_phi node evaluations (radial and
// cos1 node counts that are not multiples of the lanes leave lanes idle in the last round); T
// = ceil(n_ext / le) c wavefronts spread over the SIMDs (target_waves / 4 of them), m =
// ceil(T / SIMDs) per SIMD, and a SIMD with m wavefronts gets through rate(m) of its issue
// rate (one wavefront cannot hide its own latencies).  Estimate: m (W + per-tile set-up) /
// rate(m), plus the radial-sum pass when c > 1; the two-point families pay ~35 % more per node
// when they share cos1 nodes across lanes (their inner sums are short).
static TileShape request_shape_search(const frg_integral_desc &d, int n_ext, int target_waves) {
    const double simds = std::max(1, target_waves / 4);
    const int nphi = d.family == 3 ? d.n_phi : 1;
    auto rate = [](double m) { return m >= 4 ? 1.0 : (m >= 3 ? 0.95 : (m >= 2 ? 0.85 : 0.6)); };
    constexpr double kTileSetup = 20.0;   // node evaluations' worth per tile
    constexpr double kRadialSums = 40.0;  // the extra launch and contribution round trip
    TileShape best;
    double best_t = 1e300;
    for (int lql = 6; lql >= 0; --lql) {
        const int lq = 1 << lql;
        if (lq > d.n_q && lql > 0) continue;
        for (int lxl = 0; lql + lxl <= 6; ++lxl) {
            const int lx = 1 << lxl;
            if (lx > d.n_x && lxl > 0) break;
            const int le = kWave >> (lql + lxl);
            const long long et = (n_ext + le - 1) / le;
            const int max_c = std::max(1, std::min(d.n_q / lq, 64));
            for (int c = 1; c <= max_c; ++c) {
                const long long rq = ((d.n_q + c - 1) / c + lq - 1) / lq;
                const long long rx = (d.n_x + lx - 1) / lx;
                double W = (double)rq * (double)rx * nphi;
                if (d.family != 3 && lx > 1) W *= 1.35;
                const double T = (double)et * c;
                const double m = std::ceil(T / simds);
                const double t = m * (W + kTileSetup) / rate(m) + (c > 1 ? kRadialSums : 0.0);
                // ties: more radial lanes, then fewer chunks
                if (t < best_t * (1.0 - 1e-9)) {
                    best_t = t;
                    best.lq_log2 = lql;
                    best.lx_log2 = lxl;
                    best.chunks = c;
                }
            }
        }
    }
    return best;
}

TileShape heuristic_shape(const frg_integral_desc &desc, int n_ext, int target_waves,
                          bool allow_chunks, bool fused) {
    TileShape s;
    const frg_integral_desc d = plan_desc(desc);
    if (d.family == 1) return s;
    // a request launched alone: the estimate over every shape
    if (allow_chunks && !fused) return request_shape_search(d, n_ext, target_waves);
    // external points per wavefront: the smallest power of two >= n_ext, at least 4
    int le = kWave;
    while (le > 4 && le / 2 >= n_ext) le /= 2;
    int ext_tiles = (n_ext + le - 1) / le;
    // Prefer more lanes per point over radial chunks: a tile that holds all radial nodes of its
    // points finishes them within the wavefront, chunked tiles need the finalize pass.
    while (ext_tiles < target_waves && le > 1 && 2 * (kWave / le) <= d.n_q) {
        le /= 2;
        ext_tiles = (n_ext + le - 1) / le;
    }
    s.lq_log2 = ilog2(kWave / le);
    // integrand nodes one lane evaluates; splitting further than kMinLaneNodes would leave the
    // per-lane prologue and the cross-lane additions dominant
    constexpr int kMinLaneNodes = 16;
    auto lane_nodes = [&](int lq_log2, int lx_log2, int chunks) {
        const long long rq = (d.n_q + ((long long)chunks << lq_log2) - 1) /
                             ((long long)chunks << lq_log2);
        const long long rx = (d.n_x + (1LL << lx_log2) - 1) >> lx_log2;
        return rq * rx * (d.family == 3 ? d.n_phi : 1);
    };
    // then share the cos1 nodes of a radial node among lanes as well
    while (ext_tiles < target_waves && le > 1 && (2 << s.lx_log2) <= d.n_x &&
           lane_nodes(s.lq_log2, s.lx_log2 + 1, 1) >= kMinLaneNodes) {
        le /= 2;
        ++s.lx_log2;
        ext_tiles = (n_ext + le - 1) / le;
    }
    // Radial chunks cost a second (finalize) launch, a few microseconds: only for requests
    // with work enough to gain that back (about 15 us of the whole chip).
    const double nodes = (double)n_ext * d.n_q * d.n_x * (d.family == 3 ? d.n_phi : 1);
    if (!allow_chunks || nodes < 8.0e6) return s;
    const int lq_now = 1 << s.lq_log2;
    if (fused && d.family == 3 && n_ext >= 8 && d.n_q >= 16) {
        // three-point: 8 points x 8 radial lanes, one radial node per lane and chunk, so that a
        // wavefront's lanes share |p| and neighbouring radial nodes and often all take the exact
        // far-field path together (measured on the three-point batch: 604 -> 683 Gnodes/s)
        TileShape t;
        t.lq_log2 = 3;
        t.lx_log2 = 0;
        t.chunks = std::min(64, (d.n_q + 7) / 8);
        return t;
    }
    if (fused) {
        // A fused launch shares the chip with other requests: a request whose wavefronts hold
        // one point each gets radial chunks for about three rounds of the persistent grid
        // (twice its share of the wave target), so that the tile counter can balance the tail.
        // Two-point families only (measured: +12 % on the finite-temperature batch; sharing
        // cos1 nodes among lanes instead costs them 30-40 %).
        if (le == 1 && d.family != 3) {
            const int max_chunks = (d.n_q + lq_now - 1) / lq_now;
            const int want = (2 * target_waves + ext_tiles - 1) / ext_tiles;
            s.chunks = std::max(1, std::min(max_chunks, want));
        }
        return s;
    }
    // 64 lanes per point and still too few tiles (three-point): move radial lanes to cos1 lanes
    // and give the radial nodes freed that way to further chunks (same lanes per point, twice
    // the tiles).  The two-point families take plain radial chunks below instead (their cos1
    // sums shared across lanes cost more than they gain).
    while (d.family == 3 && le == 1 && ext_tiles * s.chunks < target_waves && s.lq_log2 > 0 &&
           (2 << s.lx_log2) <= d.n_x &&
           lane_nodes(s.lq_log2 - 1, s.lx_log2 + 1, s.chunks * 2) >= kMinLaneNodes) {
        --s.lq_log2;
        ++s.lx_log2;
        s.chunks *= 2;
    }
    if (s.chunks > 1) return s;
    int lq = 1 << s.lq_log2;
    int max_chunks = (d.n_q + lq - 1) / lq;  // at least one radial node per lane and chunk
    // chunks only when even the narrowest tiles leave the chip mostly idle
    int want = ext_tiles * 4 >= target_waves ? 1 : (target_waves + ext_tiles - 1) / ext_tiles;
    s.chunks = std::max(1, std::min(max_chunks, want));
    return s;
}

TileShape choose_shape(frg_context *ctx, const frg_integral_desc &desc, int n_ext,
                       int target_waves, ShapeUse use) {
    // finite-temperature requests share the tuned shapes of their vacuum counterparts
    const frg_integral_desc d = plan_desc(desc);
    std::vector<int> key = {d.family, d.precision, d.n_q, d.n_x, d.n_phi, n_ext, target_waves};
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end() && (use != ShapeUse::kNoChunks || it->second.chunks == 1))
        return it->second;
    return heuristic_shape(d, n_ext, target_waves, use != ShapeUse::kNoChunks,
                           use == ShapeUse::kFused);
}

// Only radially chunked requests hand contributions between workgroups; a single-chunk tile
// reduces its points within the wavefront and needs neither scratch nor counters.
size_t contrib_doubles(const ReqDev &r) {
    if (r.family == 1 || r.chunks == 1) return 0;
    // [n_q][n_ext] contributions (and as many derivative contributions)
    return (size_t)r.n_q * (size_t)r.n_ext * (r.dout ? 2 : 1);
}

int counter_count(const ReqDev &r) {
    // float32 form: one amplification slot per point and the dressing table's relative step
    if (r.family == 1 || r.chunks == 1 || r.precision == 0) return 0;
    return r.n_ext + 1;
}

int tile_count(const ReqDev &r) { return r.ext_tiles * r.chunks; }

int finalize_blocks(const ReqDev &r) {
    return (r.family == 1 || r.chunks <= 1) ? 0 : (r.n_ext + kWave - 1) / kWave;
}

int lds_bytes_for(const ReqDev &r) {
    // logarithm table and dressing pairs (the float32 form rounds the float64 pairs at use)
    if (r.family == 1) return 0;
    return (kLogTable + r.nZ + 1) * (int)sizeof(double2);
}

frg_status make_request(frg_context *ctx, const frg_integral_desc &d, const frg_batch &b,
                        const TileShape &shape, int m2_mode, double m2_floor, double coef,
                        ReqDev *out, const RadialRule *rad, const AngleRule *ang,
                        const PhiRule *phi) {
    ReqDev r;
    std::memset(&r, 0, sizeof r);
    // kernel family: LPA at finite temperature runs the LPA kernel on the frequency-folded rule
    const bool lpa = is_lpa(d.family), vertex = is_vertex(d.family);
    FreqRule fr;
    if (is_ft(d.family)) {
        const frg_status fs = freq_rule(d, &fr);
        if (fs != FRG_OK) return fs;
    }
    r.family = d.family == FRG_FAMILY_LPA_T ? FRG_FAMILY_LPA : d.family;
    if (d.complex_freq)
        r.family = d.family == FRG_FAMILY_THREE_POINT_T ? kFamThreePointComplex
                                                        : kFamTwoPointComplex;
    r.d = d.d;
    r.n_q = is_ft(d.family) ? d.n_q * fr.n_f : d.n_q;
    r.n_x = vertex ? d.n_x : 0;
    r.n_phi = has_phi(d.family) ? d.n_phi : 0;
    r.precision = d.precision;
    r.n_ext = b.n_ext;
    r.lq_log2 = lpa ? 0 : shape.lq_log2;
    r.lx_log2 = vertex ? shape.lx_log2 : 0;
    r.chunks = lpa ? 1 : shape.chunks;
    int le = kWave >> (r.lq_log2 + r.lx_log2);
    r.ext_tiles = (b.n_ext + le - 1) / le;
    r.k = d.k;
    r.k2 = d.k * d.k;
    const double pi = 3.141592653589793238462643383279502884;
    double omega;
    if (d.family == FRG_FAMILY_LPA)
        omega = 2.0 * std::pow(pi, 0.5 * d.d) / std::tgamma(0.5 * d.d) / std::pow(2.0 * pi, d.d);
    else if (d.family == FRG_FAMILY_TWO_POINT)
        omega = 4.0 * pi / std::pow(2.0 * pi, 4);
    else if (d.family == FRG_FAMILY_THREE_POINT)
        omega = 2.0 * pi / std::pow(2.0 * pi, 4);
    else if (d.family == FRG_FAMILY_LPA_T)
        omega = 4.0 * pi / std::pow(2.0 * pi, 3);  // int d^3q/(2pi)^3, radial
    else if (d.family == FRG_FAMILY_TWO_POINT_T)
        omega = 2.0 * pi / std::pow(2.0 * pi, 3);  // int d^3q/(2pi)^3 = 2pi int q^2 dq dx/(2pi)^3
    else
        omega = 2.0 / std::pow(2.0 * pi, 3);  // = int q^2 dq dx dphi/(2pi)^3, phi over [0, pi] x 2
    // vacuum: k^(d+2) from the k-scaled nodes, weights and Rdot; finite temperature: k^5 from the
    // spatial part and one k from the frequency weights, which the rule holds as c_j/k
    r.pref = omega * std::pow(d.k, d.d + 2) * coef;
    r.m2_mode = b.m2 ? m2_mode : 0;
    r.reg = d.regulator;
    r.reg_n = reg_order(d);
    r.far_y = d.regulator == FRG_REG_POLY_EXP ? poly_exp_far_y(r.reg_n, 760.0) : 38.0;
    // the float32 form drops e^-S_N below e^-24 (its bound carries that term)
    r.far_y32 = d.regulator == FRG_REG_POLY_EXP
                    ? std::nextafter((float)poly_exp_far_y(r.reg_n, 24.0), 3.0e38f)
                    : 3.0e38f;
    r.m2s = b.m2_scalar;
    r.m2_floor = m2_floor;
    r.tau = d.precision == 1 ? d.near_pole_tau : 0.0;
    if (vertex) {
        // without a dressing table the kernels look up a two-entry table of ones (Z == 1 exactly),
        // which keeps the inner loops free of branches
        const bool has = b.Z.values != nullptr;
        r.nZ = has ? b.Z.n : 2;
        double xmin = has ? b.Z.x_min : 1.0, xmax = has ? b.Z.x_max : 2.0;
        double lmin = std::log(xmin), lmax = std::log(xmax);
        double delta = (lmax - lmin) / (double)(r.nZ - 1);
        r.za = 0.5 / delta;
        r.zb = -lmin / delta;
        r.zbk = r.zb + r.za * std::log(r.k2);
        r.Z = has ? b.Z.values : (const double *)ctx->ones.ptr;
    }
    frg_status st = FRG_OK;
    if (rad)
        r.rad = *rad;
    else
        st = is_ft(d.family) ? get_ft_radial(ctx, d, fr, &r.rad)
                             : get_radial(ctx, d.n_q, d.q_max, d.d, d.regulator, reg_order(d),
                                          &r.rad);
    if (st != FRG_OK) return st;
    if (vertex) {
        if (ang)
            r.ang = *ang;
        else
            st = get_cos1(ctx, d.n_x, &r.ang, is_ft(d.family));
        if (st != FRG_OK) return st;
    }
    if (has_phi(d.family)) {
        if (phi)
            r.phi = *phi;
        else
            st = get_phi(ctx, d.n_phi, &r.phi, is_ft(d.family));
        if (st != FRG_OK) return st;
    }
    r.logt = (const double2 *)ctx->logtab.ptr;
    r.ext = b.ext;
    r.m2 = b.m2;
    r.out = b.out;
    r.err = b.err_out;
    // complex frequencies: the imaginary parts take the derivative's place, after the real ones
    r.dout = d.complex_freq ? b.out + b.n_ext : b.dout_dm2;
    *out = r;
    return FRG_OK;
}

// ---------------------------------------------------------------------------------------------
// Scratch and launches
// ---------------------------------------------------------------------------------------------
static frg_status grow(DeviceBuffer &buf, size_t bytes, hipStream_t s, bool zero_u32) {
    if (buf.bytes >= bytes && buf.ptr) return FRG_OK;
    if (buf.ptr) {
        // queued work on this stream may still use the old buffer
        FRG_HIP_CHECK(hipStreamSynchronize(s));
        FRG_HIP_CHECK(hipFree(buf.ptr));
        buf.ptr = nullptr;
        buf.bytes = 0;
    }
    size_t want = std::max<size_t>(bytes, 4096);
    want = want + want / 2;
    FRG_HIP_CHECK(buf.alloc(want));
    if (zero_u32) FRG_HIP_CHECK(launch_fill_zero_u32((unsigned *)buf.ptr, want / 4, s));
    return FRG_OK;
}

frg_status get_scratch(frg_context *ctx, hipStream_t s, size_t n_contrib, size_t n_counters,
                       size_t n_reqs, size_t n_tiles, Scratch **out) {
    auto &slot = ctx->scratch[s];
    if (!slot) slot = std::make_unique<Scratch>();
    Scratch *sc = slot.get();
    frg_status st;
    if ((st = grow(sc->contrib, n_contrib * sizeof(double), s, false)) != FRG_OK) return st;
    if ((st = grow(sc->counters, n_counters * sizeof(unsigned), s, true)) != FRG_OK) return st;
    if ((st = grow(sc->work, 2 * sizeof(unsigned), s, true)) != FRG_OK) return st;
    sc->last_key.clear();
    sc->last_dz.clear();
    if ((st = grow(sc->reqs, n_reqs * sizeof(ReqDev), s, false)) != FRG_OK) return st;
    if ((st = grow(sc->tiles, n_tiles * sizeof(TileDev), s, false)) != FRG_OK) return st;
    *out = sc;
    return FRG_OK;
}

frg_status run_batch(frg_context *ctx, ReqDev &r, hipStream_t s, Scratch *sc) {
    (void)ctx;
    r.contrib_base = 0;
    r.ctr_base = 0;
    FRG_HIP_CHECK(launch_batch(&r, nullptr, tile_count(r), lds_bytes_for(r),
                               (double *)sc->contrib.ptr, (unsigned *)sc->counters.ptr, s));
    FRG_HIP_CHECK(launch_finalize(r, (const double *)sc->contrib.ptr,
                                  (unsigned *)sc->counters.ptr, s));
    return FRG_OK;
}

std::vector<TileDev> make_tiles(const std::vector<ReqDev> &reqs, int *lds_out,
                                const std::vector<std::pair<int, int>> *et_ranges) {
    std::vector<TileDev> tiles;
    std::vector<double> cost;
    int lds = 0;
    for (size_t i = 0; i < reqs.size(); ++i) {
        const ReqDev &r = reqs[i];
        lds = std::max(lds, lds_bytes_for(r));
        int lq = 1 << r.lq_log2;
        double inner = r.family == 1 ? 1.0
                                     : std::ceil((double)r.n_x / (1 << r.lx_log2)) *
                                           (req_has_phi(r.family) ? r.n_phi : 1);
        const int et0 = et_ranges ? (*et_ranges)[i].first : 0;
        const int et1 = et_ranges ? (*et_ranges)[i].second : r.ext_tiles;
        for (int et = et0; et < et1; ++et)
            for (int ch = 0; ch < r.chunks; ++ch) {
                int a0 = (int)(((long long)r.n_q * ch) / r.chunks);
                int a1 = (int)(((long long)r.n_q * (ch + 1)) / r.chunks);
                double c = r.family == 1 ? (double)r.n_q
                                         : std::ceil((double)(a1 - a0) / lq) * inner;
                tiles.push_back(TileDev{(int)i, et, ch, 0});
                cost.push_back(c);
            }
    }
    // longest-processing-time-first order; ties keep request/tile order
    std::vector<int> order(tiles.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<TileDev> sorted(tiles.size());
    for (size_t i = 0; i < order.size(); ++i) sorted[i] = tiles[order[i]];
    if (lds_out) *lds_out = lds;
    return sorted;
}

void common_kind(const std::vector<ReqDev> &reqs, int *fam, int *prec, int *reg, int *der) {
    // the LPA kernel takes its regulator from the radial rule and its derivative flag from the
    // request
    auto reg_of = [](const ReqDev &r) { return r.family == 1 ? 0 : r.reg; };
    *fam = reqs.empty() ? -1 : reqs[0].family;
    *prec = reqs.empty() ? -1 : reqs[0].precision;
    *reg = reqs.empty() ? -1 : reg_of(reqs[0]);
    *der = 0;  // 1 if any vertex request asks for the mass derivative
    for (const ReqDev &r : reqs) {
        if (r.family != *fam) *fam = -1;
        if (r.precision != *prec) *prec = -1;
        if (reg_of(r) != *reg) *reg = -1;
        if (r.family != 1 && r.dout) *der = 1;
    }
    if (*fam < 0 || *prec < 0 || *reg < 0) *fam = *prec = *reg = -1;
}

frg_status run_multi(frg_context *ctx, std::vector<ReqDev> &reqs, hipStream_t s, Scratch *sc,
                     int grid_waves) {
    sc->last_dz.clear();  // a new plan: its caller adds its derivative blocks
    long long cb = 0, ctr = 0;
    for (ReqDev &r : reqs) {
        r.contrib_base = cb;
        r.ctr_base = ctr;
        cb += (long long)contrib_doubles(r);
        ctr += counter_count(r);
    }
    int lds = 0;
    std::vector<TileDev> sorted = make_tiles(reqs, &lds);
    if (sorted.empty()) return FRG_OK;
    // radially chunked requests: (request, block of 64 points) entries of the finalize launch,
    // stored after the tiles
    const size_t n_work = sorted.size();
    for (size_t i = 0; i < reqs.size(); ++i)
        for (int b = 0; b < finalize_blocks(reqs[i]); ++b)
            sorted.push_back(TileDev{(int)i, b, 0, 0});
    const int n_fin = (int)(sorted.size() - n_work);
    size_t rb = reqs.size() * sizeof(ReqDev), tb = sorted.size() * sizeof(TileDev);
    if (!sc->staged) FRG_HIP_CHECK(hipEventCreateWithFlags(&sc->staged, hipEventDisableTiming));
    // the previous upload from the staging area must have finished before it is rewritten
    FRG_HIP_CHECK(hipEventSynchronize(sc->staged));
    if (sc->host_bytes < rb + tb) {
        if (sc->host_stage) FRG_HIP_CHECK(hipHostFree(sc->host_stage));
        sc->host_stage = nullptr;
        sc->host_bytes = 0;
        size_t want = (rb + tb) + (rb + tb) / 2 + 4096;
        FRG_HIP_CHECK(hipHostMalloc(&sc->host_stage, want, hipHostMallocDefault));
        sc->host_bytes = want;
    }
    std::memcpy(sc->host_stage, reqs.data(), rb);
    std::memcpy((char *)sc->host_stage + rb, sorted.data(), tb);
    FRG_HIP_CHECK(hipMemcpyAsync(sc->reqs.ptr, sc->host_stage, rb, hipMemcpyHostToDevice, s));
    FRG_HIP_CHECK(hipMemcpyAsync(sc->tiles.ptr, (char *)sc->host_stage + rb, tb,
                                 hipMemcpyHostToDevice, s));
    FRG_HIP_CHECK(hipEventRecord(sc->staged, s));
    sc->last_tiles = (int)n_work;
    sc->last_fin = n_fin;
    common_kind(reqs, &sc->last_fam, &sc->last_prec, &sc->last_reg, &sc->last_der);
    sc->last_grid = std::min(multi_grid((int)n_work, sc->last_fam, sc->last_prec,
                                        sc->last_reg, sc->last_der, lds, ctx->num_cus),
        std::max(grid_waves, 1));
    sc->last_lds = lds;
    sc->last_nreqs = (int)reqs.size();
    return relaunch_multi(sc, s);
}

frg_status relaunch_multi(Scratch *sc, hipStream_t s) {
    FRG_HIP_CHECK(launch_multi((const ReqDev *)sc->reqs.ptr, sc->last_fam, sc->last_prec,
                               sc->last_reg, sc->last_der, (const TileDev *)sc->tiles.ptr, sc->last_tiles, sc->last_grid,
                               sc->last_lds, (double *)sc->contrib.ptr,
                               (unsigned *)sc->counters.ptr, (unsigned *)sc->work.ptr, s));
    FRG_HIP_CHECK(launch_multi_finalize((const ReqDev *)sc->reqs.ptr,
                                        (const TileDev *)sc->tiles.ptr + sc->last_tiles,
                                        sc->last_fin, (const double *)sc->contrib.ptr,
                                        (unsigned *)sc->counters.ptr, s));
    for (const auto &d : sc->last_dz) FRG_HIP_CHECK(launch_dz(d.first, d.second, s));
    return FRG_OK;
}

// ---------------------------------------------------------------------------------------------
// Flow right-hand sides, captured as HIP graphs
// ---------------------------------------------------------------------------------------------
struct FlowGraph {
    hipGraphExec_t exec = nullptr;  // captured plan (graph mode), else launched directly
    hipGraph_t graph = nullptr;
    DeviceBuffer contrib;
    DeviceBuffer counters;
    ReqDev r{};             // the integrals of the right-hand side
    int family = 0, n = 0, n_comp = 0;
    const double *grid = nullptr, *state = nullptr;
    double m2_floor = 0.0;
    double *dstate_dt = nullptr;
    // state -> masses -> integrals -> assembly on stream s (LPA: one fused kernel)
    hipError_t enqueue(hipStream_t s) const {
        if (family == 1) return launch_lpa_rhs(r, n, n_comp, grid, state, m2_floor, dstate_dt, s);
        const hipError_t e = launch_batch(&r, nullptr, tile_count(r), lds_bytes_for(r),
                                          (double *)contrib.ptr, (unsigned *)counters.ptr, s);
        if (e != hipSuccess) return e;
        return launch_finalize(r, (const double *)contrib.ptr, (unsigned *)counters.ptr, s);
    }
    ~FlowGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

}  // namespace frg

using namespace frg;

extern "C" {

const char *frg_last_error(void) { return g_last_error.c_str(); }

frg_status frg_context_create(int device, size_t hbm_budget_bytes, frg_context **out) {
    clear_error();
    if (!out) {
        set_error("out is NULL");
        return FRG_E_INVAL;
    }
    int n = 0;
    FRG_HIP_CHECK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) {
        set_error("device %d out of range (%d devices)", device, n);
        return FRG_E_INVAL;
    }
    FRG_HIP_CHECK(hipSetDevice(device));
    auto ctx = std::make_unique<frg_context>();
    ctx->device = device;
    hipDeviceProp_t prop;
    FRG_HIP_CHECK(hipGetDeviceProperties(&prop, device));
    ctx->num_cus = prop.multiProcessorCount;
    size_t free_b = 0, total_b = 0;
    FRG_HIP_CHECK(hipMemGetInfo(&free_b, &total_b));
    ctx->hbm_budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)free_b);
    FRG_HIP_CHECK(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
    // device address of the no-allocation entry point's static scratch (once per device)
    frg_status sst = noalloc_scratch_address(device, &ctx->noalloc_scratch);
    if (sst != FRG_OK) return sst;
    FRG_HIP_CHECK(ctx->logtab.alloc(kLogTable * sizeof(double2)));
    FRG_HIP_CHECK(launch_log_table((double2 *)ctx->logtab.ptr, ctx->aux));
    {
        const double ones[2] = {1.0, 1.0};
        FRG_HIP_CHECK(ctx->ones.alloc(sizeof ones));
        FRG_HIP_CHECK(hipMemcpy(ctx->ones.ptr, ones, sizeof ones, hipMemcpyHostToDevice));
    }
    FRG_HIP_CHECK(hipStreamSynchronize(ctx->aux));
    const char *fg = std::getenv("FRG_FLOW_GRAPH");
    ctx->flow_graphs = fg && fg[0] == '1';
    const char *tp = std::getenv("FRG_AUTOTUNE_CACHE");
    if (tp) {
        // lines: family precision n_q n_x n_phi n_ext target lq_log2 chunks [lx_log2]
        ctx->tune_path = tp;
        std::ifstream f(tp);
        std::string line;
        while (std::getline(f, line)) {
            std::istringstream ls(line);
            std::vector<int> v;
            int x;
            while (ls >> x) v.push_back(x);
            if (v.size() != 9 && v.size() != 10) continue;
            const int lx = v.size() == 10 ? v[9] : 0;
            if (v[7] < 0 || lx < 0 || v[7] + lx > 6 || v[8] < 1 || v[8] > FRG_MAX_NODES) continue;
            ctx->tuned[std::vector<int>(v.begin(), v.begin() + 7)] = TileShape{v[7], v[8], lx};
        }
    }
    *out = ctx.release();
    return FRG_OK;
}

frg_status frg_context_destroy(frg_context *ctx) {
    clear_error();
    if (!ctx) return FRG_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->graphs.clear();
    ctx->scratch.clear();
    ctx->ft_radial.clear();
    ctx->radial.clear();
    ctx->cos1.clear();
    ctx->phi.clear();
    if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
    delete ctx;
    return FRG_OK;
}

frg_status frg_integrate_batch(frg_context *ctx, const frg_integral_desc *desc,
                               const frg_batch *batch, hipStream_t stream) {
    clear_error();
    if (!ctx) {
        set_error("context is NULL");
        return FRG_E_INVAL;
    }
    frg_status st = validate(desc, batch, true);
    if (st != FRG_OK) return st;
    if (batch->n_ext == 0) return FRG_OK;
    std::lock_guard<std::mutex> lk(ctx->mu);
    FRG_HIP_CHECK(hipSetDevice(ctx->device));
    TileShape shape = choose_shape(ctx, *desc, batch->n_ext, 16 * ctx->num_cus);
    ReqDev r;
    if ((st = make_request(ctx, *desc, *batch, shape, 1, 0.0, 1.0, &r)) != FRG_OK) return st;
    Scratch *sc;
    if ((st = get_scratch(ctx, stream, contrib_doubles(r), counter_count(r), 1, 1, &sc)) != FRG_OK)
        return st;
    if ((st = run_batch(ctx, r, stream, sc)) != FRG_OK) return st;
    if (batch->dout_dz) FRG_HIP_CHECK(launch_dz(r, batch->dout_dz, stream));
    return FRG_OK;
}

frg_status frg_autotune(frg_context *ctx, const frg_integral_desc *desc, const frg_batch *batch,
                        hipStream_t stream, int reps, double *best_us) {
    clear_error();
    if (!ctx || reps < 1 || reps > 1000) {
        set_error("invalid arguments to frg_autotune");
        return FRG_E_INVAL;
    }
    frg_status st = validate(desc, batch, true);
    if (st != FRG_OK) return st;
    if (batch->n_ext == 0 || is_lpa(desc->family)) return FRG_OK;  // LPA has a single shape
    const frg_integral_desc pd = plan_desc(*desc);  // finite temperature: n_q n_f radial nodes
    std::lock_guard<std::mutex> lk(ctx->mu);
    FRG_HIP_CHECK(hipSetDevice(ctx->device));
    const int target = 16 * ctx->num_cus;
    std::vector<TileShape> cands;
    for (int lq = 0; lq <= 6; ++lq) {
        const int le = kWave >> lq;
        if (lq > 0 && le / 2 >= batch->n_ext) continue;  // narrower than needed
        const int max_chunks = (pd.n_q + (1 << lq) - 1) >> lq;
        for (int ch = 1; ch <= max_chunks; ch *= 2) cands.push_back(TileShape{lq, ch});
        if ((max_chunks & (max_chunks - 1)) != 0) cands.push_back(TileShape{lq, max_chunks});
        // cos1 nodes shared among lanes as well (single radial chunk)
        for (int lx = 1; lq + lx <= 6 && (1 << lx) <= desc->n_x; ++lx) {
            if ((kWave >> (lq + lx)) / 2 >= batch->n_ext && lq + lx > 0) continue;
            cands.push_back(TileShape{lq, 1, lx});
        }
    }
    cands.push_back(heuristic_shape(*desc, batch->n_ext, target, true, false));
    hipEvent_t e0, e1;
    FRG_HIP_CHECK(hipEventCreate(&e0));
    FRG_HIP_CHECK(hipEventCreate(&e1));
    double best = 1e300;
    TileShape best_shape = cands.back();
    frg_status res = FRG_OK;
    for (const TileShape &c : cands) {
        ReqDev r;
        if ((res = make_request(ctx, *desc, *batch, c, 1, 0.0, 1.0, &r)) != FRG_OK) break;
        Scratch *sc;
        if ((res = get_scratch(ctx, stream, contrib_doubles(r), counter_count(r), 1, 1, &sc)) !=
            FRG_OK)
            break;
        if ((res = run_batch(ctx, r, stream, sc)) != FRG_OK) break;  // warm-up
        double t_best = 1e300;
        for (int k = 0; k < reps && res == FRG_OK; ++k) {
            if (hipEventRecord(e0, stream) != hipSuccess) res = FRG_E_DEVICE;
            if (res == FRG_OK) res = run_batch(ctx, r, stream, sc);
            if (res == FRG_OK && hipEventRecord(e1, stream) != hipSuccess) res = FRG_E_DEVICE;
            if (res == FRG_OK && hipEventSynchronize(e1) != hipSuccess) res = FRG_E_DEVICE;
            float ms = 0.f;
            if (res == FRG_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) res = FRG_E_DEVICE;
            t_best = std::min(t_best, (double)ms * 1e3);
        }
        if (res != FRG_OK) break;
        if (const char *lp = std::getenv("FRG_AUTOTUNE_LOG")) {
            std::ofstream lf(lp, std::ios::app);
            if (lf)
                lf << pd.family << ' ' << pd.precision << ' ' << pd.n_q << ' ' << pd.n_x << ' '
                   << pd.n_phi << ' ' << batch->n_ext << ' ' << c.lq_log2
                   << ' ' << c.chunks << ' ' << c.lx_log2 << ' ' << t_best << '\n';
        }
        if (t_best < best) {
            best = t_best;
            best_shape = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (res != FRG_OK) {
        if (res == FRG_E_DEVICE && g_last_error.empty()) set_error("autotune launch failed");
        return res;
    }
    std::vector<int> key = {pd.family, pd.precision, pd.n_q, pd.n_x, pd.n_phi, batch->n_ext,
                            target};
    ctx->tuned[key] = best_shape;
    if (best_us) *best_us = best;
    if (!ctx->tune_path.empty()) {
        std::ofstream f(ctx->tune_path, std::ios::app);
        if (f) {
            for (int v : key) f << v << ' ';
            f << best_shape.lq_log2 << ' ' << best_shape.chunks << ' ' << best_shape.lx_log2
              << '\n';
        }
    }
    return FRG_OK;
}

frg_status frg_integrate_multi(frg_context *ctx, int n, const frg_integral_desc *descs,
                               const frg_batch *batches, hipStream_t stream) {
    clear_error();
    if (!ctx || n < 0 || (n > 0 && (!descs || !batches))) {
        set_error("invalid arguments to frg_integrate_multi");
        return FRG_E_INVAL;
    }
    frg_status st;
    // plan cache: the same arguments as the previous fused call on this stream relaunch the
    // uploaded plan directly (flows re-evaluate the same batches every stage)
    std::vector<char> key((size_t)n * (sizeof(frg_integral_desc) + sizeof(frg_batch)));
    if (n > 0) {
        std::memcpy(key.data(), descs, (size_t)n * sizeof(frg_integral_desc));
        std::memcpy(key.data() + (size_t)n * sizeof(frg_integral_desc), batches,
                    (size_t)n * sizeof(frg_batch));
    }
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->scratch.find(stream);
        if (n > 0 && it != ctx->scratch.end() && it->second->last_key == key &&
            it->second->last_tiles > 0) {
            FRG_HIP_CHECK(hipSetDevice(ctx->device));
            return relaunch_multi(it->second.get(), stream);
        }
    }
    double total_nodes = 0.0;
    std::vector<double> nodes(n);
    for (int i = 0; i < n; ++i) {
        if ((st = validate(&descs[i], &batches[i], true)) != FRG_OK) {
            std::string m = g_last_error;
            set_error("batch %d: %s", i, m.c_str());
            return st;
        }
        nodes[i] = nodes_per_point(descs[i]) * batches[i].n_ext;
        total_nodes += nodes[i];
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    FRG_HIP_CHECK(hipSetDevice(ctx->device));
    std::vector<ReqDev> reqs;
    std::vector<std::pair<ReqDev, double *>> dz;  // dressing-table derivatives, after the launch
    size_t n_contrib = 0, n_ctr = 0, n_tiles = 0;
    const int target_total = 32 * ctx->num_cus;  // about twice the resident waves
    int n_active = 0;
    for (int i = 0; i < n; ++i) n_active += batches[i].n_ext > 0;
    for (int i = 0; i < n; ++i) {
        if (batches[i].n_ext == 0) continue;
        int target = std::max(1, (int)std::lround(target_total * nodes[i] / total_nodes));
        // radially chunked (tuned) shapes are summed by one finalize launch after the fused one;
        // a launch of one request is planned as that request alone
        const ShapeUse use = n_active == 1 ? ShapeUse::kRequest : ShapeUse::kFused;
        if (n_active == 1) target = 16 * ctx->num_cus;
        TileShape shape = choose_shape(ctx, descs[i], batches[i].n_ext, target, use);
        ReqDev r;
        if ((st = make_request(ctx, descs[i], batches[i], shape, 1, 0.0, 1.0, &r)) != FRG_OK)
            return st;
        n_contrib += contrib_doubles(r);
        n_ctr += counter_count(r);
        n_tiles += tile_count(r) + finalize_blocks(r);
        reqs.push_back(r);
        if (batches[i].dout_dz) dz.emplace_back(r, batches[i].dout_dz);
    }
    if (reqs.empty()) return FRG_OK;
    Scratch *sc;
    if ((st = get_scratch(ctx, stream, n_contrib, n_ctr, reqs.size(), n_tiles, &sc)) != FRG_OK)
        return st;
    sc->last_key.clear();
    if ((st = run_multi(ctx, reqs, stream, sc, 1 << 30)) != FRG_OK) return st;
    for (const auto &d : dz) FRG_HIP_CHECK(launch_dz(d.first, d.second, stream));
    sc->last_dz = std::move(dz);
    sc->last_key = std::move(key);
    return FRG_OK;
}

frg_status frg_flow_rhs(frg_context *ctx, const frg_integral_desc *desc,
                        const frg_flow_state *state, double *dstate_dt, hipStream_t stream) {
    clear_error();
    if (!ctx || !desc || !state || !dstate_dt) {
        set_error("null argument to frg_flow_rhs");
        return FRG_E_INVAL;
    }
    if (state->family != desc->family) {
        set_error("flow state family %d does not match descriptor family %d", state->family,
                  desc->family);
        return FRG_E_INVAL;
    }
    if (desc->complex_freq) {
        set_error("complex external frequencies give complex integrals: no flow right-hand side");
        return FRG_E_UNSUPPORTED;
    }
    const int n = state->n_ext;
    const bool lpa = is_lpa(desc->family);
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
    // the batch the integrals run on (pointers filled below)
    frg_batch b;
    std::memset(&b, 0, sizeof b);
    b.n_ext = lpa ? 2 * n : n;
    b.ext = lpa ? nullptr : state->grid;
    b.m2 = state->state;
    b.Z = state->Z;
    b.out = dstate_dt;
    frg_status st = FRG_OK;

    std::lock_guard<std::mutex> lk(ctx->mu);
    FRG_HIP_CHECK(hipSetDevice(ctx->device));
    // the plan's key holds every descriptor and state field and every pointer: a plan found
    // under it was validated when it was built
    std::vector<long long> key = {desc->family, desc->d, desc->n_q, desc->n_x, desc->n_phi,
                                  desc->precision, n, state->n_comp, (long long)stream,
                                  (long long)state->state, (long long)state->grid,
                                  (long long)state->Z.values, state->Z.n, (long long)dstate_dt};
    key.push_back(desc->statistics);
    key.push_back(desc->n_tail);
    key.push_back(desc->freq_scaled);
    key.push_back(desc->regulator);
    key.push_back(desc->reg_order);
    double dk[9] = {desc->q_max, desc->k,        desc->near_pole_tau, state->m2_floor, state->coef,
                    state->Z.x_min, state->Z.x_max, desc->T, desc->freq_max};
    for (double v : dk) {
        long long bits;
        std::memcpy(&bits, &v, sizeof bits);
        key.push_back(bits);
    }
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        if ((st = validate(desc, &b, true)) != FRG_OK) return st;
        auto g = std::make_unique<FlowGraph>();
        TileShape shape = choose_shape(ctx, *desc, b.n_ext, 16 * ctx->num_cus);
        ReqDev r;
        if (lpa) {
            // the fused kernel takes rules, prefactor and precision from r; masses come from
            // the state inside it
            if ((st = make_request(ctx, *desc, b, shape, 1, 0.0, 1.0, &r)) != FRG_OK) return st;
        } else {
            if ((st = make_request(ctx, *desc, b, shape, 2, state->m2_floor, state->coef, &r)) !=
                FRG_OK)
                return st;
        }
        FRG_HIP_CHECK(g->contrib.alloc(std::max<size_t>(contrib_doubles(r), 1) * sizeof(double)));
        FRG_HIP_CHECK(
            g->counters.alloc(std::max<size_t>(counter_count(r), 1) * sizeof(unsigned)));
        FRG_HIP_CHECK(launch_fill_zero_u32((unsigned *)g->counters.ptr,
                                           std::max<size_t>(counter_count(r), 1), ctx->aux));
        FRG_HIP_CHECK(hipStreamSynchronize(ctx->aux));
        r.contrib_base = 0;
        r.ctr_base = 0;
        g->r = r;
        g->family = r.family;  // kernel family: 1 for both LPA families
        g->n = n;
        g->n_comp = state->n_comp;
        g->grid = state->grid;
        g->state = state->state;
        g->m2_floor = state->m2_floor;
        g->dstate_dt = dstate_dt;
        if (ctx->flow_graphs) {
            FRG_HIP_CHECK(hipStreamBeginCapture(ctx->aux, hipStreamCaptureModeThreadLocal));
            const hipError_t e1 = g->enqueue(ctx->aux);
            const hipError_t e2 = hipStreamEndCapture(ctx->aux, &g->graph);
            if (e1 != hipSuccess || e2 != hipSuccess) {
                set_error("graph capture failed: %s / %s", hipGetErrorString(e1),
                          hipGetErrorString(e2));
                return FRG_E_DEVICE;
            }
            FRG_HIP_CHECK(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
        }
        it = ctx->graphs.emplace(key, std::move(g)).first;
    }
    if (it->second->exec) {
        FRG_HIP_CHECK(hipGraphLaunch(it->second->exec, stream));
    } else {
        FRG_HIP_CHECK(it->second->enqueue(stream));
    }
    return FRG_OK;
}

}  // extern "C"
