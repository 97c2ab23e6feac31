/*
 * frg_oracle.c -- plain FP64 CPU oracle for the batched fRG loop integrals.
 *
 * TEST INFRASTRUCTURE ONLY (see frg_oracle.h).  Deliberately simple: every node term is
 * evaluated in full from the definitions, in nested loops, with libm math and
 * Neumaier-compensated sums.  No hoisting, no blocking, no reordering beyond the sum order.
 */
#include "frg_oracle.h"

#include <complex.h>
#include <math.h>
#include <stddef.h>

#define PI 3.14159265358979323846264338327950288

/* ---------------------------------------------------------------------------------------- */
/* Neumaier (improved Kahan-Babuska) compensated summation.                                  */
/* ---------------------------------------------------------------------------------------- */
typedef struct {
    double s, c;
} nsum;

static void nsum_add(nsum *acc, double v) {
    double t = acc->s + v;
    if (fabs(acc->s) >= fabs(v))
        acc->c += (acc->s - t) + v;
    else
        acc->c += (v - t) + acc->s;
    acc->s = t;
}

static double nsum_get(const nsum *acc) { return acc->s + acc->c; }

/* ---------------------------------------------------------------------------------------- */
/* Gauss-Legendre: nodes are the roots of P_n, found by Newton's method on the three-term    */
/* recurrence (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}; weights 2/((1-x^2) P_n'(x)^2).       */
/* Computed in long double, mapped affinely to [a, b].                                      */
/* ---------------------------------------------------------------------------------------- */
static void legendre_eval(int n, long double x, long double *pn, long double *dpn) {
    long double p0 = 1.0L, p1 = x;
    if (n == 0) {
        *pn = 1.0L;
        *dpn = 0.0L;
        return;
    }
    for (int j = 1; j < n; ++j) {
        long double p2 = ((2.0L * j + 1.0L) * x * p1 - (long double)j * p0) / (j + 1.0L);
        p0 = p1;
        p1 = p2;
    }
    *pn = p1;
    /* P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1) */
    *dpn = (long double)n * (x * p1 - p0) / (x * x - 1.0L);
}

int frgo_gauss_legendre(int n, double a, double b, double *nodes, double *weights) {
    if (n < 1 || !(b > a) || nodes == NULL || weights == NULL) return -1;
    const long double pi = 3.141592653589793238462643383279502884L;
    long double half = 0.5L * ((long double)b - (long double)a);
    long double mid = 0.5L * ((long double)b + (long double)a);
    for (int i = 0; i < n; ++i) {
        /* i-th root from the largest down; Tricomi-type starting value */
        long double x = cosl(pi * (i + 0.75L) / (n + 0.5L));
        long double pn = 0, dpn = 1;
        for (int it = 0; it < 40; ++it) {
            legendre_eval(n, x, &pn, &dpn);
            long double dx = pn / dpn;
            x -= dx;
            /* quadratic convergence: once a step is this small the next error is negligible */
            if (fabsl(dx) < 1e-18L) break;
        }
        legendre_eval(n, x, &pn, &dpn);
        long double w = 2.0L / ((1.0L - x * x) * dpn * dpn);
        /* store ascending: root i (descending order) goes to slot n-1-i */
        nodes[n - 1 - i] = (double)(mid + half * x);
        weights[n - 1 - i] = (double)(half * w);
    }
    return 0;
}

/* ---------------------------------------------------------------------------------------- */
/* Regulators.                                                                               */
/*   exponential:  R = l2/(exp(y) - 1), y = l2/k^2.  At fixed l2, k dy/dk = -2 y, so         */
/*   k dR/dk = l2 e^y 2y/(e^y - 1)^2 = 2 k^2 y^2 e^y/(e^y - 1)^2 (> 0).  Both are written     */
/*   with E = expm1(-y), e = exp(-y): R = k^2 y e/(-E), Rdot = 2 k^2 y^2 e/E^2, so that no   */
/*   cancellation (small y) or overflow (large y) occurs.                                    */
/*   flat (Litim):  R = (k^2 - l2) Theta(k^2 - l2), k dR/dk = 2 k^2 Theta(k^2 - l2).         */
/* ---------------------------------------------------------------------------------------- */
static void exp_pair(double y, double *e, double *E) {
    /* e = exp(-y), E = exp(-y) - 1, each to full relative precision */
    if (y < 0.69314718055994530942) {
        *E = expm1(-y);
        *e = 1.0 + *E;
    } else {
        *e = exp(-y);
        *E = *e - 1.0;
    }
}

/* polynomial-exponential shape (Sec. 3.1): S = sum_{i=1}^{N} y^i / i and P = sum_{i=1}^{N} y^i,
 * each term from its own power of y; R = k^2 e^{-S}; at fixed l2, k dy/dk = -2y gives
 * k dR/dk = 2 k^2 e^{-S} + k^2 e^{-S} (-S'(y)) (-2y) = 2 k^2 e^{-S} (1 + y S'(y)), y S' = P. */
static void polyexp_sums(int N, double y, double *S, double *P) {
    double s = 0.0, p = 0.0, yi = 1.0;
    for (int i = 1; i <= N; ++i) {
        yi *= y;
        s += yi / (double)i;
        p += yi;
    }
    *S = s;
    *P = p;
}

double frgo_regulator(int kind, double l2, double k) {
    double k2 = k * k;
    if (l2 < 0.0) l2 = 0.0;
    if (kind == FRGO_REG_LITIM) return (l2 < k2) ? (k2 - l2) : 0.0;
    if (kind > FRGO_REG_POLYEXP && kind <= FRGO_REG_POLYEXP + 64) {
        double S, P;
        polyexp_sums(kind - FRGO_REG_POLYEXP, l2 / k2, &S, &P);
        return k2 * exp(-S);
    }
    double y = l2 / k2;
    if (y == 0.0) return k2;
    double e, E;
    exp_pair(y, &e, &E);
    return k2 * y * e / (-E);
}

double frgo_regulator_dot(int kind, double l2, double k) {
    double k2 = k * k;
    if (l2 < 0.0) l2 = 0.0;
    if (kind == FRGO_REG_LITIM) return (l2 < k2) ? 2.0 * k2 : 0.0;
    if (kind > FRGO_REG_POLYEXP && kind <= FRGO_REG_POLYEXP + 64) {
        double S, P;
        polyexp_sums(kind - FRGO_REG_POLYEXP, l2 / k2, &S, &P);
        return 2.0 * k2 * exp(-S) * (1.0 + P);
    }
    double y = l2 / k2;
    if (y == 0.0) return 2.0 * k2;
    double e, E;
    exp_pair(y, &e, &E);
    return 2.0 * k2 * y * y * e / (E * E);
}

/* ---------------------------------------------------------------------------------------- */
/* Dressing: linear interpolation in u = log|l| on a log-uniform grid, clamped at the ends.  */
/* ---------------------------------------------------------------------------------------- */
double frgo_dressing(const double *Z, int nZ, double x_min, double x_max, double l2) {
    if (Z == NULL) return 1.0;
    if (nZ == 1) return Z[0];
    double u = (l2 > 0.0) ? 0.5 * log(l2) : -INFINITY;
    double lmin = log(x_min), lmax = log(x_max);
    double delta = (lmax - lmin) / (double)(nZ - 1);
    double s = (u - lmin) / delta;
    if (!(s > 0.0)) s = 0.0; /* also catches -inf */
    if (s > (double)(nZ - 1)) s = (double)(nZ - 1);
    int i = (int)floor(s);
    if (i > nZ - 2) i = nZ - 2;
    double f = s - (double)i;
    return Z[i] + f * (Z[i + 1] - Z[i]);
}

double frgo_propagator(int reg, const double *Z, int nZ, double x_min, double x_max, double l2,
                       double m2, double k) {
    if (l2 < 0.0) l2 = 0.0;
    double z = frgo_dressing(Z, nZ, x_min, x_max, l2);
    return 1.0 / (z * l2 + frgo_regulator(reg, l2, k) + m2);
}

/* Threshold function of the flat regulator: l_n^d(w) = (2/d) (n + [n == 0]) / (1 + w)^(n + 1).
 * With R = (k^2 - q^2) Theta(k^2 - q^2) the radial integral over [0, k] of
 * q^(d-1) (2 k^2) / (k^2 + m^2)^m is 2 k^(d+2) / (d (k^2 + m^2)^m), which in units of k and
 * w = m^2/k^2 is J_m = (2/d) / (1 + w)^m; l_n^d = (n + [n == 0]) J_{n+1} is the conventional
 * normalisation (dl_n/dw = -(n + [n == 0]) l_{n+1}), and l_1^d is the LPA integral itself. */
double frgo_litim_threshold(int d, int n, double w) {
    double r = 1.0 / (1.0 + w);
    double p = r;
    for (int i = 0; i < n; ++i) p *= r;
    return (2.0 / (double)d) * (double)(n == 0 ? 1 : n) * p;
}

/* ---------------------------------------------------------------------------------------- */
/* Loop integrals.                                                                           */
/* ---------------------------------------------------------------------------------------- */
static double omega(int d) {
    /* surface of the unit sphere in d dimensions: 2 pi^(d/2) / Gamma(d/2) */
    return 2.0 * pow(PI, 0.5 * d) / tgamma(0.5 * d);
}

#define MAXN 4096

/* deriv = 1: the same sums with the product of propagators replaced by its derivative in m2,
 * each propagator G contributing dG/dm2 = -G^2 (product rule, written out per family). */
static int integrate_impl(int family, int d, int n_q, int n_x, int n_phi, double q_max, double k,
                          int regulator, const double *ext, const double *m2, double m2_scalar,
                          const double *Z, int nZ, double x_min, double x_max, int n_ext,
                          int deriv, double *out) {
    if (n_ext < 0 || out == NULL) return -1;
    if (n_q < 1 || n_q > MAXN || !(q_max > 0.0) || !(k > 0.0)) return -1;
    if (Z != NULL && (nZ < 1 || !(x_min > 0.0) || !(x_max > x_min))) return -1;
    if (family == FRGO_LPA) {
        if (d < 1) return -1;
    } else if (family == FRGO_TWO_POINT || family == FRGO_THREE_POINT) {
        if (d != 4 || n_x < 1 || n_x > MAXN || ext == NULL) return -1;
        if (family == FRGO_THREE_POINT && (n_phi < 1 || n_phi > MAXN)) return -1;
    } else {
        return -1;
    }

    static __thread double qn[MAXN], qw[MAXN], xn[MAXN], xw[MAXN], fn[MAXN], fw[MAXN];
    frgo_gauss_legendre(n_q, 0.0, q_max * k, qn, qw);
    if (family != FRGO_LPA) frgo_gauss_legendre(n_x, -1.0, 1.0, xn, xw);
    if (family == FRGO_THREE_POINT) frgo_gauss_legendre(n_phi, 0.0, PI, fn, fw);

    for (int e = 0; e < n_ext; ++e) {
        double mass = m2 ? m2[e] : m2_scalar;
        nsum total = {0.0, 0.0};
        if (family == FRGO_LPA) {
            double pref = omega(d) / pow(2.0 * PI, (double)d);
            for (int a = 0; a < n_q; ++a) {
                double q = qn[a], q2 = q * q;
                double den = q2 + frgo_regulator(regulator, q2, k) + mass;
                double term = pref * qw[a] * pow(q, (double)(d - 1)) *
                              frgo_regulator_dot(regulator, q2, k) / (den * den);
                if (deriv) term *= -2.0 / den;
                nsum_add(&total, term);
            }
        } else if (family == FRGO_TWO_POINT) {
            double p = ext[e];
            double pref = 4.0 * PI / pow(2.0 * PI, 4.0);
            for (int a = 0; a < n_q; ++a) {
                nsum inner = {0.0, 0.0};
                double q = qn[a], q2 = q * q;
                for (int b = 0; b < n_x; ++b) {
                    double x = xn[b];
                    double l2 = q2 + p * p + 2.0 * q * p * x;
                    double gq = frgo_propagator(regulator, Z, nZ, x_min, x_max, q2, mass, k);
                    double gl = frgo_propagator(regulator, Z, nZ, x_min, x_max, l2, mass, k);
                    double term = pref * qw[a] * xw[b] * sqrt(1.0 - x * x) * q2 * q *
                                  frgo_regulator_dot(regulator, q2, k) * gq * gq * gl;
                    if (deriv)
                        term = pref * qw[a] * xw[b] * sqrt(1.0 - x * x) * q2 * q *
                               frgo_regulator_dot(regulator, q2, k) *
                               (-2.0 * gq * gq * gq * gl - gq * gq * gl * gl);
                    nsum_add(&inner, term);
                }
                nsum_add(&total, nsum_get(&inner));
            }
        } else {
            double p = ext[e], alpha = ext[n_ext + e];
            double ca = cos(alpha), sa = sin(alpha);
            double pref = 2.0 * PI / pow(2.0 * PI, 4.0);
            for (int a = 0; a < n_q; ++a) {
                nsum mid = {0.0, 0.0};
                double q = qn[a], q2 = q * q;
                for (int b = 0; b < n_x; ++b) {
                    nsum inner = {0.0, 0.0};
                    double x = xn[b], sx = sqrt(1.0 - x * x);
                    for (int c = 0; c < n_phi; ++c) {
                        double phi = fn[c];
                        double l1 = q2 + p * p + 2.0 * q * p * x;
                        double l2 = q2 + p * p - 2.0 * q * p * (x * ca + sx * cos(phi) * sa);
                        double gq = frgo_propagator(regulator, Z, nZ, x_min, x_max, q2, mass, k);
                        double g1 = frgo_propagator(regulator, Z, nZ, x_min, x_max, l1, mass, k);
                        double g2 = frgo_propagator(regulator, Z, nZ, x_min, x_max, l2, mass, k);
                        double term = pref * qw[a] * xw[b] * fw[c] * sx * sin(phi) * q2 * q *
                                      frgo_regulator_dot(regulator, q2, k) * gq * gq * g1 * g2;
                        if (deriv)
                            term = pref * qw[a] * xw[b] * fw[c] * sx * sin(phi) * q2 * q *
                                   frgo_regulator_dot(regulator, q2, k) *
                                   (-2.0 * gq * gq * gq * g1 * g2 - gq * gq * g1 * g1 * g2 -
                                    gq * gq * g1 * g2 * g2);
                        nsum_add(&inner, term);
                    }
                    nsum_add(&mid, nsum_get(&inner));
                }
                nsum_add(&total, nsum_get(&mid));
            }
        }
        out[e] = nsum_get(&total);
    }
    return 0;
}

int frgo_integrate(int family, int d, int n_q, int n_x, int n_phi, double q_max, double k,
                   int regulator, const double *ext, const double *m2, double m2_scalar,
                   const double *Z, int nZ, double x_min, double x_max, int n_ext, double *out) {
    return integrate_impl(family, d, n_q, n_x, n_phi, q_max, k, regulator, ext, m2, m2_scalar, Z,
                          nZ, x_min, x_max, n_ext, 0, out);
}

int frgo_integrate_dm2(int family, int d, int n_q, int n_x, int n_phi, double q_max, double k,
                       int regulator, const double *ext, const double *m2, double m2_scalar,
                       const double *Z, int nZ, double x_min, double x_max, int n_ext,
                       double *out) {
    return integrate_impl(family, d, n_q, n_x, n_phi, q_max, k, regulator, ext, m2, m2_scalar, Z,
                          nZ, x_min, x_max, n_ext, 1, out);
}

/* Cell and fraction of the dressing's interpolation at l2 (the same clamping as frgo_dressing):
 * Z(l2) = (1 - f) Z_i + f Z_{i+1} for nZ >= 2; nZ == 1 gives i = 0, f = 0 (Z(l2) = Z_0). */
static void dressing_cell(int nZ, double x_min, double x_max, double l2, int *i, double *f) {
    *i = 0;
    *f = 0.0;
    if (nZ == 1) return;
    double u = (l2 > 0.0) ? 0.5 * log(l2) : -INFINITY;
    double lmin = log(x_min), lmax = log(x_max);
    double delta = (lmax - lmin) / (double)(nZ - 1);
    double s = (u - lmin) / delta;
    if (!(s > 0.0)) s = 0.0;
    if (s > (double)(nZ - 1)) s = (double)(nZ - 1);
    int c = (int)floor(s);
    if (c > nZ - 2) c = nZ - 2;
    *i = c;
    *f = s - (double)c;
}

/* Adds v * dZ(l2)/dZ_i to acc[i] for every table entry i: (1 - f) v to the cell's first entry
 * and f v to its second. */
static void add_dressing_weights(nsum *acc, int nZ, int i, double f, double v) {
    nsum_add(&acc[i], (1.0 - f) * v);
    if (nZ > 1) nsum_add(&acc[i + 1], f * v);
}

int frgo_integrate_dz(int d, int n_q, int n_x, double q_max, double k, int regulator,
                      const double *ext, const double *m2, double m2_scalar, const double *Z,
                      int nZ, double x_min, double x_max, int n_ext, double *out) {
    if (n_ext < 0 || out == NULL || ext == NULL || Z == NULL || nZ < 1 || nZ > MAXN) return -1;
    if (d != 4 || n_q < 1 || n_q > MAXN || n_x < 1 || n_x > MAXN) return -1;
    if (!(q_max > 0.0) || !(k > 0.0) || !(x_min > 0.0) || !(x_max > x_min)) return -1;
    static __thread double qn[MAXN], qw[MAXN], xn[MAXN], xw[MAXN];
    static __thread nsum acc[MAXN];
    frgo_gauss_legendre(n_q, 0.0, q_max * k, qn, qw);
    frgo_gauss_legendre(n_x, -1.0, 1.0, xn, xw);
    double pref = 4.0 * PI / pow(2.0 * PI, 4.0);
    for (int e = 0; e < n_ext; ++e) {
        double p = ext[e];
        double mass = m2 ? m2[e] : m2_scalar;
        for (int i = 0; i < nZ; ++i) acc[i].s = acc[i].c = 0.0;
        for (int a = 0; a < n_q; ++a) {
            double q = qn[a], q2 = q * q;
            double gq = frgo_propagator(regulator, Z, nZ, x_min, x_max, q2, mass, k);
            int iq;
            double fq;
            dressing_cell(nZ, x_min, x_max, q2, &iq, &fq);
            for (int b = 0; b < n_x; ++b) {
                double x = xn[b];
                double l2 = q2 + p * p + 2.0 * q * p * x;
                if (l2 < 0.0) l2 = 0.0; /* the propagator's own clamp */
                double gl = frgo_propagator(regulator, Z, nZ, x_min, x_max, l2, mass, k);
                double c = pref * qw[a] * xw[b] * sqrt(1.0 - x * x) * q2 * q *
                           frgo_regulator_dot(regulator, q2, k);
                /* term = c G(q^2)^2 G(l2); dG(v)/dZ_i = -G(v)^2 v dZ(v)/dZ_i */
                add_dressing_weights(acc, nZ, iq, fq, -2.0 * c * gq * gq * gq * q2 * gl);
                int il;
                double fl;
                dressing_cell(nZ, x_min, x_max, l2, &il, &fl);
                add_dressing_weights(acc, nZ, il, fl, -c * gq * gq * gl * gl * l2);
            }
        }
        for (int i = 0; i < nZ; ++i) out[(size_t)e * nZ + i] = nsum_get(&acc[i]);
    }
    return 0;
}

int frgo_integrate_dz_three(int n_q, int n_x, int n_phi, double q_max, double k, int regulator,
                            const double *ext, const double *m2, double m2_scalar,
                            const double *Z, int nZ, double x_min, double x_max, int n_ext,
                            double *out) {
    if (n_ext < 0 || out == NULL || ext == NULL || Z == NULL || nZ < 1 || nZ > MAXN) return -1;
    if (n_q < 1 || n_q > MAXN || n_x < 1 || n_x > MAXN || n_phi < 1 || n_phi > MAXN) return -1;
    if (!(q_max > 0.0) || !(k > 0.0) || !(x_min > 0.0) || !(x_max > x_min)) return -1;
    static __thread double qn[MAXN], qw[MAXN], xn[MAXN], xw[MAXN], fn[MAXN], fw[MAXN];
    static __thread nsum acc[MAXN];
    frgo_gauss_legendre(n_q, 0.0, q_max * k, qn, qw);
    frgo_gauss_legendre(n_x, -1.0, 1.0, xn, xw);
    frgo_gauss_legendre(n_phi, 0.0, PI, fn, fw);
    double pref = 2.0 * PI / pow(2.0 * PI, 4.0);
    for (int e = 0; e < n_ext; ++e) {
        double p = ext[e], alpha = ext[n_ext + e];
        double ca = cos(alpha), sa = sin(alpha);
        double mass = m2 ? m2[e] : m2_scalar;
        for (int i = 0; i < nZ; ++i) acc[i].s = acc[i].c = 0.0;
        for (int a = 0; a < n_q; ++a) {
            double q = qn[a], q2 = q * q;
            double gq = frgo_propagator(regulator, Z, nZ, x_min, x_max, q2, mass, k);
            int iq;
            double fq;
            dressing_cell(nZ, x_min, x_max, q2, &iq, &fq);
            for (int b = 0; b < n_x; ++b) {
                double x = xn[b], sx = sqrt(1.0 - x * x);
                double l1 = q2 + p * p + 2.0 * q * p * x;
                if (l1 < 0.0) l1 = 0.0;
                double g1 = frgo_propagator(regulator, Z, nZ, x_min, x_max, l1, mass, k);
                int i1;
                double f1;
                dressing_cell(nZ, x_min, x_max, l1, &i1, &f1);
                for (int c = 0; c < n_phi; ++c) {
                    double phi = fn[c];
                    double l2 = q2 + p * p - 2.0 * q * p * (x * ca + sx * cos(phi) * sa);
                    if (l2 < 0.0) l2 = 0.0;
                    double g2 = frgo_propagator(regulator, Z, nZ, x_min, x_max, l2, mass, k);
                    double cw = pref * qw[a] * xw[b] * fw[c] * sx * sin(phi) * q2 * q *
                                frgo_regulator_dot(regulator, q2, k);
                    /* term = cw G(q^2)^2 G(l1) G(l2) */
                    add_dressing_weights(acc, nZ, iq, fq, -2.0 * cw * gq * gq * gq * q2 * g1 * g2);
                    add_dressing_weights(acc, nZ, i1, f1, -cw * gq * gq * g1 * g1 * l1 * g2);
                    int i2;
                    double f2;
                    dressing_cell(nZ, x_min, x_max, l2, &i2, &f2);
                    add_dressing_weights(acc, nZ, i2, f2, -cw * gq * gq * g1 * g2 * g2 * l2);
                }
            }
        }
        for (int i = 0; i < nZ; ++i) out[(size_t)e * nZ + i] = nsum_get(&acc[i]);
    }
    return 0;
}

/* ---------------------------------------------------------------------------------------- */
/* Finite temperature: Matsubara frequency rule and the d = 3 + 1 integrals.                 */
/* ---------------------------------------------------------------------------------------- */
int frgo_matsubara_rule(int statistics, double T, double lambda, int n_tail, int cap, double *w,
                        double *c) {
    if ((statistics != FRGO_BOSONIC && statistics != FRGO_FERMIONIC) || !(T > 0.0) ||
        !(lambda > 0.0) || n_tail < 0 || w == NULL || c == NULL)
        return -1;
    double eta = statistics == FRGO_FERMIONIC ? 0.5 : 0.0;
    /* largest n >= 0 with 2 pi T (n + eta) <= lambda */
    double nh = floor(lambda / (2.0 * PI * T) - eta);
    if (nh < 0.0) return -1;
    if (nh > 1e6) return -2;
    int n_hi = (int)nh;
    int n_lo = statistics == FRGO_FERMIONIC ? -n_hi - 1 : -n_hi; /* symmetric set */
    int n_exp = n_hi - n_lo + 1;
    int total = n_exp + 2 * n_tail;
    if (total > cap) return -2;
    double Omega = 2.0 * PI * T * ((double)n_hi + eta) + PI * T;
    static __thread double tn[MAXN], tw[MAXN];
    if (n_tail > 0) {
        if (n_tail > MAXN) return -2;
        frgo_gauss_legendre(n_tail, 0.0, 1.0, tn, tw);
    }
    int j = 0;
    /* negative tail, ascending w = -Omega/t: t ascending */
    for (int i = 0; i < n_tail; ++i) {
        w[j] = -Omega / tn[i];
        c[j] = Omega * tw[i] / (tn[i] * tn[i]) / (2.0 * PI);
        ++j;
    }
    for (int n = n_lo; n <= n_hi; ++n) {
        w[j] = 2.0 * PI * T * ((double)n + eta);
        c[j] = T;
        ++j;
    }
    /* positive tail, ascending w = Omega/t: t descending */
    for (int i = n_tail - 1; i >= 0; --i) {
        w[j] = Omega / tn[i];
        c[j] = Omega * tw[i] / (tn[i] * tn[i]) / (2.0 * PI);
        ++j;
    }
    return total;
}

static int integrate_ft_impl(int family, int n_q, int n_x, double q_max, double k, int regulator,
                             int statistics, double T, double freq_max, int freq_scaled,
                             int n_tail, const double *ext, const double *m2, double m2_scalar,
                             const double *Z, int nZ, double x_min, double x_max, int n_ext,
                             int deriv, double *out) {
    if (n_ext < 0 || out == NULL) return -1;
    if (n_q < 1 || n_q > MAXN || !(q_max > 0.0) || !(k > 0.0)) return -1;
    if (family != FRGO_LPA_T && family != FRGO_TWO_POINT_T) return -1;
    if (family == FRGO_TWO_POINT_T && (n_x < 1 || n_x > MAXN || ext == NULL)) return -1;
    if (Z != NULL && (nZ < 1 || !(x_min > 0.0) || !(x_max > x_min))) return -1;
    static __thread double qn[MAXN], qw[MAXN], xn[MAXN], xw[MAXN], fw_[MAXN], fc_[MAXN];
    double lambda = freq_scaled ? freq_max * k : freq_max;
    int n_f = frgo_matsubara_rule(statistics, T, lambda, n_tail, MAXN, fw_, fc_);
    if (n_f < 0) return -1;
    frgo_gauss_legendre(n_q, 0.0, q_max * k, qn, qw);
    if (family == FRGO_TWO_POINT_T) frgo_gauss_legendre(n_x, -1.0, 1.0, xn, xw);
    for (int e = 0; e < n_ext; ++e) {
        double mass = m2 ? m2[e] : m2_scalar;
        nsum total = {0.0, 0.0};
        if (family == FRGO_LPA_T) {
            double pref = 4.0 * PI / pow(2.0 * PI, 3.0);
            for (int j = 0; j < n_f; ++j) {
                for (int a = 0; a < n_q; ++a) {
                    double q = qn[a], q2 = q * q;
                    double den = fw_[j] * fw_[j] + q2 + frgo_regulator(regulator, q2, k) + mass;
                    double term = fc_[j] * pref * qw[a] * q2 *
                                  frgo_regulator_dot(regulator, q2, k) / (den * den);
                    if (deriv) term *= -2.0 / den;
                    nsum_add(&total, term);
                }
            }
        } else {
            double p = ext[e], p0 = ext[n_ext + e];
            double pref = 2.0 * PI / pow(2.0 * PI, 3.0);
            for (int j = 0; j < n_f; ++j) {
                double wq = fw_[j], wl = fw_[j] + p0;
                for (int a = 0; a < n_q; ++a) {
                    nsum inner = {0.0, 0.0};
                    double q = qn[a], q2 = q * q;
                    for (int b = 0; b < n_x; ++b) {
                        double l2 = q2 + p * p + 2.0 * q * p * xn[b];
                        if (l2 < 0.0) l2 = 0.0;
                        double gq = 1.0 / (wq * wq + frgo_dressing(Z, nZ, x_min, x_max, q2) * q2 +
                                           frgo_regulator(regulator, q2, k) + mass);
                        double gl = 1.0 / (wl * wl + frgo_dressing(Z, nZ, x_min, x_max, l2) * l2 +
                                           frgo_regulator(regulator, l2, k) + mass);
                        double term = fc_[j] * pref * qw[a] * xw[b] * q2 *
                                      frgo_regulator_dot(regulator, q2, k) * gq * gq * gl;
                        if (deriv)
                            term = fc_[j] * pref * qw[a] * xw[b] * q2 *
                                   frgo_regulator_dot(regulator, q2, k) *
                                   (-2.0 * gq * gq * gq * gl - gq * gq * gl * gl);
                        nsum_add(&inner, term);
                    }
                    nsum_add(&total, nsum_get(&inner));
                }
            }
        }
        out[e] = nsum_get(&total);
    }
    return 0;
}

int frgo_integrate_ft_dz(int n_q, int n_x, double q_max, double k, int regulator, int statistics,
                         double T, double freq_max, int freq_scaled, int n_tail,
                         const double *ext, const double *m2, double m2_scalar, const double *Z,
                         int nZ, double x_min, double x_max, int n_ext, double *out) {
    if (n_ext < 0 || out == NULL || ext == NULL || Z == NULL || nZ < 1 || nZ > MAXN) return -1;
    if (n_q < 1 || n_q > MAXN || n_x < 1 || n_x > MAXN) return -1;
    if (!(q_max > 0.0) || !(k > 0.0) || !(x_min > 0.0) || !(x_max > x_min)) return -1;
    static __thread double qn[MAXN], qw[MAXN], xn[MAXN], xw[MAXN], fw_[MAXN], fc_[MAXN];
    static __thread nsum acc[MAXN];
    double lambda = freq_scaled ? freq_max * k : freq_max;
    int n_f = frgo_matsubara_rule(statistics, T, lambda, n_tail, MAXN, fw_, fc_);
    if (n_f < 0) return -1;
    frgo_gauss_legendre(n_q, 0.0, q_max * k, qn, qw);
    frgo_gauss_legendre(n_x, -1.0, 1.0, xn, xw);
    double pref = 2.0 * PI / pow(2.0 * PI, 3.0);
    for (int e = 0; e < n_ext; ++e) {
        double p = ext[e], p0 = ext[n_ext + e];
        double mass = m2 ? m2[e] : m2_scalar;
        for (int i = 0; i < nZ; ++i) acc[i].s = acc[i].c = 0.0;
        for (int j = 0; j < n_f; ++j) {
            double wq = fw_[j], wl = fw_[j] + p0;
            for (int a = 0; a < n_q; ++a) {
                double q = qn[a], q2 = q * q;
                int iq;
                double fq;
                dressing_cell(nZ, x_min, x_max, q2, &iq, &fq);
                for (int b = 0; b < n_x; ++b) {
                    double l2 = q2 + p * p + 2.0 * q * p * xn[b];
                    if (l2 < 0.0) l2 = 0.0;
                    double gq = 1.0 / (wq * wq + frgo_dressing(Z, nZ, x_min, x_max, q2) * q2 +
                                       frgo_regulator(regulator, q2, k) + mass);
                    double gl = 1.0 / (wl * wl + frgo_dressing(Z, nZ, x_min, x_max, l2) * l2 +
                                       frgo_regulator(regulator, l2, k) + mass);
                    double c = fc_[j] * pref * qw[a] * xw[b] * q2 *
                               frgo_regulator_dot(regulator, q2, k);
                    /* term = c G(q^2)^2 G(l2): the dressing multiplies the spatial momentum */
                    add_dressing_weights(acc, nZ, iq, fq, -2.0 * c * gq * gq * gq * q2 * gl);
                    int il;
                    double fl;
                    dressing_cell(nZ, x_min, x_max, l2, &il, &fl);
                    add_dressing_weights(acc, nZ, il, fl, -c * gq * gq * gl * gl * l2);
                }
            }
        }
        for (int i = 0; i < nZ; ++i) out[(size_t)e * nZ + i] = nsum_get(&acc[i]);
    }
    return 0;
}

int frgo_integrate_ft(int family, int n_q, int n_x, double q_max, double k, int regulator,
                      int statistics, double T, double freq_max, int freq_scaled, int n_tail,
                      const double *ext, const double *m2, double m2_scalar, const double *Z,
                      int nZ, double x_min, double x_max, int n_ext, double *out) {
    return integrate_ft_impl(family, n_q, n_x, q_max, k, regulator, statistics, T, freq_max,
                             freq_scaled, n_tail, ext, m2, m2_scalar, Z, nZ, x_min, x_max, n_ext,
                             0, out);
}

int frgo_integrate_ft_dm2(int family, int n_q, int n_x, double q_max, double k, int regulator,
                          int statistics, double T, double freq_max, int freq_scaled, int n_tail,
                          const double *ext, const double *m2, double m2_scalar, const double *Z,
                          int nZ, double x_min, double x_max, int n_ext, double *out) {
    return integrate_ft_impl(family, n_q, n_x, q_max, k, regulator, statistics, T, freq_max,
                             freq_scaled, n_tail, ext, m2, m2_scalar, Z, nZ, x_min, x_max, n_ext,
                             1, out);
}

/* ---------------------------------------------------------------------------------------- */
/* Three-point at finite temperature (family 6).                                            */
/* ---------------------------------------------------------------------------------------- */
static double ft_prop(int regulator, const double *Z, int nZ, double x_min, double x_max,
                      double l2, double w, double m2, double k) {
    return 1.0 / (w * w + frgo_dressing(Z, nZ, x_min, x_max, l2) * l2 +
                  frgo_regulator(regulator, l2, k) + m2);
}

int frgo_integrate_ft_three(int n_q, int n_x, int n_phi, double q_max, double k, int regulator,
                            int statistics, double T, double freq_max, int freq_scaled,
                            int n_tail, const double *ext, const double *m2, double m2_scalar,
                            const double *Z, int nZ, double x_min, double x_max, int n_ext,
                            int deriv, double *out) {
    if (n_ext < 0 || out == NULL || ext == NULL) return -1;
    if (n_q < 1 || n_q > MAXN || n_x < 1 || n_x > MAXN || n_phi < 1 || n_phi > MAXN) return -1;
    if (!(q_max > 0.0) || !(k > 0.0)) return -1;
    if (Z != NULL && (nZ < 1 || !(x_min > 0.0) || !(x_max > x_min))) return -1;
    static __thread double qn[MAXN], qw[MAXN], xn[MAXN], xw[MAXN], fn[MAXN], fw[MAXN],
        mw[MAXN], mc[MAXN];
    double lambda = freq_scaled ? freq_max * k : freq_max;
    int n_f = frgo_matsubara_rule(statistics, T, lambda, n_tail, MAXN, mw, mc);
    if (n_f < 0) return -1;
    frgo_gauss_legendre(n_q, 0.0, q_max * k, qn, qw);
    frgo_gauss_legendre(n_x, -1.0, 1.0, xn, xw);
    frgo_gauss_legendre(n_phi, 0.0, PI, fn, fw);
    double pref = 2.0 / pow(2.0 * PI, 3.0);  /* the azimuth folded onto [0, pi] */
    for (int e = 0; e < n_ext; ++e) {
        double p = ext[e], alpha = ext[n_ext + e], p01 = ext[2 * n_ext + e],
               p02 = ext[3 * n_ext + e];
        double ca = cos(alpha), sa = sin(alpha);
        double mass = m2 ? m2[e] : m2_scalar;
        nsum total = {0.0, 0.0};
        for (int j = 0; j < n_f; ++j) {
            double w = mw[j];
            for (int a = 0; a < n_q; ++a) {
                double q = qn[a], q2 = q * q;
                double gq = ft_prop(regulator, Z, nZ, x_min, x_max, q2, w, mass, k);
                double rad = mc[j] * pref * qw[a] * q2 * frgo_regulator_dot(regulator, q2, k);
                nsum mid = {0.0, 0.0};
                for (int b = 0; b < n_x; ++b) {
                    double x = xn[b], sx = sqrt(1.0 - x * x);
                    double l1 = q2 + p * p + 2.0 * q * p * x;
                    if (l1 < 0.0) l1 = 0.0;
                    double g1 = ft_prop(regulator, Z, nZ, x_min, x_max, l1, w + p01, mass, k);
                    nsum inner = {0.0, 0.0};
                    for (int c = 0; c < n_phi; ++c) {
                        double l2 = q2 + p * p - 2.0 * q * p * (x * ca + sx * cos(fn[c]) * sa);
                        if (l2 < 0.0) l2 = 0.0;
                        double g2 = ft_prop(regulator, Z, nZ, x_min, x_max, l2, w + p02, mass, k);
                        double term = rad * xw[b] * fw[c] * gq * gq * g1 * g2;
                        if (deriv)
                            term = rad * xw[b] * fw[c] *
                                   (-2.0 * gq * gq * gq * g1 * g2 - gq * gq * g1 * g1 * g2 -
                                    gq * gq * g1 * g2 * g2);
                        nsum_add(&inner, term);
                    }
                    nsum_add(&mid, nsum_get(&inner));
                }
                nsum_add(&total, nsum_get(&mid));
            }
        }
        out[e] = nsum_get(&total);
    }
    return 0;
}

int frgo_integrate_ft_three_dz(int n_q, int n_x, int n_phi, double q_max, double k,
                               int regulator, int statistics, double T, double freq_max,
                               int freq_scaled, int n_tail, const double *ext, const double *m2,
                               double m2_scalar, const double *Z, int nZ, double x_min,
                               double x_max, int n_ext, double *out) {
    if (n_ext < 0 || out == NULL || ext == NULL || Z == NULL || nZ < 1 || nZ > MAXN) return -1;
    if (n_q < 1 || n_q > MAXN || n_x < 1 || n_x > MAXN || n_phi < 1 || n_phi > MAXN) return -1;
    if (!(q_max > 0.0) || !(k > 0.0) || !(x_min > 0.0) || !(x_max > x_min)) return -1;
    static __thread double qn[MAXN], qw[MAXN], xn[MAXN], xw[MAXN], fn[MAXN], fw[MAXN],
        mw[MAXN], mc[MAXN];
    static __thread nsum acc[MAXN];
    double lambda = freq_scaled ? freq_max * k : freq_max;
    int n_f = frgo_matsubara_rule(statistics, T, lambda, n_tail, MAXN, mw, mc);
    if (n_f < 0) return -1;
    frgo_gauss_legendre(n_q, 0.0, q_max * k, qn, qw);
    frgo_gauss_legendre(n_x, -1.0, 1.0, xn, xw);
    frgo_gauss_legendre(n_phi, 0.0, PI, fn, fw);
    double pref = 2.0 / pow(2.0 * PI, 3.0);
    for (int e = 0; e < n_ext; ++e) {
        double p = ext[e], alpha = ext[n_ext + e], p01 = ext[2 * n_ext + e],
               p02 = ext[3 * n_ext + e];
        double ca = cos(alpha), sa = sin(alpha);
        double mass = m2 ? m2[e] : m2_scalar;
        for (int i = 0; i < nZ; ++i) acc[i].s = acc[i].c = 0.0;
        for (int j = 0; j < n_f; ++j) {
            double w = mw[j];
            for (int a = 0; a < n_q; ++a) {
                double q = qn[a], q2 = q * q;
                double gq = ft_prop(regulator, Z, nZ, x_min, x_max, q2, w, mass, k);
                int iq;
                double fq;
                dressing_cell(nZ, x_min, x_max, q2, &iq, &fq);
                for (int b = 0; b < n_x; ++b) {
                    double x = xn[b], sx = sqrt(1.0 - x * x);
                    double l1 = q2 + p * p + 2.0 * q * p * x;
                    if (l1 < 0.0) l1 = 0.0;
                    double g1 = ft_prop(regulator, Z, nZ, x_min, x_max, l1, w + p01, mass, k);
                    int i1;
                    double f1;
                    dressing_cell(nZ, x_min, x_max, l1, &i1, &f1);
                    for (int c = 0; c < n_phi; ++c) {
                        double l2 = q2 + p * p - 2.0 * q * p * (x * ca + sx * cos(fn[c]) * sa);
                        if (l2 < 0.0) l2 = 0.0;
                        double g2 = ft_prop(regulator, Z, nZ, x_min, x_max, l2, w + p02, mass, k);
                        double cw = mc[j] * pref * qw[a] * xw[b] * fw[c] * q2 *
                                    frgo_regulator_dot(regulator, q2, k);
                        /* term = cw G(q^2)^2 G(l1) G(l2); dG(v)/dZ_i = -G(v)^2 v w_i(v) */
                        add_dressing_weights(acc, nZ, iq, fq,
                                             -2.0 * cw * gq * gq * gq * q2 * g1 * g2);
                        add_dressing_weights(acc, nZ, i1, f1, -cw * gq * gq * g1 * g1 * l1 * g2);
                        int i2;
                        double f2;
                        dressing_cell(nZ, x_min, x_max, l2, &i2, &f2);
                        add_dressing_weights(acc, nZ, i2, f2, -cw * gq * gq * g1 * g2 * g2 * l2);
                    }
                }
            }
        }
        for (int i = 0; i < nZ; ++i) out[(size_t)e * nZ + i] = nsum_get(&acc[i]);
    }
    return 0;
}

/* ---------------------------------------------------------------------------------------- */
/* Complex external frequencies of the inner legs (families 5 and 6).                        */
/* ---------------------------------------------------------------------------------------- */
static double complex ft_prop_c(int regulator, const double *Z, int nZ, double x_min,
                                double x_max, double l2, double complex w, double m2, double k) {
    return 1.0 / (w * w + frgo_dressing(Z, nZ, x_min, x_max, l2) * l2 +
                  frgo_regulator(regulator, l2, k) + m2);
}

int frgo_integrate_ft_complex(int family, int n_q, int n_x, int n_phi, double q_max, double k,
                              int regulator, int statistics, double T, double freq_max,
                              int freq_scaled, int n_tail, const double *ext, const double *m2,
                              double m2_scalar, const double *Z, int nZ, double x_min,
                              double x_max, int n_ext, double *out) {
    if (n_ext < 0 || out == NULL || ext == NULL) return -1;
    if (family != FRGO_TWO_POINT_T && family != FRGO_THREE_POINT_T) return -1;
    if (n_q < 1 || n_q > MAXN || n_x < 1 || n_x > MAXN) return -1;
    if (family == FRGO_THREE_POINT_T && (n_phi < 1 || n_phi > MAXN)) return -1;
    if (!(q_max > 0.0) || !(k > 0.0)) return -1;
    if (Z != NULL && (nZ < 1 || !(x_min > 0.0) || !(x_max > x_min))) return -1;
    static __thread double qn[MAXN], qw[MAXN], xn[MAXN], xw[MAXN], fn[MAXN], fw[MAXN],
        mw[MAXN], mc[MAXN];
    double lambda = freq_scaled ? freq_max * k : freq_max;
    int n_f = frgo_matsubara_rule(statistics, T, lambda, n_tail, MAXN, mw, mc);
    if (n_f < 0) return -1;
    frgo_gauss_legendre(n_q, 0.0, q_max * k, qn, qw);
    frgo_gauss_legendre(n_x, -1.0, 1.0, xn, xw);
    int three = family == FRGO_THREE_POINT_T;
    if (three) frgo_gauss_legendre(n_phi, 0.0, PI, fn, fw);
    /* int d^3q/(2pi)^3: 2pi int q^2 dq dx (two-point), 2 int q^2 dq dx dphi, phi on [0, pi] */
    double pref = (three ? 2.0 : 2.0 * PI) / pow(2.0 * PI, 3.0);
    for (int e = 0; e < n_ext; ++e) {
        double p = ext[e];
        double ca = 1.0, sa = 0.0;
        double complex s1, s2 = 0.0;
        if (three) {
            ca = cos(ext[n_ext + e]);
            sa = sin(ext[n_ext + e]);
            s1 = ext[2 * n_ext + e] + ext[4 * n_ext + e] * _Complex_I;
            s2 = ext[3 * n_ext + e] + ext[5 * n_ext + e] * _Complex_I;
        } else {
            s1 = ext[n_ext + e] + ext[2 * n_ext + e] * _Complex_I;
        }
        double mass = m2 ? m2[e] : m2_scalar;
        nsum tre = {0.0, 0.0}, tim = {0.0, 0.0};
        for (int j = 0; j < n_f; ++j) {
            double w = mw[j];
            for (int a = 0; a < n_q; ++a) {
                double q = qn[a], q2 = q * q;
                double gq = ft_prop(regulator, Z, nZ, x_min, x_max, q2, w, mass, k);
                double rad = mc[j] * pref * qw[a] * q2 * frgo_regulator_dot(regulator, q2, k) *
                             gq * gq;
                nsum mre = {0.0, 0.0}, mim = {0.0, 0.0};
                for (int b = 0; b < n_x; ++b) {
                    double x = xn[b], sx = sqrt(1.0 - x * x);
                    double l1 = q2 + p * p + 2.0 * q * p * x;
                    if (l1 < 0.0) l1 = 0.0;
                    double complex h1 = ft_prop_c(regulator, Z, nZ, x_min, x_max, l1, w + s1,
                                                  mass, k);
                    if (!three) {
                        double complex term = rad * xw[b] * h1;
                        nsum_add(&mre, creal(term));
                        nsum_add(&mim, cimag(term));
                        continue;
                    }
                    for (int c = 0; c < n_phi; ++c) {
                        double l2 = q2 + p * p - 2.0 * q * p * (x * ca + sx * cos(fn[c]) * sa);
                        if (l2 < 0.0) l2 = 0.0;
                        double complex h2 = ft_prop_c(regulator, Z, nZ, x_min, x_max, l2,
                                                      w + s2, mass, k);
                        double complex term = rad * xw[b] * fw[c] * h1 * h2;
                        nsum_add(&mre, creal(term));
                        nsum_add(&mim, cimag(term));
                    }
                }
                nsum_add(&tre, nsum_get(&mre));
                nsum_add(&tim, nsum_get(&mim));
            }
        }
        out[e] = nsum_get(&tre);
        out[n_ext + e] = nsum_get(&tim);
    }
    return 0;
}

int frgo_vertex_ft_spherical(int n_q, int n_t1, int n_t2, double q_max, double k, int regulator,
                             int statistics, double T, double freq_max, int freq_scaled,
                             int n_tail, const double p1[3], const double p2[3], double p01,
                             double p02, double m2, const double *Z, int nZ, double x_min,
                             double x_max, double *out) {
    if (n_q < 1 || n_t1 < 1 || n_t2 < 1 || n_q > MAXN || n_t1 > MAXN || n_t2 > MAXN) return -1;
    if (out == NULL || p1 == NULL || p2 == NULL || !(q_max > 0.0) || !(k > 0.0)) return -1;
    static __thread double qn[MAXN], qw[MAXN], t1n[MAXN], t1w[MAXN], t2n[MAXN], t2w[MAXN],
        mw[MAXN], mc[MAXN];
    double lambda = freq_scaled ? freq_max * k : freq_max;
    int n_f = frgo_matsubara_rule(statistics, T, lambda, n_tail, MAXN, mw, mc);
    if (n_f < 0) return -1;
    frgo_gauss_legendre(n_q, 0.0, q_max * k, qn, qw);
    frgo_gauss_legendre(n_t1, 0.0, PI, t1n, t1w);
    frgo_gauss_legendre(n_t2, 0.0, 2.0 * PI, t2n, t2w);
    double pref = 1.0 / pow(2.0 * PI, 3.0);
    nsum total = {0.0, 0.0};
    for (int j = 0; j < n_f; ++j) {
        double w = mw[j];
        for (int a = 0; a < n_q; ++a) {
            double q = qn[a], q2 = q * q;
            double gq = ft_prop(regulator, Z, nZ, x_min, x_max, q2, w, m2, k);
            double rad = mc[j] * pref * qw[a] * q2 * frgo_regulator_dot(regulator, q2, k) * gq * gq;
            nsum s1 = {0.0, 0.0};
            for (int i = 0; i < n_t1; ++i) {
                double t1 = t1n[i];
                nsum s2 = {0.0, 0.0};
                for (int c = 0; c < n_t2; ++c) {
                    double t2 = t2n[c];
                    double v[3] = {q * cos(t1), q * sin(t1) * cos(t2), q * sin(t1) * sin(t2)};
                    double a1 = 0.0, a2 = 0.0;
                    for (int m = 0; m < 3; ++m) {
                        a1 += (v[m] + p1[m]) * (v[m] + p1[m]);
                        a2 += (v[m] - p2[m]) * (v[m] - p2[m]);
                    }
                    double g1 = ft_prop(regulator, Z, nZ, x_min, x_max, a1, w + p01, m2, k);
                    double g2 = ft_prop(regulator, Z, nZ, x_min, x_max, a2, w + p02, m2, k);
                    nsum_add(&s2, t2w[c] * g1 * g2);
                }
                nsum_add(&s1, t1w[i] * sin(t1) * nsum_get(&s2));
            }
            nsum_add(&total, rad * nsum_get(&s1));
        }
    }
    out[0] = nsum_get(&total);
    return 0;
}

/* ---------------------------------------------------------------------------------------- */
/* Hyperspherical reference rule (rotation-invariance pin).                                  */
/* q = |q| (cos t1, sin t1 cos t2, sin t1 sin t2 cos t3, sin t1 sin t2 sin t3),              */
/* d^4q = q^3 sin^2 t1 sin t2 dq dt1 dt2 dt3.                                                */
/* ---------------------------------------------------------------------------------------- */
static double dot4(const double *a, const double *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3];
}

int frgo_vertex_hyperspherical(int n_legs, int n_q, int n_t1, int n_t2, int n_t3, double q_max,
                               double k, int regulator, const double p1[4], const double p2[4],
                               double m2, const double *Z, int nZ, double x_min, double x_max,
                               double *out) {
    if ((n_legs != 2 && n_legs != 3) || n_q < 1 || n_t1 < 1 || n_t2 < 1 || n_t3 < 1) return -1;
    if (n_q > MAXN || n_t1 > MAXN || n_t2 > MAXN || n_t3 > MAXN || out == NULL) return -1;
    static __thread double qn[MAXN], qw[MAXN], t1n[MAXN], t1w[MAXN], t2n[MAXN], t2w[MAXN],
        t3n[MAXN], t3w[MAXN];
    frgo_gauss_legendre(n_q, 0.0, q_max * k, qn, qw);
    frgo_gauss_legendre(n_t1, 0.0, PI, t1n, t1w);
    frgo_gauss_legendre(n_t2, 0.0, PI, t2n, t2w);
    frgo_gauss_legendre(n_t3, 0.0, 2.0 * PI, t3n, t3w);
    double pref = 1.0 / pow(2.0 * PI, 4.0);
    nsum total = {0.0, 0.0};
    for (int a = 0; a < n_q; ++a) {
        double q = qn[a], q2 = q * q;
        double gq = frgo_propagator(regulator, Z, nZ, x_min, x_max, q2, m2, k);
        double rad = pref * qw[a] * q2 * q * frgo_regulator_dot(regulator, q2, k) * gq * gq;
        nsum s1 = {0.0, 0.0};
        for (int i = 0; i < n_t1; ++i) {
            double t1 = t1n[i];
            nsum s2 = {0.0, 0.0};
            for (int j = 0; j < n_t2; ++j) {
                double t2 = t2n[j];
                nsum s3 = {0.0, 0.0};
                for (int c = 0; c < n_t3; ++c) {
                    double t3 = t3n[c];
                    double v[4] = {q * cos(t1), q * sin(t1) * cos(t2),
                                   q * sin(t1) * sin(t2) * cos(t3), q * sin(t1) * sin(t2) * sin(t3)};
                    double a1[4], a2[4];
                    for (int m = 0; m < 4; ++m) {
                        a1[m] = v[m] + p1[m];
                        a2[m] = v[m] - p2[m];
                    }
                    double g = frgo_propagator(regulator, Z, nZ, x_min, x_max, dot4(a1, a1), m2, k);
                    if (n_legs == 3)
                        g *= frgo_propagator(regulator, Z, nZ, x_min, x_max, dot4(a2, a2), m2, k);
                    nsum_add(&s3, t3w[c] * g);
                }
                nsum_add(&s2, t2w[j] * sin(t2) * nsum_get(&s3));
            }
            nsum_add(&s1, t1w[i] * sin(t1) * sin(t1) * nsum_get(&s2));
        }
        nsum_add(&total, rad * nsum_get(&s1));
    }
    *out = nsum_get(&total);
    return 0;
}

/* ---------------------------------------------------------------------------------------- */
/* LPA flow right-hand side.                                                                 */
/* ---------------------------------------------------------------------------------------- */
int frgo_fd_derivatives(const double *x, const double *f, int n, double *d1, double *d2) {
    /* derivatives of the quadratic through three neighbouring points (Lagrange form) */
    if (n < 3 || x == NULL || f == NULL || d1 == NULL || d2 == NULL) return -1;
    for (int i = 0; i < n; ++i) {
        int c = (i == 0) ? 1 : (i == n - 1 ? n - 2 : i); /* centre of the stencil */
        double x0 = x[c - 1], x1 = x[c], x2 = x[c + 1];
        double f0 = f[c - 1], f1 = f[c], f2 = f[c + 1];
        double xe = x[i];
        /* L_j'(xe) and L_j'' for the three Lagrange basis polynomials */
        double l0d = ((xe - x1) + (xe - x2)) / ((x0 - x1) * (x0 - x2));
        double l1d = ((xe - x0) + (xe - x2)) / ((x1 - x0) * (x1 - x2));
        double l2d = ((xe - x0) + (xe - x1)) / ((x2 - x0) * (x2 - x1));
        double l0s = 2.0 / ((x0 - x1) * (x0 - x2));
        double l1s = 2.0 / ((x1 - x0) * (x1 - x2));
        double l2s = 2.0 / ((x2 - x0) * (x2 - x1));
        d1[i] = f0 * l0d + f1 * l1d + f2 * l2d;
        d2[i] = f0 * l0s + f1 * l1s + f2 * l2s;
    }
    return 0;
}

int frgo_lpa_flow_rhs(int d, int n_q, double q_max, double k, int regulator, int n_comp,
                      double m2_floor, const double *rho, const double *u, int n, double *dudt) {
    if (n < 3 || n > MAXN || n_comp < 1 || rho == NULL || u == NULL || dudt == NULL) return -1;
    static __thread double d1[MAXN], d2[MAXN], ms[MAXN], mp[MAXN], Is[MAXN], Ip[MAXN];
    if (frgo_fd_derivatives(rho, u, n, d1, d2) != 0) return -1;
    for (int i = 0; i < n; ++i) {
        ms[i] = u[i] + 2.0 * rho[i] * d1[i];
        mp[i] = u[i];
        if (ms[i] < m2_floor) ms[i] = m2_floor;
        if (mp[i] < m2_floor) mp[i] = m2_floor;
    }
    int rc = frgo_integrate(FRGO_LPA, d, n_q, 0, 0, q_max, k, regulator, NULL, ms, 0.0, NULL, 0,
                            0.0, 0.0, n, Is);
    if (rc != 0) return rc;
    rc = frgo_integrate(FRGO_LPA, d, n_q, 0, 0, q_max, k, regulator, NULL, mp, 0.0, NULL, 0, 0.0,
                        0.0, n, Ip);
    if (rc != 0) return rc;
    for (int i = 0; i < n; ++i)
        dudt[i] = 0.5 * (Is[i] * (3.0 * d1[i] + 2.0 * rho[i] * d2[i]) +
                         (double)(n_comp - 1) * Ip[i] * d1[i]);
    return 0;
}
