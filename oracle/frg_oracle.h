/*
 * frg_oracle.h -- plain, slow, FP64 CPU oracle for the batched fRG loop integrals.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls this code;
 * only the test suite, the smoke check and the CPU-baseline leg of the benchmark do.  It shares
 * no source with the HIP library: its own Gauss-Legendre generator (Newton on the Legendre
 * three-term recurrence in long double), libm transcendentals, Neumaier-compensated sums.
 *
 * Everything follows the paper (Sattler & Pawlowski, "DiFfRG: A Discretisation Framework for
 * functional Renormalisation Group flows", arXiv 2412.13043):
 *   - RG-time convention t = log(Lambda/k), k d/dk = -d/dt                     (Sec. 2.1)
 *   - k d/dk = -2 x d/dx for x = p^2/k^2, used for the regulator derivative    (Sec. 3.1)
 *   - flat (Litim) regulator r(x) = (1/x - 1) Theta(1 - x)                      (Sec. 3.1, fig. polyExpReg)
 *   - vacuum "Quadrature" integrator: tensor-product quadrature over |q| and
 *     the loop angles, d = 4 angle names cos1, cos2, phi                      (Sec. 5.3, App. F)
 *   - log-coordinate linear interpolation of dressing functions               (App. F, FunctionTex1D)
 * and the exponential regulator R_k(q) = q^2/(exp(q^2/k^2) - 1) of the benchmark workloads.
 *
 * All arrays are host memory owned by the caller.  Functions return 0 on success and a negative
 * value on invalid arguments (nothing is written then).
 */
#ifndef FRG_ORACLE_H
#define FRG_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Regulators: exponential, flat (Litim), and the polynomial-exponential shape of Sec. 3.1,
 * R = k^2 exp(-sum_{i=1}^{N} (l2/k^2)^i / i), selected as FRGO_REG_POLYEXP + N (1 <= N <= 64). */
enum { FRGO_REG_EXP = 0, FRGO_REG_LITIM = 1, FRGO_REG_POLYEXP = 100 };
enum { FRGO_LPA = 1, FRGO_TWO_POINT = 2, FRGO_THREE_POINT = 3, FRGO_LPA_T = 4, FRGO_TWO_POINT_T = 5,
       FRGO_THREE_POINT_T = 6 };

/* n-point Gauss-Legendre rule on [a, b]; nodes ascending. */
int frgo_gauss_legendre(int n, double a, double b, double *nodes, double *weights);

/* Regulator R_k(l2) and its scale derivative k dR_k/dk at momentum squared l2 (>= 0). */
double frgo_regulator(int kind, double l2, double k);
double frgo_regulator_dot(int kind, double l2, double k);

/* Dressing Z(l2) from a table on a grid log-uniform in |l| over [x_min, x_max] (n >= 2 points),
 * linear in log|l|, constant outside.  Z == NULL means Z == 1. */
double frgo_dressing(const double *Z, int nZ, double x_min, double x_max, double l2);

/* Propagator G(l2) = 1/(Z(l2) l2 + R_k(l2) + m2). */
double frgo_propagator(int reg, const double *Z, int nZ, double x_min, double x_max,
                       double l2, double m2, double k);

/*
 * Loop integral I_e for every external point e in [0, n_ext):
 *   family 1 (LPA, any d >= 1, no angles):
 *       I = Omega_d/(2pi)^d  sum_a w_a q_a^(d-1) Rdot(q_a^2) / (q_a^2 + R(q_a^2) + m2_e)^2      (Z == 1)
 *   family 2 (two-point, d = 4, angle cos1 = x):
 *       I = 4pi/(2pi)^4 sum_ab w_a w_b sqrt(1-x_b^2) q^3 Rdot(q^2) G(q^2)^2 G((q+p)^2)
 *   family 3 (three-point, d = 4, angles cos1 = x and phi in [0, pi]):
 *       I = 2pi/(2pi)^4 sum_abc w_a w_b w_c sqrt(1-x^2) sin(phi) q^3 Rdot G(q^2)^2 G((q+p1)^2) G((q-p2)^2)
 *       with p1 = p e1, p2 = p (cos(alpha) e1 + sin(alpha) e2).
 * Radial GL(n_q) on [0, q_max*k], x GL(n_x) on [-1, 1], phi GL(n_phi) on [0, pi].
 * ext: family 1 unused (may be NULL); family 2 p[n_ext]; family 3 p[n_ext] followed by alpha[n_ext].
 * m2: per-point masses [n_ext] (NULL -> m2_scalar).
 */
int frgo_integrate(int family, int d, int n_q, int n_x, int n_phi, double q_max, double k,
                   int regulator, const double *ext, const double *m2, double m2_scalar,
                   const double *Z, int nZ, double x_min, double x_max, int n_ext, double *out);

/*
 * dI_e/dm2_e, the derivative of frgo_integrate's integral in the point's mass (the forward-mode
 * derivative that implicit steppers need, Sec. 5.2 jacobian_variables, App. F "AD"): the same
 * sums with every propagator's dG/dm2 = -G^2 taken through the product rule.  Same arguments.
 */
int frgo_integrate_dm2(int family, int d, int n_q, int n_x, int n_phi, double q_max, double k,
                       int regulator, const double *ext, const double *m2, double m2_scalar,
                       const double *Z, int nZ, double x_min, double x_max, int n_ext,
                       double *out);

/*
 * dI_e/dZ_i, the derivatives of the two-point integral (family 2) in the entries of its dressing
 * table: out[e * nZ + i], n_ext x nZ row-major.  The integral depends on the entries through the
 * linear interpolation Z(l2) = (1 - f) Z_j + f Z_{j+1} (cell j, fraction f as in frgo_dressing;
 * nZ == 1: Z(l2) = Z_0); each propagator contributes dG(v)/dZ_i = -G(v)^2 v dZ(v)/dZ_i through
 * the product rule, and entries no node reaches get exactly 0.  Z is required.  Arguments as
 * frgo_integrate (d = 4; ext = p[n_ext]).
 */
int frgo_integrate_dz(int d, int n_q, int n_x, double q_max, double k, int regulator,
                      const double *ext, const double *m2, double m2_scalar, const double *Z,
                      int nZ, double x_min, double x_max, int n_ext, double *out);

/* dI_e/dZ_i of the three-point integral (family 3), out[e * nZ + i], as frgo_integrate_dz:
 * the product rule runs over the radial leg (weight 2) and both inner legs.  ext = p[n_ext]
 * followed by alpha[n_ext]; Z is required. */
int frgo_integrate_dz_three(int n_q, int n_x, int n_phi, double q_max, double k, int regulator,
                            const double *ext, const double *m2, double m2_scalar,
                            const double *Z, int nZ, double x_min, double x_max, int n_ext,
                            double *out);

/* Threshold function of the flat regulator, l_n^d(w) = (2/d) (n + [n == 0]) / (1 + w)^(n+1): the
 * closed form of the LPA integral with that regulator, I = Omega_d/(2 pi)^d k^(d-2) l_1^d(m2/k^2)
 * (and dI/dm2 = -Omega_d/(2 pi)^d k^(d-4) l_2^d). */
double frgo_litim_threshold(int d, int n, double w);

/*
 * General d = 4 one-loop integral with explicit external 4-vectors, on a full hyperspherical
 * product rule (GL in the polar angles theta1, theta2 in [0, pi] with the sin^2/sin Jacobian
 * and GL in the azimuth theta3 in [0, 2pi]):
 *   I = 1/(2pi)^4 \int d^4q Rdot(q^2) G(q^2)^2 G((q+p1)^2) [G((q-p2)^2) if n_legs == 3]
 * Used only to pin the reduced angle forms of families 2 and 3 (rotation invariance).
 */
int frgo_vertex_hyperspherical(int n_legs, int n_q, int n_t1, int n_t2, int n_t3, double q_max,
                               double k, int regulator, const double p1[4], const double p2[4],
                               double m2, const double *Z, int nZ, double x_min, double x_max,
                               double *out);

/*
 * Finite temperature (Sec. 5.3.2, integrator types "Quadratureq0"/"Quadraturex0": the imaginary-
 * time direction becomes a Matsubara sum; Sec. 3.1: regulators that act on the spatial momentum
 * only).  Frequencies w_n = 2 pi T (n + eta), eta = 0 (bosonic) or 1/2 (fermionic).
 *
 * Frequency rule replacing T sum_{n in Z} f(w_n) by sum_j c_j f(w_j):
 *   - every Matsubara frequency with |w_n| <= lambda, weight c = T (the bounded frequency domain);
 *   - n_tail > 0: the frequencies beyond it as an integral, (1/2pi) int_{|w| >= Omega} f(w) dw with
 *     Omega = (largest explicit |w|) + pi T, the midpoint below the first omitted frequency, each
 *     side by GL(n_tail) in t on [0, 1] after w = +-Omega/t (dw = Omega dt/t^2).
 * Nodes ascending in w.  Returns the number of nodes, -1 on invalid arguments (statistics not
 * 0/1, T or lambda not positive, no explicit frequency, n_tail < 0), -2 if cap is too small.
 */
enum { FRGO_BOSONIC = 0, FRGO_FERMIONIC = 1 };
int frgo_matsubara_rule(int statistics, double T, double lambda, int n_tail, int cap, double *w,
                        double *c);

/*
 * Finite-temperature loop integrals in d = 3 + 1 with a spatial regulator R(q^2), q = |spatial q|,
 * the frequency rule above (lambda = freq_max, or freq_max * k when freq_scaled), radial GL(n_q)
 * on [0, q_max k] and x GL(n_x) on [-1, 1]:
 *   family 4 (LPA):       I = sum_j c_j 4pi/(2pi)^3 sum_a w_a q^2 Rdot(q^2) G_j(q)^2
 *                         G_j(q) = 1/(w_j^2 + q^2 + R(q^2) + m2)                     (Z == 1)
 *   family 5 (two-point): I = sum_j c_j 2pi/(2pi)^3 sum_ab w_a w_b q^2 Rdot(q^2) G_j(q)^2 H_j(l)
 *                         G_j(q) = 1/(w_j^2 + Z(q^2) q^2 + R(q^2) + m2),
 *                         H_j(l) = 1/((w_j + p0)^2 + Z(l^2) l^2 + R(l^2) + m2),  l^2 = q^2 + p^2 + 2 q p x
 * (int d^3q = 2 pi int q^2 dq int dx; the dressing depends on the spatial momentum).
 * ext: family 5 p[n_ext] followed by p0[n_ext] (the external frequency); unused for family 4.
 */
int frgo_integrate_ft(int family, int n_q, int n_x, double q_max, double k, int regulator,
                      int statistics, double T, double freq_max, int freq_scaled, int n_tail,
                      const double *ext, const double *m2, double m2_scalar, const double *Z,
                      int nZ, double x_min, double x_max, int n_ext, double *out);

/*
 * Three-point at finite temperature (family 6), d = 3 + 1: the spatial angles are x = cos theta
 * (GL(n_x) on [-1, 1]) and the azimuth phi about the first leg, over [0, 2pi) and folded onto
 * [0, pi] by phi -> 2pi - phi (GL(n_phi) on [0, pi], weight 2; int d^3q = int q^2 dq dx dphi):
 *   I = sum_j c_j 2/(2pi)^3 sum_abc w_a w_b w_c q^2 Rdot(q^2) G_j(q)^2 H1_j(l1) H2_j(l2)
 *   G_j(q)  = 1/(w_j^2 + Z(q^2) q^2 + R(q^2) + m2)
 *   Hi_j(l) = 1/((w_j + p0i)^2 + Z(l^2) l^2 + R(l^2) + m2)
 *   l1^2 = q^2 + p^2 + 2 q p x,  l2^2 = q^2 + p^2 - 2 q p (x cos(alpha) + sqrt(1 - x^2) cos(phi)
 *   sin(alpha)) -- the legs q + p1 and q - p2, |p1| = |p2| = p at angle alpha, carrying the loop
 * frequency shifted by p01 and p02.  ext: p[n_ext], alpha[n_ext], p01[n_ext], p02[n_ext].
 * deriv = 1: dI/dm2 instead (every propagator's -G^2 by the product rule).
 */
int frgo_integrate_ft_three(int n_q, int n_x, int n_phi, double q_max, double k, int regulator,
                            int statistics, double T, double freq_max, int freq_scaled,
                            int n_tail, const double *ext, const double *m2, double m2_scalar,
                            const double *Z, int nZ, double x_min, double x_max, int n_ext,
                            int deriv, double *out);

/*
 * The same integral for one point on a product rule in explicit spatial 3-vectors (to pin the
 * reduced angle form by rotation invariance): q = |q| (cos t1, sin t1 cos t2, sin t1 sin t2),
 * GL(n_t1) in t1 on [0, pi] with the sin t1 Jacobian and GL(n_t2) in t2 on [0, 2pi]; the legs
 * are (q + p1, w_j + p01) and (q - p2, w_j + p02) for arbitrary 3-vectors p1, p2.
 */
int frgo_vertex_ft_spherical(int n_q, int n_t1, int n_t2, double q_max, double k, int regulator,
                             int statistics, double T, double freq_max, int freq_scaled,
                             int n_tail, const double p1[3], const double p2[3], double p01,
                             double p02, double m2, const double *Z, int nZ, double x_min,
                             double x_max, double *out);

/* dI_e/dZ_i of the finite-temperature three-point integral (family 6), out[e * nZ + i]: the
 * radial leg and both inner legs through the interpolation weights of their spatial momenta
 * (dG(v)/dZ_i = -G(v)^2 v w_i(v)).  Arguments as frgo_integrate_ft_three without deriv; Z is
 * required. */
int frgo_integrate_ft_three_dz(int n_q, int n_x, int n_phi, double q_max, double k,
                               int regulator, int statistics, double T, double freq_max,
                               int freq_scaled, int n_tail, const double *ext, const double *m2,
                               double m2_scalar, const double *Z, int nZ, double x_min,
                               double x_max, int n_ext, double *out);

/*
 * Complex external frequencies (families 5 and 6): the external frequency of an inner leg is
 * p0 = p0r + i p0i, as for the paper's external fermion legs at chemical potential mu, whose
 * imaginary-time component is p0f - i mu (App. "Derivation of the four-Fermi system",
 * MakeP0FormRule).  Every inner-leg propagator is continued analytically,
 *   H(l) = 1/((w_j + p0)^2 + Z(l^2) l^2 + R(l^2) + m2)    (complex),
 * the radial leg keeps its real frequency w_j; otherwise the integrals are those of
 * frgo_integrate_ft (family 5) and frgo_integrate_ft_three (family 6).
 * ext: family 5 p, p0r, p0i; family 6 p, alpha, p01r, p02r, p01i, p02i (each [n_ext]).
 * out[e] = Re I_e and out[n_ext + e] = Im I_e.
 */
int frgo_integrate_ft_complex(int family, int n_q, int n_x, int n_phi, double q_max, double k,
                              int regulator, int statistics, double T, double freq_max,
                              int freq_scaled, int n_tail, const double *ext, const double *m2,
                              double m2_scalar, const double *Z, int nZ, double x_min,
                              double x_max, int n_ext, double *out);

/* dI_e/dZ_i of the finite-temperature two-point integral (family 5), out[e * nZ + i], as
 * frgo_integrate_dz: the dressing multiplies the spatial momentum of both legs.  Arguments as
 * frgo_integrate_ft with family 5 implied; Z is required. */
int frgo_integrate_ft_dz(int n_q, int n_x, double q_max, double k, int regulator, int statistics,
                         double T, double freq_max, int freq_scaled, int n_tail,
                         const double *ext, const double *m2, double m2_scalar, const double *Z,
                         int nZ, double x_min, double x_max, int n_ext, double *out);

/* dI_e/dm2_e of frgo_integrate_ft (see frgo_integrate_dm2).  Same arguments. */
int frgo_integrate_ft_dm2(int family, int n_q, int n_x, double q_max, double k, int regulator,
                          int statistics, double T, double freq_max, int freq_scaled, int n_tail,
                          const double *ext, const double *m2, double m2_scalar, const double *Z,
                          int nZ, double x_min, double x_max, int n_ext, double *out);

/*
 * Right-hand side of the LPA flow of u(rho) = U'(rho) for the O(N) model on a rho grid (Sec. 3.1
 * flux form, vacuum, d dimensions, radial and N-1 Goldstone modes):
 *   m_s^2 = u + 2 rho u',  m_p^2 = u   (each floored at m2_floor)
 *   du/dt = +1/2 [ I(m_s^2) (3 u' + 2 rho u'') + (N-1) I(m_p^2) u' ]
 * where I is the family-1 integral and t = log(Lambda/k).  u', u'' are second-order finite
 * differences on the (possibly non-uniform) grid, one-sided at the two ends.  n >= 3.
 */
int frgo_lpa_flow_rhs(int d, int n_q, double q_max, double k, int regulator, int n_comp,
                      double m2_floor, const double *rho, const double *u, int n, double *dudt);

/* Second-order finite-difference first and second derivatives used by frgo_lpa_flow_rhs. */
int frgo_fd_derivatives(const double *x, const double *f, int n, double *d1, double *d2);

#ifdef __cplusplus
}
#endif
#endif
