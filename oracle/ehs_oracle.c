/*
 * ehs_oracle.c -- plain FP64 direct-summation oracle for the half-space sums
 * of Stokes Green's functions (stokeslet, stresslet, rotlet).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct CPU
 * reference against which the GPU library is checked.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU path.
 *
 * What it computes: the half-space representation of the paper
 * (Srinivasan & Tornberg, "Fast Ewald summation for Green's functions of
 * Stokes flow in a half-space", Sec. 3, eq. (v_sum_halfspace) with the
 * harmonic corrections of eq. (phi)), summed directly in O(N*T):
 *
 *   u(x) = sum_m  K(x - y_m) s_m  -  K(x - y_m^I) s_m^I
 *                 - x_3 grad phi_m(x) + e_3 phi_m(x)
 *
 * with y^I = (y1, y2, -y3) the reflection in the wall x3 = 0 (Sec. 3).
 *
 * Normalisation (the paper writes 8*pi*S, 8*pi*T, 4*pi*W and 4*pi*G = 1/r;
 * Sec. 2 and Sec. 3): we drop those constants and use
 *     S(r) f      = f/r + r (r.f)/r^3
 *     T(r)[g,q]   = -6 r (r.g)(r.q)/r^5
 *     2 W(r) v    = 2 (v x r)/r^3            (v = g x q)
 *     G(r)        = 1/r
 * i.e. the r -> 0 / xi -> 0 limits of the paper's Ewald real-space parts
 * (Sec. 4 and the Appendix), which is the only set for which the wall
 * velocity vanishes (no-slip).
 *
 * Correction potentials (eq. (phi)), evaluated at r~ = x - y^I:
 *     phi_S = 2 ( -f3 G - y3 grad G . f^I )                       (as printed)
 *     phi_T = 4 (g^I . q^I) dG/dx3 - 4 y3 (g^I)^T (grad grad G) q^I
 *             (the printed second coefficient, +2, violates no-slip; the
 *              harmonic function with the required wall values has -4)
 *     phi_W = 2 grad G . 2 (q3 g^I - g3 q^I)                        (as printed)
 *
 * Self interaction: the direct term m is omitted when x equals y_m exactly
 * (the paper's p != m, Sec. 2); the image and correction terms of that
 * source are kept (they are centred below the wall, Sec. 4).
 *
 * Strength layouts: stokeslet s = f (3 per source); stresslet s = (g, q)
 * (6 per source, strength then orientation); rotlet s = (g, q) (6 per
 * source), the sum depending on them only through g x q.
 *
 * A debug "mutation" switch plants deliberate mistakes (used only by tests
 * that check the pins are sensitive: 1-4 in the direct sum, 5-10 in the
 * real-space part of the split); it is 0 in normal use.
 */
#include <math.h>
#include <stddef.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_STOKESLET 0
#define ORACLE_STRESSLET 1
#define ORACLE_ROTLET 2

static int g_mutation = 0;

void oracle_set_mutation(int m) { g_mutation = m; }
int oracle_get_mutation(void) { return g_mutation; }

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double* a, const double* b, double* c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Free-space kernel applied to one source, Sec. 2:  out += K(r) s. */
static void kernel_term(int kernel, const double* r, const double* s, double sign, double* out)
{
    double r2 = dot3(r, r);
    double rn = sqrt(r2);
    double ir = 1.0 / rn;
    double ir3 = ir * ir * ir;
    if (kernel == ORACLE_STOKESLET) {
        /* S f = f/r + r (r.f)/r^3 */
        double rf = dot3(r, s);
        for (int i = 0; i < 3; ++i) out[i] += sign * (s[i] * ir + r[i] * rf * ir3);
    } else if (kernel == ORACLE_STRESSLET) {
        /* T[g,q] = -6 r (r.g)(r.q)/r^5 */
        const double* g = s;
        const double* q = s + 3;
        double ir5 = ir3 * ir * ir;
        double c = -6.0 * dot3(r, g) * dot3(r, q) * ir5;
        for (int i = 0; i < 3; ++i) out[i] += sign * c * r[i];
    } else {
        /* 2 W (g x q) = 2 (v x r)/r^3 with W v = (v x r)/r^3 (4 pi W = eps r / r^3) */
        double v[3], vr[3];
        cross3(s, s + 3, v);
        cross3(v, r, vr);
        for (int i = 0; i < 3; ++i) out[i] += sign * 2.0 * vr[i] * ir3;
    }
}

/*
 * Harmonic correction phi and its gradient for one source at y with
 * strength s, evaluated at x (eq. (phi)); G and its derivatives are taken
 * at r~ = x - y^I with G = 1/|r~|.
 */
void oracle_correction(int kernel, const double* y, const double* s, const double* x, double* phi,
                       double* gphi)
{
    double rt[3] = {x[0] - y[0], x[1] - y[1], x[2] + y[2]};
    double y3 = y[2];
    double r2 = dot3(rt, rt);
    double rn = sqrt(r2);
    double ir = 1.0 / rn;
    double ir3 = ir * ir * ir;
    double ir5 = ir3 * ir * ir;
    double ir7 = ir5 * ir * ir;
    /* G = 1/r, dG_i = -r_i/r^3, ddG_ij = -d_ij/r^3 + 3 r_i r_j / r^5,
       dddG_ijk = 3 (d_ij r_k + d_ik r_j + d_jk r_i)/r^5 - 15 r_i r_j r_k / r^7 */
    double G = ir;
    double dG[3];
    for (int i = 0; i < 3; ++i) dG[i] = -rt[i] * ir3;
    double ddG[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) ddG[i][j] = (i == j ? -ir3 : 0.0) + 3.0 * rt[i] * rt[j] * ir5;

    if (kernel == ORACLE_STOKESLET) {
        const double* f = s;
        double fI[3] = {f[0], f[1], -f[2]};
        double c3 = 2.0;
        if (g_mutation == 1) c3 = -2.0; /* planted: wrong sign of the dipole term */
        *phi = 2.0 * (-f[2] * G) - c3 * y3 * dot3(dG, fI);
        for (int k = 0; k < 3; ++k) {
            double t = 0.0;
            for (int j = 0; j < 3; ++j) t += ddG[k][j] * fI[j];
            gphi[k] = -2.0 * f[2] * dG[k] - c3 * y3 * t;
        }
    } else if (kernel == ORACLE_STRESSLET) {
        const double* g = s;
        const double* q = s + 3;
        double gI[3] = {g[0], g[1], -g[2]};
        double qI[3] = {q[0], q[1], -q[2]};
        double gq = dot3(gI, qI);
        double cq = -4.0; /* the printed coefficient is +2 (see header) */
        if (g_mutation == 2) cq = 2.0; /* planted: the coefficient exactly as printed */
        double quad = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) quad += gI[i] * ddG[i][j] * qI[j];
        *phi = 4.0 * gq * dG[2] + cq * y3 * quad;
        double rg = dot3(rt, gI), rq = dot3(rt, qI);
        for (int k = 0; k < 3; ++k) {
            /* d/dx_k of (g^I)^T ddG q^I = dddG_ijk g_i q_j */
            double t = 3.0 * (gq * rt[k] + gI[k] * rq + qI[k] * rg) * ir5 - 15.0 * rg * rq * rt[k] * ir7;
            gphi[k] = 4.0 * gq * ddG[k][2] + cq * y3 * t;
        }
    } else {
        const double* g = s;
        const double* q = s + 3;
        double gI[3] = {g[0], g[1], -g[2]};
        double qI[3] = {q[0], q[1], -q[2]};
        double w[3];
        for (int i = 0; i < 3; ++i) w[i] = 2.0 * (q[2] * gI[i] - g[2] * qI[i]);
        *phi = 2.0 * dot3(dG, w);
        for (int k = 0; k < 3; ++k) {
            double t = 0.0;
            for (int j = 0; j < 3; ++j) t += ddG[k][j] * w[j];
            gphi[k] = 2.0 * t;
        }
    }
}

static int nstr(int kernel) { return kernel == ORACLE_STOKESLET ? 3 : 6; }

/*
 * One source's full half-space contribution at x (eq. (v_sum_halfspace)),
 * formed on its own before it is added to the running sum: for a source
 * close to the wall its image and correction terms are each of size
 * 1/(2 y3)^2 and cancel to O(1), so adding them to the sum one by one would
 * round away what the other sources have contributed.
 */
static void halfspace_term(int kernel, const double* y, const double* s, const double* x, double* sum)
{
    double acc[3] = {0.0, 0.0, 0.0};
    double r[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
    int self = (r[0] == 0.0 && r[1] == 0.0 && r[2] == 0.0);
    if (!self) kernel_term(kernel, r, s, 1.0, acc);

    /* image term: - K(x - y^I) s^I, with s^I the reflected strength(s) */
    double rt[3] = {x[0] - y[0], x[1] - y[1], x[2] + y[2]};
    double sI[6];
    sI[0] = s[0];
    sI[1] = s[1];
    sI[2] = -s[2];
    if (kernel != ORACLE_STOKESLET) {
        sI[3] = s[3];
        sI[4] = s[4];
        sI[5] = -s[5];
    }
    double img_sign = -1.0;
    if (g_mutation == 3) img_sign = 1.0; /* planted: image added instead of subtracted */
    kernel_term(kernel, rt, sI, img_sign, acc);

    double phi, gphi[3];
    oracle_correction(kernel, y, s, x, &phi, gphi);
    double x3 = x[2];
    if (g_mutation == 4) x3 = 0.0; /* planted: the -x3 grad phi term dropped */
    acc[0] += -x3 * gphi[0];
    acc[1] += -x3 * gphi[1];
    acc[2] += -x3 * gphi[2] + phi;
    sum[0] += acc[0];
    sum[1] += acc[1];
    sum[2] += acc[2];
}

/*
 * u[t] = sum over all sources of the half-space contribution at x[t].
 * y: n_src x 3, s: n_src x (3 | 6) row-major, x: n_tgt x 3, u: n_tgt x 3.
 * Returns 0, or -1 for an unknown kernel.
 */
int oracle_halfspace(int kernel, const double* y, const double* s, long n_src, const double* x, long n_tgt,
                     double* u, int nthreads)
{
    if (kernel < 0 || kernel > 2) return -1;
    int ns = nstr(kernel);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    long t;
#pragma omp parallel for schedule(dynamic, 16)
    for (t = 0; t < n_tgt; ++t) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (long m = 0; m < n_src; ++m) halfspace_term(kernel, y + 3 * m, s + ns * m, x + 3 * t, acc);
        u[3 * t + 0] = acc[0];
        u[3 * t + 1] = acc[1];
        u[3 * t + 2] = acc[2];
    }
    return 0;
}

/* The free-space sum of Sec. 2 (no image, no correction), same layouts. */
int oracle_freespace(int kernel, const double* y, const double* s, long n_src, const double* x, long n_tgt,
                     double* u, int nthreads)
{
    if (kernel < 0 || kernel > 2) return -1;
    int ns = nstr(kernel);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    long t;
#pragma omp parallel for schedule(dynamic, 16)
    for (t = 0; t < n_tgt; ++t) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (long m = 0; m < n_src; ++m) {
            const double* y_m = y + 3 * m;
            double r[3] = {x[3 * t] - y_m[0], x[3 * t + 1] - y_m[1], x[3 * t + 2] - y_m[2]};
            if (r[0] == 0.0 && r[1] == 0.0 && r[2] == 0.0) continue;
            kernel_term(kernel, r, s + ns * m, 1.0, acc);
        }
        u[3 * t + 0] = acc[0];
        u[3 * t + 1] = acc[1];
        u[3 * t + 2] = acc[2];
    }
    return 0;
}

/*
 * ---------------------------------------------------------------------------
 * The real-space part of the Ewald split of the same sum (Sec. 4 and the
 * appendix), for stage checks of the GPU path: the kernels K_R of eq.
 * (kernel_real_parts) and the harmonic corrections built from
 * G_R = erfc(xi r)/r (eq. (G_R)) instead of G = 1/r, over the pairs with
 * |x - y| < r_c (direct) and |x - y^I| < r_c (image and corrections), plus
 * the stokeslet's self term -4 xi/sqrt(pi) f at a coincident source.
 * ---------------------------------------------------------------------------
 */
static const double ORACLE_PI = 3.14159265358979323846;

/* r-derivatives 0..3 of G_R(r) = erfc(xi r)/r: from those of erf(xi r)/r
 * recorded in the appendix, with G_R = 1/r - erf(xi r)/r written out in
 * erfc (no cancellation where erf is close to 1) */
static void gr_radial(double r, double xi, double g[4])
{
    double C = erfc(xi * r), E = exp(-xi * xi * r * r), c = 2.0 * xi / sqrt(ORACLE_PI);
    double r2 = r * r;
    g[0] = C / r;
    g[1] = -C / r2 - c * E / r;
    g[2] = 2.0 * C / (r2 * r) + 2.0 * c * E / r2 + (g_mutation == 8 ? 0.0 : 2.0 * c * xi * xi * E);
    g[3] = -6.0 * C / (r2 * r2) -
           (2.0 * c * E / r) * (3.0 / r2 + 2.0 * xi * xi + (g_mutation == 9 ? 0.0 : 2.0 * xi * xi * xi * xi * r2));
}

/* Cartesian derivatives of a radial function from its r-derivatives g:
 *   d1_i   = g1 n_i
 *   d2_ij  = (g2 - g1/r) n_i n_j + (g1/r) d_ij
 *   d3_ijk = (g3 - 3 g2/r + 3 g1/r^2) n_i n_j n_k + (g2/r - g1/r^2) (d_ij n_k + d_ik n_j + d_jk n_i)
 * with n = r_vec / r. */
static void radial_tensors(const double* rv, const double* g, double* d1, double d2[3][3], double d3[3][3][3])
{
    double r = sqrt(dot3(rv, rv));
    double n[3] = {rv[0] / r, rv[1] / r, rv[2] / r};
    double a2 = g[2] - g[1] / r, b2 = g[1] / r;
    double a3 = g[3] - 3.0 * g[2] / r + 3.0 * g[1] / (r * r), b3 = g[2] / r - g[1] / (r * r);
    for (int i = 0; i < 3; ++i) {
        d1[i] = g[1] * n[i];
        for (int j = 0; j < 3; ++j) {
            d2[i][j] = a2 * n[i] * n[j] + (i == j ? b2 : 0.0);
            for (int k = 0; k < 3; ++k)
                d3[i][j][k] = a3 * n[i] * n[j] * n[k] +
                              b3 * ((i == j ? n[k] : 0.0) + (i == k ? n[j] : 0.0) + (j == k ? n[i] : 0.0));
        }
    }
}

/* The correction potential of eq. (phi) and its gradient from the value and
 * derivatives (G, dG, ddG, dddG) of the harmonic kernel at r~ = x - y^I; the
 * same combinations as oracle_correction, here for any radial kernel. */
static void correction_from(int kernel, const double* y, const double* s, double G, const double* dG,
                            double ddG[3][3], double dddG[3][3][3], double* phi, double* gphi)
{
    double y3 = y[2];
    if (kernel == ORACLE_STOKESLET) {
        const double* f = s;
        double fI[3] = {f[0], f[1], -f[2]};
        *phi = -2.0 * f[2] * G - 2.0 * y3 * dot3(dG, fI);
        for (int k = 0; k < 3; ++k) {
            double t = 0.0;
            for (int j = 0; j < 3; ++j) t += ddG[k][j] * fI[j];
            gphi[k] = -2.0 * f[2] * dG[k] - 2.0 * y3 * t;
        }
    } else if (kernel == ORACLE_STRESSLET) {
        const double *g = s, *q = s + 3;
        double gI[3] = {g[0], g[1], -g[2]}, qI[3] = {q[0], q[1], -q[2]};
        double gq = dot3(gI, qI), quad = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) quad += gI[i] * ddG[i][j] * qI[j];
        *phi = 4.0 * gq * dG[2] - 4.0 * y3 * quad;
        for (int k = 0; k < 3; ++k) {
            double t = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) t += dddG[i][j][k] * gI[i] * qI[j];
            gphi[k] = 4.0 * gq * ddG[k][2] - 4.0 * y3 * t;
        }
    } else {
        const double *g = s, *q = s + 3;
        double gI[3] = {g[0], g[1], -g[2]}, qI[3] = {q[0], q[1], -q[2]};
        double w[3];
        for (int i = 0; i < 3; ++i) w[i] = 2.0 * (q[2] * gI[i] - g[2] * qI[i]);
        *phi = 2.0 * dot3(dG, w);
        for (int k = 0; k < 3; ++k) {
            double t = 0.0;
            for (int j = 0; j < 3; ++j) t += ddG[k][j] * w[j];
            gphi[k] = 2.0 * t;
        }
    }
}

/* K_R(r) s of eq. (kernel_real_parts), in the normalisation of kernel_term
 * (the xi -> 0 limit of each is the kernel above):
 *   S_R = 2 (xi E/sqrt(pi) + C/(2r)) (I + n n) - 4 xi E/sqrt(pi) I
 *   T_R[g,q]_j = -(2/r) (3C/r + c (3 + 2 xi^2 r^2) E) n_j (n.g)(n.q)
 *                + 2 c xi^2 E (g_j (r.q) + (g.q) r_j + q_j (r.g))
 * (the appendix prints unit vectors in the Gaussian term of T_R; only the
 * vector r itself gives T_R the dimension of T, 1/length^2, and makes
 * T_R - T = -T_F vanish at r = 0, as the smooth odd Fourier part does, with
 * the slope -grad T_F(0) that the Fourier multiplier gives)
 *   W_R v = 2 (C/r^2 + c E/r) (v x n),   v = g x q
 * with C = erfc(xi r), E = exp(-xi^2 r^2), c = 2 xi / sqrt(pi). */
static void kernel_real(int kernel, const double* rv, const double* s, double xi, double sign, double* out)
{
    double r = sqrt(dot3(rv, rv));
    double n[3] = {rv[0] / r, rv[1] / r, rv[2] / r};
    double C = erfc(xi * r), E = exp(-xi * xi * r * r), c = 2.0 * xi / sqrt(ORACLE_PI);
    if (kernel == ORACLE_STOKESLET) {
        double a = 2.0 * (xi * E / sqrt(ORACLE_PI) + C / (2.0 * r));
        double b = (g_mutation == 5 ? 3.0 : 4.0) * xi * E / sqrt(ORACLE_PI);
        double nf = dot3(n, s);
        for (int i = 0; i < 3; ++i) out[i] += sign * (a * (s[i] + n[i] * nf) - b * s[i]);
    } else if (kernel == ORACLE_STRESSLET) {
        const double *g = s, *q = s + 3;
        double ng = dot3(n, g), nq = dot3(n, q), gq = dot3(g, q);
        double A = -(2.0 / r) * (3.0 * C / r + c * (3.0 + 2.0 * xi * xi * r * r) * E);
        double B = (g_mutation == 6 ? 1.0 : 2.0) * c * xi * xi * E * (g_mutation == 10 ? 1.0 : r);
        for (int i = 0; i < 3; ++i) out[i] += sign * (A * n[i] * ng * nq + B * (g[i] * nq + gq * n[i] + q[i] * ng));
    } else {
        double v[3], vn[3];
        cross3(s, s + 3, v);
        cross3(v, n, vn);
        double a = 2.0 * (C / (r * r) + (g_mutation == 7 ? 0.0 : c * E / r));
        for (int i = 0; i < 3; ++i) out[i] += sign * a * vn[i];
    }
}

static void ewald_real_term(int kernel, const double* y, const double* s, const double* x, double xi, double rc2,
                            double* sum)
{
    double acc[3] = {0.0, 0.0, 0.0};
    double r[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
    double r2 = dot3(r, r);
    if (r2 == 0.0) {
        if (kernel == ORACLE_STOKESLET) /* the limit of S_R - S at r = 0 (Sec. 4) */
            for (int i = 0; i < 3; ++i) acc[i] -= 4.0 * xi / sqrt(ORACLE_PI) * s[i];
    } else if (r2 < rc2) {
        kernel_real(kernel, r, s, xi, 1.0, acc);
    }
    double rt[3] = {x[0] - y[0], x[1] - y[1], x[2] + y[2]};
    if (dot3(rt, rt) < rc2) {
        double sI[6] = {s[0], s[1], -s[2], 0.0, 0.0, 0.0};
        if (kernel != ORACLE_STOKESLET) {
            sI[3] = s[3];
            sI[4] = s[4];
            sI[5] = -s[5];
        }
        kernel_real(kernel, rt, sI, xi, -1.0, acc);
        double g[4], d1[3], d2[3][3], d3[3][3][3], phi, gphi[3];
        gr_radial(sqrt(dot3(rt, rt)), xi, g);
        radial_tensors(rt, g, d1, d2, d3);
        correction_from(kernel, y, s, g[0], d1, d2, d3, &phi, gphi);
        acc[0] += -x[2] * gphi[0];
        acc[1] += -x[2] * gphi[1];
        acc[2] += -x[2] * gphi[2] + phi;
    }
    sum[0] += acc[0];
    sum[1] += acc[1];
    sum[2] += acc[2];
}

/* u[t] = the real-space part at x[t] with cutoff r_c (layouts as oracle_halfspace). */
int oracle_ewald_real(int kernel, const double* y, const double* s, long n_src, const double* x, long n_tgt,
                      double xi, double rc, double* u, int nthreads)
{
    if (kernel < 0 || kernel > 2 || !(xi > 0.0) || !(rc > 0.0)) return -1;
    int ns = nstr(kernel);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const double rc2 = rc * rc;
    long t;
#pragma omp parallel for schedule(dynamic, 16)
    for (t = 0; t < n_tgt; ++t) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (long m = 0; m < n_src; ++m) ewald_real_term(kernel, y + 3 * m, s + ns * m, x + 3 * t, xi, rc2, acc);
        u[3 * t + 0] = acc[0];
        u[3 * t + 1] = acc[1];
        u[3 * t + 2] = acc[2];
    }
    return 0;
}

/* The correction potential and gradient with G_R (for the pins of the split). */
void oracle_correction_real(int kernel, const double* y, const double* s, const double* x, double xi, double* phi,
                            double* gphi)
{
    double rt[3] = {x[0] - y[0], x[1] - y[1], x[2] + y[2]};
    double g[4], d1[3], d2[3][3], d3[3][3][3];
    gr_radial(sqrt(dot3(rt, rt)), xi, g);
    radial_tensors(rt, g, d1, d2, d3);
    correction_from(kernel, y, s, g[0], d1, d2, d3, phi, gphi);
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
