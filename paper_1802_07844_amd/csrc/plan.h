// Parameter selection for one evaluation (host-only arithmetic).
//
// Given xi and r_c from the caller and the target relative RMS error tol:
//  * M (grid intervals over the box L) from the Fourier truncation estimate
//    of the paper's Table 1 with k_inf = pi / h = pi M / L, sources and images
//    counted (Q -> 2Q), budget tol/4 relative to sqrt(Q)/L (tol/40 for the
//    rotlet, whose correction terms are of the same order as the kernel and
//    are not covered by the free-space estimate -- paper Sec. 6);
//  * P (Gaussian support, even) from exp(-pi P c^2 / 2) <= tol/40 (tol/4 for
//    the FP32 stokeslet and rotlet when tol >= 1e-6), c = 0.95,
//    eta = P xi^2 h^2 / (c^2 pi) (Algorithm 1 step 4), M raised until eta < 0.95;
//  * the box is extended by max(P, m / (sqrt2 xi h)) nodes with
//    m = sqrt(2 ln(1/tol)): the Gaussian support of Algorithm 1 step 3 plus a
//    margin for the k-space screening exp(-(1-eta) k^2/4xi^2), which is
//    applied to the window-truncated kernel and must not reach the window's
//    edge; M~ is then rounded up to an even 7-smooth size (FFT radices 2..8);
//  * the real-space estimate of Table 2 (Q -> 2Q) is reported and flagged
//    when above tol/2;
//  * precision: FP32 in auto mode when tol >= 1e-5 and the FP32 rounding
//    estimate is at most tol/2, FP64 otherwise.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "kernels.h"

namespace ehs {

constexpr double C_SHAPE = 0.95;
constexpr size_t ZSLAB_BUDGET = (size_t)2 << 30;

inline bool smooth7(long long n)
{
    if (n < 1) return false;
    for (int p : {2, 3, 5, 7})
        while (n % p == 0) n /= p;
    return n == 1;
}

inline int next_smooth_even(double x)
{
    long long n = (long long)std::ceil(x);
    if (n < 2) n = 2;
    while (!(n % 2 == 0 && smooth7(n))) ++n;
    return (int)n;
}

// Radices of the Stockham FFT of length n: the factorisation into
// {2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 15, 16} with the fewest stages (each stage
// is one pass through LDS), ties broken by the larger per-thread capacity
// (elements a thread holds, (16 / R) R at the smallest); odd radices come
// first, since the first stage writes with a stride of its radix and an odd
// stride spreads over the LDS banks, then the even ones in decreasing order.
inline bool factor_radices(int n, std::vector<int>& r)
{
    r.clear();
    if (n < 2) return false;
    static const int R[] = {16, 15, 14, 12, 10, 8, 7, 6, 5, 4, 3, 2};
    // best[m] = (stages, capacity) for m, with the first radix used
    std::vector<int> st(n + 1, 1 << 20), cap(n + 1, 0), first(n + 1, 0);
    st[1] = 0;
    cap[1] = 16;
    for (int m = 2; m <= n; ++m) {
        if (n % m) continue;
        for (int x : R) {
            if (m % x || st[m / x] >= (1 << 20)) continue;
            int s2 = st[m / x] + 1, c2 = std::min(cap[m / x], (16 / x) * x);
            if (s2 < st[m] || (s2 == st[m] && c2 > cap[m])) {
                st[m] = s2;
                cap[m] = c2;
                first[m] = x;
            }
        }
    }
    if (st[n] >= (1 << 20)) return false;
    for (int m = n; m > 1; m /= first[m]) r.push_back(first[m]);
    std::stable_sort(r.begin(), r.end(), [](int a, int b) {
        bool oa = a & 1, ob = b & 1;
        if (oa != ob) return oa;
        return a > b;
    });
    return true;
}

inline int lds_fft_cap(int n, int nt)
{
    std::vector<int> r;
    if (!factor_radices(n, r)) return 0;
    int per = 16;
    for (int x : r) per = std::min(per, (16 / x) * x);
    return per * nt;
}

inline int bits_for(long long nkeys)
{
    int b = 4;
    while ((1LL << b) < nkeys) b += 4;
    return b;
}


// relative truncation estimates (paper Tables 1 and 2), sources and images
// counted, normalised by sqrt(Q)/L; R in Table 1 taken as sqrt(6) L
inline double est_fourier_rel(int family, double k, double xi, double L)
{
    const double pi = 3.14159265358979323846;
    double e = std::exp(-k * k / (4 * xi * xi));
    double R = std::sqrt(6.0) * L;
    if (family == 0) return std::sqrt(2.0) * R * k * k * k / (xi * xi * pi) * e;
    if (family == 1) return std::sqrt(7.0 / 3.0) * R * k * k * k * k / (xi * xi * pi) * e;
    return std::sqrt(16.0 * xi * xi / (3.0 * pi * L * k)) * e;
}

inline double est_real_rel(int family, double rc, double xi, double L)
{
    double e = std::exp(-xi * xi * rc * rc);
    if (family == 0) return std::sqrt(8.0 * rc / L) * e;
    if (family == 1) return std::sqrt(224.0 * xi * xi * xi * xi * rc * rc * rc / (9.0 * L)) * e;
    return std::sqrt(16.0 / (3.0 * L * rc)) * e;
}

inline double xi_for_cutoff(int family, double rc, double tol, double L)
{
    if (!(rc > 0) || !(tol > 0) || !(L > 0) || family < 0 || family > 2) return -1.0;
    // bisection on xi in (0, 100 / rc]: the estimate decreases for xi rc > ~1
    double lo = 0.5 / rc, hi = 100.0 / rc;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (est_real_rel(family, rc, mid, L) > 0.5 * tol)
            lo = mid;
        else
            hi = mid;
    }
    return hi;
}

// Cutoff r_c at which the real-space estimate for xi equals est: bisection
// over xi r_c in [1, 100], where every family's estimate decreases in r_c.
// Returns -1 for bad arguments or when est lies outside that range.
inline double cutoff_for_estimate(int family, double xi, double est, double L)
{
    if (!(xi > 0) || !(est > 0) || !(L > 0) || family < 0 || family > 2) return -1.0;
    double lo = 1.0 / xi, hi = 100.0 / xi;
    if (est_real_rel(family, lo, xi, L) < est || est_real_rel(family, hi, xi, L) > est) return -1.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (est_real_rel(family, mid, xi, L) > est)
            lo = mid;
        else
            hi = mid;
    }
    return hi;
}

struct PlanInput {
    int family;
    long long N, T;
    double xi, rc, tol;
    double lo[3], hi[3];
    double Q;
    int prec;  // 0 auto, 1 fp64, 2 fp32
    int force_M, force_P, force_Mt;
    int force_zg;  // > 0: k1 slabs per group of the y / x3 pipeline
    int gather_extra;  // >= 0: extra gather support nodes (even); < 0: default
    int dgrid;         // 1 / 0: force the correction density D on / off; < 0: by cost
    double tlo3;       // lowest target x3 (>= 0)
    double slo3;       // lowest source x3 (> 0): the images lie at x3 <= -slo3
    const uint32_t* zhist;  // nullable: ZH_BINS counts of the target heights, bins of width zbin
    double zbin;
    int force_nr;      // 1..3: real-space cells of side >= r_c / force_nr; else chosen by density
    bool free;         // the free-space sum (Sec. 2): no wall, no images, no corrections
};

// Real-space cells of side >= r_c / nr are walked (2 nr + 1)^3 around a
// target's cell.  Smaller cells cut the candidates' volume (27 r_c^3 for
// nr = 1, 15.6 for 2, 12.7 for 3) but leave the 64-target chunks of a cell
// emptier and add cell ranges to walk, so nr follows the number of targets
// a cell of side r_c holds, averaged over the targets (a cell's chunks cost
// in proportion to its targets): below 256, nr = 1; below 1500, nr = 2
// (60-190 targets per cell), else 3.  Measured: N = 1e6 uniform with 2000
// neighbours (480 per r_c cell) 38.6 -> 29.1 ms with nr = 2; with 600 (146)
// 11.3 -> 14.9 ms; 300 at N = 1e5 (75) 0.72 -> 1.0 ms.  The average over the
// targets comes from the height histogram with x1, x2 taken as uniform
// over the box: a set clustered at the wall has most of its targets in
// cells far fuller than the box average.
inline double weighted_occupancy(const double extent[3], double rc, long long T, const uint32_t* zhist,
                                 double zbin)
{
    int nc[3];
    for (int a = 0; a < 3; ++a) nc[a] = std::max(1, std::min(256, (int)std::floor(extent[a] / rc)));
    const double plane = (double)nc[0] * nc[1];
    if (!zhist || !(zbin > 0) || !(extent[2] > 0)) return (double)T / (plane * nc[2]);
    const double s3 = extent[2] / nc[2];
    std::vector<double> layer(nc[2], 0.0);
    for (int b = 0; b < ZH_BINS; ++b) {
        const double n = (double)zhist[b];
        if (n == 0) continue;
        if (b < ZH_BINS - 1) {
            int l = (int)std::floor((b + 0.5) * zbin / s3);
            layer[std::min(std::max(l, 0), nc[2] - 1)] += n;
        } else {
            // everything above: spread over the layers it can occupy
            int l0 = std::min(nc[2] - 1, (int)std::floor((ZH_BINS - 1) * zbin / s3));
            for (int l = l0; l < nc[2]; ++l) layer[l] += n / (nc[2] - l0);
        }
    }
    double s1 = 0, s2 = 0;
    for (double n : layer) {
        s1 += n;
        s2 += n * n;
    }
    return s1 > 0 ? s2 / (s1 * plane) : 0.0;
}

struct Plan {
    int family, prec;
    long long N, T;
    double xi, rc, tol;
    double L, h, Lt, eta, Q;
    int M, P, Ps, Pg, Mt, Qz, nf, nf3, ncin;
    bool dgrid;  // the correction sources are spread as one density D
    bool resident;
    double est_r, est_f, est32;
    CellGeom cg;
    long long ncell;
    GridArgs g;   // spreading (support P)
    GridArgs gg;  // quadrature at the targets (support Pg >= P, same Gaussian)
    long long ntiles;
    long long ntiles_g;  // quadrature tiles (8^3 nodes)
    bool gtiles;         // quadrature in node-owner form (large supports at low density), else one-wavefront forms
    bool ggroup = false; // one-wavefront form with groups of nearby targets sharing the walk
    int Bx, By;
    int zg;  // k1 slabs per group of the y / x3 pipeline
    int l3lo;  // first x3 node the inverse transforms produce (the quadrature reads no lower node)
    int lzc;   // the correction grids (components >= ncA, spread at the images only) vanish at x3 nodes >= lzc
    long long max_chunks;
    int warnings;
    double occ;  // targets per real-space cell of side r_c, averaged over the targets
    bool free;   // free space: sources only on the grid, kernel grids only, no image terms
};

// correction mode of the grid pipeline (CM_GRIDS, CM_DENSITY or CM_FREE)
inline int plan_cm(const Plan& p) { return p.free ? CM_FREE : p.dgrid ? CM_DENSITY : CM_GRIDS; }

constexpr int EHS_MT_MAX = 2048;

// lines per block of the x / y passes: one 128-byte segment of complex
// values per written (or read) row, i.e. 8 (FP64) or 16 (FP32) lines, fewer
// when the lines and the twiddle tables do not fit the LDS budget (78 KiB:
// two blocks per CU) or the 16-element register budget of the FFT
inline int choose_lines(int Mt, size_t esz)
{
    int B = (int)(128 / (2 * esz));
    int cap = lds_fft_cap(Mt, 256);
    // LDS per block: B lines of Mt + 1 values and the stage twiddles (Mt)
    while (B > 2 && (((size_t)B * (Mt + 1) + Mt) * 2 * esz > 78 * 1024 || B * Mt > cap)) B -= 2;
    return B;
}

inline int make_plan(const PlanInput& in, Plan* out)
{
    Plan p;
    std::memset(&p, 0, sizeof(p));
    p.family = in.family;
    p.free = in.free;
    p.N = in.N;
    p.T = in.T;
    p.xi = in.xi;
    p.rc = in.rc;
    p.tol = in.tol;
    p.Q = in.Q;
    {
        // FP32 rounding error of the grid path for uniform point sets, fitted
        // to the error at typical targets (FP32 minus FP64 under one plan):
        // the grid values near a source carry its own smooth field, of size
        // xi |f| (stokeslet) or xi^3 |S| (stresslet), whose FP32 quantisation
        // does not cancel at the source's own position; the rotlet's stays
        // near 1e-6.  Clustered sets have a larger RMS velocity, so their
        // relative rounding error is smaller.
        double box = std::max(std::max(in.hi[0] - in.lo[0], in.hi[1] - in.lo[1]),
                              in.free ? in.hi[2] - in.lo[2] : in.hi[2]);
        double xl = in.xi * box;
        double e32 = in.family == 0 ? 1.7e-6 * std::pow(xl / 25.0, 1.6)
                   : in.family == 1 ? 1.1e-5 * std::pow(xl / 45.0, 2.5)
                                    : 1e-6;
        p.est32 = e32;
        p.prec = in.prec == 0 ? ((in.tol >= 1e-5 && e32 <= 0.5 * in.tol) ? 2 : 1) : in.prec;
        if (p.prec == 2 && e32 > 0.5 * in.tol) p.warnings |= 4;
    }
    const double pi = 3.14159265358979323846;
    // half space: x3 measured from the wall; free space: the points' own range
    double ext1 = in.hi[0] - in.lo[0], ext2 = in.hi[1] - in.lo[1], ext3 = in.free ? in.hi[2] - in.lo[2] : in.hi[2];
    double L = std::max(std::max(ext1, ext2), ext3);
    if (!(L > 0)) return -3;
    L *= 1.0 + 1e-12;
    p.L = L;
    const double xi = in.xi, tol = in.tol;

    // Gaussian support
    int P = in.force_P;
    if (P <= 0) {
        P = 4;
        // the stresslet's near-field Fourier part (third derivatives)
        // amplifies the support truncation about tenfold; so does the FP64
        // path's quadrature of the correction gradient with grad W, whose
        // aliasing error on the grid is larger than W's by about the ratio of
        // the grid's wave number to xi (measured at P = 10: about 45 times,
        // 3.1e-5 where the Gaussian's own truncation is 6.9e-7)
        const double pbudget = (tol < 1e-6 || in.family == 1 || p.prec == 1) ? tol / 40 : tol / 4;
        while (std::exp(-pi * P * C_SHAPE * C_SHAPE / 2) > pbudget) P += 2;
        // the stresslet's correction density carries the second derivatives
        // of the Gaussian, a^2 d^2 W with a = 2 xi^2 / eta, whose rounding the
        // harmonic multiplier does not damp: its error grows like a (measured
        // at N = 1e5, tol 1e-10: 3.5e-12 and 4.7e-11 at 300 and 30
        // neighbours, rising with M at fixed xi), and two more support nodes,
        // which widen the Gaussian (eta grows with P), bring it to the
        // separate grids' level (1.2e-12, 1.2e-11)
        if (in.family == 1 && p.prec == 1 && !in.free && in.dgrid > 0) P += 2;
    }
    if (P < 2 || P > 30 || (P & 1)) return -1;
    // the quadrature forms the gradient of the correction potential with the
    // gradient of the Gaussian: it weights the smooth potential by grad W,
    // whose truncation error is larger by about sqrt(a) times the potential's
    // length scale, so the gather truncates the same Gaussian further out
    // (FP64 only: the FP32 path transforms the gradient spectrally)
    int Pg = P + (in.gather_extra >= 0 ? in.gather_extra : (p.prec == 1 && !in.free ? 2 : 0));
    if (Pg > 30 || (Pg & 1)) return -1;
    // spreading support: P, or P + 2 (P + 6 for the stresslet's second
    // derivatives) when the correction density D is spread with derivative
    // weights; the choice is made below, once M~ is known
    const int Pd = P + (in.family == 1 ? 6 : 2);
    // the density on request needs its support within the 30 nodes; by cost
    // it is only a candidate when it fits
    const bool dens_fits = Pd <= 30;
    if (in.dgrid > 0 && p.prec == 1 && !in.free && !dens_fits) return -1;
    // the density's derivative weights leave a rounding floor of about 1e-13
    // relative (measured at N = 400, ~120 neighbours, tol 1e-13: the rotlet
    // 1.1e-13 with the density and 5.7e-14 with the separate grids; the
    // stokeslet 7.2e-14 with either), so auto mode takes it only from tol
    // 1e-12 up
    const bool dens_tol = in.dgrid > 0 || tol >= 1e-12;
    // (the stresslet's density in auto mode is planned by the plan made again
    // with it, below: this plan is the separate grids' and is not widened)
    const bool dens_cand = p.prec == 1 && in.dgrid != 0 && !in.free && dens_fits && dens_tol &&
                           !(in.family == 1 && in.dgrid < 0);
    const int Pe = std::max(std::max(P, Pg), dens_cand ? Pd : P);
    // grid intervals over the box
    int M = in.force_M;
    if (M <= 0) {
        M = 4;
        const double budget = in.family == 2 ? tol / 40 : tol / 4;
        while (est_fourier_rel(in.family, pi * M / L, xi, L) > budget) {
            if (++M > EHS_MT_MAX) return -3;
        }
        while (P * xi * xi * (L / M) * (L / M) / (C_SHAPE * C_SHAPE * pi) >= 0.95) {
            if (++M > EHS_MT_MAX) return -3;
        }
    }
    double h = L / M;
    double eta = P * xi * xi * h * h / (C_SHAPE * C_SHAPE * pi);
    if (!(eta < 1.0)) return -3;
    double m = std::sqrt(2.0 * std::log(1.0 / tol));
    int ext = std::max(Pe, (int)std::ceil(m / (std::sqrt(2.0) * xi * h)));
    int Mt = in.force_Mt > 0 ? in.force_Mt : next_smooth_even(M + ext);
    if (Mt < M + Pe || (Mt & 1) || !smooth7(Mt) || Mt > EHS_MT_MAX) return -3;
    p.M = M;
    p.P = P;
    p.Pg = Pg;
    // D-grid spreading (FP64): saves (ncB - 1) forward transform components
    // of the grid at the price of (Pd^3 - P^3) more spreading work per point;
    // the unit costs are those measured on MI355X for the two passes (about
    // 10 ms per component at M~ = 480 and 4.4 ns per point and P^3 node)
    // the stresslet in auto mode: its density needs two more support nodes
    // (above), which change the whole plan, so the choice is made on this
    // plan's grid and, for the density, the plan is made again with it.  The
    // density saves 6 of 13 forward components, measured at about
    // 1.5e-7 ms Mt^3 each pass set, and its image records and larger support
    // cost about 3.5e-9 ms per point and node of ((P + 8)^3 - P^3)
    // (spreading and quadrature together; measured on MI355X: the density
    // runs 0.61-0.87 of the grids' time from 130 grid nodes per point up,
    // 1.07-1.37 below)
    if (in.family == 1 && p.prec == 1 && !in.free && in.dgrid < 0 && in.force_P <= 0 && dens_tol) {
        const double save = 1.5e-7 * (double)Mt * Mt * Mt * 6.0;
        const double cost = 3.5e-9 * (double)in.N * ((double)(P + 8) * (P + 8) * (P + 8) - (double)P * P * P);
        if (save > cost) {
            // (at the tightest tolerances the wider density support exceeds
            // the supported 30 nodes: the separate grids then remain)
            PlanInput in2 = in;
            in2.dgrid = 1;
            const int r = make_plan(in2, out);
            if (r == 0) return 0;
        }
    }
    {
        bool dg = false;
        // (the stresslet: on request, or chosen above)
        if (dens_cand && (in.family != 1 || in.dgrid > 0)) {
            int ncB = in.family == 0 ? 4 : in.family == 1 ? 7 : 2;
            double save = 10.0 * std::pow(Mt / 480.0, 3) * (ncB - 1);
            double cost = 4.4e-9 * 2.0 * (double)in.N * ((double)Pd * Pd * Pd - (double)P * P * P) *
                          (in.family == 1 ? 2.0 : 1.0);
            dg = in.dgrid > 0 || save > cost;
        }
        // the grids chosen over a candidate density: M~ without the density's
        // wider support
        if (dens_cand && !dg && in.force_Mt <= 0) {
            const int extg = std::max(std::max(P, Pg), (int)std::ceil(m / (std::sqrt(2.0) * xi * h)));
            Mt = std::min(Mt, next_smooth_even(M + extg));
        }
        p.dgrid = dg;
        p.Ps = dg ? Pd : P;
        p.ncin = ncin_for(in.family, in.free ? CM_FREE : dg ? CM_DENSITY : CM_GRIDS);
    }
    p.Mt = Mt;
    p.h = h;
    p.Lt = Mt * h;
    p.eta = eta;
    p.nf = next_smooth_even((1.0 + std::sqrt(6.0)) * Mt);
    p.nf3 = next_smooth_even((2.0 + std::sqrt(6.0)) * Mt);
    // the precompute transforms one line of each length per 256-thread block
    for (int n : {p.nf, p.nf3, 2 * Mt, 4 * Mt})
        if (n > lds_fft_cap(n, 256)) return -3;
    p.est_f = est_fourier_rel(in.family, pi / h, xi, L);
    p.est_r = est_real_rel(in.family, in.rc, xi, L);
    if (p.est_r > tol / 2) p.warnings |= 1;

    // fused x3 pass: smallest number of phases whose lines fit one wavefront's
    // FFT and whose max(ncin, 6) lines fit the LDS
    const size_t esz = p.prec == 1 ? 8 : 4;
    const int cm = plan_cm(p);
    const int nl = std::max(p.ncin, ncout_for(p.prec, cm));
    p.Qz = 0;
    for (int Q : {2, 4, 8}) {
        if ((4 * Mt) % Q) continue;
        int nq = 4 * Mt / Q;
        if (!smooth7(nq)) continue;
        if (nq > lds_fft_cap(nq, 64)) continue;  // one line per wavefront
        if (z_lds_bytes(in.family, cm, Mt, Q, esz) > 150 * 1024) continue;
        p.Qz = Q;
        break;
    }
    if (!p.Qz) return -3;
    p.resident = z_resident_ok(in.family, Mt);
    // y / x3 pipeline: groups of zg k1 slabs pass through forward y, the fused
    // x3 pass and inverse y back to back, through a buffer of zg slabs (at most
    // ZSLAB_BUDGET bytes) instead of the whole padded spectrum
    {
        size_t slab = (size_t)nl * (2 * Mt) * (2 * Mt) * 2 * esz;
        if (!p.resident) slab += (size_t)ncout_for(p.prec, cm) * (2 * Mt) * (2 * Mt) * 2 * esz;
        long long g = in.force_zg > 0 ? in.force_zg : (long long)(ZSLAB_BUDGET / slab);
        p.zg = (int)std::max(1LL, std::min(g, (long long)Mt + 1));
    }
    p.Bx = choose_lines(Mt, esz);
    p.By = p.Bx;
    if (p.Bx < 2 || p.By < 1) return -3;

    // real-space cells (x3 measured from the wall): side >= r_c / nr
    double extent[3] = {ext1, ext2, ext3};
    const double occ = weighted_occupancy(extent, in.rc, in.T, in.zhist, in.zbin);
    int nr = occ < 256.0 ? 1 : occ < 1500.0 ? 2 : 3;
    if (in.force_nr >= 1 && in.force_nr <= 3) nr = in.force_nr;
    p.occ = occ;
    p.cg.nr = nr;
    long long ncell = 1;
    for (int a = 0; a < 3; ++a) {
        int nc = (int)std::floor(extent[a] * nr / in.rc);
        nc = std::max(1, std::min(nc, 256));
        p.cg.nc[a] = nc;
        p.cg.lo[a] = (a < 2 || in.free) ? in.lo[a] : 0.0;
        double side = extent[a] > 0 ? extent[a] / nc : 1.0;
        p.cg.inv[a] = 1.0 / side;
        ncell *= nc;
    }
    p.ncell = ncell;
    p.max_chunks = (in.T + 63) / 64 + std::min(ncell, in.T);

    // spreading tiles
    GridArgs& g = p.g;
    g.Mt = Mt;
    g.P = p.Ps;
    g.o[0] = in.lo[0] - Pe * h / 2;
    g.o[1] = in.lo[1] - Pe * h / 2;
    // half space: the wall x3 = 0 is node M~ (the images below it); free
    // space: placed like x1 and x2, so that the upper half stays empty
    g.o[2] = in.free ? in.lo[2] - Pe * h / 2 : -p.Lt;
    g.h = h;
    g.a2 = 2 * xi * xi / eta;
    g.mP = magic_of((unsigned)p.Ps);
    g.pref = std::pow(2 * xi * xi / (pi * eta), 1.5);
    // spreading tile depth: 4 x3 nodes per lane where the points are dense
    // (more wavefronts per SIMD hide the records' latency), 8 where they are
    // sparse (fewer record visits); the stresslet's 13 grids always take 4.
    // Measured (ms, depth 8 -> 4): clustered N = 4e6 120 -> 87 (18.5 points
    // per 8^3 tile), N = 1e6 rotlet 24.7 -> 17.9 (31), stresslet 42.6 ->
    // 35.7; N = 1e5 at ~415 neighbours 2.62 -> 2.84 (5.1) and at ~30
    // neighbours 3.6 -> 4.5 (0.46)
    const double per_tile8 = (in.free ? 1.0 : 2.0) * (double)in.N /
                             ((double)((Mt + 7) / 8) * ((Mt + 7) / 8) * ((2 * Mt + 7) / 8));
    int tz = (in.family == 1 || per_tile8 >= 10.0) ? 4 : 8;
    int dims[3] = {Mt, Mt, 2 * Mt};
    int tl[3] = {8, 8, tz};
    p.ntiles = 1;
    for (int a = 0; a < 3; ++a) {
        g.tile[a] = tl[a];
        g.nt[a] = (dims[a] + tl[a] - 1) / tl[a];
        g.K[a] = (p.Ps - 1 + tl[a] - 1) / tl[a];
        p.ntiles *= g.nt[a];
    }
    p.gg = g;
    p.gg.P = Pg;
    p.gg.mP = magic_of((unsigned)Pg);
    // quadrature tiles: 8 x 8 x 8 nodes, each owned by one wavefront.  The
    // node-owner form reads each grid node once but pays a reduction per
    // (target, tile), about 45 ns per target on MI355X whatever the density;
    // the one-wavefront forms re-read nodes through L2, cheaper the denser
    // the targets (the grouped form shares the reads of four nearby targets).
    // Node-owner only for large supports at low target density: FP64
    // N = 1e5 (Pg = 22, 0.9e-3 targets per node) 4.6 ms against 7.0 for the
    // grouped form; N = 1e6 (1.7e-2 per node) 44 ms against 28.5 for the
    // one-target form (grouped: about 11); FP32 (Pg = 10) 0.8 ms against
    // 0.34 for the one-target form.
    {
        // nodes from the lowest target's support up (the x3 range computed
        // as l3lo below)
        double zt = in.free ? in.tlo3 : std::max(in.tlo3, 0.0);
        long long b = (long long)std::floor((zt - g.o[2]) / h) - Pg / 2;
        b = std::max(0LL, std::min(b, (long long)(2 * Mt - Pg)));
        double nodes = (double)Mt * Mt * (double)(2 * Mt - b);
        // (free space: the target-per-wavefront form, which has its output layout)
        p.gtiles = !in.free && Pg >= 16 && (double)in.T < 3e-3 * nodes;
    }
    // dense targets: several per wavefront, sharing the walk over their supports
    p.ggroup = !p.gtiles && gather_group_fits(Pg, Mt, p.prec == 1 ? 8 : 4);
    p.ntiles_g = 1;
    for (int a = 0; a < 3; ++a) {
        p.gg.tile[a] = 8;
        p.gg.nt[a] = (dims[a] + 7) / 8;
        p.gg.K[a] = (Pg - 1 + 7) / 8;
        p.ntiles_g *= p.gg.nt[a];
    }
    // The targets lie at x3 >= tlo3 >= 0, so the quadrature never reads the
    // lower part of the x3 range (the image side of the box): the inverse
    // transforms produce only nodes from the support base of the lowest
    // target, less one node of margin, rounded down to a multiple of 16 (one
    // 128-byte row segment of the y passes).
    {
        double zt = in.free ? in.tlo3 : std::max(in.tlo3, 0.0);
        long long b = (long long)std::floor((zt - g.o[2]) / h) - Pg / 2;
        b = std::max(0LL, std::min(b, (long long)(2 * Mt - Pg)));
        p.l3lo = (int)(b / 16) * 16;
    }
    // The correction sources sit at the images, x3 <= -slo3 < 0: the grids
    // spread from them (every component from ncA on) vanish above the top of
    // the highest image's support, which the forward transforms skip.  One
    // node of margin, rounded up to a multiple of 16.
    {
        // (free space: every grid vanishes above the top of the highest
        // point's support, and the forward passes skip those rows for all
        // components)
        double zi = in.free ? in.hi[2] : -std::max(in.slo3, 0.0);
        long long t = (long long)std::floor((zi - g.o[2]) / h) + p.Ps / 2 + 2;
        t = std::max(0LL, std::min(t, (long long)(2 * Mt)));
        p.lzc = (int)std::min((long long)(2 * Mt), ((t + 15) / 16) * 16);
    }
    *out = p;
    return 0;
}

}  // namespace ehs
