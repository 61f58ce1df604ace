// Real-space (short-range) part of the half-space Ewald sum.
//
// One wavefront per chunk of <= 64 targets of one cell (cells have side
// >= r_c / nr, so the neighbours lie within nr cells).  All lanes walk the
// same neighbour-cell source ranges (staged in LDS per batch); each lane
// accumulates its own target.  Direct terms
// use the Ewald real-space kernels S_R, T_R, W_R (paper Sec. 4 and Appendix);
// image and correction terms use the same kernels at r~ = x - y^I together
// with the real-space parts of G, grad G, grad grad G and grad grad grad G
// (paper eq. (G_R), written with erfc instead of 1 - erf).  Only targets in
// the bottom nr cell layers can be within r_c of an image.
#include <math.h>

#include <type_traits>

#include "common.h"
#include "erfc_poly.h"
#include "kernels.h"

namespace ehs {

// ---------------------------------------------------------------------------
// Arithmetic of one pair.  The library's sqrt, division and exp cover every
// input (denormals, overflow, infinities) in some twenty to thirty
// instructions each.  A pair here has 0 < r < r_c and 0 <= xi r <= xi r_c,
// so each is formed from the hardware estimate and one Newton step, or from a
// range reduction and a series, in about a third of that.
// ---------------------------------------------------------------------------

// a * b + c with the constant c in scalar registers.  With the coefficients
// of a polynomial in vector registers the compiler picks the accumulating
// FMA form, which overwrites its addend, and copies the coefficient before
// every use: a third more instructions for a Horner chain.
__device__ __forceinline__ double fma_sc(double a, double b, double c)
{
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
}

template <typename T>
struct PairMath;

template <>
struct PairMath<double> {
    // 1/sqrt(x), x > 0 normal: the hardware estimate y (relative error
    // about 2^-23) and one third-order Newton step y (1 + e/2 + 3e^2/8),
    // e = 1 - x y^2, which leaves an error of order e^3, below rounding
    static __device__ __forceinline__ double rsqrt(double x)
    {
        const double y = __builtin_amdgcn_rsq(x);
        const double e = fma(-x * y, y, 1.0);
        return fma(y * e, fma(e, 0.375, 0.5), y);
    }
    // 1/x, 1 <= x <= 8: the hardware estimate and the step y (1 + e + e^2),
    // e = 1 - x y
    static __device__ __forceinline__ double rcp(double x)
    {
        const double y = __builtin_amdgcn_rcp(x);
        const double e = fma(-x, y, 1.0);
        return fma(y * e, 1.0 + e, y);
    }
    // e^y, -700 < y <= 0: y = k ln2 + f, k = rint(y / ln2), |f| <= ln2 / 2,
    // with ln2 split in two parts so that k ln2 is exact to 2^-60; e^f by its
    // Taylor series to the f^12 term (truncation below 2.5e-16 relative);
    // 2^k applied to the exponent
    static __device__ __forceinline__ double exp(double y)
    {
        const double k = __builtin_rint(y * 1.4426950408889634074);
        double f = fma(-k, 6.93147180369123816490e-01, y);
        f = fma(-k, 1.90821492927058770002e-10, f);
        double p = 1.0 / 479001600.0;  // 1/12!
        p = fma_sc(p, f, 1.0 / 39916800.0);
        p = fma_sc(p, f, 1.0 / 3628800.0);
        p = fma_sc(p, f, 1.0 / 362880.0);
        p = fma_sc(p, f, 1.0 / 40320.0);
        p = fma_sc(p, f, 1.0 / 5040.0);
        p = fma_sc(p, f, 1.0 / 720.0);
        p = fma_sc(p, f, 1.0 / 120.0);
        p = fma_sc(p, f, 1.0 / 24.0);
        p = fma_sc(p, f, 1.0 / 6.0);
        p = fma_sc(p, f, 0.5);
        p = fma_sc(p, f, 1.0);
        p = fma_sc(p, f, 1.0);
        return __builtin_amdgcn_ldexp(p, (int)k);
    }
    // erfc(x), x >= 0, from E = exp(-x^2), which the Gaussian terms need
    // anyway: erfc(x) = E q(t), t = 1 / (1 + x / 2), q a fitted polynomial
    // (erfc_poly.h).  The library erfc branches over ranges of x, and a
    // wavefront's pairs span 0 <= x < xi r_c and take several branches.
    static __device__ __forceinline__ double erfc_e(double x, double E)
    {
        const double t = rcp(fma(0.5, x, 1.0));
        double q = ERFC_C64[ERFC_DEG64];
#pragma unroll
        for (int k = ERFC_DEG64 - 1; k >= 0; --k) q = fma_sc(q, t, ERFC_C64[k]);
        return E * q;
    }
};

template <>
struct PairMath<float> {
    // the FP32 estimates are within about 1 ulp: no refinement
    static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    // e^y = 2^(y log2 e) by the hardware exp2: the rounding of the product
    // adds |y| 2^-24 relative, below 1e-6 for the arguments of FP32 plans
    // (xi r_c about 3.5 at tol 1e-5, so |y| < 13)
    static __device__ __forceinline__ float exp(float y) { return __builtin_amdgcn_exp2f(y * 1.44269504088896341f); }
    static __device__ __forceinline__ float erfc_e(float x, float E)
    {
        const float t = rcp(fmaf(0.5f, x, 1.0f));
        float q = ERFC_C32[ERFC_DEG32];
#pragma unroll
        for (int k = ERFC_DEG32 - 1; k >= 0; --k) q = fmaf(q, t, ERFC_C32[k]);
        return E * q;
    }
};

// direct term K_R(r) s, r != 0, written to out
template <typename T, int K>
__device__ __forceinline__ void direct_term(T rx, T ry, T rz, T r2, const T* s, T xi, T c2, T* out)
{
    using PM = PairMath<T>;
    const T ir = PM::rsqrt(r2);
    const T r = r2 * ir;
    const T E = PM::exp(-xi * xi * r2);
    const T C = PM::erfc_e(xi * r, E);
    if (K == STOKESLET) {
        // S_R f = (a - 2 c2 E) f + a (r.f) r / r^2,  a = c2 E + C / r
        T a = c2 * E + C * ir;
        T rf = rx * s[0] + ry * s[1] + rz * s[2];
        T b = a * rf * ir * ir;
        T d = a - (T)2 * c2 * E;
        out[0] = d * s[0] + b * rx;
        out[1] = d * s[1] + b * ry;
        out[2] = d * s[2] + b * rz;
    } else if (K == STRESSLET) {
        // T_R[S] = A (r.S r) r + Bc (2 S r + r tr S)
        T ir2 = ir * ir;
        T A = (T)-2 * ir2 * ir2 * ((T)3 * C * ir + c2 * ((T)3 + (T)2 * xi * xi * r2) * E);
        T Bc = (T)2 * xi * xi * c2 * E;
        T sr0 = s[0] * rx + s[1] * ry + s[2] * rz;
        T sr1 = s[1] * rx + s[3] * ry + s[4] * rz;
        T sr2 = s[2] * rx + s[4] * ry + s[5] * rz;
        T rsr = rx * sr0 + ry * sr1 + rz * sr2;
        T tr = s[0] + s[3] + s[5];
        T g = A * rsr;
        out[0] = g * rx + Bc * ((T)2 * sr0 + rx * tr);
        out[1] = g * ry + Bc * ((T)2 * sr1 + ry * tr);
        out[2] = g * rz + Bc * ((T)2 * sr2 + rz * tr);
    } else {
        // W_R v = 2 alpha (v x r), alpha = C / r^3 + c2 E / r^2
        T al = (T)2 * (C * ir * ir * ir + c2 * E * ir * ir);
        out[0] = al * (s[1] * rz - s[2] * ry);
        out[1] = al * (s[2] * rx - s[0] * rz);
        out[2] = al * (s[0] * ry - s[1] * rx);
    }
}

// image kernel term plus the harmonic corrections -x3 grad phi_R + e3 phi_R
// of one source (strength s, height y3) at r~ = x - y^I, written to out
template <typename T, int K>
__device__ __forceinline__ void image_term(T rx, T ry, T rz, T r2, const T* s, T y3, T x3, T xi, T c2, T* out)
{
    using PM = PairMath<T>;
    const T ir = PM::rsqrt(r2);
    const T r = r2 * ir;
    const T ir2 = ir * ir;
    const T E = PM::exp(-xi * xi * r2);
    const T C = PM::erfc_e(xi * r, E);
    T xi2 = xi * xi;
    // grad G_R = -alpha r, grad grad G_R = -alpha I + beta r r,
    // grad grad grad G_R = beta (d r)_sym + gamma r r r
    T al = C * ir2 * ir + c2 * E * ir2;
    T be = (T)3 * C * ir2 * ir2 * ir + c2 * E * ((T)3 * ir2 * ir2 + (T)2 * xi2 * ir2);
    T phi, g0, g1, g2, k0, k1, k2;  // k: the image kernel term
    if (K == STOKESLET) {
        T f0 = s[0], f1 = s[1], f2 = -s[2];  // f^I
        T a = c2 * E + C * ir;
        T rf = rx * f0 + ry * f1 + rz * f2;
        T b = a * rf * ir2;
        T d = a - (T)2 * c2 * E;
        k0 = -(d * f0 + b * rx);
        k1 = -(d * f1 + b * ry);
        k2 = -(d * f2 + b * rz);
        // phi = -2 f3 G_R - 2 y3 f^I . grad G_R
        T f3 = s[2];
        phi = (T)-2 * f3 * C * ir + (T)2 * y3 * al * rf;
        T u = (T)2 * f3 * al - (T)2 * y3 * be * rf;
        T v = (T)2 * y3 * al;
        g0 = u * rx + v * f0;
        g1 = u * ry + v * f1;
        g2 = u * rz + v * f2;
    } else if (K == STRESSLET) {
        // S^I = R S R: flip the xz, yz entries
        T s0 = s[0], s1 = s[1], s2 = -s[2], s3 = s[3], s4 = -s[4], s5 = s[5];
        T A = (T)-2 * ir2 * ir2 * ((T)3 * C * ir + c2 * ((T)3 + (T)2 * xi2 * r2) * E);
        T Bc = (T)2 * xi2 * c2 * E;
        T sr0 = s0 * rx + s1 * ry + s2 * rz;
        T sr1 = s1 * rx + s3 * ry + s4 * rz;
        T sr2 = s2 * rx + s4 * ry + s5 * rz;
        T rsr = rx * sr0 + ry * sr1 + rz * sr2;
        T tr = s0 + s3 + s5;
        T gk = A * rsr;
        k0 = -(gk * rx + Bc * ((T)2 * sr0 + rx * tr));
        k1 = -(gk * ry + Bc * ((T)2 * sr1 + ry * tr));
        k2 = -(gk * rz + Bc * ((T)2 * sr2 + rz * tr));
        T ga = (T)-15 * C * ir2 * ir2 * ir2 * ir -
               c2 * E * ((T)15 * ir2 * ir2 * ir2 + (T)10 * xi2 * ir2 * ir2 + (T)4 * xi2 * xi2 * ir2);
        // phi = 4 tr dG_R/dx3 - 4 y3 grad grad G_R : S^I
        phi = (T)-4 * al * rz * tr + (T)4 * y3 * al * tr - (T)4 * y3 * be * rsr;
        // grad phi = 4 tr (-alpha e3 + beta r3 r) - 4 y3 [beta (tr r + 2 S^I r) + gamma (r.S^I r) r]
        T u = (T)4 * tr * be * rz - (T)4 * y3 * (be * tr + ga * rsr);
        T v = (T)-8 * y3 * be;
        g0 = u * rx + v * sr0;
        g1 = u * ry + v * sr1;
        g2 = u * rz + v * sr2 - (T)4 * tr * al;
    } else {
        // + W_R(r~) v^I
        T v0 = s[0], v1 = s[1], v2 = -s[2];
        T a2 = (T)2 * al;
        k0 = a2 * (v1 * rz - v2 * ry);
        k1 = a2 * (v2 * rx - v0 * rz);
        k2 = a2 * (v0 * ry - v1 * rx);
        // w = 2 (-v2, v1, 0); phi = 2 w . grad G_R; grad phi = 2 grad grad G_R w
        T w0 = (T)-2 * s[1], w1 = (T)2 * s[0];
        T rw = rx * w0 + ry * w1;
        phi = (T)-2 * al * rw;
        T u = (T)2 * be * rw;
        g0 = u * rx - (T)2 * al * w0;
        g1 = u * ry - (T)2 * al * w1;
        g2 = u * rz;
    }
    out[0] = k0 - x3 * g0;
    out[1] = k1 - x3 * g1;
    out[2] = k2 + (phi - x3 * g2);
}

// LDS add of one contribution to a target's accumulator.  All pairs of a
// chunk are evaluated by its one wavefront, so the adds to an accumulator
// happen in the order of its instructions and, within one instruction, in
// the order the LDS serves the lanes: the same for the same input.
template <typename T>
__device__ __forceinline__ void lds_add(T* p, T v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Pair compaction.  A wavefront owns <= 64 targets of one cell (one lane
// each) and walks the sources of the neighbour cells in batches of SB.  Only
// a fraction of the (target, source) candidates lie within r_c (a third for
// cells of side r_c / 3, a sixth for side r_c), and a lane-per-target loop
// would evaluate the kernel for every candidate with most lanes idle.
// Instead, per batch:
//   1. each lane tests its target against the SB sources (wave-uniform
//      loads); the hits are written, in (source, lane) order, to a pair list
//      in LDS;
//   2. the lanes evaluate the listed pairs, one pair per lane, and add each
//      contribution to its target's accumulator in LDS (lds_add).
// Batches of 16 sources keep the pair lists long (at high densities hundreds
// of pairs per batch), so the evaluation passes run with nearly every lane
// busy.  The accumulation by LDS adds replaced a per-target sum in source
// order out of a contribution buffer, whose bookkeeping cost more
// instructions per pair than the pair's own arithmetic: the clustered
// N = 4e6 set issued about 290 instructions per lane and pair.

// PASS_IMG = false: the direct terms of every chunk (and the self term),
// written to upart; PASS_IMG = true: the image and correction terms of the chunks in the
// bottom nr cell layers, in FP64, added to upart.  Two launches rather than
// one kernel: the FP64 image terms need many more registers than the direct
// ones, and in one kernel they would set the occupancy of every chunk.
// Chunks go to the XCDs in runs of RS_RUN consecutive ones: block b runs on
// XCD b % 8, and XCD k takes runs k, k + 8, k + 16, ... in order, so that
// neighbouring chunks, which read the same source cells, share an L2, while
// every XCD still takes its share of each region of the cell order (the
// dense bottom layers come first; one contiguous range per XCD would leave
// them to one or two).  The grid is padded to a multiple of 8 RS_RUN blocks;
// chunks past the count exit.  (Clustered N = 4e6 stokeslet: HBM fetch of
// the direct pass 71.5 -> 54.4 GB per evaluation, time unchanged: the pass
// is bound by instruction issue.)
constexpr int RS_RUN = 64;
__device__ __forceinline__ long long chunk_of_block(long long b)
{
    const long long q = b / NXCD;  // position in the XCD's sequence
    return ((q / RS_RUN) * NXCD + b % NXCD) * RS_RUN + q % RS_RUN;
}

template <typename T, int K, bool PASS_IMG>
__global__ void __launch_bounds__(64) k_realspace(RealArgs a, const double* __restrict__ ys,
                                                  const double* __restrict__ ss, const double* __restrict__ xt,
                                                  double* __restrict__ upart)
{
    constexpr int NS = (K == STRESSLET) ? 6 : 3;
    // sources per batch: their pairs are listed at once and evaluated in
    // windows of the contribution slots (SB 64 entries of 16 bits: the source
    // index in the batch is stored above the lane)
    constexpr int SB = 16;
    constexpr int SBI = 8;  // image sources per batch (FP64 contributions)
    constexpr int SW = 3 + NS;                  // staged values per source
    __shared__ uint16_t plist[64 * SB];
    __shared__ double sb[SB * SW];
    __shared__ double tpos[3 * 64];
    // (FP64 accumulators in both precisions: the LDS adds of FP32 values ran
    // the FP32 kernel at less than half the speed of the FP64 adds)
    __shared__ double acc_l[PASS_IMG ? 1 : 3 * 64];    // direct terms, per target
    __shared__ double acci_l[PASS_IMG ? 3 * 64 : 1];   // image terms, per target (FP64)
    const int lane = threadIdx.x;
    const long long w = chunk_of_block(blockIdx.x);
    if (w >= (long long)(*a.nchunks)) return;  // the whole (one-wavefront) block
    const uint32_t cell = a.chunk_cell[w];
    // (a target and a source can both lie within r_c of the wall only in the
    // bottom nr cell layers; the chunks run in cell order, so these come first)
    if (PASS_IMG && cell >= (uint32_t)(a.cg.nr * a.cg.nc[0] * a.cg.nc[1])) return;
    const uint32_t first = a.chunk_first[w];
    const int cnt = (int)min(64u, a.tgt_off[cell + 1] - first);
    const bool act = lane < cnt;
    const long long t = first + (act ? lane : 0);
    const long long N = a.N, TT = a.T;
    const double xd0 = xt[t], xd1 = xt[TT + t], xd2 = xt[2 * TT + t];
    tpos[lane] = xd0;
    tpos[64 + lane] = xd1;
    tpos[128 + lane] = xd2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (PASS_IMG)
            acci_l[3 * lane + c] = 0.0;
        else
            acc_l[3 * lane + c] = 0.0;
    }
    const int n0 = a.cg.nc[0], n1 = a.cg.nc[1], n2 = a.cg.nc[2];
    const int c1 = (int)(cell % (uint32_t)n0);
    const int c2i = (int)((cell / (uint32_t)n0) % (uint32_t)n1);
    const int c3 = (int)(cell / ((uint32_t)n0 * (uint32_t)n1));
    const T xi = (T)a.xi;
    const T c2 = (T)(2.0 * a.xi / 1.7724538509055160273);
    const double rc2 = a.rc2;
    double self[3] = {0.0, 0.0, 0.0};
    unsigned long long npair[2] = {0ull, 0ull};  // direct, image (wave-uniform)
    const int nr = a.cg.nr;  // cells of side >= r_c / nr: neighbours within nr cells
    const unsigned long long live = __builtin_amdgcn_ballot_w64(act);  // lanes with a target

    // one batch of sources [mb, mb + nb) of the sorted arrays; IMG: their
    // images (and harmonic corrections) instead of the direct terms; every
    // pair's contribution is added to its target's accumulator in LDS.
    // OWN: the row of cells holds the target's own cell, the only one where
    // a source can coincide with it (r = 0: excluded, with the self term)
    auto batch = [&](uint32_t mb, int nb, auto img_tag, auto own_tag) {
        constexpr bool IMG = decltype(img_tag)::value;
        constexpr bool OWN = decltype(own_tag)::value;
        constexpr int B = IMG ? SBI : SB;
        for (int f = lane; f < nb * SW; f += 64) {
            const int jj = f / SW, c = f - jj * SW;
            sb[f] = c < 3 ? ys[c * N + mb + jj] : ss[(c - 3) * N + mb + jj];
        }
        wave_sync();
        // every lane forms r^2 for every slot of the batch (slots past nb hold
        // the previous batch's sources, which the mask drops): no branches,
        // and the hits are the compare's own lane mask
        int pre = 0;  // wavefront-uniform
#pragma unroll 4
        for (int j = 0; j < B; ++j) {
            const double* s = sb + j * SW;
            const double dx = xd0 - s[0], dy = xd1 - s[1], dz = IMG ? xd2 + s[2] : xd2 - s[2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            bool in = r2 < rc2;
            if (!IMG && OWN) {
                in = in & (r2 > 0.0);
                if (K == STOKESLET && act && j < nb && r2 == 0.0) {
                    // self interaction: limit of S_R - S at r = 0 is -(4 xi / sqrt(pi)) I
                    const double cs = 4.0 * a.xi / 1.7724538509055160273;
                    self[0] -= cs * s[3];
                    self[1] -= cs * s[4];
                    self[2] -= cs * s[5];
                }
            }
            const bool hit = in & act & (j < nb);
            // (the lane mask of the compare itself: a ballot of the bool
            // would form it again from a select and a compare)
            unsigned long long m = 0ull;
            if (j < nb) m = (IMG || !OWN ? __builtin_amdgcn_fcmp(r2, rc2, 4 /* ordered < */)
                                         : __builtin_amdgcn_ballot_w64(in)) & live;
            const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            if (hit) plist[pre + below] = (uint16_t)(lane | (j << 6));
            pre += __popcll(m);
        }
        wave_sync();
        const int np = pre;
        npair[IMG ? 1 : 0] += (unsigned long long)np;
        for (int q = lane; q < np; q += 64) {
            const int pr = plist[q], tl = pr & 63, j = pr >> 6;
            const double* s = sb + j * SW;
            const double px = tpos[tl], py = tpos[64 + tl], pz = tpos[128 + tl];
            if (IMG) {
                const double y3 = s[2];
                const double dx = px - s[0], dy = py - s[1], dz = pz + y3;
                double sv[NS], ci[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int c = 0; c < NS; ++c) sv[c] = s[3 + c];
                image_term<double, K>(dx, dy, dz, dx * dx + dy * dy + dz * dz, sv, y3, pz, a.xi,
                                      2.0 * a.xi / 1.7724538509055160273, ci);
#pragma unroll
                for (int c = 0; c < 3; ++c) lds_add(&acci_l[3 * tl + c], ci[c]);
            } else {
                const double dx = px - s[0], dy = py - s[1], dz = pz - s[2];
                T sv[NS], cd[3] = {0, 0, 0};
#pragma unroll
                for (int c = 0; c < NS; ++c) sv[c] = (T)s[3 + c];
                direct_term<T, K>((T)dx, (T)dy, (T)dz, (T)(dx * dx + dy * dy + dz * dz), sv, xi, c2, cd);
#pragma unroll
                for (int c = 0; c < 3; ++c) lds_add(&acc_l[3 * tl + c], (double)cd[c]);
            }
        }
        wave_sync();  // the next batch overwrites the lists
    };

    // Only cells within r_c of the target's cell are walked: a row of cells at
    // (x2, x3) offsets whose nearest points lie m^2 apart in (x2, x3) needs
    // the x1 offsets |d1| with ((|d1| - 1) side1)^2 + m^2 < r_c^2 (the cells
    // of the (2 nr + 1)^3 block at the far corners and edges hold no pair;
    // about 9 % of the candidates for nr = 3)
    const double hc1 = 1.0 / a.cg.inv[0], hc2 = 1.0 / a.cg.inv[1], hc3 = 1.0 / a.cg.inv[2];
    auto x_reach = [&](double m2) -> int {
        if (m2 >= rc2) return -1;
        const int r = (int)ceil(sqrt(rc2 - m2) / hc1 * (1.0 + 1e-12));
        return r < nr ? r : nr;
    };
    // (the gaps are shrunk by 1e-12 relative, against the rounding of the
    // points' cell assignment)
    auto gap = [](int d, double side) {
        const int g = (d < 0 ? -d : d) - 1;
        return g > 0 ? g * side * (1.0 - 1e-12) : 0.0;
    };
    if (!PASS_IMG) {
        for (int d3 = -nr; d3 <= nr; ++d3) {
            int cc3 = c3 + d3;
            if (cc3 < 0 || cc3 >= n2) continue;
            const double g3 = gap(d3, hc3);
            for (int d2 = -nr; d2 <= nr; ++d2) {
                int cc2 = c2i + d2;
                if (cc2 < 0 || cc2 >= n1) continue;
                const double g2 = gap(d2, hc2);
                const int rx = x_reach(g2 * g2 + g3 * g3);
                if (rx < 0) continue;
                const int l1 = c1 - rx > 0 ? c1 - rx : 0, h1 = c1 + rx < n0 - 1 ? c1 + rx : n0 - 1;
                long long row = ((long long)cc3 * n1 + cc2) * n0;
                uint32_t s0 = a.src_off[row + l1], s1 = a.src_off[row + h1 + 1];
                if (d2 == 0 && d3 == 0) {
                    for (uint32_t mb = s0; mb < s1; mb += SB)
                        batch(mb, (int)min((uint32_t)SB, s1 - mb), std::false_type(), std::true_type());
                } else {
                    for (uint32_t mb = s0; mb < s1; mb += SB)
                        batch(mb, (int)min((uint32_t)SB, s1 - mb), std::false_type(), std::false_type());
                }
            }
        }
    }
    // Image and correction terms in FP64 in both precisions: for a source and
    // target near the wall they are of size 1/(x3 + y3)^2 and cancel to O(1)
    // on the wall, beyond what FP32 can resolve.  Only sources within r_c of
    // the wall have images here, and the x3 distance from a target in cell
    // layer c3 to the image of a source in layer cc3 is at least
    // (c3 + cc3) side3 (the cell layers start at the wall).
    if (PASS_IMG) {
        for (int cc3 = 0; cc3 < nr && cc3 < n2; ++cc3) {
            const double g3 = (c3 + cc3) * hc3 * (1.0 - 1e-12);
            for (int d2 = -nr; d2 <= nr; ++d2) {
                int cc2 = c2i + d2;
                if (cc2 < 0 || cc2 >= n1) continue;
                const double g2 = gap(d2, hc2);
                const int rx = x_reach(g2 * g2 + g3 * g3);
                if (rx < 0) continue;
                const int l1 = c1 - rx > 0 ? c1 - rx : 0, h1 = c1 + rx < n0 - 1 ? c1 + rx : n0 - 1;
                long long row = ((long long)cc3 * n1 + cc2) * n0;
                uint32_t s0 = a.src_off[row + l1], s1 = a.src_off[row + h1 + 1];
                for (uint32_t mb = s0; mb < s1; mb += SBI)
                    batch(mb, (int)min((uint32_t)SBI, s1 - mb), std::true_type(), std::false_type());
            }
        }
    }
    wave_sync();
    double acc[3];
    double acci[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[c] = PASS_IMG ? 0.0 : acc_l[3 * lane + c];
        acci[c] = PASS_IMG ? acci_l[3 * lane + c] : 0.0;
    }
    if (a.pairs && lane == 0) atomicAdd(a.pairs + (PASS_IMG ? 1 : 0), npair[PASS_IMG ? 1 : 0]);
    if (act) {
        long long o = a.tgt_perm[t];
        if (PASS_IMG) {
            // after the direct launch on the same stream
            upart[3 * o + 0] += acci[0];
            upart[3 * o + 1] += acci[1];
            upart[3 * o + 2] += acci[2];
        } else {
            upart[3 * o + 0] = (double)acc[0] + self[0];
            upart[3 * o + 1] = (double)acc[1] + self[1];
            upart[3 * o + 2] = (double)acc[2] + self[2];
        }
    }
}

template <typename T>
hipError_t launch_realspace(int family, const RealArgs& a, const double* ys, const double* ss, const double* xt,
                            double* upart, long long max_chunks, hipStream_t st)
{
    if (max_chunks <= 0) return hipSuccess;
    const long long span = (long long)NXCD * RS_RUN;
    dim3 grid((unsigned)((max_chunks + span - 1) / span * span));  // one wavefront per chunk
    // direct terms of every chunk, then the images of the bottom-layer chunks
    // (none in free space)
    if (!a.images) {
        switch (family) {
            case STOKESLET: hipLaunchKernelGGL((k_realspace<T, STOKESLET, false>), grid, dim3(64), 0, st, a, ys, ss, xt, upart); break;
            case STRESSLET: hipLaunchKernelGGL((k_realspace<T, STRESSLET, false>), grid, dim3(64), 0, st, a, ys, ss, xt, upart); break;
            default: hipLaunchKernelGGL((k_realspace<T, ROTLET, false>), grid, dim3(64), 0, st, a, ys, ss, xt, upart); break;
        }
        return hipGetLastError();
    }
    switch (family) {
        case STOKESLET:
            hipLaunchKernelGGL((k_realspace<T, STOKESLET, false>), grid, dim3(64), 0, st, a, ys, ss, xt, upart);
            hipLaunchKernelGGL((k_realspace<double, STOKESLET, true>), grid, dim3(64), 0, st, a, ys, ss, xt, upart);
            break;
        case STRESSLET:
            hipLaunchKernelGGL((k_realspace<T, STRESSLET, false>), grid, dim3(64), 0, st, a, ys, ss, xt, upart);
            hipLaunchKernelGGL((k_realspace<double, STRESSLET, true>), grid, dim3(64), 0, st, a, ys, ss, xt, upart);
            break;
        default:
            hipLaunchKernelGGL((k_realspace<T, ROTLET, false>), grid, dim3(64), 0, st, a, ys, ss, xt, upart);
            hipLaunchKernelGGL((k_realspace<double, ROTLET, true>), grid, dim3(64), 0, st, a, ys, ss, xt, upart);
            break;
    }
    return hipGetLastError();
}

template hipError_t launch_realspace<double>(int, const RealArgs&, const double*, const double*, const double*,
                                             double*, long long, hipStream_t);
template hipError_t launch_realspace<float>(int, const RealArgs&, const double*, const double*, const double*, double*,
                                            long long, hipStream_t);

}  // namespace ehs
