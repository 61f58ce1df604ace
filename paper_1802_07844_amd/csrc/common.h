// Shared device-side helpers of the MI355X half-space spectral Ewald library:
// complex arithmetic, the kernel-family traits and the LDS-resident mixed-radix
// Stockham FFT used by every transform pass.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ehs {

// ---------------------------------------------------------------------------
// complex numbers (interleaved re, im)
// ---------------------------------------------------------------------------
template <typename T>
struct alignas(2 * sizeof(T)) cplx {
    T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmk(T a, T b)
{
    cplx<T> r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return cmk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return cmk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b)
{
    return cmk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return cmk<T>(a.x, -a.y); }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return cmk<T>(a.x * s, a.y * s); }
// exchange of the real and imaginary parts: swap(z) = i conj(z), so that
// the inverse DFT is swap(DFT(swap(v))) (free in registers, unlike conj)
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cswap(cplx<T> a) { return cmk<T>(a.y, a.x); }
// multiply by -i
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmul_mi(cplx<T> a) { return cmk<T>(a.y, -a.x); }
// multiply by +i
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmul_pi(cplx<T> a) { return cmk<T>(-a.y, a.x); }

// ---------------------------------------------------------------------------
// kernel families and their grid-component counts
//   A-grids: the 2N consolidated sources (sources and their wall images);
//   B-grids: the correction sources, centred at the images only.
// ---------------------------------------------------------------------------
enum Family { STOKESLET = 0, STRESSLET = 1, ROTLET = 2 };

template <int K>
struct Traits;
template <>
struct Traits<STOKESLET> {
    static constexpr int nstr = 3;  // f
    static constexpr int ncA = 3;   // f at y, -f^I at y^I
    static constexpr int ncB = 4;   // f3 and y3 f^I at y^I
};
template <>
struct Traits<STRESSLET> {
    static constexpr int nstr = 6;  // (g, q)
    static constexpr int ncA = 6;   // sym(g q) at y, -R sym(g q) R at y^I
    static constexpr int ncB = 7;   // g.q and y3 R sym(g q) R at y^I
};
template <>
struct Traits<ROTLET> {
    static constexpr int nstr = 3;  // torque v = g x q
    static constexpr int ncA = 3;   // v at y, v^I at y^I
    static constexpr int ncB = 2;   // w = 2(-v2, v1) at y^I
};
// output grids of the transform pipeline: FP64 keeps Y1 (3 components) and
// the correction potential phi (1), whose gradient the quadrature forms with
// the gradient of the Gaussian; FP32 keeps Y1 and grad phi = IFFT(i k phi^)
// (3), because the FP32 quantisation of the long-range potential would be
// amplified by that gradient
// (free space keeps Y1 only: no images and no corrections).
//
// Correction modes of the grid pipeline (the CM template argument):
//   CM_GRIDS    the ncB correction grids, spread separately;
//   CM_DENSITY  the correction sources spread as one density D (FP64, below);
//   CM_FREE     the free-space sum of Sec. 2: sources only, no images, no
//               corrections, the kernel grid's three outputs.
enum CorrectionMode { CM_GRIDS = 0, CM_DENSITY = 1, CM_FREE = 2 };
constexpr int NCOUT_MAX = 6;
template <typename T, int CM>
struct Out {
    static constexpr int n = CM == CM_FREE ? 3 : sizeof(T) == 8 ? 4 : 6;
    static constexpr bool grad_quad = CM != CM_FREE && sizeof(T) == 8;  // gradient by quadrature
};
inline int ncout_for(int prec, int cm) { return cm == CM_FREE ? 3 : prec == 1 ? 4 : 6; }

// input grids: the kernel grid C1 (ncA components) and the correction
// sources.  FP64 spreads the correction sources directly as the one scalar
// density D whose transform enters the potential, phi^ = E H^R D^, using
// derivatives of the Gaussian:
//   stokeslet  D = -2 C2 - 2 div C3           (C2 = f3, C3 = y3 f^I at y^I)
//   stresslet  D = 4 d3 C2 - 4 grad grad : C3  (C2 = g.q, C3 = y3 sym(g^I q^I))
//   rotlet     D = 2 div C2                    (C2 = w)
// The derivative weights need a wider Gaussian support than plain spreading,
// so the planner uses D only where the saved transforms outweigh that (and
// only in FP64: the FP32 quantisation would be amplified by the derivative
// weights as in the quadrature); otherwise the ncB correction grids are
// spread separately.
template <int K, int CM>
struct InGrids {
    static constexpr int n = Traits<K>::ncA + (CM == CM_DENSITY ? 1 : CM == CM_FREE ? 0 : Traits<K>::ncB);
};
inline int ncin_for(int family, int cm)
{
    int ncA = family == 1 ? 6 : 3, ncB = family == 0 ? 4 : family == 1 ? 7 : 2;
    return ncA + (cm == CM_DENSITY ? 1 : cm == CM_FREE ? 0 : ncB);
}

// ---------------------------------------------------------------------------
// FFT plan for one line length: radices (each 2,3,4,5,7 or 8), the twiddle
// table tw[t] = exp(-2 pi i t / n), t < n, in device memory, and for every
// stage the index divisors with their multiply-high reciprocals (exact for
// numerators and divisors below 2^16), so that no kernel divides at run time.
// ---------------------------------------------------------------------------
constexpr int FFT_MAX_STAGES = 16;
struct FftPlanDev {
    int n;
    int nst;
    int rad[FFT_MAX_STAGES];
    int ns[FFT_MAX_STAGES];         // product of the radices before the stage
    unsigned mns[FFT_MAX_STAGES];   // reciprocal of ns (unused when ns == 1)
    int nb[FFT_MAX_STAGES];         // butterflies per line, n / rad
    unsigned mnb[FFT_MAX_STAGES];   // reciprocal of nb (unused when nb == 1)
    int tstr[FFT_MAX_STAGES];       // twiddle stride n / (ns * rad)
    int toff[FFT_MAX_STAGES];       // offset of the stage's table in tws
    const void* tw;                 // cplx<T>*: exp(-2 pi i t / n), t < n
    const void* tws;                // cplx<T>*: per stage, w^(k q) at (q - 1) ns + k, k < ns,
                                    // 1 <= q < rad; n - 1 entries in all
};

// a / d for a * d < 2^32, with m = floor((2^32 - 1) / d) + 1 (d >= 2)
__host__ __device__ __forceinline__ unsigned magic_of(unsigned d) { return d > 1 ? 0xFFFFFFFFu / d + 1u : 0u; }
__device__ __forceinline__ int fdiv(int a, int d, unsigned m) { return d == 1 ? a : (int)__umulhi((unsigned)a, m); }

// MI355X dispatches consecutive workgroups of a 1D grid round robin over its
// 8 XCDs, each with its own L2.  This maps the hardware block index to a
// logical one such that every XCD receives one contiguous range of logical
// blocks (in order), so neighbouring work shares an L2.  The result may reach
// 8 * ceil(nb / 8) - 1; callers treat logical indices >= nb as empty.
constexpr int NXCD = 8;
__device__ __forceinline__ long long xcd_block(long long b, long long nb)
{
    const long long per = (nb + NXCD - 1) / NXCD;
    return (b % NXCD) * per + b / NXCD;
}

// radix-R DFT in registers, forward sign exp(-2 pi i k q / R)
template <typename T, int R>
struct Dft;

template <typename T>
struct Dft<T, 2> {
    __device__ __forceinline__ static void run(cplx<T>* v)
    {
        cplx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};
template <typename T>
struct Dft<T, 4> {
    __device__ __forceinline__ static void run(cplx<T>* v)
    {
        cplx<T> a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
        cplx<T> b0 = cadd(v[1], v[3]), b1 = cmul_mi(csub(v[1], v[3]));
        v[0] = cadd(a0, b0);
        v[2] = csub(a0, b0);
        v[1] = cadd(a1, b1);
        v[3] = csub(a1, b1);
    }
};
template <typename T>
struct Dft<T, 8> {
    __device__ __forceinline__ static void run(cplx<T>* v)
    {
        const T s = (T)0.70710678118654752440;
        // two radix-4 on even/odd, then combine
        cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
        cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
        Dft<T, 4>::run(e);
        Dft<T, 4>::run(o);
        // twiddles exp(-2 pi i k / 8), k = 0..3
        cplx<T> t1 = cmk<T>(s * (o[1].x + o[1].y), s * (o[1].y - o[1].x));
        cplx<T> t2 = cmul_mi(o[2]);
        cplx<T> t3 = cmk<T>(s * (o[3].y - o[3].x), -s * (o[3].x + o[3].y));
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], t1);
        v[5] = csub(e[1], t1);
        v[2] = cadd(e[2], t2);
        v[6] = csub(e[2], t2);
        v[3] = cadd(e[3], t3);
        v[7] = csub(e[3], t3);
    }
};
template <typename T>
struct Dft<T, 3> {
    __device__ __forceinline__ static void run(cplx<T>* v)
    {
        const T c1 = (T)-0.5;
        const T s1 = (T)0.86602540378443864676;  // sin(2 pi / 3)
        cplx<T> a = cadd(v[1], v[2]), d = csub(v[1], v[2]);
        cplx<T> m = cmk<T>(v[0].x + c1 * a.x, v[0].y + c1 * a.y);
        cplx<T> t = cmk<T>(s1 * d.y, -s1 * d.x);  // -i s1 d
        v[0] = cadd(v[0], a);
        v[1] = cadd(m, t);
        v[2] = csub(m, t);
    }
};
template <typename T>
struct Dft<T, 5> {
    __device__ __forceinline__ static void run(cplx<T>* v)
    {
        const T c1 = (T)0.30901699437494742410;   // cos(2 pi / 5)
        const T c2 = (T)-0.80901699437494742410;  // cos(4 pi / 5)
        const T s1 = (T)0.95105651629515357212;   // sin(2 pi / 5)
        const T s2 = (T)0.58778525229247312917;   // sin(4 pi / 5)
        cplx<T> a1 = cadd(v[1], v[4]), d1 = csub(v[1], v[4]);
        cplx<T> a2 = cadd(v[2], v[3]), d2 = csub(v[2], v[3]);
        cplx<T> m1 = cmk<T>(v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y);
        cplx<T> m2 = cmk<T>(v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y);
        // -i (s1 d1 + s2 d2) and -i (s2 d1 - s1 d2)
        cplx<T> t1 = cmk<T>(s1 * d1.y + s2 * d2.y, -(s1 * d1.x + s2 * d2.x));
        cplx<T> t2 = cmk<T>(s2 * d1.y - s1 * d2.y, -(s2 * d1.x - s1 * d2.x));
        v[0] = cadd(v[0], cadd(a1, a2));
        v[1] = cadd(m1, t1);
        v[4] = csub(m1, t1);
        v[2] = cadd(m2, t2);
        v[3] = csub(m2, t2);
    }
};
template <typename T>
struct Dft<T, 7> {
    __device__ __forceinline__ static void run(cplx<T>* v)
    {
        const T c1 = (T)0.62348980185873353053;   // cos(2 pi / 7)
        const T c2 = (T)-0.22252093395631440429;  // cos(4 pi / 7)
        const T c3 = (T)-0.90096886790241912624;  // cos(6 pi / 7)
        const T s1 = (T)0.78183148246802980871;   // sin(2 pi / 7)
        const T s2 = (T)0.97492791218182360702;   // sin(4 pi / 7)
        const T s3 = (T)0.43388373911755812048;   // sin(6 pi / 7)
        cplx<T> a1 = cadd(v[1], v[6]), d1 = csub(v[1], v[6]);
        cplx<T> a2 = cadd(v[2], v[5]), d2 = csub(v[2], v[5]);
        cplx<T> a3 = cadd(v[3], v[4]), d3 = csub(v[3], v[4]);
        cplx<T> m1 = cmk<T>(v[0].x + c1 * a1.x + c2 * a2.x + c3 * a3.x, v[0].y + c1 * a1.y + c2 * a2.y + c3 * a3.y);
        cplx<T> m2 = cmk<T>(v[0].x + c2 * a1.x + c3 * a2.x + c1 * a3.x, v[0].y + c2 * a1.y + c3 * a2.y + c1 * a3.y);
        cplx<T> m3 = cmk<T>(v[0].x + c3 * a1.x + c1 * a2.x + c2 * a3.x, v[0].y + c3 * a1.y + c1 * a2.y + c2 * a3.y);
        // sin(2 pi k q / 7) for (k,q): row k=1: s1 s2 s3; k=2: s2 -s3 -s1; k=3: s3 -s1 s2
        cplx<T> p1 = cmk<T>(s1 * d1.x + s2 * d2.x + s3 * d3.x, s1 * d1.y + s2 * d2.y + s3 * d3.y);
        cplx<T> p2 = cmk<T>(s2 * d1.x - s3 * d2.x - s1 * d3.x, s2 * d1.y - s3 * d2.y - s1 * d3.y);
        cplx<T> p3 = cmk<T>(s3 * d1.x - s1 * d2.x + s2 * d3.x, s3 * d1.y - s1 * d2.y + s2 * d3.y);
        v[0] = cadd(v[0], cadd(a1, cadd(a2, a3)));
        v[1] = cadd(m1, cmul_mi(p1));
        v[6] = csub(m1, cmul_mi(p1));
        v[2] = cadd(m2, cmul_mi(p2));
        v[5] = csub(m2, cmul_mi(p2));
        v[3] = cadd(m3, cmul_mi(p3));
        v[4] = csub(m3, cmul_mi(p3));
    }
};

// Radix 16 as 4 x 4 (Cooley-Tukey): n = 4 n1 + n2, k = k1 + 4 k2, with the
// twiddles exp(-2 pi i n2 k1 / 16) between the two rounds of 4-point DFTs.
template <typename T>
struct Dft<T, 16> {
    __device__ __forceinline__ static void run(cplx<T>* v)
    {
        const T c1 = (T)0.92387953251128675613;  // cos(pi / 8)
        const T s1 = (T)0.38268343236508977173;  // sin(pi / 8)
        const T h = (T)0.70710678118654752440;   // cos(pi / 4)
        cplx<T> y[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < 4; ++n1) y[n2][n1] = v[4 * n1 + n2];
            Dft<T, 4>::run(y[n2]);  // y[n2][k1]
        }
        // w^1 = (c1, -s1), w^2 = (h, -h), w^3 = (s1, -c1), w^4 = -i, w^6 = (-h, -h), w^9 = (-c1, s1)
        y[1][1] = cmul(y[1][1], cmk<T>(c1, -s1));
        y[1][2] = cmul(y[1][2], cmk<T>(h, -h));
        y[1][3] = cmul(y[1][3], cmk<T>(s1, -c1));
        y[2][1] = cmul(y[2][1], cmk<T>(h, -h));
        y[2][2] = cmul_mi(y[2][2]);
        y[2][3] = cmul(y[2][3], cmk<T>(-h, -h));
        y[3][1] = cmul(y[3][1], cmk<T>(s1, -c1));
        y[3][2] = cmul(y[3][2], cmk<T>(-h, -h));
        y[3][3] = cmul(y[3][3], cmk<T>(-c1, s1));
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            cplx<T> t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
            Dft<T, 4>::run(t);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
        }
    }
};

// modular inverse of a (mod m), m >= 2, gcd(a, m) = 1 (compile-time use)
__host__ __device__ constexpr int inv_mod(int a, int m)
{
    int x = 1;
    while ((a * x) % m != 1) ++x;
    return x;
}

// Radix N1 N2 with coprime factors as a prime-factor (Good-Thomas) transform:
// input n = (N2 n1 + N1 n2) mod N, output by the Chinese remainder map; no
// twiddles between the rounds.
template <typename T, int N1, int N2>
struct Pfa {
    static constexpr int N = N1 * N2;
    // output map: k = (k1 E1 + k2 E2) mod N is the k with k = k1 (mod N1),
    // k = k2 (mod N2)
    static constexpr int E1 = (N2 * inv_mod(N2 % N1, N1)) % N;
    static constexpr int E2 = (N1 * inv_mod(N1 % N2, N2)) % N;
    __device__ __forceinline__ static void run(cplx<T>* v)
    {
        cplx<T> y[N2][N1];
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < N1; ++n1) y[n2][n1] = v[(N2 * n1 + N1 * n2) % N];
            Dft<T, N1>::run(y[n2]);
        }
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) {
            cplx<T> t[N2];
#pragma unroll
            for (int n2 = 0; n2 < N2; ++n2) t[n2] = y[n2][k1];
            Dft<T, N2>::run(t);
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) v[(k1 * E1 + k2 * E2) % N] = t[k2];
        }
    }
};
template <typename T>
struct Dft<T, 15> : Pfa<T, 3, 5> {};
template <typename T>
struct Dft<T, 6> : Pfa<T, 2, 3> {};
template <typename T>
struct Dft<T, 10> : Pfa<T, 2, 5> {};
template <typename T>
struct Dft<T, 12> : Pfa<T, 4, 3> {};
template <typename T>
struct Dft<T, 14> : Pfa<T, 2, 7> {};

// Copy of the n - 1 stage twiddles of plan p into LDS (all NT threads of the
// block; the caller synchronises before the first transform).
template <typename T, int NT>
__device__ __forceinline__ void load_stage_twiddles(cplx<T>* dst, const FftPlanDev& p)
{
    const cplx<T>* __restrict__ src = static_cast<const cplx<T>*>(p.tws);
    for (int t = threadIdx.x; t < p.n - 1; t += NT) dst[t] = src[t];
}

// Ordering of LDS accesses among the lanes of one wavefront: the wave's LDS
// operations execute in order, so a compiler barrier with wavefront-scope
// fences is enough (no s_barrier, no wait on other waves).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool WAVE>
__device__ __forceinline__ void group_sync()
{
    if (WAVE)
        wave_sync();
    else
        __syncthreads();
}

// One Stockham stage of radix R on `nl` lines of length n held in LDS
// (line q at buf + q * ld).  Every thread of the group calls it -- the block
// (WAVE false, NT threads) or one wavefront (WAVE true, NT = 64) -- and each
// handles up to E/R butterflies, one after the other, keeping only their
// outputs in registers until all threads have read their inputs.
template <typename T, int NT, int E, int R, bool INV, bool WAVE = false>
__device__ __forceinline__ void fft_stage(cplx<T>* buf, int ld, int nl, const FftPlanDev& p, int st,
                                          const cplx<T>* __restrict__ tws_all)
{
    constexpr int MB = (E / R) > 0 ? (E / R) : 1;
    const int nb = p.nb[st], Ns = p.ns[st];
    const cplx<T>* __restrict__ tws = tws_all + p.toff[st];
    const unsigned mnb = p.mnb[st], mns = p.mns[st];
    const int total = nl * nb;
    cplx<T> v[MB][R];
    int base[MB];
    const int tid = WAVE ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        int b = tid + i * NT;
        base[i] = -1;
        if (b < total) {
            int line = nl == 1 ? 0 : fdiv(b, nb, mnb);  // nl is a literal 1 in the single-line callers
            int j = b - line * nb;
            int jq = fdiv(j, Ns, mns);
            int k = j - jq * Ns;
            const cplx<T>* src = buf + line * ld + j;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                cplx<T> a = src[q * nb];
                v[i][q] = INV ? cswap(a) : a;
            }
            // the stage's twiddles w^(k q) (w^0 = 1 for k = 0; none in the
            // first stage, Ns = 1), read in batches of TB before their use so
            // that a batch is in flight together
            if (Ns > 1) {
                constexpr int TB = sizeof(T) == 8 ? 4 : 2;
                const cplx<T>* ws = tws + k;
#pragma unroll
                for (int q0 = 1; q0 < R; q0 += TB) {
                    cplx<T> wv[TB];
#pragma unroll
                    for (int u = 0; u < TB; ++u)
                        if (q0 + u < R) wv[u] = ws[(q0 + u - 1) * Ns];
#pragma unroll
                    for (int u = 0; u < TB; ++u)
                        if (q0 + u < R) v[i][q0 + u] = cmul(v[i][q0 + u], wv[u]);
                }
            }
            Dft<T, R>::run(v[i]);
            base[i] = line * ld + jq * Ns * R + k;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    group_sync<WAVE>();
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        if (base[i] >= 0) {
            cplx<T>* dst = buf + base[i];
#pragma unroll
            for (int q = 0; q < R; ++q) dst[q * Ns] = INV ? cswap(v[i][q]) : v[i][q];
        }
    }
    group_sync<WAVE>();
}

// Full in-place FFT (unnormalised) of nl lines of length p.n in LDS.
// Requires nl * p.n <= E * NT (checked by the host planner).  Caller must
// __syncthreads() before (data written) -- this routine ends with a barrier.
// tw: the stage twiddle tables (p.tws, or a copy of its n - 1 entries in LDS).
template <typename T, int NT, int E, bool INV, bool WAVE = false>
__device__ void lds_fft(cplx<T>* buf, int ld, int nl, const FftPlanDev& p, const cplx<T>* __restrict__ tw)
{
    for (int s = 0; s < p.nst; ++s) {
        switch (p.rad[s]) {
            case 2: fft_stage<T, NT, E, 2, INV, WAVE>(buf, ld, nl, p, s, tw); break;
            case 3: fft_stage<T, NT, E, 3, INV, WAVE>(buf, ld, nl, p, s, tw); break;
            case 4: fft_stage<T, NT, E, 4, INV, WAVE>(buf, ld, nl, p, s, tw); break;
            case 5: fft_stage<T, NT, E, 5, INV, WAVE>(buf, ld, nl, p, s, tw); break;
            case 6: fft_stage<T, NT, E, 6, INV, WAVE>(buf, ld, nl, p, s, tw); break;
            case 7: fft_stage<T, NT, E, 7, INV, WAVE>(buf, ld, nl, p, s, tw); break;
            case 10: fft_stage<T, NT, E, 10, INV, WAVE>(buf, ld, nl, p, s, tw); break;
            case 12: fft_stage<T, NT, E, 12, INV, WAVE>(buf, ld, nl, p, s, tw); break;
            case 14: fft_stage<T, NT, E, 14, INV, WAVE>(buf, ld, nl, p, s, tw); break;
            case 15: fft_stage<T, NT, E, 15, INV, WAVE>(buf, ld, nl, p, s, tw); break;
            case 16: fft_stage<T, NT, E, 16, INV, WAVE>(buf, ld, nl, p, s, tw); break;
            default: fft_stage<T, NT, E, 8, INV, WAVE>(buf, ld, nl, p, s, tw); break;
        }
    }
}

// Truncated Green's function transforms (paper Sec. 5.2).
//   kind 0, harmonic:    H^R(k) = 8 pi sin^2(R k / 2) / k^2, the transform of
//                        (1/r) 1[r < R]
//   kind 1, biharmonic:  the transform of (r - R) 1[r < R],
//                        4 pi [2 cos Rk + Rk sin Rk - 2] / k^4.
// The biharmonic kernel only enters through second and third derivatives
// (stokeslet and stresslet multipliers), which annihilate the constant -R, so
// inside the truncation radius it acts exactly as the paper's r 1[r < R]
// (whose transform is 4 pi [(2 - R^2k^2) cos Rk + 2 Rk sin Rk - 2] / k^4).
// Subtracting R removes the R^2 k^2 cos Rk edge term, which otherwise
// dominates the samples by a factor ~ (Rk)^2 / 2 and costs about five digits
// of the precomputed multiplier in double precision.  Near k = 0 both forms
// cancel catastrophically and are summed from their series.
__host__ __device__ inline double khat_truncated(int kind, double k, double R)
{
    const double pi = 3.14159265358979323846;
    double x = R * k;
    if (kind == 0) {
        if (x < 1e-4) return 2.0 * pi * R * R * (1.0 - x * x / 12.0);
        double s = sin(0.5 * x) / k;
        return 8.0 * pi * s * s;
    }
    if (x < 0.5) {
        // 4 pi R^4 sum_{m >= 2} (-1)^m 2 (1 - m) x^{2m-4} / (2m)!
        double x2 = x * x, pw = 1.0, acc = 0.0;
        double fact = 24.0;  // (2m)! for m = 2
        for (int m = 2; m < 16; ++m) {
            double c = 2.0 * (1.0 - m) / fact;
            acc += (m & 1) ? -c * pw : c * pw;
            pw *= x2;
            fact *= (double)(2 * m + 1) * (double)(2 * m + 2);
        }
        return 4.0 * pi * R * R * R * R * acc;
    }
    double k2 = k * k;
    return 4.0 * pi * (2.0 * cos(x) + x * sin(x) - 2.0) / (k2 * k2);
}

}  // namespace ehs
