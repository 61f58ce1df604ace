// Binning support: bounding-box / validation reduction, cell keys, a stable
// LSD radix sort and exclusive scans, all deterministic (no floating-point
// atomics; integer counts come from wave ballots).
#include <math.h>

#include "common.h"
#include "kernels.h"

namespace ehs {

// ---------------------------------------------------------------------------
// fill (used instead of memset so that every clear is an ordinary kernel)
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* p, uint32_t v, long long n)
{
    const long long step = (long long)gridDim.x * blockDim.x;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += step) p[i] = v;
}

hipError_t fill_u32(uint32_t* p, uint32_t v, long long n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const long long blocks = std::min((n + 255) / 256, 1LL << 16);  // grid-stride beyond 2^24 words
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

template <typename A, typename B>
__global__ void k_convert(const A* __restrict__ in, B* __restrict__ out, long long n)
{
    const long long step = (long long)gridDim.x * blockDim.x;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += step) out[i] = (B)in[i];
}

template <typename A, typename B>
hipError_t launch_convert(const A* in, B* out, long long n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const long long blocks = std::min((n + 255) / 256, 1LL << 16);
    hipLaunchKernelGGL((k_convert<A, B>), dim3((unsigned)blocks), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}
template hipError_t launch_convert<float, double>(const float*, double*, long long, hipStream_t);
template hipError_t launch_convert<double, float>(const double*, float*, long long, hipStream_t);
template hipError_t launch_convert<double, double>(const double*, double*, long long, hipStream_t);

// ---------------------------------------------------------------------------
// bounding box and validation
// ---------------------------------------------------------------------------
constexpr int BB_NT = 256;
constexpr int BB_NV = 10;

struct BBox {
    double v[BB_NV];
};

__device__ __forceinline__ void bb_init(BBox& b)
{
    for (int a = 0; a < 3; ++a) {
        b.v[a] = INFINITY;
        b.v[3 + a] = -INFINITY;
    }
    b.v[6] = INFINITY;
    b.v[7] = INFINITY;
    b.v[8] = 0.0;
    b.v[9] = 0.0;
}

__device__ __forceinline__ void bb_merge(BBox& a, const BBox& b)
{
    for (int i = 0; i < 3; ++i) {
        a.v[i] = fmin(a.v[i], b.v[i]);
        a.v[3 + i] = fmax(a.v[3 + i], b.v[3 + i]);
    }
    a.v[6] = fmin(a.v[6], b.v[6]);
    a.v[7] = fmin(a.v[7], b.v[7]);
    a.v[8] += b.v[8];
    a.v[9] += b.v[9];
}

int bbox_blocks(long long n)
{
    long long b = (n + BB_NT * 8 - 1) / (BB_NT * 8);
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int)b;
}

// besides the box: a histogram of the target heights x3 in ZH_BINS bins of
// width 1 / zbin_inv from the wall (the last bin holds everything above),
// from which the planner sizes the real-space cells by the targets' actual
// density near the wall (integer counts: the same on every run)
__global__ void __launch_bounds__(BB_NT) k_bbox(int family, const double* __restrict__ y, const double* __restrict__ s,
                                                long long N, const double* __restrict__ x, long long T,
                                                double* __restrict__ partial, double zbin_inv,
                                                uint32_t* __restrict__ zhist)
{
    __shared__ double red[BB_NT][BB_NV];
    __shared__ uint32_t hist[ZH_BINS];
    if (threadIdx.x < ZH_BINS) hist[threadIdx.x] = 0u;
    __syncthreads();
    BBox b;
    bb_init(b);
    const int ns = family == STRESSLET ? 6 : 3;
    long long stride = (long long)gridDim.x * BB_NT;
    for (long long i = blockIdx.x * (long long)BB_NT + threadIdx.x; i < N + T; i += stride) {
        const double* p = (i < N) ? (y + 3 * i) : (x + 3 * (i - N));
        double p0 = p[0], p1 = p[1], p2 = p[2];
        bool fin = isfinite(p0) && isfinite(p1) && isfinite(p2);
        if (i < N) {
            const double* q = s + ns * i;
            double qq = 0.0;
            if (family == STRESSLET) {
                double g2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
                double o2 = q[3] * q[3] + q[4] * q[4] + q[5] * q[5];
                qq = g2 * o2;  // |g (x) q|_F^2
            } else {
                qq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
            }
            fin = fin && isfinite(qq);
            if (fin) b.v[9] += qq;
            if (fin) b.v[6] = fmin(b.v[6], p2);
        } else if (fin) {
            b.v[7] = fmin(b.v[7], p2);
            const int bin = (int)fmin((double)(ZH_BINS - 1), fmax(0.0, p2 * zbin_inv));
            atomicAdd(&hist[bin], 1u);
        }
        if (!fin) {
            b.v[8] += 1.0;
            continue;
        }
        b.v[0] = fmin(b.v[0], p0);
        b.v[1] = fmin(b.v[1], p1);
        b.v[2] = fmin(b.v[2], p2);
        b.v[3] = fmax(b.v[3], p0);
        b.v[4] = fmax(b.v[4], p1);
        b.v[5] = fmax(b.v[5], p2);
    }
    for (int k = 0; k < BB_NV; ++k) red[threadIdx.x][k] = b.v[k];
    __syncthreads();
    for (int w = BB_NT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            BBox o;
            for (int k = 0; k < BB_NV; ++k) {
                b.v[k] = red[threadIdx.x][k];
                o.v[k] = red[threadIdx.x + w][k];
            }
            bb_merge(b, o);
            for (int k = 0; k < BB_NV; ++k) red[threadIdx.x][k] = b.v[k];
        }
        __syncthreads();
    }
    if (threadIdx.x < BB_NV) partial[blockIdx.x * BB_NV + threadIdx.x] = red[0][threadIdx.x];
    if (threadIdx.x < ZH_BINS && hist[threadIdx.x]) atomicAdd(&zhist[threadIdx.x], hist[threadIdx.x]);
}

__global__ void k_bbox_final(const double* __restrict__ partial, int nb, double* __restrict__ out16)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    BBox b;
    bb_init(b);
    for (int i = 0; i < nb; ++i) {
        BBox o;
        for (int k = 0; k < BB_NV; ++k) o.v[k] = partial[i * BB_NV + k];
        bb_merge(b, o);
    }
    for (int k = 0; k < BB_NV; ++k) out16[k] = b.v[k];
    for (int k = BB_NV; k < 16; ++k) out16[k] = 0.0;
}

hipError_t launch_bbox(int family, const double* y, const double* s, long long N, const double* x, long long T,
                       double* partial, int nblocks, double* out16, double zbin_inv, uint32_t* zhist, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(ZH_BINS), 0, st, zhist, 0u, (long long)ZH_BINS);
    hipLaunchKernelGGL(k_bbox, dim3(nblocks), dim3(BB_NT), 0, st, family, y, s, N, x, T, partial, zbin_inv, zhist);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, st, partial, nblocks, out16);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exclusive scan of uint32 (three kernels: block sums, top-level scan,
// block scans with offsets); blocks of SC_TILE elements
// ---------------------------------------------------------------------------
constexpr int SC_NT = 256;
constexpr int SC_PER = 4;
constexpr int SC_TILE = SC_NT * SC_PER;

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total)
{
    // Hillis-Steele inclusive scan over SC_NT values, then shift
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < SC_NT; off <<= 1) {
        uint32_t t = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0u;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    uint32_t incl = sh[threadIdx.x];
    if (total) *total = sh[SC_NT - 1];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(SC_NT) k_scan_reduce(const uint32_t* __restrict__ in, long long n,
                                                       uint32_t* __restrict__ bsum)
{
    __shared__ uint32_t sh[SC_NT];
    long long b0 = blockIdx.x * (long long)SC_TILE;
    uint32_t v = 0;
    for (int k = 0; k < SC_PER; ++k) {
        long long i = b0 + threadIdx.x * SC_PER + k;
        if (i < n) v += in[i];
    }
    uint32_t tot;
    block_excl_scan(v, sh, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(SC_NT) k_scan_top(uint32_t* __restrict__ bsum, long long nb)
{
    __shared__ uint32_t sh[SC_NT];
    uint32_t carry = 0;
    for (long long c0 = 0; c0 < nb; c0 += SC_NT) {
        long long i = c0 + threadIdx.x;
        uint32_t v = (i < nb) ? bsum[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_excl_scan(v, sh, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
}

__global__ void __launch_bounds__(SC_NT) k_scan_down(const uint32_t* in, uint32_t* out, long long n,
                                                     const uint32_t* __restrict__ bsum)
{
    __shared__ uint32_t sh[SC_NT];
    long long b0 = blockIdx.x * (long long)SC_TILE;
    uint32_t v[SC_PER];
    uint32_t t = 0;
    for (int k = 0; k < SC_PER; ++k) {
        long long i = b0 + threadIdx.x * SC_PER + k;
        v[k] = (i < n) ? in[i] : 0u;
        t += v[k];
    }
    uint32_t ex = block_excl_scan(t, sh, nullptr) + bsum[blockIdx.x];
    for (int k = 0; k < SC_PER; ++k) {
        long long i = b0 + threadIdx.x * SC_PER + k;
        if (i < n) out[i] = ex;
        ex += v[k];
    }
}

size_t scan_scratch_bytes(long long n) { return (size_t)(((n + SC_TILE - 1) / SC_TILE) + 1) * sizeof(uint32_t); }

hipError_t exclusive_scan(const uint32_t* in, uint32_t* out, long long n, void* scratch, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    long long nb = (n + SC_TILE - 1) / SC_TILE;
    uint32_t* bsum = static_cast<uint32_t*>(scratch);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SC_NT), 0, st, in, n, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SC_NT), 0, st, bsum, nb);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(SC_NT), 0, st, in, out, n, bsum);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// radix sort: 4-bit digits, tiles of 1024 keys (256 threads x 4 rounds),
// digit counts and stable ranks from wave ballots
// ---------------------------------------------------------------------------
constexpr int RS_NT = 256;
constexpr int RS_ROUNDS = 4;
constexpr int RS_TILE = RS_NT * RS_ROUNDS;
constexpr int RS_DIG = 16;
constexpr int RS_WAVES = RS_NT / 64;

__global__ void __launch_bounds__(RS_NT) k_rs_hist(const uint32_t* __restrict__ keys, long long n, int shift,
                                                   uint32_t* __restrict__ hist, long long ntiles)
{
    __shared__ uint32_t cnt[RS_WAVES][RS_DIG];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane < RS_DIG) cnt[w][lane] = 0;
    __syncthreads();
    long long t0 = blockIdx.x * (long long)RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        long long e = t0 + r * RS_NT + threadIdx.x;
        int d = (e < n) ? (int)((keys[e] >> shift) & (RS_DIG - 1)) : RS_DIG;
        for (int dd = 0; dd < RS_DIG; ++dd) {
            unsigned long long m = __ballot(d == dd);
            if (lane == 0) cnt[w][dd] += (uint32_t)__popcll(m);
        }
    }
    __syncthreads();
    if (threadIdx.x < RS_DIG) {
        uint32_t s = 0;
        for (int ww = 0; ww < RS_WAVES; ++ww) s += cnt[ww][threadIdx.x];
        hist[(long long)threadIdx.x * ntiles + blockIdx.x] = s;
    }
}

__global__ void __launch_bounds__(RS_NT) k_rs_scatter(const uint32_t* __restrict__ keys,
                                                      const uint32_t* __restrict__ vals, long long n, int shift,
                                                      const uint32_t* __restrict__ offs, long long ntiles,
                                                      uint32_t* __restrict__ kout, uint32_t* __restrict__ vout)
{
    __shared__ uint32_t wc[RS_ROUNDS * RS_WAVES][RS_DIG];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    long long t0 = blockIdx.x * (long long)RS_TILE;
    uint32_t key[RS_ROUNDS], val[RS_ROUNDS], rank[RS_ROUNDS];
    int dig[RS_ROUNDS];
    for (int r = 0; r < RS_ROUNDS; ++r) {
        long long e = t0 + r * RS_NT + threadIdx.x;
        bool ok = e < n;
        key[r] = ok ? keys[e] : 0u;
        val[r] = ok ? vals[e] : 0u;
        int d = ok ? (int)((key[r] >> shift) & (RS_DIG - 1)) : RS_DIG;
        dig[r] = d;
        rank[r] = 0;
        for (int dd = 0; dd < RS_DIG; ++dd) {
            unsigned long long m = __ballot(d == dd);
            if (d == dd) rank[r] = (uint32_t)__popcll(m & lt);
            if (lane == 0) wc[r * RS_WAVES + w][dd] = (uint32_t)__popcll(m);
        }
    }
    __syncthreads();
    if (threadIdx.x < RS_DIG) {
        uint32_t run = 0;
        for (int g = 0; g < RS_ROUNDS * RS_WAVES; ++g) {
            uint32_t c = wc[g][threadIdx.x];
            wc[g][threadIdx.x] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int r = 0; r < RS_ROUNDS; ++r) {
        int d = dig[r];
        if (d < RS_DIG) {
            uint32_t dst = offs[(long long)d * ntiles + blockIdx.x] + wc[r * RS_WAVES + w][d] + rank[r];
            kout[dst] = key[r];
            vout[dst] = val[r];
        }
    }
}

size_t radix_sort_scratch_bytes(long long n)
{
    long long ntiles = (n + RS_TILE - 1) / RS_TILE;
    long long nh = ntiles * RS_DIG;
    return (size_t)nh * sizeof(uint32_t) + scan_scratch_bytes(nh) + 256;
}

hipError_t radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp, long long n, int bits,
                      void* scratch, hipStream_t st, uint32_t** keys_out, uint32_t** vals_out)
{
    long long ntiles = (n + RS_TILE - 1) / RS_TILE;
    long long nh = ntiles * RS_DIG;
    uint32_t* hist = static_cast<uint32_t*>(scratch);
    void* sc = static_cast<void*>(hist + nh + 64);
    uint32_t *ka = keys, *va = vals, *kb = keys_tmp, *vb = vals_tmp;
    if (n > 0) {
        for (int shift = 0; shift < bits; shift += 4) {
            hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)ntiles), dim3(RS_NT), 0, st, ka, n, shift, hist, ntiles);
            hipError_t e = exclusive_scan(hist, hist, nh, sc, st);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)ntiles), dim3(RS_NT), 0, st, ka, va, n, shift, hist,
                               ntiles, kb, vb);
            uint32_t* t = ka;
            ka = kb;
            kb = t;
            t = va;
            va = vb;
            vb = t;
        }
    }
    *keys_out = ka;
    *vals_out = va;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// off[k] = first position q of the sorted keys with skeys[q] >= k, k <= ncell
// (binary search; the records of key k are [off[k], off[k+1]))
// ---------------------------------------------------------------------------
__global__ void k_key_offsets(const uint32_t* __restrict__ skeys, long long n, uint32_t* __restrict__ off,
                              long long ncell)
{
    long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (k > ncell) return;
    long long lo = 0, hi = n;
    while (lo < hi) {
        long long mid = (lo + hi) >> 1;
        if ((long long)skeys[mid] < k)
            lo = mid + 1;
        else
            hi = mid;
    }
    off[k] = (uint32_t)lo;
}

hipError_t launch_cell_ranges(const uint32_t* skeys, long long n, uint32_t* start, uint32_t* end, long long ncell,
                              hipStream_t st)
{
    // `start` receives ncell + 1 offsets; `end` is unused (kept for symmetry)
    (void)end;
    hipLaunchKernelGGL(k_key_offsets, dim3((unsigned)((ncell + 1 + 255) / 256)), dim3(256), 0, st, skeys, n, start,
                       ncell);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// real-space cell keys and chunk work list
// ---------------------------------------------------------------------------
__global__ void k_cell_keys(const double* __restrict__ p, long long n, CellGeom cg, uint32_t* __restrict__ keys,
                            uint32_t* __restrict__ idx)
{
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c[3];
    for (int a = 0; a < 3; ++a) {
        double t = floor((p[3 * i + a] - cg.lo[a]) * cg.inv[a]);
        int v = (t < 0.0) ? 0 : (t >= (double)cg.nc[a] ? cg.nc[a] - 1 : (int)t);
        c[a] = v;
    }
    keys[i] = (uint32_t)(((long long)c[2] * cg.nc[1] + c[1]) * cg.nc[0] + c[0]);
    idx[i] = (uint32_t)i;
}

hipError_t launch_cell_keys(const double* p, long long n, CellGeom cg, uint32_t* keys, uint32_t* idx, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cell_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, cg, keys, idx);
    return hipGetLastError();
}

__global__ void k_chunk_counts(const uint32_t* __restrict__ toff, long long ncell, uint32_t* __restrict__ counts)
{
    long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    uint32_t n = toff[c + 1] - toff[c];
    counts[c] = (n + 63u) / 64u;
}

__global__ void k_chunk_emit(const uint32_t* __restrict__ toff, long long ncell, const uint32_t* __restrict__ counts,
                             const uint32_t* __restrict__ offs, uint32_t* __restrict__ chunk_cell,
                             uint32_t* __restrict__ chunk_first, uint32_t* __restrict__ nchunks)
{
    long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    uint32_t n = counts[c], o = offs[c];
    for (uint32_t q = 0; q < n; ++q) {
        chunk_cell[o + q] = (uint32_t)c;
        chunk_first[o + q] = toff[c] + 64u * q;
    }
    if (c == ncell - 1) *nchunks = o + n;
}

hipError_t launch_chunks(const uint32_t* toff, const uint32_t* unused, long long ncell, uint32_t* counts,
                         uint32_t* offs, void* scan_scratch, uint32_t* chunk_cell, uint32_t* chunk_first,
                         uint32_t* nchunks, hipStream_t st)
{
    (void)unused;
    unsigned g = (unsigned)((ncell + 255) / 256);
    hipLaunchKernelGGL(k_chunk_counts, dim3(g), dim3(256), 0, st, toff, ncell, counts);
    hipError_t e = exclusive_scan(counts, offs, ncell, scan_scratch, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_chunk_emit, dim3(g), dim3(256), 0, st, toff, ncell, counts, offs, chunk_cell, chunk_first,
                       nchunks);
    return hipGetLastError();
}

// sorted source data for the real-space pass: positions SoA (3 x N) and the
// real-space strengths (stokeslet f; stresslet sym(g q) as xx xy xz yy yz zz;
// rotlet v), nstr x N
__global__ void k_gather_sources(int family, const double* __restrict__ y, const double* __restrict__ s,
                                 const uint32_t* __restrict__ perm, long long N, double* __restrict__ ys,
                                 double* __restrict__ ss)
{
    long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= N) return;
    long long p = perm[q];
    for (int a = 0; a < 3; ++a) ys[a * N + q] = y[3 * p + a];
    if (family == STRESSLET) {
        const double* g = s + 6 * p;
        const double* o = s + 6 * p + 3;
        ss[0 * N + q] = g[0] * o[0];
        ss[1 * N + q] = 0.5 * (g[0] * o[1] + g[1] * o[0]);
        ss[2 * N + q] = 0.5 * (g[0] * o[2] + g[2] * o[0]);
        ss[3 * N + q] = g[1] * o[1];
        ss[4 * N + q] = 0.5 * (g[1] * o[2] + g[2] * o[1]);
        ss[5 * N + q] = g[2] * o[2];
    } else {
        for (int a = 0; a < 3; ++a) ss[a * N + q] = s[3 * p + a];
    }
}

hipError_t launch_gather_sources(int family, const double* y, const double* s, const uint32_t* perm, long long N,
                                 double* ys, double* ss, hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_sources, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, family, y, s, perm, N,
                       ys, ss);
    return hipGetLastError();
}

__global__ void k_gather_points(const double* __restrict__ x, const uint32_t* __restrict__ perm, long long T,
                                double* __restrict__ xs)
{
    long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= T) return;
    long long p = perm[q];
    for (int a = 0; a < 3; ++a) xs[a * T + q] = x[3 * p + a];
}

hipError_t launch_gather_points(const double* x, const uint32_t* perm, long long T, double* xs, hipStream_t st)
{
    if (T <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_points, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, st, x, perm, T, xs);
    return hipGetLastError();
}

}  // namespace ehs
