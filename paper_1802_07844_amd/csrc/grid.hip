// Gaussian spreading onto the grid and Gaussian gathering (quadrature) at the
// targets -- steps 5 and 10 of the paper's Algorithm 1, with the window
// W(d) = (2 xi^2 / (pi eta))^{3/2} exp(-2 xi^2 |d|^2 / eta) truncated to P^3
// nodes.
//
// Spreading is atomic-free: the 2N points (sources and their wall images)
// are sorted by the grid tile that holds the first node of their support;
// every output tile is owned by one wavefront, which walks the records of the
// neighbouring tiles in sorted order and accumulates its own nodes in
// registers.  The result is deterministic and every grid node is written
// exactly once (zeros included).
#include <math.h>

#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace ehs {

template <int K>
struct RecLayout {
    static constexpr int ncA = Traits<K>::ncA;
    static constexpr int ncB = Traits<K>::ncB;
};

// A record: header of 4 int32 (support base x, y, z, image flag) in the first
// 16 bytes, then the 3P Gaussian factors along x1, x2, x3, the offsets
// o + base h - z of the first support node per axis (for derivative
// weights), then ncA kernel strengths and ncB correction coefficients (FP32:
// the correction strengths; FP64: the coefficients of the density D).
size_t record_stride(int family, int P, size_t esz)
{
    int nc = family == STOKESLET ? 7 : family == STRESSLET ? 13 : 5;
    return 16 / esz + 3 * (size_t)P + 3 + nc;
}

__device__ __forceinline__ int support_base(double z, double o, double h, int P, int n)
{
    int b = (int)floor((z - o) / h) - P / 2 + 1;
    if (b < 0) b = 0;
    if (b > n - P) b = n - P;
    return b;
}

// npts = 2N (sources, then their wall images) or N (free space: sources only)
__global__ void k_point_keys(const double* __restrict__ y, long long N, long long npts, GridArgs g,
                             uint32_t* __restrict__ keys, uint32_t* __restrict__ idx)
{
    long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (p >= npts) return;
    long long m = p < N ? p : p - N;
    double z[3] = {y[3 * m], y[3 * m + 1], p < N ? y[3 * m + 2] : -y[3 * m + 2]};
    int dims[3] = {g.Mt, g.Mt, 2 * g.Mt};
    int t[3];
    for (int a = 0; a < 3; ++a) t[a] = support_base(z[a], g.o[a], g.h, g.P, dims[a]) / g.tile[a];
    keys[p] = (uint32_t)(((long long)t[2] * g.nt[1] + t[1]) * g.nt[0] + t[0]);
    idx[p] = (uint32_t)p;
}

hipError_t launch_point_keys(const double* y, long long N, long long npts, GridArgs g, uint32_t* keys, uint32_t* idx,
                             hipStream_t st)
{
    if (npts <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_point_keys, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, y, N, npts, g, keys,
                       idx);
    return hipGetLastError();
}

// strengths of the consolidated sources (A-grids) and of the correction
// sources (B-grids) for point p (p >= N: image of source p - N)
template <int K>
__device__ __forceinline__ void point_strengths(const double* s, const double* y, long long p, long long N, double* cA,
                                                double* cB)
{
    bool img = p >= N;
    long long m = img ? p - N : p;
    if (K == STOKESLET) {
        const double* f = s + 3 * m;
        if (!img) {
            cA[0] = f[0];
            cA[1] = f[1];
            cA[2] = f[2];
        } else {
            // -f^I at y^I;  correction sources f3 and y3 f^I
            cA[0] = -f[0];
            cA[1] = -f[1];
            cA[2] = f[2];
            double y3 = y[3 * m + 2];
            cB[0] = f[2];
            cB[1] = y3 * f[0];
            cB[2] = y3 * f[1];
            cB[3] = -y3 * f[2];
        }
    } else if (K == STRESSLET) {
        const double* g = s + 6 * m;
        const double* q = s + 6 * m + 3;
        double S[6] = {g[0] * q[0], 0.5 * (g[0] * q[1] + g[1] * q[0]), 0.5 * (g[0] * q[2] + g[2] * q[0]),
                       g[1] * q[1], 0.5 * (g[1] * q[2] + g[2] * q[1]), g[2] * q[2]};
        if (!img) {
            for (int c = 0; c < 6; ++c) cA[c] = S[c];
        } else {
            // R S R flips xz and yz
            double SI[6] = {S[0], S[1], -S[2], S[3], -S[4], S[5]};
            for (int c = 0; c < 6; ++c) cA[c] = -SI[c];
            double y3 = y[3 * m + 2];
            cB[0] = S[0] + S[3] + S[5];
            for (int c = 0; c < 6; ++c) cB[1 + c] = y3 * SI[c];
        }
    } else {
        const double* v = s + 3 * m;
        if (!img) {
            cA[0] = v[0];
            cA[1] = v[1];
            cA[2] = v[2];
        } else {
            cA[0] = v[0];
            cA[1] = v[1];
            cA[2] = -v[2];
            cB[0] = -2.0 * v[1];
            cB[1] = 2.0 * v[0];
        }
    }
}

template <typename T, int K, int CM>
__global__ void k_records(const double* __restrict__ y, const double* __restrict__ s, const uint32_t* __restrict__ perm,
                          long long N, GridArgs g, T* __restrict__ rec)
{
    constexpr int ncA = RecLayout<K>::ncA, ncB = RecLayout<K>::ncB;
    long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= (CM == CM_FREE ? N : 2 * N)) return;  // free space: no images
    const int P = g.P;
    const long long stride = 16 / sizeof(T) + 3 * P + 3 + ncA + ncB;
    long long p = perm[q];
    long long m = p < N ? p : p - N;
    bool img = p >= N;
    double z[3] = {y[3 * m], y[3 * m + 1], img ? -y[3 * m + 2] : y[3 * m + 2]};
    int dims[3] = {g.Mt, g.Mt, 2 * g.Mt};
    T* r = rec + q * stride;
    int* hdr = reinterpret_cast<int*>(r);
    int base[3];
    for (int a = 0; a < 3; ++a) {
        base[a] = support_base(z[a], g.o[a], g.h, P, dims[a]);
        hdr[a] = base[a];
    }
    hdr[3] = img ? 1 : 0;
    T* w = r + 16 / sizeof(T);
    for (int a = 0; a < 3; ++a) {
        for (int t = 0; t < P; ++t) {
            double d = g.o[a] + (base[a] + t) * g.h - z[a];
            double v = exp(-g.a2 * d * d);
            if (a == 0) v *= g.pref;
            w[a * P + t] = (T)v;
        }
    }
    for (int a = 0; a < 3; ++a) w[3 * P + a] = (T)(g.o[a] + base[a] * g.h - z[a]);
    double cA[ncA], cB[ncB];
    for (int c = 0; c < ncB; ++c) cB[c] = 0.0;
    point_strengths<K>(s, y, p, N, cA, cB);
    if (CM == CM_DENSITY) {
        // coefficients of D (see InGrids): stokeslet (c0; cx, cy, cz) of
        // c0 W + c . grad W; stresslet (c3; Sxx, Sxy, Sxz, Syy, Syz, Szz) of
        // c3 d3 W + S : grad grad W; rotlet (cx, cy) of c . grad W
        const double k = K == STOKESLET ? -2.0 : K == STRESSLET ? -4.0 : 2.0;
        for (int c = 0; c < ncB; ++c) cB[c] *= k;
        if (K == STRESSLET) cB[0] = -cB[0];  // +4 g.q d3
    }
    T* cs = w + 3 * P + 3;
    for (int c = 0; c < ncA; ++c) cs[c] = (T)cA[c];
    for (int c = 0; c < ncB; ++c) cs[ncA + c] = (T)cB[c];
}

template <typename T, int CM>
static void launch_records_t(int family, const double* y, const double* s, const uint32_t* perm, long long N,
                             GridArgs g, T* rec, hipStream_t st)
{
    dim3 grid((unsigned)(((CM == CM_FREE ? N : 2 * N) + 255) / 256));
    switch (family) {
        case STOKESLET: hipLaunchKernelGGL((k_records<T, STOKESLET, CM>), grid, dim3(256), 0, st, y, s, perm, N, g, rec); break;
        case STRESSLET: hipLaunchKernelGGL((k_records<T, STRESSLET, CM>), grid, dim3(256), 0, st, y, s, perm, N, g, rec); break;
        default: hipLaunchKernelGGL((k_records<T, ROTLET, CM>), grid, dim3(256), 0, st, y, s, perm, N, g, rec); break;
    }
}

template <typename T>
hipError_t launch_records(int family, int cm, const double* y, const double* s, const uint32_t* perm, long long N,
                          GridArgs g, T* rec, hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    if (cm == CM_FREE)
        launch_records_t<T, CM_FREE>(family, y, s, perm, N, g, rec, st);
    else if (cm == CM_DENSITY)
        launch_records_t<T, CM_DENSITY>(family, y, s, perm, N, g, rec, st);
    else
        launch_records_t<T, CM_GRIDS>(family, y, s, perm, N, g, rec, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// spreading: one wavefront (block of 64) per output tile of 8 x 8 x TZ nodes;
// lane (i, j) owns the column of TZ nodes along x3.  Output grids: the ncA
// kernel components, then the correction grids (FP32: ncB of them) or the
// single density D (FP64), accumulated with derivative weights
//   w'(d) = -2 a d w(d),  w''(d) = (4 a^2 d^2 - 2 a) w(d),  d = x_g - z.
// ---------------------------------------------------------------------------
// records staged in LDS per chunk: few, so that the LDS leaves room for many
// one-wavefront blocks per CU (32 records allowed two per SIMD; 8 allow eight).
// Tiles of 8 x 8 x 4 nodes for dense point sets: the accumulators of 4 nodes
// per lane (28 FP64 values for the stokeslet's 7 grids) leave registers for 5
// wavefronts per SIMD, where 8 nodes per lane allowed 3, and the other
// wavefronts hide the records' latency (clustered N = 4e6 stokeslet: 120 ->
// 88 ms, with the strengths held in registers; 2 nodes per lane visit too
// many records).  Sparse sets keep 8 nodes per lane (the planner decides).
constexpr int SP_CHUNK = 8;

template <typename T, int K, int TZ, int CM>
__global__ void __launch_bounds__(64) k_spread(GridArgs g, const T* __restrict__ rec,
                                               const uint32_t* __restrict__ toff, T* __restrict__ grids, long long cs)
{
    constexpr int ncA = RecLayout<K>::ncA, ncB = RecLayout<K>::ncB;
    constexpr int nout = InGrids<K, CM>::n;
    extern __shared__ unsigned char smem_raw[];
    T* sh = reinterpret_cast<T*>(smem_raw);
    const int P = g.P;
    const int stride = 16 / sizeof(T) + 3 * P + 3 + ncA + ncB;
    const int lane = threadIdx.x;
    const int tx = blockIdx.x, ty = blockIdx.y, tz = blockIdx.z;
    const int i = tx * 8 + (lane & 7), j = ty * 8 + (lane >> 3);
    const int l0 = tz * TZ;
    const T a2 = (T)g.a2, hh = (T)g.h;
    T acc[TZ][nout];
#pragma unroll
    for (int z = 0; z < TZ; ++z)
#pragma unroll
        for (int c = 0; c < nout; ++c) acc[z][c] = (T)0;

    const int x_lo = tx - g.K[0] < 0 ? 0 : tx - g.K[0];
    for (int sz = tz - g.K[2]; sz <= tz; ++sz) {
        if (sz < 0) continue;
        for (int sy = ty - g.K[1]; sy <= ty; ++sy) {
            if (sy < 0) continue;
            long long row = ((long long)sz * g.nt[1] + sy) * g.nt[0];
            uint32_t r0 = toff[row + x_lo], r1 = toff[row + tx + 1];
            for (uint32_t c0 = r0; c0 < r1; c0 += SP_CHUNK) {
                int nr = (int)min((uint32_t)SP_CHUNK, r1 - c0);
                // stage the records of this chunk (8 independent loads per lane
                // in flight before the LDS stores)
                const T* src = rec + (long long)c0 * stride;
                for (int f0 = lane; f0 < nr * stride; f0 += 8 * 64) {
                    T v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) v[u] = (f0 + 64 * u < nr * stride) ? src[f0 + 64 * u] : (T)0;
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (f0 + 64 * u < nr * stride) sh[f0 + 64 * u] = v[u];
                }
                __syncthreads();
                for (int q = 0; q < nr; ++q) {
                    const T* r = sh + q * stride;
                    const int* hdr = reinterpret_cast<const int*>(r);
                    int dx = i - hdr[0], dy = j - hdr[1];
                    if ((unsigned)dx < (unsigned)P && (unsigned)dy < (unsigned)P) {
                        const T* w = r + 16 / sizeof(T);
                        const T wx = w[dx], wy = w[P + dy];
                        const T wxy = wx * wy;
                        const T* off = w + 3 * P;
                        // the strengths used at every node in registers: one
                        // LDS read each per record, not one per node (the
                        // density's coefficients enter once per record; with
                        // 8 nodes per lane the density keeps them in LDS, which
                        // holds its registers at 5 wavefronts per SIMD)
                        constexpr int NH = CM == CM_GRIDS ? ncA + ncB : (TZ == 4 ? ncA : 0);
                        T cvh[NH > 0 ? NH : 1];
#pragma unroll
                        for (int c = 0; c < NH; ++c) cvh[c] = off[3 + c];
                        auto cv = [&](int c) -> T { return c < NH ? cvh[c < NH ? c : 0] : off[3 + c]; };
                        const bool img = hdr[3] != 0;
                        // D: per-column factors of w(z), w'(z), w''(z)
                        T fa = 0, fb = 0, fc = 0;
                        if (CM == CM_DENSITY && img) {
                            const T ex = off[0] + (T)dx * hh, ey = off[1] + (T)dy * hh;
                            const T dwx = -2 * a2 * ex * wx, dwy = -2 * a2 * ey * wy;
                            const T* c = off + 3 + ncA;
                            if (K == STOKESLET) {
                                fa = c[0] * wxy + c[1] * dwx * wy + c[2] * wx * dwy;
                                fb = c[3] * wxy;
                            } else if (K == STRESSLET) {
                                const T d2x = (4 * a2 * a2 * ex * ex - 2 * a2) * wx;
                                const T d2y = (4 * a2 * a2 * ey * ey - 2 * a2) * wy;
                                fa = c[1] * d2x * wy + c[4] * wx * d2y + 2 * c[2] * dwx * dwy;
                                fb = c[0] * wxy + 2 * c[3] * dwx * wy + 2 * c[5] * wx * dwy;
                                fc = c[6] * wxy;
                            } else {
                                fa = c[0] * dwx * wy + c[1] * wx * dwy;
                            }
                        }
                        // depth 4: the four x3 factors read together (paired
                        // LDS reads).  A record within reach has
                        // -3 <= dz0 <= P + 2, so the reads cover factors
                        // 2P - 3 .. 3P + 5 of its 3P + 3 + nc (nc >= 5) values
                        // after the header: within the record; those outside
                        // the support are not used (spreading 2-3.5 % faster)
                        constexpr bool WZ4 = TZ == 4;
                        const int dz0 = l0 - hdr[2];
                        T wzv[TZ];
                        if (WZ4) {
#pragma unroll
                            for (int z = 0; z < TZ; ++z) wzv[z] = w[2 * P + dz0 + z];
                        }
#pragma unroll
                        for (int z = 0; z < TZ; ++z) {
                            int dz = dz0 + z;
                            if ((unsigned)dz < (unsigned)P) {
                                const T wz = WZ4 ? wzv[z] : w[2 * P + dz];
                                const T wv = wxy * wz;
#pragma unroll
                                for (int c = 0; c < ncA; ++c) acc[z][c] += wv * cv(c);
                                if (img) {
                                    if constexpr (CM == CM_DENSITY) {
                                        const T ez = off[2] + (T)dz * hh;
                                        T dsum = fa * wz;
                                        if (K != ROTLET) dsum += fb * (-2 * a2 * ez * wz);
                                        if (K == STRESSLET) dsum += fc * ((4 * a2 * a2 * ez * ez - 2 * a2) * wz);
                                        acc[z][ncA] += dsum;
                                    } else if constexpr (CM == CM_GRIDS) {
#pragma unroll
                                        for (int c = 0; c < ncB; ++c) acc[z][ncA + c] += wv * cv(ncA + c);
                                    }
                                }
                            }
                        }
                    }
                }
                __syncthreads();
            }
        }
    }
    const int Mt = g.Mt;
    if (i < Mt && j < Mt) {
#pragma unroll
        for (int z = 0; z < TZ; ++z) {
            int l = l0 + z;
            if (l < 2 * Mt) {
                long long node = ((long long)l * Mt + j) * Mt + i;
#pragma unroll
                for (int c = 0; c < nout; ++c) grids[c * cs + node] = acc[z][c];
            }
        }
    }
}

template <typename T, int CM, int TZ>
static void launch_spread_tz(int family, GridArgs g, const T* rec, const uint32_t* toff, T* grids, long long cs,
                             hipStream_t st)
{
    dim3 grid(g.nt[0], g.nt[1], g.nt[2]);
    size_t lds = (size_t)SP_CHUNK * record_stride(family, g.P, sizeof(T)) * sizeof(T);
    switch (family) {
        case STOKESLET: hipLaunchKernelGGL((k_spread<T, STOKESLET, TZ, CM>), grid, dim3(64), lds, st, g, rec, toff, grids, cs); break;
        case STRESSLET: hipLaunchKernelGGL((k_spread<T, STRESSLET, 4, CM>), grid, dim3(64), lds, st, g, rec, toff, grids, cs); break;
        default: hipLaunchKernelGGL((k_spread<T, ROTLET, TZ, CM>), grid, dim3(64), lds, st, g, rec, toff, grids, cs); break;
    }
}

template <typename T, int CM>
static void launch_spread_t(int family, GridArgs g, const T* rec, const uint32_t* toff, T* grids, long long cs,
                            hipStream_t st)
{
    // the tile depth is the planner's (the stresslet's is always 4)
    if (g.tile[2] == 8)
        launch_spread_tz<T, CM, 8>(family, g, rec, toff, grids, cs, st);
    else
        launch_spread_tz<T, CM, 4>(family, g, rec, toff, grids, cs, st);
}

template <typename T>
hipError_t launch_spread(int family, int cm, GridArgs g, const T* rec, const uint32_t* toff, T* grids, long long cs,
                         hipStream_t st)
{
    if (cm == CM_FREE)
        launch_spread_t<T, CM_FREE>(family, g, rec, toff, grids, cs, st);
    else if (cm == CM_DENSITY)
        launch_spread_t<T, CM_DENSITY>(family, g, rec, toff, grids, cs, st);
    else
        launch_spread_t<T, CM_GRIDS>(family, g, rec, toff, grids, cs, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// gather (quadrature) and the FP64 combination u = u_R + self + u_F:
//   u_F(x) = h^3 sum_nodes W(x - x_g) [T1(x_g) - x3 T2(x_g)],  T2 = grad phi.
// FP64 (GQ): the grids hold T1 (0..2) and the potential phi (3), and T2 is
// formed here as the gradient of the potential's quadrature,
//   grad_x W(x - x_g) = 2 a (x_g - x) W,  separable like W;
// FP32: the grids hold T1 (0..2) and T2 (3..5).
//
// Node-owner form, the adjoint of the spreading: the targets are sorted by
// the 8^3-node tile that holds the first node of their support; one
// wavefront owns a tile (lane = one (x1, x2) column of 8 nodes along x3, held
// in registers) and, for every target whose support reaches the tile, forms
// the six partial sums over the tile's nodes and reduces them across the
// wavefront.  Each grid node is read once (a target-per-wavefront gather
// reads every node about ten times, once per target whose support holds
// it).  The partial sums go to one slot per (target, tile); a last pass adds
// a target's slots in a fixed order, so the result is deterministic.
// ---------------------------------------------------------------------------
constexpr int GT_CHUNK = 8;  // target records staged in LDS per chunk

// header of 4 int32 (support base x, y, z; cell-sorted target index), then
// the 3 Pg factors of W along x1, x2, x3 (the first carries the prefactor)
// and, with GQ, their derivatives 2 a (x_g - x) w
__host__ __device__ __forceinline__ size_t trec_stride(int Pg, size_t esz)
{
    return 16 / esz + (esz == 8 ? 6 : 3) * (size_t)Pg;
}
size_t target_record_stride(int Pg, size_t esz) { return trec_stride(Pg, esz); }

int gather_slots(const GridArgs& gg)
{
    const int ks = gg.K[0] + 1;
    return ks * ks * ks;
}

__global__ void k_target_keys(const double* __restrict__ xs, long long TT, GridArgs gg, uint32_t* __restrict__ keys,
                              uint32_t* __restrict__ idx)
{
    long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= TT) return;
    const int dims[3] = {gg.Mt, gg.Mt, 2 * gg.Mt};
    int b[3];
    for (int a = 0; a < 3; ++a) b[a] = support_base(xs[a * TT + t], gg.o[a], gg.h, gg.P, dims[a]) / gg.tile[a];
    keys[t] = (uint32_t)(((long long)b[2] * gg.nt[1] + b[1]) * gg.nt[0] + b[0]);
    idx[t] = (uint32_t)t;
}

hipError_t launch_target_keys(const double* xs, long long TT, GridArgs gg, uint32_t* keys, uint32_t* idx,
                              hipStream_t st)
{
    if (TT <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_target_keys, dim3((unsigned)((TT + 255) / 256)), dim3(256), 0, st, xs, TT, gg, keys, idx);
    return hipGetLastError();
}

// Morton (Z-order) key of the bin (support base >> shift, per axis) of each
// target: consecutive keys stay close along all three axes
__device__ __forceinline__ uint32_t spread_bits3(uint32_t v)
{
    uint32_t r = 0;
    for (int i = 0; i < 11; ++i) r |= ((v >> i) & 1u) << (3 * i);
    return r;
}

__global__ void k_target_zkeys(const double* __restrict__ xs, long long TT, GridArgs gg, int shift,
                               uint32_t* __restrict__ keys, uint32_t* __restrict__ idx)
{
    long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= TT) return;
    const int dims[3] = {gg.Mt, gg.Mt, 2 * gg.Mt};
    uint32_t k = 0;
    for (int a = 0; a < 3; ++a)
        k |= spread_bits3((uint32_t)(support_base(xs[a * TT + t], gg.o[a], gg.h, gg.P, dims[a]) >> shift)) << a;
    keys[t] = k;
    idx[t] = (uint32_t)t;
}

hipError_t launch_target_zkeys(const double* xs, long long TT, GridArgs gg, int shift, uint32_t* keys, uint32_t* idx,
                               hipStream_t st)
{
    if (TT <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_target_zkeys, dim3((unsigned)((TT + 255) / 256)), dim3(256), 0, st, xs, TT, gg, shift, keys,
                       idx);
    return hipGetLastError();
}

// one wavefront per (tile-sorted) target
template <typename T>
__global__ void __launch_bounds__(64) k_target_records(const double* __restrict__ xs, const uint32_t* __restrict__ perm,
                                                       long long TT, GridArgs gg, T* __restrict__ rec)
{
    constexpr bool GQ = Out<T, CM_GRIDS>::grad_quad;
    const long long r = blockIdx.x;
    const int lane = threadIdx.x;
    const int Pg = gg.P;
    const long long t = perm[r];
    const double x[3] = {xs[t], xs[TT + t], xs[2 * TT + t]};
    const int dims[3] = {gg.Mt, gg.Mt, 2 * gg.Mt};
    int base[3];
    for (int a = 0; a < 3; ++a) base[a] = support_base(x[a], gg.o[a], gg.h, Pg, dims[a]);
    const long long stride = (long long)trec_stride(Pg, sizeof(T));
    T* R = rec + r * stride;
    if (lane == 0) {
        int* hdr = reinterpret_cast<int*>(R);
        hdr[0] = base[0];
        hdr[1] = base[1];
        hdr[2] = base[2];
        hdr[3] = (int)t;
    }
    T* w = R + 16 / sizeof(T);
    for (int f = lane; f < 3 * Pg; f += 64) {
        const int a = f / Pg, q = f - a * Pg;
        const double dd = gg.o[a] + (base[a] + q) * gg.h - x[a];
        double v = exp(-gg.a2 * dd * dd);
        if (a == 0) v *= gg.pref;
        w[f] = (T)v;
        if (GQ) w[3 * Pg + f] = (T)(2.0 * gg.a2 * dd * v);
    }
}

template <typename T>
hipError_t launch_target_records(const double* xs, const uint32_t* perm, long long TT, GridArgs gg, T* rec,
                                 hipStream_t st)
{
    if (TT <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_target_records<T>, dim3((unsigned)TT), dim3(64), 0, st, xs, perm, TT, gg, rec);
    return hipGetLastError();
}

// grid: (nt0, nt1, nt2 - tz0): tiles from x3 tile tz0 up (no target's support
// reaches lower)
template <typename T>
__global__ void __launch_bounds__(64) k_gather_tiles(GridArgs gg, const T* __restrict__ grids, long long cs,
                                                     const T* __restrict__ rec, const uint32_t* __restrict__ gtoff,
                                                     int tz0, T* __restrict__ part)
{
    constexpr bool GQ = Out<T, CM_GRIDS>::grad_quad;
    constexpr int NOUT = Out<T, CM_GRIDS>::n;
    extern __shared__ unsigned char smem_raw[];
    T* sh = reinterpret_cast<T*>(smem_raw);
    const int Pg = gg.P, Mt = gg.Mt;
    const int stride = (int)trec_stride(Pg, sizeof(T));
    const int lane = threadIdx.x;
    const int tx = blockIdx.x, ty = blockIdx.y, tz = tz0 + (int)blockIdx.z;
    const int i = tx * 8 + (lane & 7), j = ty * 8 + (lane >> 3), l0 = tz * 8;
    // this lane's column: NOUT grids at 8 nodes along x3 (zero outside the grid)
    T gv[8][NOUT];
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const int l = l0 + z;
        const bool ok = i < Mt && j < Mt && l < 2 * Mt;
        const long long node = ok ? ((long long)l * Mt + j) * Mt + i : 0;
#pragma unroll
        for (int c = 0; c < NOUT; ++c) gv[z][c] = ok ? grids[c * cs + node] : (T)0;
    }
    const int K = gg.K[0], KS = K + 1;
    const int x_lo = tx - K < 0 ? 0 : tx - K;
    // staged per target: its header and, for each factor array (W along x1,
    // x2, x3 and, with GQ, their derivatives), the 8 entries that fall on
    // this tile (zero outside the support), so lanes index them by their
    // own position in the tile
    constexpr int NA = GQ ? 6 : 3;
    constexpr int HS = 16 / sizeof(T);
    constexpr int SS = HS + 8 * NA;
    const int org[3] = {tx * 8, ty * 8, l0};
    for (int sz = tz - K; sz <= tz; ++sz) {
        if (sz < 0) continue;
        for (int sy = ty - K; sy <= ty; ++sy) {
            if (sy < 0) continue;
            const long long row = ((long long)sz * gg.nt[1] + sy) * gg.nt[0];
            const uint32_t r0 = gtoff[row + x_lo], r1 = gtoff[row + tx + 1];
            for (uint32_t c0 = r0; c0 < r1; c0 += GT_CHUNK) {
                const int nr = (int)min((uint32_t)GT_CHUNK, r1 - c0);
                for (int f = lane; f < nr * SS; f += 64) {
                    const int q = f / SS, e = f - q * SS;
                    const T* R = rec + (long long)(c0 + q) * stride;
                    if (e < HS) {
                        sh[f] = R[e];
                    } else {
                        const int k = e - HS, arr = k >> 3, u = k & 7, ax = arr % 3;
                        const int off = org[ax] + u - reinterpret_cast<const int*>(R)[ax];
                        sh[f] = (off >= 0 && off < Pg) ? R[HS + arr * Pg + off] : (T)0;
                    }
                }
                __syncthreads();
                for (int q = 0; q < nr; ++q) {
                    const T* r = sh + q * SS;
                    const int* hdr = reinterpret_cast<const int*>(r);
                    const int bx = hdr[0], by = hdr[1], bz = hdr[2];
                    // this tile beyond the support's last tile: nothing to add
                    // (wavefront-uniform; the first tile is never beyond this one)
                    if (tx > (bx + Pg - 1) / 8 || ty > (by + Pg - 1) / 8 || tz > (bz + Pg - 1) / 8) continue;
                    const T* w = r + HS;  // [array][8]
                    const T wx = w[lane & 7], wy = w[8 + (lane >> 3)];
                    const T dwx = GQ ? w[24 + (lane & 7)] : (T)0, dwy = GQ ? w[32 + (lane >> 3)] : (T)0;
                    T s[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
                    for (int z = 0; z < 8; ++z) {
                        const T wz = w[16 + z];
                        const T wyz = wy * wz;
                        const T wv = wx * wyz;
#pragma unroll
                        for (int c = 0; c < 3; ++c) s[c] += wv * gv[z][c];
                        if (GQ) {
                            const T ph = gv[z][3];
                            s[3] += dwx * wyz * ph;
                            s[4] += wx * dwy * wz * ph;
                            s[5] += wx * wy * w[40 + z] * ph;
                        } else {
#pragma unroll
                            for (int c = 3; c < 6; ++c) s[c] += wv * gv[z][c < NOUT ? c : 0];
                        }
                    }
#pragma unroll
                    for (int c = 0; c < 6; ++c) {
                        T v = s[c];
                        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                        s[c] = v;
                    }
                    if (lane == 0) {
                        const int slot = ((tz - bz / 8) * KS + (ty - by / 8)) * KS + (tx - bx / 8);
                        T* o = part + ((long long)(c0 + q) * (KS * KS * KS) + slot) * 6;
#pragma unroll
                        for (int c = 0; c < 6; ++c) o[c] = s[c];
                    }
                }
                __syncthreads();
            }
        }
    }
}

template <typename T>
hipError_t launch_gather_tiles(GridArgs gg, const T* grids, long long cs, const T* rec, const uint32_t* gtoff,
                               int tz0, T* part, hipStream_t st)
{
    const int nz = gg.nt[2] - tz0;
    if (nz <= 0) return hipSuccess;
    size_t lds = (size_t)GT_CHUNK * (16 / sizeof(T) + 8 * (sizeof(T) == 8 ? 6 : 3)) * sizeof(T);
    hipLaunchKernelGGL(k_gather_tiles<T>, dim3(gg.nt[0], gg.nt[1], nz), dim3(64), lds, st, gg, grids, cs, rec, gtoff,
                       tz0, part);
    return hipGetLastError();
}

// one thread per (tile-sorted) target: its slots, in order over the tiles of
// its support box, then u = u_R + h^3 (T1 - x3 T2)
template <typename T>
__global__ void k_gather_final(GridArgs gg, const T* __restrict__ rec, const T* __restrict__ part, long long TT,
                               const double* __restrict__ xs, const uint32_t* __restrict__ tperm,
                               const double* __restrict__ upart, double* __restrict__ uout)
{
    const long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (r >= TT) return;
    const int Pg = gg.P;
    const long long stride = (long long)trec_stride(Pg, sizeof(T));
    const int* hdr = reinterpret_cast<const int*>(rec + r * stride);
    const int b[3] = {hdr[0], hdr[1], hdr[2]};
    const long long t = hdr[3];
    const int KS = gg.K[0] + 1;
    const T* ps = part + r * (long long)(KS * KS * KS) * 6;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int dz = 0; dz <= (b[2] + Pg - 1) / 8 - b[2] / 8; ++dz)
        for (int dy = 0; dy <= (b[1] + Pg - 1) / 8 - b[1] / 8; ++dy)
            for (int dx = 0; dx <= (b[0] + Pg - 1) / 8 - b[0] / 8; ++dx) {
                const T* o = ps + ((dz * KS + dy) * KS + dx) * 6;
#pragma unroll
                for (int c = 0; c < 6; ++c) acc[c] += (double)o[c];
            }
    const long long o = tperm[t];
    const double x3 = xs[2 * TT + t];
    const double h3 = gg.h * gg.h * gg.h;
    for (int a = 0; a < 3; ++a) uout[3 * o + a] = upart[3 * o + a] + h3 * (acc[a] - x3 * acc[3 + a]);
}

template <typename T>
hipError_t launch_gather_final(GridArgs gg, const T* rec, const T* part, long long TT, const double* xs,
                               const uint32_t* tperm, const double* upart, double* uout, hipStream_t st)
{
    if (TT <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_final<T>, dim3((unsigned)((TT + 255) / 256)), dim3(256), 0, st, gg, rec, part, TT, xs,
                       tperm, upart, uout);
    return hipGetLastError();
}

// Target-per-wavefront form, for small supports and dense targets (where
// the per-tile reductions of the node-owner form cost more than the repeated
// reads, which then hit L2 more often): one wavefront per target, its lanes
// over whole x1 rows of the support where those fill at least 90 % of them,
// else over the flattened Pg^3 support (Pg = 22: 44 of 64 lanes in rows,
// quadrature 2.9 -> 2.5 ms at N = 1e5); blocks of 4 consecutive (cell-sorted, so
// nearby) targets, spread over the XCDs in contiguous ranges so that
// overlapping supports share an L2.
template <typename T, int CM>
__global__ void __launch_bounds__(256) k_gather(GridArgs g, const T* __restrict__ grids, long long cs,
                                                const double* __restrict__ xs, const uint32_t* __restrict__ tperm,
                                                long long TT, const double* __restrict__ upart,
                                                double* __restrict__ uout)
{
    constexpr bool GQ = Out<T, CM>::grad_quad;
    // free space: the kernel grid's three outputs only (no -x3 grad phi)
    constexpr bool FREE = CM == CM_FREE;
    __shared__ T wsh[4][3 * 32];              // W factors along x1, x2, x3
    __shared__ T dsh[4][GQ ? 3 * 32 : 1];     // their derivatives with respect to the target
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // blocks of 4 consecutive (cell-sorted, so nearby) targets, spread over the
    // XCDs in contiguous ranges so that overlapping supports share an L2
    const long long nblk = (TT + 3) / 4;
    const long long t_raw = xcd_block(blockIdx.x, nblk) * 4LL + wv;
    const bool valid = t_raw < TT;  // no early exit: every wave reaches the barrier
    const long long t = valid ? t_raw : TT - 1;
    const int P = g.P, Mt = g.Mt;
    const double x[3] = {xs[t], xs[TT + t], xs[2 * TT + t]};
    int dims[3] = {Mt, Mt, 2 * Mt};
    int base[3];
    for (int a = 0; a < 3; ++a) base[a] = support_base(x[a], g.o[a], g.h, P, dims[a]);
    for (int f = lane; f < 3 * P; f += 64) {
        int a = f / P, q = f - a * P;
        double d = g.o[a] + (base[a] + q) * g.h - x[a];
        double v = exp(-g.a2 * d * d);
        if (a == 0) v *= g.pref;
        wsh[wv][f] = (T)v;
        if (GQ) dsh[wv][f] = (T)(2.0 * g.a2 * d * v);
    }
    __syncthreads();
    T acc[6] = {0, 0, 0, 0, 0, 0};
    const int rows = 64 / P;
    if (10 * rows * P >= 9 * 64) {
        // lanes cover P consecutive x1 nodes of `rows` rows at a time (at
        // least 90 % of the lanes busy)
        const int row = fdiv(lane, P, g.mP), xi = lane - row * P;
        if (row < rows) {
            const T wx = wsh[wv][xi];
            const T dx = GQ ? dsh[wv][xi] : (T)0;
#pragma unroll 4
            for (int rr = row; rr < P * P; rr += rows) {
                int dz = fdiv(rr, P, g.mP), dy = rr - dz * P;
                const T wy = wsh[wv][P + dy], wz = wsh[wv][2 * P + dz];
                const T wyz = wy * wz;
                const T w = wx * wyz;
                long long node = ((long long)(base[2] + dz) * Mt + base[1] + dy) * Mt + base[0] + xi;
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[c] += w * grids[c * cs + node];
                if (GQ) {
                    const T gx = dx * wyz, gy = wx * dsh[wv][P + dy] * wz, gz = wx * wy * dsh[wv][2 * P + dz];
                    const T ph = grids[3 * cs + node];
                    acc[3] += gx * ph;
                    acc[4] += gy * ph;
                    acc[5] += gz * ph;
                } else if (!FREE) {
#pragma unroll
                    for (int c = 3; c < 6; ++c) acc[c] += w * grids[c * cs + node];
                }
            }
        }
    } else {
        // the P^3 support nodes, x1 fastest, flattened over the 64 lanes: lane
        // takes node f = lane + 64 i, its (x1, x2, x3) offsets advanced by those
        // of 64 with carries, so every lane is busy whatever P is
        const int P2 = P * P, n3 = P2 * P;
        const int sx = 64 - fdiv(64, P, g.mP) * P;  // 64 = (sz P + sy) P + sx
        const int q64 = fdiv(64, P, g.mP);
        const int sz = fdiv(q64, P, g.mP), sy = q64 - sz * P;
        int r0 = fdiv(lane, P, g.mP);
        int xi = lane - r0 * P;
        int dz = fdiv(r0, P, g.mP);
        int dy = r0 - dz * P;
#pragma unroll 2
        for (int f = lane; f < n3; f += 64) {
            const T wx = wsh[wv][xi], wy = wsh[wv][P + dy], wz = wsh[wv][2 * P + dz];
            const T wyz = wy * wz;
            const T w = wx * wyz;
            long long node = ((long long)(base[2] + dz) * Mt + base[1] + dy) * Mt + base[0] + xi;
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c] += w * grids[c * cs + node];
            if (GQ) {
                const T gx = dsh[wv][xi] * wyz, gy = wx * dsh[wv][P + dy] * wz, gz = wx * wy * dsh[wv][2 * P + dz];
                const T ph = grids[3 * cs + node];
                acc[3] += gx * ph;
                acc[4] += gy * ph;
                acc[5] += gz * ph;
            } else if (!FREE) {
#pragma unroll
                for (int c = 3; c < 6; ++c) acc[c] += w * grids[c * cs + node];
            }
            xi += sx;
            dy += sy;
            dz += sz;
            if (xi >= P) {
                xi -= P;
                ++dy;
            }
            if (dy >= P) {
                dy -= P;
                ++dz;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        T v = acc[c];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[c] = v;
    }
    if (lane == 0 && valid) {
        long long o = tperm[t];
        double h3 = g.h * g.h * g.h;
        for (int a = 0; a < 3; ++a)
            uout[3 * o + a] = upart[3 * o + a] + h3 * ((double)acc[a] - (FREE ? 0.0 : x[2] * (double)acc[3 + a]));
    }
}

// Quadrature for dense targets, several per wavefront.  The targets are
// sorted along a Morton curve over 2^3-node bins of their support base (so
// that consecutive ones lie close along all three axes); a wavefront takes GK
// consecutive ones and walks the union of their supports once -- lanes own
// (x1, x2) node pairs of it, 64 at a time, and walk the x3 column -- so each
// grid value is read once for the group and weighted for each of its
// targets (by zero outside the target's own support).  The 1D factors of
// each target over the union, and their derivatives, sit in LDS.  A group
// whose union is wider than GX nodes on some axis, or holds more nodes than
// the targets' own supports together, is taken one target at a time.  Per target the sums run over the same nodes with the same factors
// as in the one-target form, in another order.
constexpr int GK = 4;
constexpr int GX = GATHER_GX;

template <typename T, int CM>
__global__ void __launch_bounds__(64) k_gather_group(GridArgs g, const T* __restrict__ grids, long long cs,
                                                     const double* __restrict__ xs, const uint32_t* __restrict__ gperm,
                                                     const uint32_t* __restrict__ tperm, long long TT,
                                                     const double* __restrict__ upart, double* __restrict__ uout)
{
    constexpr bool GQ = Out<T, CM>::grad_quad;
    constexpr bool FREE = CM == CM_FREE;
    constexpr int NC = FREE ? 3 : 6;                   // sums per target
    constexpr int NG = FREE ? 3 : GQ ? 4 : 6;          // grids read per node
    __shared__ T tab[GK][3][GX][2];                    // (factor, derivative) per target, axis, union node
    __shared__ double sx[GK][3];
    __shared__ int sb[GK][3];
    __shared__ uint32_t sti[GK];
    const int lane = threadIdx.x;
    const long long ng = (TT + GK - 1) / GK;
    const long long grp = xcd_block(blockIdx.x, ng);
    if (grp >= ng) return;  // whole block
    const long long s0 = grp * GK;
    const int nt = (int)min((long long)GK, TT - s0);
    const int P = g.P, Mt = g.Mt;
    if (lane < GK * 3) {
        const int k = lane / 3, a = lane - 3 * k;
        const uint32_t t = gperm[s0 + (k < nt ? k : nt - 1)];
        const double xa = xs[a * TT + t];
        const int dims = a == 2 ? 2 * Mt : Mt;
        sx[k][a] = xa;
        sb[k][a] = support_base(xa, g.o[a], g.h, P, dims);
        if (a == 0) sti[k] = t;
    }
    __syncthreads();
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = sb[0][a];
        hi[a] = sb[0][a];
        for (int k = 1; k < nt; ++k) {
            lo[a] = min(lo[a], sb[k][a]);
            hi[a] = max(hi[a], sb[k][a]);
        }
        hi[a] += P;
    }
    // one walk over the union only where it is no longer than the targets'
    // own walks together (sparse groups go one target at a time)
    const bool together = hi[0] - lo[0] <= GX && hi[1] - lo[1] <= GX && hi[2] - lo[2] <= GX &&
                          (long long)(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]) <=
                              (long long)nt * P * P * P;

    // factors of targets k0 .. k0 + nk - 1 over the window L .. L + E - 1
    auto fill = [&](int k0, int nk, const int* L, const int* E) {
        for (int f = lane; f < GK * 3 * GX; f += 64) {
            const int kk = f / (3 * GX), r = f - kk * (3 * GX), a = r / GX, e = r - a * GX;
            T w = 0, dw = 0;
            if (kk < nk && e < E[a]) {
                const int k = k0 + kk, n = L[a] + e;
                if (n >= sb[k][a] && n < sb[k][a] + P) {
                    const double d = g.o[a] + n * g.h - sx[k][a];
                    double v = exp(-g.a2 * d * d);
                    if (a == 0) v *= g.pref;
                    w = (T)v;
                    if (GQ) dw = (T)(2.0 * g.a2 * d * v);
                }
            }
            tab[kk][a][e][0] = w;
            tab[kk][a][e][1] = dw;
        }
    };
    auto at = [&](const T* gb, int c, unsigned ob) -> T {
        return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(gb + c * cs) + ob);
    };
    // the walk over the window for NK targets, then their sums and outputs
    auto walk = [&](auto nk_c, int k0, const int* L, const int* E) {
        constexpr int NK = decltype(nk_c)::value;
        T acc[NK][6];
#pragma unroll
        for (int k = 0; k < NK; ++k)
#pragma unroll
            for (int c = 0; c < 6; ++c) acc[k][c] = (T)0;
        const T* gb = grids + ((long long)L[2] * Mt + L[1]) * Mt + L[0];
        const unsigned zstep = (unsigned)((long long)Mt * Mt * (long long)sizeof(T));
        const int E2 = E[0] * E[1];
        for (int p0 = 0; p0 < E2; p0 += 64) {
            const bool on = p0 + lane < E2;
            const int pr = on ? p0 + lane : E2 - 1;
            const int dy = pr / E[0], xi = pr - dy * E[0];
            T wxy[NK], gxy[NK], gyx[NK];
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                const T wx = on ? tab[k][0][xi][0] : (T)0, wy = tab[k][1][dy][0];
                wxy[k] = wx * wy;
                gxy[k] = GQ ? (on ? tab[k][0][xi][1] : (T)0) * wy : (T)0;
                gyx[k] = GQ ? wx * tab[k][1][dy][1] : (T)0;
            }
            unsigned ob = (unsigned)((dy * Mt + xi) * (int)sizeof(T));
#pragma unroll 2
            for (int dz = 0; dz < E[2]; ++dz) {
                T v[NG];
#pragma unroll
                for (int c = 0; c < NG; ++c) v[c] = at(gb, c, ob);
#pragma unroll
                for (int k = 0; k < NK; ++k) {
                    const T wz = tab[k][2][dz][0];
                    const T w = wxy[k] * wz;
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[k][c] += w * v[c];
                    if (GQ) {
                        acc[k][3] += (gxy[k] * wz) * v[3];
                        acc[k][4] += (gyx[k] * wz) * v[3];
                        acc[k][5] += (wxy[k] * tab[k][2][dz][1]) * v[3];
                    } else if (!FREE) {
#pragma unroll
                        for (int c = 3; c < NC; ++c) acc[k][c] += w * v[c];
                    }
                }
                ob += zstep;
            }
        }
#pragma unroll
        for (int k = 0; k < NK; ++k)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                T v = acc[k][c];
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                acc[k][c] = v;
            }
        if (lane == 0) {
            const double h3 = g.h * g.h * g.h;
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                if (k0 + k >= nt) continue;
                const long long o = tperm[sti[k0 + k]];
                const double x3 = sx[k0 + k][2];
                for (int a = 0; a < 3; ++a)
                    uout[3 * o + a] =
                        upart[3 * o + a] + h3 * ((double)acc[k][a] - (FREE ? 0.0 : x3 * (double)acc[k][3 + a]));
            }
        }
    };
    if (together) {
        const int E[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
        fill(0, nt, lo, E);
        __syncthreads();
        walk(std::integral_constant<int, GK>{}, 0, lo, E);
    } else {
        const int E[3] = {P, P, P};
        for (int k = 0; k < nt; ++k) {
            __syncthreads();  // the previous target's factors are read
            const int L[3] = {sb[k][0], sb[k][1], sb[k][2]};
            fill(k, 1, L, E);
            __syncthreads();
            walk(std::integral_constant<int, 1>{}, k, L, E);
        }
    }
}

template <typename T>
hipError_t launch_gather_group(GridArgs g, int cm, const T* grids, long long cs, const double* xs,
                               const uint32_t* gperm, const uint32_t* tperm, long long T_, const double* upart,
                               double* uout, hipStream_t st)
{
    if (T_ <= 0) return hipSuccess;
    if (!gather_group_fits(g.P, g.Mt, sizeof(T))) return hipErrorInvalidValue;
    const long long ng = (T_ + GK - 1) / GK;
    const long long nlaunch = (ng + NXCD - 1) / NXCD * NXCD;  // every XCD range padded to full length
    if (cm == CM_FREE)
        hipLaunchKernelGGL((k_gather_group<T, CM_FREE>), dim3((unsigned)nlaunch), dim3(64), 0, st, g, grids, cs, xs,
                           gperm, tperm, T_, upart, uout);
    else
        hipLaunchKernelGGL((k_gather_group<T, CM_GRIDS>), dim3((unsigned)nlaunch), dim3(64), 0, st, g, grids, cs, xs,
                           gperm, tperm, T_, upart, uout);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(GridArgs g, int cm, const T* grids, long long cs, const double* xs, const uint32_t* tperm,
                         long long T_, const double* upart, double* uout, hipStream_t st)
{
    if (T_ <= 0) return hipSuccess;
    const long long nblk = (T_ + 3) / 4;
    const long long nlaunch = (nblk + NXCD - 1) / NXCD * NXCD;  // every XCD range padded to full length
    if (cm == CM_FREE)
        hipLaunchKernelGGL((k_gather<T, CM_FREE>), dim3((unsigned)nlaunch), dim3(256), 0, st, g, grids, cs, xs, tperm,
                           T_, upart, uout);
    else
        hipLaunchKernelGGL((k_gather<T, CM_GRIDS>), dim3((unsigned)nlaunch), dim3(256), 0, st, g, grids, cs, xs, tperm,
                           T_, upart, uout);
    return hipGetLastError();
}

template hipError_t launch_records<double>(int, int, const double*, const double*, const uint32_t*, long long,
                                           GridArgs, double*, hipStream_t);
template hipError_t launch_records<float>(int, int, const double*, const double*, const uint32_t*, long long,
                                          GridArgs, float*, hipStream_t);
template hipError_t launch_spread<double>(int, int, GridArgs, const double*, const uint32_t*, double*, long long,
                                          hipStream_t);
template hipError_t launch_spread<float>(int, int, GridArgs, const float*, const uint32_t*, float*, long long,
                                         hipStream_t);
template hipError_t launch_gather_group<double>(GridArgs, int, const double*, long long, const double*,
                                                const uint32_t*, const uint32_t*, long long, const double*, double*,
                                                hipStream_t);
template hipError_t launch_gather_group<float>(GridArgs, int, const float*, long long, const double*, const uint32_t*,
                                               const uint32_t*, long long, const double*, double*, hipStream_t);
template hipError_t launch_gather<double>(GridArgs, int, const double*, long long, const double*, const uint32_t*,
                                          long long, const double*, double*, hipStream_t);
template hipError_t launch_gather<float>(GridArgs, int, const float*, long long, const double*, const uint32_t*, long long,
                                         const double*, double*, hipStream_t);
template hipError_t launch_target_records<double>(const double*, const uint32_t*, long long, GridArgs, double*,
                                                  hipStream_t);
template hipError_t launch_target_records<float>(const double*, const uint32_t*, long long, GridArgs, float*,
                                                 hipStream_t);
template hipError_t launch_gather_tiles<double>(GridArgs, const double*, long long, const double*, const uint32_t*,
                                                int, double*, hipStream_t);
template hipError_t launch_gather_tiles<float>(GridArgs, const float*, long long, const float*, const uint32_t*, int,
                                               float*, hipStream_t);
template hipError_t launch_gather_final<double>(GridArgs, const double*, const double*, long long, const double*,
                                                const uint32_t*, const double*, double*, hipStream_t);
template hipError_t launch_gather_final<float>(GridArgs, const float*, const float*, long long, const double*,
                                               const uint32_t*, const double*, double*, hipStream_t);

}  // namespace ehs
