// Zero-padded 3D transforms of the Fourier-space pipeline and the truncated
// Green's-function precompute.
//
// Grid conventions (one component shown; components are stacked):
//   real grid   R[l][j][i]      i,j < Mt (x1, x2), l < 2 Mt (x3)
//   after X     A[k1][l][j]     k1 <= Mt (half spectrum of the 2Mt padded x1 axis)
//   after Y     Z[k1][k2][l]    k2 < 2Mt (padded x2 axis), l < 2Mt (unpadded x3)
// The x3 transform (padded to 4 Mt), the k-space scaling and the inverse x3
// transform are fused into one pass over Z, so the 2Mt x 2Mt x 4Mt spectrum is
// never written to memory.  The inverse passes mirror the forward ones and keep
// only the unpadded M~ x M~ x 2M~ block.
//
// Zero padding by 2 along an axis is done without touching the zeros: for a
// line x_t, t < n, padded to 2n, the even outputs X[2m] are DFT_n(x)[m] and the
// odd outputs X[2m+1] are DFT_n(x_t e^{-i pi t/n})[m].  Along x3 the same
// identity is used with Q "phases" k3 = Q m + s.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace ehs {

constexpr int PASS_NT = 256;  // threads of the y passes
constexpr int XPASS_NT = 512; // threads of the x passes
constexpr int PASS_E = 16;    // complex elements per thread in the LDS FFT
constexpr int Z_E = 16;

// ---------------------------------------------------------------------------
// forward x pass: real lines of Mt values, zero-padded to 2Mt, half spectrum
// k1 = 0..Mt.  Two real lines are packed into one complex line; both padding
// halves of every packed line are transformed together (2 * B/2 lines).
// grid: (ceil(Mt / B), 2Mt, ncomp); B even.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(XPASS_NT, 4) k_fwd_x(const T* __restrict__ in, cplx<T>* __restrict__ out, PassArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
    const int Mt = a.Mt, B = a.B, ld = Mt + 1;
    const int j0 = blockIdx.x * B, l = blockIdx.y, c = blockIdx.z;
    if (c >= a.czero && l >= a.lzc) return;  // a vanishing row: never read downstream
    const int nb = min(B, Mt - j0);
    const cplx<T>* tw2 = static_cast<const cplx<T>*>(a.tw2);
    const T* src = in + (long long)c * a.cs_in + ((long long)l * Mt + j0) * Mt;
    const int np = B / 2;
    cplx<T>* twl = buf + B * ld;
    load_stage_twiddles<T, XPASS_NT>(twl, a.fM);
    constexpr int LB = 4;  // independent loads in flight per thread
    for (int f0 = threadIdx.x; f0 < np * Mt; f0 += LB * XPASS_NT) {
        T va[LB], vb[LB];
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            int f = f0 + u * XPASS_NT;
            int p = fdiv(f, Mt, a.mMt), i = f - p * Mt;
            const bool ok = f < np * Mt;
            va[u] = (ok && 2 * p < nb) ? src[(2 * p) * Mt + i] : (T)0;
            vb[u] = (ok && 2 * p + 1 < nb) ? src[(2 * p + 1) * Mt + i] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            int f = f0 + u * XPASS_NT;
            if (f < np * Mt) {
                int p = fdiv(f, Mt, a.mMt), i = f - p * Mt;
                cplx<T> z = cmk<T>(va[u], vb[u]);
                buf[(2 * p) * ld + i] = z;
                buf[(2 * p + 1) * ld + i] = cmul(z, tw2[i]);
            }
        }
    }
    __syncthreads();
    lds_fft<T, XPASS_NT, PASS_E, false>(buf, ld, B, a.fM, twl);
    // unpack the two real spectra: A = (Z[k] + conj Z[-k]) / 2, B = (Z[k] - conj Z[-k]) / 2i
    cplx<T>* dst = out + (long long)c * a.cs_out + (long long)l * Mt + j0;
    const long long rowk = (long long)2 * Mt * Mt;  // stride of k1
    for (int f = threadIdx.x; f < (Mt + 1) * B; f += XPASS_NT) {
        int k = fdiv(f, B, a.mB), b = f - k * B;
        if (b >= nb) continue;
        int p = b >> 1, s = k & 1, m = k >> 1;
        int mm = Mt - m - s;
        if (mm >= Mt) mm -= Mt;
        cplx<T> zk = buf[(2 * p + s) * ld + m];
        cplx<T> zn = cconj(buf[(2 * p + s) * ld + mm]);
        cplx<T> r;
        if ((b & 1) == 0)
            r = cmk<T>((T)0.5 * (zk.x + zn.x), (T)0.5 * (zk.y + zn.y));
        else
            r = cmk<T>((T)0.5 * (zk.y - zn.y), (T)-0.5 * (zk.x - zn.x));
        dst[k * rowk + b] = r;
    }
}

// ---------------------------------------------------------------------------
// forward y pass: complex lines along j (Mt values, contiguous), padded to
// 2Mt; the even and odd k2 halves are transformed one after the other with
// the input lines kept in registers.  output Z[k1][k2][l] (l fastest): every
// block writes B consecutive l (one 128-byte segment) per k2.
// grid: (ceil(2Mt / B), Mt + 1, ncomp)
// ---------------------------------------------------------------------------
template <typename T, int MAXR>
__global__ void __launch_bounds__(PASS_NT) k_fwd_y(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out, PassArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
    const int Mt = a.Mt, B = a.B, ld = Mt + 1;
    const int l0 = blockIdx.x * B, k1l = blockIdx.y, k1 = a.k1base + k1l, c = blockIdx.z;
    // rows l >= lzc of the vanishing components: skipped here, treated as
    // zero by the x3 pass
    if (c >= a.czero && l0 >= a.lzc) return;
    const int nl = 2 * Mt;
    const int nb = min(B, nl - l0);
    const int nbr = c >= a.czero ? min(nb, a.lzc - l0) : nb;  // rows read (the rest are zero)
    const cplx<T>* tw2 = static_cast<const cplx<T>*>(a.tw2);
    const cplx<T>* src = in + (long long)c * a.cs_in + ((long long)k1 * nl + l0) * Mt;
    cplx<T>* twl = buf + B * ld;
    load_stage_twiddles<T, PASS_NT>(twl, a.fM);
    cplx<T> x[MAXR];
    int jj[MAXR], bb[MAXR];
#pragma unroll
    for (int i = 0; i < MAXR; ++i) {
        int f = threadIdx.x + i * PASS_NT;
        x[i] = cmk<T>(0, 0);
        jj[i] = -1;
        bb[i] = 0;
        if (f < B * Mt) {
            int b = fdiv(f, Mt, a.mMt);
            jj[i] = f - b * Mt;
            bb[i] = b;
            if (b < nbr) x[i] = src[f];
        }
    }
    cplx<T>* dst = out + (long long)c * a.cs_out + (long long)k1l * nl * nl + l0;
    for (int s = 0; s < 2; ++s) {
#pragma unroll
        for (int i = 0; i < MAXR; ++i)
            if (jj[i] >= 0) buf[bb[i] * ld + jj[i]] = s ? cmul(x[i], tw2[jj[i]]) : x[i];
        __syncthreads();
        lds_fft<T, PASS_NT, PASS_E, false>(buf, ld, B, a.fM, twl);
        for (int f = threadIdx.x; f < Mt * B; f += PASS_NT) {
            int m = fdiv(f, B, a.mB), b = f - m * B;
            if (b < nb) dst[(long long)(2 * m + s) * nl + b] = buf[b * ld + m];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// inverse y pass: lines along k2 (2Mt values, stride 2Mt), keep j < Mt; the
// even and odd k2 halves are transformed one after the other and combined in
// registers.  output D[k1][l][j] for l >= l3lo.
// grid: (ceil((2Mt - l3lo) / B), nk1, ncomp)
// ---------------------------------------------------------------------------
template <typename T, int MAXR>
__global__ void __launch_bounds__(PASS_NT) k_inv_y(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out, PassArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
    const int Mt = a.Mt, B = a.B, ld = Mt + 1;
    const int l0 = a.l3lo + blockIdx.x * B, k1l = blockIdx.y, k1 = a.k1base + k1l, c = blockIdx.z;
    const int nl = 2 * Mt;
    const int nb = min(B, nl - l0);
    const cplx<T>* tw2 = static_cast<const cplx<T>*>(a.tw2);
    const cplx<T>* src = in + (long long)c * a.cs_in + (long long)k1l * nl * nl + l0;
    cplx<T>* twl = buf + B * ld;
    load_stage_twiddles<T, PASS_NT>(twl, a.fM);
    cplx<T> acc[MAXR];
    for (int s = 0; s < 2; ++s) {
        // rows of B values (one 128-byte segment) spread over 2Mt rows: issue
        // LB independent loads per thread before their LDS stores
        constexpr int LB = 4;
        for (int f0 = threadIdx.x; f0 < Mt * B; f0 += LB * PASS_NT) {
            cplx<T> v[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                int f = f0 + u * PASS_NT;
                int m = fdiv(f, B, a.mB), b = f - m * B;
                v[u] = (f < Mt * B && b < nb) ? src[(long long)(2 * m + s) * nl + b] : cmk<T>(0, 0);
            }
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                int f = f0 + u * PASS_NT;
                if (f < Mt * B) {
                    int m = fdiv(f, B, a.mB), b = f - m * B;
                    buf[b * ld + m] = v[u];
                }
            }
        }
        __syncthreads();
        lds_fft<T, PASS_NT, PASS_E, true>(buf, ld, B, a.fM, twl);
#pragma unroll
        for (int i = 0; i < MAXR; ++i) {
            int f = threadIdx.x + i * PASS_NT;
            if (f < B * Mt) {
                int b = fdiv(f, Mt, a.mMt), t = f - b * Mt;
                cplx<T> v = buf[b * ld + t];
                acc[i] = s ? cadd(acc[i], cmul(v, cconj(tw2[t]))) : v;
            }
        }
        __syncthreads();
    }
    cplx<T>* dst = out + (long long)c * a.cs_out + ((long long)k1 * nl + l0) * Mt;
#pragma unroll
    for (int i = 0; i < MAXR; ++i) {
        int f = threadIdx.x + i * PASS_NT;
        if (f < nb * Mt) dst[f] = acc[i];
    }
}

// ---------------------------------------------------------------------------
// inverse x pass (complex-to-real): lines along k1 (Mt + 1 values of the half
// spectrum), keep i < Mt.  Two real output lines share one complex line.
// output R[l][j][i] for l >= l3lo.  grid: (ceil(Mt / B), 2Mt - l3lo, ncomp); B even.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(XPASS_NT, 4) k_inv_x(const cplx<T>* __restrict__ in, T* __restrict__ out, PassArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
    const int Mt = a.Mt, B = a.B, ld = Mt + 1;
    const int j0 = blockIdx.x * B, l = a.l3lo + blockIdx.y, c = blockIdx.z;
    const int nb = min(B, Mt - j0);
    const cplx<T>* tw2 = static_cast<const cplx<T>*>(a.tw2);
    const cplx<T>* src = in + (long long)c * a.cs_in + (long long)l * Mt + j0;
    const long long rowk = (long long)2 * Mt * Mt;
    const int hB = B / 2;
    cplx<T>* twl = buf + B * ld;
    load_stage_twiddles<T, XPASS_NT>(twl, a.fM);
    // Z_p[k] = Ya[k] + i Yb[k] over the full padded range k < 2Mt; the
    // position k = 2m + s is stored at buf[(2p + s) * ld + m].
    constexpr int LB = 4;  // independent loads in flight per thread
    for (int part = 0; part < 2; ++part) {
        for (int f0 = threadIdx.x; f0 < (Mt + 1) * hB; f0 += LB * XPASS_NT) {
          cplx<T> vv[LB];
#pragma unroll
          for (int u = 0; u < LB; ++u) {
            int f = f0 + u * XPASS_NT;
            int k = fdiv(f, hB, a.mB2), p = f - k * hB;
            int b = 2 * p + part;
            vv[u] = (f < (Mt + 1) * hB && b < nb) ? src[k * rowk + b] : cmk<T>(0, 0);
          }
#pragma unroll
          for (int u = 0; u < LB; ++u) {
            int f = f0 + u * XPASS_NT;
            if (f >= (Mt + 1) * hB) break;
            int k = fdiv(f, hB, a.mB2), p = f - k * hB;
            cplx<T> v = vv[u];
            if (k == 0 || k == Mt) v.y = 0;  // self-conjugate bins are real
            cplx<T> w1 = part ? cmul_pi(v) : v;
            int s = k & 1, m = k >> 1;
            cplx<T>* d1 = &buf[(2 * p + s) * ld + m];
            *d1 = part ? cadd(*d1, w1) : w1;
            if (k > 0 && k < Mt) {
                int k2 = 2 * Mt - k;
                cplx<T> v2 = cconj(v);
                cplx<T> w2 = part ? cmul_pi(v2) : v2;
                cplx<T>* d2 = &buf[(2 * p + (k2 & 1)) * ld + (k2 >> 1)];
                *d2 = part ? cadd(*d2, w2) : w2;
            }
          }
        }
        __syncthreads();
    }
    lds_fft<T, XPASS_NT, PASS_E, true>(buf, ld, B, a.fM, twl);
    T* dst = out + (long long)c * a.cs_out + ((long long)l * Mt + j0) * Mt;
    for (int f = threadIdx.x; f < nb * Mt; f += XPASS_NT) {
        int b = fdiv(f, Mt, a.mMt), t = f - b * Mt;
        int p = b >> 1;
        cplx<T> r0 = buf[(2 * p) * ld + t];
        cplx<T> r1 = buf[(2 * p + 1) * ld + t];
        cplx<T> y = cadd(r0, cmul(r1, cconj(tw2[t])));
        dst[f] = (b & 1) ? y.y : y.x;
    }
}

// ---------------------------------------------------------------------------
// k-space multipliers (the scaling step).  X: the ncin transformed grids at
// one wave vector; Y: the six outputs Y1 = t1 + e3 phi, Y2 = i k phi.
//   gB = (1 + k^2/4xi^2) e^{-(1-eta) k^2/4xi^2} B^R(k) / Npad
//   gH =                e^{-(1-eta) k^2/4xi^2} H^R(k) / Npad
// ---------------------------------------------------------------------------
template <typename U, bool GQ, int CM>
__device__ __forceinline__ void mult_stokeslet(const cplx<U>* X, cplx<U>* Y, U kx, U ky, U kz, U gB, U gH)
{
    U k2 = kx * kx + ky * ky + kz * kz;
    // t1 = -(k^2 I - k k) C1 * gB   (the A^S(k) of the stokeslet)
    cplx<U> kc = cmk<U>(kx * X[0].x + ky * X[1].x + kz * X[2].x, kx * X[0].y + ky * X[1].y + kz * X[2].y);
    U kv[3] = {kx, ky, kz};
#pragma unroll
    for (int q = 0; q < 3; ++q) Y[q] = cmk<U>(-gB * (k2 * X[q].x - kv[q] * kc.x), -gB * (k2 * X[q].y - kv[q] * kc.y));
    if (CM == CM_FREE) return;
    // phi = gH (-2 C2 - 2 i k.C3), or gH D when the density D was spread
    cplx<U> phi;
    if (CM == CM_DENSITY) {
        phi = cmk<U>(gH * X[3].x, gH * X[3].y);
    } else {
        cplx<U> kc3 = cmk<U>(kx * X[4].x + ky * X[5].x + kz * X[6].x, kx * X[4].y + ky * X[5].y + kz * X[6].y);
        phi = cmk<U>(gH * (-2 * X[3].x + 2 * kc3.y), gH * (-2 * X[3].y - 2 * kc3.x));
    }
    Y[2] = cadd(Y[2], phi);
    if (GQ) {
        Y[3] = phi;
    } else {
#pragma unroll
        for (int q = 0; q < 3; ++q) Y[3 + q] = cmk<U>(-kv[q] * phi.y, kv[q] * phi.x);  // i k phi
    }
}

template <typename U, bool GQ, int CM>
__device__ __forceinline__ void mult_stresslet(const cplx<U>* X, cplx<U>* Y, U kx, U ky, U kz, U gB, U gH)
{
    U k2 = kx * kx + ky * ky + kz * kz;
    // C1 symmetric: xx xy xz yy yz zz
    cplx<U> ck[3];
    ck[0] = cmk<U>(X[0].x * kx + X[1].x * ky + X[2].x * kz, X[0].y * kx + X[1].y * ky + X[2].y * kz);
    ck[1] = cmk<U>(X[1].x * kx + X[3].x * ky + X[4].x * kz, X[1].y * kx + X[3].y * ky + X[4].y * kz);
    ck[2] = cmk<U>(X[2].x * kx + X[4].x * ky + X[5].x * kz, X[2].y * kx + X[4].y * ky + X[5].y * kz);
    cplx<U> tr = cmk<U>(X[0].x + X[3].x + X[5].x, X[0].y + X[3].y + X[5].y);
    cplx<U> kck = cmk<U>(kx * ck[0].x + ky * ck[1].x + kz * ck[2].x, kx * ck[0].y + ky * ck[1].y + kz * ck[2].y);
    U kv[3] = {kx, ky, kz};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        // t1 = -i gB [k^2 (2 C k + k trC) - 2 k (k.C k)]
        cplx<U> s = cmk<U>(k2 * (2 * ck[q].x + kv[q] * tr.x) - 2 * kv[q] * kck.x,
                           k2 * (2 * ck[q].y + kv[q] * tr.y) - 2 * kv[q] * kck.y);
        Y[q] = cmk<U>(gB * s.y, -gB * s.x);
    }
    if (CM == CM_FREE) return;
    // C3 symmetric (indices 7..12), phi = gH (4 i kz C2 + 4 k.C3.k), or gH D
    cplx<U> phi;
    if (CM == CM_DENSITY) {
        phi = cmk<U>(gH * X[6].x, gH * X[6].y);
    } else {
        const cplx<U>* B3 = X + 7;
        U kbk_x = kx * kx * B3[0].x + ky * ky * B3[3].x + kz * kz * B3[5].x +
                  2 * (kx * ky * B3[1].x + kx * kz * B3[2].x + ky * kz * B3[4].x);
        U kbk_y = kx * kx * B3[0].y + ky * ky * B3[3].y + kz * kz * B3[5].y +
                  2 * (kx * ky * B3[1].y + kx * kz * B3[2].y + ky * kz * B3[4].y);
        phi = cmk<U>(gH * (-4 * kz * X[6].y + 4 * kbk_x), gH * (4 * kz * X[6].x + 4 * kbk_y));
    }
    Y[2] = cadd(Y[2], phi);
    if (GQ) {
        Y[3] = phi;
    } else {
#pragma unroll
        for (int q = 0; q < 3; ++q) Y[3 + q] = cmk<U>(-kv[q] * phi.y, kv[q] * phi.x);  // i k phi
    }
}

template <typename U, bool GQ, int CM>
__device__ __forceinline__ void mult_rotlet(const cplx<U>* X, cplx<U>* Y, U kx, U ky, U kz, U gH)
{
    // t1 = -2 i gH (C1 x k)
    cplx<U> cx[3];
    cx[0] = cmk<U>(X[1].x * kz - X[2].x * ky, X[1].y * kz - X[2].y * ky);
    cx[1] = cmk<U>(X[2].x * kx - X[0].x * kz, X[2].y * kx - X[0].y * kz);
    cx[2] = cmk<U>(X[0].x * ky - X[1].x * kx, X[0].y * ky - X[1].y * kx);
    U kv[3] = {kx, ky, kz};
#pragma unroll
    for (int q = 0; q < 3; ++q) Y[q] = cmk<U>(2 * gH * cx[q].y, -2 * gH * cx[q].x);
    if (CM == CM_FREE) return;
    // phi = gH 2 i (kx w1 + ky w2), or gH D
    cplx<U> phi;
    if (CM == CM_DENSITY) {
        phi = cmk<U>(gH * X[3].x, gH * X[3].y);
    } else {
        cplx<U> kw = cmk<U>(kx * X[3].x + ky * X[4].x, kx * X[3].y + ky * X[4].y);
        phi = cmk<U>(-2 * gH * kw.y, 2 * gH * kw.x);
    }
    Y[2] = cadd(Y[2], phi);
    if (GQ) {
        Y[3] = phi;
    } else {
#pragma unroll
        for (int q = 0; q < 3; ++q) Y[3 + q] = cmk<U>(-kv[q] * phi.y, kv[q] * phi.x);  // i k phi
    }
}

template <typename U, int K, bool GQ, int CM>
__device__ __forceinline__ void apply_mult(const cplx<U>* X, cplx<U>* Y, U kx, U ky, U kz, U gB, U gH)
{
    if (K == STOKESLET)
        mult_stokeslet<U, GQ, CM>(X, Y, kx, ky, kz, gB, gH);
    else if (K == STRESSLET)
        mult_stresslet<U, GQ, CM>(X, Y, kx, ky, kz, gB, gH);
    else
        mult_rotlet<U, GQ, CM>(X, Y, kx, ky, kz, gH);
}

// ---------------------------------------------------------------------------
// fused x3 pass: for one (k1, k2) line, zero-padded forward transform along
// x3 (length 4Mt, input 2Mt), scaling by the multiplier, inverse transform,
// keep l < 2Mt.  The padded axis is split into Q phases,
//   X[Q m + s] = DFT_{4Mt/Q}( sum_h x[l' + h nq] w^{s (l' + h nq)} )[m],
// w = exp(-2 pi i / 4Mt), and the inverse accumulates the phases back.
//
// One block per (k1, k2) line with one wavefront per component line (at most
// 8); wavefront w owns the input components w, w + 8 and the output
// component w.  Folding, the forward and inverse
// transforms and unfolding of a component touch only its own LDS line, so
// they run at wavefront scope without block barriers and the waves proceed
// independently; only the scaling, which couples the components at each k,
// is bracketed by two block barriers per phase.  Outputs are produced for
// l >= l3lo only (the nodes the quadrature reads).  EPL > 0: each lane holds
// its EPL output elements (l = l3lo + lane + 64 e) in registers, and with
// HOLD its 2 EPL input elements (l = lane + 64 e) too, so inputs are read
// once and outputs written once; EPL = 0: inputs re-read and outputs
// accumulated in zout.
// grid: (2Mt, nk1)
// ---------------------------------------------------------------------------
// wavefronts per block: one per line, at most 8
template <typename T, int K, int CM>
struct ZWaves {
    static constexpr int lines = InGrids<K, CM>::n > Out<T, CM>::n ? InGrids<K, CM>::n : Out<T, CM>::n;
    static constexpr int n = lines < 8 ? lines : 8;
};

// occupancy target (wavefronts per SIMD): two blocks per CU.  With four
// wavefronts per block that is two per SIMD.  FP32 stokeslet and rotlet
// blocks have six or seven wavefronts and need four per SIMD (128 registers,
// which their variants with at most 4 outputs per lane and no held inputs
// fit; their LDS allows it); FP64 blocks of more wavefronts are held to one
// block per CU by the LDS anyway, and the FP32 stresslet's 13 input lines do
// not fit 128 registers.
template <typename T, int K, int CM, int EPL>
struct ZOcc {
    static constexpr int n = (sizeof(T) == 4 && ZWaves<T, K, CM>::n > 4 && K != STRESSLET && EPL <= 4) ? 4 : 2;
};

// inputs held in registers (HOLD): 2 EPL elements per lane cover the whole
// input line when 128 EPL >= 2Mt; only where they fit a register budget of
// 32 per lane (more spills in the FP64 variants)
template <typename T, int K, int CM, int EPL>
constexpr bool z_hold_fits()
{
    constexpr int zw = ZWaves<T, K, CM>::n;
    constexpr int cpw = (InGrids<K, CM>::n + zw - 1) / zw;
    return EPL > 0 && EPL <= 8 && cpw * 2 * EPL * (int)sizeof(cplx<T>) <= 128 && ZOcc<T, K, CM, EPL>::n == 2;
}

template <typename T, int K, int EPL, bool HOLD, int CM>
__global__ void __launch_bounds__((64 * ZWaves<T, K, CM>::n), (ZOcc<T, K, CM, EPL>::n))
    k_z_scale(const cplx<T>* zb, cplx<T>* zout, ZArgs a)
{
    constexpr int ZW = ZWaves<T, K, CM>::n;
    constexpr int Z_NT = 64 * ZW;
    constexpr int ncin = InGrids<K, CM>::n;
    constexpr int NCOUT = Out<T, CM>::n;
    constexpr bool GQ = Out<T, CM>::grad_quad;
    // the harmonic kernel's octant: the corrections, and the rotlet's kernel
    constexpr bool NEED_H = CM != CM_FREE || K == ROTLET;
    constexpr int CPW = (ncin + ZW - 1) / ZW;  // input components per wavefront
    static_assert(!HOLD || z_hold_fits<T, K, CM, EPL>(), "held inputs exceed the register budget");
    constexpr int EPI = HOLD ? 2 * EPL : 1;  // held input elements per lane and component
    constexpr int NX = HOLD ? CPW * EPI : 1;
    constexpr int NY = EPL > 0 ? EPL : 1;
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
    const int Mt = a.Mt, Q = a.Q;
    const int nz = 2 * Mt, n4 = 4 * Mt, nq = n4 / Q, ld = nq + 1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int k2 = blockIdx.x, k1 = a.k1base + (int)blockIdx.y;
    const long long cs = a.cs;
    const long long base = ((long long)blockIdx.y * nz + k2) * nz;
    const cplx<T>* tw4 = static_cast<const cplx<T>*>(a.tw4);
    const unsigned mnq = a.mnq, mn4 = a.mn4;
    const int nh = nz / nq;  // 1 (Q = 2), 2 (Q = 4) or 4 (Q = 8)
    const int l3lo = a.l3lo;  // output element e of a lane is l = l3lo + lane + 64 e
    constexpr int NL = ncin > NCOUT ? ncin : NCOUT;  // LDS lines
    cplx<T>* twl = buf + NL * ld;                    // stage twiddles of the line FFT
    load_stage_twiddles<T, Z_NT>(twl, a.fq);
    __syncthreads();
    constexpr int MJ = (1024 + Z_NT - 1) / Z_NT;  // wave numbers per thread (4Mt / Q <= 1024)

    cplx<T> xin[NX];
    cplx<T> yout[NY];
#pragma unroll
    for (int e = 0; e < NY; ++e) yout[e] = cmk<T>(0, 0);
    if (HOLD) {
#pragma unroll
        for (int ci = 0; ci < CPW; ++ci) {
            const int c = w + ci * ZW;
#pragma unroll
            for (int e = 0; e < EPI; ++e) {
                const int l = lane + 64 * e;
                const bool rd = c < ncin && l < nz && (c < a.czero || l < a.lzc);
                xin[ci * EPI + e] = rd ? zb[c * cs + base + l] : cmk<T>(0, 0);
            }
        }
    }

    // signed wave numbers of this line
    const int k2s = (k2 < Mt) ? k2 : k2 - nz;
    const int ak2 = k2s < 0 ? -k2s : k2s;
    const bool nyq12 = (k1 == Mt) || (k2 == Mt);
    const double kxd = a.dk12 * k1, kyd = a.dk12 * k2s;
    const long long oct_line = ((long long)k1 * (Mt + 1) + ak2) * (2 * Mt + 1);
    // the screening factor exp(-c k^2) is separable: the in-plane part once
    // per line, the x3 part from the table ez[|k3|]
    const double exy = exp(-a.c_exp * (kxd * kxd + kyd * kyd));

    for (int s = 0; s < Q; ++s) {
        // the multiplier samples of this phase's wave numbers k3 = Q m + s:
        // raw loads (every index valid, m clamped), issued before the fold so
        // that their latency overlaps the forward transform; they are combined
        // into the multipliers only in the scaling step
        using OT = typename std::conditional<sizeof(T) == 8, double, float>::type;
        const OT* octH = sizeof(T) == 8 ? (const OT*)a.octH64 : (const OT*)a.octH32;
        const OT* octB = sizeof(T) == 8 ? (const OT*)a.octB64 : (const OT*)a.octB32;
        // (with 16 outputs per lane the registers do not allow it: loaded in
        // the scaling step instead)
        constexpr bool PREF = EPL < 16;
        double pez[MJ];
        OT poh[MJ], pob[MJ];
        auto load_mult = [&](int j) {
            const int m = min((int)threadIdx.x + j * Z_NT, nq - 1);
            const int k3 = Q * m + s;
            const int k3s = (k3 < nz) ? k3 : k3 - n4;
            const int ak3 = k3s < 0 ? -k3s : k3s;
            pez[j] = a.ez[ak3];
            poh[j] = NEED_H ? octH[oct_line + ak3] : (OT)0;
            pob[j] = K != ROTLET ? octB[oct_line + ak3] : (OT)0;
        };
        if (PREF) {
#pragma unroll
            for (int j = 0; j < MJ; ++j) load_mult(j);
        }
        // fold and twist each owned input component into its LDS line:
        //   line c holds sum_h x_c[l' + h nq] w^{s (l' + h nq)},  l' < nq
        // (the twist factors are loaded with the data, ahead of their use)
#pragma unroll
        for (int ci = 0; ci < CPW; ++ci) {
            const int c = w + ci * ZW;
            if (c >= ncin) break;  // wavefront-uniform
            cplx<T>* line = buf + c * ld;
            for (int h = 0; h < nh; ++h) {
                if (h) wave_sync();
                if (HOLD) {
                    cplx<T> t[EPI];
#pragma unroll
                    for (int e = 0; e < EPI; ++e) {
                        const int l = min(lane + 64 * e, nz - 1);
                        int ti = s * l;  // < 4Mt when Q = 2 (nh = 1)
                        if (nh != 1) ti -= fdiv(ti, n4, mn4) * n4;
                        t[e] = s ? tw4[ti] : cmk<T>(1, 0);
                    }
#pragma unroll
                    for (int e = 0; e < EPI; ++e) {
                        const int l = lane + 64 * e;
                        if (l < nz) {
                            const int lq = nh == 1 ? 0 : fdiv(l, nq, mnq);
                            if (lq == h) {
                                cplx<T> v = xin[ci * EPI + e];
                                if (s) v = cmul(v, t[e]);
                                const int lp = l - lq * nq;
                                if (h == 0)
                                    line[lp] = v;
                                else
                                    line[lp] = cadd(line[lp], v);
                            }
                        }
                    }
                } else {
                    // LB loads of data and twist factors per lane in flight
                    // before their stores
                    constexpr int LB = EPL >= 16 ? (CPW > 1 ? 2 : 4) : 8;
                    for (int lp0 = lane; lp0 < nq; lp0 += LB * 64) {
                        cplx<T> v[LB], t[LB];
#pragma unroll
                        for (int u = 0; u < LB; ++u) {
                            const int lp = lp0 + u * 64;
                            const bool rd = lp < nq && (c < a.czero || lp + h * nq < a.lzc);
                            v[u] = rd ? zb[c * cs + base + lp + h * nq] : cmk<T>(0, 0);
                            int ti = s * (min(lp, nq - 1) + h * nq);
                            if (nh != 1) ti -= fdiv(ti, n4, mn4) * n4;
                            t[u] = s ? tw4[ti] : cmk<T>(1, 0);
                        }
                        if (h == 0) {
#pragma unroll
                            for (int u = 0; u < LB; ++u) {
                                const int lp = lp0 + u * 64;
                                if (lp < nq) line[lp] = s ? cmul(v[u], t[u]) : v[u];
                            }
                        } else {
#pragma unroll
                            for (int u = 0; u < LB; ++u) {
                                const int lp = lp0 + u * 64;
                                if (lp < nq) line[lp] = cadd(line[lp], s ? cmul(v[u], t[u]) : v[u]);
                            }
                        }
                    }
                }
            }
            wave_sync();
            lds_fft<T, 64, Z_E, false, true>(line, ld, 1, a.fq, twl);
        }
        __syncthreads();

        // scaling at k3 = Q m + s (couples the components)
#pragma unroll
        for (int j = 0; j < MJ; ++j) {
            const int m = threadIdx.x + j * Z_NT;
            if (m >= nq) break;
            if (!PREF) load_mult(j);
            int k3 = Q * m + s;
            int k3s = (k3 < nz) ? k3 : k3 - n4;
            int ak3 = k3s < 0 ? -k3s : k3s;
            cplx<T> X[ncin];
#pragma unroll
            for (int c = 0; c < ncin; ++c) X[c] = buf[c * ld + m];
            cplx<T> Y[NCOUT];
            if (nyq12 || k3 == nz) {
#pragma unroll
                for (int c = 0; c < NCOUT; ++c) Y[c] = cmk<T>(0, 0);
            } else {
                double kzd = a.dk3 * k3s;
                bool near0 = (k1 <= a.near0) && (ak2 <= a.near0) && (ak3 <= 2 * a.near0);
                if (sizeof(T) == 8 || near0) {
                    double k2v = kxd * kxd + kyd * kyd + kzd * kzd;
                    double gB, gH;
                    if (sizeof(T) == 8) {
                        const double ep = exy * pez[j];
                        gH = ep * a.cH * (double)poh[j];
                        gB = K != ROTLET ? (1.0 + a.c_has * k2v) * (ep * a.cB * (double)pob[j]) : 0.0;
                    } else {
                        // FP32 path near k = 0: FP64 multipliers
                        const long long oi = oct_line + ak3;
                        const double ep = exy * a.ez[ak3];
                        gH = NEED_H ? ep * a.cH * a.octH64[oi] : 0.0;
                        gB = K != ROTLET ? (1.0 + a.c_has * k2v) * (ep * a.cB * a.octB64[oi]) : 0.0;
                    }
                    cplx<double> Xd[ncin], Yd[NCOUT_MAX];
#pragma unroll
                    for (int c = 0; c < ncin; ++c) Xd[c] = cmk<double>((double)X[c].x, (double)X[c].y);
                    apply_mult<double, K, GQ, CM>(Xd, Yd, kxd, kyd, kzd, gB, gH);
#pragma unroll
                    for (int c = 0; c < NCOUT; ++c) Y[c] = cmk<T>((T)Yd[c].x, (T)Yd[c].y);
                } else {
                    float kx = (float)kxd, ky = (float)kyd, kz = (float)kzd;
                    float k2v = kx * kx + ky * ky + kz * kz;
                    const double ep = exy * pez[j];
                    float gH = (float)(ep * a.cH) * (float)poh[j];
                    float gB = K != ROTLET ? (1.f + (float)a.c_has * k2v) * ((float)(ep * a.cB) * (float)pob[j]) : 0.f;
                    cplx<float> Xf[ncin], Yf[NCOUT_MAX];
#pragma unroll
                    for (int c = 0; c < ncin; ++c) Xf[c] = cmk<float>((float)X[c].x, (float)X[c].y);
                    apply_mult<float, K, GQ, CM>(Xf, Yf, kx, ky, kz, gB, gH);
#pragma unroll
                    for (int c = 0; c < NCOUT; ++c) Y[c] = cmk<T>((T)Yf[c].x, (T)Yf[c].y);
                }
            }
#pragma unroll
            for (int c = 0; c < NCOUT; ++c) buf[c * ld + m] = Y[c];
        }
        __syncthreads();

        // inverse transform and unfold of the owned output component:
        //   out_c[l] += line_c[l mod nq] w^{-s l},  l < 2Mt
        if (w < NCOUT) {
            cplx<T>* line = buf + w * ld;
            lds_fft<T, 64, Z_E, true, true>(line, ld, 1, a.fq, twl);
            if (EPL > 0) {
                // twist factors loaded in batches of UB ahead of their use
                constexpr int UB = NY >= 16 ? 4 : (NY < 8 ? NY : 8);
#pragma unroll
                for (int e0 = 0; e0 < NY; e0 += UB) {
                    cplx<T> t[UB];
                    if (s) {
#pragma unroll
                        for (int u = 0; u < UB; ++u) {
                            int ti = s * min(l3lo + lane + 64 * (e0 + u), nz - 1);
                            if (nh != 1) ti -= fdiv(ti, n4, mn4) * n4;
                            t[u] = tw4[ti];
                        }
                    }
                    // with at most 8 outputs per lane no branch per element
                    // (the LDS reads of a batch are in flight together):
                    // positions past the line are clamped, and their sums are
                    // never written; with more the registers do not allow it
#pragma unroll
                    for (int u = 0; u < UB; ++u) {
                        const int l = l3lo + lane + 64 * (e0 + u);
                        if (NY > 8 && l >= nz) continue;
                        const int lc = min(l, nz - 1);
                        const int lq = nh == 1 ? 0 : fdiv(lc, nq, mnq);
                        cplx<T> v = line[lc - lq * nq];
                        if (s) v = cmul(v, cconj(t[u]));
                        yout[e0 + u] = cadd(yout[e0 + u], v);
                    }
                }
            } else {
                for (int l = l3lo + lane; l < nz; l += 64) {
                    const int lq = nh == 1 ? 0 : fdiv(l, nq, mnq);
                    cplx<T> v = line[l - lq * nq];
                    if (s) {
                        int ti = s * l;
                        if (nh != 1) ti -= fdiv(ti, n4, mn4) * n4;
                        v = cmul(v, cconj(tw4[ti]));
                    }
                    cplx<T>* o = zout + w * a.cs_out + base + l;
                    *o = (s == 0) ? v : cadd(*o, v);
                }
            }
            wave_sync();
        }
    }
    if (EPL > 0 && w < NCOUT) {
#pragma unroll
        for (int e = 0; e < NY; ++e) {
            const int l = l3lo + lane + 64 * e;
            if (l < nz) zout[w * a.cs_out + base + l] = yout[e];
        }
    }
}

// ---------------------------------------------------------------------------
// precompute: one real, even line transform per block.
//   v[t] = in[min(t, n - t)] (even extension of the stored half line), t < n
//   out[k] = scale * Re sum_t v[t] exp(-2 pi i k t / n),  k < nkeep
// In generate mode the input is the analytic kernel K^R(|k|) sampled on the
// oversampled grid, for the octant indices (o1, o2) of the block.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_even_line(const double* __restrict__ in, double* __restrict__ out,
                                                    EvenArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    cplx<double>* buf = reinterpret_cast<cplx<double>*>(smem_raw);
    long long g = blockIdx.x + (long long)gridDim.x * blockIdx.y;
    if (g >= (long long)a.n1 * a.n2) return;
    int o1 = (int)(g / a.n2), o2 = (int)(g - (long long)o1 * a.n2);
    const int n = a.f.n;
    for (int t = threadIdx.x; t < n; t += 256) {
        int tt = (t <= n - t) ? t : n - t;
        double v;
        if (a.generate) {
            // octant indices (o1, o2) along the two oversampled in-plane axes and
            // tt along the current axis
            double k1 = a.dkg1 * o1, k2 = a.dkg1 * o2, k3 = a.dkg3 * tt;
            v = khat_truncated(a.kind, sqrt(k1 * k1 + k2 * k2 + k3 * k3), a.R);
        } else {
            v = in[(long long)o1 * a.si1 + (long long)o2 * a.si2 + (long long)tt * a.st];
        }
        buf[t] = cmk<double>(v, 0.0);
    }
    __syncthreads();
    lds_fft<double, 256, 16, false>(buf, n, 1, a.f, static_cast<const cplx<double>*>(a.f.tws));
    for (int k = threadIdx.x; k < a.nkeep; k += 256)
        out[(long long)o1 * a.so1 + (long long)o2 * a.so2 + (long long)k * a.sk] = a.scale * buf[k].x;
}

// ez[t] = exp(-c (dk t)^2), t < n: the x3 factor of the screening exponential
__global__ void k_exp_table(double* __restrict__ ez, int n, double c, double dk)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        double k = dk * t;
        ez[t] = exp(-c * k * k);
    }
}

hipError_t launch_exp_table(double* ez, int n, double c, double dk, hipStream_t st)
{
    hipLaunchKernelGGL(k_exp_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ez, n, c, dk);
    return hipGetLastError();
}

__global__ void k_oct_to_f32(const double* __restrict__ in, float* __restrict__ out, long long n)
{
    long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

// debug / unit-test entry: nl independent FFTs of length p.n, each line
// contiguous, one block handling `per` lines.
template <typename T, bool INV>
__global__ void __launch_bounds__(PASS_NT) k_line_fft(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out, int nl,
                                                       int per, FftPlanDev p)
{
    extern __shared__ unsigned char smem_raw[];
    cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem_raw);
    const int n = p.n, ld = n + 1;
    int l0 = blockIdx.x * per;
    int nb = min(per, nl - l0);
    for (int f = threadIdx.x; f < per * n; f += PASS_NT) {
        int b = f / n, t = f - b * n;  // debug kernel: plain division
        buf[b * ld + t] = (b < nb) ? in[(long long)(l0 + b) * n + t] : cmk<T>(0, 0);
    }
    __syncthreads();
    lds_fft<T, PASS_NT, PASS_E, INV>(buf, ld, per, p, static_cast<const cplx<T>*>(p.tws));
    for (int f = threadIdx.x; f < nb * n; f += PASS_NT) {
        int b = f / n, t = f - b * n;
        out[(long long)(l0 + b) * n + t] = buf[b * ld + t];
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
// B lines of Mt + 1 complex values and the Mt - 1 stage twiddles (rounded up to Mt)
size_t pass_lds(int Mt, int B, size_t esz) { return ((size_t)B * (Mt + 1) + Mt) * 2 * esz; }

template <typename T>
hipError_t launch_fwd_x(const T* in, cplx<T>* out, const PassArgs& a, int ncomp, hipStream_t st)
{
    dim3 grid((a.Mt + a.B - 1) / a.B, 2 * a.Mt, ncomp);
    hipLaunchKernelGGL(k_fwd_x<T>, grid, dim3(XPASS_NT), pass_lds(a.Mt, a.B, sizeof(T)), st, in, out, a);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_fwd_y(const cplx<T>* in, cplx<T>* out, const PassArgs& a, int ncomp, hipStream_t st)
{
    dim3 grid((2 * a.Mt + a.B - 1) / a.B, a.nk1, ncomp);
    size_t lds = pass_lds(a.Mt, a.B, sizeof(T));
    if (a.B * a.Mt <= 8 * PASS_NT)
        hipLaunchKernelGGL((k_fwd_y<T, 8>), grid, dim3(PASS_NT), lds, st, in, out, a);
    else
        hipLaunchKernelGGL((k_fwd_y<T, 16>), grid, dim3(PASS_NT), lds, st, in, out, a);  // B Mt <= 16 PASS_NT
    return hipGetLastError();
}
template <typename T>
hipError_t launch_inv_y(const cplx<T>* in, cplx<T>* out, const PassArgs& a, int ncomp, hipStream_t st)
{
    dim3 grid((2 * a.Mt - a.l3lo + a.B - 1) / a.B, a.nk1, ncomp);
    size_t lds = pass_lds(a.Mt, a.B, sizeof(T));
    if (a.B * a.Mt <= 8 * PASS_NT)
        hipLaunchKernelGGL((k_inv_y<T, 8>), grid, dim3(PASS_NT), lds, st, in, out, a);
    else
        hipLaunchKernelGGL((k_inv_y<T, 16>), grid, dim3(PASS_NT), lds, st, in, out, a);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_inv_x(const cplx<T>* in, T* out, const PassArgs& a, int ncomp, hipStream_t st)
{
    dim3 grid((a.Mt + a.B - 1) / a.B, 2 * a.Mt - a.l3lo, ncomp);
    hipLaunchKernelGGL(k_inv_x<T>, grid, dim3(XPASS_NT), pass_lds(a.Mt, a.B, sizeof(T)), st, in, out, a);
    return hipGetLastError();
}

template <typename T, int K, int CM, int EPL>
static void launch_z_e(cplx<T>* zb, cplx<T>* zout, const ZArgs& a, hipStream_t st)
{
    dim3 grid(2 * a.Mt, a.nk1);
    size_t lds = z_lds_bytes(K, CM, a.Mt, a.Q, sizeof(T));
    const dim3 blk(64 * ZWaves<T, K, CM>::n);
    if constexpr (z_hold_fits<T, K, CM, EPL>()) {
        if (128 * EPL >= 2 * a.Mt) {
            hipLaunchKernelGGL((k_z_scale<T, K, EPL, true, CM>), grid, blk, lds, st, zb, zout, a);
            return;
        }
    }
    hipLaunchKernelGGL((k_z_scale<T, K, EPL, false, CM>), grid, blk, lds, st, zb, zout, a);
}

template <typename T, int K, int CM>
static void launch_z_t(cplx<T>* zb, cplx<T>* zout, const ZArgs& a, bool res, hipStream_t st)
{
    const int no = 2 * a.Mt - a.l3lo;  // outputs per line
    if (!res)
        launch_z_e<T, K, CM, 0>(zb, zout, a, st);
    else if (no <= 256)
        launch_z_e<T, K, CM, 4>(zb, zout, a, st);
    else if (no <= 512)
        launch_z_e<T, K, CM, 8>(zb, zout, a, st);
    else
        launch_z_e<T, K, CM, 16>(zb, zout, a, st);  // no <= 1024 (the planner's audit)
}

template <typename T, int CM>
static void launch_z_f(int family, cplx<T>* zb, cplx<T>* zout, const ZArgs& a, bool res, hipStream_t st)
{
    switch (family) {
        case STOKESLET: launch_z_t<T, STOKESLET, CM>(zb, zout, a, res, st); break;
        case STRESSLET: launch_z_t<T, STRESSLET, CM>(zb, zout, a, res, st); break;
        default: launch_z_t<T, ROTLET, CM>(zb, zout, a, res, st); break;
    }
}

template <typename T>
hipError_t launch_z(int family, int cm, cplx<T>* zb, cplx<T>* zout, const ZArgs& a, bool res, hipStream_t st)
{
    // the correction density is only used in FP64
    if (cm == CM_FREE) {
        launch_z_f<T, CM_FREE>(family, zb, zout, a, res, st);
    } else {
        if constexpr (sizeof(T) == 8) {
            if (cm == CM_DENSITY) {
                launch_z_f<T, CM_DENSITY>(family, zb, zout, a, res, st);
                return hipGetLastError();
            }
        }
        launch_z_f<T, CM_GRIDS>(family, zb, zout, a, res, st);
    }
    return hipGetLastError();
}

hipError_t launch_even_line(const double* in, double* out, const EvenArgs& a, hipStream_t st)
{
    long long nlines = (long long)a.n1 * a.n2;
    unsigned gx = (unsigned)(nlines < 65535 ? nlines : 65535);
    unsigned gy = (unsigned)((nlines + gx - 1) / gx);
    size_t lds = (size_t)a.f.n * sizeof(cplx<double>);
    hipLaunchKernelGGL(k_even_line, dim3(gx, gy), dim3(256), lds, st, in, out, a);
    return hipGetLastError();
}

hipError_t launch_oct_to_f32(const double* in, float* out, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(k_oct_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_line_fft(const cplx<T>* in, cplx<T>* out, int nl, int per, const FftPlanDev& p, bool inv,
                           hipStream_t st)
{
    dim3 grid((nl + per - 1) / per);
    size_t lds = (size_t)per * (p.n + 1) * sizeof(cplx<T>);
    if (inv)
        hipLaunchKernelGGL((k_line_fft<T, true>), grid, dim3(PASS_NT), lds, st, in, out, nl, per, p);
    else
        hipLaunchKernelGGL((k_line_fft<T, false>), grid, dim3(PASS_NT), lds, st, in, out, nl, per, p);
    return hipGetLastError();
}

template hipError_t launch_fwd_x<double>(const double*, cplx<double>*, const PassArgs&, int, hipStream_t);
template hipError_t launch_fwd_x<float>(const float*, cplx<float>*, const PassArgs&, int, hipStream_t);
template hipError_t launch_fwd_y<double>(const cplx<double>*, cplx<double>*, const PassArgs&, int, hipStream_t);
template hipError_t launch_fwd_y<float>(const cplx<float>*, cplx<float>*, const PassArgs&, int, hipStream_t);
template hipError_t launch_inv_y<double>(const cplx<double>*, cplx<double>*, const PassArgs&, int, hipStream_t);
template hipError_t launch_inv_y<float>(const cplx<float>*, cplx<float>*, const PassArgs&, int, hipStream_t);
template hipError_t launch_inv_x<double>(const cplx<double>*, double*, const PassArgs&, int, hipStream_t);
template hipError_t launch_inv_x<float>(const cplx<float>*, float*, const PassArgs&, int, hipStream_t);
template hipError_t launch_z<double>(int, int, cplx<double>*, cplx<double>*, const ZArgs&, bool, hipStream_t);
template hipError_t launch_z<float>(int, int, cplx<float>*, cplx<float>*, const ZArgs&, bool, hipStream_t);
template hipError_t launch_line_fft<double>(const cplx<double>*, cplx<double>*, int, int, const FftPlanDev&, bool,
                                            hipStream_t);
template hipError_t launch_line_fft<float>(const cplx<float>*, cplx<float>*, int, int, const FftPlanDev&, bool,
                                           hipStream_t);

}  // namespace ehs
