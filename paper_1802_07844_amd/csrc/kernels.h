// Kernel argument blocks and host-side launchers of the device kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace ehs {

// x / y transform passes
struct PassArgs {
    int Mt;              // grid nodes along x1 and x2 (2 Mt along x3)
    int B;               // lines per block
    unsigned mMt, mB, mB2;  // reciprocals for division by Mt, B and B/2 (see magic_of)
    long long cs_in;     // elements between components of the input
    long long cs_out;    // elements between components of the output
    const void* tw2;     // exp(-2 pi i t / 2Mt), t < 2Mt
    FftPlanDev fM;       // FFT of length Mt
    int k1base, nk1;     // y passes: k1 slabs [k1base, k1base + nk1); the Z side
                         // is a buffer of slabs indexed k1 - k1base
    int l3lo;            // inverse passes: only x3 nodes l >= l3lo are produced
    int czero, lzc;      // forward passes: components >= czero vanish at x3 nodes l >= lzc
                         // (neither read nor written there)
};

// fused x3 transform + scaling
struct ZArgs {
    int Mt;
    int Q;                 // phases of the 4Mt padded axis; line length 4Mt / Q
    unsigned mnz, mnq, mn4;  // reciprocals for division by 2Mt, 4Mt / Q and 4Mt
    long long cs;          // elements between input components
    long long cs_out;      // elements between output components
    const void* tw4;       // exp(-2 pi i t / 4Mt), t < 4Mt
    FftPlanDev fq;         // FFT of length 4Mt / Q
    double dk12, dk3;      // wave-number steps: pi / L~ (x1, x2) and pi / (2 L~) (x3)
    double c_exp;          // (1 - eta) / (4 xi^2)
    double c_has;          // 1 / (4 xi^2)
    double cB, cH;         // L~^4 / Npad and L~^2 / Npad
    const double* octB64;  // truncated biharmonic kernel, octant (Mt+1) x (Mt+1) x (2Mt+1)
    const double* octH64;  // truncated harmonic kernel, same layout
    const float* octB32;
    const float* octH32;
    int near0;             // index radius of the k ~ 0 region computed in FP64
    int k1base, nk1;       // k1 slabs of this launch; data indexed k1 - k1base
    int l3lo;              // outputs are written for l >= l3lo only
    const double* ez;      // exp(-c_exp (dk3 t)^2), t <= 2Mt
    int czero, lzc;        // input components >= czero are zero at l >= lzc (not read)
};

// one even real line transform per block (precompute)
struct EvenArgs {
    int n1, n2;          // outer index ranges (one line per pair)
    FftPlanDev f;        // FFT of the period n
    int generate;        // 1: analytic input (K^R sampled on the oversampled grid)
    int kind;            // 0: H^R, 1: B^R
    double R;            // truncation radius (units of L~)
    double dkg1, dkg3;   // oversampled wave-number steps (in-plane, x3)
    long long si1, si2, st;  // input strides (outer 1, outer 2, along the line)
    long long so1, so2, sk;  // output strides
    int nkeep;           // outputs kept (k < nkeep)
    double scale;
};

// LDS of one block of the fused x3 pass: its component lines of 4 Mt / Q
// points and the nq - 1 stage twiddles (host arithmetic, also the planner's)
inline size_t z_lds_bytes(int family, int cm, int Mt, int Q, size_t esz)
{
    int ncin = ncin_for(family, cm);
    int nout = ncout_for(esz == 8 ? 1 : 2, cm);
    int nl = ncin > nout ? ncin : nout;
    int nq = 4 * Mt / Q;
    return ((size_t)nl * (nq + 1) + nq) * 2 * esz;
}
size_t pass_lds(int Mt, int B, size_t esz);
// the x3 pass writes its output over its input slab (lines of up to 1536 points)
inline bool z_resident_ok(int family, int Mt)
{
    (void)family;
    return 2 * Mt <= 3 * 512;
}

template <typename T>
hipError_t launch_fwd_x(const T* in, cplx<T>* out, const PassArgs& a, int ncomp, hipStream_t st);
template <typename T>
hipError_t launch_fwd_y(const cplx<T>* in, cplx<T>* out, const PassArgs& a, int ncomp, hipStream_t st);
template <typename T>
hipError_t launch_inv_y(const cplx<T>* in, cplx<T>* out, const PassArgs& a, int ncomp, hipStream_t st);
template <typename T>
hipError_t launch_inv_x(const cplx<T>* in, T* out, const PassArgs& a, int ncomp, hipStream_t st);
template <typename T>
hipError_t launch_z(int family, int cm, cplx<T>* zb, cplx<T>* zout, const ZArgs& a, bool res, hipStream_t st);
hipError_t launch_even_line(const double* in, double* out, const EvenArgs& a, hipStream_t st);
hipError_t launch_oct_to_f32(const double* in, float* out, long long n, hipStream_t st);
hipError_t launch_exp_table(double* ez, int n, double c, double dk, hipStream_t st);
template <typename T>
hipError_t launch_line_fft(const cplx<T>* in, cplx<T>* out, int nl, int per, const FftPlanDev& p, bool inv,
                           hipStream_t st);

// ---------------------------------------------------------------------------
// binning: bounding box, keys, radix sort, scans, cell ranges
// ---------------------------------------------------------------------------
// bbox / validation reduction over sources and targets; 16 doubles out:
// [0..2] min over all points, [3..5] max, [6] min source x3, [7] min target x3,
// [8] non-finite count, [9] Q (sum of squared strength norms); and zhist,
// ZH_BINS counts of the target heights in bins of width 1 / zbin_inv
constexpr int ZH_BINS = 64;
hipError_t launch_bbox(int family, const double* y, const double* s, long long N, const double* x, long long T,
                       double* partial, int nblocks, double* out16, double zbin_inv, uint32_t* zhist,
                       hipStream_t st);
int bbox_blocks(long long n);

// stable LSD radix sort of (key, value) pairs on `bits` low key bits
size_t radix_sort_scratch_bytes(long long n);
hipError_t radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp, long long n, int bits,
                      void* scratch, hipStream_t st, uint32_t** keys_out, uint32_t** vals_out);
// exclusive scan of n uint32 values (in place allowed); scratch from scan_scratch_bytes
size_t scan_scratch_bytes(long long n);
hipError_t exclusive_scan(const uint32_t* in, uint32_t* out, long long n, void* scratch, hipStream_t st);
hipError_t fill_u32(uint32_t* p, uint32_t v, long long n, hipStream_t st);
// out[i] = (B) in[i], i < n (float <-> double, double -> double)
template <typename A, typename B>
hipError_t launch_convert(const A* in, B* out, long long n, hipStream_t st);
// off[c] (c <= ncell) = first sorted position with key >= c, written to `start`
hipError_t launch_cell_ranges(const uint32_t* skeys, long long n, uint32_t* start, uint32_t* end, long long ncell,
                              hipStream_t st);

// ---------------------------------------------------------------------------
// real-space sum
// ---------------------------------------------------------------------------
struct CellGeom {
    int nc[3];        // cells per axis
    double lo[3];     // origin of the cell grid (x3 origin is the wall)
    double inv[3];    // 1 / cell side
    int nr;           // neighbour reach in cells per axis: side >= r_c / nr
};

struct RealArgs {
    CellGeom cg;
    long long N, T;
    double xi, rc2;
    const uint32_t* src_off;      // ncell + 1 offsets into the sorted sources
    const uint32_t* tgt_off;      // ncell + 1 offsets into the sorted targets
    const uint32_t* chunk_cell;   // work list: cell of each 64-target chunk
    const uint32_t* chunk_first;  // first sorted target of each chunk
    const uint32_t* nchunks;      // device count of chunks
    const uint32_t* tgt_perm;     // sorted target -> original target
    unsigned long long* pairs;    // nullable: in-range (direct, image) pairs evaluated, added up
    int images;                   // 1: half space (image and correction terms); 0: free space
};

hipError_t launch_cell_keys(const double* p, long long n, CellGeom cg, uint32_t* keys, uint32_t* idx, hipStream_t st);
hipError_t launch_chunks(const uint32_t* tstart, const uint32_t* tend, long long ncell, uint32_t* counts,
                         uint32_t* offs, void* scan_scratch, uint32_t* chunk_cell, uint32_t* chunk_first,
                         uint32_t* nchunks, hipStream_t st);
hipError_t launch_gather_points(const double* x, const uint32_t* perm, long long T, double* xs, hipStream_t st);
// gathers sorted source data: positions (SoA, 3 x N) and strengths (nstr x N), FP64
hipError_t launch_gather_sources(int family, const double* y, const double* s, const uint32_t* perm, long long N,
                                 double* ys, double* ss, hipStream_t st);
template <typename T>
hipError_t launch_realspace(int family, const RealArgs& a, const double* ys, const double* ss, const double* xt,
                            double* upart, long long max_chunks, hipStream_t st);

// ---------------------------------------------------------------------------
// spreading and gathering
// ---------------------------------------------------------------------------
// spreading tiles: 8 x 8 x tile[2] nodes, one wavefront each (lane = an x3
// column of tile[2] nodes); tile[2] is 4 or 8 (chosen by the planner)

struct GridArgs {
    int Mt, P;
    double o[3];        // grid origin
    double h;
    double a2;          // 2 xi^2 / eta (Gaussian exponent factor)
    unsigned mP;        // reciprocal for division by P
    double pref;        // (2 xi^2 / (pi eta))^{3/2}
    int tile[3];        // spread tile edge per axis (nodes)
    int nt[3];          // tiles per axis
    int K[3];           // neighbour tiles per axis: ceil((P - 1) / tile)
};

// npts points (sources, then their images when npts = 2N): support base tile keys
hipError_t launch_point_keys(const double* y, long long N, long long npts, GridArgs g, uint32_t* keys, uint32_t* idx,
                             hipStream_t st);
// records of the sorted points (base, 1D weights, strengths) in precision T
size_t record_stride(int family, int P, size_t esz);
template <typename T>
hipError_t launch_records(int family, int cm, const double* y, const double* s, const uint32_t* perm, long long N, GridArgs g,
                          T* rec, hipStream_t st);
template <typename T>
hipError_t launch_spread(int family, int cm, GridArgs g, const T* rec, const uint32_t* toff, T* grids, long long cs,
                         hipStream_t st);
// quadrature at the targets, one wavefront per target (for grids too large for
// the grouped form below)
template <typename T>
hipError_t launch_gather(GridArgs g, int cm, const T* grids, long long cs, const double* x, const uint32_t* tperm,
                         long long T_, const double* upart, double* uout, hipStream_t st);
// the grouped form takes union windows of at most GATHER_GX nodes per axis,
// with 32-bit byte offsets within one window
constexpr int GATHER_GX = 48;
inline bool gather_group_fits(int Pg, long long Mt, size_t esz)
{
    return Pg <= GATHER_GX && (long long)GATHER_GX * Mt * Mt * (long long)esz < (1LL << 32);
}
// Morton keys of the targets' support bases >> shift (bins of 2^shift nodes)
hipError_t launch_target_zkeys(const double* xs, long long TT, GridArgs gg, int shift, uint32_t* keys, uint32_t* idx,
                               hipStream_t st);
// quadrature at dense targets, several targets per wavefront sharing one walk
// over their supports (gperm: targets sorted by the Morton keys above, as
// indices into the cell-sorted xs)
template <typename T>
hipError_t launch_gather_group(GridArgs g, int cm, const T* grids, long long cs, const double* xs,
                               const uint32_t* gperm, const uint32_t* tperm, long long T_, const double* upart,
                               double* uout, hipStream_t st);
// quadrature at the targets, node-owner form (see grid.hip):
//   keys: quadrature tile of each target's support base (xs: cell-sorted SoA targets)
hipError_t launch_target_keys(const double* xs, long long T_, GridArgs gg, uint32_t* keys, uint32_t* idx,
                              hipStream_t st);
//   records of the tile-sorted targets: support base, cell-sorted index, 1D factors
size_t target_record_stride(int Pg, size_t esz);
template <typename T>
hipError_t launch_target_records(const double* xs, const uint32_t* perm, long long T_, GridArgs gg, T* rec,
                                 hipStream_t st);
//   slots per target of the partial sums (one per tile of its support box)
int gather_slots(const GridArgs& gg);
//   one wavefront per tile: partial sums of every target whose support reaches it
template <typename T>
hipError_t launch_gather_tiles(GridArgs gg, const T* grids, long long cs, const T* rec, const uint32_t* gtoff,
                               int tz0, T* part, hipStream_t st);
//   per target: the partial sums in a fixed order, and the FP64 combination
template <typename T>
hipError_t launch_gather_final(GridArgs gg, const T* rec, const T* part, long long T_, const double* xs,
                               const uint32_t* tperm, const double* upart, double* uout, hipStream_t st);

}  // namespace ehs
