// Host side of the C ABI: validation, parameter selection (plan), workspace,
// the truncated-kernel cache and the stage-by-stage orchestration of one
// half-space Ewald evaluation on a HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "../../include/ehs.h"
#include "ctx.h"
#include "kernels.h"
#include "plan.h"

using namespace ehs;

namespace {

constexpr size_t ALIGN = 256;
inline size_t al(size_t n) { return (n + ALIGN - 1) / ALIGN * ALIGN; }

#define HIPCHK(x)                              \
    do {                                       \
        hipError_t e_ = (x);                   \
        if (e_ != hipSuccess) return EHS_EHIP; \
    } while (0)

// device memory for one table: carved from the table region of a fixed
// region, else allocated
int table_alloc(Tables* t, size_t bytes, void** out)
{
    *out = nullptr;
    if (t->arena) {
        size_t off = al(t->used);
        if (off + bytes > t->cap) return EHS_ENOMEM;
        *out = t->arena + off;
        t->used = off + bytes;
        return EHS_OK;
    }
    if (hipMalloc(out, bytes) != hipSuccess) {
        *out = nullptr;
        hipGetLastError();
        return EHS_ENOMEM;
    }
    return EHS_OK;
}

int tw_table(ehs_ctx* c, int n, int esz, void** out)
{
    std::lock_guard<std::mutex> lk(c->tables->mu);
    auto key = std::make_pair(n, esz);
    auto& tables = c->tables->m;
    auto it = tables.find(key);
    if (it != tables.end()) {
        *out = it->second;
        return EHS_OK;
    }
    std::vector<double> h(2 * (size_t)n);
    const double tp = 6.283185307179586476925286766559;
    for (int t = 0; t < n; ++t) {
        // exp(-2 pi i t / n), reduced to the first half period for accuracy
        double a = tp * (double)t / (double)n;
        h[2 * t] = std::cos(a);
        h[2 * t + 1] = -std::sin(a);
    }
    void* d = nullptr;
    size_t bytes = (size_t)n * 2 * esz;
    if (int rc = table_alloc(c->tables, bytes, &d)) return rc;
    if (esz == 8) {
        if (hipMemcpy(d, h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) return EHS_EHIP;
    } else {
        std::vector<float> f(h.begin(), h.end());
        if (hipMemcpy(d, f.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) return EHS_EHIP;
    }
    tables[key] = d;
    *out = d;
    return EHS_OK;
}

// per-stage twiddles of the Stockham stages: for stage s with radix R and
// span Ns, entries w^(k q), w = exp(-2 pi i / (Ns R)), k < Ns, 1 <= q < R
int stage_table(ehs_ctx* c, int n, int esz, const std::vector<int>& r, FftPlanDev* p)
{
    std::lock_guard<std::mutex> lk(c->tables->mu);
    auto key = std::make_pair(-n, esz);  // negative key: stage tables
    auto& tables = c->tables->m;
    auto it = tables.find(key);
    std::vector<int> offs;
    size_t total = 0;
    int ns = 1;
    for (int R : r) {
        offs.push_back((int)total);
        total += (size_t)ns * (R - 1);
        ns *= R;
    }
    for (size_t i = 0; i < r.size(); ++i) p->toff[i] = offs[i];
    if (it != tables.end()) {
        p->tws = it->second;
        return EHS_OK;
    }
    std::vector<double> h(2 * std::max<size_t>(total, 1));
    const double tp = 6.283185307179586476925286766559;
    ns = 1;
    for (size_t s = 0; s < r.size(); ++s) {
        int R = r[s];
        for (int k = 0; k < ns; ++k)
            for (int q = 1; q < R; ++q) {
                // exp(-2 pi i k q / (ns R)) = table entry (k q n / (ns R)) mod n
                long long t = ((long long)k * q * (n / (ns * R))) % n;
                double a = tp * (double)t / (double)n;
                size_t e = offs[s] + (size_t)(q - 1) * ns + k;
                h[2 * e] = std::cos(a);
                h[2 * e + 1] = -std::sin(a);
            }
        ns *= R;
    }
    void* d = nullptr;
    size_t bytes = (h.size() / 2) * 2 * esz;
    if (int rc = table_alloc(c->tables, bytes, &d)) return rc;
    if (esz == 8) {
        if (hipMemcpy(d, h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) return EHS_EHIP;
    } else {
        std::vector<float> f(h.begin(), h.end());
        if (hipMemcpy(d, f.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) return EHS_EHIP;
    }
    tables[key] = d;
    p->tws = d;
    return EHS_OK;
}

int fft_plan(ehs_ctx* c, int n, int esz, FftPlanDev* p)
{
    std::vector<int> r;
    if (!factor_radices(n, r) || (int)r.size() > FFT_MAX_STAGES) return EHS_ERANGE;
    std::memset(p, 0, sizeof(*p));
    p->n = n;
    p->nst = (int)r.size();
    int ns = 1;
    for (size_t i = 0; i < r.size(); ++i) {
        p->rad[i] = r[i];
        p->ns[i] = ns;
        p->mns[i] = magic_of((unsigned)ns);
        p->nb[i] = n / r[i];
        p->mnb[i] = magic_of((unsigned)(n / r[i]));
        p->tstr[i] = n / (ns * r[i]);
        ns *= r[i];
    }
    void* t = nullptr;
    int rc = tw_table(c, n, esz, &t);
    if (rc) return rc;
    p->tw = t;
    return stage_table(c, n, esz, r, p);
}

// ---------------------------------------------------------------------------
// truncated-kernel precompute (Sec. 5.2, the three precompute steps), in
// units of L~ = 1, h = 1 / M~:
//   sample K^R(|k|) on the oversampled grid (nf x nf x nf3, R = sqrt 6),
//   inverse transform, keep the window |j1|, |j2| <= M~, |j3| <= 2 M~,
//   forward transform on the 2M~ x 2M~ x 4M~ grid, keep the octant.
// Every transform is a real even one done axis by axis on octant data.
// ---------------------------------------------------------------------------
int precompute_kind(ehs_ctx* c, int Mt, int nf, int nf3, int kind, double* scratch, double* oct, hipStream_t st)
{
    const long long h1 = nf / 2 + 1, m1 = Mt + 1, z1 = 2 * Mt + 1;
    double* out1 = scratch;                // h1 x h1 x z1
    double* out2 = scratch + h1 * h1 * z1; // h1 x m1 x z1
    double* out3 = out1;                   // m1 x m1 x z1
    double* out4 = out2;
    double* out5 = out1;
    FftPlanDev pf3, pf, p4, p2;
    int rc;
    if ((rc = fft_plan(c, nf3, 8, &pf3)) || (rc = fft_plan(c, nf, 8, &pf)) || (rc = fft_plan(c, 4 * Mt, 8, &p4)) ||
        (rc = fft_plan(c, 2 * Mt, 8, &p2)))
        return rc;
    const double tp = 6.283185307179586476925286766559;
    EvenArgs a;
    std::memset(&a, 0, sizeof(a));
    a.R = std::sqrt(6.0);
    a.kind = kind;
    a.dkg1 = tp * Mt / nf;
    a.dkg3 = tp * Mt / nf3;
    // P1: along n3, analytic input, lines (n1, n2)
    a.n1 = (int)h1; a.n2 = (int)h1; a.f = pf3; a.generate = 1;
    a.so1 = h1 * z1; a.so2 = z1; a.sk = 1; a.nkeep = (int)z1; a.scale = 1.0;
    HIPCHK(launch_even_line(nullptr, out1, a, st));
    // P2: along n2, lines (n1, j3)
    a.generate = 0; a.f = pf; a.n1 = (int)h1; a.n2 = (int)z1;
    a.si1 = h1 * z1; a.si2 = 1; a.st = z1;
    a.so1 = m1 * z1; a.so2 = 1; a.sk = z1; a.nkeep = (int)m1;
    HIPCHK(launch_even_line(out1, out2, a, st));
    // P3: along n1, lines (j2, j3); normalisation of the inverse transform
    a.n1 = (int)m1; a.n2 = (int)z1;
    a.si1 = z1; a.si2 = 1; a.st = m1 * z1;
    a.so1 = z1; a.so2 = 1; a.sk = m1 * z1; a.nkeep = (int)m1;
    a.scale = 1.0 / ((double)nf * (double)nf * (double)nf3);
    HIPCHK(launch_even_line(out2, out3, a, st));
    // Q1: along j3 (period 4 M~), lines (j1, j2)
    a.scale = 1.0; a.f = p4; a.n1 = (int)m1; a.n2 = (int)m1;
    a.si1 = m1 * z1; a.si2 = z1; a.st = 1;
    a.so1 = m1 * z1; a.so2 = z1; a.sk = 1; a.nkeep = (int)z1;
    HIPCHK(launch_even_line(out3, out4, a, st));
    // Q2: along j2 (period 2 M~), lines (j1, k3)
    a.f = p2; a.n1 = (int)m1; a.n2 = (int)z1;
    a.si1 = m1 * z1; a.si2 = 1; a.st = z1;
    a.so1 = m1 * z1; a.so2 = 1; a.sk = z1; a.nkeep = (int)m1;
    HIPCHK(launch_even_line(out4, out5, a, st));
    // Q3: along j1, lines (k2, k3) -> octant [k1][k2][k3]
    a.n1 = (int)m1; a.n2 = (int)z1;
    a.si1 = z1; a.si2 = 1; a.st = m1 * z1;
    a.so1 = z1; a.so2 = 1; a.sk = m1 * z1; a.nkeep = (int)m1;
    HIPCHK(launch_even_line(out5, oct, a, st));
    return EHS_OK;
}

}  // namespace

int ehs::precompute_octant(ehs_ctx* c, const Plan& p, int kind, double* oct, hipStream_t st)
{
    return precompute_kind(c, p.Mt, p.nf, p.nf3, kind, static_cast<double*>(c->ws), oct, st);
}

namespace {

size_t cache_bytes(const ehs_ctx* c)
{
    size_t b = 0;
    for (auto& kv : c->cache) {
        const size_t n = (size_t)octant_elems(kv.first);
        const Octants& o = kv.second;
        b += (o.H64 ? 8 * n : 0) + (o.B64 ? 8 * n : 0) + (o.H32 ? 4 * n : 0) + (o.B32 ? 4 * n : 0);
    }
    return b;
}

void free_octants(Octants& o)
{
    if (o.B64) hipFree(o.B64);
    if (o.H64) hipFree(o.H64);
    if (o.B32) hipFree(o.B32);
    if (o.H32) hipFree(o.H32);
    o = Octants();
}

// Drop every cached grid size except `keep` (hipFree waits for the device).
void evict_octants_except(ehs_ctx* c, int keep)
{
    for (auto it = c->cache.begin(); it != c->cache.end();) {
        if (it->first == keep) {
            ++it;
            continue;
        }
        free_octants(it->second);
        it = c->cache.erase(it);
    }
}

// Device memory for one more octant array: under a memory cap the workspace
// and every cached array count against it, and other grid sizes are evicted
// to make room.
int octant_alloc(ehs_ctx* c, int Mt, size_t bytes, void** out)
{
    *out = nullptr;
    if (c->mem_cap > 0) {
        if ((double)(c->ws_bytes + cache_bytes(c) + bytes) > c->mem_cap) evict_octants_except(c, Mt);
        if ((double)(c->ws_bytes + cache_bytes(c) + bytes) > c->mem_cap) return EHS_ENOMEM;
    }
    if (hipMalloc(out, bytes) != hipSuccess) {
        *out = nullptr;
        hipGetLastError();
        return EHS_ENOMEM;
    }
    return EHS_OK;
}

// the test hook of EHS_OPT_FAIL_PRECOMPUTE: fail before launching anything
int take_injected_failure(int* counter)
{
    if (*counter > 0) {
        --*counter;
        return EHS_EHIP;
    }
    return EHS_OK;
}

// standalone contexts: octants by M~ in the context's own cache; an array is
// entered into the cache only once its production has been enqueued without
// error, so a failed precompute leaves nothing behind; the stream is
// synchronised after a precompute so that later calls on other streams see it
int ensure_octants(ehs_ctx* c, const Plan& p, hipStream_t st, bool* ran, Octants** out)
{
    const bool needB = p.family != EHS_ROTLET;
    const bool needH = !(p.free && p.family != EHS_ROTLET);  // free space: the kernel's octant only
    const bool need32 = p.prec == 2;
    const long long n = octant_elems(p.Mt);
    *ran = false;
    Octants cur;
    auto it = c->cache.find(p.Mt);
    if (it != c->cache.end()) cur = it->second;
    cur.nf = p.nf;
    cur.nf3 = p.nf3;
    double* scratch = static_cast<double*>(c->ws);
    auto publish = [&]() { c->cache[p.Mt] = cur; };
    for (int kind = 0; kind < 2; ++kind) {
        if (kind == 1 && !needB) continue;
        if (kind == 0 && !needH) continue;
        double*& d64 = kind == 0 ? cur.H64 : cur.B64;
        float*& d32 = kind == 0 ? cur.H32 : cur.B32;
        if (!d64) {
            void* tmp = nullptr;
            int rc = octant_alloc(c, p.Mt, n * sizeof(double), &tmp);
            if (rc) return rc;
            if (!rc) rc = take_injected_failure(&c->fail_precompute);
            if (!rc) rc = precompute_kind(c, p.Mt, p.nf, p.nf3, kind, scratch, static_cast<double*>(tmp), st);
            if (rc) {
                hipFree(tmp);
                return rc;
            }
            d64 = static_cast<double*>(tmp);
            publish();
            *ran = true;
        }
        if (need32 && !d32) {
            void* tmp = nullptr;
            int rc = octant_alloc(c, p.Mt, n * sizeof(float), &tmp);
            if (rc) return rc;
            if (launch_oct_to_f32(d64, static_cast<float*>(tmp), n, st) != hipSuccess) {
                hipFree(tmp);
                return EHS_EHIP;
            }
            d32 = static_cast<float*>(tmp);
            publish();
            *ran = true;
        }
    }
    if (*ran) HIPCHK(hipStreamSynchronize(st));
    *out = &c->cache[p.Mt];
    return EHS_OK;
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
struct Layout {
    size_t X, Y, ZS, Zo, rec, keys, sortsc, toff, soff, tgoff, chunks, ys, ss, xs, upart, bb, ez, gkeys, gtoff, grec,
        gpart, cnt, total;
};

// Host-side audit: the largest extent every pass writes or reads must fit the
// region it is given.  Returns 0 or EHS_ERANGE (never launches an
// out-of-bounds kernel).
int check_extents(const Plan& p, const Layout& L, size_t esz)
{
    const size_t Mt = p.Mt;
    const size_t c = 2 * esz;
    const size_t real = Mt * Mt * 2 * Mt * esz;
    const size_t a = (Mt + 1) * 2 * Mt * Mt * c;
    const size_t zs = (size_t)p.zg * 2 * Mt * 2 * Mt * c;  // one component of the slab buffer
    const size_t nin = (size_t)p.ncin;
    const size_t nout = (size_t)ncout_for(p.prec, plan_cm(p));
    const size_t xreg = L.Y - L.X, yreg = L.ZS - L.Y, zsreg = L.Zo - L.ZS, zoreg = L.rec - L.Zo;
    auto fits = [](size_t need, size_t have) { return need <= have; };
    // in place (resident), the fused x3 pass keeps at most 16 outputs per lane
    bool ok = p.zg >= 1 && p.zg <= p.Mt + 1 && p.l3lo >= 0 && p.l3lo < 2 * p.Mt && p.lzc >= 0 &&
              p.lzc <= 2 * p.Mt &&
              (!p.resident || 2 * p.Mt - p.l3lo <= 1024)
              && fits(nin * real, xreg)                 // spread -> X
              && fits(nin * a, yreg)                    // forward x1 -> Y
              && fits(nin * zs, zsreg)                  // forward x2 -> slab buffer
              && fits(nout * zs, p.resident ? zsreg : zoreg)  // fused x3 outputs
              && fits(nout * a, yreg)                  // inverse x2 -> Y (in place of A)
              && fits(nout * real, xreg)               // inverse x1 -> X (read by the gather)
              && fits((size_t)2 * p.N * record_stride(p.family, p.g.P, esz) * esz, L.keys - L.rec)
              && fits((size_t)(4 * p.N + 4 * p.T + 8 * p.N) * 4, L.sortsc - L.keys)
              && fits((size_t)(p.ntiles + 1) * 4, L.soff - L.toff)
              && fits((size_t)(p.ncell + 1) * 4, L.tgoff - L.soff)
              && fits((size_t)(p.ncell + 1) * 4, L.chunks - L.tgoff)
              && fits((size_t)(2 * p.ncell + 2 * p.max_chunks + 1) * 4, L.ys - L.chunks)
              && fits((size_t)3 * p.N * 8, L.ss - L.ys) && fits((size_t)6 * p.N * 8, L.xs - L.ss)
              && fits((size_t)3 * p.T * 8, L.upart - L.xs) && fits((size_t)3 * p.T * 8, L.bb - L.upart)
              && fits((size_t)(2 * Mt + 1) * 8, L.gkeys - L.ez)
              && (!p.ggroup || fits((size_t)4 * p.T * 4, L.gtoff - L.gkeys))
              && (!p.gtiles || (fits((size_t)4 * p.T * 4, L.gtoff - L.gkeys)
                                && fits((size_t)(p.ntiles_g + 1) * 4, L.grec - L.gtoff)
                                && fits((size_t)p.T * target_record_stride(p.gg.P, esz) * esz, L.gpart - L.grec)
                                && fits((size_t)p.T * gather_slots(p.gg) * 6 * esz, L.total - L.gpart)))
              && p.gg.tile[0] == 8 && p.gg.tile[1] == 8 && p.gg.tile[2] == 8 && p.gg.K[0] == p.gg.K[1] &&
              p.gg.K[0] == p.gg.K[2] && p.gg.K[0] * 8 >= p.gg.P - 1;
    // precompute scratch in X
    size_t h1 = p.nf / 2 + 1;
    ok = ok && fits((h1 * h1 * (2 * Mt + 1) + h1 * (Mt + 1) * (2 * Mt + 1)) * 8, xreg);
    // the fused x3 pass holds lines of length 4Mt/Q for max(ncin, outputs) components,
    // each transformed by one wavefront
    int nq = 4 * p.Mt / p.Qz;
    ok = ok && (4 * p.Mt) % p.Qz == 0 && z_lds_bytes(p.family, plan_cm(p), p.Mt, p.Qz, esz) <= 160 * 1024 &&
         nq <= lds_fft_cap(nq, 64);
    // x / y passes: B lines of Mt in LDS and in the 16-element register budget
    ok = ok && p.Bx * p.Mt <= lds_fft_cap(p.Mt, 256) && p.By * p.Mt <= lds_fft_cap(p.Mt, 256) &&
         p.By * p.Mt <= 16 * 256 && (p.Bx % 2) == 0 && p.By >= 1 &&
         pass_lds(p.Mt, p.By, esz) <= 160 * 1024 && pass_lds(p.Mt, p.Bx, esz) <= 160 * 1024;
    // magic-number division is exact for numerator * divisor < 2^32
    ok = ok && (long long)(p.Mt + 1) * std::max(p.Bx, 2 * p.By) * std::max(p.Mt, 2 * p.By) < (1LL << 31) &&
         (long long)std::max(p.ncin, ncout_for(p.prec, plan_cm(p))) * 2 * p.Mt * 2 * p.Mt < (1LL << 31);
    // gather weights table (3P <= 96) and spread support within the grid
    // supports: the kernels read them from the grid arguments, which must agree
    // with the plan (spreading g.P = Ps >= P, quadrature gg.P = Pg >= P)
    ok = ok && p.g.P == p.Ps && p.gg.P == p.Pg && p.Ps >= p.P && p.Pg >= p.P && 3 * p.Pg <= 96 &&
         p.Ps <= p.Mt && p.Pg <= p.Mt && p.M + std::max(p.Ps, p.Pg) <= p.Mt;
    return ok ? EHS_OK : EHS_ERANGE;
}

Layout layout(const Plan& p, size_t esz)
{
    Layout L;
    const long long Mt = p.Mt;
    const int ncin = p.ncin;
    const int nl = std::max(ncin, ncout_for(p.prec, plan_cm(p)));
    size_t czs = (size_t)p.zg * 2 * Mt * 2 * Mt * 2 * esz;  // one slab-buffer component (complex)
    size_t cy = (size_t)(Mt + 1) * 2 * Mt * Mt * 2 * esz;   // one A / D component
    size_t x_bytes = (size_t)nl * (size_t)(Mt * Mt * 2 * Mt) * esz;
    // the precompute scratch also lives in X
    long long h1 = p.nf / 2 + 1;
    size_t pre = (size_t)(h1 * h1 * (2 * Mt + 1) + h1 * (Mt + 1) * (2 * Mt + 1)) * sizeof(double);
    x_bytes = std::max(x_bytes, pre);
    size_t off = 0;
    L.X = off; off += al(x_bytes);
    L.Y = off; off += al((size_t)nl * cy);  // A (ncin components), then D (outputs) in place
    L.ZS = off; off += al((size_t)nl * czs);
    L.Zo = off; off += p.resident ? 0 : al((size_t)ncout_for(p.prec, plan_cm(p)) * czs);
    long long N = p.N, T = p.T;
    // records carry 3 g.P weights: g.P is the spreading support the kernels use
    L.rec = off; off += al((size_t)2 * N * record_stride(p.family, p.g.P, esz) * esz);
    // keys / values: sources (4 N), targets (4 T), points (4 * 2N)
    L.keys = off; off += al((size_t)(4 * N + 4 * T + 8 * N) * sizeof(uint32_t));
    L.sortsc = off; off += al(radix_sort_scratch_bytes(std::max(2 * N, T)) + scan_scratch_bytes(p.ncell + 1) + 1024);
    L.toff = off; off += al((size_t)(p.ntiles + 1) * sizeof(uint32_t));
    L.soff = off; off += al((size_t)(p.ncell + 1) * sizeof(uint32_t));
    L.tgoff = off; off += al((size_t)(p.ncell + 1) * sizeof(uint32_t));
    // chunk work list: counts, offsets (ncell each), cell + first (max_chunks each), count
    L.chunks = off; off += al((size_t)(2 * p.ncell + 2 * p.max_chunks + 4) * sizeof(uint32_t));
    L.ys = off; off += al((size_t)3 * N * sizeof(double));
    L.ss = off; off += al((size_t)6 * N * sizeof(double));
    L.xs = off; off += al((size_t)3 * T * sizeof(double));
    L.upart = off; off += al((size_t)3 * T * sizeof(double));
    L.bb = off; off += al((size_t)(1024 * 10 + 16) * sizeof(double));
    L.ez = off; off += al((size_t)(2 * Mt + 1) * sizeof(double));
    // quadrature: target keys / values (4 T), tile offsets, target records and
    // the partial sums (6 per target and tile of its support box)
    const size_t gt = p.gtiles ? 1 : 0;  // regions of the node-owner quadrature only
    L.gkeys = off; off += al((p.gtiles || p.ggroup ? 4 : 0) * T * sizeof(uint32_t));
    L.gtoff = off; off += al(gt * (p.ntiles_g + 1) * sizeof(uint32_t));
    L.grec = off; off += al(gt * T * target_record_stride(p.gg.P, esz) * esz);
    L.gpart = off; off += al(gt * T * gather_slots(p.gg) * 6 * esz);
    L.cnt = off; off += al(2 * sizeof(unsigned long long));  // real-space pair counters (timing)
    L.total = off;
    return L;
}

// Workspace of at least `bytes`; under a memory cap the cached octants count
// too, and grid sizes other than keep_Mt are evicted to make room.
int ensure_ws(ehs_ctx* c, size_t bytes, hipStream_t st, int keep_Mt)
{
    if (c->mem_cap > 0) {
        if ((double)bytes > c->mem_cap) return EHS_ENOMEM;
        if ((double)(std::max(bytes, c->ws_bytes) + cache_bytes(c)) > c->mem_cap) evict_octants_except(c, keep_Mt);
        if ((double)(std::max(bytes, c->ws_bytes) + cache_bytes(c)) > c->mem_cap) return EHS_ENOMEM;
    }
    if (bytes <= c->ws_bytes) return EHS_OK;
    HIPCHK(hipStreamSynchronize(st));
    if (c->ws) hipFree(c->ws);
    c->ws = nullptr;
    c->ws_bytes = 0;
    if (hipMalloc(&c->ws, bytes) != hipSuccess) {
        c->ws = nullptr;
        hipGetLastError();
        return EHS_ENOMEM;
    }
    c->ws_bytes = bytes;
    return EHS_OK;
}

// ---------------------------------------------------------------------------
// one evaluation
// ---------------------------------------------------------------------------
template <typename T>
int run(ehs_ctx* c, Plan& p, const Octants& oct, const double* y, const double* s, const double* x, double* u,
        hipStream_t st, bool alias)
{
    const size_t esz = sizeof(T);
    Layout Lo = layout(p, esz);
    int rc = check_extents(p, Lo, esz);
    if (rc) return rc;
    if (!c->ws || c->ws_bytes < Lo.total) return EHS_ENOMEM;
    char* base = static_cast<char*>(c->ws);
    auto rec_ev = [&](int i) {
        if (c->opt_timing && c->ev_ok) hipEventRecord(c->ev[i], st);
    };
    rec_ev(EHS_ST_BIN);

    const long long N = p.N, TT = p.T;
    uint32_t* kbase = reinterpret_cast<uint32_t*>(base + Lo.keys);
    uint32_t *ks = kbase, *vs = ks + N, *ks2 = vs + N, *vs2 = ks2 + N;
    uint32_t *kt = vs2 + N, *vt = kt + TT, *kt2 = vt + TT, *vt2 = kt2 + TT;
    uint32_t *kp = vt2 + TT, *vp = kp + 2 * N, *kp2 = vp + 2 * N, *vp2 = kp2 + 2 * N;
    void* sortsc = base + Lo.sortsc;
    uint32_t* toff = reinterpret_cast<uint32_t*>(base + Lo.toff);
    uint32_t* soff = reinterpret_cast<uint32_t*>(base + Lo.soff);
    uint32_t* tgoff = reinterpret_cast<uint32_t*>(base + Lo.tgoff);
    uint32_t* ch = reinterpret_cast<uint32_t*>(base + Lo.chunks);
    uint32_t *ch_counts = ch, *ch_offs = ch + p.ncell, *ch_cell = ch_offs + p.ncell,
             *ch_first = ch_cell + p.max_chunks, *ch_n = ch_first + p.max_chunks;
    double* ys = reinterpret_cast<double*>(base + Lo.ys);
    double* ss = reinterpret_cast<double*>(base + Lo.ss);
    double* xs = reinterpret_cast<double*>(base + Lo.xs);
    double* upart = reinterpret_cast<double*>(base + Lo.upart);

    // -- real-space binning: sort sources (and targets) by cell
    int cbits = bits_for(p.ncell);
    uint32_t *sk, *sperm;
    HIPCHK(launch_cell_keys(y, N, p.cg, ks, vs, st));
    HIPCHK(radix_sort(ks, vs, ks2, vs2, N, cbits, sortsc, st, &sk, &sperm));
    HIPCHK(launch_cell_ranges(sk, N, soff, nullptr, p.ncell, st));
    HIPCHK(launch_gather_sources(p.family, y, s, sperm, N, ys, ss, st));
    uint32_t *tk, *tperm;
    if (alias) {
        tk = sk;
        tperm = sperm;
        HIPCHK(hipMemcpyAsync(tgoff, soff, (p.ncell + 1) * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
    } else {
        HIPCHK(launch_cell_keys(x, TT, p.cg, kt, vt, st));
        HIPCHK(radix_sort(kt, vt, kt2, vt2, TT, cbits, sortsc, st, &tk, &tperm));
        HIPCHK(launch_cell_ranges(tk, TT, tgoff, nullptr, p.ncell, st));
    }
    HIPCHK(launch_gather_points(x, tperm, TT, xs, st));
    HIPCHK(launch_chunks(tgoff, nullptr, p.ncell, ch_counts, ch_offs, sortsc, ch_cell, ch_first, ch_n, st));
    rec_ev(EHS_ST_REAL);

    // -- real-space sum
    RealArgs ra;
    ra.cg = p.cg;
    ra.N = N;
    ra.T = TT;
    ra.xi = p.xi;
    ra.rc2 = p.rc * p.rc;
    ra.src_off = soff;
    ra.tgt_off = tgoff;
    ra.chunk_cell = ch_cell;
    ra.chunk_first = ch_first;
    ra.nchunks = ch_n;
    ra.tgt_perm = tperm;
    ra.images = p.free ? 0 : 1;
    ra.pairs = nullptr;
    c->pairs_dev = nullptr;
    if (c->opt_timing && c->ev_ok) {
        ra.pairs = reinterpret_cast<unsigned long long*>(base + Lo.cnt);
        c->pairs_dev = ra.pairs;
        HIPCHK(fill_u32(reinterpret_cast<uint32_t*>(ra.pairs), 0u, 4, st));
    }
    // The real-space sum (bound by the vector ALU) runs on the side stream
    // beside the spreading and the transforms (bound by memory and latency);
    // they share only read-only inputs, and the quadrature, which adds the
    // real-space part, waits for it.  Every return after the fork makes the
    // caller's stream wait for the side stream (the workspace is reused).
    const bool ovl = c->overlap && c->side;
    c->last_overlap = ovl && c->opt_timing && c->ev_ok;
    struct Join {
        ehs_ctx* c;
        hipStream_t st;
        bool armed;
        void now()
        {
            if (!armed) return;
            armed = false;
            hipEventRecord(c->join, c->side);
            hipStreamWaitEvent(st, c->join, 0);
        }
        ~Join() { now(); }
    } join{c, st, false};
    hipStream_t rst = st;
    if (ovl) {
        HIPCHK(hipEventRecord(c->fork, st));
        HIPCHK(hipStreamWaitEvent(c->side, c->fork, 0));
        join.armed = true;
        rst = c->side;
    }
    if (c->parts != 2 && !c->tap_quad) {
        HIPCHK(launch_realspace<T>(p.family, ra, ys, ss, xs, upart, p.max_chunks, rst));
    } else if (TT > 0) {  // Fourier part only: the quadrature adds it to zero
        HIPCHK(fill_u32(reinterpret_cast<uint32_t*>(upart), 0u, 6 * TT, rst));
    }
    if (c->last_overlap) HIPCHK(hipEventRecord(c->ev_rs_end, rst));
    rec_ev(EHS_ST_SPREAD);

    // -- spreading
    T* X = reinterpret_cast<T*>(base + Lo.X);
    cplx<T>* Yc = reinterpret_cast<cplx<T>*>(base + Lo.Y);
    T* rec = reinterpret_cast<T*>(base + Lo.rec);
    uint32_t *pk, *pperm;
    const int cm = plan_cm(p);
    const long long npts = p.free ? N : 2 * N;  // sources and (half space) their images
    HIPCHK(launch_point_keys(y, N, npts, p.g, kp, vp, st));
    HIPCHK(radix_sort(kp, vp, kp2, vp2, npts, bits_for(p.ntiles), sortsc, st, &pk, &pperm));
    HIPCHK(launch_cell_ranges(pk, npts, toff, nullptr, p.ntiles, st));
    HIPCHK(launch_records<T>(p.family, cm, y, s, pperm, N, p.g, rec, st));
    const long long Mt = p.Mt;
    const long long csR = Mt * Mt * 2 * Mt;          // real grid component
    const long long csA = (Mt + 1) * 2 * Mt * Mt;    // A / D component (complex)
    HIPCHK(launch_spread<T>(p.family, cm, p.g, rec, toff, X, csR, st));
    c->tap_grids[0] = p.ncin;
    if (c->tap_spread) {
        if (c->tap_spread_cap < p.ncin * csR) return EHS_EINVAL;
        HIPCHK(launch_convert(X, c->tap_spread, p.ncin * csR, st));
    }
    rec_ev(EHS_ST_FWDX);

    // -- forward transforms
    PassArgs pa;
    std::memset(&pa, 0, sizeof(pa));
    pa.Mt = p.Mt;
    pa.k1base = 0;
    pa.nk1 = p.Mt + 1;
    void* tw2 = nullptr;
    if ((rc = tw_table(c, 2 * p.Mt, (int)esz, &tw2))) return rc;
    pa.tw2 = tw2;
    if ((rc = fft_plan(c, p.Mt, (int)esz, &pa.fM))) return rc;
    pa.mMt = magic_of((unsigned)p.Mt);
    auto set_b = [&](int B) {
        pa.B = B;
        pa.mB = magic_of((unsigned)B);
        pa.mB2 = magic_of((unsigned)(B / 2));
    };
    set_b(p.Bx);
    pa.cs_in = csR;
    pa.cs_out = csA;
    // components from ncA on (the correction grids, spread at the images)
    // vanish at x3 nodes >= lzc: the forward passes skip them there
    // (free space: every component vanishes there)
    pa.czero = p.free ? 0 : p.family == STRESSLET ? 6 : 3;  // the kernel-grid components come first
    pa.lzc = p.lzc;
    HIPCHK(launch_fwd_x<T>(X, Yc, pa, p.ncin, st));
    rec_ev(EHS_ST_FWDY);

    // -- y / x3 pipeline over groups of zg k1 slabs: forward y into the slab
    //    buffer, fused x3 transform + scaling + inverse x3, inverse y back into
    //    Y (D[k1] replaces A[k1], which the forward y pass of the group has read)
    ZArgs za;
    std::memset(&za, 0, sizeof(za));
    za.Mt = p.Mt;
    za.Q = p.Qz;
    za.mnz = magic_of((unsigned)(2 * p.Mt));
    za.mnq = magic_of((unsigned)(4 * p.Mt / p.Qz));
    za.mn4 = magic_of((unsigned)(4 * p.Mt));
    const long long csS = (long long)p.zg * 2 * Mt * 2 * Mt;  // slab-buffer component
    za.cs = csS;
    za.cs_out = csS;
    void* tw4 = nullptr;
    if ((rc = tw_table(c, 4 * p.Mt, (int)esz, &tw4))) return rc;
    za.tw4 = tw4;
    if ((rc = fft_plan(c, 4 * p.Mt / p.Qz, (int)esz, &za.fq))) return rc;
    const double pi = 3.14159265358979323846;
    za.dk12 = pi / p.Lt;
    za.dk3 = pi / (2.0 * p.Lt);
    za.c_exp = (1.0 - p.eta) / (4.0 * p.xi * p.xi);
    za.c_has = 1.0 / (4.0 * p.xi * p.xi);
    double npad = 16.0 * (double)Mt * (double)Mt * (double)Mt;
    za.cB = std::pow(p.Lt, 4) / npad;
    za.cH = p.Lt * p.Lt / npad;
    za.octB64 = oct.B64;
    za.octH64 = oct.H64;
    za.octB32 = oct.B32;
    za.octH32 = oct.H32;
    za.near0 = 2;
    double* ez = reinterpret_cast<double*>(base + Lo.ez);
    HIPCHK(launch_exp_table(ez, 2 * p.Mt + 1, za.c_exp, za.dk3, st));
    za.ez = ez;
    cplx<T>* ZS = reinterpret_cast<cplx<T>*>(base + Lo.ZS);
    cplx<T>* ZO = p.resident ? ZS : reinterpret_cast<cplx<T>*>(base + Lo.Zo);
    const int ngroups = (p.Mt + p.zg) / p.zg;
    const bool slab_ev = c->opt_timing && c->ev_ok;
    if (slab_ev) {
        size_t need = (size_t)3 * ngroups + 1;
        while (c->sev.size() < need) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            c->sev.push_back(e);
        }
        c->nsev = 0;
        HIPCHK(hipEventRecord(c->sev[c->nsev++], st));
    }
    set_b(p.By);
    za.l3lo = p.l3lo;
    za.czero = pa.czero;
    za.lzc = p.lzc;
    for (int k0 = 0; k0 <= p.Mt; k0 += p.zg) {
        const int cnt = std::min(p.zg, p.Mt + 1 - k0);
        pa.k1base = k0;
        pa.nk1 = cnt;
        za.k1base = k0;
        za.nk1 = cnt;
        pa.cs_in = csA;
        pa.cs_out = csS;
        HIPCHK(launch_fwd_y<T>(Yc, ZS, pa, p.ncin, st));
        if (slab_ev) HIPCHK(hipEventRecord(c->sev[c->nsev++], st));
        HIPCHK(launch_z<T>(p.family, cm, ZS, ZO, za, p.resident, st));
        if (slab_ev) HIPCHK(hipEventRecord(c->sev[c->nsev++], st));
        pa.cs_in = csS;
        pa.cs_out = csA;
        pa.l3lo = p.l3lo;
        HIPCHK(launch_inv_y<T>(ZO, Yc, pa, ncout_for(p.prec, cm), st));
        pa.l3lo = 0;
        if (slab_ev) HIPCHK(hipEventRecord(c->sev[c->nsev++], st));
    }
    rec_ev(EHS_ST_ZSCALE);
    rec_ev(EHS_ST_INVY);

    rec_ev(EHS_ST_INVX);
    set_b(p.Bx);
    pa.cs_in = csA;
    pa.cs_out = csR;
    pa.l3lo = p.l3lo;
    HIPCHK(launch_inv_x<T>(Yc, X, pa, ncout_for(p.prec, cm), st));
    if (c->parts == 1)  // real-space part only: the quadrature reads a cleared grid
        HIPCHK(fill_u32(reinterpret_cast<uint32_t*>(X), 0u, (long long)((Lo.Y - Lo.X) / 4), st));
    c->tap_grids[1] = ncout_for(p.prec, cm);
    if (c->tap_quad) {
        const long long nq = ncout_for(p.prec, cm) * csR;
        if (c->tap_quad_cap < nq) return EHS_EINVAL;
        HIPCHK(launch_convert(c->tap_quad, X, nq, st));
    }
    if (c->last_overlap) HIPCHK(hipEventRecord(c->ev_pre_join, st));
    join.now();
    rec_ev(EHS_ST_GATHER);

    // -- quadrature at the targets and FP64 combination with the real part:
    //    dense targets four per wavefront, sharing the walk over their
    //    supports (grouped form); large supports at low target density in
    //    node-owner form (targets sorted by the quadrature tile of their
    //    support base, one wavefront per tile for the partial sums, then a
    //    fixed-order sum per target); one wavefront per target only for grids
    //    too large for the grouped form's 32-bit offsets
    if (p.ggroup) {
        // targets sorted along a Morton curve over 2^3-node bins of their
        // support base (wider bins on grids of 1024 nodes and more, so that
        // the three 10-bit indices fit a 32-bit key), so that consecutive
        // targets share most of their supports
        int sh = 1;
        while (((2LL * p.Mt) >> sh) >= 1024) ++sh;
        int nb = 1;
        while ((1LL << nb) < ((2LL * p.Mt) >> sh) + 1) ++nb;  // bits of a bin index
        uint32_t* gk = reinterpret_cast<uint32_t*>(base + Lo.gkeys);
        uint32_t *gv = gk + TT, *gk2 = gv + TT, *gv2 = gk2 + TT;
        uint32_t *gks, *gperm;
        HIPCHK(launch_target_zkeys(xs, TT, p.gg, sh, gk, gv, st));
        HIPCHK(radix_sort(gk, gv, gk2, gv2, TT, (3 * nb + 3) / 4 * 4, sortsc, st, &gks, &gperm));
        HIPCHK(launch_gather_group<T>(p.gg, cm, X, csR, xs, gperm, tperm, TT, upart, u, st));
    } else if (!p.gtiles) {
        HIPCHK(launch_gather<T>(p.gg, cm, X, csR, xs, tperm, TT, upart, u, st));
    } else {
        uint32_t* gk = reinterpret_cast<uint32_t*>(base + Lo.gkeys);
        uint32_t *gv = gk + TT, *gk2 = gv + TT, *gv2 = gk2 + TT;
        uint32_t* gtoff = reinterpret_cast<uint32_t*>(base + Lo.gtoff);
        T* grec = reinterpret_cast<T*>(base + Lo.grec);
        T* gpart = reinterpret_cast<T*>(base + Lo.gpart);
        uint32_t *gks, *gperm;
        HIPCHK(launch_target_keys(xs, TT, p.gg, gk, gv, st));
        HIPCHK(radix_sort(gk, gv, gk2, gv2, TT, bits_for(p.ntiles_g), sortsc, st, &gks, &gperm));
        HIPCHK(launch_cell_ranges(gks, TT, gtoff, nullptr, p.ntiles_g, st));
        HIPCHK(launch_target_records<T>(xs, gperm, TT, p.gg, grec, st));
        HIPCHK(launch_gather_tiles<T>(p.gg, X, csR, grec, gtoff, p.l3lo / 8, gpart, st));
        HIPCHK(launch_gather_final<T>(p.gg, grec, gpart, TT, xs, tperm, upart, u, st));
    }
    rec_ev(EHS_ST_TOTAL);
    return EHS_OK;
}

}  // namespace

int ehs::plan_request(ehs_ctx* c, int family, const double* y, const double* s, int64_t N, const double* x,
                      int64_t T, double xi, double rc, double tol, int prec, hipStream_t st, Plan* p, bool free_space)
{
    if (family < 0 || family > 2) return EHS_EINVAL;
    if (prec < 0 || prec > 2) return EHS_EINVAL;
    if (!y || !s || N < 1 || T < 0 || (T > 0 && !x)) return EHS_EINVAL;
    if (!(xi > 0) || !(rc > 0) || !std::isfinite(xi) || !std::isfinite(rc)) return EHS_EINVAL;
    if (!(tol >= 1e-14 && tol <= 1e-2)) return EHS_EINVAL;
    if (N >= (1LL << 30) || T >= (1LL << 31)) return EHS_EINVAL;
    // bounding box, validation, Q and the target heights (one readback)
    size_t need = al((size_t)(1024 * 10 + 16 + ZH_BINS / 2) * sizeof(double));
    if (c->ws_external) {
        if (c->ws_bytes < need) return EHS_ENOMEM;
    } else {
        int rc0 = ensure_ws(c, std::max(need, c->ws_bytes), st, -1);
        if (rc0) return rc0;
    }
    char* base = static_cast<char*>(c->ws);
    double* partial = reinterpret_cast<double*>(base);
    double* out16 = partial + 1024 * 10;
    uint32_t* zhist = reinterpret_cast<uint32_t*>(out16 + 16);
    const double zbin = rc / 6.0;  // layers of r_c, r_c / 2 and r_c / 3 are whole numbers of bins
    int nb = bbox_blocks(N + T);
    HIPCHK(launch_bbox(family, y, s, N, x, T, partial, nb, out16, 1.0 / zbin, zhist, st));
    HIPCHK(hipMemcpyAsync(c->host_bbox, out16, 16 * sizeof(double) + ZH_BINS * sizeof(uint32_t),
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double* b = c->host_bbox;
    if (b[8] > 0) return EHS_EDOMAIN;
    // the half space: sources above the wall, targets not below it
    if (!free_space && !(b[6] > 0)) return EHS_EDOMAIN;
    if (!free_space && T > 0 && !(b[7] >= 0)) return EHS_EDOMAIN;
    PlanInput in;
    in.family = family;
    in.N = N;
    in.T = T;
    in.xi = xi;
    in.rc = rc;
    in.tol = tol;
    for (int a = 0; a < 3; ++a) {
        in.lo[a] = b[a];
        in.hi[a] = b[3 + a];
    }
    in.Q = b[9];
    in.prec = prec;
    in.force_M = c->force_M;
    in.force_P = c->force_P;
    in.force_Mt = c->force_Mt;
    in.force_zg = c->force_zg;
    in.gather_extra = c->gather_extra;
    in.dgrid = c->dgrid;
    in.tlo3 = T > 0 ? b[7] : 0.0;
    in.slo3 = b[6];
    // (the height histogram counts from the wall: none in free space)
    in.zhist = free_space ? nullptr : reinterpret_cast<const uint32_t*>(b + 16);
    in.zbin = zbin;
    in.force_nr = c->force_nr;
    in.free = free_space;
    return make_plan(in, p);
}

int ehs::plan_workspace(const Plan& p, size_t* bytes)
{
    size_t esz = p.prec == 1 ? 8 : 4;
    Layout Lo = layout(p, esz);
    int rc = check_extents(p, Lo, esz);
    if (rc) return rc;
    *bytes = Lo.total;
    return EHS_OK;
}

int ehs::execute(ehs_ctx* c, Plan& p, const Octants& o, const double* y, const double* s, const double* x, double* u,
                 hipStream_t st)
{
    if (p.T == 0) return EHS_OK;
    bool alias = (x == y) && (p.T == p.N);
    return (p.prec == 1) ? run<double>(c, p, o, y, s, x, u, st, alias) : run<float>(c, p, o, y, s, x, u, st, alias);
}

void ehs::fill_report(const Plan& p, ehs_report* r)
{
    std::memset(r, 0, sizeof(*r));
    r->M = p.M;
    r->P = p.P;
    r->Mt = p.Mt;
    r->precision = p.prec;
    r->Q = p.Qz;
    r->nf = p.nf;
    r->nf3 = p.nf3;
    r->warnings = p.warnings;
    for (int a = 0; a < 3; ++a) {
        r->ncell[a] = p.cg.nc[a];
        r->origin[a] = p.g.o[a];
    }
    r->family = p.family;
    r->L = p.L;
    r->h = p.h;
    r->Lt = p.Lt;
    r->eta = p.eta;
    r->xi = p.xi;
    r->r_c = p.rc;
    r->tol = p.tol;
    r->est_real = p.est_r;
    r->est_fourier = p.est_f;
    r->zslab = p.zg;
    r->Pg = p.Pg;
    r->Ps = p.Ps;
    r->dgrid = p.dgrid ? 1 : 0;
    r->est_fp32 = p.est32;
    r->x3_first = p.l3lo;
    r->x3_corr_end = p.lzc;
    r->cell_reach = p.cg.nr;
    r->occupancy = p.occ;
    r->free_space = p.free ? 1 : 0;
}

namespace {

// report of a finished evaluation, with the stage times when timing is on
int finish_report(ehs_ctx* c, const Plan& p, size_t need, ehs_report* rep)
{
    if (!rep) return EHS_OK;
    fill_report(p, rep);
    rep->workspace_bytes = (double)need;
    if (!(c->opt_timing && c->ev_ok)) return EHS_OK;
    if (hipEventSynchronize(c->ev[EHS_ST_TOTAL]) != hipSuccess) return EHS_EHIP;
    for (int i = 0; i < EHS_ST_TOTAL; ++i) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]);
        rep->ms_stage[i] = ms;
    }
    if (c->last_overlap) {
        // the real-space sum on the side stream; the inverse x1 pass ends
        // where the caller's stream starts waiting for it
        float mr = 0.f, mi = 0.f;
        hipEventElapsedTime(&mr, c->ev[EHS_ST_REAL], c->ev_rs_end);
        hipEventElapsedTime(&mi, c->ev[EHS_ST_INVX], c->ev_pre_join);
        rep->ms_stage[EHS_ST_REAL] = mr;
        rep->ms_stage[EHS_ST_INVX] = mi;
    }
    float tot = 0.f;
    hipEventElapsedTime(&tot, c->ev[EHS_ST_BBOX], c->ev[EHS_ST_TOTAL]);
    rep->ms_stage[EHS_ST_TOTAL] = tot;
    if (c->pairs_dev) {
        unsigned long long h[2] = {0ull, 0ull};
        if (hipMemcpy(h, c->pairs_dev, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return EHS_EHIP;
        rep->pairs_direct = (double)h[0];
        rep->pairs_image = (double)h[1];
    }
    // the y / x3 pipeline: per-kernel sums over the slab groups
    double sy = 0, sz = 0, si = 0;
    for (int g = 0; 3 * g + 3 < c->nsev; ++g) {
        float m0 = 0.f, m1 = 0.f, m2 = 0.f;
        hipEventElapsedTime(&m0, c->sev[3 * g], c->sev[3 * g + 1]);
        hipEventElapsedTime(&m1, c->sev[3 * g + 1], c->sev[3 * g + 2]);
        hipEventElapsedTime(&m2, c->sev[3 * g + 2], c->sev[3 * g + 3]);
        sy += m0;
        sz += m1;
        si += m2;
    }
    if (c->nsev > 1) {
        rep->ms_stage[EHS_ST_FWDY] = sy;
        rep->ms_stage[EHS_ST_ZSCALE] = sz;
        rep->ms_stage[EHS_ST_INVY] = si;
    }
    return EHS_OK;
}

void start_timing(ehs_ctx* c, hipStream_t st)
{
    if (c->opt_timing && !c->ev_ok) {
        bool ok = true;
        for (int i = 0; i <= EHS_NSTAGES; ++i) ok = ok && hipEventCreate(&c->ev[i]) == hipSuccess;
        c->ev_ok = ok;
    }
    if (c->opt_timing && c->ev_ok) hipEventRecord(c->ev[EHS_ST_BBOX], st);
}

int evaluate(ehs_ctx* c, int family, const double* y, const double* s, int64_t N, const double* x, int64_t T,
             double xi, double rc, double tol, double* u, void* stream, ehs_report* rep, bool free_space = false)
{
    if (!c) return EHS_EINVAL;
    if (c->fixed)
        return evaluate_fixed(c, c->fixed, family, y, s, N, x, T, xi, rc, tol, u, stream, rep, EHS_ENOMEM,
                              free_space);
    if (T > 0 && !u) return EHS_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return EHS_EHIP;
    hipStream_t st = static_cast<hipStream_t>(stream);
    start_timing(c, st);
    Plan p;
    int r = plan_request(c, family, y, s, N, x, T, xi, rc, tol, c->opt_prec, st, &p, free_space);
    if (r) return r;
    if (T == 0) {
        if (rep) fill_report(p, rep);
        return EHS_OK;
    }
    size_t need = 0;
    if ((r = plan_workspace(p, &need))) return r;
    if ((r = ensure_ws(c, need, st, p.Mt))) return r;
    if (c->opt_timing && c->ev_ok) hipEventRecord(c->ev[EHS_ST_PRECOMP], st);
    bool ran = false;
    Octants* oct = nullptr;
    if ((r = ensure_octants(c, p, st, &ran, &oct))) return r;
    if (ran) p.warnings |= 2;
    if ((r = execute(c, p, *oct, y, s, x, u, st))) return r;
    return finish_report(c, p, need, rep);
}

// ---------------------------------------------------------------------------
// evaluations from a fixed region (no device allocation)
// ---------------------------------------------------------------------------
// offsets of the octant arrays held for `mask` (bit 0 H64, 1 B64, 2 H32,
// 3 B32), in that order; returns the bytes of the octant part
size_t fixed_oct_layout(int Mt, unsigned mask, size_t off[4])
{
    const size_t n = (size_t)octant_elems(Mt);
    size_t o = 0;
    for (int i = 0; i < 4; ++i) {
        off[i] = o;
        if (mask & (1u << i)) o += al(n * (i < 2 ? 8 : 4));
    }
    return o;
}

unsigned octant_mask(const Plan& p)
{
    const bool needH = !(p.free && p.family != EHS_ROTLET), needB = p.family != EHS_ROTLET;
    unsigned m = 0u;
    if (needH) m |= p.prec == 2 ? 5u : 1u;  // H64 (and H32)
    if (needB) m |= p.prec == 2 ? 10u : 2u;  // B64 (and B32)
    return m;
}

// restores the fields of a context that a fixed-region evaluation borrows
struct Borrow {
    ehs_ctx* c;
    void* ws;
    size_t ws_bytes;
    bool ws_external;
    Tables* tables;
    int timing;
    explicit Borrow(ehs_ctx* c_)
        : c(c_), ws(c_->ws), ws_bytes(c_->ws_bytes), ws_external(c_->ws_external), tables(c_->tables),
          timing(c_->opt_timing)
    {
    }
    ~Borrow()
    {
        c->ws = ws;
        c->ws_bytes = ws_bytes;
        c->ws_external = ws_external;
        c->tables = tables;
        c->opt_timing = timing;
    }
};

}  // namespace

int ehs::evaluate_fixed(ehs_ctx* c, Fixed* fx, int family, const double* y, const double* s, int64_t N,
                        const double* x, int64_t T, double xi, double rc, double tol, double* u, void* stream,
                        ehs_report* rep, int too_big, bool free_space)
{
    if (!c || !fx || !fx->base) return EHS_EINVAL;
    if (T > 0 && !u) return EHS_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return EHS_EHIP;
    std::lock_guard<std::mutex> lk(fx->mu);
    hipStream_t st = static_cast<hipStream_t>(stream);
    Borrow keep(c);
    // the scratch of the allocation-free entry point is not the context's:
    // no timing events there (their creation is the context's business)
    if (fx != c->fixed) c->opt_timing = 0;
    start_timing(c, st);
    c->tables = &fx->tables;
    c->ws_external = true;
    c->ws = fx->base + FIXED_TABLE_BYTES;  // the bounding-box scratch first
    c->ws_bytes = FIXED_BB_BYTES;
    Plan p;
    // (the bounding-box readback synchronises the stream: every earlier call
    // on it has finished reading the tables and octants rewritten below)
    int r = plan_request(c, family, y, s, N, x, T, xi, rc, tol, c->opt_prec, st, &p, free_space);
    if (r) return r;
    if (T == 0) {
        if (rep) fill_report(p, rep);
        return EHS_OK;
    }
    const size_t head = FIXED_TABLE_BYTES + FIXED_BB_BYTES;
    const unsigned need_mask = octant_mask(p);
    const bool reuse = fx->oct_Mt == p.Mt && (fx->oct_mask & need_mask) == need_mask;
    const unsigned mask = reuse ? fx->oct_mask : need_mask;
    size_t off[4];
    const size_t oct_bytes = fixed_oct_layout(p.Mt, mask, off);
    if (head + oct_bytes >= fx->bytes) return too_big;
    const size_t avail = fx->bytes - head - al(oct_bytes);
    // the slab groups of the y / x3 pipeline shrink until the workspace fits
    size_t need = 0;
    for (;;) {
        if ((r = plan_workspace(p, &need))) return r;
        if (need <= avail) break;
        if (p.zg == 1) return too_big;
        p.zg = std::max(1, p.zg / 2);
    }
    c->ws = fx->base + head + al(oct_bytes);
    c->ws_bytes = avail;
    // tables: start afresh when half of the table region is used (one plan
    // needs a few MB at most)
    if (fx->tables.used > fx->tables.cap / 2) {
        fx->tables.m.clear();
        fx->tables.used = 0;
    }
    if (c->opt_timing && c->ev_ok) hipEventRecord(c->ev[EHS_ST_PRECOMP], st);
    char* ob = fx->base + head;
    Octants o;
    o.H64 = (mask & 1u) ? reinterpret_cast<double*>(ob + off[0]) : nullptr;
    o.B64 = (mask & 2u) ? reinterpret_cast<double*>(ob + off[1]) : nullptr;
    o.H32 = (mask & 4u) ? reinterpret_cast<float*>(ob + off[2]) : nullptr;
    o.B32 = (mask & 8u) ? reinterpret_cast<float*>(ob + off[3]) : nullptr;
    if (!reuse) {
        fx->oct_Mt = 0;  // invalid until every array is produced
        fx->oct_mask = 0;
        double* scratch = static_cast<double*>(c->ws);
        for (int kind = 0; kind < 2; ++kind) {
            double* d64 = kind == 0 ? o.H64 : o.B64;
            if (!d64) continue;
            if ((r = take_injected_failure(&c->fail_precompute))) return r;
            if ((r = precompute_kind(c, p.Mt, p.nf, p.nf3, kind, scratch, d64, st))) return r;
            float* d32 = kind == 0 ? o.H32 : o.B32;
            if (d32) HIPCHK(launch_oct_to_f32(d64, d32, octant_elems(p.Mt), st));
        }
        HIPCHK(hipStreamSynchronize(st));
        fx->oct_Mt = p.Mt;
        fx->oct_mask = mask;
        fx->nf = p.nf;
        fx->nf3 = p.nf3;
        p.warnings |= 2;
    }
    if ((r = execute(c, p, o, y, s, x, u, st))) return r;
    return finish_report(c, p, need, rep);
}

void ehs::free_tables(Tables* t)
{
    if (!t) return;
    if (!t->arena)
        for (auto& kv : t->m) hipFree(kv.second);
    t->m.clear();
    t->used = 0;
}

int ehs::ctx_init(ehs_ctx* c, int device, Tables* shared)
{
    c->device = device;
    if (shared) {
        c->tables = shared;
        c->own_tables = false;
    } else {
        c->tables = new (std::nothrow) Tables();
        c->own_tables = true;
        if (!c->tables) return EHS_ENOMEM;
    }
    if (hipHostMalloc((void**)&c->host_bbox, 16 * sizeof(double) + ZH_BINS * sizeof(uint32_t),
                      hipHostMallocDefault) != hipSuccess) {
        c->host_bbox = nullptr;
        return EHS_ENOMEM;
    }
    // the real-space sum's stream (default priority) and its fork / join
    // events; without them the sum runs on the caller's stream
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&c->ev_rs_end) != hipSuccess || hipEventCreate(&c->ev_pre_join) != hipSuccess) {
        hipGetLastError();
        c->overlap = 0;
    }
    return EHS_OK;
}

void ehs::ctx_release(ehs_ctx* c)
{
    if (c->ws && !c->ws_external) hipFree(c->ws);
    c->ws = nullptr;
    for (auto& kv : c->cache) free_octants(kv.second);
    c->cache.clear();
    if (c->fixed) {
        free_tables(&c->fixed->tables);
        if (c->fixed->base) hipFree(c->fixed->base);
        delete c->fixed;
        c->fixed = nullptr;
    }
    if (c->own_tables && c->tables) {
        free_tables(c->tables);
        delete c->tables;
    }
    c->tables = nullptr;
    if (c->ev_ok)
        for (int i = 0; i <= EHS_NSTAGES; ++i) hipEventDestroy(c->ev[i]);
    c->ev_ok = false;
    for (hipEvent_t e : c->sev) hipEventDestroy(e);
    c->sev.clear();
    if (c->host_bbox) hipHostFree(c->host_bbox);
    c->host_bbox = nullptr;
    for (hipEvent_t* e : {&c->fork, &c->join, &c->ev_rs_end, &c->ev_pre_join}) {
        if (*e) hipEventDestroy(*e);
        *e = nullptr;
    }
    if (c->side) hipStreamDestroy(c->side);
    c->side = nullptr;
}

extern "C" {

int ehs_create(ehs_ctx** out, int hip_device, size_t arena_bytes)
{
    if (!out) return EHS_EINVAL;
    *out = nullptr;
    if (arena_bytes > 0 && arena_bytes < EHS_ARENA_MIN_BYTES) return EHS_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return EHS_EINVAL;
    if (hipSetDevice(hip_device) != hipSuccess) return EHS_EHIP;
    ehs_ctx* c = new (std::nothrow) ehs_ctx();
    if (!c) return EHS_ENOMEM;
    int rc = ctx_init(c, hip_device, nullptr);
    // the static scratch of the allocation-free entry point on this device
    if (!rc) rc = noalloc_attach(hip_device);
    if (!rc && arena_bytes > 0) {
        // one region for tables, octants and workspace: no allocation later
        c->fixed = new (std::nothrow) Fixed();
        if (!c->fixed) rc = EHS_ENOMEM;
        if (!rc && hipMalloc((void**)&c->fixed->base, arena_bytes) != hipSuccess) {
            c->fixed->base = nullptr;
            hipGetLastError();
            rc = EHS_ENOMEM;
        }
        if (!rc) {
            c->fixed->bytes = arena_bytes;
            c->fixed->tables.arena = c->fixed->base;
            c->fixed->tables.cap = FIXED_TABLE_BYTES;
        }
    }
    if (rc) {
        ctx_release(c);
        delete c;
        return rc;
    }
    *out = c;
    return EHS_OK;
}

void ehs_destroy(ehs_ctx* c)
{
    if (!c) return;
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    ctx_release(c);
    delete c;
}

int ehs_set_option(ehs_ctx* c, int option, double value)
{
    if (!c) return EHS_EINVAL;
    switch (option) {
        case EHS_OPT_PRECISION:
            if (value != 0 && value != 1 && value != 2) return EHS_EINVAL;
            c->opt_prec = (int)value;
            return EHS_OK;
        case EHS_OPT_TIMING: c->opt_timing = value != 0; return EHS_OK;
        case EHS_OPT_FORCE_M: c->force_M = (int)value; return EHS_OK;
        case EHS_OPT_FORCE_P: c->force_P = (int)value; return EHS_OK;
        case EHS_OPT_FORCE_MT: c->force_Mt = (int)value; return EHS_OK;
        case EHS_OPT_MEM_CAP: c->mem_cap = value; return EHS_OK;
        case EHS_OPT_ZSLAB: c->force_zg = (int)value; return EHS_OK;
        case EHS_OPT_GATHER_EXTRA: c->gather_extra = (int)value; return EHS_OK;
        case EHS_OPT_DGRID: c->dgrid = (int)value; return EHS_OK;
        case EHS_OPT_FAIL_PRECOMPUTE: c->fail_precompute = std::max(0, (int)value); return EHS_OK;
        case EHS_OPT_CELL_REACH:
            if (value < 0 || value > 3) return EHS_EINVAL;
            c->force_nr = (int)value;
            return EHS_OK;
        case EHS_OPT_OVERLAP:
            if (value != 0 && value != 1) return EHS_EINVAL;
            c->overlap = (value == 1 && c->side) ? 1 : 0;
            return EHS_OK;
        case EHS_OPT_PARTS:
            if (value != 0 && value != 1 && value != 2) return EHS_EINVAL;
            c->parts = (int)value;
            return EHS_OK;
        default: return EHS_EINVAL;
    }
}

int ewald_halfspace_stokeslet(ehs_ctx* c, const double* sources, const double* f, int64_t N, const double* targets,
                              int64_t T, double xi, double r_c, double tol, double* u_out, void* stream,
                              ehs_report* rep)
{
    return evaluate(c, EHS_STOKESLET, sources, f, N, targets, T, xi, r_c, tol, u_out, stream, rep);
}

int ewald_halfspace_stresslet(ehs_ctx* c, const double* sources, const double* gq, int64_t N, const double* targets,
                              int64_t T, double xi, double r_c, double tol, double* u_out, void* stream,
                              ehs_report* rep)
{
    return evaluate(c, EHS_STRESSLET, sources, gq, N, targets, T, xi, r_c, tol, u_out, stream, rep);
}

int ewald_halfspace_rotlet(ehs_ctx* c, const double* sources, const double* v, int64_t N, const double* targets,
                           int64_t T, double xi, double r_c, double tol, double* u_out, void* stream, ehs_report* rep)
{
    return evaluate(c, EHS_ROTLET, sources, v, N, targets, T, xi, r_c, tol, u_out, stream, rep);
}

int ewald_freespace_stokeslet(ehs_ctx* c, const double* sources, const double* f, int64_t N, const double* targets,
                              int64_t T, double xi, double r_c, double tol, double* u_out, void* stream,
                              ehs_report* rep)
{
    return evaluate(c, EHS_STOKESLET, sources, f, N, targets, T, xi, r_c, tol, u_out, stream, rep, true);
}

int ewald_freespace_stresslet(ehs_ctx* c, const double* sources, const double* gq, int64_t N, const double* targets,
                              int64_t T, double xi, double r_c, double tol, double* u_out, void* stream,
                              ehs_report* rep)
{
    return evaluate(c, EHS_STRESSLET, sources, gq, N, targets, T, xi, r_c, tol, u_out, stream, rep, true);
}

int ewald_freespace_rotlet(ehs_ctx* c, const double* sources, const double* v, int64_t N, const double* targets,
                           int64_t T, double xi, double r_c, double tol, double* u_out, void* stream, ehs_report* rep)
{
    return evaluate(c, EHS_ROTLET, sources, v, N, targets, T, xi, r_c, tol, u_out, stream, rep, true);
}

int ehs_debug_grid_taps(ehs_ctx* c, int family, int free_space, const double* sources, const double* strengths,
                        int64_t N, const double* targets, int64_t T, double xi, double r_c, double tol,
                        double* u_out, double* spread_out, int64_t spread_elems, const double* quad_in,
                        int64_t quad_elems, int32_t* n_grids, void* stream, ehs_report* rep)
{
    if (!c || c->fixed) return EHS_EINVAL;
    if ((spread_out && spread_elems < 1) || (quad_in && quad_elems < 1)) return EHS_EINVAL;
    struct Untap {
        ehs_ctx* c;
        ~Untap()
        {
            c->tap_spread = nullptr;
            c->tap_quad = nullptr;
            c->tap_spread_cap = c->tap_quad_cap = 0;
        }
    } untap{c};
    c->tap_spread = spread_out;
    c->tap_spread_cap = spread_out ? spread_elems : 0;
    c->tap_quad = quad_in;
    c->tap_quad_cap = quad_in ? quad_elems : 0;
    c->tap_grids[0] = c->tap_grids[1] = 0;
    int r = evaluate(c, family, sources, strengths, N, targets, T, xi, r_c, tol, u_out, stream, rep,
                     free_space != 0);
    if (n_grids) {
        n_grids[0] = c->tap_grids[0];
        n_grids[1] = c->tap_grids[1];
    }
    return r;
}

const char* ehs_strerror(int code)
{
    switch (code) {
        case EHS_OK: return "success";
        case EHS_EINVAL: return "invalid argument (null pointer, size or parameter out of range)";
        case EHS_EDOMAIN: return "point outside the half space (source y3 <= 0, target x3 < 0) or non-finite input";
        case EHS_ERANGE: return "no admissible grid for the requested accuracy";
        case EHS_ENOMEM: return "device memory exhausted or above the memory cap";
        case EHS_EHIP: return "HIP runtime error";
        case EHS_ETIMEDOUT: return "request not completed within the timeout";
        case EHS_ETOOBIG:
            return "problem larger than the fixed scratch buffer of the allocation-free entry point";
        default: return "unknown error";
    }
}

double ehs_xi_for_cutoff(int family, double r_c, double tol, double L) { return xi_for_cutoff(family, r_c, tol, L); }

double ehs_cutoff_for_estimate(int family, double xi, double est, double L)
{
    return cutoff_for_estimate(family, xi, est, L);
}

int ehs_tune(ehs_ctx* c, int family, const double* y, const double* s, int64_t N, const double* x, int64_t T,
             double xi0, double rc0, double tol, int max_evals, double* u, double* best, double* trace, int* ntrace,
             void* stream, ehs_report* rep)
{
    if (!c || !u || !best || T < 1 || family < 0 || family > 2) return EHS_EINVAL;
    if (max_evals < 1 || max_evals > 64 || !(xi0 > 0) || !(rc0 > 0)) return EHS_EINVAL;
    if (ntrace) *ntrace = 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // grid sizes cached before the search stay; of the candidates' own, only
    // the fastest candidate's octants are kept
    std::vector<int> before;
    for (auto& kv : c->cache) before.push_back(kv.first);
    // the starting point fixes the box and the real-space estimate
    ehs_report r0;
    int r = evaluate(c, family, y, s, N, x, T, xi0, rc0, tol, u, stream, &r0);
    if (r) return r;
    const double L = r0.L, est = r0.est_real;
    auto drop_unless = [&](int Mt, int keep) {
        if (Mt == keep || std::find(before.begin(), before.end(), Mt) != before.end()) return;
        auto it = c->cache.find(Mt);
        if (it == c->cache.end()) return;
        free_octants(it->second);
        c->cache.erase(it);
    };

    struct Cand {
        int k;  // xi = xi0 2^(k/8)
        double xi, rc, ms;
        int Mt;
    };
    std::vector<Cand> tried;
    // 0: timed; 1: inadmissible (ends the walk in its direction); < 0: error
    auto probe = [&](int k) -> int {
        if ((int)tried.size() >= max_evals) return 1;
        const double xi = xi0 * std::pow(2.0, 0.125 * k);
        const double rc = k == 0 ? rc0 : cutoff_for_estimate(family, xi, est, L);
        if (!(rc > 0) || rc > 0.5 * L) return 1;
        ehs_report rw;
        int e = evaluate(c, family, y, s, N, x, T, xi, rc, tol, u, stream, &rw);  // untimed
        if (e == EHS_ERANGE || e == EHS_ENOMEM) return 1;
        if (e) return e;
        // forced FP32 whose rounding estimate exceeds tol/2 where the start's did not
        if ((rw.warnings & 4) && !(r0.warnings & 4)) return 1;
        double ms = 1e300;
        for (int k = 0; k < 2; ++k) {
            if (hipStreamSynchronize(st) != hipSuccess) return EHS_EHIP;
            auto t0 = std::chrono::steady_clock::now();
            if ((e = evaluate(c, family, y, s, N, x, T, xi, rc, tol, u, stream, nullptr))) return e;
            if (hipStreamSynchronize(st) != hipSuccess) return EHS_EHIP;
            ms = std::min(ms, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
        }
        tried.push_back({k, xi, rc, ms, rw.Mt});
        // (the octants of a slower candidate are released: under
        // EHS_OPT_MEM_CAP they would otherwise crowd out later candidates)
        size_t b = 0;
        for (size_t i = 1; i < tried.size(); ++i)
            if (tried[i].ms < tried[b].ms) b = i;
        for (const Cand& t : tried) drop_unless(t.Mt, tried[b].Mt);
        return 0;
    };
    auto fastest = [&]() {
        size_t b = 0;
        for (size_t i = 1; i < tried.size(); ++i)
            if (tried[i].ms < tried[b].ms) b = i;
        return b;
    };
    if ((r = probe(0)) < 0) return r;
    if (r > 0) return EHS_ERANGE;  // the starting point itself is not admissible
    // the walk in quarter octaves: first down in xi (larger cutoff, smaller
    // grid), else up
    int dir = -1;
    if ((r = probe(-2)) < 0) return r;
    if (r > 0 || tried.back().ms >= tried[0].ms) {
        dir = +1;
        if ((r = probe(+2)) < 0) return r;
        if (r > 0 || tried.back().ms >= tried[0].ms) dir = 0;
    }
    if (dir != 0) {
        double last = tried.back().ms;
        for (int j = 2 * dir;; j += dir) {
            if ((r = probe(2 * j)) < 0) return r;
            if (r > 0 || tried.back().ms >= last) break;
            last = tried.back().ms;
        }
    }
    // then the two eighth-octave neighbours of the fastest
    const int kb = tried[fastest()].k;
    for (int dk : {-1, +1})
        if ((r = probe(kb + dk)) < 0) return r;
    const Cand* b = &tried[fastest()];
    best[0] = b->xi;
    best[1] = b->rc;
    best[2] = b->ms;
    if (trace)
        for (size_t i = 0; i < tried.size(); ++i) {
            trace[3 * i] = tried[i].xi;
            trace[3 * i + 1] = tried[i].rc;
            trace[3 * i + 2] = tried[i].ms;
        }
    if (ntrace) *ntrace = (int)tried.size();
    return evaluate(c, family, y, s, N, x, T, b->xi, b->rc, tol, u, stream, rep);
}

int ehs_plan_query(int family, int64_t N, int64_t T, const double* lo, const double* hi, double Q, double xi,
                   double r_c, double tol, int precision, ehs_report* rep)
{
    if (!lo || !hi || !rep || family < 0 || family > 2 || N < 1 || T < 0) return EHS_EINVAL;
    if (!(xi > 0) || !(r_c > 0) || !(tol >= 1e-14 && tol <= 1e-2)) return EHS_EINVAL;
    PlanInput in;
    std::memset(&in, 0, sizeof(in));
    in.family = family;
    in.N = N;
    in.T = T;
    in.xi = xi;
    in.rc = r_c;
    in.tol = tol;
    for (int a = 0; a < 3; ++a) {
        in.lo[a] = lo[a];
        in.hi[a] = hi[a];
    }
    in.Q = Q;
    in.prec = precision;
    in.gather_extra = -1;
    in.dgrid = -1;
    in.tlo3 = std::max(lo[2], 0.0);  // lowest point of the box: no target lies lower
    in.slo3 = std::max(lo[2], 0.0);  // nor any source
    Plan p;
    int rc = make_plan(in, &p);
    if (rc) return rc;
    fill_report(p, rep);
    Layout Lo = layout(p, p.prec == 1 ? 8 : 4);
    rc = check_extents(p, Lo, p.prec == 1 ? 8 : 4);
    if (rc) return rc;
    rep->workspace_bytes = (double)Lo.total;
    return EHS_OK;
}

int ehs_context_memory(const ehs_ctx* c, double* workspace_bytes, double* cache_bytes_out, int* cache_entries)
{
    if (!c) return EHS_EINVAL;
    double ws = c->fixed ? (double)c->fixed->bytes : (double)c->ws_bytes;
    double cb = (double)cache_bytes(c);
    int ne = (int)c->cache.size();
    if (workspace_bytes) *workspace_bytes = ws;
    if (cache_bytes_out) *cache_bytes_out = cb;
    if (cache_entries) *cache_entries = ne;
    return EHS_OK;
}

double ehs_truncated_kernel_hat(int kind, double k, double R) { return khat_truncated(kind, k, R); }

int ehs_debug_line_fft(ehs_ctx* c, int n, int nl, const void* in, void* out, int inverse, int fp32, void* stream)
{
    if (!c || !in || !out || n < 1 || nl < 1) return EHS_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return EHS_EHIP;
    hipStream_t st = static_cast<hipStream_t>(stream);
    FftPlanDev p;
    int esz = fp32 ? 4 : 8;
    int rc = fft_plan(c, n, esz, &p);
    if (rc) return rc;
    int cap = lds_fft_cap(n, 256);
    int per = std::max(1, std::min(cap / n, 16));
    if (n > cap) return EHS_ERANGE;
    if ((size_t)per * (n + 1) * 2 * esz > 160 * 1024) per = std::max(1, (int)(160 * 1024 / ((n + 1) * 2 * esz)));
    if (fp32)
        HIPCHK(launch_line_fft<float>(static_cast<const cplx<float>*>(in), static_cast<cplx<float>*>(out), nl, per, p,
                                      inverse != 0, st));
    else
        HIPCHK(launch_line_fft<double>(static_cast<const cplx<double>*>(in), static_cast<cplx<double>*>(out), nl, per,
                                       p, inverse != 0, st));
    return EHS_OK;
}

}  // extern "C"
