// Internal host-side state shared by the single-call path (api.cpp) and the
// serving scheduler (serve.cpp).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/ehs.h"
#include "kernels.h"
#include "plan.h"

namespace ehs {

// Truncated-kernel multipliers on the octant k1, k2 <= M~, |k3| <= 2M~
// (FP64, plus FP32 copies for the FP32 path).
struct Octants {
    double* B64 = nullptr;
    double* H64 = nullptr;
    float* B32 = nullptr;
    float* H32 = nullptr;
    int nf = 0, nf3 = 0;
};

// Twiddle and Stockham stage tables by (length, element size); immutable once
// built, the map is guarded by mu.  One per standalone context, one per server
// (shared by its slots), one per fixed region.  With `arena` set the tables
// are carved from that device region (bump allocation, never freed one by
// one) instead of allocated.
struct Tables {
    std::mutex mu;
    std::map<std::pair<int, int>, void*> m;
    char* arena = nullptr;
    size_t cap = 0, used = 0;
};

void free_tables(Tables* t);

// A fixed device region from which an evaluation takes everything it needs,
// so that it allocates nothing: the stage tables, the octants of one grid
// size and the workspace, laid out as
//   [tables: FIXED_TABLE_BYTES][bounding-box scratch: FIXED_BB_BYTES]
//   [octants of grid size oct_Mt][workspace: the rest].
// The region of a context created with arena_bytes > 0, or the per-device
// static scratch of the allocation-free entry point.  The octants are kept
// between calls and recomputed when the grid size or the arrays needed change.
constexpr size_t FIXED_TABLE_BYTES = (size_t)16 << 20;
constexpr size_t FIXED_BB_BYTES = (size_t)128 << 10;

struct Fixed {
    char* base = nullptr;
    size_t bytes = 0;
    Tables tables;
    int oct_Mt = 0;          // grid size of the octants held (0: none)
    unsigned oct_mask = 0;   // arrays held: bit 0 H64, 1 B64, 2 H32, 3 B32
    int nf = 0, nf3 = 0;
    std::mutex mu;           // host-side state; calls overlapping on the device still race
};

}  // namespace ehs

struct ehs_ctx {
    int device = 0;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_external = false;                // workspace lent by a server arena
    std::map<int, ehs::Octants> cache;       // by M~ (standalone contexts only)
    ehs::Tables* tables = nullptr;
    bool own_tables = true;
    double* host_bbox = nullptr;             // pinned: 16 doubles, then ZH_BINS uint32 counts
    hipEvent_t ev[EHS_NSTAGES + 1] = {};
    bool ev_ok = false;
    int opt_prec = 0, opt_timing = 0, force_M = 0, force_P = 0, force_Mt = 0, force_zg = 0, gather_extra = -1, dgrid = -1;
    std::vector<hipEvent_t> sev;             // per-launch events of the slab pipeline (timing)
    int nsev = 0;                            // events recorded in the last evaluation
    double mem_cap = 0.0;
    ehs::Fixed* fixed = nullptr;             // arena_bytes > 0 at creation: everything from one region
    int fail_precompute = 0;                 // test hook: the next octant production fails (EHS_EHIP)
    int force_nr = 0;                        // real-space cell reach (0: by density)
    unsigned long long* pairs_dev = nullptr; // the last timed evaluation's pair counters (workspace)
    // the real-space sum runs on `side`, beside the grid stages on the
    // caller's stream (fork and join by events); created with the context
    int overlap = 1;
    int parts = 0;  // EHS_OPT_PARTS: 0 the whole sum, 1 real-space part only, 2 Fourier part only
    // stage taps of ehs_debug_grid_taps (null outside that call): the spread
    // grids copied out, the quadrature's grids replaced, and their counts
    double* tap_spread = nullptr;
    long long tap_spread_cap = 0;
    const double* tap_quad = nullptr;
    long long tap_quad_cap = 0;
    int tap_grids[2] = {0, 0};
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipEvent_t ev_rs_end = nullptr, ev_pre_join = nullptr;  // timing of the overlapped sum
    bool last_overlap = false;               // the last timed evaluation overlapped
};

namespace ehs {

// Context set-up on the current device; `shared` (may be null) lends the
// table cache of a server.
int ctx_init(ehs_ctx* c, int device, Tables* shared);
void ctx_release(ehs_ctx* c);

// Argument checks, bounding box / validation reduction (one readback on st)
// and parameter selection with precision `prec` (0 auto, 1 FP64, 2 FP32).
int plan_request(ehs_ctx* c, int family, const double* y, const double* s, int64_t N, const double* x, int64_t T,
                 double xi, double rc, double tol, int prec, hipStream_t st, Plan* p, bool free_space = false);

// Workspace bytes of one evaluation under plan p (after the extent audit).
int plan_workspace(const Plan& p, size_t* bytes);

// Elements of one octant array for grid size Mt.
inline long long octant_elems(int Mt) { return (long long)(Mt + 1) * (Mt + 1) * (2 * Mt + 1); }

// Enqueue the precompute of one FP64 octant (kind 0: harmonic, 1: biharmonic)
// into `oct`, using the context workspace as scratch.
int precompute_octant(ehs_ctx* c, const Plan& p, int kind, double* oct, hipStream_t st);

// Enqueue one evaluation under plan p with ready octants (the workspace
// c->ws must hold plan_workspace(p) bytes).
int execute(ehs_ctx* c, Plan& p, const Octants& o, const double* y, const double* s, const double* x, double* u,
            hipStream_t st);

void fill_report(const Plan& p, ehs_report* r);

// One evaluation that takes its tables, octants and workspace from the fixed
// region fx (no device allocation); `too_big` is returned when the plan does
// not fit the region even with the smallest slab group.
int evaluate_fixed(ehs_ctx* c, Fixed* fx, int family, const double* y, const double* s, int64_t N, const double* x,
                   int64_t T, double xi, double rc, double tol, double* u, void* stream, ehs_report* rep,
                   int too_big, bool free_space = false);

// Resolve the device address of the static scratch of the allocation-free
// entry point for `device` (which must be current); called once per device
// at context creation.  Returns EHS_OK or EHS_EHIP.
int noalloc_attach(int device);

}  // namespace ehs
