// Host-side checks of the planner, the arena allocator and the multiply-high
// reciprocals, built with AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/test_sanitizers.py).  Exit status 0 when every check holds and the
// sanitizers report nothing.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <map>
#include <random>
#include <vector>

#include "arena.h"
#include "plan.h"

using namespace ehs;

static int fails = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            if (fails < 20) std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++fails;                                                              \
        }                                                                         \
    } while (0)

int main()
{
    std::mt19937_64 g(20240611);
    auto U = [&](double a, double b) { return std::uniform_real_distribution<double>(a, b)(g); };

    // the planner over random problems: every plan it returns keeps its
    // supports within the kernels' limits and its grids 7-smooth
    int planned = 0;
    std::vector<uint32_t> zh(ZH_BINS);
    for (int it = 0; it < 20000; ++it) {
        PlanInput in{};
        in.family = (int)(g() % 3);
        in.N = 1 + (long long)(g() % 5000000);
        in.T = 1 + (long long)(g() % 5000000);
        in.free = g() % 4 == 0;
        const double L = U(0.01, 10.0);
        for (int a = 0; a < 3; ++a) {
            in.lo[a] = U(-1.0, 1.0) * L;
            in.hi[a] = in.lo[a] + U(0.05, 1.0) * L;
        }
        if (!in.free) {
            in.lo[2] = U(1e-9, 0.1) * L;
            in.hi[2] = in.lo[2] + U(0.05, 1.0) * L;
        }
        in.tol = std::pow(10.0, -U(2.0, 14.0));
        in.rc = U(0.005, 0.5) * L;
        in.xi = xi_for_cutoff(in.family, in.rc, in.tol / 2, L);
        in.Q = (double)in.N;
        in.prec = (int)(g() % 3);
        in.gather_extra = -1;
        in.dgrid = (int)(g() % 3) - 1;
        in.tlo3 = in.free ? 0.0 : in.lo[2];
        in.slo3 = in.free ? 0.0 : in.lo[2];
        in.zbin = in.rc / 6.0;
        in.zhist = nullptr;
        if (!in.free && g() % 2) {
            for (auto& v : zh) v = (uint32_t)(g() % 100000);
            in.zhist = zh.data();
        }
        in.force_nr = (int)(g() % 4);
        Plan p;
        if (make_plan(in, &p) != 0) continue;
        ++planned;
        CHECK(p.P >= 2 && p.P <= 30 && p.P % 2 == 0);
        CHECK(p.Ps <= 30 && p.Pg <= 30 && p.Ps >= p.P);
        CHECK(p.Mt % 2 == 0 && smooth7(p.Mt) && p.Mt <= EHS_MT_MAX);
        CHECK(p.Mt >= p.M + p.P);
        CHECK(p.eta > 0.0 && p.eta < 1.0);
        CHECK(p.cg.nr >= 1 && p.cg.nr <= 3);
        for (int a = 0; a < 3; ++a) {
            CHECK(p.cg.nc[a] >= 1 && p.cg.nc[a] <= 256);
            CHECK(p.g.tile[a] * p.g.K[a] >= p.g.P - 1);
            CHECK(p.g.nt[a] * p.g.tile[a] >= (a < 2 ? p.Mt : 2 * p.Mt));
            // cells of side >= r_c / nr
            CHECK(1.0 / p.cg.inv[a] * p.cg.nr >= in.rc * (1.0 - 1e-12) || p.cg.nc[a] == 1);
        }
        CHECK(p.g.tile[2] == 4 || p.g.tile[2] == 8);
        CHECK(p.ncin >= 3);
    }
    CHECK(planned > 1000);
    std::printf("planner: %d of 20000 random problems planned\n", planned);

    // the arena against a shadow map of its live ranges: no overlap, every
    // range inside the capacity and aligned, used == sum of the live sizes,
    // and a full release leaves one free range
    for (int round = 0; round < 50; ++round) {
        Arena ar;
        const size_t cap = (size_t)(1 + g() % 4096) * ARENA_ALIGN + (size_t)(g() % ARENA_ALIGN);
        ar.init(cap);
        std::map<size_t, size_t> live;  // offset -> rounded bytes
        size_t sum = 0;
        for (int op = 0; op < 2000; ++op) {
            if (live.empty() || g() % 3) {
                const size_t n = 1 + (size_t)(g() % (64 * ARENA_ALIGN));
                size_t off = 0;
                if (ar.alloc(n, &off)) {
                    const size_t r = Arena::round(n);
                    CHECK(off % ARENA_ALIGN == 0 && off + r <= ar.cap);
                    auto nx = live.lower_bound(off);
                    if (nx != live.end()) CHECK(off + r <= nx->first);
                    if (nx != live.begin()) {
                        auto pv = std::prev(nx);
                        CHECK(pv->first + pv->second <= off);
                    }
                    live[off] = r;
                    sum += r;
                }
            } else {
                auto it = live.begin();
                std::advance(it, (long)(g() % live.size()));
                ar.release(it->first, it->second);
                sum -= it->second;
                live.erase(it);
            }
            CHECK(ar.used == sum && ar.peak >= ar.used && ar.used <= ar.cap);
        }
        for (auto& kv : live) ar.release(kv.first, kv.second);
        CHECK(ar.used == 0 && ar.free_.size() == 1 && ar.free_.begin()->second == ar.cap);
    }
    std::printf("arena: 50 rounds of 2000 operations\n");

    // the multiply-high reciprocals: a / d exactly for a, d < 2^16
    long long bad = 0;
    for (unsigned d = 2; d < 4096; ++d) {
        const unsigned m = magic_of(d);
        for (unsigned a = 0; a < 65536; a += (d < 64 ? 1 : 7))
            bad += (unsigned)(((unsigned long long)a * m) >> 32) != a / d;
    }
    for (int k = 0; k < 2000000; ++k) {
        const unsigned d = 2 + (unsigned)(g() % 65534), a = (unsigned)(g() % 65536);
        bad += (unsigned)(((unsigned long long)a * magic_of(d)) >> 32) != a / d;
    }
    CHECK(bad == 0);
    std::printf("reciprocals: %lld mismatches\n", bad);
    return fails ? 1 : 0;
}
