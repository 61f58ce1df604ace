// Serving: continuous batching of half-space Ewald requests on one device.
//
// A server owns one device arena.  Every admitted request gets a workspace
// carved from it, plus the truncated-kernel octants it needs, which are
// shared between requests and kept in the arena as a cache.  Requests run on
// `nslots` slots, each a host worker thread with its own stream and context;
// their device work overlaps.  Admission happens whenever a request arrives
// or one completes.  First-come (EHS_OPT_ADMISSION 0): the oldest queued
// request that fits a free slot and the arena is started; younger requests
// may overtake a head that does not fit, at most MAX_BYPASS times per head.
// Smallest-first (1, the default): among the queued requests that fit, the
// one with the smallest workspace (a measure of its grid and point work)
// starts first, and one slot is kept for requests of at most EXPRESS_POINTS
// points, so that small requests neither queue behind large ones nor wait
// for a slot they hold; the oldest request may still be overtaken at most
// MAX_BYPASS times, after which the general slots wait for it.
//
// Octant sharing: a request that finds an octant missing allocates it and
// enqueues its precompute on its own stream, then records an event.  Others
// that need it wait for that event on their streams (hipStreamWaitEvent), not
// on the host.  A cached octant is evicted (least recently used first) only
// when no admitted request references it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/ehs.h"
#include "arena.h"
#include "ctx.h"

using namespace ehs;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int MAX_BYPASS = 8;
constexpr long long EXPRESS_POINTS = 65536;  // N + T of a request the kept slot takes

// one cached octant array in the arena
struct Unit {
    int Mt = 0, kind = 0;
    bool f32 = false;
    size_t off = 0, bytes = 0;
    hipEvent_t ready = nullptr;  // recorded after its production
    bool recorded = false, failed = false;
    int refs = 0;
    uint64_t last_use = 0;
};

inline long long unit_key(int Mt, int kind, bool f32) { return (long long)Mt * 4 + kind * 2 + (f32 ? 1 : 0); }

enum { REQ_QUEUED = 1, REQ_RUNNING = 2, REQ_DONE = 0 };

struct Req {
    uint64_t ticket = 0;
    ehs_request r;
    Plan plan;
    size_t ws_bytes = 0, ws_off = 0, footprint = 0;
    std::vector<Unit*> units;    // every octant it reads (references held while admitted)
    std::vector<Unit*> produce;  // those it allocated and must produce (FP64 before FP32)
    int state = REQ_QUEUED, code = EHS_OK, slot = -1, bypassed = 0;
    double t_submit = 0, t_admit = 0, t_done = 0, gpu_ms = 0;
};

struct Slot {
    ehs_ctx ctx;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    Req* job = nullptr;
    std::condition_variable cv;
    std::thread th;
};

}  // namespace

struct ehs_server {
    int device = 0;
    char* mem = nullptr;
    Arena arena;
    Tables tables;
    ehs_ctx admin;
    hipStream_t admin_st = nullptr;
    std::mutex admin_mu;  // planning (bounding-box readback) of submissions

    std::mutex mu;  // everything below
    std::condition_variable cv_done, cv_units;
    std::deque<Req*> pending;
    std::map<uint64_t, Req*> reqs;
    std::map<long long, Unit*> units;
    std::vector<Slot*> slots;
    bool stop = false;
    uint64_t next_ticket = 1, use_clock = 0;
    int running = 0;
    std::atomic<int> fail_productions{0};  // test hook (EHS_OPT_FAIL_PRECOMPUTE)
    int admission = 1;                     // EHS_OPT_ADMISSION
    int64_t submitted = 0, completed = 0, failed = 0, rejected = 0, hits = 0, misses = 0, evictions = 0;
    size_t cache_bytes = 0;
    Clock::time_point t0;

    double now_ms() const { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }
};

namespace {

void destroy_unit(ehs_server* s, Unit* u)
{
    s->arena.release(u->off, u->bytes);
    s->cache_bytes -= Arena::round(u->bytes);
    if (u->ready) hipEventDestroy(u->ready);
    auto it = s->units.find(unit_key(u->Mt, u->kind, u->f32));
    if (it != s->units.end() && it->second == u) s->units.erase(it);
    delete u;
}

// allocate, evicting unreferenced cached octants (least recently used first)
bool alloc_evict(ehs_server* s, size_t bytes, size_t* off)
{
    while (!s->arena.alloc(bytes, off)) {
        Unit* victim = nullptr;
        for (auto& kv : s->units) {
            Unit* u = kv.second;
            if (u->refs == 0 && u->recorded && (!victim || u->last_use < victim->last_use)) victim = u;
        }
        if (!victim) return false;
        destroy_unit(s, victim);
        ++s->evictions;
    }
    return true;
}

// octants a plan reads: H always, B unless rotlet; FP32 copies in FP32 mode
void needed_units(const Plan& p, std::vector<long long>& keys)
{
    keys.clear();
    for (int kind = 0; kind < 2; ++kind) {
        if (kind == 1 && p.family == EHS_ROTLET) continue;
        keys.push_back(unit_key(p.Mt, kind, false));
        if (p.prec == 2) keys.push_back(unit_key(p.Mt, kind, true));
    }
}

size_t unit_bytes(int Mt, bool f32) { return (size_t)octant_elems(Mt) * (f32 ? 4 : 8); }

// Try to admit r (lock held): workspace and missing octants from the arena.
bool admit(ehs_server* s, Req* r)
{
    std::vector<long long> keys;
    needed_units(r->plan, keys);
    std::vector<Unit*> have;
    for (long long k : keys) {
        auto it = s->units.find(k);
        if (it != s->units.end()) {
            it->second->refs++;  // pin against eviction while admitting
            have.push_back(it->second);
        }
    }
    auto unpin = [&]() {
        for (Unit* u : have) u->refs--;
    };
    size_t off = 0;
    if (!alloc_evict(s, r->ws_bytes, &off)) {
        unpin();
        return false;
    }
    std::vector<Unit*> made;
    bool ok = true;
    for (long long k : keys) {
        if (s->units.count(k)) continue;
        Unit* u = new (std::nothrow) Unit();
        if (!u) {
            ok = false;
            break;
        }
        u->Mt = (int)(k / 4);
        u->kind = (int)((k / 2) % 2);
        u->f32 = (k % 2) != 0;
        u->bytes = unit_bytes(u->Mt, u->f32);
        if (!alloc_evict(s, u->bytes, &u->off)) {
            delete u;
            ok = false;
            break;
        }
        if (hipEventCreateWithFlags(&u->ready, hipEventDisableTiming) != hipSuccess) {
            s->arena.release(u->off, u->bytes);
            delete u;
            ok = false;
            break;
        }
        u->refs = 1;
        s->units[k] = u;
        s->cache_bytes += Arena::round(u->bytes);
        made.push_back(u);
    }
    if (!ok) {
        for (Unit* u : made) {
            u->refs = 0;
            u->recorded = true;
            destroy_unit(s, u);
        }
        s->arena.release(off, r->ws_bytes);
        unpin();
        return false;
    }
    r->ws_off = off;
    r->units = have;
    r->units.insert(r->units.end(), made.begin(), made.end());
    // produce FP64 arrays before their FP32 copies
    std::stable_sort(made.begin(), made.end(), [](const Unit* a, const Unit* b) { return !a->f32 && b->f32; });
    r->produce = made;
    s->hits += (int64_t)have.size();
    s->misses += (int64_t)made.size();
    for (Unit* u : r->units) u->last_use = ++s->use_clock;
    return true;
}

void start(ehs_server* s, Req* r, Slot* sl)
{
    r->state = REQ_RUNNING;
    r->t_admit = s->now_ms();
    r->slot = (int)(std::find(s->slots.begin(), s->slots.end(), sl) - s->slots.begin());
    sl->job = r;
    s->running++;
    sl->cv.notify_one();
}

bool is_small(const Req* r) { return r->r.N + r->r.T <= EXPRESS_POINTS; }

// Smallest-first admission (lock held): the last slot (with two or more) is
// kept for small requests.
void try_admit_smallest(ehs_server* s)
{
    const size_t ns = s->slots.size();
    Slot* express = ns >= 2 ? s->slots.back() : nullptr;
    for (;;) {
        Slot *gen = nullptr, *exp = nullptr;
        for (Slot* sl : s->slots)
            if (!sl->job) {
                if (sl == express)
                    exp = sl;
                else if (!gen)
                    gen = sl;
            }
        if ((!gen && !exp) || s->pending.empty()) return;
        Req* head = s->pending.front();
        const bool aged = head->bypassed >= MAX_BYPASS;
        // candidates by workspace size, oldest first among equals
        std::vector<Req*> cand(s->pending.begin(), s->pending.end());
        std::stable_sort(cand.begin(), cand.end(), [](const Req* a, const Req* b) { return a->ws_bytes < b->ws_bytes; });
        // a request that does not fit the arena stops the search for its slot
        // (larger ones would not fit either; each try may evict cached octants)
        bool started = false;
        for (Req* r : cand) {
            Slot* sl = nullptr;
            if (is_small(r) && exp)
                sl = exp;
            else if (gen && (!aged || r == head))
                sl = gen;
            if (!sl) continue;
            if (!admit(s, r)) {
                if (sl == exp)
                    exp = nullptr;
                else
                    gen = nullptr;
                continue;
            }
            if (r != head) head->bypassed++;
            start(s, r, sl);
            s->pending.erase(std::find(s->pending.begin(), s->pending.end(), r));
            started = true;
            break;
        }
        if (!started) return;
    }
}

// Start queued requests while slots and memory allow (lock held).
void try_admit(ehs_server* s)
{
    if (s->admission == 1) {
        try_admit_smallest(s);
        return;
    }
    auto it = s->pending.begin();
    while (it != s->pending.end()) {
        Slot* free_slot = nullptr;
        for (Slot* sl : s->slots)
            if (!sl->job) {
                free_slot = sl;
                break;
            }
        if (!free_slot) return;
        Req* r = *it;
        if (admit(s, r)) {
            if (it != s->pending.begin()) s->pending.front()->bypassed++;
            start(s, r, free_slot);
            it = s->pending.erase(it);
            continue;
        }
        if (it == s->pending.begin() && r->bypassed >= MAX_BYPASS) return;
        ++it;
    }
}

void complete(ehs_server* s, Slot* sl, Req* r, int code, double gpu_ms)
{
    std::lock_guard<std::mutex> lk(s->mu);
    r->code = code;
    r->gpu_ms = gpu_ms;
    r->state = REQ_DONE;
    r->t_done = s->now_ms();
    s->arena.release(r->ws_off, r->ws_bytes);
    for (Unit* u : r->units) {
        u->refs--;
        // a unit whose production failed left the cache when the failure was
        // recorded; its memory goes back once no admitted request holds it
        if (u->failed && u->refs == 0) destroy_unit(s, u);
    }
    r->units.clear();
    r->produce.clear();
    sl->job = nullptr;
    s->running--;
    if (code == EHS_OK)
        s->completed++;
    else
        s->failed++;
    try_admit(s);
    s->cv_done.notify_all();
}

int run_job(ehs_server* s, Slot* sl, Req* r)
{
    ehs_ctx* c = &sl->ctx;
    hipStream_t st = sl->st;
    c->ws = s->mem + r->ws_off;
    c->ws_bytes = r->ws_bytes;
    Plan& p = r->plan;
    int code = EHS_OK;
    if (hipEventRecord(sl->e0, st) != hipSuccess) code = EHS_EHIP;
    // 1. produce the octants this request allocated, then publish them
    for (Unit* u : r->produce) {
        if (code == EHS_OK) {
            if (!u->f32) {
                if (s->fail_productions.load() > 0 && s->fail_productions.fetch_sub(1) > 0) code = EHS_EHIP;
                if (code == EHS_OK)
                    code = precompute_octant(c, p, u->kind, reinterpret_cast<double*>(s->mem + u->off), st);
            } else {
                Unit* src = nullptr;
                for (Unit* v : r->units)
                    if (!v->f32 && v->kind == u->kind) src = v;
                bool own = std::find(r->produce.begin(), r->produce.end(), src) != r->produce.end();
                if (!own && src) {
                    std::unique_lock<std::mutex> lk(s->mu);
                    s->cv_units.wait(lk, [&] { return src->recorded; });
                    if (src->failed) code = EHS_EHIP;
                }
                if (!src) code = EHS_EHIP;
                if (code == EHS_OK && !own && hipStreamWaitEvent(st, src->ready, 0) != hipSuccess) code = EHS_EHIP;
                if (code == EHS_OK &&
                    launch_oct_to_f32(reinterpret_cast<const double*>(s->mem + src->off),
                                      reinterpret_cast<float*>(s->mem + u->off), octant_elems(p.Mt), st) != hipSuccess)
                    code = EHS_EHIP;
            }
        }
        if (code == EHS_OK && hipEventRecord(u->ready, st) != hipSuccess) code = EHS_EHIP;
        std::lock_guard<std::mutex> lk(s->mu);
        u->recorded = true;
        u->failed = code != EHS_OK;
        if (u->failed) {
            // out of the cache at once: the next request that needs this
            // array allocates and produces it again
            auto it = s->units.find(unit_key(u->Mt, u->kind, u->f32));
            if (it != s->units.end() && it->second == u) s->units.erase(it);
        }
        s->cv_units.notify_all();
    }
    // 2. wait (on the stream) for octants produced by other requests
    Octants o;
    for (Unit* u : r->units) {
        bool own = std::find(r->produce.begin(), r->produce.end(), u) != r->produce.end();
        if (!own) {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_units.wait(lk, [&] { return u->recorded; });
            if (u->failed) code = EHS_EHIP;
            lk.unlock();
            if (code == EHS_OK && hipStreamWaitEvent(st, u->ready, 0) != hipSuccess) code = EHS_EHIP;
        }
        void* ptr = s->mem + u->off;
        if (u->kind == 0) {
            if (u->f32)
                o.H32 = static_cast<float*>(ptr);
            else
                o.H64 = static_cast<double*>(ptr);
        } else {
            if (u->f32)
                o.B32 = static_cast<float*>(ptr);
            else
                o.B64 = static_cast<double*>(ptr);
        }
    }
    // 3. the evaluation
    if (code == EHS_OK) code = execute(c, p, o, r->r.sources, r->r.strengths, r->r.targets, r->r.u_out, st);
    if (hipEventRecord(sl->e1, st) != hipSuccess && code == EHS_OK) code = EHS_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess && code == EHS_OK) code = EHS_EHIP;
    float ms = 0.f;
    if (code == EHS_OK) hipEventElapsedTime(&ms, sl->e0, sl->e1);
    r->gpu_ms = ms;
    c->ws = nullptr;
    c->ws_bytes = 0;
    return code;
}

void worker(ehs_server* s, Slot* sl)
{
    hipSetDevice(s->device);
    for (;;) {
        Req* r = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            sl->cv.wait(lk, [&] { return s->stop || sl->job != nullptr; });
            if (!sl->job) return;  // stop with nothing assigned
            r = sl->job;
        }
        int code = run_job(s, sl, r);
        complete(s, sl, r, code, r->gpu_ms);
    }
}

void server_free(ehs_server* s)
{
    hipSetDevice(s->device);
    for (Slot* sl : s->slots) {
        if (sl->e0) hipEventDestroy(sl->e0);
        if (sl->e1) hipEventDestroy(sl->e1);
        if (sl->st) hipStreamDestroy(sl->st);
        sl->ctx.ws = nullptr;
        ctx_release(&sl->ctx);
        delete sl;
    }
    s->slots.clear();
    while (!s->units.empty()) {
        Unit* u = s->units.begin()->second;
        if (u->ready) hipEventDestroy(u->ready);
        delete u;
        s->units.erase(s->units.begin());
    }
    for (auto& kv : s->reqs) delete kv.second;
    s->reqs.clear();
    ctx_release(&s->admin);
    if (s->admin_st) hipStreamDestroy(s->admin_st);
    free_tables(&s->tables);
    if (s->mem) hipFree(s->mem);
    delete s;
}

}  // namespace

extern "C" {

int ehs_server_create(ehs_server** out, int hip_device, size_t arena_bytes, int nslots)
{
    if (!out) return EHS_EINVAL;
    *out = nullptr;
    if (nslots < 1 || nslots > 16 || arena_bytes < ARENA_ALIGN) return EHS_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return EHS_EINVAL;
    if (hipSetDevice(hip_device) != hipSuccess) return EHS_EHIP;
    ehs_server* s = new (std::nothrow) ehs_server();
    if (!s) return EHS_ENOMEM;
    s->device = hip_device;
    s->t0 = Clock::now();
    s->arena.init(arena_bytes);
    int rc = EHS_OK;
    if (hipMalloc((void**)&s->mem, s->arena.cap) != hipSuccess) {
        s->mem = nullptr;
        hipGetLastError();
        rc = EHS_ENOMEM;
    }
    if (!rc) rc = ctx_init(&s->admin, hip_device, &s->tables);
    if (!rc && hipStreamCreateWithFlags(&s->admin_st, hipStreamNonBlocking) != hipSuccess) rc = EHS_EHIP;
    for (int i = 0; !rc && i < nslots; ++i) {
        Slot* sl = new (std::nothrow) Slot();
        if (!sl) {
            rc = EHS_ENOMEM;
            break;
        }
        s->slots.push_back(sl);
        rc = ctx_init(&sl->ctx, hip_device, &s->tables);
        sl->ctx.ws_external = true;
        if (!rc && (hipStreamCreateWithFlags(&sl->st, hipStreamNonBlocking) != hipSuccess ||
                    hipEventCreate(&sl->e0) != hipSuccess || hipEventCreate(&sl->e1) != hipSuccess))
            rc = EHS_EHIP;
    }
    if (rc) {
        server_free(s);
        return rc;
    }
    for (Slot* sl : s->slots) sl->th = std::thread(worker, s, sl);
    *out = s;
    return EHS_OK;
}

void ehs_server_destroy(ehs_server* s)
{
    if (!s) return;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] { return s->pending.empty() && s->running == 0; });
        s->stop = true;
        for (Slot* sl : s->slots) sl->cv.notify_all();
    }
    for (Slot* sl : s->slots)
        if (sl->th.joinable()) sl->th.join();
    server_free(s);
}

int ehs_submit(ehs_server* s, const ehs_request* rq, uint64_t* ticket)
{
    if (!s || !rq || !ticket) return EHS_EINVAL;
    *ticket = 0;
    if (rq->T > 0 && !rq->u_out) return EHS_EINVAL;
    Req* r = new (std::nothrow) Req();
    if (!r) return EHS_ENOMEM;
    r->r = *rq;
    r->t_submit = s->now_ms();
    int rc;
    {
        std::lock_guard<std::mutex> lk(s->admin_mu);
        if (hipSetDevice(s->device) != hipSuccess) {
            delete r;
            return EHS_EHIP;
        }
        rc = plan_request(&s->admin, rq->family, rq->sources, rq->strengths, rq->N, rq->targets, rq->T, rq->xi,
                          rq->r_c, rq->tol, rq->precision, s->admin_st, &r->plan);
    }
    if (!rc && rq->T > 0) rc = plan_workspace(r->plan, &r->ws_bytes);
    if (!rc && rq->T > 0) {
        std::vector<long long> keys;
        needed_units(r->plan, keys);
        size_t need = Arena::round(r->ws_bytes);
        for (long long k : keys) need += Arena::round(unit_bytes(r->plan.Mt, (k % 2) != 0));
        r->footprint = need;
        if (need > s->arena.cap) rc = EHS_ENOMEM;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (rc) {
        s->rejected++;
        delete r;
        return rc;
    }
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    s->reqs[r->ticket] = r;
    s->submitted++;
    if (rq->T == 0) {
        r->state = REQ_DONE;
        r->t_admit = r->t_done = r->t_submit;
        s->completed++;
        s->cv_done.notify_all();
        return EHS_OK;
    }
    s->pending.push_back(r);
    try_admit(s);
    return EHS_OK;
}

int ehs_wait(ehs_server* s, uint64_t ticket, int timeout_ms, ehs_request_status* status)
{
    if (!s) return EHS_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return EHS_EINVAL;
    Req* r = it->second;
    auto done = [&] { return r->state == REQ_DONE; };
    if (timeout_ms < 0)
        s->cv_done.wait(lk, done);
    else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done))
        return EHS_ETIMEDOUT;
    if (status) {
        std::memset(status, 0, sizeof(*status));
        status->code = r->code;
        status->slot = r->slot;
        status->t_submit_ms = r->t_submit;
        status->t_admit_ms = r->t_admit;
        status->t_done_ms = r->t_done;
        status->gpu_ms = r->gpu_ms;
        status->footprint_bytes = (double)r->footprint;
        fill_report(r->plan, &status->report);
        status->report.workspace_bytes = (double)r->ws_bytes;
    }
    int code = r->code;
    s->reqs.erase(it);
    delete r;
    return code;
}

int ehs_server_set_option(ehs_server* s, int option, double value)
{
    if (!s) return EHS_EINVAL;
    if (option == EHS_OPT_FAIL_PRECOMPUTE) {
        s->fail_productions.store(std::max(0, (int)value));
        return EHS_OK;
    }
    if (option == EHS_OPT_ADMISSION) {
        if (value != 0 && value != 1) return EHS_EINVAL;
        std::lock_guard<std::mutex> lk(s->mu);
        s->admission = (int)value;
        try_admit(s);
        return EHS_OK;
    }
    return EHS_EINVAL;
}

int ehs_server_stats(ehs_server* s, ehs_serve_stats* out)
{
    if (!s || !out) return EHS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->failed = s->failed;
    out->rejected = s->rejected;
    out->queued = (int32_t)s->pending.size();
    out->running = s->running;
    out->nslots = (int32_t)s->slots.size();
    out->cache_entries = (int32_t)s->units.size();
    out->cache_hits = s->hits;
    out->cache_misses = s->misses;
    out->evictions = s->evictions;
    out->arena_bytes = (double)s->arena.cap;
    out->arena_used = (double)s->arena.used;
    out->arena_peak = (double)s->arena.peak;
    out->cache_bytes = (double)s->cache_bytes;
    return EHS_OK;
}

}  // extern "C"
