// sf_api.hip -- the C ABI of libsfgrav.so: argument checks, handle life
// cycle, path selection.  Every entry point returns an sf_status; nothing
// here aborts or prints.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "sf_build.h"
#include "sf_prims.h"

namespace {
thread_local char g_msg[512] = "";
}

sf_status sf_fail(sf_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
    return st;
}

namespace sf {

// Device memory cache.  Every build and call allocates and frees a few
// dozen arrays; the runtime's stream-ordered allocator costs tens of
// microseconds per call, which adds up to milliseconds per force evaluation.
// Freed blocks are kept here by (size class, device, stream) and handed out
// again in stream order, so reuse on the same stream needs no
// synchronisation.  Blocks of another stream are never reused.
namespace {
struct BlockKey {
    size_t bytes;
    int dev;
    hipStream_t s;
    bool operator<(const BlockKey &o) const {
        if (bytes != o.bytes) return bytes < o.bytes;
        if (dev != o.dev) return dev < o.dev;
        return (uintptr_t)s < (uintptr_t)o.s;
    }
};
struct LiveBlock {
    size_t bytes;
    int dev;
};
std::mutex g_mu;
std::multimap<BlockKey, void *> g_free;
std::unordered_map<void *, LiveBlock> g_live;
size_t g_cached_bytes = 0;
const size_t kCacheLimit = size_t(64) << 30;   // keep at most 64 GiB cached

size_t size_class(size_t b) {
    if (b < 256) return 256;
    size_t c = 256;
    while (c < b) c <<= 1;
    return c;
}
}  // namespace

void cache_release(void *p, hipStream_t s) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) {
        (void)hipFreeAsync(p, s);
        return;
    }
    const LiveBlock lb = it->second;
    g_live.erase(it);
    if (g_cached_bytes + lb.bytes > kCacheLimit) {
        (void)hipFreeAsync(p, s);
        return;
    }
    g_free.emplace(BlockKey{lb.bytes, lb.dev, s}, p);
    g_cached_bytes += lb.bytes;
}

// Allocation-failure injection (test hook): with SF_GRAV_FAIL_ALLOC=k in the
// environment, the k-th device allocation of each entry-point call fails.
namespace {
thread_local long t_alloc_count = 0;
thread_local long t_fail_at = 0;
}  // namespace

void fail_alloc_arm() {
    const char *e = getenv("SF_GRAV_FAIL_ALLOC");
    t_fail_at = e ? atol(e) : 0;
    t_alloc_count = 0;
}

sf_status DevArena::alloc(void **p, size_t bytes, bool temp) {
    *p = nullptr;
    if (fixed) {   // bump mode: no HIP allocation, nothing to release
        const size_t off = (fixed_used + 255) & ~(size_t)255;
        if (off > fixed_cap || bytes > fixed_cap - off)
            return sf_fail(SF_E_INTERNAL, "fixed scratch of %zu bytes exhausted (%zu more needed)",
                           fixed_cap, off + bytes - fixed_cap);
        *p = fixed + off;
        fixed_used = off + bytes;
        return SF_OK;
    }
    if (t_fail_at > 0 && ++t_alloc_count == t_fail_at)
        return sf_fail(SF_E_NOMEM, "device allocation %ld of this call failed (SF_GRAV_FAIL_ALLOC)",
                       t_alloc_count);
    const size_t cls = size_class(bytes);
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_free.find(BlockKey{cls, dev, s});
        if (it != g_free.end()) {
            *p = it->second;
            g_free.erase(it);
            g_cached_bytes -= cls;
            g_live[*p] = LiveBlock{cls, dev};
        }
    }
    if (!*p) {
        hipError_t e = hipMallocAsync(p, cls, s);
        if (e != hipSuccess || *p == nullptr) {
            (void)hipGetLastError();
            *p = nullptr;
            return sf_fail(SF_E_NOMEM, "device allocation of %zu bytes failed: %s", bytes,
                           hipGetErrorString(e));
        }
        std::lock_guard<std::mutex> lk(g_mu);
        g_live[*p] = LiveBlock{cls, dev};
    }
    (temp ? tmp : keep).push_back(*p);
    return SF_OK;
}

void DevArena::free_tmp() {
    for (void *p : tmp) cache_release(p, s);
    tmp.clear();
}

void DevArena::free_keep() {
    for (void *p : keep) cache_release(p, s);
    keep.clear();
}

// Return every cached block to HIP (after the devices that own them have
// finished their work) and trim the devices' default memory pools; report
// the bytes still handed out (held by live handles or running calls).
sf_status release_cache(size_t *live_bytes) {
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return sf_fail(SF_E_DEVICE, "hipGetDevice failed");
    bool used[64] = {};
    for (auto &kv : g_free)
        if (kv.first.dev >= 0 && kv.first.dev < 64) used[kv.first.dev] = true;
    sf_status st = SF_OK;
    for (int d = 0; d < 64; ++d) {
        if (!used[d]) continue;
        if (hipSetDevice(d) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
            st = sf_fail(SF_E_DEVICE, "synchronising device %d failed", d);
            continue;
        }
        for (auto it = g_free.begin(); it != g_free.end();) {
            if (it->first.dev != d) {
                ++it;
                continue;
            }
            (void)hipFreeAsync(it->second, nullptr);
            g_cached_bytes -= it->first.bytes;
            it = g_free.erase(it);
        }
        (void)hipDeviceSynchronize();
        hipMemPool_t pool = nullptr;
        if (hipDeviceGetDefaultMemPool(&pool, d) == hipSuccess && pool)
            (void)hipMemPoolTrimTo(pool, 0);
    }
    (void)hipSetDevice(cur);
    (void)hipGetLastError();
    size_t live = 0;
    for (auto &kv : g_live) live += kv.second.bytes;
    if (live_bytes) *live_bytes = live;
    return st;
}

// hipEvents for the phase timers, reused across handles.
static std::mutex g_ev_mu;
static std::vector<hipEvent_t> g_events;

static hipEvent_t event_get() {
    {
        std::lock_guard<std::mutex> lk(g_ev_mu);
        if (!g_events.empty()) {
            hipEvent_t e = g_events.back();
            g_events.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static void event_put(hipEvent_t e) {
    if (!e) return;
    std::lock_guard<std::mutex> lk(g_ev_mu);
    g_events.push_back(e);
}

void phase_begin(sf_grav_tree_s *t, int ph, hipStream_t st) {
    if (!t->timing) return;
    if (!t->ev0[ph]) {
        t->ev0[ph] = event_get();
        t->ev1[ph] = event_get();
        if (!t->ev0[ph] || !t->ev1[ph]) {
            event_put(t->ev0[ph]);
            event_put(t->ev1[ph]);
            t->ev0[ph] = t->ev1[ph] = nullptr;
            return;
        }
    }
    (void)hipEventRecord(t->ev0[ph], st ? st : t->stream);
}

void phase_end(sf_grav_tree_s *t, int ph, hipStream_t st) {
    if (!t->timing || !t->ev0[ph]) return;
    (void)hipEventRecord(t->ev1[ph], st ? st : t->stream);
    t->ev_used[ph] = true;
}

// One side stream per device, created on first use (default priority,
// non-blocking) and kept until the process ends.
static std::mutex g_side_mu;
static hipStream_t g_side[64] = {};

hipStream_t side_stream(int device) {
    if (device < 0 || device >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_side_mu);
    if (!g_side[device]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) return nullptr;
        if (cur != device && hipSetDevice(device) != hipSuccess) return nullptr;
        hipStream_t st = nullptr;
        const hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_side[device] = st;
    }
    return g_side[device];
}

static sf_status ensure_event(hipEvent_t *e) {
    if (*e) return SF_OK;
    if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        *e = nullptr;
        return sf_fail(SF_E_INTERNAL, "hipEventCreateWithFlags failed");
    }
    return SF_OK;
}

sf_status side_fork(sf_grav_tree_s *t, hipStream_t side) {
    if (side == t->stream) return SF_OK;
    // both events exist before anything is queued on the side stream, so the
    // join cannot fail for want of an event
    sf_status st = ensure_event(&t->ev_fork);
    if (st == SF_OK) st = ensure_event(&t->ev_join);
    if (st != SF_OK) return st;
    SF_HIP(hipEventRecord(t->ev_fork, t->stream));
    SF_HIP(hipStreamWaitEvent(side, t->ev_fork, 0));
    return SF_OK;
}

sf_status side_join(sf_grav_tree_s *t, hipStream_t side) {
    if (side == t->stream) return SF_OK;
    hipError_t e = hipEventRecord(t->ev_join, side);
    if (e == hipSuccess) e = hipStreamWaitEvent(t->stream, t->ev_join, 0);
    if (e != hipSuccess) {
        // the caller's stream cannot wait for the side work: finish it here,
        // before the caller releases the scratch it uses
        (void)hipGetLastError();
        (void)hipStreamSynchronize(side);
        return sf_fail(SF_E_DEVICE, "joining the side stream failed: %s", hipGetErrorString(e));
    }
    return SF_OK;
}

static void phase_reset(sf_grav_tree_s *t, int lo, int hi) {
    for (int p = lo; p < hi; ++p) t->ev_used[p] = false;
}

}  // namespace sf

using sf::DevArena;

static sf_status check_opts(const sf_grav_opts *o, int64_t n, bool need_tree_caps) {
    if (!o) return sf_fail(SF_E_INVALID, "opts is NULL");
    if (o->struct_size != sizeof(sf_grav_opts))
        return sf_fail(SF_E_INVALID, "opts.struct_size %u != %zu", o->struct_size, sizeof(sf_grav_opts));
    if (o->form != SF_FP32C && o->form != SF_FP32 && o->form != SF_FP64)
        return sf_fail(SF_E_INVALID, "opts.form %d unknown", o->form);
    if (!(o->theta >= 0.0) || !(o->theta < 1e30))
        return sf_fail(SF_E_INVALID, "opts.theta must be finite and >= 0");
    if (o->order != 0 && o->order != 2) return sf_fail(SF_E_INVALID, "opts.order must be 0 or 2");
    if (need_tree_caps) {
        if (o->leaf_cap < 1 || o->leaf_cap > 64)
            return sf_fail(SF_E_INVALID, "opts.leaf_cap must be in [1, 64]");
        if (o->group_cap < 1 || o->group_cap > 64)
            return sf_fail(SF_E_INVALID, "opts.group_cap must be in [1, 64]");
    }
    if (!(o->G == o->G) || o->G > 1e300 || o->G < -1e300)
        return sf_fail(SF_E_INVALID, "opts.G must be finite");
    if (o->alpha != o->alpha) return sf_fail(SF_E_INVALID, "opts.alpha is NaN");
    const int64_t ng = o->n_gas < 0 ? n : o->n_gas;
    if (ng > n) return sf_fail(SF_E_INVALID, "opts.n_gas %lld > n %lld", (long long)ng, (long long)n);
    return SF_OK;
}

static const int64_t kMaxN = 1ll << 25;

static sf_status check_arrays(const void *pos, const void *mass, const void *soft, int64_t n,
                              sf_dtype dt) {
    if (dt != SF_F32 && dt != SF_F64) return sf_fail(SF_E_INVALID, "dtype %d unknown", (int)dt);
    if (n < 1) return sf_fail(SF_E_INVALID, "n must be >= 1 (got %lld)", (long long)n);
    if (n > kMaxN)
        return sf_fail(SF_E_UNSUPPORTED, "n = %lld exceeds the supported maximum %lld",
                       (long long)n, (long long)kMaxN);
    if (!pos || !mass || !soft) return sf_fail(SF_E_INVALID, "pos, mass and soft must be non-NULL");
    return SF_OK;
}

static void free_handle_memory(sf_grav_tree_s *t) {
    if (!t) return;
    (void)hipStreamSynchronize(t->stream);
    for (void *p : t->allocs) sf::cache_release(p, t->stream);
    t->allocs.clear();
    for (int p = 0; p < sf_grav_tree_s::kPhases; ++p) {
        sf::event_put(t->ev0[p]);
        sf::event_put(t->ev1[p]);
        t->ev0[p] = t->ev1[p] = nullptr;
    }
    if (t->ev_fork) (void)hipEventDestroy(t->ev_fork);
    if (t->ev_join) (void)hipEventDestroy(t->ev_join);
    t->ev_fork = t->ev_join = nullptr;
}

extern "C" {

void sf_grav_opts_default(sf_grav_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(sf_grav_opts);
    o->form = SF_FP32C;
    o->G = 1.0;
    o->theta = 0.5;
    o->order = 2;
    o->leaf_cap = 32;
    o->group_cap = 32;
    o->validate = 0;
    o->n_gas = -1;
    o->collect_stats = 0;
    o->timing = 0;
    o->alpha = -1.0;
}

const char *sf_grav_strerror(sf_status s) {
    switch (s) {
        case SF_OK: return "ok";
        case SF_E_INVALID: return "invalid argument";
        case SF_E_NOMEM: return "out of memory";
        case SF_E_DEVICE: return "device error";
        case SF_E_STATE: return "handle does not match the call";
        case SF_E_UNSUPPORTED: return "unsupported";
        case SF_E_INTERNAL: return "internal capacity exceeded";
    }
    return "unknown status";
}

const char *sf_grav_last_error(void) { return g_msg; }

// Build everything for the tree path into a fresh handle.
static sf_status build_all(sf_grav_tree_s *t, const void *pos, const void *mass, const void *soft,
                           const sf_grav_opts *o, DevArena &ar) {
    t->timing = o->timing != 0;
    sf::phase_reset(t, 0, sf_grav_tree_s::kPhases);
    sf::phase_begin(t, 0);
    sf_status st = sf::build_sorted(pos, mass, soft, t->n, t->n_gas, t->dt, false, o->validate != 0,
                                    t, ar);
    if (st != SF_OK) return st;
    sf::phase_end(t, 0);
    SF_HIP(hipMemcpyAsync(&t->hframe, t->frame, sizeof(sf::Frame), hipMemcpyDeviceToHost, t->stream));
    sf::phase_begin(t, 1);
    st = sf::build_topology(t, ar);   // synchronises the stream once
    if (st != SF_OK) return st;
    sf::phase_end(t, 1);
    if (o->validate && t->hframe.bad)
        return sf_fail(SF_E_INVALID, "inputs contain non-finite values, h <= 0 or m < 0");
    if (t->n_nodes >= (1ll << 27))
        return sf_fail(SF_E_UNSUPPORTED, "tree has %lld nodes (limit 2^27)", (long long)t->n_nodes);
    sf::phase_begin(t, 2);
    st = sf::build_moments(t, ar, false);
    if (st != SF_OK) return st;
    sf::phase_end(t, 2);
    sf::phase_begin(t, 3);
    st = sf::build_groups(t, ar);
    sf::phase_end(t, 3);
    return st;
}

sf_status sf_grav_build_tree(const void *pos, const void *mass, const void *soft, int64_t n,
                             sf_dtype dt, const sf_grav_opts *o, void *stream, sf_grav_tree *out) {
    g_msg[0] = 0;
    if (!out) return sf_fail(SF_E_INVALID, "out is NULL");
    *out = nullptr;
    sf_status st = check_arrays(pos, mass, soft, n, dt);
    if (st != SF_OK) return st;
    st = check_opts(o, n, true);
    if (st != SF_OK) return st;
    sf::fail_alloc_arm();
    sf_grav_tree_s *t = new (std::nothrow) sf_grav_tree_s();
    if (!t) return sf_fail(SF_E_NOMEM, "host allocation failed");
    t->stream = (hipStream_t)stream;
    t->n = n;
    t->n_gas = o->n_gas < 0 ? n : o->n_gas;
    t->n_sink = n - t->n_gas;
    t->dt = dt;
    t->leaf_cap = o->leaf_cap;
    t->group_cap = o->group_cap;
    hipGetDevice(&t->device);
    {
        DevArena ar(t->stream);
        st = build_all(t, pos, mass, soft, o, ar);
        if (st != SF_OK) {
            (void)hipStreamSynchronize(t->stream);
            ar.free_keep();
            ar.free_tmp();
            for (int p = 0; p < sf_grav_tree_s::kPhases; ++p) {
                sf::event_put(t->ev0[p]);
                sf::event_put(t->ev1[p]);
            }
            delete t;
            return st;
        }
        t->allocs.insert(t->allocs.end(), ar.keep.begin(), ar.keep.end());
        ar.keep.clear();
    }
    *out = t;
    return SF_OK;
}

static sf_status eval_opts(const sf_grav_opts *o, sf::EvalOpts &e) {
    e.form = o->form;
    e.order = o->order;
    e.G = o->G;
    e.theta = o->theta;
    e.alpha = o->alpha;
    e.stats = o->collect_stats != 0;
    return SF_OK;
}

// The relative criterion needs a previous field on the handle.
static sf_status check_field(const sf_grav_tree_s *t, const sf_grav_opts *o) {
    if (o->alpha >= 0.0 && !t->have_field)
        return sf_fail(SF_E_STATE,
                       "opts.alpha >= 0 needs a previous field: call sf_grav_tree_set_field first");
    return SF_OK;
}

// Direct paths with validate = 1: read the flag the input pass raised
// (synchronises the stream once).
static sf_status validation_result(const sf_grav_tree_s &t) {
    sf::Frame hf;
    hipError_t he = hipMemcpyAsync(&hf, t.frame, sizeof(hf), hipMemcpyDeviceToHost, t.stream);
    if (he == hipSuccess) he = hipStreamSynchronize(t.stream);
    if (he != hipSuccess) return sf_fail(SF_E_DEVICE, "%s", hipGetErrorString(he));
    if (hf.bad) return sf_fail(SF_E_INVALID, "inputs contain non-finite values, h <= 0 or m < 0");
    return SF_OK;
}

sf_status sf_grav_accel(sf_grav_tree tree, const void *pos, const void *mass, const void *soft,
                        int64_t n, sf_dtype dt, const sf_grav_opts *o, void *acc, void *pot,
                        void *stream) {
    g_msg[0] = 0;
    if (!acc) return sf_fail(SF_E_INVALID, "acc is NULL");
    sf::EvalOpts e;
    if (tree) {
        sf_status st = check_opts(o, n, false);
        if (st != SF_OK) return st;
        if (tree->direct_only) return sf_fail(SF_E_STATE, "handle has no tree");
        if (n != tree->n || dt != tree->dt)
            return sf_fail(SF_E_STATE, "n/dtype (%lld, %d) differ from the handle's (%lld, %d)",
                           (long long)n, (int)dt, (long long)tree->n, (int)tree->dt);
        st = check_field(tree, o);
        if (st != SF_OK) return st;
        sf::fail_alloc_arm();
        eval_opts(o, e);
        hipStream_t prev = tree->stream;
        tree->stream = (hipStream_t)stream;
        tree->timing = o->timing != 0;
        sf::phase_reset(tree, 4, 7);
        DevArena ar(tree->stream);
        st = sf::tree_accel(tree, e, acc, pot, ar);
        if (st != SF_OK) {
            tree->stream = prev;
            return st;
        }
        return SF_OK;
    }
    sf_status st = check_arrays(pos, mass, soft, n, dt);
    if (st != SF_OK) return st;
    st = check_opts(o, n, false);
    if (st != SF_OK) return st;
    eval_opts(o, e);
    sf::fail_alloc_arm();
    sf_grav_tree_s t;
    t.stream = (hipStream_t)stream;
    t.direct_only = true;
    {
        DevArena ar(t.stream);
        const int64_t ng = o->n_gas < 0 ? n : o->n_gas;
        st = sf::build_sorted(pos, mass, soft, n, ng, dt, true, o->validate != 0, &t, ar);
        if (st == SF_OK && o->validate) st = validation_result(t);
        if (st == SF_OK) st = sf::direct_accel(&t, e, acc, pot, ar);
        // the handle's own arrays are released once the stream reaches here
        ar.free_keep();
    }
    return st;
}

sf_status sf_grav_accel_backward(sf_grav_tree tree, const void *pos, const void *mass,
                                 const void *soft, int64_t n, sf_dtype dt, const sf_grav_opts *o,
                                 const void *g_acc, const void *g_pot, void *g_pos, void *g_mass,
                                 void *g_soft, void *stream) {
    g_msg[0] = 0;
    if (!g_acc) return sf_fail(SF_E_INVALID, "g_acc is NULL");
    sf::EvalOpts e;
    if (tree) {
        sf_status st = check_opts(o, n, false);
        if (st != SF_OK) return st;
        if (tree->direct_only) return sf_fail(SF_E_STATE, "handle has no tree");
        if (n != tree->n || dt != tree->dt)
            return sf_fail(SF_E_STATE, "n/dtype differ from the handle's");
        st = check_field(tree, o);
        if (st != SF_OK) return st;
        sf::fail_alloc_arm();
        eval_opts(o, e);
        tree->stream = (hipStream_t)stream;
        tree->timing = o->timing != 0;
        sf::phase_reset(tree, 7, 11);
        DevArena ar(tree->stream);
        return sf::tree_backward(tree, e, g_acc, g_pot, g_pos, g_mass, g_soft, ar);
    }
    sf_status st = check_arrays(pos, mass, soft, n, dt);
    if (st != SF_OK) return st;
    st = check_opts(o, n, false);
    if (st != SF_OK) return st;
    eval_opts(o, e);
    sf::fail_alloc_arm();
    sf_grav_tree_s t;
    t.stream = (hipStream_t)stream;
    t.direct_only = true;
    {
        DevArena ar(t.stream);
        const int64_t ng = o->n_gas < 0 ? n : o->n_gas;
        st = sf::build_sorted(pos, mass, soft, n, ng, dt, true, o->validate != 0, &t, ar);
        if (st == SF_OK && o->validate) st = validation_result(t);
        if (st == SF_OK) st = sf::direct_backward(&t, e, g_acc, g_pot, g_pos, g_mass, g_soft, ar);
        ar.free_keep();
    }
    return st;
}

sf_status sf_grav_get_timings(sf_grav_tree t, sf_grav_timings *out) {
    g_msg[0] = 0;
    if (!t || !out) return sf_fail(SF_E_INVALID, "NULL argument");
    if (out->struct_size != sizeof(sf_grav_timings))
        return sf_fail(SF_E_INVALID, "timings.struct_size mismatch");
    out->n_phases = sf_grav_tree_s::kPhases;
    for (int p = 0; p < 16; ++p) out->ms[p] = -1.0;
    for (int p = 0; p < sf_grav_tree_s::kPhases; ++p) {
        if (!t->ev_used[p]) continue;
        SF_HIP(hipEventSynchronize(t->ev1[p]));
        float ms = 0.f;
        SF_HIP(hipEventElapsedTime(&ms, t->ev0[p], t->ev1[p]));
        out->ms[p] = ms;
    }
    return SF_OK;
}

sf_status sf_grav_tree_free(sf_grav_tree tree) {
    if (!tree) return SF_OK;
    free_handle_memory(tree);
    delete tree;
    return SF_OK;
}

sf_status sf_grav_get_tree_info(sf_grav_tree t, sf_grav_tree_info *info) {
    g_msg[0] = 0;
    if (!t || !info) return sf_fail(SF_E_INVALID, "NULL argument");
    if (info->struct_size != sizeof(sf_grav_tree_info))
        return sf_fail(SF_E_INVALID, "info.struct_size mismatch");
    if (t->direct_only) return sf_fail(SF_E_STATE, "handle has no tree");
    uint32_t st[2] = {0, 0};
    int32_t ng = 0;
    SF_HIP(hipMemcpyAsync(st, t->info_dev, sizeof(st), hipMemcpyDeviceToHost, t->stream));
    SF_HIP(hipMemcpyAsync(&ng, t->n_groups_dev, sizeof(ng), hipMemcpyDeviceToHost, t->stream));
    SF_HIP(hipStreamSynchronize(t->stream));
    t->n_groups = ng;
    t->max_level = (int)st[0];
    t->n_leaves = st[1];
    info->max_level = t->max_level;
    info->n = t->n;
    info->n_gas = t->n_gas;
    info->n_nodes = t->n_nodes;
    info->n_groups = t->n_groups;
    info->n_leaves = t->n_leaves;
    return SF_OK;
}

sf_status sf_grav_tree_export(sf_grav_tree t, int32_t what, void *host_dst, size_t bytes) {
    g_msg[0] = 0;
    if (!t || !host_dst) return sf_fail(SF_E_INVALID, "NULL argument");
    if (t->direct_only) return sf_fail(SF_E_STATE, "handle has no tree");
    int32_t ng = 0;
    SF_HIP(hipMemcpyAsync(&ng, t->n_groups_dev, sizeof(ng), hipMemcpyDeviceToHost, t->stream));
    SF_HIP(hipStreamSynchronize(t->stream));
    t->n_groups = ng;
    const void *src = nullptr;
    size_t need = 0;
    const size_t nn = (size_t)t->n_nodes, n = (size_t)t->n, g = (size_t)ng;
    switch (what) {
        case SF_EXPORT_KEYS: src = t->keys; need = n * 8; break;
        case SF_EXPORT_ORDER: src = t->order; need = n * 4; break;
        case SF_EXPORT_NODE_LEVEL: src = t->nlevel; need = nn * 4; break;
        case SF_EXPORT_NODE_FIRST: src = t->nfirst; need = nn * 4; break;
        case SF_EXPORT_NODE_COUNT: src = t->ncount; need = nn * 4; break;
        case SF_EXPORT_NODE_PARENT: src = t->nparent; need = nn * 4; break;
        case SF_EXPORT_NODE_CHILD: src = t->nchild; need = nn * 4; break;
        case SF_EXPORT_NODE_NCHILD: src = t->nnchild; need = nn * 4; break;
        case SF_EXPORT_GROUP_FIRST: src = t->gfirst; need = g * 4; break;
        case SF_EXPORT_GROUP_COUNT: src = t->gcount; need = g * 4; break;
        case SF_EXPORT_NODE_MASS: src = t->M[0]; need = nn * 8; break;
        case SF_EXPORT_NODE_COM: src = t->com[0]; need = nn * 24; break;
        case SF_EXPORT_NODE_QUAD: src = t->Q[0]; need = nn * 48; break;
        case SF_EXPORT_GROUP_NPC:
        case SF_EXPORT_GROUP_NPP:
            if (!t->have_stats) return sf_fail(SF_E_STATE, "no statistics collected");
            src = what == SF_EXPORT_GROUP_NPC ? (const void *)t->gnpc : (const void *)t->gnpp;
            need = g * 4;
            break;
        case SF_EXPORT_GROUP_CKS:
            if (!t->have_stats) return sf_fail(SF_E_STATE, "no statistics collected");
            src = t->gcks;
            need = g * 8;
            break;
        default: return sf_fail(SF_E_INVALID, "unknown export id %d", what);
    }
    if (bytes != need)
        return sf_fail(SF_E_INVALID, "export %d needs %zu bytes, got %zu", what, need, bytes);
    if (need == 0) return SF_OK;
    SF_HIP(hipMemcpyAsync(host_dst, src, need, hipMemcpyDeviceToHost, t->stream));
    SF_HIP(hipStreamSynchronize(t->stream));
    return SF_OK;
}

sf_status sf_grav_accel_tidal(sf_grav_tree tree, const void *vel, const sf_grav_opts *o, void *acc,
                              void *pot, void *tidal, void *jerk, void *stream) {
    g_msg[0] = 0;
    if (!tree) return sf_fail(SF_E_UNSUPPORTED, "the tidal tensor needs a tree (theta = 0 gives "
                              "the all-pairs sum)");
    if (!acc) return sf_fail(SF_E_INVALID, "acc is NULL");
    if (jerk && !vel) return sf_fail(SF_E_INVALID, "the jerk needs velocities");
    sf_status st = check_opts(o, tree->n, false);
    if (st != SF_OK) return st;
    if (tree->direct_only) return sf_fail(SF_E_STATE, "handle has no tree");
    st = check_field(tree, o);
    if (st != SF_OK) return st;
    sf::fail_alloc_arm();
    sf::EvalOpts e;
    eval_opts(o, e);
    tree->stream = (hipStream_t)stream;
    DevArena ar(tree->stream);
    return sf::tidal_accel(tree, e, jerk ? vel : nullptr, acc, pot, tidal, jerk, ar);
}

sf_status sf_grav_accel_adaptive(sf_grav_tree tree, const sf_grav_opts *o, void *acc, void *pot,
                                 void *aux, void *stream) {
    g_msg[0] = 0;
    if (!tree) return sf_fail(SF_E_INVALID, "tree is NULL");
    if (!acc) return sf_fail(SF_E_INVALID, "acc is NULL");
    sf_status st = check_opts(o, tree->n, false);
    if (st != SF_OK) return st;
    if (tree->direct_only) return sf_fail(SF_E_STATE, "handle has no tree");
    st = check_field(tree, o);
    if (st != SF_OK) return st;
    sf::fail_alloc_arm();
    sf::EvalOpts e;
    eval_opts(o, e);
    tree->stream = (hipStream_t)stream;
    DevArena ar(tree->stream);
    return sf::adaptive_accel(tree, e, acc, pot, aux, ar);
}

sf_status sf_grav_rad_sums(sf_grav_tree tree, const void *lum, double c_light,
                           const sf_grav_opts *o, void *column, void *e_ir, void *stream) {
    g_msg[0] = 0;
    if (!tree) return sf_fail(SF_E_INVALID, "tree is NULL");
    if (!column && !e_ir) return sf_fail(SF_E_INVALID, "column and e_ir are both NULL");
    if (e_ir && !(c_light > 0.0)) return sf_fail(SF_E_INVALID, "c_light must be > 0");
    sf_status st = check_opts(o, tree->n, false);
    if (st != SF_OK) return st;
    if (tree->direct_only) return sf_fail(SF_E_STATE, "handle has no tree");
    st = check_field(tree, o);
    if (st != SF_OK) return st;
    sf::fail_alloc_arm();
    sf::EvalOpts e;
    eval_opts(o, e);
    tree->stream = (hipStream_t)stream;
    DevArena ar(tree->stream);
    return sf::rad_sums(tree, e, lum, c_light > 0.0 ? c_light : 1.0, column, e_ir, ar);
}

sf_status sf_grav_tree_set_field(sf_grav_tree t, const void *acc_prev, void *stream) {
    g_msg[0] = 0;
    if (!t || !acc_prev) return sf_fail(SF_E_INVALID, "NULL argument");
    if (t->direct_only) return sf_fail(SF_E_STATE, "handle has no tree");
    sf::fail_alloc_arm();
    t->stream = (hipStream_t)stream;
    return sf::set_field(t, acc_prev);
}

sf_status sf_grav_tree_refit(sf_grav_tree t, const void *pos, const void *mass, const void *soft,
                             void *stream) {
    g_msg[0] = 0;
    if (!t || !pos || !mass || !soft) return sf_fail(SF_E_INVALID, "NULL argument");
    if (t->direct_only) return sf_fail(SF_E_STATE, "handle has no tree");
    sf::fail_alloc_arm();
    t->stream = (hipStream_t)stream;
    DevArena ar(t->stream);
    return sf::refit(t, pos, mass, soft, ar);
}

sf_status sf_grav_get_stats(sf_grav_tree t, sf_grav_stats *out) {
    g_msg[0] = 0;
    if (!t || !out) return sf_fail(SF_E_INVALID, "NULL argument");
    if (out->struct_size != sizeof(sf_grav_stats))
        return sf_fail(SF_E_INVALID, "stats.struct_size mismatch");
    if (t->direct_only) return sf_fail(SF_E_STATE, "handle has no tree");
    if (!t->have_stats) return sf_fail(SF_E_STATE, "no statistics collected");
    return sf::tree_stats(t, out);
}

sf_status sf_grav_release_cache(size_t *live_bytes) {
    g_msg[0] = 0;
    return sf::release_cache(live_bytes);
}

}  // extern "C"
