// sf_build.h -- host-side pieces shared by the library's translation units:
// error reporting, a device-allocation arena and the build/eval entry points.
#pragma once
#include <vector>

#include "sf_internal.h"

// Record a failure message for sf_grav_last_error() and return the status.
sf_status sf_fail(sf_status st, const char *fmt, ...);

namespace sf {

// Stream-ordered device allocations.  `keep` allocations belong to a tree
// handle; `tmp` ones are released when the arena is destroyed (at the end of
// a call).  On failure every allocation made so far can be released.
// Bump mode (set_fixed): every allocation is carved, 256-byte aligned, out
// of one caller-supplied device region and nothing is ever released or
// allocated from HIP; running past the region's end is SF_E_INTERNAL.
struct DevArena {
    hipStream_t s = nullptr;
    std::vector<void *> keep, tmp;
    char *fixed = nullptr;
    size_t fixed_cap = 0, fixed_used = 0;
    explicit DevArena(hipStream_t st) : s(st) {}
    ~DevArena() { free_tmp(); }
    void set_fixed(void *base, size_t cap) {
        fixed = (char *)base;
        fixed_cap = cap;
        fixed_used = 0;
    }
    sf_status alloc(void **p, size_t bytes, bool temp);   // cached, stream ordered
    void free_tmp();
    void free_keep();
};

// Return a block from DevArena::alloc to the library's cache (stream ordered).
void cache_release(void *p, hipStream_t s);
// Give every cached block back to HIP; *live_bytes = bytes still handed out.
sf_status release_cache(size_t *live_bytes);
// Read SF_GRAV_FAIL_ALLOC and restart the per-call allocation count.
void fail_alloc_arm();

// Allocations that a call adds to an existing handle: released again unless
// committed to the handle.
struct HandleAlloc {
    DevArena ar;
    sf_grav_tree_s *t;
    explicit HandleAlloc(sf_grav_tree_s *tt) : ar(tt->stream), t(tt) {}
    ~HandleAlloc() { ar.free_keep(); }
    void commit() {
        t->allocs.insert(t->allocs.end(), ar.keep.begin(), ar.keep.end());
        ar.keep.clear();
    }
};

}  // namespace sf

#define SF_ALLOC(ar, p, count)                                                                  \
    do {                                                                                        \
        sf_status _st = (ar).alloc((void **)&(p), sizeof(*(p)) * (size_t)(count), false);     \
        if (_st != SF_OK) return _st;                                                           \
    } while (0)
#define SF_ALLOC_TMP(ar, p, count)                                                              \
    do {                                                                                        \
        sf_status _st = (ar).alloc((void **)&(p), sizeof(*(p)) * (size_t)(count), true);      \
        if (_st != SF_OK) return _st;                                                           \
    } while (0)
#define SF_HIP(expr)                                                                            \
    do {                                                                                        \
        hipError_t _e = (expr);                                                                 \
        if (_e != hipSuccess)                                                                   \
            return sf_fail(SF_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(_e));         \
    } while (0)

namespace sf {

// A1-A4: bounding box, keys, radix sort, sorted SoA, sink positions.
sf_status build_sorted(const void *pos, const void *mass, const void *soft, int64_t n,
                       int64_t n_gas, sf_dtype dt, bool type_major, bool validate,
                       sf_grav_tree_s *t, DevArena &ar);
sf_status build_topology(sf_grav_tree_s *t, DevArena &ar);   // A5 (one stream sync)
sf_status build_moments(sf_grav_tree_s *t, DevArena &ar, bool refit);   // A6
sf_status build_groups(sf_grav_tree_s *t, DevArena &ar);     // A7
sf_status group_boxes(sf_grav_tree_s *t);                    // A7: boxes of the built groups
// Frozen-topology refit: new pos/mass/soft, same keys, order, nodes, groups.
sf_status refit(sf_grav_tree_s *t, const void *pos, const void *mass, const void *soft,
                DevArena &ar);

struct EvalOpts {
    int form;
    int order;
    double G;
    double theta;
    double alpha;   // relative criterion tolerance; < 0: off
    bool stats;
};

// Store |g| of a previous field (caller order, handle dtype) for the
// relative criterion: per sorted particle and per group minimum.
sf_status set_field(sf_grav_tree_s *t, const void *acc_prev);
// Totals, list-length histogram and list checksum of the last walk with stats.
sf_status tree_stats(sf_grav_tree_s *t, sf_grav_stats *out);
struct WalkNodes;
void set_relative(WalkNodes &nd, const sf_grav_tree_s *t, const EvalOpts &o);

// A8-A10, A12: tree walk for gas targets, sink walk + FP64 sink-sink.  With
// groups false only the sinks' fields are written (the gas targets are left
// to another evaluator), and no statistics or costs are recorded.
sf_status tree_accel(sf_grav_tree_s *t, const EvalOpts &o, void *acc, void *pot, DevArena &ar,
                     bool groups = true);
// Tidal tensor and jerk (and g, phi) in one tree walk; vel may be NULL when
// jerk is NULL; pot/tid may be NULL.
sf_status tidal_accel(sf_grav_tree_s *t, const EvalOpts &o, const void *vel, void *acc, void *pot,
                      void *tid, void *jerk, DevArena &ar);
// Symmetrised adaptive gas-gas softening (two walks after the ordinary one);
// aux (Omega, zeta per particle, caller order) may be NULL.
sf_status adaptive_accel(sf_grav_tree_s *t, const EvalOpts &o, void *acc, void *pot, void *aux,
                         DevArena &ar);
// Tree-pass radiation sums for gas cells: 6-bin column densities and the IR
// energy density of the sinks' luminosities (lum may be NULL: no stars).
sf_status rad_sums(sf_grav_tree_s *t, const EvalOpts &o, const void *lum, double c_light,
                   void *col, void *eir, DevArena &ar);
// A11: direct path on a handle built with type-major keys (no topology).
sf_status direct_accel(sf_grav_tree_s *t, const EvalOpts &o, void *acc, void *pot, DevArena &ar);
// Bytes of one packed source record of the direct path in form `form`.
size_t direct_rec_bytes(int form);
// A13: adjoints.
sf_status tree_backward(sf_grav_tree_s *t, const EvalOpts &o, const void *g_acc,
                        const void *g_pot, void *g_pos, void *g_mass, void *g_soft,
                        DevArena &ar);
sf_status direct_backward(sf_grav_tree_s *t, const EvalOpts &o, const void *g_acc,
                          const void *g_pot, void *g_pos, void *g_mass, void *g_soft,
                          DevArena &ar);

// FP64 sink-sink direct sum into acc4 (4 doubles per sink: ax ay az phi),
// launched on stream st; rec is scratch for kSinkRec doubles per sink.
constexpr int kSinkRec = 6;
void sink_sink_accel(sf_grav_tree_s *t, double G, double *acc4, double *rec, hipStream_t st);

// Second stream of the device for the sink work, which runs beside the group
// walk: side_fork makes it wait for the work queued so far on t->stream,
// side_join makes t->stream wait for the work queued so far on it.
hipStream_t side_stream(int device);
sf_status side_fork(sf_grav_tree_s *t, hipStream_t side);
sf_status side_join(sf_grav_tree_s *t, hipStream_t side);

int device_cu_count();
int walk_grid();

// Phase timer helpers: no-ops unless t->timing.  Events go on st (t->stream
// when null).
void phase_begin(sf_grav_tree_s *t, int ph, hipStream_t st = nullptr);
void phase_end(sf_grav_tree_s *t, int ph, hipStream_t st = nullptr);

}  // namespace sf
