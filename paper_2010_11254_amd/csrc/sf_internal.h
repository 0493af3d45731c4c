// sf_internal.h -- device-side types and helpers shared by the kernels of
// libsfgrav.so (gfx950 only).  Nothing here is exported.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "sf_grav.h"

namespace sf {

constexpr int kLevels = 21;          // Morton levels: 21 bits per axis
constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kMaxGroup = 64;        // one target per lane

// Root cube of the octree: lo corner, side, quantisation scale 2^21/side.
struct Frame {
    double lo[3];
    double side;
    double scale;
    double hi[3];
    int32_t bad;      // validation: count of non-finite / h <= 0 / m < 0
    int32_t pad;
};
static_assert(sizeof(Frame) % 4 == 0, "Frame is cleared as 32-bit words");

// Status word of a decoupled look-back scan: 2 flag bits + 30-bit value.
constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagPre = 2u << 30;
constexpr uint32_t kValMask = (1u << 30) - 1;

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ double dsub(double a, double b) { return __dsub_rn(a, b); }
__device__ __forceinline__ double dadd(double a, double b) { return __dadd_rn(a, b); }
__device__ __forceinline__ double dmul(double a, double b) { return __dmul_rn(a, b); }

__device__ __forceinline__ uint64_t lane_mask_lt() {
    const int lane = threadIdx.x & (kWave - 1);
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ int popc64(uint64_t v) { return __popcll(v); }

// Common leading octal digits of two 63-bit keys (21 if equal).
__device__ __forceinline__ int lcp_digits(uint64_t a, uint64_t b) {
    uint64_t x = a ^ b;
    if (x == 0) return kLevels;
    return (__clzll(x) - 1) / 3;
}

// Spread the low 21 bits of v so that bit k lands at bit 3k.
__host__ __device__ __forceinline__ uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x001f00000000ffffull;
    v = (v | (v << 16)) & 0x001f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// Inverse of spread3.
__host__ __device__ __forceinline__ uint32_t compact3(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x001f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x001f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x00000000001fffffull;
    return (uint32_t)v;
}

// Coherent (device-scope) loads for data written by other workgroups in the
// same kernel.
__device__ __forceinline__ double ld_dev(const double *p) {
    unsigned long long v = __hip_atomic_load((const unsigned long long *)p, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)v);
}
__device__ __forceinline__ uint32_t ld_dev_u32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev_u32(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Knuth two-sum: s + e == a + b exactly (round-to-nearest FP32).
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Compensated accumulator: value = hi + lo.
struct Comp {
    float hi, lo;
    __device__ __forceinline__ void zero() { hi = 0.f; lo = 0.f; }
    __device__ __forceinline__ void add(float v) {
        float s, e;
        two_sum(hi, v, s, e);
        hi = s;
        lo += e;
    }
    __device__ __forceinline__ double value() const { return (double)hi + (double)lo; }
};

// Node record read by the walk: one 128-byte line per node and moment set.
struct alignas(128) NodeW {
    double clo[3], chi[3];     // cube corners
    double com[3];             // centre of mass of the set
    double hmax;               // largest softening radius in the set
    double M;                  // mass of the set
    int32_t first, count;      // particle range (sorted order)
    int32_t child;             // first child (-1 for leaves)
    int32_t lvl_nch;           // level << 8 | number of children
    double pad[2];
};

// Traceless quadrupole of a node (xx yy xy xz yz; zz = -xx - yy).
struct alignas(16) NodeQ {
    double q[5];
    double pad;
};

}  // namespace sf

// Opaque handle (C linkage name from the public header).
struct sf_grav_tree_s {
    int64_t n = 0, n_gas = 0, n_sink = 0;
    sf_dtype dt = SF_F32;
    int leaf_cap = 16, group_cap = 64;
    hipStream_t stream = nullptr;
    int device = 0;

    // sorted particles (dtype of the inputs), order, keys
    uint64_t *keys = nullptr;
    int32_t *order = nullptr;
    void *xs = nullptr, *ys = nullptr, *zs = nullptr, *ms = nullptr, *hs = nullptr;
    int32_t *sink_pos = nullptr;      // sorted positions of the sinks
    sf::Frame *frame = nullptr;       // device
    sf::Frame hframe{};

    // nodes (breadth-first)
    int64_t n_nodes = 0, n_leaves = 0;
    int max_level = 0;
    int64_t level_off[24] = {};                       // first node of each level
    int32_t *nlevel = nullptr, *nfirst = nullptr, *ncount = nullptr, *nparent = nullptr;
    int32_t *nchild = nullptr, *nnchild = nullptr;
    double *clo = nullptr, *chi = nullptr;            // cube corners, 3 per node
    int32_t *pleaf = nullptr;                         // leaf node of each sorted particle
    // moments, set 0 = all particles, set 1 = gas only
    double *M[2] = {nullptr, nullptr};
    double *com[2] = {nullptr, nullptr};              // 3 per node
    double *Q[2] = {nullptr, nullptr};                // 6 per node: xx yy zz xy xz yz
    double *hmax[2] = {nullptr, nullptr};
    sf::NodeW *nw[2] = {nullptr, nullptr};
    sf::NodeQ *nq[2] = {nullptr, nullptr};

    // groups
    int64_t n_groups = 0;
    int32_t *n_groups_dev = nullptr;
    int32_t *gfirst = nullptr, *gcount = nullptr;
    double *gbox = nullptr;                           // 6 per group: lo3 hi3
    double *ghmax = nullptr;
    double *gcen = nullptr;                           // 3 per group
    int32_t *gnpc = nullptr, *gnpp = nullptr;         // stats
    uint64_t *gcks = nullptr;                         // stats: list checksum per group
    bool have_stats = false;
    // previous field for the relative criterion: |g| per sorted particle and
    // smallest |g| per group
    double *fpt = nullptr, *fgrp = nullptr;
    bool have_field = false;
    // per group, written by every forward walk: (3 nodes + particles) x the
    // adjoint's lanes per target, so the adjoint can start costly groups first
    uint32_t *gcost = nullptr;
    bool have_cost = false;

    int64_t groups_cap = 0;
    uint32_t *info_dev = nullptr;                     // [0] max level, [1] leaves

    // direct path: 64-particle tiles of the (type-major) sorted order
    int64_t n_tiles = 0, n_gas_tiles = 0;
    int32_t *tfirst = nullptr, *tcount = nullptr;
    double *tbox = nullptr;                           // 8 per tile: lo3 hi3 hmax pad
    double *tcen = nullptr;                           // 3 per tile
    void *tsrc = nullptr;                             // packed source records

    bool direct_only = false;                         // built by the direct path
    // phase timers (opts.timing)
    static constexpr int kPhases = 11;
    hipEvent_t ev0[kPhases] = {}, ev1[kPhases] = {};
    bool ev_used[kPhases] = {};
    bool timing = false;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;  // side-stream fork and join
    std::vector<void *> allocs;                       // device memory owned here
};
