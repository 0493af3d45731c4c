// sf_walk.h -- the group tree walk shared by the forward and adjoint kernels
// (internal).  See sf_walk.hip for the description of the walk.
#pragma once
#include "sf_math.h"

namespace sf {

// Walk stack: kStack entries bound it (see the walk's header); the top
// kStackLds of them live in LDS, older ones are moved, 64 at a time, to a
// per-wave area in device memory when the window fills (rare at theta 0.5;
// full-tree walks at theta 0 reach it) and brought back when the top runs
// short.
constexpr int kStack = 22 * 64 + 64;
constexpr int kStackLds = 128;
constexpr uint32_t kStackMask = kStackLds - 1;

struct WalkNodes {
    int64_t n_nodes;
    const NodeW *w;                      // node records of the moment set used
    const NodeQ *q;                      // quadrupoles of that set
    double side;                         // root cube side (cell = side 2^-level)
    double th2;                          // theta^2
    // relative (acceleration-based) criterion, on when rel != 0: a task
    // opens a node when G M L^2 > ag r^4, ag = alpha |g|min of the task
    int32_t rel;
    double G, alpha;
    const double *fgrp;                  // per group: smallest previous |g| of its members
    const double *fpt;                   // per sorted particle: previous |g|
};

// Ring of opened-leaf particle ranges (first, count).
struct PPRing {
    int32_t f[128];
    int32_t c[128];
};

struct WalkLds {
    uint32_t stack[kStackLds];   // stack position p at index p & kStackMask
    int32_t pc[128];
    PPRing near;   // leaves that may hold softened pairs (incl. the task's own)
    PPRing far;    // leaves whose every pair with the task is Newtonian
    int32_t slot[128];
    uint32_t mark[64];   // pop: 1 + lane of the entry whose nodes start at this slot, else 0
};

template <typename R> struct alignas(16) PPStage { R x, y, z, m, h2, h, hinv; int32_t idx; };
// qzz = -(qxx + qyy) (Q is traceless), formed once when the node is staged.
template <typename R> struct alignas(16) PCStage { R x, y, z, M, qxx, qyy, qxy, qxz, qyz, qzz; };
// One batch is staged at a time, so the particle and node stages share LDS.
// Particle batches of the FP32 forms hold up to 128 entries.
template <typename R> constexpr uint32_t kPPBatch = sizeof(R) == 4 ? 128u : 64u;
template <typename R> union StageBuf {
    PPStage<R> pp[kPPBatch<R>];
    PCStage<R> pc[64];
};
// The group walk sums its per-lane partials (4 doubles per lane) in the stage.
static_assert(sizeof(StageBuf<float>) >= 4 * 64 * sizeof(double), "stage too small for the sums");

// Particle pair: d = source - target.  Accumulates a (F m d) and phi (-m P).
// hjinv, tiinv are the reciprocals of the two softening lengths (the support's
// reciprocal is the smaller one).  SELF = false leaves the self pair in: its
// force term is exactly zero (d = 0, F finite) and its potential term is
// m (14/5) / h of the target, which the caller then takes out once
// (self_P below).
template <typename R, bool SELF = true>
__device__ __forceinline__ void pair(R dx, R dy, R dz, R m, R hj2, R hj, R hjinv, R ti2, R ti,
                                     R tiinv, bool self, R &bx, R &by, R &bz, R &bp) {
    const R r2 = dx * dx + dy * dy + dz * dz;
    const R ri = rsq(r2);
    R P = ri;
    R F = ri * ri * ri;
    const R hh2 = pos_max(hj2, ti2);
    if (r2 < hh2) {
        soft_FP_ri<R>(r2, ri, pos_max(hj, ti), pos_min(hjinv, tiinv), F, P);
        if (SELF && self) { F = R(0); P = R(0); }
    }
    const R mF = m * F;
    bx += mF * dx;
    by += mF * dy;
    bz += mF * dz;
    bp -= m * P;
}

// The softened P at r = 0, (14/5) / h, rounded as pair<R, false> rounds it
// for a target's own particle (whose potential term is m times this).
template <typename R>
__device__ __forceinline__ R self_P(R hinv) {
    return R(14.0 / 5.0) * hinv;
}

// Newtonian particle pair (no softening possible, not a self pair).
template <typename R>
__device__ __forceinline__ void pair_newton(R dx, R dy, R dz, R m, R &bx, R &by, R &bz, R &bp) {
    const R r2 = dx * dx + dy * dy + dz * dz;
    const R ri = rsq(r2);
    const R mri = m * ri;
    const R mri3 = mri * ri * ri;
    bp -= mri;
    bx += mri3 * dx;
    by += mri3 * dy;
    bz += mri3 * dz;
}

// Multipole term: r = target - centre of mass; qzz = -(qxx + qyy).
template <typename R, int ORDER>
__device__ __forceinline__ void multipole(R rx, R ry, R rz, R M, R qxx, R qyy, R qxy, R qxz, R qyz,
                                          R qzz, R &bx, R &by, R &bz, R &bp) {
    const R r2 = rx * rx + ry * ry + rz * rz;
    const R ri = rsq(r2);
    const R ri2 = ri * ri;
    const R Mri = M * ri;
    if (ORDER == 0) {
        const R c = -Mri * ri2;
        bx += c * rx;
        by += c * ry;
        bz += c * rz;
        bp -= Mri;
    } else {
        const R qx = qxx * rx + qxy * ry + qxz * rz;
        const R qy = qxy * rx + qyy * ry + qyz * rz;
        const R qz = qxz * rx + qyz * ry + qzz * rz;
        const R rqr = qx * rx + qy * ry + qz * rz;
        const R ri5 = ri2 * ri2 * ri;
        const R t2 = rqr * ri5;                          // twice the quadrupole potential term
        bp -= fma(R(0.5), t2, Mri);
        const R c = -fma(R(2.5), t2, Mri) * ri2;
        bx = fma(c, rx, bx);
        by = fma(c, ry, by);
        bz = fma(c, rz, bz);
        bx = fma(ri5, qx, bx);
        by = fma(ri5, qy, by);
        bz = fma(ri5, qz, bz);
    }
}

// ---------------------------------------------------------------- walk core

// Test one node against the task box: cls 1 accept, 2 open leaf that may
// hold softened pairs, 3 open inner, 4 open leaf with only Newtonian pairs
// (gap to the box at least the larger max softening).  A node is opened when
// its opening angle is too large, when the relative criterion (if on) asks
// for it, when it is near the box (overlap, contact, softening) or when it
// has no mass (no centre of mass to expand about: its particles are summed
// as pairs).  All FP64 steps are separately rounded (no contraction).  The
// node record is read once, whole, and the fields the walk needs next are
// returned with the class, so a step costs one memory round trip per node.
// NEAR_ONLY walks (neighbour sums) keep only what can hold a softened pair:
// near nodes are opened as usual and every other node is dropped (class 0),
// which reaches exactly the near leaves of the full walk, because every
// ancestor of a near node is near.
struct NodeHit {
    int cls;
    int32_t first, count, child, lvl_nch;
};

template <bool NEAR_ONLY = false>
__device__ __forceinline__ NodeHit classify(const WalkNodes &nd, int node, const double blo[3],
                                            const double bhi[3], double hg, int64_t gf,
                                            int64_t gl, double ag) {
    const NodeW w = nd.w[node];
    const int64_t f = w.first, c = w.count;
    const bool open = (f < gl) && (gf < f + c);
    const bool meets = w.clo[0] <= bhi[0] && blo[0] <= w.chi[0] && w.clo[1] <= bhi[1] &&
                       blo[1] <= w.chi[1] && w.clo[2] <= bhi[2] && blo[2] <= w.chi[2];
    double g[3], e[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        g[d] = fmax(fmax(dsub(w.clo[d], bhi[d]), dsub(blo[d], w.chi[d])), 0.0);
        e[d] = fmax(fmax(dsub(blo[d], w.com[d]), dsub(w.com[d], bhi[d])), 0.0);
    }
    const double dbb2 = dadd(dadd(dmul(g[0], g[0]), dmul(g[1], g[1])), dmul(g[2], g[2]));
    const double hm = fmax(w.hmax, hg);
    const bool soft = dbb2 < dmul(hm, hm);
    const double r2 = dadd(dadd(dmul(e[0], e[0]), dmul(e[1], e[1])), dmul(e[2], e[2]));
    const double L = ldexp(nd.side, -(w.lvl_nch >> 8));
    const double L2 = dmul(L, L);
    bool far_ok = !(L2 > dmul(nd.th2, r2)) && w.M > 0.0;
    if (nd.rel) far_ok = far_ok && !(dmul(dmul(nd.G, w.M), L2) > dmul(ag, dmul(r2, r2)));
    const bool near = open || meets || soft;
    int cls = (!near && far_ok) ? 1 : ((w.lvl_nch & 255) != 0 ? 3 : (near ? 2 : 4));
    if (NEAR_ONLY && !near) cls = 0;
    return {cls, w.first, w.count, w.child, w.lvl_nch};
}

// Relative-criterion threshold of a task (alpha times the smallest previous
// |g| of its targets); unused when the criterion is off.
__device__ __forceinline__ double task_ag_group(const WalkNodes &nd, int g) {
    return nd.rel ? dmul(nd.alpha, nd.fgrp[g]) : 0.0;
}
__device__ __forceinline__ double task_ag_point(const WalkNodes &nd, int64_t p) {
    return nd.rel ? dmul(nd.alpha, nd.fpt[p]) : 0.0;
}

// Order-independent list checksum: each accepted node adds mix(node), each
// opened leaf mix(node + 2^31); the sum over the list (mod 2^64) identifies
// the set of decisions a task took.
__device__ __forceinline__ uint64_t list_mix(uint64_t v) {
    v += 0x9e3779b97f4a7c15ull;
    v = (v ^ (v >> 30)) * 0xbf58476d1ce4e5b9ull;
    v = (v ^ (v >> 27)) * 0x94d049bb133111ebull;
    return v ^ (v >> 31);
}

// Next task index for the whole wave, as a scalar (SGPR) value: lane 0 takes
// it from the counter and readfirstlane broadcasts it.  Keeping every loop
// bound of the walk in scalar registers makes all loop exits scalar
// branches; a task index broadcast through a vector register let the
// compiler structure the task loop as a divergent loop.
__device__ __forceinline__ int next_task(int32_t *ctr) {
    int g = 0;
    if ((threadIdx.x & 63) == 0) g = atomicAdd(ctr, 1);
    return __builtin_amdgcn_readfirstlane(g);
}

// XCD (the L2 domain, one of 8 on MI355X) of the executing wave, read from
// the hardware register XCC_ID.  Used only to place work and scratch copies
// near an L2; no result depends on its value.
constexpr int kXcd = 8;
__device__ __forceinline__ int xcd_id() {
    return __builtin_amdgcn_s_getreg((3 << 11) | 20) & (kXcd - 1);   // hwreg(XCC_ID, 0, 4)
}

// Task counters: the group-task counter, the sink-task counter, the error
// word and kXcd per-XCD group counters, 64 bytes apart.
constexpr int kCtrStride = 16;
constexpr int kCtrSinks = kCtrStride;
constexpr int kCtrErr = kCtrSinks + kCtrStride;
constexpr int kCtrXcd = kCtrErr + kCtrStride;
constexpr int kCtrWords = kCtrXcd + kXcd * kCtrStride;

// Group tasks placed by XCD: the groups (Morton order, so spatially compact
// runs) are cut into chunks of kXcdChunk, dealt to the XCDs in turn (chunk q
// to XCD q mod kXcd).  A wave takes the tasks of its own XCD's chunks in
// order, then helps the other XCDs (its XCD + 1, + 2, ...) until all are
// drained.  At any moment the waves of one XCD work on a run of neighbouring
// groups, which read the same node and particle records, so that XCD's L2
// holds one compact region instead of a slice of every region in flight; and
// all XCDs move through the Morton order together, so their shares of dense
// and sparse regions stay alike.  (One contiguous eighth per XCD measured 8%
// slower: the eighths' costs differ.)  Every task is taken exactly once, as
// offset t of one XCD's sequence, and a wave stops after finding all kXcd
// sequences past the last group.
constexpr int kXcdChunkLog = 10;
constexpr int kXcdChunk = 1 << kXcdChunkLog;

struct XcdTasks {
    int32_t *xc;   // kXcd counters, kCtrStride words apart
    int ng, xcd, probe;

    __device__ __forceinline__ void init(int32_t *ctr, int n_groups) {
        xc = ctr + kCtrXcd;
        ng = n_groups;
        xcd = xcd_id();
        probe = 0;
    }

    // Next task for the whole wave (a scalar), or ng when none is left.
    __device__ __forceinline__ int next() {
        while (probe < kXcd) {
            const int c = (xcd + probe) & (kXcd - 1);
            int t = 0;
            if ((threadIdx.x & 63) == 0) t = atomicAdd(xc + c * kCtrStride, 1);
            t = __builtin_amdgcn_readfirstlane(t);
            // offset t of XCD c's sequence: chunk (t / kXcdChunk) kXcd + c
            const int64_t g = ((int64_t)(t >> kXcdChunkLog) * kXcd + c) * kXcdChunk +
                              (t & (kXcdChunk - 1));
            if (g < ng) return (int)g;
            ++probe;
        }
        return ng;
    }
};

// Prefix sums and totals over the wave (called with all 64 lanes active):
// an inclusive scan by DPP, one VALU add per stage -- row shifts by 1, 2, 4
// and 8 lanes (lanes without a source add 0), then the last lane of rows 0
// and 2 added to rows 1 and 3, and the last lane of row 1 to rows 2 and 3.
// The total is lane 63's value, read into a scalar register.
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);   // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return v;
}

__device__ __forceinline__ uint32_t wave_total(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_scan_incl(v), 63);
}

// Inclusive prefix maximum over the wave, by the same DPP stages.
__device__ __forceinline__ uint32_t wave_max_incl(uint32_t v) {
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
    return v;
}

// Value of v in lane src (0..63).
__device__ __forceinline__ uint32_t lane_value(uint32_t src, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src << 2), (int)v);
}

// Gather `want` (<= 64) particle indices from the front of a range ring into
// slot[], in one pass: lane l looks at ring entry head + l, an inclusive scan
// of the entry sizes places every entry's particles, entries used up are
// dropped and a partly used one is shortened in place.  Every entry holds at
// least one particle, so 64 entries always cover `want`; returns false (and
// flags err) if the pending entries hold fewer particles, which the pending
// counts rule out.
__device__ __forceinline__ bool ring_gather(PPRing &R, uint32_t &h, uint32_t t, int32_t *slot,
                                            uint32_t *mark, uint32_t want, int32_t *err) {
    const uint32_t lane = threadIdx.x;
    const bool have = h + lane < t;
    const uint32_t q = (h + lane) & 127;
    const int32_t f = have ? R.f[q] : 0;
    const uint32_t c = have ? (uint32_t)R.c[q] : 0u;
    const uint32_t incl = wave_scan_incl(c);
    const uint32_t excl = incl - c;
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    if (total < want) {
        if (lane == 0) atomicOr(err, 4);
        return false;
    }
    // slot l takes particle f + (l - excl) of the entry whose range
    // [excl, incl) holds l: each entry marks its first slot (mark[] is zero
    // between calls), a prefix maximum spreads the marks
    if (have && excl < want) {
        mark[excl] = lane + 1u;
        if (incl > want) {   // the one entry that is used only in part
            const uint32_t take = want - excl;
            R.f[q] = f + (int32_t)take;
            R.c[q] = (int32_t)(c - take);
        }
    }
    __syncthreads();
    const uint32_t mk = wave_max_incl(mark[lane]);
    mark[lane] = 0u;   // read above by this lane only
    const uint32_t e = mk > 0u ? mk - 1u : 0u;
    const uint32_t f_e = lane_value(e, (uint32_t)f), excl_e = lane_value(e, excl);
    if (lane < want) slot[lane] = (int32_t)(f_e + (lane - excl_e));
    // entries used up: those whose inclusive count is at most want
    h += (uint32_t)popc64(__ballot(have && incl <= want));
    __syncthreads();
    return true;
}

// Gather up to 128 particle indices: ring_gather in passes of at most 64.
__device__ __forceinline__ bool ring_gather_n(PPRing &R, uint32_t &h, uint32_t t, int32_t *slot,
                                              uint32_t *mark, uint32_t want, int32_t *err) {
    if (want <= 64u) return ring_gather(R, h, t, slot, mark, want, err);
    if (!ring_gather(R, h, t, slot, mark, 64u, err)) return false;
    return ring_gather(R, h, t, slot + 64, mark, want - 64u, err);
}

// Walk one task.  Ev supplies pc_batch(L, head, nb) (nb <= pcb <= 64) and
// pp_batch<SOFT>(L, nb) (nb <= ppb <= 128; SOFT = false: every pair is
// Newtonian and none is a self pair).  Full batches hold pcb nodes and ppb
// particles; the last ones of a task may be shorter.  A range ring is
// drained before it holds more than 64 entries, and fewer than pcb <= 64
// accepted nodes wait between steps, so the next step's (at most 64) new
// entries always fit.
// Stack entries moved out of and back into LDS: device-scope relaxed
// atomics, so the wave reads back exactly what it wrote (no stale L1 line).
__device__ __forceinline__ void stack_out(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t stack_in(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// With CKS, cks receives (on every lane) the task's list checksum.  With
// NEAR_ONLY only near nodes are walked (see classify): no accepted nodes and
// no far leaves reach the evaluator.
template <bool CKS, class Ev, bool NEAR_ONLY = false>
__device__ void walk_task(const WalkNodes &nd, WalkLds &L, uint32_t *gstack, Ev &ev,
                          const double blo[3], const double bhi[3], double hg, int64_t gf,
                          int64_t gl, double ag, int32_t *err, uint32_t &n_pc, uint32_t &n_pp,
                          uint64_t &cks, uint32_t ppb = 64u, uint32_t pcb = 64u) {
    const int lane = threadIdx.x;
    const uint64_t lt = lane_mask_lt();
    uint32_t sp = 1;     // stack positions [0, sp)
    uint32_t base = 0;   // positions [base, sp) in LDS, [0, base) in gstack
    if (lane == 0) L.stack[0] = 1u;   // root (node 0), one node
    L.mark[lane] = 0u;
    uint32_t pc_h = 0, pc_t = 0;
    uint32_t nh = 0, nt = 0, npend = 0;   // near ring
    uint32_t fh = 0, ft = 0, fpend = 0;   // far ring
    n_pc = 0;
    n_pp = 0;
    uint64_t lane_cks = 0;
    __syncthreads();
    // Every node is popped at most once per task, so a task takes at most
    // n_nodes steps; the bound makes termination unconditional.
    int64_t steps = 0;
    while (sp > 0) {
        if (++steps > nd.n_nodes + 1) {
            if (lane == 0) atomicOr(err, 2);
            break;
        }
        // the top 64 positions must be in LDS: bring back the 64 older ones
        // (the window then holds at most 63 + 64 entries)
        if (base > 0 && sp - base < 64u) {
            const uint32_t nb = base - 64u;   // base is a multiple of 64
            for (uint32_t p = nb + lane; p < base; p += 64u) L.stack[p & kStackMask] = stack_in(gstack + p);
            base = nb;
            __syncthreads();
        }
        // pop whole entries from the top, at most 64 nodes
        const int ei = (int)sp - 1 - lane;
        const uint32_t ent = ei >= 0 ? L.stack[ei & kStackMask] : 0u;
        const uint32_t cnt = ent & 15u;
        const uint32_t incl = wave_scan_incl(cnt);   // an entry holds 1..8 nodes
        const bool take = ei >= 0 && incl <= 64u;
        const uint32_t ntake = (uint32_t)popc64(__ballot(take));
        const uint32_t nnodes = (uint32_t)__builtin_amdgcn_readlane((int)incl, (int)ntake - 1);
        // slot l takes node (first of entry e) + (l - start of e) for the
        // taken entry e whose slot range [incl - cnt, incl) holds l: each
        // entry marks its first slot, a prefix maximum spreads the marks
        if (take) L.mark[incl - cnt] = (uint32_t)lane + 1u;
        sp -= ntake;
        __syncthreads();
        const uint32_t mk = wave_max_incl(L.mark[lane]);
        L.mark[lane] = 0u;   // read above by this lane only; clear for the next step
        const uint32_t e = mk > 0u ? mk - 1u : 0u;
        const uint32_t ent_e = lane_value(e, ent), incl_e = lane_value(e, incl);
        const int node = lane < (int)nnodes
                             ? (int)((ent_e >> 4) + ((uint32_t)lane - (incl_e - (ent_e & 15u))))
                             : -1;
        NodeHit hit{0, 0, 0, 0, 0};
        if (node >= 0) hit = classify<NEAR_ONLY>(nd, node, blo, bhi, hg, gf, gl, ag);
        const int cls = hit.cls;
        if (CKS && (cls == 1 || cls == 2 || cls == 4))
            lane_cks += list_mix((uint64_t)node + (cls == 1 ? 0ull : (1ull << 31)));
        const uint64_t macc = __ballot(cls == 1), mnear = __ballot(cls == 2),
                       mint = __ballot(cls == 3), mfar = __ballot(cls == 4);
        if (cls == 1) L.pc[(pc_t + popc64(macc & lt)) & 127] = node;
        pc_t += (uint32_t)popc64(macc);
        uint32_t lcn = 0, lcf = 0;
        if (cls == 2) {
            const uint32_t q = (nt + popc64(mnear & lt)) & 127;
            lcn = (uint32_t)hit.count;
            L.near.f[q] = hit.first;
            L.near.c[q] = hit.count;
        }
        if (cls == 4) {
            const uint32_t q = (ft + popc64(mfar & lt)) & 127;
            lcf = (uint32_t)hit.count;
            L.far.f[q] = hit.first;
            L.far.c[q] = hit.count;
        }
        nt += (uint32_t)popc64(mnear);
        ft += (uint32_t)popc64(mfar);
        npend += wave_total(lcn);
        fpend += wave_total(lcf);
        const uint32_t npush = (uint32_t)popc64(mint);
        if (sp + npush > (uint32_t)kStack) {   // cannot happen (see header); stop safely
            if (lane == 0) atomicOr(err, 1);
            break;
        }
        // room for the push: move the oldest 64 window entries out (they all
        // exist: sp - base > kStackLds - 64 = 64 here)
        while (sp + npush - base > (uint32_t)kStackLds) {
            stack_out(gstack + base + lane, L.stack[(base + lane) & kStackMask]);
            base += 64u;
            __syncthreads();
        }
        if (cls == 3) {
            const uint32_t r = (uint32_t)popc64(mint & lt);
            L.stack[(sp + npush - 1 - r) & kStackMask] =
                ((uint32_t)hit.child << 4) | (uint32_t)(hit.lvl_nch & 255);
        }
        sp += npush;
        __syncthreads();
        while (pc_t - pc_h >= pcb) {
            ev.pc_batch(L, pc_h, pcb);
            pc_h += pcb;
            n_pc += pcb;
        }
        while (fpend >= ppb || ft - fh > 64u) {
            const uint32_t nb = fpend < ppb ? fpend : ppb;
            if (!ring_gather_n(L.far, fh, ft, L.slot, L.mark, nb, err)) { fpend = 0; break; }
            ev.template pp_batch<false>(L, nb);
            fpend -= nb;
            n_pp += nb;
        }
        while (npend >= ppb || nt - nh > 64u) {
            const uint32_t nb = npend < ppb ? npend : ppb;
            if (!ring_gather_n(L.near, nh, nt, L.slot, L.mark, nb, err)) { npend = 0; break; }
            ev.template pp_batch<true>(L, nb);
            npend -= nb;
            n_pp += nb;
        }
    }
    if (pc_t > pc_h) {
        ev.pc_batch(L, pc_h, pc_t - pc_h);
        n_pc += pc_t - pc_h;
    }
    if (fpend > 0) {
        if (ring_gather_n(L.far, fh, ft, L.slot, L.mark, fpend, err)) {
            ev.template pp_batch<false>(L, fpend);
            n_pp += fpend;
        }
    }
    if (npend > 0) {
        if (ring_gather_n(L.near, nh, nt, L.slot, L.mark, npend, err)) {
            ev.template pp_batch<true>(L, npend);
            n_pp += npend;
        }
    }
    if (CKS) {
        uint64_t v = lane_cks;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += (uint64_t)__shfl_xor((unsigned long long)v, off, 64);
        cks = v;
    }
    __syncthreads();
}

}  // namespace sf
