// sf_walk.hip -- Barnes-Hut group walk and interaction evaluation on gfx950
// (paper Sec. 2.2: node multipoles unless the opening criterion opens the
// node; Sec. 2.2.1: softened pairs r < max(h_i, h_j), Newtonian beyond).
//
// One wavefront per walk task.  A task is either a target group (up to 64
// Morton-consecutive particles, floor(64 / group size) lanes per target, node
// moments over all particles) or one sink target (node moments over gas only,
// lanes spread over the sources, sink sources skipped -- sinks see other
// sinks through the FP64 sink-sink sum).
//
// Walk: an LDS stack of child ranges (<= 8 nodes each).  Each step pops whole
// entries from the top, up to 64 nodes, one node per lane, and tests each
// against the task's bounding box in FP64 with separately rounded operations.
// A node is opened when (a) L^2 > theta^2 r^2 with r the distance from its
// centre of mass to the box, (r) with the relative criterion on,
// G M L^2 > alpha |g|min r^4 (|g|min the smallest previous field magnitude
// of the task's targets), (b) its cube meets the box or it holds one of the
// task's particles, (c) the cube-box gap is below the larger maximum
// softening, or (z) it has no mass.  Accepted nodes go to a ring of multipole interactions, opened
// leaves to a ring of particle ranges, opened inner nodes push their child
// range.  Children are pushed in reverse lane order, so levels never decrease
// from bottom to top of the stack; a new level-L entry is only pushed when a
// level L-1 node is popped, which pops every level-L entry above it first,
// so at most 64 entries per level are ever stored: 22 * 64 bounds the stack.
// Interactions are evaluated in batches as the rings fill: 64 nodes, and up
// to 128 particles in the FP32 forms of the group walk (64 otherwise).
#include <atomic>

#include "sf_build.h"
#include "sf_math.h"
#include "sf_prims.h"
#include "sf_walk.h"

namespace sf {

// ---------------------------------------------------------------- common args

template <typename T>
struct WalkArgs {
    WalkNodes nd;
    const T *xs, *ys, *zs, *ms, *hs;
    const int32_t *order;
    int64_t n, n_gas;
    // tasks
    const int32_t *n_groups_dev;
    const int32_t *gfirst, *gcount;
    const double *gbox, *ghmax, *gcen;
    const int32_t *sink_pos;
    int64_t n_sink;
    const double *ss;          // sink-sink sums (4 per sink), may be null
    int32_t *task_ctr;
    int32_t *err;
    uint32_t *gstack;          // kStack entries per block: stack overflow area
    int32_t *gnpc, *gnpp;      // stats (group mode), may be null
    uint64_t *gcks;            // stats: per-group list checksum, may be null
    uint32_t *gcost;           // per-group cost for the adjoint's task order, may be null
    T *acc, *pot;
    double G;
};

// ---------------------------------------------------------------- group mode

// Batch staging for lane splitting: entry e of a batch (e < nb <= 64) goes to
// LDS slot e; copy `sub` of a target (k copies) takes entries sub, sub + k, ...
// in floor(nb / k) steps that every lane runs, plus one step for the copies
// with an entry left over.

template <typename T, int FORM, int ORDER>
struct GroupEval {
    using R = typename FormT<FORM>::R;
    const WalkArgs<T> *a;
    PPStage<R> *spp;
    PCStage<R> *spc;
    double cen[3];
    R tx, ty, tz, th, th2, thinv;
    R bl[3], bh[3], hg2;        // group box in the form's frame, largest h squared
    uint32_t nsoft, nnewt;      // partition counts of the particle batch being staged
    int32_t tidx;
    uint32_t sub, k;            // lane splitting: lane handles entries sub, sub+k, ...
    Acc<FORM> ax, ay, az, ap;

    __device__ void pc_batch(WalkLds &L, uint32_t head, uint32_t nb) {
        const uint32_t e = threadIdx.x;
        if (e < nb) {
            PCStage<R> s;
            const int node = L.pc[(head + e) & 127];
            const WalkNodes &nd = a->nd;
            s.x = dto_frame<FORM>(nd.w[node].com[0], cen[0]);
            s.y = dto_frame<FORM>(nd.w[node].com[1], cen[1]);
            s.z = dto_frame<FORM>(nd.w[node].com[2], cen[2]);
            s.M = (R)nd.w[node].M;
            s.qxx = s.qyy = s.qxy = s.qxz = s.qyz = R(0);
            if (ORDER == 2) {
                s.qxx = (R)nd.q[node].q[0];
                s.qyy = (R)nd.q[node].q[1];
                s.qxy = (R)nd.q[node].q[2];
                s.qxz = (R)nd.q[node].q[3];
                s.qyz = (R)nd.q[node].q[4];
            }
            s.qzz = -(s.qxx + s.qyy);
            spc[e] = s;
        }
        __syncthreads();
        R bx = 0, by = 0, bz = 0, bp = 0;
        // entries sub, sub + k, ...: nb / k steps with an entry on every lane,
        // then one step for the lanes whose entry is left over
        const uint32_t mf = nb / k;
        const PCStage<R> *src = spc + sub;
        for (uint32_t j = 0; j < mf; ++j) {
            const PCStage<R> s = src[j * k];
            multipole<R, ORDER>(tx - s.x, ty - s.y, tz - s.z, s.M, s.qxx, s.qyy, s.qxy, s.qxz,
                                s.qyz, s.qzz, bx, by, bz, bp);
        }
        if (sub + mf * k < nb) {
            const PCStage<R> s = src[mf * k];
            multipole<R, ORDER>(tx - s.x, ty - s.y, tz - s.z, s.M, s.qxx, s.qyy, s.qxy, s.qxz,
                                s.qyz, s.qzz, bx, by, bz, bp);
        }
        ax.fold(bx);
        ay.fold(by);
        az.fold(bz);
        ap.fold(bp);
        __syncthreads();
    }

    template <bool SOFT>
    __device__ __forceinline__ void pp_one(const PPStage<R> &s, R &bx, R &by, R &bz, R &bp) const {
        if (SOFT)   // the self pair stays in; its potential term is taken out per target
            pair<R, false>(s.x - tx, s.y - ty, s.z - tz, s.m, s.h2, s.h, s.hinv, th2, th, thinv,
                           false, bx, by, bz, bp);
        else
            pair_newton<R>(s.x - tx, s.y - ty, s.z - tz, s.m, bx, by, bz, bp);
    }

    // Entries [lo, lo + n) of the stage, copy `sub` taking lo + sub, lo + sub + k, ...
    template <bool SOFT>
    __device__ __forceinline__ void pp_run(uint32_t lo, uint32_t n, R &bx, R &by, R &bz,
                                           R &bp) const {
        const uint32_t mf = n / k;
        const PPStage<R> *src = spp + lo + sub;
        for (uint32_t j = 0; j < mf; ++j) pp_one<SOFT>(src[j * k], bx, by, bz, bp);
        if (sub + mf * k < n) pp_one<SOFT>(src[mf * k], bx, by, bz, bp);
    }

    // SOFT batches (leaves that may hold softened pairs) are split once more
    // per source particle: a source farther from the group box than
    // max(its h, the group's largest h), with a relative margin that covers
    // the rounding of both distances, has only Newtonian pairs with the
    // group and runs the short loop; the rest (the task's own particles
    // among them) run the softened one.  Target coordinates lie inside the
    // box in the form's frame too, since rounding is monotone.
    template <bool SOFT>
    __device__ void pp_batch(WalkLds &L, uint32_t nb) {
        nsoft = nnewt = 0;
        for (uint32_t r = 0; r < nb; r += 64u) stage_pp<SOFT>(L, r + threadIdx.x, nb);
        __syncthreads();
        R bx = 0, by = 0, bz = 0, bp = 0;
        if (SOFT) {
            const uint32_t ns = nsoft;
            pp_run<false>(ns, nb - ns, bx, by, bz, bp);
            pp_run<true>(0, ns, bx, by, bz, bp);
        } else {
            pp_run<false>(0, nb, bx, by, bz, bp);
        }
        ax.fold(bx);
        ay.fold(by);
        az.fold(bz);
        ap.fold(bp);
        __syncthreads();
    }

    // Stage entry e of a particle batch; all lanes call it once per round of
    // 64 entries (SOFT: the possibly softened entries first, the Newtonian-only
    // ones after them).
    template <bool SOFT>
    __device__ __forceinline__ void stage_pp(WalkLds &L, uint32_t e, uint32_t nb) {
        PPStage<R> s;
        bool soft = false;
        if (e < nb) {
            const int p = L.slot[e];
            s.x = to_frame<FORM>(a->xs[p], cen[0]);
            s.y = to_frame<FORM>(a->ys[p], cen[1]);
            s.z = to_frame<FORM>(a->zs[p], cen[2]);
            s.m = (R)a->ms[p];
            s.h = (R)a->hs[p];
            s.h2 = s.h * s.h;
            s.hinv = rcp(s.h);
            s.idx = p;
            if (SOFT) {
                const R gx = fmax(fmax(bl[0] - s.x, s.x - bh[0]), R(0));
                const R gy = fmax(fmax(bl[1] - s.y, s.y - bh[1]), R(0));
                const R gz = fmax(fmax(bl[2] - s.z, s.z - bh[2]), R(0));
                const R d2 = gx * gx + gy * gy + gz * gz;
                const R h2 = s.h2 > hg2 ? s.h2 : hg2;
                soft = !(d2 > h2 * R(1.0001));
            }
        }
        if (SOFT) {
            // softened entries of earlier rounds of 64 are counted in nsoft,
            // Newtonian ones fill the stage from the end
            const uint64_t msoft = __ballot(e < nb && soft);
            const uint64_t mnewt = __ballot(e < nb && !soft);
            const uint64_t lt = lane_mask_lt();
            if (e < nb) {
                if (soft) spp[nsoft + (uint32_t)popc64(msoft & lt)] = s;
                else spp[nb - 1 - (nnewt + (uint32_t)popc64(mnewt & lt))] = s;
            }
            nsoft += (uint32_t)popc64(msoft);
            nnewt += (uint32_t)popc64(mnewt);
        } else if (e < nb) {
            spp[e] = s;
        }
    }
};

template <typename T, int FORM, int ORDER, bool STATS>
__global__ __launch_bounds__(64) void k_walk_groups(WalkArgs<T> a) {
    using R = typename FormT<FORM>::R;
    __shared__ WalkLds L;
    __shared__ StageBuf<R> stage;
    const int lane = threadIdx.x;
    const int ng = __builtin_amdgcn_readfirstlane(*a.n_groups_dev);
    GroupEval<T, FORM, ORDER> ev;
    ev.a = &a;
    ev.spp = stage.pp;
    ev.spc = stage.pc;
    XcdTasks tasks;
    tasks.init(a.task_ctr, ng);
    for (int g = tasks.next(); g < ng; g = tasks.next()) {
        const int64_t gf = a.gfirst[g], gc = a.gcount[g];
        double blo[3], bhi[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            blo[d] = a.gbox[6 * g + d];
            bhi[d] = a.gbox[6 * g + 3 + d];
            ev.cen[d] = a.gcen[3 * g + d];
        }
        const double hg = a.ghmax[g];
        // Lane splitting: each target gets k = floor(64 / group size) lanes;
        // lane t + gc*s (s < k) takes target t's batch entries s, s + k, ...
        // Lanes from k*gc on repeat the first copy and are left out of the sums.
        const uint32_t gcu = (uint32_t)gc;
        const uint32_t k = 64u / gcu;
        const uint32_t tl = (uint32_t)lane % gcu;
        const uint32_t sub = (uint32_t)lane / gcu;
        const bool copy = sub < k;
        ev.sub = copy ? sub : 0u;
        ev.k = k;
        const int64_t i = gf + tl;
        const bool active = a.order[i] < a.n_gas;
        uint32_t npc = 0, npp = 0;
        uint64_t cks = 0;
        if (__ballot(active) != 0ull) {   // groups of sinks only are left to the sink walk
            ev.tx = to_frame<FORM>(a.xs[i], ev.cen[0]);
            ev.ty = to_frame<FORM>(a.ys[i], ev.cen[1]);
            ev.tz = to_frame<FORM>(a.zs[i], ev.cen[2]);
            ev.th = (R)a.hs[i];
            ev.th2 = ev.th * ev.th;
            ev.thinv = rcp(ev.th);
            ev.tidx = (int32_t)i;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                ev.bl[d] = dto_frame<FORM>(blo[d], ev.cen[d]);
                ev.bh[d] = dto_frame<FORM>(bhi[d], ev.cen[d]);
            }
            {
                const R hgr = (R)hg;
                ev.hg2 = hgr * hgr;
            }
            ev.ax.zero();
            ev.ay.zero();
            ev.az.zero();
            ev.ap.zero();
            // full batches hold a multiple of k entries, so that none ends
            // with a step in which only some of the copies have an entry
            walk_task<STATS>(a.nd, L, a.gstack + (int64_t)blockIdx.x * kStack, ev, blo, bhi, hg,
                             gf, gf + gc, task_ag_group(a.nd, g), a.err, npc, npp, cks,
                             kPPBatch<R> / k * k, 64u / k * k);
            double v[4] = {ev.ax.value(), ev.ay.value(), ev.az.value(), ev.ap.value()};
            // sum the k copies of each target in a fixed order, through LDS
            // (the stage is free once the task's batches are done)
            double(*red)[64] = reinterpret_cast<double(*)[64]>(&stage);
            for (int d = 0; d < 4; ++d) red[d][lane] = v[d];
            __syncthreads();
            if ((uint32_t)lane < gcu)
                for (uint32_t c = 1; c < k; ++c)
                    for (int d = 0; d < 4; ++d) v[d] += red[d][lane + c * gcu];
            __syncthreads();
            if (active && (uint32_t)lane < gcu) {
                const int64_t o = a.order[i];
                a.acc[3 * o] = (T)(a.G * v[0]);
                a.acc[3 * o + 1] = (T)(a.G * v[1]);
                a.acc[3 * o + 2] = (T)(a.G * v[2]);
                // take out the self pair's potential term (-m P(0), added in the
                // softened loop), as the exact product of the values it used
                const double sp = (double)(R)a.ms[i] * (double)self_P<R>(ev.thinv);
                if (a.pot) a.pot[o] = (T)(a.G * (v[3] + sp));
            }
        }
        if (STATS && lane == 0) {
            a.gnpc[g] = (int32_t)npc;
            a.gnpp[g] = (int32_t)npp;
            a.gcks[g] = cks;
        }
        if (lane == 0 && a.gcost) {
            // the adjoint's steps: each of its k = floor(64 / gc) copies of
            // a target meets 1/k of the list
            const uint64_t c = ((uint64_t)3 * npc + npp) * 64u / k;
            a.gcost[g] = c > 0xffffffffull ? 0xffffffffu : (uint32_t)c;
        }
    }
}

// ---------------------------------------------------------------- sink mode

template <typename T, int FORM, int ORDER>
struct SinkEval {
    using R = typename FormT<FORM>::R;
    const WalkArgs<T> *a;
    double cen[3];
    R th, th2;
    int32_t tidx;
    Acc<FORM> ax, ay, az, ap;   // per lane partial sums

    __device__ void pc_batch(WalkLds &L, uint32_t head, uint32_t nb) {
        const int lane = threadIdx.x;
        R bx = 0, by = 0, bz = 0, bp = 0;
        if ((uint32_t)lane < nb) {
            const int node = L.pc[(head + lane) & 127];
            const WalkNodes &nd = a->nd;
            // target at the frame origin (FP32C) or at its own coordinates
            const R cx = dto_frame<FORM>(nd.w[node].com[0], cen[0]);
            const R cy = dto_frame<FORM>(nd.w[node].com[1], cen[1]);
            const R cz = dto_frame<FORM>(nd.w[node].com[2], cen[2]);
            const R tx = FormT<FORM>::rel ? R(0) : (R)cen[0];
            const R ty = FormT<FORM>::rel ? R(0) : (R)cen[1];
            const R tz = FormT<FORM>::rel ? R(0) : (R)cen[2];
            R qxx = 0, qyy = 0, qxy = 0, qxz = 0, qyz = 0;
            if (ORDER == 2) {
                qxx = (R)nd.q[node].q[0];
                qyy = (R)nd.q[node].q[1];
                qxy = (R)nd.q[node].q[2];
                qxz = (R)nd.q[node].q[3];
                qyz = (R)nd.q[node].q[4];
            }
            multipole<R, ORDER>(tx - cx, ty - cy, tz - cz, (R)nd.w[node].M, qxx, qyy, qxy, qxz, qyz,
                                -(qxx + qyy), bx, by, bz, bp);
        }
        ax.fold(bx);
        ay.fold(by);
        az.fold(bz);
        ap.fold(bp);
    }

    template <bool SOFT>
    __device__ void pp_batch(WalkLds &L, uint32_t nb) {
        const int lane = threadIdx.x;
        R bx = 0, by = 0, bz = 0, bp = 0;
        if ((uint32_t)lane < nb) {
            const int p = L.slot[lane];
            if (a->order[p] < a->n_gas) {
                const R sx = to_frame<FORM>(a->xs[p], cen[0]);
                const R sy = to_frame<FORM>(a->ys[p], cen[1]);
                const R sz = to_frame<FORM>(a->zs[p], cen[2]);
                const R tx = FormT<FORM>::rel ? R(0) : (R)cen[0];
                const R ty = FormT<FORM>::rel ? R(0) : (R)cen[1];
                const R tz = FormT<FORM>::rel ? R(0) : (R)cen[2];
                const R h = (R)a->hs[p];
                if (SOFT)
                    pair<R>(sx - tx, sy - ty, sz - tz, (R)a->ms[p], h * h, h, rcp(h), th2, th,
                            rcp(th), p == tidx, bx, by, bz, bp);
                else
                    pair_newton<R>(sx - tx, sy - ty, sz - tz, (R)a->ms[p], bx, by, bz, bp);
            }
        }
        ax.fold(bx);
        ay.fold(by);
        az.fold(bz);
        ap.fold(bp);
        __syncthreads();
    }
};

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T, int FORM, int ORDER>
__global__ __launch_bounds__(64) void k_walk_sinks(WalkArgs<T> a) {
    __shared__ WalkLds L;
    const int lane = threadIdx.x;
    SinkEval<T, FORM, ORDER> ev;
    ev.a = &a;
    for (int k = next_task(a.task_ctr); k < a.n_sink; k = next_task(a.task_ctr)) {
        const int64_t p = a.sink_pos[k];
        double b[3];
        b[0] = (double)a.xs[p];
        b[1] = (double)a.ys[p];
        b[2] = (double)a.zs[p];
        for (int d = 0; d < 3; ++d) ev.cen[d] = b[d];
        ev.th = (typename FormT<FORM>::R)a.hs[p];
        ev.th2 = ev.th * ev.th;
        ev.tidx = (int32_t)p;
        ev.ax.zero();
        ev.ay.zero();
        ev.az.zero();
        ev.ap.zero();
        uint32_t npc, npp;
        uint64_t cks;
        walk_task<false>(a.nd, L, a.gstack + (int64_t)blockIdx.x * kStack, ev, b, b,
                         (double)a.hs[p], p, p + 1, task_ag_point(a.nd, p), a.err, npc, npp, cks);
        double s[4] = {ev.ax.value(), ev.ay.value(), ev.az.value(), ev.ap.value()};
        for (int d = 0; d < 4; ++d) s[d] = wave_sum_f64(s[d]);
        if (lane == 0) {
            if (a.ss)
                for (int d = 0; d < 4; ++d) s[d] += a.ss[4 * k + d];
            const int64_t o = a.order[p];
            a.acc[3 * o] = (T)(a.G * s[0]);
            a.acc[3 * o + 1] = (T)(a.G * s[1]);
            a.acc[3 * o + 2] = (T)(a.G * s[2]);
            if (a.pot) a.pot[o] = (T)(a.G * s[3]);
        }
    }
}

// ---------------------------------------------------------------- sink-sink

// Sink records gathered once into one contiguous FP64 array (x y z m h 1/h),
// so the pair loop issues independent, coalesced loads.
template <typename T>
__global__ void k_sink_gather(const int32_t *__restrict__ sink_pos, int64_t n_sink,
                              const T *__restrict__ xs, const T *__restrict__ ys,
                              const T *__restrict__ zs, const T *__restrict__ ms,
                              const T *__restrict__ hs, double *__restrict__ rec) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_sink) return;
    const int64_t p = sink_pos[k];
    const double h = (double)hs[p];
    double *r = rec + kSinkRec * k;
    r[0] = (double)xs[p];
    r[1] = (double)ys[p];
    r[2] = (double)zs[p];
    r[3] = (double)ms[p];
    r[4] = h;
    r[5] = 1.0 / h;
}

// FP64 direct sum over sink pairs; one wave per sink target, lanes stride the
// sources; results unscaled by G.
__global__ __launch_bounds__(64) void k_sink_sink(const double *__restrict__ rec, int64_t n_sink,
                                                  double *__restrict__ ss) {
    const int lane = threadIdx.x;
    for (int64_t k = blockIdx.x; k < n_sink; k += gridDim.x) {
        const double *t = rec + kSinkRec * k;
        const double tx = t[0], ty = t[1], tz = t[2], th = t[4], thi = t[5];
        double bx = 0, by = 0, bz = 0, bp = 0;
        for (int64_t j = lane; j < n_sink; j += 64) {
            if (j == k) continue;
            const double *r = rec + kSinkRec * j;
            const double h = r[4];
            pair<double>(r[0] - tx, r[1] - ty, r[2] - tz, r[3], h * h, h, r[5], th * th, th, thi,
                         false, bx, by, bz, bp);
        }
        bx = wave_sum_f64(bx);
        by = wave_sum_f64(by);
        bz = wave_sum_f64(bz);
        bp = wave_sum_f64(bp);
        if (lane == 0) {
            ss[4 * k] = bx;
            ss[4 * k + 1] = by;
            ss[4 * k + 2] = bz;
            ss[4 * k + 3] = bp;
        }
    }
}

void sink_sink_accel(sf_grav_tree_s *t, double G, double *ss, double *rec, hipStream_t st) {
    (void)G;
    if (t->n_sink <= 0) return;
    const unsigned gb = (unsigned)((t->n_sink + 255) / 256);
    if (t->dt == SF_F32)
        hipLaunchKernelGGL(k_sink_gather<float>, dim3(gb), dim3(256), 0, st, t->sink_pos, t->n_sink,
                           (const float *)t->xs, (const float *)t->ys, (const float *)t->zs,
                           (const float *)t->ms, (const float *)t->hs, rec);
    else
        hipLaunchKernelGGL(k_sink_gather<double>, dim3(gb), dim3(256), 0, st, t->sink_pos,
                           t->n_sink, (const double *)t->xs, (const double *)t->ys,
                           (const double *)t->zs, (const double *)t->ms, (const double *)t->hs,
                           rec);
    const unsigned blocks = (unsigned)std::min<int64_t>(t->n_sink, 8192);
    hipLaunchKernelGGL(k_sink_sink, dim3(blocks), dim3(64), 0, st, (const double *)rec, t->n_sink,
                       ss);
}

// ---------------------------------------------------------------- launch

// Persistent grid of the walk kernels: 16 one-wave blocks per CU (the most
// that run at once at their register use).
int walk_grid() { return device_cu_count() * 16; }

// CU count of the current device, queried once per device (MI355X: 256, also
// the value taken if the query fails; it only sizes persistent grids).
int device_cu_count() {
    static std::atomic<int> cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int c = cus[dev].load(std::memory_order_relaxed);
    if (c == 0) {
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            c <= 0)
            c = 256;
        cus[dev].store(c, std::memory_order_relaxed);
    }
    return c;
}

// ---------------------------------------------------------------- previous field

// |g| of each sorted particle from a previous field given in caller order:
// sqrt((gx^2 + gy^2) + gz^2) in FP64, every step correctly rounded.
template <typename T>
__global__ void k_field_norm(const T *__restrict__ acc, const int32_t *__restrict__ order,
                             int64_t n, double *__restrict__ fpt) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t o = order[s];
    const double x = (double)acc[3 * o], y = (double)acc[3 * o + 1], z = (double)acc[3 * o + 2];
    fpt[s] = __dsqrt_rn(dadd(dadd(dmul(x, x), dmul(y, y)), dmul(z, z)));
}

// Smallest |g| over each group's members (all of them, as the group box).
__global__ void k_field_group(const double *__restrict__ fpt, const int32_t *__restrict__ n_groups,
                              const int32_t *__restrict__ gfirst, const int32_t *__restrict__ gcount,
                              int64_t cap, double *__restrict__ fgrp) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= cap) return;
    double v = 0.0;
    if (g < *n_groups) {
        const int64_t f = gfirst[g], c = gcount[g];
        v = fpt[f];
        for (int64_t j = 1; j < c; ++j) v = fmin(v, fpt[f + j]);
    }
    fgrp[g] = v;
}

sf_status set_field(sf_grav_tree_s *t, const void *acc_prev) {
    if (!t->fpt) {
        HandleAlloc keep(t);
        double *fpt, *fgrp;
        SF_ALLOC(keep.ar, fpt, t->n);
        SF_ALLOC(keep.ar, fgrp, t->groups_cap);
        keep.commit();
        t->fpt = fpt;
        t->fgrp = fgrp;
    }
    const unsigned nb = (unsigned)((t->n + 255) / 256);
    if (t->dt == SF_F32)
        hipLaunchKernelGGL(k_field_norm<float>, dim3(nb), dim3(256), 0, t->stream,
                           (const float *)acc_prev, t->order, t->n, t->fpt);
    else
        hipLaunchKernelGGL(k_field_norm<double>, dim3(nb), dim3(256), 0, t->stream,
                           (const double *)acc_prev, t->order, t->n, t->fpt);
    hipLaunchKernelGGL(k_field_group, dim3((unsigned)((t->groups_cap + 255) / 256)), dim3(256), 0,
                       t->stream, t->fpt, t->n_groups_dev, t->gfirst, t->gcount, t->groups_cap,
                       t->fgrp);
    SF_HIP(hipGetLastError());
    t->have_field = true;
    return SF_OK;
}

// ---------------------------------------------------------------- statistics

// One thread per group: interactions summed over the group's gas targets,
// list-length histogram (bin b: 2^b <= nodes + particles < 2^(b+1), bin 0
// also empty lists) and the combined list checksum; integer atomics only,
// so the result does not depend on their order.
__global__ void k_stats(const int32_t *__restrict__ n_groups, const int32_t *__restrict__ gfirst,
                        const int32_t *__restrict__ gcount, const int32_t *__restrict__ order,
                        int64_t n_gas, const int32_t *__restrict__ npc,
                        const int32_t *__restrict__ npp, const uint64_t *__restrict__ cks,
                        unsigned long long *__restrict__ out) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= *n_groups) return;
    const int64_t f = gfirst[g], c = gcount[g];
    uint64_t act = 0;
    for (int64_t j = 0; j < c; ++j) act += order[f + j] < n_gas ? 1u : 0u;
    atomicAdd(out + 0, (unsigned long long)(act * (uint64_t)npc[g]));
    atomicAdd(out + 1, (unsigned long long)(act * (uint64_t)npp[g]));
    atomicAdd(out + 2, (unsigned long long)list_mix(cks[g] + list_mix((uint64_t)g)));
    const uint64_t len = (uint64_t)npc[g] + (uint64_t)npp[g];
    const int bin = len <= 1 ? 0 : 63 - __clzll((long long)len);
    atomicAdd(out + 3 + (bin < 32 ? bin : 31), 1ull);
}

sf_status tree_stats(sf_grav_tree_s *t, sf_grav_stats *out) {
    DevArena ar(t->stream);
    unsigned long long *d = nullptr;
    SF_ALLOC_TMP(ar, d, 3 + 32);
    fill_u32((uint32_t *)d, 2 * (3 + 32), 0u, t->stream);
    hipLaunchKernelGGL(k_stats, dim3((unsigned)((t->groups_cap + 255) / 256)), dim3(256), 0,
                       t->stream, t->n_groups_dev, t->gfirst, t->gcount, t->order, t->n_gas,
                       t->gnpc, t->gnpp, t->gcks, d);
    unsigned long long h[3 + 32];
    uint32_t info[2] = {0, 0};
    int32_t ng = 0;
    SF_HIP(hipGetLastError());
    SF_HIP(hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, t->stream));
    SF_HIP(hipMemcpyAsync(info, t->info_dev, sizeof(info), hipMemcpyDeviceToHost, t->stream));
    SF_HIP(hipMemcpyAsync(&ng, t->n_groups_dev, sizeof(ng), hipMemcpyDeviceToHost, t->stream));
    SF_HIP(hipStreamSynchronize(t->stream));
    out->max_level = (int32_t)info[0];
    out->n_nodes = t->n_nodes;
    out->n_leaves = info[1];
    out->n_groups = ng;
    out->n_pc = (int64_t)h[0];
    out->n_pp = (int64_t)h[1];
    out->checksum = h[2];
    for (int b = 0; b < 32; ++b) out->hist[b] = (int64_t)h[3 + b];
    return SF_OK;
}

void set_relative(WalkNodes &nd, const sf_grav_tree_s *t, const EvalOpts &o) {
    nd.rel = o.alpha >= 0.0 ? 1 : 0;
    nd.G = o.G;
    nd.alpha = o.alpha;
    nd.fgrp = t->fgrp;
    nd.fpt = t->fpt;
}

template <typename T>
static WalkArgs<T> make_args(sf_grav_tree_s *t, const EvalOpts &o, int set, void *acc, void *pot,
                             int32_t *ctr, double *ss, uint32_t *gstack) {
    WalkArgs<T> a{};
    a.nd.n_nodes = t->n_nodes;
    a.nd.w = t->nw[set];
    a.nd.q = t->nq[set];
    a.nd.side = t->hframe.side;
    a.nd.th2 = o.theta * o.theta;
    set_relative(a.nd, t, o);
    a.xs = (const T *)t->xs;
    a.ys = (const T *)t->ys;
    a.zs = (const T *)t->zs;
    a.ms = (const T *)t->ms;
    a.hs = (const T *)t->hs;
    a.order = t->order;
    a.n = t->n;
    a.n_gas = t->n_gas;
    a.n_groups_dev = t->n_groups_dev;
    a.gfirst = t->gfirst;
    a.gcount = t->gcount;
    a.gbox = t->gbox;
    a.ghmax = t->ghmax;
    a.gcen = t->gcen;
    a.sink_pos = t->sink_pos;
    a.n_sink = t->n_sink;
    a.ss = ss;
    a.task_ctr = ctr;
    a.err = ctr + kCtrErr;
    a.gstack = gstack;
    a.gnpc = t->gnpc;
    a.gnpp = t->gnpp;
    a.gcks = t->gcks;
    a.gcost = set == 0 ? t->gcost : nullptr;
    a.acc = (T *)acc;
    a.pot = (T *)pot;
    a.G = o.G;
    return a;
}

// The sink walk (with the sink-sink sum before it) goes on the side stream
// first, so that its waves share the device with the group walk; each walk
// has its own task counter and stack area.
template <typename T, int FORM, int ORDER>
static void launch_walks(sf_grav_tree_s *t, const EvalOpts &o, void *acc, void *pot, int32_t *ctr,
                         double *ss, uint32_t *gstack, uint32_t *sstack, hipStream_t side,
                         bool groups) {
    const unsigned grid = (unsigned)walk_grid();
    if (t->n_sink > 0) {
        WalkArgs<T> as = make_args<T>(t, o, 1, acc, pot, ctr + kCtrSinks, ss, sstack);
        as.err = ctr + kCtrErr;
        const unsigned gs = (unsigned)std::min<int64_t>(t->n_sink, grid);
        phase_begin(t, 6, side);
        hipLaunchKernelGGL((k_walk_sinks<T, FORM, ORDER>), dim3(gs), dim3(64), 0, side, as);
        phase_end(t, 6, side);
    }
    if (!groups) return;
    WalkArgs<T> ag = make_args<T>(t, o, 0, acc, pot, ctr, ss, gstack);
    phase_begin(t, 5);
    if (o.stats)
        hipLaunchKernelGGL((k_walk_groups<T, FORM, ORDER, true>), dim3(grid), dim3(64), 0, t->stream, ag);
    else
        hipLaunchKernelGGL((k_walk_groups<T, FORM, ORDER, false>), dim3(grid), dim3(64), 0, t->stream, ag);
    phase_end(t, 5);
}

template <typename T>
static void dispatch_walks(sf_grav_tree_s *t, const EvalOpts &o, void *acc, void *pot,
                           int32_t *ctr, double *ss, uint32_t *gstack, uint32_t *sstack,
                           hipStream_t side, bool groups) {
#define SF_W(F, O) launch_walks<T, F, O>(t, o, acc, pot, ctr, ss, gstack, sstack, side, groups)
    if (o.order == 0) {
        if (o.form == SF_FP32C) SF_W(SF_FP32C, 0);
        else if (o.form == SF_FP32) SF_W(SF_FP32, 0);
        else SF_W(SF_FP64, 0);
    } else {
        if (o.form == SF_FP32C) SF_W(SF_FP32C, 2);
        else if (o.form == SF_FP32) SF_W(SF_FP32, 2);
        else SF_W(SF_FP64, 2);
    }
#undef SF_W
}

sf_status tree_accel(sf_grav_tree_s *t, const EvalOpts &o, void *acc, void *pot, DevArena &ar,
                     bool groups) {
    if (!groups && t->n_sink == 0) return SF_OK;
    int32_t *ctr = nullptr;
    double *ss = nullptr, *srec = nullptr;
    uint32_t *gstack = nullptr, *sstack = nullptr;
    SF_ALLOC_TMP(ar, ctr, kCtrWords);
    SF_ALLOC_TMP(ar, gstack, (int64_t)walk_grid() * kStack);
    fill_u32((uint32_t *)ctr, kCtrWords, 0u, t->stream);
    if (groups && o.stats) {
        if (!t->gnpc) {
            HandleAlloc keep(t);
            int32_t *npc, *npp;
            uint64_t *cks;
            SF_ALLOC(keep.ar, npc, t->groups_cap);
            SF_ALLOC(keep.ar, npp, t->groups_cap);
            SF_ALLOC(keep.ar, cks, t->groups_cap);
            keep.commit();
            t->gnpc = npc;
            t->gnpp = npp;
            t->gcks = cks;
        }
        FillRanges zero;
        zero.add(t->gnpc, t->groups_cap);
        zero.add(t->gnpp, t->groups_cap);
        zero.add(t->gcks, 2 * t->groups_cap);
        fill_ranges_u32(zero, 0u, t->stream);
        t->have_stats = true;
    }
    if (groups && !t->gcost) {   // zero beyond the groups, so a cost order is a permutation of them
        HandleAlloc keep(t);
        uint32_t *cost;
        SF_ALLOC(keep.ar, cost, t->groups_cap);
        keep.commit();
        t->gcost = cost;
        fill_u32(t->gcost, t->groups_cap, 0u, t->stream);
    }
    if (groups) t->have_cost = false;
    // every allocation precedes the fork: no early return between the fork
    // and the join
    hipStream_t side = t->stream;
    if (t->n_sink > 0) {
        SF_ALLOC_TMP(ar, ss, 4 * t->n_sink);
        SF_ALLOC_TMP(ar, srec, kSinkRec * t->n_sink);
        SF_ALLOC_TMP(ar, sstack, std::min<int64_t>(t->n_sink, walk_grid()) * kStack);
        if (hipStream_t sd = side_stream(t->device)) side = sd;
        if (side_fork(t, side) != SF_OK) side = t->stream;   // nothing queued there: run serially
        phase_begin(t, 4, side);
        sink_sink_accel(t, o.G, ss, srec, side);
        phase_end(t, 4, side);
    }
    if (t->dt == SF_F32) dispatch_walks<float>(t, o, acc, pot, ctr, ss, gstack, sstack, side, groups);
    else dispatch_walks<double>(t, o, acc, pot, ctr, ss, gstack, sstack, side, groups);
    if (t->n_sink > 0) {   // joined before any early return, so scratch outlives the side work
        sf_status st = side_join(t, side);
        if (st != SF_OK) return st;
    }
    SF_HIP(hipGetLastError());
    int32_t herr = 0;
    SF_HIP(hipMemcpyAsync(&herr, ctr + kCtrErr, sizeof(int32_t), hipMemcpyDeviceToHost, t->stream));
    SF_HIP(hipStreamSynchronize(t->stream));
    if (herr)
        return sf_fail(SF_E_INTERNAL, "tree walk stopped by a capacity guard (code %d)", herr);
    if (groups) t->have_cost = true;
    return SF_OK;
}

}  // namespace sf
