// sf_tidal.hip -- tidal tensor T = -grad grad Phi and jerk j = da/dt in the
// same tree walk as g and Phi (paper Sec. 2.2: T and j are summed in the
// same pass, from the monopole contributions of the accepted nodes and the
// spatial derivatives of the same softened kernel for particle pairs).
//
// With d = x_source - x_target, w = v_source - v_target, F and F' the
// softened force factor and its radial derivative (Newtonian beyond
// h_ij = max(h_i, h_j)):
//     T += -G m [F I + (F'/r) d d^T],      j += G m [F w + (F'/r) (d . w) d].
// A node enters with its mass, centre of mass and mass-weighted velocity
// (monopole); the acceleration and potential of the same pass keep the
// node expansion of `order`.  Sinks add an exact FP64 sum over the other
// sinks, as for g.
//
// The walk (decisions, lists) is the group walk of sf_walk.h, so the lists
// equal those of sf_grav_accel on the same handle and options.  Batch
// entries are staged in LDS; each target of the group holds floor(64 / gc)
// lanes that share its entries (lane splitting), and the copies' partial
// sums are added in a fixed order at the end of the task.
#include "sf_build.h"
#include "sf_ext.h"
#include "sf_math.h"
#include "sf_prims.h"
#include "sf_split.h"
#include "sf_walk.h"

namespace sf {

namespace {

template <typename T>
struct WalkArgsX {
    WalkNodes nd;
    const T *xs, *ys, *zs, *ms, *hs;
    const T *vx, *vy, *vz;        // sorted velocities (JERK only)
    const double *mv;             // per node: mass-weighted velocity sums (3 per node)
    const int32_t *order;
    int64_t n, n_gas;
    const int32_t *n_groups_dev, *gfirst, *gcount;
    const double *gbox, *ghmax, *gcen;
    const int32_t *sink_pos;
    int64_t n_sink;
    const double *ssx;            // sink-sink sums, kX per sink (unscaled by G), may be null
    int32_t *task_ctr, *err;
    uint32_t *gstack;
    T *acc, *pot, *tid, *jerk;    // caller order; pot/tid/jerk may be null
    double G;
};

template <typename R> struct alignas(16) XNode { R x, y, z, M, qxx, qyy, qxy, qxz, qyz, vx, vy, vz; };
template <typename R> struct alignas(16) XPart { R x, y, z, m, h, vx, vy, vz; int32_t idx; };
template <typename R> union XStage {
    XNode<R> nd[64];
    XPart<R> pp[64];
};

// Node record for the staging: centre of mass in the form's frame, mass,
// quadrupole and mass-weighted mean velocity.
template <typename T, int FORM, int ORDER, bool JERK>
__device__ __forceinline__ XNode<typename FormT<FORM>::R> stage_node(const WalkArgsX<T> &a, int node,
                                                                     const double cen[3]) {
    using R = typename FormT<FORM>::R;
    const WalkNodes &nd = a.nd;
    XNode<R> s;
    s.x = dto_frame<FORM>(nd.w[node].com[0], cen[0]);
    s.y = dto_frame<FORM>(nd.w[node].com[1], cen[1]);
    s.z = dto_frame<FORM>(nd.w[node].com[2], cen[2]);
    const double M = nd.w[node].M;
    s.M = (R)M;
    s.qxx = s.qyy = s.qxy = s.qxz = s.qyz = R(0);
    if (ORDER == 2) {
        s.qxx = (R)nd.q[node].q[0];
        s.qyy = (R)nd.q[node].q[1];
        s.qxy = (R)nd.q[node].q[2];
        s.qxz = (R)nd.q[node].q[3];
        s.qyz = (R)nd.q[node].q[4];
    }
    s.vx = s.vy = s.vz = R(0);
    if (JERK) {
        const int64_t nn = nd.n_nodes;
        s.vx = (R)(a.mv[node] / M);
        s.vy = (R)(a.mv[nn + node] / M);
        s.vz = (R)(a.mv[2 * nn + node] / M);
    }
    return s;
}

template <typename T, int FORM, int ORDER, bool JERK>
__device__ __forceinline__ void node_term(const XNode<typename FormT<FORM>::R> &s,
                                          typename FormT<FORM>::R tx, typename FormT<FORM>::R ty,
                                          typename FormT<FORM>::R tz, typename FormT<FORM>::R tvx,
                                          typename FormT<FORM>::R tvy, typename FormT<FORM>::R tvz,
                                          typename FormT<FORM>::R (&b)[kX]) {
    using R = typename FormT<FORM>::R;
    // g and phi with the node expansion of ORDER (r = target - centre of mass)
    multipole<R, ORDER>(tx - s.x, ty - s.y, tz - s.z, s.M, s.qxx, s.qyy, s.qxy, s.qxz, s.qyz,
                        -(s.qxx + s.qyy), b[0], b[1], b[2], b[3]);
    // T and j from the monopole.  Every tidal and jerk term is even in the
    // separation (products of two of its components, and (d.w) d), so the
    // expansion's r = target - centre of mass serves for d = -r exactly, and
    // r, r^2 and 1/r are the ones computed for the expansion.
    const R dx = tx - s.x, dy = ty - s.y, dz = tz - s.z;
    const R r2 = dx * dx + dy * dy + dz * dz;
    const R ri = rsq(r2);
    const R mF = s.M * ri * ri * ri;
    const R mR = R(-3) * mF * ri * ri;
    ext_term<R, JERK>(dx, dy, dz, s.vx - tvx, s.vy - tvy, s.vz - tvz, mF, mR, R(0), b, false);
}

// Group tasks: lane t + gc*s holds copy s of target t of the group.
template <typename T, int FORM, int ORDER, bool JERK>
struct GroupEvalX {
    using R = typename FormT<FORM>::R;
    const WalkArgsX<T> *a;
    XStage<R> *st;
    double cen[3];
    R tx, ty, tz, th, tvx, tvy, tvz;
    R bl[3], bh[3], hg2;        // group box in the form's frame, largest h squared
    int32_t tidx;
    bool on;                    // this lane holds a gas target
    Split sp;
    Acc<FORM> acc[kX];

    __device__ void fold(const R (&b)[kX]) {
#pragma unroll
        for (int c = 0; c < kX; ++c) acc[c].fold(b[c]);
    }

    __device__ void pc_batch(WalkLds &L, uint32_t head, uint32_t nb) {
        const uint32_t e = threadIdx.x;
        if (e < nb) st->nd[e] = stage_node<T, FORM, ORDER, JERK>(*a, L.pc[(head + e) & 127], cen);
        __syncthreads();
        R b[kX] = {};
        if (on)
            sp.each(nb, [&](uint32_t j) {
                node_term<T, FORM, ORDER, JERK>(st->nd[j], tx, ty, tz, tvx, tvy, tvz, b);
            });
        fold(b);
        __syncthreads();
    }

    // Particle batches (nb <= 64).  A SOFT batch (leaves that may hold
    // softened pairs) is split per source as in the force walk: a source
    // farther from the group box than max(its h, the group's largest h), with
    // a relative margin for the rounding of both distances, has only
    // Newtonian pairs with the group; the others (the task's own particles
    // among them) are staged first and take the softened form.
    template <bool SOFT>
    __device__ void pp_batch(WalkLds &L, uint32_t nb) {
        const uint32_t e = threadIdx.x;
        XPart<R> s;
        bool soft = false;
        if (e < nb) {
            const int p = L.slot[e];
            s.x = to_frame<FORM>(a->xs[p], cen[0]);
            s.y = to_frame<FORM>(a->ys[p], cen[1]);
            s.z = to_frame<FORM>(a->zs[p], cen[2]);
            s.m = (R)a->ms[p];
            s.h = (R)a->hs[p];
            s.vx = s.vy = s.vz = R(0);
            if (JERK) {
                s.vx = (R)a->vx[p];
                s.vy = (R)a->vy[p];
                s.vz = (R)a->vz[p];
            }
            s.idx = p;
            if (SOFT) {
                const R gx = fmax(fmax(bl[0] - s.x, s.x - bh[0]), R(0));
                const R gy = fmax(fmax(bl[1] - s.y, s.y - bh[1]), R(0));
                const R gz = fmax(fmax(bl[2] - s.z, s.z - bh[2]), R(0));
                const R d2 = gx * gx + gy * gy + gz * gz;
                soft = !(d2 > pos_max(s.h * s.h, hg2) * R(1.0001));
            }
        }
        uint32_t ns = 0;   // entries [0, ns) may hold softened pairs
        if (SOFT) {
            const uint64_t msoft = __ballot(e < nb && soft);
            const uint64_t mnewt = __ballot(e < nb && !soft);
            const uint64_t lt = lane_mask_lt();
            ns = (uint32_t)popc64(msoft);
            if (e < nb) st->pp[soft ? popc64(msoft & lt) : ns + popc64(mnewt & lt)] = s;
        } else if (e < nb) {
            st->pp[e] = s;
        }
        __syncthreads();
        R b[kX] = {};
        if (on) {
            sp.each(nb - ns, [&](uint32_t j) {
                const XPart<R> q = st->pp[ns + j];
                ext_pair<R, JERK, false>(q.x - tx, q.y - ty, q.z - tz, q.vx - tvx, q.vy - tvy,
                                         q.vz - tvz, q.m, q.h, th, false, b);
            });
            if (SOFT)
                sp.each(ns, [&](uint32_t j) {
                    const XPart<R> q = st->pp[j];
                    ext_pair<R, JERK, true>(q.x - tx, q.y - ty, q.z - tz, q.vx - tvx, q.vy - tvy,
                                            q.vz - tvz, q.m, q.h, th, q.idx == tidx, b);
                });
        }
        fold(b);
        __syncthreads();
    }
};

template <typename T>
__device__ __forceinline__ void write_out(const WalkArgsX<T> &a, int64_t o, const double (&v)[kX]) {
    const double G = a.G;
    a.acc[3 * o] = (T)(G * v[0]);
    a.acc[3 * o + 1] = (T)(G * v[1]);
    a.acc[3 * o + 2] = (T)(G * v[2]);
    if (a.pot) a.pot[o] = (T)(G * v[3]);
    if (a.tid)
        for (int c = 0; c < 6; ++c) a.tid[6 * o + c] = (T)(G * v[4 + c]);
    if (a.jerk)
        for (int c = 0; c < 3; ++c) a.jerk[3 * o + c] = (T)(G * v[10 + c]);
}

template <typename T, int FORM, int ORDER, bool JERK>
__global__ __launch_bounds__(64) void k_walk_groups_x(WalkArgsX<T> a) {
    using R = typename FormT<FORM>::R;
    __shared__ WalkLds L;
    __shared__ XStage<R> stage;
    const int lane = threadIdx.x;
    const int ng = __builtin_amdgcn_readfirstlane(*a.n_groups_dev);
    GroupEvalX<T, FORM, ORDER, JERK> ev;
    ev.a = &a;
    ev.st = &stage;
    XcdTasks tasks;
    tasks.init(a.task_ctr, ng);
    for (int g = tasks.next(); g < ng; g = tasks.next()) {
        const int64_t gf = a.gfirst[g], gc = a.gcount[g];
        double blo[3], bhi[3];
        for (int d = 0; d < 3; ++d) {
            blo[d] = a.gbox[6 * g + d];
            bhi[d] = a.gbox[6 * g + 3 + d];
            ev.cen[d] = a.gcen[3 * g + d];
        }
        ev.sp.init((uint32_t)gc, (uint32_t)lane);
        const int64_t i = gf + ev.sp.tl;
        ev.on = a.order[i] < a.n_gas;
        if (__ballot(ev.on) == 0ull) continue;   // sinks only: left to the sink walk
        ev.tx = to_frame<FORM>(a.xs[i], ev.cen[0]);
        ev.ty = to_frame<FORM>(a.ys[i], ev.cen[1]);
        ev.tz = to_frame<FORM>(a.zs[i], ev.cen[2]);
        ev.th = (R)a.hs[i];
        ev.tvx = ev.tvy = ev.tvz = R(0);
        if (JERK) {
            ev.tvx = (R)a.vx[i];
            ev.tvy = (R)a.vy[i];
            ev.tvz = (R)a.vz[i];
        }
        ev.tidx = (int32_t)i;
        for (int d = 0; d < 3; ++d) {
            ev.bl[d] = dto_frame<FORM>(blo[d], ev.cen[d]);
            ev.bh[d] = dto_frame<FORM>(bhi[d], ev.cen[d]);
        }
        {
            const R hgr = (R)a.ghmax[g];
            ev.hg2 = hgr * hgr;
        }
        for (int c = 0; c < kX; ++c) ev.acc[c].zero();
        uint32_t npc, npp;
        uint64_t cks;
        // full batches hold a multiple of the copy count (no partial last step)
        const uint32_t kb = 64u / ev.sp.k * ev.sp.k;
        walk_task<false>(a.nd, L, a.gstack + (int64_t)blockIdx.x * kStack, ev, blo, bhi,
                         a.ghmax[g], gf, gf + gc, task_ag_group(a.nd, g), a.err, npc, npp, cks,
                         kb, kb);
        double v[kX];
        for (int c = 0; c < kX; ++c) v[c] = ev.acc[c].value();
        // the stage is free once the task's batches are done
        ev.sp.template reduce<sizeof(XStage<R>) / (64 * sizeof(double))>(
            v, reinterpret_cast<double *>(&stage), (uint32_t)lane);
        if (ev.on && (uint32_t)lane < ev.sp.gc) write_out(a, a.order[i], v);
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sink tasks: one sink, lanes spread over each batch's entries, node moments
// over gas only, sink sources skipped (they come from the FP64 sink sum).
template <typename T, int FORM, int ORDER, bool JERK>
struct SinkEvalX {
    using R = typename FormT<FORM>::R;
    const WalkArgsX<T> *a;
    double cen[3];
    R th, tvx, tvy, tvz;
    int32_t tidx;
    Acc<FORM> acc[kX];

    __device__ void fold(const R (&b)[kX]) {
#pragma unroll
        for (int c = 0; c < kX; ++c) acc[c].fold(b[c]);
    }

    __device__ void pc_batch(WalkLds &L, uint32_t head, uint32_t nb) {
        R b[kX] = {};
        if (threadIdx.x < nb) {
            const XNode<R> s = stage_node<T, FORM, ORDER, JERK>(*a, L.pc[(head + threadIdx.x) & 127],
                                                                cen);
            const R t0 = FormT<FORM>::rel ? R(0) : (R)cen[0];
            const R t1 = FormT<FORM>::rel ? R(0) : (R)cen[1];
            const R t2 = FormT<FORM>::rel ? R(0) : (R)cen[2];
            node_term<T, FORM, ORDER, JERK>(s, t0, t1, t2, tvx, tvy, tvz, b);
        }
        fold(b);
    }

    template <bool SOFT>
    __device__ void pp_batch(WalkLds &L, uint32_t nb) {
        R b[kX] = {};
        if (threadIdx.x < nb) {
            const int p = L.slot[threadIdx.x];
            if (a->order[p] < a->n_gas) {
                const R t0 = FormT<FORM>::rel ? R(0) : (R)cen[0];
                const R t1 = FormT<FORM>::rel ? R(0) : (R)cen[1];
                const R t2 = FormT<FORM>::rel ? R(0) : (R)cen[2];
                R wx = R(0), wy = R(0), wz = R(0);
                if (JERK) {
                    wx = (R)a->vx[p] - tvx;
                    wy = (R)a->vy[p] - tvy;
                    wz = (R)a->vz[p] - tvz;
                }
                ext_pair<R, JERK>(to_frame<FORM>(a->xs[p], cen[0]) - t0,
                                  to_frame<FORM>(a->ys[p], cen[1]) - t1,
                                  to_frame<FORM>(a->zs[p], cen[2]) - t2, wx, wy, wz, (R)a->ms[p],
                                  (R)a->hs[p], th, p == tidx, b);
            }
        }
        fold(b);
        __syncthreads();
    }
};

template <typename T, int FORM, int ORDER, bool JERK>
__global__ __launch_bounds__(64) void k_walk_sinks_x(WalkArgsX<T> a) {
    __shared__ WalkLds L;
    using R = typename FormT<FORM>::R;
    SinkEvalX<T, FORM, ORDER, JERK> ev;
    ev.a = &a;
    for (int k = next_task(a.task_ctr); k < a.n_sink; k = next_task(a.task_ctr)) {
        const int64_t p = a.sink_pos[k];
        double b[3] = {(double)a.xs[p], (double)a.ys[p], (double)a.zs[p]};
        for (int d = 0; d < 3; ++d) ev.cen[d] = b[d];
        ev.th = (R)a.hs[p];
        ev.tvx = ev.tvy = ev.tvz = R(0);
        if (JERK) {
            ev.tvx = (R)a.vx[p];
            ev.tvy = (R)a.vy[p];
            ev.tvz = (R)a.vz[p];
        }
        ev.tidx = (int32_t)p;
        for (int c = 0; c < kX; ++c) ev.acc[c].zero();
        uint32_t npc, npp;
        uint64_t cks;
        walk_task<false>(a.nd, L, a.gstack + (int64_t)blockIdx.x * kStack, ev, b, b,
                         (double)a.hs[p], p, p + 1, task_ag_point(a.nd, p), a.err, npc, npp, cks);
        double v[kX];
        for (int c = 0; c < kX; ++c) v[c] = wave_sum(ev.acc[c].value());
        if (threadIdx.x == 0) {
            if (a.ssx)
                for (int c = 0; c < kX; ++c) v[c] += a.ssx[kX * k + c];
            write_out(a, a.order[p], v);
        }
    }
}

// FP64 sink-sink sum of g, phi, T and j: one wave per sink target, lanes
// stride the other sinks.
template <typename T, bool JERK>
__global__ __launch_bounds__(64) void k_sink_sink_x(const int32_t *__restrict__ sink_pos,
                                                    int64_t n_sink, const T *__restrict__ xs,
                                                    const T *__restrict__ ys,
                                                    const T *__restrict__ zs,
                                                    const T *__restrict__ ms,
                                                    const T *__restrict__ hs,
                                                    const T *__restrict__ vx,
                                                    const T *__restrict__ vy,
                                                    const T *__restrict__ vz,
                                                    double *__restrict__ ssx) {
    for (int64_t k = blockIdx.x; k < n_sink; k += gridDim.x) {
        const int64_t p = sink_pos[k];
        const double tx = (double)xs[p], ty = (double)ys[p], tz = (double)zs[p];
        const double th = (double)hs[p];
        double tv[3] = {0.0, 0.0, 0.0};
        if (JERK) {
            tv[0] = (double)vx[p];
            tv[1] = (double)vy[p];
            tv[2] = (double)vz[p];
        }
        double b[kX] = {};
        for (int64_t j = threadIdx.x; j < n_sink; j += 64) {
            if (j == k) continue;
            const int64_t q = sink_pos[j];
            double w[3] = {0.0, 0.0, 0.0};
            if (JERK) {
                w[0] = (double)vx[q] - tv[0];
                w[1] = (double)vy[q] - tv[1];
                w[2] = (double)vz[q] - tv[2];
            }
            ext_pair<double, JERK>((double)xs[q] - tx, (double)ys[q] - ty, (double)zs[q] - tz, w[0],
                                   w[1], w[2], (double)ms[q], (double)hs[q], th, false, b);
        }
        for (int c = 0; c < kX; ++c) b[c] = wave_sum(b[c]);
        if (threadIdx.x == 0)
            for (int c = 0; c < kX; ++c) ssx[kX * k + c] = b[c];
    }
}

// Velocities to sorted order (SoA).
template <typename T>
__global__ void k_gather_vel(const T *__restrict__ vel, const int32_t *__restrict__ order,
                             int64_t n, T *__restrict__ vx, T *__restrict__ vy,
                             T *__restrict__ vz) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t o = order[s];
    vx[s] = vel[3 * o];
    vy[s] = vel[3 * o + 1];
    vz[s] = vel[3 * o + 2];
}

// Mass-weighted velocity sums per node, bottom up: leaves sum their
// particles (gas only for set 1), inner nodes their children, one launch per
// level from the deepest up.  FP64, fixed order (deterministic).
template <typename T>
__global__ void k_vmom_leaf(int64_t nn, const int32_t *__restrict__ nfirst,
                            const int32_t *__restrict__ ncount, const int32_t *__restrict__ nnchild,
                            const T *__restrict__ ms, const T *__restrict__ vx,
                            const T *__restrict__ vy, const T *__restrict__ vz,
                            const int32_t *__restrict__ order, int64_t n_gas, int gas_only,
                            double *__restrict__ mv) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn || nnchild[k] != 0) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    const int64_t f = nfirst[k], c = ncount[k];
    for (int64_t p = f; p < f + c; ++p) {
        if (gas_only && order[p] >= n_gas) continue;
        const double m = (double)ms[p];
        s0 += m * (double)vx[p];
        s1 += m * (double)vy[p];
        s2 += m * (double)vz[p];
    }
    mv[k] = s0;
    mv[nn + k] = s1;
    mv[2 * nn + k] = s2;
}

__global__ void k_vmom_level(int64_t k0, int64_t k1, int64_t nn, const int32_t *__restrict__ nchild,
                             const int32_t *__restrict__ nnchild, double *__restrict__ mv) {
    const int64_t k = k0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= k1 || nnchild[k] == 0) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    const int64_t c0 = nchild[k], c1 = c0 + nnchild[k];
    for (int64_t ch = c0; ch < c1; ++ch) {
        s0 += mv[ch];
        s1 += mv[nn + ch];
        s2 += mv[2 * nn + ch];
    }
    mv[k] = s0;
    mv[nn + k] = s1;
    mv[2 * nn + k] = s2;
}

unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename T>
void node_velocities(sf_grav_tree_s *t, const T *vx, const T *vy, const T *vz, int gas_only,
                     double *mv) {
    hipStream_t s = t->stream;
    const int64_t nn = t->n_nodes;
    hipLaunchKernelGGL(k_vmom_leaf<T>, dim3(nblk(nn)), dim3(256), 0, s, nn, t->nfirst, t->ncount,
                       t->nnchild, (const T *)t->ms, vx, vy, vz, t->order, t->n_gas, gas_only, mv);
    for (int l = kLevels - 1; l >= 0; --l) {
        const int64_t k0 = t->level_off[l], k1 = t->level_off[l + 1];
        if (k1 <= k0 || t->level_off[l + 2] <= k1) continue;   // no nodes, or no children below
        hipLaunchKernelGGL(k_vmom_level, dim3(nblk(k1 - k0)), dim3(256), 0, s, k0, k1, nn,
                           t->nchild, t->nnchild, mv);
    }
}

template <typename T>
WalkArgsX<T> make_args_x(sf_grav_tree_s *t, const EvalOpts &o, int set, const T *v3[3],
                         const double *mv, int32_t *ctr, uint32_t *gstack, const double *ssx,
                         void *acc, void *pot, void *tid, void *jerk) {
    WalkArgsX<T> a{};
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
    a.vx = v3[0];
    a.vy = v3[1];
    a.vz = v3[2];
    a.mv = mv;
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
    a.ssx = ssx;
    a.task_ctr = ctr;
    a.err = ctr + kCtrErr;
    a.gstack = gstack;
    a.acc = (T *)acc;
    a.pot = (T *)pot;
    a.tid = (T *)tid;
    a.jerk = (T *)jerk;
    a.G = o.G;
    return a;
}

template <typename T, int FORM, int ORDER, bool JERK>
void launch_x(sf_grav_tree_s *t, const WalkArgsX<T> &ag, const WalkArgsX<T> &as) {
    const unsigned grid = (unsigned)walk_grid();
    hipLaunchKernelGGL((k_walk_groups_x<T, FORM, ORDER, JERK>), dim3(grid), dim3(64), 0, t->stream,
                       ag);
    if (t->n_sink > 0) {
        const unsigned gs = (unsigned)std::min<int64_t>(t->n_sink, grid);
        hipLaunchKernelGGL((k_walk_sinks_x<T, FORM, ORDER, JERK>), dim3(gs), dim3(64), 0,
                           t->stream, as);
    }
}

template <typename T, bool JERK>
void dispatch_x(sf_grav_tree_s *t, const EvalOpts &o, const WalkArgsX<T> &ag,
                const WalkArgsX<T> &as) {
    if (o.order == 0) {
        if (o.form == SF_FP32C) launch_x<T, SF_FP32C, 0, JERK>(t, ag, as);
        else if (o.form == SF_FP32) launch_x<T, SF_FP32, 0, JERK>(t, ag, as);
        else launch_x<T, SF_FP64, 0, JERK>(t, ag, as);
    } else {
        if (o.form == SF_FP32C) launch_x<T, SF_FP32C, 2, JERK>(t, ag, as);
        else if (o.form == SF_FP32) launch_x<T, SF_FP32, 2, JERK>(t, ag, as);
        else launch_x<T, SF_FP64, 2, JERK>(t, ag, as);
    }
}

template <typename T>
sf_status tidal_run(sf_grav_tree_s *t, const EvalOpts &o, const void *vel, void *acc, void *pot,
                    void *tid, void *jerk, DevArena &ar) {
    hipStream_t s = t->stream;
    const int64_t n = t->n, nn = t->n_nodes;
    const bool jk = jerk != nullptr;
    int32_t *ctr;
    uint32_t *gstack, *sstack = nullptr;
    T *vx = nullptr, *vy = nullptr, *vz = nullptr;
    double *mv0 = nullptr, *mv1 = nullptr, *ssx = nullptr;
    SF_ALLOC_TMP(ar, ctr, kCtrWords);
    SF_ALLOC_TMP(ar, gstack, (int64_t)walk_grid() * kStack);
    if (jk) {
        SF_ALLOC_TMP(ar, vx, n);
        SF_ALLOC_TMP(ar, vy, n);
        SF_ALLOC_TMP(ar, vz, n);
        SF_ALLOC_TMP(ar, mv0, 3 * nn);
        if (t->n_sink > 0) SF_ALLOC_TMP(ar, mv1, 3 * nn);
    }
    if (t->n_sink > 0) {
        SF_ALLOC_TMP(ar, ssx, kX * t->n_sink);
        SF_ALLOC_TMP(ar, sstack, std::min<int64_t>(t->n_sink, walk_grid()) * kStack);
    }
    fill_u32((uint32_t *)ctr, kCtrWords, 0u, s);
    if (jk) {
        hipLaunchKernelGGL(k_gather_vel<T>, dim3(nblk(n)), dim3(256), 0, s, (const T *)vel,
                           t->order, n, vx, vy, vz);
        node_velocities<T>(t, vx, vy, vz, 0, mv0);
        if (t->n_sink > 0) node_velocities<T>(t, vx, vy, vz, 1, mv1);
    }
    if (t->n_sink > 0) {
        const unsigned b = (unsigned)std::min<int64_t>(t->n_sink, 8192);
        if (jk)
            hipLaunchKernelGGL((k_sink_sink_x<T, true>), dim3(b), dim3(64), 0, s, t->sink_pos,
                               t->n_sink, (const T *)t->xs, (const T *)t->ys, (const T *)t->zs,
                               (const T *)t->ms, (const T *)t->hs, vx, vy, vz, ssx);
        else
            hipLaunchKernelGGL((k_sink_sink_x<T, false>), dim3(b), dim3(64), 0, s, t->sink_pos,
                               t->n_sink, (const T *)t->xs, (const T *)t->ys, (const T *)t->zs,
                               (const T *)t->ms, (const T *)t->hs, vx, vy, vz, ssx);
    }
    const T *v3[3] = {vx, vy, vz};
    WalkArgsX<T> ag = make_args_x<T>(t, o, 0, v3, mv0, ctr, gstack, nullptr, acc, pot, tid, jerk);
    WalkArgsX<T> as = make_args_x<T>(t, o, 1, v3, mv1, ctr + kCtrSinks, sstack, ssx, acc, pot, tid,
                                     jerk);
    as.err = ctr + kCtrErr;
    if (jk) dispatch_x<T, true>(t, o, ag, as);
    else dispatch_x<T, false>(t, o, ag, as);
    SF_HIP(hipGetLastError());
    int32_t herr = 0;
    SF_HIP(hipMemcpyAsync(&herr, ctr + kCtrErr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SF_HIP(hipStreamSynchronize(s));
    if (herr)
        return sf_fail(SF_E_INTERNAL, "tree walk stopped by a capacity guard (code %d)", herr);
    return SF_OK;
}

}  // namespace

sf_status tidal_accel(sf_grav_tree_s *t, const EvalOpts &o, const void *vel, void *acc, void *pot,
                      void *tid, void *jerk, DevArena &ar) {
    if (t->dt == SF_F32) return tidal_run<float>(t, o, vel, acc, pot, tid, jerk, ar);
    return tidal_run<double>(t, o, vel, acc, pot, tid, jerk, ar);
}

}  // namespace sf
