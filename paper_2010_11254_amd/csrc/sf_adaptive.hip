// sf_adaptive.hip -- gas-gas pairs with the symmetrised adaptive softening of
// Sec. 2.2.1 (gas softening follows each cell's kernel radius, with the
// symmetrisation and extra terms that keep momentum and energy conserved),
// on the tree of a handle.
//
// Gas-gas pairs use the average of the two cells' softened kernels,
// F_ij = (F(r, h_i) + F(r, h_j)) / 2 and P_ij likewise, and the acceleration
// of gas cell i gains
//     -(G/2) sum_j [z_i W_r(r, h_i) + (m_j/m_i) z_j W_r(r, h_j)] d / r,
// z = zeta / Omega, W the M4 cubic spline of support h normalised to 1,
// W_r = dW/dr, with, for the number density n_i = sum_j W(r_ij, h_i) (self
// included) of the constraint (4 pi/3) h_i^3 n_i = N_NGB:
//     zeta_i  = (dh_i/dn_i) sum_{j != i} m_j dP(r_ij, h_i)/dh,
//     Omega_i = 1 - (dh_i/dn_i) sum_j dW(r_ij, h_i)/dh,   dh/dn = -h/(3 n).
// These terms make the force the exact gradient of the total potential
// energy when every h_i follows the constraint (the caller's kernel radii
// are taken to satisfy it).  Gas-sink and sink-sink pairs keep the
// larger-radius rule.
//
// Two walks over the handle's groups: the first sums n, dW/dh and m dP/dh
// over each gas cell's neighbours, walking only the nodes that can hold a
// softened pair (the near leaves of sf_grav_accel's lists, reached without
// the far traversal); the second, with sf_grav_accel's decisions, evaluates
// the forces with every source's z from the first.  Each
// target holds floor(64 / gc) lanes that share its batch entries (lane
// splitting); sinks get their fields from the sink walk of sf_grav_accel.
#include "sf_build.h"
#include "sf_math.h"
#include "sf_prims.h"
#include "sf_split.h"
#include "sf_walk.h"

namespace sf {

namespace {

// M4 cubic spline normalised to 1 on a ball of radius h, for r < h: W, dW/dr
// and dW/dh.
template <typename R>
__device__ __forceinline__ void m4(R r, R hinv, R &W, R &Wr, R &Wh) {
    const R u = r * hinv;
    const R om = R(1) - u;
    const bool in = u < R(0.5);
    const R k = in ? R(1) + u * u * (R(-6) + R(6) * u) : R(2) * om * om * om;
    const R dk = in ? u * (R(-12) + R(18) * u) : R(-6) * om * om;
    const R c = R(8.0 / 3.14159265358979323846) * hinv * hinv * hinv;
    W = c * k;
    Wr = c * hinv * dk;
    Wh = -c * hinv * (R(3) * k + u * dk);
}

// Softened F and P of the M4 spline with support h (Newtonian at and beyond
// h) and the spline's radial derivative W_r = dW/dr (zero beyond h), from
// the pair's r^2, ri = rsq(r^2), r, h and 1/h.  Both spline pieces are
// evaluated and one is selected, so lanes on different pieces follow one
// instruction stream; the outer piece's 1/u is h ri (capped at 2, its value
// at u = 1/2), so no further reciprocal or square root is needed.
template <typename R>
__device__ __forceinline__ void sym_soft(R r2, R ri, R r, R h, R hinv, R &F, R &P, R &Wr) {
    const R u = r * hinv;
    const R u2 = u * u;
    const R hinv2 = hinv * hinv;
    const R hinv3 = hinv2 * hinv;
    const R us = u > R(0.5) ? u : R(0.5);
    const R iu = pos_min(h * ri, R(2));
    const R Fi = R(32.0 / 3.0) + u2 * (R(-192.0 / 5.0) + R(32.0) * u);
    const R Pi = R(14.0 / 5.0) + u2 * (R(-16.0 / 3.0) + u2 * (R(48.0 / 5.0) + R(-32.0 / 5.0) * u));
    const R Fo = R(64.0 / 3.0) + us * (R(-48.0) + us * (R(192.0 / 5.0) + us * R(-32.0 / 3.0))) -
                 R(1.0 / 15.0) * iu * iu * iu;
    const R Po = R(16.0 / 5.0) - R(1.0 / 15.0) * iu +
                 us * us * (R(-32.0 / 3.0) + us * (R(16.0) + us * (R(-48.0 / 5.0) + us * R(32.0 / 15.0))));
    const R om = R(1) - us;
    const R dk = u < R(0.5) ? u * (R(-12) + R(18) * u) : R(-6) * om * om;
    const bool inner = u < R(0.5);
    const bool inside = r2 < h * h;
    F = inside ? (inner ? Fi : Fo) * hinv3 : ri * ri * ri;
    P = inside ? (inner ? Pi : Po) * hinv : ri;
    Wr = inside ? R(8.0 / 3.14159265358979323846) * hinv2 * hinv2 * dk : R(0);
}

template <typename T>
struct AdArgs {
    WalkNodes nd;
    const T *xs, *ys, *zs, *ms, *hs;
    const int32_t *order;
    int64_t n, n_gas;
    const int32_t *n_groups_dev, *gfirst, *gcount;
    const double *gbox, *ghmax, *gcen;
    int32_t *task_ctr, *err;
    uint32_t *gstack;
    double *z;                 // per sorted particle: zeta / Omega (0 for sinks)
    T *acc, *pot, *aux;        // caller order; pot and aux (Omega, zeta) may be null
    double G;
};

template <typename R> struct alignas(16) AdPart { R x, y, z, m, h, zz; int32_t idx, gas; };
template <typename R> struct alignas(16) AdNode { R x, y, z, M, q[5]; };
// Particle batches of the force pass hold up to kPPBatch<R> entries (128 in
// the FP32 forms, as in the force walk); the neighbour sums use 64.
template <typename R> union AdStage {
    AdPart<R> pp[kPPBatch<R>];
    AdNode<R> nd[64];
};
// the copies' partial sums (up to 4 per lane) go through the stage
static_assert(sizeof(AdStage<float>) >= 4 * 64 * sizeof(double), "stage too small for the sums");

// Pass 1: neighbour sums of every gas target.
template <typename T, int FORM>
struct SumsEval {
    using R = typename FormT<FORM>::R;
    const AdArgs<T> *a;
    AdStage<R> *st;
    double cen[3];
    R tx, ty, tz, th, thinv;
    int32_t tidx;
    bool on;
    Split sp;
    R sW, sWh, sPh;

    __device__ void pc_batch(WalkLds &, uint32_t, uint32_t) {}

    template <bool SOFT>
    __device__ void pp_batch(WalkLds &L, uint32_t nb) {
        if (!SOFT) return;   // leaves with Newtonian pairs only hold no neighbours
        const uint32_t e = threadIdx.x;
        if (e < nb) {
            const int p = L.slot[e];
            AdPart<R> s;
            s.x = to_frame<FORM>(a->xs[p], cen[0]);
            s.y = to_frame<FORM>(a->ys[p], cen[1]);
            s.z = to_frame<FORM>(a->zs[p], cen[2]);
            s.m = (R)a->ms[p];
            s.h = s.zz = R(0);
            s.idx = p;
            s.gas = a->order[p] < a->n_gas ? 1 : 0;
            st->pp[e] = s;
        }
        __syncthreads();
        if (on)
            sp.each(nb, [&](uint32_t j) {
                const AdPart<R> s = st->pp[j];
                const R dx = s.x - tx, dy = s.y - ty, dz = s.z - tz;
                const R r2 = dx * dx + dy * dy + dz * dz;
                if (!s.gas || !(r2 < th * th)) return;
                const R ri = rsq(r2);
                const R r = r_of(r2, ri);
                R W, Wr, Wh;
                m4<R>(r, thinv, W, Wr, Wh);
                sW += W;
                sWh += Wh;
                if (s.idx != tidx) {   // r < h here: the softened factors, branch-free
                    R F, P, FrR, dFh, Ph;
                    dsoft_ri<R>(r2, ri, th, thinv, F, P, FrR, dFh, Ph);
                    sPh += s.m * Ph;
                }
            });
        __syncthreads();
    }
};

// Pass 2: forces with the symmetrised gas-gas law.
template <typename T, int FORM, int ORDER>
struct ForceEval {
    using R = typename FormT<FORM>::R;
    const AdArgs<T> *a;
    AdStage<R> *st;
    double cen[3];
    R tx, ty, tz, th, thinv, tminv, tz_;   // tminv = 1/m of the target; tz_: its zeta / Omega
    R bl[3], bh[3], hg2;            // group box in the form's frame, largest h squared
    int32_t tidx;
    bool on;
    Split sp;
    Acc<FORM> ax, ay, az, ap;

    __device__ void pc_batch(WalkLds &L, uint32_t head, uint32_t nb) {
        const uint32_t e = threadIdx.x;
        if (e < nb) {
            const int node = L.pc[(head + e) & 127];
            const WalkNodes &nd = a->nd;
            AdNode<R> s;
            s.x = dto_frame<FORM>(nd.w[node].com[0], cen[0]);
            s.y = dto_frame<FORM>(nd.w[node].com[1], cen[1]);
            s.z = dto_frame<FORM>(nd.w[node].com[2], cen[2]);
            s.M = (R)nd.w[node].M;
            for (int d = 0; d < 5; ++d) s.q[d] = ORDER == 2 ? (R)nd.q[node].q[d] : R(0);
            st->nd[e] = s;
        }
        __syncthreads();
        R bx = 0, by = 0, bz = 0, bp = 0;
        if (on)
            sp.each(nb, [&](uint32_t j) {
                const AdNode<R> s = st->nd[j];
                multipole<R, ORDER>(tx - s.x, ty - s.y, tz - s.z, s.M, s.q[0], s.q[1], s.q[2],
                                    s.q[3], s.q[4], -(s.q[0] + s.q[1]), bx, by, bz, bp);
            });
        ax.fold(bx);
        ay.fold(by);
        az.fold(bz);
        ap.fold(bp);
        __syncthreads();
    }

    // Particle batches (nb <= kPPBatch<R>), staged 64 entries per round.  A
    // SOFT batch (leaves that may hold softened pairs) is split per source as
    // in the force walk: a source farther from the group box than max(its h,
    // the group's largest h), with a relative margin for the rounding of both
    // distances, is beyond both softening lengths of every pair it forms with
    // the group, so its terms are Newtonian with no extra term; the others
    // (the task's own particles among them) fill the stage from the start and
    // take the symmetrised law, the Newtonian ones fill it from the end.
    template <bool SOFT>
    __device__ void pp_batch(WalkLds &L, uint32_t nb) {
        uint32_t ns = 0, nn = 0;   // entries [0, ns) may hold softened pairs
        for (uint32_t r = 0; r < nb; r += 64u) {
            const uint32_t e = r + threadIdx.x;
            AdPart<R> s;
            bool soft = false;
            if (e < nb) {
                const int p = L.slot[e];
                s.x = to_frame<FORM>(a->xs[p], cen[0]);
                s.y = to_frame<FORM>(a->ys[p], cen[1]);
                s.z = to_frame<FORM>(a->zs[p], cen[2]);
                s.m = (R)a->ms[p];
                s.h = (R)a->hs[p];
                s.zz = (R)a->z[p];
                s.idx = p;
                s.gas = a->order[p] < a->n_gas ? 1 : 0;
                if (SOFT) {
                    const R gx = fmax(fmax(bl[0] - s.x, s.x - bh[0]), R(0));
                    const R gy = fmax(fmax(bl[1] - s.y, s.y - bh[1]), R(0));
                    const R gz = fmax(fmax(bl[2] - s.z, s.z - bh[2]), R(0));
                    const R d2 = gx * gx + gy * gy + gz * gz;
                    soft = !(d2 > pos_max(s.h * s.h, hg2) * R(1.0001));
                }
            }
            if (SOFT) {
                const uint64_t msoft = __ballot(e < nb && soft);
                const uint64_t mnewt = __ballot(e < nb && !soft);
                const uint64_t lt = lane_mask_lt();
                if (e < nb) {
                    if (soft) st->pp[ns + (uint32_t)popc64(msoft & lt)] = s;
                    else st->pp[nb - 1u - (nn + (uint32_t)popc64(mnewt & lt))] = s;
                }
                ns += (uint32_t)popc64(msoft);
                nn += (uint32_t)popc64(mnewt);
            } else if (e < nb) {
                st->pp[e] = s;
            }
        }
        __syncthreads();
        R bx = 0, by = 0, bz = 0, bp = 0;
        if (on) {
            sp.each(nb - ns, [&](uint32_t j) {   // both radii below r: Newtonian, no extra terms
                const AdPart<R> q = st->pp[ns + j];
                const R dx = q.x - tx, dy = q.y - ty, dz = q.z - tz;
                const R ri = rsq(dx * dx + dy * dy + dz * dz);
                const R mri = q.m * ri, mri3 = mri * ri * ri;
                bp -= mri;
                bx += mri3 * dx;
                by += mri3 * dy;
                bz += mri3 * dz;
            });
            if (SOFT)
                sp.each(ns, [&](uint32_t j) {
                    const AdPart<R> q = st->pp[j];
                    if (q.idx == tidx) return;
                    const R dx = q.x - tx, dy = q.y - ty, dz = q.z - tz;
                    const R r2 = dx * dx + dy * dy + dz * dz;
                    const R ri = rsq(r2);
                    const R r = r_of(r2, ri);
                    R F = ri * ri * ri, P = ri;   // Newtonian beyond both radii
                    R c = R(0);                     // extra term over r
                    const R hm = pos_max(th, q.h);
                    if (r2 < hm * hm) {   // inside at least one radius: one branch for the wave
                        if (q.gas) {
                            R Fi, Pi, Wri, Fj, Pj, Wrj;
                            sym_soft<R>(r2, ri, r, th, thinv, Fi, Pi, Wri);
                            sym_soft<R>(r2, ri, r, q.h, rcp(q.h), Fj, Pj, Wrj);
                            F = R(0.5) * (Fi + Fj);
                            P = R(0.5) * (Pi + Pj);
                            if (r > R(0)) c = R(0.5) * (tz_ * Wri + q.m * tminv * q.zz * Wrj) * ri;
                        } else {
                            R Wr;
                            sym_soft<R>(r2, ri, r, hm, rcp(hm), F, P, Wr);
                        }
                    }
                    const R k = q.m * F - c;
                    bx += k * dx;
                    by += k * dy;
                    bz += k * dz;
                    bp -= q.m * P;
                });
        }
        ax.fold(bx);
        ay.fold(by);
        az.fold(bz);
        ap.fold(bp);
        __syncthreads();
    }
};

template <typename T, class Ev>
__device__ __forceinline__ bool group_target(const AdArgs<T> &a, Ev &ev, int g, int64_t &i,
                                             double blo[3], double bhi[3]) {
    using R = typename Ev::R;
    const int lane = threadIdx.x;
    const int64_t gf = a.gfirst[g], gc = a.gcount[g];
    for (int d = 0; d < 3; ++d) {
        blo[d] = a.gbox[6 * g + d];
        bhi[d] = a.gbox[6 * g + 3 + d];
        ev.cen[d] = a.gcen[3 * g + d];
    }
    ev.sp.init((uint32_t)gc, (uint32_t)lane);
    i = gf + ev.sp.tl;
    ev.on = a.order[i] < a.n_gas;
    if (__ballot(ev.on) == 0ull) return false;
    ev.tx = (R)((double)a.xs[i] - (FormT<Ev::kForm>::rel ? ev.cen[0] : 0.0));
    ev.ty = (R)((double)a.ys[i] - (FormT<Ev::kForm>::rel ? ev.cen[1] : 0.0));
    ev.tz = (R)((double)a.zs[i] - (FormT<Ev::kForm>::rel ? ev.cen[2] : 0.0));
    ev.th = (R)a.hs[i];
    ev.tidx = (int32_t)i;
    return true;
}

template <typename T, int FORM>
struct SumsEvalF : SumsEval<T, FORM> {
    static constexpr int kForm = FORM;
};
template <typename T, int FORM, int ORDER>
struct ForceEvalF : ForceEval<T, FORM, ORDER> {
    static constexpr int kForm = FORM;
};

template <typename T, int FORM>
__global__ __launch_bounds__(64) void k_adaptive_sums(AdArgs<T> a) {
    using R = typename FormT<FORM>::R;
    __shared__ WalkLds L;
    __shared__ AdStage<R> stage;
    const int ng = __builtin_amdgcn_readfirstlane(*a.n_groups_dev);
    SumsEvalF<T, FORM> ev;
    ev.a = &a;
    ev.st = &stage;
    XcdTasks tasks;
    tasks.init(a.task_ctr, ng);
    for (int g = tasks.next(); g < ng; g = tasks.next()) {
        int64_t i;
        double blo[3], bhi[3];
        if (!group_target(a, ev, g, i, blo, bhi)) continue;
        ev.thinv = rcp(ev.th);
        ev.sW = ev.sWh = ev.sPh = R(0);
        uint32_t npc, npp;
        uint64_t cks;
        walk_task<false, SumsEvalF<T, FORM>, true>(
            a.nd, L, a.gstack + (int64_t)blockIdx.x * kStack, ev, blo, bhi, a.ghmax[g],
            a.gfirst[g], a.gfirst[g] + a.gcount[g], task_ag_group(a.nd, g), a.err, npc, npp, cks);
        double v[3] = {(double)ev.sW, (double)ev.sWh, (double)ev.sPh};
        ev.sp.template reduce<3>(v, reinterpret_cast<double *>(&stage), (uint32_t)threadIdx.x);
        if (ev.on && threadIdx.x < ev.sp.gc) {
            const double h = (double)a.hs[i];
            const double n = v[0];
            const double dhdn = -h / (3.0 * n);
            const double omega = 1.0 - dhdn * v[1];
            const double zeta = dhdn * v[2];
            a.z[i] = zeta / omega;
            if (a.aux) {
                const int64_t o = a.order[i];
                a.aux[2 * o] = (T)omega;
                a.aux[2 * o + 1] = (T)zeta;
            }
        }
    }
}

template <typename T, int FORM, int ORDER>
__global__ __launch_bounds__(64) void k_adaptive_force(AdArgs<T> a) {
    using R = typename FormT<FORM>::R;
    __shared__ WalkLds L;
    __shared__ AdStage<R> stage;
    const int ng = __builtin_amdgcn_readfirstlane(*a.n_groups_dev);
    ForceEvalF<T, FORM, ORDER> ev;
    ev.a = &a;
    ev.st = &stage;
    XcdTasks tasks;
    tasks.init(a.task_ctr, ng);
    for (int g = tasks.next(); g < ng; g = tasks.next()) {
        int64_t i;
        double blo[3], bhi[3];
        if (!group_target(a, ev, g, i, blo, bhi)) continue;
        ev.thinv = rcp(ev.th);
        ev.tminv = rcp((R)a.ms[i]);
        ev.tz_ = (R)a.z[i];
        for (int d = 0; d < 3; ++d) {
            ev.bl[d] = dto_frame<FORM>(blo[d], ev.cen[d]);
            ev.bh[d] = dto_frame<FORM>(bhi[d], ev.cen[d]);
        }
        {
            const R hgr = (R)a.ghmax[g];
            ev.hg2 = hgr * hgr;
        }
        ev.ax.zero();
        ev.ay.zero();
        ev.az.zero();
        ev.ap.zero();
        uint32_t npc, npp;
        uint64_t cks;
        // full batches hold a multiple of the copy count (no partial last step)
        walk_task<false>(a.nd, L, a.gstack + (int64_t)blockIdx.x * kStack, ev, blo, bhi,
                         a.ghmax[g], a.gfirst[g], a.gfirst[g] + a.gcount[g],
                         task_ag_group(a.nd, g), a.err, npc, npp, cks,
                         kPPBatch<R> / ev.sp.k * ev.sp.k, 64u / ev.sp.k * ev.sp.k);
        double v[4] = {ev.ax.value(), ev.ay.value(), ev.az.value(), ev.ap.value()};
        ev.sp.template reduce<4>(v, reinterpret_cast<double *>(&stage), (uint32_t)threadIdx.x);
        if (ev.on && threadIdx.x < ev.sp.gc) {
            const int64_t o = a.order[i];
            a.acc[3 * o] = (T)(a.G * v[0]);
            a.acc[3 * o + 1] = (T)(a.G * v[1]);
            a.acc[3 * o + 2] = (T)(a.G * v[2]);
            if (a.pot) a.pot[o] = (T)(a.G * v[3]);
        }
    }
}

template <typename T, int FORM, int ORDER>
void launch_ad(const AdArgs<T> &a1, const AdArgs<T> &a2, hipStream_t s) {
    const unsigned grid = (unsigned)walk_grid();
    hipLaunchKernelGGL((k_adaptive_sums<T, FORM>), dim3(grid), dim3(64), 0, s, a1);
    hipLaunchKernelGGL((k_adaptive_force<T, FORM, ORDER>), dim3(grid), dim3(64), 0, s, a2);
}

template <typename T>
sf_status adaptive_run(sf_grav_tree_s *t, const EvalOpts &o, void *acc, void *pot, void *aux,
                       DevArena &ar) {
    hipStream_t s = t->stream;
    // sinks take their fields from the sink walk; gas cells from the walks below
    sf_status st = tree_accel(t, o, acc, pot, ar, false);
    if (st != SF_OK) return st;
    int32_t *ctr;
    uint32_t *gstack;
    double *z;
    SF_ALLOC_TMP(ar, ctr, 2 * kCtrWords);
    SF_ALLOC_TMP(ar, gstack, (int64_t)walk_grid() * kStack);
    SF_ALLOC_TMP(ar, z, t->n);
    FillRanges zero;
    zero.add(ctr, 2 * kCtrWords);
    zero.add(z, 2 * t->n);
    fill_ranges_u32(zero, 0u, s);
    AdArgs<T> a{};
    a.nd.n_nodes = t->n_nodes;
    a.nd.w = t->nw[0];
    a.nd.q = t->nq[0];
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
    a.gstack = gstack;
    a.z = z;
    a.acc = (T *)acc;
    a.pot = (T *)pot;
    a.aux = (T *)aux;
    a.G = o.G;
    AdArgs<T> a1 = a, a2 = a;
    a1.task_ctr = ctr;
    a1.err = ctr + kCtrErr;
    a2.task_ctr = ctr + kCtrWords;
    a2.err = ctr + kCtrErr;
    if (o.order == 0) {
        if (o.form == SF_FP32C) launch_ad<T, SF_FP32C, 0>(a1, a2, s);
        else if (o.form == SF_FP32) launch_ad<T, SF_FP32, 0>(a1, a2, s);
        else launch_ad<T, SF_FP64, 0>(a1, a2, s);
    } else {
        if (o.form == SF_FP32C) launch_ad<T, SF_FP32C, 2>(a1, a2, s);
        else if (o.form == SF_FP32) launch_ad<T, SF_FP32, 2>(a1, a2, s);
        else launch_ad<T, SF_FP64, 2>(a1, a2, s);
    }
    SF_HIP(hipGetLastError());
    int32_t herr = 0;
    SF_HIP(hipMemcpyAsync(&herr, ctr + kCtrErr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SF_HIP(hipStreamSynchronize(s));
    if (herr)
        return sf_fail(SF_E_INTERNAL, "tree walk stopped by a capacity guard (code %d)", herr);
    return SF_OK;
}

}  // namespace

sf_status adaptive_accel(sf_grav_tree_s *t, const EvalOpts &o, void *acc, void *pot, void *aux,
                         DevArena &ar) {
    if (t->dt == SF_F32) return adaptive_run<float>(t, o, acc, pot, aux, ar);
    return adaptive_run<double>(t, o, acc, pot, aux, ar);
}

}  // namespace sf
