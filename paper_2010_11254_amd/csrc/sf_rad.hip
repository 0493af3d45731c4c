// sf_rad.hip -- radiation sums that ride on the gravity walk (Sec. 3.1: FUV
// optical depths of tree nodes summed into angular bins; Sec. 3.3: the IR
// energy density from stars, sum_s L_s / (4 pi c r^2)), for gas cells.
//
// Columns: six bins, the faces of a cube around the target (a direction d =
// x_source - x_target belongs to the face of its largest |d_k|, ties to the
// lower axis, with that component's sign; each face spans 4 pi / 6 sr); a
// bin holds the gas column density averaged over its solid angle,
// sum m / (Omega_bin r^2), with a particle's r^2 softened to
// r^2 + (h / 2.8)^2 and an accepted node entering as its gas mass at its gas
// centre of mass.  e_IR: sinks' luminosities, an accepted node as its total
// sink luminosity at the luminosity-weighted centre, particles with the same
// softened r^2.  The walk and its decisions are those of sf_grav_accel (node
// moments over all particles).  Each target of a group holds
// floor(64 / gc) lanes that share its batch entries (lane splitting).
#include "sf_build.h"
#include "sf_math.h"
#include "sf_prims.h"
#include "sf_split.h"
#include "sf_walk.h"

namespace sf {

namespace {

constexpr int kR = 7;   // six bins, e_IR

template <typename T>
struct RadArgs {
    WalkNodes nd;
    const NodeW *gas;             // node records over gas only (mass, centre of mass)
    const double *lum_node;       // per node: L, L x, L y, L z (4 x nodes, component-major)
    const T *xs, *ys, *zs, *ms, *hs, *ls;   // sorted particles; ls: luminosity (sinks)
    const int32_t *order;
    int64_t n, n_gas;
    const int32_t *n_groups_dev, *gfirst, *gcount;
    const double *gbox, *ghmax, *gcen;
    int32_t *task_ctr, *err;
    uint32_t *gstack;
    T *col, *eir;                 // caller order (n x 6, n); either may be null
    double inv_omega, inv_4pic;
};

template <typename R>
struct alignas(16) RadEntry {
    R x, y, z, mw;   // gas position or centre, weight m (gas) for the columns
    R lx, ly, lz, lw;   // luminosity centre and luminosity (sinks)
    R e2;            // softening (h/2.8)^2 of a particle, 0 for nodes
};

template <typename R>
__device__ __forceinline__ void add_col(R dx, R dy, R dz, R w, R (&b)[kR]) {
    // dominant axis (ties to the lower axis), then the sign of d along it
    // (-0 counts as positive); each bin's condition is formed from the
    // comparisons as a lane mask, so a bin costs one select and one add
    const R ax = fabs(dx), ay = fabs(dy), az = fabs(dz);
    const bool xm = ax >= ay && ax >= az;
    const bool ym = !xm && ay >= az;
    const bool zm = !xm && !ym;
    const bool nx = dx < R(0), ny = dy < R(0), nz = dz < R(0);
    b[0] += (xm && !nx) ? w : R(0);
    b[1] += (xm && nx) ? w : R(0);
    b[2] += (ym && !ny) ? w : R(0);
    b[3] += (ym && ny) ? w : R(0);
    b[4] += (zm && !nz) ? w : R(0);
    b[5] += (zm && nz) ? w : R(0);
}

template <typename T, int FORM>
struct RadEval {
    using R = typename FormT<FORM>::R;
    const RadArgs<T> *a;
    RadEntry<R> *st;
    double cen[3];
    R tx, ty, tz;
    int32_t tidx;
    bool on;
    Split sp;
    Acc<FORM> acc[kR];

    __device__ void fold(const R (&b)[kR]) {
#pragma unroll
        for (int c = 0; c < kR; ++c) acc[c].fold(b[c]);
    }

    // node entries: no self term, no softening
    __device__ void run(uint32_t nb) {
        R b[kR] = {};
        if (on)
            sp.each(nb, [&](uint32_t j) {
                const RadEntry<R> s = st[j];
                if (s.mw > R(0)) {
                    const R dx = s.x - tx, dy = s.y - ty, dz = s.z - tz;
                    const R r2 = dx * dx + dy * dy + dz * dz + s.e2;
                    add_col<R>(dx, dy, dz, s.mw * rcp(r2), b);
                }
                if (s.lw > R(0)) {
                    const R dx = s.lx - tx, dy = s.ly - ty, dz = s.lz - tz;
                    b[6] += s.lw * rcp(dx * dx + dy * dy + dz * dz + s.e2);
                }
            });
        fold(b);
        __syncthreads();
    }

    __device__ void pc_batch(WalkLds &L, uint32_t head, uint32_t nb) {
        const uint32_t e = threadIdx.x;
        if (e < nb) {
            const int node = L.pc[(head + e) & 127];
            const NodeW &g = a->gas[node];
            RadEntry<R> s;
            s.x = dto_frame<FORM>(g.com[0], cen[0]);
            s.y = dto_frame<FORM>(g.com[1], cen[1]);
            s.z = dto_frame<FORM>(g.com[2], cen[2]);
            s.mw = (R)g.M;
            const int64_t nn = a->nd.n_nodes;
            const double lw = a->lum_node[node];
            s.lw = (R)lw;
            s.lx = s.ly = s.lz = R(0);
            if (lw > 0.0) {
                s.lx = dto_frame<FORM>(a->lum_node[nn + node] / lw, cen[0]);
                s.ly = dto_frame<FORM>(a->lum_node[2 * nn + node] / lw, cen[1]);
                s.lz = dto_frame<FORM>(a->lum_node[3 * nn + node] / lw, cen[2]);
            }
            s.e2 = R(0);
            st[e] = s;
        }
        __syncthreads();
        run(nb);
    }

    template <bool SOFT>
    __device__ void pp_batch(WalkLds &L, uint32_t nb) {
        const uint32_t e = threadIdx.x;
        if (e < nb) {
            const int p = L.slot[e];
            const bool gas = a->order[p] < a->n_gas;
            RadEntry<R> s;
            s.x = to_frame<FORM>(a->xs[p], cen[0]);
            s.y = to_frame<FORM>(a->ys[p], cen[1]);
            s.z = to_frame<FORM>(a->zs[p], cen[2]);
            s.lx = s.x;
            s.ly = s.y;
            s.lz = s.z;
            s.mw = gas ? (R)a->ms[p] : R(0);
            s.lw = gas ? R(0) : (R)a->ls[p];
            const R eps = (R)a->hs[p] * R(1.0 / 2.8);
            s.e2 = eps * eps;
            st[e] = s;
        }
        __syncthreads();
        // each lane skips its own target's entry (only near leaves hold it)
        R b[kR] = {};
        if (on)
            sp.each(nb, [&](uint32_t j) {
                const RadEntry<R> s = st[j];
                const R dx = s.x - tx, dy = s.y - ty, dz = s.z - tz;
                const R r2 = dx * dx + dy * dy + dz * dz + s.e2;
                const bool self = SOFT && L.slot[j] == tidx;
                if (s.mw > R(0) && !self) add_col<R>(dx, dy, dz, s.mw * rcp(r2), b);
                if (s.lw > R(0) && !self) b[6] += s.lw * rcp(r2);
            });
        fold(b);
        __syncthreads();
    }
};

template <typename T, int FORM>
__global__ __launch_bounds__(64) void k_walk_rad(RadArgs<T> a) {
    using R = typename FormT<FORM>::R;
    __shared__ WalkLds L;
    __shared__ RadEntry<R> stage[64];
    const int lane = threadIdx.x;
    const int ng = __builtin_amdgcn_readfirstlane(*a.n_groups_dev);
    RadEval<T, FORM> ev;
    ev.a = &a;
    ev.st = stage;
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
        if (__ballot(ev.on) == 0ull) continue;
        ev.tx = to_frame<FORM>(a.xs[i], ev.cen[0]);
        ev.ty = to_frame<FORM>(a.ys[i], ev.cen[1]);
        ev.tz = to_frame<FORM>(a.zs[i], ev.cen[2]);
        ev.tidx = (int32_t)i;
        for (int c = 0; c < kR; ++c) ev.acc[c].zero();
        uint32_t npc, npp;
        uint64_t cks;
        // full batches hold a multiple of the copy count (no partial last step)
        const uint32_t kb = 64u / ev.sp.k * ev.sp.k;
        walk_task<false>(a.nd, L, a.gstack + (int64_t)blockIdx.x * kStack, ev, blo, bhi,
                         a.ghmax[g], gf, gf + gc, task_ag_group(a.nd, g), a.err, npc, npp, cks,
                         kb, kb);
        double v[kR];
        for (int c = 0; c < kR; ++c) v[c] = ev.acc[c].value();
        // the stage is free once the task's batches are done
        ev.sp.template reduce<sizeof(stage) / (64 * sizeof(double))>(
            v, reinterpret_cast<double *>(stage), (uint32_t)lane);
        if (ev.on && (uint32_t)lane < ev.sp.gc) {
            const int64_t o = a.order[i];
            if (a.col)
                for (int c = 0; c < 6; ++c) a.col[6 * o + c] = (T)(a.inv_omega * v[c]);
            if (a.eir) a.eir[o] = (T)(a.inv_4pic * v[6]);
        }
    }
}

// Luminosity sums per node (L, L x, L y, L z over the node's sinks), bottom
// up as the velocity sums of the tidal walk.
template <typename T>
__global__ void k_lum_leaf(int64_t nn, const int32_t *__restrict__ nfirst,
                           const int32_t *__restrict__ ncount, const int32_t *__restrict__ nnchild,
                           const T *__restrict__ ls, const T *__restrict__ xs,
                           const T *__restrict__ ys, const T *__restrict__ zs,
                           const int32_t *__restrict__ order, int64_t n_gas,
                           double *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn || nnchild[k] != 0) return;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t p = nfirst[k]; p < nfirst[k] + ncount[k]; ++p) {
        if (order[p] < n_gas) continue;
        const double l = (double)ls[p];
        s[0] += l;
        s[1] += l * (double)xs[p];
        s[2] += l * (double)ys[p];
        s[3] += l * (double)zs[p];
    }
    for (int c = 0; c < 4; ++c) out[c * nn + k] = s[c];
}

__global__ void k_lum_level(int64_t k0, int64_t k1, int64_t nn, const int32_t *__restrict__ nchild,
                            const int32_t *__restrict__ nnchild, double *__restrict__ out) {
    const int64_t k = k0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= k1 || nnchild[k] == 0) return;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t ch = nchild[k]; ch < nchild[k] + nnchild[k]; ++ch)
        for (int c = 0; c < 4; ++c) s[c] += out[c * nn + ch];
    for (int c = 0; c < 4; ++c) out[c * nn + k] = s[c];
}

template <typename T>
__global__ void k_gather_lum(const T *__restrict__ lum, const int32_t *__restrict__ order,
                             int64_t n, T *__restrict__ ls) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) ls[s] = lum[order[s]];
}

unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

template <typename T>
sf_status rad_run(sf_grav_tree_s *t, const EvalOpts &o, const void *lum, double c_light, void *col,
                  void *eir, DevArena &ar) {
    hipStream_t s = t->stream;
    const int64_t n = t->n, nn = t->n_nodes;
    int32_t *ctr;
    uint32_t *gstack;
    T *ls;
    double *lnode;
    SF_ALLOC_TMP(ar, ctr, kCtrWords);
    SF_ALLOC_TMP(ar, gstack, (int64_t)walk_grid() * kStack);
    SF_ALLOC_TMP(ar, ls, n);
    SF_ALLOC_TMP(ar, lnode, 4 * nn);
    FillRanges zero;
    zero.add(ctr, kCtrWords);
    zero.add(ls, n * (int64_t)sizeof(T) / 4);
    fill_ranges_u32(zero, 0u, s);
    if (lum)
        hipLaunchKernelGGL(k_gather_lum<T>, dim3(nblk(n)), dim3(256), 0, s, (const T *)lum,
                           t->order, n, ls);
    hipLaunchKernelGGL(k_lum_leaf<T>, dim3(nblk(nn)), dim3(256), 0, s, nn, t->nfirst, t->ncount,
                       t->nnchild, (const T *)ls, (const T *)t->xs, (const T *)t->ys,
                       (const T *)t->zs, t->order, t->n_gas, lnode);
    for (int l = kLevels - 1; l >= 0; --l) {
        const int64_t k0 = t->level_off[l], k1 = t->level_off[l + 1];
        if (k1 <= k0 || t->level_off[l + 2] <= k1) continue;
        hipLaunchKernelGGL(k_lum_level, dim3(nblk(k1 - k0)), dim3(256), 0, s, k0, k1, nn,
                           t->nchild, t->nnchild, lnode);
    }
    RadArgs<T> a{};
    a.nd.n_nodes = nn;
    a.nd.w = t->nw[0];
    a.nd.q = t->nq[0];
    a.nd.side = t->hframe.side;
    a.nd.th2 = o.theta * o.theta;
    set_relative(a.nd, t, o);
    a.gas = t->nw[1];
    a.lum_node = lnode;
    a.xs = (const T *)t->xs;
    a.ys = (const T *)t->ys;
    a.zs = (const T *)t->zs;
    a.ms = (const T *)t->ms;
    a.hs = (const T *)t->hs;
    a.ls = ls;
    a.order = t->order;
    a.n = n;
    a.n_gas = t->n_gas;
    a.n_groups_dev = t->n_groups_dev;
    a.gfirst = t->gfirst;
    a.gcount = t->gcount;
    a.gbox = t->gbox;
    a.ghmax = t->ghmax;
    a.gcen = t->gcen;
    a.task_ctr = ctr;
    a.err = ctr + kCtrErr;
    a.gstack = gstack;
    a.col = (T *)col;
    a.eir = (T *)eir;
    a.inv_omega = 6.0 / (4.0 * 3.14159265358979323846);
    a.inv_4pic = 1.0 / (4.0 * 3.14159265358979323846 * c_light);
    const unsigned grid = (unsigned)walk_grid();
    if (o.form == SF_FP32C)
        hipLaunchKernelGGL((k_walk_rad<T, SF_FP32C>), dim3(grid), dim3(64), 0, s, a);
    else if (o.form == SF_FP32)
        hipLaunchKernelGGL((k_walk_rad<T, SF_FP32>), dim3(grid), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL((k_walk_rad<T, SF_FP64>), dim3(grid), dim3(64), 0, s, a);
    SF_HIP(hipGetLastError());
    int32_t herr = 0;
    SF_HIP(hipMemcpyAsync(&herr, ctr + kCtrErr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SF_HIP(hipStreamSynchronize(s));
    if (herr)
        return sf_fail(SF_E_INTERNAL, "tree walk stopped by a capacity guard (code %d)", herr);
    return SF_OK;
}

}  // namespace

sf_status rad_sums(sf_grav_tree_s *t, const EvalOpts &o, const void *lum, double c_light,
                   void *col, void *eir, DevArena &ar) {
    if (t->dt == SF_F32) return rad_run<float>(t, o, lum, c_light, col, eir, ar);
    return rad_run<double>(t, o, lum, c_light, col, eir, ar);
}

}  // namespace sf
