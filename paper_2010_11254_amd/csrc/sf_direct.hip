// sf_direct.hip -- direct summation path on gfx950 (all pairs; the theta -> 0
// limit of the tree, paper Sec. 2.2) and its adjoint.
//
// Particles are sorted by a type-major Morton key (gas first, then sinks, each
// in Morton order) and cut into 64-particle tiles, so a tile is spatially
// compact.  One wavefront owns one target tile (one target per lane) and
// walks every source tile; the source index is uniform across the wave, so
// source records stream through scalar loads into SGPRs and need no LDS.
// Per (target tile, source tile) one FP64 test decides whether any pair can
// be softened (box gap below the larger max softening); if not, a loop with
// no softening test or self check runs.  In FP32C, sources are stored as
// offsets from their tile centre and each target is shifted once per source
// tile by the FP64 centre difference, so the FP32 pair vector keeps the
// relative accuracy of a local difference; per-tile FP32 partials are folded
// into per-target two-sum accumulators.  Sink targets skip sink tiles and add
// the FP64 sink-sink sum.
#include "sf_build.h"
#include "sf_math.h"
#include "sf_prims.h"

namespace sf {

template <typename R> struct alignas(32) SrcRec { R x, y, z, m, h2, h; int32_t idx, pad; };

template <int FORM> using DForm = FormT<FORM>;

// ---------------------------------------------------------------- tiles

// One wave per tile: first/count, box, max softening, centre, source records.
template <typename T, int FORM>
__global__ __launch_bounds__(64) void k_tiles(int64_t n, int64_t n_gas, int64_t n_gas_tiles,
                                              int64_t n_tiles, const T *__restrict__ xs,
                                              const T *__restrict__ ys, const T *__restrict__ zs,
                                              const T *__restrict__ ms, const T *__restrict__ hs,
                                              int32_t *__restrict__ tfirst,
                                              int32_t *__restrict__ tcount,
                                              double *__restrict__ tbox, double *__restrict__ tcen,
                                              SrcRec<typename DForm<FORM>::R> *__restrict__ rec) {
    using R = typename DForm<FORM>::R;
    const int lane = threadIdx.x;
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        int64_t f, e;
        if (t < n_gas_tiles) {
            f = t * 64;
            e = f + 64 < n_gas ? f + 64 : n_gas;
        } else {
            f = n_gas + (t - n_gas_tiles) * 64;
            e = f + 64 < n ? f + 64 : n;
        }
        const int64_t c = e - f;
        const int64_t p = f + (lane < c ? lane : 0);
        const double v[3] = {(double)xs[p], (double)ys[p], (double)zs[p]};
        double lo[3], hi[3];
        double hm = lane < c ? (double)hs[p] : 0.0;
        for (int d = 0; d < 3; ++d) { lo[d] = v[d]; hi[d] = v[d]; }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            for (int d = 0; d < 3; ++d) {
                lo[d] = fmin(lo[d], __shfl_xor(lo[d], off, 64));
                hi[d] = fmax(hi[d], __shfl_xor(hi[d], off, 64));
            }
            hm = fmax(hm, __shfl_xor(hm, off, 64));
        }
        double cen[3];
        for (int d = 0; d < 3; ++d) cen[d] = DForm<FORM>::rel ? (double)(T)(0.5 * (lo[d] + hi[d])) : 0.0;
        if (lane == 0) {
            tfirst[t] = (int32_t)f;
            tcount[t] = (int32_t)c;
            for (int d = 0; d < 3; ++d) {
                tbox[8 * t + d] = lo[d];
                tbox[8 * t + 3 + d] = hi[d];
                tcen[3 * t + d] = cen[d];
            }
            tbox[8 * t + 6] = hm;
            tbox[8 * t + 7] = 0.0;
        }
        if (lane < c) {
            SrcRec<R> r;
            r.x = (R)(v[0] - cen[0]);
            r.y = (R)(v[1] - cen[1]);
            r.z = (R)(v[2] - cen[2]);
            if (!DForm<FORM>::rel) { r.x = (R)xs[p]; r.y = (R)ys[p]; r.z = (R)zs[p]; }
            r.m = (R)ms[p];
            r.h = (R)hs[p];
            r.h2 = r.h * r.h;
            r.idx = (int32_t)p;
            r.pad = 0;
            rec[p] = r;
        }
    }
}

// ---------------------------------------------------------------- forward

template <typename T, int FORM>
__global__ __launch_bounds__(256) void k_direct(int64_t n, int64_t n_gas, int64_t n_gas_tiles,
                                                int64_t n_tiles,
                                                const int32_t *__restrict__ tfirst,
                                                const int32_t *__restrict__ tcount,
                                                const double *__restrict__ tbox,
                                                const double *__restrict__ tcen,
                                                const SrcRec<typename DForm<FORM>::R> *__restrict__ rec,
                                                const int32_t *__restrict__ order,
                                                const double *__restrict__ ss, double G,
                                                T *__restrict__ acc, T *__restrict__ pot) {
    using R = typename DForm<FORM>::R;
    const int lane = threadIdx.x & 63;
    const int64_t tt = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tt >= n_tiles) return;
    const int64_t f = tfirst[tt], c = tcount[tt];
    const bool has = lane < c;
    const int64_t i = f + (has ? lane : 0);
    const SrcRec<R> me = rec[i];
    const double wlo[3] = {tbox[8 * tt], tbox[8 * tt + 1], tbox[8 * tt + 2]};
    const double whi[3] = {tbox[8 * tt + 3], tbox[8 * tt + 4], tbox[8 * tt + 5]};
    const double whm = tbox[8 * tt + 6];
    const double wc[3] = {tcen[3 * tt], tcen[3 * tt + 1], tcen[3 * tt + 2]};
    const bool sink_tile = tt >= n_gas_tiles;
    const int64_t ns = sink_tile ? n_gas_tiles : n_tiles;
    Acc<FORM> ax, ay, az, ap;
    ax.zero(); ay.zero(); az.zero(); ap.zero();
    const int32_t my_idx = (int32_t)i;
    for (int64_t s = 0; s < ns; ++s) {
        const int64_t sf0 = tfirst[s], sc = tcount[s];
        // any softened pair possible between the two tiles?
        double g2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double gd = fmax(fmax(tbox[8 * s + d] - whi[d], wlo[d] - tbox[8 * s + 3 + d]), 0.0);
            g2 += gd * gd;
        }
        const double hm = fmax(whm, tbox[8 * s + 6]);
        const bool near = g2 < hm * hm;
        // target in the source tile's frame: o_i - (c_s - c_w)
        R tx = me.x, ty = me.y, tz = me.z;
        if (DForm<FORM>::rel) {
            tx = me.x - (R)(tcen[3 * s] - wc[0]);
            ty = me.y - (R)(tcen[3 * s + 1] - wc[1]);
            tz = me.z - (R)(tcen[3 * s + 2] - wc[2]);
        }
        R bx = 0, by = 0, bz = 0, bp = 0;
        const SrcRec<R> *src = rec + sf0;
        if (!near) {
            // unrolled so that the scalar loads of several source records are
            // in flight together (a tile holds at most 64 sources)
            const uint32_t nsrc = (uint32_t)sc;
            constexpr int U = sizeof(R) == 4 ? 4 : 2;   // FP64: registers for 2 in flight
#pragma unroll U
            for (uint32_t j = 0; j < nsrc; ++j) {
                const SrcRec<R> q = src[j];
                const R dx = q.x - tx, dy = q.y - ty, dz = q.z - tz;
                const R r2 = dx * dx + dy * dy + dz * dz;
                const R ri = rsq(r2);
                const R mri = q.m * ri;
                const R mri3 = mri * ri * ri;
                bp -= mri;
                bx += mri3 * dx;
                by += mri3 * dy;
                bz += mri3 * dz;
            }
        } else {
            for (int64_t j = 0; j < sc; ++j) {
                const SrcRec<R> q = src[j];
                const R dx = q.x - tx, dy = q.y - ty, dz = q.z - tz;
                const R r2 = dx * dx + dy * dy + dz * dz;
                const R ri = rsq(r2);
                R P = ri, F = ri * ri * ri;
                const R hh2 = q.h2 > me.h2 ? q.h2 : me.h2;
                if (r2 < hh2) {
                    R FrR, dFh, dPh;
                    const R hh = pos_max(q.h, me.h);
                    dsoft_ri<R>(r2, ri, hh, rcp(hh), F, P, FrR, dFh, dPh);
                    if (q.idx == my_idx) { F = R(0); P = R(0); }
                }
                const R mF = q.m * F;
                bp -= q.m * P;
                bx += mF * dx;
                by += mF * dy;
                bz += mF * dz;
            }
        }
        ax.fold(bx); ay.fold(by); az.fold(bz); ap.fold(bp);
    }
    if (!has) return;
    double v[4] = {ax.value(), ay.value(), az.value(), ap.value()};
    if (sink_tile && ss) {
        // sinks occupy the tail of the sorted order; their FP64 sink-sink sum
        // is indexed by position among sinks
        const int64_t ks = i - n_gas;
        for (int d = 0; d < 4; ++d) v[d] += ss[4 * ks + d];
    }
    const int64_t o = order[i];
    acc[3 * o] = (T)(G * v[0]);
    acc[3 * o + 1] = (T)(G * v[1]);
    acc[3 * o + 2] = (T)(G * v[2]);
    if (pot) pot[o] = (T)(G * v[3]);
}

template <typename T, int FORM>
static sf_status direct_run(sf_grav_tree_s *t, const EvalOpts &o, void *acc, void *pot,
                            DevArena &ar) {
    using R = typename DForm<FORM>::R;
    hipStream_t s = t->stream;
    const int64_t n = t->n, ng = t->n_gas;
    t->n_gas_tiles = (ng + 63) / 64;
    t->n_tiles = t->n_gas_tiles + (n - ng + 63) / 64;
    SrcRec<R> *rec;
    SF_ALLOC_TMP(ar, t->tfirst, t->n_tiles);
    SF_ALLOC_TMP(ar, t->tcount, t->n_tiles);
    SF_ALLOC_TMP(ar, t->tbox, 8 * t->n_tiles);
    SF_ALLOC_TMP(ar, t->tcen, 3 * t->n_tiles);
    SF_ALLOC_TMP(ar, rec, n);
    const unsigned tb = (unsigned)std::min<int64_t>(t->n_tiles, 8192);
    hipLaunchKernelGGL((k_tiles<T, FORM>), dim3(tb), dim3(64), 0, s, n, ng, t->n_gas_tiles,
                       t->n_tiles, (const T *)t->xs, (const T *)t->ys, (const T *)t->zs,
                       (const T *)t->ms, (const T *)t->hs, t->tfirst, t->tcount, t->tbox, t->tcen,
                       rec);
    double *ss = nullptr, *srec = nullptr;
    if (t->n_sink > 0) {
        SF_ALLOC_TMP(ar, ss, 4 * t->n_sink);
        SF_ALLOC_TMP(ar, srec, kSinkRec * t->n_sink);
        sink_sink_accel(t, o.G, ss, srec, t->stream);
    }
    const unsigned blocks = (unsigned)((t->n_tiles + 3) / 4);
    hipLaunchKernelGGL((k_direct<T, FORM>), dim3(blocks), dim3(256), 0, s, n, ng, t->n_gas_tiles,
                       t->n_tiles, t->tfirst, t->tcount, t->tbox, t->tcen, rec, t->order, ss, o.G,
                       (T *)acc, (T *)pot);
    SF_HIP(hipGetLastError());
    return SF_OK;
}

size_t direct_rec_bytes(int form) {
    return form == SF_FP64 ? sizeof(SrcRec<double>) : sizeof(SrcRec<float>);
}

sf_status direct_accel(sf_grav_tree_s *t, const EvalOpts &o, void *acc, void *pot, DevArena &ar) {
    if (t->dt == SF_F32) {
        if (o.form == SF_FP32C) return direct_run<float, SF_FP32C>(t, o, acc, pot, ar);
        if (o.form == SF_FP32) return direct_run<float, SF_FP32>(t, o, acc, pot, ar);
        return direct_run<float, SF_FP64>(t, o, acc, pot, ar);
    }
    if (o.form == SF_FP32C) return direct_run<double, SF_FP32C>(t, o, acc, pot, ar);
    if (o.form == SF_FP32) return direct_run<double, SF_FP32>(t, o, acc, pot, ar);
    return direct_run<double, SF_FP64>(t, o, acc, pot, ar);
}

}  // namespace sf
