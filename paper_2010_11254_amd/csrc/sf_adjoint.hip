// sf_adjoint.hip -- adjoint (vector-Jacobian product) of the softened gravity.
//
// For L = sum_i (ga_i . a_i + gp_i phi_i) with a_i = G sum_j m_j F(r,h_ij) d_ij,
// phi_i = -G sum_j m_j P(r,h_ij), d_ij = x_j - x_i, h_ij = max(h_i, h_j), the
// gradient with respect to particle k gathers over its partners i (d = x_k - x_i,
// w = m_k ga_i - m_i ga_k):
//   dL/dx_k = G sum_i [ w F + (w.d) (F_r/r) d + (m_k gp_i + m_i gp_k) F d ]
//   dL/dm_k = G sum_i [ (ga_i . d) F - gp_i P ]
//   dL/dh_k = G sum_i s_ki [ m_k ((ga_i . d) F_h - gp_i P_h)
//                          + m_i (-(ga_k . d) F_h - gp_k P_h) ]
// with s_ki = 1 if h_k > h_i, 1/2 if equal, 0 otherwise (the pair's radius
// belongs to the particle with the larger one).  The pair set of the direct
// sum is symmetric, so every target gathers its own gradient: no atomics.
//
// Direct path: the tile loop of the forward kernel, one target per lane, with
// source records that also carry the cotangents.  Sink targets take their
// sink-sink part from an FP64 kernel.
#include "sf_build.h"
#include "sf_math.h"
#include "sf_prims.h"

namespace sf {

template <typename R>
struct alignas(16) SrcRecB { R x, y, z, m, h2, h, gx, gy, gz, gp; int32_t idx, pad; };

// Gradient contribution of one pair to target k.  dd = x_src - x_k.
template <typename R, bool SOFT>
__device__ __forceinline__ void adj_pair(R ddx, R ddy, R ddz, const SrcRecB<R> &q, R mk, R gkx,
                                         R gky, R gkz, R gpk, R hk2, R hk, bool self, R &ox, R &oy,
                                         R &oz, R &om, R &oh) {
    const R r2 = ddx * ddx + ddy * ddy + ddz * ddz;
    const R ri = rsq(r2);
    const R ri2 = ri * ri;
    R F = ri * ri2, P = ri, FrR = R(-3) * F * ri2, dFh = R(0), dPh = R(0);
    bool soft = false;
    if (SOFT) {
        const R hh2 = q.h2 > hk2 ? q.h2 : hk2;
        if (r2 < hh2) {
            dsoft<R>(r2, q.h > hk ? q.h : hk, F, P, FrR, dFh, dPh);
            soft = true;
            if (self) { F = R(0); P = R(0); FrR = R(0); dFh = R(0); dPh = R(0); }
        }
    }
    const R wx = mk * q.gx - q.m * gkx;
    const R wy = mk * q.gy - q.m * gky;
    const R wz = mk * q.gz - q.m * gkz;
    const R wdd = wx * ddx + wy * ddy + wz * ddz;
    const R cc = mk * q.gp + q.m * gpk;
    const R s = wdd * FrR - cc * F;
    ox += wx * F + s * ddx;
    oy += wy * F + s * ddy;
    oz += wz * F + s * ddz;
    const R adn = q.gx * ddx + q.gy * ddy + q.gz * ddz;   // ga_i . dd
    om -= adn * F + q.gp * P;
    if (SOFT && soft) {
        const R share = hk > q.h ? R(1) : (hk == q.h ? R(0.5) : R(0));
        const R akd = gkx * ddx + gky * ddy + gkz * ddz;   // ga_k . dd
        oh += share * (mk * (-adn * dFh - q.gp * dPh) + q.m * (akd * dFh - gpk * dPh));
    }
}

template <typename T, int FORM>
__global__ __launch_bounds__(64) void k_tiles_b(int64_t n, int64_t n_gas, int64_t n_gas_tiles,
                                                int64_t n_tiles, const T *__restrict__ xs,
                                                const T *__restrict__ ys, const T *__restrict__ zs,
                                                const T *__restrict__ ms, const T *__restrict__ hs,
                                                const int32_t *__restrict__ order,
                                                const T *__restrict__ g_acc,
                                                const T *__restrict__ g_pot,
                                                int32_t *__restrict__ tfirst,
                                                int32_t *__restrict__ tcount,
                                                double *__restrict__ tbox, double *__restrict__ tcen,
                                                SrcRecB<typename FormT<FORM>::R> *__restrict__ rec) {
    using R = typename FormT<FORM>::R;
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
        for (int d = 0; d < 3; ++d) cen[d] = FormT<FORM>::rel ? (double)(T)(0.5 * (lo[d] + hi[d])) : 0.0;
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
            const int64_t o = order[p];
            SrcRecB<R> r;
            if (FormT<FORM>::rel) {
                r.x = (R)(v[0] - cen[0]);
                r.y = (R)(v[1] - cen[1]);
                r.z = (R)(v[2] - cen[2]);
            } else {
                r.x = (R)xs[p];
                r.y = (R)ys[p];
                r.z = (R)zs[p];
            }
            r.m = (R)ms[p];
            r.h = (R)hs[p];
            r.h2 = r.h * r.h;
            r.gx = (R)g_acc[3 * o];
            r.gy = (R)g_acc[3 * o + 1];
            r.gz = (R)g_acc[3 * o + 2];
            r.gp = g_pot ? (R)g_pot[o] : R(0);
            r.idx = (int32_t)p;
            r.pad = 0;
            rec[p] = r;
        }
    }
}

template <typename T, int FORM>
__global__ __launch_bounds__(256) void k_direct_b(int64_t n, int64_t n_gas, int64_t n_gas_tiles,
                                                  int64_t n_tiles, const int32_t *__restrict__ tfirst,
                                                  const int32_t *__restrict__ tcount,
                                                  const double *__restrict__ tbox,
                                                  const double *__restrict__ tcen,
                                                  const SrcRecB<typename FormT<FORM>::R> *__restrict__ rec,
                                                  const int32_t *__restrict__ order,
                                                  const double *__restrict__ ssb, double G,
                                                  T *__restrict__ g_pos, T *__restrict__ g_mass,
                                                  T *__restrict__ g_soft) {
    using R = typename FormT<FORM>::R;
    const int lane = threadIdx.x & 63;
    const int64_t tt = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tt >= n_tiles) return;
    const int64_t f = tfirst[tt], c = tcount[tt];
    const bool has = lane < c;
    const int64_t i = f + (has ? lane : 0);
    const SrcRecB<R> me = rec[i];
    const double wlo[3] = {tbox[8 * tt], tbox[8 * tt + 1], tbox[8 * tt + 2]};
    const double whi[3] = {tbox[8 * tt + 3], tbox[8 * tt + 4], tbox[8 * tt + 5]};
    const double whm = tbox[8 * tt + 6];
    const double wc[3] = {tcen[3 * tt], tcen[3 * tt + 1], tcen[3 * tt + 2]};
    const bool sink_tile = tt >= n_gas_tiles;
    const int64_t ns = sink_tile ? n_gas_tiles : n_tiles;
    Acc<FORM> ax, ay, az, am, ah;
    ax.zero(); ay.zero(); az.zero(); am.zero(); ah.zero();
    const int32_t my_idx = (int32_t)i;
    for (int64_t s = 0; s < ns; ++s) {
        const int64_t sf0 = tfirst[s], sc = tcount[s];
        double g2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            const double gd = fmax(fmax(tbox[8 * s + d] - whi[d], wlo[d] - tbox[8 * s + 3 + d]), 0.0);
            g2 += gd * gd;
        }
        const double hm = fmax(whm, tbox[8 * s + 6]);
        const bool near = g2 < hm * hm;
        R tx = me.x, ty = me.y, tz = me.z;
        if (FormT<FORM>::rel) {
            tx = me.x - (R)(tcen[3 * s] - wc[0]);
            ty = me.y - (R)(tcen[3 * s + 1] - wc[1]);
            tz = me.z - (R)(tcen[3 * s + 2] - wc[2]);
        }
        R bx = 0, by = 0, bz = 0, bm = 0, bh = 0;
        const SrcRecB<R> *src = rec + sf0;
        if (!near) {
            for (int64_t j = 0; j < sc; ++j) {
                const SrcRecB<R> q = src[j];
                adj_pair<R, false>(q.x - tx, q.y - ty, q.z - tz, q, me.m, me.gx, me.gy, me.gz, me.gp,
                                   me.h2, me.h, false, bx, by, bz, bm, bh);
            }
        } else {
            for (int64_t j = 0; j < sc; ++j) {
                const SrcRecB<R> q = src[j];
                adj_pair<R, true>(q.x - tx, q.y - ty, q.z - tz, q, me.m, me.gx, me.gy, me.gz, me.gp,
                                  me.h2, me.h, q.idx == my_idx, bx, by, bz, bm, bh);
            }
        }
        ax.fold(bx); ay.fold(by); az.fold(bz); am.fold(bm); ah.fold(bh);
    }
    if (!has) return;
    double v[5] = {ax.value(), ay.value(), az.value(), am.value(), ah.value()};
    if (sink_tile && ssb) {
        const int64_t ks = i - n_gas;
        for (int d = 0; d < 5; ++d) v[d] += ssb[5 * ks + d];
    }
    const int64_t o = order[i];
    if (g_pos) {
        g_pos[3 * o] = (T)(G * v[0]);
        g_pos[3 * o + 1] = (T)(G * v[1]);
        g_pos[3 * o + 2] = (T)(G * v[2]);
    }
    if (g_mass) g_mass[o] = (T)(G * v[3]);
    if (g_soft) g_soft[o] = (T)(G * v[4]);
}

// FP64 sink-sink adjoint: one wave per sink target, lanes stride the sources.
template <typename T>
__global__ __launch_bounds__(64) void k_sink_sink_b(const int32_t *__restrict__ sink_pos,
                                                    int64_t n_sink, const T *__restrict__ xs,
                                                    const T *__restrict__ ys,
                                                    const T *__restrict__ zs,
                                                    const T *__restrict__ ms,
                                                    const T *__restrict__ hs,
                                                    const int32_t *__restrict__ order,
                                                    const T *__restrict__ g_acc,
                                                    const T *__restrict__ g_pot,
                                                    double *__restrict__ ssb) {
    const int lane = threadIdx.x;
    for (int64_t k = blockIdx.x; k < n_sink; k += gridDim.x) {
        const int64_t p = sink_pos[k];
        const int64_t ok = order[p];
        const double tx = xs[p], ty = ys[p], tz = zs[p], th = hs[p], mk = ms[p];
        const double gkx = g_acc[3 * ok], gky = g_acc[3 * ok + 1], gkz = g_acc[3 * ok + 2];
        const double gpk = g_pot ? (double)g_pot[ok] : 0.0;
        double v[5] = {0, 0, 0, 0, 0};
        for (int64_t j = lane; j < n_sink; j += 64) {
            if (j == k) continue;
            const int64_t q = sink_pos[j];
            const int64_t oq = order[q];
            SrcRecB<double> r;
            r.x = xs[q]; r.y = ys[q]; r.z = zs[q]; r.m = ms[q]; r.h = hs[q]; r.h2 = r.h * r.h;
            r.gx = g_acc[3 * oq]; r.gy = g_acc[3 * oq + 1]; r.gz = g_acc[3 * oq + 2];
            r.gp = g_pot ? (double)g_pot[oq] : 0.0;
            r.idx = (int32_t)q;
            adj_pair<double, true>(r.x - tx, r.y - ty, r.z - tz, r, mk, gkx, gky, gkz, gpk,
                                   th * th, th, false, v[0], v[1], v[2], v[3], v[4]);
        }
        for (int d = 0; d < 5; ++d) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v[d] += __shfl_xor(v[d], off, 64);
        }
        if (lane == 0)
            for (int d = 0; d < 5; ++d) ssb[5 * k + d] = v[d];
    }
}

template <typename T>
static void sink_sink_backward(sf_grav_tree_s *t, const void *g_acc, const void *g_pot, double *ssb) {
    const unsigned blocks = (unsigned)std::min<int64_t>(t->n_sink, 8192);
    hipLaunchKernelGGL(k_sink_sink_b<T>, dim3(blocks), dim3(64), 0, t->stream, t->sink_pos,
                       t->n_sink, (const T *)t->xs, (const T *)t->ys, (const T *)t->zs,
                       (const T *)t->ms, (const T *)t->hs, t->order, (const T *)g_acc,
                       (const T *)g_pot, ssb);
}

template <typename T, int FORM>
static sf_status direct_backward_run(sf_grav_tree_s *t, const EvalOpts &o, const void *g_acc,
                                     const void *g_pot, void *g_pos, void *g_mass, void *g_soft,
                                     DevArena &ar) {
    using R = typename FormT<FORM>::R;
    hipStream_t s = t->stream;
    const int64_t n = t->n, ng = t->n_gas;
    t->n_gas_tiles = (ng + 63) / 64;
    t->n_tiles = t->n_gas_tiles + (n - ng + 63) / 64;
    SrcRecB<R> *rec;
    SF_ALLOC_TMP(ar, t->tfirst, t->n_tiles);
    SF_ALLOC_TMP(ar, t->tcount, t->n_tiles);
    SF_ALLOC_TMP(ar, t->tbox, 8 * t->n_tiles);
    SF_ALLOC_TMP(ar, t->tcen, 3 * t->n_tiles);
    SF_ALLOC_TMP(ar, rec, n);
    const unsigned tb = (unsigned)std::min<int64_t>(t->n_tiles, 8192);
    hipLaunchKernelGGL((k_tiles_b<T, FORM>), dim3(tb), dim3(64), 0, s, n, ng, t->n_gas_tiles,
                       t->n_tiles, (const T *)t->xs, (const T *)t->ys, (const T *)t->zs,
                       (const T *)t->ms, (const T *)t->hs, t->order, (const T *)g_acc,
                       (const T *)g_pot, t->tfirst, t->tcount, t->tbox, t->tcen, rec);
    double *ssb = nullptr;
    if (t->n_sink > 0) {
        SF_ALLOC_TMP(ar, ssb, 5 * t->n_sink);
        sink_sink_backward<T>(t, g_acc, g_pot, ssb);
    }
    const unsigned blocks = (unsigned)((t->n_tiles + 3) / 4);
    hipLaunchKernelGGL((k_direct_b<T, FORM>), dim3(blocks), dim3(256), 0, s, n, ng, t->n_gas_tiles,
                       t->n_tiles, t->tfirst, t->tcount, t->tbox, t->tcen, rec, t->order, ssb, o.G,
                       (T *)g_pos, (T *)g_mass, (T *)g_soft);
    SF_HIP(hipGetLastError());
    return SF_OK;
}

sf_status direct_backward(sf_grav_tree_s *t, const EvalOpts &o, const void *g_acc,
                          const void *g_pot, void *g_pos, void *g_mass, void *g_soft,
                          DevArena &ar) {
#define SF_B(T, F) return direct_backward_run<T, F>(t, o, g_acc, g_pot, g_pos, g_mass, g_soft, ar)
    if (t->dt == SF_F32) {
        if (o.form == SF_FP32C) SF_B(float, SF_FP32C);
        if (o.form == SF_FP32) SF_B(float, SF_FP32);
        SF_B(float, SF_FP64);
    }
    if (o.form == SF_FP32C) SF_B(double, SF_FP32C);
    if (o.form == SF_FP32) SF_B(double, SF_FP32);
    SF_B(double, SF_FP64);
#undef SF_B
}

sf_status tree_backward(sf_grav_tree_s *t, const EvalOpts &o, const void *g_acc,
                        const void *g_pot, void *g_pos, void *g_mass, void *g_soft,
                        DevArena &ar) {
    (void)t; (void)o; (void)g_acc; (void)g_pot; (void)g_pos; (void)g_mass; (void)g_soft; (void)ar;
    return sf_fail(SF_E_UNSUPPORTED, "tree adjoint not available yet");
}

}  // namespace sf
