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
#include "sf_split.h"
#include "sf_walk.h"

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

// Sink records for the sink-sink adjoint, gathered once into one contiguous
// FP64 array: x y z m h and the cotangents a_x a_y a_z phi of the sink.
constexpr int kSinkRecB = 9;

template <typename T>
__global__ void k_sink_gather_b(const int32_t *__restrict__ sink_pos, int64_t n_sink,
                                const T *__restrict__ xs, const T *__restrict__ ys,
                                const T *__restrict__ zs, const T *__restrict__ ms,
                                const T *__restrict__ hs, const int32_t *__restrict__ order,
                                const T *__restrict__ g_acc, const T *__restrict__ g_pot,
                                double *__restrict__ rec) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_sink) return;
    const int64_t p = sink_pos[k];
    const int64_t o = order[p];
    double *r = rec + kSinkRecB * k;
    r[0] = (double)xs[p];
    r[1] = (double)ys[p];
    r[2] = (double)zs[p];
    r[3] = (double)ms[p];
    r[4] = (double)hs[p];
    r[5] = (double)g_acc[3 * o];
    r[6] = (double)g_acc[3 * o + 1];
    r[7] = (double)g_acc[3 * o + 2];
    r[8] = g_pot ? (double)g_pot[o] : 0.0;
}

// FP64 sink-sink adjoint: one wave per sink target, lanes stride the sources.
__global__ __launch_bounds__(64) void k_sink_sink_b(const double *__restrict__ rec,
                                                    int64_t n_sink, double *__restrict__ ssb) {
    const int lane = threadIdx.x;
    for (int64_t k = blockIdx.x; k < n_sink; k += gridDim.x) {
        const double *t = rec + kSinkRecB * k;
        const double tx = t[0], ty = t[1], tz = t[2], mk = t[3], th = t[4];
        const double gkx = t[5], gky = t[6], gkz = t[7], gpk = t[8];
        double v[5] = {0, 0, 0, 0, 0};
        for (int64_t j = lane; j < n_sink; j += 64) {
            if (j == k) continue;
            const double *q = rec + kSinkRecB * j;
            SrcRecB<double> r;
            r.x = q[0]; r.y = q[1]; r.z = q[2]; r.m = q[3]; r.h = q[4]; r.h2 = r.h * r.h;
            r.gx = q[5]; r.gy = q[6]; r.gz = q[7]; r.gp = q[8];
            r.idx = -1;
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

// rec: scratch for kSinkRecB doubles per sink.
template <typename T>
static void sink_sink_backward(sf_grav_tree_s *t, const void *g_acc, const void *g_pot, double *ssb,
                               double *rec, hipStream_t st) {
    const unsigned gb = (unsigned)((t->n_sink + 255) / 256);
    hipLaunchKernelGGL(k_sink_gather_b<T>, dim3(gb), dim3(256), 0, st, t->sink_pos, t->n_sink,
                       (const T *)t->xs, (const T *)t->ys, (const T *)t->zs, (const T *)t->ms,
                       (const T *)t->hs, t->order, (const T *)g_acc, (const T *)g_pot, rec);
    const unsigned blocks = (unsigned)std::min<int64_t>(t->n_sink, 8192);
    hipLaunchKernelGGL(k_sink_sink_b, dim3(blocks), dim3(64), 0, st, (const double *)rec,
                       t->n_sink, ssb);
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
        double *srec;
        SF_ALLOC_TMP(ar, ssb, 5 * t->n_sink);
        SF_ALLOC_TMP(ar, srec, kSinkRecB * t->n_sink);
        sink_sink_backward<T>(t, g_acc, g_pot, ssb, srec, s);
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

// ---------------------------------------------------------------- tree adjoint
//
// The tree result is a sum over the frozen interaction lists of pair terms
// (target i, particle j) and node terms (target i, node n with mass M, centre
// of mass c, traceless quadrupole Q).  Its gradient has three parts:
//   * target side: d/dx_i, d/dh_i of the target's own terms (gathered in the
//     registers of the lanes that own the target, as in the forward walk);
//   * source side: d/dx_j, d/dm_j, d/dh_j of pair terms (each term is
//     evaluated once, by the target's lane, and added to the source's LDS
//     accumulator; one FP64 atomic add per source and value and batch);
//   * node side: d/dM, d/dc, d/dQ of node terms (accumulated the same way),
//     later pushed down to every particle of the node through M = sum m,
//     c = sum m x / M, Q = sum m (3 y y^T - |y|^2 I), y = x - c.
// Opening decisions are held fixed, so this is the exact derivative of the
// tree approximation as evaluated.

// Pair (target i, source j), d = x_j - x_i: S = dT/dx_j (target gets -S),
// Tm = dT/dm_j, Th = dT/dh_ij, share_i = part of Th owned by the target.
// With F(r) the force factor, S = m_j (F a + (a.d F'/r + phi F) d) for
// cotangents a (acceleration) and phi (potential).
template <typename R, bool SOFT = true>
__device__ __forceinline__ void bpair(R dx, R dy, R dz, R mj, R hj2, R hj, R hi2, R hi, R gax,
                                      R gay, R gaz, R gp, bool self, R &Sx, R &Sy, R &Sz, R &Tm,
                                      R &Th, R &share_i) {
    const R r2 = dx * dx + dy * dy + dz * dz;
    const R ri = rsq(r2);
    const R ri2 = ri * ri;
    const R ad = gax * dx + gay * dy + gaz * dz;
    R F = ri * ri2, P = ri, mc1;
    Th = R(0);
    if (!SOFT) {
        // Newtonian: F'/r = -3 F / r^2
        const R mF = mj * F;
        mc1 = mF * fma(ad * ri2, R(-3), gp);
        Sx = fma(mc1, dx, mF * gax);
        Sy = fma(mc1, dy, mF * gay);
        Sz = fma(mc1, dz, mF * gaz);
    } else {
        R FrR = R(-3) * F * ri2, dFh = R(0), dPh = R(0);
        const R hh2 = hj2 > hi2 ? hj2 : hi2;
        const bool soft = r2 < hh2;
        if (soft) {
            const R hh = pos_max(hj, hi);
            dsoft_ri<R>(r2, ri, hh, rcp(hh), F, P, FrR, dFh, dPh);
            if (self) { F = R(0); P = R(0); FrR = R(0); dFh = R(0); dPh = R(0); }
            Th = mj * (ad * dFh - gp * dPh);
        }
        const R mF = mj * F;
        mc1 = mj * fma(ad, FrR, gp * F);
        Sx = fma(mc1, dx, mF * gax);
        Sy = fma(mc1, dy, mF * gay);
        Sz = fma(mc1, dz, mF * gaz);
    }
    Tm = fma(ad, F, -gp * P);
    share_i = hi > hj ? R(1) : (hi == hj ? R(0.5) : R(0));
}

// Node term, r = x_i - c: g = dL/dr (the centre of mass gets -g), gM = dL/dM,
// gq = dL/dQ as 5 numbers (zero for monopoles).  With the forward term
// phi = -M/r - s/(2 r^5), a = -M r/r^3 + q/r^5 - 5 s r/(2 r^7) (q = Q r,
// s = r.q) and L = a_bar.a + phi_bar phi:
//   g = c_r r + c_a a_bar + c_q q + Q a_bar / r^5,
//   c_r = 3 M ra/r^5 + phi_bar M/r^3 + (35/2 s ra/r^2 + 5/2 phi_bar s
//         - 5 a_bar.q)/r^7,  c_a = -M/r^3 - 5/2 s/r^7,
//   c_q = -5 ra/r^7 - phi_bar/r^5,  ra = r.a_bar.
// Q is traceless, so dL/dQ matters only up to a multiple of the identity;
// written as G = (w r^T + r w^T)/2 with w = a_bar/r^5 + (c_q/2) r, the five
// numbers are G_xx - G_zz, G_yy - G_zz, 2 G_xy, 2 G_xz, 2 G_yz.  Since
// Q w = Q a_bar/r^5 + (c_q/2) q, the g above is also c_r r + c_a a_bar
// + (c_q/2) q + Q w, which shares w with dL/dQ.
template <typename R, int ORDER>
__device__ __forceinline__ void bmultipole(R rx, R ry, R rz, R M, R qxx, R qyy, R qxy, R qxz,
                                           R qyz, R gax, R gay, R gaz, R gp, R &gx, R &gy,
                                           R &gz, R &gM, R gq[5]) {
    const R r2 = rx * rx + ry * ry + rz * rz;
    const R ri = rsq(r2);
    const R u = ri * ri;                      // 1/r^2
    const R ri3 = ri * u;
    const R ra = rx * gax + ry * gay + rz * gaz;
    const R t = ra * u;                       // (r . a_bar)/r^2
    gM = -ri * (t + gp);                      // -(ra/r^3 + phi/r)
    const R Mri3 = M * ri3;
    const R cm = Mri3 * fma(R(3), t, gp);     // monopole part of c_r: M (3 ra/r^5 + phi/r^3)
    if (ORDER != 2) {
        gx = fma(cm, rx, -Mri3 * gax);
        gy = fma(cm, ry, -Mri3 * gay);
        gz = fma(cm, rz, -Mri3 * gaz);
        for (int d = 0; d < 5; ++d) gq[d] = R(0);
        return;
    }
    const R qzz = -(qxx + qyy);
    const R qx = qxx * rx + qxy * ry + qxz * rz;
    const R qy = qxy * rx + qyy * ry + qyz * rz;
    const R qz = qxz * rx + qyz * ry + qzz * rz;
    const R sq = qx * rx + qy * ry + qz * rz;
    const R aQr = gax * qx + gay * qy + gaz * qz;
    const R ri5 = ri3 * u;
    const R ri7 = ri5 * u;
    const R s5 = R(2.5) * sq;
    // c_r = cm + (35/2 s ra/r^2 + 5/2 phi s - 5 aQr)/r^7 = cm + (s5 (7 t + phi) - 5 aQr)/r^7
    const R cr = fma(ri7, fma(s5, fma(R(7), t, gp), R(-5) * aQr), cm);
    const R ca = -fma(s5, ri7, Mri3);         // -(M/r^3 + 5/2 s/r^7)
    // hc = c_q / 2 with c_q = -(5 ra/r^7 + phi/r^5); dL/dQ's vector is
    // w = r^-5 a_bar + hc r, and c_q q + Q a_bar/r^5 = Q w + hc q
    const R hc = R(-0.5) * ri5 * fma(R(5), t, gp);
    const R wx = fma(hc, rx, ri5 * gax);
    const R wy = fma(hc, ry, ri5 * gay);
    const R wz = fma(hc, rz, ri5 * gaz);
    const R Qwx = qxx * wx + qxy * wy + qxz * wz;
    const R Qwy = qxy * wx + qyy * wy + qyz * wz;
    const R Qwz = qxz * wx + qyz * wy + qzz * wz;
    gx = fma(cr, rx, fma(ca, gax, fma(hc, qx, Qwx)));
    gy = fma(cr, ry, fma(ca, gay, fma(hc, qy, Qwy)));
    gz = fma(cr, rz, fma(ca, gaz, fma(hc, qz, Qwz)));
    const R pz = wz * rz;
    gq[0] = fma(wx, rx, -pz);
    gq[1] = fma(wy, ry, -pz);
    gq[2] = fma(wx, ry, wy * rx);
    gq[3] = fma(wx, rz, wz * rx);
    gq[4] = fma(wy, rz, wz * ry);
}

template <typename T>
struct WalkArgsB {
    WalkNodes nd;
    const T *xs, *ys, *zs, *ms, *hs;
    const int32_t *order;
    int64_t n, n_gas;
    const int32_t *n_groups_dev, *gfirst, *gcount;
    const double *gbox, *ghmax, *gcen;
    const int32_t *sink_pos;
    int64_t n_sink;
    const T *g_acc, *g_pot;     // caller order
    double *tgt;                // 5 per sorted particle: target side (x y z m h)
    // Atomic arrays, kXcd copies each.  Particle values component-major
    // (value c of particle p at c n + p): a batch's particles come from a few
    // leaves, so one add instruction over the batch touches a few cache
    // lines.  Node values of the group walk node-major (value c of node k at
    // 9 k + c): a batch's nodes are scattered, so its 9 values per node are
    // added by consecutive lanes, which keeps each add instruction on a few
    // lines.  The sink walk, one node per lane, adds component-major (value
    // c at c n_nodes + k), so a lane's 9 adds do not queue on one line.
    double *scat;               // 5 per sorted particle: source side (x y z m h)
    double *nadj;               // 9 per node: M, c(3), dQ(5)
    int64_t scat_stride, nadj_stride;   // elements between copies
    const uint32_t *gperm;      // task -> group (costly groups first), or null: Morton order
    int32_t *task_ctr, *err;
    uint32_t *gstack;           // kStack entries per block: stack overflow area
};

// Per-lane target of the group adjoint.
template <typename R> struct TgtB { R x, y, z, h, h2, gx, gy, gz, gp; int32_t idx; };

__device__ __forceinline__ void atomic_add_f64(double *p, double v) { unsafeAtomicAdd(p, v); }

// Positions of staged dummy entries and of lanes that take no part (no
// target, or a sink target): far enough that every term with them vanishes
// or underflows, near enough that no square or quadrupole product overflows
// FP32.
constexpr float kFarB = 1e15f;
constexpr float kFarT = -1e15f;

// FP64 LDS atomic add (ds_add_f64).
__device__ __forceinline__ void lds_add(double *p, double v) { unsafeAtomicAdd(p, v); }

// LDS for the FP64 form's entry-side sums (none for the FP32 forms).
template <typename R> struct BAccMem {
    __device__ double (*ptr())[64] { return nullptr; }
};
template <> struct BAccMem<double> {
    double v[9][64];
    __device__ double (*ptr())[64] { return v; }
};

// Value of v in the lane whose byte address (4 x lane) is src.
__device__ __forceinline__ float lane_take(int src, float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(v)));
}
__device__ __forceinline__ double lane_take(int src, double v) {
    const int lo = __builtin_amdgcn_ds_bpermute(src, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(src, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Group tasks, one pass per batch: each (target, entry) term is evaluated
// once and split into its target side (kept in the registers of the lanes
// that own the target) and its entry side.
//
// Lane splitting as in the forward walk: a group of gc targets gets
// k = floor(64 / gc) copies of each target, lane t + gc*c holding copy c of
// target t.  A batch holds at most k gc entries (the walk is run with
// batches of that size); entry e is staged in slot (e mod k) gc + e / k, so
// copy c owns the gc slots [c gc, c gc + gc).  In step s (of gc) the lane of
// target t takes slot c gc + (t + s) mod gc: the lanes of a step sit on
// different slots, and every lane meets every slot of its copy once.  The
// entry-side sums live in registers and travel with their slot: the slot a
// lane takes in step s + 1 is the one its right-hand neighbour (cyclically,
// within the copy) held in step s, so one lane shuffle per value hands all
// of them on.  After the last step the sums are written to LDS by slot and
// flushed with one FP64 global atomic add per entry and value.  (LDS atomic
// adds measured slower on gfx950, FP32 ones by an order of magnitude; a
// read-add-write of LDS records exposes the LDS latency in every step.)
// The FP64 form keeps FP64 LDS atomic adds instead: its hand-off needs two
// shuffles per value, which measured slower than the adds.
//
// Padding entries are zero-mass dummies far away; lanes without a target (a
// sink target, in the FP64 form the lanes past the group's size, or lanes
// from k gc on) sit far away on the other side with
// zero cotangents, so both contribute exact zeros to every real sum, and no
// step needs a predicate.  Lanes from k gc on keep to slot = their lane,
// which holds a dummy and is never flushed.
template <typename T, int FORM, int ORDER>
struct GroupEvalB {
    using R = typename FormT<FORM>::R;
    const WalkArgsB<T> *a;
    // Batch entries staged structure-of-arrays: the lanes of a step read
    // different slots, and one component of consecutive slots sits in
    // consecutive LDS words, so those reads are free of bank conflicts.
    // After a batch's steps the same rows hold its entry-side sums by slot.
    R (*stg)[64];               // [9][64]: x y z m|M, then h2 h (pairs) or Q (nodes)
    int32_t *sidx;              // [64] particle index of a pair entry
    double (*bacc)[64];         // [9][64] FP64 form: entry-side sums by slot
    double *scat, *nadj;        // this XCD's copies of the atomic arrays
    double cen[3];
    TgtB<R> me;
    static constexpr bool kShuffle = sizeof(R) == 4;
    uint32_t gc, k, nslot;      // copy width (the group size), copies, k gc slots in use
    uint32_t tl, base;          // this lane's target and the first slot of its copy
    bool inslot;                // lane < k gc
    int src;                    // byte address of the lane that hands this lane its next slot
    uint32_t held_last;         // slot this lane holds after a batch's last step
    uint32_t stslot;            // slot of the entry this lane stages
    Acc<FORM> ox, oy, oz, oh;

    // The FP64 form, whose entry sums are LDS atomic adds rather than a
    // hand-off, takes gc rounded up to a power of two as the copy width (the
    // lanes past the group's size hold no target), so that every batch holds
    // 64 entries: with no hand-off, smaller batches would only add flushes.
    __device__ void setup(uint32_t gcount, uint32_t lane) {
        gc = gcount;
        if constexpr (!kShuffle) {
            gc = 1u;
            while (gc < gcount) gc <<= 1;
        }
        k = 64u / gc;
        nslot = k * gc;
        tl = lane % gc;
        const uint32_t c = lane / gc;
        inslot = lane < nslot;
        base = c * gc;
        const uint32_t nxt = tl + 1u == gc ? 0u : tl + 1u;
        src = (int)((inslot ? base + nxt : lane) << 2);
        const uint32_t last = tl == 0u ? gc - 1u : tl - 1u;   // (tl + gc - 1) mod gc
        held_last = inslot ? base + last : lane;
        // lane e stages batch entry e: entries e < nslot fill the slots in
        // use, the other lanes their own unused slot
        stslot = inslot ? (lane % k) * gc + lane / k : lane;
    }

    template <int NV>
    __device__ __forceinline__ void pass_on(R (&acc)[NV]) const {
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = lane_take(src, acc[v]);
    }

    __device__ void pc_batch(WalkLds &L, uint32_t head, uint32_t nb) {
        constexpr int NV = ORDER == 2 ? 9 : 4;
        const uint32_t e = threadIdx.x;
        const uint32_t slot = stslot;
        int node = -1;
        if (e < nb) {
            node = L.pc[(head + e) & 127];
            const WalkNodes &nd = a->nd;
            stg[0][slot] = dto_frame<FORM>(nd.w[node].com[0], cen[0]);
            stg[1][slot] = dto_frame<FORM>(nd.w[node].com[1], cen[1]);
            stg[2][slot] = dto_frame<FORM>(nd.w[node].com[2], cen[2]);
            stg[3][slot] = (R)nd.w[node].M;
            for (int d = 0; d < 5; ++d) stg[4 + d][slot] = ORDER == 2 ? (R)nd.q[node].q[d] : R(0);
        } else {
            stg[0][slot] = stg[1][slot] = stg[2][slot] = R(kFarB);
            for (int d = 3; d < 9; ++d) stg[d][slot] = R(0);
        }
        __syncthreads();
        R acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = R(0);
        R bx = 0, by = 0, bz = 0;
        uint32_t jj = tl;   // (tl + s) mod gc
        for (uint32_t s = 0; s < gc; ++s) {
            const uint32_t j = inslot ? base + jj : threadIdx.x;
            jj = jj + 1u == gc ? 0u : jj + 1u;
            R q5[5] = {R(0), R(0), R(0), R(0), R(0)};
            if (ORDER == 2)
                for (int d = 0; d < 5; ++d) q5[d] = stg[4 + d][j];
            R gx, gy, gz, gM, gq[5];
            bmultipole<R, ORDER>(me.x - stg[0][j], me.y - stg[1][j], me.z - stg[2][j], stg[3][j],
                                 q5[0], q5[1], q5[2], q5[3], q5[4], me.gx, me.gy, me.gz, me.gp,
                                 gx, gy, gz, gM, gq);
            bx += gx;
            by += gy;
            bz += gz;
            if constexpr (kShuffle) {
                acc[0] += gM;
                acc[1] -= gx;
                acc[2] -= gy;
                acc[3] -= gz;
                if (ORDER == 2)
                    for (int d = 0; d < 5; ++d) acc[4 + d] += gq[d];
                if (s + 1 < gc) pass_on<NV>(acc);
            } else {
                lds_add(&bacc[0][j], (double)gM);
                lds_add(&bacc[1][j], (double)-gx);
                lds_add(&bacc[2][j], (double)-gy);
                lds_add(&bacc[3][j], (double)-gz);
                if (ORDER == 2)
                    for (int d = 0; d < 5; ++d) lds_add(&bacc[4 + d][j], (double)gq[d]);
            }
        }
        ox.fold(bx);
        oy.fold(by);
        oz.fold(bz);
        flush_nodes<NV>(acc, L, head, nb);
        (void)node;
    }

    // Node-side sums of a finished batch to the node-major FP64 array: the
    // nb x NV values are taken in entry-major order, 64 consecutive ones per
    // add instruction (value d of entry e at 9 node(e) + d).
    template <int NV>
    __device__ __forceinline__ void flush_nodes(const R (&acc)[NV], const WalkLds &L,
                                                uint32_t head, uint32_t nb) {
        const uint32_t e = threadIdx.x;
        sidx[e] = (int32_t)stslot;   // slot of entry e (unused by node batches otherwise)
        __syncthreads();   // every lane is done reading the staged entries
        if constexpr (kShuffle) {
#pragma unroll
            for (int v = 0; v < NV; ++v) stg[v][held_last] = acc[v];
            __syncthreads();
        }
        const uint32_t tot = nb * NV;
        for (uint32_t q = e; q < tot; q += 64u) {
            const uint32_t en = q / NV;
            const uint32_t d = q - en * NV;
            const int32_t sl = sidx[en];
            const int nd = L.pc[(head + en) & 127];
            double v;
            if constexpr (kShuffle) v = (double)stg[d][sl];
            else v = bacc[d][sl];
            atomic_add_f64(nadj + (int64_t)nd * 9 + d, v);
        }
        __syncthreads();
        if constexpr (!kShuffle) {
            for (int d = 0; d < NV; ++d) bacc[d][e] = 0.0;
            __syncthreads();
        }
    }

    // Entry-side sums of a finished batch to the global FP64 arrays: value d
    // of entry e goes to out_e[d * stride] (out_e = base array + entry index).
    template <int NV>
    __device__ __forceinline__ void flush(const R (&acc)[NV], uint32_t nb, uint32_t slot,
                                          double *out_e, int64_t stride) {
        const uint32_t e = threadIdx.x;
        __syncthreads();   // every lane is done reading the staged entries
        if constexpr (kShuffle) {
#pragma unroll
            for (int v = 0; v < NV; ++v) stg[v][held_last] = acc[v];
            __syncthreads();
            if (e < nb) {
                // all values read before the first add, so the LDS reads overlap
                R w[NV];
#pragma unroll
                for (int d = 0; d < NV; ++d) w[d] = stg[d][slot];
#pragma unroll
                for (int d = 0; d < NV; ++d) atomic_add_f64(out_e + d * stride, (double)w[d]);
            }
        } else {
            if (e < nb)
                for (int d = 0; d < NV; ++d) atomic_add_f64(out_e + d * stride, bacc[d][slot]);
            __syncthreads();
            for (int d = 0; d < NV; ++d) bacc[d][e] = 0.0;
        }
        __syncthreads();
    }

    template <bool SOFT>
    __device__ void pp_batch(WalkLds &L, uint32_t nb) {
        constexpr int NV = SOFT ? 5 : 4;
        const uint32_t e = threadIdx.x;
        const uint32_t slot = stslot;
        int p = -1;
        if (e < nb) {
            p = L.slot[e];
            stg[0][slot] = to_frame<FORM>(a->xs[p], cen[0]);
            stg[1][slot] = to_frame<FORM>(a->ys[p], cen[1]);
            stg[2][slot] = to_frame<FORM>(a->zs[p], cen[2]);
            stg[3][slot] = (R)a->ms[p];
            const R h = (R)a->hs[p];
            stg[4][slot] = h * h;
            stg[5][slot] = h;
            sidx[slot] = p;
        } else {
            stg[0][slot] = stg[1][slot] = stg[2][slot] = R(kFarB);
            stg[3][slot] = stg[4][slot] = stg[5][slot] = R(0);
            sidx[slot] = -1;
        }
        __syncthreads();
        R acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = R(0);
        R bx = 0, by = 0, bz = 0, bh = 0;
        uint32_t jj = tl;   // (tl + s) mod gc
        for (uint32_t s = 0; s < gc; ++s) {
            const uint32_t j = inslot ? base + jj : threadIdx.x;
            jj = jj + 1u == gc ? 0u : jj + 1u;
            R Sx, Sy, Sz, Tm, Th, sh;
            const R hj2 = SOFT ? stg[4][j] : R(0), hj = SOFT ? stg[5][j] : R(0);
            const bool self = SOFT && sidx[j] == me.idx;
            bpair<R, SOFT>(stg[0][j] - me.x, stg[1][j] - me.y, stg[2][j] - me.z, stg[3][j], hj2,
                           hj, me.h2, me.h, me.gx, me.gy, me.gz, me.gp, self, Sx, Sy, Sz, Tm, Th,
                           sh);
            bx -= Sx;
            by -= Sy;
            bz -= Sz;
            if (SOFT) bh += sh * Th;
            if constexpr (kShuffle) {
                acc[0] += Sx;
                acc[1] += Sy;
                acc[2] += Sz;
                acc[3] += Tm;
                if (SOFT) acc[NV - 1] += (R(1) - sh) * Th;
                if (s + 1 < gc) pass_on<NV>(acc);
            } else {
                lds_add(&bacc[0][j], (double)Sx);
                lds_add(&bacc[1][j], (double)Sy);
                lds_add(&bacc[2][j], (double)Sz);
                lds_add(&bacc[3][j], (double)Tm);
                if (SOFT) lds_add(&bacc[NV - 1][j], (double)((R(1) - sh) * Th));
            }
        }
        ox.fold(bx);
        oy.fold(by);
        oz.fold(bz);
        if (SOFT) oh.fold(bh);
        flush<NV>(acc, nb, slot, scat + p, a->n);
    }
};

// At least three waves per SIMD: binds only the FP64 form (the FP32 forms
// fit four in their registers), which without it took more registers than
// three waves allow.
template <typename T, int FORM, int ORDER>
__global__ __launch_bounds__(64, 3) void k_walk_groups_b(WalkArgsB<T> a) {
    using R = typename FormT<FORM>::R;
    __shared__ WalkLds L;
    __shared__ R stg[9][64];
    __shared__ int32_t sidx[64];
    __shared__ BAccMem<R> bmem;
    const int lane = threadIdx.x;
    const int ng = __builtin_amdgcn_readfirstlane(*a.n_groups_dev);
    GroupEvalB<T, FORM, ORDER> ev;
    ev.a = &a;
    ev.stg = stg;
    ev.sidx = sidx;
    ev.bacc = bmem.ptr();
    if (ev.bacc)
        for (int d = 0; d < 9; ++d) ev.bacc[d][lane] = 0.0;
    const int xcd = xcd_id();
    ev.scat = a.scat + xcd * a.scat_stride;
    ev.nadj = a.nadj + xcd * a.nadj_stride;
    for (int tk = next_task(a.task_ctr); tk < ng; tk = next_task(a.task_ctr)) {
        const int g = a.gperm ? __builtin_amdgcn_readfirstlane((int)a.gperm[tk]) : tk;
        if (g < 0 || g >= ng) continue;   // a cost order is a permutation of the groups
        const int64_t gf = a.gfirst[g], gc = a.gcount[g];
        double blo[3], bhi[3];
        for (int d = 0; d < 3; ++d) {
            blo[d] = a.gbox[6 * g + d];
            bhi[d] = a.gbox[6 * g + 3 + d];
            ev.cen[d] = a.gcen[3 * g + d];
        }
        const double hg = a.ghmax[g];
        ev.setup((uint32_t)gc, (uint32_t)lane);
        const bool has = ev.tl < (uint32_t)gc;   // false only past the group in the FP64 form
        const int64_t i = gf + (has ? ev.tl : 0u);
        const bool active = ev.inslot && has && a.order[i] < a.n_gas;
        if (__ballot(active) == 0ull) continue;
        const int64_t o = a.order[i];
        TgtB<R> &me = ev.me;
        if (active) {
            me.x = to_frame<FORM>(a.xs[i], ev.cen[0]);
            me.y = to_frame<FORM>(a.ys[i], ev.cen[1]);
            me.z = to_frame<FORM>(a.zs[i], ev.cen[2]);
            me.h = (R)a.hs[i];
            me.gx = (R)a.g_acc[3 * o];
            me.gy = (R)a.g_acc[3 * o + 1];
            me.gz = (R)a.g_acc[3 * o + 2];
            me.gp = a.g_pot ? (R)a.g_pot[o] : R(0);
            me.idx = (int32_t)i;
        } else {
            me.x = me.y = me.z = R(kFarT);
            me.h = me.gx = me.gy = me.gz = me.gp = R(0);
            me.idx = -1;
        }
        me.h2 = me.h * me.h;
        ev.ox.zero();
        ev.oy.zero();
        ev.oz.zero();
        ev.oh.zero();
        uint32_t npc, npp;
        uint64_t cks;
        walk_task<false>(a.nd, L, a.gstack + (int64_t)blockIdx.x * kStack, ev, blo, bhi, hg, gf,
                         gf + gc, task_ag_group(a.nd, g), a.err, npc, npp, cks, ev.nslot,
                         ev.nslot);
        double v[4] = {ev.ox.value(), ev.oy.value(), ev.oz.value(), ev.oh.value()};
        // sum the k copies of each target in a fixed order, through LDS (the
        // stage is free once the task's batches are done)
        Split sp;
        sp.gc = ev.gc;
        sp.k = ev.k;
        sp.template reduce<sizeof(stg) / (64 * sizeof(double))>(
            v, reinterpret_cast<double *>(&stg[0][0]), (uint32_t)lane);
        if (active && (uint32_t)lane < ev.gc) {
            a.tgt[5 * i] = v[0];
            a.tgt[5 * i + 1] = v[1];
            a.tgt[5 * i + 2] = v[2];
            a.tgt[5 * i + 3] = 0.0;
            a.tgt[5 * i + 4] = v[3];
        }
    }
}

template <typename T, int FORM, int ORDER>
struct SinkEvalB {
    using R = typename FormT<FORM>::R;
    const WalkArgsB<T> *a;
    double *scat, *nadj;        // this XCD's copies of the atomic arrays
    double cen[3];
    R th, th2, gx, gy, gz, gp;
    int32_t tidx;
    Acc<FORM> ox, oy, oz, oh;   // per lane partials of the target side

    __device__ void pc_batch(WalkLds &L, uint32_t head, uint32_t nb) {
        const int lane = threadIdx.x;
        R bx = 0, by = 0, bz = 0;
        if ((uint32_t)lane < nb) {
            const int node = L.pc[(head + lane) & 127];
            const WalkNodes &nd = a->nd;
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
            R g0, g1, g2, gM, gq[5];
            bmultipole<R, ORDER>(tx - cx, ty - cy, tz - cz, (R)nd.w[node].M, qxx, qyy, qxy, qxz, qyz,
                                 gx, gy, gz, gp, g0, g1, g2, gM, gq);
            bx = g0;
            by = g1;
            bz = g2;
            // component-major (one node per lane: a lane's 9 adds go to 9 lines)
            const int64_t nn = a->nd.n_nodes;
            atomic_add_f64(nadj + node, (double)gM);
            atomic_add_f64(nadj + nn + node, -(double)g0);
            atomic_add_f64(nadj + 2 * nn + node, -(double)g1);
            atomic_add_f64(nadj + 3 * nn + node, -(double)g2);
            if (ORDER == 2)
                for (int d = 0; d < 5; ++d) atomic_add_f64(nadj + (4 + d) * nn + node, (double)gq[d]);
        }
        ox.fold(bx);
        oy.fold(by);
        oz.fold(bz);
    }

    template <bool SOFT>
    __device__ void pp_batch(WalkLds &L, uint32_t nb) {
        const int lane = threadIdx.x;
        R bx = 0, by = 0, bz = 0, bh = 0;
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
                R Sx, Sy, Sz, Tm, Th, sh;
                bpair<R, SOFT>(sx - tx, sy - ty, sz - tz, (R)a->ms[p], h * h, h, th2, th, gx, gy,
                               gz, gp, p == tidx, Sx, Sy, Sz, Tm, Th, sh);
                bx = -Sx;
                by = -Sy;
                bz = -Sz;
                bh = sh * Th;
                const int64_t n = a->n;
                atomic_add_f64(scat + p, (double)Sx);
                atomic_add_f64(scat + n + p, (double)Sy);
                atomic_add_f64(scat + 2 * n + p, (double)Sz);
                atomic_add_f64(scat + 3 * n + p, (double)Tm);
                atomic_add_f64(scat + 4 * n + p, (double)((R(1) - sh) * Th));
            }
        }
        ox.fold(bx);
        oy.fold(by);
        oz.fold(bz);
        oh.fold(bh);
        __syncthreads();
    }
};

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T, int FORM, int ORDER>
__global__ __launch_bounds__(64) void k_walk_sinks_b(WalkArgsB<T> a) {
    using R = typename FormT<FORM>::R;
    __shared__ WalkLds L;
    const int lane = threadIdx.x;
    SinkEvalB<T, FORM, ORDER> ev;
    ev.a = &a;
    const int xcd = xcd_id();
    ev.scat = a.scat + xcd * a.scat_stride;
    ev.nadj = a.nadj + xcd * a.nadj_stride;
    for (int k = next_task(a.task_ctr); k < a.n_sink; k = next_task(a.task_ctr)) {
        const int64_t p = a.sink_pos[k];
        const int64_t o = a.order[p];
        double b[3] = {(double)a.xs[p], (double)a.ys[p], (double)a.zs[p]};
        for (int d = 0; d < 3; ++d) ev.cen[d] = b[d];
        ev.th = (R)a.hs[p];
        ev.th2 = ev.th * ev.th;
        ev.gx = (R)a.g_acc[3 * o];
        ev.gy = (R)a.g_acc[3 * o + 1];
        ev.gz = (R)a.g_acc[3 * o + 2];
        ev.gp = a.g_pot ? (R)a.g_pot[o] : R(0);
        ev.tidx = (int32_t)p;
        ev.ox.zero();
        ev.oy.zero();
        ev.oz.zero();
        ev.oh.zero();
        uint32_t npc, npp;
        uint64_t cks;
        walk_task<false>(a.nd, L, a.gstack + (int64_t)blockIdx.x * kStack, ev, b, b,
                         (double)a.hs[p], p, p + 1, task_ag_point(a.nd, p), a.err, npc, npp, cks);
        const double s0 = wave_sum_d(ev.ox.value()), s1 = wave_sum_d(ev.oy.value());
        const double s2 = wave_sum_d(ev.oz.value()), s4 = wave_sum_d(ev.oh.value());
        if (lane == 0) {
            a.tgt[5 * p] = s0;
            a.tgt[5 * p + 1] = s1;
            a.tgt[5 * p + 2] = s2;
            a.tgt[5 * p + 3] = 0.0;
            a.tgt[5 * p + 4] = s4;
        }
    }
}

// Sort keys for the adjoint's task order.  With at most kFineOrderGroups
// groups per resident wave (a few tasks per wave, so the last costly group
// to start sets the end): decreasing cost (a stable sort keeps Morton order
// among equal costs; 4 passes).  With more: cost classes (powers of two)
// from the most costly down and Morton order within a class, so that
// neighbouring groups, which read the same nodes, stay close in time (key
// bits 0..39: index below 2^32, class below 32; 5 passes).
constexpr int64_t kFineOrderGroups = 32;
__global__ void k_cost_keys(const uint32_t *__restrict__ cost, int64_t n, int fine,
                            uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t c = cost[i];
    if (fine) {
        keys[i] = 0xffffffffull - c;
    } else {
        const uint32_t lg = c ? 31u - (uint32_t)__clz(c) : 0u;   // floor(log2 c)
        keys[i] = ((uint64_t)(31u - lg) << 32) | (uint64_t)i;
    }
    vals[i] = (uint32_t)i;
}

// Fold the kXcd per-XCD copies of an atomic array into copy 0.
__global__ void k_sum_copies(double *__restrict__ base, int64_t len) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        double v = base[i];
#pragma unroll
        for (int x = 1; x < kXcd; ++x) v += base[x * len + i];
        base[i] = v;
    }
}

// Node adjoints summed along each leaf's ancestor path (the leaf included).
// For a node of mass Mn, centre of mass c and adjoint numbers a9 (dL/dM,
// dL/dcom, and dL/dQ up to a multiple of the identity with the zz component
// 0 and the off-diagonals stored doubled), a particle of mass m at x,
// y = x - c, receives
//   dL/dx += m (a/Mn + K y),   dL/dm += a0 + a.y/Mn + y'K y/2,
// with K = 6 Gq - 2 tr(Gq) I and Gq the symmetric dL/dQ.  Writing y = u + e
// with u = x - r (r the leaf's cube centre) and e = r - c, the sum over the
// path is one quadratic in u:
//   dL/dx += m (V + KK u),     dL/dm += S0 + V.u + u'KK u/2,
//   V = sum(a/Mn + K e), KK = sum K, S0 = sum(a0 + a.e/Mn + e'K e/2).
// poly holds per leaf and set: V (3), KK (xx yy zz xy xz yz), S0.
constexpr int kPoly = 10;

template <typename T>
__global__ __launch_bounds__(256) void k_leaf_poly(
    int64_t nn, const int32_t *__restrict__ nnchild, const int32_t *__restrict__ nparent,
    const double *__restrict__ clo, const double *__restrict__ chi,
    const double *__restrict__ M0, const double *__restrict__ com0,
    const double *__restrict__ M1, const double *__restrict__ com1,
    const double *__restrict__ nadj0, const double *__restrict__ nadj1, int sets,
    double *__restrict__ poly) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn || nnchild[k] != 0) return;
    double r[3];
    for (int d = 0; d < 3; ++d) r[d] = 0.5 * (clo[3 * k + d] + chi[3 * k + d]);
    for (int set = 0; set < sets; ++set) {
        const double *Ms = set ? M1 : M0;
        const double *cs = set ? com1 : com0;
        const double *ad = set ? nadj1 : nadj0;
        double V[3] = {0.0, 0.0, 0.0}, KK[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, S0 = 0.0;
        for (int64_t nd = k; nd >= 0; nd = nparent[nd]) {
            const double Mn = Ms[nd];
            if (!(Mn > 0.0)) continue;
            double a9[9];
            // set 0 (group walk) node-major, set 1 (sink walk) component-major
            for (int c = 0; c < 9; ++c) a9[c] = set ? ad[c * nn + nd] : ad[9 * nd + c];
            const double e0 = r[0] - cs[3 * nd], e1 = r[1] - cs[3 * nd + 1], e2 = r[2] - cs[3 * nd + 2];
            const double gxx = a9[4], gyy = a9[5], gxy = 0.5 * a9[6], gxz = 0.5 * a9[7],
                         gyz = 0.5 * a9[8];
            const double tr2 = 2.0 * (gxx + gyy);
            // K = 6 Gq - 2 tr I (Gq zz = 0)
            const double kxx = 6.0 * gxx - tr2, kyy = 6.0 * gyy - tr2, kzz = -tr2;
            const double kxy = 6.0 * gxy, kxz = 6.0 * gxz, kyz = 6.0 * gyz;
            const double Ke0 = kxx * e0 + kxy * e1 + kxz * e2;
            const double Ke1 = kxy * e0 + kyy * e1 + kyz * e2;
            const double Ke2 = kxz * e0 + kyz * e1 + kzz * e2;
            const double inv = 1.0 / Mn;
            V[0] += a9[1] * inv + Ke0;
            V[1] += a9[2] * inv + Ke1;
            V[2] += a9[3] * inv + Ke2;
            KK[0] += kxx;
            KK[1] += kyy;
            KK[2] += kzz;
            KK[3] += kxy;
            KK[4] += kxz;
            KK[5] += kyz;
            S0 += a9[0] + (a9[1] * e0 + a9[2] * e1 + a9[3] * e2) * inv +
                  0.5 * (e0 * Ke0 + e1 * Ke1 + e2 * Ke2);
        }
        double *q = poly + ((int64_t)set * nn + k) * kPoly;
        for (int d = 0; d < 3; ++d) q[d] = V[d];
        for (int d = 0; d < 6; ++d) q[3 + d] = KK[d];
        q[9] = S0;
    }
}

// Every part of each particle's adjoint, added and written in input order:
// target part, source part (all per-XCD copies), the leaf polynomials of set
// 0 (all particles) and set 1 (gas only), and the sink-sink part.
template <typename T>
__global__ void k_pushdown(int64_t n, int64_t n_gas, int64_t nn, const T *__restrict__ xs,
                           const T *__restrict__ ys, const T *__restrict__ zs,
                           const T *__restrict__ ms, const int32_t *__restrict__ order,
                           const int32_t *__restrict__ pleaf, const double *__restrict__ clo,
                           const double *__restrict__ chi, const double *__restrict__ poly,
                           int sets, const double *__restrict__ tgt, const double *__restrict__ scat,
                           const int32_t *__restrict__ sink_pos, int64_t n_sink,
                           const double *__restrict__ ssb, double G, T *__restrict__ g_pos,
                           T *__restrict__ g_mass, T *__restrict__ g_soft) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double m = (double)ms[s];
    const int64_t o = order[s];
    const bool gas = o < n_gas;
    double g[5];
    for (int d = 0; d < 5; ++d) {
        double v = tgt[5 * s + d];
#pragma unroll
        for (int x = 0; x < kXcd; ++x) v += scat[(int64_t)x * 5 * n + d * n + s];
        g[d] = v;
    }
    const int64_t lf = pleaf[s];
    const double u0 = (double)xs[s] - 0.5 * (clo[3 * lf] + chi[3 * lf]);
    const double u1 = (double)ys[s] - 0.5 * (clo[3 * lf + 1] + chi[3 * lf + 1]);
    const double u2 = (double)zs[s] - 0.5 * (clo[3 * lf + 2] + chi[3 * lf + 2]);
    for (int set = 0; set < 2; ++set) {
        if (set >= sets || (set == 1 && !gas)) break;
        const double *q = poly + ((int64_t)set * nn + lf) * kPoly;
        const double Ku0 = q[3] * u0 + q[6] * u1 + q[7] * u2;
        const double Ku1 = q[6] * u0 + q[4] * u1 + q[8] * u2;
        const double Ku2 = q[7] * u0 + q[8] * u1 + q[5] * u2;
        g[0] += m * (q[0] + Ku0);
        g[1] += m * (q[1] + Ku1);
        g[2] += m * (q[2] + Ku2);
        g[3] += q[9] + q[0] * u0 + q[1] * u1 + q[2] * u2 + 0.5 * (u0 * Ku0 + u1 * Ku1 + u2 * Ku2);
    }
    if (!gas && ssb) {
        int64_t lo = 0, hi = n_sink;   // rank of s among the sorted sink positions
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (sink_pos[mid] < s) lo = mid + 1; else hi = mid;
        }
        for (int d = 0; d < 5; ++d) g[d] += ssb[5 * lo + d];
    }
    if (g_pos) {
        g_pos[3 * o] = (T)(G * g[0]);
        g_pos[3 * o + 1] = (T)(G * g[1]);
        g_pos[3 * o + 2] = (T)(G * g[2]);
    }
    if (g_mass) g_mass[o] = (T)(G * g[3]);
    if (g_soft) g_soft[o] = (T)(G * g[4]);
}

template <typename T>
static WalkArgsB<T> make_args_b(sf_grav_tree_s *t, const EvalOpts &o, int set, const void *g_acc,
                                const void *g_pot, double *tgt, double *scat, double *nadj,
                                int32_t *ctr) {
    WalkArgsB<T> a{};
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
    a.g_acc = (const T *)g_acc;
    a.g_pot = (const T *)g_pot;
    a.tgt = tgt;
    a.scat = scat;
    a.nadj = nadj;
    a.scat_stride = 5 * t->n;
    a.nadj_stride = 9 * t->n_nodes;
    a.task_ctr = ctr;
    a.err = ctr + kCtrErr;
    return a;
}

// The sink walk goes on the side stream first (after the sink-sink part),
// the group walk on the caller's stream; each has its own task counter and
// stack area.
template <typename T, int FORM, int ORDER>
static void launch_walks_b(sf_grav_tree_s *t, const EvalOpts &o, const void *g_acc,
                           const void *g_pot, double *tgt, double *scat, double *nadj0,
                           double *nadj1, int32_t *ctr, uint32_t *gstack, uint32_t *sstack,
                           const uint32_t *gperm, hipStream_t side) {
    const unsigned grid = (unsigned)walk_grid();
    if (t->n_sink > 0) {
        WalkArgsB<T> as = make_args_b<T>(t, o, 1, g_acc, g_pot, tgt, scat, nadj1, ctr + kCtrSinks);
        as.err = ctr + kCtrErr;
        as.gstack = sstack;
        const unsigned gs = (unsigned)std::min<int64_t>(t->n_sink, grid);
        phase_begin(t, 9, side);
        hipLaunchKernelGGL((k_walk_sinks_b<T, FORM, ORDER>), dim3(gs), dim3(64), 0, side, as);
        phase_end(t, 9, side);
    }
    WalkArgsB<T> ag = make_args_b<T>(t, o, 0, g_acc, g_pot, tgt, scat, nadj0, ctr);
    ag.gstack = gstack;
    ag.gperm = gperm;
    phase_begin(t, 8);
    hipLaunchKernelGGL((k_walk_groups_b<T, FORM, ORDER>), dim3(grid), dim3(64), 0, t->stream, ag);
    phase_end(t, 8);
}

template <typename T>
static sf_status tree_backward_t(sf_grav_tree_s *t, const EvalOpts &o, const void *g_acc,
                                 const void *g_pot, void *g_pos, void *g_mass, void *g_soft,
                                 DevArena &ar) {
    hipStream_t s = t->stream;
    const int64_t n = t->n, nn = t->n_nodes;
    int32_t *ctr;
    uint32_t *gstack;
    double *tgt, *scat, *nadj0, *nadj1 = nullptr, *ssb = nullptr;
    SF_ALLOC_TMP(ar, ctr, kCtrWords);
    SF_ALLOC_TMP(ar, gstack, (int64_t)walk_grid() * kStack);
    SF_ALLOC_TMP(ar, tgt, 5 * n);
    SF_ALLOC_TMP(ar, scat, kXcd * 5 * n);
    SF_ALLOC_TMP(ar, nadj0, kXcd * 9 * nn);
    if (t->n_sink > 0) SF_ALLOC_TMP(ar, nadj1, kXcd * 9 * nn);   // the sink walk's node adjoints
    double *poly;
    SF_ALLOC_TMP(ar, poly, 2 * kPoly * nn);
    FillRanges zero;   // one launch; set 1 node adjoints exist only with sinks
    zero.add(ctr, kCtrWords);
    zero.add(tgt, 10 * n);
    zero.add(scat, kXcd * 10 * n);
    zero.add(nadj0, kXcd * 18 * nn);
    if (t->n_sink > 0) zero.add(nadj1, kXcd * 18 * nn);
    fill_ranges_u32(zero, 0u, s);
    // If a forward walk on this handle recorded each group's cost, start the
    // costly groups first: with few groups per resident wave the last costly
    // group to start sets the end of the walk.
    const uint32_t *gperm = nullptr;
    const int64_t gcap = t->groups_cap;
    if (t->have_cost && t->gcost && gcap >= 2 && gcap <= 0xffffffffll) {
        uint64_t *ckeys, *ctmp;
        uint32_t *cvals, *cvtmp, *cscr;
        SF_ALLOC_TMP(ar, ckeys, gcap);
        SF_ALLOC_TMP(ar, ctmp, gcap);
        SF_ALLOC_TMP(ar, cvals, gcap);
        SF_ALLOC_TMP(ar, cvtmp, gcap);
        const bool fine = gcap <= kFineOrderGroups * walk_grid();
        const int passes = fine ? 4 : 5;
        SF_ALLOC_TMP(ar, cscr, radix_scratch_words(gcap, passes));
        hipLaunchKernelGGL(k_cost_keys, dim3((unsigned)((gcap + 255) / 256)), dim3(256), 0, s,
                           (const uint32_t *)t->gcost, gcap, fine ? 1 : 0, ckeys, cvals);
        radix_sort_u64(ckeys, cvals, ctmp, cvtmp, gcap, passes, cscr, s);   // stable
        gperm = cvals;
    }
    uint32_t *sstack = nullptr;
    hipStream_t side = s;
    if (t->n_sink > 0) {
        double *srec;
        SF_ALLOC_TMP(ar, ssb, 5 * t->n_sink);
        SF_ALLOC_TMP(ar, srec, kSinkRecB * t->n_sink);
        SF_ALLOC_TMP(ar, sstack, std::min<int64_t>(t->n_sink, walk_grid()) * kStack);
        if (hipStream_t sd = side_stream(t->device)) side = sd;
        if (side_fork(t, side) != SF_OK) side = t->stream;   // nothing queued there: run serially
        phase_begin(t, 7, side);
        sink_sink_backward<T>(t, g_acc, g_pot, ssb, srec, side);
        phase_end(t, 7, side);
    }
#define SF_WB(F, O)                                                                                \
    launch_walks_b<T, F, O>(t, o, g_acc, g_pot, tgt, scat, nadj0, nadj1, ctr, gstack, sstack, \
                            gperm, side)
    if (o.order == 0) {
        if (o.form == SF_FP32C) SF_WB(SF_FP32C, 0);
        else if (o.form == SF_FP32) SF_WB(SF_FP32, 0);
        else SF_WB(SF_FP64, 0);
    } else {
        if (o.form == SF_FP32C) SF_WB(SF_FP32C, 2);
        else if (o.form == SF_FP32) SF_WB(SF_FP32, 2);
        else SF_WB(SF_FP64, 2);
    }
#undef SF_WB
    if (t->n_sink > 0) {
        sf_status st = side_join(t, side);
        if (st != SF_OK) return st;
    }
    phase_begin(t, 10);
    const unsigned rb = (unsigned)std::min<int64_t>(8192, (9 * nn + 255) / 256);
    const int sets = t->n_sink > 0 ? 2 : 1;   // set 1 adjoints come from the sink walk only
    hipLaunchKernelGGL(k_sum_copies, dim3(rb), dim3(256), 0, s, nadj0, (int64_t)9 * nn);
    if (t->n_sink > 0)
        hipLaunchKernelGGL(k_sum_copies, dim3(rb), dim3(256), 0, s, nadj1, (int64_t)9 * nn);
    hipLaunchKernelGGL(k_leaf_poly<T>, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, nn,
                       t->nnchild, t->nparent, t->clo, t->chi, t->M[0], t->com[0], t->M[1],
                       t->com[1], nadj0, nadj1, sets, poly);
    hipLaunchKernelGGL(k_pushdown<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       t->n_gas, nn, (const T *)t->xs, (const T *)t->ys, (const T *)t->zs,
                       (const T *)t->ms, t->order, t->pleaf, t->clo, t->chi, poly, sets, tgt, scat,
                       t->sink_pos, t->n_sink, ssb, o.G, (T *)g_pos, (T *)g_mass, (T *)g_soft);
    phase_end(t, 10);
    SF_HIP(hipGetLastError());
    int32_t herr = 0;
    SF_HIP(hipMemcpyAsync(&herr, ctr + kCtrErr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SF_HIP(hipStreamSynchronize(s));
    if (herr)
        return sf_fail(SF_E_INTERNAL, "tree walk stopped by a capacity guard (code %d)", herr);
    return SF_OK;
}

sf_status tree_backward(sf_grav_tree_s *t, const EvalOpts &o, const void *g_acc,
                        const void *g_pot, void *g_pos, void *g_mass, void *g_soft,
                        DevArena &ar) {
    if (t->dt == SF_F32)
        return tree_backward_t<float>(t, o, g_acc, g_pot, g_pos, g_mass, g_soft, ar);
    return tree_backward_t<double>(t, o, g_acc, g_pot, g_pos, g_mass, g_soft, ar);
}

}  // namespace sf
