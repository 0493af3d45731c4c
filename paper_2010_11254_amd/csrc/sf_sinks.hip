// sf_sinks.hip -- sink dynamics of Sec. 2.3 on the GPU, in FP64 throughout
// (sink-sink sums of close binaries keep FP64).
//
// * The sinks-only pass (Sec. 2.3.2 evaluates a_s and j_s of all sinks in a
//   special sinks-only gravity pass): acceleration, potential, jerk and
//   tidal tensor of every sink from all other sinks, as an exact direct sum
//   with the softened kernel (h_ss' = max(h_s, h_s')), and the two-body
//   time scales of Sec. 2.3.1 (Eqs. tcross and tdyn): the minima over s' of
//   sqrt(r^2 + eps^2) / |v_ss'| and sqrt((r^2 + eps^2)^(3/2) / (G (m_s +
//   m_s'))), eps = h_s / 2.8, with the 2-body and tidal timesteps built from
//   them.  One wavefront per target sink, lanes stride the other sinks; sums
//   and minima are reduced across the wave in a fixed order.
// * One step of the modified 4th-order Hermite scheme (Sec. 2.3.2, Eqs.
//   predictor and corrector) for all sinks with a common step: pass at the
//   start, prediction, pass at the predicted state, correction of v and then
//   of x with the corrected v.
#include "sf_build.h"
#include "sf_ext.h"
#include "sf_math.h"

namespace sf {

namespace {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wmin(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

struct SinkOut {
    double *acc, *pot, *jerk, *tidal, *times;   // times: tc, tdyn, dt_2body, dt_tidal
    double eta;
};

template <bool JERK>
__global__ __launch_bounds__(64) void k_sinks_pass(const double *__restrict__ x,
                                                   const double *__restrict__ v,
                                                   const double *__restrict__ m,
                                                   const double *__restrict__ h, int64_t n,
                                                   double G, SinkOut out) {
    const int lane = threadIdx.x;
    for (int64_t s = blockIdx.x; s < n; s += gridDim.x) {
        const double tx = x[3 * s], ty = x[3 * s + 1], tz = x[3 * s + 2];
        const double th = h[s], ms = m[s];
        double tv[3] = {0.0, 0.0, 0.0};
        if (JERK) {
            tv[0] = v[3 * s];
            tv[1] = v[3 * s + 1];
            tv[2] = v[3 * s + 2];
        }
        const double eps = th / 2.8, eps2 = eps * eps;
        double b[kX] = {};
        double tc = INFINITY, td = INFINITY;
        for (int64_t q = lane; q < n; q += 64) {
            if (q == s) continue;
            const double dx = x[3 * q] - tx, dy = x[3 * q + 1] - ty, dz = x[3 * q + 2] - tz;
            double w[3] = {0.0, 0.0, 0.0};
            if (JERK) {
                w[0] = v[3 * q] - tv[0];
                w[1] = v[3 * q + 1] - tv[1];
                w[2] = v[3 * q + 2] - tv[2];
            }
            ext_pair<double, JERK>(dx, dy, dz, w[0], w[1], w[2], m[q], h[q], th, false, b);
            if (JERK) {
                const double re2 = dx * dx + dy * dy + dz * dz + eps2;
                const double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
                const double re = sqrt(re2);
                tc = fmin(tc, re / wn);   // infinite for equal velocities
                td = fmin(td, sqrt(re2 * re / (G * (ms + m[q]))));
            }
        }
        for (int c = 0; c < kX; ++c) b[c] = wsum(b[c]);
        if (JERK) {
            tc = wmin(tc);
            td = wmin(td);
        }
        if (lane != 0) continue;
        out.acc[3 * s] = G * b[0];
        out.acc[3 * s + 1] = G * b[1];
        out.acc[3 * s + 2] = G * b[2];
        if (out.pot) out.pot[s] = G * b[3];
        if (out.tidal)
            for (int c = 0; c < 6; ++c) out.tidal[6 * s + c] = G * b[4 + c];
        if (out.jerk)
            for (int c = 0; c < 3; ++c) out.jerk[3 * s + c] = G * b[10 + c];
        if (out.times) {
            double *t = out.times + 4 * s;
            t[0] = tc;
            t[1] = td;
            double fro2 = 0.0;
            for (int c = 0; c < 3; ++c) fro2 += (G * b[4 + c]) * (G * b[4 + c]);
            for (int c = 3; c < 6; ++c) fro2 += 2.0 * (G * b[4 + c]) * (G * b[4 + c]);
            const double se = sqrt(out.eta);
            t[2] = out.eta > 0.0 ? se / (1.0 / tc + 1.0 / td) : 0.0;
            t[3] = out.eta > 0.0 ? se * pow(fro2 / 6.0, -0.25) : 0.0;
        }
    }
}

__global__ void k_predict(int64_t n, double dt, const double *__restrict__ x,
                          const double *__restrict__ v, const double *__restrict__ a0,
                          const double *__restrict__ j0, double *__restrict__ xp,
                          double *__restrict__ vp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * n) return;
    const double dt2 = dt * dt;
    xp[i] = x[i] + dt * v[i] + 0.5 * dt2 * a0[i] + dt2 * dt / 6.0 * j0[i];
    vp[i] = v[i] + dt * a0[i] + 0.5 * dt2 * j0[i];
}

// v first, then x with the corrected v (the order of the two updates matters).
__global__ void k_correct(int64_t n, double dt, double *__restrict__ x, double *__restrict__ v,
                          const double *__restrict__ a0, const double *__restrict__ j0,
                          const double *__restrict__ a1, const double *__restrict__ j1) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * n) return;
    const double dt2 = dt * dt;
    const double v0 = v[i];
    const double v1 = v0 + 0.5 * dt * (a1[i] + a0[i]) + dt2 / 12.0 * (j0[i] - j1[i]);
    v[i] = v1;
    x[i] = x[i] + 0.5 * dt * (v1 + v0) + dt2 / 12.0 * (a0[i] - a1[i]);
}

void sinks_pass(const double *x, const double *v, const double *m, const double *h, int64_t n,
                double G, const SinkOut &out, hipStream_t s) {
    const unsigned blocks = (unsigned)std::min<int64_t>(n, 16384);
    if (v)
        hipLaunchKernelGGL(k_sinks_pass<true>, dim3(blocks), dim3(64), 0, s, x, v, m, h, n, G, out);
    else
        hipLaunchKernelGGL(k_sinks_pass<false>, dim3(blocks), dim3(64), 0, s, x, v, m, h, n, G,
                           out);
}

}  // namespace

}  // namespace sf

extern "C" sf_status sf_grav_sinks(const double *pos, const double *vel, const double *mass,
                                   const double *soft, int64_t n, double G, double eta,
                                   double *acc, double *pot, double *jerk, double *tidal,
                                   double *times, void *stream) {
    if (!pos || !mass || !soft || !acc) return sf_fail(SF_E_INVALID, "pos, mass, soft, acc must be non-NULL");
    if (n < 1) return sf_fail(SF_E_INVALID, "n must be >= 1");
    if ((jerk || times) && !vel) return sf_fail(SF_E_INVALID, "jerk and time scales need vel");
    if (!(G == G) || !(eta == eta)) return sf_fail(SF_E_INVALID, "G and eta must not be NaN");
    sf::SinkOut out{acc, pot, jerk, tidal, times, eta};
    sf::sinks_pass(pos, (jerk || times) ? vel : nullptr, mass, soft, n, G, out,
                   (hipStream_t)stream);
    SF_HIP(hipGetLastError());
    return SF_OK;
}

extern "C" sf_status sf_grav_sink_hermite(double *pos, double *vel, const double *mass,
                                          const double *soft, int64_t n, double G, double dt,
                                          void *stream) {
    if (!pos || !vel || !mass || !soft) return sf_fail(SF_E_INVALID, "NULL argument");
    if (n < 1) return sf_fail(SF_E_INVALID, "n must be >= 1");
    if (!(dt == dt) || !(G == G)) return sf_fail(SF_E_INVALID, "dt and G must not be NaN");
    sf::fail_alloc_arm();
    hipStream_t s = (hipStream_t)stream;
    sf::DevArena ar(s);
    double *a0, *j0, *a1, *j1, *xp, *vp;
    SF_ALLOC_TMP(ar, a0, 3 * n);
    SF_ALLOC_TMP(ar, j0, 3 * n);
    SF_ALLOC_TMP(ar, a1, 3 * n);
    SF_ALLOC_TMP(ar, j1, 3 * n);
    SF_ALLOC_TMP(ar, xp, 3 * n);
    SF_ALLOC_TMP(ar, vp, 3 * n);
    sf::SinkOut o0{a0, nullptr, j0, nullptr, nullptr, 0.0};
    sf::sinks_pass(pos, vel, mass, soft, n, G, o0, s);
    const unsigned nb = (unsigned)((3 * n + 255) / 256);
    hipLaunchKernelGGL(sf::k_predict, dim3(nb), dim3(256), 0, s, n, dt, pos, vel, a0, j0, xp, vp);
    sf::SinkOut o1{a1, nullptr, j1, nullptr, nullptr, 0.0};
    sf::sinks_pass(xp, vp, mass, soft, n, G, o1, s);
    hipLaunchKernelGGL(sf::k_correct, dim3(nb), dim3(256), 0, s, n, dt, pos, vel, a0, j0, a1, j1);
    SF_HIP(hipGetLastError());
    return SF_OK;
}
