/*
 * oracle/direct.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow FP64 O(N^2) direct sum of kernel-softened Newtonian gravity,
 * with its exact vector-Jacobian product and a pair-local loss for central
 * finite differences.  Only the tests, the smoke check and the CPU baseline
 * leg of the benchmark call it; the GPU library never links it and shares no
 * code with it.
 *
 * What it computes (paper Sec. 2.2 "Gravity" and Sec. 2.2.1 "Softening"):
 *   g = -grad(Phi) and Phi at every particle, summing every other particle
 *   j != i.  Pairs closer than the larger of the two softening radii,
 *   r < max(S_i, S_j), use a softened force law; beyond it the law is exactly
 *   Newtonian.  The softened law is the one implied by the M4 cubic spline
 *   (the kernel of the Sec. 2.1 footnote) with compact support h = S:
 *       W(u) = 8/(pi h^3) * { 1 - 6u^2 + 6u^3   (u < 1/2)
 *                             2 (1-u)^3         (1/2 <= u < 1)
 *                             0                 (u >= 1) },   u = r/h.
 *   Taking the larger softening for both directions of every pair (the rule
 *   the paper gives for sink-gas pairs, applied here to all pairs) keeps every
 *   interaction antisymmetric.
 *
 *   a_i   =  G sum_j m_j F(r_ij, h_ij) (x_j - x_i)
 *   phi_i = -G sum_j m_j P(r_ij, h_ij)
 *   F(r,h) = q(u)/r^3 with q the kernel mass enclosed within u, and P the
 *   matching potential, P(0,h) = 2.8/h (the Plummer-equivalent radius h/2.8 of
 *   Sec. 2.3.1).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (see oracle/build.py).
 * OpenMP splits only over targets; each target sums its sources in ascending
 * index order, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

/* ---- the softened kernel and its derivatives (closed forms) ---------------
 * All take r >= 0 and h > 0.  u = r/h.
 *   F      : force factor, a = G m F d
 *   P      : potential factor, phi = -G m P
 *   FrOverR: (dF/dr)/r, written in polynomial form so r -> 0 stays finite
 *   dFdh   : dF/dh = -32 w(u)/h^4, w the bracket of W above
 *   dPdh   : dP/dh = -(psi + u psi')/h^2 with psi = h P
 */
static void kern(double r, double h, double *F, double *P, double *FrOverR,
                 double *dFdh, double *dPdh)
{
    double u = r / h;
    double h2 = h * h, h3 = h2 * h;
    if (u >= 1.0) {
        double ir = 1.0 / r;
        *F = ir * ir * ir;
        *P = ir;
        *FrOverR = -3.0 * ir * ir * ir * ir * ir;
        *dFdh = 0.0;
        *dPdh = 0.0;
        return;
    }
    double u2 = u * u, u3 = u2 * u, u4 = u3 * u, u5 = u4 * u;
    if (u < 0.5) {
        *F = (32.0 / 3.0 - 192.0 / 5.0 * u2 + 32.0 * u3) / h3;
        *P = (14.0 / 5.0 - 16.0 / 3.0 * u2 + 48.0 / 5.0 * u4 - 32.0 / 5.0 * u5) / h;
        *FrOverR = (-384.0 / 5.0 + 96.0 * u) / (h3 * h2);
        *dFdh = -32.0 * (1.0 - 6.0 * u2 + 6.0 * u3) / (h2 * h2);
        *dPdh = -(14.0 / 5.0 - 16.0 * u2 + 48.0 * u4 - 192.0 / 5.0 * u5) / h2;
    } else {
        double om = 1.0 - u;
        *F = (64.0 / 3.0 - 48.0 * u + 192.0 / 5.0 * u2 - 32.0 / 3.0 * u3
              - 1.0 / (15.0 * u3)) / h3;
        *P = (16.0 / 5.0 - 1.0 / (15.0 * u) - 32.0 / 3.0 * u2 + 16.0 * u3
              - 48.0 / 5.0 * u4 + 32.0 / 15.0 * u5) / h;
        *FrOverR = (-48.0 / u + 384.0 / 5.0 - 32.0 * u + 1.0 / (5.0 * u5)) / (h3 * h2);
        *dFdh = -32.0 * (2.0 * om * om * om) / (h2 * h2);
        /* psi + u psi' = 16/5 - 32u^2 + 64u^3 - 48u^4 + 64/5 u^5, which vanishes
           at u = 1; written as (1-u)^4 (16 - 64/5 (1-u)) so it keeps its
           relative accuracy at the edge of the support. */
        double om2 = om * om;
        *dPdh = -(om2 * om2 * (16.0 - 64.0 / 5.0 * om)) / h2;
    }
}

/* Vectorised access to the kernel for the tests. */
void or_kernel(int64_t n, const double *r, const double *h, double *F, double *P,
               double *FrOverR, double *dFdh, double *dPdh)
{
    for (int64_t k = 0; k < n; ++k)
        kern(r[k], h[k], &F[k], &P[k], &FrOverR[k], &dFdh[k], &dPdh[k]);
}

/* Accelerations and potentials at targets tidx[0..nt) (or all if tidx NULL),
 * summing every source j != target.  x is n x 3 row-major. */
void or_direct(int64_t n, const double *x, const double *m, const double *h,
               double G, int64_t nt, const int64_t *tidx, double *acc, double *pot)
{
    int64_t count = tidx ? nt : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < count; ++t) {
        int64_t i = tidx ? tidx[t] : t;
        double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2], hi = h[i];
        double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[3 * j] - xi, dy = x[3 * j + 1] - yi, dz = x[3 * j + 2] - zi;
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double hij = hi > h[j] ? hi : h[j];
            double F, P, a, b, c;
            kern(r, hij, &F, &P, &a, &b, &c);
            double mF = m[j] * F;
            ax += mF * dx;
            ay += mF * dy;
            az += mF * dz;
            ph -= m[j] * P;
        }
        acc[3 * t] = G * ax;
        acc[3 * t + 1] = G * ay;
        acc[3 * t + 2] = G * az;
        pot[t] = G * ph;
    }
}

/* Tidal tensor T = -grad grad Phi = d a / d x (at the target) and jerk
 * j = d a / dt at targets tidx[0..nt) (or all if tidx NULL), from the same
 * softened kernel (Sec. 2.2: T and j are summed with spatial derivatives of
 * the kernel used for g).  With d = x_j - x_i, w = v_j - v_i:
 *     T_i = -G sum_j m_j [F I + (F'/r) d d^T]
 *     j_i =  G sum_j m_j [F w + (F'/r) (d . w) d]
 * T is written as xx yy zz xy xz yz (6 per target); v may be NULL (then j
 * is not computed). */
void or_direct_tidal(int64_t n, const double *x, const double *m, const double *h,
                     const double *v, double G, int64_t nt, const int64_t *tidx,
                     double *T, double *J)
{
    int64_t count = tidx ? nt : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < count; ++t) {
        int64_t i = tidx ? tidx[t] : t;
        double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2], hi = h[i];
        double txx = 0.0, tyy = 0.0, tzz = 0.0, txy = 0.0, txz = 0.0, tyz = 0.0;
        double jx = 0.0, jy = 0.0, jz = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[3 * j] - xi, dy = x[3 * j + 1] - yi, dz = x[3 * j + 2] - zi;
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double hij = hi > h[j] ? hi : h[j];
            double F, P, FrR, b, c;
            kern(r, hij, &F, &P, &FrR, &b, &c);
            double mF = m[j] * F, mR = m[j] * FrR;
            txx -= mF + mR * dx * dx;
            tyy -= mF + mR * dy * dy;
            tzz -= mF + mR * dz * dz;
            txy -= mR * dx * dy;
            txz -= mR * dx * dz;
            tyz -= mR * dy * dz;
            if (v) {
                double wx = v[3 * j] - v[3 * i], wy = v[3 * j + 1] - v[3 * i + 1];
                double wz = v[3 * j + 2] - v[3 * i + 2];
                double dw = dx * wx + dy * wy + dz * wz;
                jx += mF * wx + mR * dw * dx;
                jy += mF * wy + mR * dw * dy;
                jz += mF * wz + mR * dw * dz;
            }
        }
        double *Tt = T + 6 * t;
        Tt[0] = G * txx; Tt[1] = G * tyy; Tt[2] = G * tzz;
        Tt[3] = G * txy; Tt[4] = G * txz; Tt[5] = G * tyz;
        if (v) {
            J[3 * t] = G * jx;
            J[3 * t + 1] = G * jy;
            J[3 * t + 2] = G * jz;
        }
    }
}

/* Exact gradient of L = sum_i (ga_i . a_i + gp_i phi_i) with respect to every
 * position, mass and softening radius (gather form over k).  The softening
 * derivative of a pair goes to the particle whose radius is the larger one;
 * equal radii split it half and half. */
void or_direct_vjp(int64_t n, const double *x, const double *m, const double *h,
                   double G, const double *ga, const double *gp,
                   double *gx, double *gm, double *gh)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n; ++k) {
        double xk = x[3 * k], yk = x[3 * k + 1], zk = x[3 * k + 2], hk = h[k];
        double sx = 0.0, sy = 0.0, sz = 0.0, sm = 0.0, sh = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (i == k) continue;
            /* d points from i to k */
            double dx = xk - x[3 * i], dy = yk - x[3 * i + 1], dz = zk - x[3 * i + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double hik = hk > h[i] ? hk : h[i];
            double F, P, FrR, dFh, dPh;
            kern(r, hik, &F, &P, &FrR, &dFh, &dPh);
            double wx = m[k] * ga[3 * i] - m[i] * ga[3 * k];
            double wy = m[k] * ga[3 * i + 1] - m[i] * ga[3 * k + 1];
            double wz = m[k] * ga[3 * i + 2] - m[i] * ga[3 * k + 2];
            double wd = wx * dx + wy * dy + wz * dz;
            double c = (m[k] * gp[i] + m[i] * gp[k]) * F;
            sx += wx * F + wd * FrR * dx + c * dx;
            sy += wy * F + wd * FrR * dy + c * dy;
            sz += wz * F + wd * FrR * dz + c * dz;
            /* mass: k as the source seen by target i, d_ik = x_k - x_i */
            double gid = ga[3 * i] * dx + ga[3 * i + 1] * dy + ga[3 * i + 2] * dz;
            sm += gid * F - gp[i] * P;
            /* softening: both ordered pairs (i<-k) and (k<-i) use h_ik */
            double share = (hk > h[i]) ? 1.0 : (hk == h[i] ? 0.5 : 0.0);
            if (share > 0.0) {
                double gkd = -(ga[3 * k] * dx + ga[3 * k + 1] * dy + ga[3 * k + 2] * dz);
                double t_ik = m[k] * (gid * dFh - gp[i] * dPh);   /* target i, source k */
                double t_ki = m[i] * (gkd * dFh - gp[k] * dPh);   /* target k, source i */
                sh += share * (t_ik + t_ki);
            }
        }
        gx[3 * k] = G * sx;
        gx[3 * k + 1] = G * sy;
        gx[3 * k + 2] = G * sz;
        gm[k] = G * sm;
        gh[k] = G * sh;
    }
}

/* The same gradients when only the particles act[0..nact) carry nonzero
 * cotangents: every term above is a multiple of a cotangent of i or of k, so
 * a particle k outside act receives terms only from the i in act, and the
 * terms skipped are exact zeros (checks at full size, O(nact * n)).  flag[k]
 * is nonzero exactly for the k in act. */
void or_direct_vjp_sparse(int64_t n, const double *x, const double *m, const double *h,
                          double G, const double *ga, const double *gp, int64_t nact,
                          const int64_t *act, const unsigned char *flag,
                          double *gx, double *gm, double *gh)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < n; ++k) {
        double xk = x[3 * k], yk = x[3 * k + 1], zk = x[3 * k + 2], hk = h[k];
        double sx = 0.0, sy = 0.0, sz = 0.0, sm = 0.0, sh = 0.0;
        const int64_t cnt = flag[k] ? n : nact;
        for (int64_t q = 0; q < cnt; ++q) {
            const int64_t i = flag[k] ? q : act[q];
            if (i == k) continue;
            double dx = xk - x[3 * i], dy = yk - x[3 * i + 1], dz = zk - x[3 * i + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double hik = hk > h[i] ? hk : h[i];
            double F, P, FrR, dFh, dPh;
            kern(r, hik, &F, &P, &FrR, &dFh, &dPh);
            double wx = m[k] * ga[3 * i] - m[i] * ga[3 * k];
            double wy = m[k] * ga[3 * i + 1] - m[i] * ga[3 * k + 1];
            double wz = m[k] * ga[3 * i + 2] - m[i] * ga[3 * k + 2];
            double wd = wx * dx + wy * dy + wz * dz;
            double c = (m[k] * gp[i] + m[i] * gp[k]) * F;
            sx += wx * F + wd * FrR * dx + c * dx;
            sy += wy * F + wd * FrR * dy + c * dy;
            sz += wz * F + wd * FrR * dz + c * dz;
            double gid = ga[3 * i] * dx + ga[3 * i + 1] * dy + ga[3 * i + 2] * dz;
            sm += gid * F - gp[i] * P;
            double share = (hk > h[i]) ? 1.0 : (hk == h[i] ? 0.5 : 0.0);
            if (share > 0.0) {
                double gkd = -(ga[3 * k] * dx + ga[3 * k + 1] * dy + ga[3 * k + 2] * dz);
                double t_ik = m[k] * (gid * dFh - gp[i] * dPh);
                double t_ki = m[i] * (gkd * dFh - gp[k] * dPh);
                sh += share * (t_ik + t_ki);
            }
        }
        gx[3 * k] = G * sx;
        gx[3 * k + 1] = G * sy;
        gx[3 * k + 2] = G * sz;
        gm[k] = G * sm;
        gh[k] = G * sh;
    }
}

/* The part of L that depends on particle k: every ordered pair with k as
 * target or source.  Perturbing x_k, m_k or h_k changes L by exactly the
 * change of this sum, so central differences of it need no O(N^2) cancellation.
 * xk3/mk/hk override particle k's values. */
double or_pair_loss(int64_t n, const double *x, const double *m, const double *h,
                    double G, const double *ga, const double *gp, int64_t k,
                    const double *xk3, double mk, double hk)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (i == k) continue;
        double dx = xk3[0] - x[3 * i], dy = xk3[1] - x[3 * i + 1], dz = xk3[2] - x[3 * i + 2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        double hik = hk > h[i] ? hk : h[i];
        double F, P, a, b, c;
        kern(r, hik, &F, &P, &a, &b, &c);
        /* target i, source k: d = x_k - x_i */
        s += mk * (F * (ga[3 * i] * dx + ga[3 * i + 1] * dy + ga[3 * i + 2] * dz) - gp[i] * P);
        /* target k, source i: d = x_i - x_k */
        s += m[i] * (-F * (ga[3 * k] * dx + ga[3 * k + 1] * dy + ga[3 * k + 2] * dz) - gp[k] * P);
    }
    return G * s;
}
