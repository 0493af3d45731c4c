// sf_math.h -- pair arithmetic shared by the tree and direct kernels:
// reciprocal square roots, the softened kernel of the M4 cubic spline and its
// derivatives, arithmetic forms and accumulators (internal).
#pragma once
#include "sf_internal.h"

namespace sf {

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) {
    // hardware estimate + two Newton steps: y <- y + y/2 (1 - x y^2)
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }

// Larger and smaller of two positive numbers that are finite or +inf
// (softening lengths, their squares and reciprocals, reciprocal distances).
// For such floats the order of the bit patterns read as unsigned integers is
// the order of the values, so one integer max or min returns exactly what
// fmax or fmin returns, without the instructions that quiet NaN operands
// first.  Doubles keep fmax and fmin.
__device__ __forceinline__ float pos_max(float a, float b) {
    return __uint_as_float(max(__float_as_uint(a), __float_as_uint(b)));
}
__device__ __forceinline__ float pos_min(float a, float b) {
    return __uint_as_float(min(__float_as_uint(a), __float_as_uint(b)));
}
__device__ __forceinline__ double pos_max(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ double pos_min(double a, double b) { return fmin(a, b); }

// r from r^2 and ri = rsq(r^2), 0 at r^2 = 0 (where ri is +inf): in FP32,
// ri capped at the largest finite float, which leaves every finite ri as it
// is and turns 0 * inf into 0.
__device__ __forceinline__ float r_of(float r2, float ri) {
    return r2 * pos_min(ri, __FLT_MAX__);
}
__device__ __forceinline__ double r_of(double r2, double ri) { return r2 > 0.0 ? r2 * ri : 0.0; }

// Softened force and potential factors for r^2 < h^2 (M4 cubic spline with
// support h): F = q(u)/r^3, P = psi(u)/h, u = r/h; both branches evaluated,
// the inner one selected for u < 1/2.  Taken from quantities the pair
// evaluation already holds: ri = rsq(r2), h and its reciprocal hinv; the outer
// branch's 1/u is h ri (2 at u <= 1/2, and at r = 0 where ri is infinite), so
// no further reciprocal or square root is needed.
template <typename R>
__device__ __forceinline__ void soft_FP_ri(R r2, R ri, R h, R hinv, R &F, R &P) {
    const R r = r_of(r2, ri);
    const R u = r * hinv;
    const R u2 = u * u;
    const R hinv3 = hinv * hinv * hinv;
    const R Fi = R(32.0 / 3.0) + u2 * (R(-192.0 / 5.0) + R(32.0) * u);
    const R Pi = R(14.0 / 5.0) + u2 * (R(-16.0 / 3.0) + u2 * (R(48.0 / 5.0) + R(-32.0 / 5.0) * u));
    const R us = u > R(0.5) ? u : R(0.5);
    const R hr = h * ri;
    const R iu = hr < R(2) ? hr : R(2);
    const R Fo = R(64.0 / 3.0) + us * (R(-48.0) + us * (R(192.0 / 5.0) + us * R(-32.0 / 3.0))) -
                 R(1.0 / 15.0) * iu * iu * iu;
    const R Po = R(16.0 / 5.0) - R(1.0 / 15.0) * iu +
                 us * us * (R(-32.0 / 3.0) + us * (R(16.0) + us * (R(-48.0 / 5.0) + us * R(32.0 / 15.0))));
    const bool inner = u < R(0.5);
    F = (inner ? Fi : Fo) * hinv3;
    P = (inner ? Pi : Po) * hinv;
}

template <int FORM> struct FormT;
template <> struct FormT<SF_FP32C> { using R = float; static constexpr bool rel = true, comp = true; };
template <> struct FormT<SF_FP32> { using R = float; static constexpr bool rel = false, comp = false; };
template <> struct FormT<SF_FP64> { using R = double; static constexpr bool rel = false, comp = false; };

// Per-target accumulator: compensated FP32 (batch partial folded with
// two-sum), or plain.
template <int FORM> struct Acc {
    using R = typename FormT<FORM>::R;
    R v;
    __device__ __forceinline__ void zero() { v = R(0); }
    __device__ __forceinline__ void fold(R b) { v += b; }
    __device__ __forceinline__ double value() const { return (double)v; }
};
template <> struct Acc<SF_FP32C> {
    Comp c;
    __device__ __forceinline__ void zero() { c.zero(); }
    __device__ __forceinline__ void fold(float b) { c.add(b); }
    __device__ __forceinline__ double value() const { return c.value(); }
};

// Coordinate in the form's frame: relative to `cen` for FP32C.
template <int FORM, typename T>
__device__ __forceinline__ typename FormT<FORM>::R to_frame(T x, double cen) {
    using R = typename FormT<FORM>::R;
    if (FormT<FORM>::rel) return (R)((double)x - cen);
    return (R)x;
}
template <int FORM>
__device__ __forceinline__ typename FormT<FORM>::R dto_frame(double x, double cen) {
    using R = typename FormT<FORM>::R;
    if (FormT<FORM>::rel) return (R)(x - cen);
    return (R)x;
}

// Kernel factors and h-derivatives for r^2 < h^2 (M4 cubic spline, support h):
// F, P, (dF/dr)/r, dF/dh, dP/dh.
template <typename R>
__device__ __forceinline__ void dsoft(R r2, R h, R &F, R &P, R &FrR, R &dFh, R &dPh) {
    const R hinv = rcp(h);
    const R r = r2 > R(0) ? r2 * rsq(r2) : R(0);
    const R u = r * hinv;
    const R u2 = u * u;
    const R hinv2 = hinv * hinv;
    const R hinv3 = hinv2 * hinv;
    const R us = u > R(0.5) ? u : R(0.5);
    const R iu = rcp(us);
    const R om = R(1) - us;
    const R om2 = om * om;
    if (u < R(0.5)) {
        F = (R(32.0 / 3.0) + u2 * (R(-192.0 / 5.0) + R(32.0) * u)) * hinv3;
        P = (R(14.0 / 5.0) + u2 * (R(-16.0 / 3.0) + u2 * (R(48.0 / 5.0) + R(-32.0 / 5.0) * u))) * hinv;
        FrR = (R(-384.0 / 5.0) + R(96.0) * u) * hinv3 * hinv2;
        dFh = R(-32.0) * (R(1) - R(6) * u2 + R(6) * u2 * u) * hinv2 * hinv2;
        dPh = -(R(14.0 / 5.0) + u2 * (R(-16.0) + u2 * (R(48.0) + R(-192.0 / 5.0) * u))) * hinv2;
    } else {
        const R iu2 = iu * iu;
        F = (R(64.0 / 3.0) + us * (R(-48.0) + us * (R(192.0 / 5.0) + us * R(-32.0 / 3.0))) -
             R(1.0 / 15.0) * iu2 * iu) * hinv3;
        P = (R(16.0 / 5.0) - R(1.0 / 15.0) * iu +
             us * us * (R(-32.0 / 3.0) + us * (R(16.0) + us * (R(-48.0 / 5.0) + us * R(32.0 / 15.0))))) *
            hinv;
        FrR = (R(-48.0) * iu + R(384.0 / 5.0) - R(32.0) * us + R(0.2) * iu2 * iu2 * iu) * hinv3 * hinv2;
        dFh = R(-64.0) * om2 * om * hinv2 * hinv2;
        dPh = -(om2 * om2 * (R(16.0) - R(64.0 / 5.0) * om)) * hinv2;
    }
}

// The same five factors from quantities the pair evaluation already holds:
// ri = rsq(r^2), h and 1/h.  Both spline pieces are evaluated and one is
// selected (no divergent branch), and the outer piece's 1/u is h ri capped at
// 2 (its value at u = 1/2), so no further square root or reciprocal is taken.
template <typename R>
__device__ __forceinline__ void dsoft_ri(R r2, R ri, R h, R hinv, R &F, R &P, R &FrR, R &dFh,
                                         R &dPh) {
    const R r = r_of(r2, ri);
    const R u = r * hinv;
    const R u2 = u * u;
    const R hinv2 = hinv * hinv;
    const R hinv3 = hinv2 * hinv;
    const R us = u > R(0.5) ? u : R(0.5);
    const R iu = pos_min(h * ri, R(2));
    const R iu2 = iu * iu;
    const R om = R(1) - us;
    const R om2 = om * om;
    const bool inner = u < R(0.5);
    const R Fi = R(32.0 / 3.0) + u2 * (R(-192.0 / 5.0) + R(32.0) * u);
    const R Fo = R(64.0 / 3.0) + us * (R(-48.0) + us * (R(192.0 / 5.0) + us * R(-32.0 / 3.0))) -
                 R(1.0 / 15.0) * iu2 * iu;
    const R Pi = R(14.0 / 5.0) + u2 * (R(-16.0 / 3.0) + u2 * (R(48.0 / 5.0) + R(-32.0 / 5.0) * u));
    const R Po = R(16.0 / 5.0) - R(1.0 / 15.0) * iu +
                 us * us * (R(-32.0 / 3.0) + us * (R(16.0) + us * (R(-48.0 / 5.0) + us * R(32.0 / 15.0))));
    const R Ri = R(-384.0 / 5.0) + R(96.0) * u;
    const R Ro = R(-48.0) * iu + R(384.0 / 5.0) - R(32.0) * us + R(0.2) * iu2 * iu2 * iu;
    const R Dfi = R(-32.0) * (R(1) - R(6) * u2 + R(6) * u2 * u);
    const R Dfo = R(-64.0) * om2 * om;
    const R Dpi = -(R(14.0 / 5.0) + u2 * (R(-16.0) + u2 * (R(48.0) + R(-192.0 / 5.0) * u)));
    const R Dpo = -(om2 * om2 * (R(16.0) - R(64.0 / 5.0) * om));
    F = (inner ? Fi : Fo) * hinv3;
    P = (inner ? Pi : Po) * hinv;
    FrR = (inner ? Ri : Ro) * hinv3 * hinv2;
    dFh = (inner ? Dfi : Dfo) * hinv2 * hinv2;
    dPh = (inner ? Dpi : Dpo) * hinv2;
}

}  // namespace sf
