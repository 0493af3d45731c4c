// sf_ext.h -- pair and node terms of the tidal tensor and jerk beside the
// acceleration and potential (internal; used by the tree walk with tidal
// outputs and by the sinks-only pass).
#pragma once
#include "sf_math.h"

namespace sf {

constexpr int kX = 13;   // ax ay az phi  Txx Tyy Tzz Txy Txz Tyz  jx jy jz

// One source term (pair or node monopole); mF = m F, mR = m F'/r, mP = m P.
template <typename R, bool JERK>
__device__ __forceinline__ void ext_term(R dx, R dy, R dz, R wx, R wy, R wz, R mF, R mR, R mP,
                                         R (&b)[kX], bool force) {
    if (force) {
        b[0] += mF * dx;
        b[1] += mF * dy;
        b[2] += mF * dz;
        b[3] -= mP;
    }
    const R rx = mR * dx, ry = mR * dy;
    b[4] -= mF + rx * dx;
    b[5] -= mF + ry * dy;
    b[6] -= mF + mR * dz * dz;
    b[7] -= rx * dy;
    b[8] -= rx * dz;
    b[9] -= ry * dz;
    if (JERK) {
        const R dw = dx * wx + dy * wy + dz * wz;
        b[10] += mF * wx + mR * dw * dx;
        b[11] += mF * wy + mR * dw * dy;
        b[12] += mF * wz + mR * dw * dz;
    }
}

// Particle pair with softening test and self exclusion.  SOFT = false:
// the caller knows the pair is Newtonian (its source leaf lies at least the
// larger softening length from the target box) and not a self pair.
template <typename R, bool JERK, bool SOFT = true>
__device__ __forceinline__ void ext_pair(R dx, R dy, R dz, R wx, R wy, R wz, R m, R hj, R ti,
                                         bool self, R (&b)[kX]) {
    const R r2 = dx * dx + dy * dy + dz * dz;
    const R ri = rsq(r2);
    R F = ri * ri * ri, P = ri, FrR = R(-3) * F * ri * ri;
    if (SOFT) {
        const R hh = pos_max(hj, ti);
        if (r2 < hh * hh) {
            R dFh, dPh;
            dsoft_ri<R>(r2, ri, hh, rcp(hh), F, P, FrR, dFh, dPh);
        }
        if (self) F = P = FrR = R(0);
    }
    ext_term<R, JERK>(dx, dy, dz, wx, wy, wz, m * F, m * FrR, m * P, b, true);
}

}  // namespace sf
