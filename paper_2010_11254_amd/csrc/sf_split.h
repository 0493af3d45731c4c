// sf_split.h -- lane splitting for the group evaluators that keep one target
// per lane (tidal tensor and jerk, adaptive softening, radiation sums).
//
// A group of gc targets gets k = floor(64 / gc) copies of each target: lane
// t + gc*s (s < k) holds target t and takes the entries s, s + k, s + 2k, ...
// of every staged batch, so a batch of nb entries costs about nb / k steps
// instead of nb.  Lanes from k*gc on repeat copy 0 (their sums are dropped),
// which keeps the wave's lanes on the same instruction stream.  At the end
// of the task the k partial sums of a target are added on its lane t in the
// order copy 0, 1, ..., k-1, so results do not depend on scheduling.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sf {

struct Split {
    uint32_t gc, k, tl, sub;   // group size, copies per target, this lane's target and copy

    __device__ __forceinline__ void init(uint32_t gcount, uint32_t lane) {
        gc = gcount;
        k = 64u / gc;
        tl = lane % gc;
        sub = lane / gc;
        if (sub >= k) sub = 0u;
    }

    // f(j) for this lane's entries j of a batch of nb: nb / k steps that give
    // every copy an entry, then one step for the copies with one left over.
    template <class F>
    __device__ __forceinline__ void each(uint32_t nb, F &&f) const {
        const uint32_t mf = nb / k;
        for (uint32_t j = 0; j < mf; ++j) f(sub + j * k);
        if (sub + mf * k < nb) f(sub + mf * k);
    }

    // On lanes t < gc, v[c] becomes the sum of target t's k copies.  The
    // partials go through buf, COLS x 64 doubles of LDS that no lane uses at
    // this point; every lane of the wave calls this.
    template <int COLS, int NV>
    __device__ void reduce(double (&v)[NV], double *buf, uint32_t lane) const {
#pragma unroll
        for (int c0 = 0; c0 < NV; c0 += COLS) {
            constexpr int kc = COLS;
#pragma unroll
            for (int c = 0; c < kc; ++c)
                if (c0 + c < NV) buf[c * 64 + lane] = v[c0 + c];
            __syncthreads();
            if (lane < gc)
                for (uint32_t s = 1; s < k; ++s) {
#pragma unroll
                    for (int c = 0; c < kc; ++c)
                        if (c0 + c < NV) v[c0 + c] += buf[c * 64 + lane + s * gc];
                }
            __syncthreads();
        }
    }
};

}  // namespace sf
