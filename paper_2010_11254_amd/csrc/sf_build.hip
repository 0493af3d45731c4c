// sf_build.hip -- octree construction on gfx950 (paper Sec. 2.2: the domain is
// subdivided recursively into octants).
//
//   bounding box -> 63-bit Morton keys -> stable radix sort -> sorted SoA
//   -> topology (all levels at once from key prefixes) -> FP64 moments
//   (bottom-up, last-arriving child combines) -> target groups.
//
// Topology without a level loop: for a sorted position s let c(s) be the
// number of leading octal digits s shares with s-1.  Position s starts a cell
// at every level l > c(s).  The cell of s at level l holds more than leaf_cap
// particles iff some window of leaf_cap+1 consecutive positions around s
// shares the level-l prefix, so the leaf level of s is
//     lambda(s) = min(21, 1 + max_{t in [s-cap, s]} lcp(key[t], key[t+cap])),
// and s starts one node at each level in (c(s), lambda(s)].  Nodes are
// emitted in depth-first order (by first particle, then level), then a stable
// counting pass by level yields the breadth-first array; per-node fields come
// from binary searches.
#include "sf_build.h"
#include "sf_prims.h"

namespace sf {

// ---------------------------------------------------------------- A1 bbox

constexpr int kBoxBlocks = 1024;

template <typename T>
__global__ __launch_bounds__(256) void k_bbox_partial(const T *__restrict__ pos,
                                                      const T *__restrict__ mass,
                                                      const T *__restrict__ soft, int64_t n,
                                                      int validate, double *__restrict__ part,
                                                      Frame *frame) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double v = (double)pos[3 * i + d];
            lo[d] = fmin(lo[d], v);
            hi[d] = fmax(hi[d], v);
            if (validate && !isfinite(v)) bad = 1;
        }
        if (validate) {
            double m = (double)mass[i], h = (double)soft[i];
            if (!(m >= 0.0) || !isfinite(m) || !(h > 0.0) || !isfinite(h)) bad = 1;
        }
    }
    __shared__ double sh[6][256];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        sh[d][threadIdx.x] = lo[d];
        sh[3 + d][threadIdx.x] = hi[d];
    }
    if (validate && bad) atomicAdd(&frame->bad, 1);
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                sh[d][threadIdx.x] = fmin(sh[d][threadIdx.x], sh[d][threadIdx.x + w]);
                sh[3 + d][threadIdx.x] = fmax(sh[3 + d][threadIdx.x], sh[3 + d][threadIdx.x + w]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

// Root cube: lo = per-axis minimum; side = largest extent (1 if zero);
// scale = 2^21 / side (correctly rounded FP64 division).
__global__ __launch_bounds__(256) void k_bbox_final(const double *__restrict__ part, int nblocks,
                                                    Frame *frame) {
    __shared__ double sh[6][256];
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int d = 0; d < 3; ++d) {
            v[d] = fmin(v[d], part[b * 6 + d]);
            v[3 + d] = fmax(v[3 + d], part[b * 6 + 3 + d]);
        }
    for (int d = 0; d < 6; ++d) sh[d][threadIdx.x] = v[d];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int d = 0; d < 3; ++d) {
                sh[d][threadIdx.x] = fmin(sh[d][threadIdx.x], sh[d][threadIdx.x + w]);
                sh[3 + d][threadIdx.x] = fmax(sh[3 + d][threadIdx.x], sh[3 + d][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double side = 0.0;
    for (int d = 0; d < 3; ++d) {
        const double e = dsub(sh[3 + d][0], sh[d][0]);
        side = e > side ? e : side;
        frame->lo[d] = sh[d][0];
        frame->hi[d] = sh[3 + d][0];
    }
    if (side == 0.0) side = 1.0;
    frame->side = side;
    frame->scale = 2097152.0 / side;
}

// ---------------------------------------------------------------- A2 keys

// q_d = floor((x_d - lo_d) * scale) in FP64 (separate subtract and multiply),
// clamped to [0, 2^21 - 1]; x supplies the most significant bit of each
// 3-bit digit.  type_major sets bit 63 for sinks (gas first, then sinks).
template <typename T>
__global__ void k_keys(const T *__restrict__ pos, int64_t n, int64_t n_gas,
                       const Frame *__restrict__ frame, int type_major, uint64_t *__restrict__ keys,
                       uint32_t *__restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t q[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double v = dmul(dsub((double)pos[3 * i + d], frame->lo[d]), frame->scale);
        v = floor(v);
        v = v < 0.0 ? 0.0 : (v > 2097151.0 ? 2097151.0 : v);
        q[d] = (uint64_t)v;
    }
    uint64_t k = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
    if (type_major && i >= n_gas) k |= 1ull << 63;
    keys[i] = k;
    vals[i] = (uint32_t)i;
}

// ---------------------------------------------------------------- A4 permute

template <typename T>
__global__ void k_permute(const T *__restrict__ pos, const T *__restrict__ mass,
                          const T *__restrict__ soft, const uint32_t *__restrict__ order, int64_t n,
                          T *__restrict__ xs, T *__restrict__ ys, T *__restrict__ zs,
                          T *__restrict__ ms, T *__restrict__ hs) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t i = order[s];
    xs[s] = pos[3 * i];
    ys[s] = pos[3 * i + 1];
    zs[s] = pos[3 * i + 2];
    ms[s] = mass[i];
    hs[s] = soft[i];
}

__global__ void k_sink_flags(const int32_t *__restrict__ order, int64_t n, int64_t n_gas,
                             uint32_t *__restrict__ flag) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) flag[s] = order[s] >= n_gas ? 1u : 0u;
}

__global__ void k_sink_write(const uint32_t *__restrict__ flag, const uint32_t *__restrict__ idx,
                             int64_t n, int32_t *__restrict__ sink_pos) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n && flag[s]) sink_pos[idx[s]] = (int32_t)s;
}

static inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

template <typename T>
static sf_status sort_stage(const void *pos, const void *mass, const void *soft, int64_t n,
                            int64_t n_gas, bool type_major, bool validate, sf_grav_tree_s *t,
                            DevArena &ar) {
    hipStream_t s = t->stream;
    SF_ALLOC(ar, t->frame, 1);
    fill_u32((uint32_t *)t->frame, sizeof(Frame) / 4, 0u, s);
    double *part = nullptr;
    SF_ALLOC_TMP(ar, part, kBoxBlocks * 6);
    int bb = (int)std::min<int64_t>(kBoxBlocks, (n + 255) / 256);
    hipLaunchKernelGGL(k_bbox_partial<T>, dim3(bb), dim3(256), 0, s, (const T *)pos,
                       (const T *)mass, (const T *)soft, n, validate ? 1 : 0, part, t->frame);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(256), 0, s, part, bb, t->frame);

    uint64_t *ktmp = nullptr;
    uint32_t *vtmp = nullptr, *scr = nullptr;
    SF_ALLOC(ar, t->keys, n);
    SF_ALLOC(ar, t->order, n);
    SF_ALLOC_TMP(ar, ktmp, n);
    SF_ALLOC_TMP(ar, vtmp, n);
    SF_ALLOC_TMP(ar, scr, radix_scratch_words(n, 8));
    hipLaunchKernelGGL(k_keys<T>, dim3(nblk(n)), dim3(256), 0, s, (const T *)pos, n, n_gas,
                       t->frame, type_major ? 1 : 0, t->keys, (uint32_t *)t->order);
    radix_sort_u64(t->keys, (uint32_t *)t->order, ktmp, vtmp, n, 8, scr, s);

    T *xs, *ys, *zs, *ms, *hs;
    SF_ALLOC(ar, xs, n);
    SF_ALLOC(ar, ys, n);
    SF_ALLOC(ar, zs, n);
    SF_ALLOC(ar, ms, n);
    SF_ALLOC(ar, hs, n);
    t->xs = xs; t->ys = ys; t->zs = zs; t->ms = ms; t->hs = hs;
    hipLaunchKernelGGL(k_permute<T>, dim3(nblk(n)), dim3(256), 0, s, (const T *)pos,
                       (const T *)mass, (const T *)soft, (const uint32_t *)t->order, n, xs, ys, zs,
                       ms, hs);
    // sinks in sorted order
    const int64_t n_sink = n - n_gas;
    if (n_sink > 0) {
        SF_ALLOC(ar, t->sink_pos, n_sink);
        uint32_t *flag = (uint32_t *)vtmp, *idx = nullptr, *sscr = nullptr;
        SF_ALLOC_TMP(ar, idx, n);
        SF_ALLOC_TMP(ar, sscr, scan_scratch_words(n));
        hipLaunchKernelGGL(k_sink_flags, dim3(nblk(n)), dim3(256), 0, s, t->order, n, n_gas, flag);
        scan_u32(flag, idx, n, sscr, nullptr, s);
        hipLaunchKernelGGL(k_sink_write, dim3(nblk(n)), dim3(256), 0, s, flag, idx, n, t->sink_pos);
    }
    SF_HIP(hipGetLastError());
    return SF_OK;
}

sf_status build_sorted(const void *pos, const void *mass, const void *soft, int64_t n,
                       int64_t n_gas, sf_dtype dt, bool type_major, bool validate,
                       sf_grav_tree_s *t, DevArena &ar) {
    t->n = n;
    t->n_gas = n_gas;
    t->n_sink = n - n_gas;
    t->dt = dt;
    if (dt == SF_F32) return sort_stage<float>(pos, mass, soft, n, n_gas, type_major, validate, t, ar);
    return sort_stage<double>(pos, mass, soft, n, n_gas, type_major, validate, t, ar);
}

// ---------------------------------------------------------------- A5 topology

__global__ void k_topo_lcp(const uint64_t *__restrict__ keys, int64_t n, int cap,
                           uint8_t *__restrict__ lcp, uint8_t *__restrict__ win) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint64_t k = keys[s];
    lcp[s] = s > 0 ? (uint8_t)lcp_digits(keys[s - 1], k) : 0;
    if (s + cap < n) win[s] = (uint8_t)lcp_digits(k, keys[s + cap]);
}

// Leaf level lambda(s), node count of s, and the block's level histogram,
// written to column l of part (part[l * nb + block]).  The block's window
// bytes (positions base - cap .. base + 255, cap <= 64) are staged in LDS; the
// histogram takes one ballot per level per wave.
__global__ __launch_bounds__(256) void k_topo_count(const uint8_t *__restrict__ lcp,
                                                    const uint8_t *__restrict__ win, int64_t n,
                                                    int cap, uint8_t *__restrict__ lam,
                                                    uint32_t *__restrict__ nn,
                                                    uint32_t *__restrict__ part) {
    __shared__ uint8_t sw[256 + 64];
    __shared__ uint32_t sh[kLevels + 1];
    if (threadIdx.x <= kLevels) sh[threadIdx.x] = 0;
    const int64_t base = (int64_t)blockIdx.x * blockDim.x;
    for (int i = threadIdx.x; i < 256 + cap; i += 256) {
        const int64_t t = base - cap + i;
        sw[i] = (t >= 0 && t < n - cap) ? win[t] : 0;
    }
    __syncthreads();
    const int64_t s = base + threadIdx.x;
    const bool valid = s < n;
    int lo = 1, L = 0;
    if (valid) {
        // windows t in [max(s - cap, 0), min(s, n - 1 - cap)]: empty only when n <= cap
        const int64_t t0 = s - cap > 0 ? s - cap : 0;
        const int64_t t1 = s < n - 1 - cap ? s : n - 1 - cap;
        int mx = -1;
        for (int64_t t = t0; t <= t1; ++t) mx = max(mx, (int)sw[t - (base - cap)]);
        L = mx < 0 ? 0 : min(kLevels, mx + 1);
        lo = s == 0 ? 0 : (int)lcp[s] + 1;
        lam[s] = (uint8_t)L;
        nn[s] = (uint32_t)(L >= lo ? L - lo + 1 : 0);
    }
    for (int l = 0; l <= kLevels; ++l) {
        const uint64_t b = __ballot(l >= lo && l <= L);
        if ((threadIdx.x & 63) == 0 && b) atomicAdd(&sh[l], (uint32_t)__popcll(b));
    }
    __syncthreads();
    if (threadIdx.x <= kLevels) part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = sh[threadIdx.x];
}

// Block b writes the sum of part[b * nb .. b * nb + nb) to out[b] (the level
// histogram from the per-block columns; the leaf count from per-block counts).
__global__ __launch_bounds__(256) void k_topo_levsum(const uint32_t *__restrict__ part, int64_t nb,
                                                     uint32_t *__restrict__ out) {
    __shared__ uint32_t sw[4];
    const uint32_t *col = part + (int64_t)blockIdx.x * nb;
    uint32_t v = 0;
    for (int64_t i = threadIdx.x; i < nb; i += 256) v += col[i];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = sw[0] + sw[1] + sw[2] + sw[3];
}

// level_off[0..22] (exclusive prefix of the level histogram) and the 256-entry
// digit-offset table for the counting pass by level.
__global__ void k_topo_levoff(const uint32_t *__restrict__ levhist, uint32_t *__restrict__ level_off,
                              uint32_t *__restrict__ digit_off, uint32_t *__restrict__ max_level) {
    if (threadIdx.x != 0) return;
    uint32_t run = 0, lmax = 0;
    for (int l = 0; l <= kLevels; ++l) {
        level_off[l] = run;
        digit_off[l] = run;
        run += levhist[l];
        if (levhist[l]) lmax = (uint32_t)l;
    }
    *max_level = lmax;
    level_off[kLevels + 1] = run;
    for (int d = kLevels + 1; d < 256; ++d) digit_off[d] = run;
}

// Depth-first emission: packed node = (first << 8) | level.
__global__ void k_topo_emit(const uint8_t *__restrict__ lcp, const uint8_t *__restrict__ lam,
                            const uint32_t *__restrict__ dfs_off, int64_t n,
                            uint64_t *__restrict__ packed) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int lo = s == 0 ? 0 : (int)lcp[s] + 1;
    int L = lam[s];
    uint32_t o = dfs_off[s];
    for (int l = lo; l <= L; ++l) packed[o + (l - lo)] = ((uint64_t)s << 8) | (uint64_t)l;
}

// DFS position of every BFS node: node (s, l) was emitted at
// dfs_off[s] + l - lo(s), lo(s) = lcp[s] + 1 (0 for s = 0).
__global__ void k_topo_inv(const uint64_t *__restrict__ packed, int64_t n_nodes,
                           const uint8_t *__restrict__ lcp, const uint32_t *__restrict__ dfs_off,
                           uint32_t *__restrict__ inv) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_nodes) return;
    const uint64_t pk = packed[k];
    const int l = (int)(pk & 255);
    const int64_t s = (int64_t)(pk >> 8);
    const int lo = s == 0 ? 0 : (int)lcp[s] + 1;
    inv[dfs_off[s] + (l - lo)] = (uint32_t)k;
}

// Node fields from the BFS array.  The cell end comes from a galloping search
// of the keys; an inner node (s, l) has first child (s, l + 1), the next DFS
// entry of particle s, and its children are the consecutive level-(l + 1)
// nodes whose first particle lies before the end.  Each inner node writes its
// own child fields and its children's parent links.
__global__ void k_topo_fields(const uint64_t *__restrict__ packed, int64_t n_nodes,
                              const uint64_t *__restrict__ keys, int64_t n, int cap,
                              const uint32_t *__restrict__ level_off, const Frame *__restrict__ frame,
                              const uint8_t *__restrict__ lcp, const uint32_t *__restrict__ dfs_off,
                              const uint32_t *__restrict__ inv,
                              int32_t *__restrict__ nlevel, int32_t *__restrict__ nfirst,
                              int32_t *__restrict__ ncount, int32_t *__restrict__ nparent,
                              int32_t *__restrict__ nchild, int32_t *__restrict__ nnchild,
                              double *__restrict__ clo, double *__restrict__ chi,
                              uint32_t *__restrict__ leaf_part) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = k < n_nodes;
    const uint64_t pk = valid ? packed[k] : 0ull;
    const int l = (int)(pk & 255);
    const int64_t s = (int64_t)(pk >> 8);
    int64_t end = s;
    if (valid) {
        // end of the cell: first key beyond the largest key with this prefix;
        // galloping from s (most cells are small), then bisection
        const uint64_t kmax = keys[s] | ((l == 0) ? ~0ull >> 1 : ((1ull << (3 * (kLevels - l))) - 1));
        int64_t a = s + 1, step = 1;
        while (a < n && keys[a] <= kmax) {
            a = s + 1 + step;
            step <<= 1;
        }
        // keys[lo - 1] <= kmax and (hi == n or keys[hi] > kmax)
        int64_t lo = s + 1 + (step >> 2), hi = a < n ? a : n;
        while (lo < hi) {
            const int64_t m = (lo + hi) >> 1;
            if (keys[m] <= kmax) lo = m + 1; else hi = m;
        }
        end = lo;
    }
    const int64_t cnt = end - s;
    const bool leaf = cnt <= cap || l == kLevels;
    {   // the block's leaf count (summed over blocks by a later launch)
        __shared__ uint32_t sl[4];
        const uint32_t nleaf = (uint32_t)__popcll(__ballot(valid && leaf));
        if ((threadIdx.x & 63) == 0) sl[threadIdx.x >> 6] = nleaf;
        __syncthreads();
        if (threadIdx.x == 0) leaf_part[blockIdx.x] = sl[0] + sl[1] + sl[2] + sl[3];
    }
    if (!valid) return;
    nlevel[k] = l;
    nfirst[k] = (int32_t)s;
    ncount[k] = (int32_t)cnt;
    if (l == 0) nparent[k] = -1;
    if (!leaf) {
        const int lo = s == 0 ? 0 : (int)lcp[s] + 1;
        const int64_t di = (int64_t)dfs_off[s] + (l - lo) + 1;   // below n_nodes by construction
        const int64_t c0 = di < n_nodes ? (int64_t)inv[di] : n_nodes;
        const int64_t cend = level_off[l + 2];
        int64_t c = c0;
        while (c < cend && (int64_t)(packed[c] >> 8) < end) {
            nparent[c] = (int32_t)k;
            ++c;
        }
        nchild[k] = (int32_t)c0;
        nnchild[k] = (int32_t)(c - c0);
    } else {
        nchild[k] = -1;
        nnchild[k] = 0;
    }
    // cube: lo + ix * cell, lo + (ix + 1) * cell with cell = side * 2^-l
    const uint64_t pre = l == 0 ? 0ull : (keys[s] >> (3 * (kLevels - l)));
    const double cell = ldexp(frame->side, -l);
    const uint32_t ij[3] = {compact3(pre >> 2), compact3(pre >> 1), compact3(pre)};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        clo[3 * k + d] = dadd(frame->lo[d], dmul((double)ij[d], cell));
        chi[3 * k + d] = dadd(frame->lo[d], dmul((double)(ij[d] + 1), cell));
    }
}

sf_status build_topology(sf_grav_tree_s *t, DevArena &ar) {
    hipStream_t s = t->stream;
    const int64_t n = t->n;
    const int cap = t->leaf_cap;
    uint8_t *lcp, *win, *lam;
    uint32_t *nn, *dfs, *levhist, *misc, *scr, *pscr;
    SF_ALLOC_TMP(ar, lcp, n);
    SF_ALLOC_TMP(ar, win, n);
    SF_ALLOC_TMP(ar, lam, n);
    SF_ALLOC_TMP(ar, nn, n);
    SF_ALLOC_TMP(ar, dfs, n);
    // misc: [0..22] levhist, [24..47] level_off, [48..303] digit_off,
    //       [304] total nodes, [305] max level, [306] leaves
    SF_ALLOC_TMP(ar, misc, 320);
    levhist = misc;
    SF_HIP(hipMemsetAsync(misc, 0, 320 * sizeof(uint32_t), s));
    SF_ALLOC_TMP(ar, scr, scan_scratch_words(n));
    hipLaunchKernelGGL(k_topo_lcp, dim3(nblk(n)), dim3(256), 0, s, t->keys, n, cap, lcp, win);
    const int64_t nb = nblk(n);
    uint32_t *part;
    SF_ALLOC_TMP(ar, part, (kLevels + 1) * nb);
    hipLaunchKernelGGL(k_topo_count, dim3(nb), dim3(256), 0, s, lcp, win, n, cap, lam, nn, part);
    hipLaunchKernelGGL(k_topo_levsum, dim3(kLevels + 1), dim3(256), 0, s, part, nb, levhist);
    scan_u32(nn, dfs, n, scr, misc + 304, s);
    hipLaunchKernelGGL(k_topo_levoff, dim3(1), dim3(64), 0, s, levhist, misc + 24, misc + 48,
                       misc + 305);
    uint32_t hmisc[24 + 23];
    SF_HIP(hipMemcpyAsync(hmisc, misc + 24, 23 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    SF_HIP(hipStreamSynchronize(s));
    const int64_t nn_total = hmisc[kLevels + 1];
    for (int l = 0; l <= kLevels + 1; ++l) t->level_off[l] = hmisc[l];
    t->n_nodes = nn_total;
    uint64_t *pdfs, *pbfs;
    SF_ALLOC_TMP(ar, pdfs, nn_total);
    SF_ALLOC_TMP(ar, pbfs, nn_total);
    SF_ALLOC_TMP(ar, pscr, radix_pass_scratch_words(nn_total));
    hipLaunchKernelGGL(k_topo_emit, dim3(nblk(n)), dim3(256), 0, s, lcp, lam, dfs, n, pdfs);
    radix_pass_u64(pdfs, pbfs, nn_total, 0, misc + 48, pscr, s);
    SF_ALLOC(ar, t->info_dev, 8);
    SF_ALLOC(ar, t->nlevel, nn_total);
    SF_ALLOC(ar, t->nfirst, nn_total);
    SF_ALLOC(ar, t->ncount, nn_total);
    SF_ALLOC(ar, t->nparent, nn_total);
    SF_ALLOC(ar, t->nchild, nn_total);
    SF_ALLOC(ar, t->nnchild, nn_total);
    SF_ALLOC(ar, t->clo, 3 * nn_total);
    SF_ALLOC(ar, t->chi, 3 * nn_total);
    uint32_t *inv, *leaf_part;
    SF_ALLOC_TMP(ar, inv, nn_total);
    SF_ALLOC_TMP(ar, leaf_part, nblk(nn_total));
    hipLaunchKernelGGL(k_topo_inv, dim3(nblk(nn_total)), dim3(256), 0, s, pbfs, nn_total, lcp, dfs,
                       inv);
    hipLaunchKernelGGL(k_topo_fields, dim3(nblk(nn_total)), dim3(256), 0, s, pbfs, nn_total,
                       t->keys, n, cap, misc + 24, t->frame, lcp, dfs, inv, t->nlevel, t->nfirst,
                       t->ncount, t->nparent, t->nchild, t->nnchild, t->clo, t->chi, leaf_part);
    hipLaunchKernelGGL(k_topo_levsum, dim3(1), dim3(256), 0, s, leaf_part, (int64_t)nblk(nn_total),
                       misc + 306);
    SF_HIP(hipGetLastError());
    SF_HIP(hipMemcpyAsync(t->info_dev, misc + 305, 2 * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    return SF_OK;
}

// ---------------------------------------------------------------- A6 moments

// Raw moments of a node about its cube centre g, per set (0 all, 1 gas):
//   M, D = sum m (x - g), S = sum m (x - g)(x - g)^T (xx yy zz xy xz yz), hmax.
struct RawMom {
    double M, D[3], S[6], h;
};

__device__ __forceinline__ void raw_zero(RawMom &r) {
    r.M = 0.0;
    r.h = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) r.D[d] = 0.0;
#pragma unroll
    for (int d = 0; d < 6; ++d) r.S[d] = 0.0;
}

__device__ __forceinline__ void raw_add_point(RawMom &r, double m, double y0, double y1, double y2,
                                              double h) {
    r.M += m;
    r.D[0] += m * y0;
    r.D[1] += m * y1;
    r.D[2] += m * y2;
    r.S[0] += m * y0 * y0;
    r.S[1] += m * y1 * y1;
    r.S[2] += m * y2 * y2;
    r.S[3] += m * y0 * y1;
    r.S[4] += m * y0 * y2;
    r.S[5] += m * y1 * y2;
    r.h = fmax(r.h, h);
}

// raw layout per set: 11 doubles per node (M, D0..2, S0..5, h)
__device__ __forceinline__ void raw_store(double *raw, int64_t k, const RawMom &r) {
    double *p = raw + 11 * k;
    p[0] = r.M;
    for (int d = 0; d < 3; ++d) p[1 + d] = r.D[d];
    for (int d = 0; d < 6; ++d) p[4 + d] = r.S[d];
    p[10] = r.h;
}

__device__ __forceinline__ void raw_load(const double *raw, int64_t k, RawMom &r) {
    const double *p = raw + 11 * k;
    r.M = p[0];
    for (int d = 0; d < 3; ++d) r.D[d] = p[1 + d];
    for (int d = 0; d < 6; ++d) r.S[d] = p[4 + d];
    r.h = p[10];
}

// Shift child moments from its centre gc to the parent centre g and add.
__device__ __forceinline__ void raw_add_child(RawMom &p, const RawMom &c, const double dl[3]) {
    p.M += c.M;
    p.D[0] += c.D[0] + c.M * dl[0];
    p.D[1] += c.D[1] + c.M * dl[1];
    p.D[2] += c.D[2] + c.M * dl[2];
    p.S[0] += c.S[0] + 2.0 * c.D[0] * dl[0] + c.M * dl[0] * dl[0];
    p.S[1] += c.S[1] + 2.0 * c.D[1] * dl[1] + c.M * dl[1] * dl[1];
    p.S[2] += c.S[2] + 2.0 * c.D[2] * dl[2] + c.M * dl[2] * dl[2];
    p.S[3] += c.S[3] + c.D[0] * dl[1] + c.D[1] * dl[0] + c.M * dl[0] * dl[1];
    p.S[4] += c.S[4] + c.D[0] * dl[2] + c.D[2] * dl[0] + c.M * dl[0] * dl[2];
    p.S[5] += c.S[5] + c.D[1] * dl[2] + c.D[2] * dl[1] + c.M * dl[1] * dl[2];
    p.h = fmax(p.h, c.h);
}

__device__ __forceinline__ void centre(const double *clo, const double *chi, int64_t k, double g[3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d) g[d] = 0.5 * (clo[3 * k + d] + chi[3 * k + d]);
}

// Lane exchange inside rows of the wave (DPP, a VALU operation): CTRL 0xB1
// swaps lanes 2i and 2i+1, 0x4E swaps pairs within each quad, 0x141 mirrors
// each group of eight lanes.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <int CTRL>
__device__ __forceinline__ void raw_dpp_add(RawMom &r) {
    r.M += dpp_d<CTRL>(r.M);
#pragma unroll
    for (int d = 0; d < 3; ++d) r.D[d] += dpp_d<CTRL>(r.D[d]);
#pragma unroll
    for (int d = 0; d < 6; ++d) r.S[d] += dpp_d<CTRL>(r.S[d]);
    r.h = fmax(r.h, dpp_d<CTRL>(r.h));
}

// Sum of the raw moments held by each aligned group of eight lanes (every
// lane of a group active): pairs, quads, then the mirrored quad.  Lane 0 of
// the group holds the sum, in the same order on every run.
__device__ __forceinline__ void raw_group_sum8(RawMom &r) {
    raw_dpp_add<0xB1>(r);
    raw_dpp_add<0x4E>(r);
    raw_dpp_add<0x141>(r);
}

// Leaves: sums over their particles about the cube centre (and each
// particle's leaf index, used by the adjoint).  Eight lanes per node, lane j
// taking particles j, j + 8, ...; the whole group leaves together for inner
// nodes.
template <typename T>
__global__ __launch_bounds__(256) void k_moments_leaf(
    int64_t n_nodes, const int32_t *__restrict__ nfirst, const int32_t *__restrict__ ncount,
    const int32_t *__restrict__ nnchild, const double *__restrict__ clo,
    const double *__restrict__ chi, const T *__restrict__ xs, const T *__restrict__ ys,
    const T *__restrict__ zs, const T *__restrict__ ms, const T *__restrict__ hs,
    const int32_t *__restrict__ order, int64_t n_gas, double *__restrict__ raw0,
    double *__restrict__ raw1, int32_t *__restrict__ pleaf) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = gid >> 3;
    const int j = (int)(gid & 7);
    if (k >= n_nodes || nnchild[k] != 0) return;
    double g[3];
    centre(clo, chi, k, g);
    RawMom ra, rg;
    raw_zero(ra);
    raw_zero(rg);
    const int64_t f = nfirst[k], e = f + ncount[k];
    for (int64_t p = f + j; p < e; p += 8) {
        pleaf[p] = (int32_t)k;
        const double m = (double)ms[p], h = (double)hs[p];
        const double y0 = (double)xs[p] - g[0], y1 = (double)ys[p] - g[1], y2 = (double)zs[p] - g[2];
        raw_add_point(ra, m, y0, y1, y2, h);
        if (order[p] < n_gas) raw_add_point(rg, m, y0, y1, y2, h);
    }
    raw_group_sum8(ra);
    raw_group_sum8(rg);
    if (j == 0) {
        raw_store(raw0, k, ra);
        raw_store(raw1, k, rg);
    }
}

// Inner node k from its children, eight lanes per node, lane j shifting child
// j from its centre to k's centre; lane 0 stores the group's sum.
__device__ __forceinline__ void node_from_children8(int64_t k, int j, const int32_t *__restrict__ nchild,
                                                    const int32_t *__restrict__ nnchild,
                                                    const double *__restrict__ clo,
                                                    const double *__restrict__ chi, double *raw0,
                                                    double *raw1) {
    RawMom ra, rg;
    raw_zero(ra);
    raw_zero(rg);
    if (j < nnchild[k]) {
        const int64_t ch = nchild[k] + j;
        double gp[3], gc[3], dl[3];
        centre(clo, chi, k, gp);
        centre(clo, chi, ch, gc);
        for (int d = 0; d < 3; ++d) dl[d] = gc[d] - gp[d];
        RawMom cm;
        raw_load(raw0, ch, cm);
        raw_add_child(ra, cm, dl);
        raw_load(raw1, ch, cm);
        raw_add_child(rg, cm, dl);
    }
    raw_group_sum8(ra);
    raw_group_sum8(rg);
    if (j == 0) {
        raw_store(raw0, k, ra);
        raw_store(raw1, k, rg);
    }
}

// Inner nodes of one level (their children were done by earlier launches).
__global__ __launch_bounds__(256) void k_moments_level(int64_t k0, int64_t k1,
                                                       const int32_t *__restrict__ nchild,
                                                       const int32_t *__restrict__ nnchild,
                                                       const double *__restrict__ clo,
                                                       const double *__restrict__ chi,
                                                       double *raw0, double *raw1) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = k0 + (gid >> 3);
    if (k >= k1 || nnchild[k] == 0) return;
    node_from_children8(k, (int)(gid & 7), nchild, nnchild, clo, chi, raw0, raw1);
}

struct LevelRange {
    int64_t off[kLevels + 2];
};

// Inner nodes of the small levels l_hi, l_hi - 1, ..., l_lo in one workgroup,
// deepest first, a barrier between levels (one launch instead of one per
// level where a level has few nodes).
__global__ __launch_bounds__(1024) void k_moments_levels(LevelRange lr, int l_hi, int l_lo,
                                                         const int32_t *__restrict__ nchild,
                                                         const int32_t *__restrict__ nnchild,
                                                         const double *__restrict__ clo,
                                                         const double *__restrict__ chi,
                                                         double *raw0, double *raw1) {
    for (int l = l_hi; l >= l_lo; --l) {
        for (int64_t base = lr.off[l]; base < lr.off[l + 1]; base += blockDim.x / 8) {
            const int64_t k = base + (threadIdx.x >> 3);
            if (k < lr.off[l + 1] && nnchild[k] != 0)   // uniform over each group of 8
                node_from_children8(k, threadIdx.x & 7, nchild, nnchild, clo, chi, raw0, raw1);
        }
        __syncthreads();
    }
}

__global__ void k_moments_final(int64_t n_nodes, const double *__restrict__ clo,
                                const double *__restrict__ chi, const double *__restrict__ raw,
                                double *__restrict__ M, double *__restrict__ com,
                                double *__restrict__ Q, double *__restrict__ hmax,
                                const int32_t *__restrict__ nfirst,
                                const int32_t *__restrict__ ncount,
                                const int32_t *__restrict__ nchild,
                                const int32_t *__restrict__ nnchild,
                                const int32_t *__restrict__ nlevel, NodeW *__restrict__ nw,
                                NodeQ *__restrict__ nq) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_nodes) return;
    {
        NodeW w;
        const double *pr = raw + 11 * k;
        const double m = pr[0];
        for (int d = 0; d < 3; ++d) {
            w.clo[d] = clo[3 * k + d];
            w.chi[d] = chi[3 * k + d];
            w.com[d] = m > 0.0 ? 0.5 * (clo[3 * k + d] + chi[3 * k + d]) + pr[1 + d] / m
                               : 0.5 * (clo[3 * k + d] + chi[3 * k + d]);
        }
        w.hmax = pr[10];
        w.M = m;
        w.first = nfirst[k];
        w.count = ncount[k];
        w.child = nchild[k];
        w.lvl_nch = (nlevel[k] << 8) | nnchild[k];
        w.pad[0] = w.pad[1] = 0.0;
        nw[k] = w;
    }
    double g[3];
    centre(clo, chi, k, g);
    const double *p = raw + 11 * k;
    const double m = p[0];
    M[k] = m;
    hmax[k] = p[10];
    if (m > 0.0) {
        const double c0 = p[1] / m, c1 = p[2] / m, c2 = p[3] / m;
        com[3 * k] = g[0] + c0;
        com[3 * k + 1] = g[1] + c1;
        com[3 * k + 2] = g[2] + c2;
        const double sxx = p[4] - p[1] * c0, syy = p[5] - p[2] * c1, szz = p[6] - p[3] * c2;
        const double sxy = p[7] - p[1] * c1, sxz = p[8] - p[1] * c2, syz = p[9] - p[2] * c2;
        const double tr = sxx + syy + szz;
        Q[6 * k] = 3.0 * sxx - tr;
        Q[6 * k + 1] = 3.0 * syy - tr;
        Q[6 * k + 2] = 3.0 * szz - tr;
        Q[6 * k + 3] = 3.0 * sxy;
        Q[6 * k + 4] = 3.0 * sxz;
        Q[6 * k + 5] = 3.0 * syz;
    } else {
        for (int d = 0; d < 3; ++d) com[3 * k + d] = g[d];
        for (int d = 0; d < 6; ++d) Q[6 * k + d] = 0.0;
    }
    NodeQ q;
    q.q[0] = Q[6 * k];
    q.q[1] = Q[6 * k + 1];
    q.q[2] = Q[6 * k + 3];
    q.q[3] = Q[6 * k + 4];
    q.q[4] = Q[6 * k + 5];
    q.pad = 0.0;
    nq[k] = q;
}

sf_status build_moments(sf_grav_tree_s *t, DevArena &ar, bool refit) {
    hipStream_t s = t->stream;
    const int64_t nn = t->n_nodes;
    double *raw0, *raw1;
    SF_ALLOC_TMP(ar, raw0, 11 * nn);
    SF_ALLOC_TMP(ar, raw1, 11 * nn);
    if (!refit) {   // a refit overwrites the handle's arrays in place
        SF_ALLOC(ar, t->pleaf, t->n);
        for (int set = 0; set < 2; ++set) {
            SF_ALLOC(ar, t->M[set], nn);
            SF_ALLOC(ar, t->com[set], 3 * nn);
            SF_ALLOC(ar, t->Q[set], 6 * nn);
            SF_ALLOC(ar, t->hmax[set], nn);
            SF_ALLOC(ar, t->nw[set], nn);
            SF_ALLOC(ar, t->nq[set], nn);
        }
    }
    if (t->dt == SF_F32)
        hipLaunchKernelGGL(k_moments_leaf<float>, dim3(nblk(8 * nn)), dim3(256), 0, s, nn,
                           t->nfirst, t->ncount, t->nnchild, t->clo, t->chi, (const float *)t->xs,
                           (const float *)t->ys, (const float *)t->zs, (const float *)t->ms,
                           (const float *)t->hs, t->order, t->n_gas, raw0, raw1, t->pleaf);
    else
        hipLaunchKernelGGL(k_moments_leaf<double>, dim3(nblk(8 * nn)), dim3(256), 0, s, nn,
                           t->nfirst, t->ncount, t->nnchild, t->clo, t->chi, (const double *)t->xs,
                           (const double *)t->ys, (const double *)t->zs, (const double *)t->ms,
                           (const double *)t->hs, t->order, t->n_gas, raw0, raw1, t->pleaf);
    // inner nodes, deepest level first (level offsets are known on the host);
    // runs of consecutive small levels share one single-workgroup launch
    constexpr int64_t kSmallLevel = 128;   // one pass of the 1024-lane workgroup
    LevelRange lr;
    for (int l = 0; l <= kLevels + 1; ++l) lr.off[l] = t->level_off[l];
    for (int l = kLevels - 1; l >= 0;) {
        const int64_t k0 = t->level_off[l], k1 = t->level_off[l + 1];
        if (k1 - k0 > kSmallLevel) {
            if (t->level_off[l + 2] > t->level_off[l + 1])   // some children below
                hipLaunchKernelGGL(k_moments_level, dim3(nblk(8 * (k1 - k0))), dim3(256), 0, s, k0, k1,
                                   t->nchild, t->nnchild, t->clo, t->chi, raw0, raw1);
            --l;
            continue;
        }
        int lo = l;
        while (lo > 0 && t->level_off[lo] - t->level_off[lo - 1] <= kSmallLevel) --lo;
        if (t->level_off[l + 1] > t->level_off[lo])   // some nodes in the run
            hipLaunchKernelGGL(k_moments_levels, dim3(1), dim3(1024), 0, s, lr, l, lo, t->nchild,
                               t->nnchild, t->clo, t->chi, raw0, raw1);
        l = lo - 1;
    }
    double *raws[2] = {raw0, raw1};
    for (int set = 0; set < 2; ++set)
        hipLaunchKernelGGL(k_moments_final, dim3(nblk(nn)), dim3(256), 0, s, nn, t->clo, t->chi,
                           raws[set], t->M[set], t->com[set], t->Q[set], t->hmax[set], t->nfirst,
                           t->ncount, t->nchild, t->nnchild, t->nlevel, t->nw[set], t->nq[set]);
    SF_HIP(hipGetLastError());
    return SF_OK;
}

// ---------------------------------------------------------------- A7 groups

// Group starts: a node holding at most group_cap particles is one group;
// consecutive such children of a split node are packed greedily while the
// run stays within group_cap; an over-full leaf is cut into slices.
__global__ void k_grp_mark(int64_t n_nodes, const int32_t *__restrict__ nfirst,
                           const int32_t *__restrict__ ncount, const int32_t *__restrict__ nchild,
                           const int32_t *__restrict__ nnchild, int gcap,
                           uint32_t *__restrict__ mark) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_nodes) return;
    const int64_t f = nfirst[k], c = ncount[k];
    if (k == 0 && c <= gcap) mark[0] = 1u;
    if (c <= gcap) return;
    if (nnchild[k] == 0) {
        for (int64_t s = f; s < f + c; s += gcap) mark[s] = 1u;
        return;
    }
    int64_t run = 0;
    const int64_t c0 = nchild[k], c1 = c0 + nnchild[k];
    for (int64_t ch = c0; ch < c1; ++ch) {
        const int64_t cc = ncount[ch];
        if (cc > gcap) {
            run = 0;
            continue;
        }
        if (run + cc > gcap) run = 0;
        if (run == 0) mark[nfirst[ch]] = 1u;
        run += cc;
    }
}

__global__ void k_grp_write(const uint32_t *__restrict__ mark, const uint32_t *__restrict__ idx,
                            int64_t n, int32_t *__restrict__ gfirst) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n && mark[s]) gfirst[idx[s]] = (int32_t)s;
}

// One wave per group: count, bounding box, max softening and centre.  The
// extremes are taken in the input precision (exact), the centre is the box
// midpoint in FP64 rounded to the input precision.
template <typename T>
__global__ __launch_bounds__(256) void k_grp_info(const int32_t *__restrict__ n_groups_dev, int64_t n,
                                                  int32_t *__restrict__ gfirst,
                                                  int32_t *__restrict__ gcount,
                                                  const T *__restrict__ xs, const T *__restrict__ ys,
                                                  const T *__restrict__ zs, const T *__restrict__ hs,
                                                  double *__restrict__ gbox,
                                                  double *__restrict__ ghmax,
                                                  double *__restrict__ gcen) {
    const int64_t ng = *n_groups_dev;
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; g < ng; g += nwaves) {
        const int64_t f = gfirst[g];
        const int64_t e = (g + 1 < ng) ? gfirst[g + 1] : n;
        const int64_t c = e - f;
        T lo[3] = {(T)INFINITY, (T)INFINITY, (T)INFINITY};
        T hi[3] = {-(T)INFINITY, -(T)INFINITY, -(T)INFINITY};
        T hm = (T)0;
        if (lane < c) {
            const int64_t p = f + lane;
            const T v[3] = {xs[p], ys[p], zs[p]};
            for (int d = 0; d < 3; ++d) { lo[d] = v[d]; hi[d] = v[d]; }
            hm = hs[p];
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            for (int d = 0; d < 3; ++d) {
                lo[d] = fmin(lo[d], __shfl_xor(lo[d], off, 64));
                hi[d] = fmax(hi[d], __shfl_xor(hi[d], off, 64));
            }
            hm = fmax(hm, __shfl_xor(hm, off, 64));
        }
        if (lane == 0) {
            gcount[g] = (int32_t)c;
            for (int d = 0; d < 3; ++d) {
                gbox[6 * g + d] = (double)lo[d];
                gbox[6 * g + 3 + d] = (double)hi[d];
                gcen[3 * g + d] = (double)(T)(0.5 * ((double)lo[d] + (double)hi[d]));
            }
            ghmax[g] = (double)hm;
        }
    }
}

sf_status build_groups(sf_grav_tree_s *t, DevArena &ar) {
    hipStream_t s = t->stream;
    const int64_t n = t->n, nn = t->n_nodes;
    const int gcap = t->group_cap;
    // every group is a node, a run starting at a distinct child node, or a
    // slice of an over-full leaf
    const int64_t cap_groups = 2 * nn + (n + gcap - 1) / gcap + 1;
    t->groups_cap = cap_groups;
    uint32_t *mark, *idx, *scr;
    SF_ALLOC_TMP(ar, mark, n);
    SF_ALLOC_TMP(ar, idx, n);
    SF_ALLOC_TMP(ar, scr, scan_scratch_words(n));
    SF_ALLOC(ar, t->n_groups_dev, 1);
    SF_ALLOC(ar, t->gfirst, cap_groups);
    SF_ALLOC(ar, t->gcount, cap_groups);
    SF_ALLOC(ar, t->gbox, 6 * cap_groups);
    SF_ALLOC(ar, t->ghmax, cap_groups);
    SF_ALLOC(ar, t->gcen, 3 * cap_groups);
    fill_u32(mark, n, 0u, s);
    hipLaunchKernelGGL(k_grp_mark, dim3(nblk(nn)), dim3(256), 0, s, nn, t->nfirst, t->ncount,
                       t->nchild, t->nnchild, gcap, mark);
    scan_u32(mark, idx, n, scr, (uint32_t *)t->n_groups_dev, s);
    hipLaunchKernelGGL(k_grp_write, dim3(nblk(n)), dim3(256), 0, s, mark, idx, n, t->gfirst);
    return group_boxes(t);
}

// Box, centre and largest softening of every group from the sorted particles.
sf_status group_boxes(sf_grav_tree_s *t) {
    hipStream_t s = t->stream;
    const int64_t n = t->n;
    const int blocks = 16384;   // four waves per block, one group per wave
    if (t->dt == SF_F32)
        hipLaunchKernelGGL(k_grp_info<float>, dim3(blocks), dim3(256), 0, s, t->n_groups_dev, n,
                           t->gfirst, t->gcount, (const float *)t->xs, (const float *)t->ys,
                           (const float *)t->zs, (const float *)t->hs, t->gbox, t->ghmax, t->gcen);
    else
        hipLaunchKernelGGL(k_grp_info<double>, dim3(blocks), dim3(256), 0, s, t->n_groups_dev, n,
                           t->gfirst, t->gcount, (const double *)t->xs, (const double *)t->ys,
                           (const double *)t->zs, (const double *)t->hs, t->gbox, t->ghmax,
                           t->gcen);
    SF_HIP(hipGetLastError());
    return SF_OK;
}

// New particle values on a frozen tree: the sorted SoA is re-gathered in the
// handle's order, moments and group boxes are recomputed; keys, order,
// topology, cubes and group ranges stay as built.
sf_status refit(sf_grav_tree_s *t, const void *pos, const void *mass, const void *soft,
                DevArena &ar) {
    hipStream_t s = t->stream;
    const int64_t n = t->n;
    if (t->dt == SF_F32)
        hipLaunchKernelGGL(k_permute<float>, dim3(nblk(n)), dim3(256), 0, s, (const float *)pos,
                           (const float *)mass, (const float *)soft, (const uint32_t *)t->order, n,
                           (float *)t->xs, (float *)t->ys, (float *)t->zs, (float *)t->ms,
                           (float *)t->hs);
    else
        hipLaunchKernelGGL(k_permute<double>, dim3(nblk(n)), dim3(256), 0, s, (const double *)pos,
                           (const double *)mass, (const double *)soft, (const uint32_t *)t->order,
                           n, (double *)t->xs, (double *)t->ys, (double *)t->zs, (double *)t->ms,
                           (double *)t->hs);
    sf_status st = build_moments(t, ar, true);
    if (st != SF_OK) return st;
    return group_boxes(t);
}

}  // namespace sf
