// sf_prims.hip -- device-wide primitives for the tree build on gfx950:
// fill, exclusive scan (single pass, decoupled look-back) and a stable LSD
// radix sort of 64-bit keys with 32-bit values (onesweep-style: one
// histogram pass for all digits, then one chained-scan scatter per digit).
#include "sf_prims.h"

namespace sf {

// ---------------------------------------------------------------- fill

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
}

// Several ranges in one launch: block b of the grid strides over every range.
__global__ void k_fill_ranges_u32(FillRanges r, uint32_t v) {
    for (int k = 0; k < r.count; ++k) {
        uint32_t *p = r.p[k];
        const int64_t n = r.n[k];
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * blockDim.x)
            p[i] = v;
    }
}

void fill_ranges_u32(const FillRanges &r, uint32_t v, hipStream_t s) {
    int64_t most = 0;
    for (int k = 0; k < r.count; ++k) most = r.n[k] > most ? r.n[k] : most;
    if (most <= 0) return;
    int64_t blocks = (most + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_ranges_u32, dim3((unsigned)blocks), dim3(256), 0, s, r, v);
}

// ---------------------------------------------------------------- scan

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;   // 4096 values per tile

// Wave-level inclusive scan of 32-bit values (64 lanes).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Look back over earlier tiles' status words until an inclusive prefix is
// found.  Tiles are taken from an atomic counter in start order, so every
// earlier tile belongs to a workgroup that has already started and will
// publish; the wait ends.
__device__ __forceinline__ uint32_t look_back(uint32_t *status, int64_t tile, int stride, int slot) {
    uint32_t prefix = 0;
    int64_t t = tile - 1;
    while (t >= 0) {
        uint32_t v;
        do {
            v = ld_dev_u32(&status[t * stride + slot]);
        } while ((v & ~kValMask) == 0);
        prefix += v & kValMask;
        if (v & kFlagPre) break;
        --t;
    }
    return prefix;
}

// Look-back by one wave: lane i reads the status of tile t - i.  The nearest
// tile with an inclusive prefix ends the walk once every tile between is
// published; otherwise, with all 64 published, their aggregates are added and
// the window moves 64 tiles back.  Tiles start in counter order, so every
// earlier tile belongs to a running workgroup that will publish.
__device__ __forceinline__ uint32_t wave_look_back(uint32_t *status, int64_t tile) {
    const int lane = threadIdx.x & 63;
    uint32_t prefix = 0;
    int64_t t = tile - 1;
    while (true) {
        const int64_t j = t - lane;
        const uint32_t v = j >= 0 ? ld_dev_u32(&status[j]) : kFlagPre;
        const uint64_t wait = __ballot((v & ~kValMask) == 0);
        const uint64_t pre = __ballot((v & kFlagPre) != 0);
        if (pre) {
            const int lp = __ffsll((long long)pre) - 1;
            const uint64_t upto = lp == 63 ? ~0ull : ((1ull << (lp + 1)) - 1);
            if (wait & upto) continue;
            uint32_t x = lane <= lp ? (v & kValMask) : 0u;
            for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
            return (prefix + x) & kValMask;
        }
        if (wait) continue;
        uint32_t x = v & kValMask;
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        prefix += x;
        t -= 64;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_u32(const uint32_t *__restrict__ in,
                                                           uint32_t *__restrict__ out, int64_t n,
                                                           uint32_t *status, uint32_t *tile_ctr,
                                                           uint32_t *total) {
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wave[kScanThreads / 64];
    __shared__ uint32_t s_prefix;
    if (threadIdx.x == 0) s_tile = atomicAdd(tile_ctr, 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t base = tile * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    if (base + kScanItems <= n) {   // whole run in range: four 16-byte loads
        const uint4 *p = reinterpret_cast<const uint4 *>(in + base);
#pragma unroll
        for (int q = 0; q < kScanItems / 4; ++q) {
            const uint4 w = p[q];
            v[4 * q] = w.x;
            v[4 * q + 1] = w.y;
            v[4 * q + 2] = w.z;
            v[4 * q + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = (base + k < n) ? in[base + k] : 0u;
    }
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) sum += v[k];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan(sum);
    if (lane == 63) s_wave[wid] = incl;
    __syncthreads();
    uint32_t wave_off = 0, tile_sum = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) {
        if (w < wid) wave_off += s_wave[w];
        tile_sum += s_wave[w];
    }
    if (wid == 0) {
        uint32_t p = 0;
        if (tile == 0) {
            if (lane == 0) st_dev_u32(&status[0], kFlagPre | tile_sum);
        } else {
            if (lane == 0) st_dev_u32(&status[tile], kFlagAgg | tile_sum);
            p = wave_look_back(status, tile);
            if (lane == 0) st_dev_u32(&status[tile], kFlagPre | ((p + tile_sum) & kValMask));
        }
        if (lane == 0) {
            s_prefix = p;
            const int64_t tiles = (n + kScanTile - 1) / kScanTile;
            if (tile == tiles - 1 && total) *total = p + tile_sum;
        }
    }
    __syncthreads();
    uint32_t run = s_prefix + wave_off + incl - sum;
    uint32_t o[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        o[k] = run;
        run += v[k];
    }
    if (base + kScanItems <= n) {
        uint4 *q4 = reinterpret_cast<uint4 *>(out + base);
#pragma unroll
        for (int q = 0; q < kScanItems / 4; ++q)
            q4[q] = make_uint4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (base + k < n) out[base + k] = o[k];
    }
}

int64_t scan_scratch_words(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

void scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *scratch, uint32_t *total,
              hipStream_t s) {
    int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles == 0) {
        if (total) hipMemsetAsync(total, 0, sizeof(uint32_t), s);
        return;
    }
    fill_u32(scratch, tiles + 1, 0u, s);
    hipLaunchKernelGGL(k_scan_u32, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, out, n,
                       scratch + 1, scratch, total);
}

// ---------------------------------------------------------------- radix sort

constexpr int kRsThreads = 256;
constexpr int kRsItems = 16;
constexpr int kRsWaves = kRsThreads / 64;
constexpr int kRsTile = kRsThreads * kRsItems;   // 4096 keys per tile

// Histograms of all eight 8-bit digits in one read of the keys.
__global__ __launch_bounds__(256) void k_rs_hist(const uint64_t *__restrict__ keys, int64_t n,
                                                 uint32_t *__restrict__ hist, int passes) {
    __shared__ uint32_t sh[8][256];
    for (int i = threadIdx.x; i < 8 * 256; i += blockDim.x) (&sh[0][0])[i] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k = keys[i];
        for (int p = 0; p < passes; ++p) atomicAdd(&sh[p][(k >> (8 * p)) & 255], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < passes * 256; i += blockDim.x) {
        uint32_t c = (&sh[0][0])[i];
        if (c) atomicAdd(&hist[i], c);
    }
}

// Exclusive scan of each pass's 256 digit counts (one block, one wave per pass).
__global__ void k_rs_offsets(uint32_t *hist, int passes) {
    const int p = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (p >= passes) return;
    uint32_t c[4], s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        c[k] = hist[p * 256 + lane * 4 + k];
        s += c[k];
    }
    uint32_t incl = wave_incl_scan(s);
    uint32_t run = incl - s;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        hist[p * 256 + lane * 4 + k] = run;
        run += c[k];
    }
}

// One stable scatter pass by the digit (key >> shift) & 255.  Within a tile,
// wave w owns the contiguous segment [w*1024, (w+1)*1024) read in rounds of
// 64 consecutive keys, so (round, lane) order is input order; ranks among
// equal digits come from ballots, per-wave running counts live in LDS.  The
// tile is reordered by digit in LDS first, so that the writes of each
// digit's run go out from consecutive lanes to consecutive addresses.
template <bool kHasVal>
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint64_t *__restrict__ kout,
    uint32_t *__restrict__ vout, int64_t n, int shift, const uint32_t *__restrict__ digit_off,
    uint32_t *status, uint32_t *tile_ctr) {
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_cnt[kRsWaves][256];
    __shared__ uint32_t s_base[256];     // global start of the tile's run of each digit
    __shared__ uint32_t s_start[256];    // start of each digit's run within the tile
    __shared__ uint32_t s_wsum[kRsWaves];
    __shared__ uint64_t s_key[kRsTile];
    __shared__ uint32_t s_val[kHasVal ? kRsTile : 1];
    if (threadIdx.x == 0) s_tile = atomicAdd(tile_ctr, 1u);
    for (int i = threadIdx.x; i < kRsWaves * 256; i += kRsThreads) (&s_cnt[0][0])[i] = 0;
    __syncthreads();
    const int64_t tile = s_tile;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t seg = tile * kRsTile + (int64_t)wid * (64 * kRsItems);
    const uint64_t lt = lane_mask_lt();

    uint64_t key[kRsItems];
    uint32_t val[kRsItems];
    uint32_t rank[kRsItems];
#pragma unroll
    for (int r = 0; r < kRsItems; ++r) {
        const int64_t i = seg + r * 64 + lane;
        const bool valid = i < n;
        key[r] = valid ? kin[i] : 0ull;
        if (kHasVal) val[r] = valid ? vin[i] : 0u;
        const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bb = __ballot((d >> b) & 1u);
            m &= ((d >> b) & 1u) ? bb : ~bb;
        }
        const uint32_t before = s_cnt[wid][d];
        rank[r] = before + popc64(m & lt);
        // the lowest lane of each digit class bumps the running count; the
        // reads above were issued by the same wave first, so they see the
        // value from before this round.
        if (valid && (m & lt) == 0) s_cnt[wid][d] = before + popc64(m);
        if (!valid) rank[r] = 0xffffffffu;
    }
    __syncthreads();
    // one thread per digit: per-wave exclusive offsets, tile total, the run
    // starts within the tile (a scan over digits), look-back
    {
        const int d = threadIdx.x;
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < kRsWaves; ++w) {
            uint32_t c = s_cnt[w][d];
            s_cnt[w][d] = tot;
            tot += c;
        }
        const uint32_t incl = wave_incl_scan(tot);
        if (lane == 63) s_wsum[wid] = incl;
        uint32_t prefix = 0;
        if (tile == 0) {
            st_dev_u32(&status[d], kFlagPre | tot);
        } else {
            st_dev_u32(&status[tile * 256 + d], kFlagAgg | tot);
            prefix = look_back(status, tile, 256, d);
            st_dev_u32(&status[tile * 256 + d], kFlagPre | ((prefix + tot) & kValMask));
        }
        s_base[d] = digit_off[d] + prefix;
        __syncthreads();
        uint32_t woff = 0;
#pragma unroll
        for (int w = 0; w < kRsWaves; ++w)
            if (w < wid) woff += s_wsum[w];
        s_start[d] = woff + incl - tot;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRsItems; ++r) {
        if (rank[r] == 0xffffffffu) continue;
        const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
        const uint32_t lp = s_start[d] + s_cnt[wid][d] + rank[r];
        s_key[lp] = key[r];
        if (kHasVal) s_val[lp] = val[r];
    }
    __syncthreads();
    const int64_t left = n - tile * kRsTile;
    const int tn = left < kRsTile ? (int)left : kRsTile;
    for (int i = threadIdx.x; i < tn; i += kRsThreads) {
        const uint64_t k = s_key[i];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        const uint32_t pos = s_base[d] + (uint32_t)i - s_start[d];
        kout[pos] = k;
        if (kHasVal) vout[pos] = s_val[i];
    }
}

int64_t radix_scratch_words(int64_t n, int passes) {
    int64_t tiles = (n + kRsTile - 1) / kRsTile;
    return (int64_t)passes * 256 + (int64_t)passes * (tiles * 256 + 1);
}

// Sort (keys, vals) by the low `passes` bytes of the key; the result ends in
// (keys, vals) -- an even pass count ping-pongs back, an odd count copies.
int radix_sort_u64(uint64_t *keys, uint32_t *vals, uint64_t *keys_tmp, uint32_t *vals_tmp,
                   int64_t n, int passes, uint32_t *scratch, hipStream_t s) {
    if (n <= 1) return 0;
    const int64_t tiles = (n + kRsTile - 1) / kRsTile;
    uint32_t *hist = scratch;
    uint32_t *status = scratch + passes * 256;
    fill_u32(scratch, radix_scratch_words(n, passes), 0u, s);
    int64_t hb = (n + 255) / 256;
    if (hb > 2048) hb = 2048;
    hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)hb), dim3(256), 0, s, keys, n, hist, passes);
    hipLaunchKernelGGL(k_rs_offsets, dim3(1), dim3(64 * 8), 0, s, hist, passes);
    uint64_t *ka = keys, *kb = keys_tmp;
    uint32_t *va = vals, *vb = vals_tmp;
    for (int p = 0; p < passes; ++p) {
        uint32_t *st = status + (int64_t)p * (tiles * 256 + 1);
        if (vals)
            hipLaunchKernelGGL(k_rs_scatter<true>, dim3((unsigned)tiles), dim3(kRsThreads), 0, s, ka,
                               va, kb, vb, n, 8 * p, hist + p * 256, st + 1, st);
        else
            hipLaunchKernelGGL(k_rs_scatter<false>, dim3((unsigned)tiles), dim3(kRsThreads), 0, s,
                               ka, nullptr, kb, nullptr, n, 8 * p, hist + p * 256, st + 1, st);
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    if (ka != keys) {
        hipMemcpyAsync(keys, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
        if (vals) hipMemcpyAsync(vals, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
    }
    return 0;
}

// Single stable pass by an 8-bit field at `shift`, with precomputed digit
// offsets (exclusive prefix of the digit counts); keys only.
void radix_pass_u64(const uint64_t *kin, uint64_t *kout, int64_t n, int shift,
                    const uint32_t *digit_off, uint32_t *scratch, hipStream_t s) {
    if (n <= 0) return;
    const int64_t tiles = (n + kRsTile - 1) / kRsTile;
    fill_u32(scratch, tiles * 256 + 1, 0u, s);
    hipLaunchKernelGGL(k_rs_scatter<false>, dim3((unsigned)tiles), dim3(kRsThreads), 0, s, kin,
                       nullptr, kout, nullptr, n, shift, digit_off, scratch + 1, scratch);
}

int64_t radix_pass_scratch_words(int64_t n) { return (n + kRsTile - 1) / kRsTile * 256 + 1; }

}  // namespace sf
