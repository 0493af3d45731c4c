// sf_prims.h -- device-wide primitives used by the tree build (internal).
#pragma once
#include "sf_internal.h"

namespace sf {

void fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);

// Up to kFillRanges ranges (p[k], n[k] words) set to one value in one launch.
constexpr int kFillRanges = 6;
struct FillRanges {
    uint32_t *p[kFillRanges];
    int64_t n[kFillRanges];
    int count = 0;
    void add(void *ptr, int64_t words) {
        if (count < kFillRanges && words > 0) {
            p[count] = (uint32_t *)ptr;
            n[count] = words;
            ++count;
        }
    }
};
void fill_ranges_u32(const FillRanges &r, uint32_t v, hipStream_t s);

// Exclusive scan of n 32-bit values; *total (device) receives the sum.
// scratch: scan_scratch_words(n) words.  Sums must stay below 2^30.
int64_t scan_scratch_words(int64_t n);
void scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *scratch, uint32_t *total,
              hipStream_t s);

// Stable LSD radix sort of (keys, vals) by the low `passes` bytes of the key.
// vals may be NULL.  keys_tmp/vals_tmp: n-element ping-pong buffers.
// scratch: radix_scratch_words(n, passes) words.
int64_t radix_scratch_words(int64_t n, int passes);
int radix_sort_u64(uint64_t *keys, uint32_t *vals, uint64_t *keys_tmp, uint32_t *vals_tmp,
                   int64_t n, int passes, uint32_t *scratch, hipStream_t s);

// One stable scatter pass of keys by the byte at `shift`, given the digit
// offsets (exclusive prefix of the digit counts, 256 entries).
int64_t radix_pass_scratch_words(int64_t n);
void radix_pass_u64(const uint64_t *kin, uint64_t *kout, int64_t n, int shift,
                    const uint32_t *digit_off, uint32_t *scratch, hipStream_t s);

}  // namespace sf
