// sf_noalloc.hip -- sf_grav_accel_direct_noalloc: the direct path of
// sf_grav_accel (same kernels, same results) with every scratch buffer
// carved out of one fixed device array instead of the library's allocator,
// for callers that cannot allocate device memory.
//
// The array is a file-scope __device__ object, so each device the library
// runs on holds its own copy for the life of the process.  Host code never
// uses the array's name as an address: on the first call on a device (that
// device current) hipGetSymbolAddress gives the device address of that
// device's copy, which is kept per device and handed to the kernels as their
// scratch base.  Calls that overlap on one device share the array and race.
#include <mutex>

#include "sf_build.h"
#include "sf_prims.h"

namespace {

constexpr int64_t kNoAllocMaxN = int64_t(1) << 19;
constexpr size_t kScratchBytes = size_t(96) << 20;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scr_mu;
void *g_scr_ptr[64] = {};

// Device address of the current device's copy of `scratch` (looked up once
// per device).
sf_status scratch_base(void **out) {
    *out = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return sf_fail(SF_E_DEVICE, "no usable current device");
    std::lock_guard<std::mutex> lk(g_scr_mu);
    if (!g_scr_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return sf_fail(SF_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s",
                           hipGetErrorString(e));
        }
        g_scr_ptr[dev] = p;
    }
    *out = g_scr_ptr[dev];
    return SF_OK;
}

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

// Scratch of one direct evaluation, in the order the direct path takes it:
// root frame, box partials, keys, order and their sort buffers, radix
// scratch, sorted SoA, sink positions and their scan, tile records, packed
// sources, sink-sink sums.  Each piece is rounded up to 256 bytes (the bump
// arena's alignment).
size_t scratch_need(int64_t n, int64_t n_sink, size_t tsize, size_t rsize) {
    const size_t un = (size_t)n;
    const size_t tiles = (size_t)((n - n_sink + 63) / 64 + (n_sink + 63) / 64);
    size_t b = a256(sizeof(sf::Frame)) + a256(1024 * 6 * sizeof(double));
    b += a256(8 * un) + a256(4 * un) + a256(8 * un) + a256(4 * un);
    b += a256(4 * (size_t)sf::radix_scratch_words(n, 8));
    b += 5 * a256(tsize * un);
    if (n_sink > 0)
        b += a256(4 * (size_t)n_sink) + a256(4 * un) + a256(4 * (size_t)sf::scan_scratch_words(n));
    b += a256(4 * tiles) + a256(4 * tiles) + a256(64 * tiles) + a256(24 * tiles);
    b += a256(rsize * un);
    if (n_sink > 0) b += a256(32 * (size_t)n_sink) + a256(8 * (size_t)sf::kSinkRec * n_sink);
    return b;
}

}  // namespace

extern "C" sf_status sf_grav_accel_direct_noalloc(const void *pos, const void *mass,
                                                  const void *soft, int64_t n, sf_dtype dt,
                                                  const sf_grav_opts *o, void *acc, void *pot,
                                                  void *stream) {
    if (!acc) return sf_fail(SF_E_INVALID, "acc is NULL");
    if (!pos || !mass || !soft) return sf_fail(SF_E_INVALID, "pos, mass and soft must be non-NULL");
    if (dt != SF_F32 && dt != SF_F64) return sf_fail(SF_E_INVALID, "dtype %d unknown", (int)dt);
    if (n < 1) return sf_fail(SF_E_INVALID, "n must be >= 1 (got %lld)", (long long)n);
    if (n > kNoAllocMaxN)
        return sf_fail(SF_E_UNSUPPORTED,
                       "n = %lld exceeds the allocation-free maximum %lld (fixed scratch of %zu "
                       "bytes)",
                       (long long)n, (long long)kNoAllocMaxN, kScratchBytes);
    if (!o) return sf_fail(SF_E_INVALID, "opts is NULL");
    if (o->struct_size != sizeof(sf_grav_opts))
        return sf_fail(SF_E_INVALID, "opts.struct_size %u != %zu", o->struct_size,
                       sizeof(sf_grav_opts));
    if (o->form != SF_FP32C && o->form != SF_FP32 && o->form != SF_FP64)
        return sf_fail(SF_E_INVALID, "opts.form %d unknown", o->form);
    if (!(o->G == o->G) || o->G > 1e300 || o->G < -1e300)
        return sf_fail(SF_E_INVALID, "opts.G must be finite");
    const int64_t ng = o->n_gas < 0 ? n : o->n_gas;
    if (ng > n) return sf_fail(SF_E_INVALID, "opts.n_gas %lld > n %lld", (long long)ng, (long long)n);
    const size_t need = scratch_need(n, n - ng, dt == SF_F32 ? 4 : 8, sf::direct_rec_bytes(o->form));
    if (need > kScratchBytes)
        return sf_fail(SF_E_UNSUPPORTED, "n = %lld needs %zu bytes of scratch, more than the %zu "
                       "of the allocation-free entry point", (long long)n, need, kScratchBytes);
    void *base = nullptr;
    sf_status st = scratch_base(&base);
    if (st != SF_OK) return st;
    sf::EvalOpts e;
    e.form = o->form;
    e.order = o->order;
    e.G = o->G;
    e.theta = o->theta;
    e.alpha = -1.0;
    e.stats = false;
    sf_grav_tree_s t;
    t.stream = (hipStream_t)stream;
    t.direct_only = true;
    sf::DevArena ar(t.stream);
    ar.set_fixed(base, kScratchBytes);
    st = sf::build_sorted(pos, mass, soft, n, ng, dt, true, o->validate != 0, &t, ar);
    if (st == SF_OK && o->validate) {
        sf::Frame hf;
        hipError_t he = hipMemcpyAsync(&hf, t.frame, sizeof(hf), hipMemcpyDeviceToHost, t.stream);
        if (he == hipSuccess) he = hipStreamSynchronize(t.stream);
        if (he != hipSuccess) return sf_fail(SF_E_DEVICE, "%s", hipGetErrorString(he));
        if (hf.bad) return sf_fail(SF_E_INVALID, "inputs contain non-finite values, h <= 0 or m < 0");
    }
    if (st == SF_OK) st = sf::direct_accel(&t, e, acc, pot, ar);
    return st;
}
