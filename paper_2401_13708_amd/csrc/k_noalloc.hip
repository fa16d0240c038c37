// k_noalloc.hip -- hts_gradient_exact_noalloc: the exact gradient (and cost)
// with every piece of device memory it needs beyond the caller's inputs and
// outputs taken from one fixed region per GPU, for callers that cannot
// allocate (code under graph capture, serving loops that forbid it).
//
// The region is a file-scope device array.  In host code its name only
// stands for the symbol: its address on a device is looked up once, on the
// first call on that device with the device current, and kept per device;
// every launch takes that address.  All calls on one GPU share the region
// and the last call's contents stay in it (nothing has to start at zero:
// every piece is written before it is read within a call), so calls that
// overlap on one GPU race.
#include <mutex>

#include "hts_impl.hpp"

namespace hts {

constexpr int64_t kNoAllocMaxN = HTS_NOALLOC_MAX_N;
// the largest exact_ws_bytes over n <= HTS_NOALLOC_MAX_N (17.5 MiB, both dtypes)
constexpr size_t kScratchBytes = (size_t)18 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// device address of scratch on `device`, which is current
static hts_status scratch_on(int device, char **out) {
    if (device < 0 || device >= kMaxDevices)
        return fail(HTS_EINVAL, "hts_gradient_exact_noalloc: device %d beyond the %d tracked",
                    device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(HTS_EDEVICE, "hts_gradient_exact_noalloc: no address for the workspace");
        g_scratch_ptr[device] = ptr;
    }
    *out = (char *)g_scratch_ptr[device];
    return HTS_OK;
}

}  // namespace hts

using namespace hts;

extern "C" hts_status hts_gradient_exact_noalloc(hts_ctx c, hts_stream stream, const void *Y,
                                                 int64_t n, int32_t dtype, const int64_t *row_ptr,
                                                 const int32_t *col_idx, const void *p_val,
                                                 double exaggeration, void *grad, double *z_dev,
                                                 double *kl_dev) {
    const char *fn = "hts_gradient_exact_noalloc";
    if (n < 2) return fail(HTS_EINVAL, "%s: n = %lld < 2", fn, (long long)n);
    if (n > kNoAllocMaxN)
        return fail(HTS_ECAPACITY,
                    "%s: n = %lld exceeds the fixed workspace's limit of %lld points (use "
                    "hts_gradient_exact)",
                    fn, (long long)n, (long long)kNoAllocMaxN);
    if (dtype != HTS_F32 && dtype != HTS_F64) return fail(HTS_EINVAL, "%s: bad dtype %d", fn, dtype);
    if (!(exaggeration > 0.0) || !(exaggeration < __builtin_inf()))
        return fail(HTS_EINVAL, "%s: exaggeration %g must be > 0", fn, exaggeration);
    if (!Y || !row_ptr || !col_idx || !p_val || !grad || !z_dev)
        return fail(HTS_EINVAL, "%s: NULL pointer argument", fn);
    if (!c) return fail(HTS_EINVAL, "%s: ctx is NULL", fn);
    size_t sz[6];
    const size_t need =
        dtype == HTS_F64 ? exact_ws_bytes<double>(n, sz) : exact_ws_bytes<float>(n, sz);
    if (need > kScratchBytes)  // cannot happen within the point limit
        return fail(HTS_ECAPACITY, "%s: %zu workspace bytes needed, %zu fixed", fn, need,
                    kScratchBytes);
    HTS_HIP(hipSetDevice(c->device));
    char *base = nullptr;
    HTS_OKR(scratch_on(c->device, &base));
    hipStream_t st = (hipStream_t)stream;
    if (dtype == HTS_F64)
        return exact_impl<double>(c, st, (const double *)Y, n, row_ptr, col_idx,
                                  (const double *)p_val, exaggeration, (double *)grad, z_dev,
                                  kl_dev, exact_carve<double>(base, n), false);
    return exact_impl<float>(c, st, (const float *)Y, n, row_ptr, col_idx, (const float *)p_val,
                             exaggeration, (float *)grad, z_dev, kl_dev,
                             exact_carve<float>(base, n), false);
}
