// noalloc.hip -- the residual r = 1 - Z w (FP64, Z regenerated from the
// coordinates) without any device allocation, for callers that cannot
// allocate (code under graph capture, tight serving loops).
//
// Its only device workspace is a file-scope array of kScratchDoubles doubles
// (16 MiB) that every GPU the library runs on holds until the process ends.
// Host code never uses the array's name as an address: mag_create takes the
// array's device address once per device with hipGetSymbolAddress (that
// device current) and every launch and copy uses that address.  All calls on
// one GPU share its array, so calls that overlap on one GPU race; nothing in
// it needs to start at zero (every entry the kernels read they first write).
#include "internal.hpp"

#include <mutex>

namespace mag {
namespace {

constexpr size_t kScratchDoubles = (size_t)1 << 21;  // 16 MiB
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double *g_addr[kMaxDevices] = {};

// doubles the call needs: y (npad), the split partials and block maxima, the norm
size_t needed_doubles(int64_t n)
{
    return (size_t)round_up(n, kPad) + zmv_split_partial_doubles(n) + 8;
}

}  // namespace

int noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return MAG_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_addr[device]) return MAG_OK;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return MAG_EHIP;
    if (cur != device && hipSetDevice(device) != hipSuccess) return MAG_EHIP;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return MAG_EHIP;
    }
    g_addr[device] = (double *)p;
    return MAG_OK;
}

}  // namespace mag

using namespace mag;

extern "C" {

size_t mag_residual_noalloc_max_doubles(void) { return kScratchDoubles; }

int mag_residual_noalloc(mag_ctx *c, const double *X, int64_t n, int32_t m, double t, const double *w,
                         double *r, double *rinf)
{
    if (!c || !X || !w || !r || n < 1 || m < 1 || !std::isfinite(t) || !(t > 0.0)) return MAG_EINVAL;
    if (c->device < 0 || c->device >= kMaxDevices) return MAG_EINVAL;
    if (needed_doubles(n) > kScratchDoubles) return MAG_ENOMEM;
    double *base;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        base = g_addr[c->device];
    }
    if (!base) return MAG_EINTERNAL;
    if (hipSetDevice(c->device) != hipSuccess) return MAG_EHIP;
    hipStream_t s = c->stream;
    const int64_t npad = round_up(n, kPad);
    double *y = base;
    double *partial = y + npad;
    double *nrm = partial + zmv_split_partial_doubles(n);
    launch_zmv_split(s, X, n, m, t, w, y, nullptr, 1, partial, nrm);
    if (hipGetLastError() != hipSuccess) return MAG_EHIP;
    if (hipMemcpyAsync(r, y, sizeof(double) * n, hipMemcpyDeviceToDevice, s) != hipSuccess) return MAG_EHIP;
    if (rinf && hipMemcpyAsync(c->host_scalars + 56, nrm, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
        return MAG_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return MAG_EHIP;
    if (rinf) *rinf = c->host_scalars[56];
    return MAG_OK;
}

}  // extern "C"
