// Allocation-free Gram of a block pair: the FP64 path of qo_gram_pair for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving loops).
//
// The split-K partial sums of the Gram live in one file-scope device array, `scratch`,
// of kScratchBytes.  Host code never passes the array's name to a kernel or a copy: in
// host code that name is only a stand-in, not a device address.  The device address is
// taken once per device with hipGetSymbolAddress (with that device current) at the first
// call on it, and kept per device; each GPU holds its own copy of the array until the
// process ends.
//
// Every call on a GPU shares that GPU's array and leaves its partials in it.  Nothing has
// to start at zero: every partial that the reduction reads is written by the same call
// first.  Calls that overlap on one GPU (other streams, other threads) race on the array.
#include "qo.h"
#include "qo_internal.h"

#include <cmath>
#include <mutex>
#include <string>

namespace {

constexpr size_t kScratchBytes = 32u << 20;  // 32 MiB per device
constexpr size_t kScratchDoubles = kScratchBytes / sizeof(double);
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

thread_local std::string g_err;  // message of this thread's last failing call

qo_status nfail(qo_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

// Device address of the current device's `scratch`; nullptr on failure (g_err says why).
double *scratch_ptr(int dev) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            g_err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
            return nullptr;
        }
        g_ptr[dev] = static_cast<double *>(p);
    }
    return g_ptr[dev];
}

}  // namespace

namespace qo {
const char *noalloc_last_error() { return g_err.empty() ? "no error" : g_err.c_str(); }
}  // namespace qo

extern "C" {

qo_status qo_gram_pair_noalloc(const double *X, const double *Y, long ld, long ng, int ncols,
                               double w, double *G, void *hip_stream) {
    if (!X || !Y || !G) return nfail(QO_ERR_ARG, "qo_gram_pair_noalloc: null pointer");
    if (ng < 1 || ld < ng) return nfail(QO_ERR_ARG, "qo_gram_pair_noalloc: need 1 <= ng <= ld");
    if (ncols < 1 || ncols > QO_NOALLOC_MAX_COLS)
        return nfail(QO_ERR_ARG, "qo_gram_pair_noalloc: ncols " + std::to_string(ncols) +
                                     " outside 1.." + std::to_string(QO_NOALLOC_MAX_COLS) +
                                     " (the Gram partials must fit the 32 MiB scratch array)");
    if (!(w > 0.0) || !std::isfinite(w))
        return nfail(QO_ERR_ARG, "qo_gram_pair_noalloc: weight must be positive and finite");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return nfail(QO_ERR_DEVICE, "qo_gram_pair_noalloc: no current device");
    double *part = scratch_ptr(dev);
    if (!part) return QO_ERR_DEVICE;
    // as many row chunks as the regular path would use, within the scratch array
    const size_t per_split = (size_t)4 * ncols * ncols;
    long nsplit = qo::gram_nsplit(ng, ncols);
    const long cap = (long)(kScratchDoubles / per_split);
    if (nsplit > cap) nsplit = cap;
    if (nsplit < 1) return nfail(QO_ERR_ARG, "qo_gram_pair_noalloc: partials do not fit");
    const hipError_t e = qo::launch_gram_f64(X, Y, ld, ng, ncols, w, part, (int)nsplit, G,
                                             static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess)
        return nfail(QO_ERR_DEVICE, std::string("qo_gram_pair_noalloc: launch failed: ") +
                                        hipGetErrorString(e));
    return QO_OK;
}

}  // extern "C"
