// Gram products without a caller workspace, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid allocation).  The split-K partial sums live in a file-scope
// device array; each GPU holds its own copy at its own address, which host
// code obtains with hipGetSymbolAddress once per device and uses for every
// kernel argument (the array's name is only a host-side stand-in).
//
// Every call on one GPU shares that GPU's array: calls that overlap on one
// GPU (different streams or threads) race.  The partials of each call are
// written in full before they are read, so nothing has to start at zero.
#include <mutex>

#include "stf_internal.h"

namespace stf {
namespace {

constexpr size_t kScratchBytes = STF_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The device address of this GPU's scratch array (looked up once per device,
// with that device current).
int scratch_ptr(double** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return STF_E_HIP;
    if (dev < 0 || dev >= kMaxDevices) return STF_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return STF_E_HIP;
        g_ptr[dev] = p;
    }
    *out = (double*)g_ptr[dev];
    return STF_OK;
}

}  // namespace
}  // namespace stf

using namespace stf;

extern "C" {

int stf_gram_noalloc(const stf_problem* prob, const void* X, const void* G, int32_t dtype,
                     int32_t precision, double* S, double* W, hipStream_t stream) {
    int rc = check_problem(prob);
    if (rc) return rc;
    if (!X || !G || !S || !W) return STF_E_INVALID;
    if (dtype != STF_F64 && dtype != STF_F32) return STF_E_INVALID;
    if (precision < STF_PREC_FP64 || precision > STF_PREC_MIXED) return STF_E_INVALID;
    if ((precision == STF_PREC_FP64) != (dtype == STF_F64)) return STF_E_UNSUPPORTED;
    const int64_t n = prob->n;
    const int p = prob->p;
    // the plan of stf_gram, with the split-K chunk count capped so that the
    // partials [chunk][tile][bt][bt] fit the scratch array
    GramPlan gp = make_gram_plan(n, p);
    const size_t tile_bytes = (size_t)gp.bt * gp.bt * sizeof(double);
    const size_t tiles = (size_t)gp.n_s_tiles + (size_t)gp.nb * gp.nb;
    const size_t max_ch = kScratchBytes / (tiles * tile_bytes);
    if (max_ch < 1) return STF_E_SCRATCH;
    if ((size_t)gp.nchunks > max_ch) gp = make_gram_plan(n, p, (int64_t)(max_ch * tiles));
    if ((size_t)gp.nchunks * tiles * tile_bytes > kScratchBytes) return STF_E_SCRATCH;
    double* part = nullptr;
    if ((rc = scratch_ptr(&part))) return rc;
    launch_gram(dtype, precision, gp, X, G, n, p, part, S, W, nullptr, stream);
    if ((rc = last_launch())) return rc;
    return hipStreamSynchronize(stream) == hipSuccess ? last_launch() : STF_E_HIP;
}

}  // extern "C"
