// Handle-free sketch update that allocates no device memory (usbs_sketch_update_noalloc).
//
// Same arithmetic and kernels as usbs_op_sketch_update (Sec. 4: P <- g P + W diag(lam)
// (W^T Psi)), for callers that cannot call hipMalloc (code under stream capture, serving
// loops that forbid allocation).  The reduction partials of W^T Psi and the q x r product
// live in one fixed device array per GPU; the library takes its address once per device
// with hipGetSymbolAddress and passes that address to the kernels.
#include "../../include/usbs.h"
#include "kernels.h"

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

using namespace usbs;

namespace {

// partials of the first reduction stage (kRedMaxBlocks x q*r) followed by the q x r product
constexpr int kNoallocMaxQ = USBS_NOALLOC_MAX_Q;
constexpr int kNoallocMaxR = USBS_NOALLOC_MAX_R;
constexpr size_t kPartialDoubles = (size_t)kRedMaxBlocks * kNoallocMaxQ * kNoallocMaxR;
constexpr size_t kScratchDoubles = kPartialDoubles + kNoallocMaxQ * kNoallocMaxR;
static_assert(kScratchDoubles * sizeof(double) == USBS_NOALLOC_SCRATCH_BYTES, "scratch size in the header");

// Host code never passes this name to a kernel: in host code it is a stand-in, not the
// device address.  scratch_ptr() returns the address on the current device.
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
thread_local std::string g_err;

int set_error(int code, const char *msg) {
    g_err = msg;
    return code;
}

// device address of `scratch` on the current device (looked up once per device)
int scratch_ptr(double **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return set_error(USBS_E_DEVICE, "usbs_sketch_update_noalloc: no current device");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(USBS_E_DEVICE, "usbs_sketch_update_noalloc: hipGetSymbolAddress failed");
        g_ptr[dev] = p;
    }
    *out = static_cast<double *>(g_ptr[dev]);
    return USBS_OK;
}

struct RowScale {
    double v[kNoallocMaxQ];
};

// H[a * r + c] *= lam[a]  (the product diag(lam) (W^T Psi), one workgroup)
__global__ __launch_bounds__(kWG) void k_scale_rows(int q, int r, RowScale lam, double *H) {
    for (int e = threadIdx.x; e < q * r; e += kWG) H[e] *= lam.v[e / r];
}

}  // namespace

namespace usbs_noalloc {
const char *last_error() { return g_err.empty() ? nullptr : g_err.c_str(); }
}  // namespace usbs_noalloc

extern "C" int usbs_sketch_update_noalloc(int64_t n, int32_t q, int32_t r, double g, const double *W_dev,
                                          const double *lam, const float *psi_dev, double *P_dev, void *stream) {
    if (n < 0 || n > INT32_MAX)
        return set_error(USBS_E_INVALID, "usbs_sketch_update_noalloc: n must be in [0, 2^31 - 1]");
    if (q < 1 || q > kNoallocMaxQ || r < 1 || r > kNoallocMaxR)
        return set_error(USBS_E_INVALID, "usbs_sketch_update_noalloc: q and r must be in [1, 16]");
    if (!lam || (n > 0 && (!W_dev || !psi_dev || !P_dev)))
        return set_error(USBS_E_INVALID, "usbs_sketch_update_noalloc: NULL argument");
    if (n == 0) return USBS_OK;
    double *sp = nullptr;
    if (const int rc = scratch_ptr(&sp)) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    set_tuning(nullptr);   // built-in launch shapes (the tuned ones give the same bits)
    RedScratch rs{sp, kRedMaxBlocks, q * r};
    double *H = sp + kPartialDoubles;
    RowScale ls{};
    for (int a = 0; a < q; ++a) ls.v[a] = lam[a];
    // G = W^T Psi: every workgroup writes its whole partial, the finisher writes all of G
    tn_reduce_f(s, rs, (int)n, W_dev, q, q, psi_dev, r, r, H, r, 1.0);
    hipLaunchKernelGGL(k_scale_rows, dim3(1), dim3(kWG), 0, s, q, r, ls, H);
    nn_update(s, (int)n, W_dev, q, q, H, r, r, P_dev, r, 1.0, g);
    if (hipGetLastError() != hipSuccess) return set_error(USBS_E_DEVICE, "usbs_sketch_update_noalloc: launch failed");
    g_err.clear();
    return USBS_OK;
}
