// noalloc.hip -- precode_pd_noalloc: precode_pd for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// The workspace a call needs -- the fused refinement's factors, scale and
// status, or the plain kernels' Gram / factor / scale / solve workspace --
// comes from one file-scope __device__ array, `scratch`, of kScratchBytes.
// Every GPU the library runs on holds its own copy until the process ends;
// its address is taken once per device with hipGetSymbolAddress (the array's
// name is a host-side stand-in, never used as an address here).  Calls on
// one GPU share that copy: calls that overlap on one GPU (other streams,
// other host threads) race.  Nothing in the array needs to start at zero.
#include <mutex>

#include "common.h"

namespace pc {
namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
}  // namespace
}  // namespace pc

static __device__ __align__(256) unsigned char scratch[pc::kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[pc::kMaxDevices];

// This device's copy of `scratch`: its address from hipGetSymbolAddress,
// taken with the device current on the first call for that device.
int scratch_ptr(int device, void **out) {
    if (device < 0 || device >= pc::kMaxDevices) return PRECODE_EINVAL;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) {
            (void)hipGetLastError();
            return PRECODE_EDEVICE;
        }
        if (cur != device && hipSetDevice(device) != hipSuccess) {
            (void)hipGetLastError();
            return PRECODE_EDEVICE;
        }
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return PRECODE_EDEVICE;
        }
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return PRECODE_OK;
}

}  // namespace

extern "C" int precode_pd_noalloc(precode_ctx *ctx, const void *H, const void *s, float rho, const int *cluster_sizes,
                                  int C, int mode, int B, int U, int n_sc, int K, const precode_params *params,
                                  void *x, float *beta, int *status, void *stream) {
    if (!ctx) return PRECODE_EINVAL;
    void *ws = nullptr;
    const int rc = scratch_ptr(pc::ctx_device(ctx), &ws);
    if (rc) return rc;
    return pc::pd_fixed_ws(ctx, H, s, rho, cluster_sizes, C, mode, B, U, n_sc, K, params, x, beta, status, stream, ws,
                           pc::kScratchBytes);
}
