// noalloc.hip -- tcu_join_agg_fwd_noalloc: the forward operator with the
// library's own device array as its workspace, for callers that cannot
// allocate device memory (code under graph capture, serving loops, harnesses
// that forbid hipMalloc).
//
// The array lives in the code object: every device the library runs on holds
// one copy of kScratchBytes from module load until the process ends.  Host
// code never uses the array's name as an address (on the host it is only a
// stand-in for the symbol); the device address comes from
// hipGetSymbolAddress, looked up once per device with that device current,
// and is kept per device.
#include <mutex>

#include "internal.h"

namespace tcu {
namespace {

// 64 MiB plus room for the status block and alignment: holds the FP64 form's
// X and Y for M = K = N = 2048.
constexpr size_t kScratchBytes = TCU_NOALLOC_MAX_BYTES;
static_assert(kScratchBytes == (64u << 20) + (64u << 10), "scratch size");
constexpr int kMaxDevices = 64;

}  // namespace
}  // namespace tcu

static __device__ __align__(256) unsigned char scratch[tcu::kScratchBytes];

namespace tcu {
namespace {

// The status block of the last call, copied to the caller's buffer.
__global__ void copy_status_kernel(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst) {
    dst[threadIdx.x] = src[threadIdx.x];  // 64 threads x 4 bytes
}

// Device address of `scratch` on the current device (looked up on the first
// call on that device).
hipError_t scratch_ptr(void **out) {
    static std::mutex mu;
    static void *ptrs[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (ptrs[dev] == nullptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr || ((uintptr_t)p % kAlign) != 0) return hipErrorInvalidSymbol;
        ptrs[dev] = p;
    }
    *out = ptrs[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace tcu

extern "C" {

tcu_status tcu_join_agg_fwd_noalloc(const tcu_relation *A, const tcu_relation *B, int32_t M,
                                    int32_t K, int32_t N, tcu_precision p, double tol, double *C,
                                    int32_t *count, void *status, hipStream_t stream) {
    if (status != nullptr && ((uintptr_t)status % tcu::kAlign) != 0) return TCU_ERR_ARG;
    const size_t need = tcu::join_agg_fwd_ws_bytes(A, B, M, K, N, p, count != nullptr);
    if (need == 0) return TCU_ERR_ARG;
    if (need > tcu::kScratchBytes) return TCU_ERR_WORKSPACE;
    void *ws = nullptr;
    if (tcu::scratch_ptr(&ws) != hipSuccess) return TCU_ERR_HIP;
    const tcu_status st =
        tcu::join_agg_fwd_ws(A, B, M, K, N, p, tol, C, count, ws, tcu::kScratchBytes, stream);
    if (st != TCU_OK || status == nullptr) return st;
    tcu::copy_status_kernel<<<1, 64, 0, stream>>>(static_cast<const uint32_t *>(ws),
                                                  static_cast<uint32_t *>(status));
    return hipGetLastError() == hipSuccess ? TCU_OK : TCU_ERR_HIP;
}

}  // extern "C"
