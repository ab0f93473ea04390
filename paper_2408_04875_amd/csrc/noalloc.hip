// psdp_eval_penalty_grad_noalloc: the penalty value/gradient evaluation of
// psdp_eval_penalty_grad with its workspace in a fixed device array instead
// of a stream-ordered allocation, for callers that cannot allocate (code
// under graph capture, serving loops).
//
// The workspace holds the product U = Q X (n x B, FP64 on the FMA path, the
// operand type on the MFMA path) and the MFMA path's column list, exactly as
// psdp_eval_penalty_grad lays it out; the same kernels run on it. Every word
// of U the epilogue reads is written by the product first (one K slice, no
// accumulation into old contents), so nothing needs clearing between calls.
#include <map>
#include <mutex>

#include "launch.hpp"

namespace psdp {
namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB per device

// One per device, held until the process ends. Host code never uses this
// name as an address: it uses the pointer hipGetSymbolAddress returns.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_lock;
std::map<int, void *> g_scratch_ptr;  // device -> address of that device's scratch

// The calling thread's current device's copy of scratch, looked up once
// per device with that device current.
hipError_t scratch_ptr(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_scratch_lock);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        it = g_scratch_ptr.emplace(dev, p).first;
    }
    *out = it->second;
    return hipSuccess;
}

}  // namespace
}  // namespace psdp

using namespace psdp;

extern "C" {

psdp_status psdp_eval_penalty_grad_noalloc(int32_t dtype, int32_t vtype, const void *Q, int64_t ldq,
                                           const void *b, const void *p, const void *X, int64_t n,
                                           int64_t B, void *h, void *G, hipStream_t st) {
    set_error(PSDP_OK, nullptr);
    if (dtype < PSDP_F64 || dtype > PSDP_BF16) return set_error(PSDP_E_INVALID, "dtype");
    if (vtype != PSDP_F64 && vtype != PSDP_F32) return set_error(PSDP_E_INVALID, "vtype");
    if (!Q || !b || !p || !X || !h) return set_error(PSDP_E_INVALID, "null required pointer");
    if (n < 1 || B < 1 || ldq < n) return set_error(PSDP_E_INVALID, "sizes");
    if (B > 65535) return set_error(PSDP_E_UNSUPPORTED, "B > 65535");
    // the workspace psdp_eval_penalty_grad would allocate: U (n x B, at most
    // 8 bytes an entry), the column list and its count
    const double need = (double)n * (double)B * 8.0 + (double)(B + 16) * 4.0 + 256.0;
    if (need > (double)kScratchBytes)
        return set_error(PSDP_E_UNSUPPORTED, "n * B too large for the fixed workspace (8 n B + 4 B + 320 bytes "
                                             "must not exceed 32 MiB)");
    void *ws = nullptr;
    if (scratch_ptr(&ws) != hipSuccess) return set_error(PSDP_E_DEVICE, "hipGetSymbolAddress of the workspace");
    const hipError_t e = launch_eval(dtype, vtype, Q, ldq, b, p, X, n, B, h, G, (double *)ws, st);
    if (e != hipSuccess) return set_error(PSDP_E_DEVICE, hipGetErrorString(e));
    return PSDP_OK;
}

}  // extern "C"
