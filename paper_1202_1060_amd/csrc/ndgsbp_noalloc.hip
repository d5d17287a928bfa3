// ldpc_decode_noalloc: ldpc_decode for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops, harnesses that
// forbid it). Its kernels take their work counter and, in the HBM tier,
// their frame-interleaved workspace from one fixed device array per GPU,
// `scratch`, instead of the code's counters and its on-demand workspace.
//
// `scratch` is a file-scope device array; on the host its name is only a
// stand-in for the symbol, so host code never passes it to a kernel or a
// copy. At set-up (ldpc_code_create, once per device, with that device
// current) hipGetSymbolAddress gives this device's address of the array,
// which is kept per device and used everywhere host code needs the array.
// Layout: bytes [0, 256) the launch's two work counters (zero between
// launches: cleared at set-up and before every call by a fill kernel, and
// reset by the decode's last workgroup), bytes [256, kScratchBytes) the
// HBM-tier workspace.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ndgsbp.h"
#include "ndgsbp_code.h"
#include "ndgsbp_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU
constexpr size_t kCounterBytes = 256;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};  // this device's address of `scratch`, after set-up

__global__ void clear_counters(uint32_t* w) {
    if (threadIdx.x < 2) w[threadIdx.x] = 0u;
}

}  // namespace

namespace ndgsbp {

hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[device]) return hipSuccess;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    e = hipMemset(ptr, 0, kCounterBytes);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    g_ptr[device] = ptr;
    return hipSuccess;
}

}  // namespace ndgsbp

extern "C" int ldpc_decode_noalloc(ldpc_code_t c, const float* llr, int32_t num_frames, int32_t max_iter,
                                   uint32_t flags, uint8_t* hard, float* post, int32_t* iters, uint8_t* syn_ok,
                                   void* hip_stream) {
    if (!c) return ndgsbp::record_error(LDPC_EINVAL, "code is NULL");
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (c->device >= 0 && c->device < kMaxDevices) ptr = g_ptr[c->device];
    }
    if (!ptr) return ndgsbp::record_error(LDPC_EHIP, "fixed scratch of the code's device was not set up");
    ndgsbp::Scratch s;
    s.work = static_cast<uint32_t*>(ptr);
    s.hbm = static_cast<unsigned char*>(ptr) + kCounterBytes;
    s.hbm_bytes = kScratchBytes - kCounterBytes;
    if (num_frames > 0 && llr && hard && iters) {
        int prev = -1;
        if (hipGetDevice(&prev) != hipSuccess) return ndgsbp::record_error(LDPC_EHIP, "cannot query the device");
        if (prev != c->device && hipSetDevice(c->device) != hipSuccess)
            return ndgsbp::record_error(LDPC_EHIP, "cannot select the code's device");
        hipLaunchKernelGGL(clear_counters, dim3(1), dim3(64), 0, (hipStream_t)hip_stream, s.work);
        const hipError_t e = hipGetLastError();
        if (prev != c->device) (void)hipSetDevice(prev);
        if (e != hipSuccess)
            return ndgsbp::record_error(LDPC_EHIP, (std::string("counter clear: ") + hipGetErrorString(e)).c_str());
    }
    return ndgsbp::decode_enqueue(c, llr, num_frames, max_iter, flags, hard, post, iters, syn_ok, &s, hip_stream);
}
