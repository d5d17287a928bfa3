// Issue-rate probes of the gfx950 vector ALU, for the roofline of the
// decoder's VALU-bound kernel: how many lane-operations per second the chip
// retires for the instruction classes the CN rule uses (FMA, add, exp2,
// log2, reciprocal), alone and mixed. Each lane runs independent dependency
// chains so that issue, not latency, limits the rate; the result is stored
// so that no chain is removed. Built into a library of its own
// (libndgsbp_probe.so).
#include <hip/hip_runtime.h>

namespace {

// KIND 0: FMA (8 chains); 1: exp2 then log2 (8 chains, x -> x);
// 2: reciprocal (8 chains, x -> 1/x); 3: FMA (16 chains); 4: add (16 chains);
// 5: mixed, 16 FMA chains and 4 exp2/log2 chains per trip (8 transcendentals
// and 16 FMAs)
template <int KIND>
struct Shape {
    static constexpr int chains = KIND >= 3 ? 16 : 8;
    static constexpr int extra = KIND == 5 ? 4 : 0;
};

template <int KIND>
__global__ __launch_bounds__(256) void valu_probe(float* out, int iters, float seed) {
    constexpr int C = Shape<KIND>::chains, X = Shape<KIND>::extra;
    float x[C], t[X > 0 ? X : 1];
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = seed + 0.001f * (float)(threadIdx.x + c);
#pragma unroll
    for (int c = 0; c < (X > 0 ? X : 1); ++c) t[c] = 1.5f + 0.001f * (float)(threadIdx.x + c);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if constexpr (KIND == 0 || KIND == 3 || KIND == 5) {
                x[c] = __builtin_fmaf(x[c], 0.999999f, 1e-7f);
            } else if constexpr (KIND == 1) {
                x[c] = __builtin_amdgcn_logf(__builtin_amdgcn_exp2f(x[c]));
            } else if constexpr (KIND == 2) {
                x[c] = __builtin_amdgcn_rcpf(x[c]);
            } else {
                x[c] = x[c] + 1e-7f;
            }
        }
        if constexpr (X > 0) {
#pragma unroll
            for (int c = 0; c < X; ++c) t[c] = __builtin_amdgcn_logf(__builtin_amdgcn_exp2f(t[c]));
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c) s += x[c];
    if constexpr (X > 0) {
#pragma unroll
        for (int c = 0; c < X; ++c) s += t[c];
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int KIND>
double lane_ops_per_trip() {
    if constexpr (KIND == 1) return 2.0 * Shape<KIND>::chains;
    if constexpr (KIND == 5) return Shape<KIND>::chains + 2.0 * Shape<KIND>::extra;
    return Shape<KIND>::chains;
}

template <int KIND>
hipError_t launch(int blocks, int iters, float* out, double* ops) {
    hipLaunchKernelGGL(valu_probe<KIND>, dim3(blocks), dim3(256), 0, nullptr, out, iters, 1.25f);
    *ops = (double)blocks * 256.0 * (double)iters * lane_ops_per_trip<KIND>();
    return hipGetLastError();
}

}  // namespace

// Runs probe `kind` (0..5, see valu_probe) on `blocks` x 256 threads for
// `iters` loop trips; *ms is the kernel time from HIP events and *lane_ops
// the lane-operations it retired (for kind 5, FMAs plus transcendentals).
// `out` is a device buffer of blocks * 256 floats. Returns a hipError_t code.
extern "C" int ndgsbp_probe_valu(int kind, int blocks, int iters, float* out, float* ms, double* lane_ops) {
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e != hipSuccess) return (int)e;
    e = hipEventRecord(a, nullptr);
    if (e == hipSuccess) {
        switch (kind) {
            case 0: e = launch<0>(blocks, iters, out, lane_ops); break;
            case 1: e = launch<1>(blocks, iters, out, lane_ops); break;
            case 2: e = launch<2>(blocks, iters, out, lane_ops); break;
            case 3: e = launch<3>(blocks, iters, out, lane_ops); break;
            case 4: e = launch<4>(blocks, iters, out, lane_ops); break;
            case 5: e = launch<5>(blocks, iters, out, lane_ops); break;
            default: e = hipErrorInvalidValue;
        }
    }
    if (e == hipSuccess) e = hipEventRecord(b, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return (int)e;
}
