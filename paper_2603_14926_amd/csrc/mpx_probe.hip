// mpx_probe.hip -- measurement aid: the VALU issue rate of the instruction
// kinds the multicomponent kernels are made of, used to check the FP64 / FP32
// vector peaks the rooflines are quoted against.
//
// Every thread runs 16 independent dependency chains x_c := x_c + y (or
// x_c := fma(x_c, y, z)), 4 steps each per round (64 operations per loop
// iteration, so the loop control is negligible), for `iters` rounds; y and z
// are per-lane values derived from the arguments, so the compiler can neither
// fold nor reassociate them (no fast-math), and the final sums are stored so
// nothing is dead.  The grid is
// 8 workgroups of 256 threads per CU.  Lane-operations = threads x iters x 64.
#include "mpx_internal.hpp"

#include "../../include/mpx_probe.h"

#pragma clang fp contract(off)

namespace mpx {

template <typename T, bool FMA>
__global__ void __launch_bounds__(256)
k_probe_valu(long long iters, T y0, T z0, T* __restrict__ out) {
    // per-lane operands (vector registers, as in the arithmetic kernels)
    const T y = y0 * (T)(1 + (threadIdx.x & 1)), z = z0 * (T)(1 + (threadIdx.x & 2));
    constexpr int NC = 16;
    T x[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) x[c] = (T)(threadIdx.x + c);
    for (long long i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if constexpr (FMA && sizeof(T) == 4) x[c] = __builtin_fmaf(x[c], y, z);
                else if constexpr (FMA) x[c] = __builtin_fma(x[c], y, z);
                else x[c] = x[c] + y;
            }
    }
    T s = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) s = s + x[c];
    out[(long long)blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace mpx

using namespace mpx;

extern "C" int64_t mpx_probe_threads(void) {
    int dev = 0, cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        cus = prop.multiProcessorCount;
    return (int64_t)cus * 8 * 256;
}

extern "C" int mpx_probe_valu(int kind, int64_t iters, void* out, int64_t threads, void* stream) {
    if (kind < 0 || kind > 3 || iters < 1 || threads < 256 || threads % 256 || out == nullptr)
        return MPX_EINVAL;
    const unsigned grid = (unsigned)(threads / 256);
    hipStream_t s = as_stream(stream);
    switch (kind) {
        case MPX_PROBE_F64_ADD: k_probe_valu<double, false><<<grid, 256, 0, s>>>(iters, 1e-300, 0.0, (double*)out); break;
        case MPX_PROBE_F64_FMA: k_probe_valu<double, true><<<grid, 256, 0, s>>>(iters, 1.0, 1e-300, (double*)out); break;
        case MPX_PROBE_F32_ADD: k_probe_valu<float, false><<<grid, 256, 0, s>>>(iters, 1e-30f, 0.0f, (float*)out); break;
        default: k_probe_valu<float, true><<<grid, 256, 0, s>>>(iters, 1.0f, 1e-30f, (float*)out); break;
    }
    return launch_status();
}
