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

// How much of the FP64 issue rate few waves reach: NC independent chains of
// dependent additions per lane, W waves per SIMD (one workgroup of 256 W
// threads per CU), 8 steps per round.  A lone wave on one chain waits for
// each result before the next addition can issue; more chains or more waves
// fill those gaps.
template <int NC>
__global__ void __launch_bounds__(1024)
k_probe_chains(long long iters, double y0, double* __restrict__ out) {
    const double y = y0 * (double)(1 + (threadIdx.x & 1));
    double x[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) x[c] = (double)(threadIdx.x + c);
    for (long long i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int c = 0; c < NC; ++c) x[c] = x[c] + y;
    }
    double s = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) s = s + x[c];
    out[(long long)blockIdx.x * blockDim.x + threadIdx.x] = s;
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

extern "C" int64_t mpx_probe_chains_threads(int waves_per_simd) {
    if (waves_per_simd < 1 || waves_per_simd > 4) return 0;
    return mpx_probe_threads() / 8 * waves_per_simd;
}

extern "C" int mpx_probe_chains(int chains, int waves_per_simd, int64_t iters, void* out,
                                int64_t out_len, void* stream) {
    const int64_t threads = mpx_probe_chains_threads(waves_per_simd);
    if (threads <= 0 || iters < 1 || out == nullptr || out_len < threads) return MPX_EINVAL;
    if (chains != 1 && chains != 2 && chains != 4 && chains != 8 && chains != 16) return MPX_EINVAL;
    const unsigned block = 256u * (unsigned)waves_per_simd;
    const unsigned grid = (unsigned)(threads / block);
    hipStream_t s = as_stream(stream);
    double* o = (double*)out;
    switch (chains) {
        case 1: k_probe_chains<1><<<grid, block, 0, s>>>(iters, 1e-300, o); break;
        case 2: k_probe_chains<2><<<grid, block, 0, s>>>(iters, 1e-300, o); break;
        case 4: k_probe_chains<4><<<grid, block, 0, s>>>(iters, 1e-300, o); break;
        case 8: k_probe_chains<8><<<grid, block, 0, s>>>(iters, 1e-300, o); break;
        default: k_probe_chains<16><<<grid, block, 0, s>>>(iters, 1e-300, o); break;
    }
    return launch_status();
}
