// mpx_internal.hpp -- host-side helpers shared by the libmpx translation units:
// precision decoding, argument checks and launch error mapping.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/mpx.h"

namespace mpx {

// Number of components of a precision tag, or 0 if the tag is unknown.
inline int prec_k(int prec) {
    switch (prec) {
        case MPX_DD: return 2;
        case MPX_TD: return 3;
        case MPX_QD: return 4;
        case MPX_FF: return 2;
        default: return 0;
    }
}

inline bool is_ff(int prec) { return prec == MPX_FF; }

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Map the launch status of the kernel just enqueued to an mpx status.
inline int launch_status() {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MPX_OK : MPX_EDEVICE;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace mpx

namespace mpx {
// Workspace requirements (bytes), defined next to the kernels that use them.
size_t dot_workspace(int prec, long long n);
size_t gemv_workspace(int prec, long long m, long long n, int trans);
size_t ozaki_workspace(long long m, long long n, long long k, int slices);
size_t cgemm_workspace(int prec, long long m, long long n, long long k);
}  // namespace mpx
