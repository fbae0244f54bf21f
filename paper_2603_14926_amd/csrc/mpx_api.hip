// mpx_api.hip -- library-wide C ABI entry points: version, status strings and
// workspace sizing.
#include "mpx_internal.hpp"

extern "C" int mpx_version(void) { return 100; }

extern "C" const char* mpx_status_string(int status) {
    switch (status) {
        case MPX_OK: return "ok";
        case MPX_EINVAL: return "invalid argument (size, stride, pointer or flag)";
        case MPX_EPREC: return "unknown or unsupported precision tag";
        case MPX_ENOTSUP: return "unsupported argument combination";
        case MPX_EWORKSPACE: return "workspace missing or too small";
        case MPX_EDEVICE: return "HIP launch or runtime error";
        default: return "unknown status";
    }
}

extern "C" size_t mpx_workspace_size(int op, int prec, int64_t m, int64_t n, int64_t k,
                                     int64_t extra) {
    using namespace mpx;
    const bool flags_ok = op == MPX_OP_DOT || op == MPX_OP_STRASSEN;
    if (flags_ok ? !prec_k_ar(prec) : (op != MPX_OP_OZAKI && !prec_k(prec))) return 0;
    if (m < 0 || n < 0 || k < 0 || extra < 0) return 0;
    switch (op) {
        case MPX_OP_DOT: return dot_workspace(prec, m);
        case MPX_OP_GEMV: return (k == 0 || k == 1) ? gemv_workspace(prec, m, n, (int)k) : 0;
        case MPX_OP_GEMM: return 0;
        case MPX_OP_OZAKI: return ozaki_workspace(m, n, k, (int)extra);
        case MPX_OP_CGEMM: return cgemm_workspace(prec, m, n, k);
        case MPX_OP_STRASSEN: return strassen_workspace(prec, m, n, k, extra);
        default: return 0;
    }
}
