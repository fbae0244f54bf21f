// mpx_internal.hpp -- host-side helpers shared by the libmpx translation units:
// precision decoding, argument checks and launch error mapping.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

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

// Precision tag with the arithmetic flags removed, and the flag as the
// kernels' selector (0 branch-free, 1 conventional, 2 conventional with the
// accurate DD addition).
inline int base_prec(int prec) { return prec & ~(MPX_NOBF | MPX_NOBF_ACC); }
inline int arith_of(int prec) {
    return (prec & MPX_NOBF_ACC) ? 2 : (prec & MPX_NOBF) ? 1 : 0;
}

// K of a tag that may carry an arithmetic flag, or 0 when the combination
// does not exist (flags on FF, both flags, the accurate addition beyond DD).
inline int prec_k_ar(int prec) {
    const int fl = prec & (MPX_NOBF | MPX_NOBF_ACC), b = base_prec(prec);
    if (fl == 0) return prec_k(b);
    if (fl == (MPX_NOBF | MPX_NOBF_ACC) || b == MPX_FF) return 0;
    if (fl == MPX_NOBF_ACC && b != MPX_DD) return 0;
    return prec_k(b);
}

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Map the launch status of the kernel just enqueued to an mpx status.
inline int launch_status() {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MPX_OK : MPX_EDEVICE;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Does a row-major rows x cols block with leading dimension ld fit in a
// plane of ps elements, i.e. ld >= cols and (rows - 1) ld + cols <= ps?
// Evaluated without signed overflow (a span beyond int64 does not fit).
// rows, cols >= 1.
inline bool span_fits(int64_t rows, int64_t cols, int64_t ld, int64_t ps) {
    if (ld < cols) return false;
    if (rows > 1 && ld > (INT64_MAX - cols) / (rows - 1)) return false;
    return (rows - 1) * ld + cols <= ps;
}
// a * b <= ps for a, b >= 0, without signed overflow.
inline bool prod_fits(int64_t a, int64_t b, int64_t ps) {
    return b == 0 || a <= ps / b;
}

// Bytes spanned by K component planes of a rows x cols row-major block
// (plane stride ps, leading dimension ld, elements of elt bytes), computed
// in 128 bits and saturated; 0 for an empty block.
inline uint64_t planes_bytes(int K, int64_t rows, int64_t cols, int64_t ld, int64_t ps, size_t elt) {
    if (rows <= 0 || cols <= 0) return 0;
    const unsigned __int128 e = (unsigned __int128)(K - 1) * (uint64_t)ps +
                                (unsigned __int128)(rows - 1) * (uint64_t)ld + (uint64_t)cols;
    const unsigned __int128 b = e * elt;
    return b > (unsigned __int128)UINT64_MAX ? UINT64_MAX : (uint64_t)b;
}
// Do the byte ranges [a, a + na) and [b, b + nb) intersect?
inline bool overlaps(const void* a, uint64_t na, const void* b, uint64_t nb) {
    if (na == 0 || nb == 0 || a == nullptr || b == nullptr) return false;
    const unsigned __int128 a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

// Two HIP events bracketing timed work on a stream (the autotuners); both are
// destroyed on scope exit.  Every step reports failure instead of ignoring it.
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    bool ok = false;
    EventPair() { ok = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess; }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    EventPair(const EventPair&) = delete;
    EventPair& operator=(const EventPair&) = delete;
    bool start(hipStream_t s) { return hipEventRecord(a, s) == hipSuccess; }
    bool stop(hipStream_t s) { return hipEventRecord(b, s) == hipSuccess; }
    // Waits for the stop event; milliseconds between the two.
    bool elapsed(float* ms) {
        return hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(ms, a, b) == hipSuccess;
    }
};

// The engine clock ramps up over tens of milliseconds of sustained work (a
// DD GEMM of about a millisecond runs up to 25 % slower in its first calls
// after an idle spell than after thirty calls in a row), so an autotuner
// first runs the operation for about kTuneWarmMs of GPU time (at most
// kTuneWarmCalls calls) and only then times the candidates; otherwise the
// first candidates are timed at a lower clock than the last.
constexpr float kTuneWarmMs = 100.f;
constexpr int kTuneWarmCalls = 4096;
template <typename F>
int warm_clock(EventPair& ev, hipStream_t s, F run_once) {
    float total = 0.f;
    for (int calls = 0; total < kTuneWarmMs && calls < kTuneWarmCalls; ++calls) {
        if (!ev.start(s)) return MPX_EDEVICE;
        if (int st = run_once()) return st;
        float ms = 0.f;
        if (!ev.stop(s) || !ev.elapsed(&ms)) return MPX_EDEVICE;
        total += ms;
    }
    return MPX_OK;
}

}  // namespace mpx

namespace mpx {
// Workspace requirements (bytes), defined next to the kernels that use them.
size_t dot_workspace(int prec, long long n);
size_t gemv_workspace(int prec, long long m, long long n, int trans);
size_t ozaki_workspace(long long m, long long n, long long k, int slices);
size_t cgemm_workspace(int prec, long long m, long long n, long long k);
size_t strassen_workspace(int prec, long long m, long long n, long long k, long long cutoff);

// Tuned launch choices (mpx_tune.hip): in-process, and in the MPX_TUNE_CACHE
// file when that is set.  Keys are "<op> <fields...>", choices one word.
bool tune_disabled();
bool tune_lookup(const std::string& op_key, std::string& choice);
void tune_store(const std::string& op_key, const std::string& choice);
void tune_forget(const std::string& op);
}  // namespace mpx
