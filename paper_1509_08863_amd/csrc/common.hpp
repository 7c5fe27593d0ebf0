// Internal helpers shared by the HIP translation units of libasc (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "asc.h"

namespace asc {

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
std::string &last_error_ref();
asc_status fail(asc_status st, const char *fmt, ...);

#define ASC_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::asc::fail(ASC_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define ASC_LAUNCHED()                                                                  \
    do {                                                                                \
        hipError_t e_ = hipGetLastError();                                              \
        if (e_ != hipSuccess)                                                           \
            return ::asc::fail(ASC_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)

#define ASC_TRY(expr)                          \
    do {                                       \
        asc_status s_ = (expr);                \
        if (s_ != ASC_OK) return s_;           \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// ---------------------------------------------------------------------------
// workspace carving: a bump allocator over the caller's buffer.  Run once
// with base == nullptr to size it.
// ---------------------------------------------------------------------------
struct Arena {
    char *base;
    size_t off = 0;
    explicit Arena(void *b) : base(static_cast<char *>(b)) {}
    template <typename T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += sizeof(T) * count;
        return p;
    }
    size_t size() const { return (off + 255) & ~size_t(255); }
};

asc_status check_ws(const void *ws, size_t ws_bytes, size_t need, const char *who);
asc_status check_graph_args(const asc_graph *g, bool need_strength, const char *who);
asc_status check_block(const void *p, asc_dtype dt, int64_t n, int64_t r, int64_t ld, const char *who,
                       const char *name);

// Every workspace starts with this header (flags raised by kernels).
struct WsHeader {
    uint32_t flags;
    uint32_t pad[63];
};

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block reduction of NV doubles (fixed lane and wave order).
// All threads of the block must call it; result valid in thread 0.
template <int NV, int NT>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds /* NV * NT/64 */) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) lds[q * NW + wave] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = 0.0;
            for (int w = 0; w < NW; ++w) s += lds[q * NW + w];
            v[q] = s;
        }
    }
    __syncthreads();
}

// bfloat16 <-> float32 (round to nearest even; NaN kept quiet)
__device__ __forceinline__ float bf16_lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t u) { return __uint_as_float(u & 0xffff0000u); }
__device__ __forceinline__ uint32_t f32_to_bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
    return f32_to_bf16_bits(lo) | (f32_to_bf16_bits(hi) << 16);
}

}  // namespace asc
