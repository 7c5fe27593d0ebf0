// Error reporting, argument validation and the small utility entry points.
#include "common.hpp"

#include <algorithm>

namespace asc {

std::string &last_error_ref() {
    static thread_local std::string s;
    return s;
}

asc_status fail(asc_status st, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    last_error_ref() = buf;
    return st;
}

asc_status check_ws(const void *ws, size_t ws_bytes, size_t need, const char *who) {
    if (need == 0) return ASC_OK;
    if (ws == nullptr) return fail(ASC_ERR_WORKSPACE, "%s: workspace is NULL (need %zu bytes)", who, need);
    if (!aligned(ws, 256)) return fail(ASC_ERR_WORKSPACE, "%s: workspace not 256-byte aligned", who);
    if (ws_bytes < need)
        return fail(ASC_ERR_WORKSPACE, "%s: workspace has %zu bytes, need %zu", who, ws_bytes, need);
    return ASC_OK;
}

asc_status check_graph_args(const asc_graph *g, bool need_strength, const char *who) {
    if (!g) return fail(ASC_ERR_INVALID, "%s: graph is NULL", who);
    if (g->n < 1 || g->n >= (int64_t(1) << 31)) return fail(ASC_ERR_INVALID, "%s: n=%lld out of range", who, (long long)g->n);
    if (g->nnz < 0 || g->nnz >= (int64_t(1) << 31))
        return fail(ASC_ERR_INVALID, "%s: nnz=%lld out of range", who, (long long)g->nnz);
    if (!g->row_ptr) return fail(ASC_ERR_INVALID, "%s: row_ptr is NULL", who);
    if (g->nnz > 0 && !g->col_idx) return fail(ASC_ERR_INVALID, "%s: col_idx is NULL", who);
    if (!aligned(g->row_ptr, 4) || (g->col_idx && !aligned(g->col_idx, 4)) || (g->w && !aligned(g->w, 4)))
        return fail(ASC_ERR_INVALID, "%s: graph arrays must be 4-byte aligned", who);
    if (need_strength && !g->strength)
        return fail(ASC_ERR_INVALID, "%s: graph strength is NULL (call asc_graph_prepare)", who);
    if (need_strength && !aligned(g->strength, 8)) return fail(ASC_ERR_INVALID, "%s: strength misaligned", who);
    return ASC_OK;
}

asc_status check_block(const void *p, asc_dtype dt, int64_t n, int64_t r, int64_t ld, const char *who,
                       const char *name) {
    if (dt != ASC_F32 && dt != ASC_BF16) return fail(ASC_ERR_INVALID, "%s: unknown dtype %d", who, (int)dt);
    if (!p) return fail(ASC_ERR_INVALID, "%s: %s is NULL", who, name);
    if (r < 1 || r > 65536) return fail(ASC_ERR_INVALID, "%s: %s has r=%lld (1..65536)", who, name, (long long)r);
    if (ld < r) return fail(ASC_ERR_INVALID, "%s: %s leading dimension %lld < r=%lld", who, name, (long long)ld, (long long)r);
    const int64_t q = dt == ASC_F32 ? 4 : 8;
    if (ld % q) return fail(ASC_ERR_INVALID, "%s: %s leading dimension must be a multiple of %lld", who, name, (long long)q);
    if (!aligned(p, 16)) return fail(ASC_ERR_INVALID, "%s: %s must be 16-byte aligned", who, name);
    (void)n;
    return ASC_OK;
}

}  // namespace asc

using namespace asc;

extern "C" int asc_abi_version(void) { return ASC_ABI_VERSION; }

extern "C" const char *asc_last_error(void) { return last_error_ref().c_str(); }

extern "C" asc_status asc_read_flags(const void *ws, uint32_t *flags_host, void *stream) {
    if (!ws || !aligned(ws, 256)) return fail(ASC_ERR_WORKSPACE, "asc_read_flags: bad workspace");
    uint32_t f = 0;
    ASC_HIP(hipMemcpyAsync(&f, ws, sizeof f, hipMemcpyDeviceToHost, as_stream(stream)));
    ASC_HIP(hipStreamSynchronize(as_stream(stream)));
    if (flags_host) *flags_host = f;
    if (f & ASC_FLAG_NONFINITE) return fail(ASC_ERR_NONFINITE, "non-finite value in a filtered block");
    if (f & ASC_FLAG_GROWTH)
        return fail(ASC_ERR_LMAX_TOO_SMALL, "recurrence grew: |T_p R| > 1.5 |R|, lambda_max is below lambda_N");
    return ASC_OK;
}

// plain streaming copy (16-byte vectors), the reference kernel for bandwidth
// and memory-counter calibration
namespace {
// Four 16-byte vectors in flight per lane (all loads before the stores) and
// non-temporal hints: the fastest of the plain copies measured on this device
// (about 5.1 TB/s for 2 GiB, 5.3 TB/s for 4 GiB, against 4.6-4.8 TB/s for one
// vector per lane and iteration).
typedef unsigned cp4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void stream_copy_kernel(const cp4 *__restrict__ src, cp4 *__restrict__ dst,
                                                          int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        cp4 a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = __builtin_nontemporal_load(src + i + q * stride);
#pragma unroll
        for (int q = 0; q < 4; ++q) __builtin_nontemporal_store(a[q], dst + i + q * stride);
    }
    for (; i < n16; i += stride) dst[i] = src[i];
}
// rows idx[e] of a table of 128-byte rows: 8 lanes per row (16 bytes each),
// 8 rows in flight per lane group, grid-stride over the index list; indices
// are clamped into the table; a lane writes its sum to sink[0] only when it
// equals a fixed sentinel, which keeps the loads live
__global__ __launch_bounds__(256) void gather_probe_kernel(const float4 *__restrict__ table, int64_t rows,
                                                           const int32_t *__restrict__ idx, int64_t nidx,
                                                           float *__restrict__ sink) {
    constexpr int LPR = 8, U = 8;
    const int t = threadIdx.x % LPR;
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / LPR;
    const int64_t ngrp = (int64_t)gridDim.x * blockDim.x / LPR;
    float a = 0.0f, b = 0.0f, c = 0.0f, d = 0.0f;
    for (int64_t e = grp * U; e < nidx; e += ngrp * U) {
        int64_t k[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t kk = e + u < nidx ? (int64_t)idx[e + u] : 0;
            k[u] = kk < 0 ? 0 : (kk >= rows ? rows - 1 : kk);
        }
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = table[k[u] * LPR + t];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a += v[u].x;
            b += v[u].y;
            c += v[u].z;
            d += v[u].w;
        }
    }
    const float s = a + b + c + d;
    if (s == 1.2345678e7f) sink[0] = s;
}
}  // namespace

extern "C" asc_status asc_gather_probe(const float *table, int64_t rows, const int32_t *idx, int64_t nidx,
                                       float *sink, void *stream) {
    if (!table || !idx || !sink || rows < 1 || nidx < 0 || !aligned(table, 16) || !aligned(idx, 4))
        return fail(ASC_ERR_INVALID, "asc_gather_probe: NULL or misaligned pointer, or rows < 1");
    if (nidx == 0) return ASC_OK;
    const int64_t groups = (nidx + 7) / 8;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((groups * 8 + 255) / 256, 256 * 32));
    gather_probe_kernel<<<grid, 256, 0, as_stream(stream)>>>(reinterpret_cast<const float4 *>(table), rows, idx,
                                                              nidx, sink);
    ASC_LAUNCHED();
    return ASC_OK;
}

extern "C" asc_status asc_stream_copy(const void *src, void *dst, size_t bytes, void *stream) {
    if (!src || !dst || bytes % 16 || !aligned(src, 16) || !aligned(dst, 16))
        return fail(ASC_ERR_INVALID, "asc_stream_copy: pointers must be 16-byte aligned and bytes a multiple of 16");
    const int64_t n16 = (int64_t)(bytes / 16);
    const int grid = (int)std::min<int64_t>((n16 + 255) / 256, 65536);
    if (n16 == 0) return ASC_OK;
    stream_copy_kernel<<<grid, 256, 0, as_stream(stream)>>>(static_cast<const cp4 *>(src), static_cast<cp4 *>(dst), n16);
    ASC_LAUNCHED();
    return ASC_OK;
}
