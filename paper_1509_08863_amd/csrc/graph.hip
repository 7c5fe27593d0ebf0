// Graph preparation: node strengths s_i of L = S - W (Sec. 2.1) and the
// optional device-side validation of the CSR graph.
#include "common.hpp"

namespace asc {
namespace {

// one thread per row, entries summed in CSR order (float64)
__global__ void strength_kernel(int64_t n, const int32_t *__restrict__ rp, const float *__restrict__ w,
                                double *__restrict__ s) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t e0 = rp[i], e1 = rp[i + 1];
    double acc = 0.0;
    if (w) {
        for (int32_t e = e0; e < e1; ++e) acc += (double)w[e];
    } else {
        acc = (double)(e1 - e0);
    }
    s[i] = acc;
}

__device__ __forceinline__ bool bad_w(float x) { return !(x >= 0.0f) || isinf(x); }

// row i: monotone row_ptr, columns strictly increasing, in range, no self
// loop, finite non-negative weights, and W_ik == W_ki (binary search of i in
// row k).  Any violation sets bit 0 of *bad.
__global__ void validate_kernel(int64_t n, int64_t nnz, const int32_t *__restrict__ rp,
                                const int32_t *__restrict__ ci, const float *__restrict__ w,
                                uint32_t *__restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool ok = true;
    const int64_t e0 = rp[i], e1 = rp[i + 1];
    if (i == 0 && e0 != 0) ok = false;
    if (i == n - 1 && e1 != nnz) ok = false;
    if (e1 < e0 || e0 < 0 || e1 > nnz) {
        atomicOr(bad, 1u);
        return;
    }
    int32_t prev = -1;
    for (int64_t e = e0; e < e1 && ok; ++e) {
        const int32_t k = ci[e];
        if (k <= prev || k < 0 || k >= n || k == i) { ok = false; break; }
        prev = k;
        if (w && bad_w(w[e])) { ok = false; break; }
        // symmetric entry (k, i)
        int64_t lo = rp[k], hi = rp[k + 1];
        if (lo < 0 || hi > nnz || hi < lo) { ok = false; break; }
        bool found = false;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            const int32_t c = ci[mid];
            if (c == (int32_t)i) { found = true; lo = mid; break; }
            if (c < (int32_t)i) lo = mid + 1; else hi = mid;
        }
        if (!found) { ok = false; break; }
        if (w && w[lo] != w[e]) { ok = false; break; }
    }
    if (!ok) atomicOr(bad, 1u);
}

// row_ptr must be checked before the row loop reads through it
__global__ void validate_rowptr_kernel(int64_t n, int64_t nnz, const int32_t *__restrict__ rp,
                                       uint32_t *__restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const int32_t v = rp[i];
    bool ok = v >= 0 && v <= nnz;
    if (i == 0 && v != 0) ok = false;
    if (i == n && v != nnz) ok = false;
    if (i < n && rp[i + 1] < v) ok = false;
    if (!ok) atomicOr(bad, 1u);
}

__global__ void zero_u32(uint32_t *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

// normalised Laplacian (footnote of Sec. 2.1): w'_e = w_e / sqrt(s_i s_k)
// in float64 (0 where s_i or s_k is 0) and unit strengths, so that every
// kernel built on L = S - W applies L_n = I - S^{-1/2} W S^{-1/2}
__global__ void normalize_weights_kernel(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                         const float *__restrict__ w, const double *__restrict__ s,
                                         float *__restrict__ wn, double *__restrict__ ones) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double si = s[i];
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
        const double sk = s[ci[e]];
        const double we = w ? (double)w[e] : 1.0;
        wn[e] = (si > 0.0 && sk > 0.0) ? (float)(we / sqrt(si * sk)) : 0.0f;
    }
    ones[i] = 1.0;
}

}  // namespace
}  // namespace asc

using namespace asc;

extern "C" asc_status asc_graph_normalize(const asc_graph *g, float *w_out, double *strength_out, void *stream) {
    const char *who = "asc_graph_normalize";
    ASC_TRY(check_graph_args(g, true, who));
    if ((g->nnz > 0 && (!w_out || !aligned(w_out, 4))) || !strength_out || !aligned(strength_out, 8))
        return fail(ASC_ERR_INVALID, "%s: w_out or strength_out NULL or misaligned", who);
    if (static_cast<const void *>(w_out) == static_cast<const void *>(g->w) || strength_out == g->strength)
        return fail(ASC_ERR_INVALID, "%s: outputs must not alias the input graph", who);
    const int64_t n = g->n;
    normalize_weights_kernel<<<(unsigned)((n + 255) / 256), 256, 0, as_stream(stream)>>>(
        n, g->row_ptr, g->col_idx, g->w, g->strength, w_out, strength_out);
    ASC_LAUNCHED();
    return ASC_OK;
}

extern "C" size_t asc_graph_prepare_workspace(int64_t n, int validate) {
    (void)n;
    return validate ? 256 : 0;
}

extern "C" asc_status asc_graph_prepare(const asc_graph *g, double *strength, int validate, void *ws,
                                        size_t ws_bytes, void *stream) {
    ASC_TRY(check_graph_args(g, false, "asc_graph_prepare"));
    if (!strength || !aligned(strength, 8)) return fail(ASC_ERR_INVALID, "asc_graph_prepare: strength NULL/misaligned");
    hipStream_t st = as_stream(stream);
    const int64_t n = g->n;
    if (validate) {
        ASC_TRY(check_ws(ws, ws_bytes, 256, "asc_graph_prepare"));
        uint32_t *bad = static_cast<uint32_t *>(ws);
        zero_u32<<<1, 64, 0, st>>>(bad, 2);
        ASC_LAUNCHED();
        validate_rowptr_kernel<<<(unsigned)((n + 1 + 255) / 256), 256, 0, st>>>(n, g->nnz, g->row_ptr, bad);
        ASC_LAUNCHED();
        uint32_t hbad = 0;
        ASC_HIP(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, st));
        ASC_HIP(hipStreamSynchronize(st));
        if (hbad) return fail(ASC_ERR_INVALID, "asc_graph_prepare: row_ptr is not a valid CSR offset array");
        validate_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, g->nnz, g->row_ptr, g->col_idx, g->w, bad);
        ASC_LAUNCHED();
        ASC_HIP(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, st));
        ASC_HIP(hipStreamSynchronize(st));
        if (hbad)
            return fail(ASC_ERR_INVALID,
                        "asc_graph_prepare: invalid graph (unsorted/out-of-range columns, self-loop, bad weight "
                        "or W not symmetric)");
    }
    strength_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, g->row_ptr, g->w, strength);
    ASC_LAUNCHED();
    return ASC_OK;
}
