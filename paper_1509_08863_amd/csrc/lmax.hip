// Step 1 of the algorithm (Sec. 4.1): estimate of lambda_N, the largest
// eigenvalue of L = S - W, by the Lanczos iteration in float64.
//
// Iteration j (v_j = u / beta_j, u the unnormalised Lanczos vector):
//   w = L v_j - beta_j v_{j-1};  alpha_j = <w, v_j>;  u = w - alpha_j v_j;
//   beta_{j+1} = |u|; stop when j + 1 == iters or beta_{j+1} <= 1e-12 max s.
// The largest eigenvalue theta of the m x m tridiagonal (alpha, beta) is found
// by Sturm-sequence bisection; lmax = min(1.01 theta, 2 max_i s_i).
// Reductions are two-stage (per-block partials, then one block summing them
// in index order), so the result is deterministic.
#include "common.hpp"

#include <algorithm>

namespace asc {
namespace {

constexpr int NT = 256;

struct LzState {        // device-resident scalars
    double smax;
    int32_t stopped;
    int32_t m;          // size of the tridiagonal once stopped
    double pad[6];
};

constexpr int kMaxParts = 2048;

// Sum of nparts per-block partials in a fixed order (strided per thread, then
// the fixed-order block reduction); every block computes the same value.
__device__ double sum_parts(const double *__restrict__ part, int nparts, double *lds) {
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nparts; b += NT) v[0] += part[b];
    block_sum<1, NT>(v, lds);
    __shared__ double bc;
    if (threadIdx.x == 0) bc = v[0];
    __syncthreads();
    const double r = bc;
    __syncthreads();
    return r;
}

// u = v0, vprev = 0, partial |v0|^2 and max_i s_i
__global__ void lz_init_kernel(int64_t n, const double *__restrict__ v0, const double *__restrict__ s,
                               double *__restrict__ u, double *__restrict__ vprev, double *__restrict__ part,
                               double *__restrict__ partmax) {
    __shared__ double lds[NT / 64];
    double acc[1] = {0.0};
    double mx = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const double x = v0[i];
        u[i] = x;
        vprev[i] = 0.0;
        acc[0] += x * x;
        mx = fmax(mx, s[i]);
    }
    block_sum<1, NT>(acc, lds);
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    __shared__ double lmx[NT / 64];
    if ((threadIdx.x & 63) == 0) lmx[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < NT / 64; ++w) m = fmax(m, lmx[w]);
        part[blockIdx.x] = acc[0];
        partmax[blockIdx.x] = m;
    }
}

// beta_0 = |v0|, smax; then v_0 = u / beta_0 (every block recomputes beta_0)
__global__ void lz_start_kernel(int64_t n, int nparts, const double *__restrict__ part,
                                const double *__restrict__ partmax, const double *__restrict__ u,
                                double *__restrict__ vcur, double *__restrict__ beta, LzState *st) {
    __shared__ double lds[NT / 64];
    const double b = sqrt(sum_parts(part, nparts, lds));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double m = 0.0;
        for (int q = 0; q < nparts; ++q) m = fmax(m, partmax[q]);
        beta[0] = b;
        st->smax = m;
        st->stopped = (b == 0.0) ? 1 : 0;
        st->m = 0;
    }
    if (b == 0.0) return;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) vcur[i] = u[i] / b;
}

// w = L v_j - beta_j v_{j-1}, partial <w, v_j>.  Eight lanes per row split
// the row's entries; the lane partials are combined by a fixed butterfly.
__global__ void lz_spmv_kernel(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                               const float *__restrict__ wgt, const double *__restrict__ s,
                               const double *__restrict__ v, const double *__restrict__ vprev,
                               double *__restrict__ wout, const double *__restrict__ beta, int j, const LzState *st,
                               double *__restrict__ part) {
    if (st->stopped) return;
    __shared__ double lds[NT / 64];
    constexpr int LPR = 8;
    const double b = beta[j];
    const int t = threadIdx.x & (LPR - 1);
    double acc[1] = {0.0};
    const int64_t rows_per_block = NT / LPR;
    for (int64_t i0 = (int64_t)blockIdx.x * rows_per_block; i0 < n; i0 += (int64_t)gridDim.x * rows_per_block) {
        const int64_t i = i0 + threadIdx.x / LPR;
        double sum = 0.0;
        if (i < n) {
            const int32_t e1 = rp[i + 1];
            for (int32_t e = rp[i] + t; e < e1; e += LPR) sum += (wgt ? (double)wgt[e] : 1.0) * v[ci[e]];
        }
        sum += __shfl_xor(sum, 1, 64);
        sum += __shfl_xor(sum, 2, 64);
        sum += __shfl_xor(sum, 4, 64);
        if (i < n && t == 0) {
            const double vi = v[i];
            const double wi = (s[i] * vi - sum) - b * vprev[i];
            wout[i] = wi;
            acc[0] += wi * vi;
        }
    }
    block_sum<1, NT>(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// Column blocks.  A row's gathers v[k] land anywhere in the 8n-byte vector,
// which for large n is far larger than an XCD's 4 MB L2.  The columns are cut
// into B ranges of at most kBlockBytes of v (2 MB: at n = 1e6 the 60-iteration
// estimate took 19.6 ms against 26.8 ms unblocked and 23.4 ms with 4 MB ranges)
// and the product runs as B passes:
// pass b adds, for every row, the entries whose column lies in range b (a
// contiguous segment of the row, since its columns are sorted), so the
// gathered part of v stays L2-resident.  The row sum is the sum of the B
// segment sums in range order; the last pass finishes w and its partials.
constexpr int64_t kBlockBytes = int64_t(2) << 20;
constexpr int kMaxColBlocks = 16;

int col_blocks(int64_t n) {
    const int64_t b = (8 * n + kBlockBytes - 1) / kBlockBytes;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, kMaxColBlocks));
}

// off[(b - 1) n + i] = first entry of row i with column >= b * cb, b = 1..B-1
__global__ void lz_split_kernel(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, int B,
                                int64_t cb, int32_t *__restrict__ off) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const int32_t r0 = rp[i], r1 = rp[i + 1];
        for (int b = 1; b < B; ++b) {
            const int64_t c = (int64_t)b * cb;
            int32_t lo = r0, hi = r1;  // first e in [r0, r1) with ci[e] >= c
            while (lo < hi) {
                const int32_t mid = lo + (hi - lo) / 2;
                if (ci[mid] < c) lo = mid + 1; else hi = mid;
            }
            off[(int64_t)(b - 1) * n + i] = lo;
        }
    }
}

// pass b of w = L v_j - beta_j v_{j-1}: the segment sums of column range b
// are added to the running row sums in w; the last pass forms w and the
// partial <w, v_j> as lz_spmv_kernel does.  Unit weights (w = NULL) and
// stored weights are separate instantiations, so a lane's index and weight
// loads go out together instead of the weight load waiting behind a branch.
template <bool LAST, bool WEIGHTED>
__global__ void lz_spmv_block_kernel(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                     const float *__restrict__ wgt, const int32_t *__restrict__ off, int B, int b,
                                     const double *__restrict__ s, const double *__restrict__ v,
                                     const double *__restrict__ vprev, double *__restrict__ wout,
                                     const double *__restrict__ beta, int j, const LzState *st,
                                     double *__restrict__ part) {
    if (st->stopped) return;
    __shared__ double lds[NT / 64];
    constexpr int LPR = 8;
    const int t = threadIdx.x & (LPR - 1);
    double acc[1] = {0.0};
    const int64_t rows_per_block = NT / LPR;
    for (int64_t i0 = (int64_t)blockIdx.x * rows_per_block; i0 < n; i0 += (int64_t)gridDim.x * rows_per_block) {
        const int64_t i = i0 + threadIdx.x / LPR;
        double sum = 0.0;
        if (i < n) {
            const int32_t e0 = b == 0 ? rp[i] : off[(int64_t)(b - 1) * n + i];
            const int32_t e1 = b == B - 1 ? rp[i + 1] : off[(int64_t)b * n + i];
            for (int32_t e = e0 + t; e < e1; e += LPR) sum += (WEIGHTED ? (double)wgt[e] : 1.0) * v[ci[e]];
        }
        sum += __shfl_xor(sum, 1, 64);
        sum += __shfl_xor(sum, 2, 64);
        sum += __shfl_xor(sum, 4, 64);
        if (i < n && t == 0) {
            const double row = b == 0 ? sum : wout[i] + sum;
            if (LAST) {
                const double vi = v[i];
                const double wi = (s[i] * vi - row) - beta[j] * vprev[i];
                wout[i] = wi;
                acc[0] += wi * vi;
            } else {
                wout[i] = row;
            }
        }
    }
    if (LAST) {
        block_sum<1, NT>(acc, lds);
        if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
    }
}

// alpha_j = <w, v_j>; u = w - alpha_j v_j; partial |u|^2
__global__ void lz_axpy_kernel(int64_t n, int nparts_in, const double *__restrict__ part_in,
                               const double *__restrict__ wv, const double *__restrict__ vcur, double *__restrict__ u,
                               double *__restrict__ alpha, int j, const LzState *st, double *__restrict__ part) {
    if (st->stopped) return;
    __shared__ double lds[NT / 64];
    const double a = sum_parts(part_in, nparts_in, lds);
    if (blockIdx.x == 0 && threadIdx.x == 0) alpha[j] = a;
    double acc[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const double x = wv[i] - a * vcur[i];
        u[i] = x;
        acc[0] += x * x;
    }
    block_sum<1, NT>(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// beta_{j+1} = |u|; stop on the last iteration or on breakdown; else
// v_{j+1} = u / beta_{j+1}
__global__ void lz_scale_kernel(int64_t n, int nparts, const double *__restrict__ part, const double *__restrict__ u,
                                double *__restrict__ vnext, double *__restrict__ beta, int j, int iters,
                                LzState *st) {
    if (st->stopped) return;
    __shared__ double lds[NT / 64];
    const double bn = sqrt(sum_parts(part, nparts, lds));
    const bool stop = (j + 1 == iters) || bn <= 1e-12 * st->smax;
    __syncthreads();  // every thread has read st->stopped / smax before block 0 updates them
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        beta[j + 1] = bn;
        if (stop) {
            st->stopped = 1;
            st->m = j + 1;
        }
    }
    if (stop) return;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) vnext[i] = u[i] / bn;
}

// number of eigenvalues of the tridiagonal strictly below x (Sturm sequence)
__device__ int sturm_below(const double *a, const double *b, int m, double x) {
    int cnt = 0;
    double q = a[0] - x;
    if (q < 0) ++cnt;
    for (int i = 1; i < m; ++i) {
        const double qq = (q == 0.0) ? 1e-300 : q;
        q = a[i] - x - b[i] * b[i] / qq;
        if (q < 0) ++cnt;
    }
    return cnt;
}

// largest eigenvalue of T = tridiag(beta[1..m-1], alpha[0..m-1], beta[1..m-1])
__global__ void lz_tridiag_kernel(const double *__restrict__ alpha, const double *__restrict__ beta,
                                  const LzState *st, double *__restrict__ lmax) {
    if (threadIdx.x != 0) return;
    const int m = st->m;
    const double smax = st->smax;
    if (m <= 0) {  // zero start vector or no iteration: fall back to the Gershgorin bound
        lmax[0] = 2.0 * smax;
        return;
    }
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? fabs(beta[i]) : 0.0) + (i + 1 < m ? fabs(beta[i + 1]) : 0.0);
        lo = fmin(lo, alpha[i] - r);
        hi = fmax(hi, alpha[i] + r);
    }
    // largest eigenvalue theta: sturm_below(x) == m  <=>  x > theta
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_below(alpha, beta, m, mid) == m) hi = mid; else lo = mid;
    }
    const double theta = hi;
    lmax[0] = fmin(1.01 * theta, 2.0 * smax);
}

int nblocks_for(int64_t n) {
    int64_t b = (n + NT - 1) / NT;
    if (b > kMaxParts) b = kMaxParts;
    if (b < 1) b = 1;
    return (int)b;
}

}  // namespace
}  // namespace asc

using namespace asc;

extern "C" size_t asc_lmax_workspace(int64_t n, int iters) {
    Arena a(nullptr);
    a.take<WsHeader>(1);
    a.take<LzState>(1);
    for (int q = 0; q < 5; ++q) a.take<double>((size_t)n);  // u, vA, vB, w, (spare)
    a.take<double>((size_t)iters + 2);                    // alpha
    a.take<double>((size_t)iters + 2);                    // beta
    a.take<double>(kMaxParts);                            // partials
    a.take<double>(kMaxParts);
    const int B = col_blocks(n);
    if (B > 1) a.take<int32_t>((size_t)(B - 1) * n);      // column-range offsets per row
    return a.size();
}

extern "C" asc_status asc_lmax_estimate(const asc_graph *g, const double *v0, int iters, double *lmax,
                                        double *lmax_host, void *ws, size_t ws_bytes, void *stream) {
    const char *who = "asc_lmax_estimate";
    ASC_TRY(check_graph_args(g, true, who));
    if (!v0 || !lmax || !aligned(v0, 8) || !aligned(lmax, 8)) return fail(ASC_ERR_INVALID, "%s: v0/lmax NULL or misaligned", who);
    if (iters < 1 || iters > 4096) return fail(ASC_ERR_INVALID, "%s: iters=%d not in [1, 4096]", who, iters);
    const int64_t n = g->n;
    ASC_TRY(check_ws(ws, ws_bytes, asc_lmax_workspace(n, iters), who));
    Arena a(ws);
    a.take<WsHeader>(1);
    LzState *st = a.take<LzState>(1);
    double *u = a.take<double>(n);
    double *vA = a.take<double>(n);
    double *vB = a.take<double>(n);
    double *wv = a.take<double>(n);
    a.take<double>(n);
    double *alpha = a.take<double>(iters + 2);
    double *beta = a.take<double>(iters + 2);
    double *part = a.take<double>(kMaxParts);
    double *partmax = a.take<double>(kMaxParts);
    const int B = col_blocks(n);
    const int64_t cb = (n + B - 1) / B;
    int32_t *off = B > 1 ? a.take<int32_t>((size_t)(B - 1) * n) : nullptr;
    hipStream_t s = as_stream(stream);
    const int nb = nblocks_for(n);
    const int nbs = (int)std::max<int64_t>(1, std::min<int64_t>((n + NT / 8 - 1) / (NT / 8), kMaxParts));
    lz_init_kernel<<<nb, NT, 0, s>>>(n, v0, g->strength, u, vB, part, partmax);
    ASC_LAUNCHED();
    lz_start_kernel<<<nb, NT, 0, s>>>(n, nb, part, partmax, u, vA, beta, st);
    ASC_LAUNCHED();
    if (B > 1) {
        lz_split_kernel<<<nb, NT, 0, s>>>(n, g->row_ptr, g->col_idx, B, cb, off);
        ASC_LAUNCHED();
    }
    double *vcur = vA, *vprev = vB;
    for (int j = 0; j < iters; ++j) {
        if (B == 1) {
            lz_spmv_kernel<<<nbs, NT, 0, s>>>(n, g->row_ptr, g->col_idx, g->w, g->strength, vcur, vprev, wv, beta, j,
                                              st, part);
        } else {
            // unit weights (w = NULL) and stored weights take separate
            // kernels, so no weight load sits behind a branch
            for (int b = 0; b < B; ++b) {
                const bool last = b == B - 1;
                if (g->w) {
                    if (last)
                        lz_spmv_block_kernel<true, true><<<nbs, NT, 0, s>>>(n, g->row_ptr, g->col_idx, g->w, off, B,
                                                                            b, g->strength, vcur, vprev, wv, beta, j,
                                                                            st, part);
                    else
                        lz_spmv_block_kernel<false, true><<<nbs, NT, 0, s>>>(n, g->row_ptr, g->col_idx, g->w, off, B,
                                                                             b, g->strength, vcur, vprev, wv, beta, j,
                                                                             st, part);
                } else {
                    if (last)
                        lz_spmv_block_kernel<true, false><<<nbs, NT, 0, s>>>(n, g->row_ptr, g->col_idx, g->w, off,
                                                                             B, b, g->strength, vcur, vprev, wv, beta,
                                                                             j, st, part);
                    else
                        lz_spmv_block_kernel<false, false><<<nbs, NT, 0, s>>>(n, g->row_ptr, g->col_idx, g->w, off,
                                                                              B, b, g->strength, vcur, vprev, wv,
                                                                              beta, j, st, part);
                }
            }
        }
        ASC_LAUNCHED();
        lz_axpy_kernel<<<nb, NT, 0, s>>>(n, nbs, part, wv, vcur, u, alpha, j, st, partmax);
        ASC_LAUNCHED();
        // v_{j+1} overwrites v_{j-1}
        lz_scale_kernel<<<nb, NT, 0, s>>>(n, nb, partmax, u, vprev, beta, j, iters, st);
        ASC_LAUNCHED();
        double *t = vprev;
        vprev = vcur;
        vcur = t;
    }
    lz_tridiag_kernel<<<1, 64, 0, s>>>(alpha, beta, st, lmax);
    ASC_LAUNCHED();
    if (lmax_host) {
        ASC_HIP(hipMemcpyAsync(lmax_host, lmax, sizeof(double), hipMemcpyDeviceToHost, s));
        ASC_HIP(hipStreamSynchronize(s));
    }
    return ASC_OK;
}
