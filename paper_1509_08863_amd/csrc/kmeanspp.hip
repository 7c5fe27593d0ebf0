// k-means++ seeding of the k-means step (Sec. 5 runs Matlab's k-means, whose
// default start is the D^2 draw of Arthur and Vassilvitskii: each new centre
// is a row drawn with probability proportional to its squared distance to the
// nearest centre so far).
//
// The draw is made exact: the weights are the integers
//   q_i = floor(2^30 (D_i / max_j D_j)),
// D_i the least float64 squared distance (columns in order, no fused
// multiply-add) from row i to the chosen rows, and with the caller's 53-bit
// random integer U_c the chosen row is the least i whose prefix sum of q
// exceeds floor(U_c T / 2^53), T = sum q (T = 0: row floor(U_c n / 2^53));
// the first row is floor(U_0 n / 2^53).  Integer sums do not depend on their
// order, so the blocked sums below give the same row as a sequential scan.
#include "common.hpp"

#include <algorithm>

namespace asc {
namespace {

constexpr int NT = 256;
constexpr int kBlocks = 1024;       // blocks of the weight sums
constexpr int kDistBlocks = 16384;  // blocks of the distance pass (and of its maxima)
constexpr uint64_t kUMask = (uint64_t(1) << 53) - 1;

// floor(a b / 2^53) for a < 2^53 and b < 2^63, from the 128-bit product
__device__ __forceinline__ uint64_t mulshift53(uint64_t a, uint64_t b) {
    const uint64_t lo = a * b;
    const uint64_t hi = __umul64hi(a, b);
    return (hi << 11) | (lo >> 53);
}

__device__ __forceinline__ int64_t pp_weight(double d, double dmax) {
    return dmax > 0.0 ? (int64_t)floor((d / dmax) * 1073741824.0) : 0;
}

// max of the per-block maxima, the same value in every thread of the block
__device__ double block_max(const double *__restrict__ pmax, int np) {
    __shared__ double red[NT / 64];
    __shared__ double bc;
    double m = 0.0;
    for (int b = threadIdx.x; b < np; b += NT) m = fmax(m, pmax[b]);
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0;
        for (int w = 0; w < NT / 64; ++w) x = fmax(x, red[w]);
        bc = x;
    }
    __syncthreads();
    const double r = bc;
    __syncthreads();
    return r;
}

__global__ void pp_first_kernel(const uint64_t *__restrict__ U, int64_t n, int32_t *__restrict__ rows) {
    if (threadIdx.x == 0 && blockIdx.x == 0) rows[0] = (int32_t)mulshift53(U[0] & kUMask, (uint64_t)n);
}

// D_i = d(row i, rows[c]) (c == 0) or min(D_i, d(row i, rows[c])); per-block max
__global__ __launch_bounds__(NT) void pp_dist_kernel(const float *__restrict__ F, int64_t n, int64_t r, int64_t ldf,
                                                     int vec4, const int32_t *__restrict__ rows, int c,
                                                     double *__restrict__ D, double *__restrict__ pmax) {
#pragma clang fp contract(off)
    __shared__ double red[NT / 64];
    const float *x = F + (int64_t)rows[c] * ldf;
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const float *f = F + i * ldf;
        double d = 0.0;
        if (vec4) {  // 16-byte loads, the same columns in the same order
            const float4 *f4 = reinterpret_cast<const float4 *>(f);
            const float4 *x4 = reinterpret_cast<const float4 *>(x);
            for (int64_t q = 0; q < r / 4; ++q) {
                const float4 a = f4[q], b = x4[q];
                const double d0 = (double)a.x - (double)b.x, s0 = d0 * d0;
                d = d + s0;
                const double d1 = (double)a.y - (double)b.y, s1 = d1 * d1;
                d = d + s1;
                const double d2 = (double)a.z - (double)b.z, s2 = d2 * d2;
                d = d + s2;
                const double d3 = (double)a.w - (double)b.w, s3 = d3 * d3;
                d = d + s3;
            }
        } else {
            for (int64_t col = 0; col < r; ++col) {
                const double diff = (double)f[col] - (double)x[col];
                const double sq = diff * diff;
                d = d + sq;
            }
        }
        const double v = (c == 0 || d < D[i]) ? d : D[i];
        D[i] = v;
        m = fmax(m, v);
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int w = 0; w < NT / 64; ++w) v = fmax(v, red[w]);
        pmax[blockIdx.x] = v;
    }
}

// The same pass for rows of 16-byte aligned quads (r and ldf multiples of 4):
// a wavefront takes 64 rows and brings them in through LDS, 32 columns at a
// time, with coalesced 16-byte loads (8 rows x 128 bytes per load instead of
// one 16-byte piece of 64 different rows); each lane then adds its own row's
// squared differences in column order, exactly as above.
constexpr int kPpChunk = 32;
__global__ __launch_bounds__(NT) void pp_dist_staged_kernel(const float *__restrict__ F, int64_t n, int64_t r,
                                                            int64_t ldf, const int32_t *__restrict__ rows, int c,
                                                            double *__restrict__ D, double *__restrict__ pmax) {
#pragma clang fp contract(off)
    __shared__ float Xs[NT / 64][64][kPpChunk + 1];  // +1: lane l reads row l without bank conflicts
    __shared__ double red[NT / 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const float *x = F + (int64_t)rows[c] * ldf;
    float(*S)[kPpChunk + 1] = Xs[wave];
    const int64_t ldq = ldf >> 2;
    double m = 0.0;
    for (int64_t base = ((int64_t)blockIdx.x * (NT / 64) + wave) * 64; base < n;
         base += (int64_t)gridDim.x * (NT / 64) * 64) {
        const int64_t i = base + lane;
        double d = 0.0;
        for (int64_t c0 = 0; c0 < r; c0 += kPpChunk) {
            const int w = (int)min<int64_t>(kPpChunk, r - c0);  // a multiple of 4
            const float4 *g4 = reinterpret_cast<const float4 *>(F + base * ldf + c0);
            // quad e of the chunk: row e >> 3, quad e & 7 (8 quads of a 32-column row)
            float4 v[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int e = t * 64 + lane;
                const int rl = e >> 3, cq = e & 7;
                const bool in = base + rl < n && 4 * cq < w;
                const float4 a = g4[in ? (int64_t)rl * ldq + cq : 0];
                v[t] = in ? a : float4{0.0f, 0.0f, 0.0f, 0.0f};
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int e = t * 64 + lane;
                const int rl = e >> 3, cq = e & 7;
                S[rl][4 * cq + 0] = v[t].x;
                S[rl][4 * cq + 1] = v[t].y;
                S[rl][4 * cq + 2] = v[t].z;
                S[rl][4 * cq + 3] = v[t].w;
            }
            __builtin_amdgcn_wave_barrier();
            for (int col = 0; col < w; ++col) {
                const double diff = (double)S[lane][col] - (double)x[c0 + col];
                const double sq = diff * diff;
                d = d + sq;
            }
            __builtin_amdgcn_wave_barrier();  // S is free for the next chunk
        }
        if (i < n) {
            const double v = (c == 0 || d < D[i]) ? d : D[i];
            D[i] = v;
            m = fmax(m, v);
        }
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if (lane == 0) red[wave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int w = 0; w < NT / 64; ++w) v = fmax(v, red[w]);
        pmax[blockIdx.x] = v;
    }
}

// dmax[0] = the largest of the distance pass's block maxima
__global__ __launch_bounds__(NT) void pp_max_kernel(const double *__restrict__ pmax, int np, double *__restrict__ dmax) {
    const double m = block_max(pmax, np);
    if (threadIdx.x == 0) dmax[0] = m;
}

// bsum[b] = sum of q_i over rows [b R, min(n, (b + 1) R))
__global__ __launch_bounds__(NT) void pp_wsum_kernel(const double *__restrict__ D, int64_t n, int64_t R,
                                                     const double *__restrict__ dmaxp, int64_t *__restrict__ bsum) {
    __shared__ int64_t red[NT / 64];
    const double dmax = dmaxp[0];
    const int64_t i0 = (int64_t)blockIdx.x * R, i1 = min(n, i0 + R);
    int64_t s = 0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += NT) s += pp_weight(D[i], dmax);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t v = 0;
        for (int w = 0; w < NT / 64; ++w) v += red[w];
        bsum[blockIdx.x] = v;
    }
}

// one block: the row of draw c
__global__ __launch_bounds__(NT) void pp_pick_kernel(const double *__restrict__ D, int64_t n, int64_t R, int nb,
                                                     const double *__restrict__ dmaxp,
                                                     const int64_t *__restrict__ bsum, const uint64_t *__restrict__ U,
                                                     int c, int32_t *__restrict__ rows) {
    __shared__ int64_t scan[NT];
    __shared__ int64_t sh_base;
    __shared__ int sh_block;
    __shared__ int sh_found;
    const double dmax = dmaxp[0];
    const uint64_t u = U[c] & kUMask;
    // T and the block whose prefix passes the target, by a block-wide scan:
    // thread t owns the contiguous blocks [t P, t P + P) (integer sums, so
    // the result is the sequential scan's)
    __shared__ int64_t tsum[NT];
    const int P = (nb + NT - 1) / NT;
    const int b0 = threadIdx.x * P, b1 = min(nb, b0 + P);
    int64_t own = 0;
    for (int b = b0; b < b1; ++b) own += bsum[b];
    tsum[threadIdx.x] = own;
    if (threadIdx.x == 0) {
        sh_block = -1;
        sh_found = 0;
    }
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {  // inclusive scan of the owners' sums
        const int64_t add = threadIdx.x >= off ? tsum[threadIdx.x - off] : 0;
        __syncthreads();
        tsum[threadIdx.x] += add;
        __syncthreads();
    }
    const int64_t T = tsum[NT - 1];
    if (T == 0) {
        if (threadIdx.x == 0) rows[c] = (int32_t)mulshift53(u, (uint64_t)n);
    } else {
        const int64_t target = (int64_t)mulshift53(u, (uint64_t)T);
        int64_t acc = tsum[threadIdx.x] - own;  // the sum over the blocks before b0
        if (acc <= target && target < acc + own) {
            for (int b = b0; b < b1; ++b) {
                if (acc + bsum[b] > target) {
                    sh_block = b;
                    sh_base = target - acc;  // the row is where the block's own prefix passes this
                    break;
                }
                acc += bsum[b];
            }
        }
    }
    __syncthreads();
    const int b = sh_block;
    if (b < 0) return;  // T == 0 (uniform over the block)
    int64_t rest = sh_base;
    const int64_t i0 = (int64_t)b * R, i1 = min(n, i0 + R);
    for (int64_t s = i0; s < i1; s += NT) {
        const int64_t i = s + threadIdx.x;
        scan[threadIdx.x] = i < i1 ? pp_weight(D[i], dmax) : 0;
        __syncthreads();
        for (int off = 1; off < NT; off <<= 1) {  // inclusive scan (Hillis-Steele)
            const int64_t add = threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
            __syncthreads();
            scan[threadIdx.x] += add;
            __syncthreads();
        }
        const int64_t incl = scan[threadIdx.x];
        const int64_t excl = threadIdx.x > 0 ? scan[threadIdx.x - 1] : 0;
        if (i < i1 && incl > rest && excl <= rest) {
            rows[c] = (int32_t)i;
            sh_found = 1;
        }
        const int64_t total = scan[NT - 1];
        __syncthreads();
        if (sh_found) break;
        rest -= total;
    }
}

}  // namespace
}  // namespace asc

using namespace asc;

extern "C" size_t asc_kmeanspp_workspace(int64_t n) {
    Arena a(nullptr);
    a.take<double>(n > 0 ? (size_t)n : 1);  // D
    a.take<double>(kDistBlocks);            // per-block maxima of the distance pass
    a.take<double>(1);                      // their maximum
    a.take<int64_t>(kBlocks);               // per-block weight sums
    return a.size();
}

extern "C" asc_status asc_kmeanspp(const float *F, int64_t n, int64_t r, int64_t ldf, int k, const uint64_t *U,
                                   int32_t *rows, void *ws, size_t ws_bytes, void *stream) {
    const char *who = "asc_kmeanspp";
    if (!F || n < 1 || n >= (int64_t(1) << 31) || r < 1 || r > 4096 || ldf < r || !aligned(F, 4))
        return fail(ASC_ERR_INVALID, "%s: bad features (n=%lld r=%lld ldf=%lld)", who, (long long)n, (long long)r,
                    (long long)ldf);
    if (k < 1 || k > 1024 || k > n) return fail(ASC_ERR_INVALID, "%s: k=%d not in [1, min(n, 1024)]", who, k);
    if (!U || !rows || !aligned(U, 8) || !aligned(rows, 4)) return fail(ASC_ERR_INVALID, "%s: U/rows NULL or misaligned", who);
    ASC_TRY(check_ws(ws, ws_bytes, asc_kmeanspp_workspace(n), who));
    hipStream_t s = as_stream(stream);
    Arena a(ws);
    double *D = a.take<double>((size_t)n);
    double *pmax = a.take<double>(kDistBlocks);
    double *dmax = a.take<double>(1);
    int64_t *bsum = a.take<int64_t>(kBlocks);
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kBlocks, (n + NT - 1) / NT));
    const int64_t R = (n + nb - 1) / nb;
    const int nd = (int)std::max<int64_t>(1, std::min<int64_t>(kDistBlocks, (n + NT - 1) / NT));
    const int vec4 = (r % 4 == 0 && ldf % 4 == 0 && aligned(F, 16)) ? 1 : 0;
    pp_first_kernel<<<1, 64, 0, s>>>(U, n, rows);
    ASC_LAUNCHED();
    for (int c = 0; c + 1 < k; ++c) {
        if (vec4)
            pp_dist_staged_kernel<<<nd, NT, 0, s>>>(F, n, r, ldf, rows, c, D, pmax);
        else
            pp_dist_kernel<<<nd, NT, 0, s>>>(F, n, r, ldf, vec4, rows, c, D, pmax);
        ASC_LAUNCHED();
        pp_max_kernel<<<1, NT, 0, s>>>(pmax, nd, dmax);
        ASC_LAUNCHED();
        pp_wsum_kernel<<<nb, NT, 0, s>>>(D, n, R, dmax, bsum);
        ASC_LAUNCHED();
        pp_pick_kernel<<<1, NT, 0, s>>>(D, n, R, nb, dmax, bsum, U, c + 1, rows);
        ASC_LAUNCHED();
    }
    return ASC_OK;
}
