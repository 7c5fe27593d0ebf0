// K-nearest-neighbour similarity graph (Sec. 5: K ~ log N nearest
// neighbours, union-symmetrised), built on the device from the points.
//
// The all-pairs distance work is a dense contraction: |x_i - x_j|^2 =
// |x_i|^2 + |x_j|^2 - 2 x_i . x_j, with the dot products on the matrix cores
// (v_mfma_f32_16x16x4f32: a wavefront computes a 16 x 16 tile of dot products
// in d/4 instructions).  That float32 form only proposes candidates; the
// neighbours themselves are decided on exact float64 distances, so the result
// is the exact K-nearest set with ties to the lower index:
//   A. per (query, lane class) the H = 10 nearest by the float32 form (4
//      classes: 40 candidates per query);
//   B. one wavefront per row recomputes the 40 candidates in float64 and keeps
//      the K least (distance, index).  The row is certified when its K-th
//      exact distance is below cut - e, where cut is the least of the 4
//      classes' H-th proposals (no point left out can be nearer than cut - e)
//      and e bounds the float32 error of the proposals;
//   C. rows that fail (rare) are redone by a float64 scan over all points;
//   D. the union graph: reverse lists, per-row merge of sorted lists, offsets
//      by prefix sums, columns and float64 distances (stored as float32).
#include "common.hpp"

#include <algorithm>
#include <climits>

namespace asc {
namespace {

constexpr int NT = 256;
constexpr int H = 10;           // proposals kept per (query, lane class)
constexpr int NCLASS = 4;       // lane classes per query (candidate rows 4c..4c+3 of every tile)
constexpr int NCAND = NCLASS * H;  // proposals per query
static_assert(NCAND <= 64, "one proposal per lane in the exact selection");
constexpr int QW = 32;          // query rows per wavefront (two 16-row tiles)
constexpr int QB = 4 * QW;      // query rows per block
constexpr int kMaxK = 32;
constexpr int kMaxD = 64;
constexpr int kFallbackBlocks = 64;  // at most; fewer when n is large (scratch <= 1 GiB)
constexpr int kScanTile = 2048;

typedef float v4f __attribute__((ext_vector_type(4)));

struct KnnWs {
    WsHeader *hdr;
    float *nrm;          // |x_i|^2 (float32)
    uint32_t *nmax;      // max |x|^2 as float bits
    uint32_t *nflag;     // rows that needed the float64 scan
    int32_t *flag_list;  // [n]
    float *cand_d;       // [n][NCAND]
    int32_t *cand_j;     // [n][NCAND]
    double *scratch;     // [fallback_blocks(n)][n]
    int32_t *cnt;        // [n] reverse-list lengths, then cursors
    int64_t *rev_off;    // [n + 1]
    int32_t *rev;        // [n k]
    int64_t *len;        // [n] union row lengths
    int64_t *tile_sums;  // [tiles + 1]
};

int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

// blocks of the float64 fallback scan, each with an n-long scratch row
int fallback_blocks(int64_t n) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(kFallbackBlocks, (int64_t(1) << 30) / (8 * n)));
}

size_t knn_ws_layout(int64_t n, int k, void *ws, KnnWs *out) {
    Arena a(ws);
    KnnWs w;
    w.hdr = a.take<WsHeader>(1);
    w.nrm = a.take<float>(n);
    w.nmax = a.take<uint32_t>(64);
    w.nflag = a.take<uint32_t>(64);
    w.flag_list = a.take<int32_t>(n);
    w.cand_d = a.take<float>((size_t)n * NCAND);
    w.cand_j = a.take<int32_t>((size_t)n * NCAND);
    w.scratch = a.take<double>((size_t)fallback_blocks(n) * n);
    w.cnt = a.take<int32_t>(n);
    w.rev_off = a.take<int64_t>(n + 1);
    w.rev = a.take<int32_t>((size_t)n * k);
    w.len = a.take<int64_t>(n);
    w.tile_sums = a.take<int64_t>(scan_tiles(n + 1) + 1);
    if (out) *out = w;
    return a.size();
}

__global__ void knn_clear_kernel(uint32_t *nmax, uint32_t *nflag, int32_t *cnt, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        nmax[0] = 0u;
        nflag[0] = 0u;
    }
    for (int64_t i = t; i < n; i += (int64_t)gridDim.x * blockDim.x) cnt[i] = 0;
}

__global__ void zero_i32_kernel(int32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

// |x_i|^2 in float32 (coordinates in order) and the largest of them
__global__ void sqnorm_kernel(const float *__restrict__ X, int64_t n, int d, int64_t ldx, float *__restrict__ nrm,
                              uint32_t *__restrict__ nmax) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float s = 0.0f;
    if (i < n) {
        const float *x = X + i * ldx;
        for (int c = 0; c < d; ++c) s += x[c] * x[c];
        nrm[i] = s;
        if (!(s < __builtin_inff())) s = 0.0f;  // a non-finite point does not loosen the other rows' bound
    }
    for (int off = 32; off > 0; off >>= 1) s = fmaxf(s, __shfl_xor(s, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(nmax, __float_as_uint(s));  // non-negative floats order as integers
}

__device__ __forceinline__ void propose(float (&hd)[H], int (&hj)[H], float dv, int j) {
    if (!(dv < hd[H - 1])) return;
    hd[H - 1] = dv;
    hj[H - 1] = j;
#pragma unroll
    for (int p = H - 1; p > 0; --p) {
        if (hd[p] < hd[p - 1]) {
            const float td = hd[p];
            hd[p] = hd[p - 1];
            hd[p - 1] = td;
            const int tj = hj[p];
            hj[p] = hj[p - 1];
            hj[p - 1] = tj;
        }
    }
}

// A: a wavefront owns 32 queries, the B operands (columns) of two 16 x 16
// tiles; the block stages candidate points in LDS and every wavefront sweeps
// them 16 at a time as the A operand (rows).  In the 16 x 16 x 4 MFMA output
// lane l holds column l % 16 (its query) for rows 4 (l / 16) + v, v = 0..3: the
// lane sees 4 candidates per tile and keeps its class's (l / 16) H nearest.
template <int DS, bool VEC>
__global__ __launch_bounds__(NT) void knn_propose_kernel(const float *__restrict__ X, int64_t n, int d, int64_t ldx,
                                                         const float *__restrict__ nrm, float *__restrict__ cand_d,
                                                         int32_t *__restrict__ cand_j) {
    constexpr int CB = DS <= 12 ? 256 : 128;  // candidate points staged in LDS per chunk (<= 50 KB)
    constexpr int DP = 4 * DS + 1;            // padded LDS row (conflict-free column reads)
    __shared__ float xs[CB * DP];
    __shared__ float ns[CB];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t qbase = (int64_t)blockIdx.x * QB + wave * QW;
    // B operands: -2 x_q (the MFMA then accumulates |x_q|^2 + |x_j|^2 - 2 x_q.x_j)
    float bq[2][DS];
    int qi[2];
    float nq[2];
    float hd[2][H];
    int hj[2][H];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const int64_t q = qbase + 16 * g + li;
#pragma unroll
        for (int s = 0; s < DS; ++s) {
            const int c = 4 * s + lk;
            bq[g][s] = (q < n && c < d) ? -2.0f * X[q * ldx + c] : 0.0f;
        }
        qi[g] = q < n ? (int)q : -1;
        nq[g] = q < n ? nrm[q] : 0.0f;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            hd[g][h] = __builtin_inff();
            hj[g][h] = -1;
        }
    }
    for (int64_t c0 = 0; c0 < n; c0 += CB) {
        __syncthreads();
        if constexpr (VEC) {
            // rows of 16-byte quads: four 16-byte loads per thread in flight
            // (clamped in-range addresses, always issued), then their LDS
            // stores; zero past d and past n
            const int64_t ldq = ldx >> 2;
            const v4f *X4 = reinterpret_cast<const v4f *>(X);
            for (int e0 = 0; e0 < CB * DS; e0 += 4 * NT) {
                v4f v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = e0 + u * NT + threadIdx.x;
                    const int p = e / DS, cq = e - p * DS;
                    const int64_t j = c0 + p;
                    // quads at or past d are not read (DS may exceed ceil(d / 4))
                    const bool in = e < CB * DS && j < n && 4 * cq < d;
                    const v4f x = X4[in ? j * ldq + cq : 0];
                    v[u] = in ? x : v4f{0.0f, 0.0f, 0.0f, 0.0f};
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = e0 + u * NT + threadIdx.x;
                    if (e < CB * DS) {
                        const int p = e / DS, cq = e - p * DS;
#pragma unroll
                        for (int k = 0; k < 4; ++k) xs[p * DP + 4 * cq + k] = 4 * cq + k < d ? v[u][k] : 0.0f;
                    }
                }
            }
        } else {
            for (int q = threadIdx.x; q < CB * 4 * DS; q += NT) {
                const int p = q / (4 * DS), c = q - p * (4 * DS);
                const int64_t j = c0 + p;
                xs[p * DP + c] = (j < n && c < d) ? X[j * ldx + c] : 0.0f;
            }
        }
        // rows past n: +inf norm, so their distances are +inf and never proposed
        for (int p = threadIdx.x; p < CB; p += NT) ns[p] = (c0 + p < n) ? nrm[c0 + p] : __builtin_inff();
        __syncthreads();
        const int pend = (int)min<int64_t>(CB, n - c0);
        // software pipeline: the MFMAs of tile t + 16 are issued before the
        // proposals of tile t are processed
        v4f cur[2], nxt[2];
        auto tile_mfma = [&](int t, v4f (&acc)[2]) {
            float a[DS];
#pragma unroll
            for (int s = 0; s < DS; ++s) a[s] = xs[(t + li) * DP + 4 * s + lk];
            const float n0 = ns[t + 4 * lk], n1 = ns[t + 4 * lk + 1], n2 = ns[t + 4 * lk + 2], n3 = ns[t + 4 * lk + 3];
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                acc[g] = v4f{nq[g] + n0, nq[g] + n1, nq[g] + n2, nq[g] + n3};
#pragma unroll
                for (int s = 0; s < DS; ++s)
                    acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], bq[g][s], acc[g], 0, 0, 0);
            }
        };
        // candidate indices in 32 bits (n < 2^31); two tiles per iteration so
        // the pipelined accumulators alternate instead of being copied
        // a tile's four values of a group are compared with the current H-th
        // proposal at once, since most tiles bring none; the query itself is
        // skipped there (rows past n have +inf distances)
        auto consume = [&](int t, const v4f (&acc)[2]) {
            const int j0 = (int)c0 + t + 4 * lk;
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                const float m = fminf(fminf(acc[g][0], acc[g][1]), fminf(acc[g][2], acc[g][3]));
                if (m < hd[g][H - 1]) {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (j0 + v != qi[g]) propose(hd[g], hj[g], acc[g][v], j0 + v);
                }
            }
        };
        tile_mfma(0, cur);
        for (int t = 0; t < pend; t += 32) {
            if (t + 16 < pend) tile_mfma(t + 16, nxt);
            consume(t, cur);
            if (t + 16 >= pend) break;
            if (t + 32 < pend) tile_mfma(t + 32, cur);
            consume(t + 16, nxt);
        }
    }
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        if (qi[g] < 0) continue;
        const int64_t base = (int64_t)qi[g] * NCAND + lk * H;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            cand_d[base + h] = hd[g][h];
            cand_j[base + h] = hj[g][h];
        }
    }
}

__device__ __forceinline__ double exact_d2(const float *__restrict__ X, int64_t ldx, int d, int64_t i, int64_t j) {
#pragma clang fp contract(off)
    const float *xi = X + i * ldx;
    const float *xj = X + j * ldx;
    double s = 0.0;
    for (int c = 0; c < d; ++c) {
        const double t = (double)xj[c] - (double)xi[c];
        const double sq = t * t;
        s = s + sq;
    }
    return s;
}

__device__ __forceinline__ void lexmin(double &d, int &j, double d2, int j2) {
    if (d2 < d || (d2 == d && j2 < j)) {
        d = d2;
        j = j2;
    }
}

// B: one wavefront per row, one proposal per lane (lanes >= NCAND hold none)
__global__ __launch_bounds__(NT) void knn_exact_kernel(const float *__restrict__ X, int64_t n, int d, int64_t ldx,
                                                       const float *__restrict__ nrm, const uint32_t *__restrict__ nmax,
                                                       int K, const float *__restrict__ cand_d,
                                                       const int32_t *__restrict__ cand_j, int32_t *__restrict__ nbr,
                                                       double *__restrict__ nd2, int32_t *__restrict__ flag_list,
                                                       uint32_t *__restrict__ nflag) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
    if (i >= n) return;  // uniform per wavefront
    const int j = lane < NCAND ? cand_j[i * NCAND + lane] : -1;
    const float gd = lane < NCAND ? cand_d[i * NCAND + lane] : __builtin_inff();
    const double de = j >= 0 ? exact_d2(X, ldx, d, i, j) : __builtin_huge_val();
    // the point itself and NaN (non-finite coordinates) are no candidates
    const bool valid = j >= 0 && j != (int)i && de < __builtin_huge_val();
    // the least H-th proposal over the lane classes (+inf: that class is complete)
    float cut = (lane < NCAND && lane % H == H - 1) ? (j >= 0 ? gd : __builtin_inff()) : __builtin_inff();
    for (int off = 32; off > 0; off >>= 1) cut = fminf(cut, __shfl_xor(cut, off, 64));
    bool taken = false;
    double kth = 0.0;
    for (int t = 0; t < K; ++t) {
        double bd = (valid && !taken) ? de : __builtin_huge_val();
        int bj = (valid && !taken) ? j : INT_MAX;
        for (int off = 1; off < 64; off <<= 1) {
            const double d2 = __shfl_xor(bd, off, 64);
            const int j2 = __shfl_xor(bj, off, 64);
            lexmin(bd, bj, d2, j2);
        }
        if (lane == 0) {
            nbr[i * K + t] = bj == INT_MAX ? -1 : bj;
            nd2[i * K + t] = bd;
        }
        if (valid && j == bj) taken = true;
        kth = bd;
    }
    // float32 error bound of the proposals: (2d + 8) u (|x_i|^2 + max |x|^2), u = 2^-24, with margin
    const double nm = (double)__uint_as_float(nmax[0]);
    const double e = (2.0 * d + 8.0) * 5.9604644775390625e-8 * ((double)nrm[i] + nm) * 1.01 + 1e-12 * ((double)nrm[i] + nm);
    const bool certified = (kth < __builtin_huge_val()) && (isinf(cut) || kth < (double)cut - e);
    if (!certified && lane == 0) {
        const uint32_t pos = atomicAdd(nflag, 1u);
        flag_list[pos] = (int32_t)i;
    }
}

// C: exact float64 scan for the rows that were not certified
__global__ __launch_bounds__(NT) void knn_fallback_kernel(const float *__restrict__ X, int64_t n, int d, int64_t ldx,
                                                          int K, const int32_t *__restrict__ flag_list,
                                                          const uint32_t *__restrict__ nflag,
                                                          double *__restrict__ scratch, int32_t *__restrict__ nbr,
                                                          double *__restrict__ nd2) {
    __shared__ double rd[NT / 64];
    __shared__ int rj[NT / 64];
    const uint32_t cnt = nflag[0];
    double *dd = scratch + (int64_t)blockIdx.x * n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (uint32_t f = blockIdx.x; f < cnt; f += gridDim.x) {
        const int64_t i = flag_list[f];
        for (int64_t j = threadIdx.x; j < n; j += NT) dd[j] = (j == i) ? __builtin_huge_val() : exact_d2(X, ldx, d, i, j);
        __syncthreads();
        for (int t = 0; t < K; ++t) {
            double bd = __builtin_huge_val();
            int bj = INT_MAX;
            for (int64_t j = threadIdx.x; j < n; j += NT) lexmin(bd, bj, dd[j], (int)j);
            for (int off = 1; off < 64; off <<= 1) {
                const double d2 = __shfl_xor(bd, off, 64);
                const int j2 = __shfl_xor(bj, off, 64);
                lexmin(bd, bj, d2, j2);
            }
            if (lane == 0) {
                rd[wave] = bd;
                rj[wave] = bj;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                for (int w = 1; w < NT / 64; ++w) lexmin(bd, bj, rd[w], rj[w]);
                // no finite distance left (non-finite coordinates): no neighbour
                const bool found = bd < __builtin_huge_val();
                nbr[i * K + t] = found ? bj : -1;
                nd2[i * K + t] = bd;
                if (found) dd[bj] = __builtin_huge_val();
            }
            __syncthreads();
        }
    }
}

// D: union graph
// entries -1 (no neighbour found: non-finite coordinates) are skipped by every kernel below
__global__ void rev_count_kernel(const int32_t *__restrict__ nbr, int64_t nk, int32_t *__restrict__ cnt) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nk; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = nbr[t];
        if (j >= 0) atomicAdd(&cnt[j], 1);
    }
}

// exclusive prefix sums of int32 or int64 counts into int64 offsets [n + 1],
// three passes over tiles of kScanTile elements (integer sums: exact)
template <typename T>
__global__ void scan_tile_sums_kernel(const T *__restrict__ in, int64_t n, int64_t *__restrict__ tile_sums) {
    __shared__ int64_t red[NT / 64];
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
    for (int64_t q = t0 + threadIdx.x; q < min(n, t0 + kScanTile); q += NT) s += (int64_t)in[q];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t tot = 0;
        for (int w = 0; w < NT / 64; ++w) tot += red[w];
        tile_sums[blockIdx.x] = tot;
    }
}

__global__ void scan_tile_offsets_kernel(int64_t *__restrict__ tile_sums, int64_t ntiles) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int64_t run = 0;
        for (int64_t t = 0; t < ntiles; ++t) {
            const int64_t v = tile_sums[t];
            tile_sums[t] = run;
            run += v;
        }
        tile_sums[ntiles] = run;
    }
}

// within a tile: thread 0 of the block walks its tile in order (tiles are
// 2048 elements; every block runs in parallel)
template <typename T, typename O>
__global__ void scan_apply_kernel(const T *__restrict__ in, int64_t n, const int64_t *__restrict__ tile_sums,
                                  int64_t ntiles, O *__restrict__ out) {
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
    if (threadIdx.x != 0) return;
    int64_t run = tile_sums[blockIdx.x];
    for (int64_t q = t0; q < min(n, t0 + kScanTile); ++q) {
        out[q] = (O)run;
        run += (int64_t)in[q];
    }
    if (blockIdx.x == ntiles - 1) out[n] = (O)tile_sums[ntiles];
}

__global__ void rev_fill_kernel(const int32_t *__restrict__ nbr, int64_t n, int K, const int64_t *__restrict__ rev_off,
                                int32_t *__restrict__ cursor, int32_t *__restrict__ rev) {
    const int64_t nk = n * K;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nk; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = nbr[t];
        if (j < 0) continue;
        const int32_t pos = atomicAdd(&cursor[j], 1);
        rev[rev_off[j] + pos] = (int32_t)(t / K);
    }
}

// sorted copy of row i's neighbours (K <= 32, insertion sort); returns how many
__device__ __forceinline__ int sorted_nbrs(const int32_t *__restrict__ nbr, int64_t i, int K, int32_t (&s)[kMaxK]) {
    int m = 0;
    for (int t = 0; t < K; ++t) {
        const int32_t v = nbr[i * K + t];
        if (v < 0) continue;
        int p = m;
        while (p > 0 && s[p - 1] > v) {
            s[p] = s[p - 1];
            --p;
        }
        s[p] = v;
        ++m;
    }
    return m;
}

// one thread per row: sort the reverse list in place, count the merged set
__global__ void union_count_kernel(const int32_t *__restrict__ nbr, int64_t n, int K,
                                   const int64_t *__restrict__ rev_off, int32_t *__restrict__ rev,
                                   int64_t *__restrict__ len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t *r = rev + rev_off[i];
    const int64_t m = rev_off[i + 1] - rev_off[i];
    for (int64_t a = 1; a < m; ++a) {
        const int32_t v = r[a];
        int64_t p = a;
        while (p > 0 && r[p - 1] > v) {
            r[p] = r[p - 1];
            --p;
        }
        r[p] = v;
    }
    int32_t s[kMaxK];
    const int ka = sorted_nbrs(nbr, i, K, s);
    int64_t a = 0, b = 0, c = 0;
    while (a < ka || b < m) {
        const int32_t va = a < ka ? s[a] : INT_MAX;
        const int32_t vb = b < m ? r[b] : INT_MAX;
        if (va <= vb) ++a;
        if (vb <= va) ++b;
        ++c;
    }
    len[i] = c;
}

__global__ void union_fill_kernel(const float *__restrict__ X, int64_t ldx, int d, const int32_t *__restrict__ nbr,
                                  int64_t n, int K, const int64_t *__restrict__ rev_off,
                                  const int32_t *__restrict__ rev, const int32_t *__restrict__ row_ptr,
                                  int32_t *__restrict__ col_idx, float *__restrict__ d2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t *r = rev + rev_off[i];
    const int64_t m = rev_off[i + 1] - rev_off[i];
    int32_t s[kMaxK];
    const int ka = sorted_nbrs(nbr, i, K, s);
    int64_t a = 0, b = 0, c = row_ptr[i];
    while (a < ka || b < m) {
        const int32_t va = a < ka ? s[a] : INT_MAX;
        const int32_t vb = b < m ? r[b] : INT_MAX;
        const int32_t v = va < vb ? va : vb;
        if (va <= vb) ++a;
        if (vb <= va) ++b;
        col_idx[c] = v;
        d2[c] = (float)exact_d2(X, ldx, d, i, v);
        ++c;
    }
}

template <int DS>
void launch_propose(const float *X, int64_t n, int d, int64_t ldx, const KnnWs &w, hipStream_t s) {
    const unsigned grid = (unsigned)((n + QB - 1) / QB);
    if (aligned(X, 16) && ldx % 4 == 0)
        knn_propose_kernel<DS, true><<<grid, NT, 0, s>>>(X, n, d, ldx, w.nrm, w.cand_d, w.cand_j);
    else
        knn_propose_kernel<DS, false><<<grid, NT, 0, s>>>(X, n, d, ldx, w.nrm, w.cand_d, w.cand_j);
}

void scan_i32(const int32_t *in, int64_t n, int64_t *tile_sums, int64_t *out, hipStream_t s) {
    const int64_t nt = scan_tiles(n);
    scan_tile_sums_kernel<int32_t><<<(unsigned)nt, NT, 0, s>>>(in, n, tile_sums);
    scan_tile_offsets_kernel<<<1, 64, 0, s>>>(tile_sums, nt);
    scan_apply_kernel<int32_t, int64_t><<<(unsigned)nt, 64, 0, s>>>(in, n, tile_sums, nt, out);
}

asc_status check_knn_args(const float *X, int64_t n, int d, int64_t ldx, int k, const char *who) {
    if (!X || !aligned(X, 4)) return fail(ASC_ERR_INVALID, "%s: X NULL or misaligned", who);
    if (n < 2 || n >= (int64_t(1) << 31)) return fail(ASC_ERR_INVALID, "%s: n=%lld", who, (long long)n);
    if (d < 1 || d > kMaxD || ldx < d) return fail(ASC_ERR_INVALID, "%s: d=%d (1..%d), ldx=%lld", who, d, kMaxD, (long long)ldx);
    if (k < 1 || k > kMaxK || k > n - 1) return fail(ASC_ERR_INVALID, "%s: k=%d not in [1, min(%d, n-1)]", who, k, kMaxK);
    if (n * (int64_t)k * 2 >= (int64_t(1) << 31)) return fail(ASC_ERR_INVALID, "%s: n*k too large", who);
    return ASC_OK;
}

}  // namespace
}  // namespace asc

using namespace asc;

extern "C" size_t asc_knn_workspace(int64_t n, int d, int k) {
    (void)d;
    if (n < 2 || k < 1) return 0;
    return knn_ws_layout(n, k, nullptr, nullptr);
}

extern "C" asc_status asc_knn(const float *X, int64_t n, int d, int64_t ldx, int k, int32_t *nbr, double *d2,
                              int32_t *row_ptr, uint32_t *fallback_rows, void *ws, size_t ws_bytes, void *stream) {
    const char *who = "asc_knn";
    ASC_TRY(check_knn_args(X, n, d, ldx, k, who));
    if (!nbr || !aligned(nbr, 4) || !d2 || !aligned(d2, 8) || !row_ptr || !aligned(row_ptr, 4) ||
        (fallback_rows && !aligned(fallback_rows, 4)))
        return fail(ASC_ERR_INVALID, "%s: an output is NULL or misaligned", who);
    ASC_TRY(check_ws(ws, ws_bytes, asc_knn_workspace(n, d, k), who));
    hipStream_t s = as_stream(stream);
    KnnWs w;
    knn_ws_layout(n, k, ws, &w);
    knn_clear_kernel<<<(unsigned)std::min<int64_t>((n + 255) / 256, 4096), 256, 0, s>>>(w.nmax, w.nflag, w.cnt, n);
    ASC_LAUNCHED();
    sqnorm_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(X, n, d, ldx, w.nrm, w.nmax);
    ASC_LAUNCHED();
    switch ((d + 3) / 4) {
        case 1: launch_propose<1>(X, n, d, ldx, w, s); break;
        case 2: launch_propose<2>(X, n, d, ldx, w, s); break;
        case 3: launch_propose<3>(X, n, d, ldx, w, s); break;
        case 4: launch_propose<4>(X, n, d, ldx, w, s); break;
        case 5: case 6: launch_propose<6>(X, n, d, ldx, w, s); break;
        case 7: case 8: launch_propose<8>(X, n, d, ldx, w, s); break;
        case 9: case 10: case 11: case 12: launch_propose<12>(X, n, d, ldx, w, s); break;
        default: launch_propose<16>(X, n, d, ldx, w, s); break;
    }
    ASC_LAUNCHED();
    knn_exact_kernel<<<(unsigned)((n + 3) / 4), NT, 0, s>>>(X, n, d, ldx, w.nrm, w.nmax, k, w.cand_d, w.cand_j, nbr, d2,
                                                           w.flag_list, w.nflag);
    ASC_LAUNCHED();
    knn_fallback_kernel<<<fallback_blocks(n), NT, 0, s>>>(X, n, d, ldx, k, w.flag_list, w.nflag, w.scratch, nbr, d2);
    ASC_LAUNCHED();
    if (fallback_rows) {
        ASC_HIP(hipMemcpyAsync(fallback_rows, w.nflag, sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    }
    // union graph offsets
    const int64_t nk = n * k;
    rev_count_kernel<<<(unsigned)std::min<int64_t>((nk + 255) / 256, 65536), 256, 0, s>>>(nbr, nk, w.cnt);
    ASC_LAUNCHED();
    scan_i32(w.cnt, n, w.tile_sums, w.rev_off, s);
    ASC_LAUNCHED();
    zero_i32_kernel<<<(unsigned)std::min<int64_t>((n + 255) / 256, 4096), 256, 0, s>>>(w.cnt, n);
    ASC_LAUNCHED();
    rev_fill_kernel<<<(unsigned)std::min<int64_t>((nk + 255) / 256, 65536), 256, 0, s>>>(nbr, n, k, w.rev_off, w.cnt,
                                                                                       w.rev);
    ASC_LAUNCHED();
    union_count_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(nbr, n, k, w.rev_off, w.rev, w.len);
    ASC_LAUNCHED();
    {
        const int64_t nt = scan_tiles(n);
        scan_tile_sums_kernel<int64_t><<<(unsigned)nt, NT, 0, s>>>(w.len, n, w.tile_sums);
        scan_tile_offsets_kernel<<<1, 64, 0, s>>>(w.tile_sums, nt);
        scan_apply_kernel<int64_t, int32_t><<<(unsigned)nt, 64, 0, s>>>(w.len, n, w.tile_sums, nt, row_ptr);
        ASC_LAUNCHED();
    }
    return ASC_OK;
}

extern "C" asc_status asc_knn_graph_fill(const float *X, int64_t n, int d, int64_t ldx, int k, const int32_t *nbr,
                                         const int32_t *row_ptr, int32_t *col_idx, float *d2, void *ws,
                                         size_t ws_bytes, void *stream) {
    const char *who = "asc_knn_graph_fill";
    ASC_TRY(check_knn_args(X, n, d, ldx, k, who));
    if (!nbr || !row_ptr || !col_idx || !d2 || !aligned(col_idx, 4) || !aligned(d2, 4))
        return fail(ASC_ERR_INVALID, "%s: an argument is NULL or misaligned", who);
    ASC_TRY(check_ws(ws, ws_bytes, asc_knn_workspace(n, d, k), who));
    KnnWs w;
    knn_ws_layout(n, k, ws, &w);
    union_fill_kernel<<<(unsigned)((n + 255) / 256), 256, 0, as_stream(stream)>>>(X, ldx, d, nbr, n, k, w.rev_off, w.rev,
                                                                                 row_ptr, col_idx, d2);
    ASC_LAUNCHED();
    return ASC_OK;
}
