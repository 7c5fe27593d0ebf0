// Gradients of a loss on the filtered signals with respect to the edge
// weights, the Gaussian-kernel bandwidth and the Chebyshev coefficients
// (an extension of the fast filter of Sec. 2.4; similarity weights of
// Sec. 2.2 step 1).
//
// Reverse mode of Y = sum_j a_j T_j, T_1 = Lt T_0, T_{j+1} = 2 Lt T_j - T_{j-1}:
//   A_p = a_p G,  A_j = a_j G + 2 Lt A_{j+1} - A_{j+2}  (A_{p+1} = 0),
//   dloss/dLt = M = A_1 T_0^T + sum_{j=1..p-1} 2 A_{j+1} T_j^T,
//   dw_(i,k) = (2/lmax)(M_ii - M_ik) per stored entry, da_j = <G, T_j>.
// The adjoint step gathers A_{j+1}[k] over the neighbours of row i, exactly
// like the forward step gathers T_j[k]; the same gathered rows give
// <A_{j+1}[k], T_j[i]> = (A_{j+1} T_j^T)_{k,i}, i.e. the M entry of the stored
// transpose (k, i).  These are accumulated per entry in float32 and mapped to
// dw through the transpose permutation at the end, so no second gather is
// needed.  T_j is recomputed segment by segment from the forward checkpoints
// (T_{sc}, T_{sc+1}).
#include "recurrence.hpp"

namespace asc {
namespace {

constexpr unsigned B_TOP = 1u;   // j = p-1: there is no A_{j+2}
constexpr unsigned B_OUT = 2u;   // write A_j (j >= 1)
constexpr unsigned B_DW = 4u;    // accumulate the per-entry and diagonal M terms
constexpr unsigned B_DA = 8u;    // partial <G, T_j>

struct AdjArgs {
    int64_t n;
    const int32_t *rp;
    const int32_t *ci;
    const float *w;
    const float *diag;
    const float *beta;
    const void *acur;   // panel A_{j+1}
    const void *aold;   // panel A_{j+2}
    void *aout;         // panel A_j (may equal aold)
    const void *tj;     // panel T_j
    const float *G;     // caller block, slice columns c0..
    int64_t ldg, c0, r;
    const double *coeffs;  // a_0..a_p
    int j;              // this step produces A_j
    float cj;           // 1 (j = 0) or 2
    float *mt;          // [nnz] accumulated (A T^T)_{k,i} at entry (i,k)
    float *mdiag;       // [n] accumulated M_ii
    double *partials;   // [gridDim.x] <G, T_j>
    int xcd_bands;      // tiles of XCD x (workgroups b with b mod 8 = x) form one contiguous band of rows
    int64_t nnz_hint;   // stored entries (host side: picks the kernel variant)
};

template <int VN>
__device__ __forceinline__ void load_g(const float *__restrict__ G, int64_t row, int64_t ldg, int64_t cbase, int64_t r,
                                       float (&g)[VN]) {
    const float *gr = G + row * ldg + cbase;
    if (cbase + VN <= r) {
#pragma unroll
        for (int q = 0; q < VN; q += 4) {
            const v4f x = *reinterpret_cast<const v4f *>(gr + q);
            g[q] = x.x; g[q + 1] = x.y; g[q + 2] = x.z; g[q + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < VN; ++q) g[q] = (cbase + q < r) ? gr[q] : 0.0f;
    }
}

__device__ __forceinline__ float dot_raw(const v4f &x, const float (&t)[4]) {
    return ((x.x * t[0] + x.y * t[1]) + x.z * t[2]) + x.w * t[3];
}
__device__ __forceinline__ float dot_raw(const v4u &x, const float (&t)[8]) {
    return ((((((bf16_lo(x.x) * t[0] + bf16_hi(x.x) * t[1]) + bf16_lo(x.y) * t[2]) + bf16_hi(x.y) * t[3]) +
              bf16_lo(x.z) * t[4]) + bf16_hi(x.z) * t[5]) + bf16_lo(x.w) * t[6]) + bf16_hi(x.w) * t[7];
}

// sum over the LPR lanes of a row group (all lanes get the sum)
template <int LPR>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Reduce-scatter over the 8 lanes of a row group: lane t holds partial dots
// p[0..7] of 8 entries and ends with the group's sum for entry t, in 3
// exchange steps (xor 4, 2, 1), each halving the entries a lane carries:
// 7 shuffles instead of the 24 of eight separate butterflies.
__device__ __forceinline__ float group8_reduce_scatter(const float (&p)[8], int t) {
    const bool b2 = (t & 4) != 0, b1 = (t & 2) != 0, b0 = (t & 1) != 0;
    float h[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float send = b2 ? p[q] : p[q + 4];
        const float keep = b2 ? p[q + 4] : p[q];
        h[q] = keep + __shfl_xor(send, 4, 64);  // entry 4 b2 + q
    }
    float h2[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const float send = b1 ? h[q] : h[q + 2];
        const float keep = b1 ? h[q + 2] : h[q];
        h2[q] = keep + __shfl_xor(send, 2, 64);  // entry 4 b2 + 2 b1 + q
    }
    const float send = b0 ? h2[0] : h2[1];
    const float keep = b0 ? h2[1] : h2[0];
    return keep + __shfl_xor(send, 1, 64);  // entry t
}

// Per-entry accumulator stores of a tile are staged in LDS and written out
// once the whole tile is done: the 4-byte stores of a row group come one
// neighbour group at a time, microseconds apart while the gathers are in
// flight, and written straight to memory they leave partly written lines that
// the L2 writes back more than once.  A tile of up to this many stored
// entries is staged (16 KB of LDS per workgroup); longer tiles store directly.
constexpr int kStageEntries = 4096;

// PF: the next neighbour group's indices, weights and accumulated entries are
// loaded while the current group's gathers are in flight (pays off on long
// rows; on short rows the extra registers cost more than it hides)
template <typename TS, int LPR, unsigned MODE, bool PF>
__global__ __launch_bounds__(NT) void adj_step(AdjArgs A) {
    constexpr int VN = St<TS>::VN;
    constexpr int RS = LPR * VN;
    constexpr int RPW = 64 / LPR;
    constexpr int ROWS = RPW * (NT / 64);
    constexpr int U = 8;
    typedef typename St<TS>::raw raw_t;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int t = lane % LPR;
    const int sub = lane / LPR;
    const TS *__restrict__ acur = static_cast<const TS *>(A.acur);
    const TS *__restrict__ aold = static_cast<const TS *>(A.aold);
    TS *__restrict__ aout = static_cast<TS *>(A.aout);
    const TS *__restrict__ tj = static_cast<const TS *>(A.tj);
    const float beta = A.beta[0];
    const float aj = (MODE & B_OUT) ? (float)A.coeffs[A.j] : 0.0f;
    const bool weighted = A.w != nullptr;
    double p_da = 0.0;
    const int64_t ntiles = (A.n + ROWS - 1) / ROWS;
    // tile schedule: round robin over the grid, or (for locality-ordered
    // graphs) one contiguous band of tiles per XCD, as in the forward step
    int64_t tfirst = blockIdx.x, tend = ntiles, tstep = gridDim.x;
    if (A.xcd_bands && gridDim.x >= 8) {
        const int64_t xcd = blockIdx.x % 8;
        const int64_t chunk = (ntiles + 7) / 8;
        tfirst = xcd * chunk + blockIdx.x / 8;
        tend = xcd * chunk + chunk < ntiles ? xcd * chunk + chunk : ntiles;
        tstep = (gridDim.x - xcd + 7) / 8;
    }
    constexpr bool STAGE = (MODE & B_DW) != 0;
    __shared__ float mstage[STAGE ? kStageEntries : 1];
    for (int64_t tile = tfirst; tile < tend; tile += tstep) {
        const int64_t row = tile * ROWS + (int64_t)wave * RPW + sub;
        // rows past n still run the neighbour loop (with no entries) so that
        // every lane takes part in the group reductions
        const bool live = row < A.n;
        // the tile's stored entries [te0, te1) (block-uniform)
        int32_t te0 = 0, te1 = 0;
        if (STAGE) {
            const int64_t r0 = tile * ROWS;
            const int64_t r1 = r0 + ROWS < A.n ? r0 + ROWS : A.n;
            te0 = A.rp[r0];
            te1 = A.rp[r1];
        }
        const bool staged = STAGE && (te1 - te0) <= kStageEntries;
        const int64_t rrow = live ? row : 0;
        const int32_t e0 = live ? A.rp[row] : 0;
        const int32_t e1 = live ? A.rp[row + 1] : 0;
        float tv[VN];
        unpack(ldraw(tj + rrow * RS + t * VN), tv);
        float acc[VN];
#pragma unroll
        for (int q = 0; q < VN; ++q) acc[q] = 0.0f;
        const TS *base = acur + t * VN;
        // loop trip count must be uniform across the lanes of a row group: it is
        // (e1 - e0) for the group's row, identical for its LPR lanes
        int32_t kc[U];
        float wc[U];
        float mtv[U];  // this lane's accumulated entries, loaded with the indices
        auto load_group = [&](int32_t eg, int32_t (&k_)[U], float (&w_)[U], float (&m_)[U]) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                k_[u] = (int32_t)rrow;
                w_[u] = 0.0f;
                m_[u] = 0.0f;
                if (eg + u < e1) {
                    k_[u] = A.ci[eg + u];
                    w_[u] = weighted ? A.w[eg + u] : 1.0f;
                    if ((MODE & B_DW) && (u % LPR) == t) m_[u] = A.mt[eg + u];
                }
            }
        };
        if (PF && e0 < e1) load_group(e0, kc, wc, mtv);
        for (int32_t e = e0; e < e1; e += U) {
            if (!PF) load_group(e, kc, wc, mtv);
            raw_t v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = ldraw(base + (int64_t)kc[u] * RS);
            int32_t kn[U];
            float wn[U], mn[U];
            if (PF && e + U < e1) load_group(e + U, kn, wn, mn);
#pragma unroll
            for (int u = 0; u < U; ++u) fma_raw(acc, wc[u], v[u]);
            if (MODE & B_DW) {
                if constexpr (LPR == 8 && U == 8) {
                    float pd[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) pd[u] = dot_raw(v[u], tv);
                    const float ds = group8_reduce_scatter(pd, t);  // entry e + t, owned by lane t
                    float own_m = 0.0f;
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (u == t) own_m = mtv[u];
                    if (e + t < e1) {
                        if (staged) mstage[e + t - te0] = own_m + A.cj * ds;
                        else A.mt[e + t] = own_m + A.cj * ds;
                    }
                } else {
                    float dsum[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) dsum[u] = group_sum<LPR>(dot_raw(v[u], tv));
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if ((u % LPR) == t && e + u < e1) {
                            if (staged) mstage[e + u - te0] = mtv[u] + A.cj * dsum[u];
                            else A.mt[e + u] = mtv[u] + A.cj * dsum[u];
                        }
                }
            }
            if (PF && e + U < e1) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    kc[u] = kn[u];
                    wc[u] = wn[u];
                    mtv[u] = mn[u];
                }
            }
        }
        float own[VN], g[VN];
        unpack(ldraw(acur + rrow * RS + t * VN), own);
        load_g<VN>(A.G, rrow, A.ldg, A.c0 + (int64_t)t * VN, A.r, g);
        if (MODE & B_DW) {
            float dd = 0.0f;
#pragma unroll
            for (int q = 0; q < VN; ++q) dd += own[q] * tv[q];
            dd = group_sum<LPR>(dd);
            if (live && t == 0) A.mdiag[row] += A.cj * dd;
        }
        if (MODE & B_DA) {
            if (live) {
#pragma unroll
                for (int q = 0; q < VN; ++q) p_da += (double)g[q] * (double)tv[q];
            }
        }
        if ((MODE & B_OUT) && live) {
            const float d = A.diag[row];
            float nxt[VN], stv[VN];
            if (MODE & B_TOP) {
#pragma unroll
                for (int q = 0; q < VN; ++q) nxt[q] = fmaf(aj, g[q], fmaf(d, own[q], beta * acc[q]));
            } else {
                float old[VN];
                unpack(ldraw(aold + row * RS + t * VN), old);
#pragma unroll
                for (int q = 0; q < VN; ++q) nxt[q] = fmaf(aj, g[q], fmaf(d, own[q], fmaf(beta, acc[q], -old[q])));
            }
            st16(aout + row * RS + t * VN, nxt, stv);
        }
        if (staged) {
            // the tile's entries, complete, in one pass of consecutive stores
            __syncthreads();
            for (int32_t q = (int32_t)threadIdx.x; q < te1 - te0; q += NT) A.mt[te0 + q] = mstage[q];
            __syncthreads();
        }
    }
    if (MODE & B_DA) {
        __shared__ double lds[NT / 64];
        double v[1] = {p_da};
        block_sum<1, NT>(v, lds);
        if (threadIdx.x == 0) A.partials[blockIdx.x] = v[0];
    }
}

template <typename TS, int LPR, bool PF>
hipError_t launch_adj_t(unsigned mode, const AdjArgs &A, int grid, hipStream_t s) {
    switch (mode) {
#define ASC_ADJ_CASE(m) \
    case m: adj_step<TS, LPR, m, PF><<<grid, NT, 0, s>>>(A); break;
        ASC_ADJ_CASE(0) ASC_ADJ_CASE(1) ASC_ADJ_CASE(2) ASC_ADJ_CASE(3) ASC_ADJ_CASE(4) ASC_ADJ_CASE(5)
        ASC_ADJ_CASE(6) ASC_ADJ_CASE(7) ASC_ADJ_CASE(8) ASC_ADJ_CASE(9) ASC_ADJ_CASE(10) ASC_ADJ_CASE(11)
        ASC_ADJ_CASE(12) ASC_ADJ_CASE(13) ASC_ADJ_CASE(14) ASC_ADJ_CASE(15)
#undef ASC_ADJ_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool PF>
hipError_t launch_adj_pf(asc_dtype dt, int lpr, unsigned mode, const AdjArgs &A, int grid, hipStream_t s) {
    if (dt == ASC_F32) {
        switch (lpr) {
            case 2: return launch_adj_t<float, 2, PF>(mode, A, grid, s);
            case 4: return launch_adj_t<float, 4, PF>(mode, A, grid, s);
            case 8: return launch_adj_t<float, 8, PF>(mode, A, grid, s);
            case 16: return launch_adj_t<float, 16, PF>(mode, A, grid, s);
        }
    } else {
        switch (lpr) {
            case 2: return launch_adj_t<uint16_t, 2, PF>(mode, A, grid, s);
            case 4: return launch_adj_t<uint16_t, 4, PF>(mode, A, grid, s);
            case 8: return launch_adj_t<uint16_t, 8, PF>(mode, A, grid, s);
            case 16: return launch_adj_t<uint16_t, 16, PF>(mode, A, grid, s);
        }
    }
    return hipErrorInvalidValue;
}

// the one-group-ahead index loads are used from 3 groups of 8 entries per row on average
hipError_t launch_adj(asc_dtype dt, int lpr, unsigned mode, const AdjArgs &A, int grid, hipStream_t s) {
    const bool long_rows = A.n > 0 && A.rp && A.nnz_hint >= 24 * A.n;
    return long_rows ? launch_adj_pf<true>(dt, lpr, mode, A, grid, s) : launch_adj_pf<false>(dt, lpr, mode, A, grid, s);
}

// A_p = a_p G (slice), partial <G, T_p>
template <typename TS>
__global__ void adj_init_kernel(int64_t n, const float *__restrict__ G, int64_t ldg, int64_t c0, int64_t r, int rs,
                                const double *__restrict__ coeffs, int p, const TS *__restrict__ tp,
                                TS *__restrict__ ap, double *__restrict__ part) {
    __shared__ double lds[NT / 64];
    const float a = (float)coeffs[p];
    double v[1] = {0.0};
    const int64_t total = n * rs;
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < total; q += (int64_t)gridDim.x * NT) {
        const int64_t i = q / rs, c = q - i * rs;
        const float gv = (c0 + c < r) ? G[i * ldg + c0 + c] : 0.0f;
        float tv;
        if constexpr (sizeof(TS) == 4) {
            tv = (float)tp[q];
            ap[q] = (TS)(a * gv);
        } else {
            tv = __uint_as_float(((uint32_t)tp[q]) << 16);
            ap[q] = (TS)f32_to_bf16_bits(a * gv);
        }
        v[0] += (double)gv * (double)tv;
    }
    block_sum<1, NT>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ void fill_f32(float *p, int64_t count, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void fill_f64(double *p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// tr[e] for e = (i, k): position of (k, i) in row k; -1 and a flag if absent
__global__ void transpose_map_kernel(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                     int32_t *__restrict__ tr, uint32_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int32_t k = ci[e];
        int32_t lo = rp[k], hi = rp[k + 1], pos = -1;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            const int32_t c = ci[mid];
            if (c == (int32_t)i) { pos = mid; break; }
            if (c < (int32_t)i) lo = mid + 1; else hi = mid;
        }
        tr[e] = pos;
        if (pos < 0) atomicOr(flags, (uint32_t)ASC_FLAG_BAD_GRAPH);
    }
}

// dw[tr[e]] = (2/lmax)(M_kk - mt[e]) for e = (i, k)
__global__ void dw_final_kernel(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                const int32_t *__restrict__ tr, const float *__restrict__ mt,
                                const float *__restrict__ mdiag, const double *__restrict__ lmax,
                                float *__restrict__ dw) {
    const float sc = (float)(2.0 / lmax[0]);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int32_t q = tr[e];
        if (q >= 0) dw[q] = sc * (mdiag[ci[e]] - mt[e]);
    }
}

// dsum[j] += sum_b part[j][b] (fixed order), j = 0..p
__global__ void da_accum_kernel(const double *__restrict__ part, int nparts, int64_t stride, int p,
                                double *__restrict__ dsum) {
    __shared__ double lds[NT / 64];
    const int j = blockIdx.x;
    if (j > p) return;
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nparts; b += NT) v[0] += part[(int64_t)j * stride + b];
    block_sum<1, NT>(v, lds);
    if (threadIdx.x == 0) dsum[j] += v[0];
}

__global__ void copy_f64(const double *__restrict__ src, double *__restrict__ dst, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = src[i];
}

// w = exp(-d2 / sigma^2) (evaluated in float64, stored float32)
__global__ void gauss_kernel(const float *__restrict__ d2, int64_t nnz, double sigma, float *__restrict__ w) {
    const double inv = 1.0 / (sigma * sigma);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        w[e] = (float)exp(-(double)d2[e] * inv);
}

// partial sum_e dw_e w_e 2 d2_e / sigma^3
__global__ void gauss_bwd_kernel(const float *__restrict__ d2, const float *__restrict__ w,
                                 const float *__restrict__ dw, int64_t nnz, double sigma, double *__restrict__ part) {
    __shared__ double lds[NT / 64];
    const double c = 2.0 / (sigma * sigma * sigma);
    double v[1] = {0.0};
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * NT)
        v[0] += (double)dw[e] * (double)w[e] * (double)d2[e] * c;
    block_sum<1, NT>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ void sum_to_scalar(const double *__restrict__ part, int nparts, double *__restrict__ out) {
    __shared__ double lds[NT / 64];
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nparts; b += NT) v[0] += part[b];
    block_sum<1, NT>(v, lds);
    if (threadIdx.x == 0) out[0] = v[0];
}

// loss = sum_i |y_i/|y_i| - t_i|^2 and G = dloss/dY; one wavefront per row
__global__ __launch_bounds__(NT) void rownorm_loss_kernel(const float *__restrict__ Y, int64_t ldy,
                                                          const float *__restrict__ T, int64_t ldt, int64_t n,
                                                          int64_t r, float *__restrict__ G, int64_t ldg,
                                                          double *__restrict__ part) {
    __shared__ double lds[NT / 64];
    const int lane = threadIdx.x & 63;
    const int64_t w0 = ((int64_t)blockIdx.x * NT + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * NT) >> 6;
    double loss = 0.0;
    for (int64_t i = w0; i < n; i += nw) {
        const float *y = Y + i * ldy;
        const float *tt = T + i * ldt;
        double s = 0.0;
        for (int64_t c = lane; c < r; c += 64) {
            const double v = y[c];
            s += v * v;
        }
        s = wave_sum(s);
        const double nrm = sqrt(s);
        double fg = 0.0, l = 0.0;
        for (int64_t c = lane; c < r; c += 64) {
            const double f = nrm > 0.0 ? (double)y[c] / nrm : 0.0;
            const double dlt = f - (double)tt[c];
            l += dlt * dlt;
            fg += f * 2.0 * dlt;
        }
        l = wave_sum(l);
        fg = wave_sum(fg);
        for (int64_t c = lane; c < r; c += 64) {
            double gv = 0.0;
            if (nrm > 0.0) {
                const double f = (double)y[c] / nrm;
                gv = (2.0 * (f - (double)tt[c]) - f * fg) / nrm;
            }
            G[i * ldg + c] = (float)gv;
        }
        if (lane == 0) loss += l;
    }
    double v[1] = {loss};
    block_sum<1, NT>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

struct BwdWs {
    WsHeader *hdr;
    float *diag;
    float *beta;
    int32_t *tr;
    float *mt;
    float *mdiag;
    double *dapart;   // [p+1][kMaxGrid]
    double *dsum;     // [p+1]
    void *panels;     // (c+1) state panels + 2 adjoint panels
};

size_t bwd_ws_layout(int64_t n, int64_t nnz, int64_t r, asc_dtype dt, int p, int c, void *ws, BwdWs *out) {
    Arena a(ws);
    BwdWs b;
    b.hdr = a.take<WsHeader>(1);
    b.diag = a.take<float>(n);
    b.beta = a.take<float>(64);
    b.tr = a.take<int32_t>(nnz > 0 ? nnz : 1);
    b.mt = a.take<float>(nnz > 0 ? nnz : 1);
    b.mdiag = a.take<float>(n);
    b.dapart = a.take<double>((size_t)(p + 1) * kMaxGrid);
    b.dsum = a.take<double>(p + 1 + 64);
    b.panels = a.take<char>((size_t)(c + 3) * n * rs_for_ws(r, dt) * esize(dt));
    if (out) *out = b;
    return a.size();
}

int grid1(int64_t count) { return (int)std::max<int64_t>(1, std::min<int64_t>((count + 255) / 256, 16384)); }

}  // namespace
}  // namespace asc

using namespace asc;

extern "C" asc_status asc_gauss_weights(const float *d2, int64_t nnz, double sigma, float *w, void *stream) {
    if (nnz < 0 || (nnz > 0 && (!d2 || !w)) || !(sigma > 0.0) || !std::isfinite(sigma))
        return fail(ASC_ERR_INVALID, "asc_gauss_weights: bad arguments");
    if (nnz == 0) return ASC_OK;
    gauss_kernel<<<grid1(nnz), 256, 0, as_stream(stream)>>>(d2, nnz, sigma, w);
    ASC_LAUNCHED();
    return ASC_OK;
}

extern "C" size_t asc_gauss_weights_bwd_workspace(int64_t nnz) {
    (void)nnz;
    return 256 + sizeof(double) * kMaxGrid;
}

extern "C" asc_status asc_gauss_weights_bwd(const float *d2, const float *w, const float *dW, int64_t nnz,
                                            double sigma, double *dsigma, void *ws, size_t ws_bytes, void *stream) {
    const char *who = "asc_gauss_weights_bwd";
    if (nnz < 0 || !dsigma || (nnz > 0 && (!d2 || !w || !dW)) || !(sigma > 0.0))
        return fail(ASC_ERR_INVALID, "%s: bad arguments", who);
    ASC_TRY(check_ws(ws, ws_bytes, asc_gauss_weights_bwd_workspace(nnz), who));
    double *part = reinterpret_cast<double *>(static_cast<char *>(ws) + 256);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((nnz + NT - 1) / NT, kMaxGrid));
    hipStream_t s = as_stream(stream);
    gauss_bwd_kernel<<<grid, NT, 0, s>>>(d2, w, dW, nnz, sigma, part);
    ASC_LAUNCHED();
    sum_to_scalar<<<1, NT, 0, s>>>(part, grid, dsigma);
    ASC_LAUNCHED();
    return ASC_OK;
}

extern "C" size_t asc_rownorm_loss_bwd_workspace(int64_t n) {
    (void)n;
    return 256 + sizeof(double) * kMaxGrid;
}

extern "C" asc_status asc_rownorm_loss_bwd(const float *Y, int64_t ldy, const float *target, int64_t ldt, int64_t n,
                                           int64_t r, double *loss, float *G, int64_t ldg, void *ws, size_t ws_bytes,
                                           void *stream) {
    const char *who = "asc_rownorm_loss_bwd";
    if (!Y || !target || !loss || !G || n < 1 || r < 1 || ldy < r || ldt < r || ldg < r)
        return fail(ASC_ERR_INVALID, "%s: bad arguments", who);
    ASC_TRY(check_ws(ws, ws_bytes, asc_rownorm_loss_bwd_workspace(n), who));
    double *part = reinterpret_cast<double *>(static_cast<char *>(ws) + 256);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n * 64 + NT - 1) / NT, kMaxGrid));
    hipStream_t s = as_stream(stream);
    rownorm_loss_kernel<<<grid, NT, 0, s>>>(Y, ldy, target, ldt, n, r, G, ldg, part);
    ASC_LAUNCHED();
    sum_to_scalar<<<1, NT, 0, s>>>(part, grid, loss);
    ASC_LAUNCHED();
    return ASC_OK;
}

extern "C" size_t asc_filter_bwd_workspace(int64_t n, int64_t nnz, int64_t r, asc_dtype sig, int p, int ckpt_stride) {
    if (ckpt_stride < 1) ckpt_stride = 1;
    return bwd_ws_layout(n, nnz, r, sig, p, ckpt_stride, nullptr, nullptr);
}

extern "C" asc_status asc_cheb_filter_bwd(const asc_graph *g, const double *lmax, const double *coeffs, int p,
                                          const void *R, asc_dtype sig, int64_t r, int64_t ldr, const void *ckpt,
                                          int ckpt_stride, const float *G, int64_t ldg, float *dW, double *dcoeffs,
                                          void *ws, size_t ws_bytes, void *stream) {
    const char *who = "asc_cheb_filter_bwd";
    ASC_TRY(check_common(g, lmax, p, R, sig, r, ldr, who));
    if (!coeffs || !aligned(coeffs, 8)) return fail(ASC_ERR_INVALID, "%s: coeffs NULL or misaligned", who);
    ASC_TRY(check_block(G, ASC_F32, g->n, r, ldg, who, "G"));
    if (p >= 1 && (!ckpt || ckpt_stride < 1 || !aligned(ckpt, 256)))
        return fail(ASC_ERR_INVALID, "%s: needs the forward checkpoints (ckpt_stride >= 1)", who);
    if (dW && !aligned(dW, 4)) return fail(ASC_ERR_INVALID, "%s: dW misaligned", who);
    if (dcoeffs && !aligned(dcoeffs, 8)) return fail(ASC_ERR_INVALID, "%s: dcoeffs misaligned", who);
    const int c = std::max(1, ckpt_stride);
    const bool store_all = c == 1;
    ASC_TRY(check_ws(ws, ws_bytes, asc_filter_bwd_workspace(g->n, g->nnz, r, sig, p, c), who));
    hipStream_t s = as_stream(stream);
    const int64_t n = g->n, nnz = g->nnz;
    BwdWs B;
    bwd_ws_layout(n, nnz, r, sig, p, c, ws, &B);
    uint32_t *flags = &B.hdr->flags;
    diag_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, g->strength, lmax, B.diag, B.beta, flags, 1);
    ASC_LAUNCHED();
    fill_f64<<<1, 256, 0, s>>>(B.dsum, p + 1);
    ASC_LAUNCHED();
    const bool want_dw = dW != nullptr && p >= 1 && nnz > 0;
    if (dW && nnz > 0) {
        fill_f32<<<grid1(nnz), 256, 0, s>>>(dW, nnz, 0.0f);
        ASC_LAUNCHED();
    }
    if (want_dw) {
        fill_f32<<<grid1(nnz), 256, 0, s>>>(B.mt, nnz, 0.0f);
        fill_f32<<<grid1(n), 256, 0, s>>>(B.mdiag, n, 0.0f);
        transpose_map_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, g->row_ptr, g->col_idx, B.tr, flags);
        ASC_LAUNCHED();
    }
    const Plan P = store_all ? store_plan(g, r, sig) : make_plan(g, r, sig);
    const int grid = grid_for(n, P.lpr);
    const size_t pb = (size_t)n * P.rs * esize(sig);
    auto panel = [&](int q) -> void * { return static_cast<char *>(B.panels) + (size_t)q * pb; };
    void *Acur = panel(c + 1), *Aold = panel(c + 2);
    const size_t ckb = ck_block_bytes(n, r, sig);
    const int64_t ckld = ck_ld_of(r, sig);
    const int nseg = nseg_of(p, c);
    const int64_t tot = n * P.rs;
    const int pg = (int)std::min<int64_t>((tot + 255) / 256, 65536);
    auto pack = [&](const void *src, int64_t ld, int64_t c0, void *dst) {
        if (sig == ASC_F32)
            pack_kernel<float><<<pg, 256, 0, s>>>(n, (const float *)src, ld, c0, r, P.rs, (float *)dst);
        else
            pack_kernel<uint16_t><<<pg, 256, 0, s>>>(n, (const uint16_t *)src, ld, c0, r, P.rs, (uint16_t *)dst);
    };
    for (int sl = 0; sl < P.nslices; ++sl) {
        const int64_t c0 = (int64_t)sl * P.rs;
        if (p == 0) {
            // da_0 = <G, R>: A "init" with coefficient index 0 gives it
            pack(R, ldr, c0, panel(0));
            if (sig == ASC_F32)
                adj_init_kernel<float><<<grid, NT, 0, s>>>(n, G, ldg, c0, r, P.rs, coeffs, 0, (const float *)panel(0),
                                                           (float *)Acur, B.dapart);
            else
                adj_init_kernel<uint16_t><<<grid, NT, 0, s>>>(n, G, ldg, c0, r, P.rs, coeffs, 0,
                                                              (const uint16_t *)panel(0), (uint16_t *)Acur, B.dapart);
            ASC_LAUNCHED();
            da_accum_kernel<<<1, NT, 0, s>>>(B.dapart, grid, kMaxGrid, 0, B.dsum);
            ASC_LAUNCHED();
            continue;
        }
        StepArgs F{};
        F.n = n;
        F.rp = g->row_ptr;
        F.ci = g->col_idx;
        F.w = g->w;
        F.diag = B.diag;
        F.beta = B.beta;
        AdjArgs A{};
        A.n = n;
        A.xcd_bands = (P.var & 4u) ? 1 : 0;
        A.nnz_hint = nnz;
        A.rp = g->row_ptr;
        A.ci = g->col_idx;
        A.w = g->w;
        A.diag = B.diag;
        A.beta = B.beta;
        A.G = G;
        A.ldg = ldg;
        A.c0 = c0;
        A.r = r;
        A.mt = B.mt;
        A.mdiag = B.mdiag;
        if (store_all) {
            // every state is in the store: slot(sl, j) = T_j of this slice
            const size_t spb = panel_bytes(n, P.rs, sig);
            auto slot = [&](int j) -> const void * {
                return static_cast<const char *>(ckpt) + ((size_t)sl * (p + 1) + j) * spb;
            };
            if (sig == ASC_F32)
                adj_init_kernel<float><<<grid, NT, 0, s>>>(n, G, ldg, c0, r, P.rs, coeffs, p, (const float *)slot(p),
                                                           (float *)Acur, B.dapart + (int64_t)p * kMaxGrid);
            else
                adj_init_kernel<uint16_t><<<grid, NT, 0, s>>>(n, G, ldg, c0, r, P.rs, coeffs, p,
                                                              (const uint16_t *)slot(p), (uint16_t *)Acur,
                                                              B.dapart + (int64_t)p * kMaxGrid);
            ASC_LAUNCHED();
            for (int j = p - 1; j >= 0; --j) {
                A.acur = Acur;
                A.aold = Aold;
                A.aout = Aold;
                A.tj = slot(j);
                A.cj = (j == 0) ? 1.0f : 2.0f;
                A.partials = B.dapart + (int64_t)j * kMaxGrid;
                unsigned mode = B_DA | (want_dw ? B_DW : 0u);
                if (j >= 1) mode |= B_OUT;
                if (j == p - 1) mode |= B_TOP;
                A.coeffs = coeffs;
                A.j = j;
                hipError_t e = launch_adj(sig, P.lpr, mode, A, grid, s);
                if (e != hipSuccess) return fail(ASC_ERR_HIP, "adjoint launch failed: %s", hipGetErrorString(e));
                std::swap(Acur, Aold);
            }
            da_accum_kernel<<<p + 1, NT, 0, s>>>(B.dapart, grid, kMaxGrid, p, B.dsum);
            ASC_LAUNCHED();
            continue;
        }
        for (int seg = nseg - 1; seg >= 0; --seg) {
            const int sc = seg * c;
            const int hi = std::min(sc + c, p);
            const int last_state = (hi == p) ? p : hi - 1;  // recompute T_sc .. T_last_state
            const char *ck0 = static_cast<const char *>(ckpt) + ((size_t)seg * 2) * ckb;
            pack(ck0, ckld, c0, panel(0));
            pack(ck0 + ckb, ckld, c0, panel(1));
            ASC_LAUNCHED();
            for (int q = 1; q + sc < last_state; ++q) {
                F.cur = panel(q);
                F.prev = panel(q - 1);
                F.out = panel(q + 1);
                F.j = sc + q;
                hipError_t e = launch_step(sig, P.lpr, 0u, 0u, F, grid, s);
                if (e != hipSuccess) return fail(ASC_ERR_HIP, "recompute launch failed: %s", hipGetErrorString(e));
            }
            if (hi == p) {
                // A_p = a_p G and da_p = <G, T_p>
                if (sig == ASC_F32)
                    adj_init_kernel<float><<<grid, NT, 0, s>>>(n, G, ldg, c0, r, P.rs, coeffs, p,
                                                               (const float *)panel(p - sc), (float *)Acur,
                                                               B.dapart + (int64_t)p * kMaxGrid);
                else
                    adj_init_kernel<uint16_t><<<grid, NT, 0, s>>>(n, G, ldg, c0, r, P.rs, coeffs, p,
                                                                  (const uint16_t *)panel(p - sc), (uint16_t *)Acur,
                                                                  B.dapart + (int64_t)p * kMaxGrid);
                ASC_LAUNCHED();
            }
            for (int j = hi - 1; j >= sc; --j) {
                A.acur = Acur;
                A.aold = Aold;
                A.aout = Aold;
                A.tj = panel(j - sc);
                A.cj = (j == 0) ? 1.0f : 2.0f;
                A.partials = B.dapart + (int64_t)j * kMaxGrid;
                unsigned mode = B_DA | (want_dw ? B_DW : 0u);
                if (j >= 1) mode |= B_OUT;
                if (j == p - 1) mode |= B_TOP;
                A.coeffs = coeffs;
                A.j = j;
                hipError_t e;
                e = launch_adj(sig, P.lpr, mode, A, grid, s);
                if (e != hipSuccess) return fail(ASC_ERR_HIP, "adjoint launch failed: %s", hipGetErrorString(e));
                std::swap(Acur, Aold);
            }
        }
        da_accum_kernel<<<p + 1, NT, 0, s>>>(B.dapart, grid, kMaxGrid, p, B.dsum);
        ASC_LAUNCHED();
    }
    if (want_dw) {
        dw_final_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, g->row_ptr, g->col_idx, B.tr, B.mt, B.mdiag,
                                                                    lmax, dW);
        ASC_LAUNCHED();
    }
    if (dcoeffs) {
        copy_f64<<<(p + 1 + 255) / 256, 256, 0, s>>>(B.dsum, dcoeffs, p + 1);
        ASC_LAUNCHED();
    }
    return ASC_OK;
}
