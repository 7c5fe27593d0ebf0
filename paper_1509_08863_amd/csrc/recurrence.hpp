// Recurrence-step machinery shared by the forward filter, the moment pass,
// the backward pass and the batched launch (see cheb.hip for the design).
#pragma once

#include "common.hpp"

#include <algorithm>

namespace asc {

// process-wide tuning table: kernel configuration per (n, nnz, r, dtype)
struct TuneKey {
    int64_t n, nnz, r;
    int dt;
    bool operator==(const TuneKey &o) const { return n == o.n && nnz == o.nnz && r == o.r && dt == o.dt; }
};
struct TuneEntry {
    TuneKey key;
    int rs;       // slice width (columns)
    int var;      // kernel variant bits
    float ms;     // measured time of one recurrence step over all columns
};

bool tuned(int64_t n, int64_t nnz, int64_t r, asc_dtype dt, TuneEntry *out);

namespace {

constexpr int NT = 256;          // threads per block (4 wavefronts)
constexpr int kMaxGrid = 8192;   // cap of blocks per step launch (grid-stride beyond)
constexpr unsigned M_FIRST = 1u;  // step 0: T_1 = Lt T_0 (there is no T_{-1})
constexpr unsigned M_YACC = 2u;   // Y += a_{j+1} T_{j+1}; with M_FIRST: Y = a_0 T_0 + a_1 T_1
constexpr unsigned M_PART = 4u;   // write float64 partial sums
constexpr unsigned M_YPAIR = 8u;  // with M_YACC: Y += a_j T_j + a_{j+1} T_{j+1} (Y touched every other step)

// ---------------------------------------------------------------------------
// storage element types: float (4 per 16 B) and bfloat16 bits (8 per 16 B)
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

template <typename TS> struct St;
template <> struct St<float> { static constexpr int VN = 4; typedef v4f raw; };
template <> struct St<uint16_t> { static constexpr int VN = 8; typedef v4u raw; };

// loads/stores with an optional non-temporal hint (streamed data that is not
// re-read in this step: CSR arrays, T_{j-1}, Y)
template <bool NTH, typename T>
__device__ __forceinline__ T ldx(const T *p) {
    if constexpr (NTH) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NTH, typename T>
__device__ __forceinline__ void stx(T *p, T v) {
    if constexpr (NTH) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <bool NTH = false>
__device__ __forceinline__ v4f ldraw(const float *p) { return ldx<NTH>(reinterpret_cast<const v4f *>(p)); }
template <bool NTH = false>
__device__ __forceinline__ v4u ldraw(const uint16_t *p) { return ldx<NTH>(reinterpret_cast<const v4u *>(p)); }

__device__ __forceinline__ void unpack(const v4f &x, float (&v)[4]) {
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
}
__device__ __forceinline__ void unpack(const v4u &x, float (&v)[8]) {
    v[0] = bf16_lo(x.x); v[1] = bf16_hi(x.x); v[2] = bf16_lo(x.y); v[3] = bf16_hi(x.y);
    v[4] = bf16_lo(x.z); v[5] = bf16_hi(x.z); v[6] = bf16_lo(x.w); v[7] = bf16_hi(x.w);
}
// acc += w * x (one fused multiply-add per element, in element order)
__device__ __forceinline__ void fma_raw(float (&acc)[4], float w, const v4f &x) {
    acc[0] = fmaf(w, x.x, acc[0]); acc[1] = fmaf(w, x.y, acc[1]);
    acc[2] = fmaf(w, x.z, acc[2]); acc[3] = fmaf(w, x.w, acc[3]);
}
__device__ __forceinline__ void fma_raw(float (&acc)[8], float w, const v4u &x) {
    acc[0] = fmaf(w, bf16_lo(x.x), acc[0]); acc[1] = fmaf(w, bf16_hi(x.x), acc[1]);
    acc[2] = fmaf(w, bf16_lo(x.y), acc[2]); acc[3] = fmaf(w, bf16_hi(x.y), acc[3]);
    acc[4] = fmaf(w, bf16_lo(x.z), acc[4]); acc[5] = fmaf(w, bf16_hi(x.z), acc[5]);
    acc[6] = fmaf(w, bf16_lo(x.w), acc[6]); acc[7] = fmaf(w, bf16_hi(x.w), acc[7]);
}
// store v rounded to the storage type; `r` receives the stored values
__device__ __forceinline__ v4f st16(float *p, const float (&v)[4], float (&r)[4]) {
    v4f x = {v[0], v[1], v[2], v[3]};
    *reinterpret_cast<v4f *>(p) = x;
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = v[q];
    return x;
}
__device__ __forceinline__ v4u st16(uint16_t *p, const float (&v)[8], float (&r)[8]) {
    v4u x;
    x.x = pack_bf16x2(v[0], v[1]); x.y = pack_bf16x2(v[2], v[3]);
    x.z = pack_bf16x2(v[4], v[5]); x.w = pack_bf16x2(v[6], v[7]);
    *reinterpret_cast<v4u *>(p) = x;
    unpack(x, r);
    return x;
}

struct StepArgs {
    int64_t n;
    const int32_t *rp;
    const int32_t *ci;
    const float *w;        // nullptr: unit weights
    const float *diag;     // d_i (float32)
    const float *beta;     // beta[0] = -4/lmax
    const void *cur;       // panel T_j
    const void *prev;      // panel T_{j-1} (unused with M_FIRST)
    void *out;             // panel T_{j+1} (may equal prev)
    float *Y;              // caller block (slice columns c0..)
    int64_t ldy, c0, r;
    const double *coeffs;  // a_0..a_p
    int j;                 // this step produces T_{j+1}
    double *partials;      // [gridDim.x][3]
    void *ck_a;            // if set: T_j row-major checkpoint block (columns c0.., ld ck_ld)
    void *ck_b;            // if set: T_{j+1} checkpoint block
    int64_t ck_ld;
    int64_t pstride;       // NP > 1: elements from one slice's panel to the next one's
    int64_t ystride;       // gridDim.y > 1 (state-store passes of small graphs): bytes from one
                           // slice's panels (cur, prev, out) to the next slice's; no Y, no partials
};

// The rest of a row's step for one panel: T_{j+1} from the gathered sum, its
// store and checkpoints, the Y update of caller columns c0.., partial sums.
template <typename TS, int LPR, unsigned MODE, unsigned VAR>
__device__ __forceinline__ void finish_row(const StepArgs &A, const TS *__restrict__ cur, const TS *__restrict__ prv,
                                           TS *__restrict__ out, const int64_t c0, const int64_t row, const int t,
                                           const float d, const float beta, const float aj1, const float a0,
                                           const float (&acc)[St<TS>::VN], double &p_own, double &p_cross,
                                           double &p_sq) {
    constexpr bool NTH = (VAR & 1u) != 0;
    constexpr int VN = St<TS>::VN;
    constexpr int RS = LPR * VN;
    typedef typename St<TS>::raw raw_t;
    float own[VN], nxt[VN], stv[VN];
    const raw_t own_raw = ldraw(cur + row * RS + t * VN);
    unpack(own_raw, own);
    if (A.ck_a) *reinterpret_cast<raw_t *>(static_cast<TS *>(A.ck_a) + row * A.ck_ld + c0 + t * VN) = own_raw;
    if (MODE & M_FIRST) {
#pragma unroll
        for (int q = 0; q < VN; ++q) nxt[q] = 0.5f * fmaf(d, own[q], beta * acc[q]);
    } else {
        float pv[VN];
        unpack(ldraw<NTH>(prv + row * RS + t * VN), pv);
#pragma unroll
        for (int q = 0; q < VN; ++q) nxt[q] = fmaf(d, own[q], fmaf(beta, acc[q], -pv[q]));
    }
    const raw_t nxt_raw = st16(out + row * RS + t * VN, nxt, stv);
    if (A.ck_b) *reinterpret_cast<raw_t *>(static_cast<TS *>(A.ck_b) + row * A.ck_ld + c0 + t * VN) = nxt_raw;
    if (MODE & M_YACC) {
        const int64_t cbase = c0 + (int64_t)t * VN;
        float *yrow = A.Y + row * A.ldy + cbase;
        if (cbase + VN <= A.r) {
#pragma unroll
            for (int q = 0; q < VN; q += 4) {
                v4f y;
                if (MODE & M_FIRST) {
                    y.x = a0 * own[q] + aj1 * nxt[q];
                    y.y = a0 * own[q + 1] + aj1 * nxt[q + 1];
                    y.z = a0 * own[q + 2] + aj1 * nxt[q + 2];
                    y.w = a0 * own[q + 3] + aj1 * nxt[q + 3];
                } else if (MODE & M_YPAIR) {
                    // a0 carries a_j here
                    y = ldx<NTH>(reinterpret_cast<const v4f *>(yrow + q));
                    y.x += fmaf(a0, own[q], aj1 * nxt[q]);
                    y.y += fmaf(a0, own[q + 1], aj1 * nxt[q + 1]);
                    y.z += fmaf(a0, own[q + 2], aj1 * nxt[q + 2]);
                    y.w += fmaf(a0, own[q + 3], aj1 * nxt[q + 3]);
                } else {
                    y = ldx<NTH>(reinterpret_cast<const v4f *>(yrow + q));
                    y.x = fmaf(aj1, nxt[q], y.x);
                    y.y = fmaf(aj1, nxt[q + 1], y.y);
                    y.z = fmaf(aj1, nxt[q + 2], y.z);
                    y.w = fmaf(aj1, nxt[q + 3], y.w);
                }
                stx<NTH>(reinterpret_cast<v4f *>(yrow + q), y);
            }
        } else {
#pragma unroll
            for (int q = 0; q < VN; ++q) {
                if (cbase + q < A.r) {
                    if (MODE & M_FIRST)
                        yrow[q] = a0 * own[q] + aj1 * nxt[q];
                    else if (MODE & M_YPAIR)
                        yrow[q] += fmaf(a0, own[q], aj1 * nxt[q]);
                    else
                        yrow[q] = fmaf(aj1, nxt[q], yrow[q]);
                }
            }
        }
    }
    if (MODE & M_PART) {
#pragma unroll
        for (int q = 0; q < VN; ++q) {
            const double o = own[q], x = stv[q];
            if (MODE & M_FIRST) p_own += o * o;
            p_cross += x * o;
            p_sq += x * x;
        }
    }
}

// Kernel variants (VAR bits): bit 0 = non-temporal hints on the streamed
// arrays.  The neighbour loop gathers U rows per iteration and prefetches the
// next U column indices / weights while the gathers are in flight.
// One row of a recurrence step (the LPR lanes of row group `t`): gather
// sum_k w_ik T_j[k], form T_{j+1}[i] (or T_1 at the first step), store it (and
// the checkpoints), update Y and the float64 partial sums.  With NP > 1 one
// launch covers NP consecutive slices (panels A.pstride elements apart,
// caller columns c0 + q RS): the row's column indices and weights are read
// once for all of them and every neighbour costs NP gathers.
template <typename TS, int LPR, unsigned MODE, unsigned VAR, int NP = 1>
__device__ __forceinline__ void step_row(const StepArgs &A, const int64_t row, const int t, const float beta,
                                         const float aj1, const float a0, double &p_own, double &p_cross,
                                         double &p_sq) {
    constexpr bool NTH = (VAR & 1u) != 0;
    constexpr int VN = St<TS>::VN;
    constexpr int RS = LPR * VN;
    constexpr int U = NP == 1 ? 8 : 4;
    typedef typename St<TS>::raw raw_t;
    const TS *__restrict__ cur = static_cast<const TS *>(A.cur);
    const TS *__restrict__ prv = static_cast<const TS *>(A.prev);
    TS *__restrict__ out = static_cast<TS *>(A.out);
    const int64_t ps = NP == 1 ? 0 : A.pstride;
    const bool weighted = A.w != nullptr;
    const int32_t e0 = ldx<NTH>(A.rp + row), e1 = ldx<NTH>(A.rp + row + 1);
    float acc[NP][VN];
#pragma unroll
    for (int pn = 0; pn < NP; ++pn)
#pragma unroll
        for (int q = 0; q < VN; ++q) acc[pn][q] = 0.0f;
    const TS *base = cur + t * VN;
    if constexpr ((VAR & 2u) != 0) {
        // cooperative index loads: the lanes of the row group load the next U
        // column indices / weights with one coalesced request (M per lane) and
        // broadcast them inside the group, instead of every lane loading all U
        constexpr int M = (LPR >= U) ? 1 : U / LPR;
        const int gbase = (int)(threadIdx.x & 63) & ~(LPR - 1);
        int32_t mk[M];
        float mw[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int32_t ee = e0 + t + LPR * m;
            mk[m] = (int32_t)row;
            mw[m] = 0.0f;
            if ((LPR < U || t < U) && ee < e1) {
                mk[m] = ldx<NTH>(A.ci + ee);
                mw[m] = weighted ? ldx<NTH>(A.w + ee) : 1.0f;
            }
        }
        for (int32_t e = e0; e < e1; e += U) {
            int32_t kc[U];
            float wc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int src = gbase + (LPR < U ? (u % LPR) : u);
                kc[u] = __shfl(mk[LPR < U ? u / LPR : 0], src, 64);
                wc[u] = __shfl(mw[LPR < U ? u / LPR : 0], src, 64);
            }
            raw_t v[U][NP];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int pn = 0; pn < NP; ++pn) v[u][pn] = ldraw(base + pn * ps + (int64_t)kc[u] * RS);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int32_t ee = e + U + t + LPR * m;
                mk[m] = (int32_t)row;
                mw[m] = 0.0f;
                if ((LPR < U || t < U) && ee < e1) {
                    mk[m] = ldx<NTH>(A.ci + ee);
                    mw[m] = weighted ? ldx<NTH>(A.w + ee) : 1.0f;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int pn = 0; pn < NP; ++pn) fma_raw(acc[pn], wc[u], v[u][pn]);
        }
    } else {
        // padding slots gather the row itself with weight 0
        int32_t kn[U];
        float wn[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            kn[u] = (int32_t)row;
            wn[u] = 0.0f;
            if (e0 + u < e1) {
                kn[u] = ldx<NTH>(A.ci + e0 + u);
                wn[u] = weighted ? ldx<NTH>(A.w + e0 + u) : 1.0f;
            }
        }
        for (int32_t e = e0; e < e1; e += U) {
            int32_t kc[U];
            float wc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                kc[u] = kn[u];
                wc[u] = wn[u];
            }
            raw_t v[U][NP];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int pn = 0; pn < NP; ++pn) v[u][pn] = ldraw(base + pn * ps + (int64_t)kc[u] * RS);
            const int32_t en = e + U;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                kn[u] = (int32_t)row;
                wn[u] = 0.0f;
                if (en + u < e1) {
                    kn[u] = ldx<NTH>(A.ci + en + u);
                    wn[u] = weighted ? ldx<NTH>(A.w + en + u) : 1.0f;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int pn = 0; pn < NP; ++pn) fma_raw(acc[pn], wc[u], v[u][pn]);
        }
    }
    const float d = ldx<NTH>(A.diag + row);
#pragma unroll
    for (int pn = 0; pn < NP; ++pn)
        finish_row<TS, LPR, MODE, VAR>(A, cur + pn * ps, prv + pn * ps, out + pn * ps, A.c0 + (int64_t)pn * RS, row,
                                       t, d, beta, aj1, a0, acc[pn], p_own, p_cross, p_sq);
}

template <typename TS, int LPR, unsigned MODE, unsigned VAR, int NP = 1>
__global__ __launch_bounds__(NT) void cheb_step(StepArgs A) {
    if (gridDim.y > 1) {
        // one slice per blockIdx.y: its own panels, A.ystride bytes apart
        const int64_t off = (int64_t)blockIdx.y * A.ystride;
        A.cur = static_cast<const char *>(A.cur) + off;
        A.prev = A.prev ? static_cast<const char *>(A.prev) + off : nullptr;
        A.out = static_cast<char *>(A.out) + off;
    }
    constexpr int RPW = 64 / LPR;
    constexpr int ROWS = RPW * (NT / 64);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int t = lane % LPR;
    const int sub = lane / LPR;
    const float beta = A.beta[0];
    const float aj1 = (MODE & M_YACC) ? (float)A.coeffs[A.j + 1] : 0.0f;
    const float a0 = !(MODE & M_YACC) ? 0.0f
                     : (MODE & M_FIRST) ? (float)A.coeffs[0]
                     : (MODE & M_YPAIR) ? (float)A.coeffs[A.j] : 0.0f;
    double p_own = 0.0, p_cross = 0.0, p_sq = 0.0;
    const int64_t ntiles = (A.n + ROWS - 1) / ROWS;
    if ((VAR & 4u) != 0 && gridDim.x >= 8) {
        // XCD-contiguous tiles: workgroups are dispatched round-robin over the
        // 8 XCDs, so workgroup b runs on XCD b % 8; give XCD x the x-th
        // contiguous eighth of the rows, so that each XCD's L2 serves one band
        // of a locality-ordered graph.  (A permutation of the tile order only.)
        const int64_t xcd = blockIdx.x % 8, loc = blockIdx.x / 8;
        const int64_t nx = (gridDim.x - xcd + 7) / 8;  // workgroups on this XCD
        const int64_t chunk = (ntiles + 7) / 8;
        const int64_t t0 = xcd * chunk, t1 = t0 + chunk < ntiles ? t0 + chunk : ntiles;
        for (int64_t tile = t0 + loc; tile < t1; tile += nx) {
            const int64_t row = tile * ROWS + (int64_t)wave * RPW + sub;
            if (row >= A.n) continue;
            step_row<TS, LPR, MODE, VAR, NP>(A, row, t, beta, aj1, a0, p_own, p_cross, p_sq);
        }
    } else {
        for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
            const int64_t row = tile * ROWS + (int64_t)wave * RPW + sub;
            if (row >= A.n) continue;
            step_row<TS, LPR, MODE, VAR, NP>(A, row, t, beta, aj1, a0, p_own, p_cross, p_sq);
        }
    }
    if (MODE & M_PART) {
        __shared__ double lds[3 * NT / 64];
        double v[3] = {p_own, p_cross, p_sq};
        block_sum<3, NT>(v, lds);
        if (threadIdx.x == 0) {
            double *pp = A.partials + (int64_t)blockIdx.x * 3;
            pp[0] = v[0];
            pp[1] = v[1];
            pp[2] = v[2];
        }
    }
}

// d_i = 4 s_i / lmax - 2 (float32), beta = -4 / lmax; flags a bad lmax
__global__ void diag_kernel(int64_t n, const double *__restrict__ s, const double *__restrict__ lmax,
                            float *__restrict__ diag, float *__restrict__ beta, uint32_t *flags, int clear_flags) {
    const double L = lmax[0];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        beta[0] = (float)(-4.0 / L);
        uint32_t f = clear_flags ? 0u : flags[0];
        if (!(L > 0.0) || isinf(L)) f |= ASC_FLAG_NONFINITE;
        flags[0] = f;
    }
    if (i < n) diag[i] = (float)(4.0 * s[i] / L - 2.0);
}

// panel[i][c] = R[i][c0 + c] for c0 + c < r, else 0
template <typename TS>
__global__ void pack_kernel(int64_t n, const TS *__restrict__ R, int64_t ldr, int64_t c0, int64_t r, int rs,
                            TS *__restrict__ panel) {
    const int64_t total = n * rs;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q / rs;
        const int64_t c = q - i * rs;
        panel[q] = (c0 + c < r) ? R[i * ldr + c0 + c] : TS(0);
    }
}

// Y = a_0 R (order 0 filter)
template <typename TS>
__global__ void scale_copy_kernel(int64_t n, int64_t r, const TS *__restrict__ R, int64_t ldr,
                                  const double *__restrict__ coeffs, float *__restrict__ Y, int64_t ldy) {
    const float a0 = (float)coeffs[0];
    const int64_t total = n * r;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q / r, c = q - i * r;
        float x;
        if constexpr (sizeof(TS) == 4) x = (float)R[i * ldr + c];
        else x = __uint_as_float(((uint32_t)R[i * ldr + c]) << 16);
        Y[i * ldy + c] = a0 * x;
    }
}

// sums of [nparts][3] partials in block order; out[3]
__global__ void sum_partials_kernel(int nparts, const double *__restrict__ part, int nsteps, int64_t step_stride,
                                    double *__restrict__ out) {
    // one block per step; out[step*3 + q]
    __shared__ double lds[3 * NT / 64];
    const int step = blockIdx.x;
    if (step >= nsteps) return;
    const double *p = part + step * step_stride;
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nparts; b += NT) {
        v[0] += p[b * 3 + 0];
        v[1] += p[b * 3 + 1];
        v[2] += p[b * 3 + 2];
    }
    block_sum<3, NT>(v, lds);
    if (threadIdx.x == 0) {
        out[step * 3 + 0] = v[0];
        out[step * 3 + 1] = v[1];
        out[step * 3 + 2] = v[2];
    }
}

// growth / finiteness check of one slice: |T_p|^2 vs |T_0|^2
__global__ void growth_check_kernel(const double *__restrict__ first, const double *__restrict__ last,
                                    uint32_t *flags) {
    if (threadIdx.x != 0) return;
    const double n0 = first[0], np = last[2];
    uint32_t f = flags[0];
    if (!isfinite(n0) || !isfinite(np)) f |= ASC_FLAG_NONFINITE;
    else if (np > 2.25 * n0 * (1.0 + 1e-6) + 1e-300) f |= ASC_FLAG_GROWTH;
    flags[0] = f;
}

// mu_0..mu_p from per-slice per-step sums [nslices][steps][3]
__global__ void moments_finalize_kernel(const double *__restrict__ sums, int nslices, int steps, int p,
                                        double *__restrict__ mu, uint32_t *flags) {
    if (threadIdx.x != 0) return;
    auto tot = [&](int step, int q) {
        double s = 0.0;
        for (int sl = 0; sl < nslices; ++sl) s += sums[((int64_t)sl * steps + step) * 3 + q];
        return s;
    };
    const double mu0 = tot(0, 0);
    const double mu1 = tot(0, 1);
    mu[0] = mu0;
    bool bad = !isfinite(mu0);
    for (int s = 0; s < steps; ++s) {
        const int jo = 2 * s + 1, je = 2 * s + 2;
        const double cross = tot(s, 1), sq = tot(s, 2);
        if (jo <= p) mu[jo] = (s == 0) ? cross : 2.0 * cross - mu1;
        if (je <= p) mu[je] = 2.0 * sq - mu0;
        if (!isfinite(sq)) bad = true;
        else if (sq > 2.25 * mu0 * (1.0 + 1e-6) + 1e-300) flags[0] |= ASC_FLAG_GROWTH;
    }
    if (bad) flags[0] |= ASC_FLAG_NONFINITE;
}

// ---------------------------------------------------------------------------
// host-side planning and launch
// ---------------------------------------------------------------------------
struct Plan {
    int lpr;     // lanes per row (2, 4, 8, 16)
    int rs;      // panel width in elements = lpr * VN
    int nslices;
    unsigned var;
    int np;      // slices per launch: 1, or all of them (variant bit 3)
};

int vn_of(asc_dtype dt) { return dt == ASC_F32 ? 4 : 8; }

int default_rs(int64_t r, asc_dtype dt) {
    const int vn = vn_of(dt);
    // smallest supported width covering r, capped at 32 float32 / 64 bfloat16 columns
    const int cap = dt == ASC_F32 ? 32 : 64;
    int rs = 2 * vn;
    while (rs < r && rs < cap) rs *= 2;
    return rs;
}

}  // namespace

namespace {

bool valid_rs(int rs, asc_dtype dt) {
    const int vn = dt == ASC_F32 ? 4 : 8;
    return rs == 2 * vn || rs == 4 * vn || rs == 8 * vn || rs == 16 * vn;
}

// Variant bit 3 puts every slice in one launch (np = nslices) where the
// multi-panel kernel exists: 8 lanes per row and 2 to 4 slices.
bool multi_panel(int lpr, int nslices) { return lpr == 8 && nslices >= 2 && nslices <= 4; }

Plan plan_for(int rs, unsigned var, int64_t r, asc_dtype dt) {
    Plan P;
    const int vn = vn_of(dt);
    P.rs = rs;
    P.lpr = rs / vn;
    P.nslices = (int)((r + rs - 1) / rs);
    P.var = var;
    P.np = ((var & 8u) != 0 && multi_panel(P.lpr, P.nslices)) ? P.nslices : 1;
    return P;
}

Plan make_plan(const asc_graph *g, int64_t r, asc_dtype dt) {
    TuneEntry e;
    if (tuned(g->n, g->nnz, r, dt, &e) && valid_rs(e.rs, dt)) return plan_for(e.rs, (unsigned)e.var, r, dt);
    return plan_for(default_rs(r, dt), 0u, r, dt);
}

// The state store (every T_j kept, panel layout [slice][j][n x rs]) always
// uses the default slice width for (r, dtype), whatever the tuning says, so its
// size and layout cannot change between sizing, the forward pass that writes it
// and the backward pass that reads it; the tuned variant bits still apply.
Plan store_plan(const asc_graph *g, int64_t r, asc_dtype dt) {
    TuneEntry e;
    const unsigned var = tuned(g->n, g->nnz, r, dt, &e) ? (unsigned)e.var : 0u;
    return plan_for(default_rs(r, dt), var, r, dt);
}

int grid_for(int64_t n, int lpr) {
    const int64_t rows = (64 / lpr) * (NT / 64);
    int64_t b = (n + rows - 1) / rows;
    b = std::max<int64_t>(1, std::min<int64_t>(b, kMaxGrid));
    return (int)b;
}

template <typename TS, int LPR, unsigned VAR, int NP = 1>
hipError_t launch_step_v(unsigned mode, const StepArgs &A, dim3 grid, hipStream_t s) {
    switch (mode) {
        case 0: cheb_step<TS, LPR, 0, VAR, NP><<<grid, NT, 0, s>>>(A); break;
        case 1: cheb_step<TS, LPR, 1, VAR, NP><<<grid, NT, 0, s>>>(A); break;
        case 2: cheb_step<TS, LPR, 2, VAR, NP><<<grid, NT, 0, s>>>(A); break;
        case 3: cheb_step<TS, LPR, 3, VAR, NP><<<grid, NT, 0, s>>>(A); break;
        case 4: cheb_step<TS, LPR, 4, VAR, NP><<<grid, NT, 0, s>>>(A); break;
        case 5: cheb_step<TS, LPR, 5, VAR, NP><<<grid, NT, 0, s>>>(A); break;
        case 6: cheb_step<TS, LPR, 6, VAR, NP><<<grid, NT, 0, s>>>(A); break;
        case 7: cheb_step<TS, LPR, 7, VAR, NP><<<grid, NT, 0, s>>>(A); break;
        case 10: cheb_step<TS, LPR, 10, VAR, NP><<<grid, NT, 0, s>>>(A); break;
        case 14: cheb_step<TS, LPR, 14, VAR, NP><<<grid, NT, 0, s>>>(A); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TS, int LPR>
hipError_t launch_step_t(unsigned mode, unsigned var, const StepArgs &A, dim3 grid, hipStream_t s) {
    switch (var & 7u) {
        case 1u: return launch_step_v<TS, LPR, 1u>(mode, A, grid, s);
        case 2u: return launch_step_v<TS, LPR, 2u>(mode, A, grid, s);
        case 3u: return launch_step_v<TS, LPR, 3u>(mode, A, grid, s);
        case 4u: return launch_step_v<TS, LPR, 4u>(mode, A, grid, s);
        case 5u: return launch_step_v<TS, LPR, 5u>(mode, A, grid, s);
        case 6u: return launch_step_v<TS, LPR, 6u>(mode, A, grid, s);
        case 7u: return launch_step_v<TS, LPR, 7u>(mode, A, grid, s);
        default: return launch_step_v<TS, LPR, 0u>(mode, A, grid, s);
    }
}

hipError_t launch_step(asc_dtype dt, int lpr, unsigned var, unsigned mode, const StepArgs &A, dim3 grid,
                       hipStream_t s) {
    if (dt == ASC_F32) {
        switch (lpr) {
            case 2: return launch_step_t<float, 2>(mode, var, A, grid, s);
            case 4: return launch_step_t<float, 4>(mode, var, A, grid, s);
            case 8: return launch_step_t<float, 8>(mode, var, A, grid, s);
            case 16: return launch_step_t<float, 16>(mode, var, A, grid, s);
        }
    } else {
        switch (lpr) {
            case 2: return launch_step_t<uint16_t, 2>(mode, var, A, grid, s);
            case 4: return launch_step_t<uint16_t, 4>(mode, var, A, grid, s);
            case 8: return launch_step_t<uint16_t, 8>(mode, var, A, grid, s);
            case 16: return launch_step_t<uint16_t, 16>(mode, var, A, grid, s);
        }
    }
    return hipErrorInvalidValue;
}

// Y accumulation of recurrence step j >= 1 of an order-p filter (step j
// forms T_{j+1}): with float32 states, even steps add the pair
// a_j T_j + a_{j+1} T_{j+1}, odd steps leave Y alone, except the last step,
// which adds its own a_p T_p; step 0 writes a_0 T_0 + a_1 T_1.  Every term is
// added exactly once.  With bfloat16 states every step adds its T_{j+1} as
// computed, before rounding to storage (T_j as read back would be rounded).
unsigned y_mode(int j, int p, asc_dtype dt) {
    if (dt != ASC_F32) return M_YACC;
    if (j % 2 == 0) return M_YACC | M_YPAIR;
    return j == p - 1 ? M_YACC : 0u;
}

size_t esize(asc_dtype dt) { return dt == ASC_F32 ? 4 : 2; }

// checkpoint blocks: (T_{sc}, T_{sc+1}) for segment starts sc = 0, c, 2c, ... < p,
// each row-major n x ck_ld in the storage type; ck_ld holds the widest slice
int64_t ck_ld_of(int64_t r, asc_dtype dt) {
    const int64_t w = dt == ASC_F32 ? 64 : 128;
    return (r + w - 1) / w * w;
}
int nseg_of(int p, int c) { return p <= 0 ? 0 : (p + c - 1) / c; }
size_t panel_bytes(int64_t n, int rs, asc_dtype dt) { return ((size_t)n * rs * esize(dt) + 255) & ~size_t(255); }
size_t ck_block_bytes(int64_t n, int64_t r, asc_dtype dt) {
    return ((size_t)n * ck_ld_of(r, dt) * esize(dt) + 255) & ~size_t(255);
}

// workspace layout shared by the filter and the moment pass
struct FilterWs {
    WsHeader *hdr;
    float *diag;
    float *beta;
    double *part;      // [steps_part][kMaxGrid][3]
    double *sums;      // [nslices][steps][3]
    double *first;     // [3]
    void *panelA;
    void *panelB;
};

size_t filter_ws_layout(int64_t n, int rs_max, int nslices, asc_dtype dt, int steps_part, int steps_sum,
                        void *ws, FilterWs *out) {
    Arena a(ws);
    FilterWs f;
    f.hdr = a.take<WsHeader>(1);
    f.diag = a.take<float>(n);
    f.beta = a.take<float>(64);
    f.part = a.take<double>((size_t)steps_part * kMaxGrid * 3);
    f.sums = a.take<double>((size_t)nslices * steps_sum * 3);
    f.first = a.take<double>(64);
    // room for up to 4 slice panels, each rounded up to 256 bytes
    f.panelA = a.take<char>((size_t)n * rs_max * esize(dt) + 4 * 256);
    f.panelB = a.take<char>((size_t)n * rs_max * esize(dt) + 4 * 256);
    if (out) *out = f;
    return a.size();
}

int rs_for_ws(int64_t r, asc_dtype dt) {
    // the workspace must hold the widest panel any plan may pick, and the
    // panels of every slice when one launch covers them all
    const int w8 = 8 * vn_of(dt);
    const int64_t ns8 = (r + w8 - 1) / w8;
    const int all = multi_panel(8, (int)std::min<int64_t>(ns8, 5)) ? (int)(ns8 * w8) : 0;
    return std::max(std::max(default_rs(r, dt), dt == ASC_F32 ? 64 : 128), all);
}

asc_status check_common(const asc_graph *g, const double *lmax, int p, const void *R, asc_dtype sig, int64_t r,
                        int64_t ldr, const char *who) {
    ASC_TRY(check_graph_args(g, true, who));
    if (!lmax || !aligned(lmax, 8)) return fail(ASC_ERR_INVALID, "%s: lmax NULL or misaligned", who);
    if (p < 0 || p > 100000) return fail(ASC_ERR_INVALID, "%s: p=%d not in [0, 100000]", who, p);
    ASC_TRY(check_block(R, sig, g->n, r, ldr, who, "R"));
    return ASC_OK;
}

}  // namespace
}  // namespace asc
