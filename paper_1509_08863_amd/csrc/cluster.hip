// Feature post-processing and clustering: row normalisation of the filtered
// signals (footnote of Sec. 2.1) and k-means with the Euclidean distance
// (Sec. 2.2 step 4; step 6 of the algorithm in Sec. 4.1).
#include "common.hpp"
#include "cluster.hpp"

#include <algorithm>

namespace asc {
namespace {

constexpr int NT = 256;

// Several independent problems in one launch: problem b = blockIdx.y reads
// feature block b / fdiv (replicates of one realisation share their features)
// and owns centroid block b, label block b and init-row block b.
struct Bat {
    int64_t f;       // elements between feature blocks
    int fdiv;        // problems per feature block
    int64_t c;       // elements between centroid blocks
    int64_t l;       // elements between label / distance blocks
    int64_t rows;    // elements between init-row blocks
    // optional per-problem stamps: problem b is skipped (every block of it
    // returns at once) while stamp[b] < want; an assignment that changes a
    // label of problem b sets stamp[b] = mark (when mark != 0)
    uint32_t *stamp;
    uint32_t want;
    uint32_t mark;
};
__device__ __forceinline__ int64_t fblk(const Bat &b, unsigned y) { return (int64_t)(y / b.fdiv) * b.f; }
__device__ __forceinline__ bool idle(const Bat &b) { return b.stamp && b.stamp[blockIdx.y] < b.want; }

// one wavefront per row: |y_i| accumulated in float64, y_i /= |y_i|
__global__ __launch_bounds__(NT) void normalize_kernel(float *__restrict__ Y, int64_t n, int64_t r, int64_t ldy,
                                                       float *__restrict__ norms) {
    const int lane = threadIdx.x & 63;
    const int64_t row0 = ((int64_t)blockIdx.x * NT + threadIdx.x) >> 6;
    const int64_t stride = ((int64_t)gridDim.x * NT) >> 6;
    for (int64_t i = row0; i < n; i += stride) {
        float *y = Y + i * ldy;
        double s = 0.0;
        for (int64_t c = lane; c < r; c += 64) {
            const double v = y[c];
            s += v * v;
        }
        s = wave_sum(s);
        const double nrm = sqrt(s);
        if (nrm > 0.0) {
            for (int64_t c = lane; c < r; c += 64) y[c] = (float)((double)y[c] / nrm);
        }
        if (norms && lane == 0) norms[i] = (float)nrm;
    }
}

__global__ void init_rows_kernel(const float *__restrict__ F, int64_t n, int64_t r, int64_t ldf,
                                 const int32_t *__restrict__ rows, int k, float *__restrict__ C, Bat bt) {
    F += fblk(bt, blockIdx.y);
    rows += blockIdx.y * bt.rows;
    C += blockIdx.y * bt.c;
    const int64_t total = (int64_t)k * r;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(q / r);
        const int64_t col = q - (int64_t)c * r;
        int64_t i = rows[c];
        if (i < 0 || i >= n) i = 0;  // out-of-range rows read row 0 (validated on the host when possible)
        C[q] = F[i * ldf + col];
    }
}

// One wavefront per row, one lane per centroid: lane c accumulates
// sum_col (F_i,col - C_c,col)^2 in float64 over the columns in order (no
// fused multiply-add), then the wavefront takes the minimum with the lowest
// index on ties.  The row index is wave-uniform, so F_i,col is a scalar load.
// Centroids are staged transposed in LDS (Ct[col][c]) when they fit.
__device__ __forceinline__ void better(double &d, int &c, double d2, int c2) {
    if (d2 < d || (d2 == d && c2 < c)) {
        d = d2;
        c = c2;
    }
}

__global__ __launch_bounds__(NT) void assign_kernel(const float *__restrict__ F, int64_t n, int64_t r, int64_t ldf,
                                                    const float *__restrict__ Cg, int k, int use_lds,
                                                    int32_t *__restrict__ labels, float *__restrict__ dist2,
                                                    double *__restrict__ dist64, Bat bt) {
#pragma clang fp contract(off)
    if (idle(bt)) return;
    extern __shared__ float Ct[];
    F += fblk(bt, blockIdx.y);
    Cg += blockIdx.y * bt.c;
    labels += blockIdx.y * bt.l;
    if (dist2) dist2 += blockIdx.y * bt.l;
    if (dist64) dist64 += blockIdx.y * bt.l;
    const int kp = (k + 63) & ~63;
    if (use_lds) {
        for (int64_t q = threadIdx.x; q < (int64_t)kp * r; q += NT) {
            const int64_t col = q / kp;
            const int c = (int)(q - col * kp);
            Ct[q] = c < k ? Cg[(int64_t)c * r + col] : 0.0f;
        }
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = ((int64_t)blockIdx.x * NT + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * NT) >> 6;
    for (int64_t i = wave0; i < n; i += nwaves) {
        const int64_t iu = __builtin_amdgcn_readfirstlane((int)i);
        const float *f = F + iu * ldf;
        double best = 0.0;
        int bc = 0x7fffffff;
        for (int g = 0; g < kp; g += 64) {
            const int c = g + lane;
            double d = 0.0;
            if (use_lds) {
                for (int64_t col = 0; col < r; ++col) {
                    const double diff = (double)f[col] - (double)Ct[col * kp + c];
                    const double sq = diff * diff;
                    d = d + sq;
                }
            } else {
                const int cc = c < k ? c : k - 1;
                for (int64_t col = 0; col < r; ++col) {
                    const double diff = (double)f[col] - (double)Cg[(int64_t)cc * r + col];
                    const double sq = diff * diff;
                    d = d + sq;
                }
            }
            int ci = c;
            if (c >= k) {
                d = __builtin_huge_val();
                ci = 0x7fffffff;
            }
            for (int off = 1; off < 64; off <<= 1) {
                const double d2 = __shfl_xor(d, off, 64);
                const int c2 = __shfl_xor(ci, off, 64);
                better(d, ci, d2, c2);
            }
            if (g == 0) {
                best = d;
                bc = ci;
            } else {
                better(best, bc, d, ci);
            }
        }
        if (lane == 0) {
            if (bt.mark && labels[iu] != bc) bt.stamp[blockIdx.y] = bt.mark;
            labels[iu] = bc;
            if (dist2) dist2[iu] = (float)best;
            if (dist64) dist64[iu] = best;
        }
    }
}

// k > 32 with centroids that fit LDS as float64: one lane per centroid (64
// per group) and RB rows per wavefront pass, the centroids staged transposed
// as float64 (Cd[col][kp]), so one LDS read and no conversion serve RB rows.
// Per (row, centroid) the arithmetic and the lowest-index argmin are those of
// assign_kernel (identical labels).
template <int RB>
__global__ __launch_bounds__(NT) void assign_rows_kernel(const float *__restrict__ F, int64_t n, int64_t r,
                                                         int64_t ldf, const float *__restrict__ Cg, int k,
                                                         int32_t *__restrict__ labels, float *__restrict__ dist2,
                                                         double *__restrict__ dist64, Bat bt) {
#pragma clang fp contract(off)
    if (idle(bt)) return;
    extern __shared__ double Cd[];
    F += fblk(bt, blockIdx.y);
    Cg += blockIdx.y * bt.c;
    labels += blockIdx.y * bt.l;
    if (dist2) dist2 += blockIdx.y * bt.l;
    if (dist64) dist64 += blockIdx.y * bt.l;
    const int kp = (k + 63) & ~63;
    for (int64_t q = threadIdx.x; q < (int64_t)kp * r; q += NT) {
        const int64_t col = q / kp;
        const int c = (int)(q - col * kp);
        Cd[q] = c < k ? (double)Cg[(int64_t)c * r + col] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = ((int64_t)blockIdx.x * NT + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * NT) >> 6;
    for (int64_t i = wave0 * RB; i < n; i += nwaves * RB) {
        const int64_t i0 = __builtin_amdgcn_readfirstlane((int)i);
        const float *f[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) f[q] = F + (i0 + q < n ? i0 + q : n - 1) * ldf;
        double best[RB];
        int bc[RB];
        for (int g = 0; g < kp; g += 64) {
            const int c = g + lane;
            double d[RB];
#pragma unroll
            for (int q = 0; q < RB; ++q) d[q] = 0.0;
            int64_t col = 0;
            for (; col + 4 <= r; col += 4) {
                // four columns of every row loaded per pass, summed in column order
                float fv[RB][4];
#pragma unroll
                for (int q = 0; q < RB; ++q)
#pragma unroll
                    for (int u = 0; u < 4; ++u) fv[q][u] = f[q][col + u];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const double cv = Cd[(col + u) * kp + c];
#pragma unroll
                    for (int q = 0; q < RB; ++q) {
                        const double diff = (double)fv[q][u] - cv;
                        const double sq = diff * diff;
                        d[q] = d[q] + sq;
                    }
                }
            }
            for (; col < r; ++col) {
                const double cv = Cd[col * kp + c];
#pragma unroll
                for (int q = 0; q < RB; ++q) {
                    const double diff = (double)f[q][col] - cv;
                    const double sq = diff * diff;
                    d[q] = d[q] + sq;
                }
            }
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                double dq = d[q];
                int ci = c;
                if (c >= k) {
                    dq = __builtin_huge_val();
                    ci = 0x7fffffff;
                }
                for (int off = 1; off < 64; off <<= 1) {
                    const double d2 = __shfl_xor(dq, off, 64);
                    const int c2 = __shfl_xor(ci, off, 64);
                    better(dq, ci, d2, c2);
                }
                if (g == 0) {
                    best[q] = dq;
                    bc[q] = ci;
                } else {
                    better(best[q], bc[q], dq, ci);
                }
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                if (i0 + q < n) {
                    if (bt.mark && labels[i0 + q] != bc[q]) bt.stamp[blockIdx.y] = bt.mark;
                    labels[i0 + q] = bc[q];
                    if (dist2) dist2[i0 + q] = (float)best[q];
                    if (dist64) dist64[i0 + q] = best[q];
                }
            }
        }
    }
}

// k-means assignment on the matrix cores (2 <= k <= 16 NTILE; the centroids
// are staged in LDS, and up to 32 centroids the rows too).  A wavefront takes 16
// rows: v_mfma_f32_16x16x4f32 forms the dot products with the centroids as
// the A operand and the rows as the B operand, so lane l holds row l % 16 and
// centroids 16 T + 4 (l / 16) + v (v = 0..3) of tile T; the approximate
// distance is d~ = (|f|^2 + |c|^2) - 2 f.c with the norms in float64.  With
//   E = 3 (r + 2) 2^-24 |f| max|c| + 1e-12 (|f|^2 + max|c|^2)
// over the k centroids (1.5 times the standard bound 2 gamma_r |f| |c| on
// the float32 dot product's contribution, plus the float64 definition's own
// rounding), the exact distance of every centroid c lies in
// [d~(c) - E, d~(c) + E].  Let b be the float32 winner; every centroid whose
// interval reaches below d~(b) + E, d~(c) <= d~(b) + 2E (b itself, and any
// near tie), gets its float64 distance by the definition (squared
// differences summed column by column, no fused multiply-add) from the lane
// that holds it, and the least (distance, index) among them is the row's
// result: the others cannot be nearer.  Labels and distances therefore equal
// the definition's.  A row with non-finite values evaluates every centroid.
// One bound per row instead of one per centroid, and at most 72 registers
// (7 wavefronts per SIMD), took 2.4% off both stability sweeps.
template <int NTILE, bool STAGE>
__global__ __launch_bounds__(NT, 7) void assign_mfma_kernel(const float *__restrict__ F, int64_t n, int64_t r,
                                                         int64_t ldf, const float *__restrict__ Cg, int k,
                                                         int32_t *__restrict__ labels, float *__restrict__ dist2,
                                                         double *__restrict__ dist64, Bat bt) {
#pragma clang fp contract(off)
    if (idle(bt)) return;
    typedef float v4f __attribute__((ext_vector_type(4)));
    constexpr int KC = 16 * NTILE;
    extern __shared__ double lds_d[];
    // row stride RP = 2 (mod 4): the 32 lanes of a half-wavefront, (li, lk)
    // with li < 16 and lk < 2, read li * RP + lk + const, and 2 li (RP / 2)
    // takes every even bank once as li runs over 16 rows (RP / 2 odd), so the
    // matrix-core operand reads are free of bank conflicts (with an odd
    // stride, conflicts took 7-12% of the cycles, now 1.5-3%; the time is
    // the same, the kernel being bound by vector issue)
    const int RP = (int)((r + 3) & ~int64_t(3)) + 2;
    double *cn = lds_d;                                   // |c|^2, KC values
    double *cs = lds_d + KC;                              // |c|, KC values
    float *Cs = reinterpret_cast<float *>(lds_d + 2 * KC);  // [KC][RP], zero-padded
    constexpr bool kStageRows = STAGE;
    float *Fs = Cs + KC * RP + (threadIdx.x >> 6) * 16 * RP;  // this wavefront's rows (staged only)
    F += fblk(bt, blockIdx.y);
    Cg += blockIdx.y * bt.c;
    labels += blockIdx.y * bt.l;
    if (dist2) dist2 += blockIdx.y * bt.l;
    if (dist64) dist64 += blockIdx.y * bt.l;
    for (int q = threadIdx.x; q < KC * RP; q += NT) {
        const int c = q / RP, col = q - c * RP;
        Cs[q] = (c < k && col < r) ? Cg[(int64_t)c * r + col] : 0.0f;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < KC; c += NT) {
        double a = 0.0;
        for (int col = 0; col < r; ++col) {
            const double x = Cs[c * RP + col];
            a += x * x;
        }
        cn[c] = a;
        cs[c] = sqrt(a);
    }
    __syncthreads();
    // the largest |c| and |c|^2 of the k centroids: one error bound per row
    // that holds for every centroid
    double csmax = 0.0, cnmax = 0.0;
    for (int c = 0; c < k; ++c) {
        csmax = fmax(csmax, cs[c]);
        cnmax = fmax(cnmax, cn[c]);
    }
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int steps = (int)((r + 3) >> 2);
    const double ecoef = 3.0 * (double)(r + 2) * 0x1p-24;
    // staged rows, in 16-byte quads (rows of F 16-byte aligned when staged):
    // quad qd = rl * NQ + cq of the wavefront's 16 rows; lane qd0 + lane starts
    // at (qr0, qc0), and each further load is 64 quads on, (dq64, mq64) rows
    // and quads (no division per load)
    const int NQ = (int)((r + 3) >> 2);
    const int qr0 = lane / NQ, qc0 = lane - qr0 * NQ;
    const int dq64 = 64 / NQ, mq64 = 64 - dq64 * NQ;
    const int64_t wave0 = ((int64_t)blockIdx.x * NT + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * NT) >> 6;
    for (int64_t g = wave0; g * 16 < n; g += nwaves) {
        const int64_t row = g * 16 + li;
        const bool live = row < n;
        // the row's previous label, read early (clamped, always issued) when
        // a change is to be marked
        const int32_t prev = bt.mark ? labels[live ? row : 0] : 0;
        // up to 32 centroids the wavefront's 16 rows are staged in its own LDS
        // rows with coalesced loads (little matrix work per column step to
        // hide the loads behind); above, each lane reads its row from F
        const float *fr;
        if constexpr (kStageRows) {
            // four 16-byte loads in flight per lane, from clamped in-range
            // addresses and always issued, then their LDS stores; zero past r
            // and past n (the pad columns RP - 2 and RP - 1 are never read)
            const int64_t left = n - g * 16;  // rows of this group that exist (>= 1)
            const v4f *fg = reinterpret_cast<const v4f *>(F + g * 16 * ldf);
            const int64_t ldq = ldf >> 2;
            int rl = qr0, cq = qc0;
            for (int q0 = 0; q0 < 16 * NQ; q0 += 4 * 64) {
                v4f v[4];
                int row[4], c4[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool in = rl < 16 && rl < left;
                    const v4f x = fg[in ? (int64_t)rl * ldq + cq : 0];
                    v[u] = in ? x : v4f{0.0f, 0.0f, 0.0f, 0.0f};
                    row[u] = rl;
                    c4[u] = 4 * cq;
                    rl += dq64;
                    cq += mq64;
                    if (cq >= NQ) {
                        cq -= NQ;
                        ++rl;
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (row[u] < 16) {
                        float *d = Fs + row[u] * RP + c4[u];
#pragma unroll
                        for (int e = 0; e < 4; ++e) d[e] = c4[u] + e < r ? v[u][e] : 0.0f;
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
            fr = Fs + li * RP;
        } else {
            fr = F + (live ? row : 0) * ldf;
        }
        v4f acc[NTILE];
#pragma unroll
        for (int t = 0; t < NTILE; ++t) acc[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        double nf = 0.0;
        if constexpr (kStageRows) {
            // rows in LDS (zero past r and past n): the LDS reads of four column
            // steps issued together, then their products in column order
            int st = 0;
            for (; st + 4 <= steps; st += 4) {
                float bq[4], aq[NTILE][4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int col = 4 * (st + u) + lk;
                    bq[u] = fr[col];
#pragma unroll
                    for (int t = 0; t < NTILE; ++t) aq[t][u] = Cs[(16 * t + li) * RP + col];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    nf += (double)bq[u] * (double)bq[u];
#pragma unroll
                    for (int t = 0; t < NTILE; ++t)
                        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[t][u], bq[u], acc[t], 0, 0, 0);
                }
            }
            for (; st < steps; ++st) {
                const int col = 4 * st + lk;
                const float b = fr[col];
                nf += (double)b * (double)b;
#pragma unroll
                for (int t = 0; t < NTILE; ++t) {
                    const float a = Cs[(16 * t + li) * RP + col];
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
                }
            }
        } else {
            // rows read from global memory: four column steps per pass, the
            // row values of the next pass loaded while this pass's products
            // run (products and sums still step by step, in column order;
            // clamped in-range addresses, always issued)
            float bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int col = 4 * u + lk;
                const bool in = live && col < r;
                const float x = fr[in ? col : 0];
                bv[u] = in ? x : 0.0f;
            }
            for (int st0 = 0; st0 < steps; st0 += 4) {
                float bn[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int col = 4 * (st0 + 4 + u) + lk;
                    const bool in = live && col < r;
                    const float x = fr[in ? col : 0];
                    bn[u] = in ? x : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (st0 + u >= steps) break;
                    const int col = 4 * (st0 + u) + lk;
                    const float b = bv[u];
                    nf += (double)b * (double)b;
#pragma unroll
                    for (int t = 0; t < NTILE; ++t) {
                        const float a = Cs[(16 * t + li) * RP + col];
                        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) bv[u] = bn[u];
            }
        }
        // |f|^2 of row li: the four lanes li, li+16, li+32, li+48 hold its columns
        nf += __shfl_xor(nf, 16, 64);
        nf += __shfl_xor(nf, 32, 64);
        const double sf = sqrt(nf);
        // |d~ - d| <= E for every centroid of the row
        const double E = ecoef * sf * csmax + 1e-12 * (nf + cnmax);
        // the float32 winner of the row
        double bd = __builtin_huge_val();
        int bc = 0x7fffffff;
#pragma unroll
        for (int t = 0; t < NTILE; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = 16 * t + 4 * lk + v;
                if (c < k) {
                    const double dd = (cn[c] + nf) - 2.0 * (double)acc[t][v];
                    if (dd < bd || (dd == bd && c < bc)) {
                        bd = dd;
                        bc = c;
                    }
                }
            }
#pragma unroll
        for (int off = 16; off <= 32; off <<= 1) {
            const double obd = __shfl_xor(bd, off, 64);
            const int obc = __shfl_xor(bc, off, 64);
            if (obd < bd || (obd == bd && obc < bc)) {
                bd = obd;
                bc = obc;
            }
        }
        // every centroid that could be nearest, by the float64 definition: its
        // lower bound d~ - E at most the winner's upper bound d~ + E
        const double thr = (bd + E) + E;
        const bool all = !(thr < __builtin_huge_val());  // non-finite row: every centroid
        uint32_t need = 0;  // bit 4 t + v: centroid 16 t + 4 lk + v needs its float64 distance
#pragma unroll
        for (int t = 0; t < NTILE; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = 16 * t + 4 * lk + v;
                if (c >= k) continue;
                const double dd = (cn[c] + nf) - 2.0 * (double)acc[t][v];
                if (all || dd <= thr) need |= 1u << (4 * t + v);
            }
        if (!live) need = 0;
        // A lone candidate is the float32 winner, and the float64 winner for
        // certain: every other centroid lies beyond the winner's upper bound.
        // Its float64 distance is then only needed as an output.
        bool sure = false;
        if (!dist2 && !dist64) {
            int cnt = __popc(need);
            cnt += __shfl_xor(cnt, 16, 64);
            cnt += __shfl_xor(cnt, 32, 64);
            sure = cnt == 1;
            if (sure) need = 0;
        }
        // one pass of the column loop per needed centroid of the busiest lane
        // (usually one: the winner's own lane)
        double ed = __builtin_huge_val();
        int ec = 0x7fffffff;
        while (__ballot(need != 0)) {
            const int slot = need ? __builtin_ctz(need) : -1;
            need &= need - 1;
            if (slot >= 0) {
                const int c = 16 * (slot >> 2) + 4 * lk + (slot & 3);
                const float *cr = Cs + c * RP;
                double d = 0.0;
                // rows in global memory: eight row values loaded per pass, then
                // summed in column order
                int64_t col = 0;
                if constexpr (!kStageRows) {
                    for (; col + 8 <= r; col += 8) {
                        float fv[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) fv[q] = fr[col + q];
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const double diff = (double)fv[q] - (double)cr[col + q];
                            const double sq = diff * diff;
                            d = d + sq;
                        }
                    }
                }
                for (; col < r; ++col) {
                    const double diff = (double)fr[col] - (double)cr[col];
                    const double sq = diff * diff;
                    d = d + sq;
                }
                if (ec == 0x7fffffff) {  // the first is taken as is (also when d is NaN)
                    ed = d;
                    ec = c;
                } else {
                    better(ed, ec, d, c);
                }
            }
        }
#pragma unroll
        for (int off = 16; off <= 32; off <<= 1) {
            const double od = __shfl_xor(ed, off, 64);
            const int oc = __shfl_xor(ec, off, 64);
            if (oc != 0x7fffffff && (ec == 0x7fffffff || od < ed || (od == ed && oc < ec))) {
                ed = od;
                ec = oc;
            }
        }
        if (sure) ec = bc;
        if (live && lk == 0) {
            if (bt.mark && prev != ec) bt.stamp[blockIdx.y] = bt.mark;
            labels[row] = ec;
            if (dist2) dist2[row] = (float)ed;
            if (dist64) dist64[row] = ed;
        }
        if constexpr (kStageRows) __builtin_amdgcn_wave_barrier();  // Fs is free for the next rows
    }
}

// k <= 32: 64/KP rows per wavefront and KP lanes (one per centroid) per row,
// so small k keeps the lanes busy; the centroids are staged transposed in LDS
// as float64 (Cd[col][KP]).  The arithmetic per (row, centroid) and the
// lowest-index argmin are those of assign_kernel (identical labels).
template <int KP>
__global__ __launch_bounds__(NT) void assign_grouped_kernel(const float *__restrict__ F, int64_t n, int64_t r,
                                                            int64_t ldf, const float *__restrict__ Cg, int k,
                                                            int32_t *__restrict__ labels, float *__restrict__ dist2,
                                                            double *__restrict__ dist64, Bat bt) {
#pragma clang fp contract(off)
    if (idle(bt)) return;
    extern __shared__ double Cd[];
    constexpr int RPW = 64 / KP;
    F += fblk(bt, blockIdx.y);
    Cg += blockIdx.y * bt.c;
    labels += blockIdx.y * bt.l;
    if (dist2) dist2 += blockIdx.y * bt.l;
    if (dist64) dist64 += blockIdx.y * bt.l;
    for (int64_t q = threadIdx.x; q < (int64_t)KP * r; q += NT) {
        const int64_t col = q / KP;
        const int c = (int)(q - col * KP);
        Cd[q] = c < k ? (double)Cg[(int64_t)c * r + col] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int c = lane % KP;
    const int sub = lane / KP;
    const int64_t wave0 = ((int64_t)blockIdx.x * NT + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * NT) >> 6;
    for (int64_t base = wave0 * RPW; base < n; base += nwaves * RPW) {
        const int64_t i = base + sub;
        const bool valid = i < n;
        const float *f = F + (valid ? i : 0) * ldf;
        double d = 0.0;
        // eight row values loaded per pass, then summed in column order
        int64_t col = 0;
        for (; col + 8 <= r; col += 8) {
            float fv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) fv[q] = f[col + q];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double diff = (double)fv[q] - Cd[(col + q) * KP + c];
                const double sq = diff * diff;
                d = d + sq;
            }
        }
        for (; col < r; ++col) {
            const double diff = (double)f[col] - Cd[col * KP + c];
            const double sq = diff * diff;
            d = d + sq;
        }
        int ci = c;
        if (c >= k) {
            d = __builtin_huge_val();
            ci = 0x7fffffff;
        }
        for (int off = 1; off < KP; off <<= 1) {
            const double d2 = __shfl_xor(d, off, 64);
            const int c2 = __shfl_xor(ci, off, 64);
            better(d, ci, d2, c2);
        }
        if (c == 0 && valid) {
            if (bt.mark && labels[i] != ci) bt.stamp[blockIdx.y] = bt.mark;
            labels[i] = ci;
            if (dist2) dist2[i] = (float)d;
            if (dist64) dist64[i] = d;
        }
    }
}

// per-block float64 sums of member rows, one thread per column, rows in
// order (deterministic), partial [block][k][r] and counts [block][k]
__global__ void update_partial_kernel(const float *__restrict__ F, int64_t n, int64_t r, int64_t ldf,
                                      const int32_t *__restrict__ labels, int k, int64_t rows_per_block,
                                      double *__restrict__ part, int64_t *__restrict__ pcount, Bat bt) {
    if (idle(bt)) return;
    extern __shared__ double S[];  // k*r sums then k counts (as double)
    const int64_t kr = (int64_t)k * r;
    F += fblk(bt, blockIdx.y);
    labels += blockIdx.y * bt.l;
    part += (int64_t)blockIdx.y * gridDim.x * kr;
    pcount += (int64_t)blockIdx.y * gridDim.x * k;
    for (int64_t q = threadIdx.x; q < kr + k; q += blockDim.x) S[q] = 0.0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t i1 = min(n, i0 + rows_per_block);
    // 16 rows' labels and values loaded before they are added (clamped
    // in-range addresses, always issued: no load waits behind a branch)
    constexpr int U = 16;
    if (r <= (int64_t)blockDim.x) {
        // one column per thread: the next 16 rows' loads are issued before this
        // group's additions, so they overlap (rows still added in order)
        const int64_t col = threadIdx.x;
        const bool colin = col < r;
        const int64_t colc = colin ? col : 0;
        int lab[U], labn[U];
        float v[U], vn[U];
        auto load = [&](int64_t ib, int *L, float *V) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool in = ib + u < i1;
                const int64_t i = in ? ib + u : i1 - 1;
                const int l = labels[i];
                const float x = F[i * ldf + colc];
                L[u] = in ? l : -1;
                V[u] = (in && colin) ? x : 0.0f;
            }
        };
        if (i0 < i1) load(i0, labn, vn);
        for (int64_t ib = i0; ib < i1; ib += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                lab[u] = labn[u];
                v[u] = vn[u];
            }
            if (ib + U < i1) load(ib + U, labn, vn);
            if (colin) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int c = lab[u];
                    if (c >= 0 && c < k) S[(int64_t)c * r + col] += (double)v[u];
                }
            }
            if (threadIdx.x == 0) {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (lab[u] >= 0 && lab[u] < k) S[kr + lab[u]] += 1.0;
            }
        }
        __syncthreads();
        double *out = part + (int64_t)blockIdx.x * kr;
        for (int64_t q = threadIdx.x; q < kr; q += blockDim.x) out[q] = S[q];
        for (int q = threadIdx.x; q < k; q += blockDim.x) pcount[(int64_t)blockIdx.x * k + q] = (int64_t)S[kr + q];
        return;
    }
    for (int64_t ib = i0; ib < i1; ib += U) {
        int lab[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool in = ib + u < i1;
            const int l = labels[in ? ib + u : i1 - 1];
            lab[u] = in ? l : -1;
        }
        for (int64_t col = threadIdx.x; col < r; col += blockDim.x) {
            float v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool in = ib + u < i1;
                const float x = F[(in ? ib + u : i1 - 1) * ldf + col];
                v[u] = in ? x : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = lab[u];
                if (c >= 0 && c < k) S[(int64_t)c * r + col] += (double)v[u];
            }
        }
        if (threadIdx.x == 0) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (lab[u] >= 0 && lab[u] < k) S[kr + lab[u]] += 1.0;
        }
    }
    __syncthreads();
    double *out = part + (int64_t)blockIdx.x * kr;
    for (int64_t q = threadIdx.x; q < kr; q += blockDim.x) out[q] = S[q];
    for (int q = threadIdx.x; q < k; q += blockDim.x) pcount[(int64_t)blockIdx.x * k + q] = (int64_t)S[kr + q];
}

// same with 4 wavefronts per block, each summing its own quarter of the
// block's rows into its own LDS copy (rows in order, one lane per column);
// the copies are then added in wavefront order (deterministic)
__global__ __launch_bounds__(256) void update_partial4_kernel(const float *__restrict__ F, int64_t n, int64_t r,
                                                              int64_t ldf, const int32_t *__restrict__ labels, int k,
                                                              int64_t rows_per_block, double *__restrict__ part,
                                                              int64_t *__restrict__ pcount, Bat bt) {
    if (idle(bt)) return;
    extern __shared__ double S4[];  // 4 x (k*r sums, k counts)
    const int64_t kr = (int64_t)k * r;
    const int64_t stride = kr + k;
    F += fblk(bt, blockIdx.y);
    labels += blockIdx.y * bt.l;
    part += (int64_t)blockIdx.y * gridDim.x * kr;
    pcount += (int64_t)blockIdx.y * gridDim.x * k;
    for (int64_t q = threadIdx.x; q < 4 * stride; q += blockDim.x) S4[q] = 0.0;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double *S = S4 + wave * stride;
    const int64_t b0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t b1 = min(n, b0 + rows_per_block);
    const int64_t len = b1 > b0 ? b1 - b0 : 0;
    const int64_t q4 = (len + 3) / 4;
    const int64_t i0 = min(b1, b0 + wave * q4);
    const int64_t i1 = min(b1, i0 + q4);
    // 8 rows' labels and values loaded before they are added (clamped
    // in-range addresses, always issued: no load waits behind a branch)
    constexpr int U = 8;
    for (int64_t ib = i0; ib < i1; ib += U) {
        int lab[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool in = ib + u < i1;
            const int l = labels[in ? ib + u : i1 - 1];
            lab[u] = in ? l : -1;
        }
        for (int64_t col = lane; col < r; col += 64) {
            float v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool in = ib + u < i1;
                const float x = F[(in ? ib + u : i1 - 1) * ldf + col];
                v[u] = in ? x : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = lab[u];
                if (c >= 0 && c < k) S[(int64_t)c * r + col] += (double)v[u];
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (lab[u] >= 0 && lab[u] < k) S[kr + lab[u]] += 1.0;
        }
    }
    __syncthreads();
    double *out = part + (int64_t)blockIdx.x * kr;
    for (int64_t q = threadIdx.x; q < kr; q += blockDim.x)
        out[q] = ((S4[q] + S4[stride + q]) + S4[2 * stride + q]) + S4[3 * stride + q];
    for (int q = threadIdx.x; q < k; q += blockDim.x)
        pcount[(int64_t)blockIdx.x * k + q] =
            (int64_t)S4[kr + q] + (int64_t)S4[stride + kr + q] + (int64_t)S4[2 * stride + kr + q] +
            (int64_t)S4[3 * stride + kr + q];
}

// r <= 32: the 64 lanes of a wavefront form 64 / rs slots of rs lanes (rs the
// power of two >= r, one lane per column); each of the block's 4 (64 / rs)
// slots sums its own contiguous share of the block's rows, in order, into
// its own LDS copy, and the copies are added in slot order (deterministic)
__global__ __launch_bounds__(256) void update_slots_kernel(const float *__restrict__ F, int64_t n, int64_t r,
                                                           int64_t ldf, const int32_t *__restrict__ labels, int k,
                                                           int64_t rows_per_block, double *__restrict__ part,
                                                           int64_t *__restrict__ pcount, Bat bt, int rs) {
    if (idle(bt)) return;
    extern __shared__ double SS[];  // (4 * 64 / rs) x (k*r sums, k counts)
    const int SL = 64 / rs;
    const int ncopy = 4 * SL;
    const int64_t kr = (int64_t)k * r;
    const int64_t stride = kr + k;
    F += fblk(bt, blockIdx.y);
    labels += blockIdx.y * bt.l;
    part += (int64_t)blockIdx.y * gridDim.x * kr;
    pcount += (int64_t)blockIdx.y * gridDim.x * k;
    for (int64_t q = threadIdx.x; q < ncopy * stride; q += blockDim.x) SS[q] = 0.0;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int slot = lane / rs, col = lane & (rs - 1);
    const int id = wave * SL + slot;
    double *S = SS + (int64_t)id * stride;
    const int64_t b0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t b1 = min(n, b0 + rows_per_block);
    const int64_t len = b1 > b0 ? b1 - b0 : 0;
    const int64_t q = (len + ncopy - 1) / ncopy;
    const int64_t i0 = min(b1, b0 + id * q);
    const int64_t i1 = min(b1, i0 + q);
    // 8 rows' labels and values are loaded before they are added (rows still
    // added one by one, in order).  The loads use clamped in-range addresses
    // and are always issued, so none of them waits behind a branch.
    constexpr int U = 8;
    const int colc = col < r ? col : (int)r - 1;
    for (int64_t ib = i0; ib < i1; ib += U) {
        int lab[U];
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool in = ib + u < i1;
            const int64_t i = in ? ib + u : i1 - 1;
            const int l = labels[i];
            const float x = F[i * ldf + colc];
            lab[u] = in ? l : -1;
            v[u] = (in && col < r) ? x : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = lab[u];
            if (c >= 0 && c < k) {
                if (col < r) S[(int64_t)c * r + col] += (double)v[u];
                if (col == 0) S[kr + c] += 1.0;
            }
        }
    }
    __syncthreads();
    double *out = part + (int64_t)blockIdx.x * kr;
    for (int64_t e = threadIdx.x; e < kr; e += blockDim.x) {
        double a = SS[e];
        for (int c = 1; c < ncopy; ++c) a += SS[(int64_t)c * stride + e];
        out[e] = a;
    }
    for (int e = threadIdx.x; e < k; e += blockDim.x) {
        int64_t a = 0;
        for (int c = 0; c < ncopy; ++c) a += (int64_t)SS[(int64_t)c * stride + kr + e];
        pcount[(int64_t)blockIdx.x * k + e] = a;
    }
}

// same, for k*r too large for LDS: sums kept in the partial array itself
__global__ void update_partial_global_kernel(const float *__restrict__ F, int64_t n, int64_t r, int64_t ldf,
                                             const int32_t *__restrict__ labels, int k, int64_t rows_per_block,
                                             double *__restrict__ part, int64_t *__restrict__ pcount, Bat bt) {
    if (idle(bt)) return;
    const int64_t kr = (int64_t)k * r;
    F += fblk(bt, blockIdx.y);
    labels += blockIdx.y * bt.l;
    part += (int64_t)blockIdx.y * gridDim.x * kr;
    pcount += (int64_t)blockIdx.y * gridDim.x * k;
    double *S = part + (int64_t)blockIdx.x * kr;
    for (int64_t q = threadIdx.x; q < kr; q += blockDim.x) S[q] = 0.0;
    int64_t *cnt = pcount + (int64_t)blockIdx.x * k;
    for (int q = threadIdx.x; q < k; q += blockDim.x) cnt[q] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t i1 = min(n, i0 + rows_per_block);
    for (int64_t i = i0; i < i1; ++i) {
        const int c = labels[i];
        if (c < 0 || c >= k) continue;
        for (int64_t col = threadIdx.x; col < r; col += blockDim.x) S[(int64_t)c * r + col] += (double)F[i * ldf + col];
        if (threadIdx.x == 0) cnt[c] += 1;
    }
}

// C[c][col] = (sum over blocks of the partial sums) / count; one wavefront
// per (c, col): lanes take blocks b = lane, lane+64, ... in order, then the
// fixed butterfly adds the 64 lane sums (deterministic).
__global__ void update_final_kernel(int nblocks, int64_t r, int k, const double *__restrict__ part,
                                    const int64_t *__restrict__ pcount, float *__restrict__ C,
                                    int64_t *__restrict__ counts, Bat bt) {
    if (idle(bt)) return;
    const int lane = threadIdx.x & 63;
    const int64_t kr = (int64_t)k * r;
    part += (int64_t)blockIdx.y * nblocks * kr;
    pcount += (int64_t)blockIdx.y * nblocks * k;
    C += blockIdx.y * bt.c;
    if (counts) counts += (int64_t)blockIdx.y * k;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t q = w0; q < kr; q += nw) {
        const int c = (int)(q / r);
        double s = 0.0;
        int64_t cnt = 0;
        for (int b = lane; b < nblocks; b += 64) {
            s += part[(int64_t)b * kr + q];
            cnt += pcount[(int64_t)b * k + c];
        }
        s = wave_sum(s);
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
        if (lane == 0) {
            if (cnt > 0) C[q] = (float)(s / (double)cnt);
            if (counts && q - (int64_t)c * r == 0) counts[c] = cnt;
        }
    }
}

// Up to W <= 32 partial blocks: one lane per (c, col) instead of one
// wavefront.  The lane holds the W partial sums (zero past nblocks) and adds
// them in registers by the pairing of the butterfly above: lane l of the
// wavefront adds lane l + off for off = 32, 16, ..., 1, and the levels with
// off >= W only add zeros to the canonical 0.0 + p of each lane, so the
// result is the butterfly's, bit for bit.
template <int W>
__global__ __launch_bounds__(256) void update_final_lanes_kernel(int nblocks, int64_t r, int k,
                                                                 const double *__restrict__ part,
                                                                 const int64_t *__restrict__ pcount,
                                                                 float *__restrict__ C, int64_t *__restrict__ counts,
                                                                 Bat bt) {
    if (idle(bt)) return;
    const int64_t kr = (int64_t)k * r;
    part += (int64_t)blockIdx.y * nblocks * kr;
    pcount += (int64_t)blockIdx.y * nblocks * k;
    C += blockIdx.y * bt.c;
    if (counts) counts += (int64_t)blockIdx.y * k;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < kr; q += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(q / r);
        double v[W];
        int64_t cnt = 0;
#pragma unroll
        for (int b = 0; b < W; ++b) {
            const bool in = b < nblocks;
            const double x = part[(int64_t)(in ? b : 0) * kr + q];
            const int64_t m = pcount[(int64_t)(in ? b : 0) * k + c];
            v[b] = in ? 0.0 + x : 0.0;
            cnt += in ? m : 0;
        }
#pragma unroll
        for (int off = W / 2; off >= 1; off >>= 1)
#pragma unroll
            for (int l = 0; l < off; ++l) v[l] = v[l] + v[l + off];
        if (cnt > 0) C[q] = (float)(v[0] / (double)cnt);
        if (counts && q - (int64_t)c * r == 0) counts[c] = cnt;
    }
}

// one block per problem: its inertia, the float64 sum of the rows' least
// distances (each thread's rows in order, then the fixed block sum)
__global__ __launch_bounds__(NT) void inertia_kernel(const double *__restrict__ dist64, int64_t n,
                                                     double *__restrict__ inert) {
    __shared__ double lds[NT / 64];
    const int64_t q = blockIdx.x;
    const double *d = dist64 + q * n;
    double v[1] = {0.0};
    for (int64_t i = threadIdx.x; i < n; i += NT) v[0] += d[i];
    block_sum<1, NT>(v, lds);
    if (threadIdx.x == 0) inert[q] = v[0];
}

// per group of reps problems (blockIdx.y): the problem of least inertia, the
// lowest one on ties, gives the labels (and centroids, when asked); blocks
// along x share the copy
__global__ __launch_bounds__(NT) void select_kernel(const double *__restrict__ inert,
                                                    const int32_t *__restrict__ lab_all, int64_t n, int reps,
                                                    int32_t *__restrict__ lab_out, double *__restrict__ inertia,
                                                    const float *__restrict__ C_all, int64_t ckr,
                                                    float *__restrict__ C_out) {
    __shared__ int best;
    const int j = blockIdx.y;
    const double *v = inert + (int64_t)j * reps;
    if (threadIdx.x == 0) {
        double best_v = v[0];
        int best_r = 0;
        for (int rep = 1; rep < reps; ++rep)
            if (v[rep] < best_v) {
                best_v = v[rep];
                best_r = rep;
            }
        best = best_r;
    }
    if (inertia && blockIdx.x == 0)
        for (int rep = threadIdx.x; rep < reps; rep += NT) inertia[(int64_t)j * reps + rep] = v[rep];
    __syncthreads();
    const int32_t *src = lab_all + ((int64_t)j * reps + best) * n;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        lab_out[(int64_t)j * n + i] = src[i];
    if (C_out && blockIdx.x == 0) {
        const float *cs = C_all + ((int64_t)j * reps + best) * ckr;
        for (int64_t q = threadIdx.x; q < ckr; q += NT) C_out[(int64_t)j * ckr + q] = cs[q];
    }
}

__global__ void zero_u32_kernel(uint32_t *v, int64_t m) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < m; q += (int64_t)gridDim.x * blockDim.x)
        v[q] = 0u;
}

int update_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 255) / 256)); }

asc_status check_feat(const float *F, int64_t n, int64_t r, int64_t ldf, const char *who) {
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(ASC_ERR_INVALID, "%s: n=%lld", who, (long long)n);
    if (!F) return fail(ASC_ERR_INVALID, "%s: F is NULL", who);
    if (r < 1 || r > 4096 || ldf < r) return fail(ASC_ERR_INVALID, "%s: r=%lld ldf=%lld", who, (long long)r, (long long)ldf);
    if (!aligned(F, 4)) return fail(ASC_ERR_INVALID, "%s: F misaligned", who);
    return ASC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers shared by the public entry points and the batched callers
// ---------------------------------------------------------------------------
static Bat to_bat(const KmBatch &b) {
    return Bat{b.fstride, b.fdiv, b.cstride, b.lstride, b.rows_stride, b.stamp, b.want, b.mark};
}

int km_update_blocks(int64_t n, int count) {
    const int nb = count <= 1 ? update_blocks(n)
                              : (int)std::max<int64_t>(1, std::min<int64_t>(update_blocks(n), 16384 / count));
    // 17 to 32 partial blocks become 16: the final sum then holds 16 partials
    // per lane instead of 32 (the 32-partial form spills scalar registers),
    // 55.4 -> 53.5 ms on the 5000-point stability sweep (20 blocks per problem)
    return nb > 16 && nb <= 32 ? 16 : nb;
}

void km_normalize(float *Y, int64_t n, int64_t r, int64_t ldy, float *norms, hipStream_t s) {
    const int grid = (int)std::min<int64_t>((n * 64 + NT - 1) / NT, 16384);
    normalize_kernel<<<grid, NT, 0, s>>>(Y, n, r, ldy, norms);
}

void km_init_rows(const float *F, int64_t n, int64_t r, int64_t ldf, const int32_t *rows, int k, float *C,
                  const KmBatch &b, hipStream_t s) {
    const int64_t total = (int64_t)k * r;
    const dim3 grid((unsigned)std::min<int64_t>((total + 255) / 256, 1024), (unsigned)b.count);
    init_rows_kernel<<<grid, 256, 0, s>>>(F, n, r, ldf, rows, k, C, to_bat(b));
}

template <int KP>
void assign_grouped(const float *F, int64_t n, int64_t r, int64_t ldf, const float *C, int k, int32_t *labels,
                    float *dist2, double *dist64, const KmBatch &b, hipStream_t s) {
    const int64_t rows_per_block = (NT / 64) * (64 / KP);
    const int64_t want = (n + rows_per_block - 1) / rows_per_block;
    const int64_t cap = b.count <= 1 ? 8192 : std::max<int64_t>(1, 65536 / b.count);
    const dim3 grid((unsigned)std::max<int64_t>(1, std::min(want, cap)), (unsigned)b.count);
    assign_grouped_kernel<KP><<<grid, NT, (size_t)KP * r * sizeof(double), s>>>(F, n, r, ldf, C, k, labels, dist2,
                                                                               dist64, to_bat(b));
}

// rows are staged with 16-byte loads: every problem's feature rows 16-byte aligned
static bool stage_ok(const float *F, int64_t ldf, const KmBatch &b) {
    return aligned(F, 16) && ldf % 4 == 0 && b.fstride % 4 == 0;
}

template <int NTILE>
void assign_mfma(const float *F, int64_t n, int64_t r, int64_t ldf, const float *C, int k, int32_t *labels,
                 float *dist2, double *dist64, const KmBatch &b, hipStream_t s) {
    constexpr int KC = 16 * NTILE;
    const int64_t rp = ((r + 3) & ~int64_t(3)) + 2;
    // rows staged in LDS (16-byte loads) up to 32 centroids, measured faster
    // there (1e6 x 96, k = 20: 0.24 -> 0.20 ms); with more centroids each lane
    // reads its row from F, with the loads of the next column steps in flight
    // (staging is 4% slower at k = 50, where the LDS of the staged rows costs
    // resident blocks)
    const size_t lds_staged = (size_t)2 * KC * sizeof(double) + (size_t)(KC + (NT / 64) * 16) * rp * sizeof(float);
    const bool stage = NTILE <= 2 && stage_ok(F, ldf, b) && lds_staged <= 64 * 1024;
    const size_t lds = stage ? lds_staged : (size_t)2 * KC * sizeof(double) + (size_t)KC * rp * sizeof(float);
    // many small problems: about 8 row groups per wavefront, so the centroid
    // staging of a block is spread over more rows; 4 when that still keeps
    // the launch within 8192 blocks: fewer rows per block shorten the
    // launches in which only a few problems still move (5000 rows x 400
    // problems: sweep 59.2 -> 56.7 ms; 1e5 rows x 80 problems keeps 8)
    int groups = b.count > 1 ? 8 : 1;
    if (b.count > 1 && (int64_t)b.count * ((n + (NT / 64) * 16 * 4 - 1) / ((NT / 64) * 16 * 4)) <= 8192) groups = 4;
    const int64_t rows_per_block = (NT / 64) * 16 * groups;
    const int64_t want = (n + rows_per_block - 1) / rows_per_block;
    const int64_t cap = b.count <= 1 ? 8192 : std::max<int64_t>(1, 65536 / b.count);
    const dim3 grid((unsigned)std::max<int64_t>(1, std::min(want, cap)), (unsigned)b.count);
    if constexpr (NTILE <= 2) {
        if (stage) {
            assign_mfma_kernel<NTILE, true><<<grid, NT, lds, s>>>(F, n, r, ldf, C, k, labels, dist2, dist64, to_bat(b));
            return;
        }
    }
    assign_mfma_kernel<NTILE, false><<<grid, NT, lds, s>>>(F, n, r, ldf, C, k, labels, dist2, dist64, to_bat(b));
}

void km_assign(const float *F, int64_t n, int64_t r, int64_t ldf, const float *C, int k, int32_t *labels,
               float *dist2, double *dist64, const KmBatch &b, hipStream_t s) {
    // matrix cores while the centroids fit 64 KB of LDS (the rows are staged
    // as well when they fit beside them)
    const int64_t rpad = ((r + 3) & ~int64_t(3)) + 2;
    const int kc = ((k + 15) / 16) * 16;
    if (k >= 2 && k <= 64 && (size_t)kc * 16 + (size_t)kc * rpad * 4 <= 64 * 1024) {
        switch ((k + 15) / 16) {
            case 1: assign_mfma<1>(F, n, r, ldf, C, k, labels, dist2, dist64, b, s); return;
            case 2: assign_mfma<2>(F, n, r, ldf, C, k, labels, dist2, dist64, b, s); return;
            case 3: assign_mfma<3>(F, n, r, ldf, C, k, labels, dist2, dist64, b, s); return;
            default: assign_mfma<4>(F, n, r, ldf, C, k, labels, dist2, dist64, b, s); return;
        }
    }
    int kp2 = 2;
    while (kp2 < k) kp2 *= 2;
    if (kp2 <= 32 && (size_t)kp2 * r * sizeof(double) <= 64 * 1024) {
        switch (kp2) {
            case 2: assign_grouped<2>(F, n, r, ldf, C, k, labels, dist2, dist64, b, s); return;
            case 4: assign_grouped<4>(F, n, r, ldf, C, k, labels, dist2, dist64, b, s); return;
            case 8: assign_grouped<8>(F, n, r, ldf, C, k, labels, dist2, dist64, b, s); return;
            case 16: assign_grouped<16>(F, n, r, ldf, C, k, labels, dist2, dist64, b, s); return;
            default: assign_grouped<32>(F, n, r, ldf, C, k, labels, dist2, dist64, b, s); return;
        }
    }
    const int64_t cap0 = b.count <= 1 ? 8192 : std::max<int64_t>(1, 65536 / b.count);
    const size_t dbytes = (size_t)((k + 63) & ~63) * r * sizeof(double);
    if (dbytes <= 64 * 1024) {
        constexpr int RB = 4;
        const int64_t want = (n + (NT / 64) * RB - 1) / ((NT / 64) * RB);
        const dim3 grid((unsigned)std::max<int64_t>(1, std::min(want, cap0)), (unsigned)b.count);
        assign_rows_kernel<RB><<<grid, NT, dbytes, s>>>(F, n, r, ldf, C, k, labels, dist2, dist64, to_bat(b));
        return;
    }
    const size_t cbytes = (size_t)((k + 63) & ~63) * r * sizeof(float);
    const int use_lds = cbytes <= 64 * 1024;
    const int64_t want = (n * 64 + NT - 1) / NT;
    const int64_t cap = b.count <= 1 ? 8192 : std::max<int64_t>(1, 65536 / b.count);
    const dim3 grid((unsigned)std::max<int64_t>(1, std::min(want, cap)), (unsigned)b.count);
    assign_kernel<<<grid, NT, use_lds ? cbytes : 0, s>>>(F, n, r, ldf, C, k, use_lds, labels, dist2, dist64,
                                                         to_bat(b));
}

size_t km_update_ws(int64_t n, int64_t r, int k, int count) {
    Arena a(nullptr);
    const int nb = km_update_blocks(n, count);
    a.take<double>((size_t)count * nb * k * r);
    a.take<int64_t>((size_t)count * nb * k);
    return a.size();
}

void km_update(const float *F, int64_t n, int64_t r, int64_t ldf, const int32_t *labels, int k, float *C,
               int64_t *counts, void *ws, const KmBatch &b, hipStream_t s) {
    Arena a(ws);
    const int nb = km_update_blocks(n, b.count);
    double *part = a.take<double>((size_t)b.count * nb * k * r);
    int64_t *pcount = a.take<int64_t>((size_t)b.count * nb * k);
    const int64_t rpb = (n + nb - 1) / nb;
    const size_t lds = ((size_t)k * r + k) * sizeof(double);
    const int threads = (int)std::min<int64_t>(256, ((r + 63) / 64) * 64);
    const dim3 g1((unsigned)nb, (unsigned)b.count);
    int rs = 1;
    while (rs < r) rs *= 2;
    if (b.count > 1 && rs <= 32 && (size_t)4 * (64 / rs) * lds <= 64 * 1024)
        update_slots_kernel<<<g1, 256, (size_t)4 * (64 / rs) * lds, s>>>(F, n, r, ldf, labels, k, rpb, part, pcount,
                                                                          to_bat(b), rs);
    else if (4 * lds <= 64 * 1024)
        update_partial4_kernel<<<g1, 256, 4 * lds, s>>>(F, n, r, ldf, labels, k, rpb, part, pcount, to_bat(b));
    else if (lds <= 64 * 1024)
        update_partial_kernel<<<g1, threads, lds, s>>>(F, n, r, ldf, labels, k, rpb, part, pcount, to_bat(b));
    else
        update_partial_global_kernel<<<g1, threads, 0, s>>>(F, n, r, ldf, labels, k, rpb, part, pcount, to_bat(b));
    const int64_t kr = (int64_t)k * r;
    const int64_t cap = b.count <= 1 ? 4096 : std::max<int64_t>(1, 65536 / b.count);
    if (nb <= 32) {
        const dim3 gl((unsigned)std::max<int64_t>(1, std::min((kr + 255) / 256, cap)), (unsigned)b.count);
        if (nb <= 8)
            update_final_lanes_kernel<8><<<gl, 256, 0, s>>>(nb, r, k, part, pcount, C, counts, to_bat(b));
        else if (nb <= 16)
            update_final_lanes_kernel<16><<<gl, 256, 0, s>>>(nb, r, k, part, pcount, C, counts, to_bat(b));
        else
            update_final_lanes_kernel<32><<<gl, 256, 0, s>>>(nb, r, k, part, pcount, C, counts, to_bat(b));
        return;
    }
    const int64_t want = (kr * 64 + 255) / 256;
    const dim3 g2((unsigned)std::max<int64_t>(1, std::min(want, cap)), (unsigned)b.count);
    update_final_kernel<<<g2, 256, 0, s>>>(nb, r, k, part, pcount, C, counts, to_bat(b));
}

void km_zero_stamps(uint32_t *stamp, int64_t count, hipStream_t s) {
    zero_u32_kernel<<<(unsigned)std::min<int64_t>((count + NT - 1) / NT, 256), NT, 0, s>>>(stamp, count);
}

// Lloyd's steps stop per problem at a fixed point: once an assignment leaves
// every label of a problem as it was, its update would return the centroids
// it already has (the same member sums in the same order; an empty cluster
// keeps its centroid) and every later step would repeat itself, so those
// steps are skipped, which leaves the labels and centroids bit for bit as if
// they had run.  Assignment it (it >= 1) stamps base + it + 1 on a problem
// whose labels it changes; the update of step it runs only with that stamp,
// and the assignment of step it + 1 only with the stamp of step it.
void km_lloyd(const float *F, int64_t n, int64_t r, int64_t ldf, const int32_t *rows, int k, int iters, float *C,
              int32_t *labels, double *dist64, void *ws, uint32_t *stamp, uint32_t base, const KmBatch &b,
              hipStream_t s) {
    km_init_rows(F, n, r, ldf, rows, k, C, b, s);
    for (int it = 0; it < iters; ++it) {
        KmBatch ba = b, bu = b;
        ba.stamp = bu.stamp = stamp;
        ba.want = it >= 2 ? base + (uint32_t)it : 0u;
        ba.mark = it >= 1 ? base + (uint32_t)it + 1u : 0u;
        bu.want = it >= 1 ? base + (uint32_t)it + 1u : 0u;
        km_assign(F, n, r, ldf, C, k, labels, nullptr, nullptr, ba, s);
        km_update(F, n, r, ldf, labels, k, C, nullptr, ws, bu, s);
    }
    km_assign(F, n, r, ldf, C, k, labels, nullptr, dist64, b, s);
}

void km_select(const double *dist64, const int32_t *lab_all, int64_t n, int groups, int reps, double *inert,
               int32_t *lab_out, double *inertia_out, const float *C_all, int64_t ckr, float *C_out, hipStream_t s) {
    inertia_kernel<<<(unsigned)(groups * reps), NT, 0, s>>>(dist64, n, inert);
    select_kernel<<<dim3((unsigned)std::min<int64_t>((n + NT - 1) / NT, 64), (unsigned)groups), NT, 0, s>>>(
        inert, lab_all, n, reps, lab_out, inertia_out, C_all, ckr, C_out);
}

}  // namespace asc

using namespace asc;

extern "C" asc_status asc_normalize_features(float *Y, int64_t n, int64_t r, int64_t ldy, float *norms, void *stream) {
    const char *who = "asc_normalize_features";
    if (!Y || n < 1 || n >= (int64_t(1) << 31) || r < 1 || r > 65536 || ldy < r || !aligned(Y, 4) ||
        (norms && !aligned(norms, 4)))
        return fail(ASC_ERR_INVALID, "%s: bad arguments", who);
    km_normalize(Y, n, r, ldy, norms, as_stream(stream));
    ASC_LAUNCHED();
    return ASC_OK;
}

extern "C" asc_status asc_kmeans_init_rows(const float *F, int64_t n, int64_t r, int64_t ldf, const int32_t *rows,
                                           int k, float *C, void *stream) {
    const char *who = "asc_kmeans_init_rows";
    ASC_TRY(check_feat(F, n, r, ldf, who));
    if (!rows || !C || k < 1 || k > 1024 || !aligned(rows, 4) || !aligned(C, 4))
        return fail(ASC_ERR_INVALID, "%s: bad arguments", who);
    km_init_rows(F, n, r, ldf, rows, k, C, KmBatch{}, as_stream(stream));
    ASC_LAUNCHED();
    return ASC_OK;
}

extern "C" asc_status asc_kmeans_assign(const float *F, int64_t n, int64_t r, int64_t ldf, const float *C, int k,
                                        int32_t *labels, float *dist2, void *stream) {
    const char *who = "asc_kmeans_assign";
    ASC_TRY(check_feat(F, n, r, ldf, who));
    if (!C || !labels || k < 1 || k > 1024 || !aligned(C, 4) || !aligned(labels, 4) || (dist2 && !aligned(dist2, 4)))
        return fail(ASC_ERR_INVALID, "%s: bad arguments", who);
    km_assign(F, n, r, ldf, C, k, labels, dist2, nullptr, KmBatch{}, as_stream(stream));
    ASC_LAUNCHED();
    return ASC_OK;
}

extern "C" size_t asc_kmeans_update_workspace(int64_t n, int64_t r, int k) { return km_update_ws(n, r, k, 1); }

extern "C" asc_status asc_kmeans_update(const float *F, int64_t n, int64_t r, int64_t ldf, const int32_t *labels,
                                        int k, float *C, int64_t *counts, void *ws, size_t ws_bytes, void *stream) {
    const char *who = "asc_kmeans_update";
    ASC_TRY(check_feat(F, n, r, ldf, who));
    if (!labels || !C || k < 1 || k > 1024 || !aligned(labels, 4) || !aligned(C, 4) || (counts && !aligned(counts, 8)))
        return fail(ASC_ERR_INVALID, "%s: bad arguments", who);
    ASC_TRY(check_ws(ws, ws_bytes, asc_kmeans_update_workspace(n, r, k), who));
    km_update(F, n, r, ldf, labels, k, C, counts, ws, KmBatch{}, as_stream(stream));
    ASC_LAUNCHED();
    return ASC_OK;
}

static KmBatch replicate_batch(int64_t n, int64_t r, int k, int reps) {
    KmBatch b;
    b.count = reps;
    b.fstride = 0;  // every replicate reads the same rows
    b.cstride = (int64_t)k * r;
    b.lstride = n;
    b.rows_stride = k;
    return b;
}

struct RepWs {
    float *C;
    int32_t *lab;
    double *dist64;
    double *inert;
    uint32_t *stamp;
    void *kmws;
};

static size_t replicates_layout(int64_t n, int64_t r, int k, int reps, void *ws, RepWs *out) {
    Arena a(ws);
    RepWs w;
    w.C = a.take<float>((size_t)reps * k * r);
    w.lab = a.take<int32_t>((size_t)reps * n);
    w.dist64 = a.take<double>((size_t)reps * n);
    w.inert = a.take<double>((size_t)reps);
    w.stamp = a.take<uint32_t>((size_t)reps);
    w.kmws = a.take<char>(km_update_ws(n, r, k, reps));
    if (out) *out = w;
    return a.size();
}

extern "C" size_t asc_kmeans_replicates_workspace(int64_t n, int64_t r, int k, int reps) {
    if (n < 1 || r < 1 || k < 1 || reps < 1) return 0;
    return replicates_layout(n, r, k, reps, nullptr, nullptr);
}

extern "C" asc_status asc_kmeans_replicates(const float *F, int64_t n, int64_t r, int64_t ldf, int k, int reps,
                                            int iters, const int32_t *rows, int32_t *labels, float *C,
                                            double *inertia, void *ws, size_t ws_bytes, void *stream) {
    const char *who = "asc_kmeans_replicates";
    ASC_TRY(check_feat(F, n, r, ldf, who));
    if (k < 1 || k > 1024) return fail(ASC_ERR_INVALID, "%s: k=%d not in [1, 1024]", who, k);
    if (reps < 1 || reps > 65535) return fail(ASC_ERR_INVALID, "%s: reps=%d not in [1, 65535]", who, reps);
    if (iters < 0 || iters > 10000) return fail(ASC_ERR_INVALID, "%s: iters=%d not in [0, 10000]", who, iters);
    if (!rows || !labels || !aligned(rows, 4) || !aligned(labels, 4) || (C && !aligned(C, 4)) ||
        (inertia && !aligned(inertia, 8)))
        return fail(ASC_ERR_INVALID, "%s: rows/labels NULL or an argument misaligned", who);
    ASC_TRY(check_ws(ws, ws_bytes, asc_kmeans_replicates_workspace(n, r, k, reps), who));
    hipStream_t s = as_stream(stream);
    RepWs w;
    replicates_layout(n, r, k, reps, ws, &w);
    const KmBatch b = replicate_batch(n, r, k, reps);
    km_zero_stamps(w.stamp, reps, s);
    km_lloyd(F, n, r, ldf, rows, k, iters, w.C, w.lab, w.dist64, w.kmws, w.stamp, 0u, b, s);
    km_select(w.dist64, w.lab, n, 1, reps, w.inert, labels, inertia, w.C, (int64_t)k * r, C, s);
    ASC_LAUNCHED();
    return ASC_OK;
}
