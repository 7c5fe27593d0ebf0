// Stability measure gamma(k) for choosing the number of clusters (Sec. 4.3,
// Eq. stab): for every k in [k_min, k_max], the algorithm of Sec. 4.1 runs on
// J independent realisations of its random signals, and gamma(k) is the mean
// adjusted Rand index (Hubert & Arabie) over the J(J-1)/2 pairs of the
// resulting clusterings.
//
// MI355X design.  One recurrence pass over all J * eta_max signal columns keeps
// every state T_t R in the state store (the CSR is streamed once per step for
// all realisations and all k).  Everything that depends on k is then formed
// from the store without touching the graph again:
//   * per-column moments mu_{t,c} = <R_c, T_t R_c> (float64, fixed order), so
//     the eigenvalue count of realisation j for k is (1/eta_k) sum_t a_t(lc)
//     sum_{c < eta_k} mu_{t, j eta_max + c} and every (k, j) dichotomy runs on
//     the device in one launch;
//   * per k, the features Y = sum_t a_t T_t over the first eta_k columns of
//     every realisation (one launch for all j), row normalisation, and k-means
//     for all J x reps problems at once (batched launches), the least-inertia
//     replicate per realisation, then the pairwise ARIs from exact integer
//     contingency tables in LDS.
#include "common.hpp"
#include "cluster.hpp"
#include "coeffs.hpp"
#include "store.hpp"

#include <algorithm>

namespace asc {
namespace {

constexpr int NT = 256;
constexpr int kMaxClusters = 128;  // k x k contingency table of ints in LDS (64 KB)
constexpr int kMaxNk = 256;
constexpr int kMaxJ = 1024;
constexpr int kMaxP = 8192;
constexpr int64_t kChunkRows = 2048;

__device__ __forceinline__ float elem_f32(float v) { return v; }
__device__ __forceinline__ float elem_f32(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }

// mu partial sums over one chunk of rows: block (chunk, state t, slice);
// thread = (row lane, column), rows strided by the number of row lanes, the
// row lanes then added in order (deterministic)
template <typename TS>
__global__ __launch_bounds__(NT) void colmom_partial_kernel(int64_t n, int rs, const TS *__restrict__ store,
                                                            int64_t slot_elems, int p, int64_t rows_per_chunk,
                                                            int nchunks, double *__restrict__ part) {
    __shared__ double red[NT];
    const int c = threadIdx.x % rs;
    const int rl = threadIdx.x / rs;
    const int nrl = NT / rs;
    const int64_t ch = blockIdx.x;
    const int t = blockIdx.y;
    const int64_t sl = blockIdx.z;
    const TS *T0 = store + sl * (p + 1) * slot_elems;
    const TS *Tt = T0 + (int64_t)t * slot_elems;
    const int64_t i0 = ch * rows_per_chunk;
    const int64_t i1 = min(n, i0 + rows_per_chunk);
    double acc = 0.0;
    for (int64_t i = i0 + rl; i < i1; i += nrl) acc += (double)elem_f32(T0[i * rs + c]) * (double)elem_f32(Tt[i * rs + c]);
    red[threadIdx.x] = acc;
    __syncthreads();
    if (rl == 0) {
        double sum = 0.0;
        for (int q = 0; q < nrl; ++q) sum += red[q * rs + c];
        part[((sl * (p + 1) + t) * nchunks + ch) * rs + c] = sum;
    }
}

// mu[t][col] = sum over chunks in order
__global__ void colmom_final_kernel(const double *__restrict__ part, int rs, int p, int nchunks, int64_t C,
                                    double *__restrict__ mu) {
    const int64_t total = (int64_t)(p + 1) * C;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(q / C);
        const int64_t col = q - (int64_t)t * C;
        const int64_t sl = col / rs;
        const int c = (int)(col - sl * rs);
        const double *pp = part + ((sl * (p + 1) + t) * nchunks) * rs + c;
        double s = 0.0;
        for (int ch = 0; ch < nchunks; ++ch) s += pp[(int64_t)ch * rs];
        mu[q] = s;
    }
}

struct Etas {
    int v[kMaxNk];
};

// M[kk][j][t] = (1/eta_kk) sum_{c < eta_kk} mu[t][j eta_max + c]: the moments
// of realisation j's signals at variance 1/eta (Sec. 3.1)
__global__ void msum_kernel(const double *__restrict__ mu, int64_t C, int p, int J, int64_t eta_max, int nk, Etas et,
                            double *__restrict__ M) {
    const int64_t per_k = (int64_t)J * (p + 1);
    const int64_t total = (int64_t)nk * per_k;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int kk = (int)(q / per_k);
        const int64_t rem = q - (int64_t)kk * per_k;
        const int j = (int)(rem / (p + 1));
        const int t = (int)(rem - (int64_t)j * (p + 1));
        const int eta = et.v[kk];
        const double *row = mu + (int64_t)t * C + (int64_t)j * eta_max;
        double s = 0.0;
        for (int c = 0; c < eta; ++c) s += row[c];
        M[q] = s / (double)eta;
    }
}

// one block per (realisation j, k): dichotomy on [0, lmax] (Sec. 3.2) with
// count(lc) = sum_t a_t(lc) M_t, then the coefficients at the estimate
__global__ __launch_bounds__(NT) void stab_dichotomy_kernel(const double *__restrict__ M, int p,
                                                            const double *__restrict__ lmax, int k_min, int J,
                                                            int steps, double *__restrict__ lambda_k,
                                                            double *__restrict__ traj, double *__restrict__ coeffs) {
    __shared__ double lds[NT / 64];
    __shared__ double bc;
    const int j = blockIdx.x, kk = blockIdx.y;
    const int64_t pj = (int64_t)kk * J + j;
    const double *mu = M + pj * (p + 1);
    const double L = lmax[0];
    const int k = k_min + kk;
    double lo = 0.0, hi = L;
    for (int s = 0; s < steps; ++s) {
        const double mid = 0.5 * (lo + hi);
        double v[1] = {0.0};
        for (int t = threadIdx.x; t <= p; t += NT) v[0] += cheb_coeff_dev(mid, L, p, t, 1) * mu[t];
        block_sum<1, NT>(v, lds);
        if (threadIdx.x == 0) {
            bc = v[0];
            if (traj) {
                traj[(pj * steps + s) * 2] = mid;
                traj[(pj * steps + s) * 2 + 1] = v[0];
            }
        }
        __syncthreads();
        if (bc >= k - 0.5) hi = mid; else lo = mid;
        __syncthreads();
    }
    if (threadIdx.x == 0) lambda_k[pj] = hi;
    for (int t = threadIdx.x; t <= p; t += NT) coeffs[pj * (p + 1) + t] = cheb_coeff_dev(hi, L, p, t, 1);
}

// features of one k for every realisation: Y[j][i][c] = sum_t a_{k,j,t} T_t[i][j eta_max + c],
// c < eta; coefficients staged in LDS, t summed in order with float32 fma
template <typename TS>
__global__ __launch_bounds__(NT) void stab_combine_kernel(int64_t n, int rs, const TS *__restrict__ store,
                                                          int64_t slot_elems, int p, int64_t eta_max, int eta,
                                                          const double *__restrict__ coeffs, float *__restrict__ Y,
                                                          int64_t ldy) {
    extern __shared__ float cs[];  // p + 1
    const int j = blockIdx.y;
    for (int t = threadIdx.x; t <= p; t += NT) cs[t] = (float)coeffs[(int64_t)j * (p + 1) + t];
    __syncthreads();
    const int64_t total = n * eta;
    float *Yj = Y + (int64_t)j * n * ldy;
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < total; q += (int64_t)gridDim.x * NT) {
        const int64_t i = q / eta;
        const int c = (int)(q - i * eta);
        const int64_t col = (int64_t)j * eta_max + c;
        const int64_t sl = col / rs;
        const int64_t cc = col - sl * rs;
        const TS *src = store + sl * (p + 1) * slot_elems + i * rs + cc;
        float acc = 0.0f;
        for (int t = 0; t <= p; ++t) acc = fmaf(cs[t], elem_f32(src[(int64_t)t * slot_elems]), acc);
        Yj[i * ldy + c] = acc;
    }
}

// The same features for every k at once (up to 32 values of k), from one
// read of the store instead of one per k: a lane keeps one float32
// accumulator per k and adds, for t in order, fma(a_{k,j,t}, T_t[i][col])
// exactly as stab_combine_kernel does for one k (identical features).  The
// coefficients come from cfT[j][t][u] = (float) a_{u,j,t} (zero for u >= nk),
// the same at every lane of a block, so they are scalar loads.
constexpr int kCombineAllMax = 32;
struct CombineAll {
    int nk;
    int eta[kCombineAllMax];
    int ld[kCombineAllMax];
    int64_t off[kCombineAllMax];  // element offset of the block of k_min + u in Y, laid out [J][n][ld]
};

__global__ void stab_cf_table_kernel(const double *__restrict__ coeffs, int nk, int J, int p, float *__restrict__ cfT) {
    const int64_t total = (int64_t)J * (p + 1) * kCombineAllMax;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int u = (int)(q % kCombineAllMax);
        const int64_t jt = q / kCombineAllMax;  // j (p + 1) + t
        const int j = (int)(jt / (p + 1));
        const int t = (int)(jt - (int64_t)j * (p + 1));
        cfT[q] = u < nk ? (float)coeffs[((int64_t)u * J + j) * (p + 1) + t] : 0.0f;
    }
}

template <typename TS, int NKC>
__global__ __launch_bounds__(NT) void stab_combine_all_kernel(int64_t n, int rs, const TS *__restrict__ store,
                                                              int64_t slot_elems, int p, int64_t eta_max,
                                                              int eta_used, const float *__restrict__ cfT,
                                                              float *__restrict__ Y, CombineAll ca) {
    const int j = blockIdx.y;
    const float *cfj = cfT + (int64_t)j * (p + 1) * kCombineAllMax;
    const int64_t total = n * eta_used;
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < total; q += (int64_t)gridDim.x * NT) {
        const int64_t i = q / eta_used;
        const int c = (int)(q - i * eta_used);
        const int64_t col = (int64_t)j * eta_max + c;
        const int64_t sl = col / rs;
        const int64_t cc = col - sl * rs;
        const TS *src = store + sl * (p + 1) * slot_elems + i * rs + cc;
        float acc[NKC];
#pragma unroll
        for (int u = 0; u < NKC; ++u) acc[u] = 0.0f;
        for (int t = 0; t <= p; ++t) {
            const float x = elem_f32(src[(int64_t)t * slot_elems]);
            const float *cf = cfj + (int64_t)t * kCombineAllMax;
#pragma unroll
            for (int u = 0; u < NKC; ++u) acc[u] = fmaf(cf[u], x, acc[u]);
        }
#pragma unroll
        for (int u = 0; u < NKC; ++u)
            if (u < ca.nk && c < ca.eta[u]) Y[ca.off[u] + ((int64_t)j * n + i) * ca.ld[u] + c] = acc[u];
    }
}

__device__ __forceinline__ long long wave_sum_i64(long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double i128_to_f64(__int128 x) {
    const bool neg = x < 0;
    const unsigned __int128 m = neg ? (unsigned __int128)(-x) : (unsigned __int128)x;
    const double d = (double)(uint64_t)(m >> 64) * 18446744073709551616.0 + (double)(uint64_t)m;
    return neg ? -d : d;
}

// one block per pair (a, b), a < b, in the order (0,1), (0,2), ..., (1,2), ...:
// contingency table n_uv in LDS (integer atomics), then
//   index = sum C(n_uv, 2), sa = sum_u C(row_u, 2), sb = sum_v C(col_v, 2),
//   ARI = 2 (index C(n,2) - sa sb) / ((sa + sb) C(n,2) - 2 sa sb)
// with exact 128-bit integers up to the final division (1 when it is 0/0)
__global__ __launch_bounds__(NT) void ari_kernel(const int32_t *__restrict__ labels, int64_t n, int64_t ldl, int J,
                                                 int k, double *__restrict__ ari, uint32_t *__restrict__ flags) {
    extern __shared__ int tab[];  // k * k (reused for the cross-wavefront sums: 64 KB at k = 128)
    int a = 0;
    int rem = blockIdx.x;
    while (rem >= J - 1 - a) {
        rem -= J - 1 - a;
        ++a;
    }
    const int b = a + 1 + rem;
    for (int x = threadIdx.x; x < k * k; x += NT) tab[x] = 0;
    __syncthreads();
    const int32_t *la = labels + (int64_t)a * ldl;
    const int32_t *lb = labels + (int64_t)b * ldl;
    bool bad = false;
    for (int64_t i = threadIdx.x; i < n; i += NT) {
        const int u = la[i], v = lb[i];
        if (u >= 0 && u < k && v >= 0 && v < k) atomicAdd(&tab[u * k + v], 1);
        else bad = true;
    }
    if (bad && flags) atomicOr(flags, ASC_FLAG_BAD_INPUT);
    __syncthreads();
    long long idx = 0, sa = 0, sb = 0;
    for (int x = threadIdx.x; x < k * k; x += NT) {
        const long long m = tab[x];
        idx += m * (m - 1) / 2;
    }
    for (int u = threadIdx.x; u < k; u += NT) {
        long long rs = 0, cs = 0;
        for (int v = 0; v < k; ++v) {
            rs += tab[u * k + v];
            cs += tab[v * k + u];
        }
        sa += rs * (rs - 1) / 2;
        sb += cs * (cs - 1) / 2;
    }
    idx = wave_sum_i64(idx);
    sa = wave_sum_i64(sa);
    sb = wave_sum_i64(sb);
    // the number of rows that carried valid labels in both
    long long m = 0;
    for (int x = threadIdx.x; x < k * k; x += NT) m += tab[x];
    m = wave_sum_i64(m);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();  // every read of the table is done: its memory now holds the wavefront sums
    long long *red = reinterpret_cast<long long *>(tab);  // [4][NT / 64]
    if (lane == 0) {
        red[0 * (NT / 64) + wave] = idx;
        red[1 * (NT / 64) + wave] = sa;
        red[2 * (NT / 64) + wave] = sb;
        red[3 * (NT / 64) + wave] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        idx = sa = sb = m = 0;
        for (int w = 0; w < NT / 64; ++w) {
            idx += red[0 * (NT / 64) + w];
            sa += red[1 * (NT / 64) + w];
            sb += red[2 * (NT / 64) + w];
            m += red[3 * (NT / 64) + w];
        }
        const __int128 n2 = (__int128)(m * (m - 1) / 2);
        double v = 1.0;
        if (n2 > 0) {
            const __int128 num = 2 * ((__int128)idx * n2 - (__int128)sa * sb);
            const __int128 den = (__int128)(sa + sb) * n2 - 2 * (__int128)sa * sb;
            if (den != 0) v = i128_to_f64(num) / i128_to_f64(den);
        }
        ari[blockIdx.x] = v;
    }
}

__global__ void clear_flags_kernel(uint32_t *flags) { flags[0] = 0u; }

// dynamic LDS of ari_kernel: the k x k table, at least the 4 x (NT/64) wavefront sums it later holds
size_t ari_lds(int k) {
    return std::max<size_t>((size_t)k * k * sizeof(int), 4 * (NT / 64) * sizeof(long long));
}

// gamma = mean of the pair ARIs (one wavefront, fixed order)
__global__ void gamma_kernel(const double *__restrict__ ari, int npairs, double *__restrict__ gamma) {
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    for (int q = lane; q < npairs; q += 64) s += ari[q];
    s = wave_sum(s);
    if (lane == 0) gamma[0] = s / (double)npairs;
}

struct StabWs {
    WsHeader *hdr;
    void *store;
    void *sws;
    double *part;
    double *mu;
    double *M;
    double *lam;
    double *coeffs;
    float *Y;
    float *cfT;  // all-k coefficient table (when every k's features are formed at once)
    float *C;
    int32_t *lab_all;
    double *dist64;
    double *inert;  // per (realisation, replicate) inertia
    uint32_t *stamp;  // per (realisation, replicate): the last Lloyd step that moved a label
    void *kmws;
    double *ari;
    int32_t *labels;
};

struct StabDims {
    int64_t n, C;
    int nk, J, reps, p, steps, kmax, etamax_used;
    int64_t eta_max;
    int nchunks;
    StoreLayout S;
    bool all_k;      // every k's features formed in one pass over the store
    int64_t ld_sum;  // sum over k of the feature leading dimensions
};

size_t stab_ws_layout(const asc_graph *g, const StabDims &d, asc_dtype sig, void *ws, StabWs *out) {
    Arena a(ws);
    StabWs w;
    const int64_t n = d.n;
    const int64_t npairs = (int64_t)d.J * (d.J - 1) / 2;
    const int64_t ldmax = ((int64_t)d.etamax_used + 3) & ~int64_t(3);
    // the recurrence's workspace comes first: its header (cleared by the
    // recurrence, then raised by any kernel here) is the header of ws
    w.sws = a.take<char>(store_ws_bytes(n, d.C, sig));
    w.hdr = static_cast<WsHeader *>(w.sws);
    w.store = a.take<char>((size_t)d.S.nslices * (d.p + 1) * d.S.panel_bytes);
    w.part = a.take<double>((size_t)d.S.nslices * (d.p + 1) * d.nchunks * d.S.rs);
    w.mu = a.take<double>((size_t)(d.p + 1) * d.C);
    w.M = a.take<double>((size_t)d.nk * d.J * (d.p + 1));
    w.lam = a.take<double>((size_t)d.nk * d.J);
    w.coeffs = a.take<double>((size_t)d.nk * d.J * (d.p + 1));
    w.Y = a.take<float>((size_t)d.J * n * (d.all_k ? d.ld_sum : ldmax));
    w.cfT = d.all_k ? a.take<float>((size_t)d.J * (d.p + 1) * kCombineAllMax) : nullptr;
    w.C = a.take<float>((size_t)d.J * d.reps * d.kmax * d.etamax_used);
    w.lab_all = a.take<int32_t>((size_t)d.J * d.reps * n);
    w.dist64 = a.take<double>((size_t)d.J * d.reps * n);
    w.inert = a.take<double>((size_t)d.J * d.reps);
    w.stamp = a.take<uint32_t>((size_t)d.J * d.reps);
    w.kmws = a.take<char>(km_update_ws(n, d.etamax_used, d.kmax, d.J * d.reps));
    w.ari = a.take<double>((size_t)npairs);
    w.labels = a.take<int32_t>((size_t)d.J * n);
    (void)g;
    if (out) *out = w;
    return a.size();
}

asc_status stab_dims(const asc_graph *g, int k_min, int k_max, const int *eta, int J, int reps, int p, int steps,
                     asc_dtype sig, int64_t eta_max, const char *who, StabDims *d) {
    ASC_TRY(check_graph_args(g, true, who));
    if (sig != ASC_F32 && sig != ASC_BF16) return fail(ASC_ERR_INVALID, "%s: unknown dtype", who);
    if (k_min < 1 || k_max < k_min || k_max > kMaxClusters || k_max > g->n || k_max - k_min + 1 > kMaxNk)
        return fail(ASC_ERR_INVALID, "%s: k range [%d, %d] (1 <= k_min <= k_max <= min(n, %d), at most %d values)",
                    who, k_min, k_max, kMaxClusters, kMaxNk);
    if (J < 2 || J > kMaxJ) return fail(ASC_ERR_INVALID, "%s: J=%d not in [2, %d]", who, J, kMaxJ);
    if (reps < 1 || (int64_t)J * reps > 65535) return fail(ASC_ERR_INVALID, "%s: reps=%d (J*reps <= 65535)", who, reps);
    if (p < 1 || p > kMaxP) return fail(ASC_ERR_INVALID, "%s: p=%d not in [1, %d]", who, p, kMaxP);
    if (steps < 0 || steps > 200) return fail(ASC_ERR_INVALID, "%s: steps=%d", who, steps);
    if (eta_max < 1 || (int64_t)J * eta_max > 65536)
        return fail(ASC_ERR_INVALID, "%s: eta_max=%lld (J*eta_max <= 65536)", who, (long long)eta_max);
    if (!eta) return fail(ASC_ERR_INVALID, "%s: eta_host is NULL", who);
    d->nk = k_max - k_min + 1;
    d->etamax_used = 0;
    for (int q = 0; q < d->nk; ++q) {
        if (eta[q] < 1 || eta[q] > eta_max)
            return fail(ASC_ERR_INVALID, "%s: eta[%d]=%d not in [1, eta_max=%lld]", who, q, eta[q], (long long)eta_max);
        d->etamax_used = std::max(d->etamax_used, eta[q]);
    }
    d->n = g->n;
    d->C = (int64_t)J * eta_max;
    d->J = J;
    d->reps = reps;
    d->p = p;
    d->steps = steps;
    d->kmax = k_max;
    d->eta_max = eta_max;
    d->nchunks = (int)std::max<int64_t>(1, (g->n + kChunkRows - 1) / kChunkRows);
    d->S = store_layout(g, d->C, sig);
    d->ld_sum = 0;
    for (int q = 0; q < d->nk; ++q) d->ld_sum += ((int64_t)eta[q] + 3) & ~int64_t(3);
    // all k at once while the coefficient table stays small (a few MB)
    d->all_k = d->nk <= kCombineAllMax && (size_t)J * (p + 1) * kCombineAllMax * sizeof(float) <= (size_t(64) << 20);
    return ASC_OK;
}

template <typename TS>
void launch_colmom(const StabDims &d, const StabWs &w, hipStream_t s) {
    const int64_t slot_elems = (int64_t)(d.S.panel_bytes / sizeof(TS));
    const int64_t rpc = (d.n + d.nchunks - 1) / d.nchunks;
    const dim3 grid((unsigned)d.nchunks, (unsigned)(d.p + 1), (unsigned)d.S.nslices);
    colmom_partial_kernel<TS><<<grid, NT, 0, s>>>(d.n, d.S.rs, static_cast<const TS *>(w.store), slot_elems, d.p, rpc,
                                                  d.nchunks, w.part);
}

template <typename TS>
void launch_combine(const StabDims &d, const StabWs &w, int eta, const double *coeffs_k, int64_t ldy, hipStream_t s) {
    const int64_t slot_elems = (int64_t)(d.S.panel_bytes / sizeof(TS));
    const int64_t total = d.n * eta;
    const int bx = (int)std::max<int64_t>(1, std::min<int64_t>((total + NT - 1) / NT, std::max(1, 16384 / d.J)));
    stab_combine_kernel<TS><<<dim3((unsigned)bx, (unsigned)d.J), NT, (size_t)(d.p + 1) * sizeof(float), s>>>(
        d.n, d.S.rs, static_cast<const TS *>(w.store), slot_elems, d.p, d.eta_max, eta, coeffs_k, w.Y, ldy);
}

// every k's features in one pass (d.all_k); offsets of the per-k blocks in ca
template <typename TS>
void launch_combine_all(const StabDims &d, const StabWs &w, const int *eta_host, CombineAll &ca, hipStream_t s) {
    ca.nk = d.nk;
    int64_t off = 0;
    for (int u = 0; u < d.nk; ++u) {
        ca.eta[u] = eta_host[u];
        ca.ld[u] = (eta_host[u] + 3) & ~3;
        ca.off[u] = off;
        off += (int64_t)d.J * d.n * ca.ld[u];
    }
    const int64_t tcf = (int64_t)d.J * (d.p + 1) * kCombineAllMax;
    stab_cf_table_kernel<<<(unsigned)std::min<int64_t>((tcf + 255) / 256, 16384), 256, 0, s>>>(w.coeffs, d.nk, d.J,
                                                                                              d.p, w.cfT);
    const int64_t slot_elems = (int64_t)(d.S.panel_bytes / sizeof(TS));
    const int64_t total = d.n * d.etamax_used;
    const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>((total + NT - 1) / NT, std::max(1, 16384 / d.J))),
                    (unsigned)d.J);
    const TS *st = static_cast<const TS *>(w.store);
    if (d.nk <= 8)
        stab_combine_all_kernel<TS, 8><<<grid, NT, 0, s>>>(d.n, d.S.rs, st, slot_elems, d.p, d.eta_max,
                                                           d.etamax_used, w.cfT, w.Y, ca);
    else if (d.nk <= 16)
        stab_combine_all_kernel<TS, 16><<<grid, NT, 0, s>>>(d.n, d.S.rs, st, slot_elems, d.p, d.eta_max,
                                                            d.etamax_used, w.cfT, w.Y, ca);
    else
        stab_combine_all_kernel<TS, 32><<<grid, NT, 0, s>>>(d.n, d.S.rs, st, slot_elems, d.p, d.eta_max,
                                                            d.etamax_used, w.cfT, w.Y, ca);
}

}  // namespace
}  // namespace asc

using namespace asc;

extern "C" size_t asc_stability_workspace(const asc_graph *g, int k_min, int k_max, const int *eta_host, int J,
                                          int reps, int p, int steps, asc_dtype sig, int64_t eta_max) {
    StabDims d;
    if (stab_dims(g, k_min, k_max, eta_host, J, reps, p, steps, sig, eta_max, "asc_stability_workspace", &d) != ASC_OK)
        return 0;
    return stab_ws_layout(g, d, sig, nullptr, nullptr);
}

extern "C" asc_status asc_stability(const asc_graph *g, const double *lmax, int k_min, int k_max, const int *eta_host,
                                    int J, int reps, int p, int steps, int kmeans_iters, const void *R, asc_dtype sig,
                                    int64_t eta_max, int64_t ldr, const int32_t *init_rows, double *gamma,
                                    double *ari, int32_t *labels, double *lambda_k, double *traj, double *inertia,
                                    void *ws, size_t ws_bytes, void *stream) {
    const char *who = "asc_stability";
    StabDims d;
    ASC_TRY(stab_dims(g, k_min, k_max, eta_host, J, reps, p, steps, sig, eta_max, who, &d));
    ASC_TRY(check_block(R, sig, g->n, d.C, ldr, who, "R"));
    if (!lmax || !aligned(lmax, 8)) return fail(ASC_ERR_INVALID, "%s: lmax NULL or misaligned", who);
    if (kmeans_iters < 0 || kmeans_iters > 10000) return fail(ASC_ERR_INVALID, "%s: kmeans_iters=%d", who, kmeans_iters);
    if (!init_rows || !aligned(init_rows, 4)) return fail(ASC_ERR_INVALID, "%s: init_rows NULL or misaligned", who);
    if (!gamma || !aligned(gamma, 8)) return fail(ASC_ERR_INVALID, "%s: gamma NULL or misaligned", who);
    if ((ari && !aligned(ari, 8)) || (labels && !aligned(labels, 4)) || (lambda_k && !aligned(lambda_k, 8)) ||
        (traj && !aligned(traj, 8)) || (inertia && !aligned(inertia, 8)))
        return fail(ASC_ERR_INVALID, "%s: an output is misaligned", who);
    ASC_TRY(check_ws(ws, ws_bytes, stab_ws_layout(g, d, sig, nullptr, nullptr), who));
    hipStream_t s = as_stream(stream);
    StabWs w;
    stab_ws_layout(g, d, sig, ws, &w);
    const int64_t n = d.n;
    const int npairs = J * (J - 1) / 2;
    // 1. every state of every signal column, one recurrence pass
    ASC_TRY(run_store(g, lmax, p, R, sig, d.C, ldr, w.store, w.sws, s));
    // 2. per-column moments, per-(k, j) moments and dichotomies
    if (sig == ASC_F32) launch_colmom<float>(d, w, s);
    else launch_colmom<uint16_t>(d, w, s);
    ASC_LAUNCHED();
    {
        const int64_t tot = (int64_t)(p + 1) * d.C;
        colmom_final_kernel<<<(unsigned)std::min<int64_t>((tot + 255) / 256, 16384), 256, 0, s>>>(
            w.part, d.S.rs, p, d.nchunks, d.C, w.mu);
        ASC_LAUNCHED();
        Etas et{};
        for (int q = 0; q < d.nk; ++q) et.v[q] = eta_host[q];
        const int64_t totm = (int64_t)d.nk * J * (p + 1);
        msum_kernel<<<(unsigned)std::min<int64_t>((totm + 255) / 256, 16384), 256, 0, s>>>(w.mu, d.C, p, J, eta_max,
                                                                                           d.nk, et, w.M);
        ASC_LAUNCHED();
    }
    double *lam = lambda_k ? lambda_k : w.lam;
    stab_dichotomy_kernel<<<dim3((unsigned)J, (unsigned)d.nk), NT, 0, s>>>(w.M, p, lmax, k_min, J, steps, lam, traj,
                                                                          w.coeffs);
    ASC_LAUNCHED();
    // 3. features: every k's at once, or one k at a time below
    CombineAll ca{};
    if (d.all_k) {
        if (sig == ASC_F32) launch_combine_all<float>(d, w, eta_host, ca, s);
        else launch_combine_all<uint16_t>(d, w, eta_host, ca, s);
        ASC_LAUNCHED();
    }
    // 4. per k: (features,) normalisation, batched k-means, selection, ARIs
    km_zero_stamps(w.stamp, J * reps, s);
    ASC_LAUNCHED();
    for (int kk = 0; kk < d.nk; ++kk) {
        const int k = k_min + kk;
        const int eta = eta_host[kk];
        const int64_t ld = ((int64_t)eta + 3) & ~int64_t(3);
        float *Yk = d.all_k ? w.Y + ca.off[kk] : w.Y;
        if (!d.all_k) {
            const double *co = w.coeffs + (int64_t)kk * J * (p + 1);
            if (sig == ASC_F32) launch_combine<float>(d, w, eta, co, ld, s);
            else launch_combine<uint16_t>(d, w, eta, co, ld, s);
            ASC_LAUNCHED();
        }
        km_normalize(Yk, (int64_t)J * n, eta, ld, nullptr, s);
        ASC_LAUNCHED();
        KmBatch b;
        b.count = J * reps;
        b.fstride = n * ld;
        b.fdiv = reps;
        b.cstride = (int64_t)k * eta;
        b.lstride = n;
        b.rows_stride = k_max;
        const int32_t *rows_k = init_rows + (int64_t)kk * J * reps * k_max;
        // stamps grow over the whole sweep (base rises per k), so an older
        // k's stamps never let a problem run
        km_lloyd(Yk, n, eta, ld, rows_k, k, kmeans_iters, w.C, w.lab_all, w.dist64, w.kmws, w.stamp,
                 (uint32_t)kk * (uint32_t)(kmeans_iters + 1), b, s);
        ASC_LAUNCHED();
        int32_t *lab_k = labels ? labels + (int64_t)kk * J * n : w.labels;
        km_select(w.dist64, w.lab_all, n, J, reps, w.inert, lab_k, inertia ? inertia + (int64_t)kk * J * reps : nullptr,
                  nullptr, 0, nullptr, s);
        ASC_LAUNCHED();
        double *ari_k = ari ? ari + (int64_t)kk * npairs : w.ari;
        ari_kernel<<<npairs, NT, ari_lds(k), s>>>(lab_k, n, n, J, k, ari_k, &w.hdr->flags);
        ASC_LAUNCHED();
        gamma_kernel<<<1, 64, 0, s>>>(ari_k, npairs, gamma + kk);
        ASC_LAUNCHED();
    }
    return ASC_OK;
}

extern "C" size_t asc_ari_workspace(void) { return sizeof(WsHeader); }

extern "C" asc_status asc_ari_pairs(const int32_t *labels, int64_t n, int64_t ldl, int J, int k, double *ari,
                                    double *mean, void *ws, size_t ws_bytes, void *stream) {
    const char *who = "asc_ari_pairs";
    if (!labels || !aligned(labels, 4) || n < 1 || n >= (int64_t(1) << 31) || ldl < n)
        return fail(ASC_ERR_INVALID, "%s: labels NULL/misaligned or n=%lld ldl=%lld", who, (long long)n, (long long)ldl);
    if (J < 2 || J > kMaxJ) return fail(ASC_ERR_INVALID, "%s: J=%d not in [2, %d]", who, J, kMaxJ);
    if (k < 1 || k > kMaxClusters) return fail(ASC_ERR_INVALID, "%s: k=%d not in [1, %d]", who, k, kMaxClusters);
    if (!ari || !aligned(ari, 8) || (mean && !aligned(mean, 8)))
        return fail(ASC_ERR_INVALID, "%s: ari NULL or misaligned", who);
    ASC_TRY(check_ws(ws, ws_bytes, asc_ari_workspace(), who));
    hipStream_t s = as_stream(stream);
    WsHeader *hdr = static_cast<WsHeader *>(ws);
    const int npairs = J * (J - 1) / 2;
    clear_flags_kernel<<<1, 1, 0, s>>>(&hdr->flags);
    ASC_LAUNCHED();
    ari_kernel<<<npairs, NT, ari_lds(k), s>>>(labels, n, ldl, J, k, ari, &hdr->flags);
    ASC_LAUNCHED();
    if (mean) {
        gamma_kernel<<<1, 64, 0, s>>>(ari, npairs, mean);
        ASC_LAUNCHED();
    }
    return ASC_OK;
}
