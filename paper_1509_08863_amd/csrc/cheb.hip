// Polynomial low-pass filtering of random signals (Sec. 2.4, Sec. 3.1, steps
// 3-5 of the algorithm in Sec. 4.1) and the Chebyshev moments behind the
// eigenvalue count of Sec. 3.2.
//
// Data layout.  The caller's blocks are row-major n x r.  Internally the
// columns are processed in slices of RS columns (RS = lanes-per-row x 16 bytes
// of elements); each slice runs its whole recurrence before the next one, so
// the block that is gathered at random rows (T_j of the slice, n x RS) stays
// small enough to live in the 256 MB Infinity Cache.  Slice states live in
// "panels": n x RS, contiguous, zero-padded past column r.  Two panels
// suffice because T_{j+1} overwrites T_{j-1} row by row (row i of T_{j-1} is
// read only by the lanes that write row i of T_{j+1}).
//
// One recurrence step (kernel cheb_step):
//   T_{j+1}[i] = d_i T_j[i] + beta sum_k w_ik T_j[k] - T_{j-1}[i],
//   d_i = 4 s_i / lmax - 2, beta = -4 / lmax   (= 2 Lt T_j - T_{j-1}),
//   Y[i] += a_j T_j[i] + a_{j+1} T_{j+1}[i]      (fused, float32, every other
//                                                step; bfloat16 states: Y[i] +=
//                                                a_{j+1} T_{j+1}[i] every step),
// with LPR lanes of a wavefront per row (64/LPR rows per wavefront), each
// lane owning 16 bytes of the row: the gather of T_j[k] is one coalesced
// 16*LPR-byte segment per neighbour.  Optional float64 partial sums per block
// (|T_j|^2, <T_{j+1}, T_j>, |T_{j+1}|^2) feed the moments and the growth check.
#include "recurrence.hpp"
#include "coeffs.hpp"
#include "store.hpp"

#include <cmath>
#include <mutex>
#include <vector>

namespace asc {

std::mutex &tune_mutex() {
    static std::mutex m;
    return m;
}
std::vector<TuneEntry> &tune_table() {
    static std::vector<TuneEntry> t;
    return t;
}

bool tuned(int64_t n, int64_t nnz, int64_t r, asc_dtype dt, TuneEntry *out) {
    std::lock_guard<std::mutex> lk(tune_mutex());
    for (auto &e : tune_table())
        if (e.key == TuneKey{n, nnz, r, (int)dt}) {
            if (out) *out = e;
            return true;
        }
    return false;
}



// ---------------------------------------------------------------------------
// launches of a plan: one slice per launch, or every slice in one launch
// (variant bit 3; 8 lanes per row, 2 to 4 slices; of the other bits only the
// XCD-band schedule applies there)
// ---------------------------------------------------------------------------
template <typename TS>
hipError_t launch_np_t(unsigned var, int np, unsigned mode, const StepArgs &A, int grid, hipStream_t s) {
    const bool bands = (var & 4u) != 0;
    switch (np) {
        case 2: return bands ? launch_step_v<TS, 8, 4u, 2>(mode, A, grid, s) : launch_step_v<TS, 8, 0u, 2>(mode, A, grid, s);
        case 3: return bands ? launch_step_v<TS, 8, 4u, 3>(mode, A, grid, s) : launch_step_v<TS, 8, 0u, 3>(mode, A, grid, s);
        case 4: return bands ? launch_step_v<TS, 8, 4u, 4>(mode, A, grid, s) : launch_step_v<TS, 8, 0u, 4>(mode, A, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_plan(const Plan &P, asc_dtype dt, unsigned mode, const StepArgs &A, int grid, hipStream_t s) {
    if (P.np > 1)
        return dt == ASC_F32 ? launch_np_t<float>(P.var, P.np, mode, A, grid, s)
                             : launch_np_t<uint16_t>(P.var, P.np, mode, A, grid, s);
    return launch_step(dt, P.lpr, P.var, mode, A, grid, s);
}

// R columns c0 .. c0 + np*rs - 1 into np consecutive panels `pstride` elements apart
void pack_panels(const Plan &P, int64_t n, const void *R, asc_dtype sig, int64_t ldr, int64_t r, int sl0, void *dst,
                 int64_t pstride, hipStream_t s) {
    const int64_t tot = n * P.rs;
    const int pg = (int)std::min<int64_t>((tot + 255) / 256, 65536);
    for (int q = 0; q < P.np; ++q) {
        const int64_t c0 = (int64_t)(sl0 + q) * P.rs;
        if (sig == ASC_F32)
            pack_kernel<float><<<pg, 256, 0, s>>>(n, (const float *)R, ldr, c0, r, P.rs,
                                                  static_cast<float *>(dst) + q * pstride);
        else
            pack_kernel<uint16_t><<<pg, 256, 0, s>>>(n, (const uint16_t *)R, ldr, c0, r, P.rs,
                                                     static_cast<uint16_t *>(dst) + q * pstride);
    }
}

// ---------------------------------------------------------------------------
// the filter, shared by asc_cheb_filter and the literal eigencount
// ---------------------------------------------------------------------------
asc_status run_filter(const asc_graph *g, const double *lmax, const double *coeffs, int p, const void *R,
                      asc_dtype sig, int64_t r, int64_t ldr, float *Y, int64_t ldy, void *ckpt, int ckpt_stride,
                      void *ws, bool clear_flags, hipStream_t s) {
    const int64_t n = g->n;
    FilterWs F;
    const bool store_all = ckpt && ckpt_stride == 1;
    const Plan P = store_all ? store_plan(g, r, sig) : make_plan(g, r, sig);
    filter_ws_layout(n, rs_for_ws(r, sig), 1, sig, 2, 1, ws, &F);
    uint32_t *flags = &F.hdr->flags;
    diag_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, g->strength, lmax, F.diag, F.beta, flags,
                                                           clear_flags ? 1 : 0);
    ASC_LAUNCHED();
    if (p == 0) {
        const int64_t tot = n * r;
        const int grid = (int)std::min<int64_t>((tot + 255) / 256, 65536);
        if (sig == ASC_F32)
            scale_copy_kernel<float><<<grid, 256, 0, s>>>(n, r, (const float *)R, ldr, coeffs, Y, ldy);
        else
            scale_copy_kernel<uint16_t><<<grid, 256, 0, s>>>(n, r, (const uint16_t *)R, ldr, coeffs, Y, ldy);
        ASC_LAUNCHED();
        return ASC_OK;
    }
    const int grid = grid_for(n, P.lpr);
    // ckpt_stride >= 2: (T_sc, T_sc+1) pairs, row-major blocks; ckpt_stride == 1:
    // every state in panel layout [slice][j][n x rs] (the recurrence writes its
    // states straight into their slots, nothing is overwritten)
    const size_t ckb = (ckpt && !store_all) ? ck_block_bytes(n, r, sig) : 0;
    auto ck_block = [&](int seg, int which) -> void * {
        return static_cast<char *>(ckpt) + ((size_t)seg * 2 + which) * ckb;
    };
    const size_t pbytes = panel_bytes(n, P.rs, sig);
    auto slot = [&](int sl, int j) -> void * {
        return static_cast<char *>(ckpt) + ((size_t)sl * (p + 1) + j) * pbytes;
    };
    // panels of the slices of one launch: consecutive panels of the ping-pong
    // buffers, or the slots of consecutive slices in the state store
    const int64_t pstride = (int64_t)((store_all ? (size_t)(p + 1) * pbytes : pbytes) / esize(sig));
    for (int sl = 0; sl < P.nslices; sl += P.np) {
        const int64_t c0 = (int64_t)sl * P.rs;
        void *pa = store_all ? slot(sl, 0) : F.panelA;
        void *pb = store_all ? slot(sl, 1) : F.panelB;
        pack_panels(P, n, R, sig, ldr, r, sl, pa, pstride, s);
        ASC_LAUNCHED();
        StepArgs A{};
        A.pstride = pstride;
        A.n = n;
        A.rp = g->row_ptr;
        A.ci = g->col_idx;
        A.w = g->w;
        A.diag = F.diag;
        A.beta = F.beta;
        A.Y = Y;
        A.ldy = ldy;
        A.c0 = c0;
        A.r = r;
        A.coeffs = coeffs;
        // step 0: T_1 from T_0
        A.cur = pa;
        A.prev = nullptr;
        A.out = pb;
        A.j = 0;
        A.partials = F.part;  // partial slot 0: first step
        A.ck_ld = ck_ld_of(r, sig);
        A.ck_a = ckb ? ck_block(0, 0) : nullptr;
        A.ck_b = ckb ? ck_block(0, 1) : nullptr;
        hipError_t e = launch_plan(P, sig, M_FIRST | M_YACC | M_PART, A, grid, s);
        if (e != hipSuccess) return fail(ASC_ERR_HIP, "cheb_step launch failed: %s", hipGetErrorString(e));
        sum_partials_kernel<<<1, NT, 0, s>>>(grid, F.part, 1, 0, F.first);
        ASC_LAUNCHED();
        void *cur = pb, *prev = pa;
        for (int j = 1; j < p; ++j) {
            const bool last = (j == p - 1);
            A.cur = store_all ? slot(sl, j) : cur;
            A.prev = store_all ? slot(sl, j - 1) : prev;
            A.out = store_all ? slot(sl, j + 1) : prev;  // else T_{j+1} overwrites T_{j-1}
            A.j = j;
            A.partials = F.part + (int64_t)kMaxGrid * 3;
            const bool ck = ckb && (j % ckpt_stride == 0);
            A.ck_a = ck ? ck_block(j / ckpt_stride, 0) : nullptr;
            A.ck_b = ck ? ck_block(j / ckpt_stride, 1) : nullptr;
            e = launch_plan(P, sig, y_mode(j, p, sig) | (last ? M_PART : 0u), A, grid, s);
            if (e != hipSuccess) return fail(ASC_ERR_HIP, "cheb_step launch failed: %s", hipGetErrorString(e));
            std::swap(cur, prev);
        }
        const double *lastp = F.first;  // p == 1: the first step is the last
        if (p > 1) {
            sum_partials_kernel<<<1, NT, 0, s>>>(grid, F.part + (int64_t)kMaxGrid * 3, 1, 0, F.first + 3);
            ASC_LAUNCHED();
            lastp = F.first + 3;
        }
        growth_check_kernel<<<1, 64, 0, s>>>(F.first, lastp, flags);
        ASC_LAUNCHED();
    }
    return ASC_OK;
}

asc_status run_moments(const asc_graph *g, const double *lmax, int p, const void *R, asc_dtype sig, int64_t r,
                       int64_t ldr, double *mu, void *ws, hipStream_t s) {
    const int64_t n = g->n;
    const Plan P = make_plan(g, r, sig);
    const int steps = std::max(1, (p + 1) / 2);
    FilterWs F;
    filter_ws_layout(n, rs_for_ws(r, sig), (int)((r + 2 * vn_of(sig) - 1) / (2 * vn_of(sig))), sig, steps, steps,
                     ws, &F);
    uint32_t *flags = &F.hdr->flags;
    diag_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, g->strength, lmax, F.diag, F.beta, flags, 1);
    ASC_LAUNCHED();
    const int grid = grid_for(n, P.lpr);
    const int64_t pstride = (int64_t)(panel_bytes(n, P.rs, sig) / esize(sig));
    int groups = 0;
    for (int sl = 0; sl < P.nslices; sl += P.np, ++groups) {
        pack_panels(P, n, R, sig, ldr, r, sl, F.panelA, pstride, s);
        ASC_LAUNCHED();
        StepArgs A{};
        A.pstride = pstride;
        A.n = n;
        A.rp = g->row_ptr;
        A.ci = g->col_idx;
        A.w = g->w;
        A.diag = F.diag;
        A.beta = F.beta;
        A.coeffs = nullptr;
        void *cur = F.panelA, *prev = F.panelB;
        for (int st = 0; st < steps; ++st) {
            A.cur = cur;
            A.prev = st == 0 ? nullptr : prev;
            A.out = prev;
            A.j = st;
            A.partials = F.part + (int64_t)st * kMaxGrid * 3;
            hipError_t e = launch_plan(P, sig, (st == 0 ? M_FIRST : 0u) | M_PART, A, grid, s);
            if (e != hipSuccess) return fail(ASC_ERR_HIP, "cheb_step launch failed: %s", hipGetErrorString(e));
            std::swap(cur, prev);
        }
        sum_partials_kernel<<<steps, NT, 0, s>>>(grid, F.part, steps, (int64_t)kMaxGrid * 3,
                                                 F.sums + (int64_t)groups * steps * 3);
        ASC_LAUNCHED();
    }
    moments_finalize_kernel<<<1, 64, 0, s>>>(F.sums, groups, steps, p, mu, flags);
    ASC_LAUNCHED();
    return ASC_OK;
}

size_t moments_ws(int64_t n, int64_t r, asc_dtype sig, int p) {
    const int steps = std::max(1, (p + 1) / 2);
    const int nsl_max = (int)((r + 2 * vn_of(sig) - 1) / (2 * vn_of(sig)));
    return filter_ws_layout(n, rs_for_ws(r, sig), nsl_max, sig, steps, steps, nullptr, nullptr);
}

size_t filter_ws(int64_t n, int64_t r, asc_dtype sig) {
    return filter_ws_layout(n, rs_for_ws(r, sig), 1, sig, 2, 1, nullptr, nullptr);
}

// ---------------------------------------------------------------------------
// coefficients and the dichotomy (float64 on the device)
// ---------------------------------------------------------------------------
namespace {

__global__ void coeffs_kernel(const double *__restrict__ lc, int n_cut, const double *__restrict__ lmax, int p,
                              int jackson, double *__restrict__ out) {
    const int64_t total = (int64_t)n_cut * (p + 1);
    const double L = lmax[0];
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int cut = (int)(q / (p + 1));
        const int j = (int)(q - (int64_t)cut * (p + 1));
        out[q] = cheb_coeff_dev(lc[cut], L, p, j, jackson);
    }
}

// count(lc) = sum_j a_j(lc) mu_j, summed by the block in a fixed order
__device__ double count_block(const double *mu, int p, double lc, double L, int jackson, double *lds) {
    double v[1] = {0.0};
    for (int j = threadIdx.x; j <= p; j += NT) v[0] += cheb_coeff_dev(lc, L, p, j, jackson) * mu[j];
    block_sum<1, NT>(v, lds);
    __shared__ double bc;
    if (threadIdx.x == 0) bc = v[0];
    __syncthreads();
    const double r = bc;
    __syncthreads();
    return r;
}

__global__ void dichotomy_kernel(const double *__restrict__ mu, int p, const double *__restrict__ lmax, int k,
                                 int steps, int jackson, double *__restrict__ lambda_k, double *__restrict__ traj) {
    __shared__ double lds[NT / 64];
    const double L = lmax[0];
    double lo = 0.0, hi = L;
    for (int s = 0; s < steps; ++s) {
        const double mid = 0.5 * (lo + hi);
        const double c = count_block(mu, p, mid, L, jackson, lds);
        if (threadIdx.x == 0 && traj) {
            traj[2 * s] = mid;
            traj[2 * s + 1] = c;
        }
        if (c >= k - 0.5) hi = mid; else lo = mid;
    }
    if (threadIdx.x == 0) lambda_k[0] = hi;
}

// literal mode state: [lo, hi]
__global__ void dich_lit_prepare(double *__restrict__ state, int s, const double *__restrict__ lmax, int p,
                                 int jackson, double *__restrict__ coeffs, double *__restrict__ mid_out) {
    (void)s;
    const double L = lmax[0];
    const double mid = 0.5 * (state[0] + state[1]);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j <= p; j += gridDim.x * blockDim.x)
        coeffs[j] = cheb_coeff_dev(mid, L, p, j, jackson);
    if (blockIdx.x == 0 && threadIdx.x == 0) mid_out[0] = mid;
}

__global__ void dich_lit_init(double *state, const double *lmax) {
    if (threadIdx.x == 0) {
        state[0] = 0.0;
        state[1] = lmax[0];
    }
}

// partial <R, Y> per block (float64)
template <typename TS>
__global__ void dot_RY_kernel(int64_t n, int64_t r, const TS *__restrict__ R, int64_t ldr, const float *__restrict__ Y,
                              int64_t ldy, double *__restrict__ part) {
    __shared__ double lds[NT / 64];
    double v[1] = {0.0};
    const int64_t total = n * r;
    for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < total; q += (int64_t)gridDim.x * NT) {
        const int64_t i = q / r, c = q - i * r;
        float x;
        if constexpr (sizeof(TS) == 4) x = (float)R[i * ldr + c];
        else x = __uint_as_float(((uint32_t)R[i * ldr + c]) << 16);
        v[0] += (double)x * (double)Y[i * ldy + c];
    }
    block_sum<1, NT>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ void dich_lit_update(double *__restrict__ state, int s, int k, int nparts, const double *__restrict__ part,
                                const double *__restrict__ mid_in, double *__restrict__ traj,
                                double *__restrict__ lambda_k, int last) {
    if (threadIdx.x != 0) return;
    double c = 0.0;
    for (int b = 0; b < nparts; ++b) c += part[b];
    const double mid = mid_in[0];
    if (traj) {
        traj[2 * s] = mid;
        traj[2 * s + 1] = c;
    }
    if (c >= k - 0.5) state[1] = mid; else state[0] = mid;
    if (last) lambda_k[0] = state[1];
}

__global__ void set_value_kernel(double *dst, const double *src) {
    if (threadIdx.x == 0) dst[0] = src[1];
}

}  // namespace
}  // namespace asc

using namespace asc;

extern "C" size_t asc_filter_workspace(int64_t n, int64_t r, asc_dtype sig, int p) {
    (void)p;
    return filter_ws(n, r, sig);
}

extern "C" size_t asc_ckpt_bytes(const asc_graph *g, int64_t r, asc_dtype sig, int p, int ckpt_stride) {
    if (!g || g->n < 1 || r < 1 || p < 0 || ckpt_stride < 1 || (sig != ASC_F32 && sig != ASC_BF16)) return 0;
    if (ckpt_stride == 1) {
        const Plan P = store_plan(g, r, sig);
        return (size_t)P.nslices * (p + 1) * panel_bytes(g->n, P.rs, sig);
    }
    return (size_t)nseg_of(p, ckpt_stride) * 2 * ck_block_bytes(g->n, r, sig);
}

extern "C" asc_status asc_cheb_coeffs(const double *lambda_c, int n_cut, const double *lmax, int p, int jackson,
                                      double *coeffs, void *stream) {
    const char *who = "asc_cheb_coeffs";
    if (!lambda_c || !lmax || !coeffs) return fail(ASC_ERR_INVALID, "%s: NULL pointer", who);
    if (!aligned(lambda_c, 8) || !aligned(lmax, 8) || !aligned(coeffs, 8)) return fail(ASC_ERR_INVALID, "%s: misaligned", who);
    if (n_cut < 1 || p < 0 || p > 100000) return fail(ASC_ERR_INVALID, "%s: n_cut=%d p=%d", who, n_cut, p);
    const int64_t total = (int64_t)n_cut * (p + 1);
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
    coeffs_kernel<<<grid, 256, 0, as_stream(stream)>>>(lambda_c, n_cut, lmax, p, jackson, coeffs);
    ASC_LAUNCHED();
    return ASC_OK;
}

extern "C" asc_status asc_cheb_filter(const asc_graph *g, const double *lmax, const double *coeffs, int p,
                                      const void *R, asc_dtype sig, int64_t r, int64_t ldr, float *Y, int64_t ldy,
                                      void *ckpt, int ckpt_stride, void *ws, size_t ws_bytes, void *stream) {
    const char *who = "asc_cheb_filter";
    ASC_TRY(check_common(g, lmax, p, R, sig, r, ldr, who));
    if (!coeffs || !aligned(coeffs, 8)) return fail(ASC_ERR_INVALID, "%s: coeffs NULL or misaligned", who);
    ASC_TRY(check_block(Y, ASC_F32, g->n, r, ldy, who, "Y"));
    {
        const char *rb = static_cast<const char *>(R);
        const char *re = rb + (size_t)((g->n - 1) * ldr + r) * esize(sig);
        const char *yb = reinterpret_cast<const char *>(Y);
        const char *ye = yb + (size_t)((g->n - 1) * ldy + r) * 4;
        if (rb < ye && yb < re) return fail(ASC_ERR_INVALID, "%s: Y overlaps R", who);
    }
    if (ckpt && (ckpt_stride < 1 || !aligned(ckpt, 256)))
        return fail(ASC_ERR_INVALID, "%s: ckpt needs ckpt_stride >= 1 and 256-byte alignment", who);
    ASC_TRY(check_ws(ws, ws_bytes, asc_filter_workspace(g->n, r, sig, p), who));
    return run_filter(g, lmax, coeffs, p, R, sig, r, ldr, Y, ldy, ckpt, ckpt_stride, ws, true, as_stream(stream));
}

// ---------------------------------------------------------------------------
// the filter with its workspace in a static device array (no allocation)
// ---------------------------------------------------------------------------
// One copy per device, held until the process ends.  Host code never passes
// the array's own name to a kernel: that is a host-side shadow, not a device
// address; the address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[ASC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
void *scratch_ptr[kMaxDevices] = {};

asc_status scratch_for_current_device(void **out, const char *who) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(ASC_ERR_HIP, "%s: hipGetDevice: %s", who, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(ASC_ERR_INVALID, "%s: device %d beyond %d", who, dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ASC_ERR_HIP, "%s: hipGetSymbolAddress(scratch) on device %d: %s", who, dev,
                        hipGetErrorString(e));
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return ASC_OK;
}
}  // namespace

extern "C" asc_status asc_cheb_filter_noalloc(const asc_graph *g, const double *lmax, const double *coeffs, int p,
                                              const void *R, asc_dtype sig, int64_t r, int64_t ldr, float *Y,
                                              int64_t ldy, void *ckpt, int ckpt_stride, void *stream) {
    const char *who = "asc_cheb_filter_noalloc";
    ASC_TRY(check_common(g, lmax, p, R, sig, r, ldr, who));
    const size_t need = asc_filter_workspace(g->n, r, sig, p);
    if (need > (size_t)ASC_NOALLOC_SCRATCH_BYTES)
        return fail(ASC_ERR_WORKSPACE, "%s: n=%lld, r=%lld needs %zu bytes of scratch; the static array holds %zu",
                    who, (long long)g->n, (long long)r, need, (size_t)ASC_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    ASC_TRY(scratch_for_current_device(&ws, who));
    // same checks and kernels as asc_cheb_filter; the scratch is its workspace
    return asc_cheb_filter(g, lmax, coeffs, p, R, sig, r, ldr, Y, ldy, ckpt, ckpt_stride, ws,
                           (size_t)ASC_NOALLOC_SCRATCH_BYTES, stream);
}

extern "C" size_t asc_moments_workspace(int64_t n, int64_t r, asc_dtype sig, int p) { return moments_ws(n, r, sig, p); }

extern "C" asc_status asc_cheb_moments(const asc_graph *g, const double *lmax, int p, const void *R, asc_dtype sig,
                                       int64_t r, int64_t ldr, double *mu, void *ws, size_t ws_bytes, void *stream) {
    const char *who = "asc_cheb_moments";
    ASC_TRY(check_common(g, lmax, p, R, sig, r, ldr, who));
    if (!mu || !aligned(mu, 8)) return fail(ASC_ERR_INVALID, "%s: mu NULL or misaligned", who);
    ASC_TRY(check_ws(ws, ws_bytes, moments_ws(g->n, r, sig, p), who));
    return run_moments(g, lmax, p, R, sig, r, ldr, mu, ws, as_stream(stream));
}

extern "C" asc_status asc_eigcount_dichotomy(const double *mu, int p, const double *lmax, int k, int steps,
                                             int jackson, double *lambda_k, double *traj, void *stream) {
    const char *who = "asc_eigcount_dichotomy";
    if (!mu || !lmax || !lambda_k) return fail(ASC_ERR_INVALID, "%s: NULL pointer", who);
    if (!aligned(mu, 8) || !aligned(lmax, 8) || !aligned(lambda_k, 8) || (traj && !aligned(traj, 8)))
        return fail(ASC_ERR_INVALID, "%s: misaligned", who);
    if (p < 0 || p > 100000 || k < 0 || steps < 0 || steps > 200)
        return fail(ASC_ERR_INVALID, "%s: p=%d k=%d steps=%d", who, p, k, steps);
    dichotomy_kernel<<<1, NT, 0, as_stream(stream)>>>(mu, p, lmax, k, steps, jackson, lambda_k, traj);
    ASC_LAUNCHED();
    return ASC_OK;
}

extern "C" size_t asc_eigcount_workspace(int64_t n, int64_t r, asc_dtype sig, int p, int steps, int literal) {
    (void)steps;
    Arena a(nullptr);
    if (literal) {
        a.take<char>(filter_ws(n, r, sig));
        a.take<double>(p + 1);         // coeffs
        a.take<double>(64);            // state, mid
        a.take<double>(kMaxGrid);      // dot partials
        a.take<float>((size_t)n * ((r + 3) & ~int64_t(3)));  // Y
    } else {
        a.take<char>(moments_ws(n, r, sig, p));
        a.take<double>(p + 1);  // mu
    }
    return a.size();
}

extern "C" asc_status asc_eigcount_lambda_k(const asc_graph *g, const double *lmax, int k, int p, int steps,
                                            int literal, const void *R, asc_dtype sig, int64_t r, int64_t ldr,
                                            double *lambda_k, double *traj, void *ws, size_t ws_bytes, void *stream) {
    const char *who = "asc_eigcount_lambda_k";
    ASC_TRY(check_common(g, lmax, p, R, sig, r, ldr, who));
    if (!lambda_k || !aligned(lambda_k, 8) || (traj && !aligned(traj, 8)))
        return fail(ASC_ERR_INVALID, "%s: lambda_k NULL or misaligned", who);
    if (k < 0 || steps < 0 || steps > 200) return fail(ASC_ERR_INVALID, "%s: k=%d steps=%d", who, k, steps);
    ASC_TRY(check_ws(ws, ws_bytes, asc_eigcount_workspace(g->n, r, sig, p, steps, literal), who));
    hipStream_t s = as_stream(stream);
    Arena a(ws);
    if (!literal) {
        void *mws = a.take<char>(moments_ws(g->n, r, sig, p));
        double *mu = a.take<double>(p + 1);
        ASC_TRY(run_moments(g, lmax, p, R, sig, r, ldr, mu, mws, s));
        dichotomy_kernel<<<1, NT, 0, s>>>(mu, p, lmax, k, steps, 1, lambda_k, traj);
        ASC_LAUNCHED();
        return ASC_OK;
    }
    void *fws = a.take<char>(filter_ws(g->n, r, sig));
    double *coeffs = a.take<double>(p + 1);
    double *state = a.take<double>(64);
    double *part = a.take<double>(kMaxGrid);
    const int64_t ldy = (r + 3) & ~int64_t(3);
    float *Y = a.take<float>((size_t)g->n * ldy);
    dich_lit_init<<<1, 64, 0, s>>>(state, lmax);
    ASC_LAUNCHED();
    if (steps == 0) {
        set_value_kernel<<<1, 64, 0, s>>>(lambda_k, state);
        ASC_LAUNCHED();
        return ASC_OK;
    }
    const int64_t tot = g->n * r;
    const int dg = (int)std::min<int64_t>((tot + NT - 1) / NT, kMaxGrid);
    for (int st = 0; st < steps; ++st) {
        dich_lit_prepare<<<(p + 256) / 256, 256, 0, s>>>(state, st, lmax, p, 1, coeffs, state + 2);
        ASC_LAUNCHED();
        ASC_TRY(run_filter(g, lmax, coeffs, p, R, sig, r, ldr, Y, ldy, nullptr, 0, fws, st == 0, s));
        if (sig == ASC_F32)
            dot_RY_kernel<float><<<dg, NT, 0, s>>>(g->n, r, (const float *)R, ldr, Y, ldy, part);
        else
            dot_RY_kernel<uint16_t><<<dg, NT, 0, s>>>(g->n, r, (const uint16_t *)R, ldr, Y, ldy, part);
        ASC_LAUNCHED();
        dich_lit_update<<<1, 64, 0, s>>>(state, st, k, dg, part, state + 2, traj, lambda_k, st == steps - 1);
        ASC_LAUNCHED();
    }
    return ASC_OK;
}

// ---------------------------------------------------------------------------
// autotuner: times one recurrence step (all column slices) of every candidate
// (slice width x kernel variant) on the caller's graph and signals, keeps the
// fastest in the process-wide table.  Synchronises the stream.
// ---------------------------------------------------------------------------
namespace asc {
namespace {
__global__ void zero_f64(double *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0;
}
}  // namespace

asc_status autotune_filter(const asc_graph *g, const double *lmax, const void *R, asc_dtype sig, int64_t r,
                           int64_t ldr, float *Y, int64_t ldy, int probe_steps, void *ws, hipStream_t s,
                           TuneEntry *best) {
    const int64_t n = g->n;
    FilterWs F;
    filter_ws_layout(n, rs_for_ws(r, sig), 1, sig, 2, 1, ws, &F);
    diag_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, g->strength, lmax, F.diag, F.beta, &F.hdr->flags, 1);
    ASC_LAUNCHED();
    zero_f64<<<1, 64, 0, s>>>(F.first, 64);  // coefficients read by the probe steps
    ASC_LAUNCHED();
    const int vn = vn_of(sig);
    int64_t rcap = 2 * vn;
    while (rcap < r) rcap *= 2;
    hipEvent_t e0, e1;
    ASC_HIP(hipEventCreate(&e0));
    ASC_HIP(hipEventCreate(&e1));
    TuneEntry bestE{};
    bestE.ms = 1e30f;
    asc_status st = ASC_OK;
    for (int rs = 2 * vn; rs <= 16 * vn && rs <= rcap; rs *= 2) {
        for (unsigned var = 0; var < 16; ++var) {
            const Plan P = plan_for(rs, var, r, sig);
            // bit 3 only where one launch can cover every slice, and then
            // only with the tile-schedule bit
            if ((var & 8u) != 0 && (P.np == 1 || (var & 3u) != 0)) continue;
            const int grid = grid_for(n, P.lpr);
            const int64_t pstride = (int64_t)(panel_bytes(n, P.rs, sig) / esize(sig));
            for (void *panel : {F.panelA, F.panelB}) pack_panels(P, n, R, sig, ldr, r, 0, panel, pstride, s);
            ASC_LAUNCHED();
            StepArgs A{};
            A.pstride = pstride;
            A.n = n;
            A.rp = g->row_ptr;
            A.ci = g->col_idx;
            A.w = g->w;
            A.diag = F.diag;
            A.beta = F.beta;
            A.Y = Y;
            A.ldy = ldy;
            A.r = r;
            A.coeffs = F.first;
            A.j = 0;
            void *cur = F.panelA, *prev = F.panelB;
            float ms = 0.f;
            // steps in pairs, as the filter runs them (float32: one that adds a
            // pair of terms to Y, one that leaves Y alone; bfloat16: Y on both)
            for (int it = -1; it < probe_steps && st == ASC_OK; ++it) {
                if (it == 0) (void)hipEventRecord(e0, s);
                for (int half = 0; half < 2 && st == ASC_OK; ++half) {
                    for (int sl = 0; sl < P.nslices; sl += P.np) {
                        A.c0 = (int64_t)sl * P.rs;
                        A.cur = cur;
                        A.prev = prev;
                        A.out = prev;
                        const unsigned ym = sig == ASC_F32 ? (half == 0 ? (M_YACC | M_YPAIR) : 0u) : M_YACC;
                        hipError_t e = launch_plan(P, sig, ym, A, grid, s);
                        if (e != hipSuccess) {
                            st = fail(ASC_ERR_HIP, "autotune launch failed: %s", hipGetErrorString(e));
                            break;
                        }
                    }
                    std::swap(cur, prev);
                }
            }
            if (st != ASC_OK) break;
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms /= (float)(2 * std::max(1, probe_steps));
            if (ms < bestE.ms) {
                bestE.ms = ms;
                bestE.rs = rs;
                bestE.var = (int)var;
            }
        }
        if (st != ASC_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != ASC_OK) return st;
    bestE.key = TuneKey{n, g->nnz, r, (int)sig};
    {
        std::lock_guard<std::mutex> lk(tune_mutex());
        auto &t = tune_table();
        bool found = false;
        for (auto &e : t)
            if (e.key == bestE.key) {
                e = bestE;
                found = true;
            }
        if (!found) t.push_back(bestE);
    }
    if (best) *best = bestE;
    return ASC_OK;
}
}  // namespace asc

extern "C" asc_status asc_tune_set(int64_t n, int64_t nnz, int64_t r, asc_dtype sig, int slice_cols, int variant) {
    if (sig != ASC_F32 && sig != ASC_BF16) return fail(ASC_ERR_INVALID, "asc_tune_set: dtype");
    if (slice_cols != 0 && !valid_rs(slice_cols, sig))
        return fail(ASC_ERR_INVALID, "asc_tune_set: slice_cols=%d not supported for this dtype", slice_cols);
    if (variant < 0 || variant > 15) return fail(ASC_ERR_INVALID, "asc_tune_set: variant=%d", variant);
    std::lock_guard<std::mutex> lk(tune_mutex());
    auto &t = tune_table();
    const TuneKey key{n, nnz, r, (int)sig};
    for (size_t q = 0; q < t.size(); ++q)
        if (t[q].key == key) {
            if (slice_cols == 0) t.erase(t.begin() + q);
            else t[q] = TuneEntry{key, slice_cols, variant, 0.f};
            return ASC_OK;
        }
    if (slice_cols != 0) t.push_back(TuneEntry{key, slice_cols, variant, 0.f});
    return ASC_OK;
}

extern "C" asc_status asc_tune_get(int64_t n, int64_t nnz, int64_t r, asc_dtype sig, int *slice_cols, int *variant) {
    if (!slice_cols || !variant) return fail(ASC_ERR_INVALID, "asc_tune_get: NULL output");
    TuneEntry e;
    if (tuned(n, nnz, r, sig, &e)) {
        *slice_cols = e.rs;
        *variant = e.var;
    } else {
        *slice_cols = default_rs(r, sig);
        *variant = 0;
    }
    return ASC_OK;
}

extern "C" asc_status asc_tune_save(const char *path) {
    if (!path) return fail(ASC_ERR_INVALID, "asc_tune_save: NULL path");
    FILE *f = fopen(path, "w");
    if (!f) return fail(ASC_ERR_INVALID, "asc_tune_save: cannot open %s", path);
    std::lock_guard<std::mutex> lk(tune_mutex());
    fprintf(f, "[\n");
    const auto &t = tune_table();
    for (size_t q = 0; q < t.size(); ++q) {
        const auto &e = t[q];
        fprintf(f, "{\"n\": %lld, \"nnz\": %lld, \"r\": %lld, \"dtype\": %d, \"slice_cols\": %d, \"variant\": %d, \"ms\": %.6f}%s\n",
                (long long)e.key.n, (long long)e.key.nnz, (long long)e.key.r, e.key.dt, e.rs, e.var, (double)e.ms,
                q + 1 < t.size() ? "," : "");
    }
    fprintf(f, "]\n");
    fclose(f);
    return ASC_OK;
}

extern "C" asc_status asc_tune_load(const char *path) {
    if (!path) return fail(ASC_ERR_INVALID, "asc_tune_load: NULL path");
    FILE *f = fopen(path, "r");
    if (!f) return fail(ASC_ERR_INVALID, "asc_tune_load: cannot open %s", path);
    char line[512];
    while (fgets(line, sizeof line, f)) {
        long long n, nnz, r;
        int dt, rs, var;
        double ms;
        if (sscanf(line, " {\"n\": %lld, \"nnz\": %lld, \"r\": %lld, \"dtype\": %d, \"slice_cols\": %d, \"variant\": %d, \"ms\": %lf",
                   &n, &nnz, &r, &dt, &rs, &var, &ms) == 7) {
            if ((dt == 0 || dt == 1) && valid_rs(rs, (asc_dtype)dt) && var >= 0 && var <= 15) {
                asc_tune_set(n, nnz, r, (asc_dtype)dt, rs, var);
            }
        }
    }
    fclose(f);
    return ASC_OK;
}

extern "C" asc_status asc_autotune_filter(const asc_graph *g, const double *lmax, const void *R, asc_dtype sig,
                                          int64_t r, int64_t ldr, float *Y, int64_t ldy, int probe_steps, void *ws,
                                          size_t ws_bytes, int *best_slice_cols, int *best_variant,
                                          float *best_ms_per_step, void *stream) {
    const char *who = "asc_autotune_filter";
    ASC_TRY(check_common(g, lmax, 1, R, sig, r, ldr, who));
    ASC_TRY(check_block(Y, ASC_F32, g->n, r, ldy, who, "Y"));
    if (probe_steps < 1 || probe_steps > 1000) return fail(ASC_ERR_INVALID, "%s: probe_steps=%d", who, probe_steps);
    ASC_TRY(check_ws(ws, ws_bytes, asc_filter_workspace(g->n, r, sig, 1), who));
    TuneEntry e;
    ASC_TRY(autotune_filter(g, lmax, R, sig, r, ldr, Y, ldy, probe_steps, ws, as_stream(stream), &e));
    if (best_slice_cols) *best_slice_cols = e.rs;
    if (best_variant) *best_variant = e.var;
    if (best_ms_per_step) *best_ms_per_step = e.ms;
    return ASC_OK;
}

// ---------------------------------------------------------------------------
// the state store for other translation units
// ---------------------------------------------------------------------------
namespace asc {

StoreLayout store_layout(const asc_graph *g, int64_t r, asc_dtype sig) {
    const Plan P = store_plan(g, r, sig);
    return StoreLayout{P.rs, P.nslices, panel_bytes(g->n, P.rs, sig)};
}

size_t store_ws_bytes(int64_t n, int64_t r, asc_dtype sig) {
    return filter_ws_layout(n, rs_for_ws(r, sig), 1, sig, 1, 1, nullptr, nullptr);
}

asc_status run_store(const asc_graph *g, const double *lmax, int p, const void *R, asc_dtype sig, int64_t r,
                     int64_t ldr, void *states, void *ws, hipStream_t s) {
    const int64_t n = g->n;
    const Plan P = store_plan(g, r, sig);
    FilterWs F;
    filter_ws_layout(n, rs_for_ws(r, sig), 1, sig, 1, 1, ws, &F);
    diag_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, g->strength, lmax, F.diag, F.beta, &F.hdr->flags, 1);
    ASC_LAUNCHED();
    const int grid = grid_for(n, P.lpr);
    const size_t pbytes = panel_bytes(n, P.rs, sig);
    auto slot = [&](int sl, int j) -> void * { return static_cast<char *>(states) + ((size_t)sl * (p + 1) + j) * pbytes; };
    const int64_t pstride = (int64_t)((size_t)(p + 1) * pbytes / esize(sig));
    // Small graphs: every slice in one launch per step (blockIdx.y = slice),
    // instead of one launch per slice and step, while all the slices' panels
    // stay a cache-resident set (the launches, not the memory, bound these).
    if (P.np == 1 && P.nslices > 1 && P.nslices <= 65535 && (size_t)P.nslices * pbytes <= (size_t(64) << 20)) {
        Plan Py = P;
        Py.var &= ~4u;  // the XCD-band tile order assumes a one-dimensional grid
        for (int sl = 0; sl < P.nslices; ++sl) {
            pack_panels(Py, n, R, sig, ldr, r, sl, slot(sl, 0), pstride, s);
            ASC_LAUNCHED();
        }
        StepArgs A{};
        A.pstride = pstride;
        A.ystride = (int64_t)((size_t)(p + 1) * pbytes);
        A.n = n;
        A.rp = g->row_ptr;
        A.ci = g->col_idx;
        A.w = g->w;
        A.diag = F.diag;
        A.beta = F.beta;
        const dim3 gy((unsigned)grid, (unsigned)P.nslices);
        for (int j = 0; j < p; ++j) {
            A.cur = slot(0, j);
            A.prev = j == 0 ? nullptr : slot(0, j - 1);
            A.out = slot(0, j + 1);
            A.j = j;
            hipError_t e = launch_step(sig, Py.lpr, Py.var, j == 0 ? M_FIRST : 0u, A, gy, s);
            if (e != hipSuccess) return fail(ASC_ERR_HIP, "cheb_step launch failed: %s", hipGetErrorString(e));
        }
        return ASC_OK;
    }
    for (int sl = 0; sl < P.nslices; sl += P.np) {
        pack_panels(P, n, R, sig, ldr, r, sl, slot(sl, 0), pstride, s);
        ASC_LAUNCHED();
        StepArgs A{};
        A.pstride = pstride;
        A.n = n;
        A.rp = g->row_ptr;
        A.ci = g->col_idx;
        A.w = g->w;
        A.diag = F.diag;
        A.beta = F.beta;
        for (int j = 0; j < p; ++j) {
            A.cur = slot(sl, j);
            A.prev = j == 0 ? nullptr : slot(sl, j - 1);
            A.out = slot(sl, j + 1);
            A.j = j;
            hipError_t e = launch_plan(P, sig, j == 0 ? M_FIRST : 0u, A, grid, s);
            if (e != hipSuccess) return fail(ASC_ERR_HIP, "cheb_step launch failed: %s", hipGetErrorString(e));
        }
    }
    return ASC_OK;
}

}  // namespace asc

// ---------------------------------------------------------------------------
// one-pass lambda_k + filter: states are kept, Y is formed at the end
// ---------------------------------------------------------------------------
namespace asc {
namespace {

// Y[i, c0 + c] = sum_j a_j T_j[i, c] over the stored panels of one slice;
// one thread per 16-byte chunk, coefficients summed in order j = 0..p
template <typename TS>
__global__ void combine_kernel(int64_t n, int rs, const TS *__restrict__ slots, int64_t slot_elems, int p,
                               const double *__restrict__ coeffs, float *__restrict__ Y, int64_t ldy, int64_t c0,
                               int64_t r) {
    constexpr int VN = St<TS>::VN;
    const int64_t chunks = n * (rs / VN);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < chunks; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q / (rs / VN);
        const int cc = (int)(q - i * (rs / VN)) * VN;
        float acc[VN];
#pragma unroll
        for (int e = 0; e < VN; ++e) acc[e] = 0.0f;
        const TS *src = slots + i * rs + cc;
        for (int j = 0; j <= p; ++j) fma_raw(acc, (float)coeffs[j], ldraw<true>(src + (int64_t)j * slot_elems));
        float *y = Y + i * ldy + c0 + cc;
        if (c0 + cc + VN <= r) {
#pragma unroll
            for (int e = 0; e < VN; e += 4) {
                v4f v = {acc[e], acc[e + 1], acc[e + 2], acc[e + 3]};
                *reinterpret_cast<v4f *>(y + e) = v;
            }
        } else {
#pragma unroll
            for (int e = 0; e < VN; ++e)
                if (c0 + cc + e < r) y[e] = acc[e];
        }
    }
}

size_t lkf_ws_layout(int64_t n, int64_t r, asc_dtype sig, int p, void *ws, void **mws, double **mu, double **co) {
    Arena a(ws);
    void *m = a.take<char>(moments_ws(n, r, sig, p));
    double *u = a.take<double>(p + 1);
    double *c = a.take<double>(p + 1);
    if (mws) *mws = m;
    if (mu) *mu = u;
    if (co) *co = c;
    return a.size();
}

}  // namespace
}  // namespace asc

extern "C" size_t asc_lambda_k_filter_workspace(int64_t n, int64_t r, asc_dtype sig, int p) {
    return lkf_ws_layout(n, r, sig, p, nullptr, nullptr, nullptr, nullptr);
}

extern "C" asc_status asc_lambda_k_filter(const asc_graph *g, const double *lmax, int k, int p, int steps,
                                          const void *R, asc_dtype sig, int64_t r, int64_t ldr, float *Y, int64_t ldy,
                                          double *lambda_k, double *traj, double *coeffs_out, void *states, void *ws,
                                          size_t ws_bytes, void *stream) {
    const char *who = "asc_lambda_k_filter";
    ASC_TRY(check_common(g, lmax, p, R, sig, r, ldr, who));
    if (p < 1) return fail(ASC_ERR_INVALID, "%s: p must be >= 1", who);
    ASC_TRY(check_block(Y, ASC_F32, g->n, r, ldy, who, "Y"));
    if (!lambda_k || !aligned(lambda_k, 8) || (traj && !aligned(traj, 8)) || (coeffs_out && !aligned(coeffs_out, 8)))
        return fail(ASC_ERR_INVALID, "%s: lambda_k NULL or outputs misaligned", who);
    if (k < 0 || steps < 0 || steps > 200) return fail(ASC_ERR_INVALID, "%s: k=%d steps=%d", who, k, steps);
    if (!states || !aligned(states, 256)) return fail(ASC_ERR_INVALID, "%s: states NULL or not 256-byte aligned", who);
    ASC_TRY(check_ws(ws, ws_bytes, asc_lambda_k_filter_workspace(g->n, r, sig, p), who));
    hipStream_t s = as_stream(stream);
    const int64_t n = g->n;
    void *mws;
    double *mu, *co;
    lkf_ws_layout(n, r, sig, p, ws, &mws, &mu, &co);
    if (coeffs_out) co = coeffs_out;
    const Plan P = store_plan(g, r, sig);
    const int msteps = std::max(1, (p + 1) / 2);
    FilterWs F;
    filter_ws_layout(n, rs_for_ws(r, sig), (int)((r + 2 * vn_of(sig) - 1) / (2 * vn_of(sig))), sig, msteps, msteps,
                     mws, &F);
    uint32_t *flags = &F.hdr->flags;
    diag_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, g->strength, lmax, F.diag, F.beta, flags, 1);
    ASC_LAUNCHED();
    const int grid = grid_for(n, P.lpr);
    const size_t pbytes = panel_bytes(n, P.rs, sig);
    auto slot = [&](int sl, int j) -> void * { return static_cast<char *>(states) + ((size_t)sl * (p + 1) + j) * pbytes; };
    const int64_t pstride = (int64_t)((size_t)(p + 1) * pbytes / esize(sig));
    int groups = 0;
    for (int sl = 0; sl < P.nslices; sl += P.np, ++groups) {
        pack_panels(P, n, R, sig, ldr, r, sl, slot(sl, 0), pstride, s);
        ASC_LAUNCHED();
        StepArgs A{};
        A.pstride = pstride;
        A.n = n;
        A.rp = g->row_ptr;
        A.ci = g->col_idx;
        A.w = g->w;
        A.diag = F.diag;
        A.beta = F.beta;
        for (int j = 0; j < p; ++j) {
            A.cur = slot(sl, j);
            A.prev = j == 0 ? nullptr : slot(sl, j - 1);
            A.out = slot(sl, j + 1);
            A.j = j;
            const bool part = j < msteps;
            A.partials = part ? F.part + (int64_t)j * kMaxGrid * 3 : nullptr;
            hipError_t e = launch_plan(P, sig, (j == 0 ? M_FIRST : 0u) | (part ? M_PART : 0u), A, grid, s);
            if (e != hipSuccess) return fail(ASC_ERR_HIP, "cheb_step launch failed: %s", hipGetErrorString(e));
        }
        sum_partials_kernel<<<msteps, NT, 0, s>>>(grid, F.part, msteps, (int64_t)kMaxGrid * 3,
                                                  F.sums + (int64_t)groups * msteps * 3);
        ASC_LAUNCHED();
    }
    moments_finalize_kernel<<<1, 64, 0, s>>>(F.sums, groups, msteps, p, mu, flags);
    ASC_LAUNCHED();
    dichotomy_kernel<<<1, NT, 0, s>>>(mu, p, lmax, k, steps, 1, lambda_k, traj);
    ASC_LAUNCHED();
    coeffs_kernel<<<(p + 256) / 256, 256, 0, s>>>(lambda_k, 1, lmax, p, 1, co);
    ASC_LAUNCHED();
    const int64_t chunks = n * (P.rs / vn_of(sig));
    const int cg = (int)std::min<int64_t>((chunks + 255) / 256, 65536);
    for (int sl = 0; sl < P.nslices; ++sl) {
        const int64_t slot_elems = (int64_t)(pbytes / esize(sig));
        if (sig == ASC_F32)
            combine_kernel<float><<<cg, 256, 0, s>>>(n, P.rs, (const float *)slot(sl, 0), slot_elems, p, co, Y, ldy,
                                                     (int64_t)sl * P.rs, r);
        else
            combine_kernel<uint16_t><<<cg, 256, 0, s>>>(n, P.rs, (const uint16_t *)slot(sl, 0), slot_elems, p, co, Y,
                                                        ldy, (int64_t)sl * P.rs, r);
        ASC_LAUNCHED();
    }
    return ASC_OK;
}
