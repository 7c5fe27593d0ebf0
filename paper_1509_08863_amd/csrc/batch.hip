// Batched lambda_k estimation and filtering of many graphs of uneven size
// (steps 2-5 of the algorithm in Sec. 4.1 for every graph of a batch).
//
// The batch is one block-diagonal CSR: graph g owns rows node_off[g] ..
// node_off[g+1]-1 and its columns stay inside that range.  Every graph runs
// the same sequence of recurrence levels (ceil(p/2) moment levels, one
// dichotomy, p filter levels), so the batch advances in lockstep: one launch
// per level covers the rows of all graphs, with per-graph scale beta_g and
// per-graph coefficients.  Work is cut into graph-aligned row tiles, so the
// float64 moment partials of a tile belong to one graph and are summed per
// graph in a fixed order (deterministic).  The dichotomy of all graphs runs
// in one kernel (one block per graph) that also writes each graph's filter
// coefficients, so no value returns to the host.  The whole sequence is
// captured once into a HIP graph and replayed as a single launch.
#include "recurrence.hpp"
#include "coeffs.hpp"

#include <vector>

namespace asc {
namespace {

struct Tile {
    int32_t g, r0, r1, pad;
};

struct BatchArgs {
    StepArgs S;            // n, rp, ci, w, diag, cur, prev, out, Y, ldy, c0, r, ck_*
    const Tile *tiles;
    int ntiles;
    const float *betas;    // [G]
    const double *coeffs;  // [G][p+1]
    int p1;                // p + 1
};

template <typename TS, int LPR, unsigned MODE>
__global__ __launch_bounds__(NT) void batch_step(BatchArgs B) {
    constexpr int RPW = 64 / LPR;
    constexpr int ROWS = RPW * (NT / 64);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int t = lane % LPR;
    const int sub = lane / LPR;
    __shared__ double lds[3 * NT / 64];
    for (int tile = blockIdx.x; tile < B.ntiles; tile += gridDim.x) {
        const Tile T = B.tiles[tile];
        const float beta = B.betas[T.g];
        const double *a = B.coeffs + (int64_t)T.g * B.p1;
        const float aj1 = (MODE & M_YACC) ? (float)a[B.S.j + 1] : 0.0f;
        const float a0 = !(MODE & M_YACC) ? 0.0f
                         : (MODE & M_FIRST) ? (float)a[0]
                         : (MODE & M_YPAIR) ? (float)a[B.S.j] : 0.0f;
        double p_own = 0.0, p_cross = 0.0, p_sq = 0.0;
        for (int64_t r0 = T.r0; r0 < T.r1; r0 += ROWS) {
            const int64_t row = r0 + (int64_t)wave * RPW + sub;
            if (row < T.r1) step_row<TS, LPR, MODE, 0u>(B.S, row, t, beta, aj1, a0, p_own, p_cross, p_sq);
        }
        if (MODE & M_PART) {
            double v[3] = {p_own, p_cross, p_sq};
            block_sum<3, NT>(v, lds);
            if (threadIdx.x == 0) {
                double *pp = B.S.partials + (int64_t)tile * 3;
                pp[0] = v[0];
                pp[1] = v[1];
                pp[2] = v[2];
            }
        }
    }
}

template <typename TS, int LPR>
hipError_t launch_batch_t(unsigned mode, const BatchArgs &B, int grid, hipStream_t s) {
    switch (mode) {
        case M_FIRST | M_PART: batch_step<TS, LPR, M_FIRST | M_PART><<<grid, NT, 0, s>>>(B); break;
        case M_PART: batch_step<TS, LPR, M_PART><<<grid, NT, 0, s>>>(B); break;
        case M_FIRST | M_YACC: batch_step<TS, LPR, M_FIRST | M_YACC><<<grid, NT, 0, s>>>(B); break;
        case M_YACC: batch_step<TS, LPR, M_YACC><<<grid, NT, 0, s>>>(B); break;
        case M_YACC | M_YPAIR: batch_step<TS, LPR, M_YACC | M_YPAIR><<<grid, NT, 0, s>>>(B); break;
        case 0u: batch_step<TS, LPR, 0u><<<grid, NT, 0, s>>>(B); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch(asc_dtype dt, int lpr, unsigned mode, const BatchArgs &B, int grid, hipStream_t s) {
    if (dt == ASC_F32) {
        switch (lpr) {
            case 2: return launch_batch_t<float, 2>(mode, B, grid, s);
            case 4: return launch_batch_t<float, 4>(mode, B, grid, s);
            case 8: return launch_batch_t<float, 8>(mode, B, grid, s);
            case 16: return launch_batch_t<float, 16>(mode, B, grid, s);
        }
    } else {
        switch (lpr) {
            case 2: return launch_batch_t<uint16_t, 2>(mode, B, grid, s);
            case 4: return launch_batch_t<uint16_t, 4>(mode, B, grid, s);
            case 8: return launch_batch_t<uint16_t, 8>(mode, B, grid, s);
            case 16: return launch_batch_t<uint16_t, 16>(mode, B, grid, s);
        }
    }
    return hipErrorInvalidValue;
}

// d_i = 4 s_i / lmax_g - 2 for the rows of each tile; beta_g = -4 / lmax_g
__global__ void batch_diag_kernel(const Tile *__restrict__ tiles, int ntiles, const double *__restrict__ s,
                                  const double *__restrict__ lmax, float *__restrict__ diag, float *__restrict__ betas,
                                  const int64_t *__restrict__ node_off) {
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const Tile T = tiles[tile];
        const double L = lmax[T.g];
        for (int64_t i = T.r0 + threadIdx.x; i < T.r1; i += blockDim.x) diag[i] = (float)(4.0 * s[i] / L - 2.0);
        if (T.r0 == node_off[T.g] && threadIdx.x == 0) betas[T.g] = (float)(-4.0 / L);
    }
}

// one block per graph: moments from the tile partials (doubling identities),
// dichotomy on [0, lmax_g], coefficients of the final filter
__global__ __launch_bounds__(NT) void batch_dichotomy_kernel(
    const double *__restrict__ part, int nslices, int msteps, int ntiles, const int32_t *__restrict__ tile_off,
    const int32_t *__restrict__ kk, const double *__restrict__ lmax, int p, int steps, double *__restrict__ lambda_k,
    double *__restrict__ traj, double *__restrict__ coeffs) {
    extern __shared__ double mu[];  // p + 1
    __shared__ double lds[3 * NT / 64];
    __shared__ double bc;
    const int g = blockIdx.x;
    const int t0 = tile_off[g], t1 = tile_off[g + 1];
    double mu0 = 0.0, mu1 = 0.0;
    for (int st = 0; st < msteps; ++st) {
        double v[3] = {0.0, 0.0, 0.0};
        for (int sl = 0; sl < nslices; ++sl) {
            const double *pp = part + ((int64_t)sl * msteps + st) * (int64_t)ntiles * 3;
            for (int tt = t0 + threadIdx.x; tt < t1; tt += NT) {
                v[0] += pp[(int64_t)tt * 3 + 0];
                v[1] += pp[(int64_t)tt * 3 + 1];
                v[2] += pp[(int64_t)tt * 3 + 2];
            }
        }
        block_sum<3, NT>(v, lds);
        if (threadIdx.x == 0) {
            if (st == 0) {
                mu0 = v[0];
                mu1 = v[1];
                mu[0] = mu0;
                if (p >= 1) mu[1] = mu1;
            }
            const int jo = 2 * st + 1, je = 2 * st + 2;
            if (st > 0 && jo <= p) mu[jo] = 2.0 * v[1] - mu1;
            if (je <= p) mu[je] = 2.0 * v[2] - mu0;
        }
        __syncthreads();
    }
    const double L = lmax[g];
    const int k = kk[g];
    double lo = 0.0, hi = L;
    for (int s = 0; s < steps; ++s) {
        const double mid = 0.5 * (lo + hi);
        double v[1] = {0.0};
        for (int j = threadIdx.x; j <= p; j += NT) v[0] += cheb_coeff_dev(mid, L, p, j, 1) * mu[j];
        block_sum<1, NT>(v, lds);
        if (threadIdx.x == 0) {
            bc = v[0];
            if (traj) {
                traj[((int64_t)g * steps + s) * 2] = mid;
                traj[((int64_t)g * steps + s) * 2 + 1] = v[0];
            }
        }
        __syncthreads();
        if (bc >= k - 0.5) hi = mid; else lo = mid;
        __syncthreads();
    }
    if (threadIdx.x == 0) lambda_k[g] = hi;
    for (int j = threadIdx.x; j <= p; j += NT) coeffs[(int64_t)g * (p + 1) + j] = cheb_coeff_dev(hi, L, p, j, 1);
}

struct BatchPlan {
    asc_graph g;
    int G;
    int64_t r;
    asc_dtype sig;
    int p, steps, msteps;
    Plan P;
    int tile_rows;
    std::vector<int64_t> node_off;
    std::vector<int32_t> k;
    std::vector<Tile> tiles;
    std::vector<int32_t> tile_off;
    int grid;
    // device copies live in the workspace; uploaded once per workspace pointer
    const void *uploaded_ws = nullptr;
    // captured graph and the pointers it was captured with
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *cap_key[8] = {};
};

struct BatchWs {
    WsHeader *hdr;
    Tile *tiles;
    int32_t *tile_off;
    int32_t *k;
    int64_t *node_off;
    float *diag;
    float *betas;
    double *coeffs;
    double *part;
    void *panelA;
    void *panelB;
};

size_t batch_ws_layout(const BatchPlan &b, void *ws, BatchWs *out) {
    Arena a(ws);
    BatchWs w;
    w.hdr = a.take<WsHeader>(1);
    w.tiles = a.take<Tile>(b.tiles.size());
    w.tile_off = a.take<int32_t>(b.G + 1);
    w.k = a.take<int32_t>(b.G);
    w.node_off = a.take<int64_t>(b.G + 1);
    w.diag = a.take<float>(b.g.n);
    w.betas = a.take<float>(b.G);
    w.coeffs = a.take<double>((size_t)b.G * (b.p + 1));
    w.part = a.take<double>((size_t)b.P.nslices * b.msteps * b.tiles.size() * 3);
    w.panelA = a.take<char>((size_t)b.g.n * b.P.rs * esize(b.sig));
    w.panelB = a.take<char>((size_t)b.g.n * b.P.rs * esize(b.sig));
    if (out) *out = w;
    return a.size();
}

int rows_per_pass(const Plan &P) { return (64 / P.lpr) * (NT / 64); }

// cut every graph into tiles of tile_rows rows (rounded up to whole passes of
// the step kernel; 0 = four passes) for the slice plan P; the device copies of
// the tile list and any captured graph are stale afterwards
void retile(BatchPlan &b, const Plan &P, int tile_rows) {
    const int rp = rows_per_pass(P);
    b.P = P;
    b.tile_rows = tile_rows > 0 ? ((tile_rows + rp - 1) / rp) * rp : rp * 4;
    b.tiles.clear();
    b.tile_off.assign(1, 0);
    for (int q = 0; q < b.G; ++q) {
        for (int64_t r0 = b.node_off[q]; r0 < b.node_off[q + 1]; r0 += b.tile_rows)
            b.tiles.push_back(Tile{q, (int32_t)r0, (int32_t)std::min<int64_t>(r0 + b.tile_rows, b.node_off[q + 1]), 0});
        b.tile_off.push_back((int32_t)b.tiles.size());
    }
    b.grid = (int)std::max<size_t>(1, std::min<size_t>(b.tiles.size(), kMaxGrid));
    b.uploaded_ws = nullptr;
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
}

asc_status upload_plan(BatchPlan &b, void *ws, hipStream_t s) {
    BatchWs W;
    batch_ws_layout(b, ws, &W);
    ASC_HIP(hipStreamSynchronize(s));
    ASC_HIP(hipMemcpy(W.tiles, b.tiles.data(), sizeof(Tile) * b.tiles.size(), hipMemcpyHostToDevice));
    ASC_HIP(hipMemcpy(W.tile_off, b.tile_off.data(), sizeof(int32_t) * b.tile_off.size(), hipMemcpyHostToDevice));
    ASC_HIP(hipMemcpy(W.k, b.k.data(), sizeof(int32_t) * b.k.size(), hipMemcpyHostToDevice));
    ASC_HIP(hipMemcpy(W.node_off, b.node_off.data(), sizeof(int64_t) * b.node_off.size(), hipMemcpyHostToDevice));
    b.uploaded_ws = ws;
    return ASC_OK;
}

// the candidates of the batch autotuner: every supported slice width up to
// the one covering r, times tiles of 1, 2, 4, 8, 16 or 32 passes
template <typename F>
void for_each_candidate(const BatchPlan &b, F &&f) {
    const int vn = vn_of(b.sig);
    int64_t rcap = 2 * vn;
    while (rcap < b.r) rcap *= 2;
    for (int rs = 2 * vn; rs <= 16 * vn && rs <= rcap; rs *= 2) {
        const Plan P = plan_for(rs, 0u, b.r, b.sig);
        for (int m = 1; m <= 32; m *= 2) f(P, m * rows_per_pass(P));
    }
}

asc_status enqueue_batch(BatchPlan &b, const double *lmax, const void *R, int64_t ldr, float *Y, int64_t ldy,
                         double *lambda_k, double *traj, void *ws, hipStream_t s) {
    BatchWs W;
    batch_ws_layout(b, ws, &W);
    const int nt = (int)b.tiles.size();
    const int64_t n = b.g.n;
    batch_diag_kernel<<<std::min(nt, 4096), 256, 0, s>>>(W.tiles, nt, b.g.strength, lmax, W.diag, W.betas,
                                                         W.node_off);
    ASC_LAUNCHED();
    BatchArgs B{};
    B.S.n = n;
    B.S.rp = b.g.row_ptr;
    B.S.ci = b.g.col_idx;
    B.S.w = b.g.w;
    B.S.diag = W.diag;
    B.S.Y = Y;
    B.S.ldy = ldy;
    B.S.r = b.r;
    B.tiles = W.tiles;
    B.ntiles = nt;
    B.betas = W.betas;
    B.coeffs = W.coeffs;
    B.p1 = b.p + 1;
    const int64_t tot = n * b.P.rs;
    const int pg = (int)std::min<int64_t>((tot + 255) / 256, 65536);
    auto pack = [&](int64_t c0) {
        if (b.sig == ASC_F32)
            pack_kernel<float><<<pg, 256, 0, s>>>(n, (const float *)R, ldr, c0, b.r, b.P.rs, (float *)W.panelA);
        else
            pack_kernel<uint16_t><<<pg, 256, 0, s>>>(n, (const uint16_t *)R, ldr, c0, b.r, b.P.rs,
                                                     (uint16_t *)W.panelA);
    };
    // moment levels
    for (int sl = 0; sl < b.P.nslices; ++sl) {
        pack((int64_t)sl * b.P.rs);
        ASC_LAUNCHED();
        void *cur = W.panelA, *prev = W.panelB;
        for (int st = 0; st < b.msteps; ++st) {
            B.S.cur = cur;
            B.S.prev = st == 0 ? nullptr : prev;
            B.S.out = prev;
            B.S.j = st;
            B.S.partials = W.part + ((int64_t)sl * b.msteps + st) * (int64_t)nt * 3;
            hipError_t e = launch_batch(b.sig, b.P.lpr, (st == 0 ? M_FIRST : 0u) | M_PART, B, b.grid, s);
            if (e != hipSuccess) return fail(ASC_ERR_HIP, "batch_step launch failed: %s", hipGetErrorString(e));
            std::swap(cur, prev);
        }
    }
    batch_dichotomy_kernel<<<b.G, NT, sizeof(double) * (b.p + 1), s>>>(W.part, b.P.nslices, b.msteps, nt, W.tile_off,
                                                                        W.k, lmax, b.p, b.steps, lambda_k, traj,
                                                                        W.coeffs);
    ASC_LAUNCHED();
    // filter levels at each graph's lambda_k
    for (int sl = 0; sl < b.P.nslices; ++sl) {
        pack((int64_t)sl * b.P.rs);
        ASC_LAUNCHED();
        B.S.c0 = (int64_t)sl * b.P.rs;
        void *cur = W.panelA, *prev = W.panelB;
        for (int j = 0; j < b.p; ++j) {
            B.S.cur = cur;
            B.S.prev = j == 0 ? nullptr : prev;
            B.S.out = prev;
            B.S.j = j;
            hipError_t e = launch_batch(b.sig, b.P.lpr, j == 0 ? (M_FIRST | M_YACC) : y_mode(j, b.p, b.sig), B, b.grid, s);
            if (e != hipSuccess) return fail(ASC_ERR_HIP, "batch_step launch failed: %s", hipGetErrorString(e));
            std::swap(cur, prev);
        }
    }
    return ASC_OK;
}

}  // namespace
}  // namespace asc

using namespace asc;

extern "C" asc_status asc_batch_create(const asc_graph *g, int n_graphs, const int64_t *node_off_host,
                                       const int32_t *k_host, int64_t r, asc_dtype sig, int p, int steps,
                                       int tile_rows, void **plan_out) {
    const char *who = "asc_batch_create";
    ASC_TRY(check_graph_args(g, true, who));
    if (!plan_out) return fail(ASC_ERR_INVALID, "%s: plan_out is NULL", who);
    *plan_out = nullptr;
    if (n_graphs < 1 || n_graphs > 65536 || !node_off_host || !k_host)
        return fail(ASC_ERR_INVALID, "%s: n_graphs=%d or NULL offsets/k", who, n_graphs);
    if (sig != ASC_F32 && sig != ASC_BF16) return fail(ASC_ERR_INVALID, "%s: dtype", who);
    if (r < 1 || r > 65536 || p < 1 || p > 4000 || steps < 0 || steps > 200)
        return fail(ASC_ERR_INVALID, "%s: r=%lld p=%d steps=%d", who, (long long)r, p, steps);
    if (node_off_host[0] != 0 || node_off_host[n_graphs] != g->n)
        return fail(ASC_ERR_INVALID, "%s: node offsets must run from 0 to n", who);
    for (int q = 0; q < n_graphs; ++q) {
        if (node_off_host[q + 1] <= node_off_host[q]) return fail(ASC_ERR_INVALID, "%s: empty or unsorted graph %d", who, q);
        if (k_host[q] < 0) return fail(ASC_ERR_INVALID, "%s: k[%d] < 0", who, q);
    }
    auto *b = new BatchPlan();
    b->g = *g;
    b->G = n_graphs;
    b->r = r;
    b->sig = sig;
    b->p = p;
    b->steps = steps;
    b->msteps = std::max(1, (p + 1) / 2);
    b->node_off.assign(node_off_host, node_off_host + n_graphs + 1);
    b->k.assign(k_host, k_host + n_graphs);
    retile(*b, make_plan(g, r, sig), tile_rows);
    *plan_out = b;
    return ASC_OK;
}

extern "C" size_t asc_batch_workspace(const void *plan) {
    if (!plan) return 0;
    return batch_ws_layout(*static_cast<const BatchPlan *>(plan), nullptr, nullptr);
}

extern "C" asc_status asc_batch_info(const void *plan, int *slice_cols, int *tile_rows, int *ntiles) {
    if (!plan) return fail(ASC_ERR_INVALID, "asc_batch_info: NULL plan");
    const BatchPlan *b = static_cast<const BatchPlan *>(plan);
    if (slice_cols) *slice_cols = b->P.rs;
    if (tile_rows) *tile_rows = b->tile_rows;
    if (ntiles) *ntiles = (int)b->tiles.size();
    return ASC_OK;
}

namespace asc {
namespace {

// a copy of the plan's shape only: no captured graph, nothing uploaded
BatchPlan shape_copy(const BatchPlan &b) {
    BatchPlan t;
    t.g = b.g;
    t.G = b.G;
    t.r = b.r;
    t.sig = b.sig;
    t.p = b.p;
    t.steps = b.steps;
    t.msteps = b.msteps;
    t.P = b.P;
    t.tile_rows = b.tile_rows;
    t.node_off = b.node_off;
    t.k = b.k;
    t.tiles = b.tiles;
    t.tile_off = b.tile_off;
    t.grid = b.grid;
    return t;
}

asc_status check_run_args(const BatchPlan &b, const double *lmax, const void *R, int64_t ldr, const float *Y,
                          int64_t ldy, const double *lambda_k, const double *traj, const char *who) {
    if (!lmax || !lambda_k || !aligned(lmax, 8) || !aligned(lambda_k, 8) || (traj && !aligned(traj, 8)))
        return fail(ASC_ERR_INVALID, "%s: lmax/lambda_k NULL or misaligned", who);
    ASC_TRY(check_block(R, b.sig, b.g.n, b.r, ldr, who, "R"));
    ASC_TRY(check_block(Y, ASC_F32, b.g.n, b.r, ldy, who, "Y"));
    return ASC_OK;
}

}  // namespace
}  // namespace asc

extern "C" size_t asc_batch_tune_workspace(const void *plan) {
    if (!plan) return 0;
    BatchPlan t = shape_copy(*static_cast<const BatchPlan *>(plan));
    size_t m = 0;
    for_each_candidate(t, [&](const Plan &P, int tr) {
        retile(t, P, tr);
        m = std::max(m, batch_ws_layout(t, nullptr, nullptr));
    });
    return m;
}

extern "C" asc_status asc_batch_autotune(void *plan, const double *lmax, const void *R, int64_t ldr, float *Y,
                                         int64_t ldy, double *lambda_k, double *traj, int probe_runs, void *ws,
                                         size_t ws_bytes, int *best_slice_cols, int *best_tile_rows, float *best_ms,
                                         void *stream) {
    const char *who = "asc_batch_autotune";
    if (!plan) return fail(ASC_ERR_INVALID, "%s: NULL plan", who);
    BatchPlan &b = *static_cast<BatchPlan *>(plan);
    ASC_TRY(check_run_args(b, lmax, R, ldr, Y, ldy, lambda_k, traj, who));
    if (probe_runs < 1 || probe_runs > 100) return fail(ASC_ERR_INVALID, "%s: probe_runs=%d", who, probe_runs);
    ASC_TRY(check_ws(ws, ws_bytes, asc_batch_tune_workspace(plan), who));
    hipStream_t s = as_stream(stream);
    // the candidates overwrite the tile lists in ws: whatever b uploaded or
    // captured there is stale from here on, also if tuning fails
    retile(b, b.P, b.tile_rows);
    BatchPlan t = shape_copy(b);
    hipEvent_t e0, e1;
    ASC_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ASC_ERR_HIP, "%s: event creation failed", who);
    }
    Plan bestP = b.P;
    int bestTR = b.tile_rows;
    float bestMs = 1e30f;
    bool warm = false;
    asc_status st = ASC_OK;
    for_each_candidate(t, [&](const Plan &P, int tr) {
        if (st != ASC_OK) return;
        retile(t, P, tr);
        st = upload_plan(t, ws, s);
        if (st == ASC_OK && !warm) st = enqueue_batch(t, lmax, R, ldr, Y, ldy, lambda_k, traj, ws, s);
        warm = true;
        if (st == ASC_OK && hipEventRecord(e0, s) != hipSuccess) st = fail(ASC_ERR_HIP, "%s: event record", who);
        for (int it = 0; it < probe_runs && st == ASC_OK; ++it)
            st = enqueue_batch(t, lmax, R, ldr, Y, ldy, lambda_k, traj, ws, s);
        if (st != ASC_OK) return;
        float ms = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = fail(ASC_ERR_HIP, "%s: timing failed", who);
            return;
        }
        ms /= (float)probe_runs;
        if (ms < bestMs) {
            bestMs = ms;
            bestP = P;
            bestTR = t.tile_rows;
        }
    });
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != ASC_OK) return st;
    retile(b, bestP, bestTR);
    if (best_slice_cols) *best_slice_cols = bestP.rs;
    if (best_tile_rows) *best_tile_rows = b.tile_rows;
    if (best_ms) *best_ms = bestMs;
    return ASC_OK;
}

extern "C" asc_status asc_batch_run(void *plan, const double *lmax, const void *R, int64_t ldr, float *Y, int64_t ldy,
                                    double *lambda_k, double *traj, void *ws, size_t ws_bytes, int use_graph,
                                    void *stream) {
    const char *who = "asc_batch_run";
    if (!plan) return fail(ASC_ERR_INVALID, "%s: NULL plan", who);
    BatchPlan &b = *static_cast<BatchPlan *>(plan);
    ASC_TRY(check_run_args(b, lmax, R, ldr, Y, ldy, lambda_k, traj, who));
    ASC_TRY(check_ws(ws, ws_bytes, asc_batch_workspace(plan), who));
    hipStream_t s = as_stream(stream);
    if (b.uploaded_ws != ws) ASC_TRY(upload_plan(b, ws, s));
    if (!use_graph) return enqueue_batch(b, lmax, R, ldr, Y, ldy, lambda_k, traj, ws, s);
    const void *key[8] = {lmax, R, (const void *)(intptr_t)ldr, Y, (const void *)(intptr_t)ldy, lambda_k, traj, ws};
    bool same = b.exec != nullptr;
    for (int q = 0; q < 8 && same; ++q) same = key[q] == b.cap_key[q];
    if (!same) {
        if (b.exec) {
            (void)hipGraphExecDestroy(b.exec);
            b.exec = nullptr;
        }
        if (b.graph) {
            (void)hipGraphDestroy(b.graph);
            b.graph = nullptr;
        }
        hipStream_t cs;
        ASC_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(cs);
            return fail(ASC_ERR_HIP, "%s: capture failed: %s", who, hipGetErrorString(e));
        }
        asc_status st = enqueue_batch(b, lmax, R, ldr, Y, ldy, lambda_k, traj, ws, cs);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cs, &graph);
        (void)hipStreamDestroy(cs);
        if (st != ASC_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return fail(ASC_ERR_HIP, "%s: end capture failed: %s", who, hipGetErrorString(e));
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(ASC_ERR_HIP, "%s: graph instantiate failed: %s", who, hipGetErrorString(e));
        }
        b.graph = graph;
        b.exec = exec;
        for (int q = 0; q < 8; ++q) b.cap_key[q] = key[q];
    }
    ASC_HIP(hipGraphLaunch(b.exec, s));
    return ASC_OK;
}

extern "C" asc_status asc_batch_destroy(void *plan) {
    if (!plan) return ASC_OK;
    BatchPlan *b = static_cast<BatchPlan *>(plan);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
    return ASC_OK;
}
