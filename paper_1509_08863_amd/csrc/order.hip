// Choice of the polynomial order (note on the choice of m, Sec. 2.4): the
// least m whose Jackson-damped Chebyshev approximation of the ideal low-pass
// h_{lambda_c} stays within delta of it, as a function of rho = lambda_c /
// lambda_N alone, so it can be tabulated once and looked up per graph.
//
// The sup of |h - p_m| is taken outside the transition band |lambda -
// lambda_c| < w lambda_N (at the jump no polynomial is close to h), on the
// grid x_i = cos(pi i / (G-1)) of x = 2 lambda / lambda_N - 1.  One block per
// (m, rho): the m+1 coefficients in LDS, every thread evaluates p_m at its
// grid points by the three-term recurrence in float64, and the block takes
// the maximum (order-independent, so exact).
#include "common.hpp"
#include "coeffs.hpp"

#include <algorithm>

namespace asc {
namespace {

constexpr int NT = 256;
constexpr int kMaxOrder = 8000;

__global__ __launch_bounds__(NT) void order_err_kernel(const double *__restrict__ rho, int m_max, double band,
                                                       int G, int jackson, double *__restrict__ err) {
    extern __shared__ double a[];  // m + 1
    __shared__ double red[NT / 64];
    const int m = blockIdx.x + 1;
    const int q = blockIdx.y;
    const double r = rho[q];
    const double xc = 2.0 * r - 1.0;
    for (int j = threadIdx.x; j <= m; j += NT) a[j] = cheb_coeff_dev(r, 1.0, m, j, jackson);
    __syncthreads();
    double emax = 0.0;
    for (int i = threadIdx.x; i < G; i += NT) {
        const double x = cos(kPi * (double)i / (double)(G - 1));
        if (fabs(x - xc) < 2.0 * band) continue;
        double t0 = 1.0, t1 = x;
        double s = a[0] + a[1] * x;
        for (int j = 2; j <= m; ++j) {
            const double t2 = 2.0 * x * t1 - t0;
            s += a[j] * t2;
            t0 = t1;
            t1 = t2;
        }
        const double h = x <= xc ? 1.0 : 0.0;
        emax = fmax(emax, fabs(h - s));
    }
    for (int off = 32; off > 0; off >>= 1) emax = fmax(emax, __shfl_xor(emax, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = emax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double e = red[0];
        for (int w = 1; w < NT / 64; ++w) e = fmax(e, red[w]);
        err[(int64_t)q * m_max + (m - 1)] = e;
    }
}

// m*[q][d] = least m with err[q][m-1] <= delta[d], m_max + 1 if none
__global__ void order_pick_kernel(const double *__restrict__ err, int n_rho, int m_max,
                                  const double *__restrict__ delta, int n_delta, int32_t *__restrict__ m_star) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_rho * n_delta) return;
    const int q = (int)(t / n_delta);
    const int d = (int)(t - (int64_t)q * n_delta);
    const double dl = delta[d];
    int ms = m_max + 1;
    for (int m = 1; m <= m_max; ++m)
        if (err[(int64_t)q * m_max + (m - 1)] <= dl) {
            ms = m;
            break;
        }
    m_star[t] = ms;
}

}  // namespace
}  // namespace asc

using namespace asc;

extern "C" size_t asc_order_table_workspace(int n_rho, int m_max) {
    if (n_rho < 1 || m_max < 1) return 0;
    Arena a(nullptr);
    a.take<double>((size_t)n_rho * m_max);
    return a.size();
}

extern "C" asc_status asc_order_table(const double *rho, int n_rho, const double *delta, int n_delta, double band,
                                      int m_max, int grid, int jackson, double *err, int32_t *m_star, void *ws,
                                      size_t ws_bytes, void *stream) {
    const char *who = "asc_order_table";
    if (!rho || !aligned(rho, 8) || n_rho < 1 || n_rho > 65535)
        return fail(ASC_ERR_INVALID, "%s: rho NULL/misaligned or n_rho=%d not in [1, 65535]", who, n_rho);
    if (!delta || !aligned(delta, 8) || n_delta < 1 || n_delta > 4096)
        return fail(ASC_ERR_INVALID, "%s: delta NULL/misaligned or n_delta=%d", who, n_delta);
    if (!(band >= 0.0) || !(band < 1.0)) return fail(ASC_ERR_INVALID, "%s: band=%g not in [0, 1)", who, band);
    if (m_max < 1 || m_max > kMaxOrder) return fail(ASC_ERR_INVALID, "%s: m_max=%d not in [1, %d]", who, m_max, kMaxOrder);
    if (grid < 2 || grid > (1 << 22)) return fail(ASC_ERR_INVALID, "%s: grid=%d not in [2, 2^22]", who, grid);
    if (!m_star || !aligned(m_star, 4) || (err && !aligned(err, 8)))
        return fail(ASC_ERR_INVALID, "%s: m_star NULL or outputs misaligned", who);
    double *e = err;
    if (!e) {
        ASC_TRY(check_ws(ws, ws_bytes, asc_order_table_workspace(n_rho, m_max), who));
        e = static_cast<double *>(ws);
    }
    hipStream_t s = as_stream(stream);
    order_err_kernel<<<dim3((unsigned)m_max, (unsigned)n_rho), NT, (size_t)(m_max + 1) * sizeof(double), s>>>(
        rho, m_max, band, grid, jackson ? 1 : 0, e);
    ASC_LAUNCHED();
    const int64_t tot = (int64_t)n_rho * n_delta;
    order_pick_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(e, n_rho, m_max, delta, n_delta, m_star);
    ASC_LAUNCHED();
    return ASC_OK;
}
