// Observables from the moments: the T = 0 order parameter of eq. (op1) with
// plain mixing, the local density of states of eq. (ldos) with eq. (imag2),
// and the transposes of both linear maps.  All sums are FP64.
//
// Weights.  The truncated series is damped by kernel factors g_n (Jackson,
// or the Lorentz kernel that follows eq. (ref2)).  The gap equation weights
// the anomalous moments with the Chebyshev coefficients c_n of
// w(E) = 1 - 2f(E) = sign(E) on |E| < E_c at T = 0.  In the rescaled variable
// x = cos(theta) the weight is +1 for theta in (th_hi, th_0), -1 for theta
// in (th_0, th_lo), with th_0 = acos(-b/a), th_hi = acos((E_c - b)/a) and
// th_lo = acos((-E_c - b)/a) (0 and pi without a cutoff), so
//   c_0 = (2 th_0 - th_hi - th_lo)/pi,
//   c_n = 2 (2 sin(n th_0) - sin(n th_hi) - sin(n th_lo)) / (pi n).
#include "common.hpp"

#include <algorithm>
#include <cmath>

namespace cbdg {

struct WeightParams {
    int N;
    int kernel;
    double lambda;
    double th0, thh, thl;  // angles of the sign weight
};

__device__ inline double kernel_factor(int n, const WeightParams &P)
{
    if (P.kernel == CBDG_KERNEL_LORENTZ)
        return sinh(P.lambda * (1.0 - (double)n / P.N)) / sinh(P.lambda);
    const double q = M_PI / (P.N + 1);
    return ((P.N - n + 1) * cos(q * n) + sin(q * n) * (cos(q) / sin(q))) / (P.N + 1);
}

__device__ inline double sign_coefficient(int n, const WeightParams &P)
{
    if (n == 0) return (2.0 * P.th0 - P.thh - P.thl) / M_PI;
    return 2.0 * (2.0 * sin(n * P.th0) - sin(n * P.thh) - sin(n * P.thl)) / (M_PI * n);
}

static int make_weights(const cbdg_weights *w, int N, bool need_sign, WeightParams &P, const char *who)
{
    if (!w) return fail(CBDG_EINVAL, "%s: weights must not be NULL", who);
    if (w->kernel != CBDG_KERNEL_JACKSON && w->kernel != CBDG_KERNEL_LORENTZ)
        return fail(CBDG_EINVAL, "%s: unknown kernel %d", who, w->kernel);
    if (w->kernel == CBDG_KERNEL_LORENTZ && !(w->lambda > 0.0 && std::isfinite(w->lambda)))
        return fail(CBDG_EINVAL, "%s: the Lorentz kernel needs lambda > 0", who);
    if (!(w->a > 0.0) || !std::isfinite(w->a) || !std::isfinite(w->b))
        return fail(CBDG_EINVAL, "%s: weights need a finite a > 0 and finite b", who);
    if (w->T != 0.0)
        return fail(CBDG_EUNSUPPORTED, "%s: only T = 0 weights are implemented", who);
    P.N = N;
    P.kernel = w->kernel;
    P.lambda = w->lambda;
    P.th0 = P.thh = P.thl = 0.0;
    if (need_sign) {
        const double x0 = -w->b / w->a;
        if (!(std::fabs(x0) < 1.0)) return fail(CBDG_EINVAL, "%s: E = 0 lies outside the rescaled interval", who);
        P.th0 = std::acos(x0);
        if (w->E_c > 0.0) {
            P.thh = std::acos(std::min((w->E_c - w->b) / w->a, 1.0));
            P.thl = std::acos(std::max((-w->E_c - w->b) / w->a, -1.0));
        } else {
            P.thh = 0.0;
            P.thl = M_PI;
        }
    }
    return CBDG_OK;
}

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

struct GapArgs {
    const double *mu;
    int64_t rows;
    int cplx;
    WeightParams P;
    double U;
    const double *Urows;
    const double *din;
    double alpha;
    double *dout;
    unsigned long long *resid;
};

// One wavefront per row: lanes stride over n, then a fixed-order wave
// reduction; the weights g_n c_n are built once per workgroup in LDS.
__global__ __launch_bounds__(kBlock) void k_gap(GapArgs A)
{
    extern __shared__ double wt[];
    const int N = A.P.N;
    for (int n = threadIdx.x; n < N; n += blockDim.x) wt[n] = kernel_factor(n, A.P) * sign_coefficient(n, A.P);
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int wpb = blockDim.x / kWave;
    double rmax = 0.0;
    bool saw_nan = false;
    for (int64_t r = (int64_t)blockIdx.x * wpb + wv; r < A.rows; r += (int64_t)gridDim.x * wpb) {
        double sr = 0.0, si = 0.0;
        if (A.cplx) {
            const double *row = A.mu + 2 * r * N;
            for (int n = lane; n < N; n += kWave) { sr += wt[n] * row[2 * n]; si += wt[n] * row[2 * n + 1]; }
        } else {
            const double *row = A.mu + r * N;
            for (int n = lane; n < N; n += kWave) sr += wt[n] * row[n];
        }
        sr = wave_sum(sr);
        si = wave_sum(si);
        if (lane == 0) {
            const double half_u = 0.5 * (A.Urows ? A.Urows[r] : A.U);
            if (A.cplx) {
                const double nr = half_u * sr, ni = -half_u * si;  // conj
                const double orr = A.din[2 * r], oi = A.din[2 * r + 1];
                A.dout[2 * r] = (1.0 - A.alpha) * orr + A.alpha * nr;
                A.dout[2 * r + 1] = (1.0 - A.alpha) * oi + A.alpha * ni;
                const double d = hypot(nr - orr, ni - oi);
                if (d != d) saw_nan = true; else rmax = fmax(rmax, d);
            } else {
                const double nr = half_u * sr;
                const double orr = A.din[r];
                A.dout[r] = (1.0 - A.alpha) * orr + A.alpha * nr;
                const double d = fabs(nr - orr);
                if (d != d) saw_nan = true; else rmax = fmax(rmax, d);
            }
        }
    }
    if (saw_nan) rmax = __builtin_nan("");
    __shared__ double red[kBlock / kWave];
    if (lane == 0) red[wv] = rmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        bool nan = m != m;
        for (int i = 1; i < wpb; ++i) { nan |= red[i] != red[i]; m = fmax(m, red[i]); }
        const unsigned long long bits = nan ? 0x7ff8000000000000ull : (unsigned long long)__double_as_longlong(m);
        atomicMax(A.resid, bits);
    }
}

__global__ void k_set_f64(double *p, double v) { *p = v; }

struct LdosArgs {
    const double *mu;
    int64_t rows;
    WeightParams P;
    double a, b;
    const double *E;
    int nE;
    double *out;
};

// Rows in a grid-stride loop; per row the damped moments pref_n g_n mu_n go to
// LDS and each thread sums one energy with the three-term recurrence of T_n.
__global__ __launch_bounds__(kBlock) void k_ldos(LdosArgs A)
{
    extern __shared__ double sm[];
    const int N = A.P.N;
    double *g = sm, *m = sm + N;
    for (int n = threadIdx.x; n < N; n += blockDim.x) g[n] = (n == 0 ? 1.0 : 2.0) * kernel_factor(n, A.P);
    __syncthreads();
    const double norm = 1.0 / (M_PI * A.a);
    for (int64_t r = blockIdx.x; r < A.rows; r += gridDim.x) {
        for (int n = threadIdx.x; n < N; n += blockDim.x) m[n] = g[n] * A.mu[r * N + n];
        __syncthreads();
        for (int e = threadIdx.x; e < A.nE; e += blockDim.x) {
            const double x = (A.E[e] - A.b) / A.a;
            double val;
            if (!(fabs(x) < 1.0)) {
                val = __builtin_nan("");
            } else {
                double t0 = 1.0, t1 = x;
                double acc = m[0];
                if (N > 1) acc += m[1] * x;
                for (int n = 2; n < N; ++n) {
                    const double t2 = 2.0 * x * t1 - t0;
                    acc += m[n] * t2;
                    t0 = t1;
                    t1 = t2;
                }
                val = acc * norm / sqrt(1.0 - x * x);
            }
            A.out[r * A.nE + e] = val;
        }
        __syncthreads();
    }
}

struct LdosBwdArgs {
    const double *dl;
    int64_t rows;
    WeightParams P;
    double a, b;
    const double *E;
    int nE;
    double *dmu;
};

constexpr int kLdosBwdChunk = 2048;

// d_mu[r][n] = pref_n g_n sum_m d_ldos[r][m] T_n(x_m) / (pi a sqrt(1 - x_m^2)),
// T_n(x_m) = cos(n acos x_m); energies are staged through LDS in chunks.
__global__ __launch_bounds__(kBlock) void k_ldos_bwd(LdosBwdArgs A)
{
    __shared__ double q[kLdosBwdChunk], th[kLdosBwdChunk];
    const int N = A.P.N;
    const double norm = 1.0 / (M_PI * A.a);
    for (int64_t r = blockIdx.x; r < A.rows; r += gridDim.x) {
        for (int n = threadIdx.x; n < N; n += blockDim.x) A.dmu[r * N + n] = 0.0;
        for (int e0 = 0; e0 < A.nE; e0 += kLdosBwdChunk) {
            const int ne = min(kLdosBwdChunk, A.nE - e0);
            __syncthreads();
            for (int e = threadIdx.x; e < ne; e += blockDim.x) {
                const double x = (A.E[e0 + e] - A.b) / A.a;
                const bool ok = fabs(x) < 1.0;
                th[e] = ok ? acos(x) : 0.0;
                q[e] = ok ? A.dl[r * A.nE + e0 + e] * norm / sqrt(1.0 - x * x) : __builtin_nan("");
            }
            __syncthreads();
            for (int n = threadIdx.x; n < N; n += blockDim.x) {
                double acc = 0.0;
                for (int e = 0; e < ne; ++e) acc += q[e] * cos(n * th[e]);
                A.dmu[r * N + n] += (n == 0 ? 1.0 : 2.0) * kernel_factor(n, A.P) * acc;
            }
        }
    }
}

struct GapBwdArgs {
    const double *dout;
    int64_t rows;
    WeightParams P;
    double U;
    const double *Urows;
    double alpha;
    double *dmu;
    double *din;
};

__global__ __launch_bounds__(kBlock) void k_gap_bwd(GapBwdArgs A)
{
    extern __shared__ double wt[];
    const int N = A.P.N;
    for (int n = threadIdx.x; n < N; n += blockDim.x) wt[n] = kernel_factor(n, A.P) * sign_coefficient(n, A.P);
    __syncthreads();
    for (int64_t r = blockIdx.x; r < A.rows; r += gridDim.x) {
        const double g = A.dout[r];
        const double f = A.alpha * 0.5 * (A.Urows ? A.Urows[r] : A.U) * g;
        for (int n = threadIdx.x; n < N; n += blockDim.x) A.dmu[r * N + n] = f * wt[n];
        if (threadIdx.x == 0 && A.din) A.din[r] = (1.0 - A.alpha) * g;
    }
}

static unsigned grid_rows(int64_t rows, int per_block) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(rows, per_block), 2048)); }

static int lds_ok(size_t bytes, const char *who)
{
    if (bytes > 64 * 1024) return fail(CBDG_EUNSUPPORTED, "%s: N too large for the LDS weight table", who);
    return CBDG_OK;
}

}  // namespace cbdg

using namespace cbdg;

extern "C" int cbdg_gap_update(const void *mu_he, int64_t n_rows, int32_t N, int32_t scalar,
                               const cbdg_weights *w, double U, const double *U_rows,
                               const void *delta_in, double alpha, void *delta_out, double *resid,
                               void *stream)
{
    clear_error();
    if (n_rows < 0 || N < 1) return fail(CBDG_EINVAL, "gap_update: need n_rows >= 0 and N >= 1");
    if (scalar != CBDG_REAL && scalar != CBDG_COMPLEX) return fail(CBDG_EINVAL, "gap_update: bad scalar");
    if (!resid) return fail(CBDG_EINVAL, "gap_update: resid must not be NULL");
    if (!std::isfinite(U) || !std::isfinite(alpha)) return fail(CBDG_EINVAL, "gap_update: U and alpha must be finite");
    WeightParams P;
    int rc = make_weights(w, N, true, P, "gap_update");
    if (rc) return rc;
    rc = lds_ok((size_t)N * 8, "gap_update");
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(k_set_f64, dim3(1), dim3(1), 0, st, resid, 0.0);
    CBDG_CHECK_LAUNCH("k_set_f64");
    if (n_rows == 0) return CBDG_OK;
    if (!mu_he || !delta_in || !delta_out)
        return fail(CBDG_EINVAL, "gap_update: mu_he, delta_in and delta_out must not be NULL");
    GapArgs A{(const double *)mu_he, n_rows, scalar == CBDG_COMPLEX, P, U, U_rows,
              (const double *)delta_in, alpha, (double *)delta_out, (unsigned long long *)resid};
    hipLaunchKernelGGL(k_gap, dim3(grid_rows(n_rows, kBlock / kWave)), dim3(kBlock), (size_t)N * 8, st, A);
    CBDG_CHECK_LAUNCH("k_gap");
    return CBDG_OK;
}

extern "C" int cbdg_ldos(const double *mu_ee, int64_t n_rows, int32_t N, const cbdg_weights *w,
                         const double *energies, int32_t n_E, double *ldos, void *stream)
{
    clear_error();
    if (n_rows < 0 || N < 1 || n_E < 0) return fail(CBDG_EINVAL, "ldos: need n_rows >= 0, N >= 1, n_E >= 0");
    WeightParams P;
    int rc = make_weights(w, N, false, P, "ldos");
    if (rc) return rc;
    rc = lds_ok((size_t)2 * N * 8, "ldos");
    if (rc) return rc;
    if (n_rows == 0 || n_E == 0) return CBDG_OK;
    if (!mu_ee || !energies || !ldos) return fail(CBDG_EINVAL, "ldos: mu_ee, energies and ldos must not be NULL");
    LdosArgs A{mu_ee, n_rows, P, w->a, w->b, energies, n_E, ldos};
    hipLaunchKernelGGL(k_ldos, dim3(grid_rows(n_rows, 1)), dim3(kBlock), (size_t)2 * N * 8, as_stream(stream), A);
    CBDG_CHECK_LAUNCH("k_ldos");
    return CBDG_OK;
}

extern "C" int cbdg_gap_update_backward(const double *d_delta_out, int64_t n_rows, int32_t N,
                                        const cbdg_weights *w, double U, const double *U_rows,
                                        double alpha, double *d_mu_he, double *d_delta_in, void *stream)
{
    clear_error();
    if (n_rows < 0 || N < 1) return fail(CBDG_EINVAL, "gap_update_backward: need n_rows >= 0 and N >= 1");
    WeightParams P;
    int rc = make_weights(w, N, true, P, "gap_update_backward");
    if (rc) return rc;
    rc = lds_ok((size_t)N * 8, "gap_update_backward");
    if (rc) return rc;
    if (n_rows == 0) return CBDG_OK;
    if (!d_delta_out || !d_mu_he) return fail(CBDG_EINVAL, "gap_update_backward: d_delta_out and d_mu_he must not be NULL");
    GapBwdArgs A{d_delta_out, n_rows, P, U, U_rows, alpha, d_mu_he, d_delta_in};
    hipLaunchKernelGGL(k_gap_bwd, dim3(grid_rows(n_rows, 1)), dim3(kBlock), (size_t)N * 8, as_stream(stream), A);
    CBDG_CHECK_LAUNCH("k_gap_bwd");
    return CBDG_OK;
}

extern "C" int cbdg_ldos_backward(const double *d_ldos, int64_t n_rows, int32_t N, const cbdg_weights *w,
                                  const double *energies, int32_t n_E, double *d_mu_ee, void *stream)
{
    clear_error();
    if (n_rows < 0 || N < 1 || n_E < 0) return fail(CBDG_EINVAL, "ldos_backward: need n_rows >= 0, N >= 1, n_E >= 0");
    WeightParams P;
    int rc = make_weights(w, N, false, P, "ldos_backward");
    if (rc) return rc;
    if (n_rows == 0) return CBDG_OK;
    if (!d_ldos || !d_mu_ee || (n_E > 0 && !energies))
        return fail(CBDG_EINVAL, "ldos_backward: d_ldos, energies and d_mu_ee must not be NULL");
    LdosBwdArgs A{d_ldos, n_rows, P, w->a, w->b, energies, n_E, d_mu_ee};
    hipLaunchKernelGGL(k_ldos_bwd, dim3(grid_rows(n_rows, 1)), dim3(kBlock), 0, as_stream(stream), A);
    CBDG_CHECK_LAUNCH("k_ldos_bwd");
    return CBDG_OK;
}
