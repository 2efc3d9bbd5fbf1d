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
// At T > 0 the weights tanh(E/2T) (gap) and f(E) (electron density) have no
// closed form; cbdg_sum_coefficients integrates them (k_sum_coeff) and the
// sums take those coefficients instead.
#include "common.hpp"

#include <algorithm>
#include <cmath>

namespace cbdg {

struct WeightParams {
    int N;
    int kernel;
    double lambda;
    double th0, thh, thl;  // angles of the sign weight
    const double *coeff;   // damped coefficients g_n c_n replacing the T = 0 ones, or null
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

// theta(-E) = 1 for theta > th_0: c_0 = (pi - th_0)/pi, c_n = -2 sin(n th_0)/(pi n)
__device__ inline double step_coefficient(int n, double th0)
{
    if (n == 0) return (M_PI - th0) / M_PI;
    return -2.0 * sin(n * th0) / (M_PI * n);
}

// w->T must be 0 unless the caller passes coefficients (need_sign: the sum
// uses the T-dependent weight).
static int make_weights(const cbdg_weights *w, int N, bool need_sign, WeightParams &P, const char *who,
                        const double *coeff = nullptr)
{
    if (!w) return fail(CBDG_EINVAL, "%s: weights must not be NULL", who);
    if (w->kernel != CBDG_KERNEL_JACKSON && w->kernel != CBDG_KERNEL_LORENTZ)
        return fail(CBDG_EINVAL, "%s: unknown kernel %d", who, w->kernel);
    if (w->kernel == CBDG_KERNEL_LORENTZ && !(w->lambda > 0.0 && std::isfinite(w->lambda)))
        return fail(CBDG_EINVAL, "%s: the Lorentz kernel needs lambda > 0", who);
    if (!(w->a > 0.0) || !std::isfinite(w->a) || !std::isfinite(w->b))
        return fail(CBDG_EINVAL, "%s: weights need a finite a > 0 and finite b", who);
    if (!(w->T >= 0.0) || !std::isfinite(w->T)) return fail(CBDG_EINVAL, "%s: T must be finite and >= 0", who);
    if (need_sign && w->T > 0.0 && !coeff)
        return fail(CBDG_EINVAL, "%s: T > 0 needs the coefficients of cbdg_sum_coefficients", who);
    P.N = N;
    P.kernel = w->kernel;
    P.lambda = w->lambda;
    P.th0 = P.thh = P.thl = 0.0;
    P.coeff = need_sign ? coeff : nullptr;
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
    for (int n = threadIdx.x; n < N; n += blockDim.x)
        wt[n] = A.P.coeff ? A.P.coeff[n] : kernel_factor(n, A.P) * sign_coefficient(n, A.P);
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

// LDOS(r, m) = norm / sqrt(1 - x_m^2) * sum_n mu[r][n] w_n T_n(x_m) with
// w_n = pref_n g_n, x_m = (E_m - b)/a: a product of the moments [rows x N]
// with the weighted Chebyshev table [N x nE], tiled through LDS.  A
// workgroup takes 64 rows x 64 energies; per chunk of 32 moments it stages
// the rows' moments and the table's chunk (threads 0..63 advance the
// three-term recurrence of T_n for one energy each, in order of n, so the
// table is exact to the recurrence's rounding), then each thread adds 4 x 4
// outputs, every output summed over n in order.
constexpr int kLdR = 64, kLdE = 64, kLdN = 32, kLdosTable = 4096;

__global__ __launch_bounds__(kBlock) void k_ldos(LdosArgs A)
{
    __shared__ double ms[kLdR][kLdN + 1];
    __shared__ double ts[kLdN][kLdE];
    __shared__ double gt[kLdosTable];  // pref_n g_n, once per workgroup when N fits
    const int N = A.P.N;
    const bool table = N <= kLdosTable;
    const int tid = threadIdx.x;
    if (table)
        for (int n = tid; n < N; n += blockDim.x) gt[n] = (n == 0 ? 1.0 : 2.0) * kernel_factor(n, A.P);
    const double norm = 1.0 / (M_PI * A.a);
    const int n_et = (A.nE + kLdE - 1) / kLdE;
    const int64_t n_tiles = (A.rows + kLdR - 1) / kLdR * n_et;
    const int tr = tid / 16, tc = tid % 16;  // the thread's rows tr*4.., energies tc*4..
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t r0 = tile / n_et * kLdR;
        const int e0 = (int)(tile % n_et) * kLdE;
        const double x = tid < kLdE && e0 + tid < A.nE ? (A.E[e0 + tid] - A.b) / A.a : 0.0;
        double t0 = 1.0, t1 = x;  // T_{n-2}, T_{n-1}
        double acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
        for (int c0 = 0; c0 < N; c0 += kLdN) {
            const int cn = min(kLdN, N - c0);
            __syncthreads();
            for (int i = tid; i < kLdR * kLdN; i += blockDim.x) {
                const int rr = i / kLdN, k = i % kLdN;
                const int64_t row = r0 + rr;
                ms[rr][k] = row < A.rows && k < cn ? A.mu[row * N + c0 + k] : 0.0;
            }
            if (tid < kLdE) {
                for (int k = 0; k < kLdN; ++k) {
                    const int n = c0 + k;
                    double tn;
                    if (n == 0) tn = 1.0;
                    else if (n == 1) tn = x;
                    else { tn = 2.0 * x * t1 - t0; t0 = t1; t1 = tn; }
                    const double g = k >= cn ? 0.0 : table ? gt[n] : (n == 0 ? 1.0 : 2.0) * kernel_factor(n, A.P);
                    ts[k][tid] = g * tn;
                }
            }
            __syncthreads();
            for (int k = 0; k < cn; ++k) {
                double mv[4], tv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) mv[i] = ms[tr * 4 + i][k];
#pragma unroll
                for (int j = 0; j < 4; ++j) tv[j] = ts[k][tc * 4 + j];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_fma(mv[i], tv[j], acc[i][j]);
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = e0 + tc * 4 + j;
            if (e >= A.nE) continue;
            const double xe = (A.E[e] - A.b) / A.a;
            const double f = fabs(xe) < 1.0 ? norm / sqrt(1.0 - xe * xe) : __builtin_nan("");
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t row = r0 + tr * 4 + i;
                if (row < A.rows) A.out[row * A.nE + e] = acc[i][j] * f;
            }
        }
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
    for (int n = threadIdx.x; n < N; n += blockDim.x)
        wt[n] = A.P.coeff ? A.P.coeff[n] : kernel_factor(n, A.P) * sign_coefficient(n, A.P);
    __syncthreads();
    for (int64_t r = blockIdx.x; r < A.rows; r += gridDim.x) {
        const double g = A.dout[r];
        const double f = A.alpha * 0.5 * (A.Urows ? A.Urows[r] : A.U) * g;
        for (int n = threadIdx.x; n < N; n += blockDim.x) A.dmu[r * N + n] = f * wt[n];
        if (threadIdx.x == 0 && A.din) A.din[r] = (1.0 - A.alpha) * g;
    }
}

// Chebyshev coefficients of the finite-T weights, one workgroup per n:
//   c_n = ((2 - delta_n0)/pi) int w(a cos t + b) cos(n t) dt  over [t_lo, t_hi]
// (the cutoff range for the gap, [0, pi] for the density).  Outside the
// transition zone |E| < 40 T the weight is constant to 1e-17 (+1 / -1 for
// tanh(E/2T), 0 / 1 for f(E)) and its pieces integrate in closed form; the
// zone is split into P panels of 8-point Gauss-Legendre nodes, panel width at
// most 1/(2N) (cos(n t)) and T/(4a) (the weight).  Panels are shared out over
// the threads in a fixed order and reduced in a fixed tree: reproducible bits.
struct CoeffArgs {
    int N;
    int quantity;
    WeightParams P;     // kernel factors
    double a, b, T;
    double lo, hi;      // integration range in t
    double z0, z1;      // transition zone (z0 < z1), clipped to [lo, hi]
    int64_t panels;
    double gx[8], gw[8];  // Gauss-Legendre nodes and weights on [-1, 1]
    double *out;
};

__device__ inline double piece(int n, double p, double q)
{
    if (!(q > p)) return 0.0;
    return n == 0 ? q - p : (sin(n * q) - sin(n * p)) / n;
}

__global__ __launch_bounds__(kBlock) void k_sum_coeff(CoeffArgs A)
{
    const int n = blockIdx.x;
    const bool gap = A.quantity == CBDG_QTY_GAP;
    double acc = 0.0;
    if (A.z1 > A.z0) {
        const double h = (A.z1 - A.z0) / (double)A.panels;
        for (int64_t p = threadIdx.x; p < A.panels; p += blockDim.x) {
            const double c = A.z0 + (p + 0.5) * h;
            double sp = 0.0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const double t = c + 0.5 * h * A.gx[k];
                const double th = tanh((A.a * cos(t) + A.b) / (2.0 * A.T));
                const double wv = gap ? th : 0.5 * (1.0 - th);
                sp += A.gw[k] * wv * cos(n * t);
            }
            acc += 0.5 * h * sp;
        }
    }
    __shared__ double red[kBlock];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // constant pieces: t < z0 is E above the zone, t > z1 below it
        double cst;
        if (gap) cst = piece(n, A.lo, fmin(A.z0, A.hi)) - piece(n, fmax(A.z1, A.lo), A.hi);
        else cst = piece(n, fmax(A.z1, A.lo), A.hi);
        const double c = (n == 0 ? 1.0 : 2.0) / M_PI * (cst + red[0]);
        A.out[n] = kernel_factor(n, A.P) * c;
    }
}

struct DensArgs {
    const double *mu;
    int64_t rows;
    WeightParams P;
    double th0;
    double *out;
};

// n_i = 2 sum_n g_n c_n mu_ee_n(i): one wavefront per row, weights in LDS.
__global__ __launch_bounds__(kBlock) void k_density(DensArgs A)
{
    extern __shared__ double wt[];
    const int N = A.P.N;
    for (int n = threadIdx.x; n < N; n += blockDim.x)
        wt[n] = A.P.coeff ? A.P.coeff[n] : kernel_factor(n, A.P) * step_coefficient(n, A.th0);
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int wpb = blockDim.x / kWave;
    for (int64_t r = (int64_t)blockIdx.x * wpb + wv; r < A.rows; r += (int64_t)gridDim.x * wpb) {
        const double *row = A.mu + r * N;
        double s = 0.0;
        for (int n = lane; n < N; n += kWave) s += wt[n] * row[n];
        s = wave_sum(s);
        if (lane == 0) A.out[r] = 2.0 * s;
    }
}

// d mu_ee[r][n] = 2 g_n c_n d n[r]
__global__ __launch_bounds__(kBlock) void k_density_bwd(const double *dn, int64_t rows, WeightParams P, double th0,
                                                       double *dmu)
{
    extern __shared__ double wt[];
    const int N = P.N;
    for (int n = threadIdx.x; n < N; n += blockDim.x)
        wt[n] = P.coeff ? P.coeff[n] : kernel_factor(n, P) * step_coefficient(n, th0);
    __syncthreads();
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x)
        for (int n = threadIdx.x; n < N; n += blockDim.x) dmu[r * N + n] = 2.0 * dn[r] * wt[n];
}

// Neighbour d (+x, -x, +y, -y) of site s, or -1 outside an open lattice.
__device__ inline int64_t neighbour_of(int64_t s, int d, int Lx, int Ly, int bcx, int bcy)
{
    const int x = (int)(s % Lx), y = (int)(s / Lx);
    int x2 = x + (d == 0 ? 1 : d == 1 ? -1 : 0), y2 = y + (d == 2 ? 1 : d == 3 ? -1 : 0);
    if (x2 < 0 || x2 >= Lx) { if (!bcx) return -1; x2 = (x2 + Lx) % Lx; }
    if (y2 < 0 || y2 >= Ly) { if (!bcy) return -1; y2 = (y2 + Ly) % Ly; }
    return x2 + (int64_t)Lx * y2;
}

struct BondArgs {
    const double *nb;      // [L2][4][N] (complex interleaved when cplx)
    int Lx, Ly, bcx, bcy;
    int cplx;
    WeightParams P;
    double U;
    const double *din;     // [2][L2]
    double alpha;
    double *dout;
    unsigned long long *resid;
    // current
    const void *bonds;     // operator's forward bonds (general), or null
    double t_uniform, a;
    double *cur;           // [2][L2]
};

// sum_n wt_n nb[row][d][n] by one wavefront (complex: both parts)
__device__ inline void wave_dot(const double *nb, int64_t row, int d, int N, int cplx, const double *wt, int lane,
                                double &re, double &im)
{
    re = 0.0; im = 0.0;
    const int64_t base = (row * 4 + d) * (int64_t)N;
    if (cplx) {
        for (int n = lane; n < N; n += kWave) { re += wt[n] * nb[2 * (base + n)]; im += wt[n] * nb[2 * (base + n) + 1]; }
    } else {
        for (int n = lane; n < N; n += kWave) re += wt[n] * nb[base + n];
    }
    re = wave_sum(re);
    im = wave_sum(im);
}

// Bond order parameter (symmetrised singlet) with mixing and residual: one
// wavefront per bond q = axis * L2 + s (bond s -> s + x for axis 0, s + y for
// axis 1): Delta_new = (U/4) [conj(S(s; fwd)) + conj(S(j; back))].
__global__ __launch_bounds__(kBlock) void k_bond_gap(BondArgs A)
{
    extern __shared__ double wt[];
    const int N = A.P.N;
    for (int n = threadIdx.x; n < N; n += blockDim.x)
        wt[n] = A.P.coeff ? A.P.coeff[n] : kernel_factor(n, A.P) * sign_coefficient(n, A.P);
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int wpb = blockDim.x / kWave;
    const int64_t L2 = (int64_t)A.Lx * A.Ly;
    double rmax = 0.0;
    bool saw_nan = false;
    for (int64_t q = (int64_t)blockIdx.x * wpb + wv; q < 2 * L2; q += (int64_t)gridDim.x * wpb) {
        const int axis = (int)(q / L2);
        const int64_t s = q % L2;
        const int fwd = axis == 0 ? 0 : 2, back = fwd + 1;
        const int64_t j = neighbour_of(s, fwd, A.Lx, A.Ly, A.bcx, A.bcy);
        double nr = 0.0, ni = 0.0;
        if (j >= 0) {
            double fr, fi, br, bi;
            wave_dot(A.nb, s, fwd, N, A.cplx, wt, lane, fr, fi);
            wave_dot(A.nb, j, back, N, A.cplx, wt, lane, br, bi);
            nr = 0.25 * A.U * (fr + br);
            ni = -0.25 * A.U * (fi + bi);  // conj
        }
        if (lane == 0) {
            if (A.cplx) {
                const double orr = A.din[2 * q], oi = A.din[2 * q + 1];
                A.dout[2 * q] = (1.0 - A.alpha) * orr + A.alpha * nr;
                A.dout[2 * q + 1] = (1.0 - A.alpha) * oi + A.alpha * ni;
                const double d = hypot(nr - orr, ni - oi);
                if (d != d) saw_nan = true; else rmax = fmax(rmax, d);
            } else {
                const double orr = A.din[q];
                A.dout[q] = (1.0 - A.alpha) * orr + A.alpha * nr;
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

// Particle current along bond q (both spins): J = 4 Im(t_ij <c_i^+ c_j>) with
// <c_i^+ c_j> = sum_n wt_n <j,e|T_n|i,e> and t_ij the unscaled hopping.
__global__ __launch_bounds__(kBlock) void k_bond_current(BondArgs A)
{
    extern __shared__ double wt[];
    const int N = A.P.N;
    for (int n = threadIdx.x; n < N; n += blockDim.x) wt[n] = A.P.coeff[n];
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int wpb = blockDim.x / kWave;
    const int64_t L2 = (int64_t)A.Lx * A.Ly;
    for (int64_t q = (int64_t)blockIdx.x * wpb + wv; q < 2 * L2; q += (int64_t)gridDim.x * wpb) {
        const int axis = (int)(q / L2);
        const int64_t s = q % L2;
        const int fwd = axis == 0 ? 0 : 2;
        const int64_t j = neighbour_of(s, fwd, A.Lx, A.Ly, A.bcx, A.bcy);
        double J = 0.0;
        if (j >= 0) {
            double rr, ri;
            wave_dot(A.nb, s, fwd, N, A.cplx, wt, lane, rr, ri);
            double tr = A.t_uniform, ti = 0.0;
            if (A.bonds) {
                if (A.cplx) {
                    const BondsC<double> b = reinterpret_cast<const BondsC<double> *>(A.bonds)[s];
                    tr = A.a * (axis == 0 ? b.txr : b.tyr);
                    ti = A.a * (axis == 0 ? b.txi : b.tyi);
                } else {
                    const BondsR<double> b = reinterpret_cast<const BondsR<double> *>(A.bonds)[s];
                    tr = A.a * (axis == 0 ? b.tx : b.ty);
                }
            }
            J = 4.0 * (tr * ri + ti * rr);
        }
        if (lane == 0) A.cur[q] = J;
    }
}

// Nodes and weights of n-point Gauss-Legendre quadrature on [-1, 1]: roots of
// P_n by Newton's method from cos(pi (i + 3/4) / (n + 1/2)), weights
// 2 / ((1 - x^2) P_n'(x)^2).
static void gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
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
                               const cbdg_weights *w, const double *coeff, double U, const double *U_rows,
                               const void *delta_in, double alpha, void *delta_out, double *resid,
                               void *stream)
{
    clear_error();
    if (n_rows < 0 || N < 1) return fail(CBDG_EINVAL, "gap_update: need n_rows >= 0 and N >= 1");
    if (scalar != CBDG_REAL && scalar != CBDG_COMPLEX) return fail(CBDG_EINVAL, "gap_update: bad scalar");
    if (!resid) return fail(CBDG_EINVAL, "gap_update: resid must not be NULL");
    if (!std::isfinite(U) || !std::isfinite(alpha)) return fail(CBDG_EINVAL, "gap_update: U and alpha must be finite");
    WeightParams P;
    int rc = make_weights(w, N, true, P, "gap_update", coeff);
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
    if (n_rows == 0 || n_E == 0) return CBDG_OK;
    if (!mu_ee || !energies || !ldos) return fail(CBDG_EINVAL, "ldos: mu_ee, energies and ldos must not be NULL");
    LdosArgs A{mu_ee, n_rows, P, w->a, w->b, energies, n_E, ldos};
    const int64_t tiles = ceil_div(n_rows, kLdR) * ceil_div(n_E, kLdE);
    hipLaunchKernelGGL(k_ldos, dim3((unsigned)std::min<int64_t>(tiles, 65536)), dim3(kBlock), 0, as_stream(stream), A);
    CBDG_CHECK_LAUNCH("k_ldos");
    return CBDG_OK;
}

extern "C" int cbdg_gap_update_backward(const double *d_delta_out, int64_t n_rows, int32_t N,
                                        const cbdg_weights *w, const double *coeff, double U,
                                        const double *U_rows, double alpha, double *d_mu_he,
                                        double *d_delta_in, void *stream)
{
    clear_error();
    if (n_rows < 0 || N < 1) return fail(CBDG_EINVAL, "gap_update_backward: need n_rows >= 0 and N >= 1");
    WeightParams P;
    int rc = make_weights(w, N, true, P, "gap_update_backward", coeff);
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

extern "C" int cbdg_sum_coefficients(const cbdg_weights *w, int32_t N, int32_t quantity, double *coeff,
                                     void *stream)
{
    clear_error();
    if (N < 1) return fail(CBDG_EINVAL, "sum_coefficients: N must be >= 1");
    if (quantity != CBDG_QTY_GAP && quantity != CBDG_QTY_DENSITY)
        return fail(CBDG_EINVAL, "sum_coefficients: unknown quantity %d", quantity);
    if (!coeff) return fail(CBDG_EINVAL, "sum_coefficients: coeff must not be NULL");
    WeightParams P;
    int rc = make_weights(w, N, false, P, "sum_coefficients");
    if (rc) return rc;
    const double a = w->a, b = w->b, T = w->T;
    if (!(std::fabs(b / a) < 1.0)) return fail(CBDG_EINVAL, "sum_coefficients: E = 0 lies outside the rescaled interval");
    auto th = [&](double x) { return std::acos(std::min(1.0, std::max(-1.0, x))); };
    CoeffArgs A{};
    A.N = N;
    A.quantity = quantity;
    A.P = P;
    A.a = a; A.b = b; A.T = T;
    A.lo = 0.0; A.hi = M_PI;
    if (quantity == CBDG_QTY_GAP && w->E_c > 0.0) { A.lo = th((w->E_c - b) / a); A.hi = th((-w->E_c - b) / a); }
    const double Z = 40.0 * T;  // |E| beyond which tanh(E/2T) = +-1 and f(E) = 0 or 1 to 1e-17
    A.z0 = std::max(th((Z - b) / a), A.lo);
    A.z1 = std::min(th((-Z - b) / a), A.hi);
    if (T == 0.0) A.z0 = A.z1 = th(-b / a);
    A.panels = 0;
    if (A.z1 > A.z0) {
        const double hmax = std::min(0.5 / N, 0.25 * T / a);
        const double np = std::ceil((A.z1 - A.z0) / hmax);
        if (!(np < 4.0e7)) return fail(CBDG_EINVAL, "sum_coefficients: T = %g too small for the quadrature; use T = 0", T);
        A.panels = (int64_t)np;
    }
    gauss_legendre(8, A.gx, A.gw);
    A.out = coeff;
    hipLaunchKernelGGL(k_sum_coeff, dim3((unsigned)N), dim3(kBlock), 0, as_stream(stream), A);
    CBDG_CHECK_LAUNCH("k_sum_coeff");
    return CBDG_OK;
}

extern "C" int cbdg_density(const double *mu_ee, int64_t n_rows, int32_t N, const cbdg_weights *w,
                            const double *coeff, double *density, void *stream)
{
    clear_error();
    if (n_rows < 0 || N < 1) return fail(CBDG_EINVAL, "density: need n_rows >= 0 and N >= 1");
    WeightParams P;
    int rc = make_weights(w, N, false, P, "density");
    if (rc) return rc;
    if (w->T > 0.0 && !coeff) return fail(CBDG_EINVAL, "density: T > 0 needs the coefficients of cbdg_sum_coefficients");
    if (!(std::fabs(w->b / w->a) < 1.0)) return fail(CBDG_EINVAL, "density: E = 0 lies outside the rescaled interval");
    P.coeff = coeff;
    rc = lds_ok((size_t)N * 8, "density");
    if (rc) return rc;
    if (n_rows == 0) return CBDG_OK;
    if (!mu_ee || !density) return fail(CBDG_EINVAL, "density: mu_ee and density must not be NULL");
    DensArgs A{mu_ee, n_rows, P, std::acos(-w->b / w->a), density};
    hipLaunchKernelGGL(k_density, dim3(grid_rows(n_rows, kBlock / kWave)), dim3(kBlock), (size_t)N * 8,
                       as_stream(stream), A);
    CBDG_CHECK_LAUNCH("k_density");
    return CBDG_OK;
}

extern "C" int cbdg_density_backward(const double *d_density, int64_t n_rows, int32_t N, const cbdg_weights *w,
                                     const double *coeff, double *d_mu_ee, void *stream)
{
    clear_error();
    if (n_rows < 0 || N < 1) return fail(CBDG_EINVAL, "density_backward: need n_rows >= 0 and N >= 1");
    WeightParams P;
    int rc = make_weights(w, N, false, P, "density_backward");
    if (rc) return rc;
    if (w->T > 0.0 && !coeff)
        return fail(CBDG_EINVAL, "density_backward: T > 0 needs the coefficients of cbdg_sum_coefficients");
    if (!(std::fabs(w->b / w->a) < 1.0))
        return fail(CBDG_EINVAL, "density_backward: E = 0 lies outside the rescaled interval");
    P.coeff = coeff;
    rc = lds_ok((size_t)N * 8, "density_backward");
    if (rc) return rc;
    if (n_rows == 0) return CBDG_OK;
    if (!d_density || !d_mu_ee) return fail(CBDG_EINVAL, "density_backward: d_density and d_mu_ee must not be NULL");
    hipLaunchKernelGGL(k_density_bwd, dim3(grid_rows(n_rows, 1)), dim3(kBlock), (size_t)N * 8, as_stream(stream),
                       d_density, n_rows, P, std::acos(-w->b / w->a), d_mu_ee);
    CBDG_CHECK_LAUNCH("k_density_bwd");
    return CBDG_OK;
}

extern "C" int cbdg_bond_gap_update(const void *nb_he, int32_t Lx, int32_t Ly, int32_t bc_x, int32_t bc_y,
                                    int32_t N, int32_t scalar, const cbdg_weights *w, const double *coeff,
                                    double U, const void *delta_bond_in, double alpha, void *delta_bond_out,
                                    double *resid, void *stream)
{
    clear_error();
    if (Lx < 1 || Ly < 1 || N < 1) return fail(CBDG_EINVAL, "bond_gap_update: need Lx, Ly, N >= 1");
    if ((bc_x && Lx < 3) || (bc_y && Ly < 3)) return fail(CBDG_EINVAL, "bond_gap_update: periodic directions need >= 3 sites");
    if (scalar != CBDG_REAL && scalar != CBDG_COMPLEX) return fail(CBDG_EINVAL, "bond_gap_update: bad scalar");
    if (!std::isfinite(U) || !std::isfinite(alpha)) return fail(CBDG_EINVAL, "bond_gap_update: U and alpha must be finite");
    if (!nb_he || !delta_bond_in || !delta_bond_out || !resid)
        return fail(CBDG_EINVAL, "bond_gap_update: nb_he, delta_bond_in, delta_bond_out and resid must not be NULL");
    WeightParams P;
    int rc = make_weights(w, N, true, P, "bond_gap_update", coeff);
    if (rc) return rc;
    rc = lds_ok((size_t)N * 8, "bond_gap_update");
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(k_set_f64, dim3(1), dim3(1), 0, st, resid, 0.0);
    CBDG_CHECK_LAUNCH("k_set_f64");
    BondArgs A{};
    A.nb = (const double *)nb_he;
    A.Lx = Lx; A.Ly = Ly; A.bcx = bc_x; A.bcy = bc_y;
    A.cplx = scalar == CBDG_COMPLEX;
    A.P = P;
    A.U = U;
    A.din = (const double *)delta_bond_in;
    A.alpha = alpha;
    A.dout = (double *)delta_bond_out;
    A.resid = (unsigned long long *)resid;
    const int64_t nb = 2 * (int64_t)Lx * Ly;
    hipLaunchKernelGGL(k_bond_gap, dim3(grid_rows(nb, kBlock / kWave)), dim3(kBlock), (size_t)N * 8, st, A);
    CBDG_CHECK_LAUNCH("k_bond_gap");
    return CBDG_OK;
}

extern "C" int cbdg_bond_current(const cbdg_op *op, const void *nb_ee, int32_t N, const cbdg_weights *w,
                                 const double *coeff, double *current, void *stream)
{
    clear_error();
    if (!op || N < 1) return fail(CBDG_EINVAL, "bond_current: need op and N >= 1");
    if (!nb_ee || !current) return fail(CBDG_EINVAL, "bond_current: nb_ee and current must not be NULL");
    WeightParams P;
    int rc = make_weights(w, N, false, P, "bond_current");
    if (rc) return rc;
    if (!coeff) return fail(CBDG_EINVAL, "bond_current: coeff (cbdg_sum_coefficients, CBDG_QTY_DENSITY) is required");
    P.coeff = coeff;
    rc = lds_ok((size_t)N * 8, "bond_current");
    if (rc) return rc;
    BondArgs A{};
    A.nb = (const double *)nb_ee;
    A.Lx = op->Lx; A.Ly = op->Ly; A.bcx = op->bc_x; A.bcy = op->bc_y;
    A.cplx = op->scalar == CBDG_COMPLEX;
    A.P = P;
    A.bonds = op->general ? op->bonds64 : nullptr;
    A.t_uniform = op->t;
    A.a = op->bounds.a;
    A.cur = current;
    const int64_t nb = 2 * op->L2;
    hipLaunchKernelGGL(k_bond_current, dim3(grid_rows(nb, kBlock / kWave)), dim3(kBlock), (size_t)N * 8,
                       as_stream(stream), A);
    CBDG_CHECK_LAUNCH("k_bond_current");
    return CBDG_OK;
}
