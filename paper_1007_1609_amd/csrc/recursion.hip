// Batched Chebyshev vector recursion of eq. (ref2) with fused extraction of
// the local moments of eqs. (coeff1)/(coeff2).
//
// A tile of B start vectors |s_b,e> is stored vector-major: the Nambu pair of
// vector b at site s sits at s*Bp + b (Bp = B rounded up to the wavefront).
// One launch advances the whole tile by one step,
//     a_n = 2 Ht a_{n-1} - a_{n-2}    (in place over a_{n-2}),
// and lane b stores <s_b,e|a_n> and <s_b,h|a_n> when it passes its own start
// site.  The kernel is bound by HBM bandwidth (about 16 flops per 24 bytes
// in FP64), so the design is about moving each byte once:
//   - lanes map to vectors, so every neighbour read of a wavefront is one
//     contiguous run, and the per-site coefficients are wave-uniform scalar
//     loads reused by all 64 lanes;
//   - each lane owns a strip of W sites along x and marches up a segment of
//     rows in y, keeping rows y-1, y, y+1 of a_{n-1} in registers, so a_{n-1}
//     is read about once (plus the strip's x halo and the segment's y halo,
//     which neighbouring strips on the same XCD fetch at nearly the same time);
//   - a_{n-2} is read and a_n written by the same lane at the same address.
#include "stencil.hpp"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace cbdg {

struct StepArgs {
    const void *prev1;   // a_{n-1}
    const void *prev2;   // a_{n-2} (unused on the first step)
    void *out;           // a_n (may alias prev2)
    const void *onsite;  // OnSite<T>[L2]
    const void *bonds;   // BondsR<T>/BondsC<T>[L2] (general operators)
    double th;           // t/a (uniform operators)
    int Lx, Ly, bcx, bcy;
    int Bp;              // lane stride of the tile layout
    int Bt;              // vectors in the tile
    int first;           // 1: a_1 = Ht a_0
    int n, N;            // moment index produced, moments per row
    const int32_t *sites;  // [Bt] start sites of the tile
    double *mu_ee;       // tile's first row
    double *mu_he;       // tile's first row (complex interleaved for C)
    int n_strips, n_segs, nblocks;
};

template <typename T, bool C, bool GEN, int W, int YS>
__global__ __launch_bounds__(kBlock) void k_cheb_step(StepArgs A)
{
    using P = Pair<T, C>;
    using S = typename Storage<T, C>::type;
    const int lb = xcd_remap(blockIdx.x, A.nblocks);
    const int strip = lb % A.n_strips;
    const int rest = lb / A.n_strips;
    const int seg = rest % A.n_segs;
    const int chunk = rest / A.n_segs;
    const int b = chunk * kBlock + threadIdx.x;
    if (b >= A.Bt) return;

    const int Lx = A.Lx, Ly = A.Ly;
    const int x0 = strip * W;
    const int y0 = seg * YS;
    const int y1 = min(y0 + YS, Ly);
    const int64_t Bp = A.Bp;
    const S *a1 = reinterpret_cast<const S *>(A.prev1);
    const S *a2 = reinterpret_cast<const S *>(A.prev2);
    S *ao = reinterpret_cast<S *>(A.out);
    const OnSite<T> *ons = reinterpret_cast<const OnSite<T> *>(A.onsite);
    const int my_site = A.sites[b];
    const T th = T(A.th);
    const bool first = A.first != 0;

    // column k of the register window holds x = x0 - 1 + k
    auto col_of = [&](int k) -> int {
        int x = x0 - 1 + k;
        if (x >= 0 && x < Lx) return x;
        if (A.bcx && (x == -1 || x == Lx)) return x < 0 ? x + Lx : x - Lx;
        return -1;
    };
    auto row_of = [&](int y) -> int {
        if (y >= 0 && y < Ly) return y;
        if (A.bcy && (y == -1 || y == Ly)) return y < 0 ? y + Ly : y - Ly;
        return -1;
    };
    auto load_row = [&](P *row, int y, int kbeg, int kend) {
        const int yy = row_of(y);
#pragma unroll
        for (int k = 0; k < W + 2; ++k) {
            if (k < kbeg || k >= kend) continue;
            const int xx = col_of(k);
            if (yy >= 0 && xx >= 0) row[k] = ld<T, C>(a1 + ((int64_t)yy * Lx + xx) * Bp + b);
            else row[k] = zero_pair<T, C>();
        }
    };

    P up[W + 2], cur[W + 2], dn[W + 2];
    load_row(up, y0 - 1, 1, W + 1);
    load_row(cur, y0, 0, W + 2);

    for (int y = y0; y < y1; ++y) {
        load_row(dn, y + 1, 0, W + 2);
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int x = x0 + k;
            if (x >= Lx) continue;
            const int64_t s = (int64_t)y * Lx + x;
            const OnSite<T> o = ons[s];
            P yv;
            if constexpr (GEN) {
                const int64_t sl = x > 0 ? s - 1 : (A.bcx ? s + Lx - 1 : -1);
                const int64_t sd = y > 0 ? s - Lx : (A.bcy ? s + (int64_t)(Ly - 1) * Lx : -1);
                Link<T, C> lk[4];
                links_of<T, C>(A.bonds, s, sl, sd, lk);
                P nb[4] = {cur[k + 2], cur[k], dn[k + 1], up[k + 1]};
                yv = apply_general<T, C>(o, cur[k + 1], nb, lk);
            } else {
                yv = apply_uniform<T, C>(o, th, cur[k + 1], cur[k], cur[k + 2], up[k + 1], dn[k + 1]);
            }
            P pv = first ? zero_pair<T, C>() : ld<T, C>(a2 + s * Bp + b);
            P ov = cheb_combine<T, C>(yv, pv, first);
            st<T, C>(ao + s * Bp + b, ov);
            if (s == my_site) {
                const int64_t m = (int64_t)b * A.N + A.n;
                if constexpr (C) {
                    A.mu_ee[m] = (double)ov.er;
                    A.mu_he[2 * m] = (double)ov.hr;
                    A.mu_he[2 * m + 1] = (double)ov.hi;
                } else {
                    A.mu_ee[m] = (double)ov.e;
                    A.mu_he[m] = (double)ov.h;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < W + 2; ++k) { up[k] = cur[k]; cur[k] = dn[k]; }
    }
}

// a_0 = |s_b, e> for every lane: zero the buffer ...
template <typename T, bool C>
__global__ void k_zero(typename Storage<T, C>::type *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        st<T, C>(p + i, zero_pair<T, C>());
}

// ... then set the unit entries and the zeroth moments.  A start site outside
// the lattice leaves its vector zero and fills its moment row with NaN.
template <typename T, bool C>
__global__ void k_seed(typename Storage<T, C>::type *a0, int64_t Bp, int Bt, int64_t L2,
                       const int32_t *sites, double *mu_ee, double *mu_he, int N)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= Bt) return;
    const int64_t s = sites[b];
    const int64_t m = (int64_t)b * N;
    if (s < 0 || s >= L2) {
        const double nan = __builtin_nan("");
        for (int n = 0; n < N; ++n) {
            mu_ee[m + n] = nan;
            if (C) { mu_he[2 * (m + n)] = nan; mu_he[2 * (m + n) + 1] = nan; }
            else mu_he[m + n] = nan;
        }
        return;
    }
    Pair<T, C> one = zero_pair<T, C>();
    if constexpr (C) one.er = T(1); else one.e = T(1);
    st<T, C>(a0 + s * Bp + b, one);
    mu_ee[m] = 1.0;
    if (C) { mu_he[2 * m] = 0.0; mu_he[2 * m + 1] = 0.0; }
    else mu_he[m] = 0.0;
}

template <typename T, bool C> struct StepShape;
template <> struct StepShape<double, false> { static constexpr int W = 8, YS = 32; };
template <> struct StepShape<float, false> { static constexpr int W = 8, YS = 32; };
template <> struct StepShape<double, true> { static constexpr int W = 4, YS = 32; };
template <> struct StepShape<float, true> { static constexpr int W = 8, YS = 32; };

template <typename T, bool C, bool GEN>
static int launch_step(StepArgs A, hipStream_t st)
{
    constexpr int W = StepShape<T, C>::W, YS = StepShape<T, C>::YS;
    A.n_strips = (int)ceil_div(A.Lx, W);
    A.n_segs = (int)ceil_div(A.Ly, YS);
    const int n_chunks = (int)ceil_div(A.Bt, kBlock);
    const int64_t nb = (int64_t)A.n_strips * A.n_segs * n_chunks;
    if (nb > INT32_MAX) return fail(CBDG_EINVAL, "chebyshev_moments: launch grid too large");
    A.nblocks = (int)nb;
    hipLaunchKernelGGL((k_cheb_step<T, C, GEN, W, YS>), dim3(A.nblocks), dim3(kBlock), 0, st, A);
    CBDG_CHECK_LAUNCH("k_cheb_step");
    return CBDG_OK;
}

template <typename T, bool C>
static int run_moments(const cbdg_op *op, const int32_t *sites, int64_t n_start, int N, int tile,
                       void *ws, double *mu_ee, double *mu_he, hipStream_t st)
{
    using S = typename Storage<T, C>::type;
    const int64_t L2 = op->L2;
    const int64_t Bp_max = round_up(tile, kWave);
    S *bufA = reinterpret_cast<S *>(ws);
    S *bufB = bufA + L2 * Bp_max;
    const void *onsite = std::is_same<T, double>::value ? (const void *)op->onsite64 : (const void *)op->onsite32;
    const void *bonds = std::is_same<T, double>::value ? op->bonds64 : op->bonds32;
    const int he_mult = C ? 2 : 1;
    for (int64_t t0 = 0; t0 < n_start; t0 += tile) {
        const int Bt = (int)std::min<int64_t>(tile, n_start - t0);
        const int64_t Bp = round_up(Bt, kWave);
        double *mee = mu_ee + t0 * N;
        double *mhe = mu_he + t0 * N * he_mult;
        const int32_t *ts = sites + t0;
        const int64_t nz = L2 * Bp;
        hipLaunchKernelGGL((k_zero<T, C>), dim3((unsigned)std::min<int64_t>(ceil_div(nz, kBlock), 8192)),
                           dim3(kBlock), 0, st, bufA, nz);
        CBDG_CHECK_LAUNCH("k_zero");
        hipLaunchKernelGGL((k_seed<T, C>), dim3((unsigned)ceil_div(Bt, kBlock)), dim3(kBlock), 0, st,
                           bufA, Bp, Bt, L2, ts, mee, mhe, N);
        CBDG_CHECK_LAUNCH("k_seed");
        StepArgs A{};
        A.onsite = onsite;
        A.bonds = bonds;
        A.th = op->t / op->bounds.a;
        A.Lx = op->Lx; A.Ly = op->Ly; A.bcx = op->bc_x; A.bcy = op->bc_y;
        A.Bp = (int)Bp; A.Bt = Bt; A.N = N;
        A.sites = ts; A.mu_ee = mee; A.mu_he = mhe;
        S *buf[2] = {bufA, bufB};
        for (int n = 1; n < N; ++n) {
            A.first = n == 1;
            A.n = n;
            A.prev1 = buf[(n - 1) & 1];
            A.prev2 = buf[n & 1];
            A.out = buf[n & 1];
            int rc = op->general ? launch_step<T, C, true>(A, st) : launch_step<T, C, false>(A, st);
            if (rc) return rc;
        }
    }
    return CBDG_OK;
}

static size_t pair_bytes(int scalar, int precision)
{
    const size_t base = precision == CBDG_FP64 ? 8 : 4;
    return base * (scalar == CBDG_COMPLEX ? 4 : 2);
}

__global__ void k_fill_i32(int32_t *p, int32_t v) { *p = v; }

__global__ void k_check(const double *mu_ee, const double *mu_he, int64_t n, int cplx, double lim,
                        int32_t *flag)
{
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double e = mu_ee[i];
        double h;
        if (cplx) h = hypot(mu_he[2 * i], mu_he[2 * i + 1]);
        else h = fabs(mu_he[i]);
        if (!(fabs(e) <= lim) || !(h <= lim)) bad = 1;
    }
    if (bad) atomicOr(flag, 1);
}

}  // namespace cbdg

using namespace cbdg;

extern "C" int cbdg_moments_workspace_size(const cbdg_op *op, int32_t tile, int32_t precision,
                                           size_t *bytes)
{
    clear_error();
    if (!op || !bytes) return fail(CBDG_EINVAL, "moments_workspace_size: op and bytes must not be NULL");
    if (tile < 1) return fail(CBDG_EINVAL, "moments_workspace_size: tile must be >= 1");
    if (precision != CBDG_FP64 && precision != CBDG_FP32_ACC64)
        return fail(CBDG_EINVAL, "moments_workspace_size: unknown precision %d", precision);
    *bytes = 2 * (size_t)op->L2 * (size_t)round_up(tile, kWave) * pair_bytes(op->scalar, precision);
    return CBDG_OK;
}

extern "C" int cbdg_chebyshev_moments(const cbdg_op *op, const int32_t *start_sites, int64_t n_start,
                                      int32_t N, int32_t tile, int32_t precision, void *workspace,
                                      size_t workspace_bytes, double *mu_ee, void *mu_he, void *stream)
{
    clear_error();
    if (!op) return fail(CBDG_EINVAL, "chebyshev_moments: op must not be NULL");
    if (n_start < 0) return fail(CBDG_EINVAL, "chebyshev_moments: n_start must be >= 0");
    if (N < 1) return fail(CBDG_EINVAL, "chebyshev_moments: N must be >= 1");
    if (tile < 1) return fail(CBDG_EINVAL, "chebyshev_moments: tile must be >= 1");
    if (precision != CBDG_FP64 && precision != CBDG_FP32_ACC64)
        return fail(CBDG_EINVAL, "chebyshev_moments: unknown precision %d", precision);
    if (n_start == 0) return CBDG_OK;
    if (!start_sites || !mu_ee || !mu_he || !workspace)
        return fail(CBDG_EINVAL, "chebyshev_moments: start_sites, mu_ee, mu_he and workspace must not be NULL");
    const int64_t eff_tile = std::min<int64_t>(tile, n_start);
    size_t need = 0;
    int rc = cbdg_moments_workspace_size(op, (int32_t)eff_tile, precision, &need);
    if (rc) return rc;
    if (workspace_bytes < need)
        return fail(CBDG_EINVAL, "chebyshev_moments: workspace of %zu bytes is smaller than the %zu needed",
                    workspace_bytes, need);
    hipStream_t st = as_stream(stream);
    double *mhe = reinterpret_cast<double *>(mu_he);
    const bool cplx = op->scalar == CBDG_COMPLEX;
    if (precision == CBDG_FP64)
        return cplx ? run_moments<double, true>(op, start_sites, n_start, N, (int)eff_tile, workspace, mu_ee, mhe, st)
                    : run_moments<double, false>(op, start_sites, n_start, N, (int)eff_tile, workspace, mu_ee, mhe, st);
    return cplx ? run_moments<float, true>(op, start_sites, n_start, N, (int)eff_tile, workspace, mu_ee, mhe, st)
                : run_moments<float, false>(op, start_sites, n_start, N, (int)eff_tile, workspace, mu_ee, mhe, st);
}

extern "C" int cbdg_check_moments(const double *mu_ee, const void *mu_he, int64_t n_rows, int32_t N,
                                  int32_t scalar, double tol, int32_t *flag, void *stream)
{
    clear_error();
    if (!flag) return fail(CBDG_EINVAL, "check_moments: flag must not be NULL");
    if (n_rows < 0 || N < 1) return fail(CBDG_EINVAL, "check_moments: need n_rows >= 0 and N >= 1");
    if (scalar != CBDG_REAL && scalar != CBDG_COMPLEX)
        return fail(CBDG_EINVAL, "check_moments: scalar must be REAL or COMPLEX");
    if (!(tol >= 0.0)) return fail(CBDG_EINVAL, "check_moments: tol must be >= 0");
    hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(1), 0, st, flag, 0);
    CBDG_CHECK_LAUNCH("k_fill_i32");
    const int64_t n = n_rows * (int64_t)N;
    if (n == 0) return CBDG_OK;
    if (!mu_ee || !mu_he) return fail(CBDG_EINVAL, "check_moments: mu_ee and mu_he must not be NULL");
    hipLaunchKernelGGL(k_check, dim3((unsigned)std::min<int64_t>(ceil_div(n, kBlock), 4096)), dim3(kBlock), 0,
                       st, mu_ee, (const double *)mu_he, n, scalar == CBDG_COMPLEX ? 1 : 0, 1.0 + tol, flag);
    CBDG_CHECK_LAUNCH("k_check");
    return CBDG_OK;
}
