// Reverse-mode derivative of the batched recursion (real FP64 operators).
//
// For a loss L = sum_n <w_n, a_n>, where w_n is nonzero only at the start
// site of each vector (w_n = dL/dmu_ee_n |s,e> + dL/dmu_he_n |s,h>), the
// adjoint vectors obey the transposed recursion
//     lam_n = w_n + 2 Ht^T lam_{n+1} - lam_{n+2},   lam_N = lam_{N+1} = 0,
// and the derivative with respect to an operator parameter theta is
//     dL/dtheta = sum_{n>=1} c_n <lam_n, (dHt/dtheta) a_{n-1}>,
// c_1 = 1 (a_1 = Ht a_0 carries no factor 2) and c_n = 2 otherwise.  For a
// real operator Ht^T = Ht, so the adjoint step is the forward stencil.  With
// dHt/deps_j = (|j,e><j,e| - |j,h><j,h|)/a and
// dHt/dDelta_j = (|j,e><j,h| + |j,h><j,e|)/a the per-site terms are
//     g_eps(j)   += c_n/a sum_b [lam(j,e) a(j,e) - lam(j,h) a(j,h)]
//     g_delta(j) += c_n/a sum_b [lam(j,e) a(j,h) + lam(j,h) a(j,e)].
//
// Memory: a_{n-1} is needed in reverse order.  A forward pass stores the
// pairs (a_{jk}, a_{jk+1}) every k steps (k = ceil(sqrt(N)) by default,
// ceil(sqrt(M+1)) under doubling); each segment is recomputed from its pair
// just before the adjoint walks through it.  Per tile, with V = N-1 forward
// vectors (M+1 under doubling): ceil(V/k) checkpoints, as many again when
// k > 1, max(k-2, 2) recomputed vectors and 2 adjoint vectors.
//
// With moment doubling (b = 0) the moments are functions of a_0 .. a_M only,
// M = floor(N/2):  mu_ee[2m] = 2<a_m|a_m> - 1,
// mu_ee[2m-1] = 2<a_m|a_{m-1}> - mu_ee[1],
// mu_he[2m-1] = 2(-1)^m B(a_m, a_{m-1}) - mu_he[1], mu_he[2m] = 0, with
// B(x, y) = sum_i x_e(i) y_h(i) - x_h(i) y_e(i).  Their cotangent on a_m is a
// whole vector,
//   w_m = 4 g_ee[2m] a_m + 2 g_ee[2m+1] a_{m+1} + 2 g_ee[2m-1] a_{m-1}
//       + 2(-1)^{m+1} g_he[2m+1] (-a_{m+1,h}, a_{m+1,e})
//       + 2(-1)^m g_he[2m-1] (a_{m-1,h}, -a_{m-1,e})
// (each term only where its moment index lies in 2..N-1), plus at m = 1 the
// start-site terms of mu_ee[1] and mu_he[1], whose cotangents collect
// g[1] - sum_{m>=2} g[2m-1].  The same transposed recursion then runs over
// m = M .. 1 only: half the forward and adjoint steps, at the price of one
// more vector read per adjoint step (a_m, with the halo of its strip:
// a_{m+1} is formed in registers as 2 Ht a_m - a_{m-1}).
//
// The forward pass and the segment recomputations take two recursion steps
// per launch where the operator allows it (the forward moments' two-step
// pass), so a stored or recomputed a_m moves through HBM as in the forward
// moments.
//
// The sum over the tile's vectors is a wavefront reduction per site; each
// (64-vector chunk, site) partial is owned by one wavefront, accumulated over
// n without atomics and summed over chunks in a fixed order, so results are
// bitwise reproducible.
#include "step.hpp"

#include <algorithm>
#include <cmath>

namespace cbdg {

struct AdjArgs {
    const void *lam1;    // lam_{n+1} (HAS1)
    const void *lam2;    // lam_{n+2} (HAS2)
    void *out;           // lam_n (aliases lam2 when HAS2)
    const void *aprev;   // a_{n-1}
    double th;           // t/a
    int Lx, Ly, bcx, bcy;
    int Bp, Bt;
    int n, N;
    const int32_t *sites;   // tile's start sites
    const double *dmu_ee;   // tile rows, or null
    const double *dmu_he;   // tile rows, or null
    double cscale;          // c_n / a
    double *gpart;          // [Bp/64][L2][2]
    int64_t L2;
    int n_strips, n_segs, nblocks;
    int ys;               // rows per segment
    const void *acur;     // a_m (doubling)
    const double *d1;     // [Bt][2] start-site cotangents of mu_ee[1], mu_he[1] (doubling)
};

// Cotangent coefficients of one doubling step m for one vector:
//   w_m = cA a_m + cP a_{m+1} + cQ (-a_{m+1,h}, a_{m+1,e})
//       + cR a_{m-1} + cS (a_{m-1,h}, -a_{m-1,e}) + (we, wh) at the start site
struct AdjCoef { double cA, cP, cQ, cR, cS, we, wh; };

__device__ __forceinline__ AdjCoef adj_coef(const AdjArgs &A, int m, uint32_t b, bool active)
{
    AdjCoef c{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int N = A.N;
    const int64_t row = (int64_t)b * N;
    auto gee = [&](int i) { return (active && A.dmu_ee && i >= 2 && i < N) ? A.dmu_ee[row + i] : 0.0; };
    auto ghe = [&](int i) { return (active && A.dmu_he && i >= 2 && i < N) ? A.dmu_he[row + i] : 0.0; };
    const double sg = (m & 1) ? -2.0 : 2.0;  // 2(-1)^m
    c.cA = 4.0 * gee(2 * m);
    c.cP = 2.0 * gee(2 * m + 1);
    c.cQ = -sg * ghe(2 * m + 1);
    if (m >= 2) { c.cR = 2.0 * gee(2 * m - 1); c.cS = sg * ghe(2 * m - 1); }
    if (m == 1 && active) { c.we = A.d1[2 * b]; c.wh = A.d1[2 * b + 1]; }
    return c;
}

// lam_n at one site from hl = (Ht lam_{n+1})(s), l2 = lam_{n+2}(s), the forward
// vectors mk = a_n(s), ac = a_{n-1}(s), q = a_{n+1}(s) and the cotangent
// (direct form: we, wh only).  The multiply-adds are written out and no other
// contraction is allowed, so a site's rounding is fixed by this function and
// not by how the compiler schedules the kernel around it.
template <bool HAS1, bool HAS2, bool DBL, bool NXT>
__device__ __forceinline__ Pair<double, false> adj_site(const Pair<double, false> &hl, const Pair<double, false> &l2,
                                                        const Pair<double, false> &mk, const Pair<double, false> &ac,
                                                        const Pair<double, false> &q, const AdjCoef &c, bool hit)
{
#pragma clang fp contract(off)
    Pair<double, false> lam{0.0, 0.0};
    if constexpr (HAS1) { lam.e = 2.0 * hl.e; lam.h = 2.0 * hl.h; }
    if constexpr (HAS2) { lam.e = lam.e - l2.e; lam.h = lam.h - l2.h; }
    if constexpr (DBL) {
        lam.e = lam.e + __builtin_fma(c.cA, mk.e, __builtin_fma(c.cR, ac.e, c.cS * ac.h));
        lam.h = lam.h + __builtin_fma(c.cA, mk.h, __builtin_fma(c.cR, ac.h, -(c.cS * ac.e)));
    }
    if constexpr (NXT) {
        lam.e = lam.e + __builtin_fma(c.cP, q.e, -(c.cQ * q.h));
        lam.h = lam.h + __builtin_fma(c.cP, q.h, c.cQ * q.e);
    }
    lam.e = lam.e + (hit ? c.we : 0.0);
    lam.h = lam.h + (hit ? c.wh : 0.0);
    return lam;
}

// The lane's terms of dL/deps and dL/dDelta at one site: lam_n . dHt a_{n-1}.
__device__ __forceinline__ void adj_grad_terms(const Pair<double, false> &lam, const Pair<double, false> &ac, bool active,
                                               double &ge, double &gd)
{
#pragma clang fp contract(off)
    ge = active ? __builtin_fma(lam.e, ac.e, -(lam.h * ac.h)) : 0.0;
    gd = active ? __builtin_fma(lam.e, ac.h, lam.h * ac.e) : 0.0;
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <bool HAS1, bool HAS2, int W, bool DBL, bool NXT>
__global__ __launch_bounds__(kBlock) void k_adj_step(AdjArgs A, const double2 *__restrict__ lam1,
                                                     const OnSite<double> *__restrict__ ons,
                                                     const double2 *__restrict__ aprev)
{
    using P = Pair<double, false>;
    using S = double2;
    const int lb = xcd_remap(blockIdx.x, A.nblocks);
    const int strip = lb % A.n_strips;
    const int rest = lb / A.n_strips;
    const int seg = rest % A.n_segs;
    const int chunk = rest / A.n_segs;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int wave_base = chunk * kBlock + wave * kWave;
    // whole wavefronts beyond the tile leave; partially filled ones stay for
    // the reductions, their spare lanes contribute zero
    if (wave_base >= A.Bt) return;
    const uint32_t b = wave_base + lane;
    const bool active = b < (uint32_t)A.Bt;
    const int c64 = wave_base / kWave;

    const int Lx = A.Lx, Ly = A.Ly;
    const int x0 = strip * W;
    const int y0 = seg * A.ys;
    const int y1 = min(y0 + A.ys, Ly);
    const int64_t Bp = A.Bp;
    const S *l2 = reinterpret_cast<const S *>(A.lam2);
    S *lo = reinterpret_cast<S *>(A.out);
    const double th = A.th;
    const int my_site = active ? A.sites[b] : -1;
    AdjCoef cf{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (DBL) {
        cf = adj_coef(A, A.n, b, active);
    } else {
        cf.we = (active && A.dmu_ee) ? A.dmu_ee[(int64_t)b * A.N + A.n] : 0.0;
        cf.wh = (active && A.dmu_he) ? A.dmu_he[(int64_t)b * A.N + A.n] : 0.0;
    }
    const S *am = reinterpret_cast<const S *>(A.acur);
    double *gp = A.gpart + (int64_t)c64 * A.L2 * 2;

    int cx[W + 2];
    uint32_t cm[W + 2];
#pragma unroll
    for (int k = 0; k < W + 2; ++k) {
        const int x = x0 - 1 + k;
        bool ok;
        if (x < 0) { ok = A.bcx != 0; cx[k] = A.bcx ? x + Lx : 0; }
        else if (x >= Lx) { ok = A.bcx && x == Lx; cx[k] = ok ? 0 : Lx - 1; }
        else { ok = true; cx[k] = x; }
        cm[k] = ok ? ~0u : 0u;
    }
    auto load_row = [&](const S *base_ptr, P *row, int y) -> uint32_t {
        bool ok = true;
        int yy = y;
        if (y < 0) { ok = A.bcy != 0; yy = A.bcy ? y + Ly : 0; }
        else if (y >= Ly) { ok = A.bcy != 0; yy = A.bcy ? y - Ly : Ly - 1; }
        const int64_t rbase = (int64_t)yy * Lx;
#pragma unroll
        for (int k = 0; k < W + 2; ++k) row[k] = ld<double, false>(base_ptr + (rbase + cx[k]) * Bp + b);
        return ok ? ~0u : 0u;
    };
    auto apply_mask = [&](P *row, uint32_t rm) {
#pragma unroll
        for (int k = 0; k < W + 2; ++k) row[k] = masked<double, false>(row[k], rm & cm[k]);
    };
    auto load_own = [&](const S *base_ptr, P *row, int y, bool nt) {
        const int64_t rbase = (int64_t)y * Lx;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const S *q = base_ptr + (rbase + x0 + k) * Bp + b;
            row[k] = nt ? ld_nt<double, false>(q) : ld<double, false>(q);
        }
    };

    // lam_{n+1} rows y-1 .. y+2; under doubling also a_n rows y-1 .. y+2,
    // from which a_{n+1} = 2 Ht a_n - a_{n-1} is formed in registers exactly
    // as the forward step formed it
    constexpr int WM = DBL ? W + 2 : 1;
    P up[W + 2], cur[W + 2], dn[W + 2], nx[W + 2];
    P pc[W], pn[W], ac[W], an[W];
    [[maybe_unused]] P mup[WM], mcur[WM], mdn[WM], mnx[WM];
    if constexpr (HAS1) {
        apply_mask(up, load_row(lam1, up, y0 - 1));
        apply_mask(cur, load_row(lam1, cur, y0));
        apply_mask(dn, load_row(lam1, dn, y0 + 1));
    }
    if constexpr (DBL) {
        apply_mask(mup, load_row(am, mup, y0 - 1));
        apply_mask(mcur, load_row(am, mcur, y0));
        apply_mask(mdn, load_row(am, mdn, y0 + 1));
    }
    if constexpr (HAS2) load_own(l2, pc, y0, true);
    load_own(aprev, ac, y0, true);

    // The (chunk, site) gradient partials of row y, read before the trip's
    // prefetch loads: the loads complete in issue order, so reading them
    // where they are updated would wait for the prefetch of the next rows.
    double gold[W][2];
    auto load_grad = [&](int y) {
        if (lane == 0) {
            const int64_t srow = (int64_t)y * Lx;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                gold[k][0] = gp[2 * (srow + x0 + k)];
                gold[k][1] = gp[2 * (srow + x0 + k) + 1];
            }
        }
    };
    auto compute_row = [&](int y) {
        const int64_t srow = (int64_t)y * Lx;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int64_t s = srow + x0 + k;
            [[maybe_unused]] OnSite<double> o;
            if constexpr (HAS1 || NXT) o = ons[s];
            P hl = zero_pair<double, false>(), q = zero_pair<double, false>();
            if constexpr (HAS1) hl = apply_uniform<double, false>(o, th, cur[k + 1], cur[k], cur[k + 2], up[k + 1], dn[k + 1]);
            if constexpr (NXT) {
                const P yq = apply_uniform<double, false>(o, th, mcur[k + 1], mcur[k], mcur[k + 2], mup[k + 1], mdn[k + 1]);
                q = cheb_combine<double, false>(yq, ac[k], false);
            }
            [[maybe_unused]] const P mk = DBL ? mcur[k + 1] : zero_pair<double, false>();
            const P lam = adj_site<HAS1, HAS2, DBL, NXT>(hl, HAS2 ? pc[k] : zero_pair<double, false>(), mk, ac[k], q,
                                                         cf, s == my_site);
            st_nt<double, false>(lo + s * Bp + b, lam);
            double ge, gd;
            adj_grad_terms(lam, ac[k], active, ge, gd);
            ge = wave_sum_f64(ge);
            gd = wave_sum_f64(gd);
            if (lane == 0) {
                gp[2 * s] = __builtin_fma(A.cscale, ge, gold[k][0]);
                gp[2 * s + 1] = __builtin_fma(A.cscale, gd, gold[k][1]);
            }
        }
    };

    // one row per trip: unrolling would duplicate the register window
#pragma unroll 1
    for (int y = y0; y < y1 - 1; ++y) {
        uint32_t nm = 0, mm = 0;
        load_grad(y);
        if constexpr (HAS1) nm = load_row(lam1, nx, y + 2);
        if constexpr (DBL) mm = load_row(am, mnx, y + 2);
        if constexpr (HAS2) load_own(l2, pn, y + 1, true);
        load_own(aprev, an, y + 1, true);
        compute_row(y);
        if constexpr (HAS1) {
            apply_mask(nx, nm);
#pragma unroll
            for (int k = 0; k < W + 2; ++k) { up[k] = cur[k]; cur[k] = dn[k]; dn[k] = nx[k]; }
        }
        if constexpr (DBL) {
            apply_mask(mnx, mm);
#pragma unroll
            for (int k = 0; k < W + 2; ++k) { mup[k] = mcur[k]; mcur[k] = mdn[k]; mdn[k] = mnx[k]; }
        }
#pragma unroll
        for (int k = 0; k < W; ++k) { pc[k] = pn[k]; ac[k] = an[k]; }
    }
    load_grad(y1 - 1);
    compute_row(y1 - 1);
}

// Start-site cotangents of mu_ee[1] and mu_he[1] under doubling: every odd
// moment 2m-1 >= 3 subtracts mu[1], so d1 = g[1] - sum_{m=2..M} g[2m-1].
__global__ void k_adj_d1(const double *dmu_ee, const double *dmu_he, int Bt, int N, double *d1)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= Bt) return;
    const int64_t row = (int64_t)b * N;
    double e = 0.0, h = 0.0;
    for (int i = 3; i < N; i += 2) {
        if (dmu_ee) e += dmu_ee[row + i];
        if (dmu_he) h += dmu_he[row + i];
    }
    d1[2 * b] = (dmu_ee && N > 1 ? dmu_ee[row + 1] : 0.0) - e;
    d1[2 * b + 1] = (dmu_he && N > 1 ? dmu_he[row + 1] : 0.0) - h;
}

__global__ void k_fill_f64(double *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// grad[j] += sum over chunks (in chunk order) of the partials of site j
__global__ void k_grad_reduce(const double *gpart, int nchunk, int64_t L2, double *grad_eps, double *grad_delta)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < L2; j += (int64_t)gridDim.x * blockDim.x) {
        double ge = 0.0, gd = 0.0;
        for (int c = 0; c < nchunk; ++c) {
            ge += gpart[(c * L2 + j) * 2];
            gd += gpart[(c * L2 + j) * 2 + 1];
        }
        if (grad_eps) grad_eps[j] += ge;
        if (grad_delta) grad_delta[j] += gd;
    }
}

#ifndef CBDG_ADJ_YS
#define CBDG_ADJ_YS 64
#endif
#ifndef CBDG_ADJ_TGT
#define CBDG_ADJ_TGT 2048
#endif
constexpr int kAdjW = 4, kAdjYS = CBDG_ADJ_YS;

template <bool HAS1, bool HAS2, int W, bool DBL, bool NXT>
static int launch_adj_w(AdjArgs A, const OnSite<double> *ons, hipStream_t st)
{
    A.n_strips = A.Lx / W;
    const int n_chunks = (int)ceil_div(A.Bt, kBlock);
    A.ys = kAdjYS;
    while (A.ys > 8 && (int64_t)A.n_strips * n_chunks * ceil_div(A.Ly, A.ys) < CBDG_ADJ_TGT) A.ys /= 2;
    A.n_segs = (int)ceil_div(A.Ly, A.ys);
    const int64_t nb = (int64_t)A.n_strips * A.n_segs * n_chunks;
    if (nb > INT32_MAX) return fail(CBDG_EINVAL, "chebyshev_moments_backward: launch grid too large");
    A.nblocks = (int)nb;
    hipLaunchKernelGGL((k_adj_step<HAS1, HAS2, W, DBL, NXT>), dim3(A.nblocks), dim3(kBlock), 0, st, A,
                       reinterpret_cast<const double2 *>(A.lam1), ons, reinterpret_cast<const double2 *>(A.aprev));
    CBDG_CHECK_LAUNCH("k_adj_step");
    return CBDG_OK;
}

// Strip width of the doubling-form adjoint step (three more register rows
// than the direct form).  128x128, N = 512, 4 tiles of 1024 on MI355X:
// W = 2 511 ms, W = 1 510 ms, W = 4 561 ms (256 VGPRs, one wave per SIMD).
#ifndef CBDG_ADJ_W_DBL
#define CBDG_ADJ_W_DBL 2
#endif

template <bool HAS1, bool HAS2, bool DBL, bool NXT>
static int launch_adj_d(AdjArgs A, const OnSite<double> *ons, hipStream_t st)
{
    constexpr int WB = DBL ? CBDG_ADJ_W_DBL : kAdjW;
    if (A.Lx % WB == 0) return launch_adj_w<HAS1, HAS2, WB, DBL, NXT>(A, ons, st);
    if (A.Lx % 2 == 0) return launch_adj_w<HAS1, HAS2, 2, DBL, NXT>(A, ons, st);
    return launch_adj_w<HAS1, HAS2, 1, DBL, NXT>(A, ons, st);
}

// nxt: the doubling cotangent has a_{n+1} terms (moment 2n+1 <= N-1)
template <bool HAS1, bool HAS2>
static int launch_adj(AdjArgs A, const OnSite<double> *ons, bool dbl, bool nxt, hipStream_t st)
{
    if (!dbl) return launch_adj_d<HAS1, HAS2, false, false>(A, ons, st);
    if (nxt) return launch_adj_d<HAS1, HAS2, true, true>(A, ons, st);
    return launch_adj_d<HAS1, HAS2, true, false>(A, ons, st);
}

struct Plan {
    bool dbl;        // doubling form
    int top;         // last forward vector the adjoint reads: N-2 (direct), M (doubling)
    int mtop;        // first adjoint index: N-1 (direct), M (doubling)
    int k;           // checkpoint stride
    int J;           // segments
    int J1;          // second checkpoint of each pair: J slots, none when k = 1
    int nscratch;    // segment / scratch vectors
    int64_t Bp;      // lane stride for the widest tile
};

// Checkpoint stride k = ceil(sqrt(N)) (direct) or ceil(sqrt(M + 1))
// (doubling), rounded up to a multiple of 3, unless given: three-step passes
// from a_2 on write the pairs (a_{3m}, a_{3m+1}), which then include every
// checkpoint pair (a_{jk}, a_{jk+1}).
static Plan make_plan(int N, int tile, int ckpt_stride, bool dbl)
{
    Plan p;
    p.dbl = dbl;
    p.top = dbl ? N / 2 : std::max(N - 2, 0);
    p.mtop = dbl ? N / 2 : N - 1;
    const int nvec = p.top + 1;
    const int kdef = 3 * (int)ceil_div((int64_t)std::ceil(std::sqrt((double)(dbl ? nvec : N))), 3);
    p.k = ckpt_stride > 0 ? ckpt_stride : std::max(1, kdef);
    p.J = (int)ceil_div(nvec, p.k);
    p.J1 = p.k > 1 ? p.J : 0;
    p.nscratch = std::max(p.k - 2, 2);
    p.Bp = lane_stride(tile);
    return p;
}

// Workspace of the reverse passes without checkpoints: the moments
// workspace of one tile (its four buffers hold the regenerated a_m), four
// cotangent buffers, the per-vector gradient terms G, the forward's moment
// rows (not returned) and the start-site cotangents, each region aligned to
// 256 bytes.
struct RevLayout { size_t moments, cbuf, G, mu, d1, total; };
static int rev_layout(const cbdg_op *op, int tile, int N, RevLayout *L)
{
    size_t mws = 0;
    int rc = cbdg_moments_workspace_size(op, tile, CBDG_FP64, CBDG_ALG_DOUBLING, &mws);
    if (rc) return rc;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t vec = (size_t)op->L2 * (size_t)tile * sizeof(double2);
    L->moments = 0;
    L->cbuf = al(mws);
    L->G = L->cbuf + 4 * al(vec);
    L->mu = L->G + al(vec);
    L->d1 = L->mu + al((size_t)2 * tile * N * sizeof(double));
    L->total = L->d1 + al((size_t)2 * tile * sizeof(double));
    return CBDG_OK;
}

static size_t plan_bytes(const Plan &p, int64_t L2)
{
    const size_t vec = (size_t)L2 * (size_t)p.Bp * sizeof(double2);
    const size_t gpart = (size_t)(p.Bp / kWave) * (size_t)L2 * 2 * sizeof(double);
    const size_t d1 = p.dbl ? (size_t)p.Bp * 2 * sizeof(double) : 0;
    return (size_t)(p.J + p.J1 + p.nscratch + 2) * vec + gpart + d1;
}

}  // namespace cbdg

using namespace cbdg;

static int check_backward_op(const cbdg_op *op, const char *who)
{
    if (!op) return fail(CBDG_EINVAL, "%s: op must not be NULL", who);
    if (op->scalar != CBDG_REAL || op->general)
        return fail(CBDG_EUNSUPPORTED, "%s: the adjoint is implemented for real operators with uniform "
                    "hopping and on-site pairing only", who);
    return CBDG_OK;
}

// Resolves the algorithm of the backward pass (the forward's enum): doubling
// needs b == 0; N <= 2 always takes the direct form.
static int backward_algorithm(const cbdg_op *op, int32_t algorithm, int32_t N, const char *who, bool *dbl)
{
    const bool centred = op->bounds.b == 0.0;
    switch (algorithm) {
    case CBDG_ALG_AUTO: *dbl = centred && N >= 3; return CBDG_OK;
    case CBDG_ALG_DIRECT: *dbl = false; return CBDG_OK;
    case CBDG_ALG_DOUBLING:
        if (!centred) return fail(CBDG_EINVAL, "%s: moment doubling needs a spectrum centred at b = 0 (b = %g)", who, op->bounds.b);
        *dbl = N >= 3;
        return CBDG_OK;
    default: return fail(CBDG_EINVAL, "%s: unknown algorithm %d", who, algorithm);
    }
}

// The reverse passes without checkpoints, tile by tile: the forward moments
// in the vector-contiguous passes and one step more leave (a_{M+1}, a_M);
// full reverse passes of K levels then walk m = M .. down, the last (shorter)
// pass ending at m = 1; the gradient terms of the tile's vectors are summed
// into grad_eps and grad_delta.
// With ld > 0 the terms of each start vector are written as its own row
// (row_eps/row_delta + (start index) * ld) instead of summed into grad_*.
static int backward_reversible(const cbdg_op *op, const int32_t *start_sites, int64_t n_start, int32_t N, int tile,
                               const double *dmu_ee, const double *dmu_he, void *workspace, size_t workspace_bytes,
                               double *grad_eps, double *grad_delta, hipStream_t st, double *row_eps = nullptr,
                               double *row_delta = nullptr, int64_t ld = 0)
{
    RevLayout R;
    int rc = rev_layout(op, tile, N, &R);
    if (rc) return rc;
    if (workspace_bytes < R.total)
        return fail(CBDG_EINVAL, "chebyshev_moments_backward: workspace of %zu bytes is smaller than the %zu needed",
                    workspace_bytes, R.total);
    char *base = reinterpret_cast<char *>(workspace);
    const int64_t L2 = op->L2;
    const size_t vec = ((size_t)L2 * (size_t)tile * sizeof(double2) + 255) / 256 * 256;
    void *cb[4];
    for (int i = 0; i < 4; ++i) cb[i] = base + R.cbuf + i * vec;
    double *G = reinterpret_cast<double *>(base + R.G);
    double *mu = reinterpret_cast<double *>(base + R.mu);
    double *d1 = reinterpret_cast<double *>(base + R.d1);
    const int M = N / 2, K = vc_adj_steps(op->Lx);
    for (int64_t t0 = 0; t0 < n_start; t0 += tile) {
        const int Bt = (int)std::min<int64_t>(tile, n_start - t0);
        const int32_t *ts = start_sites + t0;
        const double *tee = dmu_ee ? dmu_ee + t0 * N : nullptr;
        const double *the = dmu_he ? dmu_he + t0 * N : nullptr;
        void *last[2], *spare[2];
        const void *coef = nullptr;
        if ((rc = vc_forward_last(op, ts, Bt, N, base + R.moments, mu, mu + (int64_t)Bt * N, st, last, spare, &coef)))
            return rc;
        hipLaunchKernelGGL(k_adj_d1, dim3((unsigned)ceil_div(Bt, kBlock)), dim3(kBlock), 0, st, tee, the, Bt, N, d1);
        CBDG_CHECK_LAUNCH("k_adj_d1");
        VcAdjArgs A{};
        A.G = G;
        A.coef = coef;
        A.th = op->t / op->bounds.a;
        A.Lx = op->Lx; A.Ly = op->Ly; A.bcx = op->bc_x; A.bcy = op->bc_y;
        A.Dv = L2; A.Bt = Bt; A.N = N;
        A.n_segs = vc_segments(op->Ly, Bt, K);
        A.sites = ts; A.dmu_ee = tee; A.dmu_he = the; A.d1 = d1;
        // a_{m0+1}, a_{m0} in b[0], b[1]; lam_{m0+2}, lam_{m0+1} in c[0], c[1]
        void *b[4] = {last[0], last[1], spare[0], spare[1]};
        void *c[4] = {cb[0], cb[1], cb[2], cb[3]};
        int m0 = M;
        bool first = true;
        while (m0 >= 1) {
            const bool full = m0 >= K;
            A.m0 = m0;
            A.nlev = full ? K : m0;
            A.first = first ? 1 : 0;
            A.b0 = b[0]; A.b1 = b[1]; A.bo1 = b[2]; A.bo2 = b[3];
            A.c0 = c[0]; A.c1 = c[1]; A.co1 = c[2]; A.co2 = c[3];
            if ((rc = launch_vc_adj(A, full, st))) return rc;
            std::swap(b[0], b[2]); std::swap(b[1], b[3]);
            std::swap(c[0], c[2]); std::swap(c[1], c[3]);
            first = false;
            m0 -= A.nlev;
        }
        if (ld > 0) {
            rc = launch_vc_grad_rows(G, ts, Bt, L2, op->Lx, L2, 1.0 / op->bounds.a, row_eps ? row_eps + t0 * ld : nullptr,
                                     row_delta ? row_delta + t0 * ld : nullptr, ld, st);
        } else {
            rc = launch_vc_grad_reduce(G, ts, Bt, L2, op->Lx, L2, 1.0 / op->bounds.a, grad_eps, grad_delta, st);
        }
        if (rc) return rc;
    }
    return CBDG_OK;
}

extern "C" int cbdg_backward_workspace_size(const cbdg_op *op, int32_t tile, int32_t N, int32_t ckpt_stride,
                                            int32_t algorithm, size_t *bytes)
{
    clear_error();
    int rc = check_backward_op(op, "backward_workspace_size");
    if (rc) return rc;
    if (!bytes || tile < 1 || N < 1 || ckpt_stride < -1)
        return fail(CBDG_EINVAL, "backward_workspace_size: need bytes, tile >= 1, N >= 1, ckpt_stride >= -1");
    bool dbl = false;
    rc = backward_algorithm(op, algorithm, N, "backward_workspace_size", &dbl);
    if (rc) return rc;
    if (ckpt_stride == -1) {
        if (!dbl || !vc_adjoint_supported(op))
            return fail(CBDG_EUNSUPPORTED, "backward_workspace_size: the reverse passes without checkpoints need "
                        "moment doubling on a real operator with uniform hopping and Lx = 64 W (W = 1, 2, 4)");
        RevLayout R;
        if ((rc = rev_layout(op, tile, N, &R))) return rc;
        *bytes = R.total;
        return CBDG_OK;
    }
    *bytes = plan_bytes(make_plan(N, tile, ckpt_stride, dbl), op->L2);
    return CBDG_OK;
}

extern "C" int cbdg_chebyshev_moments_backward(const cbdg_op *op, const int32_t *start_sites,
                                               int64_t n_start, int32_t N, int32_t tile,
                                               int32_t ckpt_stride, int32_t algorithm,
                                               const double *dmu_ee, const double *dmu_he, void *workspace,
                                               size_t workspace_bytes, double *grad_eps,
                                               double *grad_delta, void *stream)
{
    clear_error();
    int rc = check_backward_op(op, "chebyshev_moments_backward");
    if (rc) return rc;
    if (n_start < 0 || N < 1 || tile < 1 || ckpt_stride < -1)
        return fail(CBDG_EINVAL, "chebyshev_moments_backward: need n_start >= 0, N >= 1, tile >= 1, ckpt_stride >= -1");
    bool dbl = false;
    rc = backward_algorithm(op, algorithm, N, "chebyshev_moments_backward", &dbl);
    if (rc) return rc;
    if (ckpt_stride == -1 && (!dbl || !vc_adjoint_supported(op)))
        return fail(CBDG_EUNSUPPORTED, "chebyshev_moments_backward: the reverse passes without checkpoints need "
                    "moment doubling on a real operator with uniform hopping and Lx = 64 W (W = 1, 2, 4)");
    if (n_start == 0 || N == 1 || (!dmu_ee && !dmu_he)) return CBDG_OK;  // nothing depends on eps or Delta
    if (!start_sites || !workspace || (!grad_eps && !grad_delta))
        return fail(CBDG_EINVAL, "chebyshev_moments_backward: start_sites, workspace and a gradient output are required");
    const int eff_tile = (int)std::min<int64_t>(tile, n_start);
    if (ckpt_stride == -1)
        return backward_reversible(op, start_sites, n_start, N, eff_tile, dmu_ee, dmu_he, workspace, workspace_bytes,
                                   grad_eps, grad_delta, as_stream(stream));
    const Plan plan = make_plan(N, eff_tile, ckpt_stride, dbl);
    const size_t need = plan_bytes(plan, op->L2);
    if (workspace_bytes < need)
        return fail(CBDG_EINVAL, "chebyshev_moments_backward: workspace of %zu bytes is smaller than the %zu needed",
                    workspace_bytes, need);
    hipStream_t st = as_stream(stream);
    const int64_t L2 = op->L2;
    const int64_t vec = L2 * plan.Bp;  // pairs per vector slot
    double2 *base = reinterpret_cast<double2 *>(workspace);
    auto C0 = [&](int j) { return base + (int64_t)j * vec; };
    auto C1 = [&](int j) { return base + (int64_t)(plan.J + j) * vec; };
    auto SC = [&](int i) { return base + (int64_t)(plan.J + plan.J1 + i) * vec; };
    double2 *LA = base + (int64_t)(plan.J + plan.J1 + plan.nscratch) * vec;
    double2 *LB = LA + vec;
    double *gpart = reinterpret_cast<double *>(LB + vec);
    double *d1 = gpart + (plan.Bp / kWave) * L2 * 2;
    const int k = plan.k;
    const int top = plan.top, mtop = plan.mtop;
    const bool two = two_step_f64_real(op);

    for (int64_t t0 = 0; t0 < n_start; t0 += eff_tile) {
        const int Bt = (int)std::min<int64_t>(eff_tile, n_start - t0);
        const int64_t Bp = lane_stride(Bt);
        const int nchunk = (int)(Bp / kWave);
        const int32_t *ts = start_sites + t0;
        const double *tee = dmu_ee ? dmu_ee + t0 * N : nullptr;
        const double *the = dmu_he ? dmu_he + t0 * N : nullptr;

        // forward: a_0 .. a_top, keeping the checkpoint pairs
        rc = seed_tile_f64_real(C0(0), L2, Bt, ts, nullptr, nullptr, N, st);
        if (rc) return rc;
        StepArgs S{};
        S.th = op->t / op->bounds.a;
        S.Lx = op->Lx; S.Ly = op->Ly; S.bcx = op->bc_x; S.bcy = op->bc_y;
        S.Bp = (int)Bp; S.Bt = Bt; S.N = N; S.sites = ts; S.mu_ee = nullptr; S.mu_he = nullptr;
        // a_n goes to its checkpoint slot, else to one of four rotating
        // buffers (two scratch slots and the adjoint vectors, free until the
        // backward walk) that is neither input of its step nor the other
        // output of a two-step pass
        double2 *const pool[4] = {SC(0), SC(1), LA, LB};
        auto dest_of = [&](int n, const double2 *x, const double2 *y, const double2 *z) -> double2 * {
            if (n % k == 0) return C0(n / k);
            if (k > 1 && n % k == 1) return C1(n / k);
            for (double2 *q : pool)
                if (q != x && q != y && q != z) return q;
            return nullptr;
        };
        const double2 *p2 = nullptr, *p1 = C0(0);
        // three-step passes store a_{n+1}, a_{n+2} only; with k a multiple of 3
        // and the passes starting at n = 2 every checkpoint is among them
        const bool three = k % 3 == 0 && three_step_f64_real(op, Bt);
        for (int n = 1; n <= top;) {
            if (three && n >= 2 && n + 2 <= top) {
                double2 *d1 = dest_of(n + 1, p1, p2, nullptr);
                double2 *d2 = dest_of(n + 2, p1, p2, d1);
                S.first = 0;
                S.n = n;
                S.prev1 = p1;
                S.prev2 = p2;
                S.out = d1;
                S.out2 = d2;
                rc = run_step3_f64_real(op, S, st);
                if (rc) return rc;
                p2 = d1;
                p1 = d2;
                n += 3;
                continue;
            }
            if (two && n >= 2 && n + 1 <= top) {
                double2 *d0 = dest_of(n, p1, p2, nullptr);
                double2 *d1 = dest_of(n + 1, p1, p2, d0);
                S.first = 0;
                S.n = n;
                S.prev1 = p1;
                S.prev2 = p2;
                S.out = d0;
                S.out2 = d1;
                rc = run_step2_f64_real(op, S, st);
                if (rc) return rc;
                p2 = d0;
                p1 = d1;
                n += 2;
                continue;
            }
            double2 *dest = dest_of(n, p1, nullptr, nullptr);
            S.first = n == 1;
            S.n = n;
            S.prev1 = p1;
            S.prev2 = p2 ? p2 : p1;
            S.out = dest;
            rc = run_step(op, CBDG_FP64, S, st);
            if (rc) return rc;
            p2 = p1;
            p1 = dest;
            ++n;
        }

        // backward over the segments in reverse
        const int64_t ng = (int64_t)nchunk * L2 * 2;
        hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)std::min<int64_t>(ceil_div(ng, kBlock), 4096)), dim3(kBlock), 0,
                           st, gpart, ng);
        CBDG_CHECK_LAUNCH("k_fill_f64");
        if (dbl) {
            hipLaunchKernelGGL(k_adj_d1, dim3((unsigned)ceil_div(Bt, kBlock)), dim3(kBlock), 0, st, tee, the, Bt, N, d1);
            CBDG_CHECK_LAUNCH("k_adj_d1");
        }
        AdjArgs A{};
        A.th = op->t / op->bounds.a;
        A.Lx = op->Lx; A.Ly = op->Ly; A.bcx = op->bc_x; A.bcy = op->bc_y;
        A.Bp = (int)Bp; A.Bt = Bt; A.N = N; A.sites = ts; A.dmu_ee = tee; A.dmu_he = the;
        A.gpart = gpart; A.L2 = L2; A.d1 = d1;
        auto lam = [&](int n) { return ((mtop - n) % 2 == 0) ? LA : LB; };
        for (int j = plan.J - 1; j >= 0; --j) {
            const int s0 = j * k, e0 = std::min(s0 + k - 1, top);
            // forward vector m: recomputed scratch inside this segment, else a
            // checkpoint (the adjoint of the doubling form also reads a_{e0+1},
            // the first vector of the next segment's pair)
            auto vec_of = [&](int m) -> const double2 * {
                if (m % k == 0) return C0(m / k);
                if (k > 1 && m % k == 1) return C1(m / k);
                return SC(m - s0 - 2);
            };
            // a_{s0+2} .. a_{e0} (none a checkpoint), two at a time
            for (int m = s0 + 2; m <= e0;) {
                S.first = 0;
                S.n = m;
                S.prev1 = vec_of(m - 1);
                S.prev2 = vec_of(m - 2);
                S.out = SC(m - s0 - 2);
                if (two && m + 1 <= e0) {
                    S.out2 = SC(m - s0 - 1);
                    rc = run_step2_f64_real(op, S, st);
                    m += 2;
                } else {
                    rc = run_step(op, CBDG_FP64, S, st);
                    ++m;
                }
                if (rc) return rc;
            }
            for (int n = std::min(e0 + 1, mtop); n >= s0 + 1; --n) {
                const bool has1 = n + 1 <= mtop, has2 = n + 2 <= mtop;
                A.n = n;
                A.lam1 = has1 ? lam(n + 1) : nullptr;
                A.lam2 = has2 ? lam(n + 2) : nullptr;
                A.out = lam(n);
                A.aprev = vec_of(n - 1);
                A.acur = dbl ? vec_of(n) : nullptr;
                A.cscale = (n == 1 ? 1.0 : 2.0) / op->bounds.a;
                const OnSite<double> *ons = op->onsite64;
                const bool nxt = dbl && 2 * n + 1 <= N - 1;
                if (has1 && has2) rc = launch_adj<true, true>(A, ons, dbl, nxt, st);
                else if (has1) rc = launch_adj<true, false>(A, ons, dbl, nxt, st);
                else rc = launch_adj<false, false>(A, ons, dbl, nxt, st);
                if (rc) return rc;
            }
        }
        hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)std::min<int64_t>(ceil_div(L2, kBlock), 4096)), dim3(kBlock), 0,
                           st, gpart, nchunk, L2, grad_eps, grad_delta);
        CBDG_CHECK_LAUNCH("k_grad_reduce");
    }
    return CBDG_OK;
}

// Per-start-vector rows of the reverse-mode derivative: the checkpoint-free
// reverse passes of cbdg_chebyshev_moments_backward with each vector's
// gradient terms written as a row of their own instead of summed.
extern "C" int cbdg_chebyshev_moments_jacobian(const cbdg_op *op, const int32_t *start_sites, int64_t n_start,
                                               int32_t N, int32_t tile, const double *dmu_ee, const double *dmu_he,
                                               void *workspace, size_t workspace_bytes, double *jac_eps,
                                               double *jac_delta, int64_t ld, void *stream)
{
    clear_error();
    int rc = check_backward_op(op, "chebyshev_moments_jacobian");
    if (rc) return rc;
    if (n_start < 0 || N < 1 || tile < 1)
        return fail(CBDG_EINVAL, "chebyshev_moments_jacobian: need n_start >= 0, N >= 1, tile >= 1");
    bool dbl = false;
    rc = backward_algorithm(op, CBDG_ALG_AUTO, N, "chebyshev_moments_jacobian", &dbl);
    if (rc) return rc;
    if (!dbl || !vc_adjoint_supported(op))
        return fail(CBDG_EUNSUPPORTED, "chebyshev_moments_jacobian: needs moment doubling (b = 0, N >= 3) on a real "
                    "operator with uniform hopping and Lx = 64 W (W = 1, 2, 4)");
    if (n_start == 0) return CBDG_OK;
    if (ld < op->L2)
        return fail(CBDG_EINVAL, "chebyshev_moments_jacobian: ld = %lld is below the %lld sites",
                    (long long)ld, (long long)op->L2);
    if (!start_sites || !workspace || (!jac_eps && !jac_delta) || (!dmu_ee && !dmu_he))
        return fail(CBDG_EINVAL, "chebyshev_moments_jacobian: start_sites, workspace, a cotangent and an output are "
                    "required");
    return backward_reversible(op, start_sites, n_start, N, (int)std::min<int64_t>(tile, n_start), dmu_ee, dmu_he,
                               workspace, workspace_bytes, nullptr, nullptr, as_stream(stream), jac_eps, jac_delta, ld);
}

namespace cbdg {
// y[r] = sum_c A[r * ld + c] x[c]: one wavefront per row, each lane summing
// the columns c = lane (mod 64) in order, then a fixed butterfly, so repeated
// calls give identical bits
__global__ __launch_bounds__(kBlock) void k_matvec(const double *__restrict__ A, int64_t rows, int64_t cols,
                                                   int64_t ld, const double *__restrict__ x, double *__restrict__ y)
{
    const int64_t r = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (r >= rows) return;  // the whole wavefront
    const int lane = threadIdx.x % kWave;
    const double *a = A + r * ld;
    double s = 0.0;
    for (int64_t c = lane; c < cols; c += kWave) s = __builtin_fma(a[c], x[c], s);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, kWave);
    if (lane == 0) y[r] = s;
}
}  // namespace cbdg

extern "C" int cbdg_jacobian_matvec(const double *A, int64_t rows, int64_t cols, int64_t ld, const double *x,
                                    double *y, void *stream)
{
    clear_error();
    if (rows < 0 || cols < 0 || ld < cols)
        return fail(CBDG_EINVAL, "jacobian_matvec: need rows >= 0, cols >= 0, ld >= cols");
    if (rows == 0) return CBDG_OK;
    if (!A || !y || (cols > 0 && !x)) return fail(CBDG_EINVAL, "jacobian_matvec: A, x and y are required");
    const int64_t nb = ceil_div(rows, kBlock / kWave);
    if (nb > INT32_MAX) return fail(CBDG_EINVAL, "jacobian_matvec: too many rows");
    hipLaunchKernelGGL(k_matvec, dim3((unsigned)nb), dim3(kBlock), 0, as_stream(stream), A, rows, cols, ld, x, y);
    CBDG_CHECK_LAUNCH("k_matvec");
    return CBDG_OK;
}
