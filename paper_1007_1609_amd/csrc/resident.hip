// Cache-resident recursion: every recursion step of one tile in a single
// persistent launch, for tiles small enough that their two vector buffers stay
// in the 256 MB Infinity Cache (the memory-side cache in front of HBM).
//
// The recursion and moments are those of eq. (ref2) with eqs. (coeff1)/
// (coeff2), by moment doubling: step n produces a_n = 2 Ht a_{n-1} - a_{n-2}
// (in place over a_{n-2}, a_1 = Ht a_0) and per (region, vector) FP64 partial
// sums of <a_n|a_n>, <a_n|a_{n-1}> and the particle-hole bilinear form, from
// which moments 2n-1 and 2n follow (the product rule of the Chebyshev
// polynomials).  The launch is cooperative (all workgroups resident at once);
// steps are separated by a grid barrier -- an atomic arrival counter with a
// bounded spin.  A barrier that does not complete within the host's spin limit
// raises an abort flag that every workgroup checks, so every workgroup leaves
// the kernel in any case and the host reports the failure.
//
// Partial sums of kResRing consecutive steps are kept in a ring; after the
// ring fills, all workgroups reduce it (each moment sum in a fixed order over
// regions, so results do not depend on scheduling) and write the moments.
#include "step.hpp"

#include <algorithm>

namespace cbdg {

constexpr int kResRing = 16;                    // steps per reduction round
constexpr int64_t kResidentBudget = 200ll << 20;  // bytes of vector buffers a resident tile may hold
constexpr int kResRows = 16;                    // rows per region
constexpr long long kResDefaultSpins = 1ll << 22;

struct ResArgs {
    void *buf0, *buf1;       // a_n lives in buffer n % 2 (a_0 seeded in buf0)
    const void *ons;         // OnSite<T>[L2]
    double th;               // t/a
    int Lx, Ly, bcx, bcy;
    int Bp, Bt, N, n_steps;
    int n_strips, n_regions, rpw;  // rpw: regions per workgroup pass (kBlock / Bp)
    const int32_t *sites;
    double *mu_ee, *mu_he;   // the tile's first row
    double *ring;            // [kResRing][n_regions][3][Bp]
    unsigned *count;         // barrier arrivals (zero at launch)
    int *abort;              // nonzero: a barrier timed out (zero at launch)
    long long spin_limit;
};

template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_resident(ResArgs A)
{
    using P = Pair<T, false>;
    using S = typename Storage<T, false>::type;
    const int Bp = A.Bp;
    const int slot = threadIdx.x / Bp;
    const int b = threadIdx.x % Bp;
    const bool lane_on = b < A.Bt;
    const int Lx = A.Lx, Ly = A.Ly;
    const int my_site = lane_on ? A.sites[b] : -1;
    const T th = T(A.th);
    const OnSite<T> *ons = reinterpret_cast<const OnSite<T> *>(A.ons);
    S *bufs[2] = {reinterpret_cast<S *>(A.buf0), reinterpret_cast<S *>(A.buf1)};
    __shared__ int s_abort;
    unsigned barrier_no = 0;

    // Grid barrier: release this workgroup's writes, arrive, wait (bounded)
    // for every workgroup, acquire theirs.  True when the launch is aborted.
    auto barrier = [&]() -> bool {
        ++barrier_no;
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            atomicAdd(A.count, 1u);
            const unsigned target = barrier_no * gridDim.x;
            long long spins = 0;
            int ab = 0;
            while (true) {
                if (__hip_atomic_load(A.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
                if (__hip_atomic_load(A.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ab = 1; break; }
                if (++spins > A.spin_limit) {
                    __hip_atomic_store(A.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ab = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            __threadfence();
            s_abort = ab;
        }
        __syncthreads();
        return s_abort != 0;
    };

    // One recursion step on one region (a strip of W columns, kResRows rows)
    // for this lane's vector: rows y-1, y, y+1 of a_{n-1} in registers, a_n
    // written over a_{n-2} in place, FP64 dot-product partials into the ring.
    auto step_region = [&](int rid, int n) {
        const int strip = rid % A.n_strips, seg = rid / A.n_strips;
        const int x0 = strip * W, y0 = seg * kResRows, y1 = min(y0 + kResRows, Ly);
        const S *a1 = bufs[(n - 1) & 1];
        S *ao = bufs[n & 1];
        const bool first = n == 1;
        int cx[W + 2];
        uint32_t cm[W + 2];
#pragma unroll
        for (int k = 0; k < W + 2; ++k) {
            const int x = x0 - 1 + k;
            if (A.bcx) { cx[k] = ((x % Lx) + Lx) % Lx; cm[k] = ~0u; }
            else { const bool ok = x >= 0 && x < Lx; cx[k] = ok ? x : 0; cm[k] = ok ? ~0u : 0u; }
        }
        auto load_row = [&](P *row, int y) {
            bool ok = true;
            int yy = y;
            if (y < 0 || y >= Ly) { ok = A.bcy != 0; yy = A.bcy ? ((y % Ly) + Ly) % Ly : 0; }
            const int64_t rb = (int64_t)yy * Lx;
#pragma unroll
            for (int k = 0; k < W + 2; ++k)
                row[k] = masked<T, false>(ld<T, false>(a1 + (rb + cx[k]) * Bp + b), (ok ? ~0u : 0u) & cm[k]);
        };
        P up[W + 2], cur[W + 2], dn[W + 2], nx[W + 2];
        load_row(up, y0 - 1);
        load_row(cur, y0);
        load_row(dn, y0 + 1);
        double d0 = 0.0, d1 = 0.0, d2 = 0.0;
        for (int y = y0; y < y1; ++y) {
            load_row(nx, y + 2);
            const int64_t srow = (int64_t)y * Lx;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const int64_t s = srow + x0 + k;
                const P yv = apply_uniform<T, false>(ons[s], th, cur[k + 1], cur[k], cur[k + 2], up[k + 1], dn[k + 1]);
                S *q = ao + s * Bp + b;
                const P ov = first ? yv : cheb_combine<T, false>(yv, ld<T, false>(q), false);
                st<T, false>(q, ov);
                if (first && s == my_site) {
                    A.mu_ee[(int64_t)b * A.N + 1] = (double)ov.e;
                    A.mu_he[(int64_t)b * A.N + 1] = (double)ov.h;
                }
                const double e = ov.e, h = ov.h, ce = cur[k + 1].e, ch = cur[k + 1].h;
                d0 += e * e + h * h;
                d1 += e * ce + h * ch;
                d2 += e * ch - h * ce;
            }
#pragma unroll
            for (int k = 0; k < W + 2; ++k) { up[k] = cur[k]; cur[k] = dn[k]; dn[k] = nx[k]; }
        }
        double *pp = A.ring + (((int64_t)((n - 1) % kResRing) * A.n_regions + rid) * 3) * Bp + b;
        pp[0] = d0;
        pp[Bp] = d1;
        pp[2 * Bp] = d2;
    };

    // Moments of the ring's steps n_first .. n_last: one unit per (step,
    // 64 vectors); wave w of the workgroup sums regions w, w + 4, ..., then
    // wave 0 adds the four wave sums in order.
    __shared__ double red[kBlock / kWave][3][kWave];
    auto reduce_ring = [&](int n_first, int n_last) {
        const int chunks = (A.Bt + kWave - 1) / kWave;
        const int units = (n_last - n_first + 1) * chunks;
        const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
        constexpr int NW = kBlock / kWave;
        for (int u = blockIdx.x; u < units; u += gridDim.x) {
            const int n = n_first + u / chunks;
            const int bb = (u % chunks) * kWave + lane;
            double acc[3] = {0.0, 0.0, 0.0};
            if (bb < A.Bt) {
                const double *base = A.ring + (int64_t)((n - 1) % kResRing) * A.n_regions * 3 * Bp + bb;
                for (int r = wv; r < A.n_regions; r += NW) {
                    const double *pp = base + (int64_t)r * 3 * Bp;
                    acc[0] += pp[0];
                    acc[1] += pp[Bp];
                    acc[2] += pp[2 * Bp];
                }
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) red[wv][k][lane] = acc[k];
            __syncthreads();
            if (wv == 0 && bb < A.Bt) {
                for (int w = 1; w < NW; ++w) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) acc[k] += red[w][k][lane];
                }
                const int64_t m = (int64_t)bb * A.N;
                if (A.mu_ee[m] == A.mu_ee[m]) {  // rows of invalid start sites stay NaN
                    const double sgn = (n & 1) ? -2.0 : 2.0;
                    if (2 * n < A.N) {
                        A.mu_ee[m + 2 * n] = 2.0 * acc[0] - A.mu_ee[m];
                        A.mu_he[m + 2 * n] = 0.0;
                    }
                    if (n >= 2 && 2 * n - 1 < A.N) {
                        A.mu_ee[m + 2 * n - 1] = 2.0 * acc[1] - A.mu_ee[m + 1];
                        A.mu_he[m + 2 * n - 1] = sgn * acc[2] - A.mu_he[m + 1];
                    }
                }
            }
            __syncthreads();
        }
    };

    const int sets = (A.n_regions + A.rpw - 1) / A.rpw;
    for (int n = 1; n <= A.n_steps; ++n) {
        for (int set = blockIdx.x; set < sets; set += gridDim.x) {
            const int rid = set * A.rpw + slot;
            if (lane_on && rid < A.n_regions) step_region(rid, n);
        }
        if (barrier()) return;
        if (n % kResRing == 0 || n == A.n_steps) {
            reduce_ring(((n - 1) / kResRing) * kResRing + 1, n);
            if (barrier()) return;
        }
    }
}

// a_0 = |s_b, e> in a zeroed buffer; mu_0 = 1 (NaN rows for invalid sites).
template <typename T>
__global__ void k_res_seed(typename Storage<T, false>::type *a0, int64_t n_pairs, int Bp, int Bt, int64_t L2,
                           const int32_t *sites, double *mu_ee, double *mu_he, int N, unsigned *count, int *abort)
{
    using S = typename Storage<T, false>::type;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_pairs;
         i += (int64_t)gridDim.x * blockDim.x)
        a0[i] = S{T(0), T(0)};
    if (blockIdx.x == 0 && threadIdx.x == 0) { *count = 0u; *abort = 0; }
}

template <typename T>
__global__ void k_res_seed_sites(typename Storage<T, false>::type *a0, int Bp, int Bt, int64_t L2,
                                 const int32_t *sites, double *mu_ee, double *mu_he, int N)
{
    using S = typename Storage<T, false>::type;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= Bt) return;
    const int64_t s = sites[b];
    const int64_t m = (int64_t)b * N;
    if (s < 0 || s >= L2) {
        const double nan = __builtin_nan("");
        for (int n = 0; n < N; ++n) { mu_ee[m + n] = nan; mu_he[m + n] = nan; }
        return;
    }
    a0[s * Bp + b] = S{T(1), T(0)};
    mu_ee[m] = 1.0;
    mu_he[m] = 0.0;
}

struct ResPlan {
    int W, n_strips, n_regions, rpw, Bp;
    int64_t buf_bytes, ring_bytes;
};

static ResPlan res_plan(const cbdg_op *op, int tile, int precision)
{
    ResPlan p;
    p.Bp = (int)lane_stride(tile);
    p.W = (op->Lx % 2 == 0) ? 2 : 1;
    p.n_strips = op->Lx / p.W;
    p.n_regions = p.n_strips * (int)ceil_div(op->Ly, kResRows);
    p.rpw = std::max(1, kBlock / p.Bp);
    const int64_t pair = precision == CBDG_FP64 ? 16 : 8;
    p.buf_bytes = round_up(op->L2 * p.Bp * pair, 256);
    p.ring_bytes = round_up((int64_t)kResRing * p.n_regions * 3 * p.Bp * (int64_t)sizeof(double), 256);
    return p;
}

static int res_check(const cbdg_op *op, int tile, int precision, const char *who)
{
    if (!op) return fail(CBDG_EINVAL, "%s: op must not be NULL", who);
    if (op->scalar != CBDG_REAL || op->general)
        return fail(CBDG_EUNSUPPORTED, "%s: resident tiles are implemented for real operators with uniform "
                    "hopping and on-site pairing", who);
    if (op->bounds.b != 0.0)
        return fail(CBDG_EINVAL, "%s: moment doubling needs a spectrum centred at b = 0 (b = %g)", who, op->bounds.b);
    if (precision != CBDG_FP64 && precision != CBDG_FP32_ACC64)
        return fail(CBDG_EINVAL, "%s: unknown precision %d", who, precision);
    if (tile < 1 || lane_stride(tile) > kBlock)
        return fail(CBDG_EINVAL, "%s: resident tiles hold 1 to %d vectors (got %d)", who, kBlock, tile);
    const ResPlan p = res_plan(op, tile, precision);
    if (2 * p.buf_bytes > kResidentBudget)
        return fail(CBDG_EINVAL, "%s: tiles of %d vectors need %lld bytes of vectors, more than the %lld a tile "
                    "resident in the Infinity Cache may hold (use fewer vectors per tile)", who, tile,
                    (long long)(2 * p.buf_bytes), (long long)kResidentBudget);
    return CBDG_OK;
}

template <typename T, int W>
static int launch_resident(const cbdg_op *op, const ResPlan &p, ResArgs A, hipStream_t st)
{
    int per_cu = 0, n_cu = 0, dev = 0;
    CBDG_CHECK_HIP(hipGetDevice(&dev));
    CBDG_CHECK_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    CBDG_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_resident<T, W>, kBlock, 0));
    if (per_cu < 1) return fail(CBDG_EHIP, "chebyshev_moments_resident: the kernel does not fit on a compute unit");
    const int sets = (int)ceil_div(p.n_regions, p.rpw);
    const int grid = std::max(1, std::min(sets, per_cu * n_cu));
    void *args[] = {&A};
    CBDG_CHECK_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_resident<T, W>), dim3(grid),
                                              dim3(kBlock), args, 0, st));
    return CBDG_OK;
}

template <typename T>
static int run_resident(const cbdg_op *op, const int32_t *sites, int64_t n_start, int N, int tile, void *ws,
                        long long spin_limit, double *mu_ee, double *mu_he, int *abort_host, hipStream_t st)
{
    using S = typename Storage<T, false>::type;
    const ResPlan p = res_plan(op, tile, std::is_same<T, double>::value ? CBDG_FP64 : CBDG_FP32_ACC64);
    char *base = reinterpret_cast<char *>(ws);
    S *buf0 = reinterpret_cast<S *>(base);
    S *buf1 = reinterpret_cast<S *>(base + p.buf_bytes);
    double *ring = reinterpret_cast<double *>(base + 2 * p.buf_bytes);
    unsigned *count = reinterpret_cast<unsigned *>(base + 2 * p.buf_bytes + p.ring_bytes);
    int *abort_flag = reinterpret_cast<int *>(count + 1);
    for (int64_t t0 = 0; t0 < n_start; t0 += tile) {
        const int Bt = (int)std::min<int64_t>(tile, n_start - t0);
        const int Bp = (int)lane_stride(Bt);
        double *mee = mu_ee + t0 * N;
        double *mhe = mu_he + t0 * N;
        const int64_t n_pairs = op->L2 * Bp;
        hipLaunchKernelGGL(k_res_seed<T>, dim3((unsigned)std::min<int64_t>(ceil_div(n_pairs, kBlock), 8192)),
                           dim3(kBlock), 0, st, buf0, n_pairs, Bp, Bt, op->L2, sites + t0, mee, mhe, N, count,
                           abort_flag);
        CBDG_CHECK_LAUNCH("k_res_seed");
        hipLaunchKernelGGL(k_res_seed_sites<T>, dim3((unsigned)ceil_div(Bt, kBlock)), dim3(kBlock), 0, st, buf0, Bp,
                           Bt, op->L2, sites + t0, mee, mhe, N);
        CBDG_CHECK_LAUNCH("k_res_seed_sites");
        const int n_steps = N >= 2 ? N / 2 : 0;
        if (n_steps > 0) {
            ResArgs A{};
            A.buf0 = buf0; A.buf1 = buf1;
            A.ons = std::is_same<T, double>::value ? (const void *)op->onsite64 : (const void *)op->onsite32;
            A.th = op->t / op->bounds.a;
            A.Lx = op->Lx; A.Ly = op->Ly; A.bcx = op->bc_x; A.bcy = op->bc_y;
            A.Bp = Bp; A.Bt = Bt; A.N = N; A.n_steps = n_steps;
            A.n_strips = p.n_strips; A.n_regions = p.n_regions; A.rpw = std::max(1, kBlock / Bp);
            A.sites = sites + t0; A.mu_ee = mee; A.mu_he = mhe;
            A.ring = ring; A.count = count; A.abort = abort_flag;
            A.spin_limit = spin_limit;
            const int rc = p.W == 2 ? launch_resident<T, 2>(op, p, A, st) : launch_resident<T, 1>(op, p, A, st);
            if (rc) return rc;
            // a timed-out barrier ends the launch early: report it before the
            // next tile reuses the buffers
            CBDG_CHECK_HIP(hipMemcpyAsync(abort_host, abort_flag, sizeof(int), hipMemcpyDeviceToHost, st));
            CBDG_CHECK_HIP(hipStreamSynchronize(st));
            if (*abort_host)
                return fail(CBDG_EHIP, "chebyshev_moments_resident: a grid barrier did not complete within %lld "
                            "spins; the launch was abandoned", spin_limit);
        }
        const int rc = bound_moments(mee, mhe, (int64_t)Bt * N, false, false,
                                     moment_limit(!std::is_same<T, double>::value), st);
        if (rc) return rc;
    }
    return CBDG_OK;
}

}  // namespace cbdg

using namespace cbdg;

extern "C" int cbdg_resident_workspace_size(const cbdg_op *op, int32_t tile, int32_t precision, size_t *bytes)
{
    clear_error();
    if (!bytes) return fail(CBDG_EINVAL, "resident_workspace_size: bytes must not be NULL");
    int rc = res_check(op, tile, precision, "resident_workspace_size");
    if (rc) return rc;
    const ResPlan p = res_plan(op, tile, precision);
    *bytes = (size_t)(2 * p.buf_bytes + p.ring_bytes + 256);
    return CBDG_OK;
}

extern "C" int cbdg_chebyshev_moments_resident(const cbdg_op *op, const int32_t *start_sites, int64_t n_start,
                                               int32_t N, int32_t tile, int32_t precision, int64_t spin_limit,
                                               void *workspace, size_t workspace_bytes, double *mu_ee,
                                               void *mu_he, void *stream)
{
    clear_error();
    if (n_start < 0 || N < 1) return fail(CBDG_EINVAL, "chebyshev_moments_resident: need n_start >= 0 and N >= 1");
    if (spin_limit < 0) return fail(CBDG_EINVAL, "chebyshev_moments_resident: spin_limit must be >= 0");
    const int32_t eff = (int32_t)std::max<int64_t>(1, std::min<int64_t>(tile, n_start));
    int rc = res_check(op, eff, precision, "chebyshev_moments_resident");
    if (rc) return rc;
    if (n_start == 0) return CBDG_OK;
    if (!start_sites || !mu_ee || !mu_he || !workspace)
        return fail(CBDG_EINVAL, "chebyshev_moments_resident: start_sites, mu_ee, mu_he and workspace must not be NULL");
    size_t need = 0;
    if ((rc = cbdg_resident_workspace_size(op, eff, precision, &need))) return rc;
    if (workspace_bytes < need)
        return fail(CBDG_EINVAL, "chebyshev_moments_resident: workspace of %zu bytes is smaller than the %zu needed",
                    workspace_bytes, need);
    int abort_host = 0;
    hipStream_t st = as_stream(stream);
    const long long spins = spin_limit > 0 ? (long long)spin_limit : kResDefaultSpins;
    double *mhe = reinterpret_cast<double *>(mu_he);
    return precision == CBDG_FP64
               ? run_resident<double>(op, start_sites, n_start, N, eff, workspace, spins, mu_ee, mhe, &abort_host, st)
               : run_resident<float>(op, start_sites, n_start, N, eff, workspace, spins, mu_ee, mhe, &abort_host, st);
}
