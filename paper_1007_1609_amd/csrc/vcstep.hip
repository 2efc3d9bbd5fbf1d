// Chebyshev recursion of eq. (ref2) over a tile stored vector-contiguous,
// for real operators with uniform hopping and moment doubling.
//
// Vector b occupies the pairs b*Dv .. b*Dv + L2 - 1, one row after the
// other.  A wavefront holds one vector and one segment of rows; lane l owns
// the W = Lx/64 neighbouring columns lW .. lW+W-1 of every row.  Inside a row
// the pairs are ordered so that every load and store instruction of a
// wavefront moves one contiguous 1 KB block (16 bytes per lane; pair_pos).
// The x-neighbours of a lane's outer columns are the outer columns of lanes
// l-1 and l+1, moved across the wavefront by DPP wave shifts (rotations for
// periodic x).  Against the vector-major passes (lanes = vectors, strips
// widened by the halo of every fused step):
//   - a pass of K steps computes each intermediate vector once per site;
//     only the K-1 rows at each end of a row segment are computed twice, so
//     K = 7 fused steps cost little more arithmetic than seven single steps
//     while the vectors cross HBM 4 times instead of 21;
//   - a lane holds W pairs per row instead of W + 6, so the seven three-row
//     windows of a pass fit one wavefront per SIMD (part in AGPRs);
//   - a vector is clipped to its own light cone: a_n vanishes outside the
//     diamond |x - x_b| + |y - y_b| <= n around its start site, rows outside
//     it are skipped, and lanes outside it neither read nor write (their
//     buffer offsets are pushed past the buffer-resource range, where loads
//     return zero and stores are dropped);
//   - the per-site coefficients (2 de, 2 Delta/a) come from a packed copy in
//     the same row layout (every vector reads the same copy, from L2) through
//     a ring in LDS instead of wave-uniform scalar loads; with b = 0 (the
//     doubling identities need it) the hole diagonal is exactly -de, and the
//     factor 2 of eq. (ref2), folded into the coefficients, saves the product
//     by t/a and the separate combination with a_{n-2} of every component.
// The first step and single steps compute a site exactly as the vector-major
// kernels do; the passes of several steps round 2 Ht a_{n-1} - a_{n-2} in
// three fused multiply-adds instead, and the doubling partials are summed in
// another (fixed) order.
//
// Nothing is read that the tile has not written: a load of a_m covers the
// rows of the diamond of radius m (on open rows only the lanes the diamond
// touches), the store of a_m the same rows and lanes (with the zeros a lane
// holds outside the diamond), and a_0 is seeded as its whole start row.
// The buffers need no clearing between tiles.
#include "step.hpp"

#include <algorithm>

namespace cbdg {

namespace {

#ifndef CBDG_VC_WG
#define CBDG_VC_WG 4
#endif
constexpr int kVcWaves = CBDG_VC_WG;       // vectors per workgroup
constexpr int kVcBlock = kVcWaves * kWave;
constexpr unsigned kOut = 0x80000000u;     // a byte offset past every buffer range
constexpr int kRsrcWord3 = 0x00020000;     // gfx9 buffer descriptor: 32-bit data format

// DPP controls of the whole-wavefront shifts by one lane
constexpr int kShl1 = 0x130;  // lane i <- lane i+1 (lane 63 <- 0)
constexpr int kRol1 = 0x134;  // lane i <- lane i+1 (lane 63 <- lane 0)
constexpr int kShr1 = 0x138;  // lane i <- lane i-1 (lane 0 <- 0)
constexpr int kRor1 = 0x13C;  // lane i <- lane i-1 (lane 0 <- lane 63)

template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL, typename T>
__device__ __forceinline__ Pair<T, false> dpp_pair(const Pair<T, false> &p)
{
    return Pair<T, false>{dpp<CTRL>(p.e), dpp<CTRL>(p.h)};
}

typedef unsigned U4 __attribute__((ext_vector_type(4)));
typedef unsigned U2 __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t vec_rsrc(const void *base, int64_t b, int64_t Dv)
{
    const char *p = reinterpret_cast<const char *>(base) + b * Dv * (int64_t)(2 * sizeof(T));
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(p), (short)0, (int)(Dv * 2 * sizeof(T)), kRsrcWord3);
}

// Every access moves 16 bytes per lane: one FP64 pair or two FP32 pairs
// (kPer pairs).  Inside a row, chunk j of lane l (its pairs k = j*kPer ..
// j*kPer + kPer - 1) sits at (j*64 + l)*kPer, so the j-th chunks of all lanes
// are one contiguous 1 KB block.
template <typename T> constexpr int kPer = 16 / (2 * (int)sizeof(T));
template <typename T> __host__ __device__ constexpr int pair_pos(int lane, int k)
{
    return ((k / kPer<T>) * kWave + lane) * kPer<T> + k % kPer<T>;
}

// Cache policy of the vector streams: nontemporal (2) for FP64, where each
// row of a vector is read or written once per pass and the streams stay out
// of the caches' way (FP64, 256x256, one 1024-vector tile: 107.2 -> 99.3 ms);
// FP32 runs faster with ordinary accesses (136.2 ms against 160.9).
#ifndef CBDG_VC_NT_F64
#define CBDG_VC_NT_F64 2
#endif
#ifndef CBDG_VC_NT_F32
#define CBDG_VC_NT_F32 0
#endif
template <typename T> constexpr int kAux = sizeof(T) == 8 ? CBDG_VC_NT_F64 : CBDG_VC_NT_F32;

// the chunk of kPer pairs at byte offset off
template <typename T>
__device__ __forceinline__ void bld(__amdgpu_buffer_rsrc_t r, unsigned off, Pair<T, false> *p)
{
    const U4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, kAux<T>);
    if constexpr (sizeof(T) == 8) {
        p[0].e = __hiloint2double((int)v[1], (int)v[0]);
        p[0].h = __hiloint2double((int)v[3], (int)v[2]);
    } else {
        p[0].e = __uint_as_float(v[0]); p[0].h = __uint_as_float(v[1]);
        p[1].e = __uint_as_float(v[2]); p[1].h = __uint_as_float(v[3]);
    }
}

template <typename T>
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, unsigned off, const Pair<T, false> *p)
{
    U4 v;
    if constexpr (sizeof(T) == 8) {
        v = U4{(unsigned)__double2loint(p[0].e), (unsigned)__double2hiint(p[0].e), (unsigned)__double2loint(p[0].h),
               (unsigned)__double2hiint(p[0].h)};
    } else {
        v = U4{__float_as_uint(p[0].e), __float_as_uint(p[0].h), __float_as_uint(p[1].e), __float_as_uint(p[1].h)};
    }
    __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, kAux<T>);
}

// Geometry of one wavefront: its vector's start site and its row segment.
// Rows are virtual (periodic y: taken modulo Ly), so a segment with its halo
// rows is always a run of consecutive integers.
template <bool BCX, bool BCY>
struct VcGeo {
    int Lx, Ly;
    int xi, yi;  // start site
    int lo;      // the lane's first column
    int lane;

    __device__ int dy(int v) const
    {
        int d = v - yi;
        if constexpr (BCY) {
            d %= Ly;
            if (d < 0) d += Ly;
            return min(d, Ly - d);
        }
        return d < 0 ? -d : d;
    }
    __device__ bool in_lattice(int v) const { return BCY || (unsigned)v < (unsigned)Ly; }
    __device__ int phys(int v) const
    {
        if constexpr (!BCY) return v;
        const int r = v % Ly;
        return r < 0 ? r + Ly : r;
    }
    // byte offset of the lane's first pair in row v of a vector that vanishes
    // outside the diamond of radius R, or past the range where it vanishes
    // (a select on the computed offset, so no lane branches)
    template <typename T, int W>
    __device__ unsigned offset(int v, int R) const
    {
        const int rr = R - dy(v);
        const unsigned at = (unsigned)((phys(v) * Lx + lane * kPer<T>) * (int)(2 * sizeof(T)));
        bool ok = in_lattice(v) & (rr >= 0);
        if constexpr (!BCX) ok = ok & (lo <= xi + rr) & (lo + W - 1 >= xi - rr);
        const unsigned keep = 0u - (unsigned)ok;
        return (at & keep) | (kOut & ~keep);
    }
    // the lane's first packed coefficient pair of row v (row 0 for rows
    // outside an open lattice, whose results are masked)
    template <typename T>
    __device__ int64_t coef_row(int v) const { return (int64_t)(in_lattice(v) ? phys(v) : 0) * Lx + lane * kPer<T>; }
};

template <typename T, int W>
__device__ __forceinline__ void load_row(__amdgpu_buffer_rsrc_t r, unsigned off, Pair<T, false> *out)
{
#pragma unroll
    for (int j = 0; j < W / kPer<T>; ++j) bld<T>(r, off + j * (unsigned)(kWave * 16), out + j * kPer<T>);
}

template <typename T, int W>
__device__ __forceinline__ void store_row(__amdgpu_buffer_rsrc_t r, unsigned off, const Pair<T, false> *v)
{
#pragma unroll
    for (int j = 0; j < W / kPer<T>; ++j) bst<T>(r, off + j * (unsigned)(kWave * 16), v + j * kPer<T>);
}

// (de, Delta/a) of the lane's W sites of one row, 16 bytes per load
template <typename T, int W>
__device__ __forceinline__ void load_coef(const typename Storage<T, false>::type *pc, int64_t at,
                                          typename Storage<T, false>::type *o)
{
    using S = typename Storage<T, false>::type;
#pragma unroll
    for (int j = 0; j < W / kPer<T>; ++j) {
        if constexpr (sizeof(T) == 8) {
            o[j] = pc[at + j * kWave];
        } else {
            const float4 v = *reinterpret_cast<const float4 *>(pc + at + j * kWave * 2);
            o[2 * j] = S{v.x, v.y};
            o[2 * j + 1] = S{v.z, v.w};
        }
    }
}

// Ht applied to row `c` (rows `d` below and `u` above), x-halo across lanes
template <typename T, int W, bool BCX>
__device__ __forceinline__ void apply_row(const typename Storage<T, false>::type *cf, T th, const Pair<T, false> *c,
                                          const Pair<T, false> *d, const Pair<T, false> *u, Pair<T, false> *y)
{
    const Pair<T, false> hl = dpp_pair<BCX ? kRor1 : kShr1>(c[W - 1]);
    const Pair<T, false> hr = dpp_pair<BCX ? kRol1 : kShl1>(c[0]);
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const OnSite<T> o{cf[k].x, -cf[k].x, cf[k].y, T(0)};
        y[k] = apply_uniform<T, false>(o, th, c[k], k > 0 ? c[k - 1] : hl, k < W - 1 ? c[k + 1] : hr, d[k], u[k]);
    }
}

// Whether the passes of several steps fold the factor 2 of eq. (ref2) into
// their coefficients (2 de, 2 Delta/a and 2 t/a are exact): 2 Ht c - p of a
// component is then three fused multiply-adds after the neighbour sum
// instead of a product, two fused multiply-adds and the combination (FP32,
// 256x256, 16 tiles of 1024 vectors at N = 2048: 1203 -> 1148 ms; FP64 at
// N = 1024 unchanged within the run-to-run spread, 3189 / 3214 ms).
#ifndef CBDG_VC_FOLD
#define CBDG_VC_FOLD 1
#endif
template <typename T> constexpr T kCoefScale = CBDG_VC_FOLD ? T(2) : T(1);

// 2 Ht c - p at one site from the doubled coefficients cf = (2 de, 2 Delta/a)
// and th2 = 2 t/a (the hole diagonal is -2 de)
template <typename T>
__device__ __forceinline__ Pair<T, false> step_site(const typename Storage<T, false>::type &cf, T th2,
                                                     const Pair<T, false> &c, const Pair<T, false> &l,
                                                     const Pair<T, false> &r, const Pair<T, false> &d,
                                                     const Pair<T, false> &u, const Pair<T, false> &p)
{
#pragma clang fp contract(off)
    const T se = (l.e + r.e) + (d.e + u.e), sh = (l.h + r.h) + (d.h + u.h);
    Pair<T, false> y;
    y.e = fma_t(cf.x, c.e, fma_t(cf.y, c.h, fma_t(-th2, se, -p.e)));
    y.h = fma_t(-cf.x, c.h, fma_t(cf.y, c.e, fma_t(th2, sh, -p.h)));
    return y;
}

// one site of a pass: 2 Ht c - p from the ring's coefficients
template <typename T>
__device__ __forceinline__ Pair<T, false> pass_site(const typename Storage<T, false>::type &cf, T th,
                                                     const Pair<T, false> &c, const Pair<T, false> &l,
                                                     const Pair<T, false> &r, const Pair<T, false> &d,
                                                     const Pair<T, false> &u, const Pair<T, false> &p)
{
    if constexpr (CBDG_VC_FOLD) {
        return step_site<T>(cf, th, c, l, r, d, u, p);
    } else {
        const OnSite<T> o{cf.x, -cf.x, cf.y, T(0)};
        return cheb_combine<T, false>(apply_uniform<T, false>(o, th, c, l, r, d, u), p, false);
    }
}

// <v|v>, <v|c> and B(v, c) of one site added to the partial sums, as two
// fused multiply-adds each (no other contraction: the sums do not depend on
// how the compiler schedules a pass)
__device__ __forceinline__ void dots3(double *acc, double e, double h, double ce, double ch)
{
    acc[0] = __builtin_fma(h, h, __builtin_fma(e, e, acc[0]));
    acc[1] = __builtin_fma(h, ch, __builtin_fma(e, ce, acc[1]));
    acc[2] = __builtin_fma(-h, ce, __builtin_fma(e, ch, acc[2]));
}

// Sum over the wavefront in a fixed order (the same butterfly in every lane);
// lane 0 stores its result.
template <int K>
__device__ __forceinline__ void wave_sum(double *d)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) d[k] += __shfl_xor(d[k], off, kWave);
    }
}

// With one row segment per vector the wavefront's sums are the whole dot
// products of step m, and its lane 0 writes the moments of the doubling
// identities itself (the arithmetic of the reduction kernels, which the
// passes need for two or more segments):
//   mu_ee[2m] = 2 <a_m|a_m> - mu_ee[0],  mu_he[2m] = 0,
//   mu_ee[2m-1] = 2 <a_m|a_{m-1}> - mu_ee[1],
//   mu_he[2m-1] = 2 (-1)^m B(a_m, a_{m-1}) - mu_he[1]   (m >= 2).
__device__ __forceinline__ void vc_moments(const VcArgs &A, int b, int m, const double *dm)
{
    const int64_t row = (int64_t)b * A.N;
    const double s0 = 0.0 + dm[0], s1 = 0.0 + dm[1], s2 = 0.0 + dm[2];
    if (2 * m < A.N) {
        A.mu_ee[row + 2 * m] = 2.0 * s0 - A.mu_ee[row];
        A.mu_he[row + 2 * m] = 0.0;
    }
    if (m >= 2 && 2 * m - 1 < A.N) {
        A.mu_ee[row + 2 * m - 1] = 2.0 * s1 - A.mu_ee[row + 1];
        A.mu_he[row + 2 * m - 1] = ((m & 1) ? -2.0 : 2.0) * s2 - A.mu_he[row + 1];
    }
}

// Common prologue: the wavefront's vector, start site and row segment for a
// pass whose last step has light-cone radius m.  Returns false when the
// wavefront has nothing to compute (its partials are written as zeros then,
// in `nparts` arrays).
template <bool BCX, bool BCY>
struct VcWave {
    int b, seg, lane, y0, y1;
    VcGeo<BCX, BCY> g;
};

template <bool BCX, bool BCY>
__device__ __forceinline__ bool vc_wave(const VcArgs &A, int m, int nparts, VcWave<BCX, BCY> &w)
{
    const int lb = xcd_remap(blockIdx.x, A.nblocks);
    w.seg = lb % A.n_segs;
    const int grp = lb / A.n_segs;
    w.lane = threadIdx.x % kWave;
    w.b = grp * kVcWaves + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (w.b >= A.Bt) return false;
    const int Lx = A.Lx, Ly = A.Ly;
    const int si = A.sites[w.b];
    int ylo = 0, yhi = -1;
    if (si >= 0 && si < Lx * Ly) {
        w.g.yi = si / Lx;
        w.g.xi = si - w.g.yi * Lx;
        if constexpr (BCY) {
            if (2 * m + 1 >= Ly) { ylo = 0; yhi = Ly - 1; }
            else { ylo = w.g.yi - m; yhi = w.g.yi + m; }
        } else {
            ylo = max(0, w.g.yi - m);
            yhi = min(Ly - 1, w.g.yi + m);
        }
    }
    const int per = max(4, (yhi - ylo + 1 + A.n_segs - 1) / A.n_segs);
    w.y0 = ylo + w.seg * per;
    w.y1 = min(w.y0 + per, yhi + 1);
    if (w.y0 >= w.y1) {
        if (w.lane < 3 * nparts)
            A.part[(w.lane / 3) * A.pstride + ((int64_t)w.seg * 3 + w.lane % 3) * A.Bp + w.b] = 0.0;
        return false;
    }
    w.g.Lx = Lx; w.g.Ly = Ly;
    return true;
}

}  // namespace

// One step: a_n (FIRST: a_1 = Ht a_0 and moment 1) and the doubling partials
// <a_n|a_n>, <a_n|a_{n-1}>, B(a_n, a_{n-1}) of the wavefront's rows.  Each
// trip issues the coefficient loads of its row before the loads of the rows
// the next trip needs, so waiting for the former leaves the latter in flight.
template <typename T, int W, bool BCX, bool BCY, bool FIRST>
__global__ __launch_bounds__(kVcBlock) void k_vc_step1(VcArgs A)
{
    using P = Pair<T, false>;
    using S = typename Storage<T, false>::type;
    VcWave<BCX, BCY> w;
    const int n = A.n;
    if (!vc_wave(A, n, 1, w)) return;
    w.g.lo = w.lane * W;
    w.g.lane = w.lane;
    const auto &g = w.g;
    const auto r1 = vec_rsrc<T>(A.a1, w.b, A.Dv);
    const auto r2 = vec_rsrc<T>(A.a2, w.b, A.Dv);
    const auto ro = vec_rsrc<T>(A.out, w.b, A.Dv);
    const S *pc = reinterpret_cast<const S *>(A.coef);
    const T th = T(A.th);
    const int y0 = w.y0, y1 = w.y1;

    P w0[W], w1[W], w2[W], nx[W], p2[W], pn[W], v[W];
    S c0[W];
#pragma unroll
    for (int k = 0; k < W; ++k) p2[k] = pn[k] = zero_pair<T, false>();
    load_row<T, W>(r1, g.template offset<T, W>(y0 - 1, n - 1), w0);
    load_row<T, W>(r1, g.template offset<T, W>(y0, n - 1), w1);
    load_row<T, W>(r1, g.template offset<T, W>(y0 + 1, n - 1), w2);
    if constexpr (!FIRST) load_row<T, W>(r2, g.template offset<T, W>(y0, n - 2), p2);
    double d[3] = {0.0, 0.0, 0.0};
    P mv = zero_pair<T, false>();
    bool found = false;
    const int kx = g.xi % W;
    const bool own_lane = w.lane == g.xi / W;
#pragma unroll 1
    for (int r = y0; r < y1; ++r) {
        load_coef<T, W>(pc, g.template coef_row<T>(r), c0);
        if constexpr (CBDG_VC_FOLD) {
#pragma unroll
            for (int k = 0; k < W; ++k) { c0[k].x *= T(0.5); c0[k].y *= T(0.5); }
        }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (!FIRST) load_row<T, W>(r2, g.template offset<T, W>(min(r + 1, y1 - 1), n - 2), pn);
        load_row<T, W>(r1, g.template offset<T, W>(min(r + 2, y1), n - 1), nx);
        apply_row<T, W, BCX>(c0, th, w1, w0, w2, v);
#pragma unroll
        for (int k = 0; k < W; ++k) {
            v[k] = cheb_combine<T, false>(v[k], p2[k], FIRST);
            dots3(d, (double)v[k].e, (double)v[k].h, (double)w1[k].e, (double)w1[k].h);
        }
        store_row<T, W>(ro, g.template offset<T, W>(r, n), v);
        if constexpr (FIRST) {
            if (g.phys(r) == g.yi) {
#pragma unroll
                for (int k = 0; k < W; ++k) mv = select_pair<T, false>(k == kx, v[k], mv);
                found = own_lane;
            }
        }
#pragma unroll
        for (int k = 0; k < W; ++k) {
            w0[k] = w1[k]; w1[k] = w2[k]; w2[k] = nx[k];
            if constexpr (!FIRST) p2[k] = pn[k];
        }
    }
    if constexpr (FIRST) {
        if (found && A.mu_ee) {
            const int64_t m = (int64_t)w.b * A.N + 1;
            A.mu_ee[m] = (double)mv.e;
            A.mu_he[m] = (double)mv.h;
        }
    }
    wave_sum<3>(d);
    if (w.lane == 0) {
        if (A.n_segs == 1) {
            vc_moments(A, w.b, n, d);
        } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) A.part[((int64_t)w.seg * 3 + k) * A.Bp + w.b] = d[k];
        }
    }
}

// Steps per pass and the wavefronts per SIMD the compiler must fit (its
// registers: 512 / waves per lane).  One 1024-vector tile of the 256x256
// workload (first / middle tile, ms; FP64 at N = 1024, FP32 at N = 2048):
// FP64 three steps 99 / 117, four 81 / 95, five 69 / 80, six 55 / 65, seven
// 46.7 / 54.9, eight 47.4 / 55.4; FP32 five 85 / 91, six 78 / 85, seven
// 72 / 78, eight 73 / 79.  At one wavefront per SIMD the registers hold the
// windows of all levels (part in AGPRs); two per SIMD would need K <= 3.
#ifndef CBDG_VC_K_F64
#define CBDG_VC_K_F64 7
#endif
#ifndef CBDG_VC_K_F32
#define CBDG_VC_K_F32 7
#endif
// Whether a pass skips the rows of a level outside the lattice or its light
// cone (they are zero) instead of computing them (FP32, 256x256, 16 tiles of
// 1024 vectors at N = 2048: 1101 -> 1083 ms; FP64 unchanged)
#ifndef CBDG_VC_DLDS_F64
#define CBDG_VC_DLDS_F64 5
#endif
#ifndef CBDG_VC_SKIP
#define CBDG_VC_SKIP 1
#endif
#ifndef CBDG_VC_DEFER_F64
#define CBDG_VC_DEFER_F64 1
#endif
#ifndef CBDG_VC_DEFER_F32
#define CBDG_VC_DEFER_F32 0
#endif
// Coefficient ring of 8 slots (a power of two: the slot of a row is a mask
// of its index, not a remainder by K = 7) instead of K; 131 KB of LDS per
// workgroup of four FP64 wavefronts at W = 4
#ifndef CBDG_VC_RING_POW2
#define CBDG_VC_RING_POW2 1
#endif
#ifndef CBDG_VC_OCC_F64
#define CBDG_VC_OCC_F64 1
#endif
#ifndef CBDG_VC_OCC_F32
#define CBDG_VC_OCC_F32 1
#endif
template <typename T> constexpr int kVcSteps = sizeof(T) == 8 ? CBDG_VC_K_F64 : CBDG_VC_K_F32;
// Trips ahead that the a_{n-1} and a_{n-2} rows are loaded (FP64 six steps:
// 55.0 ms one and one, 51.9 three and two; at seven steps the a_{n-1} rows
// go three trips ahead in the registers the LDS-held doubling sums free.
// FP32 seven steps: 73.2 -> 71.9)
#ifndef CBDG_VC_D1_F64
#define CBDG_VC_D1_F64 3
#endif
#ifndef CBDG_VC_D2_F64
#define CBDG_VC_D2_F64 1
#endif
#ifndef CBDG_VC_D1_F32
#define CBDG_VC_D1_F32 3
#endif
#ifndef CBDG_VC_D2_F32
#define CBDG_VC_D2_F32 2
#endif
template <typename T> struct VcDepth {
    static constexpr int a1 = sizeof(T) == 8 ? CBDG_VC_D1_F64 : CBDG_VC_D1_F32;
    static constexpr int a2 = sizeof(T) == 8 ? CBDG_VC_D2_F64 : CBDG_VC_D2_F32;
};
template <typename T, int K> struct VcOcc {
    static constexpr int waves = sizeof(T) == 8 ? CBDG_VC_OCC_F64 : CBDG_VC_OCC_F32;
};

// K steps in one pass: a_n .. a_{n+K-1} from a_{n-2} and a_{n-1}; the last
// two (a_{n+K-2}, a_{n+K-1}, what the next pass reads) are stored, the others
// stay in registers.  Trip r computes row r - j of level j (a_{n+j}) for
// j = 0 .. K-1: level j needs rows r-j-1 .. r-j+1 of level j-1 and row r-j
// of level j-2 (a_{n-1} and a_{n-2} for the first two levels), so every
// level keeps a window of its three newest rows.  Level j is computed on the
// segment's rows and K-1-j more at each end.
// Each trip stores the coefficient row loaded on the trip before into the
// LDS ring and loads the next one, then loads the a_{n-2} and a_{n-1} rows
// of later trips (FP64: and stores the two rows the trip before computed).  The a_{n-1} rows sit in a ring of 3 + D1 and the a_{n-2}
// rows in a ring of 1 + D2, rotated by unrolling the loop U times: a register
// that a load is still filling is never copied, so no trip waits for the
// loads it issued itself.  The trip count is rounded up to a multiple of U;
// the extra trips compute rows past the segment that are neither stored nor
// summed.
// VAR: a shorter last pass of A.nlev (2 .. K-1) levels, the rest skipped.
template <typename T, int W, bool BCX, bool BCY, int K, bool VAR>
__global__ __launch_bounds__(kVcBlock) __attribute__((amdgpu_waves_per_eu(VcOcc<T, K>::waves)))
void k_vc_pass(VcArgs A)
{
    static_assert(K >= 3, "a pass of K steps keeps the windows of levels 0 .. K-2");
    using P = Pair<T, false>;
    using S = typename Storage<T, false>::type;
    VcWave<BCX, BCY> w;
    const int n = A.n;
    const int nlev = VAR ? A.nlev : K;
    if (!vc_wave(A, n + nlev - 1, nlev, w)) return;
    w.g.lo = w.lane * W;
    w.g.lane = w.lane;
    const auto &g = w.g;
    const auto r1 = vec_rsrc<T>(A.a1, w.b, A.Dv);
    const auto r2 = vec_rsrc<T>(A.a2, w.b, A.Dv);
    const auto ro1 = vec_rsrc<T>(A.out, w.b, A.Dv);
    const auto ro2 = vec_rsrc<T>(A.out2, w.b, A.Dv);
    const T th = kCoefScale<T> * T(A.th);
    const int y0 = w.y0, y1 = w.y1;

    // a_{n-1} rows r-1 .. r+1 and the D1 rows in flight; a_{n-2} row r and
    // the D2 rows in flight
    // (the shorter last pass, one launch per tile, keeps the rows one trip
    // ahead: its stores at a run-time level leave no room for more; so do
    // narrower rows, W < 4, whose passes the deeper ring does not speed up)
    constexpr int D1 = sizeof(T) == 8 && (VAR || W < 4) ? 1 : VcDepth<T>::a1, D2 = VcDepth<T>::a2;
    constexpr int R1 = 3 + D1, R2 = 1 + D2;
    P ra[R1][W], rp[R2][W];
    P lv[K - 1][3][W];              // level j: rows r-j-2, r-j-1, r-j
    // Coefficient rows r-K+1 .. r in a ring in LDS of KR >= K slots (slot =
    // row mod KR), one row loaded per trip into registers one trip ahead of
    // its use
    constexpr int NQ = W / kPer<T>;  // 16-byte chunks per lane and row
    constexpr int KR = CBDG_VC_RING_POW2 ? (K <= 4 ? 4 : 8) : K;
    __shared__ U4 ring_all[kVcWaves][KR][NQ][kWave];
    U4 (*ring)[NQ][kWave] = ring_all[threadIdx.x / kWave];
    const U4 *pc4 = reinterpret_cast<const U4 *>(A.coef);
    auto coef_chunks = [&](int v, U4 *cp) __attribute__((always_inline)) {
        const int64_t at = g.template coef_row<T>(v) / kPer<T>;
#pragma unroll
        for (int q = 0; q < NQ; ++q) cp[q] = pc4[at + q * kWave];
    };
    auto slot = [&](int v) -> int {
        if constexpr (KR == 4 || KR == 8) return v & (KR - 1);
        else return (v % KR + KR) % KR;
    };
    U4 cpre[NQ];
    for (int v = y0 - 2 * (K - 1); v < y0 - (K - 1); ++v) {
        coef_chunks(v, cpre);
#pragma unroll
        for (int q = 0; q < NQ; ++q) ring[slot(v)][q][w.lane] = cpre[q];
    }
    coef_chunks(y0 - (K - 1), cpre);
    const int r0 = y0 - (K - 1);
#pragma unroll
    for (int i = 0; i < R1 - 1; ++i) load_row<T, W>(r1, g.template offset<T, W>(r0 - 1 + i, n - 1), ra[i]);
#pragma unroll
    for (int i = 0; i < R2 - 1; ++i) load_row<T, W>(r2, g.template offset<T, W>(r0 + i, n - 2), rp[i]);
#pragma unroll
    for (int j = 0; j < K - 1; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < W; ++k) lv[j][i][k] = zero_pair<T, false>();
    double d[3 * K];
#pragma unroll
    for (int i = 0; i < 3 * K; ++i) d[i] = 0.0;
    // FP64: the doubling sums of levels 0 .. NDL-1 collect in LDS, one slot
    // per lane, each added to once per trip; the registers they free hold the
    // a_{n-1} rows three trips ahead (256x256, N = 1024, 64 tiles: 3121-3126
    // ms against 3150-3160 with the sums in registers and the rows one trip
    // ahead; the sums alone in LDS gain nothing, nor do two trips ahead.  W =
    // 4 only: at W = 2, 128x128, N = 512, 140.5-143.0 ms with the sums in
    // registers against 140.1-144.8 ms)
    constexpr int NDL = sizeof(T) == 8 && W >= 4 ? (CBDG_VC_DLDS_F64 < K - 1 ? CBDG_VC_DLDS_F64 : K - 1) : 0;
    __shared__ double dl_all[kVcWaves][NDL > 0 ? 3 * NDL : 1][kWave];
    double (*dl)[kWave] = dl_all[threadIdx.x / kWave];
#pragma unroll
    for (int i = 0; i < 3 * NDL; ++i) dl[i][w.lane] = 0.0;

    // FP64: the two rows a trip stores (levels K-2 and K-1) go out on the next
    // trip, after its loads, so that a wait for those loads never waits for
    // these stores as well (256x256, 64 tiles of 1024 vectors: 3170 -> 3109
    // ms; FP32 1103 -> 1125 ms at N = 2048, so FP32 stores at once).  The
    // offset past the buffer range drops the stores of trips that had nothing
    // to store.
    constexpr bool DEF = !VAR && (sizeof(T) == 8 ? CBDG_VC_DEFER_F64 : CBDG_VC_DEFER_F32);
    P pend5[W], pend6[W];
    unsigned off5 = kOut, off6 = kOut;
#pragma unroll
    for (int k = 0; k < W; ++k) pend5[k] = pend6[k] = zero_pair<T, false>();
    // one trip: w0, w1, w2 = a_{n-1} rows r-1, r, r+1; row r+1+D1 is loaded
    // into w3; p = a_{n-2} row r; row r+D2 is loaded into pn
    auto trip = [&](int r, const P *w0, const P *w1, const P *w2, P *w3, const P *p, P *pn)
                    __attribute__((always_inline)) {
        {
            const int sr = slot(r);
#pragma unroll
            for (int q = 0; q < NQ; ++q) ring[sr][q][w.lane] = cpre[q];
        }
        coef_chunks(r + 1, cpre);
        __builtin_amdgcn_sched_barrier(0);
        load_row<T, W>(r2, g.template offset<T, W>(r + D2, n - 2), pn);
        load_row<T, W>(r1, g.template offset<T, W>(r + 1 + D1, n - 1), w3);
        if constexpr (DEF) {
            store_row<T, W>(ro1, off5, pend5);
            store_row<T, W>(ro2, off6, pend6);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int s = r - j;
            S cj[W];  // coefficients of row s
            {
                const int ss = slot(s);
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const U4 u = ring[ss][q][w.lane];
                    if constexpr (sizeof(T) == 8) {
                        cj[q] = S{__hiloint2double((int)u[1], (int)u[0]), __hiloint2double((int)u[3], (int)u[2])};
                    } else {
                        cj[2 * q] = S{__uint_as_float(u[0]), __uint_as_float(u[1])};
                        cj[2 * q + 1] = S{__uint_as_float(u[2]), __uint_as_float(u[3])};
                    }
                }
            }
            // center, lower and upper rows of level j-1 and row s of level j-2
            const P *cc = j == 0 ? w1 : lv[j - 1][1];
            const P *dd = j == 0 ? w0 : lv[j - 1][0];
            const P *uu = j == 0 ? w2 : lv[j - 1][2];
            const P *pp = j == 0 ? p : (j == 1 ? w0 : lv[j - 2][0]);
            const bool own = (unsigned)(s - y0) < (unsigned)(y1 - y0);  // y0 <= s < y1
            if (VAR && j >= nlev) {
                // past the last level of a shorter pass
            } else if (j < K - 1) {
#pragma unroll
                for (int k = 0; k < W; ++k) { lv[j][0][k] = lv[j][1][k]; lv[j][1][k] = lv[j][2][k]; }
                P *v = lv[j][2];
                // Rows outside the lattice or beyond a_{n+j}'s light cone are
                // zero: they are set so, not computed (a wave-uniform branch).
                // Otherwise a row past an open edge must come out zero.  Its
                // own pairs on the level below and two levels below are zero
                // already (loaded as zero, or computed so on earlier trips), so
                // with the hopping switched off for it the stencil gives zero
                // without a mask: no other row reaches it.
                const bool live = !CBDG_VC_SKIP || (g.in_lattice(s) && g.dy(s) <= n + j);
                if (live) {
                    const T ths = g.in_lattice(s) ? th : T(0);
                    const P hl = dpp_pair<BCX ? kRor1 : kShr1>(cc[W - 1]);
                    const P hr = dpp_pair<BCX ? kRol1 : kShl1>(cc[0]);
#pragma unroll
                    for (int k = 0; k < W; ++k)
                        v[k] = pass_site<T>(cj[k], ths, cc[k], k > 0 ? cc[k - 1] : hl, k < W - 1 ? cc[k + 1] : hr,
                                            dd[k], uu[k], pp[k]);
                } else {
#pragma unroll
                    for (int k = 0; k < W; ++k) v[k] = zero_pair<T, false>();
                }
                if (DEF && j == K - 2) {
                    off5 = own ? g.template offset<T, W>(s, n + j) : kOut;
#pragma unroll
                    for (int k = 0; k < W; ++k) pend5[k] = v[k];
                }
                if (own) {
                    if (live && j < NDL) {
                        double t[3] = {0.0, 0.0, 0.0};
#pragma unroll
                        for (int k = 0; k < W; ++k)
                            dots3(t, (double)v[k].e, (double)v[k].h, (double)cc[k].e, (double)cc[k].h);
#pragma unroll
                        for (int i = 0; i < 3; ++i)
                            __hip_atomic_fetch_add(&dl[3 * j + i][w.lane], t[i], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WAVEFRONT);
                    } else if (live) {
#pragma unroll
                        for (int k = 0; k < W; ++k)
                            dots3(d + 3 * j, (double)v[k].e, (double)v[k].h, (double)cc[k].e, (double)cc[k].h);
                    }
                    if (!DEF && j == nlev - 2) store_row<T, W>(ro1, g.template offset<T, W>(s, n + j), v);
                    if (VAR && j == nlev - 1) store_row<T, W>(ro2, g.template offset<T, W>(s, n + j), v);
                }
            } else if constexpr (DEF) {
                // the last level, kept for the next trip's store
                off6 = kOut;
                if (own && (!CBDG_VC_SKIP || g.dy(s) <= n + j)) {
                    off6 = g.template offset<T, W>(s, n + j);
                    const P hl = dpp_pair<BCX ? kRor1 : kShr1>(cc[W - 1]);
                    const P hr = dpp_pair<BCX ? kRol1 : kShl1>(cc[0]);
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        pend6[k] = pass_site<T>(cj[k], th, cc[k], k > 0 ? cc[k - 1] : hl, k < W - 1 ? cc[k + 1] : hr,
                                                dd[k], uu[k], pp[k]);
                        dots3(d + 3 * j, (double)pend6[k].e, (double)pend6[k].h, (double)cc[k].e, (double)cc[k].h);
                    }
                }
            } else if (own && (!CBDG_VC_SKIP || g.dy(s) <= n + j)) {
                // the last level, stored chunk by chunk
                const unsigned off = g.template offset<T, W>(s, n + j);
                const P hl = dpp_pair<BCX ? kRor1 : kShr1>(cc[W - 1]);
                const P hr = dpp_pair<BCX ? kRol1 : kShl1>(cc[0]);
#pragma unroll
                for (int q = 0; q < W / kPer<T>; ++q) {
                    P v[kPer<T>];
#pragma unroll
                    for (int i = 0; i < kPer<T>; ++i) {
                        const int k = q * kPer<T> + i;
                        v[i] = pass_site<T>(cj[k], th, cc[k], k > 0 ? cc[k - 1] : hl, k < W - 1 ? cc[k + 1] : hr,
                                            dd[k], uu[k], pp[k]);
                        dots3(d + 3 * j, (double)v[i].e, (double)v[i].h, (double)cc[k].e, (double)cc[k].h);
                    }
                    bst<T>(ro2, off + q * (unsigned)(kWave * 16), v);
                }
            }
        }
    };
    // the rings rotate by unrolling: U trips per iteration, U a multiple of
    // both ring lengths
    constexpr int U = R1 % R2 == 0 ? R1 : R1 * R2;
    const int trips = (y1 + K - 2) - r0 + 1;
    const int r_end = r0 + U * ((trips + U - 1) / U);
    __builtin_amdgcn_s_waitcnt(0);
#pragma unroll 1
    for (int r = r0; r < r_end; r += U) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            trip(r + u, ra[u % R1], ra[(u + 1) % R1], ra[(u + 2) % R1], ra[(u + R1 - 1) % R1], rp[u % R2],
                 rp[(u + R2 - 1) % R2]);
    }
    if constexpr (DEF) {
        store_row<T, W>(ro1, off5, pend5);
        store_row<T, W>(ro2, off6, pend6);
    }
#pragma unroll
    for (int i = 0; i < 3 * NDL; ++i) d[i] = dl[i][w.lane];
    wave_sum<3 * K>(d);
    if (w.lane == 0) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (j < nlev) {
                if (A.n_segs == 1) {
                    vc_moments(A, w.b, n + j, d + 3 * j);
                } else {
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        A.part[j * A.pstride + ((int64_t)w.seg * 3 + k) * A.Bp + w.b] = d[3 * j + k];
                }
            }
        }
    }
}

// Reverse passes of the doubling adjoint.  The three-term recursion runs
// backwards as well as forwards, a_{m-1} = 2 Ht a_m - a_{m+1}, so one sweep
// m = M .. 1 regenerates the forward vectors from (a_{M+1}, a_M) beside the
// transposed recursion of the cotangents,
//   lam_m = w_m + 2 Ht lam_{m+1} - lam_{m+2},
//   w_m   = cA a_m + cP a_{m+1} + cQ (-a_{m+1,h}, a_{m+1,e})
//         + cR a_{m-1} + cS (a_{m-1,h}, -a_{m-1,e})   (+ the start-site
//           cotangents of mu[1] at m = 1),
// with no checkpoints: a pass streams two vectors of each recursion in and
// out.  Rounding makes the regenerated a_m differ from the forward ones by a
// few units in the last place per step, and those differences grow at most
// linearly: on each eigenvector of Ht the two-term recursion matrix has its
// eigenvalues e^{+-i theta} on the unit circle, theta kept away from 0 and
// pi by the rescaling's margin.
// Each wavefront (one vector, one row segment) adds c_m lam_m . dHt a_{m-1}
// of its own rows to its vector's G, read and written once per pass; the
// vectors' G are summed in order afterwards.  The rows go through the
// pipeline of the forward passes (trip r computes row r-j of level j); each
// level keeps three-row windows of both recursions, and the gradient terms
// of a row collect in a ring of K rows until its last level has passed.
// Levels per reverse pass and rows of the input vectors loaded ahead, by
// lanes' width W (the trips' unrolling is a common multiple of the two ring
// lengths and K).  W <= 2: six levels, b1/c1 rows three trips ahead (128x128,
// N = 512, all 16384 start vectors in tiles of 1024: 0.627 s with four
// levels one trip ahead, 0.533 s with five levels two ahead, 0.477 s); W = 4
// takes three levels with no rows loaded ahead, its windows being twice as
// wide: deeper rings no longer fit the registers (256x256, N = 1024, two
// tiles of 1024 vectors: four levels one row ahead 1.58 s, spilling 784
// bytes per lane; two levels one row ahead 1.06 s; three levels none ahead
// 0.745 s, 480 registers; three levels one ahead spill 528 bytes).
#ifndef CBDG_VC_ADJ_K
#define CBDG_VC_ADJ_K 6
#endif
#ifndef CBDG_VC_ADJ_D1
#define CBDG_VC_ADJ_D1 3
#endif
#ifndef CBDG_VC_ADJ_D2
#define CBDG_VC_ADJ_D2 1
#endif
template <int W> struct VcAdjShape {
    static constexpr int K = W >= 4 ? 3 : CBDG_VC_ADJ_K;
    static constexpr int D1 = W >= 4 ? 0 : CBDG_VC_ADJ_D1;
    static constexpr int D2 = W >= 4 ? 0 : CBDG_VC_ADJ_D2;
};
constexpr int cx_gcd(int a, int b) { return b == 0 ? a : cx_gcd(b, a % b); }
constexpr int cx_lcm(int a, int b) { return a / cx_gcd(a, b) * b; }
int vc_adj_steps(int Lx)
{
    switch (vc_width(Lx, false)) {
    case 1: return VcAdjShape<1>::K;
    case 2: return VcAdjShape<2>::K;
    case 4: return VcAdjShape<4>::K;
    default: return 0;
    }
}

template <int W, bool BCX, bool BCY, bool VAR>
__global__ __launch_bounds__(kVcBlock) __attribute__((amdgpu_waves_per_eu(1))) void k_vc_adj(VcAdjArgs A)
{
    using T = double;
    using P = Pair<T, false>;
    using S = typename Storage<T, false>::type;
    constexpr int K = VcAdjShape<W>::K;
    static_assert(K >= 2 && K <= 8, "the coefficient ring holds at most eight rows");
    constexpr int kFar = 1 << 29;  // a radius past every lattice: no light-cone clipping
    const int blk = xcd_remap(blockIdx.x, A.nblocks);
    const int seg = blk % A.n_segs;
    const int lane = threadIdx.x % kWave;
    const int b = (blk / A.n_segs) * kVcWaves + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (b >= A.Bt) return;
    const int Lx = A.Lx, Ly = A.Ly;
    const int si = A.sites[b];
    if (si < 0 || si >= Lx * Ly) return;  // an invalid start site adds nothing
    VcGeo<BCX, BCY> g;
    g.Lx = Lx; g.Ly = Ly;
    g.yi = si / Lx; g.xi = si - g.yi * Lx;
    g.lo = lane * W; g.lane = lane;
    const int per = max(4, (Ly + A.n_segs - 1) / A.n_segs);
    const int y0 = seg * per, y1 = min(y0 + per, Ly);
    if (y0 >= y1) return;
    const int m0 = A.m0;
    const int nlev = VAR ? A.nlev : K;
    const bool first = A.first != 0;

    // cotangent coefficients of the pass's levels (wave-uniform)
    double cA[K], cP[K], cQ[K], cR[K], cS[K], cg[K];
    {
        const int N = A.N;
        const int64_t row = (int64_t)b * N;
        auto gee = [&](int i) { return (A.dmu_ee && i >= 2 && i < N) ? A.dmu_ee[row + i] : 0.0; };
        auto ghe = [&](int i) { return (A.dmu_he && i >= 2 && i < N) ? A.dmu_he[row + i] : 0.0; };
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int m = m0 - j;
            const double sg = (m & 1) ? -2.0 : 2.0;  // 2 (-1)^m
            cA[j] = 4.0 * gee(2 * m);
            cP[j] = 2.0 * gee(2 * m + 1);
            cQ[j] = -sg * ghe(2 * m + 1);
            cR[j] = m >= 2 ? 2.0 * gee(2 * m - 1) : 0.0;
            cS[j] = m >= 2 ? sg * ghe(2 * m - 1) : 0.0;
            cg[j] = m == 1 ? 1.0 : 2.0;
        }
    }
    const int j1 = m0 - 1;  // the level of m = 1, if the pass reaches it
    const double we = (j1 >= 0 && j1 < nlev) ? A.d1[2 * b] : 0.0;
    const double wh = (j1 >= 0 && j1 < nlev) ? A.d1[2 * b + 1] : 0.0;
    const bool own_x = lane == g.xi / W;
    const int kx = g.xi % W;

    const auto rb0 = vec_rsrc<T>(A.b0, b, A.Dv), rb1 = vec_rsrc<T>(A.b1, b, A.Dv);
    const auto rc0 = vec_rsrc<T>(A.c0, b, A.Dv), rc1 = vec_rsrc<T>(A.c1, b, A.Dv);
    const auto rbo1 = vec_rsrc<T>(A.bo1, b, A.Dv), rbo2 = vec_rsrc<T>(A.bo2, b, A.Dv);
    const auto rco1 = vec_rsrc<T>(A.co1, b, A.Dv), rco2 = vec_rsrc<T>(A.co2, b, A.Dv);
    const auto rg = vec_rsrc<T>(A.G, b, A.Dv);
    const T th = kCoefScale<T> * T(A.th);
    // row offsets: the forward vectors inside their cones, the cotangents and
    // G over every lattice row (not loaded at all on the first pass)
    auto off_b = [&](int v, int R) -> unsigned { return g.template offset<T, W>(v, R); };
    auto off_c = [&](int v) -> unsigned { return first ? kOut : g.template offset<T, W>(v, kFar); };
    auto own = [&](int v) -> bool { return (unsigned)(v - y0) < (unsigned)(y1 - y0); };

    constexpr int NQ = W / kPer<T>;
    constexpr int KR = K <= 4 ? 4 : 8;
    __shared__ U4 ring_all[kVcWaves][KR][NQ][kWave];
    U4 (*ring)[NQ][kWave] = ring_all[threadIdx.x / kWave];
    const U4 *pc4 = reinterpret_cast<const U4 *>(A.coef);
    auto coef_chunks = [&](int v, U4 *cp) __attribute__((always_inline)) {
        const int64_t at = g.template coef_row<T>(v) / kPer<T>;
#pragma unroll
        for (int q = 0; q < NQ; ++q) cp[q] = pc4[at + q * kWave];
    };
    U4 cpre[NQ];
    for (int v = y0 - 2 * (K - 1); v < y0 - (K - 1); ++v) {
        coef_chunks(v, cpre);
#pragma unroll
        for (int q = 0; q < NQ; ++q) ring[v & (KR - 1)][q][lane] = cpre[q];
    }
    coef_chunks(y0 - (K - 1), cpre);

    // rings of the input rows: b1/c1 rows r-1 .. r+1 and one in flight, b0/c0
    // row r and one in flight
    constexpr int D1 = VcAdjShape<W>::D1, D2 = VcAdjShape<W>::D2;
    constexpr int R1 = 3 + D1, R2 = 1 + D2;
    P ab1[R1][W], ab0[R2][W], ac1[R1][W], ac0[R2][W];
    P wb[K - 1][3][W], wc[K - 1][3][W];  // level j: rows r-j-2, r-j-1, r-j of a_{m0-j-1} and lam_{m0-j}
    P gacc[K][W];                        // gradient terms (eps, Delta) of rows r-K+1 .. r
    P gpre[W];
    const int r0 = y0 - (K - 1);
#pragma unroll
    for (int i = 0; i < R1 - 1; ++i) {
        load_row<T, W>(rb1, off_b(r0 - 1 + i, m0), ab1[i]);
        load_row<T, W>(rc1, off_c(r0 - 1 + i), ac1[i]);
    }
#pragma unroll
    for (int i = 0; i < R2 - 1; ++i) {
        load_row<T, W>(rb0, off_b(r0 + i, m0 + 1), ab0[i]);
        load_row<T, W>(rc0, off_c(r0 + i), ac0[i]);
    }
#pragma unroll
    for (int j = 0; j < K - 1; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < W; ++k) wb[j][i][k] = wc[j][i][k] = zero_pair<T, false>();
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int k = 0; k < W; ++k) gacc[i][k] = zero_pair<T, false>();

    // trip r (u = its place in the unrolled iteration, which fixes the ring
    // slots): bw/cw = b1/c1 rows r-1, r, r+1 and the slot for row r+1+D1,
    // bp/cp = b0/c0 row r and the slot for row r+D2
    auto trip = [&](int r, int u, const P *bw0, const P *bw1, const P *bw2, P *bw3, const P *bp0, P *bpn,
                    const P *cw0, const P *cw1, const P *cw2, P *cw3, const P *cp0, P *cpn)
                    __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) ring[r & (KR - 1)][q][lane] = cpre[q];
        coef_chunks(r + 1, cpre);
        __builtin_amdgcn_sched_barrier(0);
        load_row<T, W>(rb0, off_b(r + D2, m0 + 1), bpn);
        load_row<T, W>(rb1, off_b(r + 1 + D1, m0), bw3);
        load_row<T, W>(rc0, off_c(r + D2), cpn);
        load_row<T, W>(rc1, off_c(r + 1 + D1), cw3);
        const int rg_row = r - (K - 1);
        load_row<T, W>(rg, (!first && own(rg_row)) ? g.template offset<T, W>(rg_row, kFar) : kOut, gpre);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (VAR && j >= nlev) continue;
            const int s = r - j;
            S cj[W];
            {
                const int ss = s & (KR - 1);
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const U4 v = ring[ss][q][lane];
                    cj[q] = S{__hiloint2double((int)v[1], (int)v[0]), __hiloint2double((int)v[3], (int)v[2])};
                }
            }
            // a_m rows s-1, s, s+1 and a_{m+1}(s); lam_{m+1} rows and lam_{m+2}(s)
            const P *bd = j == 0 ? bw0 : wb[j - 1][0];
            const P *bc = j == 0 ? bw1 : wb[j - 1][1];
            const P *bu = j == 0 ? bw2 : wb[j - 1][2];
            const P *bq = j == 0 ? bp0 : (j == 1 ? bw0 : wb[j - 2][0]);
            const P *cd = j == 0 ? cw0 : wc[j - 1][0];
            const P *cc = j == 0 ? cw1 : wc[j - 1][1];
            const P *cu = j == 0 ? cw2 : wc[j - 1][2];
            const P *cq = j == 0 ? cp0 : (j == 1 ? cw0 : wc[j - 2][0]);
            const T ths = g.in_lattice(s) ? th : T(0);
            const bool start_row = j == j1 && g.phys(s) == g.yi && own_x;
            const P bl = dpp_pair<BCX ? kRor1 : kShr1>(bc[W - 1]);
            const P br = dpp_pair<BCX ? kRol1 : kShl1>(bc[0]);
            const P cl = dpp_pair<BCX ? kRor1 : kShr1>(cc[W - 1]);
            const P cr = dpp_pair<BCX ? kRol1 : kShl1>(cc[0]);
            P bn[W], cn[W];
#pragma unroll
            for (int k = 0; k < W; ++k) {
#pragma clang fp contract(off)
                // a_{m-1}(s)
                bn[k] = pass_site<T>(cj[k], ths, bc[k], k > 0 ? bc[k - 1] : bl, k < W - 1 ? bc[k + 1] : br, bd[k],
                                     bu[k], bq[k]);
                // w_m(s)
                double w_e = __builtin_fma(cA[j], bc[k].e, __builtin_fma(cR[j], bn[k].e, cS[j] * bn[k].h));
                double w_h = __builtin_fma(cA[j], bc[k].h, __builtin_fma(cR[j], bn[k].h, -(cS[j] * bn[k].e)));
                w_e = w_e + __builtin_fma(cP[j], bq[k].e, -(cQ[j] * bq[k].h));
                w_h = w_h + __builtin_fma(cP[j], bq[k].h, cQ[j] * bq[k].e);
                if (start_row && k == kx) { w_e = w_e + we; w_h = w_h + wh; }
                // lam_m(s)
                const P l2 = pass_site<T>(cj[k], ths, cc[k], k > 0 ? cc[k - 1] : cl, k < W - 1 ? cc[k + 1] : cr, cd[k],
                                          cu[k], cq[k]);
                cn[k] = P{l2.e + w_e, l2.h + w_h};
            }
            if (own(s)) {
                P *ga = gacc[(u - j + K * 4) % K];
#pragma unroll
                for (int k = 0; k < W; ++k) {
#pragma clang fp contract(off)
                    ga[k].e = __builtin_fma(cg[j], __builtin_fma(cn[k].e, bn[k].e, -(cn[k].h * bn[k].h)), ga[k].e);
                    ga[k].h = __builtin_fma(cg[j], __builtin_fma(cn[k].e, bn[k].h, cn[k].h * bn[k].e), ga[k].h);
                }
                if (!VAR && j == K - 2) {
                    store_row<T, W>(rbo1, off_b(s, m0 - j - 1), bn);
                    store_row<T, W>(rco1, g.template offset<T, W>(s, kFar), cn);
                }
                if (!VAR && j == K - 1) {
                    store_row<T, W>(rbo2, off_b(s, m0 - j - 1), bn);
                    store_row<T, W>(rco2, g.template offset<T, W>(s, kFar), cn);
                }
            }
            if (j < K - 1) {
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    wb[j][0][k] = wb[j][1][k]; wb[j][1][k] = wb[j][2][k]; wb[j][2][k] = bn[k];
                    wc[j][0][k] = wc[j][1][k]; wc[j][1][k] = wc[j][2][k]; wc[j][2][k] = cn[k];
                }
            }
        }
        // row r-K+1 has had all its levels: G += its terms
        P *ga = gacc[(u - (K - 1) + K * 4) % K];
        if (own(rg_row)) {
#pragma unroll
            for (int k = 0; k < W; ++k) { gpre[k].e = gpre[k].e + ga[k].e; gpre[k].h = gpre[k].h + ga[k].h; }
            store_row<T, W>(rg, g.template offset<T, W>(rg_row, kFar), gpre);
        }
#pragma unroll
        for (int k = 0; k < W; ++k) ga[k] = zero_pair<T, false>();
    };
    constexpr int U = cx_lcm(cx_lcm(R1, R2), K);  // a multiple of R1, R2 and K
    static_assert(U <= 12, "unrolling");
    const int trips = (y1 + K - 2) - r0 + 1;
    const int r_end = r0 + U * ((trips + U - 1) / U);
    __builtin_amdgcn_s_waitcnt(0);
#pragma unroll 1
    for (int r = r0; r < r_end; r += U) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            trip(r + u, u, ab1[u % R1], ab1[(u + 1) % R1], ab1[(u + 2) % R1], ab1[(u + R1 - 1) % R1], ab0[u % R2],
                 ab0[(u + R2 - 1) % R2], ac1[u % R1], ac1[(u + 1) % R1], ac1[(u + 2) % R1], ac1[(u + R1 - 1) % R1],
                 ac0[u % R2], ac0[(u + R2 - 1) % R2]);
    }
}

// grad_eps[j] += scale * sum_b G_b(j).e and grad_delta[j] += scale * sum_b
// G_b(j).h over the vectors of valid start sites (the reverse passes never
// touch the others' G), added in order; one thread per pair of the row layout
__global__ void k_vc_grad_reduce(const double2 *__restrict__ G, const int32_t *__restrict__ sites, int Bt, int64_t Dv,
                                 int Lx, int W, int64_t L2, double scale, double *grad_eps, double *grad_delta)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < L2; p += (int64_t)gridDim.x * blockDim.x) {
        double ge = 0.0, gd = 0.0;
        for (int b = 0; b < Bt; ++b) {
            const int32_t sb = sites[b];
            if (sb < 0 || sb >= L2) continue;
            const double2 v = G[b * Dv + p];
            ge += v.x;
            gd += v.y;
        }
        // position p of row y holds column lane * W + k with p % Lx = k * 64 + lane
        const int64_t y = p / Lx;
        const int q = (int)(p - y * Lx);
        const int64_t site = y * Lx + (q % kWave) * W + q / kWave;
        if (grad_eps) grad_eps[site] += scale * ge;
        if (grad_delta) grad_delta[site] += scale * gd;
    }
}

// The same terms kept apart, one row per start vector: rows[b][j] = scale *
// G_b(j).e / .h for a valid start site, zero for the others; one thread per
// (vector, pair of the row layout)
__global__ void k_vc_grad_rows(const double2 *__restrict__ G, const int32_t *__restrict__ sites, int Bt, int64_t Dv,
                               int Lx, int W, int64_t L2, double scale, double *row_eps, double *row_delta, int64_t ld)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)Bt * L2) return;
    const int b = (int)(t / L2);
    const int64_t p = t - (int64_t)b * L2;
    const int32_t sb = sites[b];
    const bool ok = sb >= 0 && sb < L2;
    const double2 v = ok ? G[b * Dv + p] : make_double2(0.0, 0.0);
    const int64_t y = p / Lx;
    const int q = (int)(p - y * Lx);
    const int64_t site = y * Lx + (q % kWave) * W + q / kWave;
    if (row_eps) row_eps[b * ld + site] = scale * v.x;
    if (row_delta) row_delta[b * ld + site] = scale * v.y;
}

// a_0 = |s_b, e> in the vector-contiguous layout, and the zeroth moments; an
// invalid start site leaves its vector untouched (no pass reads or writes it)
// and its moment row NaN.
template <typename T>
__global__ void k_vc_seed(typename Storage<T, false>::type *a0, int64_t Dv, int Lx, int W, int Bt, int64_t L2,
                          const int32_t *sites, double *mu_ee, double *mu_he, int N)
{
    // one thread per (vector, pair of the start row)
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)Bt * Lx) return;
    const int b = (int)(t / Lx), k = (int)(t % Lx);
    const int64_t s = sites[b];
    const int64_t m = (int64_t)b * N;
    if (s < 0 || s >= L2) {
        if (k == 0) {
            const double nan = __builtin_nan("");
            for (int n = 0; n < N; ++n) { mu_ee[m + n] = nan; mu_he[m + n] = nan; }
        }
        return;
    }
    // the whole start row: every pair the first step reads of a_0 (the
    // owner lane's W pairs on open rows, all lanes on periodic ones)
    const int64_t y = s / Lx, x = s % Lx;
    const int one = pair_pos<T>((int)(x / W), (int)(x % W));
    a0[b * Dv + y * Lx + k] = typename Storage<T, false>::type{k == one ? T(1) : T(0), T(0)};
    if (k == 0) {
        mu_ee[m] = 1.0;
        mu_he[m] = 0.0;
    }
}

// Packed (de, Delta/a) of every site in the row layout of the passes.
template <typename T>
__global__ void k_vc_coef(const OnSite<T> *__restrict__ ons, typename Storage<T, false>::type *__restrict__ pc,
                          int Lx, int W, int64_t L2)
{
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < L2; s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t y = s / Lx, x = s % Lx;
        const OnSite<T> o = ons[s];
        pc[y * Lx + pair_pos<T>((int)(x / W), (int)(x % W))] =
            typename Storage<T, false>::type{kCoefScale<T> * o.de, kCoefScale<T> * o.dr};
    }
}

#ifndef CBDG_VC
#define CBDG_VC 1
#endif
// Wavefronts a pass aims for: enough row segments per vector that a tile
// of Bt vectors gives at least this many.
#ifndef CBDG_VC_WAVES
#define CBDG_VC_WAVES 1024
#endif

int vc_width(int Lx, bool f32)
{
    if (!CBDG_VC || Lx % kWave) return 0;
    const int W = Lx / kWave;
    if (f32) return (W == 2 || W == 4) ? W : 0;  // two FP32 pairs per access
    return (W == 1 || W == 2 || W == 4) ? W : 0;
}

int vc_segments(int Ly, int Bt, int steps)
{
    (void)steps;
    const int want = (int)ceil_div(CBDG_VC_WAVES, std::max(Bt, 1));
    return std::max(1, std::min(want, Ly / 16));
}

template <typename T, int W, bool BCX, bool BCY>
static int launch_vc_w(VcArgs A, int steps, hipStream_t st)
{
    const int64_t nb = ceil_div(A.Bt, kVcWaves) * (int64_t)A.n_segs;
    if (nb > INT32_MAX) return fail(CBDG_EINVAL, "chebyshev_moments: launch grid too large");
    A.nblocks = (int)nb;
    constexpr int K = kVcSteps<T>;
    if (steps == K) {
        hipLaunchKernelGGL((k_vc_pass<T, W, BCX, BCY, K, false>), dim3(A.nblocks), dim3(kVcBlock), 0, st, A);
    } else if (steps >= 2) {
        A.nlev = steps;
        hipLaunchKernelGGL((k_vc_pass<T, W, BCX, BCY, K, true>), dim3(A.nblocks), dim3(kVcBlock), 0, st, A);
    } else if (A.n == 1) hipLaunchKernelGGL((k_vc_step1<T, W, BCX, BCY, true>), dim3(A.nblocks), dim3(kVcBlock), 0, st, A);
    else hipLaunchKernelGGL((k_vc_step1<T, W, BCX, BCY, false>), dim3(A.nblocks), dim3(kVcBlock), 0, st, A);
    CBDG_CHECK_LAUNCH(steps == 1 ? "k_vc_step1" : "k_vc_pass");
    return CBDG_OK;
}

template <typename T, int W>
static int launch_vc_bc(const VcArgs &A, int steps, hipStream_t st)
{
    if (A.bcx) return A.bcy ? launch_vc_w<T, W, true, true>(A, steps, st) : launch_vc_w<T, W, true, false>(A, steps, st);
    return A.bcy ? launch_vc_w<T, W, false, true>(A, steps, st) : launch_vc_w<T, W, false, false>(A, steps, st);
}

template <typename T>
static int launch_vc_t(const VcArgs &A, int steps, hipStream_t st)
{
    switch (vc_width(A.Lx, std::is_same<T, float>::value)) {
    case 1:
        if constexpr (std::is_same<T, double>::value) return launch_vc_bc<T, 1>(A, steps, st);
        break;
    case 2: return launch_vc_bc<T, 2>(A, steps, st);
    case 4: return launch_vc_bc<T, 4>(A, steps, st);
    default: break;
    }
    return fail(CBDG_EUNSUPPORTED, "vector-contiguous pass: Lx = %d is not 64 times a supported width", A.Lx);
}

int launch_vc_seed(void *a0, int64_t Dv, int Lx, bool f32, int Bt, int64_t L2, const int32_t *sites, double *mu_ee,
                   double *mu_he, int N, hipStream_t st)
{
    const int W = vc_width(Lx, f32);
    if (!W) return fail(CBDG_EUNSUPPORTED, "vector-contiguous pass: Lx = %d does not fit", Lx);
    if (f32)
        hipLaunchKernelGGL((k_vc_seed<float>), dim3((unsigned)ceil_div((int64_t)Bt * Lx, kBlock)), dim3(kBlock), 0, st,
                           reinterpret_cast<float2 *>(a0), Dv, Lx, W, Bt, L2, sites, mu_ee, mu_he, N);
    else
        hipLaunchKernelGGL((k_vc_seed<double>), dim3((unsigned)ceil_div((int64_t)Bt * Lx, kBlock)), dim3(kBlock), 0, st,
                           reinterpret_cast<double2 *>(a0), Dv, Lx, W, Bt, L2, sites, mu_ee, mu_he, N);
    CBDG_CHECK_LAUNCH("k_vc_seed");
    return CBDG_OK;
}

int launch_vc_coef(const void *onsite, void *coef, int Lx, bool f32, int64_t L2, hipStream_t st)
{
    const int W = vc_width(Lx, f32);
    if (!W) return fail(CBDG_EUNSUPPORTED, "vector-contiguous pass: Lx = %d does not fit", Lx);
    const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(L2, kBlock), 4096);
    if (f32)
        hipLaunchKernelGGL((k_vc_coef<float>), dim3(grid), dim3(kBlock), 0, st,
                           reinterpret_cast<const OnSite<float> *>(onsite), reinterpret_cast<float2 *>(coef), Lx, W, L2);
    else
        hipLaunchKernelGGL((k_vc_coef<double>), dim3(grid), dim3(kBlock), 0, st,
                           reinterpret_cast<const OnSite<double> *>(onsite), reinterpret_cast<double2 *>(coef), Lx, W, L2);
    CBDG_CHECK_LAUNCH("k_vc_coef");
    return CBDG_OK;
}

int vc_steps(bool f32) { return f32 ? kVcSteps<float> : kVcSteps<double>; }

template <int W, bool BCX, bool BCY>
static int launch_vc_adj_w(VcAdjArgs A, bool full, hipStream_t st)
{
    const int64_t nb = ceil_div(A.Bt, kVcWaves) * (int64_t)A.n_segs;
    if (nb > INT32_MAX) return fail(CBDG_EINVAL, "chebyshev_moments_backward: launch grid too large");
    A.nblocks = (int)nb;
    if (full) hipLaunchKernelGGL((k_vc_adj<W, BCX, BCY, false>), dim3(A.nblocks), dim3(kVcBlock), 0, st, A);
    else hipLaunchKernelGGL((k_vc_adj<W, BCX, BCY, true>), dim3(A.nblocks), dim3(kVcBlock), 0, st, A);
    CBDG_CHECK_LAUNCH("k_vc_adj");
    return CBDG_OK;
}

template <int W>
static int launch_vc_adj_bc(const VcAdjArgs &A, bool full, hipStream_t st)
{
    if (A.bcx)
        return A.bcy ? launch_vc_adj_w<W, true, true>(A, full, st) : launch_vc_adj_w<W, true, false>(A, full, st);
    return A.bcy ? launch_vc_adj_w<W, false, true>(A, full, st) : launch_vc_adj_w<W, false, false>(A, full, st);
}

int launch_vc_adj(VcAdjArgs A, bool full, hipStream_t st)
{
    const int K = vc_adj_steps(A.Lx);
    if (!full && (A.nlev < 1 || A.nlev > K))
        return fail(CBDG_EINVAL, "chebyshev_moments_backward: reverse pass of %d levels", A.nlev);
    if (full && A.m0 < K) return fail(CBDG_EINVAL, "chebyshev_moments_backward: full reverse pass below m = K");
    if (A.Dv * 16 > INT32_MAX) return fail(CBDG_EINVAL, "chebyshev_moments_backward: lattice too large");
    if (A.n_segs < 1) return fail(CBDG_EINVAL, "chebyshev_moments_backward: no row segments");
    switch (vc_width(A.Lx, false)) {
    case 1: return launch_vc_adj_bc<1>(A, full, st);
    case 2: return launch_vc_adj_bc<2>(A, full, st);
    case 4: return launch_vc_adj_bc<4>(A, full, st);
    default: break;
    }
    return fail(CBDG_EUNSUPPORTED, "reverse pass: Lx = %d is not 64 times a supported width", A.Lx);
}

int launch_vc_grad_reduce(const double *G, const int32_t *sites, int Bt, int64_t Dv, int Lx, int64_t L2, double scale,
                          double *grad_eps, double *grad_delta, hipStream_t st)
{
    const int W = vc_width(Lx, false);
    if (!W) return fail(CBDG_EUNSUPPORTED, "reverse pass: Lx = %d does not fit", Lx);
    const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(L2, kBlock), 4096);
    hipLaunchKernelGGL(k_vc_grad_reduce, dim3(grid), dim3(kBlock), 0, st, reinterpret_cast<const double2 *>(G), sites,
                       Bt, Dv, Lx, W, L2, scale, grad_eps, grad_delta);
    CBDG_CHECK_LAUNCH("k_vc_grad_reduce");
    return CBDG_OK;
}

int launch_vc_grad_rows(const double *G, const int32_t *sites, int Bt, int64_t Dv, int Lx, int64_t L2, double scale,
                        double *row_eps, double *row_delta, int64_t ld, hipStream_t st)
{
    const int W = vc_width(Lx, false);
    if (!W) return fail(CBDG_EUNSUPPORTED, "reverse pass: Lx = %d does not fit", Lx);
    const int64_t nb = ceil_div((int64_t)Bt * L2, kBlock);
    if (nb > INT32_MAX) return fail(CBDG_EINVAL, "jacobian: launch grid too large");
    hipLaunchKernelGGL(k_vc_grad_rows, dim3((unsigned)nb), dim3(kBlock), 0, st, reinterpret_cast<const double2 *>(G),
                       sites, Bt, Dv, Lx, W, L2, scale, row_eps, row_delta, ld);
    CBDG_CHECK_LAUNCH("k_vc_grad_rows");
    return CBDG_OK;
}

int launch_vc(const VcArgs &A, int steps, bool f32, hipStream_t st)
{
    if (steps < 1 || steps > vc_steps(f32)) return fail(CBDG_EINVAL, "vector-contiguous pass: %d steps", steps);
    if (A.Dv * 16 > INT32_MAX) return fail(CBDG_EINVAL, "vector-contiguous pass: lattice too large");
    return f32 ? launch_vc_t<float>(A, steps, st) : launch_vc_t<double>(A, steps, st);
}

}  // namespace cbdg
