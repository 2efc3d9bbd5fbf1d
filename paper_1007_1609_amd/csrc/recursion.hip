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
//   - each lane owns a strip of W sites along x (W divides Lx, so every
//     strip is full) and marches up a segment of rows in y, keeping rows y-1, y, y+1 of a_{n-1} in registers, so a_{n-1}
//     is read about once (plus the strip's x halo and the segment's y halo,
//     which neighbouring strips on the same XCD fetch at nearly the same time);
//   - a_{n-2} is read and a_n written by the same lane at the same address.
#include "step.hpp"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace cbdg {

// Load/store flavours of the three streams (1 = nontemporal) and extra
// padding of the lane stride.  a_{n-2} and a_n are touched once per step and
// stream past the caches; a_{n-1} is read through L2, where neighbouring
// strips and row segments pick up each other's halo columns and rows.
// Measured on MI355X (256x256, 1024 vectors, FP64): nontemporal a_{n-2}/a_n
// cut the step from 719 to 665 us at W = 4; a nontemporal a_{n-1} or a
// padded lane stride did not help.
#ifndef CBDG_NT_A1
#define CBDG_NT_A1 0
#endif
#ifndef CBDG_NT_A2
#define CBDG_NT_A2 1
#endif
#ifndef CBDG_NT_OUT
#define CBDG_NT_OUT 1
#endif
// Multi-step passes: issue the loads of the a_{n-2} row a pass consumes in the
// same iteration before the prefetch of the next a_{n-1} row (loads complete
// in order, so waiting for a_{n-2} then leaves the prefetch in flight).
// FP64 two-step, 256x256, 1024 vectors: 198.4 -> 191.5 us per moment index
// (spread start sites), 154.7 -> 148.7 (a block of rows); FP32 three-step
// 1 % faster.  A pipeline two rows deep (a_{n-2} one row and a_{n-1} two
// rows ahead, buffers alternating over a loop unrolled by two) needs the
// AGPRs as spill space and was slower: W = 4 239.7, W = 2 283.5 us.
#ifndef CBDG_A2_FIRST
#define CBDG_A2_FIRST 1
#endif
// Three-step passes: a_{n-2} loaded one row ahead, so each trip computes from
// registers while the next rows of a_{n-1} and a_{n-2} arrive.  FP32, one
// 1024-vector tile at 256x256: 90.9 -> 85.0 us per moment index (spread
// start sites), 80.8 -> 75.6 (a block of rows).  FP64 three-step (one wave
// per SIMD, windows partly in AGPRs) is faster without it: 186.9 / 142.2 us
// against 188.1 / 143.6 at 128-row segments, 163.6 / 127.0 against
// 169.0 / 131.5 at 256 rows.  The same prefetch in the FP64 two-step pass was
// slower too (W = 8: 192.8 -> 197.3 us; W = 4: 226.9 us).
#ifndef CBDG_PF3_F32
#define CBDG_PF3_F32 1
#endif
#ifndef CBDG_PF3_F64
#define CBDG_PF3_F64 0
#endif

#ifndef CBDG_LANE_PAD
#define CBDG_LANE_PAD 0
#endif
// Unrolling of the three-step row loop.  FP32 (two waves per SIMD), one
// 1024-vector tile at 256x256, N = 2048: 455.4 us per launch unrolled once,
// 446.0 twice, 441.0 three times (241 / 252 VGPRs, bits unchanged); the FP64
// loop is not unrolled by the compiler either way (782 us).
#ifndef CBDG_U3
#define CBDG_U3 3
#endif


// MODE 0: moments at the start site; 1: also the moment-doubling partial sums;
// 2: also the values at the four neighbours of the start site.
template <typename T, bool C, bool GEN, bool FIRST, int W, bool PF, int MODE>
__global__ __launch_bounds__(kBlock) void k_cheb_step(
    StepArgs A, const typename Storage<T, C>::type *__restrict__ a1,
    const OnSite<T> *__restrict__ ons, const void *__restrict__ bonds)
{
    constexpr bool DOT = MODE == 1, NB = MODE == 2;
    using P = Pair<T, C>;
    using S = typename Storage<T, C>::type;
    const int lb = xcd_remap(blockIdx.x, A.nblocks);
    const int strip = lb % A.n_strips;
    const int rest = lb / A.n_strips;
    const int seg = rest % A.n_segs;
    const int chunk = rest / A.n_segs;
    const uint32_t b = chunk * kBlock + threadIdx.x;
    if (b >= (uint32_t)A.Bt) return;

    const int Lx = A.Lx, Ly = A.Ly;
    const int x0 = strip * W;
    int y0 = seg * A.ys;
    int y1 = min(y0 + A.ys, Ly);
    const int64_t Bp = A.Bp;
    // Light cone: H has nearest-neighbour range, so a_n vanishes farther than
    // n sites (in x or y) from every start site; a_{n-2} (the output buffer)
    // vanishes there too, so those strips and rows are left as they are.  The
    // rows inside the cone are shared out evenly over the launch's segments
    // (at least 4 rows each), so early steps still spread over the GPU.  The
    // first step writes every site (its output buffer is not cleared).
    if constexpr (!FIRST) {
        if (A.cone) {
            const int n = A.n;
            bool skip = false;
            if (!A.bcx) skip = x0 + W - 1 < A.cone[0] - n || x0 > A.cone[1] + n;
            if (!A.bcy) {
                const int ylo = max(0, A.cone[2] - n), yhi = min(Ly - 1, A.cone[3] + n);
                const int rows = yhi - ylo + 1;
                const int per = max(4, (rows + A.n_segs - 1) / A.n_segs);
                y0 = ylo + seg * per;
                y1 = min(y0 + per, yhi + 1);
                skip = skip || rows <= 0 || y0 >= y1;
            }
            if (skip) {
                if constexpr (DOT) {
                    constexpr int K = C ? 4 : 3;
                    double *pp = A.part + (strip + (int64_t)A.n_strips * seg) * K * Bp + b;
#pragma unroll
                    for (int k = 0; k < K; ++k) pp[k * Bp] = 0.0;
                }
                return;
            }
        }
    }
    // a1 (a_{n-1}) is never written by this launch -- out aliases a_{n-2}
    // only -- and the coefficients are read-only, which lets the wave-uniform
    // coefficient reads become scalar loads.  Addresses are a wave-uniform
    // base (site * Bp) plus the lane's vector index.
    const S *a2 = reinterpret_cast<const S *>(A.prev2);
    S *ao = reinterpret_cast<S *>(A.out);
    const int my_site = A.sites[b];
    const T th = T(A.th);
    // neighbours +x, -x, +y, -y of the start site (-1: none)
    [[maybe_unused]] int nbs[4] = {-1, -1, -1, -1};
    [[maybe_unused]] bool nbf[4] = {false, false, false, false};
    [[maybe_unused]] P nbv[NB ? 4 : 1];
    if constexpr (NB) {
        if (my_site >= 0 && my_site < Lx * Ly) {
            const int mx = my_site % Lx, my = my_site / Lx;
            if (mx + 1 < Lx) nbs[0] = my_site + 1; else if (A.bcx) nbs[0] = my_site + 1 - Lx;
            if (mx > 0) nbs[1] = my_site - 1; else if (A.bcx) nbs[1] = my_site - 1 + Lx;
            if (my + 1 < Ly) nbs[2] = my_site + Lx; else if (A.bcy) nbs[2] = my_site + Lx - Lx * Ly;
            if (my > 0) nbs[3] = my_site - Lx; else if (A.bcy) nbs[3] = my_site - Lx + Lx * Ly;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) nbv[q] = zero_pair<T, C>();
    }

    // Column k of the register window holds x = x0 - 1 + k.  Every column gets
    // an in-bounds column index and a mask; a column outside an open lattice is
    // loaded from a valid column and its bits cleared, so each row is one
    // branch-free clause of loads.
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
    // Raw loads of row y; returns the row's mask (masks are applied by
    // apply_mask once the loads have had time to land).
    auto load_row = [&](P *row, int y) -> uint32_t {
        bool ok = true;
        int yy = y;
        if (y < 0) { ok = A.bcy != 0; yy = A.bcy ? y + Ly : 0; }
        else if (y >= Ly) { ok = A.bcy != 0; yy = A.bcy ? y - Ly : Ly - 1; }
        const int64_t rbase = (int64_t)yy * Lx;
#pragma unroll
        for (int k = 0; k < W + 2; ++k) {
            const S *q = a1 + (rbase + cx[k]) * Bp + b;
            row[k] = CBDG_NT_A1 ? ld_nt<T, C>(q) : ld<T, C>(q);
        }
        return ok ? ~0u : 0u;
    };
    auto apply_mask = [&](P *row, uint32_t rm) {
#pragma unroll
        for (int k = 0; k < W + 2; ++k) row[k] = masked<T, C>(row[k], rm & cm[k]);
    };
    auto load_prev2 = [&](P *row, int y) {
        const int64_t rbase = (int64_t)y * Lx;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const S *q = a2 + (rbase + x0 + k) * Bp + b;
            row[k] = CBDG_NT_A2 ? ld_nt<T, C>(q) : ld<T, C>(q);
        }
    };

    // Rows y-1, y, y+1 of a_{n-1} and row y of a_{n-2} are in registers while
    // row y is computed; the loads for row y+1 are issued first so their
    // latency overlaps the arithmetic and the stores of row y.  The lane's own
    // moment is captured with a select and stored once at the end, so the
    // loop body issues a fixed number of memory operations.
    P up[W + 2], cur[W + 2], dn[W + 2], nx[W + 2], pc[W];
    [[maybe_unused]] P pn[PF ? W : 1];
    P mval = zero_pair<T, C>();
    bool found = false;
    // moment doubling: per-lane partial sums over this block's sites of
    // <a_n|a_n>, Re<a_n|a_{n-1}> and the bilinear form
    // B(a_n, a_{n-1}) = sum_i u_n(i) v_{n-1}(i) - v_n(i) u_{n-1}(i), in FP64
    double d_nn = 0.0, d_nm = 0.0, d_br = 0.0, d_bi = 0.0;
    apply_mask(up, load_row(up, y0 - 1));
    apply_mask(cur, load_row(cur, y0));
    apply_mask(dn, load_row(dn, y0 + 1));
    if constexpr (!FIRST && PF) load_prev2(pc, y0);

    auto compute_row = [&](int y) {
        const int64_t srow = (int64_t)y * Lx;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int x = x0 + k;
            const int64_t s = srow + x;
            const OnSite<T> o = ons[s];
            P yv;
            if constexpr (GEN) {
                const int64_t sl = x > 0 ? s - 1 : (A.bcx ? s + Lx - 1 : -1);
                const int64_t sd = y > 0 ? s - Lx : (A.bcy ? s + (int64_t)(Ly - 1) * Lx : -1);
                Link<T, C> lk[4];
                links_of<T, C>(bonds, s, sl, sd, lk);
                P nb[4] = {cur[k + 2], cur[k], dn[k + 1], up[k + 1]};
                yv = apply_general<T, C>(o, cur[k + 1], nb, lk);
            } else {
                yv = apply_uniform<T, C>(o, th, cur[k + 1], cur[k], cur[k + 2], up[k + 1], dn[k + 1]);
            }
            P ov;
            if constexpr (FIRST) ov = yv;
            else ov = cheb_combine<T, C>(yv, pc[k], false);
            if constexpr (CBDG_NT_OUT) st_nt<T, C>(ao + s * Bp + b, ov);
            else st<T, C>(ao + s * Bp + b, ov);
            const bool hit = s == my_site;
            found = found || hit;
            mval = select_pair<T, C>(hit, ov, mval);
            if constexpr (NB) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool hq = s == nbs[q];
                    nbf[q] = nbf[q] || hq;
                    nbv[q] = select_pair<T, C>(hq, ov, nbv[q]);
                }
            }
            if constexpr (DOT) {
                const P &c = cur[k + 1];
                if constexpr (C) {
                    const double er = ov.er, ei = ov.ei, hr = ov.hr, hi = ov.hi;
                    const double cer = c.er, cei = c.ei, chr = c.hr, chi = c.hi;
                    d_nn += (er * er + ei * ei) + (hr * hr + hi * hi);
                    d_nm += (er * cer + ei * cei) + (hr * chr + hi * chi);
                    d_br += (er * chr - ei * chi) - (hr * cer - hi * cei);
                    d_bi += (er * chi + ei * chr) - (hr * cei + hi * cer);
                } else {
                    const double e = ov.e, h = ov.h, ce = c.e, ch = c.h;
                    d_nn += e * e + h * h;
                    d_nm += e * ce + h * ch;
                    d_br += e * ch - h * ce;
                }
            }
        }
    };
    // one row per trip: unrolling would duplicate the register window
#pragma unroll 1
    for (int y = y0; y < y1 - 1; ++y) {
        // without the a_{n-2} prefetch its loads go first, so waiting for
        // them does not wait for the next row of a_{n-1}
        if constexpr (!FIRST && !PF) load_prev2(pc, y);
        const uint32_t nm = load_row(nx, y + 2);
        if constexpr (!FIRST && PF) load_prev2(pn, y + 1);
        compute_row(y);
        apply_mask(nx, nm);
#pragma unroll
        for (int k = 0; k < W + 2; ++k) { up[k] = cur[k]; cur[k] = dn[k]; dn[k] = nx[k]; }
        if constexpr (!FIRST && PF) {
#pragma unroll
            for (int k = 0; k < W; ++k) pc[k] = pn[k];
        }
    }
    if constexpr (!FIRST && !PF) load_prev2(pc, y1 - 1);
    compute_row(y1 - 1);

    if constexpr (DOT) {
        constexpr int K = C ? 4 : 3;
        const int64_t region = strip + (int64_t)A.n_strips * seg;
        double *pp = A.part + region * K * Bp + b;
        pp[0] = d_nn;
        pp[Bp] = d_nm;
        pp[2 * Bp] = d_br;
        if constexpr (C) pp[3 * Bp] = d_bi;
    }
    if (found && A.mu_ee) {
        const int64_t m = (int64_t)b * A.N + A.n;
        if constexpr (C) {
            A.mu_ee[m] = (double)mval.er;
            A.mu_he[2 * m] = (double)mval.hr;
            A.mu_he[2 * m + 1] = (double)mval.hi;
        } else {
            A.mu_ee[m] = (double)mval.e;
            A.mu_he[m] = (double)mval.h;
        }
    }
    if constexpr (NB) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (!nbf[q]) continue;
            const int64_t m = ((int64_t)b * 4 + q) * A.N + A.n;
            if constexpr (C) {
                A.nb_ee[2 * m] = (double)nbv[q].er;
                A.nb_ee[2 * m + 1] = (double)nbv[q].ei;
                A.nb_he[2 * m] = (double)nbv[q].hr;
                A.nb_he[2 * m + 1] = (double)nbv[q].hi;
            } else {
                A.nb_ee[m] = (double)nbv[q].e;
                A.nb_he[m] = (double)nbv[q].h;
            }
        }
    }
}

// Neighbour-moment rows [Bt][4][N]: zero (n = 0, and missing neighbours), NaN
// for invalid start sites.
__global__ void k_seed_nb(double *nb_ee, double *nb_he, const int32_t *sites, int Bt, int64_t L2, int N, int cplx)
{
    const int64_t per = (int64_t)4 * N * (cplx ? 2 : 1);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)Bt * per;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = sites[i / per];
        const double v = (s < 0 || s >= L2) ? __builtin_nan("") : 0.0;
        nb_ee[i] = v;
        nb_he[i] = v;
    }
}

// Two recursion steps in one pass:
//     a_n     = 2 Ht a_{n-1} - a_{n-2}   (into A.out)
//     a_{n+1} = 2 Ht a_n     - a_{n-1}   (into A.out2)
// from a_{n-2} (A.prev2) and a_{n-1} (a1); the four buffers are distinct.  A
// lane computes a_n on its strip widened by one column on each side and on
// one row beyond each end of its segment (reading a_{n-1} two columns and two
// rows out, a_{n-2} one out), so a_{n+1} needs nothing from other
// workgroups.  Per two steps the vectors cross HBM four times (read a_{n-2},
// a_{n-1}; write a_n, a_{n+1}) instead of six; the widened a_n costs extra
// arithmetic and L2 reads only.  GEN: per-bond hopping and pairing (links of
// the site and of its -x and -y neighbours, scalar loads).
//
// Row r of a_n is computed with rows r-1, r, r+1 of a_{n-1} in registers;
// row r-1 of a_{n+1} follows from rows r-2, r-1, r of a_n.  Columns: a_{n-1}
// at x0-2 .. x0+W+1 (index k <-> x0-2+k), a_n at x0-1 .. x0+W (k <-> x0-1+k).
template <typename T, bool C, bool GEN, int W, bool DOT>
__global__ __launch_bounds__(kBlock) void k_cheb_step2(StepArgs A, const typename Storage<T, C>::type *__restrict__ a1,
                                                      const OnSite<T> *__restrict__ ons,
                                                      const void *__restrict__ bonds)
{
    using P = Pair<T, C>;
    using S = typename Storage<T, C>::type;
    constexpr int X = W + 2, Y = W + 4;
    constexpr int K = C ? 4 : 3;
    const int lb = xcd_remap(blockIdx.x, A.nblocks);
    const int strip = lb % A.n_strips;
    const int rest = lb / A.n_strips;
    const int seg = rest % A.n_segs;
    const int chunk = rest / A.n_segs;
    const uint32_t b = chunk * kBlock + threadIdx.x;
    if (b >= (uint32_t)A.Bt) return;

    const int Lx = A.Lx, Ly = A.Ly;
    const int x0 = strip * W;
    int y0 = seg * A.ys;
    int y1 = min(y0 + A.ys, Ly);
    const int64_t Bp = A.Bp;
    const int64_t region = strip + (int64_t)A.n_strips * seg;
    // light cone of a_{n+1} (that of a_n lies inside it); rows inside are
    // shared out over the segments as in the one-step kernel
    if (A.cone) {
        const int m = A.n + 1;
        bool skip = false;
        if (!A.bcx) skip = x0 + W - 1 < A.cone[0] - m || x0 > A.cone[1] + m;
        if (!A.bcy) {
            const int ylo = max(0, A.cone[2] - m), yhi = min(Ly - 1, A.cone[3] + m);
            const int rows = yhi - ylo + 1;
            const int per = max(4, (rows + A.n_segs - 1) / A.n_segs);
            y0 = ylo + seg * per;
            y1 = min(y0 + per, yhi + 1);
            skip = skip || rows <= 0 || y0 >= y1;
        }
        if (skip) {
            if constexpr (DOT) {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    A.part[(region * K + k) * Bp + b] = 0.0;
                    A.part_b[(region * K + k) * Bp + b] = 0.0;
                }
            }
            return;
        }
    }
    const S *a2 = reinterpret_cast<const S *>(A.prev2);
    S *ao = reinterpret_cast<S *>(A.out);
    S *ao2 = reinterpret_cast<S *>(A.out2);
    const int my_site = A.sites[b];
    const T th = T(A.th);

    // columns x0-2+k: an in-bounds index and a mask (0 outside an open lattice)
    int cx[Y];
    uint32_t cm[Y];
#pragma unroll
    for (int k = 0; k < Y; ++k) {
        const int x = x0 - 2 + k;
        if (A.bcx) {
            cx[k] = ((x % Lx) + Lx) % Lx;
            cm[k] = ~0u;
        } else {
            const bool ok = x >= 0 && x < Lx;
            cx[k] = ok ? x : (x < 0 ? 0 : Lx - 1);
            cm[k] = ok ? ~0u : 0u;
        }
    }
    // in-bounds row index of y and its mask
    auto row_y = [&](int y, uint32_t &ok) -> int {
        if (A.bcy) { ok = ~0u; return ((y % Ly) + Ly) % Ly; }
        const bool in = y >= 0 && y < Ly;
        ok = in ? ~0u : 0u;
        return in ? y : (y < 0 ? 0 : Ly - 1);
    };
    auto load_row1 = [&](P *row, int y) -> uint32_t {
        uint32_t ok;
        const int64_t rb = (int64_t)row_y(y, ok) * Lx;
#pragma unroll
        for (int k = 0; k < Y; ++k) row[k] = ld<T, C>(a1 + (rb + cx[k]) * Bp + b);
        return ok;
    };
    auto mask_row1 = [&](P *row, uint32_t rm) {
#pragma unroll
        for (int k = 0; k < Y; ++k) row[k] = masked<T, C>(row[k], rm & cm[k]);
    };
    // (Ht v)(s) at column xc, row yy from the centre and its four neighbours
    auto apply = [&](int64_t s, int xc, int yy, const P &c, const P &l, const P &r, const P &up, const P &dn) -> P {
        const OnSite<T> o = ons[s];
        if constexpr (GEN) {
            const int64_t sl = xc > 0 ? s - 1 : (A.bcx ? s + Lx - 1 : -1);
            const int64_t sd = yy > 0 ? s - Lx : (A.bcy ? s + (int64_t)(Ly - 1) * Lx : -1);
            Link<T, C> lk[4];
            links_of<T, C>(bonds, s, sl, sd, lk);
            const P nb[4] = {r, l, dn, up};  // +x, -x, +y, -y
            return apply_general<T, C>(o, c, nb, lk);
        } else {
            return apply_uniform<T, C>(o, th, c, l, r, up, dn);
        }
    };
    auto dots = [&](double *acc, const P &v, const P &c) {
        if constexpr (C) {
            const double er = v.er, ei = v.ei, hr = v.hr, hi = v.hi;
            const double cer = c.er, cei = c.ei, chr = c.hr, chi = c.hi;
            acc[0] += (er * er + ei * ei) + (hr * hr + hi * hi);
            acc[1] += (er * cer + ei * cei) + (hr * chr + hi * chi);
            acc[2] += (er * chr - ei * chi) - (hr * cer - hi * cei);
            acc[3] += (er * chi + ei * chr) - (hr * cei + hi * cer);
        } else {
            const double e = v.e, h = v.h, ce = c.e, ch = c.h;
            acc[0] += e * e + h * h;
            acc[1] += e * ce + h * ch;
            acc[2] += e * ch - h * ce;
        }
    };

    P w0[Y], w1[Y], w2[Y], nx[Y];      // a_{n-1} rows r-1, r, r+1, r+2
    P m2[X], m1[X], m0[X];             // a_n rows r-2, r-1, r
    P p2[X];                           // a_{n-2} row r
    P mval = zero_pair<T, C>(), mval1 = zero_pair<T, C>();
    bool found = false, found1 = false;
    double d0[K], d1[K];
#pragma unroll
    for (int k = 0; k < K; ++k) { d0[k] = 0.0; d1[k] = 0.0; }
    mask_row1(w0, load_row1(w0, y0 - 2));
    mask_row1(w1, load_row1(w1, y0 - 1));
    mask_row1(w2, load_row1(w2, y0));
#pragma unroll
    for (int k = 0; k < X; ++k) { m1[k] = zero_pair<T, C>(); m0[k] = zero_pair<T, C>(); }

    // a_n of row r and a_{n+1} of row r-1 from the windows w0..w2 (a_{n-1}
    // rows r-1 .. r+1), the a_n rows m0..m2 and the a_{n-2} row pr
    auto compute_rows = [&](int r, const P *pr) __attribute__((always_inline)) {
        uint32_t rok;
        const int ry = row_y(r, rok);
        const int64_t rb = (int64_t)ry * Lx;
#pragma unroll
        for (int k = 0; k < X; ++k) { m2[k] = m1[k]; m1[k] = m0[k]; }
        // a_n, row r, columns x0-1 .. x0+W
        const bool own_r = r >= y0 && r < y1;
#pragma unroll
        for (int k = 0; k < X; ++k) {
            const P yv = apply(rb + cx[k + 1], cx[k + 1], ry, w1[k + 1], w1[k], w1[k + 2], w0[k + 1], w2[k + 1]);
            m0[k] = masked<T, C>(cheb_combine<T, C>(yv, pr[k], false), rok & cm[k + 1]);
        }
        if (own_r) {
#pragma unroll
            for (int k = 1; k <= W; ++k) {
                const int64_t s = rb + x0 + k - 1;
                const P &v = m0[k];
                if constexpr (CBDG_NT_OUT) st_nt<T, C>(ao + s * Bp + b, v);
                else st<T, C>(ao + s * Bp + b, v);
                const bool hit = s == my_site;
                found = found || hit;
                mval = select_pair<T, C>(hit, v, mval);
                if constexpr (DOT) dots(d0, v, w1[k + 1]);
            }
        }
        // a_{n+1}, row r-1, own columns
        if (r - 1 >= y0) {
            const int64_t qb = (int64_t)(r - 1) * Lx;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const int64_t s = qb + x0 + k;
                const P yv = apply(s, x0 + k, r - 1, m1[k + 1], m1[k], m1[k + 2], m2[k + 1], m0[k + 1]);
                const P v = cheb_combine<T, C>(yv, w0[k + 2], false);
                if constexpr (CBDG_NT_OUT) st_nt<T, C>(ao2 + s * Bp + b, v);
                else st<T, C>(ao2 + s * Bp + b, v);
                const bool hit = s == my_site;
                found1 = found1 || hit;
                mval1 = select_pair<T, C>(hit, v, mval1);
                if constexpr (DOT) dots(d1, v, m1[k + 1]);
            }
        }
    };
    auto load_prev2 = [&](P *pr, int r) __attribute__((always_inline)) {
        uint32_t rok;
        const int64_t rb = (int64_t)row_y(r, rok) * Lx;
#pragma unroll
        for (int k = 0; k < X; ++k) pr[k] = CBDG_NT_A2 ? ld_nt<T, C>(a2 + (rb + cx[k + 1]) * Bp + b)
                                                      : ld<T, C>(a2 + (rb + cx[k + 1]) * Bp + b);
    };
#pragma unroll 1
    for (int r = y0 - 1; r <= y1; ++r) {
        uint32_t nm = 0;
        if constexpr (!CBDG_A2_FIRST) { if (r + 2 <= y1 + 1) nm = load_row1(nx, r + 2); }
        load_prev2(p2, r);
        if constexpr (CBDG_A2_FIRST) {
            __builtin_amdgcn_sched_barrier(0);  // keep the a_{n-2} loads ahead of the prefetch
            // unconditional (the last trip reloads row y1 + 1, unused), so the
            // waits for a_{n-2} can count the prefetch as issued
            nm = load_row1(nx, min(r + 2, y1 + 1));
        }
        compute_rows(r, p2);
        if (CBDG_A2_FIRST || r + 2 <= y1 + 1) mask_row1(nx, nm);
#pragma unroll
        for (int k = 0; k < Y; ++k) { w0[k] = w1[k]; w1[k] = w2[k]; w2[k] = nx[k]; }
    }

    if constexpr (DOT) {
        double *pp = A.part + region * K * Bp + b;
        double *qq = A.part_b + region * K * Bp + b;
#pragma unroll
        for (int k = 0; k < K; ++k) { pp[k * Bp] = d0[k]; qq[k * Bp] = d1[k]; }
    }
    if (A.mu_ee) {
        const int64_t m = (int64_t)b * A.N + A.n;
        if constexpr (C) {
            if (found) { A.mu_ee[m] = (double)mval.er; A.mu_he[2 * m] = (double)mval.hr; A.mu_he[2 * m + 1] = (double)mval.hi; }
            if (found1) {
                A.mu_ee[m + 1] = (double)mval1.er;
                A.mu_he[2 * (m + 1)] = (double)mval1.hr;
                A.mu_he[2 * (m + 1) + 1] = (double)mval1.hi;
            }
        } else {
            if (found) { A.mu_ee[m] = (double)mval.e; A.mu_he[m] = (double)mval.h; }
            if (found1) { A.mu_ee[m + 1] = (double)mval1.e; A.mu_he[m + 1] = (double)mval1.h; }
        }
    }
}

// Three recursion steps in one pass (real operators, uniform hopping):
// a_n, a_{n+1}, a_{n+2} from a_{n-2} (A.prev2) and a_{n-1} (a1); only the two
// vectors the next pass reads are written, a_{n+1} (A.out) and a_{n+2}
// (A.out2), so the vectors cross HBM four times per three steps.  A lane
// computes a_n on its strip widened by two columns and rows per side, a_{n+1}
// widened by one, a_{n+2} on the strip itself.  Columns: a_{n-1} at
// x0-3 .. x0+W+2 (k <-> x0-3+k), a_n at x0-2 .. x0+W+1, a_{n+1} at
// x0-1 .. x0+W.  Iteration r computes row r of a_n, row r-1 of a_{n+1} and
// row r-2 of a_{n+2}.
template <typename T, int W, bool DOT>
__global__ __launch_bounds__(kBlock) void k_cheb_step3(StepArgs A, const typename Storage<T, false>::type *__restrict__ a1,
                                                      const OnSite<T> *__restrict__ ons)
{
    using P = Pair<T, false>;
    using S = typename Storage<T, false>::type;
    constexpr int X2 = W + 2, X1 = W + 4, Y = W + 6;
    const int lb = xcd_remap(blockIdx.x, A.nblocks);
    const int strip = lb % A.n_strips;
    const int rest = lb / A.n_strips;
    const int seg = rest % A.n_segs;
    const int chunk = rest / A.n_segs;
    const uint32_t b = chunk * kBlock + threadIdx.x;
    if (b >= (uint32_t)A.Bt) return;

    const int Lx = A.Lx, Ly = A.Ly;
    const int x0 = strip * W;
    int y0 = seg * A.ys;
    int y1 = min(y0 + A.ys, Ly);
    const int64_t Bp = A.Bp;
    const int64_t region = strip + (int64_t)A.n_strips * seg;
    if (A.cone) {
        const int m = A.n + 2;
        bool skip = false;
        if (!A.bcx) skip = x0 + W - 1 < A.cone[0] - m || x0 > A.cone[1] + m;
        if (!A.bcy) {
            const int ylo = max(0, A.cone[2] - m), yhi = min(Ly - 1, A.cone[3] + m);
            const int rows = yhi - ylo + 1;
            const int per = max(4, (rows + A.n_segs - 1) / A.n_segs);
            y0 = ylo + seg * per;
            y1 = min(y0 + per, yhi + 1);
            skip = skip || rows <= 0 || y0 >= y1;
        }
        if (skip) {
            if constexpr (DOT) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    A.part[(region * 3 + k) * Bp + b] = 0.0;
                    A.part_b[(region * 3 + k) * Bp + b] = 0.0;
                    A.part_c[(region * 3 + k) * Bp + b] = 0.0;
                }
            }
            return;
        }
    }
    const S *a2 = reinterpret_cast<const S *>(A.prev2);
    S *ao = reinterpret_cast<S *>(A.out);
    S *ao2 = reinterpret_cast<S *>(A.out2);
    const int my_site = A.sites[b];
    const T th = T(A.th);

    int cx[Y];
    uint32_t cm[Y];
#pragma unroll
    for (int k = 0; k < Y; ++k) {
        const int x = x0 - 3 + k;
        if (A.bcx) {
            cx[k] = ((x % Lx) + Lx) % Lx;
            cm[k] = ~0u;
        } else {
            const bool ok = x >= 0 && x < Lx;
            cx[k] = ok ? x : (x < 0 ? 0 : Lx - 1);
            cm[k] = ok ? ~0u : 0u;
        }
    }
    auto row_of = [&](int y, uint32_t &ok) -> int64_t {
        if (A.bcy) { ok = ~0u; return (int64_t)(((y % Ly) + Ly) % Ly) * Lx; }
        const bool in = y >= 0 && y < Ly;
        ok = in ? ~0u : 0u;
        return (int64_t)(in ? y : (y < 0 ? 0 : Ly - 1)) * Lx;
    };
    auto load_row1 = [&](P *row, int y) -> uint32_t {
        uint32_t ok;
        const int64_t rb = row_of(y, ok);
#pragma unroll
        for (int k = 0; k < Y; ++k) row[k] = ld<T, false>(a1 + (rb + cx[k]) * Bp + b);
        return ok;
    };
    auto mask_row1 = [&](P *row, uint32_t rm) {
#pragma unroll
        for (int k = 0; k < Y; ++k) row[k] = masked<T, false>(row[k], rm & cm[k]);
    };

    P w0[Y], w1[Y], w2[Y], nx[Y];   // a_{n-1} rows r-1, r, r+1, r+2
    P m2[X1], m1[X1], m0[X1];       // a_n rows r-2, r-1, r
    P q2[X2], q1[X2], q0[X2];       // a_{n+1} rows r-3, r-2, r-1
    P p2[X1];                       // a_{n-2} row r
    P mv0 = zero_pair<T, false>(), mv1 = zero_pair<T, false>(), mv2 = zero_pair<T, false>();
    bool f0 = false, f1 = false, f2 = false;
    double d[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // <x|x>, <x|y>, B(x, y) for steps n, n+1, n+2
    auto dots = [&](double *acc, const P &v, const P &c) {
        const double e = v.e, h = v.h, ce = c.e, ch = c.h;
        acc[0] += e * e + h * h;
        acc[1] += e * ce + h * ch;
        acc[2] += e * ch - h * ce;
    };
    mask_row1(w0, load_row1(w0, y0 - 3));
    mask_row1(w1, load_row1(w1, y0 - 2));
    mask_row1(w2, load_row1(w2, y0 - 1));
#pragma unroll
    for (int k = 0; k < X1; ++k) { m1[k] = zero_pair<T, false>(); m0[k] = zero_pair<T, false>(); }
#pragma unroll
    for (int k = 0; k < X2; ++k) { q1[k] = zero_pair<T, false>(); q0[k] = zero_pair<T, false>(); }

    auto load_p2 = [&](P *pr, int r) {
        uint32_t ok;
        const int64_t rb = row_of(r, ok);
#pragma unroll
        for (int k = 0; k < X1; ++k) pr[k] = CBDG_NT_A2 ? ld_nt<T, false>(a2 + (rb + cx[k + 1]) * Bp + b)
                                                       : ld<T, false>(a2 + (rb + cx[k + 1]) * Bp + b);
    };
    constexpr bool PF3 = std::is_same<T, float>::value ? CBDG_PF3_F32 : CBDG_PF3_F64;
    [[maybe_unused]] P pn[PF3 ? X1 : 1];
    if constexpr (PF3) load_p2(p2, y0 - 2);

#pragma unroll CBDG_U3
    for (int r = y0 - 2; r <= y1 + 1; ++r) {
        uint32_t nm = 0;
        uint32_t rok;
        const int64_t rb = row_of(r, rok);
        if constexpr (PF3) {
            // a_{n-2} one row ahead: this trip computes with the row loaded on
            // the previous one (rows past the segment clamped, unused)
            nm = load_row1(nx, min(r + 2, y1 + 2));
            load_p2(pn, min(r + 1, y1 + 1));
        } else {
            if constexpr (!CBDG_A2_FIRST) { if (r + 2 <= y1 + 2) nm = load_row1(nx, r + 2); }
            load_p2(p2, r);
            if constexpr (CBDG_A2_FIRST) {
                __builtin_amdgcn_sched_barrier(0);
                nm = load_row1(nx, min(r + 2, y1 + 2));
            }
        }
#pragma unroll
        for (int k = 0; k < X1; ++k) { m2[k] = m1[k]; m1[k] = m0[k]; }
        // a_n, row r, columns x0-2 .. x0+W+1
#pragma unroll
        for (int k = 0; k < X1; ++k) {
            const OnSite<T> o = ons[rb + cx[k + 1]];
            const P yv = apply_uniform<T, false>(o, th, w1[k + 1], w1[k], w1[k + 2], w0[k + 1], w2[k + 1]);
            m0[k] = masked<T, false>(cheb_combine<T, false>(yv, p2[k], false), rok & cm[k + 1]);
        }
        if (r >= y0 && r < y1) {
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const P &v = m0[k + 2];
                const bool hit = rb + x0 + k == my_site;
                f0 = f0 || hit;
                mv0 = select_pair<T, false>(hit, v, mv0);
                if constexpr (DOT) dots(d, v, w1[k + 3]);
            }
        }
        // a_{n+1}, row r-1, columns x0-1 .. x0+W
        if (r - 1 >= y0 - 1) {
            uint32_t qok;
            const int64_t qb = row_of(r - 1, qok);
#pragma unroll
            for (int k = 0; k < X2; ++k) { q2[k] = q1[k]; q1[k] = q0[k]; }
#pragma unroll
            for (int k = 0; k < X2; ++k) {
                const OnSite<T> o = ons[qb + cx[k + 2]];
                const P yv = apply_uniform<T, false>(o, th, m1[k + 1], m1[k], m1[k + 2], m2[k + 1], m0[k + 1]);
                q0[k] = masked<T, false>(cheb_combine<T, false>(yv, w0[k + 2], false), qok & cm[k + 2]);
            }
            if (r - 1 >= y0 && r - 1 < y1) {
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    const int64_t s = qb + x0 + k;
                    const P &v = q0[k + 1];
                    if constexpr (CBDG_NT_OUT) st_nt<T, false>(ao + s * Bp + b, v);
                    else st<T, false>(ao + s * Bp + b, v);
                    const bool hit = s == my_site;
                    f1 = f1 || hit;
                    mv1 = select_pair<T, false>(hit, v, mv1);
                    if constexpr (DOT) dots(d + 3, v, m1[k + 2]);
                }
            }
        }
        // a_{n+2}, row r-2, own columns
        if (r - 2 >= y0) {
            uint32_t sok;
            const int64_t sb = row_of(r - 2, sok);
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const int64_t s = sb + x0 + k;
                const OnSite<T> o = ons[s];
                const P yv = apply_uniform<T, false>(o, th, q1[k + 1], q1[k], q1[k + 2], q2[k + 1], q0[k + 1]);
                const P v = cheb_combine<T, false>(yv, m2[k + 2], false);
                if constexpr (CBDG_NT_OUT) st_nt<T, false>(ao2 + s * Bp + b, v);
                else st<T, false>(ao2 + s * Bp + b, v);
                const bool hit = s == my_site;
                f2 = f2 || hit;
                mv2 = select_pair<T, false>(hit, v, mv2);
                if constexpr (DOT) dots(d + 6, v, q1[k + 1]);
            }
        }
        if (PF3 || CBDG_A2_FIRST || r + 2 <= y1 + 2) mask_row1(nx, nm);
#pragma unroll
        for (int k = 0; k < Y; ++k) { w0[k] = w1[k]; w1[k] = w2[k]; w2[k] = nx[k]; }
        if constexpr (PF3) {
#pragma unroll
            for (int k = 0; k < X1; ++k) p2[k] = pn[k];
        }
    }

    if constexpr (DOT) {
        double *pa = A.part + region * 3 * Bp + b;
        double *pb = A.part_b + region * 3 * Bp + b;
        double *pc = A.part_c + region * 3 * Bp + b;
#pragma unroll
        for (int k = 0; k < 3; ++k) { pa[k * Bp] = d[k]; pb[k * Bp] = d[3 + k]; pc[k * Bp] = d[6 + k]; }
    }
    if (A.mu_ee) {
        const int64_t m = (int64_t)b * A.N + A.n;
        if (f0) { A.mu_ee[m] = (double)mv0.e; A.mu_he[m] = (double)mv0.h; }
        if (f1) { A.mu_ee[m + 1] = (double)mv1.e; A.mu_he[m + 1] = (double)mv1.h; }
        if (f2) { A.mu_ee[m + 2] = (double)mv2.e; A.mu_he[m + 2] = (double)mv2.h; }
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
        if (!mu_ee) return;
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
    if (!mu_ee) return;
    mu_ee[m] = 1.0;
    if (C) { mu_he[2 * m] = 0.0; mu_he[2 * m + 1] = 0.0; }
    else mu_he[m] = 0.0;
}

// Bounding box {x_min, x_max, y_min, y_max} of the tile's valid start sites
// (an empty tile gives x_min > x_max).  One workgroup of kBlock threads.
__global__ __launch_bounds__(kBlock) void k_tile_cone(const int32_t *sites, int Bt, int Lx, int64_t L2,
                                                     int32_t *cone)
{
    __shared__ int red[4][kBlock];
    int v[4] = {INT32_MAX, -1, INT32_MAX, -1};
    for (int b = threadIdx.x; b < Bt; b += kBlock) {
        const int64_t s = sites[b];
        if (s < 0 || s >= L2) continue;
        const int x = (int)(s % Lx), y = (int)(s / Lx);
        v[0] = min(v[0], x); v[1] = max(v[1], x);
        v[2] = min(v[2], y); v[3] = max(v[3], y);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h /= 2) {
        if ((int)threadIdx.x < h) {
            const int o = threadIdx.x + h;
            red[0][threadIdx.x] = min(red[0][threadIdx.x], red[0][o]);
            red[1][threadIdx.x] = max(red[1][threadIdx.x], red[1][o]);
            red[2][threadIdx.x] = min(red[2][threadIdx.x], red[2][o]);
            red[3][threadIdx.x] = max(red[3][threadIdx.x], red[3][o]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) cone[threadIdx.x] = red[threadIdx.x][0];
}

// Launch shapes per vector type, chosen by measurement on MI355X (one
// 1024-vector step):
//   W   strip width in sites (W + 2 columns of a_{n-1} per row in registers)
//   PF  rows of a_{n-2} prefetched one row ahead (more registers) or loaded at
//       the top of their own row
//   YS  longest row segment; shortened at launch until the grid fills the GPU
// "big" is used when W_BIG divides Lx and the grid has at least 2048
// workgroups at 16-row segments, "small" otherwise.  FP64 at 256x256:
// W8+PF 508 us, W8 541, W4+PF 565, W4 556; at 128x128: W4 126, W8+PF 141.
// complex128 at 512x512: W2+PF 5.27 ms, W4 5.33, W1+PF 5.80; complex64:
// W8 2.20 ms, W4+PF 2.32.
// Complex operators (one step per launch): 32-row segments, 2048 workgroups.
// On one tile of spread start sites (512x512, N = 258) longer segments were
// faster (512 rows, 1024 workgroups: complex128 982.4 vs 1019.0 us per
// step), but on the Peierls/d-wave workload (stride-8 grid of start sites,
// N = 2048) 4840 vs 4770 us per launch: while the light cone is small a
// strip's active rows are shared by fewer, longer segments.
#ifndef CBDG_YS_C128
#define CBDG_YS_C128 32
#endif
#ifndef CBDG_YS_C64
#define CBDG_YS_C64 32
#endif
#ifndef CBDG_TGT_C
#define CBDG_TGT_C 2048
#endif
template <typename T, bool C> struct StepShape;
template <> struct StepShape<double, false> {
    static constexpr int W_BIG = 8, W_SMALL = 4, YS = 64, TGT = 2048;
    static constexpr bool PF_BIG = true, PF_SMALL = false;
};
template <> struct StepShape<float, false> {
    static constexpr int W_BIG = 8, W_SMALL = 4, YS = 32, TGT = 2048;
    static constexpr bool PF_BIG = true, PF_SMALL = false;
};
template <> struct StepShape<double, true> {
    static constexpr int W_BIG = 2, W_SMALL = 2, YS = CBDG_YS_C128, TGT = CBDG_TGT_C;
    static constexpr bool PF_BIG = true, PF_SMALL = true;
};
template <> struct StepShape<float, true> {
    static constexpr int W_BIG = 8, W_SMALL = 4, YS = CBDG_YS_C64, TGT = CBDG_TGT_C;
    static constexpr bool PF_BIG = false, PF_SMALL = false;
};

// Row-segment length: the longest of YS, YS/2, ... (not below 8) that still
// gives every CU several workgroups; shorter segments cost extra halo rows.
static int segment_rows(int Ly, int64_t other_blocks, int ys_max, int64_t target_blocks)
{
    int ys = ys_max;
    while (ys > 8 && other_blocks * ceil_div(Ly, ys) < target_blocks) ys /= 2;
    return ys;
}

struct Shape {
    int W;
    bool PF;
    int ys, n_strips, n_segs;
};

// Strip width from the shape table (else 2 or 1 so that W divides Lx), then
// the row-segment length for that width.
template <typename T, bool C>
static Shape choose_shape(int Lx, int Ly, int64_t n_chunks)
{
    using SH = StepShape<T, C>;
    Shape sh;
    if (Lx % SH::W_BIG == 0 && (Lx / SH::W_BIG) * n_chunks * ceil_div(Ly, 16) >= 2048) {
        sh.W = SH::W_BIG; sh.PF = SH::PF_BIG;
    } else if (Lx % SH::W_SMALL == 0) {
        sh.W = SH::W_SMALL; sh.PF = SH::PF_SMALL;
    } else {
        sh.W = (Lx % 2 == 0) ? 2 : 1; sh.PF = false;
    }
    sh.n_strips = Lx / sh.W;
    sh.ys = segment_rows(Ly, (int64_t)sh.n_strips * n_chunks, SH::YS, SH::TGT);
    sh.n_segs = (int)ceil_div(Ly, sh.ys);
    return sh;
}

// Largest number of (strip, segment) regions any tile of up to `tile`
// vectors launches with: the size of the moment-doubling partials.
template <typename T, bool C>
static int64_t max_regions(int Lx, int Ly, int tile)
{
    int64_t r = 0;
    for (int64_t c = 1; c <= ceil_div(tile, kBlock); ++c) {
        const Shape sh = choose_shape<T, C>(Lx, Ly, c);
        r = std::max<int64_t>(r, (int64_t)sh.n_strips * sh.n_segs);
    }
    return r;
}

template <typename T, bool C, bool GEN, int W, bool PF>
static int launch_step_w(StepArgs A, hipStream_t st)
{
    const int n_chunks = (int)ceil_div(A.Bt, kBlock);
    const int64_t nb = (int64_t)A.n_strips * A.n_segs * n_chunks;
    if (nb > INT32_MAX) return fail(CBDG_EINVAL, "chebyshev_moments: launch grid too large");
    A.nblocks = (int)nb;
    const auto *a1 = reinterpret_cast<const typename Storage<T, C>::type *>(A.prev1);
    const auto *ons = reinterpret_cast<const OnSite<T> *>(A.onsite);
    const dim3 g(A.nblocks), bl(kBlock);
    if (A.part) {
        if (A.first) hipLaunchKernelGGL((k_cheb_step<T, C, GEN, true, W, PF, 1>), g, bl, 0, st, A, a1, ons, A.bonds);
        else hipLaunchKernelGGL((k_cheb_step<T, C, GEN, false, W, PF, 1>), g, bl, 0, st, A, a1, ons, A.bonds);
    } else if (A.nb_ee) {
        if (A.first) hipLaunchKernelGGL((k_cheb_step<T, C, GEN, true, W, PF, 2>), g, bl, 0, st, A, a1, ons, A.bonds);
        else hipLaunchKernelGGL((k_cheb_step<T, C, GEN, false, W, PF, 2>), g, bl, 0, st, A, a1, ons, A.bonds);
    } else {
        if (A.first) hipLaunchKernelGGL((k_cheb_step<T, C, GEN, true, W, PF, 0>), g, bl, 0, st, A, a1, ons, A.bonds);
        else hipLaunchKernelGGL((k_cheb_step<T, C, GEN, false, W, PF, 0>), g, bl, 0, st, A, a1, ons, A.bonds);
    }
    CBDG_CHECK_LAUNCH("k_cheb_step");
    return CBDG_OK;
}

template <typename T, bool C, bool GEN>
static int launch_step(StepArgs A, hipStream_t st)
{
    using SH = StepShape<T, C>;
    const Shape sh = choose_shape<T, C>(A.Lx, A.Ly, ceil_div(A.Bt, kBlock));
    A.n_strips = sh.n_strips;
    A.ys = sh.ys;
    A.n_segs = sh.n_segs;
    if (sh.W == SH::W_BIG && sh.PF == SH::PF_BIG) return launch_step_w<T, C, GEN, SH::W_BIG, SH::PF_BIG>(A, st);
    if (sh.W == SH::W_SMALL && sh.PF == SH::PF_SMALL) return launch_step_w<T, C, GEN, SH::W_SMALL, SH::PF_SMALL>(A, st);
    if (sh.W == 2) return launch_step_w<T, C, GEN, 2, false>(A, st);
    return launch_step_w<T, C, GEN, 1, false>(A, st);
}

// Two-step passes (k_cheb_step2) for real operators with uniform hopping.
// Strip width W, longest row segment YS2 and the workgroup count the
// segments are shortened to reach (TGT2), by measurement on MI355X: one
// 1024-vector tile of the 256x256 workload, N = 514 by doubling, microseconds
// per moment index (FP64 / FP32; one-step kernel alone: 268.9 / 135.4):
//   W = 2: 295.8 / 132.8   W = 4: 219.5 / 122.0   W = 8: 203.9 / 104.7
//   W = 8, 1024 workgroups: 196.6 / 103.1; 512 workgroups: 193.1 / 102.2
//   W = 16 (FP32): 133.8; a_{n-2} prefetched a row ahead: no gain.
// At W = 8 the FP64 kernel holds 256 VGPRs plus AGPRs, one wave per SIMD.
// With the a_{n-2} loads ahead of the prefetch (FP64, spread / rows):
// segments of 64 rows, 512 workgroups 192.7 / 149.7; 32 rows 195.9 / 153.5;
// 1024 workgroups 195.9 / 153.4; 128 rows, 256 workgroups 191.2 / 147.8
// (one workgroup per CU at 256x256: fewer widened halo rows).
#ifndef CBDG_TWO_STEP
#define CBDG_TWO_STEP 1
#endif
#ifndef CBDG_W2_F64
#define CBDG_W2_F64 8
#endif
#ifndef CBDG_W2_F32
#define CBDG_W2_F32 8
#endif
#ifndef CBDG_YS2
#define CBDG_YS2 128
#endif
#ifndef CBDG_TGT2
#define CBDG_TGT2 256
#endif
// Two-step passes for complex operators and per-bond coefficients are
// available but off: on one 1024-vector tile of the 512x512 Peierls/d-wave
// lattice (N = 258 by doubling) they were slower than one step per launch,
// complex128 1371 (W = 2) / 1668 (W = 1) vs 1030 us per moment index,
// complex64 485 (W = 4 or 2) vs 432 -- the widened windows of 32-byte pairs
// and the per-site link loads outweigh the saved traffic.
#ifndef CBDG_TWO_STEP_GEN
#define CBDG_TWO_STEP_GEN 0
#endif
#ifndef CBDG_W2_C128
#define CBDG_W2_C128 2
#endif
#ifndef CBDG_W2_C64
#define CBDG_W2_C64 4
#endif
template <typename T, bool C> struct Step2Shape;
template <> struct Step2Shape<double, false> { static constexpr int W = CBDG_W2_F64; };
template <> struct Step2Shape<float, false> { static constexpr int W = CBDG_W2_F32; };
template <> struct Step2Shape<double, true> { static constexpr int W = CBDG_W2_C128; };
template <> struct Step2Shape<float, true> { static constexpr int W = CBDG_W2_C64; };

template <typename T, bool C>
static Shape choose_shape2(int Lx, int Ly, int64_t n_chunks)
{
    Shape sh;
    constexpr int WB = Step2Shape<T, C>::W;
    sh.W = (Lx % WB == 0) ? WB : (Lx % 4 == 0 && WB > 4 ? 4 : (Lx % 2 == 0 && WB > 2 ? 2 : 1));
    sh.PF = false;
    sh.n_strips = Lx / sh.W;
    int ys = CBDG_YS2;
    while (ys > 8 && (int64_t)sh.n_strips * n_chunks * ceil_div(Ly, ys) < CBDG_TGT2) ys /= 2;
    sh.ys = ys;
    sh.n_segs = (int)ceil_div(Ly, sh.ys);
    return sh;
}

template <typename T, bool C>
static int64_t max_regions2(int Lx, int Ly, int tile)
{
    int64_t r = 0;
    for (int64_t c = 1; c <= ceil_div(tile, kBlock); ++c) {
        const Shape sh = choose_shape2<T, C>(Lx, Ly, c);
        r = std::max<int64_t>(r, (int64_t)sh.n_strips * sh.n_segs);
    }
    return r;
}

template <typename T, bool C, bool GEN, int W>
static int launch_step2_w(StepArgs A, hipStream_t st)
{
    const int n_chunks = (int)ceil_div(A.Bt, kBlock);
    const int64_t nb = (int64_t)A.n_strips * A.n_segs * n_chunks;
    if (nb > INT32_MAX) return fail(CBDG_EINVAL, "chebyshev_moments: launch grid too large");
    A.nblocks = (int)nb;
    const auto *a1 = reinterpret_cast<const typename Storage<T, C>::type *>(A.prev1);
    const auto *ons = reinterpret_cast<const OnSite<T> *>(A.onsite);
    if (A.part) hipLaunchKernelGGL((k_cheb_step2<T, C, GEN, W, true>), dim3(A.nblocks), dim3(kBlock), 0, st, A, a1, ons, A.bonds);
    else hipLaunchKernelGGL((k_cheb_step2<T, C, GEN, W, false>), dim3(A.nblocks), dim3(kBlock), 0, st, A, a1, ons, A.bonds);
    CBDG_CHECK_LAUNCH("k_cheb_step2");
    return CBDG_OK;
}

template <typename T, bool C, bool GEN>
static int launch_step2(StepArgs A, hipStream_t st)
{
    const Shape sh = choose_shape2<T, C>(A.Lx, A.Ly, ceil_div(A.Bt, kBlock));
    A.n_strips = sh.n_strips;
    A.ys = sh.ys;
    A.n_segs = sh.n_segs;
    constexpr int WB = Step2Shape<T, C>::W;
    if (sh.W == WB) return launch_step2_w<T, C, GEN, WB>(A, st);
    if constexpr (WB > 4) { if (sh.W == 4) return launch_step2_w<T, C, GEN, 4>(A, st); }
    if constexpr (WB > 2) { if (sh.W == 2) return launch_step2_w<T, C, GEN, 2>(A, st); }
    return launch_step2_w<T, C, GEN, 1>(A, st);
}

static bool uses_two_step(const cbdg_op *op)
{
    if (op->scalar == CBDG_REAL && !op->general) return CBDG_TWO_STEP;
    return CBDG_TWO_STEP && CBDG_TWO_STEP_GEN;
}

// Three-step passes (k_cheb_step3) for real operators with uniform hopping.
// One 1024-vector tile of the 256x256 workload, N = 514 by doubling,
// microseconds per moment index (two-step W = 8: FP64 192.7, FP32 101.7):
//   FP32: W = 4 94.3 (222 VGPRs, two waves per SIMD), W = 8 111.2, W = 2 135.5
//   FP64: W = 4 199.1, W = 2 263.0, W = 1 329.6 (the widened register windows
//         spill into AGPRs)
// After the load-order change and 128-row segments (spread / rows): FP64
// two-step 191.4 / 148.0, three-step W = 4 186.9 / 142.2, W = 2 212.6 / 163.5.
#ifndef CBDG_THREE_STEP_F64
#define CBDG_THREE_STEP_F64 1
#endif
#ifndef CBDG_THREE_STEP_F32
#define CBDG_THREE_STEP_F32 1
#endif
#ifndef CBDG_W3_F64
#define CBDG_W3_F64 4
#endif
#ifndef CBDG_W3_F32
#define CBDG_W3_F32 4
#endif
// Longest row segment and workgroup target of the three-step passes, per
// type (FP64, spread / rows, us per moment index; FP32 widths W = 2 and
// W = 8 with 256 rows were slower, 111.2 and 105.7 against 82.8 spread):
// 256 rows 163.2 / 126.6,
// 128 rows 186.6 / 141.9, 64 rows with 512 or 1024 workgroups 191.9 / 147.1 --
// at 256x256 the 256 workgroups of 256-row segments put exactly one wave on
// every SIMD for the whole launch.  FP32 (two waves per SIMD): 128 rows
// 83.1 / 73.6, 256 rows 121.2 / 107.2, 64 rows 84.9 / 75.6.
#ifndef CBDG_YS3_F64
#define CBDG_YS3_F64 256
#endif
// Tiles of fewer vectors take two-step passes: with one or two waves per row
// segment the longer serial chain of a three-step trip is not hidden.  256x256,
// 1024 start sites, time per tile set (two-step / three-step, ms): FP64 64
// vectors 182.5 / 190.5, 128: 100.9 / 101.0, 256: 71.3 / 60.3, 1024: 62.4 /
// 53.6; FP32 64: 350 / 386, 128: 184 / 202, 256: 118 / 107, 1024: 104 / 70.
constexpr int kThreeStepMinVectors = 129;
// Tiles of at least this many vectors take the vector-contiguous passes when
// the lattice fits them.
#ifndef CBDG_VC_MIN
#define CBDG_VC_MIN 1
#endif
constexpr int kVcMinVectors = CBDG_VC_MIN;
#ifndef CBDG_YS3_F32
#define CBDG_YS3_F32 128
#endif
#ifndef CBDG_TGT3
#define CBDG_TGT3 256
#endif
template <typename T> struct Step3Shape;
template <> struct Step3Shape<double> {
    static constexpr int W = CBDG_W3_F64, YS = CBDG_YS3_F64;
    static constexpr bool ON = CBDG_THREE_STEP_F64;
};
template <> struct Step3Shape<float> {
    static constexpr int W = CBDG_W3_F32, YS = CBDG_YS3_F32;
    static constexpr bool ON = CBDG_THREE_STEP_F32;
};

template <typename T>
static Shape choose_shape3(int Lx, int Ly, int64_t n_chunks)
{
    Shape sh;
    constexpr int WB = Step3Shape<T>::W;
    sh.W = (Lx % WB == 0) ? WB : (Lx % 4 == 0 ? 4 : (Lx % 2 == 0 ? 2 : 1));
    sh.PF = false;
    sh.n_strips = Lx / sh.W;
    int ys = Step3Shape<T>::YS;
    while (ys > 8 && (int64_t)sh.n_strips * n_chunks * ceil_div(Ly, ys) < CBDG_TGT3) ys /= 2;
    sh.ys = ys;
    sh.n_segs = (int)ceil_div(Ly, sh.ys);
    return sh;
}

template <typename T>
static int64_t max_regions3(int Lx, int Ly, int tile)
{
    int64_t r = 0;
    for (int64_t c = 1; c <= ceil_div(tile, kBlock); ++c) {
        const Shape sh = choose_shape3<T>(Lx, Ly, c);
        r = std::max<int64_t>(r, (int64_t)sh.n_strips * sh.n_segs);
    }
    return r;
}

template <typename T, int W>
static int launch_step3_w(StepArgs A, hipStream_t st)
{
    const int n_chunks = (int)ceil_div(A.Bt, kBlock);
    const int64_t nb = (int64_t)A.n_strips * A.n_segs * n_chunks;
    if (nb > INT32_MAX) return fail(CBDG_EINVAL, "chebyshev_moments: launch grid too large");
    A.nblocks = (int)nb;
    const auto *a1 = reinterpret_cast<const typename Storage<T, false>::type *>(A.prev1);
    const auto *ons = reinterpret_cast<const OnSite<T> *>(A.onsite);
    if (A.part) hipLaunchKernelGGL((k_cheb_step3<T, W, true>), dim3(A.nblocks), dim3(kBlock), 0, st, A, a1, ons);
    else hipLaunchKernelGGL((k_cheb_step3<T, W, false>), dim3(A.nblocks), dim3(kBlock), 0, st, A, a1, ons);
    CBDG_CHECK_LAUNCH("k_cheb_step3");
    return CBDG_OK;
}

template <typename T>
static int launch_step3(StepArgs A, hipStream_t st)
{
    const Shape sh = choose_shape3<T>(A.Lx, A.Ly, ceil_div(A.Bt, kBlock));
    A.n_strips = sh.n_strips;
    A.ys = sh.ys;
    A.n_segs = sh.n_segs;
    // only the table width and the narrower fallbacks are instantiated
    constexpr int WB = Step3Shape<T>::W;
    if constexpr (WB >= 8) { if (sh.W == 8) return launch_step3_w<T, 8>(A, st); }
    if constexpr (WB >= 4) { if (sh.W == 4) return launch_step3_w<T, 4>(A, st); }
    if (sh.W == 2) return launch_step3_w<T, 2>(A, st);
    return launch_step3_w<T, 1>(A, st);
}

// Moments 2n-1 and 2n of every vector from the partial sums of step n:
//   mu_ee[2n]   = 2 <a_n|a_n> - mu_ee[0]
//   mu_ee[2n-1] = 2 Re<a_n|a_{n-1}> - mu_ee[1]
//   mu_he[2n-1] = 2 (-1)^n B(a_n, a_{n-1}) - mu_he[1]
//   mu_he[2n]   = 0
// (C(u,v) = (-v*, u*) anticommutes with Ht when b = 0, so T_m(Ht) C =
// (-1)^m C T_m(Ht), and the hole start vector is C applied to the electron
// one.)  The per-region partials are summed in two passes, both in a fixed
// order so that the bits do not depend on scheduling: k_doubling_groups adds
// runs of consecutive regions (one thread per vector and run, enough
// workgroups to spread over the GPU), then k_doubling_reduce adds the runs
// (one workgroup per 64 vectors; wave w takes runs w, w + 16, ..., wave 0
// adds the 16 wave sums in order) and writes the moments.  Rows of invalid
// start sites keep their NaN.
constexpr int kRedWaves = 16;
constexpr int64_t kConeDoubles = 32;  // workspace slot of the tile's bounding box (256 B)
constexpr int kMaxGroups = 256;

// Regions per run and number of runs for R regions (at most kMaxGroups runs).
static inline void doubling_groups(int64_t R, int64_t *per, int64_t *groups)
{
    *per = std::max<int64_t>(4, ceil_div(R, kMaxGroups));
    *groups = ceil_div(R, *per);
}

// blockIdx.z selects one of the steps of a multi-step pass: its partials sit
// pstride doubles after the previous step's, its run sums ostride after.
template <bool C>
__global__ __launch_bounds__(kBlock) void k_doubling_groups(
    const double *__restrict__ part, int64_t regions, int64_t per, int64_t Bp, int Bt,
    double *__restrict__ out, int64_t pstride, int64_t ostride)
{
    constexpr int K = C ? 4 : 3;
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= Bt) return;
    part += blockIdx.z * pstride;
    out += blockIdx.z * ostride;
    const int64_t g = blockIdx.y;
    const int64_t r0 = g * per, r1 = std::min<int64_t>(regions, r0 + per);
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
        const double *pp = part + r * K * Bp + b;
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += pp[k * Bp];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) out[(g * K + k) * Bp + b] = acc[k];
}

// blockIdx.y selects the step n + blockIdx.y of a multi-step pass (run sums
// ostride doubles apart); the steps write disjoint moments.
template <bool C>
__global__ __launch_bounds__(kRedWaves * kWave) void k_doubling_reduce(
    const double *__restrict__ part, int64_t regions, int64_t Bp, int Bt, int n, int N,
    double *__restrict__ mu_ee, double *__restrict__ mu_he, int64_t ostride)
{
    constexpr int K = C ? 4 : 3;
    part += blockIdx.y * ostride;
    n += blockIdx.y;
    __shared__ double red[kRedWaves][K][kWave];
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    const int b = blockIdx.x * kWave + lane;
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    if (b < Bt) {
#pragma unroll 2
        for (int64_t r = wv; r < regions; r += kRedWaves) {
            const double *pp = part + r * K * Bp + b;
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] += pp[k * Bp];
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) red[wv][k][lane] = acc[k];
    __syncthreads();
    if (wv != 0 || b >= Bt) return;
#pragma unroll 1
    for (int w = 1; w < kRedWaves; ++w) {
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += red[w][k][lane];
    }
    const int64_t m = (int64_t)b * N;
    if (!(mu_ee[m] == mu_ee[m])) return;
    const double sgn = (n & 1) ? -2.0 : 2.0;
    if (2 * n < N) {
        mu_ee[m + 2 * n] = 2.0 * acc[0] - mu_ee[m];
        if constexpr (C) { mu_he[2 * (m + 2 * n)] = 0.0; mu_he[2 * (m + 2 * n) + 1] = 0.0; }
        else mu_he[m + 2 * n] = 0.0;
    }
    if (n >= 2 && 2 * n - 1 < N) {
        mu_ee[m + 2 * n - 1] = 2.0 * acc[1] - mu_ee[m + 1];
        if constexpr (C) {
            mu_he[2 * (m + 2 * n - 1)] = sgn * acc[2] - mu_he[2 * (m + 1)];
            mu_he[2 * (m + 2 * n - 1) + 1] = sgn * acc[3] - mu_he[2 * (m + 1) + 1];
        } else {
            mu_he[m + 2 * n - 1] = sgn * acc[2] - mu_he[m + 1];
        }
    }
}

// Bound of the moments: with the spectrum of Ht inside [-1, 1], every
// <bra|T_n(Ht)|s,e> of unit vectors has magnitude at most 1.  A moment beyond
// lim (1 + the precision's rounding allowance) or not finite means the
// rescaling does not contain the spectrum; it is replaced by NaN, so that
// every quantity computed from it (gap update residual, LDOS, density) is NaN
// and the caller sees the failure without a synchronisation here.  Rows of
// invalid start sites are NaN already.
__device__ __forceinline__ void bound_entry(double *p, int64_t i, int cplx, double lim)
{
    const double nan = __builtin_nan("");
    if (cplx) {
        if (!(hypot(p[2 * i], p[2 * i + 1]) <= lim)) { p[2 * i] = nan; p[2 * i + 1] = nan; }
    } else if (!(fabs(p[i]) <= lim)) {
        p[i] = nan;
    }
}

// ee_c / he_c: the array holds complex128 entries (interleaved) instead of FP64
__global__ void k_bound_moments(double *__restrict__ ee, double *__restrict__ he, int64_t n, int ee_c, int he_c,
                                double lim)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        bound_entry(ee, i, ee_c, lim);
        bound_entry(he, i, he_c, lim);
    }
}

int bound_moments(double *ee, double *he, int64_t n, bool ee_c, bool he_c, double lim, hipStream_t st)
{
    if (n <= 0) return CBDG_OK;
    hipLaunchKernelGGL(k_bound_moments, dim3((unsigned)std::min<int64_t>(ceil_div(n, kBlock), 2048)), dim3(kBlock),
                       0, st, ee, he, n, ee_c ? 1 : 0, he_c ? 1 : 0, lim);
    CBDG_CHECK_LAUNCH("k_bound_moments");
    return CBDG_OK;
}

// Rounding allowance of the bound check: FP64 recursion vectors keep |mu| <= 1
// to ~1e-13; FP32 vectors to a few 1e-6.
double moment_limit(bool f32) { return f32 ? 1.0 + 1e-4 : 1.0 + 1e-9; }

int run_step(const cbdg_op *op, int precision, StepArgs A, hipStream_t st)
{
    const bool f64 = precision == CBDG_FP64;
    const bool cplx = op->scalar == CBDG_COMPLEX;
    A.onsite = f64 ? (const void *)op->onsite64 : (const void *)op->onsite32;
    A.bonds = f64 ? op->bonds64 : op->bonds32;
    if (f64) {
        if (cplx) return op->general ? launch_step<double, true, true>(A, st) : launch_step<double, true, false>(A, st);
        return op->general ? launch_step<double, false, true>(A, st) : launch_step<double, false, false>(A, st);
    }
    if (cplx) return op->general ? launch_step<float, true, true>(A, st) : launch_step<float, true, false>(A, st);
    return op->general ? launch_step<float, false, true>(A, st) : launch_step<float, false, false>(A, st);
}

bool two_step_f64_real(const cbdg_op *op)
{
    return op->scalar == CBDG_REAL && !op->general && CBDG_TWO_STEP;
}

bool three_step_f64_real(const cbdg_op *op, int Bt)
{
    return two_step_f64_real(op) && Step3Shape<double>::ON && Bt >= kThreeStepMinVectors;
}

int run_step3_f64_real(const cbdg_op *op, StepArgs A, hipStream_t st)
{
    if (!three_step_f64_real(op, A.Bt))
        return fail(CBDG_EUNSUPPORTED, "three-step pass: needs a real operator with uniform hopping and "
                    "a tile of at least %d vectors", kThreeStepMinVectors);
    A.onsite = op->onsite64;
    A.bonds = op->bonds64;
    A.first = 0;
    return launch_step3<double>(A, st);
}

int run_step2_f64_real(const cbdg_op *op, StepArgs A, hipStream_t st)
{
    if (!two_step_f64_real(op))
        return fail(CBDG_EUNSUPPORTED, "two-step pass: needs a real operator with uniform hopping");
    A.onsite = op->onsite64;
    A.bonds = op->bonds64;
    A.first = 0;
    return launch_step2<double, false, false>(A, st);
}

int seed_tile_f64_real(void *a0, int64_t L2, int Bt, const int32_t *sites, double *mu_ee, double *mu_he, int N,
                       hipStream_t st)
{
    using S = Storage<double, false>::type;
    const int64_t Bp = lane_stride(Bt);
    const int64_t nz = L2 * Bp;
    hipLaunchKernelGGL((k_zero<double, false>), dim3((unsigned)std::min<int64_t>(ceil_div(nz, kBlock), 8192)),
                       dim3(kBlock), 0, st, reinterpret_cast<S *>(a0), nz);
    CBDG_CHECK_LAUNCH("k_zero");
    hipLaunchKernelGGL((k_seed<double, false>), dim3((unsigned)ceil_div(Bt, kBlock)), dim3(kBlock), 0, st,
                       reinterpret_cast<S *>(a0), Bp, Bt, L2, sites, mu_ee, mu_he, N);
    CBDG_CHECK_LAUNCH("k_seed");
    return CBDG_OK;
}

// Direct: steps n = 1 .. N-1, each capturing moment n of every vector.
// Doubling: steps n = 1 .. ceil((N-1)/2); step 1 captures moment 1 and every
// step's partial sums give moments 2n-1 and 2n.  Real uniform operators take
// the steps after the first two at a time (three at a time in FP32; four tile
// buffers), the others one at a time in place (two buffers).  Workspace: the tile buffers, the
// tile's bounding box, then for doubling the partials of a pass's two steps
// [regions][K][Bp] x 2 and the run sums [runs][K][Bp].
template <typename T, bool C>
static int run_moments(const cbdg_op *op, const int32_t *sites, int64_t n_start, int N, int tile,
                       bool doubling, void *ws, double *mu_ee, double *mu_he, hipStream_t st,
                       double *nb_ee = nullptr, double *nb_he = nullptr, void **vc_out = nullptr)
{
    using S = typename Storage<T, C>::type;
    const int64_t L2 = op->L2;
    const int64_t Bp_max = lane_stride(tile);
    const bool two = uses_two_step(op) && !nb_ee;
    const int nbuf = two ? 4 : 2;
    S *buf[4];
    for (int i = 0; i < 4; ++i) buf[i] = reinterpret_cast<S *>(ws) + (i < nbuf ? i : 0) * L2 * Bp_max;
    int32_t *cone = reinterpret_cast<int32_t *>(reinterpret_cast<S *>(ws) + nbuf * L2 * Bp_max);
    constexpr int K = C ? 4 : 3;
    const bool three = two && !C && !op->general && Step3Shape<T>::ON;
    const int64_t Rmax = std::max({max_regions<T, C>(op->Lx, op->Ly, tile), two ? max_regions2<T, C>(op->Lx, op->Ly, tile) : 0,
                                   three ? max_regions3<T>(op->Lx, op->Ly, tile) : 0});
    double *part = reinterpret_cast<double *>(cone) + kConeDoubles;
    double *part_b = part + (doubling ? Rmax * K * Bp_max : 0);
    double *part_c = part_b + (doubling ? Rmax * K * Bp_max : 0);
    double *part2 = part + (doubling ? kMaxPassSteps * Rmax * K * Bp_max : 0);
    const void *onsite = std::is_same<T, double>::value ? (const void *)op->onsite64 : (const void *)op->onsite32;
    const void *bonds = std::is_same<T, double>::value ? op->bonds64 : op->bonds32;
    const int he_mult = C ? 2 : 1;
    const int64_t pstride = Rmax * K * Bp_max, ostride = (int64_t)kMaxGroups * K * Bp_max;
    // moments 2m-1, 2m for the steps m = n .. n+ns-1 of one launch, whose
    // partials sit pstride doubles apart from `part` on
    auto reduce = [&](int64_t regions, int n, int ns, int Bt, int64_t Bp, double *mee, double *mhe) -> int {
        int64_t per = 0, groups = 0;
        doubling_groups(regions, &per, &groups);
        hipLaunchKernelGGL((k_doubling_groups<C>),
                           dim3((unsigned)ceil_div(Bt, kBlock), (unsigned)groups, (unsigned)ns),
                           dim3(kBlock), 0, st, part, regions, per, Bp, Bt, part2, pstride, ostride);
        CBDG_CHECK_LAUNCH("k_doubling_groups");
        hipLaunchKernelGGL((k_doubling_reduce<C>), dim3((unsigned)ceil_div(Bt, kWave), (unsigned)ns),
                           dim3(kRedWaves * kWave), 0, st, part2, groups, Bp, Bt, n, N, mee, mhe, ostride);
        CBDG_CHECK_LAUNCH("k_doubling_reduce");
        return CBDG_OK;
    };
    // Vector-contiguous passes (real uniform operators, doubling, Lx = 64 W):
    // the same four buffers, vector b from pair b * L2 on; their packed
    // coefficients follow the run sums.
    void *vc_coef = part2 + kMaxPassSteps * (int64_t)kMaxGroups * K * Bp_max;
    constexpr bool f32 = std::is_same<T, float>::value;
    auto vc_tile = [&](int Bt) -> bool {
        return !C && !op->general && doubling && !nb_ee && two && vc_width(op->Lx, f32) > 0 && Bt >= kVcMinVectors;
    };
    // No clearing: the passes read nothing the tile has not written.  With
    // one row segment per vector a pass writes its moments itself; with more
    // the reduction kernels add the segments' partials.
    auto run_tile_vc = [&](int Bt, int64_t Bp, const int32_t *ts, double *mee, double *mhe) -> int {
        auto vc_reduce = [&](int segs, int n, int ns) -> int {
            return segs == 1 ? CBDG_OK : reduce(segs, n, ns, Bt, Bp, mee, mhe);
        };
        int rc = launch_vc_seed(buf[0], L2, op->Lx, f32, Bt, L2, ts, mee, mhe, N, st);
        if (rc) return rc;
        VcArgs V{};
        V.coef = vc_coef;
        V.th = op->t / op->bounds.a;
        V.Lx = op->Lx; V.Ly = op->Ly; V.bcx = op->bc_x; V.bcy = op->bc_y;
        V.Dv = L2; V.Bt = Bt; V.Bp = (int)Bp; V.N = N;
        V.sites = ts; V.mu_ee = mee; V.mu_he = mhe;
        const int KS = vc_steps(f32);
        const int segs1 = (int)std::min<int64_t>(vc_segments(op->Ly, Bt, 1), Rmax);
        const int segsK = (int)std::min<int64_t>(vc_segments(op->Ly, Bt, KS), Rmax);
        const int n_steps = N / 2;
        S *P2 = buf[0], *P1 = buf[1], *Q0 = buf[2], *Q1 = buf[3];
        V.part = part; V.pstride = pstride;
        V.n = 1; V.a1 = P2; V.a2 = P2; V.out = P1; V.n_segs = segs1;
        if ((rc = launch_vc(V, 1, f32, st)) || (rc = vc_reduce(segs1, 1, 1))) return rc;
        int n = 2;
        V.n_segs = segsK;
        for (; n + KS - 1 <= n_steps; n += KS) {
            V.n = n; V.a2 = P2; V.a1 = P1; V.out = Q0; V.out2 = Q1;
            if ((rc = launch_vc(V, KS, f32, st)) || (rc = vc_reduce(segsK, n, KS))) return rc;
            std::swap(P2, Q0);
            std::swap(P1, Q1);
        }
        if (n_steps - n + 1 >= 2) {
            // the steps left, fewer than a full pass, in one shorter pass
            const int rest = n_steps - n + 1;
            V.n = n; V.a2 = P2; V.a1 = P1; V.out = Q0; V.out2 = Q1;
            if ((rc = launch_vc(V, rest, f32, st)) || (rc = vc_reduce(segsK, n, rest))) return rc;
            std::swap(P2, Q0);
            std::swap(P1, Q1);
            n += rest;
        }
        V.n_segs = segs1;
        for (; n <= n_steps; ++n) {
            V.n = n; V.a1 = P1; V.a2 = P2; V.out = P2;
            if ((rc = launch_vc(V, 1, f32, st)) || (rc = vc_reduce(segs1, n, 1))) return rc;
            std::swap(P1, P2);
        }
        // P2 = a_{M-1}, P1 = a_M (M = n_steps)
        if (vc_out) {
            // one step more for the reverse pass: a_{M+1} into P2
            V.n = n_steps + 1; V.a1 = P1; V.a2 = P2; V.out = P2;
            if ((rc = launch_vc(V, 1, f32, st)) || (rc = vc_reduce(segs1, n_steps + 1, 1))) return rc;
            vc_out[0] = P2; vc_out[1] = P1; vc_out[2] = Q0; vc_out[3] = Q1; vc_out[4] = vc_coef;
        }
        return bound_moments(mee, mhe, (int64_t)Bt * N, false, false, moment_limit(f32), st);
    };
    if (n_start > 0 && vc_tile((int)std::min<int64_t>(tile, n_start))) {
        int rc = launch_vc_coef(onsite, vc_coef, op->Lx, f32, L2, st);
        if (rc) return rc;
    }
    for (int64_t t0 = 0; t0 < n_start; t0 += tile) {
        const int Bt = (int)std::min<int64_t>(tile, n_start - t0);
        const int64_t Bp = lane_stride(Bt);
        double *mee = mu_ee + t0 * N;
        double *mhe = mu_he + t0 * N * he_mult;
        const int32_t *ts = sites + t0;
        if constexpr (!C) {
            if (vc_tile(Bt)) {
                int rc = run_tile_vc(Bt, Bp, ts, mee, mhe);
                if (rc) return rc;
                continue;
            }
        }
        const int64_t nz = L2 * Bp;
        const unsigned zgrid = (unsigned)std::min<int64_t>(ceil_div(nz, kBlock), 8192);
        for (int i = 0; i < nbuf; ++i) {
            if (i == 1) continue;  // a_1 is written whole by the first step
            hipLaunchKernelGGL((k_zero<T, C>), dim3(zgrid), dim3(kBlock), 0, st, buf[i], nz);
            CBDG_CHECK_LAUNCH("k_zero");
        }
        hipLaunchKernelGGL((k_seed<T, C>), dim3((unsigned)ceil_div(Bt, kBlock)), dim3(kBlock), 0, st,
                           buf[0], Bp, Bt, L2, ts, mee, mhe, N);
        CBDG_CHECK_LAUNCH("k_seed");
        hipLaunchKernelGGL(k_tile_cone, dim3(1), dim3(kBlock), 0, st, ts, Bt, op->Lx, L2, cone);
        CBDG_CHECK_LAUNCH("k_tile_cone");
        StepArgs A{};
        if (nb_ee) {
            A.nb_ee = nb_ee + t0 * 4 * N * he_mult;
            A.nb_he = nb_he + t0 * 4 * N * he_mult;
            hipLaunchKernelGGL(k_seed_nb, dim3((unsigned)std::min<int64_t>(ceil_div((int64_t)Bt * 4 * N * he_mult, kBlock), 4096)),
                               dim3(kBlock), 0, st, A.nb_ee, A.nb_he, ts, Bt, L2, N, C ? 1 : 0);
            CBDG_CHECK_LAUNCH("k_seed_nb");
        }
        A.cone = cone;
        A.onsite = onsite;
        A.bonds = bonds;
        A.th = op->t / op->bounds.a;
        A.Lx = op->Lx; A.Ly = op->Ly; A.bcx = op->bc_x; A.bcy = op->bc_y;
        A.Bp = (int)Bp; A.Bt = Bt; A.N = N;
        A.sites = ts; A.mu_he = mhe;
        const int n_steps = doubling ? N / 2 : N - 1;
        const int64_t chunks = ceil_div(Bt, kBlock);
        const Shape sh1 = choose_shape<T, C>(op->Lx, op->Ly, chunks);
        const int64_t regions1 = (int64_t)sh1.n_strips * sh1.n_segs;
        int64_t regions2 = 0, regions3 = 0;
        if (two) {
            const Shape sh2 = choose_shape2<T, C>(op->Lx, op->Ly, chunks);
            regions2 = (int64_t)sh2.n_strips * sh2.n_segs;
        }
        if (three) {
            const Shape sh3 = choose_shape3<T>(op->Lx, op->Ly, chunks);
            regions3 = (int64_t)sh3.n_strips * sh3.n_segs;
        }
        // P2 holds a_{n-2}, P1 a_{n-1}; Q0, Q1 are free (two-step passes)
        S *P2 = buf[0], *P1 = buf[1], *Q0 = buf[2], *Q1 = buf[3];
        int n = 1;
        if (n_steps >= 1) {
            A.first = 1;
            A.n = 1;
            A.prev1 = P2;
            A.prev2 = P2;
            A.out = P1;
            A.part = doubling ? part : nullptr;
            A.mu_ee = mee;
            int rc = op->general ? launch_step<T, C, true>(A, st) : launch_step<T, C, false>(A, st);
            if (rc) return rc;
            if (doubling && (rc = reduce(regions1, 1, 1, Bt, Bp, mee, mhe))) return rc;
            n = 2;
        }
        A.first = 0;
        A.mu_ee = doubling ? nullptr : mee;
        if constexpr (!C) {
            while (three && Bt >= kThreeStepMinVectors && n + 2 <= n_steps) {
                A.n = n;
                A.prev2 = P2;
                A.prev1 = P1;
                A.out = Q0;
                A.out2 = Q1;
                A.part = doubling ? part : nullptr;
                A.part_b = doubling ? part_b : nullptr;
                A.part_c = doubling ? part_c : nullptr;
                int rc = launch_step3<T>(A, st);
                if (rc) return rc;
                if (doubling && (rc = reduce(regions3, n, 3, Bt, Bp, mee, mhe))) return rc;
                std::swap(P2, Q0);
                std::swap(P1, Q1);
                n += 3;
            }
        }
        while (two && n + 1 <= n_steps) {
            A.n = n;
            A.prev2 = P2;
            A.prev1 = P1;
            A.out = Q0;
            A.out2 = Q1;
            A.part = doubling ? part : nullptr;
            A.part_b = doubling ? part_b : nullptr;
            int rc;
#if CBDG_TWO_STEP_GEN
            rc = op->general ? launch_step2<T, C, true>(A, st) : launch_step2<T, C, false>(A, st);
#else
            if constexpr (C) rc = fail(CBDG_EUNSUPPORTED, "chebyshev_moments: two-step passes for complex operators are off");
            else if (op->general) rc = fail(CBDG_EUNSUPPORTED, "chebyshev_moments: two-step passes for bond coefficients are off");
            else rc = launch_step2<T, false, false>(A, st);
#endif
            if (rc) return rc;
            if (doubling && (rc = reduce(regions2, n, 2, Bt, Bp, mee, mhe))) return rc;
            std::swap(P2, Q0);
            std::swap(P1, Q1);
            n += 2;
        }
        for (; n <= n_steps; ++n) {
            A.n = n;
            A.prev1 = P1;
            A.prev2 = P2;
            A.out = P2;
            A.part = doubling ? part : nullptr;
            int rc = op->general ? launch_step<T, C, true>(A, st) : launch_step<T, C, false>(A, st);
            if (rc) return rc;
            if (doubling && (rc = reduce(regions1, n, 1, Bt, Bp, mee, mhe))) return rc;
            std::swap(P1, P2);
        }
        const double lim = moment_limit(std::is_same<T, float>::value);
        int rc = bound_moments(mee, mhe, (int64_t)Bt * N, false, C, lim, st);
        if (rc) return rc;
        if (nb_ee && (rc = bound_moments(A.nb_ee, A.nb_he, (int64_t)Bt * 4 * N, C, C, lim, st))) return rc;
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

// Resolves CBDG_ALG_AUTO; fails for doubling with b != 0 (the particle-hole
// partner of a_n is then no longer (-1)^n-related to it).
static int resolve_algorithm(const cbdg_op *op, int32_t algorithm, int32_t N, const char *who, bool *doubling)
{
    const bool centred = op->bounds.b == 0.0;
    switch (algorithm) {
    case CBDG_ALG_AUTO: *doubling = centred && N >= 3; return CBDG_OK;
    case CBDG_ALG_DIRECT: *doubling = false; return CBDG_OK;
    case CBDG_ALG_DOUBLING:
        if (!centred) return fail(CBDG_EINVAL, "%s: moment doubling needs a spectrum centred at b = 0 (b = %g)", who, op->bounds.b);
        *doubling = N >= 3;
        return CBDG_OK;
    default: return fail(CBDG_EINVAL, "%s: unknown algorithm %d", who, algorithm);
    }
}

static int64_t doubling_partial_bytes(const cbdg_op *op, int tile, int precision)
{
    const bool cplx = op->scalar == CBDG_COMPLEX;
    const bool two = uses_two_step(op);
    const int K = cplx ? 4 : 3;
    int64_t R;
    const bool three = two && !cplx && !op->general && (precision == CBDG_FP64 ? Step3Shape<double>::ON : Step3Shape<float>::ON);
    if (precision == CBDG_FP64)
        R = cplx ? std::max(max_regions<double, true>(op->Lx, op->Ly, tile), two ? max_regions2<double, true>(op->Lx, op->Ly, tile) : 0)
                 : std::max({max_regions<double, false>(op->Lx, op->Ly, tile), two ? max_regions2<double, false>(op->Lx, op->Ly, tile) : 0,
                             three ? max_regions3<double>(op->Lx, op->Ly, tile) : 0});
    else
        R = cplx ? std::max(max_regions<float, true>(op->Lx, op->Ly, tile), two ? max_regions2<float, true>(op->Lx, op->Ly, tile) : 0)
                 : std::max({max_regions<float, false>(op->Lx, op->Ly, tile), two ? max_regions2<float, false>(op->Lx, op->Ly, tile) : 0,
                             three ? max_regions3<float>(op->Lx, op->Ly, tile) : 0});
    // partials of up to kMaxPassSteps steps, then their run sums at a stride
    // of kMaxGroups runs
    return kMaxPassSteps * (R + (int64_t)kMaxGroups) * K * lane_stride(tile) * (int64_t)sizeof(double);
}

// Packed coefficients of the vector-contiguous passes (operators they run on)
static size_t vc_coef_bytes(const cbdg_op *op, int precision)
{
    const bool f32 = precision != CBDG_FP64;
    if (op->scalar != CBDG_REAL || op->general || !uses_two_step(op) || !vc_width(op->Lx, f32)) return 0;
    return (size_t)op->L2 * 2 * (f32 ? sizeof(float) : sizeof(double));
}

static size_t tile_buffer_bytes(const cbdg_op *op, int64_t tile, int precision)
{
    const size_t nbuf = uses_two_step(op) ? 4 : 2;
    return nbuf * (size_t)op->L2 * (size_t)lane_stride(tile) * pair_bytes(op->scalar, precision);
}

namespace cbdg {

bool vc_adjoint_supported(const cbdg_op *op)
{
    return op && op->scalar == CBDG_REAL && !op->general && op->bounds.b == 0.0 && uses_two_step(op) &&
           vc_width(op->Lx, false) > 0;
}

int vc_forward_last(const cbdg_op *op, const int32_t *sites, int Bt, int N, void *ws, double *mu_ee, double *mu_he,
                    hipStream_t st, void **last, void **spare, const void **coef)
{
    if (!vc_adjoint_supported(op) || N < 3 || Bt < kVcMinVectors)
        return fail(CBDG_EUNSUPPORTED, "chebyshev_moments_backward: the reverse passes need the vector-contiguous "
                    "forward (real operator, uniform hopping, b = 0, Lx = 64 W, N >= 3)");
    void *out[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    int rc = run_moments<double, false>(op, sites, Bt, N, Bt, true, ws, mu_ee, mu_he, st, nullptr, nullptr, out);
    if (rc) return rc;
    if (!out[0]) return fail(CBDG_EINVAL, "chebyshev_moments_backward: the forward did not take the vector-contiguous passes");
    last[0] = out[0]; last[1] = out[1]; spare[0] = out[2]; spare[1] = out[3]; *coef = out[4];
    return CBDG_OK;
}

}  // namespace cbdg

extern "C" int cbdg_moments_workspace_size(const cbdg_op *op, int32_t tile, int32_t precision, int32_t algorithm,
                                           size_t *bytes)
{
    clear_error();
    if (!op || !bytes) return fail(CBDG_EINVAL, "moments_workspace_size: op and bytes must not be NULL");
    if (tile < 1) return fail(CBDG_EINVAL, "moments_workspace_size: tile must be >= 1");
    if (precision != CBDG_FP64 && precision != CBDG_FP32_ACC64)
        return fail(CBDG_EINVAL, "moments_workspace_size: unknown precision %d", precision);
    bool doubling = false;
    // sized for any N: the partials are included whenever doubling may run
    int rc = resolve_algorithm(op, algorithm, 3, "moments_workspace_size", &doubling);
    if (rc) return rc;
    *bytes = tile_buffer_bytes(op, tile, precision) + kConeDoubles * sizeof(double);
    if (doubling) *bytes += (size_t)doubling_partial_bytes(op, tile, precision) + vc_coef_bytes(op, precision);
    return CBDG_OK;
}

extern "C" int cbdg_chebyshev_moments(const cbdg_op *op, const int32_t *start_sites, int64_t n_start,
                                      int32_t N, int32_t tile, int32_t precision, int32_t algorithm,
                                      void *workspace, size_t workspace_bytes, double *mu_ee, void *mu_he,
                                      void *stream)
{
    clear_error();
    if (!op) return fail(CBDG_EINVAL, "chebyshev_moments: op must not be NULL");
    if (n_start < 0) return fail(CBDG_EINVAL, "chebyshev_moments: n_start must be >= 0");
    if (N < 1) return fail(CBDG_EINVAL, "chebyshev_moments: N must be >= 1");
    if (tile < 1) return fail(CBDG_EINVAL, "chebyshev_moments: tile must be >= 1");
    if (precision != CBDG_FP64 && precision != CBDG_FP32_ACC64)
        return fail(CBDG_EINVAL, "chebyshev_moments: unknown precision %d", precision);
    bool doubling = false;
    int rc = resolve_algorithm(op, algorithm, N, "chebyshev_moments", &doubling);
    if (rc) return rc;
    if (n_start == 0) return CBDG_OK;
    if (!start_sites || !mu_ee || !mu_he || !workspace)
        return fail(CBDG_EINVAL, "chebyshev_moments: start_sites, mu_ee, mu_he and workspace must not be NULL");
    const int64_t eff_tile = std::min<int64_t>(tile, n_start);
    size_t need = tile_buffer_bytes(op, eff_tile, precision) + kConeDoubles * sizeof(double);
    if (doubling) need += (size_t)doubling_partial_bytes(op, (int)eff_tile, precision) + vc_coef_bytes(op, precision);
    if (workspace_bytes < need)
        return fail(CBDG_EINVAL, "chebyshev_moments: workspace of %zu bytes is smaller than the %zu needed",
                    workspace_bytes, need);
    hipStream_t st = as_stream(stream);
    double *mhe = reinterpret_cast<double *>(mu_he);
    const bool cplx = op->scalar == CBDG_COMPLEX;
    const int et = (int)eff_tile;
    if (precision == CBDG_FP64)
        return cplx ? run_moments<double, true>(op, start_sites, n_start, N, et, doubling, workspace, mu_ee, mhe, st)
                    : run_moments<double, false>(op, start_sites, n_start, N, et, doubling, workspace, mu_ee, mhe, st);
    return cplx ? run_moments<float, true>(op, start_sites, n_start, N, et, doubling, workspace, mu_ee, mhe, st)
                : run_moments<float, false>(op, start_sites, n_start, N, et, doubling, workspace, mu_ee, mhe, st);
}

extern "C" int cbdg_chebyshev_moments_nb(const cbdg_op *op, const int32_t *start_sites, int64_t n_start,
                                         int32_t N, int32_t tile, int32_t precision, void *workspace,
                                         size_t workspace_bytes, double *mu_ee, void *mu_he, void *nb_ee,
                                         void *nb_he, void *stream)
{
    clear_error();
    if (!op) return fail(CBDG_EINVAL, "chebyshev_moments_nb: op must not be NULL");
    if (n_start < 0 || N < 1 || tile < 1) return fail(CBDG_EINVAL, "chebyshev_moments_nb: need n_start >= 0, N >= 1, tile >= 1");
    if (precision != CBDG_FP64 && precision != CBDG_FP32_ACC64)
        return fail(CBDG_EINVAL, "chebyshev_moments_nb: unknown precision %d", precision);
    if (n_start == 0) return CBDG_OK;
    if (!start_sites || !mu_ee || !mu_he || !nb_ee || !nb_he || !workspace)
        return fail(CBDG_EINVAL, "chebyshev_moments_nb: start_sites, moment outputs and workspace must not be NULL");
    const int64_t eff_tile = std::min<int64_t>(tile, n_start);
    size_t need = 2 * (size_t)op->L2 * (size_t)lane_stride(eff_tile) * pair_bytes(op->scalar, precision) +
                  kConeDoubles * sizeof(double);
    if (workspace_bytes < need)
        return fail(CBDG_EINVAL, "chebyshev_moments_nb: workspace of %zu bytes is smaller than the %zu needed",
                    workspace_bytes, need);
    hipStream_t st = as_stream(stream);
    double *mhe = reinterpret_cast<double *>(mu_he);
    double *ne = reinterpret_cast<double *>(nb_ee), *nh = reinterpret_cast<double *>(nb_he);
    const bool cplx = op->scalar == CBDG_COMPLEX;
    const int et = (int)eff_tile;
    if (precision == CBDG_FP64)
        return cplx ? run_moments<double, true>(op, start_sites, n_start, N, et, false, workspace, mu_ee, mhe, st, ne, nh)
                    : run_moments<double, false>(op, start_sites, n_start, N, et, false, workspace, mu_ee, mhe, st, ne, nh);
    return cplx ? run_moments<float, true>(op, start_sites, n_start, N, et, false, workspace, mu_ee, mhe, st, ne, nh)
                : run_moments<float, false>(op, start_sites, n_start, N, et, false, workspace, mu_ee, mhe, st, ne, nh);
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

// ---------------------------------------------------------------------------
// Moments without a caller workspace, for callers that cannot allocate device
// memory.  The workspace lives in a device array of fixed size that each GPU
// holds for the life of the process; host code reaches it only through the
// address hipGetSymbolAddress reports for the current device (the array's
// name in host code is not a device address).
#include <mutex>

static __device__ __align__(256) unsigned char scratch[CBDG_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of the current device's scratch array (looked up once per
// device, with that device current).
static int static_scratch(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(CBDG_EINVAL, "chebyshev_moments_static: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CBDG_EHIP, "chebyshev_moments_static: hipGetSymbolAddress failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CBDG_OK;
}

extern "C" size_t cbdg_static_scratch_bytes(void) { return (size_t)CBDG_STATIC_SCRATCH_BYTES; }

extern "C" int cbdg_chebyshev_moments_static(const cbdg_op *op, const int32_t *start_sites, int64_t n_start,
                                             int32_t N, int32_t tile, int32_t precision, int32_t algorithm,
                                             double *mu_ee, void *mu_he, void *stream)
{
    clear_error();
    if (!op) return fail(CBDG_EINVAL, "chebyshev_moments_static: op must not be NULL");
    if (n_start < 0 || N < 1 || tile < 1)
        return fail(CBDG_EINVAL, "chebyshev_moments_static: need n_start >= 0, N >= 1, tile >= 1");
    if (precision != CBDG_FP64 && precision != CBDG_FP32_ACC64)
        return fail(CBDG_EINVAL, "chebyshev_moments_static: unknown precision %d", precision);
    int dev = -1;
    CBDG_CHECK_HIP(hipGetDevice(&dev));
    if (dev != op->device)
        return fail(CBDG_EINVAL, "chebyshev_moments_static: the operator lives on device %d, the current device is %d",
                    op->device, dev);
    if (n_start == 0) return CBDG_OK;
    size_t need = 0;
    const int32_t eff = (int32_t)std::min<int64_t>(tile, n_start);
    int rc = cbdg_moments_workspace_size(op, eff, precision, algorithm, &need);
    if (rc) return rc;
    if (need > (size_t)CBDG_STATIC_SCRATCH_BYTES)
        return fail(CBDG_EINVAL,
                    "chebyshev_moments_static: tiles of %d vectors need %zu bytes of workspace, more than the %zu "
                    "of the static scratch array (use smaller tiles or cbdg_chebyshev_moments)",
                    eff, need, (size_t)CBDG_STATIC_SCRATCH_BYTES);
    void *ws = nullptr;
    if ((rc = static_scratch(dev, &ws))) return rc;
    // every buffer the recursion reads is written first within the call
    // (tile buffers cleared per tile or written before they are read,
    // bounding box, partial and run sums), so the previous call's contents
    // need no clearing
    return cbdg_chebyshev_moments(op, start_sites, n_start, N, tile, precision, algorithm, ws, need, mu_ee, mu_he,
                                  stream);
}
