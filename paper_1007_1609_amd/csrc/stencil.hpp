// Device-side building blocks of the matrix-free Nambu BdG stencil:
// Nambu pairs of one start vector at one site, their loads and stores, and
// the action of the rescaled operator Ht on one site (eq. (hamil2)).
#pragma once

#include "common.hpp"

namespace cbdg {

// One Nambu pair (electron, hole) of one vector at one site.
template <typename T, bool C> struct Pair;
template <typename T> struct Pair<T, false> { T e, h; };
template <typename T> struct Pair<T, true> { T er, ei, hr, hi; };

template <typename T, bool C> struct Storage;
template <> struct Storage<double, false> { using type = double2; };
template <> struct Storage<float, false> { using type = float2; };
template <> struct Storage<double, true> { using type = double4; };
template <> struct Storage<float, true> { using type = float4; };

template <typename T, bool C> __device__ __forceinline__ Pair<T, C> zero_pair()
{
    Pair<T, C> p;
    if constexpr (C) { p.er = p.ei = p.hr = p.hi = T(0); }
    else { p.e = p.h = T(0); }
    return p;
}

// v with every bit cleared when mask == 0 (mask is 0 or ~0u): zeroes halo
// values without a branch and independently of their content.
__device__ __forceinline__ double mask_bits(double v, uint32_t m)
{
    const unsigned long long mm = ((unsigned long long)m << 32) | m;
    return __longlong_as_double((long long)((unsigned long long)__double_as_longlong(v) & mm));
}
__device__ __forceinline__ float mask_bits(float v, uint32_t m) { return __uint_as_float(__float_as_uint(v) & m); }

// c ? a : b component by component (a select of whole structs would be
// lowered through stack memory)
template <typename T, bool C>
__device__ __forceinline__ Pair<T, C> select_pair(bool c, const Pair<T, C> &a, const Pair<T, C> &b)
{
    Pair<T, C> r;
    if constexpr (C) {
        r.er = c ? a.er : b.er; r.ei = c ? a.ei : b.ei;
        r.hr = c ? a.hr : b.hr; r.hi = c ? a.hi : b.hi;
    } else {
        r.e = c ? a.e : b.e; r.h = c ? a.h : b.h;
    }
    return r;
}

template <typename T, bool C>
__device__ __forceinline__ Pair<T, C> masked(const Pair<T, C> &v, uint32_t mask)
{
    Pair<T, C> r;
    if constexpr (C) {
        r.er = mask_bits(v.er, mask); r.ei = mask_bits(v.ei, mask);
        r.hr = mask_bits(v.hr, mask); r.hi = mask_bits(v.hi, mask);
    } else {
        r.e = mask_bits(v.e, mask); r.h = mask_bits(v.h, mask);
    }
    return r;
}

template <typename T, bool C>
__device__ __forceinline__ Pair<T, C> ld(const typename Storage<T, C>::type *p)
{
    Pair<T, C> r;
    if constexpr (C) {
        if constexpr (sizeof(T) == 8) {
            const double2 *q = reinterpret_cast<const double2 *>(p);
            double2 u = q[0], v = q[1];
            r.er = u.x; r.ei = u.y; r.hr = v.x; r.hi = v.y;
        } else {
            float4 u = *p;
            r.er = u.x; r.ei = u.y; r.hr = u.z; r.hi = u.w;
        }
    } else {
        auto u = *p;
        r.e = u.x; r.h = u.y;
    }
    return r;
}

// Streaming (nontemporal) variants: data read or written once per step is
// marked so it does not displace the halo rows other strips still need.
template <typename T, int N> using Vec = T __attribute__((ext_vector_type(N)));

template <typename T, bool C>
__device__ __forceinline__ Pair<T, C> ld_nt(const typename Storage<T, C>::type *p)
{
    Pair<T, C> r;
    if constexpr (C) {
        if constexpr (sizeof(T) == 8) {
            const Vec<double, 2> *q = reinterpret_cast<const Vec<double, 2> *>(p);
            Vec<double, 2> u = __builtin_nontemporal_load(q), v = __builtin_nontemporal_load(q + 1);
            r.er = u.x; r.ei = u.y; r.hr = v.x; r.hi = v.y;
        } else {
            Vec<float, 4> u = __builtin_nontemporal_load(reinterpret_cast<const Vec<float, 4> *>(p));
            r.er = u.x; r.ei = u.y; r.hr = u.z; r.hi = u.w;
        }
    } else {
        Vec<T, 2> u = __builtin_nontemporal_load(reinterpret_cast<const Vec<T, 2> *>(p));
        r.e = u.x; r.h = u.y;
    }
    return r;
}

template <typename T, bool C>
__device__ __forceinline__ void st_nt(typename Storage<T, C>::type *p, const Pair<T, C> &v)
{
    if constexpr (C) {
        if constexpr (sizeof(T) == 8) {
            Vec<double, 2> *q = reinterpret_cast<Vec<double, 2> *>(p);
            __builtin_nontemporal_store(Vec<double, 2>{v.er, v.ei}, q);
            __builtin_nontemporal_store(Vec<double, 2>{v.hr, v.hi}, q + 1);
        } else {
            __builtin_nontemporal_store(Vec<float, 4>{v.er, v.ei, v.hr, v.hi}, reinterpret_cast<Vec<float, 4> *>(p));
        }
    } else {
        __builtin_nontemporal_store(Vec<T, 2>{v.e, v.h}, reinterpret_cast<Vec<T, 2> *>(p));
    }
}

template <typename T, bool C>
__device__ __forceinline__ void st(typename Storage<T, C>::type *p, const Pair<T, C> &v)
{
    if constexpr (C) {
        if constexpr (sizeof(T) == 8) {
            double2 *q = reinterpret_cast<double2 *>(p);
            q[0] = double2{v.er, v.ei};
            q[1] = double2{v.hr, v.hi};
        } else {
            *p = float4{v.er, v.ei, v.hr, v.hi};
        }
    } else {
        using S = typename Storage<T, C>::type;
        *p = S{v.e, v.h};
    }
}

// Neighbour coefficients of site i towards j: hopping t_ij and bond pairing
// Delta_ij (both divided by a).  Uniform operators carry one real t.
template <typename T, bool C> struct Link;
template <typename T> struct Link<T, false> { T t, d; };
template <typename T> struct Link<T, true> { T tr, ti, dr, di; };

// (Ht a)(i) for one vector, given the pair at i, its four neighbours and the
// four links:
//   (Ht a)(i,e) = de a(i,e) + Delta_i a(i,h) + sum_j [-t_ij a(j,e) + Delta_ij a(j,h)]
//   (Ht a)(i,h) = conj(Delta_i) a(i,e) + dh a(i,h) + sum_j [conj(Delta_ij) a(j,e) + conj(t_ij) a(j,h)]
template <typename T, bool C>
__device__ __forceinline__ Pair<T, C> apply_general(const OnSite<T> &o, const Pair<T, C> &c,
                                                    const Pair<T, C> *nb, const Link<T, C> *lk)
{
    Pair<T, C> r;
    if constexpr (C) {
        // on-site
        T er = o.de * c.er + (o.dr * c.hr - o.di * c.hi);
        T ei = o.de * c.ei + (o.dr * c.hi + o.di * c.hr);
        T hr = (o.dr * c.er + o.di * c.ei) + o.dh * c.hr;
        T hi = (o.dr * c.ei - o.di * c.er) + o.dh * c.hi;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const Pair<T, C> &a = nb[q];
            const Link<T, C> &l = lk[q];
            // -t a_e + d a_h
            er += -(l.tr * a.er - l.ti * a.ei) + (l.dr * a.hr - l.di * a.hi);
            ei += -(l.tr * a.ei + l.ti * a.er) + (l.dr * a.hi + l.di * a.hr);
            // conj(d) a_e + conj(t) a_h
            hr += (l.dr * a.er + l.di * a.ei) + (l.tr * a.hr + l.ti * a.hi);
            hi += (l.dr * a.ei - l.di * a.er) + (l.tr * a.hi - l.ti * a.hr);
        }
        r.er = er; r.ei = ei; r.hr = hr; r.hi = hi;
    } else {
        T e = o.de * c.e + o.dr * c.h;
        T h = o.dr * c.e + o.dh * c.h;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            e += -lk[q].t * nb[q].e + lk[q].d * nb[q].h;
            h += lk[q].d * nb[q].e + lk[q].t * nb[q].h;
        }
        r.e = e; r.h = h;
    }
    return r;
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Uniform real hopping t (th = t/a) and no bond pairing.  The fused
// multiply-adds are written out and no other contraction is allowed, so
// every kernel that applies Ht (one, two or three steps per launch, the
// adjoint) rounds a site's value identically.
template <typename T, bool C>
__device__ __forceinline__ Pair<T, C> apply_uniform(const OnSite<T> &o, T th, const Pair<T, C> &c,
                                                    const Pair<T, C> &l, const Pair<T, C> &r,
                                                    const Pair<T, C> &d, const Pair<T, C> &u)
{
#pragma clang fp contract(off)
    Pair<T, C> y;
    if constexpr (C) {
        const T ser = (l.er + r.er) + (d.er + u.er), sei = (l.ei + r.ei) + (d.ei + u.ei);
        const T shr = (l.hr + r.hr) + (d.hr + u.hr), shi = (l.hi + r.hi) + (d.hi + u.hi);
        y.er = fma_t(o.de, c.er, fma_t(o.dr, c.hr, fma_t(-o.di, c.hi, -(th * ser))));
        y.ei = fma_t(o.de, c.ei, fma_t(o.dr, c.hi, fma_t(o.di, c.hr, -(th * sei))));
        y.hr = fma_t(o.dh, c.hr, fma_t(o.dr, c.er, fma_t(o.di, c.ei, th * shr)));
        y.hi = fma_t(o.dh, c.hi, fma_t(o.dr, c.ei, fma_t(-o.di, c.er, th * shi)));
    } else {
        const T se = (l.e + r.e) + (d.e + u.e), sh = (l.h + r.h) + (d.h + u.h);
        y.e = fma_t(o.de, c.e, fma_t(o.dr, c.h, -(th * se)));
        y.h = fma_t(o.dh, c.h, fma_t(o.dr, c.e, th * sh));
    }
    return y;
}

// out = 2 y - p   (or y on the first step), one fused multiply-add per
// component: 2y is exact, so fma(2, y, -p) rounds 2y - p exactly as the
// product followed by the subtraction would
template <typename T, bool C>
__device__ __forceinline__ Pair<T, C> cheb_combine(const Pair<T, C> &y, const Pair<T, C> &p, bool first)
{
#pragma clang fp contract(off)
    Pair<T, C> o;
    if constexpr (C) {
        o.er = first ? y.er : fma_t(T(2), y.er, -p.er);
        o.ei = first ? y.ei : fma_t(T(2), y.ei, -p.ei);
        o.hr = first ? y.hr : fma_t(T(2), y.hr, -p.hr);
        o.hi = first ? y.hi : fma_t(T(2), y.hi, -p.hi);
    } else {
        o.e = first ? y.e : fma_t(T(2), y.e, -p.e);
        o.h = first ? y.h : fma_t(T(2), y.h, -p.h);
    }
    return o;
}

// Links of site (x, y): +x, -x, +y, -y, built from the forward bond
// coefficients of the site and of its backward neighbours (t_ji = conj(t_ij),
// Delta_ji = Delta_ij).  A missing neighbour gets a zero link; its halo pair
// is zero too.
template <typename T, bool C>
__device__ __forceinline__ void links_of(const void *bonds, int64_t s, int64_t s_left, int64_t s_down,
                                         Link<T, C> *lk)
{
    if constexpr (C) {
        const BondsC<T> *B = reinterpret_cast<const BondsC<T> *>(bonds);
        const BondsC<T> o = B[s];
        lk[0] = Link<T, C>{o.txr, o.txi, o.dxr, o.dxi};
        lk[2] = Link<T, C>{o.tyr, o.tyi, o.dyr, o.dyi};
        if (s_left >= 0) { const BondsC<T> q = B[s_left]; lk[1] = Link<T, C>{q.txr, -q.txi, q.dxr, q.dxi}; }
        else lk[1] = Link<T, C>{T(0), T(0), T(0), T(0)};
        if (s_down >= 0) { const BondsC<T> q = B[s_down]; lk[3] = Link<T, C>{q.tyr, -q.tyi, q.dyr, q.dyi}; }
        else lk[3] = Link<T, C>{T(0), T(0), T(0), T(0)};
    } else {
        const BondsR<T> *B = reinterpret_cast<const BondsR<T> *>(bonds);
        const BondsR<T> o = B[s];
        lk[0] = Link<T, C>{o.tx, o.dx};
        lk[2] = Link<T, C>{o.ty, o.dy};
        if (s_left >= 0) { const BondsR<T> q = B[s_left]; lk[1] = Link<T, C>{q.tx, q.dx}; }
        else lk[1] = Link<T, C>{T(0), T(0)};
        if (s_down >= 0) { const BondsR<T> q = B[s_down]; lk[3] = Link<T, C>{q.ty, q.dy}; }
        else lk[3] = Link<T, C>{T(0), T(0)};
    }
}

// Maps a hardware workgroup id to a logical tile id so that consecutive
// logical ids run on the same XCD (workgroups are dispatched round-robin over
// the 8 XCDs): neighbouring strips then share their halo rows in one L2.
__device__ __forceinline__ int xcd_remap(int id, int n)
{
    constexpr int kXcd = 8;
    const int q = n / kXcd, r = n % kXcd;
    const int xcd = id % kXcd, k = id / kXcd;
    return (xcd < r) ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

}  // namespace cbdg
