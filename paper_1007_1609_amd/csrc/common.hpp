// Internal definitions shared by the translation units of libcbdg.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <cstdio>

#include "cbdg.h"

namespace cbdg {

int fail(int code, const char *fmt, ...);
void clear_error();

#define CBDG_CHECK_HIP(call)                                                          \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return ::cbdg::fail(CBDG_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define CBDG_CHECK_LAUNCH(name)                                                       \
    do {                                                                              \
        hipError_t e_ = hipGetLastError();                                            \
        if (e_ != hipSuccess)                                                         \
            return ::cbdg::fail(CBDG_EHIP, "launch of %s failed: %s", name, hipGetErrorString(e_)); \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Vectors of one tile are laid out vector-major: element (site s, vector b)
// of a Nambu pair lives at index s * lane_stride + b, lane_stride a multiple
// of the wavefront width, so every neighbour access of a wavefront is one
// contiguous run.
constexpr int kWave = 64;
constexpr int kBlock = 256;

// Per-site rescaled on-site coefficients:
//   de = (eps - mu - b)/a, dh = (-(eps - mu) - b)/a, (dr, di) = Delta/a.
template <typename T> struct alignas(4 * sizeof(T)) OnSite { T de, dh, dr, di; };

// Per-site coefficients of the two bonds leaving the site forward (+x, +y),
// divided by a: t for the hopping amplitude (with its Peierls phase) and d
// for the bond pairing.  Real operators use only the .r parts.
template <typename T> struct alignas(4 * sizeof(T)) BondsR { T tx, dx, ty, dy; };
template <typename T> struct alignas(4 * sizeof(T)) BondsC {
    T txr, txi, dxr, dxi, tyr, tyi, dyr, dyi;
};

}  // namespace cbdg

struct cbdg_op {
    int32_t Lx = 0, Ly = 0, bc_x = 0, bc_y = 0, scalar = 0;
    bool general = false;      // per-bond coefficients (Peierls phases and/or bond pairing)
    bool bond_pairing = false;
    bool peierls = false;
    double t = 0, mu_c = 0;
    cbdg_bounds bounds{};
    int device = 0;
    int64_t L2 = 0;
    // device coefficient arrays, library-owned
    cbdg::OnSite<double> *onsite64 = nullptr;
    cbdg::OnSite<float> *onsite32 = nullptr;
    void *bonds64 = nullptr;   // BondsR<double> or BondsC<double> per site
    void *bonds32 = nullptr;   // BondsR<float> or BondsC<float> per site
    double *eps = nullptr;     // copy of eps (to rebuild coefficients on update)
    unsigned long long *scratch = nullptr;  // one word for reductions
};
