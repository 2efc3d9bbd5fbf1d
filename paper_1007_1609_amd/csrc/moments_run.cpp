// Native runner of one batched-moments call through the C ABI (no Python and
// no torch in the process), for profilers that read hardware counters per
// dispatch.
//
// It builds the rescaled operator of eq. (hamil2) on an Lx x Ly open lattice
// with real s-wave pairing (t = 1, mu_c = -0.4, Delta_i = 0.1, Gershgorin
// bound with the Delta cap 1.25, eta = 0.01; on-site potential +1.5 / -1.5
// on every 100th site), runs cbdg_chebyshev_moments over the start sites
// first .. first+n_start-1 (first = 0 unless given) in tiles of `tile` with
// moment doubling, checks the bound
// |mu| <= 1 on the device, and, when copy_mib > 0, copies copy_mib MiB from
// one device buffer to another: a transfer of known size that scales what
// the memory counters read.  Which kernels run, their grids and the vector
// bytes each launch moves depend on the lattice, the sites, N, the tile and
// the precision only, never on the operator's values.
//
//   cbdg_moments_run Lx Ly N tile n_start fp64|fp32 [copy_mib [first]]
//
// Prints one line per phase; exits with 1 on any failure (the library's
// message is printed).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "cbdg.h"

namespace {

int fail(const char *what, int rc) {
    std::fprintf(stderr, "cbdg_moments_run: %s failed (%d): %s\n", what, rc, cbdg_last_error());
    return 1;
}

int hip_fail(const char *what, hipError_t e) {
    std::fprintf(stderr, "cbdg_moments_run: %s: %s\n", what, hipGetErrorString(e));
    return 1;
}

#define HIP_OK(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return hip_fail(#call, e_); \
    } while (0)

}  // namespace

int main(int argc, char **argv) {
    if (argc < 7) {
        std::fprintf(stderr, "usage: %s Lx Ly N tile n_start fp64|fp32 [copy_mib [first]]\n", argv[0]);
        return 2;
    }
    const int Lx = std::atoi(argv[1]), Ly = std::atoi(argv[2]);
    const int N = std::atoi(argv[3]), tile = std::atoi(argv[4]);
    const long long n_start = std::atoll(argv[5]);
    const bool f32 = std::strcmp(argv[6], "fp32") == 0;
    if (!f32 && std::strcmp(argv[6], "fp64") != 0) {
        std::fprintf(stderr, "precision must be fp64 or fp32\n");
        return 2;
    }
    const long long copy_mib = argc > 7 ? std::atoll(argv[7]) : 0;
    const long long first = argc > 8 ? std::atoll(argv[8]) : 0;
    const long long L2 = (long long)Lx * Ly;
    if (Lx < 1 || Ly < 1 || N < 1 || tile < 1 || n_start < 1 || first < 0 || first + n_start > L2 || copy_mib < 0) {
        std::fprintf(stderr, "bad sizes\n");
        return 2;
    }

    std::vector<double> eps(L2, 0.0), delta(L2, 0.1);
    for (long long i = 0; i < L2; i += 100) eps[i] = (i / 100) % 2 ? -1.5 : 1.5;
    std::vector<int32_t> sites(n_start);
    for (long long i = 0; i < n_start; ++i) sites[i] = (int32_t)(first + i);

    double *d_eps = nullptr, *d_delta = nullptr, *mu_ee = nullptr, *mu_he = nullptr;
    int32_t *d_sites = nullptr, *d_flag = nullptr;
    void *ws = nullptr;
    HIP_OK(hipMalloc(&d_eps, L2 * sizeof(double)));
    HIP_OK(hipMalloc(&d_delta, L2 * sizeof(double)));
    HIP_OK(hipMalloc(&d_sites, n_start * sizeof(int32_t)));
    HIP_OK(hipMalloc(&d_flag, sizeof(int32_t)));
    HIP_OK(hipMalloc(&mu_ee, n_start * N * sizeof(double)));
    HIP_OK(hipMalloc(&mu_he, n_start * N * sizeof(double)));
    HIP_OK(hipMemcpy(d_eps, eps.data(), L2 * sizeof(double), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d_delta, delta.data(), L2 * sizeof(double), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d_sites, sites.data(), n_start * sizeof(int32_t), hipMemcpyHostToDevice));

    cbdg_lattice lat{};
    lat.Lx = Lx;
    lat.Ly = Ly;
    lat.bc_x = CBDG_BC_OPEN;
    lat.bc_y = CBDG_BC_OPEN;
    lat.scalar = CBDG_REAL;
    cbdg_op *op = nullptr;
    cbdg_bounds bounds{};
    int rc = cbdg_build_bdg(&lat, 1.0, -0.4, d_eps, d_delta, nullptr, nullptr, nullptr, 1.25, 0.01, nullptr,
                            &op, &bounds);
    if (rc) return fail("cbdg_build_bdg", rc);
    std::printf("operator %dx%d: a = %.6f, b = %.1f\n", Lx, Ly, bounds.a, bounds.b);
    std::fflush(stdout);

    const int prec = f32 ? CBDG_FP32_ACC64 : CBDG_FP64;
    size_t ws_bytes = 0;
    rc = cbdg_moments_workspace_size(op, tile, prec, CBDG_ALG_DOUBLING, &ws_bytes);
    if (rc) return fail("cbdg_moments_workspace_size", rc);
    HIP_OK(hipMalloc(&ws, ws_bytes));

    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipEventRecord(e0, nullptr));
    rc = cbdg_chebyshev_moments(op, d_sites, n_start, N, tile, prec, CBDG_ALG_DOUBLING, ws, ws_bytes, mu_ee, mu_he,
                                nullptr);
    if (rc) return fail("cbdg_chebyshev_moments", rc);
    HIP_OK(hipEventRecord(e1, nullptr));
    rc = cbdg_check_moments(mu_ee, mu_he, n_start, N, CBDG_REAL, f32 ? 1e-4 : 1e-9, d_flag, nullptr);
    if (rc) return fail("cbdg_check_moments", rc);
    HIP_OK(hipDeviceSynchronize());
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, e0, e1));
    int32_t flag = 1;
    double mu00 = 0.0;
    HIP_OK(hipMemcpy(&flag, d_flag, sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(&mu00, mu_ee, sizeof(double), hipMemcpyDeviceToHost));
    std::printf("moments: %lld start sites from %lld, N = %d, tiles of %d, %s: %.1f ms (%.4g moments/s), "
                "bounded %s, mu_ee[0][0] = %g\n",
                n_start, first, N, tile, f32 ? "fp32 vectors" : "fp64", ms, n_start * (double)N / (ms * 1e-3),
                flag ? "NO" : "yes", mu00);
    std::fflush(stdout);
    if (flag || mu00 != 1.0) {
        std::fprintf(stderr, "cbdg_moments_run: moments out of bound\n");
        return 1;
    }

    if (copy_mib > 0) {
        const size_t bytes = (size_t)copy_mib << 20;
        void *src = nullptr, *dst = nullptr;
        HIP_OK(hipMalloc(&src, bytes));
        HIP_OK(hipMalloc(&dst, bytes));
        HIP_OK(hipMemset(src, 1, bytes));
        HIP_OK(hipDeviceSynchronize());
        HIP_OK(hipEventRecord(e0, nullptr));
        HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, nullptr));
        HIP_OK(hipEventRecord(e1, nullptr));
        HIP_OK(hipDeviceSynchronize());
        HIP_OK(hipEventElapsedTime(&ms, e0, e1));
        std::printf("copy: %lld MiB device to device, %.3f ms (%.0f GB/s read + write)\n", copy_mib, ms,
                    2.0 * bytes / (ms * 1e-3) / 1e9);
        std::fflush(stdout);
        HIP_OK(hipFree(src));
        HIP_OK(hipFree(dst));
    }

    rc = cbdg_op_destroy(op);
    if (rc) return fail("cbdg_op_destroy", rc);
    HIP_OK(hipFree(ws));
    HIP_OK(hipFree(mu_ee));
    HIP_OK(hipFree(mu_he));
    HIP_OK(hipFree(d_sites));
    HIP_OK(hipFree(d_flag));
    HIP_OK(hipFree(d_eps));
    HIP_OK(hipFree(d_delta));
    return 0;
}
