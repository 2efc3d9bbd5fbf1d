// Operator construction: rescaled matrix-free coefficients of the Nambu BdG
// Hamiltonian, eq. (hamil2), and the spectral bound of the rescaling
// (paragraph after eq. (rec)).
#include "common.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

namespace cbdg {

static thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = '\0'; }

struct RawInputs {
    const double *eps;
    const double *delta;       // [L2] real or [L2][2] complex
    const double *delta_bond;  // [2][L2] real or [2][L2][2] complex, may be null
    const double *peierls;     // [2][L2], may be null
    int Lx, Ly, bcx, bcy, cplx;
    double t, mu_c;
};

__device__ inline bool has_fwd_bond(int x, int y, int axis, const RawInputs &in)
{
    if (axis == 0) return (x + 1 < in.Lx) || in.bcx;
    return (y + 1 < in.Ly) || in.bcy;
}

__device__ inline void raw_delta(const RawInputs &in, int64_t s, double &re, double &im)
{
    if (in.cplx) { re = in.delta[2 * s]; im = in.delta[2 * s + 1]; }
    else { re = in.delta[s]; im = 0.0; }
}

__device__ inline void raw_bond_delta(const RawInputs &in, int axis, int64_t s, int64_t L2,
                                      double &re, double &im)
{
    re = im = 0.0;
    if (!in.delta_bond) return;
    const int64_t q = axis * L2 + s;
    if (in.cplx) { re = in.delta_bond[2 * q]; im = in.delta_bond[2 * q + 1]; }
    else re = in.delta_bond[q];
}

// Gershgorin row sum of |H| at site s (the electron and hole rows of a site
// have the same sum), with |Delta_s| raised to at least cap.
__global__ void k_gershgorin(RawInputs in, double cap, unsigned long long *out)
{
    const int64_t L2 = (int64_t)in.Lx * in.Ly;
    double best = 0.0;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < L2;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(s % in.Lx), y = (int)(s / in.Lx);
        double dr, di;
        raw_delta(in, s, dr, di);
        double sum = fabs(in.eps[s] - in.mu_c) + fmax(hypot(dr, di), cap);
        // four neighbours: the forward bonds of s and of its backward neighbours
        for (int axis = 0; axis < 2; ++axis) {
            const int len = axis == 0 ? in.Lx : in.Ly;
            const int pos = axis == 0 ? x : y;
            const int periodic = axis == 0 ? in.bcx : in.bcy;
            const int64_t step = axis == 0 ? 1 : in.Lx;
            // forward bond owned by s
            if (pos + 1 < len || periodic) {
                double br, bi;
                raw_bond_delta(in, axis, s, L2, br, bi);
                sum += fabs(in.t) + hypot(br, bi);
            }
            // backward bond owned by the neighbour behind s
            if (pos > 0 || periodic) {
                const int64_t o = pos > 0 ? s - step : s + (int64_t)(len - 1) * step;
                double br, bi;
                raw_bond_delta(in, axis, o, L2, br, bi);
                sum += fabs(in.t) + hypot(br, bi);
            }
        }
        best = fmax(best, sum);
    }
    // block max, then one atomic max on the bit pattern (non-negative doubles
    // order like their unsigned bit patterns)
    __shared__ double red[kBlock];
    red[threadIdx.x] = best;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(red[0]));
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

struct CoefArgs {
    RawInputs in;
    double a, b;
    OnSite<double> *on64;
    OnSite<float> *on32;
    void *bo64, *bo32;
    int general;
    int only_delta;  // 1: update the pairing entries only
};

// Rescaled coefficients at every site.  Bonds that leave an open lattice get
// zero coefficients so the stencil may apply them to the zero halo.
__global__ void k_coefficients(CoefArgs A)
{
    const RawInputs &in = A.in;
    const int64_t L2 = (int64_t)in.Lx * in.Ly;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < L2;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(s % in.Lx), y = (int)(s / in.Lx);
        double dr, di;
        raw_delta(in, s, dr, di);
        OnSite<double> o;
        if (A.only_delta) {
            o = A.on64[s];
        } else {
            const double xi = in.eps[s] - in.mu_c;
            o.de = (xi - A.b) / A.a;
            o.dh = (-xi - A.b) / A.a;
        }
        o.dr = dr / A.a;
        o.di = di / A.a;
        A.on64[s] = o;
        A.on32[s] = OnSite<float>{(float)o.de, (float)o.dh, (float)o.dr, (float)o.di};
        if (!A.general) continue;
        double t_r[2], t_i[2], d_r[2], d_i[2];
        for (int axis = 0; axis < 2; ++axis) {
            const bool ex = has_fwd_bond(x, y, axis, in);
            const double th = in.peierls ? in.peierls[axis * L2 + s] : 0.0;
            double br, bi;
            raw_bond_delta(in, axis, s, L2, br, bi);
            t_r[axis] = ex ? in.t * cos(th) / A.a : 0.0;
            t_i[axis] = ex ? in.t * sin(th) / A.a : 0.0;
            d_r[axis] = ex ? br / A.a : 0.0;
            d_i[axis] = ex ? bi / A.a : 0.0;
        }
        if (in.cplx) {
            BondsC<double> *p = (BondsC<double> *)A.bo64 + s;
            BondsC<float> *q = (BondsC<float> *)A.bo32 + s;
            BondsC<double> v;
            if (A.only_delta) v = *p;
            else { v.txr = t_r[0]; v.txi = t_i[0]; v.tyr = t_r[1]; v.tyi = t_i[1]; }
            v.dxr = d_r[0]; v.dxi = d_i[0]; v.dyr = d_r[1]; v.dyi = d_i[1];
            *p = v;
            *q = BondsC<float>{(float)v.txr, (float)v.txi, (float)v.dxr, (float)v.dxi,
                               (float)v.tyr, (float)v.tyi, (float)v.dyr, (float)v.dyi};
        } else {
            BondsR<double> *p = (BondsR<double> *)A.bo64 + s;
            BondsR<float> *q = (BondsR<float> *)A.bo32 + s;
            BondsR<double> v;
            if (A.only_delta) v = *p;
            else { v.tx = t_r[0]; v.ty = t_r[1]; }
            v.dx = d_r[0]; v.dy = d_r[1];
            *p = v;
            *q = BondsR<float>{(float)v.tx, (float)v.dx, (float)v.ty, (float)v.dy};
        }
    }
}

static int grid_for(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>(ceil_div(n, kBlock), 1), 4096); }

// Releases the operator and its device arrays; returns the first hipFree
// error (the other arrays are released all the same).
static hipError_t free_op(cbdg_op *op)
{
    if (!op) return hipSuccess;
    hipError_t first = hipSuccess;
    for (void *p : {(void *)op->onsite64, (void *)op->onsite32, op->bonds64, op->bonds32, (void *)op->scratch}) {
        const hipError_t e = hipFree(p);
        if (first == hipSuccess) first = e;
    }
    delete op;
    return first;
}

}  // namespace cbdg

using namespace cbdg;

extern "C" const char *cbdg_last_error(void) { return cbdg::g_err; }

extern "C" int cbdg_build_bdg(const cbdg_lattice *lat, double t, double mu_c,
                              const double *eps, const void *delta, const void *delta_bond,
                              const double *peierls, const cbdg_bounds *fixed,
                              double delta_cap, double eta, void *stream,
                              cbdg_op **op_out, cbdg_bounds *out)
{
    clear_error();
    if (!lat || !op_out) return fail(CBDG_EINVAL, "build_bdg: lat and op must not be NULL");
    *op_out = nullptr;
    if (lat->Lx < 1 || lat->Ly < 1)
        return fail(CBDG_EINVAL, "build_bdg: lattice %d x %d is empty", lat->Lx, lat->Ly);
    if ((int64_t)lat->Lx * lat->Ly > (int64_t)1 << 30)
        return fail(CBDG_EINVAL, "build_bdg: lattice too large");
    if ((lat->bc_x != CBDG_BC_OPEN && lat->bc_x != CBDG_BC_PERIODIC) ||
        (lat->bc_y != CBDG_BC_OPEN && lat->bc_y != CBDG_BC_PERIODIC))
        return fail(CBDG_EINVAL, "build_bdg: boundary condition must be OPEN or PERIODIC");
    if ((lat->bc_x == CBDG_BC_PERIODIC && lat->Lx < 3) || (lat->bc_y == CBDG_BC_PERIODIC && lat->Ly < 3))
        return fail(CBDG_EINVAL, "build_bdg: a periodic direction needs at least 3 sites");
    if (lat->scalar != CBDG_REAL && lat->scalar != CBDG_COMPLEX)
        return fail(CBDG_EINVAL, "build_bdg: scalar must be REAL or COMPLEX");
    if (!eps || !delta) return fail(CBDG_EINVAL, "build_bdg: eps and delta must not be NULL");
    if (peierls && lat->scalar != CBDG_COMPLEX)
        return fail(CBDG_EINVAL, "build_bdg: Peierls phases need a COMPLEX operator");
    if (!std::isfinite(t) || !std::isfinite(mu_c))
        return fail(CBDG_EINVAL, "build_bdg: t and mu_c must be finite");
    if (fixed) {
        if (!(fixed->a > 0.0) || !std::isfinite(fixed->a) || !std::isfinite(fixed->b))
            return fail(CBDG_EINVAL, "build_bdg: fixed bounds need a finite a > 0 and finite b");
    } else {
        if (!(eta > 0.0 && eta < 1.0)) return fail(CBDG_EINVAL, "build_bdg: eta must lie in (0, 1)");
        if (!(delta_cap >= 0.0) || !std::isfinite(delta_cap))
            return fail(CBDG_EINVAL, "build_bdg: delta_cap must be finite and >= 0");
    }

    cbdg_op *op = new (std::nothrow) cbdg_op();
    if (!op) return fail(CBDG_ENOMEM, "build_bdg: host allocation failed");
    hipStream_t st = as_stream(stream);
    op->Lx = lat->Lx; op->Ly = lat->Ly; op->bc_x = lat->bc_x; op->bc_y = lat->bc_y;
    op->scalar = lat->scalar;
    op->bond_pairing = delta_bond != nullptr;
    op->peierls = peierls != nullptr;
    op->general = op->bond_pairing || op->peierls;
    op->t = t; op->mu_c = mu_c;
    op->L2 = (int64_t)lat->Lx * lat->Ly;
    const bool cplx = lat->scalar == CBDG_COMPLEX;
    const size_t L2 = (size_t)op->L2;
    const size_t b64 = cplx ? sizeof(BondsC<double>) : sizeof(BondsR<double>);
    const size_t b32 = cplx ? sizeof(BondsC<float>) : sizeof(BondsR<float>);
    if (hipGetDevice(&op->device) != hipSuccess ||
        hipMalloc(&op->onsite64, L2 * sizeof(OnSite<double>)) != hipSuccess ||
        hipMalloc(&op->onsite32, L2 * sizeof(OnSite<float>)) != hipSuccess ||
        hipMalloc(&op->scratch, 256) != hipSuccess ||
        (op->general && (hipMalloc(&op->bonds64, L2 * b64) != hipSuccess ||
                         hipMalloc(&op->bonds32, L2 * b32) != hipSuccess))) {
        const size_t bytes = L2 * (sizeof(OnSite<double>) + sizeof(OnSite<float>) + (op->general ? b64 + b32 : 0));
        (void)free_op(op);  // already failing: the first error is reported
        (void)hipGetLastError();
        return fail(CBDG_ENOMEM, "build_bdg: device allocation of %zu coefficient bytes failed", bytes);
    }

    RawInputs in{eps, (const double *)delta, (const double *)delta_bond, peierls,
                 lat->Lx, lat->Ly, lat->bc_x, lat->bc_y, cplx ? 1 : 0, t, mu_c};
    cbdg_bounds bd{};
    if (fixed) {
        bd = *fixed;
    } else {
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, st, op->scratch);
        hipLaunchKernelGGL(k_gershgorin, dim3(grid_for(op->L2)), dim3(kBlock), 0, st, in, delta_cap,
                           op->scratch);
        unsigned long long bits = 0;
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(&bits, op->scratch, sizeof(bits), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            (void)free_op(op);  // already failing: the first error is reported
            return fail(CBDG_EHIP, "build_bdg: spectral bound failed: %s", hipGetErrorString(e));
        }
        double R;
        std::memcpy(&R, &bits, sizeof(R));
        if (!std::isfinite(R) || !(R > 0.0)) {
            (void)free_op(op);  // already failing: the first error is reported
            return fail(CBDG_EINVAL, "build_bdg: spectral bound %g is not positive and finite "
                        "(non-finite inputs, or an operator that is identically zero)", R);
        }
        bd.E_min = -R;
        bd.E_max = R;
        bd.a = (bd.E_max - bd.E_min) / (2.0 - eta);
        bd.b = 0.5 * (bd.E_max + bd.E_min);
    }
    op->bounds = bd;
    CoefArgs ca{in, bd.a, bd.b, op->onsite64, op->onsite32, op->bonds64, op->bonds32,
                op->general ? 1 : 0, 0};
    hipLaunchKernelGGL(k_coefficients, dim3(grid_for(op->L2)), dim3(kBlock), 0, st, ca);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        (void)free_op(op);  // already failing: the first error is reported
        return fail(CBDG_EHIP, "build_bdg: coefficient kernel failed: %s", hipGetErrorString(e));
    }
    *op_out = op;
    if (out) *out = bd;
    return CBDG_OK;
}

extern "C" int cbdg_op_update_delta(cbdg_op *op, const void *delta, const void *delta_bond,
                                    void *stream)
{
    clear_error();
    if (!op || !delta) return fail(CBDG_EINVAL, "op_update_delta: op and delta must not be NULL");
    if (delta_bond && !op->bond_pairing)
        return fail(CBDG_EINVAL, "op_update_delta: operator was built without bond pairing");
    // Bond entries are rewritten from delta_bond; without it they stay as built.
    RawInputs in{nullptr, (const double *)delta, (const double *)delta_bond, nullptr,
                 op->Lx, op->Ly, op->bc_x, op->bc_y, op->scalar == CBDG_COMPLEX ? 1 : 0,
                 op->t, op->mu_c};
    CoefArgs ca{in, op->bounds.a, op->bounds.b, op->onsite64, op->onsite32, op->bonds64,
                op->bonds32, (op->general && delta_bond) ? 1 : 0, 1};
    hipLaunchKernelGGL(k_coefficients, dim3(grid_for(op->L2)), dim3(kBlock), 0, as_stream(stream), ca);
    CBDG_CHECK_LAUNCH("k_coefficients");
    return CBDG_OK;
}

extern "C" int cbdg_op_destroy(cbdg_op *op)
{
    clear_error();
    if (!op) return CBDG_OK;
    hipError_t e = hipDeviceSynchronize();
    const hipError_t f = free_op(op);
    if (e == hipSuccess) e = f;
    if (e != hipSuccess) return fail(CBDG_EHIP, "op_destroy: %s", hipGetErrorString(e));
    return CBDG_OK;
}

extern "C" int cbdg_op_bounds(const cbdg_op *op, cbdg_bounds *out)
{
    clear_error();
    if (!op || !out) return fail(CBDG_EINVAL, "op_bounds: op and out must not be NULL");
    *out = op->bounds;
    return CBDG_OK;
}
