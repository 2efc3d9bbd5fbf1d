// Internal interface of the recursion step, shared by the forward moments
// and the checkpointed adjoint.
#pragma once

#include "stencil.hpp"

#ifndef CBDG_LANE_PAD
#define CBDG_LANE_PAD 0
#endif

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
    int ys;              // rows per segment
    double *part;        // moment-doubling partials [regions][K][Bp], or null
    const int32_t *cone; // {x_min, x_max, y_min, y_max} of the tile's valid start
                         // sites, or null: steps n >= 2 skip strips and rows
                         // farther than n from that box (a_n is zero there)
    void *out2;          // two-step pass: a_{n+1}
    double *part_b;      // two-step pass: doubling partials of step n+1
    double *part_c;      // three-step pass: doubling partials of step n+2
    double *nb_ee;       // neighbour moments [Bt][4][N] (+x, -x, +y, -y; complex
    double *nb_he;       //   interleaved for C), tile's first row, or null
};

// Lane stride of a tile of B vectors: B rounded up to the wavefront, plus
// the stride padding.
inline int64_t lane_stride(int64_t B) { return round_up(B, kWave) + CBDG_LANE_PAD; }

// One recursion step (A.first: a_1 = Ht a_0) on the stream; A.onsite/A.bonds
// are filled from the operator.  prev1 must not alias out; prev2 may.
// mu_ee == nullptr skips the moment extraction.
int run_step(const cbdg_op *op, int precision, StepArgs A, hipStream_t st);

// Two recursion steps in one launch (FP64, real operator with uniform
// hopping): a_n -> A.out and a_{n+1} -> A.out2 from a_{n-2} (A.prev2) and
// a_{n-1} (A.prev1), n >= 2.  Neither output may alias an input or the other
// output: a lane reads its neighbours' a_{n-1} and a_{n-2} while they write.
bool two_step_f64_real(const cbdg_op *op);
int run_step2_f64_real(const cbdg_op *op, StepArgs A, hipStream_t st);

// Three recursion steps in one launch (same operators, tiles of Bt vectors
// the library runs three-step passes for): a_{n+1} -> A.out and
// a_{n+2} -> A.out2 from a_{n-2} and a_{n-1}, n >= 2; a_n is not stored.
// The same aliasing rules as the two-step pass.
bool three_step_f64_real(const cbdg_op *op, int Bt);
int run_step3_f64_real(const cbdg_op *op, StepArgs A, hipStream_t st);

// Device-side bound check of n moment entries (ee_c / he_c: complex128
// entries): a magnitude beyond lim or a non-finite value becomes NaN.
int bound_moments(double *ee, double *he, int64_t n, bool ee_c, bool he_c, double lim, hipStream_t st);
// Its limit: 1 plus the rounding allowance of FP64 or FP32 recursion vectors.
double moment_limit(bool f32);

// Most steps one pass of any kind takes (partials and run sums are sized for it).
constexpr int kMaxPassSteps = 8;

// Passes over a tile stored vector-contiguous (vector b in the pairs
// b*Dv .. b*Dv + L2 - 1, row after row, column x = lW + k of a row at k*64 + l
// for W = Lx/64; real operators with uniform hopping, moment doubling): one
// wavefront per vector and row segment, each vector clipped to its own light
// cone.  A pass of `steps` = 1 writes a_n (A.out, may alias A.a2; n = 1: a_1 =
// Ht a_0 and moment 1) and the partials of step n; `steps` = K = 2 ..
// vc_steps() writes a_{n+K-2} (A.out) and a_{n+K-1} (A.out2) from a_{n-2}
// (A.a2) and a_{n-1} (A.a1) and the partials of steps n .. n+K-1
// ([n_segs][3][Bp] each), or with n_segs = 1 the moments 2m-1 and 2m of
// those steps m themselves.  The passes read only what the tile's earlier
// passes (and the seed) wrote: the buffers need no clearing.
struct VcArgs {
    const void *a1, *a2;
    void *out, *out2;
    const void *coef;    // packed (de, Delta/a) per site, in the passes' row layout
    double th;           // t/a
    int Lx, Ly, bcx, bcy;
    int64_t Dv;          // pairs per vector
    int Bt, Bp;          // vectors; lane stride of the partials
    int n, N;
    int n_segs, nblocks;
    int nlev;            // steps of a shorter last pass (set by launch_vc)
    const int32_t *sites;
    double *part;        // partials of step n + j at part + j * pstride
    int64_t pstride;
    double *mu_ee, *mu_he;  // first step: moment 1 of each row
};
// Lanes per row: a vector-contiguous pass needs Lx = 64 W with W in the
// instantiated set; 0 when the lattice does not fit.
int vc_width(int Lx, bool f32);
// Row segments per vector of a pass over a tile of Bt vectors.
int vc_segments(int Ly, int Bt, int steps);
int launch_vc(const VcArgs &A, int steps, bool f32, hipStream_t st);
// Steps of a full multi-step vector-contiguous pass (3 .. kMaxPassSteps).
int vc_steps(bool f32);
// Reverse passes of the doubling adjoint that regenerate the forward vectors
// backwards (a_{m-1} = 2 Ht a_m - a_{m+1}) instead of reading checkpoints,
// in the vector-contiguous layout (FP64; the operators and lattices of the
// forward passes).  A pass of nlev levels takes m = m0 .. m0-nlev+1:
//   inputs   b0 = a_{m0+1}, b1 = a_{m0} (inside their light cones),
//            c0 = lam_{m0+2}, c1 = lam_{m0+1} (zero when first),
//   outputs  (full passes only) bo1 = a_{m0-K+1}, bo2 = a_{m0-K},
//            co1 = lam_{m0-K+2}, co2 = lam_{m0-K+1},
//   G        per vector and site, the terms c_m (lam_m . dHt/deps a_{m-1},
//            lam_m . dHt/dDelta a_{m-1}) * a of the gradient, added to what
//            G holds (G starts at zero when first).
// Outputs must not alias inputs.
struct VcAdjArgs {
    const void *b0, *b1, *c0, *c1;
    void *bo1, *bo2, *co1, *co2;
    double *G;
    const void *coef;    // the passes' packed coefficients
    double th;           // t/a
    int Lx, Ly, bcx, bcy;
    int64_t Dv;
    int Bt, n_segs, nblocks;
    int m0, nlev, N, first;
    const int32_t *sites;
    const double *dmu_ee, *dmu_he;  // tile rows (either may be null)
    const double *d1;               // [Bt][2] start-site cotangents at m = 1
};
// Levels of a full reverse pass on lattices of width Lx (0: unsupported).
int vc_adj_steps(int Lx);
int launch_vc_adj(VcAdjArgs A, bool full, hipStream_t st);
// grad_eps[j] += scale * sum_b G_b(j).e, grad_delta[j] += scale * sum_b G_b(j).h
// over the vectors of valid start sites (summed in order)
int launch_vc_grad_reduce(const double *G, const int32_t *sites, int Bt, int64_t Dv, int Lx, int64_t L2, double scale,
                          double *grad_eps, double *grad_delta, hipStream_t st);
// the same terms one row per vector: row_eps[b * ld + j] = scale * G_b(j).e,
// row_delta[b * ld + j] = scale * G_b(j).h (zero rows for invalid start
// sites; either output may be null)
int launch_vc_grad_rows(const double *G, const int32_t *sites, int Bt, int64_t Dv, int Lx, int64_t L2, double scale,
                        double *row_eps, double *row_delta, int64_t ld, hipStream_t st);
// The forward moments of one tile in the vector-contiguous passes, then one
// more step: a_{M+1} and a_M (M = N/2) are left in two of the four tile
// buffers of the moments workspace ws, whose addresses come back in last[0]
// and last[1]; the other two go to spare[0], spare[1], and the packed
// coefficients the passes read to coef.
int vc_forward_last(const cbdg_op *op, const int32_t *sites, int Bt, int N, void *ws, double *mu_ee, double *mu_he,
                    hipStream_t st, void **last, void **spare, const void **coef);
bool vc_adjoint_supported(const cbdg_op *op);

// a_0 (its whole start row) and the zeroth moments of a tile
int launch_vc_seed(void *a0, int64_t Dv, int Lx, bool f32, int Bt, int64_t L2, const int32_t *sites, double *mu_ee,
                   double *mu_he, int N, hipStream_t st);
// the packed coefficients (L2 pairs of the recursion's type) from the operator's
int launch_vc_coef(const void *onsite, void *coef, int Lx, bool f32, int64_t L2, hipStream_t st);

// a_0 = |s_b,e> for the tile's vectors (FP64 real layout); writes mu_0 when
// mu_ee is not null.
int seed_tile_f64_real(void *a0, int64_t L2, int Bt, const int32_t *sites, double *mu_ee, double *mu_he, int N,
                       hipStream_t st);

}  // namespace cbdg
