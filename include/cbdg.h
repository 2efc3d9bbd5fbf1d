/*
 * cbdg.h -- C ABI of the Chebyshev-BdG hot path on MI355X (gfx950).
 *
 * Method: L. Covaci, F. M. Peeters, M. Berciu, "Chebyshev-BdG: an efficient
 * numerical approach to inhomogeneous superconductivity" (arXiv:1007.1609).
 * The library builds the rescaled Nambu BdG operator of eq. (hamil2), runs
 * the vector recursion of eq. (ref2) from many start vectors |s,e> at once,
 * reads the local moments of eqs. (coeff1)/(coeff2), and turns them into the
 * order parameter (eq. (op1)) and the local density of states (eq. (ldos)).
 * Reverse-mode derivatives of each step are provided.
 *
 * Conventions fixed at this boundary
 *   - Lattice site index s = x + Lx*y (x fastest), 0 <= s < L2 = Lx*Ly.
 *   - Nambu components: e = c^dag_{s,up}|vac> (electron), h = c_{s,down}|vac>
 *     (hole); the start vector of a recursion is |s,e>.
 *   - Moments: mu_ee[k*N + n] = <s,e|T_n(Ht)|s,e> and
 *     mu_he[k*N + n] = <s,h|T_n(Ht)|s,e> for s = start_sites[k],
 *     n = 0..N-1, Ht = (H - b)/a.  They are the paper's a_n^{11}, a_n^{12}
 *     without the 1/(1 + delta_{0n}) factor, so mu_ee[k*N] = 1.
 *   - Complex values are interleaved (re, im) FP64 (complex128) unless
 *     stated.  "scalar" selects real FP64 or complex128 for Delta and mu_he.
 *   - Energies are in units of the hopping t's unit; LDOS is per spin (N_up)
 *     per unit energy.
 *
 * Memory and streams
 *   - Every array argument is a caller-owned, contiguous DEVICE pointer unless
 *     marked "host".  The library never frees or retains a caller pointer
 *     past the call.  The only library-owned object is cbdg_op (coefficient
 *     copies), released with cbdg_op_destroy.
 *   - Workspaces are caller-allocated device memory of at least the size the
 *     matching *_workspace_size call returns.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  All
 *     work is enqueued asynchronously on it; no call synchronises except
 *     cbdg_build_bdg when it computes the spectral bounds (fixed == NULL),
 *     which waits for one scalar.
 *   - Calls that share an operator or workspace on different streams race;
 *     order them on one stream.
 *
 * Errors
 *   Every call returns CBDG_OK (0) or a negative code; cbdg_last_error()
 *   returns a message for the last failure on the calling thread.  Argument
 *   errors are detected on the host before any device work is enqueued.
 *   Values that live on the device (start sites, energies) cannot be checked
 *   on the host: a start site outside [0, L2) yields a row of NaN moments and
 *   an energy outside the expansion interval yields NaN LDOS values, both of
 *   which cbdg_check_moments / the caller can detect.
 */
#ifndef CBDG_H
#define CBDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CBDG_OK            0
#define CBDG_EINVAL       -1  /* bad argument (detected on the host)          */
#define CBDG_ENOMEM       -2  /* device allocation failed                      */
#define CBDG_EHIP         -3  /* a HIP runtime call or kernel launch failed    */
#define CBDG_EBOUNDS      -4  /* spectrum not inside [-1, 1] after rescaling;
                                 device-side check, see cbdg_chebyshev_moments */
#define CBDG_EUNSUPPORTED -5  /* valid request this build does not implement   */

enum cbdg_bc { CBDG_BC_OPEN = 0, CBDG_BC_PERIODIC = 1 };
enum cbdg_scalar { CBDG_REAL = 0, CBDG_COMPLEX = 1 };
enum cbdg_precision { CBDG_FP64 = 0, CBDG_FP32_ACC64 = 1 };
enum cbdg_kernel { CBDG_KERNEL_JACKSON = 0, CBDG_KERNEL_LORENTZ = 1 };
/* How cbdg_chebyshev_moments gets moments 2..N-1 (both give the same moments
 * up to rounding):
 *   DIRECT    N - 1 recursion steps, moment n read off a_n at the start site.
 *   DOUBLING  ceil((N-1)/2) steps: the product rule of Chebyshev polynomials,
 *             2 T_m T_n = T_{m+n} + T_{|m-n|} (the Chebyshev expansion of
 *             section II), with the particle-hole symmetry of the BdG
 *             operator gives mu_ee[2n] = 2<a_n|a_n> - mu_ee[0],
 *             mu_ee[2n-1] = 2 Re<a_n|a_{n-1}> - mu_ee[1],
 *             mu_he[2n-1] = 2 (-1)^n sum_i (u_n(i) v_{n-1}(i) - v_n(i) u_{n-1}(i)) - mu_he[1],
 *             mu_he[2n] = 0, where a = (u, v) on the (e, h) components.
 *             Needs b == 0 (a spectrum centred by the rescaling).
 *   AUTO      DOUBLING when b == 0 and N >= 3, else DIRECT. */
enum cbdg_algorithm { CBDG_ALG_AUTO = 0, CBDG_ALG_DIRECT = 1, CBDG_ALG_DOUBLING = 2 };
/* Energy weight of a moment sum (cbdg_sum_coefficients):
 *   GAP      1 - 2f(E) = tanh(E/2T) on |E| < E_c (E_c <= 0: no cutoff), the
 *            weight of eq. (op1)
 *   DENSITY  f(E) = 1/(exp(E/T) + 1), the weight of the electron density */
enum cbdg_quantity { CBDG_QTY_GAP = 0, CBDG_QTY_DENSITY = 1 };

/* Lattice geometry and number type (host struct).
 * Periodic directions need at least 3 sites. */
typedef struct cbdg_lattice {
    int32_t Lx, Ly;
    int32_t bc_x, bc_y;   /* enum cbdg_bc */
    int32_t scalar;       /* enum cbdg_scalar */
} cbdg_lattice;

/* Spectral interval and rescaling Ht = (H - b)/a (host struct). */
typedef struct cbdg_bounds {
    double E_min, E_max;  /* interval that contains the spectrum of H        */
    double a, b;          /* a = (E_max - E_min)/(2 - eta), b = (E_max+E_min)/2 */
} cbdg_bounds;

/* Kernel damping and energy weighting of the truncated expansion (host).
 *   kernel  CBDG_KERNEL_JACKSON (default) or CBDG_KERNEL_LORENTZ with
 *           parameter lambda (broadening lambda/N in rescaled units)
 *   T       temperature >= 0; sums with T > 0 take coefficients from
 *           cbdg_sum_coefficients
 *   E_c     cutoff energy of the gap equation (<= 0: no cutoff)
 *   a, b    the operator's rescaling (from cbdg_bounds) */
typedef struct cbdg_weights {
    int32_t kernel;
    double lambda;
    double T;
    double E_c;
    double a, b;
} cbdg_weights;

typedef struct cbdg_op cbdg_op;

/* Message of the last failure on the calling thread ("" if none). */
const char *cbdg_last_error(void);

/*
 * Build the rescaled BdG operator of eq. (hamil2):
 *   on-site 2x2 block  [[eps_i - mu_c, Delta_i], [conj(Delta_i), -(eps_i - mu_c)]]
 *   bond 2x2 block     [[-t_ij, Delta_ij], [conj(Delta_ij), conj(t_ij)]]
 * with t_ij = t exp(i theta_ij) on the bond i -> j = i + x^ (or + y^),
 * t_ji = conj(t_ij), Delta_ji = Delta_ij (Peierls phases: the paragraph after
 * eq. (hamil2)), and the rescaling of the paragraph after eq. (rec).
 *
 *   lat          host; geometry and scalar type
 *   t, mu_c      hopping amplitude and chemical potential
 *   eps          [L2] FP64 on-site potential
 *   delta        [L2] on-site Delta_i, FP64 (REAL) or complex128 (COMPLEX)
 *   delta_bond   [2*L2] or NULL: bond Delta for the bond s -> s+x^ (first L2
 *                entries) and s -> s+y^ (next L2), same scalar type as delta;
 *                entries of bonds that leave an open lattice are ignored
 *   peierls      [2*L2] FP64 or NULL: phase theta of the same bonds; needs
 *                lat->scalar == CBDG_COMPLEX
 *   fixed        host or NULL.  NULL: compute the Gershgorin bound R = max
 *                row sum of |H| with every |Delta_i| raised to at least
 *                delta_cap, set E_max = -E_min = R, b = 0,
 *                a = 2R/(2 - eta) (synchronises on one scalar).  Otherwise
 *                use fixed->a and fixed->b as given (a > 0).
 *   delta_cap    >= 0, see fixed (U/2 keeps the bound valid for every
 *                iterate of the gap map)
 *   eta          in (0, 1): safety margin of the rescaling
 *   op           host out: new operator handle (library-owned)
 *   out          host out or NULL: the bounds used
 * The operator keeps FP64 and FP32 copies of the rescaled coefficients;
 * the input arrays are not retained.
 */
int cbdg_build_bdg(const cbdg_lattice *lat, double t, double mu_c,
                   const double *eps, const void *delta, const void *delta_bond,
                   const double *peierls, const cbdg_bounds *fixed,
                   double delta_cap, double eta, void *stream,
                   cbdg_op **op, cbdg_bounds *out);

/* Replace the operator's on-site (and, if delta_bond != NULL and the operator
 * was built with bond pairing, bond) order parameter, keeping a and b frozen:
 * the self-consistency update of the paragraph after the current density.
 * Same layouts as cbdg_build_bdg. */
int cbdg_op_update_delta(cbdg_op *op, const void *delta, const void *delta_bond,
                         void *stream);

/* Release an operator (NULL is a no-op).  Synchronises the device. */
int cbdg_op_destroy(cbdg_op *op);

/* Rescaling (a, b) of an operator (host out). */
int cbdg_op_bounds(const cbdg_op *op, cbdg_bounds *out);

/* Bytes of workspace cbdg_chebyshev_moments needs for tiles of `tile` start
 * vectors at `precision` with `algorithm` (host out): the tile's vector
 * buffers (four for real operators with uniform hopping, whose recursion
 * advances several steps per launch; two otherwise), plus FP64 partial sums
 * for DOUBLING and, where the vector-contiguous passes apply, a packed copy
 * of the coefficients.  EINVAL for DOUBLING when b != 0. */
int cbdg_moments_workspace_size(const cbdg_op *op, int32_t tile, int32_t precision,
                                int32_t algorithm, size_t *bytes);

/*
 * Chebyshev moments of eqs. (coeff1)/(coeff2) through the vector recursion
 * of eq. (ref2):  a_0 = |s,e>,  a_1 = Ht a_0,  a_n = 2 Ht a_{n-1} - a_{n-2},
 * mu_ee[k][n] = <s,e|a_n>,  mu_he[k][n] = <s,h|a_n>.
 * The start vectors are processed in tiles of `tile` vectors; all tiles run
 * inside this call.  Real operators with uniform hopping under DOUBLING on
 * lattices with Lx = 64 W (FP64: W = 1, 2, 4; FP32_ACC64: W = 2, 4) store a
 * tile vector by vector and fuse seven recursion steps per launch, each
 * vector clipped to its own light cone; the site values and doubling sums
 * agree with those of the other passes to rounding.
 *   start_sites  [n_start] int32 lattice sites (duplicates allowed)
 *   n_start      >= 0 (0: nothing is done)
 *   N            number of moments, >= 1
 *   tile         start vectors per tile, >= 1
 *   precision    CBDG_FP64, or CBDG_FP32_ACC64: recursion vectors and
 *                coefficients in FP32 (complex64 for COMPLEX), moments
 *                widened exactly to FP64 (doubling sums in FP64)
 *   algorithm    enum cbdg_algorithm; DOUBLING with b != 0 is EINVAL
 *   workspace    >= cbdg_moments_workspace_size(op, tile, precision,
 *                algorithm) bytes
 *   mu_ee        out [n_start*N] FP64
 *   mu_he        out [n_start*N] FP64 (REAL) or complex128 (COMPLEX)
 * Spectral bound (CBDG_EBOUNDS): with the spectrum of Ht inside [-1, 1] every
 * moment satisfies |mu| <= 1.  The check runs on the device, after each tile,
 * so that the call stays asynchronous: a moment with |mu| > 1 + tol or not
 * finite (tol 1e-9 for FP64, 1e-4 for FP32_ACC64 vectors) is stored as NaN.
 * The call itself cannot return CBDG_EBOUNDS; the NaN reaches the residual of
 * cbdg_gap_update (NaN), the LDOS and cbdg_check_moments, and the host loop
 * that reads the residual reports CBDG_EBOUNDS.
 */
int cbdg_chebyshev_moments(const cbdg_op *op, const int32_t *start_sites, int64_t n_start,
                           int32_t N, int32_t tile, int32_t precision, int32_t algorithm,
                           void *workspace, size_t workspace_bytes,
                           double *mu_ee, void *mu_he, void *stream);

/* Bytes of workspace cbdg_chebyshev_moments_resident needs for tiles of
 * `tile` vectors (host out): the tile's two vector buffers, the FP64 partial
 * sums of 16 recursion steps and two control words.  EINVAL / EUNSUPPORTED
 * as cbdg_chebyshev_moments_resident. */
int cbdg_resident_workspace_size(const cbdg_op *op, int32_t tile, int32_t precision, size_t *bytes);

/*
 * The moments of cbdg_chebyshev_moments by moment doubling, with every
 * recursion step of a tile in one persistent (cooperative) launch, for tiles
 * whose two vector buffers -- 2 * L2 * round_up(tile, 64) Nambu pairs, 16 B
 * (FP64) or 8 B (FP32_ACC64) each -- fit in 200 MiB, so that they stay in the
 * 256 MB Infinity Cache of the GPU: eq. (ref2) with the moments of eqs.
 * (coeff1)/(coeff2), as the paper's closing remarks note the method needs
 * only sparse matrix-vector products and little memory.  Steps are separated
 * by a grid barrier with a bounded wait.
 *   start_sites, n_start, N, precision, mu_ee, mu_he  as cbdg_chebyshev_moments
 *   tile        1 .. 256 vectors per tile
 *   spin_limit  polls of a grid barrier before the launch gives up (0: a
 *               default of about a second); a barrier that gives up makes
 *               every workgroup leave the kernel, and the call returns
 *               CBDG_EHIP with the moments of that tile incomplete
 *   workspace   >= cbdg_resident_workspace_size(op, min(tile, n_start),
 *               precision) bytes
 * Real operators with uniform hopping and on-site pairing only
 * (EUNSUPPORTED otherwise); b must be 0 (EINVAL otherwise); EINVAL when the
 * tile's vectors exceed 200 MiB.  The moments agree with
 * cbdg_chebyshev_moments to rounding (the dot products are summed over other
 * regions), with the same device-side bound check.  The call synchronises the
 * stream once per tile to read the barrier's flag.
 */
int cbdg_chebyshev_moments_resident(const cbdg_op *op, const int32_t *start_sites, int64_t n_start,
                                    int32_t N, int32_t tile, int32_t precision, int64_t spin_limit,
                                    void *workspace, size_t workspace_bytes, double *mu_ee, void *mu_he,
                                    void *stream);

/* Size of the per-GPU device array cbdg_chebyshev_moments_static works in. */
#define CBDG_STATIC_SCRATCH_BYTES (64u << 20)

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * cbdg_chebyshev_moments with its workspace taken from a library-owned device
 * array of CBDG_STATIC_SCRATCH_BYTES (64 MiB) instead of a caller argument.
 * The call allocates and frees nothing.  The array is a file-scope device
 * variable of the library: each GPU the library runs on holds its own copy
 * until the process ends.
 *   arguments   as cbdg_chebyshev_moments, without the workspace
 *   errors      EINVAL when cbdg_moments_workspace_size(op, min(tile, n_start),
 *               precision, algorithm) exceeds CBDG_STATIC_SCRATCH_BYTES (use
 *               smaller tiles), or when the current device is not the one the
 *               operator was built on
 * Every call on one GPU shares that GPU's array and leaves its contents
 * there; the call writes everything it reads from the array before reading
 * it.  Calls that overlap on one GPU (several streams or host threads) race
 * on the array: order them on one stream.  Results are bitwise those of
 * cbdg_chebyshev_moments with the same tile.
 */
int cbdg_chebyshev_moments_static(const cbdg_op *op, const int32_t *start_sites, int64_t n_start,
                                  int32_t N, int32_t tile, int32_t precision, int32_t algorithm,
                                  double *mu_ee, void *mu_he, void *stream);

/* CBDG_STATIC_SCRATCH_BYTES as built into the library. */
size_t cbdg_static_scratch_bytes(void);

/*
 * The moments of cbdg_chebyshev_moments (direct algorithm) and, from the same
 * vectors, the off-diagonal moments between each start site and its four
 * lattice neighbours j (the moments of the paragraph after eq. (ref2) with a
 * bra on another grid point):
 *   nb_ee[k][d][n] = <j,e|a_n>,  nb_he[k][d][n] = <j,h|a_n>,
 *   d = 0..3 for j = s + x, s - x, s + y, s - y (wrapping on periodic
 *   directions; a neighbour outside an open lattice gives a zero row).
 * They feed cbdg_bond_gap_update and cbdg_bond_current.
 *   nb_ee, nb_he  out [n_start*4*N] FP64 (REAL) or complex128 (COMPLEX)
 *   workspace     >= cbdg_moments_workspace_size(op, tile, precision,
 *                 CBDG_ALG_DIRECT) bytes
 * Other arguments, NaN rows for invalid sites and the device-side bound check
 * (applied to the neighbour moments too) as cbdg_chebyshev_moments.
 */
int cbdg_chebyshev_moments_nb(const cbdg_op *op, const int32_t *start_sites, int64_t n_start,
                              int32_t N, int32_t tile, int32_t precision, void *workspace,
                              size_t workspace_bytes, double *mu_ee, void *mu_he, void *nb_ee,
                              void *nb_he, void *stream);

/* Bounds check of moments: |mu| <= 1 holds for every moment when the
 * spectrum of Ht lies in [-1, 1].  Writes 1 to *flag if any |mu_ee| or
 * |mu_he| exceeds 1 + tol or is not finite, else 0.
 *   flag  out, one int32 on the device */
int cbdg_check_moments(const double *mu_ee, const void *mu_he, int64_t n_rows, int32_t N,
                       int32_t scalar, double tol, int32_t *flag, void *stream);

/*
 * Chebyshev coefficients of a weight of the moment sums, damped by the
 * kernel: coeff[n] = g_n c_n with w(a x + b) = sum_n c_n T_n(x) and
 *   CBDG_QTY_GAP      w(E) = 1 - 2f(E) = tanh(E/2T) on |E| < E_c (eq. (op1))
 *   CBDG_QTY_DENSITY  w(E) = f(E) (the electron-density equation)
 * at the weights' temperature T >= 0 (T = 0: sign(E) and theta(-E)).
 * c_n = ((2 - delta_n0)/pi) int_0^pi w(a cos t + b) cos(n t) dt: closed form
 * where |E| > 40 T, Gauss-Legendre panels (width <= min(1/(2N), T/(4a))) in
 * between.  coeff: out [N] FP64 on the device.  EINVAL when E = 0 is outside
 * [b - a, b + a] or T is too small for the panels (use T = 0).
 */
int cbdg_sum_coefficients(const cbdg_weights *w, int32_t N, int32_t quantity, double *coeff,
                          void *stream);

/*
 * One step of the gap equation, eq. (op1), from the anomalous moments:
 *   Delta_new[r] = (U_r/2) conj( sum_n g_n c_n mu_he[r][n] )
 * where g_n is the kernel and c_n are the Chebyshev coefficients of the
 * weight (1 - 2f(E)) on |E| < E_c; then plain mixing
 *   delta_out[r] = (1 - alpha) delta_in[r] + alpha Delta_new[r]
 * and the residual *resid = max_r |Delta_new[r] - delta_in[r]|.
 *   coeff      [N] g_n c_n from cbdg_sum_coefficients(CBDG_QTY_GAP), or NULL
 *              for the built-in T = 0 weight sign(E) (EINVAL when T > 0)
 *   mu_he      [n_rows*N] FP64 (REAL) or complex128 (COMPLEX)
 *   U, U_rows  coupling: U_rows ([n_rows] FP64) if not NULL, else U
 *   delta_in   [n_rows], delta_out [n_rows] (may alias delta_in)
 *   resid      out, one FP64 on the device (NaN if any Delta_new is NaN)
 */
int cbdg_gap_update(const void *mu_he, int64_t n_rows, int32_t N, int32_t scalar,
                    const cbdg_weights *w, const double *coeff, double U, const double *U_rows,
                    const void *delta_in, double alpha, void *delta_out,
                    double *resid, void *stream);

/*
 * Electron density of the electron-density equation with the spin-down LDOS
 * equal to the spin-up one (singlet pairing):
 *   density[r] = 2 sum_n g_n c_n mu_ee[r][n],  c_n the coefficients of f(E)
 *   coeff    [N] from cbdg_sum_coefficients(CBDG_QTY_DENSITY), or NULL for
 *            the built-in T = 0 weight theta(-E) (EINVAL when T > 0)
 *   density  out [n_rows] FP64
 */
int cbdg_density(const double *mu_ee, int64_t n_rows, int32_t N, const cbdg_weights *w,
                 const double *coeff, double *density, void *stream);

/* Transpose of cbdg_density: d_mu_ee[r][n] = 2 g_n c_n d_density[r]
 * (overwritten). */
int cbdg_density_backward(const double *d_density, int64_t n_rows, int32_t N,
                          const cbdg_weights *w, const double *coeff, double *d_mu_ee,
                          void *stream);

/*
 * Local density of states per spin, eq. (ldos) with eq. (imag2):
 *   ldos[r][m] = [g_0 mu_ee[r][0] + 2 sum_{n>=1} g_n mu_ee[r][n] T_n(x_m)]
 *                / (pi a sqrt(1 - x_m^2)),   x_m = (energies[m] - b)/a
 *   mu_ee     [n_rows*N] FP64
 *   energies  [n_E] FP64; |x_m| >= 1 gives NaN
 *   ldos      out [n_rows*n_E] FP64
 */
int cbdg_ldos(const double *mu_ee, int64_t n_rows, int32_t N, const cbdg_weights *w,
              const double *energies, int32_t n_E, double *ldos, void *stream);

/*
 * Bond order parameter of eq. (op1) for i != j (singlet, symmetrised), from
 * the neighbour moments of every site (rows = sites 0..Lx*Ly-1 in order):
 *   Delta_new(s, s+e) = (U/4) [conj(sum_n g_n c_n nb_he[s][+e][n])
 *                            + conj(sum_n g_n c_n nb_he[s+e][-e][n])],
 * e = x (axis 0) or y (axis 1), then plain mixing and the residual as in
 * cbdg_gap_update.  Bonds leaving an open lattice get Delta_new = 0.
 *   nb_he           [Lx*Ly*4*N] from cbdg_chebyshev_moments_nb
 *   coeff           as for cbdg_gap_update (NULL: T = 0)
 *   delta_bond_in   [2*Lx*Ly] (axis-major, the layout of cbdg_build_bdg),
 *   delta_bond_out  [2*Lx*Ly] (may alias delta_bond_in); FP64 or complex128
 */
int cbdg_bond_gap_update(const void *nb_he, int32_t Lx, int32_t Ly, int32_t bc_x, int32_t bc_y,
                         int32_t N, int32_t scalar, const cbdg_weights *w, const double *coeff,
                         double U, const void *delta_bond_in, double alpha, void *delta_bond_out,
                         double *resid, void *stream);

/*
 * Particle current along every bond, both spins (the current-density
 * equation, read as the continuity current of the hopping -t_ij c_i^+ c_j of
 * eq. (hamil2)):  J(s -> s+e) = 4 Im( t_{s,s+e} <c_s^+ c_{s+e}> ),
 *   <c_s^+ c_{s+e}> = sum_n g_n c_n nb_ee[s][+e][n],  c_n of f(E),
 * t the operator's unscaled hopping (with its Peierls phase).
 *   nb_ee    [L2*4*N] from cbdg_chebyshev_moments_nb (rows = all sites)
 *   coeff    [N] from cbdg_sum_coefficients(CBDG_QTY_DENSITY) (required)
 *   current  out [2*L2] FP64, axis-major; 0 for bonds leaving an open lattice
 */
int cbdg_bond_current(const cbdg_op *op, const void *nb_ee, int32_t N, const cbdg_weights *w,
                      const double *coeff, double *current, void *stream);

/* Transpose of cbdg_gap_update for a REAL operator:
 *   d_mu_he[r][n] = alpha (U_r/2) g_n c_n d_delta_out[r]
 *   d_delta_in[r] = (1 - alpha) d_delta_out[r]        (if d_delta_in != NULL)
 * coeff as for cbdg_gap_update.  Outputs are overwritten. */
int cbdg_gap_update_backward(const double *d_delta_out, int64_t n_rows, int32_t N,
                             const cbdg_weights *w, const double *coeff, double U,
                             const double *U_rows, double alpha, double *d_mu_he,
                             double *d_delta_in, void *stream);

/* Transpose of cbdg_ldos:  d_mu_ee[r][n] = sum_m d_ldos[r][m] W[m][n]
 * (overwritten). */
int cbdg_ldos_backward(const double *d_ldos, int64_t n_rows, int32_t N,
                       const cbdg_weights *w, const double *energies, int32_t n_E,
                       double *d_mu_ee, void *stream);

/* Bytes of workspace cbdg_chebyshev_moments_backward needs (host out).
 * ckpt_stride 0 selects k = ceil(sqrt(N)) (direct) or ceil(sqrt(N/2 + 1))
 * (doubling), rounded up to a multiple of 3; -1 the reverse passes without
 * checkpoints (a moments workspace of one tile, four cotangent buffers and
 * per-vector gradient terms of one tile; EUNSUPPORTED where they do not
 * apply). */
int cbdg_backward_workspace_size(const cbdg_op *op, int32_t tile, int32_t N,
                                 int32_t ckpt_stride, int32_t algorithm, size_t *bytes);

/*
 * Reverse-mode derivative of the moments for a REAL FP64 operator with
 * (a, b) held fixed.  For L = sum_k sum_n (dmu_ee[k][n] mu_ee[k][n] +
 * dmu_he[k][n] mu_he[k][n]) it ADDS dL/deps_j to grad_eps[j] and dL/dDelta_j
 * to grad_delta[j] (on-site, real).  Per tile: a forward pass stores the
 * vector pairs (a_{jk}, a_{jk+1}) every k = ckpt_stride steps; segments are
 * then recomputed in reverse and the transposed recursion
 *   lam_n = w_n + 2 Ht^T lam_{n+1} - lam_{n+2}
 * runs over them, accumulating sum_{n>=1} c_n <lam_n, dHt/dtheta a_{n-1}>
 * (c_1 = 1, c_n = 2).  The sum over start vectors is reduced in a fixed
 * order, so repeated calls give identical bits, whatever the stride.
 *   ckpt_stride  k; 0: ceil(sqrt(N)) (DIRECT) or ceil(sqrt(N/2 + 1)) (DOUBLING),
 *                rounded up to a multiple of 3 (the forward then advances
 *                three steps per launch on tiles of more than 128 vectors).
 *                -1: no checkpoints (DOUBLING on lattices with Lx = 64 W,
 *                W = 1, 2, 4, else EUNSUPPORTED): the forward moments keep
 *                only (a_{M+1}, a_M) and the reverse passes regenerate
 *                a_{m-1} = 2 Ht a_m - a_{m+1} beside the transposed
 *                recursion, several levels per launch in the
 *                vector-contiguous layout; the gradient agrees with the
 *                checkpointed one to rounding (the regenerated vectors differ
 *                from the forward ones by a few units in the last place).
 *   algorithm    enum cbdg_algorithm.  DOUBLING (AUTO when b == 0, N >= 3)
 *                differentiates the doubling formulas instead: forward and
 *                adjoint run over a_0 .. a_{N/2} only, the cotangent of a_m
 *                being a whole vector built from a_{m-1}, a_m, a_{m+1}; the
 *                gradient is the same up to rounding.  DOUBLING with b != 0
 *                is EINVAL.
 *   dmu_ee, dmu_he  [n_start*N] FP64 (either may be NULL: zero)
 *   grad_eps, grad_delta  [L2] FP64, accumulated into (caller zeroes)
 * COMPLEX operators, bond pairing or Peierls phases return EUNSUPPORTED.
 */
int cbdg_chebyshev_moments_backward(const cbdg_op *op, const int32_t *start_sites,
                                    int64_t n_start, int32_t N, int32_t tile,
                                    int32_t ckpt_stride, int32_t algorithm,
                                    const double *dmu_ee, const double *dmu_he, void *workspace,
                                    size_t workspace_bytes, double *grad_eps,
                                    double *grad_delta, void *stream);

/*
 * The derivative of the same L one start vector at a time: row k holds the
 * gradient of L_k = sum_n (dmu_ee[k][n] mu_ee[k][n] + dmu_he[k][n]
 * mu_he[k][n]) with respect to eps_j and Delta_j (the terms that
 * cbdg_chebyshev_moments_backward sums over k).  With dmu_he[k][n] the
 * derivative of the gap update of site k by its own moments
 * (cbdg_gap_update_backward with d_delta_out = 1), row k is row k of the
 * Jacobian dDelta_new/dDelta of the self-consistency map (the gap equation
 * after eq. (op1) with the moments of eq. (ref2)): one reverse sweep gives
 * the whole matrix.  It runs the reverse passes without checkpoints, so it
 * needs what they need (REAL operator with uniform hopping, b = 0, N >= 3,
 * Lx = 64 W with W = 1, 2, 4; else EUNSUPPORTED) and the workspace of
 * cbdg_backward_workspace_size(op, tile, N, -1, ...).
 *   dmu_ee, dmu_he  [n_start*N] FP64 (either may be NULL: zero; not both)
 *   jac_eps, jac_delta  out [n_start][ld] FP64, ld >= Lx*Ly (either may be
 *                NULL); columns Lx*Ly .. ld-1 are not written.  Rows of
 *                invalid start sites are zero.  Overwritten, not added to.
 * The rows agree with one backward call per start vector to rounding.
 */
int cbdg_chebyshev_moments_jacobian(const cbdg_op *op, const int32_t *start_sites, int64_t n_start,
                                    int32_t N, int32_t tile, const double *dmu_ee, const double *dmu_he,
                                    void *workspace, size_t workspace_bytes, double *jac_eps,
                                    double *jac_delta, int64_t ld, void *stream);

/*
 * y = A x for a dense row-major FP64 matrix on the device (the Jacobian of
 * cbdg_chebyshev_moments_jacobian applied to a Newton direction): one
 * wavefront per row, summed in a fixed order, so repeated calls give the
 * same bits.
 *   A  [rows][ld], ld >= cols;  x  [cols];  y  out [rows] (must not alias x)
 */
int cbdg_jacobian_matvec(const double *A, int64_t rows, int64_t cols, int64_t ld, const double *x,
                         double *y, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CBDG_H */
