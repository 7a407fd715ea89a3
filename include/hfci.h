/*
 * hfci.h -- C ABI of libhfci, an MI355X (gfx950) solver for the 3D Helmholtz
 * equation by contour integration and polynomial preconditioning
 * (Liu, Xi, Saad, de Hoop, arXiv 1811.12378).
 *
 * Problem (Sec. 1.1, eq. helmholtz-op / eq. lin-sys):
 *     (-Laplace_h - omega^2 / c(x)^2) u = f
 * on an nx*ny*nz grid of interior nodes with spacing h, homogeneous Dirichlet
 * ghosts, 7-point second-order differences.
 *
 * Internally the operator is normalised as in Sec. 7.1 (eq. stiff-mass):
 *     A = S - M - i D,   S = (s/h^2) * (7-point stencil),  s = c_min^2/omega^2,
 *     M = diag(kappa), kappa_i = c_min^2 / c_i^2 <= 1,
 *     D = diag(rho2 * (d_i/L)^2)  (absorbing layer of L cells, d_i = depth into it),
 * so the physical system is A u = s f.  The damping carries a minus sign so that
 * A = A1 - i A2 with A2 >= 0 as Lemma 3.1 requires.
 *
 * Memory / layout conventions (all entry points):
 *   * Grid vectors are caller-owned DEVICE buffers, x fastest then y then z:
 *     element (x, y, z) at index x + nx*(y + ny*z).  Complex values are
 *     interleaved (re, im): complex128 (hfci_c128) or complex64 (two floats),
 *     identical to torch.complex128 / torch.complex64 storage.
 *   * Batches of vectors are contiguous: vector k starts at k*n elements,
 *     n = nx*ny*nz.
 *   * Handles are library-owned and released by the matching *_destroy.
 *     Operators and contours may be destroyed before or after their context,
 *     but no call other than *_destroy may use them once the context is gone.
 *   * All device work is issued on the context's stream.  Every entry point
 *     returns after its work has completed on that stream (it synchronises).
 *   * On a negative status the outputs are unspecified and hfci_last_error()
 *     holds a message (thread-local).  HFCI_W_NOCONV (> 0) still writes the
 *     best iterate.
 */
#ifndef HFCI_H
#define HFCI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } hfci_c128;

typedef enum {
  HFCI_OK = 0,
  HFCI_W_NOCONV = 1,      /* iteration cap reached before the tolerance    */
  HFCI_E_ARG = -1,        /* invalid argument (sizes, null pointers, enum) */
  HFCI_E_HIP = -2,        /* HIP runtime error (message has the HIP text)  */
  HFCI_E_OOM = -3,        /* device allocation failed                      */
  HFCI_E_CONTOUR = -4,    /* contour violates Sec. 6.2's invariants, or the
                             delta search found no contraction (nu >= 1)   */
  HFCI_E_NUMERIC = -5,    /* NaN/Inf met in a reduction                    */
  HFCI_E_STATE = -6       /* handle mismatch (e.g. contour of another op)  */
} hfci_status;

enum { HFCI_F32 = 32, HFCI_F64 = 64 };
enum { HFCI_PRECOND_NONE = 0, HFCI_PRECOND_FCI = 1, HFCI_PRECOND_LEARNED = 2 };

typedef struct hfci_ctx hfci_ctx;
typedef struct hfci_op hfci_op;
typedef struct hfci_contour hfci_contour;
typedef struct hfci_net hfci_net;

/* Options of the FCI preconditioner and the FGMRES wrapper (Sec. 2, Alg. 1). */
typedef struct {
  size_t size;          /* = sizeof(hfci_solve_opts); set by hfci_default_opts   */
  int precision;        /* HFCI_F64 or HFCI_F32: arithmetic of the shifted-system
                           sweeps and the quadrature combine.  The Arnoldi
                           process, Givens least squares and true residuals are
                           always FP64.                         default HFCI_F64 */
  int restart;          /* m of FGMRES(m), 1..64                    default 30  */
  int max_it;           /* cap on FGMRES iterations (all cycles)    default 500 */
  double tol;           /* target ||f - A u|| / ||f|| (2-norm)      default 1e-6 */
  int fp_steps;         /* > 0: exactly this many fixed-point steps per pole
                           (lockstep mode); 0: adaptive stopping     default 0  */
  double fp_reduce;     /* adaptive: stop a pole when ||r|| <= ||f|| / fp_reduce
                           (Table 4 uses 5)                          default 5  */
  int fp_max_steps;     /* adaptive: cap on steps per pole           default 200 */
  int k_in;             /* Alg. 1 step 4: GMRES steps (0..16) on the remainder
                           f - d A w, right-preconditioned by the regularised
                           inverse of the discrete Laplacian, V diag(1/max(lambda,
                           1)) V^T with V the sine transform along each axis
                           (Sec. 6.3); FP64.  Not for case-two operators or
                           batches.                                   default 0 */
  int precond;          /* HFCI_PRECOND_FCI (default) or HFCI_PRECOND_NONE       */
  int pole_batch;       /* poles advanced together per launch (x every RHS);
                           0 = all J                                              */
  int verbose;          /* 1: one line per FGMRES cycle on stderr               */
  /* learned preconditioner (precond = HFCI_PRECOND_LEARNED): the proposal z = net(v_j)
     is scaled by the complex d minimising rho = ||v_j - d A z|| / ||v_j|| (Alg. 1 step 3)
     and kept when rho <= learned_tau * (mean rho of FCI over this solve's FCI steps)
     and rho < 0.99; otherwise, and until FCI has run once, z_j = FCI(v_j) (needs the
     contour).  0 < learned_tau <= 4.                               default 1.0 */
  hfci_net* net;
  double learned_tau;
  int learned_patience;  /* after this many consecutive rejected proposals the network
                            is no longer consulted in this solve (0 = never stop)
                                                                     default 8 */
  /* training-pair harvest: each Arnoldi step of each RHS appends (v_j, FCI(v_j)) as
     complex64 to the DEVICE arrays harvest_v / harvest_z (harvest_cap vectors of n). */
  int harvest_cap;
  void* harvest_v;
  void* harvest_z;
  int graphs;           /* fixed-point steps of the FCI: 1 = each step (its remaining
                           factors, the next step's first factor, the stopping test and
                           the read-back of the flags) replayed from a captured HIP graph,
                           one graph launch per step, every launch sized for all systems
                           (stopped ones exit at once); 0 = direct launches sized for the
                           systems still iterating; -1 = graphs when the grid has at most
                           2^16 points                                     default 0 */
  int inner_precond;    /* the right preconditioner of Alg. 1 step 4 (k_in > 0): 0 = the
                           regularised Laplacian inverse above, 1 = the learned network
                           opts->net, the inner steps then being flexible GMRES steps
                           with z_j = net(v_j) on the remainder: with k_in = 1 the result
                           is out + beta net(r), r = f - A out, beta minimising the new
                           remainder, so the network can only lower ||f - A out|| and FCI
                           stays the preconditioner.  1 needs opts->net.     default 0 */
} hfci_solve_opts;

/* Counters of one call. */
typedef struct {
  size_t size;              /* = sizeof(hfci_stats), set by the caller          */
  int its;                  /* FGMRES iterations (max over right-hand sides)     */
  int restarts;             /* FGMRES cycles                                     */
  long long matvecs;        /* stencil applications, all systems and precisions */
  long long fp_steps;       /* fixed-point steps summed over (pole, RHS) systems */
  double final_relres;      /* max over RHS of the true FP64 relative residual  */
  double time_fci_ms;       /* device time in the preconditioner                 */
  double time_arnoldi_ms;   /* device time in matvec/CGS2/update                 */
  double time_total_ms;     /* wall time of the call                             */
  int harvested;            /* pairs appended to the harvest arrays              */
  int learned_accepted;     /* Arnoldi steps that kept the network's output      */
  int learned_fallbacks;    /* Arnoldi steps that fell back to FCI               */
  double time_net_ms;       /* device time in the network                        */
  double net_rho_mean;      /* mean scaled residual rho of the network proposals */
  double fci_rho_mean;      /* mean scaled residual rho of the FCI steps taken   */
} hfci_stats;

/* Per-kernel timing collected by hfci_ctx_profile (device time from HIP events
 * recorded on the context's stream around each launch of the class). */
typedef struct {
  long long launches;   /* launches timed                                       */
  double total_ms;      /* summed device time                                   */
  double alg_bytes;     /* summed algorithmic HBM bytes (reads + writes each
                           launch must move: every active system's vectors once,
                           shared kappa and right-hand sides once per launch)   */
} hfci_kernel_prof;

enum {
  HFCI_PROF_FP_STAGE = 0,  /* middle factors w <- a (A - z0) w + b w of a fixed-point
                              step (product form of eq. fix-pt-exp)                */
  HFCI_PROF_FP_FIRST = 1,  /* first factor of a step (also forms the shifted residual) */
  HFCI_PROF_APPLY = 2,     /* hfci_apply                                           */
  HFCI_PROF_FP_LAST = 3,   /* last factor of a step (adds the constant term y1)    */
  HFCI_PROF_FP_INIT = 4,   /* first and last factor of step one (from f, to y1)    */
  HFCI_PROF_FP_TRIPLE = 5, /* three middle factors in one pass (launch shape fuse 2)  */
  HFCI_PROF_N = 6
};

/* Fill *o with the defaults listed above. */
void hfci_default_opts(hfci_solve_opts* o);

/* Thread-local message of the last failing call ("" if none). */
const char* hfci_last_error(void);

/* Library version string. */
const char* hfci_version(void);

/* ---- context -------------------------------------------------------------
 * device: HIP device ordinal.  stream: a hipStream_t to issue work on, or NULL
 * for the library's own stream.  The context owns the workspace memory. */
hfci_status hfci_ctx_create(int device, void* stream, hfci_ctx** out);
void hfci_ctx_destroy(hfci_ctx* ctx);

/* Start (enable = k >= 1, counters reset: every k-th launch of each class is timed) or
 * stop (0) kernel timing on the context.  Errors: HFCI_E_ARG for enable < 0. */
hfci_status hfci_ctx_profile(hfci_ctx* ctx, int enable);
/* Copy the counters into out[HFCI_PROF_N] (HOST array). */
hfci_status hfci_ctx_profile_read(const hfci_ctx* ctx, hfci_kernel_prof* out);

/* ---- operator (Sec. 1.1; Sec. 7.1 eq. stiff-mass) --------------------------
 * c: DEVICE float64 array of nx*ny*nz wavespeeds (> 0), x fastest; read once,
 *    not retained.  h: grid spacing.  omega: angular frequency (> 0).
 * damp_cells (L >= 0) and damp_rho2 (>= 0): absorbing layer D_i = rho2 (d_i/L)^2.
 * Errors: HFCI_E_ARG for non-positive sizes/h/omega or a non-positive c. */
hfci_status hfci_op_create(hfci_ctx* ctx, int nx, int ny, int nz, double h,
                           const double* c, double omega, int damp_cells,
                           double damp_rho2, hfci_op** out);
void hfci_op_destroy(hfci_op* op);

/* Scalars of the normalised operator, written to host array out[7]:
 *   s = c_min^2/omega^2, s/h^2, b1, b2, rho2, kappa_min, kappa_max,
 * where [b1, b2] x [-rho2, 0] is the spectrum rectangle of Lemma 3.1 (Weyl
 * bounds of S - M with the exact extreme Dirichlet Laplacian eigenvalues). */
hfci_status hfci_op_info(const hfci_op* op, double* out7);

/* Launch shape of the operator's z-marching stencil kernels for one precision
 * (HFCI_F32 or HFCI_F64), tune[6] (HOST array):
 *   tune[0] kern: 0 = in-plane neighbours as cached global loads, 1 = each plane
 *           staged through LDS with its halo, 2 (HFCI_F32 only, with fuse = 1 and
 *           ty = 8) = as 1 for the two-factor passes, but every plane of every stream
 *           is loaded from HBM straight into a ring of P + 2 LDS slots (P = 2 planes
 *           ahead for pd = 2, 4 for pd = 3) without passing through registers, so
 *           more planes are in flight; single factors, and two-factor passes on
 *           grids with an odd nx or vectors of 2 GiB or more, run as kern 1;
 *           3 (HFCI_F32 only, fuse = 1 or 2, ty = 8, pd = 2) = as 2, with the middle
 *           two-factor passes on 64 x 28 output tiles (the input halo and kappa then
 *           cost less per output point; one 1024-thread block per CU), and with
 *           fuse = 2 the middle three-factor passes on 64 x 22 tiles;
 *   tune[1] ty:   the thread tile is 64 x ty (4 or 8);
 *   tune[2] pd:   HBM streams are issued pd planes ahead (kern 0: 1 or 2;
 *                 kern 1: 1..3 with ty = 4, 2..3 with ty = 8);
 *   tune[3] cz:   z-chunk length in planes (1..4096, or 0 = chosen from the grid);
 *   tune[4] fuse: 1 = the fixed-point factors run two per pass over HBM (temporal
 *                 blocking on 64 x 12 tiles with z-chunks cz), 0 = one per pass,
 *                 2 (kern 3 only) = as 1, with the middle factors of a step (those
 *                 between its first and last pair: q - 4 of them, or of step one's
 *                 run of pairs) three per pass where they split into threes and at
 *                 most two pairs (a run of 4 stays 2 + 2), on z-chunks of 2 cz;
 *   tune[5] sg:   1..16; with fuse >= 1 on grids whose pair tiles split into 8 XCD
 *                 slabs, the systems of a launch are taken sg at a time, tile by tile,
 *                 so kappa of a tile is read once per sg systems (1 = one system's
 *                 tiles after another's).
 * Shapes change launch geometry only: every grid point gets the same arithmetic,
 * while reductions (residual norms, the step size d) sum their block partials in a
 * different order.  New operators start at {1, 8, 2, 0, 0, 1}.  Errors: HFCI_E_ARG. */
hfci_status hfci_op_set_tune(hfci_op* op, int prec, const int* tune6);
hfci_status hfci_op_get_tune(const hfci_op* op, int prec, int* tune6);

/* Launch-shape autotuner: times the middle factors of the fixed-point iteration
 * (the dominant launches) over nsys systems (1..64, e.g. the number of shifted
 * systems that usually iterate together) for every valid shape, one, two and
 * (HFCI_F32) three factors per pass, keeps the fastest per factor for this operator and precision and writes
 * it to best6 (HOST, may be NULL).  timings (HOST, may be NULL if cap = 0) receives
 * up to cap rows of {kern, ty, pd, cz, fuse, sg, milliseconds per factor}; *count
 * (may be NULL) the number of shapes timed.  Uses the context's workspace (2 nsys
 * vectors of the precision); the operator's inputs and outputs of other calls are not
 * touched.  Timing-based, so two runs may pick different shapes (results then differ
 * only in the summation order of reductions).  Errors: HFCI_E_ARG. */
hfci_status hfci_op_autotune(hfci_op* op, int prec, int nsys, int* best6, double* timings, int cap,
                             int* count);

/* y_k = (A - shift I) x_k for k < nvec (normalised A).  prec: HFCI_F64
 * (complex128 x, y) or HFCI_F32 (complex64).  x and y are DEVICE buffers of
 * nvec*n complex values and must not overlap. */
hfci_status hfci_apply(const hfci_op* op, hfci_c128 shift, int prec, int nvec,
                       const void* x, void* y);

/* ---- Fourier-spectral operator (Sec. 7.1, eq. eig-Laplacian-spectral) --------
 * As hfci_op_create, with the discrete Laplacian replaced by the Fourier-spectral one on
 * a periodic grid: S = F^H Lambda F, lambda = s sum_j (2 pi min(m_j, N_j - m_j)/(N_j h))^2
 * for the Fourier mode m (the paper's (l_min/N)^2 sum_j min(i_j^2, (N - i_j)^2)), applied
 * with library 3D FFTs; kappa and the damping layer as for hfci_op_create.  The box
 * reported by hfci_op_info is [-kappa_max, lambda_max - kappa_min] x [-rho2, 0].
 * Accepted by hfci_op_info, hfci_op_get_tune, hfci_apply, hfci_contour_create / get / q,
 * hfci_shifted_solve (one FFT pair and one epilogue launch per fixed-point factor),
 * hfci_fci_apply and hfci_solve (precond FCI or NONE, k_in = 0); the other entry points
 * return HFCI_E_STATE.  Errors: as hfci_op_create. */
hfci_status hfci_op_create_spectral(hfci_ctx* ctx, int nx, int ny, int nz, double h,
                                    const double* c, double omega, int damp_cells,
                                    double damp_rho2, hfci_op** out);

/* ---- case two: the double-size formulation (Sec. 3, eq. mat-2x2) -----------
 * Creates a second operator handle for B = iC - I, C = [[0, I], [-(A1 + I), -A2]],
 * built on op's A = A1 - i A2 (A1 = S - M, A2 = D).  Solving B [x1; x2] = [0; f] gives
 * x2 = u and x1 = i u with A u = f.  Vectors of B hold 2n complex values: x1 (n, x
 * fastest) then x2 (n).  Its spectrum box, reported by hfci_op_info as [b1, b2] (rho2
 * unchanged), is [-1 - R, -1 + R] x [-rho2, 0] with R = rho2/2 + sqrt(rho2^2/4 + rho1)
 * and rho1 = b2 + 1 from op's box (Thm 3.2 and the remark after it).
 * On the returned handle: hfci_op_info, hfci_op_get_tune, hfci_apply ((B - shift) x),
 * hfci_contour_create / hfci_contour_get (poles and delta for B's box),
 * hfci_shifted_solve (vectors of 2n values; one launch per fixed-point factor, every
 * shifted system in one grid), hfci_fci_apply (Algorithm 1 on B, all poles in one batch:
 * opts->pole_batch and opts->graphs do not apply) and hfci_solve (FGMRES on B; pass the
 * physical right-hand side [0; f] to get [i u; u]; precond FCI or NONE).  The other
 * entry points, and the learned preconditioner, return HFCI_E_STATE for it.
 * The handle copies op's medium (op may be destroyed first); release it with
 * hfci_op_destroy.  Errors: HFCI_E_ARG, HFCI_E_STATE (op is itself a case-two handle). */
hfci_status hfci_op_case_two(const hfci_op* op, hfci_op** out);

/* ---- contour and per-pole parameters (Sec. 6.1-6.2, Sec. 4.2) -------------
 * J poles on the shifted-centre ellipse of eq. quad-points with radius
 * r = (rho2/2 + eps)/sin(pi/J) (eq. quad-radius), weights
 * sigma_j = (r cos theta_j + i t r sin theta_j)/J (eq. ellipse), and per pole
 * z0_j = (b1+b2)/2 + i Im z_j and delta_j minimising eq. fix-pt-conv for the
 * exponential-Taylor polynomial of degree q (eq. exp-taylor).
 * z, sigma (HOST arrays of J, or NULL) override the computed poles/weights;
 * delta (HOST array of J, or NULL) overrides the delta search.
 * q = 0 chooses the degree by Sec. 4.2's rule for the pole closest to the origin (not
 * with given deltas): the q in 1..16 minimising the cost of reducing its residual by a
 * fixed factor, ceil(q/P) / -ln nu_q with P = 2 for the finite-difference operators
 * (whose fixed-point factors run two per pass over HBM) and P = 1 for the spectral
 * operator (then it is the smallest nu^(1/q), the rule as written); hfci_contour_q reads
 * it back.
 * Without given poles, J = 0 takes J = 6 and eps = 0 takes the eps of hfci_contour_rule
 * for this operator's box, grid, J, t, q and fp_reduce 5 (with q = 0 also its degree);
 * hfci_contour_params reads J, t and eps back.
 * Errors: HFCI_E_ARG (J < 0 or > 256, J = 0 with given poles or deltas, q < 0 or > 16,
 * t <= 0, eps < 0);
 * HFCI_E_CONTOUR (a pole with Re z > 0 or Im z in (-eps-rho2, eps) when
 * computed, or nu >= 1). */
hfci_status hfci_contour_create(const hfci_op* op, int J, double t, double eps, int q,
                                const hfci_c128* z, const hfci_c128* sigma,
                                const double* delta, hfci_contour** out);
void hfci_contour_destroy(hfci_contour* c);

/* The degree q of the contour's polynomial (the chosen one when created with q = 0),
 * written to *q (HOST).  Errors: HFCI_E_ARG. */
hfci_status hfci_contour_q(const hfci_contour* c, int* q);

/* J, t and eps of the contour (the chosen ones when created with J = 0 or eps = 0),
 * written to HOST scalars (any may be NULL).  Errors: HFCI_E_ARG. */
hfci_status hfci_contour_params(const hfci_contour* c, int* J, double* t, double* eps);

/* Contour parameters by rule, host arithmetic only (no GPU work; b1, b2, rho2 are the
 * box of hfci_op_info, npoints the grid points nx*ny*nz).  Sec. 7.3 sets eps per
 * frequency with a small fixed number of poles (six); here *J_out = J, or 6 for J = 0,
 * and *eps_out is the eps, among 31 geometric steps over [0.01, 0.64], minimising the
 * predicted solve time
 *     T(eps) = eps * (Q S + Q M * 2e6 / npoints + 100),  Q = per_pass * ceil(q / per_pass),
 *     S = sum_j c_j, M = max_j c_j, c_j = ceil(ln(fp_reduce) / 2 / -ln nu_j(eps)),
 * where nu_j is eq. fix-pt-conv's rate for pole j of eq. quad-points (J, t, eps) at the
 * degree q: ceil(ln(fp_reduce) / -ln nu_j) steps reduce pole j's residual by fp_reduce in
 * the worst case, the adaptive stops measured about half of that, so c_j is the steps the
 * rule charges and Q c_j their products, a pass of per_pass factors counting per_pass
 * (per_pass = 2 for the finite-difference operators' multi-factor kernels, 1 for the
 * spectral operator).  With q = 0 the degree at each eps is
 * the one hfci_contour_create would choose for the pole nearest the origin (1..16, in
 * passes) and *q_out receives the chosen one; else *q_out = q.  The FGMRES iteration count
 * grows about in proportion to eps (measured on the finite-difference operators for J
 * from 4 to 16); per iteration the products of all poles cost their bytes, each launch a
 * latency worth about 2e6 grid points of one system's pass, and the Arnoldi step with the
 * combine about 100 products (both fitted to measured solve times on MI355X).  The rates
 * use 200 samples per side of the box and an 80-point delta scan; ties go to the smaller
 * eps.  Outputs HOST (any may be NULL).  Errors: HFCI_E_ARG (b1 >= b2, rho2 < 0,
 * npoints < 1, J < 0 or > 256, t <= 0, q < 0 or > 16, per_pass not 1 or 2,
 * fp_reduce <= 1). */
hfci_status hfci_contour_rule(double b1, double b2, double rho2, double npoints, int J, double t, int q,
                              int per_pass, double fp_reduce, int* J_out, double* eps_out, int* q_out);

/* Copy the contour's parameters into HOST arrays of length J (any may be NULL):
 * poles z, weights sigma, delta, Taylor centres z0, and the rate nu of each. */
hfci_status hfci_contour_get(const hfci_contour* c, hfci_c128* z, hfci_c128* sigma,
                             double* delta, hfci_c128* z0, double* nu);

/* ---- shifted solves (Sec. 4.2, eq. fix-pt-exp) -----------------------------
 * For every pole j < J and right-hand side k < nrhs, iterates eq. fix-pt-exp
 * for (A - z_j I) y = f_k from y = 0, either exactly `steps` steps (steps > 0)
 * or until ||f_k - (A - z_j) y|| <= ||f_k|| / reduce (at most max_steps).
 * f: DEVICE, nrhs vectors.  y: DEVICE, J*nrhs vectors, system (j, k) at index
 * j*nrhs + k.  prec: HFCI_F64 / HFCI_F32 for f and y.
 * steps_taken: HOST int array of J*nrhs (or NULL). */
hfci_status hfci_shifted_solve(const hfci_op* op, const hfci_contour* c, int prec,
                               int nrhs, const void* f, void* y, int steps,
                               double reduce, int max_steps, int* steps_taken);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): hfci_shifted_solve with every buffer
 * beyond f and y (the iterates' step constants and factor buffers, residual partials,
 * flags, lists and step counters) taken from a static device array of 64 MiB per GPU
 * instead of the context's workspace.  Same arguments, results and errors as
 * hfci_shifted_solve, bit for bit, for a case-one operator; it calls no hipMalloc,
 * hipFree or allocating library routine.  The array is looked up once per device when a
 * context is created there and stays allocated until the process ends.  Every call on a
 * GPU shares that GPU's array: calls that overlap in time on one GPU race.  Kernel timing
 * (hfci_ctx_profile) is paused during the call.
 * Errors: as hfci_shifted_solve; HFCI_E_ARG when the solve needs more than the 64 MiB
 * (about 3 J nrhs n complex values of the precision), before any launch; HFCI_E_STATE
 * for a case-two or spectral operator. */
hfci_status hfci_shifted_solve_noalloc(const hfci_op* op, const hfci_contour* c, int prec,
                                       int nrhs, const void* f, void* y, int steps,
                                       double reduce, int max_steps, int* steps_taken);

/* ---- FCI preconditioner (Algorithm 1) --------------------------------------
 * out_k = v + d_k w_k with w_k = sum_j sigma_j/z_j y_jk (steps 1-2),
 * d_k = (A w_k)^H f_k / (A w_k)^H (A w_k) (step 3), v from opts->k_in GMRES
 * steps on A v = f_k - d_k A w_k (step 4).  f, out: DEVICE, nrhs vectors of
 * complex128 (the FCI sweeps run in opts->precision).  stats may be NULL. */
hfci_status hfci_fci_apply(const hfci_op* op, const hfci_contour* c,
                           const hfci_solve_opts* opts, int nrhs,
                           const hfci_c128* f, hfci_c128* out, hfci_stats* stats);

/* ---- solve (Sec. 2: FCI inside flexible GMRES) ----------------------------
 * Solves (-Laplace_h - omega^2/c^2) u_k = f_k for k < nrhs with FGMRES(m),
 * classical Gram-Schmidt applied twice, Givens rotations and true-residual
 * restarts, all FP64, preconditioned by FCI.  f: DEVICE complex128 (physical
 * right-hand sides); u: DEVICE complex128, in: initial guess, out: solution.
 * Returns HFCI_W_NOCONV if max_it was reached first (u holds the last iterate). */
hfci_status hfci_solve(const hfci_op* op, const hfci_contour* c,
                       const hfci_solve_opts* opts, int nrhs,
                       const hfci_c128* f, hfci_c128* u, hfci_stats* stats);

/* ---- uneven batches (independent operators of different sizes) -------------
 * count instances (1..4096), instance i = operator ops[i] with its contour cons[i]
 * (all on one context; all contours with the same q; at most 65536 shifted systems
 * in all) and ONE right-hand side each.  Every factor of the fixed-point step is a
 * single launch over the shifted systems of all instances still iterating (a work
 * table maps workgroups to (instance, pole, tile)); the FCI quadrature, the step size
 * and FGMRES run per instance, in lockstep over the Arnoldi steps.
 *
 * hfci_shifted_solve_batch: hfci_shifted_solve for every instance: f[i] DEVICE n_i
 * values of the precision, y[i] DEVICE J_i * n_i (pole-major); steps_taken HOST,
 * sum of J_i ints in instance order (may be NULL).
 * hfci_solve_batch: hfci_solve for every instance: f[i], u[i] DEVICE complex128
 * n_i (u[i] in: initial guess, out: solution), stats HOST array of count
 * (may be NULL; each .size set).  stats[i] has instance i's FGMRES iterations,
 * restarts, final relative residual and FGMRES products; the shifted-system products
 * and fixed-point steps of the whole batch are added to stats[0].  precond must be
 * HFCI_PRECOND_FCI (contours needed) or HFCI_PRECOND_NONE; no training harvest.
 * Returns HFCI_W_NOCONV if any instance stops at max_it.  Errors: HFCI_E_ARG,
 * HFCI_E_STATE (contour of another operator, operators on different contexts). */
hfci_status hfci_shifted_solve_batch(int count, const hfci_op* const* ops, const hfci_contour* const* cons,
                                     int prec, const void* const* f, void* const* y, int steps, double reduce,
                                     int max_steps, int* steps_taken);
hfci_status hfci_solve_batch(int count, const hfci_op* const* ops, const hfci_contour* const* cons,
                             const hfci_solve_opts* opts, const hfci_c128* const* f, hfci_c128* const* u,
                             hfci_stats* stats);

/* ---- learned preconditioner (not part of the paper) -------------------------
 * A 3-level 3D U-Net (16/32/64 channels, 3x3x3 kernels, ReLU, 2x2x2 average
 * pooling, nearest up-sampling, skip concatenation, 1x1x1 head 16 -> 2) on
 * channels-last BF16 activations with FP32 accumulation on the matrix cores;
 * FP32 master weights trained with Adam.  Input channels: (Re r, Im r)/rms(r) and
 * omega^2 h^2/c^2; output: the correction divided by rms(r).  Grid sizes must be
 * multiples of 4.  Parameters are one FP32 array: per layer (c1a, c1b, c2a, c2b,
 * c3a, c3b, d2a, d2b, d1a, d1b) weights [27][Cout][Cin] then biases [Cout]
 * (c1a has Cin = 16: three real input channels, the rest must stay zero), then
 * the head weights [2][16] and biases [2]. */
typedef struct {
  size_t size;                 /* = sizeof(hfci_net_desc) */
  unsigned long long seed;     /* weight initialisation */
} hfci_net_desc;

typedef struct {
  size_t size;                 /* = sizeof(hfci_train_desc) */
  int nx, ny, nz;              /* grid of the pairs (multiples of 4 >= crop) */
  int npairs;
  const void* v;               /* DEVICE complex64 [npairs][n] residuals            */
  const void* e;               /* DEVICE complex64 [npairs][n] corrections          */
  const float* kch;            /* DEVICE float [nmedia][n]: omega^2 h^2 / c^2       */
  int nmedia;
  const int* medium_of_pair;   /* HOST int [npairs]: medium index of each pair, each
                                  in [0, nmedia) (checked)                          */
  int crop;                    /* training crop edge (multiple of 4)                */
  int steps;                   /* Adam steps (one crop each)                        */
  float lr, lr_min;            /* cosine schedule from lr to lr_min                 */
  int phase_aug;               /* 1: random global phase per step                   */
  unsigned long long seed;
  int log_every;               /* loss readback period (0 = never)                  */
  int verbose;                 /* 1: print the readbacks on stderr                  */
  double* loss_curve;          /* HOST array for the readbacks, or NULL             */
  int loss_curve_cap;
  int loss_kind;               /* 0: ||out - t||^2/||t||^2; 1: 1 - |<o,t>|^2/(||o||^2||t||^2)
                                  with o, t read as complex fields (scale and phase
                                  invariant: FGMRES only needs the direction);
                                  2: the residual the output leaves, min over complex d
                                  of ||v - d Ahat out||^2/||v||^2 with v the pair's
                                  residual (e is not read) and Ahat = A/(s/h^2)
                                  without damping, from the omega^2 h^2/c^2 channel
                                  (the arbiter's measure of a proposal, Alg. 1 step 3) */
} hfci_train_desc;

hfci_status hfci_net_create(hfci_ctx* ctx, const hfci_net_desc* desc, hfci_net** out);
void hfci_net_destroy(hfci_net* net);
/* Number of FP32 parameters; copy them to / from HOST arrays. */
long long hfci_net_param_count(const hfci_net* net);
hfci_status hfci_net_get_params(const hfci_net* net, float* host);
hfci_status hfci_net_set_params(hfci_net* net, const float* host);
hfci_status hfci_net_get_grads(const hfci_net* net, float* host);
/* Raw evaluation: x16 DEVICE bf16 [nz][ny][nx][16] (channels 3..15 zero), out DEVICE
 * float [nz][ny][nx][2]. */
hfci_status hfci_net_eval(hfci_net* net, int nx, int ny, int nz, const uint16_t* x16, float* out);
/* One forward/backward pass on (x16, target float [n][2]) with the loss loss_kind
 * (as in hfci_train_desc; for kind 2 the target is the residual v itself and Ahat takes
 * omega^2 h^2/c^2 from x16's third channel, zero values outside the box); update != 0
 * also takes an Adam step with lr.
 * *loss receives the loss (HOST). */
hfci_status hfci_net_train_step(hfci_net* net, int nx, int ny, int nz, const uint16_t* x16,
                                const float* target, float lr, int update, int loss_kind, double* loss);
/* Training loop over random crops of the pairs; returns the last loss read back. */
hfci_status hfci_net_train(hfci_net* net, const hfci_train_desc* desc, double* final_loss);
/* The preconditioner itself: z_k = rms(r_k) N(r_k / rms(r_k)) for complex128 DEVICE
 * vectors on op's grid (dims multiples of 4). */
hfci_status hfci_net_apply(hfci_net* net, const hfci_op* op, int nvec, const hfci_c128* r, hfci_c128* z);
/* omega^2 h^2 / c^2 of op as a DEVICE float array of n (the medium input channel). */
hfci_status hfci_op_medium_channel(const hfci_op* op, float* out);
/* Parameters and Adam state to / from a file (little-endian, with a header). */
hfci_status hfci_net_save(const hfci_net* net, const char* path);
hfci_status hfci_net_load(hfci_net* net, const char* path);

#ifdef __cplusplus
}
#endif
#endif /* HFCI_H */
