// Internal interface between the host runtime and the HIP kernels of libhfci.
//
// Vectors are complex, interleaved (re, im) as float2 / double2, over an
// nx*ny*nz grid with x fastest.  Batches of vectors are strided by n.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

namespace hfci {

// Launch shape of the z-marching stencil kernels: kern 0 keeps the in-plane neighbours
// as cached global loads, kern 1 stages each plane through LDS; a 64 x ty thread tile,
// HBM streams prefetched pd planes ahead, z-chunks of cz planes (0: from the grid size);
// fuse 1 applies the fixed-point factors two per pass (64 x 12 tiles, z-chunks cz; loads
// one plane ahead, two when pd is 3).
struct KernelTune {
  // fuse: 0 one factor per pass, 1 two (the later steps' first and last factors and the
  // middle ones in pairs), 2 (kern 3 only) as 1 with the middle factors in threes where
  // they split so; sg: with several factors per pass, the systems of a launch are taken sg
  // at a time, tile by tile, inside each XCD's slab of tiles (1 = system after system)
  int kern = 1, ty = 8, pd = 2, cz = 0, fuse = 0, sg = 1;
};

// Geometry and operator scalars of the normalised A = (s/h^2) L7 - kappa - i D, plus
// the launch shapes used for complex64 and complex128 vectors.
struct GridDesc {
  int nx, ny, nz;
  int damp_cells;        // L
  double damp_scale;     // rho2 / L^2, so D = damp_scale * depth^2
  double s_h2;           // s / h^2
  KernelTune tune32, tune64;
};
bool tune_valid(const KernelTune& t);

// One linear factor of the product-form fixed-point step, per pole:
//   w_out = a * (A - z0) w_in + b * w_in   (+ y1 on the last factor of a step).
struct FactorCoef {
  double a_re, a_im, b_re, b_im;
};

// Per-pole constants used inside the stage kernels.
struct PoleDev {
  double z0_re, z0_im;   // Taylor centre (shift applied by the stencil)
  double zz_re, zz_im;   // z - z0 (residual of the first stage)
};

// Kinds of factor launch (bit set):
//   RESID  the input is the iterate y; also forms |f - (A - z) y|^2 partials
//   ADD    adds the step's constant vector y1 (last factor of a step)
//   DUAL   writes the output to a second vector as well
//   INF    the input is the system's right-hand side f (first factor of step one)
enum : int { kFacResid = 1, kFacAdd = 2, kFacDual = 4, kFacInF = 8 };

// Work description of one batched factor launch over the systems listed in
// list[0..count) (indices s in [0, nsys), global system gs = sys0 + s,
// pole = gs / nrhs, rhs = gs % nrhs).  Vectors are strided by n per system (per rhs for f).
template <typename T2>
struct FactorArgs {
  const T2* win;          // input w (or y with RESID), per system
  const T2* f;            // right-hand sides, per rhs
  const T2* y1;           // constant term of the step (ADD), per system
  T2* wout;               // output, per system
  T2* wout2;              // second output (DUAL), per system
  const FactorCoef* coef; // [pole][cstride]; this launch uses entry k
  const PoleDev* poles;   // [pole]
  const int* list;        // DEVICE array of the systems to run, count entries
  double* partial;        // residual partial sums [nsys][nblk] (RESID only)
  int count, sys0, nrhs, cstride, k;
};

// Case two (eq. mat-2x2): factors of the fixed-point step on B = iC - I, whose vectors
// hold 2 n values (x1 then x2).  System s = pole * nrhs + rhs, vectors strided by 2 n;
// kind bits as for the case-one factors (kFacResid, kFacAdd, kFacInF, kFacDual), and a
// system with active[s] == 0 is skipped.  Residual partials: [nsys][b2_blocks(g)].
template <typename T2>
struct B2Args {
  const T2* win;           // input, per system (the right-hand sides, per rhs, with kFacInF)
  const T2* f;             // right-hand sides, per rhs (kFacResid)
  const T2* y1;            // constant term of the step, per system (kFacAdd)
  T2* wout;                // output, per system
  T2* wout2;               // second output, per system (kFacDual)
  const FactorCoef* coef;  // [pole][cstride]; this launch uses entry k
  const PoleDev* poles;    // [pole]
  const int* active;       // [nsys]
  double* partial;         // [nsys][b2_blocks(g)] (kFacResid)
  int nrhs, cstride, k;
};
int b2_blocks(const GridDesc& g);
// false for an unsupported combination of kind bits (nothing is launched)
template <typename T2>
bool launch_b2_factor(hipStream_t st, const GridDesc& g, const void* K, int kind, int nsys, const B2Args<T2>& a);
// Fourier-spectral operator (Sec. 7.1): kernels around the library FFTs.  SpecArgs are the
// factor arguments of B2Args plus sw = S w of the inputs (indexed as the inputs).
template <typename T2>
struct SpecArgs {
  const T2* win;
  const T2* sw;
  const T2* f;
  const T2* y1;
  T2* wout;
  T2* wout2;
  const FactorCoef* coef;
  const PoleDev* poles;
  const int* active;
  double* partial;         // [nsys][spec_blocks(g)] (kFacResid)
  int nrhs, cstride, k;
};
int spec_blocks(const GridDesc& g);
// c_v *= lambda / N (the diagonal between a forward and an unnormalised inverse FFT)
template <typename T2>
void launch_spec_scale(hipStream_t st, T2* c, int nvec, const GridDesc& g, double s, double h);
template <typename T2>
bool launch_spec_factor(hipStream_t st, const GridDesc& g, const void* K, int kind, int nsys, const SpecArgs<T2>& a);
// y = (A - shift) x from sx = S x (y may alias sx)
template <typename T2>
void launch_spec_apply(hipStream_t st, const GridDesc& g, const void* K, int nvec, const T2* x, const T2* sx, T2* y,
                       double sr, double si);
// Alg. 1 step 3 partials from sw = S w, layout as launch_b2_dstep (spec_blocks(g) per row)
template <typename T2>
void launch_spec_dstep(hipStream_t st, const GridDesc& g, const void* K, int nrhs, const T2* w, const T2* sw,
                       const T2* f, double* partial);
// res = b - A u from su = S u (res may alias su), nblk partial sums of |res|^2
void launch_spec_residual64(hipStream_t st, const GridDesc& g, const double* K, const double2* b, const double2* u,
                            const double2* su, double2* res, double* partial, int nblk);

// Alg. 1 step 3 on B: partial[(3 r + c)][b2_blocks(g)] = Re, Im of (B w_r)^H f_r and |B w_r|^2
template <typename T2>
void launch_b2_dstep(hipStream_t st, const GridDesc& g, const void* K, int nrhs, const T2* w, const T2* f,
                     double* partial);
// res = b - B u in FP64 with nblk partial sums of |res|^2 (nblk >= 1 blocks)
void launch_b2_residual64(hipStream_t st, const GridDesc& g, const double* K, const double2* b, const double2* u,
                          double2* res, double* partial, int nblk);
// y_v = (B - shift) x_v for v < nvec (vectors of 2 n values, not overlapping)
template <typename T2>
void launch_b2_apply(hipStream_t st, const GridDesc& g, const void* K, int nvec, const T2* x, T2* y, double sr,
                     double si);

template <typename T2>
struct Launch {
  static void apply(hipStream_t st, const GridDesc& g, const void* kappa, double shift_re,
                    double shift_im, int nvec, const T2* x, T2* y);
  // one factor launch of the given kind (kFac* bits) over a.list; false for an
  // unsupported combination of bits (nothing is launched)
  static bool factor(hipStream_t st, const GridDesc& g, const void* kappa, const FactorArgs<T2>& a, int kind);
  // factors a.k and a.k + 1 in one pass; kind: the first factor's input bits (kFacResid,
  // kFacInF) and the second factor's epilogue bits (kFacAdd, kFacDual); the output must
  // not alias the input
  static bool factor_pair(hipStream_t st, const GridDesc& g, const void* kappa, const FactorArgs<T2>& a,
                          int kind);
  // middle factors a.k, a.k + 1 and a.k + 2 in one pass (no kind bits), on z-chunks of
  // 2 cz planes; false (nothing launched) unless the complex64 launch shape is kern 3 with
  // fuse 2 and the grid suits the pair kernels (an even nx, vectors under 2 GiB); the
  // output must not alias the input
  static bool factor_triple(hipStream_t st, const GridDesc& g, const void* kappa, const FactorArgs<T2>& a);
  // whether factor_triple launches on this grid with its current launch shape
  static bool triple_runs(const GridDesc& g);
  // a kFacInF single factor over systems s = j * nrhs + r (all listed, count a multiple of
  // nrhs, at most 64 poles): each point forms the stencil of f once for all poles; false
  // (nothing launched) when those conditions do not hold
  static bool factor_fanout(hipStream_t st, const GridDesc& g, const void* kappa, const FactorArgs<T2>& a);
  static int pair_blocks(const GridDesc& g);  // residual partials per system of a pair launch
  // whether factor_pair runs on this grid (32-bit byte offsets: each vector under 4 GiB)
  static bool pair_fits(const GridDesc& g);
  // partial sums for the step size d: conj(A w).f and |A w|^2, per rhs.
  static void dstep_partials(hipStream_t st, const GridDesc& g, const void* kappa, int nrhs,
                             const T2* w, const T2* f, double* partial);
  static int partial_blocks(const GridDesc& g);
};

// ---- uneven batches: many operators in one launch (work table) ----
// Per instance: its grid, kappa and the launch geometry of its stencil tiles.
struct MultiInst {
  GridDesc g;
  const void* kappa;  // float* or double*
  int gx, gy, nzc, czlen, xcd_slab, per_sys;
  // the same for two factors per pass (64 x 12 tiles); pper_sys = 0 where it does not run
  int pgx, pgy, pnzc, pczlen, pxcd_slab, pper_sys;
};
// Per shifted system (instance, pole): its vectors by role (0 f, 1 y, 2 y1, 3 wA, 4 wB),
// the pole's factor coefficients and constants, its residual-partial row.
enum : int { kRoleF = 0, kRoleY = 1, kRoleY1 = 2, kRoleWA = 3, kRoleWB = 4, kRoleNone = -1 };
template <typename T2>
struct MultiSys {
  T2* vec[5];
  const FactorCoef* coef;  // this pole's cstride coefficients
  const PoleDev* pole;
  double* partial;         // nblk doubles
  int inst, nblk, slot, pad;
};
// One factor launch over the systems listed in the work table seg[i] = {first block,
// system}, ascending in the first block; a block finds its system by binary search over
// the nseg rows.  A row with system -1 is a sentinel: blocks that land on it exit.
template <typename T2>
struct MultiLaunch {
  static constexpr int kTy = 8, kPd = 2;  // launch shape of the multi-instance kernel
  static void factor(hipStream_t st, const MultiInst* inst, const MultiSys<T2>* sys, const int2* seg, int nseg,
                     int nblocks, int kind, int role_in, int role_out, int role_out2, int k, int cstride,
                     bool f64);
  // factors k and k + 1 in one pass over the work table of pair tiles (kind as for
  // Launch::factor_pair); false for an unsupported kind
  static bool factor_pair(hipStream_t st, const MultiInst* inst, const MultiSys<T2>* sys, const int2* seg, int nseg,
                          int nblocks, int kind, int role_in, int role_out, int role_out2, int k, int cstride);
  // geometry of one instance for this launch shape (host)
  static MultiInst describe(const GridDesc& g, const void* kappa);
};
// fixed-point bookkeeping of a batch: per system s, its partial row (sys[s].partial,
// sys[s].nblk) against fnorm2[sys[s].slot]
template <typename T2>
void launch_fp_check_multi(hipStream_t st, const MultiSys<T2>* sys, int nsys, const double* fnorm2,
                           int fixed_steps, double reduce, int max_steps, int* active, int* steps, double* rnorm2);
// adaptive test of a batch that also rebuilds the work tables on the device: rows
// {first block, system} of the active systems in seg (bps[s].x blocks each) and segp
// (bps[s].y), then the sentinel {total, -1} and {INT_MAX, -1} up to row nsys; the flags
// also go to host_flags (device-visible pinned host memory, nsys ints)
template <typename T2>
void launch_fp_test_multi(hipStream_t st, const MultiSys<T2>* sys, int nsys, const int2* bps, const double* fnorm2,
                          double reduce, int max_steps, int* active, int* steps, double* rnorm2, int2* seg,
                          int2* segp, int* host_flags);

// FP64 residual r = b - A u (shift 0) with partial sums of |r|^2.
void launch_residual64(hipStream_t st, const GridDesc& g, const double* kappa, const double2* b,
                       const double2* u, double2* r, double* partial);

// ---- BLAS-1 and reductions (blas.hip) ----
int blas_blocks(size_t n);
// partial[k][blk] over nblk blocks -> out[k], for k < ncomp (deterministic order).
void launch_reduce(hipStream_t st, const double* partial, int nblk, int ncomp, double* out);
// FGMRES building blocks (complex128).
// Basis vector i of V starts at V + i*vstride.
void launch_multidot(hipStream_t st, const double2* V, int nv, size_t n, size_t vstride,
                     const double2* w, double* partial);     // partial[(2i+c)][blk]
void launch_multiaxpy(hipStream_t st, double2* w, const double2* V, int nv, size_t n,
                      size_t vstride, const double* h, double sign);  // w += sign * sum h_i V_i
// Classical Gram-Schmidt twice of w against V[0..nv), then |w|^2:
//   h1 = V^H w, w -= V h1, h2 = V^H w, w -= V h2, nrm2 = |w|^2  (device h1, h2: 2 nv
//   doubles each, nrm2: 1; partial: 2 nv * blas_blocks(n) doubles of scratch).
// For nv <= 32 the update and the next reduction share one pass over V.
void launch_cgs2(hipStream_t st, const double2* V, int nv, size_t n, size_t vstride, double2* w, double* partial,
                 double* h1, double* h2, double* nrm2);
void launch_norm2_partial(hipStream_t st, const void* x, bool f32, size_t n, double* partial);
void launch_scale_inv(hipStream_t st, double2* v, const double2* w, size_t n, const double* nrm2);
void launch_fill_zero(hipStream_t st, void* p, size_t bytes);
void launch_copy_scaled64(hipStream_t st, double2* dst, const double2* src, size_t n, double s);
void launch_convert_64_to_32(hipStream_t st, float2* dst, const double2* src, size_t n);
void launch_convert_32_to_64(hipStream_t st, double2* dst, const float2* src, size_t n);
// w_r = sum_p c_p y_{p,r} (+= if accumulate), systems laid out pole-major; with steps
// (device, per system) the systems with steps <= 1 read y1 instead of y.
template <typename T2>
void launch_combine(hipStream_t st, T2* w, const T2* y, const double* coef /*[npole][2]*/,
                    int npole, int nrhs, size_t n, bool accumulate, const T2* y1 = nullptr,
                    const int* steps = nullptr);
// out64_r = d_r * w_r  (d from device array d[2r], d[2r+1])
template <typename T2>
void launch_scale_out(hipStream_t st, double2* out, const T2* w, const double* d, int nrhs,
                      size_t n);
// fixed-point bookkeeping: residual norms -> active flags and step counters.
void launch_fp_check(hipStream_t st, const double* partial, int nblk, int nsys, int sys0,
                     int nrhs, const double* fnorm2, int fixed_steps, double reduce,
                     int max_steps, int* active, int* steps, double* rnorm2);
// d_r = num_r / den_r from reduced sums [nrhs][3]
void launch_dfinish(hipStream_t st, const double* sums, int nrhs, double* d);
void launch_set_int(hipStream_t st, int* p, int v, int count);
// start of the fixed-point iteration: every system active and listed, steps = 1 (or 0
// for a zero right-hand side in adaptive mode), after the first step.
void launch_fp_start(hipStream_t st, int nsys, int sys0, int nrhs, const double* fnorm2, bool fixed,
                     int* active, int* steps, int* list);
// list[0..count) = indices s with active[s] != 0, in increasing order (one block).
void launch_build_list(hipStream_t st, const int* active, int nsys, int* list);
// adaptive stopping test + list compaction in one launch; the flags also go to
// host_flags (device-visible pinned host memory, nsys ints)
void launch_fp_test(hipStream_t st, const double* partial, int nblk, int nsys, int sys0, int nrhs,
                    const double* fnorm2, double reduce, int max_steps, int* active, int* steps, double* rnorm2,
                    int* list, int* host_flags);

}  // namespace hfci
