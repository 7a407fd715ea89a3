// Complex 7-point shifted stencil (A - shift I) x on gfx950, with fused epilogues.
//
// A = (s/h^2) (6 x_p - sum of the 6 neighbours) - kappa_p x_p - i D_p x_p  (normalised
// Helmholtz operator, Sec. 7.1 eq. stiff-mass, damping sign of Lemma 3.1), Dirichlet
// ghosts = 0.  D_p = rho2 (d_p/L)^2 is computed from the index, never stored.
//
// Kernel shape: a 64x4 block of threads owns a 64(x) x 4(y) column tile and marches
// through a chunk of z-planes.  The z-neighbours live in registers (prev/cur/next:
// every plane is loaded once per chunk), x-rows are 64 lanes wide so each load
// instruction moves one contiguous 512 B (complex64) or 1 KiB (complex128) row,
// and the x/y neighbours are re-reads of lines the block already pulled into L1/L2.
// Each launch covers (x-tiles, y-tiles, z-chunks x systems) so that one launch
// holds thousands of workgroups for the 256 CUs.
//
// Epilogues fused into the sweep:
//   EpiApply    y = (A - shift) x
//   EpiStage    one Horner stage of the exponential-Taylor fixed-point step
//               (eq. fix-pt-exp re-associated, see solver.cpp); the first stage
//               also forms the residual f - (A - z) y and its squared norm.
//   EpiDstep    partial sums of (A w)^H f and |A w|^2 for Alg. 1 step 3.
//   EpiResidual r = b - A u and |r|^2 (FP64 true residual of FGMRES).
#include "kernels.h"

namespace hfci {
namespace {

constexpr int TX = 64, TY = 4, NT = TX * TY;

template <typename T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };
template <typename T2> struct Scal;
template <> struct Scal<float2> { using t = float; };
template <> struct Scal<double2> { using t = double; };

__device__ __forceinline__ int layer_depth(int i, int n, int L) {
  const int d = min(i, n - 1 - i);
  return max(0, L - d);
}

// Block-wide sum of NACC doubles; result valid in thread 0.
template <int NACC>
__device__ __forceinline__ void block_sum(double (&acc)[NACC], double* sh) {
  const int t = threadIdx.x + TX * threadIdx.y;
  const int lane = t & 63, wid = t >> 6;
#pragma unroll
  for (int k = 0; k < NACC; ++k) {
    double v = acc[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) sh[wid * NACC + k] = v;
  }
  __syncthreads();
  if (t == 0) {
#pragma unroll
    for (int k = 0; k < NACC; ++k) {
      double v = 0.0;
      for (int w = 0; w < NT / 64; ++w) v += sh[w * NACC + k];
      acc[k] = v;
    }
  }
}

template <typename T, class Epi>
__global__ __launch_bounds__(NT) void zmarch_kernel(GridDesc g, int nzc, int czlen, Epi epi) {
  using T2 = typename V2<T>::t;
  constexpr int NACC = Epi::NACC;
  __shared__ double sh[(NT / 64) * (NACC > 0 ? NACC : 1)];
  const int x = blockIdx.x * TX + threadIdx.x;
  const int y = blockIdx.y * TY + threadIdx.y;
  const int zc = blockIdx.z % nzc;
  const int s = blockIdx.z / nzc;
  if (!epi.active(s)) return;  // uniform over the block
  const bool valid = (x < g.nx) && (y < g.ny);
  const int zb = zc * czlen;
  const int ze = min(g.nz, zb + czlen);
  const size_t plane = (size_t)g.nx * (size_t)g.ny;
  const T2* __restrict__ X = epi.in(s);
  const T* __restrict__ K = epi.kappa;
  T sre, sim;
  epi.shift(s, sre, sim);
  const T sh2 = (T)g.s_h2;
  const T dsc = (T)g.damp_scale;
  const T diag0 = (T)6 * sh2 - sre;
  double acc[NACC > 0 ? NACC : 1];
#pragma unroll
  for (int k = 0; k < (NACC > 0 ? NACC : 1); ++k) acc[k] = 0.0;

  if (valid) {
    const int dxy = max(layer_depth(x, g.nx, g.damp_cells), layer_depth(y, g.ny, g.damp_cells));
    size_t p = (size_t)x + (size_t)g.nx * (size_t)y + plane * (size_t)zb;
    const T2 zero = {(T)0, (T)0};
    T2 prev = zero, cur = X[p];
    if (zb > 0) prev = X[p - plane];
    for (int z = zb; z < ze; ++z, p += plane) {
      T2 next = zero, xm = zero, xp = zero, ym = zero, yp = zero;
      if (z + 1 < g.nz) next = X[p + plane];
      if (x > 0) xm = X[p - 1];
      if (x + 1 < g.nx) xp = X[p + 1];
      if (y > 0) ym = X[p - g.nx];
      if (y + 1 < g.ny) yp = X[p + g.nx];
      const int d = max(dxy, layer_depth(z, g.nz, g.damp_cells));
      const T dre = diag0 - K[p];
      const T dim = -((T)(d * d) * dsc + sim);
      const T nbr = ((prev.x + next.x) + (xm.x + xp.x)) + (ym.x + yp.x);
      const T nbi = ((prev.y + next.y) + (xm.y + xp.y)) + (ym.y + yp.y);
      T2 Sx;
      Sx.x = dre * cur.x - dim * cur.y - sh2 * nbr;
      Sx.y = dre * cur.y + dim * cur.x - sh2 * nbi;
      epi.point(s, p, Sx, cur, acc);
      prev = cur;
      cur = next;
    }
  }
  if constexpr (NACC > 0) {
    block_sum<NACC>(acc, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
      const int nblk = gridDim.x * gridDim.y * nzc;
      const int blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * zc);
#pragma unroll
      for (int k = 0; k < NACC; ++k) epi.partial_out(s, k, nblk, blk, acc[k]);
    }
  }
}

template <typename T>
struct EpiApply {
  using T2 = typename V2<T>::t;
  static constexpr int NACC = 0;
  const T2* x;
  T2* y;
  const T* kappa;
  size_t n;
  T sre, sim;
  __device__ bool active(int) const { return true; }
  __device__ const T2* in(int s) const { return x + (size_t)s * n; }
  __device__ void shift(int, T& re, T& im) const { re = sre; im = sim; }
  __device__ void point(int s, size_t p, const T2& Sx, const T2&, double*) const {
    y[(size_t)s * n + p] = Sx;
  }
  __device__ void partial_out(int, int, int, int, double) const {}
};

template <typename T, bool FIRST>
struct EpiStage {
  using T2 = typename V2<T>::t;
  static constexpr int NACC = FIRST ? 1 : 0;
  StageArgs<T2> a;
  const T* kappa;
  size_t n;
  __device__ bool active(int s) const { return a.active[s] != 0; }
  __device__ const T2* in(int s) const { return a.win + (size_t)s * n; }
  __device__ void shift(int s, T& re, T& im) const {
    const int pole = (a.sys0 + s) / a.nrhs;
    re = (T)a.poles[pole].z0_re;
    im = (T)a.poles[pole].z0_im;
  }
  __device__ void point(int s, size_t p, const T2& Sx, const T2& cur, double* acc) const {
    const int gs = a.sys0 + s;
    const int pole = gs / a.nrhs, r = gs % a.nrhs;
    const StageCoef c = a.coef[pole * a.q + a.m];
    const T2 yv = FIRST ? cur : a.y[(size_t)s * n + p];
    const T2 fv = a.f[(size_t)r * n + p];
    T2 o;
    o.x = (T)c.cB_re * Sx.x - (T)c.cB_im * Sx.y + (T)c.al_re * yv.x - (T)c.al_im * yv.y +
          (T)c.ga_re * fv.x - (T)c.ga_im * fv.y;
    o.y = (T)c.cB_re * Sx.y + (T)c.cB_im * Sx.x + (T)c.al_re * yv.y + (T)c.al_im * yv.x +
          (T)c.ga_re * fv.y + (T)c.ga_im * fv.x;
    a.wout[(size_t)s * n + p] = o;
    if constexpr (FIRST) {
      // r = f - (A - z) y = f - (A - z0) y + (z - z0) y
      const PoleDev pd = a.poles[pole];
      const double rr = (double)fv.x - (double)Sx.x + pd.zz_re * (double)yv.x - pd.zz_im * (double)yv.y;
      const double ri = (double)fv.y - (double)Sx.y + pd.zz_re * (double)yv.y + pd.zz_im * (double)yv.x;
      acc[0] += rr * rr + ri * ri;
    }
  }
  __device__ void partial_out(int s, int, int nblk, int blk, double v) const {
    a.partial[(size_t)s * nblk + blk] = v;
  }
};

template <typename T>
struct EpiDstep {
  using T2 = typename V2<T>::t;
  static constexpr int NACC = 3;
  const T2* w;
  const T2* f;
  const T* kappa;
  double* partial;
  size_t n;
  __device__ bool active(int) const { return true; }
  __device__ const T2* in(int s) const { return w + (size_t)s * n; }
  __device__ void shift(int, T& re, T& im) const { re = (T)0; im = (T)0; }
  __device__ void point(int s, size_t p, const T2& Sx, const T2&, double* acc) const {
    const T2 fv = f[(size_t)s * n + p];
    const double ar = Sx.x, ai = Sx.y, fr = fv.x, fi = fv.y;
    acc[0] += ar * fr + ai * fi;  // Re conj(Aw) f
    acc[1] += ar * fi - ai * fr;  // Im conj(Aw) f
    acc[2] += ar * ar + ai * ai;  // |Aw|^2
  }
  __device__ void partial_out(int s, int k, int nblk, int blk, double v) const {
    partial[((size_t)s * 3 + k) * nblk + blk] = v;
  }
};

struct EpiResidual {
  static constexpr int NACC = 1;
  const double2* u;
  const double2* b;
  double2* r;
  const double* kappa;
  double* partial;
  __device__ bool active(int) const { return true; }
  __device__ const double2* in(int) const { return u; }
  __device__ void shift(int, double& re, double& im) const { re = 0.0; im = 0.0; }
  __device__ void point(int, size_t p, const double2& Sx, const double2&, double* acc) const {
    const double2 bv = b[p];
    double2 o;
    o.x = bv.x - Sx.x;
    o.y = bv.y - Sx.y;
    r[p] = o;
    acc[0] += o.x * o.x + o.y * o.y;
  }
  __device__ void partial_out(int, int, int, int blk, double v) const { partial[blk] = v; }
};

struct Shape {
  dim3 grid;
  int nzc, czlen;
};

Shape shape_for(const GridDesc& g, int nsys) {
  Shape sh;
  const int gx = (g.nx + TX - 1) / TX, gy = (g.ny + TY - 1) / TY;
  // z-chunk: keep >= ~2048 blocks per system on large grids, chunks of >= 8 planes.
  int cz = 32;
  while (cz > 8 && (long)gx * gy * ((g.nz + cz - 1) / cz) < 2048) cz /= 2;
  sh.czlen = cz;
  sh.nzc = (g.nz + cz - 1) / cz;
  sh.grid = dim3(gx, gy, sh.nzc * nsys);
  return sh;
}

template <typename T, class Epi>
void run(hipStream_t st, const GridDesc& g, int nsys, const Epi& epi) {
  if (nsys <= 0) return;
  const Shape sh = shape_for(g, nsys);
  hipLaunchKernelGGL((zmarch_kernel<T, Epi>), sh.grid, dim3(TX, TY), 0, st, g, sh.nzc, sh.czlen, epi);
}

}  // namespace

template <typename T2>
int Launch<T2>::partial_blocks(const GridDesc& g) {
  const Shape sh = shape_for(g, 1);
  return (int)(sh.grid.x * sh.grid.y * sh.nzc);
}

template <typename T2>
void Launch<T2>::apply(hipStream_t st, const GridDesc& g, const void* kappa, double sre, double sim,
                       int nvec, const T2* x, T2* y) {
  using T = typename Scal<T2>::t;
  EpiApply<T> e{x, y, (const T*)kappa, (size_t)g.nx * g.ny * g.nz, (T)sre, (T)sim};
  run<T>(st, g, nvec, e);
}

template <typename T2>
void Launch<T2>::stage(hipStream_t st, const GridDesc& g, const void* kappa, const StageArgs<T2>& a,
                       bool first) {
  using T = typename Scal<T2>::t;
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  if (first) {
    EpiStage<T, true> e{a, (const T*)kappa, n};
    run<T>(st, g, a.nsys, e);
  } else {
    EpiStage<T, false> e{a, (const T*)kappa, n};
    run<T>(st, g, a.nsys, e);
  }
}

template <typename T2>
void Launch<T2>::dstep_partials(hipStream_t st, const GridDesc& g, const void* kappa, int nrhs,
                                const T2* w, const T2* f, double* partial) {
  using T = typename Scal<T2>::t;
  EpiDstep<T> e{w, f, (const T*)kappa, partial, (size_t)g.nx * g.ny * g.nz};
  run<T>(st, g, nrhs, e);
}

void launch_residual64(hipStream_t st, const GridDesc& g, const double* kappa, const double2* b,
                       const double2* u, double2* r, double* partial) {
  EpiResidual e{u, b, r, kappa, partial};
  run<double>(st, g, 1, e);
}

template struct Launch<float2>;
template struct Launch<double2>;

}  // namespace hfci
