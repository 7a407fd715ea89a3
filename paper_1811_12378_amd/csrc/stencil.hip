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

// Lanes outside the grid (x >= nx or y >= ny) and the Dirichlet ghosts read a clamped,
// always-valid address and zero the value with a select, so the loop body has no
// divergent branches.  Loads for plane z+1 are issued before plane z is computed and
// stored (one plane of software pipelining): the stores cannot alias-block them.
template <typename T, class Epi>
__global__ __launch_bounds__(NT) void zmarch_kernel(GridDesc g, int nzc, int czlen, int xcd_slab, Epi epi) {
  using T2 = typename V2<T>::t;
  using Aux = typename Epi::Aux;
  constexpr int NACC = Epi::NACC;
  __shared__ double sh[(NT / 64) * (NACC > 0 ? NACC : 1)];
  // XCD-aware tile order: consecutive workgroups go round-robin over the 8 XCDs, so
  // workgroup b is given tile (b % 8) * slab + b / 8 and every XCD walks a contiguous
  // run of tiles whose y/z neighbours it shares in its own L2.
  const int gx = gridDim.x, gy = gridDim.y;
  const int per_sys = gx * gy * nzc;
  const int s = blockIdx.z / nzc;
  int b = blockIdx.x + gx * (blockIdx.y + gy * (blockIdx.z % nzc));
  if (xcd_slab > 0) b = (b % 8) * xcd_slab + b / 8;
  const int bx = b % gx, by = (b / gx) % gy, zc = b / (gx * gy);
  (void)per_sys;
  if (!epi.active(s)) return;  // uniform over the block
  const int x = bx * TX + threadIdx.x;
  const int y = by * TY + threadIdx.y;
  const bool valid = (x < g.nx) && (y < g.ny);
  const int zb = zc * czlen;
  const int ze = min(g.nz, zb + czlen);
  const size_t plane = (size_t)g.nx * (size_t)g.ny;
  const T2* __restrict__ X = epi.in(s);
  const T* __restrict__ K = epi.kappa;
  const typename Epi::Sys sys = epi.sys(s);
  T sre, sim;
  epi.shift(sys, sre, sim);
  const T sh2 = (T)g.s_h2;
  const T dsc = (T)g.damp_scale;
  const T diag0 = (T)6 * sh2 - sre;
  double acc[NACC > 0 ? NACC : 1];
#pragma unroll
  for (int k = 0; k < (NACC > 0 ? NACC : 1); ++k) acc[k] = 0.0;

  if (valid && zb < ze) {
    const int dxy = max(layer_depth(x, g.nx, g.damp_cells), layer_depth(y, g.ny, g.damp_cells));
    const T mxm = x > 0 ? (T)1 : (T)0, mxp = x + 1 < g.nx ? (T)1 : (T)0;
    const T mym = y > 0 ? (T)1 : (T)0, myp = y + 1 < g.ny ? (T)1 : (T)0;
    const size_t oxm = x > 0 ? 1 : 0, oxp = x + 1 < g.nx ? 1 : 0;
    const size_t oym = y > 0 ? (size_t)g.nx : 0, oyp = y + 1 < g.ny ? (size_t)g.nx : 0;
    size_t p = (size_t)x + (size_t)g.nx * (size_t)y + plane * (size_t)zb;
    // plane zb: centre, z-1 neighbour, in-plane neighbours, kappa, epilogue inputs
    T2 prev = X[zb > 0 ? p - plane : p];
    if (zb == 0) prev = T2{(T)0, (T)0};
    T2 cur = X[p];
    T2 nxt = X[zb + 1 < g.nz ? p + plane : p];
    T2 xm = X[p - oxm], xp = X[p + oxp], ym = X[p - oym], yp = X[p + oyp];
    T kap = K[p];
    Aux aux = epi.load_aux(sys, s, p);
#pragma unroll 2
    for (int z = zb; z < ze; ++z, p += plane) {
      // ---- issue the loads of plane z+1 (clamped to plane z on the last plane) ----
      const bool more = z + 1 < ze;
      const size_t q1 = more ? p + plane : p;
      const T2 nn = X[z + 2 < g.nz ? p + 2 * plane : q1];
      const T2 xm1 = X[q1 - oxm], xp1 = X[q1 + oxp], ym1 = X[q1 - oym], yp1 = X[q1 + oyp];
      const T kap1 = K[q1];
      const Aux aux1 = epi.load_aux(sys, s, q1);
      // ---- compute and store plane z ----
      const T2 zn = (z + 1 < g.nz) ? nxt : T2{(T)0, (T)0};
      const int d = max(dxy, layer_depth(z, g.nz, g.damp_cells));
      const T dre = diag0 - kap;
      const T dim = -((T)(d * d) * dsc + sim);
      const T nbr = ((prev.x + zn.x) + (mxm * xm.x + mxp * xp.x)) + (mym * ym.x + myp * yp.x);
      const T nbi = ((prev.y + zn.y) + (mxm * xm.y + mxp * xp.y)) + (mym * ym.y + myp * yp.y);
      T2 Sx;
      Sx.x = dre * cur.x - dim * cur.y - sh2 * nbr;
      Sx.y = dre * cur.y + dim * cur.x - sh2 * nbi;
      epi.point(sys, s, p, Sx, cur, aux, acc);
      // ---- rotate ----
      prev = cur;
      cur = zn;
      nxt = nn;
      xm = xm1; xp = xp1; ym = ym1; yp = yp1;
      kap = kap1;
      aux = aux1;
    }
  }
  if constexpr (NACC > 0) {
    block_sum<NACC>(acc, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
      const int nblk = gx * gy * nzc;
      const int blk = bx + gx * (by + gy * zc);
#pragma unroll
      for (int k = 0; k < NACC; ++k) epi.partial_out(s, k, nblk, blk, acc[k]);
    }
  }
}

struct NoAux {};

template <typename T>
struct EpiApply {
  using T2 = typename V2<T>::t;
  static constexpr int NACC = 0;
  struct Sys {};
  using Aux = NoAux;
  const T2* x;
  T2* y;
  const T* kappa;
  size_t n;
  T sre, sim;
  __device__ bool active(int) const { return true; }
  __device__ const T2* in(int s) const { return x + (size_t)s * n; }
  __device__ Sys sys(int) const { return Sys{}; }
  __device__ void shift(const Sys&, T& re, T& im) const { re = sre; im = sim; }
  __device__ Aux load_aux(const Sys&, int, size_t) const { return Aux{}; }
  __device__ void point(const Sys&, int s, size_t p, const T2& Sx, const T2&, const Aux&, double*) const {
    y[(size_t)s * n + p] = Sx;
  }
  __device__ void partial_out(int, int, int, int, double) const {}
};

template <typename T, bool FIRST>
struct EpiStage {
  using T2 = typename V2<T>::t;
  static constexpr int NACC = FIRST ? 1 : 0;
  struct Sys {
    T cBr, cBi, alr, ali, gar, gai, z0r, z0i;
    double zzr, zzi;
    const T2* y;
    const T2* f;
    T2* out;
  };
  struct Aux {
    T2 y, f;
  };
  StageArgs<T2> a;
  const T* kappa;
  size_t n;
  __device__ bool active(int s) const { return a.active[s] != 0; }
  __device__ const T2* in(int s) const { return a.win + (size_t)s * n; }
  __device__ Sys sys(int s) const {
    const int gs = a.sys0 + s;
    const int pole = gs / a.nrhs, r = gs % a.nrhs;
    const StageCoef c = a.coef[pole * a.q + a.m];
    const PoleDev pd = a.poles[pole];
    return Sys{(T)c.cB_re, (T)c.cB_im, (T)c.al_re, (T)c.al_im, (T)c.ga_re, (T)c.ga_im, (T)pd.z0_re,
               (T)pd.z0_im, pd.zz_re, pd.zz_im, a.y + (size_t)s * n, a.f + (size_t)r * n, a.wout + (size_t)s * n};
  }
  __device__ void shift(const Sys& c, T& re, T& im) const { re = c.z0r; im = c.z0i; }
  __device__ Aux load_aux(const Sys& c, int, size_t p) const {
    Aux x;
    if constexpr (FIRST) x.y = T2{(T)0, (T)0};
    else x.y = c.y[p];
    x.f = c.f[p];
    return x;
  }
  __device__ void point(const Sys& c, int, size_t p, const T2& Sx, const T2& cur, const Aux& ax, double* acc) const {
    const T2 yv = FIRST ? cur : ax.y;
    const T2 fv = ax.f;
    T2 o;
    o.x = c.cBr * Sx.x - c.cBi * Sx.y + c.alr * yv.x - c.ali * yv.y + c.gar * fv.x - c.gai * fv.y;
    o.y = c.cBr * Sx.y + c.cBi * Sx.x + c.alr * yv.y + c.ali * yv.x + c.gar * fv.y + c.gai * fv.x;
    c.out[p] = o;
    if constexpr (FIRST) {
      // r = f - (A - z) y = f - (A - z0) y + (z - z0) y
      const double rr = (double)fv.x - (double)Sx.x + c.zzr * (double)yv.x - c.zzi * (double)yv.y;
      const double ri = (double)fv.y - (double)Sx.y + c.zzr * (double)yv.y + c.zzi * (double)yv.x;
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
  struct Sys {
    const T2* f;
  };
  struct Aux {
    T2 f;
  };
  const T2* w;
  const T2* f;
  const T* kappa;
  double* partial;
  size_t n;
  __device__ bool active(int) const { return true; }
  __device__ const T2* in(int s) const { return w + (size_t)s * n; }
  __device__ Sys sys(int s) const { return Sys{f + (size_t)s * n}; }
  __device__ void shift(const Sys&, T& re, T& im) const { re = (T)0; im = (T)0; }
  __device__ Aux load_aux(const Sys& c, int, size_t p) const { return Aux{c.f[p]}; }
  __device__ void point(const Sys&, int, size_t, const T2& Sx, const T2&, const Aux& ax, double* acc) const {
    const double ar = Sx.x, ai = Sx.y, fr = ax.f.x, fi = ax.f.y;
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
  struct Sys {};
  struct Aux {
    double2 b;
  };
  const double2* u;
  const double2* b;
  double2* r;
  const double* kappa;
  double* partial;
  __device__ bool active(int) const { return true; }
  __device__ const double2* in(int) const { return u; }
  __device__ Sys sys(int) const { return Sys{}; }
  __device__ void shift(const Sys&, double& re, double& im) const { re = 0.0; im = 0.0; }
  __device__ Aux load_aux(const Sys&, int, size_t p) const { return Aux{b[p]}; }
  __device__ void point(const Sys&, int, size_t p, const double2& Sx, const double2&, const Aux& ax,
                        double* acc) const {
    double2 o;
    o.x = ax.b.x - Sx.x;
    o.y = ax.b.y - Sx.y;
    r[p] = o;
    acc[0] += o.x * o.x + o.y * o.y;
  }
  __device__ void partial_out(int, int, int, int blk, double v) const { partial[blk] = v; }
};

struct Shape {
  dim3 grid;
  int nzc, czlen, xcd_slab;
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
  const int per_sys = gx * gy * sh.nzc;
  sh.xcd_slab = (per_sys % 8 == 0 && per_sys >= 64) ? per_sys / 8 : 0;
  return sh;
}

template <typename T, class Epi>
void run(hipStream_t st, const GridDesc& g, int nsys, const Epi& epi) {
  if (nsys <= 0) return;
  const Shape sh = shape_for(g, nsys);
  hipLaunchKernelGGL((zmarch_kernel<T, Epi>), sh.grid, dim3(TX, TY), 0, st, g, sh.nzc, sh.czlen, sh.xcd_slab, epi);
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
