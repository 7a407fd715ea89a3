// Case two (Sec. 3, eq. mat-2x2): the double-size operator B = iC - I with
// C = [[0, I], [-(A1 + I), -A2]], A = A1 - i A2, A1 = S - M, A2 = D.  Written out,
//   B [x1; x2] = [ -x1 + i x2 ;  -i (A1 + I) x1 - (I + i A2) x2 ],
// one 7-point stencil on x1 plus pointwise terms.  A vector of B holds x1 (n values)
// then x2 (n values), n the grid points.
//
// Kernels: one factor of the product-form fixed-point step (eq. fix-pt-exp, as the
// factors of params.cpp), w_out = a (B - z0) w + b w, or two consecutive factors in one
// pass over HBM, over all shifted systems, with the epilogues of the case-one kernels
// (residual partials, adding y1, a second output): b2_zm_kernel, one thread per grid
// column marching in z.  Then the plain product (B - shift) x, the step-size partials and
// the FP64 residual: one thread per grid point.  Both blocks per thread; the neighbours come
// through the cache (no LDS staging).
#include "kernels.h"

namespace hfci {
namespace {

constexpr int NT = 256;

template <typename T> struct Vec2;
template <> struct Vec2<float> { using t = float2; };
template <> struct Vec2<double> { using t = double2; };
template <typename T2> struct Scal;
template <> struct Scal<float2> { using t = float; };
template <> struct Scal<double2> { using t = double; };

__device__ __forceinline__ int depth_in_layer(int i, int n, int L) { return max(0, L - min(i, n - 1 - i)); }

template <typename T>
struct Cx {
  T x, y;
};
template <typename T>
__device__ __forceinline__ Cx<T> cmul(T ar, T ai, Cx<T> v) {
  return Cx<T>{ar * v.x - ai * v.y, ar * v.y + ai * v.x};
}

template <typename T, typename T2>
__device__ __forceinline__ Cx<T> ldc(const T2* __restrict__ x, size_t p) {
  const T2 v = x[p];
  return Cx<T>{v.x, v.y};
}

// block 1 of (B - z0) x at a point: -(1 + z0) x1 + i x2
template <typename T>
__device__ __forceinline__ Cx<T> b2_block1(Cx<T> x1, Cx<T> x2, T z0r, T z0i) {
  const Cx<T> s1 = cmul((T)1 + z0r, z0i, x1);
  return Cx<T>{-s1.x - x2.y, -s1.y + x2.x};
}

// block 2 of (B - z0) x at a point: -i (A1 + I) x1 - (1 + z0) x2 - i D x2, from the point's
// x1 and x2, the sum (nr, ni) of x1 over its in-grid neighbours, kappa and the damping D
template <typename T>
__device__ __forceinline__ Cx<T> b2_block2(const GridDesc& g, Cx<T> x1, Cx<T> x2, T nr, T ni, T kap, T dmp, T z0r,
                                           T z0i) {
  const T sh2 = (T)g.s_h2;
  // (A1 + I) x1 = s/h^2 (6 x1 - neighbours) - kappa x1 + x1
  const T ar = sh2 * ((T)6 * x1.x - nr) + ((T)1 - kap) * x1.x;
  const T ai = sh2 * ((T)6 * x1.y - ni) + ((T)1 - kap) * x1.y;
  const Cx<T> s2 = cmul((T)1 + z0r, z0i, x2);
  return Cx<T>{ai - s2.x + dmp * x2.y, -ar - s2.y - dmp * x2.x};
}

template <typename T>
__device__ __forceinline__ T b2_damping(const GridDesc& g, int i, int j, int k) {
  const int d = max(max(depth_in_layer(i, g.nx, g.damp_cells), depth_in_layer(j, g.ny, g.damp_cells)),
                    depth_in_layer(k, g.nz, g.damp_cells));
  return (T)(d * d) * (T)g.damp_scale;
}

// one factor at a point: a o + b x, with o = (B - z0) x there
template <typename T>
__device__ __forceinline__ Cx<T> b2_fac(T ar, T ai, T br, T bi, Cx<T> o, Cx<T> x) {
  const Cx<T> u = cmul(ar, ai, o), v = cmul(br, bi, x);
  return Cx<T>{u.x + v.x, u.y + v.y};
}

// (B - z0) x at point p = i + nx (j + ny k) of the vector x (x1 at x, x2 at x + npt);
// also returns the point's x1 and x2.
template <typename T, typename T2>
__device__ __forceinline__ void b2_point(const GridDesc& g, const T* __restrict__ K, const T2* __restrict__ x,
                                         size_t npt, size_t p, int i, int j, int k, T z0r, T z0i, Cx<T>& o1,
                                         Cx<T>& o2, Cx<T>& x1, Cx<T>& x2) {
  const size_t sx = 1, sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  x1 = ldc<T>(x, p);
  x2 = ldc<T>(x, npt + p);
  T nr = (T)0, ni = (T)0;
  if (i > 0) { const T2 v = x[p - sx]; nr += v.x; ni += v.y; }
  if (i + 1 < g.nx) { const T2 v = x[p + sx]; nr += v.x; ni += v.y; }
  if (j > 0) { const T2 v = x[p - sy]; nr += v.x; ni += v.y; }
  if (j + 1 < g.ny) { const T2 v = x[p + sy]; nr += v.x; ni += v.y; }
  if (k > 0) { const T2 v = x[p - sz]; nr += v.x; ni += v.y; }
  if (k + 1 < g.nz) { const T2 v = x[p + sz]; nr += v.x; ni += v.y; }
  o1 = b2_block1(x1, x2, z0r, z0i);
  o2 = b2_block2(g, x1, x2, nr, ni, K[p], b2_damping<T>(g, i, j, k), z0r, z0i);
}

__device__ __forceinline__ double block_sum_nt(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NT / 64; ++w) t += sh[w];
  return t;
}

// NF = 1: one factor of the step, w_out = F_k(w).  NF = 2: two consecutive factors k and
// k + 1 in one pass, w_out = F_{k+1}(F_k(w)); block one of B is pointwise, so the
// intermediate x1' at a neighbour is formed from the input there (its Dirichlet ghosts stay
// zero), and a one-point halo of the input serves both factors; the intermediate x2' is
// needed at the point only.  Kind bits on the input: kFacResid (the residual partials of
// w), kFacInF (the input is the right-hand side); on the output: kFacAdd (adds y1),
// kFacDual (a second output).
//
// z-marching: a workgroup of PTX x PTY threads takes tiles of PTX x PTY columns by PCZ
// planes (a grid-stride loop over the tiles of its system, so the residual partials keep
// the single factor's layout); each thread carries x1 and x2 of planes k - 1, k and k + 1
// of its column in registers and gathers only the in-plane neighbours through the cache.
// With a grid width that is a multiple of 8 the workgroups of one XCD (blockIdx.x % 8)
// sweep one contiguous eighth of the tiles.
constexpr int PTX = 64, PTY = NT / PTX, PCZ = 32;

template <typename T>
struct Pt2 {
  Cx<T> a, b;  // x1, x2 at a point
};

// Waves per SIMD asked of the compiler: 8 (64 VGPRs) for the complex64 kinds that fit
// without spilling (single factors; the middle pairs and the first pair of step one), else
// its own choice.
template <typename T, int KIND, int NF>
constexpr int b2_zm_waves() {
  return (sizeof(T) == 4 && (NF == 1 || (KIND & (kFacResid | kFacAdd | kFacDual)) == 0)) ? 8 : 1;
}

template <typename T, int KIND, int NF>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(b2_zm_waves<T, KIND, NF>()))) void b2_zm_kernel(
    GridDesc g, const T* __restrict__ K, B2Args<typename Vec2<T>::t> a) {
  static_assert(NF == 1 || NF == 2, "one or two factors per pass");
  using T2 = typename Vec2<T>::t;
  constexpr bool RESID = (KIND & kFacResid) != 0, ADD = (KIND & kFacAdd) != 0, DUAL = (KIND & kFacDual) != 0,
                 INF = (KIND & kFacInF) != 0;
  __shared__ double sh[NT / 64];
  const int s = blockIdx.y;
  if (a.active[s] == 0) return;  // block-uniform: stopped systems are skipped
  const int pole = s / a.nrhs, r = s % a.nrhs;
  const size_t npt = (size_t)g.nx * g.ny * g.nz, n2 = 2 * npt;
  // the second coefficient only for a pair: k + 1 may lie past the pole's entries otherwise
  const FactorCoef f1 = a.coef[(size_t)pole * a.cstride + a.k];
  const FactorCoef f2 = NF == 2 ? a.coef[(size_t)pole * a.cstride + a.k + 1] : f1;
  const PoleDev pd = a.poles[pole];
  const T a1r = (T)f1.a_re, a1i = (T)f1.a_im, b1r = (T)f1.b_re, b1i = (T)f1.b_im;
  const T a2r = (T)f2.a_re, a2i = (T)f2.a_im, b2r = (T)f2.b_re, b2i = (T)f2.b_im;
  const T z0r = (T)pd.z0_re, z0i = (T)pd.z0_im;
  const T2* __restrict__ X = INF ? a.win + (size_t)r * n2 : a.win + (size_t)s * n2;
  const T2* __restrict__ F = a.f + (size_t)r * n2;
  const T2* __restrict__ Y1 = a.y1 + (size_t)s * n2;
  T2* __restrict__ O = a.wout + (size_t)s * n2;
  T2* __restrict__ O2 = DUAL ? a.wout2 + (size_t)s * n2 : nullptr;
  const size_t sy = (size_t)g.nx, sz = (size_t)g.nx * g.ny;
  const int gx = (g.nx + PTX - 1) / PTX, gy = (g.ny + PTY - 1) / PTY, gz = (g.nz + PCZ - 1) / PCZ;
  const int ntile = gx * gy * gz;
  const int nsl = gridDim.x % 8 == 0 ? 8 : 1;
  const int tps = (ntile + nsl - 1) / nsl;
  const int t_lo = (int)(blockIdx.x % nsl) * tps, t_hi = min(ntile, t_lo + tps);
  const int tx = threadIdx.x % PTX, ty = threadIdx.x / PTX;
  const Pt2<T> zero{Cx<T>{(T)0, (T)0}, Cx<T>{(T)0, (T)0}};
  auto ld2 = [&](size_t q) { return Pt2<T>{ldc<T>(X, q), ldc<T>(X, npt + q)}; };
  // the first factor's x1' at a point from x1, x2 there (zero at a ghost)
  auto fac1 = [&](const Pt2<T>& u) { return b2_fac(a1r, a1i, b1r, b1i, b2_block1(u.a, u.b, z0r, z0i), u.a); };
  double acc = 0.0;
  for (int t = t_lo + (int)(blockIdx.x / nsl); t < t_hi; t += (int)(gridDim.x / nsl)) {
    const int i = (t % gx) * PTX + tx, j = ((t / gx) % gy) * PTY + ty, zc = t / (gx * gy);
    const int zb = zc * PCZ, ze = min(g.nz, zb + PCZ);
    if (i >= g.nx || j >= g.ny) continue;  // no barrier inside the tile loop
    const size_t col = (size_t)i + sy * (size_t)j;
    Pt2<T> xm = zb > 0 ? ld2(col + sz * (size_t)(zb - 1)) : zero;
    Pt2<T> xc = ld2(col + sz * (size_t)zb);
    for (int k = zb; k < ze; ++k) {
      const size_t p = col + sz * (size_t)k;
      const Pt2<T> xp = k + 1 < g.nz ? ld2(p + sz) : zero;
      // neighbour sums of x1 (first factor) and of the first factor's x1' (second factor),
      // in the order -x, +x, -y, +y, -z, +z
      T nr = (T)0, ni = (T)0, mr = (T)0, mi = (T)0;
      auto add = [&](const Pt2<T>& u) {
        nr += u.a.x;
        ni += u.a.y;
        if constexpr (NF == 2) {
          const Cx<T> v = fac1(u);
          mr += v.x;
          mi += v.y;
        }
      };
      if (i > 0) add(ld2(p - 1));
      if (i + 1 < g.nx) add(ld2(p + 1));
      if (j > 0) add(ld2(p - sy));
      if (j + 1 < g.ny) add(ld2(p + sy));
      if (k > 0) add(xm);
      if (k + 1 < g.nz) add(xp);
      const Cx<T> x1 = xc.a, x2 = xc.b;
      const T kap = K[p], dmp = b2_damping<T>(g, i, j, k);
      const Cx<T> o1 = b2_block1(x1, x2, z0r, z0i), o2 = b2_block2(g, x1, x2, nr, ni, kap, dmp, z0r, z0i);
      // the first factor at the point (t1, t2), then the second (a pair)
      const Cx<T> t1 = b2_fac(a1r, a1i, b1r, b1i, o1, x1), t2 = b2_fac(a1r, a1i, b1r, b1i, o2, x2);
      Cx<T> c1 = t1, c2 = t2;
      if constexpr (NF == 2) {
        const Cx<T> p1 = b2_block1(t1, t2, z0r, z0i), p2 = b2_block2(g, t1, t2, mr, mi, kap, dmp, z0r, z0i);
        c1 = b2_fac(a2r, a2i, b2r, b2i, p1, t1);
        c2 = b2_fac(a2r, a2i, b2r, b2i, p2, t2);
      }
      T2 w1, w2;
      w1.x = c1.x;
      w1.y = c1.y;
      w2.x = c2.x;
      w2.y = c2.y;
      if constexpr (ADD) {
        const T2 e1 = Y1[p], e2 = Y1[npt + p];
        w1.x += e1.x;
        w1.y += e1.y;
        w2.x += e2.x;
        w2.y += e2.y;
      }
      O[p] = w1;
      O[npt + p] = w2;
      if constexpr (DUAL) {
        O2[p] = w1;
        O2[npt + p] = w2;
      }
      if constexpr (RESID) {
        const double zr = pd.zz_re, zi = pd.zz_im;
        const T2 g1 = F[p], g2 = F[npt + p];
        const double r1x = (double)g1.x - (double)o1.x + zr * (double)x1.x - zi * (double)x1.y;
        const double r1y = (double)g1.y - (double)o1.y + zr * (double)x1.y + zi * (double)x1.x;
        const double r2x = (double)g2.x - (double)o2.x + zr * (double)x2.x - zi * (double)x2.y;
        const double r2y = (double)g2.y - (double)o2.y + zr * (double)x2.y + zi * (double)x2.x;
        acc += r1x * r1x + r1y * r1y + r2x * r2x + r2y * r2y;
      }
      xm = xc;
      xc = xp;
    }
  }
  if constexpr (RESID) {
    const double t = block_sum_nt(acc, sh);
    if (threadIdx.x == 0) a.partial[(size_t)s * gridDim.x + blockIdx.x] = t;
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void b2_apply_kernel(GridDesc g, const T* __restrict__ K,
                                                      const typename Vec2<T>::t* __restrict__ x,
                                                      typename Vec2<T>::t* __restrict__ y, double sr, double si) {
  using T2 = typename Vec2<T>::t;
  const size_t npt = (size_t)g.nx * g.ny * g.nz, n2 = 2 * npt;
  const T2* __restrict__ X = x + (size_t)blockIdx.y * n2;
  T2* __restrict__ Y = y + (size_t)blockIdx.y * n2;
  const size_t stride = (size_t)gridDim.x * NT;
  for (size_t p = (size_t)blockIdx.x * NT + threadIdx.x; p < npt; p += stride) {
    const int i = (int)(p % g.nx), j = (int)((p / g.nx) % g.ny), k = (int)(p / ((size_t)g.nx * g.ny));
    Cx<T> o1, o2, x1, x2;
    b2_point<T, T2>(g, K, X, npt, p, i, j, k, (T)sr, (T)si, o1, o2, x1, x2);
    T2 w1, w2;
    w1.x = o1.x;
    w1.y = o1.y;
    w2.x = o2.x;
    w2.y = o2.y;
    Y[p] = w1;
    Y[npt + p] = w2;
  }
}

// Alg. 1 step 3 on B: per right-hand side r (grid y), partial sums of (B w)^H f (real and
// imaginary parts) and |B w|^2 over both blocks; partial[(3 r + c) * gridDim.x + block].
template <typename T>
__global__ __launch_bounds__(NT) void b2_dstep_kernel(GridDesc g, const T* __restrict__ K,
                                                      const typename Vec2<T>::t* __restrict__ w,
                                                      const typename Vec2<T>::t* __restrict__ f,
                                                      double* __restrict__ partial) {
  using T2 = typename Vec2<T>::t;
  __shared__ double sh[NT / 64];
  const size_t npt = (size_t)g.nx * g.ny * g.nz, n2 = 2 * npt;
  const int r = blockIdx.y;
  const T2* __restrict__ W = w + (size_t)r * n2;
  const T2* __restrict__ F = f + (size_t)r * n2;
  double nr = 0.0, ni = 0.0, den = 0.0;
  const size_t stride = (size_t)gridDim.x * NT;
  for (size_t p = (size_t)blockIdx.x * NT + threadIdx.x; p < npt; p += stride) {
    const int i = (int)(p % g.nx), j = (int)((p / g.nx) % g.ny), k = (int)(p / ((size_t)g.nx * g.ny));
    Cx<T> o1, o2, x1, x2;
    b2_point<T, T2>(g, K, W, npt, p, i, j, k, (T)0, (T)0, o1, o2, x1, x2);
    const T2 f1 = F[p], f2 = F[npt + p];
    nr += (double)o1.x * f1.x + (double)o1.y * f1.y + (double)o2.x * f2.x + (double)o2.y * f2.y;
    ni += (double)o1.x * f1.y - (double)o1.y * f1.x + (double)o2.x * f2.y - (double)o2.y * f2.x;
    den += (double)o1.x * o1.x + (double)o1.y * o1.y + (double)o2.x * o2.x + (double)o2.y * o2.y;
  }
  const double a = block_sum_nt(nr, sh);
  __syncthreads();
  const double b = block_sum_nt(ni, sh);
  __syncthreads();
  const double c = block_sum_nt(den, sh);
  if (threadIdx.x == 0) {
    partial[(size_t)(3 * r) * gridDim.x + blockIdx.x] = a;
    partial[(size_t)(3 * r + 1) * gridDim.x + blockIdx.x] = b;
    partial[(size_t)(3 * r + 2) * gridDim.x + blockIdx.x] = c;
  }
}

// FP64 true residual of the double-size system: res = b - B u, partial sums of |res|^2
// (one per block).
__global__ __launch_bounds__(NT) void b2_residual64_kernel(GridDesc g, const double* __restrict__ K,
                                                           const double2* __restrict__ b,
                                                           const double2* __restrict__ u,
                                                           double2* __restrict__ res, double* __restrict__ partial) {
  __shared__ double sh[NT / 64];
  const size_t npt = (size_t)g.nx * g.ny * g.nz;
  double acc = 0.0;
  const size_t stride = (size_t)gridDim.x * NT;
  for (size_t p = (size_t)blockIdx.x * NT + threadIdx.x; p < npt; p += stride) {
    const int i = (int)(p % g.nx), j = (int)((p / g.nx) % g.ny), k = (int)(p / ((size_t)g.nx * g.ny));
    Cx<double> o1, o2, x1, x2;
    b2_point<double, double2>(g, K, u, npt, p, i, j, k, 0.0, 0.0, o1, o2, x1, x2);
    const double2 b1 = b[p], b2 = b[npt + p];
    const double2 r1 = make_double2(b1.x - o1.x, b1.y - o1.y), r2 = make_double2(b2.x - o2.x, b2.y - o2.y);
    res[p] = r1;
    res[npt + p] = r2;
    acc += r1.x * r1.x + r1.y * r1.y + r2.x * r2.x + r2.y * r2.y;
  }
  const double t = block_sum_nt(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

template <typename T, int KIND>
void launch_kind(hipStream_t st, const GridDesc& g, const T* K, int nsys, int nblk,
                 const B2Args<typename Vec2<T>::t>& a) {
  hipLaunchKernelGGL((b2_zm_kernel<T, KIND, 1>), dim3((unsigned)nblk, (unsigned)nsys), dim3(NT), 0, st, g, K, a);
}

template <typename T, int KIND>
void launch_pair_kind(hipStream_t st, const GridDesc& g, const T* K, int nsys, int nblk,
                      const B2Args<typename Vec2<T>::t>& a) {
  hipLaunchKernelGGL((b2_zm_kernel<T, KIND, 2>), dim3((unsigned)nblk, (unsigned)nsys), dim3(NT), 0, st, g, K, a);
}

}  // namespace

int b2_blocks(const GridDesc& g) {
  const size_t npt = (size_t)g.nx * g.ny * g.nz;
  size_t b = (npt + NT - 1) / NT;
  if (b > 1024) b = 1024;
  return (int)b;
}

template <typename T2>
bool launch_b2_factor(hipStream_t st, const GridDesc& g, const void* K, int kind, int nsys,
                      const B2Args<T2>& a) {
  using T = typename Scal<T2>::t;
  const T* k = (const T*)K;
  const int nb = b2_blocks(g);
  if (nsys <= 0) return true;
  switch (kind) {
    case 0: launch_kind<T, 0>(st, g, k, nsys, nb, a); return true;
    case kFacResid: launch_kind<T, kFacResid>(st, g, k, nsys, nb, a); return true;
    case kFacAdd: launch_kind<T, kFacAdd>(st, g, k, nsys, nb, a); return true;
    case kFacResid | kFacAdd: launch_kind<T, kFacResid | kFacAdd>(st, g, k, nsys, nb, a); return true;
    case kFacInF: launch_kind<T, kFacInF>(st, g, k, nsys, nb, a); return true;
    case kFacInF | kFacDual: launch_kind<T, kFacInF | kFacDual>(st, g, k, nsys, nb, a); return true;
    case kFacDual: launch_kind<T, kFacDual>(st, g, k, nsys, nb, a); return true;
    default: return false;
  }
}
template bool launch_b2_factor<float2>(hipStream_t, const GridDesc&, const void*, int, int, const B2Args<float2>&);
template bool launch_b2_factor<double2>(hipStream_t, const GridDesc&, const void*, int, int,
                                        const B2Args<double2>&);

template <typename T2>
bool launch_b2_pair(hipStream_t st, const GridDesc& g, const void* K, int kind, int nsys, const B2Args<T2>& a) {
  using T = typename Scal<T2>::t;
  const T* k = (const T*)K;
  const int nb = b2_blocks(g);
  if (nsys <= 0) return true;
  switch (kind) {
    case 0: launch_pair_kind<T, 0>(st, g, k, nsys, nb, a); return true;
    case kFacResid: launch_pair_kind<T, kFacResid>(st, g, k, nsys, nb, a); return true;
    case kFacAdd: launch_pair_kind<T, kFacAdd>(st, g, k, nsys, nb, a); return true;
    case kFacResid | kFacAdd: launch_pair_kind<T, kFacResid | kFacAdd>(st, g, k, nsys, nb, a); return true;
    case kFacInF: launch_pair_kind<T, kFacInF>(st, g, k, nsys, nb, a); return true;
    case kFacDual: launch_pair_kind<T, kFacDual>(st, g, k, nsys, nb, a); return true;
    case kFacInF | kFacDual: launch_pair_kind<T, kFacInF | kFacDual>(st, g, k, nsys, nb, a); return true;
    default: return false;
  }
}
template bool launch_b2_pair<float2>(hipStream_t, const GridDesc&, const void*, int, int, const B2Args<float2>&);
template bool launch_b2_pair<double2>(hipStream_t, const GridDesc&, const void*, int, int, const B2Args<double2>&);

template <typename T2>
void launch_b2_apply(hipStream_t st, const GridDesc& g, const void* K, int nvec, const T2* x, T2* y, double sr,
                     double si) {
  using T = typename Scal<T2>::t;
  if (nvec <= 0) return;
  hipLaunchKernelGGL(b2_apply_kernel<T>, dim3((unsigned)b2_blocks(g), (unsigned)nvec), dim3(NT), 0, st, g,
                     (const T*)K, x, y, sr, si);
}
template void launch_b2_apply<float2>(hipStream_t, const GridDesc&, const void*, int, const float2*, float2*,
                                      double, double);
template void launch_b2_apply<double2>(hipStream_t, const GridDesc&, const void*, int, const double2*, double2*,
                                       double, double);

template <typename T2>
void launch_b2_dstep(hipStream_t st, const GridDesc& g, const void* K, int nrhs, const T2* w, const T2* f,
                     double* partial) {
  using T = typename Scal<T2>::t;
  if (nrhs <= 0) return;
  hipLaunchKernelGGL(b2_dstep_kernel<T>, dim3((unsigned)b2_blocks(g), (unsigned)nrhs), dim3(NT), 0, st, g,
                     (const T*)K, w, f, partial);
}
template void launch_b2_dstep<float2>(hipStream_t, const GridDesc&, const void*, int, const float2*, const float2*,
                                      double*);
template void launch_b2_dstep<double2>(hipStream_t, const GridDesc&, const void*, int, const double2*,
                                       const double2*, double*);

void launch_b2_residual64(hipStream_t st, const GridDesc& g, const double* K, const double2* b, const double2* u,
                          double2* res, double* partial, int nblk) {
  hipLaunchKernelGGL(b2_residual64_kernel, dim3((unsigned)nblk), dim3(NT), 0, st, g, K, b, u, res, partial);
}

}  // namespace hfci
