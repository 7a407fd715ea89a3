// Kernels of the Fourier-spectral operator (Sec. 7.1, eq. eig-Laplacian-spectral):
// A = S - kappa - i D with S = F^H Lambda F on a periodic grid.  The FFTs are library
// transforms (spectral.cpp); these kernels are the diagonal Lambda between them and the
// pointwise epilogues that turn S w into a factor of the fixed-point step, a product
// with A - shift, the step-size partials and the FP64 residual.
#include <cmath>

#include "kernels.h"

namespace hfci {
namespace {

constexpr int NT = 256;

template <typename T> struct Vec2s;
template <> struct Vec2s<float> { using t = float2; };
template <> struct Vec2s<double> { using t = double2; };
template <typename T2> struct Scals;
template <> struct Scals<float2> { using t = float; };
template <> struct Scals<double2> { using t = double; };

__device__ __forceinline__ int layer_d(int i, int n, int L) { return max(0, L - min(i, n - 1 - i)); }

// grid indices of point p (x fastest) and its damping D_p = damp_scale * depth^2
__device__ __forceinline__ void point_of(const GridDesc& g, size_t p, int& i, int& j, int& k, double& dmp) {
  i = (int)(p % g.nx);
  j = (int)((p / g.nx) % g.ny);
  k = (int)(p / ((size_t)g.nx * g.ny));
  const int d = max(max(layer_d(i, g.nx, g.damp_cells), layer_d(j, g.ny, g.damp_cells)),
                    layer_d(k, g.nz, g.damp_cells));
  dmp = (double)(d * d) * g.damp_scale;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
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

// c_v[p] *= lambda_p / N for every vector v (grid y): lambda of the Fourier mode of p in FFT
// order, s * sum_j (2 pi min(m_j, N_j - m_j) / (N_j h))^2; 1/N normalises the inverse FFT
template <typename T2>
__global__ __launch_bounds__(NT) void spec_scale_kernel(T2* __restrict__ c, GridDesc g, double s, double h) {
  const size_t npt = (size_t)g.nx * g.ny * g.nz;
  T2* __restrict__ C = c + (size_t)blockIdx.y * npt;
  const double inv_n = 1.0 / (double)npt;
  const double kx = 2.0 * M_PI / (g.nx * h), ky = 2.0 * M_PI / (g.ny * h), kz = 2.0 * M_PI / (g.nz * h);
  const size_t stride = (size_t)gridDim.x * NT;
  for (size_t p = (size_t)blockIdx.x * NT + threadIdx.x; p < npt; p += stride) {
    const int i = (int)(p % g.nx), j = (int)((p / g.nx) % g.ny), k = (int)(p / ((size_t)g.nx * g.ny));
    const double mx = kx * min(i, g.nx - i), my = ky * min(j, g.ny - j), mz = kz * min(k, g.nz - k);
    const double f = s * (mx * mx + my * my + mz * mz) * inv_n;
    T2 v = C[p];
    v.x = (decltype(v.x))(v.x * f);
    v.y = (decltype(v.y))(v.y * f);
    C[p] = v;
  }
}

// (A - z0) w at p from S w: sw - (kappa + z0) w - i D w
template <typename T, typename T2>
__device__ __forceinline__ void spec_point(T2 w, T2 sw, T kap, T dmp, T z0r, T z0i, T& ox, T& oy) {
  const T dr = kap + z0r;
  ox = sw.x - (dr * w.x - z0i * w.y) + dmp * w.y;
  oy = sw.y - (dr * w.y + z0i * w.x) - dmp * w.x;
}

// slot: null when S w of system s sits at a.sw + s n (indexed as the inputs), else the
// batch slot of each system's S w (a gathered batch; -1 for a system outside it)
template <typename T, int KIND>
__global__ __launch_bounds__(NT) void spec_factor_kernel(GridDesc g, const T* __restrict__ K,
                                                         SpecArgs<typename Vec2s<T>::t> a,
                                                         const int* __restrict__ slot) {
  using T2 = typename Vec2s<T>::t;
  constexpr bool RESID = (KIND & kFacResid) != 0, ADD = (KIND & kFacAdd) != 0, DUAL = (KIND & kFacDual) != 0,
                 INF = (KIND & kFacInF) != 0;
  __shared__ double sh[NT / 64];
  const int s = blockIdx.y;
  if (a.active[s] == 0) return;  // block-uniform
  const int pole = s / a.nrhs, r = s % a.nrhs;
  const size_t npt = (size_t)g.nx * g.ny * g.nz;
  const FactorCoef cf = a.coef[(size_t)pole * a.cstride + a.k];
  const PoleDev pd = a.poles[pole];
  const T car = (T)cf.a_re, cai = (T)cf.a_im, cbr = (T)cf.b_re, cbi = (T)cf.b_im;
  const T z0r = (T)pd.z0_re, z0i = (T)pd.z0_im;
  const size_t vi = INF ? (size_t)r * npt : (size_t)s * npt;
  const int sl = slot != nullptr && !INF ? slot[s] : 0;
  if (sl < 0) return;  // block-uniform: not in the gathered batch
  const T2* __restrict__ W = a.win + vi;
  const T2* __restrict__ SW = slot != nullptr && !INF ? a.sw + (size_t)sl * npt : a.sw + vi;
  const T2* __restrict__ F = a.f + (size_t)r * npt;
  const T2* __restrict__ Y1 = a.y1 + (size_t)s * npt;
  T2* __restrict__ O = a.wout + (size_t)s * npt;
  T2* __restrict__ O2 = DUAL ? a.wout2 + (size_t)s * npt : nullptr;
  double acc = 0.0;
  const size_t stride = (size_t)gridDim.x * NT;
  for (size_t p = (size_t)blockIdx.x * NT + threadIdx.x; p < npt; p += stride) {
    int i, j, k;
    double dm;
    point_of(g, p, i, j, k, dm);
    const T2 w = W[p], sw = SW[p];
    T ox, oy;
    spec_point<T, T2>(w, sw, K[p], (T)dm, z0r, z0i, ox, oy);
    T2 o;
    o.x = car * ox - cai * oy + cbr * w.x - cbi * w.y;
    o.y = car * oy + cai * ox + cbr * w.y + cbi * w.x;
    if constexpr (ADD) {
      const T2 v = Y1[p];
      o.x += v.x;
      o.y += v.y;
    }
    O[p] = o;
    if constexpr (DUAL) O2[p] = o;
    if constexpr (RESID) {
      // g - (A - z) y = g - (A - z0) y + (z - z0) y, in FP64
      const T2 gv = F[p];
      const double rx = (double)gv.x - (double)ox + pd.zz_re * (double)w.x - pd.zz_im * (double)w.y;
      const double ry = (double)gv.y - (double)oy + pd.zz_re * (double)w.y + pd.zz_im * (double)w.x;
      acc += rx * rx + ry * ry;
    }
  }
  if constexpr (RESID) {
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) a.partial[(size_t)s * gridDim.x + blockIdx.x] = t;
  }
}

// y_v = (A - shift) x_v from sx_v = S x_v (y may alias sx)
template <typename T>
__global__ __launch_bounds__(NT) void spec_apply_kernel(GridDesc g, const T* __restrict__ K,
                                                        const typename Vec2s<T>::t* __restrict__ x,
                                                        const typename Vec2s<T>::t* sx, typename Vec2s<T>::t* y,
                                                        double sr, double si) {
  using T2 = typename Vec2s<T>::t;
  const size_t npt = (size_t)g.nx * g.ny * g.nz, o = (size_t)blockIdx.y * npt;
  const size_t stride = (size_t)gridDim.x * NT;
  for (size_t p = (size_t)blockIdx.x * NT + threadIdx.x; p < npt; p += stride) {
    int i, j, k;
    double dm;
    point_of(g, p, i, j, k, dm);
    T ox, oy;
    spec_point<T, T2>(x[o + p], sx[o + p], K[p], (T)dm, (T)sr, (T)si, ox, oy);
    T2 v;
    v.x = ox;
    v.y = oy;
    y[o + p] = v;
  }
}

// Alg. 1 step 3: per rhs (grid y) partial sums of (A w)^H f and |A w|^2 from sw = S w;
// partial[(3 r + c) * gridDim.x + block]
template <typename T>
__global__ __launch_bounds__(NT) void spec_dstep_kernel(GridDesc g, const T* __restrict__ K,
                                                        const typename Vec2s<T>::t* __restrict__ w,
                                                        const typename Vec2s<T>::t* __restrict__ sw,
                                                        const typename Vec2s<T>::t* __restrict__ f,
                                                        double* __restrict__ partial) {
  using T2 = typename Vec2s<T>::t;
  __shared__ double sh[NT / 64];
  const size_t npt = (size_t)g.nx * g.ny * g.nz, o = (size_t)blockIdx.y * npt;
  double nr = 0.0, ni = 0.0, den = 0.0;
  const size_t stride = (size_t)gridDim.x * NT;
  for (size_t p = (size_t)blockIdx.x * NT + threadIdx.x; p < npt; p += stride) {
    int i, j, k;
    double dm;
    point_of(g, p, i, j, k, dm);
    T ax, ay;
    spec_point<T, T2>(w[o + p], sw[o + p], K[p], (T)dm, (T)0, (T)0, ax, ay);
    const T2 fv = f[o + p];
    nr += (double)ax * fv.x + (double)ay * fv.y;
    ni += (double)ax * fv.y - (double)ay * fv.x;
    den += (double)ax * ax + (double)ay * ay;
  }
  const double a = block_sum(nr, sh);
  __syncthreads();
  const double b = block_sum(ni, sh);
  __syncthreads();
  const double c = block_sum(den, sh);
  if (threadIdx.x == 0) {
    const int r = blockIdx.y;
    partial[(size_t)(3 * r) * gridDim.x + blockIdx.x] = a;
    partial[(size_t)(3 * r + 1) * gridDim.x + blockIdx.x] = b;
    partial[(size_t)(3 * r + 2) * gridDim.x + blockIdx.x] = c;
  }
}

// FP64 residual res = b - A u from su = S u (res may alias su), partial sums of |res|^2
__global__ __launch_bounds__(NT) void spec_residual64_kernel(GridDesc g, const double* __restrict__ K,
                                                             const double2* __restrict__ b,
                                                             const double2* __restrict__ u, const double2* su,
                                                             double2* res, double* __restrict__ partial) {
  __shared__ double sh[NT / 64];
  const size_t npt = (size_t)g.nx * g.ny * g.nz;
  double acc = 0.0;
  const size_t stride = (size_t)gridDim.x * NT;
  for (size_t p = (size_t)blockIdx.x * NT + threadIdx.x; p < npt; p += stride) {
    int i, j, k;
    double dm;
    point_of(g, p, i, j, k, dm);
    double ax, ay;
    spec_point<double, double2>(u[p], su[p], K[p], dm, 0.0, 0.0, ax, ay);
    const double2 bv = b[p];
    const double2 rv = make_double2(bv.x - ax, bv.y - ay);
    res[p] = rv;
    acc += rv.x * rv.x + rv.y * rv.y;
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

template <typename T, int KIND>
void launch_skind(hipStream_t st, const GridDesc& g, const T* K, int nsys, const SpecArgs<typename Vec2s<T>::t>& a,
                  const int* slot) {
  hipLaunchKernelGGL((spec_factor_kernel<T, KIND>), dim3((unsigned)spec_blocks(g), (unsigned)nsys), dim3(NT), 0, st,
                     g, K, a, slot);
}

// The batch of the systems still iterating: slot_sys[v] for v < nvec is the v-th active
// system in index order (-1 past the last), sys_slot[s] the slot of system s (-1 for a
// stopped system or one past nvec slots).  One thread; nsys is at most a few thousand.
__global__ void spec_slots_kernel(const int* __restrict__ active, int nsys, int nvec, int* __restrict__ slot_sys,
                                  int* __restrict__ sys_slot) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int v = 0;
  for (int s = 0; s < nsys; ++s) {
    if (active[s] != 0 && v < nvec) {
      slot_sys[v] = s;
      sys_slot[s] = v++;
    } else {
      sys_slot[s] = -1;
    }
  }
  for (; v < nvec; ++v) slot_sys[v] = -1;
}

// out_v = in_{slot_sys[v]} for v < nvec (grid y), zero for a slot past the last system
template <typename T2>
__global__ __launch_bounds__(NT) void spec_gather_kernel(const T2* __restrict__ in, T2* __restrict__ out,
                                                         const int* __restrict__ slot_sys, size_t n) {
  const int v = blockIdx.y, sys = slot_sys[v];
  T2* __restrict__ O = out + (size_t)v * n;
  const T2* __restrict__ I = in + (size_t)(sys < 0 ? 0 : sys) * n;
  const size_t stride = (size_t)gridDim.x * NT;
  for (size_t p = (size_t)blockIdx.x * NT + threadIdx.x; p < n; p += stride) {
    T2 x;
    if (sys >= 0) {
      x = I[p];
    } else {
      x.x = 0;
      x.y = 0;
    }
    O[p] = x;
  }
}

}  // namespace

int spec_blocks(const GridDesc& g) {
  const size_t npt = (size_t)g.nx * g.ny * g.nz;
  size_t b = (npt + NT - 1) / NT;
  if (b > 1024) b = 1024;
  return (int)b;
}

template <typename T2>
void launch_spec_scale(hipStream_t st, T2* c, int nvec, const GridDesc& g, double s, double h) {
  if (nvec > 0)
    hipLaunchKernelGGL(spec_scale_kernel<T2>, dim3((unsigned)spec_blocks(g), (unsigned)nvec), dim3(NT), 0, st, c, g,
                       s, h);
}
template void launch_spec_scale<float2>(hipStream_t, float2*, int, const GridDesc&, double, double);
template void launch_spec_scale<double2>(hipStream_t, double2*, int, const GridDesc&, double, double);

template <typename T2>
bool launch_spec_factor_slots(hipStream_t st, const GridDesc& g, const void* K, int kind, int nsys,
                              const SpecArgs<T2>& a, const int* slot) {
  using T = typename Scals<T2>::t;
  const T* k = (const T*)K;
  if (nsys <= 0) return true;
  switch (kind) {
    case 0: launch_skind<T, 0>(st, g, k, nsys, a, slot); return true;
    case kFacResid: launch_skind<T, kFacResid>(st, g, k, nsys, a, slot); return true;
    case kFacAdd: launch_skind<T, kFacAdd>(st, g, k, nsys, a, slot); return true;
    case kFacResid | kFacAdd: launch_skind<T, kFacResid | kFacAdd>(st, g, k, nsys, a, slot); return true;
    case kFacInF: launch_skind<T, kFacInF>(st, g, k, nsys, a, slot); return true;
    case kFacInF | kFacDual: launch_skind<T, kFacInF | kFacDual>(st, g, k, nsys, a, slot); return true;
    case kFacDual: launch_skind<T, kFacDual>(st, g, k, nsys, a, slot); return true;
    default: return false;
  }
}
template bool launch_spec_factor_slots<float2>(hipStream_t, const GridDesc&, const void*, int, int,
                                               const SpecArgs<float2>&, const int*);
template bool launch_spec_factor_slots<double2>(hipStream_t, const GridDesc&, const void*, int, int,
                                                const SpecArgs<double2>&, const int*);

template <typename T2>
bool launch_spec_factor(hipStream_t st, const GridDesc& g, const void* K, int kind, int nsys, const SpecArgs<T2>& a) {
  return launch_spec_factor_slots<T2>(st, g, K, kind, nsys, a, nullptr);
}
template bool launch_spec_factor<float2>(hipStream_t, const GridDesc&, const void*, int, int,
                                         const SpecArgs<float2>&);
template bool launch_spec_factor<double2>(hipStream_t, const GridDesc&, const void*, int, int,
                                          const SpecArgs<double2>&);

void launch_spec_slots(hipStream_t st, const int* active, int nsys, int nvec, int* slot_sys, int* sys_slot) {
  hipLaunchKernelGGL(spec_slots_kernel, dim3(1), dim3(64), 0, st, active, nsys, nvec, slot_sys, sys_slot);
}

template <typename T2>
void launch_spec_gather(hipStream_t st, const GridDesc& g, const T2* in, T2* out, const int* slot_sys, int nvec) {
  if (nvec <= 0) return;
  const size_t n = (size_t)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL(spec_gather_kernel<T2>, dim3((unsigned)spec_blocks(g), (unsigned)nvec), dim3(NT), 0, st, in, out,
                     slot_sys, n);
}
template void launch_spec_gather<float2>(hipStream_t, const GridDesc&, const float2*, float2*, const int*, int);
template void launch_spec_gather<double2>(hipStream_t, const GridDesc&, const double2*, double2*, const int*, int);

template <typename T2>
void launch_spec_apply(hipStream_t st, const GridDesc& g, const void* K, int nvec, const T2* x, const T2* sx, T2* y,
                       double sr, double si) {
  using T = typename Scals<T2>::t;
  if (nvec > 0)
    hipLaunchKernelGGL(spec_apply_kernel<T>, dim3((unsigned)spec_blocks(g), (unsigned)nvec), dim3(NT), 0, st, g,
                       (const T*)K, x, sx, y, sr, si);
}
template void launch_spec_apply<float2>(hipStream_t, const GridDesc&, const void*, int, const float2*, const float2*,
                                        float2*, double, double);
template void launch_spec_apply<double2>(hipStream_t, const GridDesc&, const void*, int, const double2*,
                                         const double2*, double2*, double, double);

template <typename T2>
void launch_spec_dstep(hipStream_t st, const GridDesc& g, const void* K, int nrhs, const T2* w, const T2* sw,
                       const T2* f, double* partial) {
  using T = typename Scals<T2>::t;
  if (nrhs > 0)
    hipLaunchKernelGGL(spec_dstep_kernel<T>, dim3((unsigned)spec_blocks(g), (unsigned)nrhs), dim3(NT), 0, st, g,
                       (const T*)K, w, sw, f, partial);
}
template void launch_spec_dstep<float2>(hipStream_t, const GridDesc&, const void*, int, const float2*, const float2*,
                                        const float2*, double*);
template void launch_spec_dstep<double2>(hipStream_t, const GridDesc&, const void*, int, const double2*,
                                         const double2*, const double2*, double*);

void launch_spec_residual64(hipStream_t st, const GridDesc& g, const double* K, const double2* b, const double2* u,
                            const double2* su, double2* res, double* partial, int nblk) {
  hipLaunchKernelGGL(spec_residual64_kernel, dim3((unsigned)nblk), dim3(NT), 0, st, g, K, b, u, su, res, partial);
}

}  // namespace hfci
