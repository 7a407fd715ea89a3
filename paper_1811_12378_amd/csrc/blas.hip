// BLAS-1 kernels and deterministic reductions for FGMRES and the FCI combine (gfx950).
//
// Reductions are two-pass and order-fixed: a grid of blas_blocks(n) blocks writes one
// partial per block (wavefront shuffle tree, then 4 waves through LDS), and a second
// kernel sums the partials of each component in a fixed order.  No floating-point
// atomics, so FP64 results are bit-reproducible run to run.
#include <climits>

#include "kernels.h"

namespace hfci {
namespace {

constexpr int NT = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Sum over the block of NV values per thread; results valid in thread 0 (v[k]).
template <int NV>
__device__ __forceinline__ void block_sum_n(double (&v)[NV], double* sh) {
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) sh[wid * NV + k] = s;
  }
  __syncthreads();
  if (t == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = sh[k] + sh[NV + k] + sh[2 * NV + k] + sh[3 * NV + k];
  }
}

__global__ __launch_bounds__(NT) void reduce_kernel(const double* __restrict__ partial, int nblk,
                                                    double* __restrict__ out) {
  __shared__ double sh[4];
  const double* row = partial + (size_t)blockIdx.x * nblk;
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < nblk; i += NT) v[0] += row[i];
  block_sum_n<1>(v, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = v[0];
}

// Partial sums of conj(V_i) . w for the vectors of group blockIdx.y (NVMAX per group):
// each thread reads w once and each vector of its group once per point.  Accumulators
// are indexed only by compile-time constants (a runtime index would put them in scratch).
template <int NVMAX>
__global__ __launch_bounds__(NT) void multidot_kernel(const double2* __restrict__ V, int nv, size_t n,
                                                      size_t vstride, const double2* __restrict__ w,
                                                      double* __restrict__ partial) {
  __shared__ double sh[4 * 2 * NVMAX];
  const int i0 = blockIdx.y * NVMAX;
  const int ng = min(NVMAX, nv - i0);
  V += (size_t)i0 * vstride;
  partial += (size_t)2 * i0 * gridDim.x;
  double acc[2 * NVMAX];
#pragma unroll
  for (int k = 0; k < 2 * NVMAX; ++k) acc[k] = 0.0;
  const size_t stride = (size_t)gridDim.x * NT;
  for (size_t p = (size_t)blockIdx.x * NT + threadIdx.x; p < n; p += stride) {
    const double2 wv = w[p];
#pragma unroll
    for (int i = 0; i < NVMAX; ++i) {
      if (i < ng) {
        const double2 v = V[(size_t)i * vstride + p];
        acc[2 * i] += v.x * wv.x + v.y * wv.y;      // Re conj(v) w
        acc[2 * i + 1] += v.x * wv.y - v.y * wv.x;  // Im conj(v) w
      }
    }
  }
  block_sum_n<2 * NVMAX>(acc, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 2 * NVMAX; ++k)
      if (k < 2 * ng) partial[(size_t)k * gridDim.x + blockIdx.x] = acc[k];
  }
}

__global__ __launch_bounds__(NT) void multiaxpy_kernel(double2* __restrict__ w, const double2* __restrict__ V,
                                                       int nv, size_t n, size_t vstride,
                                                       const double* __restrict__ h,
                                                       double sign) {
  __shared__ double hs[2 * 64];
  if (threadIdx.x < 2 * nv) hs[threadIdx.x] = sign * h[threadIdx.x];
  __syncthreads();
  const size_t stride = (size_t)gridDim.x * NT;
  for (size_t p = (size_t)blockIdx.x * NT + threadIdx.x; p < n; p += stride) {
    double2 acc = w[p];
    for (int i = 0; i < nv; ++i) {
      const double2 v = V[(size_t)i * vstride + p];
      const double hr = hs[2 * i], hi = hs[2 * i + 1];
      acc.x += hr * v.x - hi * v.y;
      acc.y += hr * v.y + hi * v.x;
    }
    w[p] = acc;
  }
}

// The passes of CGS2 over the basis V[0..nv) (nv <= 4 * NQ):
//   partial sums of conj(V_i) . w                                           (DOT, !UPD)
//   w <- w + sign * sum_i h_i V_i, then partial sums of conj(V_i) . w      (DOT)
//   w <- w + sign * sum_i h_i V_i, then partial sums of |w|^2               (NORM)
// Each point belongs to a quad of four lanes; lane q holds the vectors i = 4j + q
// (j < NQ) of that point in registers, the quad sums the update through lane shuffles,
// so V is read once from HBM for both the update and the dot products.  Lanes past nv
// read a valid vector (V_{nv-1}) with a zero coefficient.  Partial row k (= 2i + c for
// DOT, 0 for NORM) of block b is at partial[k * gridDim.x + b], as for multidot.
template <int NQ, bool DOT, bool UPD = true>
__global__ __launch_bounds__(NT) void axpy_reduce_kernel(double2* __restrict__ w, const double2* __restrict__ V,
                                                         int nv, size_t n, size_t vstride,
                                                         const double* __restrict__ h, double sign,
                                                         double* __restrict__ partial) {
  constexpr int NA = DOT ? 2 * NQ : 1;
  __shared__ double hs[2 * 4 * NQ];
  __shared__ double sh[(NT / 64) * 4 * NA];
  if constexpr (UPD) {
    for (int t = threadIdx.x; t < 2 * 4 * NQ; t += NT) hs[t] = t < 2 * nv ? sign * h[t] : 0.0;
    __syncthreads();
  }
  const int q = threadIdx.x & 3;
  double acc[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc[k] = 0.0;
  const size_t pstride = (size_t)gridDim.x * (NT / 4);
  for (size_t p = (size_t)blockIdx.x * (NT / 4) + threadIdx.x / 4; p < n; p += pstride) {
    double2 v[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      const int i = min(4 * j + q, nv - 1);
      v[j] = V[(size_t)i * vstride + p];
    }
    const double2 wv = w[p];
    double2 wn = wv;
    if constexpr (UPD) {
      double sx = 0.0, sy = 0.0;
#pragma unroll
      for (int j = 0; j < NQ; ++j) {
        const double hr = hs[2 * (4 * j + q)], hi = hs[2 * (4 * j + q) + 1];
        sx += hr * v[j].x - hi * v[j].y;
        sy += hr * v[j].y + hi * v[j].x;
      }
      sx += __shfl_xor(sx, 1, 64);
      sy += __shfl_xor(sy, 1, 64);
      sx += __shfl_xor(sx, 2, 64);
      sy += __shfl_xor(sy, 2, 64);
      wn = make_double2(wv.x + sx, wv.y + sy);
      if (q == 0) w[p] = wn;
    }
    if constexpr (DOT) {
#pragma unroll
      for (int j = 0; j < NQ; ++j) {
        acc[2 * j] += v[j].x * wn.x + v[j].y * wn.y;      // Re conj(v) w
        acc[2 * j + 1] += v[j].x * wn.y - v[j].y * wn.x;  // Im conj(v) w
      }
    } else {
      if (q == 0) acc[0] += wn.x * wn.x + wn.y * wn.y;
    }
  }
  // lanes q, q + 4, ..., q + 60 of a wave hold the same vectors: sum them into lane q
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    double x = acc[k];
#pragma unroll
    for (int o = 32; o >= 4; o >>= 1) x += __shfl_down(x, o, 64);
    if (lane < 4) sh[(wid * 4 + lane) * NA + k] = x;
  }
  __syncthreads();
  if (DOT) {
    // thread t < 4 * NA: lane group q = t / NA, entry k = t % NA -> vector 4 (k / 2) + q
    const int t = threadIdx.x;
    if (t < 4 * NA) {
      const int qq = t / NA, k = t % NA;
      double x = 0.0;
#pragma unroll
      for (int w4 = 0; w4 < NT / 64; ++w4) x += sh[(w4 * 4 + qq) * NA + k];
      const int i = 4 * (k / 2) + qq;
      if (i < nv) partial[(size_t)(2 * i + (k & 1)) * gridDim.x + blockIdx.x] = x;
    }
  } else if (threadIdx.x == 0) {
    double x = 0.0;
#pragma unroll
    for (int w4 = 0; w4 < NT / 64; ++w4) x += sh[(w4 * 4) * NA];
    partial[blockIdx.x] = x;
  }
}

__global__ __launch_bounds__(NT) void diffnorm2_kernel(const double2* __restrict__ a, const double2* __restrict__ b,
                                                       size_t n, double* __restrict__ partial) {
  __shared__ double sh[4];
  double v[1] = {0.0};
  const size_t stride = (size_t)gridDim.x * NT;
  for (size_t p = (size_t)blockIdx.x * NT + threadIdx.x; p < n; p += stride) {
    const double2 x = a[p], y = b[p];
    const double dr = x.x - y.x, di = x.y - y.y;
    v[0] += dr * dr + di * di;
  }
  block_sum_n<1>(v, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

template <typename T2>
__global__ __launch_bounds__(NT) void norm2_kernel(const T2* __restrict__ x, size_t n,
                                                   double* __restrict__ partial) {
  __shared__ double sh[4];
  double v[1] = {0.0};
  const size_t stride = (size_t)gridDim.x * NT;
  for (size_t p = (size_t)blockIdx.x * NT + threadIdx.x; p < n; p += stride) {
    const T2 a = x[p];
    v[0] += (double)a.x * (double)a.x + (double)a.y * (double)a.y;
  }
  block_sum_n<1>(v, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

__global__ void scale_inv_kernel(double2* __restrict__ v, const double2* __restrict__ w, size_t n,
                                 const double* __restrict__ nrm2) {
  const double s = 1.0 / sqrt(nrm2[0]);
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const double2 a = w[p];
    v[p] = make_double2(a.x * s, a.y * s);
  }
}

__global__ void fill_zero_kernel(uint4* __restrict__ p, size_t n16) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void fill_zero_tail(unsigned char* __restrict__ p, size_t nb) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) p[i] = 0;
}

__global__ void copy_scaled64_kernel(double2* __restrict__ d, const double2* __restrict__ s, size_t n,
                                     double a) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const double2 v = s[p];
    d[p] = make_double2(a * v.x, a * v.y);
  }
}

__global__ void cvt64to32_kernel(float2* __restrict__ d, const double2* __restrict__ s, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const double2 v = s[p];
    d[p] = make_float2((float)v.x, (float)v.y);
  }
}

__global__ void cvt32to64_kernel(double2* __restrict__ d, const float2* __restrict__ s, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const float2 v = s[p];
    d[p] = make_double2((double)v.x, (double)v.y);
  }
}

template <typename T2> struct ScalOf;
template <> struct ScalOf<float2> { using t = float; };
template <> struct ScalOf<double2> { using t = double; };

// w_r (+)= sum_j c_j y_{j,r}; with steps given, system (j, r) reads y1 instead of y when it
// took at most one fixed-point step (its iterate was left in y1)
template <typename T2>
__global__ void combine_kernel(T2* __restrict__ w, const T2* __restrict__ y, const double* __restrict__ coef,
                               int npole, int nrhs, size_t n, int accumulate, const T2* __restrict__ y1,
                               const int* __restrict__ steps) {
  using T = typename ScalOf<T2>::t;
  const int r = blockIdx.y;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    double ar = 0.0, ai = 0.0;
    if (accumulate) {
      const T2 o = w[(size_t)r * n + p];
      ar = o.x;
      ai = o.y;
    }
    for (int j = 0; j < npole; ++j) {
      const size_t ls = (size_t)j * nrhs + r;
      const T2* src = (steps != nullptr && steps[ls] <= 1) ? y1 : y;
      const T2 v = src[ls * n + p];
      const double cr = coef[2 * j], ci = coef[2 * j + 1];
      ar += cr * (double)v.x - ci * (double)v.y;
      ai += cr * (double)v.y + ci * (double)v.x;
    }
    T2 o;
    o.x = (T)ar;
    o.y = (T)ai;
    w[(size_t)r * n + p] = o;
  }
}

template <typename T2>
__global__ void scale_out_kernel(double2* __restrict__ out, const T2* __restrict__ w,
                                 const double* __restrict__ d, size_t n) {
  const int r = blockIdx.y;
  const double dr = d[2 * r], di = d[2 * r + 1];
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
    const T2 v = w[(size_t)r * n + p];
    const double vr = v.x, vi = v.y;
    out[(size_t)r * n + p] = make_double2(dr * vr - di * vi, dr * vi + di * vr);
  }
}

// One block per system: sum its residual partials, then decide whether the
// fixed-point iteration continues (stopping rule of Table 4, or a fixed count).
__global__ __launch_bounds__(NT) void fp_check_kernel(const double* __restrict__ partial, int nblk,
                                                      int sys0, int nrhs, const double* __restrict__ fnorm2,
                                                      int fixed_steps, double inv_reduce2, int max_steps,
                                                      int* __restrict__ active, int* __restrict__ steps,
                                                      double* __restrict__ rnorm2) {
  __shared__ double sh[4];
  const int s = blockIdx.x;
  if (active[s] == 0) return;  // converged earlier: its partial was not written
  const double* row = partial + (size_t)s * nblk;
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < nblk; i += NT) v[0] += row[i];
  block_sum_n<1>(v, sh);
  if (threadIdx.x == 0) {
    const double r2 = v[0];
    rnorm2[s] = r2;
    const int r = (sys0 + s) % nrhs;
    int act;
    if (fixed_steps > 0)
      act = steps[s] < fixed_steps;
    else
      act = (r2 > fnorm2[r] * inv_reduce2) && (steps[s] < max_steps);
    if (!(r2 == r2) || r2 > 1e300) act = 0;  // NaN / overflow: stop, reported by the host
    active[s] = act;
    if (act) steps[s] += 1;
  }
}

// After the first fixed-point step (from y = 0, which never meets the stopping test
// unless f = 0): every system is active and listed; one step is counted unless the
// adaptive test already holds (f = 0).
__global__ void fp_start_kernel(int nsys, int sys0, int nrhs, const double* __restrict__ fnorm2, int fixed,
                                int* __restrict__ active, int* __restrict__ steps, int* __restrict__ list) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nsys) {
    active[s] = 1;
    list[s] = s;
    steps[s] = (fixed || fnorm2[(sys0 + s) % nrhs] > 0.0) ? 1 : 0;
  }
}

// The stopping test of every listed system and the compacted list in one block (adaptive
// mode; see fp_check_kernel and build_list_kernel): wave w sums the partial row of systems
// w, w + 16, ... in a fixed order and its lane 0 decides; after the barrier the block
// compacts the flags into the list (-1 tail) and also writes them to host_flags, pinned
// host memory that the host reads once the launch's event has completed.
constexpr int FTT = 1024;
__global__ __launch_bounds__(FTT) void fp_test_kernel(const double* __restrict__ partial, int nblk, int nsys,
                                                      int sys0, int nrhs, const double* __restrict__ fnorm2,
                                                      double inv_reduce2, int max_steps, int* __restrict__ active,
                                                      int* __restrict__ steps, double* __restrict__ rnorm2,
                                                      int* __restrict__ list, int* __restrict__ host_flags) {
  __shared__ int wtot[FTT / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int s = wid; s < nsys; s += FTT / 64) {
    if (active[s] == 0) continue;  // converged earlier: its partial row was not written
    const double* row = partial + (size_t)s * nblk;
    double v = 0.0;
    for (int i = lane; i < nblk; i += 64) v += row[i];
    v = wave_sum(v);
    if (lane == 0) {
      const double r2 = v;
      rnorm2[s] = r2;
      int act = (r2 > fnorm2[(sys0 + s) % nrhs] * inv_reduce2) && (steps[s] < max_steps);
      if (!(r2 == r2) || r2 > 1e300) act = 0;  // NaN / overflow: stop, reported by the host
      active[s] = act;
      if (act) steps[s] += 1;
    }
  }
  __syncthreads();
  int base = 0;
  for (int c0 = 0; c0 < nsys; c0 += FTT) {
    const int s = c0 + threadIdx.x;
    const bool a = s < nsys && active[s] != 0;
    if (s < nsys) host_flags[s] = a ? 1 : 0;
    const unsigned long long m = __ballot(a);
    const int below = __popcll(m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
    if (lane == 0) wtot[wid] = __popcll(m);
    __syncthreads();
    int off = base;
    for (int w = 0; w < wid; ++w) off += wtot[w];
    if (a) list[off + below] = s;
    int tot = 0;
    for (int w = 0; w < FTT / 64; ++w) tot += wtot[w];
    base += tot;
    __syncthreads();
  }
  for (int s = base + threadIdx.x; s < nsys; s += FTT) list[s] = -1;
}

// Stream compaction of the active flags in one block: wave ballots give each lane its
// rank within the wave, LDS carries the wave totals, chunks of NT go in order; the
// tail of the list is filled with -1.
__global__ __launch_bounds__(NT) void build_list_kernel(const int* __restrict__ active, int nsys,
                                                        int* __restrict__ list) {
  __shared__ int wtot[NT / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int base = 0;
  for (int c0 = 0; c0 < nsys; c0 += NT) {
    const int s = c0 + threadIdx.x;
    const bool a = s < nsys && active[s] != 0;
    const unsigned long long m = __ballot(a);
    const int below = __popcll(m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
    if (lane == 0) wtot[wid] = __popcll(m);
    __syncthreads();
    int off = base;
    for (int w = 0; w < wid; ++w) off += wtot[w];
    if (a) list[off + below] = s;
    int tot = 0;
    for (int w = 0; w < NT / 64; ++w) tot += wtot[w];
    base += tot;
    __syncthreads();
  }
  // entries past the count are -1: launches sized for every system skip them
  for (int s = base + threadIdx.x; s < nsys; s += NT) list[s] = -1;
}

// Stopping test of a batch of systems from different operators (see fp_check_kernel):
// system s reduces its own partial row against the norm of its slot's right-hand side.
template <typename T2>
__global__ __launch_bounds__(NT) void fp_check_multi_kernel(const MultiSys<T2>* __restrict__ sys,
                                                            const double* __restrict__ fnorm2, int fixed_steps,
                                                            double inv_reduce2, int max_steps, int* __restrict__ active,
                                                            int* __restrict__ steps, double* __restrict__ rnorm2) {
  __shared__ double sh[4];
  const int s = blockIdx.x;
  if (active[s] == 0) return;
  const MultiSys<T2> sd = sys[s];
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < sd.nblk; i += NT) v[0] += sd.partial[i];
  block_sum_n<1>(v, sh);
  if (threadIdx.x == 0) {
    const double r2 = v[0];
    rnorm2[s] = r2;
    int act;
    if (fixed_steps > 0)
      act = steps[s] < fixed_steps;
    else
      act = (r2 > fnorm2[sd.slot] * inv_reduce2) && (steps[s] < max_steps);
    if (!(r2 == r2) || r2 > 1e300) act = 0;
    active[s] = act;
    if (act) steps[s] += 1;
  }
}

// Adaptive stopping test of a batch with the work tables rebuilt on the device (one
// block): wave w decides systems w, w + 16, ... as fp_check_multi_kernel does; then the
// active systems, in increasing order, get their rows {first block, system} of the
// single-factor table (seg, bps[s].x blocks each) and of the pair table (segp, bps[s].y
// blocks).  Exclusive prefix sums run per chunk of FTT systems: ballots give the row,
// shuffle scans the first blocks, LDS carries the wave totals.  Row `count` of each table
// is the sentinel {total blocks, -1}, the rows after it {INT_MAX, -1}: a launch sized for
// an earlier, larger set of systems searches past the live rows and its surplus blocks
// land on the sentinel and exit.  The flags also go to host_flags (pinned host memory).
template <typename T2>
__global__ __launch_bounds__(FTT) void fp_test_multi_kernel(const MultiSys<T2>* __restrict__ sys, int nsys,
                                                            const int2* __restrict__ bps,
                                                            const double* __restrict__ fnorm2, double inv_reduce2,
                                                            int max_steps, int* __restrict__ active,
                                                            int* __restrict__ steps, double* __restrict__ rnorm2,
                                                            int2* __restrict__ seg, int2* __restrict__ segp,
                                                            int* __restrict__ host_flags) {
  __shared__ int wtot[3][FTT / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int s = wid; s < nsys; s += FTT / 64) {
    if (active[s] == 0) continue;  // stopped earlier: its partial row was not written
    const MultiSys<T2>& sd = sys[s];
    double v = 0.0;
    for (int i = lane; i < sd.nblk; i += 64) v += sd.partial[i];
    v = wave_sum(v);
    if (lane == 0) {
      const double r2 = v;
      rnorm2[s] = r2;
      int act = (r2 > fnorm2[sd.slot] * inv_reduce2) && (steps[s] < max_steps);
      if (!(r2 == r2) || r2 > 1e300) act = 0;
      active[s] = act;
      if (act) steps[s] += 1;
    }
  }
  __syncthreads();
  int base = 0, bbase = 0, pbase = 0;
  for (int c0 = 0; c0 < nsys; c0 += FTT) {
    const int s = c0 + threadIdx.x;
    const bool a = s < nsys && active[s] != 0;
    if (s < nsys) host_flags[s] = a ? 1 : 0;
    const int2 w = a ? bps[s] : make_int2(0, 0);
    const unsigned long long m = __ballot(a);
    const int below = __popcll(m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
    int ib = w.x, ip = w.y;  // inclusive scans within the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int tb = __shfl_up(ib, o, 64), tp = __shfl_up(ip, o, 64);
      if (lane >= o) {
        ib += tb;
        ip += tp;
      }
    }
    if (lane == 63) {
      wtot[0][wid] = __popcll(m);
      wtot[1][wid] = ib;
      wtot[2][wid] = ip;
    }
    __syncthreads();
    int off = base, boff = bbase, poff = pbase;
    for (int v = 0; v < wid; ++v) {
      off += wtot[0][v];
      boff += wtot[1][v];
      poff += wtot[2][v];
    }
    if (a) {
      seg[off + below] = make_int2(boff + ib - w.x, s);
      segp[off + below] = make_int2(poff + ip - w.y, s);
    }
    for (int v = 0; v < FTT / 64; ++v) {
      base += wtot[0][v];
      bbase += wtot[1][v];
      pbase += wtot[2][v];
    }
    __syncthreads();
  }
  for (int r = base + threadIdx.x; r <= nsys; r += FTT) {
    seg[r] = make_int2(r == base ? bbase : INT_MAX, -1);
    segp[r] = make_int2(r == base ? pbase : INT_MAX, -1);
  }
}

__global__ void dfinish_kernel(const double* __restrict__ sums, int nrhs, double* __restrict__ d) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrhs) {
    const double nr = sums[3 * r], ni = sums[3 * r + 1], den = sums[3 * r + 2];
    d[2 * r] = den > 0 ? nr / den : 0.0;
    d[2 * r + 1] = den > 0 ? ni / den : 0.0;
  }
}

// d = s for the systems that took at most one fixed-point step (their y is y1)
template <typename T2>
__global__ void copy_unstepped_kernel(T2* __restrict__ d, const T2* __restrict__ s, const int* __restrict__ steps,
                                      size_t n) {
  const int sys = blockIdx.y;
  if (steps[sys] > 1) return;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
    d[(size_t)sys * n + p] = s[(size_t)sys * n + p];
}

template <typename T2>
__global__ void copy_active_kernel(T2* __restrict__ d, const T2* __restrict__ s, const int* __restrict__ active,
                                   size_t n) {
  const int sys = blockIdx.y;
  if (!active[sys]) return;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride)
    d[(size_t)sys * n + p] = s[(size_t)sys * n + p];
}

__global__ void set_int_kernel(int* p, int v, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

unsigned ew_blocks(size_t n) {
  size_t b = (n + NT - 1) / NT;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

int blas_blocks(size_t n) {
  size_t b = (n + 4 * NT - 1) / (4 * NT);
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

void launch_reduce(hipStream_t st, const double* partial, int nblk, int ncomp, double* out) {
  if (ncomp <= 0) return;
  hipLaunchKernelGGL(reduce_kernel, dim3(ncomp), dim3(NT), 0, st, partial, nblk, out);
}

void launch_multidot(hipStream_t st, const double2* V, int nv, size_t n, size_t vstride, const double2* w,
                     double* partial) {
  if (nv <= 0) return;
  const int nb = blas_blocks(n);
  // groups of 8 vectors along grid y; partial rows stay ordered by vector index
  hipLaunchKernelGGL(multidot_kernel<8>, dim3(nb, (nv + 7) / 8), dim3(NT), 0, st, V, nv, n, vstride, w, partial);
}

void launch_multiaxpy(hipStream_t st, double2* w, const double2* V, int nv, size_t n, size_t vstride,
                      const double* h, double sign) {
  if (nv > 32) {
    for (int i0 = 0; i0 < nv; i0 += 32)
      launch_multiaxpy(st, w, V + (size_t)i0 * vstride, nv - i0 < 32 ? nv - i0 : 32, n, vstride, h + 2 * i0, sign);
    return;
  }
  hipLaunchKernelGGL(multiaxpy_kernel, dim3(blas_blocks(n)), dim3(NT), 0, st, w, V, nv, n, vstride, h, sign);
}

template <bool DOT, bool UPD = true>
static bool launch_axpy_reduce(hipStream_t st, double2* w, const double2* V, int nv, size_t n, size_t vstride,
                               const double* h, double sign, double* partial) {
  if (nv <= 0 || nv > 32) return false;
  const dim3 grid(blas_blocks(n)), block(NT);
  if (nv <= 4)
    hipLaunchKernelGGL((axpy_reduce_kernel<1, DOT, UPD>), grid, block, 0, st, w, V, nv, n, vstride, h, sign,
                       partial);
  else if (nv <= 8)
    hipLaunchKernelGGL((axpy_reduce_kernel<2, DOT, UPD>), grid, block, 0, st, w, V, nv, n, vstride, h, sign,
                       partial);
  else if (nv <= 16)
    hipLaunchKernelGGL((axpy_reduce_kernel<4, DOT, UPD>), grid, block, 0, st, w, V, nv, n, vstride, h, sign,
                       partial);
  else
    hipLaunchKernelGGL((axpy_reduce_kernel<8, DOT, UPD>), grid, block, 0, st, w, V, nv, n, vstride, h, sign,
                       partial);
  return true;
}

void launch_cgs2(hipStream_t st, const double2* V, int nv, size_t n, size_t vstride, double2* w, double* partial,
                 double* h1, double* h2, double* nrm2) {
  const int nb = blas_blocks(n);
  // first pass: the quad-lane kernel without the update (w read once), else the multi-dot
  if (!launch_axpy_reduce<true, false>(st, w, V, nv, n, vstride, nullptr, 0.0, partial))
    launch_multidot(st, V, nv, n, vstride, w, partial);
  launch_reduce(st, partial, nb, 2 * nv, h1);
  if (launch_axpy_reduce<true>(st, w, V, nv, n, vstride, h1, -1.0, partial)) {
    launch_reduce(st, partial, nb, 2 * nv, h2);
    launch_axpy_reduce<false>(st, w, V, nv, n, vstride, h2, -1.0, partial);
    launch_reduce(st, partial, nb, 1, nrm2);
    return;
  }
  launch_multiaxpy(st, w, V, nv, n, vstride, h1, -1.0);
  launch_multidot(st, V, nv, n, vstride, w, partial);
  launch_reduce(st, partial, nb, 2 * nv, h2);
  launch_multiaxpy(st, w, V, nv, n, vstride, h2, -1.0);
  launch_norm2_partial(st, w, false, n, partial);
  launch_reduce(st, partial, nb, 1, nrm2);
}

void launch_norm2_partial(hipStream_t st, const void* x, bool f32, size_t n, double* partial) {
  if (f32)
    hipLaunchKernelGGL(norm2_kernel<float2>, dim3(blas_blocks(n)), dim3(NT), 0, st, (const float2*)x, n, partial);
  else
    hipLaunchKernelGGL(norm2_kernel<double2>, dim3(blas_blocks(n)), dim3(NT), 0, st, (const double2*)x, n, partial);
}

void launch_diffnorm2_partial(hipStream_t st, const double2* a, const double2* b, size_t n, double* partial) {
  hipLaunchKernelGGL(diffnorm2_kernel, dim3(blas_blocks(n)), dim3(NT), 0, st, a, b, n, partial);
}

void launch_scale_inv(hipStream_t st, double2* v, const double2* w, size_t n, const double* nrm2) {
  hipLaunchKernelGGL(scale_inv_kernel, dim3(ew_blocks(n)), dim3(NT), 0, st, v, w, n, nrm2);
}

void launch_fill_zero(hipStream_t st, void* p, size_t bytes) {
  const size_t n16 = bytes / 16;
  if (n16) hipLaunchKernelGGL(fill_zero_kernel, dim3(ew_blocks(n16)), dim3(NT), 0, st, (uint4*)p, n16);
  const size_t tail = bytes - n16 * 16;
  if (tail)
    hipLaunchKernelGGL(fill_zero_tail, dim3(1), dim3(64), 0, st, (unsigned char*)p + n16 * 16, tail);
}

void launch_copy_scaled64(hipStream_t st, double2* dst, const double2* src, size_t n, double s) {
  hipLaunchKernelGGL(copy_scaled64_kernel, dim3(ew_blocks(n)), dim3(NT), 0, st, dst, src, n, s);
}

void launch_convert_64_to_32(hipStream_t st, float2* dst, const double2* src, size_t n) {
  hipLaunchKernelGGL(cvt64to32_kernel, dim3(ew_blocks(n)), dim3(NT), 0, st, dst, src, n);
}

void launch_convert_32_to_64(hipStream_t st, double2* dst, const float2* src, size_t n) {
  hipLaunchKernelGGL(cvt32to64_kernel, dim3(ew_blocks(n)), dim3(NT), 0, st, dst, src, n);
}

template <typename T2>
void launch_combine(hipStream_t st, T2* w, const T2* y, const double* coef, int npole, int nrhs, size_t n,
                    bool accumulate, const T2* y1, const int* steps) {
  const unsigned bx = ew_blocks(n) / (nrhs > 8 ? 8 : (unsigned)nrhs) + 1;
  hipLaunchKernelGGL(combine_kernel<T2>, dim3(bx, nrhs), dim3(NT), 0, st, w, y, coef, npole, nrhs, n,
                     accumulate ? 1 : 0, y1, steps);
}

template <typename T2>
void launch_scale_out(hipStream_t st, double2* out, const T2* w, const double* d, int nrhs, size_t n) {
  const unsigned bx = ew_blocks(n) / (nrhs > 8 ? 8 : (unsigned)nrhs) + 1;
  hipLaunchKernelGGL(scale_out_kernel<T2>, dim3(bx, nrhs), dim3(NT), 0, st, out, w, d, n);
}

void launch_fp_check(hipStream_t st, const double* partial, int nblk, int nsys, int sys0, int nrhs,
                     const double* fnorm2, int fixed_steps, double reduce, int max_steps, int* active,
                     int* steps, double* rnorm2) {
  hipLaunchKernelGGL(fp_check_kernel, dim3(nsys), dim3(NT), 0, st, partial, nblk, sys0, nrhs, fnorm2,
                     fixed_steps, 1.0 / (reduce * reduce), max_steps, active, steps, rnorm2);
}

template <typename T2>
void launch_fp_check_multi(hipStream_t st, const MultiSys<T2>* sys, int nsys, const double* fnorm2, int fixed_steps,
                           double reduce, int max_steps, int* active, int* steps, double* rnorm2) {
  if (nsys > 0)
    hipLaunchKernelGGL(fp_check_multi_kernel<T2>, dim3(nsys), dim3(NT), 0, st, sys, fnorm2, fixed_steps,
                       1.0 / (reduce * reduce), max_steps, active, steps, rnorm2);
}
template void launch_fp_check_multi<float2>(hipStream_t, const MultiSys<float2>*, int, const double*, int, double, int,
                                            int*, int*, double*);
template void launch_fp_check_multi<double2>(hipStream_t, const MultiSys<double2>*, int, const double*, int, double,
                                             int, int*, int*, double*);

template <typename T2>
void launch_fp_test_multi(hipStream_t st, const MultiSys<T2>* sys, int nsys, const int2* bps, const double* fnorm2,
                          double reduce, int max_steps, int* active, int* steps, double* rnorm2, int2* seg,
                          int2* segp, int* host_flags) {
  if (nsys > 0)
    hipLaunchKernelGGL(fp_test_multi_kernel<T2>, dim3(1), dim3(FTT), 0, st, sys, nsys, bps, fnorm2,
                       1.0 / (reduce * reduce), max_steps, active, steps, rnorm2, seg, segp, host_flags);
}
template void launch_fp_test_multi<float2>(hipStream_t, const MultiSys<float2>*, int, const int2*, const double*,
                                           double, int, int*, int*, double*, int2*, int2*, int*);
template void launch_fp_test_multi<double2>(hipStream_t, const MultiSys<double2>*, int, const int2*, const double*,
                                            double, int, int*, int*, double*, int2*, int2*, int*);

void launch_dfinish(hipStream_t st, const double* sums, int nrhs, double* d) {
  hipLaunchKernelGGL(dfinish_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, st, sums, nrhs, d);
}

void launch_set_int(hipStream_t st, int* p, int v, int count) {
  if (count > 0) hipLaunchKernelGGL(set_int_kernel, dim3((count + 255) / 256), dim3(256), 0, st, p, v, count);
}

void launch_fp_start(hipStream_t st, int nsys, int sys0, int nrhs, const double* fnorm2, bool fixed, int* active,
                     int* steps, int* list) {
  if (nsys > 0)
    hipLaunchKernelGGL(fp_start_kernel, dim3((nsys + 255) / 256), dim3(256), 0, st, nsys, sys0, nrhs, fnorm2,
                       fixed ? 1 : 0, active, steps, list);
}

void launch_fp_test(hipStream_t st, const double* partial, int nblk, int nsys, int sys0, int nrhs,
                    const double* fnorm2, double reduce, int max_steps, int* active, int* steps, double* rnorm2,
                    int* list, int* host_flags) {
  if (nsys > 0)
    hipLaunchKernelGGL(fp_test_kernel, dim3(1), dim3(FTT), 0, st, partial, nblk, nsys, sys0, nrhs, fnorm2,
                       1.0 / (reduce * reduce), max_steps, active, steps, rnorm2, list, host_flags);
}

void launch_build_list(hipStream_t st, const int* active, int nsys, int* list) {
  if (nsys > 0) hipLaunchKernelGGL(build_list_kernel, dim3(1), dim3(NT), 0, st, active, nsys, list);
}

void launch_copy_unstepped(hipStream_t st, void* d, const void* s, bool f64, const int* steps, int nsys,
                           size_t n) {
  const dim3 grid(ew_blocks(n) / 4 + 1, nsys);
  if (f64)
    hipLaunchKernelGGL(copy_unstepped_kernel<double2>, grid, dim3(NT), 0, st, (double2*)d, (const double2*)s, steps, n);
  else
    hipLaunchKernelGGL(copy_unstepped_kernel<float2>, grid, dim3(NT), 0, st, (float2*)d, (const float2*)s, steps, n);
}

void launch_copy_active_f(hipStream_t st, float2* d, const float2* s, const int* a, int nsys, size_t n) {
  hipLaunchKernelGGL(copy_active_kernel<float2>, dim3(ew_blocks(n) / 4 + 1, nsys), dim3(NT), 0, st, d, s, a, n);
}

void launch_copy_active_d(hipStream_t st, double2* d, const double2* s, const int* a, int nsys, size_t n) {
  hipLaunchKernelGGL(copy_active_kernel<double2>, dim3(ew_blocks(n) / 4 + 1, nsys), dim3(NT), 0, st, d, s, a, n);
}

template void launch_combine<float2>(hipStream_t, float2*, const float2*, const double*, int, int, size_t, bool,
                                     const float2*, const int*);
template void launch_combine<double2>(hipStream_t, double2*, const double2*, const double*, int, int, size_t,
                                      bool, const double2*, const int*);
template void launch_scale_out<float2>(hipStream_t, double2*, const float2*, const double*, int, size_t);
template void launch_scale_out<double2>(hipStream_t, double2*, const double2*, const double*, int, size_t);

}  // namespace hfci
