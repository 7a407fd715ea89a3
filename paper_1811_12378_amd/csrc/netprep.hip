// Input/output conversions and the loss of the learned preconditioner (gfx950).
//
// The network sees a residual r as three channels (Re r, Im r)/s and omega^2 h^2 / c^2
// (= kappa / (s/h^2), a resolution-independent description of the medium), with
// s = rms(r); its two output channels are the correction e/s.  Training pairs may be
// rotated by a random global phase (the preconditioner commutes with it).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "netkern.h"

namespace hfci {
namespace {

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ long full_index(long vc, Dims full, Dims crop, int oz, int oy, int ox) {
  const int x = (int)(vc % crop.x);
  const long rr = vc / crop.x;
  const int y = (int)(rr % crop.y);
  const int z = (int)(rr / crop.y);
  return ((long)(z + oz) * full.y + (y + oy)) * full.x + (x + ox);
}

__global__ void prep_input_c64_kernel(Dims full, Dims crop, int oz, int oy, int ox, const float2* __restrict__ r,
                                      const float* __restrict__ kch, float pr, float pi,
                                      const double* __restrict__ scale, uint16_t* __restrict__ x16) {
  const long n = (long)crop.x * crop.y * crop.z;
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const long f = full_index(v, full, crop, oz, oy, ox);
  const float inv = (float)(1.0 / scale[0]);
  const float2 a = r[f];
  const float re = (pr * a.x - pi * a.y) * inv, im = (pr * a.y + pi * a.x) * inv;
  uint16_t* o = x16 + v * 16;
  o[0] = f2bf(re);
  o[1] = f2bf(im);
  o[2] = f2bf(kch[f]);
#pragma unroll
  for (int c = 3; c < 16; ++c) o[c] = 0;
}

__global__ void prep_target_c64_kernel(Dims full, Dims crop, int oz, int oy, int ox, const float2* __restrict__ e,
                                       float pr, float pi, const double* __restrict__ scale, float* __restrict__ t) {
  const long n = (long)crop.x * crop.y * crop.z;
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const long f = full_index(v, full, crop, oz, oy, ox);
  const float inv = (float)(1.0 / scale[0]);
  const float2 a = e[f];
  t[2 * v] = (pr * a.x - pi * a.y) * inv;
  t[2 * v + 1] = (pr * a.y + pi * a.x) * inv;
}

__global__ void prep_input_c128_kernel(long n, const double2* __restrict__ r, const float* __restrict__ kappa,
                                       float inv_s_h2, const double* __restrict__ scale, uint16_t* __restrict__ x16) {
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const double inv = 1.0 / scale[0];
  const double2 a = r[v];
  uint16_t* o = x16 + v * 16;
  o[0] = f2bf((float)(a.x * inv));
  o[1] = f2bf((float)(a.y * inv));
  o[2] = f2bf(kappa[v] * inv_s_h2);
#pragma unroll
  for (int c = 3; c < 16; ++c) o[c] = 0;
}

__global__ void output_c128_kernel(long n, const float* __restrict__ o, const double* __restrict__ scale,
                                   double2* __restrict__ z) {
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const double s = scale[0];
  z[v] = make_double2(s * (double)o[2 * v], s * (double)o[2 * v + 1]);
}

__device__ __forceinline__ double block_sum256(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  return sh[0];
}

constexpr int RB = 1024;  // max partial blocks

__global__ __launch_bounds__(256) void sumsq_crop_c64_kernel(Dims full, Dims crop, int oz, int oy, int ox,
                                                              const float2* __restrict__ r, double* __restrict__ part) {
  __shared__ double sh[256];
  const long n = (long)crop.x * crop.y * crop.z;
  double s = 0.0;
  for (long v = (long)blockIdx.x * 256 + threadIdx.x; v < n; v += (long)gridDim.x * 256) {
    const float2 a = r[full_index(v, full, crop, oz, oy, ox)];
    s += (double)a.x * a.x + (double)a.y * a.y;
  }
  const double t = block_sum256(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void sumsq_c128_kernel(long n, const double2* __restrict__ r,
                                                          double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (long v = (long)blockIdx.x * 256 + threadIdx.x; v < n; v += (long)gridDim.x * 256) {
    const double2 a = r[v];
    s += a.x * a.x + a.y * a.y;
  }
  const double t = block_sum256(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void finish_rms_kernel(const double* __restrict__ part, int nblk, double count,
                                                          double* __restrict__ scale) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) s += part[i];
  const double t = block_sum256(s, sh);
  if (threadIdx.x == 0) scale[0] = t > 0.0 ? sqrt(t / count) : 1.0;
}

__global__ __launch_bounds__(256) void loss_sums_kernel(long nvox, const float* __restrict__ o,
                                                         const float* __restrict__ t, double* __restrict__ part) {
  __shared__ double sh[256];
  double a = 0.0, b = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < 2 * nvox; i += (long)gridDim.x * 256) {
    const double d = (double)o[i] - (double)t[i];
    a += d * d;
    b += (double)t[i] * t[i];
  }
  const double ta = block_sum256(a, sh);
  const double tb = block_sum256(b, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ta;
    part[2 * blockIdx.x + 1] = tb;
  }
}

__global__ __launch_bounds__(256) void loss_finish_kernel(const double* __restrict__ part, int nblk,
                                                           double* __restrict__ sums) {
  __shared__ double sh[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  const double ta = block_sum256(a, sh);
  const double tb = block_sum256(b, sh);
  if (threadIdx.x == 0) {
    sums[0] = tb > 0 ? ta / tb : 0.0;  // loss
    sums[1] = tb;
  }
}

__global__ void loss_grad_kernel(long nvox, const float* __restrict__ o, const float* __restrict__ t,
                                 const double* __restrict__ sums, float* __restrict__ dout) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * nvox) return;
  const double den = sums[1] > 0 ? sums[1] : 1.0;
  dout[i] = (float)(2.0 * ((double)o[i] - (double)t[i]) / den);
}

// scale- and phase-invariant loss: S = <o, t> (complex), P = |o|^2, Q = |t|^2 per block
__global__ __launch_bounds__(256) void loss_pi_sums_kernel(long nvox, const float* __restrict__ o,
                                                            const float* __restrict__ t, double* __restrict__ part) {
  __shared__ double sh[256];
  double sr = 0.0, si = 0.0, pp = 0.0, qq = 0.0;
  for (long v = (long)blockIdx.x * 256 + threadIdx.x; v < nvox; v += (long)gridDim.x * 256) {
    const double o0 = o[2 * v], o1 = o[2 * v + 1], t0 = t[2 * v], t1 = t[2 * v + 1];
    sr += o0 * t0 + o1 * t1;
    si += o0 * t1 - o1 * t0;
    pp += o0 * o0 + o1 * o1;
    qq += t0 * t0 + t1 * t1;
  }
  const double a = block_sum256(sr, sh);
  const double b = block_sum256(si, sh);
  const double c = block_sum256(pp, sh);
  const double d = block_sum256(qq, sh);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x] = a;
    part[4 * blockIdx.x + 1] = b;
    part[4 * blockIdx.x + 2] = c;
    part[4 * blockIdx.x + 3] = d;
  }
}

__global__ __launch_bounds__(256) void loss_pi_finish_kernel(const double* __restrict__ part, int nblk,
                                                              double* __restrict__ sums) {
  __shared__ double sh[256];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nblk; i += 256)
    for (int k = 0; k < 4; ++k) acc[k] += part[4 * i + k];
  double tot[4];
  for (int k = 0; k < 4; ++k) tot[k] = block_sum256(acc[k], sh);
  if (threadIdx.x == 0) {
    const double den = tot[2] * tot[3];
    sums[0] = den > 0 ? 1.0 - (tot[0] * tot[0] + tot[1] * tot[1]) / den : 1.0;
    for (int k = 0; k < 4; ++k) sums[1 + k] = tot[k];
  }
}

// dL/dRe o + i dL/dIm o = -2 conj(S) (t - (S/P) o) / (P Q)
__global__ void loss_pi_grad_kernel(long nvox, const float* __restrict__ o, const float* __restrict__ t,
                                    const double* __restrict__ sums, float* __restrict__ dout) {
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvox) return;
  const double Sr = sums[1], Si = sums[2], P = sums[3], Q = sums[4];
  if (!(P > 0 && Q > 0)) {
    dout[2 * v] = 0.f;
    dout[2 * v + 1] = 0.f;
    return;
  }
  const double qr = Sr / P, qi = Si / P;  // S / P
  const double o0 = o[2 * v], o1 = o[2 * v + 1];
  const double ur = t[2 * v] - (qr * o0 - qi * o1), ui = t[2 * v + 1] - (qr * o1 + qi * o0);
  const double k = -2.0 / (P * Q);
  // conj(S) * u
  dout[2 * v] = (float)(k * (Sr * ur + Si * ui));
  dout[2 * v + 1] = (float)(k * (Sr * ui - Si * ur));
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// out = Ahat in on the box d, both channels: (6 - kch) in - sum of the six neighbours
// (zero outside), kch from the network input's third channel
__global__ void ahat_kernel(Dims d, const uint16_t* __restrict__ x16, const float* __restrict__ in,
                            float* __restrict__ out) {
  const long n = (long)d.x * d.y * d.z;
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int x = (int)(v % d.x);
  const long r = v / d.x;
  const int y = (int)(r % d.y), z = (int)(r / d.y);
  const long sy = d.x, sz = (long)d.x * d.y;
  const float k = 6.f - bf2f(x16[v * 16 + 2]);
  float s0 = k * in[2 * v], s1 = k * in[2 * v + 1];
  auto sub = [&](bool ok, long u) {
    if (ok) {
      s0 -= in[2 * u];
      s1 -= in[2 * u + 1];
    }
  };
  sub(x > 0, v - 1);
  sub(x + 1 < d.x, v + 1);
  sub(y > 0, v - sy);
  sub(y + 1 < d.y, v + sy);
  sub(z > 0, v - sz);
  sub(z + 1 < d.z, v + sz);
  out[2 * v] = s0;
  out[2 * v + 1] = s1;
}

__global__ void scale_f32_kernel(const float* __restrict__ in, long n, float a, float* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * in[i];
}

unsigned nb(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void launch_scale_f32(hipStream_t s, const float* in, long n, float a, float* out) {
  hipLaunchKernelGGL(scale_f32_kernel, dim3(nb(n)), dim3(256), 0, s, in, n, a, out);
}

int rms_blocks(long n) {
  long b = (n + 4095) / 4096;
  if (b > RB) b = RB;
  if (b < 1) b = 1;
  return (int)b;
}

void launch_prep_input_c64(hipStream_t s, Dims full, Dims crop, int oz, int oy, int ox, const float2* r,
                           const float* kch, float ph_re, float ph_im, const double* scale, uint16_t* x16) {
  const long n = (long)crop.x * crop.y * crop.z;
  hipLaunchKernelGGL(prep_input_c64_kernel, dim3(nb(n)), dim3(256), 0, s, full, crop, oz, oy, ox, r, kch, ph_re, ph_im,
                     scale, x16);
}

void launch_prep_target_c64(hipStream_t s, Dims full, Dims crop, int oz, int oy, int ox, const float2* e,
                            float ph_re, float ph_im, const double* scale, float* t) {
  const long n = (long)crop.x * crop.y * crop.z;
  hipLaunchKernelGGL(prep_target_c64_kernel, dim3(nb(n)), dim3(256), 0, s, full, crop, oz, oy, ox, e, ph_re, ph_im,
                     scale, t);
}

void launch_prep_input_c128(hipStream_t s, long n, const double2* r, const float* kappa, float inv_s_h2,
                            const double* scale, uint16_t* x16) {
  hipLaunchKernelGGL(prep_input_c128_kernel, dim3(nb(n)), dim3(256), 0, s, n, r, kappa, inv_s_h2, scale, x16);
}

void launch_output_c128(hipStream_t s, long n, const float* o, const double* scale, double2* z) {
  hipLaunchKernelGGL(output_c128_kernel, dim3(nb(n)), dim3(256), 0, s, n, o, scale, z);
}

void launch_sumsq_crop_c64(hipStream_t s, Dims full, Dims crop, int oz, int oy, int ox, const float2* r,
                           double* part) {
  const long n = (long)crop.x * crop.y * crop.z;
  hipLaunchKernelGGL(sumsq_crop_c64_kernel, dim3(rms_blocks(n)), dim3(256), 0, s, full, crop, oz, oy, ox, r, part);
}

void launch_sumsq_c128(hipStream_t s, long n, const double2* r, double* part) {
  hipLaunchKernelGGL(sumsq_c128_kernel, dim3(rms_blocks(n)), dim3(256), 0, s, n, r, part);
}

void launch_finish_rms(hipStream_t s, const double* part, int nblk, double count, double* scale) {
  hipLaunchKernelGGL(finish_rms_kernel, dim3(1), dim3(256), 0, s, part, nblk, count, scale);
}

void launch_loss(hipStream_t s, long nvox, const float* o, const float* t, double* part, double* sums, float* dout,
                 int kind) {
  if (kind == 1) {
    const int b = rms_blocks(nvox);
    hipLaunchKernelGGL(loss_pi_sums_kernel, dim3(b), dim3(256), 0, s, nvox, o, t, part);
    hipLaunchKernelGGL(loss_pi_finish_kernel, dim3(1), dim3(256), 0, s, part, b, sums);
    if (dout) hipLaunchKernelGGL(loss_pi_grad_kernel, dim3(nb(nvox)), dim3(256), 0, s, nvox, o, t, sums, dout);
    return;
  }
  const int b = rms_blocks(2 * nvox);
  hipLaunchKernelGGL(loss_sums_kernel, dim3(b), dim3(256), 0, s, nvox, o, t, part);
  hipLaunchKernelGGL(loss_finish_kernel, dim3(1), dim3(256), 0, s, part, b, sums);
  if (dout) hipLaunchKernelGGL(loss_grad_kernel, dim3(nb(2 * nvox)), dim3(256), 0, s, nvox, o, t, sums, dout);
}

void launch_residual_loss(hipStream_t s, Dims d, const uint16_t* x16, const float* o, const float* v, double* part,
                          double* sums, float* dout, float* p, float* dp) {
  const long n = (long)d.x * d.y * d.z;
  hipLaunchKernelGGL(ahat_kernel, dim3(nb(n)), dim3(256), 0, s, d, x16, o, p);
  launch_loss(s, n, p, v, part, sums, dout ? dp : nullptr, 1);
  if (dout) hipLaunchKernelGGL(ahat_kernel, dim3(nb(n)), dim3(256), 0, s, d, x16, dp, dout);
}

}  // namespace hfci
