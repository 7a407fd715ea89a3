// 3x3x3 "same" convolutions and the elementwise ops of the learned preconditioner
// (a small 3D U-Net), for gfx950: BF16 activations and weights, FP32 accumulation on
// the matrix cores.
//
// Layout: activations are channels-last, element (voxel v, channel c) of a view at
// p[v * cs + off + c]; a "view" lets a convolution read or write a channel slice of a
// wider buffer, so the U-Net's skip concatenations never copy.  Weights are
// [27 taps][Cout][Cin] (tap = (dz+1)*9 + (dy+1)*3 + (dx+1)), so that the Cin values a
// lane feeds to one MFMA are contiguous.
//
// Implicit GEMM: output tile = 16 voxels x 16 output channels per wavefront,
//   D[v][co] += sum_{tap, ci} X[v + off_tap][ci] * W[tap][co][ci],
// one v_mfma_f32_16x16x32_bf16 (Cin % 32 == 0) or v_mfma_f32_16x16x16_bf16 per
// (tap, 32- or 16-channel chunk, Cout tile).  Lane l supplies row (l % 16) and the
// k-range [KB*(l/16), KB*(l/16)+KB) of A (voxels x channels) and column (l % 16) of B;
// the accumulator holds rows 4*(l/16)+r, column l%16.  Voxels are numbered linearly
// (x fastest), so any grid shape fills the waves.
//
// The backward data pass is the same kernel applied to the output gradient with the
// tap-flipped, Cin/Cout-transposed weights; the weight gradient is a GEMM over voxels
// (k = voxel) whose per-chunk partial sums are reduced in a fixed order.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "netkern.h"

namespace hfci {
namespace {

typedef short s4v __attribute__((ext_vector_type(4)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}

struct Coord {
  int z, y, x;
};
__device__ __forceinline__ Coord coord_of(long v, const Dims& d) {
  Coord c;
  c.x = (int)(v % d.x);
  const long r = v / d.x;
  c.y = (int)(r % d.y);
  c.z = (int)(r / d.y);
  return c;
}

template <int KB>
struct Frag;
template <>
struct Frag<4> {  // 16x16x16: 4 bf16 per lane
  using T = s4v;
  __device__ static T load(const uint16_t* p) {
    const uint2 u = *reinterpret_cast<const uint2*>(p);
    T r;
    r[0] = (short)(u.x & 0xffff);
    r[1] = (short)(u.x >> 16);
    r[2] = (short)(u.y & 0xffff);
    r[3] = (short)(u.y >> 16);
    return r;
  }
  __device__ static T zero() { return T{0, 0, 0, 0}; }
  __device__ static f4v mma(T a, T b, f4v c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
};
template <>
struct Frag<8> {  // 16x16x32: 8 bf16 per lane
  using T = b8v;
  __device__ static T load(const uint16_t* p) {
    const uint4 u = *reinterpret_cast<const uint4*>(p);
    return __builtin_bit_cast(T, u);
  }
  __device__ static T zero() { return __builtin_bit_cast(T, make_uint4(0, 0, 0, 0)); }
  __device__ static f4v mma(T a, T b, f4v c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};

// Forward 3x3x3 convolution: one block = 64 consecutive voxels (4 waves x 16);
// each wave produces all Cout channels of its 16 voxels.  CT = Cout / 16 tiles.
template <int KB, int CT>
__global__ __launch_bounds__(256) void conv_fwd_kernel(Dims d, View in, int cin, const uint16_t* __restrict__ w,
                                                       const float* __restrict__ bias, int relu, View out) {
  using F = Frag<KB>;
  constexpr int KC = 4 * KB;  // channels per MFMA
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long nvox = (long)d.x * d.y * d.z;
  const long v0 = (long)blockIdx.x * 64 + wave * 16;
  const int row = lane & 15, kq = lane >> 4;
  const long va = v0 + row;  // voxel whose A-row this lane supplies
  const bool va_ok = va < nvox;
  const Coord ca = coord_of(va_ok ? va : 0, d);
  const int cout = CT * 16;
  f4v acc[CT];
#pragma unroll
  for (int t = 0; t < CT; ++t) acc[t] = f4v{0.f, 0.f, 0.f, 0.f};
  for (int tap = 0; tap < 27; ++tap) {
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const int zz = ca.z + dz, yy = ca.y + dy, xx = ca.x + dx;
    const bool ok = va_ok && zz >= 0 && zz < d.z && yy >= 0 && yy < d.y && xx >= 0 && xx < d.x;
    const long vin = ok ? ((long)zz * d.y + yy) * d.x + xx : 0;
    const uint16_t* ap = in.p + vin * in.cs + in.off + kq * KB;
    const uint16_t* wp = w + (size_t)tap * cout * cin + (size_t)row * cin + kq * KB;
    for (int c0 = 0; c0 < cin; c0 += KC) {
      const typename F::T a = ok ? F::load(ap + c0) : F::zero();
#pragma unroll
      for (int t = 0; t < CT; ++t) {
        const typename F::T b = F::load(wp + (size_t)t * 16 * cin + c0);
        acc[t] = F::mma(a, b, acc[t]);
      }
    }
  }
  // accumulator: rows (voxels) 4*kq + r, column (channel) row
#pragma unroll
  for (int t = 0; t < CT; ++t) {
    const int co = t * 16 + row;
    const float bv = bias ? bias[co] : 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long v = v0 + kq * 4 + r;
      if (v < nvox) {
        float val = acc[t][r] + bv;
        if (relu) val = fmaxf(val, 0.f);
        out.p[v * out.cs + out.off + co] = f2bf(val);
      }
    }
  }
}

// 16 -> 16 channel layers (the full-resolution level of the U-Net) as a z-marching
// implicit GEMM.  A block owns a 64 x 4 voxel tile of each plane of a z-chunk; the input
// tile with its one-voxel halo (66 x 6 voxels x 16 channels) of planes z-1, z, z+1 sits
// in a 3-plane LDS ring and the 27 x 16 x 16 weights in LDS, so every input voxel is read
// from memory about once per chunk instead of once per tap.  Wave w computes row y0+w:
// four 16-voxel blocks, one MFMA per (tap, block) with the weights as A (cout x cin) and
// the input as B (cin x voxels), so the accumulator of lane l holds output channels
// 4(l/16)..4(l/16)+3 of voxel l%16 and is stored as one 8-byte write.
constexpr int ZCX = 64, ZCY = 4, ZLX = ZCX + 2, ZLY = ZCY + 2;

__global__ __launch_bounds__(256) void zconv16_kernel(Dims d, View in, const uint16_t* __restrict__ w,
                                                      const float* __restrict__ bias, int relu, View out, int zlen) {
  __shared__ __align__(16) uint16_t ring[3][ZLY][ZLX][16];
  __shared__ __align__(16) uint16_t ws[27][16][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gx = (d.x + ZCX - 1) / ZCX, gy = (d.y + ZCY - 1) / ZCY;
  const int b = blockIdx.x;
  const int bx = b % gx, by = (b / gx) % gy, zc = b / (gx * gy);
  const int x0 = bx * ZCX, y0 = by * ZCY;
  const int zb = zc * zlen, ze = min(d.z, zb + zlen);
  for (int i = threadIdx.x; i < 27 * 16 * 16 / 8; i += 256)
    reinterpret_cast<uint4*>(&ws[0][0][0])[i] = reinterpret_cast<const uint4*>(w)[i];
  // plane zp of the input tile into ring slot zp mod 3 (zeros outside the grid)
  auto load_plane = [&](int zp) {
    uint4* dst = reinterpret_cast<uint4*>(&ring[(zp + 3) % 3][0][0][0]);
    for (int c = threadIdx.x; c < ZLY * ZLX * 2; c += 256) {
      const int vox = c >> 1, half = c & 1;
      const int lx = vox % ZLX, ly = vox / ZLX;
      const int xg = x0 - 1 + lx, yg = y0 - 1 + ly;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (zp >= 0 && zp < d.z && xg >= 0 && xg < d.x && yg >= 0 && yg < d.y)
        v = *reinterpret_cast<const uint4*>(in.p + (((long)zp * d.y + yg) * d.x + xg) * in.cs + in.off + half * 8);
      dst[c] = v;
    }
  };
  if (zb >= ze) return;
  load_plane(zb - 1);
  load_plane(zb);
  const int row = lane & 15, kq = lane >> 4;
  const int yo = y0 + wave;
  float bv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) bv[r] = bias ? bias[4 * kq + r] : 0.f;
  for (int z = zb; z < ze; ++z) {
    load_plane(z + 1);
    __syncthreads();
    f4v acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int tap = 0; tap < 27; ++tap) {
      const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
      const s4v wa = *reinterpret_cast<const s4v*>(&ws[tap][row][4 * kq]);
      const uint16_t(*pl)[ZLX][16] = ring[(z + dz + 3) % 3];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const s4v xb = *reinterpret_cast<const s4v*>(&pl[wave + 1 + dy][q * 16 + row + 1 + dx][4 * kq]);
        acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa, xb, acc[q], 0, 0, 0);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int xo = x0 + q * 16 + row;
      if (xo < d.x && yo < d.y) {
        uint16_t h[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float v = acc[q][r] + bv[r];
          if (relu) v = fmaxf(v, 0.f);
          h[r] = f2bf(v);
        }
        const uint2 pk = make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16));
        *reinterpret_cast<uint2*>(out.p + (((long)z * d.y + yo) * d.x + xo) * out.cs + out.off + 4 * kq) = pk;
      }
    }
    __syncthreads();
  }
}

// 48 -> 16 channel layer (the full-resolution decoder's first convolution, on the
// concatenation of the upsampled coarse features and the skip connection) as a z-marching
// implicit GEMM.  As zconv16, but the 48-channel planes are too large for a 64 x 4 tile to
// leave room for two blocks per CU: a block owns a 32 x 4 tile, its input planes (34 x 6
// voxels with the halo, 48 channels padded to 56 per voxel, so 16-byte rows stay aligned)
// sit in a 3-plane LDS ring (68.5 KB), and the weights (27 x 16 x 48, the same for every
// block) are read through the L1 cache.  Wave w computes row y0 + w: two 16-voxel blocks,
// one 16x16x16 MFMA per (tap, 16-channel chunk, block), weights as A and input as B.
constexpr int ZDX = 32, ZDY = 4, ZDLX = ZDX + 2, ZDLY = ZDY + 2, ZDC = 48, ZDCP = 56;

__global__ __launch_bounds__(256) void zconv48_kernel(Dims d, View in, const uint16_t* __restrict__ w,
                                                      const float* __restrict__ bias, int relu, View out, int zlen) {
  __shared__ __align__(16) uint16_t ring[3][ZDLY][ZDLX][ZDCP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gx = (d.x + ZDX - 1) / ZDX, gy = (d.y + ZDY - 1) / ZDY;
  const int b = blockIdx.x;
  const int bx = b % gx, by = (b / gx) % gy, zc = b / (gx * gy);
  const int x0 = bx * ZDX, y0 = by * ZDY;
  const int zb = zc * zlen, ze = min(d.z, zb + zlen);
  if (zb >= ze) return;
  constexpr int PARTS = ZDC / 8;  // 16-byte pieces per voxel
  auto load_plane = [&](int zp) {
    uint16_t(*dst)[ZDLX][ZDCP] = ring[(zp + 3) % 3];
    for (int c = threadIdx.x; c < ZDLY * ZDLX * PARTS; c += 256) {
      const int vox = c / PARTS, part = c % PARTS;
      const int lx = vox % ZDLX, ly = vox / ZDLX;
      const int xg = x0 - 1 + lx, yg = y0 - 1 + ly;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (zp >= 0 && zp < d.z && xg >= 0 && xg < d.x && yg >= 0 && yg < d.y)
        v = *reinterpret_cast<const uint4*>(in.p + (((long)zp * d.y + yg) * d.x + xg) * in.cs + in.off + part * 8);
      *reinterpret_cast<uint4*>(&dst[ly][lx][part * 8]) = v;
    }
  };
  load_plane(zb - 1);
  load_plane(zb);
  const int row = lane & 15, kq = lane >> 4;
  const int yo = y0 + wave;
  float bv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) bv[r] = bias ? bias[4 * kq + r] : 0.f;
  for (int z = zb; z < ze; ++z) {
    load_plane(z + 1);
    __syncthreads();
    f4v acc[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[q] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int tap = 0; tap < 27; ++tap) {
      const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
      const uint16_t(*pl)[ZDLX][ZDCP] = ring[(z + dz + 3) % 3];
      const uint16_t* wp = w + ((size_t)tap * 16 + row) * ZDC + 4 * kq;
#pragma unroll
      for (int c = 0; c < ZDC / 16; ++c) {
        const s4v wa = Frag<4>::load(wp + 16 * c);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const s4v xb = *reinterpret_cast<const s4v*>(&pl[wave + 1 + dy][q * 16 + row + 1 + dx][16 * c + 4 * kq]);
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa, xb, acc[q], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int xo = x0 + q * 16 + row;
      if (xo < d.x && yo < d.y) {
        uint16_t h[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float v = acc[q][r] + bv[r];
          if (relu) v = fmaxf(v, 0.f);
          h[r] = f2bf(v);
        }
        const uint2 pk = make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16));
        *reinterpret_cast<uint2*>(out.p + (((long)z * d.y + yo) * d.x + xo) * out.cs + out.off + 4 * kq) = pk;
      }
    }
    __syncthreads();
  }
}

// Weight gradient partials for one tap: P[chunk][tap][co][ci] = sum over the chunk's voxels
// of dz[v][co] * x[v + off_tap][ci].  GEMM with k = voxel (16 voxels per MFMA step);
// the 16 k-values of a lane are gathered (4 per lane) from channels-last memory.
template <int CT_OUT, int CT_IN>
__global__ __launch_bounds__(256) void conv_wgrad_kernel(Dims d, View x, View dz, int chunk, float* __restrict__ part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tap = blockIdx.y;
  const int dzz = tap / 9 - 1, dyy = (tap / 3) % 3 - 1, dxx = tap % 3 - 1;
  const long nvox = (long)d.x * d.y * d.z;
  const long vb = (long)blockIdx.x * chunk;
  const long ve = vb + chunk < nvox ? vb + chunk : nvox;
  const int row = lane & 15, kq = lane >> 4;
  constexpr int NT = CT_OUT * CT_IN;  // output tiles, distributed over the 4 waves
  constexpr int PER = (NT + 3) / 4;
  f4v acc[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) acc[i] = f4v{0.f, 0.f, 0.f, 0.f};
  for (long k0 = vb; k0 < ve; k0 += 16) {
    // this lane's 4 voxels of the k-block
    s4v bfr[CT_IN];
    s4v afr[CT_OUT];
    long vv[4];
    long vin[4];
    bool okv[4], okin[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      vv[r] = k0 + kq * 4 + r;
      okv[r] = vv[r] < ve;
      const Coord c = coord_of(okv[r] ? vv[r] : 0, d);
      const int zz = c.z + dzz, yy = c.y + dyy, xx = c.x + dxx;
      okin[r] = okv[r] && zz >= 0 && zz < d.z && yy >= 0 && yy < d.y && xx >= 0 && xx < d.x;
      vin[r] = okin[r] ? ((long)zz * d.y + yy) * d.x + xx : 0;
    }
#pragma unroll
    for (int t = 0; t < CT_OUT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        afr[t][r] = okv[r] ? (short)dz.p[vv[r] * dz.cs + dz.off + t * 16 + row] : (short)0;
#pragma unroll
    for (int t = 0; t < CT_IN; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        bfr[t][r] = okin[r] ? (short)x.p[vin[r] * x.cs + x.off + t * 16 + row] : (short)0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int tile = wave + 4 * i;
      if (tile < NT) {
        const int to = tile / CT_IN, ti = tile % CT_IN;
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(afr[to], bfr[ti], acc[i], 0, 0, 0);
      }
    }
  }
  const int cout = CT_OUT * 16, cin = CT_IN * 16;
  float* out = part + ((size_t)blockIdx.x * 27 + tap) * cout * cin;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int tile = wave + 4 * i;
    if (tile < NT) {
      const int to = tile / CT_IN, ti = tile % CT_IN;
#pragma unroll
      for (int r = 0; r < 4; ++r) out[(size_t)(to * 16 + kq * 4 + r) * cin + ti * 16 + row] = acc[i][r];
    }
  }
}

// sum over chunks, fixed order: out[i] = sum_c part[c][i]  (optionally += into out)
__global__ void sum_chunks_kernel(const float* __restrict__ part, int nchunk, long len, float* __restrict__ out,
                                  int accumulate) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float s = accumulate ? out[i] : 0.f;
  for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * len + i];
  out[i] = s;
}

// per-channel sums over voxels (bias gradient): partials per block, then sum_chunks
__global__ __launch_bounds__(256) void chan_sum_kernel(View g, int C, long nvox, int per_block, float* __restrict__ part) {
  const long vb = (long)blockIdx.x * per_block;
  const long ve = vb + per_block < nvox ? vb + per_block : nvox;
  __shared__ float sh[256];
  for (int c = 0; c < C; ++c) {
    float s = 0.f;
    for (long v = vb + threadIdx.x; v < ve; v += 256) s += bf2f(g.p[v * g.cs + g.off + c]);
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * C + c] = sh[0];
    __syncthreads();
  }
}

// W'[tap][ci][co] = W[26 - tap][co][ci]  (bf16), for the backward data pass
__global__ void flip_transpose_kernel(const uint16_t* __restrict__ w, int cout, int cin, uint16_t* __restrict__ wt) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long n = 27L * cout * cin;
  if (i >= n) return;
  const int tap = (int)(i / ((long)cin * cout));
  const int rem = (int)(i % ((long)cin * cout));
  const int ci = rem / cout, co = rem % cout;
  wt[i] = w[((size_t)(26 - tap) * cout + co) * cin + ci];
}

__global__ void f32_to_bf16_kernel(const float* __restrict__ a, long n, uint16_t* __restrict__ b) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = f2bf(a[i]);
}

// relu backward: dzo[v][c] = dh[v][c] if post[v][c] > 0 else 0
__global__ void relu_mask_kernel(View dh, View post, int C, long nvox, View dzo) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox * C) return;
  const long v = i / C;
  const int c = (int)(i % C);
  const uint16_t pv = post.p[v * post.cs + post.off + c];
  const bool pos = (pv & 0x8000u) == 0 && (pv & 0x7fffu) != 0;
  dzo.p[v * dzo.cs + dzo.off + c] = pos ? dh.p[v * dh.cs + dh.off + c] : (uint16_t)0;
}

// 2x2x2 average pooling (fine dims d, coarse dims d/2)
__global__ void pool_kernel(Dims d, View in, int C, View out) {
  const Dims e{d.z / 2, d.y / 2, d.x / 2};
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long n = (long)e.x * e.y * e.z * C;
  if (i >= n) return;
  const int c = (int)(i % C);
  const long vc = i / C;
  const Coord q = coord_of(vc, e);
  float s = 0.f;
  for (int k = 0; k < 8; ++k) {
    const long v = ((long)(2 * q.z + (k >> 2)) * d.y + 2 * q.y + ((k >> 1) & 1)) * d.x + 2 * q.x + (k & 1);
    s += bf2f(in.p[v * in.cs + in.off + c]);
  }
  out.p[vc * out.cs + out.off + c] = f2bf(0.125f * s);
}

// adjoint of pooling: out[v][c] (+)= in[parent(v)][c] / 8  (fine dims d)
__global__ void pool_back_kernel(Dims d, View in, int C, View out, View addend) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long n = (long)d.x * d.y * d.z * C;
  if (i >= n) return;
  const int c = (int)(i % C);
  const long v = i / C;
  const Coord f = coord_of(v, d);
  const long vc = ((long)(f.z / 2) * (d.y / 2) + f.y / 2) * (d.x / 2) + f.x / 2;
  float s = 0.125f * bf2f(in.p[vc * in.cs + in.off + c]);
  if (addend.p) s += bf2f(addend.p[v * addend.cs + addend.off + c]);
  out.p[v * out.cs + out.off + c] = f2bf(s);
}

// nearest-neighbour x2 up-sampling (fine dims d)
__global__ void up_kernel(Dims d, View in, int C, View out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long n = (long)d.x * d.y * d.z * C;
  if (i >= n) return;
  const int c = (int)(i % C);
  const long v = i / C;
  const Coord f = coord_of(v, d);
  const long vc = ((long)(f.z / 2) * (d.y / 2) + f.y / 2) * (d.x / 2) + f.x / 2;
  out.p[v * out.cs + out.off + c] = in.p[vc * in.cs + in.off + c];
}

// adjoint of up-sampling: out[vc][c] = sum of the 8 children (coarse dims d/2)
__global__ void up_back_kernel(Dims d, View in, int C, View out) {
  const Dims e{d.z / 2, d.y / 2, d.x / 2};
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long n = (long)e.x * e.y * e.z * C;
  if (i >= n) return;
  const int c = (int)(i % C);
  const long vc = i / C;
  const Coord q = coord_of(vc, e);
  float s = 0.f;
  for (int k = 0; k < 8; ++k) {
    const long v = ((long)(2 * q.z + (k >> 2)) * d.y + 2 * q.y + ((k >> 1) & 1)) * d.x + 2 * q.x + (k & 1);
    s += bf2f(in.p[v * in.cs + in.off + c]);
  }
  out.p[vc * out.cs + out.off + c] = f2bf(s);
}

// 1x1x1 head 16 -> 2 channels: o[v][k] = b[k] + sum_c W[k][c] h[v][c]  (FP32 out)
__global__ void head_fwd_kernel(View h, long nvox, const float* __restrict__ W, const float* __restrict__ b,
                                float* __restrict__ o) {
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvox) return;
  float o0 = b[0], o1 = b[1];
  for (int c = 0; c < 16; ++c) {
    const float x = bf2f(h.p[v * h.cs + h.off + c]);
    o0 += W[c] * x;
    o1 += W[16 + c] * x;
  }
  o[2 * v] = o0;
  o[2 * v + 1] = o1;
}

// head backward: dh[v][c] = sum_k dout[v][k] W[k][c] (bf16); partial dW/db per block
__global__ __launch_bounds__(256) void head_back_kernel(View h, long nvox, const float* __restrict__ W,
                                                        const float* __restrict__ dout, View dh,
                                                        float* __restrict__ part /* [blk][34] */) {
  __shared__ float sh[256];
  const long v = (long)blockIdx.x * 256 + threadIdx.x;
  float g0 = 0.f, g1 = 0.f;
  float x[16];
  if (v < nvox) {
    g0 = dout[2 * v];
    g1 = dout[2 * v + 1];
    for (int c = 0; c < 16; ++c) {
      x[c] = bf2f(h.p[v * h.cs + h.off + c]);
      dh.p[v * dh.cs + dh.off + c] = f2bf(g0 * W[c] + g1 * W[16 + c]);
    }
  } else {
    for (int c = 0; c < 16; ++c) x[c] = 0.f;
  }
  for (int k = 0; k < 34; ++k) {
    float val;
    if (k < 16) val = g0 * x[k];
    else if (k < 32) val = g1 * x[k - 16];
    else val = k == 32 ? g0 : g1;
    sh[threadIdx.x] = val;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * 34 + k] = sh[0];
    __syncthreads();
  }
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, long n, float lr, float b1, float b2, float eps, float c1,
                            float c2, uint16_t* __restrict__ pb) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  if (pb) pb[i] = f2bf(pi);
}

unsigned blocks_for(long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

template <int KB>
void fwd_dispatch(hipStream_t s, Dims d, View in, int cin, const uint16_t* w, const float* bias, int relu, View out,
                  int cout) {
  const long nvox = (long)d.x * d.y * d.z;
  const dim3 g((unsigned)((nvox + 63) / 64));
  switch (cout / 16) {
    case 1: hipLaunchKernelGGL((conv_fwd_kernel<KB, 1>), g, dim3(256), 0, s, d, in, cin, w, bias, relu, out); break;
    case 2: hipLaunchKernelGGL((conv_fwd_kernel<KB, 2>), g, dim3(256), 0, s, d, in, cin, w, bias, relu, out); break;
    case 3: hipLaunchKernelGGL((conv_fwd_kernel<KB, 3>), g, dim3(256), 0, s, d, in, cin, w, bias, relu, out); break;
    case 4: hipLaunchKernelGGL((conv_fwd_kernel<KB, 4>), g, dim3(256), 0, s, d, in, cin, w, bias, relu, out); break;
    case 6: hipLaunchKernelGGL((conv_fwd_kernel<KB, 6>), g, dim3(256), 0, s, d, in, cin, w, bias, relu, out); break;
    default: break;
  }
}

template <int CO>
void wgrad_dispatch_in(hipStream_t s, Dims d, View x, View dz, int cin, int chunk, unsigned nch, float* part) {
  const dim3 g(nch, 27);
  switch (cin / 16) {
    case 1: hipLaunchKernelGGL((conv_wgrad_kernel<CO, 1>), g, dim3(256), 0, s, d, x, dz, chunk, part); break;
    case 2: hipLaunchKernelGGL((conv_wgrad_kernel<CO, 2>), g, dim3(256), 0, s, d, x, dz, chunk, part); break;
    case 3: hipLaunchKernelGGL((conv_wgrad_kernel<CO, 3>), g, dim3(256), 0, s, d, x, dz, chunk, part); break;
    case 4: hipLaunchKernelGGL((conv_wgrad_kernel<CO, 4>), g, dim3(256), 0, s, d, x, dz, chunk, part); break;
    case 6: hipLaunchKernelGGL((conv_wgrad_kernel<CO, 6>), g, dim3(256), 0, s, d, x, dz, chunk, part); break;
    default: break;
  }
}

}  // namespace

bool conv_shape_ok(int cin, int cout) {
  auto ok = [](int c) { return c == 16 || c == 32 || c == 48 || c == 64 || c == 96; };
  return ok(cin) && (cout == 16 || cout == 32 || cout == 48 || cout == 64 || cout == 96);
}

void launch_conv_fwd(hipStream_t s, Dims d, View in, int cin, const uint16_t* w, const float* bias, bool relu,
                     View out, int cout) {
  // the 16 -> 16 layers take the z-marching kernel when the views allow 16-byte vector
  // access (channel stride and offset multiples of 8)
  if (cin == 16 && cout == 16 && in.cs % 8 == 0 && in.off % 8 == 0 && out.cs % 4 == 0 && out.off % 4 == 0) {
    const int gx = (d.x + ZCX - 1) / ZCX, gy = (d.y + ZCY - 1) / ZCY;
    int zlen = 32;
    while (zlen > 4 && (long)gx * gy * ((d.z + zlen - 1) / zlen) < 2048) zlen /= 2;
    const unsigned nb = (unsigned)((long)gx * gy * ((d.z + zlen - 1) / zlen));
    hipLaunchKernelGGL(zconv16_kernel, dim3(nb), dim3(256), 0, s, d, in, w, bias, relu ? 1 : 0, out, zlen);
    return;
  }
  // the 48 -> 16 layer likewise (16-byte loads of the input, 8-byte stores of the output)
  if (cin == ZDC && cout == 16 && in.cs % 8 == 0 && in.off % 8 == 0 && out.cs % 4 == 0 && out.off % 4 == 0) {
    const int gx = (d.x + ZDX - 1) / ZDX, gy = (d.y + ZDY - 1) / ZDY;
    int zlen = 32;
    while (zlen > 4 && (long)gx * gy * ((d.z + zlen - 1) / zlen) < 2048) zlen /= 2;
    const unsigned nb = (unsigned)((long)gx * gy * ((d.z + zlen - 1) / zlen));
    hipLaunchKernelGGL(zconv48_kernel, dim3(nb), dim3(256), 0, s, d, in, w, bias, relu ? 1 : 0, out, zlen);
    return;
  }
  if (cin % 32 == 0)
    fwd_dispatch<8>(s, d, in, cin, w, bias, relu ? 1 : 0, out, cout);
  else
    fwd_dispatch<4>(s, d, in, cin, w, bias, relu ? 1 : 0, out, cout);
}

int wgrad_chunk() { return 2048; }

void launch_conv_wgrad(hipStream_t s, Dims d, View x, int cin, View dz, int cout, float* part, float* dw,
                       bool accumulate) {
  const long nvox = (long)d.x * d.y * d.z;
  const int chunk = wgrad_chunk();
  const unsigned nch = (unsigned)((nvox + chunk - 1) / chunk);
  switch (cout / 16) {
    case 1: wgrad_dispatch_in<1>(s, d, x, dz, cin, chunk, nch, part); break;
    case 2: wgrad_dispatch_in<2>(s, d, x, dz, cin, chunk, nch, part); break;
    case 3: wgrad_dispatch_in<3>(s, d, x, dz, cin, chunk, nch, part); break;
    case 4: wgrad_dispatch_in<4>(s, d, x, dz, cin, chunk, nch, part); break;
    case 6: wgrad_dispatch_in<6>(s, d, x, dz, cin, chunk, nch, part); break;
    default: break;
  }
  const long len = 27L * cout * cin;
  hipLaunchKernelGGL(sum_chunks_kernel, dim3(blocks_for(len)), dim3(256), 0, s, part, (int)nch, len, dw,
                     accumulate ? 1 : 0);
}

long wgrad_part_floats(Dims d, int cin, int cout) {
  const long nvox = (long)d.x * d.y * d.z;
  const long nch = (nvox + wgrad_chunk() - 1) / wgrad_chunk();
  return nch * 27L * cin * cout;
}

long bias_part_floats(Dims d, int C) {
  const long nvox = (long)d.x * d.y * d.z;
  return ((nvox + 4095) / 4096) * C;
}

void launch_bias_grad(hipStream_t s, Dims d, View g, int C, float* part, float* db, bool accumulate) {
  const long nvox = (long)d.x * d.y * d.z;
  const int per = 4096;
  const unsigned nb = (unsigned)((nvox + per - 1) / per);
  hipLaunchKernelGGL(chan_sum_kernel, dim3(nb), dim3(256), 0, s, g, C, nvox, per, part);
  hipLaunchKernelGGL(sum_chunks_kernel, dim3(blocks_for(C)), dim3(256), 0, s, part, (int)nb, (long)C, db,
                     accumulate ? 1 : 0);
}

void launch_flip_transpose(hipStream_t s, const uint16_t* w, int cout, int cin, uint16_t* wt) {
  const long n = 27L * cout * cin;
  hipLaunchKernelGGL(flip_transpose_kernel, dim3(blocks_for(n)), dim3(256), 0, s, w, cout, cin, wt);
}

void launch_f32_to_bf16(hipStream_t s, const float* a, long n, uint16_t* b) {
  hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(blocks_for(n)), dim3(256), 0, s, a, n, b);
}

void launch_relu_mask(hipStream_t s, View dh, View post, int C, long nvox, View dz) {
  hipLaunchKernelGGL(relu_mask_kernel, dim3(blocks_for(nvox * C)), dim3(256), 0, s, dh, post, C, nvox, dz);
}

void launch_pool(hipStream_t s, Dims d, View in, int C, View out) {
  const long n = (long)(d.x / 2) * (d.y / 2) * (d.z / 2) * C;
  hipLaunchKernelGGL(pool_kernel, dim3(blocks_for(n)), dim3(256), 0, s, d, in, C, out);
}

void launch_pool_back(hipStream_t s, Dims d, View in, int C, View out, View addend) {
  const long n = (long)d.x * d.y * d.z * C;
  hipLaunchKernelGGL(pool_back_kernel, dim3(blocks_for(n)), dim3(256), 0, s, d, in, C, out, addend);
}

void launch_up(hipStream_t s, Dims d, View in, int C, View out) {
  const long n = (long)d.x * d.y * d.z * C;
  hipLaunchKernelGGL(up_kernel, dim3(blocks_for(n)), dim3(256), 0, s, d, in, C, out);
}

void launch_up_back(hipStream_t s, Dims d, View in, int C, View out) {
  const long n = (long)(d.x / 2) * (d.y / 2) * (d.z / 2) * C;
  hipLaunchKernelGGL(up_back_kernel, dim3(blocks_for(n)), dim3(256), 0, s, d, in, C, out);
}

void launch_head_fwd(hipStream_t s, View h, long nvox, const float* W, const float* b, float* o) {
  hipLaunchKernelGGL(head_fwd_kernel, dim3(blocks_for(nvox)), dim3(256), 0, s, h, nvox, W, b, o);
}

long head_part_floats(long nvox) { return ((nvox + 255) / 256) * 34; }

void launch_head_back(hipStream_t s, View h, long nvox, const float* W, const float* dout, View dh, float* part,
                      float* dWb /* [34]: dW (32) then db (2) */) {
  const unsigned nb = blocks_for(nvox);
  hipLaunchKernelGGL(head_back_kernel, dim3(nb), dim3(256), 0, s, h, nvox, W, dout, dh, part);
  hipLaunchKernelGGL(sum_chunks_kernel, dim3(1), dim3(256), 0, s, part, (int)nb, 34L, dWb, 0);
}

void launch_adam(hipStream_t s, float* p, const float* g, float* m, float* v, long n, float lr, float b1, float b2,
                 float eps, int step, uint16_t* pb) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2, pb);
}

}  // namespace hfci
