// Internal interface of the learned-preconditioner kernels (conv.hip, netprep.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hfci {

struct Dims {
  int z, y, x;
};

// Channels-last BF16 view: element (voxel v, channel c) at p[v * cs + off + c].
struct View {
  uint16_t* p;
  int cs, off;
};

bool conv_shape_ok(int cin, int cout);
void launch_conv_fwd(hipStream_t s, Dims d, View in, int cin, const uint16_t* w, const float* bias, bool relu,
                     View out, int cout);
long wgrad_part_floats(Dims d, int cin, int cout);
void launch_conv_wgrad(hipStream_t s, Dims d, View x, int cin, View dz, int cout, float* part, float* dw,
                       bool accumulate);
long bias_part_floats(Dims d, int C);
void launch_bias_grad(hipStream_t s, Dims d, View g, int C, float* part, float* db, bool accumulate);
void launch_flip_transpose(hipStream_t s, const uint16_t* w, int cout, int cin, uint16_t* wt);
void launch_f32_to_bf16(hipStream_t s, const float* a, long n, uint16_t* b);
void launch_relu_mask(hipStream_t s, View dh, View post, int C, long nvox, View dz);
void launch_pool(hipStream_t s, Dims d, View in, int C, View out);
void launch_pool_back(hipStream_t s, Dims d, View in, int C, View out, View addend);
void launch_up(hipStream_t s, Dims d, View in, int C, View out);
void launch_up_back(hipStream_t s, Dims d, View in, int C, View out);
void launch_head_fwd(hipStream_t s, View h, long nvox, const float* W, const float* b, float* o);
long head_part_floats(long nvox);
void launch_head_back(hipStream_t s, View h, long nvox, const float* W, const float* dout, View dh, float* part,
                      float* dWb);
void launch_adam(hipStream_t s, float* p, const float* g, float* m, float* v, long n, float lr, float b1, float b2,
                 float eps, int step, uint16_t* pb);

// netprep.hip: network input/output conversions and the loss
// x16[v] = (Re, Im)(phase * r[v]) / scale, kch[v], 0 ... (16 channels), over a crop of the full grid
void launch_prep_input_c64(hipStream_t s, Dims full, Dims crop, int oz, int oy, int ox, const float2* r,
                           const float* kch, float ph_re, float ph_im, const double* scale, uint16_t* x16);
void launch_prep_target_c64(hipStream_t s, Dims full, Dims crop, int oz, int oy, int ox, const float2* e,
                            float ph_re, float ph_im, const double* scale, float* t);
void launch_prep_input_c128(hipStream_t s, long n, const double2* r, const float* kappa, float inv_s_h2,
                            const double* scale, uint16_t* x16);
void launch_output_c128(hipStream_t s, long n, const float* o, const double* scale, double2* z);
// sum of |r|^2 over a crop (complex64) or a full vector (complex128), into partials
int rms_blocks(long n);
void launch_sumsq_crop_c64(hipStream_t s, Dims full, Dims crop, int oz, int oy, int ox, const float2* r,
                           double* part);
void launch_sumsq_c128(hipStream_t s, long n, const double2* r, double* part);
// scale = sqrt(sum / count) (or 1 if zero) from partials
void launch_finish_rms(hipStream_t s, const double* part, int nblk, double count, double* scale);
// kind 0: relative squared loss |o - t|^2 / |t|^2, dout = 2 (o - t) / |t|^2;
// kind 1: scale- and phase-invariant loss 1 - |<o,t>|^2 / (|o|^2 |t|^2) of the complex field.
// sums[0] receives the loss; part needs 4 * rms_blocks(2 * nvox) doubles, sums 5.
void launch_loss(hipStream_t s, long nvox, const float* o, const float* t, double* part, double* sums, float* dout,
                 int kind);
// residual loss (kind 2): p = Ahat o on the box d, the kind-1 loss of p against v, and
// dout = Ahat dL/dp (Ahat is real and symmetric); Ahat = (6 - kch) - sum of the six
// neighbours (zero outside), kch from x16's third channel; p, dp: scratch [n][2]
void launch_residual_loss(hipStream_t s, Dims d, const uint16_t* x16, const float* o, const float* v, double* part,
                          double* sums, float* dout, float* p, float* dp);

}  // namespace hfci
