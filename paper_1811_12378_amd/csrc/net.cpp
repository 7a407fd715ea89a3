// Learned preconditioner: a 3-level 3D U-Net (16/32/64 channels, 3x3x3 kernels), BF16
// activations and weights with FP32 accumulation and FP32 master weights, trained with
// Adam on (residual -> FCI correction) pairs.  Host-side orchestration of conv.hip and
// netprep.hip; see oracle/conv.py for the network's definition.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>

#include "internal.h"
#include "netkern.h"

namespace hfci {

namespace {

struct LayerSpec {
  const char* name;
  int cin, cout;
};
// cin of the first layer is the padded input width (3 real channels + 13 zero channels)
const LayerSpec kLayers[] = {{"c1a", 16, 16}, {"c1b", 16, 16}, {"c2a", 16, 32}, {"c2b", 32, 32},
                             {"c3a", 32, 64}, {"c3b", 64, 64}, {"d2a", 96, 32}, {"d2b", 32, 32},
                             {"d1a", 48, 16}, {"d1b", 16, 16}};
constexpr int kNL = 10;
enum { C1A, C1B, C2A, C2B, C3A, C3B, D2A, D2B, D1A, D1B };

View V(uint16_t* p, int cs, int off = 0) { return View{p, cs, off}; }

}  // namespace

Net::Net(Ctx* c, unsigned long long seed) : ctx(c), device(c->device) {
  long off = 0;
  for (int l = 0; l < kNL; ++l) {
    layers[l].cin = kLayers[l].cin;
    layers[l].cout = kLayers[l].cout;
    layers[l].w_off = off;
    off += 27L * kLayers[l].cin * kLayers[l].cout;
    layers[l].b_off = off;
    off += kLayers[l].cout;
  }
  head_off = off;
  off += 34;
  nparam = off;
  HFCI_HIP(hipMalloc(&p, nparam * sizeof(float)));
  HFCI_HIP(hipMalloc(&g, nparam * sizeof(float)));
  HFCI_HIP(hipMalloc(&m, nparam * sizeof(float)));
  HFCI_HIP(hipMalloc(&v, nparam * sizeof(float)));
  HFCI_HIP(hipMalloc(&wb, nparam * sizeof(uint16_t)));
  HFCI_HIP(hipMalloc(&wt, nparam * sizeof(uint16_t)));
  // He-normal kernels (the first layer over its 3 real input channels), zero biases,
  // small head; the padded input channels of the first layer stay zero.
  std::vector<float> h(nparam, 0.f);
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  for (int l = 0; l < kNL; ++l) {
    const int cin_real = l == C1A ? 3 : layers[l].cin;
    const double sd = std::sqrt(2.0 / (27.0 * cin_real));
    for (int t = 0; t < 27; ++t)
      for (int co = 0; co < layers[l].cout; ++co)
        for (int ci = 0; ci < cin_real; ++ci)
          h[layers[l].w_off + ((long)t * layers[l].cout + co) * layers[l].cin + ci] = (float)(sd * nd(rng));
  }
  for (int k = 0; k < 32; ++k) h[head_off + k] = (float)(0.1 * nd(rng));
  set_params(h.data());
  zero_moments();
}

Net::~Net() {
  (void)hipFree(p);
  (void)hipFree(g);
  (void)hipFree(m);
  (void)hipFree(v);
  (void)hipFree(wb);
  (void)hipFree(wt);
}

void Net::zero_moments() {
  launch_fill_zero(ctx->stream, m, nparam * sizeof(float));
  launch_fill_zero(ctx->stream, v, nparam * sizeof(float));
  launch_fill_zero(ctx->stream, g, nparam * sizeof(float));
  step = 0;
}

void Net::refresh_bf16() {
  hipStream_t s = ctx->stream;
  launch_f32_to_bf16(s, p, nparam, wb);
  for (int l = 0; l < kNL; ++l)
    launch_flip_transpose(s, wb + layers[l].w_off, layers[l].cout, layers[l].cin, wt + layers[l].w_off);
}

void Net::set_params(const float* host) {
  HFCI_HIP(hipMemcpy(p, host, nparam * sizeof(float), hipMemcpyHostToDevice));
  refresh_bf16();
  HFCI_HIP(hipStreamSynchronize(ctx->stream));
}

void Net::get_params(float* host) const {
  HFCI_HIP(hipStreamSynchronize(ctx->stream));
  HFCI_HIP(hipMemcpy(host, p, nparam * sizeof(float), hipMemcpyDeviceToHost));
}

void Net::get_grads(float* host) const {
  HFCI_HIP(hipStreamSynchronize(ctx->stream));
  HFCI_HIP(hipMemcpy(host, g, nparam * sizeof(float), hipMemcpyDeviceToHost));
}

Net::Acts Net::acts(Dims d, bool backward) {
  const long V1 = (long)d.x * d.y * d.z, V2 = V1 / 8, V3 = V1 / 64;
  Workspace& ws = ctx->ws;
  auto b16 = [&](const char* tag, long n) { return (uint16_t*)ws.get(tag, (size_t)n * sizeof(uint16_t)); };
  Acts a;
  a.d1 = d;
  a.d2 = Dims{d.z / 2, d.y / 2, d.x / 2};
  a.d3 = Dims{d.z / 4, d.y / 4, d.x / 4};
  a.V1 = V1;
  a.V2 = V2;
  a.V3 = V3;
  a.a1 = b16("net_a1", V1 * 16);
  a.cat1 = b16("net_cat1", V1 * 48);
  a.p1 = b16("net_p1", V2 * 16);
  a.a2 = b16("net_a2", V2 * 32);
  a.cat2 = b16("net_cat2", V2 * 96);
  a.p2 = b16("net_p2", V3 * 32);
  a.a3 = b16("net_a3", V3 * 64);
  a.b3 = b16("net_b3", V3 * 64);
  a.g2 = b16("net_g2", V2 * 32);
  a.dd2 = b16("net_d2", V2 * 32);
  a.g1 = b16("net_g1", V1 * 16);
  a.dd1 = b16("net_d1", V1 * 16);
  a.o = (float*)ws.get("net_o", (size_t)V1 * 2 * sizeof(float));
  if (backward) {
    a.gd1 = b16("net_gd1", V1 * 16);
    a.gz = b16("net_gz", V1 * 16);
    a.gg1 = b16("net_gg1", V1 * 16);
    a.gcat1 = b16("net_gcat1", V1 * 48);
    a.gd2 = b16("net_gd2", V2 * 32);
    a.gg2 = b16("net_gg2", V2 * 32);
    a.gcat2 = b16("net_gcat2", V2 * 96);
    a.gb3 = b16("net_gb3", V3 * 64);
    a.ga3 = b16("net_ga3", V3 * 64);
    a.gp2 = b16("net_gp2", V3 * 32);
    a.ge2 = b16("net_ge2", V2 * 32);
    a.ga2 = b16("net_ga2", V2 * 32);
    a.gp1 = b16("net_gp1", V2 * 16);
    a.ge1 = b16("net_ge1", V1 * 16);
    a.ga1 = b16("net_ga1", V1 * 16);
    a.dout = (float*)ws.get("net_dout", (size_t)V1 * 2 * sizeof(float));
    long part = head_part_floats(V1);
    for (int l = 0; l < kNL; ++l) {
      const Dims dl = (l < C2A || l >= D1A) ? a.d1 : ((l < C3A || l >= D2A) ? a.d2 : a.d3);
      part = std::max(part, wgrad_part_floats(dl, layers[l].cin, layers[l].cout));
      part = std::max(part, bias_part_floats(dl, layers[l].cout));
    }
    a.part = (float*)ws.get("net_part", (size_t)part * sizeof(float));
  }
  return a;
}

void Net::conv(const Acts&, int l, Dims d, View in, View out, bool relu) {
  launch_conv_fwd(ctx->stream, d, in, layers[l].cin, wb + layers[l].w_off, p + layers[l].b_off, relu, out,
                  layers[l].cout);
}

void Net::forward(Dims d, const uint16_t* x16, const Acts& a) {
  hipStream_t s = ctx->stream;
  View x{const_cast<uint16_t*>(x16), 16, 0};
  conv(a, C1A, a.d1, x, V(a.a1, 16), true);
  conv(a, C1B, a.d1, V(a.a1, 16), V(a.cat1, 48, 32), true);          // e1 -> cat1[32:48]
  launch_pool(s, a.d1, V(a.cat1, 48, 32), 16, V(a.p1, 16));
  conv(a, C2A, a.d2, V(a.p1, 16), V(a.a2, 32), true);
  conv(a, C2B, a.d2, V(a.a2, 32), V(a.cat2, 96, 64), true);          // e2 -> cat2[64:96]
  launch_pool(s, a.d2, V(a.cat2, 96, 64), 32, V(a.p2, 32));
  conv(a, C3A, a.d3, V(a.p2, 32), V(a.a3, 64), true);
  conv(a, C3B, a.d3, V(a.a3, 64), V(a.b3, 64), true);
  launch_up(s, a.d2, V(a.b3, 64), 64, V(a.cat2, 96, 0));             // up(b3) -> cat2[0:64]
  conv(a, D2A, a.d2, V(a.cat2, 96), V(a.g2, 32), true);
  conv(a, D2B, a.d2, V(a.g2, 32), V(a.dd2, 32), true);
  launch_up(s, a.d1, V(a.dd2, 32), 32, V(a.cat1, 48, 0));            // up(d2) -> cat1[0:32]
  conv(a, D1A, a.d1, V(a.cat1, 48), V(a.g1, 16), true);
  conv(a, D1B, a.d1, V(a.g1, 16), V(a.dd1, 16), true);
  launch_head_fwd(s, V(a.dd1, 16), a.V1, p + head_off, p + head_off + 32, a.o);
}

// gradient of one ReLU conv layer: dz = dh * (post > 0); weight/bias grads; optional input grad
void Net::conv_back(const Acts& a, int l, Dims d, View in, View post, View dh, View din) {
  hipStream_t s = ctx->stream;
  const long nv = (long)d.x * d.y * d.z;
  const int ci = layers[l].cin, co = layers[l].cout;
  const View dz = V(a.gz, co);
  launch_relu_mask(s, dh, post, co, nv, dz);
  launch_conv_wgrad(s, d, in, ci, dz, co, a.part, g + layers[l].w_off, false);
  launch_bias_grad(s, d, dz, co, a.part, g + layers[l].b_off, false);
  if (din.p) launch_conv_fwd(s, d, dz, co, wt + layers[l].w_off, nullptr, false, din, ci);
}

void Net::backward(const uint16_t* x16, const Acts& a) {
  hipStream_t s = ctx->stream;
  View x{const_cast<uint16_t*>(x16), 16, 0};
  const View none{nullptr, 0, 0};
  launch_head_back(s, V(a.dd1, 16), a.V1, p + head_off, a.dout, V(a.gd1, 16), a.part, g + head_off);
  conv_back(a, D1B, a.d1, V(a.g1, 16), V(a.dd1, 16), V(a.gd1, 16), V(a.gg1, 16));
  conv_back(a, D1A, a.d1, V(a.cat1, 48), V(a.g1, 16), V(a.gg1, 16), V(a.gcat1, 48));
  launch_up_back(s, a.d1, V(a.gcat1, 48, 0), 32, V(a.gd2, 32));
  conv_back(a, D2B, a.d2, V(a.g2, 32), V(a.dd2, 32), V(a.gd2, 32), V(a.gg2, 32));
  conv_back(a, D2A, a.d2, V(a.cat2, 96), V(a.g2, 32), V(a.gg2, 32), V(a.gcat2, 96));
  launch_up_back(s, a.d2, V(a.gcat2, 96, 0), 64, V(a.gb3, 64));
  conv_back(a, C3B, a.d3, V(a.a3, 64), V(a.b3, 64), V(a.gb3, 64), V(a.ga3, 64));
  conv_back(a, C3A, a.d3, V(a.p2, 32), V(a.a3, 64), V(a.ga3, 64), V(a.gp2, 32));
  // de2 = dcat2[64:96] + pool^T(dp2)
  launch_pool_back(s, a.d2, V(a.gp2, 32), 32, V(a.ge2, 32), V(a.gcat2, 96, 64));
  conv_back(a, C2B, a.d2, V(a.a2, 32), V(a.cat2, 96, 64), V(a.ge2, 32), V(a.ga2, 32));
  conv_back(a, C2A, a.d2, V(a.p1, 16), V(a.a2, 32), V(a.ga2, 32), V(a.gp1, 16));
  launch_pool_back(s, a.d1, V(a.gp1, 16), 16, V(a.ge1, 16), V(a.gcat1, 48, 32));
  conv_back(a, C1B, a.d1, V(a.a1, 16), V(a.cat1, 48, 32), V(a.ge1, 16), V(a.ga1, 16));
  conv_back(a, C1A, a.d1, x, V(a.a1, 16), V(a.ga1, 16), none);
}

double Net::train_step(Dims d, const uint16_t* x16, const float* target, float lr, bool update, bool read_loss,
                       int loss_kind) {
  hipStream_t s = ctx->stream;
  const Acts a = acts(d, true);
  double* lpart = (double*)ctx->ws.get("net_lpart", 4 * 1024 * sizeof(double));
  double* lsum = (double*)ctx->ws.get("net_lsum", 5 * sizeof(double));
  forward(d, x16, a);
  if (loss_kind == 2) {
    float* pb = (float*)ctx->ws.get("net_rp", (size_t)a.V1 * 2 * sizeof(float));
    float* dpb = (float*)ctx->ws.get("net_rdp", (size_t)a.V1 * 2 * sizeof(float));
    launch_residual_loss(s, d, x16, a.o, target, lpart, lsum, a.dout, pb, dpb);
  } else {
    launch_loss(s, a.V1, a.o, target, lpart, lsum, a.dout, loss_kind);
  }
  backward(x16, a);
  if (update) {
    ++step;
    launch_adam(s, p, g, m, v, nparam, lr, 0.9f, 0.999f, 1e-8f, step, wb);
    for (int l = 0; l < kNL; ++l)
      launch_flip_transpose(s, wb + layers[l].w_off, layers[l].cout, layers[l].cin, wt + layers[l].w_off);
  }
  if (!read_loss) return -1.0;
  double h[1];
  HFCI_HIP(hipMemcpyAsync(h, lsum, sizeof(h), hipMemcpyDeviceToHost, s));
  HFCI_HIP(hipStreamSynchronize(s));
  return h[0];
}

void Net::eval(Dims d, const uint16_t* x16, float* out) {
  const Acts a = acts(d, false);
  forward(d, x16, a);
  HFCI_HIP(hipMemcpyAsync(out, a.o, (size_t)a.V1 * 2 * sizeof(float), hipMemcpyDeviceToDevice, ctx->stream));
}

// z = s * N(r / s) with s = rms(r): the preconditioner applied to complex128 vectors.
void Net::apply(const Op& op, int nvec, const double2* r, double2* z) {
  hipStream_t s = ctx->stream;
  const Dims d{op.g.nz, op.g.ny, op.g.nx};
  const long n = (long)op.n;
  uint16_t* x16 = (uint16_t*)ctx->ws.get("net_x16", (size_t)n * 16 * sizeof(uint16_t));
  double* part = (double*)ctx->ws.get("net_rpart", 1024 * sizeof(double));
  double* scale = (double*)ctx->ws.get("net_scale", sizeof(double));
  const Acts a = acts(d, false);
  for (int k = 0; k < nvec; ++k) {
    launch_sumsq_c128(s, n, r + k * n, part);
    launch_finish_rms(s, part, rms_blocks(n), (double)n, scale);
    launch_prep_input_c128(s, n, r + k * n, op.kappa32, (float)(1.0 / op.s_h2), scale, x16);
    forward(d, x16, a);
    launch_output_c128(s, n, a.o, scale, z + k * n);
  }
}

double Net::train(const TrainData& td, const TrainOpts& to, std::vector<double>& curve) {
  hipStream_t s = ctx->stream;
  const Dims full{td.nz, td.ny, td.nx};
  const Dims crop{to.crop, to.crop, to.crop};
  const long nc = (long)to.crop * to.crop * to.crop;
  const long n = (long)td.nx * td.ny * td.nz;
  uint16_t* x16 = (uint16_t*)ctx->ws.get("net_tx16", (size_t)nc * 16 * sizeof(uint16_t));
  float* tgt = (float*)ctx->ws.get("net_tt", (size_t)nc * 2 * sizeof(float));
  double* part = (double*)ctx->ws.get("net_rpart", 1024 * sizeof(double));
  double* scale = (double*)ctx->ws.get("net_scale", sizeof(double));
  std::mt19937_64 rng(to.seed);
  std::uniform_int_distribution<int> pick(0, td.npairs - 1);
  std::uniform_int_distribution<int> oz(0, td.nz - to.crop), oy(0, td.ny - to.crop), ox(0, td.nx - to.crop);
  std::uniform_real_distribution<double> th(0.0, 2.0 * M_PI);
  double last = 0.0;
  for (int it = 0; it < to.steps; ++it) {
    const int pidx = pick(rng);
    const int z0 = oz(rng), y0 = oy(rng), x0 = ox(rng);
    const double t = to.phase_aug ? th(rng) : 0.0;
    const float pr = (float)std::cos(t), pi = (float)std::sin(t);
    const float2* vp = td.v + (size_t)pidx * n;
    const float2* ep = td.e + (size_t)pidx * n;
    const float* kp = td.kch + (size_t)td.medium_of_pair[pidx] * n;
    launch_sumsq_crop_c64(s, full, crop, z0, y0, x0, vp, part);
    launch_finish_rms(s, part, rms_blocks(nc), (double)nc, scale);
    launch_prep_input_c64(s, full, crop, z0, y0, x0, vp, kp, pr, pi, scale, x16);
    // the residual loss compares A N(v) with v itself; the other losses with the correction
    launch_prep_target_c64(s, full, crop, z0, y0, x0, to.loss_kind == 2 ? vp : ep, pr, pi, scale, tgt);
    // cosine decay from lr to lr_min
    const double frac = to.steps > 1 ? (double)it / (to.steps - 1) : 1.0;
    const float lr = (float)(to.lr_min + 0.5 * (to.lr - to.lr_min) * (1.0 + std::cos(M_PI * frac)));
    const bool read = to.log_every > 0 && (it % to.log_every == 0 || it == to.steps - 1);
    const double L = train_step(crop, x16, tgt, lr, true, read, to.loss_kind);
    if (read) {
      curve.push_back(L);
      last = L;
      if (to.verbose) {
        std::fprintf(stderr, "[hfci-net] step %d/%d loss %.4f lr %.2e\n", it, to.steps, L, lr);
        std::fflush(stderr);
      }
    }
  }
  HFCI_HIP(hipStreamSynchronize(s));
  return last;
}

}  // namespace hfci
