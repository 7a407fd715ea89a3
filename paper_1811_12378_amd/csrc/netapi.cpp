// extern "C" entry points of the learned preconditioner.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace hfci {
void launch_scale_f32(hipStream_t s, const float* in, long n, float a, float* out);
}  // namespace hfci

using namespace hfci;

namespace {

hfci_status fail(const Error& e) {
  set_last_error(e.what());
  return e.st;
}

#define NET_BEGIN try {
#define NET_END                                 \
  }                                             \
  catch (const Error& e) {                      \
    return fail(e);                             \
  }                                             \
  catch (const std::exception& e) {             \
    set_last_error(e.what());                   \
    return HFCI_E_HIP;                          \
  }

struct Dev {
  int prev = -1;
  explicit Dev(int d) {
    HFCI_HIP(hipGetDevice(&prev));
    if (prev != d) HFCI_HIP(hipSetDevice(d));
  }
  ~Dev() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

void check_dims(int nx, int ny, int nz) {
  HFCI_REQUIRE(nx >= 4 && ny >= 4 && nz >= 4 && nx % 4 == 0 && ny % 4 == 0 && nz % 4 == 0,
               "network grids need sizes that are multiples of 4 (>= 4)");
}

const char kMagic[8] = {'H', 'F', 'C', 'I', 'N', 'E', 'T', '1'};

}  // namespace

extern "C" {

hfci_status hfci_net_create(hfci_ctx* ctx, const hfci_net_desc* desc, hfci_net** out) {
  NET_BEGIN
  HFCI_REQUIRE(ctx && out, "NULL argument");
  HFCI_REQUIRE(!desc || desc->size == sizeof(hfci_net_desc), "desc->size mismatch");
  *out = nullptr;
  hfci::Ctx* c = ctx;
  Dev dg(c->device);
  *out = new hfci_net(c, desc ? desc->seed : 1234ULL);
  return HFCI_OK;
  NET_END
}

void hfci_net_destroy(hfci_net* net) {
  if (!net) return;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(net->device);
  delete net;
  if (prev >= 0) (void)hipSetDevice(prev);
}

long long hfci_net_param_count(const hfci_net* net) { return net ? net->nparam : 0; }

hfci_status hfci_net_get_params(const hfci_net* net, float* host) {
  NET_BEGIN
  HFCI_REQUIRE(net && host, "NULL argument");
  Dev dg(net->device);
  net->get_params(host);
  return HFCI_OK;
  NET_END
}

hfci_status hfci_net_set_params(hfci_net* net, const float* host) {
  NET_BEGIN
  HFCI_REQUIRE(net && host, "NULL argument");
  Dev dg(net->device);
  net->set_params(host);
  return HFCI_OK;
  NET_END
}

hfci_status hfci_net_get_grads(const hfci_net* net, float* host) {
  NET_BEGIN
  HFCI_REQUIRE(net && host, "NULL argument");
  Dev dg(net->device);
  net->get_grads(host);
  return HFCI_OK;
  NET_END
}

hfci_status hfci_net_eval(hfci_net* net, int nx, int ny, int nz, const uint16_t* x16, float* out) {
  NET_BEGIN
  HFCI_REQUIRE(net && x16 && out, "NULL argument");
  check_dims(nx, ny, nz);
  Dev dg(net->device);
  net->eval(Dims{nz, ny, nx}, x16, out);
  HFCI_HIP(hipGetLastError());
  HFCI_HIP(hipStreamSynchronize(net->ctx->stream));
  return HFCI_OK;
  NET_END
}

hfci_status hfci_net_train_step(hfci_net* net, int nx, int ny, int nz, const uint16_t* x16, const float* target,
                                float lr, int update, int loss_kind, double* loss) {
  NET_BEGIN
  HFCI_REQUIRE(net && x16 && target, "NULL argument");
  check_dims(nx, ny, nz);
  HFCI_REQUIRE(!update || (lr > 0.f && lr < 1.f), "lr must be in (0, 1)");
  HFCI_REQUIRE(loss_kind >= 0 && loss_kind <= 2, "loss_kind must be 0, 1 or 2");
  Dev dg(net->device);
  const double L = net->train_step(Dims{nz, ny, nx}, x16, target, lr, update != 0, true, loss_kind);
  HFCI_HIP(hipGetLastError());
  if (loss) *loss = L;
  return HFCI_OK;
  NET_END
}

hfci_status hfci_net_train(hfci_net* net, const hfci_train_desc* d, double* final_loss) {
  NET_BEGIN
  HFCI_REQUIRE(net && d, "NULL argument");
  HFCI_REQUIRE(d->size == sizeof(hfci_train_desc), "desc->size mismatch");
  HFCI_REQUIRE(d->v && d->e && d->kch && d->medium_of_pair && d->npairs >= 1 && d->nmedia >= 1,
               "missing training pairs");
  for (int i = 0; i < d->npairs; ++i)
    HFCI_REQUIRE(d->medium_of_pair[i] >= 0 && d->medium_of_pair[i] < d->nmedia, "medium index out of range");
  HFCI_REQUIRE(d->crop >= 4 && d->crop % 4 == 0 && d->crop <= d->nx && d->crop <= d->ny && d->crop <= d->nz,
               "crop must be a multiple of 4 no larger than the grid");
  HFCI_REQUIRE(d->steps >= 1 && d->lr > 0.f && d->lr < 1.f && d->lr_min >= 0.f, "bad schedule");
  HFCI_REQUIRE(d->loss_kind >= 0 && d->loss_kind <= 2, "loss_kind must be 0, 1 or 2");
  Dev dg(net->device);
  TrainData td{d->nx, d->ny, d->nz, d->npairs, (const float2*)d->v, (const float2*)d->e, d->kch,
               d->medium_of_pair};
  TrainOpts to{d->crop, d->steps, d->phase_aug, d->log_every, d->verbose, d->loss_kind, d->lr, d->lr_min, d->seed};
  std::vector<double> curve;
  const double L = net->train(td, to, curve);
  HFCI_HIP(hipGetLastError());
  if (d->loss_curve)
    for (int i = 0; i < (int)curve.size() && i < d->loss_curve_cap; ++i) d->loss_curve[i] = curve[i];
  if (final_loss) *final_loss = L;
  return HFCI_OK;
  NET_END
}

hfci_status hfci_net_apply(hfci_net* net, const hfci_op* op, int nvec, const hfci_c128* r, hfci_c128* z) {
  NET_BEGIN
  HFCI_REQUIRE(net && op && r && z, "NULL argument");
  const hfci::Op& o = *op;
  if (o.form != 1) throw hfci::Error(HFCI_E_STATE, "not available for a case-two operator");
  check_dims(o.g.nx, o.g.ny, o.g.nz);
  HFCI_REQUIRE(nvec >= 1, "nvec must be >= 1");
  Dev dg(net->device);
  net->apply(o, nvec, (const double2*)r, (double2*)z);
  HFCI_HIP(hipGetLastError());
  HFCI_HIP(hipStreamSynchronize(net->ctx->stream));
  return HFCI_OK;
  NET_END
}

hfci_status hfci_op_medium_channel(const hfci_op* op, float* out) {
  NET_BEGIN
  HFCI_REQUIRE(op && out, "NULL argument");
  const hfci::Op& o = *op;
  if (o.form != 1) throw hfci::Error(HFCI_E_STATE, "not available for a case-two operator");
  Dev dg(o.device);
  launch_scale_f32(o.ctx->stream, o.kappa32, (long)o.n, (float)(1.0 / o.s_h2), out);
  HFCI_HIP(hipGetLastError());
  HFCI_HIP(hipStreamSynchronize(o.ctx->stream));
  return HFCI_OK;
  NET_END
}

hfci_status hfci_net_save(const hfci_net* net, const char* path) {
  NET_BEGIN
  HFCI_REQUIRE(net && path, "NULL argument");
  Dev dg(net->device);
  const long n = net->nparam;
  std::vector<float> buf(3 * (size_t)n);
  HFCI_HIP(hipStreamSynchronize(net->ctx->stream));
  HFCI_HIP(hipMemcpy(buf.data(), net->p, n * sizeof(float), hipMemcpyDeviceToHost));
  HFCI_HIP(hipMemcpy(buf.data() + n, net->m, n * sizeof(float), hipMemcpyDeviceToHost));
  HFCI_HIP(hipMemcpy(buf.data() + 2 * n, net->v, n * sizeof(float), hipMemcpyDeviceToHost));
  FILE* f = std::fopen(path, "wb");
  if (!f) throw Error(HFCI_E_ARG, std::string("cannot open ") + path);
  const long long nn = n;
  const int st = net->step;
  bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&nn, sizeof(nn), 1, f) == 1 &&
            std::fwrite(&st, sizeof(st), 1, f) == 1 && std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) throw Error(HFCI_E_ARG, std::string("write failed: ") + path);
  return HFCI_OK;
  NET_END
}

hfci_status hfci_net_load(hfci_net* net, const char* path) {
  NET_BEGIN
  HFCI_REQUIRE(net && path, "NULL argument");
  Dev dg(net->device);
  FILE* f = std::fopen(path, "rb");
  if (!f) throw Error(HFCI_E_ARG, std::string("cannot open ") + path);
  char mg[8];
  long long nn = 0;
  int st = 0;
  bool ok = std::fread(mg, 1, 8, f) == 8 && std::memcmp(mg, kMagic, 8) == 0 && std::fread(&nn, sizeof(nn), 1, f) == 1 &&
            nn == net->nparam && std::fread(&st, sizeof(st), 1, f) == 1;
  std::vector<float> buf(3 * (size_t)net->nparam);
  ok = ok && std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  std::fclose(f);
  if (!ok) throw Error(HFCI_E_ARG, std::string("not a compatible network file: ") + path);
  const long n = net->nparam;
  net->set_params(buf.data());
  HFCI_HIP(hipMemcpy(net->m, buf.data() + n, n * sizeof(float), hipMemcpyHostToDevice));
  HFCI_HIP(hipMemcpy(net->v, buf.data() + 2 * n, n * sizeof(float), hipMemcpyHostToDevice));
  net->step = st;
  return HFCI_OK;
  NET_END
}

}  // extern "C"
