// extern "C" entry points of libhfci: argument checks, handle management, error text.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace hfci {

namespace {
thread_local std::string g_err;
constexpr size_t kPinnedInts = 2 * (size_t)kPinnedIntHalf;
constexpr size_t kPinnedDbls = 65536;
}  // namespace

void set_last_error(const char* msg) { g_err = msg; }

void throw_hip(hipError_t e, const char* what, const char* file, int line) {
  const char* base = std::strrchr(file, '/');
  std::string msg = std::string(hipGetErrorString(e)) + " in " + what + " (" + (base ? base + 1 : file) + ":" +
                    std::to_string(line) + ")";
  throw Error(e == hipErrorOutOfMemory ? HFCI_E_OOM : HFCI_E_HIP, msg);
}

void Workspace::set_arena(void* base, size_t cap) {
  arena_ = (char*)base;
  arena_cap_ = cap;
  arena_used_ = 0;
  slices_.clear();
}

void Workspace::clear_arena() {
  arena_ = nullptr;
  arena_cap_ = arena_used_ = 0;
  slices_.clear();
}

void* Workspace::get(const std::string& tag, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (arena_) {
    Buf& sl = slices_[tag];
    if (sl.bytes >= bytes) return sl.p;
    const size_t off = (arena_used_ + 255) & ~(size_t)255;
    if (off > arena_cap_ || bytes > arena_cap_ - off)
      throw Error(HFCI_E_ARG, "the call needs more than the " + std::to_string(arena_cap_) +
                                  "-byte static scratch buffer (at '" + tag + "': " + std::to_string(off + bytes) +
                                  " bytes so far)");
    sl.p = arena_ + off;
    sl.bytes = bytes;
    arena_used_ = off + bytes;
    return sl.p;
  }
  Buf& b = bufs_[tag];
  if (b.bytes >= bytes) return b.p;
  if (b.p) {
    HFCI_HIP(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(HFCI_E_OOM, "device allocation of " + std::to_string(bytes) + " bytes for '" + tag + "' failed");
  }
  b.p = p;
  b.bytes = bytes;
  return p;
}

hipGraphExec_t GraphCache::find(const std::string& key) const {
  auto it = map_.find(key);
  return it == map_.end() ? nullptr : it->second;
}

void GraphCache::put(const std::string& key, hipGraphExec_t exec) {
  if (map_.size() >= 16) clear();
  map_[key] = exec;
}

void GraphCache::clear() {
  for (auto& kv : map_) (void)hipGraphExecDestroy(kv.second);
  map_.clear();
}

void Workspace::release_all() {
  for (auto& kv : bufs_)
    if (kv.second.p) (void)hipFree(kv.second.p);
  bufs_.clear();
}

hipEvent_t Profiler::take() {
  if (!free_.empty()) {
    hipEvent_t e = free_.back();
    free_.pop_back();
    return e;
  }
  hipEvent_t e;  // timing only: no system-scope fence (no cache writeback) per record
  HFCI_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  return e;
}

void Profiler::begin(hipStream_t s) {
  open_ = take();
  HFCI_HIP(hipEventRecord(open_, s));
}

void Profiler::end(hipStream_t s, int cls, double bytes) {
  hipEvent_t b = take();
  HFCI_HIP(hipEventRecord(b, s));
  pending_.push_back(Pending{cls, open_, b, bytes});
  open_ = nullptr;
}

void Profiler::harvest() {
  for (const Pending& p : pending_) {
    float ms = 0.f;
    HFCI_HIP(hipEventSynchronize(p.b));
    HFCI_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    acc[p.cls].launches += 1;
    acc[p.cls].ms += ms;
    acc[p.cls].bytes += p.bytes;
    free_.push_back(p.a);
    free_.push_back(p.b);
  }
  pending_.clear();
}

void Profiler::reset() {
  for (auto& a : acc) a = Acc{};
  for (auto& k : seen_) k = 0;
}

void Profiler::release() {
  for (const Pending& p : pending_) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  pending_.clear();
  for (hipEvent_t e : free_) (void)hipEventDestroy(e);
  free_.clear();
}

static hfci_status fail(const Error& e) {
  g_err = e.what();
  return e.st;
}

#define HFCI_API_BEGIN try {
#define HFCI_API_END                                  \
  }                                                   \
  catch (const Error& e) {                            \
    return fail(e);                                   \
  }                                                   \
  catch (const std::exception& e) {                   \
    g_err = e.what();                                 \
    return HFCI_E_HIP;                                \
  }

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    HFCI_HIP(hipGetDevice(&prev));
    if (prev != dev) HFCI_HIP(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
  }
};

static void check_opts(const hfci_solve_opts* o) {
  HFCI_REQUIRE(o != nullptr, "opts is NULL");
  HFCI_REQUIRE(o->size == sizeof(hfci_solve_opts), "opts->size mismatch (call hfci_default_opts)");
  HFCI_REQUIRE(o->precision == HFCI_F32 || o->precision == HFCI_F64, "precision must be 32 or 64");
  HFCI_REQUIRE(o->restart >= 1 && o->restart <= 64, "restart must be in [1, 64]");
  HFCI_REQUIRE(o->max_it >= 1, "max_it must be >= 1");
  HFCI_REQUIRE(o->tol >= 0.0, "tol must be >= 0");
  HFCI_REQUIRE(o->fp_steps >= 0, "fp_steps must be >= 0");
  HFCI_REQUIRE(o->fp_steps > 0 || (o->fp_reduce > 1.0 && o->fp_max_steps >= 1),
               "adaptive stopping needs fp_reduce > 1 and fp_max_steps >= 1");
  HFCI_REQUIRE(o->k_in >= 0 && o->k_in <= 16, "k_in must be in [0, 16]");
  HFCI_REQUIRE(o->precond == HFCI_PRECOND_FCI || o->precond == HFCI_PRECOND_NONE ||
                   o->precond == HFCI_PRECOND_LEARNED,
               "unknown precond");
  HFCI_REQUIRE(o->precond != HFCI_PRECOND_LEARNED ||
                   (o->net != nullptr && o->learned_tau > 0.0 && o->learned_tau <= 4.0),
               "the learned preconditioner needs opts->net and 0 < learned_tau <= 4");
  HFCI_REQUIRE(o->learned_patience >= 0, "learned_patience must be >= 0");
  HFCI_REQUIRE(o->harvest_cap >= 0 && (o->harvest_cap == 0 || (o->harvest_v && o->harvest_z)),
               "harvest_cap > 0 needs harvest_v and harvest_z");
  HFCI_REQUIRE(o->pole_batch >= 0, "pole_batch must be >= 0");
  HFCI_REQUIRE(o->graphs >= -1 && o->graphs <= 1, "graphs must be -1, 0 or 1");
  HFCI_REQUIRE(o->inner_precond == 0 || o->inner_precond == 1, "inner_precond must be 0 or 1");
  HFCI_REQUIRE(o->inner_precond == 0 || o->net != nullptr, "inner_precond = 1 needs opts->net");
}

}  // namespace hfci

using namespace hfci;


extern "C" {

void hfci_default_opts(hfci_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->size = sizeof(hfci_solve_opts);
  o->precision = HFCI_F64;
  o->restart = 30;
  o->max_it = 500;
  o->tol = 1e-6;
  o->fp_steps = 0;
  o->fp_reduce = 5.0;
  o->fp_max_steps = 200;
  o->k_in = 0;
  o->precond = HFCI_PRECOND_FCI;
  o->pole_batch = 0;
  o->verbose = 0;
  o->net = nullptr;
  o->learned_tau = 1.0;
  o->learned_patience = 8;
  o->inner_precond = 0;
  o->harvest_cap = 0;
  o->harvest_v = nullptr;
  o->harvest_z = nullptr;
  o->graphs = 0;
}

const char* hfci_last_error(void) { return g_err.c_str(); }

const char* hfci_version(void) { return "hfci 0.1 (gfx950)"; }

hfci_status hfci_ctx_create(int device, void* stream, hfci_ctx** out) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(out != nullptr, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  HFCI_HIP(hipGetDeviceCount(&ndev));
  HFCI_REQUIRE(device >= 0 && device < ndev, "device ordinal out of range");
  DeviceGuard dg(device);
  hfci_ctx* c = new hfci_ctx();
  c->device = device;
  try {
    if (stream) {
      c->stream = (hipStream_t)stream;
    } else {
      HFCI_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
    HFCI_HIP(hipHostMalloc((void**)&c->pinned_int, kPinnedInts * sizeof(int), hipHostMallocDefault));
    HFCI_HIP(hipHostGetDevicePointer((void**)&c->pinned_int_dev, c->pinned_int, 0));
    HFCI_HIP(hipHostMalloc((void**)&c->pinned_dbl, kPinnedDbls * sizeof(double), hipHostMallocDefault));
    for (hipEvent_t& e : c->step_event) HFCI_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->noalloc_scratch = noalloc_scratch_for_device(device);
  } catch (...) {
    for (hipEvent_t e : c->step_event)
      if (e) (void)hipEventDestroy(e);
    if (c->pinned_int) (void)hipHostFree(c->pinned_int);
    if (c->pinned_dbl) (void)hipHostFree(c->pinned_dbl);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    throw;
  }
  *out = c;
  return HFCI_OK;
  HFCI_API_END
}

void hfci_ctx_destroy(hfci_ctx* c) {
  if (!c) return;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  c->prof.release();
  c->graphs.clear();
  for (hipEvent_t e : c->step_event)
    if (e) (void)hipEventDestroy(e);
  c->ws.release_all();
  inner_release(*c);
  spectral_release(*c);
  if (c->pinned_int) (void)hipHostFree(c->pinned_int);
  if (c->pinned_dbl) (void)hipHostFree(c->pinned_dbl);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  if (prev >= 0) (void)hipSetDevice(prev);
  delete c;
}

hfci_status hfci_ctx_profile(hfci_ctx* ctx, int enable) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(ctx, "NULL context");
  DeviceGuard dg(ctx->device);
  HFCI_HIP(hipStreamSynchronize(ctx->stream));
  HFCI_REQUIRE(enable >= 0, "enable must be >= 0");
  ctx->prof.harvest();
  if (enable) ctx->prof.reset();
  ctx->prof.on = enable != 0;
  ctx->prof.period = enable > 0 ? enable : 1;
  return HFCI_OK;
  HFCI_API_END
}

hfci_status hfci_ctx_profile_read(const hfci_ctx* ctx, hfci_kernel_prof* out) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(ctx && out, "NULL argument");
  for (int k = 0; k < HFCI_PROF_N; ++k)
    out[k] = hfci_kernel_prof{ctx->prof.acc[k].launches, ctx->prof.acc[k].ms, ctx->prof.acc[k].bytes};
  return HFCI_OK;
  HFCI_API_END
}

hfci_status hfci_op_create(hfci_ctx* ctx, int nx, int ny, int nz, double h, const double* c, double omega,
                           int damp_cells, double damp_rho2, hfci_op** out) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(ctx && out && c, "NULL argument");
  *out = nullptr;
  HFCI_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1, "grid sizes must be >= 1");
  HFCI_REQUIRE((double)nx * ny * nz < 4.0e9, "grid too large");
  HFCI_REQUIRE(h > 0 && std::isfinite(h) && omega > 0 && std::isfinite(omega), "h and omega must be > 0");
  HFCI_REQUIRE(damp_cells >= 0 && damp_rho2 >= 0 && std::isfinite(damp_rho2), "invalid damping layer");
  DeviceGuard dg(ctx->device);
  const size_t n = (size_t)nx * ny * nz;
  std::vector<double> hc(n);
  HFCI_HIP(hipMemcpyAsync(hc.data(), c, n * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HFCI_HIP(hipStreamSynchronize(ctx->stream));
  double cmin = hc[0], cmax = hc[0];
  for (double v : hc) {
    HFCI_REQUIRE(v > 0 && std::isfinite(v), "wavespeed must be positive and finite");
    cmin = std::min(cmin, v);
    cmax = std::max(cmax, v);
  }
  hfci_op* op = new hfci_op();
  try {
    op->ctx = ctx;
    op->device = ctx->device;
    op->n = n;
    op->h = h;
    op->omega = omega;
    op->s = cmin * cmin / (omega * omega);
    op->s_h2 = op->s / (h * h);
    op->damp_cells = damp_cells;
    op->damp_rho2 = damp_rho2;
    op->g.nx = nx;
    op->g.ny = ny;
    op->g.nz = nz;
    op->g.damp_cells = damp_cells;
    op->g.damp_scale = damp_cells > 0 ? damp_rho2 / ((double)damp_cells * damp_cells) : 0.0;
    op->g.s_h2 = op->s_h2;
    std::vector<float> k32(n);
    double kmin = 1e300, kmax = 0;
    for (size_t i = 0; i < n; ++i) {
      const double r = cmin / hc[i];
      hc[i] = r * r;  // kappa = c_min^2 / c^2
      k32[i] = (float)hc[i];
      kmin = std::min(kmin, hc[i]);
      kmax = std::max(kmax, hc[i]);
    }
    op->kmin = kmin;
    op->kmax = kmax;
    op_rectangle(*op);
    HFCI_HIP(hipMalloc(&op->kappa64, n * sizeof(double)));
    HFCI_HIP(hipMalloc(&op->kappa32, n * sizeof(float)));
    HFCI_HIP(hipMemcpy(op->kappa64, hc.data(), n * sizeof(double), hipMemcpyHostToDevice));
    HFCI_HIP(hipMemcpy(op->kappa32, k32.data(), n * sizeof(float), hipMemcpyHostToDevice));
  } catch (...) {
    if (op->kappa64) (void)hipFree(op->kappa64);
    if (op->kappa32) (void)hipFree(op->kappa32);
    delete op;
    throw;
  }
  *out = op;
  return HFCI_OK;
  HFCI_API_END
}

// Entry points that run the case-one kernels only.
static void require_case_one(const hfci::Op* op) {
  if (op && op->form != 1) throw Error(HFCI_E_STATE, "not available for a case-two or spectral operator");
}

hfci_status hfci_op_create_spectral(hfci_ctx* ctx, int nx, int ny, int nz, double h, const double* c, double omega,
                                    int damp_cells, double damp_rho2, hfci_op** out) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(out, "NULL argument");
  hfci_op* op = nullptr;
  const hfci_status st = hfci_op_create(ctx, nx, ny, nz, h, c, omega, damp_cells, damp_rho2, &op);
  if (st != HFCI_OK) return st;
  // Sec. 7.1: lambda = s sum_j (2 pi min(m_j, N_j - m_j) / (N_j h))^2, largest at m_j = floor(N_j / 2);
  // Lemma 3.1's box with lambda_min = 0
  double lmax = 0.0;
  for (int n : {nx, ny, nz}) {
    const double k = 2.0 * M_PI * (n / 2) / (n * h);
    lmax += k * k;
  }
  op->form = 3;
  op->b1 = -op->kmax;
  op->b2 = op->s * lmax - op->kmin;
  *out = op;
  return HFCI_OK;
  HFCI_API_END
}

hfci_status hfci_op_case_two(const hfci_op* op, hfci_op** out) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(op && out, "NULL argument");
  *out = nullptr;
  require_case_one(op);
  DeviceGuard dg(op->ctx->device);
  const size_t npt = op->n;
  hfci_op* o2 = new hfci_op();
  try {
    static_cast<Op&>(*o2) = static_cast<const Op&>(*op);
    o2->kappa64 = nullptr;
    o2->kappa32 = nullptr;
    o2->form = 2;
    o2->n = 2 * npt;
    // Thm 3.2 and the remark after it: spec(B) in |mu + 1| <= R, Im mu in [-rho2, 0],
    // R = rho2/2 + sqrt(rho2^2/4 + rho1), rho1 = rho(A1 + I) <= b2 + 1
    const double rho1 = op->b2 + 1.0;
    const double R = 0.5 * op->rho2 + std::sqrt(0.25 * op->rho2 * op->rho2 + rho1);
    o2->b1 = -1.0 - R;
    o2->b2 = -1.0 + R;
    HFCI_HIP(hipMalloc(&o2->kappa64, npt * sizeof(double)));
    HFCI_HIP(hipMalloc(&o2->kappa32, npt * sizeof(float)));
    HFCI_HIP(hipMemcpy(o2->kappa64, op->kappa64, npt * sizeof(double), hipMemcpyDeviceToDevice));
    HFCI_HIP(hipMemcpy(o2->kappa32, op->kappa32, npt * sizeof(float), hipMemcpyDeviceToDevice));
  } catch (...) {
    if (o2->kappa64) (void)hipFree(o2->kappa64);
    if (o2->kappa32) (void)hipFree(o2->kappa32);
    delete o2;
    throw;
  }
  *out = o2;
  return HFCI_OK;
  HFCI_API_END
}

void hfci_op_destroy(hfci_op* op) {
  if (!op) return;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(op->device);
  // hipFree waits for outstanding work on the device; the context is not touched, so an
  // operator may be released after its context.
  if (op->kappa64) (void)hipFree(op->kappa64);
  if (op->kappa32) (void)hipFree(op->kappa32);
  if (prev >= 0) (void)hipSetDevice(prev);
  delete op;
}

hfci_status hfci_op_info(const hfci_op* op, double* o) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(op && o, "NULL argument");
  o[0] = op->s;
  o[1] = op->s_h2;
  o[2] = op->b1;
  o[3] = op->b2;
  o[4] = op->rho2;
  o[5] = op->kmin;
  o[6] = op->kmax;
  return HFCI_OK;
  HFCI_API_END
}

hfci_status hfci_op_set_tune(hfci_op* op, int prec, const int* t3) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(op && t3, "NULL argument");
  require_case_one(op);
  HFCI_REQUIRE(prec == HFCI_F32 || prec == HFCI_F64, "prec must be HFCI_F32 or HFCI_F64");
  KernelTune t;
  t.kern = t3[0];
  t.ty = t3[1];
  t.pd = t3[2];
  t.cz = t3[3];
  t.fuse = t3[4];
  t.sg = t3[5];
  HFCI_REQUIRE(tune_valid(t), "tune must be {0, ty in {4, 8}, pd in {1, 2}, cz, fuse, sg} or {1, 4, pd in 1..3, cz, "
                              "fuse, sg} or {1, 8, pd in {2, 3}, cz, fuse, sg} or {2, 8, pd in {2, 3}, cz, 1, sg} or "
                              "{3, 8, 2, cz, 1, sg}, cz in [0, 4096], fuse in {0, 1}, sg in [1, 16]");
  HFCI_REQUIRE(t.kern < 2 || prec == HFCI_F32, "kerns 2 and 3 (streams loaded into LDS) are complex64 kernels");
  (prec == HFCI_F32 ? op->g.tune32 : op->g.tune64) = t;
  return HFCI_OK;
  HFCI_API_END
}

hfci_status hfci_op_get_tune(const hfci_op* op, int prec, int* t3) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(op && t3, "NULL argument");
  HFCI_REQUIRE(prec == HFCI_F32 || prec == HFCI_F64, "prec must be HFCI_F32 or HFCI_F64");
  const KernelTune& t = prec == HFCI_F32 ? op->g.tune32 : op->g.tune64;
  t3[0] = t.kern;
  t3[1] = t.ty;
  t3[2] = t.pd;
  t3[3] = t.cz;
  t3[4] = t.fuse;
  t3[5] = t.sg;
  return HFCI_OK;
  HFCI_API_END
}

hfci_status hfci_op_autotune(hfci_op* op, int prec, int nsys, int* best6, double* timings, int cap, int* count) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(op, "NULL operator");
  require_case_one(op);
  HFCI_REQUIRE(prec == HFCI_F32 || prec == HFCI_F64, "prec must be HFCI_F32 or HFCI_F64");
  HFCI_REQUIRE(nsys >= 1 && nsys <= 64, "nsys must be in [1, 64]");
  HFCI_REQUIRE(cap >= 0 && (cap == 0 || timings != nullptr), "timings is NULL");
  DeviceGuard dg(op->device);
  std::vector<std::pair<KernelTune, double>> tm;
  const KernelTune b = prec == HFCI_F32 ? autotune_shapes<float2>(*op, nsys, tm) : autotune_shapes<double2>(*op, nsys, tm);
  if (best6) {
    best6[0] = b.kern;
    best6[1] = b.ty;
    best6[2] = b.pd;
    best6[3] = b.cz;
    best6[4] = b.fuse;
    best6[5] = b.sg;
  }
  const int m = std::min<int>(cap, (int)tm.size());
  for (int k = 0; k < m; ++k) {
    timings[7 * k + 0] = tm[k].first.kern;
    timings[7 * k + 1] = tm[k].first.ty;
    timings[7 * k + 2] = tm[k].first.pd;
    timings[7 * k + 3] = tm[k].first.cz;
    timings[7 * k + 4] = tm[k].first.fuse;
    timings[7 * k + 5] = tm[k].first.sg;
    timings[7 * k + 6] = tm[k].second;
  }
  if (count) *count = (int)tm.size();
  return HFCI_OK;
  HFCI_API_END
}

hfci_status hfci_apply(const hfci_op* op, hfci_c128 shift, int prec, int nvec, const void* x, void* y) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(op && x && y, "NULL argument");
  HFCI_REQUIRE(prec == HFCI_F32 || prec == HFCI_F64, "prec must be 32 or 64");
  HFCI_REQUIRE(nvec >= 1 && nvec <= 4096, "nvec must be in [1, 4096]");
  const size_t bytes = (size_t)nvec * op->n * (prec == HFCI_F64 ? 16 : 8);
  const char* xa = (const char*)x;
  const char* ya = (const char*)y;
  HFCI_REQUIRE(xa + bytes <= ya || ya + bytes <= xa, "x and y overlap");
  DeviceGuard dg(op->ctx->device);
  hipStream_t s = op->ctx->stream;
  Profiler& pr = op->ctx->prof;
  const double e = prec == HFCI_F64 ? 16.0 : 8.0;
  const bool timed = pr.sample(HFCI_PROF_APPLY);
  if (timed) pr.begin(s);
  if (op->form == 3 && prec == HFCI_F64)
    spectral_apply<double2>(*op, nvec, (const double2*)x, (double2*)y, shift.re, shift.im);
  else if (op->form == 3)
    spectral_apply<float2>(*op, nvec, (const float2*)x, (float2*)y, shift.re, shift.im);
  else if (op->form == 2 && prec == HFCI_F64)
    launch_b2_apply<double2>(s, op->g, op->kappa64, nvec, (const double2*)x, (double2*)y, shift.re, shift.im);
  else if (op->form == 2)
    launch_b2_apply<float2>(s, op->g, op->kappa32, nvec, (const float2*)x, (float2*)y, shift.re, shift.im);
  else if (prec == HFCI_F64)
    Launch<double2>::apply(s, op->g, op->kappa64, shift.re, shift.im, nvec, (const double2*)x, (double2*)y);
  else
    Launch<float2>::apply(s, op->g, op->kappa32, shift.re, shift.im, nvec, (const float2*)x, (float2*)y);
  if (timed) pr.end(s, HFCI_PROF_APPLY, (double)op->n * (2.0 * e * nvec + e / 2.0));
  HFCI_HIP(hipGetLastError());
  HFCI_HIP(hipStreamSynchronize(s));
  if (pr.on) pr.harvest();
  return HFCI_OK;
  HFCI_API_END
}

hfci_status hfci_contour_create(const hfci_op* op, int J, double t, double eps, int q, const hfci_c128* z,
                                const hfci_c128* sigma, const double* delta, hfci_contour** out) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(op && out, "NULL argument");
  *out = nullptr;
  HFCI_REQUIRE((z == nullptr) == (sigma == nullptr), "give both poles and weights or neither");
  HFCI_REQUIRE(J >= (z ? 1 : 0) && J <= 256, "J must be in [1, 256] (or 0: chosen by the rule)");
  HFCI_REQUIRE(q >= 0 && q <= 16, "q must be in [0, 16]");
  HFCI_REQUIRE(q > 0 || delta == nullptr, "q = 0 (chosen here) cannot take given deltas");
  HFCI_REQUIRE(J > 0 || delta == nullptr, "J = 0 (chosen here) cannot take given deltas");
  if (!z) {
    HFCI_REQUIRE(t > 0 && eps >= 0 && std::isfinite(t) && std::isfinite(eps),
                 "t must be > 0 and eps >= 0 (0: chosen by the rule)");
    if (J == 0) J = kRuleJ;
    // the finite-difference forms run the fixed-point factors two per pass, the spectral
    // form one per launch
    if (eps == 0) {
      int qr = q;
      eps = rule_eps(op->b1, op->b2, op->rho2, (double)op->g.nx * op->g.ny * op->g.nz, J, t, q,
                     op->form == 3 ? 1 : 2, kRuleReduce, &qr);
      if (q == 0) q = qr;  // chosen with eps
    }
  }
  DeviceGuard dg(op->ctx->device);
  hfci_contour* c = new hfci_contour();
  try {
    c->op = op;
    c->device = op->device;
    c->J = J;
    c->t = t;
    c->eps = eps;
    if (z) {
      c->z.resize(J);
      c->sigma.resize(J);
      for (int j = 0; j < J; ++j) {
        c->z[j] = cd(z[j].re, z[j].im);
        c->sigma[j] = cd(sigma[j].re, sigma[j].im);
        if (c->z[j] == cd(0, 0)) throw Error(HFCI_E_CONTOUR, "a pole at the origin");
      }
    } else {
      contour_poles(J, t, eps, op->rho2, c->z, c->sigma);
      for (int j = 0; j < J; ++j) {
        const double re = c->z[j].real(), im = c->z[j].imag();
        if (re > 1e-12 || (im < eps - 1e-12 && im > -eps - op->rho2 + 1e-12))
          throw Error(HFCI_E_CONTOUR, "pole violates Re z <= 0 and Im z outside (-eps-rho2, eps)");
      }
    }
    if (q == 0) {
      // Sec. 4.2's rule for the pole closest to the origin, the slowest to converge
      int j0 = 0;
      for (int j = 1; j < J; ++j)
        if (std::abs(c->z[j]) < std::abs(c->z[j0])) j0 = j;
      q = choose_q(c->z[j0], op->b1, op->b2, op->rho2, kAutoQMax, op->form == 3 ? 1 : 2);
    }
    c->q = q;
    c->delta.resize(J);
    c->nu.resize(J);
    c->z0.resize(J);
    c->pz.resize(J);
    c->cstride = q + std::max(q - 1, 1);
    c->coef.resize((size_t)J * c->cstride);
    c->pdev.resize(J);
    const std::vector<cd> bd = rectangle_boundary(op->b1, op->b2, op->rho2, 2000);
    for (int j = 0; j < J; ++j) {
      const cd zj = c->z[j];
      if (zj.imag() <= 0.0 && zj.imag() >= -op->rho2)
        throw Error(HFCI_E_CONTOUR, "pole inside the imaginary band [-rho2, 0] of the spectrum");
    }
    // each pole's delta search is independent: run them on host threads
    host_parallel_for(J, [&](int j) {
      const cd zj = c->z[j];
      if (delta) {
        c->delta[j] = delta[j];
        c->z0[j] = cd(0.5 * (op->b1 + op->b2), zj.imag());
        c->nu[j] = rate_on_boundary(delta[j], zj, c->z0[j], q, bd);
      } else {
        optimise_delta(zj, op->b1, op->b2, op->rho2, q, c->delta[j], c->nu[j], c->z0[j]);
      }
    });
    for (int j = 0; j < J; ++j) {
      const cd zj = c->z[j];
      if (!(c->nu[j] < 1.0)) throw Error(HFCI_E_CONTOUR, "no contraction for a pole (nu >= 1)");
      FactorCoef* cj = &c->coef[(size_t)j * c->cstride];
      factor_coefficients(zj, c->z0[j], c->delta[j], q, cj, cj + q, c->pz[j]);
      for (int k = 0; k < c->cstride; ++k)
        if (!std::isfinite(cj[k].a_re) || !std::isfinite(cj[k].a_im) || !std::isfinite(cj[k].b_re) ||
            !std::isfinite(cj[k].b_im))
          throw Error(HFCI_E_NUMERIC, "non-finite factor coefficient");
      const cd zz = zj - c->z0[j];
      c->pdev[j] = PoleDev{c->z0[j].real(), c->z0[j].imag(), zz.real(), zz.imag()};
    }
    HFCI_HIP(hipMalloc(&c->d_coef, c->coef.size() * sizeof(FactorCoef)));
    HFCI_HIP(hipMalloc(&c->d_poles, c->pdev.size() * sizeof(PoleDev)));
    HFCI_HIP(hipMemcpy(c->d_coef, c->coef.data(), c->coef.size() * sizeof(FactorCoef), hipMemcpyHostToDevice));
    HFCI_HIP(hipMemcpy(c->d_poles, c->pdev.data(), c->pdev.size() * sizeof(PoleDev), hipMemcpyHostToDevice));
  } catch (...) {
    if (c->d_coef) (void)hipFree(c->d_coef);
    if (c->d_poles) (void)hipFree(c->d_poles);
    delete c;
    throw;
  }
  *out = c;
  return HFCI_OK;
  HFCI_API_END
}

void hfci_contour_destroy(hfci_contour* c) {
  if (!c) return;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(c->device);
  if (c->d_coef) (void)hipFree(c->d_coef);
  if (c->d_poles) (void)hipFree(c->d_poles);
  if (prev >= 0) (void)hipSetDevice(prev);
  delete c;
}

hfci_status hfci_contour_rule(double b1, double b2, double rho2, double npoints, int J, double t, int q,
                              int per_pass, double fp_reduce, int* J_out, double* eps_out, int* q_out) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(per_pass == 1 || per_pass == 2, "per_pass must be 1 or 2");
  HFCI_REQUIRE(std::isfinite(b1) && std::isfinite(b2) && b1 < b2 && std::isfinite(rho2) && rho2 >= 0,
               "need b1 < b2 and rho2 >= 0");
  HFCI_REQUIRE(npoints >= 1 && std::isfinite(npoints), "npoints must be >= 1");
  HFCI_REQUIRE(J >= 0 && J <= 256, "J must be in [0, 256]");
  HFCI_REQUIRE(t > 0 && std::isfinite(t), "t must be > 0");
  HFCI_REQUIRE(q >= 0 && q <= 16, "q must be in [0, 16]");
  HFCI_REQUIRE(fp_reduce > 1.0 && std::isfinite(fp_reduce), "fp_reduce must be > 1");
  const int Jr = J > 0 ? J : kRuleJ;
  int qr = q;
  const double e = rule_eps(b1, b2, rho2, npoints, Jr, t, q, per_pass, fp_reduce, &qr);
  if (J_out) *J_out = Jr;
  if (eps_out) *eps_out = e;
  if (q_out) *q_out = qr;
  return HFCI_OK;
  HFCI_API_END
}

hfci_status hfci_contour_params(const hfci_contour* c, int* J, double* t, double* eps) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(c, "NULL contour");
  if (J) *J = c->J;
  if (t) *t = c->t;
  if (eps) *eps = c->eps;
  return HFCI_OK;
  HFCI_API_END
}

hfci_status hfci_contour_q(const hfci_contour* c, int* q) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(c && q, "NULL argument");
  *q = c->q;
  return HFCI_OK;
  HFCI_API_END
}

hfci_status hfci_contour_get(const hfci_contour* c, hfci_c128* z, hfci_c128* sigma, double* delta, hfci_c128* z0,
                             double* nu) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(c, "NULL contour");
  for (int j = 0; j < c->J; ++j) {
    if (z) z[j] = hfci_c128{c->z[j].real(), c->z[j].imag()};
    if (sigma) sigma[j] = hfci_c128{c->sigma[j].real(), c->sigma[j].imag()};
    if (delta) delta[j] = c->delta[j];
    if (z0) z0[j] = hfci_c128{c->z0[j].real(), c->z0[j].imag()};
    if (nu) nu[j] = c->nu[j];
  }
  return HFCI_OK;
  HFCI_API_END
}

hfci_status hfci_shifted_solve(const hfci_op* op, const hfci_contour* c, int prec, int nrhs, const void* f,
                               void* y, int steps, double reduce, int max_steps, int* steps_taken) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(op && c && f && y, "NULL argument");
  if (c->op != op) throw Error(HFCI_E_STATE, "contour was created for another operator");
  HFCI_REQUIRE(prec == HFCI_F32 || prec == HFCI_F64, "prec must be 32 or 64");
  HFCI_REQUIRE(nrhs >= 1 && (long)nrhs * c->J <= 65536, "nrhs out of range");
  HFCI_REQUIRE(steps > 0 || (reduce > 1.0 && max_steps >= 1), "give steps > 0, or reduce > 1 and max_steps >= 1");
  DeviceGuard dg(op->ctx->device);
  FciStats st;
  if (op->form == 3 && prec == HFCI_F64)
    shifted_solve_spectral<double2>(*op, *c, nrhs, (const double2*)f, (double2*)y, steps, reduce, max_steps,
                                    steps_taken, st);
  else if (op->form == 3)
    shifted_solve_spectral<float2>(*op, *c, nrhs, (const float2*)f, (float2*)y, steps, reduce, max_steps,
                                   steps_taken, st);
  else if (op->form == 2 && prec == HFCI_F64)
    shifted_solve_case_two<double2>(*op, *c, nrhs, (const double2*)f, (double2*)y, steps, reduce, max_steps,
                                    steps_taken, st);
  else if (op->form == 2)
    shifted_solve_case_two<float2>(*op, *c, nrhs, (const float2*)f, (float2*)y, steps, reduce, max_steps,
                                   steps_taken, st);
  else if (prec == HFCI_F64)
    shifted_solve_batch<double2>(*op, *c, nrhs, (const double2*)f, (double2*)y, steps, reduce, max_steps,
                                 steps_taken, st);
  else
    shifted_solve_batch<float2>(*op, *c, nrhs, (const float2*)f, (float2*)y, steps, reduce, max_steps,
                                steps_taken, st);
  HFCI_HIP(hipGetLastError());
  HFCI_HIP(hipStreamSynchronize(op->ctx->stream));
  return HFCI_OK;
  HFCI_API_END
}

hfci_status hfci_shifted_solve_noalloc(const hfci_op* op, const hfci_contour* c, int prec, int nrhs, const void* f,
                                       void* y, int steps, double reduce, int max_steps, int* steps_taken) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(op && c && f && y, "NULL argument");
  require_case_one(op);
  if (c->op != op) throw Error(HFCI_E_STATE, "contour was created for another operator");
  HFCI_REQUIRE(prec == HFCI_F32 || prec == HFCI_F64, "prec must be 32 or 64");
  HFCI_REQUIRE(nrhs >= 1 && (long)nrhs * c->J <= 65536, "nrhs out of range");
  HFCI_REQUIRE(steps > 0 || (reduce > 1.0 && max_steps >= 1), "give steps > 0, or reduce > 1 and max_steps >= 1");
  Ctx& ctx = *op->ctx;
  HFCI_REQUIRE(ctx.noalloc_scratch != nullptr, "no static scratch array on this device");
  DeviceGuard dg(ctx.device);
  // Every buffer of the solve is a slice of the static array: the workspace allocates
  // nothing while the arena is set, and a solve that does not fit raises HFCI_E_ARG at
  // its first buffer request, before any launch.  Kernel timing (which takes events
  // from a pool that may grow) is paused for the call.
  const int period = ctx.prof.on ? ctx.prof.period : 0;
  ctx.prof.on = false;
  try {
    ArenaScope arena(ctx.ws, ctx.noalloc_scratch, kNoAllocScratchBytes);
    FciStats st;
    if (prec == HFCI_F64)
      shifted_solve_batch<double2>(*op, *c, nrhs, (const double2*)f, (double2*)y, steps, reduce, max_steps,
                                   steps_taken, st);
    else
      shifted_solve_batch<float2>(*op, *c, nrhs, (const float2*)f, (float2*)y, steps, reduce, max_steps,
                                  steps_taken, st);
    HFCI_HIP(hipGetLastError());
    HFCI_HIP(hipStreamSynchronize(ctx.stream));
  } catch (...) {
    if (period > 0) ctx.prof.on = true;
    throw;
  }
  if (period > 0) ctx.prof.on = true;
  return HFCI_OK;
  HFCI_API_END
}

// Common checks of a batch: handles, one context, one q across the contours.
static void check_batch(int count, const hfci_op* const* ops, const hfci_contour* const* cons, bool need_cons,
                        std::vector<const Op*>& vo, std::vector<const Contour*>& vc) {
  HFCI_REQUIRE(count >= 1 && count <= 4096, "count must be in [1, 4096]");
  HFCI_REQUIRE(ops != nullptr && (!need_cons || cons != nullptr), "NULL argument");
  long nsys = 0;
  for (int i = 0; i < count; ++i) {
    HFCI_REQUIRE(ops[i] != nullptr, "NULL operator in the batch");
    require_case_one(ops[i]);
    if (ops[i]->ctx != ops[0]->ctx) throw Error(HFCI_E_STATE, "operators of a batch must share one context");
    vo.push_back(ops[i]);
    if (need_cons) {
      HFCI_REQUIRE(cons[i] != nullptr, "NULL contour in the batch");
      if (cons[i]->op != ops[i]) throw Error(HFCI_E_STATE, "contour was created for another operator");
      if (cons[i]->q != cons[0]->q) throw Error(HFCI_E_ARG, "all contours of a batch must have the same q");
      vc.push_back(cons[i]);
      nsys += cons[i]->J;
    }
  }
  HFCI_REQUIRE(nsys <= 65536, "more than 65536 shifted systems in the batch");
}

hfci_status hfci_shifted_solve_batch(int count, const hfci_op* const* ops, const hfci_contour* const* cons, int prec,
                                     const void* const* f, void* const* y, int steps, double reduce, int max_steps,
                                     int* steps_taken) {
  HFCI_API_BEGIN
  std::vector<const Op*> vo;
  std::vector<const Contour*> vc;
  check_batch(count, ops, cons, true, vo, vc);
  HFCI_REQUIRE(f && y, "NULL argument");
  for (int i = 0; i < count; ++i) HFCI_REQUIRE(f[i] && y[i], "NULL vector in the batch");
  HFCI_REQUIRE(prec == HFCI_F32 || prec == HFCI_F64, "prec must be 32 or 64");
  HFCI_REQUIRE(steps > 0 || (reduce > 1.0 && max_steps >= 1), "give steps > 0, or reduce > 1 and max_steps >= 1");
  DeviceGuard dg(vo[0]->ctx->device);
  FciStats st;
  if (prec == HFCI_F64) {
    std::vector<const double2*> fv(count);
    std::vector<double2*> yv(count);
    for (int i = 0; i < count; ++i) {
      fv[i] = (const double2*)f[i];
      yv[i] = (double2*)y[i];
    }
    shifted_solve_multi<double2>(vo[0]->ctx, vo, vc, fv, yv, steps, reduce, max_steps, steps_taken, st);
  } else {
    std::vector<const float2*> fv(count);
    std::vector<float2*> yv(count);
    for (int i = 0; i < count; ++i) {
      fv[i] = (const float2*)f[i];
      yv[i] = (float2*)y[i];
    }
    shifted_solve_multi<float2>(vo[0]->ctx, vo, vc, fv, yv, steps, reduce, max_steps, steps_taken, st);
  }
  HFCI_HIP(hipGetLastError());
  HFCI_HIP(hipStreamSynchronize(vo[0]->ctx->stream));
  return HFCI_OK;
  HFCI_API_END
}

hfci_status hfci_solve_batch(int count, const hfci_op* const* ops, const hfci_contour* const* cons,
                             const hfci_solve_opts* o, const hfci_c128* const* f, hfci_c128* const* u,
                             hfci_stats* stats) {
  HFCI_API_BEGIN
  check_opts(o);
  HFCI_REQUIRE(o->k_in == 0, "k_in > 0 (Alg. 1 step 4) is not available for batches");
  HFCI_REQUIRE(o->precond == HFCI_PRECOND_FCI || o->precond == HFCI_PRECOND_NONE,
               "a batch takes precond = HFCI_PRECOND_FCI or HFCI_PRECOND_NONE");
  HFCI_REQUIRE(o->harvest_cap == 0, "a batch does not harvest training pairs");
  std::vector<const Op*> vo;
  std::vector<const Contour*> vc;
  check_batch(count, ops, cons, o->precond == HFCI_PRECOND_FCI, vo, vc);
  HFCI_REQUIRE(f && u, "NULL argument");
  for (int i = 0; i < count; ++i) HFCI_REQUIRE(f[i] && u[i], "NULL vector in the batch");
  if (stats)
    for (int i = 0; i < count; ++i) HFCI_REQUIRE(stats[i].size == sizeof(hfci_stats), "stats[i].size mismatch");
  DeviceGuard dg(vo[0]->ctx->device);
  std::vector<const double2*> fv(count);
  std::vector<double2*> uv(count);
  for (int i = 0; i < count; ++i) {
    fv[i] = (const double2*)f[i];
    uv[i] = (double2*)u[i];
  }
  const hfci_status st = solve_batch(vo, vc, *o, fv, uv, stats);
  HFCI_HIP(hipGetLastError());
  HFCI_HIP(hipStreamSynchronize(vo[0]->ctx->stream));
  return st;
  HFCI_API_END
}

hfci_status hfci_fci_apply(const hfci_op* op, const hfci_contour* c, const hfci_solve_opts* o, int nrhs,
                           const hfci_c128* f, hfci_c128* out, hfci_stats* stats) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(op && c && f && out, "NULL argument");
  if (c->op != op) throw Error(HFCI_E_STATE, "contour was created for another operator");
  check_opts(o);
  if (op->form != 1 && o->k_in > 0)
    throw Error(HFCI_E_STATE, "k_in > 0 is not available for a case-two or spectral operator");
  HFCI_REQUIRE(nrhs >= 1 && (long)nrhs * c->J <= 65536, "nrhs out of range");
  HFCI_REQUIRE(!stats || stats->size == sizeof(hfci_stats), "stats->size mismatch");
  DeviceGuard dg(op->ctx->device);
  FciStats st;
  fci_apply(*op, *c, *o, nrhs, (const double2*)f, (double2*)out, st);
  HFCI_HIP(hipGetLastError());
  HFCI_HIP(hipStreamSynchronize(op->ctx->stream));
  if (stats) {
    std::memset((char*)stats + sizeof(size_t), 0, sizeof(hfci_stats) - sizeof(size_t));
    stats->matvecs = st.matvecs;
    stats->fp_steps = st.fp_steps;
  }
  return HFCI_OK;
  HFCI_API_END
}

hfci_status hfci_solve(const hfci_op* op, const hfci_contour* c, const hfci_solve_opts* o, int nrhs,
                       const hfci_c128* f, hfci_c128* u, hfci_stats* stats) {
  HFCI_API_BEGIN
  HFCI_REQUIRE(op && f && u, "NULL argument");
  if (op->form != 1 && o && o->precond == HFCI_PRECOND_LEARNED)
    throw Error(HFCI_E_STATE, "the learned preconditioner is not available for a case-two or spectral operator");
  check_opts(o);
  if (op->form != 1 && o->k_in > 0)
    throw Error(HFCI_E_STATE, "k_in > 0 is not available for a case-two or spectral operator");
  if (o->precond == HFCI_PRECOND_FCI || o->precond == HFCI_PRECOND_LEARNED) {
    HFCI_REQUIRE(c != nullptr, "FCI preconditioning (or its use as the learned fallback) needs a contour");
    if (c->op != op) throw Error(HFCI_E_STATE, "contour was created for another operator");
  }
  HFCI_REQUIRE(nrhs >= 1 && nrhs <= 64, "nrhs must be in [1, 64]");
  HFCI_REQUIRE(!stats || stats->size == sizeof(hfci_stats), "stats->size mismatch");
  if (o->precond == HFCI_PRECOND_LEARNED)
    HFCI_REQUIRE(op->g.nx % 4 == 0 && op->g.ny % 4 == 0 && op->g.nz % 4 == 0 && op->g.nx >= 4 && op->g.ny >= 4 &&
                     op->g.nz >= 4,
                 "the learned preconditioner needs grid sizes that are multiples of 4");
  DeviceGuard dg(op->ctx->device);
  const hfci_status st = fgmres_solve(*op, c, *o, nrhs, (const double2*)f, (double2*)u, stats);
  HFCI_HIP(hipGetLastError());
  if (st == HFCI_W_NOCONV) g_err = "FGMRES reached max_it before the tolerance";
  return st;
  HFCI_API_END
}

}  // extern "C"
