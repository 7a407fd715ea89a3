// The Fourier-spectral operator (Sec. 7.1, eq. eig-Laplacian-spectral) on the GPU:
// S x = F^H Lambda F x with library 3D FFTs (hipFFT, batched over vectors, in place) and
// the diagonal between them (spec_scale_kernel); the shifted solves run the loop of
// fp_simple.h with one batched FFT pair and one epilogue launch per factor.
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "fp_simple.h"

namespace hfci {

namespace {

#define HFCI_FFT(x)                                                                            \
  do {                                                                                         \
    const hipfftResult _r = (x);                                                               \
    if (_r != HIPFFT_SUCCESS) throw Error(HFCI_E_HIP, "hipFFT call failed: " #x);              \
  } while (0)

template <typename T2> const void* kappa_for(const Op& op);
template <> const void* kappa_for<float2>(const Op& op) { return op.kappa32; }
template <> const void* kappa_for<double2>(const Op& op) { return op.kappa64; }

template <typename T2> hipfftType fft_type();
template <> hipfftType fft_type<float2>() { return HIPFFT_C2C; }
template <> hipfftType fft_type<double2>() { return HIPFFT_Z2Z; }

// batched in-place transform of nvec vectors of the grid (x fastest) over its axes longer
// than one point (a length-one axis transforms as the identity), cached per context;
// nullptr for a single-point grid
template <typename T2>
hipfftHandle plan_for(Ctx& ctx, const GridDesc& g, int nvec) {
  int n[3], rank = 0;
  for (int len : {g.nz, g.ny, g.nx})
    if (len > 1) n[rank++] = len;
  if (rank == 0) return nullptr;
  const std::string key = std::to_string(g.nx) + "x" + std::to_string(g.ny) + "x" + std::to_string(g.nz) + "/" +
                          std::to_string(sizeof(T2)) + "/" + std::to_string(nvec);
  auto it = ctx.fft.find(key);
  hipfftHandle p;
  if (it != ctx.fft.end()) {
    p = (hipfftHandle)it->second;
  } else {
    const int dist = g.nx * g.ny * g.nz;
    HFCI_FFT(hipfftPlanMany(&p, rank, n, nullptr, 1, dist, nullptr, 1, dist, fft_type<T2>(), nvec));
    ctx.fft[key] = (void*)p;
  }
  HFCI_FFT(hipfftSetStream(p, ctx.stream));
  return p;
}

void exec(hipfftHandle p, float2* x, int dir) { HFCI_FFT(hipfftExecC2C(p, (hipfftComplex*)x, (hipfftComplex*)x, dir)); }
void exec(hipfftHandle p, double2* x, int dir) {
  HFCI_FFT(hipfftExecZ2Z(p, (hipfftDoubleComplex*)x, (hipfftDoubleComplex*)x, dir));
}

}  // namespace

namespace {

// x_v <- S x_v for v < nvec, in place
template <typename T2>
void spectral_S_inplace(const Op& op, int nvec, T2* x) {
  Ctx& ctx = *op.ctx;
  HFCI_REQUIRE((long long)op.g.nx * op.g.ny * op.g.nz < (1LL << 31), "grid too large for the FFT plans");
  hipfftHandle p = plan_for<T2>(ctx, op.g, nvec);
  if (p) exec(p, x, HIPFFT_FORWARD);
  launch_spec_scale<T2>(ctx.stream, x, nvec, op.g, op.s, op.h);
  if (p) exec(p, x, HIPFFT_BACKWARD);
}

}  // namespace

// out_v = S in_v for v < nvec (out distinct from in)
template <typename T2>
void spectral_S(const Op& op, int nvec, const T2* in, T2* out) {
  HFCI_HIP(hipMemcpyAsync(out, in, (size_t)nvec * op.n * sizeof(T2), hipMemcpyDeviceToDevice, op.ctx->stream));
  spectral_S_inplace<T2>(op, nvec, out);
}
template void spectral_S<float2>(const Op&, int, const float2*, float2*);
template void spectral_S<double2>(const Op&, int, const double2*, double2*);

// y_v = (A - shift) x_v (y distinct from x)
template <typename T2>
void spectral_apply(const Op& op, int nvec, const T2* x, T2* y, double sr, double si) {
  spectral_S<T2>(op, nvec, x, y);
  launch_spec_apply<T2>(op.ctx->stream, op.g, kappa_for<T2>(op), nvec, x, y, y, sr, si);
}
template void spectral_apply<float2>(const Op&, int, const float2*, float2*, double, double);
template void spectral_apply<double2>(const Op&, int, const double2*, double2*, double, double);

void spectral_release(Ctx& ctx) {
  for (auto& kv : ctx.fft) (void)hipfftDestroy((hipfftHandle)kv.second);
  ctx.fft.clear();
}

template <typename T2>
void shifted_solve_spectral(const Op& op, const Contour& c, int nrhs, const T2* f, T2* y, int fixed_steps,
                            double reduce, int max_steps, int* steps_out, FciStats& st) {
  Ctx& ctx = *op.ctx;
  hipStream_t s = ctx.stream;
  const void* K = kappa_for<T2>(op);
  const int nsys = c.J * nrhs;
  T2* sw = (T2*)ctx.ws.get("sp_sw", (size_t)nsys * op.n * sizeof(T2));
  int* slot_sys = (int*)ctx.ws.get("sp_slot_sys", (size_t)nsys * sizeof(int));
  int* sys_slot = (int*)ctx.ws.get("sp_sys_slot", (size_t)nsys * sizeof(int));
  fp_simple<T2>(op, c, nrhs, f, y, fixed_steps, reduce, max_steps, steps_out, st, spec_blocks(op.g), false,
                [&](const SimpleFactor<T2>& sf) {
                  // S w of the factor's inputs, one batched transform: the right-hand sides
                  // (step one's first factor), all vectors when every system iterates, else
                  // the vectors of the systems still iterating gathered into the first slots
                  // of a batch of exactly that many vectors up to 16, else of the next
                  // multiple of 16 (at most 16 + nsys / 16 cached plans; the padding slots
                  // are zero)
                  HFCI_REQUIRE(sf.nfac == 1, "internal: the spectral factors run one per launch");
                  int nact = 0;
                  for (int k = 0; k < sf.nsys; ++k) nact += sf.host_active[k] != 0;
                  const int* slot = nullptr;
                  if ((sf.kind & kFacInF) != 0) {
                    spectral_S<T2>(op, sf.nrhs, sf.in, sw);
                  } else if (nact == sf.nsys) {
                    spectral_S<T2>(op, sf.nsys, sf.in, sw);
                  } else {
                    const int nvec = std::min(nact <= 16 ? nact : (nact + 15) / 16 * 16, sf.nsys);
                    launch_spec_slots(s, sf.active, sf.nsys, nvec, slot_sys, sys_slot);
                    launch_spec_gather<T2>(s, op.g, sf.in, sw, slot_sys, nvec);
                    spectral_S_inplace<T2>(op, nvec, sw);
                    slot = sys_slot;
                  }
                  SpecArgs<T2> a{};
                  a.win = sf.in;
                  a.sw = sw;
                  a.f = sf.f;
                  a.y1 = sf.y1;
                  a.wout = sf.out;
                  a.wout2 = sf.out2;
                  a.coef = c.d_coef;
                  a.poles = c.d_poles;
                  a.active = sf.active;
                  a.partial = sf.partial;
                  a.nrhs = sf.nrhs;
                  a.cstride = c.cstride;
                  a.k = sf.k;
                  const bool ok = launch_spec_factor_slots<T2>(s, op.g, K, sf.kind, sf.nsys, a, slot);
                  HFCI_REQUIRE(ok, "internal: unsupported factor kind");
                });
}
template void shifted_solve_spectral<float2>(const Op&, const Contour&, int, const float2*, float2*, int, double,
                                             int, int*, FciStats&);
template void shifted_solve_spectral<double2>(const Op&, const Contour&, int, const double2*, double2*, int,
                                              double, int, int*, FciStats&);

}  // namespace hfci
