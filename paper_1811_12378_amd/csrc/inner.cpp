// Alg. 1 step 4 (Sec. 6.3): after steps 1-3 give out = d w, k_in steps of GMRES on the
// remainder A v = f - A out, right-preconditioned by the regularised inverse of the
// discrete Laplacian M = V diag(1 / max(lambda, 1)) V^T, V the orthonormal sine transform
// (DST-I) along each axis, which diagonalises the Dirichlet 7-point Laplacian exactly.
// Returns out + M t with t minimising ||r - A M t|| over K_k(A M, r).  FP64 throughout.
// With a learned network as the inner preconditioner, the steps are flexible GMRES steps
// with z_j = net(v_j) (the network is not linear), and the result is out + sum_j t_j z_j.
//
// The sine transform is a dense contraction along each axis, run as three complex GEMMs
// (rocBLAS): along x, S_x X with X the nx x (ny nz) matrix of the grid (x fastest); along
// y, X_z S_y for every z-slab (a strided batch); along z, X S_z with X the (nx ny) x nz
// matrix.  S_n[j][k] = sqrt(2/(n+1)) sin(pi (j+1)(k+1)/(n+1)) is symmetric and its own
// inverse.
#include <rocblas/rocblas.h>

#include <cmath>
#include <vector>

#include "internal.h"

namespace hfci {

void launch_laplace_scale(hipStream_t st, double2* c, const GridDesc& g);

namespace {

#define HFCI_BLAS(x)                                                                         \
  do {                                                                                       \
    const rocblas_status _s = (x);                                                           \
    if (_s != rocblas_status_success)                                                        \
      throw Error(HFCI_E_HIP, std::string("rocBLAS: ") + rocblas_status_to_string(_s));      \
  } while (0)

rocblas_handle blas_of(Ctx& ctx) {
  if (!ctx.blas) {
    rocblas_handle h = nullptr;
    HFCI_BLAS(rocblas_create_handle(&h));
    ctx.blas = h;
  }
  rocblas_handle h = (rocblas_handle)ctx.blas;
  HFCI_BLAS(rocblas_set_stream(h, ctx.stream));
  return h;
}

// the orthonormal DST-I matrix of size n as complex entries (imaginary parts zero), cached
const rocblas_double_complex* sine_matrix(Ctx& ctx, int n) {
  auto it = ctx.sine.find(n);
  if (it != ctx.sine.end()) return (const rocblas_double_complex*)it->second;
  std::vector<double2> h((size_t)n * n);
  const double sc = std::sqrt(2.0 / (n + 1));
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k) h[(size_t)j * n + k] = make_double2(sc * std::sin(M_PI * (j + 1) * (k + 1) / (n + 1)), 0.0);
  double2* d = nullptr;
  HFCI_HIP(hipMalloc(&d, h.size() * sizeof(double2)));
  ctx.sine[n] = d;
  HFCI_HIP(hipMemcpy(d, h.data(), h.size() * sizeof(double2), hipMemcpyHostToDevice));
  return (const rocblas_double_complex*)d;
}

// out = (S_z (x) S_y (x) S_x) in, using tmp; in, out and tmp distinct
void sine3(Ctx& ctx, const GridDesc& g, const double2* in, double2* out, double2* tmp) {
  rocblas_handle h = blas_of(ctx);
  const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const auto* Sx = sine_matrix(ctx, nx);
  const auto* Sy = sine_matrix(ctx, ny);
  const auto* Sz = sine_matrix(ctx, nz);
  auto C = [](const double2* p) { return (const rocblas_double_complex*)p; };
  auto Cm = [](double2* p) { return (rocblas_double_complex*)p; };
  // along x: out = S_x * in (nx x ny nz)
  HFCI_BLAS(rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, nx, ny * nz, nx, &one, Sx, nx, C(in),
                          nx, &zero, Cm(out), nx));
  // along y: tmp_z = out_z * S_y for every z-slab (nx x ny)
  HFCI_BLAS(rocblas_zgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_none, nx, ny, ny, &one,
                                          C(out), nx, (rocblas_stride)nx * ny, Sy, ny, 0, &zero, Cm(tmp), nx,
                                          (rocblas_stride)nx * ny, nz));
  // along z: out = tmp * S_z ((nx ny) x nz)
  HFCI_BLAS(rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, nx * ny, nz, nz, &one, C(tmp), nx * ny,
                          Sz, nz, &zero, Cm(out), nx * ny));
}

// Givens rotation (c, s) with [c s; -conj(s) c] [a; b] = [rho; 0], c real
void rotation(cd a, cd b, double& c, cd& s, cd& rho) {
  if (std::abs(a) == 0.0) {
    c = 0.0;
    s = cd(1.0, 0.0);
    rho = b;
    return;
  }
  const double nrm = std::sqrt(std::norm(a) + std::norm(b));
  const cd ph = a / std::abs(a);
  c = std::abs(a) / nrm;
  s = ph * std::conj(b) / nrm;
  rho = ph * nrm;
}

}  // namespace

void laplace_inverse(Ctx& ctx, const GridDesc& g, const double2* x, double2* y) {
  const size_t npt = (size_t)g.nx * g.ny * g.nz;
  HFCI_REQUIRE((long long)g.ny * g.nz < (1LL << 31) && (long long)g.nx * g.ny < (1LL << 31),
               "grid too large for the inner preconditioner's GEMMs");
  double2* t1 = (double2*)ctx.ws.get("in_t1", npt * sizeof(double2));
  double2* t2 = (double2*)ctx.ws.get("in_t2", npt * sizeof(double2));
  sine3(ctx, g, x, t1, t2);
  launch_laplace_scale(ctx.stream, t1, g);
  sine3(ctx, g, t1, y, t2);
}

void inner_release(Ctx& ctx) {
  if (ctx.blas) (void)rocblas_destroy_handle((rocblas_handle)ctx.blas);
  ctx.blas = nullptr;
  for (auto& kv : ctx.sine) (void)hipFree(kv.second);
  ctx.sine.clear();
}

void inner_steps(const Op& op, int k_in, int nrhs, const double2* f, double2* out, FciStats& st, Net* net) {
  Ctx& ctx = *op.ctx;
  hipStream_t s = ctx.stream;
  const size_t n = op.n;
  const int k = k_in;
  double2* V = (double2*)ctx.ws.get("in_V", (size_t)(k + 1) * n * sizeof(double2));
  double2* Z = (double2*)ctx.ws.get("in_Z", (size_t)k * n * sizeof(double2));
  const int nbs = Launch<double2>::partial_blocks(op.g);
  const int nbb = blas_blocks(n);
  double* part = (double*)ctx.ws.get("in_part", (size_t)std::max(nbs, nbb * 2 * (k + 1)) * sizeof(double));
  // h1[2(k+1)], h2[2(k+1)], nrm2, beta2, y[2k]
  const int hs = 4 * (k + 1) + 2 + 2 * k;
  double* hd = (double*)ctx.ws.get("in_h", (size_t)hs * sizeof(double));
  double* hh = ctx.pinned_dbl + kPinnedFciOffset + 2048;
  double* h1 = hd;
  double* h2 = hd + 2 * (k + 1);
  double* nrm2 = hd + 4 * (k + 1);
  double* beta2 = nrm2 + 1;
  double* yd = beta2 + 1;
  for (int r = 0; r < nrhs; ++r) {
    double2* outr = out + (size_t)r * n;
    // remainder f - A out (= f - d A w) and its norm
    launch_residual64(s, op.g, op.kappa64, f + (size_t)r * n, outr, V, part);
    launch_reduce(s, part, nbs, 1, beta2);
    HFCI_HIP(hipMemcpyAsync(hh, beta2, sizeof(double), hipMemcpyDeviceToHost, s));
    HFCI_HIP(hipStreamSynchronize(s));
    const double beta = std::sqrt(hh[0]);
    if (!(beta > 0.0)) continue;  // nothing left (or NaN: FGMRES reports it)
    launch_scale_inv(s, V, V, n, beta2);
    std::vector<cd> H((size_t)(k + 1) * k, cd(0, 0)), G(k + 1, cd(0, 0)), SN(k);
    std::vector<double> CS(k);
    G[0] = beta;
    auto Hat = [&](int i, int j) -> cd& { return H[(size_t)i * k + j]; };
    int kk = 0;
    for (int j = 0; j < k; ++j) {
      if (net)
        net->apply(op, 1, V + (size_t)j * n, Z + (size_t)j * n);
      else
        laplace_inverse(ctx, op.g, V + (size_t)j * n, Z + (size_t)j * n);
      double2* w = V + (size_t)(j + 1) * n;
      Launch<double2>::apply(s, op.g, op.kappa64, 0.0, 0.0, 1, Z + (size_t)j * n, w);
      launch_cgs2(s, V, j + 1, n, n, w, part, h1, h2, nrm2);
      launch_scale_inv(s, w, w, n, nrm2);
      HFCI_HIP(hipMemcpyAsync(hh, hd, (4 * (k + 1) + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
      HFCI_HIP(hipStreamSynchronize(s));
      st.matvecs += 1;
      for (int i = 0; i <= j; ++i)
        Hat(i, j) = cd(hh[2 * i] + hh[2 * (k + 1) + 2 * i], hh[2 * i + 1] + hh[2 * (k + 1) + 2 * i + 1]);
      const double hn = std::sqrt(hh[4 * (k + 1)]);
      if (!(hn == hn)) throw Error(HFCI_E_NUMERIC, "NaN in the inner GMRES steps");
      Hat(j + 1, j) = hn;
      for (int i = 0; i < j; ++i) {
        const cd x = Hat(i, j), yv = Hat(i + 1, j);
        Hat(i, j) = CS[i] * x + SN[i] * yv;
        Hat(i + 1, j) = -std::conj(SN[i]) * x + CS[i] * yv;
      }
      double cs;
      cd sn, rho;
      rotation(Hat(j, j), Hat(j + 1, j), cs, sn, rho);
      CS[j] = cs;
      SN[j] = sn;
      Hat(j, j) = rho;
      Hat(j + 1, j) = 0.0;
      G[j + 1] = -std::conj(sn) * G[j];
      G[j] = cs * G[j];
      kk = j + 1;
      if (!(hn > 0.0)) break;  // the Krylov space is invariant: the remainder is solved
    }
    std::vector<cd> y(kk);
    for (int i = kk - 1; i >= 0; --i) {
      cd acc = G[i];
      for (int l = i + 1; l < kk; ++l) acc -= Hat(i, l) * y[l];
      y[i] = acc / Hat(i, i);
    }
    for (int i = 0; i < kk; ++i) {
      hh[2 * i] = y[i].real();
      hh[2 * i + 1] = y[i].imag();
    }
    HFCI_HIP(hipMemcpyAsync(yd, hh, 2 * kk * sizeof(double), hipMemcpyHostToDevice, s));
    launch_multiaxpy(s, outr, Z, kk, n, n, yd, 1.0);
    // the pinned staging is reused by the next right-hand side: wait for the copy
    HFCI_HIP(hipStreamSynchronize(s));
  }
}

}  // namespace hfci
