// Case-two shifted solves (Sec. 3 eq. mat-2x2, Sec. 4.2 eq. fix-pt-exp): for every pole
// z_j of a contour built on B's spectrum box and every right-hand side g_r (vectors of
// 2 n values), the polynomial fixed-point iteration for (B - z_j) y = g_r from y = 0,
// in the product form of params.cpp: step one builds y1 = P2(B) g / p~(z) with
// max(q-1, 1) factors; every later step is y <- L y + y1 with q factors, the first of
// which also forms the residual partials of the current y for the stopping test
// ||g - (B - z) y|| <= ||g|| / reduce.  One launch per factor covers every system still
// iterating (stopped systems skip their blocks); the host reads the flags once a step.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace hfci {

void launch_copy_active_f(hipStream_t st, float2* dst, const float2* src, const int* active, int nsys, size_t n);
void launch_copy_active_d(hipStream_t st, double2* dst, const double2* src, const int* active, int nsys,
                          size_t n);

namespace {

template <typename T2> const void* kappa_for(const Op& op);
template <> const void* kappa_for<float2>(const Op& op) { return op.kappa32; }
template <> const void* kappa_for<double2>(const Op& op) { return op.kappa64; }

void copy_active(hipStream_t st, float2* d, const float2* s, const int* a, int nsys, size_t n) {
  launch_copy_active_f(st, d, s, a, nsys, n);
}
void copy_active(hipStream_t st, double2* d, const double2* s, const int* a, int nsys, size_t n) {
  launch_copy_active_d(st, d, s, a, nsys, n);
}

}  // namespace

template <typename T2>
void shifted_solve_case_two(const Op& op, const Contour& c, int nrhs, const T2* f, T2* y, int fixed_steps,
                            double reduce, int max_steps, int* steps_out, FciStats& st) {
  Ctx& ctx = *op.ctx;
  hipStream_t s = ctx.stream;
  const GridDesc& g = op.g;
  const size_t n2 = op.n;  // 2 n values per vector of B
  const int J = c.J, q = c.q, nsys = J * nrhs;
  const bool fixed = fixed_steps > 0;
  HFCI_REQUIRE(nsys <= kPinnedIntHalf, "too many shifted systems");
  const bool f32 = sizeof(T2) == 8;
  const size_t vb = n2 * sizeof(T2);
  T2* y1 = (T2*)ctx.ws.get("c2_y1", (size_t)nsys * vb);
  T2* wA = (T2*)ctx.ws.get("c2_wA", (size_t)nsys * vb);
  T2* wB = q >= 3 ? (T2*)ctx.ws.get("c2_wB", (size_t)nsys * vb) : nullptr;
  const int nblk = b2_blocks(g);
  double* partial = (double*)ctx.ws.get("c2_partial", (size_t)nsys * nblk * sizeof(double));
  const int nbf = blas_blocks(n2);
  double* fpart = (double*)ctx.ws.get("c2_fpart", (size_t)nbf * sizeof(double));
  double* fnorm2 = (double*)ctx.ws.get("c2_fnorm2", (size_t)nrhs * sizeof(double));
  double* rnorm2 = (double*)ctx.ws.get("c2_rnorm2", (size_t)nsys * sizeof(double));
  int* active = (int*)ctx.ws.get("c2_active", (size_t)nsys * sizeof(int));
  int* steps = (int*)ctx.ws.get("c2_steps", (size_t)nsys * sizeof(int));
  int* list = (int*)ctx.ws.get("c2_list", (size_t)nsys * sizeof(int));
  for (int r = 0; r < nrhs; ++r) {
    launch_norm2_partial(s, f + (size_t)r * n2, f32, n2, fpart);
    launch_reduce(s, fpart, nbf, 1, fnorm2 + r);
  }
  // every system active for step one
  launch_fp_start(s, nsys, 0, nrhs, fnorm2, true, active, steps, list);

  B2Args<T2> a{};
  a.f = f;
  a.y1 = y1;
  a.coef = c.d_coef;
  a.poles = c.d_poles;
  a.active = active;
  a.partial = partial;
  a.nrhs = nrhs;
  a.cstride = c.cstride;
  const void* K = kappa_for<T2>(op);
  auto factor = [&](int kind, int k, const T2* in, T2* out, T2* out2) {
    a.win = in;
    a.wout = out;
    a.wout2 = out2;
    a.k = k;
    const bool ok = launch_b2_factor<T2>(s, g, K, kind, nsys, a);
    HFCI_REQUIRE(ok, "internal: unsupported factor kind");
  };

  // step one: the max(q-1, 1) factors of P2 from g; the last writes y1 and y
  const int nP = std::max(q - 1, 1);
  {
    const T2* cur = f;
    for (int i = 0; i < nP; ++i) {
      const bool first = i == 0, last = i + 1 == nP;
      T2* dst = last ? y1 : (cur == wA ? wB : wA);
      int kind = first ? kFacInF : 0;
      if (last) kind |= kFacDual;
      factor(kind, q + i, cur, dst, last ? y : nullptr);
      cur = dst;
    }
    st.matvecs += (long long)nP * nsys;
    st.fp_steps += nsys;
  }
  // after step one: zero right-hand sides stop with y = 0 (adaptive mode)
  launch_fp_start(s, nsys, 0, nrhs, fnorm2, fixed, active, steps, list);
  int nact = nsys;
  const int cap = fixed ? fixed_steps : max_steps;
  for (int it = 1; it <= cap; ++it) {
    if (fixed && it == cap) break;
    // head: the first factor of L on y (with the residual of y when adaptive)
    const int head_kind = (fixed ? 0 : kFacResid) | (q == 1 ? kFacAdd : 0);
    factor(head_kind, 0, y, wA, nullptr);
    st.matvecs += nact;
    if (!fixed) {
      launch_fp_test(s, partial, nblk, nsys, 0, nrhs, fnorm2, reduce, max_steps, active, steps, rnorm2, list,
                     ctx.pinned_int_dev);
      HFCI_HIP(hipStreamSynchronize(s));
      nact = 0;
      for (int k = 0; k < nsys; ++k) nact += ctx.pinned_int[k] != 0;
      if (nact == 0) break;
    }
    if (q == 1) {
      copy_active(s, y, wA, active, nsys, n2);
    } else {
      const T2* cur = wA;
      for (int k = 1; k < q; ++k) {
        const bool last = k + 1 == q;
        T2* dst = last ? y : (cur == wA ? wB : wA);
        factor(last ? kFacAdd : 0, k, cur, dst, nullptr);
        cur = dst;
      }
    }
    st.matvecs += (long long)(q - 1) * nact;
    st.fp_steps += nact;
  }
  if (steps_out && fixed) {
    std::fill(steps_out, steps_out + nsys, fixed_steps);
  } else if (steps_out) {
    HFCI_HIP(hipMemcpyAsync(ctx.pinned_int, steps, nsys * sizeof(int), hipMemcpyDeviceToHost, s));
    HFCI_HIP(hipStreamSynchronize(s));
    std::memcpy(steps_out, ctx.pinned_int, nsys * sizeof(int));
  }
}

template void shifted_solve_case_two<float2>(const Op&, const Contour&, int, const float2*, float2*, int, double,
                                             int, int*, FciStats&);
template void shifted_solve_case_two<double2>(const Op&, const Contour&, int, const double2*, double2*, int,
                                              double, int, int*, FciStats&);

}  // namespace hfci
