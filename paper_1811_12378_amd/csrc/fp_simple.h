// Shifted solves with one launch per factor (or per pair of factors) over every shifted
// system, for the operators without the z-marching stencil kernels (case two, the
// Fourier-spectral operator): the loop of the product-form fixed-point iteration
// (eq. fix-pt-exp, factors of params.cpp) for (A - z_j) y = g_r from y = 0.  Step one
// builds y1 = P2(A) g / p~(z) with max(q-1, 1) factors; every later step is y <- L y + y1
// with q factors, the first of which also forms the residual partials of the current y for
// the stopping test
// ||g - (A - z) y|| <= ||g|| / reduce.  Stopped systems skip their blocks; the host reads
// the flags once a step.  The operator supplies one factor launch, and optionally a launch
// of two consecutive factors in one pass: step one then runs as a leading single factor
// when q - 1 is odd plus pairs, and a later step as pairs (the first with the residual of
// its input) plus a trailing single factor when q is odd.
#pragma once

#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"

namespace hfci {

void launch_copy_active_f(hipStream_t st, float2* dst, const float2* src, const int* active, int nsys, size_t n);
void launch_copy_active_d(hipStream_t st, double2* dst, const double2* src, const int* active, int nsys,
                          size_t n);

// What a factor launch of the loop below needs: system s = pole * nrhs + rhs, vectors of
// n values strided by n (the right-hand sides per rhs), residual partials [nsys][nblk].
template <typename T2>
struct SimpleFactor {
  int kind, k;                 // kFac* bits; coefficient index within the pole's cstride
  int nfac;                    // factors of this launch: 1, or 2 (k and k + 1; kFacResid and
                               // kFacInF apply to the input, kFacAdd and kFacDual to the output)
  const T2* in;                // per system, or per rhs with kFacInF
  T2* out;                     // per system
  T2* out2;                    // per system (kFacDual)
  const T2* f;                 // right-hand sides (kFacResid, kFacInF)
  const T2* y1;                // per system (kFacAdd)
  const int* active;           // [nsys] (device)
  const int* host_active;      // [nsys] (host): the systems this launch runs
  double* partial;             // [nsys][nblk] (kFacResid)
  int nrhs, nsys;
};

inline void copy_active_sys(hipStream_t st, float2* d, const float2* s, const int* a, int nsys, size_t n) {
  launch_copy_active_f(st, d, s, a, nsys, n);
}
inline void copy_active_sys(hipStream_t st, double2* d, const double2* s, const int* a, int nsys, size_t n) {
  launch_copy_active_d(st, d, s, a, nsys, n);
}

// nblk: residual partials per system of the operator's factor launch; factor(const
// SimpleFactor<T2>&) launches sf.nfac factors over all systems, and is given nfac = 2 only
// when pairs is set.
template <typename T2, typename Factor>
void fp_simple(const Op& op, const Contour& c, int nrhs, const T2* f, T2* y, int fixed_steps, double reduce,
               int max_steps, int* steps_out, FciStats& st, int nblk, bool pairs, Factor&& factor) {
  Ctx& ctx = *op.ctx;
  hipStream_t s = ctx.stream;
  const size_t n = op.n;
  const int J = c.J, q = c.q, nsys = J * nrhs;
  const bool fixed = fixed_steps > 0;
  HFCI_REQUIRE(nsys <= kPinnedIntHalf, "too many shifted systems");
  const bool f32 = sizeof(T2) == 8;
  const size_t vb = n * sizeof(T2);
  T2* y1 = (T2*)ctx.ws.get("sf_y1", (size_t)nsys * vb);
  T2* wA = (T2*)ctx.ws.get("sf_wA", (size_t)nsys * vb);
  T2* wB = q >= 3 ? (T2*)ctx.ws.get("sf_wB", (size_t)nsys * vb) : nullptr;
  double* partial = (double*)ctx.ws.get("sf_partial", (size_t)nsys * nblk * sizeof(double));
  const int nbf = blas_blocks(n);
  double* fpart = (double*)ctx.ws.get("sf_fpart", (size_t)nbf * sizeof(double));
  double* fnorm2 = (double*)ctx.ws.get("sf_fnorm2", (size_t)nrhs * sizeof(double));
  double* rnorm2 = (double*)ctx.ws.get("sf_rnorm2", (size_t)nsys * sizeof(double));
  int* active = (int*)ctx.ws.get("sf_active", (size_t)nsys * sizeof(int));
  int* steps = (int*)ctx.ws.get("sf_steps", (size_t)nsys * sizeof(int));
  int* list = (int*)ctx.ws.get("sf_list", (size_t)nsys * sizeof(int));
  for (int r = 0; r < nrhs; ++r) {
    launch_norm2_partial(s, f + (size_t)r * n, f32, n, fpart);
    launch_reduce(s, fpart, nbf, 1, fnorm2 + r);
  }
  // every system active for step one
  launch_fp_start(s, nsys, 0, nrhs, fnorm2, true, active, steps, list);
  std::vector<int> hact(nsys, 1);
  SimpleFactor<T2> a{};
  a.host_active = hact.data();
  a.f = f;
  a.y1 = y1;
  a.active = active;
  a.partial = partial;
  a.nrhs = nrhs;
  a.nsys = nsys;
  auto run = [&](int kind, int k, const T2* in, T2* out, T2* out2, int nfac) {
    a.kind = kind;
    a.k = k;
    a.nfac = nfac;
    a.in = in;
    a.out = out;
    a.out2 = out2;
    factor(a);
  };
  // step one: the max(q-1, 1) factors of P2 from g; the last writes y1 and y
  const int nP = std::max(q - 1, 1);
  {
    const T2* cur = f;
    for (int i = 0; i < nP;) {
      const int nf = pairs && (nP - i) % 2 == 0 ? 2 : 1;
      const bool first = i == 0, last = i + nf == nP;
      T2* dst = last ? y1 : (cur == wA ? wB : wA);
      int kind = first ? kFacInF : 0;
      if (last) kind |= kFacDual;
      run(kind, q + i, cur, dst, last ? y : nullptr, nf);
      cur = dst;
      i += nf;
    }
    st.matvecs += (long long)nP * nsys;
    st.fp_steps += nsys;
  }
  // after step one: zero right-hand sides stop with y = 0 (adaptive mode)
  launch_fp_start(s, nsys, 0, nrhs, fnorm2, fixed, active, steps, list);
  int nact = nsys;
  const int cap = fixed ? fixed_steps : max_steps;
  // factors of the head launch of a later step
  const int nh = pairs && q >= 2 ? 2 : 1;
  for (int it = 1; it <= cap; ++it) {
    if (fixed && it == cap) break;
    // head: the first factor (or pair) of L on y, with the residual of y when adaptive
    const int head_kind = (fixed ? 0 : kFacResid) | (q == nh ? kFacAdd : 0);
    run(head_kind, 0, y, wA, nullptr, nh);
    st.matvecs += (long long)nh * nact;
    if (!fixed) {
      launch_fp_test(s, partial, nblk, nsys, 0, nrhs, fnorm2, reduce, max_steps, active, steps, rnorm2, list,
                     ctx.pinned_int_dev);
      HFCI_HIP(hipStreamSynchronize(s));
      nact = 0;
      for (int k = 0; k < nsys; ++k) {
        hact[k] = ctx.pinned_int[k] != 0;
        nact += hact[k];
      }
      if (nact == 0) break;
    }
    if (q == nh) {
      // the head wrote the whole step (a launch never writes its own input)
      copy_active_sys(s, y, wA, active, nsys, n);
    } else {
      const T2* cur = wA;
      for (int k = nh; k < q;) {
        const int nf = pairs && k + 1 < q ? 2 : 1;
        const bool last = k + nf == q;
        T2* dst = last ? y : (cur == wA ? wB : wA);
        run(last ? kFacAdd : 0, k, cur, dst, nullptr, nf);
        cur = dst;
        k += nf;
      }
    }
    st.matvecs += (long long)(q - nh) * nact;
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

}  // namespace hfci
