// Case-two shifted solves (Sec. 3 eq. mat-2x2, Sec. 4.2 eq. fix-pt-exp): for every pole
// z_j of a contour built on B's spectrum box and every right-hand side g_r (vectors of
// 2 n values), the polynomial fixed-point iteration for (B - z_j) y = g_r from y = 0 (the
// loop of fp_simple.h) with pairs on: two factors per launch where the step allows, one for
// a leading factor of step one or a trailing factor of an odd q (b2_zm_kernel), all systems
// at once.
#include "fp_simple.h"

namespace hfci {

namespace {

template <typename T2> const void* kappa_for(const Op& op);
template <> const void* kappa_for<float2>(const Op& op) { return op.kappa32; }
template <> const void* kappa_for<double2>(const Op& op) { return op.kappa64; }

}  // namespace

template <typename T2>
void shifted_solve_case_two(const Op& op, const Contour& c, int nrhs, const T2* f, T2* y, int fixed_steps,
                            double reduce, int max_steps, int* steps_out, FciStats& st) {
  hipStream_t s = op.ctx->stream;
  const void* K = kappa_for<T2>(op);
  fp_simple<T2>(op, c, nrhs, f, y, fixed_steps, reduce, max_steps, steps_out, st, b2_blocks(op.g), true,
                [&](const SimpleFactor<T2>& sf) {
                  B2Args<T2> a{};
                  a.win = sf.in;
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
                  const bool ok = sf.nfac == 2 ? launch_b2_pair<T2>(s, op.g, K, sf.kind, sf.nsys, a)
                                               : launch_b2_factor<T2>(s, op.g, K, sf.kind, sf.nsys, a);
                  HFCI_REQUIRE(ok, "internal: unsupported factor kind");
                });
}

template void shifted_solve_case_two<float2>(const Op&, const Contour&, int, const float2*, float2*, int, double,
                                             int, int*, FciStats&);
template void shifted_solve_case_two<double2>(const Op&, const Contour&, int, const double2*, double2*, int,
                                              double, int, int*, FciStats&);

}  // namespace hfci
