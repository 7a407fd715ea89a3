// Host-side parameters of the method: spectrum rectangle, contour poles and weights,
// the delta search of the exponential-Taylor iteration, and the Horner stage
// coefficients that the stage kernels consume.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace hfci {

// Lemma 3.1 rectangle for A = S - M - iD: Re in [lmin(S) - max kappa, lmax(S) - min kappa]
// (Weyl bounds with the exact extreme eigenvalues 2(1 -+ cos(pi/(n+1))) per axis of the
// Dirichlet 7-point Laplacian), Im in [-rho(D), 0] with rho(D) = rho2 at the boundary nodes.
void op_rectangle(Op& op) {
  double lo = 0.0, hi = 0.0;
  for (int n : {op.g.nx, op.g.ny, op.g.nz}) {
    const double c = std::cos(M_PI / (n + 1));
    lo += 2.0 * (1.0 - c);
    hi += 2.0 * (1.0 + c);
  }
  op.b1 = op.s_h2 * lo - op.kmax;
  op.b2 = op.s_h2 * hi - op.kmin;
  op.rho2 = (op.damp_cells > 0) ? op.damp_rho2 : 0.0;
}

// Sec. 6.2 eq. quad-points / quad-radius with the weights of eq. ellipse (Sec. 6.1):
// theta_j = (2j-1) pi/J, r = (rho2/2 + eps)/sin(pi/J),
// z_j = t r (cos theta_j - cos(pi/J)) + i (r sin theta_j - rho2/2),
// sigma_j = (r cos theta_j + i t r sin theta_j)/J.
void contour_poles(int J, double t, double eps, double rho2, std::vector<cd>& z, std::vector<cd>& sigma) {
  const double phi = M_PI / J;
  const double r = (0.5 * rho2 + eps) / std::sin(phi);
  z.resize(J);
  sigma.resize(J);
  for (int j = 1; j <= J; ++j) {
    const double th = (2 * j - 1) * phi;
    z[j - 1] = cd(t * r * (std::cos(th) - std::cos(phi)), r * std::sin(th) - 0.5 * rho2);
    sigma[j - 1] = cd(r * std::cos(th), t * r * std::sin(th)) / (double)J;
  }
}

// p~^(q)(lambda) = sum_{j<=q} (-i delta (lambda - z0))^j / j!   (eq. exp-taylor), Horner form.
cd ptilde(cd lam, cd z0, double delta, int q) {
  const cd x = cd(0.0, -delta) * (lam - z0);
  cd acc(1.0, 0.0);
  for (int j = q; j >= 1; --j) acc = 1.0 + acc * x / (double)j;
  return acc;
}

std::vector<cd> rectangle_boundary(double b1, double b2, double rho2, int per_side) {
  std::vector<cd> b;
  b.reserve(4 * (per_side + 1));
  for (int k = 0; k <= per_side; ++k) {
    const double t = (double)k / per_side;
    const double re = b1 + (b2 - b1) * t;
    b.emplace_back(re, 0.0);
    b.emplace_back(re, -rho2);
    b.emplace_back(b1, -rho2 * t);
    b.emplace_back(b2, -rho2 * t);
  }
  return b;
}

double rate_on_boundary(double delta, cd z, cd z0, int q, const std::vector<cd>& boundary) {
  double m = 0.0;
  for (const cd& l : boundary) m = std::max(m, std::abs(ptilde(l, z0, delta, q)));
  return m / std::abs(ptilde(z, z0, delta, q));
}

// eq. fix-pt-conv: nu = min over real delta of max over the rectangle boundary of
// |p~(lambda)/p~(z)|, with z0 = (b1+b2)/2 + i Im z and sign(delta) = sign(Im z).
// A geometric scan of |delta| brackets the minimum, golden-section search refines it.
void optimise_delta(cd z, double b1, double b2, double rho2, int q, double& delta, double& nu, cd& z0) {
  z0 = cd(0.5 * (b1 + b2), z.imag());
  const double sgn = z.imag() > 0 ? 1.0 : -1.0;
  const std::vector<cd> bd = rectangle_boundary(b1, b2, rho2, 2000);
  const int ns = 480;
  const double lo = 1e-4, hi = 50.0;
  std::vector<double> ds(ns), vs(ns);
  int best = 0;
  for (int k = 0; k < ns; ++k) {
    ds[k] = lo * std::pow(hi / lo, (double)k / (ns - 1));
    vs[k] = rate_on_boundary(sgn * ds[k], z, z0, q, bd);
    if (vs[k] < vs[best]) best = k;
  }
  double a = ds[std::max(best - 1, 0)], b = ds[std::min(best + 1, ns - 1)];
  const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
  double c = b - gr * (b - a), d = a + gr * (b - a);
  double fc = rate_on_boundary(sgn * c, z, z0, q, bd), fd = rate_on_boundary(sgn * d, z, z0, q, bd);
  for (int it = 0; it < 80 && (b - a) > 1e-12 * b; ++it) {
    if (fc < fd) {
      b = d; d = c; fd = fc;
      c = b - gr * (b - a);
      fc = rate_on_boundary(sgn * c, z, z0, q, bd);
    } else {
      a = c; c = d; fc = fd;
      d = a + gr * (b - a);
      fd = rate_on_boundary(sgn * d, z, z0, q, bd);
    }
  }
  double dm = 0.5 * (a + b);
  double vm = rate_on_boundary(sgn * dm, z, z0, q, bd);
  if (vs[best] < vm) {
    dm = ds[best];
    vm = vs[best];
  }
  delta = sgn * dm;
  nu = vm;
}

// Horner re-association of one step of eq. fix-pt-exp.  With B = -i delta (A - z0 I),
// beta = -i delta (z - z0), g = i delta f, the step's unrolled recursion gives
//   y + k_1 + ... + k_q = sum_{m=0..q} B^m a_m,  a_m = y/m! + e_m g,
//   e_m = sum_{j=m+1..q} beta^(j-1-m)/j!   (e_q = 0),
// so y_new = (Horner over m = q..0) / p~(z).  Stage m (q-1 down to 0) computes
//   w_m = cB_m (A - z0) w_{m+1} + alpha_m y + gamma_m f
// with w_q = y (the 1/q! is folded into cB_{q-1}) and 1/p~(z) folded into stage 0.
void stage_coefficients(cd z, cd z0, double delta, int q, StageCoef* out, cd& pz) {
  const cd beta = cd(0.0, -delta) * (z - z0);
  pz = ptilde(z, z0, delta, q);
  const cd inv_pz = 1.0 / pz;
  std::vector<double> fact(q + 1, 1.0);
  for (int j = 1; j <= q; ++j) fact[j] = fact[j - 1] * j;
  for (int m = 0; m < q; ++m) {
    cd e(0.0, 0.0), bp(1.0, 0.0);
    for (int j = m + 1; j <= q; ++j) {
      e += bp / fact[j];
      bp *= beta;
    }
    cd cB = cd(0.0, -delta);
    if (m == q - 1) cB /= fact[q];
    cd al = cd(1.0 / fact[m], 0.0);
    cd ga = cd(0.0, delta) * e;
    if (m == 0) {
      cB *= inv_pz;
      al *= inv_pz;
      ga *= inv_pz;
    }
    out[m] = StageCoef{cB.real(), cB.imag(), al.real(), al.imag(), ga.real(), ga.imag()};
  }
}

}  // namespace hfci
