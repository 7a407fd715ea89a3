// Host-side parameters of the method: spectrum rectangle, contour poles and weights,
// the delta search of the exponential-Taylor iteration, and the linear-factor
// coefficients of its product form that the stage kernels consume.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <exception>
#include <thread>

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
void optimise_delta(cd z, double b1, double b2, double rho2, int q, double& delta, double& nu, cd& z0, int per_side,
                    int ns) {
  z0 = cd(0.5 * (b1 + b2), z.imag());
  const double sgn = z.imag() > 0 ? 1.0 : -1.0;
  const std::vector<cd> bd = rectangle_boundary(b1, b2, rho2, per_side);
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

// Sec. 4.2: the degree q is preferred where nu^(1/q) is smallest (the cost to reduce the
// residual by a factor F is about q ln F / (-ln nu) products).  Where the products run
// per_pass at a time in one pass over HBM (the finite-difference operators' two-factor
// kernels), the cost is ceil(q / per_pass) ln F / (-ln nu) passes, and that is minimised;
// per_pass = 1 is the rule as written.  q in 1..qmax, ties to the smaller q.
int choose_q(cd z, double b1, double b2, double rho2, int qmax, int per_pass) {
  std::vector<double> nu(std::max(qmax, 0) + 1, HUGE_VAL);
  host_parallel_for(qmax, [&](int i) {
    double delta;
    cd z0;
    optimise_delta(z, b1, b2, rho2, i + 1, delta, nu[i + 1], z0);
  });
  int best = 1;
  double cost_best = HUGE_VAL;
  for (int q = 1; q <= qmax; ++q) {  // in order: ties go to the smaller q
    if (!(nu[q] < 1.0)) continue;
    const double cost = (double)((q + per_pass - 1) / per_pass) / -std::log(nu[q]);
    if (cost < cost_best) {
      best = q;
      cost_best = cost;
    }
  }
  return best;
}

// f(0), ..., f(n - 1) on up to hardware_concurrency host threads (each index once; the
// calls must be independent); the first exception a call throws is rethrown here
void host_parallel_for(int n, const std::function<void(int)>& f) {
  if (n <= 0) return;
  const int nt = std::max(1, std::min(n, (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()))));
  if (nt == 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int> next{0};
  std::exception_ptr err;
  std::atomic<bool> failed{false};
  auto work = [&] {
    for (int i; (i = next.fetch_add(1)) < n;) {
      if (failed.load()) return;
      try {
        f(i);
      } catch (...) {
        if (!failed.exchange(true)) err = std::current_exception();
        return;
      }
    }
  };
  std::vector<std::thread> th;
  th.reserve(nt - 1);
  for (int k = 1; k < nt; ++k) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
  if (err) std::rethrow_exception(err);
}

// max over the boundary of |p~(lambda)| / |p~(z)| with the complex products written out
// (the rule evaluates it some 10^5 times per call; std::complex's checked products are
// several times slower)
static double rate_plain(double delta, cd z, cd z0, int q, const std::vector<cd>& bd) {
  auto pt_abs2 = [&](double lr, double li) {
    // x = -i delta (lambda - z0) = delta (Im(lambda - z0)) - i delta Re(lambda - z0)
    const double xr = delta * (li - z0.imag()), xi = -delta * (lr - z0.real());
    double ar = 1.0, ai = 0.0;
    for (int j = q; j >= 1; --j) {
      const double inv = 1.0 / j;
      const double tr = (ar * xr - ai * xi) * inv, ti = (ar * xi + ai * xr) * inv;
      ar = 1.0 + tr;
      ai = ti;
    }
    return ar * ar + ai * ai;
  };
  double m = 0.0;
  for (const cd& l : bd) m = std::max(m, pt_abs2(l.real(), l.imag()));
  return std::sqrt(m / pt_abs2(z.real(), z.imag()));
}

// eq. fix-pt-conv's nu for the rule: a geometric scan of |delta| and a short golden-section
// refinement (the rule needs nu to a few digits)
static double rule_nu(cd z, double b1, double b2, double rho2, int q, const std::vector<cd>& bd) {
  const cd z0(0.5 * (b1 + b2), z.imag());
  const double sgn = z.imag() > 0 ? 1.0 : -1.0;
  const double lo = 1e-4, hi = 50.0;
  int best = 0;
  double vbest = HUGE_VAL;
  auto d_at = [&](int k) { return lo * std::pow(hi / lo, (double)k / (kRuleScan - 1)); };
  for (int k = 0; k < kRuleScan; ++k) {
    const double v = rate_plain(sgn * d_at(k), z, z0, q, bd);
    if (v < vbest) {
      vbest = v;
      best = k;
    }
  }
  double a = d_at(std::max(best - 1, 0)), b = d_at(std::min(best + 1, kRuleScan - 1));
  const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
  double c = b - gr * (b - a), d = a + gr * (b - a);
  double fc = rate_plain(sgn * c, z, z0, q, bd), fd = rate_plain(sgn * d, z, z0, q, bd);
  for (int it = 0; it < 40 && (b - a) > 1e-7 * b; ++it) {
    if (fc < fd) {
      b = d; d = c; fd = fc;
      c = b - gr * (b - a);
      fc = rate_plain(sgn * c, z, z0, q, bd);
    } else {
      a = c; c = d; fc = fd;
      d = a + gr * (b - a);
      fd = rate_plain(sgn * d, z, z0, q, bd);
    }
  }
  return std::min(vbest, std::min(fc, fd));
}

// Contour parameters by rule.  Sec. 7.3 sets eps per frequency with a small fixed J; here
// eps is the value, among kRuleN geometric steps over [kRuleLo, kRuleHi], that minimises a
// predicted solve time
//   T(eps) = eps * (Q sum_j c_j + Q max_j c_j * kRuleLaunch / npoints + kRuleIter),
//   c_j = ceil(kRuleStepFrac ln(reduce) / -ln nu_j),  Q = per_pass * ceil(q / per_pass),
// nu_j being eq. fix-pt-conv's rate for pole j of eq. quad-points at that eps:
// ceil(ln(reduce) / -ln nu_j) steps reduce the residual by `reduce` in the worst case, and
// the adaptive stops take about half of it (kRuleStepFrac), so c_j are the fixed-point
// steps charged to pole j and Q c_j their products (a pass of per_pass factors costs
// per_pass products).  The FGMRES iteration count grows about in proportion to eps;
// per iteration the products of all poles cost their bytes, each launch (as many as the
// slowest pole's products) a latency worth kRuleLaunch grid points of one system's pass,
// and the Arnoldi step with the combine about kRuleIter products.  With q = 0 the degree at
// each eps is Sec. 4.2's choice for the pole nearest the origin, in passes (choose_q's
// cost, over 1..kAutoQMax).  Ties go to the smaller eps; *q_out receives the degree.
double rule_eps(double b1, double b2, double rho2, double npoints, int J, double t, int q, int per_pass,
                double reduce, int* q_out) {
  const std::vector<cd> bd = rectangle_boundary(b1, b2, rho2, kRulePerSide);
  // the candidates are independent: evaluate them on host threads, then take the best in
  // order (ties to the smaller eps)
  std::vector<double> tks(kRuleN, HUGE_VAL);
  std::vector<int> qks(kRuleN, 0);
  host_parallel_for(kRuleN, [&](int k) {
    const double eps = kRuleLo * std::pow(kRuleHi / kRuleLo, (double)k / (kRuleN - 1));
    std::vector<cd> z, sigma;
    contour_poles(J, t, eps, rho2, z, sigma);
    int qk = q;
    if (qk <= 0) {
      int j0 = 0;
      for (int j = 1; j < J; ++j)
        if (std::abs(z[j]) < std::abs(z[j0])) j0 = j;
      double cost_best = HUGE_VAL;
      for (int qq = 1; qq <= kAutoQMax; ++qq) {
        const double nu = rule_nu(z[j0], b1, b2, rho2, qq, bd);
        if (!(nu < 1.0)) continue;
        const double cost = (double)((qq + per_pass - 1) / per_pass) / -std::log(nu);
        if (cost < cost_best) {
          cost_best = cost;
          qk = qq;
        }
      }
      if (qk <= 0) return;  // no degree contracts at this eps
    }
    // poles j and J-1-j are mirror images about Im = -rho2/2, as is the box, so they have
    // the same rate: evaluate the first half and count each twice (the middle pole of an
    // odd J once)
    double sum = 0.0, mx = 0.0;
    for (int j = 0; j < (J + 1) / 2 && std::isfinite(sum); ++j) {
      const double nu = rule_nu(z[j], b1, b2, rho2, qk, bd);
      const double sj = nu < 1.0 ? std::ceil(kRuleStepFrac * std::log(reduce) / -std::log(nu)) : HUGE_VAL;
      sum += (2 * j + 1 == J) ? sj : 2.0 * sj;
      mx = std::max(mx, sj);
    }
    const double Q = (double)(per_pass * ((qk + per_pass - 1) / per_pass));
    tks[k] = eps * (Q * sum + Q * mx * kRuleLaunch / npoints + kRuleIter);
    qks[k] = qk;
  });
  double best_eps = kRuleLo, best_t = HUGE_VAL;
  int best_q = q > 0 ? q : 1;
  for (int k = 0; k < kRuleN; ++k)
    if (tks[k] < best_t) {
      best_t = tks[k];
      best_eps = kRuleLo * std::pow(kRuleHi / kRuleLo, (double)k / (kRuleN - 1));
      best_q = qks[k];
    }
  if (q_out) *q_out = best_q;
  return best_eps;
}

// Roots of sum_k c[k] x^k (c.back() != 0, degree <= 16) by the Aberth-Ehrlich
// simultaneous iteration (Aberth 1973), then two Newton corrections per root.
std::vector<cd> poly_roots(std::vector<cd> c) {
  const int deg = (int)c.size() - 1;
  std::vector<cd> r;
  if (deg < 1) return r;
  const cd lead = c.back();
  for (cd& v : c) v /= lead;
  // start on a circle of the Fujiwara-type radius max |c_k|^(1/(deg-k)), rotated off the axes
  double R = 0.0;
  for (int k = 0; k < deg; ++k) R = std::max(R, std::pow(std::abs(c[k]), 1.0 / (deg - k)));
  R = std::max(R, 1e-3);
  r.resize(deg);
  for (int k = 0; k < deg; ++k) r[k] = std::polar(R, 2.0 * M_PI * k / deg + 0.4);
  auto eval = [&](cd x, cd& p, cd& dp) {
    p = c[deg];
    dp = 0.0;
    for (int k = deg - 1; k >= 0; --k) {
      dp = dp * x + p;
      p = p * x + c[k];
    }
  };
  for (int it = 0; it < 500; ++it) {
    double worst = 0.0;
    for (int k = 0; k < deg; ++k) {
      cd p, dp;
      eval(r[k], p, dp);
      if (p == cd(0.0, 0.0)) continue;
      const cd ratio = p / dp;
      cd sum(0.0, 0.0);
      for (int j = 0; j < deg; ++j)
        if (j != k) sum += 1.0 / (r[k] - r[j]);
      const cd step = ratio / (1.0 - ratio * sum);
      r[k] -= step;
      worst = std::max(worst, std::abs(step) / std::max(std::abs(r[k]), 1e-300));
    }
    if (worst < 1e-15) break;
  }
  for (cd& x : r)
    for (int k = 0; k < 2; ++k) {
      cd p, dp;
      eval(x, p, dp);
      if (dp != cd(0.0, 0.0)) x -= p / dp;
    }
  return r;
}

namespace {

// Leja order: largest modulus first, then each next root maximises the product of
// its distances to the roots already taken (keeps partial products balanced).
std::vector<cd> leja_order(std::vector<cd> r) {
  std::vector<cd> out;
  if (r.empty()) return out;
  size_t k0 = 0;
  for (size_t k = 1; k < r.size(); ++k)
    if (std::abs(r[k]) > std::abs(r[k0])) k0 = k;
  out.push_back(r[k0]);
  r.erase(r.begin() + k0);
  while (!r.empty()) {
    size_t best = 0;
    double bv = -1.0;
    for (size_t k = 0; k < r.size(); ++k) {
      double lp = 0.0;
      for (const cd& o : out) lp += std::log(std::abs(r[k] - o) + 1e-300);
      if (lp > bv) {
        bv = lp;
        best = k;
      }
    }
    out.push_back(r[best]);
    r.erase(r.begin() + best);
  }
  return out;
}

}  // namespace

// Product form of one step of eq. fix-pt-exp.  With B = -i delta (A - z0 I),
// beta = -i delta (z - z0) and g = i delta f, unrolling the k-recursion gives
//   y_new = [ p~(B) y + P2(B) g ] / p~(z),   P2(x) = sum_{m<q} e_m x^m,
//   e_m = sum_{j=m+1..q} beta^(j-1-m) / j!,
// i.e. an affine map y_new = L y + y1 with L = p~(B)/p~(z) (the error propagator of
// Thm 4.2) and y1 = P2(B) g / p~(z) (the first step from y = 0).  Both polynomials are
// applied as products of linear factors over their roots, L = s^q prod_k (B - rho_k)
// with p~(x) = (1/q!) prod (x - rho_k) and s = (q! p~(z))^(-1/q), so every factor is
//   w <- a (A - z0) w + b w,   a = -i delta s,  b = -s rho_k,
// and one full step is q such factors plus the added y1.  y1 uses the q-1 roots mu_k
// of P2 (leading coefficient e_{q-1} = 1/q!) in the same way; for q = 1, y1 = g / p~(z)
// is a single factor with a = 0.
// out_L: q factors, out_P: max(q-1, 1) factors, both in application order.
void factor_coefficients(cd z, cd z0, double delta, int q, FactorCoef* out_L, FactorCoef* out_P, cd& pz) {
  const cd beta = cd(0.0, -delta) * (z - z0);
  const cd mid(0.0, -delta);  // B = mid * (A - z0)
  pz = ptilde(z, z0, delta, q);
  std::vector<double> fact(q + 1, 1.0);
  for (int j = 1; j <= q; ++j) fact[j] = fact[j - 1] * j;
  // p~(x) = sum_m x^m / m!
  std::vector<cd> cp(q + 1);
  for (int m = 0; m <= q; ++m) cp[m] = 1.0 / fact[m];
  const std::vector<cd> rho = leja_order(poly_roots(cp));
  const cd sL = std::pow(1.0 / (fact[q] * pz), 1.0 / q);
  for (int k = 0; k < q; ++k) {
    const cd a = sL * mid, b = -sL * rho[k];
    out_L[k] = FactorCoef{a.real(), a.imag(), b.real(), b.imag()};
  }
  const cd g_scale = cd(0.0, delta) / pz;  // y1 = P2(B) (i delta f) / p~(z)
  if (q == 1) {
    // P2 = e_0 = 1
    out_P[0] = FactorCoef{0.0, 0.0, g_scale.real(), g_scale.imag()};
    return;
  }
  std::vector<cd> ce(q);
  for (int m = 0; m < q; ++m) {
    cd e(0.0, 0.0), bp(1.0, 0.0);
    for (int j = m + 1; j <= q; ++j) {
      e += bp / fact[j];
      bp *= beta;
    }
    ce[m] = e;
  }
  const std::vector<cd> mu = leja_order(poly_roots(ce));
  const cd s2 = std::pow(g_scale * ce[q - 1], 1.0 / (q - 1));
  for (int k = 0; k < q - 1; ++k) {
    const cd a = s2 * mid, b = -s2 * mu[k];
    out_P[k] = FactorCoef{a.real(), a.imag(), b.real(), b.imag()};
  }
}

}  // namespace hfci
