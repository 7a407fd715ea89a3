// Host-side structures of libhfci (context, operator, contour) and error plumbing.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdio>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hfci.h"
#include "kernels.h"

namespace hfci {

using cd = std::complex<double>;

struct Error : public std::runtime_error {
  hfci_status st;
  Error(hfci_status s, const std::string& m) : std::runtime_error(m), st(s) {}
};

[[noreturn]] void throw_hip(hipError_t e, const char* what, const char* file, int line);

#define HFCI_HIP(x)                                               \
  do {                                                            \
    hipError_t e_ = (x);                                          \
    if (e_ != hipSuccess) throw_hip(e_, #x, __FILE__, __LINE__);  \
  } while (0)

#define HFCI_REQUIRE(cond, msg)                                   \
  do {                                                            \
    if (!(cond)) throw Error(HFCI_E_ARG, msg);                    \
  } while (0)

// Device workspace owned by a context: named buffers that only grow.
class Workspace {
 public:
  void* get(const std::string& tag, size_t bytes);
  void release_all();
  ~Workspace() { release_all(); }

 private:
  struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
  };
  std::map<std::string, Buf> bufs_;
};

// Layout of Ctx::pinned_dbl: [0, kPinnedFciOffset) FGMRES scalars, then FCI weights.
constexpr size_t kPinnedFciOffset = 60000;

// Opt-in kernel timing on the context's stream: HIP events around selected launches,
// with the algorithmic bytes each launch moves.  Harvested at the driver's sync points.
class Profiler {
 public:
  bool on = false;
  struct Acc {
    long long launches = 0;
    double ms = 0.0, bytes = 0.0;
  };
  Acc acc[HFCI_PROF_N];
  void begin(hipStream_t s);
  void end(hipStream_t s, int cls, double bytes);
  void harvest();  // call after the stream has been synchronised
  void reset();
  void release();

 private:
  struct Pending {
    int cls;
    hipEvent_t a, b;
    double bytes;
  };
  hipEvent_t take();
  std::vector<hipEvent_t> free_;
  std::vector<Pending> pending_;
  hipEvent_t open_ = nullptr;
};

struct Ctx {
  int device = 0;
  Profiler prof;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Workspace ws;
  int* pinned_int = nullptr;     // host-pinned staging for small D2H reads
  double* pinned_dbl = nullptr;  // host-pinned staging (65536 doubles)
};

struct Op {
  Ctx* ctx = nullptr;
  int device = 0;        // kept so that destroy never dereferences ctx
  GridDesc g{};
  size_t n = 0;
  double h = 0, omega = 0, s = 0, s_h2 = 0;
  double b1 = 0, b2 = 0, rho2 = 0, kmin = 0, kmax = 0;
  double damp_rho2 = 0;
  int damp_cells = 0;
  double* kappa64 = nullptr;
  float* kappa32 = nullptr;
};

struct Contour {
  const Op* op = nullptr;
  int device = 0;
  int J = 0, q = 0;
  double t = 0, eps = 0;
  std::vector<cd> z, sigma, z0, pz;  // poles, weights, Taylor centres, p~(z)
  std::vector<double> delta, nu;
  std::vector<StageCoef> coef;       // [J][q]
  std::vector<PoleDev> pdev;         // [J]
  StageCoef* d_coef = nullptr;       // device copies
  PoleDev* d_poles = nullptr;
};

// ---- params.cpp ----
void op_rectangle(Op& op);
void contour_poles(int J, double t, double eps, double rho2, std::vector<cd>& z, std::vector<cd>& sigma);
cd ptilde(cd lam, cd z0, double delta, int q);
double rate_on_boundary(double delta, cd z, cd z0, int q, const std::vector<cd>& boundary);
std::vector<cd> rectangle_boundary(double b1, double b2, double rho2, int per_side);
void optimise_delta(cd z, double b1, double b2, double rho2, int q, double& delta, double& nu, cd& z0);
void stage_coefficients(cd z, cd z0, double delta, int q, StageCoef* out, cd& pz);

// ---- solver.cpp ----
struct FciStats {
  long long matvecs = 0, fp_steps = 0;
};
template <typename T2>
void shifted_solve_batch(const Op& op, const Contour& c, int nrhs, const T2* f, T2* y, int fixed_steps,
                         double reduce, int max_steps, int* steps_out, FciStats& st);
void fci_apply(const Op& op, const Contour& c, const hfci_solve_opts& o, int nrhs, const double2* f,
               double2* out, FciStats& st);
hfci_status fgmres_solve(const Op& op, const Contour* c, const hfci_solve_opts& o, int nrhs,
                         const double2* f, double2* u, hfci_stats* stats);

}  // namespace hfci
