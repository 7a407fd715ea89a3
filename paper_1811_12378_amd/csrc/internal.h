// Host-side structures of libhfci (context, operator, contour) and error plumbing.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdio>
#include <functional>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hfci.h"
#include "kernels.h"
#include "netkern.h"

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

  // While an arena is set, get() allocates nothing: it hands out 256-byte aligned slices
  // of [base, base + cap), one per tag (the same tag gets the same slice while the arena
  // is set), and throws HFCI_E_ARG when a request does not fit.  ArenaScope sets one for
  // the duration of a call.
  void set_arena(void* base, size_t cap);
  void clear_arena();
  size_t arena_used() const { return arena_used_; }

 private:
  struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
  };
  std::map<std::string, Buf> bufs_;
  char* arena_ = nullptr;
  size_t arena_cap_ = 0, arena_used_ = 0;
  std::map<std::string, Buf> slices_;
};

class ArenaScope {
 public:
  ArenaScope(Workspace& ws, void* base, size_t cap) : ws_(ws) { ws_.set_arena(base, cap); }
  ~ArenaScope() { ws_.clear_arena(); }
  ArenaScope(const ArenaScope&) = delete;
  ArenaScope& operator=(const ArenaScope&) = delete;

 private:
  Workspace& ws_;
};

// Layout of Ctx::pinned_dbl: [0, kPinnedFciOffset) FGMRES scalars, then FCI weights.
constexpr size_t kPinnedFciOffset = 60000;
// Ctx::pinned_int holds 2 * kPinnedIntHalf ints (the two flag buffers of pipelined steps).
constexpr int kPinnedIntHalf = 32768;

// Opt-in kernel timing on the context's stream: HIP events around selected launches,
// with the algorithmic bytes each launch moves.  Harvested at the solver loop's sync points.
class Profiler {
 public:
  bool on = false;
  int period = 1;  // time every period-th launch of each class
  // whether this launch of class cls is timed (counts the launch either way)
  bool sample(int cls) { return on && (seen_[cls]++ % period) == 0; }
  struct Acc {
    long long launches = 0;
    double ms = 0.0, bytes = 0.0;
  };
  Acc acc[HFCI_PROF_N];
  void begin(hipStream_t s);
  void end(hipStream_t s, int cls, double bytes);
  void harvest();  // call after the stream has been synchronised
  // index of the next pending launch, and a correction of a pending launch's bytes (for
  // launches whose work is known only after they were queued)
  size_t mark() const { return pending_.size(); }
  void set_bytes(size_t i, double bytes) {
    if (i < pending_.size()) pending_[i].bytes = bytes;
  }
  void reset();
  void release();

 private:
  struct Pending {
    int cls;
    hipEvent_t a, b;
    double bytes;
  };
  hipEvent_t take();
  long long seen_[HFCI_PROF_N] = {};
  std::vector<hipEvent_t> free_;
  std::vector<Pending> pending_;
  hipEvent_t open_ = nullptr;
};

// Instantiated HIP graphs of fixed-point steps, keyed by every value their launches
// captured (pointers, sizes, coefficients' indices, shapes).  A few entries; cleared when full.
class GraphCache {
 public:
  hipGraphExec_t find(const std::string& key) const;
  void put(const std::string& key, hipGraphExec_t exec);
  void clear();
  ~GraphCache() { clear(); }

 private:
  std::map<std::string, hipGraphExec_t> map_;
};

struct Ctx {
  int device = 0;
  Profiler prof;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Workspace ws;
  GraphCache graphs;
  hipEvent_t step_event[2] = {nullptr, nullptr};  // read-backs of the pipelined fixed-point steps
  int* pinned_int = nullptr;     // host-pinned staging for small D2H reads (65536 ints)
  int* pinned_int_dev = nullptr; // the same memory as the device addresses it
  double* pinned_dbl = nullptr;  // host-pinned staging (65536 doubles)
  void* blas = nullptr;          // rocBLAS handle of the inner preconditioner (created on first use)
  std::map<int, double2*> sine;  // orthonormal DST-I matrices by size (device, complex)
  std::map<std::string, void*> fft;  // FFT plans of spectral operators by grid, precision, batch
  void* noalloc_scratch = nullptr;   // this device's static scratch array (noalloc.cpp)
};

// The device address of the static scratch array of the no-allocation entry point, looked
// up once per device with that device current (noalloc.cpp); its size in bytes.
void* noalloc_scratch_for_device(int device);
extern const size_t kNoAllocScratchBytes;

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
  // 1: the operator A itself; 2: B = iC - I of eq. mat-2x2 built on A (n = 2 x the grid
  // points, [b1, b2] x [-rho2, 0] the box of Thm 3.2's remark); 3: A with the
  // Fourier-spectral Laplacian of Sec. 7.1 on a periodic grid
  int form = 1;
};

struct Contour {
  const Op* op = nullptr;
  int device = 0;
  int J = 0, q = 0;
  double t = 0, eps = 0;
  std::vector<cd> z, sigma, z0, pz;  // poles, weights, Taylor centres, p~(z)
  std::vector<double> delta, nu;
  // per pole: q factors of L = p~(B)/p~(z), then max(q-1, 1) factors building y1
  int cstride = 0;                   // = q + max(q-1, 1)
  std::vector<FactorCoef> coef;      // [J][cstride]
  std::vector<PoleDev> pdev;         // [J]
  FactorCoef* d_coef = nullptr;      // device copies
  PoleDev* d_poles = nullptr;
};

// ---- net.cpp: the learned preconditioner ----
struct TrainData {
  int nx, ny, nz, npairs;
  const float2* v;            // [npairs][n] residuals (complex64, device)
  const float2* e;            // [npairs][n] corrections (complex64, device)
  const float* kch;           // [nmedia][n] omega^2 h^2 / c^2 (device)
  const int* medium_of_pair;  // [npairs] (host)
};
struct TrainOpts {
  int crop, steps, phase_aug, log_every, verbose, loss_kind;
  float lr, lr_min;
  unsigned long long seed;
};

struct Net {
  struct Layer {
    int cin = 0, cout = 0;
    long w_off = 0, b_off = 0;
  };
  struct Acts {
    Dims d1, d2, d3;
    long V1, V2, V3;
    uint16_t *a1, *cat1, *p1, *a2, *cat2, *p2, *a3, *b3, *g2, *dd2, *g1, *dd1;
    float* o;
    uint16_t *gd1 = nullptr, *gz = nullptr, *gg1 = nullptr, *gcat1 = nullptr, *gd2 = nullptr, *gg2 = nullptr,
             *gcat2 = nullptr, *gb3 = nullptr, *ga3 = nullptr, *gp2 = nullptr, *ge2 = nullptr, *ga2 = nullptr,
             *gp1 = nullptr, *ge1 = nullptr, *ga1 = nullptr;
    float* dout = nullptr;
    float* part = nullptr;
  };
  Ctx* ctx;
  int device;
  Layer layers[10];
  long head_off = 0, nparam = 0;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // FP32 master, grads, Adam moments
  uint16_t *wb = nullptr, *wt = nullptr;  // BF16 copies; wt = tap-flipped, Cin/Cout-transposed
  int step = 0;

  Net(Ctx* c, unsigned long long seed);
  ~Net();
  void set_params(const float* host);
  void get_params(float* host) const;
  void get_grads(float* host) const;
  void zero_moments();
  void refresh_bf16();
  Acts acts(Dims d, bool backward);
  void forward(Dims d, const uint16_t* x16, const Acts& a);
  void backward(const uint16_t* x16, const Acts& a);
  double train_step(Dims d, const uint16_t* x16, const float* target, float lr, bool update, bool read_loss,
                    int loss_kind);
  void eval(Dims d, const uint16_t* x16, float* out);
  void apply(const Op& op, int nvec, const double2* r, double2* z);
  double train(const TrainData& td, const TrainOpts& to, std::vector<double>& curve);

 private:
  void conv(const Acts& a, int l, Dims d, View in, View out, bool relu);
  void conv_back(const Acts& a, int l, Dims d, View in, View post, View dh, View din);
};

// ---- params.cpp ----
void op_rectangle(Op& op);
void contour_poles(int J, double t, double eps, double rho2, std::vector<cd>& z, std::vector<cd>& sigma);
cd ptilde(cd lam, cd z0, double delta, int q);
double rate_on_boundary(double delta, cd z, cd z0, int q, const std::vector<cd>& boundary);
std::vector<cd> rectangle_boundary(double b1, double b2, double rho2, int per_side);
// per_side: samples per side of the rectangle boundary; ns: points of the geometric delta scan
void optimise_delta(cd z, double b1, double b2, double rho2, int q, double& delta, double& nu, cd& z0,
                    int per_side = 2000, int ns = 480);
// the eps rule (hfci_contour_rule): candidates, the J it assumes by default (Sec. 7.3's six
// poles) and its rate resolution
constexpr int kRuleN = 31, kRuleJ = 6, kRulePerSide = 200, kRuleScan = 80;
// kRuleReduce: the stopping factor hfci_contour_create assumes (Table 4's, the default
// fp_reduce); kRuleLaunch, kRuleIter: the cost model's launch latency (in grid points of one
// system's pass) and per-iteration work (in products), fitted to solve times on MI355X
constexpr double kRuleLo = 0.01, kRuleHi = 0.64, kRuleReduce = 5.0, kRuleLaunch = 2.0e6, kRuleIter = 100.0;
// the share of the worst-case step count (in the logarithm of the reduction) the rule
// charges each pole: the adaptive stops measured 0.45-0.6 of it for eps >= 0.08
constexpr double kRuleStepFrac = 0.5;
// f(0), ..., f(n - 1) on host threads (independent calls; the first exception is rethrown)
void host_parallel_for(int n, const std::function<void(int)>& f);
// per_pass: factors per pass over HBM; q = 0: the degree is chosen too (written to *q_out)
double rule_eps(double b1, double b2, double rho2, double npoints, int J, double t, int q, int per_pass,
                double reduce, int* q_out);
// largest degree hfci_contour_create considers when it chooses q (q = 0)
constexpr int kAutoQMax = 16;
// per_pass: factors applied per pass over HBM (2 for the pair kernels, 1 otherwise)
int choose_q(cd z, double b1, double b2, double rho2, int qmax, int per_pass);
std::vector<cd> poly_roots(std::vector<cd> coeffs);
void factor_coefficients(cd z, cd z0, double delta, int q, FactorCoef* out_L, FactorCoef* out_P, cd& pz);

// ---- solver.cpp ----
template <typename T2>
KernelTune autotune_shapes(Op& op, int nsys, std::vector<std::pair<KernelTune, double>>& timings);
struct FciStats {
  long long matvecs = 0, fp_steps = 0;
};

// ---- batch.cpp: uneven batches of operators ----
template <typename T2>
void shifted_solve_multi(Ctx* ctx, const std::vector<const Op*>& ops, const std::vector<const Contour*>& cons,
                         const std::vector<const T2*>& f, const std::vector<T2*>& y, int fixed_steps, double reduce,
                         int max_steps, int* steps_out, FciStats& st);
hfci_status solve_batch(const std::vector<const Op*>& ops, const std::vector<const Contour*>& cons,
                        const hfci_solve_opts& o, const std::vector<const double2*>& f, const std::vector<double2*>& u,
                        hfci_stats* stats);

template <typename T2>
void shifted_solve_batch(const Op& op, const Contour& c, int nrhs, const T2* f, T2* y, int fixed_steps,
                         double reduce, int max_steps, int* steps_out, FciStats& st);
void fci_apply(const Op& op, const Contour& c, const hfci_solve_opts& o, int nrhs, const double2* f,
               double2* out, FciStats& st);
// inner.cpp: Alg. 1 step 4, k_in GMRES steps on the remainder f - A out (FP64, nrhs
// vectors), right-preconditioned by the regularised Laplacian inverse; out is updated
// net: the inner preconditioner is this network instead of the Laplacian inverse (NULL: the latter)
void inner_steps(const Op& op, int k_in, int nrhs, const double2* f, double2* out, FciStats& st, Net* net);
// y = V diag(1 / max(lambda, 1)) V^T x on the grid g (FP64, x and y distinct)
void laplace_inverse(Ctx& ctx, const GridDesc& g, const double2* x, double2* y);
void inner_release(Ctx& ctx);
// spectral.cpp: the Fourier-spectral operator (op.form == 3)
template <typename T2>
void spectral_S(const Op& op, int nvec, const T2* in, T2* out);
template <typename T2>
void spectral_apply(const Op& op, int nvec, const T2* x, T2* y, double sr, double si);
// spectral.hip: a gathered batch of the systems still iterating.  launch_spec_slots fills
// slot_sys[nvec] (the v-th active system, -1 past the last) and sys_slot[nsys] (-1 outside
// the batch) from the device flags; launch_spec_gather copies in_{slot_sys[v]} to out_v
// (zero for -1); launch_spec_factor_slots is launch_spec_factor with S w of system s at
// a.sw + sys_slot[s] n (slot null: at a.sw + s n).
void launch_spec_slots(hipStream_t st, const int* active, int nsys, int nvec, int* slot_sys, int* sys_slot);
template <typename T2>
void launch_spec_gather(hipStream_t st, const GridDesc& g, const T2* in, T2* out, const int* slot_sys, int nvec);
template <typename T2>
bool launch_spec_factor_slots(hipStream_t st, const GridDesc& g, const void* K, int kind, int nsys,
                              const SpecArgs<T2>& a, const int* slot);
template <typename T2>
void shifted_solve_spectral(const Op& op, const Contour& c, int nrhs, const T2* f, T2* y, int fixed_steps,
                            double reduce, int max_steps, int* steps_out, FciStats& st);
void spectral_release(Ctx& ctx);
// case_two.hip: factors k and k + 1 of a case-two fixed-point step in one pass (a.k is k;
// kind: kFacResid or kFacInF on the input, kFacAdd or kFacDual on the output); false for
// other kind bits
template <typename T2>
bool launch_b2_pair(hipStream_t st, const GridDesc& g, const void* K, int kind, int nsys, const B2Args<T2>& a);
// case_two.cpp: the shifted solves of a case-two operator (op.form == 2)
template <typename T2>
void shifted_solve_case_two(const Op& op, const Contour& c, int nrhs, const T2* f, T2* y, int fixed_steps,
                            double reduce, int max_steps, int* steps_out, FciStats& st);
hfci_status fgmres_solve(const Op& op, const Contour* c, const hfci_solve_opts& o, int nrhs,
                         const double2* f, double2* u, hfci_stats* stats);
void launch_diffnorm2_partial(hipStream_t st, const double2* a, const double2* b, size_t n, double* partial);

void set_last_error(const char* msg);

}  // namespace hfci

// The opaque C handles are the internal structures.
struct hfci_ctx : public hfci::Ctx {};
struct hfci_op : public hfci::Op {};
struct hfci_contour : public hfci::Contour {};
struct hfci_net : public hfci::Net {
  using hfci::Net::Net;
};
