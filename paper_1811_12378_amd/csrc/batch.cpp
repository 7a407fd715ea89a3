// Uneven batches: many independent operators (different grids, media and frequencies,
// each with its own contour) solved together.  Every factor of the product-form
// fixed-point step (eq. fix-pt-exp, see params.cpp) is one launch over the shifted
// systems of all instances still iterating: a work table maps each workgroup to its
// (instance, pole) system and tile.  The FCI quadrature, the step size d (Alg. 1 steps
// 2-3) and the FP64 flexible GMRES (Sec. 2) of each instance run per instance, in
// lockstep over the Arnoldi steps of all instances.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "internal.h"

namespace hfci {
namespace {

template <typename T2> const void* kappa_of(const Op& op);
template <> const void* kappa_of<float2>(const Op& op) { return op.kappa32; }
template <> const void* kappa_of<double2>(const Op& op) { return op.kappa64; }

template <typename T2> void copy_vec(hipStream_t s, T2* dst, const double2* src, size_t n);
template <> void copy_vec<float2>(hipStream_t s, float2* dst, const double2* src, size_t n) {
  launch_convert_64_to_32(s, dst, src, n);
}
template <> void copy_vec<double2>(hipStream_t s, double2* dst, const double2* src, size_t n) {
  HFCI_HIP(hipMemcpyAsync(dst, src, n * sizeof(double2), hipMemcpyDeviceToDevice, s));
}

std::string tag(const char* base, int i) { return std::string(base) + "_" + std::to_string(i); }

// Device tables and per-system vectors of a batch in precision T2.
template <typename T2>
struct MultiFp {
  Ctx* ctx = nullptr;
  int count = 0, q = 0, cstride = 0, nsys = 0;
  std::vector<const Op*> ops;
  std::vector<const Contour*> cons;
  std::vector<int> sys0, J, per_sys, per_sys_p;  // per instance (single-factor and pair tiles)
  bool pairs = false;                 // factors two per pass (every instance supports it)
  std::vector<size_t> n;
  std::vector<int> slot_of;           // per system
  std::vector<T2*> f, y;              // per instance: f (n), y (J n)
  std::vector<MultiSys<T2>> h_sys;
  std::vector<int2> h_seg, h_segp;
  std::vector<int> h_init;  // host sources of asynchronous copies live as long as the batch
  MultiInst* d_inst = nullptr;
  MultiSys<T2>* d_sys = nullptr;
  int2* d_seg = nullptr;
  int2* d_segp = nullptr;
  int2* d_bps = nullptr;              // per system: {single-factor, pair} blocks
  int *active = nullptr, *steps = nullptr;
  double *rnorm2 = nullptr, *fnorm2 = nullptr, *fpart = nullptr, *dpart = nullptr;
  std::vector<double*> cc;            // per instance: sigma_j / z_j (device)
  std::vector<T2*> w;                 // per instance: the quadrature sum (n)
  int nb_max = 0, nd_max = 0;

  MultiFp(Ctx* c, const std::vector<const Op*>& o, const std::vector<const Contour*>& k) : ctx(c), ops(o), cons(k) {
    hipStream_t s = ctx->stream;
    count = (int)ops.size();
    q = cons[0]->q;
    cstride = cons[0]->cstride;
    std::vector<MultiInst> h_inst(count);
    size_t npart = 0;
    pairs = q >= 3;
    for (int i = 0; i < count; ++i) {
      h_inst[i] = MultiLaunch<T2>::describe(ops[i]->g, kappa_of<T2>(*ops[i]));
      pairs = pairs && h_inst[i].pper_sys > 0;
    }
    for (int i = 0; i < count; ++i) {
      sys0.push_back(nsys);
      J.push_back(cons[i]->J);
      n.push_back(ops[i]->n);
      per_sys.push_back(h_inst[i].per_sys);
      per_sys_p.push_back(h_inst[i].pper_sys);
      nsys += cons[i]->J;
      // residual partials: one per block of the launch that forms them (a pair when fusing)
      npart += (size_t)cons[i]->J * (pairs ? h_inst[i].pper_sys : h_inst[i].per_sys);
      nb_max = std::max(nb_max, blas_blocks(ops[i]->n));
      nd_max = std::max(nd_max, Launch<T2>::partial_blocks(ops[i]->g));
    }
    Workspace& ws = ctx->ws;
    d_inst = (MultiInst*)ws.get("mb_inst", count * sizeof(MultiInst));
    d_sys = (MultiSys<T2>*)ws.get("mb_sys", nsys * sizeof(MultiSys<T2>));
    d_seg = (int2*)ws.get("mb_seg", (nsys + 1) * sizeof(int2));
    d_segp = (int2*)ws.get("mb_segp", (nsys + 1) * sizeof(int2));
    d_bps = (int2*)ws.get("mb_bps", nsys * sizeof(int2));
    active = (int*)ws.get("mb_active", nsys * sizeof(int));
    steps = (int*)ws.get("mb_steps", nsys * sizeof(int));
    rnorm2 = (double*)ws.get("mb_rnorm2", nsys * sizeof(double));
    fnorm2 = (double*)ws.get("mb_fnorm2", count * sizeof(double));
    fpart = (double*)ws.get("mb_fpart", (size_t)nb_max * sizeof(double));
    dpart = (double*)ws.get("mb_dpart", (size_t)3 * nd_max * sizeof(double));
    double* part = (double*)ws.get("mb_partial", npart * sizeof(double));
    h_sys.resize(nsys);
    slot_of.resize(nsys);
    size_t poff = 0;
    for (int i = 0; i < count; ++i) {
      const size_t vb = n[i] * sizeof(T2);
      T2* fi = (T2*)ws.get(tag("mb_f", i), vb);
      T2* yi = (T2*)ws.get(tag("mb_y", i), J[i] * vb);
      T2* y1i = (T2*)ws.get(tag("mb_y1", i), J[i] * vb);
      T2* wAi = (T2*)ws.get(tag("mb_wA", i), J[i] * vb);
      T2* wBi = (q >= 3) ? (T2*)ws.get(tag("mb_wB", i), J[i] * vb) : nullptr;
      f.push_back(fi);
      y.push_back(yi);
      w.push_back((T2*)ws.get(tag("mb_w", i), vb));
      double* cci = (double*)ws.get(tag("mb_cc", i), 2 * J[i] * sizeof(double));
      std::vector<double> h(2 * J[i]);
      for (int j = 0; j < J[i]; ++j) {
        const cd t = cons[i]->sigma[j] / cons[i]->z[j];
        h[2 * j] = t.real();
        h[2 * j + 1] = t.imag();
      }
      HFCI_HIP(hipMemcpy(cci, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
      cc.push_back(cci);
      for (int p = 0; p < J[i]; ++p) {
        const int G = sys0[i] + p;
        MultiSys<T2>& d = h_sys[G];
        d.vec[kRoleF] = fi;
        d.vec[kRoleY] = yi + (size_t)p * n[i];
        d.vec[kRoleY1] = y1i + (size_t)p * n[i];
        d.vec[kRoleWA] = wAi + (size_t)p * n[i];
        d.vec[kRoleWB] = wBi ? wBi + (size_t)p * n[i] : nullptr;
        d.coef = cons[i]->d_coef + (size_t)p * cstride;
        d.pole = cons[i]->d_poles + p;
        d.partial = part + poff;
        d.inst = i;
        d.nblk = pairs ? per_sys_p[i] : per_sys[i];
        d.slot = i;
        d.pad = 0;
        poff += d.nblk;
        slot_of[G] = i;
      }
    }
    HFCI_HIP(hipMemcpyAsync(d_inst, h_inst.data(), count * sizeof(MultiInst), hipMemcpyHostToDevice, s));
    HFCI_HIP(hipMemcpyAsync(d_sys, h_sys.data(), nsys * sizeof(MultiSys<T2>), hipMemcpyHostToDevice, s));
    std::vector<int2> h_bps(nsys);
    for (int G = 0; G < nsys; ++G)
      h_bps[G] = int2{per_sys[slot_of[G]], pairs ? per_sys_p[slot_of[G]] : 0};
    HFCI_HIP(hipMemcpyAsync(d_bps, h_bps.data(), nsys * sizeof(int2), hipMemcpyHostToDevice, s));
    HFCI_HIP(hipStreamSynchronize(s));
  }

  // Launch bounds of the systems with hact[G] != 0: rows to search (the live rows and
  // the sentinel) and blocks of single-factor and pair launches.
  struct Tables {
    int nseg, blocks, blocks_p;
  };
  Tables bounds(const std::vector<int>& hact) const {
    Tables t{1, 0, 0};
    for (int G = 0; G < nsys; ++G)
      if (hact[G]) {
        ++t.nseg;
        t.blocks += per_sys[slot_of[G]];
        if (pairs) t.blocks_p += per_sys_p[slot_of[G]];
      }
    return t;
  }
  // the work tables of those systems, each ending in its sentinel {total blocks, -1}
  Tables upload_segments(const std::vector<int>& hact) {
    h_seg.clear();
    h_segp.clear();
    int blocks = 0, blocks_p = 0;
    for (int G = 0; G < nsys; ++G)
      if (hact[G]) {
        h_seg.push_back(int2{blocks, G});
        h_segp.push_back(int2{blocks_p, G});
        blocks += per_sys[slot_of[G]];
        if (pairs) blocks_p += per_sys_p[slot_of[G]];
      }
    h_seg.push_back(int2{blocks, -1});
    h_segp.push_back(int2{blocks_p, -1});
    HFCI_HIP(hipMemcpyAsync(d_seg, h_seg.data(), h_seg.size() * sizeof(int2), hipMemcpyHostToDevice, ctx->stream));
    HFCI_HIP(hipMemcpyAsync(d_segp, h_segp.data(), h_segp.size() * sizeof(int2), hipMemcpyHostToDevice,
                            ctx->stream));
    return Tables{(int)h_seg.size(), blocks, blocks_p};
  }

  // The fixed-point iteration of every system of the live instances (live[i] != 0) on
  // f[i], from y = 0, as in fp_run: step one builds y1 = P2(B) g / p~(z), later steps
  // y <- L y + y1 with the residual of the current y tested in the first factor.
  void run(const std::vector<char>& live, int fixed_steps, double reduce, int max_steps, FciStats& st) {
    hipStream_t s = ctx->stream;
    const bool fixed = fixed_steps > 0;
    const int cap = fixed ? fixed_steps : max_steps;
    std::vector<int> hact(nsys, 0);
    int nact = 0;
    for (int G = 0; G < nsys; ++G)
      if (live[slot_of[G]]) {
        hact[G] = 1;
        ++nact;
      }
    if (nact == 0) return;
    for (int i = 0; i < count; ++i) {
      if (!live[i]) continue;
      launch_norm2_partial(s, f[i], sizeof(T2) == 8, n[i], fpart);
      launch_reduce(s, fpart, blas_blocks(n[i]), 1, fnorm2 + i);
    }
    // state after step one: every live system active, one step taken
    HFCI_HIP(hipStreamSynchronize(s));  // earlier copies from h_init / h_seg have completed
    h_init = hact;
    HFCI_HIP(hipMemcpyAsync(active, h_init.data(), nsys * sizeof(int), hipMemcpyHostToDevice, s));
    HFCI_HIP(hipMemcpyAsync(steps, h_init.data(), nsys * sizeof(int), hipMemcpyHostToDevice, s));
    auto sg = upload_segments(hact);
    const bool f64 = sizeof(T2) == 16;
    // one launch of `width` factors from coefficient k over the listed systems
    auto launch = [&](int kind, int k, int width, int rin, int rout, int rout2) {
      if (width == 2) {
        const bool ok = MultiLaunch<T2>::factor_pair(s, d_inst, d_sys, d_segp, sg.nseg, sg.blocks_p, kind, rin, rout,
                                                     rout2, k, cstride);
        HFCI_REQUIRE(ok, "internal: unsupported factor kind");
      } else {
        MultiLaunch<T2>::factor(s, d_inst, d_sys, d_seg, sg.nseg, sg.blocks, kind, rin, rout, rout2, k, cstride, f64);
      }
    };
    struct Part {
      int k, width, kind;
    };
    // launches of cnt factors from coefficient k0, two per pass when fusing; an odd count
    // leaves one single launch, at the end or (single_first) at the start
    auto plan = [&](int k0, int cnt, int kind_first, int kind_last, bool single_first) {
      std::vector<Part> v;
      for (int j = 0; j < cnt;) {
        const bool lone = single_first && j == 0 && cnt % 2 == 1;
        const int w = (pairs && j + 1 < cnt && !lone) ? 2 : 1;
        int kind = 0;
        if (j == 0) kind |= kind_first;
        if (j + w == cnt) kind |= kind_last;
        v.push_back(Part{k0 + j, w, kind});
        j += w;
      }
      return v;
    };
    // step one: the max(q-1, 1) factors of P2 from f into y1 (and y)
    const int nP = std::max(q - 1, 1);
    {
      const std::vector<Part> pl = plan(q, nP, kFacInF, kFacDual, true);
      int cur = kRoleF;
      for (size_t i = 0; i < pl.size(); ++i) {
        const bool last = i + 1 == pl.size();
        const int dst = last ? kRoleY1 : (cur == kRoleWA ? kRoleWB : kRoleWA);
        launch(pl[i].kind, pl[i].k, pl[i].width, cur, dst, last ? kRoleY : kRoleNone);
        cur = dst;
      }
      st.matvecs += (long long)(q - 1) * nact;
      st.fp_steps += nact;
    }
    // later steps: the first launch reads y and forms the residual partials, the last adds
    // y1 into y; the launches in between ping-pong between wA and wB
    const std::vector<Part> pl = plan(0, q, kFacResid, kFacAdd, false);
    auto rest = [&]() {
      int cur = kRoleWA;
      for (size_t i = 1; i < pl.size(); ++i) {
        const bool last = i + 1 == pl.size();
        const int dst = last ? kRoleY : (cur == kRoleWA ? kRoleWB : kRoleWA);
        launch(pl[i].kind, pl[i].k, pl[i].width, cur, dst, kRoleNone);
        cur = dst;
      }
    };
    if (!fixed && pl.size() > 1 && nsys <= kPinnedIntHalf) {
      // Adaptive, pipelined as the single-operator loop: the stopping test rebuilds the
      // work tables on the device, so the rest of step `it` and the head of step it + 1
      // are queued before the host reads step it's flags.  Their launches are sized for
      // the systems active after the previous test (a superset; surplus blocks meet the
      // sentinel and exit).  Flags alternate between the halves of the pinned buffer.
      hipEvent_t ev[2] = {ctx->step_event[0], ctx->step_event[1]};
      int* flags[2] = {ctx->pinned_int, ctx->pinned_int + kPinnedIntHalf};
      int* flags_dev[2] = {ctx->pinned_int_dev, ctx->pinned_int_dev + kPinnedIntHalf};
      auto head_to = [&](int slot) {
        launch(pl[0].kind, pl[0].k, pl[0].width, kRoleY, kRoleWA, kRoleNone);
        launch_fp_test_multi<T2>(s, d_sys, nsys, d_bps, fnorm2, reduce, max_steps, active, steps, rnorm2, d_seg,
                                 d_segp, flags_dev[slot]);
        HFCI_HIP(hipEventRecord(ev[slot], s));
      };
      head_to(0);
      st.matvecs += nact;
      int slot = 0;
      for (int it = 1; it <= cap; ++it) {
        rest();
        head_to(slot ^ 1);
        HFCI_HIP(hipEventSynchronize(ev[slot]));
        nact = 0;
        for (int G = 0; G < nsys; ++G) {
          hact[G] = flags[slot][G] != 0;
          nact += hact[G];
        }
        st.matvecs += (long long)q * nact;  // the rest of step it and the head of step it + 1
        st.fp_steps += nact;
        if (nact == 0) break;  // the queued launches found only the sentinel
        sg = bounds(hact);
        slot ^= 1;
      }
      return;
    }
    for (int it = 1; it <= cap; ++it) {
      if (fixed && it == cap) break;
      launch(pl[0].kind, pl[0].k, pl[0].width, kRoleY, kRoleWA, kRoleNone);
      st.matvecs += nact;
      launch_fp_check_multi<T2>(s, d_sys, nsys, fnorm2, fixed_steps, reduce, max_steps, active, steps, rnorm2);
      if (!fixed) {
        HFCI_HIP(hipMemcpyAsync(ctx->pinned_int, active, nsys * sizeof(int), hipMemcpyDeviceToHost, s));
        HFCI_HIP(hipStreamSynchronize(s));
        nact = 0;
        for (int G = 0; G < nsys; ++G) {
          hact[G] = ctx->pinned_int[G] != 0;
          nact += hact[G];
        }
        if (nact == 0) break;
        sg = upload_segments(hact);
      }
      st.matvecs += (long long)(q - 1) * nact;
      st.fp_steps += nact;
      if (pl.size() == 1) {  // a step of one launch went to wA
        for (int G = 0; G < nsys; ++G)
          if (hact[G])
            HFCI_HIP(hipMemcpyAsync(h_sys[G].vec[kRoleY], h_sys[G].vec[kRoleWA], n[slot_of[G]] * sizeof(T2),
                                    hipMemcpyDeviceToDevice, s));
        continue;
      }
      rest();
    }
  }

  void read_steps(int* out) {
    HFCI_HIP(hipMemcpyAsync(ctx->pinned_int, steps, nsys * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HFCI_HIP(hipStreamSynchronize(ctx->stream));
    std::memcpy(out, ctx->pinned_int, nsys * sizeof(int));
  }
};

// Alg. 1 steps 1-3 for every live instance: v[i] (FP64, n_i) -> z[i] = d_i w_i.
template <typename T2>
void fci_multi(MultiFp<T2>& M, const std::vector<char>& live, const std::vector<const double2*>& v,
               const std::vector<double2*>& z, const hfci_solve_opts& o, FciStats& st) {
  Ctx& ctx = *M.ctx;
  hipStream_t s = ctx.stream;
  for (int i = 0; i < M.count; ++i)
    if (live[i]) copy_vec<T2>(s, M.f[i], v[i], M.n[i]);
  M.run(live, o.fp_steps, o.fp_reduce, o.fp_max_steps, st);
  for (int i = 0; i < M.count; ++i) {
    if (!live[i]) continue;
    const Op& op = *M.ops[i];
    const Contour& c = *M.cons[i];
    const size_t n = M.n[i];
    T2* w = M.w[i];
    launch_combine<T2>(s, w, M.y[i], M.cc[i], c.J, 1, n, false);
    const int nblk = Launch<T2>::partial_blocks(op.g);
    double* part = M.dpart;
    double* sums = (double*)ctx.ws.get(tag("mb_dsums", i), 3 * sizeof(double));
    double* d = (double*)ctx.ws.get(tag("mb_d", i), 2 * sizeof(double));
    Launch<T2>::dstep_partials(s, op.g, kappa_of<T2>(op), 1, w, M.f[i], part);
    launch_reduce(s, part, nblk, 3, sums);
    launch_dfinish(s, sums, 1, d);
    st.matvecs += 1;
    launch_scale_out<T2>(s, z[i], w, d, 1, n);
  }
}

struct Timer {
  hipEvent_t a, b;
  hipStream_t s;
  explicit Timer(hipStream_t st) : s(st) {
    HFCI_HIP(hipEventCreateWithFlags(&a, hipEventDisableSystemFence));
    HFCI_HIP(hipEventCreateWithFlags(&b, hipEventDisableSystemFence));
  }
  ~Timer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  void start() { HFCI_HIP(hipEventRecord(a, s)); }
  void stop() { HFCI_HIP(hipEventRecord(b, s)); }
  // after stop(): waits for the end event (free after a stream synchronisation)
  double elapsed_ms() {
    HFCI_HIP(hipEventSynchronize(b));
    float ms = 0;
    HFCI_HIP(hipEventElapsedTime(&ms, a, b));
    return ms;
  }
  double stop_ms() {
    stop();
    return elapsed_ms();
  }
};

// [c s; -conj(s) c] [a; b] = [rho; 0], c real
void givens(cd a, cd b, double& c, cd& s, cd& rho) {
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

template <typename T2>
void solve_multi(MultiFp<T2>* M, const std::vector<const Op*>& ops, const hfci_solve_opts& o,
                 const std::vector<const double2*>& f, const std::vector<double2*>& u, hfci_stats* stats,
                 hfci_status* status_out) {
  Ctx& ctx = *ops[0]->ctx;
  hipStream_t s = ctx.stream;
  const int count = (int)ops.size();
  const int m = o.restart;
  const int hstride = 4 * (m + 1) + 2 + 2 * m;
  std::vector<double2*> b(count), V(count), Z(count);
  std::vector<double*> hdev(count);
  int nbs_max = 0, nbb_max = 0;
  for (int i = 0; i < count; ++i) {
    const size_t n = ops[i]->n;
    b[i] = (double2*)ctx.ws.get(tag("mg_b", i), n * sizeof(double2));
    V[i] = (double2*)ctx.ws.get(tag("mg_V", i), (size_t)(m + 1) * n * sizeof(double2));
    Z[i] = (double2*)ctx.ws.get(tag("mg_Z", i), (size_t)m * n * sizeof(double2));
    hdev[i] = (double*)ctx.ws.get(tag("mg_h", i), hstride * sizeof(double));
    nbs_max = std::max(nbs_max, Launch<double2>::partial_blocks(ops[i]->g));
    nbb_max = std::max(nbb_max, blas_blocks(n));
  }
  double* part = (double*)ctx.ws.get("mg_part", (size_t)std::max(nbs_max, nbb_max * 2 * (m + 1)) * sizeof(double));
  if ((size_t)count * hstride > kPinnedFciOffset) throw Error(HFCI_E_ARG, "batch too large for the restart length");
  double* hh_all = ctx.pinned_dbl;
  auto hhost = [&](int i) { return hh_all + (size_t)i * hstride; };

  std::vector<double> bnorm(count);
  for (int i = 0; i < count; ++i) {
    const size_t n = ops[i]->n;
    launch_copy_scaled64(s, b[i], f[i], n, ops[i]->s);
    launch_norm2_partial(s, b[i], false, n, part);
    launch_reduce(s, part, blas_blocks(n), 1, hdev[i]);
    HFCI_HIP(hipMemcpyAsync(hhost(i), hdev[i], sizeof(double), hipMemcpyDeviceToHost, s));
  }
  HFCI_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < count; ++i) bnorm[i] = std::sqrt(hhost(i)[0]);

  std::vector<char> done(count, 0);
  std::vector<double> relres(count, 1.0);
  std::vector<std::vector<cd>> H(count), G(count), SN(count);
  std::vector<std::vector<double>> CS(count);
  std::vector<int> kr(count, 0), its_i(count, 0), cyc_i(count, 0);
  std::vector<long long> mv_i(count, 0);
  int its = 0, cycles = 0;
  FciStats fst;
  double t_fci = 0, t_arn = 0;
  Timer tm(s), tf(s);  // tf: the preconditioner of an Arnoldi step, read at the step's sync
  const auto t0 = std::chrono::steady_clock::now();
  hfci_status status = HFCI_OK;
  for (int i = 0; i < count; ++i)
    if (bnorm[i] == 0.0) {
      launch_fill_zero(s, u[i], ops[i]->n * sizeof(double2));
      done[i] = 1;
      relres[i] = 0.0;
    }
  while (true) {
    tm.start();
    std::vector<int> act;
    for (int i = 0; i < count; ++i) {
      if (done[i]) continue;
      const Op& op = *ops[i];
      launch_residual64(s, op.g, op.kappa64, b[i], u[i], V[i], part);
      launch_reduce(s, part, Launch<double2>::partial_blocks(op.g), 1, hdev[i] + 4 * (m + 1) + 1);
      HFCI_HIP(hipMemcpyAsync(hhost(i) + 4 * (m + 1) + 1, hdev[i] + 4 * (m + 1) + 1, sizeof(double),
                              hipMemcpyDeviceToHost, s));
      act.push_back(i);
      ++mv_i[i];
    }
    HFCI_HIP(hipStreamSynchronize(s));
    t_arn += tm.stop_ms();
    std::vector<int> cyc;
    for (int i : act) {
      const double beta = std::sqrt(hhost(i)[4 * (m + 1) + 1]);
      if (!(beta == beta)) throw Error(HFCI_E_NUMERIC, "NaN in the FGMRES residual");
      relres[i] = beta / bnorm[i];
      if (relres[i] <= o.tol) done[i] = 1;
      else cyc.push_back(i);
    }
    if (o.verbose) {
      double mx = 0.0;
      for (int i : act) mx = std::max(mx, relres[i]);
      std::fprintf(stderr, "[hfci-batch] cycle %d: its %d, max true relres %.3e, %zu of %d instances open, "
                   "fci %.0f ms, arnoldi %.0f ms\n", cycles, its, mx, cyc.size(), count, t_fci, t_arn);
      std::fflush(stderr);
    }
    if (cyc.empty()) break;
    if (its >= o.max_it) {
      status = HFCI_W_NOCONV;
      break;
    }
    ++cycles;
    for (int i : cyc) {
      ++cyc_i[i];
      launch_scale_inv(s, V[i], V[i], ops[i]->n, hdev[i] + 4 * (m + 1) + 1);
      H[i].assign((size_t)(m + 1) * m, cd(0, 0));
      G[i].assign(m + 1, cd(0, 0));
      G[i][0] = std::sqrt(hhost(i)[4 * (m + 1) + 1]);
      CS[i].assign(m, 0.0);
      SN[i].assign(m, cd(0, 0));
      kr[i] = 0;
    }
    std::vector<int> live = cyc;
    for (int j = 0; j < m && !live.empty(); ++j) {
      tf.start();
      std::vector<char> lv(count, 0);
      std::vector<const double2*> vin(count, nullptr);
      std::vector<double2*> zout(count, nullptr);
      for (int i : live) {
        lv[i] = 1;
        vin[i] = V[i] + (size_t)j * ops[i]->n;
        zout[i] = Z[i] + (size_t)j * ops[i]->n;
      }
      if (M) {
        fci_multi<T2>(*M, lv, vin, zout, o, fst);
      } else {
        for (int i : live)
          HFCI_HIP(hipMemcpyAsync(zout[i], vin[i], ops[i]->n * sizeof(double2), hipMemcpyDeviceToDevice, s));
      }
      tf.stop();  // no wait here: the Arnoldi launches queue behind the preconditioner
      tm.start();
      for (int i : live) {
        const Op& op = *ops[i];
        const size_t n = op.n;
        double2* w = V[i] + (size_t)(j + 1) * n;
        double* hb = hdev[i];
        Launch<double2>::apply(s, op.g, op.kappa64, 0.0, 0.0, 1, Z[i] + (size_t)j * n, w);
        launch_cgs2(s, V[i], j + 1, n, n, w, part, hb, hb + 2 * (m + 1), hb + 4 * (m + 1));
        launch_scale_inv(s, w, w, n, hb + 4 * (m + 1));
        HFCI_HIP(hipMemcpyAsync(hhost(i), hb, (4 * (m + 1) + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
        ++mv_i[i];
        ++its_i[i];
      }
      HFCI_HIP(hipStreamSynchronize(s));
      t_arn += tm.stop_ms();
      t_fci += tf.elapsed_ms();
      ++its;
      std::vector<int> next;
      for (int i : live) {
        const double* hh = hhost(i);
        std::vector<cd>& Hr = H[i];
        auto Hat = [&](int a, int c) -> cd& { return Hr[(size_t)a * m + c]; };
        for (int a = 0; a <= j; ++a)
          Hat(a, j) = cd(hh[2 * a] + hh[2 * (m + 1) + 2 * a], hh[2 * a + 1] + hh[2 * (m + 1) + 2 * a + 1]);
        const double hn = std::sqrt(hh[4 * (m + 1)]);
        if (!(hn == hn)) throw Error(HFCI_E_NUMERIC, "NaN in the Arnoldi process");
        Hat(j + 1, j) = hn;
        for (int a = 0; a < j; ++a) {
          const cd x = Hat(a, j), yv = Hat(a + 1, j);
          Hat(a, j) = CS[i][a] * x + SN[i][a] * yv;
          Hat(a + 1, j) = -std::conj(SN[i][a]) * x + CS[i][a] * yv;
        }
        double cs;
        cd sn, rho;
        givens(Hat(j, j), Hat(j + 1, j), cs, sn, rho);
        CS[i][j] = cs;
        SN[i][j] = sn;
        Hat(j, j) = rho;
        Hat(j + 1, j) = 0.0;
        G[i][j + 1] = -std::conj(sn) * G[i][j];
        G[i][j] = cs * G[i][j];
        kr[i] = j + 1;
        relres[i] = std::abs(G[i][j + 1]) / bnorm[i];
        if (!(relres[i] <= o.tol) && its < o.max_it && hn > 0.0) next.push_back(i);
      }
      live = next;
      if (its >= o.max_it) break;
    }
    tm.start();
    for (int i : cyc) {
      const int k = kr[i];
      std::vector<cd> yv(k);
      for (int a = k - 1; a >= 0; --a) {
        cd acc = G[i][a];
        for (int l = a + 1; l < k; ++l) acc -= H[i][(size_t)a * m + l] * yv[l];
        yv[a] = acc / H[i][(size_t)a * m + a];
      }
      double* yd = hhost(i) + 4 * (m + 1) + 2;
      for (int a = 0; a < k; ++a) {
        yd[2 * a] = yv[a].real();
        yd[2 * a + 1] = yv[a].imag();
      }
      HFCI_HIP(hipMemcpyAsync(hdev[i] + 4 * (m + 1) + 2, yd, 2 * k * sizeof(double), hipMemcpyHostToDevice, s));
      launch_multiaxpy(s, u[i], Z[i], k, ops[i]->n, ops[i]->n, hdev[i] + 4 * (m + 1) + 2, 1.0);
    }
    HFCI_HIP(hipStreamSynchronize(s));
    t_arn += tm.stop_ms();
  }
  const double wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats)
    for (int i = 0; i < count; ++i) {
      hfci_stats& st = stats[i];
      st.its = its_i[i];
      st.restarts = cyc_i[i];
      st.matvecs = mv_i[i];  // FGMRES products; the shifted sweeps are counted for the batch in stats[0]
      st.fp_steps = 0;
      st.final_relres = relres[i];
      st.time_fci_ms = t_fci;
      st.time_arnoldi_ms = t_arn;
      st.time_total_ms = wall;
      st.harvested = 0;
      st.learned_accepted = 0;
      st.learned_fallbacks = 0;
      st.time_net_ms = 0.0;
      st.net_rho_mean = 0.0;
      st.fci_rho_mean = 0.0;
    }
  if (stats) {
    stats[0].matvecs += fst.matvecs;
    stats[0].fp_steps = fst.fp_steps;
  }
  *status_out = status;
}

}  // namespace

template <typename T2>
void shifted_solve_multi(Ctx* ctx, const std::vector<const Op*>& ops, const std::vector<const Contour*>& cons,
                         const std::vector<const T2*>& f, const std::vector<T2*>& y, int fixed_steps, double reduce,
                         int max_steps, int* steps_out, FciStats& st) {
  MultiFp<T2> M(ctx, ops, cons);
  hipStream_t s = ctx->stream;
  for (int i = 0; i < M.count; ++i)
    HFCI_HIP(hipMemcpyAsync(M.f[i], f[i], M.n[i] * sizeof(T2), hipMemcpyDeviceToDevice, s));
  std::vector<char> live(M.count, 1);
  M.run(live, fixed_steps, reduce, max_steps, st);
  for (int i = 0; i < M.count; ++i)
    HFCI_HIP(hipMemcpyAsync(y[i], M.y[i], (size_t)M.J[i] * M.n[i] * sizeof(T2), hipMemcpyDeviceToDevice, s));
  if (steps_out) M.read_steps(steps_out);
}
template void shifted_solve_multi<float2>(Ctx*, const std::vector<const Op*>&, const std::vector<const Contour*>&,
                                          const std::vector<const float2*>&, const std::vector<float2*>&, int, double,
                                          int, int*, FciStats&);
template void shifted_solve_multi<double2>(Ctx*, const std::vector<const Op*>&, const std::vector<const Contour*>&,
                                           const std::vector<const double2*>&, const std::vector<double2*>&, int,
                                           double, int, int*, FciStats&);

hfci_status solve_batch(const std::vector<const Op*>& ops, const std::vector<const Contour*>& cons,
                        const hfci_solve_opts& o, const std::vector<const double2*>& f, const std::vector<double2*>& u,
                        hfci_stats* stats) {
  Ctx* ctx = ops[0]->ctx;
  hfci_status st = HFCI_OK;
  if (o.precond == HFCI_PRECOND_NONE) {
    solve_multi<float2>(nullptr, ops, o, f, u, stats, &st);
  } else if (o.precision == HFCI_F32) {
    MultiFp<float2> M(ctx, ops, cons);
    solve_multi<float2>(&M, ops, o, f, u, stats, &st);
  } else {
    MultiFp<double2> M(ctx, ops, cons);
    solve_multi<double2>(&M, ops, o, f, u, stats, &st);
  }
  return st;
}

}  // namespace hfci
