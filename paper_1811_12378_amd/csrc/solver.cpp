// Host drivers: batched polynomial fixed-point iteration (Sec. 4.2, eq. fix-pt-exp),
// the FCI preconditioner (Algorithm 1) and flexible GMRES(m) (Sec. 2) in FP64.
//
// All (pole, right-hand side) shifted systems of one FCI application advance together:
// every factor of a fixed-point step is a single launch over the systems still
// iterating, so a step at 256^3 with 16 poles x 8 RHS is one launch of ~260k
// workgroups.  Systems stop independently: the device turns residual norms into
// per-system active flags and a compacted list of the systems left, which the next
// launches read; the host reads the flags once per step to size the grid and to know
// when every system has stopped.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "internal.h"

namespace hfci {
namespace {

template <typename T2> struct Prec;
template <> struct Prec<float2> { static const void* kappa(const Op& op) { return op.kappa32; } };
template <> struct Prec<double2> { static const void* kappa(const Op& op) { return op.kappa64; } };

template <typename T2>
void copy_active(hipStream_t st, T2* dst, const T2* src, const int* active, int nsys, size_t n);

}  // namespace

void launch_copy_active_f(hipStream_t st, float2* dst, const float2* src, const int* active, int nsys, size_t n);
void launch_copy_active_d(hipStream_t st, double2* dst, const double2* src, const int* active, int nsys,
                          size_t n);
void launch_copy_unstepped(hipStream_t st, void* dst, const void* src, bool f64, const int* steps, int nsys,
                           size_t n);

namespace {
template <>
void copy_active<float2>(hipStream_t st, float2* d, const float2* s, const int* a, int nsys, size_t n) {
  launch_copy_active_f(st, d, s, a, nsys, n);
}
template <>
void copy_active<double2>(hipStream_t st, double2* d, const double2* s, const int* a, int nsys, size_t n) {
  launch_copy_active_d(st, d, s, a, nsys, n);
}
// d_s = s_s for the systems with steps[s] <= 1
template <typename T2>
void copy_unstepped(hipStream_t st, T2* d, const T2* s, const int* steps, int nsys, size_t n) {
  launch_copy_unstepped(st, d, s, sizeof(T2) == 16, steps, nsys, n);
}

// Systems whose iterate was left in y1 (they took at most one fixed-point step): the
// caller selects y1 for them through their step counts.
template <typename T2>
struct Deferred {
  const T2* y1 = nullptr;
  const int* steps = nullptr;
};

// Iterate eq. fix-pt-exp for systems gs in [sys0, sys0 + nsys) from y = 0, in the
// product form of params.cpp: step one builds y1 = P2(B) g / p~(z) (y = y1 after it),
// every later step is y <- L y + y1 as q factor launches, the first of which also forms
// the residual of the current y for the stopping test (Table 4's "reduced by 5").  With
// defer (not null), systems that took at most one step may keep their iterate in y1:
// defer->y1 and defer->steps are then set for the caller to select it (else both null).
template <typename T2>
void fp_run(const Op& op, const Contour& c, int nrhs, const T2* f, T2* y, int sys0, int nsys,
            int fixed_steps, double reduce, int max_steps, int* steps_out, FciStats& st, bool graphs = false,
            Deferred<T2>* defer = nullptr) {
  Ctx& ctx = *op.ctx;
  hipStream_t s = ctx.stream;
  const size_t n = op.n;
  const int q = c.q;
  const size_t vbytes = n * sizeof(T2);
  const bool fixed = fixed_steps > 0;
  const int cap = fixed ? fixed_steps : max_steps;
  int* steps = (int*)ctx.ws.get("fp_steps", (size_t)nsys * sizeof(int));
  if (cap <= 0) {
    launch_fill_zero(s, y, (size_t)nsys * vbytes);
    launch_set_int(s, steps, 0, nsys);
  } else {
    T2* y1 = (T2*)ctx.ws.get("fp_y1", (size_t)nsys * vbytes);
    T2* wA = (T2*)ctx.ws.get("fp_wA", (size_t)nsys * vbytes);
    T2* wB = (q >= 3) ? (T2*)ctx.ws.get("fp_wB", (size_t)nsys * vbytes) : nullptr;
    const KernelTune& tn = (sizeof(T2) == 8) ? op.g.tune32 : op.g.tune64;
    const bool fuse = tn.fuse != 0 && Launch<T2>::pair_fits(op.g);
    const bool triples = fuse && Launch<T2>::triple_runs(op.g);
    // residual partials come from the first launch of a step: a pair launch when fusing
    const int nblk = (fuse && q >= 3) ? Launch<T2>::pair_blocks(op.g) : Launch<T2>::partial_blocks(op.g);
    double* partial = (double*)ctx.ws.get("fp_partial", (size_t)nsys * nblk * sizeof(double));
    int* active = (int*)ctx.ws.get("fp_active", (size_t)nsys * sizeof(int));
    int* list = (int*)ctx.ws.get("fp_list", (size_t)nsys * sizeof(int));
    double* rnorm2 = (double*)ctx.ws.get("fp_rnorm2", (size_t)nsys * sizeof(double));
    const int nb = blas_blocks(n);
    double* fpart = (double*)ctx.ws.get("fp_fpart", (size_t)nrhs * nb * sizeof(double));
    double* fnorm2 = (double*)ctx.ws.get("fp_fnorm2", (size_t)nrhs * sizeof(double));
    for (int r = 0; r < nrhs; ++r)
      launch_norm2_partial(s, f + (size_t)r * n, sizeof(T2) == 8, n, fpart + (size_t)r * nb);
    launch_reduce(s, fpart, nb, nrhs, fnorm2);
    launch_fp_start(s, nsys, sys0, nrhs, fnorm2, fixed, active, steps, list);

    FactorArgs<T2> a{};
    a.f = f;
    a.y1 = y1;
    a.coef = c.d_coef;
    a.poles = c.d_poles;
    a.list = list;
    a.partial = partial;
    a.sys0 = sys0;
    a.nrhs = nrhs;
    a.cstride = c.cstride;
    const void* kap = Prec<T2>::kappa(op);
    Profiler& pr = ctx.prof;
    // algorithmic bytes of one launch: per listed system its own vectors (vec_per_sys of
    // them), plus kappa once and the right-hand sides of the listed systems once each
    const double e = (double)sizeof(T2), ek = e / 2.0;
    std::vector<int> hact(nsys, 1);
    auto launch_bytes = [&](double vec_per_sys, bool reads_f) {
      int na = 0;
      std::vector<char> rhs_used(nrhs, 0);
      for (int k = 0; k < nsys; ++k)
        if (hact[k]) {
          ++na;
          rhs_used[(sys0 + k) % nrhs] = 1;
        }
      int nr = 0;
      for (char u : rhs_used) nr += u;
      return (double)n * (vec_per_sys * e * na + ek + (reads_f ? e * nr : 0.0));
    };
    // launches queued before the systems they run over are known: their bytes are set
    // once the flags have been read back
    struct Fixup {
      size_t idx;
      double vecs;
      bool reads_f;
    };
    std::vector<Fixup>* fixups = nullptr;
    // One launch of `width` (1, 2 or 3) consecutive factors starting at coefficient k.  kind:
    // kFacInF / kFacResid on its first factor, kFacAdd / kFacDual on its last (none with 3).
    auto launch = [&](int kind, int k, int width, const T2* win, T2* wout, T2* wout2, bool fan = false) {
      a.k = k;
      a.win = win;
      a.wout = wout;
      a.wout2 = wout2;
      const bool inf = kind & kFacInF, resid = kind & kFacResid, add = kind & kFacAdd, dual = kind & kFacDual;
      const int cls = resid                  ? HFCI_PROF_FP_FIRST
                       : (inf || dual)       ? HFCI_PROF_FP_INIT
                       : add                 ? HFCI_PROF_FP_LAST
                       : width == 3          ? HFCI_PROF_FP_TRIPLE
                                             : HFCI_PROF_FP_STAGE;
      const double vecs = (inf ? 0.0 : 1.0) + 1.0 + (add ? 1.0 : 0.0) + (dual ? 1.0 : 0.0);
      const bool timed = pr.sample(cls);
      if (timed) pr.begin(s);
      const bool ok = width == 3   ? kind == 0 && Launch<T2>::factor_triple(s, op.g, kap, a)
                      : width == 2 ? Launch<T2>::factor_pair(s, op.g, kap, a, kind)
                                   : (fan && Launch<T2>::factor_fanout(s, op.g, kap, a)) ||
                                         Launch<T2>::factor(s, op.g, kap, a, kind);
      HFCI_REQUIRE(ok, "internal: unsupported factor kind");
      if (timed) {
        if (fixups) fixups->push_back(Fixup{pr.mark(), vecs, inf || resid});
        pr.end(s, cls, launch_bytes(vecs, inf || resid));
      }
    };
    struct Part {
      int k, width, kind;
    };
    // launches of `count` factors from coefficient k0, two per pass when fusing; an odd
    // count leaves one single launch, at the end or (single_first) at the start.  With
    // triples the run of middle pairs (kind 0), 2L factors, is split again into threes and
    // the fewest pairs that complete it (none, one or two: 4 = 2 + 2, never 3 + 1).
    auto plan = [&](int k0, int count, int kind_first, int kind_last, bool pairs, bool single_first) {
      std::vector<Part> v;
      for (int j = 0; j < count;) {
        const bool lone = single_first && j == 0 && count % 2 == 1;
        const int w = (pairs && j + 1 < count && !lone) ? 2 : 1;
        int kind = 0;
        if (j == 0) kind |= kind_first;
        if (j + w == count) kind |= kind_last;
        v.push_back(Part{k0 + j, w, kind});
        j += w;
      }
      if (!triples) return v;
      std::vector<Part> out;
      for (size_t i = 0; i < v.size();) {
        if (v[i].width != 2 || v[i].kind != 0) {
          out.push_back(v[i++]);
          continue;
        }
        size_t j = i;
        while (j < v.size() && v[j].width == 2 && v[j].kind == 0) ++j;
        const int m = 2 * (int)(j - i), np = (m % 3 == 0) ? 0 : (m % 3 == 2) ? 1 : 2;
        int k = v[i].k;
        for (int t = 0; t < (m - 2 * np) / 3; ++t, k += 3) out.push_back(Part{k, 3, 0});
        for (int t = 0; t < np; ++t, k += 2) out.push_back(Part{k, 2, 0});
        i = j;
      }
      return out;
    };

    // ---- step one: y1 = prod over the max(q-1, 1) factors of P2, applied to f ----
    // After it y = y1.  Unless a captured graph replays the later steps (their first launch
    // reads y) or no later step runs, step one writes y1 only, the first later step reads
    // y1, and the systems that stop before any later step get y = y1 at the end.  With an
    // odd number of factors the single launch comes first: it reads f, shared by the poles.
    a.count = nsys;
    const int nP = std::max(q - 1, 1);
    const bool dual = (graphs && !pr.on) || (fixed && cap <= 1);
    {
      const std::vector<Part> pl = plan(q, nP, kFacInF, dual ? kFacDual : 0, fuse, true);
      const T2* cur = nullptr;
      for (size_t i = 0; i < pl.size(); ++i) {
        const bool last = i + 1 == pl.size();
        T2* dst = last ? y1 : ((cur == wA) ? wB : wA);
        // every system is listed in order here: a lone first factor from f serves all
        // poles of a right-hand side in one pass
        const bool fan = i == 0 && pl[i].width == 1 && pl[i].kind == kFacInF;
        launch(pl[i].kind, pl[i].k, pl[i].width, cur, dst, (last && dual) ? y : nullptr, fan);
        cur = dst;
      }
      st.matvecs += (long long)(q - 1) * nsys;
      st.fp_steps += nsys;
    }
    const T2* y_first = dual ? y : y1;  // the iterate read by the first later step

    // ---- steps two and on: y <- L y + y1 ----
    // (a launch never writes its own input: a step made of a single launch goes through wA)
    const std::vector<Part> pl = plan(0, q, kFacResid, kFacAdd, fuse && q >= 3, false);
    const bool single = pl.size() == 1;
    // first launch of a step from y, with the ||f - (A - z) y||^2 partials of the current
    // iterate, the stopping test, and in adaptive mode the compacted list and the flags
    auto head = [&](bool read_flags, const T2* yin) {
      launch(pl[0].kind, pl[0].k, pl[0].width, yin, wA, nullptr);
      launch_fp_check(s, partial, nblk, nsys, sys0, nrhs, fnorm2, fixed_steps, reduce, max_steps, active, steps,
                      rnorm2);
      if (!fixed) {
        launch_build_list(s, active, nsys, list);
        if (read_flags)
          HFCI_HIP(hipMemcpyAsync(ctx.pinned_int, active, nsys * sizeof(int), hipMemcpyDeviceToHost, s));
      }
    };
    // the rest of a step: middle factors ping-pong between wA and wB, the last adds y1
    auto rest = [&]() {
      if (single) {
        copy_active<T2>(s, y, wA, active, nsys, n);
        return;
      }
      T2* cur = wA;
      for (size_t i = 1; i < pl.size(); ++i) {
        const bool last = i + 1 == pl.size();
        T2* dst = last ? y : ((cur == wA) ? wB : wA);
        launch(pl[i].kind, pl[i].k, pl[i].width, cur, dst, nullptr);
        cur = dst;
      }
    };
    auto read_active = [&]() {
      int na = 0;
      for (int k = 0; k < nsys; ++k) {
        hact[k] = ctx.pinned_int[k] != 0;
        na += hact[k];
      }
      return na;
    };
    int nact = nsys;
    if (!(graphs && !pr.on) && !fixed && nsys <= kPinnedIntHalf) {
      // Adaptive, pipelined: the launches of step `it` (sized for the systems that were
      // active after the previous test, an upper bound: the compacted list ends in -1s)
      // and the next step's head are queued before the host waits for this step's flags,
      // so the device never idles on the host's read-back.  Flags alternate between the
      // two halves of the pinned buffer; an event marks each read-back.
      hipEvent_t ev[2] = {ctx.step_event[0], ctx.step_event[1]};
      int* flags[2] = {ctx.pinned_int, ctx.pinned_int + kPinnedIntHalf};
      int* flags_dev[2] = {ctx.pinned_int_dev, ctx.pinned_int_dev + kPinnedIntHalf};
      auto head_to = [&](int slot, const T2* yin) {
        launch(pl[0].kind, pl[0].k, pl[0].width, yin, wA, nullptr);
        launch_fp_test(s, partial, nblk, nsys, sys0, nrhs, fnorm2, reduce, max_steps, active, steps, rnorm2, list,
                       flags_dev[slot]);
        HFCI_HIP(hipEventRecord(ev[slot], s));
      };
      std::vector<Fixup> fx;
      fixups = &fx;
      head_to(0, y_first);
      st.matvecs += nact;
      int slot = 0;
      for (int it = 1; it <= cap; ++it) {
        // queue the rest of step `it` and the head of step it + 1, then read step it's flags
        fx.clear();
        rest();
        head_to(slot ^ 1, y);
        HFCI_HIP(hipEventSynchronize(ev[slot]));
        int na = 0;
        for (int k = 0; k < nsys; ++k) {
          hact[k] = flags[slot][k] != 0;
          na += hact[k];
        }
        for (const Fixup& x : fx) pr.set_bytes(x.idx, launch_bytes(x.vecs, x.reads_f));
        st.matvecs += (long long)(q - 1) * na + na;
        st.fp_steps += na;
        nact = na;
        if (nact == 0) break;  // the queued rest and head found an empty list: no work
        a.count = nact;
        slot ^= 1;
      }
      fixups = nullptr;
    } else if (!(graphs && !pr.on)) {
      for (int it = 1; it <= cap; ++it) {
        if (fixed && it == cap) break;  // exact count: no final residual check needed
        head(!fixed, it == 1 ? y_first : y);
        st.matvecs += nact;
        if (!fixed) {
          HFCI_HIP(hipStreamSynchronize(s));
          if (pr.on) pr.harvest();
          nact = read_active();
        }
        if (nact == 0) break;
        a.count = nact;
        st.matvecs += (long long)(q - 1) * nact;
        st.fp_steps += nact;
        rest();
      }
    } else if (cap > 1 || !fixed) {
      // Graph replay: launches cover every system (stopped ones find -1 in the list and
      // exit), so one step's launch sequence is the same every step and is captured once:
      // adaptive [rest of step, head of the next step, read-back], fixed [head, rest].
      a.count = nsys;
      std::string key;
      auto put = [&](const void* p, size_t b) { key.append((const char*)p, b); };
      const void* ptrs[] = {f, y, y1, wA, wB, partial, active, list, steps, rnorm2, fnorm2, c.d_coef, c.d_poles,
                            kap, ctx.pinned_int};
      put(ptrs, sizeof(ptrs));
      const int ints[] = {(int)sizeof(T2), nsys, sys0, nrhs, q, c.cstride, fixed_steps, max_steps, nblk,
                          fuse ? 1 : 0, op.g.nx, op.g.ny, op.g.nz};
      put(ints, sizeof(ints));
      put(&reduce, sizeof(reduce));
      put(&op.g, sizeof(op.g));
      hipGraphExec_t exec = ctx.graphs.find(key);
      if (!exec) {
        hipGraph_t graph = nullptr;
        HFCI_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
          if (fixed) {
            head(false, y);
            rest();
          } else {
            rest();
            head(true, y);
          }
        } catch (...) {
          (void)hipStreamEndCapture(s, &graph);
          if (graph) (void)hipGraphDestroy(graph);
          throw;
        }
        HFCI_HIP(hipStreamEndCapture(s, &graph));
        const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HFCI_HIP(e);
        ctx.graphs.put(key, exec);
      }
      if (fixed) {
        for (int it = 1; it < cap; ++it) {
          HFCI_HIP(hipGraphLaunch(exec, s));
          st.matvecs += (long long)q * nsys;
          st.fp_steps += nsys;
        }
      } else {
        head(true, y);
        st.matvecs += nsys;
        HFCI_HIP(hipStreamSynchronize(s));
        nact = read_active();
        for (int it = 1; it <= cap && nact > 0; ++it) {
          st.matvecs += (long long)(q - 1) * nact;
          st.fp_steps += nact;
          HFCI_HIP(hipGraphLaunch(exec, s));
          HFCI_HIP(hipStreamSynchronize(s));
          st.matvecs += nact;
          nact = read_active();
        }
      }
    }
    // adaptive without the dual write: the systems that stopped before any later step
    // (steps <= 1) hold their iterate in y1 (fixed counts >= 2 run a later step on every
    // system); the caller selects it, or it is copied to y
    if (!dual && !fixed) {
      if (defer) {
        defer->y1 = y1;
        defer->steps = steps;
      } else {
        copy_unstepped<T2>(s, y, y1, steps, nsys, n);
      }
    }
  }
  if (steps_out) {
    HFCI_HIP(hipMemcpyAsync(ctx.pinned_int, steps, nsys * sizeof(int), hipMemcpyDeviceToHost, s));
    HFCI_HIP(hipStreamSynchronize(s));
    std::memcpy(steps_out, ctx.pinned_int, nsys * sizeof(int));
  }
  if (ctx.prof.on) {
    HFCI_HIP(hipStreamSynchronize(s));
    ctx.prof.harvest();
  }
}

}  // namespace

// Launch-shape autotuner: times the middle-factor kernel (the dominant launch of the
// fixed-point iteration) over nsys systems for every valid shape, one, two and (complex64)
// three factors per pass, and keeps the fastest per factor for this operator and precision.  Inputs are zeros and the factor is a fixed benign
// one: the kernel's time does not depend on the values.
template <typename T2>
KernelTune autotune_shapes(Op& op, int nsys, std::vector<std::pair<KernelTune, double>>& timings) {
  Ctx& ctx = *op.ctx;
  hipStream_t s = ctx.stream;
  const size_t n = op.n;
  const size_t vbytes = n * sizeof(T2);
  T2* win = (T2*)ctx.ws.get("fp_wA", (size_t)nsys * vbytes);
  T2* wout = (T2*)ctx.ws.get("fp_wB", (size_t)nsys * vbytes);
  FactorCoef* coef = (FactorCoef*)ctx.ws.get("tune_coef", 3 * sizeof(FactorCoef));
  PoleDev* pole = (PoleDev*)ctx.ws.get("tune_pole", sizeof(PoleDev));
  int* list = (int*)ctx.ws.get("tune_list", (size_t)nsys * sizeof(int));
  const FactorCoef c0[3] = {{1e-3, 0.0, 0.5, 0.0}, {1e-3, 0.0, 0.5, 0.0}, {1e-3, 0.0, 0.5, 0.0}};
  const PoleDev p0{0.5 * (op.b1 + op.b2), 0.5, 0.0, 0.0};
  std::vector<int> ids(nsys);
  for (int k = 0; k < nsys; ++k) ids[k] = k;
  HFCI_HIP(hipMemcpyAsync(coef, c0, sizeof(c0), hipMemcpyHostToDevice, s));
  HFCI_HIP(hipMemcpyAsync(pole, &p0, sizeof(p0), hipMemcpyHostToDevice, s));
  HFCI_HIP(hipMemcpyAsync(list, ids.data(), nsys * sizeof(int), hipMemcpyHostToDevice, s));
  launch_fill_zero(s, win, (size_t)nsys * vbytes);
  FactorArgs<T2> a{};
  a.win = win;
  a.wout = wout;
  a.coef = coef;
  a.poles = pole;
  a.list = list;
  a.count = nsys;
  a.sys0 = 0;
  a.nrhs = 1;
  a.cstride = 3;
  a.k = 0;
  KernelTune& cur = (sizeof(T2) == 8) ? op.g.tune32 : op.g.tune64;
  const KernelTune saved = cur;
  const void* kap = Prec<T2>::kappa(op);
  std::vector<KernelTune> cands;
  for (int cz : {0, 16, 64}) {
    for (int ty : {4, 8})
      for (int pd : {1, 2}) cands.push_back(KernelTune{0, ty, pd, cz, 0});
    for (int pd : {1, 2, 3}) cands.push_back(KernelTune{1, 4, pd, cz, 0});
    for (int pd : {2, 3}) cands.push_back(KernelTune{1, 8, pd, cz, 0});
  }
  // two factors per pass (its own 64 x 12 tiles; per-factor time = half a launch), with
  // the systems of a launch taken one, two or four at a time tile by tile
  // (kern 2: the complex64 pair kernel whose streams are loaded straight into LDS; kern 3:
  // the same with 64 x 28 tiles for the middle pairs, two planes ahead only)
  if (Launch<T2>::pair_fits(op.g))
    for (int kern : {1, 2, 3}) {
      if (kern >= 2 && sizeof(T2) != 8) continue;
      for (int cz : {0, 16, 64})
        for (int pd : {2, 3})
          for (int sg : {1, 2, 4})
            if ((sg == 1 || sg <= nsys) && !(kern == 3 && pd != 2)) cands.push_back(KernelTune{kern, 8, pd, cz, 1, sg});
    }
  // three middle factors per pass (kern 3, fuse 2; per-factor time = a third of a launch)
  if (sizeof(T2) == 8 && Launch<T2>::pair_fits(op.g))
    for (int cz : {0, 16, 64})
      for (int sg : {1, 2, 4})
        if (sg == 1 || sg <= nsys) cands.push_back(KernelTune{3, 8, 2, cz, 2, sg});
  hipEvent_t e0, e1;
  HFCI_HIP(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
  HFCI_HIP(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
  KernelTune best = saved;
  double best_ms = 1e300;
  timings.clear();
  try {
    for (const KernelTune& t : cands) {
      if (t.cz > 0 && t.cz >= op.g.nz) continue;  // same as one chunk per column: covered by cz = 0 or larger
      cur = t;
      if (t.fuse == 2 && !Launch<T2>::triple_runs(op.g)) continue;  // (an odd nx: the pairs' shape covers it)
      auto one = [&] {
        if (t.fuse == 2) Launch<T2>::factor_triple(s, op.g, kap, a);
        else if (t.fuse) Launch<T2>::factor_pair(s, op.g, kap, a, 0);
        else Launch<T2>::factor(s, op.g, kap, a, 0);
      };
      one();  // warm-up
      HFCI_HIP(hipEventRecord(e0, s));
      const int reps = 3;
      for (int r = 0; r < reps; ++r) one();
      HFCI_HIP(hipEventRecord(e1, s));
      HFCI_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      HFCI_HIP(hipEventElapsedTime(&ms, e0, e1));
      const double avg = ms / reps / (t.fuse == 2 ? 3.0 : t.fuse ? 2.0 : 1.0);  // per factor
      timings.emplace_back(t, avg);
      if (avg < best_ms) {
        best_ms = avg;
        best = t;
      }
    }
  } catch (...) {
    cur = saved;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  cur = best;
  return best;
}
template KernelTune autotune_shapes<float2>(Op&, int, std::vector<std::pair<KernelTune, double>>&);
template KernelTune autotune_shapes<double2>(Op&, int, std::vector<std::pair<KernelTune, double>>&);

namespace {

// Alg. 1 steps 1-3 in precision T2: w = sum sigma_j/z_j y_j, d = (Aw)^H f / |Aw|^2, out = d w.
template <typename T2>
void fci_body(const Op& op, const Contour& c, const hfci_solve_opts& o, int nrhs, const T2* f, double2* out,
              FciStats& st) {
  Ctx& ctx = *op.ctx;
  hipStream_t s = ctx.stream;
  const size_t n = op.n;
  const int J = c.J;
  int pb = o.pole_batch > 0 ? std::min(o.pole_batch, J) : J;
  T2* w = (T2*)ctx.ws.get("fci_w", (size_t)nrhs * n * sizeof(T2));
  T2* y = (T2*)ctx.ws.get("fci_y", (size_t)pb * nrhs * n * sizeof(T2));
  // quadrature weights of eq. rational: sigma_j / z_j
  double* cc = (double*)ctx.ws.get("fci_cc", (size_t)2 * J * sizeof(double));
  double* stage = ctx.pinned_dbl + kPinnedFciOffset;
  for (int j = 0; j < J; ++j) {
    const cd v = c.sigma[j] / c.z[j];
    stage[2 * j] = v.real();
    stage[2 * j + 1] = v.imag();
  }
  HFCI_HIP(hipMemcpyAsync(cc, stage, 2 * J * sizeof(double), hipMemcpyHostToDevice, s));
  if (op.form != 1) {
    // case two (eq. mat-2x2) or the spectral operator: every pole in one batch of shifted
    // solves, the same quadrature, and step 3 with the operator's own product
    T2* yall = (T2*)ctx.ws.get("fci_y", (size_t)J * nrhs * n * sizeof(T2));
    if (op.form == 2)
      shifted_solve_case_two<T2>(op, c, nrhs, f, yall, o.fp_steps, o.fp_reduce, o.fp_max_steps, nullptr, st);
    else
      shifted_solve_spectral<T2>(op, c, nrhs, f, yall, o.fp_steps, o.fp_reduce, o.fp_max_steps, nullptr, st);
    launch_combine<T2>(s, w, yall, cc, J, nrhs, n, false);
    const int nb2 = op.form == 2 ? b2_blocks(op.g) : spec_blocks(op.g);
    double* part2 = (double*)ctx.ws.get("fci_dpart", (size_t)nrhs * 3 * nb2 * sizeof(double));
    double* sums2 = (double*)ctx.ws.get("fci_dsums", (size_t)nrhs * 3 * sizeof(double));
    double* d2 = (double*)ctx.ws.get("fci_d", (size_t)nrhs * 2 * sizeof(double));
    if (op.form == 2) {
      launch_b2_dstep<T2>(s, op.g, Prec<T2>::kappa(op), nrhs, w, f, part2);
    } else {
      T2* sw = (T2*)ctx.ws.get("fci_sw", (size_t)nrhs * n * sizeof(T2));
      spectral_S<T2>(op, nrhs, w, sw);
      launch_spec_dstep<T2>(s, op.g, Prec<T2>::kappa(op), nrhs, w, sw, f, part2);
    }
    launch_reduce(s, part2, nb2, 3 * nrhs, sums2);
    launch_dfinish(s, sums2, nrhs, d2);
    st.matvecs += nrhs;
    launch_scale_out<T2>(s, out, w, d2, nrhs, n);
    return;
  }
  for (int p0 = 0; p0 < J; p0 += pb) {
    const int np = std::min(pb, J - p0);
    const bool graphs = o.graphs == 1 || (o.graphs < 0 && op.n <= ((size_t)1 << 16));
    Deferred<T2> dfr;
    fp_run<T2>(op, c, nrhs, f, y, p0 * nrhs, np * nrhs, o.fp_steps, o.fp_reduce, o.fp_max_steps, nullptr, st,
               graphs, &dfr);
    launch_combine<T2>(s, w, y, cc + 2 * p0, np, nrhs, n, p0 > 0, dfr.y1, dfr.steps);
  }
  // step 3: minimise ||f - d A w|| over d
  const int nblk = Launch<T2>::partial_blocks(op.g);
  double* part = (double*)ctx.ws.get("fci_dpart", (size_t)nrhs * 3 * nblk * sizeof(double));
  double* sums = (double*)ctx.ws.get("fci_dsums", (size_t)nrhs * 3 * sizeof(double));
  double* d = (double*)ctx.ws.get("fci_d", (size_t)nrhs * 2 * sizeof(double));
  Launch<T2>::dstep_partials(s, op.g, Prec<T2>::kappa(op), nrhs, w, f, part);
  launch_reduce(s, part, nblk, 3 * nrhs, sums);
  launch_dfinish(s, sums, nrhs, d);
  st.matvecs += nrhs;
  launch_scale_out<T2>(s, out, w, d, nrhs, n);
}

}  // namespace

template <typename T2>
void shifted_solve_batch(const Op& op, const Contour& c, int nrhs, const T2* f, T2* y, int fixed_steps,
                         double reduce, int max_steps, int* steps_out, FciStats& st) {
  fp_run<T2>(op, c, nrhs, f, y, 0, c.J * nrhs, fixed_steps, reduce, max_steps, steps_out, st);
}
template void shifted_solve_batch<float2>(const Op&, const Contour&, int, const float2*, float2*, int, double, int,
                                          int*, FciStats&);
template void shifted_solve_batch<double2>(const Op&, const Contour&, int, const double2*, double2*, int, double,
                                           int, int*, FciStats&);

void fci_apply(const Op& op, const Contour& c, const hfci_solve_opts& o, int nrhs, const double2* f, double2* out,
               FciStats& st) {
  Ctx& ctx = *op.ctx;
  if (o.precision == HFCI_F32) {
    float2* f32 = (float2*)ctx.ws.get("fci_f32", (size_t)nrhs * op.n * sizeof(float2));
    launch_convert_64_to_32(ctx.stream, f32, f, (size_t)nrhs * op.n);
    fci_body<float2>(op, c, o, nrhs, f32, out, st);
  } else {
    fci_body<double2>(op, c, o, nrhs, f, out, st);
  }
  if (o.k_in > 0)  // Alg. 1 step 4
    inner_steps(op, o.k_in, nrhs, f, out, st, o.inner_precond == 1 ? static_cast<Net*>(o.net) : nullptr);
}

namespace {

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

// Givens rotation (c, s) with [c s; -conj(s) c] [a; b] = [rho; 0], c real.
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

}  // namespace

// Flexible GMRES(m) with CGS2 and Givens, FP64, batched over right-hand sides.
// Krylov bases are laid out [j][rhs][n] so that the FCI of step j reads V[j] and
// writes Z[j] for all right-hand sides as two contiguous blocks.
hfci_status fgmres_solve(const Op& op, const Contour* c, const hfci_solve_opts& o, int nrhs, const double2* f,
                         double2* u, hfci_stats* stats) {
  Ctx& ctx = *op.ctx;
  hipStream_t s = ctx.stream;
  const auto t_wall0 = std::chrono::steady_clock::now();
  const size_t n = op.n;
  const int m = o.restart;
  const size_t vs = (size_t)nrhs * n;  // stride between basis vectors of the same rhs
  double2* b = (double2*)ctx.ws.get("gm_b", vs * sizeof(double2));
  double2* V = (double2*)ctx.ws.get("gm_V", (size_t)(m + 1) * vs * sizeof(double2));
  double2* Z = (double2*)ctx.ws.get("gm_Z", (size_t)m * vs * sizeof(double2));
  double2* stage_in = nullptr;
  double2* stage_out = nullptr;
  const int nbs = Launch<double2>::partial_blocks(op.g);
  const int nbb = blas_blocks(n);
  const int npart = std::max(nbs, nbb * 2 * (m + 1));
  double* part = (double*)ctx.ws.get("gm_part", (size_t)npart * sizeof(double));
  // per rhs: h1[2(m+1)], h2[2(m+1)], hn2[1], beta2[1], y[2m]
  const int hstride = 4 * (m + 1) + 2 + 2 * m;
  double* hdev = (double*)ctx.ws.get("gm_h", (size_t)nrhs * hstride * sizeof(double));
  double* hhost = ctx.pinned_dbl;
  if ((size_t)nrhs * hstride > kPinnedFciOffset) throw Error(HFCI_E_ARG, "too many right-hand sides for the restart length");

  for (int r = 0; r < nrhs; ++r) launch_copy_scaled64(s, b + r * n, f + r * n, n, op.s);
  std::vector<double> bnorm(nrhs);
  for (int r = 0; r < nrhs; ++r) launch_norm2_partial(s, b + r * n, false, n, part + (size_t)r * nbb);
  launch_reduce(s, part, nbb, nrhs, hdev);
  HFCI_HIP(hipMemcpyAsync(hhost, hdev, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
  HFCI_HIP(hipStreamSynchronize(s));
  for (int r = 0; r < nrhs; ++r) bnorm[r] = std::sqrt(hhost[r]);

  std::vector<char> done(nrhs, 0);
  std::vector<double> relres(nrhs, 1.0);
  std::vector<std::vector<cd>> H(nrhs), G(nrhs), SN(nrhs);
  std::vector<std::vector<double>> CS(nrhs);
  std::vector<int> kr(nrhs, 0);
  int its = 0, cycles = 0;
  long long res_mv = 0;
  int harvested = 0, n_accept = 0, n_fallback = 0;
  double t_net = 0.0, net_rho_sum = 0.0, fci_rho_sum = 0.0;
  long net_rho_n = 0, fci_rho_n = 0;
  int net_rejects_in_row = 0;
  FciStats fst;
  double t_fci = 0, t_arn = 0;
  Timer tm(s), tf(s);  // tf: the preconditioner of an Arnoldi step, read at the step's sync
  hfci_status status = HFCI_OK;

  for (int r = 0; r < nrhs; ++r)
    if (bnorm[r] == 0.0) {
      launch_fill_zero(s, u + r * n, n * sizeof(double2));
      done[r] = 1;
      relres[r] = 0.0;
    }

  while (true) {
    // true FP64 residual of every unfinished rhs, written into V[0]
    tm.start();
    std::vector<int> act;
    for (int r = 0; r < nrhs; ++r) {
      if (done[r]) continue;
      if (op.form == 2) {
        launch_b2_residual64(s, op.g, op.kappa64, b + r * n, u + r * n, V + r * n, part, nbs);
      } else if (op.form == 3) {
        spectral_S<double2>(op, 1, u + r * n, V + r * n);
        launch_spec_residual64(s, op.g, op.kappa64, b + r * n, u + r * n, V + r * n, V + r * n, part, nbs);
      } else
        launch_residual64(s, op.g, op.kappa64, b + r * n, u + r * n, V + r * n, part);
      launch_reduce(s, part, nbs, 1, hdev + (size_t)r * hstride + 4 * (m + 1) + 1);
      act.push_back(r);
      ++res_mv;
    }
    for (int r : act)
      HFCI_HIP(hipMemcpyAsync(hhost + r, hdev + (size_t)r * hstride + 4 * (m + 1) + 1, sizeof(double),
                              hipMemcpyDeviceToHost, s));
    HFCI_HIP(hipStreamSynchronize(s));
    t_arn += tm.stop_ms();
    std::vector<int> cyc;
    for (int r : act) {
      const double beta = std::sqrt(hhost[r]);
      if (!(beta == beta)) throw Error(HFCI_E_NUMERIC, "NaN in the FGMRES residual");
      relres[r] = beta / bnorm[r];
      if (relres[r] <= o.tol)
        done[r] = 1;
      else
        cyc.push_back(r);
    }
    if (o.verbose) {
      double mx = 0.0;
      for (int r : act) mx = std::max(mx, relres[r]);
      std::fprintf(stderr, "[hfci] cycle %d: its %d, max true relres %.3e, %zu of %d rhs open, fci %.0f ms, "
                   "arnoldi %.0f ms\n", cycles, its, mx, cyc.size(), nrhs, t_fci, t_arn);
      std::fflush(stderr);
    }
    if (cyc.empty()) break;
    if (its >= o.max_it) {
      status = HFCI_W_NOCONV;
      break;
    }
    ++cycles;
    std::vector<double> beta(nrhs, 0.0);
    for (int r : cyc) {
      beta[r] = std::sqrt(hhost[r]);
      launch_scale_inv(s, V + r * n, V + r * n, n, hdev + (size_t)r * hstride + 4 * (m + 1) + 1);
      H[r].assign((size_t)(m + 1) * m, cd(0, 0));
      G[r].assign(m + 1, cd(0, 0));
      G[r][0] = beta[r];
      CS[r].assign(m, 0.0);
      SN[r].assign(m, cd(0, 0));
      kr[r] = 0;
    }
    std::vector<int> live = cyc;  // rhs still extending this cycle
    for (int j = 0; j < m && !live.empty(); ++j) {
      // ---- preconditioner: Z[j] = FCI(V[j]) for the live right-hand sides ----
      tf.start();
      const int nl = (int)live.size();
      const bool all = (nl == nrhs);
      const double2* fin = V + (size_t)j * vs;
      double2* fout = Z + (size_t)j * vs;
      if (!all) {
        stage_in = (double2*)ctx.ws.get("gm_stage_in", (size_t)nl * n * sizeof(double2));
        stage_out = (double2*)ctx.ws.get("gm_stage_out", (size_t)nl * n * sizeof(double2));
        for (int k = 0; k < nl; ++k)
          HFCI_HIP(hipMemcpyAsync(stage_in + k * n, V + (size_t)j * vs + live[k] * n, n * sizeof(double2),
                                  hipMemcpyDeviceToDevice, s));
        fin = stage_in;
        fout = stage_out;
      }
      const bool consult_net = o.precond == HFCI_PRECOND_LEARNED &&
                               (o.learned_patience == 0 || net_rejects_in_row < o.learned_patience);
      if (o.precond == HFCI_PRECOND_LEARNED && !consult_net) {
        fci_apply(op, *c, o, nl, fin, fout, fst);
        n_fallback += nl;
      } else if (consult_net) {
        // the network proposes z = N(v).  Alg. 1 step 3 on the proposal: d = (Az)^H v / |Az|^2
        // minimises ||v - d A z||; with |v| = 1 that residual is sqrt(1 - |(Az)^H v|^2 / |Az|^2).
        // A proposal is kept (scaled by d) when that residual is at most learned_tau times the
        // mean of FCI's own scaled residual over this solve's FCI steps (and below 0.99);
        // otherwise, and until FCI has run once, z = FCI(v).
        Timer tn(s);
        tn.start();
        o.net->apply(op, nl, fin, fout);
        const int nbs2 = Launch<double2>::partial_blocks(op.g);
        double* jp = (double*)ctx.ws.get("gm_jpart", (size_t)nl * 3 * nbs2 * sizeof(double));
        double* js = (double*)ctx.ws.get("gm_jsums", (size_t)nl * 3 * sizeof(double));
        double* jd = (double*)ctx.ws.get("gm_jd", (size_t)nl * 2 * sizeof(double));
        Launch<double2>::dstep_partials(s, op.g, op.kappa64, nl, fout, fin, jp);
        launch_reduce(s, jp, nbs2, 3 * nl, js);
        launch_dfinish(s, js, nl, jd);
        launch_scale_out<double2>(s, fout, fout, jd, nl, n);
        fst.matvecs += nl;
        double* jh = ctx.pinned_dbl + kPinnedFciOffset + 1024;
        HFCI_HIP(hipMemcpyAsync(jh, js, 3 * nl * sizeof(double), hipMemcpyDeviceToHost, s));
        t_net += tn.stop_ms();
        std::vector<int> rej;
        const double thr = fci_rho_n > 0 ? std::min(0.99, o.learned_tau * fci_rho_sum / fci_rho_n) : -1.0;
        for (int k = 0; k < nl; ++k) {
          const double num2 = jh[3 * k] * jh[3 * k] + jh[3 * k + 1] * jh[3 * k + 1], den = jh[3 * k + 2];
          const double rho = den > 0.0 ? std::sqrt(std::max(0.0, 1.0 - num2 / den)) : 1.0;
          net_rho_sum += rho;
          ++net_rho_n;
          if (!(den > 0.0) || !(rho <= thr)) rej.push_back(k);
          if (o.verbose > 1)
            std::fprintf(stderr, "[hfci] step %d slot %d: network residual %.3f, threshold %.3f\n", its, k, rho, thr);
        }
        n_accept += nl - (int)rej.size();
        n_fallback += (int)rej.size();
        net_rejects_in_row = rej.size() == (size_t)nl ? net_rejects_in_row + 1 : 0;
        if (!rej.empty()) {
          const int nr = (int)rej.size();
          double2* rin = (double2*)ctx.ws.get("gm_rej_in", (size_t)nr * n * sizeof(double2));
          double2* rout = (double2*)ctx.ws.get("gm_rej_out", (size_t)nr * n * sizeof(double2));
          for (int k = 0; k < nr; ++k)
            HFCI_HIP(hipMemcpyAsync(rin + k * n, fin + rej[k] * n, n * sizeof(double2), hipMemcpyDeviceToDevice, s));
          fci_apply(op, *c, o, nr, rin, rout, fst);
          for (int k = 0; k < nr; ++k)
            HFCI_HIP(hipMemcpyAsync(fout + rej[k] * n, rout + k * n, n * sizeof(double2), hipMemcpyDeviceToDevice, s));
          // FCI's own scaled residual from its step-3 sums ((Aw)^H v, |Aw|^2; |v| = 1)
          const double* fs = (const double*)ctx.ws.get("fci_dsums", (size_t)nr * 3 * sizeof(double));
          HFCI_HIP(hipMemcpyAsync(jh, fs, 3 * nr * sizeof(double), hipMemcpyDeviceToHost, s));
          HFCI_HIP(hipStreamSynchronize(s));
          for (int k = 0; k < nr; ++k) {
            const double num2 = jh[3 * k] * jh[3 * k] + jh[3 * k + 1] * jh[3 * k + 1], den = jh[3 * k + 2];
            if (den > 0.0) {
              fci_rho_sum += std::sqrt(std::max(0.0, 1.0 - num2 / den));
              ++fci_rho_n;
            }
          }
        }
      } else if (c && o.precond == HFCI_PRECOND_FCI) {
        fci_apply(op, *c, o, nl, fin, fout, fst);
      } else {
        HFCI_HIP(hipMemcpyAsync(fout, fin, (size_t)nl * n * sizeof(double2), hipMemcpyDeviceToDevice, s));
      }
      if (!all)
        for (int k = 0; k < nl; ++k)
          HFCI_HIP(hipMemcpyAsync(Z + (size_t)j * vs + live[k] * n, stage_out + k * n, n * sizeof(double2),
                                  hipMemcpyDeviceToDevice, s));
      // training-pair harvest: (v_j, z_j) as complex64
      for (int r : live) {
        if (harvested >= o.harvest_cap) break;
        launch_convert_64_to_32(s, (float2*)o.harvest_v + (size_t)harvested * n, V + (size_t)j * vs + r * n, n);
        launch_convert_64_to_32(s, (float2*)o.harvest_z + (size_t)harvested * n, Z + (size_t)j * vs + r * n, n);
        ++harvested;
      }
      tf.stop();  // no wait here: the Arnoldi launches queue behind the preconditioner
      // ---- Arnoldi: w = A z_j, CGS2 against V[0..j], normalise ----
      tm.start();
      for (int r : live) {
        double2* w = V + (size_t)(j + 1) * vs + r * n;
        const double2* Vr = V + r * n;
        double* hb = hdev + (size_t)r * hstride;
        if (op.form == 2)
          launch_b2_apply<double2>(s, op.g, op.kappa64, 1, Z + (size_t)j * vs + r * n, w, 0.0, 0.0);
        else if (op.form == 3)
          spectral_apply<double2>(op, 1, Z + (size_t)j * vs + r * n, w, 0.0, 0.0);
        else
          Launch<double2>::apply(s, op.g, op.kappa64, 0.0, 0.0, 1, Z + (size_t)j * vs + r * n, w);
        launch_cgs2(s, Vr, j + 1, n, vs, w, part, hb, hb + 2 * (m + 1), hb + 4 * (m + 1));
        launch_scale_inv(s, w, w, n, hb + 4 * (m + 1));
        HFCI_HIP(hipMemcpyAsync(hhost + (size_t)r * hstride, hb, (4 * (m + 1) + 1) * sizeof(double),
                                hipMemcpyDeviceToHost, s));
      }
      fst.matvecs += nl;
      HFCI_HIP(hipStreamSynchronize(s));
      t_arn += tm.stop_ms();
      t_fci += tf.elapsed_ms();
      ++its;
      // ---- Givens update of the Hessenberg column on the host ----
      std::vector<int> next;
      for (int r : live) {
        const double* hh = hhost + (size_t)r * hstride;
        std::vector<cd>& Hr = H[r];
        auto Hat = [&](int i, int jj) -> cd& { return Hr[(size_t)i * m + jj]; };
        for (int i = 0; i <= j; ++i)
          Hat(i, j) = cd(hh[2 * i] + hh[2 * (m + 1) + 2 * i], hh[2 * i + 1] + hh[2 * (m + 1) + 2 * i + 1]);
        const double hn = std::sqrt(hh[4 * (m + 1)]);
        if (!(hn == hn)) throw Error(HFCI_E_NUMERIC, "NaN in the Arnoldi process");
        Hat(j + 1, j) = hn;
        for (int i = 0; i < j; ++i) {
          const cd x = Hat(i, j), yv = Hat(i + 1, j);
          Hat(i, j) = CS[r][i] * x + SN[r][i] * yv;
          Hat(i + 1, j) = -std::conj(SN[r][i]) * x + CS[r][i] * yv;
        }
        double cs;
        cd sn, rho;
        givens(Hat(j, j), Hat(j + 1, j), cs, sn, rho);
        CS[r][j] = cs;
        SN[r][j] = sn;
        Hat(j, j) = rho;
        Hat(j + 1, j) = 0.0;
        G[r][j + 1] = -std::conj(sn) * G[r][j];
        G[r][j] = cs * G[r][j];
        kr[r] = j + 1;
        relres[r] = std::abs(G[r][j + 1]) / bnorm[r];
        if (!(relres[r] <= o.tol) && its < o.max_it && hn > 0.0) next.push_back(r);
      }
      live = next;
      if (its >= o.max_it) break;
    }
    // ---- u += Z_k y_k with H_k y_k = g_k (back substitution) ----
    tm.start();
    for (int r : cyc) {
      const int k = kr[r];
      std::vector<cd> yv(k);
      for (int i = k - 1; i >= 0; --i) {
        cd acc = G[r][i];
        for (int l = i + 1; l < k; ++l) acc -= H[r][(size_t)i * m + l] * yv[l];
        yv[i] = acc / H[r][(size_t)i * m + i];
      }
      double* yd = hhost + (size_t)r * hstride + 4 * (m + 1) + 2;
      for (int i = 0; i < k; ++i) {
        yd[2 * i] = yv[i].real();
        yd[2 * i + 1] = yv[i].imag();
      }
      HFCI_HIP(hipMemcpyAsync(hdev + (size_t)r * hstride + 4 * (m + 1) + 2, yd, 2 * k * sizeof(double),
                              hipMemcpyHostToDevice, s));
      launch_multiaxpy(s, u + r * n, Z + r * n, k, n, vs, hdev + (size_t)r * hstride + 4 * (m + 1) + 2, 1.0);
    }
    HFCI_HIP(hipStreamSynchronize(s));
    t_arn += tm.stop_ms();
  }
  if (stats) {
    stats->its = its;
    stats->restarts = cycles;
    stats->matvecs = fst.matvecs + res_mv;
    stats->fp_steps = fst.fp_steps;
    double mx = 0;
    for (double v : relres) mx = std::max(mx, v);
    stats->final_relres = mx;
    stats->time_fci_ms = t_fci;
    stats->harvested = harvested;
    stats->learned_accepted = n_accept;
    stats->learned_fallbacks = n_fallback;
    stats->time_net_ms = t_net;
    stats->net_rho_mean = net_rho_n ? net_rho_sum / net_rho_n : 0.0;
    stats->fci_rho_mean = fci_rho_n ? fci_rho_sum / fci_rho_n : 0.0;
    stats->time_arnoldi_ms = t_arn;
    stats->time_total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_wall0).count();
  }
  return status;
}

}  // namespace hfci
