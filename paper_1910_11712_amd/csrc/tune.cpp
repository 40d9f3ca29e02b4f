// Autotuner of launch shapes.  A moments plan has a few launch-shape choices
// whose best setting depends on the batch (how many matrices of which sizes)
// and on the device rather than on the arithmetic:
//   * the width of the triangular solves' column groups (4, 8 or 16 right-hand
//     columns per work-group): fewer, wider groups re-read each factor less,
//     more, narrower groups fill more CUs when there are few matrices;
//   * paired 256-thread solve groups (two per CU) for the large matrices,
//     which cover each other's barrier waits when there are many of them;
//   * 256-thread panel groups for panels of at most 256 rows (two per CU)
//     against one 512-thread group per CU;
//   * the LU's look-ahead fork point: the rest of a step's update starts as
//     soon as the panel is done (best when the panels bound the time) or
//     after the update of the next panel's columns (which then does not wait
//     for CU slots behind the larger update);
//   * the LU's panel width, 64 or 128: wider panels give the trailing update
//     twice the products per C byte but lengthen the panel chain.
// Every setting computes the moments to the same accuracy; all but the panel
// width give the same bits (the panel width changes the factors' rounding).
// The tuner times each candidate with full moment passes on the plan's own
// buffers (HIP events on the caller's stream, median of a few passes), keeps
// the fastest if it beats the built-in setting by more than 2% (the built-in
// one otherwise), and caches it per plan signature for the life of the process:
// a later plan with the same launch shapes applies the cached setting without
// timing.  It searches coordinate-wise: the LU settings first (panel groups
// by fork point, with the built-in solve setting), then the solve settings
// with the winning LU one.
#include <algorithm>
#include <cfloat>
#include <climits>
#include <cstdint>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "handle.hpp"

namespace nep {

namespace {

struct TuneState {
  std::mutex mu;
  bool on = false;
  int reps = 3;
  std::map<std::string, MomentsPlan::Knobs> cache;
  std::vector<nep_tune_cand> last;  // candidates timed by the last tuning
  int last_chosen = -1, last_cached = 0;
};

TuneState& tune_state() {
  static TuneState s;
  return s;
}

// 1 when the large matrices run as paired groups under knobs k
int eff_paired(const SolvePlan& sp, int prec, const MomentsPlan::Knobs& k, int L) {
  const bool can = prec == NEP_PREC_C32_IR64 && k.lg <= 8 && sp.rpt <= 2 && sp.nbig > 0;
  if (!can) return 0;
  if (k.paired >= 0) return k.paired;
  return (long long)sp.nbig * ceil_div(L, k.lg) >= 2048 ? 1 : 0;
}

}  // namespace

nep_status MomentsPlan::apply(const Knobs& k, hipStream_t st) {
  solve_set_lg(sp_, k.lg, opt.L);
  sp_.paired = k.paired;
  if (k.jb != lu_.jb) {  // another panel width: a new LU schedule and prefix table
    NEP_CHECK(k.jb == 64 || k.jb == 128, NEP_ERR_ARG, "panel width %d", k.jb);
    lu_.build(sorted_, opt.prec, k.jb);
    const size_t need = sizeof(int) * std::max<size_t>(1, lu_.prefix.size());
    if (dlu_prefix_.bytes < need) NEP_TRY(dlu_prefix_.alloc(need));
    if (!lu_.prefix.empty())
      NEP_HIP(hipMemcpyAsync(dlu_prefix_.p, lu_.prefix.data(), sizeof(int) * lu_.prefix.size(),
                             hipMemcpyHostToDevice, st));
  }
  lu_.small_min = k.small_min;
  lu_.early_fork = k.early_fork;
  return NEP_OK;
}

void MomentsPlan::candidates(std::vector<Knobs>& lu, std::vector<Knobs>& solve) const {
  const Knobs base = knobs();
  lu.assign(1, base);
  solve.assign(1, base);
  const bool f32 = opt.prec == NEP_PREC_C32_IR64;
  std::vector<int> smins{base.small_min};
  if (f32) {
    // the steps that take the small groups under a threshold; thresholds that
    // give the same steps are the same launches
    auto steps_small = [&](int smin) {
      std::vector<char> v;
      for (const auto& s : lu_.steps) v.push_back(s.nact > s.nsmall && s.nact - s.nsmall >= smin ? 1 : 0);
      return v;
    };
    std::vector<std::vector<char>> seen{steps_small(base.small_min)};
    for (int smin : {0, INT_MAX}) {
      auto v = steps_small(smin);
      if (std::find(seen.begin(), seen.end(), v) != seen.end()) continue;
      seen.push_back(v);
      smins.push_back(smin);
    }
  }
  // panel widths: the built-in one, and the other where it differs (a plan
  // whose largest matrix has more than 64 rows); the other fork point
  // matters where a step forks at all (more than one step), the built-in one
  // being early for 64-wide complex-FP32 panels and late otherwise
  std::vector<int> jbs{base.jb};
  if (!sorted_.empty() && sorted_[0].n > 64) jbs.push_back(base.jb == 64 ? 128 : 64);
  for (int jb : jbs) {
    const int fork_base = f32 && jb == 64 ? 1 : 0;
    std::vector<int> forks{base.early_fork};
    if ((sorted_.empty() ? 0 : sorted_[0].n) > jb) forks.push_back(1 - fork_base);
    for (int fk : forks)
      for (int smin : smins) {
        if (jb == base.jb && fk == base.early_fork && smin == base.small_min) continue;  // [0]
        Knobs k = base;
        k.small_min = smin;
        k.early_fork = fk;
        k.jb = jb;
        lu.push_back(k);
      }
  }
  std::vector<std::pair<int, int>> seen{{base.lg, eff_paired(sp_, opt.prec, base, opt.L)}};
  for (int lg : {4, 8, 16}) {
    if (!solve_lg_fits(sp_, lg, opt.L, opt.prec)) continue;
    for (int pr : {0, 1}) {
      Knobs k = base;
      k.lg = lg;
      k.paired = pr;
      const std::pair<int, int> e{lg, eff_paired(sp_, opt.prec, k, opt.L)};
      if (std::find(seen.begin(), seen.end(), e) != seen.end()) continue;
      seen.push_back(e);
      solve.push_back(k);
    }
  }
}

std::string MomentsPlan::signature() const {
  std::uint64_t h = 1469598103934665603ull;  // FNV-1a over the sorted sizes
  for (const auto& m : sorted_) {
    h ^= (std::uint64_t)m.n;
    h *= 1099511628211ull;
  }
  char buf[160];
  std::snprintf(buf, sizeof buf, "prec%d N%d L%d sweeps%d fb%d m%zu sizes%016llx", opt.prec, opt.N, opt.L,
                opt.max_refine, opt.fallback, sorted_.size(), (unsigned long long)h);
  return buf;
}

nep_status MomentsPlan::time_pass(hipStream_t st, int reps, float& ms) {
  struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  NEP_HIP(hipEventCreate(&ev.a));
  NEP_HIP(hipEventCreate(&ev.b));
  NEP_TRY(enqueue(st, false));  // untimed: first touch of this setting's kernels
  std::vector<float> t;
  for (int r = 0; r < reps; ++r) {
    NEP_HIP(hipEventRecord(ev.a, st));
    NEP_TRY(enqueue(st, false));
    NEP_HIP(hipEventRecord(ev.b, st));
    NEP_HIP(hipEventSynchronize(ev.b));
    float x = 0.f;
    NEP_HIP(hipEventElapsedTime(&x, ev.a, ev.b));
    t.push_back(x);
  }
  std::sort(t.begin(), t.end());
  ms = t[t.size() / 2];
  return NEP_OK;
}

nep_status tune_plan(MomentsPlan& plan, hipStream_t st) {
  TuneState& T = tune_state();
  const std::string sig = plan.signature();
  int reps;
  {
    std::lock_guard<std::mutex> g(T.mu);
    auto it = T.cache.find(sig);
    if (it != T.cache.end()) {
      NEP_TRY(plan.apply(it->second, st));
      T.last.clear();
      T.last_chosen = -1;
      T.last_cached = 1;
      return NEP_OK;
    }
    if (!T.on) {  // the built-in setting, not timed
      T.last.clear();
      T.last_chosen = -1;
      T.last_cached = 0;
      return NEP_OK;
    }
    reps = T.reps;
  }
  std::vector<MomentsPlan::Knobs> lu, sv;
  plan.candidates(lu, sv);
  std::vector<nep_tune_cand> rec;
  MomentsPlan::Knobs best = plan.knobs();
  int chosen = 0;
  if (lu.size() + sv.size() > 2) {
    float best_ms = FLT_MAX;
    auto measure = [&](const MomentsPlan::Knobs& k) -> nep_status {
      NEP_TRY(plan.apply(k, st));
      float ms = 0.f;
      NEP_TRY(plan.time_pass(st, reps, ms));
      rec.push_back(nep_tune_cand{k.lg, k.paired, k.small_min, k.early_fork, k.jb, ms});
      if (ms < best_ms) {
        best_ms = ms;
        best = k;
        chosen = (int)rec.size() - 1;
      }
      return NEP_OK;
    };
    // a setting replaces the built-in one only if it is faster by more than
    // the passes' run-to-run spread (about 1%); within it, the built-in stays
    constexpr float kMargin = 0.98f;
    const MomentsPlan::Knobs builtin = lu[0];
    for (const auto& k : lu) NEP_TRY(measure(k));
    const float builtin_ms = rec[0].ms;
    auto settle = [&]() {
      if (chosen != 0 && best_ms > kMargin * builtin_ms) {
        best = builtin;
        best_ms = builtin_ms;
        chosen = 0;
      }
    };
    settle();
    // the built-in solve setting was timed with every LU setting above
    for (size_t i = 1; i < sv.size(); ++i) {
      MomentsPlan::Knobs k = sv[i];
      k.small_min = best.small_min;
      k.early_fork = best.early_fork;
      k.jb = best.jb;
      NEP_TRY(measure(k));
    }
    settle();
  } else {
    rec.push_back(nep_tune_cand{best.lg, best.paired, best.small_min, best.early_fork, best.jb, 0.f});  // nothing to choose
  }
  NEP_TRY(plan.apply(best, st));
  std::lock_guard<std::mutex> g(T.mu);
  T.cache[sig] = best;
  T.last = rec;
  T.last_chosen = chosen;
  T.last_cached = 0;
  return NEP_OK;
}

}  // namespace nep

using namespace nep;

extern "C" {

nep_status nep_tune_set(int on, int reps) {
  NEP_CHECK(reps >= 1 && reps <= 64, NEP_ERR_ARG, "reps must be in 1..64");
  TuneState& T = tune_state();
  std::lock_guard<std::mutex> g(T.mu);
  T.on = on != 0;
  T.reps = reps;
  return NEP_OK;
}

nep_status nep_tune_report(int max, nep_tune_cand* cand, int* ncand, int* chosen, int* cached) {
  NEP_CHECK(max >= 0 && (max == 0 || cand != nullptr), NEP_ERR_ARG, "bad candidate array");
  NEP_CHECK(ncand && chosen && cached, NEP_ERR_ARG, "null output");
  TuneState& T = tune_state();
  std::lock_guard<std::mutex> g(T.mu);
  *ncand = (int)T.last.size();
  *chosen = T.last_chosen;
  *cached = T.last_cached;
  for (int i = 0; i < max && i < (int)T.last.size(); ++i) cand[i] = T.last[i];
  return NEP_OK;
}

nep_status nep_tune_clear(void) {
  TuneState& T = tune_state();
  std::lock_guard<std::mutex> g(T.mu);
  T.cache.clear();
  T.last.clear();
  T.last_chosen = -1;
  T.last_cached = 0;
  return NEP_OK;
}

}  // extern "C"
