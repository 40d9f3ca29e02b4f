// Host-side moment plan: layout of a batch of problems x nodes on the device,
// launch tables, buffers, and the launch sequence (eager or captured).
#pragma once

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "engine.hpp"

namespace nep {

// A device memory arena: one allocation carved into 256-byte aligned blocks.
// Returning a block never synchronizes the device (hipFree does), so a
// server can recycle workspaces while other streams run.
class Arena {
 public:
  Arena() = default;
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  ~Arena();
  nep_status init(size_t bytes);
  void* take(size_t bytes);  // nullptr if no free block is large enough
  void give(void* p);
  size_t capacity() const { return size_; }
  size_t in_use() const;

 private:
  char* base_ = nullptr;
  size_t size_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length, coalesced
  std::map<size_t, size_t> used_;  // offset -> length
  mutable std::mutex mu_;
};

// While an ArenaScope is alive, DevMem allocations made on this thread come
// from the arena instead of hipMalloc.
class ArenaScope {
 public:
  explicit ArenaScope(Arena* a);
  ~ArenaScope();

 private:
  Arena* prev_;
};

// Small pinned host blocks (64 bytes) from one process-wide pinned slab, so
// plans do not pair hipHostMalloc/hipHostFree per build.
void* pinned_take();
void pinned_give(void* p);

// Device memory block owned by a plan or a handle.
struct DevMem {
  void* p = nullptr;
  size_t bytes = 0;
  Arena* arena = nullptr;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  ~DevMem() { release(); }
  nep_status alloc(size_t b);
  void release();
  template <typename T>
  T* as() const { return reinterpret_cast<T*>(p); }
};

// What the operator handle contributes to a plan.
struct SplitOperator {
  int n = 0, ell = 0;
  int a_cplx = 0;
  int is_cplx[kMaxTerms] = {0};
  const void* dA[kMaxTerms] = {nullptr};  // device row-major copies
  int is_diag[kMaxTerms] = {0};           // A_i diagonal (detected at creation)
  const c128* dDiag[kMaxTerms] = {nullptr};  // its diagonal (n complex)
  // real banded A_i (detected at creation, half-bandwidth 1..kBandMax): the
  // real-term residual runs each tile over its rows' band only
  int band_w[kMaxTerms] = {0};
  // real low-rank A_i = G H^T (detected at creation, rank 1..kLowRankMax):
  // G and H n x r row-major (device)
  int lr_rank[kMaxTerms] = {0};
  const double* dLrG[kMaxTerms] = {nullptr};
  const double* dLrH[kMaxTerms] = {nullptr};
  const double* dnormA = nullptr;
  std::vector<double> normA;
  const FnNode* dfn_nodes = nullptr;
  const c128* dfn_coef = nullptr;
  int fn_root[kMaxTerms] = {0};
};

struct PlanProblem {
  const SplitOperator* op;
  nep_contour g;
  const c128* V;
  c128* S;
  const c128* zpts = nullptr;  // explicit points (device, N) instead of g's nodes
  long long s_stride = 0;      // elements between moment blocks of S; 0: n*L
  // with zpts: coefficients c_ji (device, N x ell, at j*ell + i) that take the
  // place of f_i(z_j), so the plan factors sum_i c_ji A_i (e.g. a rational
  // interpolant of T evaluated at a shift)
  const c128* fpts = nullptr;
};

struct PlanOptions {
  int N = 32, L = 8, K = 2, prec = NEP_PREC_C32_IR64;
  int max_refine = 5, fallback = 1;
  double tol = kDefaultRefineTol;
};

struct RunResult {
  nep_status status = NEP_OK;           // first failing problem's status
  std::vector<nep_ciss_stats> stats;    // per problem
  std::vector<nep_status> pstatus;      // per problem
};

class MomentsPlan {
 public:
  MomentsPlan() = default;
  MomentsPlan(const MomentsPlan&) = delete;
  MomentsPlan& operator=(const MomentsPlan&) = delete;
  ~MomentsPlan() {
    if (hcounter_) pinned_give(hcounter_);
    if (hstat_) (void)hipHostFree(hstat_);
    if (ev_counter_) (void)hipEventDestroy(ev_counter_);
    for (hipEvent_t e : ev_lu_)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : {ls_.ev_fork, ls_.ev_join, ls_.ev_side[0], ls_.ev_side[1], ls_.ev_side_done})
      if (e) (void)hipEventDestroy(e);
    if (ls_.aux) (void)hipStreamDestroy(ls_.aux);
    if (ls_.side) (void)hipStreamDestroy(ls_.side);
  }
  // Builds layout, tables and buffers.  Problems may differ in n (ragged).
  // The device tables are uploaded on st, the stream the plan's passes run
  // on, so they are in place for the first pass on any kind of stream (an
  // upload through the null stream is not ordered before work on a
  // non-blocking stream).
  nep_status build(const std::vector<PlanProblem>& probs, const PlanOptions& o, hipStream_t st);
  // Enqueues the whole moment path on st.  eager=true lets the host stop the
  // refinement loop early (one small read-back per sweep); eager=false runs a
  // fixed number of sweeps with device-side skipping (graph capture safe).
  nep_status enqueue(hipStream_t st, bool eager, bool refactor = true);
  // A replay of a captured enqueue was launched: the next finish() starts
  // from the graph's own state (no FP64 re-solve of this run done yet).
  void replayed() {
    fallback_pending_ = false;
    lu_timed_ = false;
  }
  // Waits, reads back device status and fills per-problem stats.  With
  // allow_fallback, nodes that a fixed-sweep (non-eager) run left
  // unconverged are re-solved in FP64 and the moments recomputed (if the
  // options enable the fallback).
  nep_status finish(hipStream_t st, RunResult& out, bool allow_fallback);
  // Device buffers shared with extraction and the server.
  const c128* Y() const { return dY_.as<c128>(); }
  // Shifted solves on resident factors (a plan over explicit points or the
  // contour's nodes): factor() assembles and factors T at every node;
  // solve_rhs() then sets Y_j = T(z_j)^{-1} R_j for the right-hand sides the
  // caller wrote into R (layout [row][node][column], n x N*L per problem),
  // any number of times.
  nep_status factor(hipStream_t st);
  nep_status solve_rhs(hipStream_t st);
  c128* R_mut() { return dR_.as<c128>(); }
  c128* Y_mut() { return dY_.as<c128>(); }
  const NodeArrays& nodes() const { return na_; }
  // The factors of the plan's first (largest) matrix, for solves outside the
  // batched solve kernels: its descriptor, the factor buffer, the row map and
  // its diagonal-block inverses ([block][0: L, 1: U][64][64], row-major).
  const MatDesc& mat0() const { return sorted_[0]; }
  // element offset of problem p's block in the R and Y buffers
  long long y_offset(int p) const { return hpd_[p].offY; }
  const void* factor_base() const { return dT_.p; }
  const int* row_map() const { return drows_.as<int>(); }
  const void* dinv0() const { return ddinv_.as<char>() + dinv_off_[0] * (opt.prec == NEP_PREC_FP64 ? 16 : 8); }
  const int* info() const { return dinfo_.as<int>(); }
  // Per node (global index): log|det T(z_g)| and arg det T(z_g) in (-pi, pi]
  // from the resident factors (the product of the pivots and the sign of the
  // row permutation), read back to host arrays of nnodes entries.
  nep_status logdet(hipStream_t st, std::vector<double>& logabs, std::vector<double>& arg);
  // Rebinds caller buffers (V, S) and contours without rebuilding; the
  // descriptor upload is queued on st.
  nep_status rebind(const std::vector<PlanProblem>& probs, hipStream_t st);
  // For a pass on resident factors (enqueue with refactor=false): the listed
  // problems take new probes V and moment buffers S (s_stride n*L), every
  // other problem sits out the pass (nothing of its operator is read, its
  // previous buffers are not touched).  The descriptor upload is queued on st.
  // s_stride: elements between the moment blocks of each S (nullptr: n*L).
  nep_status rebind_members(const std::vector<int>& member, const std::vector<const c128*>& V,
                            const std::vector<c128*>& S, hipStream_t st,
                            const std::vector<long long>* s_stride = nullptr);
  // Frees the FP64 re-solve buffers (allocated again if a later pass needs them).
  void release_fallback();
  bool matches(const std::vector<PlanProblem>& probs, const PlanOptions& o) const;

  // Launch-shape knobs of the plan (see LuPlan::small_min and early_fork,
  // SolvePlan::lg and paired); every setting computes the same moments.
  struct Knobs {
    int lg, paired, small_min, early_fork, jb;
  };
  Knobs knobs() const { return Knobs{sp_.lg, sp_.paired, lu_.small_min, lu_.early_fork, lu_.jb}; }
  // applies k; a different panel width rebuilds the LU schedule and its
  // device prefix table (uploaded on st)
  nep_status apply(const Knobs& k, hipStream_t st);
  // The candidate settings that differ for this plan's shapes: [0] is the
  // built-in choice; LU candidates first, then the solve's.
  void candidates(std::vector<Knobs>& lu, std::vector<Knobs>& solve) const;
  // Identifies plans whose launches have the same shapes: precision, N, L,
  // sweeps and the multiset of matrix sizes.
  std::string signature() const;
  // Time one full moment pass (fixed sweeps, no host read-back) per rep on st
  // and return the median in ms (after one untimed pass).
  nep_status time_pass(hipStream_t st, int reps, float& ms);
  size_t device_bytes() const { return total_bytes_; }
  static size_t estimate_bytes(int n, int N, int L, int prec);

  PlanOptions opt;
  int nprob = 0, nnodes = 0, Lmax = 0;

 private:
  nep_status upload_problems(const std::vector<PlanProblem>& probs, hipStream_t st);
  template <typename P>
  nep_status enqueue_t(hipStream_t st, bool eager, bool refactor);
  template <typename P>
  nep_status run_fallback(hipStream_t st);
  template <typename P>
  nep_status factor_t(hipStream_t st);
  template <typename P>
  nep_status solve_rhs_t(hipStream_t st);

  std::vector<ProbDesc> hpd_;
  std::vector<LrJob> lr_jobs_;  // low-rank terms of real problems (Z = H^T Y per residual)
  DevMem dlrz_;                 // their Z blocks
  DevMem dlrzp_;                // partial sums of one Z block (the jobs run in turn on one stream)
  std::vector<MatDesc> sorted_;
  std::vector<int> prob_of_sorted_;
  LuPlan lu_;
  SolvePlan sp_;
  ProblemTables pt_;
  std::vector<int> hprefix_;
  DevMem dpd_, dmd_, dprefix_, dlu_prefix_;
  DevMem dT_, drows_, drows_snap_, dinfo_, dY_, dR_, dnode_, dir_, dT64_, dW_;
  DevMem ddinv_, ddinv_off_, ddinv64_, dlinv_, dlinv64_, darrive_;
  std::vector<long long> dinv_off_;
  long long dinv_elems_ = 0;
  NodeArrays na_{};
  IrState ir_{};
  int* hcounter_ = nullptr;  // pinned host read-back
  hipEvent_t ev_counter_ = nullptr;  // marks the counter read-back of a sweep
  hipEvent_t ev_lu_[2] = {nullptr, nullptr};  // around the LU of an eager pass (ms_lu)
  bool lu_timed_ = false;
  DevMem dstat_;                     // status block gathered for finish()
  char* hstat_ = nullptr;            // its pinned host copy
  size_t hstat_bytes_ = 0;
  LuStreams ls_;  // look-ahead LU streams (default priority) and events
  size_t total_bytes_ = 0;
  long long t_elems_ = 0, w_elems_ = 0, y_elems_ = 0;
  int rows_total_ = 0;
  int sweeps_run_ = 0;
  bool fallback_pending_ = false;
  std::vector<int> fallback_count_;  // per problem, nodes re-solved in FP64
  std::vector<int> na_prob_host_;    // problem of each node (host copy)
};

nep_status configure_kernels();

// Applies the cached launch-shape setting for the plan's signature, or, with
// tuning on and none cached, times the candidates on st and keeps the fastest
// (tune.cpp).
nep_status tune_plan(MomentsPlan& plan, hipStream_t st);

}  // namespace nep
