// Split-operator handle (behind the opaque nep_split of the C ABI).
#pragma once

#include <cmath>
#include <memory>
#include <vector>

#include "plan.hpp"

namespace nep {

struct ExtractWork;  // extraction workspace (extract.cpp)

struct Split {
  SplitOperator op;
  // unique over the process (never reused, unlike the handle's address):
  // keys the server's resident factors
  unsigned long long uid = next_uid();
  static unsigned long long next_uid();
  hipStream_t stream = nullptr;
  hipStream_t last_stream = nullptr;
  std::unique_ptr<DevMem> mats[kMaxTerms];
  std::unique_ptr<DevMem> diags[kMaxTerms];
  std::unique_ptr<DevMem> lrG[kMaxTerms], lrH[kMaxTerms];
  DevMem norms, fn_nodes, fn_coef, fn_roots;
  std::unique_ptr<MomentsPlan> plan;  // resident factors of the last call
  std::shared_ptr<ExtractWork> xw;
  bool pending = false;
  nep_contour last_g{};               // contour of the last moments call
  DevMem saug;                        // augmented moments of nep_eigs (grow-only)
  std::vector<FnNode> h_fn_nodes;     // host copies of the function tree
  std::vector<c128> h_fn_coef;
  struct nep_split_s* adj = nullptr;  // the adjoint operator T^*, made on demand
  ~Split();
  // T^*(z) = T(conj z)^*: conjugate-transposed A_i, functions with conjugated
  // parameters (f^*(z) = conj(f(conj z)))
  nep_status init_adjoint(const Split& src);

  nep_status init(int n, int ell, const nep_mat* A, const nep_fn* f, hipStream_t st);
  nep_status moments(const nep_contour* g, const nep_ciss_opts* o, const void* V, void* S, nep_ciss_stats* st,
                     long long s_stride = 0);
  // moments of new probes on the factors resident from the last call
  nep_status moments_more(const void* V, void* S, long long s_stride, void* stream, nep_ciss_stats* st);
  nep_status wait(nep_ciss_stats* st);
  nep_status eval_fns(int m, const c128* zh, std::vector<c128>& out, std::vector<int>& bad, bool deriv);
};

nep_status check_contour(const nep_contour* g);
nep_status check_opts(const nep_ciss_opts* o, PlanOptions& po);

// Extraction (extract.hip).  wk: the workspace to use, or nullptr for the
// handle's own.  A workspace grows and never shrinks; blocks allocated while
// an ArenaScope is alive come from that arena.
std::shared_ptr<ExtractWork> make_extract_work();
nep_status extract(Split& h, const nep_contour* g, const nep_ciss_opts* o, const void* S,
                   const nep_extract_opts* e, int* m_out, double* lambda, void* X, double* eta, int* inside,
                   double* sigma, ExtractWork* wk);
// The same with L_eff probe columns in S and moment blocks sstride elements
// apart (0: n * L_eff), for moments augmented by further probe blocks.
nep_status extract_strided(Split& h, const nep_contour* g, const nep_ciss_opts* o, int L_eff, const void* S,
                           long long sstride, const nep_extract_opts* e, int* m_out, double* lambda, void* X,
                           double* eta, int* inside, double* sigma, ExtractWork* wk);
// Winding number of det T(z) along the nodes' closed polygon from per-node
// arguments in node order: count = round(total / 2 pi), with the largest
// phase step.
void winding_count(const std::vector<double>& arg, int* count, double* max_step, double* winding);

}  // namespace nep

struct nep_split_s {
  nep::Split impl;
};
