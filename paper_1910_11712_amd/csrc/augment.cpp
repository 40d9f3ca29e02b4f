// Work on resident factors: moments of further probe blocks, the eigenvalue
// count by the argument principle, and the end-to-end eigenvalue call that
// augments the probes when the moments' rank saturates.
//
// Eigenvalues of T are the zeros of det T(z) (Section 2, eq. (nep)), so the
// number inside a contour is the winding number of det T along it.  Each
// node's LU gives det T(z_j) = sign(P) prod_k u_kk; the phase differences of
// consecutive nodes, each taken in (-pi, pi], sum to 2 pi times the count
// when the nodes are dense enough that det T turns by less than pi between
// neighbours (the largest step is reported so the caller can judge).
#include <cmath>
#include <vector>

#include "handle.hpp"

namespace nep {

static nep_status count_from_plan(MomentsPlan& plan, int n, hipStream_t st, int* count, double* max_step,
                                  double* winding) {
  const int G = plan.nnodes;
  std::vector<int> info(G), bad(G);
  NEP_HIP(hipMemcpyAsync(info.data(), plan.info(), sizeof(int) * G, hipMemcpyDeviceToHost, st));
  NEP_HIP(hipMemcpyAsync(bad.data(), plan.nodes().bad, sizeof(int) * G, hipMemcpyDeviceToHost, st));
  NEP_HIP(hipStreamSynchronize(st));
  for (int g = 0; g < G; ++g) {
    NEP_CHECK(!bad[g], NEP_ERR_NOT_HOLOMORPHIC, "node %d lies on a pole or branch cut of some f_i", g);
    NEP_CHECK(info[g] >= n, NEP_ERR_SINGULAR, "node %d: exact zero pivot", g);
  }
  std::vector<double> la, arg;
  NEP_TRY(plan.logdet(st, la, arg));
  for (int g = 0; g < G; ++g)
    NEP_CHECK(std::isfinite(la[g]) && std::isfinite(arg[g]), NEP_ERR_SINGULAR,
              "node %d: det T(z) is zero or not finite in the factor precision", g);
  winding_count(arg, count, max_step, winding);
  return NEP_OK;
}

}  // namespace nep

using namespace nep;

extern "C" {

nep_status nep_ciss_moments_more(nep_split h, const void* V, void* S, long long s_stride, nep_ciss_stats* st) {
  NEP_CHECK(h != nullptr, NEP_ERR_ARG, "null handle");
  return h->impl.moments_more(V, S, s_stride, nullptr, st);
}

nep_status nep_ciss_count(nep_split h, int* count, double* max_step, double* winding) {
  NEP_CHECK(h != nullptr && count != nullptr, NEP_ERR_ARG, "null handle or output");
  Split& s = h->impl;
  NEP_CHECK(s.plan != nullptr, NEP_ERR_ARG, "no resident factors: call nep_ciss_moments on this handle first");
  NEP_CHECK(!s.pending, NEP_ERR_ARG, "the last moments call on this handle has not been waited for");
  const hipStream_t st = s.last_stream ? s.last_stream : s.stream;
  return count_from_plan(*s.plan, s.op.n, st, count, max_step, winding);
}

nep_status nep_count_eigs(nep_split h, const nep_contour* g, int N, int prec, int* count, double* max_step,
                          double* winding) {
  NEP_CHECK(h != nullptr && count != nullptr, NEP_ERR_ARG, "null handle or output");
  NEP_TRY(check_contour(g));
  NEP_CHECK(N >= 4 && N <= 4096, NEP_ERR_ARG, "N must be in 4..4096");
  NEP_CHECK(prec == NEP_PREC_FP64 || prec == NEP_PREC_C32_IR64, NEP_ERR_ARG, "unknown precision %d", prec);
  Split& s = h->impl;
  MomentsPlan plan;
  PlanOptions po;
  po.N = N;
  po.L = 1;
  po.K = 1;
  po.prec = prec;
  po.max_refine = 0;
  po.fallback = 0;
  std::vector<PlanProblem> probs{PlanProblem{&s.op, *g, nullptr, nullptr}};
  NEP_TRY(plan.build(probs, po, s.stream));
  NEP_TRY(plan.factor(s.stream));
  return count_from_plan(plan, s.op.n, s.stream, count, max_step, winding);
}

nep_status nep_eigs(nep_split h, const nep_contour* g, const nep_ciss_opts* o, const nep_extract_opts* e,
                    const void* V, int Lmax, int* m, double* lambda, void* X, double* eta, int* inside,
                    double* sigma, int* L_used, nep_ciss_stats* st) {
  NEP_CHECK(h != nullptr && o != nullptr && e != nullptr, NEP_ERR_ARG, "null handle or options");
  NEP_CHECK(V != nullptr && m != nullptr && L_used != nullptr, NEP_ERR_ARG, "null probes or outputs");
  PlanOptions po;
  NEP_TRY(check_opts(o, po));
  NEP_CHECK(Lmax >= po.L && Lmax % po.L == 0 && Lmax <= 256, NEP_ERR_ARG,
            "Lmax must be a multiple of L, at most 256");
  Split& s = h->impl;
  const int n = s.op.n, L = po.L, KK = 2 * po.K;
  const long long stride = (long long)n * Lmax;
  if (s.saug.bytes < sizeof(c128) * (size_t)stride * KK) NEP_TRY(s.saug.alloc(sizeof(c128) * (size_t)stride * KK));
  c128* S = s.saug.as<c128>();
  const c128* Vb = static_cast<const c128*>(V);
  nep_ciss_stats tmp;
  nep_ciss_stats* stp = st ? st : &tmp;
  NEP_TRY(s.moments(g, o, Vb, S, stp, stride));
  void* strm = o->stream;
  int b = 1;
  for (;;) {
    *L_used = b * L;
    const nep_status r = extract_strided(s, g, o, b * L, S, stride, e, m, lambda, X, eta, inside, sigma, nullptr);
    // augment only on saturation (every singular value significant), not
    // when the moments vanish
    if (r != NEP_ERR_RANK || *m != po.K * b * L || b * L >= Lmax) return r;
    NEP_TRY(s.moments_more(Vb + (size_t)b * n * L, S + (size_t)b * n * L, stride, strm, stp));
    ++b;
  }
}

}  // extern "C"
