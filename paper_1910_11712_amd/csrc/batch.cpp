// Batched moments: many problems (uneven n) in one plan, optionally replayed
// from a captured HIP graph.
#include <memory>
#include <vector>

#include "handle.hpp"

namespace nep {

struct Batch {
  std::unique_ptr<MomentsPlan> plan;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use_graph = false;
  bool pending = false;  // a run was enqueued and not yet finished
  ~Batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

}  // namespace nep

struct nep_batch_s {
  nep::Batch impl;
};

using namespace nep;

extern "C" {

nep_status nep_batch_create(int nprob, const nep_split* h, const nep_contour* g, const nep_ciss_opts* o,
                            const void* const* V, void* const* S, int use_graph, void* stream, nep_batch* out) {
  NEP_CHECK(out != nullptr, NEP_ERR_ARG, "null output");
  *out = nullptr;
  NEP_CHECK(nprob >= 1 && h && g && V && S, NEP_ERR_ARG, "bad batch arrays");
  PlanOptions po;
  NEP_TRY(check_opts(o, po));
  std::vector<PlanProblem> probs;
  for (int p = 0; p < nprob; ++p) {
    NEP_CHECK(h[p] != nullptr && V[p] != nullptr && S[p] != nullptr, NEP_ERR_ARG, "problem %d: null handle/buffer",
              p);
    NEP_TRY(check_contour(&g[p]));
    probs.push_back(PlanProblem{&h[p]->impl.op, g[p], (const c128*)V[p], (c128*)S[p]});
  }
  auto b = std::make_unique<nep_batch_s>();
  b->impl.stream = (hipStream_t)stream;
  b->impl.plan = std::make_unique<MomentsPlan>();
  NEP_TRY(b->impl.plan->build(probs, po, b->impl.stream));
  NEP_TRY(tune_plan(*b->impl.plan, (hipStream_t)stream));
  b->impl.use_graph = use_graph != 0;
  if (b->impl.use_graph) {
    hipStream_t st = b->impl.stream;
    bool own = false;
    if (st == nullptr) {  // the legacy default stream cannot be captured
      NEP_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      own = true;
    }
    NEP_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    nep_status es = b->impl.plan->enqueue(st, false);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(st, &graph);
    if (own) (void)hipStreamDestroy(st);
    NEP_TRY(es);
    NEP_HIP(ce);
    b->impl.graph = graph;
    NEP_HIP(hipGraphInstantiate(&b->impl.exec, graph, nullptr, nullptr, 0));
  }
  *out = b.release();
  return NEP_OK;
}

nep_status nep_batch_run(nep_batch b, nep_ciss_stats* st) {
  NEP_CHECK(b != nullptr, NEP_ERR_ARG, "null batch");
  Batch& B = b->impl;
  if (B.use_graph) {
    NEP_HIP(hipGraphLaunch(B.exec, B.stream));
    B.plan->replayed();
  } else {
    NEP_TRY(B.plan->enqueue(B.stream, false));
  }
  B.pending = true;
  if (!st) return NEP_OK;
  return nep_batch_wait(b, st);
}

nep_status nep_batch_wait(nep_batch b, nep_ciss_stats* st) {
  NEP_CHECK(b != nullptr, NEP_ERR_ARG, "null batch");
  Batch& B = b->impl;
  NEP_CHECK(B.pending, NEP_ERR_ARG, "no batch run pending");
  B.pending = false;
  RunResult rr;
  nep_status s = B.plan->finish(B.stream, rr, true);
  if (st)
    for (int p = 0; p < B.plan->nprob && p < (int)rr.stats.size(); ++p) st[p] = rr.stats[p];
  return s;
}

nep_status nep_batch_destroy(nep_batch* b) {
  NEP_CHECK(b != nullptr, NEP_ERR_ARG, "null batch pointer");
  if (*b) {
    (void)hipStreamSynchronize((*b)->impl.stream);
    delete *b;
  }
  *b = nullptr;
  return NEP_OK;
}

nep_status nep_ciss_moments_batch(int nprob, const nep_split* h, const nep_contour* g, const nep_ciss_opts* o,
                                  const void* const* V, void* const* S, nep_ciss_stats* st) {
  nep_batch b = nullptr;
  NEP_TRY(nep_batch_create(nprob, h, g, o, V, S, 0, o ? o->stream : nullptr, &b));
  std::vector<nep_ciss_stats> tmp(nprob);
  nep_status s = nep_batch_run(b, st ? st : tmp.data());
  nep_batch_destroy(&b);
  return s;
}

}  // extern "C"
