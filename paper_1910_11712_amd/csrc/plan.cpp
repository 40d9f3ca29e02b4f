// Moment plan: layout, tables, buffers and the launch sequence of the
// contour-integral moment path for one or many problems.
#include "plan.hpp"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>

namespace nep {

static_assert(kSolveBlk == kSolveBlkLu, "the LU writes the solve's diagonal-block inverses");

// --------------------------------------------------------------------------
static thread_local Arena* tls_arena = nullptr;

ArenaScope::ArenaScope(Arena* a) : prev_(tls_arena) { tls_arena = a; }
ArenaScope::~ArenaScope() { tls_arena = prev_; }

Arena::~Arena() {
  if (base_) (void)hipFree(base_);
}

nep_status Arena::init(size_t bytes) {
  bytes = (bytes + 255) / 256 * 256;
  hipError_t e = hipMalloc((void**)&base_, bytes);
  if (e != hipSuccess) {
    base_ = nullptr;
    (void)hipGetLastError();
    set_error("arena allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    return NEP_ERR_OOM;
  }
  size_ = bytes;
  free_.clear();
  used_.clear();
  free_[0] = bytes;
  return NEP_OK;
}

void* Arena::take(size_t bytes) {
  bytes = (bytes + 255) / 256 * 256;
  std::lock_guard<std::mutex> lk(mu_);
  for (auto it = free_.begin(); it != free_.end(); ++it) {  // first fit
    if (it->second < bytes) continue;
    const size_t off = it->first, len = it->second;
    free_.erase(it);
    if (len > bytes) free_[off + bytes] = len - bytes;
    used_[off] = bytes;
    return base_ + off;
  }
  return nullptr;
}

void Arena::give(void* q) {
  std::lock_guard<std::mutex> lk(mu_);
  const size_t off = (size_t)((char*)q - base_);
  auto u = used_.find(off);
  if (u == used_.end()) return;
  size_t start = off, len = u->second;
  used_.erase(u);
  auto nx = free_.lower_bound(start);
  if (nx != free_.end() && nx->first == start + len) {  // merge with the next block
    len += nx->second;
    nx = free_.erase(nx);
  }
  if (nx != free_.begin()) {  // merge with the previous block
    auto pv = std::prev(nx);
    if (pv->first + pv->second == start) {
      start = pv->first;
      len += pv->second;
      free_.erase(pv);
    }
  }
  free_[start] = len;
}

size_t Arena::in_use() const {
  std::lock_guard<std::mutex> lk(mu_);
  size_t t = 0;
  for (const auto& kv : used_) t += kv.second;
  return t;
}

namespace {
struct PinnedSlab {
  std::mutex mu;
  char* base = nullptr;
  std::vector<int> free_slots;
  static constexpr int kSlots = 1024, kSlot = 64;
};
PinnedSlab& slab() {
  static PinnedSlab s;
  return s;
}
}  // namespace

void* pinned_take() {
  PinnedSlab& s = slab();
  std::lock_guard<std::mutex> lk(s.mu);
  if (!s.base) {
    if (hipHostMalloc((void**)&s.base, (size_t)PinnedSlab::kSlots * PinnedSlab::kSlot, hipHostMallocDefault) !=
        hipSuccess) {
      s.base = nullptr;
      (void)hipGetLastError();
      return nullptr;
    }
    for (int i = PinnedSlab::kSlots - 1; i >= 0; --i) s.free_slots.push_back(i);
  }
  if (s.free_slots.empty()) return nullptr;
  const int i = s.free_slots.back();
  s.free_slots.pop_back();
  return s.base + (size_t)i * PinnedSlab::kSlot;
}

void pinned_give(void* p) {
  PinnedSlab& s = slab();
  std::lock_guard<std::mutex> lk(s.mu);
  if (!s.base || p == nullptr) return;
  s.free_slots.push_back((int)(((char*)p - s.base) / PinnedSlab::kSlot));
}

// --------------------------------------------------------------------------
nep_status DevMem::alloc(size_t b) {
  release();
  if (b == 0) return NEP_OK;
  if (tls_arena) {
    p = tls_arena->take(b);
    if (!p) {
      set_error("arena has no free block of %zu bytes", b);
      return NEP_ERR_OOM;
    }
    arena = tls_arena;
    bytes = b;
    return NEP_OK;
  }
  hipError_t e = hipMalloc(&p, b);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    set_error("device allocation of %zu bytes failed: %s", b, hipGetErrorString(e));
    return NEP_ERR_OOM;
  }
  bytes = b;
  return NEP_OK;
}

void DevMem::release() {
  if (p) {
    if (arena) arena->give(p);
    else (void)hipFree(p);
  }
  p = nullptr;
  bytes = 0;
  arena = nullptr;
}

static int pad_ld(int n) {
  int ld = (n + 15) / 16 * 16;
  if (ld % 512 == 0) ld += 16;  // avoid power-of-two row strides
  return ld;
}

static size_t elem_size(int prec) { return prec == NEP_PREC_FP64 ? sizeof(c128) : sizeof(c64); }

size_t MomentsPlan::estimate_bytes(int n, int N, int L, int prec) {
  const size_t ld = pad_ld(n);
  size_t b = (size_t)N * ld * n * elem_size(prec);        // factors
  b += (size_t)N * n * sizeof(int);                        // row maps
  b += (size_t)N * ((n + 63) / 64) * 2 * 64 * 64 * elem_size(prec);  // diagonal-block inverses
  b += 2 * (size_t)N * kLuMaxJB * kLuMaxJB * elem_size(prec);        // panel inverses (two halves)
  b += 2 * (size_t)n * N * L * sizeof(c128);               // Y, R
  if (prec != NEP_PREC_FP64 && n >= kSolveBlockedMinN)     // blocked-solve right-hand sides
    b += (size_t)N * ((n + 63) / 64 * 64) * L * sizeof(c64);
  b += (size_t)N * (kMaxTerms + kMaxMoments + 8) * sizeof(c128) + (size_t)N * kNormStride * 16;
  return b;
}

bool MomentsPlan::matches(const std::vector<PlanProblem>& probs, const PlanOptions& o) const {
  if ((int)probs.size() != nprob) return false;
  if (o.N != opt.N || o.L != opt.L || o.K != opt.K || o.prec != opt.prec) return false;
  for (int p = 0; p < nprob; ++p)
    if (probs[p].op->n != hpd_[p].n || probs[p].op->ell != hpd_[p].ell || probs[p].op->a_cplx != hpd_[p].a_cplx)
      return false;
  return true;
}

nep_status MomentsPlan::upload_problems(const std::vector<PlanProblem>& probs, hipStream_t st) {
  // Z blocks of the low-rank terms of real problems (the complex-term
  // residual multiplies every term densely)
  size_t zelems = 0;
  for (int p = 0; p < nprob; ++p)
    if (!probs[p].op->a_cplx)
      for (int i = 0; i < probs[p].op->ell; ++i) zelems += (size_t)probs[p].op->lr_rank[i] * opt.N * opt.L;
  if (zelems > 0 && dlrz_.bytes < sizeof(c128) * zelems) NEP_TRY(dlrz_.alloc(sizeof(c128) * zelems));
  // Z = H^T Y sums over the problem's n rows: cut into S ranges (at most 16,
  // at least 256 rows each, a multiple of 32) so that enough groups run;
  // the partial sums of one job at a time live in dlrzp_.
  auto lr_split = [](int n, int& S, int& srows) {
    S = std::max(1, std::min(16, n / 256));
    srows = ((n + S - 1) / S + 31) / 32 * 32;
    S = (n + srows - 1) / srows;
  };
  size_t pelems = 0;
  for (int p = 0; p < nprob; ++p)
    if (!probs[p].op->a_cplx)
      for (int i = 0; i < probs[p].op->ell; ++i) {
        int S, srows;
        lr_split(probs[p].op->n, S, srows);
        if (probs[p].op->lr_rank[i] > 0 && S > 1)
          pelems = std::max(pelems, (size_t)S * probs[p].op->lr_rank[i] * opt.N * opt.L);
      }
  if (pelems > 0 && dlrzp_.bytes < sizeof(c128) * pelems) NEP_TRY(dlrzp_.alloc(sizeof(c128) * pelems));
  lr_jobs_.clear();
  size_t zoff = 0;
  for (int p = 0; p < nprob; ++p) {
    ProbDesc& D = hpd_[p];
    const PlanProblem& q = probs[p];
    for (int i = 0; i < kMaxTerms; ++i) {
      const int rk = (i < q.op->ell && !q.op->a_cplx) ? q.op->lr_rank[i] : 0;
      D.a_lr[i] = rk;
      D.LrG[i] = rk > 0 ? q.op->dLrG[i] : nullptr;
      D.LrZ[i] = rk > 0 ? dlrz_.as<c128>() + zoff : nullptr;
      if (rk > 0) {
        int S, srows;
        lr_split(D.n, S, srows);
        lr_jobs_.push_back(LrJob{q.op->dLrH[i], dlrz_.as<c128>() + zoff, D.offY, D.n, rk, opt.N * opt.L,
                                 S > 1 ? dlrzp_.as<c128>() : nullptr, S, srows});
        zoff += (size_t)rk * opt.N * opt.L;
      }
    }
    D.kind = q.g.kind;
    D.c = c128{q.g.c[0], q.g.c[1]};
    D.rho = q.g.rho;
    D.v = q.g.kind == 1 ? q.g.v : 1.0;
    D.V = q.V;
    D.S = q.S;
    D.ell = q.op->ell;
    D.a_cplx = q.op->a_cplx;
    for (int i = 0; i < kMaxTerms; ++i) {
      D.A[i] = i < q.op->ell ? q.op->dA[i] : nullptr;
      D.a_is_cplx[i] = i < q.op->ell ? q.op->is_cplx[i] : 0;
      D.a_is_diag[i] = i < q.op->ell ? q.op->is_diag[i] : 0;
      D.Adiag[i] = i < q.op->ell ? q.op->dDiag[i] : nullptr;
      D.a_bw[i] = i < q.op->ell ? q.op->band_w[i] : 0;
      D.fn_root[i] = i < q.op->ell ? q.op->fn_root[i] : 0;
    }
    D.normA = q.op->dnormA;
    D.fn_nodes = q.op->dfn_nodes;
    D.fn_coef = q.op->dfn_coef;
    D.zpts = q.zpts;
    D.fpts = q.zpts != nullptr ? q.fpts : nullptr;
    D.s_stride = q.s_stride > 0 ? q.s_stride : (long long)D.n * D.L;
    D.active = 1;
  }
  NEP_HIP(hipMemcpyAsync(dpd_.p, hpd_.data(), sizeof(ProbDesc) * nprob, hipMemcpyHostToDevice, st));
  return NEP_OK;
}

nep_status MomentsPlan::rebind(const std::vector<PlanProblem>& probs, hipStream_t st) {
  NEP_CHECK((int)probs.size() == nprob, NEP_ERR_ARG, "rebind: problem count changed");
  return upload_problems(probs, st);
}

nep_status MomentsPlan::rebind_members(const std::vector<int>& member, const std::vector<const c128*>& V,
                                       const std::vector<c128*>& S, hipStream_t st,
                                       const std::vector<long long>* s_stride) {
  NEP_CHECK(member.size() == V.size() && member.size() == S.size(), NEP_ERR_ARG, "rebind: size mismatch");
  NEP_CHECK(s_stride == nullptr || s_stride->size() == member.size(), NEP_ERR_ARG, "rebind: stride count");
  for (auto& D : hpd_) D.active = 0;
  for (size_t k = 0; k < member.size(); ++k) {
    const int p = member[k];
    NEP_CHECK(p >= 0 && p < nprob, NEP_ERR_ARG, "rebind: member %d out of range", p);
    NEP_CHECK(!hpd_[p].active, NEP_ERR_ARG, "rebind: member %d bound twice", p);
    ProbDesc& D = hpd_[p];
    D.active = 1;
    D.V = V[k];
    D.S = S[k];
    D.zpts = nullptr;
    D.fpts = nullptr;
    D.s_stride = s_stride != nullptr ? (*s_stride)[k] : (long long)D.n * D.L;
    NEP_CHECK(D.s_stride >= (long long)D.n * D.L, NEP_ERR_ARG, "rebind: moment stride below n*L");
  }
  NEP_HIP(hipMemcpyAsync(dpd_.p, hpd_.data(), sizeof(ProbDesc) * nprob, hipMemcpyHostToDevice, st));
  return NEP_OK;
}

void MomentsPlan::release_fallback() {
  dT64_.release();
  ddinv64_.release();
  dlinv64_.release();
}

nep_status MomentsPlan::build(const std::vector<PlanProblem>& probs, const PlanOptions& o, hipStream_t st) {
  opt = o;
  nprob = (int)probs.size();
  Lmax = o.L;
  hpd_.assign(nprob, ProbDesc{});
  std::vector<int> hprob, hj;
  std::vector<MatDesc> all;
  long long offT = 0, offW = 0, offY = 0;
  int offRow = 0, g = 0;
  for (int p = 0; p < nprob; ++p) {
    const int n = probs[p].op->n;
    ProbDesc& D = hpd_[p];
    D.n = n;
    D.N = o.N;
    D.L = o.L;
    D.KK = 2 * o.K;
    D.node0 = g;
    D.ld = pad_ld(n);
    D.offT0 = offT;
    D.strideT = (long long)D.ld * n;
    D.offW0 = offW;
    D.offY = offY;
    D.offRow0 = offRow;
    for (int j = 0; j < o.N; ++j, ++g) {
      MatDesc m;
      m.n = n;
      m.ld = D.ld;
      m.offT = offT + (long long)j * D.strideT;
      m.offRow = offRow + j * n;
      m.node = g;
      all.push_back(m);
      hprob.push_back(p);
      hj.push_back(j);
    }
    offT += (long long)o.N * D.strideT;
    offW += (long long)o.N * n * o.L;
    offY += (long long)n * o.N * o.L;
    offRow += o.N * n;
  }
  nnodes = g;
  t_elems_ = offT;
  w_elems_ = offW;
  y_elems_ = offY;
  rows_total_ = offRow;
  sorted_ = all;
  std::stable_sort(sorted_.begin(), sorted_.end(), [](const MatDesc& a, const MatDesc& b) { return a.n > b.n; });

  lu_.build(sorted_, o.prec);
  const bool mixed = o.prec == NEP_PREC_C32_IR64;

  hprefix_.clear();
  SolvePlan_build(sp_, hprefix_, sorted_, o.L, o.prec, dinv_off_, dinv_elems_);
  {
    std::vector<int> ca, cr, crr, cm;
    // real-term residual tiles: the big ones when they still give every CU
    // two groups (they halve the operand traffic per product)
    long long big_tiles = 0;
    for (int p = 0; p < nprob; ++p)
      if (probs[p].op->a_cplx == 0)
        big_tiles += (long long)ceil_div(hpd_[p].n, kResidBigTM) * ceil_div(2 * o.N * o.L, kResidBigTQ);
    pt_.resid_big = big_tiles >= 512 ? 1 : 0;
    const int rtm = pt_.resid_big ? kResidBigTM : kResidRealTM, rtq = pt_.resid_big ? kResidBigTQ : kResidRealTQ;
    for (int p = 0; p < nprob; ++p) {
      const long long n = hpd_[p].n;
      const bool cplx = probs[p].op->a_cplx != 0;
      ca.push_back((int)ceil_div_ll(n * n, 256));
      cr.push_back(cplx ? ceil_div((int)n, 64) * ceil_div(2 * o.N * o.L, 64) : 0);
      crr.push_back(cplx ? 0 : ceil_div((int)n, rtm) * ceil_div(2 * o.N * o.L, rtq));
      cm.push_back(ceil_div((int)n * o.L, 256) * ceil_div(2 * o.K, 8));  // (row, column) blocks x moment groups
    }
    build_prefix(hprefix_, pt_.assemble, ca);
    build_prefix(hprefix_, pt_.resid, cr);
    build_prefix(hprefix_, pt_.resid_real, crr);
    build_prefix(hprefix_, pt_.moments, cm);
  }

  const size_t es = elem_size(o.prec);
  total_bytes_ = 0;
  auto A = [&](DevMem& m, size_t b) -> nep_status {
    nep_status s = m.alloc(b);
    total_bytes_ += b;
    return s;
  };
  NEP_TRY(A(dpd_, sizeof(ProbDesc) * nprob));
  NEP_TRY(A(dmd_, sizeof(MatDesc) * sorted_.size()));
  NEP_TRY(A(dprefix_, sizeof(int) * hprefix_.size()));
  NEP_TRY(A(dlu_prefix_, sizeof(int) * std::max<size_t>(1, lu_.prefix.size())));
  NEP_TRY(A(dT_, es * (size_t)t_elems_));
  if (sp_.nblk > 0) {  // right-hand sides of the blocked solve
    NEP_TRY(A(dW_, sizeof(c64) * (size_t)sp_.nblk * sp_.npad * sp_.L));
    sp_.W = dW_.as<c64>();
  } else {
    dW_.release();
    sp_.W = nullptr;
  }
  NEP_TRY(A(drows_, sizeof(int) * (size_t)rows_total_));
  NEP_TRY(A(drows_snap_, sizeof(int) * (size_t)rows_total_));
  if (!ls_.aux) {
    NEP_HIP(hipStreamCreateWithFlags(&ls_.aux, hipStreamNonBlocking));
    NEP_HIP(hipStreamCreateWithFlags(&ls_.side, hipStreamNonBlocking));
    for (hipEvent_t* e : {&ls_.ev_fork, &ls_.ev_join, &ls_.ev_side[0], &ls_.ev_side[1], &ls_.ev_side_done})
      NEP_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
  }
  NEP_TRY(A(dinfo_, sizeof(int) * (size_t)nnodes));
  NEP_TRY(A(ddinv_, es * (size_t)dinv_elems_));
  NEP_TRY(A(dlinv_, 2 * es * (size_t)sorted_.size() * kLuMaxJB * kLuMaxJB));
  NEP_TRY(A(darrive_, sizeof(int) * std::max<size_t>(1, sorted_.size())));
  NEP_HIP(hipMemsetAsync(darrive_.p, 0, sizeof(int) * std::max<size_t>(1, sorted_.size()), st));
  NEP_TRY(A(ddinv_off_, sizeof(long long) * dinv_off_.size()));
  NEP_TRY(A(dY_, sizeof(c128) * (size_t)y_elems_));
  NEP_TRY(A(dR_, sizeof(c128) * (size_t)y_elems_));
  const size_t G = nnodes;
  const size_t node_bytes = G * (3 + kMaxTerms + kMaxMoments) * sizeof(c128) + G * sizeof(double) + 3 * G * sizeof(int);
  NEP_TRY(A(dnode_, node_bytes));
  const size_t ir_bytes = 2 * G * kNormStride * 8 + (size_t)nprob * 64 * 8 + G * 8 + 3 * G * 4 + 8 * 4;
  NEP_TRY(A(dir_, ir_bytes));
  NEP_TRY(A(dstat_, status_bytes((int)G)));
  if (hstat_ && hstat_bytes_ < status_bytes((int)G)) {
    (void)hipHostFree(hstat_);
    hstat_ = nullptr;
  }
  if (!hstat_) {
    hstat_bytes_ = status_bytes((int)G);
    NEP_HIP(hipHostMalloc((void**)&hstat_, hstat_bytes_, hipHostMallocDefault));
  }
  if (!ev_counter_) NEP_HIP(hipEventCreateWithFlags(&ev_counter_, hipEventDisableTiming));
  if (!ev_lu_[0]) {
    NEP_HIP(hipEventCreate(&ev_lu_[0]));
    NEP_HIP(hipEventCreate(&ev_lu_[1]));
  }

  {
    char* q = dnode_.as<char>();
    na_.z = reinterpret_cast<c128*>(q); q += G * sizeof(c128);
    na_.zeta = reinterpret_cast<c128*>(q); q += G * sizeof(c128);
    na_.w = reinterpret_cast<c128*>(q); q += G * sizeof(c128);
    na_.fz = reinterpret_cast<c128*>(q); q += G * kMaxTerms * sizeof(c128);
    na_.mcoef = reinterpret_cast<c128*>(q); q += G * kMaxMoments * sizeof(c128);
    na_.fnorm = reinterpret_cast<double*>(q); q += G * sizeof(double);
    na_.prob = reinterpret_cast<int*>(q); q += G * sizeof(int);
    na_.jnode = reinterpret_cast<int*>(q); q += G * sizeof(int);
    na_.bad = reinterpret_cast<int*>(q);
    char* r = dir_.as<char>();
    ir_.rnorm = reinterpret_cast<unsigned long long*>(r); r += G * kNormStride * 8;
    ir_.ynorm = reinterpret_cast<unsigned long long*>(r); r += G * kNormStride * 8;
    ir_.vnorm = reinterpret_cast<double*>(r); r += (size_t)nprob * 64 * 8;
    ir_.rho = reinterpret_cast<double*>(r); r += G * 8;
    ir_.conv = reinterpret_cast<int*>(r); r += G * 4;
    ir_.stalled = reinterpret_cast<int*>(r); r += G * 4;
    ir_.sweeps = reinterpret_cast<int*>(r); r += G * 4;
    ir_.counters = reinterpret_cast<int*>(r);
  }
  if (!hcounter_) {
    hcounter_ = static_cast<int*>(pinned_take());
    NEP_CHECK(hcounter_ != nullptr, NEP_ERR_OOM, "no pinned read-back slot left");
  }

  // pageable sources: each copy has taken its bytes when the call returns
  NEP_HIP(hipMemcpyAsync(dmd_.p, sorted_.data(), sizeof(MatDesc) * sorted_.size(), hipMemcpyHostToDevice, st));
  NEP_HIP(hipMemcpyAsync(dprefix_.p, hprefix_.data(), sizeof(int) * hprefix_.size(), hipMemcpyHostToDevice, st));
  if (!lu_.prefix.empty())
    NEP_HIP(hipMemcpyAsync(dlu_prefix_.p, lu_.prefix.data(), sizeof(int) * lu_.prefix.size(),
                           hipMemcpyHostToDevice, st));
  NEP_HIP(hipMemcpyAsync(ddinv_off_.p, dinv_off_.data(), sizeof(long long) * dinv_off_.size(),
                         hipMemcpyHostToDevice, st));
  NEP_HIP(hipMemcpyAsync(na_.prob, hprob.data(), sizeof(int) * G, hipMemcpyHostToDevice, st));
  na_prob_host_ = hprob;
  NEP_HIP(hipMemcpyAsync(na_.jnode, hj.data(), sizeof(int) * G, hipMemcpyHostToDevice, st));
  dT64_.release();
  ddinv64_.release();
  dlinv64_.release();
  return upload_problems(probs, st);
}

template <typename P>
nep_status MomentsPlan::enqueue_t(hipStream_t st, bool eager, bool refactor) {
  const ProbDesc* pd = dpd_.as<ProbDesc>();
  const MatDesc* md = dmd_.as<MatDesc>();
  const int* pre = dprefix_.as<int>();
  cx<P>* T = dT_.as<cx<P>>();
  c128* Y = dY_.as<c128>();
  c128* R = dR_.as<c128>();
  int* rows = drows_.as<int>();
  int* info = dinfo_.as<int>();
  NEP_HIP(ir_reset(ir_, nnodes, st));
  NEP_HIP(launch_coef(pd, na_, nnodes, ir_, st));
  if (refactor) NEP_HIP(launch_assemble<P>(pd, pre, pt_.assemble, na_, T, nullptr, st));
  // the probe norms are first read by the refinement test; queued behind the
  // assembly they start without a launch gap
  NEP_HIP(launch_vnorm(pd, nprob, opt.L, ir_, st));
  cx<P>* Dinv = ddinv_.as<cx<P>>();
  const long long* doff = ddinv_off_.as<long long>();
  if (refactor) {  // otherwise the factors (and info) of the previous pass are reused
    if (eager) NEP_HIP(hipEventRecord(ev_lu_[0], st));
    NEP_HIP(lu_run<P>(lu_, md, dlu_prefix_.as<int>(), T, rows, drows_snap_.as<int>(), rows_total_, info, nullptr,
                      dlinv_.as<cx<P>>(), Dinv, doff, darrive_.as<int>(), st, ls_));
    if (eager) {
      NEP_HIP(hipEventRecord(ev_lu_[1], st));
      lu_timed_ = true;
    }
  }
  // nodes of problems sitting out the pass are marked converged by k_coef
  NEP_HIP(solve_run<P>(sp_, pd, md, na_, T, rows, Dinv, doff, nullptr, Y, false, ir_.conv, ir_, st));
  sweeps_run_ = 0;
  if (opt.max_refine > 0) {
    // The correction solve of each sweep is queued before the host reads the
    // sweep's convergence count, so the device never waits for that round
    // trip; nodes already converged skip the solve, which makes it a no-op
    // when the count turns out to be zero.
    for (int s = 0; s <= opt.max_refine; ++s) {
      NEP_HIP(resid_run(pd, pre, pt_.resid, pt_.resid_real, pt_.resid_big, na_, Y, R, ir_, nnodes, st,
                        lr_jobs_.data(), (int)lr_jobs_.size()));
      NEP_HIP(ir_control(pd, na_, ir_, nnodes, s, opt.tol, st));
      sweeps_run_ = s;
      if (eager) {
        NEP_HIP(hipMemcpyAsync(hcounter_, ir_.counters, sizeof(int), hipMemcpyDeviceToHost, st));
        NEP_HIP(hipEventRecord(ev_counter_, st));
      }
      if (s < opt.max_refine)
        NEP_HIP(solve_run<P>(sp_, pd, md, na_, T, rows, Dinv, doff, R, Y, true, ir_.conv, ir_, st));
      if (eager) {
        NEP_HIP(hipEventSynchronize(ev_counter_));
        if (hcounter_[0] == 0) break;
      }
    }
    if (eager && hcounter_[0] > 0 && opt.fallback && sizeof(P) == 4) NEP_TRY(run_fallback<double>(st));
  }
  NEP_HIP(launch_moments(pd, pre, pt_.moments, na_, Y, st));
  return NEP_OK;
}

// FP64 re-solve of the nodes whose refinement did not converge: assemble in
// complex FP64, factor on the FP64 matrix cores, solve, overwrite Y, then
// refine with the FP64 factor (fixed-precision refinement: a backward-stable
// LU's solution can sit above a tolerance near unit roundoff on large,
// ill-conditioned nodes; one or two sweeps bring it to that level).
template <typename P>
nep_status MomentsPlan::run_fallback(hipStream_t st) {
  static_assert(sizeof(P) == 8, "fallback runs in FP64");
  if (!dT64_.p) {
    auto alloc64 = [&]() -> nep_status {
      nep_status s = dT64_.alloc(sizeof(c128) * (size_t)t_elems_);
      if (s == NEP_OK) s = ddinv64_.alloc(sizeof(c128) * (size_t)dinv_elems_);
      if (s == NEP_OK) s = dlinv64_.alloc(2 * sizeof(c128) * (size_t)sorted_.size() * kLuMaxJB * kLuMaxJB);
      if (s != NEP_OK) {
        dT64_.release();
        ddinv64_.release();
        dlinv64_.release();
      }
      return s;
    };
    nep_status s = alloc64();
    if (s == NEP_ERR_OOM) {  // an arena without room: take the rare re-solve from the device heap
      ArenaScope heap(nullptr);
      s = alloc64();
    }
    NEP_TRY(s);
  }
  const ProbDesc* pd = dpd_.as<ProbDesc>();
  const MatDesc* md = dmd_.as<MatDesc>();
  const int* pre = dprefix_.as<int>();
  c128* T = dT64_.as<c128>();
  const int* skip = ir_.conv;
  {
    std::vector<int> conv(nnodes);
    NEP_HIP(hipMemcpyAsync(conv.data(), ir_.conv, sizeof(int) * nnodes, hipMemcpyDeviceToHost, st));
    NEP_HIP(hipStreamSynchronize(st));
    fallback_count_.assign(nprob, 0);
    for (int p = 0; p < nprob; ++p)
      for (int j = 0; j < opt.N; ++j) fallback_count_[p] += conv[hpd_[p].node0 + j] ? 0 : 1;
  }
  NEP_HIP(launch_assemble<double>(pd, pre, pt_.assemble, na_, T, skip, st));
  c128* Dinv = ddinv64_.as<c128>();
  const long long* doff = ddinv_off_.as<long long>();
  {
    // factor only the unconverged matrices: a compact plan over them (in the
    // size order of the full plan), whose diagonal-block inverses land where
    // the full plan's solve looks for them
    std::vector<int> conv(nnodes);
    NEP_HIP(hipMemcpyAsync(conv.data(), ir_.conv, sizeof(int) * nnodes, hipMemcpyDeviceToHost, st));
    NEP_HIP(hipStreamSynchronize(st));
    std::vector<MatDesc> sub;
    std::vector<long long> sub_off;
    for (size_t b = 0; b < sorted_.size(); ++b)
      if (!conv[sorted_[b].node]) {
        sub.push_back(sorted_[b]);
        sub_off.push_back(dinv_off_[b]);
      }
    if (!sub.empty()) {
      LuPlan lsub;
      lsub.build(sub, NEP_PREC_FP64);
      DevMem dmd, dpre, doff_sub;
      NEP_TRY(dmd.alloc(sizeof(MatDesc) * sub.size()));
      NEP_TRY(dpre.alloc(sizeof(int) * std::max<size_t>(1, lsub.prefix.size())));
      NEP_TRY(doff_sub.alloc(sizeof(long long) * sub_off.size()));
      NEP_HIP(hipMemcpyAsync(dmd.p, sub.data(), sizeof(MatDesc) * sub.size(), hipMemcpyHostToDevice, st));
      if (!lsub.prefix.empty())
        NEP_HIP(hipMemcpyAsync(dpre.p, lsub.prefix.data(), sizeof(int) * lsub.prefix.size(), hipMemcpyHostToDevice,
                               st));
      NEP_HIP(hipMemcpyAsync(doff_sub.p, sub_off.data(), sizeof(long long) * sub_off.size(), hipMemcpyHostToDevice,
                             st));
      NEP_HIP(lu_run<double>(lsub, dmd.as<MatDesc>(), dpre.as<int>(), T, drows_.as<int>(), drows_snap_.as<int>(),
                             rows_total_, dinfo_.as<int>(), nullptr, dlinv64_.as<c128>(), Dinv,
                             doff_sub.as<long long>(), darrive_.as<int>(), st, ls_));
      NEP_HIP(hipStreamSynchronize(st));  // the compact tables leave scope
    }
  }
  NEP_HIP(solve_run<double>(sp_, pd, md, na_, T, drows_.as<int>(), Dinv, doff, nullptr, dY_.as<c128>(), false,
                            skip, ir_, st));
  for (int s = 0;; ++s) {
    NEP_HIP(resid_run(pd, pre, pt_.resid, pt_.resid_real, pt_.resid_big, na_, dY_.as<c128>(), dR_.as<c128>(), ir_, nnodes, st,
                      lr_jobs_.data(), (int)lr_jobs_.size()));
    NEP_HIP(ir_control(pd, na_, ir_, nnodes, opt.max_refine + 1 + s, opt.tol, st));
    if (s == kFallbackSweeps) break;
    NEP_HIP(hipMemcpyAsync(hcounter_, ir_.counters, sizeof(int), hipMemcpyDeviceToHost, st));
    NEP_HIP(hipStreamSynchronize(st));
    if (hcounter_[0] == 0) break;
    NEP_HIP(solve_run<double>(sp_, pd, md, na_, T, drows_.as<int>(), Dinv, doff, dR_.as<c128>(), dY_.as<c128>(),
                              true, ir_.conv, ir_, st));
  }
  fallback_pending_ = true;
  return NEP_OK;
}

template <typename P>
nep_status MomentsPlan::factor_t(hipStream_t st) {
  const ProbDesc* pd = dpd_.as<ProbDesc>();
  NEP_HIP(ir_reset(ir_, nnodes, st));
  NEP_HIP(launch_coef(pd, na_, nnodes, ir_, st));
  NEP_HIP(launch_assemble<P>(pd, dprefix_.as<int>(), pt_.assemble, na_, dT_.as<cx<P>>(), nullptr, st));
  NEP_HIP(lu_run<P>(lu_, dmd_.as<MatDesc>(), dlu_prefix_.as<int>(), dT_.as<cx<P>>(), drows_.as<int>(),
                    drows_snap_.as<int>(), rows_total_, dinfo_.as<int>(), nullptr, dlinv_.as<cx<P>>(),
                    ddinv_.as<cx<P>>(), ddinv_off_.as<long long>(), darrive_.as<int>(), st, ls_));
  return NEP_OK;
}

template <typename P>
nep_status MomentsPlan::solve_rhs_t(hipStream_t st) {
  NEP_HIP(hipMemsetAsync(dY_.p, 0, sizeof(c128) * (size_t)y_elems_, st));
  NEP_HIP(solve_run<P>(sp_, dpd_.as<ProbDesc>(), dmd_.as<MatDesc>(), na_, dT_.as<cx<P>>(), drows_.as<int>(),
                       ddinv_.as<cx<P>>(), ddinv_off_.as<long long>(), dR_.as<c128>(), dY_.as<c128>(), true,
                       nullptr, ir_, st));
  return NEP_OK;
}

nep_status MomentsPlan::factor(hipStream_t st) {
  if (opt.prec == NEP_PREC_FP64) return factor_t<double>(st);
  return factor_t<float>(st);
}

nep_status MomentsPlan::solve_rhs(hipStream_t st) {
  if (opt.prec == NEP_PREC_FP64) return solve_rhs_t<double>(st);
  return solve_rhs_t<float>(st);
}

nep_status MomentsPlan::enqueue(hipStream_t st, bool eager, bool refactor) {
  fallback_pending_ = false;
  if (opt.prec == NEP_PREC_FP64) return enqueue_t<double>(st, eager, refactor);
  return enqueue_t<float>(st, eager, refactor);
}

template <typename P>
hipError_t logdet_run(const MatDesc* md, int nmat, const cx<P>* T, const int* rows, double* out, hipStream_t st);

nep_status MomentsPlan::logdet(hipStream_t st, std::vector<double>& logabs, std::vector<double>& arg) {
  DevMem out;
  NEP_TRY(out.alloc(sizeof(double) * 2 * (size_t)nnodes));
  if (opt.prec == NEP_PREC_FP64)
    NEP_HIP(logdet_run<double>(dmd_.as<MatDesc>(), (int)sorted_.size(), dT_.as<c128>(), drows_.as<int>(),
                               out.as<double>(), st));
  else
    NEP_HIP(logdet_run<float>(dmd_.as<MatDesc>(), (int)sorted_.size(), dT_.as<c64>(), drows_.as<int>(),
                              out.as<double>(), st));
  std::vector<double> h(2 * (size_t)nnodes);
  NEP_HIP(hipMemcpyAsync(h.data(), out.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
  NEP_HIP(hipStreamSynchronize(st));
  logabs.assign(h.begin(), h.begin() + nnodes);
  arg.assign(h.begin() + nnodes, h.end());
  return NEP_OK;
}

nep_status MomentsPlan::finish(hipStream_t st, RunResult& out, bool allow_fallback) {
  const int G = nnodes;
  std::vector<int> info(G), conv(G), sweeps(G), bad(G), counters(4);
  std::vector<double> rho(G);
  std::vector<double> pmin(G);
  auto read_back = [&]() -> nep_status {  // one gathered block, one copy
    NEP_HIP(gather_status(ir_, dinfo_.as<int>(), na_.bad, G, dstat_.p, st));
    if (opt.prec == NEP_PREC_FP64)
      NEP_HIP(min_pivot<double>(dmd_.as<MatDesc>(), (int)sorted_.size(), dT_.as<c128>(), drows_.as<int>(), G,
                                dstat_.p, st));
    else
      NEP_HIP(min_pivot<float>(dmd_.as<MatDesc>(), (int)sorted_.size(), dT_.as<c64>(), drows_.as<int>(), G,
                               dstat_.p, st));
    NEP_HIP(hipMemcpyAsync(hstat_, dstat_.p, status_bytes(G), hipMemcpyDeviceToHost, st));
    NEP_HIP(hipStreamSynchronize(st));
    const int* iv = reinterpret_cast<const int*>(hstat_ + 2 * (size_t)G * sizeof(double));
    std::memcpy(rho.data(), hstat_, sizeof(double) * G);
    std::memcpy(pmin.data(), hstat_ + (size_t)G * sizeof(double), sizeof(double) * G);
    std::memcpy(info.data(), iv, sizeof(int) * G);
    std::memcpy(conv.data(), iv + G, sizeof(int) * G);
    std::memcpy(sweeps.data(), iv + 2 * G, sizeof(int) * G);
    std::memcpy(bad.data(), iv + 3 * G, sizeof(int) * G);
    std::memcpy(counters.data(), iv + 4 * G, sizeof(int) * 4);
    return NEP_OK;
  };
  NEP_TRY(read_back());
  const bool refined = opt.max_refine > 0;
  const bool mixed = opt.prec == NEP_PREC_C32_IR64;
  std::vector<int> excluded;  // unconverged nodes of problems that fail anyway
  if (allow_fallback && refined && mixed && opt.fallback && !fallback_pending_) {
    // A fixed-sweep run left nodes unconverged: re-solve them in FP64 and
    // recompute the moments (the eager path does this inside enqueue).  The
    // decision is per problem: a problem with a node on a pole or cut, or an
    // exact zero pivot, fails whatever its other nodes do, so its nodes are
    // left out, and the other problems of the batch are re-solved exactly
    // as they would be alone.
    std::vector<char> fails(nprob, 0);
    for (int g = 0; g < G; ++g) {
      const int p = na_prob_host_[g];
      if (bad[g] || info[g] < hpd_[p].n) fails[p] = 1;
    }
    bool any = false;
    for (int g = 0; g < G; ++g) {
      if (conv[g]) continue;
      if (fails[na_prob_host_[g]]) excluded.push_back(g);
      else any = true;
    }
    // (if the FP64 workspace cannot be allocated the nodes stay unconverged
    // and their problems report NEP_ERR_REFINE)
    if (any) {
      if (!excluded.empty()) {  // the re-solve skips converged nodes: mark the left-out ones so
        std::vector<int> skip(conv);
        for (int g : excluded) skip[g] = 1;
        NEP_HIP(hipMemcpyAsync(ir_.conv, skip.data(), sizeof(int) * G, hipMemcpyHostToDevice, st));
        NEP_HIP(hipStreamSynchronize(st));
      }
      if (run_fallback<double>(st) == NEP_OK) {
        NEP_HIP(launch_moments(dpd_.as<ProbDesc>(), dprefix_.as<int>(), pt_.moments, na_, dY_.as<c128>(), st));
        NEP_TRY(read_back());
        for (int g : excluded) conv[g] = 0;  // still unconverged, for the stats
      }
    }
  }
  out.stats.assign(nprob, nep_ciss_stats{});
  out.pstatus.assign(nprob, NEP_OK);
  out.status = NEP_OK;
  float lu_ms = 0.f;
  if (lu_timed_) {
    if (hipEventElapsedTime(&lu_ms, ev_lu_[0], ev_lu_[1]) != hipSuccess) {
      (void)hipGetLastError();
      lu_ms = 0.f;
    }
    lu_timed_ = false;
  }
  for (int p = 0; p < nprob; ++p) {
    nep_ciss_stats& s = out.stats[p];
    s.N = opt.N;
    s.singular_node = -1;
    s.bad_node = -1;
    s.max_rel_residual = refined ? 0.0 : -1.0;
    s.ms_lu = lu_ms;
    s.min_abs_pivot = INFINITY;
    if (fallback_pending_) s.n_fallback = fallback_count_[p];
  }
  for (int g = 0; g < G; ++g) {
    const int p = na_prob_host_[g];
    nep_ciss_stats& s = out.stats[p];
    const int j = g - hpd_[p].node0;
    if (!(pmin[g] >= s.min_abs_pivot)) s.min_abs_pivot = pmin[g];  // keeps a NaN
    if (bad[g] && s.bad_node < 0) s.bad_node = j;
    if (info[g] < hpd_[p].n && s.singular_node < 0) s.singular_node = j;
    if (refined) {
      s.refine_sweeps = std::max(s.refine_sweeps, std::min(sweeps[g] - 1, opt.max_refine));
      if (!conv[g]) s.n_unconverged++;
      if (std::isfinite(rho[g])) s.max_rel_residual = std::max(s.max_rel_residual, rho[g]);
    }
  }
  // per-problem status, in order of precedence
  for (int p = 0; p < nprob; ++p) {
    const nep_ciss_stats& s = out.stats[p];
    nep_status ps = NEP_OK;
    if (s.bad_node >= 0) {
      set_error("quadrature node %d of problem %d lies on a pole or branch cut of some f_i", s.bad_node, p);
      ps = NEP_ERR_NOT_HOLOMORPHIC;
    } else if (s.singular_node >= 0) {
      set_error("T(z_j) has an exact zero pivot at node %d of problem %d", s.singular_node, p);
      ps = NEP_ERR_SINGULAR;
    } else if (s.n_unconverged > 0 && refined && mixed) {
      set_error("refinement did not reach the tolerance at %d node(s) of problem %d", s.n_unconverged, p);
      ps = NEP_ERR_REFINE;
    }
    out.pstatus[p] = ps;
  }
  // the call's status: the most severe kind over problems, message of its first
  for (nep_status kind : {NEP_ERR_NOT_HOLOMORPHIC, NEP_ERR_SINGULAR, NEP_ERR_REFINE})
    for (int p = 0; p < nprob; ++p)
      if (out.pstatus[p] == kind) {
        const nep_ciss_stats& s = out.stats[p];
        if (kind == NEP_ERR_NOT_HOLOMORPHIC)
          set_error("quadrature node %d of problem %d lies on a pole or branch cut of some f_i", s.bad_node, p);
        else if (kind == NEP_ERR_SINGULAR)
          set_error("T(z_j) has an exact zero pivot at node %d of problem %d", s.singular_node, p);
        else
          set_error("refinement did not reach the tolerance at %d node(s) of problem %d", s.n_unconverged, p);
        out.status = kind;
        return out.status;
      }
  return NEP_OK;
}

nep_status configure_kernels() {
  static int done = 0;
  if (done) return NEP_OK;
  NEP_HIP(lu_configure());
  NEP_HIP(solve_configure());
  done = 1;
  return NEP_OK;
}

template nep_status MomentsPlan::enqueue_t<float>(hipStream_t, bool, bool);
template nep_status MomentsPlan::enqueue_t<double>(hipStream_t, bool, bool);

}  // namespace nep
