// Serving of "eigenvalues of this operator inside this contour" queries.
//
// Queries are queued by nep_server_submit and served by one host thread that
// owns nstreams device streams ("slots").  Whenever a slot is free, the
// thread takes the oldest queued query and every other queued query that
// shares its (N, L, K, precision, refinement) options, as far as the HBM
// budget and the in-flight limit allow, and runs their moments as one ragged
// batch (one plan over every (query, node) pair) on that slot's stream.
// New arrivals join the next free slot while earlier batches still run:
// continuous batching.  Each slot has a completion worker thread: it waits
// for the slot's batch, reads the per-query status, runs the extraction of
// each query and copies the results to the caller's host arrays, while the
// dispatch thread keeps feeding the other slots.  Workspaces (plans, probes,
// moments, and each slot's extraction workspace) come from one device arena
// of the budget's size, so recycling them never synchronizes the device.
//
// Factors stay resident: a finished batch's plan (its LU factors of every
// node of every query) is kept, keyed per query by (operator, contour, N, L,
// K, precision, refinement options).  A later query with the key of a
// resident member runs on those factors: probes, solves, refinement and
// moments only, no assembly or factorization (the factors are the same
// bits a new factorization would give).  Several such queries on members of
// one resident plan run as one pass; the plan's other members sit out.
// Resident plans count against the budget and are evicted least recently
// used when a new batch needs the room.  A queued query whose key repeats a
// query already in the batch being formed waits and then runs on the
// resident factors instead of factoring the same matrices twice.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "handle.hpp"

namespace nep {

namespace {

// What makes two queries' factors identical.
struct Key {
  unsigned long long uid = 0;  // operator (Split::uid)
  nep_contour g{};
  int N = 0, L = 0, K = 0, prec = 0, max_refine = 0, fallback = 0;
  double tol = 0.0;
};

bool same_key(const Key& a, const Key& b) {
  return a.uid == b.uid && a.g.kind == b.g.kind && a.g.c[0] == b.g.c[0] && a.g.c[1] == b.g.c[1] &&
         a.g.rho == b.g.rho && (a.g.kind != 1 || a.g.v == b.g.v) && a.N == b.N && a.L == b.L && a.K == b.K &&
         a.prec == b.prec && a.max_refine == b.max_refine && a.fallback == b.fallback && a.tol == b.tol;
}

struct Query {
  long long ticket = 0;
  Key key;
  nep_split h = nullptr;
  nep_contour g{};
  nep_ciss_opts o{};
  nep_extract_opts e{};
  PlanOptions po;
  int n = 0;
  int Lmax = 0;         // probe columns available: L, or a pool for rank augmentation
  std::vector<c128> V;  // host copy of the probes (n x Lmax); freed at dispatch unless Lmax > L
  double* lambda = nullptr;
  double* eta = nullptr;
  int* inside = nullptr;
  void* X = nullptr;
  size_t bytes = 0;   // a query with its own factors (plan, probes, moments, vectors)
  size_t fbytes = 0;  // a query on resident factors (probes, moments, vectors)
  nep_query_info info{};
  bool done = false;
};
using QueryPtr = std::shared_ptr<Query>;

// A finished batch's plan kept with its factors.
struct Resident {
  std::unique_ptr<MomentsPlan> plan;
  std::vector<Key> keys;    // per plan problem
  std::vector<char> valid;  // the member's last query succeeded
  size_t bytes = 0;         // counted against the budget
  double last_use = 0.0;
  bool out = false;         // a slot runs a pass on it
};

struct QueryBuffers {
  DevMem V, S, X;
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  std::unique_ptr<MomentsPlan> own;  // a new plan (factored in this batch)
  Resident* res = nullptr;           // or the resident plan the batch runs on
  MomentsPlan* plan = nullptr;       // the one in use
  std::vector<QueryPtr> q;
  std::vector<int> member;           // on a resident plan: each query's plan problem
  std::vector<std::unique_ptr<QueryBuffers>> buf;
  std::shared_ptr<ExtractWork> xw;  // extraction workspace (arena blocks)
  size_t bytes = 0;
  bool busy = false;     // a batch is on the device or being completed
  bool running = false;  // handed to the completion worker
  std::thread worker;
};

bool same_batch(const Query& a, const Query& b) {
  return a.po.N == b.po.N && a.po.L == b.po.L && a.po.K == b.po.K && a.po.prec == b.po.prec &&
         a.po.max_refine == b.po.max_refine && a.po.fallback == b.po.fallback && a.po.tol == b.po.tol;
}

}  // namespace

class Server {
 public:
  ~Server();
  nep_status init(const nep_server_opts* o);
  nep_status submit(nep_split h, const nep_contour* g, const nep_ciss_opts* o, const nep_extract_opts* e,
                    const void* V, int Lmax, double* lambda, double* eta, int* inside, void* X, long long* ticket);
  nep_status poll(long long ticket, int* done, nep_query_info* info, bool block);
  double clock() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
  }
  void shutdown();

 private:
  void loop();
  void work(Slot& s);                    // completion worker of a slot
  bool dispatch(Slot& s);                // true if a batch was started
  void complete(Slot& s);                // the slot's batch has finished
  void fail(std::vector<QueryPtr>& qs, nep_status st);
  static size_t query_bytes(const Query& q);
  static size_t query_buffer_bytes(const Query& q);
  // resident_ helpers (mu_ held)
  Resident* find_resident(const Key& k, int* member);
  void evict_lru(size_t need, std::vector<std::unique_ptr<Resident>>& out);
  void keep_resident(Slot& s, const std::vector<nep_status>& status);
  void release_slot_plan(Slot& s, bool drop_resident);
  bool evict_one();  // destroys the least recently used idle resident plan (mu_ not held)

  Arena arena_;
  int device_ = 0;
  size_t budget_ = 0, inflight_bytes_ = 0;
  int max_inflight_ = 1, inflight_ = 0, batch_cap_ = 1;
  std::vector<Slot> slots_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_, cv_slot_;
  std::deque<QueryPtr> queue_;
  std::vector<std::unique_ptr<Resident>> resident_;
  size_t resident_bytes_ = 0;
  std::unordered_map<long long, QueryPtr> tickets_;
  long long next_ticket_ = 1;
  bool stop_ = false, started_ = false;
  bool arena_full_ = false;  // a dispatch found no room; wait for a completion
  std::chrono::steady_clock::time_point t0_ = std::chrono::steady_clock::now();
  std::thread th_;
};

Server::~Server() { shutdown(); }

size_t Server::query_buffer_bytes(const Query& q) {
  const size_t c = sizeof(c128);
  size_t b = (size_t)q.n * q.po.L * c + (size_t)q.n * q.Lmax * c * 2 * q.po.K;  // V (one block) and S
  b += (size_t)q.n * q.e.max_eigs * c;                     // X
  return b + (1u << 16);                                    // alignment
}

size_t Server::query_bytes(const Query& q) {
  return MomentsPlan::estimate_bytes(q.n, q.po.N, q.po.L, q.po.prec) + query_buffer_bytes(q) +
         (1u << 20);  // tables, alignment
}

Resident* Server::find_resident(const Key& k, int* member) {
  for (auto& r : resident_) {
    if (r->out) continue;
    for (size_t m = 0; m < r->keys.size(); ++m)
      if (r->valid[m] && same_key(r->keys[m], k)) {
        *member = (int)m;
        return r.get();
      }
  }
  return nullptr;
}

// Removes least recently used resident plans that no slot runs on until
// need more bytes fit the budget (or none is left); the caller destroys them
// with mu_ released.
void Server::evict_lru(size_t need, std::vector<std::unique_ptr<Resident>>& out) {
  while (inflight_bytes_ + resident_bytes_ + need > budget_) {
    int best = -1;
    for (int i = 0; i < (int)resident_.size(); ++i)
      if (!resident_[i]->out && (best < 0 || resident_[i]->last_use < resident_[best]->last_use)) best = i;
    if (best < 0) return;
    resident_bytes_ -= resident_[best]->bytes;
    out.push_back(std::move(resident_[best]));
    resident_.erase(resident_.begin() + best);
  }
}

nep_status Server::init(const nep_server_opts* o) {
  NEP_CHECK(o != nullptr, NEP_ERR_ARG, "null server options");
  NEP_CHECK(o->hbm_budget > 0, NEP_ERR_ARG, "hbm_budget must be positive");
  NEP_CHECK(o->max_inflight >= 1, NEP_ERR_ARG, "max_inflight must be >= 1");
  NEP_CHECK(o->nstreams >= 1 && o->nstreams <= 16, NEP_ERR_ARG, "nstreams must be in 1..16");
  NEP_TRY(configure_kernels());
  NEP_HIP(hipGetDevice(&device_));
  budget_ = (size_t)o->hbm_budget;
  max_inflight_ = o->max_inflight;
  batch_cap_ = std::max(1, (max_inflight_ + o->nstreams - 1) / o->nstreams);
  NEP_TRY(arena_.init(budget_));
  slots_.resize(o->nstreams);
  for (auto& s : slots_) {
    NEP_HIP(hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking));
    NEP_HIP(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
    s.xw = make_extract_work();
  }
  for (auto& s : slots_) {
    Slot* sp = &s;
    s.worker = std::thread([this, sp] { work(*sp); });
  }
  th_ = std::thread([this] { loop(); });
  started_ = true;
  return NEP_OK;
}

nep_status Server::submit(nep_split h, const nep_contour* g, const nep_ciss_opts* o, const nep_extract_opts* e,
                          const void* V, int Lmax, double* lambda, double* eta, int* inside, void* X,
                          long long* ticket) {
  NEP_CHECK(h != nullptr && ticket != nullptr, NEP_ERR_ARG, "null handle or ticket");
  NEP_CHECK(V != nullptr && lambda != nullptr && eta != nullptr && inside != nullptr, NEP_ERR_ARG,
            "null probe or result array");
  NEP_CHECK(e != nullptr && e->max_eigs >= 1, NEP_ERR_ARG, "extract options need max_eigs >= 1");
  NEP_TRY(check_contour(g));
  auto q = std::make_shared<Query>();
  NEP_TRY(check_opts(o, q->po));
  q->h = h;
  q->g = *g;
  q->o = *o;
  q->e = *e;
  q->n = h->impl.op.n;
  q->Lmax = Lmax > 0 ? Lmax : q->po.L;
  NEP_CHECK(q->Lmax >= q->po.L && q->Lmax % q->po.L == 0 && q->Lmax <= 256 && q->Lmax <= q->n, NEP_ERR_ARG,
            "probe pool of %d columns: a multiple of L=%d, at most 256 and at most n", q->Lmax, q->po.L);
  q->key.uid = h->impl.uid;
  q->key.g = *g;
  q->key.N = q->po.N;
  q->key.L = q->po.L;
  q->key.K = q->po.K;
  q->key.prec = q->po.prec;
  q->key.max_refine = q->po.max_refine;
  q->key.fallback = q->po.fallback;
  q->key.tol = q->po.tol;
  q->fbytes = query_buffer_bytes(*q);
  q->lambda = lambda;
  q->eta = eta;
  q->inside = inside;
  q->X = X;
  q->bytes = query_bytes(*q);
  NEP_CHECK(q->bytes <= budget_, NEP_ERR_BUSY, "query needs %zu bytes, more than the server's HBM budget %zu",
            q->bytes, budget_);
  const size_t cnt = (size_t)q->n * q->Lmax;
  q->V.assign(static_cast<const c128*>(V), static_cast<const c128*>(V) + cnt);
  {
    std::lock_guard<std::mutex> lk(mu_);
    NEP_CHECK(!stop_, NEP_ERR_ARG, "server is shutting down");
    q->ticket = next_ticket_++;
    q->info.status = NEP_OK;
    q->info.L_used = q->po.L;
    q->info.t_submit = clock();
    tickets_[q->ticket] = q;
    queue_.push_back(q);
    *ticket = q->ticket;
  }
  cv_work_.notify_one();
  return NEP_OK;
}

nep_status Server::poll(long long ticket, int* done, nep_query_info* info, bool block) {
  std::unique_lock<std::mutex> lk(mu_);
  auto it = tickets_.find(ticket);
  NEP_CHECK(it != tickets_.end(), NEP_ERR_ARG, "unknown or already collected ticket %lld", ticket);
  QueryPtr q = it->second;
  if (block) cv_done_.wait(lk, [&] { return q->done; });
  if (done) *done = q->done ? 1 : 0;
  if (q->done) {
    if (info) *info = q->info;
    tickets_.erase(it);  // collected
  }
  return NEP_OK;
}

void Server::shutdown() {
  if (started_) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_work_.notify_all();
    th_.join();  // returns once the queue is drained and no slot is busy
    cv_slot_.notify_all();
    for (auto& s : slots_)
      if (s.worker.joinable()) s.worker.join();
    started_ = false;
  }
  {
    std::lock_guard<std::mutex> lk(mu_);
    resident_.clear();  // every slot is idle: no resident plan is in use
    resident_bytes_ = 0;
  }
  for (auto& s : slots_) {
    {
      ArenaScope scope(&arena_);  // the workspace's blocks go back to the arena
      s.xw.reset();
    }
    if (s.ev) (void)hipEventDestroy(s.ev);
    if (s.st) (void)hipStreamDestroy(s.st);
    s.ev = nullptr;
    s.st = nullptr;
  }
}

void Server::fail(std::vector<QueryPtr>& qs, nep_status st) {
  std::lock_guard<std::mutex> lk(mu_);
  for (auto& q : qs) {
    q->info.status = st;
    q->info.t_done = clock();
    q->done = true;
    inflight_--;
    inflight_bytes_ -= q->bytes;
  }
  cv_done_.notify_all();
}

bool Server::dispatch(Slot& s) {
  std::vector<QueryPtr> batch;
  std::vector<int> member;  // on resident factors: the plan problem of each query
  Resident* res = nullptr;
  size_t bytes = 0;
  std::vector<std::unique_ptr<Resident>> evicted;  // destroyed with mu_ released
  bool started = false, return_now = false;
  {
    std::lock_guard<std::mutex> lk(mu_);
    if (queue_.empty() || arena_full_) return false;
    // the oldest query that has resident factors, with every other queued
    // query on a member of the same resident plan (each member once per
    // pass), runs on them; such passes are short, so they go first
    QueryPtr head;
    for (auto& q : queue_) {
      int m0 = -1;
      if ((res = find_resident(q->key, &m0)) != nullptr) {
        head = q;
        break;
      }
    }
    if (res != nullptr) {
      res->out = true;
      evict_lru(head->fbytes, evicted);
      std::vector<char> taken(res->keys.size(), 0);
      for (auto it = queue_.begin(); it != queue_.end() && (int)batch.size() < batch_cap_;) {
        const Query& q = **it;
        int m = -1;
        for (size_t k = 0; k < res->keys.size() && m < 0; ++k)
          if (res->valid[k] && !taken[k] && same_key(res->keys[k], q.key)) m = (int)k;
        const bool fits = inflight_ + (int)batch.size() < max_inflight_ &&
                          inflight_bytes_ + resident_bytes_ + bytes + q.fbytes <= budget_;
        if (batch.empty() && m >= 0 && !fits) break;
        if (m < 0 || !fits) {
          ++it;
          continue;
        }
        taken[m] = 1;
        member.push_back(m);
        bytes += q.fbytes;
        batch.push_back(*it);
        it = queue_.erase(it);
      }
      if (batch.empty()) {
        res->out = false;
        if (inflight_ == 0) {  // no room beside this plan even with nothing running: give it up
          for (size_t i = 0; i < resident_.size(); ++i)
            if (resident_[i].get() == res) {
              resident_bytes_ -= res->bytes;
              evicted.push_back(std::move(resident_[i]));
              resident_.erase(resident_.begin() + i);
              break;
            }
          res = nullptr;
          return_now = true;  // retried at once as a new batch
        }
      }
    } else {
      // a new batch: queries sharing the first one's options; a query whose
      // key repeats one already taken, or names a member of a resident plan
      // that a slot is running, waits and then runs on resident factors
      const Query* first = nullptr;
      for (auto it = queue_.begin(); it != queue_.end() && (int)batch.size() < batch_cap_;) {
        const Query& q = **it;
        bool wait = false;
        for (auto& r : resident_)
          for (size_t k = 0; k < r->keys.size() && !wait; ++k) wait = r->valid[k] && same_key(r->keys[k], q.key);
        for (auto& b : batch) wait |= same_key(b->key, q.key);
        if (wait) {
          ++it;
          continue;
        }
        if (first == nullptr) evict_lru(q.bytes, evicted);
        const bool fits = inflight_ + (int)batch.size() < max_inflight_ &&
                          inflight_bytes_ + resident_bytes_ + bytes + q.bytes <= budget_;
        if (first == nullptr && !fits) break;  // the oldest query waits for room: it is never overtaken
        if (!fits || (first != nullptr && !same_batch(q, *first))) {
          ++it;
          continue;
        }
        if (first == nullptr) first = &q;
        bytes += q.bytes;
        batch.push_back(*it);
        it = queue_.erase(it);
      }
    }
    if (batch.empty()) {  // nothing runs before a completion frees room or a plan
      if (!return_now) arena_full_ = true;
    } else {
      inflight_ += (int)batch.size();
      inflight_bytes_ += bytes;
      const double t = clock();
      for (auto& q : batch) {
        q->info.t_start = t;
        q->info.reused = res != nullptr ? 1 : 0;
      }
      started = true;
    }
  }
  evicted.clear();  // their blocks go back to the arena before this batch allocates
  if (!started) return return_now;

  // workspaces and a new plan come from the arena
  ArenaScope scope(&arena_);
  s.buf.clear();
  s.res = res;  // the slot holds the resident plan (checked out) from here on
  std::vector<PlanProblem> probs;
  nep_status st = NEP_OK;
  for (auto& q : batch) {
    auto b = std::make_unique<QueryBuffers>();
    const size_t c = sizeof(c128), nl = (size_t)q->n * q->po.L;
    st = b->V.alloc(nl * c);
    if (st == NEP_OK) st = b->S.alloc((size_t)q->n * q->Lmax * 2 * q->po.K * c);
    if (st == NEP_OK) st = b->X.alloc((size_t)q->n * q->e.max_eigs * c);
    if (st != NEP_OK) break;
    if (hipMemcpyAsync(b->V.p, q->V.data(), nl * c, hipMemcpyHostToDevice, s.st) != hipSuccess) {
      (void)hipGetLastError();
      st = NEP_ERR_DEVICE;
      break;
    }
    probs.push_back(PlanProblem{&q->h->impl.op, q->g, b->V.as<c128>(), b->S.as<c128>(), nullptr,
                                (long long)q->n * q->Lmax});
    s.buf.push_back(std::move(b));
  }
  bool enqueued = false;
  if (st == NEP_OK && res != nullptr) {
    s.plan = res->plan.get();
    std::vector<const c128*> Vs;
    std::vector<c128*> Ss;
    std::vector<long long> strides;
    for (size_t k = 0; k < s.buf.size(); ++k) {
      Vs.push_back(s.buf[k]->V.as<c128>());
      Ss.push_back(s.buf[k]->S.as<c128>());
      strides.push_back((long long)batch[k]->n * batch[k]->Lmax);
    }
    st = s.plan->rebind_members(member, Vs, Ss, s.st, &strides);
    if (st == NEP_OK) {
      enqueued = true;
      st = s.plan->enqueue(s.st, false, false);
    }
  } else if (st == NEP_OK) {
    s.own = std::make_unique<MomentsPlan>();
    s.plan = s.own.get();
    st = s.plan->build(probs, batch.front()->po, s.st);
    if (st == NEP_OK) {
      enqueued = true;
      st = s.plan->enqueue(s.st, false);
    }
  }
  if (st == NEP_OK && hipEventRecord(s.ev, s.st) != hipSuccess) st = NEP_ERR_DEVICE;
  if (st == NEP_ERR_OOM && !enqueued) {
    // the arena is fragmented or the estimate was short: requeue in order,
    // with every idle resident plan evicted
    (void)hipStreamSynchronize(s.st);
    release_slot_plan(s, false);
    s.buf.clear();
    std::unique_lock<std::mutex> lk(mu_);
    for (auto it = batch.rbegin(); it != batch.rend(); ++it) queue_.push_front(*it);
    inflight_ -= (int)batch.size();
    inflight_bytes_ -= bytes;
    evict_lru(budget_, evicted);
    bool others_busy = false;
    for (auto& o : slots_) others_busy |= o.busy;
    const bool freed = !evicted.empty();
    if (others_busy && !freed) arena_full_ = true;
    lk.unlock();
    evicted.clear();
    if (others_busy || freed) return freed;
    lk.lock();  // nothing else holds the arena: this batch fails below
    for (size_t k = 0; k < batch.size(); ++k) queue_.pop_front();
    inflight_ += (int)batch.size();
    inflight_bytes_ += bytes;
  }
  if (st != NEP_OK) {
    (void)hipStreamSynchronize(s.st);
    release_slot_plan(s, enqueued);
    s.buf.clear();
    fail(batch, st);
    return true;
  }
  for (auto& q : batch)  // the device holds the probes now; a pool keeps its further blocks
    if (q->Lmax == q->po.L) std::vector<c128>().swap(q->V);
  s.q = std::move(batch);
  s.member = std::move(member);
  s.bytes = bytes;
  {
    std::lock_guard<std::mutex> lk(mu_);
    s.busy = true;
    s.running = true;
  }
  cv_slot_.notify_all();
  return true;
}

bool Server::evict_one() {
  std::unique_ptr<Resident> gone;
  {
    std::lock_guard<std::mutex> lk(mu_);
    int best = -1;
    for (int i = 0; i < (int)resident_.size(); ++i)
      if (!resident_[i]->out && (best < 0 || resident_[i]->last_use < resident_[best]->last_use)) best = i;
    if (best < 0) return false;
    resident_bytes_ -= resident_[best]->bytes;
    gone = std::move(resident_[best]);
    resident_.erase(resident_.begin() + best);
  }
  return true;  // its blocks go back to the arena here
}

// The slot's plan after its batch: a resident plan goes back to the cache
// (or, with drop, out of it: its state is unknown after a failed pass), a
// new one is destroyed.
void Server::release_slot_plan(Slot& s, bool drop) {
  std::unique_ptr<Resident> gone;
  if (s.res != nullptr) {
    std::lock_guard<std::mutex> lk(mu_);
    for (size_t i = 0; i < resident_.size(); ++i)
      if (resident_[i].get() == s.res) {
        if (drop) {
          resident_bytes_ -= s.res->bytes;
          gone = std::move(resident_[i]);
          resident_.erase(resident_.begin() + i);
        } else {
          s.res->out = false;
        }
        break;
      }
  }
  s.res = nullptr;
  s.own.reset();
  s.plan = nullptr;
}

// After a completed batch: a new plan becomes resident (if any of its
// queries succeeded), a resident one returns to the cache with its members'
// validity updated.
void Server::keep_resident(Slot& s, const std::vector<nep_status>& status) {
  std::lock_guard<std::mutex> lk(mu_);
  const double t = clock();
  if (s.res != nullptr) {
    for (size_t k = 0; k < s.member.size(); ++k) s.res->valid[s.member[k]] = status[k] == NEP_OK;
    s.res->out = false;
    s.res->last_use = t;
    s.res = nullptr;
    s.plan = nullptr;
    return;
  }
  bool any = false;
  for (nep_status x : status) any |= x == NEP_OK;
  if (!any || !s.own) return;  // destroyed by the caller
  auto r = std::make_unique<Resident>();
  for (size_t k = 0; k < s.q.size(); ++k) {
    r->keys.push_back(s.q[k]->key);
    r->valid.push_back(status[k] == NEP_OK);
    r->bytes += s.q[k]->bytes - s.q[k]->fbytes;
  }
  s.own->release_fallback();
  r->plan = std::move(s.own);
  r->last_use = t;
  resident_bytes_ += r->bytes;
  resident_.push_back(std::move(r));
  s.plan = nullptr;
}

void Server::complete(Slot& s) {
  ArenaScope scope(&arena_);  // a fallback re-solve allocates from the arena
  RunResult rr;
  (void)s.plan->finish(s.st, rr, true);
  std::vector<nep_status> status(s.q.size());
  for (size_t k = 0; k < s.q.size(); ++k) {
    Query& q = *s.q[k];
    const size_t pk = s.res != nullptr ? (size_t)s.member[k] : k;  // the query's plan problem
    nep_status st = pk < rr.pstatus.size() ? rr.pstatus[pk] : NEP_ERR_DEVICE;
    int m = 0, nin = 0;
    if (st == NEP_OK) {
      nep_ciss_opts o = q.o;
      o.stream = s.st;
      // the slot's own workspace, from the arena: no device allocation or
      // free here, and no state of the handle is touched, so slots complete
      // queries of the same operator concurrently
      const long long sstride = (long long)q.n * q.Lmax;
      int Lcur = q.po.L;
      auto run_extract = [&]() {
        nep_status r = extract_strided(q.h->impl, &q.g, &o, Lcur, s.buf[k]->S.p, sstride, &q.e, &m, q.lambda,
                                       s.buf[k]->X.p, q.eta, q.inside, nullptr, s.xw.get());
        // the extraction workspace grows from the arena: without room, idle
        // resident plans give theirs up, least recently used first
        while (r == NEP_ERR_OOM && evict_one()) {
          (void)hipGetLastError();
          r = extract_strided(q.h->impl, &q.g, &o, Lcur, s.buf[k]->S.p, sstride, &q.e, &m, q.lambda,
                              s.buf[k]->X.p, q.eta, q.inside, nullptr, s.xw.get());
        }
        return r;
      };
      st = run_extract();
      // Rank saturation (m = K * L) with probe columns left in the pool: the
      // next block of probes is solved on the same factors (no assembly or
      // LU), its moments land beside the others in S, and the extraction
      // runs again on all probes so far, as nep_eigs does on a handle.
      while (st == NEP_ERR_RANK && m == q.po.K * Lcur && Lcur < q.Lmax) {
        const size_t blk = (size_t)q.n * q.po.L;
        const size_t off = (size_t)(Lcur / q.po.L) * blk;
        c128* Sb = s.buf[k]->S.as<c128>() + off;
        const std::vector<long long> stv{sstride};
        if (hipMemcpyAsync(s.buf[k]->V.p, q.V.data() + off, sizeof(c128) * blk, hipMemcpyHostToDevice, s.st) !=
            hipSuccess) {
          (void)hipGetLastError();
          st = NEP_ERR_DEVICE;
          break;
        }
        st = s.plan->rebind_members({(int)pk}, {s.buf[k]->V.as<c128>()}, {Sb}, s.st, &stv);
        if (st == NEP_OK) st = s.plan->enqueue(s.st, false, false);
        if (st == NEP_OK) {
          // the pass's verdict for this problem (the others sat it out)
          RunResult ra;
          const nep_status fs = s.plan->finish(s.st, ra, true);
          st = pk < ra.pstatus.size() ? ra.pstatus[pk] : (fs != NEP_OK ? fs : NEP_ERR_DEVICE);
        }
        if (st != NEP_OK) break;
        Lcur += q.po.L;
        st = run_extract();
      }
      q.info.L_used = Lcur;
      if (st == NEP_OK && q.X != nullptr && m > 0) {
        if (hipMemcpyAsync(q.X, s.buf[k]->X.p, sizeof(c128) * (size_t)q.n * m, hipMemcpyDeviceToHost, s.st) !=
                hipSuccess ||
            hipStreamSynchronize(s.st) != hipSuccess) {
          (void)hipGetLastError();
          st = NEP_ERR_DEVICE;
        }
      }
      if (st == NEP_OK)
        for (int i = 0; i < m; ++i) nin += q.inside[i] ? 1 : 0;
    }
    // the factors' own verdict decides residency (an extraction failure,
    // such as a saturated rank, does not make them invalid)
    status[k] = pk < rr.pstatus.size() ? rr.pstatus[pk] : NEP_ERR_DEVICE;
    q.info.status = st;
    q.info.m = m;
    q.info.n_inside = nin;
  }
  keep_resident(s, status);
  s.own.reset();
  s.buf.clear();
  s.member.clear();
  {
    std::lock_guard<std::mutex> lk(mu_);
    const double t = clock();
    for (auto& q : s.q) {
      q->info.t_done = t;
      q->done = true;
    }
    inflight_ -= (int)s.q.size();
    inflight_bytes_ -= s.bytes;
    arena_full_ = false;
  }
  cv_done_.notify_all();
  s.q.clear();
  s.bytes = 0;
}

// Completion worker of a slot: waits (on this thread only) for the slot's
// batch, completes it, and hands the slot back to the dispatch thread.
void Server::work(Slot& s) {
  (void)hipSetDevice(device_);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_slot_.wait(lk, [&] { return s.running || (stop_ && !s.busy); });
      if (!s.running) return;
    }
    const hipError_t e = hipEventSynchronize(s.ev);
    if (e == hipSuccess) {
      complete(s);
    } else {
      (void)hipGetLastError();
      std::vector<QueryPtr> qs = std::move(s.q);
      {
        ArenaScope scope(&arena_);
        release_slot_plan(s, true);
        s.buf.clear();
        s.member.clear();
      }
      s.bytes = 0;
      fail(qs, NEP_ERR_DEVICE);
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      s.running = false;
      s.busy = false;
    }
    cv_work_.notify_all();
  }
}

void Server::loop() {
  (void)hipSetDevice(device_);
  for (;;) {
    bool progress = false;
    for (auto& s : slots_) {
      bool free_slot;
      {
        std::lock_guard<std::mutex> lk(mu_);
        free_slot = !s.busy;
      }
      if (free_slot && dispatch(s)) progress = true;
    }
    if (progress) continue;
    std::unique_lock<std::mutex> lk(mu_);
    bool busy = false;
    for (auto& s : slots_) busy |= s.busy;
    if (stop_ && queue_.empty() && !busy) break;
    // wake on a submission or a completion (a slot freed, room back)
    cv_work_.wait(lk, [&] {
      bool free_now = false, busy_now = false;
      for (auto& s : slots_) {
        free_now |= !s.busy;
        busy_now |= s.busy;
      }
      return (free_now && !queue_.empty() && !arena_full_) || (stop_ && queue_.empty() && !busy_now) ||
             (!busy_now && arena_full_);
    });
    bool busy_now = false;
    for (auto& s : slots_) busy_now |= s.busy;
    if (!busy_now && arena_full_) arena_full_ = false;  // nothing left to wait for
  }
}

}  // namespace nep

struct nep_server_s {
  nep::Server impl;
};

using namespace nep;

extern "C" {

nep_status nep_server_create(const nep_server_opts* o, nep_server* out) {
  NEP_CHECK(out != nullptr, NEP_ERR_ARG, "null output");
  *out = nullptr;
  auto s = std::make_unique<nep_server_s>();
  NEP_TRY(s->impl.init(o));
  *out = s.release();
  return NEP_OK;
}

nep_status nep_server_submit(nep_server s, nep_split h, const nep_contour* g, const nep_ciss_opts* o,
                             const nep_extract_opts* e, const void* V, double* lambda, double* eta, int* inside,
                             void* X, long long* ticket) {
  NEP_CHECK(s != nullptr, NEP_ERR_ARG, "null server");
  return s->impl.submit(h, g, o, e, V, 0, lambda, eta, inside, X, ticket);
}

nep_status nep_server_submit_pool(nep_server s, nep_split h, const nep_contour* g, const nep_ciss_opts* o,
                                  const nep_extract_opts* e, const void* V, int Lmax, double* lambda, double* eta,
                                  int* inside, void* X, long long* ticket) {
  NEP_CHECK(s != nullptr, NEP_ERR_ARG, "null server");
  NEP_CHECK(Lmax >= 1, NEP_ERR_ARG, "Lmax must be >= 1");
  return s->impl.submit(h, g, o, e, V, Lmax, lambda, eta, inside, X, ticket);
}

nep_status nep_server_poll(nep_server s, long long ticket, int* done, nep_query_info* info) {
  NEP_CHECK(s != nullptr && done != nullptr, NEP_ERR_ARG, "null server or output");
  return s->impl.poll(ticket, done, info, false);
}

nep_status nep_server_wait(nep_server s, long long ticket, nep_query_info* info) {
  NEP_CHECK(s != nullptr, NEP_ERR_ARG, "null server");
  int done = 0;
  return s->impl.poll(ticket, &done, info, true);
}

double nep_server_clock(nep_server s) { return s ? s->impl.clock() : 0.0; }

nep_status nep_server_destroy(nep_server* s) {
  NEP_CHECK(s != nullptr, NEP_ERR_ARG, "null server pointer");
  if (*s) {
    (*s)->impl.shutdown();
    delete *s;
  }
  *s = nullptr;
  return NEP_OK;
}

}  // extern "C"
