// Continuous-batching server of libmgrit (include/mgrit_serve.h).
//
// Threads: `setup_threads` workers compute coarse operators on the host
// (with a cache); `slots` workers each own a HIP stream and run one admitted
// group at a time on it -- a request and up to max_batch-1 later ones of the
// same shape, solved together with merged relaxation launches -- so the
// kernels of all resident requests overlap on the device.  Admission (under
// one mutex) happens whenever a request becomes ready or a slot frees its
// memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/mgrit.h"
#include "../../include/mgrit_serve.h"
#include "plan.h"
#include "setup.h"

namespace mgr {

static double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Req {
  long long id = 0;
  mgrit_request r = {};
  std::vector<double> u0;
  std::vector<Taps> psi;
  int levels = 0;
  size_t bytes = 0;
  enum { SETUP, READY, RUNNING, DONE } state = SETUP;
  int bypassed = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  mgrit_result res = {0, 0, 0, 0, 0.0, 0.0, 0.0, 0.0, 0, -1};
  std::vector<double> ufinal;
};

// The coarse-operator cache, keyed by (scheme, Courant number, m).  An
// entry holds the eq. (9) hierarchy computed for some n_x_ref, deep enough
// for every request it served (a hierarchy of L levels is the first L-1
// operators of a deeper one).  A request on n_x points with n_x dividing
// n_x_ref takes the stencils folded onto its periodic line (offsets mod n_x):
// the circulant that the n_x_ref one folds to, fitted on a superset of its
// modes (theta_k on n_x points is theta_{k n_x_ref/n_x} on the longer line).
// Psi decides only how fast MGRIT converges, not its fixed point (Sec. 2.2).
// The Courant number is matched exactly: Psi_l approximates Phi^(m^(l-1)),
// whose characteristic shift of c m^(l-1) points moves by whole grid points
// on deep levels for Courant numbers 1 % apart, which stalls or breaks the
// convergence.
using PsiKey = std::tuple<int, unsigned long long, int>;
struct PsiEntry {
  int nx = 0;
  std::vector<Taps> ops;  // offsets in [0, nx)
};

struct Server {
  std::mutex mu;
  std::condition_variable cv;
  std::map<long long, std::shared_ptr<Req>> reqs;
  typedef std::vector<std::shared_ptr<Req>> Group;  // requests run as one batch
  std::deque<std::shared_ptr<Req>> setup_q;
  std::list<std::shared_ptr<Req>> ready_q;  // by submission order
  std::deque<Group> run_q;
  std::map<PsiKey, std::vector<PsiEntry>> psi_cache;
  long long next_id = 1, submitted = 0, completed = 0, admitted = 0, hits = 0, misses = 0;
  size_t budget = 0, in_use = 0, peak = 0;
  int free_slots = 0, max_bypass = 0, max_batch = 1, device = 0;
  long long batches = 0, batched = 0;  // groups of >= 2 requests, their requests
  bool stopping = false;
  std::vector<std::thread> workers;

  // Requests run as one group: the same line (n_x), scheme, coarsening
  // factor, cycle, relaxation and precision, so that the fine-level passes --
  // most of a solve -- have the same stencil kernel, and n_t within a factor
  // of two (the number of levels may differ by one): a group returns when
  // its last member has converged, so members of very different size would
  // hold the small ones back.  Launches of the same kernel and launch shape
  // merge into one grid (Batch in plan.h); the others of the group go out
  // one after another on its stream.
  static bool same_shape(const Req& a, const Req& b) {
    const int lo = std::min(a.r.nt, b.r.nt), hi = std::max(a.r.nt, b.r.nt);
    return a.r.nx == b.r.nx && a.r.scheme == b.r.scheme && a.r.m == b.r.m &&
           a.r.cycle == b.r.cycle && a.r.relax == b.r.relax &&
           a.r.precision == b.r.precision && hi <= 2 * (long long)lo;
  }

  void admit(Req& q, Group& g, const std::shared_ptr<Req>& sp) {
    in_use += q.bytes;
    if (in_use > peak) peak = in_use;
    q.state = Req::RUNNING;
    q.t_admit = now_ms();
    q.res.admit_seq = admitted++;
    g.push_back(sp);
  }

  // Admit ready requests in submission order while slots and budget allow.
  // A ready request that does not fit may be passed (a later one admitted
  // before it) at most max_bypass times; then admission waits for it.
  // Requests still in setup do not hold others back.  An admitted request
  // takes a slot and brings along up to max_batch-1 later ready requests of
  // the same shape that fit (solved with it as one batch); each of those
  // passes the requests between, which counts against their bypass limit
  // too.  Caller holds `mu`.
  void try_admit() {
    std::vector<Req*> blocked;
    for (auto it = ready_q.begin(); it != ready_q.end() && free_slots > 0;) {
      Req& q = **it;
      if (in_use + q.bytes <= budget) {
        bool stop = false;
        for (Req* bq : blocked) stop |= ++bq->bypassed >= max_bypass;
        Group g;
        admit(q, g, *it);
        it = ready_q.erase(it);
        std::vector<Req*> passed;
        for (auto jt = it; !stop && jt != ready_q.end() && (int)g.size() < max_batch;) {
          Req& x = **jt;
          if (!same_shape(q, x) || in_use + x.bytes > budget) {
            passed.push_back(&x);
            ++jt;
            continue;
          }
          bool full = false;
          for (Req* p : passed) full |= p->bypassed >= max_bypass;
          for (Req* bq : blocked) full |= bq->bypassed >= max_bypass;
          if (full) break;
          for (Req* p : passed) ++p->bypassed;
          for (Req* bq : blocked) ++bq->bypassed;
          const bool at_it = jt == it;
          admit(x, g, *jt);
          jt = ready_q.erase(jt);
          if (at_it) it = jt;
        }
        if (g.size() > 1) {
          ++batches;
          batched += (long long)g.size();
        }
        --free_slots;
        run_q.push_back(std::move(g));
        cv.notify_all();
        if (stop) break;
        continue;
      }
      if (q.bypassed >= max_bypass) break;  // nobody may pass it any more
      blocked.push_back(&q);
      ++it;
    }
  }

  // Psi_2..Psi_L for request q (L = q.levels) on its n_x: folded from a
  // cached hierarchy on a multiple of n_x points, or fitted for the request
  // (and cached) on a miss.
  int coarse_operators(const Req& q, std::vector<Taps>& psi) {
    const mgrit_request& r = q.r;
    PsiKey key{r.scheme, 0ULL, r.m};
    std::memcpy(&std::get<1>(key), &r.cfl, sizeof(double));
    PsiEntry hit;
    {
      std::lock_guard<std::mutex> lk(mu);
      auto f = psi_cache.find(key);
      if (f != psi_cache.end())
        for (const PsiEntry& e : f->second)
          if (e.nx % r.nx == 0 && (int)e.ops.size() >= q.levels - 1 && e.nx > hit.nx) hit = e;
      ++(hit.nx ? hits : misses);
    }
    if (!hit.nx) {
      double mi = 0.0;
      int rc;
      try {
        rc = psi_hierarchy(r.scheme, r.cfl, r.nx, r.m, q.levels, MGRIT_PSI_AUTO, nullptr, 0.0,
                           psi, mi);
      } catch (...) {
        rc = MGRIT_ENOMEM;
      }
      if (rc != MGRIT_OK) return rc;
      std::lock_guard<std::mutex> lk(mu);
      auto& es = psi_cache[key];
      bool have = false;
      for (PsiEntry& e : es)
        if (e.nx == r.nx) {
          if (e.ops.size() < psi.size()) e.ops = psi;
          have = true;
        }
      if (!have) es.push_back({r.nx, psi});
      return MGRIT_OK;
    }
    psi.assign(q.levels - 1, Taps());
    for (int l = 0; l < q.levels - 1; ++l) {
      std::map<int, double> folded;
      for (size_t t = 0; t < hit.ops[l].off.size(); ++t)
        folded[hit.ops[l].off[t] % r.nx] += hit.ops[l].w[t];
      for (auto& a : folded) {
        psi[l].off.push_back(a.first);
        psi[l].w.push_back(a.second);
      }
    }
    return MGRIT_OK;
  }

  void setup_loop() {
    for (;;) {
      std::shared_ptr<Req> q;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stopping || !setup_q.empty(); });
        if (setup_q.empty()) return;
        q = setup_q.front();
        setup_q.pop_front();
      }
      std::vector<Taps> psi;
      int rc = coarse_operators(*q, psi);
      std::lock_guard<std::mutex> lk(mu);
      if (rc != MGRIT_OK) {
        q->res.status = rc;
        q->state = Req::DONE;
        q->t_done = now_ms();
        ++completed;
      } else {
        q->psi = std::move(psi);
        q->state = Req::READY;
        auto pos = ready_q.begin();
        while (pos != ready_q.end() && (*pos)->id < q->id) ++pos;
        ready_q.insert(pos, q);
        try_admit();
      }
      cv.notify_all();
    }
  }

  void slot_loop() {
    (void)hipSetDevice(device);
    hipStream_t stream = nullptr;
    // non-blocking: no implicit ordering against the null stream, so one
    // slot's setup never waits for the kernels of the others
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
    for (;;) {
      Group g;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stopping || !run_q.empty(); });
        if (run_q.empty()) break;
        g = std::move(run_q.front());
        run_q.pop_front();
      }
      run(g, stream);
      std::lock_guard<std::mutex> lk(mu);
      const double t = now_ms();
      for (auto& q : g) {
        in_use -= q->bytes;
        q->state = Req::DONE;
        q->t_done = t;
        ++completed;
      }
      ++free_slots;
      try_admit();
      cv.notify_all();
    }
    if (stream) (void)hipStreamDestroy(stream);
  }

  // One group on the slot's stream: a plan per request, then all solves
  // together (mgrit_solve_batch), the final time levels back to the host,
  // and the plans released.
  void run(Group& g, hipStream_t stream) {
    struct Run {
      Req* q;
      mgrit_plan_t plan = nullptr;
      double* dev = nullptr;  // u0 and the final time level
    };
    std::vector<Run> rs;
    for (auto& sp : g) {
      Req& q = *sp;
      const mgrit_request& r = q.r;
      std::vector<mgrit_taps> taps(q.psi.size());
      for (size_t l = 0; l < q.psi.size(); ++l) {
        taps[l].nnz = (int)q.psi[l].off.size();
        taps[l].offset = q.psi[l].off.data();
        taps[l].weight = q.psi[l].w.data();
      }
      Run x{&q};
      int rc = mgrit_plan_create(&x.plan, r.nx, r.nt, r.alpha, r.cfl, r.scheme, r.m, q.levels,
                                 taps.data(), r.cycle, r.relax, r.precision, stream);
      const size_t row = (size_t)r.nx * sizeof(double);
      if (rc == MGRIT_OK && mgr::dev_alloc((void**)&x.dev, 2 * row) != MGRIT_OK)
        rc = MGRIT_ENOMEM;
      if (rc == MGRIT_OK &&
          hipMemcpyAsync(x.dev, q.u0.data(), row, hipMemcpyHostToDevice, stream) != hipSuccess)
        rc = MGRIT_EHIP;
      q.res.status = rc;
      if (rc != MGRIT_OK) {
        mgr::dev_free(x.dev);
        mgrit_destroy(x.plan);
        continue;
      }
      size_t pb = 0;
      mgrit_plan_bytes(x.plan, &pb);
      q.res.hbm_bytes = pb + 2 * row;
      mgrit_plan_set_seed(x.plan, r.seed);
      rs.push_back(x);
    }
    const int n = (int)rs.size();
    if (n > 0) {
      std::vector<mgrit_plan_t> plans(n);
      std::vector<const double*> u0(n);
      std::vector<double*> out(n);
      std::vector<double> tol(n);
      std::vector<int> maxit(n), kind(n, MGRIT_OUT_FINAL), iters(n, 0), status(n, MGRIT_OK);
      for (int i = 0; i < n; ++i) {
        plans[i] = rs[i].plan;
        u0[i] = rs[i].dev;
        out[i] = rs[i].dev + rs[i].q->r.nx;
        tol[i] = rs[i].q->r.tol;
        maxit[i] = rs[i].q->r.maxit;
      }
      const int rc = mgrit_solve_batch(n, plans.data(), u0.data(), nullptr, tol.data(),
                                       maxit.data(), out.data(), kind.data(), nullptr,
                                       iters.data(), status.data());
      for (int i = 0; i < n; ++i) {
        Req& q = *rs[i].q;
        mgrit_stats st;
        mgrit_get_stats(rs[i].plan, &st);
        q.res.status = rc == MGRIT_EINVAL ? rc : status[i];
        q.res.iterations = iters[i];
        q.res.final_residual = st.final_residual;
        q.ufinal.resize(q.r.nx);
        if (hipMemcpyAsync(q.ufinal.data(), out[i], (size_t)q.r.nx * sizeof(double),
                           hipMemcpyDeviceToHost, stream) != hipSuccess)
          q.res.status = MGRIT_EHIP;
      }
      if (hipStreamSynchronize(stream) != hipSuccess)
        for (auto& x : rs) x.q->res.status = MGRIT_EHIP;
    }
    for (auto& x : rs) {
      mgr::dev_free(x.dev);
      mgrit_destroy(x.plan);
    }
  }
};

static int auto_levels(int nt, int m) {
  int L = 2;
  long long span = (long long)m * m;  // m^(L) for the candidate L+1 levels
  while (nt % span == 0 && nt / span >= 8) {
    ++L;
    span *= m;
  }
  return L;
}

}  // namespace mgr

using namespace mgr;

extern "C" {

int mgrit_server_create(mgrit_server_t* out, size_t budget, int slots, int setup_threads,
                        int max_bypass, int max_batch) {
  if (!out || slots < 1 || setup_threads < 1 || max_bypass < 0 || budget == 0 ||
      max_batch < 1 || max_batch > kMaxBatch)
    return MGRIT_EINVAL;
  *out = nullptr;
  Server* S = new (std::nothrow) Server();
  if (!S) return MGRIT_ENOMEM;
  S->budget = budget;
  S->free_slots = slots;
  S->max_bypass = max_bypass;
  S->max_batch = max_batch;
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return MGRIT_ENODEV;
  }
  try {
    for (int i = 0; i < setup_threads; ++i) S->workers.emplace_back([S] { S->setup_loop(); });
    for (int i = 0; i < slots; ++i) S->workers.emplace_back([S] { S->slot_loop(); });
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stopping = true;
    }
    S->cv.notify_all();
    for (auto& t : S->workers)
      if (t.joinable()) t.join();
    delete S;
    return MGRIT_ENOMEM;
  }
  *out = reinterpret_cast<mgrit_server_t>(S);
  return MGRIT_OK;
}

int mgrit_server_submit(mgrit_server_t server, const mgrit_request* r, long long* id) {
  if (!server || !r || !id || !r->u0 || r->nx < 2 || r->nt < 1 || r->m < 2 ||
      r->maxit < 0 || !(r->tol >= 0.0) || !(r->cfl > 0.0) || !(r->alpha > 0.0))
    return MGRIT_EINVAL;
  Server* S = reinterpret_cast<Server*>(server);
  const int levels = r->levels > 0 ? r->levels : auto_levels(r->nt, r->m);
  long long span = 1;
  for (int l = 1; l < levels; ++l) span *= r->m;
  if (r->nt % span) return MGRIT_EINVAL;
  size_t bytes = 0;
  if (mgrit_plan_estimate_bytes(r->nx, r->nt, r->m, levels, r->precision, &bytes) != MGRIT_OK)
    return MGRIT_EINVAL;
  bytes += 2 * (size_t)r->nx * sizeof(double);
  if (bytes > S->budget) return MGRIT_EBUSY;
  auto q = std::make_shared<Req>();
  q->r = *r;
  q->u0.assign(r->u0, r->u0 + r->nx);
  q->r.u0 = nullptr;
  q->levels = levels;
  q->bytes = bytes;
  q->t_submit = now_ms();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    q->id = S->next_id++;
    q->res.id = q->id;
    q->res.levels = levels;
    S->reqs[q->id] = q;
    S->setup_q.push_back(q);
    ++S->submitted;
  }
  S->cv.notify_all();
  *id = q->id;
  return MGRIT_OK;
}

int mgrit_server_wait(mgrit_server_t server, long long id, int timeout_ms, mgrit_result* res,
                      double* u_final) {
  if (!server) return MGRIT_EINVAL;
  Server* S = reinterpret_cast<Server*>(server);
  std::unique_lock<std::mutex> lk(S->mu);
  auto f = S->reqs.find(id);
  if (f == S->reqs.end()) return MGRIT_EINVAL;
  std::shared_ptr<Req> q = f->second;
  auto done = [&] { return q->state == Req::DONE; };
  if (timeout_ms < 0) S->cv.wait(lk, done);
  else if (!S->cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), done))
    return MGRIT_EBUSY;
  q->res.queue_ms = q->t_admit > 0 ? q->t_admit - q->t_submit : q->t_done - q->t_submit;
  q->res.run_ms = q->t_admit > 0 ? q->t_done - q->t_admit : 0.0;
  q->res.latency_ms = q->t_done - q->t_submit;
  if (res) *res = q->res;
  if (u_final && q->ufinal.size() == (size_t)q->r.nx)
    std::memcpy(u_final, q->ufinal.data(), q->ufinal.size() * sizeof(double));
  S->reqs.erase(f);
  return MGRIT_OK;
}

int mgrit_server_get_stats(mgrit_server_t server, mgrit_server_stats* st) {
  if (!server || !st) return MGRIT_EINVAL;
  Server* S = reinterpret_cast<Server*>(server);
  std::lock_guard<std::mutex> lk(S->mu);
  st->submitted = S->submitted;
  st->completed = S->completed;
  long long active = 0, waiting = 0;
  for (auto& kv : S->reqs) {
    if (kv.second->state == Req::RUNNING) ++active;
    if (kv.second->state == Req::SETUP || kv.second->state == Req::READY) ++waiting;
  }
  st->active = active;
  st->waiting = waiting;
  st->hbm_in_use = S->in_use;
  st->hbm_peak = S->peak;
  st->hbm_budget = S->budget;
  st->psi_cache_hits = S->hits;
  st->psi_cache_misses = S->misses;
  st->batches = S->batches;
  st->batched_requests = S->batched;
  return MGRIT_OK;
}

void mgrit_server_destroy(mgrit_server_t server) {
  if (!server) return;
  Server* S = reinterpret_cast<Server*>(server);
  {
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv.wait(lk, [&] { return S->completed >= S->submitted; });
    S->stopping = true;
  }
  S->cv.notify_all();
  for (auto& t : S->workers)
    if (t.joinable()) t.join();
  // hand the blocks the plans released back to the driver
  mgr::dev_trim();
  delete S;
}

}  // extern "C"
