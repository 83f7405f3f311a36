// Request server: continuous batching of operator applications and filter
// passes over resident meshes.
//
// Requests name a resident mesh (its tables, coefficients and projectors stay
// on the device between requests) and a caller-owned block.  The scheduler
// works in ticks on one stream:
//   retire   requests whose completion event has fired leave the batch and
//            give back their budget;
//   admit    queued requests join while there is a free slot, their mesh is
//            idle and the device bytes the meshes would hold after setting up
//            the request stay within the HBM budget (idle meshes' request
//            workspaces are released first when that makes room);
//   step     every active request advances by one filter step (an H X
//            request completes in its first step): the local operators of
//            all active requests of one launch class run as ONE persistent
//            batched launch per colour phase, then each request's nonlocal
//            part and bookkeeping follow.
// At most two ticks are in flight ahead of the host, so a request that
// arrives while others run joins at the next step boundary.  Each request's
// arithmetic is the same whether it runs alone or batched with others (the
// batched kernel runs the identical per-item code), so results are
// independent of the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <mutex>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "fe_internal.h"

namespace {

using fehx::FilterPlan;
using fehx::set_error;
using fehx::LocalLaunch;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
  int64_t id = 0;
  fe_request r{};
  int state = 0;              // 0 queued, 1 active, 2 done, 3 failed
  FilterPlan P;
  bool stepped = false;       // H X request: its launch has been enqueued
  hipEvent_t done = nullptr;
  double t_submit = 0, t_admit = 0, t_done = 0;
  fe_status err = FE_OK;
};

size_t elem_bytes(int prec) { return prec == FE_F64 ? 8 : (prec == FE_F32 ? 4 : 2); }
// element bytes of a filter request's recurrence blocks (BF16 steps keep FP32 state)
size_t filter_elem_bytes(int prec) { return prec == FE_F64 ? 8 : 4; }

// request workspace slots: the filter blocks (see the mesh's workspace list)
constexpr int REQ_SLOTS[] = {0, 1, 2, 3, 4, 8, 9};

// the workspace bytes a request needs on its mesh, per slot, and its
// projector reduction block
void request_needs(const fe_request &q, int64_t need[fehx::Mesh::NWS], int64_t &nl_need) {
  fehx::Mesh *m = q.mesh;
  const int C = m->cplx ? 2 : 1;
  const int64_t lanes = q.nvec * C, n = m->m * lanes;
  for (int i = 0; i < fehx::Mesh::NWS; ++i) need[i] = 0;
  if (q.kind == FE_REQ_FILTER) {
    const int64_t eb = (int64_t)filter_elem_bytes(q.prec);
    need[1] = need[2] = n * eb;
    if (q.prec != FE_F64) {   // FP64 Y inside the R_X + H D^-1 R_Y block
      need[2] = fehx::filter_shared_bytes(n, eb);
    } else {
      need[0] = n * 8;
      need[8] = n * eb;
    }
    need[3] = q.prec != FE_F64 ? n * eb : 0;
    need[4] = (int64_t)(q.degree + 1) * q.nvec * 8;
    if (m->mass_kind == FE_MASS_CONSISTENT) need[9] = n * 8;
  }
  nl_need = m->ns > 0 ? fehx::nl_workspace_bytes(m, (int)lanes) : 0;
}

// bytes a request needs on its mesh beyond what the mesh holds
int64_t extra_bytes(const fe_request &q) {
  fehx::Mesh *m = q.mesh;
  int64_t need[fehx::Mesh::NWS], nl_need;
  request_needs(q, need, nl_need);
  int64_t extra = 0;
  for (int i = 0; i < fehx::Mesh::NWS; ++i)
    if (need[i] > m->ws_bytes[i]) extra += need[i] - m->ws_bytes[i];
  if (nl_need > m->nl_W_lanes) extra += nl_need - m->nl_W_lanes;
  return extra;
}

// Idle request workspaces, kept by size for the next admissions: a request
// takes the smallest idle buffer that holds a slot (at most four times the
// slot's size) and allocates only when none does, so a stream of requests of
// recurring shapes stops allocating after its first requests.  The pool's
// bytes count against the server's budget; under pressure the buffers the
// next admission does not use are freed, largest first.
struct Pool {
  std::multimap<int64_t, void *> idle;
  int64_t bytes = 0;
  int64_t allocs = 0, frees = 0;

  static bool fits(int64_t have, int64_t need) { return have >= need && have <= 4 * need; }
  void give(void *p, int64_t size) {
    if (!p) return;
    idle.emplace(size, p);
    bytes += size;
  }
  // the smallest idle buffer for 'need' bytes, removed from the pool
  bool take(int64_t need, void *&p, int64_t &size) {
    auto it = idle.lower_bound(need);
    if (it == idle.end() || !fits(it->first, need)) return false;
    size = it->first;
    p = it->second;
    bytes -= size;
    idle.erase(it);
    return true;
  }
  // bytes an admission would allocate given the idle buffers, and the
  // buffers it would take
  int64_t plan(const std::vector<int64_t> &needs, std::vector<void *> *used) const {
    std::multimap<int64_t, void *> sim = idle;
    int64_t fresh = 0;
    for (int64_t need : needs) {
      auto it = sim.lower_bound(need);
      if (it != sim.end() && fits(it->first, need)) {
        if (used) used->push_back(it->second);
        sim.erase(it);
      } else {
        fresh += need;
      }
    }
    return fresh;
  }
  void clear() {
    for (auto &kv : idle) { hipFree(kv.second); ++frees; }
    idle.clear();
    bytes = 0;
  }
};

// the slots of a request that its mesh does not hold yet, as byte counts
std::vector<int64_t> missing(const fe_request &q) {
  fehx::Mesh *m = q.mesh;
  int64_t need[fehx::Mesh::NWS], nl_need;
  request_needs(q, need, nl_need);
  std::vector<int64_t> out;
  for (int i : REQ_SLOTS)
    if (need[i] > m->ws_bytes[i]) out.push_back(need[i]);
  if (nl_need > m->nl_W_lanes) out.push_back(nl_need);
  return out;
}

// an idle mesh's request workspaces go back to the pool
void release_request_workspace(fehx::Mesh *m, Pool &pool) {
  for (int i : REQ_SLOTS)
    if (m->ws[i]) {
      pool.give(m->ws[i], m->ws_bytes[i]);
      m->footprint -= m->ws_bytes[i];
      m->ws[i] = nullptr;
      m->ws_bytes[i] = 0;
    }
  if (m->nl_W) {
    pool.give(m->nl_W, m->nl_W_lanes);
    m->footprint -= m->nl_W_lanes;
    m->nl_W = nullptr;
    m->nl_W_lanes = 0;
  }
}

// give the mesh every slot the request needs, from the pool where it can
fe_status provision(const fe_request &q, Pool &pool) {
  fehx::Mesh *m = q.mesh;
  if (m->graphs > 0) return FE_OK;   // a live graph holds the mesh's buffers: the operator calls decide
  int64_t need[fehx::Mesh::NWS], nl_need;
  request_needs(q, need, nl_need);
  auto fill = [&](void *&slot, int64_t &slot_bytes, int64_t want) -> fe_status {
    if (want <= slot_bytes) return FE_OK;
    if (slot) {
      pool.give(slot, slot_bytes);
      m->footprint -= slot_bytes;
      slot = nullptr;
      slot_bytes = 0;
    }
    void *p = nullptr;
    int64_t size = 0;
    if (!pool.take(want, p, size)) {
      if (hipMalloc(&p, (size_t)want) != hipSuccess) return set_error(FE_ENOMEM, "request workspace allocation failed");
      ++pool.allocs;
      size = want;
    }
    slot = p;
    slot_bytes = size;
    m->footprint += size;
    return FE_OK;
  };
  for (int i : REQ_SLOTS) {
    const fe_status st = fill(m->ws[i], m->ws_bytes[i], need[i]);
    if (st) return st;
  }
  return fill(m->nl_W, m->nl_W_lanes, nl_need);
}

}  // namespace

using fehx::set_error;

struct fe_server_s {
  int device = 0;
  int64_t budget = 0;
  int max_active = 1;
  hipStream_t s = nullptr;
  std::deque<Req *> queue;
  std::vector<Req *> active;
  std::unordered_map<int64_t, Req *> all;
  std::unordered_set<fehx::Mesh *> meshes, busy;
  std::deque<hipEvent_t> ticks;
  std::vector<hipEvent_t> spare;
  int64_t next_id = 1;
  int64_t nticks = 0;
  int64_t work_cap = 0;   // admission stops while the active requests hold this many DoF x lanes (0: no cap)
  Pool pool;
  std::mutex mu;

  int64_t held() const {
    int64_t b = pool.bytes;
    for (fehx::Mesh *m : meshes) b += m->footprint;
    return b;
  }

  hipEvent_t event() {
    if (!spare.empty()) { hipEvent_t e = spare.back(); spare.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }

  void finish(Req *q, int state, fe_status err) {
    q->state = state;
    q->err = err;
    q->t_done = now_s();
    busy.erase(q->r.mesh);
    if (q->done) { spare.push_back(q->done); q->done = nullptr; }
    // the mesh's request workspaces serve the next admissions (unless a
    // captured graph holds them)
    if (q->r.mesh->graphs == 0) release_request_workspace(q->r.mesh, pool);
  }

  fe_status retire() {
    for (size_t i = 0; i < active.size();) {
      Req *q = active[i];
      if (q->done) {
        const hipError_t e = hipEventQuery(q->done);
        if (e == hipErrorNotReady) { ++i; continue; }
        if (e != hipSuccess) return set_error(FE_EDEVICE, "device error while a request ran");
        finish(q, 2, FE_OK);
        active.erase(active.begin() + (long)i);
        continue;
      }
      ++i;
    }
    while (!ticks.empty() && hipEventQuery(ticks.front()) == hipSuccess) {
      spare.push_back(ticks.front());
      ticks.pop_front();
    }
    return FE_OK;
  }

  // room for an admission: idle meshes' workspaces go to the pool, then the
  // idle buffers the admission will not take are freed, largest first
  bool make_room(const fe_request &r) {
    fehx::Mesh *keep = r.mesh;
    if (held() + pool.plan(missing(r), nullptr) <= budget) return true;
    for (fehx::Mesh *m : meshes) {
      if (m == keep || busy.count(m) || m->graphs > 0) continue;   // a live graph holds its workspaces
      bool has = m->nl_W != nullptr;
      for (int i : REQ_SLOTS) has = has || m->ws[i] != nullptr;
      if (!has) continue;
      release_request_workspace(m, pool);
    }
    std::vector<void *> used;
    const int64_t fresh = pool.plan(missing(r), &used);
    for (auto it = pool.idle.end(); it != pool.idle.begin() && held() + fresh > budget;) {
      --it;
      if (std::find(used.begin(), used.end(), it->second) != used.end()) continue;
      hipFree(it->second);
      ++pool.frees;
      pool.bytes -= it->first;
      it = pool.idle.erase(it);
    }
    return held() + fresh <= budget;
  }

  // DoF x real lanes one step of a request applies H to
  static int64_t work(const fe_request &r) { return r.mesh->m * r.nvec * (r.mesh->cplx ? 2 : 1); }

  fe_status admit() {
    int64_t active_work = 0;
    for (Req *q : active) active_work += work(q->r);
    for (auto it = queue.begin(); it != queue.end() && (int)active.size() < max_active;) {
      Req *q = *it;
      fehx::Mesh *m = q->r.mesh;
      // past the work cap the queue waits in arrival order (a request that
      // fills the device runs alone; small ones share the steps)
      if (work_cap > 0 && !active.empty() && active_work + work(q->r) > work_cap) break;
      if (busy.count(m)) { ++it; continue; }
      meshes.insert(m);
      if (!make_room(q->r)) { ++it; continue; }
      const fe_request &r = q->r;
      const int C = m->cplx ? 2 : 1;
      fe_status st = provision(r, pool);
      if (st) {
      } else if (r.kind == FE_REQ_FILTER) {
        st = fehx::filter_setup(q->P, m, (double *)r.X, r.ldx * C, r.lam, r.nvec, r.degree, r.lam_min, r.lam_T,
                                r.lam_max, r.prec);
        if (st == FE_OK) st = fehx::filter_prologue(q->P, s);
      } else {
        st = fehx::ensure_nl_workspace(m, (int)(r.nvec * C));
      }
      it = queue.erase(it);
      q->t_admit = now_s();
      if (st) { finish(q, 3, st); continue; }
      q->state = 1;
      busy.insert(m);
      active.push_back(q);
      active_work += work(r);
    }
    return FE_OK;
  }

  // one step of every active request, local parts batched per launch class
  fe_status step() {
    struct Item { Req *q; LocalLaunch L; };
    std::vector<Item> items;
    for (Req *q : active) {
      if (q->done) continue;   // finished enqueueing, waiting for its event
      const fe_request &r = q->r;
      if (r.kind == FE_REQ_FILTER) {
        if (q->P.k <= q->P.degree) items.push_back({q, fehx::filter_step_local(q->P)});
      } else if (!q->stepped) {
        const int C = r.mesh->cplx ? 2 : 1;
        LocalLaunch L;
        L.X = r.X; L.Y = r.Y; L.ldx = r.ldx * C; L.ldy = r.ldy * C; L.nlanes = (int)(r.nvec * C);
        L.prec = r.prec; L.vt = r.mesh->vt_pref[r.prec][0];
        items.push_back({q, L});
      }
    }
    // projector reductions of the step's requests, before the batched local
    // launches (FP32 / BF16: on the meshes' second streams, beside them)
    for (Item &it : items) {
      Req *q = it.q;
      const fe_request &r = q->r;
      fe_status st;
      if (r.kind == FE_REQ_FILTER) {
        st = fehx::filter_step_reduce(q->P, s);
      } else {
        const int C = r.mesh->cplx ? 2 : 1;
        st = fehx::nonlocal_reduce(r.mesh, r.X, r.ldx * C, (int)(r.nvec * C), r.prec, nullptr, s);
      }
      if (st) return st;
    }
    std::vector<int> done(items.size(), 0);
    for (size_t i = 0; i < items.size(); ++i) {
      if (done[i]) continue;
      std::vector<fehx::Mesh *> ms;
      std::vector<LocalLaunch> Ls;
      const fehx::Mesh *a = items[i].q->r.mesh;
      const LocalLaunch &La = items[i].L;
      for (size_t j = i; j < items.size(); ++j) {
        const fehx::Mesh *b = items[j].q->r.mesh;
        const LocalLaunch &Lb = items[j].L;
        if (done[j] || b->np != a->np || b->nq != a->nq || b->cplx != a->cplx || Lb.prec != La.prec ||
            Lb.vt != La.vt || Lb.store32 != La.store32)
          continue;
        ms.push_back(items[j].q->r.mesh);
        Ls.push_back(Lb);
        done[j] = 1;
      }
      fehx::LocalBatch B;
      B.ms = ms.data();
      B.Ls = Ls.data();
      B.n = (int)ms.size();
      B.persistent = true;
      fe_status st = fehx::launch_local_batch(B, s);
      if (st) return st;
    }
    for (Item &it : items) {
      Req *q = it.q;
      const fe_request &r = q->r;
      fe_status st;
      if (r.kind == FE_REQ_FILTER) {
        st = fehx::filter_step_rest(q->P, s);
      } else {
        const int C = r.mesh->cplx ? 2 : 1;
        st = fehx::nonlocal_update(r.mesh, r.Y, r.ldy * C, (int)(r.nvec * C), r.prec, 1.0, s);
        q->stepped = true;
      }
      if (st) return st;
    }
    // requests with nothing left to enqueue: final combine and completion event
    for (Req *q : active) {
      if (q->done) continue;
      const bool filter = q->r.kind == FE_REQ_FILTER;
      if (filter ? q->P.k <= q->P.degree : !q->stepped) continue;
      if (filter) {
        fe_status st = fehx::filter_final(q->P, s);
        if (st) return st;
      }
      q->done = event();
      if (!q->done) return set_error(FE_EDEVICE, "hipEventCreate failed");
      FE_HIP_TRY(hipEventRecord(q->done, s));
    }
    hipEvent_t t = event();
    if (!t) return set_error(FE_EDEVICE, "hipEventCreate failed");
    FE_HIP_TRY(hipEventRecord(t, s));
    ticks.push_back(t);
    ++nticks;
    return FE_OK;
  }

  fe_status progress(bool block) {
    fe_status st;
    if ((st = retire())) return st;
    if ((st = admit())) return st;
    if (active.empty() && !queue.empty()) {
      // nothing runs and the head request still does not fit next to the
      // resident meshes: it never will
      Req *q = queue.front();
      queue.pop_front();
      finish(q, 3, set_error(FE_ENOMEM, "request does not fit the HBM budget next to the resident meshes"));
      return FE_OK;
    }
    if (ticks.size() >= 2) {
      if (!block) return FE_OK;
      FE_HIP_TRY(hipEventSynchronize(ticks.front()));
      if ((st = retire())) return st;
      if ((st = admit())) return st;
    }
    bool work = false;
    for (Req *q : active) work = work || !q->done;
    if (work) return step();
    if (block && !active.empty()) {
      for (Req *q : active)
        if (q->done) { FE_HIP_TRY(hipEventSynchronize(q->done)); break; }
      return retire();
    }
    return FE_OK;
  }
};

extern "C" {

fe_status fe_server_create(int32_t device, int64_t hbm_budget, int32_t max_active, fe_server_t *out) {
  if (!out) return set_error(FE_EINVAL, "NULL output handle");
  *out = nullptr;
  if (hbm_budget <= 0 || max_active <= 0) return set_error(FE_EINVAL, "budget and max_active must be positive");
  if (hipSetDevice(device) != hipSuccess) return set_error(FE_EDEVICE, "hipSetDevice failed");
  fe_server_s *S = new fe_server_s();
  S->device = device;
  S->budget = hbm_budget;
  S->max_active = max_active;
  if (hipStreamCreate(&S->s) != hipSuccess) { delete S; return set_error(FE_EDEVICE, "hipStreamCreate failed"); }
  *out = S;
  return FE_OK;
}

fe_status fe_server_submit(fe_server_t S, const fe_request *r, int64_t *id) {
  if (!S || !r || !id) return set_error(FE_EINVAL, "NULL argument");
  fehx::Mesh *m = r->mesh;
  if (!m || !r->X) return set_error(FE_EINVAL, "request without mesh or block");
  if (m->host_only || m->device != S->device) return set_error(FE_EINVAL, "request mesh is not on the server's device");
  if (r->nvec <= 0 || r->ldx < r->nvec) return set_error(FE_EINVAL, "bad nvec / ldx");
  if (r->prec < FE_F64 || r->prec > FE_BF16) return set_error(FE_EINVAL, "unknown precision");
  if (r->kind == FE_REQ_APPLY) {
    if (!r->Y || r->ldy < r->nvec || r->Y == r->X) return set_error(FE_EINVAL, "bad output block");
  } else if (r->kind == FE_REQ_FILTER) {
    if (!r->lam || r->degree < 1) return set_error(FE_EINVAL, "filter request needs lam and degree >= 1");
    if (!(r->lam_max > r->lam_T) || !(r->lam_min < r->lam_T)) return set_error(FE_EINVAL, "need lam_min < lam_T < lam_max");
  } else {
    return set_error(FE_EINVAL, "unknown request kind");
  }
  std::lock_guard<std::mutex> g(S->mu);
  if (hipSetDevice(S->device) != hipSuccess) return set_error(FE_EDEVICE, "hipSetDevice failed");
  if (extra_bytes(*r) + m->footprint > S->budget) return set_error(FE_ENOMEM, "request can never fit the HBM budget");
  S->meshes.insert(m);   // resident from now on: counted against the budget
  Req *q = new Req();
  q->id = S->next_id++;
  q->r = *r;
  q->t_submit = now_s();
  S->queue.push_back(q);
  S->all[q->id] = q;
  *id = q->id;
  return FE_OK;
}

fe_status fe_server_progress(fe_server_t S, int32_t block, int32_t *n_active, int32_t *n_queued) {
  if (!S) return set_error(FE_EINVAL, "NULL server");
  std::lock_guard<std::mutex> g(S->mu);
  if (hipSetDevice(S->device) != hipSuccess) return set_error(FE_EDEVICE, "hipSetDevice failed");
  fe_status st = S->progress(block != 0);
  if (n_active) *n_active = (int32_t)S->active.size();
  if (n_queued) *n_queued = (int32_t)S->queue.size();
  return st;
}

fe_status fe_server_drain(fe_server_t S) {
  if (!S) return set_error(FE_EINVAL, "NULL server");
  for (;;) {
    int32_t a = 0, q = 0;
    fe_status st = fe_server_progress(S, 1, &a, &q);
    if (st) return st;
    if (a == 0 && q == 0) return FE_OK;
  }
}

fe_status fe_server_status(fe_server_t S, int64_t id, int32_t *state, double *times, int32_t *err) {
  if (!S) return set_error(FE_EINVAL, "NULL server");
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->all.find(id);
  if (it == S->all.end()) return set_error(FE_EINVAL, "unknown request id");
  Req *q = it->second;
  if (state) *state = q->state;
  if (times) { times[0] = q->t_submit; times[1] = q->t_admit; times[2] = q->t_done; }
  if (err) *err = q->err;
  return FE_OK;
}

fe_status fe_server_stats(fe_server_t S, int64_t *ticks, int64_t *held_bytes) {
  if (!S) return set_error(FE_EINVAL, "NULL server");
  std::lock_guard<std::mutex> g(S->mu);
  if (ticks) *ticks = S->nticks;
  if (held_bytes) *held_bytes = S->held();
  return FE_OK;
}

fe_status fe_server_set_work_cap(fe_server_t S, int64_t cap) {
  if (!S) return set_error(FE_EINVAL, "NULL server");
  if (cap < 0) return set_error(FE_EINVAL, "work cap must be >= 0");
  std::lock_guard<std::mutex> g(S->mu);
  S->work_cap = cap;
  return FE_OK;
}

fe_status fe_server_pool_stats(fe_server_t S, int64_t *allocs, int64_t *frees, int64_t *idle_bytes) {
  if (!S) return set_error(FE_EINVAL, "NULL server");
  std::lock_guard<std::mutex> g(S->mu);
  if (allocs) *allocs = S->pool.allocs;
  if (frees) *frees = S->pool.frees;
  if (idle_bytes) *idle_bytes = S->pool.bytes;
  return FE_OK;
}

fe_status fe_server_destroy(fe_server_t S) {
  if (!S) return FE_OK;
  hipSetDevice(S->device);
  hipStreamSynchronize(S->s);
  S->pool.clear();
  for (auto &kv : S->all) {
    if (kv.second->done) hipEventDestroy(kv.second->done);
    delete kv.second;
  }
  for (hipEvent_t e : S->ticks) hipEventDestroy(e);
  for (hipEvent_t e : S->spare) hipEventDestroy(e);
  hipStreamDestroy(S->s);
  delete S;
  return FE_OK;
}

}  // extern "C"
