// Serving: continuous batching of solve requests (qxd_serve_*).
//
// A scheduler thread admits queued requests in arrival order when the device
// memory their right-hand sides need fits the budget; admitted right-hand
// sides join the batch of their group -- same gauge field, inner precision and
// solver parameters -- at the next step boundary.  Each group has a worker
// thread with its own HIP stream, so groups (for example lattices of
// different sizes) overlap on the device.  A worker repeatedly advances all
// its right-hand sides by one inner iteration (BatchSolver::step) and hands
// finished ones back; a finished right-hand side frees its slot at once.
// Gauge fields stay resident: requests refer to fields uploaded beforehand.
//
// Memory charged against the budget: for every group, the larger of the
// solver slots its worker holds (slots are pooled for reuse and released when
// the group runs idle) and the slots its admitted right-hand sides need; the
// operators (Pauli term, inverse, folded links) the fields of the requests
// have built and keep cached; and, for every admitted request whose operator
// was not built at admission, that operator until its worker has built it
// (from then on the field's cache accounts for it).  Operators a field
// already held when the scheduler first saw it are not charged: they were
// outside the free memory a default budget is taken from.
//
// Besides the budget, right-hand sides are admitted only while the device's
// free memory, less what admitted work has still to allocate (slots and
// operators), covers what they will allocate plus a floor kept for the
// runtime (kernels' private memory is allocated at dispatch, and a dispatch
// that cannot get it ends the process) and other users of the device.
// Nothing else in the process is counted, so this check bounds what the
// budget cannot see.  A request whose right-hand sides do not all fit is
// admitted in pieces, as many as fit at a time; it stays at the head of the
// queue (later requests wait) until all of them are in.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "batch_solver.h"
#include "host.h"
#include "qxd_debug.h"
#include "solver.h"

using namespace qxd;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
  uint64_t ticket;
  qxd_request r;
  double t_submit = 0, t_admit = 0;
  int remaining = 0;
  int status = QXD_OK;
  std::string err;      // why the request failed (its first failure)
  int next_rhs = 0;     // right-hand sides admitted so far (admission may come in pieces)
  int max_iters = 0;
  double max_res = 0;
  size_t op_bytes = 0;  // charged operator memory not yet built (cleared once built or done)
};

struct Rhs {  // one right-hand side handed to a worker
  Req *req;
  int idx;
};

using GroupKey = std::tuple<qxd_field *, int, int, int, int, double, double, int, int>;

GroupKey key_of(const qxd_request &r) {
  const qxd_solver &s = r.solver;
  return GroupKey(r.field, s.inner_prec, s.nkv, s.ncy, s.nmr, s.tol, s.inner_tol, s.maxiter, s.max_outer);
}

}  // namespace

struct Worker;

struct qxd_serve {
  qxd_ctx *ctx = nullptr;
  size_t budget = 0;
  int max_active = 0;
  std::mutex mu;
  std::condition_variable cv;
  bool stopping = false;
  uint64_t next_ticket = 1;
  std::deque<Req *> queue;
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  std::map<uint64_t, qxd_result> results;
  std::map<GroupKey, std::unique_ptr<Worker>> workers;
  size_t op_pending = 0;  // operators admitted requests still have to build
  // fields of the requests seen, with the operator bytes they held when first
  // seen (growth beyond that is charged: what they held is already outside
  // the device memory the budget was taken from)
  std::vector<std::pair<qxd_field *, size_t>> fields;
  int active_rhs = 0;
  std::thread sched;
  std::string error;
};

struct Worker {
  qxd_serve *sv;
  qxd_request proto;
  hipStream_t st = nullptr;
  std::unique_ptr<BatchSolver> bs;
  std::deque<Rhs> inbox;  // guarded by sv->mu
  std::thread th;
  bool quit = false;      // guarded by sv->mu
  size_t slot_b = 0;      // bytes of one solver slot of this group
  size_t held = 0;        // slot bytes the worker's solver holds (guarded by sv->mu)
  int admitted = 0;       // admitted right-hand sides not yet finished (guarded by sv->mu)
  size_t charge() const { return std::max(held, (size_t)admitted * slot_b); }

  void run() {
    (void)hipSetDevice(sv->ctx->device);
    for (;;) {
      std::vector<Rhs> take;
      {
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv.wait_for(lk, std::chrono::milliseconds(20),
                        [&] { return quit || !inbox.empty() || (bs && bs->active() > 0); });
        if (quit && inbox.empty() && (!bs || bs->active() == 0)) return;
        while (!inbox.empty()) {
          take.push_back(inbox.front());
          inbox.pop_front();
        }
      }
      if (!bs) continue;
      std::vector<Finished> fin;
      std::string step_msg;  // why a failed step failed
      {
        qxd_field *f = proto.field;
        std::lock_guard<std::recursive_mutex> flk(f->mu);
        // every admitted right-hand side gets a slot (the scheduler has
        // already charged its memory to the budget)
        if (!take.empty() && bs->free_slots() < (int)take.size()) {
          qxd_status s = bs->reserve(bs->active() + (int)take.size());
          {
            std::lock_guard<std::mutex> lk(sv->mu);
            held = (size_t)bs->capacity() * slot_b;
          }
          if (s != QXD_OK) {
            const std::string msg = qxd_last_error();
            std::lock_guard<std::mutex> lk(sv->mu);
            for (auto &x : take) {
              Finished e;
              e.slot = -1;
              e.tag = x.req;
              e.info = qxd_solve_info{s, 0, 0, 0.0, 0.0};
              fin.push_back(e);
              if (x.req->err.empty()) x.req->err = msg;
            }
            take.clear();
          }
        }
        std::vector<Req *> built;  // requests whose operator now exists
        for (auto &x : take) {
          qxd_status s = bs->add(x.req->r.quark, x.req->r.eta_dev + (int64_t)x.idx * 24 * f->g.V,
                                 x.req->r.psi_dev + (int64_t)x.idx * 24 * f->g.V, false, x.req);
          if (s != QXD_OK) {
            Finished e;
            e.slot = -1;
            e.tag = x.req;
            e.info = qxd_solve_info{s, 0, 0, 0.0, 0.0};
            fin.push_back(e);
            std::lock_guard<std::mutex> lk(sv->mu);
            if (x.req->err.empty()) x.req->err = qxd_last_error();
          } else {
            built.push_back(x.req);
          }
        }
        if (!built.empty()) {
          // the field's operator cache holds these operators now
          std::lock_guard<std::mutex> lk(sv->mu);
          for (Req *q : built) {
            sv->op_pending -= q->op_bytes;
            q->op_bytes = 0;
          }
        }
        if (bs->active() > 0) {
          qxd_status s = bs->step();
          if (s != QXD_OK) {
            // the batch cannot go on: every right-hand side in it ends with
            // the error, so their requests complete and stop() can join
            step_msg = qxd_last_error();
            {
              std::lock_guard<std::mutex> lk(sv->mu);
              sv->error = step_msg;
            }
            bs->abort_all(s);
          }
        }
        for (auto &x : bs->take_finished()) fin.push_back(x);
      }
      if (!fin.empty()) {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (auto &x : fin) {
          Req *q = (Req *)x.tag;
          if (x.info.status != QXD_OK && q->status == QXD_OK) q->status = x.info.status;
          if (x.info.status != QXD_OK && q->err.empty()) q->err = step_msg;
          if (x.info.inner_iters > q->max_iters) q->max_iters = x.info.inner_iters;
          if (x.info.true_resid > q->max_res) q->max_res = x.info.true_resid;
          sv->active_rhs--;
          admitted--;
          if (--q->remaining == 0) {
            qxd_result res;
            res.status = q->status;
            res.nrhs = q->r.nrhs;
            res.latency_s = now_s() - q->t_submit;
            res.queue_s = q->t_admit - q->t_submit;
            res.inner_iters = q->max_iters;
            res.true_resid = q->max_res;
            sv->results[q->ticket] = res;
            sv->op_pending -= q->op_bytes;
            q->op_bytes = 0;
          }
        }
        sv->cv.notify_all();
      }
      // a group that has run idle gives its pooled slots back to the device
      bool idle;
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        idle = inbox.empty() && bs->active() == 0 && bs->capacity() > 0;
      }
      if (idle) {
        qxd_status s = bs->release_slots();
        std::lock_guard<std::mutex> lk(sv->mu);
        if (s == QXD_OK)
          held = 0;
        else
          sv->error = qxd_last_error();
        sv->cv.notify_all();
      }
    }
  }
};

// free device memory admission leaves untouched: 4 GiB plus 2% of the device
static size_t device_floor(size_t total) { return ((size_t)4 << 30) + total / 50; }

static void scheduler(qxd_serve *sv) {
  (void)hipSetDevice(sv->ctx->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    // admit in arrival order while the footprint fits
    while (!sv->queue.empty()) {
      Req *q = sv->queue.front();
      qxd_field *f = q->r.field;
      const size_t slot_b = BatchSolver::slot_bytes(f, q->r.solver.inner_prec, q->r.solver);
      const bool first = q->next_rhs == 0;
      const size_t op_b = first ? f->pending_op_bytes_nowait(q->r.quark, q->r.solver.inner_prec) : 0;
      if (std::find_if(sv->fields.begin(), sv->fields.end(), [&](const std::pair<qxd_field *, size_t> &x) {
            return x.first == f;
          }) == sv->fields.end())
        sv->fields.emplace_back(f, f->op_mem.load());
      GroupKey gk = key_of(q->r);
      auto wit = sv->workers.find(gk);
      Worker *w0 = wit == sv->workers.end() ? nullptr : wit->second.get();
      // work charged for admitted requests (slots, operators being built),
      // and the operators resident on the fields (built and cached)
      size_t work = sv->op_pending, resident = 0;
      for (auto &kv : sv->workers) work += kv.second->charge();
      for (auto &fd : sv->fields) {
        const size_t now = fd.first->op_mem.load();
        resident += now > fd.second ? now - fd.second : 0;
      }
      const size_t before = w0 ? w0->charge() : 0;
      const size_t held0 = w0 ? w0->held : 0;
      const int adm0 = w0 ? w0->admitted : 0;
      // what admitted work of the other groups has still to allocate
      size_t pend_base = sv->op_pending;
      for (auto &kv : sv->workers) {
        const Worker *w = kv.second.get();
        if (w == w0) continue;
        const size_t need = (size_t)w->admitted * w->slot_b;
        pend_base += need > w->held ? need - w->held : 0;
      }
      size_t dev_free = 0, dev_total = 0;
      const bool have_info = hipMemGetInfo(&dev_free, &dev_total) == hipSuccess;
      // can k more right-hand sides of this request be admitted?
      auto ok = [&](int k) {
        const size_t need0 = (size_t)(adm0 + k) * slot_b;
        const size_t after = std::max(held0, need0);
        const size_t to_alloc = pend_base + (need0 > held0 ? need0 - held0 : 0) + op_b;
        const bool budget_ok = work - before + after + op_b + resident <= sv->budget;
        const bool dev_ok = have_info && dev_free >= to_alloc && dev_free - to_alloc >= device_floor(dev_total);
        const bool room = sv->max_active <= 0 || sv->active_rhs + k <= sv->max_active;
        return budget_ok && dev_ok && room;
      };
      // the most of its remaining right-hand sides that fit (the conditions
      // only tighten as k grows); a request may be admitted in pieces, and
      // holds back the later ones until all its right-hand sides are in
      const int left = q->r.nrhs - q->next_rhs;
      int k = 0;
      for (int lo = 1, hi = left; lo <= hi;) {
        const int mid = lo + (hi - lo) / 2;
        if (ok(mid)) {
          k = mid;
          lo = mid + 1;
        } else {
          hi = mid - 1;
        }
      }
      // one right-hand side always runs when no other work is charged,
      // whatever the cached operators hold (if the device cannot hold it, it
      // ends with QXD_ENOMEM)
      if (k == 0 && work == 0 && sv->active_rhs == 0) k = 1;
      if (k == 0) break;
      auto &w = sv->workers[gk];
      if (!w) {
        w.reset(new Worker());
        w->sv = sv;
        w->proto = q->r;
        w->slot_b = slot_b;
        lk.unlock();
        hipStream_t st = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        std::unique_ptr<BatchSolver> bs(new BatchSolver(f, q->r.solver.inner_prec, q->r.solver, st));
        lk.lock();
        if (e != hipSuccess) {
          sv->error = "hipStreamCreate failed";
        }
        w->st = st;
        w->bs = std::move(bs);
        w->th = std::thread([wp = w.get()] { wp->run(); });
      }
      if (first) {
        q->t_admit = now_s();
        q->remaining = q->r.nrhs;
        q->op_bytes = op_b;
        sv->op_pending += op_b;
      }
      w->admitted += k;
      sv->active_rhs += k;
      for (int i = 0; i < k; i++) w->inbox.push_back(Rhs{q, q->next_rhs + i});
      q->next_rhs += k;
      sv->cv.notify_all();
      if (q->next_rhs < q->r.nrhs) break;  // the rest waits for room
      sv->queue.pop_front();
    }
    if (sv->stopping && sv->queue.empty()) break;
    sv->cv.wait_for(lk, std::chrono::milliseconds(20));
  }
  for (auto &kv : sv->workers) kv.second->quit = true;
  sv->cv.notify_all();
  std::vector<Worker *> ws;
  for (auto &kv : sv->workers) ws.push_back(kv.second.get());
  lk.unlock();
  for (auto *w : ws)
    if (w->th.joinable()) w->th.join();
  for (auto *w : ws) {
    w->bs.reset();
    if (w->st) (void)hipStreamDestroy(w->st);
  }
}

static bool valid_request(const qxd_request *r) {
  if (!r || !r->field || !r->eta_dev || !r->psi_dev || r->nrhs < 1) return false;
  const qxd_solver &s = r->solver;
  return s.kind == QXD_SOLVER_SAP_GCR && s.tol > 0 && s.tol < 1 && s.inner_prec >= QXD_F64 &&
         s.inner_prec <= QXD_BF16 && s.nkv >= 0 && s.nkv <= 64 && s.ncy >= 0 && s.nmr >= 0 &&
         s.inner_tol >= 0 && s.inner_tol < 1;
}

extern "C" {

qxd_status qxd_debug_serve_charges(qxd_ctx *ctx, size_t out[4]) {
  if (!ctx || !ctx->serve || !out) {
    set_error("serving not started or out is NULL");
    return QXD_EINVAL;
  }
  qxd_serve *sv = ctx->serve;
  std::lock_guard<std::mutex> lk(sv->mu);
  size_t resident = 0, slots = 0;
  for (auto &fd : sv->fields) {
    const size_t now = fd.first->op_mem.load();
    resident += now > fd.second ? now - fd.second : 0;
  }
  for (auto &kv : sv->workers) slots += kv.second->charge();
  out[0] = sv->op_pending;
  out[1] = resident;
  out[2] = slots;
  out[3] = sv->budget;
  return QXD_OK;
}

qxd_status qxd_serve_start(qxd_ctx *ctx, size_t budget_bytes, int max_active) {
  if (!ctx) {
    set_error("ctx is NULL");
    return QXD_EINVAL;
  }
  if (ctx->serve) {
    set_error("serving already started on this context");
    return QXD_EINVAL;
  }
  QXD_HIP_CHECK(hipSetDevice(ctx->device));
  if (budget_bytes == 0) {
    size_t fr = 0, tot = 0;
    QXD_HIP_CHECK(hipMemGetInfo(&fr, &tot));
    // the rest stays free for the runtime, the fields' operator caches (a few
    // unused operators per field are kept) and other users of the device
    budget_bytes = (size_t)(0.7 * fr);
  }
  qxd_serve *sv = new qxd_serve();
  sv->ctx = ctx;
  sv->budget = budget_bytes;
  sv->max_active = max_active;
  ctx->serve = sv;
  sv->sched = std::thread(scheduler, sv);
  return QXD_OK;
}

qxd_status qxd_serve_submit(qxd_ctx *ctx, const qxd_request *req, uint64_t *ticket) {
  if (!ctx || !ctx->serve || !ticket) {
    set_error("serving not started or ticket is NULL");
    return QXD_EINVAL;
  }
  if (!valid_request(req)) {
    set_error("invalid request (SAP_GCR solver, nrhs >= 1, device buffers and a field are required)");
    return QXD_EINVAL;
  }
  if (req->field->ctx != ctx) {
    set_error("the request's field belongs to another context");
    return QXD_EINVAL;
  }
  {
    qxd_status s = check_sap_blocks(req->field);
    if (s != QXD_OK) return s;
  }
  qxd_serve *sv = ctx->serve;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->stopping) {
    set_error("serving is stopping");
    return QXD_EINVAL;
  }
  std::unique_ptr<Req> q(new Req());
  q->ticket = sv->next_ticket++;
  q->r = *req;
  q->t_submit = now_s();
  *ticket = q->ticket;
  sv->queue.push_back(q.get());
  sv->reqs[q->ticket] = std::move(q);
  sv->cv.notify_all();
  return QXD_OK;
}

qxd_status qxd_serve_poll(qxd_ctx *ctx, uint64_t ticket, qxd_result *out) {
  if (!ctx || !ctx->serve || !out) {
    set_error("serving not started or out is NULL");
    return QXD_EINVAL;
  }
  qxd_serve *sv = ctx->serve;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->results.find(ticket);
  if (it == sv->results.end()) {
    if (sv->reqs.count(ticket)) return QXD_EBUSY;
    set_error("unknown ticket %llu", (unsigned long long)ticket);
    return QXD_ENOTFOUND;
  }
  *out = it->second;
  if (out->status != QXD_OK) {
    auto rq = sv->reqs.find(ticket);
    const std::string &why = rq != sv->reqs.end() ? rq->second->err : std::string();
    set_error("request %llu failed: %s", (unsigned long long)ticket, why.empty() ? "(no message)" : why.c_str());
  }
  sv->results.erase(it);
  sv->reqs.erase(ticket);
  return QXD_OK;
}

qxd_status qxd_serve_stop(qxd_ctx *ctx) {
  if (!ctx) {
    set_error("ctx is NULL");
    return QXD_EINVAL;
  }
  qxd_serve *sv = ctx->serve;
  if (!sv) return QXD_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stopping = true;
    sv->cv.notify_all();
  }
  if (sv->sched.joinable()) sv->sched.join();
  ctx->serve = nullptr;
  delete sv;
  return QXD_OK;
}

}  // extern "C"
