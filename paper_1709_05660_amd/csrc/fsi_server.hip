// Solve server: continuous batching of independent systems on one GPU.
//
// Setup threads admit queued requests in arrival order while a slot is free
// and the estimated device footprint fits the budget and set them up; each
// admitted hierarchy stays resident.  Each system's Krylov work runs on its
// own stream.  Its V-cycles run either there too (tick threads advance each
// system by one unit of FGMRES work as soon as its previous unit finished,
// the systems' kernels overlapping on the device) or, with batch_vcycles, in
// lockstep ticks: every tick takes the systems whose previous unit finished,
// and the V-cycles of those that are at an Arnoldi step run together, one
// batched launch per phase of the cycle over all of them, on the server's
// batch stream between the steps' two halves on the systems' own streams.
// A system that finishes is retired (result copied to host, device memory
// returned to the server's caching pool) and the next request admitted.  Device memory and streams are recycled: while
// serving no hipFree (a device-wide synchronisation) and no stream creation
// happens once the pool has warmed up.
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <functional>
#include <tuple>
#include <thread>

#include "fsi_internal.h"

namespace fsi {

using Clock = std::chrono::steady_clock;
constexpr int kSetupThreads = 6;   // concurrent setups (each on its system's stream)
constexpr int kTickThreads = 2;    // threads that advance the active systems (each owns a share)
constexpr int kCopyThreads = 4;    // threads that copy submitted requests (with the submitting thread)

struct Request {
  uint64_t ticket = 0;
  std::unique_ptr<char[]> buf;   // every array of the request, one uninitialised host block
  std::vector<fsi_level> levels;
  std::vector<double> b;
  fsi_mg_opts mo{};
  fsi_krylov_opts ko{};
  int64_t footprint = 0, transient = 0;
  Clock::time_point t_submit;
};

struct Active {
  std::unique_ptr<Request> req;
  MG *mg = nullptr;
  hipStream_t side = nullptr;
  size_t b_bytes = 0, x_bytes = 0;
  int owner = 0;   // the tick thread that advances this system
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;   // batched mode: the first half of a step on st is done
  double *d_b = nullptr, *d_x = nullptr;
  FgmresRun run;
  Clock::time_point t_ready;
};

struct Done {
  std::vector<double> x;
  fsi_solve_info info{};
  fsi_status status = FSI_OK;
  std::string msg;
};

// Copies of large requests are split in chunks over the server's copy
// threads (and the submitting thread): one thread's memcpy bandwidth bounded
// the serving rate.  Each submit waits for its own chunks only.
struct CopyPool {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::function<void()>> jobs;
  std::vector<std::thread> th;
  bool stop = false;
  void start(int n) {
    for (int i = 0; i < n; ++i)
      th.emplace_back([this] {
        while (true) {
          std::function<void()> job;
          {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return stop || !jobs.empty(); });
            if (jobs.empty()) return;
            job = std::move(jobs.front());
            jobs.pop_front();
          }
          job();
        }
      });
  }
  // runs the copies (dst, src, bytes) in chunks; returns when all are done
  void copy(const std::vector<std::tuple<void *, const void *, size_t>> &cps) {
    constexpr size_t kChunk = 1u << 21;
    struct Wait {
      std::mutex mu;
      std::condition_variable cv;
      int left = 0;
    };
    auto w = std::make_shared<Wait>();
    std::vector<std::function<void()>> mine;
    for (auto &c : cps)
      for (size_t off = 0; off < std::get<2>(c); off += kChunk) {
        char *d = static_cast<char *>(std::get<0>(c)) + off;
        const char *sp = static_cast<const char *>(std::get<1>(c)) + off;
        const size_t nb = std::min(kChunk, std::get<2>(c) - off);
        mine.push_back([d, sp, nb, w] {
          std::memcpy(d, sp, nb);
          std::lock_guard<std::mutex> lk(w->mu);
          if (--w->left == 0) w->cv.notify_all();
        });
      }
    w->left = (int)mine.size();
    if (mine.empty()) return;
    {
      std::lock_guard<std::mutex> lk(mu);
      for (size_t i = 1; i < mine.size(); ++i) jobs.push_back(mine[i]);
    }
    cv.notify_all();
    mine[0]();   // the submitting thread copies too
    for (;;) {   // and takes further chunks while any are queued
      std::function<void()> job;
      {
        std::lock_guard<std::mutex> lk(mu);
        if (jobs.empty()) break;
        job = std::move(jobs.front());
        jobs.pop_front();
      }
      job();
    }
    std::unique_lock<std::mutex> lk(w->mu);
    w->cv.wait(lk, [&] { return w->left == 0; });
  }
  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    for (auto &t : th)
      if (t.joinable()) t.join();
  }
};

struct Server {
  fsi_server_opts o{};
  DevicePool pool;   // destroyed after every system (declared first)
  CopyPool copies;   // request copies at submit
  std::mutex mu;
  std::vector<std::pair<hipStream_t, hipStream_t>> free_streams;   // (main, side) pairs
  std::condition_variable cv;
  std::deque<std::unique_ptr<Request>> queue;
  std::map<uint64_t, Done> done;
  std::set<uint64_t> live;
  std::vector<std::unique_ptr<Active>> active;
  int setting_up = 0;
  std::vector<std::thread> setup_threads;
  std::vector<std::thread> tick_threads;
  int next_owner = 0;
  std::atomic<bool> stop{false};
  uint64_t next_ticket = 1;
  int64_t used = 0, peak = 0, submitted = 0, finished = 0, ticks = 0, max_coresident = 0;
  // batched V-cycles, per tick thread: their stream and the event that ends a
  // group's cycles; the number of groups and of the systems in them
  hipStream_t bst[kTickThreads] = {};
  hipEvent_t bev[kTickThreads] = {};
  int64_t bgroups = 0, bsystems = 0;
};

// device bytes of one system: operators, block inverses, coarse inverse,
// vectors and the Krylov basis; plus the transient dense blocks of the setup
static int64_t footprint(const fsi_level *lv, int nl, const fsi_mg_opts &mo,
                         const fsi_krylov_opts &ko, int64_t *transient_out) {
  const bool mixed = mo.precision != FSI_PREC_FP64;
  const int wbytes = mo.precision == FSI_PREC_FP64 ? 8 : (mo.precision == FSI_PREC_MIXED_FP32 ? 4 : 2);
  int64_t res = 0, transient = 0;
  for (int l = 0; l < nl; ++l) {
    const int64_t n = lv[l].J.nrows;
    auto csr = [&](const fsi_csr &A) { return (A.nrows + 1) * 4 + A.nnz * (4 + 8 + (mixed ? 4 : 0)); };
    res += csr(lv[l].J) + 6 * n * 8;
    if (l == 0) {
      res += n * n * 8;
      transient = std::max<int64_t>(transient, n * ((n + 15) / 16 * 16) * 8 + 2 * n * 8);
      continue;
    }
    res += csr(lv[l].P) + csr(lv[l].R);
    const fsi_patches &P = lv[l].patches;
    // solid blocks apart (solid_precision / refine_sweeps): FP32 owned rows,
    // or full FP32 inverses plus their local block rows
    const bool split = mixed && ((mo.solid_precision != -1 && mo.solid_precision != mo.precision) ||
                                 mo.refine_sweeps > 0);
    int64_t om = 0, m2 = 0, slots = 0, solid_bytes = 0, mlarge = 0;
    for (int k = 0; k < P.npatch; ++k) {
      const int64_t m = P.ptr[k + 1] - P.ptr[k];
      if (m > kMaxPatch) mlarge = std::max(mlarge, m);
      int64_t o = 0, ks = 0;
      for (int64_t p = P.ptr[k]; p < P.ptr[k + 1]; ++p) {
        o += P.owned[p] ? 1 : 0;
        ks += lv[l].J.rowptr[P.dof[p] + 1] - lv[l].J.rowptr[P.dof[p]];
      }
      slots += ks;
      if (split && P.kind && P.kind[k] == 1)
        solid_bytes += mo.refine_sweeps > 0 ? m * m * 4 + ks * 8 + (m + 1) * 4 : o * m * 4;
      else
        om += o * m;
      m2 += m * m;
    }
    res += om * wbytes + solid_bytes + P.ptr[P.npatch] * 48;
    // all levels' dense blocks share one setup scratch; the extraction map
    // (two ints per slot, an offset per block row) is setup scratch too
    transient += m2 * 8 + slots * 8 + P.ptr[P.npatch] * 8;
    // blocks above kMaxPatch dofs: the Gauss-Jordan chain's padded working
    // copy and (mixed forms) the FP64 inverse before its cast
    if (mlarge) res += mlarge * ((mlarge + 15) / 16 * 16) * 8 + (mixed ? mlarge * mlarge * 8 : 0) + mlarge * 12;
  }
  // Krylov: V (m+1 columns), Z (m), w, b and x; H and the rotations; the
  // reductions' chunk sums (two sets of kMaxKrylovCols columns) and norms
  const int64_t nf = lv[nl - 1].J.nrows, m = ko.restart;
  const int64_t kb = krylov_blocks((int)nf);
  res += nf * 8 * (2 * m + 4) + ((m + 1) * m + 6 * (m + 2)) * 8;
  res += (2 * kb * kMaxKrylovCols + kb + 12) * 8;
  // the caching pool may hand out a block up to a quarter (+ 4 KiB) larger
  // than asked for: admission counts that slack too
  const int64_t slack = (res + transient) / 4 + 96 * 4096;
  if (transient_out) *transient_out = transient;
  return res + transient + slack;
}

// The request's arrays in one host block (8-byte aligned pieces), copied by
// the pool: J, P, R, patch lists and Dirichlet flags of every level, b.
static std::unique_ptr<Request> copy_request(const fsi_level *lv, int nl, const double *b,
                                             const fsi_mg_opts &mo, const fsi_krylov_opts &ko,
                                             CopyPool &pool) {
  std::unique_ptr<Request> r(new Request());
  r->levels.resize(nl);
  std::vector<std::tuple<void *, const void *, size_t>> cps;
  size_t total = 0;
  auto room = [&](size_t bytes) {
    const size_t off = total;
    total += (bytes + 7) / 8 * 8;
    return off;
  };
  // first pass: offsets; second pass: pointers and copies
  struct Piece {
    const void *src;
    size_t bytes, off;
    const void **dst;
  };
  std::vector<Piece> pieces;
  auto add = [&](const void *src, size_t bytes, const void **dst) {
    if (src && bytes) pieces.push_back({src, bytes, room(bytes), dst});
    else *dst = src;
  };
  for (int l = 0; l < nl; ++l) {
    fsi_level &L = r->levels[l];
    std::memset(&L, 0, sizeof L);
    auto csr = [&](const fsi_csr &A, fsi_csr &C) {
      C = A;
      add(A.rowptr, sizeof(int64_t) * (size_t)(A.nrows + 1), (const void **)&C.rowptr);
      add(A.colind, sizeof(int32_t) * (size_t)A.nnz, (const void **)&C.colind);
      add(A.val, sizeof(double) * (size_t)A.nnz, (const void **)&C.val);
    };
    csr(lv[l].J, L.J);
    add(lv[l].dirichlet, (size_t)lv[l].J.nrows, (const void **)&L.dirichlet);
    if (l > 0) {
      csr(lv[l].P, L.P);
      csr(lv[l].R, L.R);
      const fsi_patches &P = lv[l].patches;
      const int64_t tot = P.ptr[P.npatch];
      L.patches.npatch = P.npatch;
      add(P.ptr, sizeof(int64_t) * (size_t)(P.npatch + 1), (const void **)&L.patches.ptr);
      add(P.dof, sizeof(int32_t) * (size_t)tot, (const void **)&L.patches.dof);
      add(P.owned, (size_t)tot, (const void **)&L.patches.owned);
      add(P.kind, (size_t)P.npatch, (const void **)&L.patches.kind);
    }
  }
  r->buf.reset(new char[std::max<size_t>(total, 8)]);
  for (auto &pc : pieces) {
    *pc.dst = r->buf.get() + pc.off;
    cps.emplace_back(r->buf.get() + pc.off, pc.src, pc.bytes);
  }
  pool.copy(cps);
  r->b.assign(b, b + lv[nl - 1].J.nrows);
  r->mo = mo;
  r->mo.tuning_db = nullptr;   // served systems are not autotuned per request
  r->ko = ko;
  r->ko.history = nullptr;
  return r;
}

static void finish(Server &S, Active &a, fsi_status st, const std::string &msg, bool have_x) {
  Done d;
  d.status = st;
  d.msg = msg;
  const int n = (int)a.req->b.size();
  if (have_x) {
    d.x.resize(n);
    if (hipMemcpyAsync(d.x.data(), a.d_x, sizeof(double) * n, hipMemcpyDeviceToHost, a.st) != hipSuccess ||
        hipStreamSynchronize(a.st) != hipSuccess) {
      d.status = FSI_E_DEVICE;
      d.msg = "result copy failed";
    }
    a.run.fill_info(&d.info);
  }
  const auto now = Clock::now();
  d.info.setup_ms = std::chrono::duration<double, std::milli>(a.t_ready - a.req->t_submit).count();
  d.info.solve_ms = std::chrono::duration<double, std::milli>(now - a.t_ready).count();
  if (a.st) (void)hipStreamSynchronize(a.st);
  if (a.ev) (void)hipEventDestroy(a.ev);
  if (a.mg) destroy_mg(a.mg);
  if (a.d_b) S.pool.put(a.d_b, a.b_bytes);
  if (a.d_x) S.pool.put(a.d_x, a.x_bytes);
  std::lock_guard<std::mutex> lk(S.mu);
  if (a.st) S.free_streams.push_back({a.st, a.side});
  S.used -= a.req->footprint;
  S.done[a.req->ticket] = std::move(d);
  S.finished++;
  S.cv.notify_all();
}

// Admission + setup threads: requests leave the queue in arrival order while
// a slot is free and the footprint fits the budget; each system is set up on
// its own stream, so setups overlap with each other and with the other
// systems' iterations run by the tick thread.
static void setup_loop(Server *S) {
  (void)hipSetDevice(S->o.device);
  while (true) {
    std::unique_ptr<Request> req;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait_for(lk, std::chrono::milliseconds(5), [&] {
        return S->stop.load() ||
               (!S->queue.empty() && (int)S->active.size() + S->setting_up < S->o.max_slots &&
                S->used + S->queue.front()->footprint <= S->o.hbm_budget_bytes);
      });
      if (S->stop.load()) return;
      if (S->queue.empty() || (int)S->active.size() + S->setting_up >= S->o.max_slots ||
          S->used + S->queue.front()->footprint > S->o.hbm_budget_bytes)
        continue;
      req = std::move(S->queue.front());
      S->queue.pop_front();
      S->used += req->footprint;
      S->peak = std::max(S->peak, S->used);
      S->setting_up++;
    }
    std::unique_ptr<Active> a(new Active());
    a->req = std::move(req);
    const int n = (int)a->req->b.size();
    try {
      {
        std::lock_guard<std::mutex> lk(S->mu);
        if (!S->free_streams.empty()) {
          a->st = S->free_streams.back().first;
          a->side = S->free_streams.back().second;
          S->free_streams.pop_back();
        }
      }
      if (!a->st) {
        hip_check(hipStreamCreate(&a->st), "stream");
        hip_check(hipStreamCreateWithFlags(&a->side, hipStreamNonBlocking), "stream");
      }
      if (S->o.batch_vcycles) hip_check(hipEventCreateWithFlags(&a->ev, hipEventDisableTiming), "event");
      a->mg = mg_setup(a->req->levels.data(), (int)a->req->levels.size(), &a->req->mo, a->st, a->st,
                       &S->pool, a->side);
      a->d_b = static_cast<double *>(S->pool.get(sizeof(double) * n, &a->b_bytes));
      a->d_x = static_cast<double *>(S->pool.get(sizeof(double) * n, &a->x_bytes));
      hip_check(hipMemcpyAsync(a->d_b, a->req->b.data(), sizeof(double) * n, hipMemcpyHostToDevice, a->st), "H2D");
      a->run.start(*a->mg, a->d_b, a->d_x, a->req->ko, a->st);
      a->t_ready = Clock::now();
      release_setup_scratch(*a->mg);      // the setup scratch is only needed during setup
      std::lock_guard<std::mutex> lk(S->mu);
      S->used -= a->req->transient;
      a->req->footprint -= a->req->transient;
      a->owner = S->next_owner++ % kTickThreads;
      S->active.push_back(std::move(a));
      S->setting_up--;
      S->max_coresident = std::max<int64_t>(S->max_coresident, (int64_t)S->active.size());
      S->cv.notify_all();
    } catch (const Error &e) {
      a->t_ready = Clock::now();
      finish(*S, *a, e.code, e.msg, false);
      std::lock_guard<std::mutex> lk(S->mu);
      S->setting_up--;
      S->cv.notify_all();
    }
  }
}

// Tick threads: each owns a share of the active systems and polls their
// streams; a system whose previous unit of FGMRES work has finished is
// advanced by one unit at once, so no system waits for another.
static void tick_loop(Server *S, int me) {
  (void)hipSetDevice(S->o.device);
  while (!S->stop.load()) {
    std::vector<Active *> cur;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (auto &p : S->active)
        if (p->owner == me) cur.push_back(p.get());
      if (cur.empty()) {
        S->cv.wait_for(lk, std::chrono::milliseconds(2), [&] {
          if (S->stop.load()) return true;
          for (auto &p : S->active)
            if (p->owner == me) return true;
          return false;
        });
        continue;
      }
      S->ticks++;
    }
    std::vector<Active *> retired;
    bool progressed = false;
    for (Active *a : cur) {
      try {
        const hipError_t q = hipStreamQuery(a->st);
        if (q == hipErrorNotReady) continue;
        hip_check(q, "tick");
        progressed = true;
        if (a->run.complete()) {
          finish(*S, *a, a->run.converged ? FSI_OK : FSI_NOT_CONVERGED, "", true);
          retired.push_back(a);
        } else {
          a->run.enqueue();
        }
      } catch (const Error &e) {
        finish(*S, *a, e.code, e.msg, false);
        retired.push_back(a);
      }
    }
    if (!retired.empty()) {
      std::lock_guard<std::mutex> lk(S->mu);
      for (Active *r : retired)
        for (size_t i = 0; i < S->active.size(); ++i)
          if (S->active[i].get() == r) {
            S->active.erase(S->active.begin() + i);
            break;
          }
      S->cv.notify_all();
    }
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

// Batched mode, one group of compatible systems at an Arnoldi step: each
// system's first half on its stream, the group's V-cycles on the batch
// stream after all of them, each second half after the V-cycles.
static void run_group(Server *S, int me, const std::vector<Active *> &grp, std::vector<Active *> &retired) {
  hipStream_t bst = S->bst[me];
  hipEvent_t bev = S->bev[me];
  std::vector<BatchItem> items;
  std::vector<Active *> ok;
  for (Active *a : grp) {
    try {
      const double *vin = nullptr;
      double *vout = nullptr;
      a->run.enqueue_step_pre(&vin, &vout);
      hip_check(hipEventRecord(a->ev, a->st), "event");
      hip_check(hipStreamWaitEvent(bst, a->ev, 0), "wait");
      items.push_back(BatchItem{a->mg, vin, vout});
      ok.push_back(a);
    } catch (const Error &e) {
      (void)hipStreamSynchronize(bst);
      finish(*S, *a, e.code, e.msg, false);
      retired.push_back(a);
    }
  }
  if (items.empty()) return;
  try {
    batched_vcycle(items, bst);
    hip_check(hipEventRecord(bev, bst), "event");
  } catch (const Error &e) {
    (void)hipStreamSynchronize(bst);
    for (Active *a : ok) {
      finish(*S, *a, e.code, e.msg, false);
      retired.push_back(a);
    }
    return;
  }
  for (Active *a : ok) {
    try {
      hip_check(hipStreamWaitEvent(a->st, bev, 0), "wait");
      a->run.enqueue_step_post();
    } catch (const Error &e) {
      (void)hipStreamSynchronize(bst);
      finish(*S, *a, e.code, e.msg, false);
      retired.push_back(a);
    }
  }
  std::lock_guard<std::mutex> lk(S->mu);
  S->bgroups++;
  S->bsystems += (int64_t)ok.size();
}

// Batched mode: each tick thread owns a share of the active systems (two
// cohorts, so that one cohort's launches are issued while the other's run)
// and advances its share in lockstep.  A tick first waits until the previous
// unit of every system of the share has finished (at most kLockstepWait; a system still busy then joins
// a later tick), so that systems stay in step and their V-cycles can run
// together.  A finished system then either ends, has its next phase already
// queued (the checks between cycles), or is at an Arnoldi step, and those
// steps run in groups of batch-compatible systems.
constexpr auto kLockstepWait = std::chrono::milliseconds(5);
static void batch_tick_loop(Server *S, int me) {
  (void)hipSetDevice(S->o.device);
  while (!S->stop.load()) {
    std::vector<Active *> cur;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (auto &p : S->active)
        if (p->owner == me) cur.push_back(p.get());
      if (cur.empty()) {
        S->cv.wait_for(lk, std::chrono::milliseconds(2), [&] {
          if (S->stop.load()) return true;
          for (auto &p : S->active)
            if (p->owner == me) return true;
          return false;
        });
        continue;
      }
      S->ticks++;
    }
    const auto t_wait = Clock::now();
    for (bool busy = true; busy && Clock::now() - t_wait < kLockstepWait;) {
      busy = false;
      for (Active *a : cur)
        if (hipStreamQuery(a->st) == hipErrorNotReady) busy = true;
      if (busy) std::this_thread::sleep_for(std::chrono::microseconds(10));
    }
    std::vector<Active *> retired, steps;
    bool progressed = false;
    for (Active *a : cur) {
      try {
        const hipError_t q = hipStreamQuery(a->st);
        if (q == hipErrorNotReady) continue;
        hip_check(q, "tick");
        progressed = true;
        if (a->run.complete()) {
          finish(*S, *a, a->run.converged ? FSI_OK : FSI_NOT_CONVERGED, "", true);
          retired.push_back(a);
        } else if (a->run.phase == FgmresRun::kIter) {
          steps.push_back(a);
        }
      } catch (const Error &e) {
        finish(*S, *a, e.code, e.msg, false);
        retired.push_back(a);
      }
    }
    std::vector<char> taken(steps.size(), 0);
    for (size_t i = 0; i < steps.size(); ++i) {
      if (taken[i]) continue;
      std::vector<Active *> grp;
      for (size_t k = i; k < steps.size() && (int)grp.size() < kMaxBatch; ++k)
        if (!taken[k] && batch_compatible(*steps[k]->mg, *steps[i]->mg)) {
          taken[k] = 1;
          grp.push_back(steps[k]);
        }
      run_group(S, me, grp, retired);
    }
    if (!retired.empty()) {
      std::lock_guard<std::mutex> lk(S->mu);
      for (Active *r : retired)
        for (size_t i = 0; i < S->active.size(); ++i)
          if (S->active[i].get() == r) {
            S->active.erase(S->active.begin() + i);
            break;
          }
      S->cv.notify_all();
    }
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

static void drain(Server *S) {
  for (hipStream_t b : S->bst)
    if (b) (void)hipStreamSynchronize(b);
  for (auto &a : S->active) {
    (void)hipStreamSynchronize(a->st);
    finish(*S, *a, FSI_E_DEVICE, "server destroyed", false);
  }
  S->active.clear();
}

}  // namespace fsi

using namespace fsi;

extern "C" {

fsi_status fsi_server_create(const fsi_server_opts *o, struct fsi_server **out) {
  try {
    if (!o || !out || o->max_slots < 1 || o->hbm_budget_bytes <= 0 ||
        (o->batch_vcycles != 0 && o->batch_vcycles != 1) || o->reserved != 0)
      throw Error(FSI_E_INVALID, "invalid server options");
    Server *S = new Server();
    S->o = *o;
    (void)hipSetDevice(o->device);
    for (int i = 0; o->batch_vcycles && i < kTickThreads; ++i)
      if (hipStreamCreate(&S->bst[i]) != hipSuccess ||
          hipEventCreateWithFlags(&S->bev[i], hipEventDisableTiming) != hipSuccess) {
        for (int k = 0; k <= i; ++k) {
          if (S->bst[k]) (void)hipStreamDestroy(S->bst[k]);
          if (S->bev[k]) (void)hipEventDestroy(S->bev[k]);
        }
        delete S;
        throw Error(FSI_E_DEVICE, "batch stream");
      }
    // the slots' streams are created up front (a stream's first creation is
    // slow), then recycled
    for (int i = 0; i < o->max_slots; ++i) {
      hipStream_t a = nullptr, b = nullptr;
      if (hipStreamCreate(&a) != hipSuccess) break;
      if (hipStreamCreateWithFlags(&b, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(a);
        break;
      }
      S->free_streams.push_back({a, b});
    }
    S->copies.start(kCopyThreads);
    for (int i = 0; i < kSetupThreads; ++i) S->setup_threads.emplace_back(setup_loop, S);
    for (int i = 0; i < kTickThreads; ++i)
      S->tick_threads.emplace_back(o->batch_vcycles ? batch_tick_loop : tick_loop, S, i);
    *out = reinterpret_cast<fsi_server *>(S);
    return FSI_OK;
  } catch (const Error &e) {
    set_error(e.msg);
    return e.code;
  }
}

fsi_status fsi_serve_submit(struct fsi_server *h, const fsi_level *levels, int32_t nlevels,
                            const double *b_host, const fsi_mg_opts *mo, const fsi_krylov_opts *ko,
                            uint64_t *ticket) {
  try {
    Server *S = reinterpret_cast<Server *>(h);
    if (!S || !levels || nlevels < 1 || !b_host || !mo || !ko || !ticket)
      throw Error(FSI_E_INVALID, "null argument");
    // the checks that the footprint estimate and the copy rely on; the full
    // check of every CSR entry and patch list runs in a setup thread (a
    // malformed request fails there and its ticket reports FSI_E_INVALID)
    validate_levels_light(levels, nlevels, mo);
    validate_krylov(*ko);
    if (ko->x0_nonzero) throw Error(FSI_E_INVALID, "a served request starts from x0 = 0");
    int64_t transient = 0;
    const int64_t fp = footprint(levels, nlevels, *mo, *ko, &transient);
    if (fp > S->o.hbm_budget_bytes) throw Error(FSI_E_CAPACITY, "request larger than the memory budget");
    std::unique_ptr<Request> r = copy_request(levels, nlevels, b_host, *mo, *ko, S->copies);
    r->footprint = fp;
    r->transient = transient;
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(S->mu);
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    S->live.insert(r->ticket);
    S->queue.push_back(std::move(r));
    S->submitted++;
    S->cv.notify_all();
    return FSI_OK;
  } catch (const Error &e) {
    set_error(e.msg);
    return e.code;
  }
}

fsi_status fsi_serve_poll(struct fsi_server *h, uint64_t ticket, double *x_host, fsi_solve_info *info) {
  Server *S = reinterpret_cast<Server *>(h);
  if (!S) return FSI_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->done.find(ticket);
  if (it == S->done.end()) return S->live.count(ticket) ? FSI_PENDING : FSI_E_UNKNOWN_TICKET;
  Done &d = it->second;
  if (x_host && !d.x.empty()) std::copy(d.x.begin(), d.x.end(), x_host);
  if (info) *info = d.info;
  const fsi_status st = d.status;
  if (st < 0) set_error(d.msg);
  S->done.erase(it);
  S->live.erase(ticket);
  return st;
}

fsi_status fsi_server_stats(struct fsi_server *h, int64_t out[12]) {
  Server *S = reinterpret_cast<Server *>(h);
  if (!S || !out) return FSI_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  out[0] = S->submitted;
  out[1] = S->finished;
  out[2] = (int64_t)S->active.size();
  out[3] = (int64_t)S->queue.size();
  out[4] = S->used;
  out[5] = S->peak;
  out[6] = S->ticks;
  out[7] = S->max_coresident;
  std::lock_guard<std::mutex> lp(S->pool.mu);
  out[8] = S->pool.allocated;
  out[9] = S->pool.peak_in_use;
  out[10] = S->bgroups;
  out[11] = S->bsystems;
  return FSI_OK;
}

fsi_status fsi_server_destroy(struct fsi_server *h) {
  Server *S = reinterpret_cast<Server *>(h);
  if (!S) return FSI_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  for (auto &t : S->setup_threads)
    if (t.joinable()) t.join();
  for (auto &t : S->tick_threads)
    if (t.joinable()) t.join();
  S->copies.shutdown();
  drain(S);
  for (auto &p : S->free_streams) {
    (void)hipStreamDestroy(p.first);
    (void)hipStreamDestroy(p.second);
  }
  for (int i = 0; i < kTickThreads; ++i) {
    if (S->bev[i]) (void)hipEventDestroy(S->bev[i]);
    if (S->bst[i]) (void)hipStreamDestroy(S->bst[i]);
  }
  delete S;
  return FSI_OK;
}

}  // extern "C"
