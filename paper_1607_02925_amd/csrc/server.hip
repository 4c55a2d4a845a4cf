// Request server: continuous batching of independent low-rank problems on one
// GPU.  Requests of any shape and storage type queue in arrival order; a
// request is admitted when a worker slot is idle and its whole device
// workspace fits in what is left of the server's HBM arena.  Each slot is a
// host thread with its own HIP stream, so the solves of admitted requests
// overlap on the device while every request runs exactly the kernels, in
// exactly the order, that lowrank_solve runs for it alone: results do not
// depend on what else is in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena.h"
#include "engine.h"
#include "lowrank.h"

namespace {

lr_status fail(lr_status s, const std::string& msg) {
  lr::set_last_error(msg);
  return s;
}

struct Request {
  uint64_t ticket = 0;
  lr_matrix X{};
  int k = 0, p = 0;
  double eps = 0;
  lr_options opt{};
  lr_schedule replay{};
  std::vector<int32_t> replay_epochs;
  double* U = nullptr;
  double* theta = nullptr;
  size_t bytes = 0, off = 0;
  int state = 0;  // 0 queued, 1 running, 2 done
  lr_status status = LR_OK;
  std::string err;
  lr_report rep{};
  lr_ticket_info info{};
};

struct Slot {
  hipStream_t st = nullptr;
  lr::HostRes host{};
  std::thread th;
};

}  // namespace

struct lr_server_s {
  int device = 0;
  char* base = nullptr;
  lr::Arena arena;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  bool stop = false;
  uint64_t next_ticket = 1;
  int64_t submitted = 0, completed = 0;
  int running = 0, peak_running = 0;
  size_t peak_bytes = 0;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  void run(Request* r, Slot& sl) {
    lr_plan_s* pl = nullptr;
    lr_status s = lr::plan_make(&pl, &r->X, r->k, r->p, r->eps, &r->opt, sl.st, base + r->off,
                                r->bytes, &sl.host);
    if (s == LR_OK) {
      s = lowrank_solve(pl, r->U, r->theta, &r->rep);
      if (s != LR_OK) r->err = lr::last_error();
      lowrank_destroy(pl);
    } else {
      r->err = lr::last_error();
    }
    // nothing of this request may still run on its workspace once released
    const hipError_t e = hipStreamSynchronize(sl.st);
    if (e != hipSuccess && s == LR_OK) {
      s = LR_EDEVICE;
      r->err = std::string("hipStreamSynchronize: ") + hipGetErrorString(e);
    }
    r->status = s;
  }

  void worker(int si) {
    (void)hipSetDevice(device);
    Slot& sl = slots[si];
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      // FIFO admission: the head request starts as soon as its workspace fits.
      cv_work.wait(lk, [&] {
        return (!queue.empty() && arena.fits(queue.front()->bytes)) || (stop && queue.empty());
      });
      if (queue.empty()) return;
      Request* r = queue.front();
      queue.pop_front();
      size_t off = 0;
      arena.alloc(r->bytes, &off);
      r->off = off;
      r->state = 1;
      r->info.t_admit = now();
      r->info.slot = si;
      ++running;
      peak_running = std::max(peak_running, running);
      peak_bytes = std::max(peak_bytes, arena.used());
      cv_work.notify_all();  // the next head may fit as well
      lk.unlock();
      run(r, sl);
      lk.lock();
      arena.release(r->off, r->bytes);
      r->state = 2;
      r->info.t_done = now();
      --running;
      ++completed;
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }

  // Under the lock: hand a finished request's results to the caller and
  // forget the ticket.
  lr_status collect(std::unordered_map<uint64_t, std::unique_ptr<Request>>::iterator it,
                    lr_report* rep, lr_ticket_info* info, std::string* err) {
    Request* r = it->second.get();
    if (rep) *rep = r->rep;
    if (info) *info = r->info;
    const lr_status s = r->status;
    *err = r->err;
    reqs.erase(it);
    return s;
  }
};

extern "C" {

lr_status lowrank_server_create(lr_server* out, size_t hbm_budget_bytes, int slots) {
  if (!out) return fail(LR_EINVAL, "null server pointer");
  *out = nullptr;
  if (slots < 1 || slots > LR_MAX_SLOTS) return fail(LR_EINVAL, "slots must be in [1, 16]");
  if (hbm_budget_bytes < lr::Arena::ALIGN) return fail(LR_EINVAL, "budget too small");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LR_EDEVICE, "no HIP device");
  }
  std::unique_ptr<lr_server_s> sv;
  try {
    sv.reset(new lr_server_s());
  } catch (...) {
    return fail(LR_ENOMEM, "host allocation failed");
  }
  sv->device = dev;
  const size_t cap = hbm_budget_bytes & ~(lr::Arena::ALIGN - 1);
  if (hipMalloc((void**)&sv->base, cap) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LR_ENOMEM, "cannot allocate the server's HBM budget");
  }
  sv->arena.reset(cap);
  sv->slots.resize(slots);
  lr_status s = LR_OK;
  for (auto& sl : sv->slots) {
    if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess) {
      s = fail(LR_EDEVICE, "hipStreamCreate failed");
      break;
    }
    s = lr::host_res_create(&sl.host.hpin, sl.host.ev);
    if (s != LR_OK) break;
  }
  if (s == LR_OK) {
    try {
      for (int i = 0; i < slots; ++i)
        sv->slots[i].th = std::thread(&lr_server_s::worker, sv.get(), i);
    } catch (...) {
      s = fail(LR_EDEVICE, "cannot start worker threads");
    }
  }
  if (s != LR_OK) {
    lowrank_server_destroy(sv.release());
    return s;
  }
  *out = sv.release();
  return LR_OK;
}

lr_status lowrank_submit(lr_server sv, const lr_matrix* X, int k, int p, double eps,
                         const lr_options* opt, double* U_out, double* theta_out,
                         uint64_t* ticket) {
  if (!sv || !ticket) return fail(LR_EINVAL, "null argument");
  *ticket = 0;
  if (X && X->layout != LR_DENSE_COLMAJOR)
    return fail(LR_EINVAL, "the server takes dense column-major X");
  lr_status s = lr::plan_check(X, k, p, eps, opt);
  if (s != LR_OK) return s;
  size_t bytes = 0;
  s = lr::plan_bytes(X, k, p, opt, &bytes);
  if (s != LR_OK) return s;
  if (lr::Arena::round_up(bytes) > sv->arena.capacity())
    return fail(LR_ENOMEM, "request workspace exceeds the server's HBM budget");
  std::unique_ptr<Request> r;
  try {
    r.reset(new Request());
    r->X = *X;
    r->k = k;
    r->p = p;
    r->eps = eps;
    if (opt)
      r->opt = *opt;
    else
      lowrank_options_default(&r->opt);
    if (r->opt.replay) {
      r->replay = *r->opt.replay;
      r->replay_epochs.assign(r->replay.epochs, r->replay.epochs + r->replay.outer);
      r->replay.epochs = r->replay_epochs.data();
      r->opt.replay = &r->replay;
    }
  } catch (...) {
    return fail(LR_ENOMEM, "host allocation failed");
  }
  r->U = U_out;
  r->theta = theta_out;
  r->bytes = bytes;
  r->info.workspace_bytes = bytes;
  r->info.slot = -1;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return fail(LR_EINVAL, "server is shutting down");
    r->ticket = sv->next_ticket++;
    r->info.t_submit = sv->now();
    *ticket = r->ticket;
    sv->queue.push_back(r.get());
    sv->reqs.emplace(r->ticket, std::move(r));
    ++sv->submitted;
  }
  sv->cv_work.notify_all();
  return LR_OK;
}

lr_status lowrank_poll(lr_server sv, uint64_t ticket, lr_report* rep, lr_ticket_info* info) {
  if (!sv) return fail(LR_EINVAL, "null server");
  std::string err;
  lr_status s;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return fail(LR_EINVAL, "unknown ticket");
    if (it->second->state != 2) return fail(LR_EBUSY, "request not finished");
    s = sv->collect(it, rep, info, &err);
  }
  if (s != LR_OK) lr::set_last_error(err);
  return s;
}

lr_status lowrank_wait(lr_server sv, uint64_t ticket, lr_report* rep, lr_ticket_info* info) {
  if (!sv) return fail(LR_EINVAL, "null server");
  std::string err;
  lr_status s;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    if (sv->reqs.find(ticket) == sv->reqs.end()) return fail(LR_EINVAL, "unknown ticket");
    // look the ticket up on every wake-up: another waiter may have collected it
    sv->cv_done.wait(lk, [&] {
      auto it = sv->reqs.find(ticket);
      return it == sv->reqs.end() || it->second->state == 2;
    });
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return fail(LR_EINVAL, "ticket collected by another caller");
    s = sv->collect(it, rep, info, &err);
  }
  if (s != LR_OK) lr::set_last_error(err);
  return s;
}

lr_status lowrank_server_stats(lr_server sv, lr_server_stats* out) {
  if (!sv || !out) return fail(LR_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  *out = lr_server_stats{};
  out->submitted = sv->submitted;
  out->completed = sv->completed;
  out->queued = (int64_t)sv->queue.size();
  out->running = sv->running;
  out->budget_bytes = sv->arena.capacity();
  out->bytes_in_use = sv->arena.used();
  out->peak_bytes = sv->peak_bytes;
  out->slots = (int32_t)sv->slots.size();
  out->peak_running = sv->peak_running;
  out->elapsed = sv->now();
  return LR_OK;
}

void lowrank_server_destroy(lr_server sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  for (auto& sl : sv->slots)
    if (sl.th.joinable()) sl.th.join();
  for (auto& sl : sv->slots) {
    if (sl.st) (void)hipStreamDestroy(sl.st);
    lr::host_res_destroy(sl.host.hpin, sl.host.ev);
  }
  if (sv->base) (void)hipFree(sv->base);
  delete sv;
}

}  // extern "C"
