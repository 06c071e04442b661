// server.cpp -- continuous-batching solve server (pa_server_*).
//
// Requests (a problem and GA parameters) are queued by any thread; one worker
// thread per server owns a HIP stream, a table of slots (resident requests)
// and one device arena of the HBM budget, from which each admitted request
// takes exactly the bytes its own sizes need (first fit; freed blocks merge
// with their free neighbours).  Every tick the worker
//   0. retires requests cancelled while resident;
//   1. admits queued requests, in arrival order, while a slot is free and the
//      arena holds the head request's bytes (upload, per-BS normalisation,
//      descriptor), and seeds them (K-means, initial population);
//   2. runs ONE generation for every resident request -- each at its own
//      generation number, read per task from a device array -- with one
//      launch of the fused generation kernel per class of (L, padded K, SE
//      mode) (admitted requests get their initial fitness in the same
//      launches);
//   3. for requests that reached their last generation, takes the best
//      chromosome, copies the result to pinned host memory and frees the
//      slot.
// Requests therefore join and leave the running batch between generations.
// A request's result is bit-identical to pa_solve of the same instance.  A
// tick that fails on the device fails the requests resident at that moment;
// the worker keeps serving the queue if the device still answers, and stops
// (failing everything) if it does not.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <iterator>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "pa_host.h"

namespace pa {
namespace {

// side streams of a server: a tick's size classes run on them concurrently
// (as many as the hardware queues a process gets by default)
constexpr int kServerSideStreams = 4;

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Request {
  uint64_t ticket = 0;
  pa_problem prob{};  // arrays point into the vectors below
  std::vector<double> beta, user_xy, bs_xy;
  pa_ga_params params{};
  size_t bytes = 0;        // device bytes of its arena block
  bool cancel = false;     // cancelled while resident: retired at the next tick
  bool done = false;
  pa_status status = PA_OK;
  std::string error;
  std::vector<uint8_t> best;
  std::vector<float> trace;
  float best_fit = 0.0f;
  int32_t best_index = 0;
  double t_submit = 0.0, t_done = 0.0;
};

// A resident request: its block of the device arena (laid out for its own
// sizes) and the pinned host staging of its result (sized for the largest
// accepted request).
struct Slot {
  DevProblem p;
  uint8_t *pop[2] = {nullptr, nullptr};
  float *fit[2] = {nullptr, nullptr};
  uint8_t *result = nullptr;  // device: best_idx | best_fit | trace[G+1] | best[L*K]
  uint8_t *h_result = nullptr;  // pinned copy of `result`
  Request *req = nullptr;
  size_t off = 0;  // arena block
  int gen = 0;  // next generation to run (-1: initial fitness)
};

// First-fit sub-allocator over [0, size) in 256-byte granules; free blocks
// are kept by offset and merged with their neighbours when released.
struct Arena {
  size_t size = 0, used = 0, peak = 0;
  std::map<size_t, size_t> free_blocks;  // offset -> bytes
  void reset(size_t bytes) {
    size = bytes;
    used = peak = 0;
    free_blocks.clear();
    if (bytes) free_blocks[0] = bytes;
  }
  bool take(size_t bytes, size_t *off) {
    for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, at = it->first + bytes;
      free_blocks.erase(it);
      if (rest) free_blocks[at] = rest;
      used += bytes;
      peak = std::max(peak, used);
      return true;
    }
    return false;
  }
  void give(size_t off, size_t bytes) {
    used -= bytes;
    auto next = free_blocks.lower_bound(off);
    if (next != free_blocks.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_blocks.erase(next);
    }
    if (next != free_blocks.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_blocks[off] = bytes;
  }
};

}  // namespace
}  // namespace pa

struct pa_server {
  pa_context *ctx = nullptr;
  pa_server_cfg cfg{};
  hipStream_t stream = nullptr;
  // a tick's size classes run on these (forked from and joined to `stream`)
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  std::vector<pa::Slot> slots;
  void *arena = nullptr;          // device memory of every resident request
  pa::Arena heap;                 // its sub-allocation (worker thread only)
  void *pinned = nullptr;         // pinned staging (results, descriptors, tasks)
  size_t max_request_bytes = 0;   // arena bytes of the largest accepted request
  size_t result_bytes = 0;        // pinned staging per slot
  pa::GenInst *d_insts = nullptr, *h_insts = nullptr;
  int32_t *d_gens = nullptr, *h_gens = nullptr;
  int32_t *d_which = nullptr, *h_which = nullptr;  // [3][nslots]: kmeans | init | best lists
  pa::GenTask *d_tasks = nullptr, *h_tasks = nullptr;
  size_t task_cap = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<pa::Request *> queue;
  std::unordered_map<uint64_t, pa::Request *> reqs;
  uint64_t next_ticket = 1;
  int resident = 0;
  bool stop = false;
  pa_status failed = PA_OK;
  std::string fail_msg;
  uint64_t submitted = 0, completed = 0, ticks = 0, cancelled = 0, failed_reqs = 0;
  int max_chunk = 0;     // most tasks one workgroup ran in a launch (worker thread)
  int max_resident = 0;  // most requests resident at once
  uint64_t fault_tick = 0;  // test hook: this tick reports an injected device error
  std::thread worker;
};

namespace pa {
namespace {

// Layout of a request's arena block, for its own sizes.
struct SlotLayout {
  size_t beta, T2, T1, T2z, Town, lconst, user_xy, bs_xy, seed, cent, labels, iters, pop0, pop1,
      fit0, fit1, result, total;
};

SlotLayout layout(int Lq, int Kq, int Nq, int Gq) {
  const size_t L = Lq, K = Kq, TP = pad_pilots(Kq), N = Nq;
  SlotLayout a{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += up256(bytes);
    return at;
  };
  a.beta = take(8 * L * L * K);
  a.T2 = take(4 * L * L * TP);
  a.T1 = take(4 * L * L * TP);
  a.T2z = take(4 * L * L * TP);
  a.Town = take(4 * L * TP);
  a.lconst = take(4 * 2 * L);
  a.user_xy = take(8 * L * K * 2);
  a.bs_xy = take(8 * L * 2);
  a.seed = take(L * K);
  a.cent = take(4 * 2 * K);
  a.labels = take(4 * L * K);
  a.iters = take(4);
  a.pop0 = take(N * L * K);
  a.pop1 = take(N * L * K);
  a.fit0 = take(4 * N);
  a.fit1 = take(4 * N);
  a.result = take(8 + 4 * ((size_t)Gq + 1) + L * K);
  a.total = o;
  return a;
}

size_t result_staging(const pa_server_cfg &c) {
  return up256(8 + 4 * ((size_t)c.max_gens + 1) + (size_t)c.max_L * c.max_K);
}

void fail_all(pa_server *S, pa_status st, const std::string &msg) {
  // caller holds S->mu
  for (auto &kv : S->reqs) {
    pa::Request *r = kv.second;
    if (!r->done) {
      r->done = true;
      r->status = st;
      r->error = msg;
      r->t_done = now_s();
    }
  }
  S->queue.clear();
  for (auto &sl : S->slots) sl.req = nullptr;
  S->resident = 0;
  S->heap.reset(S->heap.size);
}

// Ends the resident request of slot i with status st (not OK): frees its
// arena block and slot.  Caller holds S->mu.
void retire(pa_server *S, int i, pa_status st, const std::string &msg) {
  Slot &sl = S->slots[i];
  Request *r = sl.req;
  r->done = true;
  r->status = st;
  r->error = msg;
  r->t_done = now_s();
  S->heap.give(sl.off, r->bytes);
  sl.req = nullptr;
  --S->resident;
  if (st == PA_ECANCELED) ++S->cancelled;
  else ++S->failed_reqs;
}

// Lays out request r in its arena block (slot i, block at sl.off), uploads it
// and writes its descriptor.
hipError_t admit(pa_server *S, int i, Request *r) {
  Slot &sl = S->slots[i];
  sl.req = r;
  sl.gen = -1;
  const pa_problem &pr = r->prob;
  DevProblem &p = sl.p;
  {
    const SlotLayout lay = layout(pr.L, pr.K, r->params.pop, r->params.gens);
    uint8_t *b = static_cast<uint8_t *>(S->arena) + sl.off;
    p.beta = reinterpret_cast<double *>(b + lay.beta);
    p.T2 = reinterpret_cast<float *>(b + lay.T2);
    p.T1 = reinterpret_cast<float *>(b + lay.T1);
    p.T2z = reinterpret_cast<float *>(b + lay.T2z);
    p.Town = reinterpret_cast<float *>(b + lay.Town);
    p.lconst = reinterpret_cast<float *>(b + lay.lconst);
    p.user_xy = reinterpret_cast<double *>(b + lay.user_xy);
    p.bs_xy = reinterpret_cast<double *>(b + lay.bs_xy);
    p.seed = b + lay.seed;
    p.km_cent = reinterpret_cast<int32_t *>(b + lay.cent);
    p.km_labels = reinterpret_cast<int32_t *>(b + lay.labels);
    p.km_iters = reinterpret_cast<int32_t *>(b + lay.iters);
    sl.pop[0] = b + lay.pop0;
    sl.pop[1] = b + lay.pop1;
    sl.fit[0] = reinterpret_cast<float *>(b + lay.fit0);
    sl.fit[1] = reinterpret_cast<float *>(b + lay.fit1);
    sl.result = b + lay.result;
  }
  p.L = pr.L;
  p.K = pr.K;
  p.TP = pad_pilots(pr.K);
  p.se_mode = pr.se_mode;
  p.objective = pr.objective;
  p.prelog = pr.T > 0 ? (float)(1.0 - (double)pr.K / (double)pr.T) : 1.0f;
  const size_t L = p.L, K = p.K;
  hipStream_t s = S->stream;
  hipError_t e = hipMemcpyAsync(p.beta, r->beta.data(), 8 * L * L * K, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(p.lconst, 0, 4 * 2 * L, s);
  if (e == hipSuccess) e = hipMemsetAsync(p.km_iters, 0, 4, s);
  if (e == hipSuccess && pr.user_xy) {
    e = hipMemcpyAsync(p.user_xy, r->user_xy.data(), 8 * L * K * 2, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(p.bs_xy, r->bs_xy.data(), 8 * L * 2, hipMemcpyHostToDevice, s);
  }
  if (e == hipSuccess) e = launch_prep(p, pr.M, pr.rho, s);
  if (e != hipSuccess) return e;
  GenInst &I = S->h_insts[i];
  std::memset(&I, 0, sizeof I);
  I.T2 = p.T2;
  I.T1 = p.T1;
  I.T2z = p.T2z;
  I.Town = p.Town;
  I.lconst = p.lconst;
  I.pop[0] = sl.pop[0];
  I.pop[1] = sl.pop[1];
  I.fit[0] = sl.fit[0];
  I.fit[1] = sl.fit[1];
  I.best_idx = reinterpret_cast<int32_t *>(sl.result);
  I.best_fit = reinterpret_cast<float *>(sl.result + 4);
  I.trace = reinterpret_cast<float *>(sl.result + 8);
  I.best_out = sl.result + 8 + 4 * ((size_t)r->params.gens + 1);
  I.user_xy = pr.user_xy ? p.user_xy : nullptr;
  I.bs_xy = pr.user_xy ? p.bs_xy : nullptr;
  I.seed = p.seed;
  I.km_cent = p.km_cent;
  I.km_labels = p.km_labels;
  I.km_iters = p.km_iters;
  I.L = p.L;
  I.K = p.K;
  I.TP = p.TP;
  I.N = r->params.pop;
  I.E = r->params.elite;
  I.G = r->params.gens;
  I.prelog = p.prelog;
  I.se_mode = p.se_mode;
  I.objective = p.objective;
  I.ga = ga_from_params(&r->params);
  return hipMemcpyAsync(S->d_insts + i, &S->h_insts[i], sizeof(GenInst), hipMemcpyHostToDevice, s);
}

struct ClassKey {
  int L, TP, mode;
  bool operator<(const ClassKey &o) const {
    return L != o.L ? L < o.L : TP != o.TP ? TP < o.TP : mode < o.mode;
  }
};

// One tick; returns the first HIP error.
hipError_t tick(pa_server *S, std::vector<int> &finished) {
  const int ns = (int)S->slots.size();
  hipStream_t s = S->stream;
  std::vector<int> fresh;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    // requests cancelled while resident leave before this tick's work
    for (int i = 0; i < ns; ++i)
      if (S->slots[i].req && S->slots[i].req->cancel)
        retire(S, i, PA_ECANCELED, "request cancelled");
    // admission in arrival order while a slot is free and the arena holds the
    // head request's own bytes
    for (int i = 0; i < ns && !S->queue.empty(); ++i) {
      if (S->slots[i].req) continue;
      Request *r = S->queue.front();
      size_t off = 0;
      if (!S->heap.take(r->bytes, &off)) break;
      S->queue.pop_front();
      S->slots[i].req = r;  // reserved; uploaded below
      S->slots[i].off = off;
      S->slots[i].gen = -1;
      ++S->resident;
      fresh.push_back(i);
    }
    S->max_resident = std::max(S->max_resident, S->resident);
  }
  hipError_t e = hipSuccess;
  int nkm = 0;
  int32_t *kmw = S->h_which, *initw = S->h_which + ns, *bestw = S->h_which + 2 * ns;
  int maxN = 0;
  for (int i : fresh) {
    if (e == hipSuccess) e = admit(S, i, S->slots[i].req);
    const Request *r = S->slots[i].req;
    if (r->params.kmeans_frac > 0.0) kmw[nkm++] = i;
    maxN = std::max(maxN, r->params.pop);
  }
  for (size_t k = 0; k < fresh.size(); ++k) initw[k] = fresh[k];
  if (e == hipSuccess && !fresh.empty()) {
    e = hipMemcpyAsync(S->d_which, S->h_which, sizeof(int32_t) * 2 * ns, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_kmeans_batch(S->d_insts, S->d_which, nkm, s);
    if (e == hipSuccess)
      e = launch_init_batch(S->d_insts, (int)fresh.size(), maxN, s, S->d_which + ns);
  }
  // tasks of every resident request at its own generation, by class
  std::map<ClassKey, std::vector<int>> classes;
  for (int i = 0; i < ns; ++i) {
    const Slot &sl = S->slots[i];
    if (!sl.req) continue;
    classes[ClassKey{sl.p.L, sl.p.TP, sl.p.se_mode}].push_back(i);
    S->h_gens[i] = sl.gen;
  }
  size_t nt = 0;
  struct Launch {
    GenClass c;
    size_t off;
  };
  std::vector<Launch> launches;
  for (auto &kv : classes) {
    int maxK = 0;
    for (int i : kv.second) maxK = std::max(maxK, S->slots[i].p.K);
    GenClass c;
    c.L = kv.first.L;
    c.TP = kv.first.TP;
    c.mode = kv.first.mode;
    c.block = gen_class_block(c.L, c.TP, c.mode, maxK);
    const size_t off = nt;
    for (int i : kv.second) {
      const Slot &sl = S->slots[i];
      const int N = sl.req->params.pop, E = sl.req->params.elite, K = sl.p.K;
      const int cpr = std::max(1, c.block / K);
      if (sl.gen < 0) {
        for (int a = 0; a < N; a += cpr)
          S->h_tasks[nt++] = GenTask{i, kTaskEval, a, std::min(N, a + cpr)};
      } else {
        S->h_tasks[nt++] = GenTask{i, kTaskElite, 0, E};
        for (int a = E; a < N; a += cpr)
          S->h_tasks[nt++] = GenTask{i, kTaskChild, a, std::min(N, a + cpr)};
      }
    }
    c.ntasks = (int)(nt - off);
    c.grid = gen_class_grid(c.L, c.TP, c.mode, c.block, c.ntasks, S->ctx->info.cus);
    launches.push_back(Launch{c, off});
    S->max_chunk = std::max(S->max_chunk, (c.ntasks + c.grid - 1) / std::max(1, c.grid));
  }
  if (e == hipSuccess && nt > 0) {
    e = hipMemcpyAsync(S->d_tasks, S->h_tasks, sizeof(GenTask) * nt, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(S->d_gens, S->h_gens, sizeof(int32_t) * ns, hipMemcpyHostToDevice, s);
    // several size classes: each on a side stream, so that they overlap
    const size_t nside = launches.size() > 1 ? std::min(launches.size(), S->side.size()) : 0;
    if (nside > 0 && e == hipSuccess) e = hipEventRecord(S->fork, s);
    for (size_t j = 0; j < nside && e == hipSuccess; ++j)
      e = hipStreamWaitEvent(S->side[j], S->fork, 0);
    for (size_t k = 0; k < launches.size(); ++k) {
      if (e != hipSuccess) break;
      Launch &L = launches[k];
      L.c.tasks = S->d_tasks + L.off;
      L.c.gens = S->d_gens;
      e = launch_gen(S->d_insts, L.c, 0, S->ctx->info, nside > 0 ? S->side[k % nside] : s);
    }
    for (size_t j = 0; j < nside && e == hipSuccess; ++j) {
      e = hipEventRecord(S->join[j], S->side[j]);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, S->join[j], 0);
    }
  }
  // advance; requests past their last generation finish
  int nb = 0;
  finished.clear();
  for (int i = 0; i < ns; ++i) {
    Slot &sl = S->slots[i];
    if (!sl.req) continue;
    ++sl.gen;
    if (sl.gen >= sl.req->params.gens) {
      bestw[nb++] = i;
      finished.push_back(i);
    }
  }
  if (e == hipSuccess && nb > 0) {
    e = hipMemcpyAsync(S->d_which + 2 * ns, bestw, sizeof(int32_t) * nb, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_best_batch(S->d_insts, nb, -1, s, S->d_which + 2 * ns);
    for (int i : finished) {
      if (e != hipSuccess) break;
      const Slot &sl = S->slots[i];
      const size_t LK = (size_t)sl.p.L * sl.p.K;
      e = hipMemcpyAsync(sl.h_result, sl.result, 8 + 4 * ((size_t)sl.req->params.gens + 1) + LK,
                         hipMemcpyDeviceToHost, s);
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && S->fault_tick != 0 && S->ticks + 1 == S->fault_tick)
    e = hipErrorLaunchFailure;  // test hook (the tick's work itself completed)
  return e;
}

// Waits for every stream of the server (errors ignored): after it no kernel
// or copy of the server is in flight.
void drain(pa_server *S) {
  for (hipStream_t st : S->side)
    if (st) (void)hipStreamSynchronize(st);
  if (S->stream) (void)hipStreamSynchronize(S->stream);
}

void complete(pa_server *S, const std::vector<int> &finished) {
  const double t = now_s();
  std::lock_guard<std::mutex> lk(S->mu);
  for (int i : finished) {
    Slot &sl = S->slots[i];
    Request *r = sl.req;
    const size_t LK = (size_t)sl.p.L * sl.p.K;
    const uint8_t *h = sl.h_result;
    std::memcpy(&r->best_index, h, 4);
    std::memcpy(&r->best_fit, h + 4, 4);
    r->trace.assign(reinterpret_cast<const float *>(h + 8),
                    reinterpret_cast<const float *>(h + 8) + r->params.gens + 1);
    const uint8_t *b = h + 8 + 4 * ((size_t)r->params.gens + 1);
    r->best.assign(b, b + LK);
    r->done = true;
    r->t_done = t;
    S->heap.give(sl.off, r->bytes);
    sl.req = nullptr;
    --S->resident;
    ++S->completed;
  }
  S->cv_done.notify_all();
}

void worker_main(pa_server *S) {
  (void)hipSetDevice(S->ctx->device);
  std::vector<int> finished;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty() || S->resident > 0; });
      if (S->stop) return;
    }
    const hipError_t e = tick(S, finished);
    if (e != hipSuccess) {
      // no work of the failed tick may still run when its requests' memory
      // is reused: wait for every stream first
      drain(S);
      (void)hipGetLastError();
      const std::string msg = std::string("server worker: ") + hipGetErrorString(e);
      std::lock_guard<std::mutex> lk(S->mu);
      ++S->ticks;
      for (int i = 0; i < (int)S->slots.size(); ++i)
        if (S->slots[i].req) retire(S, i, PA_EDEVICE, msg);
      // keep serving when the device still answers, else fail everything
      const hipError_t h = hipStreamSynchronize(S->stream);
      if (h != hipSuccess || hipGetLastError() != hipSuccess) {
        S->failed = PA_EDEVICE;
        S->fail_msg = msg;
        fail_all(S, PA_EDEVICE, S->fail_msg);
        S->cv_done.notify_all();
        return;
      }
      S->cv_done.notify_all();
      continue;
    }
    ++S->ticks;
    if (!finished.empty()) complete(S, finished);
  }
}

void free_server(pa_server *S) {
  if (!S) return;
  if (S->ctx) (void)hipSetDevice(S->ctx->device);
  drain(S);  // no kernel or copy of the server runs when its memory is freed
  if (S->arena) (void)hipFree(S->arena);
  if (S->d_insts) (void)hipFree(S->d_insts);
  if (S->d_gens) (void)hipFree(S->d_gens);
  if (S->d_which) (void)hipFree(S->d_which);
  if (S->d_tasks) (void)hipFree(S->d_tasks);
  if (S->pinned) (void)hipHostFree(S->pinned);
  for (hipStream_t st : S->side)
    if (st) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : S->join)
    if (ev) (void)hipEventDestroy(ev);
  if (S->fork) (void)hipEventDestroy(S->fork);
  if (S->stream) (void)hipStreamDestroy(S->stream);
  for (auto &kv : S->reqs) delete kv.second;
  delete S;
}

}  // namespace
}  // namespace pa

using namespace pa;

extern "C" {

pa_status pa_server_create(pa_context *ctx, const pa_server_cfg *cfg, pa_server **out) {
  if (!ctx || !out) return set_error(PA_EINVAL, "context or out is NULL");
  *out = nullptr;
  pa_server_cfg c{};
  if (cfg) c = *cfg;
  if (c.max_slots == 0) c.max_slots = 512;
  if (c.max_queue == 0) c.max_queue = 1 << 20;
  if (c.max_L == 0) c.max_L = 37;
  if (c.max_K == 0) c.max_K = 32;
  if (c.max_pop == 0) c.max_pop = 1024;
  if (c.max_gens == 0) c.max_gens = 1000;
  if (c.max_slots < 1 || c.max_queue < 1 || c.max_L < 1 || c.max_L > kMaxL || c.max_K < 1 ||
      c.max_K > kMaxK || c.max_pop < 2 || c.max_pop > 65536 || c.max_gens < 1 ||
      c.hbm_budget < 0.0)
    return set_error(PA_EINVAL, "server configuration out of range");
  pa_status st = use_device(ctx);
  if (st != PA_OK) return st;
  pa_server *S = new (std::nothrow) pa_server;
  if (!S) return set_error(PA_ENOMEM, "host allocation failed");
  std::unique_ptr<pa_server, void (*)(pa_server *)> guard(S, free_server);
  S->ctx = ctx;
  S->max_request_bytes = layout(c.max_L, c.max_K, c.max_pop, c.max_gens).total;
  S->result_bytes = result_staging(c);
  double budget = c.hbm_budget;
  if (budget == 0.0) {
    size_t freeb = 0, total = 0;
    if (hipMemGetInfo(&freeb, &total) != hipSuccess) return set_error(PA_EDEVICE, "hipMemGetInfo");
    budget = 0.8 * (double)freeb;
  }
  // the arena: the budget, but never more than max_slots largest requests
  const double cap = (double)S->max_request_bytes * c.max_slots;
  const size_t arena = (size_t)std::min(budget, cap) & ~(size_t)255;
  if (arena < 256)
    return set_error(PA_ENOMEM, "HBM budget %.0f B holds no request", budget);
  const int ns = c.max_slots;
  c.hbm_budget = budget;
  S->cfg = c;
  S->slots.resize(ns);
  S->task_cap = (size_t)ns * (c.max_pop + 1);
  if (const char *f = std::getenv("PA_SERVER_FAULT_TICK")) S->fault_tick = std::strtoull(f, nullptr, 10);
  hipError_t e = hipMalloc(&S->arena, arena);
  if (e == hipSuccess) S->heap.reset(arena);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&S->d_insts), sizeof(GenInst) * ns);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&S->d_gens), sizeof(int32_t) * ns);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&S->d_which), sizeof(int32_t) * 3 * ns);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&S->d_tasks), sizeof(GenTask) * S->task_cap);
  const size_t pin_bytes = up256(S->result_bytes * ns) + up256(sizeof(GenInst) * ns) +
                           up256(sizeof(int32_t) * 4 * ns) + sizeof(GenTask) * S->task_cap;
  if (e == hipSuccess) e = hipHostMalloc(&S->pinned, pin_bytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&S->fork, hipEventDisableTiming);
  for (int j = 0; j < kServerSideStreams && e == hipSuccess; ++j) {
    S->side.push_back(nullptr);
    S->join.push_back(nullptr);
    e = hipStreamCreateWithFlags(&S->side.back(), hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->join.back(), hipEventDisableTiming);
  }
  if (e != hipSuccess) return hip_error(e, "server allocation");
  uint8_t *pin = static_cast<uint8_t *>(S->pinned);
  uint8_t *h_results = pin;
  pin += up256(S->result_bytes * ns);
  S->h_insts = reinterpret_cast<GenInst *>(pin);
  pin += up256(sizeof(GenInst) * ns);
  S->h_gens = reinterpret_cast<int32_t *>(pin);
  S->h_which = S->h_gens + ns;
  pin += up256(sizeof(int32_t) * 4 * ns);
  S->h_tasks = reinterpret_cast<GenTask *>(pin);
  for (int i = 0; i < ns; ++i) S->slots[i].h_result = h_results + S->result_bytes * i;
  S->worker = std::thread(worker_main, S);
  *out = guard.release();
  return PA_OK;
}

pa_status pa_server_submit(pa_server *S, const pa_problem *prob, const pa_ga_params *params,
                           uint64_t *ticket) {
  if (!S || !prob || !params || !ticket) return set_error(PA_EINVAL, "NULL argument");
  pa_status st = pa_params_check(prob, params);
  if (st != PA_OK) return st;
  if (prob->L > S->cfg.max_L || prob->K > S->cfg.max_K || params->pop > S->cfg.max_pop ||
      params->gens > S->cfg.max_gens)
    return set_error(PA_EINVAL, "request (L=%d K=%d pop=%d gens=%d) exceeds the server's slots "
                     "(L<=%d K<=%d pop<=%d gens<=%d)", prob->L, prob->K, params->pop,
                     params->gens, S->cfg.max_L, S->cfg.max_K, S->cfg.max_pop, S->cfg.max_gens);
  Request *r = new (std::nothrow) Request;
  if (!r) return set_error(PA_ENOMEM, "host allocation failed");
  const size_t L = prob->L, K = prob->K;
  r->beta.assign(prob->beta, prob->beta + L * L * K);
  if (prob->user_xy) {
    r->user_xy.assign(prob->user_xy, prob->user_xy + L * K * 2);
    r->bs_xy.assign(prob->bs_xy, prob->bs_xy + L * 2);
  }
  r->bytes = layout(prob->L, prob->K, params->pop, params->gens).total;
  if (r->bytes > S->heap.size) {
    const size_t need = r->bytes, have = S->heap.size;
    delete r;
    return set_error(PA_ENOMEM, "request needs %zu bytes of device memory, the server has %zu",
                     need, have);
  }
  r->prob = *prob;
  r->prob.beta = r->beta.data();
  r->prob.user_xy = prob->user_xy ? r->user_xy.data() : nullptr;
  r->prob.bs_xy = prob->user_xy ? r->bs_xy.data() : nullptr;
  r->params = *params;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->failed != PA_OK) {
      delete r;
      return set_error(S->failed, "%s", S->fail_msg.c_str());
    }
    if ((long)S->queue.size() >= S->cfg.max_queue) {
      delete r;
      return set_error(PA_EAGAIN, "queue full (%d requests)", S->cfg.max_queue);
    }
    r->ticket = S->next_ticket++;
    r->t_submit = now_s();
    S->queue.push_back(r);
    S->reqs[r->ticket] = r;
    ++S->submitted;
    *ticket = r->ticket;
  }
  S->cv_work.notify_one();
  return PA_OK;
}

pa_status pa_server_poll(pa_server *S, uint64_t ticket, pa_result *out, int32_t block) {
  if (!S || !out) return set_error(PA_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return set_error(PA_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  Request *r = it->second;
  if (!r->done) {
    if (!block) return set_error(PA_EAGAIN, "ticket %llu not done", (unsigned long long)ticket);
    S->cv_done.wait(lk, [&] { return r->done; });
  }
  const pa_status st = r->status;
  if (st == PA_OK) {
    if (out->best) std::memcpy(out->best, r->best.data(), r->best.size());
    if (out->trace) std::memcpy(out->trace, r->trace.data(), sizeof(float) * r->trace.size());
    out->best_fit = r->best_fit;
    out->best_index = r->best_index;
    out->device_ms = (r->t_done - r->t_submit) * 1e3;
  }
  const std::string msg = r->error;
  S->reqs.erase(it);
  delete r;
  if (st != PA_OK) return set_error(st, "%s", msg.c_str());
  return PA_OK;
}

pa_status pa_server_cancel(pa_server *S, uint64_t ticket) {
  if (!S) return set_error(PA_EINVAL, "NULL argument");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end())
      return set_error(PA_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    if (r->done) return set_error(PA_EINVAL, "ticket %llu has already finished", (unsigned long long)ticket);
    auto q = std::find(S->queue.begin(), S->queue.end(), r);
    if (q != S->queue.end()) {
      S->queue.erase(q);
      r->done = true;
      r->status = PA_ECANCELED;
      r->error = "request cancelled";
      r->t_done = now_s();
      ++S->cancelled;
    } else {
      r->cancel = true;  // resident: the worker retires it before its next tick
    }
  }
  S->cv_done.notify_all();
  S->cv_work.notify_one();
  return PA_OK;
}

pa_status pa_server_stats(pa_server *S, pa_server_counters *out) {
  if (!S || !out) return set_error(PA_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  out->slots = (int32_t)S->slots.size();
  out->resident = S->resident;
  out->queued = (int32_t)S->queue.size();
  out->submitted = S->submitted;
  out->completed = S->completed;
  out->ticks = S->ticks;
  out->slot_bytes = (double)S->max_request_bytes;
  out->max_tasks_per_workgroup = S->max_chunk;
  out->max_resident = S->max_resident;
  out->cancelled = S->cancelled;
  out->failed = S->failed_reqs;
  out->arena_bytes = (double)S->heap.size;
  out->arena_peak_bytes = (double)S->heap.peak;
  return PA_OK;
}

void pa_server_destroy(pa_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();  // finishes its current tick
  free_server(S);
}

}  // extern "C"
