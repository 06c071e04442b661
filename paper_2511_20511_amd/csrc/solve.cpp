// solve.cpp -- whole solves of one instance (pa_solve) or many
// (pa_solve_batch): a plan holds the device descriptors, task lists and
// double-buffered populations of its instances.  Two execution forms:
//  - graph: the whole solve (K-means seeding, initial population and
//    fitness, one generation kernel per generation and class, best of the
//    last population) is captured once into a hipGraph and replayed;
//  - persistent: when the plan has one class whose tasks all fit on the
//    device at once (small instances: the generation kernel would be a few
//    microseconds of latency), every generation runs inside one launch of
//    co-resident workgroups separated by grid barriers, so the table stays
//    in LDS and no per-generation launch is paid;
//  - one-workgroup: when an instance's population and table fit one CU's
//    LDS, one workgroup per instance runs every generation with the
//    population resident in LDS (no grid barrier, no global round trip).
//    The autotuner times it beside the persistent shapes.
// Either way a solve ends with one copy of the results.
#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <string>

#include "pa_host.h"

namespace pa {

struct PlanClass {
  GenClass c;
  int cpt_div = 1;  // children per task = ceil(block / K / cpt_div)
  GenTask *d_tasks = nullptr, *d_evals = nullptr;
  int32_t *d_bounds = nullptr;  // runs of the generation launches (grid + 1)
  double work = 0.0;     // table gathers of one generation (for the class order)
  bool tuned = false;    // the shape came from timing candidates (not the cache)
};

struct SolvePlan {
  int device = 0;
  std::vector<pa_instance *> insts;
  std::vector<pa_ga_params> params;
  std::vector<PlanClass> classes;
  std::vector<void *> owned;  // device allocations
  GenInst *d_insts = nullptr;
  int32_t *d_which = nullptr;
  int nwhich = 0;
  int Gmax = 0, maxN = 0;
  int32_t *d_best_idx = nullptr;
  float *d_best_fit = nullptr;
  float *d_trace = nullptr;      // [n][Gmax + 1]
  uint8_t *d_best = nullptr;     // concatenated best chromosomes
  std::vector<size_t> best_off;  // offsets into d_best
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool persist = false;          // persistent form (one class, co-resident tasks)
  int wg_block = 0;              // one-workgroup form: its threads (0: not this form)
  int wg_maxN = 0, wg_maxK = 0;  // its largest instance
  int pgrid = 0;                 // its workgroups
  uint32_t *d_sync = nullptr;    // [0]: grid-barrier counter, [1]: barrier time-out flag
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int cur_gen = -1;  // stepwise solve: generations done (-1: not started)
  int done_gen = -1; // generations the populations have reached (-1: never run)
  bool seeded = false;  // the populations hold a seeded generation (tuning)
  std::vector<GenInst> h_inst;  // host copy of the descriptors
  std::vector<int32_t> h_idx;
  std::vector<float> h_fit, h_trace;
  std::vector<uint8_t> h_best;
};

void free_plan(SolvePlan *plan) {
  if (!plan) return;
  (void)hipSetDevice(plan->device);
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  if (plan->ev0) (void)hipEventDestroy(plan->ev0);
  if (plan->ev1) (void)hipEventDestroy(plan->ev1);
  for (void *p : plan->owned)
    if (p) (void)hipFree(p);
  delete plan;
}

namespace {

template <class T>
hipError_t alloc(SolvePlan *pl, T **p, size_t count) {
  hipError_t e = hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * (count ? count : 1));
  if (e == hipSuccess) pl->owned.push_back(*p);
  return e;
}

#define PTRY(call, what)                             \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hip_error(e_, what); \
  } while (0)

bool exact_variant(int L, int TP) { return (L == 7 || L == 19 || L == 37) && TP <= 32; }

// A table too large to sit in LDS beside a 256-thread task's buffers (about
// 40 KiB) is tiled by the generation kernel.
bool big_table(int L, int TP, int mode) {
  return (long)L * L * TP * 4 * (mode == 1 ? 2 : 1) + 40 * 1024 > 160 * 1024;
}

struct ClassKey {
  int L, TP, mode;
  bool operator<(const ClassKey &o) const {
    return L != o.L ? L < o.L : TP != o.TP ? TP < o.TP : mode < o.mode;
  }
  bool operator==(const ClassKey &o) const { return L == o.L && TP == o.TP && mode == o.mode; }
};

// Tasks of a class when each task holds ceil(block / K / div) children.
int count_tasks(const std::vector<int> &members, const std::vector<pa_instance *> &insts,
                const std::vector<pa_ga_params> &params, int block, int div = 1) {
  int n = 0;
  for (int i : members) {
    const int cpr = std::max(1, (block / insts[i]->p.K + div - 1) / div);
    n += 1 + (params[i].pop - params[i].elite + cpr - 1) / cpr;
  }
  return n;
}

// Launch shape of a class: threads per workgroup and children per task
// (ceil(block / K / cpt_div)).
struct Shape {
  int block, cpt_div;
};

// Runs of a generation launch's task list for `grid` workgroups, cut by task
// cost: a child task costs about the same whatever its number of children
// (every lane of the workgroup runs the gathers), an elite task about a
// quarter of one.  The runs are contiguous (a workgroup keeps an instance's
// table across its tasks) and their largest cost is the smallest any cut
// into `grid` contiguous runs achieves (binary search on the cap, greedy
// filling); bounds[r] .. bounds[r + 1] is run r, unused runs are empty.
std::vector<int32_t> cost_runs(const std::vector<GenTask> &tasks, int grid) {
  const int n = (int)tasks.size();
  std::vector<int64_t> w(n);
  int64_t total = 0, wmax = 0;
  for (int i = 0; i < n; ++i) {
    w[i] = tasks[i].kind == kTaskElite ? 1 : 4;
    total += w[i];
    wmax = std::max(wmax, w[i]);
  }
  auto runs_for = [&](int64_t cap) {
    int runs = 1;
    int64_t cur = 0;
    for (int i = 0; i < n; ++i) {
      if (cur + w[i] > cap) {
        ++runs;
        cur = 0;
      }
      cur += w[i];
    }
    return runs;
  };
  int64_t lo = std::max(wmax, (total + grid - 1) / std::max(grid, 1)), hi = std::max(total, lo);
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (runs_for(mid) <= grid)
      hi = mid;
    else
      lo = mid + 1;
  }
  std::vector<int32_t> bounds(grid + 1, n);
  bounds[0] = 0;
  int r = 0;
  int64_t cur = 0;
  for (int i = 0; i < n; ++i) {
    if (cur + w[i] > lo) {
      bounds[++r] = i;
      cur = 0;
    }
    cur += w[i];
  }
  return bounds;
}

// Task lists (device) of a class of instances for a launch shape.
pa_status make_class(SolvePlan *pl, const ClassKey &key, const std::vector<int> &members,
                     const std::vector<GenInst> &hi, const Shape &sh, int cus, PlanClass *out) {
  PlanClass pc;
  pc.c.L = key.L;
  pc.c.TP = key.TP;
  pc.c.mode = key.mode;
  pc.c.block = sh.block;
  pc.cpt_div = sh.cpt_div;
  std::vector<GenTask> tasks, evals;
  for (int i : members) {
    const int K = hi[i].K, N = hi[i].N, E = hi[i].E;
    pc.work += (double)(N - E) * key.L * key.L * K;
    const int cpr = std::max(1, (pc.c.block / K + sh.cpt_div - 1) / sh.cpt_div);
    tasks.push_back(GenTask{i, kTaskElite, 0, E});
    for (int s = E; s < N; s += cpr) tasks.push_back(GenTask{i, kTaskChild, s, std::min(N, s + cpr)});
    for (int s = 0; s < N; s += cpr) evals.push_back(GenTask{i, kTaskEval, s, std::min(N, s + cpr)});
  }
  const int per_cu = gen_class_per_cu(key.L, key.TP, key.mode, pc.c.block);
  if (per_cu < 1)
    return set_error(PA_EUNSUPPORTED, "no generation kernel of L=%d TP=%d at %d threads fits a CU",
                     key.L, key.TP, pc.c.block);
  pc.c.grid = std::min((int)tasks.size(), cus * per_cu);
  pc.c.ntasks = (int)tasks.size();
  const std::vector<int32_t> bounds = cost_runs(tasks, pc.c.grid);
  pc.c.neval = (int)evals.size();
  PTRY(alloc(pl, &pc.d_tasks, tasks.size()), "hipMalloc(tasks)");
  PTRY(alloc(pl, &pc.d_evals, evals.size()), "hipMalloc(tasks)");
  PTRY(hipMemcpy(pc.d_tasks, tasks.data(), sizeof(GenTask) * tasks.size(), hipMemcpyHostToDevice),
       "upload");
  PTRY(hipMemcpy(pc.d_evals, evals.data(), sizeof(GenTask) * evals.size(), hipMemcpyHostToDevice),
       "upload");
  PTRY(alloc(pl, &pc.d_bounds, bounds.size()), "hipMalloc(tasks)");
  PTRY(hipMemcpy(pc.d_bounds, bounds.data(), sizeof(int32_t) * bounds.size(),
                 hipMemcpyHostToDevice),
       "upload");
  pc.c.tasks = pc.d_tasks;
  pc.c.eval_tasks = pc.d_evals;
  pc.c.bounds = pc.d_bounds;
  *out = pc;
  return PA_OK;
}

hipError_t launch_start(SolvePlan *pl, hipStream_t s);
hipError_t launch_persist(SolvePlan *pl, const DeviceInfo &dev, int g0, int g1, bool best,
                          hipStream_t s);
hipError_t launch_wg(SolvePlan *pl, int block, int g0, int g1, bool best, hipStream_t s);

// Autotuning of the small-instance forms: every persistent shape (block size
// from `blocks`, each with its co-residency cap; children per task = block /
// K / div for div = 1, 2, 4, ..., all tasks co-resident) and every
// one-workgroup shape (`wg_blocks`) runs the start and the first 8 and 40
// generations of the plan's own instances; the shape whose cost extrapolated
// to the plan's generation count is smallest is kept (within 3%: the
// one-workgroup form, which leaves the other CUs free, then the larger
// workgroup).  PA_SMALL_FORM=persistent or workgroup keeps only that form's
// shapes.  Shapes and forms change the schedule, never a result bit.
pa_status tune_persistent(SolvePlan *pl, pa_context *ctx, const ClassKey &key,
                          const std::vector<int> &members, const std::vector<GenInst> &hi,
                          const std::vector<std::pair<int, int>> &blocks,
                          const std::vector<int> &wg_blocks) {
  int maxK = 0;
  for (int i : members) maxK = std::max(maxK, hi[i].K);
  const char *form_env = std::getenv("PA_SMALL_FORM");
  const std::string form = form_env ? form_env : "";
  std::vector<PlanClass> cands;
  if (form != "workgroup") {
    for (const auto &bc : blocks) {
      const int block = bc.first, cap = bc.second;
      int last_tasks = -1;
      for (int div = 1; div <= std::max(1, block / maxK); div *= 2) {
        const int nt = count_tasks(members, pl->insts, pl->params, block, div);
        if (nt > cap) break;
        if (nt == last_tasks) continue;
        last_tasks = nt;
        PlanClass pc;
        pa_status st = make_class(pl, key, members, hi, Shape{block, div}, ctx->info.cus, &pc);
        if (st != PA_OK) return st;
        cands.push_back(pc);
      }
    }
  }
  // candidates: persistent shapes (wg = 0, index into cands), then
  // one-workgroup shapes (wg = threads)
  struct Cand {
    size_t pc;
    int wg;
  };
  std::vector<Cand> all;
  for (size_t c = 0; c < cands.size(); ++c) all.push_back({c, 0});
  if (form != "persistent")
    for (int b : wg_blocks) all.push_back({0, b});
  if (all.empty()) return set_error(PA_EINTERNAL, "no persistent or one-workgroup shape");
  auto select = [&](const Cand &cd) {
    pl->persist = cd.wg == 0;
    pl->wg_block = cd.wg;
    if (cd.wg == 0) {
      pl->classes.assign(1, cands[cd.pc]);
      pl->pgrid = cands[cd.pc].c.ntasks;
    } else {
      pl->classes.clear();
    }
  };
  size_t best = 0;
  if (all.size() > 1) {
    // each shape's start-up and per-generation cost from a short and a long
    // run (best of two each), extrapolated to the plan's generation count
    hipStream_t cs = ctx->stream;
    const int gs = std::min(pl->Gmax, 8), gl = std::min(pl->Gmax, 40);
    std::vector<float> ests(all.size(), 0.0f);
    for (size_t c = 0; c < all.size(); ++c) {
      select(all[c]);
      float t[2] = {0.0f, 0.0f};
      for (int k = 0; k < (gl > gs ? 2 : 1); ++k) {
        for (int rep = 0; rep < 2; ++rep) {
          PTRY(launch_start(pl, cs), "tuning");
          PTRY(hipEventRecord(pl->ev0, cs), "hipEventRecord");
          if (all[c].wg)
            PTRY(launch_wg(pl, all[c].wg, -1, k == 0 ? gs : gl, false, cs), "tuning");
          else
            PTRY(launch_persist(pl, ctx->info, -1, k == 0 ? gs : gl, false, cs), "tuning");
          PTRY(hipEventRecord(pl->ev1, cs), "hipEventRecord");
          PTRY(hipEventSynchronize(pl->ev1), "hipEventSynchronize");
          float ms = 0.0f;
          PTRY(hipEventElapsedTime(&ms, pl->ev0, pl->ev1), "hipEventElapsedTime");
          t[k] = rep == 0 ? ms : std::min(t[k], ms);
        }
      }
      const float est =
          gl > gs ? t[0] + (t[1] - t[0]) * (float)(pl->Gmax - gs) / (float)(gl - gs) : t[0];
      uint32_t sync[2] = {0, 0};
      PTRY(hipMemcpy(sync, pl->d_sync, sizeof sync, hipMemcpyDeviceToHost), "tuning");
      if (sync[1] != 0) return set_error(PA_EINTERNAL, "persistent solve: a grid barrier wait timed out");
      ests[c] = est;
    }
    // estimates within 3% of the best count as equal (run-to-run noise is of
    // that order); among them the one-workgroup form, then the larger
    // workgroup, then the cheaper, wins
    auto block_of = [&](const Cand &cd) { return cd.wg ? cd.wg : cands[cd.pc].c.block; };
    const float lo = *std::min_element(ests.begin(), ests.end());
    for (size_t c = 0; c < all.size(); ++c) {
      if (ests[c] > lo * 1.03f) continue;
      const bool bwg = all[best].wg != 0, cwg = all[c].wg != 0;
      if (ests[best] > lo * 1.03f || (cwg && !bwg) ||
          (cwg == bwg && (block_of(all[c]) > block_of(all[best]) ||
                          (block_of(all[c]) == block_of(all[best]) && ests[c] < ests[best]))))
        best = c;
    }
  }
  select(all[best]);
  return PA_OK;
}

// Releases the device task lists of a candidate class that was not kept.
void drop_class(SolvePlan *pl, const PlanClass &pc) {
  for (void *p : {(void *)pc.d_tasks, (void *)pc.d_evals}) {
    auto it = std::find(pl->owned.begin(), pl->owned.end(), p);
    if (it != pl->owned.end()) {
      (void)hipFree(p);
      pl->owned.erase(it);
    }
  }
}

// Tuned shapes of the graph form, keyed by device and class signature; kept
// for the process and, when PA_TUNE_CACHE names a file, in that file (one
// "key block div" line per entry).
struct TuneCache {
  std::mutex mu;
  std::map<std::string, Shape> map;
  bool loaded = false;
};
TuneCache &tune_cache() {
  static TuneCache c;
  return c;
}

std::string class_signature(const pa_context *ctx, const ClassKey &key,
                            const std::vector<int> &members, const std::vector<GenInst> &hi) {
  hipDeviceProp_t prop;
  std::string arch = "gfx";
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  long sumN = 0;
  int maxK = 0, minK = 1 << 30, maxG = 0;
  for (int i : members) {
    sumN += hi[i].N;
    maxK = std::max(maxK, hi[i].K);
    minK = std::min(minK, hi[i].K);
    maxG = std::max(maxG, hi[i].G);
  }
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s/cu%d/L%d/TP%d/m%d/n%d/N%ld/K%d-%d/G%d", arch.c_str(),
                ctx->info.cus, key.L, key.TP, key.mode, (int)members.size(), sumN, minK, maxK,
                maxG > 0 ? 1 : 0);
  return buf;
}

bool cache_lookup(const std::string &sig, Shape *out) {
  TuneCache &c = tune_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  if (!c.loaded) {
    c.loaded = true;
    if (const char *path = std::getenv("PA_TUNE_CACHE")) {
      if (FILE *f = std::fopen(path, "r")) {
        char k[200];
        int b, d;
        while (std::fscanf(f, "%199s %d %d", k, &b, &d) == 3) c.map[k] = Shape{b, d};
        std::fclose(f);
      }
    }
  }
  auto it = c.map.find(sig);
  if (it == c.map.end()) return false;
  *out = it->second;
  return true;
}

void cache_store(const std::string &sig, const Shape &sh) {
  TuneCache &c = tune_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  c.map[sig] = sh;
  if (const char *path = std::getenv("PA_TUNE_CACHE")) {
    if (FILE *f = std::fopen(path, "a")) {
      std::fprintf(f, "%s %d %d\n", sig.c_str(), sh.block, sh.cpt_div);
      std::fclose(f);
    }
  }
}

// Autotuning of the graph form, one class at a time: the candidate shapes are
// the workgroup sizes the class's kernel comes in (256 and 512 threads for the
// unrolled variants, one size for the runtime-L variant) times children per
// task ceil(block / K / div), div = 1, 2, 4, 8 (while the task count changes).
// Each candidate's generation launch is timed on the plan's own instances
// (seeded, initial fitness evaluated): two runs of kTuneGens launches, the
// faster kept; the cheapest candidate wins, within 3% the one with fewer
// tasks.  The winner is cached per device architecture and class signature
// (process, and PA_TUNE_CACHE), so a replanned batch of the same shape is not
// timed again.  Shapes change the schedule, never a result bit.
constexpr int kTuneGens = 3;

pa_status tune_graph_class(SolvePlan *pl, pa_context *ctx, const ClassKey &key,
                           const std::vector<int> &members, const std::vector<GenInst> &hi,
                           PlanClass *out) {
  const int cus = ctx->info.cus;
  int maxK = 0, maxG = 0;
  for (int i : members) {
    maxK = std::max(maxK, hi[i].K);
    maxG = std::max(maxG, hi[i].G);
  }
  std::vector<int> blocks;
  if (exact_variant(key.L, key.TP)) {
    if (!big_table(key.L, key.TP, key.mode)) blocks.push_back(256);
    blocks.push_back(512);
  } else {
    blocks.push_back(std::max(256, (maxK + 63) / 64 * 64));
  }
  // PA_GRAPH_SHAPE="block,div" in the environment forces one shape when the
  // class's kernel comes in that size (for tests and reproducible profiles)
  if (const char *force = std::getenv("PA_GRAPH_SHAPE")) {
    int b = 0, d = 0;
    if (std::sscanf(force, "%d,%d", &b, &d) == 2 && d >= 1 &&
        std::find(blocks.begin(), blocks.end(), b) != blocks.end() &&
        gen_class_per_cu(key.L, key.TP, key.mode, b) >= 1)
      return make_class(pl, key, members, hi, Shape{b, d}, cus, out);
  }
  const std::string sig = class_signature(ctx, key, members, hi);
  Shape cached{0, 0};
  if (cache_lookup(sig, &cached))
    return make_class(pl, key, members, hi, cached, cus, out);
  std::vector<Shape> cands;
  for (int block : blocks) {
    if (gen_class_per_cu(key.L, key.TP, key.mode, block) < 1) continue;
    int last = -1;
    for (int div = 1; div <= 8 && div <= std::max(1, block / maxK); div *= 2) {
      const int nt = count_tasks(members, pl->insts, pl->params, block, div);
      if (nt == last) continue;
      last = nt;
      cands.push_back(Shape{block, div});
    }
  }
  if (cands.empty())
    return set_error(PA_EUNSUPPORTED, "no generation kernel of L=%d TP=%d fits a CU", key.L, key.TP);
  if (cands.size() == 1 || maxG < 1) {
    const Shape sh = cands.size() == 1 ? cands[0] : Shape{blocks.back(), 1};
    return make_class(pl, key, members, hi, sh, cus, out);
  }
  hipStream_t cs = ctx->stream;
  if (!pl->seeded) {
    PTRY(launch_start(pl, cs), "tuning");
    pl->seeded = true;
  }
  std::vector<float> cost(cands.size(), 0.0f);
  std::vector<int> ntasks(cands.size(), 0);
  std::vector<PlanClass> built(cands.size());
  for (size_t k = 0; k < cands.size(); ++k) {
    pa_status st = make_class(pl, key, members, hi, cands[k], cus, &built[k]);
    if (st != PA_OK) return st;
    ntasks[k] = built[k].c.ntasks;
    PTRY(launch_gen(pl->d_insts, built[k].c, -1, ctx->info, cs), "tuning");
    float best = 0.0f;
    for (int rep = 0; rep < 2; ++rep) {
      PTRY(hipEventRecord(pl->ev0, cs), "hipEventRecord");
      for (int g = 0; g < kTuneGens; ++g)
        PTRY(launch_gen(pl->d_insts, built[k].c, std::min(g, maxG - 1), ctx->info, cs), "tuning");
      PTRY(hipEventRecord(pl->ev1, cs), "hipEventRecord");
      PTRY(hipEventSynchronize(pl->ev1), "hipEventSynchronize");
      float ms = 0.0f;
      PTRY(hipEventElapsedTime(&ms, pl->ev0, pl->ev1), "hipEventElapsedTime");
      best = rep == 0 ? ms : std::min(best, ms);
    }
    cost[k] = best;
  }
  const float lo = *std::min_element(cost.begin(), cost.end());
  size_t win = 0;
  for (size_t k = 0; k < cands.size(); ++k) {
    if (cost[k] > lo * 1.03f) continue;
    if (cost[win] > lo * 1.03f || ntasks[k] < ntasks[win] ||
        (ntasks[k] == ntasks[win] && cost[k] < cost[win]))
      win = k;
  }
  for (size_t k = 0; k < cands.size(); ++k)
    if (k != win) drop_class(pl, built[k]);
  built[win].tuned = true;
  *out = built[win];
  cache_store(sig, cands[win]);
  return PA_OK;
}

pa_status build_plan(pa_context *ctx, int n, pa_instance *const *insts,
                     const pa_ga_params *params, SolvePlan **out) {
  SolvePlan *pl = new (std::nothrow) SolvePlan;
  if (!pl) return set_error(PA_ENOMEM, "host allocation failed");
  std::unique_ptr<SolvePlan, void (*)(SolvePlan *)> guard(pl, free_plan);
  pl->device = ctx->device;
  pl->insts.assign(insts, insts + n);
  pl->params.assign(params, params + n);
  for (int i = 0; i < n; ++i) {
    pl->Gmax = std::max(pl->Gmax, params[i].gens);
    pl->maxN = std::max(pl->maxN, params[i].pop);
  }
  const int TG = pl->Gmax + 1;
  PTRY(alloc(pl, &pl->d_best_idx, n), "hipMalloc(plan)");
  PTRY(alloc(pl, &pl->d_best_fit, n), "hipMalloc(plan)");
  PTRY(alloc(pl, &pl->d_trace, (size_t)n * TG), "hipMalloc(plan)");
  size_t best_total = 0;
  for (int i = 0; i < n; ++i) {
    pl->best_off.push_back(best_total);
    best_total += (size_t)insts[i]->p.L * insts[i]->p.K;
  }
  PTRY(alloc(pl, &pl->d_best, best_total), "hipMalloc(plan)");
  std::vector<GenInst> hi(n);
  std::vector<int32_t> which;
  for (int i = 0; i < n; ++i) {
    const DevProblem &p = insts[i]->p;
    const pa_ga_params &g = params[i];
    GenInst &I = hi[i];
    std::memset(&I, 0, sizeof I);
    const size_t LK = (size_t)p.L * p.K;
    for (int b = 0; b < 2; ++b) {
      PTRY(alloc(pl, &I.pop[b], LK * g.pop), "hipMalloc(population)");
      PTRY(alloc(pl, &I.fit[b], (size_t)g.pop), "hipMalloc(fitness)");
    }
    I.T2 = p.T2;
    I.T1 = p.T1;
    I.T2z = p.T2z;
    I.Town = p.Town;
    I.lconst = p.lconst;
    I.trace = pl->d_trace + (size_t)i * TG;
    I.best_idx = pl->d_best_idx + i;
    I.best_fit = pl->d_best_fit + i;
    I.best_out = pl->d_best + pl->best_off[i];
    I.user_xy = p.user_xy;
    I.bs_xy = p.bs_xy;
    I.seed = p.seed;
    I.km_cent = p.km_cent;
    I.km_labels = p.km_labels;
    I.km_iters = p.km_iters;
    I.L = p.L;
    I.K = p.K;
    I.TP = p.TP;
    I.N = g.pop;
    I.E = g.elite;
    I.G = g.gens;
    I.prelog = p.prelog;
    I.se_mode = p.se_mode;
    I.objective = p.objective;
    I.ga = ga_from_params(&g);
    if (I.ga.n_km > 0) which.push_back(i);
  }
  pl->h_inst = hi;
  PTRY(alloc(pl, &pl->d_insts, (size_t)n), "hipMalloc(plan)");
  PTRY(hipMemcpy(pl->d_insts, hi.data(), sizeof(GenInst) * n, hipMemcpyHostToDevice), "upload");
  pl->nwhich = (int)which.size();
  if (pl->nwhich) {
    PTRY(alloc(pl, &pl->d_which, which.size()), "hipMalloc(plan)");
    PTRY(hipMemcpy(pl->d_which, which.data(), sizeof(int32_t) * which.size(),
                   hipMemcpyHostToDevice),
         "upload");
  }
  // classes of (L, TP, mode), members in input order
  std::vector<std::pair<ClassKey, std::vector<int>>> groups;
  for (int i = 0; i < n; ++i) {
    const ClassKey key{hi[i].L, hi[i].TP, hi[i].se_mode};
    auto it = std::find_if(groups.begin(), groups.end(),
                           [&](const std::pair<ClassKey, std::vector<int>> &g) { return g.first == key; });
    if (it == groups.end()) groups.push_back({key, {i}});
    else it->second.push_back(i);
  }
  // persistent form: one class with an unrolled variant whose full tasks
  // (block / K children each) all fit on the device at once, for 256- and
  // 512-thread workgroups (512 only for tiled tables; PA_PERSIST_BLOCK=256 or
  // 512 in the environment keeps only that size, for reproducible profiles)
  std::vector<std::pair<int, int>> pblocks;
  const char *only_env = std::getenv("PA_PERSIST_BLOCK");
  const int only = only_env ? std::atoi(only_env) : 0;
  if (groups.size() == 1 && exact_variant(groups[0].first.L, groups[0].first.TP)) {
    const ClassKey &key = groups[0].first;
    for (int block : {256, 512}) {
      if (only != 0 && block != only) continue;
      if (block == 256 && big_table(key.L, key.TP, key.mode)) continue;
      GenClass q;
      q.L = key.L;
      q.TP = key.TP;
      q.mode = key.mode;
      q.block = block;
      int cap = 0;
      PersistLaunch ql{};
      ql.grid = 1;
      PTRY(launch_gen_persist(pl->d_insts, q, ql, ctx->info, &cap, nullptr), "occupancy query");
      if (cap > 0 && count_tasks(groups[0].second, pl->insts, pl->params, block) <= cap)
        pblocks.push_back({block, cap});
    }
  }
  // one-workgroup form: the same class, when the largest instance's
  // population, fitness, inverse rows, codes and table fit one CU's LDS and
  // its elites one wave's ranking
  std::vector<int> wgblocks;
  if (!pblocks.empty()) {
    const ClassKey &key = groups[0].first;
    int maxN = 0, maxK = 0, maxE = 0;
    for (int i : groups[0].second) {
      maxN = std::max(maxN, hi[i].N);
      maxK = std::max(maxK, hi[i].K);
      maxE = std::max(maxE, hi[i].E);
    }
    pl->wg_maxN = maxN;
    pl->wg_maxK = maxK;
    for (int block : {256, 512}) {
      if (only != 0 && block != only) continue;
      int lds = 0;
      if (maxE <= wg_max_elites() &&
          launch_gen_wg(nullptr, 0, key.L, key.TP, key.mode, block, 0, 0, false, maxN, maxK, &lds,
                        nullptr) == hipSuccess &&
          lds <= 160 * 1024)
        wgblocks.push_back(block);
    }
  }
  PTRY(alloc(pl, &pl->d_sync, 2), "hipMalloc(plan)");
  PTRY(hipMemset(pl->d_sync, 0, 2 * sizeof(uint32_t)), "hipMemset");
  PTRY(hipEventCreate(&pl->ev0), "hipEventCreate");
  PTRY(hipEventCreate(&pl->ev1), "hipEventCreate");
  if (!pblocks.empty()) {
    pa_status st =
        tune_persistent(pl, ctx, groups[0].first, groups[0].second, hi, pblocks, wgblocks);
    if (st != PA_OK) return st;
  } else {
    for (auto &grp : groups) {
      PlanClass pc;
      pa_status st = tune_graph_class(pl, ctx, grp.first, grp.second, hi, &pc);
      if (st != PA_OK) return st;
      pl->classes.push_back(pc);
    }
    // longest class first: the classes run as concurrent graph branches, so
    // the one with the most work starts first (largest-processing-time order)
    std::stable_sort(pl->classes.begin(), pl->classes.end(),
                     [](const PlanClass &a, const PlanClass &b) { return a.work > b.work; });
  }
  pl->h_idx.resize(n);
  pl->h_fit.resize(n);
  pl->h_trace.resize((size_t)n * TG);
  pl->h_best.resize(best_total);
  if (pl->persist || pl->wg_block) {
    *out = guard.release();
    return PA_OK;
  }
  // capture the whole solve.  Size classes share no buffers, so with more
  // than one class each class's chain of launches is captured on a stream
  // of its own, forked after the seeding and joined before the best: the
  // chains are independent branches of the graph and may run concurrently
  // (the streams serve the capture only)
  hipStream_t cs = ctx->stream;
  const size_t ncls = pl->classes.size();
  std::vector<hipStream_t> side(ncls > 1 ? ncls : 0, nullptr);
  std::vector<hipEvent_t> join(side.size(), nullptr);
  hipEvent_t fork = nullptr;
  auto release_side = [&]() {
    for (hipStream_t st : side)
      if (st) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : join)
      if (ev) (void)hipEventDestroy(ev);
    if (fork) (void)hipEventDestroy(fork);
  };
  hipError_t e = hipSuccess;
  if (!side.empty()) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  for (size_t c = 0; c < side.size() && e == hipSuccess; ++c) {
    e = hipStreamCreateWithFlags(&side[c], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join[c], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    release_side();
    return hip_error(e, "capture streams");
  }
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    release_side();
    return hip_error(e, "hipStreamBeginCapture");
  }
  e = launch_kmeans_batch(pl->d_insts, pl->d_which, pl->nwhich, cs);
  if (e == hipSuccess) e = launch_init_batch(pl->d_insts, n, pl->maxN, cs);
  if (side.empty()) {
    for (size_t c = 0; c < ncls && e == hipSuccess; ++c)
      e = launch_gen(pl->d_insts, pl->classes[c].c, -1, ctx->info, cs);
    for (int g = 0; g < pl->Gmax && e == hipSuccess; ++g)
      for (size_t c = 0; c < ncls && e == hipSuccess; ++c)
        e = launch_gen(pl->d_insts, pl->classes[c].c, g, ctx->info, cs);
  } else {
    if (e == hipSuccess) e = hipEventRecord(fork, cs);
    for (size_t c = 0; c < ncls && e == hipSuccess; ++c) {
      e = hipStreamWaitEvent(side[c], fork, 0);
      if (e == hipSuccess) e = launch_gen(pl->d_insts, pl->classes[c].c, -1, ctx->info, side[c]);
      for (int g = 0; g < pl->Gmax && e == hipSuccess; ++g)
        e = launch_gen(pl->d_insts, pl->classes[c].c, g, ctx->info, side[c]);
      if (e == hipSuccess) e = hipEventRecord(join[c], side[c]);
      if (e == hipSuccess) e = hipStreamWaitEvent(cs, join[c], 0);
    }
  }
  if (e == hipSuccess) e = launch_best_batch(pl->d_insts, n, -1, cs);
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(cs, &graph);
  release_side();
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_error(e, "capturing the solve");
  }
  PTRY(e2, "hipStreamEndCapture");
  pl->graph = graph;
  PTRY(hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  *out = guard.release();
  return PA_OK;
}

// Copies best index / fitness / trace / chromosome of every instance to the
// host (after the work enqueued on s) and fills results; `gens_done` limits
// the trace (< 0: each instance's full trace).
pa_status copy_results(SolvePlan *pl, hipStream_t s, pa_result *results, int gens_done);

// Persistent launch of generations [g0, g1) of the plan's single class.
hipError_t launch_persist(SolvePlan *pl, const DeviceInfo &dev, int g0, int g1, bool best,
                          hipStream_t s) {
  hipError_t e = hipMemsetAsync(pl->d_sync, 0, sizeof(uint32_t), s);
  if (e != hipSuccess) return e;
  PersistLaunch L{};
  L.g0 = g0;
  L.g1 = g1;
  L.best = best ? 1 : 0;
  L.ninst = (int)pl->insts.size();
  L.grid = pl->pgrid;
  L.bar = pl->d_sync;
  L.err = reinterpret_cast<int32_t *>(pl->d_sync + 1);
  return launch_gen_persist(pl->d_insts, pl->classes[0].c, L, dev, nullptr, s);
}

// One-workgroup launch of generations [g0, g1) of every instance of the plan.
hipError_t launch_wg(SolvePlan *pl, int block, int g0, int g1, bool best, hipStream_t s) {
  const GenInst &I0 = pl->h_inst[0];
  return launch_gen_wg(pl->d_insts, (int)pl->insts.size(), I0.L, I0.TP, I0.se_mode, block, g0, g1,
                       best, pl->wg_maxN, pl->wg_maxK, nullptr, s);
}

// Seeding, initial population and (persistent form) the time-out flag.
hipError_t launch_start(SolvePlan *pl, hipStream_t s) {
  hipError_t e = launch_kmeans_batch(pl->d_insts, pl->d_which, pl->nwhich, s);
  if (e == hipSuccess) e = launch_init_batch(pl->d_insts, (int)pl->insts.size(), pl->maxN, s);
  if (e == hipSuccess && pl->persist) e = hipMemsetAsync(pl->d_sync, 0, 2 * sizeof(uint32_t), s);
  return e;
}

pa_status run_plan(SolvePlan *pl, const DeviceInfo &dev, hipStream_t s, pa_result *results) {
  PTRY(hipEventRecord(pl->ev0, s), "hipEventRecord");
  if (pl->wg_block) {
    PTRY(launch_start(pl, s), "launching the solve");
    PTRY(launch_wg(pl, pl->wg_block, -1, pl->Gmax, true, s), "one-workgroup solve kernel");
  } else if (pl->persist) {
    PTRY(launch_start(pl, s), "launching the solve");
    PTRY(launch_persist(pl, dev, -1, pl->Gmax, true, s), "persistent generation kernel");
  } else {
    PTRY(hipGraphLaunch(pl->exec, s), "hipGraphLaunch");
  }
  PTRY(hipEventRecord(pl->ev1, s), "hipEventRecord");
  pl->cur_gen = -1;
  pl->done_gen = pl->Gmax;
  return copy_results(pl, s, results, -1);
}

pa_status copy_results(SolvePlan *pl, hipStream_t s, pa_result *results, int gens_done) {
  const int n = (int)pl->insts.size();
  const int TG = pl->Gmax + 1;
  PTRY(hipMemcpyAsync(pl->h_idx.data(), pl->d_best_idx, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s),
       "copy results");
  PTRY(hipMemcpyAsync(pl->h_fit.data(), pl->d_best_fit, sizeof(float) * n, hipMemcpyDeviceToHost, s),
       "copy results");
  PTRY(hipMemcpyAsync(pl->h_trace.data(), pl->d_trace, sizeof(float) * n * TG, hipMemcpyDeviceToHost,
                      s),
       "copy results");
  PTRY(hipMemcpyAsync(pl->h_best.data(), pl->d_best, pl->h_best.size(), hipMemcpyDeviceToHost, s),
       "copy results");
  uint32_t sync[2] = {0, 0};
  PTRY(hipMemcpyAsync(sync, pl->d_sync, sizeof sync, hipMemcpyDeviceToHost, s), "copy results");
  PTRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (sync[1] != 0)
    return set_error(PA_EINTERNAL, "persistent solve: a grid barrier wait timed out");
  float ms = 0.0f;
  PTRY(hipEventElapsedTime(&ms, pl->ev0, pl->ev1), "hipEventElapsedTime");
  for (int i = 0; i < n; ++i) {
    pa_result &r = results[i];
    const DevProblem &p = pl->insts[i]->p;
    const size_t LK = (size_t)p.L * p.K;
    if (r.best) std::memcpy(r.best, pl->h_best.data() + pl->best_off[i], LK);
    r.best_fit = pl->h_fit[i];
    r.best_index = pl->h_idx[i];
    const int upto = gens_done < 0 ? pl->params[i].gens : std::min(gens_done, pl->params[i].gens);
    if (r.trace) std::memcpy(r.trace, pl->h_trace.data() + (size_t)i * TG, sizeof(float) * (upto + 1));
    r.device_ms = ms;
  }
  return PA_OK;
}

bool same_params(const pa_ga_params &a, const pa_ga_params &b) {
  return a.pop == b.pop && a.gens == b.gens && a.elite == b.elite && a.p_cross == b.p_cross &&
         a.p_mut == b.p_mut && a.kmeans_frac == b.kmeans_frac && a.p_init == b.p_init &&
         a.seed == b.seed && a.instance_id == b.instance_id;
}

bool plan_matches(const SolvePlan *pl, int n, pa_instance *const *insts, const pa_ga_params *params) {
  if (!pl || (int)pl->insts.size() != n) return false;
  for (int i = 0; i < n; ++i)
    if (pl->insts[i] != insts[i] || !same_params(pl->params[i], params[i])) return false;
  return true;
}

}  // namespace

pa_status check_batch(pa_context *ctx, int32_t n, pa_instance *const *insts,
                      const pa_ga_params *params) {
  if (!ctx || !insts || !params) return set_error(PA_EINVAL, "NULL argument");
  if (n < 1) return set_error(PA_EINVAL, "n=%d must be >= 1", n);
  for (int i = 0; i < n; ++i) {
    if (!insts[i]) return set_error(PA_EINVAL, "instance %d is NULL", i);
    if (insts[i]->ctx != ctx) return set_error(PA_EINVAL, "instance %d belongs to another context", i);
    for (int k = 0; k < i; ++k)
      if (insts[k] == insts[i]) return set_error(PA_EINVAL, "instance %d appears twice", i);
    pa_status st = validate_ga(insts[i], &params[i]);
    if (st != PA_OK) return set_error(st, "instance %d: %s", i, pa_last_error());
  }
  return PA_OK;
}

// Stepwise solve of a plan: seeding and initial fitness (begin), ngens more
// generations (next), best of the current populations (state).
pa_status plan_begin(SolvePlan *pl, const DeviceInfo &dev, hipStream_t s) {
  hipError_t e = launch_start(pl, s);
  if (e == hipSuccess && pl->wg_block) e = launch_wg(pl, pl->wg_block, -1, 0, false, s);
  if (e == hipSuccess && pl->persist) e = launch_persist(pl, dev, -1, 0, false, s);
  for (size_t c = 0; c < pl->classes.size() && e == hipSuccess && !pl->persist && !pl->wg_block;
       ++c)
    e = launch_gen(pl->d_insts, pl->classes[c].c, -1, dev, s);
  if (e != hipSuccess) return hip_error(e, "solve begin");
  pl->cur_gen = 0;
  pl->done_gen = 0;
  return PA_OK;
}

pa_status plan_next(SolvePlan *pl, const DeviceInfo &dev, int ngens, hipStream_t s) {
  if (!pl || pl->cur_gen < 0) return set_error(PA_EINVAL, "the stepwise solve was not begun");
  if (ngens < 0 || pl->cur_gen + ngens > pl->Gmax)
    return set_error(PA_EINVAL, "%d more generations exceed gens=%d (done %d)", ngens, pl->Gmax,
                     pl->cur_gen);
  if (pl->persist || pl->wg_block) {
    if (ngens == 0) return PA_OK;
    hipError_t e = pl->wg_block
                       ? launch_wg(pl, pl->wg_block, pl->cur_gen, pl->cur_gen + ngens, false, s)
                       : launch_persist(pl, dev, pl->cur_gen, pl->cur_gen + ngens, false, s);
    if (e != hipSuccess) return hip_error(e, "solve next");
    pl->cur_gen += ngens;
    pl->done_gen = pl->cur_gen;
    return PA_OK;
  }
  for (int k = 0; k < ngens; ++k) {
    for (size_t c = 0; c < pl->classes.size(); ++c) {
      hipError_t e = launch_gen(pl->d_insts, pl->classes[c].c, pl->cur_gen, dev, s);
      if (e != hipSuccess) return hip_error(e, "solve next");
    }
    ++pl->cur_gen;
    pl->done_gen = pl->cur_gen;
  }
  return PA_OK;
}

pa_status plan_state(SolvePlan *pl, pa_result *out, int32_t *gens_done, hipStream_t s) {
  if (!pl || pl->cur_gen < 0) return set_error(PA_EINVAL, "the stepwise solve was not begun");
  PTRY(hipEventRecord(pl->ev0, s), "hipEventRecord");
  PTRY(launch_best_batch(pl->d_insts, (int)pl->insts.size(), pl->cur_gen, s), "launch best");
  PTRY(hipEventRecord(pl->ev1, s), "hipEventRecord");
  if (gens_done) *gens_done = pl->cur_gen;
  return copy_results(pl, s, out, pl->cur_gen);
}

int gen_class_block(int L, int TP, int mode, int maxK) {
  if (!exact_variant(L, TP)) return std::max(256, (maxK + 63) / 64 * 64);
  return big_table(L, TP, mode) ? 512 : 256;
}

int gen_class_per_cu(int L, int TP, int mode, int block) {
  static std::mutex mu;
  static std::map<std::array<int, 4>, int> cache;
  const std::array<int, 4> key{L, TP, mode, block};
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  GenClass q;
  q.L = L;
  q.TP = TP;
  q.mode = mode;
  q.block = block;
  int nb = 0;
  q.query_per_cu = &nb;
  if (launch_gen(nullptr, q, 0, DeviceInfo{}, nullptr) != hipSuccess) nb = 0;
  std::lock_guard<std::mutex> lk(mu);
  cache[key] = nb;
  return nb;
}

int gen_class_grid(int L, int TP, int mode, int block, int ntasks, int cus) {
  const int per_cu = std::max(1, gen_class_per_cu(L, TP, mode, block));
  return std::max(1, std::min(ntasks, cus * per_cu));
}

namespace {
}  // namespace
}  // namespace pa

using namespace pa;

extern "C" {

pa_status pa_solve(pa_instance *in, const pa_ga_params *g, pa_result *out, void *stream) {
  if (!in || !out) return set_error(PA_EINVAL, "instance or result is NULL");
  pa_status st = validate_ga(in, g);
  if (st != PA_OK) return st;
  if ((st = use_device(in->ctx)) != PA_OK) return st;
  if (!plan_matches(in->plan, 1, &in, g)) {
    free_plan(in->plan);
    in->plan = nullptr;
    if ((st = build_plan(in->ctx, 1, &in, g, &in->plan)) != PA_OK) return st;
  }
  return run_plan(in->plan, in->ctx->info, (hipStream_t)stream, out);
}

pa_status pa_solve_batch(pa_context *ctx, int32_t n, pa_instance *const *insts,
                         const pa_ga_params *params, pa_result *results, void *stream) {
  if (!results) return set_error(PA_EINVAL, "NULL argument");
  pa_status st = check_batch(ctx, n, insts, params);
  if (st != PA_OK) return st;
  st = use_device(ctx);
  if (st != PA_OK) return st;
  if (!plan_matches(ctx->batch_plan, n, insts, params)) {
    free_plan(ctx->batch_plan);
    ctx->batch_plan = nullptr;
    if ((st = build_plan(ctx, n, insts, params, &ctx->batch_plan)) != PA_OK) return st;
  }
  return run_plan(ctx->batch_plan, ctx->info, (hipStream_t)stream, results);
}

pa_status pa_solve_begin(pa_instance *in, const pa_ga_params *g, void *stream) {
  if (!in) return set_error(PA_EINVAL, "instance is NULL");
  pa_status st = validate_ga(in, g);
  if (st != PA_OK) return st;
  if ((st = use_device(in->ctx)) != PA_OK) return st;
  if (!plan_matches(in->plan, 1, &in, g)) {
    free_plan(in->plan);
    in->plan = nullptr;
    if ((st = build_plan(in->ctx, 1, &in, g, &in->plan)) != PA_OK) return st;
  }
  return plan_begin(in->plan, in->ctx->info, (hipStream_t)stream);
}

pa_status pa_solve_next(pa_instance *in, int32_t ngens, void *stream) {
  if (!in) return set_error(PA_EINVAL, "instance is NULL");
  pa_status st = use_device(in->ctx);
  if (st != PA_OK) return st;
  return plan_next(in->plan, in->ctx->info, ngens, (hipStream_t)stream);
}

pa_status pa_solve_state(pa_instance *in, pa_result *out, int32_t *gens_done, void *stream) {
  if (!in || !out) return set_error(PA_EINVAL, "instance or result is NULL");
  pa_status st = use_device(in->ctx);
  if (st != PA_OK) return st;
  return plan_state(in->plan, out, gens_done, (hipStream_t)stream);
}

pa_status pa_solve_batch_begin(pa_context *ctx, int32_t n, pa_instance *const *insts,
                               const pa_ga_params *params, void *stream) {
  pa_status st = check_batch(ctx, n, insts, params);
  if (st != PA_OK) return st;
  if ((st = use_device(ctx)) != PA_OK) return st;
  if (!plan_matches(ctx->batch_plan, n, insts, params)) {
    free_plan(ctx->batch_plan);
    ctx->batch_plan = nullptr;
    if ((st = build_plan(ctx, n, insts, params, &ctx->batch_plan)) != PA_OK) return st;
  }
  return plan_begin(ctx->batch_plan, ctx->info, (hipStream_t)stream);
}

pa_status pa_solve_batch_next(pa_context *ctx, int32_t ngens, void *stream) {
  if (!ctx) return set_error(PA_EINVAL, "context is NULL");
  pa_status st = use_device(ctx);
  if (st != PA_OK) return st;
  return plan_next(ctx->batch_plan, ctx->info, ngens, (hipStream_t)stream);
}

pa_status pa_solve_batch_state(pa_context *ctx, pa_result *results, int32_t *gens_done,
                               void *stream) {
  if (!ctx || !results) return set_error(PA_EINVAL, "context or results is NULL");
  pa_status st = use_device(ctx);
  if (st != PA_OK) return st;
  return plan_state(ctx->batch_plan, results, gens_done, (hipStream_t)stream);
}

pa_status pa_solve_population(pa_context *ctx, pa_instance *in, int32_t index, uint8_t *pop,
                              float *fit, int32_t *gen, void *stream) {
  SolvePlan *pl = in ? in->plan : (ctx ? ctx->batch_plan : nullptr);
  if (!pl) return set_error(PA_EINVAL, "no solve plan (solve first)");
  if (pl->done_gen < 0) return set_error(PA_EINVAL, "the plan has not run");
  if (index < 0 || index >= (int)pl->insts.size())
    return set_error(PA_EINVAL, "index %d outside [0, %d)", index, (int)pl->insts.size());
  pa_status st = use_device(in ? in->ctx : ctx);
  if (st != PA_OK) return st;
  const pa_ga_params &g = pl->params[index];
  const DevProblem &p = pl->insts[index]->p;
  const int G = std::min(pl->done_gen, g.gens);
  const GenInst &I = pl->h_inst[index];
  const size_t LK = (size_t)p.L * p.K;
  hipStream_t s = (hipStream_t)stream;
  if (pop) PTRY(hipMemcpyAsync(pop, I.pop[G & 1], LK * g.pop, hipMemcpyDeviceToHost, s), "copy population");
  if (fit)
    PTRY(hipMemcpyAsync(fit, I.fit[G & 1], sizeof(float) * g.pop, hipMemcpyDeviceToHost, s),
         "copy fitness");
  PTRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (gen) *gen = G;
  return PA_OK;
}

pa_status pa_solve_resume(pa_instance *in, const pa_ga_params *g, int32_t gen, const uint8_t *pop,
                          const float *fit, const float *trace, void *stream) {
  if (!in || !pop) return set_error(PA_EINVAL, "instance or population is NULL");
  pa_status st = validate_ga(in, g);
  if (st != PA_OK) return st;
  if (gen < 0 || gen > g->gens)
    return set_error(PA_EINVAL, "gen=%d outside [0, gens=%d]", gen, g->gens);
  const int L = in->p.L, K = in->p.K, N = g->pop;
  // every row of the restored population must be a permutation of the pilots
  for (int64_t r = 0; r < (int64_t)N * L; ++r) {
    uint64_t seen = 0;
    const uint8_t *row = pop + r * K;
    for (int k = 0; k < K; ++k) {
      if (row[k] >= K || ((seen >> row[k]) & 1u))
        return set_error(PA_EINVAL, "chromosome %lld, cell %lld is not a permutation of 0..%d",
                         (long long)(r / L), (long long)(r % L), K - 1);
      seen |= uint64_t(1) << row[k];
    }
  }
  if ((st = use_device(in->ctx)) != PA_OK) return st;
  if (!plan_matches(in->plan, 1, &in, g)) {
    free_plan(in->plan);
    in->plan = nullptr;
    if ((st = build_plan(in->ctx, 1, &in, g, &in->plan)) != PA_OK) return st;
  }
  SolvePlan *pl = in->plan;
  const GenInst &I = pl->h_inst[0];
  hipStream_t s = (hipStream_t)stream;
  const size_t LK = (size_t)L * K;
  // the generation's buffers of the double-buffered population and fitness
  PTRY(hipMemcpyAsync(I.pop[gen & 1], pop, LK * N, hipMemcpyHostToDevice, s), "copy population");
  if (fit) {
    PTRY(hipMemcpyAsync(I.fit[gen & 1], fit, sizeof(float) * N, hipMemcpyHostToDevice, s),
         "copy fitness");
  } else {
    // recomputed: the same bits as the fitness the solve computed
    if ((st = pa_fitness(in, I.pop[gen & 1], N, I.fit[gen & 1], stream)) != PA_OK) return st;
  }
  // trace entries before gen from the caller (NaN without one); entry gen
  // and later are written by the generations and the state call to come
  std::vector<float> tr((size_t)pl->Gmax + 1, std::numeric_limits<float>::quiet_NaN());
  if (trace) std::memcpy(tr.data(), trace, sizeof(float) * gen);
  PTRY(hipMemcpyAsync(I.trace, tr.data(), sizeof(float) * tr.size(), hipMemcpyHostToDevice, s),
       "copy trace");
  if (pl->persist) PTRY(hipMemsetAsync(pl->d_sync, 0, 2 * sizeof(uint32_t), s), "hipMemsetAsync");
  PTRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  pl->cur_gen = gen;
  pl->done_gen = gen;
  return PA_OK;
}

pa_status pa_solve_shape(pa_context *ctx, pa_instance *in, int32_t *persistent, int32_t *block,
                         int32_t *children_per_task, int32_t *workgroups) {
  const SolvePlan *pl = in ? in->plan : (ctx ? ctx->batch_plan : nullptr);
  if (!pl) return set_error(PA_EINVAL, "no solve plan (solve first)");
  if (pl->wg_block) {
    if (persistent) *persistent = 2;
    if (block) *block = pl->wg_block;
    if (children_per_task) *children_per_task = pl->params[0].pop - pl->params[0].elite;
    if (workgroups) *workgroups = (int32_t)pl->insts.size();
    return PA_OK;
  }
  const PlanClass &pc = pl->classes[0];
  const int K = pl->insts[0]->p.K;
  if (persistent) *persistent = pl->persist ? 1 : 0;
  if (block) *block = pc.c.block;
  if (children_per_task) *children_per_task = std::max(1, (pc.c.block / K + pc.cpt_div - 1) / pc.cpt_div);
  if (workgroups) *workgroups = pl->persist ? pl->pgrid : pc.c.grid;
  return PA_OK;
}

}  // extern "C"
