// k_gen.hip -- runtime-L generation kernels and the dispatch of a class of
// instances to the unrolled (k_gen_L*.hip) or runtime-L variant.
#include "gen_core.h"

namespace pa {

namespace {

template <int LMAX, int MODE>
hipError_t gen_launch_generic(const GenInst *insts, const GenClass &c, int gen, hipStream_t s) {
  const int n = gen < 0 ? c.neval : c.ntasks;
  const int block = c.block;
  const int L = c.L, TP = c.TP;
  const int child = (block * L + 15) / 16 * 16;
  const int eb = block * 4, idxb = 256, selb = block * 8;
  const int row_bytes = L * TP * 4 * (MODE == 1 ? 2 : 1);
  const int budget = kLdsBytes - 2 * child - eb - idxb - selb - 256;
  const int max_rows = budget / row_bytes;
  if (max_rows < 1) return hipErrorInvalidValue;
  const int tiles = (L + max_rows - 1) / max_rows;
  GenGenericPlan pl;
  pl.tile_rows = (L + tiles - 1) / tiles;
  pl.child_off = pl.tile_rows * row_bytes;
  pl.inv_off = pl.child_off + child;
  pl.e_off = pl.inv_off + child;
  pl.idx_off = pl.e_off + eb;
  pl.sel_off = pl.idx_off + idxb;
  const int total = pl.sel_off + selb;
  auto kern = k_gen_generic<LMAX, MODE>;
  static LdsAttr attr;
  const hipError_t ae = allow_lds_once(attr, reinterpret_cast<const void *>(kern), kLdsBytes);
  if (c.query_per_cu)
    return per_cu_query(reinterpret_cast<const void *>(kern), block, total, c.query_per_cu);
  if (n <= 0) return hipSuccess;
  const int grid = c.grid < 1 ? 1 : (c.grid > n ? n : c.grid);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(block), total, s, gen_args(insts, c, gen), pl);
  return launch_status(ae);
}

template <int MODE>
hipError_t gen_generic_mode(const GenInst *insts, const GenClass &c, int gen, hipStream_t s) {
  if (c.L <= 8) return gen_launch_generic<8, MODE>(insts, c, gen, s);
  if (c.L <= 16) return gen_launch_generic<16, MODE>(insts, c, gen, s);
  if (c.L <= 32) return gen_launch_generic<32, MODE>(insts, c, gen, s);
  return gen_launch_generic<64, MODE>(insts, c, gen, s);
}

}  // namespace

hipError_t gen_dispatch_generic(const GenInst *insts, const GenClass &c, int gen, hipStream_t s) {
  return c.mode == 1 ? gen_generic_mode<1>(insts, c, gen, s) : gen_generic_mode<0>(insts, c, gen, s);
}

int gen_default_block(int L, int TP, int mode) {
  const bool exact = (L == 7 || L == 19 || L == 37) && TP <= 32;
  const long table = (long)L * L * TP * 4 * (mode == 1 ? 2 : 1);
  if (!exact) return 256;
  return table <= 40 * 1024 ? 256 : 512;
}

int gen_children_per_task(int L, int K, int TP, int mode, int block) {
  (void)L;
  (void)TP;
  (void)mode;
  return block / K;
}

// The unrolled variant of (L, SE mode, form), or null when there is none.
GenDispatchFn unrolled_fn(int L, int mode, bool persist) {
  static const GenDispatchFn table[3][2][2] = {
      {{gen_dispatch_L7_m0_x, gen_dispatch_L7_m0_p}, {gen_dispatch_L7_m1_x, gen_dispatch_L7_m1_p}},
      {{gen_dispatch_L19_m0_x, gen_dispatch_L19_m0_p},
       {gen_dispatch_L19_m1_x, gen_dispatch_L19_m1_p}},
      {{gen_dispatch_L37_m0_x, gen_dispatch_L37_m0_p},
       {gen_dispatch_L37_m1_x, gen_dispatch_L37_m1_p}}};
  const int li = L == 7 ? 0 : L == 19 ? 1 : L == 37 ? 2 : -1;
  if (li < 0 || mode < 0 || mode > 1) return nullptr;
  return table[li][mode][persist ? 1 : 0];
}

hipError_t launch_gen(const GenInst *insts, const GenClass &c, int gen, const DeviceInfo &dev,
                      hipStream_t s) {
  (void)dev;
  bool handled = false;
  hipError_t e = hipSuccess;
  if (const GenDispatchFn fn = unrolled_fn(c.L, c.mode, false))
    e = fn(insts, c, gen, s, &handled, nullptr);
  if (handled) return e;
  return gen_dispatch_generic(insts, c, gen, s);
}

hipError_t launch_gen_persist(const GenInst *insts, const GenClass &c, const PersistLaunch &pl,
                              const DeviceInfo &dev, int *capacity, hipStream_t s) {
  PersistCall pc;
  pc.args.insts = insts;
  pc.args.tasks = c.tasks;
  pc.args.ntasks = c.ntasks;
  pc.args.chunk = (c.ntasks + pl.grid - 1) / (pl.grid > 0 ? pl.grid : 1);
  pc.args.evals = c.eval_tasks;
  pc.args.neval = c.neval;
  pc.args.echunk = (c.neval + pl.grid - 1) / (pl.grid > 0 ? pl.grid : 1);
  pc.args.g0 = pl.g0;
  pc.args.g1 = pl.g1;
  pc.args.best = pl.best;
  pc.args.ninst = pl.ninst;
  pc.args.bar = pl.bar;
  pc.args.err = pl.err;
  pc.grid = pl.grid;
  pc.cus = dev.cus;
  pc.capacity = capacity;
  if (capacity) *capacity = 0;
  bool handled = false;
  hipError_t e = hipSuccess;
  if (const GenDispatchFn fn = unrolled_fn(c.L, c.mode, true))
    e = fn(insts, c, 0, s, &handled, &pc);
  if (!handled) return capacity ? hipSuccess : hipErrorNotSupported;
  return e;
}

}  // namespace pa
