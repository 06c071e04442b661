// k_gen_L19.hip -- unrolled generation kernels (per-generation and persistent
// forms) for L = 19 cells, one translation unit per cell count so the
// variants compile in parallel.
#include "gen_core.h"

namespace pa {
hipError_t gen_dispatch_L19(const GenInst *insts, const GenClass &c, int gen, hipStream_t s,
                           bool *handled, const PersistCall *pc) {
  return gen_dispatch_L<19>(insts, c, gen, s, handled, pc);
}
}  // namespace pa
