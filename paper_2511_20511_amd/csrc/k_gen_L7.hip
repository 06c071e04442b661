// k_gen_L7.hip -- unrolled generation kernels (per-generation and persistent
// forms) for L = 7 cells, one translation unit per cell count so the
// variants compile in parallel.
#include "gen_core.h"

namespace pa {
hipError_t gen_dispatch_L7(const GenInst *insts, const GenClass &c, int gen, hipStream_t s,
                           bool *handled, const PersistCall *pc) {
  return gen_dispatch_L<7>(insts, c, gen, s, handled, pc);
}
}  // namespace pa
