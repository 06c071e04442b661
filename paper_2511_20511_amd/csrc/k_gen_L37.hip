// k_gen_L37.hip -- unrolled generation kernels (per-generation and persistent
// forms) for L = 37 cells, one translation unit per cell count so the
// variants compile in parallel.
#include "gen_core.h"

namespace pa {
hipError_t gen_dispatch_L37(const GenInst *insts, const GenClass &c, int gen, hipStream_t s,
                           bool *handled, const PersistCall *pc) {
  return gen_dispatch_L<37>(insts, c, gen, s, handled, pc);
}
}  // namespace pa
