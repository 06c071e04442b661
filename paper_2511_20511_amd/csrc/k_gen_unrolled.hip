// k_gen_unrolled.hip -- the unrolled generation kernels of one cell count,
// SE mode and form (per-generation or persistent).  The build compiles this
// file once per (PA_GEN_L, PA_GEN_MODE, PA_GEN_FORM) so that the variants
// compile in parallel; each object defines the one dispatch function
// gen_dispatch_L<L>_m<mode>_<form> declared in gen_core.h (form x: one
// launch per generation, p: the persistent kernel).
#include "gen_core.h"

#if !defined(PA_GEN_L) || !defined(PA_GEN_MODE) || !defined(PA_GEN_FORM) || \
    !defined(PA_GEN_PERSIST)
#error "compile with -DPA_GEN_L=<7|19|37> -DPA_GEN_MODE=<0|1> -DPA_GEN_FORM=<x|p> -DPA_GEN_PERSIST=<0|1>"
#endif

#define PA_CAT(a, b) a##b
#define PA_XCAT(a, b) PA_CAT(a, b)
#define PA_GEN_NAME \
  PA_XCAT(PA_XCAT(PA_XCAT(PA_XCAT(gen_dispatch_L, PA_GEN_L), _m), PA_GEN_MODE), PA_XCAT(_, PA_GEN_FORM))

namespace pa {
hipError_t PA_GEN_NAME(const GenInst *insts, const GenClass &c, int gen, hipStream_t s,
                       bool *handled, const PersistCall *pc) {
  return gen_dispatch_unrolled<PA_GEN_L, PA_GEN_MODE, PA_GEN_PERSIST != 0>(insts, c, gen, s,
                                                                          handled, pc);
}
}  // namespace pa
