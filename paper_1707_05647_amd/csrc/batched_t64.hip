// Batched star kernel instantiated for uint64-bit table values (planar
// and interleaved layouts); see batched.hip.
#include "batched_kernel.h"

namespace oss {

hipError_t batch_p64(const BuildGeom &g, const void *L, const void *R, const void *Rp,
                     const BatchDevPlan &bp, const EmitOut &eo, const StarSweep &sw, bool staged,
                     hipStream_t st)
{
    return batch_t<uint64_t>(g, L, R, Rp, bp, eo, sw, staged, st);
}

}  // namespace oss
