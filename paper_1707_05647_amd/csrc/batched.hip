// Batched screen: every probe of every template in one persistent launch
// over one reference's tables (Algorithm 1's patch loop for all templates
// and scales at once).  With central-star rings (Sec. "Scale Invariance",
// central areas of sizes n, n/lambda, n/lambda^2) each probe also has
// entries at its central radii; a probe's bit survives where its own star
// passes and none of its central stars fails.  A wave skips a radius whose
// probes have all failed a central star at each of its positions.
//
// Templates are sorted by radius and cut into groups of at most
// BATCH_GROUP; within a group the probes are grouped by reference radius, so
// the star features of a radius are computed once per position and
// compared against every probe of every template of the group at that
// radius.  The scale bits of the group's templates live in registers
// (indexed by the probe's uniform template slot).  Each radius also carries
// the hull of its entries' intervals: a position outside it fails every
// entry, so it skips the probe loop (central-star entries record the
// failure), and a wave with no position inside skips the loop altogether.
//
// A group's distinct radii are split into buckets of consecutive radii.
// A pass = (group, bucket); the launch walks all passes in order, each pass a
// full sweep of the image with the plain kernel's persistent XCD-aware strip
// schedule.  A bucket of nearby radii only touches table rows near y +- r
// for its radii, which keeps an XCD's L2 footprint small when the radius
// range is wide.  A group with several passes carries its scale bits from
// pass to pass in scale-bit words (the first pass writes them, later passes
// OR into them); every pass assigns the same positions to the same block and
// thread, so each word is only ever read and written by one thread, in pass
// order.  The group's last pass (the only one, without buckets) emits the
// final bits: the mask, the segment counts and the staged candidates, from
// which the list pass builds the candidate list.
#include "batched_kernel.h"

namespace oss {

hipError_t batch_mix(const BuildGeom &g, const void *L, const void *R, const void *Rp,
                            const BatchDevPlan &bp, const EmitOut &eo, const StarSweep &sw,
                            bool staged, hipStream_t st)
{
    if (g.planar) {
        if (g.rec)
            batch_launch<TabPR>(g, L, R, Rp, bp, eo, sw, staged, st);
        else if (g.nq == 3 && g.sqi == 1)
            batch_launch<TabPS<3, 1>>(g, L, R, Rp, bp, eo, sw, staged, st);
        else if (g.nq == 2 && g.sqi == 1)
            batch_launch<TabPS<2, 1>>(g, L, R, Rp, bp, eo, sw, staged, st);
        else if (g.nq == 2 && g.sqi == 0)
            batch_launch<TabPS<2, 0>>(g, L, R, Rp, bp, eo, sw, staged, st);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    if (g.nq == 3 && g.sqi == 1)
        batch_launch<TabMix<3, 1>>(g, L, R, Rp, bp, eo, sw, staged, st);
    else if (g.nq == 2 && g.sqi == 1)
        batch_launch<TabMix<2, 1>>(g, L, R, Rp, bp, eo, sw, staged, st);
    else if (g.nq == 2 && g.sqi == 0)
        batch_launch<TabMix<2, 0>>(g, L, R, Rp, bp, eo, sw, staged, st);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_star_batch(const BuildGeom &g, const void *L, const void *R, const void *Rp,
                             const BatchDevPlan &bp, const EmitOut &eo, const StarSweep &sw,
                             bool staged, hipStream_t stream, Profiler *prof)
{
    if (sw.strip < 64 || sw.strip > STAR_MAX_THREADS || sw.strip % 64 || sw.blocks_per_xcd < 1 ||
        bp.max_group > (bp.rings > 1 ? BATCH_GROUP_RINGS : BATCH_GROUP))
        return hipErrorInvalidValue;
    if (!emit_ok(eo, g))
        return hipErrorInvalidValue;
    ProfScope ps(prof, K_STAR_BATCH, stream);
    if (g.sqi >= 0)
        return batch_mix(g, L, R, Rp, bp, eo, sw, staged, stream);
    if (g.ebytes == 4)
        return batch_p32(g, L, R, Rp, bp, eo, sw, staged, stream);
    return batch_p64(g, L, R, Rp, bp, eo, sw, staged, stream);
}

}  // namespace oss
