// The batched star kernel and its launch templates, shared by the
// translation units that instantiate it for the table layouts (split so the
// instantiations compile in parallel).
#pragma once

#include "star_common.h"

namespace oss {

// STAGED (planar layouts): per radius the wave first looks up the first
// quantity alone and tests it against the hull; the other quantities are
// looked up only where it lies inside (the plain screen's staged form).

template <typename Tab, int MT, bool RINGS, bool STAGED>
__global__ __launch_bounds__(STAR_MAX_THREADS) void star_batch_kernel(
    const void *__restrict__ L, const void *__restrict__ R, const void *__restrict__ Rp,
    int64_t pitch_e, int64_t plane, int H, int W, const DevBatchPass *__restrict__ passes,
    int n_passes,
    const DevBatchGroup *__restrict__ groups, const DevBatchRadius *__restrict__ radii,
    const DevBatchProbe *__restrict__ probes, const uint32_t *__restrict__ core_bits,
    uint8_t *const *__restrict__ mask_of, EmitOut eo, StarSweep sw)
{
    constexpr int NQ = Tab::NQ;
    constexpr int64_t ES = Tab::ES;
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int units = (sw.n_units - xcd + 7) / 8;
    const int items = units * sw.rows_per_part;
    const uint32_t lane_off = (uint32_t)((threadIdx.x + 1) * ES);
    const int64_t row_bytes = pitch_e * ES;
    const int64_t hw = (int64_t)H * W;
    const TabBases tb{static_cast<const char *>(L), static_cast<const char *>(R),
                      static_cast<const char *>(Rp)};
    for (int ip = 0; ip < n_passes; ++ip) {
        const DevBatchPass ps = passes[ip];
        const DevBatchGroup *grp = groups + ps.group;
        const int nt = grp->n_t;
        for (int it = j; it < items; it += sw.blocks_per_xcd) {
            int y, x0;
            sweep_item(sw, xcd, it, (int)blockDim.x, &y, &x0);
            if (y >= H)
                continue;
            const int x = x0 + threadIdx.x;
            const char *Lb = reinterpret_cast<const char *>(L) + (int64_t)x0 * ES;
            const char *Rb = reinterpret_cast<const char *>(R) + (int64_t)x0 * ES;
            const char *Rpb = reinterpret_cast<const char *>(Rp) + (int64_t)x0 * ES;
            // table row y (image row y - 1) of each table at the strip
            const int64_t yrow = (int64_t)y * row_bytes;
            const char *Ly = Lb + yrow, *Ry = Rb + yrow, *Rpy = Rpb + yrow;
            // Scale bits per template slot: whose own star passes (acc) and
            // which a central star fails (fail).  An array indexed by the
            // wave-uniform slot stays in registers up to 32 entries, so a
            // group of 64 (no rings) keeps a second half, picked by a
            // uniform branch.
            static_assert(!RINGS || MT <= 32, "groups with rings hold at most 32 templates");
            uint32_t acc[MT > 32 ? 32 : MT];
            uint32_t acc_hi[MT > 32 ? MT - 32 : 1];
            uint32_t fail[RINGS ? MT : 1];
#pragma unroll
            for (int t = 0; t < (MT > 32 ? 32 : MT); ++t) {
                acc[t] = 0;
                if constexpr (RINGS)
                    fail[t] = 0;
            }
#pragma unroll
            for (int t = 0; t < (MT > 32 ? MT - 32 : 1); ++t)
                acc_hi[t] = 0;
            for (int jr = ps.j0; jr < ps.j1; ++jr) {
                const DevBatchRadius &rd = radii[jr];
                const int r = rd.r, s = rd.s;
                if (y < r || y > H - 1 - r)
                    continue;
                const bool xv = x >= r && x <= W - 1 - r;
                if constexpr (RINGS) {
                    // skip the radius where every probe it serves has failed a
                    // central star already (its bit is then 0 whatever this
                    // radius gives); radii ascend, so a probe's central stars,
                    // smaller than its own, come first
                    bool need = false;
                    if (xv)
                        for (int p = rd.first; p < rd.first + rd.count; ++p) {
                            const DevBatchProbe &pr = probes[p];
                            need = need | !((fail[pr.t] >> pr.k) & 1u);
                        }
                    if (__builtin_amdgcn_ballot_w64(need) == 0)
                        continue;
                }
                // a valid position outside the radius' hull fails every entry
                // of the radius: central-star entries record that failure
                auto fail_all = [&]() {
                    if constexpr (RINGS) {
                        if (xv)
                            for (int p = rd.first; p < rd.first + rd.count; ++p) {
                                const DevBatchProbe &pr = probes[p];
                                if (pr.ring)
                                    fail[pr.t] |= 1u << pr.k;
                            }
                    }
                };
                int64_t F[NQ];
                bool in = false;  // inside the radius' hull
                if constexpr (STAGED && Tab::STAGE && NQ > 1) {
                    constexpr int C = Tab::C;
                    const StarAddr ad = star_addr_rows<Tab>(Ly, Ry, Rpy, rd.roff, lane_off, r, s);
                    bool in_c = false;
                    if (xv) {
                        F[C] = star_sum_c<Tab>(ad, plane);
                        in_c = (F[C] >= rd.lo[C]) & (F[C] <= rd.hi[C]);
                    }
                    if (__builtin_amdgcn_ballot_w64(in_c) == 0) {
                        fail_all();
                        continue;
                    }
                    if (in_c)
                        star_sums_rest<Tab>(ad, tb, plane, F);
                    in = in_c;
                    if (in_c) {
#pragma unroll
                        for (int q = 0; q < NQ; ++q)
                            in = in & (F[q] >= rd.lo[q]) & (F[q] <= rd.hi[q]);
                    }
                    if (__builtin_amdgcn_ballot_w64(in) == 0 || !in) {
                        fail_all();
                        continue;
                    }
                } else {
                    in = xv;
                    if (xv) {
                        star_sums_at<Tab>(star_addr_rows<Tab>(Ly, Ry, Rpy, rd.roff, lane_off, r, s),
                                          tb, F, plane);
#pragma unroll
                        for (int q = 0; q < NQ; ++q)
                            in = in & (F[q] >= rd.lo[q]) & (F[q] <= rd.hi[q]);
                    }
                    // skip the probe loop when no lane of the wave lies in the hull
                    if (__builtin_amdgcn_ballot_w64(in) == 0 || !in) {
                        fail_all();
                        continue;
                    }
                }
                // every hull lane of the wave inside the core passes every
                // probe of the radius.  Up to 16 slots: the radius' bits per
                // slot at once, from the core words.  Larger groups skip the
                // probes' compares inside the one probe loop instead: a second
                // site updating their accumulators held a second copy of them
                // in registers (64 more for 64 slots: half the occupancy).
                bool core_all = false;
                if constexpr (!RINGS) {
                    if (rd.cb_first >= 0) {
                        bool inc = in;
#pragma unroll
                        for (int q = 0; q < NQ; ++q)
                            inc = inc & (F[q] >= rd.clo[q]) & (F[q] <= rd.chi[q]);
                        core_all = __builtin_amdgcn_ballot_w64(in && !inc) == 0;
                        if (MT <= 16 && core_all) {
                            const uint32_t *cb = core_bits + rd.cb_first;
#pragma unroll
                            for (int t = 0; t < MT; ++t) {
                                if (t < nt) {
                                    const uint32_t b = inc ? cb[t] : 0u;
                                    if (t < 32)
                                        acc[t < 32 ? t : 0] |= b;
                                    else
                                        acc_hi[t >= 32 ? t - 32 : 0] |= b;
                                }
                            }
                            continue;
                        }
                    }
                }
                {
                    for (int p = rd.first; p < rd.first + rd.count; ++p) {
                        const DevBatchProbe pr = probes[p];
                        bool pass = in;
                        if (!core_all) {
#pragma unroll
                            for (int q = 0; q < NQ; ++q)
                                pass = pass & (F[q] >= pr.lo[q]) & (F[q] <= pr.hi[q]);
                        }
                        const uint32_t bit = pass ? (1u << pr.k) : 0u;
                        if constexpr (RINGS) {
                            if (pr.ring)
                                fail[pr.t] |= pass ? 0u : (1u << pr.k);
                            else
                                acc[pr.t] |= bit;
                        } else if constexpr (MT > 32) {
                            if (pr.t < 32)
                                acc[pr.t] |= bit;
                            else
                                acc_hi[pr.t - 32] |= bit;
                        } else {
                            acc[pr.t] |= bit;
                        }
                    }
                }
            }
            // the pass's scale bits per slot, with the bits carried in from
            // the group's earlier passes; a group's last pass emits them
            // (mask, segment counts, staged candidates), an earlier pass
            // carries them on in scale-bit words.  (No lambda reads the
            // accumulators: one capturing them by reference put them in
            // scratch memory in the ring kernels.)
            EmitRow er;
            const bool emit = ps.last && emit_begin(eo, y, x, &er);
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                if (t < nt) {
                    uint32_t v = t < 32 ? acc[t < 32 ? t : 0] : acc_hi[t >= 32 ? t - 32 : 0];
                    if constexpr (RINGS)
                        v &= ~fail[t];  // one pass per group: final here
                    const int tg = grp->tmap[t];
                    const int64_t wi = (int64_t)tg * hw + (int64_t)y * W + x;
                    if (!ps.first && x < W)
                        v |= eo.dense[wi];
                    if (!ps.last && x < W)
                        eo.dense[wi] = v;
                    if (emit)
                        emit_slot(eo, er, y, x, v, tg, mask_of ? mask_of[tg] : nullptr);
                }
            }
        }
    }
}

template <typename Tab, bool STAGED>
inline void batch_launch_s(const BuildGeom &g, const void *L, const void *R, const void *Rp,
                           const BatchDevPlan &bp, const EmitOut &eo, const StarSweep &sw,
                           hipStream_t st)
{
#define OSS_BATCH_LAUNCH(MT, RINGS)                                                               \
    do {                                                                                          \
        auto *k = &star_batch_kernel<Tab, MT, RINGS, STAGED>;                                     \
        const StarSweep rs = resident_sweep(reinterpret_cast<const void *>(k), sw, 0);            \
        hipLaunchKernelGGL(k, dim3(8 * rs.blocks_per_xcd), dim3(rs.strip), 0, st, L, R, Rp,       \
                           g.pitch_e, g.plane, g.H, g.W, bp.passes, bp.n_passes, bp.groups,        \
                           bp.radii, bp.probes, bp.core_bits, bp.mask_of, eo, rs);                \
    } while (0)
    if (bp.rings > 1) {
        if (bp.max_group <= 8)
            OSS_BATCH_LAUNCH(8, true);
        else
            OSS_BATCH_LAUNCH(32, true);
    } else if (bp.max_group <= 8) {
        OSS_BATCH_LAUNCH(8, false);
    } else if (bp.max_group <= 16) {
        OSS_BATCH_LAUNCH(16, false);
    } else if (bp.max_group <= 32) {
        OSS_BATCH_LAUNCH(32, false);
    } else {
        OSS_BATCH_LAUNCH(64, false);
    }
#undef OSS_BATCH_LAUNCH
}

template <typename Tab>
inline void batch_launch(const BuildGeom &g, const void *L, const void *R, const void *Rp,
                         const BatchDevPlan &bp, const EmitOut &eo, const StarSweep &sw, bool staged,
                         hipStream_t st)
{
    if (staged && Tab::STAGE)
        batch_launch_s<Tab, true>(g, L, R, Rp, bp, eo, sw, st);
    else
        batch_launch_s<Tab, false>(g, L, R, Rp, bp, eo, sw, st);
}

template <typename T>
inline hipError_t batch_t(const BuildGeom &g, const void *L, const void *R, const void *Rp,
                          const BatchDevPlan &bp, const EmitOut &eo, const StarSweep &sw,
                          bool staged, hipStream_t st)
{
    if (g.planar) {
        switch (g.nq) {
        case 1: batch_launch<TabP<T, 1>>(g, L, R, Rp, bp, eo, sw, staged, st); break;
        case 2: batch_launch<TabP<T, 2>>(g, L, R, Rp, bp, eo, sw, staged, st); break;
        case 3: batch_launch<TabP<T, 3>>(g, L, R, Rp, bp, eo, sw, staged, st); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (g.nq) {
    case 1: batch_launch<TabU<T, 1>>(g, L, R, Rp, bp, eo, sw, staged, st); break;
    case 2: batch_launch<TabU<T, 2>>(g, L, R, Rp, bp, eo, sw, staged, st); break;
    case 3: batch_launch<TabU<T, 3>>(g, L, R, Rp, bp, eo, sw, staged, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}


// Per-layout launchers, one translation unit each.
hipError_t batch_p32(const BuildGeom &g, const void *L, const void *R, const void *Rp,
                     const BatchDevPlan &bp, const EmitOut &eo, const StarSweep &sw, bool staged,
                     hipStream_t st);
hipError_t batch_p64(const BuildGeom &g, const void *L, const void *R, const void *Rp,
                     const BatchDevPlan &bp, const EmitOut &eo, const StarSweep &sw, bool staged,
                     hipStream_t st);
hipError_t batch_mix(const BuildGeom &g, const void *L, const void *R, const void *Rp,
                     const BatchDevPlan &bp, const EmitOut &eo, const StarSweep &sw, bool staged,
                     hipStream_t st);

}  // namespace oss
