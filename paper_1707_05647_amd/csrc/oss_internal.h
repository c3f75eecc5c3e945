// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/oss.h"

namespace oss {

// ---------------------------------------------------------------------------
// Builder geometry.
//
// The tables are built in row bands of KBAND rows.  Band b covers image rows
// y in [y_s, y_s + rows) with y_s = -1 + b * KBAND (row -1 is the all-zero
// leading row).  Within a band every table follows a one-row recurrence on
// the row prefix P_y(x) = sum_{i<=x} q(i, y):
//     L(x,y)    = L(x, y-1)      + P_y(x)
//     T_ad(x,y) = T_ad(x+1, y-1) + P_y(x)      (anti-diagonal carry)
//     T_d(x,y)  = T_d(x-1, y-1)  + P_y(x)      (diagonal carry)
//     R(x,y)    = T_ad(x,y) - T_d(x-1,y),   R'(x,y) = T_ad(x+1,y) - T_d(x-1,y)
// The carries entering a band (the three tables at row y_s - 1) are found in
// three steps: a zero-carry pass gives each band's own contribution, a line
// walk across bands accumulates them, and the final pass starts from them.
// Carry arrays span x in [CX0, CX1] = [-2-KBAND, W+KBAND].
// ---------------------------------------------------------------------------
constexpr int KBAND = 32;          // rows per band
constexpr int BAND_THREADS = 512;  // threads (= columns) per band tile
constexpr int BAND_HALO = KBAND + 1;
constexpr int BAND_CORE_MAX = BAND_THREADS - 2 * BAND_HALO;  // 446 columns

struct BuildGeom {
    int H, W, nq;
    int64_t pitch_e;   // table entries per row (>= W+1)
    int nb;            // bands
    int cx0, cw;       // carry range start (-2-K) and width (W+2K+3)
    int nch_agg, wc_agg;   // zero-carry pass: chunk count and core width over [cx0, cx0+cw)
    int nch_fin, wc_fin;   // final pass: chunk count and core width over [-1, W-1]
};

BuildGeom make_geom(int H, int W, int nq);

// ---------------------------------------------------------------------------
// Screening plan uploaded per call.
// ---------------------------------------------------------------------------
struct DevProbe {
    int64_t lo[3];   // inclusive bounds on the feature sums at radius r
    int64_t hi[3];
    int32_t k;       // scale bit
    int32_t pad;
};

struct DevRadius {
    int32_t r, s;        // star radius and square half-width
    int32_t first, count;  // probes [first, first + count) in the template's probe array
};

struct DevTemplatePlan {
    int32_t n_radii;
    int32_t pad;
    DevRadius radii[OSS_MAX_SCALES];
    DevProbe probes[OSS_MAX_SCALES];
};

// exact bounds: F passes feature f of a probe iff lo <= F <= hi
void feature_bounds(int f, int64_t FT, int r, int rho, int P, int Q, int64_t *lo, int64_t *hi);

int square_half(int r);
int64_t star_area(int r);

// ---------------------------------------------------------------------------
// Per-kernel timing with HIP events recorded on the launch stream.
// ---------------------------------------------------------------------------
enum KernelId {
    K_ROW_BASE,
    K_BAND_AGG,
    K_CARRY,
    K_BAND_FINAL,
    K_STAR,
    K_COMPACT_COUNT,
    K_COMPACT_SCAN,
    K_COMPACT_WRITE,
    K_COUNT
};
extern const char *const kKernelNames[K_COUNT];

struct Profiler {
    bool on = false;
    struct Rec {
        int id;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    int64_t launches[K_COUNT] = {};
    double total_ms[K_COUNT] = {};
    double max_ms[K_COUNT] = {};
    void clear();
    hipError_t resolve();  // waits for the recorded events and accumulates
    ~Profiler();
};

// Records a start event on construction and a stop event on destruction
// when profiling is on.
struct ProfScope {
    Profiler *p;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    int id;
    ProfScope(Profiler *p_, int id_, hipStream_t st_);
    ~ProfScope();
};

// ---------------------------------------------------------------------------
// Kernel launchers (asynchronous, on `stream`).
// ---------------------------------------------------------------------------
struct BuildBuffers {
    int64_t *L, *R, *Rp;          // tables
    int64_t *bp_agg, *bp_fin;     // [H][nch][nq] row-prefix bases
    int64_t *agg_L, *agg_AD, *agg_D;  // [nb][cw][nq]
    int64_t *c_L, *c_AD, *c_D;        // [nb][cw][nq]
};

hipError_t launch_build(const BuildGeom &g, const void *pixels, int64_t pitch_bytes, int dtype,
                        uint32_t feat_mask, const BuildBuffers &bb, hipStream_t stream,
                        Profiler *prof);

hipError_t launch_star_plain(const BuildGeom &g, const int64_t *L, const int64_t *R,
                             const int64_t *Rp, const DevTemplatePlan *plan, uint32_t *bits,
                             hipStream_t stream, Profiler *prof);

// compaction over n = n_tmpl * H * W scale-bit words in (t, y, x) order
size_t compact_workspace_bytes(int64_t n);
hipError_t launch_compact(const uint32_t *bits, int64_t n_tmpl, int H, int W, uint8_t *mask,
                          oss_candidate *list, int64_t list_cap, int64_t *count, void *workspace,
                          hipStream_t stream, Profiler *prof);

}  // namespace oss
