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
// The carries entering a band (the three tables at row y_s - 1) come from a
// projection pass (each band's own contribution), a line walk across bands
// and are consumed by the final pass.
//
// Band tiles are 512 threads wide, one column per thread; a tile whose
// threads start at column X0 (a multiple of 64) owns the core columns
// [X0 + BAND_HALO, X0 + BAND_HALO + BAND_STRIDE - 1]; consecutive tiles are
// BAND_STRIDE apart.  The halos absorb the one-column-per-row drift of the
// diagonal carries.  Row prefixes enter a tile through its base
// P_y(X0 - 1), taken from the per-row prefix at every 64th column.
// ---------------------------------------------------------------------------
constexpr int KBAND = 30;          // rows per band
constexpr int BAND_THREADS = 512;  // threads (= columns) per band tile
constexpr int BAND_HALO = KBAND + 1;
constexpr int BAND_STRIDE = 448;   // core width, a multiple of 64
static_assert(BAND_HALO + BAND_STRIDE + BAND_HALO <= BAND_THREADS, "tile too narrow");
static_assert(BAND_STRIDE % 64 == 0, "tile starts must stay 64-aligned");

struct BuildGeom {
    int H, W, nq;
    int ebytes;        // bytes per accumulated quantity: 4 (mod 2^32) or 8
    int sqi;           // mixed entries: slot of the squares among the quantities, else -1
    int planar;        // 1: one plane per quantity (entry stride ebytes; 4 with sqi >= 0)
    int tab_es;        // entry stride in bytes: nq * ebytes, 16 (mixed) or ebytes (planar)
    int64_t plane;     // planar: bytes from one plane to the next, else 0
    int64_t tab_bytes; // bytes of one table
    int tab_off;       // bytes from a table's (plane's) allocation start to entry 0
    int64_t pitch_e;   // table entries per row (>= W+1)
    int nb;            // bands
    int nfin, fin_x0;  // final tiles: first thread column of tile c is fin_x0 + c*BAND_STRIDE
    int nagg, agg_x0;  // projection tiles
    int cx0, cw;       // carry range [cx0, cx0 + cw): the union of the final tiles' columns
    int nbp;           // row-prefix bases per row: P_y(64 j - 1), j in [0, nbp)
    int nt;            // 1: table entries stored non-temporally (streaming)
    int rec;           // planar record layout (sum, squares, gradient; squares'
                       // region sums below 2^40): sum plane, 8-byte {squares low
                       // word, gradient} records, byte plane of squares bits 32..39
};

// Table entries hold the nq quantities in feature order, each in ebytes
// bytes; with sqi >= 0 (ebytes 8) an entry is 16 bytes instead: the squares
// (quantity slot sqi) as 64 bits, then the other quantities in feature order
// as 32 bits each (modulo 2^32), zero padded.  planar: each quantity in a
// plane of its own, plane allocations 256-byte aligned; with sqi >= 0 every
// plane holds 32-bit values and the squares take two planes, low word then
// high word, unless rec: then (sum, squares, gradient only) the sum plane is
// followed by an 8-byte {squares low word, gradient} record per entry and a
// byte plane of the squares' bits 32..39 (see TabPR).  Rows are a multiple of
// TAB_LINE bytes, and entry 0 of a table (plane) sits tab_off = TAB_LINE -
// tab_es bytes into its allocation.
constexpr int TAB_LINE = 128;
BuildGeom make_geom(int H, int W, int nq, int ebytes, int sqi = -1, int planar = 0, int rec = 0);

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

// Batched plan (all templates of a screen in one persistent launch).
constexpr int BATCH_GROUP = 64;        // templates per group (scale bits kept in registers)
constexpr int BATCH_GROUP_RINGS = 32;  // with central-star rings (pass and fail bits)

struct DevBatchProbe {
    int64_t lo[3];
    int64_t hi[3];
    int32_t t;     // template slot within its group
    int32_t k;     // scale bit
    int32_t ring;  // 0: the probe's own star; j > 0: its j-th central star
    int32_t pad;
};

struct DevBatchGroup {
    int32_t n_t;                  // templates in the group
    int32_t tmap[BATCH_GROUP];    // slot -> template index of the screen
    int32_t pad;
};

struct DevBatchPass {
    int32_t group;
    int32_t j0, j1;  // radii [j0, j1) of the global radius array
    int32_t first;   // 1: the group's first pass (nothing carried in)
    int32_t last;    // 1: the group's last pass (emits the mask, counts and candidates);
                     // 0: stores the scale-bit words for the next pass
    int32_t pad;
};

// One radius of a batched group: its probes, the hull of their intervals
// per feature slot (a position outside it fails every probe) and their
// intersection, the core (a position inside it passes every probe).  With a
// core, core_bits[cb_first + slot] holds the scale bits the radius' probes
// set for each template slot of the group; cb_first < 0: no core (empty, or
// central-star entries).
struct DevBatchRadius {
    int32_t r, s;
    int32_t first, count;
    int64_t lo[3], hi[3];
    int64_t clo[3], chi[3];
    int64_t roff[4];  // byte offsets of table rows y-s-1, y+s, y-r-1, y+r from row y-1
    int32_t cb_first;
    int32_t pad;
};

constexpr int MAX_RINGS = 4;

struct BatchDevPlan {
    uint8_t *const *mask_of;  // per template of the screen (null: no mask)
    const DevBatchPass *passes;
    int n_passes;
    const DevBatchGroup *groups;
    const DevBatchRadius *radii;
    const DevBatchProbe *probes;
    const uint32_t *core_bits;
    int max_group;
    int rings;  // 1: plain probes; > 1: central-star rings (one pass per group)
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
    K_STAR_BATCH,
    K_COMPACT_SCAN,
    K_COMPACT_LIST,
    K_STAR_MOM,
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
// All arrays hold `ebytes`-wide unsigned integers (mod 2^32 or 2^64).
struct BuildBuffers {
    void *L, *R, *Rp;             // tables [H+1][pitch_e][nq]
    void *bp;                     // [H][nbp][nq] row-prefix bases
    void *agg_L, *agg_AD, *agg_D; // [nb][cw][nq] band contributions
    void *c_L, *c_AD, *c_D;       // [nb][cw][nq] carry rows
};

hipError_t launch_build(const BuildGeom &g, const void *pixels, int64_t pitch_bytes, int dtype,
                        uint32_t feat_mask, const BuildBuffers &bb, hipStream_t stream,
                        Profiler *prof);

// ---------------------------------------------------------------------------
// Fused compaction (Algorithm 1: R <- R u {P}).  A segment is (template t,
// image row y, chunk c): the 64 columns [64 c, 64 c + 64) of row y, which
// one wave of a star pass covers.  For every row it screens, a wave writes,
// per template, the mask bytes of its segment, the number of candidates in
// it (one ballot) and the candidates themselves ({x, scale bits}, in column
// order) to the segment's 64 staging slots: no barrier, no shared memory.
// Segments in (t, y, c) order are in canonical (t, y, x) order; a sum per
// 64 segments, a scan of those sums and a list pass then place the staged
// candidates in the list.  The scale bits never reach memory as one word
// per position.
// ---------------------------------------------------------------------------
constexpr int SEG_W = 64;  // columns per segment (one wave)

struct EmitOut {
    uint8_t *mask;              // plain launches: this template's mask [H][W] (or null);
                                // batched launches take a mask per template beside it
    uint8_t *seg_count;         // [T][H][n_chunks] candidates per segment (<= 64), or null:
                                // the mask alone
    uint2 *stage;               // [T][H][n_chunks][SEG_W]: {x, scale bits}
    uint32_t *dense;            // batched launches over several passes of a group: scale-bit
                                // words [T][H][W] carried between passes, else null
    int H, W, n_chunks;         // n_chunks = ceil(W / SEG_W)
};

// Persistent strip sweep of the star kernel: strips `strip` columns wide (one
// block), each split into `parts` row ranges when there are fewer than 8
// strips; units are dealt to the 8 XCDs round-robin.
constexpr int STAR_MAX_THREADS = 512;
struct StarSweep {
    int strip, n_strips, parts, rows_per_part, n_units, blocks_per_xcd;
};
StarSweep make_sweep(int H, int W, int strip, int blocks_per_xcd);

// LDS staging of the shared table rows is used when it needs at most
// STAR_LDS_MAX bytes per block (smax / rmax: the largest square half-width
// and radius among the template's probes).
constexpr size_t STAR_LDS_MAX = 64 * 1024;
size_t star_lds_bytes(int strip, int nq, int ebytes, int smax, int rmax);
// variant: 0 one radius at a time, 1 LDS-staged rows (32/64-bit
// interleaved entries only), 2 software-pipelined radii, 3 staged lookups
// on planar tables (the first quantity alone, the others only where it
// passes)
hipError_t launch_star_plain(const BuildGeom &g, const void *L, const void *R, const void *Rp,
                             const DevTemplatePlan *plan, const EmitOut &eo, const StarSweep &sw,
                             int smax, int rmax, int variant, hipStream_t stream,
                             Profiler *prof);

// staged: look up the first quantity alone and the others only where it
// lies in the radius' hull (as variant 3 of the plain screen)
hipError_t launch_star_batch(const BuildGeom &g, const void *L, const void *R, const void *Rp,
                             const BatchDevPlan &bp, const EmitOut &eo, const StarSweep &sw,
                             bool staged, hipStream_t stream, Profiler *prof);


// segments of a screen of n_tmpl templates of H x W
int64_t emit_segments(int64_t n_tmpl, int H, int W);
// bytes of the emission workspace (counts, staging, scan) for n_tmpl templates
size_t emit_workspace_bytes(int64_t n_tmpl, int H, int W);
// carve the workspace: counts, staging, then the scan area
void emit_carve(void *ws, int64_t n_tmpl, int H, int W, uint8_t **seg_count, uint2 **stage,
                void **scan_ws);

// The mask is written by the star pass; this places the staged candidates of
// n_tmpl templates' segments (seg_count / stage as carved, possibly offset by
// whole templates) into the list in (t, y, x) order and the total into
// *count.  scan_ws: the carved scan area (one at a time per workspace).
hipError_t launch_list(const uint8_t *seg_count, const uint2 *stage, int64_t n_tmpl, int H,
                       int W, oss_candidate *list, int64_t list_cap, int64_t *count,
                       void *scan_ws, hipStream_t stream, Profiler *prof);
hipError_t launch_region_scatter(const oss_candidate *list, int64_t list_cap,
                                 const int64_t *count, int t, uint32_t bits, int H, int W,
                                 int pad, int64_t wp, uint8_t *ind, hipStream_t st);
hipError_t launch_region_or(const uint8_t *hit, int H, int W, int pad, int64_t wp,
                            uint8_t *region, hipStream_t st);

// The paper's own features (mean, variance, first-moment magnitude) per
// probe: bounds on F1, on V = A(r) F2 - F1^2 and on M = Sx^2 + Sy^2 (128-bit
// unsigned, low word first); tests = which of the three apply.
struct DevMomProbe {
    int64_t lo1, hi1;
    int64_t loV, hiV;
    uint64_t loM[2], hiM[2];
    int32_t k, tests;
};

struct DevMomPlan {
    int32_t n_radii;
    int32_t pad;
    DevRadius radii[OSS_MAX_SCALES];
    DevMomProbe probes[OSS_MAX_SCALES];
};

hipError_t launch_star_moments(const BuildGeom &g, uint32_t fm, const void *L, const void *R,
                               const void *Rp, const DevMomPlan *plan, const EmitOut &eo,
                               const StarSweep &sw, hipStream_t stream, Profiler *prof);

}  // namespace oss
