// Host-side state behind the C ABI handles, shared by the screening entry
// points and the serving loop.
#pragma once

#include "oss_internal.h"

#include <vector>

namespace oss {

// One pinned staging buffer + device copy of a launch plan, reusable once
// the event recorded after the launch that read it has completed.
struct PlanSlot {
    void *host = nullptr;  // pinned staging
    void *dev = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool used = false;
};

constexpr int NSLOTS = 4;

}  // namespace oss

struct oss_ctx {
    int device = 0;
    void *ews = nullptr;       // emission workspace: segment counts, staged candidates, scan
    size_t ews_cap = 0;        // bytes
    uint32_t *bits = nullptr;  // scale-bit words n_tmpl * H * W, only for batched groups
    size_t bits_cap = 0;       // that span several passes (bytes)
    oss::PlanSlot slots[oss::NSLOTS];
    int next_slot = 0;
    oss::Profiler prof;
    int star_strip = 512;          // OSS_OPT_STAR_STRIP
    int star_blocks_per_xcd = 96;  // OSS_OPT_STAR_BLOCKS_PER_XCD
    int star_lds = 0;              // OSS_OPT_STAR_LDS
    int batch_bucket = 0;          // OSS_OPT_BATCH_BUCKET
    int table_planar = 1;          // OSS_OPT_TABLE_PLANAR
    int table_rec = 1;             // OSS_OPT_TABLE_REC
    int star_pipe = 0;             // OSS_OPT_STAR_PIPE
    int star_staged = 1;           // OSS_OPT_STAR_STAGED
    int build_stream = 1;          // OSS_OPT_BUILD_STREAM
    void *rws = nullptr;           // preserved-region workspace (tables of the padded
    size_t rws_cap = 0;            // indicator image, the image, the star pass output)
    // a context used on one stream only (a serving lane): its workspaces,
    // plan buffers and reference tables are allocated and freed in stream
    // order on that stream, so growing them never synchronises the device
    hipStream_t alloc_stream = nullptr;
};

struct oss_ref {
    oss_ctx *ctx = nullptr;
    oss_image_desc desc{};
    uint32_t feat_mask = 0;
    int32_t max_radius = 0;
    oss::BuildGeom geom{};
    void *mem = nullptr;  // one allocation for everything below
    size_t bytes = 0;
    hipStream_t free_stream = nullptr;  // stream-ordered allocation: freed on this stream
    oss::BuildBuffers bb{};
};

namespace oss {

// Host plan of a batched launch: templates sorted by radius in groups of at
// most BATCH_GROUP, each group's probes sorted by reference radius, passes
// over runs of at most `bucket` distinct radii.
struct BatchHostPlan {
    int n_tmpl = 0;
    std::vector<DevBatchPass> passes;
    std::vector<DevBatchGroup> groups;
    std::vector<DevBatchRadius> radii;
    std::vector<DevBatchProbe> probes;
    std::vector<uint32_t> core_bits;  // per radius with a core: one word per template slot
    int max_group = 0;
    int rings = 1;
};

// Tolerance and feature set per template (tols[t], fms[t]); every fms[t]
// must be a subset of the reference's quantities.  With n_rings > 1,
// tmpl is [n_tmpl][n_rings] (ring j of template t at tmpl[t * n_rings + j])
// and every probe is also tested at its central radii s(r), s(s(r)), ...
// against the template's rings; the plan then has one pass per group.
int make_batch_plan(const oss_ref *ref, const oss_template_feat *tmpl, int32_t n_tmpl,
                    const oss_probe *probes, int32_t n_probes, const oss_tolerance *tols,
                    const uint32_t *fms, int bucket, BatchHostPlan &bp, int n_rings = 1);

// Upload the plan and launch the batched star pass on `st`: the mask of
// template t goes to masks[t] (masks null, or an entry null: no mask), the
// segment counts and staged candidates to ctx's emission workspace, which
// must have been grown for bp.n_tmpl templates (screen_workspace); *slot is the plan slot to mark used once an event
// follows the launch.
int batch_star(oss_ctx *ctx, const oss_ref *ref, const BatchHostPlan &bp, int strip, int blocks,
               uint8_t *const *masks, hipStream_t st, PlanSlot **slot);

// Passes of the plan that carry scale bits to a later pass (need ctx->bits).
bool plan_carries(const BatchHostPlan &bp);

// Probe list valid for the reference (ids, radii, scales per template).
int check_probes(const oss_ref *ref, int32_t n_tmpl, const oss_probe *probes, int32_t n_probes);

// Argument checks shared by the screens (before anything is launched).
int check_screen_args(oss_ctx *ctx, const oss_ref *ref, const oss_template_feat *tmpl,
                      int32_t n_tmpl, const oss_probe *probes, int32_t n_probes,
                      const oss_tolerance *tol, uint32_t feat_mask, int64_t list_cap,
                      const oss_candidate *dev_list, const int64_t *dev_count);

// Template t's launch plan from checked probes (no heap allocation).
void template_plan(const oss_ref *ref, const oss_template_feat &tf, int32_t t,
                   const oss_probe *probes, int32_t n_probes, const oss_tolerance *tol,
                   uint32_t fm, DevTemplatePlan *pl);

// Grow every plan slot of ctx to at least `bytes` now (a serving lane does
// this once, so its launches do not grow slots later).
int reserve_plan_slots(oss_ctx *ctx, size_t bytes);

// Look up the no-allocation screen's scratch on `device` (current), once per
// device; called when a context is created.
int noalloc_init(int device);

// Image descriptor valid (sizes, dtype, depth, pitch).
bool desc_ok(const oss_image_desc *d);

// int64 table accumulation cannot overflow for this image and feature set.
bool overflow_ok(const oss_image_desc *d, uint32_t fm);

// Grow ctx's emission workspace for n_tmpl templates of H x W, and with
// `carry` its scale-bit words to n_tmpl * H * W.
int screen_workspace(oss_ctx *ctx, int64_t n_tmpl, int H, int W, bool carry);

// Carve ctx's emission workspace (grown by screen_workspace) for n_tmpl
// templates: EmitOut fields seg_count / stage / geometry, and the scan area.
EmitOut emit_out(oss_ctx *ctx, int64_t n_tmpl, int H, int W, void **scan_ws);

}  // namespace oss
