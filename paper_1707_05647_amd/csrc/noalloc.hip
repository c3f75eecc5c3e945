// The plain screen without allocation (oss_screen_noalloc): oss_screen's
// kernels with their scratch -- the launch plans, the per-segment candidate
// counts, the staged candidates and the scan -- in one fixed array of device
// memory instead of context workspaces, for callers that cannot allocate.
//
// The array is a file-scope device variable.  Its name in host code is only
// a host-side stand-in, not a device address, so its address on each GPU is
// looked up once (hipGetSymbolAddress, with that device current, when the
// first context on it is created) and only that address is handed to
// kernels.  Plans reach the array through a kernel argument, so no host
// buffer, pinned staging or copy is involved.
#include "api_internal.h"

#include <algorithm>
#include <mutex>

namespace oss {

// Shared by every call on a GPU (each GPU holds its own copy).
static __device__ __align__(256) char scratch[OSS_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES];

int noalloc_init(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES)
        return OSS_E_ARG;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device])
        return OSS_OK;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
        return OSS_E_DEVICE;
    g_scratch_ptr[device] = p;
    return OSS_OK;
}

static void *scratch_on(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

// One template's plan, passed by value, stored to its slot in the scratch.
__global__ __launch_bounds__(256) void plan_store_kernel(DevTemplatePlan plan,
                                                         DevTemplatePlan *__restrict__ dst)
{
    const int32_t *src = reinterpret_cast<const int32_t *>(&plan);
    int32_t *out = reinterpret_cast<int32_t *>(dst);
    for (int i = threadIdx.x; i < (int)(sizeof(DevTemplatePlan) / 4); i += blockDim.x)
        out[i] = src[i];
}

static size_t al256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace oss

using namespace oss;

extern "C" int oss_screen_noalloc(oss_ctx *ctx, const oss_ref *ref,
                                  const oss_template_feat *tmpl, int32_t n_tmpl,
                                  const oss_probe *probes, int32_t n_probes,
                                  const oss_tolerance *tol, uint32_t feat_mask, uint8_t *dev_mask,
                                  oss_candidate *dev_list, int64_t list_cap, int64_t *dev_count,
                                  void *stream)
{
    int rc = check_screen_args(ctx, ref, tmpl, n_tmpl, probes, n_probes, tol, feat_mask, list_cap,
                               dev_list, dev_count);
    if (rc != OSS_OK)
        return rc;
    rc = check_probes(ref, n_tmpl, probes, n_probes);
    if (rc != OSS_OK)
        return rc;
    const BuildGeom &g = ref->geom;
    // scratch layout: the plans, then the emission workspace (counts,
    // staging, scan) carved as the context workspace would be
    const size_t plan_bytes = al256((size_t)n_tmpl * sizeof(DevTemplatePlan));
    const size_t need = plan_bytes + emit_workspace_bytes(n_tmpl, g.H, g.W);
    if (need > OSS_NOALLOC_SCRATCH_BYTES)
        return OSS_E_LIMIT;
    char *base = static_cast<char *>(scratch_on(ctx->device));
    if (!base)
        return OSS_E_STATE;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return OSS_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    DevTemplatePlan *dplan = reinterpret_cast<DevTemplatePlan *>(base);
    EmitOut all{};
    void *scan_ws = nullptr;
    emit_carve(base + plan_bytes, n_tmpl, g.H, g.W, &all.seg_count, &all.stage, &scan_ws);
    all.H = g.H;
    all.W = g.W;
    all.n_chunks = (g.W + SEG_W - 1) / SEG_W;
    const int64_t hw = (int64_t)g.H * g.W;
    const int64_t segs_t = (int64_t)g.H * all.n_chunks;
    const StarSweep sw = make_sweep(g.H, g.W, ctx->star_strip, ctx->star_blocks_per_xcd);
    const int variant = ctx->star_lds ? 1 : ctx->star_pipe ? 2 : ctx->star_staged ? 3 : 0;
    for (int t = 0; t < n_tmpl; ++t) {
        DevTemplatePlan pl;
        template_plan(ref, tmpl[t], t, probes, n_probes, tol, feat_mask, &pl);
        hipLaunchKernelGGL(plan_store_kernel, dim3(1), dim3(256), 0, st, pl, dplan + t);
        if (hipGetLastError() != hipSuccess)
            return OSS_E_DEVICE;
        int smax = 0, rmax = 0;
        for (int j = 0; j < pl.n_radii; ++j) {
            smax = std::max(smax, (int)pl.radii[j].s);
            rmax = std::max(rmax, (int)pl.radii[j].r);
        }
        EmitOut eo = all;
        eo.mask = dev_mask ? dev_mask + hw * t : nullptr;
        eo.seg_count = all.seg_count + segs_t * t;
        eo.stage = all.stage + segs_t * SEG_W * t;
        if (launch_star_plain(g, ref->bb.L, ref->bb.R, ref->bb.Rp, dplan + t, eo, sw, smax, rmax,
                              variant, st, nullptr) != hipSuccess)
            return OSS_E_DEVICE;
    }
    if (launch_list(all.seg_count, all.stage, n_tmpl, g.H, g.W, dev_list, list_cap, dev_count,
                    scan_ws, st, nullptr) != hipSuccess)
        return OSS_E_DEVICE;
    return OSS_OK;
}
