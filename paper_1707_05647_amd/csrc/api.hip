// C ABI of the octagonal-star screening library (include/oss.h).
#include "api_internal.h"

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>

using namespace oss;

namespace oss {

int square_half(int r)
{
    int s = 0;
    while ((int64_t)(2 * s + 1) * (2 * s + 1) < 2LL * r * r)
        ++s;
    return s;
}

int64_t star_area(int r)
{
    const int64_t s = square_half(r);
    return (2 * s + 1) * (2 * s + 1) + 2LL * r * r + 2LL * r + 1;
}

static __int128 floor_div(__int128 a, __int128 b)  // b > 0
{
    __int128 q = a / b;
    if ((a % b != 0) && (a < 0))
        --q;
    return q;
}

static int64_t clamp64(__int128 v)
{
    if (v > (__int128)INT64_MAX)
        return INT64_MAX;
    if (v < (__int128)INT64_MIN)
        return INT64_MIN;
    return (int64_t)v;
}

// (Q-P) X_T <= Q X_ref <= (Q+P) X_T with X_ref = F A(rho) c_ref and
// X_T = FT A(r) c_T, solved for the integer F: F in [lo, hi].
void feature_bounds(int f, int64_t FT, int r, int rho, int P, int Q, int64_t *lo, int64_t *hi)
{
    const __int128 c_ref = (f == 2) ? r : 1;
    const __int128 c_t = (f == 2) ? rho : 1;
    const __int128 xt = (__int128)FT * star_area(r) * c_t;
    const __int128 k = (__int128)Q * star_area(rho) * c_ref;
    const __int128 lo_num = (__int128)(Q - P) * xt;
    const __int128 hi_num = (__int128)(Q + P) * xt;
    if (k == 0) {
        // X_ref is 0 whatever F is
        const bool ok = lo_num <= 0 && 0 <= hi_num;
        *lo = ok ? INT64_MIN : 1;
        *hi = ok ? INT64_MAX : 0;
        return;
    }
    *lo = clamp64(-floor_div(-lo_num, k));
    *hi = clamp64(floor_div(hi_num, k));
}

}  // namespace oss

static int popc(uint32_t m) { return __builtin_popcount(m); }

bool oss::desc_ok(const oss_image_desc *d)
{
    if (!d || d->H <= 0 || d->W <= 0)
        return false;
    if (d->dtype == OSS_U8) {
        if (d->bit_depth < 1 || d->bit_depth > 8)
            return false;
    } else if (d->dtype == OSS_U16) {
        if (d->bit_depth < 1 || d->bit_depth > 16)
            return false;
    } else {
        return false;
    }
    const int64_t px = d->dtype == OSS_U8 ? 1 : 2;
    if (d->pitch_bytes < (int64_t)d->W * px || d->pitch_bytes % px != 0)
        return false;
    return true;
}

// Device allocation and release: in stream order on `async` when given (a
// context used on that stream only), else plain (a free synchronises the
// device).
static hipError_t dev_alloc(void **p, size_t bytes, hipStream_t async)
{
    return async ? hipMallocAsync(p, bytes, async) : hipMalloc(p, bytes);
}

static void dev_free(void *p, hipStream_t async)
{
    if (!p)
        return;
    if (async)
        (void)hipFreeAsync(p, async);
    else
        (void)hipFree(p);
}

static int hip_status(hipError_t e) { return e == hipSuccess ? OSS_OK : OSS_E_DEVICE; }

extern "C" {

const char *oss_status_string(int status)
{
    switch (status) {
    case OSS_OK: return "OSS_OK";
    case OSS_E_ARG: return "OSS_E_ARG";
    case OSS_E_NOMEM: return "OSS_E_NOMEM";
    case OSS_E_OVERFLOW: return "OSS_E_OVERFLOW";
    case OSS_E_DEVICE: return "OSS_E_DEVICE";
    case OSS_E_STATE: return "OSS_E_STATE";
    case OSS_E_LIMIT: return "OSS_E_LIMIT";
    case OSS_E_CANCELLED: return "OSS_E_CANCELLED";
    case OSS_E_TIMEOUT: return "OSS_E_TIMEOUT";
    default: return "OSS_E_UNKNOWN";
    }
}

int oss_ctx_create(int device, oss_ctx **out)
{
    if (!out)
        return OSS_E_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess)
        return OSS_E_DEVICE;
    if (device < 0 || device >= n)
        return OSS_E_ARG;
    if (hipSetDevice(device) != hipSuccess)
        return OSS_E_DEVICE;
    oss_ctx *c = new (std::nothrow) oss_ctx();
    if (!c)
        return OSS_E_NOMEM;
    c->device = device;
    // the no-allocation screen's scratch address on this device
    if (noalloc_init(device) != OSS_OK) {
        delete c;
        return OSS_E_DEVICE;
    }
    for (auto &s : c->slots) {
        if (hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess) {
            oss_ctx_destroy(c);
            return OSS_E_DEVICE;
        }
    }
    *out = c;
    return OSS_OK;
}

int oss_ctx_destroy(oss_ctx *ctx)
{
    if (!ctx)
        return OSS_E_ARG;
    (void)hipSetDevice(ctx->device);
    hipStream_t as = ctx->alloc_stream;
    for (auto &s : ctx->slots) {
        if (s.ev) {
            if (s.used)
                (void)hipEventSynchronize(s.ev);
            (void)hipEventDestroy(s.ev);
        }
        if (s.host)
            (void)hipHostFree(s.host);
        dev_free(s.dev, as);
    }
    dev_free(ctx->bits, as);
    dev_free(ctx->ews, as);
    dev_free(ctx->rws, as);
    if (as)
        (void)hipStreamSynchronize(as);
    delete ctx;
    return OSS_OK;
}

// Device layout of a reference: 3 tables, the row-prefix bases, 3 band
// contribution arrays and 3 carry arrays, each 256-byte aligned.
enum { A_L, A_R, A_RP, A_BP, A_AGL, A_AGAD, A_AGD, A_CL, A_CAD, A_CD, A_COUNT };

static size_t ref_layout(const BuildGeom &g, size_t off[A_COUNT])
{
    const size_t e = (size_t)g.ebytes * (size_t)g.nq;
    const size_t table = (size_t)g.tab_bytes;
    const size_t bp = (size_t)g.H * g.nbp * e;
    const size_t car = (size_t)g.nb * g.cw * e;
    const size_t sizes[A_COUNT] = {table, table, table, bp, car, car, car, car, car, car};
    size_t acc = 0;
    for (int i = 0; i < A_COUNT; ++i) {
        off[i] = acc;
        acc += (sizes[i] + 255) / 256 * 256;
    }
    return acc;
}

static __int128 max_quantity(const oss_image_desc *d, uint32_t fm)
{
    const __int128 maxv = ((__int128)1 << d->bit_depth) - 1;
    __int128 maxq = 0;
    if (fm & OSS_F_SUM)
        maxq = std::max(maxq, maxv);
    if (fm & OSS_F_SQ)
        maxq = std::max(maxq, maxv * maxv);
    if (fm & OSS_F_GRAD)
        maxq = std::max(maxq, 2 * maxv);
    return maxq;
}

}  // extern "C"

bool oss::overflow_ok(const oss_image_desc *d, uint32_t fm)
{
    return (__int128)d->H * d->W * max_quantity(d, fm) < ((__int128)1 << 62);
}

extern "C" {

static int32_t resolve_max_radius(const oss_image_desc *d, int32_t max_radius)
{
    const int32_t fit = (std::min(d->H, d->W) - 1) / 2;
    return max_radius < 0 ? fit : max_radius;
}

// A quantity can be stored modulo 2^32 when every square and every diamond
// sum of it up to the maximum radius stays below 2^32.  All quantities fit:
// 32-bit values.  Only the squares do not: the squares in 64 bits, the others
// in 32.  Otherwise 64-bit values.  Planar (the default) or interleaved
// entries as the context asks.  Planar tables of the sum, the squares and
// the gradient whose squares' square and diamond sums stay below 2^40 use
// the record layout when the context asks (rec): the squares' low words and
// the gradient in one 8-byte record per entry, the squares' bits 32..39 in a
// byte plane.
static BuildGeom ref_geom(const oss_image_desc *d, uint32_t fm, int32_t R, int planar,
                          int rec = 0)
{
    const __int128 s = square_half(R);
    const __int128 area = std::max((2 * s + 1) * (2 * s + 1),
                                   (__int128)2 * R * R + 2 * (__int128)R + 1);
    auto fits = [&](uint32_t m) { return max_quantity(d, m) * area < ((__int128)1 << 32); };
    const int nq = popc(fm);
    if (fm & OSS_F_MOMENTS) {
        // a region's first moment sum (i - x) I is at most maxv R |region| in
        // magnitude: stored modulo 2^32 when that stays below 2^31
        const __int128 maxv = ((__int128)1 << d->bit_depth) - 1;
        const bool m32 = maxv * R * area < ((__int128)1 << 31);
        return make_geom(d->H, d->W, nq, (fits(fm & OSS_F_ALL) && m32) ? 4 : 8, -1, planar);
    }
    if (fits(fm))
        return make_geom(d->H, d->W, nq, 4, -1, planar);
    if ((fm & OSS_F_SQ) && nq >= 2 && fits(fm & ~(uint32_t)OSS_F_SQ)) {
        const bool sq40 = max_quantity(d, OSS_F_SQ) * area < ((__int128)1 << 40);
        return make_geom(d->H, d->W, nq, 8, (fm & OSS_F_SUM) ? 1 : 0, planar,
                         (rec && planar && fm == OSS_F_ALL && sq40) ? 1 : 0);
    }
    return make_geom(d->H, d->W, nq, 8, -1, planar);
}

}  // extern "C"

// Feature sets a reference may hold: any non-empty subset of sum, squares
// and gradient, or the sum and both first moments (with or without squares).
static bool ref_fm_ok(uint32_t fm)
{
    if (fm & OSS_F_MOMENTS)
        return fm == (OSS_F_SUM | OSS_F_MOMENTS) || fm == (OSS_F_SUM | OSS_F_SQ | OSS_F_MOMENTS);
    return fm != 0 && !(fm & ~OSS_F_ALL);
}

extern "C" {

int oss_ref_bytes(const oss_image_desc *desc, uint32_t feat_mask, int32_t max_radius, size_t *out)
{
    if (!out || !desc_ok(desc) || !ref_fm_ok(feat_mask))
        return OSS_E_ARG;
    // the larger of the interleaved and the planar layout
    const int32_t R = resolve_max_radius(desc, max_radius);
    size_t off[A_COUNT];
    *out = std::max(ref_layout(ref_geom(desc, feat_mask, R, 0), off),
                    ref_layout(ref_geom(desc, feat_mask, R, 1), off));
    return OSS_OK;
}

int oss_ref_create(oss_ctx *ctx, const oss_image_desc *desc, uint32_t feat_mask,
                   int32_t max_radius, oss_ref **out)
{
    if (!ctx || !out || !desc_ok(desc) || !ref_fm_ok(feat_mask))
        return OSS_E_ARG;
    *out = nullptr;
    if (!overflow_ok(desc, feat_mask))
        return OSS_E_OVERFLOW;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return OSS_E_DEVICE;
    oss_ref *r = new (std::nothrow) oss_ref();
    if (!r)
        return OSS_E_NOMEM;
    r->ctx = ctx;
    r->desc = *desc;
    r->feat_mask = feat_mask;
    r->max_radius = resolve_max_radius(desc, max_radius);
    r->geom = ref_geom(desc, feat_mask, r->max_radius, ctx->table_planar, ctx->table_rec);
    size_t off[A_COUNT];
    r->bytes = ref_layout(r->geom, off);
    r->free_stream = ctx->alloc_stream;
    if (dev_alloc(&r->mem, r->bytes, r->free_stream) != hipSuccess) {
        delete r;
        return OSS_E_NOMEM;
    }
    char *m = static_cast<char *>(r->mem);
    auto at = [&](int i) { return static_cast<void *>(m + off[i]); };
    const int to = r->geom.tab_off;  // entry 0 of each table (plane)
    r->bb.L = m + off[A_L] + to;
    r->bb.R = m + off[A_R] + to;
    r->bb.Rp = m + off[A_RP] + to;
    r->bb.bp = at(A_BP);
    r->bb.agg_L = at(A_AGL);
    r->bb.agg_AD = at(A_AGAD);
    r->bb.agg_D = at(A_AGD);
    r->bb.c_L = at(A_CL);
    r->bb.c_AD = at(A_CAD);
    r->bb.c_D = at(A_CD);
    *out = r;
    return OSS_OK;
}

int oss_ref_build(oss_ref *ref, const void *dev_pixels, void *stream)
{
    if (!ref || !dev_pixels)
        return OSS_E_ARG;
    if (hipSetDevice(ref->ctx->device) != hipSuccess)
        return OSS_E_DEVICE;
    oss::BuildGeom g = ref->geom;
    g.nt = ref->ctx->build_stream;
    return hip_status(launch_build(g, dev_pixels, ref->desc.pitch_bytes, ref->desc.dtype,
                                   ref->feat_mask, ref->bb, static_cast<hipStream_t>(stream),
                                   &ref->ctx->prof));
}

int oss_ref_release(oss_ref *ref)
{
    if (!ref)
        return OSS_E_ARG;
    (void)hipSetDevice(ref->ctx->device);
    // with stream-ordered tables the caller guarantees that no work reading
    // them is still pending (or is ordered before the free on that stream)
    dev_free(ref->mem, ref->free_stream);
    delete ref;
    return OSS_OK;
}

int oss_ref_tables(const oss_ref *ref, const void **L, const void **R, const void **Rp,
                   int64_t *pitch_entries, int32_t *nq, int32_t *value_bits,
                   int32_t *max_radius)
{
    if (!ref)
        return OSS_E_ARG;
    if (L)
        *L = ref->bb.L;
    if (R)
        *R = ref->bb.R;
    if (Rp)
        *Rp = ref->bb.Rp;
    if (pitch_entries)
        *pitch_entries = ref->geom.pitch_e;
    if (nq)
        *nq = ref->geom.nq;
    if (value_bits)
        *value_bits = 8 * ref->geom.ebytes;
    if (max_radius)
        *max_radius = ref->max_radius;
    return OSS_OK;
}

int oss_ref_layout_q(const oss_ref *ref, oss_quantity_layout out[OSS_MAX_QUANTITIES],
                     int32_t *nq, int64_t *plane_bytes)
{
    if (!ref || !out || !nq || !plane_bytes)
        return OSS_E_ARG;
    const BuildGeom &g = ref->geom;
    *nq = g.nq;
    *plane_bytes = g.plane;
    int j = 0;
    for (int q = 0; q < OSS_MAX_QUANTITIES; ++q) {
        oss_quantity_layout &o = out[q];
        o = oss_quantity_layout{-1, 0, 0, -1, 0, 0};
        if (q >= g.nq)
            continue;
        if (g.rec) {
            // sum plane; {squares low word, gradient} records; squares' byte plane
            o.stride = q == 0 ? 4 : 8;
            o.bits = 32;
            o.offset = q == 0 ? 0 : q == 1 ? g.plane - 4 : g.plane;
            if (q == 1) {
                o.hi_offset = 3 * g.plane + 3;
                o.hi_stride = 1;
                o.hi_bits = 8;
            }
        } else if (g.planar && g.sqi >= 0) {
            const int pl = q <= g.sqi ? q : q + 1;
            o.offset = pl * g.plane;
            o.stride = 4;
            o.bits = 32;
            if (q == g.sqi) {
                o.hi_offset = (pl + 1) * g.plane;
                o.hi_stride = 4;
                o.hi_bits = 32;
            }
        } else if (g.planar) {
            o.offset = q * g.plane;
            o.stride = g.ebytes;
            o.bits = 8 * g.ebytes;
        } else if (g.sqi < 0) {
            o.offset = q * g.ebytes;
            o.stride = g.tab_es;
            o.bits = 8 * g.ebytes;
        } else {
            o.stride = 16;
            o.offset = q == g.sqi ? 0 : 8 + 4 * j++;
            o.bits = q == g.sqi ? 64 : 32;
        }
    }
    return OSS_OK;
}

int oss_ref_layout(const oss_ref *ref, int32_t *entry_stride, int64_t offset[OSS_MAX_QUANTITIES],
                   int32_t bits[OSS_MAX_QUANTITIES], int64_t *plane_bytes)
{
    if (!ref || !entry_stride || !offset || !bits || !plane_bytes)
        return OSS_E_ARG;
    const BuildGeom &g = ref->geom;
    if (g.rec)
        return OSS_E_STATE;  // per-quantity strides: oss_ref_layout_q
    *entry_stride = g.tab_es;
    *plane_bytes = g.plane;
    int j = 0;
    for (int q = 0; q < OSS_MAX_QUANTITIES; ++q) {
        offset[q] = -1;
        bits[q] = 0;
    }
    for (int q = 0; q < g.nq; ++q) {
        if (g.planar && g.sqi >= 0) {
            offset[q] = (q <= g.sqi ? q : q + 1) * g.plane;
            bits[q] = q == g.sqi ? 64 : 32;
        } else if (g.planar) {
            offset[q] = q * g.plane;
            bits[q] = 8 * g.ebytes;
        } else if (g.sqi < 0) {
            offset[q] = q * g.ebytes;
            bits[q] = 8 * g.ebytes;
        } else if (q == g.sqi) {
            offset[q] = 0;
            bits[q] = 64;
        } else {
            offset[q] = 8 + 4 * j++;
            bits[q] = 32;
        }
    }
    return OSS_OK;
}

// Template features on the host: star sums at the template centre, summed
// row by row over the square's and the diamond's spans.
}  // extern "C"

// Star sums of radius rho at (cx, cy) of a host image (gradient clamped to
// the image), for the enabled features (others 0).  The star must fit.
static void star_feats_at(const void *host_pixels, const oss_image_desc *desc, int cx, int cy,
                          int rho, uint32_t feat_mask, int64_t F[3])
{
    const int H = desc->H, W = desc->W;
    const unsigned char *base = static_cast<const unsigned char *>(host_pixels);
    auto pix = [&](int x, int y) -> int64_t {
        const unsigned char *row = base + (int64_t)y * desc->pitch_bytes;
        if (desc->dtype == OSS_U8)
            return row[x];
        uint16_t v;
        std::memcpy(&v, row + 2 * (int64_t)x, 2);
        return v;
    };
    auto grad = [&](int x, int y) -> int64_t {
        const int xr = std::min(x + 1, W - 1), xl = std::max(x - 1, 0);
        const int yd = std::min(y + 1, H - 1), yu = std::max(y - 1, 0);
        const int64_t gx = pix(xr, y) - pix(xl, y), gy = pix(x, yd) - pix(x, yu);
        return (gx < 0 ? -gx : gx) + (gy < 0 ? -gy : gy);
    };
    int64_t f1 = 0, f2 = 0, fg = 0;
    auto span = [&](int y, int x0, int x1) {
        for (int x = x0; x <= x1; ++x) {
            const int64_t v = pix(x, y);
            f1 += v;
            f2 += v * v;
            if (feat_mask & OSS_F_GRAD)
                fg += grad(x, y);
        }
    };
    const int s = square_half(rho);
    for (int dy = -s; dy <= s; ++dy)
        span(cy + dy, cx - s, cx + s);
    for (int dy = -rho; dy <= rho; ++dy) {
        const int h = rho - (dy < 0 ? -dy : dy);
        span(cy + dy, cx - h, cx + h);
    }
    F[0] = (feat_mask & OSS_F_SUM) ? f1 : 0;
    F[1] = (feat_mask & OSS_F_SQ) ? f2 : 0;
    F[2] = (feat_mask & OSS_F_GRAD) ? fg : 0;
}

extern "C" {

int oss_template_features(const void *host_pixels, const oss_image_desc *desc, int32_t rho,
                          uint32_t feat_mask, oss_template_feat *out)
{
    if (!host_pixels || !out || !desc_ok(desc) || feat_mask == 0 || (feat_mask & ~OSS_F_ALL))
        return OSS_E_ARG;
    const int H = desc->H, W = desc->W;
    const int cx = (W - 1) / 2, cy = (H - 1) / 2;
    const int rmax = std::min(std::min(cx, W - 1 - cx), std::min(cy, H - 1 - cy));
    // with the gradient the star must keep off the template's border: a tip
    // on the border sees a clamped gradient there that the same pixel inside
    // the reference does not have, and an exact copy could then fail
    const int rcap = rmax - ((feat_mask & OSS_F_GRAD) ? 1 : 0);
    if (rho < 0)
        rho = rcap;
    if (rho < 0 || rho > rcap)
        return OSS_E_ARG;
    star_feats_at(host_pixels, desc, cx, cy, rho, feat_mask, out->F);
    out->rho = rho;
    out->feat_mask = feat_mask;
    return OSS_OK;
}

int oss_template_features_rings(const void *host_pixels, const oss_image_desc *desc,
                                int32_t rho, uint32_t feat_mask, int32_t n_rings,
                                oss_template_feat *out)
{
    if (!out || n_rings < 1 || n_rings > MAX_RINGS)
        return OSS_E_ARG;
    int rc = oss_template_features(host_pixels, desc, rho, feat_mask, &out[0]);
    for (int j = 1; j < n_rings && rc == OSS_OK; ++j)
        rc = oss_template_features(host_pixels, desc, square_half(out[j - 1].rho), feat_mask,
                                   &out[j]);
    return rc;
}

int oss_ctx_set_option(oss_ctx *ctx, int32_t option, int32_t value)
{
    if (!ctx)
        return OSS_E_ARG;
    switch (option) {
    case OSS_OPT_STAR_STRIP:
        if (value < 64 || value > 512 || value % 64)
            return OSS_E_ARG;
        ctx->star_strip = value;
        return OSS_OK;
    case OSS_OPT_STAR_BLOCKS_PER_XCD:
        if (value < 1 || value > 4096)
            return OSS_E_ARG;
        ctx->star_blocks_per_xcd = value;
        return OSS_OK;
    case OSS_OPT_STAR_LDS:
        if (value != 0 && value != 1)
            return OSS_E_ARG;
        ctx->star_lds = value;
        return OSS_OK;
    case OSS_OPT_BATCH_BUCKET:
        if (value < 0 || value > 4096)
            return OSS_E_ARG;
        ctx->batch_bucket = value;
        return OSS_OK;
    case OSS_OPT_TABLE_PLANAR:
        if (value != 0 && value != 1)
            return OSS_E_ARG;
        ctx->table_planar = value;
        return OSS_OK;
    case OSS_OPT_STAR_PIPE:
        if (value != 0 && value != 1)
            return OSS_E_ARG;
        ctx->star_pipe = value;
        return OSS_OK;
    case OSS_OPT_STAR_STAGED:
        if (value != 0 && value != 1)
            return OSS_E_ARG;
        ctx->star_staged = value;
        return OSS_OK;
    case OSS_OPT_BUILD_STREAM:
        if (value != 0 && value != 1)
            return OSS_E_ARG;
        ctx->build_stream = value;
        return OSS_OK;
    case OSS_OPT_TABLE_REC:
        if (value != 0 && value != 1)
            return OSS_E_ARG;
        ctx->table_rec = value;
        return OSS_OK;
    default:
        return OSS_E_ARG;
    }
}

int oss_ctx_get_option(oss_ctx *ctx, int32_t option, int32_t *value)
{
    if (!ctx || !value)
        return OSS_E_ARG;
    switch (option) {
    case OSS_OPT_STAR_STRIP: *value = ctx->star_strip; return OSS_OK;
    case OSS_OPT_STAR_BLOCKS_PER_XCD: *value = ctx->star_blocks_per_xcd; return OSS_OK;
    case OSS_OPT_STAR_LDS: *value = ctx->star_lds; return OSS_OK;
    case OSS_OPT_BATCH_BUCKET: *value = ctx->batch_bucket; return OSS_OK;
    case OSS_OPT_TABLE_PLANAR: *value = ctx->table_planar; return OSS_OK;
    case OSS_OPT_STAR_PIPE: *value = ctx->star_pipe; return OSS_OK;
    case OSS_OPT_STAR_STAGED: *value = ctx->star_staged; return OSS_OK;
    case OSS_OPT_BUILD_STREAM: *value = ctx->build_stream; return OSS_OK;
    case OSS_OPT_TABLE_REC: *value = ctx->table_rec; return OSS_OK;
    default: return OSS_E_ARG;
    }
}

int oss_ctx_profile(oss_ctx *ctx, int enable)
{
    if (!ctx)
        return OSS_E_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return OSS_E_DEVICE;
    if (enable) {
        ctx->prof.clear();
        ctx->prof.on = true;
    } else {
        ctx->prof.on = false;
    }
    return OSS_OK;
}

int oss_ctx_profile_read(oss_ctx *ctx, oss_kernel_stat *out, int32_t cap, int32_t *n)
{
    if (!ctx || !n || cap < 0 || (cap > 0 && !out))
        return OSS_E_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return OSS_E_DEVICE;
    if (ctx->prof.resolve() != hipSuccess)
        return OSS_E_DEVICE;
    int32_t k = 0;
    for (int i = 0; i < K_COUNT; ++i) {
        if (ctx->prof.launches[i] == 0)
            continue;
        if (k < cap) {
            std::memset(out[k].name, 0, sizeof(out[k].name));
            std::strncpy(out[k].name, kKernelNames[i], sizeof(out[k].name) - 1);
            out[k].launches = ctx->prof.launches[i];
            out[k].total_ms = ctx->prof.total_ms[i];
            out[k].max_ms = ctx->prof.max_ms[i];
        }
        ++k;
    }
    *n = k < cap ? k : cap;
    return OSS_OK;
}

int oss_feature_bounds(int32_t feature, int64_t FT, int32_t r, int32_t rho,
                       const oss_tolerance *tol, int64_t *lo, int64_t *hi)
{
    if (!tol || !lo || !hi || feature < 0 || feature > 2 || r < 0 || rho < 0 || tol->Q <= 0 ||
        tol->P[feature] < 0)
        return OSS_E_ARG;
    feature_bounds(feature, FT, r, rho, tol->P[feature], tol->Q, lo, hi);
    return OSS_OK;
}

}  // extern "C"

// grow a device buffer; the old one may still be read by work enqueued on
// the context's streams: without a stream of its own the context waits for
// the device before freeing it, with one the free is ordered after that work
static int grow(void **p, size_t *cap, size_t need, hipStream_t async)
{
    if (*cap >= need)
        return OSS_OK;
    if (*p) {
        if (!async && hipDeviceSynchronize() != hipSuccess)
            return OSS_E_DEVICE;
        dev_free(*p, async);
        *p = nullptr;
        *cap = 0;
    }
    if (dev_alloc(p, need, async) != hipSuccess) {
        *p = nullptr;
        return OSS_E_NOMEM;
    }
    *cap = need;
    return OSS_OK;
}

// copy `bytes` of host data to a device plan buffer through a pinned slot
static int upload_plan(oss_ctx *ctx, const void *src, size_t bytes, hipStream_t st, PlanSlot **used)
{
    PlanSlot &s = ctx->slots[ctx->next_slot];
    ctx->next_slot = (ctx->next_slot + 1) % NSLOTS;
    if (s.used && hipEventSynchronize(s.ev) != hipSuccess)
        return OSS_E_DEVICE;
    if (s.cap < bytes) {
        // the slot's last use has completed (its event, above)
        if (s.host)
            (void)hipHostFree(s.host);
        dev_free(s.dev, ctx->alloc_stream);
        s.host = s.dev = nullptr;
        s.cap = 0;
        if (hipHostMalloc(&s.host, bytes, hipHostMallocDefault) != hipSuccess)
            return OSS_E_NOMEM;
        if (dev_alloc(&s.dev, bytes, ctx->alloc_stream) != hipSuccess) {
            s.dev = nullptr;
            return OSS_E_NOMEM;
        }
        s.cap = bytes;
    }
    std::memcpy(s.host, src, bytes);
    if (hipMemcpyAsync(s.dev, s.host, bytes, hipMemcpyHostToDevice, st) != hipSuccess)
        return OSS_E_DEVICE;
    *used = &s;
    return OSS_OK;
}

// Probe list valid for a reference: template and scale ids in range, radii
// within the tables' reach, at most OSS_MAX_SCALES probes per template.
int oss::check_probes(const oss_ref *ref, int32_t n_tmpl, const oss_probe *probes,
                      int32_t n_probes)
{
    for (int i = 0; i < n_probes; ++i) {
        const oss_probe &p = probes[i];
        if (p.template_id < 0 || p.template_id >= n_tmpl || p.scale_id < 0 ||
            p.scale_id >= OSS_MAX_SCALES || p.r < 0 || p.r > ref->max_radius)
            return OSS_E_ARG;
    }
    for (int t = 0; t < n_tmpl; ++t) {
        int k = 0;
        for (int i = 0; i < n_probes; ++i)
            k += probes[i].template_id == t;
        if (k > OSS_MAX_SCALES)
            return OSS_E_ARG;
    }
    return OSS_OK;
}

// Template t's plan (probes already checked): its distinct radii in
// increasing order, and for each the probes with their exact feature-sum
// bounds in table slot order.  No heap allocation.
void oss::template_plan(const oss_ref *ref, const oss_template_feat &tf, int32_t t,
                        const oss_probe *probes, int32_t n_probes, const oss_tolerance *tol,
                        uint32_t fm, DevTemplatePlan *pl)
{
    *pl = DevTemplatePlan{};
    // the template's probes, stably sorted by radius (insertion sort)
    oss_probe v[OSS_MAX_SCALES];
    int n = 0;
    for (int i = 0; i < n_probes; ++i) {
        if (probes[i].template_id != t)
            continue;
        int j = n++;
        while (j > 0 && v[j - 1].r > probes[i].r) {
            v[j] = v[j - 1];
            --j;
        }
        v[j] = probes[i];
    }
    // feature f -> table slot (the reference's quantities in bit order)
    int slot_of[3], slot = 0;
    for (int f = 0; f < 3; ++f)
        slot_of[f] = (ref->feat_mask & (1u << f)) ? slot++ : -1;
    int nr = 0;
    for (int i = 0; i < n; ++i) {
        if (nr == 0 || pl->radii[nr - 1].r != v[i].r) {
            pl->radii[nr].r = v[i].r;
            pl->radii[nr].s = square_half(v[i].r);
            pl->radii[nr].first = (int32_t)i;
            pl->radii[nr].count = 0;
            ++nr;
        }
        pl->radii[nr - 1].count++;
        DevProbe &dp = pl->probes[i];
        dp.k = v[i].scale_id;
        for (int q = 0; q < 3; ++q) {
            dp.lo[q] = INT64_MIN;
            dp.hi[q] = INT64_MAX;
        }
        for (int f = 0; f < 3; ++f) {
            if (!(fm & (1u << f)))
                continue;
            feature_bounds(f, tf.F[f], v[i].r, tf.rho, tol->P[f], tol->Q, &dp.lo[slot_of[f]],
                           &dp.hi[slot_of[f]]);
        }
    }
    pl->n_radii = nr;
}

int oss::reserve_plan_slots(oss_ctx *ctx, size_t bytes)
{
    for (PlanSlot &s : ctx->slots) {
        if (s.cap >= bytes)
            continue;
        if (s.used && hipEventSynchronize(s.ev) != hipSuccess)
            return OSS_E_DEVICE;
        if (s.host)
            (void)hipHostFree(s.host);
        dev_free(s.dev, ctx->alloc_stream);
        s.host = s.dev = nullptr;
        s.cap = 0;
        if (hipHostMalloc(&s.host, bytes, hipHostMallocDefault) != hipSuccess)
            return OSS_E_NOMEM;
        if (dev_alloc(&s.dev, bytes, ctx->alloc_stream) != hipSuccess) {
            s.dev = nullptr;
            return OSS_E_NOMEM;
        }
        s.cap = bytes;
    }
    return OSS_OK;
}

// Build the per-template plans.
static int make_plans(const oss_ref *ref, const oss_template_feat *tmpl, int32_t n_tmpl,
                      const oss_probe *probes, int32_t n_probes, const oss_tolerance *tol,
                      uint32_t fm, std::vector<DevTemplatePlan> &plans)
{
    int rc = check_probes(ref, n_tmpl, probes, n_probes);
    if (rc != OSS_OK)
        return rc;
    plans.assign(n_tmpl, DevTemplatePlan{});
    for (int t = 0; t < n_tmpl; ++t)
        template_plan(ref, tmpl[t], t, probes, n_probes, tol, fm, &plans[t]);
    return OSS_OK;
}

// Argument checks shared by the screens (before anything is launched).
int oss::check_screen_args(oss_ctx *ctx, const oss_ref *ref, const oss_template_feat *tmpl,
                             int32_t n_tmpl, const oss_probe *probes, int32_t n_probes,
                             const oss_tolerance *tol, uint32_t feat_mask, int64_t list_cap,
                             const oss_candidate *dev_list, const int64_t *dev_count)
{
    if (!ctx || !ref || !tmpl || n_tmpl <= 0 || (n_probes > 0 && !probes) || n_probes < 0 || !tol ||
        !dev_count || list_cap < 0 || (list_cap > 0 && !dev_list))
        return OSS_E_ARG;
    if (ref->ctx != ctx)
        return OSS_E_STATE;
    if (feat_mask == 0 || (feat_mask & ~ref->feat_mask) || (ref->feat_mask & OSS_F_MOMENTS))
        return OSS_E_ARG;
    if (tol->Q <= 0)
        return OSS_E_ARG;
    for (int f = 0; f < 3; ++f)
        if ((feat_mask & (1u << f)) && tol->P[f] < 0)
            return OSS_E_ARG;
    for (int t = 0; t < n_tmpl; ++t)
        if ((tmpl[t].feat_mask & feat_mask) != feat_mask || tmpl[t].rho < 0)
            return OSS_E_ARG;
    return OSS_OK;
}

int oss::screen_workspace(oss_ctx *ctx, int64_t n_tmpl, int H, int W, bool carry)
{
    if (carry) {
        int rc = grow(reinterpret_cast<void **>(&ctx->bits), &ctx->bits_cap,
                      (size_t)n_tmpl * H * W * sizeof(uint32_t), ctx->alloc_stream);
        if (rc != OSS_OK)
            return rc;
    }
    return grow(&ctx->ews, &ctx->ews_cap, emit_workspace_bytes(n_tmpl, H, W),
                ctx->alloc_stream);
}

EmitOut oss::emit_out(oss_ctx *ctx, int64_t n_tmpl, int H, int W, void **scan_ws)
{
    EmitOut eo{};
    emit_carve(ctx->ews, n_tmpl, H, W, &eo.seg_count, &eo.stage, scan_ws);
    eo.H = H;
    eo.W = W;
    eo.n_chunks = (W + SEG_W - 1) / SEG_W;
    return eo;
}

extern "C" int oss_screen(oss_ctx *ctx, const oss_ref *ref, const oss_template_feat *tmpl,
                          int32_t n_tmpl, const oss_probe *probes, int32_t n_probes,
                          const oss_tolerance *tol, uint32_t feat_mask, uint8_t *dev_mask,
                          oss_candidate *dev_list, int64_t list_cap, int64_t *dev_count,
                          void *stream)
{
    int rc = check_screen_args(ctx, ref, tmpl, n_tmpl, probes, n_probes, tol, feat_mask, list_cap,
                               dev_list, dev_count);
    if (rc != OSS_OK)
        return rc;
    std::vector<DevTemplatePlan> plans;
    rc = make_plans(ref, tmpl, n_tmpl, probes, n_probes, tol, feat_mask, plans);
    if (rc != OSS_OK)
        return rc;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return OSS_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const BuildGeom &g = ref->geom;
    const int64_t hw = (int64_t)g.H * g.W;
    const int strip = ctx->star_strip;
    rc = screen_workspace(ctx, n_tmpl, g.H, g.W, false);
    if (rc != OSS_OK)
        return rc;
    PlanSlot *slot = nullptr;
    rc = upload_plan(ctx, plans.data(), plans.size() * sizeof(DevTemplatePlan), st, &slot);
    if (rc != OSS_OK)
        return rc;
    const DevTemplatePlan *dplan = static_cast<const DevTemplatePlan *>(slot->dev);
    void *scan_ws = nullptr;
    const EmitOut all = emit_out(ctx, n_tmpl, g.H, g.W, &scan_ws);
    const int64_t segs_t = (int64_t)g.H * all.n_chunks;
    for (int t = 0; t < n_tmpl; ++t) {
        const StarSweep sw = make_sweep(g.H, g.W, strip, ctx->star_blocks_per_xcd);
        int smax = 0, rmax = 0;
        for (int j = 0; j < plans[t].n_radii; ++j) {
            smax = std::max(smax, (int)plans[t].radii[j].s);
            rmax = std::max(rmax, (int)plans[t].radii[j].r);
        }
        // template t's segments, staging slots and mask
        EmitOut eo = all;
        eo.mask = dev_mask ? dev_mask + hw * t : nullptr;
        eo.seg_count = all.seg_count + segs_t * t;
        eo.stage = all.stage + segs_t * SEG_W * t;
        hipError_t e = launch_star_plain(g, ref->bb.L, ref->bb.R, ref->bb.Rp, dplan + t, eo, sw,
                                         smax, rmax,
                                         ctx->star_lds ? 1 : ctx->star_pipe ? 2 : ctx->star_staged ? 3 : 0, st,
                                         &ctx->prof);
        if (e != hipSuccess)
            return OSS_E_DEVICE;
    }
    hipError_t e = launch_list(all.seg_count, all.stage, n_tmpl, g.H, g.W, dev_list, list_cap,
                               dev_count, scan_ws, st, &ctx->prof);
    if (e != hipSuccess)
        return OSS_E_DEVICE;
    if (hipEventRecord(slot->ev, st) != hipSuccess)
        return OSS_E_DEVICE;
    slot->used = true;
    return OSS_OK;
}

// ---------------------------------------------------------------------------
// Batched screen.
// ---------------------------------------------------------------------------
// Templates sorted by radius and cut into groups of BATCH_GROUP (with rings
// BATCH_GROUP_RINGS); each group's
// probes sorted by reference radius; every run of at most `bucket` distinct
// radii (0: all) becomes one pass.
// One entry of a template's part of a batched plan: a test at radius r
// with bounds per table slot, setting (ring 0) or vetoing (ring > 0) bit k.
struct PlanEntry {
    int r, k, ring;
    int64_t lo[3], hi[3];
};

// Groups of at most BATCH_GROUP (with rings BATCH_GROUP_RINGS) templates in
// `order`, each group's entries sorted by radius, passes over runs of at most
// `bucket` distinct radii.  bp.rings must be set.
static void build_groups(const std::vector<std::vector<PlanEntry>> &per,
                         const std::vector<int> &order, int bucket, BatchHostPlan &bp)
{
    const int n_tmpl = (int)order.size();
    const int gmax = bp.rings > 1 ? BATCH_GROUP_RINGS : BATCH_GROUP;
    for (int g0 = 0; g0 < n_tmpl; g0 += gmax) {
        const int nt = std::min(gmax, n_tmpl - g0);
        DevBatchGroup grp{};
        grp.n_t = nt;
        struct Item {
            int slot;
            const PlanEntry *e;
        };
        std::vector<Item> items;
        for (int i = 0; i < nt; ++i) {
            const int t = order[g0 + i];
            grp.tmap[i] = t;
            for (const PlanEntry &e : per[t])
                items.push_back({i, &e});
        }
        std::stable_sort(items.begin(), items.end(),
                         [](const Item &a, const Item &b) { return a.e->r < b.e->r; });
        const int gi = (int)bp.groups.size();
        bp.groups.push_back(grp);
        bp.max_group = std::max(bp.max_group, nt);
        const int rad_begin = (int)bp.radii.size();
        for (const Item &it : items) {
            const PlanEntry &e = *it.e;
            if ((int)bp.radii.size() == rad_begin || bp.radii.back().r != e.r) {
                DevBatchRadius rd{};
                rd.r = e.r;
                rd.s = square_half(e.r);
                rd.first = (int32_t)bp.probes.size();
                rd.count = 0;
                for (int q = 0; q < 3; ++q) {
                    rd.lo[q] = INT64_MAX;
                    rd.hi[q] = INT64_MIN;
                }
                bp.radii.push_back(rd);
            }
            DevBatchRadius &cur = bp.radii.back();
            cur.count++;
            DevBatchProbe dp{};
            dp.t = it.slot;
            dp.k = e.k;
            dp.ring = e.ring;
            for (int q = 0; q < 3; ++q) {
                dp.lo[q] = e.lo[q];
                dp.hi[q] = e.hi[q];
                // outside the hull every entry fails (central-star entries
                // then record their failure without the probe loop)
                cur.lo[q] = std::min(cur.lo[q], dp.lo[q]);
                cur.hi[q] = std::max(cur.hi[q], dp.hi[q]);
            }
            bp.probes.push_back(dp);
        }
        const int rad_end = (int)bp.radii.size();
        // each radius' core: the intersection of its probes' intervals, and
        // the scale bits its probes set per template slot
        for (int j = rad_begin; j < rad_end; ++j) {
            DevBatchRadius &rd = bp.radii[j];
            rd.cb_first = -1;
            bool core = bp.rings == 1;
            for (int q = 0; q < 3; ++q) {
                rd.clo[q] = INT64_MIN;
                rd.chi[q] = INT64_MAX;
            }
            for (int p = rd.first; p < rd.first + rd.count && core; ++p) {
                const DevBatchProbe &pr = bp.probes[p];
                for (int q = 0; q < 3; ++q) {
                    rd.clo[q] = std::max(rd.clo[q], pr.lo[q]);
                    rd.chi[q] = std::min(rd.chi[q], pr.hi[q]);
                    core = core && rd.clo[q] <= rd.chi[q];
                }
            }
            if (!core)
                continue;
            rd.cb_first = (int32_t)bp.core_bits.size();
            bp.core_bits.resize(bp.core_bits.size() + nt, 0u);
            for (int p = rd.first; p < rd.first + rd.count; ++p)
                bp.core_bits[rd.cb_first + bp.probes[p].t] |= 1u << bp.probes[p].k;
        }
        const int step = bucket > 0 ? bucket : std::max(1, rad_end - rad_begin);
        int j0 = rad_begin;
        do {
            const int j1 = std::min(rad_end, j0 + step);
            bp.passes.push_back({gi, j0, j1, j0 == rad_begin ? 1 : 0, j1 == rad_end ? 1 : 0, 0});
            j0 = j1;
        } while (j0 < rad_end);
    }
}

// Each radius' table-row offsets from row y-1: rows y-s-1, y+s, y-r-1, y+r.
static void set_row_offsets(const oss_ref *ref, BatchHostPlan &bp)
{
    const int64_t rb = ref->geom.pitch_e * ref->geom.tab_es;
    for (DevBatchRadius &rd : bp.radii) {
        rd.roff[0] = -(int64_t)rd.s * rb;
        rd.roff[1] = (int64_t)(rd.s + 1) * rb;
        rd.roff[2] = -(int64_t)rd.r * rb;
        rd.roff[3] = (int64_t)(rd.r + 1) * rb;
    }
}

// feature f -> table slot (the reference's quantities in bit order), -1 if absent
static void slots_of(uint32_t ref_fm, int slot_of[3])
{
    int slot = 0;
    for (int f = 0; f < 3; ++f)
        slot_of[f] = (ref_fm & (1u << f)) ? slot++ : -1;
}

int oss::make_batch_plan(const oss_ref *ref, const oss_template_feat *tmpl, int32_t n_tmpl,
                         const oss_probe *probes, int32_t n_probes, const oss_tolerance *tols,
                         const uint32_t *fms, int bucket, BatchHostPlan &bp, int n_rings)
{
    if (n_rings < 1 || n_rings > MAX_RINGS)
        return OSS_E_ARG;
    bp.rings = n_rings;
    bp.n_tmpl = n_tmpl;
    if (n_rings > 1)
        bucket = 0;  // the ring tests of a probe combine in registers: one pass
    std::vector<int> count(n_tmpl, 0);
    int slot_of[3];
    slots_of(ref->feat_mask, slot_of);
    std::vector<std::vector<PlanEntry>> per(n_tmpl);
    for (int i = 0; i < n_probes; ++i) {
        const oss_probe &p = probes[i];
        if (p.template_id < 0 || p.template_id >= n_tmpl || p.scale_id < 0 ||
            p.scale_id >= OSS_MAX_SCALES || p.r < 0 || p.r > ref->max_radius)
            return OSS_E_ARG;
        const int t = p.template_id;
        if (++count[t] > OSS_MAX_SCALES)
            return OSS_E_ARG;
        int rj = p.r;
        for (int j = 0; j < n_rings; ++j) {
            PlanEntry e{};
            e.r = rj;
            e.k = p.scale_id;
            e.ring = j;
            for (int q = 0; q < 3; ++q) {
                e.lo[q] = INT64_MIN;
                e.hi[q] = INT64_MAX;
            }
            const oss_template_feat &tf = tmpl[(int64_t)t * n_rings + j];
            const oss_tolerance &tol = tols[t];
            for (int f = 0; f < 3; ++f) {
                if (!(fms[t] & (1u << f)))
                    continue;
                feature_bounds(f, tf.F[f], rj, tf.rho, tol.P[f], tol.Q, &e.lo[slot_of[f]],
                               &e.hi[slot_of[f]]);
            }
            per[t].push_back(e);
            rj = square_half(rj);
        }
    }
    std::vector<int> order(n_tmpl);
    for (int t = 0; t < n_tmpl; ++t)
        order[t] = t;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return tmpl[(int64_t)a * n_rings].rho < tmpl[(int64_t)b * n_rings].rho;
    });
    build_groups(per, order, bucket, bp);
    set_row_offsets(ref, bp);
    return OSS_OK;
}

// Plan of caller-given interval probes (bounds in feature order).
static int make_interval_plan(const oss_ref *ref, int32_t n_tmpl, const oss_interval_probe *probes,
                              int32_t n_probes, uint32_t fm, int bucket, BatchHostPlan &bp)
{
    int slot_of[3];
    slots_of(ref->feat_mask, slot_of);
    bp.n_tmpl = n_tmpl;
    std::vector<std::vector<PlanEntry>> per(n_tmpl);
    for (int i = 0; i < n_probes; ++i) {
        const oss_interval_probe &p = probes[i];
        if (p.template_id < 0 || p.template_id >= n_tmpl || p.scale_id < 0 ||
            p.scale_id >= OSS_MAX_SCALES || p.r < 0 || p.r > ref->max_radius)
            return OSS_E_ARG;
        PlanEntry e{};
        e.r = p.r;
        e.k = p.scale_id;
        e.ring = 0;
        for (int q = 0; q < 3; ++q) {
            e.lo[q] = INT64_MIN;
            e.hi[q] = INT64_MAX;
        }
        for (int f = 0; f < 3; ++f) {
            if (!(fm & (1u << f)))
                continue;
            e.lo[slot_of[f]] = p.lo[f];
            e.hi[slot_of[f]] = p.hi[f];
        }
        per[p.template_id].push_back(e);
    }
    std::vector<int> order(n_tmpl);
    for (int t = 0; t < n_tmpl; ++t)
        order[t] = t;
    bp.rings = 1;
    build_groups(per, order, bucket, bp);
    set_row_offsets(ref, bp);
    return OSS_OK;
}

// Pack the plan into one upload; returns device pointers into the slot.
static int upload_batch_plan(oss_ctx *ctx, const BatchHostPlan &bp, uint8_t *const *masks,
                             hipStream_t st, BatchDevPlan *dev, PlanSlot **slot)
{
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t o_mask = 0;
    const size_t o_pass = al(o_mask + (size_t)std::max(1, bp.n_tmpl) * sizeof(uint8_t *));
    const size_t o_grp = al(o_pass + bp.passes.size() * sizeof(DevBatchPass));
    const size_t o_rad = al(o_grp + bp.groups.size() * sizeof(DevBatchGroup));
    const size_t o_prb = al(o_rad + bp.radii.size() * sizeof(DevBatchRadius));
    const size_t o_cb = al(o_prb + std::max<size_t>(1, bp.probes.size()) * sizeof(DevBatchProbe));
    const size_t total = al(o_cb + std::max<size_t>(1, bp.core_bits.size()) * sizeof(uint32_t));
    std::vector<char> buf(total, 0);
    if (masks)
        std::memcpy(buf.data() + o_mask, masks, (size_t)bp.n_tmpl * sizeof(uint8_t *));
    std::memcpy(buf.data() + o_pass, bp.passes.data(), bp.passes.size() * sizeof(DevBatchPass));
    std::memcpy(buf.data() + o_grp, bp.groups.data(), bp.groups.size() * sizeof(DevBatchGroup));
    std::memcpy(buf.data() + o_rad, bp.radii.data(), bp.radii.size() * sizeof(DevBatchRadius));
    std::memcpy(buf.data() + o_prb, bp.probes.data(), bp.probes.size() * sizeof(DevBatchProbe));
    std::memcpy(buf.data() + o_cb, bp.core_bits.data(), bp.core_bits.size() * sizeof(uint32_t));
    int rc = upload_plan(ctx, buf.data(), total, st, slot);
    if (rc != OSS_OK)
        return rc;
    const char *d = static_cast<const char *>((*slot)->dev);
    dev->mask_of = masks ? reinterpret_cast<uint8_t *const *>(d + o_mask) : nullptr;
    dev->passes = reinterpret_cast<const DevBatchPass *>(d + o_pass);
    dev->n_passes = (int)bp.passes.size();
    dev->groups = reinterpret_cast<const DevBatchGroup *>(d + o_grp);
    dev->radii = reinterpret_cast<const DevBatchRadius *>(d + o_rad);
    dev->probes = reinterpret_cast<const DevBatchProbe *>(d + o_prb);
    dev->core_bits = reinterpret_cast<const uint32_t *>(d + o_cb);
    dev->max_group = bp.max_group;
    dev->rings = bp.rings;
    return OSS_OK;
}

bool oss::plan_carries(const BatchHostPlan &bp)
{
    for (const DevBatchPass &p : bp.passes)
        if (!p.last)
            return true;
    return false;
}

// The batched star pass alone (mask, segment counts and staged candidates
// into the context's emission workspace).
int oss::batch_star(oss_ctx *ctx, const oss_ref *ref, const BatchHostPlan &bp, int strip,
                    int blocks, uint8_t *const *masks, hipStream_t st, PlanSlot **slot)
{
    BatchDevPlan dev{};
    int rc = upload_batch_plan(ctx, bp, masks, st, &dev, slot);
    if (rc != OSS_OK)
        return rc;
    const BuildGeom &g = ref->geom;
    const StarSweep sw = make_sweep(g.H, g.W, strip, blocks);
    void *scan_ws = nullptr;
    EmitOut eo = emit_out(ctx, bp.n_tmpl, g.H, g.W, &scan_ws);
    eo.dense = plan_carries(bp) ? ctx->bits : nullptr;
    if (launch_star_batch(g, ref->bb.L, ref->bb.R, ref->bb.Rp, dev, eo, sw,
                          ctx->star_staged != 0, st, &ctx->prof) != hipSuccess)
        return OSS_E_DEVICE;
    return OSS_OK;
}

// Per-template mask pointers of a screen's [n_tmpl][H][W] mask (empty: none).
static std::vector<uint8_t *> mask_ptrs(uint8_t *dev_mask, int32_t n_tmpl, int64_t hw)
{
    std::vector<uint8_t *> m;
    if (dev_mask)
        for (int t = 0; t < n_tmpl; ++t)
            m.push_back(dev_mask + hw * t);
    return m;
}

// Batched star pass + list for one screen over ctx's workspaces.
static int batched_screen(oss_ctx *ctx, const oss_ref *ref, const BatchHostPlan &bp,
                          uint8_t *dev_mask, oss_candidate *dev_list, int64_t list_cap,
                          int64_t *dev_count, hipStream_t st)
{
    const BuildGeom &g = ref->geom;
    const int strip = ctx->star_strip;
    int rc = screen_workspace(ctx, bp.n_tmpl, g.H, g.W, plan_carries(bp));
    if (rc != OSS_OK)
        return rc;
    const std::vector<uint8_t *> masks = mask_ptrs(dev_mask, bp.n_tmpl, (int64_t)g.H * g.W);
    PlanSlot *slot = nullptr;
    rc = batch_star(ctx, ref, bp, strip, ctx->star_blocks_per_xcd,
                    masks.empty() ? nullptr : masks.data(), st, &slot);
    if (rc != OSS_OK)
        return rc;
    void *scan_ws = nullptr;
    const EmitOut eo = emit_out(ctx, bp.n_tmpl, g.H, g.W, &scan_ws);
    if (launch_list(eo.seg_count, eo.stage, bp.n_tmpl, g.H, g.W, dev_list, list_cap, dev_count,
                    scan_ws, st, &ctx->prof) != hipSuccess)
        return OSS_E_DEVICE;
    if (hipEventRecord(slot->ev, st) != hipSuccess)
        return OSS_E_DEVICE;
    slot->used = true;
    return OSS_OK;
}

extern "C" int oss_screen_batched(oss_ctx *ctx, const oss_ref *ref,
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
    const std::vector<oss_tolerance> tols(n_tmpl, *tol);
    const std::vector<uint32_t> fms(n_tmpl, feat_mask);
    BatchHostPlan bp;
    rc = make_batch_plan(ref, tmpl, n_tmpl, probes, n_probes, tols.data(), fms.data(),
                         ctx->batch_bucket, bp);
    if (rc != OSS_OK)
        return rc;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return OSS_E_DEVICE;
    return batched_screen(ctx, ref, bp, dev_mask, dev_list, list_cap, dev_count,
                          static_cast<hipStream_t>(stream));
}

extern "C" int oss_screen_rings(oss_ctx *ctx, const oss_ref *ref, const oss_template_feat *tmpl,
                                int32_t n_tmpl, int32_t n_rings, const oss_probe *probes,
                                int32_t n_probes, const oss_tolerance *tol, uint32_t feat_mask,
                                uint8_t *dev_mask, oss_candidate *dev_list, int64_t list_cap,
                                int64_t *dev_count, void *stream)
{
    if (n_rings < 1 || n_rings > MAX_RINGS || n_tmpl <= 0 || !tmpl)
        return OSS_E_ARG;
    // the outer template features are checked like oss_screen's, the rings
    // for their feature set and radius
    std::vector<oss_template_feat> outer(n_tmpl);
    for (int t = 0; t < n_tmpl; ++t) {
        outer[t] = tmpl[(int64_t)t * n_rings];
        for (int j = 1; j < n_rings; ++j) {
            const oss_template_feat &f = tmpl[(int64_t)t * n_rings + j];
            if ((f.feat_mask & feat_mask) != feat_mask || f.rho < 0)
                return OSS_E_ARG;
        }
    }
    int rc = check_screen_args(ctx, ref, outer.data(), n_tmpl, probes, n_probes, tol, feat_mask,
                               list_cap, dev_list, dev_count);
    if (rc != OSS_OK)
        return rc;
    const std::vector<oss_tolerance> tols(n_tmpl, *tol);
    const std::vector<uint32_t> fms(n_tmpl, feat_mask);
    BatchHostPlan bp;
    rc = make_batch_plan(ref, tmpl, n_tmpl, probes, n_probes, tols.data(), fms.data(),
                         ctx->batch_bucket, bp, n_rings);
    if (rc != OSS_OK)
        return rc;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return OSS_E_DEVICE;
    return batched_screen(ctx, ref, bp, dev_mask, dev_list, list_cap, dev_count,
                          static_cast<hipStream_t>(stream));
}

// Empirical search over the batched launch's shape: each candidate (strip
// width, blocks per XCD, radius bucket) runs the star pass once to warm up
// and once timed with HIP events on `stream`; the fastest is kept in the
// context's options.
extern "C" int oss_autotune_batched(oss_ctx *ctx, const oss_ref *ref,
                                    const oss_template_feat *tmpl, int32_t n_tmpl,
                                    const oss_probe *probes, int32_t n_probes,
                                    const oss_tolerance *tol, uint32_t feat_mask, void *stream,
                                    oss_tune_result *out)
{
    const int64_t dummy_count = 0;
    int rc = check_screen_args(ctx, ref, tmpl, n_tmpl, probes, n_probes, tol, feat_mask, 0,
                               nullptr, &dummy_count);
    if (rc != OSS_OK)
        return rc;
    if (!out)
        return OSS_E_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return OSS_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const BuildGeom &g = ref->geom;
    // distinct radii per group bound the useful bucket sizes
    const std::vector<oss_tolerance> tols(n_tmpl, *tol);
    const std::vector<uint32_t> fms(n_tmpl, feat_mask);
    BatchHostPlan whole;
    rc = make_batch_plan(ref, tmpl, n_tmpl, probes, n_probes, tols.data(), fms.data(), 0, whole);
    if (rc != OSS_OK)
        return rc;
    int max_radii = 0;
    for (const DevBatchPass &p : whole.passes)
        max_radii = std::max(max_radii, p.j1 - p.j0);
    const int strips[] = {256, 512};
    const int blocks[] = {32, 64, 128};
    std::vector<int> buckets = {0};
    for (int b : {16, 8, 4})
        if (b < max_radii)
            buckets.push_back(b);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return OSS_E_DEVICE;
    std::memset(out, 0, sizeof(*out));
    float best = 1e30f;
    int n = 0;
    rc = OSS_OK;
    for (int bk : buckets) {
        BatchHostPlan bp;
        rc = make_batch_plan(ref, tmpl, n_tmpl, probes, n_probes, tols.data(), fms.data(), bk,
                             bp);
        if (rc != OSS_OK)
            break;
        for (int sp : strips) {
            rc = screen_workspace(ctx, n_tmpl, g.H, g.W, plan_carries(bp));
            if (rc != OSS_OK)
                break;
            for (int bl : blocks) {
                PlanSlot *slot = nullptr;
                rc = batch_star(ctx, ref, bp, sp, bl, nullptr, st, &slot);  // warm-up
                if (rc != OSS_OK)
                    break;
                if (hipEventRecord(e0, st) != hipSuccess) {
                    rc = OSS_E_DEVICE;
                    break;
                }
                rc = batch_star(ctx, ref, bp, sp, bl, nullptr, st, &slot);
                if (rc != OSS_OK)
                    break;
                float ms = 0.f;
                if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    rc = OSS_E_DEVICE;
                    break;
                }
                if (n < OSS_TUNE_MAX) {
                    out->tried[n][0] = sp;
                    out->tried[n][1] = bl;
                    out->tried[n][2] = bk;
                    out->tried_ms[n] = ms;
                    ++n;
                }
                if (ms < best) {
                    best = ms;
                    out->strip = sp;
                    out->blocks_per_xcd = bl;
                    out->bucket_radii = bk;
                }
            }
            if (rc != OSS_OK)
                break;
        }
        if (rc != OSS_OK)
            break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != OSS_OK)
        return rc;
    out->n_tried = n;
    out->ms = best;
    ctx->star_strip = out->strip;
    ctx->star_blocks_per_xcd = out->blocks_per_xcd;
    ctx->batch_bucket = out->bucket_radii;
    return OSS_OK;
}

// ---------------------------------------------------------------------------
// Preserved region (dilation of the candidates by their stars through the
// tables of a zero-padded indicator image; see csrc/region.hip).
// ---------------------------------------------------------------------------
extern "C" int oss_region(oss_ctx *ctx, int32_t H, int32_t W, int32_t n_tmpl,
                          const oss_probe *probes, int32_t n_probes, const oss_candidate *dev_list,
                          int64_t list_cap, const int64_t *dev_count, uint8_t *dev_region,
                          void *stream)
{
    if (!ctx || H <= 0 || W <= 0 || n_tmpl <= 0 || n_probes < 0 || (n_probes > 0 && !probes) ||
        list_cap < 0 || (list_cap > 0 && !dev_list) || !dev_count || !dev_region)
        return OSS_E_ARG;
    // scale bits of each (template, radius); radii that cannot fit carry no candidates
    std::vector<std::pair<std::pair<int, int>, uint32_t>> groups;
    int R = 0;
    for (int i = 0; i < n_probes; ++i) {
        const oss_probe &p = probes[i];
        if (p.template_id < 0 || p.template_id >= n_tmpl || p.scale_id < 0 ||
            p.scale_id >= OSS_MAX_SCALES || p.r < 0)
            return OSS_E_ARG;
        if (2 * (int64_t)p.r + 1 > std::min(H, W))
            continue;
        const std::pair<int, int> key(p.template_id, p.r);
        auto it = std::find_if(groups.begin(), groups.end(),
                               [&](const auto &g) { return g.first == key; });
        if (it == groups.end())
            groups.push_back({key, 1u << p.scale_id});
        else
            it->second |= 1u << p.scale_id;
        R = std::max(R, (int)p.r);
    }
    if (hipSetDevice(ctx->device) != hipSuccess)
        return OSS_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMemsetAsync(dev_region, 0, (size_t)n_tmpl * H * W, st) != hipSuccess)
        return OSS_E_DEVICE;
    if (groups.empty())
        return OSS_OK;
    const int Hp = H + 2 * R, Wp = W + 2 * R;
    const oss_image_desc d{Hp, Wp, (int64_t)Wp, OSS_U8, 1};
    const BuildGeom g = ref_geom(&d, OSS_F_SUM, R, 0);
    size_t off[A_COUNT];
    const size_t tb = ref_layout(g, off);
    const size_t o_ind = (tb + 255) / 256 * 256;
    const size_t o_hit = o_ind + ((size_t)Hp * Wp + 255) / 256 * 256;
    const size_t total = o_hit + (size_t)Hp * Wp;
    int rc = grow(&ctx->rws, &ctx->rws_cap, total, ctx->alloc_stream);
    if (rc != OSS_OK)
        return rc;
    char *m = static_cast<char *>(ctx->rws);
    BuildBuffers bb{};
    bb.L = m + off[A_L] + g.tab_off;
    bb.R = m + off[A_R] + g.tab_off;
    bb.Rp = m + off[A_RP] + g.tab_off;
    bb.bp = m + off[A_BP];
    bb.agg_L = m + off[A_AGL];
    bb.agg_AD = m + off[A_AGAD];
    bb.agg_D = m + off[A_AGD];
    bb.c_L = m + off[A_CL];
    bb.c_AD = m + off[A_CAD];
    bb.c_D = m + off[A_CD];
    uint8_t *ind = reinterpret_cast<uint8_t *>(m + o_ind);
    uint8_t *hit = reinterpret_cast<uint8_t *>(m + o_hit);
    const StarSweep sw = make_sweep(Hp, Wp, ctx->star_strip, ctx->star_blocks_per_xcd);
    for (const auto &grp : groups) {
        const int t = grp.first.first, r = grp.first.second;
        if (hipMemsetAsync(ind, 0, (size_t)Hp * Wp, st) != hipSuccess ||
            launch_region_scatter(dev_list, list_cap, dev_count, t, grp.second, H, W, R, Wp, ind,
                                  st) !=
                hipSuccess ||
            launch_build(g, ind, Wp, OSS_U8, OSS_F_SUM, bb, st, &ctx->prof) != hipSuccess)
            return OSS_E_DEVICE;
        // one radius, one interval: star sum of the indicator >= 1
        DevTemplatePlan pl{};
        pl.n_radii = 1;
        pl.radii[0].r = r;
        pl.radii[0].s = square_half(r);
        pl.radii[0].first = 0;
        pl.radii[0].count = 1;
        for (int q = 0; q < 3; ++q) {
            pl.probes[0].lo[q] = INT64_MIN;
            pl.probes[0].hi[q] = INT64_MAX;
        }
        pl.probes[0].lo[0] = 1;
        pl.probes[0].k = 0;
        PlanSlot *slot = nullptr;
        rc = upload_plan(ctx, &pl, sizeof(pl), st, &slot);
        if (rc != OSS_OK)
            return rc;
        // the star pass's mask alone: hit[y][x] = 1 where the star holds a candidate
        EmitOut eo{};
        eo.mask = hit;
        eo.H = Hp;
        eo.W = Wp;
        eo.n_chunks = (Wp + SEG_W - 1) / SEG_W;
        if (launch_star_plain(g, bb.L, bb.R, bb.Rp, static_cast<const DevTemplatePlan *>(slot->dev),
                              eo, sw, 0, 0, ctx->star_pipe ? 2 : 0, st, &ctx->prof) !=
                hipSuccess ||
            hipEventRecord(slot->ev, st) != hipSuccess)
            return OSS_E_DEVICE;
        slot->used = true;
        if (launch_region_or(hit, H, W, R, Wp, dev_region + (int64_t)t * H * W, st) != hipSuccess)
            return OSS_E_DEVICE;
    }
    return OSS_OK;
}

// ---------------------------------------------------------------------------
// Interval probes and Algorithm 1's template side.
// ---------------------------------------------------------------------------
extern "C" int oss_screen_intervals(oss_ctx *ctx, const oss_ref *ref, int32_t n_tmpl,
                                    const oss_interval_probe *probes, int32_t n_probes,
                                    uint32_t feat_mask, uint8_t *dev_mask,
                                    oss_candidate *dev_list, int64_t list_cap, int64_t *dev_count,
                                    void *stream)
{
    if (!ctx || !ref || n_tmpl <= 0 || n_probes < 0 || (n_probes > 0 && !probes) ||
        !dev_count || list_cap < 0 || (list_cap > 0 && !dev_list))
        return OSS_E_ARG;
    if (ref->ctx != ctx)
        return OSS_E_STATE;
    if (feat_mask == 0 || (feat_mask & ~ref->feat_mask) || (ref->feat_mask & OSS_F_MOMENTS))
        return OSS_E_ARG;
    BatchHostPlan bp;
    int rc = make_interval_plan(ref, n_tmpl, probes, n_probes, feat_mask, ctx->batch_bucket, bp);
    if (rc != OSS_OK)
        return rc;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return OSS_E_DEVICE;
    return batched_screen(ctx, ref, bp, dev_mask, dev_list, list_cap, dev_count,
                          static_cast<hipStream_t>(stream));
}

namespace {

uint64_t isqrt_u64(unsigned __int128 v)
{
    uint64_t x = (uint64_t)std::sqrt((long double)v);
    while ((unsigned __int128)x * x > v)
        --x;
    while ((unsigned __int128)(x + 1) * (x + 1) <= v)
        ++x;
    return x;
}

// floor(a / (d sqrt2^e)) and its ceiling, a >= 0, d > 0: exact (an odd
// power leaves sqrt(2 a^2), irrational for a > 0, so never an integer).
int64_t floor_sqrt2(int64_t a, int64_t d, int e)
{
    if (e % 2 == 0)
        return a / (d << (e / 2));
    return (int64_t)(isqrt_u64((unsigned __int128)2 * a * a) / (uint64_t)(d << ((e + 1) / 2)));
}

int64_t ceil_sqrt2(int64_t a, int64_t d, int e)
{
    if (e % 2 == 0) {
        const int64_t den = d << (e / 2);
        return (a + den - 1) / den;
    }
    return a == 0 ? 0 : floor_sqrt2(a, d, e) + 1;
}

// Bilinear n x n -> k x k, pixel centres aligned, edges replicated, rounded
// half up; weights in units of 1/(2k), exact integers.  Only the window of
// rows and columns [w0, w0 + ws) of the k x k result is formed, as a ws x ws
// image.
void resize_square(const std::vector<int64_t> &src, int n, int k, int w0, int ws,
                   std::vector<uint16_t> &dst)
{
    std::vector<int> i0(k), i1(k);
    std::vector<int64_t> w(k);
    const int64_t D = 2 * (int64_t)k;
    for (int i = 0; i < k; ++i) {
        const int64_t num = (2 * (int64_t)i + 1) * n - k;  // source coordinate times 2k
        int64_t x0 = 0, wx = 0;
        if (num >= 0) {
            x0 = num / D;
            wx = num % D;
        }
        if (x0 >= n - 1) {
            x0 = n - 1;
            wx = 0;
        }
        i0[i] = (int)x0;
        i1[i] = (int)std::min<int64_t>(x0 + 1, n - 1);
        w[i] = wx;
    }
    dst.assign((size_t)ws * ws, 0);
    const int64_t den = D * D;
    for (int y = w0; y < w0 + ws; ++y) {
        for (int x = w0; x < w0 + ws; ++x) {
            const int64_t t0 = (D - w[x]) * src[(size_t)i0[y] * n + i0[x]] +
                               w[x] * src[(size_t)i0[y] * n + i1[x]];
            const int64_t t1 = (D - w[x]) * src[(size_t)i1[y] * n + i0[x]] +
                               w[x] * src[(size_t)i1[y] * n + i1[x]];
            const int64_t v = (D - w[y]) * t0 + w[y] * t1;
            dst[(size_t)(y - w0) * ws + (x - w0)] = (uint16_t)((2 * v + den) / (2 * den));
        }
    }
}

}  // namespace

extern "C" int oss_alg1_probes(const void *host_pixels, const oss_image_desc *desc, int32_t t,
                               const oss_alg1_params *p, oss_interval_probe *out, int32_t cap,
                               int32_t *n_out)
{
    if (!host_pixels || !desc_ok(desc) || !p || !n_out || cap < 0 || (cap > 0 && !out) ||
        t < 0 || desc->H != desc->W || p->alpha_num <= 0 || p->alpha_den <= 0 ||
        p->beta_num <= 0 || p->beta_den <= 0 || p->feat_mask == 0 ||
        (p->feat_mask & ~OSS_F_ALL))
        return OSS_E_ARG;
    // alpha <= beta
    if ((int64_t)p->alpha_num * p->beta_den > (int64_t)p->beta_num * p->alpha_den)
        return OSS_E_ARG;
    for (int f = 0; f < 3; ++f)
        if ((p->feat_mask & (1u << f)) && p->q[f] <= 0)
            return OSS_E_ARG;
    const int n = desc->W;
    // B: smallest with 2^B (alpha_num beta_den)^2 >= (beta_num alpha_den)^2
    const __int128 num2 = (__int128)p->beta_num * p->alpha_den * p->beta_num * p->alpha_den;
    const __int128 den2 = (__int128)p->alpha_num * p->beta_den * p->alpha_num * p->beta_den;
    int B = 0;
    while (((__int128)den2 << B) < num2) {
        if (++B > OSS_MAX_SCALES)
            return OSS_E_ARG;
    }
    // the template as int64 pixels
    std::vector<int64_t> px((size_t)n * n);
    const unsigned char *base = static_cast<const unsigned char *>(host_pixels);
    for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) {
            const unsigned char *row = base + (int64_t)y * desc->pitch_bytes;
            if (desc->dtype == OSS_U8) {
                px[(size_t)y * n + x] = row[x];
            } else {
                uint16_t v;
                std::memcpy(&v, row + 2 * (int64_t)x, 2);
                px[(size_t)y * n + x] = v;
            }
        }
    const int64_t a = (int64_t)p->beta_num * n, d = p->beta_den;  // beta n = a / d
    // every (band, size) item: the template resized to k x k, the features of
    // the central star of its band's radius, the probe of its quantised cell
    struct Item {
        int b, m, r;
        int64_t k, A;
    };
    std::vector<Item> items;
    for (int b = 0; b < B; ++b) {
        const int64_t k_lo = ceil_sqrt2(a, d, b + 1), k_hi = floor_sqrt2(a, d, b);
        const int m = (int)k_lo;
        if (m < 1)
            continue;
        const int r = (m - 1) / 2;
        for (int64_t k = k_lo; k <= k_hi; ++k)
            items.push_back({b, m, r, k, star_area(r)});
    }
    std::vector<oss_interval_probe> per(items.size());
    auto work = [&](size_t i) {
        const Item &it = items[i];
        const int64_t k = it.k;
        const int m = it.m, r = it.r;
        // the star at the crop centre c reads [c - r, c + r] and, for the
        // gradient, one more pixel each way (clamped to the k x k image):
        // a window that holds those is exact, its clamping the image's
        const int c = (int)((k - m) / 2 + (m - 1) / 2);
        const int w0 = std::max(0, c - r - 1);
        const int ws = std::min((int)k - 1, c + r + 1) - w0 + 1;
        std::vector<uint16_t> Y;
        resize_square(px, n, (int)k, w0, ws, Y);
        oss_image_desc yd{ws, ws, 2 * (int64_t)ws, OSS_U16, 16};
        int64_t F[3];
        star_feats_at(Y.data(), &yd, c - w0, c - w0, r, p->feat_mask, F);
        oss_interval_probe pr{};
        pr.template_id = t;
        pr.scale_id = it.b;
        pr.r = r;
        for (int f = 0; f < 3; ++f) {
            pr.lo[f] = INT64_MIN;
            pr.hi[f] = INT64_MAX;
            if (!(p->feat_mask & (1u << f)))
                continue;
            const int64_t q = (int64_t)p->q[f] * it.A;
            const int64_t c0 = F[f] / q;  // F >= 0: floor(F / q)
            pr.lo[f] = q * c0 - q / 2;
            pr.hi[f] = q * (c0 + 2) - q / 2 - 1;
        }
        per[i] = pr;
    };
    // the items on a few host threads (each writes only its own slot)
    const size_t nthr = std::min<size_t>({items.size(), 8,
                                          std::max(1u, std::thread::hardware_concurrency())});
    if (nthr <= 1) {
        for (size_t i = 0; i < items.size(); ++i)
            work(i);
    } else {
        std::atomic<size_t> next{0};
        std::vector<std::thread> pool;
        for (size_t w = 0; w < nthr; ++w)
            pool.emplace_back([&]() {
                for (size_t i = next++; i < items.size(); i = next++)
                    work(i);
            });
        for (auto &th : pool)
            th.join();
    }
    // in (band, size) order, one probe per distinct interval set of a band
    std::vector<oss_interval_probe> res;
    size_t band_first = 0;
    for (size_t i = 0; i < items.size(); ++i) {
        if (i == 0 || items[i].b != items[i - 1].b)
            band_first = res.size();
        const oss_interval_probe &pr = per[i];
        bool dup = false;
        for (size_t j = band_first; j < res.size() && !dup; ++j)
            dup = std::memcmp(res[j].lo, pr.lo, sizeof(pr.lo)) == 0 &&
                  std::memcmp(res[j].hi, pr.hi, sizeof(pr.hi)) == 0;
        if (!dup)
            res.push_back(pr);
    }
    *n_out = (int32_t)res.size();
    if ((int64_t)res.size() > cap)
        return OSS_E_NOMEM;
    std::copy(res.begin(), res.end(), out);
    return OSS_OK;
}

// ---------------------------------------------------------------------------
// The paper's own features: template moments and the moments screen.
// ---------------------------------------------------------------------------
extern "C" int oss_template_moments(const void *host_pixels, const oss_image_desc *desc,
                                    int32_t rho, oss_template_mom *out)
{
    if (!host_pixels || !out || !desc_ok(desc))
        return OSS_E_ARG;
    const int H = desc->H, W = desc->W;
    const int cx = (W - 1) / 2, cy = (H - 1) / 2;
    const int rmax = std::min(std::min(cx, W - 1 - cx), std::min(cy, H - 1 - cy));
    if (rho < 0)
        rho = rmax;
    if (rho > rmax)
        return OSS_E_ARG;
    const unsigned char *base = static_cast<const unsigned char *>(host_pixels);
    auto pix = [&](int x, int y) -> int64_t {
        const unsigned char *row = base + (int64_t)y * desc->pitch_bytes;
        if (desc->dtype == OSS_U8)
            return row[x];
        uint16_t v;
        std::memcpy(&v, row + 2 * (int64_t)x, 2);
        return v;
    };
    int64_t f1 = 0, f2 = 0, mx = 0, my = 0;
    auto span = [&](int dy, int h) {  // the row cy + dy, columns cx - h .. cx + h
        for (int dx = -h; dx <= h; ++dx) {
            const int64_t v = pix(cx + dx, cy + dy);
            f1 += v;
            f2 += v * v;
            mx += dx * v;
            my += dy * v;
        }
    };
    const int s = square_half(rho);
    for (int dy = -s; dy <= s; ++dy)
        span(dy, s);
    for (int dy = -rho; dy <= rho; ++dy)
        span(dy, rho - (dy < 0 ? -dy : dy));
    out->F1 = f1;
    out->F2 = f2;
    out->Sx = mx;
    out->Sy = my;
    out->rho = rho;
    out->pad = 0;
    return OSS_OK;
}

namespace {

using u128 = unsigned __int128;

int64_t ceil_div_i128(__int128 a, __int128 b)  // b > 0
{
    __int128 q = a / b;
    if (a % b != 0 && a > 0)
        ++q;
    return (int64_t)std::max<__int128>(INT64_MIN, std::min<__int128>(INT64_MAX, q));
}

int64_t floor_div_i128(__int128 a, __int128 b)  // b > 0
{
    __int128 q = a / b;
    if (a % b != 0 && a < 0)
        --q;
    return (int64_t)std::max<__int128>(INT64_MIN, std::min<__int128>(INT64_MAX, q));
}

// a * b * c with a 128-bit overflow check (false on overflow)
bool mul3(u128 a, u128 b, u128 c, u128 *out)
{
    const long double est = (long double)a * (long double)b * (long double)c;
    if (est > 1.7e38L)
        return false;
    *out = a * b * c;
    return true;
}

void put128(uint64_t w[2], u128 v)
{
    w[0] = (uint64_t)v;
    w[1] = (uint64_t)(v >> 64);
}

}  // namespace

extern "C" int oss_screen_moments(oss_ctx *ctx, const oss_ref *ref, const oss_template_mom *tmpl,
                                  int32_t n_tmpl, const oss_probe *probes, int32_t n_probes,
                                  const oss_tolerance *tol, uint32_t tests, uint8_t *dev_mask,
                                  oss_candidate *dev_list, int64_t list_cap, int64_t *dev_count,
                                  void *stream)
{
    if (!ctx || !ref || !tmpl || n_tmpl <= 0 || n_probes < 0 || (n_probes > 0 && !probes) ||
        !tol || !dev_count || list_cap < 0 || (list_cap > 0 && !dev_list))
        return OSS_E_ARG;
    if (ref->ctx != ctx)
        return OSS_E_STATE;
    if (!(ref->feat_mask & OSS_F_MOMENTS) || tests == 0 || (tests & ~7u) ||
        ((tests & OSS_T_VAR) && !(ref->feat_mask & OSS_F_SQ)) || tol->Q <= 0)
        return OSS_E_ARG;
    for (int f = 0; f < 3; ++f)
        if ((tests & (1u << f)) && tol->P[f] < 0)
            return OSS_E_ARG;
    for (int t = 0; t < n_tmpl; ++t)
        if (tmpl[t].rho < 0 || tmpl[t].F1 < 0 || tmpl[t].F2 < 0)
            return OSS_E_ARG;
    std::vector<DevMomPlan> plans(n_tmpl, DevMomPlan{});
    std::vector<std::vector<oss_probe>> per(n_tmpl);
    for (int i = 0; i < n_probes; ++i) {
        const oss_probe &p = probes[i];
        if (p.template_id < 0 || p.template_id >= n_tmpl || p.scale_id < 0 ||
            p.scale_id >= OSS_MAX_SCALES || p.r < 0 || p.r > ref->max_radius)
            return OSS_E_ARG;
        per[p.template_id].push_back(p);
        if ((int)per[p.template_id].size() > OSS_MAX_SCALES)
            return OSS_E_ARG;
    }
    const __int128 Q = tol->Q;
    const int64_t maxv = ((int64_t)1 << ref->desc.bit_depth) - 1;  // largest pixel value
    for (int t = 0; t < n_tmpl; ++t) {
        auto &v = per[t];
        std::stable_sort(v.begin(), v.end(),
                         [](const oss_probe &a, const oss_probe &b) { return a.r < b.r; });
        const oss_template_mom &T = tmpl[t];
        const __int128 A_rho = star_area(T.rho);
        const __int128 VT = A_rho * T.F2 - (__int128)T.F1 * T.F1;
        const u128 MT = (u128)((__int128)T.Sx * T.Sx) + (u128)((__int128)T.Sy * T.Sy);
        const u128 N_rho = (u128)T.rho * (u128)A_rho;
        DevMomPlan &pl = plans[t];
        int nr = 0;
        for (size_t i = 0; i < v.size(); ++i) {
            const int r = v[i].r;
            if (nr == 0 || pl.radii[nr - 1].r != r) {
                pl.radii[nr].r = r;
                pl.radii[nr].s = square_half(r);
                pl.radii[nr].first = (int32_t)i;
                pl.radii[nr].count = 0;
                ++nr;
            }
            pl.radii[nr - 1].count++;
            DevMomProbe &dp = pl.probes[i];
            dp.k = v[i].scale_id;
            dp.tests = (int32_t)tests;
            const __int128 A_r = star_area(r);
            feature_bounds(0, T.F1, r, T.rho, tol->P[0], tol->Q, &dp.lo1, &dp.hi1);
            if (tests & OSS_T_VAR) {
                // the kernel forms V = A(r) F2 - F1^2 in int64: both terms are
                // at most A(r)^2 maxv^2, which must stay below 2^63
                const long double a2m2 = (long double)A_r * (long double)A_r *
                                         (long double)maxv * (long double)maxv;
                if (a2m2 >= 9.2e18L)
                    return OSS_E_OVERFLOW;
            }
            // variance: (Q-P) VT A(r)^2 <= Q V A(rho)^2 <= (Q+P) VT A(r)^2,
            // the products checked against 128 bits (VT >= 0)
            const __int128 den_v = Q * A_rho * A_rho;
            const u128 vt = VT > 0 ? (u128)VT : 0;
            const u128 ar2 = (u128)A_r * (u128)A_r;
            const __int128 qmv = Q - tol->P[1];
            u128 lo_v = 0, hi_v = 0;
            if (!mul3((u128)(Q + tol->P[1]), vt, ar2, &hi_v) ||
                !mul3(qmv > 0 ? (u128)qmv : 0, vt, ar2, &lo_v))
                return OSS_E_OVERFLOW;
            dp.loV = qmv > 0 ? ceil_div_i128((__int128)lo_v, den_v) : INT64_MIN;
            dp.hiV = floor_div_i128((__int128)hi_v, den_v);
            // magnitude: (Q-P)^2 MT N(r)^2 <= Q^2 M N(rho)^2 <= (Q+P)^2 MT N(r)^2
            const u128 N_r = (u128)r * (u128)A_r;
            const u128 qp = (u128)(Q + tol->P[2]), qm = Q >= tol->P[2] ? (u128)(Q - tol->P[2]) : 0;
            u128 hi_num = 0, lo_num = 0;
            if (!mul3(qp * qp, MT, N_r * N_r, &hi_num) || !mul3(qm * qm, MT, N_r * N_r, &lo_num))
                return OSS_E_OVERFLOW;
            const long double den_est = (long double)(Q * Q) * (long double)N_rho *
                                        (long double)N_rho;
            if (den_est > 1.7e38L)
                return OSS_E_OVERFLOW;
            const u128 den_m = (u128)(Q * Q) * N_rho * N_rho;
            if (den_m == 0) {
                // rho = 0: the middle term is 0 whatever M is
                const bool ok = lo_num == 0;
                put128(dp.loM, ok ? 0 : 1);
                put128(dp.hiM, ok ? ~(u128)0 : 0);
            } else {
                put128(dp.loM, lo_num / den_m + (lo_num % den_m != 0 ? 1 : 0));
                put128(dp.hiM, hi_num / den_m);
            }
        }
        pl.n_radii = nr;
    }
    if (hipSetDevice(ctx->device) != hipSuccess)
        return OSS_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const BuildGeom &g = ref->geom;
    const int64_t hw = (int64_t)g.H * g.W;
    const int strip = ctx->star_strip;
    int rc = screen_workspace(ctx, n_tmpl, g.H, g.W, false);
    if (rc != OSS_OK)
        return rc;
    PlanSlot *slot = nullptr;
    rc = upload_plan(ctx, plans.data(), plans.size() * sizeof(DevMomPlan), st, &slot);
    if (rc != OSS_OK)
        return rc;
    const DevMomPlan *dplan = static_cast<const DevMomPlan *>(slot->dev);
    const StarSweep sw = make_sweep(g.H, g.W, strip, ctx->star_blocks_per_xcd);
    void *scan_ws = nullptr;
    const EmitOut all = emit_out(ctx, n_tmpl, g.H, g.W, &scan_ws);
    const int64_t segs_t = (int64_t)g.H * all.n_chunks;
    for (int t = 0; t < n_tmpl; ++t) {
        EmitOut eo = all;
        eo.mask = dev_mask ? dev_mask + hw * t : nullptr;
        eo.seg_count = all.seg_count + segs_t * t;
        eo.stage = all.stage + segs_t * SEG_W * t;
        if (launch_star_moments(g, ref->feat_mask, ref->bb.L, ref->bb.R, ref->bb.Rp, dplan + t,
                                eo, sw, st, &ctx->prof) != hipSuccess)
            return OSS_E_DEVICE;
    }
    if (launch_list(all.seg_count, all.stage, n_tmpl, g.H, g.W, dev_list, list_cap, dev_count,
                    scan_ws, st, &ctx->prof) != hipSuccess)
        return OSS_E_DEVICE;
    if (hipEventRecord(slot->ev, st) != hipSuccess)
        return OSS_E_DEVICE;
    slot->used = true;
    return OSS_OK;
}
