/*
 * oss.h - octagonal-star screening library for AMD Instinct MI355X (gfx950).
 *
 * A pre-screen for rotation- and scale-invariant template matching
 * (Liu, Shu & Wu, "Fast Screening Algorithm for Rotation and Scale
 * Invariant Template Matching", Algorithm 1): every position of a reference
 * image whose octagonal-star patch features cannot match a template's, at
 * any of the probed scales, is ruled out.  The survivors are returned as a
 * per-template mask and as a list of candidates.
 *
 * Definitions used throughout (pixel (x, y): column x, row y, 0-based):
 *   star of radius r     superposition of the diamond |dx|+|dy| <= r and
 *                        the congruent square max(|dx|,|dy|) <= s(r),
 *                        s(r) = max{ s : (2s-1)^2 < 2 r^2 } = round(r/sqrt 2)
 *                        (Sec. "Rotation Invariance", Fig. os, Eq. S_os);
 *                        pixels in both count twice.  Weighted area
 *                        A(r) = (2 s(r)+1)^2 + 2 r^2 + 2 r + 1.
 *   features             F_q(x,y,r) = sum of q over the star for the
 *                        quantities q = I (OSS_F_SUM), I^2 (OSS_F_SQ) and
 *                        G = |I(x+1,y)-I(x-1,y)| + |I(x,y+1)-I(x,y-1)|
 *                        (OSS_F_GRAD, indices clamped to the image)
 *                        (Sec. "Patch Features"; Sec. "Rotation Invariance"
 *                        for the rotation-robust gradient magnitude).
 *   valid position       the star fits: r <= x <= W-1-r and r <= y <= H-1-r.
 *   probe (t, k, r)      template t screened at reference radius r; k is
 *                        the scale's bit in the candidate's scale bits.
 *   feature test         with rho the template's radius, (c_ref, c_T) =
 *                        (r, rho) for the gradient and (1, 1) otherwise,
 *                        X_ref = F(x,y,r) A(rho) c_ref, X_T = F_T A(r) c_T:
 *                        pass iff (Q-P) X_T <= Q X_ref <= (Q+P) X_T, exact.
 *                        A probe passes where the position is valid and
 *                        every compared feature passes (Algorithm 1, patch
 *                        loop; Sec. "Scale Invariance", set membership with
 *                        an exact relative interval in place of the
 *                        quantised membership array).
 *
 * Conventions.  Every call returns an int status: OSS_OK (0) or a negative
 * OSS_E_* code; oss_status_string names it.  No C++ exception crosses this
 * interface.  Argument errors are reported before anything is launched.
 * "stream" arguments are hipStream_t values passed as void* (NULL = the
 * null stream); work is enqueued asynchronously on that stream.  The
 * caller owns every pixel, mask, list and count buffer; the library owns
 * the oss_ctx / oss_ref handles and the device memory behind them.  A
 * context's internal workspaces are reused by every screen issued on it, so
 * issue the calls of one context on one stream (or synchronise between
 * streams); use one context per concurrently used stream.
 */
#ifndef OSS_H
#define OSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define OSS_OK 0
#define OSS_E_ARG (-1)      /* invalid argument (null, range, shape, dtype) */
#define OSS_E_NOMEM (-2)    /* device or pinned host allocation failed */
#define OSS_E_OVERFLOW (-3) /* an integer table could overflow int64 */
#define OSS_E_DEVICE (-4)   /* a HIP runtime call failed */
#define OSS_E_STATE (-5)    /* handle used with the wrong context or shape */
#define OSS_E_LIMIT (-6)    /* the call needs more than a fixed capacity (the scratch of
                             * oss_screen_noalloc) */
#define OSS_E_CANCELLED (-7) /* a queued serving request cancelled by the caller */
#define OSS_E_TIMEOUT (-8)   /* a serving request queued longer than the server's limit */

/* pixel types */
#define OSS_U8 0
#define OSS_U16 1

/* feature bits */
#define OSS_F_SUM 1u
#define OSS_F_SQ 2u
#define OSS_F_GRAD 4u
#define OSS_F_ALL 7u
/* first moments sum (i - x) I and sum (j - y) I of the star (the extended
 * Prewitt ramps of Sec. "Patch Features"); table quantities i I and j I.
 * A reference holds both or neither, and with them OSS_F_SUM: the feature
 * sets with moments are SUM|XMOM|YMOM and SUM|SQ|XMOM|YMOM.  Only
 * oss_screen_moments uses them. */
#define OSS_F_XMOM 8u
#define OSS_F_YMOM 16u
#define OSS_F_MOMENTS 24u
#define OSS_MAX_QUANTITIES 5

#define OSS_MAX_SCALES 32 /* scale ids 0..31 per template (bits of a uint32) */

typedef struct oss_ctx oss_ctx;
typedef struct oss_ref oss_ref;

/* An image in memory: H rows of W pixels, rows pitch_bytes apart.
 * dtype OSS_U8 (bit_depth 1..8) or OSS_U16 (bit_depth 1..16); pixel values
 * must not exceed 2^bit_depth - 1 (the bound is used to prove the integer
 * tables cannot overflow). */
typedef struct oss_image_desc {
    int32_t H, W;
    int64_t pitch_bytes;
    int32_t dtype;
    int32_t bit_depth;
} oss_image_desc;

/* Template features: F[0] sum, F[1] sum of squares, F[2] gradient sum of
 * the radius-rho star at the template centre ((w-1)/2, (h-1)/2) (floors);
 * entries for features not in feat_mask are 0. */
typedef struct oss_template_feat {
    int64_t F[3];
    int32_t rho;
    uint32_t feat_mask;
} oss_template_feat;

/* One probe: template index, scale id (0..31), reference radius r >= 0. */
typedef struct oss_probe {
    int32_t template_id, scale_id, r;
} oss_probe;

/* Relative tolerance P[f]/Q per feature f (0 sum, 1 squares, 2 gradient);
 * Q > 0, P[f] >= 0. */
typedef struct oss_tolerance {
    int32_t P[3];
    int32_t Q;
} oss_tolerance;

/* One candidate: template, row, column and the bits of the scales whose
 * probes pass there.  Lists are in (t, y, x) order. */
typedef struct oss_candidate {
    int32_t t, y, x;
    uint32_t scale_bits;
} oss_candidate;

/* Create a context on HIP device `device` (makes it current on the calling
 * thread).  *out receives the handle; destroy it with oss_ctx_destroy after
 * releasing its references and synchronising the streams it used. */
int oss_ctx_create(int device, oss_ctx **out);
int oss_ctx_destroy(oss_ctx *ctx);

/* Launch-shape options of a context (values are validated):
 *   OSS_OPT_STAR_STRIP           column-strip width of the star kernel's
 *                                sweep = threads per block (64..512, a
 *                                multiple of 64; default 512)
 *   OSS_OPT_STAR_BLOCKS_PER_XCD  persistent star blocks per XCD, about the
 *                                rows of one strip an XCD has in flight
 *                                (default 96); a launch uses at most as
 *                                many as the GPU holds at once for its
 *                                kernel
 *   OSS_OPT_STAR_LDS             1: oss_screen stages the table rows that
 *                                several lookups share in LDS (interleaved
 *                                tables with one value width only); 0: load
 *                                every lookup directly (default)
 *   OSS_OPT_BATCH_BUCKET         oss_screen_batched: at most this many distinct
 *                                radii per pass (0: all radii of a template
 *                                group in one pass; default 0)
 *   OSS_OPT_TABLE_PLANAR         1: references created afterwards store each
 *                                quantity in a table plane of its own
 *                                (default); 0: side by side in one entry
 *   OSS_OPT_STAR_PIPE            1: oss_screen's star pass issues the next
 *                                radius' lookups before comparing the
 *                                current one (software pipelining); the LDS
 *                                option takes precedence; default 0
 *   OSS_OPT_STAR_STAGED          1: on planar tables the star passes of
 *                                oss_screen, oss_screen_batched and the
 *                                server look up the first feature quantity
 *                                alone and the others only where some probe
 *                                (batched: the radius' interval hull) admits
 *                                it (default); 0: every quantity at every
 *                                lookup.  The pipelining option takes
 *                                precedence
 *   OSS_OPT_BUILD_STREAM         1: oss_ref_build stores the table entries
 *                                with non-temporal (streaming) stores, so
 *                                that a star pass running beside the build
 *                                on another stream keeps more of its lines
 *                                in L2 (default); 0: ordinary stores, faster
 *                                for a build that runs alone
 *   OSS_OPT_TABLE_REC            1: planar references of the sum, the squares
 *                                and the gradient whose squares' square and
 *                                diamond sums stay below 2^40 (12-bit pixels
 *                                up to radius ~180, 8-bit beyond the 32-bit
 *                                limit) store the sum plane, one 8-byte
 *                                record {squares low word, gradient} per
 *                                entry and a byte plane of the squares' bits
 *                                32..39: 13 bytes per entry instead of 16,
 *                                and a staged star pass's second lookups
 *                                read one record line and one byte line per
 *                                lane instead of three plane lines
 *                                (default); 0: four 32-bit planes
 * They change speed only, never results. */
#define OSS_OPT_STAR_STRIP 1
#define OSS_OPT_STAR_BLOCKS_PER_XCD 2
#define OSS_OPT_STAR_LDS 3
#define OSS_OPT_BATCH_BUCKET 4
#define OSS_OPT_TABLE_PLANAR 5
#define OSS_OPT_STAR_PIPE 6
#define OSS_OPT_STAR_STAGED 7
#define OSS_OPT_BUILD_STREAM 8
#define OSS_OPT_TABLE_REC 9
int oss_ctx_set_option(oss_ctx *ctx, int32_t option, int32_t value);
int oss_ctx_get_option(oss_ctx *ctx, int32_t option, int32_t *value);

/* Timing of one kernel over the launches recorded since profiling was
 * (re)enabled. */
typedef struct oss_kernel_stat {
    char name[32];
    int64_t launches;
    double total_ms;
    double max_ms;
} oss_kernel_stat;

/* enable != 0: clear the statistics and record a HIP event pair around every
 * kernel this context (or a reference created on it) launches, on the
 * launch stream.  enable == 0: stop recording (statistics are kept). */
int oss_ctx_profile(oss_ctx *ctx, int enable);

/* Wait for the recorded events and return one entry per kernel that ran:
 * up to `cap` entries in out, the number written in *n. */
int oss_ctx_profile_read(oss_ctx *ctx, oss_kernel_stat *out, int32_t cap, int32_t *n);

/* Static name of a status code ("OSS_OK", "OSS_E_ARG", ...). */
const char *oss_status_string(int status);

/* Device bytes oss_ref_create would allocate for an image of this shape,
 * feature set and maximum radius: the three integral tables per feature
 * (below) plus the builder's carry workspace.  Used for admission by
 * footprint. */
int oss_ref_bytes(const oss_image_desc *desc, uint32_t feat_mask, int32_t max_radius,
                  size_t *out);

/*
 * Allocate the integral tables of one reference image (Sec. "Patch
 * Features", Eq. T_1 and the summed triangular table of Sec. "Rotation
 * Invariance").  For each feature quantity q in feat_mask the library keeps,
 * for x in [-1, W-1] and y in [-1, H-1]:
 *   L(x,y)  = sum of q(i,j) over i <= x, j <= y               (Eq. T_1)
 *   R(x,y)  = sum over j <= y, |i-x| <= y-j     (45-degree table, apex at
 *             the pixel centre; the paper's triangular sum table)
 *   R'(x,y) = R with the apex moved to the pixel corner (x+1/2, y+1/2):
 *             sum over j <= y, x-(y-j) <= i <= x+1+(y-j)
 * so that square sums take 4 lookups into L (Eq. S_1) and diamond sums 4
 * lookups into R and R'.  One table entry holds the quantities of (x, y) in
 * feature-bit order.
 *
 * max_radius is the largest probe radius this reference will be screened
 * with (< 0: the largest star that fits the image); screens with a larger
 * radius are rejected.  It fixes the value width: when every square and
 * every diamond sum of every quantity up to max_radius is provably below
 * 2^32 (from bit_depth), the tables are stored modulo 2^32 in 32-bit
 * words and each region sum is still exact; otherwise they are int64.
 * Feature sums and comparisons are int64 either way.  Returns
 * OSS_E_OVERFLOW if H * W * max(q) could exceed 2^62.
 */
int oss_ref_create(oss_ctx *ctx, const oss_image_desc *desc, uint32_t feat_mask,
                   int32_t max_radius, oss_ref **out);

/* Build (or rebuild) the tables of `ref` from device pixels laid out as the
 * descriptor says.  Asynchronous on `stream`; the pixels must stay valid
 * until the stream reaches this point. */
int oss_ref_build(oss_ref *ref, const void *dev_pixels, void *stream);

/* Release the tables (the caller synchronises the streams using them). */
int oss_ref_release(oss_ref *ref);

/*
 * Read-only device view of the tables: entry (x, y) of table T starts at
 * byte ((y+1) * pitch_entries + (x+1)) * entry_bytes of T, with x in
 * [-1, W-1], y in [-1, H-1] (oss_ref_layout gives entry_bytes and where each
 * quantity sits in an entry); nq = number of bits in the feature mask;
 * value_bits = the accumulation width (32: every sum modulo 2^32, or 64).
 * Rows span a whole number of 128-byte lines, and entry (0, y) of every row
 * (of every plane) starts a line.  Any output pointer may be NULL.
 */
int oss_ref_tables(const oss_ref *ref, const void **L, const void **R, const void **Rp,
                   int64_t *pitch_entries, int32_t *nq, int32_t *value_bits,
                   int32_t *max_radius);

/*
 * Layout of the tables of `ref` (L, R and R' share it): quantity slot q
 * (feature order: sum, squares, gradient, x and y moments, enabled ones
 * only) of entry
 * (x, y) is the bits[q]-wide value (32: stored modulo 2^32, 64: two's
 * complement) at byte ((y+1) * pitch_entries + (x+1)) * entry_stride +
 * offset[q] of the table; slots q >= nq get offset -1, width 0.  Interleaved
 * entries are 4 * nq bytes (all 32-bit), 8 * nq bytes (all 64-bit) or 16
 * bytes when only the squares need 64 bits (squares at offset 0, the other
 * quantities at 8 and 12).  Planar tables (OSS_OPT_TABLE_PLANAR) hold one
 * quantity per plane, *plane_bytes apart (0 for interleaved tables), with
 * entry_stride = the value width; when only the squares need 64 bits every
 * plane holds 32-bit values (entry_stride 4) and the squares take two: the
 * low words at offset[q], the high words at offset[q] + *plane_bytes.
 */
int oss_ref_layout(const oss_ref *ref, int32_t *entry_stride, int64_t offset[OSS_MAX_QUANTITIES],
                   int32_t bits[OSS_MAX_QUANTITIES], int64_t *plane_bytes);
/* (oss_ref_layout returns OSS_E_STATE for record tables, OSS_OPT_TABLE_REC:
 * their quantities have different strides; oss_ref_layout_q describes every
 * layout.) */

/* Where one quantity of table entry e = (y+1) * pitch_entries + (x+1) sits,
 * relative to the table pointer of oss_ref_tables: its low `bits` bits at
 * byte offset + e * stride, and, when hi_bits > 0, its next hi_bits bits at
 * byte hi_offset + e * hi_stride.  The value is stored modulo
 * 2^(bits + hi_bits), which keeps every square and diamond sum of it exact
 * (it is below that bound). */
typedef struct oss_quantity_layout {
    int64_t offset;
    int32_t stride, bits;
    int64_t hi_offset;  /* -1: no high part */
    int32_t hi_stride, hi_bits;
} oss_quantity_layout;

/* The layout of each quantity slot q < *nq (feature order, enabled ones
 * only) of the tables of `ref` (L, R and R' share it); slots q >= *nq get
 * offset -1.  *plane_bytes: the first plane's size for planar tables (the
 * distance between planes of equal width), 0 for interleaved entries.
 * Host, synchronous. */
int oss_ref_layout_q(const oss_ref *ref, oss_quantity_layout out[OSS_MAX_QUANTITIES],
                     int32_t *nq, int64_t *plane_bytes);

/* Template features (host, synchronous): the radius-rho star at the centre
 * of a host image, G taken on the template itself.  rho < 0 picks the
 * largest radius whose star fits, less one when OSS_F_GRAD is requested (the
 * template's border pixels have a clamped gradient); with OSS_F_GRAD a star
 * touching the border is refused (OSS_E_ARG).  Algorithm 1, "features(Z)"
 * of the template loop. */
int oss_template_features(const void *host_pixels, const oss_image_desc *desc, int32_t rho,
                          uint32_t feat_mask, oss_template_feat *out);

/* The exact set of feature sums that pass one feature test: F passes iff
 * *lo <= F <= *hi (host, synchronous).  feature 0 sum, 1 squares,
 * 2 gradient; FT the template's feature sum, r the reference radius, rho the
 * template radius.  The screen uses the same interval (Algorithm 1, patch
 * loop: the cross-multiplied relative test solved once per probe). */
int oss_feature_bounds(int32_t feature, int64_t FT, int32_t r, int32_t rho,
                       const oss_tolerance *tol, int64_t *lo, int64_t *hi);

/*
 * Screen one reference against n_tmpl templates and n_probes probes
 * (Algorithm 1, patch loop, for every probed scale).  feat_mask selects the
 * compared features (a subset of the reference's).  Outputs, all caller
 * owned device memory written on `stream`:
 *   dev_mask  [n_tmpl][H][W] uint8, 1 where some probe of template t passes
 *             (may be NULL)
 *   dev_list  up to list_cap candidates in (t, y, x) order (may be NULL
 *             with list_cap 0)
 *   dev_count int64, the total number of candidates (may exceed list_cap;
 *             the list then holds the first list_cap)
 * Each template's probes are screened by one launch of the star kernel.
 */
int oss_screen(oss_ctx *ctx, const oss_ref *ref, const oss_template_feat *tmpl, int32_t n_tmpl,
               const oss_probe *probes, int32_t n_probes, const oss_tolerance *tol,
               uint32_t feat_mask, uint8_t *dev_mask, oss_candidate *dev_list, int64_t list_cap,
               int64_t *dev_count, void *stream);

/*
 * oss_screen without allocation, for callers that cannot allocate device
 * memory during a screen: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, outputs, kernels and
 * results as oss_screen (the same options apply); the context and the
 * reference are made beforehand.  Its scratch (the launch plans, the
 * per-segment candidate counts, the staged candidates and the scan) lives in
 * one fixed device array of OSS_NOALLOC_SCRATCH_BYTES per GPU, held by the
 * library until the process ends; the call makes no hipMalloc, hipFree or
 * other allocation, host or device, and is not profiled (oss_ctx_profile
 * does not see its kernels).  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (several streams, threads or contexts) race
 * and must be serialised by the caller.  Nothing in the array needs clearing
 * between calls (each call writes every count it reads).  OSS_E_LIMIT when
 * the screen needs more scratch than the array holds: about
 * n_tmpl * H * ceil(W / 64) * 513 bytes of counts and staging plus 2.5 KB
 * per template; a 4096 x 4096 screen of one template fits.
 */
#define OSS_NOALLOC_SCRATCH_BYTES ((size_t)160 << 20)
int oss_screen_noalloc(oss_ctx *ctx, const oss_ref *ref, const oss_template_feat *tmpl,
                       int32_t n_tmpl, const oss_probe *probes, int32_t n_probes,
                       const oss_tolerance *tol, uint32_t feat_mask, uint8_t *dev_mask,
                       oss_candidate *dev_list, int64_t list_cap, int64_t *dev_count,
                       void *stream);

/*
 * Same contract and outputs as oss_screen, with all templates and probes in
 * one persistent launch over the reference's tables (Algorithm 1's patch
 * loop for every template and scale together).  Templates are sorted by
 * radius and taken in groups of 64 (32 by oss_screen_rings); within a
 * group the star features of
 * each distinct radius are computed once per position and compared with
 * every probe of the group at that radius.  A group's radii are walked in
 * passes of at most OSS_OPT_BATCH_BUCKET distinct radii.  Results are
 * identical to oss_screen's.
 */
int oss_screen_batched(oss_ctx *ctx, const oss_ref *ref, const oss_template_feat *tmpl,
                       int32_t n_tmpl, const oss_probe *probes, int32_t n_probes,
                       const oss_tolerance *tol, uint32_t feat_mask, uint8_t *dev_mask,
                       oss_candidate *dev_list, int64_t list_cap, int64_t *dev_count,
                       void *stream);

/* ------------------------------------------------------------------------
 * Multi-central-area screen (Sec. "Scale Invariance", central areas of
 * sizes n, n/lambda, n/lambda^2 with lambda = sqrt 2, Fig. ring): a probe
 * (t, k, r) passes where its star of radius r passes and so do the
 * concentric central stars of radii r_1 = s(r), r_2 = s(r_1), ... (s(r) =
 * round(r / sqrt 2), the square half-width above), each compared with the
 * template's central star of the matching ring by the same feature test.
 * ------------------------------------------------------------------------ */
#define OSS_MAX_RINGS 4

/* Features of the template's central stars of radii rho, s(rho), ...
 * (n_rings of them, 1..OSS_MAX_RINGS) into out[0..n_rings-1]; rho < 0
 * picks the default radius as oss_template_features does.  Host-side,
 * synchronous. */
int oss_template_features_rings(const void *host_pixels, const oss_image_desc *desc,
                                int32_t rho, uint32_t feat_mask, int32_t n_rings,
                                oss_template_feat *out);

/* Screen with n_rings central stars per probe.  tmpl is [n_tmpl][n_rings]:
 * tmpl[t * n_rings + j] holds template t's ring-j features and radius (as
 * from oss_template_features_rings).  Ring j of probe (t, k, r) compares the
 * reference star of radius r_j with tmpl[t * n_rings + j].  Other arguments,
 * outputs and errors as oss_screen_batched (one pass per template group:
 * OSS_OPT_BATCH_BUCKET does not apply).  n_rings = 1 gives oss_screen's
 * results. */
int oss_screen_rings(oss_ctx *ctx, const oss_ref *ref, const oss_template_feat *tmpl,
                     int32_t n_tmpl, int32_t n_rings, const oss_probe *probes, int32_t n_probes,
                     const oss_tolerance *tol, uint32_t feat_mask, uint8_t *dev_mask,
                     oss_candidate *dev_list, int64_t list_cap, int64_t *dev_count,
                     void *stream);

/*
 * Preserved region of a screen (Sec. "Experimental Results", Exp. I: the
 * regions the pre-processor keeps; one minus their share of the image is
 * the pruned region).  dev_region [n_tmpl][H][W] (uint8, caller-owned) gets
 * 1 where the pixel lies inside the star of radius r of a candidate of
 * template t in dev_list whose scale bits include k, for some probe
 * (t, k, r) in `probes` (the probe set of the screen that produced the
 * list), and 0 elsewhere.  The list and its count are read on the device
 * (entries past min(*dev_count, list_cap) are ignored), so the call needs no
 * synchronisation after the screen on the same stream.  Works in a context
 * workspace of about 50 bytes per pixel of the image padded by the largest
 * radius; one table build and one single-radius star pass per distinct
 * (template, radius).  Asynchronous on `stream`.
 */
int oss_region(oss_ctx *ctx, int32_t H, int32_t W, int32_t n_tmpl, const oss_probe *probes,
               int32_t n_probes, const oss_candidate *dev_list, int64_t list_cap,
               const int64_t *dev_count, uint8_t *dev_region, void *stream);

/* ------------------------------------------------------------------------
 * Interval probes and Algorithm 1 taken literally.
 * ------------------------------------------------------------------------ */

/* A probe given by explicit inclusive bounds on the star's feature sums
 * (feature order: sum, squares, gradient; bounds of features outside the
 * screen's feature mask are ignored). */
typedef struct oss_interval_probe {
    int32_t template_id;  /* result row t */
    int32_t scale_id;     /* result bit k (0..31) */
    int32_t r;            /* star radius, 0..the reference's max radius */
    int32_t pad;
    int64_t lo[3], hi[3];
} oss_interval_probe;

/*
 * Screen with interval probes: bit k of template t is set where, for some
 * probe (t, k, r), the radius-r star fits and every enabled feature sum lies
 * in [lo, hi] (several probes sharing (t, k) give the union of their boxes).
 * One batched launch (OSS_OPT_STAR_* and OSS_OPT_BATCH_BUCKET apply);
 * outputs, ownership and errors as oss_screen.
 */
int oss_screen_intervals(oss_ctx *ctx, const oss_ref *ref, int32_t n_tmpl,
                         const oss_interval_probe *probes, int32_t n_probes, uint32_t feat_mask,
                         uint8_t *dev_mask, oss_candidate *dev_list, int64_t list_cap,
                         int64_t *dev_count, void *stream);

/* Parameters of Algorithm 1: the scale range [alpha, beta] as fractions and
 * the quantisation step of each feature in units of its per-pixel mean
 * (grey levels, squared grey levels, gradient units). */
typedef struct oss_alg1_params {
    int32_t alpha_num, alpha_den, beta_num, beta_den;
    int32_t q[3];
    uint32_t feat_mask;
} oss_alg1_params;

/*
 * The template side of Algorithm 1 (Sec. "Scale Invariance", Algorithm 1,
 * Eq. F_n) for one square template of width n, as interval probes of
 * template t: lambda = sqrt 2; band b = 0 .. B-1, B = the smallest integer
 * with lambda^B >= beta/alpha, covers the template sizes k = ceil(m_b) ..
 * floor(lambda m_b), m_b = beta n / lambda^(b+1), and screens patches of
 * size m = ceil(m_b) with the star of radius (m-1)/2.  For each k the
 * template is resized to k x k (bilinear, pixel centres aligned, edges
 * replicated, rounded half up, exact integers), its central m x m crop's
 * star features F are quantised with Q(f) = floor(f/q + 1/2), q = q_f A(r),
 * and the cells Q(F - q/2), Q(F), Q(F + q/2) of every feature are marked;
 * the marked box of k becomes one probe (scale_id = b) bounding the sums to
 * the cells floor(F/q) .. floor(F/q) + 1.  Identical boxes are emitted
 * once.  Writes up to `cap` probes to out and the number needed to *n_out;
 * OSS_E_NOMEM if cap is smaller.  Host-side, synchronous.  Errors: a
 * non-square template, alpha > beta, non-positive fractions or steps, more
 * than 32 bands.
 */
int oss_alg1_probes(const void *host_pixels, const oss_image_desc *desc, int32_t t,
                    const oss_alg1_params *params, oss_interval_probe *out, int32_t cap,
                    int32_t *n_out);

/* ------------------------------------------------------------------------
 * The paper's own features (Sec. "Patch Features": mean, Eq. S_sigma
 * variance, gradients as inner products with the extended Prewitt ramps;
 * Sec. "Rotation Invariance": the gradient magnitude), over the star.
 * ------------------------------------------------------------------------ */
#define OSS_T_MEAN 1u
#define OSS_T_VAR 2u
#define OSS_T_MAG 4u

/* Star sums at the template centre (as oss_template_features): F1 = sum w I,
 * F2 = sum w I^2, Sx = sum w (i - x) I, Sy = sum w (j - y) I, radius rho. */
typedef struct oss_template_mom {
    int64_t F1, F2, Sx, Sy;
    int32_t rho, pad;
} oss_template_mom;

/* Template moments at radius rho (rho < 0: the largest that fits).  Host,
 * synchronous. */
int oss_template_moments(const void *host_pixels, const oss_image_desc *desc, int32_t rho,
                         oss_template_mom *out);

/*
 * Screen with the paper's features: a position passes probe (t, k, r) where
 * the radius-r star fits and each test in `tests` passes, with A = the
 * star's weighted area, N(r) = r A(r), V = A F2 - F1^2 (A^2 times the
 * variance) and M = Sx^2 + Sy^2 (the squared gradient magnitude), rho the
 * template's radius and P = tol->P[0..2] for mean, variance, magnitude:
 *   OSS_T_MEAN  (Q-P) FT1 A(r)     <= Q F1 A(rho)     <= (Q+P) FT1 A(r)
 *   OSS_T_VAR   (Q-P) VT A(r)^2    <= Q V A(rho)^2    <= (Q+P) VT A(r)^2
 *   OSS_T_MAG   (Q-P)^2 MT N(r)^2  <= Q^2 M N(rho)^2  <= (Q+P)^2 MT N(r)^2
 * (the magnitude's lower bound is void when P > Q), all exact.  The
 * reference must hold OSS_F_SUM and the moments, and OSS_F_SQ for the
 * variance.  OSS_E_OVERFLOW when a magnitude bound exceeds 128 bits.
 * Outputs, ownership and errors otherwise as oss_screen (one launch per
 * template).
 */
int oss_screen_moments(oss_ctx *ctx, const oss_ref *ref, const oss_template_mom *tmpl,
                       int32_t n_tmpl, const oss_probe *probes, int32_t n_probes,
                       const oss_tolerance *tol, uint32_t tests, uint8_t *dev_mask,
                       oss_candidate *dev_list, int64_t list_cap, int64_t *dev_count,
                       void *stream);

#define OSS_TUNE_MAX 64
/* Autotuner result: the chosen shape, its time, and every candidate tried
 * (strip, blocks per XCD, bucket) with its time in ms. */
typedef struct oss_tune_result {
    int32_t strip, blocks_per_xcd, bucket_radii;
    float ms;
    int32_t n_tried;
    int32_t tried[OSS_TUNE_MAX][3];
    float tried_ms[OSS_TUNE_MAX];
} oss_tune_result;

/*
 * Autotune oss_screen_batched for this reference and probe set: time the
 * batched star pass (HIP events on `stream`, one warm-up and one timed run
 * per candidate) over strip widths {256, 512}, blocks per XCD {32, 64, 128}
 * and radius buckets {all, 16, 8, 4}, keep the fastest in the context's
 * options (OSS_OPT_STAR_STRIP, OSS_OPT_STAR_BLOCKS_PER_XCD,
 * OSS_OPT_BATCH_BUCKET) and report every candidate in *out.  Synchronises
 * `stream`; overwrites the context's screen workspace.
 */
int oss_autotune_batched(oss_ctx *ctx, const oss_ref *ref, const oss_template_feat *tmpl,
                         int32_t n_tmpl, const oss_probe *probes, int32_t n_probes,
                         const oss_tolerance *tol, uint32_t feat_mask, void *stream,
                         oss_tune_result *out);


/* ------------------------------------------------------------------------
 * Serving loop.  A server owns one device, a device-memory budget, a set of
 * lanes (one context + one stream each) and a cache of resident reference
 * tables keyed by the caller's reference id.  Requests are queued by
 * oss_server_submit and run by oss_server_pump: the oldest queued request is
 * admitted when its footprint fits the budget (its reference tables unless
 * resident, its mask of n_tmpl*H*W bytes, 16 bytes per list entry of
 * capacity, and the lane's emission workspace of about 8*n_tmpl*H*W bytes),
 * evicting least recently used resident references that no queued or
 * running request needs (a request that does not fit waits for running
 * work to finish or for results to be released).  Every queued request on the same reference that
 * fits joins the admitted one in a single batched launch (oss_screen_batched
 * over the union of their templates, each template keeping its request's
 * tolerance and feature set); each request then gets its own compaction into
 * its own mask and list, so its result is identical to a screen of that
 * request alone.  Work of different references runs concurrently on the
 * lanes: requests submitted while launches run are admitted as lanes and
 * memory free up, and the server's own device memory (lane workspaces,
 * output blocks, reference tables) is allocated and freed in stream order on
 * the lanes' streams, so scheduling never waits for the whole device.  A
 * queued request can be cancelled, and one that waits longer than the
 * configured queue timeout fails with OSS_E_TIMEOUT instead of running.
 * This is an addition to the paper's method (its Algorithm 1 screens one
 * reference against one template).
 * ------------------------------------------------------------------------ */
typedef struct oss_server oss_server;

typedef struct oss_server_config {
    int64_t memory_budget;        /* device bytes the server may hold (> 0) */
    int32_t lanes;                /* concurrent lanes, 1..8 */
    int32_t max_batch_templates;  /* templates per merged launch (>= 1); a
                                     request with more still runs alone */
    int64_t queue_timeout_ns;     /* a request still queued this long after its
                                     arrival fails with OSS_E_TIMEOUT (0: none) */
} oss_server_config;

typedef struct oss_request {
    uint64_t ref_key;        /* equal keys promise equal pixels and desc */
    const void *dev_pixels;  /* device pixels, read only when the reference
                                is not resident; caller-owned, valid until
                                the request completes */
    oss_image_desc desc;
    const oss_template_feat *tmpl;  /* copied by oss_server_submit */
    int32_t n_tmpl;
    const oss_probe *probes;        /* copied by oss_server_submit */
    int32_t n_probes;
    oss_tolerance tol;
    uint32_t feat_mask;
    int64_t list_cap;        /* candidate list capacity */
    int64_t arrival_ns;      /* CLOCK_MONOTONIC arrival time; 0 = at submit */
} oss_request;

typedef struct oss_result {
    int32_t status;          /* OSS_OK done, OSS_E_STATE pending, else the
                                error the request failed with */
    int32_t n_tmpl, H, W;
    const uint8_t *dev_mask;       /* [n_tmpl][H][W], server-owned */
    const oss_candidate *dev_list; /* list_cap entries, server-owned */
    int64_t list_cap;
    int64_t count;           /* candidates found (may exceed list_cap) */
    double latency_ms;       /* arrival -> completion seen by the server */
    double queue_ms;         /* arrival -> launch */
    int32_t batch_requests;  /* requests merged into its launch */
    int32_t resident_hit;    /* 1 if its reference tables were resident */
    int32_t lane;
    int32_t pad;
} oss_result;

typedef struct oss_server_stats {
    int64_t submitted, completed, failed, launches;
    int64_t resident_hits, builds, evictions;
    int64_t bytes_in_use, bytes_peak, memory_budget;
    int32_t queued, running;
} oss_server_stats;

/* Create / destroy a server on `device`.  Destroy waits for running work
 * and frees everything the server holds, including unreleased results. */
int oss_server_create(int device, const oss_server_config *cfg, oss_server **out);
int oss_server_destroy(oss_server *srv);

/* Validate and queue a request (nothing is launched).  *id identifies it.
 * OSS_E_NOMEM if its footprint (with its reference not resident) exceeds
 * the whole budget; OSS_E_ARG for invalid arguments, with the same rules as
 * oss_screen. */
int oss_server_submit(oss_server *srv, const oss_request *req, int64_t *id);

/* Retire finished launches and admit / launch queued requests on free
 * lanes.  If `wait_us` > 0 and nothing completed yet, polls for up to that
 * long for a completion.  *n_completed (optional) = requests completed by
 * this call. */
int oss_server_pump(oss_server *srv, int64_t wait_us, int32_t *n_completed);

/* Pump until no request is queued or running.  OSS_E_NOMEM if queued
 * requests cannot be admitted until completed results are released. */
int oss_server_drain(oss_server *srv);

/* Cancel a queued request: it leaves the queue and completes with status
 * OSS_E_CANCELLED (release it as any other).  OSS_E_STATE if it has been
 * launched or has finished (a running launch is not interrupted; its result
 * arrives as usual), OSS_E_ARG for an unknown id or a null server. */
int oss_server_cancel(oss_server *srv, int64_t id);

/* Status and output of a request (status OSS_E_STATE while pending). */
int oss_server_result(oss_server *srv, int64_t id, oss_result *out);

/* Free a completed (or failed) request's outputs; its id becomes invalid. */
int oss_server_release(oss_server *srv, int64_t id);

int oss_server_stats_read(oss_server *srv, oss_server_stats *out);

#ifdef __cplusplus
}
#endif

#endif /* OSS_H */
