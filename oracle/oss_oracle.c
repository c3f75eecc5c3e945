/*
 * Octagonal-star screening oracle: plain, slow CPU reference.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  It shares no
 * code, header or constant with the GPU library and must never be called
 * from the product path.
 *
 * What it computes (Liu, Shu & Wu, "Fast Screening Algorithm for Rotation
 * and Scale Invariant Template Matching"):
 *
 *  - Star region (Sec. "Rotation Invariance", Eq. S_os and Fig. os): the
 *    superposition of a square and a 45-degree diamond of the same size.
 *    Discretised pixel-centred: the diamond is |dx|+|dy| <= r, the square
 *    max(|dx|,|dy|) <= s(r), with s(r) the half-width of the square that is
 *    congruent to the diamond, s(r) = max{ s : (2s-1)^2 < 2 r^2 }.  Pixels in
 *    both count twice (superposition); the sum of the two region sums is
 *    twice the paper's averaged form up to the area normalisation.
 *  - Features (Sec. "Patch Features"): sum of intensities, sum of squared
 *    intensities (the second moment of Eq. S_sigma) and the sum of a
 *    rotation-robust gradient magnitude |Gx|+|Gy| (Sec. "Rotation
 *    Invariance", the magnitude replacing the directional gradients), with
 *    Gx, Gy undivided central differences and clamp-to-edge indexing.
 *  - Screen (Algorithm 1, patch loop; Sec. "Scale Invariance", feature set
 *    membership): a position survives a probe when every enabled feature,
 *    normalised by the star's weighted area (and, for the gradient, by the
 *    radius, since gradients shrink as 1/scale), lies within a relative
 *    tolerance P/Q of the template's.  The comparison is done literally,
 *    cross-multiplied in 128-bit integers.
 *
 * Everything is summed pixel by pixel; there are no tables, no tiling and
 * no reuse beyond computing one radius' features once per position.
 */
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __int128 i128;

/* Number of threads the parallel loops below use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Square half-width congruent with the radius-r diamond. */
int oracle_square_half(int r)
{
    int s = 0;
    while ((int64_t)(2 * s + 1) * (2 * s + 1) < 2LL * r * r)
        s++;
    return s;
}

static int iabs(int v) { return v < 0 ? -v : v; }

/* Star weight at offset (dx, dy) for radius r and square half-width s:
 * 0, 1 or 2. */
static int weight_rs(int dx, int dy, int r, int s)
{
    int adx = iabs(dx), ady = iabs(dy);
    int in_square = (adx <= s && ady <= s);
    int in_diamond = (adx + ady <= r);
    return in_square + in_diamond;
}

int oracle_star_weight(int dx, int dy, int r)
{
    return weight_rs(dx, dy, r, oracle_square_half(r));
}

/* Weighted star area A(r): the weights summed over the bounding box. */
int64_t oracle_star_area(int r)
{
    int64_t a = 0;
    for (int dy = -r; dy <= r; dy++)
        for (int dx = -r; dx <= r; dx++)
            a += oracle_star_weight(dx, dy, r);
    return a;
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* |I(x+1,y) - I(x-1,y)| + |I(x,y+1) - I(x,y-1)| with indices clamped to the image. */
void oracle_gradient(const uint16_t *img, int H, int W, int64_t stride, int32_t *G)
{
    for (int y = 0; y < H; y++) {
        for (int x = 0; x < W; x++) {
            int xr = clampi(x + 1, 0, W - 1), xl = clampi(x - 1, 0, W - 1);
            int yd = clampi(y + 1, 0, H - 1), yu = clampi(y - 1, 0, H - 1);
            int gx = (int)img[(int64_t)y * stride + xr] - (int)img[(int64_t)y * stride + xl];
            int gy = (int)img[(int64_t)yd * stride + x] - (int)img[(int64_t)yu * stride + x];
            G[(int64_t)y * W + x] = iabs(gx) + iabs(gy);
        }
    }
}

/* Star sums of I, I^2 and G at (x, y) with radius r.  Returns 0, or -1 when
 * the star does not fit inside the image. */
static int star_at(const uint16_t *img, const int32_t *G, int H, int W, int64_t stride,
                   int x, int y, int r, int64_t F[3])
{
    if (x < r || x > W - 1 - r || y < r || y > H - 1 - r)
        return -1;
    int s = oracle_square_half(r);
    int64_t f1 = 0, f2 = 0, fg = 0;
    for (int dy = -r; dy <= r; dy++) {
        for (int dx = -r; dx <= r; dx++) {
            int w = weight_rs(dx, dy, r, s);
            if (!w)
                continue;
            int64_t v = img[(int64_t)(y + dy) * stride + (x + dx)];
            f1 += w * v;
            f2 += w * v * v;
            fg += (int64_t)w * G[(int64_t)(y + dy) * W + (x + dx)];
        }
    }
    F[0] = f1;
    F[1] = f2;
    F[2] = fg;
    return 0;
}

/* Features at n positions for one radius.  F is [n][3]; positions where the
 * star does not fit get -1 in all three slots.  G must be the gradient image
 * of img (W columns, dense). */
void oracle_features(const uint16_t *img, const int32_t *G, int H, int W, int64_t stride,
                     const int32_t *xs, const int32_t *ys, int64_t n, int r, int64_t *F)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        int64_t f[3];
        if (star_at(img, G, H, W, stride, xs[i], ys[i], r, f) != 0)
            f[0] = f[1] = f[2] = -1;
        F[3 * i + 0] = f[0];
        F[3 * i + 1] = f[1];
        F[3 * i + 2] = f[2];
    }
}

/* One feature test, cross-multiplied (feature index f: 0 sum, 1 squares,
 * 2 gradient).  X_ref = F * A(rho) * c_ref, X_T = FT * A(r) * c_T with
 * (c_ref, c_T) = (r, rho) for the gradient and (1, 1) otherwise; the
 * feature passes iff (Q-P) X_T <= Q X_ref <= (Q+P) X_T. */
static int feature_pass(int f, int64_t F, int64_t FT, int r, int rho, int64_t area_r,
                        int64_t area_rho, int P, int Q)
{
    i128 c_ref = (f == 2) ? r : 1;
    i128 c_t = (f == 2) ? rho : 1;
    i128 x_ref = (i128)F * area_rho * c_ref;
    i128 x_t = (i128)FT * area_r * c_t;
    i128 lhs = (i128)(Q - P) * x_t;
    i128 mid = (i128)Q * x_ref;
    i128 rhs = (i128)(Q + P) * x_t;
    return lhs <= mid && mid <= rhs;
}

int oracle_feature_pass(int f, int64_t F, int64_t FT, int r, int rho, int P, int Q)
{
    return feature_pass(f, F, FT, r, rho, oracle_star_area(r), oracle_star_area(rho), P, Q);
}

/*
 * Screen n positions against a probe list.
 *   probes: [n_probes][3] = (template id, scale id, reference radius r)
 *   FT:     [n_tmpl][3] template features, rho: [n_tmpl] template radii
 *   feat_mask: bit 0 sum, bit 1 squares, bit 2 gradient
 *   bits:   [n_tmpl][n] output; bit k set iff probe (t, k) passes there
 * A probe passes when the star of radius r fits at the position and every
 * enabled feature passes.  Consecutive probes with the same radius share
 * one feature computation (the caller may sort the probes by radius).
 */
int oracle_screen(const uint16_t *img, const int32_t *G, int H, int W, int64_t stride,
                  const int32_t *xs, const int32_t *ys, int64_t n,
                  const int32_t *probes, int n_probes, const int64_t *FT, const int32_t *rho,
                  int n_tmpl, int feat_mask, const int32_t *P, int Q, uint32_t *bits)
{
    for (int p = 0; p < n_probes; p++) {
        int t = probes[3 * p], k = probes[3 * p + 1], r = probes[3 * p + 2];
        if (t < 0 || t >= n_tmpl || k < 0 || k > 31 || r < 0)
            return -1;
    }
    if (Q <= 0)
        return -1;
    int64_t *area_r = malloc(sizeof(int64_t) * (n_probes > 0 ? n_probes : 1));
    int64_t *area_rho = malloc(sizeof(int64_t) * (n_tmpl > 0 ? n_tmpl : 1));
    if (!area_r || !area_rho) {
        free(area_r);
        free(area_rho);
        return -1;
    }
    for (int p = 0; p < n_probes; p++)
        area_r[p] = oracle_star_area(probes[3 * p + 2]);
    for (int t = 0; t < n_tmpl; t++)
        area_rho[t] = oracle_star_area(rho[t]);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        for (int t = 0; t < n_tmpl; t++)
            bits[(int64_t)t * n + i] = 0;
        int last_r = -1, last_ok = 0;
        int64_t F[3] = {0, 0, 0};
        for (int p = 0; p < n_probes; p++) {
            int t = probes[3 * p], k = probes[3 * p + 1], r = probes[3 * p + 2];
            if (r != last_r) {
                last_ok = star_at(img, G, H, W, stride, xs[i], ys[i], r, F) == 0;
                last_r = r;
            }
            if (!last_ok)
                continue;
            int pass = 1;
            for (int f = 0; f < 3 && pass; f++) {
                if (!(feat_mask & (1 << f)))
                    continue;
                pass = feature_pass(f, F[f], FT[3 * t + f], r, rho[t], area_r[p],
                                    area_rho[t], P[f], Q);
            }
            if (pass)
                bits[(int64_t)t * n + i] |= 1u << k;
        }
    }
    free(area_r);
    free(area_rho);
    return 0;
}

/*
 * Multi-central-area screen (Sec. "Scale Invariance", the paragraph on
 * central areas of different sizes and Fig. ring): besides the star of the
 * probe's radius r, the concentric central stars of radii r_1 = s(r) and
 * r_{j+1} = s(r_j) (s(r) = round(r / sqrt 2): each ring a factor lambda =
 * sqrt 2 smaller) must match the template's central stars of radii
 * rho_j, and the probe passes only if every one of the n_rings areas
 * passes every enabled feature test.
 *   FT:  [n_tmpl][n_rings][3] template features of ring j at radius rho_j
 *   rho: [n_tmpl][n_rings] template ring radii rho_j
 * n_rings = 1 is oracle_screen.  A probe needs the outer star (radius r)
 * to fit; the inner ones then fit too.
 */
int oracle_screen_rings(const uint16_t *img, const int32_t *G, int H, int W, int64_t stride,
                        const int32_t *xs, const int32_t *ys, int64_t n,
                        const int32_t *probes, int n_probes, const int64_t *FT,
                        const int32_t *rho, int n_tmpl, int n_rings, int feat_mask,
                        const int32_t *P, int Q, uint32_t *bits)
{
    if (Q <= 0 || n_rings < 1 || n_rings > 8)
        return -1;
    for (int p = 0; p < n_probes; p++) {
        int t = probes[3 * p], k = probes[3 * p + 1], r = probes[3 * p + 2];
        if (t < 0 || t >= n_tmpl || k < 0 || k > 31 || r < 0)
            return -1;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        for (int t = 0; t < n_tmpl; t++)
            bits[(int64_t)t * n + i] = 0;
        for (int p = 0; p < n_probes; p++) {
            int t = probes[3 * p], k = probes[3 * p + 1], r = probes[3 * p + 2];
            int pass = 1;
            int rj = r;
            for (int j = 0; j < n_rings && pass; j++) {
                int64_t F[3];
                if (star_at(img, G, H, W, stride, xs[i], ys[i], rj, F) != 0) {
                    pass = 0;
                    break;
                }
                int rho_j = rho[t * n_rings + j];
                const int64_t *ft = FT + 3 * ((int64_t)t * n_rings + j);
                for (int f = 0; f < 3 && pass; f++) {
                    if (!(feat_mask & (1 << f)))
                        continue;
                    pass = feature_pass(f, F[f], ft[f], rj, rho_j, oracle_star_area(rj),
                                        oracle_star_area(rho_j), P[f], Q);
                }
                rj = oracle_square_half(rj);
            }
            if (pass)
                bits[(int64_t)t * n + i] |= 1u << k;
        }
    }
    return 0;
}

/*
 * The paper's own patch features over the star (Sec. "Patch Features":
 * mean, Eq. S_sigma variance, and the horizontal / vertical gradients as
 * inner products with the extended Prewitt ramps, Eq. T_x; Sec. "Rotation
 * Invariance": their magnitude).  For n positions and radius r, F is
 * [n][4] = (sum I, sum I^2, sum (i - x) I, sum (j - y) I) over the star with
 * its 0/1/2 weights, summed pixel by pixel; -1 ... when the star does not
 * fit (slot 0 = -1 marks it).
 */
void oracle_moments(const uint16_t *img, int H, int W, int64_t stride, const int32_t *xs,
                    const int32_t *ys, int64_t n, int r, int64_t *F)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        int x = xs[i], y = ys[i];
        int64_t *o = F + 4 * i;
        if (x < r || x > W - 1 - r || y < r || y > H - 1 - r) {
            o[0] = o[1] = o[2] = o[3] = -1;
            continue;
        }
        int s = oracle_square_half(r);
        int64_t f1 = 0, f2 = 0, mx = 0, my = 0;
        for (int dy = -r; dy <= r; dy++) {
            for (int dx = -r; dx <= r; dx++) {
                int w = weight_rs(dx, dy, r, s);
                if (!w)
                    continue;
                int64_t v = img[(int64_t)(y + dy) * stride + x + dx];
                f1 += w * v;
                f2 += (int64_t)w * v * v;
                mx += (int64_t)w * dx * v;
                my += (int64_t)w * dy * v;
            }
        }
        o[0] = f1;
        o[1] = f2;
        o[2] = mx;
        o[3] = my;
    }
}
