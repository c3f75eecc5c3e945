// Host-side calls of the library and of the C oracle, built with
// AddressSanitizer and UndefinedBehaviorSanitizer and run without a GPU.
// Each call's result is also checked: template features against the
// oracle's pixel-by-pixel star sums, feature bounds against the oracle's
// cross-multiplied compare at and around each bound, and argument errors.
// Exits non-zero on the first mismatch (a sanitizer report aborts first).
#include "oss.h"

#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

extern "C" {
void oracle_gradient(const uint16_t *img, int H, int W, int64_t stride, int32_t *G);
void oracle_features(const uint16_t *img, const int32_t *G, int H, int W, int64_t stride,
                     const int32_t *xs, const int32_t *ys, int64_t n, int r, int64_t *F);
int oracle_feature_pass(int f, int64_t F, int64_t FT, int r, int rho, int P, int Q);
int oracle_screen(const uint16_t *img, const int32_t *G, int H, int W, int64_t stride,
                  const int32_t *xs, const int32_t *ys, int64_t n, const int32_t *probes,
                  int n_probes, const int64_t *FT, const int32_t *rho, int n_tmpl, int feat_mask,
                  const int32_t *P, int Q, uint32_t *bits);
void oracle_moments(const uint16_t *img, int H, int W, int64_t stride, const int32_t *xs,
                    const int32_t *ys, int64_t n, int r, int64_t *F);
}

static int g_fail = 0;
#define CHECK(c, ...)                                     \
    do {                                                  \
        if (!(c)) {                                       \
            std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);            \
            std::fprintf(stderr, "\n");                   \
            ++g_fail;                                     \
        }                                                 \
    } while (0)

// A template image of h x w pixels (16-bit storage, values < 2^depth).
struct Img {
    int h, w, depth;
    std::vector<uint16_t> px;
};

static Img make_img(std::mt19937 &rng, int h, int w, int depth)
{
    Img im{h, w, depth, std::vector<uint16_t>((size_t)h * w)};
    std::uniform_int_distribution<int> d(0, (1 << depth) - 1);
    for (auto &v : im.px)
        v = (uint16_t)d(rng);
    return im;
}

static void check_template_features(std::mt19937 &rng)
{
    for (int trial = 0; trial < 40; ++trial) {
        const int depth = trial % 2 ? 12 : 8;
        const int h = 9 + (int)(rng() % 30), w = 9 + (int)(rng() % 30);
        Img im = make_img(rng, h, w, depth);
        // the library takes uint8 or uint16 pixels with a pitch
        std::vector<uint8_t> u8;
        oss_image_desc d{};
        d.H = h;
        d.W = w;
        d.bit_depth = depth;
        const void *pix;
        if (depth <= 8) {
            u8.assign(im.px.begin(), im.px.end());
            d.dtype = OSS_U8;
            d.pitch_bytes = w;
            pix = u8.data();
        } else {
            d.dtype = OSS_U16;
            d.pitch_bytes = 2 * (int64_t)w;
            pix = im.px.data();
        }
        const uint32_t fm = (trial % 3 == 0) ? (OSS_F_SUM | OSS_F_SQ) : OSS_F_ALL;
        oss_template_feat tf{};
        int rc = oss_template_features(pix, &d, -1, fm, &tf);
        CHECK(rc == OSS_OK, "template features rc %d", rc);
        if (rc != OSS_OK)
            continue;
        std::vector<int32_t> G((size_t)h * w);
        oracle_gradient(im.px.data(), h, w, w, G.data());
        const int32_t cx = (w - 1) / 2, cy = (h - 1) / 2;
        int64_t F[3];
        oracle_features(im.px.data(), G.data(), h, w, w, &cx, &cy, 1, tf.rho, F);
        CHECK(F[0] >= 0, "oracle says the chosen radius %d does not fit", tf.rho);
        for (int q = 0; q < 3; ++q)
            if (fm & (1u << q))
                CHECK(F[q] == tf.F[q], "feature %d: library %" PRId64 ", oracle %" PRId64, q,
                      tf.F[q], F[q]);
        // a radius that does not fit is refused
        rc = oss_template_features(pix, &d, (h < w ? h : w), fm, &tf);
        CHECK(rc == OSS_E_ARG, "oversized radius rc %d", rc);
        // rings
        oss_template_feat rings[3];
        rc = oss_template_features_rings(pix, &d, -1, fm, 3, rings);
        CHECK(rc == OSS_OK || rc == OSS_E_ARG, "rings rc %d", rc);
        // moments
        oss_template_mom tm{};
        rc = oss_template_moments(pix, &d, -1, &tm);
        CHECK(rc == OSS_OK, "moments rc %d", rc);
        if (rc == OSS_OK) {
            int64_t M[4];
            oracle_moments(im.px.data(), h, w, w, &cx, &cy, 1, tm.rho, M);
            CHECK(M[0] == tm.F1 && M[1] == tm.F2 && M[2] == tm.Sx && M[3] == tm.Sy,
                  "moments differ from the oracle at rho %d", tm.rho);
        }
    }
}

static void check_bounds(std::mt19937 &rng)
{
    for (int trial = 0; trial < 3000; ++trial) {
        const int f = trial % 3;
        const int r = 1 + (int)(rng() % 200), rho = 1 + (int)(rng() % 200);
        const int64_t FT = (int64_t)(rng() % 100000000ull);
        oss_tolerance tol{};
        tol.Q = 1 + (int)(rng() % 1000);
        for (int q = 0; q < 3; ++q)
            tol.P[q] = (int)(rng() % (2 * tol.Q));
        int64_t lo = 0, hi = 0;
        int rc = oss_feature_bounds(f, FT, r, rho, &tol, &lo, &hi);
        CHECK(rc == OSS_OK, "bounds rc %d", rc);
        if (rc != OSS_OK || lo > hi)
            continue;
        const int P = tol.P[f], Q = tol.Q;
        CHECK(oracle_feature_pass(f, lo, FT, r, rho, P, Q), "lo %" PRId64 " fails", lo);
        CHECK(oracle_feature_pass(f, hi, FT, r, rho, P, Q), "hi %" PRId64 " fails", hi);
        CHECK(!oracle_feature_pass(f, lo - 1, FT, r, rho, P, Q), "lo-1 passes");
        CHECK(!oracle_feature_pass(f, hi + 1, FT, r, rho, P, Q), "hi+1 passes");
    }
    int64_t lo, hi;
    CHECK(oss_feature_bounds(3, 1, 1, 1, nullptr, &lo, &hi) == OSS_E_ARG, "bad feature accepted");
}

static void check_alg1(std::mt19937 &rng)
{
    Img im = make_img(rng, 33, 33, 8);
    std::vector<uint8_t> u8(im.px.begin(), im.px.end());
    oss_image_desc d{33, 33, 33, OSS_U8, 8};
    oss_alg1_params pa{1, 2, 2, 1, {4, 300, 6}, OSS_F_ALL};
    std::vector<oss_interval_probe> out(4096);
    int32_t n = 0;
    int rc = oss_alg1_probes(u8.data(), &d, 0, &pa, out.data(), (int32_t)out.size(), &n);
    CHECK(rc == OSS_OK && n > 0, "alg1 rc %d n %d", rc, n);
    for (int i = 0; i < n && i < (int)out.size(); ++i)
        for (int q = 0; q < 3; ++q)
            CHECK(out[i].lo[q] <= out[i].hi[q], "alg1 probe %d empty box", i);
    // too small a buffer: the count needed, OSS_E_NOMEM
    int32_t n2 = 0;
    rc = oss_alg1_probes(u8.data(), &d, 0, &pa, out.data(), 1, &n2);
    CHECK((n <= 1 && rc == OSS_OK) || (rc == OSS_E_NOMEM && n2 == n), "alg1 cap 1: rc %d", rc);
    oss_image_desc bad{33, 32, 32, OSS_U8, 8};
    CHECK(oss_alg1_probes(u8.data(), &bad, 0, &pa, out.data(), 16, &n2) == OSS_E_ARG,
          "non-square template accepted");
}

static void check_oracle_screen(std::mt19937 &rng)
{
    const int H = 48, W = 40;
    Img im = make_img(rng, H, W, 12);
    std::vector<int32_t> G((size_t)H * W);
    oracle_gradient(im.px.data(), H, W, W, G.data());
    std::vector<int32_t> xs, ys;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            xs.push_back(x);
            ys.push_back(y);
        }
    const int32_t probes[] = {0, 0, 3, 0, 1, 5, 1, 0, 4, 1, 3, 9};
    const int64_t FT[] = {1000, 400000, 3000, 2000, 900000, 5000};
    const int32_t rho[] = {4, 5};
    const int32_t P[] = {50, 80, 200};
    std::vector<uint32_t> bits(2 * xs.size());
    int rc = oracle_screen(im.px.data(), G.data(), H, W, W, xs.data(), ys.data(),
                           (int64_t)xs.size(), probes, 4, FT, rho, 2, 7, P, 100, bits.data());
    CHECK(rc == 0, "oracle screen rc %d", rc);
}

static void check_misc()
{
    for (int c = -10; c <= 1; ++c)
        CHECK(oss_status_string(c) != nullptr, "status %d", c);
    oss_image_desc d{4096, 4096, 4096, OSS_U8, 8};
    size_t b = 0;
    CHECK(oss_ref_bytes(&d, OSS_F_ALL, 64, &b) == OSS_OK && b > 0, "ref bytes");
    CHECK(oss_ref_bytes(nullptr, OSS_F_ALL, 64, &b) == OSS_E_ARG, "null desc accepted");
    oss_image_desc bad{4096, 4096, 100, OSS_U8, 8};  // pitch < width
    CHECK(oss_ref_bytes(&bad, OSS_F_ALL, 64, &b) == OSS_E_ARG, "short pitch accepted");
    oss_template_feat tf{};
    CHECK(oss_template_features(nullptr, &d, 3, OSS_F_ALL, &tf) == OSS_E_ARG, "null pixels");
}

int main()
{
    std::mt19937 rng(1707);
    check_misc();
    check_template_features(rng);
    check_bounds(rng);
    check_alg1(rng);
    check_oracle_screen(rng);
    if (g_fail) {
        std::fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("host sanitize driver: all checks passed\n");
    return 0;
}
