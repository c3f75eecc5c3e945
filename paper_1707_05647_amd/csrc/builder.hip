// Integral-table builder: L (axis summed-area table, Eq. T_1), R and R'
// (45-degree triangular tables with the apex at the pixel centre / at the
// pixel corner; the summed triangular table of Sec. "Rotation Invariance")
// for each feature quantity q in {I, I^2, G}.
//
// The paper builds its tables by one horizontal and one vertical cumulative
// pass (Sec. "Patch Features") and "two diagonal passes" for the triangular
// one.  Here every table is written exactly once, in row bands of KBAND
// rows, from the row prefix P_y(x) of the band's own rows plus a carry row
// (the three tables at the row above the band):
//
//   K0 row_base   per image row, P_y at the left edge of every band tile
//                 (one block per row: segment sums + block scan)
//   K1 band<agg>  per band tile, the band's own contribution with zero
//                 carries, kept only at the band's last row
//   K2 carry      per line across bands, the carry rows: a running sum of
//                 the band contributions along columns (L), anti-diagonals
//                 (T_ad) and diagonals (T_d)
//   K3 band<fin>  per band tile, the final tables from the carry row, one
//                 coalesced store per entry
//
// Inside a band a tile of 512 threads owns 512 consecutive columns (one
// column per thread): each row it computes q, the row prefix by an
// LDS-staged block scan (64-lane wavefront scans combined through LDS), and
// advances the three recurrences, exchanging the shifted diagonal carries
// with its neighbours through LDS.  A tile writes only its core columns;
// the 33-column halos on both sides absorb the diagonal dependencies
// (a diagonal carry moves one column per row).
#include "oss_internal.h"

namespace oss {

static int cdiv(int a, int b) { return (a + b - 1) / b; }

BuildGeom make_geom(int H, int W, int nq)
{
    BuildGeom g;
    g.H = H;
    g.W = W;
    g.nq = nq;
    g.pitch_e = ((int64_t)W + 1 + 15) / 16 * 16;
    g.nb = cdiv(H + 1, KBAND);
    g.cx0 = -2 - KBAND;
    g.cw = W + 2 * KBAND + 3;
    g.nch_agg = cdiv(g.cw, BAND_CORE_MAX);
    g.wc_agg = cdiv(g.cw, g.nch_agg);
    g.nch_fin = cdiv(W + 1, BAND_CORE_MAX);
    g.wc_fin = cdiv(W + 1, g.nch_fin);
    return g;
}

template <unsigned FM>
struct Feat {
    static constexpr int NQ = ((FM >> 0) & 1) + ((FM >> 1) & 1) + ((FM >> 2) & 1);
};

// q values of pixel (x, y) (inside the image) in feature-bit order.
template <typename Pix, unsigned FM>
__device__ __forceinline__ void load_q(const Pix *__restrict__ img, int64_t pitch, int H, int W,
                                       int x, int y, int64_t *q)
{
    const Pix *row = img + (int64_t)y * pitch;
    const int v = row[x];
    int slot = 0;
    if (FM & OSS_F_SUM)
        q[slot++] = v;
    if (FM & OSS_F_SQ)
        q[slot++] = (int64_t)v * v;
    if (FM & OSS_F_GRAD) {
        const int xr = x + 1 < W ? x + 1 : W - 1;
        const int xl = x > 0 ? x - 1 : 0;
        const int yd = y + 1 < H ? y + 1 : H - 1;
        const int yu = y > 0 ? y - 1 : 0;
        const int gx = (int)row[xr] - (int)row[xl];
        const int gy = (int)img[(int64_t)yd * pitch + x] - (int)img[(int64_t)yu * pitch + x];
        q[slot++] = (gx < 0 ? -gx : gx) + (gy < 0 ? -gy : gy);
    }
}

// Inclusive scan of NQ int64 values over the block (NWAVES waves of 64).
// s_w holds NWAVES*NQ partial sums; the caller must separate two uses of
// s_w by a barrier.
template <int NQ, int NWAVES>
__device__ __forceinline__ void block_incl_scan(int64_t *v, int64_t *s_w, int64_t *total)
{
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int64_t t = __shfl_up(v[q], d, 64);
            if (lane >= d)
                v[q] += t;
        }
    }
    if (lane == 63) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            s_w[wid * NQ + q] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        int64_t off = 0, tot = 0;
        for (int w = 0; w < NWAVES; ++w) {
            const int64_t s = s_w[w * NQ + q];
            off += (w < wid) ? s : 0;
            tot += s;
        }
        v[q] += off;
        if (total)
            total[q] = tot;
    }
}

// ---------------------------------------------------------------------------
// K0: bases of the row prefix.  For image row y and each tile c of each pass,
// writes P_y(x_start(c) - 1), x_start = first column of the tile's threads.
// ---------------------------------------------------------------------------
constexpr int ROWBASE_THREADS = 256;

template <typename Pix, unsigned FM>
__global__ __launch_bounds__(ROWBASE_THREADS) void row_base_kernel(
    const Pix *__restrict__ img, int64_t pitch, BuildGeom g, int64_t *__restrict__ bp_agg,
    int64_t *__restrict__ bp_fin)
{
    constexpr int NQ = Feat<FM>::NQ;
    __shared__ int64_t s_w[(ROWBASE_THREADS / 64) * NQ];
    const int y = blockIdx.x;
    const int W = g.W;
    const int seg = (W + ROWBASE_THREADS - 1) / ROWBASE_THREADS;
    const int x0 = threadIdx.x * seg;
    const int x1 = min(x0 + seg, W);
    int64_t sum[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        sum[q] = 0;
    for (int x = x0; x < x1; ++x) {
        int64_t qv[NQ];
        load_q<Pix, FM>(img, pitch, g.H, W, x, y, qv);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            sum[q] += qv[q];
    }
    int64_t incl[NQ], tot[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        incl[q] = sum[q];
    block_incl_scan<NQ, ROWBASE_THREADS / 64>(incl, s_w, tot);
    // exclusive prefix at x0
    int64_t excl[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        excl[q] = incl[q] - sum[q];

    for (int pass = 0; pass < 2; ++pass) {
        const int nch = pass == 0 ? g.nch_agg : g.nch_fin;
        const int wc = pass == 0 ? g.wc_agg : g.wc_fin;
        const int core0 = pass == 0 ? g.cx0 : -1;
        int64_t *out = pass == 0 ? bp_agg : bp_fin;
        for (int c = 0; c < nch; ++c) {
            const int col = core0 + c * wc - BAND_HALO - 1;
            int64_t *dst = out + ((int64_t)y * nch + c) * NQ;
            if (col < 0 || col >= W - 1) {
                if (threadIdx.x == 0) {
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        dst[q] = col < 0 ? 0 : tot[q];
                }
            } else if (col >= x0 && col < x1) {
                int64_t acc[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    acc[q] = excl[q];
                for (int x = x0; x <= col; ++x) {
                    int64_t qv[NQ];
                    load_q<Pix, FM>(img, pitch, g.H, W, x, y, qv);
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        acc[q] += qv[q];
                }
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    dst[q] = acc[q];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// K1 / K3: one band tile.  FINAL = false: zero carries, store the band's own
// contribution at its last row into (outA, outB, outC) = (agg_L, agg_AD,
// agg_D) over the carry range.  FINAL = true: start from the carry row and
// store L, R, R' for every row of the band.
// ---------------------------------------------------------------------------
template <typename Pix, unsigned FM, bool FINAL>
__global__ __launch_bounds__(BAND_THREADS) void band_kernel(
    const Pix *__restrict__ img, int64_t pitch, BuildGeom g, const int64_t *__restrict__ bp,
    const int64_t *__restrict__ cL, const int64_t *__restrict__ cAD,
    const int64_t *__restrict__ cD, int64_t *__restrict__ outA, int64_t *__restrict__ outB,
    int64_t *__restrict__ outC)
{
    constexpr int NQ = Feat<FM>::NQ;
    constexpr int NW = BAND_THREADS / 64;
    __shared__ int64_t s_w[NW * NQ];
    __shared__ int64_t s_ta[2][NQ][BAND_THREADS];
    __shared__ int64_t s_td[2][NQ][BAND_THREADS];

    const int c = blockIdx.x;
    const int b = blockIdx.y;
    const int tid = threadIdx.x;
    const int nch = FINAL ? g.nch_fin : g.nch_agg;
    const int wc = FINAL ? g.wc_fin : g.wc_agg;
    const int core0 = FINAL ? -1 : g.cx0;
    const int core_last = FINAL ? g.W - 1 : g.cx0 + g.cw - 1;
    const int xs = core0 + c * wc;
    const int xe = min(xs + wc - 1, core_last);
    const int x = xs - BAND_HALO + tid;
    const bool in_core = x >= xs && x <= xe;
    const int ys = -1 + b * KBAND;
    const int rows = min(KBAND, g.H - ys);
    const int W = g.W, H = g.H;

    // L(x, y-1), T_ad(x+1, y-1), T_d(x-1, y-1)
    int64_t Lc[NQ], ta_r[NQ], td_l[NQ], TA[NQ], TD[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        Lc[q] = 0;
        ta_r[q] = 0;
        td_l[q] = 0;
        TA[q] = 0;
        TD[q] = 0;
    }
    if (FINAL) {
        const int64_t row = (int64_t)b * g.cw;
        const int ci = x - g.cx0;
        if (ci >= 0 && ci < g.cw) {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                Lc[q] = cL[(row + ci) * NQ + q];
        }
        if (ci + 1 >= 0 && ci + 1 < g.cw) {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                ta_r[q] = cAD[(row + ci + 1) * NQ + q];
        }
        if (ci - 1 >= 0 && ci - 1 < g.cw) {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                td_l[q] = cD[(row + ci - 1) * NQ + q];
        }
    }

    for (int k = 0; k < rows; ++k) {
        const int y = ys + k;
        int64_t P[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            P[q] = 0;
        if (y >= 0 && x >= 0 && x < W)
            load_q<Pix, FM>(img, pitch, H, W, x, y, P);
        block_incl_scan<NQ, NW>(P, s_w, nullptr);
        if (y >= 0) {
            const int64_t *base = bp + ((int64_t)y * nch + c) * NQ;
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                P[q] += base[q];
        }
        const int buf = k & 1;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            Lc[q] += P[q];
            TA[q] = ta_r[q] + P[q];
            TD[q] = td_l[q] + P[q];
            s_ta[buf][q][tid] = TA[q];
            s_td[buf][q][tid] = TD[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            ta_r[q] = tid + 1 < BAND_THREADS ? s_ta[buf][q][tid + 1] : 0;
            td_l[q] = tid > 0 ? s_td[buf][q][tid - 1] : 0;
        }
        if (FINAL && in_core) {
            const int64_t e = ((int64_t)(y + 1) * g.pitch_e + (x + 1)) * NQ;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                outA[e + q] = Lc[q];
                outB[e + q] = TA[q] - td_l[q];
                outC[e + q] = ta_r[q] - td_l[q];
            }
        }
    }
    if (!FINAL && in_core) {
        const int64_t e = ((int64_t)b * g.cw + (x - g.cx0)) * NQ;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            outA[e + q] = Lc[q];
            outB[e + q] = TA[q];
            outC[e + q] = TD[q];
        }
    }
}

// ---------------------------------------------------------------------------
// K2: carry rows.  C^0 = 0 and, for band b with KBAND rows,
//   C_L^{b+1}[x]  = C_L^b[x]           + agg_L^b[x]
//   C_AD^{b+1}[x] = C_AD^b[x + KBAND]  + agg_AD^b[x]
//   C_D^{b+1}[x]  = C_D^b[x - KBAND]   + agg_D^b[x]
// walked by one thread per line.  Beyond the right end of the carry range
// the anti-diagonal table equals the full row total L(W-1, .); left of it
// the diagonal table is zero.
// ---------------------------------------------------------------------------
template <int NQ>
__global__ __launch_bounds__(256) void carry_kernel(BuildGeom g, const int64_t *__restrict__ aL,
                                                    const int64_t *__restrict__ aAD,
                                                    const int64_t *__restrict__ aD,
                                                    int64_t *__restrict__ cL,
                                                    int64_t *__restrict__ cAD,
                                                    int64_t *__restrict__ cD)
{
    const int kind = blockIdx.y;
    const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int cw = g.cw, nb = g.nb;
    const int span = (nb - 1) * KBAND;
    const int ci_tot = (g.W - 1) - g.cx0;  // index of x = W-1
    int64_t v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        v[q] = 0;
    if (kind == 0) {
        if (line >= cw)
            return;
        for (int b = 0; b < nb; ++b) {
            const int64_t e = ((int64_t)b * cw + line) * NQ;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                cL[e + q] = v[q];
                v[q] += aL[e + q];
            }
        }
    } else if (kind == 1) {
        // lines lambda in [0, cw + span): index of x at band b is lambda - b*K
        if (line >= cw + span)
            return;
        for (int b = 0; b < nb; ++b) {
            const int64_t xb = line - (int64_t)b * KBAND;
            if (xb < 0)
                break;
            if (xb < cw) {
                const int64_t e = ((int64_t)b * cw + xb) * NQ;
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    cAD[e + q] = v[q];
            }
            const int64_t xn = xb - KBAND;
            const int64_t et = ((int64_t)b * cw + ci_tot) * NQ;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int64_t bt = aL[et + q];
                int64_t a;
                if (xn >= cw)
                    a = bt;
                else if (xn >= 0)
                    a = aAD[((int64_t)b * cw + xn) * NQ + q];
                else
                    a = 0;
                v[q] += a;
            }
        }
    } else {
        // lines lambda in [-span, cw): index of x at band b is lambda + b*K
        if (line >= cw + span)
            return;
        const int64_t lam = line - span;
        for (int b = 0; b < nb; ++b) {
            const int64_t xb = lam + (int64_t)b * KBAND;
            if (xb >= cw)
                break;
            if (xb >= 0) {
                const int64_t e = ((int64_t)b * cw + xb) * NQ;
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    cD[e + q] = v[q];
            }
            const int64_t xn = xb + KBAND;
            if (xn >= 0 && xn < cw) {
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    v[q] += aD[((int64_t)b * cw + xn) * NQ + q];
            }
        }
    }
}

template <typename Pix, unsigned FM>
static hipError_t build_t(const BuildGeom &g, const void *pixels, int64_t pitch_bytes,
                          const BuildBuffers &bb, hipStream_t st, Profiler *prof)
{
    constexpr int NQ = Feat<FM>::NQ;
    const Pix *img = static_cast<const Pix *>(pixels);
    const int64_t pitch = pitch_bytes / (int64_t)sizeof(Pix);
    {
        ProfScope ps(prof, K_ROW_BASE, st);
        hipLaunchKernelGGL((row_base_kernel<Pix, FM>), dim3(g.H), dim3(ROWBASE_THREADS), 0, st,
                           img, pitch, g, bb.bp_agg, bb.bp_fin);
    }
    {
        ProfScope ps(prof, K_BAND_AGG, st);
        hipLaunchKernelGGL((band_kernel<Pix, FM, false>), dim3(g.nch_agg, g.nb),
                           dim3(BAND_THREADS), 0, st, img, pitch, g, bb.bp_agg, nullptr, nullptr,
                           nullptr, bb.agg_L, bb.agg_AD, bb.agg_D);
    }
    {
        ProfScope ps(prof, K_CARRY, st);
        const int span = (g.nb - 1) * KBAND;
        const int lines = g.cw + span;
        hipLaunchKernelGGL((carry_kernel<NQ>), dim3((lines + 255) / 256, 3), dim3(256), 0, st, g,
                           bb.agg_L, bb.agg_AD, bb.agg_D, bb.c_L, bb.c_AD, bb.c_D);
    }
    {
        ProfScope ps(prof, K_BAND_FINAL, st);
        hipLaunchKernelGGL((band_kernel<Pix, FM, true>), dim3(g.nch_fin, g.nb), dim3(BAND_THREADS),
                           0, st, img, pitch, g, bb.bp_fin, bb.c_L, bb.c_AD, bb.c_D, bb.L, bb.R,
                           bb.Rp);
    }
    return hipGetLastError();
}

template <typename Pix>
static hipError_t build_pix(const BuildGeom &g, const void *px, int64_t pb, uint32_t fm,
                            const BuildBuffers &bb, hipStream_t st, Profiler *pr)
{
    switch (fm) {
    case 1: return build_t<Pix, 1>(g, px, pb, bb, st, pr);
    case 2: return build_t<Pix, 2>(g, px, pb, bb, st, pr);
    case 3: return build_t<Pix, 3>(g, px, pb, bb, st, pr);
    case 4: return build_t<Pix, 4>(g, px, pb, bb, st, pr);
    case 5: return build_t<Pix, 5>(g, px, pb, bb, st, pr);
    case 6: return build_t<Pix, 6>(g, px, pb, bb, st, pr);
    case 7: return build_t<Pix, 7>(g, px, pb, bb, st, pr);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_build(const BuildGeom &g, const void *pixels, int64_t pitch_bytes, int dtype,
                        uint32_t feat_mask, const BuildBuffers &bb, hipStream_t stream,
                        Profiler *prof)
{
    if (dtype == OSS_U8)
        return build_pix<uint8_t>(g, pixels, pitch_bytes, feat_mask, bb, stream, prof);
    return build_pix<uint16_t>(g, pixels, pitch_bytes, feat_mask, bb, stream, prof);
}

}  // namespace oss
