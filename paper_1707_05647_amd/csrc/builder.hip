// Integral-table builder: L (axis summed-area table, Eq. T_1), R and R'
// (45-degree triangular tables with the apex at the pixel centre / at the
// pixel corner; the summed triangular table of Sec. "Rotation Invariance")
// for each feature quantity q in {I, I^2, G}.
//
// The paper builds its tables by one horizontal and one vertical cumulative
// pass (Sec. "Patch Features") and "two diagonal passes" for the triangular
// one.  Here every table entry is written exactly once, in row bands of
// KBAND rows, from the band's own row prefixes plus the carry row above it:
//
//   row_base   per image row, the row prefix at every 64th column
//              (wavefront reductions of 64-column chunks + a block scan)
//   band_agg   per band tile, the band's own contribution to the carries
//              from its column, anti-diagonal and diagonal projections
//              (LDS atomics) and three block scans, not a row-by-row walk
//   carry      per line across bands, the carry rows: running sums of the
//              band contributions along columns (L), anti-diagonals (T_ad)
//              and diagonals (T_d)
//   band_final per band tile, the tables from the carry row: each row one
//              wavefront scan (DPP), one barrier, and one coalesced store
//              per entry (the row's R/R' are stored one row late, once the
//              neighbouring waves' diagonal carries are visible)
//
// Arithmetic is unsigned and wraps: with 32-bit storage every table is the
// exact sum modulo 2^32, which keeps every square and diamond sum exact as
// long as it is below 2^32 (the host checks that bound for the declared
// maximum radius before choosing 32-bit storage).
#include "oss_internal.h"

namespace oss {

static int cdiv(int a, int b) { return (a + b - 1) / b; }

BuildGeom make_geom(int H, int W, int nq, int ebytes, int sqi, int planar, int rec)
{
    BuildGeom g;
    g.H = H;
    g.W = W;
    g.nq = nq;
    g.ebytes = ebytes;
    g.sqi = sqi;
    g.planar = planar ? 1 : 0;
    g.rec = (rec && g.planar && sqi == 1 && nq == 3) ? 1 : 0;
    // Rows of a whole number of 128-byte lines, and entry index 0 (x = -1)
    // TAB_LINE - tab_es bytes into each table (plane) allocation: image
    // column 0 of every row then starts a line, so the final pass's 64-column
    // waves store whole lines and a star pass's centre-column lookups read
    // two lines per wave instead of three.
    g.pitch_e = ((int64_t)W + 1 + 31) / 32 * 32;
    if (g.planar) {
        g.tab_es = sqi >= 0 ? 4 : ebytes;
        g.plane = ((int64_t)(H + 1) * g.pitch_e * g.tab_es + TAB_LINE + 255) / 256 * 256;
        g.tab_bytes = g.plane * (sqi >= 0 ? nq + 1 : nq);
        if (g.rec)  // sum plane, record plane (twice its size), byte plane
            g.tab_bytes = 3 * g.plane +
                          ((int64_t)(H + 1) * g.pitch_e + TAB_LINE + 255) / 256 * 256;
    } else {
        g.tab_es = sqi >= 0 ? 16 : nq * ebytes;
        g.plane = 0;
        g.tab_bytes = (int64_t)(H + 1) * g.pitch_e * g.tab_es + TAB_LINE;
    }
    g.tab_off = TAB_LINE - g.tab_es;
    g.nb = cdiv(H + 1, KBAND);
    // final tiles: cores cover [-1, W-1]; the first core starts at -64+HALO <= -1
    g.fin_x0 = -64;
    g.nfin = cdiv((W - 1) - (g.fin_x0 + BAND_HALO) + 1, BAND_STRIDE);
    g.cx0 = g.fin_x0;
    g.cw = (g.nfin - 1) * BAND_STRIDE + BAND_THREADS;
    // projection tiles: cores cover the carry range
    g.agg_x0 = -128;
    g.nagg = cdiv((g.cx0 + g.cw - 1) - (g.agg_x0 + BAND_HALO) + 1, BAND_STRIDE);
    g.nbp = cdiv(W, 64) + 1;
    g.nt = 0;
    return g;
}

template <unsigned FM>
struct Feat {
    static constexpr int NQ = ((FM >> 0) & 1) + ((FM >> 1) & 1) + ((FM >> 2) & 1) +
                              ((FM >> 3) & 1) + ((FM >> 4) & 1);
};

// ---------------------------------------------------------------------------
// Wavefront primitives (DPP; 64-bit values move as two 32-bit halves).
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ uint32_t dpp(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, BOUND);
}

template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ uint64_t dpp(uint64_t v)
{
    const uint32_t lo = dpp<CTRL, ROW_MASK, BOUND>((uint32_t)v);
    const uint32_t hi = dpp<CTRL, ROW_MASK, BOUND>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// inclusive scan across the 64 lanes of a wavefront
template <typename T>
__device__ __forceinline__ T wave_scan(T v)
{
    v += dpp<0x111, 0xf, true>(v);  // row_shr:1
    v += dpp<0x112, 0xf, true>(v);  // row_shr:2
    v += dpp<0x114, 0xf, true>(v);  // row_shr:4
    v += dpp<0x118, 0xf, true>(v);  // row_shr:8
    v += dpp<0x142, 0xa, false>(v); // row_bcast:15 into rows 1, 3
    v += dpp<0x143, 0xc, false>(v); // row_bcast:31 into rows 2, 3
    return v;
}

// value of lane - 1 (lane 0: 0) / of lane + 1 (lane 63: 0)
template <typename T>
__device__ __forceinline__ T from_left(T v)
{
    return dpp<0x138, 0xf, false>(v);  // wave_shr:1
}
template <typename T>
__device__ __forceinline__ T from_right(T v)
{
    return dpp<0x130, 0xf, false>(v);  // wave_shl:1
}

// value of lane `src` (wave-uniform) for every lane
template <typename T>
__device__ __forceinline__ T read_lane(T v, int src)
{
    return (T)__builtin_amdgcn_readlane((int)v, src);
}
template <>
__device__ __forceinline__ uint64_t read_lane<uint64_t>(uint64_t v, int src)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

template <typename T>
__device__ __forceinline__ T lane63(T v)
{
    return read_lane(v, 63);
}

// Sum of the first `n` (wave-uniform, 0 <= n <= 8) of eight per-wave values:
// lane i < 8 holds value i (the others 0); a three-step prefix inside the
// first row of 16 lanes, then lane n-1's prefix.  Every lane must be active.
template <typename T>
__device__ __forceinline__ T first_n_sum(T v_lane, int n)
{
    v_lane += dpp<0x111, 0xf, true>(v_lane);  // row_shr:1
    v_lane += dpp<0x112, 0xf, true>(v_lane);  // row_shr:2
    v_lane += dpp<0x114, 0xf, true>(v_lane);  // row_shr:4
    return n > 0 ? read_lane(v_lane, n - 1) : (T)0;
}

// q values of the pixel (x, y) inside the image, in feature-bit order, from
// the pixel c, its left / right neighbours l, r and the pixels above / below
// u, d (neighbour indices clamped to the image); the first moments' column
// and row weights x c, y c are taken in T (modulo 2^32 for 32-bit tables).
template <unsigned FM, typename T>
__device__ __forceinline__ void quantities(int c, int l, int r, int u, int d, int x, int y, T *q)
{
    int slot = 0;
    if (FM & OSS_F_SUM)
        q[slot++] = (T)c;
    if (FM & OSS_F_SQ)
        q[slot++] = (T)((uint64_t)c * (uint64_t)c);
    if (FM & OSS_F_GRAD) {
        const int gx = r - l, gy = d - u;
        q[slot++] = (T)((gx < 0 ? -gx : gx) + (gy < 0 ? -gy : gy));
    }
    if (FM & OSS_F_XMOM)
        q[slot++] = (T)((uint64_t)x * (uint64_t)c);
    if (FM & OSS_F_YMOM)
        q[slot++] = (T)((uint64_t)y * (uint64_t)c);
}

template <typename Pix, unsigned FM, typename T>
__device__ __forceinline__ void load_q(const Pix *__restrict__ img, int64_t pitch, int H, int W,
                                       int x, int y, T *q)
{
    const Pix *row = img + (int64_t)y * pitch;
    const int xl = x > 0 ? x - 1 : 0, xr = x + 1 < W ? x + 1 : W - 1;
    const int yu = y > 0 ? y - 1 : 0, yd = y + 1 < H ? y + 1 : H - 1;
    int u = 0, d = 0, l = 0, r = 0;
    const int c = row[x];
    if (FM & OSS_F_GRAD) {
        l = row[xl];
        r = row[xr];
        u = img[(int64_t)yu * pitch + x];
        d = img[(int64_t)yd * pitch + x];
    }
    quantities<FM, T>(c, l, r, u, d, x, y, q);
}

// base P_y(X0 - 1) of a tile whose threads start at column X0 (a multiple of 64)
template <typename T>
__device__ __forceinline__ const T *tile_base(const T *__restrict__ bp, const BuildGeom &g, int y,
                                              int X0, int NQ)
{
    int j = X0 / 64;
    j = j < 0 ? 0 : (j > g.nbp - 1 ? g.nbp - 1 : j);
    return bp + ((int64_t)y * g.nbp + j) * NQ;
}

// ---------------------------------------------------------------------------
// row_base: bp[y][j] = P_y(64 j - 1) for j in [0, nbp); the last entry is
// the row total.  One block per row; a wave reduces 64-column chunks.
// ---------------------------------------------------------------------------
constexpr int RB_THREADS = 256;
constexpr int RB_MU = 4;  // chunks whose loads a wave has in flight together

template <typename Pix, unsigned FM, typename T>
__global__ __launch_bounds__(RB_THREADS) void row_base_kernel(const Pix *__restrict__ img,
                                                              int64_t pitch, BuildGeom g,
                                                              T *__restrict__ bp)
{
    constexpr int NQ = Feat<FM>::NQ;
    __shared__ T s_chunk[NQ][RB_THREADS];
    __shared__ T s_w[RB_THREADS / 64][NQ];
    const int y = blockIdx.x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nch = g.nbp - 1;  // 64-column chunks
    T carry[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        carry[q] = 0;
    T *out = bp + (int64_t)y * g.nbp * NQ;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            out[q] = 0;
    }
    constexpr int NWV = RB_THREADS / 64;
    for (int m0 = 0; m0 < nch; m0 += RB_THREADS) {
        // chunk sums for chunks m0 .. m0 + 255; a wave loads RB_MU chunks
        // before it scans any (clamped reads, out-of-range values zeroed)
        const int mend = min(m0 + RB_THREADS, nch);
        for (int mb = m0 + wid; mb < mend; mb += NWV * RB_MU) {
            T q[RB_MU][NQ];
#pragma unroll
            for (int u = 0; u < RB_MU; ++u) {
                const int m = mb + NWV * u;
                const int x = m * 64 + lane;
                const bool ok = m < mend && x < g.W;
                load_q<Pix, FM, T>(img, pitch, g.H, g.W, ok ? x : g.W - 1, y, q[u]);
#pragma unroll
                for (int k = 0; k < NQ; ++k)
                    q[u][k] = ok ? q[u][k] : (T)0;
            }
#pragma unroll
            for (int u = 0; u < RB_MU; ++u) {
                const int m = mb + NWV * u;
#pragma unroll
                for (int k = 0; k < NQ; ++k) {
                    const T s = lane63(wave_scan(q[u][k]));
                    if (lane == 0 && m < mend)
                        s_chunk[k][m - m0] = s;
                }
            }
        }
        __syncthreads();
        // block scan of the chunk sums
        const int m = m0 + threadIdx.x;
        T v[NQ];
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            v[k] = m < nch ? s_chunk[k][threadIdx.x] : (T)0;
            v[k] = wave_scan(v[k]);
            if (lane == 63)
                s_w[wid][k] = v[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            T off = carry[k], tot = carry[k];
            for (int w = 0; w < RB_THREADS / 64; ++w) {
                off += (w < wid) ? s_w[w][k] : (T)0;
                tot += s_w[w][k];
            }
            if (m < nch)
                out[(int64_t)(m + 1) * NQ + k] = off + v[k];
            carry[k] = tot;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// A band tile's pixels in LDS: px[rr][cc] = image pixel (clamped row
// ys - 1 + rr, clamped column X0 - 1 + cc) for rr < KBAND + 2, cc < PXW, so
// pixel (x, y) of the band and its clamped neighbours are px[y - ys + 1]
// [x - X0 + 1 +- 1] and the rows above and below.  Every row's load is in
// flight together (no branch between them; rows past the band are clamped
// reads that nothing uses).  Followed by a barrier in the caller.
// ---------------------------------------------------------------------------
constexpr int PXW = BAND_THREADS + 2;

template <typename Pix>
__device__ __forceinline__ void stage_band_pixels(Pix (*px)[PXW], const Pix *__restrict__ img,
                                                  int64_t pitch, int X0, int ys, int H, int W)
{
    static_assert(PXW - BAND_THREADS == 2, "two extra staged columns");
    const int tid = threadIdx.x;
    int xa = X0 - 1 + tid;
    xa = xa < 0 ? 0 : (xa > W - 1 ? W - 1 : xa);
    int va[KBAND + 2];
#pragma unroll
    for (int rr = 0; rr < KBAND + 2; ++rr) {
        int yy = ys - 1 + rr;
        yy = yy < 0 ? 0 : (yy > H - 1 ? H - 1 : yy);
        va[rr] = img[(int64_t)yy * pitch + xa];
    }
#pragma unroll
    for (int rr = 0; rr < KBAND + 2; ++rr)
        px[rr][tid] = (Pix)va[rr];
    if (tid < PXW - BAND_THREADS) {  // columns 512 and 513
        int xb = X0 - 1 + BAND_THREADS + tid;
        xb = xb < 0 ? 0 : (xb > W - 1 ? W - 1 : xb);
        int vb[KBAND + 2];
#pragma unroll
        for (int rr = 0; rr < KBAND + 2; ++rr) {
            int yy = ys - 1 + rr;
            yy = yy < 0 ? 0 : (yy > H - 1 ? H - 1 : yy);
            vb[rr] = img[(int64_t)yy * pitch + xb];
        }
#pragma unroll
        for (int rr = 0; rr < KBAND + 2; ++rr)
            px[rr][BAND_THREADS + tid] = (Pix)vb[rr];
    }
}

// ---------------------------------------------------------------------------
// band_agg: the band's contribution to the carry rows, for the core columns
// x of the tile (threads from X0 = agg_x0 + c * STRIDE, band rows y_s..y_e):
//   agg_L[x]  = sum_y P_y(x)             = B + sum_{X0 <= i <= x} colsum(i)
//   agg_AD[x] = sum_y P_y(x + y_e - y)   = B + sum over the tile's pixels with
//                                          (i - X0) + (y - y_s) <= (x - X0) + (y_e - y_s)
//   agg_D[x]  = sum_y P_y(x - (y_e - y)) = B + sum over the tile's pixels with
//                                          (i - X0) - (y - y_s) <= (x - X0) - (y_e - y_s)
// with B = sum_y P_y(X0 - 1).  The pixels are projected onto columns,
// anti-diagonals and diagonals (LDS atomic adds) and each projection is
// scanned once.
// ---------------------------------------------------------------------------
constexpr int PROJ = BAND_THREADS + KBAND;  // projection slots per tile

template <typename T, int NQ>
__device__ __forceinline__ void block_scan_lds(T (*arr)[PROJ], T (*s_w)[NQ])
{
    // inclusive scan of arr[q][0..PROJ) in place; thread t owns slots 2t, 2t+1
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int i0 = 2 * threadIdx.x;
    T a[NQ], b[NQ], s[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        a[q] = i0 < PROJ ? arr[q][i0] : (T)0;
        b[q] = i0 + 1 < PROJ ? arr[q][i0 + 1] : (T)0;
        s[q] = wave_scan((T)(a[q] + b[q]));
        if (lane == 63)
            s_w[wid][q] = s[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        T off = 0;
        for (int w = 0; w < BAND_THREADS / 64; ++w)
            off += (w < wid) ? s_w[w][q] : (T)0;
        const T incl = off + s[q];
        if (i0 < PROJ)
            arr[q][i0] = incl - b[q];
        if (i0 + 1 < PROJ)
            arr[q][i0 + 1] = incl;
    }
    __syncthreads();
}

template <typename Pix, unsigned FM, typename T>
__global__ __launch_bounds__(BAND_THREADS) void band_agg_kernel(
    const Pix *__restrict__ img, int64_t pitch, BuildGeom g, const T *__restrict__ bp,
    T *__restrict__ aL, T *__restrict__ aAD, T *__restrict__ aD)
{
    constexpr int NQ = Feat<FM>::NQ;
    constexpr int NW = BAND_THREADS / 64;
    __shared__ T s_ad[NQ][PROJ];
    __shared__ T s_d[NQ][PROJ];
    __shared__ T s_col[NQ][PROJ];
    __shared__ T s_w[NW][NQ];
    const int tid = threadIdx.x;
    const int X0 = g.agg_x0 + blockIdx.x * BAND_STRIDE;
    const int b = blockIdx.y;
    const int x = X0 + tid;
    const int ys = -1 + b * KBAND;
    const int rows = min(KBAND, g.H - ys);
    for (int i = tid; i < PROJ; i += BAND_THREADS) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            s_ad[q][i] = 0;
            s_d[q][i] = 0;
            s_col[q][i] = 0;
        }
    }
    __syncthreads();
    T col[NQ], B[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        col[q] = 0;
        B[q] = 0;
    }
    const bool inside = x >= 0 && x < g.W;
    // the band's pixels and row-prefix bases in LDS first: no global load
    // waits inside the row loop
    __shared__ Pix s_px[KBAND + 2][PXW];
    __shared__ T s_base[KBAND][NQ];
    stage_band_pixels<Pix>(s_px, img, pitch, X0, ys, g.H, g.W);
    if (tid < rows * NQ) {
        const int k = tid / NQ, q = tid - k * NQ;
        const int y = ys + k;
        s_base[k][q] = y >= 0 ? tile_base(bp, g, y, X0, NQ)[q] : (T)0;
    }
    __syncthreads();
    const int cx = x - X0 + 1;  // LDS column of image column x
    for (int k = 0; k < rows; ++k) {
        const int y = ys + k;
        if (y < 0)
            continue;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            B[q] += s_base[k][q];
        if (!inside)
            continue;
        T qv[NQ];
        quantities<FM, T>(s_px[k + 1][cx], s_px[k + 1][cx - 1], s_px[k + 1][cx + 1],
                          s_px[k][cx], s_px[k + 2][cx], x, y, qv);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            col[q] += qv[q];
            atomicAdd(&s_ad[q][tid + k], qv[q]);
            atomicAdd(&s_d[q][tid - k + KBAND - 1], qv[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        s_col[q][tid] = col[q];
    __syncthreads();
    block_scan_lds<T, NQ>(s_col, s_w);
    block_scan_lds<T, NQ>(s_ad, s_w);
    block_scan_lds<T, NQ>(s_d, s_w);
    const int core0 = X0 + BAND_HALO;
    if (x >= core0 && x < core0 + BAND_STRIDE && x >= g.cx0 && x < g.cx0 + g.cw) {
        const int64_t e = ((int64_t)b * g.cw + (x - g.cx0)) * NQ;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            aL[e + q] = B[q] + s_col[q][tid];
            aAD[e + q] = B[q] + s_ad[q][tid + rows - 1];
            aD[e + q] = B[q] + s_d[q][tid - rows + KBAND];
        }
    }
}

// ---------------------------------------------------------------------------
// carry: C^0 = 0 and, for a band of KBAND rows,
//   C_L^{b+1}[x]  = C_L^b[x]          + agg_L^b[x]
//   C_AD^{b+1}[x] = C_AD^b[x + KBAND] + agg_AD^b[x]
//   C_D^{b+1}[x]  = C_D^b[x - KBAND]  + agg_D^b[x]
// one thread per line; right of the carry range the anti-diagonal table
// equals the full row total L(W-1, .), left of it the diagonal table is 0.
// The loads of a group of bands are issued before the dependent sums.
// ---------------------------------------------------------------------------
constexpr int CW_UNROLL = 8;

template <typename T, int NQ>
__global__ __launch_bounds__(256) void carry_kernel(BuildGeom g, const T *__restrict__ aL,
                                                    const T *__restrict__ aAD,
                                                    const T *__restrict__ aD,
                                                    T *__restrict__ cL, T *__restrict__ cAD,
                                                    T *__restrict__ cD)
{
    const int kind = blockIdx.y;
    const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cw = g.cw;
    const int nb = g.nb;
    const int64_t span = (int64_t)(nb - 1) * KBAND;
    const int64_t ci_tot = (g.W - 1) - g.cx0;  // carry index of x = W-1
    T v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        v[q] = 0;
    if (kind == 0) {
        if (line >= cw)
            return;
        for (int b0 = 0; b0 < nb; b0 += CW_UNROLL) {
            T a[CW_UNROLL][NQ];
#pragma unroll
            for (int u = 0; u < CW_UNROLL; ++u)
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    a[u][q] = b0 + u < nb ? aL[(((int64_t)(b0 + u)) * cw + line) * NQ + q] : (T)0;
#pragma unroll
            for (int u = 0; u < CW_UNROLL; ++u) {
                if (b0 + u >= nb)
                    break;
                const int64_t e = (((int64_t)(b0 + u)) * cw + line) * NQ;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    cL[e + q] = v[q];
                    v[q] += a[u][q];
                }
            }
        }
    } else if (kind == 1) {
        // line lambda: carry index lambda - b*K at band b
        if (line >= cw + span)
            return;
        for (int b0 = 0; b0 < nb; b0 += CW_UNROLL) {
            if (line - (int64_t)b0 * KBAND < 0)
                break;
            T a[CW_UNROLL][NQ];
#pragma unroll
            for (int u = 0; u < CW_UNROLL; ++u) {
                const int b = b0 + u;
                const int64_t xn = line - (int64_t)(b + 1) * KBAND;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    T val = 0;
                    if (b < nb) {
                        if (xn >= cw)
                            val = aL[((int64_t)b * cw + ci_tot) * NQ + q];
                        else if (xn >= 0)
                            val = aAD[((int64_t)b * cw + xn) * NQ + q];
                    }
                    a[u][q] = val;
                }
            }
#pragma unroll
            for (int u = 0; u < CW_UNROLL; ++u) {
                const int b = b0 + u;
                if (b >= nb)
                    break;
                const int64_t xb = line - (int64_t)b * KBAND;
                if (xb >= 0 && xb < cw) {
                    const int64_t e = ((int64_t)b * cw + xb) * NQ;
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        cAD[e + q] = v[q];
                }
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    v[q] += a[u][q];
            }
        }
    } else {
        // line lambda - span: carry index lambda - span + b*K at band b
        if (line >= cw + span)
            return;
        const int64_t lam = line - span;
        for (int b0 = 0; b0 < nb; b0 += CW_UNROLL) {
            if (lam + (int64_t)b0 * KBAND >= cw)
                break;
            T a[CW_UNROLL][NQ];
#pragma unroll
            for (int u = 0; u < CW_UNROLL; ++u) {
                const int b = b0 + u;
                const int64_t xn = lam + (int64_t)(b + 1) * KBAND;
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    a[u][q] = (b < nb && xn >= 0 && xn < cw)
                                  ? aD[((int64_t)b * cw + xn) * NQ + q]
                                  : (T)0;
            }
#pragma unroll
            for (int u = 0; u < CW_UNROLL; ++u) {
                const int b = b0 + u;
                if (b >= nb)
                    break;
                const int64_t xb = lam + (int64_t)b * KBAND;
                if (xb >= 0 && xb < cw) {
                    const int64_t e = ((int64_t)b * cw + xb) * NQ;
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        cD[e + q] = v[q];
                }
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    v[q] += a[u][q];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// band_final: one tile of one band.  Thread state after row k-1: L, T_ad and
// T_d at its column.  Row k: q, wavefront scan, one barrier (which also
// publishes the previous row's T_ad of lane 0 and T_d of lane 63 of every
// wave), then
//   ta_r = T_ad(x+1, y-1), td_l = T_d(x-1, y-1)   (DPP, or the wave edges)
//   store row y-1:  L, R = T_ad(x) - td_l, R' = ta_r - td_l
//   advance:        L += P, T_ad = ta_r + P, T_d = td_l + P
// The last row is stored after one more barrier.
// ---------------------------------------------------------------------------
// Entry e of a table, by layout LAY: NQ values of T side by side
// (LAY_INTER), one value in each of NQ planes (LAY_PLANAR), the 16-byte mixed
// entry (64-bit squares from slot SQI, the other quantities modulo 2^32,
// written as one 16-byte store; LAY_MIX), or 32-bit planes with the squares
// split into a low-word and a high-word plane (LAY_PLANAR_MIX), or the sum
// plane, {squares low word, gradient} records and a byte plane of the
// squares' bits 32..39 (LAY_PLANAR_REC: sum, squares, gradient).  plane_b is
// the byte distance between planes (the sum plane's size).
enum { LAY_INTER = 0, LAY_PLANAR = 1, LAY_MIX = 2, LAY_PLANAR_MIX = 3, LAY_PLANAR_REC = 4 };

// One table value; NT: a non-temporal (streaming) store.  A compile-time
// choice: a run-time branch between the two stores is merged by the
// compiler into one ordinary store.
template <bool NT, typename V>
__device__ __forceinline__ void put(V *p, V v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename T, int NQ, int LAY, int SQI, bool NT>
__device__ __forceinline__ void store_entry(T *__restrict__ tab, int64_t e, const T *v,
                                            int64_t plane_b)
{
    if constexpr (LAY == LAY_PLANAR) {
        const int64_t pe = plane_b / (int64_t)sizeof(T);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            put<NT>(tab + q * pe + e, v[q]);
    } else if constexpr (LAY == LAY_PLANAR_MIX) {
        uint32_t *t32 = reinterpret_cast<uint32_t *>(tab);
        const int64_t pe = plane_b / 4;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int pl = q <= SQI ? q : q + 1;  // plane of quantity q
            put<NT>(t32 + pl * pe + e, (uint32_t)v[q]);
            if (q == SQI)
                put<NT>(t32 + (pl + 1) * pe + e, (uint32_t)((uint64_t)v[q] >> 32));
        }
    } else if constexpr (LAY == LAY_PLANAR_REC) {
        char *b = reinterpret_cast<char *>(tab);
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 rec = {(uint32_t)v[1], (uint32_t)v[2]};
        put<NT>(reinterpret_cast<uint32_t *>(b) + e, (uint32_t)v[0]);
        put<NT>(reinterpret_cast<u32x2 *>(b + plane_b - 4 + 8 * e), rec);
        put<NT>(reinterpret_cast<uint8_t *>(b + 3 * plane_b + 3 + e),
                (uint8_t)((uint64_t)v[1] >> 32));
    } else if constexpr (LAY == LAY_INTER) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            put<NT>(tab + e * NQ + q, v[q]);
    } else {
        uint32_t o[2] = {0u, 0u};
        int j = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (q != SQI)
                o[j++] = (uint32_t)v[q];
        const uint64_t sq = (uint64_t)v[SQI];
        const u32x4 w = {(uint32_t)sq, (uint32_t)(sq >> 32), o[0], o[1]};
        put<NT>(reinterpret_cast<u32x4 *>(reinterpret_cast<char *>(tab) + e * 16), w);
    }
}

template <typename Pix, unsigned FM, typename T, int LAY, int SQI, bool NT>
__global__ __launch_bounds__(BAND_THREADS) void band_final_kernel(
    const Pix *__restrict__ img, int64_t pitch, BuildGeom g, const T *__restrict__ bp,
    const T *__restrict__ cL, const T *__restrict__ cAD, const T *__restrict__ cD,
    T *__restrict__ tL, T *__restrict__ tR, T *__restrict__ tRp)
{
    constexpr int NQ = Feat<FM>::NQ;
    const int64_t plane_b = g.plane;
    constexpr int NW = BAND_THREADS / 64;
    static_assert(NW == 8, "first_n_sum adds eight wave totals");
    __shared__ T s_wt[2][NW][NQ];
    __shared__ T s_eta[2][NW][NQ];
    __shared__ T s_etd[2][NW][NQ];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int X0 = g.fin_x0 + blockIdx.x * BAND_STRIDE;
    const int b = blockIdx.y;
    const int x = X0 + tid;
    const int ys = -1 + b * KBAND;
    const int rows = min(KBAND, g.H - ys);
    const int W = g.W, H = g.H;
    const int core0 = X0 + BAND_HALO;
    const bool store = x >= core0 && x < core0 + BAND_STRIDE && x >= -1 && x <= W - 1;
    const bool inside = x >= 0 && x < W;

    T Lc[NQ], TA[NQ], TD[NQ];
    {
        const int64_t e = ((int64_t)b * g.cw + (x - g.cx0)) * NQ;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            Lc[q] = cL[e + q];
            TA[q] = cAD[e + q];
            TD[q] = cD[e + q];
        }
    }
    // The band's pixels (rows ys-1 .. ys+rows, columns X0-1 .. X0+512, both
    // clamped into the image) and row-prefix bases are staged in LDS first,
    // so the row loop issues no global loads: a global load consumed while
    // the previous rows' table stores are in flight would wait for those
    // stores too (loads and stores share one counter), one store round trip
    // per row.
    __shared__ Pix s_px[KBAND + 2][PXW];
    __shared__ T s_base[KBAND][NQ];
    stage_band_pixels<Pix>(s_px, img, pitch, X0, ys, H, W);
    if (tid < rows * NQ) {
        const int k = tid / NQ, q = tid - k * NQ;
        const int y = ys + k;
        s_base[k][q] = y >= 0 ? tile_base(bp, g, y, X0, NQ)[q] : (T)0;
    }
    __syncthreads();
    const int cx = x - X0 + 1;  // LDS column of image column x

    for (int k = 0; k < rows; ++k) {
        const int y = ys + k;
        T s[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            s[q] = 0;
        if (y >= 0 && inside) {
            // LDS row k + 1 holds image row y; rows k and k + 2 the clamped
            // rows above and below; columns cx -+ 1 the clamped neighbours
            quantities<FM, T>(s_px[k + 1][cx], s_px[k + 1][cx - 1], s_px[k + 1][cx + 1],
                              s_px[k][cx], s_px[k + 2][cx], x, y, s);
        }
        const int buf = k & 1;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            s[q] = wave_scan(s[q]);
            if (lane == 63) {
                s_wt[buf][wid][q] = s[q];
                s_etd[buf][wid][q] = TD[q];
            }
            if (lane == 0)
                s_eta[buf][wid][q] = TA[q];
        }
        __syncthreads();
        T ta_r[NQ], td_l[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            // the row prefix of the tile start plus the totals of the waves
            // to the left of this one
            const T wt = lane < NW ? s_wt[buf][lane & (NW - 1)][q] : (T)0;
            const T off = s_base[k][q] + first_n_sum(wt, wid);
            const T P = off + s[q];
            ta_r[q] = from_right(TA[q]);
            td_l[q] = from_left(TD[q]);
            if (lane == 63)
                ta_r[q] = wid + 1 < NW ? s_eta[buf][wid + 1][q] : (T)0;
            if (lane == 0)
                td_l[q] = wid > 0 ? s_etd[buf][wid - 1][q] : (T)0;
            s[q] = P;
        }
        if (k > 0 && store) {
            const int64_t e = (int64_t)y * g.pitch_e + (x + 1);  // row y-1
            T r[NQ], rp[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                r[q] = TA[q] - td_l[q];
                rp[q] = ta_r[q] - td_l[q];
            }
            store_entry<T, NQ, LAY, SQI, NT>(tL, e, Lc, plane_b);
            store_entry<T, NQ, LAY, SQI, NT>(tR, e, r, plane_b);
            store_entry<T, NQ, LAY, SQI, NT>(tRp, e, rp, plane_b);
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            Lc[q] += s[q];
            TA[q] = ta_r[q] + s[q];
            TD[q] = td_l[q] + s[q];
        }
    }
    // the band's last row
    const int buf = rows & 1;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (lane == 63)
            s_etd[buf][wid][q] = TD[q];
        if (lane == 0)
            s_eta[buf][wid][q] = TA[q];
    }
    __syncthreads();
    // neighbour values first, with every lane active (DPP reads from lanes
    // that are switched off return 0)
    T r[NQ], rp[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        T ta_r = from_right(TA[q]);
        T td_l = from_left(TD[q]);
        if (lane == 63)
            ta_r = wid + 1 < NW ? s_eta[buf][wid + 1][q] : (T)0;
        if (lane == 0)
            td_l = wid > 0 ? s_etd[buf][wid - 1][q] : (T)0;
        r[q] = TA[q] - td_l;
        rp[q] = ta_r - td_l;
    }
    if (store) {
        const int64_t e = (int64_t)(ys + rows) * g.pitch_e + (x + 1);
        store_entry<T, NQ, LAY, SQI, NT>(tL, e, Lc, plane_b);
        store_entry<T, NQ, LAY, SQI, NT>(tR, e, r, plane_b);
        store_entry<T, NQ, LAY, SQI, NT>(tRp, e, rp, plane_b);
    }
}

template <typename Pix, unsigned FM, typename T, int LAY = LAY_INTER, int SQI = -1>
static hipError_t build_t(const BuildGeom &g, const void *pixels, int64_t pitch_bytes,
                          const BuildBuffers &bb, hipStream_t st, Profiler *prof)
{
    constexpr int NQ = Feat<FM>::NQ;
    const Pix *img = static_cast<const Pix *>(pixels);
    const int64_t pitch = pitch_bytes / (int64_t)sizeof(Pix);
    T *bp = static_cast<T *>(bb.bp);
    T *aL = static_cast<T *>(bb.agg_L), *aAD = static_cast<T *>(bb.agg_AD),
      *aD = static_cast<T *>(bb.agg_D);
    T *cL = static_cast<T *>(bb.c_L), *cAD = static_cast<T *>(bb.c_AD),
      *cD = static_cast<T *>(bb.c_D);
    {
        ProfScope ps(prof, K_ROW_BASE, st);
        hipLaunchKernelGGL((row_base_kernel<Pix, FM, T>), dim3(g.H), dim3(RB_THREADS), 0, st, img,
                           pitch, g, bp);
    }
    {
        ProfScope ps(prof, K_BAND_AGG, st);
        hipLaunchKernelGGL((band_agg_kernel<Pix, FM, T>), dim3(g.nagg, g.nb), dim3(BAND_THREADS),
                           0, st, img, pitch, g, bp, aL, aAD, aD);
    }
    {
        ProfScope ps(prof, K_CARRY, st);
        const int lines = g.cw + (g.nb - 1) * KBAND;
        hipLaunchKernelGGL((carry_kernel<T, NQ>), dim3((lines + 255) / 256, 3), dim3(256), 0, st,
                           g, aL, aAD, aD, cL, cAD, cD);
    }
    {
        ProfScope ps(prof, K_BAND_FINAL, st);
        if (g.nt)
            hipLaunchKernelGGL((band_final_kernel<Pix, FM, T, LAY, SQI, true>),
                               dim3(g.nfin, g.nb), dim3(BAND_THREADS), 0, st, img, pitch, g, bp,
                               cL, cAD, cD, static_cast<T *>(bb.L), static_cast<T *>(bb.R),
                               static_cast<T *>(bb.Rp));
        else
            hipLaunchKernelGGL((band_final_kernel<Pix, FM, T, LAY, SQI, false>),
                               dim3(g.nfin, g.nb), dim3(BAND_THREADS), 0, st, img, pitch, g, bp,
                               cL, cAD, cD, static_cast<T *>(bb.L), static_cast<T *>(bb.R),
                               static_cast<T *>(bb.Rp));
    }
    return hipGetLastError();
}

template <typename Pix, typename T>
static hipError_t build_pix(const BuildGeom &g, const void *px, int64_t pb, uint32_t fm,
                            const BuildBuffers &bb, hipStream_t st, Profiler *pr)
{
    if (g.sqi >= 0) {
        // 64-bit accumulation, the squares stored in 64 bits
        if (g.planar) {
            switch (fm) {
            case 3: return build_t<Pix, 3, uint64_t, LAY_PLANAR_MIX, 1>(g, px, pb, bb, st, pr);
            case 6: return build_t<Pix, 6, uint64_t, LAY_PLANAR_MIX, 0>(g, px, pb, bb, st, pr);
            case 7:
                return g.rec ? build_t<Pix, 7, uint64_t, LAY_PLANAR_REC, 1>(g, px, pb, bb, st, pr)
                             : build_t<Pix, 7, uint64_t, LAY_PLANAR_MIX, 1>(g, px, pb, bb, st, pr);
            default: return hipErrorInvalidValue;
            }
        }
        switch (fm) {
        case 3: return build_t<Pix, 3, uint64_t, LAY_MIX, 1>(g, px, pb, bb, st, pr);
        case 6: return build_t<Pix, 6, uint64_t, LAY_MIX, 0>(g, px, pb, bb, st, pr);
        case 7: return build_t<Pix, 7, uint64_t, LAY_MIX, 1>(g, px, pb, bb, st, pr);
        default: return hipErrorInvalidValue;
        }
    }
    if (g.planar) {
        switch (fm) {
        case 1: return build_t<Pix, 1, T, LAY_PLANAR>(g, px, pb, bb, st, pr);
        case 2: return build_t<Pix, 2, T, LAY_PLANAR>(g, px, pb, bb, st, pr);
        case 3: return build_t<Pix, 3, T, LAY_PLANAR>(g, px, pb, bb, st, pr);
        case 4: return build_t<Pix, 4, T, LAY_PLANAR>(g, px, pb, bb, st, pr);
        case 5: return build_t<Pix, 5, T, LAY_PLANAR>(g, px, pb, bb, st, pr);
        case 6: return build_t<Pix, 6, T, LAY_PLANAR>(g, px, pb, bb, st, pr);
        case 7: return build_t<Pix, 7, T, LAY_PLANAR>(g, px, pb, bb, st, pr);
        case 25: return build_t<Pix, 25, T, LAY_PLANAR>(g, px, pb, bb, st, pr);
        case 27: return build_t<Pix, 27, T, LAY_PLANAR>(g, px, pb, bb, st, pr);
        default: return hipErrorInvalidValue;
        }
    }
    switch (fm) {
    case 25: return build_t<Pix, 25, T>(g, px, pb, bb, st, pr);
    case 27: return build_t<Pix, 27, T>(g, px, pb, bb, st, pr);
    case 1: return build_t<Pix, 1, T>(g, px, pb, bb, st, pr);
    case 2: return build_t<Pix, 2, T>(g, px, pb, bb, st, pr);
    case 3: return build_t<Pix, 3, T>(g, px, pb, bb, st, pr);
    case 4: return build_t<Pix, 4, T>(g, px, pb, bb, st, pr);
    case 5: return build_t<Pix, 5, T>(g, px, pb, bb, st, pr);
    case 6: return build_t<Pix, 6, T>(g, px, pb, bb, st, pr);
    case 7: return build_t<Pix, 7, T>(g, px, pb, bb, st, pr);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_build(const BuildGeom &g, const void *pixels, int64_t pitch_bytes, int dtype,
                        uint32_t feat_mask, const BuildBuffers &bb, hipStream_t stream,
                        Profiler *prof)
{
    if (g.sqi >= 0 && g.ebytes != 8)
        return hipErrorInvalidValue;
    if (g.ebytes == 4) {
        if (dtype == OSS_U8)
            return build_pix<uint8_t, uint32_t>(g, pixels, pitch_bytes, feat_mask, bb, stream,
                                                prof);
        return build_pix<uint16_t, uint32_t>(g, pixels, pitch_bytes, feat_mask, bb, stream, prof);
    }
    if (dtype == OSS_U8)
        return build_pix<uint8_t, uint64_t>(g, pixels, pitch_bytes, feat_mask, bb, stream, prof);
    return build_pix<uint16_t, uint64_t>(g, pixels, pitch_bytes, feat_mask, bb, stream, prof);
}

}  // namespace oss
