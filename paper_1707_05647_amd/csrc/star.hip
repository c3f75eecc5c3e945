// Star features + screening compare (plain form: one launch per template).
//
// For a position (x, y) and radius r, with s = s(r) (Sec. "Rotation
// Invariance", Eq. S_os: square and diamond superimposed) the feature sum of
// every quantity is 8 table lookups by inclusion-exclusion:
//   square  (Eq. S_1)      L(x+s,y+s) - L(x-s-1,y+s) - L(x+s,y-s-1) + L(x-s-1,y-s-1)
//   diamond (triangular)   R(x,y+r) - R'(x-r-1,y-1) - R'(x+r,y-1) + R(x,y-r-1)
// In the rotated coordinates u = x+y, v = y-x a diamond is a rectangle; the
// four corners fall on pixel centres (R) and on pixel corners (R').  Every
// lookup of a valid position stays inside x in [-1, W-1], y in [-1, H-1].
//
// The compare (Algorithm 1, patch loop) is the exact relative interval
// (Q-P) X_T <= Q X_ref <= (Q+P) X_T, solved once per probe on the host for
// the feature sum itself: lo <= F <= hi with integer lo, hi.  Each thread
// therefore does two int64 compares per feature and probe.
//
// One thread per position; a wave covers 64 consecutive columns of one row,
// so each lookup is a coalesced, wave-uniform-offset read of the tables
// (the feature quantities of one entry sit next to each other).  With
// 32-bit tables the square and the diamond sums are formed modulo 2^32
// (each is below 2^32, so exact) and widened before they are added.  A
// thread walks all radii of its template (up to 32) and ORs the passing
// scales' bits.  Blocks are assigned XCD-major: the blocks that one XCD
// receives (every 8th block id) cover a contiguous run of rows, so the rows
// a radius' lookups revisit 2r+1 rows later stay in that XCD's L2 / the
// shared Infinity Cache.
#include "oss_internal.h"

namespace oss {

constexpr int STAR_THREADS = 256;

template <typename T, int NQ>
__device__ __forceinline__ void ld(const T *__restrict__ tab, int64_t e, T *v)
{
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        v[q] = tab[e * NQ + q];
}

// Sum of two region sums that were formed in T: with 32-bit tables each
// region sum is exact modulo 2^32 and below 2^32, so it zero-extends.
__device__ __forceinline__ int64_t widen(uint32_t v) { return (int64_t)v; }
__device__ __forceinline__ int64_t widen(uint64_t v) { return (int64_t)v; }

template <typename T, int NQ>
__global__ __launch_bounds__(STAR_THREADS) void star_plain_kernel(
    const T *__restrict__ L, const T *__restrict__ R, const T *__restrict__ Rp, int64_t pitch_e,
    int H, int W, const DevTemplatePlan *__restrict__ plan, uint32_t *__restrict__ bits,
    int tiles_x, int n_tiles)
{
    const int per_xcd = gridDim.x >> 3;
    const int tile = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (tile >= n_tiles)
        return;
    const int y = tile / tiles_x;
    const int x = (tile - y * tiles_x) * STAR_THREADS + threadIdx.x;
    uint32_t acc = 0;
    const int nr = plan->n_radii;
    for (int j = 0; j < nr; ++j) {
        const int r = plan->radii[j].r;
        const int s = plan->radii[j].s;
        if (y < r || y > H - 1 - r)
            continue;
        if (x < r || x > W - 1 - r)
            continue;
        // entry index of (x, y) is (y+1)*pitch_e + (x+1)
        const int64_t e0 = (int64_t)(y + 1) * pitch_e + (x + 1);
        const int64_t dys = (int64_t)s * pitch_e;
        const int64_t dys1 = (int64_t)(s + 1) * pitch_e;
        const int64_t dyr = (int64_t)r * pitch_e;
        const int64_t dyr1 = (int64_t)(r + 1) * pitch_e;
        T a[NQ], b[NQ], c[NQ], d[NQ];
        int64_t F[NQ];
        ld<T, NQ>(L, e0 + dys + s, a);
        ld<T, NQ>(L, e0 + dys - s - 1, b);
        ld<T, NQ>(L, e0 - dys1 + s, c);
        ld<T, NQ>(L, e0 - dys1 - s - 1, d);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            F[q] = widen((T)(a[q] - b[q] - c[q] + d[q]));
        ld<T, NQ>(R, e0 + dyr, a);
        ld<T, NQ>(Rp, e0 - pitch_e - r - 1, b);
        ld<T, NQ>(Rp, e0 - pitch_e + r, c);
        ld<T, NQ>(R, e0 - dyr1, d);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            F[q] += widen((T)(a[q] - b[q] - c[q] + d[q]));
        const int p0 = plan->radii[j].first;
        const int p1 = p0 + plan->radii[j].count;
        for (int p = p0; p < p1; ++p) {
            const DevProbe &pr = plan->probes[p];
            bool pass = true;
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                pass = pass && F[q] >= pr.lo[q] && F[q] <= pr.hi[q];
            acc |= pass ? (1u << pr.k) : 0u;
        }
    }
    if (x < W)
        bits[(int64_t)y * W + x] = acc;
}

template <typename T>
static hipError_t star_t(const BuildGeom &g, const void *L, const void *R, const void *Rp,
                         const DevTemplatePlan *plan, uint32_t *bits, hipStream_t stream)
{
    const int tiles_x = (g.W + STAR_THREADS - 1) / STAR_THREADS;
    const int n_tiles = tiles_x * g.H;
    const int nblk = (n_tiles + 7) / 8 * 8;
    const T *l = static_cast<const T *>(L), *r = static_cast<const T *>(R),
            *rp = static_cast<const T *>(Rp);
    switch (g.nq) {
    case 1:
        hipLaunchKernelGGL((star_plain_kernel<T, 1>), dim3(nblk), dim3(STAR_THREADS), 0, stream,
                           l, r, rp, g.pitch_e, g.H, g.W, plan, bits, tiles_x, n_tiles);
        break;
    case 2:
        hipLaunchKernelGGL((star_plain_kernel<T, 2>), dim3(nblk), dim3(STAR_THREADS), 0, stream,
                           l, r, rp, g.pitch_e, g.H, g.W, plan, bits, tiles_x, n_tiles);
        break;
    case 3:
        hipLaunchKernelGGL((star_plain_kernel<T, 3>), dim3(nblk), dim3(STAR_THREADS), 0, stream,
                           l, r, rp, g.pitch_e, g.H, g.W, plan, bits, tiles_x, n_tiles);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_star_plain(const BuildGeom &g, const void *L, const void *R, const void *Rp,
                             const DevTemplatePlan *plan, uint32_t *bits, hipStream_t stream,
                             Profiler *prof)
{
    ProfScope ps(prof, K_STAR, stream);
    if (g.ebytes == 4)
        return star_t<uint32_t>(g, L, R, Rp, plan, bits, stream);
    return star_t<uint64_t>(g, L, R, Rp, plan, bits, stream);
}

}  // namespace oss
