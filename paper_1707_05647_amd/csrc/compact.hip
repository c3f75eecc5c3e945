// Candidate list from the star passes' segment output (Algorithm 1:
// R <- R u {P}; the list in (t, y, x) order).
//
// A star pass has already written, per segment (template t, image row y,
// 64-column chunk c), the mask bytes, the number of candidates (at most 64)
// and the candidates themselves ({x, scale bits}, in column order) into the
// segment's 64 staging slots.  Segments in (t, y, c) order are in canonical
// (t, y, x) order.  Groups of 64 consecutive segments ("blocks" of the list)
// are then placed:
//   sum    one thread per group: the candidates of its 64 segments (64 count
//          bytes)
//   scan   exclusive scan of the group sums (and the total): one block, or
//          for many groups blocks over spans, their totals, and the span
//          offsets added back
//   list   one wave per group: lane i holds segment i's count, a wave scan
//          gives each segment's offset in the group, and the lanes then walk
//          the group's candidates k = lane, lane + 64, ...: a binary search
//          over the 64 segment offsets finds candidate k's segment and its
//          slot there
// The list pass moves bytes in proportion to the candidates; the count
// bytes are read twice (one byte per 64 positions and template).
#include "oss_internal.h"

#include <algorithm>

namespace oss {

constexpr int GROUP = 64;  // segments per group of the list

int64_t emit_segments(int64_t n_tmpl, int H, int W)
{
    return n_tmpl * (int64_t)H * ((W + SEG_W - 1) / SEG_W);
}

constexpr int SCAN_THREADS = 1024;
constexpr int SCAN_PER = 8;  // consecutive segment counts per thread and round
constexpr int64_t SCAN_CHUNK = (int64_t)SCAN_THREADS * SCAN_PER;
// Segments scanned by one block; more segments are scanned by blocks of
// SCAN_SPAN each, then their totals, then the offsets are added.
constexpr int64_t SCAN_SPAN = 4 * SCAN_CHUNK;

static size_t al256(size_t v) { return (v + 255) / 256 * 256; }

static int64_t n_groups(int64_t nseg) { return (nseg + GROUP - 1) / GROUP; }

static size_t scan_bytes(int64_t nseg)
{
    const int64_t ng = n_groups(nseg);
    const int64_t nblk = (ng + SCAN_SPAN - 1) / SCAN_SPAN;
    // group sums, group offsets, span totals and span offsets
    return 2 * al256((size_t)ng * sizeof(int64_t)) + al256((size_t)(2 * nblk + 2) * sizeof(int64_t));
}

size_t emit_workspace_bytes(int64_t n_tmpl, int H, int W)
{
    const int64_t nseg = emit_segments(n_tmpl, H, W);
    return al256((size_t)nseg) + al256((size_t)nseg * SEG_W * sizeof(uint2)) + scan_bytes(nseg);
}

void emit_carve(void *ws, int64_t n_tmpl, int H, int W, uint8_t **seg_count, uint2 **stage,
                void **scan_ws)
{
    const int64_t nseg = emit_segments(n_tmpl, H, W);
    char *p = static_cast<char *>(ws);
    *seg_count = reinterpret_cast<uint8_t *>(p);
    p += al256((size_t)nseg);
    *stage = reinterpret_cast<uint2 *>(p);
    p += al256((size_t)nseg * SEG_W * sizeof(uint2));
    *scan_ws = p;
}

// Candidates per group of 64 segments (the segments past nseg count 0).
__global__ __launch_bounds__(256) void compact_sum_kernel(const uint8_t *__restrict__ seg_count,
                                                          int64_t nseg, int64_t ng,
                                                          int64_t *__restrict__ sums)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= ng)
        return;
    const int64_t s0 = g * GROUP;
    int64_t tot = 0;
    if (s0 + GROUP <= nseg && ((uintptr_t)(seg_count + s0) & 15) == 0) {
        const uint4 *p = reinterpret_cast<const uint4 *>(seg_count + s0);
#pragma unroll
        for (int i = 0; i < GROUP / 16; ++i) {
            const uint4 v = p[i];
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; ++j)
                tot += (w[j] & 0xff) + ((w[j] >> 8) & 0xff) + ((w[j] >> 16) & 0xff) + (w[j] >> 24);
        }
    } else {
        for (int64_t s = s0; s < min(nseg, s0 + GROUP); ++s)
            tot += seg_count[s];
    }
    sums[g] = tot;
}

// Exclusive scan of counts[0, n) into offs, in rounds of SCAN_CHUNK; the sum
// goes to totals[blockIdx.x].  One block; blockIdx.x selects the chunk
// [b * span, (b + 1) * span) of a longer array when several blocks scan
// chunks apart.
template <typename C>
__global__ __launch_bounds__(SCAN_THREADS) void compact_scan_kernel(
    const C *__restrict__ counts, int64_t n, int64_t span, int64_t *__restrict__ offs,
    int64_t *__restrict__ totals)
{
    __shared__ int64_t s_w[SCAN_THREADS / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t first = (int64_t)blockIdx.x * span;
    const int64_t last = min(n, first + span);
    int64_t carry = 0;
    for (int64_t base = first; base < last; base += SCAN_CHUNK) {
        const int64_t i0 = base + (int64_t)threadIdx.x * SCAN_PER;
        int64_t v[SCAN_PER], tsum = 0;
#pragma unroll
        for (int u = 0; u < SCAN_PER; ++u) {
            v[u] = i0 + u < last ? (int64_t)counts[i0 + u] : 0;
            tsum += v[u];
        }
        int64_t s = tsum;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t t = __shfl_up(s, d, 64);
            if (lane >= d)
                s += t;
        }
        if (lane == 63)
            s_w[wid] = s;
        __syncthreads();
        int64_t off = 0, chunk = 0;
        for (int w = 0; w < SCAN_THREADS / 64; ++w) {
            off += (w < wid) ? s_w[w] : 0;
            chunk += s_w[w];
        }
        off += carry + s - tsum;  // exclusive prefix of this thread's first count
#pragma unroll
        for (int u = 0; u < SCAN_PER; ++u) {
            if (i0 + u < last)
                offs[i0 + u] = off;
            off += v[u];
        }
        carry += chunk;
        __syncthreads();
    }
    if (threadIdx.x == 0)
        totals[blockIdx.x] = carry;
}

// offs[i] += add[i / span]: the chunk offsets of a multi-block scan.
__global__ __launch_bounds__(256) void compact_add_kernel(int64_t *__restrict__ offs, int64_t n,
                                                          int64_t span,
                                                          const int64_t *__restrict__ add)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        offs[i] += add[i / span];
}

constexpr int LTHREADS = 256;
constexpr int LWAVES = LTHREADS / 64;

// One wave per group of 64 segments (grid-stride).  Candidate k of the group
// (k < the group's total) lies in the segment j with off[j] <= k < off[j+1]
// (off: the wave's exclusive scan of the counts); it is staged at slot
// k - off[j] of segment j.  Records at or past `cap` are dropped (the count
// still holds the total).
__global__ __launch_bounds__(LTHREADS) void compact_list_kernel(
    const uint8_t *__restrict__ seg_count, const int64_t *__restrict__ grp_off,
    const uint2 *__restrict__ stage, int64_t nseg, int64_t segs_per_t, int n_chunks,
    oss_candidate *__restrict__ list, int64_t cap)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * LWAVES + (threadIdx.x >> 6);
    const int64_t n_waves = (int64_t)gridDim.x * LWAVES;
    const int64_t ng = (nseg + GROUP - 1) / GROUP;
    for (int64_t g = wave; g < ng; g += n_waves) {
        const int64_t base = grp_off[g];
        if (base >= cap)
            continue;
        const int64_t s = g * GROUP + lane;
        const int c = s < nseg ? seg_count[s] : 0;
        int incl = c;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(incl, d, 64);
            if (lane >= d)
                incl += t;
        }
        const int off = incl - c;
        const int total = __shfl(incl, 63, 64);
        // every lane takes part in every round: the shuffles read other
        // lanes' offsets, and a lane that has left the loop reads as 0
        for (int k0 = 0; k0 < total && base + k0 < cap; k0 += 64) {
            const int k = k0 + lane;
            // largest j with off[j] <= k (off is non-decreasing, off[0] = 0)
            int j = 0;
#pragma unroll
            for (int step = 32; step > 0; step >>= 1) {
                const int o = __shfl(off, j + step, 64);
                if (o <= k)
                    j += step;
            }
            const int oj = __shfl(off, j, 64);
            const int64_t pos = base + k;
            if (k < total && pos < cap) {
                const int64_t seg = g * GROUP + j;
                const uint2 rec = stage[seg * SEG_W + (k - oj)];
                const int32_t t = (int32_t)(seg / segs_per_t);
                const int64_t rem = seg - (int64_t)t * segs_per_t;
                oss_candidate cd;
                cd.t = t;
                cd.y = (int32_t)(rem / n_chunks);
                cd.x = (int32_t)rec.x;
                cd.scale_bits = rec.y;
                list[pos] = cd;
            }
        }
    }
}

hipError_t launch_list(const uint8_t *seg_count, const uint2 *stage, int64_t n_tmpl, int H,
                       int W, oss_candidate *list, int64_t list_cap, int64_t *count,
                       void *scan_ws, hipStream_t stream, Profiler *prof)
{
    const int n_chunks = (W + SEG_W - 1) / SEG_W;
    const int64_t nseg = emit_segments(n_tmpl, H, W);
    const int64_t ng = n_groups(nseg);
    const int64_t nblk = (ng + SCAN_SPAN - 1) / SCAN_SPAN;
    char *p = static_cast<char *>(scan_ws);
    int64_t *sums = reinterpret_cast<int64_t *>(p);
    int64_t *grp_off = reinterpret_cast<int64_t *>(p + al256((size_t)ng * sizeof(int64_t)));
    int64_t *blk_sum = reinterpret_cast<int64_t *>(p + 2 * al256((size_t)ng * sizeof(int64_t)));
    int64_t *blk_off = blk_sum + nblk + 1;
    {
        ProfScope ps(prof, K_COMPACT_SCAN, stream);
        hipLaunchKernelGGL(compact_sum_kernel, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0,
                           stream, seg_count, nseg, ng, sums);
        if (nblk <= 1) {
            hipLaunchKernelGGL(compact_scan_kernel<int64_t>, dim3(1), dim3(SCAN_THREADS), 0,
                               stream, sums, ng, ng, grp_off, count);
        } else {
            // spans of SCAN_SPAN groups scanned in parallel, their totals
            // scanned by one block (the grand total into *count), the span
            // offsets added back
            hipLaunchKernelGGL(compact_scan_kernel<int64_t>, dim3((unsigned)nblk),
                               dim3(SCAN_THREADS), 0, stream, sums, ng, SCAN_SPAN, grp_off,
                               blk_sum);
            hipLaunchKernelGGL(compact_scan_kernel<int64_t>, dim3(1), dim3(SCAN_THREADS), 0,
                               stream, blk_sum, nblk, nblk, blk_off, count);
            hipLaunchKernelGGL(compact_add_kernel, dim3((unsigned)((ng + 255) / 256)), dim3(256),
                               0, stream, grp_off, ng, SCAN_SPAN, blk_off);
        }
    }
    if (list && list_cap > 0) {
        ProfScope ps(prof, K_COMPACT_LIST, stream);
        const int64_t blocks = std::min<int64_t>((ng + LWAVES - 1) / LWAVES, 32768);
        hipLaunchKernelGGL(compact_list_kernel, dim3((unsigned)blocks), dim3(LTHREADS), 0, stream,
                           seg_count, grp_off, stage, nseg, (int64_t)H * n_chunks, n_chunks, list,
                           list_cap);
    }
    return hipGetLastError();
}

}  // namespace oss
