// Candidate compaction: scale-bit words in (t, y, x) order -> uint8 mask and
// a candidate list in the same order (Algorithm 1: R <- R u {P}).
//
// Deterministic two-pass stream compaction over segments of CSEG words:
//   count  one block per segment; each wave ballots 64 words at a time and
//          popcounts the ballot
//   scan   exclusive scan of the segment counts (and the total): one block,
//          or for many segments blocks over chunks, their totals, and the
//          chunk offsets added back
//   write  one block per segment; the wave offsets come from a block scan of
//          per-wave counts, a lane's slot from the popcount of the ballot
//          bits below it (mbcnt); the mask is written for every word
#include "oss_internal.h"

namespace oss {

constexpr int CTHREADS = 256;
constexpr int CWAVES = CTHREADS / 64;
constexpr int CITER = 16;                         // ballots per wave
constexpr int64_t CSEG = (int64_t)CTHREADS * CITER;  // 4096 words per block

__device__ __forceinline__ int lane_prefix(uint64_t ballot)
{
    // number of set ballot bits below this lane
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(ballot >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)ballot, 0u));
}

__global__ __launch_bounds__(CTHREADS) void compact_count_kernel(const uint32_t *__restrict__ bits,
                                                                 int64_t n,
                                                                 int64_t *__restrict__ seg_count)
{
    __shared__ int s_cnt[CWAVES];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * CSEG + (int64_t)wid * 64 * CITER;
    int cnt = 0;
#pragma unroll 4
    for (int it = 0; it < CITER; ++it) {
        const int64_t i = base + it * 64 + lane;
        const bool on = i < n && bits[i] != 0u;
        cnt += __popcll(__ballot(on));
    }
    if (lane == 0)
        s_cnt[wid] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < CWAVES; ++w)
            t += s_cnt[w];
        seg_count[blockIdx.x] = t;
    }
}

constexpr int SCAN_THREADS = 1024;
constexpr int SCAN_PER = 8;  // consecutive segment counts per thread and round
constexpr int64_t SCAN_CHUNK = (int64_t)SCAN_THREADS * SCAN_PER;

// Exclusive scan of counts[0, n) into offs, in rounds of SCAN_CHUNK; the sum
// goes to *total.  One block; blockIdx.x selects the chunk [b * span,
// (b + 1) * span) of a longer array when several blocks scan chunks apart.
__global__ __launch_bounds__(SCAN_THREADS) void compact_scan_kernel(
    const int64_t *__restrict__ counts, int64_t n, int64_t span, int64_t *__restrict__ offs,
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
            v[u] = i0 + u < last ? counts[i0 + u] : 0;
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

__global__ __launch_bounds__(CTHREADS) void compact_write_kernel(
    const uint32_t *__restrict__ bits, int64_t n, int64_t hw, int W,
    const int64_t *__restrict__ seg_off, uint8_t *__restrict__ mask,
    oss_candidate *__restrict__ list, int64_t cap)
{
    __shared__ int s_cnt[CWAVES];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * CSEG + (int64_t)wid * 64 * CITER;
    uint32_t v[CITER];
    int cnt = 0;
#pragma unroll
    for (int it = 0; it < CITER; ++it) {
        const int64_t i = base + it * 64 + lane;
        v[it] = i < n ? bits[i] : 0u;
        cnt += __popcll(__ballot(v[it] != 0u));
    }
    if (lane == 0)
        s_cnt[wid] = cnt;
    __syncthreads();
    int64_t off = seg_off[blockIdx.x];
    for (int w = 0; w < wid; ++w)
        off += s_cnt[w];
#pragma unroll
    for (int it = 0; it < CITER; ++it) {
        const int64_t i = base + it * 64 + lane;
        const bool on = v[it] != 0u;
        const uint64_t bal = __ballot(on);
        if (mask && i < n)
            mask[i] = on ? 1 : 0;
        if (on) {
            const int64_t pos = off + lane_prefix(bal);
            if (pos < cap) {
                const int64_t t = i / hw;
                const int64_t rem = i - t * hw;
                const int64_t y = rem / W;
                oss_candidate c;
                c.t = (int32_t)t;
                c.y = (int32_t)y;
                c.x = (int32_t)(rem - y * W);
                c.scale_bits = v[it];
                list[pos] = c;
            }
        }
        off += __popcll(bal);
    }
}

// Segments scanned by one block; more segments are scanned by blocks of
// SCAN_SPAN each, then their totals, then the offsets are added.
constexpr int64_t SCAN_SPAN = 4 * SCAN_CHUNK;

size_t compact_workspace_bytes(int64_t n)
{
    const int64_t nseg = (n + CSEG - 1) / CSEG;
    const int64_t nblk = (nseg + SCAN_SPAN - 1) / SCAN_SPAN;
    return (size_t)(2 * nseg + 2 * nblk) * sizeof(int64_t);
}

hipError_t launch_compact(const uint32_t *bits, int64_t n_tmpl, int H, int W, uint8_t *mask,
                          oss_candidate *list, int64_t list_cap, int64_t *count, void *workspace,
                          hipStream_t stream, Profiler *prof)
{
    const int64_t hw = (int64_t)H * W;
    const int64_t n = n_tmpl * hw;
    const int64_t nseg = (n + CSEG - 1) / CSEG;
    const int64_t nblk = (nseg + SCAN_SPAN - 1) / SCAN_SPAN;
    int64_t *seg_count = static_cast<int64_t *>(workspace);
    int64_t *seg_off = seg_count + nseg;
    int64_t *blk_sum = seg_off + nseg, *blk_off = blk_sum + nblk;
    {
        ProfScope ps(prof, K_COMPACT_COUNT, stream);
        hipLaunchKernelGGL(compact_count_kernel, dim3((unsigned)nseg), dim3(CTHREADS), 0, stream,
                           bits, n, seg_count);
    }
    {
        ProfScope ps(prof, K_COMPACT_SCAN, stream);
        if (nblk <= 1) {
            hipLaunchKernelGGL(compact_scan_kernel, dim3(1), dim3(SCAN_THREADS), 0, stream,
                               seg_count, nseg, nseg, seg_off, count);
        } else {
            // chunks of SCAN_SPAN segments scanned in parallel, their totals
            // scanned by one block (the grand total into *count), the chunk
            // offsets added back
            hipLaunchKernelGGL(compact_scan_kernel, dim3((unsigned)nblk), dim3(SCAN_THREADS), 0,
                               stream, seg_count, nseg, SCAN_SPAN, seg_off, blk_sum);
            hipLaunchKernelGGL(compact_scan_kernel, dim3(1), dim3(SCAN_THREADS), 0, stream,
                               blk_sum, nblk, nblk, blk_off, count);
            hipLaunchKernelGGL(compact_add_kernel, dim3((unsigned)((nseg + 255) / 256)), dim3(256),
                               0, stream, seg_off, nseg, SCAN_SPAN, blk_off);
        }
    }
    {
        ProfScope ps(prof, K_COMPACT_WRITE, stream);
        hipLaunchKernelGGL(compact_write_kernel, dim3((unsigned)nseg), dim3(CTHREADS), 0, stream,
                           bits, n, hw, W, seg_off, mask, list, list ? list_cap : 0);
    }
    return hipGetLastError();
}

}  // namespace oss
