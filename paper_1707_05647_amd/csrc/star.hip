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
// scales' bits.
//
// Schedule (cache reuse): a table entry serves the positions 2s+1 and 2r+1
// rows apart, so a row-major sweep re-reads each table row from beyond L2
// once per use unless the rows in between stay cached.  The image is cut
// into column strips one block wide; strip units are dealt round-robin to
// the 8 XCDs (a hardware block id b runs on XCD b mod 8), and the blocks_per_xcd
// persistent blocks of an XCD walk its strips row by row in lockstep.  An
// XCD then has about blocks_per_xcd rows of one strip in flight, and its L2
// holds the strip's table rows from 2 r_max rows above to the rows in
// flight: (rows in flight + 2 r_max + 2) x (strip + 2 r_max) entries.
#include "star_common.h"

namespace oss {

// STAGED (planar layouts with more than one quantity): per radius a wave
// first looks up quantity Tab::C alone (one load of 64 consecutive values
// per lookup) and compares it with the radius' probes; only if some
// position of the wave passes does it look up the other quantities, and
// only for the positions that passed.  A position fails a probe when any
// feature fails, so the result is the same; the saving is the table reads of
// the quantities that are never needed (most positions fail the first
// feature: the screen's premise).  Interleaved entries are never staged: a
// lone quantity is then a strided read that costs about as much as the
// whole entry.
template <typename Tab, bool STAGED>
__global__ __launch_bounds__(STAR_MAX_THREADS) void star_plain_kernel(
    const void *__restrict__ L, const void *__restrict__ R, const void *__restrict__ Rp,
    int64_t pitch_e, int64_t plane, int H, int W, const DevTemplatePlan *__restrict__ plan,
    EmitOut eo, StarSweep sw)
{
    constexpr int NQ = Tab::NQ;
    constexpr int64_t ES = Tab::ES;  // bytes per table entry
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int units = (sw.n_units - xcd + 7) / 8;  // units u = xcd + 8 t of this XCD
    const int items = units * sw.rows_per_part;
    // byte offset of column x0 + tid + 1 relative to column x0
    const uint32_t lane_off = (uint32_t)((threadIdx.x + 1) * ES);
    const int64_t row_bytes = pitch_e * ES;
    const TabBases tb{static_cast<const char *>(L), static_cast<const char *>(R),
                      static_cast<const char *>(Rp)};
    // the plan (radii, probe bounds) in LDS once per block: per radius it is
    // read there instead of through the scalar cache
    __shared__ DevTemplatePlan s_plan;
    {
        const int32_t *src = reinterpret_cast<const int32_t *>(plan);
        int32_t *dst = reinterpret_cast<int32_t *>(&s_plan);
        for (int i = threadIdx.x; i < (int)(sizeof(DevTemplatePlan) / 4); i += blockDim.x)
            dst[i] = src[i];
        __syncthreads();
        plan = &s_plan;
    }
    const int nr = plan->n_radii;
    for (int it = j; it < items; it += sw.blocks_per_xcd) {
        int y, x0;
        sweep_item(sw, xcd, it, (int)blockDim.x, &y, &x0);
        if (y >= H)
            continue;
        const int x = x0 + threadIdx.x;
        const char *Lb = reinterpret_cast<const char *>(L) + (int64_t)x0 * ES;
        const char *Rb = reinterpret_cast<const char *>(R) + (int64_t)x0 * ES;
        const char *Rpb = reinterpret_cast<const char *>(Rp) + (int64_t)x0 * ES;
        uint32_t acc = 0;
        for (int jr = 0; jr < nr; ++jr) {
            const DevRadius rd = plan->radii[jr];
            const int r = rd.r, s = rd.s;
            if (y < r || y > H - 1 - r)
                continue;
            const bool xv = x >= r && x <= W - 1 - r;
            if constexpr (STAGED && Tab::STAGE && NQ > 1) {
                constexpr int C = Tab::C;
                const StarAddr ad = star_addr<Tab>(Lb, Rb, Rpb, row_bytes, lane_off, y, r, s);
                int64_t F[NQ];
                bool maybe = false;
                if (xv) {
                    F[C] = star_sum_c<Tab>(ad, plane);
                    for (int p = rd.first; p < rd.first + rd.count; ++p) {
                        const DevProbe pr = plan->probes[p];
                        maybe = maybe | ((F[C] >= pr.lo[C]) & (F[C] <= pr.hi[C]));
                    }
                }
                if (__builtin_amdgcn_ballot_w64(maybe) == 0)
                    continue;
                if (maybe) {
                    star_sums_rest<Tab>(ad, tb, plane, F);
                    for (int p = rd.first; p < rd.first + rd.count; ++p) {
                        const DevProbe pr = plan->probes[p];
                        bool pass = true;
#pragma unroll
                        for (int q = 0; q < NQ; ++q)
                            pass = pass & (F[q] >= pr.lo[q]) & (F[q] <= pr.hi[q]);
                        acc |= pass ? (1u << pr.k) : 0u;
                    }
                }
            } else if (xv) {
                int64_t F[NQ];
                star_sums<Tab>(Lb, Rb, Rpb, row_bytes, lane_off, y, r, s, tb, F, plane);
                for (int p = rd.first; p < rd.first + rd.count; ++p) {
                    const DevProbe pr = plan->probes[p];
                    bool pass = true;
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        pass = pass & (F[q] >= pr.lo[q]) & (F[q] <= pr.hi[q]);
                    acc |= pass ? (1u << pr.k) : 0u;
                }
            }
        }
        emit_row<1>(eo, 1, y, x, [&](int) { return acc; }, [](int) { return 0; },
                    [&](int) { return eo.mask; });
    }
}

// Software-pipelined form of the same screen: the 8 lookups of the next
// radius are issued before the current radius is reduced and compared, so
// every wave keeps two radii of loads in flight.  Lookups use the column
// clamped into the radius' valid range (every lane loads, no lane masking;
// lanes outside the range discard the result), and only radii whose star
// fits the row and the image width are walked: with the radii ascending
// they are a prefix of the template's list.
template <typename Tab>
struct Looks {
    typename Tab::E a, b, c, d, e, f, h, k;
};

template <typename Tab>
__device__ __forceinline__ void star_load(Looks<Tab> &o, const char *L, const char *R,
                                          const char *Rp, int64_t row_bytes, int xc, int y,
                                          int r, int s, int64_t plane)
{
    constexpr uint32_t ES = (uint32_t)Tab::ES;
    const char *l_top = L + (int64_t)(y - s) * row_bytes;      // row y-s-1
    const char *l_bot = L + (int64_t)(y + s + 1) * row_bytes;  // row y+s
    const char *r_top = R + (int64_t)(y - r) * row_bytes;      // row y-r-1
    const char *r_bot = R + (int64_t)(y + r + 1) * row_bytes;  // row y+r
    const char *rp_mid = Rp + (int64_t)y * row_bytes;           // row y-1
    // byte offsets of table columns (image column + 1) from the row start
    const uint32_t c0 = (uint32_t)(xc + 1) * ES;                 // x
    const uint32_t cs = (uint32_t)(xc + s + 1) * ES;             // x+s
    const uint32_t cs1 = (uint32_t)(xc - s) * ES;                // x-s-1
    const uint32_t cr = (uint32_t)(xc + r + 1) * ES;             // x+r
    const uint32_t cr1 = (uint32_t)(xc - r) * ES;                // x-r-1
    o.a = tab_load<Tab>(l_bot + cs, L, plane);     // L(x+s,   y+s)
    o.b = tab_load<Tab>(l_bot + cs1, L, plane);    // L(x-s-1, y+s)
    o.c = tab_load<Tab>(l_top + cs, L, plane);     // L(x+s,   y-s-1)
    o.d = tab_load<Tab>(l_top + cs1, L, plane);    // L(x-s-1, y-s-1)
    o.e = tab_load<Tab>(r_bot + c0, R, plane);     // R(x, y+r)
    o.f = tab_load<Tab>(rp_mid + cr1, Rp, plane);  // R'(x-r-1, y-1)
    o.h = tab_load<Tab>(rp_mid + cr, Rp, plane);   // R'(x+r, y-1)
    o.k = tab_load<Tab>(r_top + c0, R, plane);     // R(x, y-r-1)
}

template <typename Tab>
__global__ __launch_bounds__(STAR_MAX_THREADS) void star_pipe_kernel(
    const void *__restrict__ L, const void *__restrict__ R, const void *__restrict__ Rp,
    int64_t pitch_e, int64_t plane, int H, int W, const DevTemplatePlan *__restrict__ plan,
    EmitOut eo, StarSweep sw)
{
    constexpr int NQ = Tab::NQ;
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int units = (sw.n_units - xcd + 7) / 8;
    const int items = units * sw.rows_per_part;
    const int64_t row_bytes = pitch_e * Tab::ES;
    const char *Lt = static_cast<const char *>(L);
    const char *Rt = static_cast<const char *>(R);
    const char *Rpt = static_cast<const char *>(Rp);
    const int nr = plan->n_radii;
    for (int it = j; it < items; it += sw.blocks_per_xcd) {
        int y, x0;
        sweep_item(sw, xcd, it, (int)blockDim.x, &y, &x0);
        if (y >= H)
            continue;
        const int x = x0 + threadIdx.x;
        int nv = 0;
        while (nv < nr) {
            const int r = plan->radii[nv].r;
            if (y < r || y > H - 1 - r || 2 * r + 1 > W)
                break;
            ++nv;
        }
        uint32_t acc = 0;
        if (nv > 0) {
            DevRadius rd = plan->radii[0];
            Looks<Tab> cur;
            star_load<Tab>(cur, Lt, Rt, Rpt, row_bytes, min(max(x, rd.r), W - 1 - rd.r), y, rd.r,
                           rd.s, plane);
            for (int jr = 0; jr < nv; ++jr) {
                const bool more = jr + 1 < nv;
                Looks<Tab> nxt;
                DevRadius rn = rd;
                if (more) {
                    rn = plan->radii[jr + 1];
                    star_load<Tab>(nxt, Lt, Rt, Rpt, row_bytes, min(max(x, rn.r), W - 1 - rn.r), y,
                                   rn.r, rn.s, plane);
                }
                int64_t F[NQ];
                Tab::reduce(cur.a, cur.b, cur.c, cur.d, cur.e, cur.f, cur.h, cur.k, F);
                const bool xv = x >= rd.r && x <= W - 1 - rd.r;
                for (int p = rd.first; p < rd.first + rd.count; ++p) {
                    const DevProbe pr = plan->probes[p];
                    bool pass = xv;
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        pass = pass & (F[q] >= pr.lo[q]) & (F[q] <= pr.hi[q]);
                    acc |= pass ? (1u << pr.k) : 0u;
                }
                if (more) {
                    cur = nxt;
                    rd = rn;
                }
            }
        }
        emit_row<1>(eo, 1, y, x, [&](int) { return acc; }, [](int) { return 0; },
                    [&](int) { return eo.mask; });
    }
}

// Same screen with the rows that several lookups share staged in LDS: per
// block row (strip columns [x0, x0 + strip) of image row y) the R' row y-1
// is loaded once for all radii over [x0 - r_max - 1, x0 + strip - 1 + r_max],
// and for each radius the two L rows y+s and y-s-1 are loaded once over
// [x0 - s - 1, x0 + strip - 1 + s], serving both of their lookups.  The two R
// lookups have no neighbour to share with and stay direct loads.  LDS is
// quantity-major (one column of T per quantity) so lanes hit consecutive
// banks.
template <typename T, int NQ>
__device__ __forceinline__ void stage_row(T *__restrict__ dst, int cap, const char *row_base,
                                          int col0, int n, int pitch_e)
{
    // dst[q * cap + i] = entry (column col0 + i) of the table row at row_base
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int c = col0 + i + 1;  // table column
        if (c >= 0 && c < pitch_e) {
            const Entry<T, NQ> v =
                *reinterpret_cast<const Entry<T, NQ> *>(row_base + (int64_t)c * sizeof(T) * NQ);
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                dst[q * cap + i] = v.v[q];
        }
    }
}

template <typename T, int NQ>
__global__ __launch_bounds__(STAR_MAX_THREADS) void star_lds_kernel(
    const T *__restrict__ L, const T *__restrict__ R, const T *__restrict__ Rp, int64_t pitch_e,
    int H, int W, const DevTemplatePlan *__restrict__ plan, EmitOut eo, StarSweep sw, int smax,
    int rmax)
{
    extern __shared__ char smem_raw[];
    constexpr int64_t ES = (int64_t)sizeof(T) * NQ;
    const int strip = blockDim.x;
    const int capL = strip + 2 * smax + 1, capR = strip + 2 * rmax + 1;
    T *lt = reinterpret_cast<T *>(smem_raw);  // L row y-s-1   [NQ][capL]
    T *lb = lt + NQ * capL;                    // L row y+s     [NQ][capL]
    T *rw = lb + NQ * capL;                    // R' row y-1    [NQ][capR]
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int units = (sw.n_units - xcd + 7) / 8;
    const int items = units * sw.rows_per_part;
    const uint32_t lane_off = (uint32_t)((threadIdx.x + 1) * ES);
    const int64_t row_bytes = pitch_e * ES;
    const int tid = threadIdx.x;
    const int nr = plan->n_radii;
    for (int it = j; it < items; it += sw.blocks_per_xcd) {
        int y, x0;
        sweep_item(sw, xcd, it, strip, &y, &x0);
        if (y >= H)
            continue;
        const int x = x0 + tid;
        const char *Lb = reinterpret_cast<const char *>(L);
        const char *Rb = reinterpret_cast<const char *>(R) + (int64_t)x0 * ES;
        const char *Rpb = reinterpret_cast<const char *>(Rp);
        __syncthreads();  // the previous row's readers are done with LDS
        stage_row<T, NQ>(rw, capR, Rpb + (int64_t)y * row_bytes, x0 - rmax - 1,
                         strip + 2 * rmax + 1, (int)pitch_e);
        uint32_t acc = 0;
        for (int jr = 0; jr < nr; ++jr) {
            const DevRadius rd = plan->radii[jr];
            const int r = rd.r, s = rd.s;
            if (y < r || y > H - 1 - r)
                continue;
            const bool valid = x >= r && x <= W - 1 - r;
            Entry<T, NQ> e, k;
            if (valid) {
                e = entry_at<Entry<T, NQ>>(Rb + (int64_t)(y + r + 1) * row_bytes,
                                           lane_off);  // R(x, y+r)
                k = entry_at<Entry<T, NQ>>(Rb + (int64_t)(y - r) * row_bytes,
                                           lane_off);  // R(x, y-r-1)
            }
            __syncthreads();  // the previous radius' L readers are done
            const int n = strip + 2 * s + 1;
            stage_row<T, NQ>(lt, capL, Lb + (int64_t)(y - s) * row_bytes, x0 - s - 1, n,
                             (int)pitch_e);
            stage_row<T, NQ>(lb, capL, Lb + (int64_t)(y + s + 1) * row_bytes, x0 - s - 1, n,
                             (int)pitch_e);
            __syncthreads();
            if (valid) {
                int64_t F[NQ];
                const int ia = tid + 2 * s + 1, ib = tid;          // x+s, x-s-1 in the L window
                const int jf = tid + rmax - r, jh = tid + rmax + r + 1;  // x-r-1, x+r in the R' window
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const T sq = lb[q * capL + ia] - lb[q * capL + ib] - lt[q * capL + ia] +
                                 lt[q * capL + ib];
                    const T dm = e.v[q] - rw[q * capR + jf] - rw[q * capR + jh] + k.v[q];
                    F[q] = widen(sq) + widen(dm);
                }
                for (int p = rd.first; p < rd.first + rd.count; ++p) {
                    const DevProbe pr = plan->probes[p];
                    bool pass = true;
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        pass = pass & (F[q] >= pr.lo[q]) & (F[q] <= pr.hi[q]);
                    acc |= pass ? (1u << pr.k) : 0u;
                }
            }
        }
        emit_row<1>(eo, 1, y, x, [&](int) { return acc; }, [](int) { return 0; },
                    [&](int) { return eo.mask; });
    }
}

size_t star_lds_bytes(int strip, int nq, int ebytes, int smax, int rmax)
{
    return (size_t)nq * ebytes * (2 * (size_t)(strip + 2 * smax + 1) + (strip + 2 * rmax + 1));
}

StarSweep make_sweep(int H, int W, int strip, int blocks_per_xcd)
{
    StarSweep sw;
    sw.strip = strip;
    sw.n_strips = (W + strip - 1) / strip;
    sw.parts = sw.n_strips >= 8 ? 1 : (8 + sw.n_strips - 1) / sw.n_strips;
    sw.rows_per_part = (H + sw.parts - 1) / sw.parts;
    sw.n_units = sw.n_strips * sw.parts;
    sw.blocks_per_xcd = blocks_per_xcd;
    return sw;
}

template <typename T, int NQ>
static void star_lds_launch(const BuildGeom &g, const T *l, const T *r, const T *rp,
                            const DevTemplatePlan *plan, const EmitOut &eo, const StarSweep &sw,
                            int smax, int rmax, hipStream_t stream)
{
    const size_t lds = star_lds_bytes(sw.strip, NQ, sizeof(T), smax, rmax);
    auto *k = &star_lds_kernel<T, NQ>;
    const StarSweep rs = resident_sweep(reinterpret_cast<const void *>(k), sw, lds);
    hipLaunchKernelGGL(k, dim3(8 * rs.blocks_per_xcd), dim3(rs.strip), lds, stream, l, r, rp,
                       g.pitch_e, g.H, g.W, plan, eo, rs, smax, rmax);
}

template <typename Tab>
static void star_plain_launch(const BuildGeom &g, const void *L, const void *R, const void *Rp,
                              const DevTemplatePlan *plan, const EmitOut &eo, const StarSweep &sw,
                              hipStream_t stream, int variant)
{
    auto go = [&](auto *k) {
        const StarSweep rs = resident_sweep(reinterpret_cast<const void *>(k), sw, 0);
        hipLaunchKernelGGL(k, dim3(8 * rs.blocks_per_xcd), dim3(rs.strip), 0, stream, L, R, Rp,
                           g.pitch_e, g.plane, g.H, g.W, plan, eo, rs);
    };
    if (variant == 2) {
        go(&star_pipe_kernel<Tab>);
        return;
    }
    if constexpr (Tab::STAGE && Tab::NQ > 1) {
        if (variant == 3) {
            go(&star_plain_kernel<Tab, true>);
            return;
        }
    }
    go(&star_plain_kernel<Tab, false>);
}

template <typename T>
static hipError_t star_t(const BuildGeom &g, const void *L, const void *R, const void *Rp,
                         const DevTemplatePlan *plan, const EmitOut &eo, const StarSweep &sw,
                         int smax, int rmax, bool lds, int variant, hipStream_t stream)
{
    const T *l = static_cast<const T *>(L), *r = static_cast<const T *>(R),
            *rp = static_cast<const T *>(Rp);
    if (g.planar) {
        switch (g.nq) {
        case 1: star_plain_launch<TabP<T, 1>>(g, L, R, Rp, plan, eo, sw, stream, variant); break;
        case 2: star_plain_launch<TabP<T, 2>>(g, L, R, Rp, plan, eo, sw, stream, variant); break;
        case 3: star_plain_launch<TabP<T, 3>>(g, L, R, Rp, plan, eo, sw, stream, variant); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (lds) {
        switch (g.nq) {
        case 1: star_lds_launch<T, 1>(g, l, r, rp, plan, eo, sw, smax, rmax, stream); break;
        case 2: star_lds_launch<T, 2>(g, l, r, rp, plan, eo, sw, smax, rmax, stream); break;
        case 3: star_lds_launch<T, 3>(g, l, r, rp, plan, eo, sw, smax, rmax, stream); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (g.nq) {
    case 1: star_plain_launch<TabU<T, 1>>(g, L, R, Rp, plan, eo, sw, stream, variant); break;
    case 2: star_plain_launch<TabU<T, 2>>(g, L, R, Rp, plan, eo, sw, stream, variant); break;
    case 3: star_plain_launch<TabU<T, 3>>(g, L, R, Rp, plan, eo, sw, stream, variant); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// 64-bit squares (mixed 16-byte entries or split planes): no LDS variant.
static hipError_t star_mix(const BuildGeom &g, const void *L, const void *R, const void *Rp,
                           const DevTemplatePlan *plan, const EmitOut &eo, const StarSweep &sw,
                           hipStream_t stream, int variant)
{
    if (g.planar) {
        if (g.rec)
            star_plain_launch<TabPR>(g, L, R, Rp, plan, eo, sw, stream, variant);
        else if (g.nq == 3 && g.sqi == 1)
            star_plain_launch<TabPS<3, 1>>(g, L, R, Rp, plan, eo, sw, stream, variant);
        else if (g.nq == 2 && g.sqi == 1)
            star_plain_launch<TabPS<2, 1>>(g, L, R, Rp, plan, eo, sw, stream, variant);
        else if (g.nq == 2 && g.sqi == 0)
            star_plain_launch<TabPS<2, 0>>(g, L, R, Rp, plan, eo, sw, stream, variant);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    if (g.nq == 3 && g.sqi == 1)
        star_plain_launch<TabMix<3, 1>>(g, L, R, Rp, plan, eo, sw, stream, variant);
    else if (g.nq == 2 && g.sqi == 1)
        star_plain_launch<TabMix<2, 1>>(g, L, R, Rp, plan, eo, sw, stream, variant);
    else if (g.nq == 2 && g.sqi == 0)
        star_plain_launch<TabMix<2, 0>>(g, L, R, Rp, plan, eo, sw, stream, variant);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_star_plain(const BuildGeom &g, const void *L, const void *R, const void *Rp,
                             const DevTemplatePlan *plan, const EmitOut &eo, const StarSweep &sw,
                             int smax, int rmax, int variant, hipStream_t stream,
                             Profiler *prof)
{
    bool lds = variant == 1;
    if (sw.strip < 64 || sw.strip > STAR_MAX_THREADS || sw.strip % 64 || sw.blocks_per_xcd < 1)
        return hipErrorInvalidValue;
    if (!emit_ok(eo, g))
        return hipErrorInvalidValue;
    if (lds && star_lds_bytes(sw.strip, g.nq, g.ebytes, smax, rmax) > STAR_LDS_MAX)
        lds = false;
    ProfScope ps(prof, K_STAR, stream);
    if (g.sqi >= 0)
        return star_mix(g, L, R, Rp, plan, eo, sw, stream, variant);
    if (g.ebytes == 4)
        return star_t<uint32_t>(g, L, R, Rp, plan, eo, sw, smax, rmax, lds, variant, stream);
    return star_t<uint64_t>(g, L, R, Rp, plan, eo, sw, smax, rmax, lds, variant, stream);
}

}  // namespace oss
