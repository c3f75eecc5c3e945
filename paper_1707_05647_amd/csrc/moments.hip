// The paper's own patch features over the star (Sec. "Patch Features":
// mean, Eq. S_sigma variance, the horizontal and vertical gradients as inner
// products with the extended Prewitt ramps, Eq. S_x / Eq. T_x; Sec.
// "Rotation Invariance": their magnitude), screened per probe.
//
// The tables hold I, (I^2,) i I and j I.  For each region (square, diamond)
// the first moment about the centre is the region sum of i I less x times
// the region sum of I, formed in the table's width (modulo 2^32 for 32-bit
// tables, where every region moment is below 2^31 in magnitude) and sign
// extended; the star's moment is the sum of the two regions'.  Per probe:
//   mean:      lo1 <= F1 <= hi1
//   variance:  loV <= V = A(r) F2 - F1^2 <= hiV          (int64)
//   magnitude: loM <= M = Sx^2 + Sy^2 <= hiM             (128-bit)
// with the bounds solved on the host from the template's features and the
// tolerance.  Same persistent XCD-aware strip sweep as the plain screen.
// With planar tables the lookups are staged as in the plain screen: the sum
// plane first (the mean test), the other planes only for the positions where
// some probe of the radius passes it.
#include "star_common.h"

namespace oss {

__device__ __forceinline__ int64_t sext(uint32_t v) { return (int64_t)(int32_t)v; }
__device__ __forceinline__ int64_t sext(uint64_t v) { return (int64_t)v; }

template <typename T, unsigned FM, bool PLANAR>
__global__ __launch_bounds__(STAR_MAX_THREADS) void star_moments_kernel(
    const T *__restrict__ L, const T *__restrict__ R, const T *__restrict__ Rp, int64_t pitch_e,
    int64_t plane, int H, int W, const DevMomPlan *__restrict__ plan, EmitOut eo,
    StarSweep sw)
{
    constexpr bool HAS_SQ = (FM & OSS_F_SQ) != 0;
    constexpr int NQ = HAS_SQ ? 4 : 3;
    constexpr int XM = NQ - 2, YM = NQ - 1;
    using E = Entry<T, NQ>;
    constexpr int64_t ES = PLANAR ? (int64_t)sizeof(T) : (int64_t)sizeof(E);
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int units = (sw.n_units - xcd + 7) / 8;
    const int items = units * sw.rows_per_part;
    const uint32_t lane_off = (uint32_t)((threadIdx.x + 1) * ES);
    const int64_t row_bytes = pitch_e * ES;
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
            if (x < r || x > W - 1 - r)
                continue;
            const char *l_top = Lb + (int64_t)(y - s) * row_bytes;
            const char *l_bot = Lb + (int64_t)(y + s + 1) * row_bytes;
            const char *r_top = Rb + (int64_t)(y - r) * row_bytes;
            const char *r_bot = Rb + (int64_t)(y + r + 1) * row_bytes;
            const char *rp_mid = Rpb + (int64_t)y * row_bytes;
            const int64_t ds = (int64_t)s * ES, ds1 = (int64_t)(s + 1) * ES;
            const int64_t dr = (int64_t)r * ES, dr1 = (int64_t)(r + 1) * ES;
            T sq[NQ], dm[NQ];
            if constexpr (PLANAR) {
                // quantity q of a lookup: plane q at the same entry offset
                const char *pa = l_bot + ds + lane_off, *pb = l_bot - ds1 + lane_off;
                const char *pc = l_top + ds + lane_off, *pd = l_top - ds1 + lane_off;
                const char *pe = r_bot + lane_off, *pf = rp_mid - dr1 + lane_off;
                const char *ph = rp_mid + dr + lane_off, *pk = r_top + lane_off;
                auto at = [&](const char *p, int q) {
                    return *reinterpret_cast<const T *>(p + q * plane);
                };
                sq[0] = (T)(at(pa, 0) - at(pb, 0) - at(pc, 0) + at(pd, 0));
                dm[0] = (T)(at(pe, 0) - at(pf, 0) - at(ph, 0) + at(pk, 0));
                const int64_t F1 = (int64_t)sq[0] + (int64_t)dm[0];
                bool maybe = false;
                for (int p = rd.first; p < rd.first + rd.count; ++p) {
                    const DevMomProbe &pr = plan->probes[p];
                    maybe = maybe | !(pr.tests & 1) | ((F1 >= pr.lo1) & (F1 <= pr.hi1));
                }
                if (__builtin_amdgcn_ballot_w64(maybe) == 0 || !maybe)
                    continue;
#pragma unroll
                for (int q = 1; q < NQ; ++q) {
                    sq[q] = (T)(at(pa, q) - at(pb, q) - at(pc, q) + at(pd, q));
                    dm[q] = (T)(at(pe, q) - at(pf, q) - at(ph, q) + at(pk, q));
                }
            } else {
                const E a = entry_at<E>(l_bot + ds, lane_off), b = entry_at<E>(l_bot - ds1, lane_off);
                const E c = entry_at<E>(l_top + ds, lane_off), d = entry_at<E>(l_top - ds1, lane_off);
                const E e = entry_at<E>(r_bot, lane_off), f = entry_at<E>(rp_mid - dr1, lane_off);
                const E h = entry_at<E>(rp_mid + dr, lane_off), k = entry_at<E>(r_top, lane_off);
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    sq[q] = (T)(a.v[q] - b.v[q] - c.v[q] + d.v[q]);
                    dm[q] = (T)(e.v[q] - f.v[q] - h.v[q] + k.v[q]);
                }
            }
            const int64_t F1 = (int64_t)sq[0] + (int64_t)dm[0];
            const int64_t Sx = sext((T)(sq[XM] - (T)x * sq[0])) + sext((T)(dm[XM] - (T)x * dm[0]));
            const int64_t Sy = sext((T)(sq[YM] - (T)y * sq[0])) + sext((T)(dm[YM] - (T)y * dm[0]));
            int64_t V = 0;
            if constexpr (HAS_SQ) {
                const int64_t F2 = (int64_t)sq[1] + (int64_t)dm[1];
                const int64_t A = (int64_t)(2 * s + 1) * (2 * s + 1) + 2LL * r * r + 2LL * r + 1;
                V = A * F2 - F1 * F1;
            }
            const unsigned __int128 M =
                (unsigned __int128)((__int128)Sx * Sx) + (unsigned __int128)((__int128)Sy * Sy);
            for (int p = rd.first; p < rd.first + rd.count; ++p) {
                const DevMomProbe pr = plan->probes[p];
                bool pass = true;
                if (pr.tests & 1)
                    pass = pass & (F1 >= pr.lo1) & (F1 <= pr.hi1);
                if (pr.tests & 2)
                    pass = pass & (V >= pr.loV) & (V <= pr.hiV);
                if (pr.tests & 4) {
                    const unsigned __int128 lo = ((unsigned __int128)pr.loM[1] << 64) | pr.loM[0];
                    const unsigned __int128 hi = ((unsigned __int128)pr.hiM[1] << 64) | pr.hiM[0];
                    pass = pass & (M >= lo) & (M <= hi);
                }
                acc |= pass ? (1u << pr.k) : 0u;
            }
        }
        emit_row<1>(eo, 1, y, x, [&](int) { return acc; }, [](int) { return 0; },
                    [&](int) { return eo.mask; });
    }
}

template <typename T>
static hipError_t moments_t(const BuildGeom &g, uint32_t fm, const void *L, const void *R,
                            const void *Rp, const DevMomPlan *plan, const EmitOut &eo,
                            const StarSweep &sw, hipStream_t st)
{
    const T *l = static_cast<const T *>(L), *r = static_cast<const T *>(R),
            *rp = static_cast<const T *>(Rp);
    constexpr unsigned F3 = OSS_F_SUM | OSS_F_MOMENTS, F4 = OSS_F_SUM | OSS_F_SQ | OSS_F_MOMENTS;
#define OSS_MOM_LAUNCH(FMV, PL)                                                                   \
    do {                                                                                          \
        auto *k = &star_moments_kernel<T, FMV, PL>;                                               \
        const StarSweep rs = resident_sweep(reinterpret_cast<const void *>(k), sw, 0);            \
        hipLaunchKernelGGL(k, dim3(8 * rs.blocks_per_xcd), dim3(rs.strip), 0, st, l, r, rp,       \
                           g.pitch_e, g.plane, g.H, g.W, plan, eo, rs);                           \
    } while (0)
    if (fm == F3 && g.planar)
        OSS_MOM_LAUNCH(F3, true);
    else if (fm == F3)
        OSS_MOM_LAUNCH(F3, false);
    else if (fm == F4 && g.planar)
        OSS_MOM_LAUNCH(F4, true);
    else if (fm == F4)
        OSS_MOM_LAUNCH(F4, false);
    else
        return hipErrorInvalidValue;
#undef OSS_MOM_LAUNCH
    return hipGetLastError();
}

hipError_t launch_star_moments(const BuildGeom &g, uint32_t fm, const void *L, const void *R,
                               const void *Rp, const DevMomPlan *plan, const EmitOut &eo,
                               const StarSweep &sw, hipStream_t stream, Profiler *prof)
{
    if (sw.strip < 64 || sw.strip > STAR_MAX_THREADS || sw.strip % 64 || sw.blocks_per_xcd < 1 ||
        g.sqi >= 0)
        return hipErrorInvalidValue;
    if (!emit_ok(eo, g))
        return hipErrorInvalidValue;
    ProfScope ps(prof, K_STAR_MOM, stream);
    if (g.ebytes == 4)
        return moments_t<uint32_t>(g, fm, L, R, Rp, plan, eo, sw, stream);
    return moments_t<uint64_t>(g, fm, L, R, Rp, plan, eo, sw, stream);
}

}  // namespace oss
