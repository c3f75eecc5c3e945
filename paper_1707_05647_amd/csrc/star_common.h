// Device helpers shared by the plain and the batched star kernels.
#pragma once

#include "oss_internal.h"

#include <type_traits>

namespace oss {

template <typename T, int NQ>
struct Entry {
    T v[NQ];
};

// Sum of two region sums that were formed in T: with 32-bit tables each
// region sum is exact modulo 2^32 and below 2^32, so it zero-extends.
__device__ __forceinline__ int64_t widen(uint32_t v) { return (int64_t)v; }
__device__ __forceinline__ int64_t widen(uint64_t v) { return (int64_t)v; }


// Table entry layouts.  TabU: NQ quantities of T in feature order.  TabMix:
// 16-byte entries with the squares (feature slot SQI) as 64 bits and the
// other quantities, in feature order, as 32 bits modulo 2^32.  reduce()
// forms the square and the diamond sum of every quantity in the entry's
// width (a - b - c + d) and adds the two widened sums in 64 bits: a region
// sum below 2^32 is exact modulo 2^32.
template <typename T, int NQ_>
struct TabU {
    static constexpr int NQ = NQ_;
    static constexpr int64_t ES = (int64_t)sizeof(T) * NQ;
    static constexpr bool STAGE = false;  // no narrow load of one quantity pays off
    using E = Entry<T, NQ>;
    __device__ static __forceinline__ E load(const char *p, int64_t)
    {
        return *reinterpret_cast<const E *>(p);
    }
    __device__ static __forceinline__ void reduce(const E &a, const E &b, const E &c, const E &d,
                                                  const E &e, const E &f, const E &h, const E &k,
                                                  int64_t *F)
    {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            F[q] = widen((T)(a.v[q] - b.v[q] - c.v[q] + d.v[q])) +
                   widen((T)(e.v[q] - f.v[q] - h.v[q] + k.v[q]));
    }
};

struct MixEntry {
    uint64_t sq;
    uint32_t o[2];
};

template <int NQ_, int SQI>
struct TabMix {
    static constexpr int NQ = NQ_;
    static constexpr int64_t ES = 16;
    static constexpr bool STAGE = false;
    using E = MixEntry;
    __device__ static __forceinline__ E load(const char *p, int64_t)
    {
        return *reinterpret_cast<const E *>(p);
    }
    __device__ static __forceinline__ void reduce(const E &a, const E &b, const E &c, const E &d,
                                                  const E &e, const E &f, const E &h, const E &k,
                                                  int64_t *F)
    {
        F[SQI] = widen((uint64_t)(a.sq - b.sq - c.sq + d.sq)) +
                 widen((uint64_t)(e.sq - f.sq - h.sq + k.sq));
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if (q == SQI)
                continue;
            const int j = q < SQI ? q : q - 1;
            F[q] = widen((uint32_t)(a.o[j] - b.o[j] - c.o[j] + d.o[j])) +
                   widen((uint32_t)(e.o[j] - f.o[j] - h.o[j] + k.o[j]));
        }
    }
};

// Planar tables: quantity q of an entry sits `plane` bytes after quantity
// q-1; the entry stride is sizeof(T).  A wave's lookup is then NQ loads of
// 64 consecutive values each instead of one load of 64 interleaved entries.
template <typename T, int NQ_>
struct TabP {
    static constexpr int NQ = NQ_;
    static constexpr int64_t ES = (int64_t)sizeof(T);
    static constexpr bool STAGE = true;
    using E = Entry<T, NQ>;
    __device__ static __forceinline__ E load(const char *p, int64_t plane)
    {
        E e;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            e.v[q] = *reinterpret_cast<const T *>(p + q * plane);
        return e;
    }
    __device__ static __forceinline__ void reduce(const E &a, const E &b, const E &c, const E &d,
                                                  const E &e, const E &f, const E &h, const E &k,
                                                  int64_t *F)
    {
        TabU<T, NQ>::reduce(a, b, c, d, e, f, h, k, F);
    }
    // Staged lookup: quantity C (plane 0) alone, then the other planes.
    static constexpr int C = 0;
    using V = T;
    struct Rest {
        T v[NQ > 1 ? NQ - 1 : 1];
    };
    __device__ static __forceinline__ V load_c(const char *p, int64_t)
    {
        return *reinterpret_cast<const T *>(p);
    }
    __device__ static __forceinline__ Rest load_rest(const char *p, int64_t plane)
    {
        Rest e;
#pragma unroll
        for (int q = 1; q < NQ; ++q)
            e.v[q - 1] = *reinterpret_cast<const T *>(p + q * plane);
        return e;
    }
    __device__ static __forceinline__ void reduce_rest(const Rest &a, const Rest &b, const Rest &c,
                                                       const Rest &d, const Rest &e, const Rest &f,
                                                       const Rest &h, const Rest &k, int64_t *F)
    {
#pragma unroll
        for (int q = 1; q < NQ; ++q)
            F[q] = widen((T)(a.v[q - 1] - b.v[q - 1] - c.v[q - 1] + d.v[q - 1])) +
                   widen((T)(e.v[q - 1] - f.v[q - 1] - h.v[q - 1] + k.v[q - 1]));
    }
};

// Planar tables whose squares need 64 bits: every plane holds 32-bit values
// and the squares (slot SQI) take two planes, low word then high word, so a
// wave's lookup of one quantity is 64 consecutive 32-bit words.  The other
// quantities are exact modulo 2^32 as in TabMix.
template <int NQ_, int SQI>
struct TabPS {
    static constexpr int NQ = NQ_;
    static constexpr int64_t ES = 4;
    static constexpr bool STAGE = true;
    static constexpr int NP = NQ + 1;  // planes
    struct E {
        uint32_t v[NP];
    };
    // plane of quantity q (the squares: this plane and the next)
    static constexpr int pl(int q) { return q <= SQI ? q : q + 1; }
    __device__ static __forceinline__ uint32_t word(const char *p, int64_t plane, int i)
    {
        return *reinterpret_cast<const uint32_t *>(p + i * plane);
    }
    __device__ static __forceinline__ E load(const char *p, int64_t plane)
    {
        E e;
#pragma unroll
        for (int i = 0; i < NP; ++i)
            e.v[i] = word(p, plane, i);
        return e;
    }
    __device__ static __forceinline__ uint64_t sq(const E &e)
    {
        return (uint64_t)e.v[SQI] | ((uint64_t)e.v[SQI + 1] << 32);
    }
    // F[q] for every quantity q != skip
    __device__ static __forceinline__ void reduce_skip(const E &a, const E &b, const E &c,
                                                       const E &d, const E &e, const E &f,
                                                       const E &h, const E &k, int64_t *F,
                                                       int skip)
    {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if (q == skip)
                continue;
            if (q == SQI) {
                F[q] = widen((uint64_t)(sq(a) - sq(b) - sq(c) + sq(d))) +
                       widen((uint64_t)(sq(e) - sq(f) - sq(h) + sq(k)));
            } else {
                const int i = pl(q);
                F[q] = widen((uint32_t)(a.v[i] - b.v[i] - c.v[i] + d.v[i])) +
                       widen((uint32_t)(e.v[i] - f.v[i] - h.v[i] + k.v[i]));
            }
        }
    }
    __device__ static __forceinline__ void reduce(const E &a, const E &b, const E &c, const E &d,
                                                  const E &e, const E &f, const E &h, const E &k,
                                                  int64_t *F)
    {
        reduce_skip(a, b, c, d, e, f, h, k, F, -1);
    }
    // Staged lookup: the first 32-bit quantity alone, then the other planes.
    static constexpr int C = SQI == 0 ? 1 : 0;
    using V = uint32_t;
    using Rest = E;
    __device__ static __forceinline__ V load_c(const char *p, int64_t plane)
    {
        return word(p, plane, pl(C));
    }
    __device__ static __forceinline__ Rest load_rest(const char *p, int64_t plane)
    {
        E e;
#pragma unroll
        for (int i = 0; i < NP; ++i)
            e.v[i] = i == pl(C) ? 0u : word(p, plane, i);
        return e;
    }
    __device__ static __forceinline__ void reduce_rest(const Rest &a, const Rest &b, const Rest &c,
                                                       const Rest &d, const Rest &e, const Rest &f,
                                                       const Rest &h, const Rest &k, int64_t *F)
    {
        reduce_skip(a, b, c, d, e, f, h, k, F, C);
    }
};

// Planar record tables (sum, squares, gradient, with every square and
// diamond sum of the squares below 2^40): the sum plane (32-bit values, as
// the other planar layouts), then per entry one 8-byte record {squares low
// word, gradient}, then a byte plane with the squares' bits 32..39.  A
// square or diamond sum of the squares is formed modulo 2^40 from these
// and is exact; the other quantities are exact modulo 2^32 as in TabPS.
// With plane = the sum plane's bytes and base = the table's entry 0:
//   sum of entry e      at base + 4 e
//   record of entry e   at base + plane - 4 + 8 e  (entry (0, y) starts a line)
//   byte of entry e     at base + 3 plane + 3 + e  (likewise)
// so a lookup at sum address p finds its record and byte from p - base; the
// second-stage lookups of a staged pass touch one record line and one byte
// line per lane instead of three plane lines.
struct TabPR {
    static constexpr int NQ = 3;
    static constexpr int64_t ES = 4;
    static constexpr bool STAGE = true;
    static constexpr bool REC = true;
    static constexpr int C = 0;  // the sum: looked up first, alone
    using V = uint32_t;
    struct Rest {
        uint32_t lo, g, hi;
    };
    struct E {
        uint32_t c;
        Rest r;
    };
    __device__ static __forceinline__ V load_c(const char *p, int64_t)
    {
        return *reinterpret_cast<const uint32_t *>(p);
    }
    __device__ static __forceinline__ Rest load_rest(const char *p, const char *base,
                                                     int64_t plane)
    {
        const int64_t off = p - base;
        const uint2 r = *reinterpret_cast<const uint2 *>(base + (plane - 4) + 2 * off);
        const uint8_t h = *reinterpret_cast<const uint8_t *>(base + 3 * plane + 3 + (off >> 2));
        return {r.x, r.y, (uint32_t)h};
    }
    __device__ static __forceinline__ E load(const char *p, const char *base, int64_t plane)
    {
        return {load_c(p, plane), load_rest(p, base, plane)};
    }
    __device__ static __forceinline__ uint64_t sq(const Rest &r)
    {
        return (uint64_t)r.lo | ((uint64_t)r.hi << 32);
    }
    __device__ static __forceinline__ int64_t w40(uint64_t v)
    {
        return (int64_t)(v & ((1ull << 40) - 1));
    }
    __device__ static __forceinline__ void reduce_rest(const Rest &a, const Rest &b, const Rest &c,
                                                       const Rest &d, const Rest &e, const Rest &f,
                                                       const Rest &h, const Rest &k, int64_t *F)
    {
        F[1] = w40(sq(a) - sq(b) - sq(c) + sq(d)) + w40(sq(e) - sq(f) - sq(h) + sq(k));
        F[2] = widen((uint32_t)(a.g - b.g - c.g + d.g)) + widen((uint32_t)(e.g - f.g - h.g + k.g));
    }
    __device__ static __forceinline__ void reduce(const E &a, const E &b, const E &c, const E &d,
                                                  const E &e, const E &f, const E &h, const E &k,
                                                  int64_t *F)
    {
        F[0] = widen((uint32_t)(a.c - b.c - c.c + d.c)) + widen((uint32_t)(e.c - f.c - h.c + k.c));
        reduce_rest(a.r, b.r, c.r, d.r, e.r, f.r, h.r, k.r, F);
    }
};

// Layouts whose loads need the table's entry-0 pointer (TabPR).
template <typename T, typename = void>
struct IsRec : std::false_type {};
template <typename T>
struct IsRec<T, std::void_t<decltype(T::REC)>> : std::true_type {};

// The entry-0 pointers of the three tables of a reference.
struct TabBases {
    const char *L, *R, *Rp;
};

// Load the entry at p of table base (any layout).
template <typename Tab>
__device__ __forceinline__ typename Tab::E tab_load(const char *p, const char *base,
                                                    int64_t plane)
{
    if constexpr (IsRec<Tab>::value)
        return Tab::load(p, base, plane);
    else
        return Tab::load(p, plane);
}

template <typename Tab>
__device__ __forceinline__ auto tab_load_rest(const char *p, const char *base, int64_t plane)
{
    if constexpr (IsRec<Tab>::value)
        return Tab::load_rest(p, base, plane);
    else
        return Tab::load_rest(p, plane);
}

// Entry at a wave-uniform row base plus this lane's byte offset.
template <typename E>
__device__ __forceinline__ E entry_at(const char *row, uint32_t lane_off)
{
    return *reinterpret_cast<const E *>(row + lane_off);
}

// Addresses of the 8 lookups of the star at (x0 + lane, y) for radius r
// (square half-width s): the square by 4 lookups into L (Eq. S_1), the
// diamond by 2 into R and 2 into R'.  Lb/Rb/Rpb point at table column x0
// (the lane adds lane_off = (lane + 1) entries: table column = image column
// + 1); table row = image row + 1.  Only used for positions where the star
// fits.
struct StarAddr {
    const char *a, *b, *c, *d, *e, *f, *h, *k;
};

template <typename Tab>
__device__ __forceinline__ StarAddr star_addr(const char *Lb, const char *Rb, const char *Rpb,
                                              int64_t row_bytes, uint32_t lane_off, int y, int r,
                                              int s)
{
    constexpr int64_t ES = Tab::ES;
    const char *l_top = Lb + (int64_t)(y - s) * row_bytes;      // row y-s-1
    const char *l_bot = Lb + (int64_t)(y + s + 1) * row_bytes;  // row y+s
    const char *r_top = Rb + (int64_t)(y - r) * row_bytes;      // row y-r-1
    const char *r_bot = Rb + (int64_t)(y + r + 1) * row_bytes;  // row y+r
    const char *rp_mid = Rpb + (int64_t)y * row_bytes;           // row y-1
    const int64_t ds = (int64_t)s * ES, ds1 = (int64_t)(s + 1) * ES;
    const int64_t dr = (int64_t)r * ES, dr1 = (int64_t)(r + 1) * ES;
    StarAddr o;
    o.a = l_bot + ds + lane_off;    // L(x+s,   y+s)
    o.b = l_bot - ds1 + lane_off;   // L(x-s-1, y+s)
    o.c = l_top + ds + lane_off;    // L(x+s,   y-s-1)
    o.d = l_top - ds1 + lane_off;   // L(x-s-1, y-s-1)
    o.e = r_bot + lane_off;         // R(x, y+r)
    o.f = rp_mid - dr1 + lane_off;  // R'(x-r-1, y-1)
    o.h = rp_mid + dr + lane_off;   // R'(x+r, y-1)
    o.k = r_top + lane_off;         // R(x, y-r-1)
    return o;
}

// The same addresses from the item's row bases (table row y of L, R and R':
// image row y - 1) and the radius' row offsets roff = {-s, s+1, -r, r+1}
// table rows in bytes (computed once per plan), so no per-radius multiply.
template <typename Tab>
__device__ __forceinline__ StarAddr star_addr_rows(const char *Ly, const char *Ry,
                                                   const char *Rpy, const int64_t *roff,
                                                   uint32_t lane_off, int r, int s)
{
    constexpr int64_t ES = Tab::ES;
    const char *l_top = Ly + roff[0];  // row y-s-1
    const char *l_bot = Ly + roff[1];  // row y+s
    const char *r_top = Ry + roff[2];  // row y-r-1
    const char *r_bot = Ry + roff[3];  // row y+r
    const int64_t ds = (int64_t)s * ES, ds1 = (int64_t)(s + 1) * ES;
    const int64_t dr = (int64_t)r * ES, dr1 = (int64_t)(r + 1) * ES;
    StarAddr o;
    o.a = l_bot + ds + lane_off;    // L(x+s,   y+s)
    o.b = l_bot - ds1 + lane_off;   // L(x-s-1, y+s)
    o.c = l_top + ds + lane_off;    // L(x+s,   y-s-1)
    o.d = l_top - ds1 + lane_off;   // L(x-s-1, y-s-1)
    o.e = r_bot + lane_off;         // R(x, y+r)
    o.f = Rpy - dr1 + lane_off;     // R'(x-r-1, y-1)
    o.h = Rpy + dr + lane_off;      // R'(x+r, y-1)
    o.k = r_top + lane_off;         // R(x, y-r-1)
    return o;
}

// Star feature sums of every quantity (tb: the tables' entry-0 pointers; the
// lookups a..d are in L, e and k in R, f and h in R').
template <typename Tab>
__device__ __forceinline__ void star_sums_at(const StarAddr &p, const TabBases &tb, int64_t *F,
                                             int64_t plane)
{
    Tab::reduce(tab_load<Tab>(p.a, tb.L, plane), tab_load<Tab>(p.b, tb.L, plane),
                tab_load<Tab>(p.c, tb.L, plane), tab_load<Tab>(p.d, tb.L, plane),
                tab_load<Tab>(p.e, tb.R, plane), tab_load<Tab>(p.f, tb.Rp, plane),
                tab_load<Tab>(p.h, tb.Rp, plane), tab_load<Tab>(p.k, tb.R, plane), F);
}

template <typename Tab>
__device__ __forceinline__ void star_sums(const char *Lb, const char *Rb, const char *Rpb,
                                          int64_t row_bytes, uint32_t lane_off, int y, int r,
                                          int s, const TabBases &tb, int64_t *F, int64_t plane)
{
    star_sums_at<Tab>(star_addr<Tab>(Lb, Rb, Rpb, row_bytes, lane_off, y, r, s), tb, F, plane);
}

// Staged form (planar layouts, Tab::STAGE): the feature sum of quantity
// Tab::C alone (one load of 64 consecutive values per wave and lookup), and,
// for the positions that pass its compare, the others.
template <typename Tab>
__device__ __forceinline__ int64_t star_sum_c(const StarAddr &p, int64_t plane)
{
    using V = typename Tab::V;
    const V a = Tab::load_c(p.a, plane), b = Tab::load_c(p.b, plane);
    const V c = Tab::load_c(p.c, plane), d = Tab::load_c(p.d, plane);
    const V e = Tab::load_c(p.e, plane), f = Tab::load_c(p.f, plane);
    const V h = Tab::load_c(p.h, plane), k = Tab::load_c(p.k, plane);
    return widen((V)(a - b - c + d)) + widen((V)(e - f - h + k));
}

template <typename Tab>
__device__ __forceinline__ void star_sums_rest(const StarAddr &p, const TabBases &tb,
                                               int64_t plane, int64_t *F)
{
    Tab::reduce_rest(tab_load_rest<Tab>(p.a, tb.L, plane), tab_load_rest<Tab>(p.b, tb.L, plane),
                     tab_load_rest<Tab>(p.c, tb.L, plane), tab_load_rest<Tab>(p.d, tb.L, plane),
                     tab_load_rest<Tab>(p.e, tb.R, plane), tab_load_rest<Tab>(p.f, tb.Rp, plane),
                     tab_load_rest<Tab>(p.h, tb.Rp, plane), tab_load_rest<Tab>(p.k, tb.R, plane),
                     F);
}

// ---------------------------------------------------------------------------
// Emission of one screened row segment: the wave's 64 columns of row y with
// the final scale bits of MT template slots; per slot the mask bytes, the
// segment's candidate count and its candidates in column order (see
// EmitOut; with eo.seg_count null only the mask).  Wave-local: a ballot
// gives the count, the lane's rank among the set ballot bits its slot.
// ---------------------------------------------------------------------------

// The emission geometry matches the tables (host check).
inline bool emit_ok(const EmitOut &eo, const BuildGeom &g)
{
    return eo.H == g.H && eo.W == g.W && eo.n_chunks == (g.W + SEG_W - 1) / SEG_W &&
           (eo.seg_count == nullptr) == (eo.stage == nullptr);
}

// Emission stores: through global-memory pointers (a store through a
// generic pointer becomes a flat store, which also counts on the scalar-load
// counter and would make the next scalar load wait for it), and streaming
// (non-temporal), so the mask and staged candidates do not take L2 lines
// from the tables the star pass is still reading (workload 5: star pass
// 54.0 -> 53.4 ms).
__device__ __forceinline__ void store_u8_global(uint8_t *p, uint8_t v)
{
    __builtin_nontemporal_store(v, (__attribute__((address_space(1))) uint8_t *)p);
}

__device__ __forceinline__ void store_u32x2_global(uint2 *p, uint32_t a, uint32_t b)
{
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 v = {a, b};
    __builtin_nontemporal_store(v, (__attribute__((address_space(1))) u32x2 *)p);
}

__device__ __forceinline__ int lane_rank(uint64_t ballot)
{
    // set ballot bits below this lane
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(ballot >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)ballot, 0u));
}

// Emission of one image row of a wave: x is this lane's column (the wave
// covers a 64-aligned run of columns).  emit_begin is false for a wave wholly
// right of the image (uniform); emit_slot then writes one template's mask
// bytes, segment count and staged candidates from this lane's scale bits v.
// tg is the template index of the slot in the screen, m its mask (or null);
// both should come from read-only kernel arguments (scalar loads): a vector
// load here would wait for every store in flight, since one counter counts
// both.
struct EmitRow {
    int64_t srow;  // segment within a template
    int64_t tseg;  // segments per template
    int lane;
    bool inw;      // this lane's column lies in the image
};

__device__ __forceinline__ bool emit_begin(const EmitOut &eo, int y, int x, EmitRow *er)
{
    er->lane = threadIdx.x & 63;
    er->inw = x < eo.W;
    er->srow = (int64_t)y * eo.n_chunks + (x >> 6);
    er->tseg = (int64_t)eo.H * eo.n_chunks;
    return x - er->lane < eo.W;
}

__device__ __forceinline__ void emit_slot(const EmitOut &eo, const EmitRow &er, int y, int x,
                                          uint32_t v, int tg, uint8_t *m)
{
    const bool on = er.inw && v != 0u;
    if (m && er.inw)
        store_u8_global(m + (int64_t)y * eo.W + x, on ? 1 : 0);
    if (eo.seg_count) {
        const uint64_t bal = __builtin_amdgcn_ballot_w64(on);
        const int64_t seg = (int64_t)tg * er.tseg + er.srow;
        if (er.lane == 0)
            store_u8_global(eo.seg_count + seg, (uint8_t)__popcll(bal));
        if (on)
            store_u32x2_global(eo.stage + seg * SEG_W + lane_rank(bal), (uint32_t)x, v);
    }
}

// The whole row for slots 0..nt-1: val(t) -> scale bits of slot t
// (compile-time t), tg(t) -> template index, mk(t) -> mask (or null).
template <int MT, typename Val, typename Tg, typename Mk>
__device__ __forceinline__ void emit_row(const EmitOut &eo, int nt, int y, int x, Val val, Tg tg,
                                         Mk mk)
{
    EmitRow er;
    if (!emit_begin(eo, y, x, &er))
        return;
#pragma unroll
    for (int t = 0; t < MT; ++t)
        if (t < nt)
            emit_slot(eo, er, y, x, val(t), tg(t), mk(t));
}

// The sweep with at most as many blocks per XCD as the GPU holds at once for
// this kernel (host side).  Items are dealt to blocks statically, so a block
// that cannot be resident until others finish would run its share as a tail
// after them.
inline StarSweep resident_sweep(const void *kernel, StarSweep sw, size_t lds_bytes)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, sw.strip, lds_bytes) !=
            hipSuccess)
        return sw;
    const int cap = per_cu * (cus / 8);
    if (cap > 0 && sw.blocks_per_xcd > cap)
        sw.blocks_per_xcd = cap;
    return sw;
}

// Position of sweep item `it` of XCD `xcd`: image row y and the strip's first
// column x0 (y >= H marks an empty item of a short last part).
__device__ __forceinline__ void sweep_item(const StarSweep &sw, int xcd, int it, int strip_w, int *y,
                                           int *x0)
{
    const int t = it / sw.rows_per_part;
    const int u = xcd + 8 * t;
    const int strip = u / sw.parts, part = u - strip * sw.parts;
    *y = part * sw.rows_per_part + (it - t * sw.rows_per_part);
    *x0 = strip * strip_w;
}

}  // namespace oss
