// Device helpers shared by the plain and the batched star kernels.
#pragma once

#include "oss_internal.h"

namespace oss {

template <typename T, int NQ>
struct Entry {
    T v[NQ];
};

// Sum of two region sums that were formed in T: with 32-bit tables each
// region sum is exact modulo 2^32 and below 2^32, so it zero-extends.
__device__ __forceinline__ int64_t widen(uint32_t v) { return (int64_t)v; }
__device__ __forceinline__ int64_t widen(uint64_t v) { return (int64_t)v; }

// Entry at a wave-uniform row base plus this lane's byte offset.
template <typename T, int NQ>
__device__ __forceinline__ Entry<T, NQ> at(const char *row, uint32_t lane_off)
{
    return *reinterpret_cast<const Entry<T, NQ> *>(row + lane_off);
}

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
};

// Entry at a wave-uniform row base plus this lane's byte offset.
template <typename E>
__device__ __forceinline__ E entry_at(const char *row, uint32_t lane_off)
{
    return *reinterpret_cast<const E *>(row + lane_off);
}

// Star feature sums at (x0 + lane, y) for radius r (square half-width s):
// the square by 4 lookups into L (Eq. S_1), the diamond by 2 into R and 2
// into R'.  Lb/Rb/Rpb point at table column x0 (the lane adds lane_off =
// (lane + 1) entries: table column = image column + 1); table row = image
// row + 1.  Only called for positions where the star fits.
template <typename Tab>
__device__ __forceinline__ void star_sums(const char *Lb, const char *Rb, const char *Rpb,
                                          int64_t row_bytes, uint32_t lane_off, int y, int r,
                                          int s, int64_t *F, int64_t plane)
{
    using E = typename Tab::E;
    constexpr int64_t ES = Tab::ES;
    const char *l_top = Lb + (int64_t)(y - s) * row_bytes;      // row y-s-1
    const char *l_bot = Lb + (int64_t)(y + s + 1) * row_bytes;  // row y+s
    const char *r_top = Rb + (int64_t)(y - r) * row_bytes;      // row y-r-1
    const char *r_bot = Rb + (int64_t)(y + r + 1) * row_bytes;  // row y+r
    const char *rp_mid = Rpb + (int64_t)y * row_bytes;           // row y-1
    const int64_t ds = (int64_t)s * ES, ds1 = (int64_t)(s + 1) * ES;
    const int64_t dr = (int64_t)r * ES, dr1 = (int64_t)(r + 1) * ES;
    const E a = Tab::load(l_bot + ds + lane_off, plane);    // L(x+s,   y+s)
    const E b = Tab::load(l_bot - ds1 + lane_off, plane);   // L(x-s-1, y+s)
    const E c = Tab::load(l_top + ds + lane_off, plane);    // L(x+s,   y-s-1)
    const E d = Tab::load(l_top - ds1 + lane_off, plane);   // L(x-s-1, y-s-1)
    const E e = Tab::load(r_bot + lane_off, plane);         // R(x, y+r)
    const E f = Tab::load(rp_mid - dr1 + lane_off, plane);  // R'(x-r-1, y-1)
    const E h = Tab::load(rp_mid + dr + lane_off, plane);   // R'(x+r, y-1)
    const E k = Tab::load(r_top + lane_off, plane);         // R(x, y-r-1)
    Tab::reduce(a, b, c, d, e, f, h, k, F);
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
