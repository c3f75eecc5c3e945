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

// Star feature sums at (x0 + lane, y) for radius r (square half-width s):
// the square by 4 lookups into L (Eq. S_1), the diamond by 2 into R and 2
// into R'.  Lb/Rb/Rpb point at table column x0 (the lane adds lane_off =
// (lane + 1) entries: table column = image column + 1); table row = image
// row + 1.  Only called for positions where the star fits.
template <typename T, int NQ>
__device__ __forceinline__ void star_sums(const char *Lb, const char *Rb, const char *Rpb,
                                          int64_t row_bytes, uint32_t lane_off, int y, int r,
                                          int s, int64_t *F)
{
    constexpr int64_t ES = (int64_t)sizeof(T) * NQ;
    const char *l_top = Lb + (int64_t)(y - s) * row_bytes;      // row y-s-1
    const char *l_bot = Lb + (int64_t)(y + s + 1) * row_bytes;  // row y+s
    const char *r_top = Rb + (int64_t)(y - r) * row_bytes;      // row y-r-1
    const char *r_bot = Rb + (int64_t)(y + r + 1) * row_bytes;  // row y+r
    const char *rp_mid = Rpb + (int64_t)y * row_bytes;           // row y-1
    const int64_t ds = (int64_t)s * ES, ds1 = (int64_t)(s + 1) * ES;
    const int64_t dr = (int64_t)r * ES, dr1 = (int64_t)(r + 1) * ES;
    const Entry<T, NQ> a = at<T, NQ>(l_bot + ds, lane_off);    // L(x+s,   y+s)
    const Entry<T, NQ> b = at<T, NQ>(l_bot - ds1, lane_off);   // L(x-s-1, y+s)
    const Entry<T, NQ> c = at<T, NQ>(l_top + ds, lane_off);    // L(x+s,   y-s-1)
    const Entry<T, NQ> d = at<T, NQ>(l_top - ds1, lane_off);   // L(x-s-1, y-s-1)
    const Entry<T, NQ> e = at<T, NQ>(r_bot, lane_off);         // R(x, y+r)
    const Entry<T, NQ> f = at<T, NQ>(rp_mid - dr1, lane_off);  // R'(x-r-1, y-1)
    const Entry<T, NQ> h = at<T, NQ>(rp_mid + dr, lane_off);   // R'(x+r, y-1)
    const Entry<T, NQ> k = at<T, NQ>(r_top, lane_off);         // R(x, y-r-1)
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        F[q] = widen((T)(a.v[q] - b.v[q] - c.v[q] + d.v[q])) +
               widen((T)(e.v[q] - f.v[q] - h.v[q] + k.v[q]));
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
