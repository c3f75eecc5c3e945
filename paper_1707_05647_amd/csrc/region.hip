// Preserved region of a screen (Sec. "Experimental Results", Exp. I: the
// regions the pre-processor keeps; their complement is the pruned region).
//
// A pixel is preserved for template t when it lies inside the star of
// radius r_{t,k} of some candidate of t carrying scale bit k.  The star is
// symmetric, so that is the same as: the star of radius r centred on the
// pixel contains such a candidate, i.e. the star sum of the candidates'
// indicator image is at least 1 there.  The library therefore dilates with
// its own tables: per (template, radius) it scatters the indicator into a
// zero-padded image (padding = the largest radius, so that every pixel of
// the image is a position where the star fits), builds that image's tables
// and runs the star pass with the single interval [1, max], then ORs the
// result into the region.  Cost: one build and one single-radius star pass
// over (H + 2R) x (W + 2R) per (template, radius), independent of the
// number of candidates.
#include "oss_internal.h"

#include <algorithm>

namespace oss {

// ind[(y + pad) * wp + x + pad] = 1 for list entries of template t with a
// bit of `bits` set; entries past *count (or list_cap), and entries outside
// the H x W image, are ignored.
__global__ void region_scatter_kernel(const oss_candidate *__restrict__ list, int64_t list_cap,
                                      const int64_t *__restrict__ count, int t, uint32_t bits,
                                      int H, int W, int pad, int64_t wp,
                                      uint8_t *__restrict__ ind)
{
    const int64_t n = min(*count, list_cap);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const oss_candidate c = list[i];
        if (c.t == t && (c.scale_bits & bits) && c.y >= 0 && c.y < H && c.x >= 0 && c.x < W)
            ind[(int64_t)(c.y + pad) * wp + (c.x + pad)] = 1;
    }
}

// region[y][x] |= hit[(y + pad) * wp + x + pad] != 0
__global__ void region_or_kernel(const uint8_t *__restrict__ hit, int H, int W, int pad,
                                 int64_t wp, uint8_t *__restrict__ region)
{
    const int64_t n = (int64_t)H * W;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
        if (hit[(int64_t)(y + pad) * wp + (x + pad)])
            region[i] = 1;
    }
}

hipError_t launch_region_scatter(const oss_candidate *list, int64_t list_cap,
                                 const int64_t *count, int t, uint32_t bits, int H, int W,
                                 int pad, int64_t wp, uint8_t *ind, hipStream_t st)
{
    const int64_t blocks = std::min<int64_t>(4096, std::max<int64_t>(1, (list_cap + 255) / 256));
    hipLaunchKernelGGL(region_scatter_kernel, dim3((unsigned)blocks), dim3(256), 0, st, list,
                       list_cap, count, t, bits, H, W, pad, wp, ind);
    return hipGetLastError();
}

hipError_t launch_region_or(const uint8_t *hit, int H, int W, int pad, int64_t wp,
                            uint8_t *region, hipStream_t st)
{
    const int64_t n = (int64_t)H * W;
    const int64_t blocks = std::min<int64_t>(8192, std::max<int64_t>(1, (n + 255) / 256));
    hipLaunchKernelGGL(region_or_kernel, dim3((unsigned)blocks), dim3(256), 0, st, hit, H, W,
                       pad, wp, region);
    return hipGetLastError();
}

}  // namespace oss
