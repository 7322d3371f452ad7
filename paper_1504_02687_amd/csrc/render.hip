// Width encoding of the bundles (Section 3.4): the density map controls the width of the
// line segments of every polyline, so that the bundle weight shows as width as well as
// through alpha blending. Per point, the density of its edge's layer at the point; per point,
// the width from that density on a linear or logarithmic scale.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "render.h"

namespace hb {

// One wave per edge, its points 64 at a time (coalesced): bilinear density at each point in
// its edge's layer (the taps and fractions of the advection's density samples), clamped at 0;
// a wave maximum, then one atomic max on the float bits (non-negative floats order as their
// bits).
__global__ __launch_bounds__(kBlock) void k_point_density(const GDesc *__restrict__ gd, int ng,
                                                          float *__restrict__ dens,
                                                          uint32_t *maxbits) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_edge);
    if (stopped(d)) return;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t e = (blk - d.blk_edge) * kWavesPerBlock + wid;
    if (e >= d.n_edges) return;
    const int W = d.W, H = d.H;
    const int64_t o0 = d.off_s[e], n = d.off_s[e + 1] - o0;
    const float *rho = d.rho + (int64_t)d.group[e] * ((int64_t)W * H);
    float m = 0.0f;
    for (int64_t j0 = 0; j0 < n; j0 += 64) {
        const int64_t j = j0 + lane;
        if (j < n) {
            const float2 x = d.samples[o0 + j];
            const Taps t = taps_of(x.x, x.y, W, H);
            float r = bilerp(rho[t.o00], rho[t.o10], rho[t.o01], rho[t.o11], t.tx, t.ty);
            r = r > 0.0f ? r : 0.0f;
            dens[o0 + j] = r;
            m = fmaxf(m, r);
        }
    }
    for (int s = 32; s >= 1; s >>= 1) m = fmaxf(m, __shfl_xor(m, s, 64));
    if (lane == 0 && m > 0.0f) atomicMax(maxbits, __float_as_uint(m));
}

__global__ __launch_bounds__(kBlock) void k_widths(const float *__restrict__ dens, int64_t n,
                                                   const uint32_t *__restrict__ maxbits, double w_min,
                                                   double w_max, int log_scale,
                                                   float *__restrict__ widths) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double rmax = (double)__uint_as_float(*maxbits), r = (double)dens[i];
    const double fmax = log_scale ? log1p(rmax) : rmax;
    const double f = log_scale ? log1p(r) : r;
    widths[i] = (float)(fmax > 0.0 ? w_min + (w_max - w_min) * (f / fmax) : w_min);
}

hipError_t launch_point_density(const GDesc *desc, const Shape &tot, float *dens, uint32_t *maxbits,
                                hipStream_t st) {
    if (tot.edge <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_point_density, dim3((unsigned)tot.edge), dim3(kBlock), 0, st, desc, 1, dens,
                       maxbits);
    return hipGetLastError();
}

hipError_t launch_widths(const float *dens, int64_t n, const uint32_t *maxbits, double w_min,
                         double w_max, int log_scale, float *widths, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_widths, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, dens,
                       n, maxbits, w_min, w_max, log_scale, widths);
    return hipGetLastError();
}

}  // namespace hb
