// Width encoding of the bundles (Section 3.4): the density map controls the width of the
// line segments of every polyline, so that the bundle weight shows as width as well as
// through alpha blending. Per point, the density of its edge's layer at the point; per point,
// the width from that density on a linear or logarithmic scale.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "render.h"

namespace hb {

// One wave per edge, its points 64 at a time (coalesced), four such chunks in flight per
// trip: bilinear density at each point in its edge's layer, from the strip map of its layer
// (the four clamped taps in one 16-byte load, the same taps, fractions and rounding as the
// advection's density samples), clamped at 0; a wave maximum, then one
// atomic max on the float bits (non-negative floats order as their bits).
constexpr int kDensChunks = 4;

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
    const HB_G float *__restrict__ rho = glb(d.rhos + (int64_t)d.group[e] * rho_strip_plane(W, H));
    const HB_G float2 *__restrict__ xs = glb(d.samples + o0);
    HB_G float *__restrict__ out = glb(dens + o0);
    float m = 0.0f;
    for (int64_t j0 = 0; j0 < n; j0 += 64 * kDensChunks) {
        float2 x[kDensChunks];
#pragma unroll
        for (int u = 0; u < kDensChunks; ++u) {
            const int64_t j = j0 + 64 * u + lane;
            x[u] = make_float2(0.5f, 0.5f);
            if (j < n) x[u] = ld2(xs + j);
        }
        STap c[kDensChunks];
        Quad q[kDensChunks];
#pragma unroll
        for (int u = 0; u < kDensChunks; ++u) {
            c[u] = stap_of(x[u].x, x[u].y, W, H);
            q[u] = ld_rho(rho, c[u].od);
        }
#pragma unroll
        for (int u = 0; u < kDensChunks; ++u) {
            const int64_t j = j0 + 64 * u + lane;
            float r = interp1q(q[u], c[u]);
            r = r > 0.0f ? r : 0.0f;
            if (j < n) {
                out[j] = r;
                m = fmaxf(m, r);
            }
        }
    }
    for (int s = 32; s >= 1; s >>= 1) m = fmaxf(m, __shfl_xor(m, s, 64));
    if (lane == 0 && m > 0.0f) atomicMax(maxbits, __float_as_uint(m));
}

// Four points per thread, kBlock apart (coalesced, all loads issued before the arithmetic).
// FP32: t = f(rho) / f(max) with f the identity or log2(1 + x) by the hardware base-2
// logarithm (the ratio of two logarithms does not depend on their base), as one product
// with the reciprocal of f(max); width = w_min + t (w_max - w_min), and the largest density
// gets w_max itself.
constexpr int kWidthPts = 4;

__global__ __launch_bounds__(kBlock) void k_widths(const float *__restrict__ dens, int64_t n,
                                                   const uint32_t *__restrict__ maxbits, float w_min,
                                                   float w_max, int log_scale,
                                                   float *__restrict__ widths) {
    const int64_t i0 = (int64_t)blockIdx.x * (kBlock * kWidthPts) + threadIdx.x;
    const float rmax = __uint_as_float(*maxbits);
    const float fmax = log_scale ? __log2f(1.0f + rmax) : rmax;
    const float inv = fmax > 0.0f ? 1.0f / fmax : 0.0f;
    const float range = w_max - w_min;
    float r[kWidthPts];
#pragma unroll
    for (int u = 0; u < kWidthPts; ++u) {
        const int64_t i = i0 + (int64_t)u * kBlock;
        r[u] = i < n ? dens[i] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kWidthPts; ++u) {
        const int64_t i = i0 + (int64_t)u * kBlock;
        if (i >= n) continue;
        float w = w_min;
        if (fmax > 0.0f) {
            const float f = log_scale ? __log2f(1.0f + r[u]) : r[u];
            w = r[u] >= rmax ? w_max : fminf(__builtin_fmaf(f * inv, range, w_min), w_max);
        }
        widths[i] = w;
    }
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
    const int64_t per = (int64_t)kBlock * kWidthPts;
    hipLaunchKernelGGL(k_widths, dim3((unsigned)((n + per - 1) / per)), dim3(kBlock), 0, st, dens, n,
                       maxbits, (float)w_min, (float)w_max, log_scale, widths);
    return hipGetLastError();
}

}  // namespace hb
