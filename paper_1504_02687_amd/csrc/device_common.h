// Device helpers shared by the forward and adjoint kernels of the bundling library.
#pragma once

#include <hip/hip_runtime.h>

#include "hb_internal.h"

namespace hb {

// ---------------------------------------------------------------- helpers

#define HB_FIND(field)                                                   \
    int g = 0;                                                           \
    {                                                                    \
        int lo_ = 0, hi_ = ng - 1;                                       \
        while (lo_ < hi_) {                                              \
            int mid_ = (lo_ + hi_ + 1) >> 1;                             \
            if (gd[mid_].field <= blk) lo_ = mid_; else hi_ = mid_ - 1;  \
        }                                                                \
        g = lo_;                                                         \
    }                                                                    \
    const GDesc &d = gd[g];

__device__ __forceinline__ bool stopped(const GDesc &d) {
    return (*(volatile const int32_t *)d.status & ST_STOP) != 0;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Butterfly sum: every lane ends with the same value (IEEE addition is commutative).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Exclusive block scan of one int64 per thread (kBlock threads); *total gets the sum.
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t *total) {
    __shared__ int64_t ws[kWavesPerBlock];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t incl = wave_incl_scan<int64_t>(v, lane);
    if (lane == 63) ws[wid] = incl;
    __syncthreads();
    int64_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) {
        if (w < wid) pre += ws[w];
        tot += ws[w];
    }
    __syncthreads();
    *total = tot;
    return pre + incl - v;
}

// Edge handled by wave `wid` of block `blk_local` of a graph. Blocks are dealt to the XCDs
// round-robin, so block b is mapped to chunk c of the visiting order with consecutive
// chunks on the same XCD: each XCD walks one contiguous range of the order (edges sorted
// by group and position), which keeps its share of the density maps small enough for its
// L2. Returns -1 past the last edge.
__device__ __forceinline__ int64_t edge_of(const GDesc &d, int64_t blk_local, int wid) {
    const int64_t nblk = (d.n_edges + kWavesPerBlock - 1) / kWavesPerBlock;
    const int64_t nx = d.nxcd;
    const int64_t x = blk_local % nx, i = blk_local / nx;
    const int64_t q = nblk / nx, r = nblk % nx;
    const int64_t c = x * q + (x < r ? x : r) + i;
    const int64_t idx = c * kWavesPerBlock + wid;
    if (idx >= d.n_edges) return -1;
    return d.perm ? (int64_t)d.perm[idx] : idx;
}

__device__ __forceinline__ int64_t sample_count(double L, double delta) {
    double q = ceil(L / delta);
    if (!(q >= 1.0)) q = 1.0;          // also catches NaN
    if (q > 4.0e15) q = 4.0e15;
    return (int64_t)q + 1;
}

// Explicit roundings (no contraction choices left to the compiler), so that every kernel
// variant computes the same bits.
__device__ __forceinline__ double seg_len(float2 a, float2 b) {
    const double dx = (double)b.x - (double)a.x, dy = (double)b.y - (double)a.y;
    return sqrt(__fma_rn(dx, dx, __dmul_rn(dy, dy)));
}

// ---------------------------------------------------------------- spatial binning

// Histogram tile (key) of a sample and its pixel inside the tile: the pixel the sample
// falls in (floor of its coordinates), clamped to the grid.
__device__ __forceinline__ void bin_of(const GDesc &d, int layer, float2 p, int &key,
                                       uint32_t &local) {
    const float fu = fminf(fmaxf(floorf(p.x), 0.0f), (float)(d.W - 1));
    const float fv = fminf(fmaxf(floorf(p.y), 0.0f), (float)(d.H - 1));
    const int u = (int)fu, v = (int)fv;
    key = (layer * d.tiles_y + (v >> kTileShift)) * d.tiles_x + (u >> kTileShift);
    local = (uint32_t)(((v & (kTile - 1)) << kTileShift) | (u & (kTile - 1)));
}

// Runs of equal keys among lanes 0..cnt-1 of a wave, which hold consecutive samples of one
// edge (about 64 of them share one or two tiles). Ballot of the lanes that start a run.
__device__ __forceinline__ uint64_t run_heads(int key, int lane, int cnt) {
    const int prev = __shfl_up(key, 1, 64);
    return __ballot(lane < cnt && (lane == 0 || prev != key));
}

// Length of the run that starts at lane `lane`.
__device__ __forceinline__ int run_length(uint64_t heads, int lane, int cnt) {
    const uint64_t after = lane == 63 ? 0ull : (heads >> (lane + 1));
    return (after ? lane + 1 + __builtin_ctzll(after) : cnt) - lane;
}

// First lane of the run that holds lane `lane` (lane < cnt).
__device__ __forceinline__ int run_head(uint64_t heads, int lane) {
    const uint64_t upto = lane == 63 ? heads : (heads & ((2ull << lane) - 1));
    return 63 - __builtin_clzll(upto | 1ull);
}

// ---------------------------------------------------------------- bilinear sampling

struct Bilin {
    int64_t i00, i10, i01, i11;
    double tx, ty;
};

// Taps of a bilinear sample at (x - 1/2, y - 1/2), clamped into the grid.
__device__ __forceinline__ Bilin bilin_taps(double x, double y, int W, int H) {
    double fx = fmin(fmax(x - 0.5, -1.0), (double)W);
    double fy = fmin(fmax(y - 0.5, -1.0), (double)H);
    double u0f = floor(fx), v0f = floor(fy);
    Bilin b;
    b.tx = fx - u0f;
    b.ty = fy - v0f;
    int u0 = (int)u0f, v0 = (int)v0f;
    int u1 = u0 + 1, v1 = v0 + 1;
    u0 = u0 < 0 ? 0 : (u0 > W - 1 ? W - 1 : u0);
    u1 = u1 < 0 ? 0 : (u1 > W - 1 ? W - 1 : u1);
    v0 = v0 < 0 ? 0 : (v0 > H - 1 ? H - 1 : v0);
    v1 = v1 < 0 ? 0 : (v1 > H - 1 ? H - 1 : v1);
    b.i00 = (int64_t)v0 * W + u0;
    b.i10 = (int64_t)v0 * W + u1;
    b.i01 = (int64_t)v1 * W + u0;
    b.i11 = (int64_t)v1 * W + u1;
    return b;
}

// FP32 taps and density sample for the acceptance tests (the precision of the stored map).
__device__ __forceinline__ float bilin1f(const float *__restrict__ m, float x, float y, int W,
                                         int H) {
    const float fx = fminf(fmaxf(x - 0.5f, -1.0f), (float)W);
    const float fy = fminf(fmaxf(y - 0.5f, -1.0f), (float)H);
    const float u0f = floorf(fx), v0f = floorf(fy);
    const float tx = fx - u0f, ty = fy - v0f;
    int u0 = (int)u0f, v0 = (int)v0f;
    int u1 = u0 + 1, v1 = v0 + 1;
    u0 = u0 < 0 ? 0 : (u0 > W - 1 ? W - 1 : u0);
    u1 = u1 < 0 ? 0 : (u1 > W - 1 ? W - 1 : u1);
    v0 = v0 < 0 ? 0 : (v0 > H - 1 ? H - 1 : v0);
    v1 = v1 < 0 ? 0 : (v1 > H - 1 ? H - 1 : v1);
    const float *r0 = m + v0 * W, *r1 = m + v1 * W;
    return (1.0f - tx) * (1.0f - ty) * r0[u0] + tx * (1.0f - ty) * r0[u1] +
           (1.0f - tx) * ty * r1[u0] + tx * ty * r1[u1];
}

// Density sample with the FP64 taps of the gradient sample.
__device__ __forceinline__ float bilin1(const float *__restrict__ m, const Bilin &b) {
    const float tx = (float)b.tx, ty = (float)b.ty;
    return (1.0f - tx) * (1.0f - ty) * m[b.i00] + tx * (1.0f - ty) * m[b.i10] +
           (1.0f - tx) * ty * m[b.i01] + tx * ty * m[b.i11];
}

// Gradient sample in FP64: the direction of a small gradient between taps of opposite
// sign keeps the precision of the stored taps.
__device__ __forceinline__ void bilin2(const float2 *__restrict__ m, const Bilin &b, double &gx,
                                       double &gy) {
    const double tx = b.tx, ty = b.ty;
    const double w00 = (1.0 - tx) * (1.0 - ty), w10 = tx * (1.0 - ty);
    const double w01 = (1.0 - tx) * ty, w11 = tx * ty;
    const float2 f00 = m[b.i00], f10 = m[b.i10], f01 = m[b.i01], f11 = m[b.i11];
    gx = w00 * f00.x + w10 * f10.x + w01 * f01.x + w11 * f11.x;
    gy = w00 * f00.y + w10 * f10.y + w01 * f01.y + w11 * f11.y;
}

}  // namespace hb
