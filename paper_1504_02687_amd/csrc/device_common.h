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

// Pointers into device memory (global address space): loads and stores through them are
// global (not flat) instructions, which take an SGPR base and wait only on the vector
// memory counter.
#define HB_G __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ HB_G T *glb(T *p) {
    return (HB_G T *)p;
}

// float2 through global pointers (one 8-byte access; the vector type's operators only
// take generic references).
__device__ __forceinline__ float2 ld2(const HB_G float2 *p) {
    const uint64_t v = *(const HB_G uint64_t *)p;
    return make_float2(__uint_as_float((uint32_t)v), __uint_as_float((uint32_t)(v >> 32)));
}
__device__ __forceinline__ float2 ld2(const float2 *p) { return *p; }
__device__ __forceinline__ void st2(HB_G float2 *p, float2 v) {
    *(HB_G uint64_t *)p = (uint64_t)__float_as_uint(v.x) | ((uint64_t)__float_as_uint(v.y) << 32);
}

// ---------------------------------------------------------------- cross-lane moves (DPP)

// DPP controls of gfx9 wave64: whole-wave shifts by one lane, row (16-lane) shifts, and the
// broadcasts of lane 15 / lane 31 into the following rows.
enum : int {
    kDppWaveShl1 = 0x130,   // lane l reads lane l + 1
    kDppWaveShr1 = 0x138,   // lane l reads lane l - 1
    kDppRowShr = 0x110,     // + n: lane l reads lane l - n of its row
    kDppRowBcast15 = 0x142,
    kDppRowBcast31 = 0x143,
};

// v of the lane selected by CTRL; lanes without a source, or outside the row mask, get old.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ int dpp(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp(float old, float v) {
    return __int_as_float(dpp<CTRL, ROWS>(__float_as_int(old), __float_as_int(v)));
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ int64_t dpp(int64_t old, int64_t v) {
    const int lo = dpp<CTRL, ROWS>((int)(uint32_t)old, (int)(uint32_t)v);
    const int hi = dpp<CTRL, ROWS>((int)(old >> 32), (int)(v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp(double old, double v) {
    return __longlong_as_double(dpp<CTRL, ROWS>((int64_t)__double_as_longlong(old),
                                                (int64_t)__double_as_longlong(v)));
}

// v of the lane selected by CTRL in every row; lanes without a source read 0 (the hardware
// bound control: no copy of an old value is needed).
template <int CTRL>
__device__ __forceinline__ int dpp0(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp0(float v) {
    return __int_as_float(dpp0<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ int64_t dpp0(int64_t v) {
    const int lo = dpp0<CTRL>((int)(uint32_t)v), hi = dpp0<CTRL>((int)(v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <int CTRL>
__device__ __forceinline__ double dpp0(double v) {
    return __longlong_as_double(dpp0<CTRL>((int64_t)__double_as_longlong(v)));
}

// Value of lane l - 1 (lane 0 gets fill, or 0) and of lane l + 1 (lane 63 gets fill, or 0).
// Every lane of the wave must be active.
template <typename T>
__device__ __forceinline__ T lane_prev(T v, T fill) {
    return dpp<kDppWaveShr1>(fill, v);
}
template <typename T>
__device__ __forceinline__ T lane_next(T v, T fill) {
    return dpp<kDppWaveShl1>(fill, v);
}
template <typename T>
__device__ __forceinline__ T lane_prev(T v) {
    return dpp0<kDppWaveShr1>(v);
}
template <typename T>
__device__ __forceinline__ T lane_next(T v) {
    return dpp0<kDppWaveShl1>(v);
}

// Value of lane 63, in every lane.
__device__ __forceinline__ double last_lane(double v) {
    const int64_t b = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ int64_t last_lane(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(v >> 32), 63);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Value of lane l (wave-uniform l), in every lane.
__device__ __forceinline__ double read_lane(double v, int l) {
    const int64_t b = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Inclusive sum over lanes 0..l (every lane active): shifts by 1, 2, 4, 8 inside each row
// of 16 lanes, then the row totals through the lane 15 and lane 31 broadcasts. The order of
// the additions is fixed, so the result is reproducible.
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v, int lane) {
    (void)lane;
    v += dpp0<kDppRowShr + 1>(v);
    v += dpp0<kDppRowShr + 2>(v);
    v += dpp0<kDppRowShr + 4>(v);
    v += dpp0<kDppRowShr + 8>(v);
    v += dpp<kDppRowBcast15, 0xa>((T)0, v);
    v += dpp<kDppRowBcast31, 0xc>((T)0, v);
    return v;
}

// Inclusive sum inside each half of the wave (lanes 0..31 and 32..63 separately): the same
// steps without the lane 31 broadcast, so lane 32 + r adds in the order lane r does.
template <typename T>
__device__ __forceinline__ T half_incl_scan(T v) {
    v += dpp0<kDppRowShr + 1>(v);
    v += dpp0<kDppRowShr + 2>(v);
    v += dpp0<kDppRowShr + 4>(v);
    v += dpp0<kDppRowShr + 8>(v);
    v += dpp<kDppRowBcast15, 0xa>((T)0, v);
    return v;
}

// Sum over the wave, the same value in every lane (every lane active).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    return last_lane(wave_incl_scan<T>(v, 0));
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
    // at most 2^31 edges (checked when the graph is set): block numbers fit 32 bits, and
    // 32-bit divisions are far shorter than 64-bit ones
    const uint32_t nblk = (uint32_t)((d.n_edges + kWavesPerBlock - 1) / kWavesPerBlock);
    const uint32_t nx = (uint32_t)d.nxcd, b = (uint32_t)blk_local;
    const uint32_t x = b % nx, i = b / nx;
    const uint32_t q = nblk / nx, r = nblk % nx;
    const int64_t c = (int64_t)x * q + (x < r ? x : r) + i;
    const int64_t idx = c * kWavesPerBlock + wid;
    if (idx >= d.n_edges) return -1;
    return idx;
}

__device__ __forceinline__ int64_t sample_count(double L, double delta) {
    double q = ceil(L / delta);
    if (!(q >= 1.0)) q = 1.0;          // also catches NaN
    if (q > 4.0e15) q = 4.0e15;
    return (int64_t)q + 1;
}

// FP64 operations rounded on their own: compiled with contraction off, so the compiler
// cannot fuse them with a neighbouring add or multiply, whatever the surrounding code.
__device__ __forceinline__ double mul_rn(double a, double b) {
#pragma clang fp contract(off)
    return a * b;
}
__device__ __forceinline__ double add_rn(double a, double b) {
#pragma clang fp contract(off)
    return a + b;
}
__device__ __forceinline__ double sub_rn(double a, double b) {
#pragma clang fp contract(off)
    return a - b;
}

// Length of the segment (a, b) and its reciprocal (both 0 for a zero-length segment) for
// the arclength walks of the resampling and its adjoint: the hardware reciprocal square root
// refined by one Newton step in FP64 (relative error of order 1e-15, instead of a correctly
// rounded square root and division). Sample counts come from seg_len below.
__device__ __forceinline__ void seg_len_rcp(float2 a, float2 b, double &len, double &rcp) {
    const double dx = sub_rn((double)b.x, (double)a.x), dy = sub_rn((double)b.y, (double)a.y);
    const double q = __builtin_fma(dx, dx, mul_rn(dy, dy));
    const double y0 = __builtin_amdgcn_rsq(q);
    const double e = __builtin_fma(-mul_rn(q, y0), y0, 1.0);       // 1 - q y0^2
    const double y1 = __builtin_fma(mul_rn(0.5, y0), e, y0);        // y0 (3 - q y0^2) / 2
    const bool pos = q > 0.0;
    len = pos ? mul_rn(q, y1) : 0.0;
    rcp = pos ? y1 : 0.0;
}

// 1 / sqrt(q) for q > 0: the hardware FP64 reciprocal square root refined by one Newton step
// (about 1 ulp; in place of a correctly rounded square root and a division).
__device__ __forceinline__ double rsqrt_nr(double q) {
    const double y0 = __builtin_amdgcn_rsq(q);
    const double e = __builtin_fma(-mul_rn(q, y0), y0, 1.0);
    return __builtin_fma(mul_rn(0.5, y0), e, y0);
}

// Explicit roundings (no contraction choices left to the compiler), so that every kernel
// variant computes the same bits.
__device__ __forceinline__ double seg_len(float2 a, float2 b) {
    const double dx = sub_rn((double)b.x, (double)a.x), dy = sub_rn((double)b.y, (double)a.y);
    return sqrt(__builtin_fma(dx, dx, mul_rn(dy, dy)));
}

// ---------------------------------------------------------------- spatial binning

// Histogram tile (key) of a sample and its pixel inside the tile: the pixel the sample
// falls in (floor of its coordinates), clamped to the grid.
__device__ __forceinline__ void pixel_of(float2 p, int W, int H, int &u, int &v) {
    u = (int)fminf(fmaxf(floorf(p.x), 0.0f), (float)(W - 1));
    v = (int)fminf(fmaxf(floorf(p.y), 0.0f), (float)(H - 1));
}

// Tile (key) of pixel (u, v) of a layer and the pixel's place inside the tile.
__device__ __forceinline__ void tile_of(const GDesc &d, int layer, int u, int v, int &key,
                                        uint32_t &local) {
    // at most 64 layers of at most 128 x 128 tiles: every factor fits the 24-bit multiplier
    key = (int)(__umul24(__umul24((uint32_t)layer, (uint32_t)d.tiles_y) + (uint32_t)(v >> kTileShift),
                         (uint32_t)d.tiles_x) + (uint32_t)(u >> kTileShift));
    local = (uint32_t)(((v & (kTile - 1)) << kTileShift) | (u & (kTile - 1)));
}

__device__ __forceinline__ void bin_of(const GDesc &d, int layer, float2 p, int &key,
                                       uint32_t &local) {
    int u, v;
    pixel_of(p, d.W, d.H, u, v);
    tile_of(d, layer, u, v, key, local);
}

// Runs of equal keys among lanes 0..cnt-1 of a wave, which hold consecutive samples of one
// edge (about 64 of them share one or two tiles). Ballot of the lanes that start a run.
__device__ __forceinline__ uint64_t run_heads(int key, int lane, int cnt) {
    const int prev = lane_prev(key, -1);
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

// Taps of a bilinear sample at (x - 1/2, y - 1/2), clamped into the grid: columns ua, ub
// and rows va, vb of the four taps (ua, va), (ub, va), (ua, vb), (ub, vb), and the FP32
// fractions between them. For x >= 1/2 the FP32 subtraction and the fraction are exact; below
// 1/2 (and at the far border) both taps of the axis are the same column or row, so the
// fraction has no effect.
struct Taps {
    int ua, ub, va, vb;
    float tx, ty;
};

__device__ __forceinline__ Taps taps_of(float x, float y, int W, int H) {
    const float fx = __builtin_amdgcn_fmed3f(x - 0.5f, -1.0f, (float)W);
    const float fy = __builtin_amdgcn_fmed3f(y - 0.5f, -1.0f, (float)H);
    const float u0f = floorf(fx), v0f = floorf(fy);
    Taps t;
    t.tx = fx - u0f;
    t.ty = fy - v0f;
    const int u0 = (int)u0f, v0 = (int)v0f;
    t.ua = min(max(u0, 0), W - 1);
    t.ub = min(max(u0 + 1, 0), W - 1);
    t.va = min(max(v0, 0), H - 1);
    t.vb = min(max(v0 + 1, 0), H - 1);
    return t;
}

// Wait for every outstanding vector-memory load of the wave (s_waitcnt vmcnt(0); the
// export and LDS/scalar counters are left alone).
__device__ __forceinline__ void vm_wait_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Bilinear interpolation of four taps a (u0,v0), b (u0+1,v0), c (u0,v0+1), d (u0+1,v0+1)
// at fractions (tx, ty), with one fixed rounding order (products of the weights rounded,
// the four terms summed a, b, c, d with fused multiply-adds; no contraction left to the
// compiler), so every kernel and every unrolled variant computes the same bits.
__device__ __forceinline__ float bilerp(float a, float b, float c, float d, float tx, float ty) {
#pragma clang fp contract(off)
    const float sx = 1.0f - tx, sy = 1.0f - ty;
    float r = (sx * sy) * a;
    r = __builtin_fmaf(tx * sy, b, r);
    r = __builtin_fmaf(sx * ty, c, r);
    return __builtin_fmaf(tx * ty, d, r);
}
__device__ __forceinline__ double bilerp(double a, double b, double c, double d, double tx,
                                         double ty) {
#pragma clang fp contract(off)
    const double sx = 1.0 - tx, sy = 1.0 - ty;
    double r = (sx * sy) * a;
    r = __builtin_fma(tx * sy, b, r);
    r = __builtin_fma(sx * ty, c, r);
    return __builtin_fma(tx * ty, d, r);
}

// Bilinear sample of the strip maps (see strip_rows): od is the offset of its density taps,
// og of its first gradient pair (the second is five pairs on); the same taps (clamped into the
// grid by the padding) and fractions as taps_of.
struct STap {
    uint32_t od, og;
    float tx, ty;
};

// The sample at (fx, fy) = (x - 1/2, y - 1/2) already inside [-1, W] x [-1, H].
__device__ __forceinline__ STap stap_at(float fx, float fy, int W, int H) {
    const float u0f = floorf(fx), v0f = floorf(fy);
    STap t;
    t.tx = fx - u0f;
    t.ty = fy - v0f;
    const uint32_t c = (uint32_t)(min((int)u0f, W - 1) + 1), r = (uint32_t)(min((int)v0f, H - 1) + 1);
    // grid sides are at most 8192, so the products fit the 24-bit multiplier
    const uint32_t s = r >> 2, k = r & 3u;
    t.od = ((__umul24(s, (uint32_t)W + 1u) + c) * 5u + k) * 2u;
    t.og = (__umul24(s, (uint32_t)W + 2u) + c) * 5u + k;
    return t;
}

__device__ __forceinline__ STap stap_of(float x, float y, int W, int H) {
    return stap_at(__builtin_amdgcn_fmed3f(x - 0.5f, -1.0f, (float)W),
                   __builtin_amdgcn_fmed3f(y - 0.5f, -1.0f, (float)H), W, H);
}

// The sample of a point already clamped into [0, W) x [0, H) (an advection candidate): the
// clamp of stap_of is then the identity and is left out.
__device__ __forceinline__ STap stap_inside(float x, float y, int W, int H) {
    return stap_at(x - 0.5f, y - 0.5f, W, H);
}

// Vector loads of 8-byte-aligned words: global loads of several dwords need only dword
// alignment.
typedef float hb_f4u __attribute__((ext_vector_type(4), aligned(8)));

// Density taps of a sample: one 16-byte load.
__device__ __forceinline__ Quad ld_rho(const HB_G float *m, uint32_t o) {
    const hb_f4u p = *(const HB_G hb_f4u *)(m + o);
    Quad r;
    r.a = p.x;
    r.b = p.y;
    r.c = p.z;
    r.d = p.w;
    return r;
}

// Gradient taps of a sample: two 16-byte loads, p = g(u0, v0), g(u0, v0 + 1) and
// q = g(u0 + 1, v0), g(u0 + 1, v0 + 1), (x, y) each.
__device__ __forceinline__ void ld_grad(const HB_G float2 *m, uint32_t o, Quad &p, Quad &q) {
    const hb_f4u a = *(const HB_G hb_f4u *)(m + o);
    const hb_f4u b = *(const HB_G hb_f4u *)(m + o + 5);
    p.a = a.x;
    p.b = a.y;
    p.c = a.z;
    p.d = a.w;
    q.a = b.x;
    q.b = b.y;
    q.c = b.z;
    q.d = b.w;
}

// Density sample from its taps, in FP32 (the precision of the stored map; the acceptance
// tests).
__device__ __forceinline__ float interp1q(const Quad &q, const STap &t) {
    return bilerp(q.a, q.b, q.c, q.d, t.tx, t.ty);
}

// Gradient sample from its taps (see ld_grad), in FP64: the direction of a small gradient
// between taps of opposite sign keeps the precision of the stored taps.
__device__ __forceinline__ void interp2q(const Quad &p, const Quad &q, const STap &t, double &gx,
                                         double &gy) {
    const double tx = t.tx, ty = t.ty;
    gx = bilerp((double)p.a, (double)q.a, (double)p.c, (double)q.c, tx, ty);
    gy = bilerp((double)p.b, (double)q.b, (double)p.d, (double)q.d, tx, ty);
}

}  // namespace hb
