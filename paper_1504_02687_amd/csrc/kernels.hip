// HIP kernels of the bundling iteration for gfx950 (CDNA4, wave64).
//
// Work shapes:
//   - point work runs one wavefront per edge, streaming the edge's points in chunks of
//     64 lanes (coalesced 8-byte loads/stores), with wave-level scans for arclength;
//   - map work runs one block per map row (row prefix sums in LDS) or one thread per
//     column segment (sliding column sums), coalesced along rows;
//   - every kernel takes an array of per-graph descriptors and finds its graph from
//     blockIdx, so a batch of graphs runs in one launch per stage.
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

__device__ __forceinline__ int64_t sample_count(double L, double delta) {
    double q = ceil(L / delta);
    if (!(q >= 1.0)) q = 1.0;          // also catches NaN
    if (q > 4.0e15) q = 4.0e15;
    return (int64_t)q + 1;
}

__device__ __forceinline__ double seg_len(float2 a, float2 b) {
    double dx = (double)b.x - (double)a.x, dy = (double)b.y - (double)a.y;
    return sqrt(dx * dx + dy * dy);
}

__device__ __forceinline__ void splat_point(int32_t *hist, int W, int H, float2 p, int w) {
    float fu = fminf(fmaxf(floorf(p.x), 0.0f), (float)(W - 1));
    float fv = fminf(fmaxf(floorf(p.y), 0.0f), (float)(H - 1));
    int u = (int)fu, v = (int)fv;
    atomicAdd(hist + (int64_t)v * W + u, w);
}

// ---------------------------------------------------------------- initial polylines

// Straight two-point polylines from the node positions, in pixel units, plus the
// lengths and first sample counts. One thread per edge.
__global__ __launch_bounds__(kBlock) void k_init_state(const GDesc *__restrict__ gd, int ng,
                                                       const float2 *__restrict__ nodes,
                                                       const int32_t *__restrict__ src,
                                                       const int32_t *__restrict__ dst,
                                                       double x0, double y0, double x1,
                                                       double y1) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_edget);
    const int64_t e = (blk - d.blk_edget) * kBlock + threadIdx.x;
    if (e > d.n_edges) return;
    if (e == d.n_edges) {
        d.off_s[e] = 2 * e;
        return;
    }
    float2 a = nodes[src[e]], b = nodes[dst[e]];
    float2 pa, pb;
    pa.x = (float)(((double)a.x - x0) / (x1 - x0) * (double)d.W);
    pa.y = (float)(((double)a.y - y0) / (y1 - y0) * (double)d.H);
    pb.x = (float)(((double)b.x - x0) / (x1 - x0) * (double)d.W);
    pb.y = (float)(((double)b.y - y0) / (y1 - y0) * (double)d.H);
    d.pnew[2 * e] = pa;
    d.pnew[2 * e + 1] = pb;
    d.off_s[e] = 2 * e;
    double L = seg_len(pa, pb);
    d.lens[e] = L;
    d.counts[e] = sample_count(L, d.delta);
}

// Lengths and next sample counts of the polylines (pin, off_in). One wave per edge.
__global__ __launch_bounds__(kBlock) void k_lengths(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_edge);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t e = (blk - d.blk_edge) * kWavesPerBlock + wid;
    if (e >= d.n_edges) return;
    const int64_t i0 = d.off_in[e], m = d.off_in[e + 1] - i0;
    const float2 *p = d.pin + i0;
    double L = 0.0;
    for (int64_t j0 = 0; j0 < m - 1; j0 += 64) {
        const int64_t j = j0 + lane;
        double s = 0.0;
        if (j < m - 1) s = seg_len(p[j], p[j + 1]);
        L += wave_sum(s);
    }
    if (lane == 0) {
        d.lens[e] = L;
        d.counts[e] = sample_count(L, d.delta);
    }
}

// ---------------------------------------------------------------- count scan -> offsets

__global__ __launch_bounds__(kBlock) void k_scan_tiles(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_scan);
    if (stopped(d)) return;
    const int64_t tile = blk - d.blk_scan;
    const int64_t base = tile * kScanTile;
    int64_t s = 0;
    for (int i = threadIdx.x; i < kScanTile; i += kBlock) {
        int64_t e = base + i;
        if (e < d.n_edges) s += d.counts[e];
    }
    int64_t tot;
    (void)block_excl_scan(s, &tot);
    if (threadIdx.x == 0) d.tsum[tile] = tot;
}

// One block per graph: exclusive scan of the tile sums, total and range checks.
__global__ __launch_bounds__(kBlock) void k_scan_top(const GDesc *__restrict__ gd, int ng) {
    const GDesc &d = gd[blockIdx.x];
    if (stopped(d)) return;
    const int64_t ntiles = (d.n_edges + kScanTile - 1) / kScanTile;
    int64_t carry = 0;
    for (int64_t t0 = 0; t0 < ntiles; t0 += kBlock) {
        int64_t t = t0 + threadIdx.x;
        int64_t v = t < ntiles ? d.tsum[t] : 0;
        int64_t tot;
        int64_t ex = block_excl_scan(v, &tot);
        if (t < ntiles) d.tsum[t] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        *d.total = carry;
        d.off_s[d.n_edges] = carry;
        int32_t st = 0;
        if (carry > d.cap) st |= ST_POINT_OVERFLOW;
        double wsum = (double)carry * (double)d.wmax;
        double grow = 1.0;
        for (int k = 1; k < d.P; ++k) grow *= (double)(2 * d.r + 1) * (double)(2 * d.r + 1);
        if (wsum >= 2147483647.0 || wsum * grow >= 9.2e18) st |= ST_HIST_OVERFLOW;
        if (st) atomicOr(d.status, st);
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_scan);
    if (stopped(d)) return;
    const int64_t tile = blk - d.blk_scan;
    const int64_t base = tile * kScanTile + (int64_t)threadIdx.x * 4;
    int64_t c[4];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int64_t e = base + i;
        c[i] = e < d.n_edges ? d.counts[e] : 0;
        s += c[i];
    }
    int64_t tot;
    int64_t ex = block_excl_scan(s, &tot) + d.tsum[tile];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int64_t e = base + i;
        if (e < d.n_edges) d.off_s[e] = ex;
        ex += c[i];
    }
}

// ---------------------------------------------------------------- resample + splat

// One wave per edge. The polyline (pin) is streamed in chunks of 64 segments; lane j of a
// chunk holds segment j, its FP64 length and the arclength at its start (wave scan). The
// samples whose arclength s_k = k L / (n-1) falls in the chunk are produced 64 at a time:
// each lane finds its segment by binary search in LDS and interpolates in FP64. Every
// sample is stored (coalesced, float2) and splatted into the group's histogram.
__global__ __launch_bounds__(kBlock) void k_resample_splat(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_edge);
    if (stopped(d)) return;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t e = (blk - d.blk_edge) * kWavesPerBlock + wid;
    if (e >= d.n_edges) return;

    __shared__ double sC[kWavesPerBlock][64];
    __shared__ float2 sP[kWavesPerBlock][65];

    const int64_t i0 = d.off_in[e], m = d.off_in[e + 1] - i0;
    const int64_t o0 = d.off_s[e], n = d.off_s[e + 1] - o0;
    const double L = d.lens[e];
    const float2 *p = d.pin + i0;
    float2 *q = d.samples + o0;
    const int W = d.W, H = d.H;
    int32_t *hist = d.hist + (int64_t)d.group[e] * W * H;
    const int w = d.weight ? d.weight[e] : 1;
    const double nm1 = (double)(n - 1);

    double Cbase = 0.0;
    int64_t knext = 0;
    for (int64_t j0 = 0; j0 < m - 1; j0 += 64) {
        const int nseg = (int)((m - 1 - j0) < 64 ? (m - 1 - j0) : 64);
        float2 a = make_float2(0.0f, 0.0f);
        if (lane <= nseg && lane < 64) a = p[j0 + lane];
        float2 b;
        b.x = __shfl_down(a.x, 1, 64);
        b.y = __shfl_down(a.y, 1, 64);
        if (lane == 63 && nseg == 64) b = p[j0 + 64];
        const double ell = lane < nseg ? seg_len(a, b) : 0.0;
        const double incl = wave_incl_scan<double>(ell, lane);
        double excl = __shfl_up(incl, 1, 64);
        if (lane == 0) excl = 0.0;
        if (lane < nseg) {
            sC[wid][lane] = Cbase + excl;
            sP[wid][lane] = a;
        }
        if (lane == nseg - 1) sP[wid][nseg] = b;
        const double Cend = Cbase + __shfl(incl, nseg - 1, 64);
        __builtin_amdgcn_wave_barrier();

        const bool last = (j0 + 64 >= m - 1);
        int64_t kend;
        if (last) {
            kend = n;
        } else if (!(L > 0.0)) {
            kend = knext;
        } else {
            double kf = ceil(Cend * nm1 / L);
            int64_t kk = kf < (double)knext ? knext : (kf > nm1 ? n - 1 : (int64_t)kf);
            while (kk > knext && (double)(kk - 1) * L / nm1 >= Cend) --kk;
            while (kk < n - 1 && (double)kk * L / nm1 < Cend) ++kk;
            kend = kk;
        }
        for (int64_t kb = knext; kb < kend; kb += 64) {
            const int64_t k = kb + lane;
            if (k < kend) {
                float2 out;
                if (k == 0) {
                    out = p[0];
                } else if (k == n - 1) {
                    out = p[m - 1];
                } else {
                    const double s = (double)k * L / nm1;
                    int lo = 0, hi = nseg - 1;
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (sC[wid][mid] <= s) lo = mid; else hi = mid - 1;
                    }
                    const float2 pa = sP[wid][lo], pb = sP[wid][lo + 1];
                    const double ex = (double)pb.x - (double)pa.x, ey = (double)pb.y - (double)pa.y;
                    const double el = sqrt(ex * ex + ey * ey);
                    double t = el > 0.0 ? (s - sC[wid][lo]) / el : 0.0;
                    t = fmin(fmax(t, 0.0), 1.0);
                    out.x = (float)((double)pa.x + t * ex);
                    out.y = (float)((double)pa.y + t * ey);
                }
                q[k] = out;
                splat_point(hist, W, H, out, w);
            }
        }
        __builtin_amdgcn_wave_barrier();
        knext = kend;
        Cbase = Cend;
    }
}

// Splat the given sample points (no resampling). One wave per edge.
__global__ __launch_bounds__(kBlock) void k_splat_given(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_edge);
    if (stopped(d)) return;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t e = (blk - d.blk_edge) * kWavesPerBlock + wid;
    if (e >= d.n_edges) return;
    const int64_t o0 = d.off_s[e], n = d.off_s[e + 1] - o0;
    int32_t *hist = d.hist + (int64_t)d.group[e] * d.W * d.H;
    const int w = d.weight ? d.weight[e] : 1;
    for (int64_t j = lane; j < n; j += 64) splat_point(hist, d.W, d.H, d.samples[o0 + j], w);
}

// ---------------------------------------------------------------- maps

__global__ __launch_bounds__(kBlock) void k_clear_hist(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_pxb);
    if (stopped(d)) return;
    const int64_t i = (blk - d.blk_pxb) * kBlock + threadIdx.x;
    if (i < (int64_t)d.B * d.W * d.H) d.hist[i] = 0;
}

// Row pass of one box filter: out(u) = sum of in(u') over |u'-u| <= r inside the row,
// from the row's prefix sums in LDS. One block per row of one group.
template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_box_rows(const GDesc *__restrict__ gd, int ng,
                                                     int pass) {
    extern __shared__ int64_t srow[];
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_row);
    if (stopped(d)) return;
    const int64_t row = blk - d.blk_row;
    const int W = d.W, r = d.r;
    const int64_t plane = (int64_t)d.B * d.W * d.H;
    const Tin *in = (pass == 0 ? (const Tin *)d.hist : (const Tin *)(d.box + (pass - 1) * plane)) +
                    row * W;
    for (int u = threadIdx.x; u < W; u += kBlock) srow[u] = (int64_t)in[u];
    __syncthreads();
    const int items = (W + kBlock - 1) / kBlock;
    const int beg = threadIdx.x * items;
    const int end = beg + items < W ? beg + items : W;
    int64_t run = 0;
    for (int u = beg; u < end; ++u) {
        run += srow[u];
        srow[u] = run;
    }
    int64_t tot;
    const int64_t ex = block_excl_scan(run, &tot);
    for (int u = beg; u < end; ++u) srow[u] += ex;
    __syncthreads();
    int64_t *out = d.tmp + row * W;
    for (int u = threadIdx.x; u < W; u += kBlock) {
        const int hi = u + r < W - 1 ? u + r : W - 1;
        const int lo = u - r - 1;
        out[u] = srow[hi] - (lo >= 0 ? srow[lo] : 0);
    }
}

// Column pass: sliding window sum down a column segment of kColSeg rows. One thread per
// (group, segment, column); neighbouring threads read neighbouring columns.
__global__ __launch_bounds__(kBlock) void k_box_cols(const GDesc *__restrict__ gd, int ng,
                                                     int pass) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_col);
    if (stopped(d)) return;
    const int W = d.W, H = d.H, r = d.r;
    const int nseg = (H + kColSeg - 1) / kColSeg;
    const int64_t t = (blk - d.blk_col) * kBlock + threadIdx.x;
    if (t >= (int64_t)d.B * nseg * W) return;
    const int u = (int)(t % W);
    const int64_t rest = t / W;
    const int seg = (int)(rest % nseg);
    const int64_t b = rest / nseg;
    const int64_t plane = (int64_t)W * H;
    const int64_t *in = d.tmp + b * plane + u;
    int64_t *out = d.box + (int64_t)pass * d.B * plane + b * plane + u;
    const int v0 = seg * kColSeg;
    const int v1 = v0 + kColSeg < H ? v0 + kColSeg : H;
    const int lo = v0 - r > 0 ? v0 - r : 0;
    const int hi = v0 + r < H - 1 ? v0 + r : H - 1;
    int64_t acc = 0;
    for (int v = lo; v <= hi; ++v) acc += in[(int64_t)v * W];
    out[(int64_t)v0 * W] = acc;
    for (int v = v0 + 1; v < v1; ++v) {
        if (v + r < H) acc += in[(int64_t)(v + r) * W];
        if (v - r - 1 >= 0) acc -= in[(int64_t)(v - r - 1) * W];
        out[(int64_t)v * W] = acc;
    }
}

// Density stack and its gradient in one pass. rho_l = sum_b M[l][b] * Sbar_b with
// Sbar_b = sum_k a_k S_b^k / (2r+1)^(2k), and the central-difference gradient of rho_l
// taken from exact int64 differences of the box sums (zero outside the grid), so the
// gradient keeps full relative precision where it is small compared with rho. Every sum
// runs in FP64; rho and the gradient are stored as FP32. One thread per pixel, layers in
// chunks of LCH accumulators.
template <int LCH>
__global__ __launch_bounds__(kBlock) void k_density_grad(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_px);
    if (stopped(d)) return;
    const int W = d.W, H = d.H;
    const int64_t plane = (int64_t)W * H;
    const int64_t px = (blk - d.blk_px) * kBlock + threadIdx.x;
    if (px >= plane) return;
    const int u = (int)(px % W), v = (int)(px / W);
    const bool hasl = u > 0, hasr = u + 1 < W, hasd = v > 0, hasu = v + 1 < H;
    const int B = d.B;
    for (int l0 = 0; l0 < B; l0 += LCH) {
        double rr[LCH], gx[LCH], gy[LCH];
#pragma unroll
        for (int l = 0; l < LCH; ++l) rr[l] = gx[l] = gy[l] = 0.0;
        for (int b = 0; b < B; ++b) {
            double sc = 0.0, sx = 0.0, sy = 0.0;
            for (int k = 0; k < d.P; ++k) {
                const double ak = d.a[k];
                if (ak == 0.0) continue;
                const int64_t *S = d.box + ((int64_t)k * B + b) * plane + px;
                const int64_t c0 = S[0];
                const int64_t xr = hasr ? S[1] : 0, xl = hasl ? S[-1] : 0;
                const int64_t yu = hasu ? S[W] : 0, yd = hasd ? S[-W] : 0;
                sc += ak * ((double)c0 / d.ck[k]);
                sx += ak * ((double)(xr - xl) / d.ck[k]);
                sy += ak * ((double)(yu - yd) / d.ck[k]);
            }
#pragma unroll
            for (int l = 0; l < LCH; ++l) {
                if (l0 + l < B) {
                    const double m = (double)d.M[(l0 + l) * B + b];
                    rr[l] += m * sc;
                    gx[l] += m * sx;
                    gy[l] += m * sy;
                }
            }
        }
#pragma unroll
        for (int l = 0; l < LCH; ++l) {
            if (l0 + l < B) {
                const int64_t i = (int64_t)(l0 + l) * plane + px;
                d.rho[i] = (float)rr[l];
                d.grad[i] = make_float2((float)(0.5 * gx[l]), (float)(0.5 * gy[l]));
            }
        }
    }
}

// ---------------------------------------------------------------- advection + smoothing

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

// Density sample for the acceptance test, in FP32 (the precision of the stored map).
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

// One wave per edge, chunks of 62 output points with a one-point halo on each side: lane
// l of a chunk advects point j0 - 1 + l (end points stay), neighbours come from lanes l-1
// and l+1, and lanes 1..62 write the Laplacian-smoothed point. The FP64 polyline length
// of the smoothed edge gives the next sample count.
__global__ __launch_bounds__(kBlock) void k_advect_smooth(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_edge);
    if (stopped(d)) return;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t e = (blk - d.blk_edge) * kWavesPerBlock + wid;
    if (e >= d.n_edges) return;

    const int W = d.W, H = d.H;
    const int64_t plane = (int64_t)W * H;
    const int64_t o0 = d.off_s[e], n = d.off_s[e + 1] - o0;
    const int64_t lay = (int64_t)d.group[e] * plane;
    const float *__restrict__ rho = d.rho + lay;
    const float2 *__restrict__ grad = d.grad + lay;
    const float2 *__restrict__ xs = d.samples + o0;
    float2 *__restrict__ ys = d.pnew + o0;
    const double h = d.h, s = d.s;
    const double eps = d.eps;
    const int K = d.K;
    const double xmax = (double)W - 1.0 / 256.0, ymax = (double)H - 1.0 / 256.0;

    double L = 0.0;
    float2 yprev = make_float2(0.0f, 0.0f);
    for (int64_t j0 = 0; j0 < n; j0 += 62) {
        const int64_t j = j0 - 1 + lane;
        const bool inr = j >= 0 && j < n;
        float2 x = make_float2(0.0f, 0.0f);
        if (inr) x = xs[j];
        double ax = x.x, ay = x.y;
        int jj = -2;
        if (inr && j > 0 && j < n - 1) {
            const Bilin t0 = bilin_taps(ax, ay, W, H);
            double gx, gy;
            bilin2(grad, t0, gx, gy);
            const double nrm = sqrt(gx * gx + gy * gy);
            const double den = nrm > eps ? nrm : eps;
            const double dx = gx / den, dy = gy / den;
            const float r0 = bilin1(rho, t0);
            double m = h;
            jj = -1;
            for (int k = 0; k <= K; ++k) {
                const double cx = fmin(fmax((double)x.x + m * dx, 0.0), xmax);
                const double cy = fmin(fmax((double)x.y + m * dy, 0.0), ymax);
                const float r1 = bilin1(rho, bilin_taps(cx, cy, W, H));
                if (r1 >= r0) {
                    ax = cx;
                    ay = cy;
                    jj = k;
                    break;
                }
                m *= 0.5;
            }
        }
        const double lx = __shfl_up(ax, 1, 64), ly = __shfl_up(ay, 1, 64);
        const double rx = __shfl_down(ax, 1, 64), ry = __shfl_down(ay, 1, 64);
        const bool out = lane >= 1 && lane <= 62 && j < n;
        float2 y = x;
        if (out && j > 0 && j < n - 1) {
            y.x = (float)((1.0 - s) * ax + 0.5 * s * (lx + rx));
            y.y = (float)((1.0 - s) * ay + 0.5 * s * (ly + ry));
        }
        if (out) {
            ys[j] = y;
            if (d.record) d.jacc[o0 + j] = (int8_t)jj;
        }
        float2 yl;
        yl.x = __shfl_up(y.x, 1, 64);
        yl.y = __shfl_up(y.y, 1, 64);
        if (lane == 1) yl = yprev;
        const double sl = (out && j >= 1) ? seg_len(yl, y) : 0.0;
        L += wave_sum(sl);
        yprev.x = __shfl(y.x, 62, 64);
        yprev.y = __shfl(y.y, 62, 64);
    }
    if (lane == 0) {
        d.lens[e] = L;
        d.counts[e] = sample_count(L, d.delta);
    }
}

// ---------------------------------------------------------------- launchers

Shape shape_of(int64_t n_edges, int32_t B, int32_t W, int32_t H) {
    Shape s;
    const int64_t plane = (int64_t)W * H;
    const int64_t nseg = (H + kColSeg - 1) / kColSeg;
    s.edge = (n_edges + kWavesPerBlock - 1) / kWavesPerBlock;
    s.scan = (n_edges + kScanTile - 1) / kScanTile;
    s.row = (int64_t)B * H;
    s.col = ((int64_t)B * nseg * W + kBlock - 1) / kBlock;
    s.px = (plane + kBlock - 1) / kBlock;
    s.pxb = ((int64_t)B * plane + kBlock - 1) / kBlock;
    s.edget = (n_edges + 1 + kBlock - 1) / kBlock;
    return s;
}

static inline dim3 grid_of(int64_t blocks) { return dim3((unsigned)(blocks > 0 ? blocks : 0)); }

hipError_t launch_init_state(const GDesc *desc, int ng, const Shape &tot, const float2 *nodes,
                             const int32_t *src, const int32_t *dst, double x0, double y0,
                             double x1, double y1, hipStream_t st) {
    if (tot.edget <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_state, grid_of(tot.edget), dim3(kBlock), 0, st, desc, ng, nodes,
                       src, dst, x0, y0, x1, y1);
    return hipGetLastError();
}

hipError_t launch_lengths(const GDesc *desc, int ng, const Shape &tot, hipStream_t st) {
    if (tot.edge <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lengths, grid_of(tot.edge), dim3(kBlock), 0, st, desc, ng);
    return hipGetLastError();
}

hipError_t launch_scan(const GDesc *desc, int ng, const Shape &tot, hipStream_t st) {
    if (tot.scan > 0)
        hipLaunchKernelGGL(k_scan_tiles, grid_of(tot.scan), dim3(kBlock), 0, st, desc, ng);
    hipLaunchKernelGGL(k_scan_top, dim3(ng), dim3(kBlock), 0, st, desc, ng);
    if (tot.scan > 0)
        hipLaunchKernelGGL(k_scan_apply, grid_of(tot.scan), dim3(kBlock), 0, st, desc, ng);
    return hipGetLastError();
}

hipError_t launch_resample_splat(const GDesc *desc, int ng, const Shape &tot, hipStream_t st) {
    if (tot.edge <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_resample_splat, grid_of(tot.edge), dim3(kBlock), 0, st, desc, ng);
    return hipGetLastError();
}

hipError_t launch_splat_given(const GDesc *desc, int ng, const Shape &tot, hipStream_t st) {
    if (tot.edge <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_splat_given, grid_of(tot.edge), dim3(kBlock), 0, st, desc, ng);
    return hipGetLastError();
}

hipError_t launch_clear_hist(const GDesc *desc, int ng, const Shape &tot, hipStream_t st) {
    if (tot.pxb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear_hist, grid_of(tot.pxb), dim3(kBlock), 0, st, desc, ng);
    return hipGetLastError();
}

hipError_t launch_box_pass(const GDesc *desc, int ng, const Shape &tot, int max_w, int pass,
                           hipStream_t st) {
    const size_t lds = sizeof(int64_t) * (size_t)max_w;
    if (pass == 0)
        hipLaunchKernelGGL(k_box_rows<int32_t>, grid_of(tot.row), dim3(kBlock), lds, st, desc,
                           ng, pass);
    else
        hipLaunchKernelGGL(k_box_rows<int64_t>, grid_of(tot.row), dim3(kBlock), lds, st, desc,
                           ng, pass);
    hipLaunchKernelGGL(k_box_cols, grid_of(tot.col), dim3(kBlock), 0, st, desc, ng, pass);
    return hipGetLastError();
}

hipError_t launch_density_grad(const GDesc *desc, int ng, const Shape &tot, int bmax,
                               hipStream_t st) {
    dim3 gr = grid_of(tot.px), bl(kBlock);
    if (bmax <= 1) hipLaunchKernelGGL(k_density_grad<1>, gr, bl, 0, st, desc, ng);
    else if (bmax <= 2) hipLaunchKernelGGL(k_density_grad<2>, gr, bl, 0, st, desc, ng);
    else if (bmax <= 4) hipLaunchKernelGGL(k_density_grad<4>, gr, bl, 0, st, desc, ng);
    else if (bmax <= 8) hipLaunchKernelGGL(k_density_grad<8>, gr, bl, 0, st, desc, ng);
    else hipLaunchKernelGGL(k_density_grad<16>, gr, bl, 0, st, desc, ng);
    return hipGetLastError();
}

hipError_t launch_advect_smooth(const GDesc *desc, int ng, const Shape &tot, hipStream_t st) {
    if (tot.edge <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_advect_smooth, grid_of(tot.edge), dim3(kBlock), 0, st, desc, ng);
    return hipGetLastError();
}

}  // namespace hb
