// Adjoint of one bundling iteration with the discrete choices of the forward run held
// fixed: the sample counts and the segment each sample is interpolated on (resampling), the
// histograms (so the int64 box sums are constants), and the accepted halving of every point
// (advection). With those frozen the iteration is a piecewise smooth function of the point
// positions, of the interaction matrix M and of the pass weights a (density of Section 3.2
// Eq. 3, advection of Section 3.3 Eq. 5, Laplacian smoothing of Section 3.3); these kernels
// apply its transposed Jacobian.
//
// The density gradient seen by a point of layer l is
//   g_l(x) = bilinear( sum_b M[l][b] sum_k a_k G_bk , x ),  G_bk = grad(S_b^k) / (2r+1)^(2k),
// so dL/dM and dL/da are contractions of m v (step times direction adjoint) at the moved
// points with bilinear samples of the maps G_bk. They are summed tile by tile: m v is splatted
// with the bilinear weights into LDS as 64-bit fixed point (exact in any order) and the
// splat is contracted with the maps; every floating-point reduction runs in a fixed order,
// so the results are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace hb {

// Gradient maps the parameter gradients gather, from exact int64 differences of the box
// sums (zero outside the grid), with D_bk = 1/2 grad(S_b^k) / (2r+1)^(2k):
//   gb[b]    = sum_k a_k D_bk        dL/dM[l][b] = sum over moved points of layer l of
//                                    m v . bilinear(gb[b])
//   gl[l][k] = sum_b M[l][b] D_bk    dL/da_k     = sum over moved points of layer l of
//                                    m v . bilinear(gl[l][k])
// gb does not depend on the layer: one record of B float2 per pixel serves every layer, and
// layer l has its own record of P float2 per pixel (records padded to 16-byte multiples, so a
// bilinear tap is a few 16-byte loads). One thread per pixel, all layers.
template <int BMAX>
__global__ __launch_bounds__(kBlock) void k_adj_maps(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_px);
    const int W = d.W, H = d.H, B = d.B, P = d.P, bp = d.bp, pp = d.pp;
    const int64_t plane = (int64_t)W * H;
    const int64_t px = (blk - d.blk_px) * kBlock + threadIdx.x;
    if (px >= plane) return;
    const int u = (int)(px % W), v = (int)(px / W);
    const bool hasr = u + 1 < W, hasl = u > 0, hasu = v + 1 < H, hasd = v > 0;
    float2 *gb = d.gbm + px * bp;
    float gbx[BMAX], gby[BMAX];
#pragma unroll
    for (int b = 0; b < BMAX; ++b) gbx[b] = gby[b] = 0.0f;
    for (int l = 0; l < B; ++l)
        for (int k = P; k < pp; ++k) d.gkm[((int64_t)l * plane + px) * pp + k] = make_float2(0.0f, 0.0f);
    for (int k = 0; k < P; ++k) {
        // D_bk of every group at this pixel, read once per pass
        double dxs[BMAX], dys[BMAX];
#pragma unroll
        for (int b = 0; b < BMAX; ++b) {
            dxs[b] = dys[b] = 0.0;
            if (b < B) {
                const int64_t *S = d.box + ((int64_t)k * B + b) * plane + px;
                const int64_t xr = hasr ? S[1] : 0, xl = hasl ? S[-1] : 0;
                const int64_t yu = hasu ? S[W] : 0, yd = hasd ? S[-W] : 0;
                dxs[b] = 0.5 * ((double)(xr - xl) / d.ck[k]);
                dys[b] = 0.5 * ((double)(yu - yd) / d.ck[k]);
                if (d.a[k] != 0.0) {
                    gbx[b] = (float)((double)gbx[b] + d.a[k] * dxs[b]);
                    gby[b] = (float)((double)gby[b] + d.a[k] * dys[b]);
                }
            }
        }
        for (int l = 0; l < B; ++l) {
            double ax = 0.0, ay = 0.0;
#pragma unroll
            for (int b = 0; b < BMAX; ++b) {
                if (b < B) {
                    const double mlb = (double)d.M[l * B + b];
                    ax += mlb * dxs[b];
                    ay += mlb * dys[b];
                }
            }
            d.gkm[((int64_t)l * plane + px) * pp + k] = make_float2((float)ax, (float)ay);
        }
    }
#pragma unroll
    for (int b = 0; b < BMAX; ++b)
        if (b < bp) gb[b] = make_float2(b < B ? gbx[b] : 0.0f, b < B ? gby[b] : 0.0f);
}

// Transposed Laplacian smoothing and advection, fused. One wave per edge, chunks of 62
// points with a one-point halo (like the forward): with y_bar the adjoint of the smoothed
// points (adj_in), lane l computes the adjoint x'_bar of the advected point j from y_bar of
// j-1, j, j+1, then the adjoint of the sample x_bar = w + m (dg/dx)^T v, where w is x'_bar
// without the clamped coordinates, v = (dd/dg)^T w with d = g / max(|g|, eps), and m the
// frozen step h / 2^j. m v is stored for every sample (zero where the sample did not move):
// the parameter gradients are its contractions with the gradient maps (k_adj_params); mvmax
// gets its largest component.
__global__ __launch_bounds__(kBlock) void k_adj_advect(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_edge);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // edges in the given order (by group, then position), dealt round-robin: the blocks in
    // flight work on one or two layers of the maps
    const int64_t idx = (blk - d.blk_edge) * kWavesPerBlock + wid;
    if (idx >= d.n_edges) return;
    const int64_t e = d.order ? (int64_t)d.order[idx] : idx;

    const int W = d.W, H = d.H;
    const int64_t plane = (int64_t)W * H;
    const int64_t o0 = d.off_s[e], n = d.off_s[e + 1] - o0;
    const int l = d.group[e];
    (void)plane;
    const HB_G float2 *__restrict__ grad = glb(d.grads + (int64_t)l * grad_strip_plane(W, H));
    const HB_G float2 *__restrict__ xs = glb(d.samples + o0);
    HB_G float2 *__restrict__ xb = glb(d.adj_out + o0);
    HB_G float2 *__restrict__ mvp = glb(d.mv + o0);
    const HB_G int8_t *__restrict__ jv = glb(d.jacc + o0);
    // the output polylines are the final ones when ink_pts is set: y_bar_j = u_(j-1) - u_j,
    // u the unit vectors of the adjacent segments (the gradient of the ink)
    const bool ink = d.ink_pts != nullptr;
    const HB_G float2 *__restrict__ pp = glb((ink ? d.ink_pts : d.adj_in) + o0);
    const double h = d.h, s = d.s, eps = d.eps;
    const double xmax = (double)W - 1.0 / 256.0, ymax = (double)H - 1.0 / 256.0;

    // loads of one trip (lane l: point j0 - 1 + l), which do not depend on the arithmetic of
    // the trip before: the decision, the sample, and y_bar or the final point (lane 63 also
    // the final point after the chunk, lane 0 the one before it)
    struct Base {
        int8_t jr;
        float2 x, y, pn, pl;
    };
    auto load = [&](int64_t j0) {
        Base b;
        const int64_t j = j0 - 1 + lane;
        b.jr = -2;
        b.x = b.y = b.pn = b.pl = make_float2(0.0f, 0.0f);
        if (j >= 0 && j < n) {
            b.jr = jv[j];
            b.x = ld2(xs + j);
            b.y = ld2(pp + j);
            if (ink && lane == 0 && j >= 1) b.pl = ld2(pp + (j - 1));
            if (ink && lane == 63 && j + 1 < n) b.pn = ld2(pp + (j + 1));
        }
        return b;
    };

    float mbig = 0.0f;
    // one trip of 62 output points from the loads cu; it issues the loads of the trip after it
    // into nx (none past the edge's end)
    auto trip = [&](int64_t j0, const Base &cu, Base &nx) {
        const int64_t j = j0 - 1 + lane;
        const bool inr = j >= 0 && j < n;
        const bool interior = inr && j > 0 && j < n - 1;
        const bool out = lane >= 1 && lane <= 62 && j < n;
        const int jj = interior ? (int)cu.jr : -2;
        // the gradient taps of a moved sample go out first, then the next trip's loads, so
        // both are in flight during this trip's arithmetic
        STap t0;
        Quad q0, q1;
        if (out && jj >= 0) {
            t0 = stap_of(cu.x.x, cu.x.y, W, H);
            ld_grad(grad, t0.og, q0, q1);
        }
        nx = load(j0 + 62);
        float2 ybar = cu.y;
        if (ink) {
            const float2 c = cu.y;
            float nxx = lane_next(c.x), nxy = lane_next(c.y);
            if (lane == 63) {
                nxx = cu.pn.x;
                nxy = cu.pn.y;
            }
            // unit vectors from the segment's reciprocal length (0 for a zero-length segment)
            double ux = 0.0, uy = 0.0;
            if (inr && j + 1 < n) {
                double l, r;
                seg_len_rcp(c, make_float2(nxx, nxy), l, r);
                ux = ((double)nxx - c.x) * r;
                uy = ((double)nxy - c.y) * r;
            }
            double pux = lane_prev(ux), puy = lane_prev(uy);
            if (lane == 0) {
                pux = puy = 0.0;
                if (inr && j >= 1) {
                    const float2 a = cu.pl;
                    double l, r;
                    seg_len_rcp(a, c, l, r);
                    pux = ((double)c.x - a.x) * r;
                    puy = ((double)c.y - a.y) * r;
                }
            }
            ybar = inr ? make_float2((float)(pux - ux), (float)(puy - uy)) : make_float2(0.0f, 0.0f);
        }
        const double qx = interior ? (double)ybar.x : 0.0, qy = interior ? (double)ybar.y : 0.0;
        const double qlx = lane_prev(qx), qly = lane_prev(qy);
        const double qrx = lane_next(qx), qry = lane_next(qy);
        if (!out) return;
        const double cf = interior ? 1.0 - s : 1.0;
        double wx = cf * (double)ybar.x + 0.5 * s * (qlx + qrx);
        double wy = cf * (double)ybar.y + 0.5 * s * (qly + qry);
        double gxb = wx, gyb = wy;
        float2 mvv = make_float2(0.0f, 0.0f);
        if (jj >= 0) {
            const float2 x = cu.x;
            const float2 g00 = make_float2(q0.a, q0.b), g01 = make_float2(q0.c, q0.d);
            const float2 g10 = make_float2(q1.a, q1.b), g11 = make_float2(q1.c, q1.d);
            double gx, gy;
            interp2q(q0, q1, t0, gx, gy);   // the forward's bilinear gradient sample
            // 1 / max(|g|, eps) for d and v (reciprocal square root and a Newton step)
            const double q = gx * gx + gy * gy;
            const bool big = q > eps * eps;
            const double inv = big ? rsqrt_nr(q) : 1.0 / eps;
            const double dx = gx * inv, dy = gy * inv;
            const double m = ldexp(h, -jj);
            const double cx = (double)x.x + m * dx, cy = (double)x.y + m * dy;
            if (cx < 0.0 || cx > xmax) wx = 0.0;
            if (cy < 0.0 || cy > ymax) wy = 0.0;
            double vx, vy;
            if (big) {
                const double dw = dx * wx + dy * wy;
                vx = (wx - dx * dw) * inv;
                vy = (wy - dy * dw) * inv;
            } else {
                vx = wx * inv;
                vy = wy * inv;
            }
            const double v00 = g00.x * vx + g00.y * vy, v10 = g10.x * vx + g10.y * vy;
            const double v01 = g01.x * vx + g01.y * vy, v11 = g11.x * vx + g11.y * vy;
            const double tx = t0.tx, ty = t0.ty;
            gxb = wx + m * ((1.0 - ty) * (v10 - v00) + ty * (v11 - v01));
            gyb = wy + m * ((1.0 - tx) * (v01 - v00) + tx * (v11 - v10));
            mvv = make_float2((float)(m * vx), (float)(m * vy));
            mbig = fmaxf(mbig, fmaxf(fabsf(mvv.x), fabsf(mvv.y)));
        }
        st2(xb + j, make_float2((float)gxb, (float)gyb));
        st2(mvp + j, mvv);
    };
    // two trips per turn with the two load buffers alternating: the next trip's loads are in
    // flight during this trip's arithmetic, with no register copies that would wait for them
    Base ba = load(0), bb;
    for (int64_t j0 = 0; j0 < n; j0 += 124) {
        trip(j0, ba, bb);
        if (j0 + 62 >= n) break;
        trip(j0 + 62, bb, ba);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mbig = fmaxf(mbig, __shfl_xor(mbig, o, 64));
    if (lane == 0 && mbig > 0.0f) atomicMax(d.mvmax, __float_as_uint(mbig));
}

// The nearest integer of v (ties to even; |v| < 2^51) as a two's-complement 64-bit value: v
// (exact in FP64) plus 1.5 * 2^52 keeps its integer part in the low bits of the mantissa.
__device__ __forceinline__ unsigned long long fixed64(float v) {
    const double t = (double)v + 6755399441055744.0;
    return (unsigned long long)(__double_as_longlong(t) - 0x4338000000000000ll);
}

// Threads of a k_adj_params block: its (64 + 2)^2 LDS grid of two 64-bit sums (70 KB) allows
// two blocks per CU, so a block of eight waves keeps sixteen waves per CU in flight.
constexpr int kParBlock = 512;
constexpr int kParWaves = kParBlock / 64;

// Parameter gradients, tile by tile. A moved sample p contributes m v_p . g(x_p), g the
// bilinear sample of a gradient-map record (Eq. 3 differentiated with respect to M and a);
// summed by pixel instead, that is the sum over pixels of A(px) . record(px), with
// A(px) = sum over samples of w_px(x_p) m v_p. A block takes work items of the iteration's
// checkpointed tile bins (up to kSegEntries samples of one tile), adds w m v into a
// (64 + 2)^2 LDS grid (the tile and a one-pixel border, where the taps of its samples fall)
// as 64-bit fixed point with unit 2^-S, max |m v| 2^S < 2^40 (exact sums in any order), then
// contracts the grid with the records in FP64 and writes the item's B + P partial sums; all
// reductions run in a fixed order, so the gradients are bit-reproducible.
template <int BMAX>
__global__ __launch_bounds__(kParBlock) void k_adj_params(const GDesc *__restrict__ gd, int ng) {
    const GDesc &d = gd[0];
    constexpr int GW = kTile + 2, GN = GW * GW, NQ = BMAX + HB_MAX_PASSES;
    __shared__ unsigned long long sA[2][GN];
    __shared__ double sred[kParWaves][NQ];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nt = d.n_tiles, B = d.B, P = d.P, W = d.W, H = d.H, bp = d.bp, pp = d.pp;
    const int64_t nitems = d.aseg_off[nt];
    const int64_t plane = (int64_t)W * H;
    const int per_layer = d.tiles_x * d.tiles_y;
    const float mmax = __uint_as_float(*d.mvmax);
    int ex = 0;
    if (mmax > 0.0f) (void)frexpf(mmax, &ex);
    const float scale = ldexpf(1.0f, 40 - ex);
    const double unit = ldexp(1.0, ex - 40);
    const HB_G int64_t *__restrict__ aseg = glb(d.aseg_off);
    const HB_G uint32_t *__restrict__ src = glb(d.abin_src);
    const HB_G float2 *__restrict__ mvs = glb(d.mv);
    const HB_G float2 *__restrict__ xs = glb(d.samples);
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        int lo = 0, hi = nt - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (aseg[mid] <= it) lo = mid; else hi = mid - 1;
        }
        const int t = lo;
        const int64_t beg = d.atile_off[t] + (it - d.aseg_off[t]) * d.item_entries;
        const int64_t lim = d.atile_off[t + 1];
        const int64_t end = beg + d.item_entries < lim ? beg + d.item_entries : lim;
        const int layer = t / per_layer, rem = t - layer * per_layer;
        const int ty = rem / d.tiles_x, tx = rem - ty * d.tiles_x;
        const int X0 = tx * kTile - 1, Y0 = ty * kTile - 1;   // grid cell (0, 0)
        for (int c = threadIdx.x; c < 2 * GN; c += kParBlock) (&sA[0][0])[c] = 0ull;
        __syncthreads();
        // four entries per thread in flight: every index load, then every gather of m v and
        // x (an entry past the item's end reads the item's first entry and is dropped)
        for (int64_t i0 = beg + threadIdx.x; i0 < end; i0 += 4 * kParBlock) {
            uint32_t pe[4];
            bool ok[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + r * kParBlock;
                ok[r] = i < end;
                pe[r] = src[ok[r] ? i : beg];
            }
            float2 me[4], xe[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                me[r] = ld2(mvs + pe[r]);
                xe[r] = ld2(xs + pe[r]);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float2 m = me[r], x = xe[r];
                if (!ok[r] || (m.x == 0.0f && m.y == 0.0f)) continue;
                const Taps tp = taps_of(x.x, x.y, W, H);
                const float ftx = tp.tx, fty = tp.ty;
                const float w[4] = {(1.0f - ftx) * (1.0f - fty), ftx * (1.0f - fty),
                                    (1.0f - ftx) * fty, ftx * fty};
                // grid cells of the taps (ua, va), (ub, va), (ua, vb), (ub, vb): rows and
                // columns within [0, GW) of the tile's grid
                const int ca = __mul24(tp.va - Y0, GW) - X0, cb = __mul24(tp.vb - Y0, GW) - X0;
                const int cq[4] = {ca + tp.ua, ca + tp.ub, cb + tp.ua, cb + tp.ub};
                const float mx = m.x * scale, my = m.y * scale;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int c = cq[q];
                    atomicAdd(&sA[0][c], fixed64(w[q] * mx));
                    atomicAdd(&sA[1][c], fixed64(w[q] * my));
                }
            }
        }
        __syncthreads();
        double acc[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
        for (int c = threadIdx.x; c < GN; c += kParBlock) {
            const long long ax = (long long)sA[0][c], ay = (long long)sA[1][c];
            if (ax == 0 && ay == 0) continue;
            const int v = Y0 + c / GW, u = X0 + c % GW;
            const int64_t px = (int64_t)v * W + u;
            const double fx = (double)ax * unit, fy = (double)ay * unit;
            const HB_G float2 *gb = glb(d.gbm) + px * bp;
            const HB_G float2 *gk = glb(d.gkm) + ((int64_t)layer * plane + px) * pp;
#pragma unroll
            for (int b = 0; b < BMAX; ++b) {
                if (b >= B) break;
                const float2 g = ld2(gb + b);
                acc[b] += fx * g.x + fy * g.y;
            }
#pragma unroll
            for (int k = 0; k < HB_MAX_PASSES; ++k) {
                if (k >= P) break;
                const float2 g = ld2(gk + k);
                acc[BMAX + k] += fx * g.x + fy * g.y;
            }
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const bool used = q < BMAX ? q < B : q - BMAX < P;
            if (!used) continue;
            const double v = wave_sum(acc[q]);
            if (lane == 0) sred[wid][q] = v;
        }
        __syncthreads();
        if ((int)threadIdx.x < B + P) {
            const int q = (int)threadIdx.x < B ? (int)threadIdx.x : BMAX + ((int)threadIdx.x - B);
            double sum = 0.0;
            for (int w2 = 0; w2 < kParWaves; ++w2) sum += sred[w2][q];
            d.partials[(int64_t)threadIdx.x * d.max_items + it] = sum;
        }
        __syncthreads();
    }
}

// Transposed resampling. Sample k of an edge is x_k = p_j + t (p_(j+1) - p_j) with
// t = (k L/(n-1) - C_j) / l_j, C_j the arclength at p_j, l_j the segment length and L the
// polyline length; the end points are copies. One wave per edge, two passes:
//  A) chunks of 64 segments as in the forward; the samples of a chunk add (1-t) x_bar and
//     t x_bar to the segment's end points and -t_bar/l, -t_bar t/l to C_bar_j and l_bar_j
//     (segmented scans over the lanes, in a fixed order); each point's adjoint is written
//     from its two segments, with everything except the terms proportional to L_bar and
//     to the total of C_bar, which are only known at the end of the edge;
//  B) add (L_bar + sum_j C_bar_j)(u_(i-1) - u_i) to every point (u: unit segment vectors).
// Point i is always handled by lane i mod 64, so pass B re-reads only its own writes.
__global__ __launch_bounds__(kBlock, 6) void k_adj_resample(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_edge);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t e = (blk - d.blk_edge) * kWavesPerBlock + wid;
    if (e >= d.n_edges) return;

    __shared__ double sC[kWavesPerBlock][64];
    __shared__ double sR[kWavesPerBlock][64];
    __shared__ float2 sP[kWavesPerBlock][65];
    __shared__ double acc[kWavesPerBlock][6][64];

    // per-edge point and sample counts are below 2^31 (checked by the count scan)
    const int64_t i0 = d.off_in[e], o0 = d.off_s[e];
    const int m = (int)(d.off_in[e + 1] - i0), n = (int)(d.off_s[e + 1] - o0);
    const double L = d.lens[e];
    const HB_G float2 *p = glb(d.pin + i0);
    const HB_G float2 *xb = glb(d.adj_in + o0);
    HB_G float2 *pb = glb(d.adj_out + i0);
    const double nm1 = (double)(n - 1);
    const double ds = L / nm1;
    const double inv_ds = 1.0 / ds;
    const double inv_nm1 = 1.0 / nm1;   // d s_k / d L = k / (n - 1)

    double Cbase = 0.0, Lbar = 0.0, carryP = 0.0;
    double carryBx = 0.0, carryBy = 0.0, carryVx = 0.0, carryVy = 0.0;
    int knext = 0;
    for (int j0 = 0; j0 < m - 1; j0 += 64) {
        const int rem = m - 1 - j0;
        const int nseg = rem < 64 ? rem : 64;
        float2 a = make_float2(0.0f, 0.0f);
        if (lane <= nseg && lane < 64) a = ld2(p + (j0 + lane));
        float2 b;
        b.x = lane_next(a.x);
        b.y = lane_next(a.y);
        if (lane == 63 && nseg == 64) b = ld2(p + (j0 + 64));
        double ell, rcp;
        seg_len_rcp(a, b, ell, rcp);
        if (lane >= nseg) ell = 0.0;
        const double incl = wave_incl_scan<double>(ell, lane);
        const double excl = lane_prev(incl);
        // arclengths past the chunk's last segment read as +inf (no bound check in the search)
        sC[wid][lane] = lane < nseg ? Cbase + excl : __builtin_huge_val();
        if (lane < nseg) {
            sR[wid][lane] = rcp;
            sP[wid][lane] = a;
            for (int c = 0; c < 6; ++c) acc[wid][c][lane] = 0.0;
        }
        if (lane == nseg - 1) sP[wid][nseg] = b;
        const double Cend = Cbase + last_lane(incl);
        __builtin_amdgcn_wave_barrier();

        const bool last = (j0 + 64 >= m - 1);
        int kend;
        if (last) {
            kend = n;
        } else if (!(L > 0.0)) {
            kend = knext;
        } else {
            const double kf = ceil(Cend * inv_ds);     // corrected by the exact tests below
            int kk = kf < (double)knext ? knext : (kf > nm1 ? n - 1 : (int)kf);
            while (kk > knext && (double)(kk - 1) * ds >= Cend) --kk;
            while (kk < n - 1 && (double)kk * ds < Cend) ++kk;
            kend = kk;
        }
        if (j0 == 0 && kend < 1) kend = 1;   // the first end point belongs to point 0
        for (int kb = knext; kb < kend; kb += 64) {
            const int k = kb + lane;
            const bool valid = k < kend;
            int jl = 64 + lane;   // distinct keys for idle lanes
            double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            if (valid) {
                const float2 xv = ld2(xb + k);
                double t = 0.0, tb = 0.0;
                if (k == 0) {
                    jl = 0;
                } else if (k == n - 1) {
                    jl = nseg - 1;
                    t = 1.0;
                } else {
                    const double sk = mul_rn((double)k, ds);
                    // last segment that starts at or before sk (binary search; lo + step < 64)
                    int lo = 0;
#pragma unroll
                    for (int step = 32; step >= 1; step >>= 1)
                        lo = sC[wid][lo + step] <= sk ? lo + step : lo;
                    jl = lo;
                    const double traw = mul_rn(sub_rn(sk, sC[wid][lo]), sR[wid][lo]);
                    t = fmin(fmax(traw, 0.0), 1.0);
                    if (traw > 0.0 && traw < 1.0 && sR[wid][lo] > 0.0) {
                        const float2 pa = sP[wid][lo], pz = sP[wid][lo + 1];
                        tb = xv.x * ((double)pz.x - pa.x) + xv.y * ((double)pz.y - pa.y);
                        Lbar += tb * sR[wid][lo] * ((double)k * inv_nm1);
                    }
                }
                v[0] = (1.0 - t) * xv.x;
                v[1] = (1.0 - t) * xv.y;
                v[2] = t * xv.x;
                v[3] = t * xv.y;
                v[4] = -tb * sR[wid][jl];
                v[5] = -tb * t * sR[wid][jl];
            }
            // per-segment sums: runs of equal segment index are contiguous lanes (the index
            // grows with the sample; idle lanes carry larger, distinct keys). Runs of one or two
            // samples (segments about as long as the sampling step) take one lane shift;
            // longer runs the difference of plain inclusive wave sums at the run's last lane
            // and before its first. (Lane moves run on every lane: a DPP read from a disabled
            // lane is not defined.)
            const int jprev = lane_prev(jl, -1), jnext = lane_next(jl, -1);
            const uint64_t heads = __ballot(lane == 0 || jprev != jl);
            const bool tail = lane == 63 || jnext != jl;
            if ((heads | (heads << 1) | 1ull) == ~0ull) {
                // every lane is a head or directly follows one: runs of length <= 2
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    const double pv = lane_prev(v[c]);
                    if (jprev == jl) v[c] += pv;
                }
            } else {
                const int hd = run_head(heads, lane);
                const int src = (hd > 0 ? hd - 1 : 0) * 4;
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    const double pc = wave_incl_scan<double>(v[c], lane);
                    const int64_t pb = __builtin_amdgcn_ds_bpermute(src, (int)__double_as_longlong(pc)) & 0xffffffffll;
                    const int64_t pt = __builtin_amdgcn_ds_bpermute(src, (int)(__double_as_longlong(pc) >> 32));
                    const double before = hd > 0 ? __longlong_as_double((long long)(((uint64_t)pt << 32) | (uint64_t)pb)) : 0.0;
                    v[c] = pc - before;
                }
            }
            if (valid && tail)
                for (int c = 0; c < 6; ++c) acc[wid][c][jl] += v[c];
            __builtin_amdgcn_wave_barrier();
        }
        // point adjoints of this chunk (all but the L_bar and sum C_bar terms)
        double Ax = 0.0, Ay = 0.0, Bx = 0.0, By = 0.0, Cb = 0.0, lb = 0.0, ux = 0.0, uy = 0.0;
        if (lane < nseg) {
            Ax = acc[wid][0][lane];
            Ay = acc[wid][1][lane];
            Bx = acc[wid][2][lane];
            By = acc[wid][3][lane];
            Cb = acc[wid][4][lane];
            lb = acc[wid][5][lane];
            const double r = sR[wid][lane];
            ux = ((double)b.x - a.x) * r;
            uy = ((double)b.y - a.y) * r;
        }
        const double Pin = carryP + wave_incl_scan<double>(Cb, lane);
        const double Vx = lane < nseg ? (lb - Pin) * ux : 0.0;
        const double Vy = lane < nseg ? (lb - Pin) * uy : 0.0;
        double Bpx = lane_prev(Bx), Bpy = lane_prev(By);
        double Vpx = lane_prev(Vx), Vpy = lane_prev(Vy);
        if (lane == 0) {
            Bpx = carryBx;
            Bpy = carryBy;
            Vpx = carryVx;
            Vpy = carryVy;
        }
        if (lane < nseg || (last && lane == nseg))
            st2(pb + (j0 + lane), make_float2((float)(Ax + Bpx - Vx + Vpx), (float)(Ay + Bpy - Vy + Vpy)));
        carryBx = read_lane(Bx, nseg - 1);
        carryBy = read_lane(By, nseg - 1);
        carryVx = read_lane(Vx, nseg - 1);
        carryVy = read_lane(Vy, nseg - 1);
        carryP = read_lane(Pin, nseg - 1);
        if (last && nseg == 64 && lane == 0)
            st2(pb + (j0 + 64), make_float2((float)(carryBx + carryVx), (float)(carryBy + carryVy)));
        __builtin_amdgcn_wave_barrier();
        knext = kend;
        Cbase = Cend;
    }
    // pass B: L_bar and the total of C_bar enter every segment length alike
    const double G = wave_sum(Lbar) + carryP;
    if (G == 0.0) return;
    // G (u_(i-1) - u_i) with u the unit vectors of the segments: one segment per lane, 63
    // points per trip, u_(i-1) from lane l-1 (lane 0: from the previous trip)
    double cux = 0.0, cuy = 0.0;
    for (int q0 = 0; q0 < m; q0 += 63) {
        const int i = q0 + lane;
        const float2 c = i < m ? ld2(p + i) : make_float2(0.0f, 0.0f);
        float nxx = lane_next(c.x), nxy = lane_next(c.y);
        if (lane == 63 && i + 1 < m) {
            const float2 nx = ld2(p + (i + 1));
            nxx = nx.x;
            nxy = nx.y;
        }
        double ux = 0.0, uy = 0.0;
        if (lane < 63 && i + 1 < m) {
            double l, r;
            seg_len_rcp(c, make_float2(nxx, nxy), l, r);   // r = 0 for a zero-length segment
            ux = ((double)nxx - c.x) * r;
            uy = ((double)nxy - c.y) * r;
        }
        double pux = lane_prev(ux), puy = lane_prev(uy);
        if (lane == 0) {
            pux = cux;
            puy = cuy;
        }
        if (lane < 63 && i < m) {
            const float2 cur = ld2(pb + i);
            st2(pb + i, make_float2((float)((double)cur.x + G * (pux - ux)), (float)((double)cur.y + G * (puy - uy))));
        }
        cux = read_lane(ux, 62);
        cuy = read_lane(uy, 62);
    }
}

// dL/dM[l][b] += sum over the work items of layer l of their partial b; dL/da_k += sum over
// all work items of their partial B + k (items are in tile order, so a layer's items are
// contiguous). Two fixed-order stages: block (q, slice) sums one slice of parameter q's
// range (fixed per-thread order and a fixed tree), then one thread per parameter adds its
// slice sums in order.
__global__ __launch_bounds__(kBlock) void k_adj_reduce(const GDesc *__restrict__ gd, int ng) {
    const GDesc &d = gd[0];
    const int B = d.B;
    const int q = (int)blockIdx.x / kRedSlices, sl = (int)blockIdx.x % kRedSlices;
    const int per_layer = d.tiles_x * d.tiles_y;
    int64_t lo = 0, hi = d.aseg_off[d.n_tiles];
    int col;
    if (q < B * B) {
        const int l = q / B;
        col = q % B;
        lo = d.aseg_off[l * per_layer];
        hi = d.aseg_off[(l + 1) * per_layer];
    } else {
        col = B + (q - B * B);
    }
    const int64_t per = (hi - lo + kRedSlices - 1) / kRedSlices;
    const int64_t a = lo + sl * per, b = a + per < hi ? a + per : hi;
    const double *p = d.partials + (int64_t)col * d.max_items;
    double s = 0.0;
    for (int64_t i = a + threadIdx.x; i < b; i += kBlock) s += p[i];
    __shared__ double red[kBlock];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) d.red[(int64_t)q * kRedSlices + sl] = red[0];
}

__global__ __launch_bounds__(kBlock) void k_adj_reduce_sum(const GDesc *__restrict__ gd, int ng) {
    const GDesc &d = gd[0];
    const int nq = d.B * d.B + d.P;
    for (int q = threadIdx.x; q < nq; q += kBlock) {
        double s = 0.0;
        for (int sl = 0; sl < kRedSlices; ++sl) s += d.red[(int64_t)q * kRedSlices + sl];
        d.grad_param[q] += s;
    }
}

// ---------------------------------------------------------------- launchers

static inline dim3 grid1(int64_t blocks) { return dim3((unsigned)(blocks > 0 ? blocks : 0)); }

hipError_t launch_adj_maps(const GDesc *desc, const Shape &tot, int bmax, hipStream_t st) {
    if (bmax <= 8) hipLaunchKernelGGL(k_adj_maps<8>, grid1(tot.px), dim3(kBlock), 0, st, desc, 1);
    else hipLaunchKernelGGL(k_adj_maps<16>, grid1(tot.px), dim3(kBlock), 0, st, desc, 1);
    return hipGetLastError();
}

hipError_t launch_adj_advect(const GDesc *desc, const Shape &tot, hipStream_t st) {
    if (tot.edge <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_advect, grid1(tot.edge), dim3(kBlock), 0, st, desc, 1);
    return hipGetLastError();
}

hipError_t launch_adj_params(const GDesc *desc, const Shape &tot, int bmax, hipStream_t st) {
    if (tot.tile <= 0) return hipSuccess;
    const dim3 gr = grid1(tot.tile), bl(kParBlock);
    if (bmax <= 8) hipLaunchKernelGGL(k_adj_params<8>, gr, bl, 0, st, desc, 1);
    else hipLaunchKernelGGL(k_adj_params<16>, gr, bl, 0, st, desc, 1);
    return hipGetLastError();
}

hipError_t launch_adj_resample(const GDesc *desc, const Shape &tot, hipStream_t st) {
    if (tot.edge <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_resample, grid1(tot.edge), dim3(kBlock), 0, st, desc, 1);
    return hipGetLastError();
}

hipError_t launch_adj_reduce(const GDesc *desc, int B, int P, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_reduce, dim3((B * B + P) * kRedSlices), dim3(kBlock), 0, st, desc, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_reduce_sum, dim3(1), dim3(kBlock), 0, st, desc, 1);
    return hipGetLastError();
}

}  // namespace hb
