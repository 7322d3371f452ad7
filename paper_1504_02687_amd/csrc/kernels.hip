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

#include "device_common.h"

namespace hb {

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
    int big = 0;
    for (int i = threadIdx.x; i < kScanTile; i += kBlock) {
        int64_t e = base + i;
        if (e < d.n_edges) {
            const int64_t c = d.counts[e];
            s += c;
            big |= c >= kMaxEdgeSamples;
        }
    }
    int64_t tot;
    (void)block_excl_scan(s, &tot);
    // the point kernels index the samples of one edge with 32-bit integers
    if (__syncthreads_or(big) && threadIdx.x == 0) atomicOr(d.status, (int32_t)ST_HIST_OVERFLOW);
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
        for (int k = 1; k < d.P; ++k) grow *= (double)(2 * d.rp[k] + 1) * (double)(2 * d.rp[k] + 1);
        // int64 box sums stay below N w prod_{k>=1} (2 r_k + 1)^2 (a first pass never exceeds
        // the total); the int32 counts are bounded tile by tile when the samples are binned
        if (wsum * grow >= 9.2e18) st |= ST_HIST_OVERFLOW;
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

// ---------------------------------------------------------------- resample + bin

// One wave per edge. The polyline (pin) is streamed 64 U segments at a time, with their
// FP64 lengths and the arclengths at their starts (pair sums, 32-lane scans per block of 64
// segments, blocks chained). The samples whose arclength s_k = k L / (n-1) falls in those
// segments are produced 64 at a time: each lane finds its segment by binary search in LDS
// and interpolates in FP64. Every sample is stored (coalesced, float2) and counted in its
// histogram tile: one atomic per run of consecutive samples in the same tile, into the
// counter set of this block (block mod n_sets). DIR: the directed push along the segment's
// normal is compiled in (launches with a graph that has a directed offset).
template <int U, bool DIR>
__global__ __launch_bounds__(kBlock, 7) void k_resample_count(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_edge);
    if (stopped(d)) return;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t bl = blk - d.blk_edge;
    const int64_t e = edge_of(d, bl, wid);
    if (e < 0 || d.insdel) return;

    __shared__ double sC[kWavesPerBlock][64 * U];
    __shared__ double sR[kWavesPerBlock][64 * U];
    __shared__ float2 sP[kWavesPerBlock][64 * U + 1];

    // per-edge point and sample counts are below 2^31 (checked by the count scan)
    const int64_t i0 = d.off_in[e], o0 = d.off_s[e];
    const int m = (int)(d.off_in[e + 1] - i0), n = (int)(d.off_s[e + 1] - o0);
    const double L = d.lens[e];
    const HB_G float2 *p = glb(d.pin + i0);
    HB_G float2 *q = glb(d.samples + o0);
    const int layer = d.group[e];
    HB_G unsigned long long *ctr =
        glb((unsigned long long *)d.bin_cnt) + (bl & (d.n_sets - 1)) * d.n_tiles;
    const double nm1 = (double)(n - 1);
    const double ds = L / nm1;          // arclength between consecutive samples
    const double inv_ds = 1.0 / ds;
    const double doff = d.doff;

    double Cbase = 0.0;
    int knext = 0;
    for (int j0 = 0; j0 < m - 1; j0 += 64 * U) {
        const int rem = m - 1 - j0;
        const int nseg = rem < 64 * U ? rem : 64 * U;   // segments of this chunk
        // blocks of 64 segments, each summed the same way whatever U is (so every U gives the
        // same bits): lane r of a half holds two consecutive segments of a block, their sum
        // enters a 32-lane scan, and the block's base is the previous block's base plus that
        // block's total. Pass q holds blocks 2q (lanes 0-31) and 2q + 1 (lanes 32-63), i.e.
        // lane l holds segments 128 q + 2 l and 128 q + 2 l + 1 of the chunk.
        double cb = Cbase;               // base of block 2q
#pragma unroll
        for (int q = 0; q < (U + 1) / 2; ++q) {
            const int sj = 128 * q + 2 * lane;
            float2 a[3];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = make_float2(0.0f, 0.0f);
                if (sj + i <= nseg) a[i] = ld2(p + (j0 + sj + i));
            }
            a[2].x = lane_next(a[0].x);
            a[2].y = lane_next(a[0].y);
            if (lane == 63 && 128 * q + 128 <= nseg) a[2] = ld2(p + (j0 + 128 * q + 128));
            double ell[2], rcp[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                seg_len_rcp(a[i], a[i + 1], ell[i], rcp[i]);
                if (sj + i >= nseg) ell[i] = 0.0;
            }
            const double incl = half_incl_scan<double>(ell[0] + ell[1]);
            const double prev = lane_prev(incl);
            const double t0 = read_lane(incl, 31), t1 = read_lane(incl, 63);   // block totals
            const double bb = lane < 32 ? cb : cb + t0;                        // block base
            const double c0 = (lane & 31) ? bb + prev : bb;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int sg = sj + i;
                if (sg < 64 * U) {
                    // arclengths past the chunk's last segment read as +inf: the search
                    // needs no bound check
                    sC[wid][sg] = sg < nseg ? (i == 0 ? c0 : c0 + ell[0]) : __builtin_huge_val();
                    if (sg < nseg) {
                        sR[wid][sg] = rcp[i];
                        sP[wid][sg] = a[i];
                    }
                    if (sg == nseg - 1) sP[wid][nseg] = a[i + 1];
                }
            }
            cb = (cb + t0) + t1;
        }
        const double Cend = cb;
        __builtin_amdgcn_wave_barrier();

        const bool last = (j0 + 64 * U >= m - 1);
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
        for (int kb = knext; kb < kend; kb += 64) {
            const int k = kb + lane;
            int key = 0;
            uint32_t loc = 0;
            if (k < kend) {
                float2 out;
                if (k == 0) {
                    out = ld2(p);
                } else if (k == n - 1) {
                    out = ld2(p + (m - 1));
                } else {
                    const double s = mul_rn((double)k, ds);
                    // last segment of the chunk that starts at or before s (binary search
                    // over the LDS arclengths; lo + step < 64 U always)
                    int lo = 0;
#pragma unroll
                    for (int step = 32 * U; step >= 1; step >>= 1)
                        lo = sC[wid][lo + step] <= s ? lo + step : lo;
                    const float2 pa = sP[wid][lo], pb = sP[wid][lo + 1];
                    const double ex = (double)pb.x - (double)pa.x, ey = (double)pb.y - (double)pa.y;
                    double t = mul_rn(sub_rn(s, sC[wid][lo]), sR[wid][lo]);
                    t = fmin(fmax(t, 0.0), 1.0);
                    double ox = __builtin_fma(t, ex, (double)pa.x);
                    double oy = __builtin_fma(t, ey, (double)pa.y);
                    if (DIR && doff != 0.0) {
                        // directed graphs: along the left normal of the segment, doff / |e|
                        // (-ey, ex) with 1 / |e| the segment's stored reciprocal length
                        const double f = mul_rn(doff, sR[wid][lo]);
                        ox = __builtin_fma(-f, ey, ox);
                        oy = __builtin_fma(f, ex, oy);
                    }
                    out.x = (float)ox;
                    out.y = (float)oy;
                }
                st2(q + k, out);
                bin_of(d, layer, out, key, loc);
            }
            if (!d.strip) {
                // the samples are counted in their tiles here; line strips are counted by
                // k_strip_bins once every sample is known
                const int cnt = kend - kb < 64 ? kend - kb : 64;
                const uint64_t heads = run_heads(key, lane, cnt);
                if ((heads >> lane) & 1ull)
                    atomicAdd((unsigned long long *)(ctr + key), (unsigned long long)run_length(heads, lane, cnt));
            }
        }
        __builtin_amdgcn_wave_barrier();
        knext = kend;
        Cbase = Cend;
    }
}

// Insert/delete resampling (the pipeline of Section 3: points are created where consecutive
// points are too far apart and removed where they are too close). One wave per edge, the
// input polyline 64 points at a time. An interior point is kept when its squared distance to
// its input predecessor is at least dmin^2; the gap g between consecutive kept points a, b is
// cut into c = max(1, ceil(g / delta)) equal parts: a, then a + (t / c)(b - a), t = 1..c-1.
// A kept lane owns the gap to the next kept point of its chunk; the last kept point of a
// chunk is carried into the next one, whose first kept lane also owns the carried gap; the
// edge's last point closes it. WRITE = false: the point count of each edge (into counts);
// WRITE = true: the points, at the edge's sample offset. FP64 throughout, every operation
// rounded on its own.
__device__ __forceinline__ int64_t insdel_parts(float2 a, float2 b, double dmax) {
    const double dx = sub_rn((double)b.x, (double)a.x), dy = sub_rn((double)b.y, (double)a.y);
    const double c = ceil(sqrt(add_rn(mul_rn(dx, dx), mul_rn(dy, dy))) / dmax);
    return c < 1.0 ? 1 : (int64_t)c;
}

__device__ __forceinline__ float2 insdel_point(float2 a, float2 b, int64_t t, int64_t c) {
    const double f = (double)t / (double)c;
    float2 o;
    o.x = (float)add_rn((double)a.x, mul_rn(f, sub_rn((double)b.x, (double)a.x)));
    o.y = (float)add_rn((double)a.y, mul_rn(f, sub_rn((double)b.y, (double)a.y)));
    return o;
}

template <bool WRITE>
__global__ __launch_bounds__(kBlock) void k_insdel(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_edge);
    if (stopped(d)) return;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t bl = blk - d.blk_edge;
    const int64_t e = edge_of(d, bl, wid);
    if (e < 0 || !d.insdel) return;
    const int64_t i0 = d.off_in[e], m = d.off_in[e + 1] - i0;
    const HB_G float2 *p = glb(d.pin + i0);
    HB_G float2 *q = glb(d.samples + (WRITE ? d.off_s[e] : 0));
    const double dmin2 = mul_rn(d.dmin, d.dmin), dmax = d.delta;
    bool carried = false;          // a kept point is carried from the previous chunk
    float2 cp = make_float2(0.0f, 0.0f);
    int64_t base = 0;              // points of the edge before this chunk
    for (int64_t j0 = 0; j0 < m; j0 += 64) {
        const int64_t j = j0 + lane;
        const bool inr = j < m;
        const float2 a = inr ? ld2(p + j) : make_float2(0.0f, 0.0f);
        float2 pr;
        pr.x = lane_prev(a.x);
        pr.y = lane_prev(a.y);
        if (lane == 0 && j0 > 0) pr = ld2(p + (j0 - 1));
        bool keep = false;
        if (inr) {
            if (j == 0 || j == m - 1) {
                keep = true;
            } else {
                const double dx = sub_rn((double)a.x, (double)pr.x), dy = sub_rn((double)a.y, (double)pr.y);
                keep = add_rn(mul_rn(dx, dx), mul_rn(dy, dy)) >= dmin2;
            }
        }
        const uint64_t K = __ballot(keep);
        const uint64_t above = lane == 63 ? 0ull : (K >> (lane + 1));
        const int nxt = above ? lane + 1 + __builtin_ctzll(above) : lane;
        float2 b;
        b.x = __shfl(a.x, nxt, 64);
        b.y = __shfl(a.y, nxt, 64);
        const int first = K ? __builtin_ctzll(K) : 64;
        const int lastk = K ? 63 - __builtin_clzll(K) : 0;
        const bool final_chunk = j0 + 64 >= m;
        int64_t c0 = 0, c1 = 0;
        if (keep) {
            if (lane == first && carried) c0 = insdel_parts(cp, a, dmax);
            if (above) c1 = insdel_parts(a, b, dmax);
            else if (final_chunk) c1 = 1;      // the edge's last point
        }
        const int64_t cnt = c0 + c1;
        const int64_t incl = wave_incl_scan<int64_t>(cnt, lane);
        if (WRITE) {
            int64_t o = base + incl - cnt;
            for (int64_t t = 0; t < c0; ++t) st2(q + o++, insdel_point(cp, a, t, c0));
            if (above) {
                for (int64_t t = 0; t < c1; ++t) st2(q + o++, insdel_point(a, b, t, c1));
            } else if (c1) {
                st2(q + o, a);
            }
        }
        base += last_lane(incl);
        if (K) {
            carried = true;
            cp.x = __shfl(a.x, lastk, 64);
            cp.y = __shfl(a.y, lastk, 64);
        }
    }
    if (!WRITE && lane == 0) d.counts[e] = base;
}

// Samples of every edge in its histogram tile, one wave per edge, 64 consecutive samples
// at a time. Counting (SCATTER = false): one atomic per run of samples in the same tile, as
// k_resample_count does for samples it makes. Binning (SCATTER = true): the run takes its
// place from the write cursor of its tile and set (returning atomic) and stores one entry
// per sample. Both passes map an edge to the same block, so to the same counter set.
constexpr int kBinChunks = 8;

template <bool SCATTER>
__global__ __launch_bounds__(kBlock) void k_bin_samples(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_edge);
    if (stopped(d)) return;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t bl = blk - d.blk_edge;
    const int64_t e = edge_of(d, bl, wid);
    if (e < 0 || d.strip || (!SCATTER && !d.count_given)) return;
    HB_G unsigned long long *ctr =
        glb((unsigned long long *)(SCATTER ? d.bin_cur : d.bin_cnt)) + (bl & (d.n_sets - 1)) * d.n_tiles;
    const int64_t o0 = d.off_s[e], n = d.off_s[e + 1] - o0;
    const int layer = d.group[e];
    const uint32_t wbits = (uint32_t)(d.weight ? d.weight[e] : 1) << kLocalBits;
    const HB_G float2 *__restrict__ xs = glb(d.samples + o0);
    HB_G uint32_t *bins = glb(d.bins);
    // kBinChunks chunks per trip: their atomics are in flight together
    constexpr int U = kBinChunks;
    for (int64_t j0 = 0; j0 < n; j0 += 64 * U) {
        int key[U], cnt[U];
        uint32_t loc[U];
        uint64_t heads[U];
        unsigned long long base[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = j0 + 64 * u + lane;
            const int64_t r = n - j0 - 64 * u;
            cnt[u] = (int)(r <= 0 ? 0 : (r < 64 ? r : 64));
            key[u] = 0;
            loc[u] = 0;
            if (k < n) bin_of(d, layer, ld2(xs + k), key[u], loc[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            heads[u] = run_heads(key[u], lane, cnt[u]);
            base[u] = 0;
            if ((heads[u] >> lane) & 1ull) {
                unsigned long long *c = (unsigned long long *)(ctr + key[u]);
                const unsigned long long len = (unsigned long long)run_length(heads[u], lane, cnt[u]);
                if (SCATTER) base[u] = atomicAdd(c, len);
                else atomicAdd(c, len);
            }
        }
        if (SCATTER) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int h = run_head(heads[u], lane);
                const unsigned long long b0 = __shfl(base[u], h, 64);
                if (lane < cnt[u]) {
                    const unsigned long long pos = b0 + (unsigned long long)(lane - h);
                    if (pos < (unsigned long long)d.ent_cap) {
                        if (d.narrow) ((HB_G uint16_t *)bins)[pos] = (uint16_t)loc[u];
                        else bins[pos] = loc[u] | wbits;
                        if (d.bin_src) d.bin_src[pos] = (uint32_t)(o0 + j0 + 64 * u + lane);
                    } else {
                        atomicOr(d.status, ST_BIN_MISMATCH);
                    }
                }
            }
        }
    }
}

// Line-strip splat (the rasterised drawing of Eq. 1): the polyline of each edge drawn
// through the pixels of its samples, one wave per edge, 64 segments at a time. Lane k draws
// segment (k, k+1): the n = max(|du|, |dv|) pixels (u0 + round(t du / n), v0 + round(t dv /
// n)), t = 0 .. n-1, halves rounded up in exact integer arithmetic, and not its end pixel,
// which starts the next segment; the last sample of the edge draws its own pixel. At each
// step t the drawn pixels of the wave are counted in their tiles (SCATTER = false) or
// written as entries (SCATTER = true) with one atomic per run of drawing lanes in one tile,
// into the counter set of this block, as k_bin_samples does for samples.
template <bool SCATTER>
__global__ __launch_bounds__(kBlock) void k_strip_bins(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_edge);
    if (stopped(d)) return;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t bl = blk - d.blk_edge;
    const int64_t e = edge_of(d, bl, wid);
    if (e < 0 || !d.strip) return;
    HB_G unsigned long long *ctr =
        glb((unsigned long long *)(SCATTER ? d.bin_cur : d.bin_cnt)) + (bl & (d.n_sets - 1)) * d.n_tiles;
    const int64_t o0 = d.off_s[e], n = d.off_s[e + 1] - o0;
    const int layer = d.group[e];
    const uint32_t wbits = (uint32_t)(d.weight ? d.weight[e] : 1) << kLocalBits;
    const HB_G float2 *__restrict__ xs = glb(d.samples + o0);
    HB_G uint32_t *bins = glb(d.bins);
    const int W = d.W, H = d.H;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));    // lanes < lane
    for (int64_t j0 = 0; j0 < n; j0 += 64) {
        const int64_t k = j0 + lane;
        int u0 = 0, v0 = 0;
        if (k < n) pixel_of(ld2(xs + k), W, H, u0, v0);
        int u1 = lane_next(u0), v1 = lane_next(v0);
        if (lane == 63 && k + 1 < n) pixel_of(ld2(xs + k + 1), W, H, u1, v1);
        const int du = u1 - u0, dv = v1 - v0;
        const int adu = du < 0 ? -du : du, adv = dv < 0 ? -dv : dv;
        const int steps = adu > adv ? adu : adv;
        const int npx = k + 1 < n ? steps : (k + 1 == n ? 1 : 0);
        const int twon = 2 * steps;
        for (int t = 0; __any(t < npx); ++t) {
            const bool act = t < npx;
            int key = -1;
            uint32_t loc = 0;
            if (act) {
                int u = u0, v = v0;
                if (k + 1 < n) {
                    // floor((2 t du + n) / 2n) with a floor for negative numerators
                    const int a = 2 * t * du + steps, b = 2 * t * dv + steps;
                    const int qa = a >= 0 ? a / twon : -((-a + twon - 1) / twon);
                    const int qb = b >= 0 ? b / twon : -((-b + twon - 1) / twon);
                    u = u0 + qa;
                    v = v0 + qb;
                }
                tile_of(d, layer, u, v, key, loc);
            }
            const uint64_t am = __ballot(act);
            const uint64_t prev_m = am & below;
            const int pl = prev_m ? 63 - __builtin_clzll(prev_m) : lane;
            const int pkey = __shfl(key, pl, 64);
            const bool head = act && (prev_m == 0 || pkey != key);
            const uint64_t hm = __ballot(head);
            // this lane's run: from the last head at or below it to the next head above it
            const uint64_t upto = hm & (below | (1ull << lane));
            const int h = upto ? 63 - __builtin_clzll(upto) : lane;
            const uint64_t above = lane == 63 ? 0ull : (hm >> (lane + 1));
            const int nxt = above ? lane + 1 + __builtin_ctzll(above) : 64;
            unsigned long long base = 0;
            if (head) {
                const uint64_t span = (nxt >= 64 ? ~0ull : ((1ull << nxt) - 1)) & ~below;
                const unsigned long long len = (unsigned long long)__builtin_popcountll(am & span);
                unsigned long long *c = (unsigned long long *)(ctr + key);
                if (SCATTER) base = atomicAdd(c, len);
                else atomicAdd(c, len);
            }
            if (SCATTER) {
                const unsigned long long b0 = __shfl(base, h, 64);
                if (act) {
                    const uint64_t before = am & below & ~(h == 0 ? 0ull : (~0ull >> (64 - h)));
                    const unsigned long long pos = b0 + (unsigned long long)__builtin_popcountll(before);
                    if (pos < (unsigned long long)d.ent_cap) {
                        if (d.narrow) ((HB_G uint16_t *)bins)[pos] = (uint16_t)loc;
                        else bins[pos] = loc | wbits;
                    }
                    else atomicOr(d.status, ST_BIN_MISMATCH);
                }
            }
        }
    }
}

// Tile offsets of one graph (one block per graph): the entries of tile t start at
// tile_off[t], those of set s of tile t right after the sets before it (the cursors), and
// tile t is cut into work items of item_entries entries numbered from seg_off[t].
__global__ __launch_bounds__(kBlock) void k_bin_scan(const GDesc *__restrict__ gd, int ng) {
    if ((int)blockIdx.x >= ng) return;
    const GDesc &d = gd[blockIdx.x];
    if (stopped(d)) return;
    const int nt = d.n_tiles;
    int64_t base_off = 0, base_seg = 0;
    bool big = false;
    for (int t0 = 0; t0 < nt; t0 += kBlock) {
        const int t = t0 + (int)threadIdx.x;
        int64_t tot = 0;
        if (t < nt)
            for (int q = 0; q < d.n_sets; ++q) tot += d.bin_cnt[(int64_t)q * nt + t];
        // the int32 count of a pixel is at most its tile's entries times the largest weight
        big |= (double)tot * (double)d.wmax >= 2147483647.0;
        const int64_t segs = (tot + d.item_entries - 1) / d.item_entries;
        int64_t sum_tot, sum_seg;
        const int64_t xo = block_excl_scan(tot, &sum_tot);
        const int64_t xg = block_excl_scan(segs, &sum_seg);
        if (t < nt) {
            int64_t at = base_off + xo;
            d.tile_off[t] = at;
            d.seg_off[t] = base_seg + xg;
            for (int q = 0; q < d.n_sets; ++q) {
                d.bin_cur[(int64_t)q * nt + t] = at;
                at += d.bin_cnt[(int64_t)q * nt + t];
            }
        }
        base_off += sum_tot;
        base_seg += sum_seg;
    }
    if (__syncthreads_or(big) && threadIdx.x == 0) atomicOr(d.status, (int32_t)ST_HIST_OVERFLOW);
    if (threadIdx.x == 0) {
        d.tile_off[nt] = base_off;
        d.seg_off[nt] = base_seg;
        if (d.strip) {
            // one entry per drawn pixel: the buffer bound and the histogram ranges are checked
            // here, on the actual count
            int32_t st = 0;
            if (base_off > d.ent_cap) st |= ST_ENTRY_OVERFLOW;
            const double wsum = (double)base_off * (double)d.wmax;
            double grow = 1.0;
            for (int k = 1; k < d.P; ++k) grow *= (double)(2 * d.rp[k] + 1) * (double)(2 * d.rp[k] + 1);
            if (wsum * grow >= 9.2e18) st |= ST_HIST_OVERFLOW;
            if (st) atomicOr(d.status, st);
        } else if (base_off != d.off_s[d.n_edges] || base_off > d.ent_cap) {
            atomicOr(d.status, ST_BIN_MISMATCH);
        }
    }
}

// LDS counter of a pixel inside a 64 x 64 tile (row v, column u; local = 64 v + u): the low
// five bits of the column are XORed with those of the row, so the pixels of one tile column
// (polylines running vertically) fall into different LDS banks. An involution within the row:
// the slot of a slot is the pixel.
__device__ __forceinline__ uint32_t lds_slot(uint32_t local) {
    local &= (uint32_t)(kTilePx - 1);
    return local ^ ((local >> kTileShift) & 31u);
}

// Histogram tiles in LDS. Each block takes work items (up to item_entries entries of one
// tile) round-robin, adds the entries' weights to its LDS copy of the tile with LDS
// atomics, then adds the non-zero counters to the histogram (first copy of histx).
__global__ __launch_bounds__(kBlock) void k_tile_hist(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_tile);
    if (stopped(d)) return;
    __shared__ int32_t lh[kTilePx];
    const int nt = d.n_tiles;
    const int64_t nseg = d.seg_off[nt];
    const int W = d.W, H = d.H;
    const int64_t plane = (int64_t)W * H;
    const int per_layer = d.tiles_x * d.tiles_y;
    const HB_G uint32_t *__restrict__ bins = glb(d.bins);
    for (int64_t sg = blk - d.blk_tile; sg < nseg; sg += d.tile_blocks) {
        int lo = 0, hi = nt - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (d.seg_off[mid] <= sg) lo = mid; else hi = mid - 1;
        }
        const int t = lo;
        const int64_t beg = d.tile_off[t] + (sg - d.seg_off[t]) * d.item_entries;
        const int64_t lim = d.tile_off[t + 1];
        const int64_t end = beg + d.item_entries < lim ? beg + d.item_entries : lim;
        for (int i = threadIdx.x; i < kTilePx; i += kBlock) lh[i] = 0;
        __syncthreads();
        int64_t i = beg + threadIdx.x;
        if (d.narrow) {
            // unit weights: 16-bit entries, one count each
            const HB_G uint16_t *__restrict__ b16 = (const HB_G uint16_t *)bins;
            for (; i + 3 * kBlock < end; i += 4 * kBlock) {
                const uint32_t a0 = b16[i], a1 = b16[i + kBlock];
                const uint32_t a2 = b16[i + 2 * kBlock], a3 = b16[i + 3 * kBlock];
                atomicAdd(&lh[lds_slot(a0)], 1);
                atomicAdd(&lh[lds_slot(a1)], 1);
                atomicAdd(&lh[lds_slot(a2)], 1);
                atomicAdd(&lh[lds_slot(a3)], 1);
            }
            for (; i < end; i += kBlock) atomicAdd(&lh[lds_slot(b16[i])], 1);
        } else {
            for (; i + 3 * kBlock < end; i += 4 * kBlock) {
                const uint32_t a0 = bins[i], a1 = bins[i + kBlock];
                const uint32_t a2 = bins[i + 2 * kBlock], a3 = bins[i + 3 * kBlock];
                atomicAdd(&lh[lds_slot(a0)], (int32_t)(a0 >> kLocalBits));
                atomicAdd(&lh[lds_slot(a1)], (int32_t)(a1 >> kLocalBits));
                atomicAdd(&lh[lds_slot(a2)], (int32_t)(a2 >> kLocalBits));
                atomicAdd(&lh[lds_slot(a3)], (int32_t)(a3 >> kLocalBits));
            }
            for (; i < end; i += kBlock) {
                const uint32_t a0 = bins[i];
                atomicAdd(&lh[lds_slot(a0)], (int32_t)(a0 >> kLocalBits));
            }
        }
        __syncthreads();
        const int layer = t / per_layer, rem = t - layer * per_layer;
        const int ty = rem / d.tiles_x, tx = rem - ty * d.tiles_x;
        HB_G int32_t *hist = glb(d.histx) + (int64_t)layer * plane;
        for (int q = threadIdx.x; q < kTilePx; q += kBlock) {
            const int32_t v = lh[q];
            const int p = (int)lds_slot((uint32_t)q);
            const int y = ty * kTile + (p >> kTileShift), x = tx * kTile + (p & (kTile - 1));
            if (v != 0 && x < W && y < H) atomicAdd((int32_t *)(hist + (int64_t)y * W + x), v);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- maps

// Clear the histogram accumulator and the tile counters. One thread per layer pixel.
__global__ __launch_bounds__(kBlock) void k_clear_hist(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_pxb);
    if (stopped(d)) return;
    const int64_t n = (int64_t)d.B * d.W * d.H;
    const int64_t i = (blk - d.blk_pxb) * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < d.nx; ++c) d.histx[c * n + i] = 0;
    for (int64_t j = i; j < (int64_t)d.n_sets * d.n_tiles; j += n) d.bin_cnt[j] = 0;
}

// Row pass of one box filter: out(u) = sum of in(u') over |u'-u| <= r inside the row,
// from the row's prefix sums in LDS. One block per row of one group. The first pass sums
// the per-XCD histogram copies, stores the histogram row and flags int32 overflow.
template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_box_rows(const GDesc *__restrict__ gd, int ng,
                                                     int pass) {
    extern __shared__ int64_t srow[];
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_row);
    if (stopped(d) || pass >= d.P) return;
    const int64_t row = blk - d.blk_row;
    const int W = d.W, r = d.rp[pass];
    const int64_t plane = (int64_t)d.B * d.W * d.H;
    if (pass == 0) {
        bool bad = false;
        for (int u = threadIdx.x; u < W; u += kBlock) {
            int64_t x = 0;
            for (int c = 0; c < d.nx; ++c) {
                const int32_t v = d.histx[c * plane + row * W + u];
                bad |= v < 0;
                x += v;
            }
            bad |= x > 2147483647;
            srow[u] = x;
            d.hist[row * W + u] = (int32_t)x;
        }
        if (bad) atomicOr(d.status, ST_HIST_OVERFLOW);
    } else {
        const Tin *in = (const Tin *)(d.box + (pass - 1) * plane) + row * W;
        for (int u = threadIdx.x; u < W; u += kBlock) srow[u] = (int64_t)in[u];
    }
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

// Column pass: sliding window sum down a column segment of col_rows rows. One thread per
// (group, segment, column); neighbouring threads read neighbouring columns.
__global__ __launch_bounds__(kBlock) void k_box_cols(const GDesc *__restrict__ gd, int ng,
                                                     int pass) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_col);
    if (stopped(d) || pass >= d.P) return;
    const int W = d.W, H = d.H, r = d.rp[pass];
    const int rows = d.col_rows;
    const int nseg = (H + rows - 1) / rows;
    const int64_t t = (blk - d.blk_col) * kBlock + threadIdx.x;
    if (t >= (int64_t)d.B * nseg * W) return;
    const int u = (int)(t % W);
    const int64_t rest = t / W;
    const int seg = (int)(rest % nseg);
    const int64_t b = rest / nseg;
    const int64_t plane = (int64_t)W * H;
    const int64_t *in = d.tmp + b * plane + u;
    int64_t *out = d.box + (int64_t)pass * d.B * plane + b * plane + u;
    const int v0 = seg * rows;
    const int v1 = v0 + rows < H ? v0 + rows : H;
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

// Strip maps of the density and gradient (see strip_rows): one thread per row k of a gradient
// record (strip s, stored column c) writes that row's gradient pair and, for c <= W, the
// density pair of columns c and c + 1 (consecutive threads write consecutive 8-byte words);
// rows and columns clamped into the grid.
__global__ __launch_bounds__(kBlock) void k_strips(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_strip);
    if (stopped(d)) return;
    const int W = d.W, H = d.H, WC = W + 2;
    const int64_t per = strip_rows(H) * WC * 5, plane = (int64_t)W * H;
    const int64_t i = (blk - d.blk_strip) * kBlock + threadIdx.x;
    if (i >= (int64_t)d.B * per) return;
    const int64_t l = i / per, r = i - l * per, rec = r / 5;
    const int k = (int)(r - rec * 5), s = (int)(rec / WC), c = (int)(rec - (int64_t)s * WC);
    const int64_t row = (int64_t)min(max(4 * s + k - 1, 0), H - 1) * W;
    const int u0 = min(max(c - 1, 0), W - 1), u1 = min(c, W - 1);
    d.grads[l * grad_strip_plane(W, H) + r] = d.grad[l * plane + row + u0];
    // a density record is ten floats (five pairs) at a multiple of ten floats
    if (c <= W) {
        float2 *ro = (float2 *)(d.rhos + l * rho_strip_plane(W, H));
        ro[((int64_t)s * (W + 1) + c) * 5 + k] = make_float2(d.rho[l * plane + row + u0], d.rho[l * plane + row + u1]);
    }
}

// ---------------------------------------------------------------- advection + smoothing

// Step halvings tested per round of the advection (candidates loaded together).
constexpr int kTriesPerRound = 2;
constexpr float kRoundScale = 1.0f / (float)(1 << kTriesPerRound);   // step ratio per round

// One round of step halvings k .. k + kTriesPerRound - 1 (step mf, mf/2, ...) for UU
// sub-chunks: every candidate of the round is loaded first, then the first candidate whose
// FP32 bilinear density is not lower than r0 is accepted (jj = its halving, act cleared).
template <int UU>
__device__ __forceinline__ void halving_round(const HB_G float *__restrict__ rho, const float2 *x,
                                              const float *dx, const float *dy, const float *r0,
                                              bool *act, int *jj, int k, int K, float mf,
                                              float xmaxf, float ymaxf, int W, int H) {
    STap c[kTriesPerRound][UU];
    Quad q[kTriesPerRound][UU];
    float mt = mf;
#pragma unroll
    for (int i = 0; i < kTriesPerRound; ++i) {
#pragma unroll
        for (int u = 0; u < UU; ++u) {
            const float cx = __builtin_amdgcn_fmed3f(__builtin_fmaf(mt, dx[u], x[u].x), 0.0f, xmaxf);
            const float cy = __builtin_amdgcn_fmed3f(__builtin_fmaf(mt, dy[u], x[u].y), 0.0f, ymaxf);
            c[i][u] = stap_inside(cx, cy, W, H);
        }
        mt *= 0.5f;
    }
#pragma unroll
    for (int i = 0; i < kTriesPerRound; ++i)
#pragma unroll
        for (int u = 0; u < UU; ++u)
            if (act[u] && k + i <= K) q[i][u] = ld_rho(rho, c[i][u].od);
#pragma unroll
    for (int i = 0; i < kTriesPerRound; ++i) {
#pragma unroll
        for (int u = 0; u < UU; ++u) {
            if (act[u] && k + i <= K && interp1q(q[i][u], c[i][u]) >= r0[u]) {
                jj[u] = k + i;
                act[u] = false;
            }
        }
    }
    // no load of this round is left in flight (a lane that skipped its test skipped the wait
    // as well): the next round's loads then go out without waiting
    vm_wait_all();
}

// One wave per edge. Each trip handles U sub-chunks of 62 output points with a one-point
// halo on each side (U independent gather chains in flight): lane l of sub-chunk u
// advects point j0 + 62u - 1 + l (end points stay), neighbours come from lanes l-1 and l+1,
// and lanes 1..62 write the Laplacian-smoothed point. The FP64 length of the smoothed
// polyline gives the next sample count. Up to two sub-chunks the kernel is held to five
// waves per SIMD (at most 96 VGPRs).
template <int U>
__global__ __launch_bounds__(kBlock, U <= 2 ? 5 : 1) void k_advect_smooth(const GDesc *__restrict__ gd, int ng) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_edge);
    if (stopped(d)) return;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // edges by group, then position, dealt round-robin: the blocks in flight read one or
    // two layers of the maps, around nearby edges
    const int64_t idx = (blk - d.blk_edge) * kWavesPerBlock + wid;
    if (idx >= d.n_edges) return;
    const int64_t e = d.order ? (int64_t)d.order[idx] : idx;

    const int W = d.W, H = d.H;
    const int64_t plane = (int64_t)W * H;
    const int64_t o0 = d.off_s[e], n = d.off_s[e + 1] - o0;
    (void)plane;
    const HB_G float *__restrict__ rho = glb(d.rhos + (int64_t)d.group[e] * rho_strip_plane(W, H));
    const HB_G float2 *__restrict__ grad = glb(d.grads + (int64_t)d.group[e] * grad_strip_plane(W, H));
    const HB_G float2 *__restrict__ xs = glb(d.samples + o0);
    HB_G float2 *__restrict__ ys = glb(d.pnew + o0);
    HB_G int8_t *__restrict__ jrec = glb(d.jacc + o0);
    const double h = d.h, s = d.s;
    const float eps2 = (float)(d.eps * d.eps), inv_eps = (float)(1.0 / d.eps);
    const int K = d.K;
    const double xmax = (double)W - 1.0 / 256.0, ymax = (double)H - 1.0 / 256.0;
    const float xmaxf = (float)xmax, ymaxf = (float)ymax;

    double Lp = 0.0;
    float2 yprev = make_float2(0.0f, 0.0f);
    for (int64_t j0 = 0; j0 < n; j0 += 62 * U) {
        float2 x[U];
        double ax[U], ay[U];
        float dx[U], dy[U], r0[U];
        int jj[U];
        bool act[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = j0 + 62 * u - 1 + lane;
            const bool inr = j >= 0 && j < n;
            x[u] = make_float2(0.0f, 0.0f);
            if (inr) x[u] = ld2(xs + j);
            ax[u] = x[u].x;
            ay[u] = x[u].y;
            act[u] = inr && j > 0 && j < n - 1;
            jj[u] = act[u] ? -1 : -2;
        }
        // every sub-chunk's taps first, then all their loads, then the arithmetic, so the
        // U gather chains are in flight together (inactive lanes read valid taps)
        STap t0[U];
        Quad g0[U], g1[U], rq[U];
#pragma unroll
        for (int u = 0; u < U; ++u) t0[u] = stap_of(x[u].x, x[u].y, W, H);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ld_grad(grad, t0[u].og, g0[u], g1[u]);
            rq[u] = ld_rho(rho, t0[u].od);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // the interpolated gradient in FP64 keeps its direction where the taps nearly
            // cancel; its normalisation only needs FP32
            double gx, gy;
            interp2q(g0[u], g1[u], t0[u], gx, gy);
            const float fx = (float)gx, fy = (float)gy;
            // d = g / max(|g|, eps), through one reciprocal square root (about 1 ulp)
            const float n2 = __builtin_fmaf(fy, fy, fx * fx);
            const float inv = n2 > eps2 ? __builtin_amdgcn_rsqf(n2) : inv_eps;
            dx[u] = act[u] ? fx * inv : 0.0f;
            dy[u] = act[u] ? fy * inv : 0.0f;
            r0[u] = act[u] ? interp1q(rq[u], t0[u]) : 0.0f;
        }
        // K < 0: the original fixed step (every interior point moves by h, no test)
        if (K < 0) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (act[u]) jj[u] = 0;
                act[u] = false;
            }
        }
        // acceptance tests in FP32, kTriesPerRound halvings per round: the candidates of a
        // round are loaded together (all sub-chunks too) and the first accepted one in order
        // wins, so the decisions are those of testing one halving after the other, with
        // fewer dependent round trips to memory; the accepted point is recomputed in FP64
        float mf = (float)h;
        int k = 0;
        if (K >= 0) {
            bool any = false;
#pragma unroll
            for (int u = 0; u < U; ++u) any |= act[u];
            if (__any(any)) {
                halving_round<U>(rho, x, dx, dy, r0, act, jj, 0, K, mf, xmaxf, ymaxf, W, H);
                k = kTriesPerRound;
                mf *= kRoundScale;
            }
        }
        for (; k <= K; k += kTriesPerRound) {
            bool any = false;
#pragma unroll
            for (int u = 0; u < U; ++u) any |= act[u];
            if (!__any(any)) break;
            halving_round<U>(rho, x, dx, dy, r0, act, jj, k, K, mf, xmaxf, ymaxf, W, H);
            mf *= kRoundScale;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (jj[u] >= 0) {
                const double m = ldexp(h, -jj[u]);
                ax[u] = fmin(fmax(__builtin_fma(m, (double)dx[u], (double)x[u].x), 0.0), xmax);
                ay[u] = fmin(fmax(__builtin_fma(m, (double)dy[u], (double)x[u].y), 0.0), ymax);
            }
        }
        float2 y[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = j0 + 62 * u - 1 + lane;
            const double lx = lane_prev(ax[u]), ly = lane_prev(ay[u]);
            const double rx = lane_next(ax[u]), ry = lane_next(ay[u]);
            const bool out = lane >= 1 && lane <= 62 && j < n;
            y[u] = x[u];
            if (out && j > 0 && j < n - 1) {
                y[u].x = (float)__builtin_fma(0.5 * s, add_rn(lx, rx), mul_rn(1.0 - s, ax[u]));
                y[u].y = (float)__builtin_fma(0.5 * s, add_rn(ly, ry), mul_rn(1.0 - s, ay[u]));
            }
            if (out) {
                st2(ys + j, y[u]);
                if (d.record) jrec[j] = (int8_t)jj[u];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = j0 + 62 * u - 1 + lane;
            const bool out = lane >= 1 && lane <= 62 && j < n;
            float2 yl;
            yl.x = lane_prev(y[u].x);
            yl.y = lane_prev(y[u].y);
            if (lane == 1) yl = yprev;
            // each lane sums its own segments, in the same order whatever U; one wave sum at
            // the end of the edge
            if (out && j >= 1) {
                // next sample count: a relative error of 1e-15 per segment only matters for
                // lengths within rounding of a multiple of delta, where either count is valid
                double len, rcp;
                seg_len_rcp(yl, y[u], len, rcp);
                Lp += len;
            }
            yprev.x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(y[u].x), 62));
            yprev.y = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(y[u].y), 62));
        }
    }
    const double L = wave_sum(Lp);
    if (lane == 0) {
        d.lens[e] = L;
        d.counts[e] = sample_count(L, d.delta);
    }
}

// Orientation slice of every edge (one thread per edge): the direction (dx, dy) from the
// first to the last point of its polyline, slice k for angles in [90k - 45, 90k + 45)
// degrees, decided by exact comparisons of dx and dy; coincident end points give slice 0.
__global__ __launch_bounds__(kBlock) void k_orientation(const GDesc *__restrict__ gd, int ng,
                                                        int32_t *group) {
    const int64_t blk = blockIdx.x;
    HB_FIND(blk_edget);
    const int64_t e = (blk - d.blk_edget) * kBlock + threadIdx.x;
    if (e >= d.n_edges) return;
    const float2 a = d.pin[d.off_in[e]], b = d.pin[d.off_in[e + 1] - 1];
    const double dx = (double)b.x - (double)a.x, dy = (double)b.y - (double)a.y;
    int k = 0;
    if (dy > 0.0 && -dy < dx && dx <= dy) k = 1;           // [45, 135)
    else if (dx < 0.0 && dx < dy && dy <= -dx) k = 2;      // [135, 225)
    else if (dy < 0.0 && dy <= dx && dx < -dy) k = 3;      // [225, 315)
    group[e] = k;
}

// Total length of the polylines (the ink): sum of the per-edge lengths in a fixed order.
// Stage 1: block j sums its contiguous slice (fixed per-thread order, fixed tree) into
// part[j]; stage 2: one block sums the kInkSlices slice sums in order into part[kInkSlices].
__global__ __launch_bounds__(kBlock) void k_ink_slices(const double *__restrict__ lens,
                                                       int64_t n, double *part) {
    const int64_t per = (n + kInkSlices - 1) / kInkSlices;
    const int64_t a = (int64_t)blockIdx.x * per, b = a + per < n ? a + per : n;
    double s = 0.0;
    for (int64_t i = a + threadIdx.x; i < b; i += kBlock) s += lens[i];
    __shared__ double red[kBlock];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void k_ink_total(double *part) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int j = 0; j < kInkSlices; ++j) s += part[j];
    part[kInkSlices] = s;
}

// Mark the per-iteration sample totals of every graph as not produced yet (-1). One block
// per graph; desc[g] is graph g's descriptor of the first iteration.
__global__ __launch_bounds__(kBlock) void k_fill_totals(const GDesc *__restrict__ gd, int T) {
    int64_t *t = gd[blockIdx.x].total;
    for (int i = threadIdx.x; i < T; i += kBlock) t[i] = -1;
}

// ---------------------------------------------------------------- launchers

Shape shape_of(int64_t n_edges, int32_t B, int32_t W, int32_t H, const Tiling &tg) {
    Shape s;
    const int64_t plane = (int64_t)W * H;
    const int64_t nseg = (H + tg.col_rows - 1) / tg.col_rows;
    s.edge = (n_edges + kWavesPerBlock - 1) / kWavesPerBlock;
    s.scan = (n_edges + kScanTile - 1) / kScanTile;
    s.row = (int64_t)B * H;
    s.col = ((int64_t)B * nseg * W + kBlock - 1) / kBlock;
    s.px = (plane + kBlock - 1) / kBlock;
    s.pxb = ((int64_t)B * plane + kBlock - 1) / kBlock;
    s.edget = (n_edges + 1 + kBlock - 1) / kBlock;
    s.tile = tiles_of(B, W, H, tg.sets_max).blocks;
    s.strip = ((int64_t)B * strip_rows(H) * (W + 2) * 5 + kBlock - 1) / kBlock;
    return s;
}

Tiles tiles_of(int32_t B, int32_t W, int32_t H, int32_t sets_max) {
    Tiles t;
    t.x = (W + kTile - 1) / kTile;
    t.y = (H + kTile - 1) / kTile;
    t.n = B * t.x * t.y;
    t.blocks = t.n < kTileBlocksMax ? t.n : kTileBlocksMax;
    t.sets = 1;
    while (t.sets < sets_max && (int64_t)t.sets * 2 * t.n <= kBinCounters) t.sets *= 2;
    return t;
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

hipError_t launch_fill_totals(const GDesc *desc, int ng, int T, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_totals, dim3(ng), dim3(kBlock), 0, st, desc, T);
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

hipError_t launch_resample_count(const GDesc *desc, int ng, const Shape &tot, int u,
                                 bool directed, hipStream_t st) {
    if (tot.edge <= 0) return hipSuccess;
    const dim3 gr = grid_of(tot.edge), bl(kBlock);
    if (directed) {
        switch (u) {
            case 1: hipLaunchKernelGGL((k_resample_count<1, true>), gr, bl, 0, st, desc, ng); break;
            case 4: hipLaunchKernelGGL((k_resample_count<4, true>), gr, bl, 0, st, desc, ng); break;
            default: hipLaunchKernelGGL((k_resample_count<2, true>), gr, bl, 0, st, desc, ng); break;
        }
    } else {
        switch (u) {
            case 1: hipLaunchKernelGGL((k_resample_count<1, false>), gr, bl, 0, st, desc, ng); break;
            case 4: hipLaunchKernelGGL((k_resample_count<4, false>), gr, bl, 0, st, desc, ng); break;
            default: hipLaunchKernelGGL((k_resample_count<2, false>), gr, bl, 0, st, desc, ng); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_count_given(const GDesc *desc, int ng, const Shape &tot, hipStream_t st) {
    if (tot.edge <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bin_samples<false>, grid_of(tot.edge), dim3(kBlock), 0, st, desc, ng);
    return hipGetLastError();
}

hipError_t launch_insdel(const GDesc *desc, int ng, const Shape &tot, bool write, hipStream_t st) {
    if (tot.edge <= 0) return hipSuccess;
    if (write) hipLaunchKernelGGL(k_insdel<true>, grid_of(tot.edge), dim3(kBlock), 0, st, desc, ng);
    else hipLaunchKernelGGL(k_insdel<false>, grid_of(tot.edge), dim3(kBlock), 0, st, desc, ng);
    return hipGetLastError();
}

hipError_t launch_strip_bins(const GDesc *desc, int ng, const Shape &tot, bool scatter,
                             hipStream_t st) {
    if (tot.edge <= 0) return hipSuccess;
    if (scatter) hipLaunchKernelGGL(k_strip_bins<true>, grid_of(tot.edge), dim3(kBlock), 0, st, desc, ng);
    else hipLaunchKernelGGL(k_strip_bins<false>, grid_of(tot.edge), dim3(kBlock), 0, st, desc, ng);
    return hipGetLastError();
}

hipError_t launch_bin_hist(const GDesc *desc, int ng, const Shape &tot, bool strip, bool points,
                           hipStream_t st) {
    if (ng <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bin_scan, dim3((unsigned)ng), dim3(kBlock), 0, st, desc, ng);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || tot.edge <= 0) return e;
    if (strip) {
        hipLaunchKernelGGL(k_strip_bins<true>, grid_of(tot.edge), dim3(kBlock), 0, st, desc, ng);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (points)
        hipLaunchKernelGGL(k_bin_samples<true>, grid_of(tot.edge), dim3(kBlock), 0, st, desc, ng);
    if ((e = hipGetLastError()) != hipSuccess || tot.tile <= 0) return e;
    hipLaunchKernelGGL(k_tile_hist, grid_of(tot.tile), dim3(kBlock), 0, st, desc, ng);
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

hipError_t launch_density_strips(const GDesc *desc, int ng, const Shape &tot, int bmax,
                                 hipStream_t st) {
    hipError_t e = launch_density_grad(desc, ng, tot, bmax, st);
    if (e != hipSuccess || tot.strip <= 0) return e;
    hipLaunchKernelGGL(k_strips, grid_of(tot.strip), dim3(kBlock), 0, st, desc, ng);
    return hipGetLastError();
}

hipError_t launch_orientation(const GDesc *desc, const Shape &tot, int32_t *group, hipStream_t st) {
    if (tot.edget <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_orientation, grid_of(tot.edget), dim3(kBlock), 0, st, desc, 1, group);
    return hipGetLastError();
}

hipError_t launch_ink(const double *lens, int64_t n, double *part, hipStream_t st) {
    hipLaunchKernelGGL(k_ink_slices, dim3(kInkSlices), dim3(kBlock), 0, st, lens, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ink_total, dim3(1), dim3(64), 0, st, part);
    return hipGetLastError();
}

hipError_t launch_advect_smooth(const GDesc *desc, int ng, const Shape &tot, int u,
                                hipStream_t st) {
    if (tot.edge <= 0) return hipSuccess;
    const dim3 gr = grid_of(tot.edge), bl(kBlock);
    switch (u) {
        case 1: hipLaunchKernelGGL(k_advect_smooth<1>, gr, bl, 0, st, desc, ng); break;
        case 4: hipLaunchKernelGGL(k_advect_smooth<4>, gr, bl, 0, st, desc, ng); break;
        default: hipLaunchKernelGGL(k_advect_smooth<2>, gr, bl, 0, st, desc, ng); break;
    }
    return hipGetLastError();
}

}  // namespace hb
