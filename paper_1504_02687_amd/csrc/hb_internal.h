// Internal declarations of the HIP bundling library: the per-graph launch descriptor
// shared by every kernel, status bits, and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hb.h"

namespace hb {

// Device status bits (a single int32 per context, read by every kernel at entry).
enum : int32_t {
    ST_POINT_OVERFLOW = 1,   // the next sample set does not fit the point buffers
    ST_HIST_OVERFLOW = 2,    // counts could exceed int32 / int64 box sums could overflow
    ST_BIN_MISMATCH = 4,     // tile counts and binned samples disagree (internal error)
    ST_ENTRY_OVERFLOW = 8,   // the drawn line strips need more entries than the entry buffer
    ST_STOP = ST_POINT_OVERFLOW | ST_HIST_OVERFLOW | ST_BIN_MISMATCH | ST_ENTRY_OVERFLOW,
};

constexpr int kBlock = 256;            // threads per block of every kernel
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kScanTile = 1024;        // edges per scan tile (4 per thread)
constexpr int kColSeg = 128;           // rows per thread in the column box pass (default)

// Spatial binning of the samples: the histogram is built tile by tile in LDS.
constexpr int kTileShift = 6;                       // tiles of 64 x 64 pixels
constexpr int kTile = 1 << kTileShift;
constexpr int kTilePx = kTile * kTile;              // LDS counters of one tile
constexpr int kLocalBits = 2 * kTileShift;          // pixel inside the tile, low bits of an entry
constexpr int kBinSetsMax = 64;                     // tile-count sets (edge block mod sets), default
constexpr int64_t kBinCounters = 1 << 18;          // counters of all sets, at most (unless 1 set)
constexpr int64_t kSegEntries = 1 << 16;            // entries per tile-histogram work item, default
constexpr int kTileBlocksMax = 2048;                // blocks of one graph in k_tile_hist
constexpr int kRedSlices = 32;                      // slices per parameter in k_adj_reduce
constexpr int kInkSlices = 256;                     // slices of the ink sum
constexpr int64_t kMaxEdgeSamples = int64_t(1) << 31;  // samples of one edge, exclusive bound
static_assert(HB_MAX_EDGE_WEIGHT < (1u << (32 - kLocalBits)), "weights must fit an entry");
constexpr int kKmMaxK = HB_KMEANS_MAX_K;            // clusters of the grouping k-means
constexpr int kKmMaxDim = HB_KMEANS_MAX_DIM;        // coordinates per point
static_assert(kKmMaxK <= kBlock, "one thread per cluster in k_km_db");

// Four map values of one bilinear sample: a (u0, v0), b (u0 + 1, v0), c (u0, v0 + 1),
// d (u0 + 1, v0 + 1).
struct alignas(16) Quad {
    float a, b, c, d;
};

// Strip maps for bilinear sampling. The grid padded by one clamped row and column on each
// side (stored row r = v + 1 in [0, H + 1], stored column c = u + 1 in [0, W + 1]) is cut into
// strips of four stored rows; a strip keeps, per column, its four rows and the first row of the
// next strip (five rows), so the two rows r, r + 1 of a bilinear sample (r in [0, H]) always
// fall in strip r / 4.
//   density: record (strip s, column c), c in [0, W], holds the five rows of columns c and
//     c + 1 interleaved, (rho(c, 4s + k), rho(c + 1, 4s + k)) for k = 0..4 (ten values), so
//     the four taps of a sample are one 16-byte load at ((s (W + 1) + c) * 5 + r % 4) * 2;
//   gradient: record (s, c), c in [0, W + 1], holds the five rows of column c (five (x, y)
//     pairs), so a sample's taps are two 16-byte loads at (s (W + 2) + c) * 5 + r % 4 and five
//     pairs on.
// A 128-byte line then covers about 3 x 4 sample positions of either map, which the samples
// around a point share.
__host__ __device__ inline int64_t strip_rows(int32_t H) { return (int64_t)(H >> 2) + 1; }
__host__ __device__ inline int64_t rho_strip_plane(int32_t W, int32_t H) {
    return strip_rows(H) * (W + 1) * 10;      // floats per layer
}
__host__ __device__ inline int64_t grad_strip_plane(int32_t W, int32_t H) {
    return strip_rows(H) * (W + 2) * 5;       // (x, y) pairs per layer
}

// One graph of one iteration. Every kernel takes an array of these (one per graph of a
// batch) and finds its graph from blockIdx via the blk_* prefixes, so a single graph is
// a batch of one.
struct GDesc {
    // first block of this graph in each launch shape
    int64_t blk_edge;    // one wave per edge, kWavesPerBlock edges per block
    int64_t blk_scan;    // one block per scan tile
    int64_t blk_row;     // one block per map row (B * H rows)
    int64_t blk_col;     // one thread per (group, row segment, column)
    int64_t blk_px;      // one thread per pixel (W * H)
    int64_t blk_pxb;     // one thread per layer pixel (B * W * H)
    int64_t blk_edget;   // one thread per edge
    int64_t blk_tile;    // tile-histogram blocks (tile_blocks per graph)
    int64_t blk_strip;   // one thread per gradient strip pair (B * grad_strip_plane(W, H))

    int64_t n_edges;
    int64_t cap;         // capacity of the point buffers, in points
    int32_t B, W, H, P;
    int32_t r, K, record, wmax;
    double h, eps, s, delta;
    double doff;                // directed offset of interior samples along the left normal
    int32_t strip;              // 1: histogram of the drawn line strips (entries per pixel drawn)
    int32_t insdel;             // 1: insert/delete resampling (k_insdel) instead of the uniform one
    int32_t count_given;        // 1: k_bin_samples<false> counts this graph's samples in tiles
    int32_t narrow;             // 1: unit edge weights, entries are 16-bit (pixel in the tile only)
    double dmin;                // removal spacing of the insert/delete resampling
    int64_t ent_cap;            // capacity of bins, in entries (cap for the point splat)
    double a[HB_MAX_PASSES];    // density weight of each pass
    double ck[HB_MAX_PASSES];   // prod_{q<=k} (2 r_q + 1)^2: the normalisation of pass k
    int32_t rp[HB_MAX_PASSES];  // box radius of every pass

    const int32_t *order;       // edge order of the advection kernels (by group, then position;
                                // dealt round-robin; nullptr: 0..E-1)
    const int32_t *group;
    const int32_t *weight;      // nullptr: unit weights
    const float *M;             // B x B, M[l * B + b]

    const float2 *pin;          // polylines read by resampling
    const int64_t *off_in;      // their offsets
    float2 *samples;            // sample points written by resampling / read by advection
    int64_t *off_s;             // sample offsets (also the offsets of the new polylines)
    float2 *pnew;               // new polylines written by advection + smoothing

    int64_t *counts;            // per edge: sample count of the next resampling
    double *lens;               // per edge: length of the polyline the counts come from
    int64_t *tsum;              // per scan tile partial sums
    int64_t *total;             // sample count of this iteration (device scalar)

    int32_t *hist;              // [B][H][W] histogram (sum of the per-XCD copies)
    int32_t *histx;             // [nx][B][H][W] per-XCD copies the splat kernels add into
    int32_t nx;                 // number of copies (XCDs of the device)
    int32_t nxcd;               // XCDs of the device (block-to-edge mapping)

    // spatial binning: tile t = (layer * tiles_y + ty) * tiles_x + tx
    int32_t tiles_x, tiles_y, n_tiles, tile_blocks;
    int32_t n_sets;             // counter sets (power of two): edge block b counts in set b % n_sets
    int32_t col_rows;           // rows per thread of the column box pass
    int64_t item_entries;       // entries per tile-histogram work item
    int64_t *bin_cnt;           // [n_sets][n_tiles] samples per tile, per set of edge blocks
    int64_t *bin_cur;           // [n_sets][n_tiles] write cursors of the binning pass
    int64_t *tile_off;          // [n_tiles + 1] first entry of each tile
    int64_t *seg_off;           // [n_tiles + 1] first work item (kSegEntries entries) of each tile
    uint32_t *bins;             // [ent_cap] entries: pixel in tile | edge weight << kLocalBits
                                // (narrow: [ent_cap] uint16 pixels in tile, weight 1)
    uint32_t *bin_src;          // [cap] sample of each entry (runs that record it; else null)
    int64_t *box;               // [P][B][H][W]
    int64_t *tmp;               // [B][H][W] row-pass output
    float *rho;                 // [B][H][W]
    float2 *grad;               // [B][H][W]
    // strip maps of rho and grad (bilinear taps clamped into the grid; see strip_rows)
    float *rhos;                // [B][rho_strip_plane]
    float2 *grads;              // [B][grad_strip_plane]
    int8_t *jacc;               // [cap] accepted halving per sample (record != 0)
    int32_t *status;

    // adjoint of one iteration (frozen decisions)
    const float2 *adj_in;       // adjoint of this stage's output points
    const float2 *ink_pts;      // if set: the output points are the final polylines and their
                                // adjoint is the gradient of the ink, computed in place
    float2 *adj_out;            // adjoint of this stage's input points
    // D_bk = grad(pass k of group b) / (2r+1)^(2k); records padded to an even float2 count
    float2 *gbm;                // [H][W][bp]: sum_k a_k D_bk for every group b (all layers)
    float2 *gkm;                // [B][H][W][pp]: sum_b M[l][b] D_bk for every pass k, layer l
    int32_t bp, pp;             // record lengths in float2 (B and P rounded up to even)
    // parameter gradients, tile by tile: the samples of the iteration binned by histogram
    // tile (checkpointed bins), m v of every sample from the advection adjoint, a fixed-point
    // splat of w m v per tile in LDS and its contraction with the gradient-map records
    const uint32_t *abin_src;   // [N] checkpointed sample of each entry, in tile order
    const int64_t *atile_off;   // [n_tiles + 1] checkpointed first entry of each tile
    const int64_t *aseg_off;    // [n_tiles + 1] checkpointed first work item of each tile
    float2 *mv;                 // [N] m v of every sample (zero where it does not move)
    uint32_t *mvmax;            // largest |component| of m v (bits of a non-negative float)
    double *partials;           // [B + P][n_items] parameter partials of each work item
    int64_t max_items;          // capacity of partials per parameter
    double *red;                // [B*B + P][kRedSlices] slice sums of the reduction
    double *grad_param;         // [B*B + P] accumulated dL/dM (row-major) and dL/da
};

// Launch-shape block counts of one graph (host side).
struct Shape {
    int64_t edge, scan, row, col, px, pxb, edget, tile, strip;
};
// Launch shapes that the autotuner may change, per context: rows per thread of the column
// box pass, the most tile-count sets (privatised copies of the tile counters) and the
// entries per tile-histogram work item.
struct Tiling {
    int32_t col_rows = kColSeg;
    int32_t sets_max = kBinSetsMax;
    int64_t item_entries = kSegEntries;
};
Shape shape_of(int64_t n_edges, int32_t B, int32_t W, int32_t H, const Tiling &tg);

// Tiling of the B histogram layers of a W x H grid.
struct Tiles {
    int32_t x, y, n, blocks, sets;
};
Tiles tiles_of(int32_t B, int32_t W, int32_t H, int32_t sets_max);

// Launchers (all asynchronous on `st`). desc points to device memory holding ng
// descriptors; tot is the sum of the per-graph shapes.
hipError_t launch_init_state(const GDesc *desc, int ng, const Shape &tot, const float2 *nodes,
                             const int32_t *src, const int32_t *dst, double x0, double y0,
                             double x1, double y1, hipStream_t st);
hipError_t launch_lengths(const GDesc *desc, int ng, const Shape &tot, hipStream_t st);
hipError_t launch_scan(const GDesc *desc, int ng, const Shape &tot, hipStream_t st);
// u: chunks of 64 segments (resampling) / 62 points (advection) per trip: 1, 2 or 4;
// directed: some graph of the launch has a directed offset (the push is compiled in)
hipError_t launch_resample_count(const GDesc *desc, int ng, const Shape &tot, int u,
                                 bool directed, hipStream_t st);
hipError_t launch_count_given(const GDesc *desc, int ng, const Shape &tot, hipStream_t st);
// insert/delete resampling: sample counts of the current polylines (write = false, into
// counts) or the samples (write = true, at off_s)
hipError_t launch_insdel(const GDesc *desc, int ng, const Shape &tot, bool write, hipStream_t st);
// tile counts (scatter = false) or entries (scatter = true) of the drawn line strips
hipError_t launch_strip_bins(const GDesc *desc, int ng, const Shape &tot, bool scatter,
                             hipStream_t st);
// tile offsets, binning of the samples and the tile histograms (three kernels)
// (strip / points: some graph of the batch uses the line-strip / the point splat)
hipError_t launch_bin_hist(const GDesc *desc, int ng, const Shape &tot, bool strip, bool points,
                           hipStream_t st);
hipError_t launch_clear_hist(const GDesc *desc, int ng, const Shape &tot, hipStream_t st);
hipError_t launch_box_pass(const GDesc *desc, int ng, const Shape &tot, int max_w, int pass,
                           hipStream_t st);
hipError_t launch_density_grad(const GDesc *desc, int ng, const Shape &tot, int bmax,
                               hipStream_t st);
// density and gradient, then their strip maps (what the advection reads)
hipError_t launch_density_strips(const GDesc *desc, int ng, const Shape &tot, int bmax,
                                 hipStream_t st);
hipError_t launch_advect_smooth(const GDesc *desc, int ng, const Shape &tot, int u,
                                hipStream_t st);
hipError_t launch_fill_totals(const GDesc *desc, int ng, int T, hipStream_t st);
// orientation slice in [0, 4) of every edge, from the end points of its polyline
hipError_t launch_orientation(const GDesc *desc, const Shape &tot, int32_t *group, hipStream_t st);
// grouping (k-means on edge features, Davies-Bouldin index)
hipError_t launch_edge_features(const GDesc *desc, int64_t E, int kind, float *out, hipStream_t st);
hipError_t launch_km_gather(const float *X, int dim, int k, const int64_t *idx, double *centers,
                            hipStream_t st);
// one assignment round (mode 0), or the sums of the given labels (mode 1: coordinates and
// squared distances, mode 2: distances); tot receives k (dim+1) + 2 fixed-order sums (the
// clusters, the squared distances, the changed or out-of-range labels)
hipError_t launch_km_round(const float *X, int64_t n, int dim, int k, const double *centers,
                           int32_t *labels, int mode, double *part, double *tot, hipStream_t st);
hipError_t launch_km_means(const double *tot, int dim, int k, int keep, double *centers,
                           hipStream_t st);
hipError_t launch_km_db(const double *tot, const double *centers, int dim, int k, double *db,
                        hipStream_t st);
// acc[0..w) = tot (first) or acc + tot: the sums of the point chunks, added in chunk order
hipError_t launch_km_accum(double *acc, const double *tot, int w, int first, hipStream_t st);
// x[0..n) = 0
hipError_t launch_zero_d(double *x, int n, hipStream_t st);
// ink = sum of n polyline lengths, fixed order; part[kInkSlices] receives it (device)
hipError_t launch_ink(const double *lens, int64_t n, double *part, hipStream_t st);

// Adjoint kernels (one graph per launch).
hipError_t launch_adj_maps(const GDesc *desc, const Shape &tot, int bmax, hipStream_t st);
hipError_t launch_adj_advect(const GDesc *desc, const Shape &tot, hipStream_t st);
hipError_t launch_adj_params(const GDesc *desc, const Shape &tot, int bmax, hipStream_t st);
hipError_t launch_adj_resample(const GDesc *desc, const Shape &tot, hipStream_t st);
hipError_t launch_adj_reduce(const GDesc *desc, int B, int P, hipStream_t st);

}  // namespace hb
