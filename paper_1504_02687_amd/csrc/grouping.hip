// Grouping of the edges (Section 5): edge features, Lloyd's k-means and the Davies-Bouldin
// index on the GPU. Bins can be found by k-means on an edge property with the Euclidean
// distance, the number of bins being the one with the lowest Davies-Bouldin index over
// several random initialisations. One thread per point; every reduction over points is
// a fixed-order block reduction followed by a fixed-order sum over blocks, so the results
// are bit-reproducible.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace hb {

// Squared distance summed over the coordinates in order, every operation rounded on its own.
__device__ __forceinline__ double km_sqdist(const float *x, const double *c, int dim) {
    double s = 0.0;
    for (int j = 0; j < dim; ++j) {
        const double t = sub_rn((double)x[j], c[j]);
        s = add_rn(s, mul_rn(t, t));
    }
    return s;
}

// Sum over the block of one double per thread, in a fixed order: wave scans, then the four
// wave totals in order. The result is returned to every thread.
__device__ __forceinline__ double block_sum_d(double v) {
    __shared__ double ws[kWavesPerBlock];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const double w = last_lane(wave_incl_scan<double>(v, lane));
    if (lane == 0) ws[wid] = w;
    __syncthreads();
    double s = ws[0];
#pragma unroll
    for (int q = 1; q < kWavesPerBlock; ++q) s += ws[q];
    __syncthreads();
    return s;
}

// Sum over the wave of one double per lane (fixed DPP order), in every lane.
__device__ __forceinline__ double wave_sum_d(double v) {
    return last_lane(wave_incl_scan<double>(v, (int)(threadIdx.x & 63)));
}

// Edge features from the end points of the current polylines (pixel units): kind 0 origin
// (x_s, y_s), 1 destination (x_t, y_t), 2 both (x_s, y_s, x_t, y_t), 3 the distance from
// origin to destination (FP64, rounded to FP32). One thread per edge.
__global__ __launch_bounds__(kBlock) void k_edge_features(const GDesc *__restrict__ gd, int kind,
                                                          float *out) {
    const GDesc &d = gd[0];
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= d.n_edges) return;
    const float2 a = d.pin[d.off_in[e]], b = d.pin[d.off_in[e + 1] - 1];
    if (kind == 0) {
        out[2 * e] = a.x;
        out[2 * e + 1] = a.y;
    } else if (kind == 1) {
        out[2 * e] = b.x;
        out[2 * e + 1] = b.y;
    } else if (kind == 2) {
        out[4 * e] = a.x;
        out[4 * e + 1] = a.y;
        out[4 * e + 2] = b.x;
        out[4 * e + 3] = b.y;
    } else {
        const double dx = sub_rn((double)b.x, (double)a.x), dy = sub_rn((double)b.y, (double)a.y);
        out[e] = (float)sqrt(add_rn(mul_rn(dx, dx), mul_rn(dy, dy)));
    }
}

// Centres of a k-means start: rows idx[0..k) of X.
__global__ __launch_bounds__(kBlock) void k_km_gather(const float *X, int dim, int k,
                                                      const int64_t *idx, double *centers) {
    for (int t = threadIdx.x; t < k * dim; t += kBlock) centers[t] = (double)X[idx[t / dim] * dim + t % dim];
}

// One Lloyd assignment over the points (mode 0): each point to its nearest centre (ties to
// the lower index); or (mode 1) the given labels kept, labels outside [0, k) left out. Per
// wave (64 points, row blockIdx * 4 + wave of part): part[row][c][0..dim) the coordinate
// sums of cluster c, part[row][c][dim] its count, part[row][k (dim+1)] the sum of the squared
// distances to the assigned centres and part[row][k (dim+1) + 1] the number of labels that
// changed (mode 0) or were out of range (modes 1, 2); with mode 2, part[row][c][0] is
// instead the sum of the distances (square roots) of the points of c.
__global__ __launch_bounds__(kBlock) void k_km_assign(const float *__restrict__ X, int64_t n,
                                                      int dim, int k,
                                                      const double *__restrict__ centers,
                                                      int32_t *__restrict__ labels, int mode,
                                                      double *__restrict__ part) {
    __shared__ double cen[kKmMaxK * kKmMaxDim];
    for (int i = threadIdx.x; i < k * dim; i += kBlock) cen[i] = centers[i];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool in = i < n;
    float x[kKmMaxDim];
#pragma unroll
    for (int j = 0; j < kKmMaxDim; ++j) x[j] = (in && j < dim) ? X[i * dim + j] : 0.0f;
    int lab = -1;
    double bd = 0.0;
    if (in) {
        if (mode == 0) {
            lab = 0;
            bd = km_sqdist(x, cen, dim);
            for (int c = 1; c < k; ++c) {
                const double dd = km_sqdist(x, cen + c * dim, dim);
                if (dd < bd) {
                    bd = dd;
                    lab = c;
                }
            }
        } else {
            lab = labels[i];
            if (lab >= 0 && lab < k) {
                bd = km_sqdist(x, cen + lab * dim, dim);
                if (mode == 2) bd = sqrt(bd);
            }
        }
    }
    // mode 0: labels that changed; modes 1 and 2: labels outside [0, k) (left out of the sums)
    bool flag;
    if (mode == 0) {
        flag = in && labels[i] != lab;
        if (in) labels[i] = lab;
    } else {
        flag = in && (lab < 0 || lab >= k);
        if (flag) lab = -1;
    }
    const double nflag = (double)__builtin_popcountll(__ballot(flag));
    // the wave's sums: its points, labels and distances through LDS; lane t adds value t
    // (cluster t / (dim+1), coordinate t % (dim+1), the count at dim; the last value the
    // squared distances) over the 64 points in order
    __shared__ float sx[kWavesPerBlock][64][kKmMaxDim];
    __shared__ int32_t sl[kWavesPerBlock][64];
    __shared__ double sd[kWavesPerBlock][64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < kKmMaxDim; ++j) sx[wid][lane][j] = x[j];
    sl[wid][lane] = lab;
    sd[wid][lane] = bd;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);   // LDS writes of the wave done before the reads
    const int w = k * (dim + 1) + 2;
    double *out = part + ((int64_t)blockIdx.x * kWavesPerBlock + wid) * w;
    if (lane == 0) out[w - 1] = nflag;
    for (int t = lane; t < w - 1; t += 64) {
        double s = 0.0;
        if (t == w - 2) {
            if (mode != 2)
                for (int p = 0; p < 64; ++p) s += sd[wid][p];
        } else {
            const int c = t / (dim + 1), j = t - c * (dim + 1);
            for (int p = 0; p < 64; ++p) {
                if (sl[wid][p] != c) continue;
                if (j == dim) s += 1.0;
                else if (mode == 2) s += j == 0 ? sd[wid][p] : 0.0;
                else s += (double)sx[wid][p][j];
            }
        }
        out[t] = s;
    }
}

// Sum of the per-wave partials over the rows, in a fixed order: one block per value t;
// thread i adds rows [i S, (i+1) S) in order, then the block adds the 256 thread sums.
__global__ __launch_bounds__(kBlock) void k_km_reduce(const double *__restrict__ part, int64_t rows,
                                                      int w, double *__restrict__ tot) {
    const int t = blockIdx.x;
    const int64_t S = (rows + kBlock - 1) / kBlock;
    const int64_t r0 = (int64_t)threadIdx.x * S, r1 = r0 + S < rows ? r0 + S : rows;
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) s += part[r * w + t];
    s = block_sum_d(s);
    if (threadIdx.x == 0) tot[t] = s;
}

// New centres: the mean of every cluster with points; a cluster without points keeps its
// centre (keep = 1) or gets the origin (keep = 0).
__global__ __launch_bounds__(kBlock) void k_km_means(const double *__restrict__ tot, int dim, int k,
                                                     int keep, double *__restrict__ centers) {
    for (int t = threadIdx.x; t < k * dim; t += kBlock) {
        const int c = t / dim, j = t - c * dim;
        const double cnt = tot[c * (dim + 1) + dim];
        if (cnt > 0.0) centers[t] = tot[c * (dim + 1) + j] / cnt;
        else if (!keep) centers[t] = 0.0;
    }
}

// Davies-Bouldin index from the centroids, the distance sums (tot[c (dim+1)]) and counts
// (tot[c (dim+1) + dim]) of the clusters: the mean over non-empty clusters a of the largest
// (s_a + s_b) / |c_a - c_b| over the other non-empty clusters b (0 for coincident
// centroids); 0 with fewer than two clusters. One block, one thread per cluster.
__global__ __launch_bounds__(kBlock) void k_km_db(const double *__restrict__ tot,
                                                  const double *__restrict__ centers, int dim,
                                                  int k, double *db) {
    __shared__ double worst[kKmMaxK];
    __shared__ int used[kKmMaxK];
    const int a = threadIdx.x;
    if (a < k) {
        const double ca = tot[a * (dim + 1) + dim];
        double wv = 0.0;
        if (ca > 0.0) {
            const double sa = tot[a * (dim + 1)] / ca;
            for (int b = 0; b < k; ++b) {
                const double cb = tot[b * (dim + 1) + dim];
                if (b == a || !(cb > 0.0)) continue;
                double d2 = 0.0;
                for (int j = 0; j < dim; ++j) {
                    const double t = sub_rn(centers[a * dim + j], centers[b * dim + j]);
                    d2 = add_rn(d2, mul_rn(t, t));
                }
                const double dd = sqrt(d2);
                const double r = dd > 0.0 ? (sa + tot[b * (dim + 1)] / cb) / dd : 0.0;
                if (r > wv) wv = r;
            }
        }
        worst[a] = wv;
        used[a] = ca > 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int u = 0;
        double s = 0.0;
        for (int q = 0; q < k; ++q) {
            if (!used[q]) continue;
            ++u;
            s += worst[q];
        }
        *db = u > 1 ? s / (double)u : 0.0;
    }
}

// Chunk sums added in chunk order (one thread per value).
__global__ __launch_bounds__(kBlock) void k_km_accum(double *__restrict__ acc,
                                                     const double *__restrict__ tot, int w,
                                                     int first) {
    for (int t = threadIdx.x; t < w; t += kBlock) acc[t] = first ? tot[t] : acc[t] + tot[t];
}

__global__ __launch_bounds__(kBlock) void k_zero_d(double *__restrict__ x, int n) {
    for (int t = threadIdx.x; t < n; t += kBlock) x[t] = 0.0;
}

// ---------------------------------------------------------------- launchers

hipError_t launch_edge_features(const GDesc *desc, int64_t E, int kind, float *out, hipStream_t st) {
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_edge_features, dim3((unsigned)((E + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       st, desc, kind, out);
    return hipGetLastError();
}

hipError_t launch_km_gather(const float *X, int dim, int k, const int64_t *idx, double *centers,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_km_gather, dim3(1), dim3(kBlock), 0, st, X, dim, k, idx, centers);
    return hipGetLastError();
}

hipError_t launch_km_round(const float *X, int64_t n, int dim, int k, const double *centers,
                           int32_t *labels, int mode, double *part, double *tot, hipStream_t st) {
    const int64_t nblk = (n + kBlock - 1) / kBlock;
    if (nblk <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_km_assign, dim3((unsigned)nblk), dim3(kBlock), 0, st, X, n, dim, k, centers,
                       labels, mode, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int w = k * (dim + 1) + 2;
    hipLaunchKernelGGL(k_km_reduce, dim3((unsigned)w), dim3(kBlock), 0, st, part,
                       nblk * kWavesPerBlock, w, tot);
    return hipGetLastError();
}

hipError_t launch_km_means(const double *tot, int dim, int k, int keep, double *centers,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_km_means, dim3(1), dim3(kBlock), 0, st, tot, dim, k, keep, centers);
    return hipGetLastError();
}

hipError_t launch_km_db(const double *tot, const double *centers, int dim, int k, double *db,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_km_db, dim3(1), dim3(kBlock), 0, st, tot, centers, dim, k, db);
    return hipGetLastError();
}

hipError_t launch_km_accum(double *acc, const double *tot, int w, int first, hipStream_t st) {
    hipLaunchKernelGGL(k_km_accum, dim3(1), dim3(kBlock), 0, st, acc, tot, w, first);
    return hipGetLastError();
}

hipError_t launch_zero_d(double *x, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_d, dim3(1), dim3(kBlock), 0, st, x, n);
    return hipGetLastError();
}

}  // namespace hb
