/*
 * Plain FP64 CPU oracle of one iteration of 3D-density-histogram edge bundling
 * (Moura, "3D Density Histograms for Criteria-driven Edge Bundling", arXiv 1504.02687).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, obviously correct statement of
 * what the GPU path computes. Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load it. It shares no code, header, table or helper with
 * the GPU library, and the GPU library never calls it.
 *
 * Conventions (the readings of the paper that the GPU path follows too):
 *   - points are in pixel units; pixel (u,v) covers [u,u+1) x [v,v+1);
 *   - polylines are stored in CSR form: off[E+1] (int64) and xy[2*N] (x,y interleaved);
 *   - maps are [B][H][W] row-major, index (b*H + v)*W + u;
 *   - every function is a direct loop over its definition: no blocking or fusion.
 *
 * Parity pins: every function here is pinned by the CPU tests against closed forms,
 * brute force or invariants (see the header comment of each function). The
 * whole-method behaviour against the paper's drawings is parity unpinned: the
 * paper's figures and datasets are not available.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EXPORT __attribute__((visibility("default")))

EXPORT double orc_bilinear(int32_t W, int32_t H, const double *map, int32_t stride, int32_t comp,
                           double x, double y);

/* ------------------------------------------------------------------ threads */

EXPORT int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

EXPORT void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------ O7: iteration schedule (Sec. 3.3)
 * The bandwidth decays geometrically, h_i = lambda^i * h_max (Sec. 2.1 and 3.3), with
 * h_max a multiple of sigma (2 sigma in the paper's convergence figure).
 * Reading: sigma of P passes of a (2r+1)-wide box is the standard deviation of the
 * P-fold convolution of a discrete uniform on {-r..r}: each has variance r(r+1)/3,
 * so sigma^2 = P r (r+1) / 3.
 * Pins: the variance of the P-pass impulse response computed by the box chain.
 */
EXPORT double orc_sigma(int r, int passes) {
    return sqrt((double)passes * (double)r * (double)(r + 1) / 3.0);
}

EXPORT double orc_bandwidth(int iter, double h_max, double lambda) {
    double h = h_max;
    for (int i = 0; i < iter; ++i) h *= lambda;
    return h;
}

/* ------------------------------------------------ O1: resampling (Sec. 2.1, Sec. 3)
 * Edges are polylines of sample points spaced by the sampling step delta with fixed
 * end points; at the start of every iteration each polyline is resampled so that its
 * points are equally spaced again. Reading: uniform arclength, n = max(1, ceil(L/delta))
 * + 1 points, point k at arclength k L / (n-1), linear interpolation on the segment
 * that holds that arclength, end points copied exactly.
 * Pins: closed form on straight segments, exact end points, counts of axis-aligned
 * integer-length edges, idempotence on already uniform polylines.
 */
EXPORT double orc_polyline_length(const double *xy, int64_t m) {
    double L = 0.0;
    for (int64_t j = 0; j + 1 < m; ++j) {
        double dx = xy[2 * (j + 1)] - xy[2 * j];
        double dy = xy[2 * (j + 1) + 1] - xy[2 * j + 1];
        L += sqrt(dx * dx + dy * dy);
    }
    return L;
}

EXPORT int64_t orc_sample_count(double L, double delta) {
    double q = ceil(L / delta);
    int64_t n = (int64_t)q;
    if (n < 1) n = 1;
    return n + 1;
}

/* Per-edge lengths and sample counts of the polylines (off, xy); returns the total. */
EXPORT int64_t orc_resample_counts(int64_t E, const int64_t *off, const double *xy,
                                   double delta, int64_t *counts, double *lens) {
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : total)
    for (int64_t e = 0; e < E; ++e) {
        double L = orc_polyline_length(xy + 2 * off[e], off[e + 1] - off[e]);
        lens[e] = L;
        counts[e] = orc_sample_count(L, delta);
        total += counts[e];
    }
    return total;
}

/* Resample every polyline into off_out/xy_out; lens[] are the lengths from above. seg (may
 * be NULL) receives, for every sample, the index within its edge of the segment it was
 * interpolated on (-1 for the two end points). */
EXPORT void orc_resample(int64_t E, const int64_t *off_in, const double *xy_in,
                         const int64_t *off_out, const double *lens, double *xy_out,
                         int64_t *seg) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t e = 0; e < E; ++e) {
        const double *p = xy_in + 2 * off_in[e];
        int64_t m = off_in[e + 1] - off_in[e];
        double *o = xy_out + 2 * off_out[e];
        int64_t n = off_out[e + 1] - off_out[e];
        double L = lens[e];
        o[0] = p[0];
        o[1] = p[1];
        o[2 * (n - 1)] = p[2 * (m - 1)];
        o[2 * (n - 1) + 1] = p[2 * (m - 1) + 1];
        if (seg) {
            seg[off_out[e]] = -1;
            seg[off_out[e] + n - 1] = -1;
        }
        int64_t j = 0;          /* current segment (p_j, p_j+1) */
        double C = 0.0;         /* arclength at p_j */
        double ell = hypot(p[2] - p[0], p[3] - p[1]);
        for (int64_t k = 1; k + 1 < n; ++k) {
            double s = (double)k * L / (double)(n - 1);
            /* move to the last segment whose start arclength is <= s */
            while (j < m - 2 && C + ell <= s) {
                C += ell;
                ++j;
                ell = hypot(p[2 * (j + 1)] - p[2 * j], p[2 * (j + 1) + 1] - p[2 * j + 1]);
            }
            double t = ell > 0.0 ? (s - C) / ell : 0.0;
            if (t < 0.0) t = 0.0;
            if (t > 1.0) t = 1.0;
            o[2 * k] = p[2 * j] + t * (p[2 * (j + 1)] - p[2 * j]);
            o[2 * k + 1] = p[2 * j + 1] + t * (p[2 * (j + 1) + 1] - p[2 * j + 1]);
            if (seg) seg[off_out[e] + k] = j;
        }
    }
}

/* Insert/delete resampling (the variant of Sec. 3, the pipeline: each iteration starts by
 * creating sample points where consecutive points are too far apart and removing them where
 * they are too close). Reading, with spacings dmin < dmax: an interior point is removed when
 * it lies closer than dmin to its predecessor in the input polyline (squared distances
 * compared in FP64); the end points stay. Between consecutive kept points a, b the gap
 * g = |b - a| (FP64) is cut into c = max(1, ceil(g / dmax)) equal parts: a, then the c - 1
 * points a + (t / c)(b - a), t = 1 .. c-1; the last kept point closes the polyline. From a
 * straight two-point edge this is the uniform resampling with delta = dmax.
 * Pins: every gap of the result is at most dmax; every input point at least dmin from its
 * predecessor is in the result, and every removed one was closer; a uniform polyline with
 * spacing in [dmin, dmax] is a fixed point; closed forms on collinear points; equality with
 * the uniform resampling on two-point edges.
 */
static int32_t insdel_keep(const double *p, int64_t j, int64_t m, double dmin) {
    if (j == 0 || j == m - 1) return 1;
    double dx = p[2 * j] - p[2 * (j - 1)], dy = p[2 * j + 1] - p[2 * (j - 1) + 1];
    return dx * dx + dy * dy >= dmin * dmin;
}

static int64_t insdel_parts(const double *a, const double *b, double dmax) {
    double dx = b[0] - a[0], dy = b[1] - a[1];
    double g = sqrt(dx * dx + dy * dy);
    double c = ceil(g / dmax);
    return c < 1.0 ? 1 : (int64_t)c;
}

EXPORT int64_t orc_insdel_counts(int64_t E, const int64_t *off, const double *xy, double dmin,
                                 double dmax, int64_t *counts) {
    int64_t total = 0;
    for (int64_t e = 0; e < E; ++e) {
        const double *p = xy + 2 * off[e];
        int64_t m = off[e + 1] - off[e];
        int64_t n = 0, last = 0;
        for (int64_t j = 1; j < m; ++j) {
            if (!insdel_keep(p, j, m, dmin)) continue;
            n += insdel_parts(p + 2 * last, p + 2 * j, dmax);
            last = j;
        }
        counts[e] = n + 1;
        total += n + 1;
    }
    return total;
}

EXPORT void orc_insdel(int64_t E, const int64_t *off_in, const double *xy_in, double dmin,
                       double dmax, const int64_t *off_out, double *xy_out) {
    for (int64_t e = 0; e < E; ++e) {
        const double *p = xy_in + 2 * off_in[e];
        int64_t m = off_in[e + 1] - off_in[e];
        double *o = xy_out + 2 * off_out[e];
        int64_t k = 0, last = 0;
        for (int64_t j = 1; j < m; ++j) {
            if (!insdel_keep(p, j, m, dmin)) continue;
            const double *a = p + 2 * last, *b = p + 2 * j;
            int64_t c = insdel_parts(a, b, dmax);
            for (int64_t t = 0; t < c; ++t) {
                double f = (double)t / (double)c;
                o[2 * k] = a[0] + f * (b[0] - a[0]);
                o[2 * k + 1] = a[1] + f * (b[1] - a[1]);
                ++k;
            }
            last = j;
        }
        o[2 * k] = p[2 * (m - 1)];
        o[2 * k + 1] = p[2 * (m - 1) + 1];
    }
}

/* ------------------------------------------------ directed graphs (Sec. 3, the pipeline)
 * For directed graphs whose bundling criterion follows the flow direction, every sample
 * except the two end points is pushed sideways by a fixed distance along the normal of the
 * edge at that sample, so that edges running in opposite directions part at once.
 * Reading: the normal is that of the polyline segment the sample was interpolated on (the
 * segment index seg from orc_resample, taken in the input polyline), on its left-hand side:
 * (-t_y, t_x) for the unit direction t of the segment, oriented from source to target; the
 * signed distance d is in pixels; the push is applied to a set of samples straight after
 * their resampling and before the histogram. The pipeline pushes once, after the first
 * sampling, and then loops from the resampling, which interpolates along the pushed
 * polyline and so keeps the offset; the loop (oracle/__init__.py, iterate) applies it in
 * iteration 0 only, or after every resampling when asked to.
 * Pins: closed form on straight edges (interior samples at signed distance d from the line,
 * the along-edge coordinate unchanged), edges in opposite directions part by 2|d|, d = 0 is
 * the identity, a rotation by 90 degrees commutes with the push.
 */
EXPORT void orc_directed_offset(int64_t E, const int64_t *off_in, const double *xy_in,
                                const int64_t *off_out, const int64_t *seg, double d,
                                double *xy) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t e = 0; e < E; ++e) {
        const double *p = xy_in + 2 * off_in[e];
        for (int64_t i = off_out[e] + 1; i + 1 < off_out[e + 1]; ++i) {
            int64_t j = seg[i];
            double ex = p[2 * (j + 1)] - p[2 * j];
            double ey = p[2 * (j + 1) + 1] - p[2 * j + 1];
            double len = sqrt(ex * ex + ey * ey);
            if (len == 0.0) continue;      /* no direction: the sample stays */
            double tx = ex / len, ty = ey / len;
            xy[2 * i] = xy[2 * i] + d * (-ty);
            xy[2 * i + 1] = xy[2 * i + 1] + d * tx;
        }
    }
}

/* ------------------------------------------------ orientation bins (Sec. 5)
 * Edges can be binned by orientation: the angle of the edge, discretised into 4 slices
 * centred on 0, 90, 180 and 270 degrees. Reading: the angle is that of the direction
 * (dx, dy) from source to target in grid coordinates, measured from +x towards +y; slice k
 * holds the angles in [90k - 45, 90k + 45) degrees; a zero direction is in slice 0.
 * Test of slice k: turning the direction by -90k degrees, (x, y) -> (y, -x) k times (exact
 * in floating point), must bring it into the slice around 0 degrees, angles in [-45, 45),
 * that is u > 0 and -u <= v < u for the turned direction (u, v).
 * Pins: atan2 on random directions away from the slice borders, the four axes, the four
 * diagonals (the border angles), a 90-degree turn adds 1 modulo 4, the zero direction.
 */
EXPORT void orc_orientation(int64_t n, const double *dxy, int32_t *bin) {
    for (int64_t i = 0; i < n; ++i) {
        double u = dxy[2 * i], v = dxy[2 * i + 1];
        int32_t found = 0;
        for (int32_t k = 0; k < 4; ++k) {
            if (u > 0.0 && -u <= v && v < u) {
                found = k;
                break;
            }
            double t = u;      /* turn by -90 degrees */
            u = v;
            v = -t;
        }
        bin[i] = found;
    }
}

/* ------------------------------------------------ frozen-decision surrogate (for gradients)
 * Holding the discrete choices of a base run fixed (sample counts, the segment each sample
 * is interpolated on, the histograms, the accepted halving of every point) makes one
 * iteration a piecewise smooth function of the positions, the interaction matrix and the
 * pass weights; its derivatives are what the adjoint computes.
 *
 * Resampling with frozen counts (off_out) and segment indices (seg): the arclengths are
 * recomputed from the current positions; t is clamped to [0, 1] as in orc_resample.
 */
EXPORT void orc_resample_frozen(int64_t E, const int64_t *off_in, const double *xy_in,
                                const int64_t *off_out, const int64_t *seg, double *xy_out) {
    for (int64_t e = 0; e < E; ++e) {
        const double *p = xy_in + 2 * off_in[e];
        int64_t m = off_in[e + 1] - off_in[e];
        double *o = xy_out + 2 * off_out[e];
        int64_t n = off_out[e + 1] - off_out[e];
        double L = orc_polyline_length(p, m);
        o[0] = p[0];
        o[1] = p[1];
        o[2 * (n - 1)] = p[2 * (m - 1)];
        o[2 * (n - 1) + 1] = p[2 * (m - 1) + 1];
        for (int64_t k = 1; k + 1 < n; ++k) {
            int64_t j = seg[off_out[e] + k];
            double C = orc_polyline_length(p, j + 1);     /* arclength at p_j */
            double ell = hypot(p[2 * (j + 1)] - p[2 * j], p[2 * (j + 1) + 1] - p[2 * j + 1]);
            double s = (double)k * L / (double)(n - 1);
            double t = ell > 0.0 ? (s - C) / ell : 0.0;
            if (t < 0.0) t = 0.0;
            if (t > 1.0) t = 1.0;
            o[2 * k] = p[2 * j] + t * (p[2 * (j + 1)] - p[2 * j]);
            o[2 * k + 1] = p[2 * j + 1] + t * (p[2 * (j + 1) + 1] - p[2 * j + 1]);
        }
    }
}

/* Advection with frozen accepted halvings jacc (-1: no move, -2: end point): the direction
 * is recomputed from the current maps and position (Eq. 5), the step is h / 2^jacc, and the
 * result is clamped like orc_advect. */
EXPORT void orc_advect_frozen(int64_t E, const int64_t *off, const double *xy, const int32_t *group,
                              int32_t W, int32_t H, const double *grad, double h,
                              const int32_t *jacc, double eps, double *xy_out) {
    int64_t plane = (int64_t)W * H;
    double xmax = (double)W - 1.0 / 256.0, ymax = (double)H - 1.0 / 256.0;
    for (int64_t e = 0; e < E; ++e) {
        const double *gl = grad + (int64_t)group[e] * plane * 2;
        for (int64_t i = off[e]; i < off[e + 1]; ++i) {
            double x = xy[2 * i], y = xy[2 * i + 1];
            xy_out[2 * i] = x;
            xy_out[2 * i + 1] = y;
            if (jacc[i] < 0) continue;
            double gx = orc_bilinear(W, H, gl, 2, 0, x, y);
            double gy = orc_bilinear(W, H, gl, 2, 1, x, y);
            double nrm = sqrt(gx * gx + gy * gy);
            double den = nrm > eps ? nrm : eps;
            double m = ldexp(h, -jacc[i]);
            double cx = x + m * gx / den, cy = y + m * gy / den;
            if (cx < 0.0) cx = 0.0;
            if (cx > xmax) cx = xmax;
            if (cy < 0.0) cy = 0.0;
            if (cy > ymax) cy = ymax;
            xy_out[2 * i] = cx;
            xy_out[2 * i + 1] = cy;
        }
    }
}

/* ------------------------------------------------ O2: splatting (Sec. 3.1 Eq. 1, Sec. 3.2 Eq. 3)
 * H(u,v,b) is the weighted count of edges of bin b present at pixel (u,v). Reading: every
 * sample point of an edge (end points included) adds the edge weight to the pixel that
 * contains it, index clamp(floor(x), 0, W-1), clamp(floor(y), 0, H-1). Mixing across bins
 * is applied after smoothing (linearity), so each point lands in one layer only.
 * Pins: total mass = sum of n_e * w_e, brute force, edge-permutation invariance, transpose.
 */
static int64_t clamp_index(double x, int64_t n) {
    double f = floor(x);
    if (f < 0.0) return 0;
    if (f > (double)(n - 1)) return n - 1;
    return (int64_t)f;
}

EXPORT void orc_splat(int64_t E, const int64_t *off, const double *xy, const int32_t *group,
                      const int32_t *weight, int32_t B, int32_t W, int32_t H, int64_t *hist) {
    memset(hist, 0, sizeof(int64_t) * (size_t)B * (size_t)W * (size_t)H);
    for (int64_t e = 0; e < E; ++e) {
        int64_t w = weight ? weight[e] : 1;
        int64_t b = group[e];
        for (int64_t k = off[e]; k < off[e + 1]; ++k) {
            int64_t u = clamp_index(xy[2 * k], W);
            int64_t v = clamp_index(xy[2 * k + 1], H);
            hist[(b * H + v) * W + u] += w;
        }
    }
}

/* Line-strip splat (the rasterised variant of Eq. 1): the paper's implementation draws
 * the edges with Bresenham's algorithm, drawing them into the histogram as lines.
 * Reading: the polyline of an edge is drawn as a line strip through the pixels of its
 * points (the pixel of a point as in orc_splat). Segment j, from pixel (u0, v0) to pixel
 * (u1, v1), draws the n = max(|u1 - u0|, |v1 - v0|) pixels t = 0 .. n-1 of the digital line
 * between them, (u0 + round(t (u1-u0) / n), v0 + round(t (v1-v0) / n)) with halves rounded
 * up, and not its last pixel, which starts the next segment; the last point's pixel is
 * drawn once at the end. Every drawn pixel adds the edge weight, so a pixel the strip
 * leaves and enters again counts again, and consecutive points in one pixel draw it once.
 * Pins: the strip is 8-connected and ends on the last point's pixel; mass = sum over edges
 * of w (1 + sum of n_j); on segments without a rounding tie the pixels are those of the
 * textbook (error-accumulator) Bresenham; every point's pixel is drawn (so the strip
 * histogram is >= the point histogram); a straight row gives one count per pixel.
 */
static int64_t floor_div(int64_t a, int64_t b) {   /* b > 0 */
    int64_t q = a / b;
    if (a % b != 0 && a < 0) q -= 1;
    return q;
}

EXPORT void orc_splat_strip(int64_t E, const int64_t *off, const double *xy, const int32_t *group,
                            const int32_t *weight, int32_t B, int32_t W, int32_t H, int64_t *hist) {
    memset(hist, 0, sizeof(int64_t) * (size_t)B * (size_t)W * (size_t)H);
    for (int64_t e = 0; e < E; ++e) {
        int64_t w = weight ? weight[e] : 1;
        int64_t *hb = hist + (int64_t)group[e] * H * W;
        if (off[e + 1] <= off[e]) continue;
        for (int64_t k = off[e]; k + 1 < off[e + 1]; ++k) {
            int64_t u0 = clamp_index(xy[2 * k], W), v0 = clamp_index(xy[2 * k + 1], H);
            int64_t u1 = clamp_index(xy[2 * k + 2], W), v1 = clamp_index(xy[2 * k + 3], H);
            int64_t du = u1 - u0, dv = v1 - v0;
            int64_t n = (du < 0 ? -du : du) > (dv < 0 ? -dv : dv) ? (du < 0 ? -du : du)
                                                                     : (dv < 0 ? -dv : dv);
            for (int64_t t = 0; t < n; ++t) {
                /* round(t du / n) with halves up = floor((2 t du + n) / (2 n)) */
                int64_t u = u0 + floor_div(2 * t * du + n, 2 * n);
                int64_t v = v0 + floor_div(2 * t * dv + n, 2 * n);
                hb[v * W + u] += w;
            }
        }
        int64_t kl = off[e + 1] - 1;
        hb[clamp_index(xy[2 * kl + 1], H) * W + clamp_index(xy[2 * kl], W)] += w;
    }
}

/* ------------------------------------------------ O3: box smoothing (Sec. 3.1)
 * The Gaussian of Eq. 2 is approximated by P repeated averaging (box) filters computed
 * from integral images. Reading: zero padding outside the grid and integer window sums;
 * the (2r+1)^2 divisors are applied once at the end (in the density step).
 * orc_box_brute is the literal window sum; orc_box_integral computes the same sums from
 * an integral image and its four corners. The tests require both to agree exactly.
 */
EXPORT void orc_box_brute(int32_t W, int32_t H, const int64_t *in, int32_t r, int64_t *out) {
    for (int64_t v = 0; v < H; ++v)
        for (int64_t u = 0; u < W; ++u) {
            int64_t acc = 0;
            for (int64_t dv = -r; dv <= r; ++dv)
                for (int64_t du = -r; du <= r; ++du) {
                    int64_t x = u + du, y = v + dv;
                    if (x >= 0 && x < W && y >= 0 && y < H) acc += in[y * W + x];
                }
            out[v * W + u] = acc;
        }
}

/* I has (H+1) x (W+1) entries; I(u,v) = sum of in(u',v') over u' < u, v' < v. */
EXPORT void orc_integral_image(int32_t W, int32_t H, const int64_t *in, int64_t *I) {
    int64_t W1 = (int64_t)W + 1;
    for (int64_t u = 0; u <= W; ++u) I[u] = 0;
    for (int64_t v = 0; v < H; ++v) {
        I[(v + 1) * W1] = 0;
        for (int64_t u = 0; u < W; ++u)
            I[(v + 1) * W1 + u + 1] = in[v * W + u] + I[v * W1 + u + 1] + I[(v + 1) * W1 + u]
                                      - I[v * W1 + u];
    }
}

EXPORT void orc_box_integral(int32_t W, int32_t H, const int64_t *in, int32_t r, int64_t *out) {
    int64_t W1 = (int64_t)W + 1;
    int64_t *I = (int64_t *)malloc(sizeof(int64_t) * (size_t)W1 * (size_t)(H + 1));
    orc_integral_image(W, H, in, I);
    for (int64_t v = 0; v < H; ++v) {
        int64_t v0 = v - r < 0 ? 0 : v - r;
        int64_t v1 = v + r + 1 > H ? H : v + r + 1;
        for (int64_t u = 0; u < W; ++u) {
            int64_t u0 = u - r < 0 ? 0 : u - r;
            int64_t u1 = u + r + 1 > W ? W : u + r + 1;
            out[v * W + u] = I[v1 * W1 + u1] - I[v0 * W1 + u1] - I[v1 * W1 + u0] + I[v0 * W1 + u0];
        }
    }
    free(I);
}

/* S[k][b] for k = 0..P-1 is pass k+1 applied to pass k (pass 0 input is hist[b]). */
EXPORT void orc_box_chain(int32_t B, int32_t W, int32_t H, int32_t P, int32_t r,
                          const int64_t *hist, int64_t *S, int32_t brute) {
    int64_t plane = (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t kb = 0; kb < B; ++kb) {
        const int64_t *src = hist + kb * plane;
        for (int64_t k = 0; k < P; ++k) {
            int64_t *dst = S + (k * B + kb) * plane;
            if (brute)
                orc_box_brute(W, H, src, r, dst);
            else
                orc_box_integral(W, H, src, r, dst);
            src = dst;
        }
    }
}

/* ------------------------------------------------ O4: density stack (Sec. 3.2 Eq. 3-4)
 * Layer l of the 3D density is the smoothed histogram of every bin b weighted by the
 * interaction matrix, rho_l = sum_b M[l][b] * Sbar_b (Eq. 3 with smoothing moved after
 * mixing, which is exact because the box chain is linear). Sbar_b = sum_k a_k S_b^k /
 * (2r+1)^(2k) normalises pass k to an average; the plain method uses a = (0,...,0,1).
 * Pins: M = identity gives each group's own map; B = 1 is the 2D method; permutation
 * equivariance in the group labels.
 */
EXPORT void orc_density(int32_t B, int32_t W, int32_t H, int32_t P, int32_t r, const int64_t *S,
                        const double *a, const double *M, double *rho) {
    int64_t plane = (int64_t)W * H;
    double c = (double)(2 * r + 1) * (double)(2 * r + 1);
#pragma omp parallel for schedule(static)
    for (int64_t px = 0; px < plane; ++px) {
        for (int64_t l = 0; l < B; ++l) {
            double acc = 0.0;
            for (int64_t b = 0; b < B; ++b) {
                double sbar = 0.0, ck = 1.0;
                for (int64_t k = 0; k < P; ++k) {
                    ck *= c;
                    sbar += a[k] * ((double)S[(k * B + b) * plane + px] / ck);
                }
                acc += M[l * B + b] * sbar;
            }
            rho[l * plane + px] = acc;
        }
    }
}

/* Box widths for a real sigma (the variant of the box chain for a radius that is not an
 * integer): the P passes mix two odd widths, following Kovesi's rule for almost-Gaussian
 * filtering with repeated boxes (P. Kovesi, "Fast almost-Gaussian filtering", 2010): the ideal
 * width w = sqrt(12 sigma^2 / P + 1), w_l the largest odd integer <= w, w_u = w_l + 2, and
 * m = round((12 sigma^2 - P w_l^2 - 4 P w_l - 3 P) / (-4 w_l - 4)) passes of w_l first, the
 * other P - m of w_u; radius = (width - 1) / 2. The variance of the chain is
 * sum_k r_k (r_k + 1) / 3.
 * Pins: a sigma that equal radii reach exactly gives those radii; the achieved sigma is close
 * to the requested one; the impulse response of the chain has the stated variance.
 */
EXPORT void orc_kovesi_radii(double sigma, int32_t P, int32_t *radii) {
    double wi = sqrt(12.0 * sigma * sigma / (double)P + 1.0);
    int64_t wl = (int64_t)floor(wi);
    if (wl % 2 == 0) wl -= 1;
    if (wl < 1) wl = 1;
    int64_t wu = wl + 2;
    double mi = (12.0 * sigma * sigma - (double)P * (double)(wl * wl) - 4.0 * (double)P * (double)wl -
                 3.0 * (double)P) / (-4.0 * (double)wl - 4.0);
    int64_t m = (int64_t)round(mi);
    if (m < 0) m = 0;
    if (m > P) m = P;
    for (int32_t k = 0; k < P; ++k) radii[k] = (int32_t)(((k < m ? wl : wu) - 1) / 2);
}

/* The box chain and the density with one radius per pass (pass k of radius radii[k]; the
 * normalisation of pass k is prod_{q <= k} (2 r_q + 1)^2). */
EXPORT void orc_box_chain_radii(int32_t B, int32_t W, int32_t H, int32_t P, const int32_t *radii,
                                const int64_t *hist, int64_t *S, int32_t brute) {
    int64_t plane = (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t kb = 0; kb < B; ++kb) {
        const int64_t *src = hist + kb * plane;
        for (int64_t k = 0; k < P; ++k) {
            int64_t *dst = S + (k * B + kb) * plane;
            if (brute)
                orc_box_brute(W, H, src, radii[k], dst);
            else
                orc_box_integral(W, H, src, radii[k], dst);
            src = dst;
        }
    }
}

EXPORT void orc_density_radii(int32_t B, int32_t W, int32_t H, int32_t P, const int32_t *radii,
                              const int64_t *S, const double *a, const double *M, double *rho) {
    int64_t plane = (int64_t)W * H;
#pragma omp parallel for schedule(static)
    for (int64_t px = 0; px < plane; ++px) {
        for (int64_t l = 0; l < B; ++l) {
            double acc = 0.0;
            for (int64_t b = 0; b < B; ++b) {
                double sbar = 0.0, ck = 1.0;
                for (int64_t k = 0; k < P; ++k) {
                    ck *= (double)(2 * radii[k] + 1) * (double)(2 * radii[k] + 1);
                    sbar += a[k] * ((double)S[(k * B + b) * plane + px] / ck);
                }
                acc += M[l * B + b] * sbar;
            }
            rho[l * plane + px] = acc;
        }
    }
}

/* Gradient of the density (Sec. 3.3 Eq. 5). Reading: central differences at pixel
 * centres with zero density outside the grid; grad has [B][H][W][2] entries (gx, gy).
 * Pins: exact on linear maps in the interior; sign and factor 1/2.
 */
EXPORT void orc_gradient(int32_t B, int32_t W, int32_t H, const double *rho, double *grad) {
    int64_t plane = (int64_t)W * H;
#pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < B; ++l)
        for (int64_t v = 0; v < H; ++v)
            for (int64_t u = 0; u < W; ++u) {
                const double *m = rho + l * plane;
                double xl = u > 0 ? m[v * W + u - 1] : 0.0;
                double xr = u + 1 < W ? m[v * W + u + 1] : 0.0;
                double yd = v > 0 ? m[(v - 1) * W + u] : 0.0;
                double yu = v + 1 < H ? m[(v + 1) * W + u] : 0.0;
                int64_t i = l * plane + v * W + u;
                grad[2 * i] = 0.5 * (xr - xl);
                grad[2 * i + 1] = 0.5 * (yu - yd);
            }
}

/* Bilinear sample of a map whose pixel (u,v) value sits at the pixel centre (u+1/2, v+1/2);
 * taps are clamped into the grid. stride/comp select one component of an interleaved map.
 * Pins: reproduces linear functions exactly away from the border.
 */
EXPORT double orc_bilinear(int32_t W, int32_t H, const double *map, int32_t stride, int32_t comp,
                           double x, double y) {
    double fx = x - 0.5, fy = y - 0.5;
    double u0f = floor(fx), v0f = floor(fy);
    double tx = fx - u0f, ty = fy - v0f;
    int64_t u0 = (int64_t)u0f, v0 = (int64_t)v0f, u1 = u0 + 1, v1 = v0 + 1;
    if (u0 < 0) u0 = 0;
    if (u0 > W - 1) u0 = W - 1;
    if (u1 < 0) u1 = 0;
    if (u1 > W - 1) u1 = W - 1;
    if (v0 < 0) v0 = 0;
    if (v0 > H - 1) v0 = H - 1;
    if (v1 < 0) v1 = 0;
    if (v1 > H - 1) v1 = H - 1;
    double f00 = map[(v0 * W + u0) * stride + comp], f10 = map[(v0 * W + u1) * stride + comp];
    double f01 = map[(v1 * W + u0) * stride + comp], f11 = map[(v1 * W + u1) * stride + comp];
    return (1.0 - tx) * (1.0 - ty) * f00 + tx * (1.0 - ty) * f10 + (1.0 - tx) * ty * f01 +
           tx * ty * f11;
}

/* ------------------------------------------------ O5: advection with step halving (Sec. 3.3)
 * Each interior point x of an edge in bin b moves along the normalised gradient of layer
 * l = b (Eq. 5): d = g / max(|g|, eps) with g the bilinear gradient at x. The step starts
 * at m = h and is halved until the density at the new place is not lower than at x, or
 * until m reaches zero. Readings: at most K halvings (tries m = h / 2^j for j = 0..K),
 * then the point stays; candidates are clamped into [0, W - 2^-8] x [0, H - 2^-8] before
 * their density is read; end points never move.
 *
 * Outputs per point: the moved position, jacc = accepted j (-1: no move, -2: end point),
 * dir = d, and for decision parity amb = bitmask of tries whose density margin is within
 * amb_tol * (|rho(x)| + |rho(x')|) of zero (ambiguous in finite precision), evaluated up
 * to the first unambiguous acceptance, whose index is written to jfirm (-1 if none).
 * Pins: every accepted move satisfies rho(x') >= rho(x); zero gradient gives no move; a
 * point near an isolated smoothed impulse moves radially in closed form; a straight edge
 * on a pixel-centre row of a symmetric map never leaves the row; the decision record
 * (jacc, jfirm, amb) written out by hand on maps whose tries land on pixel centres of known
 * value, including margins just inside, just outside and exactly on the band edge.
 *
 * K < 0 selects the original advection step that Section 2 describes for KDEEB and Section
 * 3.3 compares against: every interior point moves by m = h along d with no density test
 * (then clamped); jacc = jfirm = 0 and no try is ambiguous.
 */
EXPORT void orc_advect(int64_t E, const int64_t *off, const double *xy, const int32_t *group,
                       int32_t B, int32_t W, int32_t H, const double *rho, const double *grad,
                       double h, int32_t K, double eps, double amb_tol, double *xy_out,
                       int32_t *jacc, int32_t *jfirm, uint32_t *amb, double *dir) {
    (void)B;
    int64_t plane = (int64_t)W * H;
    double xmax = (double)W - 1.0 / 256.0, ymax = (double)H - 1.0 / 256.0;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t e = 0; e < E; ++e) {
        const double *rl = rho + (int64_t)group[e] * plane;
        const double *gl = grad + (int64_t)group[e] * plane * 2;
        for (int64_t i = off[e]; i < off[e + 1]; ++i) {
            double x = xy[2 * i], y = xy[2 * i + 1];
            xy_out[2 * i] = x;
            xy_out[2 * i + 1] = y;
            dir[2 * i] = 0.0;
            dir[2 * i + 1] = 0.0;
            amb[i] = 0;
            if (i == off[e] || i == off[e + 1] - 1) {
                jacc[i] = -2;
                jfirm[i] = -2;
                continue;
            }
            double gx = orc_bilinear(W, H, gl, 2, 0, x, y);
            double gy = orc_bilinear(W, H, gl, 2, 1, x, y);
            double nrm = sqrt(gx * gx + gy * gy);
            double den = nrm > eps ? nrm : eps;
            double dx = gx / den, dy = gy / den;
            dir[2 * i] = dx;
            dir[2 * i + 1] = dy;
            if (K < 0) {
                double cx = x + h * dx, cy = y + h * dy;
                if (cx < 0.0) cx = 0.0;
                if (cx > xmax) cx = xmax;
                if (cy < 0.0) cy = 0.0;
                if (cy > ymax) cy = ymax;
                xy_out[2 * i] = cx;
                xy_out[2 * i + 1] = cy;
                jacc[i] = 0;
                jfirm[i] = 0;
                continue;
            }
            double r0 = orc_bilinear(W, H, rl, 1, 0, x, y);
            int32_t acc = -1, firm = -1;
            uint32_t mask = 0;
            double m = h;
            for (int32_t j = 0; j <= K; ++j, m *= 0.5) {
                double cx = x + m * dx, cy = y + m * dy;
                if (cx < 0.0) cx = 0.0;
                if (cx > xmax) cx = xmax;
                if (cy < 0.0) cy = 0.0;
                if (cy > ymax) cy = ymax;
                double r1 = orc_bilinear(W, H, rl, 1, 0, cx, cy);
                double margin = r1 - r0;
                int ambiguous = fabs(margin) <= amb_tol * (fabs(r0) + fabs(r1));
                if (ambiguous) mask |= 1u << j;
                if (acc < 0 && r1 >= r0) {
                    acc = j;
                    xy_out[2 * i] = cx;
                    xy_out[2 * i + 1] = cy;
                }
                if (!ambiguous && r1 >= r0) {
                    firm = j;
                    break;
                }
            }
            jacc[i] = acc;
            jfirm[i] = firm;
            amb[i] = mask;
        }
    }
}

/* ------------------------------------------------ O6: Laplacian smoothing (Sec. 2.1, Sec. 3.3)
 * After advection every polyline is smoothed like FDEB/KDEEB do. Reading: Jacobi passes
 * y_j = (1-s) x_j + (s/2)(x_{j-1} + x_{j+1}) on interior points, end points fixed.
 * Pins: uniform straight polylines and linear sequences are fixed points; zig-zag closed form.
 */
EXPORT void orc_laplacian(int64_t E, const int64_t *off, const double *xy_in, double s,
                          int32_t passes, double *xy_out) {
    int64_t N = off[E];
    double *tmp = (double *)malloc(sizeof(double) * 2 * (size_t)(N > 0 ? N : 1));
    memcpy(xy_out, xy_in, sizeof(double) * 2 * (size_t)N);
    for (int32_t p = 0; p < passes; ++p) {
        memcpy(tmp, xy_out, sizeof(double) * 2 * (size_t)N);
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t e = 0; e < E; ++e)
            for (int64_t i = off[e] + 1; i + 1 < off[e + 1]; ++i)
                for (int c = 0; c < 2; ++c)
                    xy_out[2 * i + c] =
                        (1.0 - s) * tmp[2 * i + c] + 0.5 * s * (tmp[2 * (i - 1) + c] + tmp[2 * (i + 1) + c]);
    }
    free(tmp);
}

/* Total polyline length ("ink") in FP64. */
EXPORT double orc_ink(int64_t E, const int64_t *off, const double *xy) {
    double total = 0.0;
    for (int64_t e = 0; e < E; ++e) total += orc_polyline_length(xy + 2 * off[e], off[e + 1] - off[e]);
    return total;
}

/* ------------------------------------------------ grouping (Sec. 5)
 * Bins can be found by k-means clustering of an edge property (origin, destination, both,
 * or the origin-destination distance) with the Euclidean distance, the number of bins B
 * being the one between 4 and 16 with the lowest Davies-Bouldin index, with k-means run
 * from several random initialisations for every B.
 * Reading: Lloyd's algorithm from k given centres. A point goes to its nearest centre by
 * the squared distance sum_j (x_j - c_j)^2, summed over the coordinates in order in FP64
 * (ties to the lower index); each centre moves to the mean of its points (a centre left
 * without points stays); this repeats until no label changes, or for max_iters rounds.
 * Inertia = sum of the squared distances to the assigned centres. Of the restarts of one B
 * the run of lowest inertia is kept (the first one on a tie). The random initialisations
 * take k distinct points, drawn with a counter-based SplitMix64 stream (orc_draw).
 * Davies-Bouldin index: with s_i the mean distance of the points of cluster i to its
 * centroid (the mean of its points) and d_ij the distance between centroids, the mean over
 * the non-empty clusters i of max over j != i of (s_i + s_j) / d_ij (a pair of coincident
 * centroids counts 0); one cluster or none gives 0.
 * Pins: scikit-learn's Lloyd k-means from the same centres (labels, centres, inertia) and
 * its Davies-Bouldin score, brute force on tiny inputs, invariance under point order.
 */
EXPORT double orc_sqdist(const float *x, const double *c, int32_t dim) {
    double s = 0.0;
    for (int32_t j = 0; j < dim; ++j) {
        double t = (double)x[j] - c[j];
        s += t * t;
    }
    return s;
}

/* Lloyd iterations; centers [k][dim] are the starting centres on entry and the final ones on
 * exit. Returns the number of assignment rounds made. */
EXPORT int32_t orc_kmeans(int64_t n, int32_t dim, const float *X, int32_t k, double *centers,
                          int32_t max_iters, int32_t *labels, double *inertia) {
    double *sum = (double *)calloc((size_t)k * (size_t)dim, sizeof(double));
    int64_t *cnt = (int64_t *)calloc((size_t)k, sizeof(int64_t));
    int32_t rounds = 0;
    for (int64_t i = 0; i < n; ++i) labels[i] = -1;
    for (int32_t it = 0; it < max_iters; ++it) {
        int64_t changed = 0;
        double in = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            int32_t best = 0;
            double bd = orc_sqdist(X + i * dim, centers, dim);
            for (int32_t c = 1; c < k; ++c) {
                double dd = orc_sqdist(X + i * dim, centers + (int64_t)c * dim, dim);
                if (dd < bd) {
                    bd = dd;
                    best = c;
                }
            }
            if (labels[i] != best) ++changed;
            labels[i] = best;
            in += bd;
        }
        rounds = it + 1;
        *inertia = in;
        if (changed == 0) break;
        memset(sum, 0, sizeof(double) * (size_t)k * (size_t)dim);
        memset(cnt, 0, sizeof(int64_t) * (size_t)k);
        for (int64_t i = 0; i < n; ++i) {
            for (int32_t j = 0; j < dim; ++j) sum[(int64_t)labels[i] * dim + j] += (double)X[i * dim + j];
            cnt[labels[i]] += 1;
        }
        for (int32_t c = 0; c < k; ++c)
            if (cnt[c] > 0)
                for (int32_t j = 0; j < dim; ++j) centers[(int64_t)c * dim + j] = sum[(int64_t)c * dim + j] / (double)cnt[c];
        if (it + 1 == max_iters) {
            /* the inertia of the final centres */
            in = 0.0;
            for (int64_t i = 0; i < n; ++i) in += orc_sqdist(X + i * dim, centers + (int64_t)labels[i] * dim, dim);
            *inertia = in;
        }
    }
    free(sum);
    free(cnt);
    return rounds;
}

EXPORT double orc_davies_bouldin(int64_t n, int32_t dim, const float *X, int32_t k, const int32_t *labels) {
    double *cen = (double *)calloc((size_t)k * (size_t)dim, sizeof(double));
    double *s = (double *)calloc((size_t)k, sizeof(double));
    int64_t *cnt = (int64_t *)calloc((size_t)k, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t j = 0; j < dim; ++j) cen[(int64_t)labels[i] * dim + j] += (double)X[i * dim + j];
        cnt[labels[i]] += 1;
    }
    for (int32_t c = 0; c < k; ++c)
        if (cnt[c] > 0)
            for (int32_t j = 0; j < dim; ++j) cen[(int64_t)c * dim + j] /= (double)cnt[c];
    for (int64_t i = 0; i < n; ++i) s[labels[i]] += sqrt(orc_sqdist(X + i * dim, cen + (int64_t)labels[i] * dim, dim));
    int32_t used = 0;
    double total = 0.0;
    for (int32_t a = 0; a < k; ++a) {
        if (cnt[a] == 0) continue;
        ++used;
        double worst = 0.0;
        for (int32_t b = 0; b < k; ++b) {
            if (b == a || cnt[b] == 0) continue;
            double d2 = 0.0;
            for (int32_t j = 0; j < dim; ++j) {
                double t = cen[(int64_t)a * dim + j] - cen[(int64_t)b * dim + j];
                d2 += t * t;
            }
            double d = sqrt(d2);
            double r = d > 0.0 ? (s[a] / (double)cnt[a] + s[b] / (double)cnt[b]) / d : 0.0;
            if (r > worst) worst = r;
        }
        total += worst;
    }
    free(cen);
    free(s);
    free(cnt);
    return used > 1 ? total / (double)used : 0.0;
}

/* SplitMix64 (Steele, Lea and Flood, 2014) as a counter-based stream: value t of stream
 * (seed, B, r) is the SplitMix64 output mix of seed + gamma * (1 + t + 4096 (r + 1024 B)),
 * gamma = 0x9E3779B97F4A7C15. */
EXPORT uint64_t orc_draw(uint64_t seed, int32_t B, int32_t r, int64_t t) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(1 + t + 4096 * ((int64_t)r + 1024 * (int64_t)B));
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* k distinct point indices of restart r for B = k: the values t = 0, 1, ... of stream
 * (seed, k, r) taken modulo n, skipping repeats (n >= k). */
EXPORT void orc_init_indices(uint64_t seed, int32_t k, int32_t r, int64_t n, int64_t *idx) {
    int32_t got = 0;
    for (int64_t t = 0; got < k; ++t) {
        int64_t v = (int64_t)(orc_draw(seed, k, r, t) % (uint64_t)n);
        int32_t dup = 0;
        for (int32_t q = 0; q < got; ++q) dup |= idx[q] == v;
        if (!dup) idx[got++] = v;
    }
}

/* For every B in [kmin, kmax]: `restarts` k-means runs from orc_init_indices, the lowest
 * inertia kept, its Davies-Bouldin index in db[B - kmin]; returns the B of the lowest index
 * (the smallest B on a tie) and its labels. */
EXPORT int32_t orc_choose_groups(int64_t n, int32_t dim, const float *X, int32_t kmin, int32_t kmax,
                                 int32_t restarts, uint64_t seed, int32_t max_iters,
                                 int32_t *labels, double *db) {
    int32_t *lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *best_lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *cen = (double *)malloc(sizeof(double) * (size_t)kmax * (size_t)dim);
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)kmax);
    int32_t chosen = kmin;
    double chosen_db = 0.0;
    for (int32_t k = kmin; k <= kmax; ++k) {
        double best_in = 0.0;
        for (int32_t r = 0; r < restarts; ++r) {
            orc_init_indices(seed, k, r, n, idx);
            for (int32_t c = 0; c < k; ++c)
                for (int32_t j = 0; j < dim; ++j) cen[(int64_t)c * dim + j] = (double)X[idx[c] * dim + j];
            double in = 0.0;
            orc_kmeans(n, dim, X, k, cen, max_iters, lab, &in);
            if (r == 0 || in < best_in) {
                best_in = in;
                memcpy(best_lab, lab, sizeof(int32_t) * (size_t)n);
            }
        }
        double d = orc_davies_bouldin(n, dim, X, k, best_lab);
        db[k - kmin] = d;
        if (k == kmin || d < chosen_db) {
            chosen_db = d;
            chosen = k;
            memcpy(labels, best_lab, sizeof(int32_t) * (size_t)n);
        }
    }
    free(lab);
    free(best_lab);
    free(cen);
    free(idx);
    return chosen;
}

/* ------------------------------------------------ width encoding (Sec. 3.4)
 * Bundle weight is also encoded by line width: the width of the polyline between
 * consecutive sample points follows the density map at the sample points, on a linear or a
 * logarithmic scale. Reading: per point, rho = the density of its edge's layer at the point
 * (bilinear, as the advection samples it; negative values, possible with repelling
 * interactions, count as 0), the width w = w_min + (w_max - w_min) f(rho) / f(rho_max) with
 * f(rho) = rho (linear) or log(1 + rho) (log scale; rho in samples per pixel) and rho_max the
 * largest rho over all points; all points get w_min when rho_max is 0. A renderer draws the
 * segment (x_j, x_j+1) with the mean of its two end widths.
 * Pins: closed form on linear maps, w_max at the densest point and w_min where the density is
 * 0, monotone in the density, the log scale compresses.
 */
EXPORT void orc_point_widths(int64_t E, const int64_t *off, const double *xy, const int32_t *group,
                             int32_t W, int32_t H, const double *rho, double w_min, double w_max,
                             int32_t log_scale, double *dens, double *widths) {
    int64_t plane = (int64_t)W * H;
    double rmax = 0.0;
    for (int64_t e = 0; e < E; ++e)
        for (int64_t i = off[e]; i < off[e + 1]; ++i) {
            double r = orc_bilinear(W, H, rho + (int64_t)group[e] * plane, 1, 0, xy[2 * i], xy[2 * i + 1]);
            if (!(r > 0.0)) r = 0.0;
            dens[i] = r;
            if (r > rmax) rmax = r;
        }
    double fmax = log_scale ? log1p(rmax) : rmax;
    for (int64_t i = 0; i < off[E]; ++i) {
        double f = log_scale ? log1p(dens[i]) : dens[i];
        widths[i] = fmax > 0.0 ? w_min + (w_max - w_min) * (f / fmax) : w_min;
    }
}
