// Host runtime of the bundling library: contexts, parameter validation, device buffers,
// the per-iteration launch schedule, automatic growth of the point buffers, and the C ABI
// declared in include/hb.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hb_internal.h"
#include "render.h"

using hb::GDesc;
using hb::Shape;

#define HB_API extern "C" __attribute__((visibility("default")))

static thread_local std::string g_thread_err;

struct hb_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t side = nullptr;          // second stream of the backward (parameter gradients)
    std::vector<hipEvent_t> adj_ev;      // events ordering the two streams of the backward
    bool sticky = false;
    std::string err;

    // parameters
    hb_params P{};
    std::vector<int32_t> radii;
    std::vector<float> sigmas;           // sigma per iteration (Kovesi widths), or empty
    std::vector<float> passw;
    bool have_params = false;

    // graph and groups
    int64_t E = 0;
    int32_t wmax = 1;
    bool have_graph = false;
    int32_t B = 0;
    bool have_groups = false;
    int32_t *d_group = nullptr, *d_weight = nullptr;
    int32_t *d_perm_adj = nullptr;       // edge order of the advection kernels (built on use)
    std::vector<int32_t> h_group;
    std::vector<uint32_t> h_morton;     // Morton code of each straight edge's midpoint
    float *d_M = nullptr;

    // points: state = (pts[ps], off[os]); last samples = (pts[ss], off[so])
    float2 *pts[2] = {nullptr, nullptr};
    int64_t *off[2] = {nullptr, nullptr};
    int64_t cap = 0;
    uint32_t *d_bins = nullptr;          // [ent_cap] entries of the splat (samples or drawn pixels)
    int64_t ent_cap = 0;
    uint32_t *d_binsrc = nullptr;        // [cap] sample of each binned entry (checkpointed runs)
    int64_t binsrc_cap = 0;
    int ps = 0, os = 0, ss = 0, so = 0;
    int64_t n_state = 0, n_samples = 0;
    bool have_samples = false;

    int64_t *d_counts = nullptr, *d_tsum = nullptr, *d_totals = nullptr;
    double *d_lens = nullptr;
    int32_t *d_status = nullptr;
    double *d_ink = nullptr;             // [kInkSlices + 1] ink slice sums and total
    int totals_cap = 0;

    // maps of the last iteration
    int32_t *d_hist = nullptr, *d_histx = nullptr;
    int32_t nx = 1;                      // XCDs of the device
    int64_t *d_bin_cnt = nullptr, *d_bin_cur = nullptr, *d_tile_off = nullptr, *d_seg_off = nullptr;
    int64_t *d_box = nullptr, *d_tmp = nullptr;
    float *d_rho = nullptr;
    float2 *d_grad = nullptr;
    float *d_rhos = nullptr;
    float2 *d_grads = nullptr;
    int32_t map_B = 0, map_W = 0, map_H = 0, map_P = 0;
    bool have_maps = false;

    int8_t *d_jacc = nullptr;
    float *d_render = nullptr;     // point densities, widths and the largest density (bits)
    int64_t render_cap = 0;
    int64_t jacc_cap = 0;
    bool have_jacc = false;

    // descriptor table: pinned staging + device copy
    GDesc *h_desc = nullptr, *d_desc = nullptr;
    size_t desc_cap = 0;
    hipEvent_t desc_done = nullptr;

    int32_t iter = 0;
    std::vector<int64_t> last_counts;

    // per-stage timing
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<int> ev_stage;           // stage of each recorded pair
    double stage_ms[HB_NUM_STAGES] = {0};
    int64_t stage_n[HB_NUM_STAGES] = {0};

    // checkpoints of a differentiable run: the polylines entering each iteration
    struct Ckpt {
        float2 *pts = nullptr, *xs = nullptr;      // polylines entering / samples of the iteration
        int64_t *off = nullptr, *xoff = nullptr;   // their offsets
        int64_t *counts = nullptr;
        double *lens = nullptr;
        int8_t *jacc = nullptr;                    // accepted halvings of the samples
        int32_t *hist = nullptr;                   // [B][H][W] histogram of the samples
        uint32_t *bsrc = nullptr;                  // samples binned by histogram tile
        int64_t *toff = nullptr, *soff = nullptr;  // tile offsets and work-item offsets
        int64_t n = 0, ns = 0;
        int32_t iter = 0;
        int64_t cap_n = 0, cap_ns = 0, cap_e = 0, cap_px = 0;   // allocated sizes (reused)
        int64_t cap_bs = 0, cap_t = 0;
    };
    std::vector<Ckpt> ckpts;       // checkpoints of the last hb_forward_ckpt
    std::vector<Ckpt> ckpt_pool;   // allocated checkpoint buffers for reuse
    int32_t ckpt_end_iter = -1;
    int64_t ckpt_gen = 0;          // generation of the checkpoints (one more per forward)

    // adjoint work buffers, kept between backward passes
    struct AdjBufs {
        float2 *a0 = nullptr, *a1 = nullptr;
        float2 *gb[2] = {nullptr, nullptr};   // gradient-map records, by iteration parity
        double *partials = nullptr, *gparam = nullptr, *red = nullptr;
        float2 *mv[2] = {nullptr, nullptr};   // m v of every sample, by iteration parity
        uint32_t *mvmax = nullptr;
        int64_t cap_pts = 0, cap_a1 = 0, cap_gb[2] = {0, 0}, cap_part = 0, cap_gp = 0, cap_red = 0;
        int64_t cap_mv[2] = {0, 0}, cap_mm = 0;
    } adj;

    // kernel variants (chunks of 64 per trip in resampling / advection)
    int tune_ru = 2, tune_au = 2;
    hb::Tiling tiling;             // box column rows, tile-count sets, tile work-item size
    int map_sets = 0;              // tile-count sets the map buffers were sized for

    // captured iteration sequence, replayed while the batch layout is unchanged
    hipGraphExec_t gexec = nullptr;
    std::vector<int64_t> gkey;

    // pending asynchronous run
    hb_ctx *pend_lead = nullptr;
    bool pending = false;
    int32_t pend_start = 0, pend_T = 0;
    uint32_t pend_flags = 0;
    std::vector<int> pend_ps, pend_os;
};

// ------------------------------------------------------------------ errors

static hb_status fail(hb_ctx *c, hb_status st, const std::string &msg) {
    if (c) c->err = msg; else g_thread_err = msg;
    return st;
}

static hb_status fail_dev(hb_ctx *c, hipError_t e, const char *what) {
    c->sticky = true;
    char buf[512];
    snprintf(buf, sizeof buf, "HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
    c->err = buf;
    return HB_EDEVICE;
}

#define HIPCHK(c, expr)                                   \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return fail_dev(c, e_, #expr); \
    } while (0)

#define CHKST(expr)                       \
    do {                                  \
        hb_status s_ = (expr);            \
        if (s_ != HB_OK) return s_;       \
    } while (0)

// Makes ctx's device current for the duration of an API call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

#define ENTER(c)                                                                  \
    if (!(c)) return fail(nullptr, HB_EINVAL, "null context");                    \
    if ((c)->sticky) return fail(c, HB_EDEVICE, "context has a sticky HIP error: " + (c)->err); \
    DeviceGuard guard_(c->device);                                                \
    if (!guard_.ok) return fail(c, HB_EDEVICE, "hipSetDevice failed");

// ------------------------------------------------------------------ allocation

template <typename T>
static hb_status dalloc(hb_ctx *c, T **p, size_t count, const char *what) {
    if (*p) {
        (void)hipFree(*p);
        *p = nullptr;
    }
    if (count == 0) count = 1;
    if (getenv("HB_TEST_FAIL_ALLOC")) return fail(c, HB_ENOMEM, std::string("simulated allocation failure: ") + what);
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        char buf[256];
        snprintf(buf, sizeof buf, "hipMalloc of %zu bytes for %s failed", count * sizeof(T), what);
        return fail(c, HB_ENOMEM, buf);
    }
    return HB_OK;
}

template <typename T>
static void dfree(T **p) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
}

// ------------------------------------------------------------------ parameters

static double sigma_of(int r, int passes) {
    return std::sqrt((double)passes * (double)r * (double)(r + 1) / 3.0);
}

HB_API void hb_default_params(hb_params *p, int32_t grid_w, int32_t grid_h) {
    if (!p) return;
    static thread_local int32_t r_default[1];
    memset(p, 0, sizeof *p);
    p->struct_size = sizeof(hb_params);
    p->grid_w = grid_w;
    p->grid_h = grid_h;
    p->bbox[0] = 0.0f;
    p->bbox[1] = 0.0f;
    p->bbox[2] = 1.0f;
    p->bbox[3] = 1.0f;
    p->delta_px = 1.0f;
    p->box_passes = 3;
    r_default[0] = std::max(1, std::min(grid_w, grid_h) / 32);
    p->n_radii = 1;
    p->radius_per_iter = r_default;
    p->h_max_px = 0.0f;
    p->lambda = 0.9f;
    p->eps = 1e-6f;
    p->max_halvings = 8;
    p->smooth_weight = 0.5f;
    p->smooth_passes = 1;
    p->pass_weights = nullptr;
    p->capacity_factor = 2.0f;
    p->directed_offset_px = 0.0f;
    p->splat_mode = HB_SPLAT_POINTS;
    p->resample_mode = HB_RESAMPLE_UNIFORM;
    p->delta_min_px = 0.0f;
    p->n_sigmas = 0;
    p->sigma_per_iter = nullptr;
    p->directed_mode = HB_DIRECTED_ONCE;
}

static void kovesi_radii(double sigma, int P, int32_t *radii);


static hb_status validate(hb_ctx *c, const hb_params *p) {
    if (!p) return fail(c, HB_EINVAL, "params is NULL");
    if (p->struct_size != sizeof(hb_params))
        return fail(c, HB_EINVAL, "params.struct_size does not match sizeof(hb_params)");
    if (p->grid_w < 2 || p->grid_h < 2 || p->grid_w > HB_MAX_GRID || p->grid_h > HB_MAX_GRID)
        return fail(c, HB_EINVAL, "grid size out of range [2, 8192]");
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(p->bbox[i])) return fail(c, HB_EINVAL, "bbox is not finite");
    if (!(p->bbox[2] > p->bbox[0]) || !(p->bbox[3] > p->bbox[1]))
        return fail(c, HB_EINVAL, "bbox must have x1 > x0 and y1 > y0");
    if (!(p->delta_px > 0.0f) || !std::isfinite(p->delta_px))
        return fail(c, HB_EINVAL, "delta_px must be positive");
    if (p->box_passes < 1 || p->box_passes > HB_MAX_PASSES)
        return fail(c, HB_EINVAL, "box_passes out of range [1, 8]");
    const int side = std::min(p->grid_w, p->grid_h);
    if (p->n_sigmas < 0) return fail(c, HB_EINVAL, "n_sigmas must be >= 0");
    if (p->n_sigmas > 0) {
        if (!p->sigma_per_iter) return fail(c, HB_EINVAL, "sigma_per_iter is NULL");
        for (int i = 0; i < p->n_sigmas; ++i) {
            const float s = p->sigma_per_iter[i];
            if (!std::isfinite(s) || !(s > 0.0f)) return fail(c, HB_EINVAL, "sigma_per_iter must be finite and > 0");
            int32_t rp[HB_MAX_PASSES];
            kovesi_radii((double)s, std::max(1, std::min(p->box_passes, HB_MAX_PASSES)), rp);
            for (int k = 0; k < std::max(1, std::min(p->box_passes, HB_MAX_PASSES)); ++k)
                if (2 * rp[k] + 1 > side) return fail(c, HB_EINVAL, "box width of a sigma exceeds min(W, H)");
        }
    } else {
        if (p->n_radii < 1 || !p->radius_per_iter)
            return fail(c, HB_EINVAL, "radius_per_iter needs at least one value");
        for (int i = 0; i < p->n_radii; ++i) {
            int r = p->radius_per_iter[i];
            if (r < 0 || 2 * r + 1 > side)
                return fail(c, HB_EINVAL, "box radius must satisfy 0 <= r and 2r+1 <= min(W, H)");
        }
    }
    if (!std::isfinite(p->h_max_px)) return fail(c, HB_EINVAL, "h_max_px is not finite");
    if (!(p->lambda > 0.0f) || p->lambda > 1.0f) return fail(c, HB_EINVAL, "lambda must be in (0, 1]");
    if (!(p->eps > 0.0f) || !std::isfinite(p->eps)) return fail(c, HB_EINVAL, "eps must be positive");
    if (p->max_halvings < -1 || p->max_halvings > HB_MAX_HALVINGS)
        return fail(c, HB_EINVAL, "max_halvings out of range [-1, 30]");
    if (!(p->smooth_weight >= 0.0f) || p->smooth_weight > 1.0f)
        return fail(c, HB_EINVAL, "smooth_weight must be in [0, 1]");
    if (p->smooth_passes != 1) return fail(c, HB_EINVAL, "smooth_passes must be 1");
    if (p->pass_weights)
        for (int k = 0; k < p->box_passes; ++k)
            if (!std::isfinite(p->pass_weights[k])) return fail(c, HB_EINVAL, "pass_weights not finite");
    if (!(p->capacity_factor == 0.0f || (p->capacity_factor >= 1.1f && p->capacity_factor <= 64.0f)))
        return fail(c, HB_EINVAL, "capacity_factor must be 0 (default) or in [1.1, 64]");
    if (!std::isfinite(p->directed_offset_px) ||
        std::fabs(p->directed_offset_px) > (float)std::max(p->grid_w, p->grid_h) / 16.0f)
        return fail(c, HB_EINVAL, "directed_offset_px must be finite with |value| <= max(W, H) / 16");
    if (p->splat_mode != HB_SPLAT_POINTS && p->splat_mode != HB_SPLAT_STRIP)
        return fail(c, HB_EINVAL, "splat_mode must be HB_SPLAT_POINTS or HB_SPLAT_STRIP");
    if (p->resample_mode != HB_RESAMPLE_UNIFORM && p->resample_mode != HB_RESAMPLE_INSERT_DELETE)
        return fail(c, HB_EINVAL, "resample_mode must be HB_RESAMPLE_UNIFORM or HB_RESAMPLE_INSERT_DELETE");
    if (!std::isfinite(p->delta_min_px) || p->delta_min_px < 0.0f || p->delta_min_px >= p->delta_px)
        return fail(c, HB_EINVAL, "delta_min_px must be 0 (delta_px / 2) or in (0, delta_px)");
    if (p->resample_mode == HB_RESAMPLE_INSERT_DELETE && p->directed_offset_px != 0.0f)
        return fail(c, HB_EINVAL, "the directed offset needs the uniform resampling");
    if (p->directed_mode != HB_DIRECTED_ONCE && p->directed_mode != HB_DIRECTED_EVERY_ITER)
        return fail(c, HB_EINVAL, "directed_mode must be HB_DIRECTED_ONCE or HB_DIRECTED_EVERY_ITER");
    return HB_OK;
}

HB_API hb_status hb_validate_params(const hb_params *p) { return validate(nullptr, p); }

static int radius_at(const hb_ctx *c, int it) {
    return c->radii[std::min<size_t>((size_t)it, c->radii.size() - 1)];
}

// Kovesi's two-width rule (Kovesi, "Fast almost-Gaussian filtering", 2010): P passes of odd
// widths w_l and w_l + 2 whose variances add up closest to sigma^2; radii = (width - 1) / 2.
static void kovesi_radii(double sigma, int P, int32_t *radii) {
    const double wi = std::sqrt(12.0 * sigma * sigma / (double)P + 1.0);
    int64_t wl = (int64_t)std::floor(wi);
    if (wl % 2 == 0) wl -= 1;
    if (wl < 1) wl = 1;
    const int64_t wu = wl + 2;
    const double mi = (12.0 * sigma * sigma - (double)P * (double)(wl * wl) - 4.0 * (double)P * (double)wl -
                       3.0 * (double)P) / (-4.0 * (double)wl - 4.0);
    int64_t m = (int64_t)std::round(mi);
    m = std::min<int64_t>(std::max<int64_t>(m, 0), P);
    for (int k = 0; k < P; ++k) radii[k] = (int32_t)(((k < m ? wl : wu) - 1) / 2);
}

// Box radius of every pass of iteration it.
static void pass_radii(const hb_ctx *c, int it, int32_t *rp) {
    const int P = c->P.box_passes;
    if (!c->sigmas.empty()) {
        kovesi_radii((double)c->sigmas[std::min<size_t>((size_t)it, c->sigmas.size() - 1)], P, rp);
        return;
    }
    for (int k = 0; k < P; ++k) rp[k] = radius_at(c, it);
}

static double hmax_of(const hb_ctx *c) {
    if (c->P.h_max_px > 0.0f) return (double)c->P.h_max_px;
    if (!c->sigmas.empty()) return 2.0 * (double)c->sigmas[0];
    return 2.0 * sigma_of(radius_at(c, 0), c->P.box_passes);
}

static double bandwidth_at(const hb_ctx *c, int it) {
    double h = hmax_of(c);
    for (int i = 0; i < it; ++i) h *= (double)c->P.lambda;
    return h;
}

// ------------------------------------------------------------------ buffers

static hb_status ensure_totals(hb_ctx *c, int n) {
    if (n <= c->totals_cap) return HB_OK;
    CHKST(dalloc(c, &c->d_totals, (size_t)n, "iteration totals"));
    c->totals_cap = n;
    return HB_OK;
}

static hb_status ensure_desc(hb_ctx *c, size_t n) {
    if (n <= c->desc_cap) return HB_OK;
    if (c->desc_done) HIPCHK(c, hipEventSynchronize(c->desc_done));
    if (c->h_desc) (void)hipHostFree(c->h_desc);
    c->h_desc = nullptr;
    HIPCHK(c, hipHostMalloc((void **)&c->h_desc, n * sizeof(GDesc), hipHostMallocDefault));
    CHKST(dalloc(c, &c->d_desc, n, "descriptor table"));
    c->desc_cap = n;
    return HB_OK;
}

// Grow both point buffers to hold at least `need` points, keeping the state and samples.
// Splat entries per point of capacity: 1 for the point splat; for the line strips, the
// pixels a segment between consecutive samples can draw (its chord is at most the sample
// spacing delta plus twice the directed offset, and at most one more pixel comes from the
// pixel grid) plus one of margin.
static int64_t entry_factor(const hb_ctx *c) {
    if (c->P.splat_mode != HB_SPLAT_STRIP) return 1;
    const double reach = (double)c->P.delta_px + 2.0 * std::fabs((double)c->P.directed_offset_px);
    return (int64_t)std::ceil(reach) + 2;
}

// 32-bit words of an entry buffer of n entries: graphs whose edges all weigh 1 write 16-bit
// entries (the pixel inside the tile; the count is 1), the others 32-bit ones (pixel and
// weight).
static size_t entry_words(const hb_ctx *c, int64_t n) {
    return c->wmax == 1 ? (size_t)((n + 1) / 2) : (size_t)n;
}

static hb_status ensure_bins(hb_ctx *c) {
    const int64_t need = c->cap * entry_factor(c);
    if (need <= c->ent_cap && c->d_bins) return HB_OK;
    CHKST(dalloc(c, &c->d_bins, entry_words(c, need), "splat entries"));
    c->ent_cap = need;
    return HB_OK;
}

// Grows the point buffers to at least `need` points (1.25 times the old capacity at least),
// one buffer at a time so that at most three point buffers are held at once: the splat
// entries are rebuilt every iteration and are dropped first.
static hb_status ensure_capacity(hb_ctx *c, int64_t need) {
    if (need <= c->cap) return HB_OK;
    int64_t ncap = std::max<int64_t>(need, c->cap + c->cap / 4);
    ncap = std::max<int64_t>(ncap, 1024);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dfree(&c->d_bins);
    c->ent_cap = 0;
    for (int i = 0; i < 2; ++i) {
        float2 *np = nullptr;
        CHKST(dalloc(c, &np, (size_t)ncap, "point buffer"));
        int64_t keep = 0;   // points of this buffer that later calls still read
        if (i == c->ps && c->n_state > 0) keep = c->n_state;
        if (c->have_samples && i == c->ss && c->ss != c->ps) keep = c->n_samples;
        if (c->pts[i] && keep > 0) {
            hipError_t e = hipMemcpyAsync(np, c->pts[i], sizeof(float2) * keep,
                                          hipMemcpyDeviceToDevice, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) {
                dfree(&np);
                return fail_dev(c, e, "point buffer copy");
            }
        }
        dfree(&c->pts[i]);
        c->pts[i] = np;
        if (i == 0) c->cap = std::min(c->cap, ncap);   // both buffers hold at least cap
    }
    c->cap = ncap;
    c->have_jacc = false;   // the decisions buffer is kept; it grows when a run records
    return ensure_bins(c);
}

static hb_status ensure_maps(hb_ctx *c) {
    const int B = c->B, W = c->P.grid_w, H = c->P.grid_h, P = c->P.box_passes;
    const hb::Tiles tl = hb::tiles_of(B, W, H, c->tiling.sets_max);
    if (c->d_hist && c->map_B == B && c->map_W == W && c->map_H == H && c->map_P == P &&
        c->map_sets == tl.sets)
        return HB_OK;
    const size_t plane = (size_t)B * W * H;
    c->have_maps = false;
    CHKST(dalloc(c, &c->d_hist, plane, "histogram"));
    CHKST(dalloc(c, &c->d_histx, plane, "histogram accumulator"));
    CHKST(dalloc(c, &c->d_bin_cnt, (size_t)tl.sets * tl.n, "tile counts"));
    CHKST(dalloc(c, &c->d_bin_cur, (size_t)tl.sets * tl.n, "tile cursors"));
    CHKST(dalloc(c, &c->d_tile_off, (size_t)tl.n + 1, "tile offsets"));
    CHKST(dalloc(c, &c->d_seg_off, (size_t)tl.n + 1, "tile work items"));
    CHKST(dalloc(c, &c->d_box, plane * P, "box passes"));
    CHKST(dalloc(c, &c->d_tmp, plane, "row-pass scratch"));
    CHKST(dalloc(c, &c->d_rho, plane, "density"));
    CHKST(dalloc(c, &c->d_grad, plane, "gradient"));
    CHKST(dalloc(c, &c->d_rhos, (size_t)B * hb::rho_strip_plane(W, H), "density strips"));
    CHKST(dalloc(c, &c->d_grads, (size_t)B * hb::grad_strip_plane(W, H), "gradient strips"));
    c->map_B = B;
    c->map_W = W;
    c->map_H = H;
    c->map_P = P;
    c->map_sets = tl.sets;
    return HB_OK;
}

// Descriptor with every field that does not change between iterations.
static GDesc base_desc(const hb_ctx *c) {
    GDesc d;
    memset(&d, 0, sizeof d);

    d.n_edges = c->E;
    d.cap = c->cap;
    d.B = std::max(1, c->B);
    d.W = c->P.grid_w;
    d.H = c->P.grid_h;
    d.P = c->P.box_passes;
    d.K = c->P.max_halvings;
    d.wmax = c->wmax;
    d.eps = (double)c->P.eps;
    d.s = (double)c->P.smooth_weight;
    d.delta = (double)c->P.delta_px;
    d.doff = 0.0;   // per iteration, set_iter_scalars
    d.strip = c->P.splat_mode == HB_SPLAT_STRIP ? 1 : 0;
    d.ent_cap = c->ent_cap;
    d.insdel = c->P.resample_mode == HB_RESAMPLE_INSERT_DELETE ? 1 : 0;
    d.narrow = c->wmax == 1 ? 1 : 0;   // 16-bit splat entries: every edge weighs 1
    d.dmin = c->P.delta_min_px > 0.0f ? (double)c->P.delta_min_px : 0.5 * (double)c->P.delta_px;
    d.count_given = 0;
    for (int k = 0; k < d.P; ++k)
        d.a[k] = c->passw.empty() ? (k == d.P - 1 ? 1.0 : 0.0) : (double)c->passw[k];
    d.group = c->d_group;
    d.order = c->d_perm_adj;
    d.weight = c->d_weight;
    d.M = c->d_M;
    d.counts = c->d_counts;
    d.lens = c->d_lens;
    d.tsum = c->d_tsum;
    d.total = c->d_totals;
    d.hist = c->d_hist;
    d.histx = c->d_histx;
    d.nx = 1;
    d.nxcd = c->nx;
    const hb::Tiles tl = hb::tiles_of(d.B, d.W, d.H, c->tiling.sets_max);
    d.tiles_x = tl.x;
    d.tiles_y = tl.y;
    d.n_tiles = tl.n;
    d.tile_blocks = tl.blocks;
    d.n_sets = tl.sets;
    d.col_rows = c->tiling.col_rows;
    d.item_entries = c->tiling.item_entries;
    d.bin_cnt = c->d_bin_cnt;
    d.bin_cur = c->d_bin_cur;
    d.tile_off = c->d_tile_off;
    d.seg_off = c->d_seg_off;
    d.bins = c->d_bins;
    d.box = c->d_box;
    d.tmp = c->d_tmp;
    d.rho = c->d_rho;
    d.grad = c->d_grad;
    d.rhos = c->d_rhos;
    d.grads = c->d_grads;
    d.jacc = c->d_jacc;
    d.status = c->d_status;
    return d;
}

static void set_iter_scalars(const hb_ctx *c, GDesc &d, int it) {
    // the directed push follows the first sampling (iteration 0), or every resampling
    const bool push = it == 0 || c->P.directed_mode == HB_DIRECTED_EVERY_ITER;
    d.doff = push ? (double)c->P.directed_offset_px : 0.0;
    pass_radii(c, it, d.rp);
    d.r = d.rp[d.P - 1];
    d.h = bandwidth_at(c, it);
    double ck = 1.0;
    for (int k = 0; k < d.P; ++k) {
        ck *= (double)(2 * d.rp[k] + 1) * (double)(2 * d.rp[k] + 1);
        d.ck[k] = ck;
    }
}

// Upload n descriptors from the pinned staging table.
static hb_status upload_desc(hb_ctx *c, size_t n) {
    HIPCHK(c, hipMemcpyAsync(c->d_desc, c->h_desc, n * sizeof(GDesc), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipEventRecord(c->desc_done, c->stream));
    return HB_OK;
}

static hb_status wait_desc(hb_ctx *c) {
    if (c->desc_done) HIPCHK(c, hipEventSynchronize(c->desc_done));
    return HB_OK;
}

static hb_status read_scalar(hb_ctx *c, const int64_t *dptr, int64_t *out) {
    HIPCHK(c, hipMemcpyAsync(out, dptr, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HB_OK;
}

// ------------------------------------------------------------------ stage timing

// Record the start event of a stage launch; returns the pair index or -1.
static hb_status stage_begin(hb_ctx *c, int stage, int *pair) {
    *pair = -1;
    if (!c->profiling) return HB_OK;
    size_t need = c->ev_used + 2;
    while (c->ev_pool.size() < need) {
        hipEvent_t e;
        HIPCHK(c, hipEventCreate(&e));
        c->ev_pool.push_back(e);
    }
    HIPCHK(c, hipEventRecord(c->ev_pool[c->ev_used], c->stream));
    *pair = (int)(c->ev_used / 2);
    c->ev_stage.push_back(stage);
    c->ev_used += 2;
    return HB_OK;
}

static hb_status stage_end(hb_ctx *c, int pair) {
    if (pair < 0) return HB_OK;
    HIPCHK(c, hipEventRecord(c->ev_pool[(size_t)pair * 2 + 1], c->stream));
    return HB_OK;
}

// After the stream has drained: fold the recorded pairs into the accumulators.
static hb_status stage_collect(hb_ctx *c) {
    for (size_t i = 0; i < c->ev_stage.size(); ++i) {
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pool[2 * i], c->ev_pool[2 * i + 1]));
        c->stage_ms[c->ev_stage[i]] += (double)ms;
        c->stage_n[c->ev_stage[i]] += 1;
    }
    c->ev_stage.clear();
    c->ev_used = 0;
    return HB_OK;
}

#define STAGE(c, id, launch)                      \
    do {                                          \
        int pair_;                                \
        CHKST(stage_begin(c, id, &pair_));        \
        HIPCHK(c, launch);                        \
        CHKST(stage_end(c, pair_));               \
    } while (0)

// ------------------------------------------------------------------ lifecycle

// ------------------------------------------------------------------ allocation-free scratch
//
// hb_davies_bouldin_noalloc works in this fixed device array instead of allocating: the
// partial sums of one chunk of at most kNaChunk points (kNaRows rows of kNaW values: 64
// blocks of 4 waves), the chunk totals, their running sum over the chunks, the centroids and
// the index. Every GPU holds its own copy for the life of the process; its address on a
// device comes from hipGetSymbolAddress, taken once per device by hb_create with that device
// current, and only that address is handed to kernels and copies.
static constexpr int kNaRows = 256;
static constexpr int64_t kNaChunk = (int64_t)kNaRows * 64;
static constexpr int kNaW = HB_KMEANS_MAX_K * (HB_KMEANS_MAX_DIM + 1) + 2;
static constexpr size_t kNaDoubles =
    (size_t)kNaRows * kNaW + 2 * (size_t)kNaW + (size_t)HB_KMEANS_MAX_K * HB_KMEANS_MAX_DIM + 1;
static __device__ __align__(256) double scratch[kNaDoubles];

static std::mutex g_scratch_mu;
static std::vector<double *> g_scratch_ptr;      // per device; nullptr until set up
static std::vector<std::string> g_scratch_err;   // per device: why the address is missing

// Called with `device` current. Takes the array's address on that device once.
static void scratch_setup(int device, int ndev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() < ndev) {
        g_scratch_ptr.resize((size_t)ndev, nullptr);
        g_scratch_err.resize((size_t)ndev);
    }
    if (g_scratch_ptr[(size_t)device]) return;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        g_scratch_err[(size_t)device] = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
        return;
    }
    g_scratch_ptr[(size_t)device] = (double *)ptr;
}

static double *scratch_of(int device, std::string *why) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= (int)g_scratch_ptr.size()) {
        *why = "scratch not set up on this device";
        return nullptr;
    }
    if (!g_scratch_ptr[(size_t)device]) *why = g_scratch_err[(size_t)device];
    return g_scratch_ptr[(size_t)device];
}

HB_API hb_status hb_create(hb_ctx **out, int32_t device, void *hip_stream) {
    if (!out) return fail(nullptr, HB_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
        return fail(nullptr, HB_EDEVICE, "no HIP device");
    if (device < 0 || device >= ndev) return fail(nullptr, HB_EINVAL, "device index out of range");
    hb_ctx *c = new hb_ctx();
    c->device = device;
    DeviceGuard guard(device);
    if (!guard.ok) {
        delete c;
        return fail(nullptr, HB_EDEVICE, "hipSetDevice failed");
    }
    scratch_setup(device, ndev);
    {
        int nx = 1;
        if (hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, device) != hipSuccess || nx < 1)
            nx = 1;
        c->nx = nx > 16 ? 16 : nx;
        (void)hipGetLastError();
    }
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return fail(nullptr, HB_EDEVICE, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    if (hipEventCreateWithFlags(&c->desc_done, hipEventDisableTiming) != hipSuccess ||
        dalloc(c, &c->d_status, 1, "status") != HB_OK) {
        std::string m = c->err.empty() ? "event creation failed" : c->err;
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        if (c->desc_done) (void)hipEventDestroy(c->desc_done);
        delete c;
        return fail(nullptr, HB_ENOMEM, m);
    }
    if (hipMemsetAsync(c->d_status, 0, sizeof(int32_t), c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        dfree(&c->d_status);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        (void)hipEventDestroy(c->desc_done);
        delete c;
        return fail(nullptr, HB_EDEVICE, "status initialisation failed");
    }
    *out = c;
    return HB_OK;
}

static void free_ckpts(hb_ctx *c);

HB_API void hb_destroy(hb_ctx *c) {
    if (!c) return;
    {
        DeviceGuard guard(c->device);
        (void)hipStreamSynchronize(c->stream);
        dfree(&c->d_group);
        dfree(&c->d_perm_adj);
        dfree(&c->d_weight);
        dfree(&c->d_M);
        for (int i = 0; i < 2; ++i) {
            dfree(&c->pts[i]);
            dfree(&c->off[i]);
        }
        dfree(&c->d_counts);
        dfree(&c->d_tsum);
        dfree(&c->d_totals);
        dfree(&c->d_lens);
        dfree(&c->d_status);
        dfree(&c->d_ink);
        dfree(&c->d_hist);
        dfree(&c->d_histx);
        dfree(&c->d_bins);
        dfree(&c->d_binsrc);
        dfree(&c->d_bin_cnt);
        dfree(&c->d_bin_cur);
        dfree(&c->d_tile_off);
        dfree(&c->d_seg_off);
        dfree(&c->d_box);
        dfree(&c->d_tmp);
        dfree(&c->d_rho);
        dfree(&c->d_grad);
        dfree(&c->d_rhos);
        dfree(&c->d_grads);
        dfree(&c->d_jacc);
        dfree(&c->d_render);
        free_ckpts(c);
        dfree(&c->d_desc);
        if (c->h_desc) (void)hipHostFree(c->h_desc);
        if (c->desc_done) (void)hipEventDestroy(c->desc_done);
        for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
        if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
        for (hipEvent_t e : c->adj_ev) (void)hipEventDestroy(e);
        if (c->side) (void)hipStreamDestroy(c->side);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
    }
    delete c;
}

HB_API const char *hb_last_error(const hb_ctx *c) { return c ? c->err.c_str() : g_thread_err.c_str(); }

HB_API const char *hb_version(void) { return "hb 0.1 gfx950"; }

static hb_status finish_pending(hb_ctx *c);
static hb_status ensure_order(hb_ctx *c);

HB_API hb_status hb_set_params(hb_ctx *c, const hb_params *p) {
    ENTER(c);
    CHKST(finish_pending(c));
    CHKST(validate(c, p));
    if (c->have_graph && (p->grid_w != c->P.grid_w || p->grid_h != c->P.grid_h))
        c->have_samples = false;
    c->P = *p;
    if (p->n_sigmas > 0) {
        c->sigmas.assign(p->sigma_per_iter, p->sigma_per_iter + p->n_sigmas);
        int32_t rp[HB_MAX_PASSES];
        kovesi_radii((double)c->sigmas[0], p->box_passes, rp);
        c->radii.assign(1, rp[p->box_passes - 1]);
    } else {
        c->sigmas.clear();
        c->radii.assign(p->radius_per_iter, p->radius_per_iter + p->n_radii);
    }
    c->passw.clear();
    if (p->pass_weights) c->passw.assign(p->pass_weights, p->pass_weights + p->box_passes);
    c->P.radius_per_iter = nullptr;
    c->P.pass_weights = nullptr;
    c->P.sigma_per_iter = nullptr;
    if (c->P.capacity_factor == 0.0f) c->P.capacity_factor = 2.0f;
    c->have_params = true;
    c->ckpt_end_iter = -1;
    c->have_maps = false;
    return HB_OK;
}

// Copy `count` elements of a caller array (host, or device with HB_DEVICE_PTRS) to host.
template <typename T>
static hb_status to_host(hb_ctx *c, std::vector<T> &dst, const T *src, size_t count, uint32_t flags) {
    dst.resize(count);
    if (count == 0) return HB_OK;
    if (flags & HB_DEVICE_PTRS) {
        HIPCHK(c, hipMemcpyAsync(dst.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        memcpy(dst.data(), src, count * sizeof(T));
    }
    return HB_OK;
}

template <typename T>
static hb_status upload(hb_ctx *c, T *dst, const std::vector<T> &src) {
    if (src.empty()) return HB_OK;
    HIPCHK(c, hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HB_OK;
}

// Lay out the descriptor of a setup kernel on the state (pin/off_in) in slot 0.
static const char *const kOverflowMsg =
    "sample count too large for int32 histograms or int64 box sums, or 2^31 samples or more "
    "on one edge";
static const char *const kEntryMsg =
    "the line strips draw more pixels than the entry buffer holds (given polylines with "
    "segments much longer than delta_px)";

// Error of a non-zero device status word (cleared on the device).
static hb_status read_status(hb_ctx *c) {
    int32_t status = 0;
    HIPCHK(c, hipMemcpy(&status, c->d_status, sizeof status, hipMemcpyDeviceToHost));
    if (status == 0) return HB_OK;
    int32_t zero = 0;
    HIPCHK(c, hipMemcpy(c->d_status, &zero, sizeof zero, hipMemcpyHostToDevice));
    if (status & hb::ST_BIN_MISMATCH)
        return fail(c, HB_EINTERNAL, "binned samples disagree with the tile counts");
    if (status & hb::ST_ENTRY_OVERFLOW) return fail(c, HB_EOVERFLOW, kEntryMsg);
    return fail(c, HB_EOVERFLOW, kOverflowMsg);
}

static hb_status setup_scan_total(hb_ctx *c, int64_t *total_out) {
    // Scan the counts of the current state into off[1 - os] to learn the next sample count.
    CHKST(ensure_desc(c, 1));
    CHKST(ensure_totals(c, 1));
    CHKST(wait_desc(c));
    GDesc d = base_desc(c);
    set_iter_scalars(c, d, c->iter);
    d.cap = INT64_MAX;
    d.wmax = 0;   // no range checks: this scan only sizes the buffers
    d.off_s = c->off[1 - c->os];
    d.total = c->d_totals;
    d.r = 0;
    c->h_desc[0] = d;
    CHKST(upload_desc(c, 1));
    const Shape s = hb::shape_of(c->E, d.B, d.W, d.H, c->tiling);
    HIPCHK(c, hb::launch_scan(c->d_desc, 1, s, c->stream));
    CHKST(read_scalar(c, c->d_totals, total_out));
    CHKST(read_status(c));   // an edge with 2^31 samples or more
    return HB_OK;
}

HB_API hb_status hb_set_graph(hb_ctx *c, int32_t n_nodes, const float *node_xy, int64_t n_edges,
                              const int32_t *src, const int32_t *dst, const int32_t *weight,
                              uint32_t flags) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (!c->have_params) return fail(c, HB_ESTATE, "hb_set_params must come before hb_set_graph");
    if (n_edges < 0 || n_nodes < 0) return fail(c, HB_EINVAL, "negative size");
    if (n_edges > ((int64_t)1 << 31)) return fail(c, HB_EINVAL, "too many edges");
    if (n_edges > 0 && (n_nodes < 1 || !node_xy || !src || !dst))
        return fail(c, HB_EINVAL, "nodes, src and dst are required");
    std::vector<float> hx;
    std::vector<int32_t> hs, ht, hw;
    CHKST(to_host(c, hx, node_xy, (size_t)n_nodes * 2, flags));
    CHKST(to_host(c, hs, src, (size_t)n_edges, flags));
    CHKST(to_host(c, ht, dst, (size_t)n_edges, flags));
    if (weight) CHKST(to_host(c, hw, weight, (size_t)n_edges, flags));
    for (float v : hx)
        if (!std::isfinite(v)) return fail(c, HB_EINVAL, "node coordinates must be finite");
    for (int64_t e = 0; e < n_edges; ++e)
        if (hs[e] < 0 || hs[e] >= n_nodes || ht[e] < 0 || ht[e] >= n_nodes)
            return fail(c, HB_EINVAL, "edge end point out of range");
    int32_t wmax = 1;
    for (int32_t w : hw) {
        if (w < 1 || w > HB_MAX_EDGE_WEIGHT)
            return fail(c, HB_EINVAL, "edge weights must be in [1, HB_MAX_EDGE_WEIGHT]");
        wmax = std::max(wmax, w);
    }
    const int64_t E = n_edges;
    {
        // Morton code (16 bits per axis) of each edge's midpoint in the grid, for the
        // visiting order of the point kernels
        auto spread = [](uint32_t v) {
            v &= 0xffff;
            v = (v | (v << 8)) & 0x00ff00ffu;
            v = (v | (v << 4)) & 0x0f0f0f0fu;
            v = (v | (v << 2)) & 0x33333333u;
            v = (v | (v << 1)) & 0x55555555u;
            return v;
        };
        const double x0 = c->P.bbox[0], y0 = c->P.bbox[1], sx = c->P.bbox[2] - x0, sy = c->P.bbox[3] - y0;
        c->h_morton.resize((size_t)E);
        for (int64_t e = 0; e < E; ++e) {
            const float *a = &hx[2 * (size_t)hs[e]], *b = &hx[2 * (size_t)ht[e]];
            double mx = (0.5 * ((double)a[0] + b[0]) - x0) / sx, my = (0.5 * ((double)a[1] + b[1]) - y0) / sy;
            mx = std::min(std::max(mx, 0.0), 1.0);
            my = std::min(std::max(my, 0.0), 1.0);
            c->h_morton[e] = spread((uint32_t)(mx * 65535.0)) | (spread((uint32_t)(my * 65535.0)) << 1);
        }
        dfree(&c->d_perm_adj);
    }
    c->have_graph = false;
    c->have_samples = false;
    c->have_jacc = false;
    if (E != c->E) c->have_groups = false;
    c->E = E;
    c->wmax = wmax;
    CHKST(dalloc(c, &c->d_weight, hw.empty() ? 1 : hw.size(), "weights"));
    if (hw.empty()) dfree(&c->d_weight);
    else CHKST(upload(c, c->d_weight, hw));
    if (!c->have_groups) {
        CHKST(dalloc(c, &c->d_group, (size_t)E, "groups"));
        std::vector<int32_t> zero((size_t)E, 0);
        CHKST(upload(c, c->d_group, zero));
    }
    for (int i = 0; i < 2; ++i) CHKST(dalloc(c, &c->off[i], (size_t)E + 1, "offsets"));
    CHKST(dalloc(c, &c->d_counts, (size_t)E, "counts"));
    CHKST(dalloc(c, &c->d_lens, (size_t)E, "lengths"));
    CHKST(dalloc(c, &c->d_tsum, (size_t)(E / hb::kScanTile + 1), "scan tiles"));
    for (int i = 0; i < 2; ++i) dfree(&c->pts[i]);
    c->cap = 0;
    c->n_state = 0;
    c->n_samples = 0;
    c->ps = c->os = 0;
    CHKST(ensure_capacity(c, std::max<int64_t>(2 * E, 1024)));

    // straight two-point polylines from the nodes
    float2 *d_nodes = nullptr;
    int32_t *d_src = nullptr, *d_dst = nullptr;
    hb_status st = dalloc(c, &d_nodes, (size_t)std::max(1, n_nodes), "nodes");
    if (st == HB_OK) st = dalloc(c, &d_src, (size_t)E, "src");
    if (st == HB_OK) st = dalloc(c, &d_dst, (size_t)E, "dst");
    if (st == HB_OK && n_nodes > 0) {
        if (hipMemcpyAsync(d_nodes, hx.data(), hx.size() * sizeof(float), hipMemcpyHostToDevice, c->stream) != hipSuccess)
            st = fail_dev(c, hipGetLastError(), "node upload");
    }
    if (st == HB_OK) st = upload(c, d_src, hs);
    if (st == HB_OK) st = upload(c, d_dst, ht);
    if (st == HB_OK) st = ensure_desc(c, 1);
    if (st == HB_OK) st = wait_desc(c);
    if (st == HB_OK) {
        GDesc d = base_desc(c);
        set_iter_scalars(c, d, 0);
        d.pnew = c->pts[0];
        d.off_s = c->off[0];
        c->h_desc[0] = d;
        st = upload_desc(c, 1);
        if (st == HB_OK) {
            const Shape s = hb::shape_of(E, d.B, d.W, d.H, c->tiling);
            hipError_t e = hb::launch_init_state(c->d_desc, 1, s, d_nodes, d_src, d_dst,
                                                 c->P.bbox[0], c->P.bbox[1], c->P.bbox[2],
                                                 c->P.bbox[3], c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) st = fail_dev(c, e, "initial polylines");
        }
    }
    dfree(&d_nodes);
    dfree(&d_src);
    dfree(&d_dst);
    if (st != HB_OK) return st;
    c->ps = 0;
    c->os = 0;
    c->n_state = 2 * E;
    c->iter = 0;
    int64_t n0 = 0;
    CHKST(setup_scan_total(c, &n0));
    CHKST(ensure_capacity(c, (int64_t)std::ceil((double)n0 * c->P.capacity_factor) + 64));
    c->have_graph = true;
    c->ckpt_end_iter = -1;
    if (c->have_groups) CHKST(ensure_order(c));   // the edges' midpoints have changed
    return HB_OK;
}

// Edges sorted by group, then by the Morton code of their straight midpoint on a 256 x 256
// grid of cells (a stable counting sort, linear in the edge count).
static std::vector<int32_t> spatial_order(const hb_ctx *c) {
    const int64_t E = c->E;
    const std::vector<uint32_t> &mc = c->h_morton;
    const std::vector<int32_t> &g = c->h_group;
    const bool by_group = (int64_t)g.size() == E;
    int32_t B = 1;
    if (by_group)
        for (int32_t v : g) B = std::max(B, v + 1);
    const int64_t nkey = (int64_t)B << 16;
    auto key = [&](int64_t e) -> int64_t {
        return ((int64_t)(by_group ? g[e] : 0) << 16) | (int64_t)(mc[e] >> 16);
    };
    std::vector<int64_t> start((size_t)nkey + 1, 0);
    for (int64_t e = 0; e < E; ++e) ++start[(size_t)key(e) + 1];
    for (int64_t k = 0; k < nkey; ++k) start[(size_t)k + 1] += start[(size_t)k];
    std::vector<int32_t> perm((size_t)E);
    for (int64_t e = 0; e < E; ++e) perm[(size_t)start[(size_t)key(e)]++] = (int32_t)e;
    return perm;
}

HB_API hb_status hb_set_groups(hb_ctx *c, int32_t n_groups, const int32_t *group, const float *M,
                               uint32_t flags) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (!c->have_graph) return fail(c, HB_ESTATE, "hb_set_graph must come before hb_set_groups");
    if (n_groups < 1 || n_groups > HB_MAX_GROUPS) return fail(c, HB_EINVAL, "n_groups out of range [1, 64]");
    if (!M || (c->E > 0 && !group)) return fail(c, HB_EINVAL, "group and M are required");
    std::vector<int32_t> hg;
    std::vector<float> hm;
    CHKST(to_host(c, hg, group, (size_t)c->E, flags));
    CHKST(to_host(c, hm, M, (size_t)n_groups * n_groups, flags));
    for (int32_t b : hg)
        if (b < 0 || b >= n_groups) return fail(c, HB_EINVAL, "group index out of range [0, B)");
    for (float v : hm)
        if (!std::isfinite(v)) return fail(c, HB_EINVAL, "interaction matrix must be finite");
    CHKST(dalloc(c, &c->d_group, std::max<size_t>(1, hg.size()), "groups"));
    CHKST(upload(c, c->d_group, hg));
    CHKST(dalloc(c, &c->d_M, hm.size(), "interaction matrix"));
    CHKST(upload(c, c->d_M, hm));
    // the advection's edge order is rebuilt from the new groups when it is next needed (the
    // resampling and splat kernels visit the edges in index order)
    dfree(&c->d_perm_adj);
    c->h_group = hg;
    c->B = n_groups;
    c->have_groups = true;
    c->ckpt_end_iter = -1;
    c->have_maps = false;
    return ensure_order(c);   // the advection's edge order (host counting sort), built here
}

// ------------------------------------------------------------------ the iteration loop

// Edge order of the advection kernels (by group, then position): a counting sort on the host
// of the (group, Morton cell of the straight midpoint) keys, uploaded once; built when the
// groups are set (and again when the graph changes under them), so that no run pays for it.
static hb_status ensure_order(hb_ctx *c) {
    if (c->d_perm_adj) return HB_OK;
    const std::vector<int32_t> order = spatial_order(c);
    CHKST(dalloc(c, &c->d_perm_adj, std::max<size_t>(1, order.size()), "advection edge order"));
    CHKST(upload(c, c->d_perm_adj, order));
    return HB_OK;
}

// Internal run flag of hb_forward_ckpt: record the sample of every splat entry.
static const uint32_t kRunRecordBins = 1u << 30;

static hb_status prepare_ctx(hb_ctx *c, int T, uint32_t flags) {
    CHKST(ensure_order(c));
    CHKST(ensure_maps(c));
    CHKST(ensure_bins(c));
    CHKST(ensure_totals(c, T));
    if ((flags & HB_RUN_RECORD_DECISIONS) && c->jacc_cap < c->cap) {
        CHKST(dalloc(c, &c->d_jacc, (size_t)c->cap, "decisions"));
        c->jacc_cap = c->cap;
    }
    if ((flags & kRunRecordBins) && c->binsrc_cap < c->cap) {
        CHKST(dalloc(c, &c->d_binsrc, (size_t)c->cap, "binned samples"));
        c->binsrc_cap = c->cap;
    }
    return HB_OK;
}

static void shape_add(Shape &a, const Shape &b) {
    a.edge += b.edge; a.scan += b.scan; a.row += b.row; a.col += b.col;
    a.px += b.px; a.pxb += b.pxb; a.edget += b.edget; a.tile += b.tile; a.strip += b.strip;
}

// Enqueue T iterations of the graphs cs[0..n) on lead's stream: the descriptor table holds
// [T][n] entries (iteration-major) and every stage of an iteration is one launch for the
// whole batch. With use_graph the launches are captured once as a hipGraph and replayed
// while the batch layout is unchanged (only the descriptor contents change between runs).
static hb_status enqueue_batch(hb_ctx *lead, hb_ctx *const *cs, int n, int T, uint32_t flags,
                               bool use_graph) {
    for (int g = 0; g < n; ++g) {
        hb_status st = prepare_ctx(cs[g], T, flags);
        if (st != HB_OK) {
            if (cs[g] != lead) lead->err = cs[g]->err;
            return st;
        }
    }
    CHKST(ensure_desc(lead, (size_t)T * n));
    CHKST(wait_desc(lead));

    std::vector<Shape> base((size_t)n);
    Shape tot{};
    int max_w = 2, bmax = 1, pmax = 1;
    bool strip = false, points = false;   // graphs with line strips / with the point splat
    bool insdel = false;                  // graphs with the insert/delete resampling
    bool directed = false;                // graphs with a directed offset
    for (int g = 0; g < n; ++g) {
        const hb_ctx *c = cs[g];
        base[g] = tot;
        shape_add(tot, hb::shape_of(c->E, c->B, c->P.grid_w, c->P.grid_h, c->tiling));
        max_w = std::max(max_w, c->P.grid_w);
        bmax = std::max(bmax, c->B);
        pmax = std::max(pmax, c->P.box_passes);
        strip = strip || c->P.splat_mode == HB_SPLAT_STRIP;
        points = points || c->P.splat_mode != HB_SPLAT_STRIP;
        insdel = insdel || c->P.resample_mode == HB_RESAMPLE_INSERT_DELETE;
        directed = directed || c->P.directed_offset_px != 0.0f;
    }
    const bool given0 = (flags & HB_RUN_SAMPLES_GIVEN) != 0;
    const bool record = (flags & HB_RUN_RECORD_DECISIONS) != 0;
    for (int g = 0; g < n; ++g) {
        hb_ctx *c = cs[g];
        c->pend_ps.assign(T, 0);
        c->pend_os.assign(T, 0);
        int ps = c->ps, os = c->os, last_ss = 0, last_so = 0;
        for (int it = 0; it < T; ++it) {
            c->pend_ps[it] = ps;
            c->pend_os[it] = os;
            const bool given = it == 0 && given0;
            last_ss = given ? ps : 1 - ps;
            last_so = given ? os : 1 - os;
            GDesc d = base_desc(c);
            set_iter_scalars(c, d, c->iter + it);
            d.blk_edge = base[g].edge;
            d.blk_scan = base[g].scan;
            d.blk_row = base[g].row;
            d.blk_col = base[g].col;
            d.blk_px = base[g].px;
            d.blk_pxb = base[g].pxb;
            d.blk_edget = base[g].edget;
            d.blk_tile = base[g].tile;
            d.blk_strip = base[g].strip;
            d.record = record && it == T - 1;
            d.bin_src = (d.record && (flags & kRunRecordBins)) ? c->d_binsrc : nullptr;
            // samples not made by the uniform resampling are counted in tiles afterwards
            d.count_given = !d.strip && (given || d.insdel);
            d.total = c->d_totals + it;
            if (given) {
                d.samples = c->pts[ps];
                d.off_s = c->off[os];
                d.pnew = c->pts[1 - ps];
                ps = 1 - ps;
            } else {
                d.pin = c->pts[ps];
                d.off_in = c->off[os];
                d.samples = c->pts[1 - ps];
                d.off_s = c->off[1 - os];
                d.pnew = c->pts[ps];
                os = 1 - os;
            }
            lead->h_desc[(size_t)it * n + g] = d;
        }
        c->pending = true;
        c->ckpt_end_iter = -1;
        c->pend_start = c->iter;
        c->pend_T = T;
        c->pend_flags = flags;
        c->pend_lead = lead;
        // bookkeeping as if the run completes; finish_pending corrects it on overflow
        c->ss = last_ss;
        c->so = last_so;
        c->ps = ps;
        c->os = os;
        c->iter += T;
    }
    CHKST(upload_desc(lead, (size_t)T * n));

    const int ru = lead->tune_ru, au = lead->tune_au;
    auto launch_all = [&](bool timed) -> hb_status {
        HIPCHK(lead, hb::launch_fill_totals(lead->d_desc, n, T, lead->stream));
        for (int it = 0; it < T; ++it) {
            const GDesc *dd = lead->d_desc + (size_t)it * n;
            hb_ctx *c = lead;
            const bool given = it == 0 && given0;
            if (!timed) {
                if (!given && insdel) HIPCHK(c, hb::launch_insdel(dd, n, tot, false, c->stream));
                if (!given) HIPCHK(c, hb::launch_scan(dd, n, tot, c->stream));
                HIPCHK(c, hb::launch_clear_hist(dd, n, tot, c->stream));
                if (given) HIPCHK(c, hb::launch_count_given(dd, n, tot, c->stream));
                else HIPCHK(c, hb::launch_resample_count(dd, n, tot, ru, directed, c->stream));
                if (!given && insdel) {
                    HIPCHK(c, hb::launch_insdel(dd, n, tot, true, c->stream));
                    HIPCHK(c, hb::launch_count_given(dd, n, tot, c->stream));
                }
                if (strip) HIPCHK(c, hb::launch_strip_bins(dd, n, tot, false, c->stream));
                HIPCHK(c, hb::launch_bin_hist(dd, n, tot, strip, points, c->stream));
                for (int k = 0; k < pmax; ++k) HIPCHK(c, hb::launch_box_pass(dd, n, tot, max_w, k, c->stream));
                HIPCHK(c, hb::launch_density_strips(dd, n, tot, bmax, c->stream));
                HIPCHK(c, hb::launch_advect_smooth(dd, n, tot, au, c->stream));
                continue;
            }
            if (!given && insdel) STAGE(c, HB_STAGE_RESAMPLE_SPLAT, hb::launch_insdel(dd, n, tot, false, c->stream));
            if (!given) STAGE(c, HB_STAGE_SCAN, hb::launch_scan(dd, n, tot, c->stream));
            STAGE(c, HB_STAGE_CLEAR, hb::launch_clear_hist(dd, n, tot, c->stream));
            if (given) STAGE(c, HB_STAGE_RESAMPLE_SPLAT, hb::launch_count_given(dd, n, tot, c->stream));
            else STAGE(c, HB_STAGE_RESAMPLE_SPLAT, hb::launch_resample_count(dd, n, tot, ru, directed, c->stream));
            if (!given && insdel) {
                STAGE(c, HB_STAGE_RESAMPLE_SPLAT, hb::launch_insdel(dd, n, tot, true, c->stream));
                STAGE(c, HB_STAGE_BIN, hb::launch_count_given(dd, n, tot, c->stream));
            }
            if (strip) STAGE(c, HB_STAGE_BIN, hb::launch_strip_bins(dd, n, tot, false, c->stream));
            STAGE(c, HB_STAGE_BIN, hb::launch_bin_hist(dd, n, tot, strip, points, c->stream));
            for (int k = 0; k < pmax; ++k)
                STAGE(c, HB_STAGE_BOX, hb::launch_box_pass(dd, n, tot, max_w, k, c->stream));
            STAGE(c, HB_STAGE_DENSITY_GRAD, hb::launch_density_strips(dd, n, tot, bmax, c->stream));
            STAGE(c, HB_STAGE_ADVECT_SMOOTH, hb::launch_advect_smooth(dd, n, tot, au, c->stream));
        }
        return HB_OK;
    };

    if (!use_graph) return launch_all(lead->profiling);

    std::vector<int64_t> key = {n, T, (int64_t)flags, (int64_t)(intptr_t)lead->d_desc, ru, au,
                                max_w, bmax, pmax};
    for (int g = 0; g < n; ++g) {
        const hb_ctx *c = cs[g];
        key.insert(key.end(), {(int64_t)(intptr_t)c, c->E, c->B, c->P.grid_w, c->P.grid_h,
                               c->P.box_passes, c->P.splat_mode, c->P.resample_mode,
                               (int64_t)(c->P.directed_offset_px != 0.0f)});
    }
    if (!lead->gexec || key != lead->gkey) {
        if (lead->gexec) {
            (void)hipGraphExecDestroy(lead->gexec);
            lead->gexec = nullptr;
        }
        hipGraph_t graph = nullptr;
        HIPCHK(lead, hipStreamBeginCapture(lead->stream, hipStreamCaptureModeThreadLocal));
        hb_status st = launch_all(false);
        hipError_t e = hipStreamEndCapture(lead->stream, &graph);
        if (st != HB_OK) return st;
        if (e != hipSuccess) return fail_dev(lead, e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&lead->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail_dev(lead, e, "hipGraphInstantiate");
        lead->gkey = key;
    }
    HIPCHK(lead, hipGraphLaunch(lead->gexec, lead->stream));
    return HB_OK;
}

static hb_status enqueue_run(hb_ctx *c, int T, uint32_t flags) {
    hb_ctx *cs[1] = {c};
    return enqueue_batch(c, cs, 1, T, flags, (flags & HB_RUN_GRAPH) != 0);
}

static const uint32_t kRunFlags =
    HB_RUN_SAMPLES_GIVEN | HB_RUN_RECORD_DECISIONS | HB_RUN_ASYNC | HB_RUN_GRAPH;

HB_API hb_status hb_run(hb_ctx *c, int32_t n_iters, uint32_t flags) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (!c->have_params || !c->have_graph || !c->have_groups)
        return fail(c, HB_ESTATE, "hb_run needs parameters, graph and groups");
    if (n_iters < 0) return fail(c, HB_EINVAL, "n_iters must be >= 0");
    if (flags & ~kRunFlags) return fail(c, HB_EINVAL, "unknown run flags");
    c->last_counts.clear();
    if (n_iters == 0) return HB_OK;
    CHKST(enqueue_run(c, n_iters, flags));
    if (flags & HB_RUN_ASYNC) return HB_OK;
    return finish_pending(c);
}

// Wait for an enqueued run; on a point-buffer overflow grow the buffers and run the
// remaining iterations again from the last complete state.
static hb_status finish_pending(hb_ctx *c) {
    while (c->pending) {
        c->pending = false;
        hb_ctx *lead = c->pend_lead ? c->pend_lead : c;
        c->pend_lead = nullptr;
        HIPCHK(c, hipStreamSynchronize(lead->stream));
        if (lead == c) CHKST(stage_collect(c));
        int32_t status = 0;
        HIPCHK(c, hipMemcpy(&status, c->d_status, sizeof status, hipMemcpyDeviceToHost));
        const int T = c->pend_T;
        std::vector<int64_t> tot((size_t)T);
        HIPCHK(c, hipMemcpy(tot.data(), c->d_totals, sizeof(int64_t) * T, hipMemcpyDeviceToHost));
        const bool given0 = (c->pend_flags & HB_RUN_SAMPLES_GIVEN) != 0;
        if (given0) tot[0] = c->n_state;
        if (status == 0) {
            c->last_counts.insert(c->last_counts.end(), tot.begin(), tot.end());
            c->n_state = tot[T - 1];
            c->n_samples = tot[T - 1];
            c->have_samples = true;
            c->have_maps = true;
            c->have_jacc = (c->pend_flags & HB_RUN_RECORD_DECISIONS) != 0;
            return HB_OK;
        }
        // first iteration that stopped
        int f = 0;
        while (f < T && !(tot[f] < 0 || tot[f] > c->cap)) ++f;
        if (f >= T) f = T - 1;
        const int64_t need = tot[f] > 0 ? tot[f] : c->cap;
        c->last_counts.insert(c->last_counts.end(), tot.begin(), tot.begin() + f);
        c->ps = c->pend_ps[f];
        c->os = c->pend_os[f];
        c->iter = c->pend_start + f;
        if (f > 0) c->n_state = tot[f - 1];
        c->have_samples = false;
        int32_t zero = 0;
        HIPCHK(c, hipMemcpy(c->d_status, &zero, sizeof zero, hipMemcpyHostToDevice));
        if (status & hb::ST_BIN_MISMATCH)
            return fail(c, HB_EINTERNAL, "binned samples disagree with the tile counts");
        if (status & hb::ST_HIST_OVERFLOW)
            return fail(c, HB_EOVERFLOW, kOverflowMsg);
        if (status & hb::ST_ENTRY_OVERFLOW)
            return fail(c, HB_EOVERFLOW, kEntryMsg);
        CHKST(ensure_capacity(c, 2 * need + 64));
        uint32_t flags = c->pend_flags & ~(uint32_t)(HB_RUN_ASYNC | HB_RUN_GRAPH);
        if (f > 0) flags &= ~(uint32_t)HB_RUN_SAMPLES_GIVEN;
        CHKST(enqueue_run(c, T - f, flags));
    }
    return HB_OK;
}

HB_API hb_status hb_sync(hb_ctx *c) {
    ENTER(c);
    return finish_pending(c);
}

// ------------------------------------------------------------------ batches

static hb_status check_batch(hb_ctx *const *ctxs, int32_t n) {
    if (!ctxs || n < 1) return fail(nullptr, HB_EINVAL, "need at least one context");
    if (!ctxs[0]) return fail(nullptr, HB_EINVAL, "null context");
    for (int g = 0; g < n; ++g) {
        hb_ctx *c = ctxs[g];
        if (!c) return fail(ctxs[0], HB_EINVAL, "null context in batch");
        if (c->sticky) return fail(ctxs[0], HB_EDEVICE, "a context of the batch has a sticky HIP error");
        if (c->device != ctxs[0]->device) return fail(ctxs[0], HB_EINVAL, "contexts on different devices");
        for (int h = 0; h < g; ++h)
            if (ctxs[h] == c) return fail(ctxs[0], HB_EINVAL, "context listed twice");
        if (!c->have_params || !c->have_graph || !c->have_groups)
            return fail(ctxs[0], HB_ESTATE, "every context needs parameters, graph and groups");
    }
    return HB_OK;
}

HB_API hb_status hb_batch_run(hb_ctx *const *ctxs, int32_t n, int32_t n_iters, uint32_t flags) {
    CHKST(check_batch(ctxs, n));
    hb_ctx *lead = ctxs[0];
    ENTER(lead);
    if (n_iters < 0) return fail(lead, HB_EINVAL, "n_iters must be >= 0");
    if (flags & ~(uint32_t)(HB_RUN_ASYNC | HB_RUN_GRAPH | HB_RUN_RECORD_DECISIONS))
        return fail(lead, HB_EINVAL,
                    "batch runs take HB_RUN_ASYNC, HB_RUN_GRAPH and HB_RUN_RECORD_DECISIONS only");
    for (int g = 0; g < n; ++g) {
        hb_status st = finish_pending(ctxs[g]);
        if (st != HB_OK) return fail(lead, st, ctxs[g]->err);
        HIPCHK(lead, hipStreamSynchronize(ctxs[g]->stream));
        ctxs[g]->last_counts.clear();
    }
    if (n_iters == 0) return HB_OK;
    CHKST(enqueue_batch(lead, ctxs, n, n_iters, flags, (flags & HB_RUN_GRAPH) != 0));
    if (flags & HB_RUN_ASYNC) return HB_OK;
    hb_status first = HB_OK;
    for (int g = 0; g < n; ++g) {
        hb_status st = finish_pending(ctxs[g]);
        if (st != HB_OK && first == HB_OK) {
            first = st;
            lead->err = ctxs[g]->err;
        }
    }
    return first;
}

// Snapshot of the polylines and counts of a context (for trial runs of the autotuner).
struct Snapshot {
    float2 *pts = nullptr;
    int64_t *off = nullptr, *counts = nullptr;
    double *lens = nullptr;
    int64_t n = 0;
    int ps = 0, os = 0, iter = 0;
};

static hb_status take_snapshot(hb_ctx *c, Snapshot &s) {
    s.n = c->n_state;
    s.ps = c->ps;
    s.os = c->os;
    s.iter = c->iter;
    CHKST(dalloc(c, &s.pts, (size_t)std::max<int64_t>(1, s.n), "snapshot"));
    CHKST(dalloc(c, &s.off, (size_t)c->E + 1, "snapshot"));
    CHKST(dalloc(c, &s.counts, (size_t)std::max<int64_t>(1, c->E), "snapshot"));
    CHKST(dalloc(c, &s.lens, (size_t)std::max<int64_t>(1, c->E), "snapshot"));
    HIPCHK(c, hipMemcpyAsync(s.pts, c->pts[c->ps], sizeof(float2) * s.n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(s.off, c->off[c->os], sizeof(int64_t) * (c->E + 1), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(s.counts, c->d_counts, sizeof(int64_t) * c->E, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(s.lens, c->d_lens, sizeof(double) * c->E, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HB_OK;
}

static hb_status restore_snapshot(hb_ctx *c, Snapshot &s) {
    c->ps = s.ps;
    c->os = s.os;
    c->iter = s.iter;
    c->n_state = s.n;
    c->have_samples = false;
    c->have_jacc = false;
    HIPCHK(c, hipMemcpyAsync(c->pts[c->ps], s.pts, sizeof(float2) * s.n, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->off[c->os], s.off, sizeof(int64_t) * (c->E + 1), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_counts, s.counts, sizeof(int64_t) * c->E, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_lens, s.lens, sizeof(double) * c->E, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dfree(&s.pts);
    dfree(&s.off);
    dfree(&s.counts);
    dfree(&s.lens);
    return HB_OK;
}

// Tiling values the autotuner and hb_set_tiling accept.
static constexpr int kSetsLimit = hb::kBinSetsMax;
static bool tiling_ok(int32_t col_rows, int32_t sets_max, int64_t item_entries) {
    auto pow2 = [](int64_t v) { return v > 0 && (v & (v - 1)) == 0; };
    return pow2(col_rows) && col_rows >= 16 && col_rows <= 1024 && pow2(sets_max) &&
           sets_max <= kSetsLimit && pow2(item_entries) && item_entries >= (1 << 12) &&
           item_entries <= (1 << 20);
}

// One setting of every tunable launch shape of a batch.
struct TuneSet {
    int ru, au;
    hb::Tiling tg;
};

static void apply_tune(hb_ctx *const *ctxs, int n, const TuneSet &t) {
    for (int g = 0; g < n; ++g) {
        ctxs[g]->tune_ru = t.ru;
        ctxs[g]->tune_au = t.au;
        ctxs[g]->tiling = t.tg;
    }
}

// Chooses the launch shapes of a batch by timing n_iters iterations of each candidate from
// the current polylines (restored afterwards), one shape at a time: the work chunks per
// trip of the resampling and advection kernels, then the rows per thread of the column box
// pass, the tile-count sets of the splat (how many privatised copies of the tile counters
// the edge blocks spread their atomics over) and the entries per tile-histogram work item.
HB_API hb_status hb_autotune(hb_ctx *const *ctxs, int32_t n, int32_t n_iters, int32_t *choice) {
    CHKST(check_batch(ctxs, n));
    hb_ctx *lead = ctxs[0];
    ENTER(lead);
    if (n_iters < 1) return fail(lead, HB_EINVAL, "n_iters must be >= 1");
    for (int g = 0; g < n; ++g) CHKST(finish_pending(ctxs[g]));
    hipEvent_t e0, e1;
    HIPCHK(lead, hipEventCreate(&e0));
    HIPCHK(lead, hipEventCreate(&e1));
    const bool prof = lead->profiling;
    lead->profiling = false;
    hb_status st = HB_OK;
    auto trial = [&](const TuneSet &t, float *ms) -> hb_status {
        std::vector<Snapshot> snap((size_t)n);
        for (int g = 0; g < n; ++g) CHKST(take_snapshot(ctxs[g], snap[g]));
        apply_tune(ctxs, n, t);
        for (int g = 0; g < n; ++g) CHKST(ensure_maps(ctxs[g]));
        if (hipEventRecord(e0, lead->stream) != hipSuccess) return fail_dev(lead, hipGetLastError(), "event");
        CHKST(enqueue_batch(lead, ctxs, n, n_iters, 0, false));
        if (hipEventRecord(e1, lead->stream) != hipSuccess) return fail_dev(lead, hipGetLastError(), "event");
        for (int g = 0; g < n; ++g) CHKST(finish_pending(ctxs[g]));
        if (hipEventElapsedTime(ms, e0, e1) != hipSuccess) return fail_dev(lead, hipGetLastError(), "event");
        for (int g = 0; g < n; ++g) CHKST(restore_snapshot(ctxs[g], snap[g]));
        return HB_OK;
    };
    TuneSet best{lead->tune_ru, lead->tune_au, lead->tiling};
    float best_ms = -1.0f;
    // stage 1: work chunks per trip
    static const int cand[][2] = {{1, 1}, {1, 2}, {2, 2}, {1, 4}, {2, 4}, {4, 4}};
    std::vector<TuneSet> sets;
    for (const auto &c : cand) sets.push_back(TuneSet{c[0], c[1], best.tg});
    auto pick = [&](std::vector<TuneSet> cs) -> hb_status {
        for (const TuneSet &t : cs) {
            float ms = 0.0f;
            CHKST(trial(t, &ms));
            if (best_ms < 0.0f || ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
        return HB_OK;
    };
    st = pick(sets);
    // stage 2: rows per thread of the column box pass
    if (st == HB_OK) {
        sets.clear();
        for (int rows : {64, 256}) {
            TuneSet t = best;
            t.tg.col_rows = rows;
            sets.push_back(t);
        }
        st = pick(sets);
    }
    // stage 3: tile-count sets (privatised copies of the tile counters)
    if (st == HB_OK) {
        sets.clear();
        for (int k : {4, 16}) {
            TuneSet t = best;
            t.tg.sets_max = k;
            sets.push_back(t);
        }
        st = pick(sets);
    }
    // stage 4: entries per tile-histogram work item
    if (st == HB_OK) {
        sets.clear();
        for (int64_t v : {int64_t(1) << 14, int64_t(1) << 15, int64_t(1) << 17}) {
            TuneSet t = best;
            t.tg.item_entries = v;
            sets.push_back(t);
        }
        st = pick(sets);
    }
    lead->profiling = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != HB_OK) return st;
    apply_tune(ctxs, n, best);
    for (int g = 0; g < n; ++g) {
        CHKST(ensure_maps(ctxs[g]));
        ctxs[g]->last_counts.clear();
        ctxs[g]->ckpt_end_iter = -1;
    }
    if (choice) {
        choice[0] = best.ru;
        choice[1] = best.au;
        choice[2] = best.tg.col_rows;
        choice[3] = best.tg.sets_max;
        int lg = 0;
        while ((int64_t(1) << lg) < best.tg.item_entries) ++lg;
        choice[4] = lg;
    }
    return HB_OK;
}

HB_API hb_status hb_set_tiling(hb_ctx *c, int32_t col_rows, int32_t sets_max, int32_t item_entries_log2) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (item_entries_log2 < 0 || item_entries_log2 > 30 ||
        !tiling_ok(col_rows, sets_max, int64_t(1) << item_entries_log2))
        return fail(c, HB_EINVAL, "tiling: col_rows a power of two in [16, 1024], sets_max a power of "
                                  "two in [1, 64], item_entries_log2 in [12, 20]");
    c->tiling.col_rows = col_rows;
    c->tiling.sets_max = sets_max;
    c->tiling.item_entries = int64_t(1) << item_entries_log2;
    c->ckpt_end_iter = -1;
    if (c->have_graph && c->have_groups) CHKST(ensure_maps(c));
    return HB_OK;
}

HB_API hb_status hb_get_tiling(hb_ctx *c, int32_t *col_rows, int32_t *sets_max, int32_t *item_entries_log2) {
    ENTER(c);
    if (!col_rows || !sets_max || !item_entries_log2) return fail(c, HB_EINVAL, "null output");
    *col_rows = c->tiling.col_rows;
    *sets_max = c->tiling.sets_max;
    int lg = 0;
    while ((int64_t(1) << lg) < c->tiling.item_entries) ++lg;
    *item_entries_log2 = lg;
    return HB_OK;
}

HB_API hb_status hb_set_tuning(hb_ctx *c, int32_t resample_chunks, int32_t advect_chunks) {
    ENTER(c);
    auto ok = [](int v) { return v == 1 || v == 2 || v == 4; };
    if (!ok(resample_chunks) || !ok(advect_chunks)) return fail(c, HB_EINVAL, "chunk counts are 1, 2 or 4");
    c->tune_ru = resample_chunks;
    c->tune_au = advect_chunks;
    return HB_OK;
}

HB_API hb_status hb_get_tuning(hb_ctx *c, int32_t *resample_chunks, int32_t *advect_chunks) {
    ENTER(c);
    if (!resample_chunks || !advect_chunks) return fail(c, HB_EINVAL, "null output");
    *resample_chunks = c->tune_ru;
    *advect_chunks = c->tune_au;
    return HB_OK;
}

// ------------------------------------------------------------------ data movement

static hb_status copy_out(hb_ctx *c, void *dst, const void *src, size_t bytes, uint32_t flags) {
    if (bytes == 0) return HB_OK;
    HIPCHK(c, hipMemcpyAsync(dst, src, bytes,
                             (flags & HB_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HB_OK;
}

HB_API hb_status hb_get_num_points(hb_ctx *c, int32_t which, int64_t *n) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (!n) return fail(c, HB_EINVAL, "n_points is NULL");
    if (!c->have_graph) return fail(c, HB_ESTATE, "no graph");
    if (which == HB_POINTS_STATE) *n = c->n_state;
    else if (which == HB_POINTS_SAMPLES) {
        if (!c->have_samples) return fail(c, HB_ESTATE, "no samples: run an iteration first");
        *n = c->n_samples;
    } else return fail(c, HB_EINVAL, "unknown point set");
    return HB_OK;
}

HB_API hb_status hb_get_points(hb_ctx *c, int32_t which, int64_t *offsets, float *xy,
                               int64_t cap_points, uint32_t flags) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (!c->have_graph) return fail(c, HB_ESTATE, "no graph");
    int pi, oi;
    int64_t n;
    if (which == HB_POINTS_STATE) {
        pi = c->ps; oi = c->os; n = c->n_state;
    } else if (which == HB_POINTS_SAMPLES) {
        if (!c->have_samples) return fail(c, HB_ESTATE, "no samples: run an iteration first");
        pi = c->ss; oi = c->so; n = c->n_samples;
    } else return fail(c, HB_EINVAL, "unknown point set");
    if (cap_points < n) return fail(c, HB_EINVAL, "xy buffer too small");
    if (!offsets || (n > 0 && !xy)) return fail(c, HB_EINVAL, "offsets and xy are required");
    CHKST(copy_out(c, offsets, c->off[oi], sizeof(int64_t) * (size_t)(c->E + 1), flags));
    CHKST(copy_out(c, xy, c->pts[pi], sizeof(float2) * (size_t)n, flags));
    return HB_OK;
}

HB_API hb_status hb_set_points(hb_ctx *c, const int64_t *offsets, const float *xy, int64_t n_points,
                               uint32_t flags) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (!c->have_graph) return fail(c, HB_ESTATE, "hb_set_graph must come first");
    if (!offsets || (n_points > 0 && !xy)) return fail(c, HB_EINVAL, "offsets and xy are required");
    std::vector<int64_t> ho;
    CHKST(to_host(c, ho, offsets, (size_t)c->E + 1, flags));
    if (ho[0] != 0 || ho[c->E] != n_points) return fail(c, HB_EINVAL, "offsets must run from 0 to n_points");
    for (int64_t e = 0; e < c->E; ++e)
        if (ho[e + 1] - ho[e] < 2) return fail(c, HB_EINVAL, "every polyline needs at least two points");
    std::vector<float> hx;
    CHKST(to_host(c, hx, xy, (size_t)n_points * 2, flags));
    for (float v : hx)
        if (!std::isfinite(v)) return fail(c, HB_EINVAL, "point coordinates must be finite");
    c->have_samples = false;
    c->have_jacc = false;
    c->n_state = 0;
    CHKST(ensure_capacity(c, n_points));
    c->ps = 0;
    c->os = 0;
    CHKST(upload(c, c->off[0], ho));
    if (n_points > 0)
        HIPCHK(c, hipMemcpy(c->pts[0], hx.data(), hx.size() * sizeof(float), hipMemcpyHostToDevice));
    c->n_state = n_points;
    c->ckpt_end_iter = -1;
    CHKST(ensure_desc(c, 1));
    CHKST(wait_desc(c));
    GDesc d = base_desc(c);
    set_iter_scalars(c, d, c->iter);
    d.pin = c->pts[0];
    d.off_in = c->off[0];
    c->h_desc[0] = d;
    CHKST(upload_desc(c, 1));
    const Shape s = hb::shape_of(c->E, d.B, d.W, d.H, c->tiling);
    HIPCHK(c, hb::launch_lengths(c->d_desc, 1, s, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HB_OK;
}

HB_API hb_status hb_get_map(hb_ctx *c, int32_t kind, int32_t group, int32_t pass, void *out,
                            int64_t bytes, uint32_t flags) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (!c->have_maps) return fail(c, HB_ESTATE, "no maps: run an iteration first");
    if (!out) return fail(c, HB_EINVAL, "out is NULL");
    if (group < 0 || group >= c->map_B) return fail(c, HB_EINVAL, "group index out of range");
    const size_t plane = (size_t)c->map_W * c->map_H;
    const size_t gofs = (size_t)group * plane;
    const void *src;
    size_t need;
    switch (kind) {
        case HB_MAP_HIST: src = c->d_hist + gofs; need = plane * sizeof(int32_t); break;
        case HB_MAP_BOX:
            if (pass < 1 || pass > c->map_P) return fail(c, HB_EINVAL, "pass out of range [1, P]");
            src = c->d_box + (size_t)(pass - 1) * c->map_B * plane + gofs;
            need = plane * sizeof(int64_t);
            break;
        case HB_MAP_DENSITY: src = c->d_rho + gofs; need = plane * sizeof(float); break;
        case HB_MAP_GRAD: src = c->d_grad + gofs; need = plane * sizeof(float2); break;
        default: return fail(c, HB_EINVAL, "unknown map kind");
    }
    if (bytes < (int64_t)need) return fail(c, HB_EINVAL, "output buffer too small");
    return copy_out(c, out, src, need, flags);
}

HB_API hb_status hb_get_decisions(hb_ctx *c, int8_t *jacc, int64_t cap_points, uint32_t flags) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (!c->have_jacc || !c->have_samples)
        return fail(c, HB_ESTATE, "no decisions: run with HB_RUN_RECORD_DECISIONS");
    if (!jacc || cap_points < c->n_samples) return fail(c, HB_EINVAL, "buffer too small");
    return copy_out(c, jacc, c->d_jacc, (size_t)c->n_samples, flags);
}

HB_API hb_status hb_get_iter_counts(hb_ctx *c, int64_t *counts, int32_t cap) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (!counts || cap < (int32_t)c->last_counts.size()) return fail(c, HB_EINVAL, "buffer too small");
    std::copy(c->last_counts.begin(), c->last_counts.end(), counts);
    return HB_OK;
}

HB_API hb_status hb_get_ink(hb_ctx *c, double *ink) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (!ink) return fail(c, HB_EINVAL, "ink is NULL");
    if (!c->have_graph) return fail(c, HB_ESTATE, "no graph");
    if (!c->d_ink) CHKST(dalloc(c, &c->d_ink, (size_t)hb::kInkSlices + 1, "ink"));
    HIPCHK(c, hb::launch_ink(c->d_lens, c->E, c->d_ink, c->stream));
    HIPCHK(c, hipMemcpyAsync(ink, c->d_ink + hb::kInkSlices, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HB_OK;
}

// ------------------------------------------------------------------ grouping (Section 5)

HB_API hb_status hb_edge_features(hb_ctx *c, int32_t kind, float *out, int64_t cap_floats,
                                  uint32_t flags) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (flags & ~(uint32_t)HB_DEVICE_PTRS) return fail(c, HB_EINVAL, "unknown flags");
    if (!c->have_graph) return fail(c, HB_ESTATE, "hb_edge_features needs hb_set_graph");
    static const int kDim[4] = {2, 2, 4, 1};
    if (kind < 0 || kind > 3) return fail(c, HB_EINVAL, "unknown edge feature kind");
    const int64_t need = c->E * kDim[kind];
    if (!out || cap_floats < need) return fail(c, HB_EINVAL, "output buffer missing or too small");
    if (c->E == 0) return HB_OK;
    CHKST(ensure_desc(c, 1));
    CHKST(wait_desc(c));
    GDesc d = base_desc(c);
    d.pin = c->pts[c->ps];       // the end points never move
    d.off_in = c->off[c->os];
    c->h_desc[0] = d;
    CHKST(upload_desc(c, 1));
    float *dst = out, *tmp = nullptr;
    if (!(flags & HB_DEVICE_PTRS)) {
        CHKST(dalloc(c, &tmp, (size_t)need, "edge features"));
        dst = tmp;
    }
    hipError_t e = hb::launch_edge_features(c->d_desc, c->E, kind, dst, c->stream);
    if (e == hipSuccess && tmp)
        e = hipMemcpyAsync(out, tmp, sizeof(float) * (size_t)need, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dfree(&tmp);
    if (e != hipSuccess) return fail_dev(c, e, "edge features");
    return HB_OK;
}

// Device buffers of one grouping call, freed on return.
struct KmBufs {
    float *X = nullptr;
    int32_t *lab = nullptr, *best = nullptr, *chosen = nullptr;
    double *part = nullptr, *tot = nullptr, *cen = nullptr, *db = nullptr;
    int64_t *idx = nullptr;
    ~KmBufs() {
        dfree(&X);
        dfree(&lab);
        dfree(&best);
        dfree(&chosen);
        dfree(&part);
        dfree(&tot);
        dfree(&cen);
        dfree(&db);
        dfree(&idx);
    }
};

static hb_status km_check(hb_ctx *c, const float *X, int64_t n, int32_t dim, int32_t kmax,
                          uint32_t flags) {
    if (flags & ~(uint32_t)HB_DEVICE_PTRS) return fail(c, HB_EINVAL, "unknown flags");
    if (!X) return fail(c, HB_EINVAL, "X is NULL");
    if (dim < 1 || dim > HB_KMEANS_MAX_DIM) return fail(c, HB_EINVAL, "dim must be in [1, HB_KMEANS_MAX_DIM]");
    if (kmax < 1 || kmax > HB_KMEANS_MAX_K) return fail(c, HB_EINVAL, "k must be in [1, HB_KMEANS_MAX_K]");
    if (n < kmax) return fail(c, HB_EINVAL, "need at least k points");
    if (n > ((int64_t)1 << 31)) return fail(c, HB_EINVAL, "at most 2^31 points");
    return HB_OK;
}

// Points on the device (copied when given in host memory) and the work buffers for up to
// kmax clusters.
static hb_status km_setup(hb_ctx *c, KmBufs &b, const float *X, int64_t n, int32_t dim, int32_t kmax,
                          uint32_t flags, const float **dX) {
    if (flags & HB_DEVICE_PTRS) {
        *dX = X;
    } else {
        CHKST(dalloc(c, &b.X, (size_t)(n * dim), "k-means points"));
        HIPCHK(c, hipMemcpyAsync(b.X, X, sizeof(float) * (size_t)(n * dim), hipMemcpyHostToDevice, c->stream));
        *dX = b.X;
    }
    const int64_t nblk = (n + hb::kBlock - 1) / hb::kBlock;
    const int64_t w = (int64_t)kmax * (dim + 1) + 2;
    CHKST(dalloc(c, &b.part, (size_t)(nblk * hb::kWavesPerBlock * w), "k-means partial sums"));
    CHKST(dalloc(c, &b.tot, (size_t)w, "k-means sums"));
    CHKST(dalloc(c, &b.cen, (size_t)kmax * dim, "k-means centres"));
    CHKST(dalloc(c, &b.db, 1, "Davies-Bouldin index"));
    CHKST(dalloc(c, &b.idx, (size_t)kmax, "k-means start indices"));
    return HB_OK;
}

// Lloyd rounds from the centres in b.cen; labels in dlab (device).
static hb_status km_run(hb_ctx *c, KmBufs &b, const float *dX, int64_t n, int32_t dim, int32_t k,
                        int32_t max_iters, int32_t *dlab, double *inertia, int32_t *rounds) {
    HIPCHK(c, hipMemsetAsync(dlab, 0xff, sizeof(int32_t) * (size_t)n, c->stream));   // -1: none yet
    const int w = k * (dim + 1) + 2;
    int32_t r = 0;
    for (int32_t it = 0; it < max_iters; ++it) {
        HIPCHK(c, hb::launch_km_round(dX, n, dim, k, b.cen, dlab, 0, b.part, b.tot, c->stream));
        double changed = 0.0;
        HIPCHK(c, hipMemcpyAsync(&changed, b.tot + (w - 1), sizeof changed, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        r = it + 1;
        if (changed == 0.0) break;
        HIPCHK(c, hb::launch_km_means(b.tot, dim, k, 1, b.cen, c->stream));
        if (it + 1 == max_iters)   // the sums of squared distances to the final centres
            HIPCHK(c, hb::launch_km_round(dX, n, dim, k, b.cen, dlab, 1, b.part, b.tot, c->stream));
    }
    double in = 0.0;
    HIPCHK(c, hipMemcpyAsync(&in, b.tot + (w - 2), sizeof in, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (inertia) *inertia = in;
    if (rounds) *rounds = r;
    return HB_OK;
}

// Davies-Bouldin index of the labels dlab (device); invalid labels give HB_EINVAL.
static hb_status km_db(hb_ctx *c, KmBufs &b, const float *dX, int64_t n, int32_t dim, int32_t k,
                       int32_t *dlab, double *db) {
    const int w = k * (dim + 1) + 2;
    HIPCHK(c, hipMemsetAsync(b.cen, 0, sizeof(double) * (size_t)k * dim, c->stream));
    HIPCHK(c, hb::launch_km_round(dX, n, dim, k, b.cen, dlab, 1, b.part, b.tot, c->stream));
    HIPCHK(c, hb::launch_km_means(b.tot, dim, k, 0, b.cen, c->stream));       // centroids
    HIPCHK(c, hb::launch_km_round(dX, n, dim, k, b.cen, dlab, 2, b.part, b.tot, c->stream));
    HIPCHK(c, hb::launch_km_db(b.tot, b.cen, dim, k, b.db, c->stream));
    double bad = 0.0;
    HIPCHK(c, hipMemcpyAsync(&bad, b.tot + (w - 1), sizeof bad, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(db, b.db, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (bad != 0.0) return fail(c, HB_EINVAL, "labels outside [0, k)");
    return HB_OK;
}

HB_API hb_status hb_kmeans(hb_ctx *c, const float *X, int64_t n, int32_t dim, int32_t k,
                           double *centers, int32_t max_iters, int32_t *labels, double *inertia,
                           int32_t *rounds, uint32_t flags) {
    ENTER(c);
    CHKST(finish_pending(c));
    CHKST(km_check(c, X, n, dim, k, flags));
    if (!centers || !labels) return fail(c, HB_EINVAL, "centers or labels is NULL");
    if (max_iters < 1) return fail(c, HB_EINVAL, "max_iters must be >= 1");
    for (int64_t i = 0; i < (int64_t)k * dim; ++i)
        if (!std::isfinite(centers[i])) return fail(c, HB_EINVAL, "starting centres not finite");
    KmBufs b;
    const float *dX = nullptr;
    CHKST(km_setup(c, b, X, n, dim, k, flags, &dX));
    int32_t *dlab = labels;
    if (!(flags & HB_DEVICE_PTRS)) {
        CHKST(dalloc(c, &b.lab, (size_t)n, "k-means labels"));
        dlab = b.lab;
    }
    HIPCHK(c, hipMemcpyAsync(b.cen, centers, sizeof(double) * (size_t)k * dim, hipMemcpyHostToDevice, c->stream));
    CHKST(km_run(c, b, dX, n, dim, k, max_iters, dlab, inertia, rounds));
    HIPCHK(c, hipMemcpyAsync(centers, b.cen, sizeof(double) * (size_t)k * dim, hipMemcpyDeviceToHost, c->stream));
    if (b.lab)
        HIPCHK(c, hipMemcpyAsync(labels, b.lab, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return HB_OK;
}

HB_API hb_status hb_davies_bouldin(hb_ctx *c, const float *X, int64_t n, int32_t dim, int32_t k,
                                   const int32_t *labels, double *db, uint32_t flags) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (!labels || !db) return fail(c, HB_EINVAL, "labels or db is NULL");
    if (n < 1) return fail(c, HB_EINVAL, "no points");
    CHKST(km_check(c, X, n, dim, 1, flags));
    if (k < 1 || k > HB_KMEANS_MAX_K) return fail(c, HB_EINVAL, "k must be in [1, HB_KMEANS_MAX_K]");
    KmBufs b;
    const float *dX = nullptr;
    CHKST(km_setup(c, b, X, n, dim, k, flags, &dX));
    int32_t *dlab = const_cast<int32_t *>(labels);
    if (!(flags & HB_DEVICE_PTRS)) {
        CHKST(dalloc(c, &b.lab, (size_t)n, "labels"));
        HIPCHK(c, hipMemcpyAsync(b.lab, labels, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, c->stream));
        dlab = b.lab;
    }
    return km_db(c, b, dX, n, dim, k, dlab, db);
}

// hb_davies_bouldin on device inputs with the fixed scratch array: the points are taken in
// chunks of kNaChunk, each chunk's sums reduced in a fixed order and added in chunk order.
HB_API hb_status hb_davies_bouldin_noalloc(hb_ctx *c, const float *X, int64_t n, int32_t dim,
                                           int32_t k, const int32_t *labels, double *db) {
    ENTER(c);
    if (c->pending) return fail(c, HB_ESTATE, "an asynchronous run is pending (hb_sync first)");
    if (!labels || !db) return fail(c, HB_EINVAL, "labels or db is NULL");
    if (n < 1) return fail(c, HB_EINVAL, "no points");
    CHKST(km_check(c, X, n, dim, 1, HB_DEVICE_PTRS));
    if (k < 1 || k > HB_KMEANS_MAX_K) return fail(c, HB_EINVAL, "k must be in [1, HB_KMEANS_MAX_K]");
    const int w = k * (dim + 1) + 2;
    if (w > kNaW) return fail(c, HB_EINVAL, "k (dim + 1) + 2 exceeds the scratch row (578 values)");
    std::string why;
    double *base = scratch_of(c->device, &why);
    if (!base) return fail(c, HB_EDEVICE, "allocation-free scratch unavailable: " + why);
    double *part = base;
    double *tot = part + (size_t)kNaRows * kNaW;
    double *acc = tot + kNaW;
    double *cen = acc + kNaW;
    double *dbd = cen + (size_t)HB_KMEANS_MAX_K * HB_KMEANS_MAX_DIM;
    int32_t *lab = const_cast<int32_t *>(labels);   // modes 1 and 2 only read the labels
    // mode 1: centroid sums of the given labels; mode 2: distance sums to the centroids
    auto pass = [&](int mode) -> hipError_t {
        for (int64_t c0 = 0; c0 < n; c0 += kNaChunk) {
            const int64_t nc = std::min<int64_t>(kNaChunk, n - c0);
            hipError_t e = hb::launch_km_round(X + c0 * dim, nc, dim, k, cen, lab + c0, mode, part,
                                               tot, c->stream);
            if (e == hipSuccess) e = hb::launch_km_accum(acc, tot, w, c0 == 0 ? 1 : 0, c->stream);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    hipError_t e = hb::launch_zero_d(cen, k * dim, c->stream);
    if (e == hipSuccess) e = pass(1);
    if (e == hipSuccess) e = hb::launch_km_means(acc, dim, k, 0, cen, c->stream);   // centroids
    if (e == hipSuccess) e = pass(2);
    if (e == hipSuccess) e = hb::launch_km_db(acc, cen, dim, k, dbd, c->stream);
    double bad = 0.0, val = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, acc + (w - 1), sizeof bad, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&val, dbd, sizeof val, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail_dev(c, e, "Davies-Bouldin index (allocation-free)");
    if (bad != 0.0) return fail(c, HB_EINVAL, "labels outside [0, k)");
    *db = val;
    return HB_OK;
}

// SplitMix64 (Steele, Lea and Flood 2014) as a counter-based stream: value t of stream
// (seed, B, r) is the output function applied to seed + gamma (1 + t + 4096 (r + 1024 B)).
static uint64_t km_draw(uint64_t seed, int32_t B, int32_t r, int64_t t) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(1 + t + 4096 * ((int64_t)r + 1024 * (int64_t)B));
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

HB_API hb_status hb_choose_groups(hb_ctx *c, const float *X, int64_t n, int32_t dim, int32_t kmin,
                                  int32_t kmax, int32_t restarts, uint64_t seed, int32_t max_iters,
                                  int32_t *labels, int32_t *n_groups, double *db, uint32_t flags) {
    ENTER(c);
    CHKST(finish_pending(c));
    CHKST(km_check(c, X, n, dim, kmax, flags));
    if (kmin < 1 || kmin > kmax) return fail(c, HB_EINVAL, "need 1 <= kmin <= kmax");
    if (restarts < 1 || max_iters < 1) return fail(c, HB_EINVAL, "restarts and max_iters must be >= 1");
    if (!labels || !n_groups || !db) return fail(c, HB_EINVAL, "labels, n_groups or db is NULL");
    KmBufs b;
    const float *dX = nullptr;
    CHKST(km_setup(c, b, X, n, dim, kmax, flags, &dX));
    CHKST(dalloc(c, &b.lab, (size_t)n, "k-means labels"));
    CHKST(dalloc(c, &b.best, (size_t)n, "k-means best labels"));
    int32_t *dchosen = labels;
    if (!(flags & HB_DEVICE_PTRS)) {
        CHKST(dalloc(c, &b.chosen, (size_t)n, "chosen labels"));
        dchosen = b.chosen;
    }
    std::vector<int64_t> idx((size_t)kmax);
    int32_t chosen = kmin;
    double chosen_db = 0.0;
    for (int32_t k = kmin; k <= kmax; ++k) {
        double best_in = 0.0;
        for (int32_t r = 0; r < restarts; ++r) {
            int32_t got = 0;
            for (int64_t t = 0; got < k; ++t) {
                const int64_t v = (int64_t)(km_draw(seed, k, r, t) % (uint64_t)n);
                bool dup = false;
                for (int32_t q = 0; q < got; ++q) dup = dup || idx[(size_t)q] == v;
                if (!dup) idx[(size_t)got++] = v;
            }
            HIPCHK(c, hipMemcpyAsync(b.idx, idx.data(), sizeof(int64_t) * (size_t)k, hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hb::launch_km_gather(dX, dim, k, b.idx, b.cen, c->stream));
            double in = 0.0;
            CHKST(km_run(c, b, dX, n, dim, k, max_iters, b.lab, &in, nullptr));
            if (r == 0 || in < best_in) {
                best_in = in;
                HIPCHK(c, hipMemcpyAsync(b.best, b.lab, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, c->stream));
            }
        }
        double d = 0.0;
        CHKST(km_db(c, b, dX, n, dim, k, b.best, &d));
        db[k - kmin] = d;
        if (k == kmin || d < chosen_db) {
            chosen_db = d;
            chosen = k;
            HIPCHK(c, hipMemcpyAsync(dchosen, b.best, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, c->stream));
        }
    }
    if (b.chosen)
        HIPCHK(c, hipMemcpyAsync(labels, b.chosen, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *n_groups = chosen;
    return HB_OK;
}

HB_API hb_status hb_orientation_groups(hb_ctx *c, int32_t *group, uint32_t flags) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (flags & ~(uint32_t)HB_DEVICE_PTRS) return fail(c, HB_EINVAL, "unknown flags");
    if (!c->have_graph) return fail(c, HB_ESTATE, "hb_orientation_groups needs hb_set_graph");
    if (c->E == 0) return HB_OK;
    if (!group) return fail(c, HB_EINVAL, "group is NULL");
    CHKST(ensure_desc(c, 1));
    CHKST(wait_desc(c));
    GDesc d = base_desc(c);
    d.pin = c->pts[c->ps];       // the end points never move: any iteration's polylines
    d.off_in = c->off[c->os];
    c->h_desc[0] = d;
    CHKST(upload_desc(c, 1));
    int32_t *out = group, *tmp = nullptr;
    if (!(flags & HB_DEVICE_PTRS)) {
        CHKST(dalloc(c, &tmp, (size_t)c->E, "orientation bins"));
        out = tmp;
    }
    const Shape s = hb::shape_of(c->E, d.B, d.W, d.H, c->tiling);
    hipError_t e = hb::launch_orientation(c->d_desc, s, out, c->stream);
    if (e == hipSuccess && tmp)
        e = hipMemcpyAsync(group, tmp, sizeof(int32_t) * (size_t)c->E, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dfree(&tmp);
    if (e != hipSuccess) return fail_dev(c, e, "orientation bins");
    return HB_OK;
}

HB_API hb_status hb_point_widths(hb_ctx *c, int32_t iter, float w_min, float w_max, int32_t log_scale,
                                 float *dens, float *widths, int64_t cap_points, uint32_t flags) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (flags & ~(uint32_t)HB_DEVICE_PTRS) return fail(c, HB_EINVAL, "unknown flags");
    if (!c->have_params || !c->have_graph || !c->have_groups)
        return fail(c, HB_ESTATE, "hb_point_widths needs parameters, graph and groups");
    if (iter < 0) return fail(c, HB_EINVAL, "iter must be >= 0");
    if (!std::isfinite(w_min) || !std::isfinite(w_max) || w_min < 0.0f || w_max < w_min)
        return fail(c, HB_EINVAL, "widths need finite 0 <= w_min <= w_max");
    if (log_scale != 0 && log_scale != 1) return fail(c, HB_EINVAL, "log_scale must be 0 or 1");
    const int64_t N = c->n_state;
    if (cap_points < N) return fail(c, HB_EINVAL, "output buffers too small");
    if (N > 0 && !widths) return fail(c, HB_EINVAL, "widths is NULL");
    CHKST(prepare_ctx(c, 1, 0));
    if (c->render_cap < 2 * N + 1) {
        dfree(&c->d_render);
        c->render_cap = 0;
        CHKST(dalloc(c, &c->d_render, (size_t)(2 * N + 1), "point widths"));
        c->render_cap = 2 * N + 1;
    }
    CHKST(ensure_desc(c, 1));
    CHKST(wait_desc(c));
    GDesc d = base_desc(c);
    set_iter_scalars(c, d, iter);
    d.samples = c->pts[c->ps];
    d.off_s = c->off[c->os];
    d.count_given = !d.strip;
    c->h_desc[0] = d;
    CHKST(upload_desc(c, 1));
    const GDesc *dd = c->d_desc;
    const Shape s = hb::shape_of(c->E, d.B, d.W, d.H, c->tiling);
    const bool strip = d.strip != 0;
    float *pd = c->d_render, *pw = c->d_render + N;
    uint32_t *pmax = reinterpret_cast<uint32_t *>(c->d_render + 2 * N);
    if (flags & HB_DEVICE_PTRS) {
        if (dens) pd = dens;
        pw = widths;
    }
    HIPCHK(c, hb::launch_clear_hist(dd, 1, s, c->stream));
    if (!strip) HIPCHK(c, hb::launch_count_given(dd, 1, s, c->stream));
    else HIPCHK(c, hb::launch_strip_bins(dd, 1, s, false, c->stream));
    HIPCHK(c, hb::launch_bin_hist(dd, 1, s, strip, !strip, c->stream));
    for (int k = 0; k < d.P; ++k) HIPCHK(c, hb::launch_box_pass(dd, 1, s, d.W, k, c->stream));
    HIPCHK(c, hb::launch_density_strips(dd, 1, s, d.B, c->stream));
    HIPCHK(c, hipMemsetAsync(pmax, 0, sizeof(uint32_t), c->stream));
    HIPCHK(c, hb::launch_point_density(dd, s, pd, pmax, c->stream));
    HIPCHK(c, hb::launch_widths(pd, N, pmax, (double)w_min, (double)w_max, log_scale, pw, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    CHKST(read_status(c));
    c->have_maps = true;
    if (!(flags & HB_DEVICE_PTRS)) {
        if (dens) CHKST(copy_out(c, dens, pd, sizeof(float) * (size_t)N, 0));
        CHKST(copy_out(c, widths, pw, sizeof(float) * (size_t)N, 0));
    }
    return HB_OK;
}

HB_API hb_status hb_get_iteration(hb_ctx *c, int32_t *iter) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (!iter) return fail(c, HB_EINVAL, "iter is NULL");
    *iter = c->iter;
    return HB_OK;
}

HB_API hb_status hb_set_iteration(hb_ctx *c, int32_t iter) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (iter < 0) return fail(c, HB_EINVAL, "iteration must be >= 0");
    c->iter = iter;
    c->ckpt_end_iter = -1;
    return HB_OK;
}

HB_API hb_status hb_set_profiling(hb_ctx *c, int32_t enable) {
    ENTER(c);
    CHKST(finish_pending(c));
    c->profiling = enable != 0;
    return HB_OK;
}

HB_API hb_status hb_get_stage_times(hb_ctx *c, double *ms, int64_t *launches, int32_t n_stages,
                                    int32_t reset) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (n_stages < 0 || n_stages > HB_NUM_STAGES) return fail(c, HB_EINVAL, "n_stages out of range");
    if ((n_stages > 0 && (!ms || !launches))) return fail(c, HB_EINVAL, "ms and launches are required");
    for (int i = 0; i < n_stages; ++i) {
        ms[i] = c->stage_ms[i];
        launches[i] = c->stage_n[i];
    }
    if (reset)
        for (int i = 0; i < HB_NUM_STAGES; ++i) {
            c->stage_ms[i] = 0.0;
            c->stage_n[i] = 0;
        }
    return HB_OK;
}

// ------------------------------------------------------------------ adjoint

static void free_ckpts(hb_ctx *c) {
    for (auto &k : c->ckpt_pool) c->ckpts.push_back(k);
    c->ckpt_pool.clear();
    for (auto &k : c->ckpts) {
        dfree(&k.pts);
        dfree(&k.xs);
        dfree(&k.off);
        dfree(&k.xoff);
        dfree(&k.counts);
        dfree(&k.lens);
        dfree(&k.jacc);
        dfree(&k.hist);
        dfree(&k.bsrc);
        dfree(&k.toff);
        dfree(&k.soff);
    }
    c->ckpts.clear();
    c->ckpt_end_iter = -1;
    dfree(&c->adj.a0);
    dfree(&c->adj.a1);
    for (int i = 0; i < 2; ++i) {
        dfree(&c->adj.gb[i]);
        dfree(&c->adj.mv[i]);
    }
    dfree(&c->adj.partials);
    dfree(&c->adj.gparam);
    dfree(&c->adj.red);
    dfree(&c->adj.mvmax);
    c->adj = hb_ctx::AdjBufs();
}

template <typename T>
static hb_status grow(hb_ctx *c, T **p, int64_t &cap, int64_t need, const char *what) {
    if (need <= cap && *p) return HB_OK;
    CHKST(dalloc(c, p, (size_t)std::max<int64_t>(1, need), what));
    cap = need;
    return HB_OK;
}

// One descriptor of a checkpointed iteration, on explicit buffers.
static GDesc ckpt_desc(hb_ctx *c, const float2 *pin, const int64_t *off_in, float2 *xs, int64_t *xoff,
                       int64_t cap) {
    GDesc d = base_desc(c);
    set_iter_scalars(c, d, c->iter);
    d.pin = pin;
    d.off_in = off_in;
    d.samples = xs;
    d.off_s = xoff;
    d.cap = cap;
    d.total = c->d_totals;
    return d;
}

// The iterations write straight into the checkpoints: iteration t reads the polylines of
// checkpoint t, writes its samples, decisions and splat bins into checkpoint t and its new
// polylines into checkpoint t + 1 (the last one into the context's state buffer). Each
// iteration first scans the sample counts alone, so every buffer is sized exactly.
HB_API hb_status hb_forward_ckpt(hb_ctx *c, int32_t n_iters, uint32_t flags, int64_t *generation) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (!c->have_params || !c->have_graph || !c->have_groups)
        return fail(c, HB_ESTATE, "hb_forward_ckpt needs parameters, graph and groups");
    if (n_iters < 1) return fail(c, HB_EINVAL, "n_iters must be >= 1");
    if (flags != 0) return fail(c, HB_EINVAL, "hb_forward_ckpt takes no flags");
    if (c->B > 16) return fail(c, HB_EINVAL, "the adjoint supports at most 16 groups");
    if (c->P.directed_offset_px != 0.0f)
        return fail(c, HB_EINVAL, "the adjoint does not differentiate directed_offset_px (set it to 0)");
    if (c->P.splat_mode != HB_SPLAT_POINTS)
        return fail(c, HB_EINVAL, "the adjoint needs the point splat (splat_mode HB_SPLAT_POINTS)");
    if (c->P.resample_mode != HB_RESAMPLE_UNIFORM)
        return fail(c, HB_EINVAL, "the adjoint needs the uniform resampling (resample_mode HB_RESAMPLE_UNIFORM)");
    if (!c->sigmas.empty())
        return fail(c, HB_EINVAL, "the adjoint needs one box radius per iteration (n_sigmas = 0)");
    // earlier checkpoint buffers go back to the pool and are reused when large enough
    for (auto &k : c->ckpts) c->ckpt_pool.push_back(k);
    c->ckpts.clear();
    c->ckpt_end_iter = -1;
    c->ckpt_gen += 1;
    CHKST(prepare_ctx(c, 1, 0));
    CHKST(ensure_desc(c, 1));
    CHKST(wait_desc(c));
    const int T = n_iters;
    const int64_t E = c->E;
    const int64_t plane = (int64_t)c->B * c->P.grid_w * c->P.grid_h;
    const size_t E1 = (size_t)E + 1;
    const int64_t nt1 = (int64_t)hb::tiles_of(std::max(1, c->B), c->P.grid_w, c->P.grid_h, c->tiling.sets_max).n + 1;
    const Shape sh = hb::shape_of(E, std::max(1, c->B), c->P.grid_w, c->P.grid_h, c->tiling);
    auto take = [&]() {
        hb_ctx::Ckpt k;
        if (!c->ckpt_pool.empty()) {
            k = c->ckpt_pool.front();        // slot t reuses the buffers of the last slot t
            c->ckpt_pool.erase(c->ckpt_pool.begin());
        }
        return k;
    };
    auto fail_free = [&](hb_status st) {
        free_ckpts(c);
        return st;
    };
    // checkpoint 0: the polylines that enter the run
    {
        hb_ctx::Ckpt k = take();
        k.n = c->n_state;
        hb_status st = grow(c, &k.pts, k.cap_n, std::max<int64_t>(1, k.n), "checkpoint");
        c->ckpts.push_back(k);
        if (st != HB_OK) return fail_free(st);
        HIPCHK(c, hipMemcpyAsync(k.pts, c->pts[c->ps], sizeof(float2) * k.n, hipMemcpyDeviceToDevice, c->stream));
    }
    std::vector<int64_t> counts;
    for (int t = 0; t < T; ++t) {
        hb_ctx::Ckpt &k = c->ckpts[t];
        k.iter = c->iter;
        int64_t cap_e = k.cap_e, cap_e2 = k.cap_e, cap_e3 = k.cap_e, cap_e4 = k.cap_e;
        hb_status st = grow(c, &k.off, cap_e, E + 1, "checkpoint");
        if (st == HB_OK) st = grow(c, &k.xoff, cap_e2, E + 1, "checkpoint");
        if (st == HB_OK) st = grow(c, &k.counts, cap_e3, E + 1, "checkpoint");
        if (st == HB_OK) st = grow(c, &k.lens, cap_e4, E + 1, "checkpoint");
        k.cap_e = std::min(std::min(cap_e, cap_e2), std::min(cap_e3, cap_e4));
        if (st == HB_OK) st = grow(c, &k.hist, k.cap_px, plane, "checkpoint");
        if (st != HB_OK) return fail_free(st);
        // offsets, sample counts and lengths of the polylines entering iteration t
        const int64_t *off_in = t == 0 ? c->off[c->os] : c->ckpts[t - 1].xoff;
        HIPCHK(c, hipMemcpyAsync(k.off, off_in, sizeof(int64_t) * E1, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(k.counts, c->d_counts, sizeof(int64_t) * E, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(k.lens, c->d_lens, sizeof(double) * E, hipMemcpyDeviceToDevice, c->stream));
        // the sample offsets, and the sample count that sizes this iteration's buffers
        GDesc d = ckpt_desc(c, k.pts, k.off, nullptr, k.xoff, INT64_MAX);
        CHKST(wait_desc(c));   // the staging copy of the last upload has been consumed
        c->h_desc[0] = d;
        CHKST(upload_desc(c, 1));
        HIPCHK(c, hb::launch_scan(c->d_desc, 1, sh, c->stream));
        // one synchronisation per iteration: the sample count, and the status of the previous
        // iteration's kernels and of this scan
        int64_t ns = 0;
        CHKST(read_scalar(c, c->d_totals, &ns));
        CHKST(read_status(c));
        k.ns = ns;
        if (ns >= (int64_t(1) << 32))   // the tile bins record their samples as 32-bit indices
            return fail_free(fail(c, HB_EOVERFLOW, "the checkpointed forward takes fewer than 2^32 samples per iteration"));
        int64_t cap_ns2 = k.cap_ns, cap_t2 = k.cap_t;
        st = grow(c, &k.xs, k.cap_ns, std::max<int64_t>(1, ns), "checkpoint");
        if (st == HB_OK) st = grow(c, &k.jacc, cap_ns2, std::max<int64_t>(1, ns), "checkpoint");
        if (st == HB_OK) st = grow(c, &k.bsrc, k.cap_bs, std::max<int64_t>(1, ns), "checkpoint");
        if (st == HB_OK) st = grow(c, &k.toff, k.cap_t, nt1, "checkpoint");
        if (st == HB_OK) st = grow(c, &k.soff, cap_t2, nt1, "checkpoint");
        k.cap_ns = std::min(k.cap_ns, cap_ns2);
        k.cap_t = std::min(k.cap_t, cap_t2);
        if (st == HB_OK) st = ensure_capacity(c, ns + 64);   // splat bins and the final state
        if (st != HB_OK) return fail_free(st);
        float2 *pnew = c->pts[c->ps];
        if (t + 1 < T) {
            hb_ctx::Ckpt kn = take();
            kn.n = ns;
            st = grow(c, &kn.pts, kn.cap_n, std::max<int64_t>(1, ns), "checkpoint");
            c->ckpts.push_back(kn);
            if (st != HB_OK) return fail_free(st);
            pnew = kn.pts;
        }
        hb_ctx::Ckpt &kk = c->ckpts[t];
        // the iteration, on the checkpoint buffers
        d = ckpt_desc(c, kk.pts, kk.off, kk.xs, kk.xoff, ns);
        d.pnew = pnew;
        d.jacc = kk.jacc;
        d.bin_src = kk.bsrc;
        d.record = 1;
        CHKST(wait_desc(c));
        c->h_desc[0] = d;
        CHKST(upload_desc(c, 1));
        const GDesc *dd = c->d_desc;
        HIPCHK(c, hb::launch_clear_hist(dd, 1, sh, c->stream));
        // the checkpointed forward takes no directed offset
        HIPCHK(c, hb::launch_resample_count(dd, 1, sh, c->tune_ru, false, c->stream));
        HIPCHK(c, hb::launch_bin_hist(dd, 1, sh, false, true, c->stream));
        for (int kp = 0; kp < c->P.box_passes; ++kp)
            HIPCHK(c, hb::launch_box_pass(dd, 1, sh, c->P.grid_w, kp, c->stream));
        HIPCHK(c, hb::launch_density_strips(dd, 1, sh, std::max(1, c->B), c->stream));
        HIPCHK(c, hb::launch_advect_smooth(dd, 1, sh, c->tune_au, c->stream));
        HIPCHK(c, hipMemcpyAsync(kk.hist, c->d_hist, sizeof(int32_t) * plane, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(kk.toff, c->d_tile_off, sizeof(int64_t) * nt1, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(kk.soff, c->d_seg_off, sizeof(int64_t) * nt1, hipMemcpyDeviceToDevice, c->stream));
        counts.push_back(ns);
        c->iter += 1;
    }
    // the state after the run: polylines in pts[ps] with the last sample offsets
    const hb_ctx::Ckpt &kl = c->ckpts[T - 1];
    HIPCHK(c, hipMemcpyAsync(c->off[c->os], kl.xoff, sizeof(int64_t) * E1, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    CHKST(read_status(c));
    c->n_state = kl.ns;
    c->have_samples = false;   // the samples stay in the checkpoints
    c->have_jacc = false;
    c->have_maps = true;
    c->last_counts = counts;
    c->ckpt_end_iter = c->iter;
    if (generation) *generation = c->ckpt_gen;
    return HB_OK;
}

// Gradient of the loss L = total length of the polylines after the checkpointed run, with
// respect to M (B x B), the pass weights a (P) and the polylines that entered the run. The
// maps of each iteration are rebuilt from its checkpointed histogram; the samples and the
// accepted halvings come from the checkpoints, so nothing else is recomputed.
HB_API hb_status hb_backward(hb_ctx *c, int64_t generation, const float *dL_dxy_T,
                             int64_t n_points_T, double *loss, float *dL_dM, float *dL_da,
                             float *dL_dxy0, int64_t cap_points, uint32_t flags) {
    ENTER(c);
    CHKST(finish_pending(c));
    if (c->ckpts.empty() || c->iter != c->ckpt_end_iter)
        return fail(c, HB_ESTATE, "hb_backward needs hb_forward_ckpt just before it");
    if (generation >= 0 && generation != c->ckpt_gen)
        return fail(c, HB_ESTATE, "the checkpoints of that generation have been replaced");
    if (generation < -1) return fail(c, HB_EINVAL, "generation must be -1 or a generation");
    if (flags & ~(uint32_t)HB_DEVICE_PTRS) return fail(c, HB_EINVAL, "unknown flags");
    const int T = (int)c->ckpts.size();
    const int B = c->B, P = c->P.box_passes, W = c->P.grid_w, H = c->P.grid_h;
    const int64_t E = c->E, n0 = c->ckpts[0].n;
    if (dL_dxy0 && cap_points < n0) return fail(c, HB_EINVAL, "dL_dxy0 buffer too small");
    if (dL_dxy_T && n_points_T != c->n_state)
        return fail(c, HB_EINVAL, "n_points_T must equal the point count of the final polylines");
    int64_t nmax = c->n_state;
    for (auto &k : c->ckpts) nmax = std::max(nmax, std::max(k.n, k.ns));
    CHKST(ensure_maps(c));
    CHKST(ensure_desc(c, (size_t)(2 * T)));
    CHKST(wait_desc(c));
    const int64_t plane = (int64_t)W * H;
    hb_ctx::AdjBufs &A = c->adj;
    CHKST(grow(c, &A.a0, A.cap_pts, nmax, "adjoint"));
    CHKST(grow(c, &A.a1, A.cap_a1, nmax, "adjoint"));
    const int bp = (B + 1) / 2 * 2, pp = (P + 1) / 2 * 2;
    for (int i = 0; i < 2 && i < T; ++i)
        CHKST(grow(c, &A.gb[i], A.cap_gb[i], plane * (bp + (int64_t)B * pp), "gradient maps"));
    // work items of the tile bins: at most one per item_entries samples plus one per tile
    const int64_t nt = hb::tiles_of(B, W, H, c->tiling.sets_max).n;
    int64_t max_items = 1;
    for (auto &k : c->ckpts) max_items = std::max(max_items, k.ns / c->tiling.item_entries + nt + 1);
    CHKST(grow(c, &A.partials, A.cap_part, max_items * (B + P), "partials"));
    for (int i = 0; i < 2 && i < T; ++i)
        CHKST(grow(c, &A.mv[i], A.cap_mv[i], std::max<int64_t>(1, nmax), "adjoint steps"));
    CHKST(grow(c, &A.mvmax, A.cap_mm, (int64_t)T, "adjoint step scale"));
    CHKST(grow(c, &A.gparam, A.cap_gp, (int64_t)(B * B + P), "parameter gradients"));
    CHKST(grow(c, &A.red, A.cap_red, (int64_t)(B * B + P) * hb::kRedSlices, "reduction"));
    CHKST(ensure_order(c));
    HIPCHK(c, hipMemsetAsync(A.gparam, 0, sizeof(double) * (B * B + P), c->stream));

    // loss: total length of the final polylines (the lengths the last advection wrote)
    if (!c->d_ink) CHKST(dalloc(c, &c->d_ink, (size_t)hb::kInkSlices + 1, "ink"));
    HIPCHK(c, hb::launch_ink(c->d_lens, E, c->d_ink, c->stream));
    double ink = 0.0;
    HIPCHK(c, hipMemcpyAsync(&ink, c->d_ink + hb::kInkSlices, sizeof(double), hipMemcpyDeviceToHost, c->stream));

    const Shape s = hb::shape_of(E, B, W, H, c->tiling);
    float2 *cur = A.a0, *other = A.a1;   // cur: adjoint of the polylines leaving iteration t
    if (dL_dxy_T && c->n_state > 0)      // the caller's loss gradient enters the last iteration
        HIPCHK(c, hipMemcpyAsync(cur, dL_dxy_T, sizeof(float2) * c->n_state,
                                 (flags & HB_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                 c->stream));
    for (int t = T - 1; t >= 0; --t) {
        const hb_ctx::Ckpt &k = c->ckpts[t];
        const size_t slot = 2 * (size_t)(T - 1 - t);
        GDesc a = base_desc(c);                 // maps, smoothing and advection adjoint
        set_iter_scalars(c, a, k.iter);
        a.histx = k.hist;                       // one histogram copy: the checkpoint
        a.nx = 1;
        a.samples = k.xs;
        a.off_s = k.xoff;
        a.jacc = k.jacc;
        a.gbm = A.gb[t & 1];
        a.gkm = A.gb[t & 1] + plane * bp;
        a.bp = bp;
        a.pp = pp;
        a.adj_in = cur;
        a.adj_out = other;
        // the ink gradient is computed in place from the final polylines, unless given
        if (t == T - 1 && !dL_dxy_T) a.ink_pts = c->pts[c->ps];
        a.partials = A.partials;
        a.max_items = max_items;
        a.abin_src = k.bsrc;
        a.atile_off = k.toff;
        a.aseg_off = k.soff;
        a.mv = A.mv[t & 1];
        a.mvmax = A.mvmax + t;
        a.red = A.red;
        a.grad_param = A.gparam;
        GDesc q = a;                            // resampling adjoint
        q.pin = k.pts;
        q.off_in = k.off;
        q.lens = k.lens;
        q.adj_in = other;
        q.adj_out = cur;
        c->h_desc[slot] = a;
        c->h_desc[slot + 1] = q;
    }
    CHKST(upload_desc(c, (size_t)(2 * T)));
    HIPCHK(c, hipMemsetAsync(A.mvmax, 0, sizeof(uint32_t) * T, c->stream));
    // The parameter gradients of iteration t (tile splat + reduction) run on a second stream,
    // beside the resampling adjoint of t and iteration t - 1; the gradient-map records and m v
    // are double-buffered by iteration parity, so only iteration t - 2 waits for them before
    // it overwrites their buffers.
    if (!c->side) HIPCHK(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    while (c->adj_ev.size() < (size_t)(2 * T)) {
        hipEvent_t ev;
        HIPCHK(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        c->adj_ev.push_back(ev);
    }
    hipEvent_t params_done = nullptr;
    for (int t = T - 1; t >= 0; --t) {
        const GDesc *a = c->d_desc + 2 * (size_t)(T - 1 - t);
        hipEvent_t adv_done = c->adj_ev[2 * (size_t)t], par_done = c->adj_ev[2 * (size_t)t + 1];
        for (int kk = 0; kk < P; ++kk) HIPCHK(c, hb::launch_box_pass(a, 1, s, W, kk, c->stream));
        HIPCHK(c, hb::launch_density_strips(a, 1, s, B, c->stream));
        if (t + 2 < T) HIPCHK(c, hipStreamWaitEvent(c->stream, c->adj_ev[2 * (size_t)(t + 2) + 1], 0));
        HIPCHK(c, hb::launch_adj_maps(a, s, B, c->stream));
        HIPCHK(c, hb::launch_adj_advect(a, s, c->stream));
        HIPCHK(c, hipEventRecord(adv_done, c->stream));
        HIPCHK(c, hipStreamWaitEvent(c->side, adv_done, 0));
        HIPCHK(c, hb::launch_adj_params(a, s, B, c->side));
        HIPCHK(c, hb::launch_adj_reduce(a, B, P, c->side));
        HIPCHK(c, hipEventRecord(par_done, c->side));
        params_done = par_done;
        HIPCHK(c, hb::launch_adj_resample(a + 1, s, c->stream));
    }
    if (params_done) HIPCHK(c, hipStreamWaitEvent(c->stream, params_done, 0));
    std::vector<double> gp((size_t)(B * B + P));
    HIPCHK(c, hipMemcpyAsync(gp.data(), A.gparam, sizeof(double) * gp.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int32_t status = 0;
    HIPCHK(c, hipMemcpy(&status, c->d_status, sizeof status, hipMemcpyDeviceToHost));
    if (status != 0) {
        int32_t zero = 0;
        HIPCHK(c, hipMemcpy(c->d_status, &zero, sizeof zero, hipMemcpyHostToDevice));
        return fail(c, HB_EOVERFLOW, "rebuilt maps exceeded a range check");
    }
    c->have_maps = false;   // the maps buffers now hold the rebuilt maps of the first iteration
    if (loss) *loss = ink;
    if (dL_dM)
        for (int i = 0; i < B * B; ++i) dL_dM[i] = (float)gp[i];
    if (dL_da)
        for (int k = 0; k < P; ++k) dL_da[k] = (float)gp[B * B + k];
    if (dL_dxy0) {
        // cur holds the adjoint of the polylines that entered the run
        HIPCHK(c, hipMemcpyAsync(dL_dxy0, cur, sizeof(float2) * n0,
                                 (flags & HB_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return HB_OK;
}

HB_API hb_status hb_get_ckpt_decisions(hb_ctx *c, int32_t t, int64_t *offsets, int8_t *jacc,
                                       int64_t cap_points, uint32_t flags) {
    ENTER(c);
    if (t < 0 || t >= (int32_t)c->ckpts.size()) return fail(c, HB_EINVAL, "no such checkpoint");
    const hb_ctx::Ckpt &k = c->ckpts[t];
    if (!offsets || cap_points < k.ns || (k.ns > 0 && !jacc)) return fail(c, HB_EINVAL, "buffer too small");
    CHKST(copy_out(c, offsets, k.xoff, sizeof(int64_t) * (size_t)(c->E + 1), flags));
    CHKST(copy_out(c, jacc, k.jacc, sizeof(int8_t) * (size_t)k.ns, flags));
    return HB_OK;
}

HB_API hb_status hb_get_ckpt_points(hb_ctx *c, int32_t t, int64_t *offsets, float *xy,
                                    int64_t cap_points, uint32_t flags) {
    ENTER(c);
    if (t < 0 || t >= (int32_t)c->ckpts.size()) return fail(c, HB_EINVAL, "no such checkpoint");
    const hb_ctx::Ckpt &k = c->ckpts[t];
    if (!offsets || cap_points < k.n || (k.n > 0 && !xy)) return fail(c, HB_EINVAL, "buffer too small");
    CHKST(copy_out(c, offsets, k.off, sizeof(int64_t) * (size_t)(c->E + 1), flags));
    CHKST(copy_out(c, xy, k.pts, sizeof(float2) * (size_t)k.n, flags));
    return HB_OK;
}
