// Host side of the C ABI: argument validation, workspace layout, the launch
// sequence of a frame, HIP-graph batch plans, the tile-shape autotuner and
// per-stage event timing.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace rgs {
// backward.hip: zeroes the record gradients of the kept Gaussian-views
// order[0, *kept) (grad_floats_per floats each, a multiple of 4).
hipError_t launch_zero_kept_grads(const uint32_t *order, const int64_t *kept, int64_t n_max, int grad_floats_per,
                                  float *grads, int num_cus, hipStream_t stream);
// calib.hip: FP32 FMA TFLOP/s, exp2 Top/s and device copy GB/s (read + write)
// measured on `stream` (allocates and frees its own buffers, synchronises).
hipError_t measure_ceilings(int num_cus, hipStream_t stream, double *fma_tflops, double *exp_tops, double *copy_gbs);
}  // namespace rgs

using namespace rgs;

namespace {

constexpr int kNumStages = 9;
const char *const kStageNames =
    "preprocess;depth_sort;scan;emit;tile_sort;tile_ranges;blend;blend_backward;preprocess_backward";
enum Stage { ST_PRE, ST_DSORT, ST_SCAN, ST_EMIT, ST_TSORT, ST_RANGES, ST_BLEND, ST_BLEND_BWD, ST_PRE_BWD };

constexpr size_t kAlign = 256;
// Quads with a vertex at z <= 0 clipped per launch; more keep the whole view.
constexpr int64_t kCrossingCap = 1 << 16;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t counters, views, records, keys_a, keys_b, order_a, order_b, boxes, bin_boxes, sorted_boxes, conics,
        tile_counts,
        offsets, block_sums;
    size_t crossing;          // quads with a vertex at z <= 0, awaiting frustum clipping
    uint32_t crossing_cap;    // entries of the crossing list
    size_t inst_tiles_a, inst_tiles_b, inst_ids_a, inst_ids_b, hist, row_total, ranges, sched, tile_order;
    size_t row_offsets, row_owner, item_clock;
    size_t record_grads, total;
    int64_t nv_records, capacity, total_tiles;
    int tile_w, tile_h, tile_bits;
};

struct FrameEvents {
    hipEvent_t ev[kNumStages + 1];
    int first, last;  // stages [first, last) were recorded
};

// Layout-determining parameters of a rendered frame.
struct FrameShape {
    TileShape tile;
    int32_t mip, divergence, n_views;
    int64_t n, capacity;
    int32_t flags;
};

}  // namespace

namespace {

// Device scratch of rgs_render_noalloc: the whole frame workspace of that
// entry point lives here instead of in caller memory.  Each device the
// library runs on holds its own copy until the process ends.  In host code
// `scratch` only names the symbol; its device address on each device is
// looked up once (rgs_create, with that device current) and kept in
// g_scratch, and only that address is ever handed to kernels or copies.
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch[kMaxDevices] = {};
hipError_t g_scratch_error[kMaxDevices] = {};

// Looks up the scratch address of `device` (once per device).  Returns the
// runtime's error when the lookup failed.
hipError_t scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch[device] || g_scratch_error[device] != hipSuccess) return g_scratch_error[device];
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess) e = hipSetDevice(device);
    void *p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    (void)hipSetDevice(prev);
    if (e == hipSuccess && !p) e = hipErrorInvalidSymbol;
    if (e == hipSuccess)
        g_scratch[device] = p;
    else
        g_scratch_error[device] = e;
    return e;
}

}  // namespace

struct rgs_context {
    int device = 0;
    int num_cus = 256;
    std::string err;
    bool timing = false;
    std::vector<FrameEvents> pending;
    std::vector<FrameEvents> pool;
    double stage_ms[kNumStages] = {0};
    int64_t frames = 0;
    int grid_fwd[64] = {0}, grid_fwd_exact[64] = {0}, grid_bwd[64] = {0}, grid_bwd_exact[64] = {0};
    unsigned long long *view_stamps = nullptr;  // rgs_set_view_clocks (caller-owned device memory)
    int view_stamps_views = 0;
    std::map<std::string, TileShape> tune_cache;  // autotuned tile shapes by configuration class
    // What the last frame rendered into each workspace (keyed by its device
    // address) was laid out for: the backward pass reads that frame's buffers.
    std::map<const void *, FrameShape> ws_frames;
    // Host image of a frame header for rgs_render_noalloc, sized for the
    // largest batch when the context is made, so that call allocates nothing.
    std::vector<unsigned char> noalloc_header;
};

struct rgs_plan {
    rgs_context *ctx = nullptr;
    int64_t n = 0;
    int32_t sh_degree = 0;
    std::vector<rgs_camera> cams;
    rgs_options opts{};
    int64_t capacity = 0;
    int32_t flags = 0;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool captured = false;
    rgs_gaussians g{};
    void *ws_ptr = nullptr;
    hipStream_t last_stream = nullptr;  // stream of the last launch
    bool launched = false;
    std::vector<rgs_view_out> outs;
};

namespace {

// A small host block (the workspace header: counters and view table) goes to
// the device as the argument of a one-block kernel rather than through a
// host-to-device copy, whose staging and copy kernel take longer per frame.
// Larger blocks, and sizes that are not whole words, are copied.
constexpr size_t kArgBlockBytes = 3072;
struct ArgBlock {
    uint32_t w[kArgBlockBytes / 4];
};

__global__ __launch_bounds__(256) void k_put_words(uint32_t *__restrict__ dst, ArgBlock b, int n_words)
{
    for (int i = threadIdx.x; i < n_words; i += 256) dst[i] = b.w[i];
}

hipError_t put_bytes(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    if (bytes > kArgBlockBytes || bytes % 4 != 0 || reinterpret_cast<uintptr_t>(dst) % 4 != 0)
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    ArgBlock b;
    std::memcpy(b.w, src, bytes);
    k_put_words<<<1, 256, 0, s>>>(static_cast<uint32_t *>(dst), b, (int)(bytes / 4));
    return hipGetLastError();
}

rgs_status fail(rgs_context *ctx, rgs_status st, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
rgs_status fail(rgs_context *ctx, rgs_status st, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

#define RGS_HIP(ctx, call)                                                                                  \
    do {                                                                                                    \
        hipError_t e_ = (call);                                                                             \
        if (e_ != hipSuccess) return fail((ctx), RGS_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));  \
    } while (0)

constexpr TileShape kDefaultTile{8, 16};

TileShape shape_of(const rgs_options &o)
{
    if (o.tile_w == 0 && o.tile_h == 0) return kDefaultTile;
    return TileShape{o.tile_w, o.tile_h};
}

// Configuration class of the tile-shape cache: render or training step,
// MIP, the Gaussian count in octaves and each view's pixel count in
// half-octaves (sorted).
std::string tune_class(bool training, int64_t n, const rgs_camera *cams, int32_t n_views, const rgs_options &o)
{
    std::vector<int> px;
    for (int v = 0; v < n_views; ++v)
        px.push_back((int)std::lround(2.0 * std::log2(std::max(1.0, (double)cams[v].width * (double)cams[v].height))));
    std::sort(px.begin(), px.end());
    std::string k = std::string(training ? "t" : "r") + std::to_string(o.mip) + "d" + std::to_string(o.divergence) + "/" +
                    std::to_string((int)std::floor(std::log2((double)n + 1.0)));
    for (int x : px) k += "," + std::to_string(x);
    return k;
}

// Options with tile_w = tile_h = 0 resolved: the shape the autotuners last
// chose on this context for the same configuration class (a training-step
// choice first), else the default.
rgs_options resolve_tiles(const rgs_context *ctx, int64_t n, const rgs_camera *cams, int32_t n_views,
                          const rgs_options *opts)
{
    rgs_options o = *opts;
    if (o.tile_w != 0 || o.tile_h != 0) return o;
    TileShape s = kDefaultTile;
    if (ctx && cams && n_views > 0 && n >= 0) {
        for (const bool training : {true, false}) {
            const auto it = ctx->tune_cache.find(tune_class(training, n, cams, n_views, o));
            if (it != ctx->tune_cache.end()) {
                s = it->second;
                break;
            }
        }
    }
    o.tile_w = s.w;
    o.tile_h = s.h;
    return o;
}

int shape_index(TileShape s)
{
    const int w = s.w == 8 ? 0 : (s.w == 16 ? 1 : 2);
    const int h = s.h == 8 ? 0 : (s.h == 16 ? 1 : 2);
    return w * 3 + h;
}

int bits_for(int64_t count)
{
    int b = 1;
    while (b < 40 && (int64_t(1) << b) < count) ++b;
    return b;
}

rgs_status check_cameras(rgs_context *ctx, const rgs_camera *cams, int32_t n_views)
{
    if (!cams) return fail(ctx, RGS_EINVAL, "cams is NULL");
    if (n_views < 1 || n_views > kMaxViews) return fail(ctx, RGS_EINVAL, "n_views=%d outside [1, %d]", n_views, kMaxViews);
    for (int v = 0; v < n_views; ++v) {
        const rgs_camera &c = cams[v];
        if (c.width < 1 || c.width > 16384 || c.height < 1 || c.height > 16384)
            return fail(ctx, RGS_EINVAL, "view %d: size %dx%d outside [1, 16384]", v, c.width, c.height);
        bool finite = std::isfinite(c.fx) && std::isfinite(c.fy) && std::isfinite(c.cx) && std::isfinite(c.cy);
        for (int k = 0; k < 12; ++k) finite = finite && std::isfinite(c.world_to_cam[k]);
        if (!finite) return fail(ctx, RGS_EINVAL, "view %d: non-finite camera parameter", v);
        if (!(c.fx > 0.0) || !(c.fy > 0.0)) return fail(ctx, RGS_EINVAL, "view %d: focal lengths must be > 0", v);
    }
    return RGS_OK;
}

rgs_status check_options(rgs_context *ctx, const rgs_options *o)
{
    if (!o) return fail(ctx, RGS_EINVAL, "opts is NULL");
    if (!(o->p_min > 0.0 && o->p_min < 1.0)) return fail(ctx, RGS_EINVAL, "p_min must lie in (0, 1)");
    if (!(o->alpha_max > o->p_min && o->alpha_max < 1.0))
        return fail(ctx, RGS_EINVAL, "alpha_max must lie in (p_min, 1)");
    if (!(o->t_eps >= 0.0 && o->t_eps < 1.0)) return fail(ctx, RGS_EINVAL, "t_eps must lie in [0, 1)");
    if (!(o->near_z > 0.0) || !std::isfinite(o->near_z))
        return fail(ctx, RGS_EINVAL, "near_z must be finite and > 0");
    if (o->mip < 0 || o->mip > 3) return fail(ctx, RGS_EINVAL, "mip must be 0, 1, 2 or 3");
    if (o->divergence != RGS_DIVERGENCE_RAY && o->divergence != RGS_DIVERGENCE_GS)
        return fail(ctx, RGS_EINVAL, "divergence must be RGS_DIVERGENCE_RAY or RGS_DIVERGENCE_GS");
    if (o->divergence == RGS_DIVERGENCE_GS && o->mip != 0)
        return fail(ctx, RGS_EINVAL, "MIP applies to the ray-based divergence only");
    if (!(o->mip_sigma2_px >= 0.0) || !std::isfinite(o->mip_sigma2_px))
        return fail(ctx, RGS_EINVAL, "mip_sigma2_px must be finite and >= 0");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(o->background[k])) return fail(ctx, RGS_EINVAL, "background must be finite");
    const TileShape s = shape_of(*o);
    if (!tile_shape_supported(s.w, s.h))
        return fail(ctx, RGS_EINVAL, "tile shape %dx%d not supported (width and height in {8, 16, 32})", s.w, s.h);
    return RGS_OK;
}

rgs_status compute_layout(rgs_context *ctx, int64_t n, const rgs_camera *cams, int32_t n_views,
                          const rgs_options *opts, int64_t capacity, int32_t flags, Layout &L)
{
    rgs_status st = check_cameras(ctx, cams, n_views);
    if (st != RGS_OK) return st;
    if ((st = check_options(ctx, opts)) != RGS_OK) return st;
    if (n < 0) return fail(ctx, RGS_EINVAL, "n=%lld < 0", (long long)n);
    if (n * (int64_t)n_views > (int64_t)kIdMask)
        return fail(ctx, RGS_EINVAL, "n * n_views must be below 2^28");
    if (capacity < 1 || capacity > 0xffffffffLL) return fail(ctx, RGS_EINVAL, "capacity must lie in [1, 2^32)");
    if (flags & ~RGS_WS_BACKWARD) return fail(ctx, RGS_EINVAL, "unknown workspace flags 0x%x", flags);
    const TileShape s = shape_of(*opts);
    L.tile_w = s.w;
    L.tile_h = s.h;
    int64_t tiles = 0;
    for (int v = 0; v < n_views; ++v)
        tiles += (int64_t)((cams[v].width + s.w - 1) / s.w) * ((cams[v].height + s.h - 1) / s.h);
    if (tiles >= (int64_t(1) << 29)) return fail(ctx, RGS_EINVAL, "too many tiles (at most 2^29 - 1)");
    L.total_tiles = tiles;
    L.tile_bits = bits_for(tiles + 1);  // 2^tile_bits - 1 (the empty-instance tile) >= tiles
    L.nv_records = n * n_views;
    L.capacity = capacity;
    const size_t NV = (size_t)L.nv_records;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.counters = take(8 * sizeof(int64_t));
    L.views = take(sizeof(DevView) * n_views);
    L.records = take(NV * record_floats(opts->mip) * sizeof(float));
    L.keys_a = take(NV * 4);
    L.keys_b = take(NV * 4);
    L.order_a = take(NV * 4);
    L.order_b = take(NV * 4);
    L.boxes = take(NV * 8);
    L.bin_boxes = take(NV * 8);
    L.sorted_boxes = take(NV * 8);
    L.conics = take(NV * sizeof(Conic));
    L.tile_counts = take(NV * 4);
    L.crossing_cap = (uint32_t)std::min<int64_t>((int64_t)NV, kCrossingCap);
    L.crossing = take((size_t)L.crossing_cap * kCrossingDoubles * sizeof(double));
    L.offsets = take(NV * 4);
    L.row_offsets = take(NV * 4);
    L.block_sums = take(scan_block_entries((int64_t)NV) * 8);
    L.inst_tiles_a = take((size_t)capacity * 4);
    L.inst_tiles_b = take((size_t)capacity * 4);
    L.inst_ids_a = take((size_t)capacity * 4);
    L.inst_ids_b = take((size_t)capacity * 4);
    L.hist = take(radix_hist_entries(std::max<int64_t>((int64_t)NV, capacity)) * 4);
    L.row_total = take(256 * 4);
    L.ranges = take((size_t)tiles * 8);
    L.sched = take(sched_words() * 4);
    L.tile_order = take((size_t)tiles * 2 * 4);  // work items: up to two per tile
    L.row_owner = take((size_t)capacity * 4);
    L.item_clock = take((size_t)tiles * 2 * 8);  // per work item, for per-view completion clocks
    L.record_grads = (flags & RGS_WS_BACKWARD) ? take(NV * grad_floats(opts->mip) * sizeof(float)) : 0;
    L.total = off;
    return RGS_OK;
}

void fill_public_layout(const Layout &L, rgs_workspace_layout *o)
{
    std::memset(o, 0, sizeof *o);
    o->counters = L.counters;
    o->views = L.views;
    o->records = L.records;
    o->depth_keys = L.keys_a;
    o->boxes = L.boxes;
    o->bin_boxes = L.bin_boxes;
    o->conics = L.conics;
    o->tile_counts = L.tile_counts;
    o->order = L.order_a;
    o->offsets = L.offsets;
    o->inst_tiles = L.inst_tiles_a;
    o->inst_ids = L.inst_ids_a;
    o->tile_ranges = L.ranges;
    o->record_grads = L.record_grads;
    o->total_bytes = L.total;
    o->n_records = L.nv_records;
    o->capacity = L.capacity;
    o->total_tiles = L.total_tiles;
    o->tile_w = L.tile_w;
    o->tile_h = L.tile_h;
    o->tile_bits = L.tile_bits;
}

DevOptions dev_options(const rgs_options &o)
{
    DevOptions d{};
    d.p_min = o.p_min;
    d.alpha_max = o.alpha_max;
    d.t_eps = o.t_eps;
    d.near_z = o.near_z;
    d.mip_sigma2_px = o.mip_sigma2_px;
    d.mip = o.mip;
    d.divergence = o.divergence;
    const TileShape s = shape_of(o);
    d.tile_w = s.w;
    d.tile_h = s.h;
    d.tile_wshift = __builtin_ctz((unsigned)s.w);
    d.tile_hshift = __builtin_ctz((unsigned)s.h);
    for (int k = 0; k < 3; ++k) d.bg[k] = (float)o.background[k];
    return d;
}

// Host image of the workspace header: counters followed by the view table,
// written to buf (header_bytes(L, n_views) bytes).
size_t header_bytes(const Layout &L, int n_views) { return L.views + sizeof(DevView) * n_views; }

void write_header(unsigned char *buf, const Layout &L, const rgs_camera *cams, int n_views, const rgs_view_out *outs,
                  const float *const *dL)
{
    std::memset(buf, 0, header_bytes(L, n_views));
    int64_t *counters = reinterpret_cast<int64_t *>(buf + L.counters);
    counters[0] = 0;
    counters[1] = L.capacity;
    DevView *views = reinterpret_cast<DevView *>(buf + L.views);
    int base = 0;
    for (int v = 0; v < n_views; ++v) {
        const rgs_camera &c = cams[v];
        DevView &d = views[v];
        std::memcpy(d.w2c, c.world_to_cam, sizeof d.w2c);
        d.fx = c.fx;
        d.fy = c.fy;
        d.ifx = 1.0 / c.fx;  // correctly rounded, as the same division on the device
        d.ify = 1.0 / c.fy;
        d.cx = c.cx;
        d.cy = c.cy;
        const double *W = c.world_to_cam;
        for (int k = 0; k < 3; ++k) d.centre[k] = -(W[k] * W[3] + W[4 + k] * W[7] + W[8 + k] * W[11]);
        d.width = c.width;
        d.height = c.height;
        d.tiles_x = (c.width + L.tile_w - 1) / L.tile_w;
        d.tiles_y = (c.height + L.tile_h - 1) / L.tile_h;
        d.tile_base = base;
        base += d.tiles_x * d.tiles_y;
        d.rgb = outs ? outs[v].rgb : nullptr;
        d.final_T = outs ? outs[v].final_T : nullptr;
        d.n_contrib = outs ? outs[v].n_contrib : nullptr;
        d.dL_drgb = dL ? dL[v] : nullptr;
    }
}

std::vector<unsigned char> build_header(const Layout &L, const rgs_camera *cams, int n_views,
                                        const rgs_view_out *outs, const float *const *dL)
{
    std::vector<unsigned char> buf(header_bytes(L, n_views));
    write_header(buf.data(), L, cams, n_views, outs, dL);
    return buf;
}

template <typename T>
T *at(void *ws, size_t off)
{
    return reinterpret_cast<T *>(static_cast<unsigned char *>(ws) + off);
}

struct Timer {
    rgs_context *ctx;
    hipStream_t stream;
    FrameEvents fe{};
    bool on;
    Timer(rgs_context *c, hipStream_t s, bool enable, int first) : ctx(c), stream(s), on(enable && c->timing)
    {
        if (!on) return;
        if (!ctx->pool.empty()) {
            fe = ctx->pool.back();
            ctx->pool.pop_back();
        } else {
            for (auto &e : fe.ev) (void)hipEventCreate(&e);
        }
        fe.first = first;
        fe.last = first;
        (void)hipEventRecord(fe.ev[first], stream);
    }
    void mark(int stage_done)
    {
        if (!on) return;
        (void)hipEventRecord(fe.ev[stage_done + 1], stream);
        fe.last = stage_done + 1;
    }
    ~Timer()
    {
        if (on) ctx->pending.push_back(fe);
    }
};

void ensure_grids(rgs_context *ctx, TileShape s)
{
    const int k = shape_index(s);
    if (!ctx->grid_fwd[k]) ctx->grid_fwd[k] = blend_grid(s, false, ctx->num_cus);
    if (!ctx->grid_fwd_exact[k]) ctx->grid_fwd_exact[k] = blend_grid(s, true, ctx->num_cus);
    if (!ctx->grid_bwd[k]) ctx->grid_bwd[k] = blend_backward_grid(s, false, ctx->num_cus);
    if (!ctx->grid_bwd_exact[k]) ctx->grid_bwd_exact[k] = blend_backward_grid(s, true, ctx->num_cus);
}

// Enqueue the forward pipeline after the header copy.
rgs_status enqueue_forward(rgs_context *ctx, const rgs_gaussians &g, int n_views, const rgs_options &opts,
                           const Layout &L, void *ws, hipStream_t stream, bool timing,
                           unsigned long long *view_stamps = nullptr)
{
    const DevOptions dopt = dev_options(opts);
    const TileShape s = shape_of(opts);
    ensure_grids(ctx, s);
    const DevView *views = at<DevView>(ws, L.views);
    int64_t *counters = at<int64_t>(ws, L.counters);
    const int64_t NV = L.nv_records;
    // pass parity decides where the producers write so results land in "a"
    const int dpasses = radix_passes(32);
    const int tpasses = radix_passes(L.tile_bits);
    uint32_t *keys_in = at<uint32_t>(ws, dpasses % 2 ? L.keys_b : L.keys_a);
    uint32_t *keys_alt = at<uint32_t>(ws, dpasses % 2 ? L.keys_a : L.keys_b);
    uint32_t *ord_in = at<uint32_t>(ws, dpasses % 2 ? L.order_b : L.order_a);
    uint32_t *ord_alt = at<uint32_t>(ws, dpasses % 2 ? L.order_a : L.order_b);
    uint32_t *tiles_in = at<uint32_t>(ws, tpasses % 2 ? L.inst_tiles_b : L.inst_tiles_a);
    uint32_t *tiles_alt = at<uint32_t>(ws, tpasses % 2 ? L.inst_tiles_a : L.inst_tiles_b);
    uint32_t *ids_in = at<uint32_t>(ws, tpasses % 2 ? L.inst_ids_b : L.inst_ids_a);
    uint32_t *ids_alt = at<uint32_t>(ws, tpasses % 2 ? L.inst_ids_a : L.inst_ids_b);
    float4 *records = at<float4>(ws, L.records);
    uint2 *boxes = at<uint2>(ws, L.boxes);
    Conic *conics = at<Conic>(ws, L.conics);
    uint32_t *tile_counts = at<uint32_t>(ws, L.tile_counts);
    uint32_t *hist = at<uint32_t>(ws, L.hist);
    uint32_t *row_total = at<uint32_t>(ws, L.row_total);
    uint2 *ranges = at<uint2>(ws, L.ranges);
    uint32_t *sched = at<uint32_t>(ws, L.sched);
    const uint32_t *tile_order = at<uint32_t>(ws, L.tile_order);

    if (view_stamps) RGS_HIP(ctx, launch_view_clock_start(view_stamps, n_views, stream));
    unsigned long long *item_clock = view_stamps ? at<unsigned long long>(ws, L.item_clock) : nullptr;
    Timer tm(ctx, stream, timing, ST_PRE);
    uint2 *bin_boxes = at<uint2>(ws, L.bin_boxes);
    RGS_HIP(ctx, launch_preprocess(g, views, n_views, dopt, records, keys_in, boxes, bin_boxes, conics, tile_counts,
                                   at<double>(ws, L.crossing), counters + 5, L.crossing_cap, stream));
    tm.mark(ST_PRE);
    // counters: [0] box instances, [1] capacity, [2] tile rows, [3] listed instances, [4] kept views,
    // [5] quads with a vertex at z <= 0
    int64_t *listed = counters + 3, *kept = counters + 4;
    // the values of the first pass are the Gaussian-view ids, not read
    RGS_HIP(ctx, radix_sort(keys_in, ord_in, keys_alt, ord_alt, NV, nullptr, 32, true, 0xffffffffu, kept, hist,
                            row_total, stream, true));
    tm.mark(ST_DSORT);
    const uint32_t *order = at<uint32_t>(ws, L.order_a);
    uint32_t *offsets = at<uint32_t>(ws, L.offsets);
    uint32_t *row_offsets = at<uint32_t>(ws, L.row_offsets);
    uint32_t *row_owner = at<uint32_t>(ws, L.row_owner);
    uint2 *sorted_boxes = at<uint2>(ws, L.sorted_boxes);
    RGS_HIP(ctx, binning_scan(at<uint32_t>(ws, L.keys_a), bin_boxes, order, NV, kept, s.w, s.h, L.capacity, offsets,
                              row_offsets, row_owner, sorted_boxes,
                              at<unsigned long long>(ws, L.block_sums), counters, stream));
    tm.mark(ST_SCAN);
    const uint32_t empty_tile = (uint32_t)((int64_t(1) << L.tile_bits) - 1);
    RGS_HIP(ctx, launch_emit(order, offsets, row_offsets, row_owner, sorted_boxes, conics, views, g.n, n_views, counters,
                             L.capacity, s.w, s.h, empty_tile, tiles_in, ids_in, ranges, L.total_tiles, sched,
                             emit_grid(ctx->num_cus), stream));
    tm.mark(ST_EMIT);
    RGS_HIP(ctx, radix_sort(tiles_in, ids_in, tiles_alt, ids_alt, L.capacity, counters, L.tile_bits, true, empty_tile,
                            listed, hist, row_total, stream));
    tm.mark(ST_TSORT);
    const uint32_t *inst_tiles = at<uint32_t>(ws, L.inst_tiles_a);
    const uint32_t *inst_ids = at<uint32_t>(ws, L.inst_ids_a);
    const uint32_t split_min = slot_layout(s.w, s.h).slots >= 2 ? (uint32_t)RGS_SPLIT_LEN : 0u;
    const int blend_blocks = opts.mip == 2 ? ctx->grid_fwd_exact[shape_index(s)] : ctx->grid_fwd[shape_index(s)];
    const uint32_t waves = (uint32_t)(4 * blend_blocks);
    RGS_HIP(ctx, launch_tile_ranges(inst_tiles, listed, L.capacity, L.total_tiles, split_min, waves, ranges, sched,
                                    at<uint32_t>(ws, L.tile_order), stream));
    tm.mark(ST_RANGES);
    RGS_HIP(ctx, launch_blend(s, ranges, tile_order, sched + sched_item_count(), inst_ids, records, views, n_views,
                              L.total_tiles, NV, dopt, sched, blend_blocks, item_clock, stream));
    tm.mark(ST_BLEND);
    if (view_stamps)
        RGS_HIP(ctx, launch_view_clock_max(item_clock, tile_order, sched + sched_item_count(), 2 * L.total_tiles,
                                           views, n_views, view_stamps, stream));
    return RGS_OK;
}

rgs_status check_gaussians(rgs_context *ctx, const rgs_gaussians *g)
{
    if (!g) return fail(ctx, RGS_EINVAL, "g is NULL");
    if (g->n < 0) return fail(ctx, RGS_EINVAL, "n < 0");
    if (g->sh_degree < 0 || g->sh_degree > 3) return fail(ctx, RGS_EINVAL, "sh_degree=%d outside 0..3", g->sh_degree);
    if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh))
        return fail(ctx, RGS_EINVAL, "NULL Gaussian parameter pointer");
    return RGS_OK;
}

rgs_status check_outs(rgs_context *ctx, const rgs_view_out *outs, int n_views)
{
    if (!outs) return fail(ctx, RGS_EINVAL, "outs is NULL");
    for (int v = 0; v < n_views; ++v)
        if (!outs[v].rgb || !outs[v].final_T || !outs[v].n_contrib)
            return fail(ctx, RGS_EINVAL, "view %d: NULL output pointer", v);
    return RGS_OK;
}

rgs_status check_workspace(rgs_context *ctx, const rgs_workspace *ws, const Layout &L)
{
    if (!ws || !ws->ptr) return fail(ctx, RGS_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws->ptr) % kAlign)
        return fail(ctx, RGS_EINVAL, "workspace must be %zu-byte aligned", kAlign);
    if (ws->bytes < L.total)
        return fail(ctx, RGS_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws->bytes, L.total);
    return RGS_OK;
}

FrameShape frame_shape(const rgs_options &o, int64_t n, int32_t n_views, const rgs_workspace &ws)
{
    return FrameShape{shape_of(o), o.mip, o.divergence, n_views, n, ws.capacity, ws.flags};
}

// Options of the backward pass of the frame last rendered into `ws`: tile
// (0, 0) takes that frame's tile shape; anything that would lay the
// workspace out differently from that frame is an error.
rgs_status backward_options(rgs_context *ctx, int64_t n, const rgs_camera *cams, int32_t n_views,
                            const rgs_options *opts, const rgs_workspace *ws, rgs_options &out)
{
    const auto it = ctx->ws_frames.find(ws->ptr);
    if (it == ctx->ws_frames.end()) {
        out = resolve_tiles(ctx, n, cams, n_views, opts);
        return RGS_OK;
    }
    const FrameShape &f = it->second;
    out = *opts;
    if (out.tile_w == 0 && out.tile_h == 0) {
        out.tile_w = f.tile.w;
        out.tile_h = f.tile.h;
    }
    if (out.tile_w != f.tile.w || out.tile_h != f.tile.h)
        return fail(ctx, RGS_EINVAL, "tile %dx%d differs from the %dx%d of the frame last rendered into this workspace",
                    out.tile_w, out.tile_h, f.tile.w, f.tile.h);
    if (out.mip != f.mip || out.divergence != f.divergence || n != f.n || n_views != f.n_views ||
        ws->capacity != f.capacity || ws->flags != f.flags)
        return fail(ctx, RGS_EINVAL, "options, Gaussian count, views or workspace differ from the frame last "
                                     "rendered into this workspace");
    return RGS_OK;
}

}  // namespace

extern "C" {

rgs_status rgs_create(int device, rgs_context **out)
{
    if (!out) return RGS_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return RGS_EINVAL;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return RGS_EHIP;
    rgs_context *ctx = new rgs_context();
    ctx->device = device;
    ctx->num_cus = cus > 0 ? cus : 256;
    ctx->err.reserve(512);  // error messages are at most 511 characters
    ctx->noalloc_header.resize(align_up(8 * sizeof(int64_t)) + sizeof(DevView) * kMaxViews);
    // the scratch of rgs_render_noalloc; a failed lookup is reported by that call
    (void)scratch_setup(device);
    *out = ctx;
    return RGS_OK;
}

void rgs_destroy(rgs_context *ctx)
{
    if (!ctx) return;
    for (auto &fe : ctx->pending)
        for (auto &e : fe.ev) (void)hipEventDestroy(e);
    for (auto &fe : ctx->pool)
        for (auto &e : fe.ev) (void)hipEventDestroy(e);
    delete ctx;
}

const char *rgs_last_error(const rgs_context *ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

const char *rgs_stage_names(void) { return kStageNames; }

rgs_status rgs_workspace_size(rgs_context *ctx, int64_t n, const rgs_camera *cams, int32_t n_views,
                              const rgs_options *opts, int64_t capacity, int32_t flags, size_t *bytes)
{
    if (!bytes || !opts) return fail(ctx, RGS_EINVAL, "NULL argument");
    const rgs_options ro = resolve_tiles(ctx, n, cams, n_views, opts);
    Layout L;
    const rgs_status st = compute_layout(ctx, n, cams, n_views, &ro, capacity, flags, L);
    if (st != RGS_OK) return st;
    *bytes = L.total;
    return RGS_OK;
}

rgs_status rgs_get_workspace_layout(rgs_context *ctx, int64_t n, const rgs_camera *cams, int32_t n_views,
                                    const rgs_options *opts, int64_t capacity, int32_t flags,
                                    rgs_workspace_layout *out)
{
    if (!out || !opts) return fail(ctx, RGS_EINVAL, "NULL argument");
    const rgs_options ro = resolve_tiles(ctx, n, cams, n_views, opts);
    Layout L;
    const rgs_status st = compute_layout(ctx, n, cams, n_views, &ro, capacity, flags, L);
    if (st != RGS_OK) return st;
    fill_public_layout(L, out);
    return RGS_OK;
}

rgs_status rgs_render(rgs_context *ctx, const rgs_gaussians *g, const rgs_camera *cams, int32_t n_views,
                      const rgs_options *opts, const rgs_workspace *ws, const rgs_view_out *outs, void *stream)
{
    if (!ctx) return RGS_EINVAL;
    ctx->err.clear();
    rgs_status st = check_gaussians(ctx, g);
    if (st != RGS_OK) return st;
    if (!ws) return fail(ctx, RGS_EINVAL, "workspace is NULL");
    if (!opts) return fail(ctx, RGS_EINVAL, "opts is NULL");
    const rgs_options ro = resolve_tiles(ctx, g->n, cams, n_views, opts);
    opts = &ro;
    Layout L;
    if ((st = compute_layout(ctx, g->n, cams, n_views, opts, ws->capacity, ws->flags, L)) != RGS_OK) return st;
    if ((st = check_workspace(ctx, ws, L)) != RGS_OK) return st;
    if ((st = check_outs(ctx, outs, n_views)) != RGS_OK) return st;
    if (ctx->view_stamps && n_views > ctx->view_stamps_views)
        return fail(ctx, RGS_EINVAL, "%d views exceed the %d of the view clock buffer", n_views,
                    ctx->view_stamps_views);
    hipStream_t s = static_cast<hipStream_t>(stream);
    RGS_HIP(ctx, hipSetDevice(ctx->device));
    const std::vector<unsigned char> hdr = build_header(L, cams, n_views, outs, nullptr);
    RGS_HIP(ctx, put_bytes(ws->ptr, hdr.data(), hdr.size(), s));
    st = enqueue_forward(ctx, *g, n_views, *opts, L, ws->ptr, s, true, ctx->view_stamps);
    if (st == RGS_OK) ctx->ws_frames[ws->ptr] = frame_shape(*opts, g->n, n_views, *ws);
    if (st == RGS_OK && ctx->timing) ++ctx->frames;  // frames whose stages were timed
    return st;
}

rgs_status rgs_render_noalloc(rgs_context *ctx, const rgs_gaussians *g, const rgs_camera *cams, int32_t n_views,
                              const rgs_options *opts, const rgs_view_out *outs, int64_t *instances_needed,
                              void *stream)
{
    if (!ctx) return RGS_EINVAL;
    ctx->err.clear();
    rgs_status st = check_gaussians(ctx, g);
    if (st != RGS_OK) return st;
    if (!opts) return fail(ctx, RGS_EINVAL, "opts is NULL");
    if (ctx->device < 0 || ctx->device >= kMaxDevices || !g_scratch[ctx->device])
        return fail(ctx, RGS_EHIP, "no scratch on device %d: %s", ctx->device,
                    hipGetErrorString(ctx->device >= 0 && ctx->device < kMaxDevices ? g_scratch_error[ctx->device]
                                                                                     : hipErrorInvalidDevice));
    void *const ws = g_scratch[ctx->device];
    // tile (0, 0) is the default shape: the tuned-shape cache is not consulted
    // (its key is built on the heap)
    rgs_options o = *opts;
    if (o.tile_w == 0 && o.tile_h == 0) {
        o.tile_w = kDefaultTile.w;
        o.tile_h = kDefaultTile.h;
    }
    // the largest instance capacity whose layout fits the scratch
    Layout L;
    if ((st = compute_layout(ctx, g->n, cams, n_views, &o, 1, 0, L)) != RGS_OK) return st;
    if (L.total > kScratchBytes)
        return fail(ctx, RGS_EINVAL, "the frame needs %zu bytes of scratch with room for a single instance; the "
                                     "scratch holds %zu (fewer Gaussians or views, or rgs_render)",
                    L.total, kScratchBytes);
    int64_t lo = 1, hi = 0xffffffffLL;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        Layout M;
        if (compute_layout(ctx, g->n, cams, n_views, &o, mid, 0, M) == RGS_OK && M.total <= kScratchBytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    ctx->err.clear();
    if ((st = compute_layout(ctx, g->n, cams, n_views, &o, lo, 0, L)) != RGS_OK) return st;
    if ((st = check_outs(ctx, outs, n_views)) != RGS_OK) return st;
    if (reinterpret_cast<uintptr_t>(instances_needed) % 8)
        return fail(ctx, RGS_EINVAL, "instances_needed must be 8-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    RGS_HIP(ctx, hipSetDevice(ctx->device));
    unsigned char *hdr = ctx->noalloc_header.data();
    write_header(hdr, L, cams, n_views, outs, nullptr);
    RGS_HIP(ctx, hipMemcpyAsync(ws, hdr, header_bytes(L, n_views), hipMemcpyHostToDevice, s));
    if ((st = enqueue_forward(ctx, *g, n_views, o, L, ws, s, false)) != RGS_OK) return st;
    if (instances_needed) RGS_HIP(ctx, launch_copy_i64(at<int64_t>(ws, L.counters), instances_needed, s));
    return RGS_OK;
}

rgs_status rgs_render_status(rgs_context *ctx, const rgs_workspace *ws, void *stream, int64_t *instances)
{
    if (!ctx) return RGS_EINVAL;
    if (!ws || !ws->ptr) return fail(ctx, RGS_EINVAL, "workspace is NULL");
    RGS_HIP(ctx, hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    int64_t c[2] = {0, 0};
    RGS_HIP(ctx, hipMemcpy(c, ws->ptr, sizeof c, hipMemcpyDeviceToHost));
    if (instances) *instances = c[0];
    if (c[0] > ws->capacity)
        return fail(ctx, RGS_EOVERFLOW, "frame needed %lld instances, capacity %lld", (long long)c[0],
                    (long long)ws->capacity);
    return RGS_OK;
}

rgs_status rgs_render_backward(rgs_context *ctx, const rgs_gaussians *g, const rgs_camera *cams, int32_t n_views,
                               const rgs_options *opts, const rgs_workspace *ws, const rgs_view_out *outs,
                               const float *const *dL_drgb, const rgs_gaussian_grads *grads, void *stream)
{
    if (!ctx) return RGS_EINVAL;
    ctx->err.clear();
    rgs_status st = check_gaussians(ctx, g);
    if (st != RGS_OK) return st;
    if (!ws) return fail(ctx, RGS_EINVAL, "workspace is NULL");
    if (!opts) return fail(ctx, RGS_EINVAL, "opts is NULL");
    if (!cams || n_views < 1) return fail(ctx, RGS_EINVAL, "no cameras");
    rgs_options ro;
    if ((st = backward_options(ctx, g->n, cams, n_views, opts, ws, ro)) != RGS_OK) return st;
    opts = &ro;
    Layout L;
    if ((st = compute_layout(ctx, g->n, cams, n_views, opts, ws->capacity, ws->flags, L)) != RGS_OK) return st;
    if ((st = check_workspace(ctx, ws, L)) != RGS_OK) return st;
    if ((st = check_outs(ctx, outs, n_views)) != RGS_OK) return st;
    if (!(ws->flags & RGS_WS_BACKWARD)) return fail(ctx, RGS_EINVAL, "workspace lacks RGS_WS_BACKWARD");
    if (!dL_drgb) return fail(ctx, RGS_EINVAL, "dL_drgb is NULL");
    for (int v = 0; v < n_views; ++v)
        if (!dL_drgb[v]) return fail(ctx, RGS_EINVAL, "dL_drgb[%d] is NULL", v);
    if (!grads) return fail(ctx, RGS_EINVAL, "grads is NULL");
    if (opts->mip == 3) return fail(ctx, RGS_EUNSUPPORTED, "mip = 3 (dilation only) is not differentiated");
    if (g->n > 0 && (!grads->means || !grads->log_scales || !grads->quats || !grads->opacity_logits || !grads->sh))
        return fail(ctx, RGS_EINVAL, "NULL gradient pointer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    RGS_HIP(ctx, hipSetDevice(ctx->device));
    // refresh the view table with the upstream gradients (counters untouched)
    const std::vector<unsigned char> hdr = build_header(L, cams, n_views, outs, dL_drgb);
    RGS_HIP(ctx, hipMemcpyAsync(at<unsigned char>(ws->ptr, L.views), hdr.data() + L.views, hdr.size() - L.views,
                                hipMemcpyHostToDevice, s));
    const TileShape sh = shape_of(*opts);
    ensure_grids(ctx, sh);
    const DevOptions dopt = dev_options(*opts);
    uint32_t *sched = at<uint32_t>(ws->ptr, L.sched);
    float *rgrads = at<float>(ws->ptr, L.record_grads);
    RGS_HIP(ctx, launch_zero_kept_grads(at<uint32_t>(ws->ptr, L.order_a), at<int64_t>(ws->ptr, L.counters) + 4,
                                        L.nv_records, grad_floats(opts->mip), rgrads, ctx->num_cus, s));
    uint32_t *bwd_heads = sched + sched_backward_heads();
    RGS_HIP(ctx, launch_fill_u32(bwd_heads, 0u, (int64_t)kQueues * kQueueStride, s));
    // the stage times cover the compositing backward kernel alone, then the per-Gaussian chain
    Timer tm(ctx, s, true, ST_BLEND_BWD);
    RGS_HIP(ctx, launch_blend_backward(sh, at<uint2>(ws->ptr, L.ranges), at<uint32_t>(ws->ptr, L.tile_order),
                                       sched + sched_item_count(),
                                       at<uint32_t>(ws->ptr, L.inst_ids_a), at<float4>(ws->ptr, L.records),
                                       at<DevView>(ws->ptr, L.views), n_views, L.total_tiles, L.nv_records, dopt,
                                       rgrads, bwd_heads,
                                       opts->mip == 2 ? ctx->grid_bwd_exact[shape_index(sh)] : ctx->grid_bwd[shape_index(sh)],
                                       s));
    tm.mark(ST_BLEND_BWD);
    RGS_HIP(ctx, launch_preprocess_backward(*g, at<DevView>(ws->ptr, L.views), n_views, dopt,
                                            at<uint32_t>(ws->ptr, L.tile_counts), rgrads, *grads, s));
    tm.mark(ST_PRE_BWD);
    return RGS_OK;
}

rgs_status rgs_batch_plan(rgs_context *ctx, int64_t n, int32_t sh_degree, const rgs_camera *cams, int32_t n_views,
                          const rgs_options *opts, int64_t capacity, int32_t flags, size_t *ws_bytes, rgs_plan **out)
{
    if (!ctx || !out || !ws_bytes) return fail(ctx, RGS_EINVAL, "NULL argument");
    *out = nullptr;
    if (sh_degree < 0 || sh_degree > 3) return fail(ctx, RGS_EINVAL, "sh_degree outside 0..3");
    if (!opts) return fail(ctx, RGS_EINVAL, "opts is NULL");
    const rgs_options ro = resolve_tiles(ctx, n, cams, n_views, opts);
    opts = &ro;
    Layout L;
    const rgs_status st = compute_layout(ctx, n, cams, n_views, opts, capacity, flags, L);
    if (st != RGS_OK) return st;
    rgs_plan *p = new rgs_plan();
    p->ctx = ctx;
    p->n = n;
    p->sh_degree = sh_degree;
    p->cams.assign(cams, cams + n_views);
    p->opts = *opts;
    p->capacity = capacity;
    p->flags = flags;
    if (hipSetDevice(ctx->device) != hipSuccess ||
        hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        delete p;
        return fail(ctx, RGS_EHIP, "cannot create the capture stream");
    }
    ensure_grids(ctx, shape_of(*opts));
    *ws_bytes = L.total;
    *out = p;
    return RGS_OK;
}

void rgs_plan_destroy(rgs_plan *p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    delete p;
}

rgs_status rgs_batch_launch(rgs_plan *p, const rgs_gaussians *g, const rgs_camera *cams, const rgs_workspace *ws,
                            const rgs_view_out *outs, void *stream)
{
    if (!p) return RGS_EINVAL;
    rgs_context *ctx = p->ctx;
    ctx->err.clear();
    rgs_status st = check_gaussians(ctx, g);
    if (st != RGS_OK) return st;
    const int nv = (int)p->cams.size();
    if (g->n != p->n || g->sh_degree != p->sh_degree)
        return fail(ctx, RGS_EINVAL, "Gaussian count or SH degree differs from the plan");
    if (!cams) return fail(ctx, RGS_EINVAL, "cams is NULL");
    for (int v = 0; v < nv; ++v)
        if (cams[v].width != p->cams[v].width || cams[v].height != p->cams[v].height)
            return fail(ctx, RGS_EINVAL, "view %d: image size differs from the plan", v);
    if (!ws) return fail(ctx, RGS_EINVAL, "workspace is NULL");
    if (ws->capacity != p->capacity || ws->flags != p->flags)
        return fail(ctx, RGS_EINVAL, "workspace capacity or flags differ from the plan");
    Layout L;
    if ((st = compute_layout(ctx, p->n, cams, nv, &p->opts, p->capacity, p->flags, L)) != RGS_OK) return st;
    if ((st = check_workspace(ctx, ws, L)) != RGS_OK) return st;
    if ((st = check_outs(ctx, outs, nv)) != RGS_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    RGS_HIP(ctx, hipSetDevice(ctx->device));
    bool same = p->captured && ws->ptr == p->ws_ptr && std::memcmp(g, &p->g, sizeof *g) == 0;
    for (int v = 0; same && v < nv; ++v)
        same = outs[v].rgb == p->outs[v].rgb && outs[v].final_T == p->outs[v].final_T &&
               outs[v].n_contrib == p->outs[v].n_contrib;
    if (!same) {
        if (p->exec) {
            (void)hipGraphExecDestroy(p->exec);
            p->exec = nullptr;
        }
        if (p->graph) {
            (void)hipGraphDestroy(p->graph);
            p->graph = nullptr;
        }
        p->captured = false;
        RGS_HIP(ctx, hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal));
        st = enqueue_forward(ctx, *g, nv, p->opts, L, ws->ptr, p->capture_stream, false);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(p->capture_stream, &graph);
        if (st != RGS_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess || !graph) return fail(ctx, RGS_ECAPTURE, "capture failed: %s", hipGetErrorString(e));
        p->graph = graph;
        if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
            return fail(ctx, RGS_ECAPTURE, "graph instantiation failed");
        p->captured = true;
        p->g = *g;
        p->ws_ptr = ws->ptr;
        p->outs.assign(outs, outs + nv);
    }
    const std::vector<unsigned char> hdr = build_header(L, cams, nv, outs, nullptr);
    RGS_HIP(ctx, put_bytes(ws->ptr, hdr.data(), hdr.size(), s));
    RGS_HIP(ctx, hipGraphLaunch(p->exec, s));
    p->last_stream = s;
    p->launched = true;
    ctx->ws_frames[ws->ptr] = frame_shape(p->opts, p->n, nv, *ws);
    return RGS_OK;
}

rgs_status rgs_batch_status(rgs_plan *p, int64_t *instances_needed)
{
    if (!p) return RGS_EINVAL;
    rgs_context *ctx = p->ctx;
    if (!p->launched || !p->ws_ptr) return fail(ctx, RGS_EINVAL, "the plan has not been launched");
    RGS_HIP(ctx, hipSetDevice(ctx->device));
    RGS_HIP(ctx, hipStreamSynchronize(p->last_stream));
    int64_t c = 0;
    RGS_HIP(ctx, hipMemcpy(&c, p->ws_ptr, sizeof c, hipMemcpyDeviceToHost));
    if (instances_needed) *instances_needed = c;
    if (c > p->capacity)
        return fail(ctx, RGS_EOVERFLOW, "frame needed %lld instances, plan capacity %lld", (long long)c,
                    (long long)p->capacity);
    return RGS_OK;
}

}  // extern "C"

namespace {

// Times every supported tile shape: `reps` forward renders (each followed by
// a backward pass when dL_drgb is given) after one untimed step; shapes whose
// instances exceed the workspace capacity are skipped.
rgs_status autotune_shapes(rgs_context *ctx, const rgs_gaussians *g, const rgs_camera *cams, int32_t n_views,
                           const rgs_options *opts, const rgs_workspace *ws, const rgs_view_out *outs,
                           const float *const *dL_drgb, const rgs_gaussian_grads *grads, int32_t reps, void *stream,
                           rgs_options *best, double *best_ms)
{
    if (!ctx || !best || !best_ms || !opts) return fail(ctx, RGS_EINVAL, "NULL argument");
    if (reps < 1) return fail(ctx, RGS_EINVAL, "reps must be >= 1");
    static const TileShape shapes[] = {{8, 8}, {8, 16}, {8, 32}, {16, 8}, {16, 16}, {16, 32}, {32, 8}, {32, 16}, {32, 32}};
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    RGS_HIP(ctx, hipEventCreate(&e0));
    RGS_HIP(ctx, hipEventCreate(&e1));
    double best_t = 1e300;
    rgs_options chosen = *opts;
    rgs_status result = RGS_EOVERFLOW;
    const bool timing = ctx->timing;
    unsigned long long *const view_stamps = ctx->view_stamps;
    ctx->timing = false;
    ctx->view_stamps = nullptr;
    for (const TileShape &sh : shapes) {
        rgs_options o = *opts;
        o.tile_w = sh.w;
        o.tile_h = sh.h;
        auto step = [&]() {
            rgs_status st = rgs_render(ctx, g, cams, n_views, &o, ws, outs, stream);
            if (st == RGS_OK && dL_drgb)
                st = rgs_render_backward(ctx, g, cams, n_views, &o, ws, outs, dL_drgb, grads, stream);
            return st;
        };
        rgs_status st = rgs_render(ctx, g, cams, n_views, &o, ws, outs, stream);
        if (st == RGS_OK) st = rgs_render_status(ctx, ws, stream, nullptr);
        if (st == RGS_EOVERFLOW || st == RGS_EWORKSPACE) continue;
        if (st == RGS_OK && dL_drgb) st = rgs_render_backward(ctx, g, cams, n_views, &o, ws, outs, dL_drgb, grads, stream);
        if (st != RGS_OK) {
            result = st;
            break;
        }
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps && st == RGS_OK; ++r) st = step();
        (void)hipEventRecord(e1, s);
        if (st != RGS_OK) {
            result = st;
            break;
        }
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double t = ms / reps;
        if (t < best_t) {
            best_t = t;
            chosen = o;
        }
        result = RGS_OK;
    }
    ctx->timing = timing;
    ctx->view_stamps = view_stamps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != RGS_OK)
        return result == RGS_EOVERFLOW ? fail(ctx, RGS_EOVERFLOW, "no tile shape fits the workspace capacity")
                                       : result;
    *best = chosen;
    *best_ms = best_t;
    ctx->tune_cache[tune_class(dL_drgb != nullptr, g->n, cams, n_views, *opts)] = shape_of(chosen);
    return RGS_OK;
}

}  // namespace

extern "C" {

rgs_status rgs_autotune(rgs_context *ctx, const rgs_gaussians *g, const rgs_camera *cams, int32_t n_views,
                        const rgs_options *opts, const rgs_workspace *ws, const rgs_view_out *outs, int32_t reps,
                        void *stream, rgs_options *best, double *best_ms)
{
    return autotune_shapes(ctx, g, cams, n_views, opts, ws, outs, nullptr, nullptr, reps, stream, best, best_ms);
}

rgs_status rgs_autotune_training(rgs_context *ctx, const rgs_gaussians *g, const rgs_camera *cams, int32_t n_views,
                                 const rgs_options *opts, const rgs_workspace *ws, const rgs_view_out *outs,
                                 const float *const *dL_drgb, const rgs_gaussian_grads *grads, int32_t reps,
                                 void *stream, rgs_options *best, double *best_ms)
{
    if (!dL_drgb) return fail(ctx, RGS_EINVAL, "dL_drgb is NULL");
    return autotune_shapes(ctx, g, cams, n_views, opts, ws, outs, dL_drgb, grads, reps, stream, best, best_ms);
}

rgs_status rgs_set_view_clocks(rgs_context *ctx, uint64_t *stamps, int32_t max_views)
{
    if (!ctx) return RGS_EINVAL;
    if (stamps && (max_views < 1 || max_views > kMaxViews))
        return fail(ctx, RGS_EINVAL, "max_views=%d outside 1..%d", max_views, kMaxViews);
    if (reinterpret_cast<uintptr_t>(stamps) % 8) return fail(ctx, RGS_EINVAL, "stamps must be 8-byte aligned");
    ctx->view_stamps = reinterpret_cast<unsigned long long *>(stamps);
    ctx->view_stamps_views = stamps ? max_views : 0;
    return RGS_OK;
}

double rgs_wall_clock_hz(rgs_context *ctx)
{
    if (!ctx) return 0.0;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess) return 0.0;
    return 1e3 * khz;
}

rgs_status rgs_downsample_box(rgs_context *ctx, const float *src, int32_t width, int32_t height, int32_t factor,
                              int32_t planes, float *dst, void *stream)
{
    if (!ctx) return RGS_EINVAL;
    ctx->err.clear();
    if (!src || !dst) return fail(ctx, RGS_EINVAL, "src or dst is NULL");
    if (factor < 1 || factor > 16) return fail(ctx, RGS_EINVAL, "factor=%d outside [1, 16]", factor);
    if (width < 1 || width > 16384 || height < 1 || height > 16384)
        return fail(ctx, RGS_EINVAL, "size %dx%d outside [1, 16384]", width, height);
    if (planes < 1 || planes > 4) return fail(ctx, RGS_EINVAL, "planes=%d outside [1, 4]", planes);
    RGS_HIP(ctx, hipSetDevice(ctx->device));
    RGS_HIP(ctx, launch_downsample_box(src, width, height, factor, planes, dst, static_cast<hipStream_t>(stream)));
    return RGS_OK;
}

rgs_status rgs_calibrate(rgs_context *ctx, void *stream, double *fma_tflops, double *exp_tops, double *copy_gbs)
{
    if (!ctx) return RGS_EINVAL;
    ctx->err.clear();
    if (!fma_tflops || !exp_tops || !copy_gbs) return fail(ctx, RGS_EINVAL, "NULL output");
    RGS_HIP(ctx, hipSetDevice(ctx->device));
    RGS_HIP(ctx, measure_ceilings(ctx->num_cus, static_cast<hipStream_t>(stream), fma_tflops, exp_tops, copy_gbs));
    return RGS_OK;
}

rgs_status rgs_set_stage_timing(rgs_context *ctx, int32_t enable)
{
    if (!ctx) return RGS_EINVAL;
    ctx->timing = enable != 0;
    return RGS_OK;
}

int32_t rgs_stage_times(rgs_context *ctx, double *ms, int32_t n, int64_t *frames)
{
    if (!ctx) return 0;
    for (auto &fe : ctx->pending) {
        (void)hipEventSynchronize(fe.ev[fe.last]);
        for (int st = fe.first; st < fe.last; ++st) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, fe.ev[st], fe.ev[st + 1]) == hipSuccess) ctx->stage_ms[st] += t;
        }
        ctx->pool.push_back(fe);
    }
    ctx->pending.clear();
    if (ms)
        for (int k = 0; k < n && k < kNumStages; ++k) ms[k] = ctx->stage_ms[k];
    if (frames) *frames = ctx->frames;
    for (double &v : ctx->stage_ms) v = 0.0;
    ctx->frames = 0;
    return kNumStages;
}

}  // extern "C"
