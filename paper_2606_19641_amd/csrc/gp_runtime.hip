// C ABI runtime of the Gigapixel hot path: argument checks, workspace
// layout, scene upload (with spatial sorting of road strips into culling
// bins), launch scheduling (per-scene, persistent work queue, hipGraph
// replay) and error reporting.  The declarations and their contract are in
// include/gp.h.
#include "../../include/gp.h"
#include "gp_device.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <climits>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

namespace {

thread_local std::string g_last_error;

gp_status fail(gp_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
gp_status fail(gp_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

gp_status hip_fail(hipError_t e, const char *what)
{
    return fail(GP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr int64_t kAlign = 256;
int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Bins a scene of n_roads strips may use: twice the count-limited number, so
// that bins can also be closed on extent (sort_roads).
int64_t n_bins_of(int32_t n_roads) { return 2 * ((n_roads + gp::kBinQuads - 1) / gp::kBinQuads); }
constexpr float kBinExtent = 32.0f;   // metres

struct Layout {
    int64_t halted, infr, actu, signals, signal_color;
    int64_t scenes, views, state, cs, dims, agent_color, roads, road_index, road_color, bins, palette,
        queue, order, counter;
    int64_t upload_end;   // the sections above are uploaded at creation
    // the chip-wide rgb raster's buffers (present when chip is true); ctl and
    // cov are zeroed at creation, the others need no initial value
    bool chip;
    int64_t chip_ctl, chip_cov, chip_sbins, chip_vinfo, chip_btri, chip_rinfo, chip_rtri, chip_rrows, chip_items,
        chip_end;
    int64_t bins_stride, btri_cap, rtri_cap;
    int64_t total;
    int64_t n_agents, n_roads, n_views, n_bins, n_static, n_signals;
};

// box triangles one view's list holds in the chip-wide raster (a view with
// more is set up again per resolve item)
constexpr int64_t kChipBoxTris = 128;

// can the chip-wide raster serve this image size?
bool chip_size_ok(int32_t width, int32_t height)
{
    return width % 16 == 0 && width >= 64 && width <= 1024 && height >= 1;
}

bool finite_cfg(const gp_config *c)
{
    return std::isfinite(c->focal_px) && std::isfinite(c->cam_height) && std::isfinite(c->z_near) &&
           std::isfinite(c->z_far) && std::isfinite(c->dt);
}

gp_status check_inputs(const gp_config *cfg, const gp_scene_desc *sc, int32_t n)
{
    if (!cfg) return fail(GP_EINVAL, "cfg is NULL");
    if (cfg->width < 1 || cfg->width > 1024 || cfg->height < 1 || cfg->height > 1024)
        return fail(GP_EINVAL, "image size %dx%d outside 1..1024", cfg->width, cfg->height);
    if (cfg->n_cams < 1 || cfg->n_cams > GP_MAX_CAMS)
        return fail(GP_EINVAL, "n_cams %d outside 1..%d", cfg->n_cams, GP_MAX_CAMS);
    if (!finite_cfg(cfg) || !(cfg->focal_px > 0.0f) || !(cfg->z_near > 0.0f) || !(cfg->z_far > cfg->z_near) ||
        !(cfg->dt >= 0.0f) || !(cfg->cam_height > 0.0f))
        return fail(GP_EINVAL, "camera/dynamics constants out of range");
    if (cfg->focal_px > 1024.0f) return fail(GP_EINVAL, "focal length above 1024 px");
    for (int k = 0; k < cfg->n_cams; ++k)
        if (!std::isfinite(cfg->cam_dir[k][0]) || !std::isfinite(cfg->cam_dir[k][1]))
            return fail(GP_EINVAL, "camera direction %d not finite", k);
    if (n < 1) return fail(GP_EINVAL, "n_scenes must be >= 1");
    if (!sc) return fail(GP_EINVAL, "scenes is NULL");
    int64_t na = 0, nr = 0;
    for (int s = 0; s < n; ++s) {
        const gp_scene_desc &d = sc[s];
        if (d.n_agents < 1 || d.n_roads < 0)
            return fail(GP_EINVAL, "scene %d: n_agents must be >= 1 and n_roads >= 0", s);
        if (d.n_static < 0) return fail(GP_EINVAL, "scene %d: n_static must be >= 0", s);
        if (d.n_signals < 0) return fail(GP_EINVAL, "scene %d: n_signals must be >= 0", s);
        if (6LL * ((int64_t)d.n_agents + d.n_static) + d.n_roads + d.n_signals >= gp::kMaxPrims)
            return fail(GP_EINVAL, "scene %d: more than %d primitives", s, gp::kMaxPrims);
        if (d.n_static > 0 && (!d.static_xyp || !d.static_dims || !d.static_color))
            return fail(GP_EINVAL, "scene %d: static obstacle arrays are NULL", s);
        for (int64_t i = 0; i < 3LL * d.n_static; ++i)
            if (!std::isfinite(d.static_xyp[i]) || !std::isfinite(d.static_dims[i]))
                return fail(GP_EINVAL, "scene %d: static obstacle not finite", s);
        if (d.n_signals > 0 && (!d.signal_xyzr || !d.signal_color))
            return fail(GP_EINVAL, "scene %d: traffic light arrays are NULL", s);
        for (int64_t g = 0; g < d.n_signals; ++g) {
            for (int k = 0; k < 4; ++k)
                if (!std::isfinite(d.signal_xyzr[4 * g + k]))
                    return fail(GP_EINVAL, "scene %d: traffic light not finite", s);
            if (!(d.signal_xyzr[4 * g + 3] > 0.0f) || d.signal_xyzr[4 * g + 3] > 100.0f)
                return fail(GP_EINVAL, "scene %d: traffic light radius outside (0, 100] m", s);
        }
        if (!d.agent_state || !d.agent_dims || !d.agent_color)
            return fail(GP_EINVAL, "scene %d: agent arrays are NULL", s);
        if (d.n_roads > 0 && (!d.road_xy || !d.road_color))
            return fail(GP_EINVAL, "scene %d: road arrays are NULL", s);
        for (int64_t i = 0; i < 8LL * d.n_roads; ++i)
            if (!std::isfinite(d.road_xy[i])) return fail(GP_EINVAL, "scene %d: road corner not finite", s);
        na += d.n_agents;
        nr += d.n_roads;
    }
    int64_t ns = 0;
    for (int s = 0; s < n; ++s) ns += sc[s].n_static;
    if (na * cfg->n_cams >= (1LL << 31)) return fail(GP_EINVAL, "too many views");
    if (na + ns >= (1LL << 31)) return fail(GP_EINVAL, "too many boxes");
    if (nr >= (1LL << 31)) return fail(GP_EINVAL, "too many roads");
    return GP_OK;
}

Layout make_layout(const gp_config *cfg, const gp_scene_desc *sc, int32_t n)
{
    Layout L{};
    for (int s = 0; s < n; ++s) {
        L.n_agents += sc[s].n_agents;
        L.n_static += sc[s].n_static;
        L.n_signals += sc[s].n_signals;
        L.n_roads += sc[s].n_roads;
        L.n_bins += n_bins_of(sc[s].n_roads);
    }
    L.n_views = L.n_agents * cfg->n_cams;
    int64_t o = 0;
    auto take = [&](int64_t bytes) { int64_t at = o; o = align_up(o + std::max<int64_t>(bytes, 1)); return at; };
    L.scenes = take(sizeof(gp::SceneRec) * (int64_t)n);
    L.views = take(sizeof(gp::ViewRec) * L.n_views);
    // box arrays: the agents, then the static obstacles
    const int64_t n_box = L.n_agents + L.n_static;
    L.state = take(16 * n_box);
    L.cs = take(8 * n_box);
    L.dims = take(16 * n_box);
    L.agent_color = take(n_box);
    L.roads = take(32 * L.n_roads);
    L.road_index = take(4 * L.n_roads);
    L.road_color = take(L.n_roads);
    L.bins = take(sizeof(gp::RoadBin) * L.n_bins);
    L.palette = take(768);
    L.halted = take(L.n_agents);
    L.infr = take(L.n_agents);
    L.actu = take(16 * L.n_agents);
    L.signals = take(16 * L.n_signals);
    L.signal_color = take(L.n_signals);
    L.queue = take(4 * L.n_views);
    L.order = take(4 * L.n_views);
    L.counter = take(4 * (gp::kQueues + 2) * gp::kCtrStride);
    L.upload_end = o;
    L.chip = chip_size_ok(cfg->width, cfg->height);
    if (L.chip) {
        int64_t max_bins = 1, units = 0, max_roads = 0;
        for (int s = 0; s < n; ++s) {
            const int64_t nb = n_bins_of(sc[s].n_roads);
            max_bins = std::max(max_bins, nb);
            max_roads = std::max<int64_t>(max_roads, sc[s].n_roads);
            units += (int64_t)sc[s].n_agents * cfg->n_cams * ((nb + 3) / 4);
        }
        const int64_t nw = (cfg->width + 63) / 64;
        L.bins_stride = max_bins;
        L.btri_cap = kChipBoxTris;
        // road triangles a view's list holds (more go to the coverage words)
        L.rtri_cap = std::min<int64_t>(1024, std::max<int64_t>(256, (max_roads / 8 + 63) / 64 * 64));
        L.chip_ctl = take(4 * gp::CHIP_NCTL);
        L.chip_cov = take(8 * nw * cfg->height * L.n_views);
        L.chip_sbins = take(4 * L.bins_stride * L.n_views);
        L.chip_vinfo = take(16 * L.n_views);
        L.chip_btri = take(48 * L.btri_cap * L.n_views);
        L.chip_rinfo = take(16 * L.n_views);
        L.chip_rtri = take(32 * L.rtri_cap * L.n_views);
        L.chip_rrows = take(4 * L.rtri_cap * L.n_views);
        L.chip_items = take(8 * units);
        L.chip_end = o;
    }
    L.total = o;
    return L;
}

bool valid_launch(const gp_launch &l)
{
    const bool br = l.band_rows == 8 || l.band_rows == 16 || l.band_rows == 32 || l.band_rows == 64;
    const bool bt = l.batch_tris == 256 || l.batch_tris == 512 || l.batch_tris == 1024 || l.batch_tris == 2048;
    const bool th = l.block_threads == 256 || l.block_threads == 512 || l.block_threads == 1024;
    const bool sc = l.sched == GP_SCHED_PLAIN || l.sched == GP_SCHED_PERSISTENT;
    const bool ra = l.raster == GP_RASTER_BANDED || l.raster == GP_RASTER_SPLIT || l.raster == GP_RASTER_CHIP;
    const bool vw = l.view_waves == 1 || l.view_waves == 2 || l.view_waves == 4;
    const bool cw = l.road_wgs_per_cu >= 1 && l.road_wgs_per_cu <= 16;
    return br && bt && th && sc && ra && vw && cw && l.blocks_per_cu >= 1 && l.blocks_per_cu <= 16;
}

// 2-D Morton code of 16-bit coordinates
uint32_t morton16(uint32_t x, uint32_t y)
{
    auto spread = [](uint32_t v) {
        v &= 0xFFFFu;
        v = (v | (v << 8)) & 0x00FF00FFu;
        v = (v | (v << 4)) & 0x0F0F0F0Fu;
        v = (v | (v << 2)) & 0x33333333u;
        v = (v | (v << 1)) & 0x55555555u;
        return v;
    };
    return spread(x) | (spread(y) << 1);
}

// Order the road strips of one scene along a Morton curve of their centres
// and cut the order into bins of at most kBinQuads strips; each bin keeps the
// exact float bounding box of its strips' corners.  Where the curve jumps, a
// bin of 16 consecutive strips can span most of the map, which makes its box
// useless for culling; so a bin is also closed before a strip that would
// stretch its box beyond kBinExtent metres on either axis, as long as the
// remaining strips still fit in n_bins_of(n) bins.  Returns the slot -> input
// index map.
std::vector<int32_t> sort_roads(const gp_scene_desc &d, std::vector<gp::RoadBin> &bins)
{
    const int n = d.n_roads;
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    if (n == 0) return order;
    double xmin = 1e300, ymin = 1e300, xmax = -1e300, ymax = -1e300;
    std::vector<double> cx(n), cy(n);
    for (int r = 0; r < n; ++r) {
        double sx = 0, sy = 0;
        for (int k = 0; k < 4; ++k) {
            sx += d.road_xy[8 * r + 2 * k];
            sy += d.road_xy[8 * r + 2 * k + 1];
        }
        cx[r] = sx / 4;
        cy[r] = sy / 4;
        xmin = std::min(xmin, cx[r]);
        xmax = std::max(xmax, cx[r]);
        ymin = std::min(ymin, cy[r]);
        ymax = std::max(ymax, cy[r]);
    }
    const double sx = xmax > xmin ? 65535.0 / (xmax - xmin) : 0.0;
    const double sy = ymax > ymin ? 65535.0 / (ymax - ymin) : 0.0;
    std::vector<uint32_t> code(n);
    for (int r = 0; r < n; ++r)
        code[r] = morton16((uint32_t)((cx[r] - xmin) * sx), (uint32_t)((cy[r] - ymin) * sy));
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return code[a] < code[b]; });
    const int64_t budget = n_bins_of(n);
    gp::RoadBin bn{};
    bn.xmin = bn.ymin = INFINITY;
    bn.xmax = bn.ymax = -INFINITY;
    for (int k = 0; k < n; ++k) {
        const int r = order[k];
        float x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
        for (int c = 0; c < 4; ++c) {
            const float x = d.road_xy[8 * r + 2 * c], y = d.road_xy[8 * r + 2 * c + 1];
            x0 = std::min(x0, x);
            x1 = std::max(x1, x);
            y0 = std::min(y0, y);
            y1 = std::max(y1, y);
        }
        if (bn.count > 0) {
            const bool full = bn.count == gp::kBinQuads;
            const bool wide = std::max(bn.xmax, x1) - std::min(bn.xmin, x0) > kBinExtent ||
                              std::max(bn.ymax, y1) - std::min(bn.ymin, y0) > kBinExtent;
            // closing here leaves n - k strips for budget - (bins + 1) bins
            const int64_t need = (int64_t)bins.size() + 1 + (n - k + gp::kBinQuads - 1) / gp::kBinQuads;
            if (full || (wide && need <= budget)) {
                bins.push_back(bn);
                bn = gp::RoadBin{};
                bn.start = k;
                bn.xmin = bn.ymin = INFINITY;
                bn.xmax = bn.ymax = -INFINITY;
            }
        }
        bn.count += 1;
        bn.xmin = std::min(bn.xmin, x0);
        bn.ymin = std::min(bn.ymin, y0);
        bn.xmax = std::max(bn.xmax, x1);
        bn.ymax = std::max(bn.ymax, y1);
    }
    bins.push_back(bn);
    return order;
}

}  // namespace

struct gp_sim {
    gp_config cfg;
    int32_t n_scenes = 0;
    Layout lay{};
    std::vector<gp::SceneRec> scenes;
    gp::DevSim dev{};
    gp_launch launch{};
    int device = 0;
    int n_cu = 256;
    size_t max_lds = 65536;
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphNode_t g_step = nullptr;   // the step's kernel node (its action pointer is updated in place)
    const float *g_act = nullptr;
    uint8_t *g_rgb = nullptr;
    gp_launch g_launch{};
    gp::ChipBufs chip{};        // the chip-wide raster's buffers (lay.chip)
    int32_t road_uniform = 0;   // every road strip of every scene has one colour
    int32_t bins_cap = 1;       // culling bins of the largest scene
};

namespace {

gp::LaunchCfg launch_cfg(const gp_launch &l)
{
    gp::LaunchCfg c;
    c.band_rows = l.band_rows;
    c.batch_tris = l.batch_tris;
    c.block_threads = l.block_threads;
    return c;
}

gp_status check_lds(const gp_sim *sim, const gp_launch &l)
{
    const size_t need = std::max(gp::render_lds_bytes(sim->dev, launch_cfg(l), 0),
                                 sim->road_uniform ? gp::render_lds_bytes(sim->dev, launch_cfg(l), 1) : 0);
    if (need > sim->max_lds)
        return fail(GP_EINVAL, "launch needs %zu B of LDS, the device allows %zu", need, sim->max_lds);
    return GP_OK;
}

// box triangles one view's list holds in the split rasteriser (at least the
// 96 that its streaming pass can need)
constexpr int kSplitBoxTris = 96;

gp::RgbCfg rgb_cfg(const gp_sim *sim, const gp_launch &l)
{
    gp::RgbCfg c;
    c.waves = l.view_waves;
    c.bcap = kSplitBoxTris;
    c.bins_cap = sim->bins_cap;
    return c;
}

// can this render take the chip-wide rasteriser?
bool chip_ok(const gp_sim *sim, const gp::RenderOut &o, const gp_launch &l, int kind)
{
    return l.raster == GP_RASTER_CHIP && kind == 1 && sim->lay.chip && sim->cfg.cam_height > 0.0f &&
           reinterpret_cast<uintptr_t>(o.rgb) % 16 == 0 && sim->bins_cap <= sim->lay.bins_stride;
}

// can this render take the split rasteriser?
bool split_ok(const gp_sim *sim, const gp::RenderOut &o, const gp_launch &l, int kind)
{
    return l.raster == GP_RASTER_SPLIT && kind == 1 && sim->cfg.width % 16 == 0 &&
           reinterpret_cast<uintptr_t>(o.rgb) % 16 == 0 && sim->cfg.cam_height > 0.0f &&
           gp::rgb_lds_bytes(sim->cfg.width, sim->cfg.height, rgb_cfg(sim, l)) <= sim->max_lds;
}

gp_status render_impl(gp_sim *sim, const gp::RenderOut &o, const gp_launch &l, hipStream_t st)
{
    const gp::LaunchCfg c = launch_cfg(l);
    // the rgb-only kernels serve renders without depth / primitive id when
    // every road strip has the same colour; everything else takes the general one
    // (scenes with traffic lights take the general kernel's instances with lights)
    const int kind = sim->lay.n_signals > 0 ? 2 : (!o.depth && !o.primid && sim->dev.road_color_uniform) ? 1 : 0;
    const bool split = split_ok(sim, o, l, kind);
    const gp::RgbCfg rc = rgb_cfg(sim, l);
    hipError_t e;
    if (chip_ok(sim, o, l, kind)) {
        const int rg = l.road_wgs_per_cu * sim->n_cu;
        if (l.sched == GP_SCHED_PLAIN) {
            for (int s = 0; s < sim->n_scenes; ++s) {
                const gp::SceneRec &r = sim->scenes[s];
                e = gp::launch_render_chip(sim->dev, o, sim->chip, 0, r.view_base, r.n_agents * sim->cfg.n_cams, rg,
                                           st);
                if (e != hipSuccess) return hip_fail(e, "render launch");
            }
            return GP_OK;
        }
        e = gp::launch_render_chip(sim->dev, o, sim->chip, 1, 0, (int)sim->lay.n_views, rg, st);
        if (e != hipSuccess) return hip_fail(e, "render launch");
        return GP_OK;
    }
    if (l.sched == GP_SCHED_PLAIN) {
        for (int s = 0; s < sim->n_scenes; ++s) {
            const gp::SceneRec &r = sim->scenes[s];
            const int nv = r.n_agents * sim->cfg.n_cams;
            e = split ? gp::launch_render_rgb(sim->dev, o, rc, 0, r.view_base, nv, st)
                      : gp::launch_render(sim->dev, o, c, kind, 0, r.view_base, nv, st);
            if (e != hipSuccess) return hip_fail(e, "render launch");
        }
        return GP_OK;
    }
    const int64_t resident = (int64_t)l.blocks_per_cu * sim->n_cu;
    if (sim->lay.n_views <= resident || split) {
        // every view gets a workgroup of its own: one launch over all views,
        // without the queue (whose empty segments would cost each workgroup a
        // chain of device-scope atomics before it finds its view).  The
        // wave-split raster always launches so: with more views than fit the
        // chip at once, the dispatcher hands each freed slot the next view
        // (XCD-ordered), which balances uneven views without atomics
        e = split ? gp::launch_render_rgb(sim->dev, o, rc, 1, 0, (int)sim->lay.n_views, st)
                  : gp::launch_render(sim->dev, o, c, kind, 0, 0, (int)sim->lay.n_views, st);
    } else {
        e = gp::launch_render(sim->dev, o, c, kind, 1, 0, (int)resident, st);
    }
    if (e != hipSuccess) return hip_fail(e, "render launch");
    return GP_OK;
}

gp_status step_impl(gp_sim *sim, const float *act, const gp_launch &l, hipStream_t st)
{
    hipError_t e;
    if (l.sched == GP_SCHED_PLAIN) {
        for (int s = 0; s < sim->n_scenes; ++s) {
            const gp::SceneRec &r = sim->scenes[s];
            e = gp::launch_step(sim->dev, act, r.agent_base, r.n_agents, st);
            if (e != hipSuccess) return hip_fail(e, "step launch");
        }
        return GP_OK;
    }
    e = gp::launch_step(sim->dev, act, 0, (int)sim->lay.n_agents, st);
    if (e != hipSuccess) return hip_fail(e, "step launch");
    return GP_OK;
}

void drop_graph(gp_sim *sim)
{
    if (sim->gexec) (void)hipGraphExecDestroy(sim->gexec);
    if (sim->graph) (void)hipGraphDestroy(sim->graph);
    sim->gexec = nullptr;
    sim->graph = nullptr;
    sim->g_step = nullptr;
}

bool same_launch(const gp_launch &a, const gp_launch &b)
{
    return a.sched == b.sched && a.band_rows == b.band_rows && a.batch_tris == b.batch_tris &&
           a.block_threads == b.block_threads && a.blocks_per_cu == b.blocks_per_cu && a.raster == b.raster &&
           a.view_waves == b.view_waves && a.road_wgs_per_cu == b.road_wgs_per_cu;
}

}  // namespace

extern "C" {

const char *gp_last_error(void) { return g_last_error.c_str(); }

int64_t gp_sim_required_bytes(const gp_config *cfg, const gp_scene_desc *scenes, int32_t n_scenes)
{
    if (check_inputs(cfg, scenes, n_scenes) != GP_OK) return -1;
    return make_layout(cfg, scenes, n_scenes).total;
}

gp_status gp_sim_create(const gp_config *cfg, const gp_scene_desc *scenes, int32_t n_scenes,
                        void *d_workspace, int64_t workspace_bytes, void *stream, gp_sim **out)
{
    if (!out) return fail(GP_EINVAL, "out is NULL");
    *out = nullptr;
    gp_status st = check_inputs(cfg, scenes, n_scenes);
    if (st != GP_OK) return st;
    const Layout L = make_layout(cfg, scenes, n_scenes);
    if (!d_workspace) return fail(GP_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign != 0)
        return fail(GP_EINVAL, "workspace must be %lld-byte aligned", (long long)kAlign);
    if (workspace_bytes < L.total)
        return fail(GP_ENOMEM, "workspace has %lld bytes, %lld needed", (long long)workspace_bytes,
                    (long long)L.total);

    gp_sim *sim = new (std::nothrow) gp_sim();
    if (!sim) return fail(GP_ENOMEM, "host allocation failed");
    sim->cfg = *cfg;
    sim->n_scenes = n_scenes;
    sim->lay = L;
    // host image of the workspace
    std::vector<unsigned char> host((size_t)L.upload_end, 0);
    auto at = [&](int64_t off) { return host.data() + off; };
    sim->scenes.resize(n_scenes);
    auto *views = reinterpret_cast<gp::ViewRec *>(at(L.views));
    auto *state = reinterpret_cast<float *>(at(L.state));
    auto *dims = reinterpret_cast<float *>(at(L.dims));
    auto *acol = at(L.agent_color);
    auto *roads = reinterpret_cast<float *>(at(L.roads));
    auto *ridx = reinterpret_cast<int32_t *>(at(L.road_index));
    auto *rcol = at(L.road_color);
    auto *bins = reinterpret_cast<gp::RoadBin *>(at(L.bins));
    int32_t abase = 0, rbase = 0, bbase = 0, sbase = (int32_t)L.n_agents, gbase = 0;
    auto *sig = reinterpret_cast<float *>(at(L.signals));
    auto *sigc = at(L.signal_color);
    bool uniform = true;
    int color0 = -1;
    for (int s = 0; s < n_scenes; ++s) {
        const gp_scene_desc &d = scenes[s];
        gp::SceneRec &r = sim->scenes[s];
        std::vector<gp::RoadBin> sb;
        const std::vector<int32_t> order = sort_roads(d, sb);
        r.agent_base = abase;
        r.n_agents = d.n_agents;
        r.road_base = rbase;
        r.n_roads = d.n_roads;
        r.view_base = abase * cfg->n_cams;
        r.bin_base = bbase;
        r.n_bins = (int32_t)sb.size();
        r.static_base = sbase;
        r.n_static = d.n_static;
        for (int k = 0; k < d.n_static; ++k) {     // static obstacles: v = 0, never stepped
            const int g = sbase + k;
            for (int c = 0; c < 3; ++c) state[4 * g + c] = d.static_xyp[3 * k + c];
            state[4 * g + 3] = 0.0f;
            for (int c = 0; c < 3; ++c) dims[4 * g + c] = d.static_dims[3 * k + c];
            dims[4 * g + 3] = 0.0f;
            acol[g] = d.static_color[k];
        }
        sbase += d.n_static;
        r.signal_base = gbase;
        r.n_signals = d.n_signals;
        if (d.n_signals > 0) {
            std::memcpy(sig + 4 * (int64_t)gbase, d.signal_xyzr, 16 * (size_t)d.n_signals);
            std::memcpy(sigc + gbase, d.signal_color, (size_t)d.n_signals);
        }
        gbase += d.n_signals;
        for (int a = 0; a < d.n_agents; ++a) {
            const int g = r.agent_base + a;
            for (int k = 0; k < 4; ++k) state[4 * g + k] = d.agent_state[4 * a + k];
            for (int k = 0; k < 3; ++k) dims[4 * g + k] = d.agent_dims[3 * a + k];
            dims[4 * g + 3] = 0.0f;
            acol[g] = d.agent_color[a];
            for (int c = 0; c < cfg->n_cams; ++c) {
                gp::ViewRec &v = views[(int64_t)g * cfg->n_cams + c];
                v.scene = s;
                v.ego_cam = a * 4 + c;
            }
        }
        for (int k = 0; k < d.n_roads; ++k) {
            const int src = order[k];
            std::memcpy(roads + 8 * (int64_t)(rbase + k), d.road_xy + 8 * (int64_t)src, 32);
            ridx[rbase + k] = src;
            rcol[rbase + k] = d.road_color[src];
            if (color0 < 0) color0 = d.road_color[src];
            uniform = uniform && d.road_color[src] == color0;
        }
        if (!sb.empty()) std::memcpy(bins + bbase, sb.data(), sizeof(gp::RoadBin) * sb.size());
        abase += d.n_agents;
        rbase += d.n_roads;
        bbase += (int32_t)sb.size();
        sim->bins_cap = std::max<int32_t>(sim->bins_cap, (int32_t)sb.size());
    }
    std::memcpy(at(L.scenes), sim->scenes.data(), sizeof(gp::SceneRec) * n_scenes);
    std::memcpy(at(L.palette), cfg->palette, 768);
    // persistent queue: kQueues segments, one per XCD, each holding whole
    // scenes so that a scene's geometry is read through one L2.  Scenes go to
    // the segment with the least work so far, heaviest first (work of a view
    // ~ its candidate primitives); inside a segment heavier scenes come first
    // and the views of a scene are adjacent.
    std::vector<int> order(n_scenes);
    std::iota(order.begin(), order.end(), 0);
    auto view_work = [&](int s) {
        return 6LL * (scenes[s].n_agents + scenes[s].n_static) + scenes[s].n_roads + 4LL * scenes[s].n_signals + 64;
    };
    auto scene_work = [&](int s) { return view_work(s) * (int64_t)scenes[s].n_agents * cfg->n_cams; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return scene_work(a) > scene_work(b); });
    std::vector<std::vector<int>> seg(gp::kQueues);
    std::vector<int64_t> load(gp::kQueues, 0);
    for (int s : order) {
        const int q = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        seg[q].push_back(s);
        load[q] += scene_work(s);
    }
    auto *queue = reinterpret_cast<int32_t *>(at(L.queue));
    int64_t qi = 0;
    for (int q = 0; q < gp::kQueues; ++q) {
        std::stable_sort(seg[q].begin(), seg[q].end(), [&](int a, int b) { return view_work(a) > view_work(b); });
        sim->dev.qseg[q] = (int32_t)qi;
        for (int s : seg[q]) {
            const gp::SceneRec &r = sim->scenes[s];
            for (int v = 0; v < r.n_agents * cfg->n_cams; ++v) queue[qi++] = r.view_base + v;
        }
    }
    sim->dev.qseg[gp::kQueues] = (int32_t)qi;
    // direct order: workgroup b (dispatched to XCD b mod kQueues) renders the
    // next view of segment b mod kQueues; once that segment is used up, the
    // next view of the segment with the most views left
    {
        auto *ord = reinterpret_cast<int32_t *>(at(L.order));
        std::vector<int64_t> next(gp::kQueues);
        for (int q = 0; q < gp::kQueues; ++q) next[q] = sim->dev.qseg[q];
        auto left = [&](int q) { return (int64_t)sim->dev.qseg[q + 1] - next[q]; };
        for (int64_t b = 0; b < L.n_views; ++b) {
            int q = (int)(b % gp::kQueues);
            if (left(q) == 0)
                for (int r = 0; r < gp::kQueues; ++r)
                    if (left(r) > left(q)) q = r;
            ord[b] = queue[next[q]++];
        }
    }

    // the device (everything above is host work on the host image)
    hipError_t e = hipGetDevice(&sim->device);
    if (e != hipSuccess) { delete sim; return hip_fail(e, "hipGetDevice"); }
    (void)hipDeviceGetAttribute(&sim->n_cu, hipDeviceAttributeMultiprocessorCount, sim->device);
    int lds = 0;
    (void)hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, sim->device);
    if (lds > 0) sim->max_lds = (size_t)lds;

    unsigned char *base = static_cast<unsigned char *>(d_workspace);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    e = hipMemcpyAsync(base, host.data(), (size_t)L.upload_end, hipMemcpyHostToDevice, hs);
    // the chip-wide raster's counters and coverage words start at zero
    if (e == hipSuccess && L.chip) e = hipMemsetAsync(base + L.chip_ctl, 0, (size_t)(L.chip_sbins - L.chip_ctl), hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) { delete sim; return hip_fail(e, "workspace upload"); }

    gp::DevSim &D = sim->dev;
    D.scenes = reinterpret_cast<const gp::SceneRec *>(base + L.scenes);
    D.views = reinterpret_cast<const gp::ViewRec *>(base + L.views);
    D.state = reinterpret_cast<float4 *>(base + L.state);
    D.cs = reinterpret_cast<float2 *>(base + L.cs);
    D.dims = reinterpret_cast<const float4 *>(base + L.dims);
    D.agent_color = base + L.agent_color;
    D.roads = reinterpret_cast<const float4 *>(base + L.roads);
    D.road_index = reinterpret_cast<const int32_t *>(base + L.road_index);
    D.road_color = base + L.road_color;
    D.bins = reinterpret_cast<const gp::RoadBin *>(base + L.bins);
    D.palette = base + L.palette;
    D.halted = base + L.halted;
    D.infr = base + L.infr;
    D.actu = reinterpret_cast<float4 *>(base + L.actu);
    D.signals = reinterpret_cast<const float4 *>(base + L.signals);
    D.signal_color = base + L.signal_color;
    D.queue = reinterpret_cast<const int32_t *>(base + L.queue);
    D.order = reinterpret_cast<const int32_t *>(base + L.order);
    D.counter = reinterpret_cast<uint32_t *>(base + L.counter);
    if (L.chip) {
        gp::ChipBufs &C = sim->chip;
        C.ctl = reinterpret_cast<uint32_t *>(base + L.chip_ctl);
        C.cov = reinterpret_cast<unsigned long long *>(base + L.chip_cov);
        C.sbins = reinterpret_cast<int32_t *>(base + L.chip_sbins);
        C.vinfo = reinterpret_cast<int4 *>(base + L.chip_vinfo);
        C.btri = base + L.chip_btri;
        C.rinfo = reinterpret_cast<int4 *>(base + L.chip_rinfo);
        C.rtri = base + L.chip_rtri;
        C.rrows = reinterpret_cast<int32_t *>(base + L.chip_rrows);
        C.rtri_cap = (int32_t)L.rtri_cap;
        C.items = reinterpret_cast<uint2 *>(base + L.chip_items);
        C.bins_stride = (int32_t)L.bins_stride;
        C.btri_cap = (int32_t)L.btri_cap;
        C.nw = (cfg->width + 63) / 64;
        C.rows_per_item = std::max(1, 64 / (cfg->width / 16));
        C.items_per_view = (cfg->height + C.rows_per_item - 1) / C.rows_per_item;
    }
    D.n_scenes = n_scenes;
    D.n_agents = (int32_t)L.n_agents;
    D.n_boxes = (int32_t)(L.n_agents + L.n_static);
    D.n_views = (int32_t)L.n_views;
    D.width = cfg->width;
    D.height = cfg->height;
    D.n_cams = cfg->n_cams;
    sim->road_uniform = uniform ? 1 : 0;
    // the rgb kernel needs unlit frames without traffic lights
    D.road_color_uniform = (sim->road_uniform && L.n_signals == 0) ? 1 : 0;
    D.shade = 0;
    D.road_color0 = color0 < 0 ? 0 : color0;
    for (int k = 0; k < gp::kMaxCams; ++k) {
        D.cam_dir[k][0] = cfg->cam_dir[k][0];
        D.cam_dir[k][1] = cfg->cam_dir[k][1];
    }
    D.focal = cfg->focal_px;
    D.cam_height = cfg->cam_height;
    D.z_near = cfg->z_near;
    D.z_far = cfg->z_far;
    D.dt = cfg->dt;
    // Road points project to row v = cy + h f / z.  Rows whose sample is below
    // the horizon and not more than 4 subpixels above the far line can show
    // road; the farthest depth they look at, plus 2% (>= 2.5 subpixels of
    // clearance at the nearest-to-horizon row), bounds every visible road point.
    {
        const double hf = (double)cfg->cam_height * (double)cfg->focal_px;
        const double v_far = hf / (double)cfg->z_far;
        const double cy = 0.5 * cfg->height;
        double zmax = 0.0;
        for (int j = 0; j < cfg->height; ++j) {
            const double dv = j + 0.5 - cy;
            if (dv > 0.0 && dv >= v_far - 4.0 / 256.0) zmax = std::max(zmax, hf / dv);
        }
        D.road_zmax = (float)(zmax * 1.02);
    }

    e = gp::launch_cs(D, 0, hs);
    if (e != hipSuccess) { delete sim; return hip_fail(e, "heading cosines"); }

    // default launch: persistent queue, a band buffer of at most 32 KB
    gp_launch l{};
    l.sched = GP_SCHED_PERSISTENT;
    l.band_rows = 64;
    while (l.band_rows > 8 && 8LL * l.band_rows * cfg->width > 32768) l.band_rows /= 2;
    l.batch_tris = 256;
    l.block_threads = 256;
    l.blocks_per_cu = 3;
    // rgb renders take the split rasteriser (two wavefronts per view, eight
    // views per CU) where it can run
    l.raster = GP_RASTER_BANDED;
    l.view_waves = 2;
    l.road_wgs_per_cu = 8;
    {
        // rgb renders: the wave-split raster where eight views fit a CU, else
        // the chip-wide passes where the image size allows them
        gp_launch t = l;
        t.raster = GP_RASTER_SPLIT;
        if (cfg->width % 16 == 0 && cfg->cam_height > 0.0f &&
            gp::rgb_lds_bytes(cfg->width, cfg->height, rgb_cfg(sim, t)) * 8 <= 160u * 1024u) {
            l.raster = GP_RASTER_SPLIT;
            l.blocks_per_cu = 8;
        } else if (L.chip && cfg->cam_height > 0.0f) {
            l.raster = GP_RASTER_CHIP;
        }
    }
    sim->launch = l;
    if (check_lds(sim, l) != GP_OK) { delete sim; return GP_EINVAL; }
    e = hipStreamCreateWithFlags(&sim->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) { delete sim; return hip_fail(e, "capture stream"); }
    *out = sim;
    return GP_OK;
}

gp_status gp_sim_set_launch(gp_sim *sim, const gp_launch *l)
{
    if (!sim || !l) return fail(GP_EINVAL, "NULL argument");
    if (!valid_launch(*l)) return fail(GP_EINVAL, "launch settings out of range");
    gp_status st = check_lds(sim, *l);
    if (st != GP_OK) return st;
    sim->launch = *l;
    return GP_OK;
}

gp_status gp_sim_get_launch(const gp_sim *sim, gp_launch *l)
{
    if (!sim || !l) return fail(GP_EINVAL, "NULL argument");
    *l = sim->launch;
    return GP_OK;
}

gp_status gp_sim_step(gp_sim *sim, const float *d_actions, void *stream)
{
    if (!sim || !d_actions) return fail(GP_EINVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(d_actions) % 8 != 0) return fail(GP_EINVAL, "actions must be 8-byte aligned");
    return step_impl(sim, d_actions, sim->launch, static_cast<hipStream_t>(stream));
}

gp_status gp_sim_render(gp_sim *sim, uint8_t *d_rgb, float *d_depth, int32_t *d_primid, void *stream)
{
    if (!sim || !d_rgb) return fail(GP_EINVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(d_rgb) % 4 != 0) return fail(GP_EINVAL, "rgb must be 4-byte aligned");
    if ((d_depth && reinterpret_cast<uintptr_t>(d_depth) % 4) || (d_primid && reinterpret_cast<uintptr_t>(d_primid) % 4))
        return fail(GP_EINVAL, "depth/primid must be 4-byte aligned");
    gp::RenderOut o{d_rgb, d_depth, d_primid};
    return render_impl(sim, o, sim->launch, static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace {

// The scratch of gp_sim_render_noalloc: the chip-wide raster's counters,
// coverage words, surviving-bin lists, box and road triangle lists and road
// items, in one file-scope device array instead of the sim's workspace.  Each
// GPU the library runs on holds its own copy until the process ends; every
// call on that GPU shares it.  In host code `scratch` names a host-side
// stand-in, not the device array: its device address is taken once per
// device with hipGetSymbolAddress, with that device current, and only that
// address is ever passed to kernels.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

gp_status scratch_of(int device, unsigned char **out)
{
    if (device < 0 || device >= kMaxDevices) return fail(GP_EINVAL, "device %d out of range", device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "address of the static scratch");
        g_scratch_ptr[device] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[device];
    return GP_OK;
}

}  // namespace

extern "C" {

gp_status gp_sim_render_noalloc(gp_sim *sim, uint8_t *d_rgb, void *stream)
{
    if (!sim || !d_rgb) return fail(GP_EINVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(d_rgb) % 16 != 0) return fail(GP_EINVAL, "rgb must be 16-byte aligned");
    if (!sim->lay.chip)
        return fail(GP_EINVAL, "image size %dx%d: the chip-wide raster needs width %% 16 == 0 and 64 <= width <= 1024",
                    sim->cfg.width, sim->cfg.height);
    if (!sim->dev.road_color_uniform)
        return fail(GP_EINVAL, "rgb renders of this sim need the general kernel (road colours, light or traffic lights)");
    if (sim->bins_cap > sim->lay.bins_stride) return fail(GP_EINVAL, "culling bins exceed the layout");
    const int64_t need = sim->lay.chip_end - sim->lay.chip_ctl;
    if (need > (int64_t)kNoAllocScratchBytes)
        return fail(GP_EINVAL, "this sim needs %lld bytes of scratch, the static buffer holds %lld",
                    (long long)need, (long long)kNoAllocScratchBytes);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != sim->device) return fail(GP_EINVAL, "the sim's device (%d) must be current (%d is)", sim->device, dev);
    unsigned char *base = nullptr;
    gp_status st = scratch_of(dev, &base);
    if (st != GP_OK) return st;
    const Layout &L = sim->lay;
    gp::ChipBufs C = sim->chip;
    C.ctl = reinterpret_cast<uint32_t *>(base);
    C.cov = reinterpret_cast<unsigned long long *>(base + (L.chip_cov - L.chip_ctl));
    C.sbins = reinterpret_cast<int32_t *>(base + (L.chip_sbins - L.chip_ctl));
    C.vinfo = reinterpret_cast<int4 *>(base + (L.chip_vinfo - L.chip_ctl));
    C.btri = base + (L.chip_btri - L.chip_ctl);
    C.rinfo = reinterpret_cast<int4 *>(base + (L.chip_rinfo - L.chip_ctl));
    C.rtri = base + (L.chip_rtri - L.chip_ctl);
    C.rrows = reinterpret_cast<int32_t *>(base + (L.chip_rrows - L.chip_ctl));
    C.items = reinterpret_cast<uint2 *>(base + (L.chip_items - L.chip_ctl));
    hipStream_t hs = static_cast<hipStream_t>(stream);
    // the previous call (maybe of another sim, with another layout) leaves
    // anything in the array: zero the counters and coverage words first
    e = gp::launch_chip_clear(C, (size_t)((L.chip_sbins - L.chip_cov) / 8), hs);
    if (e != hipSuccess) return hip_fail(e, "scratch clear");
    const gp::RenderOut o{d_rgb, nullptr, nullptr};
    e = gp::launch_render_chip(sim->dev, o, C, 1, 0, (int)L.n_views, std::max(1, sim->launch.road_wgs_per_cu) * sim->n_cu,
                               hs);
    if (e != hipSuccess) return hip_fail(e, "render launch");
    return GP_OK;
}

// sims of at most this many views step and render by direct launches
constexpr int64_t kGraphMinViews = 64;

gp_status gp_sim_step_render_graph(gp_sim *sim, const float *d_actions, uint8_t *d_rgb, void *stream)
{
    if (!sim || !d_actions || !d_rgb) return fail(GP_EINVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(d_rgb) % 4 != 0 || reinterpret_cast<uintptr_t>(d_actions) % 8 != 0)
        return fail(GP_EINVAL, "misaligned pointer");
    gp_launch l = sim->launch;
    l.sched = GP_SCHED_PERSISTENT;
    if (sim->lay.n_views <= kGraphMinViews) {
        // a few views render in less time than a graph replay costs on the
        // host: the step and the render are launched directly
        hipStream_t hs = static_cast<hipStream_t>(stream);
        gp_status st = step_impl(sim, d_actions, l, hs);
        if (st != GP_OK) return st;
        const gp::RenderOut o{d_rgb, nullptr, nullptr};
        return render_impl(sim, o, l, hs);
    }
    if (!sim->gexec || sim->g_rgb != d_rgb || !same_launch(l, sim->g_launch)) {
        // the step as an explicit kernel node (so that a new action buffer
        // only updates that node's arguments), then the render's kernels,
        // captured into the same graph behind it
        drop_graph(sim);
        hipGraph_t g = nullptr;
        hipError_t e = hipGraphCreate(&g, 0);
        if (e != hipSuccess) return hip_fail(e, "graph create");
        sim->graph = g;
        if (sim->lay.n_agents > 0) {
            e = gp::step_graph_node(g, nullptr, &sim->g_step, sim->dev, d_actions);
            if (e != hipSuccess) { drop_graph(sim); return hip_fail(e, "step node"); }
        }
        // the render's kernels captured into the same graph, after the step node
        e = hipStreamBeginCaptureToGraph(sim->capture_stream, g, sim->g_step ? &sim->g_step : nullptr, nullptr,
                                         sim->g_step ? 1 : 0, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) { drop_graph(sim); return hip_fail(e, "begin capture"); }
        gp::RenderOut o{d_rgb, nullptr, nullptr};
        gp_status st = render_impl(sim, o, l, sim->capture_stream);
        hipGraph_t rg = nullptr;
        e = hipStreamEndCapture(sim->capture_stream, &rg);
        if (st != GP_OK) { drop_graph(sim); return st; }
        if (e != hipSuccess) { drop_graph(sim); return hip_fail(e, "end capture"); }
        e = hipGraphInstantiate(&sim->gexec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) { drop_graph(sim); return hip_fail(e, "graph instantiate"); }
        sim->g_act = d_actions;
        sim->g_rgb = d_rgb;
        sim->g_launch = l;
    } else if (sim->g_act != d_actions) {
        if (sim->g_step) {
            hipError_t e = gp::step_graph_node(nullptr, sim->gexec, &sim->g_step, sim->dev, d_actions);
            if (e != hipSuccess) { drop_graph(sim); return hip_fail(e, "step node update"); }
        }
        sim->g_act = d_actions;
    }
    hipError_t e = hipGraphLaunch(sim->gexec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return GP_OK;
}

// ---- batched step + render over several sims (serving)

namespace {

struct BatchLayout {
    int64_t ctl, table, items, actions, total;
};

BatchLayout batch_layout(int32_t n_sims, int64_t n_agents, int64_t n_views)
{
    BatchLayout B{};
    int64_t o = 0;
    auto take = [&](int64_t bytes) { int64_t at = o; o = align_up(o + std::max<int64_t>(bytes, 1)); return at; };
    B.ctl = take(4 * 4);                                   // two queue heads + exit counters
    B.table = take((int64_t)sizeof(gp::SimEntry) * n_sims);
    B.items = take(8 * n_views);
    B.actions = take(8 * n_agents);
    B.total = o;
    return B;
}

}  // namespace

int64_t gp_batch_required_bytes(int32_t n_sims, int64_t n_agents, int64_t n_views)
{
    if (n_sims < 1 || n_agents < 0 || n_views < 0) return -1;
    return batch_layout(n_sims, n_agents, n_views).total;
}

gp_status gp_batch_step_render(gp_sim *const *sims, int32_t n_sims, const float *const *h_actions,
                               uint8_t *const *d_rgb, void *d_ws, int64_t ws_bytes, void *h_staging,
                               int64_t staging_bytes, void *stream)
{
    if (!sims || !h_actions || !d_rgb || !d_ws || !h_staging) return fail(GP_EINVAL, "NULL argument");
    if (n_sims < 1) return fail(GP_EINVAL, "n_sims must be >= 1");
    if (reinterpret_cast<uintptr_t>(d_ws) % kAlign != 0 || reinterpret_cast<uintptr_t>(h_staging) % 16 != 0)
        return fail(GP_EINVAL, "batch workspace must be %lld-byte aligned, staging 16-byte aligned",
                    (long long)kAlign);
    int64_t n_agents = 0, n_views = 0;
    int max_agents = 0;
    for (int k = 0; k < n_sims; ++k) {
        const gp_sim *sim = sims[k];
        if (!sim || !h_actions[k] || !d_rgb[k]) return fail(GP_EINVAL, "NULL entry %d", k);
        if (reinterpret_cast<uintptr_t>(d_rgb[k]) % 4 != 0) return fail(GP_EINVAL, "rgb %d must be 4-byte aligned", k);
        if (sim->cfg.width != sims[0]->cfg.width || sim->cfg.height != sims[0]->cfg.height)
            return fail(GP_EINVAL, "every sim of a batch must have the same image size");
        if (sim->device != sims[0]->device) return fail(GP_EINVAL, "every sim of a batch must be on one device");
        for (int j = 0; j < k; ++j)
            if (sims[j] == sim) return fail(GP_EINVAL, "sim %d appears twice in the batch", k);
        n_agents += sim->lay.n_agents;
        n_views += sim->lay.n_views;
        max_agents = std::max<int>(max_agents, (int)sim->lay.n_agents);
    }
    const BatchLayout B = batch_layout(n_sims, n_agents, n_views);
    if (ws_bytes < B.total || staging_bytes < B.total)
        return fail(GP_ENOMEM, "batch needs %lld bytes of workspace and staging", (long long)B.total);
    if (n_views > INT32_MAX) return fail(GP_EINVAL, "too many views in one batch");

    // host image of the batch buffer: zeroed queue counters, the sim table,
    // the (sim, view) items (rgb-kernel sims first), the packed actions
    unsigned char *h = static_cast<unsigned char *>(h_staging);
    unsigned char *d = static_cast<unsigned char *>(d_ws);
    std::memset(h + B.ctl, 0, 16);
    auto *tab = reinterpret_cast<gp::SimEntry *>(h + B.table);
    auto *items = reinterpret_cast<int32_t *>(h + B.items);
    auto *act = reinterpret_cast<float *>(h + B.actions);
    int64_t a0 = 0, n_fast = 0;
    bool lights = false;          // the general launch takes the instances with traffic lights
    for (int k = 0; k < n_sims; ++k) {
        const gp_sim *sim = sims[k];
        gp::SimEntry e{};
        e.s = sim->dev;
        e.o = gp::RenderOut{d_rgb[k], nullptr, nullptr};
        e.act = reinterpret_cast<const float2 *>(d + B.actions + 8 * a0);
        std::memcpy(&tab[k], &e, sizeof(e));
        std::memcpy(act + 2 * a0, h_actions[k], 8 * (size_t)sim->lay.n_agents);
        a0 += sim->lay.n_agents;
        if (sim->dev.road_color_uniform) n_fast += sim->lay.n_views;
        lights = lights || sim->lay.n_signals > 0;
    }
    int64_t qf = 0, qg = n_fast;
    for (int k = 0; k < n_sims; ++k) {
        const gp_sim *sim = sims[k];
        int64_t &q = sim->dev.road_color_uniform ? qf : qg;
        for (int64_t v = 0; v < sim->lay.n_views; ++v) {
            items[2 * q] = k;
            items[2 * q + 1] = (int32_t)v;
            ++q;
        }
    }
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(d, h, (size_t)B.total, hipMemcpyHostToDevice, hs);
    if (e != hipSuccess) return hip_fail(e, "batch upload");
    const auto *dtab = reinterpret_cast<const gp::SimEntry *>(d + B.table);
    const auto *ditems = reinterpret_cast<const int2 *>(d + B.items);
    auto *ctl = reinterpret_cast<uint32_t *>(d + B.ctl);
    e = gp::launch_step_multi(dtab, n_sims, max_agents, hs);
    if (e != hipSuccess) return hip_fail(e, "batch step launch");
    const gp_launch &l = sims[0]->launch;
    const gp::LaunchCfg c = launch_cfg(l);
    const int W = sims[0]->cfg.width, H = sims[0]->cfg.height;
    for (int fast = 1; fast >= 0; --fast) {
        const int64_t n = fast ? n_fast : n_views - n_fast;
        if (n == 0) continue;
        if (gp::render_lds_bytes(W, H, c, fast) > sims[0]->max_lds)
            return fail(GP_EINVAL, "launch setting needs more LDS than the device has");
        const int grid = (int)std::min<int64_t>(n, (int64_t)l.blocks_per_cu * sims[0]->n_cu);
        e = gp::launch_render_multi(dtab, ditems + (fast ? 0 : n_fast), (int)n, ctl + (fast ? 0 : 2), c,
                                    fast ? 1 : (lights ? 2 : 0), W, H, grid, hs);
        if (e != hipSuccess) return hip_fail(e, "batch render launch");
    }
    return GP_OK;
}

gp_status gp_sim_get_state(gp_sim *sim, float *d_dst, void *stream)
{
    if (!sim || !d_dst) return fail(GP_EINVAL, "NULL argument");
    hipError_t e = hipMemcpyAsync(d_dst, sim->dev.state, 16 * (size_t)sim->lay.n_agents,
                                  hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GP_OK : hip_fail(e, "get_state copy");
}

gp_status gp_sim_set_state(gp_sim *sim, const float *d_src, void *stream)
{
    if (!sim || !d_src) return fail(GP_EINVAL, "NULL argument");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(sim->dev.state, d_src, 16 * (size_t)sim->lay.n_agents,
                                  hipMemcpyDeviceToDevice, hs);
    if (e != hipSuccess) return hip_fail(e, "set_state copy");
    e = gp::launch_cs(sim->dev, 1, hs);
    return e == hipSuccess ? GP_OK : hip_fail(e, "heading cosines");
}

gp_status gp_sim_set_light(gp_sim *sim, const float *h_light)
{
    if (!sim) return fail(GP_EINVAL, "NULL argument");
    if (h_light) {
        for (int k = 0; k < 4; ++k)
            if (!std::isfinite(h_light[k])) return fail(GP_EINVAL, "light not finite");
        const double n = std::sqrt((double)h_light[0] * h_light[0] + (double)h_light[1] * h_light[1] +
                                   (double)h_light[2] * h_light[2]);
        if (std::fabs(n - 1.0) > 1e-3) return fail(GP_EINVAL, "light direction is not a unit vector (norm %g)", n);
        if (!(h_light[3] >= 0.0f && h_light[3] <= 1.0f)) return fail(GP_EINVAL, "ambient outside [0, 1]");
    }
    drop_graph(sim);            // a captured graph holds the old kernel arguments
    sim->dev.shade = h_light ? 1 : 0;
    for (int k = 0; k < 4; ++k) sim->dev.light[k] = h_light ? h_light[k] : 0.0f;
    // lit frames are resolved by the general kernel
    sim->dev.road_color_uniform = (sim->road_uniform && !h_light && sim->lay.n_signals == 0) ? 1 : 0;
    return GP_OK;
}

gp_status gp_sim_render_raycast(gp_sim *sim, uint8_t *d_rgb, float *d_depth, int32_t *d_primid, void *stream)
{
    if (!sim || !d_rgb) return fail(GP_EINVAL, "NULL argument");
    if (gp::raycast_lds_bytes() > sim->max_lds) return fail(GP_EINVAL, "ray caster needs more LDS than the device has");
    gp::RenderOut o{d_rgb, d_depth, d_primid};
    hipError_t e = gp::launch_raycast(sim->dev, o, 0, (int)sim->lay.n_views, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GP_OK : hip_fail(e, "ray-cast launch");
}

gp_status gp_sim_set_signal_colors(gp_sim *sim, const uint8_t *d_colors, void *stream)
{
    if (!sim || !d_colors) return fail(GP_EINVAL, "NULL argument");
    if (sim->lay.n_signals == 0) return GP_OK;
    hipError_t e = hipMemcpyAsync(sim->dev.signal_color, d_colors, (size_t)sim->lay.n_signals,
                                  hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GP_OK : hip_fail(e, "set_signal_colors copy");
}

int64_t gp_sim_num_signals(const gp_sim *sim) { return sim ? sim->lay.n_signals : -1; }

gp_status gp_sim_step_jerk(gp_sim *sim, const uint8_t *d_actions, void *stream)
{
    if (!sim || !d_actions) return fail(GP_EINVAL, "NULL argument");
    hipError_t e = gp::launch_step_jerk(sim->dev, d_actions, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GP_OK : hip_fail(e, "jerk step launch");
}

gp_status gp_sim_get_actuators(gp_sim *sim, float *d_dst, void *stream)
{
    if (!sim || !d_dst) return fail(GP_EINVAL, "NULL argument");
    hipError_t e = hipMemcpyAsync(d_dst, sim->dev.actu, 16 * (size_t)sim->lay.n_agents,
                                  hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GP_OK : hip_fail(e, "get_actuators copy");
}

gp_status gp_sim_check_infractions(gp_sim *sim, uint8_t *d_flags, void *stream)
{
    if (!sim) return fail(GP_EINVAL, "NULL argument");
    int max_agents = 0;
    for (const gp::SceneRec &r : sim->scenes) max_agents = std::max(max_agents, r.n_agents);
    hipError_t e = gp::launch_infractions(sim->dev, max_agents, d_flags, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? GP_OK : hip_fail(e, "infraction check launch");
}

gp_status gp_sim_fork(gp_sim *dst, const gp_sim *src, void *stream)
{
    if (!dst || !src) return fail(GP_EINVAL, "NULL argument");
    if (dst == src) return GP_OK;
    if (dst->n_scenes != src->n_scenes) return fail(GP_EINVAL, "fork needs sims over the same scenes");
    for (int k = 0; k < src->n_scenes; ++k)
        if (dst->scenes[k].n_agents != src->scenes[k].n_agents || dst->scenes[k].n_roads != src->scenes[k].n_roads ||
            dst->scenes[k].n_static != src->scenes[k].n_static || dst->scenes[k].n_signals != src->scenes[k].n_signals)
            return fail(GP_EINVAL, "fork needs sims over the same scenes (scene %d differs)", k);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const size_t n = (size_t)src->lay.n_agents;
    hipError_t e = hipMemcpyAsync(dst->dev.state, src->dev.state, 16 * n, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(dst->dev.cs, src->dev.cs, 8 * n, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(dst->dev.halted, src->dev.halted, n, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(dst->dev.actu, src->dev.actu, 16 * n, hipMemcpyDeviceToDevice, hs);
    if (e == hipSuccess && src->lay.n_signals > 0)
        e = hipMemcpyAsync(dst->dev.signal_color, src->dev.signal_color, (size_t)src->lay.n_signals,
                           hipMemcpyDeviceToDevice, hs);
    return e == hipSuccess ? GP_OK : hip_fail(e, "fork copy");
}

int64_t gp_sim_num_views(const gp_sim *sim) { return sim ? sim->lay.n_views : -1; }
int64_t gp_sim_num_agents(const gp_sim *sim) { return sim ? sim->lay.n_agents : -1; }
int32_t gp_sim_num_scenes(const gp_sim *sim) { return sim ? sim->n_scenes : -1; }

void gp_sim_destroy(gp_sim *sim)
{
    if (!sim) return;
    drop_graph(sim);
    if (sim->capture_stream) (void)hipStreamDestroy(sim->capture_stream);
    delete sim;
}

}  // extern "C"
