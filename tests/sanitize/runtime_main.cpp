// Driver for an AddressSanitizer / UndefinedBehaviorSanitizer build of the
// library's host code: argument checks, workspace layout, the Morton sort of
// road strips into culling bins, the view queue and the direct order.  On a
// machine without a GPU gp_sim_create runs all of that on its host image and
// then fails at the device query (GP_EDEVICE); with a GPU it succeeds and the
// sim is destroyed again.  Built and run by tests/test_sanitize.py.
#include "../../include/gp.h"

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

namespace {

uint64_t lcg = 0x5EED0F00ull;
float urand(float lo, float hi)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return lo + (hi - lo) * (float)((lcg >> 40) * (1.0 / 16777216.0));
}

struct HostScene {
    std::vector<float> state, dims, roads, sxp, sdm, sig;
    std::vector<uint8_t> acol, rcol, scol, gcol;
    gp_scene_desc d{};
};

HostScene make(int na, int nr, int ns, int ng, float extent)
{
    HostScene h;
    for (int a = 0; a < na; ++a) {
        h.state.insert(h.state.end(), {urand(-extent, extent), urand(-extent, extent), urand(-3.2f, 3.2f), urand(0, 20)});
        h.dims.insert(h.dims.end(), {urand(4.0f, 5.5f), urand(1.8f, 2.2f), urand(1.4f, 2.0f)});
        h.acol.push_back(2);
    }
    for (int q = 0; q < nr; ++q) {
        const float cx = urand(-extent, extent), cy = urand(-extent, extent), hx = urand(0.5f, 30.0f), hy = 1.75f;
        h.roads.insert(h.roads.end(), {cx - hx, cy - hy, cx + hx, cy - hy, cx + hx, cy + hy, cx - hx, cy + hy});
        h.rcol.push_back(1);
    }
    for (int k = 0; k < ns; ++k) {
        h.sxp.insert(h.sxp.end(), {urand(-extent, extent), urand(-extent, extent), urand(-3, 3)});
        h.sdm.insert(h.sdm.end(), {urand(1, 6), urand(0.5f, 2.2f), urand(0.8f, 2)});
        h.scol.push_back(3);
    }
    for (int g = 0; g < ng; ++g) {
        h.sig.insert(h.sig.end(), {urand(-extent, extent), urand(-extent, extent), urand(3.5f, 5.5f), urand(0.25f, 0.4f)});
        h.gcol.push_back(4);
    }
    h.d.n_agents = na;
    h.d.n_roads = nr;
    h.d.agent_state = h.state.data();
    h.d.agent_dims = h.dims.data();
    h.d.agent_color = h.acol.data();
    h.d.road_xy = h.roads.data();
    h.d.road_color = h.rcol.data();
    h.d.n_static = ns;
    h.d.static_xyp = ns ? h.sxp.data() : nullptr;
    h.d.static_dims = ns ? h.sdm.data() : nullptr;
    h.d.static_color = ns ? h.scol.data() : nullptr;
    h.d.n_signals = ng;
    h.d.signal_xyzr = ng ? h.sig.data() : nullptr;
    h.d.signal_color = ng ? h.gcol.data() : nullptr;
    return h;
}

gp_config config(int w, int h, int cams)
{
    gp_config c{};
    c.width = w;
    c.height = h;
    c.n_cams = cams;
    const float dirs[4][2] = {{1, 0}, {0.5f, 0.8660254f}, {0.5f, -0.8660254f}, {-1, 0}};
    for (int k = 0; k < GP_MAX_CAMS; ++k) {
        c.cam_dir[k][0] = dirs[k][0];
        c.cam_dir[k][1] = dirs[k][1];
    }
    c.focal_px = 0.5f * (float)w;
    c.cam_height = 1.6f;
    c.z_near = 0.5f;
    c.z_far = 100.0f;
    c.dt = 0.1f;
    for (int i = 0; i < 256 * 3; ++i) c.palette[i / 3][i % 3] = (uint8_t)i;
    return c;
}

int failures = 0;
void expect(bool ok, const char *what)
{
    if (!ok) {
        std::printf("FAILED: %s (%s)\n", what, gp_last_error());
        ++failures;
    }
}

// layout and creation of one set of scenes; returns the workspace size
int64_t create(const gp_config &c, std::vector<HostScene> &hs)
{
    std::vector<gp_scene_desc> d;
    for (auto &h : hs) d.push_back(h.d);
    const int64_t need = gp_sim_required_bytes(&c, d.data(), (int32_t)d.size());
    expect(need > 0, "required bytes");
    if (need <= 0) return need;
    void *ws = std::aligned_alloc(256, (size_t)((need + 255) / 256 * 256));
    gp_sim *sim = nullptr;
    const gp_status st = gp_sim_create(&c, d.data(), (int32_t)d.size(), ws, need, nullptr, &sim);
    expect(st == GP_OK || st == GP_EDEVICE, "create runs its host work and stops only at the device");
    // a workspace one byte short is refused before anything else
    gp_sim *s2 = nullptr;
    expect(gp_sim_create(&c, d.data(), (int32_t)d.size(), ws, need - 1, nullptr, &s2) == GP_ENOMEM, "short workspace");
    if (sim) gp_sim_destroy(sim);
    std::free(ws);
    return need;
}

}  // namespace

int main()
{
    // ordinary scenes, uneven ones, scenes without roads, strip counts around
    // the bin size, static obstacles and traffic lights, several image shapes
    {
        std::vector<HostScene> hs;
        hs.push_back(make(8, 200, 0, 0, 100));
        hs.push_back(make(1, 0, 0, 0, 100));
        hs.push_back(make(3, 1, 2, 1, 100));
        hs.push_back(make(5, 15, 0, 0, 30));
        hs.push_back(make(5, 16, 0, 0, 30));
        hs.push_back(make(5, 17, 1, 0, 30));
        hs.push_back(make(128, 8000, 8, 12, 100));
        create(config(128, 128, 3), hs);
        create(config(210, 126, 4), hs);
        create(config(1, 1, 1), hs);
        create(config(1024, 1024, 1), hs);
    }
    {
        // every strip on one point of the map (one Morton code) and far apart
        std::vector<HostScene> hs;
        hs.push_back(make(4, 300, 0, 0, 0.0f));
        hs.push_back(make(4, 300, 0, 0, 1.0e6f));
        create(config(64, 64, 1), hs);
    }
    // argument checks
    {
        std::vector<HostScene> hs;
        hs.push_back(make(4, 10, 0, 0, 100));
        gp_scene_desc d = hs[0].d;
        gp_config c = config(64, 64, 1);
        expect(gp_sim_required_bytes(nullptr, &d, 1) == -1, "NULL config");
        expect(gp_sim_required_bytes(&c, nullptr, 1) == -1, "NULL scenes");
        expect(gp_sim_required_bytes(&c, &d, 0) == -1, "no scenes");
        gp_config bad = c;
        bad.width = 0;
        expect(gp_sim_required_bytes(&bad, &d, 1) == -1, "zero width");
        bad = c;
        bad.n_cams = 5;
        expect(gp_sim_required_bytes(&bad, &d, 1) == -1, "too many cameras");
        bad = c;
        bad.z_far = NAN;
        expect(gp_sim_required_bytes(&bad, &d, 1) == -1, "NaN far plane");
        bad = c;
        bad.cam_dir[0][1] = INFINITY;
        expect(gp_sim_required_bytes(&bad, &d, 1) == -1, "infinite camera direction");
        gp_scene_desc e = d;
        e.n_agents = 0;
        expect(gp_sim_required_bytes(&c, &e, 1) == -1, "no agents");
        e = d;
        e.n_roads = -1;
        expect(gp_sim_required_bytes(&c, &e, 1) == -1, "negative strips");
        e = d;
        e.agent_state = nullptr;
        expect(gp_sim_required_bytes(&c, &e, 1) == -1, "NULL agent state");
        e = d;
        e.n_static = 2;
        expect(gp_sim_required_bytes(&c, &e, 1) == -1, "static count without arrays");
        std::vector<float> nan_state = hs[0].state;
        nan_state[1] = NAN;
        e = d;
        e.agent_state = nan_state.data();
        const int64_t r = gp_sim_required_bytes(&c, &e, 1);
        expect(r == -1 || r > 0, "non-finite agent state: refused or accepted, never undefined");
        gp_sim *sim = nullptr;
        expect(gp_sim_create(&c, &d, 1, nullptr, 1 << 20, nullptr, &sim) == GP_EINVAL, "NULL workspace");
        expect(gp_sim_create(&c, &d, 1, reinterpret_cast<void *>(uintptr_t(0x1001)), 1 << 20, nullptr, &sim) ==
                   GP_EINVAL,
               "unaligned workspace");
        expect(gp_sim_create(&c, &d, 1, nullptr, 0, nullptr, nullptr) == GP_EINVAL, "NULL out");
    }
    expect(gp_batch_required_bytes(4, 100, 300) > 0, "batch bytes");
    expect(gp_batch_required_bytes(0, 100, 300) == -1, "batch of no sims");
    expect(gp_batch_required_bytes(4, -1, 300) == -1, "negative agents");
    if (failures == 0) std::printf("runtime sanitize driver ok\n");
    return failures == 0 ? 0 : 1;
}
