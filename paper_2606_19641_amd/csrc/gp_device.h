// Device-side data layout shared by the kernels and the host runtime of the
// Gigapixel hot path.  Everything here describes memory inside the caller's
// workspace; no pointer is owned by the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gp {

constexpr int kMaxCams = 4;

// Per-scene record: first agent, agent count, first road, road count, first view.
struct SceneRec {
    int32_t agent_base, n_agents, road_base, n_roads;
    int32_t view_base, pad0, pad1, pad2;
};

// One view: scene index and (ego agent local index, camera index).
struct ViewRec {
    int32_t scene;
    int32_t ego_cam;   // ego * 4 + cam
};

// Everything a kernel needs, passed by value.
struct DevSim {
    const SceneRec *scenes;
    const ViewRec *views;
    float4 *state;            // [A] x, y, psi, v
    float2 *cs;               // [A] cos psi, sin psi
    const float4 *dims;       // [A] L, W, H, 0
    const uint8_t *agent_color;
    const float4 *roads;      // [R][2] corners (x0 y0 x1 y1) (x2 y2 x3 y3)
    const uint8_t *road_color;
    const uint8_t *palette;   // [256*3]
    const int32_t *queue;     // [V] view order for the persistent schedule
    uint32_t *counter;        // work-queue head
    int32_t n_scenes, n_agents, n_views;
    int32_t width, height, n_cams;
    float cam_dir[kMaxCams][2];
    float focal, cam_height, z_near, z_far, dt;
};

struct RenderOut {
    uint8_t *rgb;
    float *depth;
    int32_t *primid;
};

struct LaunchCfg {
    int band_rows;
    int batch_tris;
    int block_threads;
};

// Host-side launch helpers (defined in gp_kernels.hip).
hipError_t launch_step(const DevSim &s, const float *actions, int agent_begin, int agent_count,
                       hipStream_t st);
hipError_t launch_cs(const DevSim &s, hipStream_t st);
hipError_t launch_reset_counter(const DevSim &s, hipStream_t st);
hipError_t launch_render(const DevSim &s, const RenderOut &o, const LaunchCfg &c, int persistent,
                         int view_begin, int grid, hipStream_t st);
size_t render_lds_bytes(const DevSim &s, const LaunchCfg &c);

}  // namespace gp
