// Device-side data layout shared by the kernels and the host runtime of the
// Gigapixel hot path.  Everything here describes memory inside the caller's
// workspace; no pointer is owned by the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gp {

constexpr int kMaxCams = 4;
constexpr int kBinQuads = 16;            // road strips per culling bin
constexpr int kMaxPrims = 1 << 23;       // primitives per scene (key packs 23 bits)
constexpr int kQueues = 8;               // work-queue segments, one per XCD of the MI355X
// Spacing of the queue's counters in 32-bit words: one counter per 256 bytes.
// Device-scope atomics on one cache line serialise (about 12 ns each on the
// MI355X), on distinct lines they proceed in parallel.
constexpr int kCtrStride = 64;

// Per-scene record.
struct SceneRec {
    int32_t agent_base, n_agents;   // agents [agent_base, agent_base + n_agents)
    int32_t road_base, n_roads;     // road slots [road_base, road_base + n_roads)
    int32_t view_base;              // first view of the scene
    int32_t bin_base, n_bins;       // culling bins [bin_base, bin_base + n_bins)
    int32_t static_base, n_static;  // static obstacles: box slots [static_base, static_base + n_static)
    int32_t signal_base, n_signals; // traffic lights [signal_base, signal_base + n_signals)
};

// Box b of a scene (the agents, then the static obstacles) -> its slot in the
// box arrays (state, cs, dims, agent_color): every agent first, then every
// static obstacle.
__host__ __device__ inline int box_slot(const SceneRec &sc, int b)
{
    return b < sc.n_agents ? sc.agent_base + b : sc.static_base + (b - sc.n_agents);
}

// One view: scene index and (ego agent local index, camera index).
struct ViewRec {
    int32_t scene;
    int32_t ego_cam;   // ego * 4 + cam
};

// Road culling bin: bounding box of up to kBinQuads consecutive road slots.
struct RoadBin {
    float xmin, ymin, xmax, ymax;
    int32_t start, count;           // slot range, relative to the scene's road_base
    int32_t pad0, pad1;
};

// Everything a kernel needs, passed by value.
struct DevSim {
    const SceneRec *scenes;
    const ViewRec *views;
    float4 *state;            // [A + S] x, y, psi, v: the A agents, then the S static obstacles (v = 0)
    float2 *cs;               // [A + S] cos psi, sin psi
    const float4 *dims;       // [A + S] L, W, H, 0
    const uint8_t *agent_color;   // [A + S]
    const float4 *roads;      // [R][2] corners of road slot r: (x0 y0 x1 y1) (x2 y2 x3 y3)
    const int32_t *road_index;// [R] index of road slot r in its scene's input order
    const uint8_t *road_color;// [R] colour of road slot r
    const RoadBin *bins;
    const uint8_t *palette;   // [256*3]
    const int32_t *queue;     // [V] view order for the persistent schedule, kQueues segments
    const int32_t *order;     // [V] view of workgroup b when every view has a workgroup: consecutive
                              // workgroups (which go to the XCDs in turn) take the segments in turn
    uint32_t *counter;        // [(kQueues + 2) * kCtrStride] segment heads, finished workgroups,
                              // exhausted segment mask, kCtrStride words apart (all zero
                              // between launches)
    int32_t qseg[kQueues + 1];// segment q of the queue is [qseg[q], qseg[q + 1])
    int32_t n_scenes, n_agents, n_views;
    int32_t n_boxes;          // A + S
    int32_t width, height, n_cams;
    int32_t road_color_uniform;   // 1 if every road strip has the colour road_color0
    int32_t road_color0;
    float road_zmax;          // no pixel sample sees the road plane beyond this depth
    uint8_t *halted;          // [A] 1 once the agent committed an infraction (frozen in place)
    uint8_t *infr;            // [A] infractions found by the last check (bit 0 collision, 1 off-road)
    float4 *actu;             // [A] jerk actuators: a_lon, a_lat, steering angle, 0
    const float4 *signals;    // [G] traffic lights: x, y, z (centre), radius
    uint8_t *signal_color;    // [G] palette index of each light's state
    float cam_dir[kMaxCams][2];
    float focal, cam_height, z_near, z_far, dt;
    float light[4];           // unit direction towards the light (world frame), ambient
    int32_t shade;            // 1: faces lit by the directional light
};

struct RenderOut {
    uint8_t *rgb;
    float *depth;
    int32_t *primid;
};

// One sim of a batched (serving) launch.
struct SimEntry {
    DevSim s;
    RenderOut o;
    const float2 *act;        // the sim's actions [n_agents] (accel, steer)
    const void *pad;
};

struct LaunchCfg {
    int band_rows;
    int batch_tris;
    int block_threads;
};

// Settings of the wave-split rgb raster (gp_raster.hip).
struct RgbCfg {
    int waves;        // wavefronts per view: 1, 2 or 4
    int bcap;         // box triangles one view's list holds
    int bins_cap;     // culling bins of the largest scene (surviving bins are listed in LDS)
};

// Buffers of the chip-wide rgb raster (gp_chip.hip), all inside the
// workspace.  The coverage words and the counters are zero between renders.
enum { CHIP_NITEMS = 0, CHIP_NCTL = 8 };
struct ChipBufs {
    unsigned long long *cov;  // [V][H][nw] road coverage: bit i of word w of a row is sample 64 w + i
    int32_t *sbins;           // [V][bins_stride] surviving culling bins: start * 128 + count
    int4 *vinfo;              // [V] surviving bins, box triangles (-1: the list overflowed), box rows min, max
    void *btri;               // [V][btri_cap] the view's box triangles (TriRec)
    int4 *rinfo;              // [V] road triangles appended (may pass rtri_cap), coverage words used, 0, 0
    void *rtri;               // [V][rtri_cap] the view's road triangles (TriGeo)
    int32_t *rrows;           // [V][rtri_cap] their sample rows j0 | j1 << 16
    uint2 *items;             // road work items (view, unit of four surviving bins)
    uint32_t *ctl;            // [CHIP_NCTL] road item count (the others unused)
    int32_t bins_stride, btri_cap, rtri_cap, nw, rows_per_item, items_per_view;
};

// Host-side launch helpers (defined in gp_kernels.hip and gp_raster.hip).
hipError_t launch_step(const DevSim &s, const float *actions, int agent_begin, int agent_count,
                       hipStream_t st);
// The direct step of every agent as a graph kernel node: added to g when exec
// is null (the node returned in *node), else the arguments of *node in the
// instantiated graph exec replaced (a new action buffer, no re-capture).
hipError_t step_graph_node(hipGraph_t g, hipGraphExec_t exec, hipGraphNode_t *node, const DevSim &s,
                           const float *actions);
// clear_halted = 1 also clears the halted flags and the jerk actuators
hipError_t launch_cs(const DevSim &s, int clear_halted, hipStream_t st);
// jerk-actuated step of every agent; actions [A] uint8 indices 0..11
hipError_t launch_step_jerk(const DevSim &s, const uint8_t *actions, hipStream_t st);
// infraction check of every agent; flags_out (optional) [A] gets bit 0
// collision, bit 1 off-road, bit 2 halted after the check
hipError_t launch_infractions(const DevSim &s, int max_agents, uint8_t *flags_out, hipStream_t st);
// kind 1: rgb-only kernel for a uniform road colour; 0: general kernel;
// 2: general kernel with traffic lights
hipError_t launch_render(const DevSim &s, const RenderOut &o, const LaunchCfg &c, int kind,
                         int persistent, int view_begin, int grid, hipStream_t st);
size_t render_lds_bytes(const DevSim &s, const LaunchCfg &c, int fast);
size_t render_lds_bytes(int width, int height, const LaunchCfg &c, int fast);
// ray-cast backend (gp_raycast.hip): one workgroup per view of [view_begin, view_begin + n_views)
hipError_t launch_raycast(const DevSim &s, const RenderOut &o, int view_begin, int n_views, hipStream_t st);
size_t raycast_lds_bytes();
// wave-split rgb raster (gp_raster.hip) for uniform road colours, no depth /
// primitive id, width a multiple of 16 and a 16-byte aligned image.
// mode 0: workgroup b renders view view_begin + b; 1: view order[b]; 2: the
// persistent work queue
hipError_t launch_render_rgb(const DevSim &s, const RenderOut &o, const RgbCfg &c, int mode, int view_begin,
                             int grid, hipStream_t st);
size_t rgb_lds_bytes(int width, int height, const RgbCfg &c);
// chip-wide rgb raster (gp_chip.hip), same conditions as the wave-split one
// plus 64 <= width <= 1024: the setup pass over views [view_begin,
// view_begin + n_views) (mode 0) or every view in order[] (mode 1), the road
// pass on road_grid workgroups, the resolve pass on a workgroup per group of
// sixteen tiles of a view
hipError_t launch_render_chip(const DevSim &s, const RenderOut &o, const ChipBufs &cb, int mode, int view_begin,
                              int n_views, int road_grid, hipStream_t st);
// zero the chip-wide raster's counters and the first cov_words coverage words
hipError_t launch_chip_clear(const ChipBufs &cb, size_t cov_words, hipStream_t st);
// batched (serving) launches over a device table of sims
hipError_t launch_step_multi(const SimEntry *tab, int n_sims, int max_agents, hipStream_t st);
hipError_t launch_render_multi(const SimEntry *tab, const int2 *items, int n_items, uint32_t *ctl,
                               const LaunchCfg &c, int kind, int width, int height, int grid, hipStream_t st);

}  // namespace gp
