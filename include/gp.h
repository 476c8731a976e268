/*
 * gp.h -- C ABI of the Gigapixel hot path on MI355X (gfx950).
 *
 * The library advances a batch of driving scenes with a kinematic agent step
 * and renders, for every agent, an ego-centric perspective view of a
 * bounding-box world (agent cuboids plus flat road strips) into a uint8 RGB
 * image that stays on the GPU.
 *
 * Paper passages (Gigapixel, "Scaling Self-Play for End-to-End Driving"):
 *   - Sec. 3.1: the state S_t = (A_t, M, L_t) of agent boxes and map polylines;
 *     O_pixel(S_t) renders S_t into an ego-centric perspective view on a
 *     batched GPU renderer; agents are cuboids and lane polylines are thin
 *     planar strips.
 *   - App. A, "High-Throughput Batched Rendering": one world per ego agent,
 *     all worlds rendered together in one batched launch; per-instance colour;
 *     images exposed to the learner as a GPU tensor with no per-step CPU
 *     transfer; image resolution and the camera set are configurable.
 *   - App. A, "Action Space and Dynamics": kinematic bicycle with the
 *     wheelbase at 60% of the vehicle length and clipped acceleration, speed
 *     and steering; App. B (student hyper-parameters): dt = 0.1 s.
 * The paper fixes no numeric conventions of the raster or the dynamics
 * constants.  The conventions implemented (documented with each call below):
 *   camera at the ego box centre, 1.6 m high, pitch 0; planar depth; pixel
 *   samples at pixel centres, row 0 at the top; vertices snapped to 1/256
 *   pixel (round half to even); top-left fill rule; box faces one-sided, road
 *   strips two-sided; near/far clip at z_near/z_far; per-pixel winner = the
 *   largest (1/z, agent-above-road, lower primitive index); the ego's own box
 *   is not drawn; acceleration in [-6, 3] m/s^2, steering in [-0.5, 0.5] rad,
 *   speed in [0, 30] m/s; project-owned sin/cos.
 *
 * Conventions of the ABI:
 *   - Every device pointer argument is a plain device address (e.g. a torch
 *     tensor's data_ptr()); every `stream` is a hipStream_t (NULL = default).
 *   - Ownership: the caller owns all device memory, including the workspace
 *     handed to gp_sim_create.  The library allocates no device memory; it
 *     keeps only a small host-side handle.
 *   - Calls are stream-ordered and return without synchronising the host.
 *     The returned status reports argument and launch errors; a device fault
 *     surfaces as GP_EDEVICE on a later call.
 *   - No call aborts the process and no C++ exception crosses the ABI.
 *   - One gp_sim is used by one host thread at a time.
 */
#ifndef GP_H
#define GP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gp_sim gp_sim;

typedef enum {
    GP_OK = 0,
    GP_EINVAL = -1,   /* bad argument; nothing was launched            */
    GP_ENOMEM = -2,   /* workspace too small                          */
    GP_EDEVICE = -3,  /* HIP runtime or launch error                  */
    GP_ESTATE = -4    /* call not valid in the handle's current state */
} gp_status;

#define GP_MAX_CAMS 4

/* Rendering and dynamics configuration, shared by every scene of a sim. */
typedef struct {
    int32_t width, height;            /* pixels, 1..1024 each                              */
    int32_t n_cams;                   /* cameras per agent, 1..GP_MAX_CAMS                 */
    float cam_dir[GP_MAX_CAMS][2];    /* (cos, sin) of each camera's yaw offset             */
    float focal_px;                   /* focal length in pixels (width/2 for 90 deg HFOV)  */
    float cam_height;                 /* camera height above the road plane, m (1.6)       */
    float z_near, z_far;              /* clip distances along the view axis, m (0.5, 100)  */
    float dt;                         /* step length, s (0.1)                              */
    uint8_t palette[256][3];          /* RGB per colour index; entry 0 is the background   */
} gp_config;

/* One scene as host arrays (copied into the workspace by gp_sim_create). */
typedef struct {
    int32_t n_agents;                 /* >= 1 (the ego of each view is one of them)        */
    int32_t n_roads;                  /* >= 0                                              */
    const float *agent_state;         /* [n_agents][4] x, y (m), psi (rad), v (m/s)        */
    const float *agent_dims;          /* [n_agents][3] length, width, height (m)           */
    const uint8_t *agent_color;       /* [n_agents] palette index                          */
    const float *road_xy;             /* [n_roads][4][2] corners (m) at z = 0, any winding */
    const uint8_t *road_color;        /* [n_roads] palette index                           */
    /* Static obstacles (Sec. 3.1: static objects are cuboids like the
     * vehicles): boxes that never move and own no view.  They are rendered,
     * and an agent overlapping one collides (gp_sim_check_infractions).
     * Their primitive indices follow the agents': box b = n_agents + k has
     * primitives 6 b + face, and road r becomes 6 (n_agents + n_static) + r.
     * All NULL / 0 for none. */
    int32_t n_static;                 /* >= 0                                              */
    const float *static_xyp;          /* [n_static][3] x, y (m), psi (rad)                 */
    const float *static_dims;         /* [n_static][3] length, width, height (m)           */
    const uint8_t *static_color;      /* [n_static] palette index                          */
    /* Traffic lights (Sec. 3.1: small spheres).  The sample of a pixel shows
     * a light when its ray passes the centre closer than the radius; the
     * fragment is the near intersection, at planar depth in [z_near, z_far].
     * Light g has primitive index 6 (n_agents + n_static) + n_roads + g; its
     * colour is the palette entry of its state (gp_sim_set_signal_colors), not
     * lit by the directional light.  NULL / 0 for none. */
    int32_t n_signals;                /* >= 0                                              */
    const float *signal_xyzr;         /* [n_signals][4] x, y, z of the centre (m), radius  */
    const uint8_t *signal_color;      /* [n_signals] palette index of the initial state    */
} gp_scene_desc;

/* Launch settings of the renderer.  Every setting gives bit-identical images;
 * they only change speed (the autotuner picks among them). */
typedef enum {
    GP_SCHED_PLAIN = 0,       /* one launch per scene                                  */
    GP_SCHED_PERSISTENT = 1   /* one launch; workgroups pull views from a work queue   */
} gp_sched;
/* With GP_SCHED_PERSISTENT and no more views than blocks_per_cu * CUs, the one
 * launch gives every view a workgroup of its own and uses no queue. */

/* Rasteriser of rgb-only renders (no depth / primitive id) of sims whose road
 * strips share one colour, without traffic lights or shading.  Other renders
 * always take the banded rasteriser. */
typedef enum {
    GP_RASTER_BANDED = 0,     /* one workgroup of block_threads per view; LDS key bands of
                                 band_rows rows; triangle lists of batch_tris             */
    GP_RASTER_SPLIT = 1,      /* view_waves wavefronts per view sharing the view's work
                                 through an LDS work counter; about 19 KB of LDS per view
                                 at 128 x 128; needs width % 16 == 0 and a 16-byte aligned
                                 image (else the banded rasteriser runs)                  */
    GP_RASTER_CHIP = 2        /* three chip-wide passes: per-view setup (bin culling, box
                                 triangle lists), road items over the whole chip (coverage
                                 bitmasks in the workspace), resolve items of whole rows;
                                 road_wgs_per_cu workgroups per CU for the road pass;
                                 needs width % 16 == 0, 64 <= width <= 1024 and a 16-byte
                                 aligned image (else the banded rasteriser runs)          */
} gp_raster;

typedef struct {
    int32_t sched;            /* gp_sched                                             */
    int32_t band_rows;        /* banded: image rows per LDS depth-buffer band: 8, 16, 32 or 64 */
    int32_t batch_tris;       /* banded: triangles per LDS batch: 256, 512, 1024 or 2048 */
    int32_t block_threads;    /* banded: threads per workgroup: 256, 512 or 1024       */
    int32_t blocks_per_cu;    /* persistent grid = blocks_per_cu * CUs (1..16)         */
    int32_t raster;           /* gp_raster                                            */
    int32_t view_waves;       /* split: wavefronts per view: 1, 2 or 4                 */
    int32_t road_wgs_per_cu;  /* chip: road-pass workgroups (4 wavefronts) per CU, 1..16 */
} gp_launch;

/* Workspace bytes needed for these scenes (>= 0), or -1 on bad arguments. */
int64_t gp_sim_required_bytes(const gp_config *cfg, const gp_scene_desc *scenes, int32_t n_scenes);

/* Create a sim over n_scenes scenes.  Views are numbered scene-major, then
 * agent, then camera: view = ((agent_base(s) + a) * n_cams + k).  Copies the
 * scene arrays into d_workspace (stream-ordered on `stream`) and computes the
 * initial heading cosines on the device.  The workspace must stay allocated
 * until gp_sim_destroy. */
gp_status gp_sim_create(const gp_config *cfg, const gp_scene_desc *scenes, int32_t n_scenes,
                        void *d_workspace, int64_t workspace_bytes, void *stream, gp_sim **out);

gp_status gp_sim_set_launch(gp_sim *sim, const gp_launch *launch);
gp_status gp_sim_get_launch(const gp_sim *sim, gp_launch *launch);

/* One kinematic step of every agent (App. A dynamics).  d_actions: device
 * float [total_agents][2] = (acceleration m/s^2, steering angle rad), in the
 * agent order of the scenes.  Non-finite actions are clamped with fmin/fmax
 * semantics (NaN becomes the lower bound). */
gp_status gp_sim_step(gp_sim *sim, const float *d_actions, void *stream);

/* Render every view of the current state.  d_rgb: device uint8
 * [num_views][height][width][3] (required).  d_depth: optional device float
 * [num_views][height][width], planar depth in m, +inf for background.
 * d_primid: optional device int32 [num_views][height][width], -1 for
 * background, else 6*box + face (0 front, 1 left, 2 back, 3 right, 4 top,
 * 5 bottom) for boxes (box = agent, or n_agents + k for static obstacle k),
 * 6*(n_agents + n_static) + road for road strips and, after the roads,
 * 6*(n_agents + n_static) + n_roads + light for traffic lights; indices
 * local to the scene. */
gp_status gp_sim_render(gp_sim *sim, uint8_t *d_rgb, float *d_depth, int32_t *d_primid, void *stream);

/* Render every view with the ray-cast backend (App. A: the renderer can
 * rasterise or ray-trace the same scene): one primary ray per pixel sample
 * through the sample's centre; boxes by slab tests in each box's frame
 * (entering hits only), road strips by the ray's ground point (strictly
 * inside a strip; the lowest road index wins), traffic lights by the same
 * sphere test as gp_sim_render; the same winner order (nearest, boxes and
 * lights above roads on ties, then the lower primitive index), colours,
 * light and outputs as gp_sim_render.  The images agree with the raster's
 * except at primitive edges, where exact rays and snapped triangles can
 * differ.  Arguments as gp_sim_render (rgb need not be 4-byte aligned). */
gp_status gp_sim_render_raycast(gp_sim *sim, uint8_t *d_rgb, float *d_depth, int32_t *d_primid, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): gp_sim_render
 * of the rgb image only, through the chip-wide raster, with that raster's
 * scratch (work counters, coverage words, culling-bin, box- and road-triangle
 * lists, road items) taken from a static device array of 64 MiB instead of
 * the sim's workspace.  The call allocates nothing; each GPU holds its own
 * array until the process ends.  d_rgb: device uint8
 * [num_views][height][width][3], 16-byte aligned.  The sim's device must be
 * current.  Every call on a GPU shares that GPU's array and clears what must
 * start at zero, so calls that overlap on one GPU (other streams, other host
 * threads) race: serialise them.  Returns GP_EINVAL when the sim's scratch
 * would exceed 64 MiB (for instance 4,096 views at 512x512), when the image
 * width is not a multiple of 16 in 64..1024, or when the sim's rgb renders
 * need the general kernel (mixed road colours, the light, traffic lights);
 * images are bit-identical to gp_sim_render's. */
gp_status gp_sim_render_noalloc(gp_sim *sim, uint8_t *d_rgb, void *stream);

/* Step then render (rgb only) as one hipGraph replay.  The graph is built on
 * first use and rebuilt when the image pointer or the launch settings change;
 * a new d_actions pointer only updates the step node's arguments, so callers
 * may pass each step's own action buffer without a copy.  Uses the persistent
 * schedule whatever the current launch setting.  A sim of at most 64 views
 * launches the step and the render directly instead (same kernels and
 * images): at that size a graph replay costs more host time than the two
 * launches. */
gp_status gp_sim_step_render_graph(gp_sim *sim, const float *d_actions, uint8_t *d_rgb, void *stream);

/* Traffic-light states: d_colors, device uint8 [num_signals], the palette
 * index of every light (scene order, then the lights' order in each scene),
 * copied into the sim on `stream`.  fork copies the states too. */
gp_status gp_sim_set_signal_colors(gp_sim *sim, const uint8_t *d_colors, void *stream);
int64_t gp_sim_num_signals(const gp_sim *sim);

/* Jerk-actuated step of every agent (App. A, "Action Space and Dynamics":
 * twelve discrete actions, the product of longitudinal jerks {-15, -4, 0, 4}
 * m/s^3 and lateral jerks {-4, 0, 4} m/s^3, integrated into accelerations,
 * then into speed and steering; wheelbase 60% of the length).  d_actions:
 * device uint8 [total_agents], index 3 * lon + lat (lon over the longitudinal
 * set, lat over the lateral one); any index above 11 coasts (both jerks 0).
 * The sim keeps each agent's actuators (longitudinal and lateral
 * acceleration, steering angle), zero after create and set_state.  Limits:
 * longitudinal acceleration in [-6, 3] m/s^2, lateral within 4 m/s^2, speed
 * in [0, 30] m/s, steering angle within 0.5 rad moving at most 0.6 rad/s; the
 * lateral acceleration sets the steering through the bicycle's path
 * curvature (tan(angle) = a_lat * 0.6 L / v^2, v floored at 1 m/s).  Halted
 * agents keep state and actuators.  gp_sim_step (direct acceleration and
 * steering) leaves the actuators untouched.  Stream-ordered; GP_EINVAL on a
 * NULL argument. */
gp_status gp_sim_step_jerk(gp_sim *sim, const uint8_t *d_actions, void *stream);

/* Copy the jerk actuators out: device float [total_agents][4] = longitudinal
 * acceleration (m/s^2; 0 where the speed clip cancelled it), lateral
 * acceleration (v^2 times the path curvature of the last jerk step), steering
 * angle (rad), 0.  Device to device, stream-ordered. */
gp_status gp_sim_get_actuators(gp_sim *sim, float *d_dst, void *stream);

/* Directional light (App. A: shading is one directional light per world with
 * a colour per instance).  h_light: host float[4] = unit direction towards
 * the light in the world frame (norm within 1e-3 of 1) and the ambient term a
 * in [0, 1], the same light in every ego's world; NULL turns shading off (the
 * default: flat palette colours).  With the light on, a face with outward
 * normal n shows each channel c of its palette colour as (c q + 127) / 255,
 * q = floor(255 (a + (1 - a) max(0, n . l)) + 0.5) in binary32; box faces
 * turn with the box heading, road strips face up, the background is unlit.
 * Lit frames are rendered by the general kernel.  Host-side only (takes
 * effect at the next render, drops a captured step + render graph); GP_EINVAL
 * on a bad light. */
gp_status gp_sim_set_light(gp_sim *sim, const float *h_light);

/* Copy the agent state [total_agents][4] out of / into the sim (device to
 * device, stream-ordered).  set_state also refreshes the heading cosines and
 * clears every agent's halted flag and jerk actuators (a new episode). */
gp_status gp_sim_get_state(gp_sim *sim, float *d_dst, void *stream);
gp_status gp_sim_set_state(gp_sim *sim, const float *d_src, void *stream);

/* ---- Batched step + render over several sims (continuous batching in a
 * serving loop; no paper passage: the paper batches all worlds of one
 * training run, App. A "High-Throughput Batched Rendering").
 *
 * gp_batch_required_bytes: bytes of device batch workspace (and of host
 * staging) for a batch of n_sims sims with n_agents agents and n_views
 * views in total; -1 on bad arguments.
 *
 * gp_batch_step_render: for each sims[k], one kinematic step with the host
 * actions h_actions[k] (float [n_agents_k][2]) followed by an rgb render of
 * every view into d_rgb[k] (device uint8 [n_views_k][H][W][3], 4-byte
 * aligned), all sims in one step launch and at most two render launches.
 * Each sim's result is bit-identical to gp_sim_step + gp_sim_render on that
 * sim alone.  Every sim must have the same image size; a sim may appear once.
 * The library packs the batch into h_staging (host memory, pinned for an
 * asynchronous copy, 16-byte aligned) and copies it to d_ws (device,
 * 256-byte aligned) on `stream`: the caller must leave h_staging and d_ws
 * untouched until the stream has passed this call (record an event), and
 * must not render the same sims on another stream meanwhile.  Launch
 * settings are those of sims[0].  Returns GP_EINVAL / GP_ENOMEM with nothing
 * launched on bad arguments. */
int64_t gp_batch_required_bytes(int32_t n_sims, int64_t n_agents, int64_t n_views);
gp_status gp_batch_step_render(gp_sim *const *sims, int32_t n_sims, const float *const *h_actions,
                               uint8_t *const *d_rgb, void *d_ws, int64_t ws_bytes, void *h_staging,
                               int64_t staging_bytes, void *stream);

/* Infraction check of the current state (App. A, "Action Space and
 * Dynamics" / episode rules: an agent that collides or leaves the drivable
 * area is halted in place, speed zeroed, and keeps being observed).  An agent
 * collides when its footprint (length x width rectangle about the box centre,
 * along the heading) overlaps another agent's of the same scene with positive
 * area; it is off-road when its centre lies in no road strip of its scene.
 * Offending agents become halted: their speed is set to 0 and gp_sim_step
 * leaves them in place until gp_sim_set_state.  d_flags (optional, device
 * uint8 [total_agents]) receives bit 0 collision, bit 1 off-road (this check),
 * bit 2 halted (after it).  Stream-ordered. */
gp_status gp_sim_check_infractions(gp_sim *sim, uint8_t *d_flags, void *stream);

/* Fork: make dst's dynamic state (agent state, heading cosines, halted flags,
 * jerk actuators, traffic-light states) a copy of src's (the paper rolls a teacher out in a forked
 * copy of the simulator, Sec. 3 "Pixel-based student training").  Both sims must have
 * been created over the same scenes.  Device-to-device, stream-ordered. */
gp_status gp_sim_fork(gp_sim *dst, const gp_sim *src, void *stream);

int64_t gp_sim_num_views(const gp_sim *sim);
int64_t gp_sim_num_agents(const gp_sim *sim);
int32_t gp_sim_num_scenes(const gp_sim *sim);

/* Free the host handle (and its graph).  Never frees the workspace. */
void gp_sim_destroy(gp_sim *sim);

/* Message for the last non-OK status returned on this thread. */
const char *gp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GP_H */
