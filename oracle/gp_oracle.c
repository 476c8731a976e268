/*
 * CPU oracle for the Gigapixel hot path: the kinematic agent step and the
 * per-agent egocentric raster of a bounding-box world.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU baseline leg of
 * the benchmark do.  It shares no source with the HIP library.
 *
 * What it follows (Gigapixel paper):
 *   - Sec. 3.1: state S_t = (A_t, M, L_t); agents are cuboids, lane polylines
 *     are thin planar strips; each agent gets an ego-centric perspective view.
 *   - App. A, "High-Throughput Batched Rendering": one world (view) per ego
 *     agent, cuboids and planes, per-instance colour (agents blue),
 *     configurable resolution and camera set.
 *   - App. A, "Action Space and Dynamics": kinematic bicycle model with the
 *     wheelbase at 60% of the vehicle length, clipped acceleration, speed and
 *     steering.  App. B, student table: dt = 0.1 s.
 * The paper fixes no numeric conventions of the raster (fill rule, snapping,
 * depth, ties) nor the dynamics constants; the readings taken here are listed
 * in the design notes of the repository and restated beside each function.
 *
 * Precision: every decision in the method (vertex snap, coverage, depth test,
 * winner) is taken in IEEE binary32, the precision of the kernels; the
 * oracle therefore computes in binary32 with every fused multiply-add written
 * as fmaf, correctly rounded division, and no contraction
 * (-ffp-contract=off, no fast-math).  Coverage uses exact int64 arithmetic.
 *
 * Algorithm shape: plain definition.  For each view, every primitive is
 * transformed, clipped, projected and split into triangles; every pixel
 * sample inside a triangle's bounding box is tested; each pixel keeps the
 * fragment with the largest total-order key.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* ------------------------------------------------------------- constants */
#define PIO2_HI   1.57079637e+00f   /* binary32 nearest to pi/2            */
#define PIO2_LO  -4.37113883e-08f   /* binary32 nearest to pi/2 - PIO2_HI  */
#define TWO_OVER_PI 0.636619747f
#define PI_F      3.14159274f
#define TWO_PI_F  6.28318548f

/* dynamics constants: the paper names clipping but gives no values */
#define ACC_MIN  -6.0f
#define ACC_MAX   3.0f
#define STEER_MAX 0.5f
#define V_MIN     0.0f
#define V_MAX    30.0f
#define WHEELBASE_FRAC 0.6f          /* App. A: wheelbase = 60% of length */

/* --------------------------------------------------------------- sincos
 * sin and cos of t for |t| <= 4 (larger t still gives a deterministic,
 * slightly less accurate value).  Written from the mathematics:
 *   - Cody-Waite reduction t = k*pi/2 + r, with pi/2 split in two binary32
 *     terms, k = round-half-even(t * 2/pi);
 *   - Taylor polynomials on |r| <= pi/4, evaluated by Horner with fmaf:
 *       sin r = r + r^3 (-1/3! + r^2 (1/5! + r^2 (-1/7! + r^2 / 9!)))
 *       cos r = 1 + r^2 (-1/2! + r^2 (1/4! + r^2 (-1/6! + r^2 (1/8! - r^2/10!))))
 *   - quadrant k mod 4 selects (+-sin r, +-cos r).
 */
void gpo_sincos(float t, float *s_out, float *c_out)
{
    float kf = rintf(t * TWO_OVER_PI);
    float r = fmaf(-kf, PIO2_HI, t);
    r = fmaf(-kf, PIO2_LO, r);
    float r2 = r * r;
    float ps = fmaf(r2, 2.75573188e-06f, -1.98412701e-04f);
    ps = fmaf(r2, ps, 8.33333377e-03f);
    ps = fmaf(r2, ps, -1.66666672e-01f);
    float sr = fmaf(r * r2, ps, r);
    float pc = fmaf(r2, -2.75573200e-07f, 2.48015876e-05f);
    pc = fmaf(r2, pc, -1.38888892e-03f);
    pc = fmaf(r2, pc, 4.16666679e-02f);
    pc = fmaf(r2, pc, -0.5f);
    float cr = fmaf(r2, pc, 1.0f);
    int q = ((int)kf) & 3;
    float s, c;
    switch (q) {
    case 0: s = sr;  c = cr;  break;
    case 1: s = cr;  c = -sr; break;
    case 2: s = -sr; c = -cr; break;
    default: s = -cr; c = sr; break;
    }
    *s_out = s;
    *c_out = c;
}

static float clampf(float x, float lo, float hi) { return fminf(fmaxf(x, lo), hi); }

/* ----------------------------------------------------------- agent step
 * Kinematic bicycle, semi-implicit Euler, reference point at the box centre.
 * state [n][4] = x, y, psi, v  (updated in place); dims [n][3] = L, W, H;
 * act [n][2] = accel, steer.  cs_out [n][2] = cos psi, sin psi (optional).
 *   a = clamp(accel, -6, 3); delta = clamp(steer, -0.5, 0.5)
 *   v' = clamp(v + a dt, 0, 30)
 *   kappa = sin(delta) / (cos(delta) * 0.6 L)        (App. A wheelbase)
 *   psi' = psi + v' dt kappa, wrapped once into (-pi, pi]
 *   x' = x + v' dt cos psi',  y' = y + v' dt sin psi'
 * An agent flagged in `halted` (optional) keeps its state (App. A: an agent
 * that commits an infraction is halted in place).
 */

/* one bicycle update of st[4] = x, y, psi, v; writes cos/sin psi' to cs[2]
 * (if given) and returns the path curvature kappa */
static float bicycle(float *st, float L, float accel, float steer, float dt, float *cs)
{
    float x = st[0], y = st[1], psi = st[2], v = st[3];
    float a = clampf(accel, ACC_MIN, ACC_MAX);
    float delta = clampf(steer, -STEER_MAX, STEER_MAX);
    float v1 = clampf(fmaf(a, dt, v), V_MIN, V_MAX);
    float sd, cd;
    gpo_sincos(delta, &sd, &cd);
    float kappa = sd / (cd * (WHEELBASE_FRAC * L));
    float vdt = v1 * dt;
    float psi1 = fmaf(vdt, kappa, psi);
    if (psi1 > PI_F)
        psi1 = psi1 - TWO_PI_F;
    else if (psi1 <= -PI_F)
        psi1 = psi1 + TWO_PI_F;
    float sp, cp;
    gpo_sincos(psi1, &sp, &cp);
    st[0] = fmaf(vdt, cp, x);
    st[1] = fmaf(vdt, sp, y);
    st[2] = psi1;
    st[3] = v1;
    if (cs) {
        cs[0] = cp;
        cs[1] = sp;
    }
    return kappa;
}

void gpo_step(int n, float *state, const float *dims, const float *act, float dt, float *cs_out,
              const uint8_t *halted)
{
    for (int i = 0; i < n; ++i) {
        if (halted && halted[i]) {              /* halted in place: state unchanged */
            if (cs_out) gpo_sincos(state[4 * i + 2], &cs_out[2 * i + 1], &cs_out[2 * i + 0]);
            continue;
        }
        bicycle(state + 4 * i, dims[3 * i + 0], act[2 * i + 0], act[2 * i + 1], dt,
                cs_out ? cs_out + 2 * i : NULL);
    }
}

/* ------------------------------------------------------- jerk actuation
 * App. A, "Action Space and Dynamics": twelve discrete actions, the product of
 * the longitudinal jerks {-15, -4, 0, 4} m/s^3 and the lateral jerks
 * {-4, 0, 4} m/s^3.  The jerks are integrated into the longitudinal and
 * lateral accelerations, and those into the speed and the steering, with the
 * accelerations clipped to g-force limits, the speed to the speed limit and
 * the steering angle and its rate bounded; the wheelbase is 60% of the
 * length.  The paper leaves the derivation and the constants to Gigaflow, so
 * the following are readings:
 *   - action k = 3 * lon + lat, lon indexing the longitudinal set and lat the
 *     lateral one; an index outside 0..11 coasts (both jerks zero);
 *   - limits: a_lon in [-6, 3] m/s^2 (as the direct step), |a_lat| <= 4 m/s^2,
 *     |steering rate| <= 0.6 rad/s, |delta| <= 0.5 rad, v in [0, 30] m/s;
 *   - the lateral acceleration sets the steering through the path curvature
 *     of the bicycle, a_lat = v^2 tan(delta) / l with l = 0.6 L, the speed
 *     floored at 1 m/s;
 *   - the actuator state keeps the accelerations the vehicle realised:
 *     a_lon is dropped to 0 where the speed clip cancelled it, a_lat is
 *     v'^2 kappa of the step taken.
 * One step, binary32 with explicit fmaf:
 *   a_lon1 = clamp(fmaf(j_lon, dt, a_lon), -6, 3)
 *   a_lat1 = clamp(fmaf(j_lat, dt, a_lat), -4, 4)
 *   v1     = clamp(fmaf(a_lon1, dt, v), 0, 30)
 *   tau    = clamp((a_lat1 * l) / max(v1 * v1, 1), -T, T),  T = binary32 tan 0.5
 *   delta1 = clamp(atan(tau), fmaf(-R, dt, delta), fmaf(R, dt, delta)), R = 0.6,
 *            then clamp(delta1, -0.5, 0.5)
 *   pose   = bicycle(a_lon1, delta1) as in the direct step (its clamps are
 *            then identities), giving kappa
 *   actuators' = (v1 == fmaf(a_lon1, dt, v) ? a_lon1 : 0, (v1 * v1) * kappa, delta1)
 * state [n][4] and actuators [n][4] = a_lon, a_lat, delta, 0 are updated in
 * place; actions [n] are uint8 indices.  Halted agents keep both.
 */
#define JERK_LAT_ACC_MAX 4.0f
#define JERK_STEER_RATE  0.6f
#define JERK_V_FLOOR2    1.0f
#define TAN_STEER_MAX    0.546302497f   /* binary32 nearest to tan(0.5) */

static const float JERK_LON[4] = {-15.0f, -4.0f, 0.0f, 4.0f};
static const float JERK_LAT[3] = {-4.0f, 0.0f, 4.0f};

/* atan(x) for |x| <= tan(0.5): the Maclaurin series
 *   atan x = x - x^3/3 + x^5/5 - ... + x^25/25
 * (truncation below 3e-9 there), as x + x^3 Q(x^2) with Q evaluated by
 * Horner in fmaf; each coefficient is the binary32 quotient 1 / (2k + 1). */
float gpo_atan_small(float x)
{
    float u = x * x;
    float q = 1.0f / 25.0f;
    q = fmaf(u, q, -1.0f / 23.0f);
    q = fmaf(u, q, 1.0f / 21.0f);
    q = fmaf(u, q, -1.0f / 19.0f);
    q = fmaf(u, q, 1.0f / 17.0f);
    q = fmaf(u, q, -1.0f / 15.0f);
    q = fmaf(u, q, 1.0f / 13.0f);
    q = fmaf(u, q, -1.0f / 11.0f);
    q = fmaf(u, q, 1.0f / 9.0f);
    q = fmaf(u, q, -1.0f / 7.0f);
    q = fmaf(u, q, 1.0f / 5.0f);
    q = fmaf(u, q, -1.0f / 3.0f);
    return fmaf(x * u, q, x);
}

void gpo_step_jerk(int n, float *state, const float *dims, float *actuators, const uint8_t *actions,
                   float dt, float *cs_out, const uint8_t *halted)
{
    for (int i = 0; i < n; ++i) {
        float *st = state + 4 * i, *ac = actuators + 4 * i;
        if (halted && halted[i]) {
            if (cs_out) gpo_sincos(st[2], &cs_out[2 * i + 1], &cs_out[2 * i + 0]);
            continue;
        }
        int k = actions[i];
        float jl = 0.0f, jt = 0.0f;
        if (k < 12) {
            jl = JERK_LON[k / 3];
            jt = JERK_LAT[k % 3];
        }
        float L = dims[3 * i + 0];
        float l = WHEELBASE_FRAC * L;
        float v = st[3];
        float a_lon1 = clampf(fmaf(jl, dt, ac[0]), ACC_MIN, ACC_MAX);
        float a_lat1 = clampf(fmaf(jt, dt, ac[1]), -JERK_LAT_ACC_MAX, JERK_LAT_ACC_MAX);
        float v_free = fmaf(a_lon1, dt, v);
        float v1 = clampf(v_free, V_MIN, V_MAX);
        float tau = clampf((a_lat1 * l) / fmaxf(v1 * v1, JERK_V_FLOOR2), -TAN_STEER_MAX, TAN_STEER_MAX);
        float d1 = clampf(gpo_atan_small(tau), fmaf(-JERK_STEER_RATE, dt, ac[2]),
                          fmaf(JERK_STEER_RATE, dt, ac[2]));
        d1 = clampf(d1, -STEER_MAX, STEER_MAX);
        float kappa = bicycle(st, L, a_lon1, d1, dt, cs_out ? cs_out + 2 * i : NULL);
        ac[0] = v1 == v_free ? a_lon1 : 0.0f;
        ac[1] = (v1 * v1) * kappa;
        ac[2] = d1;
        ac[3] = 0.0f;
    }
}

/* ----------------------------------------------------------- rendering */

typedef struct {
    int n_agents, n_roads;
    const float *agent_state;     /* [n_agents][4] x, y, psi, v */
    const float *agent_dims;      /* [n_agents][3] L, W, H */
    const uint8_t *agent_color;   /* [n_agents] */
    const float *road_xy;         /* [n_roads][4][2] */
    const uint8_t *road_color;    /* [n_roads] */
    int n_static;                 /* static obstacles: cuboids that never move */
    const float *static_xyp;      /* [n_static][3] x, y, psi */
    const float *static_dims;     /* [n_static][3] L, W, H */
    const uint8_t *static_color;  /* [n_static] */
    int n_signals;                /* traffic lights: spheres */
    const float *signal_xyzr;     /* [n_signals][4] x, y, z (centre, m), radius */
    const uint8_t *signal_color;  /* [n_signals] palette index of the light's state */
} gpo_scene;

typedef struct {
    int width, height;
    float focal_px, cam_height, z_near, z_far;
    const uint8_t *palette;       /* [256][3] */
    int shade;                    /* 1: directional light, see shade_level */
    float light[3];               /* unit vector towards the light, world frame */
    float ambient;                /* in [0, 1] */
} gpo_camera;

typedef struct { float x, y, z; } v3;

/* one view's camera: position, forward (fx, fy) in the ground plane */
typedef struct {
    float px, py, fx, fy, h;
    float f, cx, cy, F256, CX256, CY256, G;
    float z_near, z_far;
    int W, H;
} view_t;

/* world point relative to the camera (dx, dy, Z) -> camera space:
 * x right, y up, z forward (planar depth) */
static v3 to_cam(const view_t *vw, float dx, float dy, float Z)
{
    v3 p;
    p.z = fmaf(dx, vw->fx, dy * vw->fy);
    p.x = fmaf(dx, vw->fy, -(dy * vw->fx));
    p.y = Z - vw->h;
    return p;
}

/* world direction -> camera space (same rotation, no translation) */
static v3 dir_to_cam(const view_t *vw, float nx, float ny, float nz)
{
    v3 n;
    n.z = fmaf(nx, vw->fx, ny * vw->fy);
    n.x = fmaf(nx, vw->fy, -(ny * vw->fx));
    n.y = nz;
    return n;
}

/* -- clipping: Sutherland-Hodgman against one half-space at a time.
 * Planes, in order: z >= near, z <= far, and the guard band |x|, |y| <= G z
 * that keeps snapped coordinates below 2^29 subpixels.  Output order: walk
 * the input vertices; keep a vertex that is inside; if the edge to the next
 * vertex crosses the plane, emit the crossing.  The crossing is always
 * computed from the inside endpoint towards the outside one, so an edge shared
 * by two primitives is cut at the same point. */
#define MAXV 12

static float plane_dist(int plane, const view_t *vw, v3 p)
{
    switch (plane) {
    case 0: return p.z - vw->z_near;
    case 1: return vw->z_far - p.z;
    case 2: return fmaf(vw->G, p.z, p.x);
    case 3: return fmaf(vw->G, p.z, -p.x);
    case 4: return fmaf(vw->G, p.z, p.y);
    default: return fmaf(vw->G, p.z, -p.y);
    }
}

static v3 crossing(int plane, const view_t *vw, v3 in, v3 out, float din, float dout)
{
    v3 r;
    float t = din / (din - dout);
    r.x = fmaf(t, out.x - in.x, in.x);
    r.y = fmaf(t, out.y - in.y, in.y);
    r.z = fmaf(t, out.z - in.z, in.z);
    if (plane == 0) r.z = vw->z_near;
    if (plane == 1) r.z = vw->z_far;
    return r;
}

/* Returns the output count, or -1 if the output would exceed MAXV vertices
 * (possible only for a self-intersecting input quad; such a polygon is
 * dropped). */
static int clip_plane(int plane, const view_t *vw, const v3 *in, int n, v3 *out)
{
    int m = 0;
    for (int i = 0; i < n; ++i) {
        v3 a = in[i], b = in[(i + 1) % n];
        float da = plane_dist(plane, vw, a), db = plane_dist(plane, vw, b);
        int ia = da >= 0.0f, ib = db >= 0.0f;
        if (ia) {
            if (m == MAXV) return -1;
            out[m++] = a;
        }
        if (ia != ib) {
            if (m == MAXV) return -1;
            out[m++] = ia ? crossing(plane, vw, a, b, da, db) : crossing(plane, vw, b, a, db, da);
        }
    }
    return m;
}

static int clip_polygon(const view_t *vw, v3 *poly, int n)
{
    v3 tmp[MAXV];
    for (int plane = 0; plane < 6 && n > 0; ++plane) {
        n = clip_plane(plane, vw, poly, n, tmp);
        if (n < 0) return 0;
        memcpy(poly, tmp, sizeof(v3) * (size_t)n);
    }
    return n;
}

/* -- per-pixel resolve state */
typedef struct {
    uint64_t *key;     /* [H*W] */
    const view_t *vw;
    long long frags;   /* fragments that passed coverage and invz > 0 */
} target_t;

static uint32_t f32_bits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }

/* Is sample (Sx, Sy) inside the triangle?  Vertices in 1/256 pixel, positive
 * orientation.  Edge k runs from vertex k to k+1;
 * E_k = (X1-X0)(Sy-Y0) - (Y1-Y0)(Sx-X0).  Inside iff every E_k > 0, or
 * E_k == 0 on a top edge (dY == 0, dX > 0) or a left edge (dY < 0). */
static int covers(const int32_t *X, const int32_t *Y, int64_t Sx, int64_t Sy)
{
    for (int k = 0; k < 3; ++k) {
        int64_t dX = (int64_t)X[(k + 1) % 3] - X[k], dY = (int64_t)Y[(k + 1) % 3] - Y[k];
        int64_t E = dX * (Sy - Y[k]) - dY * (Sx - X[k]);
        int top_left = (dY < 0) || (dY == 0 && dX > 0);
        if (!(E > 0 || (E == 0 && top_left))) return 0;
    }
    return 1;
}

/* Test hook: add 1 to count[j*W + i] for every pixel sample the triangle
 * covers (vertices in any orientation; zero area covers nothing). */
void gpo_cover_tri(const int32_t *Xin, const int32_t *Yin, int W, int H, uint8_t *count)
{
    int32_t X[3] = {Xin[0], Xin[1], Xin[2]}, Y[3] = {Yin[0], Yin[1], Yin[2]};
    int64_t area2 = ((int64_t)X[1] - X[0]) * ((int64_t)Y[2] - Y[0])
                  - ((int64_t)X[2] - X[0]) * ((int64_t)Y[1] - Y[0]);
    if (area2 == 0) return;
    if (area2 < 0) {
        int32_t sx = X[1], sy = Y[1];
        X[1] = X[2]; Y[1] = Y[2]; X[2] = sx; Y[2] = sy;
    }
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i)
            if (covers(X, Y, 256 * (int64_t)i + 128, 256 * (int64_t)j + 128))
                count[j * W + i]++;
}

/* Coverage of one triangle with vertices (X[k], Y[k]) in 1/256 pixel,
 * oriented so that twice its signed area is positive.  Sample of pixel (i, j)
 * is (256 i + 128, 256 j + 128), row 0 at the top.  Every covered sample with
 * 1/z > 0 is a fragment; the pixel keeps the largest key
 * (1/z bits, class, inverted primitive index). */
static void raster_tri(target_t *t, const int32_t *X, const int32_t *Y,
                       float A, float B, float C, uint32_t cls, uint32_t prim)
{
    const view_t *vw = t->vw;
    int64_t xmin = X[0], xmax = X[0], ymin = Y[0], ymax = Y[0];
    for (int k = 1; k < 3; ++k) {
        if (X[k] < xmin) xmin = X[k];
        if (X[k] > xmax) xmax = X[k];
        if (Y[k] < ymin) ymin = Y[k];
        if (Y[k] > ymax) ymax = Y[k];
    }
    /* pixels whose sample can lie in the bounding box */
    int64_t i0 = (xmin - 128 + 255) >> 8;        /* ceil((xmin-128)/256) */
    int64_t i1 = (xmax - 128) >> 8;              /* floor((xmax-128)/256) */
    int64_t j0 = (ymin - 128 + 255) >> 8;
    int64_t j1 = (ymax - 128) >> 8;
    if (i0 < 0) i0 = 0;
    if (j0 < 0) j0 = 0;
    if (i1 > vw->W - 1) i1 = vw->W - 1;
    if (j1 > vw->H - 1) j1 = vw->H - 1;
    for (int64_t j = j0; j <= j1; ++j) {
        for (int64_t i = i0; i <= i1; ++i) {
            if (!covers(X, Y, 256 * i + 128, 256 * j + 128)) continue;
            float du = ((float)i + 0.5f) - vw->cx;
            float dv = ((float)j + 0.5f) - vw->cy;
            float invz = fmaf(A, du, fmaf(B, dv, C));
            if (!(invz > 0.0f)) continue;
            t->frags++;
            uint64_t key = ((uint64_t)f32_bits(invz) << 32) | ((uint64_t)cls << 31)
                         | (uint64_t)(0x7FFFFFFFu - prim);
            uint64_t *slot = &t->key[j * vw->W + i];
            if (key > *slot) *slot = key;
        }
    }
}

/* Sphere (a traffic light, Sec. 3.1) with camera-space centre c and radius r.
 * Reading: the sample of pixel (i, j) casts the ray s D, D = (a, b, f) with
 * a = (i + 0.5) - cx, b = cy - (j + 0.5); the ray meets the sphere when the
 * centre's distance to it is below r, found from the closest approach
 *     s0 = (D . c) / (D . D),  w = c - s0 D,  q = r^2 - w . w  (> 0: covered)
 * and the fragment is the near hit s = s0 - sqrt(q / (D . D)) at planar depth
 * z = s f, kept when z_near <= z <= z_far (the part of a sphere nearer than
 * the near plane is clipped away, nothing behind it shows through).  binary32
 * with fmaf, correctly rounded division and square root.  Spheres rank with
 * the boxes on depth ties (class 1). */
static void raster_sphere(target_t *t, v3 c, float r, uint32_t prim)
{
    const view_t *vw = t->vw;
    const float f = vw->f, r2 = r * r, ff = f * f, fz = f * c.z;
    for (int j = 0; j < vw->H; ++j) {
        for (int i = 0; i < vw->W; ++i) {
            const float a = ((float)i + 0.5f) - vw->cx;
            const float b = vw->cy - ((float)j + 0.5f);
            const float dd = fmaf(a, a, fmaf(b, b, ff));
            const float dc = fmaf(a, c.x, fmaf(b, c.y, fz));
            const float s0 = dc / dd;
            const float wx = fmaf(-s0, a, c.x), wy = fmaf(-s0, b, c.y), wz = fmaf(-s0, f, c.z);
            const float q = r2 - fmaf(wx, wx, fmaf(wy, wy, wz * wz));
            if (!(q > 0.0f)) continue;
            const float z = (s0 - sqrtf(q / dd)) * f;
            if (!(z >= vw->z_near && z <= vw->z_far)) continue;
            const float invz = 1.0f / z;
            t->frags++;
            uint64_t key = ((uint64_t)f32_bits(invz) << 32) | ((uint64_t)1u << 31)
                         | (uint64_t)(0x7FFFFFFFu - prim);
            uint64_t *slot = &t->key[j * vw->W + i];
            if (key > *slot) *slot = key;
        }
    }
}

/* Clip, project, snap and raster one planar polygon (a box face or a road
 * quad).  nc = camera-space normal, p0 = a point of the face (camera space).
 * Boxes are one-sided: kept only if the camera is on the outer side (d < 0)
 * and, per triangle, if the snapped triangle is front-facing.  Roads are
 * two-sided: a triangle is flipped to positive orientation; zero area drops. */
static int raster_polygon(target_t *t, v3 *poly, int n, v3 nc, v3 p0,
                          int one_sided, uint32_t cls, uint32_t prim)
{
    const view_t *vw = t->vw;
    float d = fmaf(nc.x, p0.x, fmaf(nc.y, p0.y, nc.z * p0.z));
    if (one_sided && !(d < 0.0f)) return 0;
    n = clip_polygon(vw, poly, n);
    if (n < 3) return 0;
    /* depth plane: 1/z = A du + B dv + C at pixel offsets du, dv from the centre */
    float fd = vw->f * d;
    float A = nc.x / fd;
    float B = -nc.y / fd;
    float C = nc.z / d;
    int32_t X[MAXV], Y[MAXV];
    for (int k = 0; k < n; ++k) {
        float u = poly[k].x / poly[k].z;
        float w = -(poly[k].y / poly[k].z);
        X[k] = (int32_t)rintf(fmaf(u, vw->F256, vw->CX256));
        Y[k] = (int32_t)rintf(fmaf(w, vw->F256, vw->CY256));
    }
    int ntri = 0;
    for (int k = 1; k + 1 < n; ++k) {
        int32_t tx[3] = {X[0], X[k], X[k + 1]};
        int32_t ty[3] = {Y[0], Y[k], Y[k + 1]};
        int64_t area2 = ((int64_t)tx[1] - tx[0]) * ((int64_t)ty[2] - ty[0])
                      - ((int64_t)tx[2] - tx[0]) * ((int64_t)ty[1] - ty[0]);
        if (one_sided) {
            if (area2 >= 0) continue;   /* front faces come out negative in y-down screen space */
        } else if (area2 == 0) {
            continue;
        }
        if (area2 < 0) {               /* store with positive orientation */
            int32_t sx = tx[1], sy = ty[1];
            tx[1] = tx[2]; ty[1] = ty[2];
            tx[2] = sx; ty[2] = sy;
        }
        raster_tri(t, tx, ty, A, B, C, cls, prim);
        ++ntri;
    }
    return ntri;
}

static void make_view(view_t *vw, const gpo_scene *sc, const gpo_camera *cam, int ego, float ck, float sk)
{
    const float *st = sc->agent_state + 4 * ego;
    float se, ce;
    gpo_sincos(st[2], &se, &ce);
    vw->px = st[0];
    vw->py = st[1];
    vw->fx = fmaf(ce, ck, -(se * sk));
    vw->fy = fmaf(se, ck, ce * sk);
    vw->h = cam->cam_height;
    vw->W = cam->width;
    vw->H = cam->height;
    vw->f = cam->focal_px;
    vw->cx = 0.5f * (float)cam->width;
    vw->cy = 0.5f * (float)cam->height;
    vw->F256 = 256.0f * vw->f;
    vw->CX256 = 256.0f * vw->cx;
    vw->CY256 = 256.0f * vw->cy;
    vw->G = 268435456.0f / vw->F256;    /* guard band: |x/z| <= 2^28 / F256 */
    vw->z_near = cam->z_near;
    vw->z_far = cam->z_far;
}

/* ------------------------------------------------------------- shading
 * App. A: shading is minimal, one directional light per world with a colour
 * per instance.  Reading: the light is a unit direction l towards the light in
 * the world frame, the same in every ego's world, with an ambient term a; a
 * surface with outward unit normal n is lit by
 *     s = a + (1 - a) max(0, n . l)
 * turned into an integer level q = floor(255 s + 0.5) (binary32, fmaf), and
 * each colour channel c becomes (c q + 127) / 255 in integers.  The box faces'
 * normals follow the box heading (front (c, s, 0), left (-s, c, 0), back,
 * right, top +z, bottom -z, with (c, s) the project's sincos of the heading);
 * road strips face +z; the background is not lit. */
static uint32_t shade_level(const gpo_camera *cam, float nx, float ny, int face)
{
    float d;
    if (face < 4)
        d = fmaf(nx, cam->light[0], ny * cam->light[1]);
    else
        d = face == 4 ? cam->light[2] : -cam->light[2];
    float s = fmaf(1.0f - cam->ambient, fmaxf(d, 0.0f), cam->ambient);
    return (uint32_t)fmaf(s, 255.0f, 0.5f);
}

/* Keys -> colour (lit as the camera says), depth 1/invz (+inf for
 * background) and primitive index (-1), for one W x H view. */
static void resolve_keys(const gpo_scene *sc, const gpo_camera *cam, const uint64_t *key_scratch, uint8_t *rgb,
                         float *depth, int32_t *primid)
{
    const int W = cam->width, H = cam->height;
    const uint32_t n_a = (uint32_t)sc->n_agents;
    const uint32_t n_box = n_a + (uint32_t)sc->n_static;
    const uint32_t sig0 = 6 * n_box + (uint32_t)sc->n_roads;
    for (int p = 0; p < W * H; ++p) {
        uint64_t key = key_scratch[p];
        int32_t prim = -1;
        uint8_t color = 0;
        float dep = INFINITY;
        if (key != 0) {
            uint32_t zb = (uint32_t)(key >> 32);
            float invz;
            memcpy(&invz, &zb, 4);
            prim = (int32_t)(0x7FFFFFFFu - (uint32_t)(key & 0x7FFFFFFFu));
            const int32_t b = prim / 6;
            color = prim >= (int32_t)sig0       ? sc->signal_color[prim - (int32_t)sig0]
                    : prim >= (int32_t)(6 * n_box) ? sc->road_color[prim - 6 * (int32_t)n_box]
                    : b < (int32_t)n_a            ? sc->agent_color[b]
                                                  : sc->static_color[b - (int32_t)n_a];
            dep = 1.0f / invz;
        }
        if (rgb) {
            uint32_t q = 255;
            if (cam->shade && prim >= 0 && prim < (int32_t)sig0) {     /* lights are emissive */
                if (prim < (int32_t)(6 * n_box)) {
                    const int32_t b = prim / 6;
                    const float psi = b < (int32_t)n_a ? sc->agent_state[4 * b + 2]
                                                       : sc->static_xyp[3 * (b - (int32_t)n_a) + 2];
                    float sj, cj;
                    gpo_sincos(psi, &sj, &cj);
                    const int f = prim % 6;
                    const float nx[4] = { cj, -sj, -cj, sj }, ny[4] = { sj, cj, -sj, -cj };
                    q = shade_level(cam, f < 4 ? nx[f] : 0.0f, f < 4 ? ny[f] : 0.0f, f);
                } else {
                    q = shade_level(cam, 0.0f, 0.0f, 4);
                }
            }
            for (int ch = 0; ch < 3; ++ch) {
                uint32_t c = cam->palette[3 * color + ch];
                rgb[3 * p + ch] = (uint8_t)(cam->shade && prim >= 0 && prim < (int32_t)sig0 ? (c * q + 127u) / 255u
                                                                                            : c);
            }
        }
        if (depth) depth[p] = dep;
        if (primid) primid[p] = prim;
    }
}

/* Render the view of agent `ego` through the camera whose yaw offset is
 * (ck, sk) = (cos, sin).  Outputs (any may be NULL): rgb [H][W][3], depth
 * [H][W] (1/invz, +inf for background), primid [H][W] (-1 for background).
 * Primitive index: 6*b + face for box b (the agents 0..n_agents-1, then the
 * static obstacles), 6*(n_agents + n_static) + road for roads, then
 * 6*(n_agents + n_static) + n_roads + g for traffic light g (unlit: lights
 * are emissive).
 * Faces: 0 front, 1 left, 2 back, 3 right, 4 top, 5 bottom.
 * `key_scratch` must hold H*W uint64.  Returns the number of rasterised
 * triangles; *frags_out (optional) receives the fragment count. */
long long gpo_render_view(const gpo_scene *sc, const gpo_camera *cam, int ego, float ck, float sk,
                          uint64_t *key_scratch, uint8_t *rgb, float *depth, int32_t *primid,
                          long long *frags_out)
{
    view_t vw;
    make_view(&vw, sc, cam, ego, ck, sk);
    const int W = vw.W, H = vw.H;
    target_t t = { key_scratch, &vw, 0 };
    for (int p = 0; p < W * H; ++p) key_scratch[p] = 0;
    long long ntri = 0;
    const uint32_t n_a = (uint32_t)sc->n_agents;

    /* cuboids: the agents, the ego's own box excluded (one world per ego
     * agent), then the static obstacles (Sec. 3.1: static objects are
     * cuboids too); box b has primitives 6 b + face */
    const uint32_t n_box = n_a + (uint32_t)sc->n_static;
    for (uint32_t b = 0; b < n_box; ++b) {
        if ((int)b == ego) continue;
        const int is_static = b >= n_a;
        const float *st = is_static ? sc->static_xyp + 3 * (b - n_a) : sc->agent_state + 4 * b;
        const float *dm = is_static ? sc->static_dims + 3 * (b - n_a) : sc->agent_dims + 3 * b;
        float sj, cj;
        gpo_sincos(st[2], &sj, &cj);
        float ox = st[0] - vw.px, oy = st[1] - vw.py;
        float hl = 0.5f * dm[0], hw = 0.5f * dm[1], Hb = dm[2];
        float ax = hl * cj, ay = hl * sj;        /* half length along the heading */
        float bx = -(hw * sj), by = hw * cj;     /* half width to the left */
        /* footprint, counter-clockwise seen from above:
         * 0 front-right, 1 front-left, 2 back-left, 3 back-right */
        float fxp[4] = { (ox + ax) - bx, (ox + ax) + bx, (ox - ax) + bx, (ox - ax) - bx };
        float fyp[4] = { (oy + ay) - by, (oy + ay) + by, (oy - ay) + by, (oy - ay) - by };
        v3 bot[4], top[4];
        for (int k = 0; k < 4; ++k) {
            bot[k] = to_cam(&vw, fxp[k], fyp[k], 0.0f);
            top[k] = to_cam(&vw, fxp[k], fyp[k], Hb);
        }
        /* outward world normals per face */
        float nwx[6] = { cj, -sj, -cj, sj, 0.0f, 0.0f };
        float nwy[6] = { sj, cj, -sj, -cj, 0.0f, 0.0f };
        float nwz[6] = { 0.0f, 0.0f, 0.0f, 0.0f, 1.0f, -1.0f };
        for (int f = 0; f < 6; ++f) {
            v3 poly[MAXV];
            if (f < 4) {            /* side face over footprint edge f -> f+1 */
                int a = f, c = (f + 1) & 3;
                poly[0] = bot[a]; poly[1] = bot[c]; poly[2] = top[c]; poly[3] = top[a];
            } else if (f == 4) {
                poly[0] = top[0]; poly[1] = top[1]; poly[2] = top[2]; poly[3] = top[3];
            } else {
                poly[0] = bot[3]; poly[1] = bot[2]; poly[2] = bot[1]; poly[3] = bot[0];
            }
            v3 nc = dir_to_cam(&vw, nwx[f], nwy[f], nwz[f]);
            v3 p0 = poly[0];
            ntri += raster_polygon(&t, poly, 4, nc, p0, 1, 1u, (uint32_t)(6 * b + f));
        }
    }
    /* road quads at z = 0, two-sided */
    for (int r = 0; r < sc->n_roads; ++r) {
        const float *q = sc->road_xy + 8 * r;
        v3 poly[MAXV];
        for (int k = 0; k < 4; ++k)
            poly[k] = to_cam(&vw, q[2 * k] - vw.px, q[2 * k + 1] - vw.py, 0.0f);
        v3 nc = dir_to_cam(&vw, 0.0f, 0.0f, 1.0f);
        v3 p0 = poly[0];
        ntri += raster_polygon(&t, poly, 4, nc, p0, 0, 0u, (uint32_t)(6 * n_box + r));
    }
    /* traffic lights, numbered after every road */
    const uint32_t sig0 = 6 * n_box + (uint32_t)sc->n_roads;
    for (int g = 0; g < sc->n_signals; ++g) {
        const float *q = sc->signal_xyzr + 4 * g;
        raster_sphere(&t, to_cam(&vw, q[0] - vw.px, q[1] - vw.py, q[2]), q[3], sig0 + (uint32_t)g);
    }

    resolve_keys(sc, cam, key_scratch, rgb, depth, primid);
    if (frags_out) *frags_out = t.frags;
    return ntri;
}


/* ------------------------------------------------------------ ray casting
 * The paper's other backend (App. A: rasterised or ray-traced; the ray tracer
 * is its default).  One primary ray per pixel sample, the same scene and the
 * same winner order as the raster (largest key: 1/z, then class, then the
 * lower primitive index), the same resolve.  Reading, binary32 with fmaf:
 *   - camera at (px, py, h) with forward (fx, fy, 0), right (fy, -fx, 0) and
 *     up (0, 0, 1); the sample of pixel (i, j) has offsets a = i + 0.5 - cx,
 *     b = cy - (j + 0.5) and world direction
 *       d = (fmaf(a, fy, f fx), fmaf(a, -fx, f fy), b);
 *     a hit at parameter s has planar depth z = s f, kept in [z_near, z_far];
 *   - box b (heading cos/sin (c, s) from the project's sincos, half length hl,
 *     half width hw, height H): the ray in the box frame
 *       o = (fmaf(ox, c, oy s), fmaf(oy, c, -(ox s)), h),  ox = px - x_b, oy = py - y_b,
 *       e = (fmaf(dx, c, dy s), fmaf(dy, c, -(dx s)), b)
 *     against the slabs [-hl, hl] x [-hw, hw] x [0, H]: per axis with e != 0
 *     the entry (lo - o) / e or (hi - o) / e on the side the ray comes from,
 *     with e = 0 the slab is all (-inf, inf) when lo < o < hi and empty
 *     otherwise; the entry is the largest axis entry (the first axis on a
 *     tie), its face the side entered (front / back on the first axis, left /
 *     right on the second, top / bottom on the third); a hit needs
 *     entry <= exit and entry > 0 (only rays that enter from outside: boxes
 *     are one-sided);
 *   - road strips (two-sided, z = 0): a downward ray (b < 0) meets the plane
 *     at s = -h / b, point (fmaf(s, dx, px), fmaf(s, dy, py)); the strips
 *     that hold the point strictly inside (all four edge cross products
 *     fmaf(ex, wy, -(ey wx)) of one sign) are candidates, the lowest road
 *     index wins (all share the depth);
 *   - traffic lights: the sphere test of the raster (same arithmetic).
 */
static void cast_boxes(const gpo_scene *sc, const view_t *vw, int ego, uint64_t *keys)
{
    const uint32_t n_a = (uint32_t)sc->n_agents, n_box = n_a + (uint32_t)sc->n_static;
    const float f = vw->f;
    for (uint32_t bi = 0; bi < n_box; ++bi) {
        if ((int)bi == ego) continue;
        const int is_static = bi >= n_a;
        const float *st = is_static ? sc->static_xyp + 3 * (bi - n_a) : sc->agent_state + 4 * bi;
        const float *dm = is_static ? sc->static_dims + 3 * (bi - n_a) : sc->agent_dims + 3 * bi;
        float sn, cs;
        gpo_sincos(st[2], &sn, &cs);
        const float ox = vw->px - st[0], oy = vw->py - st[1];
        const float o[3] = { fmaf(ox, cs, oy * sn), fmaf(oy, cs, -(ox * sn)), vw->h };
        const float lo[3] = { -(0.5f * dm[0]), -(0.5f * dm[1]), 0.0f };
        const float hi[3] = { 0.5f * dm[0], 0.5f * dm[1], dm[2] };
        const int face_lo[3] = { 2, 3, 5 }, face_hi[3] = { 0, 1, 4 };
        for (int j = 0; j < vw->H; ++j) {
            for (int i = 0; i < vw->W; ++i) {
                const float a = ((float)i + 0.5f) - vw->cx;
                const float b = vw->cy - ((float)j + 0.5f);
                const float dx = fmaf(a, vw->fy, f * vw->fx), dy = fmaf(a, -vw->fx, f * vw->fy);
                const float e[3] = { fmaf(dx, cs, dy * sn), fmaf(dy, cs, -(dx * sn)), b };
                float t_in = -INFINITY, t_out = INFINITY;
                int face = -1;
                for (int k = 0; k < 3; ++k) {
                    float en, lv;
                    int fk;
                    if (e[k] > 0.0f) {
                        en = (lo[k] - o[k]) / e[k]; lv = (hi[k] - o[k]) / e[k]; fk = face_lo[k];
                    } else if (e[k] < 0.0f) {
                        en = (hi[k] - o[k]) / e[k]; lv = (lo[k] - o[k]) / e[k]; fk = face_hi[k];
                    } else {
                        const int in = lo[k] < o[k] && o[k] < hi[k];
                        en = in ? -INFINITY : INFINITY; lv = in ? INFINITY : -INFINITY; fk = -1;
                    }
                    if (en > t_in) { t_in = en; face = fk; }
                    if (lv < t_out) t_out = lv;
                }
                if (!(t_in <= t_out && t_in > 0.0f && t_in < INFINITY)) continue;
                const float z = t_in * f;
                if (!(z >= vw->z_near && z <= vw->z_far)) continue;
                const float invz = 1.0f / z;
                const uint32_t prim = 6 * bi + (uint32_t)face;
                const uint64_t key = ((uint64_t)f32_bits(invz) << 32) | ((uint64_t)1u << 31)
                                   | (uint64_t)(0x7FFFFFFFu - prim);
                if (key > keys[j * vw->W + i]) keys[j * vw->W + i] = key;
            }
        }
    }
}

static void cast_roads(const gpo_scene *sc, const view_t *vw, uint64_t *keys)
{
    const uint32_t n_box = (uint32_t)(sc->n_agents + sc->n_static);
    const float f = vw->f;
    for (int j = 0; j < vw->H; ++j) {
        for (int i = 0; i < vw->W; ++i) {
            const float a = ((float)i + 0.5f) - vw->cx;
            const float b = vw->cy - ((float)j + 0.5f);
            if (!(b < 0.0f)) continue;
            const float dx = fmaf(a, vw->fy, f * vw->fx), dy = fmaf(a, -vw->fx, f * vw->fy);
            const float s = -vw->h / b;
            const float z = s * f;
            if (!(z >= vw->z_near && z <= vw->z_far)) continue;
            const float x = fmaf(s, dx, vw->px), y = fmaf(s, dy, vw->py);
            int best = -1;
            for (int r = 0; r < sc->n_roads && best < 0; ++r) {
                const float *q = sc->road_xy + 8 * r;
                int pos = 0, neg = 0;
                for (int k = 0; k < 4; ++k) {
                    const int k1 = (k + 1) & 3;
                    const float ex = q[2 * k1] - q[2 * k], ey = q[2 * k1 + 1] - q[2 * k + 1];
                    const float wx = x - q[2 * k], wy = y - q[2 * k + 1];
                    const float c = fmaf(ex, wy, -(ey * wx));
                    pos += c > 0.0f;
                    neg += c < 0.0f;
                }
                if (pos == 4 || neg == 4) best = r;
            }
            if (best < 0) continue;
            const float invz = 1.0f / z;
            const uint32_t prim = 6 * n_box + (uint32_t)best;
            const uint64_t key = ((uint64_t)f32_bits(invz) << 32) | (uint64_t)(0x7FFFFFFFu - prim);
            if (key > keys[j * vw->W + i]) keys[j * vw->W + i] = key;
        }
    }
}

/* Ray-cast view of agent `ego` (outputs as gpo_render_view). */
void gpo_raycast_view(const gpo_scene *sc, const gpo_camera *cam, int ego, float ck, float sk,
                      uint64_t *key_scratch, uint8_t *rgb, float *depth, int32_t *primid)
{
    view_t vw;
    make_view(&vw, sc, cam, ego, ck, sk);
    for (int p = 0; p < vw.W * vw.H; ++p) key_scratch[p] = 0;
    target_t t = { key_scratch, &vw, 0 };
    cast_boxes(sc, &vw, ego, key_scratch);
    cast_roads(sc, &vw, key_scratch);
    const uint32_t sig0 = 6 * (uint32_t)(sc->n_agents + sc->n_static) + (uint32_t)sc->n_roads;
    for (int g = 0; g < sc->n_signals; ++g) {
        const float *q = sc->signal_xyzr + 4 * g;
        raster_sphere(&t, to_cam(&vw, q[0] - vw.px, q[1] - vw.py, q[2]), q[3], sig0 + (uint32_t)g);
    }
    resolve_keys(sc, cam, key_scratch, rgb, depth, primid);
}

/* ----------------------------------------------------------- infractions
 * App. A ("halted in place ... continues to receive observations"): an agent
 * that collides with another vehicle or leaves the drivable area is halted,
 * its speed zeroed, for the rest of the episode.  The paper gives no
 * geometric definitions; the readings are:
 *   - collision: the two footprints (length x width rectangles about the box
 *     centre, along the heading) overlap with positive area.  Tested with the
 *     separating axes of both rectangles; boxes that only touch do not collide.
 *     The other box is another agent of the scene or one of its static
 *     obstacles (static_xyp [n_static][3] = x, y, psi; static_dims [n][3]).
 *   - off-road: the agent's centre lies in no road strip of its scene (a strip
 *     contains the point when the point is on the inner side of, or on, each
 *     of its four edges, in either winding).
 * Heading cos/sin come from gpo_sincos.  binary32 throughout, fused
 * operations written as fmaf.
 *
 * One scene: state [n][4] (v zeroed for newly halted agents), dims [n][3],
 * roads [n_roads][4][2], halted [n] (in/out), flags [n] (out):
 * bit 0 collision now, bit 1 off-road now, bit 2 halted after this check.
 */
static float dot2(float ax, float ay, float bx, float by) { return fmaf(ax, bx, ay * by); }

/* half-extent of a rectangle (half sizes hl along u, hw along v) on axis a */
static float reach(float hl, float hw, float ux, float uy, float ax, float ay)
{
    /* v = (-uy, ux) */
    return fmaf(hl, fabsf(dot2(ux, uy, ax, ay)), hw * fabsf(dot2(-uy, ux, ax, ay)));
}

int gpo_overlap(const float *si, const float *di, const float *sj, const float *dj)
{
    float ci, sni, cj, snj;
    gpo_sincos(si[2], &sni, &ci);
    gpo_sincos(sj[2], &snj, &cj);
    const float hli = 0.5f * di[0], hwi = 0.5f * di[1], hlj = 0.5f * dj[0], hwj = 0.5f * dj[1];
    const float dx = sj[0] - si[0], dy = sj[1] - si[1];
    const float ax[4] = {ci, -sni, cj, -snj}, ay[4] = {sni, ci, snj, cj};
    for (int k = 0; k < 4; ++k) {
        const float ri = reach(hli, hwi, ci, sni, ax[k], ay[k]);
        const float rj = reach(hlj, hwj, cj, snj, ax[k], ay[k]);
        if (fabsf(dot2(dx, dy, ax[k], ay[k])) >= ri + rj) return 0;   /* separated (or touching) */
    }
    return 1;
}

int gpo_in_strip(const float *q, float px, float py)
{
    int pos = 0, neg = 0;
    for (int k = 0; k < 4; ++k) {
        const int k1 = (k + 1) & 3;
        const float ex = q[2 * k1] - q[2 * k], ey = q[2 * k1 + 1] - q[2 * k + 1];
        const float wx = px - q[2 * k], wy = py - q[2 * k + 1];
        const float c = fmaf(ex, wy, -(ey * wx));
        pos |= c > 0.0f;
        neg |= c < 0.0f;
    }
    return !(pos && neg);
}

void gpo_infractions(int n, float *state, const float *dims, int n_roads, const float *roads,
                     uint8_t *halted, uint8_t *flags, int n_static, const float *static_xyp,
                     const float *static_dims)
{
    for (int i = 0; i < n; ++i) {
        int col = 0;
        for (int j = 0; j < n && !col; ++j)
            if (j != i) col = gpo_overlap(state + 4 * i, dims + 3 * i, state + 4 * j, dims + 3 * j);
        /* static obstacles are vehicles' obstacles too */
        for (int k = 0; k < n_static && !col; ++k)
            col = gpo_overlap(state + 4 * i, dims + 3 * i, static_xyp + 3 * k, static_dims + 3 * k);
        int on = 0;
        for (int r = 0; r < n_roads && !on; ++r) on = gpo_in_strip(roads + 8 * r, state[4 * i], state[4 * i + 1]);
        flags[i] = (uint8_t)(col | (on ? 0 : 2));
    }
    for (int i = 0; i < n; ++i) {
        if (flags[i]) halted[i] = 1;
        if (halted[i]) {
            state[4 * i + 3] = 0.0f;
            flags[i] |= 4;
        }
    }
}
