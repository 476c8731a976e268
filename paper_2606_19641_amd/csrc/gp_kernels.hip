// HIP kernels of the Gigapixel hot path for gfx950 (MI355X).
//
//   k_step    kinematic bicycle step, one thread per agent
//             (App. A, "Action Space and Dynamics"; dt from App. B)
//   k_cs      heading cosines of the current state (used after create/set_state)
//   k_render  per-agent ego-centric raster of cuboids and road strips
//             (Sec. 3.1 O_pixel; App. A "High-Throughput Batched Rendering")
//
// Numerics: every float operation below is written out explicitly (fmaf for
// fused operations) and the file is compiled with -ffp-contract=off,
// correctly rounded division and IEEE denormals, so that each result is a
// deterministic function of the inputs.  Coverage is exact integer work.
//
// Render design (one workgroup per view):
//   1. cull + setup: every box face and road strip of the scene is moved to
//      camera space and tested against the view frustum; survivors that need
//      no clipping are projected and snapped at once, the rest go to a small
//      LDS queue that is clipped in a dense second pass.  Triangles whose
//      bounding box holds at least one pixel sample are appended to an LDS
//      triangle list with wave ballot + prefix-count compaction.
//   2. raster: the image is walked in bands of rows; each band has a 64-bit
//      depth/winner key per pixel in LDS.  Each wave takes triangles from
//      the list and its lanes sweep the triangle's sample box, testing the
//      three edge functions exactly and folding covered fragments into the
//      key buffer with LDS atomic max.
//   3. resolve: keys become palette colours (and optional depth / primitive
//      id) and are stored with packed dword writes.
//   If a view produces more triangles than the LDS list holds, the view is
//   redone band by band, flushing the list into the band's key buffer
//   whenever it fills (same result: the per-pixel key is a maximum).

#include "gp_device.h"

namespace gp {

// ------------------------------------------------------------ constants
#define GP_PIO2_HI 1.57079637e+00f
#define GP_PIO2_LO -4.37113883e-08f
#define GP_2_OVER_PI 0.636619747f
#define GP_PI 3.14159274f
#define GP_2PI 6.28318548f

__device__ __forceinline__ void dev_sincos(float t, float &s, float &c)
{
    // Cody-Waite reduction by pi/2 (two binary32 parts), Taylor polynomials
    // of sin (to r^9) and cos (to r^10) on the reduced argument, quadrant swap.
    const float k = rintf(t * GP_2_OVER_PI);
    float r = fmaf(-k, GP_PIO2_HI, t);
    r = fmaf(-k, GP_PIO2_LO, r);
    const float r2 = r * r;
    float p = fmaf(r2, 2.75573188e-06f, -1.98412701e-04f);
    p = fmaf(r2, p, 8.33333377e-03f);
    p = fmaf(r2, p, -1.66666672e-01f);
    const float sr = fmaf(r * r2, p, r);
    float q = fmaf(r2, -2.75573200e-07f, 2.48015876e-05f);
    q = fmaf(r2, q, -1.38888892e-03f);
    q = fmaf(r2, q, 4.16666679e-02f);
    q = fmaf(r2, q, -0.5f);
    const float cr = fmaf(r2, q, 1.0f);
    const int quad = ((int)k) & 3;
    s = (quad == 0) ? sr : (quad == 1) ? cr : (quad == 2) ? -sr : -cr;
    c = (quad == 0) ? cr : (quad == 1) ? -sr : (quad == 2) ? -cr : sr;
}

// ------------------------------------------------------------ agent step

__global__ void k_step(DevSim s, const float2 *__restrict__ act, int begin, int count)
{
    const int i = begin + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= begin + count) return;
    const float4 st = s.state[i];
    const float L = s.dims[i].x;
    const float2 u = act[i];
    const float a = fminf(fmaxf(u.x, -6.0f), 3.0f);
    const float delta = fminf(fmaxf(u.y, -0.5f), 0.5f);
    const float v1 = fminf(fmaxf(fmaf(a, s.dt, st.w), 0.0f), 30.0f);
    float sd, cd;
    dev_sincos(delta, sd, cd);
    const float kappa = sd / (cd * (0.6f * L));      // wheelbase = 60% of the length
    const float vdt = v1 * s.dt;
    float psi = fmaf(vdt, kappa, st.z);
    if (psi > GP_PI)
        psi = psi - GP_2PI;
    else if (psi <= -GP_PI)
        psi = psi + GP_2PI;
    float sp, cp;
    dev_sincos(psi, sp, cp);
    s.state[i] = make_float4(fmaf(vdt, cp, st.x), fmaf(vdt, sp, st.y), psi, v1);
    s.cs[i] = make_float2(cp, sp);
}

__global__ void k_cs(DevSim s)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.n_agents) return;
    float sp, cp;
    dev_sincos(s.state[i].z, sp, cp);
    s.cs[i] = make_float2(cp, sp);
}

__global__ void k_reset_counter(uint32_t *c) { *c = 0u; }

// ------------------------------------------------------------ render

struct V3 { float x, y, z; };

// per-view camera constants
struct Cam {
    float px, py, fx, fy, h;
    float f, cx, cy, F256, CX256, CY256, G, zn, zf;
    float t_left, t_right, t_top, t_bottom;   // frustum slopes for culling
    int W, H;
};

// triangle in the LDS list: vertices in 1/256 px with positive orientation,
// depth plane, key low word, pixel-sample bounding box (inclusive)
struct TriRec {
    int32_t X0, Y0, X1, Y1, X2, Y2;
    float A, B, C;
    uint32_t keylo;
    int16_t i0, i1, j0, j1;
};
static_assert(sizeof(TriRec) == 48, "TriRec layout");

__device__ __forceinline__ V3 to_cam(const Cam &c, float dx, float dy, float Z)
{
    V3 p;
    p.z = fmaf(dx, c.fx, dy * c.fy);
    p.x = fmaf(dx, c.fy, -(dy * c.fx));
    p.y = Z - c.h;
    return p;
}

__device__ __forceinline__ V3 dir_to_cam(const Cam &c, float nx, float ny, float nz)
{
    V3 n;
    n.z = fmaf(nx, c.fx, ny * c.fy);
    n.x = fmaf(nx, c.fy, -(ny * c.fx));
    n.y = nz;
    return n;
}

// A candidate polygon: 4 camera-space corners, the face normal and the key.
struct Poly {
    V3 v[4];
    V3 n;
    uint32_t keylo;
    bool one_sided;
};

// Build candidate c of the scene: c < 6*n_a is face (c % 6) of agent c / 6,
// otherwise road strip c - 6*n_a.  Returns false for the ego's own faces.
__device__ __forceinline__ bool build_poly(const DevSim &s, const SceneRec &sc, const Cam &cam,
                                           int ego, int c, Poly &P)
{
    const int nbox = 6 * sc.n_agents;
    if (c < nbox) {
        const int j = c / 6, f = c - 6 * j;
        if (j == ego) return false;
        const int ga = sc.agent_base + j;
        const float4 st = s.state[ga];
        const float2 csj = s.cs[ga];
        const float4 dm = s.dims[ga];
        const float cj = csj.x, sj = csj.y;
        const float ox = st.x - cam.px, oy = st.y - cam.py;
        const float hl = 0.5f * dm.x, hw = 0.5f * dm.y, Hb = dm.z;
        const float ax = hl * cj, ay = hl * sj;
        const float bx = -(hw * sj), by = hw * cj;
        // footprint corners, counter-clockwise from above:
        // 0 front-right, 1 front-left, 2 back-left, 3 back-right
        float cx4[4], cy4[4];
        cx4[0] = (ox + ax) - bx; cy4[0] = (oy + ay) - by;
        cx4[1] = (ox + ax) + bx; cy4[1] = (oy + ay) + by;
        cx4[2] = (ox - ax) + bx; cy4[2] = (oy - ay) + by;
        cx4[3] = (ox - ax) - bx; cy4[3] = (oy - ay) - by;
        float nx, ny, nz;
        if (f < 4) {
            const int a = f, b = (f + 1) & 3;
            P.v[0] = to_cam(cam, cx4[a], cy4[a], 0.0f);
            P.v[1] = to_cam(cam, cx4[b], cy4[b], 0.0f);
            P.v[2] = to_cam(cam, cx4[b], cy4[b], Hb);
            P.v[3] = to_cam(cam, cx4[a], cy4[a], Hb);
            nx = (f == 0) ? cj : (f == 1) ? -sj : (f == 2) ? -cj : sj;
            ny = (f == 0) ? sj : (f == 1) ? cj : (f == 2) ? -sj : -cj;
            nz = 0.0f;
        } else if (f == 4) {
            for (int k = 0; k < 4; ++k) P.v[k] = to_cam(cam, cx4[k], cy4[k], Hb);
            nx = 0.0f; ny = 0.0f; nz = 1.0f;
        } else {
            for (int k = 0; k < 4; ++k) P.v[k] = to_cam(cam, cx4[3 - k], cy4[3 - k], 0.0f);
            nx = 0.0f; ny = 0.0f; nz = -1.0f;
        }
        P.n = dir_to_cam(cam, nx, ny, nz);
        P.keylo = (1u << 31) | (0x7FFFFFFFu - (uint32_t)c);
        P.one_sided = true;
    } else {
        const int r = c - nbox;
        const float4 q0 = s.roads[2 * (sc.road_base + r)];
        const float4 q1 = s.roads[2 * (sc.road_base + r) + 1];
        P.v[0] = to_cam(cam, q0.x - cam.px, q0.y - cam.py, 0.0f);
        P.v[1] = to_cam(cam, q0.z - cam.px, q0.w - cam.py, 0.0f);
        P.v[2] = to_cam(cam, q1.x - cam.px, q1.y - cam.py, 0.0f);
        P.v[3] = to_cam(cam, q1.z - cam.px, q1.w - cam.py, 0.0f);
        P.n = dir_to_cam(cam, 0.0f, 0.0f, 1.0f);
        P.keylo = 0x7FFFFFFFu - (uint32_t)c;
        P.one_sided = false;
    }
    return true;
}

// Conservative frustum rejection: true if the polygon certainly covers no
// pixel sample.  Near and far use the clipper's own predicates; the four side
// planes use the tile slopes with a relative margin, valid for every point of
// the polygon's convex hull, so clipping cannot bring a vertex back inside.
__device__ __forceinline__ bool outside(const Cam &c, const V3 *v)
{
    bool n = true, fa = true, l = true, r = true, t = true, b = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float ax = fabsf(v[k].x), ay = fabsf(v[k].y), az = fabsf(v[k].z);
        n = n && (v[k].z - c.zn < 0.0f);
        fa = fa && (c.zf - v[k].z < 0.0f);
        const float mx = 1e-3f * (ax + az) + 1e-6f;
        const float my = 1e-3f * (ay + az) + 1e-6f;
        r = r && (fmaf(-c.t_right, v[k].z, v[k].x) > mx);
        l = l && (fmaf(-c.t_left, v[k].z, -v[k].x) > mx);
        t = t && (fmaf(-c.t_top, v[k].z, v[k].y) > my);
        b = b && (fmaf(-c.t_bottom, v[k].z, -v[k].y) > my);
    }
    return n || fa || l || r || t || b;
}

// clip plane signed distance; >= 0 is inside
__device__ __forceinline__ float plane_dist(int plane, const Cam &c, const V3 &p)
{
    switch (plane) {
    case 0: return p.z - c.zn;
    case 1: return c.zf - p.z;
    case 2: return fmaf(c.G, p.z, p.x);
    case 3: return fmaf(c.G, p.z, -p.x);
    case 4: return fmaf(c.G, p.z, p.y);
    default: return fmaf(c.G, p.z, -p.y);
    }
}

__device__ __forceinline__ bool needs_clip(const Cam &c, const V3 *v)
{
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int pl = 0; pl < 6; ++pl) ok = ok && (plane_dist(pl, c, v[k]) >= 0.0f);
    return !ok;
}

__device__ __forceinline__ void snap(const Cam &c, const V3 &p, int32_t &X, int32_t &Y)
{
    const float u = p.x / p.z;
    const float w = -(p.y / p.z);
    X = (int32_t)rintf(fmaf(u, c.F256, c.CX256));
    Y = (int32_t)rintf(fmaf(w, c.F256, c.CY256));
}

struct Plane { float A, B, C; };

__device__ __forceinline__ Plane face_plane(const Cam &c, const V3 &n, float d)
{
    const float fd = c.f * d;
    Plane pl;
    pl.A = n.x / fd;
    pl.B = -n.y / fd;
    pl.C = n.z / d;
    return pl;
}

// Orient and bound one fan triangle.  Returns false if it is culled or its
// bounding box holds no sample within rows [r0, r1).
__device__ __forceinline__ bool make_tri(const Cam &c, bool one_sided, int32_t X0, int32_t Y0,
                                         int32_t X1, int32_t Y1, int32_t X2, int32_t Y2, int r0,
                                         int r1, TriRec &t)
{
    const int64_t area2 = (int64_t)(X1 - X0) * (int64_t)(Y2 - Y0) - (int64_t)(X2 - X0) * (int64_t)(Y1 - Y0);
    if (one_sided) {
        if (area2 >= 0) return false;      // front faces are negative in y-down screen space
    } else if (area2 == 0) {
        return false;
    }
    if (area2 < 0) {
        const int32_t sx = X1, sy = Y1;
        X1 = X2; Y1 = Y2; X2 = sx; Y2 = sy;
    }
    const int32_t xmin = min(X0, min(X1, X2)), xmax = max(X0, max(X1, X2));
    const int32_t ymin = min(Y0, min(Y1, Y2)), ymax = max(Y0, max(Y1, Y2));
    int i0 = (xmin - 128 + 255) >> 8, i1 = (xmax - 128) >> 8;
    int j0 = (ymin - 128 + 255) >> 8, j1 = (ymax - 128) >> 8;
    i0 = max(i0, 0); i1 = min(i1, c.W - 1);
    j0 = max(j0, r0); j1 = min(j1, r1 - 1);
    if (i0 > i1 || j0 > j1) return false;
    t.X0 = X0; t.Y0 = Y0; t.X1 = X1; t.Y1 = Y1; t.X2 = X2; t.Y2 = Y2;
    t.i0 = (int16_t)i0; t.i1 = (int16_t)i1; t.j0 = (int16_t)j0; t.j1 = (int16_t)j1;
    return true;
}

struct Lds {
    TriRec *tris;
    unsigned long long *zbuf;
    uint8_t *palette;
    int32_t *clipq;
    int32_t *cnt;      // [0] list count, [1] overflow flag, [2] clip-queue count
    int cap;
};

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// Append up to two triangles per lane with one LDS atomic per wave.
__device__ __forceinline__ void append2(Lds &L, bool v0, const TriRec &t0, bool v1, const TriRec &t1)
{
    const unsigned long long b0 = __ballot(v0), b1 = __ballot(v1);
    const int n0 = __popcll(b0), n = n0 + __popcll(b1);
    if (n == 0) return;
    const unsigned long long lt = (1ull << lane_id()) - 1ull;
    int base = 0;
    const int leader = __ffsll((long long)(b0 | b1)) - 1;
    if ((int)lane_id() == leader) base = atomicAdd(&L.cnt[0], n);
    base = __shfl(base, leader);
    if (base + n > L.cap) {
        if ((int)lane_id() == leader) L.cnt[1] = 1;
    }
    if (v0) {
        const int pos = base + __popcll(b0 & lt);
        if (pos < L.cap) L.tris[pos] = t0;
    }
    if (v1) {
        const int pos = base + n0 + __popcll(b1 & lt);
        if (pos < L.cap) L.tris[pos] = t1;
    }
}

__device__ __forceinline__ void append1(Lds &L, const TriRec &t)
{
    const int pos = atomicAdd(&L.cnt[0], 1);
    if (pos < L.cap)
        L.tris[pos] = t;
    else
        L.cnt[1] = 1;
}

// Fast path for one candidate: returns true if it must go through the clipper.
__device__ __forceinline__ bool fast_candidate(const DevSim &s, const SceneRec &sc, const Cam &cam,
                                               int ego, int c, bool active, int r0, int r1, Lds &L)
{
    Poly P;
    bool live = active && build_poly(s, sc, cam, ego, c, P);
    bool clip = false;
    TriRec t0, t1;
    bool v0 = false, v1 = false;
    if (live) {
        live = !outside(cam, P.v);
        if (live) {
            const V3 &p0 = P.v[0];
            const float d = fmaf(P.n.x, p0.x, fmaf(P.n.y, p0.y, P.n.z * p0.z));
            if (P.one_sided && !(d < 0.0f)) live = false;
            if (live) {
                clip = needs_clip(cam, P.v);
                if (!clip) {
                    int32_t X[4], Y[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) snap(cam, P.v[k], X[k], Y[k]);
                    v0 = make_tri(cam, P.one_sided, X[0], Y[0], X[1], Y[1], X[2], Y[2], r0, r1, t0);
                    v1 = make_tri(cam, P.one_sided, X[0], Y[0], X[2], Y[2], X[3], Y[3], r0, r1, t1);
                    if (v0 || v1) {
                        const Plane pl = face_plane(cam, P.n, d);
                        t0.A = pl.A; t0.B = pl.B; t0.C = pl.C; t0.keylo = P.keylo;
                        t1.A = pl.A; t1.B = pl.B; t1.C = pl.C; t1.keylo = P.keylo;
                    }
                }
            }
        }
    }
    append2(L, v0, t0, v1, t1);
    return clip;
}

// Sutherland-Hodgman against one plane.  Walk the vertices; keep an inside
// vertex; if the edge to the next vertex crosses the plane emit the crossing,
// computed from the inside end towards the outside end.
// Returns the output count, or -1 when more than kMaxVerts vertices would
// result (only a self-intersecting input quad can do that; it is dropped).
constexpr int kMaxVerts = 12;
constexpr int kMaxTrisPerCand = kMaxVerts - 2;

__device__ int clip_one(int plane, const Cam &c, const V3 *in, int n, V3 *out)
{
    int m = 0;
    for (int i = 0; i < n; ++i) {
        const V3 a = in[i];
        const V3 b = in[(i + 1 == n) ? 0 : i + 1];
        const float da = plane_dist(plane, c, a), db = plane_dist(plane, c, b);
        const bool ia = da >= 0.0f, ib = db >= 0.0f;
        if (ia) {
            if (m == kMaxVerts) return -1;
            out[m++] = a;
        }
        if (ia != ib) {
            if (m == kMaxVerts) return -1;
            const V3 pin = ia ? a : b, pout = ia ? b : a;
            const float din = ia ? da : db, dout = ia ? db : da;
            const float t = din / (din - dout);
            V3 r;
            r.x = fmaf(t, pout.x - pin.x, pin.x);
            r.y = fmaf(t, pout.y - pin.y, pin.y);
            r.z = fmaf(t, pout.z - pin.z, pin.z);
            if (plane == 0) r.z = c.zn;
            if (plane == 1) r.z = c.zf;
            out[m++] = r;
        }
    }
    return m;
}

// Slow path: clip, project and emit the fan of one candidate.
__device__ __noinline__ void clip_candidate(const DevSim &s, const SceneRec &sc, const Cam &cam,
                                            int ego, int c, int r0, int r1, Lds &L)
{
    Poly P;
    if (!build_poly(s, sc, cam, ego, c, P)) return;
    const V3 p0 = P.v[0];
    const float d = fmaf(P.n.x, p0.x, fmaf(P.n.y, p0.y, P.n.z * p0.z));
    if (P.one_sided && !(d < 0.0f)) return;
    V3 a[kMaxVerts], b[kMaxVerts];
    int n = 4;
    for (int k = 0; k < 4; ++k) a[k] = P.v[k];
    for (int pl = 0; pl < 6 && n > 0; ++pl) {
        n = clip_one(pl, cam, a, n, b);
        if (n < 0) return;
        for (int k = 0; k < n; ++k) a[k] = b[k];
    }
    if (n < 3) return;
    const Plane pln = face_plane(cam, P.n, d);
    int32_t X[kMaxVerts], Y[kMaxVerts];
    for (int k = 0; k < n; ++k) snap(cam, a[k], X[k], Y[k]);
    for (int k = 1; k + 1 < n; ++k) {
        TriRec t;
        if (make_tri(cam, P.one_sided, X[0], Y[0], X[k], Y[k], X[k + 1], Y[k + 1], r0, r1, t)) {
            t.A = pln.A; t.B = pln.B; t.C = pln.C; t.keylo = P.keylo;
            append1(L, t);
        }
    }
}

__device__ __forceinline__ bool covers(const TriRec &t, int64_t Sx, int64_t Sy)
{
    const int32_t X[3] = {t.X0, t.X1, t.X2}, Y[3] = {t.Y0, t.Y1, t.Y2};
    bool in = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3;
        const int64_t dX = (int64_t)X[k1] - X[k], dY = (int64_t)Y[k1] - Y[k];
        const int64_t E = dX * (Sy - Y[k]) - dY * (Sx - X[k]);
        const bool tl = (dY < 0) || (dY == 0 && dX > 0);
        in = in && ((E > 0) || (E == 0 && tl));
    }
    return in;
}

// Fold list triangles into the key buffer of rows [b0, b1).
__device__ void raster_list(const Cam &cam, Lds &L, int ntri, int b0, int b1)
{
    const int nw = blockDim.x >> 6, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int ti = w; ti < ntri; ti += nw) {
        const TriRec t = L.tris[ti];
        const int j0 = max((int)t.j0, b0), j1 = min((int)t.j1, b1 - 1);
        if (j0 > j1) continue;
        const int bw = t.i1 - t.i0 + 1;
        const int n = bw * (j1 - j0 + 1);
        const float inv_bw = 1.0f / (float)bw;
        for (int sidx = lane; sidx < n; sidx += 64) {
            const int dj = (int)(((float)sidx + 0.5f) * inv_bw);
            const int di = sidx - dj * bw;
            const int i = t.i0 + di, j = j0 + dj;
            if (di < 0 || di >= bw || j > j1) continue;     // cannot happen for n < 2^20
            if (!covers(t, 256 * (int64_t)i + 128, 256 * (int64_t)j + 128)) continue;
            const float du = ((float)i + 0.5f) - cam.cx;
            const float dv = ((float)j + 0.5f) - cam.cy;
            const float invz = fmaf(t.A, du, fmaf(t.B, dv, t.C));
            if (!(invz > 0.0f)) continue;
            const unsigned long long key =
                ((unsigned long long)__float_as_uint(invz) << 32) | (unsigned long long)t.keylo;
            atomicMax(&L.zbuf[(j - b0) * cam.W + i], key);
        }
    }
}

__device__ __forceinline__ void clear_band(Lds &L, int npix)
{
    for (int p = threadIdx.x; p < npix; p += blockDim.x) L.zbuf[p] = 0ull;
}

__device__ __forceinline__ uint8_t color_of(const DevSim &s, const SceneRec &sc, int32_t prim)
{
    const int nbox = 6 * sc.n_agents;
    return prim < nbox ? s.agent_color[sc.agent_base + prim / 6]
                       : s.road_color[sc.road_base + (prim - nbox)];
}

__device__ void resolve_band(const DevSim &s, const SceneRec &sc, const Cam &cam, Lds &L,
                             const RenderOut &o, int64_t view, int b0, int b1)
{
    const int W = cam.W;
    const int npix = (b1 - b0) * W;
    const int64_t pix0 = view * (int64_t)cam.W * cam.H + (int64_t)b0 * W;
    if ((W & 3) == 0) {
        uint32_t *rgb32 = reinterpret_cast<uint32_t *>(o.rgb + 3 * pix0);
        for (int q = threadIdx.x; q < (npix >> 2); q += blockDim.x) {
            uint8_t c[12];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int p = 4 * q + k;
                const unsigned long long key = L.zbuf[p];
                int32_t prim = -1;
                uint8_t ci = 0;
                if (key != 0ull) {
                    prim = (int32_t)(0x7FFFFFFFu - (uint32_t)(key & 0x7FFFFFFFull));
                    ci = color_of(s, sc, prim);
                }
                c[3 * k + 0] = L.palette[3 * ci + 0];
                c[3 * k + 1] = L.palette[3 * ci + 1];
                c[3 * k + 2] = L.palette[3 * ci + 2];
                if (o.depth) {
                    const float invz = __uint_as_float((uint32_t)(key >> 32));
                    o.depth[pix0 + p] = (key != 0ull) ? 1.0f / invz : __int_as_float(0x7F800000);
                }
                if (o.primid) o.primid[pix0 + p] = prim;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const uint32_t w = (uint32_t)c[4 * k] | ((uint32_t)c[4 * k + 1] << 8) |
                                   ((uint32_t)c[4 * k + 2] << 16) | ((uint32_t)c[4 * k + 3] << 24);
                rgb32[3 * q + k] = w;
            }
        }
    } else {
        for (int p = threadIdx.x; p < npix; p += blockDim.x) {
            const unsigned long long key = L.zbuf[p];
            int32_t prim = -1;
            uint8_t ci = 0;
            if (key != 0ull) {
                prim = (int32_t)(0x7FFFFFFFu - (uint32_t)(key & 0x7FFFFFFFull));
                ci = color_of(s, sc, prim);
            }
            uint8_t *dst = o.rgb + 3 * (pix0 + p);
            dst[0] = L.palette[3 * ci + 0];
            dst[1] = L.palette[3 * ci + 1];
            dst[2] = L.palette[3 * ci + 2];
            if (o.depth) {
                const float invz = __uint_as_float((uint32_t)(key >> 32));
                o.depth[pix0 + p] = (key != 0ull) ? 1.0f / invz : __int_as_float(0x7F800000);
            }
            if (o.primid) o.primid[pix0 + p] = prim;
        }
    }
}

__device__ __forceinline__ Cam make_cam(const DevSim &s, const SceneRec &sc, int ego, int k)
{
    Cam c;
    const int ga = sc.agent_base + ego;
    const float4 st = s.state[ga];
    const float2 cs = s.cs[ga];
    const float ce = cs.x, se = cs.y;
    const float ck = s.cam_dir[k][0], sk = s.cam_dir[k][1];
    c.px = st.x;
    c.py = st.y;
    c.fx = fmaf(ce, ck, -(se * sk));
    c.fy = fmaf(se, ck, ce * sk);
    c.h = s.cam_height;
    c.W = s.width;
    c.H = s.height;
    c.f = s.focal;
    c.cx = 0.5f * (float)s.width;
    c.cy = 0.5f * (float)s.height;
    c.F256 = 256.0f * c.f;
    c.CX256 = 256.0f * c.cx;
    c.CY256 = 256.0f * c.cy;
    c.G = 268435456.0f / c.F256;
    c.zn = s.z_near;
    c.zf = s.z_far;
    c.t_right = ((float)s.width - c.cx) / c.f;
    c.t_left = c.cx / c.f;
    c.t_top = c.cy / c.f;
    c.t_bottom = ((float)s.height - c.cy) / c.f;
    return c;
}

// Run the cull/setup pass over every candidate, emitting triangles that touch
// rows [r0, r1).  With flush = false an overflow only raises the flag; with
// flush = true the list is rastered into the band buffer when it gets full.
__device__ void setup_pass(const DevSim &s, const SceneRec &sc, const Cam &cam, int ego, int r0,
                           int r1, Lds &L, bool flush)
{
    const int ncand = 6 * sc.n_agents + sc.n_roads;
    const int B = blockDim.x;
    // while flushing, limit each round so that a full round always fits
    const int per_round = flush ? min(B, L.cap / kMaxTrisPerCand) : B;
    for (int base = 0; base < ncand; base += per_round) {
        if (flush) {
            __syncthreads();
            if (L.cnt[0] + per_round * kMaxTrisPerCand > L.cap) {
                raster_list(cam, L, min(L.cnt[0], L.cap), r0, r1);
                __syncthreads();
                if (threadIdx.x == 0) L.cnt[0] = 0;
                __syncthreads();
            }
        }
        const int c = base + (int)threadIdx.x;
        const bool active = (int)threadIdx.x < per_round && c < ncand;
        const bool clip = fast_candidate(s, sc, cam, ego, c, active, r0, r1, L);
        if (clip) {
            const int q = atomicAdd(&L.cnt[2], 1);
            L.clipq[q] = c;
        }
        __syncthreads();
        const int nq = L.cnt[2];
        for (int q = threadIdx.x; q < nq; q += B) clip_candidate(s, sc, cam, ego, L.clipq[q], r0, r1, L);
        __syncthreads();
        if (threadIdx.x == 0) L.cnt[2] = 0;
        if (!flush && L.cnt[1]) break;      // uniform: read after the barrier above
        __syncthreads();
    }
    __syncthreads();
}

__device__ void render_view(const DevSim &s, const RenderOut &o, const LaunchCfg &lc, Lds &L, int view)
{
    const ViewRec vr = s.views[view];
    const SceneRec sc = s.scenes[vr.scene];
    const int ego = vr.ego_cam >> 2, k = vr.ego_cam & 3;
    const Cam cam = make_cam(s, sc, ego, k);
    const int H = cam.H, W = cam.W, BR = lc.band_rows;
    if (threadIdx.x == 0) { L.cnt[0] = 0; L.cnt[1] = 0; L.cnt[2] = 0; }
    __syncthreads();
    setup_pass(s, sc, cam, ego, 0, H, L, false);
    const bool overflow = L.cnt[1] != 0;
    const int ntri = min(L.cnt[0], L.cap);
    __syncthreads();
    for (int b0 = 0; b0 < H; b0 += BR) {
        const int b1 = min(H, b0 + BR);
        clear_band(L, (b1 - b0) * W);
        __syncthreads();
        if (!overflow) {
            raster_list(cam, L, ntri, b0, b1);
        } else {
            if (threadIdx.x == 0) { L.cnt[0] = 0; L.cnt[1] = 0; L.cnt[2] = 0; }
            __syncthreads();
            setup_pass(s, sc, cam, ego, b0, b1, L, true);
            raster_list(cam, L, min(L.cnt[0], L.cap), b0, b1);
        }
        __syncthreads();
        resolve_band(s, sc, cam, L, o, view, b0, b1);
        __syncthreads();
    }
}

__global__ void k_render(DevSim s, RenderOut o, LaunchCfg lc, int persistent, int view_begin)
{
    extern __shared__ __align__(16) unsigned char smem[];
    Lds L;
    L.cap = lc.batch_tris;
    size_t off = 0;
    L.tris = reinterpret_cast<TriRec *>(smem + off);
    off += sizeof(TriRec) * (size_t)lc.batch_tris;
    L.zbuf = reinterpret_cast<unsigned long long *>(smem + off);
    off += sizeof(unsigned long long) * (size_t)lc.band_rows * s.width;
    L.clipq = reinterpret_cast<int32_t *>(smem + off);
    off += sizeof(int32_t) * blockDim.x;
    L.cnt = reinterpret_cast<int32_t *>(smem + off);
    off += 16;
    L.palette = smem + off;
    for (int p = threadIdx.x; p < 768; p += blockDim.x) L.palette[p] = s.palette[p];
    __shared__ int s_item;
    if (!persistent) {
        __syncthreads();
        render_view(s, o, lc, L, view_begin + blockIdx.x);
        return;
    }
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(s.counter, 1u);
        __syncthreads();
        const int it = s_item;
        if (it >= s.n_views) break;
        render_view(s, o, lc, L, s.queue[it]);
    }
}

// ------------------------------------------------------------ launchers

size_t render_lds_bytes(const DevSim &s, const LaunchCfg &c)
{
    return sizeof(TriRec) * (size_t)c.batch_tris + 8u * (size_t)c.band_rows * s.width +
           4u * (size_t)c.block_threads + 16u + 768u;
}

hipError_t launch_step(const DevSim &s, const float *actions, int agent_begin, int agent_count,
                       hipStream_t st)
{
    if (agent_count <= 0) return hipSuccess;
    const int B = 256;
    hipLaunchKernelGGL(k_step, dim3((agent_count + B - 1) / B), dim3(B), 0, st, s,
                       reinterpret_cast<const float2 *>(actions), agent_begin, agent_count);
    return hipGetLastError();
}

hipError_t launch_cs(const DevSim &s, hipStream_t st)
{
    const int B = 256;
    hipLaunchKernelGGL(k_cs, dim3((s.n_agents + B - 1) / B), dim3(B), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_reset_counter(const DevSim &s, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, s.counter);
    return hipGetLastError();
}

hipError_t launch_render(const DevSim &s, const RenderOut &o, const LaunchCfg &c, int persistent,
                         int view_begin, int grid, hipStream_t st)
{
    if (grid <= 0) return hipSuccess;
    const size_t lds = render_lds_bytes(s, c);
    hipLaunchKernelGGL(k_render, dim3(grid), dim3(c.block_threads), lds, st, s, o, c, persistent,
                       view_begin);
    return hipGetLastError();
}

}  // namespace gp
