// Device-side geometry of the ego-centric raster, shared by the render
// kernels: the per-view camera, camera-space transforms, conservative
// frustum tests, clipping predicates, vertex snapping, triangle setup and the
// exact per-row coverage spans.  Every float operation is written out (fmaf
// for fused operations); the sources including this header are compiled with
// -ffp-contract=off, correctly rounded division and IEEE denormals, so each
// result is a deterministic function of the inputs.
#pragma once

#include "gp_device.h"

namespace gp {

// ------------------------------------------------------------ geometry

struct V3 { float x, y, z; };
struct Plane { float A, B, C; };

__device__ __forceinline__ float uniform_f(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// per-view camera constants (kCamFloats floats, then the image size)
struct Cam {
    float px, py, fx, fy, h;
    float f, cx, cy, F256, CX256, CY256, G, zn, zf;
    float t_left, t_right, t_top, t_bottom;   // frustum slopes for culling
    Plane road;                               // depth plane shared by every road strip
    float road_zmax;                          // farthest road depth a sample row can see
    int W, H;
};
constexpr int kCamFloats = 22;
static_assert(offsetof(Cam, W) == 4 * kCamFloats && sizeof(Cam) == 4 * (kCamFloats + 2), "Cam layout");

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

__device__ __forceinline__ float plane_d(const V3 &n, const V3 &p0)
{
    return fmaf(n.x, p0.x, fmaf(n.y, p0.y, n.z * p0.z));
}

// 1/z = A du + B dv + C at pixel offsets du, dv from the principal point
__device__ __forceinline__ Plane face_plane(const Cam &c, const V3 &n, float d)
{
    const float fd = c.f * d;
    Plane pl;
    pl.A = n.x / fd;
    pl.B = -n.y / fd;
    pl.C = n.z / d;
    return pl;
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
    c.road_zmax = s.road_zmax;
    // every road corner has camera y = -h, so d = n.p0 = -h for every strip
    const V3 n = dir_to_cam(c, 0.0f, 0.0f, 1.0f);
    V3 p0;
    p0.x = 0.0f; p0.y = 0.0f - c.h; p0.z = 0.0f;
    c.road = face_plane(c, n, plane_d(n, p0));
    // one view per workgroup: every field is wave-uniform; keep them in
    // scalar registers
    float *f = &c.px;
#pragma unroll
    for (int q = 0; q < kCamFloats; ++q) f[q] = uniform_f(f[q]);
    c.W = __builtin_amdgcn_readfirstlane(c.W);
    c.H = __builtin_amdgcn_readfirstlane(c.H);
    return c;
}

// A candidate polygon: 4 camera-space corners, its normal and its key word.
struct Poly {
    V3 v[4];
    V3 n;
    uint32_t keylo;
    bool one_sided;
};

// key low word: agent-above-road bit, inverted primitive index (23 bits), colour
__device__ __forceinline__ uint32_t key_low(uint32_t cls, int prim, uint32_t color)
{
    return (cls << 31) | ((uint32_t)(kMaxPrims - 1 - prim) << 8) | color;
}

// face f (0 front, 1 left, 2 back, 3 right, 4 top, 5 bottom) of box j (an
// agent, or a static obstacle for j >= n_agents)
__device__ __forceinline__ void build_face(const DevSim &s, const SceneRec &sc, const Cam &cam, int j,
                                           int f, Poly &P)
{
    const int ga = box_slot(sc, j);
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
#pragma unroll
        for (int k = 0; k < 4; ++k) P.v[k] = to_cam(cam, cx4[k], cy4[k], Hb);
        nx = 0.0f; ny = 0.0f; nz = 1.0f;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) P.v[k] = to_cam(cam, cx4[3 - k], cy4[3 - k], 0.0f);
        nx = 0.0f; ny = 0.0f; nz = -1.0f;
    }
    P.n = dir_to_cam(cam, nx, ny, nz);
    P.keylo = key_low(1u, 6 * j + f, s.agent_color[ga]);
    P.one_sided = true;
}

// road slot `slot` (relative to the scene's road_base) with corners q0, q1
__device__ __forceinline__ void build_road(const DevSim &s, const SceneRec &sc, const Cam &cam, int slot,
                                           const float4 &q0, const float4 &q1, Poly &P)
{
    const int g = sc.road_base + slot;
    P.v[0] = to_cam(cam, q0.x - cam.px, q0.y - cam.py, 0.0f);
    P.v[1] = to_cam(cam, q0.z - cam.px, q0.w - cam.py, 0.0f);
    P.v[2] = to_cam(cam, q1.x - cam.px, q1.y - cam.py, 0.0f);
    P.v[3] = to_cam(cam, q1.z - cam.px, q1.w - cam.py, 0.0f);
    P.n = dir_to_cam(cam, 0.0f, 0.0f, 1.0f);
    P.keylo = key_low(0u, 6 * (sc.n_agents + sc.n_static) + s.road_index[g], s.road_color[g]);
    P.one_sided = false;
}

// Conservative frustum rejection of a convex set given by 4 points: true if
// it certainly covers no pixel sample.  Near and far use the clipper's own
// predicates; the side planes use a relative margin that dominates rounding,
// and hold for every point of the convex hull, so clipping cannot bring a
// point back inside.
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

// Whole-box rejection by the box's bounding cylinder (radius hl + hw >= half
// diagonal, height H) with the same margins as outside().
__device__ __forceinline__ bool box_outside(const DevSim &s, const SceneRec &sc, const Cam &c, int j)
{
    const int ga = box_slot(sc, j);
    const float4 st = s.state[ga];
    const float4 dm = s.dims[ga];
    const float ox = st.x - c.px, oy = st.y - c.py;
    const float r = 0.5f * (dm.x + dm.y);
    const float z = fmaf(ox, c.fx, oy * c.fy);
    const float x = fmaf(ox, c.fy, -(oy * c.fx));
    const float m = 1e-3f * (fabsf(x) + fabsf(z) + r + dm.z + c.h) + 1e-4f;
    const float zmax = z + r, zmin = z - r;
    if (zmax < c.zn - m) return true;
    if (zmin > c.zf + m) return true;
    if (x - c.t_right * z - r * (1.0f + c.t_right) > m) return true;
    if (-x - c.t_left * z - r * (1.0f + c.t_left) > m) return true;
    if (-(dm.z - c.h) - c.t_bottom * zmax > m) return true;
    if (-c.h - c.t_top * zmax > m) return true;
    return false;
}

// Road geometry lies at camera height -h, so a road point at depth z projects
// to image row v = cy + h f / z.  The host computes road_zmax, 2% beyond the
// largest depth that a sample row at or before the far plane looks at; a set
// whose points are all farther projects strictly between two sample rows (or
// above the horizon) and covers no sample.
__device__ __forceinline__ bool road_beyond(const Cam &c, const V3 *v)
{
    return v[0].z > c.road_zmax && v[1].z > c.road_zmax && v[2].z > c.road_zmax && v[3].z > c.road_zmax;
}

__device__ __forceinline__ bool bin_outside(const DevSim &s, const Cam &c, const RoadBin &b)
{
    V3 v[4];
    v[0] = to_cam(c, b.xmin - c.px, b.ymin - c.py, 0.0f);
    v[1] = to_cam(c, b.xmax - c.px, b.ymin - c.py, 0.0f);
    v[2] = to_cam(c, b.xmax - c.px, b.ymax - c.py, 0.0f);
    v[3] = to_cam(c, b.xmin - c.px, b.ymax - c.py, 0.0f);
    return outside(c, v) || road_beyond(c, v);
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

// ------------------------------------------------------------ triangle lists

// A snapped triangle with positive orientation, its sample rows [j0, j1] and
// whether its coordinates need the int64 span path (|coord| >= 2^25).
struct TriGeo {
    int32_t X0, Y0, X1, Y1, X2, Y2;
    int16_t j0, j1;
    int16_t huge, pad;
};
static_assert(sizeof(TriGeo) == 32, "TriGeo layout");

// A triangle with its depth plane and key word (boxes; every primitive in
// the general kernel).
struct TriRec {
    TriGeo g;
    float A, B, C;
    uint32_t keylo;
};
static_assert(sizeof(TriRec) == 48, "TriRec layout");

// Orient and bound one fan triangle.  Returns false if it is culled or its
// bounding box holds no sample within rows [r0, r1).
__device__ __forceinline__ bool make_tri(const Cam &c, bool one_sided, int32_t X0, int32_t Y0,
                                         int32_t X1, int32_t Y1, int32_t X2, int32_t Y2, int r0,
                                         int r1, TriGeo &t)
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
    const int i0 = max((xmin - 128 + 255) >> 8, 0), i1 = min((xmax - 128) >> 8, c.W - 1);
    const int j0 = max((ymin - 128 + 255) >> 8, r0), j1 = min((ymax - 128) >> 8, r1 - 1);
    if (i0 > i1 || j0 > j1) return false;
    t.X0 = X0; t.Y0 = Y0; t.X1 = X1; t.Y1 = Y1; t.X2 = X2; t.Y2 = Y2;
    t.j0 = (int16_t)j0;
    t.j1 = (int16_t)j1;
    const int32_t lim = 1 << 25;
    t.huge = (int16_t)(xmin <= -lim || xmax >= lim || ymin <= -lim || ymax >= lim);
    t.pad = 0;
    return true;
}

// ------------------------------------------------------------ exact row spans

__device__ __forceinline__ int64_t floor_div64(int64_t a, int64_t b)   // b > 0
{
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) --q;
    return q;
}

// Samples i of row j covered by the triangle: [xl, xr] clipped to [0, W).
// Edge k runs from vertex k to k+1; E_k(i) = P_k - 256 dY_k i with
// P_k = dX_k (Sy - Y_k) + dY_k (X_k - 128); a sample is inside iff every
// E_k >= t_k, t_k = 0 on top (dY == 0, dX > 0) and left (dY < 0) edges, else 1.
// The same span in exact int64 arithmetic, for triangles with a coordinate
// of 2^25 subpixels or more (guard-band geometry).
__device__ __forceinline__ bool row_span_int64(const TriGeo &t, int j, int W, int &xl_out, int &xr_out)
{
    const int32_t X[3] = {t.X0, t.X1, t.X2}, Y[3] = {t.Y0, t.Y1, t.Y2};
    int xl = 0, xr = W - 1;
    const int64_t Sy = 256 * (int64_t)j + 128;
    for (int k = 0; k < 3; ++k) {
        const int k1 = (k == 2) ? 0 : k + 1;
        const int64_t dX = (int64_t)X[k1] - X[k], dY = (int64_t)Y[k1] - Y[k];
        const int64_t tk = (dY < 0 || (dY == 0 && dX > 0)) ? 0 : 1;
        const int64_t P = dX * (Sy - Y[k]) + dY * ((int64_t)X[k] - 128);
        if (dY == 0) {
            if (P < tk) return false;
            continue;
        }
        if (dY > 0) {
            const int64_t ic = floor_div64(P - tk, 256 * dY);
            xr = (int)min((int64_t)xr, max(ic, (int64_t)-1));
        } else {
            // i >= (tk - P) / (256 |dY|), rounded up: ceil(-x) = -floor(x)
            const int64_t ic = -floor_div64(P - tk, 256 * (-dY));
            xl = (int)max((int64_t)xl, min(ic, (int64_t)W));
        }
    }
    xl_out = xl;
    xr_out = xr;
    return xl <= xr;
}

__device__ __forceinline__ bool row_span(const TriGeo &t, int j, int W, int &xl_out, int &xr_out)
{
    const int32_t X[3] = {t.X0, t.X1, t.X2}, Y[3] = {t.Y0, t.Y1, t.Y2};
    int xl = 0, xr = W - 1;
    if (!t.huge) {
        // every term is an integer below 2^53: fp64 is exact here
        const double Sy = 256.0 * (double)j + 128.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int k1 = (k == 2) ? 0 : k + 1;
            const int32_t dX = X[k1] - X[k], dY = Y[k1] - Y[k];
            const double tk = (dY < 0 || (dY == 0 && dX > 0)) ? 0.0 : 1.0;
            const double P = fma((double)dX, Sy - (double)Y[k], (double)dY * ((double)X[k] - 128.0));
            if (dY == 0) {
                if (P < tk) return false;
                continue;
            }
            const double D = 256.0 * (double)dY;
            // estimate of (P - tk) / D from a binary32 reciprocal: relative
            // error below 2^-21, so within 1 of the quotient wherever the
            // quotient lies in [-2, W + 1]; outside that range the clamp
            // below decides, and the exact test that follows moves the
            // estimate by at most one to the exact boundary
            const double q = (double)((float)(P - tk) * __builtin_amdgcn_rcpf((float)D));
            if (dY > 0) {            // E decreases with i: i <= q
                double ic = fmin(fmax(floor(q), -1.0), (double)W);
                if (P - D * ic < tk) ic -= 1.0;
                else if (P - D * (ic + 1.0) >= tk) ic += 1.0;
                xr = min(xr, (int)ic);
            } else {                 // E increases with i: i >= q
                double ic = fmin(fmax(ceil(q), -1.0), (double)W);
                if (P - D * ic < tk) ic += 1.0;
                else if (P - D * (ic - 1.0) >= tk) ic -= 1.0;
                xl = max(xl, (int)ic);
            }
        }
    } else {
        return row_span_int64(t, j, W, xl_out, xr_out);
    }
    xl_out = xl;
    xr_out = xr;
    return xl <= xr;
}

// Pointers into LDS keep their address space in the type, so every access
// through them is a ds_* instruction (a generic pointer would make the
// compiler issue flat instructions, which go through the vector-memory path).
#define GP_LDS __attribute__((address_space(3)))
template <class T> using lptr = GP_LDS T *;

// LDS atomics (relaxed; the barriers order them)
__device__ __forceinline__ int lds_add(lptr<int32_t> p, int v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_min(lptr<int32_t> p, int v)
{
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_max(lptr<int32_t> p, int v)
{
    __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_max64(lptr<unsigned long long> p, unsigned long long v)
{
    __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_or64(lptr<unsigned long long> p, unsigned long long v)
{
    __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

static_assert(kBinQuads < 128, "bin count packs into 7 bits");
constexpr int kMaxVerts = 12;
constexpr int kMaxTrisPerCand = kMaxVerts - 2;

// the low 16 bits of x moved to the even bit positions
__device__ __forceinline__ uint32_t spread_bits(uint32_t x)
{
    x &= 0xFFFFu;
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

// Component-wise choice; a conditional expression on whole records would go
// through memory.
__device__ __forceinline__ V3 sel_v3(bool c, const V3 &a, const V3 &b)
{
    V3 r;
    r.x = c ? a.x : b.x;
    r.y = c ? a.y : b.y;
    r.z = c ? a.z : b.z;
    return r;
}

__device__ __forceinline__ V3 shfl_v3(const V3 &v, int src)
{
    V3 r;
    r.x = __shfl(v.x, src);
    r.y = __shfl(v.y, src);
    r.z = __shfl(v.z, src);
    return r;
}

constexpr int kClipSeg = 16;
static_assert(kMaxVerts <= kClipSeg, "a clipped polygon fits a segment");

__device__ __forceinline__ SceneRec uniform_scene(const SceneRec &r)
{
    SceneRec u;
    u.agent_base = __builtin_amdgcn_readfirstlane(r.agent_base);
    u.n_agents = __builtin_amdgcn_readfirstlane(r.n_agents);
    u.road_base = __builtin_amdgcn_readfirstlane(r.road_base);
    u.n_roads = __builtin_amdgcn_readfirstlane(r.n_roads);
    u.view_base = __builtin_amdgcn_readfirstlane(r.view_base);
    u.bin_base = __builtin_amdgcn_readfirstlane(r.bin_base);
    u.n_bins = __builtin_amdgcn_readfirstlane(r.n_bins);
    u.static_base = __builtin_amdgcn_readfirstlane(r.static_base);
    u.n_static = __builtin_amdgcn_readfirstlane(r.n_static);
    u.signal_base = __builtin_amdgcn_readfirstlane(r.signal_base);
    u.n_signals = __builtin_amdgcn_readfirstlane(r.n_signals);
    return u;
}

}  // namespace gp
