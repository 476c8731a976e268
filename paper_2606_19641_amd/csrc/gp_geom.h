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
        n = n & (v[k].z - c.zn < 0.0f);
        fa = fa & (c.zf - v[k].z < 0.0f);
        const float mx = 1e-3f * (ax + az) + 1e-6f;
        const float my = 1e-3f * (ay + az) + 1e-6f;
        r = r & (fmaf(-c.t_right, v[k].z, v[k].x) > mx);
        l = l & (fmaf(-c.t_left, v[k].z, -v[k].x) > mx);
        t = t & (fmaf(-c.t_top, v[k].z, v[k].y) > my);
        b = b & (fmaf(-c.t_bottom, v[k].z, -v[k].y) > my);
    }
    return n | fa | l | r | t | b;
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
    // the six tests combined bitwise (no divergent early exits)
    return (zmax < c.zn - m) | (zmin > c.zf + m) | (x - c.t_right * z - r * (1.0f + c.t_right) > m) |
           (-x - c.t_left * z - r * (1.0f + c.t_left) > m) | (-(dm.z - c.h) - c.t_bottom * zmax > m) |
           (-c.h - c.t_top * zmax > m);
}

// Road geometry lies at camera height -h, so a road point at depth z projects
// to image row v = cy + h f / z.  The host computes road_zmax, 2% beyond the
// largest depth that a sample row at or before the far plane looks at; a set
// whose points are all farther projects strictly between two sample rows (or
// above the horizon) and covers no sample.
__device__ __forceinline__ bool road_beyond(const Cam &c, const V3 *v)
{
    return (v[0].z > c.road_zmax) & (v[1].z > c.road_zmax) & (v[2].z > c.road_zmax) & (v[3].z > c.road_zmax);
}

__device__ __forceinline__ bool bin_outside(const DevSim &s, const Cam &c, const RoadBin &b)
{
    V3 v[4];
    v[0] = to_cam(c, b.xmin - c.px, b.ymin - c.py, 0.0f);
    v[1] = to_cam(c, b.xmax - c.px, b.ymin - c.py, 0.0f);
    v[2] = to_cam(c, b.xmax - c.px, b.ymax - c.py, 0.0f);
    v[3] = to_cam(c, b.xmin - c.px, b.ymax - c.py, 0.0f);
    return ((int)outside(c, v) | (int)road_beyond(c, v)) != 0;
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
        for (int pl = 0; pl < 6; ++pl) ok = ok & (plane_dist(pl, c, v[k]) >= 0.0f);
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
// of 2^25 subpixels or more (guard-band geometry).  Rare: kept out of line
// (its 64-bit divisions are long), with scalar arguments.  Returns (xl, xr).
__device__ __noinline__ int2 row_span_int64(int32_t X0, int32_t Y0, int32_t X1, int32_t Y1, int32_t X2, int32_t Y2,
                                            int j, int W)
{
    const int32_t X[3] = {X0, X1, X2}, Y[3] = {Y0, Y1, Y2};
    int xl = 0, xr = W - 1;
    const int64_t Sy = 256 * (int64_t)j + 128;
    for (int k = 0; k < 3; ++k) {
        const int k1 = (k == 2) ? 0 : k + 1;
        const int64_t dX = (int64_t)X[k1] - X[k], dY = (int64_t)Y[k1] - Y[k];
        const int64_t tk = (dY < 0 || (dY == 0 && dX > 0)) ? 0 : 1;
        const int64_t P = dX * (Sy - Y[k]) + dY * ((int64_t)X[k] - 128);
        if (dY == 0) {
            if (P < tk) return make_int2(0, -1);
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
    return make_int2(xl, xr);
}

__device__ __forceinline__ bool row_span(const TriGeo &t, int j, int W, int &xl_out, int &xr_out)
{
    const int32_t X[3] = {t.X0, t.X1, t.X2}, Y[3] = {t.Y0, t.Y1, t.Y2};
    int xl = 0, xr = W - 1;
    if (!t.huge) {
        // every term is an integer below 2^53: fp64 is exact here.  With
        // N = P - t_k and D = 256 |dY|, edge k holds sample i iff
        // N - D i >= 0 (dY > 0: i <= floor(N / D)), N + D i >= 0 (dY < 0:
        // i >= -floor(N / D)) or N >= 0 (dY = 0); the same instructions serve
        // every orientation (no branch on the sign)
        const double Sy = 256.0 * (double)j + 128.0;
        const double Wd = (double)W;
        double lo = 0.0, hi = Wd - 1.0;
        bool empty = false;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int k1 = (k == 2) ? 0 : k + 1;
            const int32_t dX = X[k1] - X[k], dY = Y[k1] - Y[k];
            const double tk = (dY < 0 || (dY == 0 && dX > 0)) ? 0.0 : 1.0;
            const double P = fma((double)dX, Sy - (double)Y[k], (double)dY * ((double)X[k] - 128.0));
            const double N = P - tk;
            empty = empty | ((dY == 0) & (N < 0.0));
            const double D = 256.0 * (double)abs(dY);
            // floor(N / D) from a binary32 reciprocal estimate (relative
            // error below 2^-21, so within 1 of the quotient wherever it lies
            // within W + 2 of zero; farther out the clamp decides, and only
            // the clamped side of the range is used), moved by at most one to
            // the exact value by the exact remainder N - D f
            const double q = (double)((float)N * __builtin_amdgcn_rcpf((float)D));
            double f = fmin(fmax(floor(q), -Wd - 1.0), Wd + 1.0);
            const double r = fma(-D, f, N);
            f = r < 0.0 ? f - 1.0 : (r >= D ? f + 1.0 : f);
            hi = dY > 0 ? fmin(hi, f) : hi;
            lo = dY < 0 ? fmax(lo, -f) : lo;
        }
        xl = (int)lo;
        xr = empty ? -1 : (int)hi;
    } else {
        const int2 r = row_span_int64(t.X0, t.Y0, t.X1, t.Y1, t.X2, t.Y2, j, W);
        xl = r.x;
        xr = r.y;
    }
    xl_out = xl;
    xr_out = xr;
    return xl <= xr;
}

// The same exact spans, written with a branch per edge orientation and the
// int64 path inline: the banded kernels' form (fewer registers live there
// than with row_span's branch-free form and out-of-line int64 path, which
// keeps them at three wavefronts per SIMD).  Identical results.
__device__ __forceinline__ bool row_span_int64_inl(const TriGeo &t, int j, int W, int &xl_out, int &xr_out)
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

__device__ __forceinline__ bool row_span_banded(const TriGeo &t, int j, int W, int &xl_out, int &xr_out)
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
        return row_span_int64_inl(t, j, W, xl_out, xr_out);
    }
    xl_out = xl;
    xr_out = xr;
    return xl <= xr;
}

// ------------------------------------------------------------ road quads
//
// A road strip's two fan triangles (0, 1, 2) and (0, 2, 3) cover, together,
// exactly the samples of the quad's own four-edge test (the same top-left
// rule on each edge) when the snapped quad is strictly convex and neither end
// of the shared diagonal 0-2 lies on a sample point:
//  - a sample strictly on one side of the diagonal can only be in the
//    triangle on that side, and there the two quad edges the triangle lacks
//    are strictly positive (strict convexity: the triangle meets their lines
//    only at the diagonal's ends), so the triangle's test is the quad's;
//  - a sample on the diagonal line has E = 0 for the diagonal in both
//    triangles, run in opposite directions, so exactly one of the two counts
//    it as a top-left edge; strictly between the ends it is inside the quad
//    and inside that triangle, beyond an end both fail an edge through that
//    end, as the quad does;
//  - only the diagonal's ends themselves can differ (two edges meet there), so
//    a quad with an end on a sample point keeps its triangles.
// Coverage is all a road strip contributes in the rgb rasters (strips share
// one plane and colour), so such a strip is rasterised as one quad.

// A road primitive: a positively oriented triangle (nv 3, vertices 0..2) or
// convex quad (nv 4), its sample rows [j0, j1], and whether it needs the
// int64 span path (triangles only).
struct Prim {
    int32_t X0, Y0, X1, Y1, X2, Y2, X3, Y3;
    int16_t j0, j1;
    int16_t huge, nv;
    int32_t pad0, pad1;
};
static_assert(sizeof(Prim) == 48, "Prim layout");

__device__ __forceinline__ Prim prim_of(const TriGeo &t)
{
    Prim p;
    p.X0 = t.X0; p.Y0 = t.Y0; p.X1 = t.X1; p.Y1 = t.Y1; p.X2 = t.X2; p.Y2 = t.Y2;
    p.X3 = t.X0; p.Y3 = t.Y0;
    p.j0 = t.j0; p.j1 = t.j1; p.huge = t.huge; p.nv = 3;
    p.pad0 = 0; p.pad1 = 0;
    return p;
}

// The quad of snapped corners X[k], Y[k] when it may replace its two fan
// triangles (see above; also below 2^25 subpixels, the fp64 span range):
// returns 1 with q set (positively oriented, rows [j0, j1] within [r0, r1)),
// 0 if it covers no sample (bounding box without a sample), -1 when the
// triangles must be used.
__device__ __forceinline__ int make_quad(const Cam &c, const int32_t *X, const int32_t *Y, int r0, int r1, Prim &q)
{
    const int32_t lim = 1 << 25;
    int32_t xmin = X[0], xmax = X[0], ymin = Y[0], ymax = Y[0];
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        xmin = min(xmin, X[k]); xmax = max(xmax, X[k]);
        ymin = min(ymin, Y[k]); ymax = max(ymax, Y[k]);
    }
    if (xmin <= -lim || xmax >= lim || ymin <= -lim || ymax >= lim) return -1;
    // the diagonal's ends on a sample point
    if ((((X[0] - 128) & 255) == 0 && ((Y[0] - 128) & 255) == 0) ||
        (((X[2] - 128) & 255) == 0 && ((Y[2] - 128) & 255) == 0))
        return -1;
    // strict convexity: the turn at every corner has one strict sign
    int npos = 0, nneg = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int a = k, b = (k + 1) & 3, d = (k + 2) & 3;
        const int64_t cr = (int64_t)(X[b] - X[a]) * (int64_t)(Y[d] - Y[b]) -
                           (int64_t)(Y[b] - Y[a]) * (int64_t)(X[d] - X[b]);
        npos += cr > 0;
        nneg += cr < 0;
    }
    if (!(npos == 4 || nneg == 4)) return -1;
    const int i0 = max((xmin - 128 + 255) >> 8, 0), i1 = min((xmax - 128) >> 8, c.W - 1);
    const int j0 = max((ymin - 128 + 255) >> 8, r0), j1 = min((ymax - 128) >> 8, r1 - 1);
    if (i0 > i1 || j0 > j1) return 0;
    // positive orientation (every corner turn > 0, the orientation make_tri
    // gives road triangles after its swap): reverse a quad turning the other
    // way, keeping corner 0 and the diagonal 0-2 (its fan triangles are then
    // the two swapped ones)
    if (npos == 4) {
        q.X0 = X[0]; q.Y0 = Y[0]; q.X1 = X[1]; q.Y1 = Y[1]; q.X2 = X[2]; q.Y2 = Y[2]; q.X3 = X[3]; q.Y3 = Y[3];
    } else {
        q.X0 = X[0]; q.Y0 = Y[0]; q.X1 = X[3]; q.Y1 = Y[3]; q.X2 = X[2]; q.Y2 = Y[2]; q.X3 = X[1]; q.Y3 = Y[1];
    }
    q.j0 = (int16_t)j0; q.j1 = (int16_t)j1;
    q.huge = 0; q.nv = 4;
    q.pad0 = 0; q.pad1 = 0;
    return 1;
}

// Samples [xl, xr] of row j covered by a primitive (row_span for triangles;
// the same exact per-edge bounds over the quad's four edges).
__device__ __forceinline__ bool prim_span(const Prim &p, int j, int W, int &xl_out, int &xr_out)
{
    if (p.nv == 3) {
        TriGeo t;
        t.X0 = p.X0; t.Y0 = p.Y0; t.X1 = p.X1; t.Y1 = p.Y1; t.X2 = p.X2; t.Y2 = p.Y2;
        t.j0 = p.j0; t.j1 = p.j1; t.huge = p.huge; t.pad = 0;
        return row_span(t, j, W, xl_out, xr_out);
    }
    const int32_t X[4] = {p.X0, p.X1, p.X2, p.X3}, Y[4] = {p.Y0, p.Y1, p.Y2, p.Y3};
    const double Sy = 256.0 * (double)j + 128.0;
    const double Wd = (double)W;
    double lo = 0.0, hi = Wd - 1.0;
    bool empty = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int k1 = (k + 1) & 3;
        const int32_t dX = X[k1] - X[k], dY = Y[k1] - Y[k];
        const double tk = (dY < 0 || (dY == 0 && dX > 0)) ? 0.0 : 1.0;
        const double P = fma((double)dX, Sy - (double)Y[k], (double)dY * ((double)X[k] - 128.0));
        const double N = P - tk;
        empty = empty | ((dY == 0) & (N < 0.0));
        const double D = 256.0 * (double)abs(dY);
        const double qe = (double)((float)N * __builtin_amdgcn_rcpf((float)D));
        double f = fmin(fmax(floor(qe), -Wd - 1.0), Wd + 1.0);
        const double r = fma(-D, f, N);
        f = r < 0.0 ? f - 1.0 : (r >= D ? f + 1.0 : f);
        hi = dY > 0 ? fmin(hi, f) : hi;
        lo = dY < 0 ? fmax(lo, -f) : lo;
    }
    const int xl = (int)lo, xr = empty ? -1 : (int)hi;
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

// Whole-record LDS copies as 16-byte vectors (the records' implicit copy
// operators only bind to generic addresses).
typedef int gp_v4i __attribute__((ext_vector_type(4)));

template <class T>
__device__ __forceinline__ T lds_load(lptr<T> p)
{
    constexpr int N = sizeof(T) / 16;
    static_assert(sizeof(T) == 16 * N, "record size");
    union { T t; gp_v4i v[N]; } u;
    lptr<gp_v4i> q = (lptr<gp_v4i>)p;
#pragma unroll
    for (int k = 0; k < N; ++k) u.v[k] = q[k];
    return u.t;
}

template <class T>
__device__ __forceinline__ void lds_store(lptr<T> p, const T &t)
{
    constexpr int N = sizeof(T) / 16;
    union { T t; gp_v4i v[N]; } u;
    u.t = t;
    lptr<gp_v4i> q = (lptr<gp_v4i>)p;
#pragma unroll
    for (int k = 0; k < N; ++k) q[k] = u.v[k];
}


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

// Fast path for one live candidate polygon: cull, project and orient its two
// triangles (kept if their bounding box holds a sample within rows [r0, r1))
// unless it needs the clipper (then `clip` is set).  PLANE: the triangles
// need their depth plane and key (not for road strips of the rgb kernels).
template <bool PLANE>
__device__ __forceinline__ void fast_poly(const Cam &cam, const Poly &P, int r0, int r1, TriRec &t0, bool &v0,
                                          TriRec &t1, bool &v1, bool &clip)
{
    if (outside(cam, P.v)) return;
    if (!P.one_sided && road_beyond(cam, P.v)) return;
    const float d = plane_d(P.n, P.v[0]);
    if (P.one_sided && !(d < 0.0f)) return;
    clip = needs_clip(cam, P.v);
    if (clip) return;
    int32_t X[4], Y[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) snap(cam, P.v[k], X[k], Y[k]);
    v0 = make_tri(cam, P.one_sided, X[0], Y[0], X[1], Y[1], X[2], Y[2], r0, r1, t0.g);
    v1 = make_tri(cam, P.one_sided, X[0], Y[0], X[2], Y[2], X[3], Y[3], r0, r1, t1.g);
    if (PLANE && (v0 || v1)) {
        const Plane pl = face_plane(cam, P.n, d);
        t0.A = pl.A; t0.B = pl.B; t0.C = pl.C; t0.keylo = P.keylo;
        t1.A = pl.A; t1.B = pl.B; t1.C = pl.C; t1.keylo = P.keylo;
    }
}

// Sutherland-Hodgman clipping of one candidate by a whole wave, in registers.
// Lane k holds vertex k of the current polygon.  Against each plane, in the
// order near, far, guard band left / right / top / bottom, the edge from
// vertex k to vertex k+1 (cyclically) contributes vertex k when it is inside
// and then the crossing point when the edge crosses the plane; the crossing
// is computed from the inside end towards the outside end.  The outputs are
// ordered by k, vertex before crossing, exactly as a sequential walk emits
// them; output p is fetched by lane p from the lane that produced it.  A
// polygon that would need more than kMaxVerts vertices (only a
// self-intersecting input quad can) is dropped.
// Each 16-lane segment of the wave clips its own candidate (lane k of a
// segment holds vertex k; a clip never has more than kMaxVerts = 12
// vertices), so a wave clips four candidates at a time.  Within a segment the
// walk is the sequential one: per plane each lane emits its vertex if inside
// and the crossing of its edge if the edge crosses, the outputs placed by a
// prefix over the segment's part of the ballots, which keeps the sequential
// walk's vertex order and arithmetic exactly.  A segment whose vertices are
// all inside a plane keeps its polygon unchanged (the same outputs).  live:
// the segment has a candidate.  Returns true on the lanes that hold a fan
// triangle (lane k of a segment: triangle (0, k, k+1)) with a sample in its
// bounding box within rows [r0, r1), written to t (its depth plane and key
// word too when PLANE).

template <bool PLANE>
__device__ __forceinline__ bool clip_seg(const Cam &cam, const Poly &P, bool live, int r0, int r1, TriRec &t)
{
    const int lane = (int)lane_id();
    const int sl = lane & (kClipSeg - 1), base = lane - sl;     // lane in the segment, segment's first lane
    const float d = plane_d(P.n, P.v[0]);
    int n = (live && !(P.one_sided && !(d < 0.0f))) ? 4 : 0;
    const int l4 = sl & 3;
    V3 v = sel_v3(l4 == 0, P.v[0], sel_v3(l4 == 1, P.v[1], sel_v3(l4 == 2, P.v[2], P.v[3])));
    for (int pl = 0; pl < 6; ++pl) {
        const V3 b = shfl_v3(v, base + (sl + 1 >= n ? 0 : sl + 1));
        const float da = plane_dist(pl, cam, v), db = plane_dist(pl, cam, b);
        const bool act = sl < n;
        const bool ia = da >= 0.0f, ib = db >= 0.0f;
        // every vertex of every segment inside: the walks emit the polygons unchanged
        if (__ballot(act && !ia) == 0ull) continue;
        const bool e0 = act & ia, e1 = act & (ia != ib);
        V3 r = v;
        if (e1) {
            const V3 pin = sel_v3(ia, v, b), pout = sel_v3(ia, b, v);
            const float din = ia ? da : db, dout = ia ? db : da;
            const float t = din / (din - dout);
            r.x = fmaf(t, pout.x - pin.x, pin.x);
            r.y = fmaf(t, pout.y - pin.y, pin.y);
            r.z = fmaf(t, pout.z - pin.z, pin.z);
            if (pl == 0) r.z = cam.zn;
            if (pl == 1) r.z = cam.zf;
        }
        const uint32_t m0 = (uint32_t)(__ballot(e0) >> base) & 0xFFFFu;
        const uint32_t m1 = (uint32_t)(__ballot(e1) >> base) & 0xFFFFu;
        const int total = __popc(m0) + __popc(m1);
        // bit 2k: vertex of lane k, bit 2k+1: crossing of lane k; output p is the
        // (p+1)-th set bit
        uint32_t M = spread_bits(m0) | (spread_bits(m1) << 1);
        const int drop = min(sl, max(total - 1, 0));
        for (int k = 0; k < drop; ++k) M &= M - 1u;
        const int bit = M ? __ffs(M) - 1 : 0;
        const int src = base + (bit >> 1);
        const V3 fv = shfl_v3(v, src), fr = shfl_v3(r, src);
        v = sel_v3(bit & 1, fr, fv);
        // nothing left, or more than kMaxVerts: the polygon is dropped
        n = (total == 0 || total > kMaxVerts) ? 0 : total;
    }
    int32_t X, Y;
    snap(cam, v, X, Y);
    const int32_t X0 = __shfl(X, base), Y0 = __shfl(Y, base);
    const int nx = sl + 1 < n ? sl + 1 : 0;
    const int32_t X2 = __shfl(X, base + nx), Y2 = __shfl(Y, base + nx);
    // fan triangle (0, k, k+1) on lane k of the segment
    bool ok = false;
    if (n >= 3 && sl >= 1 && sl + 1 < n) {
        ok = make_tri(cam, P.one_sided, X0, Y0, X, Y, X2, Y2, r0, r1, t.g);
        if (PLANE) {
            const Plane pln = face_plane(cam, P.n, d);
            t.A = pln.A; t.B = pln.B; t.C = pln.C; t.keylo = P.keylo;
        }
    }
    return ok;
}


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


// ------------------------------------------------------------ wave helpers

// inclusive prefix sum over the wavefront: Hillis-Steele within each row of
// 16 lanes (DPP row shifts), then the row totals carried across rows (DPP row
// broadcasts of lanes 15 and 31)
__device__ __forceinline__ int wave_incl_scan(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast:15 into rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast:31 into rows 2, 3
    return v;
}

// number of lanes whose inclusive prefix (non-decreasing over the lanes) is
// <= g, at most 63: the lane that owns item g.  A binary search whose first
// three levels probe lanes that are the same for every lane (31; 15 or 47; 7,
// 23, 39 or 55), read as scalars, and whose last three levels are replaced by
// counting lanes t .. t + 6 with seven independent shuffles: one cross-lane
// round trip instead of six dependent ones.  Every lane of the wavefront takes
// part.
__device__ __forceinline__ int owner_of(int incl, int g)
{
    const int s31 = __builtin_amdgcn_readlane(incl, 31);
    const int s15 = __builtin_amdgcn_readlane(incl, 15), s47 = __builtin_amdgcn_readlane(incl, 47);
    const int s7 = __builtin_amdgcn_readlane(incl, 7), s23 = __builtin_amdgcn_readlane(incl, 23);
    const int s39 = __builtin_amdgcn_readlane(incl, 39), s55 = __builtin_amdgcn_readlane(incl, 55);
    int t = s31 <= g ? 32 : 0;
    t += (t ? s47 : s15) <= g ? 16 : 0;
    const int c8 = t == 0 ? s7 : (t == 16 ? s23 : (t == 32 ? s39 : s55));
    t += c8 <= g ? 8 : 0;
    int n = 0;
#pragma unroll
    for (int k = 0; k < 7; ++k) n += __shfl(incl, t + k) <= g ? 1 : 0;
    return t + n;
}

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int lanes_below(unsigned long long m)
{
    return __popcll(m & ((1ull << lane_id()) - 1ull));
}

// keep the compiler from moving LDS accesses across this point (the
// wavefront's own LDS operations execute in order)
__device__ __forceinline__ void wave_lds_order() { __asm__ __volatile__("" ::: "memory"); }

// ------------------------------------------------------------ road tests

// Road points lie at camera height -h, so a road vertex at depth z snaps to
// the row coordinate Y(z) = rint(fmaf(h / z, F256, CY256)), a non-increasing
// function of z (correctly rounded division, fmaf and rint are monotone).
// Every vertex a strip's clip can produce has a depth within
// [max(zmin, z_near), min(zmax, z_far)] up to a rounding of the guard-band
// crossings, so its triangles' sample rows lie among the rows whose sample
// 256 j + 128 falls within [Y(zhi), Y(zlo)].  The estimate below uses the
// hardware reciprocal; its error (below 2^-20 relative on the quotient term)
// and the rounding of rint are covered by the margins.  True if no image row
// has its sample in the widened range: then the set covers no sample.
__device__ __forceinline__ bool road_rows_empty(const Cam &c, float zmin, float zmax)
{
    const float zlo = fmaxf(zmin, c.zn) * (1.0f - 0x1p-20f);
    const float zhi = fminf(zmax, c.zf) * (1.0f + 0x1p-20f);
    const float hF = c.h * c.F256;
    const float ylo = fmaf(hF, __builtin_amdgcn_rcpf(zhi), c.CY256);
    const float yhi = fmaf(hF, __builtin_amdgcn_rcpf(zlo), c.CY256);
    const float a = fmaf(-fabsf(ylo), 0x1p-18f, ylo) - 4.0f;
    const float b = fmaf(fabsf(yhi), 0x1p-18f, yhi) + 4.0f;
    const float j0 = fmaxf(ceilf((a - 128.0f) * (1.0f / 256.0f)), 0.0f);
    const float j1 = fminf(floorf((b - 128.0f) * (1.0f / 256.0f)), (float)(c.H - 1));
    return !(j0 <= j1);
}

// Cheap rejection of a road strip (BIN false) or of a culling bin's bounding
// box (BIN true) with camera-space corners (x[k], -h, z[k]): true only if it
// certainly covers no sample.  The tests are the near, far and side tests of
// outside() (same predicates and margins), the road depth limit of
// road_beyond(), and the row-gap test.  A strip's corners are computed here
// exactly as the setup computes them, so its near and far predicates are the
// clipper's own; a bin's strips have corners inside its box, whose computed
// depths can differ from the box corners' by rounding (below 2^-22 of
// |x| + |z|), so a bin's depth tests carry that margin.
template <bool BIN>
__device__ __forceinline__ bool road_culled(const Cam &c, const float *x, const float *z)
{
    bool n = true, fa = true, l = true, r = true;
    float zmin = INFINITY, zmax = -INFINITY;
    const float zlim = fminf(c.road_zmax, c.zf);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float ax = fabsf(x[k]), az = fabsf(z[k]);
        const float dz = BIN ? fmaf(ax + az, 0x1p-20f, 1e-6f) : 0.0f;
        n = n & (z[k] - c.zn < -dz);
        fa = fa & (z[k] - zlim > dz);
        const float mx = 1e-3f * (ax + az) + 1e-6f;
        r = r & (fmaf(-c.t_right, z[k], x[k]) > mx);
        l = l & (fmaf(-c.t_left, z[k], -x[k]) > mx);
        zmin = fminf(zmin, z[k] - dz);
        zmax = fmaxf(zmax, z[k] + dz);
    }
    // combined bitwise (no branch; the row test is cheap next to a divergent exit)
    return n | fa | l | r | road_rows_empty(c, zmin, zmax);
}

// camera-space x and z of a ground point (world x, y)
__device__ __forceinline__ void ground_xz(const Cam &c, float wx, float wy, float &x, float &z)
{
    const float dx = wx - c.px, dy = wy - c.py;
    z = fmaf(dx, c.fx, dy * c.fy);
    x = fmaf(dx, c.fy, -(dy * c.fx));
}

// camera-space corners of road slot g (global), as the setup computes them
__device__ __forceinline__ void road_corners(const DevSim &s, const Cam &cam, int g, V3 *v)
{
    const float4 q0 = s.roads[2 * g], q1 = s.roads[2 * g + 1];
    const float y = 0.0f - cam.h;
    ground_xz(cam, q0.x, q0.y, v[0].x, v[0].z);
    ground_xz(cam, q0.z, q0.w, v[1].x, v[1].z);
    ground_xz(cam, q1.x, q1.y, v[2].x, v[2].z);
    ground_xz(cam, q1.z, q1.w, v[3].x, v[3].z);
    v[0].y = y; v[1].y = y; v[2].y = y; v[3].y = y;
}

// 16 pixels' RGB (byte 0 red) packed into the 48 bytes of their samples
__device__ __forceinline__ void store16(uint8_t *dst, const uint32_t *c)
{
    typedef uint32_t u4v __attribute__((ext_vector_type(4)));
    uint32_t w[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        // bytes 4k .. 4k + 3 belong to pixels p = 4k / 3 and p + 1
        const int p = (4 * k) / 3;
        uint32_t sel = 0;
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) {
            const int b = 4 * k + bb, px = b / 3, ch = b - 3 * px;
            sel |= (uint32_t)(px == p ? ch : 4 + ch) << (8 * bb);
        }
        w[k] = __builtin_amdgcn_perm(c[p + 1 < 16 ? p + 1 : 15], c[p], sel);
    }
    u4v *out = reinterpret_cast<u4v *>(dst);
    out[0] = u4v{w[0], w[1], w[2], w[3]};
    out[1] = u4v{w[4], w[5], w[6], w[7]};
    out[2] = u4v{w[8], w[9], w[10], w[11]};
}

// ------------------------------------------------------------ work queue

// Take the next view of the persistent work queue: kQueues segments of the
// view order, one per XCD, each holding whole scenes (a scene's geometry is
// then read through one L2).  Workgroups are dispatched to the XCDs in turn,
// so workgroup b starts on segment b mod kQueues (`cur`); an exhausted
// segment is marked in the shared mask, which the same atomic returns, and
// the caller moves on to the next segment not yet marked.  counter[q k] is the
// head of segment q, counter[kQueues k] counts the workgroups that have left,
// counter[(kQueues + 1) k] is the exhausted mask (k = kCtrStride, one counter
// per 256 bytes).  Returns a queue position, or
// n_views when every segment is exhausted.  Called by one thread.
__device__ __forceinline__ int queue_take(const DevSim &s, int &cur)
{
    for (;;) {
        const int pos = (int)atomicAdd(&s.counter[cur * kCtrStride], 1u);
        if (pos < s.qseg[cur + 1] - s.qseg[cur]) return s.qseg[cur] + pos;
        const uint32_t mask = atomicOr(&s.counter[(kQueues + 1) * kCtrStride], 1u << cur) | (1u << cur);
        if (mask == (1u << kQueues) - 1u) return s.n_views;
        do cur = (cur + 1) % kQueues; while ((mask >> cur) & 1u);
    }
}

// A workgroup leaves the persistent loop; the last one zeroes the counters,
// so the next launch on the stream starts from full queues without a
// separate reset (and a captured graph holds no memset node).  Called by one
// thread.
__device__ __forceinline__ void queue_leave(const DevSim &s)
{
    __threadfence();
    const uint32_t done = atomicAdd(&s.counter[kQueues * kCtrStride], 1u);
    if (done == gridDim.x - 1) {
        for (int q = 0; q < kQueues + 2; ++q) atomicExch(&s.counter[q * kCtrStride], 0u);
        __threadfence();
    }
}

}  // namespace gp
