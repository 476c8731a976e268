// Ray-cast backend of the Gigapixel renderer for gfx950 (MI355X): the
// paper's renderer can rasterise or ray-trace the same scene (App. A,
// "High-Throughput Batched Rendering"); this kernel casts one primary ray per
// pixel sample and keeps, per pixel, the largest key in the raster's order
// (1/z bits, class, inverted primitive index, colour), so both backends
// resolve alike.
//
// Per-sample arithmetic (binary32, every fused operation an fmaf, correctly
// rounded division and square root):
//   ray      offsets a = i + 0.5 - cx, b = cy - (j + 0.5); world direction
//            d = (fmaf(a, fy, f fx), fmaf(a, -fx, f fy), b) from the camera at
//            (px, py, h) with forward (fx, fy); a hit at parameter s has
//            planar depth z = s f, kept in [z_near, z_far]
//   boxes    the ray in the box frame, o = (fmaf(ox, c, oy s), fmaf(oy, c,
//            -(ox s)), h), e = (fmaf(dx, c, dy s), fmaf(dy, c, -(dx s)), b)
//            with (ox, oy) = camera - box centre and (c, s) the heading
//            cosines, against the slabs [-L/2, L/2] x [-W/2, W/2] x [0, H]:
//            the entry is the largest per-axis entry (first axis on ties),
//            its face the side entered; a hit needs entry <= exit
//   roads    a downward ray meets z = 0 at s = -h / b, point (fmaf(s, dx, px),
//            fmaf(s, dy, py)); a strip holds it when its four edge cross
//            products fmaf(ex, wy, -(ey wx)) share one strict sign
//   lights   the raster's sphere test in camera space
//
// Layout: one workgroup of 256 threads per view; the view is processed in
// bands of about 4096 pixels whose keys live in LDS; between two barriers
// each key is updated by one thread only (no atomics).  Boxes, road bins and
// lights are culled against the view frustum in chunks of up to 256 and the
// survivors staged in LDS; every pixel of the band then tests the staged
// records (boxes only where their image rectangle holds the pixel, road bins
// per sub-band of rows by the ground depths the rows see, their strips staged
// in LDS sixteen bins at a time).  Colours come
// from the keys as in the raster's general kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gp_device.h"

namespace gp {

namespace {

constexpr int kRcThreads = 256;
constexpr int kRcBandPixels = 4096;
constexpr int kRcRoadPixels = 512;        // pixels of a road sub-band
constexpr int kRcStageWords = 10;         // words per staged record
constexpr int kRcStripWords = 9;          // words per staged road strip: 8 corner coordinates, index and colour
constexpr int kRcGroupBins = kRcThreads / kBinQuads;   // bins whose strips are staged together
static_assert(kRcGroupBins * kBinQuads == kRcThreads, "one staged strip per thread");

#define GP_RC_LDS __attribute__((address_space(3)))

struct RcCam {
    float px, py, h, fx, fy, f, cx, cy, zn, zf, tx;   // tx: horizontal frustum slope bound
    int W, H;
};

// a value that is the same in every lane, kept in a scalar register
__device__ __forceinline__ float uniform_float(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ uint32_t key_word(uint32_t cls, int prim, uint32_t color)
{
    return (cls << 31) | ((uint32_t)(kMaxPrims - 1 - prim) << 8) | color;
}

__device__ __forceinline__ unsigned long long make_key(float invz, uint32_t word)
{
    return ((unsigned long long)__float_as_uint(invz) << 32) | word;
}

// lighting of the raster's general kernel: s = a + (1 - a) max(0, n . l),
// level floor(255 s + 0.5), channel (c q + 127) / 255
__device__ __forceinline__ uint32_t rc_level(const DevSim &s, float nx, float ny, int face)
{
    const float lx = s.light[0], ly = s.light[1], lz = s.light[2], amb = s.light[3];
    const float side = fmaf(nx, lx, ny * ly);
    const float d = face < 4 ? side : (face == 4 ? lz : -lz);
    const float sh = fmaf(1.0f - amb, fmaxf(d, 0.0f), amb);
    return (uint32_t)fmaf(sh, 255.0f, 0.5f);
}

__device__ __forceinline__ uint32_t rc_scale(uint32_t c, uint32_t q)
{
    const uint32_t r = ((c & 0xFFu) * q + 127u) / 255u;
    const uint32_t g = (((c >> 8) & 0xFFu) * q + 127u) / 255u;
    const uint32_t b = (((c >> 16) & 0xFFu) * q + 127u) / 255u;
    return r | (g << 8) | (b << 16);
}

__device__ __forceinline__ void rc_sample(const RcCam &c, int i, int j, float &a, float &b, float &dx, float &dy)
{
    a = ((float)i + 0.5f) - c.cx;
    b = c.cy - ((float)j + 0.5f);
    dx = fmaf(a, c.fy, c.f * c.fx);
    dy = fmaf(a, -c.fx, c.f * c.fy);
}

__global__ __launch_bounds__(kRcThreads) void k_raycast(DevSim s, RenderOut o, int view_begin)
{
    extern __shared__ __align__(16) unsigned char smem[];
    GP_RC_LDS unsigned long long *keys = (GP_RC_LDS unsigned long long *)smem;
    GP_RC_LDS float *stg = (GP_RC_LDS float *)(smem + 8 * kRcBandPixels);       // [kRcStageWords][256]
    GP_RC_LDS int32_t *cnt = (GP_RC_LDS int32_t *)(smem + 8 * kRcBandPixels + 4 * kRcStageWords * kRcThreads);
    GP_RC_LDS uint32_t *pal = (GP_RC_LDS uint32_t *)(cnt + 4);
    GP_RC_LDS float *sst = (GP_RC_LDS float *)(pal + 256);                         // [kRcStripWords][256]
    GP_RC_LDS int32_t *isst = (GP_RC_LDS int32_t *)sst;
    GP_RC_LDS int32_t *istg = (GP_RC_LDS int32_t *)stg;
    const int tid = threadIdx.x, B = kRcThreads;
    const int view = view_begin + blockIdx.x;
    const int scene = __builtin_amdgcn_readfirstlane(s.views[view].scene);
    const int ego_cam = __builtin_amdgcn_readfirstlane(s.views[view].ego_cam);
    const SceneRec sc = s.scenes[scene];
    const int ego = ego_cam >> 2, k = ego_cam & 3;
    const int n_box = sc.n_agents + sc.n_static;
    RcCam cam;
    {
        const int ga = sc.agent_base + ego;
        const float4 st = s.state[ga];
        const float2 cs = s.cs[ga];
        const float ck = s.cam_dir[k][0], sk = s.cam_dir[k][1];
        cam.px = uniform_float(st.x);
        cam.py = uniform_float(st.y);
        cam.fx = uniform_float(fmaf(cs.x, ck, -(cs.y * sk)));
        cam.fy = uniform_float(fmaf(cs.y, ck, cs.x * sk));
        cam.h = s.cam_height;
        cam.f = s.focal;
        cam.W = s.width;
        cam.H = s.height;
        cam.cx = 0.5f * (float)s.width;
        cam.cy = 0.5f * (float)s.height;
        cam.zn = s.z_near;
        cam.zf = s.z_far;
        cam.tx = (0.5f * (float)s.width / s.focal) * 1.001f + 1e-3f;
    }
    for (int p = tid; p < 256; p += B)
        pal[p] = (uint32_t)s.palette[3 * p] | ((uint32_t)s.palette[3 * p + 1] << 8) |
                 ((uint32_t)s.palette[3 * p + 2] << 16);
    const int W = cam.W, H = cam.H;
    const int rows = max(1, kRcBandPixels / W);
    const int rrows = max(1, kRcRoadPixels / W);      // rows of a road sub-band
    const int64_t img0 = (int64_t)view * W * H;
    const int sig0 = 6 * n_box + sc.n_roads;
    for (int j0 = 0; j0 < H; j0 += rows) {
        const int j1 = min(H, j0 + rows), npix = (j1 - j0) * W;
        for (int p = tid; p < npix; p += B) keys[p] = 0ull;

        // ---- boxes: cull a chunk, stage the survivors, test every pixel
        for (int u0 = 0; u0 < n_box; u0 += B) {
            __syncthreads();
            if (tid == 0) cnt[0] = 0;
            __syncthreads();
            const int u = u0 + tid;
            if (u < n_box && u != ego) {
                const int g = box_slot(sc, u);
                const float4 st = s.state[g];
                const float4 dm = s.dims[g];
                const float ox = st.x - cam.px, oy = st.y - cam.py;
                const float z = fmaf(ox, cam.fx, oy * cam.fy), x = fmaf(ox, cam.fy, -(oy * cam.fx));
                const float R = 0.5f * (dm.x + dm.y) + 1e-3f;      // bounds the footprint's reach from its centre
                const bool keep = !(z + R < cam.zn) && !(z - R > cam.zf) && !(fabsf(x) - R > (z + R) * cam.tx);
                if (keep) {
                    const int q = __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    const float2 cs = s.cs[g];
                    // pixel rectangle that holds every sample whose ray can hit the
                    // box: with every corner in front of the camera, the box's
                    // image is the hull of its corners' images (a pixel of margin
                    // for rounding); otherwise the whole image
                    int i0 = 0, i1 = cam.W - 1, jr0 = 0, jr1 = cam.H - 1;
                    {
                        const float ax = 0.5f * dm.x * cs.x, ay = 0.5f * dm.x * cs.y;
                        const float bx = -(0.5f * dm.y * cs.y), by = 0.5f * dm.y * cs.x;
                        float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY, zmin = INFINITY;
#pragma unroll
                        for (int c4 = 0; c4 < 4; ++c4) {
                            const float sa = (c4 & 1) ? -1.0f : 1.0f, sb = (c4 & 2) ? -1.0f : 1.0f;
                            const float wx = ox + sa * ax + sb * bx, wy = oy + sa * ay + sb * by;
                            const float zc = fmaf(wx, cam.fx, wy * cam.fy), xc = fmaf(wx, cam.fy, -(wy * cam.fx));
                            zmin = fminf(zmin, zc);
                            const float iz = 1.0f / zc;
                            const float u = fmaf(cam.f * xc, iz, cam.cx);
                            const float v0 = fmaf(-cam.f * (0.0f - cam.h), iz, cam.cy), v1 = fmaf(-cam.f * (dm.z - cam.h), iz, cam.cy);
                            umin = fminf(umin, u);
                            umax = fmaxf(umax, u);
                            vmin = fminf(vmin, fminf(v0, v1));
                            vmax = fmaxf(vmax, fmaxf(v0, v1));
                        }
                        if (zmin > 0.05f) {
                            i0 = max(0, (int)fminf(fmaxf(floorf(umin - 0.5f) - 1.0f, -1.0f), (float)cam.W));
                            i1 = min(cam.W - 1, (int)fminf(fmaxf(ceilf(umax - 0.5f) + 1.0f, -1.0f), (float)cam.W));
                            jr0 = max(0, (int)fminf(fmaxf(floorf(vmin - 0.5f) - 1.0f, -1.0f), (float)cam.H));
                            jr1 = min(cam.H - 1, (int)fminf(fmaxf(ceilf(vmax - 0.5f) + 1.0f, -1.0f), (float)cam.H));
                        }
                    }
                    istg[8 * B + q] = i0 | (jr0 << 16);
                    istg[9 * B + q] = i1 | (jr1 << 16);
                    stg[0 * B + q] = st.x;
                    stg[1 * B + q] = st.y;
                    stg[2 * B + q] = cs.x;
                    stg[3 * B + q] = cs.y;
                    stg[4 * B + q] = 0.5f * dm.x;
                    stg[5 * B + q] = 0.5f * dm.y;
                    stg[6 * B + q] = dm.z;
                    istg[7 * B + q] = (u << 8) | s.agent_color[g];
                }
            }
            __syncthreads();
            const int nb = cnt[0];
            for (int p = tid; p < npix; p += B) {
                const int j = j0 + p / W, i = p - (p / W) * W;
                float a, b, dx, dy;
                rc_sample(cam, i, j, a, b, dx, dy);
                unsigned long long best = keys[p];
                for (int r = 0; r < nb; ++r) {
                    const int lo = istg[8 * B + r], hi = istg[9 * B + r];
                    if (i < (lo & 0xFFFF) || j < (lo >> 16) || i > (hi & 0xFFFF) || j > (hi >> 16)) continue;
                    const float bxr = stg[r], byr = stg[B + r], cb = stg[2 * B + r], sb = stg[3 * B + r];
                    const float hl = stg[4 * B + r], hw = stg[5 * B + r], Hb = stg[6 * B + r];
                    const int tag = istg[7 * B + r];
                    const float ox = cam.px - bxr, oy = cam.py - byr;
                    const float o0 = fmaf(ox, cb, oy * sb), o1 = fmaf(oy, cb, -(ox * sb)), o2 = cam.h;
                    const float e0 = fmaf(dx, cb, dy * sb), e1 = fmaf(dy, cb, -(dx * sb)), e2 = b;
                    float t_in = -INFINITY, t_out = INFINITY;
                    int face = -1;
                    // axis 0: [-hl, hl], faces back (2) / front (0)
                    {
                        float en, lv;
                        int fk;
                        if (e0 > 0.0f) { en = (-hl - o0) / e0; lv = (hl - o0) / e0; fk = 2; }
                        else if (e0 < 0.0f) { en = (hl - o0) / e0; lv = (-hl - o0) / e0; fk = 0; }
                        else { const bool in = -hl < o0 && o0 < hl; en = in ? -INFINITY : INFINITY; lv = in ? INFINITY : -INFINITY; fk = -1; }
                        if (en > t_in) { t_in = en; face = fk; }
                        t_out = fminf(t_out, lv);
                    }
                    {
                        float en, lv;
                        int fk;
                        if (e1 > 0.0f) { en = (-hw - o1) / e1; lv = (hw - o1) / e1; fk = 3; }
                        else if (e1 < 0.0f) { en = (hw - o1) / e1; lv = (-hw - o1) / e1; fk = 1; }
                        else { const bool in = -hw < o1 && o1 < hw; en = in ? -INFINITY : INFINITY; lv = in ? INFINITY : -INFINITY; fk = -1; }
                        if (en > t_in) { t_in = en; face = fk; }
                        t_out = fminf(t_out, lv);
                    }
                    {
                        float en, lv;
                        int fk;
                        if (e2 > 0.0f) { en = (0.0f - o2) / e2; lv = (Hb - o2) / e2; fk = 5; }
                        else if (e2 < 0.0f) { en = (Hb - o2) / e2; lv = (0.0f - o2) / e2; fk = 4; }
                        else { const bool in = 0.0f < o2 && o2 < Hb; en = in ? -INFINITY : INFINITY; lv = in ? INFINITY : -INFINITY; fk = -1; }
                        if (en > t_in) { t_in = en; face = fk; }
                        t_out = fminf(t_out, lv);
                    }
                    if (!(t_in <= t_out && t_in > 0.0f && t_in < INFINITY)) continue;
                    const float z = t_in * cam.f;
                    if (!(z >= cam.zn && z <= cam.zf)) continue;
                    const unsigned long long key =
                        make_key(1.0f / z, key_word(1u, 6 * (tag >> 8) + face, (uint32_t)tag & 0xFFu));
                    best = key > best ? key : best;
                }
                keys[p] = best;
            }
        }

        // ---- road strips by culling bin: the ground point of each pixel, in
        // sub-bands of rows.  A row's ground points share the depth -h f / b,
        // so a sub-band sees the ground only between the depths of its lowest
        // row and of its highest row below the horizon; bins outside that
        // range are culled as well
        for (int r0 = j0; r0 < j1; r0 += rrows) {
            const int r1 = min(j1, r0 + rrows);
            const float b_low = cam.cy - ((float)(r1 - 1) + 0.5f);
            const int j_top = max(r0, (int)floorf(cam.cy - 0.5f) + 1);
            const float b_top = cam.cy - ((float)j_top + 0.5f);
            const float gz_lo = b_low < 0.0f ? fmaxf(cam.zn, -(cam.h * cam.f) / b_low) : cam.zf;
            const float gz_hi = b_top < 0.0f ? fminf(cam.zf, -(cam.h * cam.f) / b_top) : cam.zf;
            for (int u0 = 0; b_low < 0.0f && u0 < sc.n_bins; u0 += B) {
                __syncthreads();
                if (tid == 0) cnt[0] = 0;
                __syncthreads();
                const int u = u0 + tid;
                if (u < sc.n_bins) {
                    const RoadBin bn = s.bins[sc.bin_base + u];
                    // ground points a sample can show lie at depth [zn, zf] inside the
                    // horizontal frustum; reject bins whose corners are all out on one side
                    const float xs[4] = {bn.xmin, bn.xmax, bn.xmax, bn.xmin}, ys[4] = {bn.ymin, bn.ymin, bn.ymax, bn.ymax};
                    bool nz = true, fz = true, lft = true, rgt = true;
    #pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const float ox = xs[q] - cam.px, oy = ys[q] - cam.py;
                        const float z = fmaf(ox, cam.fx, oy * cam.fy), x = fmaf(ox, cam.fy, -(oy * cam.fx));
                        const float m = 1e-3f * (fabsf(x) + fabsf(z)) + 1e-3f;
                        nz = nz && (z < gz_lo - m);
                        fz = fz && (z > gz_hi + m);
                        rgt = rgt && (x - cam.tx * z > m);
                        lft = lft && (-x - cam.tx * z > m);
                    }
                    if (!(nz || fz || lft || rgt)) {
                        const int q = __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        stg[0 * B + q] = bn.xmin - 1e-2f;
                        stg[1 * B + q] = bn.ymin - 1e-2f;
                        stg[2 * B + q] = bn.xmax + 1e-2f;
                        stg[3 * B + q] = bn.ymax + 1e-2f;
                        istg[4 * B + q] = bn.start;
                        istg[5 * B + q] = bn.count;
                    }
                }
                __syncthreads();
                const int nb = cnt[0];
                if (nb == 0) continue;
                // the staged bins in groups of kRcGroupBins: a group's strips go
                // to LDS (thread k holds strip k mod kBinQuads of bin k / kBinQuads),
                // then every pixel tests them and folds its best road into its
                // key; the largest key over the groups is the lowest road index
                for (int g0 = 0; g0 < nb; g0 += kRcGroupBins) {
                    const int g1 = min(nb, g0 + kRcGroupBins);
                    {
                        const int r = g0 + tid / kBinQuads, q = tid % kBinQuads;
                        if (r < g1 && q < istg[5 * B + r]) {
                            const int g = sc.road_base + istg[4 * B + r] + q;
                            const float4 q0 = s.roads[2 * g], q1 = s.roads[2 * g + 1];
                            sst[0 * B + tid] = q0.x;
                            sst[1 * B + tid] = q0.y;
                            sst[2 * B + tid] = q0.z;
                            sst[3 * B + tid] = q0.w;
                            sst[4 * B + tid] = q1.x;
                            sst[5 * B + tid] = q1.y;
                            sst[6 * B + tid] = q1.z;
                            sst[7 * B + tid] = q1.w;
                            isst[8 * B + tid] = (s.road_index[g] << 8) | (int)s.road_color[g];
                        }
                    }
                    __syncthreads();
                    for (int p = (r0 - j0) * W + tid; p < (r1 - j0) * W; p += B) {
                        const int j = j0 + p / W, i = p - (p / W) * W;
                        float a, b, dx, dy;
                        rc_sample(cam, i, j, a, b, dx, dy);
                        if (!(b < 0.0f)) continue;
                        const float sp = -cam.h / b;
                        const float z = sp * cam.f;
                        if (!(z >= cam.zn && z <= cam.zf)) continue;
                        const float x = fmaf(sp, dx, cam.px), y = fmaf(sp, dy, cam.py);
                        int best = INT32_MAX;          // (road index << 8) | colour of the best strip
                        for (int r = g0; r < g1; ++r) {
                            if (x < stg[r] || y < stg[B + r] || x > stg[2 * B + r] || y > stg[3 * B + r]) continue;
                            const int n = istg[5 * B + r], base = (r - g0) * kBinQuads;
                            for (int q = 0; q < n; ++q) {
                                const int k = base + q;
                                const float qx[4] = {sst[k], sst[2 * B + k], sst[4 * B + k], sst[6 * B + k]};
                                const float qy[4] = {sst[B + k], sst[3 * B + k], sst[5 * B + k], sst[7 * B + k]};
                                int pos = 0, neg = 0;
    #pragma unroll
                                for (int e = 0; e < 4; ++e) {
                                    const int e1 = (e + 1) & 3;
                                    const float ex = qx[e1] - qx[e], ey = qy[e1] - qy[e];
                                    const float wx = x - qx[e], wy = y - qy[e];
                                    const float c = fmaf(ex, wy, -(ey * wx));
                                    pos += c > 0.0f;
                                    neg += c < 0.0f;
                                }
                                const int rc = isst[8 * B + k];
                                if ((pos == 4 || neg == 4) && rc < best) best = rc;
                            }
                        }
                        if (best != INT32_MAX) {
                            const unsigned long long key =
                                make_key(1.0f / z, key_word(0u, 6 * n_box + (best >> 8), (uint32_t)best & 0xFFu));
                            if (key > keys[p]) keys[p] = key;
                        }
                    }
                    __syncthreads();                   // the next group overwrites the strips
                }
            }
        }

        // ---- traffic lights: the raster's sphere test
        for (int u0 = 0; u0 < sc.n_signals; u0 += B) {
            __syncthreads();
            if (tid == 0) cnt[0] = 0;
            __syncthreads();
            const int u = u0 + tid;
            if (u < sc.n_signals) {
                const int g = sc.signal_base + u;
                const float4 q = s.signals[g];
                const float dxw = q.x - cam.px, dyw = q.y - cam.py;
                const float cz = fmaf(dxw, cam.fx, dyw * cam.fy), cxx = fmaf(dxw, cam.fy, -(dyw * cam.fx));
                const float cy = q.z - cam.h;
                const bool keep = !(cz + q.w < cam.zn) && !(cz - q.w > cam.zf) &&
                                  !(fabsf(cxx) - q.w > (cz + q.w) * cam.tx);
                if (keep) {
                    const int k2 = __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    stg[0 * B + k2] = cxx;
                    stg[1 * B + k2] = cy;
                    stg[2 * B + k2] = cz;
                    stg[3 * B + k2] = q.w * q.w;
                    stg[4 * B + k2] = cam.f * cz;
                    istg[5 * B + k2] = (int)key_word(1u, sig0 + u, s.signal_color[g]);
                }
            }
            __syncthreads();
            const int nb = cnt[0];
            const float f = cam.f, ff = f * f;
            for (int p = tid; p < npix; p += B) {
                const int j = j0 + p / W, i = p - (p / W) * W;
                const float a = ((float)i + 0.5f) - cam.cx;
                const float b = cam.cy - ((float)j + 0.5f);
                unsigned long long best = keys[p];
                for (int r = 0; r < nb; ++r) {
                    const float xc = stg[r], yc = stg[B + r], zc = stg[2 * B + r], r2 = stg[3 * B + r], fz = stg[4 * B + r];
                    const float dd = fmaf(a, a, fmaf(b, b, ff));
                    const float dc = fmaf(a, xc, fmaf(b, yc, fz));
                    const float s0 = dc / dd;
                    const float wx = fmaf(-s0, a, xc), wy = fmaf(-s0, b, yc), wz = fmaf(-s0, f, zc);
                    const float qq = r2 - fmaf(wx, wx, fmaf(wy, wy, wz * wz));
                    if (!(qq > 0.0f)) continue;
                    const float z = (s0 - sqrtf(qq / dd)) * f;
                    if (!(z >= cam.zn && z <= cam.zf)) continue;
                    const unsigned long long key = make_key(1.0f / z, (uint32_t)istg[5 * B + r]);
                    best = key > best ? key : best;
                }
                keys[p] = best;
            }
        }
        __syncthreads();

        // ---- resolve the band (as the raster's general kernel)
        const uint32_t q_road = s.shade ? rc_level(s, 0.0f, 0.0f, 4) : 255u;
        for (int p = tid; p < npix; p += B) {
            const unsigned long long key = keys[p];
            const int64_t px = img0 + (int64_t)j0 * W + p;
            uint32_t c = pal[key ? ((uint32_t)key & 0xFFu) : 0u];
            const int prim = key ? (kMaxPrims - 1) - (int)(((uint32_t)key >> 8) & (uint32_t)(kMaxPrims - 1)) : -1;
            if (s.shade && key) {
                if (prim < 6 * n_box) {
                    const int bi = prim / 6, fc = prim - 6 * bi;
                    const float2 cs = s.cs[box_slot(sc, bi)];
                    const float nx = fc == 0 ? cs.x : fc == 1 ? -cs.y : fc == 2 ? -cs.x : cs.y;
                    const float ny = fc == 0 ? cs.y : fc == 1 ? cs.x : fc == 2 ? -cs.y : -cs.x;
                    c = rc_scale(c, rc_level(s, nx, ny, fc));
                } else if (prim < sig0) {
                    c = rc_scale(c, q_road);
                }
            }
            o.rgb[3 * px] = (uint8_t)c;
            o.rgb[3 * px + 1] = (uint8_t)(c >> 8);
            o.rgb[3 * px + 2] = (uint8_t)(c >> 16);
            if (o.depth) o.depth[px] = key ? 1.0f / __uint_as_float((uint32_t)(key >> 32)) : __int_as_float(0x7F800000);
            if (o.primid) o.primid[px] = prim;
        }
        __syncthreads();
    }
}

}  // namespace

size_t raycast_lds_bytes()
{
    return 8 * kRcBandPixels + 4 * kRcStageWords * kRcThreads + 16 + 1024 + 4 * kRcStripWords * kRcThreads;
}

hipError_t launch_raycast(const DevSim &s, const RenderOut &o, int view_begin, int n_views, hipStream_t st)
{
    if (n_views <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_raycast, dim3(n_views), dim3(kRcThreads), raycast_lds_bytes(), st, s, o, view_begin);
    return hipGetLastError();
}

}  // namespace gp
