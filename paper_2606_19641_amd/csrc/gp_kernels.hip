// HIP kernels of the Gigapixel hot path for gfx950 (MI355X).
//
//   k_step         kinematic bicycle step, one thread per agent
//                  (App. A, "Action Space and Dynamics"; dt from App. B)
//   k_step_jerk    jerk-actuated step over the twelve discrete actions
//   k_cs           heading cosines of the current state (after create / set_state)
//   k_infr_flags   collision and off-road checks, one wavefront per agent
//   k_infr_apply   halting of the offenders
//   k_render<0>    general ego-centric raster: rgb + optional depth and
//                  primitive id, any road colours
//   k_render<1>    rgb-only raster for scenes whose road strips share one colour
//                  (Sec. 3.1 O_pixel; App. A "High-Throughput Batched Rendering")
//
// Numerics: every float operation is written out (fmaf for fused operations)
// and the file is compiled with -ffp-contract=off, correctly rounded division
// and IEEE denormals, so each result is a deterministic function of the
// inputs.  Coverage is exact: edge functions are evaluated in fp64 where every
// intermediate is an integer below 2^53, and in int64 otherwise.
//
// Render design, one workgroup per view (persistent work queue or one launch
// per scene):
//   cull    boxes are tested against the view frustum by their bounding
//           cylinder, road strips by the bounding box of their culling bin
//           (<= 64 spatially sorted strips); survivors are compacted with
//           wave ballots into LDS.
//   setup   the faces / strips of the survivors go to camera space, are
//           rejected against the frustum, and those that need no clipping are
//           projected and snapped at once; the rest are clipped in a dense
//           second pass.  Triangles whose bounding box holds a pixel sample
//           are appended to LDS lists (ballot + popcount compaction).
//   raster  per (triangle, pixel row) the exact span of covered samples is
//           computed from the three edge functions.  Road spans of the rgb
//           kernel are OR-ed into a per-row coverage bitmask: all strips lie in
//           one plane, so their depth at a pixel does not depend on the strip,
//           and with one road colour only coverage matters.  Box spans (and
//           every span of the general kernel) give fragments whose 64-bit key
//           (1/z, agent-above-road, lower primitive index, colour) is folded
//           into a band of LDS with atomic max.
//   resolve keys and road coverage become palette colours, stored with packed
//           dword writes (optional depth / primitive id in the general kernel).

#include "gp_device.h"
#include "gp_geom.h"

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

// One bicycle update of agent i from state st (App. A: wheelbase 60% of the
// length; acceleration, speed and steering clipped); returns the curvature.
__device__ __forceinline__ float bicycle(const DevSim &s, int i, float4 st, float L, float accel, float steer)
{
    const float a = fminf(fmaxf(accel, -6.0f), 3.0f);
    const float delta = fminf(fmaxf(steer, -0.5f), 0.5f);
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
    return kappa;
}

__device__ __forceinline__ void step_agent(const DevSim &s, const float2 *act, int i)
{
    if (s.halted[i]) return;                      // halted in place (App. A): state unchanged
    const float2 u = act[i];
    (void)bicycle(s, i, s.state[i], s.dims[i].x, u.x, u.y);
}

__global__ void k_step(DevSim s, const float2 *__restrict__ act, int begin, int count)
{
    const int i = begin + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= begin + count) return;
    step_agent(s, act, i);
}

// batch of sims: sim blockIdx.y, its actions indexed from its first agent
__global__ void k_step_multi(const SimEntry *__restrict__ tab)
{
    const SimEntry &e = tab[blockIdx.y];
    const DevSim s = e.s;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.n_agents) return;
    step_agent(s, e.act, i);
}

// ------------------------------------------------------- jerk actuation
//
// App. A: twelve discrete actions, longitudinal jerk {-15, -4, 0, 4} m/s^3 x
// lateral jerk {-4, 0, 4} m/s^3 (index 3 * lon + lat; any other index coasts
// with both jerks zero).  The jerks integrate into the accelerations (a_lon
// in [-6, 3], |a_lat| <= 4 m/s^2), a_lon into the speed, a_lat into the
// steering angle whose path curvature gives that lateral acceleration
// (tan delta = a_lat l / v^2, l = 0.6 L, v floored at 1 m/s), the angle moving
// at most 0.6 rad/s and staying within 0.5 rad; the pose then follows the
// bicycle.  The actuator record keeps what the vehicle realised: a_lon, or 0
// where the speed clip cancelled it, and v^2 kappa as a_lat.  binary32, every
// fused operation an explicit fmaf.

__constant__ float kJerkLon[4] = {-15.0f, -4.0f, 0.0f, 4.0f};
__constant__ float kJerkLat[3] = {-4.0f, 0.0f, 4.0f};

// atan x for |x| <= tan 0.5 from its Maclaurin series through x^25
// (truncation below 3e-9 there): x + x^3 Q(x^2), Q by Horner in fmaf, each
// coefficient the binary32 quotient 1 / (2k + 1)
__device__ __forceinline__ float atan_small(float x)
{
    const float u = x * x;
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

__global__ void k_step_jerk(DevSim s, const uint8_t *__restrict__ act)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.n_agents || s.halted[i]) return;
    const int k = act[i];
    const float jl = k < 12 ? kJerkLon[k / 3] : 0.0f;
    const float jt = k < 12 ? kJerkLat[k % 3] : 0.0f;
    const float4 st = s.state[i];
    const float4 ac = s.actu[i];
    const float L = s.dims[i].x, l = 0.6f * L;
    const float a_lon = fminf(fmaxf(fmaf(jl, s.dt, ac.x), -6.0f), 3.0f);
    const float a_lat = fminf(fmaxf(fmaf(jt, s.dt, ac.y), -4.0f), 4.0f);
    const float v_free = fmaf(a_lon, s.dt, st.w);
    const float v1 = fminf(fmaxf(v_free, 0.0f), 30.0f);
    const float tan_max = 0.546302497f;      // binary32 nearest to tan 0.5
    const float tau = fminf(fmaxf((a_lat * l) / fmaxf(v1 * v1, 1.0f), -tan_max), tan_max);
    float d1 = fminf(fmaxf(atan_small(tau), fmaf(-0.6f, s.dt, ac.z)), fmaf(0.6f, s.dt, ac.z));
    d1 = fminf(fmaxf(d1, -0.5f), 0.5f);
    const float kappa = bicycle(s, i, st, L, a_lon, d1);
    s.actu[i] = make_float4(v1 == v_free ? a_lon : 0.0f, (v1 * v1) * kappa, d1, 0.0f);
}

__global__ void k_cs(DevSim s, int clear_halted)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.n_boxes) return;                 // agents and static obstacles
    if (clear_halted && i < s.n_agents) {
        s.halted[i] = 0;
        s.actu[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    float sp, cp;
    dev_sincos(s.state[i].z, sp, cp);
    s.cs[i] = make_float2(cp, sp);
}

// ------------------------------------------------------------ infractions
//
// App. A: an agent that collides with another vehicle or leaves the drivable
// area is halted in place (speed zeroed) and keeps being observed.  Readings:
// a collision is a positive-area overlap of two footprints (length x width
// rectangles about the box centres along the headings), tested on the four
// separating axes of the pair, touching not counting; an agent is off-road
// when its centre lies in no road strip of its scene (on or inside each of
// the strip's four edges, either winding).  binary32 with every fused
// operation written as fmaf; heading cos/sin from the state's cosines.

__device__ __forceinline__ float dot2(float ax, float ay, float bx, float by) { return fmaf(ax, bx, ay * by); }

__device__ __forceinline__ float reach(float hl, float hw, float ux, float uy, float ax, float ay)
{
    return fmaf(hl, fabsf(dot2(ux, uy, ax, ay)), hw * fabsf(dot2(-uy, ux, ax, ay)));
}

// Strips' bounding boxes are widened by this much before the exact test: the
// binary32 edge test can only call a point inside when it lies within about
// 1e-5 m of the strip, far inside the margin.
#define GP_STRIP_MARGIN 0.01f

// Flags of every agent into s.infr, one wavefront per agent.  The lanes share
// out the scene's other agents (pair tests) and its culling bins (box tests);
// the strips of the bins whose widened box holds the agent's centre are then
// tested four bins at a time, lane l taking strip l % 16 of hit bin l / 16.
constexpr int kInfrWaves = 4;   // agents per 256-thread workgroup

__device__ __forceinline__ bool footprints_overlap(float4 si, float2 ci, float hli, float hwi, float4 sj,
                                                   float2 cj, float hlj, float hwj)
{
    const float dx = sj.x - si.x, dy = sj.y - si.y;
    const float ax[4] = {ci.x, -ci.y, cj.x, -cj.y}, ay[4] = {ci.y, ci.x, cj.y, cj.x};
    bool sep = false;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float ri = reach(hli, hwi, ci.x, ci.y, ax[e], ay[e]);
        const float rj = reach(hlj, hwj, cj.x, cj.y, ax[e], ay[e]);
        sep = sep | (fabsf(dot2(dx, dy, ax[e], ay[e])) >= ri + rj);
    }
    return !sep;
}

// the centre (x, y) is on or inside every edge of the strip, either winding
__device__ __forceinline__ bool in_strip(float4 q0, float4 q1, float x, float y)
{
    const float qx[4] = {q0.x, q0.z, q1.x, q1.z}, qy[4] = {q0.y, q0.w, q1.y, q1.w};
    bool pos = false, neg = false;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int e1 = (e + 1) & 3;
        const float ex = qx[e1] - qx[e], ey = qy[e1] - qy[e];
        const float wx = x - qx[e], wy = y - qy[e];
        const float c = fmaf(ex, wy, -(ey * wx));
        pos = pos || c > 0.0f;
        neg = neg || c < 0.0f;
    }
    return !(pos && neg);
}

__global__ __launch_bounds__(256) void k_infr_flags(DevSim s)
{
    const int lane = (int)__lane_id();
    const int i = blockIdx.x * kInfrWaves + (int)(threadIdx.x >> 6);   // one agent per wavefront
    if (i >= s.n_agents) return;                                        // the whole wavefront
    const SceneRec sc = s.scenes[s.views[(int64_t)i * s.n_cams].scene];
    const float4 si = s.state[i];
    const float2 ci = s.cs[i];
    const float4 di = s.dims[i];
    const float hli = 0.5f * di.x, hwi = 0.5f * di.y;

    bool col = false;
    for (int j0 = 0; j0 < sc.n_agents && !col; j0 += 64) {
        const int gj = sc.agent_base + j0 + lane;
        bool hit = false;
        if (j0 + lane < sc.n_agents && gj != i) {
            const float4 dj = s.dims[gj];
            hit = footprints_overlap(si, ci, hli, hwi, s.state[gj], s.cs[gj], 0.5f * dj.x, 0.5f * dj.y);
        }
        col = __ballot(hit) != 0ull;
    }
    for (int k0 = 0; k0 < sc.n_static && !col; k0 += 64) {      // static obstacles
        bool hit = false;
        if (k0 + lane < sc.n_static) {
            const int gk = sc.static_base + k0 + lane;
            const float4 dk = s.dims[gk];
            hit = footprints_overlap(si, ci, hli, hwi, s.state[gk], s.cs[gk], 0.5f * dk.x, 0.5f * dk.y);
        }
        col = __ballot(hit) != 0ull;
    }

    bool on = false;
    const int grp = lane >> 4, q = lane & 15;
    for (int b0 = 0; b0 < sc.n_bins && !on; b0 += 64) {
        const int b = b0 + lane;
        bool in = false;
        int start = 0, count = 0;
        if (b < sc.n_bins) {
            const RoadBin bn = s.bins[sc.bin_base + b];
            in = !(si.x < bn.xmin - GP_STRIP_MARGIN || si.x > bn.xmax + GP_STRIP_MARGIN ||
                   si.y < bn.ymin - GP_STRIP_MARGIN || si.y > bn.ymax + GP_STRIP_MARGIN);
            start = bn.start;
            count = bn.count;
        }
        unsigned long long m = __ballot(in);
        while (m != 0ull && !on) {
            // the lowest four hit bins, as lanes of this pass (-1: none)
            int src[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                src[k] = m != 0ull ? __ffsll((long long)m) - 1 : -1;
                m &= m - 1ull;
            }
            const int my = grp == 0 ? src[0] : grp == 1 ? src[1] : grp == 2 ? src[2] : src[3];
            const int st = __shfl(start, my < 0 ? 0 : my), ct = __shfl(count, my < 0 ? 0 : my);
            bool ok = false;
            if (my >= 0 && q < ct) {
                const int g = sc.road_base + st + q;
                ok = in_strip(s.roads[2 * g], s.roads[2 * g + 1], si.x, si.y);
            }
            on = __ballot(ok) != 0ull;
        }
    }
    if (lane == 0) s.infr[i] = (uint8_t)((col ? 1 : 0) | (on ? 0 : 2));
}

// latch halted, zero the speed of halted agents, report flags
__global__ void k_infr_apply(DevSim s, uint8_t *flags_out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s.n_agents) return;
    const uint8_t f = s.infr[i];
    uint8_t h = s.halted[i];
    if (f) {
        h = 1;
        s.halted[i] = 1;
    }
    if (h) s.state[i].w = 0.0f;
    if (flags_out) flags_out[i] = (uint8_t)(f | (h ? 4 : 0));
}

// ------------------------------------------------------------ LDS context

// LDS counters: list lengths, overflow flag, clip-queue and survivor counts,
// pending triangles of the current round (two parities, roads / others), and
// the row range touched by box triangles (rgb kernel)
enum { C_TRIS = 0, C_RTRIS, C_OVF, C_CLIPQ, C_SURV, C_PR0, C_PR1, C_PT0, C_PT1, C_BMIN, C_BMAX, C_CLIPQ1,
       C_NCNT = 16 };

// List capacities: the general kernel keeps every triangle in one list of
// batch_tris entries.  The rgb kernel keeps box triangles (far fewer) in a
// list of batch_tris / 2 entries and road triangles in a list that shares the
// key band's memory: the band is idle while the road list is in use (setup
// ends with a final flush of the road list, and the band-by-band redo after a
// box-list overflow appends no road triangle).
constexpr int kMaxRoadList = 1024;
__host__ __device__ inline void list_caps(int fast, int batch_tris, int band_bytes, int &tcap, int &rcap)
{
    tcap = fast ? max(128, batch_tris / 2) : batch_tris;
    rcap = fast ? min(kMaxRoadList, band_bytes / 32) : 0;
}

struct Lds {
    lptr<TriRec> tris;              // boxes (rgb kernel) or everything (general kernel)
    lptr<TriGeo> rtris;             // road strips (rgb kernel)
    lptr<unsigned long long> zb;    // band of 64-bit keys
    lptr<unsigned long long> road;  // rgb kernel: per-row road coverage bits [H][nw]
    lptr<int32_t> scan;             // [cap + 4] row-count prefix
    lptr<int32_t> surv;             // [B] surviving boxes / bins
    lptr<int32_t> clipq;            // [2][B] candidates that need clipping, a ring per round parity
    lptr<int32_t> cnt;              // counters (C_*)
    lptr<int32_t> wsum;             // [16] per-wave partial sums
    lptr<uint32_t> pal;             // [256] RGB as u32
    lptr<uint32_t> lut;             // rgb kernel: [16][4] the 16 four-pixel road/background
                                    // patterns as 3 packed RGB dwords (+1 pad), 16-byte aligned
    int tcap;                       // capacity of tris
    int rcap;                       // capacity of rtris (rgb kernel)
    int nw;                         // 64-bit words per image row
    __device__ int cap_of(int which) const { return which == C_RTRIS ? rcap : tcap; }
};

// Block-wide exclusive scan of L.scan[0..n) in place; L.scan[n] = total.
// Every thread must call it.
__device__ int block_scan(Lds &L, int n)
{
    const int B = blockDim.x, tid = threadIdx.x;
    const int per = (n + B - 1) / B;
    const int beg = min(n, tid * per), end = min(n, beg + per);
    int local = 0;
    for (int i = beg; i < end; ++i) local += L.scan[i];
    // inclusive scan of `local` across the wave
    int v = local;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o);
        if ((int)lane_id() >= o) v += u;
    }
    const int w = tid >> 6;
    if ((int)lane_id() == 63) L.wsum[w] = v;
    __syncthreads();
    int wbase = 0;
    for (int k = 0; k < w; ++k) wbase += L.wsum[k];
    int run = wbase + v - local;
    for (int i = beg; i < end; ++i) {
        const int c = L.scan[i];
        L.scan[i] = run;
        run += c;
    }
    if (tid == B - 1) L.scan[n] = run;
    __syncthreads();
    return L.scan[n];
}

// index t with scan[t] <= g < scan[t+1]
__device__ __forceinline__ int find_row_owner(const Lds &L, int n, int g)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.scan[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Road strips of the rgb kernel: OR every covered sample into the row bitmask.
__device__ __noinline__ void raster_roads(Lds L, int W, int n)
{
    if (n <= 0) return;
    for (int t = threadIdx.x; t < n; t += blockDim.x) L.scan[t] = L.rtris[t].j1 - L.rtris[t].j0 + 1;
    __syncthreads();
    const int total = block_scan(L, n);
    // row items dealt to the waves in turn, so a partial last pass is shared
    const int nwv = (int)blockDim.x >> 6, wv = (int)threadIdx.x >> 6, ln = (int)lane_id();
    for (int g0 = 0; g0 < total; g0 += blockDim.x) {
        const int gi = g0 + ln * nwv + wv;
        if (gi >= total) continue;
        const int t = find_row_owner(L, n, gi);
        const TriGeo tg = lds_load(L.rtris + t);
        const int j = tg.j0 + (gi - L.scan[t]);
        int xl, xr;
        if (!row_span_banded(tg, j, W, xl, xr)) continue;
        lptr<unsigned long long> row = L.road + (size_t)j * L.nw;
        const int w0 = xl >> 6, w1 = xr >> 6;
        for (int wd = w0; wd <= w1; ++wd) {
            const int lo = (wd == w0) ? (xl & 63) : 0;
            const int hi = (wd == w1) ? (xr & 63) : 63;
            const unsigned long long m = (hi == 63 ? ~0ull : ((1ull << (hi + 1)) - 1ull)) & (~0ull << lo);
            lds_or64(row + wd, m);
        }
    }
    __syncthreads();
}

// Fragments of listed triangles in rows [b0, b1) folded into the key band.
// Row items are dealt to the waves in turn (item g goes to wave g mod the
// wave count); each wave then fills its items' spans together, 64 pixels per
// pass, so a long span is not left to one lane.
__device__ __noinline__ void raster_tris(Lds L, int W, float cx, float cy, int n, int b0, int b1)
{
    if (n <= 0) return;
    const int nwv = (int)blockDim.x >> 6, wv = (int)threadIdx.x >> 6, ln = (int)lane_id();
    // Row counts per triangle and their prefix.  Up to 64 triangles every wave
    // scans them in registers (no barrier); more go through the block scan.
    const bool small = n <= 64;
    int cnt = 0, incl = 0, total;
    if (small) {
        if (ln < n) {
            const int j0 = max((int)L.tris[ln].g.j0, b0), j1 = min((int)L.tris[ln].g.j1, b1 - 1);
            cnt = max(0, j1 - j0 + 1);
        }
        incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(incl, o);
            if (ln >= o) incl += u;
        }
        total = __builtin_amdgcn_readlane(incl, 63);
        if (ln >= n) incl = INT_MAX;
    } else {
        for (int t = threadIdx.x; t < n; t += blockDim.x) {
            const int j0 = max((int)L.tris[t].g.j0, b0), j1 = min((int)L.tris[t].g.j1, b1 - 1);
            L.scan[t] = max(0, j1 - j0 + 1);
        }
        __syncthreads();
        total = block_scan(L, n);
    }
    for (int g0 = 0; g0 < total; g0 += blockDim.x) {
        const int gi = g0 + ln * nwv + wv;
        int t = 0, start = 0;
        if (small) {
            // owner: the number of triangles whose inclusive prefix is <= gi
            // (branchless search over the 64 lanes, every lane active)
#pragma unroll
            for (int step = 32; step > 0; step >>= 1)
                if (__shfl(incl, t + step - 1) <= gi) t += step;
            const int tt = min(t, 63);
            start = __shfl(incl, tt) - __shfl(cnt, tt);
        }
        int xl = 0, xr = -1, j = 0;
        float A = 0.0f, B = 0.0f, Cc = 0.0f;
        uint32_t key = 0u;
        bool has = false;
        if (gi < total) {
            if (!small) {
                t = find_row_owner(L, n, gi);
                start = L.scan[t];
            }
            const TriRec tr = lds_load(L.tris + t);
            j = max((int)tr.g.j0, b0) + (gi - start);
            has = row_span_banded(tr.g, j, W, xl, xr);
            A = tr.A; B = tr.B; Cc = tr.C; key = tr.keylo;
        }
        unsigned long long m = __ballot(has);
        while (m) {
            const int src = __ffsll((long long)m) - 1;
            m &= m - 1ull;
            // src is wave-uniform: read the item out of its lane with scalar reads
            const int sxl = __builtin_amdgcn_readlane(xl, src), sxr = __builtin_amdgcn_readlane(xr, src);
            const int sj = __builtin_amdgcn_readlane(j, src);
            const float sA = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(A), src));
            const float sB = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(B), src));
            const float sC = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(Cc), src));
            const uint32_t skey = (uint32_t)__builtin_amdgcn_readlane((int)key, src);
            const float dv = ((float)sj + 0.5f) - cy;
            lptr<unsigned long long> row = L.zb + (size_t)(sj - b0) * W;
            for (int i = sxl + ln; i <= sxr; i += 64) {
                const float du = ((float)i + 0.5f) - cx;
                const float invz = fmaf(sA, du, fmaf(sB, dv, sC));
                if (!(invz > 0.0f)) continue;
                lds_max64(row + i, ((unsigned long long)__float_as_uint(invz) << 32) | skey);
            }
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------ setup

// How triangles are consumed during a setup pass.
struct Sink {
    int fast;        // rgb kernel: road strips go to the road list
    int flush_tris;  // L.tris may be flushed into the key band [r0, r1)
    int r0, r1;      // rows kept; flushes of L.tris go to this band
};

__device__ __forceinline__ void flush_tris(const Cam &cam, Lds &L, const Sink &K)
{
    raster_tris(L, cam.W, cam.cx, cam.cy, min(L.cnt[C_TRIS], L.tcap), K.r0, K.r1);
    if (threadIdx.x == 0) L.cnt[C_TRIS] = 0;
    __syncthreads();
}

__device__ __forceinline__ void flush_roads(const Cam &cam, Lds &L)
{
    raster_roads(L, cam.W, min(L.cnt[C_RTRIS], L.rcap));
    if (threadIdx.x == 0) L.cnt[C_RTRIS] = 0;
    __syncthreads();
}

// Flush the lists that cannot take `need_r` road / `need_t` other triangles.
// Called by every thread after a barrier.  The decision is read by every
// thread before the second barrier and acted on only after it, so a wave that
// appends right after this call cannot change another wave's decision.
// Returns the road list's length after the call (the same for every thread).
__device__ __forceinline__ int make_room(const Cam &cam, Lds &L, const Sink &K, int need_r, int need_t)
{
    const int cr = L.cnt[C_RTRIS];
    const bool fr = K.fast && cr + need_r > L.rcap;
    const bool ft = K.flush_tris && L.cnt[C_TRIS] + need_t > L.tcap;
    __syncthreads();
    if (fr) flush_roads(cam, L);
    if (ft) flush_tris(cam, L, K);
    return fr ? 0 : cr;
}

// Append with one LDS atomic per wave; lanes whose triangle does not fit
// raise the overflow flag (only possible for a list that cannot be flushed).
__device__ __forceinline__ void append_wave(Lds &L, int which, bool v0, const TriRec &t0, bool v1,
                                            const TriRec &t1)
{
    const unsigned long long b0 = __ballot(v0), b1 = __ballot(v1);
    const int n0 = __popcll(b0), n = n0 + __popcll(b1);
    if (n == 0) return;
    const unsigned long long lt = (1ull << lane_id()) - 1ull;
    const int leader = __ffsll((long long)(b0 | b1)) - 1;
    int base = 0;
    if ((int)lane_id() == leader) {
        base = lds_add(L.cnt + which, n);
        if (base + n > L.cap_of(which)) L.cnt[C_OVF] = 1;
    }
    base = __shfl(base, leader);
    const int p0 = base + __popcll(b0 & lt), p1 = base + n0 + __popcll(b1 & lt);
    if (which == C_RTRIS) {
        if (v0 && p0 < L.rcap) lds_store(L.rtris + p0, t0.g);
        if (v1 && p1 < L.rcap) lds_store(L.rtris + p1, t1.g);
    } else {
        if (v0 && p0 < L.tcap) lds_store(L.tris + p0, t0);
        if (v1 && p1 < L.tcap) lds_store(L.tris + p1, t1);
    }
}

__device__ __forceinline__ void append_one(Lds &L, int which, const TriRec &t)
{
    const int pos = lds_add(L.cnt + which, 1);
    if (pos < L.cap_of(which)) {
        if (which == C_RTRIS) lds_store(L.rtris + pos, t.g);
        else lds_store(L.tris + pos, t);
    } else {
        L.cnt[C_OVF] = 1;
    }
}

// Clip one candidate per 16-lane segment (clip_seg) and append the fan
// triangles to the lists.
__device__ __forceinline__ void clip_wave(const Cam &cam, const Poly &P, bool live, bool road, const Sink &K, Lds &L)
{
    TriRec t;
    const bool ok = clip_seg<true>(cam, P, live, K.r0, K.r1, t);
    append_wave(L, road ? C_RTRIS : C_TRIS, ok, t, false, t);
    if (K.fast && !road && ok) {
        lds_min(L.cnt + C_BMIN, (int)t.g.j0);
        lds_max(L.cnt + C_BMAX, (int)t.g.j1);
    }
}

// Candidate code for the clip queue: boxes j*8 + f, roads -(slot + 1).
__device__ __forceinline__ void build_code(const DevSim &s, const SceneRec &sc, const Cam &cam, int code,
                                           Poly &P)
{
    if (code >= 0) {
        build_face(s, sc, cam, code >> 3, code & 7, P);
    } else {
        const int slot = -code - 1, g = sc.road_base + slot;
        build_road(s, sc, cam, slot, s.roads[2 * g], s.roads[2 * g + 1], P);
    }
}

// One setup pass over boxes (KIND 0) or road bins (KIND 1); FAST selects the
// rgb kernel, where road triangles go to the road list.  Both are template
// parameters so that each pass carries only the records it can emit.
template <int KIND, int FAST>
__device__ void setup_source(const DevSim &s, const SceneRec &sc, const Cam &cam, int ego, const Sink &K,
                             Lds &L)
{
    constexpr int kind = KIND;
    constexpr bool road = FAST && KIND == 1;     // triangles of this pass go to the road list
    const int B = blockDim.x, tid = threadIdx.x;
    const int n_units = kind == 0 ? sc.n_agents + sc.n_static : sc.n_bins;
    const bool can_flush = road || K.flush_tris;
    // the list that may be flushed during this pass, and its capacity; with
    // flushing a round adds at most 2 triangles per lane, so keep it below half
    const int fcap = road ? L.rcap : L.tcap;
    const int per_round = can_flush ? max(1, min(B, fcap / 2)) : B;
    // The clip queue is two rings of B entries, one per round parity, whose
    // counters only grow during a view: a round queues at most B candidates
    // and clips them before the round ends.  A round reads its parity's
    // counter after its last barrier; the next append to that ring comes two
    // rounds later, after the next round's barrier, so every thread reads the
    // same value without a barrier at the end of the round.
    int head0 = L.cnt[C_CLIPQ], head1 = L.cnt[C_CLIPQ1];   // two scalars (no indexed array)
    int r_up = L.cnt[C_RTRIS];                   // bound on the road list's length
    for (int u0 = 0; u0 < n_units; u0 += B) {
        // ---- cull units, compact the survivors
        // survivors are recorded as the agent index (boxes) or as the bin's
        // slot range start * 128 + count (roads)
        const int u = u0 + tid;
        bool keep = false;
        int rec = u;
        if (u < n_units) {
            if (kind == 0) {
                keep = (u != ego) && !box_outside(s, sc, cam, u);
            } else {
                const RoadBin bn = s.bins[sc.bin_base + u];
                keep = !bin_outside(s, cam, bn);
                rec = bn.start * 128 + bn.count;
            }
        }
        if (tid == 0) {
            L.cnt[C_SURV] = 0;
            L.cnt[C_PR0] = L.cnt[C_PR1] = L.cnt[C_PT0] = L.cnt[C_PT1] = 0;
        }
        __syncthreads();
        {
            const unsigned long long bm = __ballot(keep);
            const int nk = __popcll(bm);
            int base = 0;
            if (nk > 0) {
                const int leader = __ffsll((long long)bm) - 1;
                if ((int)lane_id() == leader) base = lds_add(L.cnt + C_SURV, nk);
                base = __shfl(base, leader);
            }
            if (keep) L.surv[base + __popcll(bm & ((1ull << lane_id()) - 1ull))] = rec;
        }
        __syncthreads();
        const int ns = L.cnt[C_SURV];
        const int ncand = kind == 0 ? 6 * ns : kBinQuads * ns;
        // ---- rounds over the candidates of the survivors; the road strips of
        // the next round are fetched while this round is processed
        float4 nq0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), nq1 = nq0;
        auto fetch = [&](int cn) {
            if (kind == 1 && tid < per_round && cn < ncand) {
                const int pk = L.surv[cn / kBinQuads], k = cn % kBinQuads;
                if (k < (pk & 127)) {
                    const int g = sc.road_base + (pk >> 7) + k;
                    nq0 = s.roads[2 * g];
                    nq1 = s.roads[2 * g + 1];
                }
            }
        };
        fetch(tid);
        int par = 0;
        for (int c0 = 0; c0 < ncand; c0 += per_round, par ^= 1) {
            const int c = c0 + tid;
            const float4 q0 = nq0, q1 = nq1;
            if (c0 + per_round < ncand) fetch(c + per_round);
            bool live = tid < per_round && c < ncand;
            int code = 0;
            Poly P;
            if (live) {
                if (kind == 0) {
                    const int j = L.surv[c / 6], f = c - 6 * (c / 6);
                    code = j * 8 + f;
                    build_face(s, sc, cam, j, f, P);
                } else {
                    const int pk = L.surv[c / kBinQuads], k = c % kBinQuads;
                    live = k < (pk & 127);
                    if (live) {
                        const int slot = (pk >> 7) + k;
                        code = -(slot + 1);
                        build_road(s, sc, cam, slot, q0, q1, P);
                    }
                }
            }
            TriRec t0, t1;
            bool v0 = false, v1 = false, clip = false;
            if (live) fast_poly<!road>(cam, P, K.r0, K.r1, t0, v0, t1, v1, clip);
            if (clip) {
                const int q = lds_add(L.cnt + (par ? C_CLIPQ1 : C_CLIPQ), 1);
                L.clipq[par * B + q % B] = code;
            }
            if (can_flush) {
                // While the bound r_up on the road list's length leaves room
                // for two triangles per candidate, the round needs no check
                // (and no barrier); otherwise count this round's triangles and
                // flush first if they would not fit.  r_up is computed from
                // values every thread sees alike, so the choice is uniform.
                if (K.fast && !K.flush_tris && r_up + 2 * per_round <= L.rcap) {
                    r_up += 2 * per_round;
                } else {
                    const int nr = __popcll(__ballot(v0 && road)) + __popcll(__ballot(v1 && road));
                    const int nt = __popcll(__ballot(v0 && !road)) + __popcll(__ballot(v1 && !road));
                    if (lane_id() == 0 && (nr | nt)) {
                        lds_add(L.cnt + C_PR0 + par, nr);
                        lds_add(L.cnt + C_PT0 + par, nt);
                    }
                    __syncthreads();
                    const int pr = L.cnt[C_PR0 + par];
                    r_up = make_room(cam, L, K, pr, L.cnt[C_PT0 + par]) + pr;
                }
                if (tid == 0) { L.cnt[C_PR0 + (par ^ 1)] = 0; L.cnt[C_PT0 + (par ^ 1)] = 0; }
            }
            if (road) append_wave(L, C_RTRIS, v0, t0, v1, t1);
            else append_wave(L, C_TRIS, v0, t0, v1, t1);
            if (FAST && !road) {
                if (v0) { lds_min(L.cnt + C_BMIN, (int)t0.g.j0); lds_max(L.cnt + C_BMAX, (int)t0.g.j1); }
                if (v1) { lds_min(L.cnt + C_BMIN, (int)t1.g.j0); lds_max(L.cnt + C_BMAX, (int)t1.g.j1); }
            }
            __syncthreads();
            // this round's clip candidates are entries [head, tail) of its parity's ring
            const int head = par ? head1 : head0;
            const int tail = L.cnt[par ? C_CLIPQ1 : C_CLIPQ], nq = tail - head;
            // the clipper may emit up to kMaxTrisPerCand triangles per candidate
            const int chunk = can_flush ? max(1, fcap / kMaxTrisPerCand) : B;
            // one 16-lane segment per queued candidate, four per wave
            for (int q0 = 0; q0 < nq; q0 += chunk) {
                const int qn = min(chunk, nq - q0);
                if (can_flush) r_up = make_room(cam, L, K, qn * kMaxTrisPerCand, qn * kMaxTrisPerCand) + qn * kMaxTrisPerCand;
                for (int qb = q0; qb < q0 + qn; qb += B / kClipSeg) {
                    const int q = qb + tid / kClipSeg;
                    const bool live = q < q0 + qn;
                    Poly Q = {};
                    if (live) build_code(s, sc, cam, L.clipq[par * B + (head + q) % B], Q);
                    clip_wave(cam, Q, live, road, K, L);
                }
                __syncthreads();
            }
            if (par) head1 = tail;
            else head0 = tail;
        }
    }
}

// ------------------------------------------------------------ resolve

__device__ __forceinline__ void clear_band(Lds &L, int npix)
{
    for (int p = threadIdx.x; p < npix; p += blockDim.x) L.zb[p] = 0ull;
}

// ------------------------------------------------------------ shading
//
// App. A: one directional light per world, a colour per instance.  With the
// light on, a face with outward unit normal n is lit by
// s = a + (1 - a) max(0, n . l) (l towards the light, world frame, a the
// ambient term), quantised to the level q = floor(255 s + 0.5) in binary32,
// and each channel c of its colour becomes (c q + 127) / 255.  Box normals
// follow the heading cosines (front, left, back, right, top, bottom), road
// strips face up; the background is not lit.  Lit frames are resolved by the
// general kernel only.

__device__ __forceinline__ uint32_t shade_level(const DevSim &s, float nx, float ny, int face)
{
    // the light is read into scalars first: selecting between fields of the
    // kernel-argument record would make the compiler keep it in memory
    const float lx = s.light[0], ly = s.light[1], lz = s.light[2], amb = s.light[3];
    const float side = fmaf(nx, lx, ny * ly);
    const float d = face < 4 ? side : (face == 4 ? lz : -lz);
    const float sh = fmaf(1.0f - amb, fmaxf(d, 0.0f), amb);
    return (uint32_t)fmaf(sh, 255.0f, 0.5f);
}

__device__ __forceinline__ uint32_t shade_rgb(uint32_t c, uint32_t q)
{
    const uint32_t r = ((c & 0xFFu) * q + 127u) / 255u;
    const uint32_t g = (((c >> 8) & 0xFFu) * q + 127u) / 255u;
    const uint32_t b = (((c >> 16) & 0xFFu) * q + 127u) / 255u;
    return r | (g << 8) | (b << 16);
}

// lit colour c of the box face that a winning key names (box and face from
// the key's primitive index)
__device__ __forceinline__ uint32_t lit_box(const DevSim &s, const SceneRec &sc, uint32_t c, unsigned long long key)
{
    const int prim = (kMaxPrims - 1) - (int)(((uint32_t)key >> 8) & (uint32_t)(kMaxPrims - 1));
    const int j = prim / 6, f = prim - 6 * j;
    const float2 cs = s.cs[box_slot(sc, j)];
    const float nx = f == 0 ? cs.x : f == 1 ? -cs.y : f == 2 ? -cs.x : cs.y;
    const float ny = f == 0 ? cs.y : f == 1 ? cs.x : f == 2 ? -cs.y : -cs.x;
    return shade_rgb(c, shade_level(s, nx, ny, f));
}

// rgb kernel: rows [r0, r1) from the road coverage bits and, with keys, the
// box key band whose first row is zb0.
//
// Every road strip shares the depth plane (A, B, C) with A = +-0, so the road
// 1/z of pixel (i, j) is fma(A, du, y) = y for y = fma(B, dv, C) != 0: one
// value per row, positive exactly below the horizon.  A box fragment beats
// the road where its 1/z is not smaller (agents rank above roads on ties).

// colour of a pixel of the rgb kernel: a box fragment wins where its 1/z is
// not below the road's (agents rank above roads on ties); else road or
// background by the coverage bit
template <bool KEYS>
__device__ __forceinline__ uint32_t fast_color(const Lds &L, bool road, float rz, unsigned long long kb,
                                              uint32_t road_rgb, uint32_t bg_rgb)
{
    if (KEYS) {
        // branch-free: both tests combined bitwise, the palette read
        // unconditional (every index is an entry), then one select
        const bool box = (kb != 0ull) & (!road | ((uint32_t)(kb >> 32) >= __float_as_uint(rz)));
        const uint32_t boxc = L.pal[(uint32_t)kb & 0xFFu];
        return box ? boxc : (road ? road_rgb : bg_rgb);
    }
    return road ? road_rgb : bg_rgb;
}

template <bool KEYS>
__device__ __forceinline__ uint32_t fast_pixel(const Cam &cam, const Lds &L, int j, int i, int zb0,
                                              uint32_t road_rgb, uint32_t bg_rgb)
{
    const float dv = ((float)j + 0.5f) - cam.cy;
    const float rz = fmaf(cam.road.B, dv, cam.road.C);
    const bool road = (rz > 0.0f) & (((L.road[(size_t)j * L.nw + (i >> 6)] >> (i & 63)) & 1ull) != 0ull);
    const unsigned long long kb = KEYS ? L.zb[(size_t)(j - zb0) * cam.W + i] : 0ull;
    return fast_color<KEYS>(L, road, rz, kb, road_rgb, bg_rgb);
}

__device__ __forceinline__ void put_rgb(uint8_t *dst, uint32_t c)
{
    dst[0] = (uint8_t)c;
    dst[1] = (uint8_t)(c >> 8);
    dst[2] = (uint8_t)(c >> 16);
}

template <bool KEYS>
__device__ void resolve_fast(const DevSim &s, const Cam &cam, Lds &L, uint8_t *rgb, int64_t view, int r0,
                             int r1, int zb0)
{
    const int W = cam.W;
    const int64_t img = view * (int64_t)W * cam.H;
    const uint32_t road_rgb = L.pal[s.road_color0];
    const uint32_t bg_rgb = L.pal[0];
    if ((W & 3) == 0) {
        const int tpr = W >> 2;                       // threads per row, 4 pixels each
        const int rpi = (int)blockDim.x / tpr;        // rows per pass (W <= 4 * blockDim)
        const int rr = (int)threadIdx.x / tpr, qi = (int)threadIdx.x - rr * tpr;
        if (rr >= rpi) return;
        const int i = 4 * qi;
        for (int j = r0 + rr; j < r1; j += rpi) {
            const float dv = ((float)j + 0.5f) - cam.cy;
            const float rz = fmaf(cam.road.B, dv, cam.road.C);
            const bool rowok = rz > 0.0f;
            const uint32_t bits = rowok ? (uint32_t)(L.road[(size_t)j * L.nw + (i >> 6)] >> (i & 63)) & 0xFu : 0u;
            lptr<unsigned long long> kp = L.zb + (KEYS ? (size_t)(j - zb0) * W + i : 0);
            uint32_t c[4];
#pragma unroll
            for (int m = 0; m < 4; ++m)
                c[m] = fast_color<KEYS>(L, (bits >> m) & 1u, rz, KEYS ? kp[m] : 0ull, road_rgb, bg_rgb);
            uint32_t *out = reinterpret_cast<uint32_t *>(rgb + 3 * (img + (int64_t)j * W + i));
            out[0] = (c[0] & 0xFFFFFFu) | (c[1] << 24);
            out[1] = ((c[1] >> 8) & 0xFFFFu) | (c[2] << 16);
            out[2] = ((c[2] >> 16) & 0xFFu) | (c[3] << 8);
        }
        return;
    }
    // rows are not a whole number of dwords: walk the rows' pixels as one
    // flat run, 4 pixels (3 dwords) per thread; a group may cross a row end.
    // The whole groups need a 4-byte aligned image (W * H a multiple of 4);
    // the partial groups at the run's two ends are written bytewise.
    const int pbeg = r0 * W, pend = r1 * W;
    const bool dwords = ((W * cam.H) & 3) == 0;
    const int g0 = dwords ? (pbeg + 3) >> 2 : 0, g1 = dwords ? pend >> 2 : 0;
    if (g0 < g1) {
        uint32_t *base = reinterpret_cast<uint32_t *>(rgb + 3 * img);
        for (int g = g0 + (int)threadIdx.x; g < g1; g += blockDim.x) {
            int j = (4 * g) / W, i = 4 * g - j * W;
            uint32_t c[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                c[k] = fast_pixel<KEYS>(cam, L, j, i, zb0, road_rgb, bg_rgb);
                if (++i == W) { i = 0; ++j; }
            }
            uint32_t *out = base + 3 * (size_t)g;
            out[0] = (c[0] & 0xFFFFFFu) | (c[1] << 24);
            out[1] = ((c[1] >> 8) & 0xFFFFu) | (c[2] << 16);
            out[2] = ((c[2] >> 16) & 0xFFu) | (c[3] << 8);
        }
        const int head = 4 * g0 - pbeg, tail = pend - 4 * g1;   // 0..3 pixels each
        int p = -1;
        if ((int)threadIdx.x < head) p = pbeg + (int)threadIdx.x;
        else if ((int)threadIdx.x >= 4 && (int)threadIdx.x < 4 + tail) p = 4 * g1 + (int)threadIdx.x - 4;
        if (p >= 0) {
            const int j = p / W, i = p - j * W;
            put_rgb(rgb + 3 * (img + (int64_t)p), fast_pixel<KEYS>(cam, L, j, i, zb0, road_rgb, bg_rgb));
        }
    } else {
        for (int p = pbeg + (int)threadIdx.x; p < pend; p += blockDim.x) {
            const int j = p / W, i = p - j * W;
            put_rgb(rgb + 3 * (img + (int64_t)p), fast_pixel<KEYS>(cam, L, j, i, zb0, road_rgb, bg_rgb));
        }
    }
}

// rgb kernel, rows [r0, r1) that no box fragment touches: the colour of a
// pixel is road or background by its coverage bit alone (the road depth of a
// row is positive exactly below the horizon).  A lane writes 16 pixels, 48
// bytes, as three 16-byte stores assembled from the pattern table.  Needs
// W % 16 == 0, W / 16 <= blockDim.x and a 16-byte aligned image.
__device__ void resolve_rows_lut(const Cam &cam, Lds &L, uint8_t *rgb, int64_t view, int r0, int r1)
{
    const int W = cam.W;
    const int tpr = W >> 4;                       // lanes per row
    const int rpi = (int)blockDim.x / tpr;        // rows per pass
    const int rr = (int)threadIdx.x / tpr, ci = (int)threadIdx.x - rr * tpr;
    if (rr >= rpi) return;
    const int i = ci << 4;
    uint8_t *img = rgb + 3 * (view * (int64_t)W * cam.H);
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    const lptr<u4> lut = (lptr<u4>)L.lut;
    for (int j = r0 + rr; j < r1; j += rpi) {
        const float dv = ((float)j + 0.5f) - cam.cy;
        const float rz = fmaf(cam.road.B, dv, cam.road.C);
        const uint32_t bits = rz > 0.0f ? (uint32_t)(L.road[(size_t)j * L.nw + (i >> 6)] >> (i & 63)) & 0xFFFFu : 0u;
        const u4 a = lut[bits & 15u], b = lut[(bits >> 4) & 15u], c = lut[(bits >> 8) & 15u], d = lut[bits >> 12];
        u4 *out = reinterpret_cast<u4 *>(img + 3 * ((int64_t)j * W + i));
        out[0] = u4{a.x, a.y, a.z, b.x};
        out[1] = u4{b.y, b.z, c.x, c.y};
        out[2] = u4{c.z, d.x, d.y, d.z};
    }
}

// general kernel: key band -> colour (lit when the light is on), depth,
// primitive id.
__device__ void resolve_general(const DevSim &s, const SceneRec &sc, const Cam &cam, Lds &L, const RenderOut &o,
                                int64_t view, int b0, int b1)
{
    const int W = cam.W;
    const int npix = (b1 - b0) * W;
    const int64_t pix0 = view * (int64_t)W * cam.H + (int64_t)b0 * W;
    const uint32_t q_road = s.shade ? shade_level(s, 0.0f, 0.0f, 4) : 255u;
    for (int p = threadIdx.x; p < npix; p += blockDim.x) {
        const unsigned long long key = L.zb[p];
        uint32_t c = L.pal[key ? ((uint32_t)key & 0xFFu) : 0u];
        if (s.shade && key) {
            // boxes hold the primitives below 6 (n_agents + n_static), then
            // come the roads, then the (unlit) traffic lights
            const uint32_t inv = ((uint32_t)key >> 8) & (uint32_t)(kMaxPrims - 1);
            const int n_box = sc.n_agents + sc.n_static;
            if (inv > (uint32_t)(kMaxPrims - 1 - 6 * n_box)) c = lit_box(s, sc, c, key);
            else if (inv > (uint32_t)(kMaxPrims - 1 - 6 * n_box - sc.n_roads)) c = shade_rgb(c, q_road);
        }
        uint8_t *dst = o.rgb + 3 * (pix0 + p);
        dst[0] = (uint8_t)c;
        dst[1] = (uint8_t)(c >> 8);
        dst[2] = (uint8_t)(c >> 16);
        if (o.depth) {
            const float invz = __uint_as_float((uint32_t)(key >> 32));
            o.depth[pix0 + p] = key ? 1.0f / invz : __int_as_float(0x7F800000);
        }
        if (o.primid)
            o.primid[pix0 + p] = key ? (int32_t)(kMaxPrims - 1) - (int32_t)(((uint32_t)key >> 8) & (kMaxPrims - 1)) : -1;
    }
}

// ------------------------------------------------------------ traffic lights
//
// Sec. 3.1: traffic lights are small spheres.  The sample of pixel (i, j)
// casts the ray s D, D = (a, b, f), a = i + 0.5 - cx, b = cy - (j + 0.5); it
// meets a sphere of camera-space centre c and radius r when, at the closest
// approach s0 = (D . c) / (D . D), the miss w = c - s0 D has w . w < r^2; the
// fragment is the near hit at planar depth z = (s0 - sqrt((r^2 - w . w) /
// (D . D))) f, kept for z_near <= z <= z_far.  binary32 with fmaf and
// correctly rounded division and square root.  Lights rank with the boxes on
// depth ties, are numbered after the roads and are not lit (emissive).

// Conservative pixel bounds of the sphere's part in [z_near, z_far]: the
// projection of its bounding box, widened by a pixel; false if none.
__device__ __forceinline__ bool signal_bounds(const Cam &cam, const V3 &c, float r, int &i0, int &i1, int &j0,
                                              int &j1)
{
    if (c.z + r < cam.zn || c.z - r > cam.zf) return false;
    const float zlo = fmaxf(c.z - r, cam.zn), zhi = fminf(c.z + r, cam.zf);
    const float xm = c.x - r, xM = c.x + r, ym = c.y - r, yM = c.y + r;
    const float xr0 = xm >= 0.0f ? xm / zhi : xm / zlo, xr1 = xM >= 0.0f ? xM / zlo : xM / zhi;
    const float yr0 = ym >= 0.0f ? ym / zhi : ym / zlo, yr1 = yM >= 0.0f ? yM / zlo : yM / zhi;
    const float u0 = fmaf(cam.f, xr0, cam.cx), u1 = fmaf(cam.f, xr1, cam.cx);
    const float v0 = fmaf(-cam.f, yr1, cam.cy), v1 = fmaf(-cam.f, yr0, cam.cy);
    const float Wf = (float)cam.W, Hf = (float)cam.H;
    i0 = max((int)fminf(fmaxf(floorf(u0 - 0.5f) - 1.0f, -1.0f), Wf), 0);
    i1 = min((int)fminf(fmaxf(ceilf(u1 - 0.5f) + 1.0f, -1.0f), Wf), cam.W - 1);
    j0 = max((int)fminf(fmaxf(floorf(v0 - 0.5f) - 1.0f, -1.0f), Hf), 0);
    j1 = min((int)fminf(fmaxf(ceilf(v1 - 0.5f) + 1.0f, -1.0f), Hf), cam.H - 1);
    return i0 <= i1 && j0 <= j1;
}

// Lights of the scene into the key band of rows [b0, b1), in chunks staged
// through the setup's survivor and clip-queue space (free during the band
// pass): 8 words per light, one array per word.
__device__ void raster_signals(const DevSim &s, const SceneRec &sc, const Cam &cam, Lds &L, int b0, int b1)
{
    const int B = blockDim.x, tid = threadIdx.x, W = cam.W;
    const int cap = (12 * B) / 32;
    lptr<float> fr = (lptr<float>)L.surv;              // xc, yc, zc, r^2, f zc: fr[k * cap + g]
    lptr<int32_t> ir = L.surv + 5 * cap;               // key word, (i0, j0), (i1, j1)
    const int sig0 = 6 * (sc.n_agents + sc.n_static) + sc.n_roads;
    const float f = cam.f, ff = f * f;
    for (int g0 = 0; g0 < sc.n_signals; g0 += cap) {
        const int ng = min(cap, sc.n_signals - g0);
        __syncthreads();
        if (tid < ng) {
            const int g = sc.signal_base + g0 + tid;
            const float4 q = s.signals[g];
            const V3 c = to_cam(cam, q.x - cam.px, q.y - cam.py, q.z);
            int i0, i1, j0, j1;
            const bool vis = signal_bounds(cam, c, q.w, i0, i1, j0, j1);
            j0 = max(j0, b0);
            j1 = min(j1, b1 - 1);
            const bool keep = vis && j0 <= j1;
            fr[tid] = c.x;
            fr[cap + tid] = c.y;
            fr[2 * cap + tid] = c.z;
            fr[3 * cap + tid] = q.w * q.w;
            fr[4 * cap + tid] = f * c.z;
            ir[tid] = (int32_t)key_low(1u, sig0 + g0 + tid, s.signal_color[g]);
            ir[cap + tid] = keep ? (i0 | (j0 << 16)) : 1;           // empty: i0 > i1
            ir[2 * cap + tid] = keep ? (i1 | (j1 << 16)) : 0;
        }
        __syncthreads();
        for (int k = 0; k < ng; ++k) {
            const int p0 = ir[cap + k], p1 = ir[2 * cap + k];
            const int i0 = p0 & 0xFFFF, j0 = p0 >> 16, i1 = p1 & 0xFFFF, j1 = p1 >> 16;
            if (i0 > i1) continue;
            const float xc = fr[k], yc = fr[cap + k], zc = fr[2 * cap + k], r2 = fr[3 * cap + k], fz = fr[4 * cap + k];
            const uint32_t keylo = (uint32_t)ir[k];
            const int w = i1 - i0 + 1, n = w * (j1 - j0 + 1);
            for (int p = tid; p < n; p += B) {
                const int dj = p / w, i = i0 + (p - dj * w), j = j0 + dj;
                const float a = ((float)i + 0.5f) - cam.cx;
                const float b = cam.cy - ((float)j + 0.5f);
                const float dd = fmaf(a, a, fmaf(b, b, ff));
                const float dc = fmaf(a, xc, fmaf(b, yc, fz));
                const float s0 = dc / dd;
                const float wx = fmaf(-s0, a, xc), wy = fmaf(-s0, b, yc), wz = fmaf(-s0, f, zc);
                const float qq = r2 - fmaf(wx, wx, fmaf(wy, wy, wz * wz));
                if (!(qq > 0.0f)) continue;
                const float z = (s0 - sqrtf(qq / dd)) * f;
                if (!(z >= cam.zn && z <= cam.zf)) continue;
                const float invz = 1.0f / z;
                lds_max64(L.zb + (size_t)(j - b0) * W + i, ((unsigned long long)__float_as_uint(invz) << 32) | keylo);
            }
        }
    }
}

// ------------------------------------------------------------ per view

__device__ __forceinline__ void reset_counts(Lds &L)
{
    const int t = threadIdx.x;
    if (t < C_NCNT) L.cnt[t] = (t == C_BMIN) ? 0x7FFFFFFF : (t == C_BMAX ? -1 : 0);
}

// KIND 0: general kernel; 1: rgb kernel; 2: general kernel with traffic
// lights (their code lives in its own instances so that it does not add to
// the registers of the other two)
template <int KIND>
__device__ void render_view(const DevSim &s, const RenderOut &o, const LaunchCfg &lc, Lds &L, int view)
{
    constexpr int FAST = KIND == 1 ? 1 : 0;
    // the view's records are the same for the whole workgroup: scalar registers
    const int scene = __builtin_amdgcn_readfirstlane(s.views[view].scene);
    const int ego_cam = __builtin_amdgcn_readfirstlane(s.views[view].ego_cam);
    const SceneRec sc = uniform_scene(s.scenes[scene]);
    const int ego = ego_cam >> 2, k = ego_cam & 3;
    const Cam cam = make_cam(s, sc, ego, k);
    const int H = cam.H, W = cam.W, BR = lc.band_rows;
    reset_counts(L);
    if (FAST) {
        for (int p = threadIdx.x; p < H * L.nw; p += blockDim.x) L.road[p] = 0ull;
    }
    __syncthreads();
    Sink K;
    K.fast = FAST;
    K.flush_tris = 0;
    K.r0 = 0;
    K.r1 = H;
    setup_source<0, FAST>(s, sc, cam, ego, K, L);           // boxes
    setup_source<1, FAST>(s, sc, cam, ego, K, L);           // road strips
    if (FAST) flush_roads(cam, L);
    const bool overflow = L.cnt[C_OVF] != 0;
    const int ntri = min(L.cnt[C_TRIS], L.tcap);
    // rows that need the key band: every row for the general kernel; for the
    // rgb kernel the rows touched by box triangles (all rows after an overflow)
    int kr0 = 0, kr1 = H;
    if (FAST && !overflow) {
        kr0 = min(L.cnt[C_BMIN], H);
        kr1 = max(L.cnt[C_BMAX] + 1, kr0);
    }
    __syncthreads();
    if (FAST) {
        if ((W & 15) == 0 && (W >> 4) <= (int)blockDim.x && ((uintptr_t)o.rgb & 15) == 0) {
            resolve_rows_lut(cam, L, o.rgb, view, 0, kr0);
            resolve_rows_lut(cam, L, o.rgb, view, kr1, H);
        } else {
            resolve_fast<false>(s, cam, L, o.rgb, view, 0, kr0, 0);
            resolve_fast<false>(s, cam, L, o.rgb, view, kr1, H, 0);
        }
    }
    for (int b0 = kr0; b0 < kr1; b0 += BR) {
        const int b1 = min(kr1, b0 + BR);
        clear_band(L, (b1 - b0) * W);
        __syncthreads();
        if (!overflow) {
            raster_tris(L, cam.W, cam.cx, cam.cy, ntri, b0, b1);
        } else {
            // the list did not hold every triangle: redo this band's setup
            // with flushes into the band
            reset_counts(L);
            __syncthreads();
            Sink KB;
            KB.fast = FAST;
            KB.flush_tris = 1;
            KB.r0 = b0;
            KB.r1 = b1;
            setup_source<0, FAST>(s, sc, cam, ego, KB, L);
            if (!FAST) setup_source<1, FAST>(s, sc, cam, ego, KB, L);
            flush_tris(cam, L, KB);
        }
        if (KIND == 2 && sc.n_signals > 0) {
            raster_signals(s, sc, cam, L, b0, b1);
            __syncthreads();
        }
        if (FAST) resolve_fast<true>(s, cam, L, o.rgb, view, b0, b1, b0);
        else resolve_general(s, sc, cam, L, o, view, b0, b1);
        __syncthreads();
    }
}

// LDS layout of a render workgroup for W x H images (sizes as render_lds_bytes)
__device__ __forceinline__ void carve_lds(unsigned char *smem, Lds &L, int W, int H, const LaunchCfg &lc, int fast)
{
    list_caps(fast, lc.batch_tris, 8 * lc.band_rows * W, L.tcap, L.rcap);
    L.nw = (W + 63) >> 6;
    size_t off = 0;
    L.tris = (lptr<TriRec>)(smem + off);
    off += sizeof(TriRec) * (size_t)L.tcap;
    L.zb = (lptr<unsigned long long>)(smem + off);
    L.rtris = (lptr<TriGeo>)(smem + off);       // rgb kernel: shares the band's memory
    off += 8u * (size_t)lc.band_rows * W;
    L.road = (lptr<unsigned long long>)(smem + off);
    off += fast ? 8u * (size_t)H * L.nw : 0;
    L.scan = (lptr<int32_t>)(smem + off);
    off += 4u * (size_t)(max(L.tcap, L.rcap) + 4);
    L.surv = (lptr<int32_t>)(smem + off);
    off += 4u * blockDim.x;
    L.clipq = (lptr<int32_t>)(smem + off);
    off += 8u * blockDim.x;
    L.cnt = (lptr<int32_t>)(smem + off);
    off += 4u * 16;
    L.wsum = (lptr<int32_t>)(smem + off);
    off += 4u * 16;
    L.pal = (lptr<uint32_t>)(smem + off);
    off += 4u * 256;
    off = (off + 15) & ~(size_t)15;
    L.lut = (lptr<uint32_t>)(smem + off);
}

// The sim's palette, and for the rgb kernel its road/background pattern
// table, into LDS; published by the caller's next barrier.
__device__ __forceinline__ void load_palette(const DevSim &s, Lds &L, int fast)
{
    for (int p = threadIdx.x; p < 256; p += blockDim.x)
        L.pal[p] = (uint32_t)s.palette[3 * p] | ((uint32_t)s.palette[3 * p + 1] << 8) |
                   ((uint32_t)s.palette[3 * p + 2] << 16);
    if (fast && threadIdx.x < 16) {
        // pattern b: pixel k is road where bit k of b is set, background elsewhere
        auto rgb_of = [&](int idx) -> uint32_t {
            return (uint32_t)s.palette[3 * idx] | ((uint32_t)s.palette[3 * idx + 1] << 8) |
                   ((uint32_t)s.palette[3 * idx + 2] << 16);
        };
        const uint32_t road = rgb_of(s.road_color0), bg = rgb_of(0);
        const int b = threadIdx.x;
        const uint32_t c0 = (b & 1) ? road : bg, c1 = (b & 2) ? road : bg;
        const uint32_t c2 = (b & 4) ? road : bg, c3 = (b & 8) ? road : bg;
        L.lut[4 * b + 0] = c0 | (c1 << 24);
        L.lut[4 * b + 1] = (c1 >> 8) | (c2 << 16);
        L.lut[4 * b + 2] = (c2 >> 16) | (c3 << 8);
        L.lut[4 * b + 3] = 0u;
    }
}

// BLOCK is the launch's block size: the bound lets the register allocator
// use what a BLOCK-thread workgroup can have instead of assuming 1024 threads.
template <int KIND, int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(BLOCK == 256 ? 3 : 1))) void k_render(DevSim s, RenderOut o, LaunchCfg lc, int persistent,
                                                  int view_begin)
{
    constexpr int FAST = KIND == 1 ? 1 : 0;
    extern __shared__ __align__(16) unsigned char smem[];
    Lds L;
    carve_lds(smem, L, s.width, s.height, lc, FAST);
    load_palette(s, L, FAST);
    __shared__ int s_item;
    if (!persistent) {
        __syncthreads();
        render_view<KIND>(s, o, lc, L, view_begin + blockIdx.x);
        return;
    }
    int cur = (int)(blockIdx.x % kQueues);       // thread 0's current segment
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = queue_take(s, cur);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= s.n_views) break;
        render_view<KIND>(s, o, lc, L, s.queue[it]);
    }
    if (threadIdx.x == 0) queue_leave(s);
}


// Batched render over several sims (serving): items are (sim, view) pairs,
// workgroups pull them from one queue.  ctl[0] is the queue head, ctl[1]
// counts the workgroups that have left; the last one zeroes both.  Every sim
// of the batch has W x H images; the palette is reloaded when the sim changes.
template <int KIND, int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(BLOCK == 256 ? 3 : 1))) void k_render_multi(const SimEntry *__restrict__ tab,
                                                        const int2 *__restrict__ items, int n_items,
                                                        uint32_t *ctl, LaunchCfg lc, int W, int H)
{
    constexpr int FAST = KIND == 1 ? 1 : 0;
    extern __shared__ __align__(16) unsigned char smem[];
    Lds L;
    carve_lds(smem, L, W, H, lc, FAST);
    __shared__ int s_item;
    int cur = -1;                                 // sim whose palette is in LDS
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(&ctl[0], 1u);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= n_items) break;
        const int2 item = items[it];
        const int k = __builtin_amdgcn_readfirstlane(item.x), view = __builtin_amdgcn_readfirstlane(item.y);
        // the sim's record is read in place (a local copy of it would be
        // indexed by camera and live in scratch memory)
        const DevSim &s = tab[k].s;
        const RenderOut o = tab[k].o;
        if (k != cur) {
            load_palette(s, L, FAST);
            cur = k;
            __syncthreads();
        }
        render_view<KIND>(s, o, lc, L, view);
    }
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t done = atomicAdd(&ctl[1], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&ctl[0], 0u);
            atomicExch(&ctl[1], 0u);
            __threadfence();
        }
    }
}

// ------------------------------------------------------------ launchers

size_t render_lds_bytes(int width, int height, const LaunchCfg &c, int fast)
{
    int tcap, rcap;
    list_caps(fast, c.batch_tris, 8 * c.band_rows * width, tcap, rcap);
    const size_t nw = (size_t)(width + 63) / 64;
    size_t b = sizeof(TriRec) * (size_t)tcap +
               8u * (size_t)c.band_rows * width + 4u * (size_t)(max(tcap, rcap) + 4) +
               12u * (size_t)c.block_threads + 64u + 64u + 1024u + 16u + 256u;
    if (fast) b += 8u * (size_t)height * nw;
    return b;
}

size_t render_lds_bytes(const DevSim &s, const LaunchCfg &c, int fast)
{
    return render_lds_bytes(s.width, s.height, c, fast);
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

hipError_t step_graph_node(hipGraph_t g, hipGraphExec_t exec, hipGraphNode_t *node, const DevSim &s,
                           const float *actions)
{
    const int B = 256;
    DevSim sv = s;
    const float2 *act = reinterpret_cast<const float2 *>(actions);
    int begin = 0, count = s.n_agents;
    void *args[] = {&sv, &act, &begin, &count};
    hipKernelNodeParams p{};
    p.func = reinterpret_cast<void *>(k_step);
    p.gridDim = dim3((count + B - 1) / B);
    p.blockDim = dim3(B);
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    p.extra = nullptr;
    if (exec) return hipGraphExecKernelNodeSetParams(exec, *node, &p);
    return hipGraphAddKernelNode(node, g, nullptr, 0, &p);
}

hipError_t launch_step_jerk(const DevSim &s, const uint8_t *actions, hipStream_t st)
{
    if (s.n_agents <= 0) return hipSuccess;
    const int B = 256;
    hipLaunchKernelGGL(k_step_jerk, dim3((s.n_agents + B - 1) / B), dim3(B), 0, st, s, actions);
    return hipGetLastError();
}

hipError_t launch_step_multi(const SimEntry *tab, int n_sims, int max_agents, hipStream_t st)
{
    if (n_sims <= 0 || max_agents <= 0) return hipSuccess;
    const int B = 256;
    hipLaunchKernelGGL(k_step_multi, dim3((max_agents + B - 1) / B, n_sims), dim3(B), 0, st, tab);
    return hipGetLastError();
}

hipError_t launch_render_multi(const SimEntry *tab, const int2 *items, int n_items, uint32_t *ctl,
                               const LaunchCfg &c, int kind, int width, int height, int grid, hipStream_t st)
{
    if (n_items <= 0 || grid <= 0) return hipSuccess;
    const size_t lds = render_lds_bytes(width, height, c, kind == 1);
#define GP_LAUNCH(F, B)                                                                                 \
    hipLaunchKernelGGL((k_render_multi<F, B>), dim3(grid), dim3(B), lds, st, tab, items, n_items, ctl, c, width, height)
    switch (c.block_threads) {
    case 256:
        if (kind == 1) GP_LAUNCH(1, 256); else if (kind == 2) GP_LAUNCH(2, 256); else GP_LAUNCH(0, 256);
        break;
    case 512:
        if (kind == 1) GP_LAUNCH(1, 512); else if (kind == 2) GP_LAUNCH(2, 512); else GP_LAUNCH(0, 512);
        break;
    case 1024:
        if (kind == 1) GP_LAUNCH(1, 1024); else if (kind == 2) GP_LAUNCH(2, 1024); else GP_LAUNCH(0, 1024);
        break;
    default:
        return hipErrorInvalidValue;
    }
#undef GP_LAUNCH
    return hipGetLastError();
}

hipError_t launch_cs(const DevSim &s, int clear_halted, hipStream_t st)
{
    const int B = 256;
    hipLaunchKernelGGL(k_cs, dim3((s.n_boxes + B - 1) / B), dim3(B), 0, st, s, clear_halted);
    return hipGetLastError();
}

hipError_t launch_infractions(const DevSim &s, int max_agents, uint8_t *flags_out, hipStream_t st)
{
    if (s.n_agents <= 0) return hipSuccess;
    const int B = 256;
    (void)max_agents;
    hipLaunchKernelGGL(k_infr_flags, dim3((s.n_agents + kInfrWaves - 1) / kInfrWaves), dim3(B), 0, st, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_infr_apply, dim3((s.n_agents + B - 1) / B), dim3(B), 0, st, s, flags_out);
    return hipGetLastError();
}

hipError_t launch_render(const DevSim &s, const RenderOut &o, const LaunchCfg &c, int kind,
                         int persistent, int view_begin, int grid, hipStream_t st)
{
    if (grid <= 0) return hipSuccess;
    const size_t lds = render_lds_bytes(s, c, kind == 1);
#define GP_LAUNCH(F, B)                                                                                 \
    hipLaunchKernelGGL((k_render<F, B>), dim3(grid), dim3(B), lds, st, s, o, c, persistent, view_begin)
    switch (c.block_threads) {
    case 256:
        if (kind == 1) GP_LAUNCH(1, 256); else if (kind == 2) GP_LAUNCH(2, 256); else GP_LAUNCH(0, 256);
        break;
    case 512:
        if (kind == 1) GP_LAUNCH(1, 512); else if (kind == 2) GP_LAUNCH(2, 512); else GP_LAUNCH(0, 512);
        break;
    case 1024:
        if (kind == 1) GP_LAUNCH(1, 1024); else if (kind == 2) GP_LAUNCH(2, 1024); else GP_LAUNCH(0, 1024);
        break;
    default:
        return hipErrorInvalidValue;
    }
#undef GP_LAUNCH
    return hipGetLastError();
}

}  // namespace gp
