// Chip-wide rgb raster of the Gigapixel hot path for gfx950 (MI355X).
//
// The rgb-only ego-centric render (Sec. 3.1 O_pixel; App. A "High-Throughput
// Batched Rendering": one world per ego agent, all views rendered together)
// for sims whose road strips share one colour and renders that need neither
// depth nor primitive ids.  Its images are bit-identical to the other
// rasterisers and to the plain definition (same clip, snap, fill rule and
// winner order); only the division of the work differs.  No view's work is a
// serial chain on one compute unit: three passes each spread their items
// over the whole chip.
//   1 setup    workgroups of sixteen wavefronts for eight views.  For each
//              view one wavefront tests the scene's road culling bins against
//              it (frustum, road depth limit, row gap) and lists the
//              survivors; another culls the boxes, sets up and clips their
//              faces and writes the view's box triangle list and its row
//              range.  The workgroup then reserves its views' road items (four
//              surviving bins each) in a global list with one device atomic.
//   2 roads    the road items are dealt to the wavefronts in turn.  An item's
//              strips meet the cheap test; survivors are set up (snap, the two
//              fan triangles, or the clipper); the exact span of covered
//              samples of every (triangle, row) is OR-ed into the view's road
//              coverage bitmask in global memory with device atomics (a few KB
//              per view).
//   3 resolve  (view, rows) items dealt to the wavefronts in turn: whole
//              image rows, one group of 16 pixels per lane.  Rows no box
//              triangle touches come from the table of the sixteen four-pixel
//              road/background patterns; rows with box triangles stage the
//              triangles that reach them, compute every (triangle, row) span
//              once and fold each pixel's 64-bit key in registers.  Each lane
//              writes its 48 bytes with three 16-byte stores and clears the
//              coverage words it consumed, so the next render starts from
//              zero.
// Work is dealt statically: a device-scope atomic on one address serialises
// across the XCDs (about 10 ns each), so per-item work counters would cost
// more than the work.
// Every float operation is written out (fmaf for fused operations) and the
// file is compiled with -ffp-contract=off, correctly rounded division and
// IEEE denormals.

#include "gp_device.h"
#include "gp_geom.h"

namespace gp {

namespace {

constexpr int kUnitBins = 4;          // culling bins per road item (64 strip slots)
constexpr int kRoadStage = 128;       // road triangles staged per wavefront
constexpr int kMaxItemRows = 16;      // rows of a resolve item (64 lanes, at least 4 groups per row)
// coverage words of a resolve item: floor(64 / G) rows of ceil(G / 4) words for
// G >= 4 groups of 16 samples per row, at most 16 + 64 / G <= 32
constexpr int kItemWords = 32;

// ------------------------------------------------------------ pass 1: setup

// the view of setup workgroup b / resolve view index vi
__device__ __forceinline__ int view_of(const DevSim &s, int mode, int view_begin, int i)
{
    return mode == 0 ? view_begin + i : s.order[i];
}

// The view's surviving bins listed; returns their number.
__device__ __forceinline__ int setup_bins(const DevSim &s, const ChipBufs &cb, const SceneRec &sc, const Cam &cam,
                                          int view)
{
    const int ln = (int)lane_id();
    int32_t *sb = cb.sbins + (size_t)view * cb.bins_stride;
    int nsb = 0;
    for (int b0 = 0; b0 < sc.n_bins; b0 += 64) {
        const int b = b0 + ln;
        bool keep = false;
        int rec = 0;
        if (b < sc.n_bins) {
            const RoadBin bn = s.bins[sc.bin_base + b];
            float x[4], z[4];
            ground_xz(cam, bn.xmin, bn.ymin, x[0], z[0]);
            ground_xz(cam, bn.xmax, bn.ymin, x[1], z[1]);
            ground_xz(cam, bn.xmax, bn.ymax, x[2], z[2]);
            ground_xz(cam, bn.xmin, bn.ymax, x[3], z[3]);
            keep = !road_culled<true>(cam, x, z);
            rec = bn.start * 128 + bn.count;
        }
        const unsigned long long bm = __ballot(keep);
        if (keep) sb[nsb + lanes_below(bm)] = rec;
        nsb += __popcll(bm);
    }
    if (ln == 0) {
        reinterpret_cast<int32_t *>(cb.vinfo + view)[0] = nsb;
        cb.rinfo[view] = make_int4(0, 0, 0, 0);      // the road pass appends from here
    }
    return nsb;
}

__device__ __forceinline__ void track_rows(const TriRec &t, int &bmin, int &bmax)
{
    bmin = min(bmin, (int)t.g.j0);
    bmax = max(bmax, (int)t.g.j1);
}

// Every box of the scene but the ego culled; the faces of the survivors set
// up (fast path or the clipper, four faces per wavefront) into the view's
// box triangle list.  A list that would exceed its capacity is marked
// overflowed (-1); the resolve pass then sets the boxes up again per item.
__device__ __forceinline__ void setup_boxes(const DevSim &s, const ChipBufs &cb, const SceneRec &sc, const Cam &cam,
                                            int ego, int view, lptr<int32_t> surv, lptr<int32_t> cq)
{
    const int ln = (int)lane_id();
    TriRec *out = reinterpret_cast<TriRec *>(cb.btri) + (size_t)view * cb.btri_cap;
    const int cap = cb.btri_cap;
    const int nbox = sc.n_agents + sc.n_static;
    int nbt = 0, bmin = 0x7FFFFFFF, bmax = -1;
    bool ovf = false;
    for (int b0 = 0; b0 < nbox && !ovf; b0 += 64) {
        const int jb = b0 + ln;
        const bool keep = jb < nbox && jb != ego && !box_outside(s, sc, cam, jb);
        const unsigned long long bm = __ballot(keep);
        if (keep) surv[lanes_below(bm)] = jb;
        const int ns = __popcll(bm);
        wave_lds_order();
        for (int c0 = 0; c0 < 6 * ns && !ovf; c0 += 64) {
            const int c = c0 + ln;
            const bool live = c < 6 * ns;
            int j = 0, f = 0;
            if (live) {
                j = surv[c / 6];
                f = c - 6 * (c / 6);
            }
            Poly P;
            TriRec t0, t1;
            bool v0 = false, v1 = false, clip = false;
            if (live) {
                build_face(s, sc, cam, j, f, P);
                fast_poly<true>(cam, P, 0, cam.H, t0, v0, t1, v1, clip);
            }
            const unsigned long long m0 = __ballot(v0), m1 = __ballot(v1), mc = __ballot(clip);
            const int n0 = __popcll(m0), nf = n0 + __popcll(m1), ncl = __popcll(mc);
            if (nbt + nf > cap) {
                ovf = true;
                break;
            }
            if (v0) {
                out[nbt + lanes_below(m0)] = t0;
                track_rows(t0, bmin, bmax);
            }
            if (v1) {
                out[nbt + n0 + lanes_below(m1)] = t1;
                track_rows(t1, bmin, bmax);
            }
            nbt += nf;
            if (clip) cq[lanes_below(mc)] = j * 8 + f;
            wave_lds_order();
            for (int q0 = 0; q0 < ncl; q0 += 4) {
                const int q = q0 + (ln >> 4);
                const bool lv = q < ncl;
                Poly Q = {};
                if (lv) {
                    const int code = cq[q];
                    build_face(s, sc, cam, code >> 3, code & 7, Q);
                }
                TriRec t;
                const bool ok = clip_seg<true>(cam, Q, lv, 0, cam.H, t);
                const unsigned long long mo = __ballot(ok);
                if (nbt + __popcll(mo) > cap) {
                    ovf = true;
                    break;
                }
                if (ok) {
                    out[nbt + lanes_below(mo)] = t;
                    track_rows(t, bmin, bmax);
                }
                nbt += __popcll(mo);
            }
            wave_lds_order();
        }
        wave_lds_order();
    }
    bmin = wave_min(bmin);
    bmax = wave_max(bmax);
    if (ln == 0) {
        int32_t *vi = reinterpret_cast<int32_t *>(cb.vinfo + view);
        vi[1] = ovf ? -1 : nbt;
        vi[2] = bmin;
        vi[3] = bmax;
    }
}

constexpr int kSetupViews = 8;   // views per setup workgroup (wavefronts 0..7 bins, 8..15 boxes)

__global__ __launch_bounds__(64 * 2 * kSetupViews) void k_chip_setup(DevSim s, ChipBufs cb, int mode, int view_begin,
                                                                    int n_views)
{
    __shared__ int32_t s_surv[kSetupViews][64];
    __shared__ int32_t s_cq[kSetupViews][64];
    __shared__ int32_t s_nu[kSetupViews];
    __shared__ int32_t s_base[kSetupViews];
    const int wv = (int)(threadIdx.x >> 6), ln = (int)lane_id();
    const int slot = wv % kSetupViews;
    const int vi = (int)blockIdx.x * kSetupViews + slot;
    const bool has = vi < n_views;
    int view = 0;
    if (has) {
        view = view_of(s, mode, view_begin, vi);
        const int scene = __builtin_amdgcn_readfirstlane(s.views[view].scene);
        const int ego_cam = __builtin_amdgcn_readfirstlane(s.views[view].ego_cam);
        const SceneRec sc = uniform_scene(s.scenes[scene]);
        const Cam cam = make_cam(s, sc, ego_cam >> 2, ego_cam & 3);
        if (wv < kSetupViews) {
            const int nsb = setup_bins(s, cb, sc, cam, view);
            if (ln == 0) s_nu[slot] = (nsb + kUnitBins - 1) / kUnitBins;
        } else {
            setup_boxes(s, cb, sc, cam, ego_cam >> 2, view, (lptr<int32_t>)&s_surv[slot][0],
                        (lptr<int32_t>)&s_cq[slot][0]);
        }
    } else if (wv < kSetupViews && ln == 0) {
        s_nu[slot] = 0;
    }
    __syncthreads();
    // one device atomic per workgroup reserves the road items of its views
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int k = 0; k < kSetupViews; ++k) {
            s_base[k] = tot;
            tot += s_nu[k];
        }
        const int base = tot > 0 ? (int)atomicAdd(&cb.ctl[CHIP_NITEMS], (uint32_t)tot) : 0;
        for (int k = 0; k < kSetupViews; ++k) s_base[k] += base;
    }
    __syncthreads();
    if (has && wv < kSetupViews) {
        const int nu = s_nu[slot], base = s_base[slot];
        for (int u = ln; u < nu; u += 64) cb.items[base + u] = make_uint2((uint32_t)view, (uint32_t)u);
    }
}

// ------------------------------------------------------------ pass 2: roads

// OR the samples [xl, xr] of one row into its coverage words (global)
__device__ __forceinline__ void or_span_g(unsigned long long *row, int xl, int xr)
{
    const int w0 = xl >> 6, w1 = xr >> 6;
    for (int w = w0; w <= w1; ++w) {
        const int lo = (w == w0) ? (xl & 63) : 0;
        const int hi = (w == w1) ? (xr & 63) : 63;
        const unsigned long long m = (hi == 63 ? ~0ull : ((1ull << (hi + 1)) - 1ull)) & (~0ull << lo);
        __hip_atomic_fetch_or(row + w, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Rasterise the n staged road triangles into the view's coverage words: lane
// t takes the first row of triangle t, then the further rows of the
// triangles that span several are dealt to the lanes by a prefix over their
// counts; per (triangle, row) the exact span of covered samples is OR-ed in.
__device__ __forceinline__ void road_spans_g(unsigned long long *cov, int nw, const Cam &cam, lptr<TriGeo> tris,
                                             int n)
{
    const int ln = (int)lane_id();
    wave_lds_order();
    for (int t0 = 0; t0 < n; t0 += 64) {
        const int t = t0 + ln;
        int c = 0;
        if (t < n) {
            const int32_t jj = ((lptr<const int32_t>)(tris + t))[6];     // j0 | j1 << 16
            c = (jj >> 16) - (int)(int16_t)(jj & 0xFFFF);
        }
        const int incl = wave_incl_scan(c);
        const int total = __builtin_amdgcn_readlane(incl, 63);
        const int excl = incl - c;
        for (int g0 = -64; g0 < total; g0 += 64) {
            // g0 < 0: lane t's own first row; then the dealt further rows
            const int gi = g0 + ln;
            int o = ln, extra = 0;
            bool act = t < n;
            if (g0 >= 0) {
                o = owner_of(incl, gi);
                extra = 1 + gi - __shfl(excl, o);
                act = gi < total;
            }
            if (act) {
                const TriGeo tg = lds_load(tris + t0 + o);
                const int j = tg.j0 + extra;
                int xl, xr;
                if (row_span(tg, j, cam.W, xl, xr)) or_span_g(cov + (size_t)j * nw, xl, xr);
            }
        }
    }
    wave_lds_order();
}

// Append the n staged road triangles to the view's list (one device atomic on
// the view's own counter); triangles past the list's capacity are rasterised
// into the view's coverage words instead, and the view marked as using them.
__device__ __forceinline__ void append_tris(const ChipBufs &cb, const Cam &cam, int view, lptr<TriGeo> tris, int n)
{
    const int ln = (int)lane_id();
    int32_t *cnt = reinterpret_cast<int32_t *>(cb.rinfo + view);
    int base = 0;
    if (ln == 0) base = atomicAdd(cnt, n);
    base = __builtin_amdgcn_readfirstlane(__shfl(base, 0));
    const int nfit = min(max(cb.rtri_cap - base, 0), n);
    TriGeo *out = reinterpret_cast<TriGeo *>(cb.rtri) + (size_t)view * cb.rtri_cap;
    int32_t *rows = cb.rrows + (size_t)view * cb.rtri_cap;
    for (int t = ln; t < nfit; t += 64) {
        const TriGeo tg = lds_load(tris + t);
        out[base + t] = tg;
        rows[base + t] = ((lptr<const int32_t>)(tris + t))[6];
    }
    if (nfit < n) {
        if (ln == 0) cnt[1] = 1;
        road_spans_g(cb.cov + (size_t)view * cam.H * cb.nw, cb.nw, cam, tris + nfit, n - nfit);
    }
}

// stage the triangles held by the lanes (v0: t0, v1: t1); returns how many
__device__ __forceinline__ int stage2(lptr<TriGeo> tris, bool v0, const TriGeo &t0, bool v1, const TriGeo &t1)
{
    const unsigned long long b0 = __ballot(v0), b1 = __ballot(v1);
    const int n0 = __popcll(b0);
    if (v0) lds_store(tris + lanes_below(b0), t0);
    if (v1) lds_store(tris + n0 + lanes_below(b1), t1);
    return n0 + __popcll(b1);
}

// One road item: the strips of four surviving bins of one view.
__device__ __forceinline__ void road_item(const DevSim &s, const ChipBufs &cb, int view, int u, lptr<TriGeo> tris,
                                          lptr<int32_t> clipq)
{
    const int ln = (int)lane_id();
    const int scene = __builtin_amdgcn_readfirstlane(s.views[view].scene);
    const int ego_cam = __builtin_amdgcn_readfirstlane(s.views[view].ego_cam);
    const SceneRec sc = uniform_scene(s.scenes[scene]);
    const Cam cam = make_cam(s, sc, ego_cam >> 2, ego_cam & 3);
    const int nsb = __builtin_amdgcn_readfirstlane(reinterpret_cast<const int32_t *>(cb.vinfo + view)[0]);
    const int32_t *sb = cb.sbins + (size_t)view * cb.bins_stride;
    const int bi = kUnitBins * u + (ln >> 4), k = ln & 15;
    bool live = false;
    int g = 0;
    V3 v[4] = {};
    if (bi < nsb) {
        const int pk = sb[bi];
        live = k < (pk & 127);
        if (live) {
            g = sc.road_base + (pk >> 7) + k;
            road_corners(s, cam, g, v);
        }
    }
    float x[4], z[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        x[q] = v[q].x;
        z[q] = v[q].z;
    }
    const bool pass = live && !road_culled<false>(cam, x, z);
    const bool clip = pass && needs_clip(cam, v);
    TriGeo t0 = {}, t1 = {};
    bool v0 = false, v1 = false;
    if (pass && !clip) {
        int32_t X[4], Y[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) snap(cam, v[q], X[q], Y[q]);
        v0 = make_tri(cam, false, X[0], Y[0], X[1], Y[1], X[2], Y[2], 0, cam.H, t0);
        v1 = make_tri(cam, false, X[0], Y[0], X[2], Y[2], X[3], Y[3], 0, cam.H, t1);
    }
    const unsigned long long mc = __ballot(clip);
    if (clip) clipq[lanes_below(mc)] = g;
    const int ncl = __popcll(mc);
    const int n = stage2(tris, v0, t0, v1, t1);
    if (n > 0) append_tris(cb, cam, view, tris, n);
    // strips that need the clipper: four per wavefront, one per 16-lane segment
    for (int q0 = 0; q0 < ncl; q0 += 4) {
        const int q = q0 + (ln >> 4);
        const bool lv = q < ncl;
        Poly P = {};
        if (lv) road_corners(s, cam, clipq[q], P.v);
        P.n = dir_to_cam(cam, 0.0f, 0.0f, 1.0f);
        P.one_sided = false;
        P.keylo = 0u;
        TriRec t;
        const bool ok = clip_seg<false>(cam, P, lv, 0, cam.H, t);
        const TriGeo none = {};
        const int m = stage2(tris, ok, t.g, false, none);
        if (m > 0) append_tris(cb, cam, view, tris, m);
    }
}

__global__ __launch_bounds__(256) void k_chip_roads(DevSim s, ChipBufs cb)
{
    __shared__ __align__(16) TriGeo s_tris[4][kRoadStage];
    __shared__ int32_t s_clip[4][64];
    const int wv = (int)(threadIdx.x >> 6), ln = (int)lane_id();
    lptr<TriGeo> tris = (lptr<TriGeo>)&s_tris[wv][0];
    lptr<int32_t> clipq = (lptr<int32_t>)&s_clip[wv][0];
    (void)ln;
    // the items are dealt to the wavefronts in turn (no work counter: a
    // device-scope atomic on one address serialises across the XCDs)
    const uint32_t total = (uint32_t)__builtin_amdgcn_readfirstlane((int)cb.ctl[CHIP_NITEMS]);
    const uint32_t nwaves = 4u * gridDim.x;
    for (uint32_t pos = 4u * blockIdx.x + (uint32_t)wv; pos < total; pos += nwaves) {
        const uint2 it = cb.items[pos];
        road_item(s, cb, __builtin_amdgcn_readfirstlane((int)it.x), __builtin_amdgcn_readfirstlane((int)it.y), tris,
                  clipq);
    }
}

// ------------------------------------------------------------ pass 3: resolve

constexpr int kTilesPerGroup = 16;     // resolve items (tiles) of one workgroup, all of one view
constexpr int kRoadChunk = 256;        // entries of the view's road list staged per round
constexpr int kBoxCap = 128;           // box triangles a view's list holds (the host's capacity)
constexpr int kBoxBatch = 32;          // box triangles folded per batch

// What the resolve needs of a view's camera beyond its triangle lists: the
// image size, the principal point and the road's depth plane.  Every camera
// is level, so the road plane is the same in every view: make_cam computes
// 1/z = A du + B dv + C with A and C zeros (of either sign) and B = -1 / (f d),
// d = -h.  The sign of a zero cannot change a decision here (1/z of the road
// is compared only where it is positive), so the values below, computed with
// make_cam's operations, decide exactly as make_cam's plane does.
struct RCam {
    float cx, cy, rB, rC;
    int W, H;
};

__device__ __forceinline__ RCam resolve_cam(const DevSim &s)
{
    RCam c;
    c.W = s.width;
    c.H = s.height;
    c.cx = 0.5f * (float)s.width;
    c.cy = 0.5f * (float)s.height;
    const float d = 0.0f - s.cam_height;
    const float fd = s.focal * d;
    c.rB = -1.0f / fd;
    c.rC = 0.0f;
    return c;
}

// A lane's share of a tile: row j (tile row lr), samples i .. i + 15.
struct Px {
    int lr, j, i;
    bool act;
    float dv, du0;
};

__device__ __forceinline__ Px lane_px(const RCam &rc, int G, int r0, int nrows)
{
    const int ln = (int)lane_id();
    Px p;
    p.lr = ln / G;
    p.act = p.lr < nrows;
    p.j = r0 + min(p.lr, nrows - 1);
    p.i = (ln - p.lr * G) << 4;
    p.dv = ((float)p.j + 0.5f) - rc.cy;
    p.du0 = ((float)p.i + 0.5f) - rc.cx;
    return p;
}

// per-wavefront LDS
struct WaveLds {
    lptr<unsigned long long> bits;   // [4][kItemWords] road coverage of the wavefront's tiles, nw words per row
    lptr<int32_t> idx;               // [64] staged triangles that reach the current tile
    lptr<TriRec> tri;                // [kBoxBatch] box faces set up per tile (views whose list overflowed)
    lptr<int32_t> q;                 // [64] box faces waiting for the clipper (same)
    lptr<unsigned long long> keys;   // [1024] the tile's 64-bit keys, (row - r0) * W + sample
};

// OR the samples [xl, xr] of one row into its coverage words (LDS)
__device__ __forceinline__ void or_span_l(lptr<unsigned long long> row, int xl, int xr)
{
    const int w0 = xl >> 6, w1 = xr >> 6;
    for (int w = w0; w <= w1; ++w) {
        const int lo = (w == w0) ? (xl & 63) : 0;
        const int hi = (w == w1) ? (xr & 63) : 63;
        const unsigned long long m = (hi == 63 ? ~0ull : ((1ull << (hi + 1)) - 1ull)) & (~0ull << lo);
        lds_or64(row + w, m);
    }
}

// The spans of the n road triangles sr[idx[0..n)] on rows [r0, r0 + nrows)
// OR-ed into the tile's coverage words: the (triangle, row) pairs inside each
// triangle's rows are dealt to the lanes by a prefix over their counts.
__device__ __forceinline__ void road_rows(lptr<const TriGeo> sr, lptr<const int32_t> idx, int n,
                                          lptr<unsigned long long> bits, int W, int nw, int r0, int nrows)
{
    const int ln = (int)lane_id();
    wave_lds_order();
    int c = 0, a = 0, tix = 0;
    if (ln < n) {
        tix = idx[ln];
        const int32_t jj = ((lptr<const int32_t>)(sr + tix))[6];
        a = max((int)(int16_t)(jj & 0xFFFF), r0);
        c = max(0, min(jj >> 16, r0 + nrows - 1) - a + 1);
    }
    const int incl = wave_incl_scan(c);
    const int total = __builtin_amdgcn_readlane(incl, 63);
    const int excl = incl - c;
    for (int g0 = 0; g0 < total; g0 += 64) {
        const int gi = g0 + ln;
        // every lane takes part in the shuffles; lanes past the total idle after
        const int o = owner_of(incl, gi);
        const int j = __shfl(a, o) + (gi - __shfl(excl, o));
        const int t = __shfl(tix, o);
        if (gi < total) {
            const TriGeo tg = lds_load(sr + t);
            int xl, xr;
            if (row_span(tg, j, W, xl, xr)) or_span_l(bits + (j - r0) * nw, xl, xr);
        }
    }
    wave_lds_order();
}

// Fold n box triangles (tris[idx[c]] for c < n, or tris[c] without idx) into
// the tile's key band: the spans of every (triangle, tile row) pair are cut
// into pieces of up to 16 samples, the pieces dealt to the lanes by a prefix
// over their counts, and each lane folds its piece's samples into the band
// with LDS atomic max.
__device__ __forceinline__ void fold_tris(const WaveLds &L, lptr<const TriRec> tris, lptr<const int32_t> idx, bool use_idx,
                                          int n, int W, float cx, float cy, int r0, int nrows)
{
    const int ln = (int)lane_id();
    wave_lds_order();
    for (int p0 = 0; p0 < n * nrows; p0 += 64) {
        const int pi = p0 + ln;
        int xl = 0, xr = -1, tc = 0, rr = 0;
        if (pi < n * nrows) {
            tc = pi / nrows;
            rr = pi - tc * nrows;
            const int t = use_idx ? idx[tc] : tc;
            const TriGeo tg = lds_load((lptr<const TriGeo>)(tris + t));
            const int jr = r0 + rr;
            if (!(jr >= tg.j0 && jr <= tg.j1 && row_span(tg, jr, W, xl, xr))) {
                xl = 0;
                xr = -1;
            }
        }
        const int np = (xr - xl + 16) >> 4;            // pieces of up to 16 samples (0 if empty)
        const int incl = wave_incl_scan(np);
        const int total = __builtin_amdgcn_readlane(incl, 63);
        const int excl = incl - np;
        for (int q0 = 0; q0 < total; q0 += 64) {
            const int q = q0 + ln;
            const int o = owner_of(incl, q);
            const int k = q - __shfl(excl, o);
            const int sxl = __shfl(xl, o), sxr = __shfl(xr, o), srr = __shfl(rr, o), stc = __shfl(tc, o);
            if (q < total) {
                const int t = use_idx ? idx[stc] : stc;
                typedef float f4v __attribute__((ext_vector_type(4)));
                const f4v pk = *(lptr<const f4v>)((lptr<const unsigned char>)(tris + t) + 32);   // A B C keylo
                const float dv = ((float)(r0 + srr) + 0.5f) - cy;
                const float bdv = fmaf(pk.y, dv, pk.z);
                const uint32_t keylo = __float_as_uint(pk.w);
                const int i0 = sxl + 16 * k, i1 = min(i0 + 15, sxr);
                lptr<unsigned long long> row = L.keys + srr * W;
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    const int i = i0 + m;
                    const float invz = fmaf(pk.x, ((float)i + 0.5f) - cx, bdv);
                    if (i <= i1 && invz > 0.0f)
                        lds_max64(row + i, ((unsigned long long)__float_as_uint(invz) << 32) | keylo);
                }
            }
        }
    }
    wave_lds_order();
}

// stage the lanes' triangles (ok) into L.tri, kBoxBatch at a time, folding each batch
__device__ __forceinline__ void stage_fold(const WaveLds &L, bool ok, const TriRec &t, int W, float cx, float cy,
                                           int r0, int nrows)
{
    const unsigned long long m = __ballot(ok);
    const int n = __popcll(m), rank = lanes_below(m);
    for (int b = 0; b < n; b += kBoxBatch) {
        if (ok && rank >= b && rank < b + kBoxBatch) lds_store(L.tri + (rank - b), t);
        fold_tris(L, (lptr<const TriRec>)L.tri, L.idx, false, min(kBoxBatch, n - b), W, cx, cy, r0, nrows);
    }
}

// The box fragments of rows [r0, r0 + nrows) set up from the scene (views
// whose triangle list overflowed): every face of every box but the ego,
// triangles kept only where they reach these rows.
__device__ __forceinline__ void boxes_from_scene(const WaveLds &L, const DevSim &s, const SceneRec &sc,
                                                 const Cam &cam, int ego, int r0, int nrows)
{
    const int ln = (int)lane_id();
    const int r1 = r0 + nrows;
    const int ncand = 6 * (sc.n_agents + sc.n_static);
    for (int c0 = 0; c0 < ncand; c0 += 64) {
        const int c = c0 + ln;
        const int jb = c / 6, f = c - 6 * jb;
        const bool live = c < ncand && jb != ego && !box_outside(s, sc, cam, jb);
        Poly P;
        TriRec t0, t1;
        bool v0 = false, v1 = false, clip = false;
        if (live) {
            build_face(s, sc, cam, jb, f, P);
            fast_poly<true>(cam, P, r0, r1, t0, v0, t1, v1, clip);
        }
        stage_fold(L, v0, t0, cam.W, cam.cx, cam.cy, r0, nrows);
        stage_fold(L, v1, t1, cam.W, cam.cx, cam.cy, r0, nrows);
        const unsigned long long mc = __ballot(clip);
        if (clip) L.q[lanes_below(mc)] = jb * 8 + f;
        const int ncl = __popcll(mc);
        wave_lds_order();
        for (int q0 = 0; q0 < ncl; q0 += 4) {
            const int q = q0 + (ln >> 4);
            const bool lv = q < ncl;
            Poly Q = {};
            if (lv) {
                const int code = L.q[q];
                build_face(s, sc, cam, code >> 3, code & 7, Q);
            }
            TriRec t;
            const bool ok = clip_seg<true>(cam, Q, lv, r0, r1, t);
            stage_fold(L, ok, t, cam.W, cam.cx, cam.cy, r0, nrows);
        }
        wave_lds_order();
    }
}

typedef uint32_t u4 __attribute__((ext_vector_type(4)));

// One workgroup renders up to kTilesPerGroup tiles of one view (a tile: the
// rows that 64 lanes of 16 samples cover).  The view's road and box triangles
// that reach the group's rows are staged in LDS once; then each wavefront
// builds its tiles' road coverage from them and resolves the tiles.
__global__ __launch_bounds__(256) void k_chip_resolve(DevSim s, RenderOut o, ChipBufs cb, int mode, int view_begin,
                                                      int n_views, int groups_per_view)
{
    __shared__ uint32_t s_pal[256];
    __shared__ __align__(16) uint32_t s_lut[64];
    __shared__ __align__(16) TriGeo s_sr[kRoadChunk];
    __shared__ __align__(16) TriRec s_sb[kBoxCap];
    __shared__ int32_t s_cnt[2];
    __shared__ unsigned long long s_bits[4][4][kItemWords];
    __shared__ int32_t s_idx[4][64];
    __shared__ __align__(16) TriRec s_tri[4][kBoxBatch];
    __shared__ int32_t s_q[4][64];
    __shared__ unsigned long long s_keys[4][1024];
    const int tid = (int)threadIdx.x, wv = tid >> 6, ln = (int)lane_id();
    // the road pass has read the item count: zero it for the next render
    // (a plain store; no memset node in a captured graph)
    if (blockIdx.x == 0 && tid == 0) cb.ctl[CHIP_NITEMS] = 0u;
    auto rgb_of = [&](int k) -> uint32_t {
        return (uint32_t)s.palette[3 * k] | ((uint32_t)s.palette[3 * k + 1] << 8) |
               ((uint32_t)s.palette[3 * k + 2] << 16);
    };
    for (int k = tid; k < 256; k += 256) s_pal[k] = rgb_of(k);
    if (tid < 16) {
        // pattern b: pixel k is road where bit k of b is set, background elsewhere
        const uint32_t road = rgb_of(s.road_color0), bg = rgb_of(0);
        const uint32_t c0 = (tid & 1) ? road : bg, c1 = (tid & 2) ? road : bg;
        const uint32_t c2 = (tid & 4) ? road : bg, c3 = (tid & 8) ? road : bg;
        s_lut[4 * tid + 0] = c0 | (c1 << 24);
        s_lut[4 * tid + 1] = (c1 >> 8) | (c2 << 16);
        s_lut[4 * tid + 2] = (c2 >> 16) | (c3 << 8);
        s_lut[4 * tid + 3] = 0u;
    }
    if (tid < 2) s_cnt[tid] = 0;
    __syncthreads();        // the counters are zero before any wavefront stages
    WaveLds L;
    L.bits = (lptr<unsigned long long>)&s_bits[wv][0][0];
    L.idx = (lptr<int32_t>)&s_idx[wv][0];
    L.tri = (lptr<TriRec>)&s_tri[wv][0];
    L.q = (lptr<int32_t>)&s_q[wv][0];
    L.keys = (lptr<unsigned long long>)&s_keys[wv][0];
    lptr<TriGeo> sr = (lptr<TriGeo>)s_sr;
    lptr<TriRec> sb = (lptr<TriRec>)s_sb;

    // the group: views fastest (neighbouring workgroups take neighbouring views)
    const int vi = (int)(blockIdx.x % (uint32_t)n_views), grp = (int)(blockIdx.x / (uint32_t)n_views);
    const int view = __builtin_amdgcn_readfirstlane(view_of(s, mode, view_begin, vi));
    const RCam rc = resolve_cam(s);
    const int W = rc.W, H = rc.H, G = W >> 4, R = cb.rows_per_item, nw = cb.nw;
    const int t_begin = grp * kTilesPerGroup;
    const int n_tiles = min(kTilesPerGroup, cb.items_per_view - t_begin);
    const int g_r0 = t_begin * R, g_r1 = min((t_begin + n_tiles) * R, H) - 1;
    const int4 ri = cb.rinfo[view];
    const int nrt = min(__builtin_amdgcn_readfirstlane(ri.x), cb.rtri_cap);
    const bool covused = __builtin_amdgcn_readfirstlane(ri.y) != 0;
    const int4 vinf = cb.vinfo[view];
    const int nbt = __builtin_amdgcn_readfirstlane(vinf.y);
    const int bmin = __builtin_amdgcn_readfirstlane(vinf.z), bmax = __builtin_amdgcn_readfirstlane(vinf.w);
    const TriGeo *rlist = reinterpret_cast<const TriGeo *>(cb.rtri) + (size_t)view * cb.rtri_cap;
    const int32_t *rrows = cb.rrows + (size_t)view * cb.rtri_cap;

    // this wavefront's tiles: wv, wv + 4, ...; clear their coverage and OR in
    // the coverage words of a view whose road list overflowed (clearing those
    // for the next render)
    const int my_tiles = n_tiles > wv ? (n_tiles - wv + 3) / 4 : 0;
    for (int k = ln; k < 4 * kItemWords; k += 64) L.bits[k] = 0ull;
    wave_lds_order();
    if (covused) {
        for (int k = 0; k < my_tiles; ++k) {
            const int r0 = (t_begin + wv + 4 * k) * R, nrows = min(R, H - r0);
            const Px p = lane_px(rc, G, r0, nrows);
            if (p.act && (p.i & 63) == 0) {
                unsigned long long *cw = cb.cov + ((size_t)view * H + p.j) * nw + (p.i >> 6);
                const unsigned long long w = *cw;
                if (w != 0ull) {
                    lds_or64(L.bits + k * kItemWords + p.lr * nw + (p.i >> 6), w);
                    *cw = 0ull;
                }
            }
        }
    }
    // stage the box triangles that reach the group's rows
    if (nbt > 0) {
        const TriRec *blist = reinterpret_cast<const TriRec *>(cb.btri) + (size_t)view * cb.btri_cap;
        for (int t0 = 64 * wv; t0 < nbt; t0 += 256) {
            const int t = t0 + ln;
            bool in = false;
            if (t < nbt) {
                const int32_t jj = reinterpret_cast<const int32_t *>(blist + t)[6];
                in = (int)(int16_t)(jj & 0xFFFF) <= g_r1 && (jj >> 16) >= g_r0;
            }
            const unsigned long long m = __ballot(in);
            int base = 0;
            if (m != 0ull && ln == 0) base = lds_add((lptr<int32_t>)&s_cnt[1], __popcll(m));
            base = __shfl(base, 0);
            if (in) lds_store(sb + base + lanes_below(m), blist[t]);
        }
    }
    // the road list in rounds of kRoadChunk entries: stage the triangles that
    // reach the group's rows, then every wavefront adds them to its tiles
    for (int c0 = 0;; c0 += kRoadChunk) {
        {
            const int t = c0 + tid;
            bool in = false;
            if (t < nrt) {
                const int32_t jj = rrows[t];
                in = (int)(int16_t)(jj & 0xFFFF) <= g_r1 && (jj >> 16) >= g_r0;
            }
            const unsigned long long m = __ballot(in);
            int base = 0;
            if (m != 0ull && ln == 0) base = lds_add((lptr<int32_t>)&s_cnt[0], __popcll(m));
            base = __shfl(base, 0);
            if (in) lds_store(sr + base + lanes_below(m), rlist[t]);
        }
        __syncthreads();
        const int nsr = s_cnt[0];
        for (int k = 0; k < my_tiles; ++k) {
            const int r0 = (t_begin + wv + 4 * k) * R, nrows = min(R, H - r0), rl = r0 + nrows - 1;
            for (int s0 = 0; s0 < nsr; s0 += 64) {
                const int t = s0 + ln;
                bool in = false;
                if (t < nsr) {
                    const int32_t jj = ((lptr<const int32_t>)(sr + t))[6];
                    in = ((int)(int16_t)(jj & 0xFFFF) <= rl) & ((jj >> 16) >= r0);
                }
                const unsigned long long m = __ballot(in);
                if (m == 0ull) continue;
                if (in) L.idx[lanes_below(m)] = t;
                road_rows((lptr<const TriGeo>)sr, (lptr<const int32_t>)L.idx, __popcll(m),
                          L.bits + k * kItemWords, W, nw, r0, nrows);
            }
        }
        __syncthreads();
        if (c0 + kRoadChunk >= nrt) break;
        if (tid == 0) s_cnt[0] = 0;
        __syncthreads();
    }
    const int nsb = s_cnt[1];

    // resolve this wavefront's tiles
    const uint32_t road_rgb = s_pal[s.road_color0], bg_rgb = s_pal[0];
    for (int k = 0; k < my_tiles; ++k) {
        const int r0 = (t_begin + wv + 4 * k) * R, nrows = min(R, H - r0), rl = r0 + nrows - 1;
        const Px p = lane_px(rc, G, r0, nrows);
        const unsigned long long word = p.act ? L.bits[k * kItemWords + p.lr * nw + (p.i >> 6)] : 0ull;
        const float rz = fmaf(rc.rB, p.dv, rc.rC);
        const uint32_t bits = rz > 0.0f ? (uint32_t)(word >> (p.i & 63)) & 0xFFFFu : 0u;
        u4 *out = reinterpret_cast<u4 *>(o.rgb + 3 * ((int64_t)view * W * H + (int64_t)p.j * W + p.i));
        if (nbt == 0 || (nbt > 0 && (bmax < r0 || bmin > rl))) {
            // no box fragment here: the pattern table
            const lptr<u4> lut = (lptr<u4>)s_lut;
            const u4 a = lut[bits & 15u], b = lut[(bits >> 4) & 15u], c = lut[(bits >> 8) & 15u], d = lut[bits >> 12];
            if (p.act) {
                out[0] = u4{a.x, a.y, a.z, b.x};
                out[1] = u4{b.y, b.z, c.x, c.y};
                out[2] = u4{c.z, d.x, d.y, d.z};
            }
            continue;
        }
        // the tile's key band starts empty (1024 keys, 16 per lane)
        {
            typedef unsigned long long u2v __attribute__((ext_vector_type(2)));
#pragma unroll
            for (int m = 0; m < 8; ++m) ((lptr<u2v>)L.keys)[64 * m + ln] = u2v{0ull, 0ull};
        }
        if (nbt > 0) {
            for (int s0 = 0; s0 < nsb; s0 += kBoxBatch) {
                const int t = s0 + (ln & (kBoxBatch - 1));
                bool in = false;
                if (ln < kBoxBatch && t < nsb) {
                    const int32_t jj = ((lptr<const int32_t>)(sb + t))[6];
                    in = ((int)(int16_t)(jj & 0xFFFF) <= rl) & ((jj >> 16) >= r0);
                }
                const unsigned long long m = __ballot(in);
                if (m == 0ull) continue;
                if (in) L.idx[lanes_below(m)] = t;
                fold_tris(L, (lptr<const TriRec>)sb, (lptr<const int32_t>)L.idx, true, __popcll(m), W, rc.cx, rc.cy,
                          r0, nrows);
            }
        } else {
            const int scene = __builtin_amdgcn_readfirstlane(s.views[view].scene);
            const int ego_cam = __builtin_amdgcn_readfirstlane(s.views[view].ego_cam);
            const SceneRec sc = uniform_scene(s.scenes[scene]);
            const Cam cam = make_cam(s, sc, ego_cam >> 2, ego_cam & 3);
            boxes_from_scene(L, s, sc, cam, ego_cam >> 2, r0, nrows);
        }
        wave_lds_order();
        unsigned long long best[16];
        {
            typedef unsigned long long u2v __attribute__((ext_vector_type(2)));
            const lptr<const u2v> kp = (lptr<const u2v>)(L.keys + p.lr * W + p.i);
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const u2v v = p.act ? kp[m] : u2v{0ull, 0ull};
                best[2 * m] = v.x;
                best[2 * m + 1] = v.y;
            }
        }
        // a box fragment wins where its 1/z is not below the road's (agents
        // rank above roads on equal depth); otherwise road or background
        const uint32_t rzb = __float_as_uint(rz);
        uint32_t c[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const unsigned long long kb = best[m];
            const bool road = (bits >> m) & 1u;
            const bool box = (kb != 0ull) & (!road | ((uint32_t)(kb >> 32) >= rzb));
            const uint32_t boxc = s_pal[(uint32_t)kb & 0xFFu];   // any index is a palette entry
            c[m] = box ? boxc : (road ? road_rgb : bg_rgb);
        }
        if (p.act) store16(reinterpret_cast<uint8_t *>(out), c);
    }
}

}  // namespace

// zero the counters and the coverage words (a fill kernel, not a memset node:
// callers may capture this into a graph)
__global__ void k_chip_clear(ChipBufs cb, size_t cov_words)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < CHIP_NCTL) cb.ctl[i] = 0u;
    for (size_t k = i; k < cov_words; k += (size_t)gridDim.x * blockDim.x) cb.cov[k] = 0ull;
}

hipError_t launch_chip_clear(const ChipBufs &cb, size_t cov_words, hipStream_t st)
{
    hipLaunchKernelGGL(k_chip_clear, dim3(1024), dim3(256), 0, st, cb, cov_words);
    return hipGetLastError();
}

hipError_t launch_render_chip(const DevSim &s, const RenderOut &o, const ChipBufs &cb, int mode, int view_begin,
                              int n_views, int road_grid, hipStream_t st)
{
    if (n_views <= 0) return hipSuccess;
    if (road_grid <= 0 || cb.rows_per_item < 1 || cb.rows_per_item > kMaxItemRows || cb.btri_cap > kBoxCap)
        return hipErrorInvalidValue;
    const int gpv = (cb.items_per_view + kTilesPerGroup - 1) / kTilesPerGroup;
    hipLaunchKernelGGL(k_chip_setup, dim3((n_views + kSetupViews - 1) / kSetupViews), dim3(64 * 2 * kSetupViews), 0, st,
                       s, cb, mode, view_begin, n_views);
    hipLaunchKernelGGL(k_chip_roads, dim3(road_grid), dim3(256), 0, st, s, cb);
    hipLaunchKernelGGL(k_chip_resolve, dim3((unsigned)n_views * (unsigned)gpv), dim3(256), 0, st, s, o, cb, mode,
                       view_begin, n_views, gpv);
    return hipGetLastError();
}

}  // namespace gp
