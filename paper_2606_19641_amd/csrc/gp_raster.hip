// Wave-split rgb raster of the Gigapixel hot path for gfx950 (MI355X).
//
// The rgb-only ego-centric render (Sec. 3.1 O_pixel; App. A "High-Throughput
// Batched Rendering": one world per ego agent, all views in one batched
// launch) for sims whose road strips share one colour and renders that need
// neither depth nor primitive ids.  Its results are bit-identical to the
// banded kernel (k_render) and to the plain definition: the same clip, snap,
// fill rule and winner order, only organised for throughput.
//
// One workgroup of K wavefronts (K = 1, 2 or 4) renders one view, with about
// 19 KB of LDS at 128 x 128, so that a CU keeps eight views in flight:
//   A  bins    the scene's road culling bins are tested against the view
//              (frustum, road depth limit and the row-gap test below); the
//              surviving bins are listed in LDS.
//   B  units   the waves deal out work units through an LDS counter.  Unit 0
//              is the boxes: cull, face setup and clipping into the view's
//              box triangle list.  Every further unit is four surviving bins
//              (64 strip slots).  A strip first meets a cheap test that can
//              only reject strips covering no sample: the frustum, the road
//              depth limit, and the row-gap test (every vertex a strip's clip
//              can produce lies at camera height -h, so its snapped row
//              coordinate is a non-increasing function of its depth; a strip
//              whose depth range maps between two sample rows covers none).
//              Survivors' camera-space corners go to the wave's ring; full
//              setup (clip test, snap, a quad or the two fan triangles) runs 48 at a
//              time, and each batch of triangles is rasterised at once: per
//              (triangle, row) the exact span of covered samples is OR-ed
//              into the view's road coverage bitmask.  Strips that need
//              clipping are queued and clipped four per wavefront.
//   C  resolve rows no box triangle touches are written from the table of the
//              sixteen four-pixel road/background patterns, 16 pixels (48
//              bytes) per lane; box rows go band by band through a band of
//              64-bit keys that reuses the waves' staging memory: box
//              fragments are dealt to lanes (span lengths prefix-summed over
//              the wavefront) and folded in with LDS atomic max, and the band
//              is resolved against the road coverage.
//
// Every float operation is written out (fmaf for fused operations) and the
// file is compiled with -ffp-contract=off, correctly rounded division and
// IEEE denormals.

#include "gp_device.h"
#include "gp_geom.h"

namespace gp {

namespace {

constexpr int kSharedRing = 768;   // strips passed by the cheap test, one ring per view (road slot indices)
constexpr int kWTris = 64;      // road primitives (quads, triangles) staged for one span pass
constexpr int kSetupBatch = kWTris;       // strips of one set-up job at most (one quad each; the rest are queued)
constexpr int kWClip = kSetupBatch;       // strips of one job waiting for the clipper (from the front) or
                                          // for their fan triangles (from the back)
constexpr int kWaveBytes = kWTris * 48 + kWClip * 4;
static_assert(kWaveBytes % 16 == 0, "wave regions stay 16-byte aligned");
static_assert(sizeof(Prim) == 48, "staged primitive size");

// LDS counters
enum { R_NSB = 0, R_NEXT, R_NBT, R_BOVF, R_BMIN, R_BMAX, R_RING, R_RESV, R_JOB, R_NCNT = 12 };
constexpr int kBoxClip = 64;     // box faces waiting for the clipper (one setup pass)

struct RgbLds {
    lptr<int32_t> cnt;               // [R_NCNT]
    lptr<uint32_t> pal;              // [256] RGB of each palette entry
    lptr<uint32_t> lut;              // [16][4] four-pixel road/background patterns, 3 packed dwords
    lptr<unsigned long long> bits;   // [H][nw] road coverage, bit i of word w: column 64 w + i
    lptr<TriRec> btris;              // [bcap] the view's box triangles
    lptr<int32_t> sbins;             // [bins_cap] surviving bins: start * 128 + count
    lptr<int32_t> cq;                // [kBoxClip] box faces to clip (box * 8 + face)
    lptr<int32_t> sring;             // [kSharedRing] strips that passed the cheap test (this round)
    lptr<unsigned char> waves;       // K regions of kWaveBytes
    int nw, bcap, krows;
    int region;                      // bytes from sbins to the end (free after the units)
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// byte offsets of the LDS sections (shared by the carve and the size query)
struct RgbLayout {
    size_t cnt, pal, lut, bits, btris, sbins, cq, sring, waves, total;
};

__host__ __device__ inline RgbLayout rgb_layout(int W, int H, const RgbCfg &c)
{
    RgbLayout l;
    const size_t nw = (size_t)(W + 63) / 64;
    size_t o = 0;
    l.cnt = o; o = align16(o + 4 * R_NCNT);
    l.pal = o; o = align16(o + 4 * 256);
    l.lut = o; o = align16(o + 4 * 64);
    l.bits = o; o = align16(o + 8 * nw * (size_t)H);
    l.btris = o; o = align16(o + sizeof(TriRec) * (size_t)c.bcap);
    l.cq = o; o = align16(o + 4 * (size_t)kBoxClip);
    l.sbins = o; o = align16(o + 4 * (size_t)c.bins_cap);
    l.sring = o; o = align16(o + 4 * (size_t)kSharedRing);
    l.waves = o; o = align16(o + (size_t)kWaveBytes * (size_t)c.waves);
    l.total = o;
    return l;
}

// ------------------------------------------------------------ per-wave state

struct WaveSt {
    lptr<Prim> tris;         // [kWTris] road primitives
    lptr<int32_t> clipq;     // [kWClip] road slots (global): nclip for the clipper at the front,
                             // nfan for their two fan triangles at the back
    int nclip, nfan;         // queued strips
};

// OR the samples [xl, xr] of one row into its coverage words
__device__ __forceinline__ void or_span(lptr<unsigned long long> row, int xl, int xr)
{
    const int w0 = xl >> 6, w1 = xr >> 6;
    for (int w = w0; w <= w1; ++w) {
        const int lo = (w == w0) ? (xl & 63) : 0;
        const int hi = (w == w1) ? (xr & 63) : 63;
        const unsigned long long m = (hi == 63 ? ~0ull : ((1ull << (hi + 1)) - 1ull)) & (~0ull << lo);
        lds_or64(row + w, m);
    }
}

// Rasterise the n staged road triangles into the coverage bitmask.  Lane t
// first takes the first row of triangle t; the further rows of triangles
// that span several rows are then dealt to the lanes by a prefix over their
// counts.  Per (triangle, row) the exact span of covered samples is OR-ed
// into the row's coverage words.
__device__ __forceinline__ void road_spans(const RgbLds &L, const Cam &cam, const WaveSt &ws, int n)
{
    const int ln = (int)lane_id();
    wave_lds_order();
    for (int t0 = 0; t0 < n; t0 += 64) {
        const int t = t0 + ln;
        int c = 0;
        if (t < n) {
            const int32_t jj = ((lptr<const int32_t>)(ws.tris + t))[8];     // j0 | j1 << 16
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
                const Prim pr = lds_load(ws.tris + t0 + o);
                const int j = pr.j0 + extra;
                int xl, xr;
                if (prim_span(pr, j, cam.W, xl, xr)) or_span(L.bits + (size_t)j * L.nw, xl, xr);
            }
        }
    }
    wave_lds_order();
}

// Stage the triangles held by the lanes (v0: t0, v1: t1); returns how many.
__device__ __forceinline__ int stage_tris(const WaveSt &ws, bool v0, const Prim &t0, bool v1, const Prim &t1)
{
    const unsigned long long b0 = __ballot(v0), b1 = __ballot(v1);
    const int n0 = __popcll(b0);
    if (v0) lds_store(ws.tris + lanes_below(b0), t0);
    if (v1) lds_store(ws.tris + n0 + lanes_below(b1), t1);
    return n0 + __popcll(b1);
}

// Clip up to four queued strips (the last ones of the queue), one per 16-lane
// segment; stages their fan triangles and returns how many.
__device__ __forceinline__ int road_clip(const DevSim &s, const Cam &cam, WaveSt &ws)
{
    const int m = min(ws.nclip, 4);
    const int seg = (int)lane_id() >> 4;
    const bool live = seg < m;
    Poly P = {};
    if (live) {
        const int g = ws.clipq[ws.nclip - m + seg];
        road_corners(s, cam, g, P.v);
    }
    P.n = dir_to_cam(cam, 0.0f, 0.0f, 1.0f);
    P.one_sided = false;
    P.keylo = 0u;
    ws.nclip -= m;
    TriRec t;
    const bool ok = clip_seg<false>(cam, P, live, 0, cam.H, t);
    Prim none = {};
    return stage_tris(ws, ok, prim_of(t.g), false, none);
}

// The two fan triangles of up to 32 queued strips (the last ones queued at
// the back of the queue); stages them and returns how many.  Their corners
// and snap are computed again, as the set-up computed them.
__device__ __forceinline__ int road_fan(const DevSim &s, const Cam &cam, WaveSt &ws)
{
    const int m = min(ws.nfan, 32);
    const int ln = (int)lane_id();
    Prim p0 = {}, p1 = {};
    bool v0 = false, v1 = false;
    if (ln < m) {
        const int g = ws.clipq[kWClip - ws.nfan + ln];
        V3 v[4];
        road_corners(s, cam, g, v);
        int32_t X[4], Y[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) snap(cam, v[k], X[k], Y[k]);
        TriGeo t0, t1;
        v0 = make_tri(cam, false, X[0], Y[0], X[1], Y[1], X[2], Y[2], 0, cam.H, t0);
        v1 = make_tri(cam, false, X[0], Y[0], X[2], Y[2], X[3], Y[3], 0, cam.H, t1);
        if (v0) p0 = prim_of(t0);
        if (v1) p1 = prim_of(t1);
    }
    ws.nfan -= m;
    return stage_tris(ws, v0, p0, v1, p1);
}

// Full setup of the n (<= kSetupBatch) strips ring[a .. a + n): clip test,
// snap, and the quad of the strips whose quad covers exactly what their two
// fan triangles cover (staged; returns how many); strips that need the
// clipper join the front of the wave's queue, strips that need their fan
// triangles its back (both empty when a job starts).
__device__ __forceinline__ int road_setup(const DevSim &s, const Cam &cam, const RgbLds &L, WaveSt &ws, int a, int n)
{
    const int ln = (int)lane_id();
    wave_lds_order();
    const bool live = ln < n;
    int g = 0;
    V3 v[4] = {};
    if (live) {
        g = L.sring[a + ln];
        road_corners(s, cam, g, v);
    }
    const bool clip = live && needs_clip(cam, v);
    const unsigned long long cb = __ballot(clip);
    if (clip) ws.clipq[ws.nclip + lanes_below(cb)] = g;
    ws.nclip += __popcll(cb);
    Prim p0 = {};
    bool v0 = false, fan = false;
    if (live && !clip) {
        int32_t X[4], Y[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) snap(cam, v[k], X[k], Y[k]);
        // one quad where it covers exactly what the two fan triangles cover
        const int qs = make_quad(cam, X, Y, 0, cam.H, p0);
        v0 = qs > 0;
        fan = qs < 0;
    }
    const unsigned long long fb = __ballot(fan);
    if (fan) ws.clipq[kWClip - 1 - (ws.nfan + lanes_below(fb))] = g;
    ws.nfan += __popcll(fb);
    Prim none = {};
    return stage_tris(ws, v0, p0, false, none);
}

// One set-up job: the n ring strips from a set up, their primitives
// rasterised into the coverage bitmask, then the strips that needed their fan
// triangles (32 at a time) and those that needed the clipper (four at a time).
__device__ __forceinline__ void setup_job(const DevSim &s, const Cam &cam, const RgbLds &L, WaveSt &ws, int a, int n)
{
    int ntri = road_setup(s, cam, L, ws, a, n);
    for (;;) {
        if (ntri > 0) road_spans(L, cam, ws, ntri);
        if (ws.nfan > 0)
            ntri = road_fan(s, cam, ws);
        else if (ws.nclip > 0)
            ntri = road_clip(s, cam, ws);
        else
            break;
    }
}

// The cheap test of one unit's strips (loaded by load_unit into q0, q1); the
// survivors' slots go to the view's ring (64 entries were reserved).
__device__ __forceinline__ void road_unit(const Cam &cam, const RgbLds &L, bool live, int g, const float4 &q0,
                                          const float4 &q1)
{
    float x[4], z[4];
    ground_xz(cam, q0.x, q0.y, x[0], z[0]);
    ground_xz(cam, q0.z, q0.w, x[1], z[1]);
    ground_xz(cam, q1.x, q1.y, x[2], z[2]);
    ground_xz(cam, q1.z, q1.w, x[3], z[3]);
    const bool pass = live && !road_culled<false>(cam, x, z);
    const unsigned long long bm = __ballot(pass);
    int base = 0;
    if (lane_id() == 0 && bm != 0ull) base = lds_add(L.cnt + R_RING, __popcll(bm));
    base = __shfl(base, 0);
    if (pass) L.sring[base + lanes_below(bm)] = g;
}

// strip data of unit u (lane l: strip l % 16 of surviving bin 4 u + l / 16)
__device__ __forceinline__ bool load_unit(const DevSim &s, const SceneRec &sc, const RgbLds &L, int nsb, int u,
                                          int &g, float4 &q0, float4 &q1)
{
    const int ln = (int)lane_id();
    const int bi = 4 * u + (ln >> 4), k = ln & 15;
    bool live = false;
    if (u >= 0 && bi < nsb) {
        const int pk = L.sbins[bi];
        live = k < (pk & 127);
        if (live) {
            g = sc.road_base + (pk >> 7) + k;
            q0 = s.roads[2 * g];
            q1 = s.roads[2 * g + 1];
        }
    }
    return live;
}

// ------------------------------------------------------------ boxes

// Reserve n entries of the box list: at the wave's own count nbt (shared
// false: the overflow path's private list), or through the view's LDS
// counter (shared: several wavefronts append); returns the first entry, or
// -1 (marking the view overflowed when shared) if they would not fit.
__device__ __forceinline__ int box_reserve(const RgbLds &L, bool shared, int &nbt, int n)
{
    if (!shared) {
        if (nbt + n > L.bcap) return -1;
        const int at = nbt;
        nbt += n;
        return at;
    }
    int at = 0;
    if (lane_id() == 0 && n > 0) at = lds_add(L.cnt + R_NBT, n);
    at = __builtin_amdgcn_readfirstlane(__shfl(at, 0));
    if (at + n > L.bcap) {
        if (lane_id() == 0) L.cnt[R_BOVF] = 1;
        return -1;
    }
    return at;
}

// One setup pass over box face candidates [c0, c0 + P) (P <= 64): candidate c
// is face c % 6 of box surv[c / 6] (use_surv), or of box c / 6 culled here.
// Fast triangles and clipped faces (clip queue cq) are appended to the box
// list (box_reserve); returns false as soon as the triangles would not fit
// (the list is then incomplete: the view takes the overflow path, which
// ignores it).  Eight candidates at a time never overflow a private list of
// 96 (at most 10 triangles each).
__device__ __forceinline__ bool box_pass(const DevSim &s, const SceneRec &sc, const Cam &cam, int ego, const RgbLds &L,
                         lptr<const int32_t> surv, bool use_surv, int ncand, int c0, int P, lptr<int32_t> cq,
                         bool shared, int &nbt, int &bmin, int &bmax)
{
    const int ln = (int)lane_id();
    const int c = c0 + ln;
    bool live = ln < P && c < ncand;
    int j = 0, f = 0;
    if (live) {
        j = use_surv ? surv[c / 6] : c / 6;
        f = c - 6 * (c / 6);
        if (!use_surv) live = j != ego && !box_outside(s, sc, cam, j);
    }
    Poly Pf;
    TriRec t0, t1;
    bool v0 = false, v1 = false, clip = false;
    if (live) {
        build_face(s, sc, cam, j, f, Pf);
        fast_poly<true>(cam, Pf, 0, cam.H, t0, v0, t1, v1, clip);
    }
    const unsigned long long b0 = __ballot(v0), b1 = __ballot(v1), bc = __ballot(clip);
    const int n0 = __popcll(b0), nf = n0 + __popcll(b1), ncl = __popcll(bc);
    const int at = box_reserve(L, shared, nbt, nf);
    if (at < 0) return false;
    if (v0) lds_store(L.btris + at + lanes_below(b0), t0);
    if (v1) lds_store(L.btris + at + n0 + lanes_below(b1), t1);
    if (v0) { bmin = min(bmin, (int)t0.g.j0); bmax = max(bmax, (int)t0.g.j1); }
    if (v1) { bmin = min(bmin, (int)t1.g.j0); bmax = max(bmax, (int)t1.g.j1); }
    if (clip) cq[lanes_below(bc)] = j * 8 + f;
    wave_lds_order();
    // the clipped faces, four per wavefront
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
        const unsigned long long bo = __ballot(ok);
        const int ato = box_reserve(L, shared, nbt, __popcll(bo));
        if (ato < 0) return false;
        if (ok) {
            lds_store(L.btris + ato + lanes_below(bo), t);
            bmin = min(bmin, (int)t.g.j0);
            bmax = max(bmax, (int)t.g.j1);
        }
    }
    return true;
}

// Box unit k: cull boxes [kBoxUnit k, kBoxUnit (k + 1)) of the scene, list
// the survivors, set up their faces into the view's box triangle list
// (shared by the wavefronts; its row range kept with LDS min / max).  scr:
// 128 ints of the wavefront's staging (survivors, then the clip queue).
constexpr int kBoxUnit = 16;
__device__ __forceinline__ void do_boxes(const DevSim &s, const SceneRec &sc, const Cam &cam, int ego, const RgbLds &L,
                                         int k, lptr<int32_t> scr)
{
    const int ln = (int)lane_id();
    const int nbox = sc.n_agents + sc.n_static;
    const int j = kBoxUnit * k + ln;
    const bool keep = ln < kBoxUnit && j < nbox && j != ego && !box_outside(s, sc, cam, j);
    const unsigned long long bm = __ballot(keep);
    if (keep) scr[lanes_below(bm)] = j;
    const int ns = __popcll(bm);
    wave_lds_order();
    int nbt = 0, bmin = 0x7FFFFFFF, bmax = -1;
    for (int c0 = 0; c0 < 6 * ns; c0 += 64)
        if (!box_pass(s, sc, cam, ego, L, scr, true, 6 * ns, c0, 64, scr + 64, true, nbt, bmin, bmax)) break;
    bmin = wave_min(bmin);
    bmax = wave_max(bmax);
    if (ln == 0 && bmax >= 0) {
        lds_min(L.cnt + R_BMIN, bmin);
        lds_max(L.cnt + R_BMAX, bmax);
    }
}

// Box fragments of the list's n triangles in rows [b0, b1) folded into the
// key band.  The (triangle, row) items are dealt to the lanes by a prefix
// over row counts, item passes shared out over the view's wavefronts (wave w
// of nw takes passes w, w + nw, ...); each lane computes its item's exact
// span; the spans are cut into pieces of up to 16 samples, which are dealt to
// the lanes by a prefix over piece counts, and each lane folds its piece's
// samples into the band with LDS atomic max.
__device__ __forceinline__ void box_band(const RgbLds &L, const Cam &cam, lptr<unsigned long long> keys, int n,
                                         int wv, int nwv, int b0, int b1)
{
    const int ln = (int)lane_id();
    const int W = cam.W;
    int pass = 0;
    for (int t0 = 0; t0 < n; t0 += 64) {
        const int t = t0 + ln;
        int c = 0;
        if (t < n) {
            const int32_t jj = ((lptr<const int32_t>)(L.btris + t))[6];
            const int j0 = max((int)(int16_t)(jj & 0xFFFF), b0), j1 = min(jj >> 16, b1 - 1);
            c = max(0, j1 - j0 + 1);
        }
        const int incl = wave_incl_scan(c);
        const int total = __builtin_amdgcn_readlane(incl, 63);
        const int excl = incl - c;
        for (int g0 = 0; g0 < total; g0 += 64, ++pass) {
            if (pass % nwv != wv) continue;
            const int gi = g0 + ln;
            const int o = owner_of(incl, gi);
            const int ex = __shfl(excl, o);
            int xl = 0, xr = -1, j = 0;
            float A = 0.0f, B = 0.0f, Cc = 0.0f;
            uint32_t key = 0u;
            if (gi < total) {
                const TriRec tr = lds_load(L.btris + t0 + o);
                j = max((int)tr.g.j0, b0) + (gi - ex);
                if (!row_span(tr.g, j, W, xl, xr)) { xl = 0; xr = -1; }
                A = tr.A; B = tr.B; Cc = tr.C; key = tr.keylo;
            }
            const int np = (xr - xl + 16) >> 4;            // pieces of up to 16 samples (0 if empty)
            const int inc2 = wave_incl_scan(np);
            const int npt = __builtin_amdgcn_readlane(inc2, 63);
            const int ex2 = inc2 - np;
            const float dv = ((float)j + 0.5f) - cam.cy;
            for (int p0 = 0; p0 < npt; p0 += 64) {
                const int pi = p0 + ln;
                const int o2 = owner_of(inc2, pi);
                const int k = pi - __shfl(ex2, o2);
                const int sxl = __shfl(xl, o2), sxr = __shfl(xr, o2), sj = __shfl(j, o2);
                const float sA = __shfl(A, o2), sB = __shfl(B, o2), sC = __shfl(Cc, o2), sdv = __shfl(dv, o2);
                const uint32_t skey = (uint32_t)__shfl((int)key, o2);
                const int i0 = sxl + 16 * k, i1 = pi < npt ? min(i0 + 15, sxr) : i0 - 1;
                lptr<unsigned long long> row = keys + (size_t)(sj - b0) * W;
                for (int i = i0; i <= i1; ++i) {
                    const float du = ((float)i + 0.5f) - cam.cx;
                    const float invz = fmaf(sA, du, fmaf(sB, sdv, sC));
                    if (invz > 0.0f) lds_max64(row + i, ((unsigned long long)__float_as_uint(invz) << 32) | skey);
                }
            }
        }
    }
}

// ------------------------------------------------------------ box rows by group masks
//
// The box rows [c0, c1) without a key band: the exact span of every (box
// triangle, row) item is computed once and stored, and every group of 16
// samples of a row gets a mask of the triangles whose span meets it.  The
// resolve then walks, for its 16 samples, the triangles of its group's mask
// and keeps the largest key of each sample in registers.  Memory (the free
// region): the masks M[c1 - c0][W / 16][2], then the spans S[t][c1 - c0].
constexpr int kMaskTris = 128;     // triangles a mask holds (two 64-bit words)

__host__ __device__ inline int mask_rows_fit(int region, int n, int W)
{
    // rows per chunk so that the masks and a span of every triangle in every row fit
    return region / (16 * (W / 16) + 4 * n);
}

__device__ __forceinline__ void box_spans(const RgbLds &L, const Cam &cam, int n, int c0, int c1, int wv, int nwv)
{
    const int ln = (int)lane_id();
    const int R = c1 - c0, G = cam.W >> 4;
    lptr<unsigned long long> M = (lptr<unsigned long long>)L.sbins;
    lptr<int32_t> S = (lptr<int32_t>)(M + 2 * G * R);
    int pass = 0;
    for (int t0 = 0; t0 < n; t0 += 64) {
        const int t = t0 + ln;
        int c = 0;
        if (t < n) {
            const int32_t jj = ((lptr<const int32_t>)(L.btris + t))[6];
            const int j0c = max((int)(int16_t)(jj & 0xFFFF), c0);
            c = max(0, min(jj >> 16, c1 - 1) - j0c + 1);
        }
        const int incl = wave_incl_scan(c);
        const int total = __builtin_amdgcn_readlane(incl, 63);
        const int excl = incl - c;
        for (int g0 = 0; g0 < total; g0 += 64, ++pass) {
            if (pass % nwv != wv) continue;
            const int gi = g0 + ln;
            const int o = owner_of(incl, gi);
            const int ex = __shfl(excl, o);
            if (gi < total) {
                const int tt = t0 + o;
                const TriGeo tg = lds_load((lptr<TriGeo>)(L.btris + tt));
                const int j = max((int)tg.j0, c0) + (gi - ex);
                int xl, xr;
                if (row_span(tg, j, cam.W, xl, xr)) {
                    S[tt * R + (j - c0)] = xl | (xr << 16);
                    lptr<unsigned long long> mrow = M + 2 * G * (j - c0) + (tt >> 6);
                    const unsigned long long bit = 1ull << (tt & 63);
                    for (int g = xl >> 4; g <= (xr >> 4); ++g) lds_or64(mrow + 2 * g, bit);
                }
            }
        }
    }
}

// rows [c0, c1) from the group masks and spans: 16 samples (48 bytes) per
// task; tasks alternate over the view's wavefronts in blocks of 32 lanes so
// that a few box rows still keep every wavefront busy
__device__ __forceinline__ void resolve_masks(const RgbLds &L, const Cam &cam, uint8_t *img, uint32_t road_rgb,
                                              uint32_t bg_rgb, int c0, int c1, int wv, int nwv)
{
    typedef float f4v __attribute__((ext_vector_type(4)));
    const int R = c1 - c0, G = cam.W >> 4;
    lptr<const unsigned long long> M = (lptr<const unsigned long long>)L.sbins;
    lptr<const int32_t> S = (lptr<const int32_t>)(M + 2 * G * R);
    const int W = cam.W;
    const int n = R * G;
    const int ln = (int)lane_id();
    const int half = ln >> 5, sub = ln & 31;
    for (int blk = 2 * wv + half; 32 * blk < n; blk += 2 * nwv) {
        const int task = 32 * blk + sub;
        if (task >= n) continue;
        const int r = task / G, g = task - r * G, i = g << 4, j = c0 + r;
        const float dv = ((float)j + 0.5f) - cam.cy;
        const float rz = fmaf(cam.road.B, dv, cam.road.C);
        const uint32_t bits = rz > 0.0f ? (uint32_t)(L.bits[(size_t)j * L.nw + (i >> 6)] >> (i & 63)) & 0xFFFFu : 0u;
        const uint32_t rzb = __float_as_uint(rz);
        // sample offsets ((float)(i + m) + 0.5f) - cx are small exact values: du0 + m
        const float du0 = ((float)i + 0.5f) - cam.cx;
        unsigned long long best[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) best[m] = 0ull;
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            unsigned long long mk = M[2 * (G * r + g) + w];
            while (mk != 0ull) {
                const int t = 64 * w + (__ffsll((long long)mk) - 1);
                mk &= mk - 1ull;
                // span and plane read together (both depend on t only)
                const int sp = S[t * R + r];
                const f4v pk = *(lptr<const f4v>)((lptr<const unsigned char>)(L.btris + t) + 32);   // A B C keylo
                // the span's samples within this group as a bit mask
                const int lo = max((sp & 0xFFFF) - i, 0), hi = min((sp >> 16) - i, 15);
                const uint32_t in = ((2u << hi) - 1u) & ~((1u << lo) - 1u);
                const float bdv = fmaf(pk.y, dv, pk.z);
                const uint32_t keylo = __float_as_uint(pk.w);
                // branch-free: the three tests combined bitwise, so that each
                // sample is a select and not a branch around the compare
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    const float invz = fmaf(pk.x, du0 + (float)m, bdv);
                    const unsigned long long key = ((unsigned long long)__float_as_uint(invz) << 32) | keylo;
                    const bool take = (((in >> m) & 1u) != 0u) & (invz > 0.0f) & (key > best[m]);
                    best[m] = take ? key : best[m];
                }
            }
        }
        uint32_t c[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const unsigned long long kb = best[m];
            const bool road = (bits >> m) & 1u;
            const bool box = (kb != 0ull) & (!road | ((uint32_t)(kb >> 32) >= rzb));
            const uint32_t boxc = L.pal[(uint32_t)kb & 0xFFu];   // any index is a palette entry
            c[m] = box ? boxc : (road ? road_rgb : bg_rgb);
        }
        store16(img + 3 * ((int64_t)j * W + i), c);
    }
}

// ------------------------------------------------------------ resolve

typedef uint32_t u4 __attribute__((ext_vector_type(4)));

// rows [r0, r1) that no box fragment touches: 16 pixels (48 bytes) per lane
// from the pattern table (road where the coverage bit is set and the row is
// below the horizon, background elsewhere); two tasks per iteration so that
// their LDS reads overlap
__device__ __forceinline__ void resolve_lut(const RgbLds &L, const Cam &cam, uint8_t *img, int r0, int r1)
{
    const int W = cam.W, gpr = W >> 4;
    const int n = (r1 - r0) * gpr;
    const lptr<u4> lut = (lptr<u4>)L.lut;
    const int B = (int)blockDim.x;
    for (int task = (int)threadIdx.x; task < n; task += 2 * B) {
        uint32_t bits[2];
        u4 *out[2];
        bool act[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int tk = task + h * B;
            act[h] = tk < n;
            const int tc = act[h] ? tk : task;
            const int r = tc / gpr, i = (tc - r * gpr) << 4, j = r0 + r;
            const float dv = ((float)j + 0.5f) - cam.cy;
            const float rz = fmaf(cam.road.B, dv, cam.road.C);
            bits[h] = rz > 0.0f ? (uint32_t)(L.bits[(size_t)j * L.nw + (i >> 6)] >> (i & 63)) & 0xFFFFu : 0u;
            out[h] = reinterpret_cast<u4 *>(img + 3 * ((int64_t)j * W + i));
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t b = bits[h];
            const u4 a = lut[b & 15u], bb = lut[(b >> 4) & 15u], c = lut[(b >> 8) & 15u], d = lut[b >> 12];
            if (act[h]) {
                out[h][0] = u4{a.x, a.y, a.z, bb.x};
                out[h][1] = u4{bb.y, bb.z, c.x, c.y};
                out[h][2] = u4{c.z, d.x, d.y, d.z};
            }
        }
    }
}

// rows [b0, b1) of the key band: a box fragment wins where its 1/z is not
// below the road's (agents rank above roads on equal depth); otherwise road
// or background by the coverage bit
__device__ __forceinline__ void resolve_band(const RgbLds &L, const Cam &cam, lptr<unsigned long long> keys, uint8_t *img,
                             uint32_t road_rgb, uint32_t bg_rgb, int b0, int b1)
{
    const int W = cam.W, gpr = W >> 4;
    const int n = (b1 - b0) * gpr;
    for (int task = (int)threadIdx.x; task < n; task += (int)blockDim.x) {
        const int r = task / gpr, i = (task - r * gpr) << 4, j = b0 + r;
        const float dv = ((float)j + 0.5f) - cam.cy;
        const float rz = fmaf(cam.road.B, dv, cam.road.C);
        const bool rowok = rz > 0.0f;
        const uint32_t bits = rowok ? (uint32_t)(L.bits[(size_t)j * L.nw + (i >> 6)] >> (i & 63)) & 0xFFFFu : 0u;
        const uint32_t rzb = __float_as_uint(rz);
        lptr<unsigned long long> kp = keys + (size_t)r * W + i;
        uint32_t c[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const unsigned long long kb = kp[m];
            const bool road = (bits >> m) & 1u;
            const bool box = (kb != 0ull) & (!road | ((uint32_t)(kb >> 32) >= rzb));
            const uint32_t boxc = L.pal[(uint32_t)kb & 0xFFu];   // any index is a palette entry
            c[m] = box ? boxc : (road ? road_rgb : bg_rgb);
        }
        u4 *out = reinterpret_cast<u4 *>(img + 3 * ((int64_t)j * W + i));
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            // 16 pixels = 48 bytes = 12 dwords; dword k holds bytes 4k .. 4k + 3
            uint32_t w[4];
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const int k = 4 * q + d;     // dword index
                uint32_t v = 0;
#pragma unroll
                for (int bb = 0; bb < 4; ++bb) {
                    const int byte = 4 * k + bb, px = byte / 3, ch = byte - 3 * px;
                    v |= ((c[px] >> (8 * ch)) & 0xFFu) << (8 * bb);
                }
                w[d] = v;
            }
            out[q] = u4{w[0], w[1], w[2], w[3]};
        }
    }
}

// Box rows [kr0, kr1) through bands of 64-bit keys (the whole workgroup; the
// region from the surviving-bin list on is free): the view's box triangle
// list, or, if it overflowed (ovf), the box faces streamed through it eight
// candidates at a time (at most 96 triangles per pass) with the boxes culled
// again.  wv / nwv: this wavefront among the workgroup's.
__device__ __forceinline__ void key_band_rows(const DevSim &s, const SceneRec &sc, const Cam &cam, int ego, const RgbLds &L,
                                              uint8_t *img, uint32_t road_rgb, uint32_t bg_rgb, int kr0, int kr1, bool ovf,
                                              int nbt, int wv, int nwv)
{
    const int W = cam.W;
    lptr<unsigned long long> keys = (lptr<unsigned long long>)L.sbins;
    for (int b0 = kr0; b0 < kr1; b0 += L.krows) {
        const int b1 = min(b0 + L.krows, kr1);
        __syncthreads();
        for (int p = (int)threadIdx.x; p < (b1 - b0) * W; p += (int)blockDim.x) keys[p] = 0ull;
        __syncthreads();
        if (!ovf) {
            box_band(L, cam, keys, nbt, wv, nwv, b0, b1);
        } else if (wv == 0) {
            const int ncand = 6 * (sc.n_agents + sc.n_static);
            for (int c0 = 0; c0 < ncand; c0 += 8) {
                int n = 0, bmn = 0, bmx = 0;
                (void)box_pass(s, sc, cam, ego, L, (lptr<const int32_t>)L.sbins, false, ncand, c0, 8, L.cq, false, n, bmn,
                               bmx);
                wave_lds_order();
                box_band(L, cam, keys, n, 0, 1, b0, b1);
                wave_lds_order();
            }
        }
        __syncthreads();
        resolve_band(L, cam, keys, img, road_rgb, bg_rgb, b0, b1);
    }
}

// ------------------------------------------------------------ per view

// Issue priority of the view's wavefronts (0..3) against the other views'
// on the same SIMDs.  Every view of a launch is resident at once, so the
// launch lasts as long as its slowest view: a view with much work left
// raises its priority and the views with little fill the gaps.  Only the
// instruction issue order changes, never a result.
__device__ __forceinline__ void view_priority(int p)
{
    p = __builtin_amdgcn_readfirstlane(p);
    if (p >= 3) __builtin_amdgcn_s_setprio(3);
    else if (p == 2) __builtin_amdgcn_s_setprio(2);
    else if (p == 1) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

// The scene's road culling bins [b0, b0 + 64) against the view (frustum, road
// depth limit and row-gap test); the survivors are appended to the view's
// list of surviving bins.
__device__ __forceinline__ void cull_bins(const DevSim &s, const SceneRec &sc, const Cam &cam, const RgbLds &L, int b0)
{
    const int ln = (int)lane_id();
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
    const int nk = __popcll(bm);
    int base = 0;
    if (nk > 0) {
        const int leader = __ffsll((long long)bm) - 1;
        if (ln == leader) base = lds_add(L.cnt + R_NSB, nk);
        base = __shfl(base, leader);
    }
    if (keep) L.sbins[base + lanes_below(bm)] = rec;
}

template <int K>
__device__ __forceinline__ void render_view_rgb(const DevSim &s, const RenderOut &o, const RgbLds &L, int view)
{
    constexpr int B = 64 * K;
    const int tid = (int)threadIdx.x, ln = (int)lane_id(), wv = tid >> 6;
    const int scene = __builtin_amdgcn_readfirstlane(s.views[view].scene);
    const int ego_cam = __builtin_amdgcn_readfirstlane(s.views[view].ego_cam);
    const SceneRec sc = uniform_scene(s.scenes[scene]);
    const int ego = ego_cam >> 2;
    const Cam cam = make_cam(s, sc, ego, ego_cam & 3);
    const int W = cam.W, H = cam.H;

    for (int p = tid; p < H * L.nw; p += B) L.bits[p] = 0ull;
    // road units are numbered after the box units (dealt as jobs, below)
    if (tid < R_NCNT)
        L.cnt[tid] = tid == R_BMIN ? 0x7FFFFFFF
                   : (tid == R_BMAX ? -1 : (tid == R_NEXT ? (sc.n_agents + sc.n_static + kBoxUnit - 1) / kBoxUnit : 0));
    __syncthreads();

    // ---- A: road culling bins
    for (int b0 = 64 * wv; b0 < sc.n_bins; b0 += B) cull_bins(s, sc, cam, L, b0);
    __syncthreads();

    // ---- B: rounds of two steps, each dealt over the view's wavefronts
    // through LDS counters.  B1: the road units (four surviving bins each,
    // numbered from nbu on): the cheap test of the unit's strips with the
    // survivors appended to the view's ring (a unit is taken only with 64
    // free ring entries reserved).  B2: the jobs -- in the first round the box
    // units first (boxes kBoxUnit k .. kBoxUnit k + kBoxUnit - 1: cull, face
    // set-up and clipping into the box list, which is needed only by the
    // resolve, so a long box unit overlaps the other wavefront's road jobs),
    // then set-up jobs of up to kSetupBatch ring strips: set-up, the fan
    // triangles and the clipper for the strips that need them, and the spans
    // of every primitive.  A round ends when the ring is full or the units
    // are used up.
    const int nsb = L.cnt[R_NSB];
    // road work ahead grows with the surviving bins (a mean view keeps about a dozen)
    const int prio_b = nsb >= 24 ? 2 : (nsb >= 16 ? 1 : 0);
    view_priority(prio_b);
    const int nbu = (sc.n_agents + sc.n_static + kBoxUnit - 1) / kBoxUnit;
    const int n_units = nbu + (nsb + 3) / 4;
    lptr<unsigned char> wbase = L.waves + (size_t)wv * kWaveBytes;
    WaveSt ws;
    ws.tris = (lptr<Prim>)wbase;
    ws.clipq = (lptr<int32_t>)(wbase + kWTris * 48);
    ws.nclip = 0;
    ws.nfan = 0;
    // the next unit with its ring entries reserved, or n_units (none left, or
    // the ring cannot take another road unit this round)
    auto take = [&]() -> int {
        int u = n_units;
        if (ln == 0) {
            const int r = lds_add(L.cnt + R_RESV, 64);
            if (r + 64 <= kSharedRing) {
                u = min(lds_add(L.cnt + R_NEXT, 1), n_units);
                if (u == n_units) lds_add(L.cnt + R_RESV, -64);   // no unit left
            } else {
                lds_add(L.cnt + R_RESV, -64);
            }
        }
        return __builtin_amdgcn_readfirstlane(__shfl(u, 0));
    };
    int box_jobs = nbu;          // box units still to deal (first round)
    for (;;) {
        // B1, the next unit's strips loaded while the current one is tested
        int u = take();
        float4 q0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), q1 = q0;
        int gq = 0;
        bool live = u < n_units && load_unit(s, sc, L, nsb, u - nbu, gq, q0, q1);
        while (u < n_units) {
            const int un = take();
            float4 n0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), n1 = n0;
            int gn = 0;
            const bool nlive = un < n_units && load_unit(s, sc, L, nsb, un - nbu, gn, n0, n1);
            road_unit(cam, L, live, gq, q0, q1);
            u = un;
            q0 = n0;
            q1 = n1;
            gq = gn;
            live = nlive;
        }
        __syncthreads();
        const int nring = L.cnt[R_RING];
        const bool more = L.cnt[R_NEXT] < n_units;
        // the ring cut into jobs of at most kSetupBatch strips, as many as a
        // multiple of the wavefronts, of equal size: a job's set-up takes about
        // the same time for any number of strips up to a wavefront's width
        const int njobs = (max(K, (nring + kSetupBatch - 1) / kSetupBatch) + K - 1) / K * K;
        const int jsz = (nring + njobs - 1) / njobs;
        // B2
        for (;;) {
            int j = 0;
            if (ln == 0) j = lds_add(L.cnt + R_JOB, 1);
            j = __builtin_amdgcn_readfirstlane(__shfl(j, 0)) - box_jobs;
            if (j < 0) {
                do_boxes(s, sc, cam, ego, L, j + box_jobs, (lptr<int32_t>)ws.tris);   // the staging is free here
                continue;
            }
            const int a = j * jsz;
            if (a >= nring) break;
            setup_job(s, cam, L, ws, a, min(jsz, nring - a));
        }
        __syncthreads();
        box_jobs = 0;
        if (!more) break;
        if (tid == 0) {
            L.cnt[R_RING] = 0;
            L.cnt[R_RESV] = 0;
            L.cnt[R_JOB] = 0;
        }
        __syncthreads();
    }

    // ---- C: resolve
    uint8_t *img = o.rgb + 3 * ((int64_t)view * W * H);
    const int nbt = L.cnt[R_NBT];
    const bool ovf = L.cnt[R_BOVF] != 0;
    int kr0 = H, kr1 = H;          // rows that need the key band
    if (ovf) {
        kr0 = 0;
    } else if (nbt > 0) {
        kr0 = L.cnt[R_BMIN];
        kr1 = L.cnt[R_BMAX] + 1;
    }
    // the box rows are the costly part of the resolve (a mean view has about a dozen)
    view_priority(max(prio_b, kr1 - kr0 >= 64 ? 3 : (kr1 - kr0 >= 32 ? 2 : 0)));
    const uint32_t road_rgb = L.pal[s.road_color0], bg_rgb = L.pal[0];
    const int mrows = mask_rows_fit(L.region, nbt, W);
    if (!ovf && nbt <= kMaskTris && mrows >= 1 && kr0 < kr1) {
        // box rows through row masks, in chunks of rows whose items fit; the
        // rows outside them (the pattern table: coverage bits and table only)
        // go with the first chunk's spans (which write the free region only)
        for (int c0 = kr0; c0 < kr1; c0 += mrows) {
            const int c1 = min(c0 + mrows, kr1);
            if (c0 != kr0) __syncthreads();
            lptr<unsigned long long> M = (lptr<unsigned long long>)L.sbins;
            for (int p = tid; p < 2 * (W >> 4) * (c1 - c0); p += B) M[p] = 0ull;
            __syncthreads();
            if (c0 == kr0) {
                resolve_lut(L, cam, img, 0, kr0);
                resolve_lut(L, cam, img, kr1, H);
            }
            box_spans(L, cam, nbt, c0, c1, wv, K);
            __syncthreads();
            resolve_masks(L, cam, img, road_rgb, bg_rgb, c0, c1, wv, K);
        }
        return;
    }
    resolve_lut(L, cam, img, 0, kr0);
    resolve_lut(L, cam, img, kr1, H);
    if (kr0 < kr1) key_band_rows(s, sc, cam, ego, L, img, road_rgb, bg_rgb, kr0, kr1, ovf, nbt, wv, K);
}

__device__ __forceinline__ void carve_rgb(unsigned char *smem, RgbLds &L, int W, int H, const RgbCfg &c)
{
    const RgbLayout l = rgb_layout(W, H, c);
    L.cnt = (lptr<int32_t>)(smem + l.cnt);
    L.pal = (lptr<uint32_t>)(smem + l.pal);
    L.lut = (lptr<uint32_t>)(smem + l.lut);
    L.bits = (lptr<unsigned long long>)(smem + l.bits);
    L.btris = (lptr<TriRec>)(smem + l.btris);
    L.sbins = (lptr<int32_t>)(smem + l.sbins);
    L.cq = (lptr<int32_t>)(smem + l.cq);
    L.sring = (lptr<int32_t>)(smem + l.sring);
    L.waves = (lptr<unsigned char>)(smem + l.waves);
    L.nw = (W + 63) >> 6;
    L.bcap = c.bcap;
    // the key band takes the surviving-bin list, the box clip queue and the
    // waves' staging, all idle by then
    L.region = (int)(l.total - l.sbins);
    L.krows = max(1, L.region / (8 * W));
}

__device__ __forceinline__ void load_palette_rgb(const DevSim &s, const RgbLds &L)
{
    auto rgb_of = [&](int idx) -> uint32_t {
        return (uint32_t)s.palette[3 * idx] | ((uint32_t)s.palette[3 * idx + 1] << 8) |
               ((uint32_t)s.palette[3 * idx + 2] << 16);
    };
    for (int p = threadIdx.x; p < 256; p += blockDim.x) L.pal[p] = rgb_of(p);
    if (threadIdx.x < 16) {
        // pattern b: pixel k is road where bit k of b is set, background elsewhere
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

// mode 0: view view_begin + blockIdx.x; 1: view order[blockIdx.x]; 2: the
// persistent work queue
template <int K>
__global__ __launch_bounds__(64 * K) __attribute__((amdgpu_waves_per_eu(4))) void k_render_rgb(DevSim s, RenderOut o, RgbCfg c, int mode, int view_begin)
{
    extern __shared__ __align__(16) unsigned char smem[];
    RgbLds L;
    carve_rgb(smem, L, s.width, s.height, c);
    load_palette_rgb(s, L);
    __shared__ int s_item;
    if (mode != 2) {
        __syncthreads();
        const int view = mode == 0 ? view_begin + (int)blockIdx.x : s.order[blockIdx.x];
        render_view_rgb<K>(s, o, L, view);
        return;
    }
    int cur = (int)(blockIdx.x % kQueues);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = queue_take(s, cur);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= s.n_views) break;
        render_view_rgb<K>(s, o, L, s.queue[it]);
    }
    if (threadIdx.x == 0) queue_leave(s);
}

}  // namespace

size_t rgb_lds_bytes(int width, int height, const RgbCfg &c) { return rgb_layout(width, height, c).total; }

hipError_t launch_render_rgb(const DevSim &s, const RenderOut &o, const RgbCfg &c, int mode, int view_begin,
                             int grid, hipStream_t st)
{
    if (grid <= 0) return hipSuccess;
    const size_t lds = rgb_lds_bytes(s.width, s.height, c);
    switch (c.waves) {
    case 1: hipLaunchKernelGGL(k_render_rgb<1>, dim3(grid), dim3(64), lds, st, s, o, c, mode, view_begin); break;
    case 2: hipLaunchKernelGGL(k_render_rgb<2>, dim3(grid), dim3(128), lds, st, s, o, c, mode, view_begin); break;
    case 4: hipLaunchKernelGGL(k_render_rgb<4>, dim3(grid), dim3(256), lds, st, s, o, c, mode, view_begin); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gp
