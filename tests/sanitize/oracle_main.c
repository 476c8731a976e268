/* Driver that runs every entry point of the oracle on generated scenes, for
 * an AddressSanitizer / UndefinedBehaviorSanitizer build on the host (the
 * oracle is test infrastructure; this only checks that it stays in bounds
 * and free of undefined behaviour on the inputs the tests give it, including
 * the degenerate ones).  Built and run by tests/test_sanitize.py. */
#include "../../oracle/gp_oracle.c"

#include <stdio.h>
#include <stdlib.h>

static uint64_t lcg_state = 0x5EED5A17ull;
static float urand(float lo, float hi)
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return lo + (hi - lo) * (float)((lcg_state >> 40) * (1.0 / 16777216.0));
}

int main(void)
{
    enum { NA = 24, NR = 60, NS = 4, NG = 3 };
    float st[NA * 4], dm[NA * 3], roads[NR * 8], sxp[NS * 3], sdm[NS * 3], sig[NG * 4], act[NA * 2];
    uint8_t acol[NA], rcol[NR], scol[NS], gcol[NG], pal[256 * 3], halted[NA], flags[NA], jact[NA];
    float actu[NA * 4], cs[NA * 2];
    for (int i = 0; i < 256 * 3; ++i) pal[i] = (uint8_t)(i * 37);
    for (int a = 0; a < NA; ++a) {
        /* some boxes right next to the ego (near-plane and guard-band clips) */
        const float r = a < 6 ? urand(0.3f, 3.0f) : urand(3.0f, 60.0f);
        const float t = urand(-3.14159f, 3.14159f);
        st[4 * a] = a == 0 ? 0.0f : r * cosf(t);
        st[4 * a + 1] = a == 0 ? 0.0f : r * sinf(t);
        st[4 * a + 2] = urand(-3.2f, 3.2f);
        st[4 * a + 3] = urand(0.0f, 20.0f);
        dm[3 * a] = urand(4.0f, 5.5f);
        dm[3 * a + 1] = urand(1.8f, 2.2f);
        dm[3 * a + 2] = urand(0.2f, 2.0f);
        acol[a] = (uint8_t)(a % 7);
        halted[a] = 0;
    }
    for (int q = 0; q < NR; ++q) {
        /* ordinary strips, a few enormous ones (guard band), degenerate ones */
        const float cx = urand(-80.0f, 80.0f), cy = urand(-80.0f, 80.0f);
        const float hx = q % 10 == 0 ? 1.0e5f : urand(0.5f, 20.0f), hy = q % 13 == 0 ? 0.0f : urand(1.0f, 2.0f);
        const float x[4] = {cx - hx, cx + hx, cx + hx, cx - hx}, y[4] = {cy - hy, cy - hy, cy + hy, cy + hy};
        for (int k = 0; k < 4; ++k) {
            roads[8 * q + 2 * k] = x[k];
            roads[8 * q + 2 * k + 1] = y[k];
        }
        rcol[q] = 1;
    }
    for (int k = 0; k < NS; ++k) {
        sxp[3 * k] = urand(-10.0f, 10.0f);
        sxp[3 * k + 1] = urand(-10.0f, 10.0f);
        sxp[3 * k + 2] = urand(-3.0f, 3.0f);
        sdm[3 * k] = urand(1.0f, 6.0f);
        sdm[3 * k + 1] = urand(0.5f, 2.2f);
        sdm[3 * k + 2] = urand(0.8f, 2.0f);
        scol[k] = 3;
    }
    for (int gi = 0; gi < NG; ++gi) {
        sig[4 * gi] = gi == 0 ? 0.2f : urand(-30.0f, 30.0f);   /* one light around the camera */
        sig[4 * gi + 1] = urand(-30.0f, 30.0f);
        sig[4 * gi + 2] = urand(0.5f, 5.0f);
        sig[4 * gi + 3] = urand(0.25f, 0.4f);
        gcol[gi] = 4;
    }
    gpo_scene sc = {NA, NR, st, dm, acol, roads, rcol, NS, sxp, sdm, scol, NG, sig, gcol};
    const int res[][2] = {{1, 1}, {3, 5}, {64, 64}, {210, 126}};
    long long checksum = 0;
    for (int ri = 0; ri < 4; ++ri) {
        const int W = res[ri][0], H = res[ri][1];
        gpo_camera cam = {W, H, 0.5f * (float)W, 1.6f, 0.5f, 100.0f, pal, ri & 1, {0.3f, 0.4f, 0.866f}, 0.3f};
        uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)W * H);
        uint8_t *rgb = (uint8_t *)malloc((size_t)3 * W * H);
        float *depth = (float *)malloc(sizeof(float) * (size_t)W * H);
        int32_t *prim = (int32_t *)malloc(sizeof(int32_t) * (size_t)W * H);
        for (int ego = 0; ego < 8; ++ego) {
            const float dirs[3][2] = {{1.0f, 0.0f}, {0.5f, 0.8660254f}, {-1.0f, 0.0f}};
            for (int k = 0; k < 3; ++k) {
                long long frags = 0;
                checksum += gpo_render_view(&sc, &cam, ego, dirs[k][0], dirs[k][1], keys, rgb, depth, prim, &frags);
                gpo_raycast_view(&sc, &cam, ego, dirs[k][0], dirs[k][1], keys, rgb, depth, prim);
                checksum += rgb[0] + prim[W * H - 1];
            }
        }
        free(keys);
        free(rgb);
        free(depth);
        free(prim);
    }
    /* the steps with ordinary, extreme and non-finite actions */
    for (int a = 0; a < NA; ++a) {
        act[2 * a] = a % 5 == 0 ? NAN : urand(-100.0f, 100.0f);
        act[2 * a + 1] = a % 7 == 0 ? INFINITY : urand(-2.0f, 2.0f);
        jact[a] = (uint8_t)(a % 14);
        for (int k = 0; k < 4; ++k) actu[4 * a + k] = 0.0f;
    }
    for (int s = 0; s < 20; ++s) {
        gpo_step(NA, st, dm, act, 0.1f, cs, halted);
        gpo_step_jerk(NA, st, dm, actu, jact, 0.1f, cs, halted);
        gpo_infractions(NA, st, dm, NR, roads, halted, flags, NS, sxp, sdm);
    }
    /* coverage of snapped triangles, some past the screen */
    uint8_t count[16 * 9];
    for (int t = 0; t < 50; ++t) {
        int32_t X[3], Y[3];
        for (int k = 0; k < 3; ++k) {
            X[k] = (int32_t)urand(-2000.0f, 6000.0f);
            Y[k] = (int32_t)urand(-2000.0f, 4000.0f);
        }
        for (int p = 0; p < 16 * 9; ++p) count[p] = 0;
        gpo_cover_tri(X, Y, 16, 9, count);
        checksum += count[t % (16 * 9)];
    }
    float sv, cv;
    gpo_sincos(1.0e6f, &sv, &cv);
    checksum += (long long)(gpo_atan_small(0.3f) * 1000.0f);
    printf("oracle sanitize driver ok (checksum %lld)\n", checksum);
    return 0;
}
