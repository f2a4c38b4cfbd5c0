// Drives libimask's host code (argument validation, workspace and table
// sizing, batch buffer sizing, the launch-shape table, host draws and the
// step-size rules) for a build with host-side AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_sanitize_cpu.py).  Nothing here
// reaches a device: every call either is host-only or is rejected during
// validation.  Exit status 0 on success.
#include <cmath>
#include <cstdio>
#include <vector>

#include "imask.h"

static int fails = 0;
#define EXPECT(cond)                                               \
    do {                                                           \
        if (!(cond)) {                                             \
            std::printf("line %d: %s\n", __LINE__, #cond);         \
            ++fails;                                               \
        }                                                          \
    } while (0)

static imask_levels levels(std::vector<int> l, int mode = IMASK_FULL_PAPER, int blocks = 1)
{
    imask_levels lv{};
    lv.r = (int)l.size();
    for (int j = 0; j < lv.r; ++j) {
        lv.log2f[j] = l[j];
        lv.p[j] = 1.0 / lv.r;
    }
    lv.full_mode = mode;
    lv.n_blocks = blocks;
    return lv;
}

int main()
{
    // sizes over a range of geometries (parallel, listed angles, fan beam)
    std::vector<double> ang(50);
    for (int a = 0; a < 50; ++a) ang[a] = 0.13 * a - 2.0;
    const int sides[] = {16, 48, 64, 96, 256, 384, 512, 1024, 4096};
    for (int n : sides)
        for (int fan = 0; fan < 2; ++fan)
            for (int listed = 0; listed < 2; ++listed) {
                imask_geometry g{};
                g.n = n;
                g.n_angles = listed ? 50 : 3 * n / 2;
                g.n_det = 3 * n / 2 + 3;
                g.angles = listed ? ang.data() : nullptr;
                g.src_dist = fan ? 4.0 : 0.0;
                g.det_dist = fan ? 2.0 : 0.0;
                g.extent = 1.3;
                const size_t ws = imask_workspace_bytes(&g);
                EXPECT(ws > 0);
                imask_levels lv = levels({0, 1, 2});
                EXPECT(imask_phi_floats(&g, &lv) > 0);
                EXPECT(imask_constants_scratch_bytes(&g) > 0);
            }
    // invalid geometries and level sets are refused with 0 bytes
    imask_geometry bad{};
    bad.n = 63;
    bad.n_angles = 10;
    bad.n_det = 10;
    EXPECT(imask_workspace_bytes(&bad) == 0);
    bad.n = 64;
    bad.extent = std::nan("");
    EXPECT(imask_workspace_bytes(&bad) == 0);
    imask_geometry g{};
    g.n = 64;
    g.n_angles = 90;
    g.n_det = 92;
    imask_levels lbad = levels({1, 2});
    EXPECT(imask_phi_floats(&g, &lbad) == 0);
    // batch buffers of mixed problems
    {
        std::vector<imask_geometry> gs(40, g);
        std::vector<imask_levels> ls(40);
        for (int q = 0; q < 40; ++q) {
            gs[q].n = 32 << (q % 4);
            gs[q].n_angles = gs[q].n_det = 3 * gs[q].n / 2;
            ls[q] = q % 3 == 0 ? levels({0, 1, 2, 3}) : q % 3 == 1 ? levels({0, 2}, IMASK_FULL_UNBIASED) : levels({0});
        }
        EXPECT(imask_batch_bytes(40, gs.data(), ls.data()) > 0);
        EXPECT(imask_batch_bytes(-1, gs.data(), ls.data()) == 0);
    }
    // the launch-shape table
    imask_tiles t{2, 4, 2048, 78}, got{};
    EXPECT(imask_set_tiles(256, 384, 384, &t) == IMASK_OK);
    EXPECT(imask_get_tiles(256, 384, 384, &got) == IMASK_OK && got.bp_wg == 2048 && got.fwd_lds_kb == 78);
    imask_tiles tb{3, 3, 0, 0};
    EXPECT(imask_set_tiles(256, 384, 384, &tb) == IMASK_EINVAL);
    EXPECT(imask_set_tiles(256, 384, 384, nullptr) == IMASK_OK);
    // host draws
    imask_params prm{};
    prm.sigma = 0.01;
    prm.seed = 42;
    prm.stream_id = 3;
    imask_levels lv = levels({0, 1, 2, 3});
    std::vector<int32_t> dr(1000), bl(1000);
    EXPECT(imask_draws(&prm, &lv, 5, 1000, dr.data()) == IMASK_OK);
    for (int v : dr) EXPECT(v >= 0 && v < 4);
    imask_levels lvb = levels({0, 1}, IMASK_FULL_PAPER, 6);
    EXPECT(imask_block_draws(&prm, &lvb, 5, 1000, bl.data()) == IMASK_OK);
    for (int v : bl) EXPECT(v >= 0 && v < 6);
    EXPECT(imask_draws(&prm, &lv, 5, -1, dr.data()) == IMASK_EINVAL);
    // step-size rules
    double s = 0.0, th = 0.0;
    EXPECT(imask_sigma_thm3(5431.0, 1358.0, 5432.0, 0.25, 64, &s, &th) == IMASK_OK && s > 0.0 && th < 1.0);
    EXPECT(imask_sigma_balamurugan(5431.0, 1358.0, &s) == IMASK_OK && s > 0.0);
    EXPECT(imask_sigma_thm3(-1.0, 1.0, 1.0, 0.25, 64, &s, &th) == IMASK_EINVAL);
    // validation of the device entry points (nothing is launched)
    imask_reg reg{IMASK_REG_TIKHONOV, 0.01, 0.0, 1e-3, 10};
    imask_state st{};
    const float* b = nullptr;
    EXPECT(imask_step(1, &g, &lv, &reg, &prm, &b, &st, 1, nullptr) == IMASK_EINVAL);
    EXPECT(imask_solve(1, &g, &lv, &reg, &prm, &b, &st, -1.0, IMASK_BUDGET_ITERS, nullptr) == IMASK_EINVAL);
    EXPECT(imask_step_timed(&g, &lv, &reg, &prm, nullptr, &st, -1, nullptr, nullptr) == IMASK_EINVAL);
    EXPECT(imask_project(&g, 9, nullptr, nullptr, nullptr, nullptr) == IMASK_EINVAL);
    EXPECT(imask_backproject(&g, -1, nullptr, nullptr, nullptr, nullptr) == IMASK_EINVAL);
    EXPECT(imask_resample(63, 1, IMASK_RESTRICT, nullptr, nullptr, nullptr, nullptr) == IMASK_EINVAL);
    EXPECT(imask_backproject_noalloc(&g, 0, nullptr, nullptr, nullptr) == IMASK_EINVAL);
    imask_geometry huge = g;
    huge.n = 1024;
    float dummy = 0.0f;
    EXPECT(imask_backproject_noalloc(&huge, 0, &dummy, &dummy, nullptr) == IMASK_ESIZE);
    EXPECT(imask_batch_step(1, &g, &lv, nullptr, 1, nullptr) == IMASK_EINVAL);
    EXPECT(imask_batch_step_part(1, &g, &lv, &dummy, 7, nullptr) == IMASK_EINVAL);
    std::printf(fails ? "FAILED %d\n" : "ok\n", fails);
    return fails ? 1 : 0;
}
