// Host driver for the sanitizer build of the library's host runtime: the
// entry points that run without a device (argument checks, orientation
// stencil taps, batch validation and tile lists, the allocation hook).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/se2n.h"

int main() {
    int bad = 0;
    // argument checks that fail before any device work
    se2n_plan p = nullptr;
    bad += se2n_plan_create(nullptr, 64, 16, SE2N_F32) != SE2N_EINVAL;
    bad += se2n_plan_create(&p, 100, 16, SE2N_F32) != SE2N_EINVAL;
    bad += se2n_plan_create(&p, 64, 3, SE2N_F32) != SE2N_EINVAL;
    bad += std::strlen(se2n_last_error()) == 0;
    bad += se2n_workspace_bytes(nullptr) != 0;
    bad += se2n_debug_fail_allocations(-2) != SE2N_EINVAL;
    bad += se2n_debug_fail_allocations(-1) != SE2N_OK;
    // orientation taps for every side class and several widths
    std::vector<float> g(65), d(65);
    int radius = 0;
    const int sides[] = {16, 36, 64, 96, 108, 256, 324, 512, 972, 2048, 4096};
    for (int M : sides)
        for (double sigma : {0.7, 2.0, 5.0}) {
            if (se2n_orient_stencil_taps(M, sigma, g.data(), d.data(), &radius) != SE2N_OK) ++bad;
            for (int j = 0; j < 65; ++j)
                if (!std::isfinite(g[j]) || !std::isfinite(d[j])) ++bad;
        }
    bad += se2n_orient_stencil_taps(100, 2.0, g.data(), d.data(), &radius) != SE2N_EINVAL;
    // batch validation and tile lists (host only)
    std::vector<float> img(1);
    std::vector<uint8_t> m8(1);
    std::vector<se2n_item> items;
    const int Ms[] = {128, 192, 256, 384, 512, 768, 1024};
    for (int i = 0; i < 14; ++i) {
        se2n_item it{};
        it.M = Ms[i % 7];
        it.N = 16 + 8 * (i % 3);
        it.n_steps = 50 + i;
        it.scheme = SE2N_CN;
        it.proj = SE2N_PROJ_MAX;
        it.T = 0.5 + 0.1 * i;
        it.beta = 1.0;
        it.sigma = 2.0;
        it.f = img.data();
        it.mask = m8.data();
        it.out = img.data() + 0;
        items.push_back(it);
    }
    // outputs must not overlap: give each item its own dummy address
    std::vector<float> outs(items.size() * 4);
    for (size_t i = 0; i < items.size(); ++i) items[i].out = outs.data() + 4 * i;
    bad += se2n_batch_workspace_bytes(items.data(), (int)items.size()) == 0;
    for (int pass = 0; pass <= 9; ++pass) {
        int nt = 0;
        if (se2n_batch_tiles(items.data(), (int)items.size(), nullptr, pass, nullptr, 0, &nt) != SE2N_OK) ++bad;
        std::vector<int> tiles(4 * (size_t)nt + 4);
        if (se2n_batch_tiles(items.data(), (int)items.size(), nullptr, pass, tiles.data(), nt, &nt) != SE2N_OK) ++bad;
    }
    se2n_item broken = items[0];
    broken.M = 100;
    bad += se2n_batch_workspace_bytes(&broken, 1) != 0;
    std::printf("host runtime: %d unexpected results\n", bad);
    return bad == 0 ? 0 : 1;
}
