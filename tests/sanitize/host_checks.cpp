// The library's host-side code (kernel-set builder, row-kernel table image,
// Marching Cubes case tables, sweep constants) run under AddressSanitizer and
// UndefinedBehaviorSanitizer. Built with g++ by tests/test_sanitizers.py; no
// device is touched. Exit status 0 and "ok" on success.
#include <cmath>
#include <cstdio>
#include <memory>
#include <string>
#include <vector>

#include "../../paper_2509_20081_amd/csrc/runtime.h"

namespace dbtsdf {
void set_error(const std::string &) {}   // the C ABI's error slot is not linked here
}

int main() {
    using namespace dbtsdf;
    struct Case {
        uint32_t K, binning, baz, bel;
        int32_t r2;
        uint32_t metric, model;
        float cone;
    };
    const Case cases[] = {
        {3, DBTSDF_BIN_CUBE26, 0, 0, 1, DBTSDF_DIST_L2, DBTSDF_SHADOW_HEMISPHERE, 90.0f},
        {11, DBTSDF_BIN_CUBE26, 0, 0, 9, DBTSDF_DIST_L2, DBTSDF_SHADOW_HEMISPHERE, 90.0f},
        {11, DBTSDF_BIN_CUBE26, 0, 0, 9, DBTSDF_DIST_L2, DBTSDF_SHADOW_CONE, 35.0f},
        {7, DBTSDF_BIN_AZEL, 8, 5, 6, DBTSDF_DIST_L1, DBTSDF_SHADOW_HEMISPHERE, 90.0f},
        {21, DBTSDF_BIN_AZEL, 40, 40, 9, DBTSDF_DIST_L2, DBTSDF_SHADOW_HEMISPHERE, 90.0f},
        {37, DBTSDF_BIN_CUBE26, 0, 0, 36, DBTSDF_DIST_L2, DBTSDF_SHADOW_CONE, 50.0f},
        {5, DBTSDF_BIN_AZEL, 256, 130, 4, DBTSDF_DIST_L2, DBTSDF_SHADOW_HEMISPHERE, 90.0f},
    };
    unsigned long long sum = 0;
    for (const Case &c : cases) {
        dbtsdf_kernel_params p{};
        p.kernel_size = c.K;
        p.binning = c.binning;
        p.bins_az = c.baz;
        p.bins_el = c.bel;
        p.shadow_r2 = c.r2;
        p.metric = c.metric;
        p.shadow_model = c.model;
        p.cone_deg = c.cone;
        std::string err;
        std::unique_ptr<KernelSet> ks(build_kernel_set(p, &err));
        if (!ks) {
            std::printf("kernel set K=%u rejected: %s\n", c.K, err.c_str());
            return 1;
        }
        std::vector<uint32_t> img;
        if (build_row_image(*ks, img))
            for (uint32_t w : img) sum += w;
        for (uint32_t m : ks->mask_by_q) sum += m;
        sum += ks->sh_off.size();
    }
    // invalid parameter sets are rejected, not read past
    dbtsdf_kernel_params bad{};
    bad.kernel_size = 4;
    std::string err;
    std::unique_ptr<KernelSet> none(build_kernel_set(bad, &err));
    if (none) return 2;
    const MeshTable &t = mesh_table();
    for (int cs = 0; cs < 256; ++cs)
        for (uint32_t k = 0; k < kMeshCaseBytes; ++k) sum += t.b[cs][k] + t.tri[cs][k % kMeshTriBytes];
    // sweep constants over a range of turns, both modes, and the degenerate ones
    for (int i = 0; i < 2000; ++i) {
        const double a = 0.0031 * i, c = std::cos(a), s = std::sin(a);
        const float p0[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
        const float p1[16] = {(float)c, (float)-s, 0, 0.5f, (float)s, (float)c, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
        float out[7];
        for (int mode = 0; mode < 2; ++mode) {
            if (!sweep_constants(p0, p1, mode, out)) return 3;
            sum += (unsigned long long)(out[0] * 1000.0f);
        }
    }
    const float up[16] = {0, 0, 1, 0, 0, 1, 0, 0, -1, 0, 0, 0, 0, 0, 0, 1};   // x axis taken to the vertical
    const float eye[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
    float out[7];
    if (!sweep_constants(eye, up, DBTSDF_DESKEW_YAW, out) || out[0] != 1.0f) return 4;
    if (sweep_constants(eye, up, 9, out)) return 5;
    std::printf("ok %llu\n", sum);
    return 0;
}
