// Host-side construction of the directional kernel set (Sec. III-B).
//
// The eq. 3 mask depends only on the offset's distance, so the device keeps
// one small table indexed by the metric value q (|o|^2 for L2, |o|_1 for L1)
// instead of one K^3 mask kernel per bin; the per-bin part of a kernel is its
// hemispherical shadow, stored as a compressed list of offsets per bin.
#include <math.h>

#include <algorithm>
#include <cstring>

#include "internal.h"

namespace dbtsdf {

namespace {

// integer ceil(sqrt(q)) for q < 2^31
uint32_t isqrt_ceil(uint32_t q) {
    uint32_t r = (uint32_t)sqrt((double)q);
    while ((uint64_t)r * r < q) ++r;
    while (r > 0 && (uint64_t)(r - 1) * (r - 1) >= q) --r;
    return r;
}

uint32_t low_ones(uint32_t n) { return n == 0 ? 0u : (n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u)); }

// the 26 lattice directions in bin order: (sx, sy, sz) enumerated with sx
// slowest, each in -1, 0, 1, skipping the zero vector
void cube26_vectors(int v[26][3]) {
    int b = 0;
    for (int sx = -1; sx <= 1; ++sx)
        for (int sy = -1; sy <= 1; ++sy)
            for (int sz = -1; sz <= 1; ++sz) {
                if (sx == 0 && sy == 0 && sz == 0) continue;
                v[b][0] = sx;
                v[b][1] = sy;
                v[b][2] = sz;
                ++b;
            }
}

double zero_tiny(double v) { return fabs(v) < 1e-12 ? 0.0 : v; }

}  // namespace

// fl32(tan(pi/8)): the CUBE26 sector half-width (22.5 degrees) as a slope.
static const float kTanPi8 = 0.414213562373095f;

int host_bin(const KernelSet &ks, float dx, float dy, float dz) {
    if (ks.p.binning == DBTSDF_BIN_CUBE26) {
        float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
        float m = std::max(ax, std::max(ay, az));
        float lim = kTanPi8 * m;
        int sx = ax >= lim ? (dx > 0.0f ? 1 : -1) : 0;
        int sy = ay >= lim ? (dy > 0.0f ? 1 : -1) : 0;
        int sz = az >= lim ? (dz > 0.0f ? 1 : -1) : 0;
        int code = (sx + 1) * 9 + (sy + 1) * 3 + (sz + 1);
        return code - (code > 13 ? 1 : 0);
    }
    const int baz = (int)ks.p.bins_az, bel = (int)ks.p.bins_el;
    int b_az = 0;
    if (dx != 0.0f || dy != 0.0f) {
        bool lower = dy < 0.0f || (dy == 0.0f && dx < 0.0f);
        float ux = lower ? -dx : dx, uy = lower ? -dy : dy;
        int c = 0;
        for (int k = 1; k < baz / 2; ++k) c += ((ks.az_c[k] * uy) - (ks.az_s[k] * ux)) >= 0.0f;
        b_az = (lower ? baz / 2 : 0) + c;
    }
    float q = ((dx * dx) + (dy * dy)) + (dz * dz);
    float zz = dz * dz;
    int b_el = 0;
    for (int k = 1; k < bel; ++k) {
        float rhs = ks.el_s2[k] * q;
        bool up = dz >= 0.0f;
        b_el += ks.el_neg[k] ? (up || zz <= rhs) : (up && zz >= rhs);
    }
    return b_el * baz + b_az;
}

KernelSet *build_kernel_set(const dbtsdf_kernel_params &p, std::string *err) {
    auto fail = [&](const char *m) -> KernelSet * {
        if (err) *err = m;
        return nullptr;
    };
    if (p.kernel_size < 3 || p.kernel_size > (uint32_t)kMaxK || (p.kernel_size & 1u) == 0)
        return fail("kernel_size must be odd and in 3..37");
    if (p.metric != DBTSDF_DIST_L2 && p.metric != DBTSDF_DIST_L1) return fail("unknown metric");
    if (p.metric == DBTSDF_DIST_L1 && p.kernel_size > 21) return fail("L1 masks need kernel_size <= 21");
    if (p.binning == DBTSDF_BIN_AZEL) {
        if (p.bins_az < 2 || (p.bins_az & 1u) || p.bins_el < 1) return fail("bins_az must be even >= 2, bins_el >= 1");
        if ((uint64_t)p.bins_az * p.bins_el > 65536) return fail("too many bins");
    } else if (p.binning != DBTSDF_BIN_CUBE26) {
        return fail("unknown binning");
    }
    if (p.shadow_model == DBTSDF_SHADOW_CONE) {
        if (!(p.cone_deg > 0.0f && p.cone_deg <= 90.0f)) return fail("cone_deg must be in (0, 90]");
    } else if (p.shadow_model != DBTSDF_SHADOW_HEMISPHERE) {
        return fail("unknown shadow model");
    }

    KernelSet *ks = new KernelSet();
    ks->p = p;
    const int K = (int)p.kernel_size, R = (K - 1) / 2;
    ks->K = K;
    ks->R = R;
    const size_t K3 = (size_t)K * K * K;

    // eq. 3 distance masks
    const uint32_t n_q = p.metric == DBTSDF_DIST_L2 ? (uint32_t)(3 * R * R + 1) : (uint32_t)(3 * R + 1);
    ks->mask_by_q.resize(n_q);
    for (uint32_t q = 0; q < n_q; ++q)
        ks->mask_by_q[q] = low_ones(p.metric == DBTSDF_DIST_L2 ? isqrt_ceil(q) : q);
    ks->cell_mask.resize(K3);
    for (int z = -R; z <= R; ++z)
        for (int y = -R; y <= R; ++y)
            for (int x = -R; x <= R; ++x) {
                uint32_t q = p.metric == DBTSDF_DIST_L2 ? (uint32_t)(x * x + y * y + z * z)
                                                        : (uint32_t)(abs(x) + abs(y) + abs(z));
                ks->cell_mask[((size_t)(z + R) * K + (y + R)) * K + (x + R)] = ks->mask_by_q[q];
            }

    // bin centres and boundary tables
    int cube[26][3];
    cube26_vectors(cube);
    if (p.binning == DBTSDF_BIN_CUBE26) {
        ks->n_bins = 26;
        ks->dirs.resize(26 * 3);
        for (int b = 0; b < 26; ++b) {
            double len = sqrt((double)(cube[b][0] * cube[b][0] + cube[b][1] * cube[b][1] + cube[b][2] * cube[b][2]));
            for (int a = 0; a < 3; ++a) ks->dirs[3 * b + a] = cube[b][a] / len;
        }
    } else {
        const int baz = (int)p.bins_az, bel = (int)p.bins_el;
        ks->n_bins = (uint32_t)(baz * bel);
        ks->dirs.resize((size_t)ks->n_bins * 3);
        for (int e = 0; e < bel; ++e) {
            double el = -M_PI / 2 + M_PI * (e + 0.5) / bel;
            for (int a = 0; a < baz; ++a) {
                double az = 2 * M_PI * (a + 0.5) / baz;
                size_t b = (size_t)e * baz + a;
                ks->dirs[3 * b + 0] = cos(el) * cos(az);
                ks->dirs[3 * b + 1] = cos(el) * sin(az);
                ks->dirs[3 * b + 2] = sin(el);
            }
        }
        ks->az_c.assign(baz / 2 + 1, 0.0f);
        ks->az_s.assign(baz / 2 + 1, 0.0f);
        for (int k = 1; k < baz / 2; ++k) {
            double th = 2 * M_PI * k / baz;
            ks->az_c[k] = (float)zero_tiny(cos(th));
            ks->az_s[k] = (float)zero_tiny(sin(th));
        }
        ks->el_s2.assign(bel + 1, 0.0f);
        ks->el_neg.assign(bel + 1, 0u);
        for (int k = 1; k < bel; ++k) {
            float s = (float)zero_tiny(sin((2.0 * k - bel) * M_PI / (2.0 * bel)));
            ks->el_s2[k] = s * s;
            ks->el_neg[k] = s < 0.0f ? 1u : 0u;
        }
    }
    if (ks->az_c.empty()) {  // keep device pointers valid for CUBE26
        ks->az_c.assign(1, 0.0f);
        ks->az_s.assign(1, 0.0f);
        ks->el_s2.assign(1, 0.0f);
        ks->el_neg.assign(1, 0u);
    }

    // shadows: inside the r_s ball and not in front of the contact voxel
    // (hemisphere), or within the half-angle of the bin direction (cone)
    const bool cone = p.shadow_model == DBTSDF_SHADOW_CONE;
    const double cos_a = cone ? zero_tiny(cos((double)p.cone_deg * M_PI / 180.0)) : 0.0;
    ks->shadow.assign((size_t)ks->n_bins * K3, 0);
    ks->sh_start.assign(ks->n_bins + 1, 0);
    for (uint32_t b = 0; b < ks->n_bins; ++b) {
        ks->sh_start[b] = (uint32_t)ks->sh_off.size();
        if (p.shadow_r2 < 0) continue;
        for (int z = -R; z <= R; ++z)
            for (int y = -R; y <= R; ++y)
                for (int x = -R; x <= R; ++x) {
                    const int r2 = x * x + y * y + z * z;
                    if (r2 > p.shadow_r2) continue;
                    bool back;
                    if (p.binning == DBTSDF_BIN_CUBE26) {
                        const int dot = x * cube[b][0] + y * cube[b][1] + z * cube[b][2];
                        const int s2 = cube[b][0] * cube[b][0] + cube[b][1] * cube[b][1] + cube[b][2] * cube[b][2];
                        back = dot >= 0 && (!cone || (double)dot * (double)dot >= (double)(r2 * s2) * (cos_a * cos_a));
                    } else {
                        const double dot = x * ks->dirs[3 * b] + y * ks->dirs[3 * b + 1] + z * ks->dirs[3 * b + 2];
                        back = cone ? dot >= sqrt((double)r2) * cos_a - 1e-9 : dot >= -1e-9;
                    }
                    if (!back) continue;
                    ks->shadow[(size_t)b * K3 + ((size_t)(z + R) * K + (y + R)) * K + (x + R)] = 1;
                    ks->sh_off.push_back((uint32_t)(x + R) | ((uint32_t)(y + R) << 8) | ((uint32_t)(z + R) << 16));
                }
    }
    ks->sh_start[ks->n_bins] = (uint32_t)ks->sh_off.size();
    if (!build_row_image(*ks, ks->row_image)) ks->row_image.clear();
    if (ks->sh_off.empty()) ks->sh_off.push_back(0);  // non-empty device allocation
    return ks;
}

bool build_row_image(const KernelSet &ks, std::vector<uint32_t> &img) {
    const int K = ks.K, R = ks.R;
    if (K * K > (int)kRowPad || ks.n_bins + 1 > kRowBins || ks.p.shadow_r2 > 9 || ks.sh_off.size() > kShadowTable)
        return false;
    for (uint32_t b = 0; b < ks.n_bins; ++b)
        if (ks.sh_start[b + 1] - ks.sh_start[b] > 128) return false;
    for (uint32_t m : ks.mask_by_q)
        if (m >= 0x8000u) return false;
    img.assign(kImgWords, 0u);
    const bool l1 = ks.p.metric == DBTSDF_DIST_L1;
    for (uint32_t sel = 0; sel < kRowSel; ++sel)
        for (uint32_t row = 0; row < kRowPad; ++row) {
            const int dy = (int)(row % K) - R, dz = (int)(row / K) - R;
            uint32_t m16[4];
            for (int j = 0; j < 4; ++j) {
                const int dx = (int)sel - 3 - R + j;
                m16[j] = 0xFFFFu;
                if (row < (uint32_t)(K * K) && dx >= -R && dx <= R) {
                    const uint32_t q = l1 ? (uint32_t)(abs(dx) + abs(dy) + abs(dz)) : (uint32_t)(dx * dx + dy * dy + dz * dz);
                    m16[j] = ks.mask_by_q[q] & 0xFFFFu;
                }
            }
            img[kImgMtab + 2 * (sel * kRowPad + row) + 0] = m16[0] | (m16[1] << 16);
            img[kImgMtab + 2 * (sel * kRowPad + row) + 1] = m16[2] | (m16[3] << 16);
        }
    const uint32_t n_sh = ks.sh_start[ks.n_bins];
    for (uint32_t j = 0; j < n_sh; ++j) img[kImgShPk + j] = ks.sh_off[j];
    for (uint32_t b = 0; b < ks.n_bins; ++b)
        for (uint32_t j = ks.sh_start[b]; j < ks.sh_start[b + 1]; ++j) {
            const uint32_t pk = ks.sh_off[j];
            const int dx = (int)(pk & 255u) - R, dy = (int)((pk >> 8) & 255u) - R, dz = (int)((pk >> 16) & 255u) - R;
            const uint32_t idx = (uint32_t)((dx + 3) + 7 * (dy + 3) + 49 * (dz + 3));
            img[kImgShBits + b * kShadowSetWords + idx / 32] |= 1u << (idx % 32);
        }
    for (uint32_t b = 0; b <= ks.n_bins; ++b) img[kImgShRng + b] = ks.sh_start[b];
    return true;
}

}  // namespace dbtsdf
