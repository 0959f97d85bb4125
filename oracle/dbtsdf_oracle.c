/*
 * Plain single-threaded CPU oracle of DB-TSDF scan integration
 * (Maese, Merino, Caballero, "DB-TSDF: Directional Bitmask-based Truncated
 * Signed Distance Fields for Efficient Volumetric Mapping", arXiv 2509.20081).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the reference the GPU library is
 * checked against. It is called from the test suite, from the package's smoke
 * check and from the benchmark's CPU-baseline leg, and from nowhere else. It
 * shares no code, header, table or constant with the GPU library: every table
 * is rebuilt here from the paper's definitions.
 *
 * Every step is written the slow, obvious way, in the paper's order:
 *   Sec. III-C  transform each return into the map frame with the pose,
 *               discard returns whose K^3 neighbourhood leaves the map,
 *               quantise the direction into a bin (eq. 2), then per voxel of
 *               the neighbourhood AND the kernel mask (eq. 4) and, inside the
 *               bin's shadow, bump the saturating hit counter (eq. 5) and set
 *               the sign on the threshold crossing (eq. 6).
 *   Sec. III-A  voxel = 32-bit distance mask + sign + hit counter; start state
 *               mask all ones, sign free, counter zero.
 *   Sec. III-B  direction bins, distance-mask kernel (eq. 3), hemispherical
 *               L2 shadow of radius r_s behind the contact voxel.
 *   Sec. IV-B   within one frame only the first return per voxel is integrated.
 *
 * Readings of the paper where it is silent or ambiguous (the same readings
 * the library implements):
 *   - mask distance is the L2 norm of eq. 3 (the text also says "L1"; L1 is an
 *     option, n = |x|+|y|+|z|);
 *   - the counter is a 16-bit field (h in bits 0-15), the sign is bit 31 of a
 *     second 32-bit word, bits 16-30 stay zero ("packed" word);
 *   - the sign is cleared when h_old < T <= h_new (eq. 6 with ">= T");
 *   - the direction used for binning and for the shadow is d = R p, the
 *     sensor-to-point vector in map axes;
 *   - azimuth/elevation bins of eq. 2 are decided by sign tests against fp32
 *     boundary tables (bin 0 starts at +x, counter-clockwise; elevation bin 0
 *     at the nadir), so no libm call sits on the per-point path;
 *   - a 26-direction cube binning (8 azimuths x 3 elevations + 2 poles) is the
 *     alternative kernel set, with exact integer shadows;
 *   - the shadow is {o : o.o <= r_s^2, o.u_b >= 0}, contact voxel and the planar
 *     face included;
 *   - the conical shadow the paper contrasts with it (Sec. IV-A, no aperture
 *     given) is {o : o.o <= r_s^2, o = 0 or the angle between o and u_b at
 *     most alpha}: o.u_b >= |o| cos(alpha), with cos(alpha) computed in fp64
 *     and snapped to 0 below 1e-12 (so alpha = 90 deg is the hemisphere);
 *     cube bins test (o.s)^2 >= (o.o)(s.s) cos^2(alpha) with o.s >= 0 on the
 *     integer direction s;
 *   - "first return" = lowest input index among valid, in-bounds returns;
 *   - non-finite or zero-range returns are skipped and counted;
 *   - the front end is fp32, one IEEE operation at a time, no FMA contraction
 *     (build with -ffp-contract=off);
 *   - motion compensation (Sec. III-C, "yaw-only or full SE(3)", no scheme
 *     given): a sweep has a start pose (R0, t0) and an end pose (R1, t1), each
 *     return a time fraction tau in [0, 1] (outside, or not a number: the
 *     return is invalid). The rotation over the sweep, Q = R1 R0^T (fp64),
 *     becomes a unit quaternion q with w >= 0 (Shepperd's method; for
 *     yaw-only, the rotation about z that takes Q's x axis, projected on the
 *     xy plane, to where Q takes it: q = (c, 0, 0, s) with (c, s) the unit
 *     half-angle vector, (1, 0, 0, 0) when the projection vanishes), rounded
 *     to fp32, and dt = t1 - t0 (fp32). Per return, in fp32: the normalised
 *     linear interpolation between the identity and q, p(tau) = (1 - tau, 0,
 *     0, 0) + tau q, taken as the rotation matrix M of a quaternion of any
 *     length (2 / |p|^2 in place of 2), R(tau) = M R0 and t(tau) = t0 + tau dt;
 *     the return is then transformed with (R(tau), t(tau)) as above. No sine,
 *     cosine or square root sits on the per-return path.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_BIN_AZEL 0
#define ORC_BIN_CUBE26 1
#define ORC_METRIC_L2 0
#define ORC_METRIC_L1 1
#define ORC_SHADOW_HEMISPHERE 0
#define ORC_SHADOW_CONE 1

typedef struct {
    uint32_t kernel_size;     /* K, odd */
    uint32_t binning;         /* ORC_BIN_* */
    uint32_t bins_az;         /* azimuth bins (AZEL), even */
    uint32_t bins_el;         /* elevation bins (AZEL) */
    int32_t shadow_r2;        /* r_s^2 in voxel^2; negative = no shadow */
    uint32_t metric;          /* ORC_METRIC_* */
    uint32_t dims[3];         /* Nx, Ny, Nz */
    float voxel_size;         /* metres */
    float origin[3];          /* map coordinate of the min corner of voxel (0,0,0) */
    uint32_t hit_threshold;   /* T */
    uint32_t hit_max;         /* H_max */
    uint32_t dedup;           /* 1 = integrate only the first return per voxel per scan */
    uint32_t shadow_model;    /* ORC_SHADOW_* */
    float cone_deg;           /* half-angle alpha of the conical shadow, degrees in (0, 90] */
} orc_params;

typedef struct {
    uint64_t n_in, n_invalid, n_out_of_bounds, n_duplicate, n_integrated;
    uint64_t voxel_updates, shadow_updates;
    uint64_t u_mask, c_mask, u_shadow; /* unique mask words read (kernel mask not all ones) / changed, unique shadow words */
} orc_stats;

typedef struct {
    orc_params p;
    int R;
    int K;
    uint32_t n_bins;
    uint32_t *mask_k;        /* K^3 eq. 3 masks, index ((dz+R)*K + (dy+R))*K + (dx+R) */
    uint8_t *shadow_k;       /* n_bins * K^3 flags */
    double *dirs;            /* n_bins * 3 bin-centre unit vectors */
    float *az_c, *az_s;      /* AZEL azimuth boundary tables, k = 1..B_az/2-1 */
    float *el_s2;            /* squared elevation boundary sines, k = 1..B_el-1 */
    int8_t *el_neg;          /* 1 when the boundary sine is negative */
    /* per-scan dedup set */
    uint64_t *seen;
    uint64_t seen_cap;
    /* optional traffic bitmaps */
    uint8_t *bm_touch, *bm_change, *bm_shadow;
} orc_ctx;

static const float ORC_TAN_PI_8 = 0.414213562373095f; /* fl32(tan(pi/8)) */

/* ---- eq. 3: distance-mask kernel ---------------------------------------- */

/* smallest n >= 0 with n*n >= q (integer ceil of the square root) */
static uint32_t ceil_sqrt_u32(uint32_t q)
{
    uint32_t n = 0;
    while (n * n < q)
        n++;
    return n;
}

static uint32_t cell_bits(const orc_params *p, int dx, int dy, int dz)
{
    if (p->metric == ORC_METRIC_L1)
        return (uint32_t)(abs(dx) + abs(dy) + abs(dz));
    return ceil_sqrt_u32((uint32_t)(dx * dx + dy * dy + dz * dz));
}

static uint32_t mask_of_bits(uint32_t n)
{
    if (n == 0)
        return 0u;
    return 0xFFFFFFFFu >> (32u - n);
}

/* ---- eq. 2: direction bins ---------------------------------------------- */

static double snap(double v) { return fabs(v) < 1e-12 ? 0.0 : v; }

static int bin_cube26(const float d[3])
{
    float a[3], m, t;
    int s[3], k, idx;
    for (k = 0; k < 3; k++)
        a[k] = fabsf(d[k]);
    m = a[0];
    if (a[1] > m)
        m = a[1];
    if (a[2] > m)
        m = a[2];
    t = ORC_TAN_PI_8 * m;
    for (k = 0; k < 3; k++) {
        if (a[k] >= t)
            s[k] = d[k] > 0.0f ? 1 : -1;
        else
            s[k] = 0;
    }
    idx = 9 * (s[0] + 1) + 3 * (s[1] + 1) + (s[2] + 1);
    return idx > 13 ? idx - 1 : idx;
}

static int bin_azel(const orc_ctx *c, const float d[3])
{
    const int baz = (int)c->p.bins_az, bel = (int)c->p.bins_el;
    int b_az = 0, b_el = 0, k;
    float x = d[0], y = d[1], z = d[2];
    if (!(x == 0.0f && y == 0.0f)) {
        int half = (y < 0.0f) || (y == 0.0f && x < 0.0f);
        float xp = half ? -x : x, yp = half ? -y : y;
        int cnt = 0;
        for (k = 1; k <= baz / 2 - 1; k++) {
            float lhs = c->az_c[k] * yp;
            float rhs = c->az_s[k] * xp;
            if (lhs - rhs >= 0.0f)
                cnt++;
        }
        b_az = half * (baz / 2) + cnt;
    }
    {
        float xx = x * x, yy = y * y, zz = z * z;
        float q = (xx + yy) + zz;
        for (k = 1; k <= bel - 1; k++) {
            float rhs = c->el_s2[k] * q;
            int pass;
            if (!c->el_neg[k])
                pass = (z >= 0.0f) && (zz >= rhs);
            else
                pass = (z >= 0.0f) || (zz <= rhs);
            if (pass)
                b_el++;
        }
    }
    return b_el * baz + b_az;
}

static int bin_of(const orc_ctx *c, const float d[3])
{
    if (c->p.binning == ORC_BIN_CUBE26)
        return bin_cube26(d);
    return bin_azel(c, d);
}

/* ---- context: kernel tables built from the definitions ------------------ */

static int params_ok(const orc_params *p)
{
    int k;
    if (p->kernel_size < 3 || p->kernel_size > 37 || (p->kernel_size % 2) == 0)
        return 0;
    if (p->metric == ORC_METRIC_L1 && p->kernel_size > 21)
        return 0;
    if (p->metric != ORC_METRIC_L1 && p->metric != ORC_METRIC_L2)
        return 0;
    if (p->binning == ORC_BIN_AZEL) {
        if (p->bins_az < 2 || (p->bins_az % 2) != 0 || p->bins_el < 1)
            return 0;
    } else if (p->binning != ORC_BIN_CUBE26) {
        return 0;
    }
    for (k = 0; k < 3; k++)
        if (p->dims[k] < p->kernel_size)
            return 0;
    if (!(p->voxel_size > 0.0f) || !isfinite(p->voxel_size))
        return 0;
    if (p->hit_max < 1 || p->hit_max > 65535)
        return 0;
    if (p->shadow_model == ORC_SHADOW_CONE) {
        if (!(p->cone_deg > 0.0f && p->cone_deg <= 90.0f))
            return 0;
    } else if (p->shadow_model != ORC_SHADOW_HEMISPHERE) {
        return 0;
    }
    return 1;
}

orc_ctx *orc_create(const orc_params *p)
{
    orc_ctx *c;
    int K, R, b, dx, dy, dz, k;
    if (!params_ok(p))
        return NULL;
    c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    c->p = *p;
    K = (int)p->kernel_size;
    R = (K - 1) / 2;
    c->K = K;
    c->R = R;
    c->n_bins = p->binning == ORC_BIN_CUBE26 ? 26u : p->bins_az * p->bins_el;

    c->mask_k = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)K * K * K);
    for (dz = -R; dz <= R; dz++)
        for (dy = -R; dy <= R; dy++)
            for (dx = -R; dx <= R; dx++)
                c->mask_k[((dz + R) * K + (dy + R)) * K + (dx + R)] =
                    mask_of_bits(cell_bits(p, dx, dy, dz));

    /* bin-centre directions */
    c->dirs = (double *)malloc(sizeof(double) * 3 * c->n_bins);
    if (p->binning == ORC_BIN_CUBE26) {
        for (b = 0; b < 26; b++) {
            int idx = b >= 13 ? b + 1 : b;
            int sx = idx / 9 - 1, sy = (idx / 3) % 3 - 1, sz = idx % 3 - 1;
            double nrm = sqrt((double)(sx * sx + sy * sy + sz * sz));
            c->dirs[3 * b + 0] = sx / nrm;
            c->dirs[3 * b + 1] = sy / nrm;
            c->dirs[3 * b + 2] = sz / nrm;
        }
    } else {
        int baz = (int)p->bins_az, bel = (int)p->bins_el, ia, ie;
        for (ie = 0; ie < bel; ie++)
            for (ia = 0; ia < baz; ia++) {
                double a = 2.0 * M_PI * (ia + 0.5) / baz;
                double e = -M_PI / 2.0 + M_PI * (ie + 0.5) / bel;
                b = ie * baz + ia;
                c->dirs[3 * b + 0] = cos(e) * cos(a);
                c->dirs[3 * b + 1] = cos(e) * sin(a);
                c->dirs[3 * b + 2] = sin(e);
            }
        c->az_c = (float *)calloc((size_t)baz / 2 + 1, sizeof(float));
        c->az_s = (float *)calloc((size_t)baz / 2 + 1, sizeof(float));
        for (k = 1; k <= baz / 2 - 1; k++) {
            double th = 2.0 * M_PI * k / baz;
            c->az_c[k] = (float)snap(cos(th));
            c->az_s[k] = (float)snap(sin(th));
        }
        c->el_s2 = (float *)calloc((size_t)bel + 1, sizeof(float));
        c->el_neg = (int8_t *)calloc((size_t)bel + 1, 1);
        for (k = 1; k <= bel - 1; k++) {
            float sg = (float)snap(sin((2.0 * k - bel) * M_PI / (2.0 * bel)));
            c->el_s2[k] = sg * sg;
            c->el_neg[k] = sg < 0.0f ? 1 : 0;
        }
    }

    /* shadow: o.o <= r_s^2 and o behind the contact voxel: o.u_b >= 0
     * (hemisphere), or within alpha of u_b (cone) */
    c->shadow_k = (uint8_t *)calloc((size_t)c->n_bins * K * K * K, 1);
    {
        const int cone = p->shadow_model == ORC_SHADOW_CONE;
        const double cos_a = cone ? snap(cos((double)p->cone_deg * M_PI / 180.0)) : 0.0;
        for (b = 0; b < (int)c->n_bins; b++) {
        for (dz = -R; dz <= R; dz++)
            for (dy = -R; dy <= R; dy++)
                for (dx = -R; dx <= R; dx++) {
                    int oo = dx * dx + dy * dy + dz * dz;
                    int in_ball = oo <= p->shadow_r2;
                    int behind;
                    if (p->binning == ORC_BIN_CUBE26) {
                        int idx = b >= 13 ? b + 1 : b;
                        int sx = idx / 9 - 1, sy = (idx / 3) % 3 - 1, sz = idx % 3 - 1;
                        int os = dx * sx + dy * sy + dz * sz;
                        behind = os >= 0;
                        if (cone && behind) {
                            int ss = sx * sx + sy * sy + sz * sz;
                            behind = (double)os * (double)os >= (double)(oo * ss) * (cos_a * cos_a);
                        }
                    } else {
                        double dot = dx * c->dirs[3 * b + 0] + dy * c->dirs[3 * b + 1] +
                                     dz * c->dirs[3 * b + 2];
                        behind = cone ? dot >= sqrt((double)oo) * cos_a - 1e-9 : dot >= -1e-9;
                    }
                    if (p->shadow_r2 >= 0 && in_ball && behind)
                        c->shadow_k[(size_t)b * K * K * K + ((dz + R) * K + (dy + R)) * K + (dx + R)] = 1;
                }
        }
    }
    return c;
}

void orc_destroy(orc_ctx *c)
{
    if (!c)
        return;
    free(c->mask_k);
    free(c->shadow_k);
    free(c->dirs);
    free(c->az_c);
    free(c->az_s);
    free(c->el_s2);
    free(c->el_neg);
    free(c->seen);
    free(c->bm_touch);
    free(c->bm_change);
    free(c->bm_shadow);
    free(c);
}

uint32_t orc_n_bins(const orc_ctx *c) { return c->n_bins; }

void orc_export(const orc_ctx *c, uint32_t *masks, uint8_t *shadow, double *dirs)
{
    size_t k3 = (size_t)c->K * c->K * c->K;
    if (masks)
        memcpy(masks, c->mask_k, k3 * sizeof(uint32_t));
    if (shadow)
        memcpy(shadow, c->shadow_k, c->n_bins * k3);
    if (dirs)
        memcpy(dirs, c->dirs, sizeof(double) * 3 * c->n_bins);
}

int orc_bin(const orc_ctx *c, float dx, float dy, float dz)
{
    float d[3] = {dx, dy, dz};
    return bin_of(c, d);
}

/* ---- grid state --------------------------------------------------------- */

void orc_grid_init(const orc_ctx *c, uint32_t *mask, uint32_t *packed)
{
    uint64_t n = (uint64_t)c->p.dims[0] * c->p.dims[1] * c->p.dims[2], i;
    for (i = 0; i < n; i++) {
        mask[i] = 0xFFFFFFFFu;  /* all bits set */
        packed[i] = 0x80000000u; /* sign = free (1), h = 0 */
    }
}

/* ---- front end: transform, validity, voxel, bounds, bin ----------------- */

enum { ST_OK = 0, ST_INVALID = 1, ST_OOB = 2 };

static int front_end(const orc_ctx *c, const float pose[16], const float pt[3], int v[3], int *bin)
{
    float d[3], w[3];
    float inv_s = 1.0f / c->p.voxel_size;
    int k;
    if (!isfinite(pt[0]) || !isfinite(pt[1]) || !isfinite(pt[2]))
        return ST_INVALID;
    for (k = 0; k < 3; k++) {
        float a = pose[4 * k + 0] * pt[0];
        float b = pose[4 * k + 1] * pt[1];
        float e = pose[4 * k + 2] * pt[2];
        d[k] = (a + b) + e;
        w[k] = d[k] + pose[4 * k + 3];
    }
    if (d[0] == 0.0f && d[1] == 0.0f && d[2] == 0.0f)
        return ST_INVALID;
    for (k = 0; k < 3; k++) {
        float f = floorf((w[k] - c->p.origin[k]) * inv_s);
        float lo = (float)c->R;
        float hi = (float)((int)c->p.dims[k] - 1 - c->R);
        if (!(f >= lo && f <= hi))
            return ST_OOB;
        v[k] = (int)f;
    }
    *bin = bin_of(c, d);
    return ST_OK;
}

void orc_front_end(const orc_ctx *c, const float pose[16], const float *pts, uint64_t n,
                   int32_t *vox, int32_t *bins, int32_t *status)
{
    uint64_t i;
    for (i = 0; i < n; i++) {
        int v[3] = {0, 0, 0}, b = -1;
        int st = front_end(c, pose, pts + 3 * i, v, &b);
        status[i] = st;
        vox[3 * i + 0] = v[0];
        vox[3 * i + 1] = v[1];
        vox[3 * i + 2] = v[2];
        bins[i] = st == ST_OK ? b : -1;
    }
}

/* ---- motion compensation (deskew) ---------------------------------------- */

#define ORC_DESKEW_SE3 0
#define ORC_DESKEW_YAW 1

/* unit quaternion (w, x, y, z), w >= 0, of a rotation matrix (row-major),
   Shepperd's method: the branch on the largest of the trace and the diagonal */
static void quat_of_matrix(const double Q[9], double q[4])
{
    double tr = (Q[0] + Q[4]) + Q[8], S, n;
    int k;
    if (tr > 0.0) {
        S = sqrt(tr + 1.0) * 2.0;
        q[0] = 0.25 * S;
        q[1] = (Q[7] - Q[5]) / S;
        q[2] = (Q[2] - Q[6]) / S;
        q[3] = (Q[3] - Q[1]) / S;
    } else if (Q[0] > Q[4] && Q[0] > Q[8]) {
        S = sqrt(((1.0 + Q[0]) - Q[4]) - Q[8]) * 2.0;
        q[0] = (Q[7] - Q[5]) / S;
        q[1] = 0.25 * S;
        q[2] = (Q[1] + Q[3]) / S;
        q[3] = (Q[2] + Q[6]) / S;
    } else if (Q[4] > Q[8]) {
        S = sqrt(((1.0 + Q[4]) - Q[0]) - Q[8]) * 2.0;
        q[0] = (Q[2] - Q[6]) / S;
        q[1] = (Q[1] + Q[3]) / S;
        q[2] = 0.25 * S;
        q[3] = (Q[5] + Q[7]) / S;
    } else {
        S = sqrt(((1.0 + Q[8]) - Q[0]) - Q[4]) * 2.0;
        q[0] = (Q[3] - Q[1]) / S;
        q[1] = (Q[2] + Q[6]) / S;
        q[2] = (Q[5] + Q[7]) / S;
        q[3] = 0.25 * S;
    }
    n = sqrt(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]);
    for (k = 0; k < 4; k++)
        q[k] = q[k] / n;
    if (q[0] < 0.0)
        for (k = 0; k < 4; k++)
            q[k] = -q[k];
}

/* the sweep's constants: out[0..3] = q (fp32), out[4..6] = t1 - t0 (fp32) */
int orc_deskew_constants(const float p0[16], const float p1[16], int mode, float out[7])
{
    double Q[9], q[4];
    int i, j;
    if (mode != ORC_DESKEW_SE3 && mode != ORC_DESKEW_YAW)
        return 1;
    for (i = 0; i < 16; i++)
        if (!isfinite(p0[i]) || !isfinite(p1[i]))
            return 1;
    /* Q = R1 R0^T: Q_ij = sum_k R1_ik R0_jk */
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++)
            Q[3 * i + j] = ((double)p1[4 * i + 0] * (double)p0[4 * j + 0] +
                            (double)p1[4 * i + 1] * (double)p0[4 * j + 1]) +
                           (double)p1[4 * i + 2] * (double)p0[4 * j + 2];
    if (mode == ORC_DESKEW_SE3) {
        quat_of_matrix(Q, q);
    } else {
        /* yaw: Q's x axis projected on the xy plane at angle psi; the half
           angle's unit vector is proportional to (|v| + v_x, v_y) */
        double L = sqrt(Q[0] * Q[0] + Q[3] * Q[3]);
        double hx = L + Q[0], hy = Q[3], H = sqrt(hx * hx + hy * hy);
        q[1] = 0.0;
        q[2] = 0.0;
        if (L == 0.0) {
            q[0] = 1.0;
            q[3] = 0.0;
        } else if (H == 0.0) {
            q[0] = 0.0; /* psi = 180 degrees */
            q[3] = 1.0;
        } else {
            q[0] = hx / H;
            q[3] = hy / H;
        }
    }
    for (i = 0; i < 4; i++)
        out[i] = (float)q[i];
    for (i = 0; i < 3; i++)
        out[4 + i] = p1[4 * i + 3] - p0[4 * i + 3];
    return 0;
}

/* the pose of a return at time fraction tau (fp32, one operation at a time) */
static void deskew_pose(const float p0[16], const float k[7], float tau, float pose[16])
{
    float a = 1.0f - tau;
    float w = a + tau * k[0], x = tau * k[1], y = tau * k[2], z = tau * k[3];
    float ww = w * w, xx = x * x, yy = y * y, zz = z * z;
    float wx = w * x, wy = w * y, wz = w * z, xy = x * y, xz = x * z, yz = y * z;
    float n2 = ((ww + xx) + yy) + zz;
    float s2 = 2.0f / n2;
    float M[9];
    int i, j;
    M[0] = 1.0f - s2 * (yy + zz);
    M[1] = s2 * (xy - wz);
    M[2] = s2 * (xz + wy);
    M[3] = s2 * (xy + wz);
    M[4] = 1.0f - s2 * (xx + zz);
    M[5] = s2 * (yz - wx);
    M[6] = s2 * (xz - wy);
    M[7] = s2 * (yz + wx);
    M[8] = 1.0f - s2 * (xx + yy);
    for (i = 0; i < 3; i++) {
        for (j = 0; j < 3; j++) {
            float u = M[3 * i + 0] * p0[4 * 0 + j];
            float v = M[3 * i + 1] * p0[4 * 1 + j];
            float e = M[3 * i + 2] * p0[4 * 2 + j];
            pose[4 * i + j] = (u + v) + e;
        }
        pose[4 * i + 3] = p0[4 * i + 3] + tau * k[4 + i];
    }
    pose[12] = 0.0f;
    pose[13] = 0.0f;
    pose[14] = 0.0f;
    pose[15] = 1.0f;
}

/* per-return pose of a deskewed sweep, exported for the tests */
void orc_deskew_pose(const float p0[16], const float k[7], float tau, float pose[16]) { deskew_pose(p0, k, tau, pose); }

/* ---- per-scan "already integrated this voxel" set ----------------------- */

static const uint64_t SEEN_EMPTY = ~(uint64_t)0;

static void seen_reset(orc_ctx *c, uint64_t n)
{
    uint64_t cap = 16, i;
    while (cap < 2 * n + 16)
        cap *= 2;
    if (cap != c->seen_cap) {
        free(c->seen);
        c->seen = (uint64_t *)malloc(sizeof(uint64_t) * cap);
        c->seen_cap = cap;
    }
    for (i = 0; i < cap; i++)
        c->seen[i] = SEEN_EMPTY;
}

/* returns 1 if key was already present, inserts it otherwise */
static int seen_test_and_insert(orc_ctx *c, uint64_t key)
{
    uint64_t h = (key * 0x9E3779B97F4A7C15ull) & (c->seen_cap - 1);
    for (;;) {
        if (c->seen[h] == key)
            return 1;
        if (c->seen[h] == SEEN_EMPTY) {
            c->seen[h] = key;
            return 0;
        }
        h = (h + 1) & (c->seen_cap - 1);
    }
}

/* ---- traffic bitmaps ---------------------------------------------------- */

static int bm_set(uint8_t *bm, uint64_t i)
{
    uint8_t bit = (uint8_t)(1u << (i & 7));
    int was = (bm[i >> 3] & bit) != 0;
    bm[i >> 3] |= bit;
    return was;
}

/* ---- one scan ----------------------------------------------------------- */

/* one scan; with times, a deskewed sweep from pose to pose_end (mode ORC_DESKEW_*) */
static int integrate(orc_ctx *c, uint32_t *mask, uint32_t *packed, const float pose[16], const float *pose_end,
                     int mode, const float *times, const float *pts, uint64_t n, orc_stats *st, int count_traffic)
{
    const int K = c->K, R = c->R;
    const uint64_t nx = c->p.dims[0], ny = c->p.dims[1], nz = c->p.dims[2];
    const uint64_t nvox = nx * ny * nz;
    const uint32_t T = c->p.hit_threshold, HMAX = c->p.hit_max;
    uint64_t i, bm_bytes = (nvox + 7) / 8;
    orc_stats s;
    int k;

    float kdesk[7];
    for (k = 0; k < 16; k++)
        if (!isfinite(pose[k]))
            return 1;
    if (times && orc_deskew_constants(pose, pose_end, mode, kdesk) != 0)
        return 1;
    memset(&s, 0, sizeof(s));
    s.n_in = n;
    if (n == 0) {
        if (st)
            *st = s;
        return 0;
    }
    seen_reset(c, n);
    if (count_traffic) {
        if (!c->bm_touch) {
            c->bm_touch = (uint8_t *)calloc(bm_bytes, 1);
            c->bm_change = (uint8_t *)calloc(bm_bytes, 1);
            c->bm_shadow = (uint8_t *)calloc(bm_bytes, 1);
        } else {
            memset(c->bm_touch, 0, bm_bytes);
            memset(c->bm_change, 0, bm_bytes);
            memset(c->bm_shadow, 0, bm_bytes);
        }
    }

    for (i = 0; i < n; i++) {
        int v[3], b, dx, dy, dz;
        int res;
        uint64_t key;
        if (times) {
            float tau = times[i], pp[16];
            if (!(tau >= 0.0f && tau <= 1.0f)) {
                res = ST_INVALID;
            } else {
                deskew_pose(pose, kdesk, tau, pp);
                res = front_end(c, pp, pts + 3 * i, v, &b);
            }
        } else {
            res = front_end(c, pose, pts + 3 * i, v, &b);
        }
        const uint8_t *sh;
        if (res == ST_INVALID) {
            s.n_invalid++;
            continue;
        }
        if (res == ST_OOB) {
            s.n_out_of_bounds++;
            continue;
        }
        key = (uint64_t)v[0] + nx * ((uint64_t)v[1] + ny * (uint64_t)v[2]);
        if (c->p.dedup && seen_test_and_insert(c, key)) {
            s.n_duplicate++;
            continue;
        }
        s.n_integrated++;
        sh = c->shadow_k + (size_t)b * K * K * K;
        for (dz = -R; dz <= R; dz++)
            for (dy = -R; dy <= R; dy++)
                for (dx = -R; dx <= R; dx++) {
                    int cell = ((dz + R) * K + (dy + R)) * K + (dx + R);
                    uint64_t u = (uint64_t)(v[0] + dx) +
                                 nx * ((uint64_t)(v[1] + dy) + ny * (uint64_t)(v[2] + dz));
                    /* eq. 4: AND, write skipped when unchanged */
                    uint32_t g = mask[u];
                    uint32_t g2 = g & c->mask_k[cell];
                    s.voxel_updates++;
                    /* a word whose kernel mask is all ones is left as it is by
                       the AND and need not be read: only the others count */
                    if (count_traffic && c->mask_k[cell] != 0xFFFFFFFFu)
                        bm_set(c->bm_touch, u);
                    if (g2 != g) {
                        mask[u] = g2;
                        if (count_traffic)
                            bm_set(c->bm_change, u);
                    }
                    /* eqs. 5-6: saturating counter and sign on the crossing */
                    if (sh[cell]) {
                        uint32_t word = packed[u];
                        uint32_t h0 = word & 0xFFFFu;
                        uint32_t h1 = h0 + 1 < HMAX ? h0 + 1 : HMAX;
                        uint32_t sign = word & 0x80000000u;
                        if (h0 < T && h1 >= T)
                            sign = 0;
                        packed[u] = sign | h1;
                        s.shadow_updates++;
                        if (count_traffic)
                            bm_set(c->bm_shadow, u);
                    }
                }
    }
    if (count_traffic) {
        uint64_t j;
        for (j = 0; j < bm_bytes; j++) {
            s.u_mask += (uint64_t)__builtin_popcount(c->bm_touch[j]);
            s.c_mask += (uint64_t)__builtin_popcount(c->bm_change[j]);
            s.u_shadow += (uint64_t)__builtin_popcount(c->bm_shadow[j]);
        }
    }
    if (st)
        *st = s;
    return 0;
}

int orc_integrate(orc_ctx *c, uint32_t *mask, uint32_t *packed, const float pose[16],
                  const float *pts, uint64_t n, orc_stats *st, int count_traffic)
{
    return integrate(c, mask, packed, pose, NULL, 0, NULL, pts, n, st, count_traffic);
}

int orc_integrate_deskew(orc_ctx *c, uint32_t *mask, uint32_t *packed, const float pose_start[16],
                         const float pose_end[16], int mode, const float *times, const float *pts, uint64_t n,
                         orc_stats *st, int count_traffic)
{
    return integrate(c, mask, packed, pose_start, pose_end, mode, times, pts, n, st, count_traffic);
}

/* ---- the same scan on every host core (OpenMP) --------------------------

   For timing the CPU on the headline workload only. The front end runs in
   parallel (it reads the tables and writes one slot per return), the
   first-return test stays sequential (the lowest index of each voxel wins, as
   above), and the windows are applied in parallel with an atomic fetch-and
   per mask word and a compare-and-swap loop per counter word. Both updates
   commute (eq. 4 is an AND; c unit steps of eqs. 5-6 in any order end in the
   same word), so the planes equal those of orc_integrate bit for bit.
   Statistics as orc_integrate without the traffic counts. Returns 1 on a
   non-finite pose, 2 when the library was built without OpenMP, 3 when out
   of memory. *threads receives the threads used. */
int orc_integrate_omp(orc_ctx *c, uint32_t *mask, uint32_t *packed, const float pose[16], const float *pts,
                      uint64_t n, orc_stats *st, int *threads)
{
#ifndef _OPENMP
    (void)c; (void)mask; (void)packed; (void)pose; (void)pts; (void)n; (void)st;
    if (threads)
        *threads = 0;
    return 2;
#else
    const int K = c->K, R = c->R;
    const uint64_t nx = c->p.dims[0], ny = c->p.dims[1];
    const uint32_t T = c->p.hit_threshold, HMAX = c->p.hit_max;
    orc_stats s;
    int k;
    int64_t i;
    for (k = 0; k < 16; k++)
        if (!isfinite(pose[k]))
            return 1;
    memset(&s, 0, sizeof(s));
    s.n_in = n;
    if (threads)
        *threads = omp_get_max_threads();
    if (n == 0) {
        if (st)
            *st = s;
        return 0;
    }
    int *vox = (int *)malloc(sizeof(int) * 3 * n);
    int *bins = (int *)malloc(sizeof(int) * n);
    int8_t *res = (int8_t *)malloc(n);
    if (!vox || !bins || !res) {
        free(vox);
        free(bins);
        free(res);
        return 3;
    }
#pragma omp parallel for schedule(static)
    for (i = 0; i < (int64_t)n; i++)
        res[i] = (int8_t)front_end(c, pose, pts + 3 * i, vox + 3 * i, bins + i);
    seen_reset(c, n);
    for (i = 0; i < (int64_t)n; i++) {
        if (res[i] == ST_INVALID) {
            s.n_invalid++;
            continue;
        }
        if (res[i] == ST_OOB) {
            s.n_out_of_bounds++;
            continue;
        }
        const int *v = vox + 3 * i;
        const uint64_t key = (uint64_t)v[0] + nx * ((uint64_t)v[1] + ny * (uint64_t)v[2]);
        if (c->p.dedup && seen_test_and_insert(c, key)) {
            s.n_duplicate++;
            res[i] = -1;   /* lost the first-return test */
            continue;
        }
        s.n_integrated++;
    }
    uint64_t vu = 0, su = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : vu, su)
    for (i = 0; i < (int64_t)n; i++) {
        int dx, dy, dz;
        if (res[i] != ST_OK)
            continue;
        const int *v = vox + 3 * i;
        const uint8_t *sh = c->shadow_k + (size_t)bins[i] * K * K * K;
        for (dz = -R; dz <= R; dz++)
            for (dy = -R; dy <= R; dy++)
                for (dx = -R; dx <= R; dx++) {
                    const int cell = ((dz + R) * K + (dy + R)) * K + (dx + R);
                    const uint64_t u = (uint64_t)(v[0] + dx) + nx * ((uint64_t)(v[1] + dy) + ny * (uint64_t)(v[2] + dz));
                    const uint32_t mk = c->mask_k[cell];
                    vu++;
                    /* words only lose bits: one already inside mk stays inside it */
                    if (mk != 0xFFFFFFFFu) {
                        const uint32_t g = __atomic_load_n(&mask[u], __ATOMIC_RELAXED);
                        if ((g & mk) != g)
                            __atomic_fetch_and(&mask[u], mk, __ATOMIC_RELAXED);
                    }
                    if (sh[cell]) {
                        uint32_t word = __atomic_load_n(&packed[u], __ATOMIC_RELAXED), nw;
                        do {
                            const uint32_t h0 = word & 0xFFFFu;
                            const uint32_t h1 = h0 + 1 < HMAX ? h0 + 1 : HMAX;
                            uint32_t sign = word & 0x80000000u;
                            if (h0 < T && h1 >= T)
                                sign = 0;
                            nw = sign | h1;
                        } while (!__atomic_compare_exchange_n(&packed[u], &word, nw, 0, __ATOMIC_RELAXED,
                                                              __ATOMIC_RELAXED));
                        su++;
                    }
                }
    }
    s.voxel_updates = vu;
    s.shadow_updates = su;
    free(vox);
    free(bins);
    free(res);
    if (st)
        *st = s;
    return 0;
#endif
}

/* signed distance readout: (sign ? +1 : -1) * popcount(mask) */
void orc_read_distance(const orc_ctx *c, const uint32_t *mask, const uint32_t *packed, int8_t *out)
{
    uint64_t n = (uint64_t)c->p.dims[0] * c->p.dims[1] * c->p.dims[2], i;
    for (i = 0; i < n; i++) {
        int pc = __builtin_popcount(mask[i]);
        out[i] = (int8_t)((packed[i] & 0x80000000u) ? pc : -pc);
    }
}
