// Constants of a motion-compensated sweep (host side, fp64).
//
// The paper transforms each return with the estimated pose, optionally with
// yaw-only or full SE(3) motion compensation (Sec. III-C), without fixing a
// scheme. Here a sweep runs from the start pose (R0, t0) to the end pose
// (R1, t1); the rotation over it, Q = R1 R0^T, is reduced once per sweep to a
// unit quaternion q (w >= 0) by Shepperd's method (branch on the largest of
// the trace and the diagonal, one square root), or for yaw-only to the
// rotation about z that turns Q's x axis, projected on the xy plane, to where
// Q turns it: its half-angle unit vector is proportional to (|v| + v_x, v_y).
// The per-return interpolation (fp32, no sine or square root) runs in the
// front kernel.
#include <cmath>

#include "runtime.h"

namespace dbtsdf {

namespace {

void shepperd(const double Q[9], double q[4]) {
    const double tr = (Q[0] + Q[4]) + Q[8];
    if (tr > 0.0) {
        const double S = std::sqrt(tr + 1.0) * 2.0;
        q[0] = 0.25 * S;
        q[1] = (Q[7] - Q[5]) / S;
        q[2] = (Q[2] - Q[6]) / S;
        q[3] = (Q[3] - Q[1]) / S;
    } else if (Q[0] > Q[4] && Q[0] > Q[8]) {
        const double S = std::sqrt(((1.0 + Q[0]) - Q[4]) - Q[8]) * 2.0;
        q[0] = (Q[7] - Q[5]) / S;
        q[1] = 0.25 * S;
        q[2] = (Q[1] + Q[3]) / S;
        q[3] = (Q[2] + Q[6]) / S;
    } else if (Q[4] > Q[8]) {
        const double S = std::sqrt(((1.0 + Q[4]) - Q[0]) - Q[8]) * 2.0;
        q[0] = (Q[2] - Q[6]) / S;
        q[1] = (Q[1] + Q[3]) / S;
        q[2] = 0.25 * S;
        q[3] = (Q[5] + Q[7]) / S;
    } else {
        const double S = std::sqrt(((1.0 + Q[8]) - Q[0]) - Q[4]) * 2.0;
        q[0] = (Q[3] - Q[1]) / S;
        q[1] = (Q[2] + Q[6]) / S;
        q[2] = (Q[5] + Q[7]) / S;
        q[3] = 0.25 * S;
    }
    const double n = std::sqrt(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) q[k] = q[k] / n;
    if (q[0] < 0.0)
        for (int k = 0; k < 4; ++k) q[k] = -q[k];
}

}  // namespace

bool sweep_constants(const float p0[16], const float p1[16], int mode, float out[7]) {
    if (mode != DBTSDF_DESKEW_SE3 && mode != DBTSDF_DESKEW_YAW) return false;
    for (int k = 0; k < 16; ++k)
        if (!std::isfinite(p0[k]) || !std::isfinite(p1[k])) return false;
    double Q[9], q[4];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            Q[3 * i + j] = ((double)p1[4 * i + 0] * (double)p0[4 * j + 0] + (double)p1[4 * i + 1] * (double)p0[4 * j + 1]) +
                           (double)p1[4 * i + 2] * (double)p0[4 * j + 2];
    if (mode == DBTSDF_DESKEW_SE3) {
        shepperd(Q, q);
    } else {
        const double L = std::sqrt(Q[0] * Q[0] + Q[3] * Q[3]);
        const double hx = L + Q[0], hy = Q[3];
        const double H = std::sqrt(hx * hx + hy * hy);
        q[1] = q[2] = 0.0;
        if (L == 0.0) {
            q[0] = 1.0;
            q[3] = 0.0;
        } else if (H == 0.0) {   // a half turn
            q[0] = 0.0;
            q[3] = 1.0;
        } else {
            q[0] = hx / H;
            q[3] = hy / H;
        }
    }
    for (int k = 0; k < 4; ++k) out[k] = (float)q[k];
    for (int k = 0; k < 3; ++k) out[4 + k] = p1[4 * k + 3] - p0[4 * k + 3];
    return true;
}

}  // namespace dbtsdf

extern "C" dbtsdf_status dbtsdf_deskew_constants(const float pose_start[16], const float pose_end[16], int mode,
                                                 float out[7]) {
    if (!pose_start || !pose_end || !out) {
        dbtsdf::set_error("NULL argument");
        return DBTSDF_ERR_INVALID_ARG;
    }
    if (!dbtsdf::sweep_constants(pose_start, pose_end, mode, out)) {
        dbtsdf::set_error("non-finite pose or unknown deskew mode");
        return DBTSDF_ERR_INVALID_ARG;
    }
    return DBTSDF_OK;
}
