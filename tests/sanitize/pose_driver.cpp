// Sanitizer driver for the host half of pose estimation (cyl_pose.cpp), built
// with that source in the same program: point tracking on exact and noisy
// detector points (with masked views), the pose from two axis points and the
// azimuthal phase of a shifted signal.  Exit status 0 when every call succeeds
// and its result is finite and close to the known answer.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <vector>

#include "cyl_internal.h"

namespace cyl {
void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vfprintf(stderr, fmt, ap);
    va_end(ap);
    fputc('\n', stderr);
}
}  // namespace cyl

// Detector point (u, v) of X for view w (12-vector: S, D, U, V) on an H x W detector.
static void project(const double *w, int H, int W, const double X[3], double *uv) {
    const double cu = 0.5 * (W - 1), cv = 0.5 * (H - 1);
    double d[3], o[3];
    for (int i = 0; i < 3; ++i) {
        d[i] = X[i] - w[i];
        o[i] = w[3 + i] - cu * w[6 + i] - cv * w[9 + i] - w[i];
    }
    // solve lam d = o + u U + v V for (lam, u, v) by Cramer's rule
    const double *U = w + 6, *V = w + 9;
    auto det = [](const double *a, const double *b, const double *c) {
        return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) + a[2] * (b[0] * c[1] - b[1] * c[0]);
    };
    const double mU[3] = {-U[0], -U[1], -U[2]}, mV[3] = {-V[0], -V[1], -V[2]};
    const double D = det(d, mU, mV);
    uv[0] = det(d, o, mV) / D;
    uv[1] = det(d, mU, o) / D;
}

int main() {
    const int n = 24, H = 256, W = 320;
    std::vector<double> views(12 * n);
    for (int k = 0; k < n; ++k) {
        const double phi = 6.283185307179586 * k / n, c = std::cos(phi), s = std::sin(phi);
        double *w = &views[12 * k];
        const double v[12] = {-200 * c, -200 * s, 0, 200 * c, 200 * s, 0, -0.2 * s, 0.2 * c, 0, 0, 0, 0.2};
        for (int i = 0; i < 12; ++i) w[i] = v[i];
    }
    cyl_traj traj{n, H, W, views.data()};
    const double X[3] = {5.0, -3.0, 7.0};
    std::vector<double> uv(2 * n);
    std::vector<uint8_t> valid(n, 1);
    for (int k = 0; k < n; ++k) project(&views[12 * k], H, W, X, &uv[2 * k]);
    for (int k = 0; k < n; k += 5) valid[k] = 0;
    double got[3], rms = -1.0;
    if (cyl_track_point(&traj, uv.data(), valid.data(), got, &rms) != CYL_OK) return 1;
    for (int i = 0; i < 3; ++i)
        if (!(std::fabs(got[i] - X[i]) < 1e-6)) return 2;
    for (int k = 0; k < n; ++k) uv[2 * k] += 0.3 * std::sin(1.7 * k);
    if (cyl_track_point(&traj, uv.data(), nullptr, got, &rms) != CYL_OK || !std::isfinite(rms)) return 3;
    // errors are reported, not crashed on
    if (cyl_track_point(nullptr, uv.data(), nullptr, got, &rms) == CYL_OK) return 4;
    const double top[3] = {0.5, -0.2, 20.0}, bottom[3] = {0.3, 0.1, -20.0};
    cyl_pose pose;
    if (cyl_pose_from_axis(top, bottom, 20.0, -20.0, 0.4, &pose) != CYL_OK) return 5;
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(pose.R[i])) return 6;
    std::vector<double> sig(n), ref(n);
    for (int k = 0; k < n; ++k) {
        const double phi = 6.283185307179586 * k / n;
        ref[k] = std::cos(phi) + 0.3 * std::sin(2 * phi);
        sig[k] = std::cos(phi - 0.5) + 0.3 * std::sin(2 * (phi - 0.5));
    }
    double alpha = 0.0;
    // the shift is 0.5 rad in one sense or the other (the convention is pinned
    // by the pose tests; here the call only has to run clean and find it)
    if (cyl_azimuth_phase(n, sig.data(), ref.data(), &alpha) != CYL_OK) return 7;
    if (!(std::fabs(std::fabs(std::remainder(alpha, 6.283185307179586)) - 0.5) < 1e-6)) return 8;
    std::printf("pose sanitizer run: ok\n");
    return 0;
}
