// Pose estimation on the host (Sec. 2.1): point tracking (Eq. 3-4) by
// Levenberg-Marquardt with analytic derivatives, and the object pose (Eq. 1)
// from two tracked points of its symmetry axis.

#include <cmath>
#include <cstdint>
#include <vector>

#include "cyl_internal.h"

namespace cyl {
namespace {

// View i maps a stage-frame point X to detector coordinates (u, v):
// X - S = M (w0, w1, w2) with M = [d0 | U | V], d0 the direction to pixel
// (0, 0), and (u, v) = (w1 / w0, w2 / w0).  Minv = M^-1 (row-major).
struct ViewH {
    double S[3];
    double Minv[9];
};

bool invert3(const double c0[3], const double c1[3], const double c2[3], double inv[9]) {
    // M has columns c0, c1, c2; inv = adj(M) / det(M)
    const double m[9] = {c0[0], c1[0], c2[0], c0[1], c1[1], c2[1], c0[2], c1[2], c2[2]};
    const double a = m[4] * m[8] - m[5] * m[7], b = m[5] * m[6] - m[3] * m[8], c = m[3] * m[7] - m[4] * m[6];
    const double det = m[0] * a + m[1] * b + m[2] * c;
    if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return false;
    const double id = 1.0 / det;
    inv[0] = a * id;
    inv[1] = (m[2] * m[7] - m[1] * m[8]) * id;
    inv[2] = (m[1] * m[5] - m[2] * m[4]) * id;
    inv[3] = b * id;
    inv[4] = (m[0] * m[8] - m[2] * m[6]) * id;
    inv[5] = (m[2] * m[3] - m[0] * m[5]) * id;
    inv[6] = c * id;
    inv[7] = (m[1] * m[6] - m[0] * m[7]) * id;
    inv[8] = (m[0] * m[4] - m[1] * m[3]) * id;
    return true;
}

// Residuals r = V(X) - uv and Jacobian rows d(u, v)/dX of one view; false if
// X is not in front of the source.
bool project(const ViewH &w, const double X[3], double uv[2], double J[6]) {
    const double d[3] = {X[0] - w.S[0], X[1] - w.S[1], X[2] - w.S[2]};
    double q[3];
    for (int r = 0; r < 3; ++r) q[r] = w.Minv[3 * r] * d[0] + w.Minv[3 * r + 1] * d[1] + w.Minv[3 * r + 2] * d[2];
    if (!(q[0] > 0.0)) return false;
    const double i0 = 1.0 / q[0];
    uv[0] = q[1] * i0;
    uv[1] = q[2] * i0;
    for (int c = 0; c < 3; ++c) {
        J[c] = (w.Minv[3 + c] - uv[0] * w.Minv[c]) * i0;
        J[3 + c] = (w.Minv[6 + c] - uv[1] * w.Minv[c]) * i0;
    }
    return true;
}

bool solve3(double A[9], double b[3], double x[3]) {
    double inv[9];
    const double c0[3] = {A[0], A[3], A[6]}, c1[3] = {A[1], A[4], A[7]}, c2[3] = {A[2], A[5], A[8]};
    if (!invert3(c0, c1, c2, inv)) return false;
    for (int r = 0; r < 3; ++r) x[r] = inv[3 * r] * b[0] + inv[3 * r + 1] * b[1] + inv[3 * r + 2] * b[2];
    return true;
}

}  // namespace
}  // namespace cyl

using namespace cyl;

extern "C" int cyl_track_point(const cyl_traj *traj, const double *uv, const uint8_t *valid, double *xyz,
                               double *rms) {
    if (!traj || !traj->views || !uv || !xyz || traj->n_views < 1 || traj->det_rows < 1 || traj->det_cols < 1) {
        set_error("cyl_track_point: NULL argument or empty trajectory");
        return CYL_EINVAL;
    }
    const int n = traj->n_views;
    const double cu = 0.5 * (traj->det_cols - 1), cv = 0.5 * (traj->det_rows - 1);
    std::vector<ViewH> vs;
    std::vector<int> idx;
    for (int k = 0; k < n; ++k) {
        if (valid && !valid[k]) continue;
        if (!std::isfinite(uv[2 * k]) || !std::isfinite(uv[2 * k + 1])) {
            set_error("cyl_track_point: non-finite detector point of view %d", k);
            return CYL_EINVAL;
        }
        const double *q = traj->views + 12 * k;
        ViewH w;
        double d0[3];
        for (int i = 0; i < 3; ++i) {
            w.S[i] = q[i];
            d0[i] = q[3 + i] - cu * q[6 + i] - cv * q[9 + i] - q[i];
        }
        if (!invert3(d0, q + 6, q + 9, w.Minv)) {
            set_error("cyl_track_point: view %d has a degenerate detector", k);
            return CYL_EINVAL;
        }
        vs.push_back(w);
        idx.push_back(k);
    }
    if (vs.size() < 2) {
        set_error("cyl_track_point: need at least two valid views");
        return CYL_EINVAL;
    }
    // start: the point nearest (least squares) to all back-projected rays
    double A[9] = {0}, b[3] = {0}, X[3];
    for (size_t i = 0; i < vs.size(); ++i) {
        const double *q = traj->views + 12 * idx[i];
        const double u = uv[2 * idx[i]], v = uv[2 * idx[i] + 1];
        double r[3];
        for (int c = 0; c < 3; ++c) r[c] = q[3 + c] + (u - cu) * q[6 + c] + (v - cv) * q[9 + c] - q[c];
        const double nr = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        for (int c = 0; c < 3; ++c) r[c] /= nr;
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) {
                const double p = (a == c ? 1.0 : 0.0) - r[a] * r[c];
                A[3 * a + c] += p;
                b[a] += p * q[c];
            }
    }
    if (!solve3(A, b, X)) {
        set_error("cyl_track_point: the rays are parallel");
        return CYL_EINVAL;
    }
    // Levenberg-Marquardt on the reprojection error (Eq. 4)
    auto cost = [&](const double *P, double *g, double *H) -> double {
        double s = 0.0;
        if (g)
            for (int i = 0; i < 3; ++i) g[i] = 0.0;
        if (H)
            for (int i = 0; i < 9; ++i) H[i] = 0.0;
        for (size_t i = 0; i < vs.size(); ++i) {
            double p[2], J[6];
            if (!project(vs[i], P, p, J)) return INFINITY;
            const double e0 = p[0] - uv[2 * idx[i]], e1 = p[1] - uv[2 * idx[i] + 1];
            s += e0 * e0 + e1 * e1;
            if (g)
                for (int c = 0; c < 3; ++c) g[c] += J[c] * e0 + J[3 + c] * e1;
            if (H)
                for (int a = 0; a < 3; ++a)
                    for (int c = 0; c < 3; ++c) H[3 * a + c] += J[a] * J[c] + J[3 + a] * J[3 + c];
        }
        return s;
    };
    double g[3], H[9];
    double f = cost(X, g, H);
    if (!std::isfinite(f)) {
        set_error("cyl_track_point: the start point is behind a source");
        return CYL_EINVAL;
    }
    double mu = 1e-3;
    for (int it = 0; it < 200; ++it) {
        double Hd[9], rhs[3], dx[3];
        for (int i = 0; i < 9; ++i) Hd[i] = H[i];
        for (int i = 0; i < 3; ++i) {
            Hd[4 * i] += mu * (H[4 * i] > 0.0 ? H[4 * i] : 1.0);
            rhs[i] = -g[i];
        }
        if (!solve3(Hd, rhs, dx)) break;
        const double Xn[3] = {X[0] + dx[0], X[1] + dx[1], X[2] + dx[2]};
        double gn[3], Hn[9];
        const double fn = cost(Xn, gn, Hn);
        const double step = std::sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
        if (fn <= f) {
            for (int i = 0; i < 3; ++i) X[i] = Xn[i];
            for (int i = 0; i < 3; ++i) g[i] = gn[i];
            for (int i = 0; i < 9; ++i) H[i] = Hn[i];
            const double df = f - fn;
            f = fn;
            mu = mu / 3.0 > 1e-12 ? mu / 3.0 : 1e-12;
            if (step <= 1e-13 * (1.0 + std::sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2])) || df <= 1e-30) break;
        } else {
            mu *= 4.0;
            if (mu > 1e12) break;
        }
    }
    for (int i = 0; i < 3; ++i) xyz[i] = X[i];
    if (rms) *rms = std::sqrt(f / (2.0 * vs.size()));
    return CYL_OK;
}

extern "C" int cyl_pose_from_axis(const double *top, const double *bottom, double h_top, double h_bottom,
                                  double alpha, cyl_pose *out) {
    if (!top || !bottom || !out) {
        set_error("cyl_pose_from_axis: NULL argument");
        return CYL_EINVAL;
    }
    double d[3] = {top[0] - bottom[0], top[1] - bottom[1], top[2] - bottom[2]};
    const double nd = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (!(nd > 0.0) || !std::isfinite(nd) || !(h_top > h_bottom) || !std::isfinite(alpha)) {
        set_error("cyl_pose_from_axis: need distinct finite points, h_top > h_bottom and a finite angle");
        return CYL_EINVAL;
    }
    for (int i = 0; i < 3; ++i) d[i] /= nd;
    // axis in the stage frame: R^T z = (sin b sin g, sin b cos g, cos b), R = Rz(a) Rx(b) Rz(g)
    const double beta = std::acos(d[2] < -1.0 ? -1.0 : (d[2] > 1.0 ? 1.0 : d[2]));
    const double gamma = std::hypot(d[0], d[1]) > 0.0 ? std::atan2(d[0], d[1]) : 0.0;
    const double ca = std::cos(alpha), sa = std::sin(alpha), cb = std::cos(beta), sb = std::sin(beta);
    const double cg = std::cos(gamma), sg = std::sin(gamma);
    const double Rza[9] = {ca, -sa, 0, sa, ca, 0, 0, 0, 1};
    const double Rxb[9] = {1, 0, 0, 0, cb, -sb, 0, sb, cb};
    const double Rzg[9] = {cg, -sg, 0, sg, cg, 0, 0, 0, 1};
    double T1[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            T1[3 * r + c] = 0.0;
            for (int k = 0; k < 3; ++k) T1[3 * r + c] += Rza[3 * r + k] * Rxb[3 * k + c];
        }
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            out->R[3 * r + c] = 0.0;
            for (int k = 0; k < 3; ++k) out->R[3 * r + c] += T1[3 * r + k] * Rzg[3 * k + c];
        }
    // the object origin is the axis point at height 0
    double centre[3];
    for (int i = 0; i < 3; ++i) centre[i] = 0.5 * (top[i] + bottom[i]) - 0.5 * (h_top + h_bottom) * d[i];
    for (int r = 0; r < 3; ++r)
        out->T[r] = -(out->R[3 * r] * centre[0] + out->R[3 * r + 1] * centre[1] + out->R[3 * r + 2] * centre[2]);
    return CYL_OK;
}

extern "C" int cyl_azimuth_phase(int32_t n, const double *s, const double *s_ref, double *alpha) {
    if (n < 3 || !s || !s_ref || !alpha) {
        set_error("cyl_azimuth_phase: need n >= 3 and non-NULL arrays");
        return CYL_EINVAL;
    }
    for (int k = 0; k < n; ++k)
        if (!std::isfinite(s[k]) || !std::isfinite(s_ref[k])) {
            set_error("cyl_azimuth_phase: non-finite signal value at %d", k);
            return CYL_EINVAL;
        }
    // cross-power X_m = S_m conj(R_m) of the DFTs (S_m = sum_k s_k e^{-2 pi i m k / n})
    const int M = (n - 1) / 2;
    std::vector<double> amp(M), th(M);
    for (int m = 1; m <= M; ++m) {
        double sr = 0, si = 0, rr = 0, ri = 0;
        for (int k = 0; k < n; ++k) {
            const double a = -2.0 * M_PI * (double)((long long)m * k % n) / n;
            const double ca = std::cos(a), sa = std::sin(a);
            sr += s[k] * ca;
            si += s[k] * sa;
            rr += s_ref[k] * ca;
            ri += s_ref[k] * sa;
        }
        const double xr = sr * rr + si * ri, xi = si * rr - sr * ri;
        amp[m - 1] = 2.0 * std::hypot(xr, xi);
        th[m - 1] = std::atan2(xi, xr);
    }
    // C(t) = sum_m amp_m cos(m t - th_m): best of a 0.1-degree grid, then Newton
    double best_t = 0.0, best_c = -INFINITY;
    for (int i = 0; i < 3600; ++i) {
        const double t = 2.0 * M_PI * i / 3600.0;
        double c = 0.0;
        for (int m = 1; m <= M; ++m) c += amp[m - 1] * std::cos(m * t - th[m - 1]);
        if (c > best_c) {
            best_c = c;
            best_t = t;
        }
    }
    double t = best_t;
    for (int it = 0; it < 8; ++it) {
        double d1 = 0.0, d2 = 0.0;
        for (int m = 1; m <= M; ++m) {
            d1 -= amp[m - 1] * m * std::sin(m * t - th[m - 1]);
            d2 -= amp[m - 1] * m * m * std::cos(m * t - th[m - 1]);
        }
        if (!(d2 < 0.0)) break;
        t -= d1 / d2;
    }
    t = std::fmod(t, 2.0 * M_PI);
    if (t < 0.0) t += 2.0 * M_PI;
    *alpha = t;
    return CYL_OK;
}

extern "C" int cyl_gamma_from_phase(double phi_p, double phi_g, double a1, double a2, double *gamma) {
    if (!gamma || !std::isfinite(phi_p) || !std::isfinite(phi_g) || !std::isfinite(a1) || !std::isfinite(a2) ||
        std::cos(a2) == 0.0) {
        set_error("cyl_gamma_from_phase: NULL output, non-finite angle or cos(a2) = 0");
        return CYL_EINVAL;
    }
    // Eq. 5, the arctangent of tan(a1) / cos(a2) as a continuous atan2
    const double corr = std::atan2(std::sin(a1), std::cos(a1) * std::cos(a2));
    double g = phi_p - phi_g - corr;
    g -= 2.0 * M_PI * std::floor(g / (2.0 * M_PI));
    *gamma = g >= 2.0 * M_PI ? 0.0 : g;
    return CYL_OK;
}

extern "C" int cyl_axis_points(int32_t n_views, const int32_t *corners, double *top, double *bottom,
                               uint8_t *valid) {
    if (n_views < 1 || !corners || !top || !bottom || !valid) {
        set_error("cyl_axis_points: n_views < 1 or NULL array");
        return CYL_EINVAL;
    }
    for (int k = 0; k < n_views; ++k) {
        const int32_t *c = corners + 9 * (size_t)k;
        const bool ok = c[8] > 0;
        valid[k] = ok ? 1 : 0;
        for (int i = 0; i < 2; ++i) {
            top[2 * k + i] = ok ? 0.5 * ((double)c[i] + (double)c[2 + i]) : -1.0;
            bottom[2 * k + i] = ok ? 0.5 * ((double)c[4 + i] + (double)c[6 + i]) : -1.0;
        }
    }
    return CYL_OK;
}
