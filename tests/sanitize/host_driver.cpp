// Sanitizer driver for the host set-up of the library (cyl_host.cpp): the
// argument checks of cyl_geom_create on malformed grids, trajectories and
// poses, and a well-formed call, which on a machine without a GPU ends at the
// device query with CYL_EDEVICE.  Exit status 0 when every call returns the
// expected code and leaves an error message.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "cyl.h"

int main() {
    const int n = 4;
    std::vector<double> views(12 * n);
    for (int k = 0; k < n; ++k) {
        const double phi = 6.283185307179586 * k / n, c = std::cos(phi), s = std::sin(phi);
        const double v[12] = {-200 * c, -200 * s, 0, 200 * c, 200 * s, 0, -0.2 * s, 0.2 * c, 0, 0, 0, 0.2};
        for (int i = 0; i < 12; ++i) views[12 * k + i] = v[i];
    }
    cyl_grid g{8, 24, 6, 0.0, 6.0, -3.0, 3.0, 0.0};
    cyl_traj t{n, 16, 20, views.data()};
    cyl_pose p;
    std::memset(&p, 0, sizeof p);
    p.R[0] = p.R[4] = p.R[8] = 1.0;
    cyl_geom *G = nullptr;
    int bad = 0;
    auto expect = [&](int rc, int want, const char *what) {
        if (rc != want || std::strlen(cyl_last_error()) == 0) {
            std::printf("%s: rc %d, want %d\n", what, rc, want);
            ++bad;
        }
    };
    expect(cyl_geom_create(nullptr, &t, &p, 0, &G), CYL_EINVAL, "null grid");
    cyl_grid g2 = g;
    g2.n_r = 0;
    expect(cyl_geom_create(&g2, &t, &p, 0, &G), CYL_EINVAL, "empty grid");
    g2 = g;
    g2.r_max = g2.r_min;
    expect(cyl_geom_create(&g2, &t, &p, 0, &G), CYL_EINVAL, "zero radial extent");
    std::vector<double> v2 = views;
    v2[5] = NAN;
    cyl_traj t2{n, 16, 20, v2.data()};
    expect(cyl_geom_create(&g, &t2, &p, 0, &G), CYL_EINVAL, "non-finite view");
    cyl_pose p2 = p;
    p2.R[8] = -1.0;
    expect(cyl_geom_create(&g, &t, &p2, 0, &G), CYL_EINVAL, "reflection");
    const int rc = cyl_geom_create(&g, &t, &p, 0, &G);
    if (rc == CYL_OK) {
        cyl_geom_destroy(G);
    } else {
        expect(rc, CYL_EDEVICE, "no device");
    }
    if (bad) return 1;
    std::printf("host sanitizer run: ok\n");
    return 0;
}
