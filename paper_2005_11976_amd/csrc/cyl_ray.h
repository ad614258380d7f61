// Per-ray geometry and the walk of the exact cylindrical traversal (Sec. 2.2,
// Eq. 6; cells of Sec. 2, Eq. 2), shared by the forward projection, the
// back-projection on super-blocks and the matrix recording.
//
// A ray is parametrised by its arc length sigma (mm) from a reference point
// X0 on it: the ray point nearest a target point (the grid centre for a whole
// ray, the super-block centre for the back-projection), computed exactly on
// the FP64 ray.  All FP32 crossing parameters are then differences measured
// from a point inside the region walked, so their rounding scales with the
// size of that region, not with the distance to the axis, and rays nearly
// parallel to the axis (whose closest approach to it lies far away) stay
// well conditioned.  The xy coordinates are taken in a frame rotated about
// the axis (by the super-block's middle edge), so sector-edge tests near the
// super-block are small differences as well.
//
// With X(sigma) = X0 + sigma e (|e| = 1), beta = X0_xy . e_xy and
// kappa^2 = |e_xy|^2:
//   r-shells      |X_xy(sigma)|^2 = r_i^2, i.e. kappa^2 sigma^2 + 2 beta sigma = r_i^2 - r0^2 = W_i.
//                 With G_i = kappa sqrt(r_i^2 - b^2) + |beta| (b the xy distance of the
//                 line from the axis, r0 = |X0_xy|) the two roots are W_i / G_i and
//                 -G_i / kappa^2 (beta >= 0; mirrored for beta < 0): the first form is
//                 the small difference computed without cancellation, the second a sum.
//   sector edges  n_b . X(sigma) = 0                  ->  sigma = -(n_b . X0) / (n_b . e)
//   axial planes  z(sigma) = h_m                      ->  sigma = (h_m - z0) / e_z
// r_i - b and r_i - r0 are formed from two-word FP32 radii rebased at the
// shell nearest b (resp. r0), so both keep their precision at grazing
// incidence; z0 is a two-word value as well.
#pragma once

#include "cyl_internal.h"
#include "cyl_isa.h"

namespace cyl {

#define CYL_INF __builtin_huge_valf()

enum : int { RAY_HIT = 1, RAY_AXIAL = 2, RAY_THRU = 4 };

// Grid tables as seen by a walk.  r, h: n_r + 1 shell radii and n_h + 1 axial
// planes as (hi, lo) words.  cs: sector edges cs_lo .. cs_lo + cs_n as
// (cos, sin) of their angle in the walk frame.
struct Tabs {
    const float2 *r;
    const float2 *h;
    const float2 *cs;
    int cs_lo, cs_n;
};

// Sector edge b of an edge table that may hold only part of the edges (a
// super-block's wedge and one edge either side).  A walk reads the edge ahead
// before it checks its box, so on the step that leaves the box b may lie
// outside the table; that read is clamped and its value is never used.
template <bool CLAMP>
__device__ __forceinline__ float2 edge_at(const Tabs &T, int b) {
    if (!CLAMP) return T.cs[b];
    return T.cs[min((unsigned)(b - T.cs_lo), (unsigned)T.cs_n)];
}

// Walk frame: rotation by angle w about the axis (X_frame = Rz(-w) X) and the
// target point whose nearest ray point is the reference point.
struct Frame {
    double cw, sw;     // cos w, sin w
    float gx, gy, gz;  // target point, object frame
    float wsec;        // (w - theta0) / dtheta, for the sector of a point
};

struct Ray {
    float px, py, pz, pzlo;  // reference point X0: frame xy, z as hi + lo
    float ex, ey, ez;        // unit direction (frame xy)
    float beta;              // X0_xy . e_xy
    float k2, ik2;           // kappa^2 = |e_xy|^2 and 1 / kappa^2
    float b, blo;            // xy distance of the line from the axis, hi + lo
    float r0, r0lo;          // |X0_xy|, hi + lo
    float sc;                // parameter of the xy closest approach, -beta / kappa^2
    float cx, cy;            // the xy closest approach (frame xy; X0 for axial rays)
    float inv_ez;            // 1 / e_z (+inf for level rays)
    float s_in, s_out;       // parameter interval to walk
    float tref, len;         // X0 = a + tref d (tref an FP32 value); len = |d|
    int flags;
    int it_in, it_out;       // rays through the axis: sectors before / after it
    int pix;                 // u | v << 16 (the rare FP64 paths rebuild the ray from it)
    int sg;                  // sense of the theta sweep along the ray: +1, -1 or 0
};

// Sector containing the global direction (x, y).
__device__ __forceinline__ int sector_of(const GeomDev &g, float x, float y) {
    if (g.n_theta == 1) return 0;
    const float two_pi = 6.28318530717958647692f;
    float th = atan2f(y, x) - g.theta0;
    th -= two_pi * floorf(th * (1.0f / two_pi));
    int it = (int)floorf(th * g.inv_dtheta);
    it = it < 0 ? 0 : it;
    return it >= g.n_theta ? g.n_theta - 1 : it;
}

// Set-up of the ray of pixel (u, v) in frame F.  FP64 for the direction, the
// reference point, its distance from the axis and the distance b of the ray's
// line from the axis (from the FP64 cross product a x d, the same for every
// point of the line).  The interval [s_in, s_out] is the source -> pixel
// segment; callers clip it.
__device__ __forceinline__ void ray_setup(const GeomDev &g, const ViewDev &V, int u, int v, const Frame &F, Ray &r,
                                          double &dxo, double &dyo, double &dzo) {
    const double fu = (double)u, fv = (double)v;
    const double dx = fma(fv, V.V[0], fma(fu, V.U[0], V.d0[0]));
    const double dy = fma(fv, V.V[1], fma(fu, V.U[1], V.d0[1]));
    const double dz = fma(fv, V.V[2], fma(fu, V.U[2], V.d0[2]));
    dxo = dx;
    dyo = dy;
    dzo = dz;
    const double A = fma(dx, dx, dy * dy);
    const double dd = fma(dz, dz, A);
    const float fdx = (float)dx, fdy = (float)dy, fdz = (float)dz;
    const float len = fsqrt((float)dd);
    const float il = frcp(len);
    // reference parameter: the ray point nearest the target (any FP32 value
    // will do; X0 is then computed for exactly this parameter)
    const float tref =
        ((F.gx - V.af[0]) * fdx + (F.gy - V.af[1]) * fdy + (F.gz - V.af[2]) * fdz) * (il * il);
    const double tr = (double)tref;
    const double X = fma(tr, dx, V.a[0]), Y = fma(tr, dy, V.a[1]), Z = fma(tr, dz, V.a[2]);
    const double Xr = fma(F.cw, X, F.sw * Y), Yr = fma(F.cw, Y, -(F.sw * X));
    const double dxr = fma(F.cw, dx, F.sw * dy), dyr = fma(F.cw, dy, -(F.sw * dx));
    r.px = (float)Xr;
    r.py = (float)Yr;
    r.pz = (float)Z;
    r.pzlo = (float)(Z - (double)r.pz);
    r.ex = (float)dxr * il;
    r.ey = (float)dyr * il;
    r.ez = fdz * il;
    r.len = len;
    r.tref = tref;
    r.pix = u | (v << 16);
    r.flags = 0;
    r.it_in = r.it_out = 0;
    const double r02 = fma(Xr, Xr, Yr * Yr);
    const float r0 = fsqrt((float)r02);
    r.r0 = r0;
    r.r0lo = r0 > 0.0f ? (float)fma(-(double)r0, (double)r0, r02) * (0.5f * frcp(r0)) : 0.0f;
    r.beta = (float)fma(Xr, dxr, Yr * dyr) * il;
    r.inv_ez = (fdz != 0.0f) ? len / fdz : CYL_INF;
    const double cross = fma(V.a[0], dy, -(V.a[1] * dx));
    r.sg = cross > 0.0 ? 1 : (cross < 0.0 ? -1 : 0);
    const float k2 = (float)A * (il * il);
    if (k2 > 0.0f) {
        const double b2 = cross * cross / A;
        const float bf = fsqrt((float)b2);
        r.b = bf;
        r.blo = bf > 0.0f ? (float)fma(-(double)bf, (double)bf, b2) * (0.5f * frcp(bf)) : 0.0f;
        r.k2 = k2;
        r.ik2 = frcp(k2);
        r.sc = -r.beta * r.ik2;
        if (b2 <= 1e-24 * fma(V.a[0], V.a[0], fma(V.a[1], V.a[1], V.a[2] * V.a[2])) && g.n_theta > 1) {
            // the line passes through the axis, to within 1e-12 of the source's
            // distance from the origin: below that the side on which it passes
            // is FP64 rounding (and the sectors it sweeps there have no length),
            // so the sector simply jumps at the axis
            r.sg = 0;
            r.flags |= RAY_THRU;
            r.it_in = sector_of(g, -fdx, -fdy);
            r.it_out = sector_of(g, fdx, fdy);
        }
        // the closest approach itself, as b times the unit normal of the xy
        // direction on the side the sweep sense gives (exact in direction even
        // where b is below the rounding of X0): positions near the axis are
        // then small offsets from a small point
        const float bk = (float)r.sg * bf * frsq(k2);
        r.cx = bk * r.ey;
        r.cy = -bk * r.ex;
    } else {
        // parallel to the axis (to FP32 resolution): a fixed ring and sector
        r.flags |= RAY_AXIAL;
        r.b = CYL_INF;
        r.blo = 0.0f;
        r.k2 = 0.0f;
        r.ik2 = CYL_INF;
        r.sc = 0.0f;
        r.cx = r.px;
        r.cy = r.py;
    }
    r.s_in = -tref * len;
    r.s_out = (1.0f - tref) * len;
}

// Both crossings lo <= hi of the ray with the shell of radius rt (hi, lo
// words); false if its line passes inside the shell's radius or runs along
// the axis (callers test axial rays against r0).
__device__ __forceinline__ bool shell_roots(float2 rt, const Ray &r, float &lo, float &hi) {
    const float d = (rt.x - r.b) + (rt.y - r.blo);  // r_t - b
    if (!(d > 0.0f)) return false;
    const float D = r.k2 * (d * (d + 2.0f * r.b));
    const float G = fmaxf(fsqrt(D) + fabsf(r.beta), 1e-30f);
    const float d2 = (rt.x - r.r0) + (rt.y - r.r0lo);  // r_t - r0
    const float W = d2 * (d2 + 2.0f * r.r0);
    const float nearr = W * frcp(G), farr = G * r.ik2;
    if (r.beta >= 0.0f) {
        hi = nearr;
        lo = -farr;
    } else {
        hi = farr;
        lo = -nearr;
    }
    return true;
}

// Parameter where the ray meets the axial plane ht (hi, lo words).
__device__ __forceinline__ float plane_s(float2 ht, const Ray &r) {
    return ((ht.x - r.pz) + (ht.y - r.pzlo)) * r.inv_ez;
}

// Crossing of sector edge b's full line through the axis, solved in FP64 on
// the unrounded ray (for rays nearly parallel to the line, where the FP32
// quotient is ill-conditioned); c = (cos, sin) of the edge in the object
// frame.  on_edge: the meeting lies on the edge's half-line.
__device__ __forceinline__ void edge_cross_fp64(double2 c, const ViewDev &V, const Ray &r, float &s, bool &on_edge) {
    // the per-ray inputs pass through an empty asm statement so that the
    // compiler does not hoist their FP64 forms out of the walk loop (where
    // they would hold registers on every step for a path that rarely runs)
    int pix = r.pix;
    float tref = r.tref, len = r.len;
    asm volatile("" : "+v"(pix), "+v"(tref), "+v"(len));
    const double fu = (double)(pix & 0xffff), fv = (double)(pix >> 16);
    const double dx = fma(fv, V.V[0], fma(fu, V.U[0], V.d0[0]));
    const double dy = fma(fv, V.V[1], fma(fu, V.U[1], V.d0[1]));
    const double nd = c.x * dy - c.y * dx;
    const double na = c.x * V.a[1] - c.y * V.a[0];
    if (nd == 0.0) {
        on_edge = false;
        s = CYL_INF;
        return;
    }
    const double t = -na / nd;
    const double px = fma(t, dx, V.a[0]), py = fma(t, dy, V.a[1]);
    on_edge = (c.x * px + c.y * py) > 0.0;
    s = (float)((t - (double)tref) * (double)len);
}

// Below this |n.e| the FP32 edge quotient is re-solved in FP64 (only rays
// nearly parallel to an edge line, that is rays passing close to the axis,
// or running nearly along it, whose crossing lies far outside the walk and
// is skipped without the re-solve).
constexpr float kEdgeTau = 0.03125f;

// Cell at parameter s (indices clamped into the grid; ir = -1 inside the hole)
// for a walk that proceeds from s in the direction of the ray.  The xy
// position is taken from whichever of X0 and the closest approach lies
// nearer, so that points near the axis keep their precision.  A point closer
// to the axis than the rounding of these coordinates (a few ulp of |s|, and of
// |X0| when measured from it) has no reliable sector of its own: the walk then starts in the sector
// the ray heads into, which it reaches within that distance anyway.
__device__ __forceinline__ void cell_at(const GeomDev &g, const Ray &r, const Frame &F, float s, int &ih, int &it,
                                        int &ir) {
    const float ds = s - r.sc;
    const bool nearc = fabsf(ds) < fabsf(s);
    const float x = nearc ? fmaf(ds, r.ex, r.cx) : fmaf(s, r.ex, r.px);
    const float y = nearc ? fmaf(ds, r.ey, r.cy) : fmaf(s, r.ey, r.py);
    const float z = fmaf(s, r.ez, r.pz);
    const float rr = sqrtf(fmaf(x, x, y * y));
    const int h = (int)floorf((z - g.h_min) * g.inv_dh);
    ih = h < 0 ? 0 : (h >= g.n_h ? g.n_h - 1 : h);
    const int ri = (int)floorf((rr - g.r_min) * g.inv_dr);
    ir = ri < -1 ? -1 : (ri >= g.n_r ? g.n_r - 1 : ri);
    if (g.n_theta == 1) {
        it = 0;
    } else if (r.flags & RAY_THRU) {
        it = (s < r.sc) ? r.it_in : r.it_out;
    } else {
        const float nt = (float)g.n_theta;
        const float eps = 4e-6f * (nearc ? 2.0f * fabsf(s) : fabsf(s) + r.r0);
        const bool at_axis = fmaf(x, x, y * y) <= eps * eps;
        float th = fmaf(at_axis ? atan2f(r.ey, r.ex) : atan2f(y, x), g.inv_dtheta, F.wsec);
        th -= nt * floorf(th * (1.0f / nt));
        const int t = (int)floorf(th);
        it = t < 0 ? 0 : (t >= g.n_theta ? g.n_theta - 1 : t);
    }
}

__device__ __forceinline__ int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Per-ray constants of the walk.
//  planes: sigma_m = k zA + (k zAlo + zB), k = m - mc, i.e. (h_m - z0) / e_z
//    rebased at the plane nearest z0 (zB = +inf for level rays);
//  shells: r_i - b = k dr + (k dr_lo + drc), k = i - ic, and r_i - r0 the same
//    with k + dk and drc2 (rebased at the shells nearest b and r0); ib is the
//    innermost shell the ray reaches (r_ib > b), so the next shell before the
//    closest approach (sigma < sc) is r_ir if ir >= ib, else the ray turns and
//    leaves through r_{ir+1};
//  sector edges: with (px, py, ex, ey) multiplied by the sweep sense the
//    edge's half-line is met ahead iff n.e > 0, at sigma = -(n.X0)/(n.e).
struct Walk {
    float zA, zAlo, zB;
    int kz, dir_h;
    float drc, drc2, twob, twor, abeta, ik;
    int ic, dk, ib;
    bool pos;
    float tpx, tpy, tex, tey;
    int dir_t, up_t, tstep, twrap;
};

__device__ __forceinline__ Walk walk_setup(const GeomDev &g, const Tabs &T, const Ray &r, int it) {
    Walk w;
    w.dir_h = r.ez > 0.0f ? 1 : (r.ez < 0.0f ? -1 : 0);
    const int mc = clampi((int)floorf((r.pz - g.h_min) * g.inv_dh + 0.5f), 0, g.n_h);
    if (w.dir_h != 0) {
        const float2 ht = T.h[mc];
        w.zA = g.dh * r.inv_ez;
        w.zAlo = g.dh_lo * r.inv_ez;
        w.zB = ((ht.x - r.pz) + (ht.y - r.pzlo)) * r.inv_ez;
    } else {
        w.zA = w.zAlo = 0.0f;
        w.zB = CYL_INF;
    }
    w.kz = (w.dir_h > 0 ? 1 : 0) - mc;
    const bool axial = (r.flags & RAY_AXIAL) != 0;
    w.ic = axial ? 0 : clampi((int)floorf((r.b - g.r_min) * g.inv_dr + 0.5f), 0, g.n_r);
    const int jc = clampi((int)floorf((r.r0 - g.r_min) * g.inv_dr + 0.5f), 0, g.n_r);
    const float2 rb = T.r[w.ic], r0t = T.r[jc];
    w.drc = (rb.x - r.b) + (rb.y - r.blo);
    w.drc2 = (r0t.x - r.r0) + (r0t.y - r.r0lo);
    w.dk = w.ic - jc;
    w.ib = axial ? 0x7fffffff : w.ic + (w.drc > 0.0f ? 0 : 1);
    w.twob = 2.0f * r.b;
    w.twor = 2.0f * r.r0;
    w.abeta = fabsf(r.beta);
    w.pos = r.beta >= 0.0f;
    w.ik = axial ? 0.0f : frsq(r.k2);
    const int nt = g.n_theta;
    w.dir_t = (nt == 1 || (r.flags & (RAY_AXIAL | RAY_THRU))) ? 0 : r.sg;
    w.up_t = w.dir_t > 0 ? 1 : 0;
    // a ray through the axis jumps from the start sector to the one ahead
    w.tstep = (r.flags & RAY_THRU) ? r.it_out - it : w.dir_t;
    w.twrap = w.dir_t * nt;
    const float sg = w.dir_t < 0 ? -1.0f : 1.0f;
    w.tpx = sg * r.px;
    w.tpy = sg * r.py;
    w.tex = sg * r.ex;
    w.tey = sg * r.ey;
    return w;
}

// Crossing of shell i on the inward (before the closest approach) or
// outward side.  PRECISE: the root as the small difference W / G or the sum
// G / kappa^2 (rounding scaled by |sigma|, for walks whose reference point is
// far from the closest approach); otherwise sc -+ |s_i|, with s_i the arc
// length from the closest approach (rounding scaled by |s_i|: for walks whose
// reference point lies near the closest approach, and whose rays are not
// close to the axis direction).
template <bool PRECISE>
__device__ __forceinline__ float shell_root(const GeomDev &g, const Walk &w, const Ray &r, int i, bool inward) {
    const float k = (float)(i - w.ic);
    const float d = fmaxf(fmaf(k, g.dr, fmaf(k, g.dr_lo, w.drc)), 0.0f);  // r_i - b
    if (!PRECISE) {
        const float x = fsqrt(d * (d + w.twob)) * w.ik;
        return (inward ? -x : x) + r.sc;
    }
    const float G = fmaxf(fsqrt(r.k2 * (d * (d + w.twob))) + w.abeta, 1e-30f);
    const float k2 = k + (float)w.dk;
    const float d2 = fmaf(k2, g.dr, fmaf(k2, g.dr_lo, w.drc2));  // r_i - r0
    const float W = d2 * (d2 + w.twor);
    const float v = (inward == w.pos) ? G * r.ik2 : W * frcp(G);
    return inward ? -v : v;
}

// Next shell crossing after s from ring ir (not clamped to s).
template <bool PRECISE>
__device__ __forceinline__ float shell_next(const GeomDev &g, const Walk &w, const Ray &r, int ir, float s,
                                            int &r_dir) {
    const bool inward = (s < r.sc) && (ir >= w.ib);
    r_dir = inward ? -1 : 1;
    return shell_root<PRECISE>(g, w, r, inward ? ir : ir + 1, inward);
}

// Crossing of plane m = ih + (dir_h > 0).
__device__ __forceinline__ float plane_next(const Walk &w, int ih) {
    const float k = (float)(ih + w.kz);
    return fmaf(k, w.zA, fmaf(k, w.zAlo, w.zB));
}

// Crossing of sector edge be (cs = its cos, sin in the walk frame) ahead of
// s, or +inf.  An edge-half-line meeting behind s means the start cell was
// one sector short (rounding at entry): cross it at once.  Near-parallel
// cases (|n.e| below kEdgeTau) whose crossing may fall before s_end are
// re-solved in FP64 when REFINE and `refine` are set (walks that cannot meet
// such a case, see needs_refine, are compiled without the test).
template <bool REFINE>
__device__ __forceinline__ float edge_next(const ViewDev &V, const GeomDev &g, const Walk &w, const Ray &r,
                                           float2 cs, int be, float s, float s_end, bool refine) {
    const float nc = cs.x * w.tpy - cs.y * w.tpx;
    const float ne = cs.x * w.tey - cs.y * w.tex;
    float x = -nc * frcp(ne);
    bool ahead = ne > 0.0f;
    if (REFINE && refine && w.dir_t != 0 && fabsf(ne) < kEdgeTau) {
        if (fabsf(nc) <= fabsf(ne) * (s_end - s + 1.0f)) edge_cross_fp64(g.cs64[be], V, r, x, ahead);
    }
    return (w.dir_t != 0 && ahead) ? vmax(x, s) : CYL_INF;
}

// Whether a walk of the ray over [s0, s1] may meet an edge crossing that
// edge_next re-solves in FP64.  The crossing of edge b at distance rho_b from
// the axis has |n_b . e| = kappa b / rho_b, and a crossing that the test
// considers (|sigma| <= s1 - s0 + 1) lies within r0 + kappa (s1 - s0 + 1) of
// the axis; so |n_b . e| < kEdgeTau needs kappa b below kEdgeTau times that
// radius (taken with a margin of 1 %).
__device__ __forceinline__ bool needs_refine(const Ray &r, float s0, float s1) {
    if ((r.flags & (RAY_AXIAL | RAY_THRU)) || !(r.flags & RAY_HIT)) return false;
    const float kappa = fsqrt(r.k2);
    const float rho = r.r0 + kappa * (s1 - s0 + 1.0f) + 1.0f;
    return kappa * r.b < 1.01f * kEdgeTau * rho;
}

// Walk the ray from s to s_end starting in cell (ih, it, ir) and call
// visit(ih, it, ir, length) for every piece (length 0 allowed; ir = -1 is the
// hole).  Each step takes the nearest of the three next-crossing candidates
// and recomputes the candidate of that kind with selects (no divergent branch
// but the rare FP64 edge case); shell and plane crossings are arithmetic, so
// the only table read per step is the next sector edge, issued before the
// visitor so that its latency overlaps the visitor's work.  Plane and shell
// candidates after their own event are monotone in the index, so only the
// first ones and the edge candidates are clamped to s.  The walk ends at
// s_end, which its caller has clipped to the region walked with the same
// crossing formulas, so the indices stay in that region up to a step of
// rounding at its faces (visitors clamp what they index).  WRAP: the sector
// index wraps around the circle (walks whose region is the whole circle);
// CLAMP: the edge table holds only the region's edges.
template <bool WRAP, bool CLAMP, bool PRECISE, bool REFINE, class Visit>
__device__ __forceinline__ void traverse(const GeomDev &g, const Tabs &T, const ViewDev &V, const Ray &r, float s,
                                         const float s_end, int ih, int it, int ir, Visit &visit) {
    const int nt = g.n_theta;
    const Walk w = walk_setup(g, T, r, it);
    const bool axial = (r.flags & RAY_AXIAL) != 0;
    // Start cell consistent with the walk's own crossings: the start point's
    // FP32 coordinates may put it one cell past a face that the walk's
    // crossing formulas place just ahead of s (a shallow ray near an axial
    // plane, a grazing one near a shell, one nearly along an edge), and the
    // walk only moves forward; step such an index back.  An index one short
    // needs nothing: that face's crossing lies behind s and is taken at once.
    if (w.dir_h != 0) {
        const float kp = (float)(ih + w.kz - w.dir_h);  // the plane behind the start slab
        if (fmaf(kp, w.zA, fmaf(kp, w.zAlo, w.zB)) > s) ih -= w.dir_h;
    }
    if (!axial) {
        const bool inward = (s < r.sc) && (ir >= w.ib);
        const int ibh = inward ? ir + 1 : ir;  // the shell behind the start ring
        if (ibh >= w.ib && ibh >= 0 && shell_root<PRECISE>(g, w, r, ibh, inward) > s) ir += inward ? 1 : -1;
    }
    if (w.dir_t != 0) {
        const int bb = it + 1 - w.up_t;  // the edge behind the start sector in the sweep
        const float2 cs = edge_at<CLAMP>(T, bb);
        const float nc = cs.x * w.tpy - cs.y * w.tpx, ne = cs.x * w.tey - cs.y * w.tex;
        if (ne > 0.0f && -nc > s * ne) {
            it -= w.dir_t;
            if (WRAP) it += ((unsigned)it >= (unsigned)nt) ? w.twrap : 0;
        }
    }
    int r_dir = 1;
    float s_z = fmaxf(plane_next(w, ih), s);
    float s_r = axial ? CYL_INF : fmaxf(shell_next<PRECISE>(g, w, r, ir, s, r_dir), s);
    float s_t;
    if (r.flags & RAY_THRU)
        s_t = s < r.sc ? r.sc : CYL_INF;
    else
        s_t = edge_next<true>(V, g, w, r, edge_at<CLAMP>(T, it + w.up_t), it + w.up_t, s, s_end, true);
    // the edge ahead of sector it is entry it + up_t of the table (it + up_t -
    // cs_lo of a partial table, clamped into it)
    const int cofs = w.up_t - (CLAMP ? T.cs_lo : 0);
    const float2 *__restrict__ csb = T.cs + cofs;
    // a guard on the step count (the walk ends at s_end on its own)
    const int max_steps = 2 * g.n_r + nt + g.n_h + 8;
    for (int n = 0; n < max_steps; ++n) {
        const float sn = vmin(vmin3(s_z, s_r, s_t), s_end);
        const bool ev_z = (sn == s_z);
        const bool ev_r = !ev_z && (sn == s_r);
        const bool ev_t = !ev_z && !ev_r;
        int itn = it + (ev_t ? w.tstep : 0);
        if (WRAP) itn -= ((unsigned)itn >= (unsigned)nt) ? w.twrap : 0;
        const int be = itn + w.up_t;
        const float2 cse = CLAMP ? T.cs[min((unsigned)(itn + cofs), (unsigned)T.cs_n)] : csb[itn];
        visit(ih, it, ir, sn - s);
        s = sn;
        ih += ev_z ? w.dir_h : 0;
        ir += ev_r ? r_dir : 0;
        it = itn;
        if (!(sn < s_end)) break;
        int rd;
        const float nz = plane_next(w, ih);
        const float nrr = shell_next<PRECISE>(g, w, r, ir, s, rd);
        const float ntt = edge_next<REFINE>(V, g, w, r, cse, be, s, s_end, ev_t);
        s_z = ev_z ? nz : s_z;
        s_r = ev_r ? nrr : s_r;
        r_dir = ev_r ? rd : r_dir;
        s_t = ev_t ? ntt : s_t;
    }
}

// Interval of the ray inside the grid support r_min..r_max x h_min..h_max
// (the hole r < r_min included); false if it misses.
__device__ __forceinline__ bool clip_support(const GeomDev &g, const Tabs &T, Ray &r) {
    float s0 = r.s_in, s1 = r.s_out;
    const float2 rt = T.r[g.n_r];
    if (r.flags & RAY_AXIAL) {
        if (!((rt.x - r.r0) + (rt.y - r.r0lo) > 0.0f)) return false;
    } else {
        float lo, hi;
        if (!shell_roots(rt, r, lo, hi)) return false;
        s0 = fmaxf(s0, lo);
        s1 = fminf(s1, hi);
    }
    if (r.ez != 0.0f) {
        const float t1 = plane_s(T.h[0], r), t2 = plane_s(T.h[g.n_h], r);
        s0 = fmaxf(s0, fminf(t1, t2));
        s1 = fminf(s1, fmaxf(t1, t2));
    } else if (!(r.pz >= T.h[0].x && r.pz < T.h[g.n_h].x)) {
        return false;
    }
    r.s_in = s0;
    r.s_out = s1;
    return s1 > s0;
}

// Closed-form row sum L_j in FP64 (Eq. 7's denominator): the length of the
// source -> pixel segment inside the support minus the part inside the hole,
// parametrised from the segment's point nearest the grid centre.
__device__ __forceinline__ float row_sum_fp64(const GeomDev &g, const ViewDev &V, double dx, double dy, double dz) {
    const double A = fma(dx, dx, dy * dy);
    const double dd = fma(dz, dz, A);
    const double len = sqrt(dd);
    const double zmid = 0.5 * (g.h_min_d + g.h_max_d);
    const double t0 = -(V.a[0] * dx + V.a[1] * dy + (V.a[2] - zmid) * dz) / dd;
    const double X = fma(t0, dx, V.a[0]), Y = fma(t0, dy, V.a[1]), Z = fma(t0, dz, V.a[2]);
    // sigma in mm from X0 = a + t0 d along e = d / len
    double lo = -t0 * len, hi = (1.0 - t0) * len;
    const double cross = V.a[0] * dy - V.a[1] * dx;
    const double b2 = A > 0.0 ? cross * cross / A : fma(X, X, Y * Y);
    const double beta = (X * dx + Y * dy) / len, k2 = A / dd, r02 = fma(X, X, Y * Y);
    // interval where |X_xy(sigma)| < R: kappa^2 sigma^2 + 2 beta sigma < R^2 - r0^2
    auto disc = [&](double R, double &a, double &c) -> bool {
        if (!(b2 < R * R)) return false;
        if (!(A > 0.0)) {
            a = -1e300;
            c = 1e300;
            return true;
        }
        const double Dq = k2 * (R * R - b2);
        const double q = beta + (beta >= 0.0 ? sqrt(Dq) : -sqrt(Dq));
        const double W = R * R - r02;
        const double x1 = -q / k2, x2 = W / q;
        a = fmin(x1, x2);
        c = fmax(x1, x2);
        return true;
    };
    double a, c;
    if (!disc(g.r_max_d, a, c)) return 0.0f;
    lo = fmax(lo, a);
    hi = fmin(hi, c);
    if (dz != 0.0) {
        const double iz = len / dz;
        const double t1 = (g.h_min_d - Z) * iz, t2 = (g.h_max_d - Z) * iz;
        lo = fmax(lo, fmin(t1, t2));
        hi = fmin(hi, fmax(t1, t2));
    } else if (!(Z >= g.h_min_d && Z < g.h_max_d)) {
        return 0.0f;
    }
    if (!(hi > lo)) return 0.0f;
    double L = hi - lo;
    if (g.r_min_d > 0.0 && disc(g.r_min_d, a, c)) L -= fmax(0.0, fmin(hi, c) - fmax(lo, a));
    return (float)fmax(L, 0.0);
}

}  // namespace cyl
