// Back-projection blocks: the super-block decomposition of the grid, the
// walk frame of a super-block, and the walk of one ray through a super-block
// (clipped to its hull, split at its inner hole, boxed to its cells), shared
// by the back-projection kernels.
#pragma once

#include "cyl_ray.h"

namespace cyl {

struct Block {
    int hA, hB, tA, tB, rA, rB;
};

// Super-block of the back-projection: sbb = 4 or 8 blocks of the
// decomposition merged by factors ft (theta) x fr (r) x fh (h) = sbb.  Merging
// in theta and r cuts the pixels that must be set up more than merging in h
// (rays are nearly level): on 256x720x128, 4.3 M (ray, block) pairs per view
// for 2 x 2 x 1 against 6.0 M for 4 blocks stacked in h and 7.1 M for single
// blocks; h takes the rest of the factor.  The merged wedge stays within pi
// (the hull clip takes it as the intersection of two half-planes) or covers
// the whole circle.  sbb blocks' slots always hold the merged block's, with
// words to spare.
// A super-block merges sbb = 4 or 8 blocks; its workgroup has one wave per
// block (64 sbb lanes).

struct SbShape {
    int fh, ft, fr, nsh, nst, nsr;
};

__host__ __device__ __forceinline__ SbShape sb_shape(const GeomDev &g, int sbb) {
    SbShape s;
    s.ft = (g.nbt >= 2 && 2 * g.bt <= g.n_theta / 2) ? 2 : 1;
    s.fr = g.nbr >= 2 ? 2 : 1;
    s.fh = sbb / (s.ft * s.fr);
    s.nsh = (g.nbh + s.fh - 1) / s.fh;
    s.nst = (g.nbt + s.ft - 1) / s.ft;
    s.nsr = (g.nbr + s.fr - 1) / s.fr;
    return s;
}

// Sector-edge entries a super-block stages in LDS: its wedge's edges and one
// either side, at most ft bt + 3.
__host__ __device__ __forceinline__ int sb_edge_words(const GeomDev &g, const SbShape &sb) {
    return sb.ft * g.bt + 3;
}

// Walk frame of a super-block: rotated to its middle sector edge m (so the
// block's edges are small angles in it), with the reference point of each ray
// the point nearest the block's centre, or, for blocks around the axis
// (r_A = 0), nearest the axis at the block's mid-height: a ray that passes the
// axis inside such a block then has its reference point next to the axis, and
// the sector it enters there is decided by small, precise coordinates.
__device__ __forceinline__ Frame block_frame(const GeomDev &g, const Block &B, int &m) {
    m = (B.tA + B.tB) >> 1;
    const double2 cm = g.cs64[m];
    Frame F;
    F.cw = cm.x;
    F.sw = cm.y;
    const float rc = B.rA == 0 ? 0.0f : 0.5f * (g.r_tab[B.rA].x + g.r_tab[B.rB].x);
    F.gx = rc * (float)cm.x;
    F.gy = rc * (float)cm.y;
    F.gz = 0.5f * (g.h_tab[B.hA].x + g.h_tab[B.hB].x);
    F.wsec = (float)m;
    return F;
}

// Entry j of a super-block's edge table: edge tA - 1 + j (j = 0 .. tB - tA + 2)
// as (cos, sin) of its angle relative to edge m, formed in FP64 from the FP64
// edge table.
__device__ __forceinline__ float2 block_edge(const GeomDev &g, const Block &B, int m, int j) {
    const int nt = g.n_theta;
    int b = B.tA - 1 + j;
    b = b < 0 ? b + nt : (b > nt ? b - nt : b);
    const double2 c = g.cs64[b], cm = g.cs64[m];
    return make_float2((float)fma(c.x, cm.x, c.y * cm.y), (float)fma(c.y, cm.x, -(c.x * cm.y)));
}

// Parameter interval of the ray inside the block hull (slab x wedge x disc),
// with the same crossing formulas as the traversal, in the super-block's frame
// (T.cs holds the edges tA - 1 .. tB + 1 of the block in that frame).
__device__ __forceinline__ bool clip_block(const GeomDev &g, const Tabs &T, const ViewDev &V, const Ray &r,
                                           const Block &B, float &s0, float &s1) {
    s0 = r.s_in;
    s1 = r.s_out;
    if (r.ez != 0.0f) {
        const float t1 = plane_s(T.h[B.hA], r), t2 = plane_s(T.h[B.hB], r);
        s0 = fmaxf(s0, fminf(t1, t2));
        s1 = fminf(s1, fmaxf(t1, t2));
    } else if (!(r.pz >= T.h[B.hA].x && r.pz < T.h[B.hB].x)) {
        return false;
    }
    const float2 rt = T.r[B.rB];
    if (r.flags & RAY_AXIAL) {
        if (!((rt.x - r.r0) + (rt.y - r.r0lo) > 0.0f)) return false;
    } else {
        float lo, hi;
        if (!shell_roots(rt, r, lo, hi)) return false;
        s0 = fmaxf(s0, lo);
        s1 = fminf(s1, hi);
    }
    if (B.tB - B.tA >= g.n_theta) return s1 > s0;
    if (r.flags & RAY_THRU) {
        // a line through the axis lies in sector it_in before it and in it_out
        // after it (its own edge tests would be ties at the axis)
        const bool in_ok = (unsigned)(r.it_in - B.tA) < (unsigned)(B.tB - B.tA);
        const bool out_ok = (unsigned)(r.it_out - B.tA) < (unsigned)(B.tB - B.tA);
        if (!in_ok) s0 = fmaxf(s0, r.sc);
        if (!out_ok) s1 = fminf(s1, r.sc);
        return s1 > s0;
    }
    {
        // lower edge: n_A . p >= 0 ; upper edge: n_B . p <= 0
        for (int e = 0; e < 2; ++e) {
            const int eb = e == 0 ? B.tA : B.tB;
            const float2 cs = edge_at<true>(T, eb);
            const float nc = cs.x * r.py - cs.y * r.px;
            float ne = cs.x * r.ey - cs.y * r.ex;
            float x = -nc * frcp(ne);
            if (fabsf(ne) < kEdgeTau && !(r.flags & RAY_AXIAL) && fabsf(nc) <= fabsf(ne) * (s1 - s0 + 1.0f)) {
                bool on_edge;
                edge_cross_fp64(g.cs64[eb], V, r, x, on_edge);
            }
            const float sg = e == 0 ? 1.0f : -1.0f;
            if (ne == 0.0f) {
                // parallel to the edge line: a ray on the line belongs to the
                // sector on the + side, i.e. to the block whose lower edge it is
                if (e == 0 ? (nc < 0.0f) : (nc >= 0.0f)) return false;
                continue;
            }
            if (sg * ne > 0.0f)
                s0 = fmaxf(s0, x);
            else
                s1 = fminf(s1, x);
        }
    }
    return s1 > s0;
}

template <class Visit>
__device__ __forceinline__ void walk_block_ray(const GeomDev &g, const Tabs &T, const Frame &F, const ViewDev &V,
                                               const Block &B, int u, int v, Visit &visit) {
    Ray r;
    double dx, dy, dz;
    ray_setup(g, V, u, v, F, r, dx, dy, dz);
    float s0, s1;
    if (!clip_block(g, T, V, r, B, s0, s1)) return;
    // the hull includes the block's inner hole r < r_A: split the interval
    // there so the walk covers the block cells only
    float pa0 = s0, pa1 = s1, pb0 = 1.0f, pb1 = 0.0f;
    const float2 rtA = T.r[B.rA];
    if (rtA.x > 0.0f) {
        if (r.flags & RAY_AXIAL) {
            if ((rtA.x - r.r0) + (rtA.y - r.r0lo) > 0.0f) return;
        } else {
            float lo, hi;
            if (shell_roots(rtA, r, lo, hi)) {
                pa1 = fminf(s1, lo);
                pb0 = fmaxf(s0, hi);
                pb1 = s1;
            }
        }
    }
    // Walk the first non-empty piece first: most rays that meet the hole have
    // only the piece after it, and a ray with two pieces is rare (nearly
    // tangent to r_A within the wedge), so the second walk is then skipped by
    // whole waves instead of idling every lane whose piece came first.
    if (!(pa1 > pa0)) {
        pa0 = pb0;
        pa1 = pb1;
        pb0 = 1.0f;
        pb1 = 0.0f;
    }
    for (int piece = 0; piece < 2; ++piece) {
        const float a0 = piece ? pb0 : pa0, a1 = piece ? pb1 : pa1;
        if (!(a1 > a0)) continue;
        int ih, it, ir;
        cell_at(g, r, F, a0, ih, it, ir);
        ih = ih < B.hA ? B.hA : (ih >= B.hB ? B.hB - 1 : ih);
        ir = ir < B.rA ? B.rA : (ir >= B.rB ? B.rB - 1 : ir);
        if (it < B.tA || it >= B.tB) {
            // nearest block edge on the circle
            int dlo = B.tA - it;
            if (dlo < 0) dlo += g.n_theta;
            int dhi = it - (B.tB - 1);
            if (dhi < 0) dhi += g.n_theta;
            it = dlo <= dhi ? B.tA : B.tB - 1;
        }
        if (B.tB - B.tA >= g.n_theta)
            traverse<true, true, true, true>(g, T, V, r, a0, a1, ih, it, ir, visit);
        else if (__ballot(needs_refine(r, a0, a1)))
            traverse<false, true, true, true>(g, T, V, r, a0, a1, ih, it, ir, visit);
        else
            traverse<false, true, true, false>(g, T, V, r, a0, a1, ih, it, ir, visit);
    }
}


}  // namespace cyl
