// Host/device walker of the projected circles: octant pieces of a circle in a
// grid frame and the exact per-line transition walk.  Compiled for the GPU in
// kernels.hip; the same functions build on the host for CPU checks of the
// indexing (nothing on the host product path calls them).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "geometry.h"
#include "kernels.h"

namespace aoresp {

// --------------------------------------------------------------------------
// Octant pieces of one circle in one grid frame
// --------------------------------------------------------------------------

AOR_HD __forceinline__ int clamp_index(double t, int lo, int hi) {
    if (!(t > (double)lo)) return lo;   // also catches NaN
    if (t > (double)hi) return hi;
    return (int)t;
}

// Restrict a monotone octant [s, e] (vertex indices along x) to the vertex
// lines where its crossing lies in [ylo, yhi].  side selects the along-root
// (0: smaller, 1: larger) when solving for x at a given cross value.
AOR_HD void clip_octant(double aL, double bL, double c, int sel, int side, double x0, double hx,
                            double ylo, double yhi, int nmax, int& s, int& e) {
    if (s >= e) return;
    double xs = x0 + s * hx, xe = x0 + e * hx;
    double ys = cross_root(aL, bL, c, xs, sel), ye = cross_root(aL, bL, c, xe, sel);
    double xa = xs, xb = xe;
    if (ye >= ys) {
        if (ys > yhi || ye < ylo) { e = s; return; }
        if (ys < ylo) xa = cross_root(bL, aL, c, ylo, side);
        if (ye > yhi) xb = cross_root(bL, aL, c, yhi, side);
    } else {
        if (ye > yhi || ys < ylo) { e = s; return; }
        if (ys > yhi) xa = cross_root(bL, aL, c, yhi, side);
        if (ye < ylo) xb = cross_root(bL, aL, c, ylo, side);
    }
    int sa = clamp_index(floor((xa - x0) / hx) - 1.0, -2, nmax + 2);
    int eb = clamp_index(ceil((xb - x0) / hx) + 1.0, -2, nmax + 2);
    if (sa > s) s = sa;
    if (eb < e) e = eb;
    if (e < s) e = s;
}

// Pieces of the curve of (a, b, c) (c >= 0, not degenerate, not risky) in the
// frame u = u0 + j*hu (j in [0, nu]), v = v0 + k*hv (k in [0, nv]).
// colp: vertex-column ranges of the column-mode octants (lower root left /
// right of the bottom point, upper root left / right of the top point).
// rowp: vertex-row ranges of the row-mode octants (lower u-root below / above
// the left point, upper u-root below / above the right point), extended by 3
// rows past the 45-degree points so that the cells around those points are
// owned by exactly one piece.  clip = (ja, jb): lower-u-root cells must have
// column < ja, upper-u-root cells column >= jb.
AOR_HD void circle_pieces(float af, float bf, float cf, bool line, double u0, double hu, int nu,
                              double v0, double hv, int nv, double margin, int4& colp, int4& rowp,
                              int32_t& clip) {
    const int E = pack_range(0, 0);
    colp = make_int4(E, E, E, E);
    rowp = make_int4(E, E, E, E);
    double a = af, b = bf, c = cf;
    double ulo = u0 - margin, uhi = u0 + nu * hu + margin;
    double vlo = v0 - margin, vhi = v0 + nv * hv + margin;
    int s, e;
    if (line) {
        // One monotone piece: column mode if |slope| <= 1, else row mode; below
        // (left of) the line sigma*F > 0 with sigma = -sign(b) (-sign(a)).
        if (fabs(a) <= fabs(b)) {
            s = 0;
            e = nu;
            clip_octant(a, b, 0.0, 0, 0, u0, hu, vlo, vhi, nu, s, e);
            if (s < 0) s = 0;
            if (e > nu) e = nu;
            int32_t pr = pack_range(s, e > s ? e : s);
            if (b < 0.0) colp.x = pr; else colp.z = pr;
            clip = pack_range(0, nu);
        } else {
            s = 0;
            e = nv;
            clip_octant(b, a, 0.0, 0, 0, v0, hv, ulo, uhi, nv, s, e);
            if (s < 0) s = 0;
            if (e > nv) e = nv;
            int32_t pr = pack_range(s, e > s ? e : s);
            if (a < 0.0) rowp.x = pr; else rowp.z = pr;
            clip = pack_range(nu, 0);
        }
        return;
    }
    double cu = -a / c, cv = -b / c;
    double r = sqrt(a * a + b * b + c * c) / c;
    double q = r * 0.70710678118654752440;
    // Indices are clamped 8 lines outside the frame so that the 3-line
    // extension of a clamped band never reaches into the frame.
    int lim_u = nu + 8, lim_v = nv + 8;
    int ja = clamp_index(ceil((cu - q - u0) / hu), -8, lim_u);
    int jb = clamp_index(floor((cu + q - u0) / hu), -8, lim_u);
    int ka = clamp_index(ceil((cv - q - v0) / hv), -8, lim_v);
    int kb = clamp_index(floor((cv + q - v0) / hv), -8, lim_v);
    if (jb < ja) jb = ja;
    if (kb < ka) kb = ka;
    int jm = clamp_index(floor((cu - u0) / hu), ja, jb);
    int km = clamp_index(floor((cv - v0) / hv), ka, kb);
    // column-mode octants: along = u, cross = v
    int cs[4] = {ja, jm, ja, jm}, ce[4] = {jm, jb, jm, jb};
    int32_t cp[4];
    for (int p = 0; p < 4; ++p) {
        s = cs[p] < 0 ? 0 : cs[p];
        e = ce[p] > nu ? nu : ce[p];
        if (s < e) clip_octant(a, b, c, p >> 1, p & 1, u0, hu, vlo, vhi, nu, s, e);
        if (s < 0) s = 0;
        if (e > nu) e = nu;
        cp[p] = pack_range(s, e > s ? e : s);
    }
    colp = make_int4(cp[0], cp[1], cp[2], cp[3]);
    // row-mode octants: along = v, cross = u
    int rs[4] = {ka - 3, km, ka - 3, km}, re[4] = {km, kb + 3, km, kb + 3};
    int32_t rp[4];
    for (int p = 0; p < 4; ++p) {
        s = rs[p] < 0 ? 0 : rs[p];
        e = re[p] > nv ? nv : re[p];
        if (s < e) clip_octant(b, a, c, p >> 1, p & 1, v0, hv, ulo, uhi, nv, s, e);
        if (s < 0) s = 0;
        if (e > nv) e = nv;
        rp[p] = pack_range(s, e > s ? e : s);
    }
    rowp = make_int4(rp[0], rp[1], rp[2], rp[3]);
    clip = pack_range(ja, jb);
}

AOR_HD __forceinline__ uint32_t classify(float a, float b, float c) {
    if (!(isfinite(a) && isfinite(b) && isfinite(c))) return kFlagDegenerate;
    if (a == 0.0f && b == 0.0f && c == 0.0f) return kFlagDegenerate;
    float m = fmaxf(fabsf(a), fmaxf(fabsf(b), fabsf(c)));
    if (m < 0x1p-100f || m > 0x1p120f) return kFlagRisky;
    if (c == 0.0f) return kFlagLine;
    return 0u;
}

// --------------------------------------------------------------------------
// Transition search on one vertex line
// --------------------------------------------------------------------------

constexpr int kMaxSteps = 24;

// lo = first vertex (upward from g) with sigma*F <= 0, hi = last with
// sigma*F >= 0, given the sign pattern "+ ... + [0] - ... -" near g.
AOR_HD __forceinline__ void find_transition(float sb, float sc, float xx, float ax, float y0, float hy,
                                                int g, int& lo, int& hi, uint32_t& bad) {
    int k = g;
    float y = y0 + (float)k * hy;
    float f = vertex_F(sb, sc, xx, ax, y);
    int steps = 0;
    if (f > 0.0f) {
        do {
            ++k;
            y += hy;
            f = vertex_F(sb, sc, xx, ax, y);
        } while (f > 0.0f && ++steps < kMaxSteps);
        lo = k;
        hi = k - 1;
        if (!(f < 0.0f)) {
            if (f > 0.0f) bad = 1u;
            while (steps++ < kMaxSteps) {
                y += hy;
                if (vertex_F(sb, sc, xx, ax, y) != 0.0f) break;
                ++k;
            }
            hi = k;
        }
    } else if (f < 0.0f) {
        do {
            --k;
            y -= hy;
            f = vertex_F(sb, sc, xx, ax, y);
        } while (f < 0.0f && ++steps < kMaxSteps);
        hi = k;
        lo = k + 1;
        if (!(f > 0.0f)) {
            if (f < 0.0f) bad = 1u;
            while (steps++ < kMaxSteps) {
                y -= hy;
                if (vertex_F(sb, sc, xx, ax, y) != 0.0f) break;
                --k;
            }
            lo = k;
        }
    } else {
        int kk = k;
        float yy = y;
        while (steps++ < kMaxSteps) {
            yy += hy;
            if (vertex_F(sb, sc, xx, ax, yy) != 0.0f) break;
            ++kk;
        }
        hi = kk;
        kk = k;
        yy = y;
        while (steps++ < kMaxSteps) {
            yy -= hy;
            if (vertex_F(sb, sc, xx, ax, yy) != 0.0f) break;
            --kk;
        }
        lo = kk;
        if (steps >= 2 * kMaxSteps) bad = 1u;
    }
}

// Walk one octant piece over cell lines [cs, ce) of a frame.  emit(j, klo, khi)
// receives the voted cross range of cell line j (before clipping).
template <class Emit>
AOR_HD __forceinline__ void walk_piece(float aL, float bL, float c, int sel, float x0, float hx, float y0,
                                           float hy, int cs, int ce, Emit& emit, uint32_t& bad) {
    float sigma = sel ? -1.0f : 1.0f;
    double xr = (double)x0 + (double)cs * (double)hx;
    double yr = cross_root(aL, bL, c, xr, sel);
    double gt = floor((yr - (double)y0) / (double)hy);
    int g = clamp_index(gt, -8, 1 << 14);
    float sa = sigma * aL, sb = sigma * bL, sc = sigma * c;
    float x = x0 + (float)cs * hx;
    float xx = x * x, ax = sa * x;
    int lo0, hi0, lo1, hi1;
    find_transition(sb, sc, xx, ax, y0, hy, g, lo0, hi0, bad);
    for (int j = cs; j < ce; ++j) {
        x += hx;
        xx = x * x;
        ax = sa * x;
        find_transition(sb, sc, xx, ax, y0, hy, lo0, lo1, hi1, bad);
        int rlo = (lo0 < lo1 ? lo0 : lo1) - 1;
        int rhi = hi0 > hi1 ? hi0 : hi1;
        emit(j, rlo, rhi);
        lo0 = lo1;
        hi0 = hi1;
    }
}


}  // namespace aoresp
