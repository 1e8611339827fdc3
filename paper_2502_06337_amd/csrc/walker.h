// Host/device walker of the projected circles: octant pieces of a circle in a
// grid frame and the per-line transition walk that lists the voted cells.
// Compiled for the GPU in kernels.hip; the same functions build on the host so
// the indexing can be checked on a CPU (no host product path calls them).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "geometry.h"
#include "kernels.h"

namespace aoresp {

AOR_HD __forceinline__ int clamp_index(double t, int lo, int hi) {
    if (!(t > (double)lo)) return lo;   // also catches NaN
    if (t > (double)hi) return hi;
    return (int)t;
}

// Index of coordinate t on the lattice x0 + k * hx, before rounding: (t - x0)
// / hx, computed as a product with 1 / hx when the step is a power of two
// (then both give the same value).
template <bool kPow2Step>
AOR_HD __forceinline__ double lattice_index(double t, double x0, double hx) {
    if (kPow2Step) return (t - x0) * (1.0 / hx);
    return (t - x0) / hx;
}

// Restrict a monotone octant [s, e] (vertex indices along x) to the vertex
// lines where its crossing lies in [ylo, yhi].  side selects the along-root
// (0: smaller, 1: larger) when solving for x at a given cross value.
template <bool kPow2Step>
AOR_HD inline void clip_octant(double aL, double bL, double c, int sel, int side, double x0, double hx, double ylo,
                               double yhi, int nmax, int& s, int& e) {
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
    int sa = clamp_index(floor(lattice_index<kPow2Step>(xa, x0, hx)) - 1.0, -2, nmax + 2);
    int eb = clamp_index(ceil(lattice_index<kPow2Step>(xb, x0, hx)) + 1.0, -2, nmax + 2);
    if (sa > s) s = sa;
    if (eb < e) e = eb;
    if (e < s) e = s;
}

AOR_HD __forceinline__ uint32_t classify(float a, float b, float c) {
    if (!(isfinite(a) && isfinite(b) && isfinite(c))) return kFlagDegenerate;
    if (a == 0.0f && b == 0.0f && c == 0.0f) return kFlagDegenerate;
    float m = fmaxf(fabsf(a), fmaxf(fabsf(b), fabsf(c)));
    if (m < 0x1p-100f || m > 0x1p120f) return kFlagRisky;
    if (c == 0.0f) return kFlagLine;
    return 0u;
}

// Certification threshold of the coarse walk, T = 1.2e-6 (|a| + |b| + |c|); a
// refinement grid uses 1.5 T.  Evaluated vertices have |u| <= 1 and |v| <=
// 1 + 5h <= 1.16 (the crossing stays within the frame plus the clip margin
// and the walk evaluates the row next to it), so |W| <= 1.35.  Let E bound
// the binary32 error of F at a vertex with sigma*F > T, and S = |a| + |b| +
// |c|.  On the coarse lattice W is exact; the products c*W, a*u, b*v, the
// inner sum and the outer sum each round once (relative 2^-24), and the
// doubling is exact, so |F~ - F| <= 2^-24 (1.35 |c| + 4.7 (|a| + |b|)) +
// 2^-24 |F~|, and near the threshold E <= 4.7 * 2^-24 S.  A refinement grid
// rounds W as well (at most 2^-22, times |c|), so there E <= 5.4 * 2^-24 S.
// The coarse walk's line pairs use the Horner form of vertex_F_fast instead:
// fma(c, x, 2a) and fma(c, y, 2b) round once each (at most 2^-24 (|c| +
// 2|a|) and 2^-24 (1.16 |c| + 2|b|)), K = fma(., x, -c) once more (2^-24
// (2|c| + 2|a|)) and the result once, so its error is at most 2^-24 (4.35 |c|
// + 4 |a| + 2.32 |b|) + 2^-24 |F~| <= 4.4 * 2^-24 S near the threshold.  A
// fast value beyond T (= 20.1 * 2^-24 S) is at least 15.7 * 2^-24 S from zero
// in exact arithmetic, more than E, so vertex_F has its sign.
// (i) sigma*F > T gives an exact F > T - E; along a vertex line |dF/dy| =
// 2 |c y + b| <= L = 2 (1.16 |c| + |b|) <= 3.07 |d|, so the vertex lies
// beyond the curve by a cross gap g >= (T - E) / L.  (ii) The gap carries over
// to the row of the next line that the certificate speaks for, and on an
// octant of slope <= 1 a cross gap g means a distance >= g / sqrt(2) from the
// curve.  (iii) At distance delta from the projected circle (centre C, radius
// R = |d| / c >= 1) |F| = c |rho - R| (rho + R) >= 2 |d| delta (1 - delta / 2R),
// and |F| = 2 |d| delta for a line, so binary32 gets the sign of every vertex
// farther than E / (1.99 |d|).  T must therefore exceed
// E (1 + sqrt(2) L / (1.99 |d|)) <= 3.19 E: 8.9e-7 S on the coarse lattice
// (for either evaluation) and 1.03e-6 S on a refinement grid, margins of 1.34x
// and 1.75x.
AOR_HD __forceinline__ float cert_threshold(float a, float b, float c) {
    return 1.2e-6f * ((fabsf(a) + fabsf(b)) + fabsf(c));
}
constexpr float kFineCertScale = 1.5f;   // refinement grids certify with 1.5 T

// sigma*F at vertex (x, y) in Horner form, from sc = sigma c, tsa = 2 sigma a,
// tsb = 2 sigma b and nsc = -sigma c: fma(fma(sc, y, tsb), y, fma(fma(sc, x,
// tsa), x, nsc)).  Not the rule's binary32 value, but within 4.4 * 2^-24 S of
// the exact one near the threshold, so a value beyond T has vertex_F's sign.
AOR_HD __forceinline__ float vertex_F_fast(float sc, float tsa, float tsb, float nsc, float x, float y) {
    return fmaf(fmaf(sc, y, tsb), y, fmaf(fmaf(sc, x, tsa), x, nsc));
}

// Octant pieces of the curve of (a, b, c) (c >= 0; not degenerate, not risky)
// in the frame u = u0 + j*hu (j in [0, nu]), v = v0 + k*hv (k in [0, nv]).
//
// The circle is cut where its slope in grid-index units is 1 (its 45-degree
// points on a square grid): the top and bottom quarters (|dv/du| <= hv/hu)
// are scanned along vertex columns, the left and right quarters
// (|du/dv| <= hu/hv) along vertex rows, so the crossing moves by at most one
// index per scanned line.  Each quarter is split at its
// extreme point into two monotone octants.  Octant p of a quarter:
//   colp: p = 0 lower root left of the bottom point, 1 lower root right of it,
//         2 upper root left of the top point, 3 upper root right of it;
//   rowp: p = 0 lower u-root below the left point, 1 above it, 2 upper u-root
//         below the right point, 3 above it.
// Cells are owned by exactly one piece: column pieces own cell columns
// [ja, jb); row pieces own rows [ka - 3, kb + 3) but only columns < ja (lower
// u-root) or >= jb (upper u-root); the 3 extra rows cover the cells around the
// 45-degree points.  geo = (ja | jb << 16, jm | km << 16, ka | kb << 16, flags)
// with jm, km the lines just before the extreme points.  kCoarse: the frame
// is the coarse lattice (hu = hv, a power of two), so divisions by the step
// are products and the slope ratio rho is 1.
template <bool kCoarse>
AOR_HD inline void circle_pieces(float af, float bf, float cf, uint32_t flags, double u0, double hu, int nu,
                                 double v0, double hv, int nv, double margin, int4& colp, int4& rowp, int4& geo) {
    const int E = pack_range(0, 0);
    colp = make_int4(E, E, E, E);
    rowp = make_int4(E, E, E, E);
    double a = af, b = bf, c = cf;
    double ulo = u0 - margin, uhi = u0 + nu * hu + margin;
    double vlo = v0 - margin, vhi = v0 + nv * hv + margin;
    int s, e;
    if (flags & kFlagLine) {
        // One straight piece: column mode if |slope| <= 1, else row mode.  Below
        // (left of) the line sigma*F > 0 with sigma = -sign(b) (-sign(a)).
        uint32_t fl = flags;
        if (fabs(a) * hu <= fabs(b) * hv) {
            s = 0;
            e = nu;
            clip_octant<kCoarse>(a, b, 0.0, 0, 0, u0, hu, vlo, vhi, nu, s, e);
            if (s < 0) s = 0;
            if (e > nu) e = nu;
            int32_t pr = pack_range(s, e > s ? e : s);
            if (b < 0.0) colp.x = pr; else colp.z = pr;
            if (a * b > 0.0) fl |= kFlagLineDown;   // v = -(a/b) u decreases
            geo = make_int4(pack_range(-8, nu + 8), pack_range(nu + 8, 0), pack_range(-8, nv + 8), (int)fl);
        } else {
            s = 0;
            e = nv;
            clip_octant<kCoarse>(b, a, 0.0, 0, 0, v0, hv, ulo, uhi, nv, s, e);
            if (s < 0) s = 0;
            if (e > nv) e = nv;
            int32_t pr = pack_range(s, e > s ? e : s);
            if (a < 0.0) rowp.x = pr; else rowp.z = pr;
            if (a * b > 0.0) fl |= kFlagLineDown;   // u = -(b/a) v decreases
            // every column allowed for either root; strict everywhere
            geo = make_int4(pack_range(nu + 8, -8), pack_range(nu + 8, nv + 8), pack_range(-8, nv + 8), (int)fl);
        }
        return;
    }
    double cu = -a / c, cv = -b / c;
    double r = sqrt(a * a + b * b + c * c) / c;
    // Split where the slope in index units is 1: |dv/du| = hv/hu.  With
    // rho = hv/hu the column band is |u - cu| <= r rho / sqrt(1 + rho^2) and
    // the row band |v - cv| <= r / sqrt(1 + rho^2) (r / sqrt(2) each on a
    // square grid).
    // on the coarse lattice rho = 1 and qn folds to a constant
    const double rho = kCoarse ? 1.0 : hv / hu;
    const double qn = 1.0 / sqrt(1.0 + rho * rho);
    double qu = r * rho * qn, qv = r * qn;
    // Indices are clamped 8 lines outside the frame so that the 3-line
    // extension of a clamped band never reaches into the frame.
    int lim_u = nu + 8, lim_v = nv + 8;
    int ja = clamp_index(ceil(lattice_index<kCoarse>(cu - qu, u0, hu)), -8, lim_u);
    int jb = clamp_index(floor(lattice_index<kCoarse>(cu + qu, u0, hu)), -8, lim_u);
    int ka = clamp_index(ceil(lattice_index<kCoarse>(cv - qv, v0, hv)), -8, lim_v);
    int kb = clamp_index(floor(lattice_index<kCoarse>(cv + qv, v0, hv)), -8, lim_v);
    if (jb < ja) jb = ja;
    if (kb < ka) kb = ka;
    int jm = clamp_index(floor(lattice_index<kCoarse>(cu, u0, hu)), ja, jb);
    int km = clamp_index(floor(lattice_index<kCoarse>(cv, v0, hv)), ka, kb);
    int cs[4] = {ja, jm, ja, jm}, ce[4] = {jm, jb, jm, jb};
    int32_t cp[4];
    for (int p = 0; p < 4; ++p) {
        s = cs[p] < 0 ? 0 : cs[p];
        e = ce[p] > nu ? nu : ce[p];
        if (s < e) clip_octant<kCoarse>(a, b, c, p >> 1, p & 1, u0, hu, vlo, vhi, nu, s, e);
        if (s < 0) s = 0;
        if (e > nu) e = nu;
        cp[p] = pack_range(s, e > s ? e : s);
    }
    colp = make_int4(cp[0], cp[1], cp[2], cp[3]);
    int rs[4] = {ka - 3, km, ka - 3, km}, re[4] = {km, kb + 3, km, kb + 3};
    int32_t rp[4];
    for (int p = 0; p < 4; ++p) {
        s = rs[p] < 0 ? 0 : rs[p];
        e = re[p] > nv ? nv : re[p];
        if (s < e) clip_octant<kCoarse>(b, a, c, p >> 1, p & 1, v0, hv, ulo, uhi, nv, s, e);
        if (s < 0) s = 0;
        if (e > nv) e = nv;
        rp[p] = pack_range(s, e > s ? e : s);
    }
    rowp = make_int4(rp[0], rp[1], rp[2], rp[3]);
    geo = make_int4(pack_range(ja, jb), pack_range(jm, km), pack_range(ka, kb), (int)flags);
}

// Direction of the transition index along octant p (+1 grows, -1 shrinks) and
// the vertex lines [lo, hi] on which the octant is monotone with |slope| <= 1.
// A row octant's range loses `shrink` lines at its end away from the extreme
// point (next to the 45-degree point, where its cells meet the columns owned
// by the column pieces).  With shrink = 2 on the coarse lattice no cell of the
// remaining lines reaches an owned column: on vertex row k of the lower
// u-root with |v_k - cv| <= qv - 2h the crossing lies left of cu - qu by
// sqrt(r^2 - (qv - 2h)^2) - qu >= 4h (qv - h) / ((1 + 1/sqrt(2)) r) >= 1.58 h
// (qu = qv = r / sqrt(2), r >= 1, h <= 1/32), so its cell index is at most
// ceil((cu - qu - u0) / h) - 2 = ja - 2; the upper u-root mirrors this with
// cells >= jb + 1.  The walk therefore needs no column bound on those lines.
constexpr int kCoarseRowShrink = 2;
AOR_HD __forceinline__ void octant_walk_info(int mode, int p, const int4& geo, int& dir, int& slo, int& shi,
                                             int shrink = 0) {
    int ja, jb, jm, km, ka, kb;
    unpack_range(geo.x, ja, jb);
    unpack_range(geo.y, jm, km);
    unpack_range(geo.z, ka, kb);
    uint32_t fl = (uint32_t)geo.w;
    if (fl & kFlagLine) {
        dir = (fl & kFlagLineDown) ? -1 : 1;
        slo = -(1 << 20);
        shi = 1 << 20;
        return;
    }
    // column octants: 0 falls, 1 rises, 2 rises, 3 falls; the same for rows
    dir = (p == 0 || p == 3) ? -1 : 1;
    if (mode == 0) {
        slo = (p & 1) ? jm + 1 : ja;
        shi = (p & 1) ? jb : jm;
    } else {
        slo = (p & 1) ? km + 1 : ka + shrink;
        shi = (p & 1) ? kb - shrink : km;
    }
}

// --------------------------------------------------------------------------
// Transition search on one vertex line
// --------------------------------------------------------------------------

constexpr int kMaxSteps = 24;

// Exact search from vertex g: lo = first vertex with sigma*F <= 0, hi = last
// with sigma*F >= 0, for the pattern "+ ... + [0] - ... -" around the crossing.
// flo / fhi return sigma*F at lo and hi when hi == lo - 1 (no zero).
AOR_HD __forceinline__ void find_transition(float sb, float sc, float xx, float ax, float y0, float hy, int g,
                                            int& lo, int& hi, float& flo, float& fhi, uint32_t& bad) {
    int k = g;
    float y = y0 + (float)k * hy;
    float f = vertex_F(sb, sc, xx, ax, y);
    float fprev = f;
    int steps = 0;
    flo = 0.0f;
    fhi = 0.0f;
    if (f > 0.0f) {
#pragma unroll 1
        do {
            fprev = f;
            ++k;
            y += hy;
            f = vertex_F(sb, sc, xx, ax, y);
        } while (f > 0.0f && ++steps < kMaxSteps);
        lo = k;
        hi = k - 1;
        flo = f;
        fhi = fprev;
        if (!(f < 0.0f)) {
            if (f > 0.0f) bad = 1u;
#pragma unroll 1
            while (steps++ < kMaxSteps) {
                y += hy;
                if (vertex_F(sb, sc, xx, ax, y) != 0.0f) break;
                ++k;
            }
            hi = k;
        }
    } else if (f < 0.0f) {
#pragma unroll 1
        do {
            fprev = f;
            --k;
            y -= hy;
            f = vertex_F(sb, sc, xx, ax, y);
        } while (f < 0.0f && ++steps < kMaxSteps);
        hi = k;
        lo = k + 1;
        fhi = f;
        flo = fprev;
        if (!(f > 0.0f)) {
            if (f < 0.0f) bad = 1u;
#pragma unroll 1
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
#pragma unroll 1
        while (steps++ < kMaxSteps) {
            yy += hy;
            if (vertex_F(sb, sc, xx, ax, yy) != 0.0f) break;
            ++kk;
        }
        hi = kk;
        kk = k;
        yy = y;
#pragma unroll 1
        while (steps++ < kMaxSteps) {
            yy -= hy;
            if (vertex_F(sb, sc, xx, ax, yy) != 0.0f) break;
            --kk;
        }
        lo = kk;
        if (steps >= 2 * kMaxSteps) bad = 1u;
    }
}

// Walks over octant cells [cs, ce) of a frame.  The voted cells of cell line
// j are cross indices min(lo_j, lo_j+1) - 1 .. max(hi_j, hi_j+1), handed to
// emit(j, klo, khi) (unclipped).  Both walks start with an exact search on
// line cs, seeded by the float64 crossing.

// Seed: first-above index near the crossing of line cs, and the exact state.
AOR_HD __forceinline__ void walk_start(float sb, float sc, float aL, float bL, float c, int sel, float x0, float hx,
                                       float y0, float hy, int cs, float xx, float ax, int& lo, int& hi, float& flo,
                                       float& fhi, uint32_t& bad) {
    double xr = (double)x0 + (double)cs * (double)hx;
    double yr = cross_root(aL, bL, c, xr, sel);
    double gt = floor((yr - (double)y0) / (double)hy);
    int g = clamp_index(gt, -16, 1 << 14);
    find_transition(sb, sc, xx, ax, y0, hy, g, lo, hi, flo, fhi, bad);
}

// Seed for a certified part.  Where the octant's slope is at most 1 the
// crossing is well conditioned (|c y + b| >= |d| / sqrt(2) there), so the
// binary32 root of the scaled equation lies within a small fraction of a row
// of the exact one; the exact search from the seed fixes the transition.
AOR_HD __forceinline__ void walk_start_cert(float sb, float sc, float aL, float bL, float c, int sel, float x0,
                                            float hx, float y0, float hy, int cs, float xx, float ax, int& lo, int& hi,
                                            float& flo, float& fhi, uint32_t& bad) {
    const float inv = seed_rcp((fabsf(aL) + fabsf(bL)) + c);
    const float yr = cross_root_f(aL * inv, bL * inv, c * inv, x0 + (float)cs * hx, sel);
    const float gt = floorf((yr - y0) * seed_rcp(hy));
    const int g = !(gt > -16.0f) ? -16 : (gt > 16384.0f ? 16384 : (int)gt);
    find_transition(sb, sc, xx, ax, y0, hy, g, lo, hi, flo, fhi, bad);
}

// General walk: an exact search on every line.  Used on the few lines where an
// octant is not known to be monotone with |slope| <= 1 (the line through its
// extreme point, the three lines past a 45-degree point).
template <class Emit>
AOR_HD __forceinline__ void walk_search(float aL, float bL, float c, int sel, float x0, float hx, float y0, float hy,
                                        int cs, int ce, Emit& emit, uint32_t& bad) {
    float sigma = sel ? -1.0f : 1.0f;
    float sa = sigma * aL, sb = sigma * bL, sc = sigma * c;
    float x = x0 + (float)cs * hx;
    float xx = x * x, ax = sa * x;
    int lo, hi, lo1, hi1;
    float flo, fhi;
    walk_start(sb, sc, aL, bL, c, sel, x0, hx, y0, hy, cs, xx, ax, lo, hi, flo, fhi, bad);
    for (int j = cs; j < ce; ++j) {
        x += hx;
        xx = x * x;
        ax = sa * x;
        find_transition(sb, sc, xx, ax, y0, hy, lo, lo1, hi1, flo, fhi, bad);
        emit(j, (lo < lo1 ? lo : lo1) - 1, hi > hi1 ? hi : hi1);
        lo = lo1;
        hi = hi1;
    }
}

// Certified walk on lines where the octant is monotone (direction dir) with
// |slope| <= 1, so the crossing moves by at most one line spacing per step.
//
// State on line j: lo/hi and two certificates, cb ("vertex lo-1 lies below the
// curve by a margin") and ca ("vertex hi+1 lies above it by a margin"); a
// value sigma*F > T (< -T) certifies a vertex.  A certified cross gap carries
// over to the same index on the next line on the side the curve moves away
// from, and to the next index on the side it moves towards.  So on line j+1
// only one or two rows next to the old transition can change side (rows
// lo .. hi+1 of a rising octant, lo-1 .. hi of a falling one, one more where a
// certificate is missing); they are evaluated, every other row keeps its
// certified side.  An evaluated vertex that is not certified is the one
// nearest the crossing (at most one per line), its neighbours are certain, and
// its binary32 sign decides the pattern exactly.
//
// Clean state (both certificates, no zero vertex, hi = lo - 1): the only row
// to evaluate is r = lo - off (off = 1 on a falling octant), the transition
// moves to r + (F > 0), and the voted cells of the column are r - 1 + off and,
// if (F > 0) != off, also r - off.  Such a line costs one vertex evaluation
// and goes to emit.pair(cursor, r, second_voted).  A value |F| <= T leaves one
// certificate missing; the next line and any zero vertex go through the
// general step, which evaluates one or two rows and emits the range
// min(lo) - 1 .. max(hi) of the two lines.
//
// Emitter interface: start(j, off) returns a cursor for line j (and may set
// up the pair offsets for this octant), next(cursor) advances it by a line,
// pair(cursor, r, second) emits the clean-state cells, and emit(j, klo, khi)
// a general range.  An emitter with kPairedLines set stores lines 2m and
// 2m + 1 in one row m instead: row_start(j, off) returns the row of line j,
// next_row(row) the following one, rows_after(row, n) the n-th following
// one, range_h<H>(row, klo, khi) emits a general range of the line with
// parity H in that row, pair_h<H>(row, r, second) its clean-state cells;
// cell_of(row, r) is a handle of cross index r in a row, index_of(row, cell)
// gives r back, next_cell(cell) is the same index in the following row, and
// pair2(cell, up0, up1) emits the cells of both lines of a row walked clean
// from row r0 = the cell's index (r1 = r0 + up0 - off, r2 = r1 + up1 - off;
// line 2m: cell r0 - 1 + off, and r1 - 1 + off if it differs; line 2m + 1:
// cell r1 - 1 + off, and r2 - 1 + off if it differs) and returns r2's handle.
// An emitter with kAudit set also receives, on every clean line, the values
// at the two rows next to the evaluated one (audit(fb, fa)), so that a host
// test can check what the certificates claim.  kLattice: every vertex
// coordinate y0 + k*hy is exact and
// so are sums of them (the coarse grid), so the evaluated row's coordinate is
// carried from line to line instead of recomputed.
template <bool kLattice = false, class Emit>
AOR_HD __forceinline__ void walk_certified(float aL, float bL, float c, int sel, int dir, float T, float x0, float hx,
                                           float y0, float hy, int cs, int ce, Emit& emit, uint32_t& bad) {
    float sigma = sel ? -1.0f : 1.0f;
    float sa = sigma * aL, sb = sigma * bL, sc = sigma * c;
    float x = x0 + (float)cs * hx;
    float xx = x * x, ax = sa * x;
    int lo, hi;
    float flo, fhi;
    walk_start_cert(sb, sc, aL, bL, c, sel, x0, hx, y0, hy, cs, xx, ax, lo, hi, flo, fhi, bad);
    // certificates of the bracketing vertices after the search
    bool cb = (hi == lo - 1) ? (fhi > T) : true;
    bool ca = (hi == lo - 1) ? (flo < -T) : true;
    if (hi >= lo) {
        // a zero vertex at lo..hi: its neighbours were found non-zero by the
        // search; certify them by evaluation
        float yb = y0 + (float)(lo - 1) * hy, ya = y0 + (float)(hi + 1) * hy;
        cb = vertex_F(sb, sc, xx, ax, yb) > T;
        ca = vertex_F(sb, sc, xx, ax, ya) < -T;
    }
    const int off = dir < 0 ? 1 : 0;
    // The state between lines lives in registers that the clean path either
    // leaves alone or overwrites, never in execution masks (whose merging at
    // every join would cost scalar instructions on each line).  cert holds the
    // certificates (bit 0: cb, bit 1: ca).  lastf holds the state class:
    //   |lastf| > T      clean (the value evaluated on the previous line, or
    //                    +inf after a general step that ended clean);
    //   0 < |lastf| <= T the previous line left the clean state there: lo,
    //                    hi, cb and ca are rebuilt from r and lastf's sign;
    //   lastf == 0       not clean, lo, hi and cert hold the state.
    const bool clean0 = cb && ca && hi == lo - 1;
    int cert = (cb ? 1 : 0) | (ca ? 2 : 0);
    const float kCleanMark = __builtin_huge_valf();
    int r = lo - off;   // the row evaluated next while clean
    float yr = y0 + (float)r * hy;
    float dy_up = (float)(1 - off) * hy, dy_dn = -(float)off * hy;   // exact: off is 0 or 1
#if defined(__HIP_DEVICE_COMPILE__)
    // opaque to the optimiser, so that the row update below stays one select
    // of these two values instead of a select of 1 - off / -off times hy
    __asm__("" : "+v"(dy_up), "+v"(dy_dn));
#endif
    float lastf = clean0 ? kCleanMark : 0.0f;
    // One cell line.  clean = fabsf(lastf) > T (the caller's, so that a
    // comparison it already made is not repeated); clean_pair(r, second)
    // emits the clean-state cells of the line, range(klo, khi) a general range.
    auto step = [&](bool clean, auto&& range, auto&& clean_pair) {
        x += hx;
        xx = x * x;
        ax = sa * x;
        // evaluated on every lane; only clean lanes use it
        const float f = vertex_F(sb, sc, xx, ax, kLattice ? yr : y0 + (float)r * hy);
        if (clean && f != 0.0f) {
            if constexpr (Emit::kAudit) {
                // test builds only: the certificates vouch for sigma*F > 0 at
                // row r - 1 and sigma*F < 0 at row r + 1 of this line
                emit.audit(vertex_F(sb, sc, xx, ax, y0 + (float)(r - 1) * hy),
                           vertex_F(sb, sc, xx, ax, y0 + (float)(r + 1) * hy));
            }
            const bool up = f > 0.0f;
            clean_pair(r, up != (off != 0));
            r += (up ? 1 : 0) - off;
            if (kLattice) yr += up ? dy_up : dy_dn;
            lastf = f;
            return;
        }
        cb = (cert & 1) != 0;
        ca = (cert & 2) != 0;
        if (!clean && lastf != 0.0f) {
            // the evaluated vertex of the previous line was not certified
            lo = r + off;
            hi = lo - 1;
            cb = !(lastf > 0.0f);
            ca = !(lastf < 0.0f);
        }
        lastf = 0.0f;
        if (clean) {
            // zero vertex on the evaluated row: rebuild the full state
            lo = r + off;
            hi = lo - 1;
            cb = true;
            ca = true;
        } else if (hi == lo - 1) {
            // One certificate missing, no zero vertex: rows r0 and r0 + 1.
            // This is the general step below with its zero-free outcomes.
            const int r0 = lo - off - (cb ? 0 : 1);
            const float ym = y0 + (float)r0 * hy;
            const float f0 = vertex_F(sb, sc, xx, ax, ym);
            const float f1 = vertex_F(sb, sc, xx, ax, ym + hy);
            const int lo1 = f0 < 0.0f ? r0 : (f1 < 0.0f ? r0 + 1 : r0 + 2);
            const bool cb1 = lo1 == r0 ? true : ((lo1 == r0 + 1 ? f0 : f1) > T);
            const bool ca1 = lo1 == r0 + 2 ? true : ((lo1 == r0 ? f0 : f1) < -T);
            if (f0 != 0.0f && f1 != 0.0f && !(f0 < 0.0f && f1 > 0.0f) && (cb1 || ca1)) {
                range((lo < lo1 ? lo : lo1) - 1, (lo > lo1 ? lo : lo1) - 1);
                lo = lo1;
                hi = lo1 - 1;
                cert = (cb1 ? 1 : 0) | (ca1 ? 2 : 0);
                lastf = (cb1 && ca1) ? kCleanMark : 0.0f;
                r = lo - off;
                if (kLattice) yr = y0 + (float)r * hy;
                return;
            }
        }
        // General step.  Rows that may change side on line j+1 (all others
        // keep a certified side): rising, lo .. hi+1 widened by one below
        // without cb and one above without ca; falling, lo-1 .. hi widened the
        // same way.
        const int r0 = lo - off - (cb ? 0 : 1);
        const int r1 = hi + 1 - off + (ca ? 0 : 1);
        if (r1 > r0 + 1) bad |= 8u;   // cannot happen: one uncertain vertex per line
        const float y = y0 + (float)r0 * hy;
        const float f0 = vertex_F(sb, sc, xx, ax, y);
        float f1 = f0;
        if (r1 > r0) f1 = vertex_F(sb, sc, xx, ax, y + hy);
        int lo1, hi1;
        if (f0 <= 0.0f) lo1 = r0; else if (r1 > r0 && f1 <= 0.0f) lo1 = r1; else lo1 = r1 + 1;
        if (r1 > r0 && f1 >= 0.0f) hi1 = r1; else if (f0 >= 0.0f) hi1 = r0; else hi1 = r0 - 1;
        // certificates on line j+1
        const int bv = lo1 - 1, av = hi1 + 1;
        bool cb1 = bv < r0 ? true : ((bv == r0 ? f0 : f1) > T);
        bool ca1 = av > r1 ? true : ((av == r0 ? f0 : f1) < -T);
        if ((r1 > r0 && f0 < 0.0f && f1 > 0.0f) || (!cb1 && !ca1) || (bv > r1) || (av < r0)) {
            // pattern inconsistent with the analysis: exact search instead
            float flo2, fhi2;
            find_transition(sb, sc, xx, ax, y0, hy, lo, lo1, hi1, flo2, fhi2, bad);
            cb1 = false;
            ca1 = false;
            if (hi1 == lo1 - 1) {
                cb1 = fhi2 > T;
                ca1 = flo2 < -T;
            }
            if (!cb1 || !ca1) {
                // certify the bracketing vertices directly (rare path)
                float yb = y0 + (float)(lo1 - 1) * hy, ya = y0 + (float)(hi1 + 1) * hy;
                cb1 = vertex_F(sb, sc, xx, ax, yb) > T;
                ca1 = vertex_F(sb, sc, xx, ax, ya) < -T;
                if (!cb1 || !ca1) bad |= 4u;
            }
        }
        range((lo < lo1 ? lo : lo1) - 1, hi > hi1 ? hi : hi1);
        lo = lo1;
        hi = hi1;
        cert = (cb1 ? 1 : 0) | (ca1 ? 2 : 0);
        lastf = (cb1 && ca1 && hi == lo - 1) ? kCleanMark : 0.0f;
        r = lo - off;
        if (kLattice) yr = y0 + (float)r * hy;
    };
    if constexpr (Emit::kPairedLines) {
        // Lines 2m and 2m + 1 share the emitter's row m: walk them in pairs,
        // so that the row advances once per pair and each half of the pair
        // has a fixed slot (an odd first line and an even last line alone).
        // A pair whose state is clean and whose two fast values (vertex_F_fast,
        // the second at the row the first one moves to) both lie beyond T is
        // decided by their signs and emitted at once; any other pair goes line
        // by line through the exact step.
        static_assert(kLattice, "line pairs are walked on the coarse lattice");
        const float tsa = 2.0f * sa, tsb = 2.0f * sb, nsc = -sc;
        auto row = emit.row_start(cs, off);
        auto range0 = [&](int klo, int khi) { emit.template range_h<0>(row, klo, khi); };
        auto range1 = [&](int klo, int khi) { emit.template range_h<1>(row, klo, khi); };
        auto pair0 = [&](int rr, bool s2) { emit.template pair_h<0>(row, rr, s2); };
        auto pair1 = [&](int rr, bool s2) { emit.template pair_h<1>(row, rr, s2); };
        int j = cs;
        if (j & 1) {
            step(fabsf(lastf) > T, range1, pair1);
            ++j;
            row = emit.next_row(row);
        }
        const auto row_end = emit.rows_after(row, (ce - j) >> 1);
        const bool last_alone = ((ce - j) & 1) != 0;
        // fast pairs carry a handle of cell r of the row (r itself is taken
        // back from it where the exact step needs it)
        auto cell = emit.cell_of(row, r);
        for (; row != row_end; row = emit.next_row(row), cell = emit.next_cell(cell)) {
            const float xa = x + hx, xb = xa + hx;
            const float f0 = vertex_F_fast(sc, tsa, tsb, nsc, xa, yr);
            const bool up0 = f0 > 0.0f;
            const float y1 = yr + (up0 ? dy_up : dy_dn);
            const float f1 = vertex_F_fast(sc, tsa, tsb, nsc, xb, y1);
            // one three-way minimum of magnitudes and one compare (the values
            // are finite: risky curves never reach the walk)
            if (fminf(fminf(fabsf(lastf), fabsf(f0)), fabsf(f1)) > T) {
                const bool up1 = f1 > 0.0f;
                if constexpr (Emit::kAudit) {
                    // test builds only: the rule's values agree in sign with the
                    // fast ones, and the certificates hold on both lines
                    const int rc = emit.index_of(row, cell);
                    const int r1 = rc + (up0 ? 1 : 0) - off;
                    const float xxa = xa * xa, axa = sa * xa, xxb = xb * xb, axb = sa * xb;
                    const float ea = vertex_F(sb, sc, xxa, axa, yr), eb = vertex_F(sb, sc, xxb, axb, y1);
                    emit.audit(up0 ? ea : -ea, -1.0f);
                    emit.audit(up1 ? eb : -eb, -1.0f);
                    emit.audit(vertex_F(sb, sc, xxa, axa, y0 + (float)(rc - 1) * hy),
                               vertex_F(sb, sc, xxa, axa, y0 + (float)(rc + 1) * hy));
                    emit.audit(vertex_F(sb, sc, xxb, axb, y0 + (float)(r1 - 1) * hy),
                               vertex_F(sb, sc, xxb, axb, y0 + (float)(r1 + 1) * hy));
                }
                cell = emit.pair2(cell, up0, up1);   // now at r2
                yr = y1 + (up1 ? dy_up : dy_dn);
                x = xb;
                // the state stays clean: lastf keeps a value beyond T
            } else {
                r = emit.index_of(row, cell);
                step(fabsf(lastf) > T, range0, pair0);
                step(fabsf(lastf) > T, range1, pair1);
                cell = emit.cell_of(row, r);
            }
        }
        r = emit.index_of(row, cell);
        if (last_alone) step(fabsf(lastf) > T, range0, pair0);
    } else {
        auto cur = emit.start(cs, off);
        int j = cs;
        auto range = [&](int klo, int khi) { emit(j, klo, khi); };
        auto pair = [&](int rr, bool s2) { emit.pair(cur, rr, s2); };
        for (; j < ce; ++j, cur = emit.next(cur)) step(fabsf(lastf) > T, range, pair);
    }
}

// Cells [cs, ce) of octant p split into the certified part and the lines
// around it that need a search: parts[0..2] = head (search), body
// (certified), tail (search); empty parts have s >= e.
AOR_HD __forceinline__ void split_piece(int cs, int ce, int slo, int shi, int2* parts) {
    int b0 = cs > slo ? cs : slo;
    int b1 = ce < shi ? ce : shi;
    if (b1 < b0) b1 = b0;
    parts[0] = make_int2(cs, b0 < ce ? b0 : ce);
    parts[1] = make_int2(b0, b1);
    parts[2] = make_int2(b1 > cs ? b1 : cs, ce);
}

// Part q of split_piece alone (selects only, so nothing goes to scratch).
AOR_HD __forceinline__ int2 piece_part(int cs, int ce, int slo, int shi, int q) {
    int b0 = cs > slo ? cs : slo;
    int b1 = ce < shi ? ce : shi;
    if (b1 < b0) b1 = b0;
    int s = q == 0 ? cs : (q == 1 ? b0 : (b1 > cs ? b1 : cs));
    int e = q == 0 ? (b0 < ce ? b0 : ce) : (q == 1 ? b1 : ce);
    return make_int2(s, e);
}

}  // namespace aoresp
