// Device geometry of the projected great circles and the exact vertex rule.
//
// A correspondence (p, q) with displacement d = p - q = (a, b, c) admits the
// rotation axes r with r . d = 0 (Sec. III-A, Eq. (4)): a great circle of the
// unit sphere.  Stereographic projection from the north pole (Eq. (7)) maps the
// closed southern hemisphere onto the closed unit disk and the great circle
// onto the curve
//     F(u, v) = c (u^2 + v^2 - 1) + 2 (a u + b v) = 0,
// the projected-circle equation of Sec. IV with D = 0, multiplied out.  For
// c != 0 it is the circle with centre -(a, b)/c and radius |d|/|c| >= 1; for
// c = 0 it is the line a u + b v = 0.
//
// Voting rule (Fig. 3(c): a cell counts the circles through it): a cell gets
// one vote from a correspondence iff it meets the closed unit disk, one of its
// corners has F <= 0 and one has F >= 0.  F at a vertex is the binary32
// expression (c*W) + 2*((a*u) + (b*v)), W = ((u*u) + (v*v)) - 1, every
// operation rounded once (the build disables contraction).
//
// Why the walk below is exact.  For 2^-100 <= max(|a|,|b|,|c|) <= 2^120 the
// binary32 value differs from the real F by at most
// E = 2^-22 (|c| + 2|a| + 2|b|) + 2^-140, and |F| >= |d| * dist(vertex, curve),
// so every vertex farther than E/|d| < 1e-6 from the curve gets the sign of
// the real F.  The circle is split at its four 45-degree points: on the top
// and bottom quarters |dv/du| <= 1 and on the left and right quarters
// |du/dv| <= 1 (in grid-index units).  Scanning a quarter across the vertex lines it crosses at 45
// degrees or steeper, at most one vertex per line lies within 1.5e-6 of the
// crossing (grid steps are >= 1.5e-5), so along each line the signs read
// "+ ... +, at most one zero, - ... -" around the crossing.  With lo = first
// vertex with sigma*F <= 0 and hi = last vertex with sigma*F >= 0 on the two
// lines that bound a cell column, the voted cells of that column are exactly
// rows min(lo) - 1 .. max(hi).
//
// Local frame: a walk scans "along" vertex lines x_j (columns in column mode,
// rows in row mode) and locates the crossing in the "cross" coordinate y.  The
// roles of (a, u) and (b, v) swap in row mode; the binary32 value of F at a
// vertex is unchanged because + and * commute exactly.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef AOR_HD
#define AOR_HD __host__ __device__
#endif

namespace aoresp {

// sigma * F-hat at (x, y): a, b, c already multiplied by sigma (exact negation).
// xx = x*x and ax = a_loc*x are per-line terms.
AOR_HD __forceinline__ float vertex_F(float b_loc, float c, float xx, float ax, float y) {
    float yy = y * y;
    float w = (xx + yy) - 1.0f;
    float cw = c * w;
    float by = b_loc * y;
    float s = ax + by;
    float s2 = 2.0f * s;
    return cw + s2;
}

// Roots y of c y^2 + 2 b y + K = 0 with K = c (x^2 - 1) + 2 a x, i.e. where
// the curve crosses the vertex line at along-coordinate x (float64; c >= 0).
// sel = 0 returns the lower root, 1 the upper one; a line (c == 0) has one.
AOR_HD __forceinline__ double cross_root(double a, double b, double c, double x, int sel) {
    double K = c * (x * x - 1.0) + 2.0 * a * x;
    if (c == 0.0) return -K / (2.0 * b);
    double t = c * x + a;
    double disc = (a * a + b * b + c * c) - t * t;   // = b^2 - c K
    if (disc < 0.0) disc = 0.0;
    double sq = sqrt(disc);
    double qq = -(b + copysign(sq, b));
    // qq / c and K / qq are the two roots; qq / c is the lower one when b has
    // a positive sign bit (then qq <= 0) and the upper one otherwise, so only
    // the requested root is divided out
    const bool r1_wanted = (sel == 0) != (bool)signbit(b);
    if (r1_wanted || qq == 0.0) return qq / c;
    return K / qq;
}

// Reciprocal and square root to about one ulp (the hardware instructions on
// the GPU), for values that only seed an exact search.
AOR_HD __forceinline__ float seed_rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
AOR_HD __forceinline__ float seed_sqrt(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#else
    return sqrtf(x);
#endif
}

// The same root in binary32, for a, b, c scaled to |a| + |b| + |c| = 1 (the
// roots do not depend on the scale), to about an ulp.  Used only to seed an
// exact search.
AOR_HD __forceinline__ float cross_root_f(float a, float b, float c, float x, int sel) {
    const float K = c * (x * x - 1.0f) + 2.0f * a * x;
    if (c == 0.0f) return -K * seed_rcp(2.0f * b);
    const float t = c * x + a;
    float disc = (a * a + b * b + c * c) - t * t;
    if (disc < 0.0f) disc = 0.0f;
    const float qq = -(b + copysignf(seed_sqrt(disc), b));
    const bool r1_wanted = (sel == 0) != (bool)signbit(b);
    if (r1_wanted || qq == 0.0f) return qq * seed_rcp(c);
    return K * seed_rcp(qq);
}

AOR_HD __forceinline__ int32_t pack_range(int s, int e) {
    return (int32_t)((uint32_t)(uint16_t)(int16_t)s | ((uint32_t)(uint16_t)(int16_t)e << 16));
}
AOR_HD __forceinline__ void unpack_range(int32_t v, int& s, int& e) {
    s = (int)(int16_t)(uint16_t)((uint32_t)v & 0xFFFFu);
    e = (int)(int16_t)(uint16_t)((uint32_t)v >> 16);
}

}  // namespace aoresp
