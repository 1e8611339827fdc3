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

// Correctly rounded 1/x for x in [1, 4) (device only): the hardware
// reciprocal (within an ulp) corrected by one fused Newton step.
// tests/recip_check.hip compares it with the correctly rounded division for
// every binary32 x in [1, 4) on the device; the sampling rule calls it with
// x = 1 - s_z in [1, 2].
__device__ __forceinline__ float recip_1_4(float x) {
    const float y = __builtin_amdgcn_rcpf(x);
    const float e = __builtin_fmaf(-x, y, 1.0f);
    return __builtin_fmaf(e, y, y);
}

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

// Eigenvector of the largest eigenvalue of a symmetric 4x4 matrix, by cyclic
// Jacobi rotations (each annihilates one off-diagonal pair; the accumulated
// rotations hold the eigenvectors).
AOR_HD inline void top_eigvec4(double A[4][4], double out[4]) {
    double V[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) V[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 32; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < 4; ++i) {
            diag += A[i][i] * A[i][i];
            for (int j = i + 1; j < 4; ++j) off += A[i][j] * A[i][j];
        }
        if (!(off > 1e-32 * diag)) break;
        for (int p = 0; p < 3; ++p)
            for (int q = p + 1; q < 4; ++q) {
                const double apq = A[p][q];
                if (apq == 0.0) continue;
                const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                A[p][p] -= t * apq;
                A[q][q] += t * apq;
                A[p][q] = A[q][p] = 0.0;
                for (int r = 0; r < 4; ++r) {
                    if (r != p && r != q) {
                        const double arp = A[r][p], arq = A[r][q];
                        A[r][p] = A[p][r] = c * arp - sn * arq;
                        A[r][q] = A[q][r] = sn * arp + c * arq;
                    }
                    const double vrp = V[r][p], vrq = V[r][q];
                    V[r][p] = c * vrp - sn * vrq;
                    V[r][q] = sn * vrp + c * vrq;
                }
            }
    }
    int best = 0;
    for (int i = 1; i < 4; ++i)
        if (A[i][i] > A[best][best]) best = i;
    for (int i = 0; i < 4; ++i) out[i] = V[i][best];
}

// Determinant of the 3x3 matrix left by removing row r and column c of a 4x4.
AOR_HD inline double minor3(const double M[4][4], int r, int c) {
    int ri[3], ci[3];
    for (int k = 0, a = 0, b = 0; k < 4; ++k) {
        if (k != r) ri[a++] = k;
        if (k != c) ci[b++] = k;
    }
    const double* m0 = M[ri[0]];
    const double* m1 = M[ri[1]];
    const double* m2 = M[ri[2]];
    return m0[ci[0]] * (m1[ci[1]] * m2[ci[2]] - m1[ci[2]] * m2[ci[1]]) -
           m0[ci[1]] * (m1[ci[0]] * m2[ci[2]] - m1[ci[2]] * m2[ci[0]]) +
           m0[ci[2]] * (m1[ci[0]] * m2[ci[1]] - m1[ci[1]] * m2[ci[0]]);
}

// Eigenvector of the largest eigenvalue of a symmetric trace-free 4x4 matrix
// N: the eigenvalue by Newton's method on the characteristic polynomial
// lambda^4 + c2 lambda^2 + c1 lambda + c0 (c2 = -tr(N^2)/2, c1 = -tr(N^3)/3,
// c0 = det N), started at sqrt(tr(N^2)) >= lambda_max, where the iteration
// decreases monotonically (all roots are real); the eigenvector is a column of
// the adjugate of N - lambda I, the one with the largest diagonal entry.
// Returns false when that column is too small for a clean direction (a
// near-repeated top eigenvalue); the caller then uses the Jacobi rotations.
AOR_HD inline bool top_eigvec4_newton(const double N[4][4], double out[4]) {
    double N2[4][4];
    double tr2 = 0.0, tr3 = 0.0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 4; ++k) acc += N[i][k] * N[k][j];
            N2[i][j] = acc;
            tr2 += N[i][j] * N[i][j];
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) tr3 += N2[i][j] * N[j][i];
    if (!(tr2 > 0.0)) return false;
    double detN = 0.0;
    for (int j = 0; j < 4; ++j) detN += ((j & 1) ? -1.0 : 1.0) * N[0][j] * minor3(N, 0, j);
    const double c2 = -0.5 * tr2, c1 = -tr3 / 3.0, c0 = detN;
    double lam = sqrt(tr2);
    for (int it = 0; it < 100; ++it) {
        const double l2 = lam * lam;
        const double f = ((l2 + c2) * lam + c1) * lam + c0;
        const double fp = (4.0 * l2 + 2.0 * c2) * lam + c1;
        if (!(fp > 0.0)) break;
        const double step = f / fp;
        lam -= step;
        if (!(fabs(step) > 1e-15 * fabs(lam))) break;
    }
    double M[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) M[i][j] = N[i][j] - (i == j ? lam : 0.0);
    int best = 0;
    double dbest = 0.0;
    for (int i = 0; i < 4; ++i) {
        const double d = fabs(minor3(M, i, i));
        if (d > dbest) {
            dbest = d;
            best = i;
        }
    }
    // a simple top eigenvalue leaves adj(M) = mu v v^T with |mu| about the
    // product of the other three eigenvalue gaps; demand a clear margin
    if (!(dbest > 1e-12 * tr2 * sqrt(tr2))) return false;
    for (int j = 0; j < 4; ++j) out[j] = (((best + j) & 1) ? -1.0 : 1.0) * minor3(M, best, j);
    return true;
}

// Rotation maximising sum q_i . (R p_i) from the sums S[3a + b] = sum p_a q_b
// (equivalently minimising sum ||R p_i - q_i||^2): the unit quaternion
// (w, x, y, z) is the top eigenvector of the symmetric 4x4 matrix N built from
// S (the quaternion method of least-squares registration), then R from the
// quaternion; float64 throughout, rounded once.
AOR_HD inline void ls_rotation_from_sums(const double* S, float* R) {
    double N4[4][4] = {
        {S[0] + S[4] + S[8], S[5] - S[7], S[6] - S[2], S[1] - S[3]},
        {S[5] - S[7], S[0] - S[4] - S[8], S[1] + S[3], S[6] + S[2]},
        {S[6] - S[2], S[1] + S[3], -S[0] + S[4] - S[8], S[5] + S[7]},
        {S[1] - S[3], S[6] + S[2], S[5] + S[7], -S[0] - S[4] + S[8]}};
    double qv[4];
    if (!top_eigvec4_newton(N4, qv)) top_eigvec4(N4, qv);
    const double nq = sqrt(qv[0] * qv[0] + qv[1] * qv[1] + qv[2] * qv[2] + qv[3] * qv[3]);
    const double w = qv[0] / nq, x = qv[1] / nq, y = qv[2] / nq, z = qv[3] / nq;
    const double Rd[9] = {w * w + x * x - y * y - z * z, 2.0 * (x * y - w * z), 2.0 * (x * z + w * y),
                          2.0 * (x * y + w * z), w * w - x * x + y * y - z * z, 2.0 * (y * z - w * x),
                          2.0 * (x * z - w * y), 2.0 * (y * z + w * x), w * w - x * x - y * y + z * z};
    for (int k = 0; k < 9; ++k) R[k] = (float)Rd[k];
}

AOR_HD __forceinline__ int32_t pack_range(int s, int e) {
    return (int32_t)((uint32_t)(uint16_t)(int16_t)s | ((uint32_t)(uint16_t)(int16_t)e << 16));
}
AOR_HD __forceinline__ void unpack_range(int32_t v, int& s, int& e) {
    s = (int)(int16_t)(uint16_t)((uint32_t)v & 0xFFFFu);
    e = (int)(int16_t)(uint16_t)((uint32_t)v >> 16);
}

}  // namespace aoresp
