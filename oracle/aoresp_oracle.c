/*
 * aoresp_oracle.c -- plain, slow, single-threaded CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code, header, table or constant generator with the HIP library; the two
 * sides meet only through the seeded input generator.
 *
 * What it computes (paper: "Accelerating Outlier-robust Rotation Estimation by
 * Stereographic Projection", Xu, Liu, Wang, Yang):
 *   - Sec. III-A, Eq. (2)-(4): each correspondence (p, q) restricts the rotation
 *     axis r to the great circle r . (p - q) = 0.
 *   - Sec. IV, Eq. (7)-(9): stereographic projection from the north pole maps
 *     the closed southern hemisphere onto the closed unit disk; the great
 *     circle normal to d = (a, b, c) becomes the plane curve
 *         F(u, v) = c (u^2 + v^2 - 1) + 2 (a u + b v) = 0
 *     (the projected-circle equation with D = 0, multiplied out; no division).
 *   - Sec. IV-A, Fig. 3(c): a 2D accumulator whose cell value is the number
 *     of circles that pass through the cell; the peak cell, back-projected
 *     (Eq. (8)), is the axis.
 *   - Sec. IV-B, Eq. (10) and Algorithm 1: with the axis fixed, every pair gives
 *     an angle; the angle is the peak of a histogram vote.
 *   - Sec. IV-C, Eq. (2): R by Rodrigues' formula.
 *   - Sec. IV-D: several peaks of the same accumulator give several rotations.
 *
 * Every floating-point step is the IEEE binary32 operation written in the
 * comment next to it (round to nearest even), built with -ffp-contract=off
 * and without -ffast-math, so that no multiply-add is fused and no step is
 * reordered.  Integer decisions (vote / no vote, bin index, argmax) are taken
 * in that same binary32 precision on both sides of the parity tests.
 *
 * Readings taken where the paper is silent (each one is listed in the design
 * notes with its justification):
 *   - x == p, y == q, and R maps p onto q (Eq. (1) vs Algorithm 1 naming).
 *   - d = p - q is used unnormalised: scaling d and flipping its sign leave the
 *     zero set of F, hence every vote, unchanged.
 *   - a cell gets at most one vote per correspondence (Fig. 3(c)), decided by
 *     the signs of F at its four corners: it is voted iff it meets the closed
 *     unit disk, some corner has F <= 0 and some corner has F >= 0.
 *   - ties in every argmax go to the lowest index.
 *   - several rotations (Sec. IV-D): the peaks are the accumulator's local
 *     maxima within the suppression radius, taken by decreasing votes; a cell
 *     within that radius of a peak already taken, or of its antipodal twin
 *     at the rim, is skipped.
 *   - the angle is signed, theta = atan2(r.(p x q), (r x p).(r x q)), binned
 *     over [-pi, pi) without transcendental functions: by comparison with a
 *     table of bin-boundary directions.
 *   - a correspondence whose displacement is zero or non-finite casts no axis
 *     vote; one whose (X, Y) is (0, 0) or non-finite casts no angle vote.
 *   - the literal sampling rule of Algorithm 1 (kept as a selectable
 *     alternative): the garbled sample expression is read as
 *     alpha1 cos(theta_j) + alpha2 sin(theta_j), alpha0 as the coordinate axis
 *     of z's smallest component, theta_j = -pi + j 2pi/J; only samples on the
 *     closed southern hemisphere vote, one vote per sample.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#if defined(__FAST_MATH__)
#error "the oracle must be built without -ffast-math"
#endif

#define OR_EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Displacement and the projected circle (Sec. III-A, Eq. (4); Sec. IV)      */
/* ------------------------------------------------------------------------ */

/* d = p - q componentwise; returns 1 if the correspondence casts votes. */
OR_EXPORT int or_displacement(const float* p, const float* q, float d[3]) {
    d[0] = p[0] - q[0];
    d[1] = p[1] - q[1];
    d[2] = p[2] - q[2];
    if (!isfinite(d[0]) || !isfinite(d[1]) || !isfinite(d[2])) return 0;
    if (d[0] == 0.0f && d[1] == 0.0f && d[2] == 0.0f) return 0;
    return 1;
}

/* Coarse-grid vertex coordinate u_j = -1 + j*h, h = 2/G (exact). */
OR_EXPORT float or_coarse_coord(int G, int j) {
    float h = 2.0f / (float)G;
    return -1.0f + (float)j * h;
}

/* W = u^2 + v^2 - 1 on a coarse vertex.  Exact there (G <= 4096), so the
 * evaluation order does not matter; written as ((u*u) + (v*v)) - 1. */
OR_EXPORT float or_W(float u, float v) {
    float uu = u * u;
    float vv = v * v;
    float s = uu + vv;
    return s - 1.0f;
}

/* F = (c*W) + 2*((a*u) + (b*v)), each operation rounded once. */
OR_EXPORT float or_F(float a, float b, float c, float u, float v, float W) {
    float cw = c * W;
    float au = a * u;
    float bv = b * v;
    float s = au + bv;
    float s2 = 2.0f * s;
    return cw + s2;
}

/* Hit rule on one cell given its four corner values of W and F. */
OR_EXPORT int or_cell_rule(const float W4[4], const float F4[4]) {
    float wmin = W4[0];
    for (int k = 1; k < 4; ++k) if (W4[k] < wmin) wmin = W4[k];
    if (!(wmin <= 0.0f)) return 0;
    int le = 0, ge = 0;
    for (int k = 0; k < 4; ++k) {
        if (F4[k] <= 0.0f) le = 1;
        if (F4[k] >= 0.0f) ge = 1;
    }
    return le && ge;
}

/* Does correspondence (p, q) vote for coarse cell (ix, iy) of a G x G grid? */
OR_EXPORT int or_coarse_hit(const float* p, const float* q, int G, int ix, int iy) {
    float d[3];
    if (!or_displacement(p, q, d)) return 0;
    float W4[4], F4[4];
    for (int k = 0; k < 4; ++k) {
        float u = or_coarse_coord(G, ix + (k & 1));
        float v = or_coarse_coord(G, iy + (k >> 1));
        W4[k] = or_W(u, v);
        F4[k] = or_F(d[0], d[1], d[2], u, v, W4[k]);
    }
    return or_cell_rule(W4, F4);
}

static void gather(const float* S, long n, long i, float out[3]) {
    out[0] = S[i];
    out[1] = S[n + i];
    out[2] = S[2 * n + i];
}

/* Full coarse accumulator by brute force over every cell (Sec. IV-A):
 * grid[iy*G + ix] = #{i : correspondence i votes for cell (ix, iy)}.
 * P, Q are SoA (3, n) float32. */
OR_EXPORT void or_coarse_grid(const float* P, const float* Q, long n, int G, uint32_t* grid) {
    long nv = (long)(G + 1) * (G + 1);
    float* W = (float*)malloc(sizeof(float) * nv);
    float* F = (float*)malloc(sizeof(float) * nv);
    for (int k = 0; k <= G; ++k)
        for (int j = 0; j <= G; ++j)
            W[(long)k * (G + 1) + j] = or_W(or_coarse_coord(G, j), or_coarse_coord(G, k));
    memset(grid, 0, sizeof(uint32_t) * (size_t)G * G);
    for (long i = 0; i < n; ++i) {
        float p[3], q[3], d[3];
        gather(P, n, i, p);
        gather(Q, n, i, q);
        if (!or_displacement(p, q, d)) continue;
        for (int k = 0; k <= G; ++k) {
            float v = or_coarse_coord(G, k);
            for (int j = 0; j <= G; ++j) {
                long o = (long)k * (G + 1) + j;
                F[o] = or_F(d[0], d[1], d[2], or_coarse_coord(G, j), v, W[o]);
            }
        }
        for (int iy = 0; iy < G; ++iy)
            for (int ix = 0; ix < G; ++ix) {
                long o = (long)iy * (G + 1) + ix;
                float W4[4] = {W[o], W[o + 1], W[o + G + 1], W[o + G + 2]};
                float F4[4] = {F[o], F[o + 1], F[o + G + 1], F[o + G + 2]};
                if (or_cell_rule(W4, F4)) grid[(long)iy * G + ix] += 1u;
            }
    }
    free(W);
    free(F);
}

/* One cell of the coarse accumulator, O(n): used to check sampled cells of a
 * grid too large for the brute-force pass. */
OR_EXPORT uint32_t or_coarse_cell(const float* P, const float* Q, long n, int G, int ix, int iy) {
    uint32_t cnt = 0;
    for (long i = 0; i < n; ++i) {
        float p[3], q[3];
        gather(P, n, i, p);
        gather(Q, n, i, q);
        cnt += (uint32_t)or_coarse_hit(p, q, G, ix, iy);
    }
    return cnt;
}

/* Angle-vote gate (coarse-to-fine angle voting, a variant of Sec. IV-B):
 * gate[i] = 1 iff correspondence i votes for at least one cell of the
 * (2w+1)^2 window of coarse cells centred on cell (px, py), clipped to the
 * grid (the per-cell rule of Sec. IV-A). */
OR_EXPORT void or_window_gate(const float* P, const float* Q, long n, int G, int px, int py, int w, uint8_t* gate) {
    int x0 = px - w < 0 ? 0 : px - w, x1 = px + w > G - 1 ? G - 1 : px + w;
    int y0 = py - w < 0 ? 0 : py - w, y1 = py + w > G - 1 ? G - 1 : py + w;
    for (long i = 0; i < n; ++i) {
        float p[3], q[3];
        gather(P, n, i, p);
        gather(Q, n, i, q);
        int g = 0;
        for (int iy = y0; iy <= y1 && !g; ++iy)
            for (int ix = x0; ix <= x1 && !g; ++ix) g = or_coarse_hit(p, q, G, ix, iy);
        gate[i] = (uint8_t)g;
    }
}

/* Number of coarse cells one correspondence votes for (brute force). */
OR_EXPORT long or_arc_votes(const float* p, const float* q, int G) {
    long cnt = 0;
    for (int iy = 0; iy < G; ++iy)
        for (int ix = 0; ix < G; ++ix) cnt += or_coarse_hit(p, q, G, ix, iy);
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* Literal sampling rule (Algorithm 1's inner loop; a selectable alternative */
/* to the per-cell rule above)                                              */
/* ------------------------------------------------------------------------ */

/* Sample directions theta_j = -pi + j*(2pi/J), j = 0..J-1 (Algorithm 1:
 * [-pi, pi] discretised uniformly; pi itself is -pi), cos and sin computed
 * in double and rounded once. */
OR_EXPORT void or_sample_dirs(int J, float* cs, float* sn) {
    double step = (2.0 * M_PI) / (double)J;
    for (int j = 0; j < J; ++j) {
        double th = -M_PI + (double)j * step;
        cs[j] = (float)cos(th);
        sn[j] = (float)sin(th);
    }
}

/* Orthonormal basis of the plane normal to z = (q - p)/|q - p| (Algorithm 1):
 * alpha0 = e_k with k = argmin |z_k| (lowest k on ties), alpha1 = alpha0 minus
 * its projection onto z, normalised, alpha2 = alpha1 x z.  Returns 0 (no
 * samples) when |q - p|^2 is zero, subnormal-underflowed or not finite. */
OR_EXPORT int or_sample_basis(const float* p, const float* q, float z[3], float a1[3], float a2[3]) {
    float d[3];
    d[0] = q[0] - p[0];
    d[1] = q[1] - p[1];
    d[2] = q[2] - p[2];
    float n2 = ((d[0] * d[0]) + (d[1] * d[1])) + (d[2] * d[2]);
    if (!(n2 > 0.0f) || !isfinite(n2)) return 0;
    float nz = sqrtf(n2);
    for (int k = 0; k < 3; ++k) z[k] = d[k] / nz;
    int k0 = 0;
    for (int k = 1; k < 3; ++k)
        if (fabsf(z[k]) < fabsf(z[k0])) k0 = k;
    /* alpha0 - (alpha0 . z) z with alpha0 = e_k0: alpha0 . z = z[k0] */
    float t[3];
    for (int k = 0; k < 3; ++k) {
        float e = (k == k0) ? 1.0f : 0.0f;
        float pz = z[k0] * z[k];
        t[k] = e - pz;
    }
    float m2 = ((t[0] * t[0]) + (t[1] * t[1])) + (t[2] * t[2]);
    float m = sqrtf(m2);
    for (int k = 0; k < 3; ++k) a1[k] = t[k] / m;
    /* alpha2 = alpha1 x z */
    a2[0] = (a1[1] * z[2]) - (a1[2] * z[1]);
    a2[1] = (a1[2] * z[0]) - (a1[0] * z[2]);
    a2[2] = (a1[0] * z[1]) - (a1[1] * z[0]);
    return 1;
}

/* Sample s = alpha1 cos(theta) + alpha2 sin(theta) on the great circle. */
OR_EXPORT void or_sample_point(const float a1[3], const float a2[3], float c, float s, float out[3]) {
    for (int k = 0; k < 3; ++k) {
        float x = a1[k] * c;
        float y = a2[k] * s;
        out[k] = x + y;
    }
}

/* Cell of a sample: only the closed southern hemisphere (s_z <= 0) votes
 * (its antipodes name the same axes); projection from the north pole,
 * (u, v) = (s_x, s_y) * (1 / (1 - s_z)) (Eq. (7)); cell index
 * floor((u + 1) * G/2), clamped to [0, G-1] (u = 1 lies on the last cell's
 * closed edge).  Returns -1 for a northern sample, else iy*G + ix. */
OR_EXPORT long or_sample_cell(const float s[3], int G) {
    if (!(s[2] <= 0.0f)) return -1;
    float den = 1.0f - s[2];
    float rinv = 1.0f / den;
    float u = s[0] * rinv;
    float v = s[1] * rinv;
    float hg = 0.5f * (float)G;
    float tu = (u + 1.0f) * hg;
    float tv = (v + 1.0f) * hg;
    long ix = (long)floorf(tu), iy = (long)floorf(tv);
    if (ix < 0) ix = 0;
    if (ix > G - 1) ix = G - 1;
    if (iy < 0) iy = 0;
    if (iy > G - 1) iy = G - 1;
    return iy * G + ix;
}

/* Coarse accumulator by the literal sampling rule: every sample of every
 * correspondence adds one vote to its cell (a circle can vote several times
 * for one cell).  grid is G*G, zeroed here. */
OR_EXPORT void or_sample_grid(const float* P, const float* Q, long n, int G, int J, uint32_t* grid) {
    float* cs = (float*)malloc(sizeof(float) * (size_t)J);
    float* sn = (float*)malloc(sizeof(float) * (size_t)J);
    or_sample_dirs(J, cs, sn);
    memset(grid, 0, sizeof(uint32_t) * (size_t)G * G);
    for (long i = 0; i < n; ++i) {
        float p[3], q[3], z[3], a1[3], a2[3];
        gather(P, n, i, p);
        gather(Q, n, i, q);
        if (!or_sample_basis(p, q, z, a1, a2)) continue;
        for (int j = 0; j < J; ++j) {
            float s[3];
            or_sample_point(a1, a2, cs[j], sn[j], s);
            long c = or_sample_cell(s, G);
            if (c >= 0) grid[c] += 1u;
        }
    }
    free(cs);
    free(sn);
}

/* ------------------------------------------------------------------------ */
/* Peak search (Algorithm 1: the accumulator's maximum cell)                */
/* ------------------------------------------------------------------------ */

/* Argmax, ties to the lowest index.  Returns the maximum value. */
OR_EXPORT uint32_t or_argmax(const uint32_t* a, long count, long* idx) {
    uint32_t best = 0;
    long bi = 0;
    for (long i = 0; i < count; ++i)
        if (a[i] > best) { best = a[i]; bi = i; }
    *idx = bi;
    return best;
}

/* ------------------------------------------------------------------------ */
/* Refinement window (64 x 64 fine grid over the 3 x 3 coarse cells around   */
/* the peak; a workload parameter, not a step of the paper)                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    float U0, V0, hx, hy;
    int ix_lo, iy_lo, nx, ny, M;
} or_window;

OR_EXPORT void or_fine_window(int G, int M, int w, int ix, int iy, or_window* win) {
    int x0 = ix - w < 0 ? 0 : ix - w;
    int x1 = ix + w > G - 1 ? G - 1 : ix + w;
    int y0 = iy - w < 0 ? 0 : iy - w;
    int y1 = iy + w > G - 1 ? G - 1 : iy + w;
    float h = 2.0f / (float)G;
    win->ix_lo = x0;
    win->iy_lo = y0;
    win->nx = x1 - x0 + 1;
    win->ny = y1 - y0 + 1;
    win->M = M;
    win->U0 = or_coarse_coord(G, x0);
    win->V0 = or_coarse_coord(G, y0);
    win->hx = ((float)win->nx * h) / (float)M;   /* exact: small int times 2^-k */
    win->hy = ((float)win->ny * h) / (float)M;
}

/* Fine vertex coordinate U0 + j*hx (exact: few significant bits). */
OR_EXPORT float or_fine_coord(float U0, float hx, int j) {
    float t = (float)j * hx;
    return U0 + t;
}

/* W' on a fine vertex: ((u*u) + (v*v)) - 1, each step rounded once. */
OR_EXPORT float or_W_fine(float u, float v) { return or_W(u, v); }

OR_EXPORT int or_fine_hit(const float* p, const float* q, const or_window* win, int jx, int jy) {
    float d[3];
    if (!or_displacement(p, q, d)) return 0;
    float W4[4], F4[4];
    for (int k = 0; k < 4; ++k) {
        float u = or_fine_coord(win->U0, win->hx, jx + (k & 1));
        float v = or_fine_coord(win->V0, win->hy, jy + (k >> 1));
        W4[k] = or_W_fine(u, v);
        F4[k] = or_F(d[0], d[1], d[2], u, v, W4[k]);
    }
    return or_cell_rule(W4, F4);
}

/* Fine accumulator (M x M) over all n correspondences, brute force. */
OR_EXPORT void or_fine_grid(const float* P, const float* Q, long n, const or_window* win, uint32_t* fine) {
    int M = win->M;
    memset(fine, 0, sizeof(uint32_t) * (size_t)M * M);
    for (long i = 0; i < n; ++i) {
        float p[3], q[3];
        gather(P, n, i, p);
        gather(Q, n, i, q);
        float d[3];
        if (!or_displacement(p, q, d)) continue;
        for (int jy = 0; jy < M; ++jy)
            for (int jx = 0; jx < M; ++jx)
                fine[(long)jy * M + jx] += (uint32_t)or_fine_hit(p, q, win, jx, jy);
    }
}

OR_EXPORT uint32_t or_fine_cell(const float* P, const float* Q, long n, const or_window* win, int jx, int jy) {
    uint32_t cnt = 0;
    for (long i = 0; i < n; ++i) {
        float p[3], q[3];
        gather(P, n, i, p);
        gather(Q, n, i, q);
        cnt += (uint32_t)or_fine_hit(p, q, win, jx, jy);
    }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* Axis: inverse stereographic projection of a cell centre (Eq. (8))        */
/* ------------------------------------------------------------------------ */

OR_EXPORT void or_axis(float u, float v, float r[3]) {
    float uu = u * u;
    float vv = v * v;
    float s = uu + vv;
    float den = 1.0f + s;
    float u2 = 2.0f * u;
    float v2 = 2.0f * v;
    float sm1 = s - 1.0f;
    r[0] = u2 / den;
    r[1] = v2 / den;
    r[2] = sm1 / den;
}

/* Centre of coarse cell (ix, iy): u = -1 + (ix + 1/2) h, exact. */
OR_EXPORT void or_coarse_center(int G, int ix, int iy, float* u, float* v) {
    float h = 2.0f / (float)G;
    *u = -1.0f + ((float)ix + 0.5f) * h;
    *v = -1.0f + ((float)iy + 0.5f) * h;
}

/* Centre of fine cell (jx, jy): U0 + (jx + 1/2) hx, exact. */
OR_EXPORT void or_fine_center(const or_window* win, int jx, int jy, float* u, float* v) {
    *u = win->U0 + ((float)jx + 0.5f) * win->hx;
    *v = win->V0 + ((float)jy + 0.5f) * win->hy;
}

/* ------------------------------------------------------------------------ */
/* Angle (Sec. IV-B, Eq. (10); Algorithm 1 angle loop)                       */
/* ------------------------------------------------------------------------ */

/* beta = r x p, gamma = r x q, X = beta . gamma, Y = r . (p x q). */
OR_EXPORT void or_angle_xy(const float r[3], const float p[3], const float q[3], float* X, float* Y) {
    float bx = (r[1] * p[2]) - (r[2] * p[1]);
    float by = (r[2] * p[0]) - (r[0] * p[2]);
    float bz = (r[0] * p[1]) - (r[1] * p[0]);
    float gx = (r[1] * q[2]) - (r[2] * q[1]);
    float gy = (r[2] * q[0]) - (r[0] * q[2]);
    float gz = (r[0] * q[1]) - (r[1] * q[0]);
    float xx = bx * gx;
    float xy = by * gy;
    float xz = bz * gz;
    *X = (xx + xy) + xz;
    float wx = (p[1] * q[2]) - (p[2] * q[1]);
    float wy = (p[2] * q[0]) - (p[0] * q[2]);
    float wz = (p[0] * q[1]) - (p[1] * q[0]);
    float yx = r[0] * wx;
    float yy = r[1] * wy;
    float yz = r[2] * wz;
    *Y = (yx + yy) + yz;
}

/* Bin boundaries phi_k = -pi + k*(2pi/B), k = 1..B-1, as float directions
 * (cos, sin) computed in double and rounded once.  Tc/Ts have B entries;
 * index 0 is unused (set to the direction of -pi). */
OR_EXPORT void or_angle_boundaries(int B, float* Tc, float* Ts) {
    double step = (2.0 * M_PI) / (double)B;
    for (int k = 0; k < B; ++k) {
        double phi = -M_PI + (double)k * step;
        Tc[k] = (float)cos(phi);
        Ts[k] = (float)sin(phi);
    }
}

/* Bin centres phi = -pi + (k + 1/2)*(2pi/B): angle, cos and sin, rounded once. */
OR_EXPORT void or_angle_centers(int B, float* th, float* ct, float* st) {
    double step = (2.0 * M_PI) / (double)B;
    for (int k = 0; k < B; ++k) {
        double phi = -M_PI + ((double)k + 0.5) * step;
        th[k] = (float)phi;
        ct[k] = (float)cos(phi);
        st[k] = (float)sin(phi);
    }
}

static int half_plane(float X, float Y) {
    if (Y < 0.0f) return 0;
    if (Y == 0.0f && X < 0.0f) return 0;
    return 1;
}

/* bin(X, Y) = number of boundaries k in [1, B-1] at or below the direction
 * (X, Y) in angular order over [-pi, pi).  Returns -1 for no vote. */
OR_EXPORT int or_angle_bin(const float* Tc, const float* Ts, int B, float X, float Y) {
    if (!isfinite(X) || !isfinite(Y)) return -1;
    if (X == 0.0f && Y == 0.0f) return -1;
    int hv = half_plane(X, Y);
    int cnt = 0;
    for (int k = 1; k < B; ++k) {
        int ht = half_plane(Tc[k], Ts[k]);
        int le;
        if (ht != hv) {
            le = ht < hv;
        } else {
            float t1 = Tc[k] * Y;
            float t2 = Ts[k] * X;
            le = (t1 - t2) >= 0.0f;
        }
        cnt += le;
    }
    return cnt;
}

/* Histogram of signed angles about axis r over all n correspondences. */
OR_EXPORT void or_angle_hist(const float* P, const float* Q, long n, const float r[3], int B, uint32_t* hist) {
    float* Tc = (float*)malloc(sizeof(float) * B);
    float* Ts = (float*)malloc(sizeof(float) * B);
    or_angle_boundaries(B, Tc, Ts);
    memset(hist, 0, sizeof(uint32_t) * (size_t)B);
    for (long i = 0; i < n; ++i) {
        float p[3], q[3], X, Y;
        gather(P, n, i, p);
        gather(Q, n, i, q);
        or_angle_xy(r, p, q, &X, &Y);
        int b = or_angle_bin(Tc, Ts, B, X, Y);
        if (b >= 0) hist[b] += 1u;
    }
    free(Tc);
    free(Ts);
}

/* ------------------------------------------------------------------------ */
/* Rotation recovery (Eq. (2), Sec. IV-C) and inlier set (Eq. (1))          */
/* ------------------------------------------------------------------------ */

/* R = I + sin(t) K + (1 - cos(t)) K^2, K = [r]x, row-major. */
OR_EXPORT void or_rotation(const float r[3], float ct, float st, float R[9]) {
    float K[9] = {0.0f, -r[2], r[1],
                  r[2], 0.0f, -r[0],
                  -r[1], r[0], 0.0f};
    float K2[9];
    for (int j = 0; j < 3; ++j)
        for (int l = 0; l < 3; ++l) {
            float t0 = K[j * 3 + 0] * K[0 * 3 + l];
            float t1 = K[j * 3 + 1] * K[1 * 3 + l];
            float t2 = K[j * 3 + 2] * K[2 * 3 + l];
            K2[j * 3 + l] = (t0 + t1) + t2;
        }
    float om = 1.0f - ct;
    for (int j = 0; j < 3; ++j)
        for (int l = 0; l < 3; ++l) {
            float delta = (j == l) ? 1.0f : 0.0f;
            float a = st * K[j * 3 + l];
            float b = om * K2[j * 3 + l];
            R[j * 3 + l] = (delta + a) + b;
        }
}

/* ||R p - q||^2 <= tau^2 for every correspondence; returns the count. */
OR_EXPORT long or_inliers(const float R[9], const float* P, const float* Q, long n, float tau, uint8_t* mask) {
    float tt = tau * tau;
    long cnt = 0;
    for (long i = 0; i < n; ++i) {
        float p[3], q[3], e[3];
        gather(P, n, i, p);
        gather(Q, n, i, q);
        for (int j = 0; j < 3; ++j) {
            float t0 = R[j * 3 + 0] * p[0];
            float t1 = R[j * 3 + 1] * p[1];
            float t2 = R[j * 3 + 2] * p[2];
            float s = (t0 + t1) + t2;
            e[j] = s - q[j];
        }
        float e0 = e[0] * e[0];
        float e1 = e[1] * e[1];
        float e2 = e[2] * e[2];
        float res2 = (e0 + e1) + e2;
        uint8_t m = (res2 <= tt) ? 1 : 0;
        if (mask) mask[i] = m;
        cnt += m;
    }
    return cnt;
}

/* Rotation error (experiments, Sec. V): arccos((tr(Rgt^T R) - 1) / 2) in
 * degrees, argument clamped to [-1, 1]. */
OR_EXPORT double or_rotation_error_deg(const double Rgt[9], const float R[9]) {
    double tr = 0.0;
    for (int j = 0; j < 3; ++j)
        for (int l = 0; l < 3; ++l) tr += Rgt[l * 3 + j] * (double)R[l * 3 + j];
    double c = 0.5 * (tr - 1.0);
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    return acos(c) * 180.0 / M_PI;
}

/* ------------------------------------------------------------------------ */
/* Top-k peak selection with suppression (Sec. IV-D, multi-model)           */
/* ------------------------------------------------------------------------ */

/* Is coarse cell (ix, iy) suppressed by peak (px, py)?  Integer disk of
 * radius rad cells around the peak, plus the disk of radius rad*h around the
 * projection of the antipodal axis, -(u, v)/(u^2 + v^2). */
OR_EXPORT int or_suppressed(int G, int rad, int px, int py, int ix, int iy) {
    long dx = ix - px, dy = iy - py;
    if (dx * dx + dy * dy <= (long)rad * rad) return 1;
    float pu, pv, cu, cv;
    or_coarse_center(G, px, py, &pu, &pv);
    or_coarse_center(G, ix, iy, &cu, &cv);
    float s = (pu * pu) + (pv * pv);
    float au = (-pu) / s;
    float av = (-pv) / s;
    float du = cu - au;
    float dv = cv - av;
    float d2 = (du * du) + (dv * dv);
    float h = 2.0f / (float)G;
    float rh = (float)rad * h;
    float rr = rh * rh;
    return d2 <= rr;
}

/* Is coarse cell (ix, iy) a local maximum of the accumulator within the
 * integer disk of radius rad?  Every other cell of the grid in that disk must
 * hold fewer votes, or as many at a higher linear index (the tie-break of the
 * argmax).  This is what non-maximum suppression means for peak detection: the
 * flank of a strong peak is never a peak of its own, however far from the
 * summit the flank reaches. */
OR_EXPORT int or_local_max(const uint32_t* grid, int G, int rad, int ix, int iy) {
    long c = (long)iy * G + ix;
    for (int dy = -rad; dy <= rad; ++dy) {
        for (int dx = -rad; dx <= rad; ++dx) {
            if (dx == 0 && dy == 0) continue;
            if ((long)dx * dx + (long)dy * dy > (long)rad * rad) continue;
            int jx = ix + dx, jy = iy + dy;
            if (jx < 0 || jx >= G || jy < 0 || jy >= G) continue;
            long o = (long)jy * G + jx;
            if (grid[o] > grid[c]) return 0;
            if (grid[o] == grid[c] && o < c) return 0;
        }
    }
    return 1;
}

/* Top-k over the coarse grid (Sec. IV-D): in order of decreasing votes (ties to
 * the lowest index), the cells with at least one vote that are local maxima
 * within radius rad and are not suppressed by a peak already taken (its disk,
 * or the disk around its antipodal twin at the rim).  Returns the number of
 * peaks found. */
OR_EXPORT int or_topk_peaks(const uint32_t* grid, int G, int k, int rad, long* peaks, uint32_t* votes) {
    int found = 0;
    for (int t = 0; t < k; ++t) {
        uint32_t best = 0;
        long bi = -1;
        for (long c = 0; c < (long)G * G; ++c) {
            int ix = (int)(c % G), iy = (int)(c / G);
            if (grid[c] <= best) continue;
            if (!or_local_max(grid, G, rad, ix, iy)) continue;
            int sup = 0;
            for (int s = 0; s < found && !sup; ++s)
                sup = or_suppressed(G, rad, (int)(peaks[s] % G), (int)(peaks[s] / G), ix, iy);
            if (sup) continue;
            best = grid[c];
            bi = c;
        }
        if (bi < 0 || best == 0) break;
        peaks[found] = bi;
        votes[found] = best;
        ++found;
    }
    return found;
}

/* ------------------------------------------------------------------------ */
/* Whole solve                                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    float R[9];
    float axis[3];
    float angle;
    uint32_t grid, peak_cell, fine_cell, angle_bin;
    uint32_t axis_votes, fine_votes, angle_votes, n_inliers;
} or_result;

/* Steps after the coarse peak for one peak cell: refinement, axis, angle
 * histogram, Rodrigues, inliers.  fine/hist are caller-provided scratch. */
OR_EXPORT void or_finish_peak(const float* P, const float* Q, long n, int G, int M, int w, int B, float tau,
                              long peak, uint32_t peak_votes, or_result* res, uint8_t* mask,
                              uint32_t* fine_out, uint32_t* hist_out) {
    int ix = (int)(peak % G), iy = (int)(peak / G);
    float u, v;
    res->grid = (uint32_t)G;
    res->peak_cell = (uint32_t)peak;
    res->axis_votes = peak_votes;
    if (M > 0) {
        or_window win;
        or_fine_window(G, M, w, ix, iy, &win);
        uint32_t* fine = fine_out ? fine_out : (uint32_t*)malloc(sizeof(uint32_t) * (size_t)M * M);
        or_fine_grid(P, Q, n, &win, fine);
        long fi;
        res->fine_votes = or_argmax(fine, (long)M * M, &fi);
        res->fine_cell = (uint32_t)fi;
        or_fine_center(&win, (int)(fi % M), (int)(fi / M), &u, &v);
        if (!fine_out) free(fine);
    } else {
        res->fine_votes = 0;
        res->fine_cell = 0;
        or_coarse_center(G, ix, iy, &u, &v);
    }
    or_axis(u, v, res->axis);
    uint32_t* hist = hist_out ? hist_out : (uint32_t*)malloc(sizeof(uint32_t) * (size_t)B);
    or_angle_hist(P, Q, n, res->axis, B, hist);
    long bi;
    res->angle_votes = or_argmax(hist, B, &bi);
    res->angle_bin = (uint32_t)bi;
    if (!hist_out) free(hist);
    float* th = (float*)malloc(sizeof(float) * B);
    float* ct = (float*)malloc(sizeof(float) * B);
    float* st = (float*)malloc(sizeof(float) * B);
    or_angle_centers(B, th, ct, st);
    res->angle = th[bi];
    or_rotation(res->axis, ct[bi], st[bi], res->R);
    free(th);
    free(ct);
    free(st);
    res->n_inliers = (uint32_t)or_inliers(res->R, P, Q, n, tau, mask);
}

static void identity_result(or_result* res, int G) {
    memset(res, 0, sizeof(*res));
    res->R[0] = res->R[4] = res->R[8] = 1.0f;
    res->grid = (uint32_t)G;
}

/* Single rotation.  Returns 0 on success, -4 (no data) if n < 2 or the grid
 * is empty.  grid_out (G*G), fine_out (M*M), hist_out (B) may be NULL. */
OR_EXPORT int or_solve(const float* P, const float* Q, long n, int G, int M, int w, int B, float tau,
                       or_result* res, uint8_t* mask, uint32_t* grid_out, uint32_t* fine_out, uint32_t* hist_out) {
    identity_result(res, G);
    if (n < 2) return -4;
    uint32_t* grid = grid_out ? grid_out : (uint32_t*)malloc(sizeof(uint32_t) * (size_t)G * G);
    or_coarse_grid(P, Q, n, G, grid);
    long peak;
    uint32_t pv = or_argmax(grid, (long)G * G, &peak);
    if (!grid_out) free(grid);
    if (pv == 0) return -4;
    or_finish_peak(P, Q, n, G, M, w, B, tau, peak, pv, res, mask, fine_out, hist_out);
    return 0;
}

/* Several rotations: greedy top-k with suppression, then one full finish per
 * peak.  masks is k*n bytes or NULL.  Returns the number found. */
OR_EXPORT int or_solve_topk(const float* P, const float* Q, long n, int G, int M, int w, int B, float tau,
                            int k, int rad, or_result* res, uint8_t* masks) {
    for (int t = 0; t < k; ++t) identity_result(&res[t], G);
    if (n < 2) return 0;
    uint32_t* grid = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)G * G);
    or_coarse_grid(P, Q, n, G, grid);
    long* peaks = (long*)malloc(sizeof(long) * (size_t)k);
    uint32_t* votes = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)k);
    int found = or_topk_peaks(grid, G, k, rad, peaks, votes);
    for (int t = 0; t < found; ++t)
        or_finish_peak(P, Q, n, G, M, w, B, tau, peaks[t], votes[t], &res[t],
                       masks ? masks + (size_t)t * n : NULL, NULL, NULL);
    free(grid);
    free(peaks);
    free(votes);
    return found;
}
