// Host build of the library's octant pieces and line walks (walker.h), for
// CPU tests: the coarse and refinement accumulators are rebuilt here with the
// same pieces, band split and walks as the kernels, but cells are counted in
// host memory.  A walk emitter with kAudit set also checks, on every line of
// the certified walk's clean path, the two vertex signs that the certificates
// vouch for.  Test code only: nothing in the library calls this file.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../paper_2502_06337_amd/csrc/walker.h"

using namespace aoresp;

namespace {

struct Audit {
    long long steps = 0, violations = 0;
};

// In-disk cross range of every coarse line (cells whose closest corner lies
// in the closed unit disk), in integer arithmetic.
std::vector<int16_t> disk_ranges(int G) {
    std::vector<int16_t> h(2 * (size_t)G);
    auto nearest = [G](int j) {
        long a = labs(2L * j - G), b = labs(2L * j + 2 - G);
        return a < b ? a : b;
    };
    const long GG = (long)G * G;
    for (int j = 0; j < G; ++j) {
        const long mu = nearest(j);
        int lo = G, hi = -1;
        for (int k = 0; k < G; ++k) {
            const long mv = nearest(k);
            if (mu * mu + mv * mv <= GG) {
                if (k < lo) lo = k;
                hi = k;
            }
        }
        h[2 * j] = (int16_t)lo;
        h[2 * j + 1] = (int16_t)hi;
    }
    return h;
}

struct CoarseHostEmit {
    static constexpr bool kAudit = true;
    static constexpr bool kPairedLines = true;   // the line-pair loop of the coarse kernel
    uint32_t* grid;
    const int16_t* disk;
    int mode, G, clo, chi;
    Audit* counts;
    int offs = 0;
    void operator()(int j, int klo, int khi) {
        klo = klo < disk[2 * j] ? disk[2 * j] : klo;
        khi = khi > disk[2 * j + 1] ? disk[2 * j + 1] : khi;
        klo = klo < clo ? clo : klo;
        khi = khi > chi ? chi : khi;
        for (int k = klo; k <= khi; ++k) grid[mode == 0 ? (size_t)k * G + j : (size_t)j * G + k] += 1;
    }
    // A cell of a clean line: the kernel writes it without a bound check, into
    // its tile's pad words when it lies outside the grid.  A cell beyond the
    // column bound of a row quarter, or farther out than the pads reach, is
    // counted as the kernel would count it and recorded as a violation.
    void clean_cell(int j, int k) {
        const bool lo_ok = clo > 0 ? k >= clo : k >= -kTilePad;
        const bool hi_ok = chi < G - 1 ? k <= chi : k <= G - 1 + kTilePad;
        if (!lo_ok || !hi_ok) counts->violations++;
        if (k < 0 || k >= G || k < disk[2 * j] || k > disk[2 * j + 1]) return;
        grid[mode == 0 ? (size_t)k * G + j : (size_t)j * G + k] += 1;
    }
    // rows are line pairs: the row handle is the even line
    int row_start(int j, int off) {
        offs = off;
        return j & ~1;
    }
    int next_row(int row) const { return row + 2; }
    int rows_after(int row, int n) const { return row + 2 * n; }
    template <int H>
    void range_h(int row, int klo, int khi) { (*this)(row + H, klo, khi); }
    template <int H>
    void pair_h(int row, int r, bool second) {
        clean_cell(row + H, r - 1 + offs);
        if (second) clean_cell(row + H, r - offs);
    }
    // a cell handle: row and cross index
    struct Cell {
        int row, r;
    };
    static Cell cell_of(int row, int r) { return {row, r}; }
    static int index_of(int row, Cell c) { return c.r; }
    static Cell next_cell(Cell c) { return {c.row + 2, c.r}; }
    Cell pair2(Cell c, bool up0, bool up1) {
        const int r0 = c.r, r1 = r0 + (up0 ? 1 : 0) - offs, r2 = r1 + (up1 ? 1 : 0) - offs;
        clean_cell(c.row, r0 - 1 + offs);
        if (up0 != (offs != 0)) clean_cell(c.row, r1 - 1 + offs);
        clean_cell(c.row + 1, r1 - 1 + offs);
        if (up1 != (offs != 0)) clean_cell(c.row + 1, r2 - 1 + offs);
        return {c.row, r2};
    }
    void audit(float below, float above) {
        counts->steps++;
        if (!(below > 0.0f)) counts->violations++;
        if (!(above < 0.0f)) counts->violations++;
    }
};

struct FineHostEmit {
    static constexpr bool kAudit = true;
    static constexpr bool kPairedLines = false;
    uint32_t* tile;
    int mode, M;
    float U0, V0, hx, hy;
    int clo, chi;
    Audit* counts;
    int offs = 0;
    bool in_disk(int jx, int jy) const {
        const float u0 = U0 + (float)jx * hx, u1 = U0 + (float)(jx + 1) * hx;
        const float v0 = V0 + (float)jy * hy, v1 = V0 + (float)(jy + 1) * hy;
        const float w00 = ((u0 * u0) + (v0 * v0)) - 1.0f, w10 = ((u1 * u1) + (v0 * v0)) - 1.0f;
        const float w01 = ((u0 * u0) + (v1 * v1)) - 1.0f, w11 = ((u1 * u1) + (v1 * v1)) - 1.0f;
        return (w00 <= 0.0f) | (w10 <= 0.0f) | (w01 <= 0.0f) | (w11 <= 0.0f);
    }
    void operator()(int j, int klo, int khi) {
        klo = klo < clo ? clo : klo;
        khi = khi > chi ? chi : khi;
        klo = klo < 0 ? 0 : klo;
        khi = khi > M - 1 ? M - 1 : khi;
        for (int k = klo; k <= khi; ++k) {
            const int jx = mode == 0 ? j : k, jy = mode == 0 ? k : j;
            if (in_disk(jx, jy)) tile[jy * M + jx] += 1;
        }
    }
    int start(int j, int off) {
        offs = off;
        return j;
    }
    int next(int j) const { return j + 1; }
    void pair(int j, int r, bool second) {
        (*this)(j, r - 1 + offs, r - 1 + offs);
        if (second) (*this)(j, r - offs, r - offs);
    }
    void audit(float below, float above) {
        counts->steps++;
        if (!(below > 0.0f)) counts->violations++;
        if (!(above < 0.0f)) counts->violations++;
    }
};

// Displacement of correspondence i with c >= 0, and its flags.
uint32_t displacement(const float* P, const float* Q, long n, long i, float& a, float& b, float& c) {
    a = P[i] - Q[i];
    b = P[n + i] - Q[n + i];
    c = P[2 * n + i] - Q[2 * n + i];
    const uint32_t fl = classify(a, b, c);
    if (!(fl & kFlagDegenerate) && c < 0.0f) {
        a = -a;
        b = -b;
        c = -c;
    }
    return fl;
}

}  // namespace

extern "C" {

// Coarse G x G grid of n correspondences (P, Q: (3, n) float32 SoA), grid
// zeroed by the caller.  audit_out[0..1] = clean lines audited, violations.
// Returns the walks' internal-check flags (0 when every walk was consistent).
int hw_coarse_grid(const float* P, const float* Q, long n, int G, uint32_t* grid, long long* audit_out) {
    const std::vector<int16_t> disk = disk_ranges(G);
    const float h = 2.0f / (float)G;
    const int bw = coarse_band_width(G);
    uint32_t bad = 0;
    Audit audit;
    for (long i = 0; i < n; ++i) {
        float a, b, c;
        const uint32_t fl = displacement(P, Q, n, i, a, b, c);
        if (fl & kFlagDegenerate) continue;
        if (fl & kFlagRisky) {
            // outside the walk's range of validity: every cell's corners
            for (int k = 0; k < G; ++k)
                for (int j = 0; j < G; ++j) {
                    if (k < disk[2 * j] || k > disk[2 * j + 1]) continue;
                    const float u0 = -1.0f + (float)j * h, u1 = -1.0f + (float)(j + 1) * h;
                    const float v0 = -1.0f + (float)k * h, v1 = -1.0f + (float)(k + 1) * h;
                    const float f0 = vertex_F(b, c, u0 * u0, a * u0, v0), f1 = vertex_F(b, c, u1 * u1, a * u1, v0);
                    const float f2 = vertex_F(b, c, u0 * u0, a * u0, v1), f3 = vertex_F(b, c, u1 * u1, a * u1, v1);
                    const bool le = (f0 <= 0.0f) | (f1 <= 0.0f) | (f2 <= 0.0f) | (f3 <= 0.0f);
                    const bool ge = (f0 >= 0.0f) | (f1 >= 0.0f) | (f2 >= 0.0f) | (f3 >= 0.0f);
                    if (le && ge) grid[(size_t)k * G + j] += 1;
                }
            continue;
        }
        int4 colp, rowp, geo;
        const double hd = 2.0 / G;
        circle_pieces<true>(a, b, c, fl, -1.0, hd, G, -1.0, hd, G, 2.0 * hd, colp, rowp, geo);
        const int32_t ranges[2][4] = {{colp.x, colp.y, colp.z, colp.w}, {rowp.x, rowp.y, rowp.z, rowp.w}};
        int ja, jb;
        unpack_range(geo.x, ja, jb);
        const float T = cert_threshold(a, b, c);
        for (int mode = 0; mode < 2; ++mode)
            for (int p = 0; p < 4; ++p) {
                int s, e;
                unpack_range(ranges[mode][p], s, e);
                if (s >= e) continue;
                CoarseHostEmit em{grid, disk.data(), mode, G, 0, G - 1, &audit};
                if (mode == 1) {
                    if ((p >> 1) == 0) em.chi = ja - 1; else em.clo = jb;
                }
                const float aL = mode == 0 ? a : b, bL = mode == 0 ? b : a;
                int dir, slo, shi;
                octant_walk_info(mode, p, geo, dir, slo, shi, kCoarseRowShrink);
                for (int b0 = 0; b0 < G; b0 += bw) {
                    const int cs = s > b0 ? s : b0, ce = e < b0 + bw ? e : b0 + bw;
                    if (cs >= ce) continue;
                    int2 parts[3];
                    split_piece(cs, ce, slo, shi, parts);
                    for (int q = 0; q < 3; ++q) {
                        if (parts[q].x >= parts[q].y) continue;
                        if (q == 1)
                            walk_certified<true>(aL, bL, c, p >> 1, dir, T, -1.0f, h, -1.0f, h, parts[q].x, parts[q].y,
                                                 em, bad);
                        else
                            walk_search(aL, bL, c, p >> 1, -1.0f, h, -1.0f, h, parts[q].x, parts[q].y, em, bad);
                    }
                }
            }
    }
    if (audit_out) {
        audit_out[0] = audit.steps;
        audit_out[1] = audit.violations;
    }
    return (int)bad;
}

// Refinement grid (M x M cells of the window U0 + jx hx, V0 + jy hy) of n
// correspondences; fine zeroed by the caller.  Same outputs as above.
int hw_fine_grid(const float* P, const float* Q, long n, float U0, float V0, float hx, float hy, int M, uint32_t* fine,
                 long long* audit_out) {
    uint32_t bad = 0;
    Audit audit;
    for (long i = 0; i < n; ++i) {
        float a, b, c;
        const uint32_t fl = displacement(P, Q, n, i, a, b, c);
        if (fl & (kFlagDegenerate | kFlagRisky)) continue;
        int4 colp, rowp, geo;
        circle_pieces<false>(a, b, c, fl, U0, hx, M, V0, hy, M, 2.0 * (double)(hx > hy ? hx : hy), colp, rowp, geo);
        const int32_t ranges[2][4] = {{colp.x, colp.y, colp.z, colp.w}, {rowp.x, rowp.y, rowp.z, rowp.w}};
        int ja, jb;
        unpack_range(geo.x, ja, jb);
        const float T = kFineCertScale * cert_threshold(a, b, c);
        for (int mode = 0; mode < 2; ++mode)
            for (int p = 0; p < 4; ++p) {
                int s, e;
                unpack_range(ranges[mode][p], s, e);
                if (s >= e) continue;
                FineHostEmit em{fine, mode, M, U0, V0, hx, hy, -(1 << 20), 1 << 20, &audit};
                if (mode == 1) {
                    if ((p >> 1) == 0) em.chi = ja - 1; else em.clo = jb;
                }
                const float aL = mode == 0 ? a : b, bL = mode == 0 ? b : a;
                const float x0 = mode == 0 ? U0 : V0, hxl = mode == 0 ? hx : hy;
                const float y0 = mode == 0 ? V0 : U0, hyl = mode == 0 ? hy : hx;
                int dir, slo, shi;
                octant_walk_info(mode, p, geo, dir, slo, shi);
                int2 parts[3];
                split_piece(s, e, slo, shi, parts);
                for (int q = 0; q < 3; ++q) {
                    if (parts[q].x >= parts[q].y) continue;
                    if (q == 1)
                        walk_certified(aL, bL, c, p >> 1, dir, T, x0, hxl, y0, hyl, parts[q].x, parts[q].y, em, bad);
                    else
                        walk_search(aL, bL, c, p >> 1, x0, hxl, y0, hyl, parts[q].x, parts[q].y, em, bad);
                }
            }
    }
    if (audit_out) {
        audit_out[0] = audit.steps;
        audit_out[1] = audit.violations;
    }
    return (int)bad;
}

// Least-squares rotation from the sums S[3a + b] = sum p_a q_b (the library's
// quaternion solve, host build).
void hw_ls_rotation(const double* S, float* R) { ls_rotation_from_sums(S, R); }

}  // extern "C"
