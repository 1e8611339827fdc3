// HIP kernels of the stereographic-projection rotation vote (gfx950).
//
// Pipeline (paper: Algorithm 1; Sec. IV), every kernel over a batch of
// instances (a single solve is a batch of one):
//   k_arc_setup      per correspondence: displacement, octant pieces
//   k_vote           coarse accumulator: column pass over vertical LDS bands
//                    and row pass over horizontal LDS bands, persistent
//                    work-groups pulling (instance, band, chunk) items
//                    (Sec. IV-A, Fig. 3(c))
//   k_sample_setup / k_sample_vote / k_sample_reduce
//                    alternative coarse accumulator by the literal sampling
//                    loop of Algorithm 1: per-circle records, LDS band tiles,
//                    sum of the per-chunk partial tiles
//   k_local_max      multi-model estimation (Sec. IV-D): bitmap of the cells
//                    that are local maxima within the suppression radius
//   k_peak           argmax (ties to the lowest index); later peaks of a
//                    multi-model instance must be local maxima and not
//                    suppressed by an earlier peak
//   k_fine_vote      refinement accumulator around each peak
//   k_fine_peak      refined cell, inverse projection to the axis (Eq. (8))
//   k_angle_hist     signed angle of every pair about the axis, binned
//                    (Sec. IV-B, Eq. (10)); optionally only the pairs whose
//                    curve crosses the peak's window of coarse cells
//   k_angle_peak     histogram peak, Rodrigues rotation (Eq. (2))
//   k_angle_fine_hist / k_angle_fine_peak
//                    optional B*F-bin histogram read on the three coarse bins
//                    around the angle peak; its argmax replaces the angle
//   k_inliers        residual mask against Eq. (1)
//   k_ls_accum       float64 sums of p q^T over the inliers, per item
//   k_ls_finish      least-squares rotation on the inlier set (quaternion
//                    method; a refinement after Eq. (1), not in the paper)
// Nothing here is a dense contraction: the vote kernels are bound by VALU
// work per vote and LDS atomics, the rest by HBM streaming.
#include <hip/hip_runtime.h>
#include <math.h>

#include <cmath>
#include <stdint.h>

#include "geometry.h"
#include "kernels.h"
#include "walker.h"

namespace aoresp {

__device__ __forceinline__ int find_inst(const Inst* insts, int ninst, int64_t col) {
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (insts[mid].off <= col) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// --------------------------------------------------------------------------
// Per-correspondence setup
// --------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_arc_setup(const float* __restrict__ P, const float* __restrict__ Q,
                                                   int64_t N, const Inst* __restrict__ insts, int ninst,
                                                   ArcRecs R) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int G = insts[find_inst(insts, ninst, i)].G;
    float a = P[i] - Q[i];
    float b = P[N + i] - Q[N + i];
    float c = P[2 * N + i] - Q[2 * N + i];
    uint32_t fl = classify(a, b, c);
    if (!(fl & kFlagDegenerate) && c < 0.0f) {
        a = -a;
        b = -b;
        c = -c;
    }
    const int E = pack_range(0, 0);
    int4 colp = make_int4(E, E, E, E), rowp = colp;
    int4 geo = make_int4(0, 0, 0, (int)fl);
    if (fl & kFlagRisky) {
        colp.x = kRiskyMark;
    } else if (!(fl & kFlagDegenerate)) {
        double h = 2.0 / G;
        circle_pieces<true>(a, b, c, fl, -1.0, h, G, -1.0, h, G, 2.0 * h, colp, rowp, geo);
    }
    R.abc[i] = make_float4(a, b, c, cert_threshold(a, b, c));
    R.colp[i] = colp;
    R.rowp[i] = rowp;
    R.geo[i] = geo;
}

// --------------------------------------------------------------------------
// Coarse accumulator: banded LDS tiles, persistent work-groups
// --------------------------------------------------------------------------

// Set bits of a wave mask in the lanes below this one.
__device__ __forceinline__ int lanes_below(unsigned long long m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Cells of a band tile: 16-bit counters, the cells (j, k) and (j + 1, k) of
// an even/odd line pair in the low and high half of one word, word rows of
// Sw = G + kTilePad words per line pair (pair m, cross k at word kTilePad +
// m * Sw + k).  Sw is odd, so the lanes of a wave (different curves, mostly on
// the same line) hit spread-out banks and the column pass's flush, which reads
// across lines, is conflict-free.  The kTilePad words between rows take the
// cells that a clean line counts outside the frame, so the clean path writes
// without a bound check: a certified body's octant is clipped to the frame
// plus two cells and a line, and its crossing moves by at most one cell per
// line, so its cells have cross indices -4 .. G + 4; in the row pass its
// lines also stop short of the columns owned by the column quarters
// (kCoarseRowShrink).  Pads are never flushed, and cells outside the disk are
// counted here and dropped at the flush.
struct CoarseEmit {
    static constexpr bool kAudit = false;
    static constexpr bool kPairedLines = true;
    uint32_t* tile;        // cross index 0 of the band's first line pair
    int jofs, sw;          // sw = G + kTilePad words per line pair, jofs = -(band0 / 2) * sw
    int clo, chi;          // allowed cross indices of a general range (callers skip a walk when chi < clo)
    int db = 0;            // second cell of a clean line relative to its first: 1 - 2 off
    int sh = 0;            // cell k of a row handle at handle[k + sh]: 1 - off
    uint32_t d_up = 0, d_dn = 0, e_up = 0, e_dn = 0;   // pair2's increments by each line's step
    int du = 0, dd = 0;    // pair2's cell moves (1 - off up, -off down)
    __device__ __forceinline__ uint32_t* row_of(int j) const { return tile + ((int)__umul24(j >> 1, sw) + jofs); }
    __device__ __forceinline__ static uint32_t inc_of(int j) { return 1u << ((j & 1) << 4); }
    __device__ __forceinline__ void operator()(int j, int klo, int khi) {
        uint32_t* row = row_of(j);
        const uint32_t inc = inc_of(j);
        klo = max(klo, clo);
        khi = min(khi, chi);
#pragma unroll 1
        for (int k = klo; k <= khi; ++k) atomicAdd(row + k, inc);
    }
    // word row of line j's pair, shifted so that row[r] is cell r - 1 + off
    __device__ __forceinline__ uint32_t* row_start(int j, int off) {
        db = 1 - 2 * off;
        sh = 1 - off;
        d_up = off ? 0x10000u : 0x10001u;
        d_dn = off ? 0x10001u : 0x10000u;
        e_up = off ? 0u : 0x10000u;
        e_dn = off ? 0x10000u : 0u;
        du = 1 - off;
        dd = -off;
        return row_of(j) + (off - 1);
    }
    // a cell handle (the word of cell r of a row handle) and its index
    __device__ __forceinline__ static uint32_t* cell_of(uint32_t* row, int r) { return row + r; }
    __device__ __forceinline__ static int index_of(uint32_t* row, uint32_t* cell) { return (int)(cell - row); }
    __device__ __forceinline__ uint32_t* next_cell(uint32_t* cell) const { return cell + sw; }
    __device__ __forceinline__ uint32_t* next_row(uint32_t* row) const { return row + sw; }
    __device__ __forceinline__ uint32_t* rows_after(uint32_t* row, int n) const { return row + n * sw; }
    // a general range of the line with parity H
    template <int H>
    __device__ __forceinline__ void range_h(uint32_t* row, int klo, int khi) const {
        constexpr uint32_t inc = 1u << (16 * H);
        uint32_t* base = row + sh;
        klo = max(klo, clo);
        khi = min(khi, chi);
#pragma unroll 1
        for (int k = klo; k <= khi; ++k) atomicAdd(base + k, inc);
    }
    // cells r - 1 + off and, if second, r - off of the line with parity H
    // (low half of the word for H = 0, high half for H = 1)
    template <int H>
    __device__ __forceinline__ void pair_h(uint32_t* row, int r, bool second) const {
        constexpr uint32_t inc = 1u << (16 * H);
        atomicAdd(row + r, inc);
        atomicAdd(row + r + db, second ? inc : 0u);
    }
    // both lines of the row from the cell handle of r0 -> r1 -> r2 (r1 = r0 +
    // (up0 ? 1 : 0) - off, r2 likewise): the line 2m + 1 cell r1 - 1 + off
    // shares its word with line 2m's second cell, if any; returns r2's handle
    __device__ __forceinline__ uint32_t* pair2(uint32_t* c0, bool up0, bool up1) const {
        uint32_t* c1 = c0 + (up0 ? du : dd);
        uint32_t* c2 = c1 + (up1 ? du : dd);
        atomicAdd(c0, 1u);
        atomicAdd(c1, up0 ? d_up : d_dn);
        atomicAdd(c2, up1 ? e_up : e_dn);
        return c2;
    }
};

// One work-group per item (instance, pass, band, correspondence range).  The
// band tile is zeroed, then every wave works on its own: it takes groups of
// 64 correspondences, appends the parts of each octant that fall in the band
// to two per-wave rings in LDS (certified bodies, searched lines), and walks
// 64 parts at a time whenever a ring holds a full round, so there is no
// block-wide barrier between listing and walking.  At the end the rings are
// drained, and the tile is flushed (disk mask applied) with global atomics.
__global__ __launch_bounds__(kVoteThreads) void k_vote(const ArcRecs R, const Inst* __restrict__ insts,
                                                       const int4* __restrict__ items, const VoteQueues vq,
                                                       uint32_t* __restrict__ counters,
                                                       uint32_t* __restrict__ grid_arena,
                                                       uint32_t* __restrict__ err) {
    constexpr int kWaves = kVoteThreads / 64;
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ int item_id;
    __shared__ int group_next;   // next unclaimed group of 64 correspondences
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    uint32_t* tile = smem + kTilePad;
    uint32_t* rbody = smem + kTileWords + wid * (kRingBody + kRingLine);
    uint32_t* rline = rbody + kRingBody;
    int16_t* dlim = reinterpret_cast<int16_t*>(smem + kTileWords + kWaves * (kRingBody + kRingLine));
    uint32_t bad = 0;

    // the queue of this work-group's XCD first; its chunks' records stay in
    // that XCD's L2 while the work-groups there take the chunks' bands
    const int home = (int)(blockIdx.x % kVoteQueues);
    int q_left = (1 << kVoteQueues) - 1;   // thread 0: queues not yet found empty
    for (;;) {
        if (tid == 0) {
            int got = -1;
            for (int k = 0; k < kVoteQueues && got < 0; ++k) {
                const int q = (home + k) & (kVoteQueues - 1);
                if (!((q_left >> q) & 1)) continue;
                const int len = vq.first[q + 1] - vq.first[q];
                const int t = len > 0 ? (int)atomicAdd(&counters[q], 1u) : len;
                if (t < len) got = vq.first[q] + t;
                else q_left &= ~(1 << q);
            }
            item_id = got;
            group_next = kWaves * 64;
        }
        __syncthreads();
        const int it = item_id;
        if (it < 0) break;
        const int4 wi = items[it];
        const Inst& I = insts[wi.x];
        const int G = I.G;
        const int mode = wi.y & 1;
        const int band = wi.y >> 1;
        const int bw = I.bw;
        const int band0 = band * bw;
        const int bwb = (band0 + bw <= G) ? bw : (G - band0);
        const int Sw = G + kTilePad;         // words per line pair
        const int tile_words = kTilePad + (bwb >> 1) * Sw;
        const int lbw = 31 - __clz(bwb), lg = 31 - __clz(G);   // both powers of two
        const float h = 2.0f / (float)G;
        for (int t = tid; t < tile_words; t += kVoteThreads) smem[t] = 0u;
        for (int t = tid; t < bwb; t += kVoteThreads) {
            dlim[2 * t] = I.disk[2 * (band0 + t)];
            dlim[2 * t + 1] = I.disk[2 * (band0 + t) + 1];
        }
        __syncthreads();
        const int64_t base = I.off + wi.z;   // entries hold li - wi.z
        const int64_t nli = (int64_t)wi.w - wi.z;
        const int4* __restrict__ prange = mode == 0 ? R.colp : R.rowp;

        // wave state (uniform): ring heads and fills, next group, octant step.
        // The first group of each wave is fixed, later ones are claimed from
        // the block's counter, so waves with lighter groups take more.
        int bh = 0, bn = 0, lh = 0, ln = 0;
        int64_t g0 = (int64_t)wid * 64;
        int step = 4;
        bool draining = false;
        int64_t li = 0;
        int4 pc = make_int4(0, 0, 0, 0);
        int slo_e = 0, shi_e = 0, slo_o = 0, shi_o = 0;   // body lines of the even / odd octants
        int4 pc_next = pc;
        if (g0 + lane < nli) pc_next = prange[base + g0 + lane];
        for (;;) {
            const bool take_b = bn >= 64 || (draining && bn > 0);
            const bool take_l = !take_b && (ln >= 64 || (draining && ln > 0));
            if (take_b || take_l) {
                // one round: lane k walks the k-th oldest part of the chosen ring
                const int cnt = take_b ? min(bn, 64) : min(ln, 64);
                if (lane < cnt) {
                    const uint32_t ent = take_b ? rbody[(bh + lane) & (kRingBody - 1)]
                                                : rline[(lh + lane) & (kRingLine - 1)];
                    const int64_t gi = base + (ent >> 4);
                    const int p = (ent >> 2) & 3;
                    const int part = ent & 3;
                    const float4 abc = R.abc[gi];
                    const int4 pc2 = prange[gi];
                    const int4 geo2 = R.geo[gi];
                    const int32_t pr = p == 0 ? pc2.x : (p == 1 ? pc2.y : (p == 2 ? pc2.z : pc2.w));
                    int s, e;
                    unpack_range(pr, s, e);
                    int dir, slo, shi;
                    octant_walk_info(mode, p, geo2, dir, slo, shi, kCoarseRowShrink);
                    const int2 pp = piece_part(max(s, band0), min(e, band0 + bwb), slo, shi, part);
                    const int sel = p >> 1;
                    CoarseEmit em{tile, -(band0 >> 1) * Sw, Sw, 0, G - 1};
                    float aL = abc.x, bL = abc.y;
                    if (mode == 1) {
                        int ja, jb;
                        unpack_range(geo2.x, ja, jb);
                        if (sel == 0) em.chi = min(G - 1, ja - 1); else em.clo = max(0, jb);
                        aL = abc.y;
                        bL = abc.x;
                    }
                    if (em.chi < em.clo) {
                        // this quarter owns no column in the band: nothing to vote
                    } else if (take_b) {
                        walk_certified<true>(aL, bL, abc.z, sel, dir, abc.w, -1.0f, h, -1.0f, h, pp.x, pp.y, em, bad);
                    } else {
                        walk_search(aL, bL, abc.z, sel, -1.0f, h, -1.0f, h, pp.x, pp.y, em, bad);
                    }
                }
                if (take_b) {
                    bh += cnt;
                    bn -= cnt;
                } else {
                    lh += cnt;
                    ln -= cnt;
                }
                continue;
            }
            if (draining) break;
            if (step == 4) {
                // next group of 64 correspondences
                if (g0 >= nli) {
                    draining = true;
                    continue;
                }
                li = g0 + lane;
                pc = pc_next;
                const bool live = li < nli;
                int gn = 0;
                if (lane == 0) gn = atomicAdd(&group_next, 64);
                g0 = __builtin_amdgcn_readlane(gn, 0);
                if (g0 + lane < nli) pc_next = prange[base + g0 + lane];
                // correspondences outside the walk's range of validity (column
                // pass only): exhaustive cell test of the band by the whole wave
                unsigned long long rk = __ballot(live && pc.x == kRiskyMark);
                while (rk) {
                    const int l = __ffsll((long long)rk) - 1;
                    rk &= rk - 1ull;
                    const float4 abc = R.abc[base + li - lane + l];
                    for (int t = lane; t < bwb * G; t += 64) {
                        const int k = t >> lbw;
                        const int jl = t & (bwb - 1);
                        if (k < dlim[2 * jl] || k > dlim[2 * jl + 1]) continue;
                        const int j = band0 + jl;
                        float u0 = -1.0f + (float)j * h, u1 = -1.0f + (float)(j + 1) * h;
                        float v0 = -1.0f + (float)k * h, v1 = -1.0f + (float)(k + 1) * h;
                        float uu0 = u0 * u0, uu1 = u1 * u1;
                        float au0 = abc.x * u0, au1 = abc.x * u1;
                        float f0 = vertex_F(abc.y, abc.z, uu0, au0, v0);
                        float f1 = vertex_F(abc.y, abc.z, uu1, au1, v0);
                        float f2 = vertex_F(abc.y, abc.z, uu0, au0, v1);
                        float f3 = vertex_F(abc.y, abc.z, uu1, au1, v1);
                        bool le = (f0 <= 0.0f) | (f1 <= 0.0f) | (f2 <= 0.0f) | (f3 <= 0.0f);
                        bool ge = (f0 >= 0.0f) | (f1 >= 0.0f) | (f2 >= 0.0f) | (f3 >= 0.0f);
                        if (le && ge) atomicAdd(&tile[(jl >> 1) * Sw + k], 1u << ((jl & 1) << 4));
                    }
                }
                bool any = false;
                if (live && pc.x != kRiskyMark) {
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        const int32_t pr = p == 0 ? pc.x : (p == 1 ? pc.y : (p == 2 ? pc.z : pc.w));
                        int s, e;
                        unpack_range(pr, s, e);
                        any |= max(s, band0) < min(e, band0 + bwb);
                    }
                }
                if (any) {
                    // the body range depends on the octant only through its parity
                    const int4 geo = R.geo[base + li];
                    int d;
                    octant_walk_info(mode, 0, geo, d, slo_e, shi_e, kCoarseRowShrink);
                    octant_walk_info(mode, 1, geo, d, slo_o, shi_o, kCoarseRowShrink);
                }
                step = __ballot(any) ? 0 : 4;
                if (!any) li = nli;   // nothing of this one in the band
                continue;
            }
            // append the parts of octant `step` that fall in the band
            {
                const int p = step;
                bool hb = false, h0 = false, h2 = false;
                if (li < nli) {
                    const int32_t pr = p == 0 ? pc.x : (p == 1 ? pc.y : (p == 2 ? pc.z : pc.w));
                    int s, e;
                    unpack_range(pr, s, e);
                    const int cs = max(s, band0), ce = min(e, band0 + bwb);
                    if (cs < ce) {
                        const int slo = (p & 1) ? slo_o : slo_e, shi = (p & 1) ? shi_o : shi_e;
                        int2 parts[3];
                        split_piece(cs, ce, slo, shi, parts);
                        hb = parts[1].x < parts[1].y;
                        h0 = parts[0].x < parts[0].y;
                        h2 = parts[2].x < parts[2].y;
                    }
                }
                const uint32_t key = ((uint32_t)li << 4) | ((uint32_t)p << 2);
                const unsigned long long mb = __ballot(hb), m0 = __ballot(h0), m2 = __ballot(h2);
                if (hb) rbody[(bh + bn + lanes_below(mb)) & (kRingBody - 1)] = key | 1u;
                const int n0 = __popcll(m0);
                if (h0) rline[(lh + ln + lanes_below(m0)) & (kRingLine - 1)] = key | 0u;
                if (h2) rline[(lh + ln + n0 + lanes_below(m2)) & (kRingLine - 1)] = key | 2u;
                bn += __popcll(mb);
                ln += n0 + __popcll(m2);
                ++step;
            }
        }
        __syncthreads();
        // flush the band's cells that meet the disk into this instance's
        // accumulator; consecutive threads take consecutive words (line pairs
        // of one cross index in the column pass, cross indices of one line
        // pair in the row pass)
        uint32_t* grid = grid_arena + I.grid_off;
        const int lhb = lbw - 1;
        for (int t = tid; t < (bwb >> 1) * G; t += kVoteThreads) {
            int m, k;
            size_t g0, g1;
            if (mode == 0) {
                k = t >> lhb;
                m = t & ((bwb >> 1) - 1);
                g0 = (size_t)k * G + band0 + 2 * m;
                g1 = g0 + 1;
            } else {
                m = t >> lg;
                k = t & (G - 1);
                g0 = (size_t)(band0 + 2 * m) * G + k;
                g1 = g0 + G;
            }
            const uint32_t w = tile[m * Sw + k];
            if (!w) continue;
            const uint32_t v0 = w & 0xFFFFu, v1 = w >> 16;
            if (v0 && k >= dlim[4 * m] && k <= dlim[4 * m + 1]) atomicAdd(&grid[g0], v0);
            if (v1 && k >= dlim[4 * m + 2] && k <= dlim[4 * m + 3]) atomicAdd(&grid[g1], v1);
        }
        __syncthreads();
    }
    if (bad) atomicOr(err, bad);
}

// --------------------------------------------------------------------------
// Peaks
// --------------------------------------------------------------------------

// Suppression test of multi-model peak search: integer disk of radius rad
// around an earlier peak, and the disk of radius rad*h around the projection
// -(u, v)/(u^2 + v^2) of its antipodal axis (binary32, as written).
__device__ __forceinline__ bool suppressed(int G, int rad, int px, int py, int ix, int iy) {
    long dx = ix - px, dy = iy - py;
    if (dx * dx + dy * dy <= (long)rad * rad) return true;
    float h = 2.0f / (float)G;
    float pu = -1.0f + ((float)px + 0.5f) * h;
    float pv = -1.0f + ((float)py + 0.5f) * h;
    float cu = -1.0f + ((float)ix + 0.5f) * h;
    float cv = -1.0f + ((float)iy + 0.5f) * h;
    float pu2 = pu * pu;
    float pv2 = pv * pv;
    float s = pu2 + pv2;
    float au = (-pu) / s;
    float av = (-pv) / s;
    float du = cu - au;
    float dv = cv - av;
    float du2 = du * du;
    float dv2 = dv * dv;
    float d2 = du2 + dv2;
    float rh = (float)rad * h;
    float rr = rh * rh;
    return d2 <= rr;
}

// Is cell (ix, iy), holding v votes, a local maximum within the integer disk
// of radius rad: every other cell of the grid in the disk holds fewer votes,
// or as many at a higher linear index.
__device__ bool local_max(const uint32_t* __restrict__ a, int G, int rad, int ix, int iy, uint32_t v) {
    const int y0 = max(0, iy - rad), y1 = min(G - 1, iy + rad);
    for (int y = y0; y <= y1; ++y) {
        const int dy = y - iy;
        const int rem = rad * rad - dy * dy;
        int dx = (int)sqrtf((float)rem);
        while (dx * dx > rem) --dx;
        while ((dx + 1) * (dx + 1) <= rem) ++dx;
        const int x0 = max(0, ix - dx), x1 = min(G - 1, ix + dx);
        const uint32_t* row = a + (size_t)y * (size_t)G;
        for (int x = x0; x <= x1; ++x) {
            const uint32_t o = row[x];
            if (o > v) return false;
            // equal count: the lower linear index wins
            if (o == v && (y < iy || (y == iy && x < ix))) return false;
        }
    }
    return true;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(k, off, 64);
        k = o > k ? o : k;
    }
    return k;
}

// Block-wide max of a u64 key (blockDim a multiple of 64, <= 1024); the
// result is valid in thread 0.
__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long k, unsigned long long* red) {
    k = wave_max_u64(k);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = k;
    __syncthreads();
    unsigned long long b = 0ull;
    if (threadIdx.x == 0) {
        b = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b = red[w] > b ? red[w] : b;
    }
    return b;
}

// Local-maximum bitmap of an instance with several peaks: bit c set iff
// cell c holds a vote and is a local maximum within radius rad.  A work-group
// takes the whole rows [c0/G, c1/G) of a cell item (item bounds are whole
// rows) and the 64 columns blockIdx.y * 64 + [0, 64): it stages those cells
// with a margin of rad cells (zero outside the grid, which never beats a cell
// with a vote) in LDS and tests every disk neighbour of each cell without
// early exits, so that neighbouring lanes advance together.  A wave's 64
// lanes cover 64 consecutive cells of a row, so its ballot is two words of
// the bitmap.  Radii above kLocalMaxLdsRad read the grid directly.
constexpr int kLocalMaxLdsRad = 32;
constexpr int kLocalMaxRows = 64;   // rows of a cell item at most (8192 cells, G >= 128; or the 64 x 64 grid)

size_t local_max_lds_bytes() {
    return ((size_t)(kLocalMaxRows + 2 * kLocalMaxLdsRad) * (64 + 2 * kLocalMaxLdsRad) + 2 * kLocalMaxLdsRad + 1) * 4;
}

__global__ __launch_bounds__(256) void k_local_max(const uint32_t* __restrict__ grid_arena,
                                                   const Inst* __restrict__ insts, const int4* __restrict__ items,
                                                   uint32_t* __restrict__ lmax) {
    extern __shared__ __align__(16) uint32_t lm[];
    const int4 wi = items[blockIdx.x];
    const Inst& I = insts[wi.x];
    if (I.npk < 2) return;
    const int G = I.G, rad = I.rad;
    const int x0 = (int)blockIdx.y * 64;
    if (x0 >= G) return;
    const uint32_t* a = grid_arena + I.grid_off;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int y0 = wi.y / G, nr = (wi.z - wi.y) / G;
    if (rad > kLocalMaxLdsRad) {
        for (int r = wave; r < nr; r += nwaves) {
            const int c = (y0 + r) * G + x0 + lane;
            const uint32_t v = a[c];
            const bool f = v != 0u && local_max(a, G, rad, x0 + lane, y0 + r, v);
            const unsigned long long m = __ballot(f);
            if (lane == 0) {
                uint32_t* out = lmax + I.lmax_off + ((c - lane) >> 5);
                out[0] = (uint32_t)m;
                out[1] = (uint32_t)(m >> 32);
            }
        }
        return;
    }
    int* ext = reinterpret_cast<int*>(lm);   // half-width of the disk on row dy, at ext[dy + rad]
    uint32_t* tile = lm + 2 * kLocalMaxLdsRad + 1;
    const int TW = 64 + 2 * rad, TH = nr + 2 * rad;
    for (int d = threadIdx.x; d <= 2 * rad; d += blockDim.x) {
        const int dy = d - rad, rem = rad * rad - dy * dy;
        int dx = 0;
        while ((dx + 1) * (dx + 1) <= rem) ++dx;
        ext[d] = dx;
    }
    for (int t = threadIdx.x; t < TW * TH; t += blockDim.x) {
        const int ty = t / TW, tx = t - ty * TW;
        const int gy = y0 - rad + ty, gx = x0 - rad + tx;
        tile[t] = (gy >= 0 && gy < G && gx >= 0 && gx < G) ? a[gy * G + gx] : 0u;
    }
    __syncthreads();
    for (int r = wave; r < nr; r += nwaves) {
        const uint32_t* centre = tile + (r + rad) * TW + rad + lane;
        const uint32_t v = *centre;
        bool f = v != 0u;
        // rows above: any neighbour with as many votes comes first (lower index)
        for (int dy = -rad; dy < 0; ++dy) {
            const int e = ext[dy + rad];
            const uint32_t* row = centre + dy * TW;
            for (int dx = -e; dx <= e; ++dx) f &= row[dx] < v;
        }
        // the cell's own row: equal counts on the left come first
        {
            const int e = ext[rad];
            for (int dx = -e; dx < 0; ++dx) f &= centre[dx] < v;
            for (int dx = 1; dx <= e; ++dx) f &= centre[dx] <= v;
        }
        // rows below: equal counts come later
        for (int dy = 1; dy <= rad; ++dy) {
            const int e = ext[dy + rad];
            const uint32_t* row = centre + dy * TW;
            for (int dx = -e; dx <= e; ++dx) f &= row[dx] <= v;
        }
        const unsigned long long m = __ballot(f);
        if (lane == 0) {
            uint32_t* out = lmax + I.lmax_off + (((y0 + r) * G + x0) >> 5);
            out[0] = (uint32_t)m;
            out[1] = (uint32_t)(m >> 32);
        }
    }
}

// Argmax (ties to the lowest index) of cells [c0, c1) of an instance's grid.
__global__ __launch_bounds__(256) void k_peak(const uint32_t* __restrict__ grid_arena, const Inst* __restrict__ insts,
                                              const int4* __restrict__ items, const PeakState* st, int slot,
                                              const uint32_t* __restrict__ lmax, unsigned long long* keys) {
    __shared__ unsigned long long red[4];
    const int4 wi = items[blockIdx.x];
    const Inst& I = insts[wi.x];
    if (slot >= I.npk) return;
    const uint32_t* a = grid_arena + I.grid_off;
    const int G = I.G;
    const PeakState* prev = st + I.res_off;
    unsigned long long best = 0ull;
    // four cells per 16-byte load (item bounds and grid offsets are multiples of 4)
    const uint4* a4 = reinterpret_cast<const uint4*>(a);
    for (int c4 = (wi.y >> 2) + threadIdx.x; c4 < (wi.z >> 2); c4 += blockDim.x) {
        const uint4 q = a4[c4];
        const uint32_t vv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t v = vv[u];
            const int c = 4 * c4 + u;
            if (v == 0u) continue;
            unsigned long long k = ((unsigned long long)v << 32) | (unsigned long long)(~(uint32_t)c);
            if (k <= best) continue;
            if (slot > 0) {
                // later peaks: local maxima (the first peak is the global
                // maximum, which is one) not suppressed by an earlier peak
                if (!((lmax[I.lmax_off + (c >> 5)] >> (c & 31)) & 1u)) continue;
                int ix = c % G, iy = c / G;
                bool sup = false;
                for (int t = 0; t < slot && !sup; ++t) {
                    uint32_t pc = prev[t].peak_cell;
                    sup = suppressed(G, I.rad, (int)(pc % (uint32_t)G), (int)(pc / (uint32_t)G), ix, iy);
                }
                if (sup) continue;
            }
            best = k;
        }
    }
    best = block_max_u64(best, red);
    if (threadIdx.x == 0 && best) atomicMax(&keys[I.res_off + slot], best);
}

__device__ void window_of(int G, int M, int w, uint32_t cell, FineWin& fw) {
    int ix = (int)(cell % (uint32_t)G), iy = (int)(cell / (uint32_t)G);
    int x0 = ix - w < 0 ? 0 : ix - w;
    int x1 = ix + w > G - 1 ? G - 1 : ix + w;
    int y0 = iy - w < 0 ? 0 : iy - w;
    int y1 = iy + w > G - 1 ? G - 1 : iy + w;
    float h = 2.0f / (float)G;
    fw.nx = x1 - x0 + 1;
    fw.ny = y1 - y0 + 1;
    fw.U0 = -1.0f + (float)x0 * h;
    fw.V0 = -1.0f + (float)y0 * h;
    fw.hx = ((float)fw.nx * h) / (float)M;
    fw.hy = ((float)fw.ny * h) / (float)M;
}

// Peak cell and votes from the key, plus its refinement window.
__global__ void k_peak_finish(const Inst* __restrict__ insts, int ninst, const unsigned long long* keys,
                              PeakState* st, int slot) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= ninst) return;
    const Inst& I = insts[b];
    if (slot >= I.npk) return;
    unsigned long long k = keys[I.res_off + slot];
    PeakState& s = st[I.res_off + slot];
    s.valid = k != 0ull;
    s.peak_cell = k ? ~(uint32_t)(k & 0xFFFFFFFFull) : 0u;
    s.axis_votes = (uint32_t)(k >> 32);
    if (I.M > 0 && s.valid) window_of(I.G, I.M, I.w, s.peak_cell, s.win);
}

// --------------------------------------------------------------------------
// Refinement window
// --------------------------------------------------------------------------

struct FineEmit {
    static constexpr bool kAudit = false;
    static constexpr bool kPairedLines = false;
    uint32_t* tile;
    int mode, M;
    float U0, V0, hx, hy;
    bool all_in;   // every cell of the window meets the disk
    int clo, chi;  // row pass: allowed columns
    __device__ __forceinline__ bool in_disk(int jx, int jy) const {
        float u0 = U0 + (float)jx * hx, u1 = U0 + (float)(jx + 1) * hx;
        float v0 = V0 + (float)jy * hy, v1 = V0 + (float)(jy + 1) * hy;
        float w00 = ((u0 * u0) + (v0 * v0)) - 1.0f;
        float w10 = ((u1 * u1) + (v0 * v0)) - 1.0f;
        float w01 = ((u0 * u0) + (v1 * v1)) - 1.0f;
        float w11 = ((u1 * u1) + (v1 * v1)) - 1.0f;
        return (w00 <= 0.0f) | (w10 <= 0.0f) | (w01 <= 0.0f) | (w11 <= 0.0f);
    }
    // Cells outside the disk are counted too and dropped at the flush.
    __device__ __forceinline__ void operator()(int j, int klo, int khi) {
        klo = max(klo, max(0, clo));
        khi = min(khi, min(M - 1, chi));
#pragma unroll 1
        for (int k = klo; k <= khi; ++k) {
            int jx = mode == 0 ? j : k, jy = mode == 0 ? k : j;
            atomicAdd(&tile[jy * M + (jx ^ (jy & (M - 1)))], 1u);
        }
    }
    __device__ __forceinline__ void add(int j, int k) {
        const int jx = mode == 0 ? j : k, jy = mode == 0 ? k : j;
        atomicAdd(&tile[jy * M + (jx ^ (jy & (M - 1)))], 1u);
    }
    int offs = 0;
    __device__ __forceinline__ int start(int j, int off) {
        offs = off;
        return j;
    }
    __device__ __forceinline__ int next(int j) const { return j + 1; }
    __device__ __forceinline__ void pair(int j, int r, bool second) {
        const int lo = max(0, clo), hi = min(M - 1, chi);
        if (hi < lo) return;
        const unsigned span = (unsigned)(hi - lo);
        const int k0 = r - 1 + offs, k1 = r - offs;
        if ((unsigned)(k0 - lo) <= span) add(j, k0);
        if (second && (unsigned)(k1 - lo) <= span) add(j, k1);
    }
};

// The refinement window of a peak and the quick-reject geometry.
struct FineGeom {
    FineWin fw;
    bool all_in;   // every fine cell meets the disk
    double Uc, Vc, Rw, margin;
};

__device__ __forceinline__ void fine_geom(const FineWin& fw, int M, FineGeom& g) {
    g.fw = fw;
    // The window is [U0, U0 + M hx] x [V0, V0 + M hy].  If its corner farthest
    // from the origin is inside the disk with room to spare, every fine cell
    // meets the disk and the per-cell test is skipped.
    double wu = (double)fw.hx * M, wv = (double)fw.hy * M;
    double ue = fmax(fabs((double)fw.U0), fabs((double)fw.U0 + wu));
    double ve = fmax(fabs((double)fw.V0), fabs((double)fw.V0 + wv));
    g.all_in = ue * ue + ve * ve < 1.0 - 1e-4;
    g.Uc = (double)fw.U0 + 0.5 * wu;
    g.Vc = (double)fw.V0 + 0.5 * wv;
    g.Rw = 0.5 * sqrt(wu * wu + wv * wv);
    g.margin = 2.0 * (double)(fw.hx > fw.hy ? fw.hx : fw.hy);
}

// Quick reject: over the window |F(x) - F(centre)| <= |grad F(centre)| Rw +
// |c| Rw^2; if |F| stays above the binary32 error bound everywhere, every
// vertex has the same sign and no fine cell is voted.
__device__ __forceinline__ bool fine_may_cross(const float4& abc, uint32_t fl, const FineGeom& g) {
    if (fl & kFlagDegenerate) return false;
    if (fl & kFlagRisky) return true;
    double a = abc.x, b = abc.y, c = abc.z;
    double Fc = c * (g.Uc * g.Uc + g.Vc * g.Vc - 1.0) + 2.0 * (a * g.Uc + b * g.Vc);
    double gx = 2.0 * (c * g.Uc + a), gy = 2.0 * (c * g.Vc + b);
    double bound = sqrt(gx * gx + gy * gy) * g.Rw + fabs(c) * g.Rw * g.Rw;
    double ebound = 2e-6 * (fabs(a) + fabs(b) + fabs(c));
    return !(fabs(Fc) > 1.0001 * bound + ebound);
}

// Fine vote of peak `slot`, one work-group per range of correspondences.
// The group lists the curves that may cross the refinement window (quick
// reject above), computes their octant pieces in the window frame, queues one
// entry per non-empty part (certified bodies first, searched lines after) and
// walks the entries one per thread, so threads walk parts side by side rather
// than each running through all eight octants of its own curve.  Candidates
// are processed in batches of at most kFineCand; the M x M tile is flushed
// (disk mask applied) at the end.
constexpr int kFineThreads = 256;
constexpr int kFineCand = 512;                 // candidate records per batch
constexpr int kFineBody = kFineCand * 8;       // <= 8 octants x 1 body
constexpr int kFineLine = kFineCand * 16;      // <= 8 octants x 2 searched parts

size_t fine_lds_bytes(int maxM) {
    return (size_t)maxM * maxM * 4 + (size_t)kFineCand * (16 + 16 + 16 + 16) + (size_t)kFineBody * 2 +
           (size_t)kFineLine * 2;
}

__global__ __launch_bounds__(kFineThreads) void k_fine_vote(const ArcRecs R, const Inst* __restrict__ insts,
                                                            const int4* __restrict__ items, const PeakState* st,
                                                            int slot, uint32_t* __restrict__ fine_arena,
                                                            uint32_t* __restrict__ err) {
    extern __shared__ __align__(16) uint32_t fsm[];
    __shared__ int ncand, nbody, nline;
    const int4 wi = items[blockIdx.x];
    const Inst& I = insts[wi.x];
    if (I.M <= 0 || slot >= I.npk) return;
    const PeakState& s = st[I.res_off + slot];
    if (!s.valid) return;
    const int M = I.M;
    FineGeom g;
    fine_geom(s.win, M, g);
    const FineWin& fw = g.fw;
    uint32_t* ftile = fsm;
    float4* cabc = reinterpret_cast<float4*>(fsm + M * M);
    int4* ccol = reinterpret_cast<int4*>(cabc + kFineCand);
    int4* crow = ccol + kFineCand;
    int4* cgeo = crow + kFineCand;
    uint16_t* qbody = reinterpret_cast<uint16_t*>(cgeo + kFineCand);
    uint16_t* qline = qbody + kFineBody;
    int32_t* cidx = reinterpret_cast<int32_t*>(qline);   // candidate offsets, reused as queue space later
    const int tid = threadIdx.x;
    for (int t = tid; t < M * M; t += kFineThreads) ftile[t] = 0u;
    if (tid == 0) ncand = 0;
    __syncthreads();
    uint32_t bad = 0;
    for (int64_t c0 = wi.y; c0 < wi.z; c0 += kFineThreads) {
        // list this chunk's candidates
        const int64_t li = c0 + tid;
        if (li < wi.z) {
            const int64_t gi = I.off + li;
            if (fine_may_cross(R.abc[gi], (uint32_t)R.geo[gi].w, g)) cidx[atomicAdd(&ncand, 1)] = (int32_t)li;
        }
        __syncthreads();
        const int nc = ncand;
        __syncthreads();   // every thread has read ncand before it changes again
        if (nc <= kFineCand - kFineThreads && c0 + kFineThreads < wi.z) continue;   // room for another chunk
        // pieces of each candidate in the window frame; queue their parts
        int myc[2] = {-1, -1};
        for (int c = tid, q = 0; c < nc; c += kFineThreads, ++q) myc[q] = cidx[c];
        __syncthreads();   // cidx is overwritten by the line queue below
        if (tid == 0) {
            nbody = 0;
            nline = 0;
        }
        __syncthreads();
        for (int q = 0; q < 2; ++q) {
            const int c = tid + q * kFineThreads;
            if (c >= nc) break;
            const int64_t gi = I.off + myc[q];
            const float4 abc = R.abc[gi];
            const uint32_t fl = (uint32_t)R.geo[gi].w;
            if (fl & kFlagRisky) {
                // outside the walk's range of validity: every cell of the window
                for (int jy = 0; jy < M; ++jy)
                    for (int jx = 0; jx < M; ++jx) {
                        float u0 = fw.U0 + (float)jx * fw.hx, u1 = fw.U0 + (float)(jx + 1) * fw.hx;
                        float v0 = fw.V0 + (float)jy * fw.hy, v1 = fw.V0 + (float)(jy + 1) * fw.hy;
                        float uu0 = u0 * u0, uu1 = u1 * u1, au0 = abc.x * u0, au1 = abc.x * u1;
                        float f0 = vertex_F(abc.y, abc.z, uu0, au0, v0);
                        float f1 = vertex_F(abc.y, abc.z, uu1, au1, v0);
                        float f2 = vertex_F(abc.y, abc.z, uu0, au0, v1);
                        float f3 = vertex_F(abc.y, abc.z, uu1, au1, v1);
                        bool le = (f0 <= 0.0f) | (f1 <= 0.0f) | (f2 <= 0.0f) | (f3 <= 0.0f);
                        bool ge = (f0 >= 0.0f) | (f1 >= 0.0f) | (f2 >= 0.0f) | (f3 >= 0.0f);
                        if (le && ge) atomicAdd(&ftile[jy * M + (jx ^ (jy & (M - 1)))], 1u);
                    }
                continue;
            }
            int4 colp, rowp, geo;
            circle_pieces<false>(abc.x, abc.y, abc.z, fl, fw.U0, fw.hx, M, fw.V0, fw.hy, M, g.margin, colp, rowp, geo);
            cabc[c] = abc;
            ccol[c] = colp;
            crow[c] = rowp;
            cgeo[c] = geo;
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const int4 pc = m == 0 ? colp : rowp;
                    const int32_t pr = p == 0 ? pc.x : (p == 1 ? pc.y : (p == 2 ? pc.z : pc.w));
                    int s0, e0, dir, slo, shi;
                    unpack_range(pr, s0, e0);
                    if (s0 >= e0) continue;
                    octant_walk_info(m, p, geo, dir, slo, shi);
                    int2 parts[3];
                    split_piece(s0, e0, slo, shi, parts);
                    const uint16_t key = (uint16_t)((c << 5) | (m << 4) | (p << 2));
                    if (parts[1].x < parts[1].y) qbody[atomicAdd(&nbody, 1)] = key | 1u;
                    if (parts[0].x < parts[0].y) qline[atomicAdd(&nline, 1)] = key | 0u;
                    if (parts[2].x < parts[2].y) qline[atomicAdd(&nline, 1)] = key | 2u;
                }
        }
        __syncthreads();
        // walk the queued parts, bodies first
        const int nb = nbody, nl = nline;
        for (int e = tid; e < nb + nl; e += kFineThreads) {
            const int ent = e < nb ? qbody[e] : qline[e - nb];
            const int c = ent >> 5, m = (ent >> 4) & 1, p = (ent >> 2) & 3, part = ent & 3;
            const float4 abc = cabc[c];
            const int4 pc = m == 0 ? ccol[c] : crow[c];
            const int4 geo = cgeo[c];
            const int32_t pr = p == 0 ? pc.x : (p == 1 ? pc.y : (p == 2 ? pc.z : pc.w));
            int s0, e0, dir, slo, shi;
            unpack_range(pr, s0, e0);
            octant_walk_info(m, p, geo, dir, slo, shi);
            const int2 pp = piece_part(s0, e0, slo, shi, part);
            int ja, jb;
            unpack_range(geo.x, ja, jb);
            FineEmit em{ftile, m, M, fw.U0, fw.V0, fw.hx, fw.hy, g.all_in,
                        (m == 1 && (p >> 1)) ? jb : -(1 << 20), (m == 1 && !(p >> 1)) ? ja - 1 : (1 << 20)};
            const float aL = m == 0 ? abc.x : abc.y, bL = m == 0 ? abc.y : abc.x;
            const float x0 = m == 0 ? fw.U0 : fw.V0, hx = m == 0 ? fw.hx : fw.hy;
            const float y0 = m == 0 ? fw.V0 : fw.U0, hy = m == 0 ? fw.hy : fw.hx;
            if (part == 1)
                walk_certified(aL, bL, abc.z, p >> 1, dir, kFineCertScale * abc.w, x0, hx, y0, hy, pp.x, pp.y, em,
                               bad);
            else
                walk_search(aL, bL, abc.z, p >> 1, x0, hx, y0, hy, pp.x, pp.y, em, bad);
        }
        __syncthreads();
        if (tid == 0) ncand = 0;
        __syncthreads();
    }
    if (bad) atomicOr(err, bad << 8);
    uint32_t* fine = fine_arena + I.fine_off + (size_t)slot * M * M;
    FineEmit em{ftile, 0, M, fw.U0, fw.V0, fw.hx, fw.hy, g.all_in, 0, 0};
    for (int t = tid; t < M * M; t += kFineThreads) {
        uint32_t v = ftile[t];
        if (!v) continue;
        const int jy = t / M;
        const int jx = (t - jy * M) ^ (jy & (M - 1));
        if (!g.all_in && !em.in_disk(jx, jy)) continue;
        atomicAdd(&fine[jy * M + jx], v);
    }
}

// Fine argmax (one block per instance), then the axis by inverse projection
// (Eq. (8)): s = u*u + v*v, den = 1 + s, r = (2u/den, 2v/den, (s - 1)/den).
__global__ __launch_bounds__(1024) void k_fine_peak(const uint32_t* __restrict__ fine_arena,
                                                    const Inst* __restrict__ insts, PeakState* st, int slot) {
    __shared__ unsigned long long red[16];
    const Inst& I = insts[blockIdx.x];
    if (slot >= I.npk) return;
    PeakState& s = st[I.res_off + slot];
    if (!s.valid) return;
    const int M = I.M;
    unsigned long long best = 0ull;
    if (M > 0) {
        const uint32_t* fine = fine_arena + I.fine_off + (size_t)slot * M * M;
        for (int c = threadIdx.x; c < M * M; c += blockDim.x) {
            unsigned long long k = ((unsigned long long)fine[c] << 32) | (unsigned long long)(~(uint32_t)c);
            best = k > best ? k : best;
        }
    }
    best = block_max_u64(best, red);
    if (threadIdx.x != 0) return;
    float u, v;
    if (M > 0) {
        uint32_t fc = ~(uint32_t)(best & 0xFFFFFFFFull);
        s.fine_cell = fc;
        s.fine_votes = (uint32_t)(best >> 32);
        int jx = (int)(fc % (uint32_t)M), jy = (int)(fc / (uint32_t)M);
        u = s.win.U0 + ((float)jx + 0.5f) * s.win.hx;
        v = s.win.V0 + ((float)jy + 0.5f) * s.win.hy;
    } else {
        s.fine_cell = 0u;
        s.fine_votes = 0u;
        const int G = I.G;
        float h = 2.0f / (float)G;
        int ix = (int)(s.peak_cell % (uint32_t)G), iy = (int)(s.peak_cell / (uint32_t)G);
        u = -1.0f + ((float)ix + 0.5f) * h;
        v = -1.0f + ((float)iy + 0.5f) * h;
    }
    float uu = u * u;
    float vv = v * v;
    float ss = uu + vv;
    float den = 1.0f + ss;
    float u2 = 2.0f * u;
    float v2 = 2.0f * v;
    float sm1 = ss - 1.0f;
    s.axis[0] = u2 / den;
    s.axis[1] = v2 / den;
    s.axis[2] = sm1 / den;
}

// --------------------------------------------------------------------------
// Literal sampling rule (Algorithm 1's inner loop; selectable alternative to
// the per-cell rule of the coarse vote)
// --------------------------------------------------------------------------

// Frame of the great circle of (p, q): z = (q - p)/|q - p|, alpha1 = e_k minus
// its projection onto z, normalised (k = index of z's smallest component,
// lowest on ties), alpha2 = alpha1 x z.  False when |q - p|^2 is zero or not
// finite (no samples).  Every value is one rounded binary32 operation in the
// order written; square root and division are correctly rounded.
__device__ __forceinline__ bool sample_frame(const float* p, const float* q, float* a1, float* a2) {
    const float d0 = q[0] - p[0], d1 = q[1] - p[1], d2 = q[2] - p[2];
    const float n2 = ((d0 * d0) + (d1 * d1)) + (d2 * d2);
    if (!(n2 > 0.0f) || !isfinite(n2)) return false;
    const float nz = sqrtf(n2);
    const float z[3] = {d0 / nz, d1 / nz, d2 / nz};
    int k0 = 0;
    if (fabsf(z[1]) < fabsf(z[k0])) k0 = 1;
    if (fabsf(z[2]) < fabsf(z[k0])) k0 = 2;
    const float zk = z[k0];
    float t[3];
    for (int k = 0; k < 3; ++k) {
        const float e = (k == k0) ? 1.0f : 0.0f;
        const float pz = zk * z[k];
        t[k] = e - pz;
    }
    const float m = sqrtf(((t[0] * t[0]) + (t[1] * t[1])) + (t[2] * t[2]));
    for (int k = 0; k < 3; ++k) a1[k] = t[k] / m;
    a2[0] = (a1[1] * z[2]) - (a1[2] * z[1]);
    a2[1] = (a1[2] * z[0]) - (a1[0] * z[2]);
    a2[2] = (a1[0] * z[1]) - (a1[1] * z[0]);
    return true;
}

// floor(x) as an int in one instruction (x finite, |x| < 2^31)
__device__ __forceinline__ int floor_to_int(float x) {
    int r;
    __asm__("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// x clamped to [0, hi] (hi >= 0 and the same on every lane) in one instruction
__device__ __forceinline__ int clamp_int(int x, int hi) {
    int r;
    __asm__("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(x), "s"(hi));
    return r;
}

// Cell of sample s = alpha1 cos + alpha2 sin, or false on the open northern
// hemisphere: projection from the north pole (Eq. (7)) as
// (s_x, s_y) * (1 / (1 - s_z)), cell floor((u + 1) G/2) clamped to [0, G-1].
// (u + 1) G/2 is one fused multiply-add u hg + hg: hg = G/2 is a power of
// two, so rounding u hg + hg once gives round(u + 1) hg, the rule's value.
__device__ __forceinline__ bool sample_cell(const float* a1, const float* a2, float c, float sn, int G, float hg,
                                            int& ix, int& iy) {
    const float s0 = (a1[0] * c) + (a2[0] * sn);
    const float s1 = (a1[1] * c) + (a2[1] * sn);
    const float s2 = (a1[2] * c) + (a2[2] * sn);
    if (!(s2 <= 0.0f)) return false;
    const float rinv = recip_1_4(1.0f - s2);
    const float u = s0 * rinv, v = s1 * rinv;
    // |u|, |v| <= 1 here (up to rounding), so both values are small and finite
    ix = clamp_int(floor_to_int(__builtin_fmaf(u, hg, hg)), G - 1);
    iy = clamp_int(floor_to_int(__builtin_fmaf(v, hg, hg)), G - 1);
    return true;
}

// Per-circle record of the band pass (kSampleRec words): the frame (alpha1,
// alpha2), the window of sample indices [js, js + L) (mod J) that holds every
// southern sample, a row margin M (word 7 = L | M << 17), and the rows
// floor((v + 1) G/2), clamped to [-2, G + 1], of the 64
// checkpoints js + (k L)/63, k = 0..63, as int16.  Every sample between
// checkpoints k and k+1 has its row within M of theirs: the projected arc
// between them is shorter than l = dtheta (L/63 + 1) * 1.02 (the projection
// scales lengths by 1/(1 - s_z) <= 1.02 in the window) and, as an arc of a
// circle of radius at least 1 (or a line), leaves their chord by at most
// l^2/8.
__device__ __forceinline__ float sample_row_coord(const float* a1, const float* a2, float c, float sn, float hg) {
    const float s1 = (a1[1] * c) + (a2[1] * sn);
    const float s2 = (a1[2] * c) + (a2[2] * sn);
    return ((s1 / (1.0f - s2)) + 1.0f) * hg;
}

// One lane per circle for the frame and window (its inputs are read
// coalesced, and the slow parts of the frame run once per circle), then the
// 64 checkpoint rows of each circle of the wave, one lane per checkpoint, from
// the circle's values read into scalar registers.
__global__ __launch_bounds__(256) void k_sample_setup(const float* __restrict__ P, const float* __restrict__ Q,
                                                      int64_t N, const Inst* __restrict__ insts,
                                                      const int4* __restrict__ items, uint32_t* __restrict__ recs) {
    extern __shared__ __align__(16) float sdir[];
    const int4 wi = items[blockIdx.x];
    const Inst& I = insts[wi.x];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int J = I.J, G = I.G;
    const float hg = 0.5f * (float)G;
    const float dth = 6.28318531f / (float)J;
    // the 64 checkpoints of a circle read directions far apart: from LDS when
    // the tables fit (J <= kSetupLdsDirs), else from global memory
    const bool lds = J <= kSetupLdsDirs;
    if (lds) {
        for (int e = threadIdx.x; e < J; e += blockDim.x) {
            sdir[e] = I.scs[e];
            sdir[J + e] = I.ssn[e];
        }
        __syncthreads();
    }
    const float* dcs = lds ? sdir : I.scs;
    const float* dsn = lds ? sdir + J : I.ssn;
    for (int64_t base = wi.y + 64 * wave; base < wi.z; base += 64 * nw) {
        const int64_t li = base + lane;
        float a1[3] = {0.0f, 0.0f, 0.0f}, a2[3] = {0.0f, 0.0f, 0.0f};
        int js = 0, L = 0, M = 0;
        if (li < wi.z) {
            const int64_t i = I.off + li;
            const float p[3] = {P[i], P[N + i], P[2 * N + i]};
            const float q[3] = {Q[i], Q[N + i], Q[2 * N + i]};
            if (sample_frame(p, q, a1, a2)) {
                // s_z = a1z cos t + a2z sin t is at most 0 on the half circle
                // centred on t = atan2(a2z, a1z) + pi; within 0.01 of the
                // equator plane every sample may be southern
                const float rz2 = (a1[2] * a1[2]) + (a2[2] * a2[2]);
                float scale = 1.0102f;   // bound on 1/(1 - s_z) over the window
                bool all_rows = false;
                if (rz2 < 1e-4f) {
                    js = 0;
                    L = J;
                } else {
                    const float t0 = atan2f(a2[2], a1[2]) + 1.57079633f;   // start of the southern half
                    const int j0 = (int)ceilf((t0 + 3.14159265f) / dth) - 4;
                    L = (int)ceilf(3.14159265f / dth) + 9;
                    js = ((j0 % J) + J) % J;
                    // the window reaches 4.5 sample steps past the southern half
                    const float sm = sqrtf(rz2) * sinf(fminf(4.5f * dth, 1.57079633f));
                    if (L >= J || sm > 0.5f) {   // few samples: walk the whole circle in every band
                        js = 0;
                        L = J;
                        all_rows = true;
                    } else {
                        scale = 1.0f / (1.0f - sm);
                    }
                }
                const float l = dth * ((float)L / 63.0f + 1.0f) * scale * 1.01f;
                // stored rows lie in [-2, G + 1], so a margin of G + 4 reaches every row
                M = all_rows ? G + 4 : (int)ceilf(fminf(l * l * 0.125f * hg + 0.05f, (float)G)) + 1;
                M = M < G + 4 ? M : G + 4;
            }
            // header: the frame, js, L | M << 17 (L = 0: no samples)
            uint32_t* rec = recs + (I.ssetup_off + li) * kSampleRec;
            for (int k = 0; k < 3; ++k) {
                rec[k] = __float_as_uint(a1[k]);
                rec[3 + k] = __float_as_uint(a2[k]);
            }
            rec[6] = (uint32_t)js;
            rec[7] = (uint32_t)L | ((uint32_t)M << 17);
        }
        const int ncirc = wi.z - base < 64 ? (int)(wi.z - base) : 64;
        for (int k = 0; k < ncirc; ++k) {
            const int Lk = __builtin_amdgcn_readlane(L, k);
            if (Lk == 0) continue;   // uniform
            auto bcast = [k](float v) { return __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(v), k)); };
            const float b1[3] = {bcast(a1[0]), bcast(a1[1]), bcast(a1[2])};
            const float b2[3] = {bcast(a2[0]), bcast(a2[1]), bcast(a2[2])};
            int c = __builtin_amdgcn_readlane(js, k) + (lane * Lk) / 63;
            if (c >= J) c -= J;
            float t = sample_row_coord(b1, b2, dcs[c], dsn[c], hg);
            t = fminf(fmaxf(t, -2.0f), (float)(G + 1));   // also maps NaN to -2
            const int r = (int)floorf(t);
            reinterpret_cast<int16_t*>(recs + (I.ssetup_off + base + k) * kSampleRec + 8)[lane] = (int16_t)r;
        }
    }
}

// The circles of a band item, walked by the waves of its work-group into the
// band tile.  kLdsDirs: the sample directions were staged in LDS (else they
// are read from global memory); kHalf: 16-bit counters, cells 2m and 2m + 1
// in word m.  Each wave walks 64 samples per step with the exact per-sample
// cell; the directions of the next step are loaded into the other of two
// register pairs while this step is evaluated.
typedef __attribute__((address_space(3))) uint32_t lds_u32;   // a word of LDS
template <bool B>
struct BoolTag {
    static constexpr bool value = B;
};

template <bool kLdsDirs, bool kHalf>
__device__ __forceinline__ void sample_band_walk(const Inst& I, const int4 wi, const uint32_t* __restrict__ recs,
                                                 const float* ldir, uint32_t* tile, int r0, int r1) {
    const int G = I.G, J = I.J;
    const int lane = threadIdx.x & 63;
    // the wave index is uniform: say so, so that the circle index and the
    // record offsets live in scalar registers
    int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __asm__("" : "+s"(wave));   // kept in a scalar register (not recomputed inside the loops)
    const int nw = blockDim.x >> 6;
    const float hg = 0.5f * (float)G;
    const int tw = (kHalf ? G >> 1 : G) + 1;   // words per tile row (odd: rows start in different banks)
    const uint32_t tw4 = 4u * (uint32_t)tw;
    const uint32_t tb = (uint32_t)(uintptr_t)(lds_u32*)tile;   // LDS address of the tile
    // buffer resources over the direction tables and over the instance's
    // circle records; reads past the end return 0, so the loads of a step are
    // issued unconditionally (the wait for a step then counts exactly the
    // loads issued after it)
    // one resource over both direction tables: the sines follow the cosines
    // and their pads (I.ssn = I.scs + J + kDirPad), reached through a scalar
    // offset of 4 (J + kDirPad) bytes
    const __amdgpu_buffer_rsrc_t rdir =
        __builtin_amdgcn_make_buffer_rsrc((void*)I.scs, (short)0, 8 * (J + kDirPad), 0x00020000);
    const int sn_off = 4 * (J + kDirPad);
    const __amdgpu_buffer_rsrc_t rrec = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(recs + I.ssetup_off * kSampleRec), (short)0, I.n * kSampleRec * 4, 0x00020000);
    const int lane4 = lane << 2;
    // directions jb + lane (a run that passes J is split there; indices past
    // J belong to samples that are not voted)
    auto dir = [&](int jb, float& c, float& sn) {
        if (kLdsDirs) {
            const int jc = jb + lane < J ? jb + lane : J - 1;
            c = ldir[jc];
            sn = ldir[J + jc];
        } else {
            // indices J..J+63 read NaN pads (never voted), beyond them sines
            // or zeros (loads of a step past the run, not used)
            const int off = lane4 + (jb << 2);
            c = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rdir, off, 0, 0));
            sn = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rdir, off, sn_off, 0));
        }
    };
    // circle li's record: lanes 0..7 take the header words, every lane its
    // checkpoint row (the scalar offset carries the circle)
    const int hoff = (lane < 8 ? lane : 7) << 2, roff = 32 + (lane << 1);
    auto load_rec = [&](int64_t li, uint32_t& h, int& row) {
        const int base = __builtin_amdgcn_readfirstlane((int)li * (kSampleRec * 4));   // uniform
        h = __builtin_amdgcn_raw_buffer_load_b32(rrec, hoff, base, 0);
        row = (int)(int16_t)__builtin_amdgcn_raw_buffer_load_b16(rrec, roff, base, 0);
    };
    // the next circle's record is loaded while the current one is walked
    int64_t li = wi.z + wave;
    uint32_t hn = 0u;
    int rn_row = 0;
    if (li < wi.w) load_rec(li, hn, rn_row);
    for (; li < wi.w; li += nw) {
        const uint32_t hw = hn;
        const int rk = rn_row;
        if (li + nw < wi.w) load_rec(li + nw, hn, rn_row);
        // the record's words are uniform: read them into scalar registers
        const uint32_t lw = __builtin_amdgcn_readlane(hw, 7);
        const int L = (int)(lw & 0x1FFFFu), M = (int)(lw >> 17);   // L <= 65536, M <= G + 4 <= 4100
        if (L == 0) continue;   // uniform
        const float a1[3] = {__uint_as_float(__builtin_amdgcn_readlane(hw, 0)),
                             __uint_as_float(__builtin_amdgcn_readlane(hw, 1)),
                             __uint_as_float(__builtin_amdgcn_readlane(hw, 2))};
        const float a2[3] = {__uint_as_float(__builtin_amdgcn_readlane(hw, 3)),
                             __uint_as_float(__builtin_amdgcn_readlane(hw, 4)),
                             __uint_as_float(__builtin_amdgcn_readlane(hw, 5))};
        const int js = (int)__builtin_amdgcn_readlane(hw, 6);
        // row and first sample of checkpoint lane + 1 (wavefront shift by one
        // lane; lane 63 keeps its own)
        const int rn = __builtin_amdgcn_update_dpp(rk, rk, 0x130, 0xf, 0xf, false);
        // (lane L) / 63 for lane L < 2^22: multiply-high by ceil(2^37 / 63)
        const int ck = (int)(__umulhi(__umul24((uint32_t)lane, (uint32_t)L), 2181570691u) >> 5);
        const int cn = __builtin_amdgcn_update_dpp(ck, ck, 0x130, 0xf, 0xf, false);
        const int lo = (rk < rn ? rk : rn) - M, hi = (rk > rn ? rk : rn) + M;
        const bool hit = lane < 63 && cn > ck && hi >= r0 && lo < r1;
        unsigned long long mask = __ballot(hit);
        // one sample: its cell in the band tile, or nothing
        const unsigned rows = (unsigned)(r1 - r0);
        // Without branches: every lane evaluates the rule (a northern sample's
        // values are garbage and unused) and adds to the tile, 0 when the
        // sample is not voted in this band (to its own word lane).  LDS
        // atomics: lanes of a run of equal cells serialise on one address,
        // which costs less here than merging the run.
        auto vote = [&](bool valid, float c, float sn) {
            const float s0 = (a1[0] * c) + (a2[0] * sn);
            const float s1 = (a1[1] * c) + (a2[1] * sn);
            const float s2 = (a1[2] * c) + (a2[2] * sn);
            const float rinv = recip_1_4(1.0f - s2);
            const float u = s0 * rinv, v = s1 * rinv;
            const int ixf = floor_to_int(__builtin_fmaf(u, hg, hg));
            const int iyf = floor_to_int(__builtin_fmaf(v, hg, hg));
            // 16-bit tiles: rows -1 and G have tile rows of their own in the
            // first and the last band (folded into rows 0 and G - 1 when the
            // tile is stored, like the columns below)
            const int iy = kHalf ? iyf : clamp_int(iyf, G - 1);
            const int ry = iy - r0;
            const bool ok = valid && s2 <= 0.0f && (unsigned)ry < rows;
            // tile rows of tw words: G/2 (+1 pad) with 16-bit counters, cells
            // 2m and 2m + 1 of a row in word m; G (+1) with 32-bit ones
            if (kHalf) {
                // Neither coordinate is clamped here.  A voted sample has s_z <= 0,
                // and the frame and the directions are unit vectors to a few
                // ulps, so |u|, |v| <= 1 + 2^-16 and ixf, iyf lie in [-1, G] (G <= 4096).
                // Cell G of row r lands in the low half of the row's pad word,
                // cell -1 in the high half of the word before the row (the pad
                // of row r - 1, or a word before the tile); the tile store adds
                // them to cells G - 1 and 0, which is the rule's clamp.
                // LDS address tb + ry (4 tw) + 4 (ixf >> 1) = tb + 2 (ixf & ~1) + ry (4 tw)
                // in three instructions (a garbage ry of an unvoted lane is
                // never used)
                uint32_t addr;
                __asm__("v_and_b32 %0, -2, %1\n\tv_lshl_add_u32 %0, %0, 1, %2\n\tv_mad_u32_u24 %0, %3, %4, %0"
                        : "=&v"(addr)
                        : "v"(ixf), "s"(tb), "v"(ry), "s"(tw4));
                const uint32_t inc = 1u << ((ixf & 1) << 4);
                if (ok)
                    __hip_atomic_fetch_add((lds_u32*)(uintptr_t)addr, inc, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
            } else {
                const int ix = clamp_int(ixf, G - 1);
                const int word = (int)__umul24((uint32_t)ry, (uint32_t)tw) + ix;
                if (ok) atomicAdd(&tile[word], 1u);
            }
        };
        // samples [b, f) of indices below J, 64 per step from the uniform
        // base j0: three register pairs of directions, step t uses one while
        // steps t + 1 and t + 2 are in flight in the others
        // Checked: lanes past f are not voted.  Unchecked: the last step's
        // lanes past f are evaluated too, which is exact when (a) checkpoint
        // intervals hold at least 64 samples, so the up to 63 samples past a
        // run's end lie in the interval after it, which reaches no row of the
        // band (else it would be part of the run) or lies outside the window,
        // where every sample is northern (L + 64 <= J, or the window is the
        // whole circle), and (b) indices J..J+62 read the tables' NaN pads, so
        // s_z <= 0 fails there.
        auto walk = [&](auto checked, int b, int f) {
            auto valid = [&](int j0) { return decltype(checked)::value ? lane < f - j0 : true; };
            float c0, s0, c1, s1, c2, s2;
            dir(b, c0, s0);
            dir(b + 64, c1, s1);
            for (int j0 = b; j0 < f; j0 += 192) {
                dir(j0 + 128, c2, s2);
                vote(valid(j0), c0, s0);
                if (j0 + 64 >= f) break;   // uniform
                dir(j0 + 192, c0, s0);
                vote(valid(j0 + 64), c1, s1);
                if (j0 + 128 >= f) break;   // uniform
                dir(j0 + 256, c1, s1);
                vote(valid(j0 + 128), c2, s2);
            }
        };
        auto runs = [&](auto checked) {
            while (mask) {
                const int k = __builtin_ctzll(mask);
                const int e = k + __builtin_ctzll(~(mask >> k));   // bit 63 is never set
                mask &= ~(((1ull << (e - k)) - 1ull) << k);
                const int jb = js + (k * L) / 63, je = js + (e * L) / 63;   // js < J, je <= js + J
                if (jb < J) walk(checked, jb, je < J ? je : J);
                if (je > J) walk(checked, jb > J ? jb - J : 0, je - J);
            }
        };
        // intervals of floor(L / 63) >= 64 samples (uniform)
        if (!kLdsDirs && L >= 64 * 63 && (L == J || L + 64 <= J)) runs(BoolTag<false>{});
        else runs(BoolTag<true>{});
    }
}

// Band pass: one work item = (instance, band of rows [r0, r1), circles
// [c0, c1)).  A wave takes one circle at a time (its record loaded while the
// previous circle is walked), finds the checkpoint intervals whose rows may
// reach the band, and walks only their samples, 64 per step, with the exact
// per-sample cell, counting them in the LDS tile.  The tile is then stored
// whole to the item's slot of the partial arena (no global atomics).
__global__ __launch_bounds__(1024) void k_sample_vote(const Inst* __restrict__ insts, const int4* __restrict__ items,
                                                      const uint32_t* __restrict__ recs,
                                                      uint32_t* __restrict__ part) {
    extern __shared__ __align__(16) uint32_t sm[];
    const int4 wi = items[blockIdx.x];
    const Inst& I = insts[wi.x];
    const int G = I.G, J = I.J, bw = I.sbw;
    const int band = wi.y;
    const int cells = bw * G;
    const bool half = I.shalf != 0;   // 16-bit counters: cells 2m and 2m + 1 share word m
    const int words = half ? cells >> 1 : cells;
    // 16-bit tiles of the first and the last band take row -1, resp. row G,
    // in a tile row of their own: the walk counts rows [r0, r1)
    const bool top = half && band == 0, bottom = half && band == I.snb - 1;
    const int r0 = band * bw - (top ? 1 : 0), r1 = (band + 1) * bw + (bottom ? 1 : 0);
    // the tile's rows carry one pad word each (an odd stride spreads the
    // cells of one column over the LDS banks)
    const int lrw = half ? 30 - __clz(G) : 31 - __clz(G);   // log2 of the words of a row
    const int padded = (r1 - r0) * ((1 << lrw) + 1);
    // LDS: the sample directions (when they fit), then the band tile (16-bit
    // counters: after one more word, which takes cell -1 of the first row)
    const bool lds_dirs = I.sdir_lds != 0;
    float* ldir = reinterpret_cast<float*>(sm);
    const int pre = half ? 1 : 0;
    uint32_t* tile = sm + (lds_dirs ? 2 * J : 0) + pre;
    for (int e = threadIdx.x; e < padded + pre; e += blockDim.x) tile[e - pre] = 0u;
    if (lds_dirs)
        for (int e = threadIdx.x; e < J; e += blockDim.x) {
            ldir[e] = I.scs[e];
            ldir[J + e] = I.ssn[e];
        }
    __syncthreads();
    if (lds_dirs) {
        if (half) sample_band_walk<true, true>(I, wi, recs, ldir, tile, r0, r1);
        else sample_band_walk<true, false>(I, wi, recs, ldir, tile, r0, r1);
    } else {
        if (half) sample_band_walk<false, true>(I, wi, recs, ldir, tile, r0, r1);
        else sample_band_walk<false, false>(I, wi, recs, ldir, sm, r0, r1);   // tile == sm: its base folds away
    }
    __syncthreads();
    const int chunk = wi.z / I.schunk;
    uint32_t* dst = part + I.spart_off + ((int64_t)chunk * I.snb + band) * words;
    if (half) {
        // cells -1 and G of a row (see the band walk) join cells 0 and G - 1,
        // rows -1 and G join rows 0 and G - 1
        const int last = (1 << lrw) - 1, tw = last + 2;
        auto word = [&](int t, int m) {   // tile row t, word m, with its row's outer cells
            const int pe = t * tw + m;
            uint32_t v = tile[pe];
            if (m == 0) v += tile[pe - 1] >> 16;
            if (m == last) v += tile[pe + 1] << 16;
            return v;
        };
        const int t0 = top ? 1 : 0;
        for (int e = threadIdx.x; e < words; e += blockDim.x) {
            const int m = e & last, r = e >> lrw;
            uint32_t v = word(r + t0, m);
            if (top && r == 0) v += word(0, m);
            if (bottom && r == bw - 1) v += word(r + t0 + 1, m);
            dst[e] = v;
        }
    } else {
        for (int e = threadIdx.x; e < words; e += blockDim.x) dst[e] = tile[e + (e >> lrw)];
    }
}

// grid cell = sum over the instance's circle chunks of its band slot.  With
// 16-bit counters a thread sums one word, i.e. the two cells 2m and 2m + 1.
__global__ __launch_bounds__(256) void k_sample_reduce(const Inst* __restrict__ insts, const int4* __restrict__ items,
                                                       const uint32_t* __restrict__ part,
                                                       uint32_t* __restrict__ grid_arena) {
    const int4 wi = items[blockIdx.x];
    const Inst& I = insts[wi.x];
    if (I.rule != 1 || I.n == 0) return;
    const int G = I.G, bw = I.sbw, cells = bw * G;
    const bool half = I.shalf != 0;
    const int words = half ? cells >> 1 : cells;
    const int nch = (I.n + I.schunk - 1) / I.schunk;
    const int64_t stride = (int64_t)I.snb * words;
    uint32_t* grid = grid_arena + I.grid_off;
    const int step = half ? 2 : 1;   // cells per thread (item bounds are even)
    for (int c = wi.y + step * (int)(blockIdx.y * blockDim.x + threadIdx.x); c < wi.z;
         c += step * (int)(gridDim.y * blockDim.x)) {
        const int band = (c / G) / bw;
        const int within = c - band * cells;
        const uint32_t* src = part + I.spart_off + (int64_t)band * words + (half ? within >> 1 : within);
        if (half) {
            uint32_t lo = 0u, hi = 0u;
            for (int h = 0; h < nch; ++h) {
                const uint32_t v = src[h * stride];
                lo += v & 0xFFFFu;
                hi += v >> 16;
            }
            grid[c] = lo;
            grid[c + 1] = hi;
        } else {
            uint32_t acc = 0u;
            for (int h = 0; h < nch; ++h) acc += src[h * stride];
            grid[c] = acc;
        }
    }
}

// --------------------------------------------------------------------------
// Angle histogram (Sec. IV-B)
// --------------------------------------------------------------------------

// beta = r x p, gamma = r x q, X = beta . gamma, Y = r . (p x q).
__device__ __forceinline__ void angle_xy(const float* r, const float* p, const float* q, float& X, float& Y) {
    float bx = (r[1] * p[2]) - (r[2] * p[1]);
    float by = (r[2] * p[0]) - (r[0] * p[2]);
    float bz = (r[0] * p[1]) - (r[1] * p[0]);
    float gx = (r[1] * q[2]) - (r[2] * q[1]);
    float gy = (r[2] * q[0]) - (r[0] * q[2]);
    float gz = (r[0] * q[1]) - (r[1] * q[0]);
    float xx = bx * gx;
    float xy = by * gy;
    float xz = bz * gz;
    X = (xx + xy) + xz;
    float wx = (p[1] * q[2]) - (p[2] * q[1]);
    float wy = (p[2] * q[0]) - (p[0] * q[2]);
    float wz = (p[0] * q[1]) - (p[1] * q[0]);
    float yx = r[0] * wx;
    float yy = r[1] * wy;
    float yz = r[2] * wz;
    Y = (yx + yy) + yz;
}

__device__ __forceinline__ int half_plane(float X, float Y) {
    return (Y < 0.0f || (Y == 0.0f && X < 0.0f)) ? 0 : 1;
}

// "boundary k is at or below direction (X, Y)" in angular order over [-pi, pi).
__device__ __forceinline__ bool at_or_below(float tc, float ts, int hv, float X, float Y) {
    int ht = half_plane(tc, ts);
    if (ht != hv) return ht < hv;
    float t1 = tc * Y;
    float t2 = ts * X;
    return (t1 - t2) >= 0.0f;
}

// Bin = number of boundaries k in [1, B-1] at or below (X, Y).  The predicate
// is monotone in k (boundaries are far apart compared with binary32 rounding),
// so a binary search returns the count.  -1 = no vote.
__device__ __forceinline__ int angle_bin(const float* tc, const float* ts, int B, float X, float Y) {
    if (!(isfinite(X) && isfinite(Y))) return -1;
    if (X == 0.0f && Y == 0.0f) return -1;
    int hv = half_plane(X, Y);
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (at_or_below(tc[mid], ts[mid], hv, X, Y)) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Angle gate (coarse-to-fine angle voting): does the correspondence with
// displacement d = p - q vote for a coarse cell of [x0, x1] x [y0, y1] by the
// per-cell rule of Sec. IV-A (a corner in the closed disk, corners with
// F <= 0 and with F >= 0)?  Vertex values are formed in the same order as the
// accumulator's: W = ((u u) + (v v)) - 1, F = (c W) + 2 ((a u) + (b v)).  Each
// row of cells is swept left to right, reusing the shared edge.
__device__ __forceinline__ void gate_vertex(float a, float b, float c, float u, float v, float& W, float& F) {
    float uu = u * u;
    float vv = v * v;
    W = (uu + vv) - 1.0f;
    float cw = c * W;
    float au = a * u;
    float bv = b * v;
    float t = au + bv;
    float t2 = 2.0f * t;
    F = cw + t2;
}

__device__ bool window_hit(const float* p, const float* q, int G, uint32_t cell, int w) {
    const float a = p[0] - q[0], b = p[1] - q[1], c = p[2] - q[2];
    if (!(isfinite(a) && isfinite(b) && isfinite(c))) return false;
    if (a == 0.0f && b == 0.0f && c == 0.0f) return false;
    const int px = (int)(cell % (uint32_t)G), py = (int)(cell / (uint32_t)G);
    const int x0 = px - w < 0 ? 0 : px - w, x1 = px + w > G - 1 ? G - 1 : px + w;
    const int y0 = py - w < 0 ? 0 : py - w, y1 = py + w > G - 1 ? G - 1 : py + w;
    const float h = 2.0f / (float)G;
    for (int iy = y0; iy <= y1; ++iy) {
        const float v0 = -1.0f + (float)iy * h, v1 = -1.0f + (float)(iy + 1) * h;
        const float ul = -1.0f + (float)x0 * h;
        float w0, f0, w1, f1;
        gate_vertex(a, b, c, ul, v0, w0, f0);
        gate_vertex(a, b, c, ul, v1, w1, f1);
        for (int ix = x0; ix <= x1; ++ix) {
            const float ur = -1.0f + (float)(ix + 1) * h;
            float w2, f2, w3, f3;
            gate_vertex(a, b, c, ur, v0, w2, f2);
            gate_vertex(a, b, c, ur, v1, w3, f3);
            const bool disk = (w0 <= 0.0f) | (w1 <= 0.0f) | (w2 <= 0.0f) | (w3 <= 0.0f);
            const bool le = (f0 <= 0.0f) | (f1 <= 0.0f) | (f2 <= 0.0f) | (f3 <= 0.0f);
            const bool ge = (f0 >= 0.0f) | (f1 >= 0.0f) | (f2 >= 0.0f) | (f3 >= 0.0f);
            if (disk && le && ge) return true;
            w0 = w2;
            f0 = f2;
            w1 = w3;
            f1 = f3;
        }
    }
    return false;
}

// Histograms of every valid peak of the item's instance over correspondences
// [i0, i1) of that instance (those that pass the peak's gate when it is on).
__global__ __launch_bounds__(512) void k_angle_hist(const float* __restrict__ P, const float* __restrict__ Q,
                                                    int64_t N, const Inst* __restrict__ insts,
                                                    const int4* __restrict__ items, const PeakState* st,
                                                    uint32_t* __restrict__ hist_arena) {
    extern __shared__ __align__(16) uint32_t sm[];
    const int4 wi = items[blockIdx.x];
    const Inst& I = insts[wi.x];
    const int B = I.B, npk = I.npk, G = I.G, w = I.w;
    const bool gate = I.gate != 0;
    float* tc = reinterpret_cast<float*>(sm);
    float* ts = tc + B;
    uint32_t* hl = reinterpret_cast<uint32_t*>(ts + B);
    for (int t = threadIdx.x; t < B; t += blockDim.x) {
        tc[t] = I.tc[t];
        ts[t] = I.ts[t];
    }
    for (int t = threadIdx.x; t < npk * B; t += blockDim.x) hl[t] = 0u;
    float ax[kMaxPeaks][3];
    bool valid[kMaxPeaks];
    uint32_t pc[kMaxPeaks];
    for (int t = 0; t < kMaxPeaks; ++t) {
        valid[t] = t < npk && st[I.res_off + t].valid;
        ax[t][0] = valid[t] ? st[I.res_off + t].axis[0] : 0.0f;
        ax[t][1] = valid[t] ? st[I.res_off + t].axis[1] : 0.0f;
        ax[t][2] = valid[t] ? st[I.res_off + t].axis[2] : 0.0f;
        pc[t] = valid[t] ? st[I.res_off + t].peak_cell : 0u;
    }
    __syncthreads();
    for (int64_t li = wi.y + threadIdx.x; li < wi.z; li += blockDim.x) {
        const int64_t i = I.off + li;
        float p[3] = {P[i], P[N + i], P[2 * N + i]};
        float q[3] = {Q[i], Q[N + i], Q[2 * N + i]};
        for (int t = 0; t < npk; ++t) {
            if (!valid[t]) continue;
            if (gate && !window_hit(p, q, G, pc[t], w)) continue;
            float X, Y;
            angle_xy(ax[t], p, q, X, Y);
            int bin = angle_bin(tc, ts, B, X, Y);
            if (bin >= 0) atomicAdd(&hl[t * B + bin], 1u);
        }
    }
    __syncthreads();
    uint32_t* hist = hist_arena + I.hist_off;
    for (int t = threadIdx.x; t < npk * B; t += blockDim.x) {
        uint32_t v = hl[t];
        if (v) atomicAdd(&hist[t], v);
    }
}

// R = I + sin K + (1 - cos) K^2 with K = [r]x (Eq. (2)), row-major.
__device__ void rodrigues(const float* r, float ct, float sn, float* R) {
    float K[9] = {0.0f, -r[2], r[1], r[2], 0.0f, -r[0], -r[1], r[0], 0.0f};
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
            float a = sn * K[j * 3 + l];
            float bb = om * K2[j * 3 + l];
            R[j * 3 + l] = (delta + a) + bb;
        }
}

// Histogram peak (ties to the lowest bin), then R from the bin centre.  One
// block per instance.
__global__ __launch_bounds__(1024) void k_angle_peak(const uint32_t* __restrict__ hist_arena,
                                                     const Inst* __restrict__ insts, PeakState* st, int slot,
                                                     aoresp_result* res) {
    __shared__ unsigned long long red[16];
    const Inst& I = insts[blockIdx.x];
    if (slot >= I.npk) return;
    const PeakState& s = st[I.res_off + slot];
    aoresp_result& o = res[I.res_off + slot];
    const int B = I.B;
    unsigned long long best = 0ull;
    if (s.valid) {
        const uint32_t* h = hist_arena + I.hist_off + (size_t)slot * B;
        for (int c = threadIdx.x; c < B; c += blockDim.x) {
            unsigned long long k = ((unsigned long long)h[c] << 32) | (unsigned long long)(~(uint32_t)c);
            best = k > best ? k : best;
        }
    }
    best = block_max_u64(best, red);
    if (threadIdx.x != 0) return;
    o.grid = (uint32_t)I.G;
    o.n_inliers = 0u;
    if (!s.valid) {
        for (int j = 0; j < 9; ++j) o.R[j] = (j % 4 == 0) ? 1.0f : 0.0f;
        o.axis[0] = o.axis[1] = o.axis[2] = 0.0f;
        o.angle = 0.0f;
        o.peak_cell = o.fine_cell = o.angle_bin = 0u;
        o.axis_votes = o.fine_votes = o.angle_votes = 0u;
        return;
    }
    uint32_t bin = ~(uint32_t)(best & 0xFFFFFFFFull);
    rodrigues(s.axis, I.ct[bin], I.st[bin], o.R);
    o.axis[0] = s.axis[0];
    o.axis[1] = s.axis[1];
    o.axis[2] = s.axis[2];
    o.angle = I.th[bin];
    o.peak_cell = s.peak_cell;
    o.fine_cell = s.fine_cell;
    o.angle_bin = bin;
    o.axis_votes = s.axis_votes;
    o.fine_votes = s.fine_votes;
    o.angle_votes = (uint32_t)(best >> 32);
}

// Coarse bin of window slot j (0, 1, 2 = k-1, k, k+1, cyclic) around bin k.
__device__ __forceinline__ int fine_slot_bin(int k, int j, int B) { return (k + j + B - 1) % B; }

// LDS of the fine pass: per peak and window slot, the F+1 boundary directions
// cF .. cF+F of the B*F table (cos and sin), then 3F counters per peak.
size_t angle_fine_lds_bytes(int npk, int F) {
    return (size_t)npk * 3 * (size_t)(F + 1) * 8 + (size_t)npk * 3 * (size_t)F * 4;
}

// Fine angle votes.  With the boundary predicate monotone in the boundary
// index, a direction lies in coarse slot c's fine bins [cF, (c+1)F) iff
// boundary cF is at or below it (always, for c = 0) and boundary (c+1)F is
// not (always, for c = B-1); its fine bin is then cF plus the number of the
// slot's interior boundaries at or below it, found by binary search.  A slot
// that repeats a coarse bin (B < 3) counts the same votes again, as a window
// read of the full B*F histogram would.
__global__ __launch_bounds__(512) void k_angle_fine_hist(const float* __restrict__ P, const float* __restrict__ Q,
                                                         int64_t N, const Inst* __restrict__ insts,
                                                         const int4* __restrict__ items, const PeakState* st,
                                                         const aoresp_result* res,
                                                         uint32_t* __restrict__ hist_arena) {
    extern __shared__ __align__(16) uint32_t sm[];
    const int4 wi = items[blockIdx.x];
    const Inst& I = insts[wi.x];
    const int F = I.F;
    if (F <= 1) return;
    const int B = I.B, npk = I.npk, G = I.G, w = I.w, BF = B * F, nb = F + 1;
    const bool gate = I.gate != 0;
    float* bc = reinterpret_cast<float*>(sm);
    float* bs = bc + (size_t)npk * 3 * nb;
    uint32_t* hl = reinterpret_cast<uint32_t*>(bs + (size_t)npk * 3 * nb);
    float ax[kMaxPeaks][3];
    bool valid[kMaxPeaks];
    uint32_t pc[kMaxPeaks];
    int kb[kMaxPeaks];
    for (int t = 0; t < kMaxPeaks; ++t) {
        valid[t] = t < npk && st[I.res_off + t].valid;
        ax[t][0] = valid[t] ? st[I.res_off + t].axis[0] : 0.0f;
        ax[t][1] = valid[t] ? st[I.res_off + t].axis[1] : 0.0f;
        ax[t][2] = valid[t] ? st[I.res_off + t].axis[2] : 0.0f;
        pc[t] = valid[t] ? st[I.res_off + t].peak_cell : 0u;
        kb[t] = valid[t] ? (int)res[I.res_off + t].angle_bin : 0;
    }
    for (int e = threadIdx.x; e < npk * 3 * nb; e += blockDim.x) {
        const int t = e / (3 * nb), j = (e / nb) % 3, m = e % nb;
        const int kt = t < npk ? (int)res[I.res_off + t].angle_bin : 0;
        const int g = fine_slot_bin(kt % B, j, B) * F + m;
        bc[e] = g < BF ? I.ftc[g] : 0.0f;
        bs[e] = g < BF ? I.fts[g] : 0.0f;
    }
    for (int e = threadIdx.x; e < npk * 3 * F; e += blockDim.x) hl[e] = 0u;
    __syncthreads();
    for (int64_t li = wi.y + threadIdx.x; li < wi.z; li += blockDim.x) {
        const int64_t i = I.off + li;
        float p[3] = {P[i], P[N + i], P[2 * N + i]};
        float q[3] = {Q[i], Q[N + i], Q[2 * N + i]};
        for (int t = 0; t < npk; ++t) {
            if (!valid[t]) continue;
            if (gate && !window_hit(p, q, G, pc[t], w)) continue;
            float X, Y;
            angle_xy(ax[t], p, q, X, Y);
            if (!(isfinite(X) && isfinite(Y))) continue;
            if (X == 0.0f && Y == 0.0f) continue;
            const int hv = half_plane(X, Y);
            for (int j = 0; j < 3; ++j) {
                const int c = fine_slot_bin(kb[t], j, B);
                const float* tc = bc + (size_t)(t * 3 + j) * nb;
                const float* ts = bs + (size_t)(t * 3 + j) * nb;
                if (c != 0 && !at_or_below(tc[0], ts[0], hv, X, Y)) continue;
                if (c != B - 1 && at_or_below(tc[F], ts[F], hv, X, Y)) continue;
                int lo = 0, hi = F - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (at_or_below(tc[mid], ts[mid], hv, X, Y)) lo = mid; else hi = mid - 1;
                }
                atomicAdd(&hl[(t * 3 + j) * F + lo], 1u);
            }
        }
    }
    __syncthreads();
    uint32_t* hist = hist_arena + I.fhist_off;
    for (int e = threadIdx.x; e < npk * 3 * F; e += blockDim.x) {
        const uint32_t v = hl[e];
        if (v) atomicAdd(&hist[e], v);
    }
}

// Argmax of the 3F window counters (ties to the first in window order); the
// fine bin's centre replaces the angle and R.  One block per instance.
__global__ __launch_bounds__(256) void k_angle_fine_peak(const uint32_t* __restrict__ hist_arena,
                                                         const Inst* __restrict__ insts, const PeakState* st, int slot,
                                                         aoresp_result* res) {
    __shared__ unsigned long long red[4];
    const Inst& I = insts[blockIdx.x];
    if (slot >= I.npk || I.F <= 1) return;
    const PeakState& s = st[I.res_off + slot];
    if (!s.valid) return;
    aoresp_result& o = res[I.res_off + slot];
    const int F = I.F, B = I.B, W3 = 3 * F;
    const uint32_t* h = hist_arena + I.fhist_off + (size_t)slot * W3;
    unsigned long long best = 0ull;
    for (int e = threadIdx.x; e < W3; e += blockDim.x) {
        unsigned long long k = ((unsigned long long)h[e] << 32) | (unsigned long long)(~(uint32_t)e);
        best = k > best ? k : best;
    }
    best = block_max_u64(best, red);
    if (threadIdx.x != 0) return;
    // keys carry ~index, so an all-zero window yields its first entry
    const int e = (int)~(uint32_t)(best & 0xFFFFFFFFull);
    const int jf = fine_slot_bin((int)o.angle_bin, e / F, B) * F + e % F;
    rodrigues(s.axis, I.fct[jf], I.fst[jf], o.R);
    o.angle = I.fth[jf];
    o.angle_fine_bin = (uint32_t)jf;
    o.angle_fine_votes = (uint32_t)(best >> 32);
}

// ||R p - q||^2 <= tau^2 per correspondence (Eq. (1)); masks[slot*N + i] if
// masks is non-null; counts land in res[..].n_inliers (one atomic per block
// and slot when the block lies in one instance, else one per wave or lane).
// Inlier counts: a block that lies inside one instance adds its count to one
// of kCountSlots partial counters of the result (chosen by block index), so
// that no single address takes one atomic per block; k_inliers_total sums
// the partials into the result.  Blocks that straddle two instances add per
// correspondence straight into the result.
// Squared residual ||R p - q||^2 of Eq. (1) in binary32, in the fixed order
// that decides inlier membership everywhere (mask, count, least squares).
__device__ __forceinline__ float residual2(const float* R, float p0, float p1, float p2, const float* qv) {
    float e[3];
    for (int j = 0; j < 3; ++j) {
        float t0 = R[j * 3 + 0] * p0;
        float t1 = R[j * 3 + 1] * p1;
        float t2 = R[j * 3 + 2] * p2;
        float sm = (t0 + t1) + t2;
        e[j] = sm - qv[j];
    }
    float e0 = e[0] * e[0];
    float e1 = e[1] * e[1];
    float e2 = e[2] * e[2];
    return (e0 + e1) + e2;
}

// One block per kInlierSub x 256 consecutive columns: the columns' inputs
// are loaded first, then each is tested against every peak of its instance.
constexpr int kInlierSub = 4;
__global__ __launch_bounds__(256) void k_inliers(const float* __restrict__ P, const float* __restrict__ Q,
                                                 int64_t N, const Inst* __restrict__ insts, int ninst,
                                                 const PeakState* st, aoresp_result* res,
                                                 uint8_t* __restrict__ masks, uint32_t* __restrict__ partial) {
    __shared__ uint32_t cnt[kMaxPeaks];
    const int64_t first = (int64_t)blockIdx.x * blockDim.x * kInlierSub;
    const int64_t last = min(first + (int64_t)blockDim.x * kInlierSub, N) - 1;
    const int bfirst = find_inst(insts, ninst, first);
    const bool block_uniform = find_inst(insts, ninst, last) == bfirst;
    if (threadIdx.x < kMaxPeaks) cnt[threadIdx.x] = 0u;
    __syncthreads();
    float pv[kInlierSub][3], qv[kInlierSub][3];
#pragma unroll
    for (int u = 0; u < kInlierSub; ++u) {
        const int64_t i = first + (int64_t)u * blockDim.x + threadIdx.x;
        const bool live = i < N;
        for (int k = 0; k < 3; ++k) {
            pv[u][k] = live ? P[k * N + i] : 0.0f;
            qv[u][k] = live ? Q[k * N + i] : 0.0f;
        }
    }
    const int npk = insts[bfirst].npk;
#pragma unroll
    for (int u = 0; u < kInlierSub; ++u) {
        const int64_t i = first + (int64_t)u * blockDim.x + threadIdx.x;
        const bool live = i < N;
        const int b = live ? (block_uniform ? bfirst : find_inst(insts, ninst, i)) : bfirst;
        const Inst& I = insts[b];
        const float tt = I.tau * I.tau;
        for (int t = 0; t < kMaxPeaks; ++t) {
            if (block_uniform && t >= npk) break;
            bool act = live && t < I.npk;
            if (!block_uniform && !__any(act)) break;
            uint8_t m = 0;
            if (act && I.n >= 2 && st[I.res_off + t].valid)
                m = residual2(res[I.res_off + t].R, pv[u][0], pv[u][1], pv[u][2], qv[u]) <= tt ? 1 : 0;
            if (act && masks) masks[(size_t)t * N + i] = m;
            if (block_uniform) {
                unsigned long long bal = __ballot(m != 0);
                if ((threadIdx.x & 63) == 0 && bal) atomicAdd(&cnt[t], (uint32_t)__popcll(bal));
            } else if (m) {
                atomicAdd(&res[I.res_off + t].n_inliers, 1u);
            }
        }
    }
    if (block_uniform) {
        __syncthreads();
        if (threadIdx.x < npk && cnt[threadIdx.x])
            atomicAdd(&partial[(size_t)(insts[bfirst].res_off + threadIdx.x) * kCountSlots +
                               (blockIdx.x & (kCountSlots - 1))],
                      cnt[threadIdx.x]);
    }
}

__global__ void k_inliers_total(const uint32_t* __restrict__ partial, int nres, aoresp_result* res) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nres) return;
    uint32_t sum = 0u;
    for (int k = 0; k < kCountSlots; ++k) sum += partial[(size_t)r * kCountSlots + k];
    res[r].n_inliers += sum;
}

// --------------------------------------------------------------------------
// Least-squares rotation on the inlier set
// --------------------------------------------------------------------------

// Sum of kLsWords doubles over a 256-thread block, in a fixed order.
__device__ __forceinline__ void block_sum_ls(double* v, double (*red)[256]) {
    const int t = threadIdx.x;
    for (int k = 0; k < kLsWords; ++k) red[k][t] = v[k];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
            for (int k = 0; k < kLsWords; ++k) red[k][t] += red[k][t + h];
        __syncthreads();
    }
    for (int k = 0; k < kLsWords; ++k) v[k] = red[k][0];
}

// Per correspondence item: S_ab = sum p_a q_b over the inliers of slot `slot`
// (the residual test of the inlier mask), and their count; each thread sums
// its columns in order, then the block in a fixed tree.
__global__ __launch_bounds__(256) void k_ls_accum(const float* __restrict__ P, const float* __restrict__ Q,
                                                  int64_t N, const Inst* __restrict__ insts,
                                                  const int4* __restrict__ items, const PeakState* st,
                                                  const aoresp_result* res, int slot, double* __restrict__ partial) {
    __shared__ double red[kLsWords][256];
    const int4 wi = items[blockIdx.x];
    const Inst& I = insts[wi.x];
    double acc[kLsWords];
    for (int k = 0; k < kLsWords; ++k) acc[k] = 0.0;
    if (slot < I.npk && I.n >= 2 && st[I.res_off + slot].valid) {
        float R[9];
        for (int k = 0; k < 9; ++k) R[k] = res[I.res_off + slot].R[k];
        const float tt = I.tau * I.tau;
        for (int64_t li = wi.y + threadIdx.x; li < wi.z; li += blockDim.x) {
            const int64_t i = I.off + li;
            const float p0 = P[i], p1 = P[N + i], p2 = P[2 * N + i];
            const float qv[3] = {Q[i], Q[N + i], Q[2 * N + i]};
            if (!(residual2(R, p0, p1, p2, qv) <= tt)) continue;
            const double pd[3] = {p0, p1, p2};
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) acc[3 * a + b] += pd[a] * (double)qv[b];
            acc[9] += 1.0;
        }
    }
    block_sum_ls(acc, red);
    if (threadIdx.x < kLsWords) partial[(size_t)blockIdx.x * kLsWords + threadIdx.x] = acc[threadIdx.x];
}

// Per instance: the sums of its items in a fixed order, then the rotation
// (ls_rotation_from_sums).  Fewer than three inliers (or an invalid peak):
// R_ls = R.
__global__ __launch_bounds__(256) void k_ls_finish(const Inst* __restrict__ insts, const double* __restrict__ partial,
                                                   const PeakState* st, aoresp_result* res, int slot) {
    __shared__ double red[kLsWords][256];
    const Inst& I = insts[blockIdx.x];
    if (slot >= I.npk) return;
    double acc[kLsWords];
    for (int k = 0; k < kLsWords; ++k) acc[k] = 0.0;
    for (int it = threadIdx.x; it < I.nitems; it += blockDim.x)
        for (int k = 0; k < kLsWords; ++k) acc[k] += partial[(size_t)(I.item0 + it) * kLsWords + k];
    block_sum_ls(acc, red);
    if (threadIdx.x != 0) return;
    aoresp_result& o = res[I.res_off + slot];
    if (!st[I.res_off + slot].valid || I.n < 2 || acc[9] < 3.0) {
        for (int k = 0; k < 9; ++k) o.R_ls[k] = o.R[k];
        return;
    }
    ls_rotation_from_sums(acc, o.R_ls);
}

__global__ void k_zero_u32(uint32_t* p, size_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Every span of the list zeroed by one grid-stride pass.
__global__ void k_zero_list(ZeroList zl) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int k = 0; k < zl.count; ++k) {
        uint32_t* p = zl.ptr[k];
        const size_t n = zl.words[k];
        for (size_t i = t0; i < n; i += stride) p[i] = 0u;
    }
}

// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------

size_t coarse_lds_bytes() {
    // tile (bw / 2 line pairs of G + 1 words, bw <= 256) + per-wave rings
    // (u32) + sink row + in-disk limits (2 x int16 per band line, <= 256 lines)
    return (size_t)kTileWords * 4 + (size_t)(kVoteThreads / 64) * (kRingBody + kRingLine) * 4 + 2 * 2 * 256;
}

static void set_lds_limit(const void* fn) {
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess)
        (void)hipGetLastError();
}

void init_kernel_attributes() {
    // the kernels that take more than the default dynamic LDS; done once per
    // device before any launch (and so outside any stream capture)
    set_lds_limit((const void*)k_vote);
    set_lds_limit((const void*)k_local_max);
    set_lds_limit((const void*)k_fine_vote);
    set_lds_limit((const void*)k_angle_hist);
    set_lds_limit((const void*)k_angle_fine_hist);
    set_lds_limit((const void*)k_sample_vote);
    set_lds_limit((const void*)k_sample_setup);
}

void launch_zero_list(const ZeroList& zl, hipStream_t s) {
    size_t most = 0;
    for (int k = 0; k < zl.count; ++k) most = zl.words[k] > most ? zl.words[k] : most;
    if (!most) return;
    size_t blocks = (most + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero_list, dim3((unsigned)blocks), dim3(256), 0, s, zl);
}

void launch_zero_u32(uint32_t* p, size_t count, hipStream_t s) {
    if (!count) return;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, count);
}

void launch_arc_setup(const float* P, const float* Q, int64_t N, const Inst* insts, int ninst, ArcRecs recs,
                      hipStream_t s) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_arc_setup, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, P, Q, N, insts, ninst, recs);
}

void launch_vote(ArcRecs recs, const Inst* insts, const int4* items, VoteQueues q, uint32_t* counters,
                 uint32_t* grid_arena, uint32_t* err, int blocks, hipStream_t s) {
    const int nitems = q.first[kVoteQueues];
    if (nitems <= 0) return;
    if (blocks > nitems) blocks = nitems;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_vote, dim3((unsigned)blocks), dim3(kVoteThreads), coarse_lds_bytes(), s, recs, insts, items,
                       q, counters, grid_arena, err);
}

void launch_local_max(const uint32_t* grid_arena, const Inst* insts, const int4* items, int nitems, uint32_t* lmax,
                      int maxG, hipStream_t s) {
    if (nitems <= 0) return;
    hipLaunchKernelGGL(k_local_max, dim3((unsigned)nitems, (unsigned)((maxG + 63) / 64)), dim3(256),
                       local_max_lds_bytes(), s, grid_arena, insts, items, lmax);
}

void launch_peak(const uint32_t* grid_arena, const Inst* insts, const int4* items, int nitems, const PeakState* st,
                 int slot, const uint32_t* lmax, unsigned long long* keys, hipStream_t s) {
    if (nitems <= 0) return;
    hipLaunchKernelGGL(k_peak, dim3((unsigned)nitems), dim3(256), 0, s, grid_arena, insts, items, st, slot, lmax,
                       keys);
}

void launch_peak_finish(const Inst* insts, int ninst, const unsigned long long* keys, PeakState* st, int slot,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_peak_finish, dim3((unsigned)((ninst + 63) / 64)), dim3(64), 0, s, insts, ninst, keys, st,
                       slot);
}

void launch_fine_vote(ArcRecs recs, const Inst* insts, const int4* items, int nitems, const PeakState* st, int slot,
                      uint32_t* fine_arena, uint32_t* err, int maxM, hipStream_t s) {
    if (nitems <= 0 || maxM <= 0) return;
    hipLaunchKernelGGL(k_fine_vote, dim3((unsigned)nitems), dim3(kFineThreads), fine_lds_bytes(maxM), s, recs, insts,
                       items, st, slot, fine_arena, err);
}

void launch_fine_peak(const uint32_t* fine_arena, const Inst* insts, int ninst, PeakState* st, int slot,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_fine_peak, dim3((unsigned)ninst), dim3(1024), 0, s, fine_arena, insts, st, slot);
}

SampleLayout sample_plan(int G, int J, int64_t n) {
    SampleLayout L;
    const int64_t GG = (int64_t)G * G;
    const auto round16 = [](int64_t x) { return (x + 15) / 16 * 16; };
    // 16-bit counters when one item cannot carry a counter: the samples one
    // circle puts in one cell lie on an arc inside the cell, shorter than
    // 1.01 times its diagonal sqrt(2) h (a circle of radius >= 1 through a cell
    // of side h = 2/G <= 1/32).  Consecutive southern samples are at least
    // 0.495 dtheta apart in the plane (dtheta = 2 pi / J): on the southern half
    // the projection scales lengths by 1/(1 - s_z) >= 1/2, and for J >= 64 the
    // chord of one sample step is within 1% of its arc, on the sphere and in
    // the plane.  So a cell takes at most
    // 1 + 1.01 sqrt(2) h / (0.495 dtheta) = 1 + 0.919 J / G samples per
    // circle; spc below uses the larger 1 + ceil(1.01 J / G), and an item of
    // at most 65535 / spc circles cannot overflow.
    const int64_t spc = 1 + (int64_t)std::ceil(1.01 * (double)J / (double)G);
    const int64_t cap16 = (65535 / spc) / 16 * 16;
    if (J >= 64 && cap16 >= 1024) {
        int64_t ch = round16((n + 31) / 32);
        ch = ch < 2048 ? 2048 : ch;
        ch = ch < cap16 ? ch : cap16;
        const int64_t nch = n > 0 ? (n + ch - 1) / ch : 0;
        const int64_t cells = GG < 65536 ? GG : 65536;
        if (nch * (GG / 2) <= ((int64_t)1 << 27)) {
            L.half = 1;
            L.bw = (int)(cells / G);
            L.chunk = ch;
            L.part_words = nch * (GG / 2);
            // rows of G/2 + 1 words (one pad), two more rows (rows -1 and G
            // in the first and the last band), one word before
            const size_t tile = ((size_t)(cells / G) + 2) * ((size_t)G * 2 + 4) + 4;
            L.dirs_lds = tile + (size_t)J * 8 <= 160 * 1024 ? 1 : 0;
            L.lds_bytes = tile + (L.dirs_lds ? (size_t)J * 8 : 0);
            return L;
        }
    }
    // 32-bit counters: at most 32 chunks, and at most 2^27 partial words
    int64_t maxch = ((int64_t)1 << 27) / GG;
    maxch = maxch < 1 ? 1 : (maxch > 32 ? 32 : maxch);
    int64_t ch = (n + maxch - 1) / maxch;
    ch = ch < 2048 ? 2048 : round16(ch);
    const int64_t cells = GG < kSampleTile ? GG : kSampleTile;
    L.half = 0;
    L.bw = (int)(cells / G);
    L.chunk = ch;
    L.part_words = (n > 0 ? (n + ch - 1) / ch : 0) * GG;
    const size_t tile = (size_t)cells * 4 + (size_t)(cells / G) * 4;   // + one pad word per row
    L.dirs_lds = tile + (size_t)J * 8 <= 160 * 1024 ? 1 : 0;
    L.lds_bytes = tile + (L.dirs_lds ? (size_t)J * 8 : 0);
    return L;
}

void launch_sample_vote(const float* P, const float* Q, int64_t N, const Inst* insts, const int4* setup_items,
                        int nsetup, const int4* band_items, int nband, const int4* cell_items, int ncell,
                        uint32_t* recs, uint32_t* part, uint32_t* grid_arena, size_t lds_bytes, hipStream_t s) {
    if (nband <= 0) return;
    // room for the direction tables of the largest J staged in LDS (instances
    // with a larger J read them from global memory)
    const size_t setup_lds = (size_t)kSetupLdsDirs * 2 * sizeof(float);
    hipLaunchKernelGGL(k_sample_setup, dim3((unsigned)nsetup), dim3(256), setup_lds, s, P, Q, N, insts, setup_items,
                       recs);
    hipLaunchKernelGGL(k_sample_vote, dim3((unsigned)nband), dim3(1024), lds_bytes, s, insts, band_items, recs, part);
    hipLaunchKernelGGL(k_sample_reduce, dim3((unsigned)ncell, 32), dim3(256), 0, s, insts, cell_items, part,
                       grid_arena);
}

void launch_angle_hist(const float* P, const float* Q, int64_t N, const Inst* insts, const int4* items, int nitems,
                       const PeakState* st, uint32_t* hist_arena, size_t lds_bytes, hipStream_t s) {
    if (nitems <= 0) return;
    hipLaunchKernelGGL(k_angle_hist, dim3((unsigned)nitems), dim3(512), lds_bytes, s, P, Q, N, insts, items, st,
                       hist_arena);
}

void launch_angle_peak(const uint32_t* hist_arena, const Inst* insts, int ninst, PeakState* st, int slot,
                       aoresp_result* res, hipStream_t s) {
    hipLaunchKernelGGL(k_angle_peak, dim3((unsigned)ninst), dim3(1024), 0, s, hist_arena, insts, st, slot, res);
}

void launch_angle_fine_hist(const float* P, const float* Q, int64_t N, const Inst* insts, const int4* items,
                            int nitems, const PeakState* st, const aoresp_result* res, uint32_t* hist_arena,
                            size_t lds_bytes, hipStream_t s) {
    if (nitems <= 0 || lds_bytes == 0) return;
    hipLaunchKernelGGL(k_angle_fine_hist, dim3((unsigned)nitems), dim3(512), lds_bytes, s, P, Q, N, insts, items, st,
                       res, hist_arena);
}

void launch_angle_fine_peak(const uint32_t* hist_arena, const Inst* insts, int ninst, const PeakState* st, int slot,
                            aoresp_result* res, hipStream_t s) {
    if (ninst <= 0) return;
    hipLaunchKernelGGL(k_angle_fine_peak, dim3((unsigned)ninst), dim3(256), 0, s, hist_arena, insts, st, slot, res);
}

void launch_ls_accum(const float* P, const float* Q, int64_t N, const Inst* insts, const int4* items, int nitems,
                     const PeakState* st, const aoresp_result* res, int slot, double* partial, hipStream_t s) {
    if (nitems <= 0) return;
    hipLaunchKernelGGL(k_ls_accum, dim3((unsigned)nitems), dim3(256), 0, s, P, Q, N, insts, items, st, res, slot,
                       partial);
}

void launch_ls_finish(const Inst* insts, int ninst, const double* partial, const PeakState* st, aoresp_result* res,
                      int slot, hipStream_t s) {
    if (ninst <= 0) return;
    hipLaunchKernelGGL(k_ls_finish, dim3((unsigned)ninst), dim3(256), 0, s, insts, partial, st, res, slot);
}

void launch_inliers(const float* P, const float* Q, int64_t N, const Inst* insts, int ninst, const PeakState* st,
                    aoresp_result* res, int nres, uint8_t* masks, uint32_t* partial, hipStream_t s) {
    if (N <= 0) return;
    const int64_t per_block = 256 * kInlierSub;
    hipLaunchKernelGGL(k_inliers, dim3((unsigned)((N + per_block - 1) / per_block)), dim3(256), 0, s, P, Q, N, insts,
                       ninst, st, res, masks, partial);
    hipLaunchKernelGGL(k_inliers_total, dim3((unsigned)((nres + 63) / 64)), dim3(64), 0, s, partial, nres, res);
}

}  // namespace aoresp
