// HIP kernels of the stereographic-projection rotation vote (gfx950).
//
// Pipeline of one solve (paper: Algorithm 1; Sec. IV):
//   k_arc_setup      per correspondence: displacement, quarter/octant pieces
//   k_vote_bands     coarse accumulator: column pass over vertical LDS bands,
//                    row pass over horizontal LDS bands (Sec. IV-A, Fig. 3(c))
//   k_peak           argmax (ties to the lowest index), optional suppression
//                    of earlier peaks for multi-model estimation (Sec. IV-D)
//   k_fine_vote      refinement accumulator around each peak
//   k_fine_peak      refined cell, inverse projection to the axis (Eq. (8))
//   k_angle_hist     signed angle of every pair about each axis, binned
//                    (Sec. IV-B, Eq. (10))
//   k_angle_peak     histogram peak, Rodrigues rotation (Eq. (2))
//   k_inliers        residual mask against Eq. (1)
// Nothing here is a dense contraction; the vote kernels are bound by VALU
// work per vote and LDS atomics, the rest by HBM streaming.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "geometry.h"
#include "kernels.h"
#include "walker.h"

namespace aoresp {

__global__ __launch_bounds__(256) void k_arc_setup(const float* __restrict__ P, const float* __restrict__ Q,
                                                   int64_t n, int G, ArcRecs R) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float a = P[i] - Q[i];
    float b = P[n + i] - Q[n + i];
    float c = P[2 * n + i] - Q[2 * n + i];
    uint32_t fl = classify(a, b, c);
    if (!(fl & kFlagDegenerate) && c < 0.0f) { a = -a; b = -b; c = -c; }
    const int E = pack_range(0, 0);
    int4 colp = make_int4(E, E, E, E), rowp = colp;
    int32_t clip = pack_range(0, 0);
    if (!(fl & (kFlagDegenerate | kFlagRisky))) {
        double h = 2.0 / G;
        circle_pieces(a, b, c, (fl & kFlagLine) != 0, -1.0, h, G, -1.0, h, G, 2.0 * h, colp, rowp, clip);
    }
    R.abc[i] = make_float4(a, b, c, __uint_as_float(fl));
    R.colp[i] = colp;
    R.rowp[i] = rowp;
    R.clip[i] = clip;
}

// --------------------------------------------------------------------------
// Coarse accumulator: banded LDS tiles
// --------------------------------------------------------------------------

struct CoarseEmit {
    uint32_t* tile;
    const int16_t* disk;   // 2*G: in-disk cross range per cell line (symmetric grid)
    int mode;              // 0: column pass (tile rows = G, cols = bw), 1: row pass
    int band0;             // first along index of the band
    int bw;                // band width (along)
    int G;
    int clo, chi;          // row pass: allowed cross range from the quarter clip
    __device__ __forceinline__ void operator()(int j, int klo, int khi) {
        int dlo = disk[2 * j], dhi = disk[2 * j + 1];
        if (klo < dlo) klo = dlo;
        if (khi > dhi) khi = dhi;
        if (klo < clo) klo = clo;
        if (khi > chi) khi = chi;
        if (mode == 0) {
            uint32_t* t = tile + (j - band0);
            for (int k = klo; k <= khi; ++k) atomicAdd(t + k * bw, 1u);
        } else {
            uint32_t* t = tile + (size_t)(j - band0) * G;
            for (int k = klo; k <= khi; ++k) atomicAdd(t + k, 1u);
        }
    }
};

__global__ __launch_bounds__(1024) void k_vote_bands(const ArcRecs R, int64_t n, int G, int bw, int nbands,
                                                     int chunks, const int16_t* __restrict__ disk,
                                                     uint32_t* __restrict__ grid, uint32_t* __restrict__ err) {
    extern __shared__ __align__(16) uint32_t smem[];
    __shared__ uint32_t qcount, rcount;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    int blk = blockIdx.x;
    const int mode = blk / (nbands * chunks);
    blk -= mode * nbands * chunks;
    const int band = blk / chunks;
    const int chunk = blk - band * chunks;
    const int band0 = band * bw;
    const int bwb = (band0 + bw <= G) ? bw : (G - band0);
    const int tile_cells = G * bwb;
    uint32_t* tile = smem;
    uint16_t* queue = reinterpret_cast<uint16_t*>(smem + (size_t)G * bw);
    uint16_t* risky = queue + 4 * 1024;

    for (int t = tid; t < tile_cells; t += nthr) tile[t] = 0u;

    const int64_t per = (n + chunks - 1) / chunks;
    const int64_t i0 = (int64_t)chunk * per;
    const int64_t i1 = (i0 + per < n) ? (i0 + per) : n;
    const float h = 2.0f / (float)G;
    uint32_t bad = 0;

    for (int64_t base = i0; base < i1; base += nthr) {
        if (tid == 0) {
            qcount = 0u;
            rcount = 0u;
        }
        __syncthreads();
        int64_t i = base + tid;
        if (i < i1) {
            uint32_t fl = __float_as_uint(R.abc[i].w);
            if (!(fl & kFlagDegenerate)) {
                if (fl & kFlagRisky) {
                    if (mode == 0) risky[atomicAdd(&rcount, 1u)] = (uint16_t)tid;
                } else {
                    int4 pc = mode == 0 ? R.colp[i] : R.rowp[i];
                    int32_t pcs[4] = {pc.x, pc.y, pc.z, pc.w};
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        int s, e;
                        unpack_range(pcs[p], s, e);
                        int cs = s > band0 ? s : band0;
                        int ce = e < band0 + bwb ? e : band0 + bwb;
                        if (cs < ce) queue[atomicAdd(&qcount, 1u)] = (uint16_t)((tid << 2) | p);
                    }
                }
            }
        }
        __syncthreads();
        const int qn = (int)qcount;
        for (int t = tid; t < qn; t += nthr) {
            int ent = queue[t];
            int64_t ai = base + (ent >> 2);
            int p = ent & 3;
            float4 abc = R.abc[ai];
            int32_t pr;
            int4 pc = mode == 0 ? R.colp[ai] : R.rowp[ai];
            pr = p == 0 ? pc.x : (p == 1 ? pc.y : (p == 2 ? pc.z : pc.w));
            int s, e;
            unpack_range(pr, s, e);
            int cs = s > band0 ? s : band0;
            int ce = e < band0 + bwb ? e : band0 + bwb;
            CoarseEmit em{tile, disk, mode, band0, bwb, G, 0, G - 1};
            int sel = p >> 1;
            if (mode == 1) {
                int ja, jb;
                unpack_range(R.clip[ai], ja, jb);
                if (sel == 0) em.chi = ja - 1; else em.clo = jb;
                walk_piece(abc.y, abc.x, abc.z, sel, -1.0f, h, -1.0f, h, cs, ce, em, bad);
            } else {
                walk_piece(abc.x, abc.y, abc.z, sel, -1.0f, h, -1.0f, h, cs, ce, em, bad);
            }
        }
        if (mode == 0) {
            const int rn = (int)rcount;
            for (int r = 0; r < rn; ++r) {
                float4 abc = R.abc[base + risky[r]];
                for (int t = tid; t < tile_cells; t += nthr) {
                    int k = t / bwb;
                    int j = band0 + (t - k * bwb);
                    if (k < disk[2 * j] || k > disk[2 * j + 1]) continue;
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
                    if (le && ge) atomicAdd(&tile[t], 1u);
                }
            }
        }
        __syncthreads();
    }
    if (bad) atomicOr(err, 1u);
    // flush the band into the global accumulator
    for (int t = tid; t < tile_cells; t += nthr) {
        uint32_t v = tile[t];
        if (!v) continue;
        size_t gi;
        if (mode == 0) {
            int k = t / bwb;
            gi = (size_t)k * G + band0 + (t - k * bwb);
        } else {
            gi = (size_t)band0 * G + t;
        }
        atomicAdd(&grid[gi], v);
    }
}

// --------------------------------------------------------------------------
// Peaks
// --------------------------------------------------------------------------

// Suppression test of multi-model peak search: integer disk of radius rad
// around an earlier peak, and the disk of radius rad*h around the projection
// -(u, v)/(u^2 + v^2) of the antipodal axis.  Same binary32 steps as the
// definition: s = u*u + v*v, p = (-u)/s, d2 = du*du + dv*dv <= (rad*h)^2.
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

__device__ __forceinline__ unsigned long long peak_key(uint32_t v, uint32_t idx) {
    return ((unsigned long long)v << 32) | (unsigned long long)(~idx);
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(k, off, 64);
        k = o > k ? o : k;
    }
    return k;
}

// Argmax of a u32 array (ties to the lowest index) into *key (pre-zeroed).
// If prev_count > 0, cells suppressed by any earlier peak are skipped.
__global__ __launch_bounds__(256) void k_peak(const uint32_t* __restrict__ a, int G, int64_t count,
                                              const PeakState* prev, int prev_count, int rad,
                                              unsigned long long* key) {
    __shared__ unsigned long long red[4];
    unsigned long long best = 0ull;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < count;
         c += (int64_t)gridDim.x * blockDim.x) {
        uint32_t v = a[c];
        if (v == 0u) continue;
        if (prev_count > 0) {
            int ix = (int)(c % G), iy = (int)(c / G);
            bool sup = false;
            for (int t = 0; t < prev_count && !sup; ++t) {
                uint32_t pc = prev[t].peak_cell;
                sup = suppressed(G, rad, (int)(pc % (uint32_t)G), (int)(pc / (uint32_t)G), ix, iy);
            }
            if (sup) continue;
        }
        unsigned long long k = peak_key(v, (uint32_t)c);
        best = k > best ? k : best;
    }
    best = wave_max_u64(best);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b = red[w] > b ? red[w] : b;
        if (b) atomicMax(key, b);
    }
}

// --------------------------------------------------------------------------
// Refinement window
// --------------------------------------------------------------------------

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

// Writes the peak cell/votes from key, and the refinement window.
__global__ void k_peak_finish(const unsigned long long* key, int G, int M, int w, PeakState* st, int slot) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    unsigned long long k = *key;
    PeakState& s = st[slot];
    s.valid = k != 0ull;
    s.peak_cell = k ? ~(uint32_t)(k & 0xFFFFFFFFull) : 0u;
    s.axis_votes = (uint32_t)(k >> 32);
    if (M > 0 && s.valid) window_of(G, M, w, s.peak_cell, s.win);
}

struct FineEmit {
    uint32_t* tile;
    int mode, M;
    float U0, V0, hx, hy;
    bool all_in;   // every cell of the window meets the disk
    __device__ __forceinline__ bool in_disk(int jx, int jy) const {
        float u0 = U0 + (float)jx * hx, u1 = U0 + (float)(jx + 1) * hx;
        float v0 = V0 + (float)jy * hy, v1 = V0 + (float)(jy + 1) * hy;
        float w00 = ((u0 * u0) + (v0 * v0)) - 1.0f;
        float w10 = ((u1 * u1) + (v0 * v0)) - 1.0f;
        float w01 = ((u0 * u0) + (v1 * v1)) - 1.0f;
        float w11 = ((u1 * u1) + (v1 * v1)) - 1.0f;
        return (w00 <= 0.0f) | (w10 <= 0.0f) | (w01 <= 0.0f) | (w11 <= 0.0f);
    }
    __device__ __forceinline__ void operator()(int j, int klo, int khi) {
        if (klo < 0) klo = 0;
        if (khi > M - 1) khi = M - 1;
        for (int k = klo; k <= khi; ++k) {
            int jx = mode == 0 ? j : k, jy = mode == 0 ? k : j;
            if (!all_in && !in_disk(jx, jy)) continue;
            atomicAdd(&tile[jy * M + jx], 1u);
        }
    }
};

// Fine accumulator of peak `slot`: every correspondence whose curve crosses
// the window walks it on the M x M fine grid (LDS), then flushes.
__global__ __launch_bounds__(256) void k_fine_vote(const ArcRecs R, int64_t n, int M, const PeakState* st,
                                                   int slot, uint32_t* __restrict__ fine,
                                                   uint32_t* __restrict__ err) {
    extern __shared__ __align__(16) uint32_t ftile[];
    const PeakState& s = st[slot];
    if (!s.valid) return;
    const FineWin fw = s.win;
    for (int t = threadIdx.x; t < M * M; t += blockDim.x) ftile[t] = 0u;
    __syncthreads();
    // The window is [U0, U0 + M hx] x [V0, V0 + M hy].  If its corner farthest
    // from the origin is inside the disk with room to spare, every fine cell
    // meets the disk and the per-cell test is skipped.
    double wu = (double)fw.hx * M, wv = (double)fw.hy * M;
    double ue = fmax(fabs((double)fw.U0), fabs((double)fw.U0 + wu));
    double ve = fmax(fabs((double)fw.V0), fabs((double)fw.V0 + wv));
    bool all_in = ue * ue + ve * ve < 1.0 - 1e-4;
    double Uc = (double)fw.U0 + 0.5 * wu, Vc = (double)fw.V0 + 0.5 * wv;
    double Rw = 0.5 * sqrt(wu * wu + wv * wv);
    uint32_t bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float4 abc = R.abc[i];
        uint32_t fl = __float_as_uint(abc.w);
        if (fl & kFlagDegenerate) continue;
        double a = abc.x, b = abc.y, c = abc.z;
        // Quick reject: over the window |F(x) - F(centre)| <= |grad F(centre)| Rw
        // + |c| Rw^2; if |F| stays above the binary32 error bound everywhere,
        // every vertex has the same sign and no fine cell is voted.
        if (!(fl & kFlagRisky)) {
            double Fc = c * (Uc * Uc + Vc * Vc - 1.0) + 2.0 * (a * Uc + b * Vc);
            double gx = 2.0 * (c * Uc + a), gy = 2.0 * (c * Vc + b);
            double bound = sqrt(gx * gx + gy * gy) * Rw + fabs(c) * Rw * Rw;
            double ebound = 2e-6 * (fabs(a) + fabs(b) + fabs(c));
            if (fabs(Fc) > 1.0001 * bound + ebound) continue;
        }
        FineEmit em{ftile, 0, M, fw.U0, fw.V0, fw.hx, fw.hy, all_in};
        if (fl & kFlagRisky) {
            for (int jy = 0; jy < M; ++jy)
                for (int jx = 0; jx < M; ++jx) {
                    if (!all_in && !em.in_disk(jx, jy)) continue;
                    float u0 = fw.U0 + (float)jx * fw.hx, u1 = fw.U0 + (float)(jx + 1) * fw.hx;
                    float v0 = fw.V0 + (float)jy * fw.hy, v1 = fw.V0 + (float)(jy + 1) * fw.hy;
                    float uu0 = u0 * u0, uu1 = u1 * u1, au0 = abc.x * u0, au1 = abc.x * u1;
                    float f0 = vertex_F(abc.y, abc.z, uu0, au0, v0);
                    float f1 = vertex_F(abc.y, abc.z, uu1, au1, v0);
                    float f2 = vertex_F(abc.y, abc.z, uu0, au0, v1);
                    float f3 = vertex_F(abc.y, abc.z, uu1, au1, v1);
                    bool le = (f0 <= 0.0f) | (f1 <= 0.0f) | (f2 <= 0.0f) | (f3 <= 0.0f);
                    bool ge = (f0 >= 0.0f) | (f1 >= 0.0f) | (f2 >= 0.0f) | (f3 >= 0.0f);
                    if (le && ge) atomicAdd(&ftile[jy * M + jx], 1u);
                }
            continue;
        }
        int4 colp, rowp;
        int32_t clip;
        circle_pieces(abc.x, abc.y, abc.z, (fl & kFlagLine) != 0, fw.U0, fw.hx, M, fw.V0, fw.hy, M,
                      2.0 * (double)(fw.hx > fw.hy ? fw.hx : fw.hy), colp, rowp, clip);
        int32_t cps[4] = {colp.x, colp.y, colp.z, colp.w};
        int32_t rps[4] = {rowp.x, rowp.y, rowp.z, rowp.w};
        int ja, jb;
        unpack_range(clip, ja, jb);
        for (int p = 0; p < 4; ++p) {
            int s0, e0;
            unpack_range(cps[p], s0, e0);
            if (s0 < e0) {
                em.mode = 0;
                walk_piece(abc.x, abc.y, abc.z, p >> 1, fw.U0, fw.hx, fw.V0, fw.hy, s0, e0, em, bad);
            }
        }
        for (int p = 0; p < 4; ++p) {
            int s0, e0;
            unpack_range(rps[p], s0, e0);
            if (s0 < e0) {
                // row pass cells restricted to columns < ja (lower u-root) or >= jb
                struct RowClipEmit {
                    FineEmit* f;
                    int lo, hi;
                    __device__ __forceinline__ void operator()(int j, int klo, int khi) {
                        if (klo < lo) klo = lo;
                        if (khi > hi) khi = hi;
                        (*f)(j, klo, khi);
                    }
                } rc{&em, (p >> 1) ? jb : -(1 << 20), (p >> 1) ? (1 << 20) : ja - 1};
                em.mode = 1;
                walk_piece(abc.y, abc.x, abc.z, p >> 1, fw.V0, fw.hy, fw.U0, fw.hx, s0, e0, rc, bad);
            }
        }
    }
    if (bad) atomicOr(err, 2u);
    __syncthreads();
    for (int t = threadIdx.x; t < M * M; t += blockDim.x) {
        uint32_t v = ftile[t];
        if (v) atomicAdd(&fine[t], v);
    }
}

// Fine argmax (single block), then the axis by inverse projection (Eq. (8)):
// s = u*u + v*v, den = 1 + s, r = (2u/den, 2v/den, (s - 1)/den).
__global__ __launch_bounds__(1024) void k_fine_peak(const uint32_t* __restrict__ fine, int G, int M,
                                                    PeakState* st, int slot) {
    __shared__ unsigned long long red[16];
    PeakState& s = st[slot];
    if (!s.valid) return;
    unsigned long long best = 0ull;
    if (M > 0) {
        for (int c = threadIdx.x; c < M * M; c += blockDim.x) {
            uint32_t v = fine[c];
            unsigned long long k = ((unsigned long long)v << 32) | (unsigned long long)(~(uint32_t)c);
            best = k > best ? k : best;
        }
        best = wave_max_u64(best);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    float u, v;
    if (M > 0) {
        unsigned long long b = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b = red[w] > b ? red[w] : b;
        uint32_t fc = ~(uint32_t)(b & 0xFFFFFFFFull);
        s.fine_cell = fc;
        s.fine_votes = (uint32_t)(b >> 32);
        int jx = (int)(fc % (uint32_t)M), jy = (int)(fc / (uint32_t)M);
        u = s.win.U0 + ((float)jx + 0.5f) * s.win.hx;
        v = s.win.V0 + ((float)jy + 0.5f) * s.win.hy;
    } else {
        s.fine_cell = 0u;
        s.fine_votes = 0u;
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
    int lo = 0, hi = B - 1;   // answer in [lo, hi]; k <= lo satisfied (k = 0 is vacuous)
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (at_or_below(tc[mid], ts[mid], hv, X, Y)) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Histograms for `npk` axes (one per peak) over all correspondences.
__global__ __launch_bounds__(512) void k_angle_hist(const float* __restrict__ P, const float* __restrict__ Q,
                                                    int64_t n, const PeakState* st, int npk, int B,
                                                    const float* __restrict__ tcg, const float* __restrict__ tsg,
                                                    uint32_t* __restrict__ hist) {
    extern __shared__ __align__(16) uint32_t sm[];
    float* tc = reinterpret_cast<float*>(sm);
    float* ts = tc + B;
    uint32_t* hl = reinterpret_cast<uint32_t*>(ts + B);
    for (int t = threadIdx.x; t < B; t += blockDim.x) {
        tc[t] = tcg[t];
        ts[t] = tsg[t];
    }
    for (int t = threadIdx.x; t < npk * B; t += blockDim.x) hl[t] = 0u;
    float ax[kMaxPeaks][3];
    bool valid[kMaxPeaks];
    for (int t = 0; t < npk; ++t) {
        valid[t] = st[t].valid;
        ax[t][0] = st[t].axis[0];
        ax[t][1] = st[t].axis[1];
        ax[t][2] = st[t].axis[2];
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float p[3] = {P[i], P[n + i], P[2 * n + i]};
        float q[3] = {Q[i], Q[n + i], Q[2 * n + i]};
        for (int t = 0; t < npk; ++t) {
            if (!valid[t]) continue;
            float X, Y;
            angle_xy(ax[t], p, q, X, Y);
            int bin = angle_bin(tc, ts, B, X, Y);
            if (bin >= 0) atomicAdd(&hl[t * B + bin], 1u);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < npk * B; t += blockDim.x) {
        uint32_t v = hl[t];
        if (v) atomicAdd(&hist[t], v);
    }
}

// Histogram peak (ties to the lowest bin), then R = I + sin K + (1 - cos) K^2
// with K = [r]x (Eq. (2)), written into the result of that peak.
__global__ __launch_bounds__(1024) void k_angle_peak(const uint32_t* __restrict__ hist, int B,
                                                     const float* __restrict__ cth, const float* __restrict__ cct,
                                                     const float* __restrict__ cst, PeakState* st, int slot,
                                                     int G, aoresp_result* out) {
    __shared__ unsigned long long red[16];
    PeakState& s = st[slot];
    aoresp_result& o = out[slot];
    unsigned long long best = 0ull;
    const uint32_t* h = hist + (size_t)slot * B;
    if (s.valid) {
        for (int c = threadIdx.x; c < B; c += blockDim.x) {
            unsigned long long k = ((unsigned long long)h[c] << 32) | (unsigned long long)(~(uint32_t)c);
            best = k > best ? k : best;
        }
    }
    best = wave_max_u64(best);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (!s.valid) {
        for (int j = 0; j < 9; ++j) o.R[j] = (j % 4 == 0) ? 1.0f : 0.0f;
        o.axis[0] = o.axis[1] = o.axis[2] = 0.0f;
        o.angle = 0.0f;
        o.grid = (uint32_t)G;
        o.peak_cell = o.fine_cell = o.angle_bin = 0u;
        o.axis_votes = o.fine_votes = o.angle_votes = o.n_inliers = 0u;
        return;
    }
    unsigned long long b = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b = red[w] > b ? red[w] : b;
    uint32_t bin = ~(uint32_t)(b & 0xFFFFFFFFull);
    float ct = cct[bin], sn = cst[bin];
    const float* r = s.axis;
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
            o.R[j * 3 + l] = (delta + a) + bb;
        }
    o.axis[0] = r[0];
    o.axis[1] = r[1];
    o.axis[2] = r[2];
    o.angle = cth[bin];
    o.grid = (uint32_t)G;
    o.peak_cell = s.peak_cell;
    o.fine_cell = s.fine_cell;
    o.angle_bin = bin;
    o.axis_votes = s.axis_votes;
    o.fine_votes = s.fine_votes;
    o.angle_votes = (uint32_t)(b >> 32);
    o.n_inliers = 0u;
}

// ||R p - q||^2 <= tau^2 per correspondence (Eq. (1)); masks is npk*n bytes
// or null; counts land in out[t].n_inliers.
__global__ __launch_bounds__(256) void k_inliers(const float* __restrict__ P, const float* __restrict__ Q,
                                                 int64_t n, const PeakState* st, int npk, float tau,
                                                 aoresp_result* out, uint8_t* __restrict__ masks) {
    __shared__ uint32_t cnt[kMaxPeaks];
    if (threadIdx.x < kMaxPeaks) cnt[threadIdx.x] = 0u;
    __syncthreads();
    float tt = tau * tau;
    for (int t = 0; t < npk; ++t) {
        bool valid = st[t].valid;
        float R[9];
        for (int j = 0; j < 9; ++j) R[j] = out[t].R[j];
        uint32_t local = 0;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * blockDim.x) {
            uint8_t m = 0;
            if (valid) {
                float p0 = P[i], p1 = P[n + i], p2 = P[2 * n + i];
                float q0 = Q[i], q1 = Q[n + i], q2 = Q[2 * n + i];
                float e[3];
                float qv[3] = {q0, q1, q2};
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
                float res2 = (e0 + e1) + e2;
                m = res2 <= tt ? 1 : 0;
            }
            if (masks) masks[(size_t)t * n + i] = m;
            local += m;
        }
        if (local) atomicAdd(&cnt[t], local);
    }
    __syncthreads();
    if (threadIdx.x < npk && cnt[threadIdx.x]) atomicAdd(&out[threadIdx.x].n_inliers, cnt[threadIdx.x]);
}

__global__ void k_zero_u32(uint32_t* p, size_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------

int coarse_band_width(int G) {
    int bw = kTileCells / G;
    if (bw > G) bw = G;
    if (bw < 1) bw = 1;
    return bw;
}

size_t coarse_lds_bytes(int G) {
    return (size_t)G * coarse_band_width(G) * 4 + 4 * 1024 * 2 + 1024 * 2;
}

void launch_zero_u32(uint32_t* p, size_t count, hipStream_t s) {
    if (!count) return;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, count);
}

void launch_arc_setup(const float* P, const float* Q, int64_t n, int G, ArcRecs recs, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_arc_setup, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, P, Q, n, G, recs);
}

void launch_coarse_vote(ArcRecs recs, int64_t n, int G, const int16_t* disk, uint32_t* grid, uint32_t* err,
                        int chunks, hipStream_t s) {
    if (n <= 0) return;
    int bw = coarse_band_width(G);
    int nbands = (G + bw - 1) / bw;
    if (chunks < 1) chunks = 1;
    size_t lds = coarse_lds_bytes(G);
    static bool attr = false;
    if (!attr) {
        if (hipFuncSetAttribute((const void*)k_vote_bands, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) !=
            hipSuccess)
            (void)hipGetLastError();
        attr = true;
    }
    unsigned blocks = (unsigned)(2 * nbands * chunks);
    hipLaunchKernelGGL(k_vote_bands, dim3(blocks), dim3(1024), lds, s, recs, n, G, bw, nbands, chunks, disk, grid,
                       err);
}

void launch_peak(const uint32_t* a, int G, int64_t count, const PeakState* prev, int prev_count, int rad,
                 unsigned long long* key, hipStream_t s) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_peak, dim3((unsigned)blocks), dim3(256), 0, s, a, G, count, prev, prev_count, rad, key);
}

void launch_peak_finish(const unsigned long long* key, int G, int M, int w, PeakState* st, int slot,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_peak_finish, dim3(1), dim3(64), 0, s, key, G, M, w, st, slot);
}

void launch_fine_vote(ArcRecs recs, int64_t n, int M, const PeakState* st, int slot, uint32_t* fine, uint32_t* err,
                      hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    static bool attr = false;
    if (!attr) {
        if (hipFuncSetAttribute((const void*)k_fine_vote, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) !=
            hipSuccess)
            (void)hipGetLastError();
        attr = true;
    }
    hipLaunchKernelGGL(k_fine_vote, dim3((unsigned)blocks), dim3(256), (size_t)M * M * 4, s, recs, n, M, st, slot,
                       fine, err);
}

void launch_fine_peak(const uint32_t* fine, int G, int M, PeakState* st, int slot, hipStream_t s) {
    hipLaunchKernelGGL(k_fine_peak, dim3(1), dim3(1024), 0, s, fine, G, M, st, slot);
}

void launch_angle_hist(const float* P, const float* Q, int64_t n, const PeakState* st, int npk, int B,
                       const float* tc, const float* ts, uint32_t* hist, hipStream_t s) {
    int64_t blocks = (n + 511) / 512;
    if (blocks > 512) blocks = 512;
    if (blocks < 1) blocks = 1;
    size_t lds = (size_t)B * 8 + (size_t)npk * B * 4;
    static bool attr = false;
    if (!attr) {
        if (hipFuncSetAttribute((const void*)k_angle_hist, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) !=
            hipSuccess)
            (void)hipGetLastError();
        attr = true;
    }
    hipLaunchKernelGGL(k_angle_hist, dim3((unsigned)blocks), dim3(512), lds, s, P, Q, n, st, npk, B, tc, ts, hist);
}

void launch_angle_peak(const uint32_t* hist, int B, const float* cth, const float* cct, const float* cst,
                       PeakState* st, int slot, int G, aoresp_result* out, hipStream_t s) {
    hipLaunchKernelGGL(k_angle_peak, dim3(1), dim3(1024), 0, s, hist, B, cth, cct, cst, st, slot, G, out);
}

void launch_inliers(const float* P, const float* Q, int64_t n, const PeakState* st, int npk, float tau,
                    aoresp_result* out, uint8_t* masks, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_inliers, dim3((unsigned)blocks), dim3(256), 0, s, P, Q, n, st, npk, tau, out, masks);
}

}  // namespace aoresp
