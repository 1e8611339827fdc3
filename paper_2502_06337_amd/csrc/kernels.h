// Internal interface between the HIP kernels (kernels.hip) and the host
// runtime of libaoresp.  Not part of the public C ABI (include/aoresp.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/aoresp.h"

namespace aoresp {

constexpr uint32_t kFlagDegenerate = 1u;  // d = 0 or non-finite: no axis vote
constexpr uint32_t kFlagRisky = 2u;       // max |d_k| outside [2^-100, 2^120]: exhaustive cell test
constexpr uint32_t kFlagLine = 4u;        // c == 0: the projected curve is a line

constexpr int kMaxPeaks = 8;
constexpr int kTileCells = 32768;         // u32 cells of one coarse LDS band (128 KiB)

// Per-correspondence records of the setup kernel (SoA, n entries each).
//  abc : displacement (a, b, c) negated if needed so that c >= 0; .w = flags.
//  colp: vertex-column ranges [s, e] of the four column-mode octants
//        (lower root left / right of the bottom point, upper root left / right
//        of the top point), each packed as int16 s | int16 e << 16.
//  rowp: vertex-row ranges of the four row-mode octants (lower u-root below /
//        above the left point, upper u-root below / above the right point).
//  clip: (ja, jb): lower-u-root cells need column < ja, upper ones >= jb.
struct ArcRecs {
    float4* abc;
    int4* colp;
    int4* rowp;
    int32_t* clip;
};

struct FineWin {
    float U0, V0, hx, hy;
    int nx, ny;
};

// Device-side state of one peak (axis hypothesis).
struct PeakState {
    int valid;
    uint32_t peak_cell, axis_votes;
    uint32_t fine_cell, fine_votes;
    float axis[3];
    FineWin win;
};

int coarse_band_width(int G);
size_t coarse_lds_bytes(int G);

void launch_zero_u32(uint32_t* p, size_t count, hipStream_t s);
void launch_arc_setup(const float* P, const float* Q, int64_t n, int G, ArcRecs recs, hipStream_t s);
void launch_coarse_vote(ArcRecs recs, int64_t n, int G, const int16_t* disk, uint32_t* grid, uint32_t* err,
                        int chunks, hipStream_t s);
void launch_peak(const uint32_t* a, int G, int64_t count, const PeakState* prev, int prev_count, int rad,
                 unsigned long long* key, hipStream_t s);
void launch_peak_finish(const unsigned long long* key, int G, int M, int w, PeakState* st, int slot,
                        hipStream_t s);
void launch_fine_vote(ArcRecs recs, int64_t n, int M, const PeakState* st, int slot, uint32_t* fine, uint32_t* err,
                      hipStream_t s);
void launch_fine_peak(const uint32_t* fine, int G, int M, PeakState* st, int slot, hipStream_t s);
void launch_angle_hist(const float* P, const float* Q, int64_t n, const PeakState* st, int npk, int B,
                       const float* tc, const float* ts, uint32_t* hist, hipStream_t s);
void launch_angle_peak(const uint32_t* hist, int B, const float* cth, const float* cct, const float* cst,
                       PeakState* st, int slot, int G, aoresp_result* out, hipStream_t s);
void launch_inliers(const float* P, const float* Q, int64_t n, const PeakState* st, int npk, float tau,
                    aoresp_result* out, uint8_t* masks, hipStream_t s);

}  // namespace aoresp
