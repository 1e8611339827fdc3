// Internal interface between the HIP kernels (kernels.hip) and the host
// runtime of libaoresp.  Not part of the public C ABI (include/aoresp.h).
//
// Every kernel works on a batch of independent instances described by an
// instance table; a single solve is a batch of one.  Per-correspondence data
// is indexed by global column (instance offset + local index).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/aoresp.h"

namespace aoresp {

constexpr uint32_t kFlagDegenerate = 1u;  // d = 0 or non-finite: no axis vote
constexpr uint32_t kFlagRisky = 2u;       // max |d_k| outside [2^-100, 2^120]: exhaustive cell test
constexpr uint32_t kFlagLine = 4u;        // c == 0: the projected curve is a line
constexpr uint32_t kFlagLineDown = 8u;    // line whose cross coordinate decreases along the scan

constexpr int kMaxPeaks = 8;
// NaN entries after the cosine and the sine table of every angle table
// (B = J for the sampling rule's directions): a sample index in [J, J + 64)
// reads NaN, so its s_z <= 0 test fails
constexpr int kDirPad = 64;
// A coarse LDS band tile holds 16-bit counters, two per u32 word: the cells
// (j, k) and (j + 1, k) of an even/odd pair of cell lines share a word.  A
// counter takes at most one vote per correspondence of its work item, so items
// are capped at kMaxItemArcs (< 2^16) correspondences and never overflow it.
constexpr int kTileCells = 65536;         // 16-bit cells of one band tile (128 KiB)
// Words between two rows of a tile (and before the first, after the last)
// that take the cells a certified walk counts just outside the frame.
constexpr int kTilePad = 7;
// kTilePad + bw/2 rows of G + kTilePad words (bw G <= kTileCells, bw <= 256),
// rounded up to 16 bytes
constexpr int kTileWords = (kTileCells / 2 + 129 * kTilePad + 3) & ~3;
constexpr int kMaxItemArcs = 63 * 1024;
constexpr int kVoteThreads = 1024;
constexpr int kCountSlots = 64;   // partial inlier counters per result
constexpr int kRingBody = 128;     // per-wave ring of certified parts: < 64 left over + <= 64 appended
constexpr int kRingLine = 256;     // per-wave ring of searched parts: < 64 left over + <= 128 appended

// Per-correspondence records (SoA, one entry per global column).
//  abc : displacement (a, b, c) negated if needed so that c >= 0; .w = the
//        certification threshold of the walk.
//  colp: vertex-column ranges [s, e] of the four column-mode octants, each
//        packed as int16 s | int16 e << 16 (empty when s >= e); a risky
//        correspondence carries kRiskyMark in colp.x.
//  rowp: the same for the four row-mode octants.
//  geo : (ja | jb << 16, jm | km << 16, ka | kb << 16, flags), see walker.h.
struct ArcRecs {
    float4* abc;
    int4* colp;
    int4* rowp;
    int4* geo;
};
constexpr int32_t kRiskyMark = 0x7FFF7FFF;

// One instance of a batch.
struct Inst {
    int64_t off;          // first global column
    int32_t n;            // correspondences
    int32_t G, M, w, B, rad, npk, res_off;
    float tau;
    int32_t bw;           // coarse band width (cell lines per LDS tile), a power of two >= 2
    int64_t grid_off;     // u32 offset of its G*G coarse grid in the grid arena
    int64_t fine_off;     // u32 offset of its npk fine grids (M*M each)
    int64_t hist_off;     // u32 offset of its npk histograms (B each)
    int32_t item0, nitems;   // its correspondence items (first index, count)
    const int16_t* disk;  // in-disk cross range per cell line (G pairs)
    const float* tc;      // angle tables for B: boundary cos / sin, centre angle / cos / sin
    const float* ts;
    const float* th;
    const float* ct;
    const float* st;
    int32_t gate;         // angle gate: only correspondences voting for a cell of the peak's window vote
    int32_t F;            // fine angle factor (1 = none): B*F-bin tables below, 3F window counters per peak
    int64_t fhist_off;    // u32 offset of its npk fine-angle windows (3F each) in the histogram arena
    const float* ftc;     // angle tables for B*F
    const float* fts;
    const float* fth;
    const float* fct;
    const float* fst;
    int32_t rule;         // coarse accumulator rule: 0 per-cell rule, 1 literal sampling rule
    int32_t J;            // samples per great circle (rule 1)
    const float* scs;     // sample directions: cos, sin of -pi + j 2pi/J (rule 1); each
    const float* ssn;     // table is followed by kDirPad NaNs, ssn = scs + J + kDirPad
    int32_t sbw, snb;     // rule 1: rows per band tile, bands
    int32_t sdir_lds;     // rule 1: sample directions staged in LDS
    int32_t shalf;        // rule 1: 16-bit band counters (partial tiles hold two per word)
    int32_t schunk;       // rule 1: circles per band item
    int64_t ssetup_off;   // rule 1: first circle record
    int64_t spart_off;    // rule 1: u32 offset of its partial tiles (chunks x bands x tile words)
    int64_t lmax_off;     // npk > 1: u32 offset of its local-maximum bitmap (G*G bits) in the bitmap arena
};

struct FineWin {
    float U0, V0, hx, hy;
    int nx, ny;
};

// Device-side state of one peak (axis hypothesis); index res_off + slot.
struct PeakState {
    int valid;
    uint32_t peak_cell, axis_votes;
    uint32_t fine_cell, fine_votes;
    float axis[3];
    FineWin win;
};

// Band width (cell lines) of a coarse tile of `tile_cells` cells (at most
// kTileCells) for a G x G grid: a power of two in [2, G], so lines pair up.
__host__ __device__ inline int coarse_band_width(int G, int tile_cells = kTileCells) {
    int bw = tile_cells / G;
    if (bw > G) bw = G;
    if (bw < 2) bw = 2;
    return bw;
}
size_t coarse_lds_bytes();
void init_kernel_attributes();   // once per device, before the first launch

void launch_zero_u32(uint32_t* p, size_t count, hipStream_t s);
// Up to kZeroSpans buffers of u32 words zeroed by one launch.
constexpr int kZeroSpans = 8;
struct ZeroList {
    uint32_t* ptr[kZeroSpans];
    size_t words[kZeroSpans];
    int count;
};
void launch_zero_list(const ZeroList& zl, hipStream_t s);
void launch_arc_setup(const float* P, const float* Q, int64_t N, const Inst* insts, int ninst, ArcRecs recs,
                      hipStream_t s);
// items: int4 (inst, mode | band << 1, i0, i1), processed by `blocks`
// persistent work-groups.  The items form kVoteQueues consecutive queues, one
// per XCD: queue q holds items [first[q], first[q + 1]) and its counter is
// counters[q] (all zero on entry).  Work-group b runs on XCD b mod 8 (the
// hardware deals work-groups to the XCDs in turn) and pulls from queue
// b mod kVoteQueues, then from the others once its own is empty.
constexpr int kVoteQueues = 8;
struct VoteQueues {
    int32_t first[kVoteQueues + 1];
};
void launch_vote(ArcRecs recs, const Inst* insts, const int4* items, VoteQueues q, uint32_t* counters,
                 uint32_t* grid_arena, uint32_t* err, int blocks, hipStream_t s);
// cell items: int4 (inst, c0, c1, -); one block each.  Slots after the first
// read the local-maximum bitmap of instances with npk > 1, written once by
// launch_local_max over the same items.
void launch_local_max(const uint32_t* grid_arena, const Inst* insts, const int4* items, int nitems, uint32_t* lmax,
                      int maxG, hipStream_t s);
void launch_peak(const uint32_t* grid_arena, const Inst* insts, const int4* items, int nitems, const PeakState* st,
                 int slot, const uint32_t* lmax, unsigned long long* keys, hipStream_t s);
void launch_peak_finish(const Inst* insts, int ninst, const unsigned long long* keys, PeakState* st, int slot,
                        hipStream_t s);
// correspondence items: int4 (inst, i0, i1, -); one block each.  A block
// lists the correspondences of its range whose curve may cross the window of
// result slot `slot`, builds their pieces in the window frame, walks them into
// an LDS tile and adds the tile to that slot's fine grid.
void launch_fine_vote(ArcRecs recs, const Inst* insts, const int4* items, int nitems, const PeakState* st, int slot,
                      uint32_t* fine_arena, uint32_t* err, int maxM, hipStream_t s);
void launch_fine_peak(const uint32_t* fine_arena, const Inst* insts, int ninst, PeakState* st, int slot,
                      hipStream_t s);
// Literal sampling rule of Algorithm 1 (instances with rule 1): every one of
// J samples of each great circle that lies on the closed southern hemisphere
// adds one vote to the coarse cell of its projection.  Three launches: a
// per-circle record (frame, window of southern sample indices, 64 checkpoint
// rows) over setup items (instance, first, last circle); the band pass over
// band items (instance, band, first, last circle), each accumulating one band
// of kSampleTile cells in LDS and storing it to its slot of the partial arena
// (chunk-major, kSampleTile-cell tiles); and the reduction over cell items
// (instance, first, last cell) that writes the instance's grid.
constexpr int kSampleTile = 32768;    // u32 counters per band tile (128 KiB of LDS), or the whole grid if smaller
constexpr int kSampleRec = 40;        // u32 words per circle record
constexpr int kSampleSetupChunk = 1024;
constexpr int kSetupLdsDirs = 8192;   // sample counts J whose direction tables the setup stages in LDS
// Layout of the sampling band pass for an instance of n circles: band tile
// rows (a power of two), 16-bit counters (two per word) where the per-item
// count bound allows it, else 32-bit, circles per band item, partial arena
// words, whether the sample directions are staged in LDS beside the tile
// (when both fit in 160 KiB), and the LDS bytes of a block.
struct SampleLayout {
    int bw = 0, half = 0, dirs_lds = 0;
    int64_t chunk = 0, part_words = 0;
    size_t lds_bytes = 0;
};
SampleLayout sample_plan(int G, int J, int64_t n);
void launch_sample_vote(const float* P, const float* Q, int64_t N, const Inst* insts, const int4* setup_items,
                        int nsetup, const int4* band_items, int nband, const int4* cell_items, int ncell,
                        uint32_t* recs, uint32_t* part, uint32_t* grid_arena, size_t lds_bytes, hipStream_t s);
void launch_angle_hist(const float* P, const float* Q, int64_t N, const Inst* insts, const int4* items, int nitems,
                       const PeakState* st, uint32_t* hist_arena, size_t lds_bytes, hipStream_t s);
void launch_angle_peak(const uint32_t* hist_arena, const Inst* insts, int ninst, PeakState* st, int slot,
                       aoresp_result* res, hipStream_t s);
// Coarse-to-fine angle voting: the B*F-bin histogram of every valid peak,
// counted only on the 3F fine bins of coarse bins k-1, k, k+1 around the
// coarse angle peak k (cyclic, in that order), then its argmax (ties to the
// first) replaces the angle and R.  Instances with F = 1 are skipped.
size_t angle_fine_lds_bytes(int npk, int F);
void launch_angle_fine_hist(const float* P, const float* Q, int64_t N, const Inst* insts, const int4* items,
                            int nitems, const PeakState* st, const aoresp_result* res, uint32_t* hist_arena,
                            size_t lds_bytes, hipStream_t s);
void launch_angle_fine_peak(const uint32_t* hist_arena, const Inst* insts, int ninst, const PeakState* st, int slot,
                            aoresp_result* res, hipStream_t s);
// Least-squares rotation on the inlier set of result slot `slot`: per
// correspondence item, the float64 sums of p q^T over the inliers and their
// count (kLsWords doubles per item, in partial); then per instance the sums of
// its items in a fixed order and the rotation (res[..].R_ls).
constexpr int kLsWords = 10;
void launch_ls_accum(const float* P, const float* Q, int64_t N, const Inst* insts, const int4* items, int nitems,
                     const PeakState* st, const aoresp_result* res, int slot, double* partial, hipStream_t s);
void launch_ls_finish(const Inst* insts, int ninst, const double* partial, const PeakState* st, aoresp_result* res,
                      int slot, hipStream_t s);
// partial: nres * kCountSlots counters, zero on entry.
void launch_inliers(const float* P, const float* Q, int64_t N, const Inst* insts, int ninst, const PeakState* st,
                    aoresp_result* res, int nres, uint8_t* masks, uint32_t* partial, hipStream_t s);

}  // namespace aoresp
