/*
 * aoresp.h -- C ABI of libaoresp: outlier-robust rotation estimation by
 * stereographic projection and spatial voting, on AMD Instinct MI355X (gfx950).
 *
 * Paper: T. Xu, Y. Liu, X. Wang, Z.-X. Yang, "Accelerating Outlier-robust
 * Rotation Estimation by Stereographic Projection" (arXiv 2502.06337).
 *
 * Problem (Sec. I, Eq. (1)): given point sets P = {p_i} and Q = {q_i} with
 * correspondence by index, find a rotation R (or several) and the inlier set
 * C = {i : q_i = R p_i + noise}.  Method (Algorithm 1, Sec. III-IV):
 *   1. every pair restricts the axis to the great circle r . (p_i - q_i) = 0
 *      (Eq. (4)); stereographic projection (Eq. (7)) maps it to a circle or
 *      line in the unit disk (Sec. IV, projected-circle equation);
 *   2. the circles vote into a G x G accumulator over [-1, 1]^2: a cell gets
 *      one vote per circle through it (Fig. 3(c));
 *   3. the peak cell (optionally refined on an M x M grid over the 3 x 3
 *      cells around it), back-projected by Eq. (8), is the axis;
 *   4. every pair votes its signed rotation angle about that axis into a
 *      B-bin histogram over [-pi, pi) (Sec. IV-B, Eq. (10));
 *   5. R = Rodrigues(axis, angle) (Eq. (2)); inliers: ||R p_i - q_i|| <= tau.
 * Several rotations (Sec. IV-D): the top-k peaks of the same accumulator with
 * non-maximum suppression, each with its own histogram and R.
 *
 * Conventions for every entry point:
 *   - P and Q are structure-of-arrays float32 of shape (3, n): x[0..n),
 *     y[0..n), z[0..n).  Host variants take host pointers; *_dev variants take
 *     device pointers on the current HIP device and a hipStream_t (as void*,
 *     NULL = default stream) and return after the work is enqueued and the
 *     small result struct has been copied back (they synchronise the stream).
 *   - The library never keeps or frees caller memory.  It caches a workspace
 *     per device (grown on demand) and serialises calls that share it.
 *   - Results depend only on (P, Q, n, params): binary32 arithmetic with no
 *     contraction, integer votes, ties broken towards the lowest index.
 *   - Outputs are written only when the status is AORESP_OK or AORESP_ENODATA.
 *   - A correspondence with p_i - q_i = 0 or a non-finite coordinate casts no
 *     axis vote; one whose angle inputs are (0, 0) or non-finite casts no
 *     angle vote; its mask entry is 0 unless its residual passes the test.
 */
#ifndef AORESP_H
#define AORESP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AORESP_OK = 0,
    AORESP_EINVAL = -1,    /* null pointer, parameter out of range */
    AORESP_ENOMEM = -2,    /* device memory or budget exhausted */
    AORESP_EDEVICE = -3,   /* HIP error, or an internal consistency check failed */
    AORESP_ENODATA = -4,   /* n < 2 or no vote: R = I, counts 0 */
    AORESP_EBUSY = -5,     /* request not finished yet (poll) */
    AORESP_ETIMEDOUT = -6  /* request exceeded its deadline */
} aoresp_status;

/* Solve parameters.  Zero-initialised fields take the documented defaults. */
typedef struct {
    uint32_t grid;           /* G: power of two in [64, 4096]; 0 = aoresp_grid_for_n(n) */
    uint32_t refine_grid;    /* M: 0 = no refinement, else power of two in [8, 128], G*M <= 262144 */
    uint32_t refine_halfwin; /* w: refinement window (2w+1)^2 coarse cells, clipped; 0 -> 1 */
    uint32_t angle_bins;     /* B: bins over [-pi, pi); 0 -> 360; at most 8192 */
    uint32_t nms_radius;     /* top-k suppression radius in coarse cells; 0 -> 5 */
    float inlier_thresh;     /* tau on ||R p - q||; <= 0 -> 0.05 */
    uint32_t angle_gate;     /* 1: only correspondences that vote for a coarse cell of the (2w+1)^2 window
                                around the peak (w = refine_halfwin, clipped; the per-cell rule of
                                Sec. IV-A) cast angle votes; 0: every correspondence (Sec. IV-B) */
    uint32_t angle_refine;   /* F: 0 or 1 = angle from the B-bin histogram; else in [2, 256] with
                                B*F <= 65536: a second histogram over B*F bins, read on the 3F fine bins
                                of coarse bins k-1, k, k+1 around the coarse peak k, gives the angle */
    uint32_t vote_rule;      /* coarse accumulator: 0 = per-cell rule (a cell counts the circles crossing it,
                                Fig. 3(c)); 1 = literal sampling rule of Algorithm 1 (J samples per great
                                circle, each southern sample adds one vote to the cell of its projection) */
    uint32_t circle_samples; /* J for vote_rule 1: 0 -> 8*G (plane step at most h/2); else in [4, 65536] */
} aoresp_params;

/* Result of one rotation. */
typedef struct {
    float R[9];              /* row-major, maps p to q */
    float axis[3];           /* unit axis on the southern hemisphere (Eq. (8)) */
    float angle;             /* signed angle in [-pi, pi): histogram bin centre */
    uint32_t grid;           /* G used */
    uint32_t peak_cell;      /* iy*G + ix of the coarse peak */
    uint32_t fine_cell;      /* jy*M + jx of the refined peak (0 without refinement) */
    uint32_t angle_bin;      /* histogram bin of the angle */
    uint32_t axis_votes;     /* votes of the coarse peak */
    uint32_t fine_votes;     /* votes of the refined peak */
    uint32_t angle_votes;    /* votes of the angle bin */
    uint32_t n_inliers;      /* number of i with ||R p_i - q_i|| <= tau */
    float R_ls[9];           /* least-squares rotation on that inlier set (float64 accumulation and solve,
                                rounded); equals R when there are fewer than three inliers */
    uint32_t angle_fine_bin;   /* bin of the B*F-bin histogram the angle comes from (0 without it) */
    uint32_t angle_fine_votes; /* its votes (0 without it) */
} aoresp_result;

/* Grid resolution chosen for n when params.grid == 0: a pure function of n
 * (so batched, served and one-at-a-time solves agree), looked up by
 * floor(log2 n) in a table the library is built with.  The table comes from
 * an offline sweep (paper_2502_06337_amd/tune_grid.py) of rotation error and
 * solve time at G = 128..1024 on seeded problems shaped like the batched
 * workload: the smallest G whose mean error (capped at 5 degrees) is within a
 * factor 1.25 of the best, non-decreasing in n.  Its scores and version are in
 * paper_2502_06337_amd/grid_table.json. */
uint32_t aoresp_grid_for_n(uint64_t n);

/* Single rotation (Sec. I; Algorithm 1).  P, Q: host (3, n) float32.
 * inlier_mask: n bytes or NULL.  ENODATA if n < 2 or the accumulator is empty. */
aoresp_status est_rotation(const float* P, const float* Q, size_t n, const aoresp_params* prm,
                           aoresp_result* out, uint8_t* inlier_mask);
aoresp_status est_rotation_dev(const float* P, const float* Q, size_t n, const aoresp_params* prm,
                               aoresp_result* out, uint8_t* inlier_mask, void* hip_stream);

/* est_rotation_dev without any allocation, for callers that cannot allocate
 * device memory (code near graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and results as est_rotation_dev, bit for
 * bit.  Every device buffer of the solve (tables, 64 B of records per
 * correspondence, the grid and the refinement, histogram and result arenas)
 * is carved from one static device array of 96 MiB that each GPU the library
 * runs on holds until the process ends; host staging comes from one static
 * host array of 8 MiB.  It calls no hipMalloc, hipFree or hipHostMalloc (the
 * plan itself is built in ordinary host memory).  A solve that does not fit
 * (about n = 1.2e6 at G = 1024; the literal sampling rule's partial tiles
 * at paper scale) returns ENOMEM and runs nothing.  Calls are serialised
 * inside the process and return after the stream has been synchronised, so
 * the array is never shared by two solves at a time; every accumulator in it
 * is cleared by the solve's first kernel, and records are written before
 * they are read.  Work a caller leaves running on another stream against an
 * earlier call's outputs is unaffected: outputs live in caller memory. */
aoresp_status est_rotation_noalloc_dev(const float* P, const float* Q, size_t n, const aoresp_params* prm,
                                       aoresp_result* out, uint8_t* inlier_mask, void* hip_stream);

/* Several rotations (Sec. IV-D): the peaks are the accumulator's local maxima
 * within an integer disk of nms_radius cells (every other cell of the disk
 * holds fewer votes, or as many at a higher index), taken by decreasing votes
 * (ties to the lowest index); a cell within the disk of an earlier peak or
 * within nms_radius*h of the projection of its antipodal axis is skipped.
 * The first peak is the global maximum, as in est_rotation.  out: k entries;
 * masks: k*n bytes (row t = peak t) or NULL; *k_found = peaks found (<= k).
 * k in [1, 8]. */
aoresp_status est_rotations_topk(const float* P, const float* Q, size_t n, uint32_t k,
                                 const aoresp_params* prm, aoresp_result* out, uint8_t* masks,
                                 uint32_t* k_found);
aoresp_status est_rotations_topk_dev(const float* P, const float* Q, size_t n, uint32_t k,
                                     const aoresp_params* prm, aoresp_result* out, uint8_t* masks,
                                     uint32_t* k_found, void* hip_stream);

/* Many independent instances in one launch per stage.  Instance b owns
 * columns [off[b], off[b+1]) of the (3, off[batch]) SoA arrays P and Q.
 * prm: 1 shared entry or `batch` entries (prm_count).  out: batch entries;
 * masks: off[batch] bytes or NULL.  Instance b's result equals est_rotation
 * on its own columns with the same parameters (grid included). */
aoresp_status est_rotation_batch(const float* P, const float* Q, const uint64_t* off, uint32_t batch,
                                 const aoresp_params* prm, uint32_t prm_count, aoresp_result* out,
                                 uint8_t* masks);
aoresp_status est_rotation_batch_dev(const float* P, const float* Q, const uint64_t* off, uint32_t batch,
                                     const aoresp_params* prm, uint32_t prm_count, aoresp_result* out,
                                     uint8_t* masks, void* hip_stream);

/* Steps of the path, exposed for verification.  All device pointers.
 * Coarse accumulator: grid = G*G uint32 (iy*G + ix).                        */
aoresp_status aoresp_coarse_grid_dev(const float* P, const float* Q, size_t n, uint32_t G, uint32_t* grid,
                                     void* hip_stream);
/* Full single solve that also copies the coarse grid (G*G), the fine grid
 * (M*M, if refining) and the angle histogram (B) to the given device buffers
 * (each may be NULL). */
aoresp_status aoresp_solve_debug_dev(const float* P, const float* Q, size_t n, const aoresp_params* prm,
                                     aoresp_result* out, uint8_t* inlier_mask, uint32_t* grid_out,
                                     uint32_t* fine_out, uint32_t* hist_out, void* hip_stream);

/* One single solve with HIP events recorded on hip_stream between its stages;
 * ms_out receives *n_stages durations in milliseconds, in this order: setup
 * (per-correspondence records, zeroing), coarse vote, peak search,
 * refinement (fine vote, fine peak, axis), angle histogram and rotation,
 * inlier mask and least-squares rotation.  For measurement; results are
 * discarded. */
aoresp_status aoresp_stage_times_dev(const float* P, const float* Q, size_t n, const aoresp_params* prm,
                                     float* ms_out, uint32_t* n_stages, void* hip_stream);

/* Autotuner of the coarse vote's work split (LDS tile size and votes per
 * work item) for one (grid, n bucket = floor(log2 n)) key.  Not a step of
 * the paper's method: every choice gives bit-identical results (the votes are
 * integer sums), only speed differs, and G itself is never tuned (it stays
 * aoresp_grid_for_n(n) or the caller's value).  aoresp_autotune_dev times the
 * coarse-vote stage of a solve of (P, Q) (device pointers, as est_rotation_dev)
 * under each candidate, records the fastest in this device's table (used by
 * every later plan with that key) and returns it in *chosen (may be NULL).
 * The table lives until the process ends; save/load write and read it as JSON
 * lines keyed by GPU architecture (entries for another architecture and
 * malformed lines are skipped on load).  EINVAL on a NULL path or n < 2. */
typedef struct {
    uint32_t grid;
    uint32_t n_bucket;
    uint32_t tile_cells;  /* LDS tile of the coarse vote, 16-bit cells, a power of two in [1024, 65536]
                             (band width = tile_cells / grid lines, clamped to [2, grid]) */
    float vote_target;    /* votes per coarse work item (items hold at most 64512 correspondences) */
    float vote_ms;        /* measured coarse-vote time of this choice; -1 if not measured */
} aoresp_tuning;
aoresp_status aoresp_autotune_dev(const float* P, const float* Q, size_t n, const aoresp_params* prm,
                                  aoresp_tuning* chosen, void* hip_stream);
aoresp_status aoresp_tuner_get(uint32_t grid, uint64_t n, aoresp_tuning* out);
aoresp_status aoresp_tuner_save(const char* path);
aoresp_status aoresp_tuner_load(const char* path);
aoresp_status aoresp_tuner_clear(void);

/* Request loop: continuous batching of solves under a device-memory budget.
 * aoresp_submit copies the inputs and returns at once; requests that arrive
 * while others run are admitted in arrival order as memory and slots free up
 * and run in the next batched step (two steps can be in flight).  Results
 * equal est_rotation on the same inputs.  The budget bounds what the loop
 * holds on the device: both pipelines' cached workspaces and batch arrays,
 * not only the requests in flight (the library's small per-device angle and
 * disk tables are outside it).  A request whose deadline passes while it
 * waits, or before its step finishes, completes with ETIMEDOUT; a step the
 * device fails completes its requests with EDEVICE; a step whose buffers
 * cannot be allocated is retried once at the exact size, else ENOMEM.    */
typedef struct aoresp_server aoresp_server;
typedef struct {
    size_t hbm_budget_bytes;  /* device bytes the loop may hold; 0 -> 8 GiB */
    uint32_t max_slots;       /* requests in one batched step; 0 -> 256 */
    uint32_t timeout_us;      /* per-request deadline from submit; 0 = none */
} aoresp_server_cfg;

aoresp_status aoresp_server_create(const aoresp_server_cfg* cfg, aoresp_server** out);
/* P, Q: host (3, n) float32, copied.  ENOMEM if the request alone, in buffers
 * sized exactly for it, exceeds the budget.  *req_id identifies the request
 * for aoresp_poll.  EINVAL once the server is being destroyed. */
aoresp_status aoresp_submit(aoresp_server* s, const float* P, const float* Q, size_t n, const aoresp_params* prm,
                            uint64_t* req_id);
/* timeout_us: 0 = do not wait, < 0 = wait until done.  EBUSY if not done.
 * On completion the request is released; mask (n bytes) may be NULL. */
aoresp_status aoresp_poll(aoresp_server* s, uint64_t req_id, aoresp_result* out, uint8_t* mask,
                          int64_t timeout_us);
/* Latency percentiles (submit to completion) over completed requests. */
aoresp_status aoresp_server_stats(aoresp_server* s, double* p50_us, double* p99_us, double* req_per_s,
                                  uint64_t* completed);
/* Drains queued and running requests, then frees everything. */
void aoresp_server_destroy(aoresp_server* s);

const char* aoresp_strerror(aoresp_status st);
/* Library build identification (string constant). */
const char* aoresp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* AORESP_H */
