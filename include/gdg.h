/*
 * gdg.h -- C ABI of the MI355X (gfx950) sliding-window GDG decoder.
 *
 * GDG (belief propagation with guided decimation and guessing) from Gong,
 * Cammerer and Renes, "Toward Low-latency Iterative Decoding of QLDPC Codes
 * Under Circuit-Level Noise" (arXiv 2403.18901). The library decodes one
 * window of a (W,1) sliding window (Sec. III, Eq. 6) for many shots at once:
 * a window syndrome goes in, the window's correction comes out, and
 * gdg_commit applies the committed part to the detector record (Eq. 7-8).
 *
 * Conventions for every entry point:
 *  - Return 0 on success or a negative GDG_E* code; gdg_last_error() gives a
 *    message (thread-local). No C++ exception crosses this boundary.
 *  - Pointers named d_* are device pointers (HIP global memory) owned by the
 *    caller; all other pointers are host pointers, read during the call only.
 *  - Device work is enqueued asynchronously on `hip_stream` (a hipStream_t;
 *    NULL = the null stream). Results are ready once the stream is synchronised.
 *  - A decode failure is not a call failure: it shows in d_pm (+infinity) and
 *    d_flags, and the shot counts as a logical failure (Sec. III).
 *  - Decode scratch: a shot counter and the path checkpoints where Fig. 2's
 *    tree splits (C2: about 150 MB at full occupancy). gdg_decode_batch takes
 *    it from the caller's workspace when one is given; otherwise, like the
 *    other decode entry points, from a library pool per (device, stream) that
 *    is allocated on the first decode on that stream, grown (after
 *    synchronising the stream) when a larger window needs more, and kept
 *    until gdg_release_scratch or the process ends. Decodes that share
 *    scratch (one stream's pool, one workspace, or the fixed array of
 *    gdg_decode_batch_noalloc) must not overlap in time.
 */
#ifndef GDG_H
#define GDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GDG_OK 0
#define GDG_EINVAL (-22)   /* bad argument */
#define GDG_ENOMEM (-12)   /* device allocation failed */
#define GDG_EDEVICE (-5)   /* a HIP call failed */
#define GDG_ESHAPE (-34)   /* the window exceeds a supported size */

/* Flags per shot in gdg_decode_batch's d_flags. */
#define GDG_FLAG_SATISFIED 1      /* some path met the window syndrome (Eq. 5 finite) */
#define GDG_FLAG_CONTRADICTION 2  /* every path ended in a peeling contradiction */
#define GDG_FLAG_EXHAUSTED 4      /* no path met the syndrome and one ran to D_max */
#define GDG_FLAG_FALLBACK 8       /* the learned proposer's answer failed; plain GDG was used */
#define GDG_FLAG_CAPACITY 16      /* internal: the shot's truncated graph exceeded the window's
                                     slot table (not expected: the table is sized for the worst
                                     case); the output is not a decode */

/*
 * Detector error model (Sec. II-B): the circuit-code parity-check matrix
 * H_circ (n_rows detectors x n_cols fault columns) in CSC form, the logical
 * observable matrix L (n_obs x n_cols, Sec. III) in CSC form, and each
 * column's prior flip probability. Rows are grouped by detector round, w rows
 * per round, n_rounds rounds; row indices within a column are ascending and no
 * column touches more than two consecutive rounds (Sec. II-B). Host memory,
 * read during gdg_build_window only.
 */
typedef struct gdg_dem {
  int32_t n_rows, n_cols, n_obs, w, n_rounds;
  const int32_t* h_ptr;  /* [n_cols+1] */
  const int32_t* h_idx;  /* [h_ptr[n_cols]] detector rows */
  const int32_t* l_ptr;  /* [n_cols+1] */
  const int32_t* l_idx;  /* [l_ptr[n_cols]] observable indices */
  const double* priors;  /* [n_cols], in (0, 1/2] */
} gdg_dem;

/* Decoder parameters (Sec. II-A, Sec. IV, Fig. 2, Alg. 1-3). */
typedef struct gdg_params {
  float alpha;              /* min-sum scaling factor (Sec. II-A): 1.0 circuit level, 0.625 C1 */
  float clip;               /* VN-to-CN messages clipped to [-clip, clip] (Sec. IV-D): 50 */
  int32_t iters_per_step;   /* BP iterations per decimation step (Fig. 2): 6, at least 4 */
  int32_t pre_iters;        /* BP iterations on the whole window before ranking (Sec. IV-C); 0 = off */
  int32_t trunc_factor;     /* keep the first trunc_factor * m ranked columns (Sec. III: 2) */
  int32_t g;                /* guessing depth: paths 0..2^g-1 (Alg. 2); 0 = main path only */
  int32_t dmax_main;        /* D_max of the main path (Fig. 2: 25) */
  int32_t extra_steps;      /* steps after the split of non-main paths (Fig. 2: 10) */
  int32_t side_max_depth;   /* extra side paths split at depths g+1..side_max_depth; 0 = none */
  int32_t low_error;        /* 1 = low-error mode: Alg. 3 off (Sec. IV-A, p <= 0.002) */
} gdg_params;

typedef struct gdg_window gdg_window;

/* Summary of a built window. */
typedef struct gdg_window_info {
  int32_t k, W, m, n;       /* window index, rounds in it, rows, columns (incl. merged unit columns) */
  int32_t row0;             /* first DEM row of the window */
  int32_t n_act;            /* columns GDG runs on after truncation */
  int32_t n_paths;          /* decision paths per shot */
  int32_t n_edges;          /* edges of the window graph */
  int32_t max_sub_edges;    /* bound on edges of a truncated sub-graph */
  int32_t n_commit;         /* committed columns */
  int32_t last;             /* 1 for the final window (commits everything) */
  int32_t lds_bytes;        /* least LDS per workgroup of the decode kernel (a launch
                               allocates up to its CU share at full occupancy) */
  int32_t waves;            /* wavefronts per workgroup of the decode kernel */
  int32_t n_msg;            /* message slots of the preprocessing BP: the per-shot
                               length of gdg_decode_batch_warm's buffers */
} gdg_window_info;

/*
 * Build window k of a (W,F) sliding window over `dem` (Sec. III, Eq. 6; App. E
 * for F > 1): the detector rows of rounds kF..kF+W-1 and the fault columns
 * starting in them. The last window is the first with kF + W >= n_rounds; it
 * covers the remaining rounds (fewer than W when the schedule does not end
 * evenly) and commits every column.
 * Columns that reach past the window's last round (the bottom-right H_1
 * block) are replaced by one unit column per last-round row they touch, with
 * prior p_j = (1 - prod (1 - 2 p_c))/2 over the merged columns, product in DEM
 * column order (Sec. III, the H_1 merge into unit columns). Window column
 * order: kept DEM columns in DEM order, then unit columns by row. Committed
 * columns: those starting in rounds kF..kF+F-1 (no later window contains
 * them), or all of them in the last window. GDG_EINVAL unless 1 <= F <= W and
 * kF < n_rounds; GDG_ESHAPE for windows of more than 512 rows.
 * Uploads the window graph to the current device; *out is owned by the caller
 * and released with gdg_window_free. The window is immutable afterwards and
 * may be used from several streams at once.
 */
int gdg_build_window(const gdg_dem* dem, int32_t k, int32_t W, int32_t F,
                     const gdg_params* prm, gdg_window** out);
void gdg_window_free(gdg_window* win);
int gdg_window_get_info(const gdg_window* win, gdg_window_info* info);

/* Host copies of the window's column table: src[n] = DEM column or -1-row for
 * a unit column (row local to the window), llr[n] = log((1-p)/p) in double,
 * commit[n] = 1 if committed. Any pointer may be NULL. */
int gdg_window_columns(const gdg_window* win, int32_t* src, double* llr, uint8_t* commit);

/* Bytes of device workspace with which gdg_decode_batch decodes n_shots shots
 * with every workgroup keeping its path checkpoints: 256 (the shot counter)
 * plus workgroups x (2^g - 1) checkpoint slots. 0 on a bad window. */
size_t gdg_workspace_bytes(const gdg_window* win, int32_t n_shots);

/*
 * Optional per-shot diagnostics of gdg_decode_batch (all device pointers,
 * each may be NULL):
 *  sel        [n_shots][n_act] int32: kept window columns in ranked order
 *  dec        [n_shots][n_paths][log_cap][3] int32: per decimation step the
 *             selected VN (ranked index), its value, and the number of Alg. 3
 *             decimations at that step; -1 past the last step
 *  ends       [n_shots][n_paths][2] int32: end reason (1 satisfied, 2 D_max,
 *             3 contradiction, 4 no eligible VN) and steps taken
 *  first_post [n_shots][n_act] float: main-path posteriors after its first
 *             step (NaN for decimated VNs)
 *  edge_iters [n_shots] int64: active edges summed over the BP iterations run
 *             (paths of Fig. 2's tree share their iterations until they split)
 * When dec, ends or step_lsum is requested every path runs to its end; without
 * them a path stops once the priors of its VNs fixed to 1 exceed a converged
 * path's Eq. 5 metric (it cannot be the answer). The answer, its metric and
 * the flags are the same either way; edge_iters can be lower without them.
 *  step_lsum  [n_shots][n_paths][log_cap][n_act] float: each VN's sum of its
 *             last four posteriors at the end of every step's BP run (the
 *             Alg. 1 key), NaN for decimated VNs and unused steps
 *  pre_post   [n_shots][pre_iters][n] float: the posteriors (Eq. 2) of every
 *             preprocessing BP iteration on the whole window, in window
 *             column order; NaN for iterations not run (the preprocessing
 *             stops once its hard decision meets the syndrome)
 */
typedef struct gdg_trace {
  int32_t* sel;
  int32_t* dec;
  int32_t log_cap;
  int32_t* ends;
  float* first_post;
  int64_t* edge_iters;
  float* step_lsum;
  float* pre_post;
} gdg_trace;

/*
 * Decode n_shots window syndromes (Alg. 2 inside the window, Sec. III-IV):
 * optional preprocessing BP on the whole window, ranking by the sum of the
 * last four posteriors and truncation to trunc_factor*m columns (Sec. III,
 * IV-C), peeling (Sec. IV-D), then every decision path of Fig. 2 (main, tree
 * and side paths; min-sum BP in steps of iters_per_step flooding iterations,
 * Alg. 1 selection with Alg. 3 unless low_error, Alg. 2 values), path metric
 * Eq. 5 in double precision and the smallest path metric (ties: lowest path
 * id); if no path meets the syndrome, the main path's final decision.
 *   d_syndrome: uint8 0/1, shot s's row r at d_syndrome[s*syn_stride + r],
 *               r < m (e.g. the DEM detector record offset by row0).
 *   d_ehat:     [n_shots][n] uint8 output, the window correction.
 *   d_pm:       [n_shots] double output, +inf when no path met the syndrome.
 *   d_flags:    [n_shots] int32 output, GDG_FLAG_* bits.
 *   d_workspace: NULL (the library's per-stream pool) or caller-owned device
 *               memory, 256-byte aligned, of workspace_bytes >= 256 bytes: the
 *               shot counter, then path checkpoints for as many workgroups as
 *               fit (gdg_workspace_bytes(win, n_shots) fits all of them; the
 *               other workgroups replay their paths from the root, which
 *               gives the same results more slowly). With a workspace the call
 *               allocates nothing and never synchronises. GDG_EINVAL if it is
 *               misaligned or under 256 bytes.
 *   trace:      NULL or diagnostics as above (host struct of device pointers).
 */
int gdg_decode_batch(const gdg_window* win, int32_t n_shots, const uint8_t* d_syndrome,
                     int64_t syn_stride, uint8_t* d_ehat, double* d_pm, int32_t* d_flags,
                     void* d_workspace, size_t workspace_bytes, const gdg_trace* trace,
                     void* hip_stream);

/*
 * gdg_decode_batch for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same decode, with its scratch in a fixed 64 MiB device array of the
 * library that every GPU it runs on holds until the process ends. The array
 * takes the shot counter (cleared by a fill kernel at every call) and the
 * path checkpoints of as many workgroups as fit (C2: 341 of 768; the others
 * replay their paths from the root, which gives identical results). Calls on
 * one GPU share the array and must not overlap in time (they race). Outputs
 * and errors as gdg_decode_batch, plus GDG_ESHAPE when one workgroup's
 * checkpoints exceed the array. No traces.
 */
int gdg_decode_batch_noalloc(const gdg_window* win, int32_t n_shots, const uint8_t* d_syndrome,
                             int64_t syn_stride, uint8_t* d_ehat, double* d_pm, int32_t* d_flags,
                             void* hip_stream);

/*
 * Releases the library's decode scratch pool of (current device, hip_stream),
 * after synchronising that stream. The next decode on the stream without a
 * workspace allocates it again.
 */
int gdg_release_scratch(void* hip_stream);

/*
 * Chained window decoding for streaming (Sec. III: window k + 1 needs the
 * commit of window k): one launch takes n_items experiments, each a shot's
 * detector record, and decodes and commits windows k_begin[i] .. k_end[i]-1 of
 * item i in order inside the same workgroup, so an experiment whose rounds
 * have all arrived needs one launch, not one per window. Each window is
 * decoded as gdg_decode_batch decodes it, straight from the record, and
 * committed as gdg_commit_indexed commits it.
 *   first, middle, last: the window objects of k = 0, of k = 1 (standing for
 *               every middle window of a time-uniform DEM; NULL if n_windows
 *               <= 2) and of k = n_windows - 1 (may equal first when
 *               n_windows = 1); built from one DEM with the same parameters.
 *   d_k_begin, d_k_end: [n_items] int32 window ranges (clamped to 0..n_windows).
 *   d_det:      detector records; item i's DEM row r at d_det[d_det_off[i] + r]
 *               (int64 offsets); updated in place by every commit.
 *   d_obs:      observable accumulators at d_obs[d_obs_off[i] + o]; XORed by
 *               every commit.
 *   d_ehat:     [n_items][ehat_stride] scratch for one window's correction,
 *               ehat_stride >= the largest window's n.
 *   d_pm, d_flags: [n_items][n_windows] outputs for each window decoded.
 * Items must not share records. Errors: GDG_EINVAL for missing windows or
 * buffers, windows out of order or of different launch shapes, unequal
 * window steps, or a small ehat_stride.
 */
int gdg_decode_chain(const gdg_window* first, const gdg_window* middle, const gdg_window* last,
                     int32_t n_windows, int32_t n_items, const int32_t* d_k_begin,
                     const int32_t* d_k_end, uint8_t* d_det, const int64_t* d_det_off,
                     uint8_t* d_obs, const int64_t* d_obs_off, uint8_t* d_ehat,
                     int64_t ehat_stride, double* d_pm, int32_t* d_flags, void* hip_stream);

/*
 * Cross-window message reuse (Sec. V, where the paper leaves it as future
 * work; readings below). gdg_link_windows prepares `next` to start its
 * preprocessing BP from messages `prev` hands over: for every edge of next's
 * window graph it finds the edge of prev between the same detector row and
 * the same DEM column (unit columns of merged faults have none). Both windows
 * must come from the same DEM; next must have preprocessing (pre_iters > 0).
 * Call it before decoding with next, not while a decode with next runs; a
 * second call replaces the link. GDG_EINVAL for a null window or a window
 * without preprocessing.
 */
int gdg_link_windows(gdg_window* next, const gdg_window* prev);

/*
 * The message slot of every edge of the window graph in the warm-start
 * buffers: slot[e] for edge e of the row-major window CSR (rows in window
 * order, columns ascending; gdg_window_info.n_edges entries), values below
 * gdg_window_info.n_msg. Host array owned by the caller.
 */
int gdg_window_edge_slots(const gdg_window* win, int32_t* slot);

/*
 * gdg_decode_batch with a warm start (Sec. V's message reuse). Reading: the
 * window's preprocessing BP -- the one BP that covers the whole window graph,
 * and the whole decoder for shots it already solves -- starts its CN-to-VN
 * messages on edges the previous window also had from the previous window's
 * handed-over messages, zero elsewhere, followed by one VN update (Eqs. 2-3)
 * that forms the first posteriors and VN-to-CN messages; it then runs as in
 * gdg_decode_batch. The messages a window hands over are one CN update (Eq. 1)
 * of its preprocessing BP's final VN-to-CN messages, whether or not that BP met
 * the syndrome. The decision paths restart from fresh messages on the
 * truncated graph as without warm start.
 *   d_warm_in:  NULL (cold start) or [n_shots][warm_in_stride] float, the
 *               previous window's d_warm_out for the same shots; the window
 *               must be linked (gdg_link_windows) and warm_in_stride at least
 *               the previous window's n_msg.
 *   d_warm_out: NULL or [n_shots][warm_out_stride] float output, this window's
 *               handed-over messages in its slot order (gdg_window_edge_slots),
 *               warm_out_stride >= n_msg. It may not alias d_warm_in.
 * Other arguments and errors as gdg_decode_batch; GDG_EINVAL also for warm
 * buffers on a window without preprocessing, or strides below those bounds.
 */
int gdg_decode_batch_warm(const gdg_window* win, int32_t n_shots, const uint8_t* d_syndrome,
                          int64_t syn_stride, const float* d_warm_in, int64_t warm_in_stride,
                          float* d_warm_out, int64_t warm_out_stride, uint8_t* d_ehat,
                          double* d_pm, int32_t* d_flags, void* d_workspace,
                          size_t workspace_bytes, const gdg_trace* trace, void* hip_stream);

/*
 * Several decode jobs in one persistent launch: windows of different codes
 * (sizes) and their shot batches share one kernel. Workgroup b decodes items
 * b, b + workgroups, ... of the concatenated job list (jobs in the order given;
 * put the costliest first). Same semantics per shot as gdg_decode_batch.
 */
#define GDG_MAX_JOBS 8
typedef struct gdg_job {
  const gdg_window* win;
  int32_t n_shots;
  const uint8_t* d_syndrome;   /* as in gdg_decode_batch */
  int64_t syn_stride;
  uint8_t* d_ehat;             /* [n_shots][n of this window] */
  double* d_pm;                /* [n_shots] */
  int32_t* d_flags;            /* [n_shots] */
} gdg_job;

typedef struct gdg_launch_cfg {
  int32_t waves;        /* wavefronts per workgroup, 1..8 (0 = 4) */
  int32_t workgroups;   /* persistent grid size (0 = one workgroup per shot) */
} gdg_launch_cfg;

int gdg_decode_jobs(const gdg_job* jobs, int32_t n_jobs, const gdg_launch_cfg* cfg,
                    void* hip_stream);

/* Least LDS bytes per workgroup the jobs need at `waves` wavefronts (negative on
 * error); a launch allocates up to the CU's share at the kernel's occupancy (a
 * larger share when it has fewer shots than that many workgroups per CU), and
 * each shot uses as many path wavefronts as fit in it. */
int gdg_jobs_lds_bytes(const gdg_job* jobs, int32_t n_jobs, int32_t waves);

/*
 * Commit (Eq. 7-8): for each shot, XOR the DEM columns of the committed window
 * columns with d_ehat = 1 into the detector record (updating the next window's
 * syndrome, s_2' = s_2 + H_2 e_1) and their observable effect into d_obs
 * (Eq. 9's L e).
 *   d_ehat:       [n_shots][n] uint8 from gdg_decode_batch.
 *   d_detectors:  uint8, shot s's DEM row r at d_detectors[s*det_stride + r], in/out.
 *   d_obs:        uint8, shot s's observable o at d_obs[s*obs_stride + o], in/out.
 */
int gdg_commit(const gdg_window* win, int32_t n_shots, const uint8_t* d_ehat,
               uint8_t* d_detectors, int64_t det_stride, uint8_t* d_obs, int64_t obs_stride,
               void* hip_stream);

/*
 * Streaming form of the sliding window (Sec. III, Eq. 6-8) for blocks that sit
 * at different windows: a time-uniform DEM gives every middle window the same
 * graph, priors and commit set up to a shift of w rows per window, so one
 * window object serves all middle windows of all blocks.
 *
 * gdg_copy_rows copies n rows of m bytes between per-row offsets:
 *   d_dst[d_dst_off[i] + j] = d_src[d_src_off[i] + j], j < m, or
 *   d_dst[i*m + j] when d_dst_off is null (offsets: [n] int64 element offsets
 *   on the device, e.g. block base + k*w to gather window k's syndrome).
 *
 * gdg_commit_indexed is gdg_commit with per-shot offsets: shot i's DEM row r
 * of the window (row0 <= r, r - row0 < (F+1)w) is d_detectors[d_det_off[i] + r - row0]
 * and observable o is d_obs[d_obs_off[i] + o]; d_det_off / d_obs_off are [n]
 * int64 on the device. Offsets are the caller's: they must stay inside the
 * buffers. Both calls are asynchronous on hip_stream; errors as gdg_commit.
 */
int gdg_copy_rows(int32_t n, int32_t m, const uint8_t* d_src, const int64_t* d_src_off,
                  uint8_t* d_dst, const int64_t* d_dst_off, void* hip_stream);
int gdg_commit_indexed(const gdg_window* win, int32_t n_shots, const uint8_t* d_ehat,
                       uint8_t* d_detectors, const int64_t* d_det_off, uint8_t* d_obs,
                       const int64_t* d_obs_off, void* hip_stream);

/*
 * Plain flooding min-sum BP on the whole window, no decimation (Eqs. 1-4):
 * n_iters iterations from fresh messages; d_post [n_shots][n_iters][n] float
 * receives every iteration's posteriors (Eq. 2), d_first_ok [n_shots] int32
 * the first iteration whose hard decision met the syndrome (0 = none). It runs
 * the decode kernel's own whole-window BP (the preprocessing of Sec. III and
 * Sec. IV-C) without its early stop, so the message passing can be checked
 * for any iteration count and on windows decoded without preprocessing.
 * GDG_ESHAPE if the window does not fit one workgroup's LDS.
 */
int gdg_bp(const gdg_window* win, int32_t n_shots, const uint8_t* d_syndrome, int64_t syn_stride,
           int32_t n_iters, float* d_post, int32_t* d_first_ok, void* hip_stream);

/*
 * BP+OSD on the window (the comparator of Sec. II-A's OSD paragraph and Sec.
 * III; App. E decodes last windows with it): flooding min-sum BP on the whole
 * window, at most bp_iters iterations, stopping once its hard decision meets
 * the syndrome (that decision is then the answer). Otherwise the columns are
 * ranked by posterior LLR ascending (ties: column index) and the first n_keep
 * kept (n_keep <= 0: all; Sec. III's shortening keeps 2m); Gauss-Jordan
 * elimination over GF(2) in rank order picks the information set (each pivot
 * at its lowest row not yet a pivot row). OSD-0 solves the syndrome on it; with
 * cs != 0 the combination sweep of order lambda also tries every single
 * non-pivot kept column and every pair among the first lambda of them (OSD-CS,
 * Sec. II-A). The least Eq. 5 cost wins (summed as the swept columns, then the
 * information-set columns by ascending pivot row), ties to the earlier
 * candidate (OSD-0, singles in rank order, pairs lexicographically).
 *   d_ehat [n_shots][n] uint8, d_pm [n_shots] (Eq. 5 in window-column order;
 *   +inf if the syndrome is outside the span of the kept columns: the answer is
 *   then BP's hard decision), d_flags [n_shots] (GDG_FLAG_SATISFIED or 0).
 *   d_order [n_shots][n] int32 or NULL: the ranking used (-1 where BP met the
 *   syndrome). d_bp_iters [n_shots] or NULL: BP iterations run.
 * One workgroup per shot. GDG_ESHAPE for windows of more than 512 rows or 4096
 * columns, or whose bit-columns do not fit in LDS (keep fewer columns).
 */
int gdg_decode_osd(const gdg_window* win, int32_t n_shots, const uint8_t* d_syndrome,
                   int64_t syn_stride, int32_t bp_iters, int32_t cs, int32_t lambda,
                   int32_t n_keep, uint8_t* d_ehat, double* d_pm, int32_t* d_flags,
                   int32_t* d_order, int32_t* d_bp_iters, void* hip_stream);

/*
 * Device copy of a DEM for sampling and evaluation. gdg_dem_upload copies the
 * CSC arrays, a CSR copy of H and uint32 sampling thresholds floor(p 2^32).
 */
typedef struct gdg_dem_dev gdg_dem_dev;
int gdg_dem_upload(const gdg_dem* dem, gdg_dem_dev** out);
void gdg_dem_free(gdg_dem_dev* d);

/*
 * Synthetic shots: column c of shot s fires iff word (c mod 4) of
 * Philox4x32-10(counter = (c div 4, shot0 + s, stream, 0xC0DE),
 * key = (seed low, seed high)) is below floor(p_c 2^32) (Salmon et al.,
 * SC'11). Writes detectors H e [n_shots][n_rows] and observables L e
 * [n_shots][n_obs] (uint8). Inputs for the decoder, not part of it.
 */
int gdg_sample(const gdg_dem_dev* d, int32_t n_shots, uint64_t seed, uint32_t stream,
               uint64_t shot0, uint8_t* d_detectors, uint8_t* d_obs, void* hip_stream);

/*
 * Shot evaluation (Sec. III, Eq. 8 and Eq. 9): d_fail[s] = 1 unless every
 * residual detector of shot s is 0 and its observable accumulator (true
 * observables XOR the committed L e) is 0.
 */
int gdg_evaluate(int32_t n_shots, int32_t n_rows, int32_t n_obs, const uint8_t* d_detectors,
                 const uint8_t* d_obs, uint8_t* d_fail, void* hip_stream);

/*
 * The error vectors behind gdg_sample's shots: d_err[s][c] = 1 iff DEM
 * column c fired in shot shot0 + s (same seed/stream/shot convention).
 * Training labels for the learned proposer; not part of decoding.
 */
int gdg_sample_errors(const gdg_dem_dev* d, int32_t n_shots, uint64_t seed, uint32_t stream,
                      uint64_t shot0, uint8_t* d_err, void* hip_stream);

/*
 * Learned decimation proposer -- an addition to the paper's method (GDG's own
 * selection is Alg. 1). A 17-64-64-1 perceptron with ReLU hidden layers
 * scores a candidate VN from its last 16 BP posteriors and its degree; the
 * output is the logit that the candidate is in error (its error bit is 1).
 *
 * Parameters: GDG_MLP_PARAMS floats, W1 [17][64] (input-major), b1 [64],
 * W2 [64][64], b2 [64], w3 [64], b3. Features x [n][17]: posteriors squashed
 * as p / (8 + |p|), oldest first, then degree / 8.
 *
 * Training (FP32, device buffers, asynchronous on hip_stream):
 *   gdg_mlp_forward  z[n] = network(x);
 *   gdg_mlp_grad     mean binary cross-entropy of logits z against labels
 *                    y [n] (0/1 floats): d_grad [GDG_MLP_PARAMS] gradient,
 *                    d_loss [1] (may be null); reduction order is fixed, so
 *                    results are deterministic. d_work: caller's scratch of
 *                    gdg_mlp_grad_work_bytes(n) bytes.
 *   gdg_mlp_adam     one Adam step (Kingma and Ba, bias-corrected, step >= 1)
 *                    on params with moment buffers d_m, d_v [GDG_MLP_PARAMS].
 * Inference (BF16 matrix cores, FP32 accumulation):
 *   gdg_model_create copies host FP32 parameters into a device model (weights
 *                    rounded to BF16, nearest even); owned by the library.
 *   gdg_mlp_infer    z[n] = network(x) with that model (for testing).
 */
#define GDG_MLP_PARAMS 5377
/*
 * Decoding with the proposer. Mode 1: each path of a small learned tree
 * (2^guesses paths) decimates, at every step, the candidate with the highest
 * logit among the first n_cand VNs in Alg. 1's order (ties: the earlier one),
 * to 1 if that logit is >= 0, else to 0; a step whose best logit has
 * magnitude below tau is a guess point (bit i of the path id: take the other
 * value at the i-th guess point), up to `guesses` of them. The best
 * converged path by Eq. 5 wins; if no learned path meets the syndrome, or the
 * winner's metric exceeds pm_fallback, the window's plain GDG tree decodes
 * the shot instead and its flags gain GDG_FLAG_FALLBACK. Mode 2 (training data): plain
 * GDG, and on the main path's first rec_steps steps the features of the first
 * 16 candidates go to d_rec_x [n_shots][rec_steps][16][17], their window
 * columns to d_rec_col (entries not reached stay as the caller filled them)
 * and their favoured values to d_rec_fav.
 * Outputs as gdg_decode_batch. d_work: gdg_learned_work_bytes(win) bytes of
 * device scratch (posterior history), not shared between concurrent calls.
 */
typedef struct gdg_learn_cfg {
  int32_t mode;        /* 1 learned + plain fallback; 2 record */
  int32_t n_cand;      /* candidates scored per step, 1..16 */
  int32_t guesses;     /* mode 1: guess points per path (2^guesses <= window paths) */
  float tau;           /* mode 1: guess when the best logit is below tau */
  int32_t rec_steps;   /* mode 2 */
  float* d_rec_x;
  int32_t* d_rec_col;
  int32_t* d_rec_fav;
  int64_t* d_edge_iters;   /* optional [n_shots]: BP edge updates spent on each shot */
  float pm_fallback;       /* mode 1: plain GDG also decodes when the best learned
                              path metric (Eq. 5) exceeds this (+inf: only when no
                              learned path meets the syndrome) */
  int32_t tree;            /* mode 1: 1 = guess at depths 1..guesses instead (Fig. 2's
                              tree, paths 1.. split and run g + extra_steps steps),
                              0 = guess at low-confidence steps */
} gdg_learn_cfg;
typedef struct gdg_model gdg_model;
int gdg_mlp_forward(int32_t n, const float* d_params, const float* d_x, float* d_z,
                    void* hip_stream);
size_t gdg_mlp_grad_work_bytes(int32_t n);
int gdg_mlp_grad(int32_t n, const float* d_params, const float* d_x, const float* d_y,
                 float* d_grad, float* d_loss, void* d_work, size_t work_bytes,
                 void* hip_stream);
int gdg_mlp_adam(int32_t step, float lr, float beta1, float beta2, float eps, float* d_params,
                 const float* d_grad, float* d_m, float* d_v, void* hip_stream);
int gdg_model_create(const float* h_params, gdg_model** out);
void gdg_model_free(gdg_model* m);
int gdg_mlp_infer(const gdg_model* m, int32_t n, const float* d_x, float* d_z, void* hip_stream);
size_t gdg_learned_work_bytes(const gdg_window* win);
int gdg_decode_learned(const gdg_window* win, const gdg_model* model, const gdg_learn_cfg* cfg,
                       int32_t n_shots, const uint8_t* d_syndrome, int64_t syn_stride,
                       uint8_t* d_ehat, double* d_pm, int32_t* d_flags, void* d_work,
                       size_t work_bytes, void* hip_stream);

const char* gdg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GDG_H */
