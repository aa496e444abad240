// Internal interface between the host side (gdg_host.cpp) and the kernels
// (gdg_kernels.hip). Plain structs of device pointers and sizes, passed by
// value to the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gdg_mlp.h"

// Slot metadata word of the lane-group CN layout (one per lane and slot column).
constexpr uint32_t kMetaEdge = 0x3fffu;      // first CSR edge of the batch
constexpr int kMetaRowShift = 14;            // row, 10 bits
constexpr int kMetaLogKShift = 24;           // log2 of the group size, 3 bits
constexpr uint32_t kMetaSyn = 1u << 27;      // window syndrome bit of the row
constexpr uint32_t kMetaLead = 1u << 28;     // first lane of the group
constexpr uint32_t kMetaValid = 1u << 29;    // the slot holds a row

// Window graph on the device plus decoder parameters.
struct gdg_win_dev {
  int m, n, n_act, e_full, n_paths;
  int g, dmax_main, extra, side_max_depth, low_error, iters, pre_iters;
  int bound_ok;             // every prior LLR > 0: a path's fixed 1s bound its Eq. 5 metric
  float alpha, clip;
  const int* row_ptr;       // [m+1] window CSR
  const uint16_t* row_col;  // [e_full] column of each CSR edge (ascending per row)
  const uint8_t* row_kcol;  // [e_full] position of that edge in its column's CSC list
  const uint32_t* row_cs;   // [e_full] column | (column-order slot << 16) of each CSR edge
  const int* col_ptr;       // [n+1] window CSC
  const float* llr;         // [n] prior LLR rounded to float
  const double* llr64;      // [n] prior LLR in double (path metric, Eq. 5)
  const uint8_t* deg;       // [n] column degree
  // the whole window graph in the decode kernel's lane-group layout (used by
  // the preprocessing BP): rows by decreasing degree, padded to multiples of 4
  // edges with dummy VN n; column slots padded to multiples of 4
  int fr_T, fr_epad;        // slot columns, padded CSR edges
  const uint32_t* fr_meta;  // [fr_T + 24][64] slot metadata (row field: window row)
  const uint4* fr_rec;      // [fr_T + 24][64] (metadata, the batch's four VN offsets)
  const uint16_t* fr_rvn;   // [fr_epad + 8] 4 * column of each padded CSR edge
  const uint16_t* fr_cidx;  // [padded column slots] 4 * CSR position (padding: 4 * fr_epad)
  const int* fr_cptr;       // [n + 1] first column slot
  // per VN, one 16-byte record for the preprocessing VN pass: the message
  // offsets of its first four column slots (u16 each), the fifth's (the zero
  // message below degree five) | degree << 16, the prior's float bits
  const uint4* fr_vrec;     // [n]
  // warm start from the previous window (Sec. V): for each padded CSR edge,
  // the message slot of the same edge in the previous window, or -1; null
  // until the window is linked
  const int* warm_map;      // [fr_epad]
  int warm_prev_slots;      // fr_epad of the linked previous window
};

// Byte offsets of the decode kernel's dynamic LDS regions. A header lives for
// the whole shot; the area from u_base holds first the preprocessing and the
// ranking, then the truncated sub-graph and the per-wavefront path regions.
// The sub-graph's variable-size arrays and the path regions are placed per
// shot from its actual sizes (gdg_dyn_layout, gdg_path_layout): the plan only
// guarantees room for the worst truncation with one path wavefront, and a shot
// uses as many path wavefronts as fit in the launch's allocation.
struct gdg_lds {
  int total;   // minimum dynamic LDS bytes
  // header (offsets from the start of the dynamic LDS)
  int sorig, sel, misc, obits, eacc;
  int pbits_words, obits_words, meta_cols;
  int u_base;
  // from u_base: preprocessing and ranking
  int p_post, p_c2v, p_lsum, p_keys, sort_n;
  // from u_base: sub-graph arrays of fixed size, then the variable part
  int psyn, rptr, cptr, vdeg, st0, sres0, ppm, pend, pbits, tq, tready;
  int dyn_base;
  // from u_base: sub-graph build scratch, above the largest variable part
  int p_loc, p_iscan, p_llr, p_deg;
};

__host__ __device__ inline int gdg_align16(int x) { return (x + 15) & ~15; }

// Variable-size sub-graph arrays (offsets from u_base) for e_pad padded CSR
// edges, col_slots padded column slots and T slot columns.
struct gdg_dyn_layout {
  int rvn, cidx, crow, meta, end;
};
// The column slots' rows (crow) serve Alg. 3 only, so low-error mode has none.
__host__ __device__ inline gdg_dyn_layout gdg_dyn(int dyn_base, int e_pad, int col_slots, int T,
                                                  bool with_crow) {
  gdg_dyn_layout d;
  d.rvn = dyn_base;                                        // [e_pad + 8] u16
  d.cidx = gdg_align16(d.rvn + 2 * (e_pad + 8));           // [col_slots + 4] u16
  d.crow = gdg_align16(d.cidx + 2 * (col_slots + 4));      // [col_slots] u16, or none
  d.meta = gdg_align16(d.crow + (with_crow ? 2 * col_slots : 0));   // [T + 3][64] u32
  d.end = gdg_align16(d.meta + 4 * 64 * (T + 3));
  return d;
}

// One path wavefront's region (offsets within it) for e_pad padded CSR edges.
struct gdg_path_layout {
  int post, status, c2v, unsat, prop, bits, stride;
};
__host__ __device__ inline gdg_path_layout gdg_paths(int e_pad, int n_act, int m, int obits_words) {
  gdg_path_layout p;
  p.post = 0;                                              // [n_act + 1] f32
  p.status = gdg_align16(4 * (n_act + 1));                 // [n_act + 1] i8
  p.c2v = gdg_align16(p.status + n_act + 1);               // [e_pad + 8] f32, also n_act f64
  const int c2v_bytes = 4 * (e_pad + 8) > 8 * n_act ? 4 * (e_pad + 8) : 8 * n_act;
  p.unsat = gdg_align16(p.c2v + c2v_bytes);                // [m] u8
  p.prop = gdg_align16(p.unsat + m);                       // [ceil(n_act / 4)] u32
  p.bits = gdg_align16(p.prop + 4 * ((n_act + 3) / 4));    // [obits_words] u32
  p.stride = gdg_align16(p.bits + 4 * obits_words);
  return p;
}

struct gdg_trace_dev {
  int* sel;
  int* dec;
  int log_cap;
  int* ends;
  float* first_post;
  long long* edge_iters;
  float* step_lsum;
  float* pre_post;
};

// Commit tables: affected DEM rows with the committed window columns touching
// each (CSR), and per observable the committed window columns in its L row.
struct gdg_commit_dev {
  int n_rows, n_obs, n_win;
  const int* row_global;  // [n_rows] DEM row index
  const int* row_ptr;     // [n_rows+1]
  const int* row_col;     // window columns
  const int* obs_ptr;     // [n_obs+1]
  const int* obs_col;
};

struct gdg_dem_dev_k {
  int n_rows, n_cols, n_obs;
  const int* h_ptr;
  const int* h_idx;
  const int* l_ptr;
  const int* l_idx;
  const uint32_t* thr;
};

// One decode job: shots [item0, item0 + n_shots) of the launch decode window
// `w` (laid out in LDS as `L`) on syndromes syn[s*syn_stride ...].
constexpr int kMaxJobs = 8;
struct gdg_job_dev {
  const gdg_win_dev* w;   // device copies, uploaded with the window
  const gdg_lds* L;
  int item0, n_shots;
  const uint8_t* syn;
  long long syn_stride;
  uint8_t* ehat;
  double* pm;
  int* flags;
};
// Learned proposer settings of a launch (mode 0: plain GDG).
struct gdg_learn_dev {
  int mode;          // 0 plain; 1 learned paths, plain GDG fallback; 2 record candidates
  int n_cand;        // candidates scored per step (<= 16)
  int guesses;       // guess points of the learned path set (1 << guesses paths)
  int tree;          // 1: guesses at depths 1..guesses (Fig. 2); 0: at low-confidence steps
  float tau;         // a step is a guess point when the best logit is below tau
  float pm_fallback; // plain GDG also runs when the best learned path metric exceeds this
  gdg_model_dev model;
  float* ring;       // posterior history: [gridDim.x][waves][16][ring_stride]
  int ring_stride;   // >= n_act
  int rec_steps;     // mode 2: main-path steps recorded per shot
  float* rec_x;      // [n_shots][rec_steps][16][17] candidate features
  int* rec_col;      // [n_shots][rec_steps][16] window column (caller fills -1)
  int* rec_fav;      // [n_shots][rec_steps][16] favoured value
};

// A path checkpoint (global memory): the state of a decision path where the
// tree splits, so that one branch continues and the other restarts from it.
struct gdg_ck_layout {
  int post, status, c2v, sres, bytes;
};
__host__ __device__ inline gdg_ck_layout gdg_ck(int n_act, int e_pad) {
  gdg_ck_layout c;
  c.post = 0;                                           // [n_act + 1] f32
  c.status = gdg_align16(4 * (n_act + 1));              // [n_act + 1] i8
  c.c2v = gdg_align16(c.status + n_act + 1);            // [e_pad + 8] f32
  c.sres = gdg_align16(c.c2v + 4 * (e_pad + 8));        // [64] u32
  c.bytes = c.sres + 4 * 64;
  return c;
}

// A chained launch (streaming): each item is one experiment whose windows
// k_begin..k_end-1 are decoded and committed in order by one workgroup, the
// commit of window k feeding the syndrome of window k+1 in device memory.
struct gdg_chain_dev {
  const gdg_win_dev* w[3];   // window graphs: first, middle, last (device copies)
  const gdg_lds* L[3];       // their LDS plans at the launch's wavefronts
  gdg_commit_dev cm[3];      // their commit tables
  int row0[3];               // first DEM row of each shape's window object
  int K, row_step;           // windows per experiment; rows between windows
  long long ehat_stride;     // per-item correction scratch
  uint8_t* det;              // detector records; item i's at det + det_off[i]
  uint8_t* obs;              // observable accumulators at obs + obs_off[i]
  const long long* det_off;
  const long long* obs_off;
  const int* k_begin;
  const int* k_end;
  uint8_t* ehat;             // [items][ehat_stride]
  double* pm;                // [items][K]: each decoded window's path metric
  int* flags;                // [items][K]: and flags
};

struct gdg_jobs_dev {
  int n_jobs, total;
  int lds;   // the launch's dynamic LDS bytes
  int* work;             // shot counter of a persistent launch (zeroed), or null: grid stride
  char* ckpt;            // path checkpoints: [ckpt_wgs][ckpt_slots] of ckpt_stride bytes, or null
  long long ckpt_stride;
  int ckpt_slots;
  int ckpt_wgs;          // workgroups 0..ckpt_wgs-1 own checkpoint slots; the others
                         // replay their paths from the root (same results)
  gdg_job_dev job[kMaxJobs];
  gdg_learn_dev learn;
  // optional warm start of a one-job launch: the previous window's handed-over
  // CN-to-VN messages per shot (its slot order) and this window's; may be null
  const float* warm_in;
  float* warm_out;
  long long warm_in_stride, warm_out_stride;
  gdg_chain_dev chain;       // the chained launch's experiments (gdg_chain_kernel)
};

// LDS plan of the BP+OSD kernel (byte offsets): fixed arrays, then one region
// reused by the window BP (posteriors, messages), the ranking sort keys and
// the GF(2) bit-columns of the kept columns.
struct gdg_osd_lds {
  int syn, order, rank_of, obits, sv, pcol, llrp, isp, freec, misc;   // fixed
  int A, post, c2v, keys, mat, sort_p, mw, nk, obits_words, total;
};
hipError_t gdg_launch_osd(const gdg_win_dev& w, const gdg_osd_lds& L, int n_shots,
                          const uint8_t* syn, long long syn_stride, int n_iters, int cs,
                          int lambda, uint8_t* ehat, double* pm, int* flags, int* order,
                          int* iters, hipStream_t st);

hipError_t gdg_launch_zero(int* p, int n, hipStream_t st);
// The fixed device scratch of gdg_decode_batch_noalloc on the current device:
// its address (looked up once per device) and size.
hipError_t gdg_static_scratch(void** ptr, size_t* bytes);
hipError_t gdg_launch_chain(const gdg_jobs_dev& J, int bucket, bool low, int waves, int grid,
                            int lds, hipStream_t st);
hipError_t gdg_launch_jobs(const gdg_jobs_dev& J, int bucket, bool low, int waves, int grid,
                           int lds, const gdg_trace_dev& tr, hipStream_t st);
int gdg_kernel_bucket(int m, int n_act);
int gdg_decode_waves_per_simd(int bucket, bool learn);   // occupancy the kernel is built for
hipError_t gdg_decode_set_lds_limit(int bucket, int bytes);
hipError_t gdg_launch_bp(const gdg_win_dev& w, int n_shots, const uint8_t* syn, long long stride,
                         int n_iters, float* post, int* first_ok, hipStream_t st);
hipError_t gdg_launch_commit(const gdg_commit_dev& cm, int n_shots, const uint8_t* ehat,
                             uint8_t* det, long long det_stride, uint8_t* obs,
                             long long obs_stride, const long long* det_off,
                             const long long* obs_off, int row0, hipStream_t st);
hipError_t gdg_launch_copy_rows(int n, int m, const uint8_t* src, const long long* src_off,
                                uint8_t* dst, const long long* dst_off, hipStream_t st);
hipError_t gdg_launch_sample(const gdg_dem_dev_k& d, int n_shots, uint64_t seed, uint32_t stream,
                             uint64_t shot0, uint8_t* det, uint8_t* obs, hipStream_t st);
hipError_t gdg_launch_sample_errors(const gdg_dem_dev_k& d, int n_shots, uint64_t seed,
                                    uint32_t stream, uint64_t shot0, uint8_t* err,
                                    hipStream_t st);
hipError_t gdg_launch_evaluate(int n_shots, int n_rows, int n_obs, const uint8_t* det,
                               const uint8_t* obs, uint8_t* fail, hipStream_t st);
