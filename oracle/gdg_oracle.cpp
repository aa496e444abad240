// FP64 CPU oracle for the sliding-window GDG decoder (Gong, Cammerer, Renes,
// "Toward Low-latency Iterative Decoding of QLDPC Codes Under Circuit-Level
// Noise", arXiv 2403.18901).
//
// TEST INFRASTRUCTURE. This file is the plain, slow reference the GPU path is
// checked against. Only the tests, the smoke check and the benchmark's CPU
// baseline may load it. It shares no code with the GPU library: the window
// builder, belief propagation, decimation, peeling, guessing tree, path metric
// and commit are all written here again, step by step, in the paper's order.
//
// Everything is double precision; loops are the obvious ones. Where the paper
// is silent the reading taken is stated at the point of use.
//
// Pins (see tests/test_oracle_*.py): Eqs. 1-4 on a hand-computed example;
// min-sum posteriors equal exact min-marginal differences and sum-product
// posteriors equal exact marginals on tree graphs (brute force); Alg. 1 / 3 and
// the Alg. 2 branch rule on hand-made tables; peeling closure invariant under
// CN/VN relabelling; brute-force minimum-weight decoding for every fault of
// weight <= 2 on the [[72,12,6]] code; every satisfied window reproduces its
// syndrome and the per-window equations (Eq. 7) compose to Eq. 8.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <numeric>
#include <thread>
#include <vector>

namespace {

const double kInf = std::numeric_limits<double>::infinity();

// ------------------------------------------------------------------ DEM input

struct Dem {
  int n_rows = 0, n_cols = 0, n_obs = 0, w = 0, n_rounds = 0;
  std::vector<int> h_ptr, h_idx, l_ptr, l_idx;
  std::vector<double> prior;
};

// ------------------------------------------------------------------ window
//
// Window k of a (W,F) sliding window (Sec. III, Eq. 6, Fig. 1; App. E for
// F > 1): the detector rows of rounds kF..kF+W-1 and the fault columns that
// start in those rounds. The last window is the first with kF + W >= the
// number of rounds; it covers the remaining rounds (possibly fewer than W) and
// commits every column (reading: the paper does not say how the schedule
// ends when the rounds are not a multiple of F).
// A column that reaches past the window (it starts in the last window round and
// also triggers the next round: the bottom-right H_1 block) is not kept;
// instead every last-round row touched by such columns gets one unit column
// (the H_1 -> identity merge of Sec. III). Its prior (the paper only says the
// priors are recalculated) is the probability that an odd number of the merged
// columns fire: p_j = (1 - prod_c (1 - 2 p_c)) / 2, product in DEM column order.
// Column order: kept DEM columns in DEM order, then unit columns in row order.
// Committed columns: those starting in rounds kF..kF+F-1 (the columns no later
// window contains, Sec. III); in the last window, all.

struct Window {
  int k = 0, W = 0, row0 = 0, m = 0, n = 0;
  bool last = false;
  std::vector<int> src;             // DEM column, or -1 - local row (unit column)
  std::vector<double> prior, llr;   // per column
  std::vector<char> commit;
  std::vector<std::vector<int>> col_rows;   // local rows of each column, ascending
  std::vector<std::vector<int>> row_cols;   // local columns of each row, ascending
};

int col_first_round(const Dem& d, int c) { return d.h_idx[d.h_ptr[c]] / d.w; }
int col_last_round(const Dem& d, int c) { return d.h_idx[d.h_ptr[c + 1] - 1] / d.w; }

bool build_window(const Dem& d, int k, int W, int F, Window& win) {
  if (W < 1 || F < 1 || F > W || k < 0 || k * F >= d.n_rounds) return false;
  const int r0 = k * F;
  const int Wk = std::min(W, d.n_rounds - r0);
  win = Window();
  win.k = k;
  win.W = Wk;
  win.row0 = r0 * d.w;
  win.m = Wk * d.w;
  win.last = (r0 + W >= d.n_rounds);
  const int last_round = r0 + Wk - 1;
  std::vector<int> spill_cols;
  for (int c = 0; c < d.n_cols; ++c) {
    int f = col_first_round(d, c), l = col_last_round(d, c);
    if (l - f > 1) return false;   // no fault spans more than two rounds (Sec. II-B)
    if (f < r0 || f > last_round) continue;
    if (l > last_round) {
      spill_cols.push_back(c);
      continue;
    }
    win.src.push_back(c);
    win.prior.push_back(d.prior[c]);
    win.commit.push_back(win.last || f < r0 + F);
    std::vector<int> rows;
    for (int e = d.h_ptr[c]; e < d.h_ptr[c + 1]; ++e) rows.push_back(d.h_idx[e] - win.row0);
    win.col_rows.push_back(rows);
  }
  // unit columns for rows of the last window round touched by spilling columns
  std::vector<double> keep(win.m, 1.0);
  std::vector<char> touched(win.m, 0);
  for (int c : spill_cols) {
    for (int e = d.h_ptr[c]; e < d.h_ptr[c + 1]; ++e) {
      int r = d.h_idx[e];
      if (r / d.w != last_round) continue;
      int lr = r - win.row0;
      keep[lr] *= (1.0 - 2.0 * d.prior[c]);
      touched[lr] = 1;
    }
  }
  for (int lr = 0; lr < win.m; ++lr) {
    if (!touched[lr]) continue;
    win.src.push_back(-1 - lr);
    win.prior.push_back(0.5 * (1.0 - keep[lr]));
    win.commit.push_back(0);
    win.col_rows.push_back(std::vector<int>{lr});
  }
  win.n = (int)win.src.size();
  win.llr.resize(win.n);
  for (int c = 0; c < win.n; ++c) win.llr[c] = std::log((1.0 - win.prior[c]) / win.prior[c]);
  win.row_cols.assign(win.m, {});
  for (int c = 0; c < win.n; ++c)
    for (int r : win.col_rows[c]) win.row_cols[r].push_back(c);
  return true;
}

// ------------------------------------------------------------------ params

}  // namespace

extern "C" {

typedef struct {
  double alpha;          // min-sum scaling factor (Sec. II-A)
  double clip;           // VN-to-CN messages are clipped to [-clip, clip] (Sec. IV-D)
  int iters_per_step;    // BP iterations per decimation step (Fig. 2: six)
  int pre_iters;         // BP iterations on the full window before ranking (Sec. IV-C); 0 = off
  int trunc_factor;      // keep the first trunc_factor * m ranked columns (Sec. III: 2w')
  int g;                 // guessing depth; 2^g paths (ids 0..2^g-1); 0 = main path only
  int dmax_main;         // D_max of the main path (Fig. 2: 25)
  int extra_steps;       // steps after the split for non-main paths (Fig. 2: 10)
  int side_max_depth;    // extra side paths split at depths g+1..side_max_depth (Fig. 2: 10); 0 = none
  int low_error;         // 1 = low-error mode (no Alg. 3)
  int sum_product;       // 1 = sum-product CN rule instead of min-sum (oracle only, for the tree pin)
} orc_params;

typedef struct {
  int n_paths;
  int converged_path;    // best path id, -1 if none
  int pre_converged;     // preprocessing alone satisfied the syndrome
  long long bp_iters;    // BP iterations summed over preprocessing and all paths
  long long edge_iters;  // active edges summed over those iterations
  int steps_main;        // decimation steps taken by the main path
} orc_stats;

}  // extern "C"

namespace {

// ------------------------------------------------------------------ BP state
//
// One decoding problem: rows 0..m-1, columns 0..n-1 (a window or the truncated
// window), with explicit per-edge messages in both directions.

struct Graph {
  int m = 0, n = 0;
  std::vector<std::vector<int>> col_rows, row_cols;
  std::vector<std::vector<int>> col_edge;    // edge id of (col_rows[c][t], c)
  std::vector<int> edge_row, edge_col;       // edge id -> (row, col); edges in row-major order
  std::vector<int> row_ptr;                  // first edge id of each row
  std::vector<int> deg;                      // static column degree (Appendix C)
  std::vector<double> llr;
};

void finish_graph(Graph& g) {
  g.row_cols.assign(g.m, {});
  for (int c = 0; c < g.n; ++c)
    for (int r : g.col_rows[c]) g.row_cols[r].push_back(c);
  g.edge_row.clear();
  g.edge_col.clear();
  std::vector<std::vector<int>> edge_of_rc(g.m);
  g.row_ptr.assign(g.m + 1, 0);
  for (int r = 0; r < g.m; ++r) {
    g.row_ptr[r + 1] = g.row_ptr[r] + (int)g.row_cols[r].size();
    for (int c : g.row_cols[r]) {
      edge_of_rc[r].push_back((int)g.edge_row.size());
      g.edge_row.push_back(r);
      g.edge_col.push_back(c);
    }
  }
  g.col_edge.assign(g.n, {});
  for (int c = 0; c < g.n; ++c) {
    for (int r : g.col_rows[c]) {
      const auto& rc = g.row_cols[r];
      int pos = (int)(std::find(rc.begin(), rc.end(), c) - rc.begin());
      g.col_edge[c].push_back(edge_of_rc[r][pos]);
    }
  }
  g.deg.resize(g.n);
  for (int c = 0; c < g.n; ++c) g.deg[c] = (int)g.col_rows[c].size();
}

// The status snapshot of Appendix C: ternary VN mask, residual syndrome,
// active CN degree.
struct Status {
  std::vector<int> vn;      // -1 active, 0/1 decimated
  std::vector<int> s;       // residual syndrome
  std::vector<int> cdeg;    // number of active VNs per CN
};

Status initial_status(const Graph& g, const uint8_t* syn) {
  Status st;
  st.vn.assign(g.n, -1);
  st.s.resize(g.m);
  st.cdeg.resize(g.m);
  for (int r = 0; r < g.m; ++r) {
    st.s[r] = syn[r] & 1;
    st.cdeg[r] = (int)g.row_cols[r].size();
  }
  return st;
}

// Decimate VN c to value v (Sec. II-A): if v = 1 the syndromes of its CNs flip;
// its CNs lose one active neighbour.
void decimate(const Graph& g, Status& st, int c, int v) {
  st.vn[c] = v;
  for (int r : g.col_rows[c]) {
    if (v) st.s[r] ^= 1;
    st.cdeg[r] -= 1;
  }
}

bool has_dead_check(const Graph& g, const Status& st) {
  for (int r = 0; r < g.m; ++r)
    if (st.cdeg[r] == 0 && st.s[r]) return true;
  return false;
}

// Peeling (Sec. IV-D, Appendix C): a CN with one active neighbour decides that
// neighbour as its residual syndrome; repeat until no such CN is left. Reading:
// synchronous rounds -- all degree-one CNs of a round propose at once; two
// different proposals for one VN, or a CN left with no active neighbour and
// residual 1, is a contradiction (the path dies, PM = infinity). The state at a
// contradiction is the state before the offending round is applied.
// Returns false on contradiction.
bool peel(const Graph& g, Status& st) {
  if (has_dead_check(g, st)) return false;
  for (;;) {
    std::vector<int> prop(g.n, -1);
    bool any = false;
    for (int r = 0; r < g.m; ++r) {
      if (st.cdeg[r] != 1) continue;
      int only = -1;
      for (int c : g.row_cols[r])
        if (st.vn[c] < 0) only = c;
      int v = st.s[r];
      if (prop[only] >= 0 && prop[only] != v) return false;
      prop[only] = v;
      any = true;
    }
    if (!any) return true;
    for (int c = 0; c < g.n; ++c)
      if (prop[c] >= 0) decimate(g, st, c, prop[c]);
    if (has_dead_check(g, st)) return false;
  }
}

struct Messages {
  std::vector<double> v2c, c2v;   // per edge
  std::vector<double> post;       // per column
};

void init_messages(const Graph& g, const orc_params& P, Messages& ms) {
  size_t ne = g.edge_row.size();
  ms.v2c.assign(ne, 0.0);
  ms.c2v.assign(ne, 0.0);
  ms.post = g.llr;
  for (size_t e = 0; e < ne; ++e) {
    double x = g.llr[g.edge_col[e]];   // t = 0: mu_{i->j} = Lambda_i (Sec. II-A)
    ms.v2c[e] = std::min(P.clip, std::max(-P.clip, x));
  }
}

int sgn(double x) { return x < 0.0 ? -1 : 1; }   // sign(0) = +1 (irrelevant, see below)

// One flooding iteration (Sec. II-A): every active CN updates (Eq. 1, scaled by
// alpha, over its active neighbours only -- stale messages of decimated VNs are
// ignored, Sec. II-A), then every active VN forms its posterior (Eq. 2) and new
// extrinsic messages (Eq. 3), clipped to [-clip, clip] (Sec. IV-D). A CN with a
// single active neighbour has an empty min; it sends +clip (reading: peeling
// keeps BP from ever seeing one). sign(0) = +1: a zero magnitude zeroes every
// other outgoing message anyway.
long long cn_update(const Graph& g, const Status& st, const orc_params& P, Messages& ms,
                    double* cn_min_abs) {
  long long active_edges = 0;
  if (cn_min_abs)
    for (int r = 0; r < g.m; ++r) {
      // smallest incoming |VN-to-CN message| of each active CN (the sign-tie detector)
      double mn = kInf;
      for (size_t a = 0; a < g.row_cols[r].size(); ++a)
        if (st.vn[g.row_cols[r][a]] < 0) mn = std::min(mn, std::fabs(ms.v2c[g.row_ptr[r] + a]));
      cn_min_abs[r] = mn;
    }
  for (int r = 0; r < g.m; ++r) {
    if (st.cdeg[r] == 0) continue;
    const auto& rc = g.row_cols[r];
    const int e0 = g.row_ptr[r];   // edges of row r are contiguous
    for (size_t a = 0; a < rc.size(); ++a) {
      int ca = rc[a];
      if (st.vn[ca] >= 0) continue;
      ++active_edges;
      if (P.sum_product) {
        double prod = 1.0;
        for (size_t b = 0; b < rc.size(); ++b) {
          if (b == a || st.vn[rc[b]] >= 0) continue;
          prod *= std::tanh(ms.v2c[e0 + b] / 2.0);
        }
        double val = 2.0 * std::atanh(prod);
        ms.c2v[e0 + a] = (st.s[r] ? -1.0 : 1.0) * val;
        continue;
      }
      double mn = kInf;
      int sign = 1;
      for (size_t b = 0; b < rc.size(); ++b) {
        if (b == a || st.vn[rc[b]] >= 0) continue;
        double x = ms.v2c[e0 + b];
        mn = std::min(mn, std::fabs(x));
        sign *= sgn(x);
      }
      if (mn == kInf) mn = P.clip;
      ms.c2v[e0 + a] = P.alpha * (st.s[r] ? -1.0 : 1.0) * sign * mn;
    }
  }
  return active_edges;
}

// The VN half of an iteration: posteriors (Eq. 2) and clipped extrinsic
// messages (Eq. 3) of every active VN from the current CN-to-VN messages.
void vn_update(const Graph& g, const Status& st, const orc_params& P, Messages& ms) {
  for (int c = 0; c < g.n; ++c) {
    if (st.vn[c] >= 0) continue;
    double sum = g.llr[c];
    for (int e : g.col_edge[c]) sum += ms.c2v[e];
    ms.post[c] = sum;
    for (int e : g.col_edge[c]) {
      double x = sum - ms.c2v[e];
      ms.v2c[e] = P.sum_product ? x : std::min(P.clip, std::max(-P.clip, x));
    }
  }
}

long long bp_iteration(const Graph& g, const Status& st, const orc_params& P, Messages& ms,
                       double* cn_min_abs = nullptr) {
  const long long active_edges = cn_update(g, st, P, ms, cn_min_abs);
  vn_update(g, st, P, ms);
  return active_edges;
}

// Hard decision (Eq. 4): 1 iff posterior <= 0; decimated VNs keep their value.
int hard(const Status& st, const Messages& ms, int c) {
  if (st.vn[c] >= 0) return st.vn[c];
  return ms.post[c] <= 0.0 ? 1 : 0;
}

// Residual syndrome check: every CN's residual syndrome equals the XOR of its
// active neighbours' hard decisions (equivalently H e = s with the decimated
// values included). unsat[r] receives the per-CN result.
bool syndrome_ok(const Graph& g, const Status& st, const Messages& ms, std::vector<int>* unsat) {
  bool ok = true;
  if (unsat) unsat->assign(g.m, 0);
  for (int r = 0; r < g.m; ++r) {
    int x = st.s[r];
    for (int c : g.row_cols[r])
      if (st.vn[c] < 0) x ^= hard(st, ms, c);
    if (x) {
      ok = false;
      if (unsat) (*unsat)[r] = 1;
    }
  }
  return ok;
}

// ------------------------------------------------------------------ Alg. 1 / Alg. 3

struct History {
  std::vector<double> sum, mn, mx;   // over the last four posteriors
  std::vector<int> count;
  void reset(int n) {
    sum.assign(n, 0.0);
    mn.assign(n, kInf);
    mx.assign(n, -kInf);
    count.assign(n, 0);
  }
  void add(int c, double x) {
    sum[c] += x;
    mn[c] = std::min(mn[c], x);
    mx[c] = std::max(mx[c], x);
    count[c] += 1;
  }
};

// Alg. 3 (aggressive decimation) for one VN's four-value history at depth D.
// Element-wise comparisons: "all four < P_A" is max < P_A, "all > P_C" is min > P_C.
int agg_dec(double hsum, double hmin, double hmax, int D, bool on_main, int n_unsat) {
  double PA = on_main ? -3.0 : 0.0;
  double PB = on_main ? -12.0 : -10.0;
  if (D == 1) PB = -16.0;
  const double PC = 30.0, PD = 3.0;
  if (hmax < PA && hsum < PB) return 1;
  if ((hmin > PC && D <= 4) || (hmin > PD && n_unsat >= 3)) return 0;
  return -1;
}

// Alg. 1 (select-VN): over active VNs of degree >= 3, the smallest sum of the
// last four posteriors among VNs whose four values are all <= 0 (favoured
// value 1), else the smallest sum overall (favoured value = its sign, 1 iff
// sum <= 0, the Eq. 4 convention). Strict '<' in index order: ties go to the
// lowest VN index. When not in low-error mode, Alg. 3 runs first on each
// candidate and the VNs it decides leave the selection (agg receives them).
// Returns the chosen VN or -1 if none is eligible.
int select_vn(const std::vector<int>& vn, const std::vector<int>& deg, const History& h,
              bool low_error, int D, bool on_main, const std::vector<int>& n_unsat,
              std::vector<int>* agg, int* fav) {
  double lmin = kInf, lmin_neg = kInf;
  int gmin = -1, gmin_neg = -1;
  int n = (int)vn.size();
  if (agg) agg->assign(n, -1);
  for (int i = 0; i < n; ++i) {
    if (vn[i] != -1) continue;
    if (deg[i] <= 2) continue;
    if (!low_error) {
      int b = agg_dec(h.sum[i], h.mn[i], h.mx[i], D, on_main, n_unsat[i]);
      if (b != -1) {
        if (agg) (*agg)[i] = b;
        continue;
      }
    }
    if (h.sum[i] < lmin) {
      lmin = h.sum[i];
      gmin = i;
    }
    if (h.mx[i] <= 0.0 && h.sum[i] < lmin_neg) {
      lmin_neg = h.sum[i];
      gmin_neg = i;
    }
  }
  if (gmin_neg != -1) {
    *fav = 1;
    return gmin_neg;
  }
  if (gmin == -1) return -1;
  *fav = lmin <= 0.0 ? 1 : 0;
  return gmin;
}

// ------------------------------------------------------------------ Alg. 2 paths
//
// Path ids (Fig. 2; the tree labels are pinned by the figure under its stated
// all-favoured-is-one demonstration): id in [0, 2^g). At depth D <= g the path
// takes the favoured value if bit D of id (D = 1 the most significant of g
// bits) is 0 and the other value if it is 1 (Alg. 2: b + (-1)^b f); past depth
// g it follows the favoured value. id 0 is the main path (D_max = dmax_main),
// id 1 is the side path splitting at depth g, ids 2.. the tree paths; all
// non-main paths get D_max = (split depth) + extra_steps where the split depth
// of ids < 2^g is g. Extra side paths (ids 2^g + j) split at depth g + 1 + j,
// for g + 1 + j <= side_max_depth, with D_max = split + extra_steps.

struct PathSpec {
  int id, split, dmax;
};

std::vector<PathSpec> path_set(const orc_params& P) {
  std::vector<PathSpec> ps;
  if (P.g <= 0) {
    ps.push_back({0, 0, P.dmax_main});
    return ps;
  }
  int nb = 1 << P.g;
  for (int id = 0; id < nb; ++id)
    ps.push_back({id, id == 0 ? 0 : P.g, id == 0 ? P.dmax_main : P.g + P.extra_steps});
  for (int d = P.g + 1; d <= P.side_max_depth; ++d)
    ps.push_back({nb + (d - P.g - 1), d, d + P.extra_steps});
  return ps;
}

// value decimated at depth D for favoured value f on path ps (Alg. 2)
int path_value(const PathSpec& ps, int g, int D, int f) {
  if (ps.id == 0) return f;
  if (g > 0 && ps.id < (1 << g)) {
    if (D > g) return f;
    int b = (ps.id >> (g - D)) & 1;
    return b ? 1 - f : f;
  }
  return D == ps.split ? 1 - f : f;
}

// Alg. 3 uses the main-path thresholds while the path has taken only favoured
// values (reading: its decisions so far coincide with the main path's).
bool path_on_main(const PathSpec& ps, int g, int D) {
  if (ps.id == 0) return true;
  if (g > 0 && ps.id < (1 << g)) {
    int taken = std::min(D - 1, g);   // decisions made before depth D
    if (taken <= 0) return true;
    return (ps.id >> (g - taken)) == 0;
  }
  return D <= ps.split;
}

// ------------------------------------------------------------------ one path

enum { END_CONVERGED = 1, END_EXHAUSTED = 2, END_CONTRADICTION = 3, END_NO_CANDIDATE = 4 };

struct PathResult {
  int end = 0;
  int steps = 0;
  long long iters = 0, edge_iters = 0;
  std::vector<int> e;                // hard decisions over the graph's columns
  std::vector<int> dec_g, dec_v;     // decision log: selected VN and value per step
  std::vector<int> n_agg;            // Alg. 3 decimations per step
  std::vector<double> first_post;   // posteriors after the first step's iterations
};

// Diagnostics of one path, per decimation step (test hooks only; nothing here
// feeds back into the decoding): the posteriors and the four-value history at
// the end of the step's BP run, the VN status before the step's Alg. 3 pass,
// each VN's count of unsatisfied CN neighbours and its Alg. 3 decision.
struct PathProbe {
  int max_steps = 0, steps = 0;
  double *post = nullptr, *hsum = nullptr, *hmin = nullptr, *hmax = nullptr;
  int *status = nullptr, *n_unsat = nullptr, *agg = nullptr;
};

PathResult run_path(const Graph& g, const Status& st0, const orc_params& P, const PathSpec& ps,
                    const int* forced_g, const int* forced_v, int n_forced,
                    PathProbe* probe = nullptr) {
  PathResult res;
  Status st = st0;
  Messages ms;
  init_messages(g, P, ms);
  History h;
  std::vector<int> unsat;
  for (int D = 1; D <= ps.dmax; ++D) {
    h.reset(g.n);
    bool ok = false;
    for (int t = 1; t <= P.iters_per_step; ++t) {
      res.edge_iters += bp_iteration(g, st, P, ms);
      res.iters += 1;
      if (t > P.iters_per_step - 4)
        for (int c = 0; c < g.n; ++c)
          if (st.vn[c] < 0) h.add(c, ms.post[c]);
      if (syndrome_ok(g, st, ms, nullptr)) {   // checked after every iteration (Eq. 4)
        ok = true;
        break;
      }
    }
    if (D == 1) res.first_post = ms.post;
    res.steps = D;
    if (ok) {
      res.end = END_CONVERGED;
      break;
    }
    if (D == ps.dmax) {   // no selection after the last BP run: it could not be used
      res.end = END_EXHAUSTED;
      break;
    }
    bool on_main = path_on_main(ps, P.g, D);
    std::vector<int> n_unsat(g.n, 0);
    if (!P.low_error) {
      syndrome_ok(g, st, ms, &unsat);
      for (int c = 0; c < g.n; ++c)
        for (int r : g.col_rows[c]) n_unsat[c] += unsat[r];
    }
    std::vector<int> agg;
    int fav = 0;
    int sel = select_vn(st.vn, g.deg, h, P.low_error != 0, D, on_main, n_unsat, &agg, &fav);
    if (probe && D - 1 < probe->max_steps) {
      const size_t o = (size_t)(D - 1) * g.n;
      for (int c = 0; c < g.n; ++c) {
        probe->post[o + c] = ms.post[c];
        probe->hsum[o + c] = h.sum[c];
        probe->hmin[o + c] = h.mn[c];
        probe->hmax[o + c] = h.mx[c];
        probe->status[o + c] = st.vn[c];
        probe->n_unsat[o + c] = n_unsat[c];
        probe->agg[o + c] = agg[c];
      }
      probe->steps = D;
    }
    int n_agg = 0;
    for (int c = 0; c < g.n; ++c)
      if (agg[c] >= 0) {
        decimate(g, st, c, agg[c]);
        ++n_agg;
      }
    res.n_agg.push_back(n_agg);
    if (sel < 0) {
      res.end = END_NO_CANDIDATE;
      break;
    }
    int val = path_value(ps, P.g, D, fav);
    if (forced_g && D - 1 < n_forced) {   // replay of another implementation's decision
      sel = forced_g[D - 1];
      val = forced_v[D - 1];
    }
    res.dec_g.push_back(sel);
    res.dec_v.push_back(val);
    decimate(g, st, sel, val);
    if (!peel(g, st)) {
      res.end = END_CONTRADICTION;
      break;
    }
  }
  res.e.resize(g.n);
  for (int c = 0; c < g.n; ++c) res.e[c] = hard(st, ms, c);
  return res;
}

// ------------------------------------------------------------------ window decode

struct WindowResult {
  std::vector<uint8_t> e;    // window columns
  double pm = kInf;
  int flags = 0;
  orc_stats stats{};
  std::vector<int> selected;              // ranked columns kept (window indices)
  std::vector<double> pre_lsum;           // ranking keys (window columns)
  std::vector<PathResult> paths;
};

// Path metric (Eq. 5): sum of prior LLRs over columns decided 1, ascending
// window column order, if the decision satisfies the window syndrome.
double path_metric(const Window& win, const std::vector<uint8_t>& e, const uint8_t* syn) {
  for (int r = 0; r < win.m; ++r) {
    int x = syn[r] & 1;
    for (int c : win.row_cols[r]) x ^= e[c];
    if (x) return kInf;
  }
  double pm = 0.0;
  for (int c = 0; c < win.n; ++c)
    if (e[c]) pm += win.llr[c];
  return pm;
}

Graph window_graph(const Window& win) {
  Graph g;
  g.m = win.m;
  g.n = win.n;
  g.col_rows = win.col_rows;
  g.llr = win.llr;
  finish_graph(g);
  return g;
}

// Preprocessing + ranking + truncation (Sec. III, Sec. IV-C): pre_iters BP
// iterations on the whole window with fresh messages (stop early if the
// syndrome is met), rank columns by the sum of the last four posteriors
// ascending (ties: lower column index first), keep the first trunc_factor * m.
// GDG then runs on the kept columns, in ranked order, with fresh messages.
//
// Warm start (Sec. V's message reuse; readings in the header of warm_map):
// with warm_in (one value per edge of the window graph, NaN where the edge
// has no counterpart in the previous window) the preprocessing BP starts from
// those CN-to-VN messages instead of zeros, followed by one VN update (so its
// first VN-to-CN messages carry them); with warm_out the messages handed to
// the next window are one CN update of the BP's final VN-to-CN messages.
void decode_window(const Window& win, const orc_params& P, const uint8_t* syn, WindowResult& out,
                   const int* forced_sel, const int* forced_g, const int* forced_v,
                   int n_forced, int forced_path, const std::vector<double>* warm_in = nullptr,
                   std::vector<double>* warm_out = nullptr) {
  out = WindowResult();
  out.e.assign(win.n, 0);
  Graph full = window_graph(win);
  std::vector<int> keep(win.n);
  std::iota(keep.begin(), keep.end(), 0);
  int n_act = win.n;
  if (P.pre_iters > 0) {
    Status st = initial_status(full, syn);
    Messages ms;
    init_messages(full, P, ms);
    if (warm_in) {
      for (size_t e = 0; e < ms.c2v.size(); ++e)
        if (!std::isnan((*warm_in)[e])) ms.c2v[e] = (*warm_in)[e];
      vn_update(full, st, P, ms);
    }
    std::vector<double> lsum(win.n, 0.0);
    bool ok = false;
    int t;
    for (t = 1; t <= P.pre_iters; ++t) {
      out.stats.edge_iters += bp_iteration(full, st, P, ms);
      out.stats.bp_iters += 1;
      if (t > P.pre_iters - 4)
        for (int c = 0; c < win.n; ++c) lsum[c] += ms.post[c];
      if (syndrome_ok(full, st, ms, nullptr)) {
        ok = true;
        break;
      }
    }
    out.pre_lsum = lsum;
    if (warm_out) {
      cn_update(full, st, P, ms, nullptr);
      *warm_out = ms.c2v;
    }
    if (ok) {
      for (int c = 0; c < win.n; ++c) out.e[c] = ms.post[c] <= 0.0 ? 1 : 0;
      out.pm = path_metric(win, out.e, syn);
      out.flags = 1;
      out.stats.pre_converged = 1;
      out.stats.converged_path = -1;
      return;
    }
    std::stable_sort(keep.begin(), keep.end(),
                     [&](int a, int b) { return lsum[a] < lsum[b]; });
    n_act = std::min(win.n, P.trunc_factor * win.m);
    keep.resize(n_act);
    if (forced_sel)
      for (int i = 0; i < n_act; ++i) keep[i] = forced_sel[i];
  }
  out.selected = keep;
  Graph sub;
  sub.m = win.m;
  sub.n = n_act;
  sub.col_rows.resize(n_act);
  sub.llr.resize(n_act);
  for (int v = 0; v < n_act; ++v) {
    sub.col_rows[v] = win.col_rows[keep[v]];
    sub.llr[v] = win.llr[keep[v]];
  }
  finish_graph(sub);
  Status st0 = initial_status(sub, syn);
  auto paths = path_set(P);
  out.stats.n_paths = (int)paths.size();
  out.stats.converged_path = -1;
  bool init_ok = peel(sub, st0);   // peel at init as well (reading: BP never sees degree-1 CNs)
  double best = kInf;
  int best_i = -1;
  int n_contra = 0, n_exh = 0;
  for (size_t i = 0; i < paths.size(); ++i) {
    PathResult pr;
    if (!init_ok) {
      pr.end = END_CONTRADICTION;
      pr.e.resize(sub.n);
      Messages ms;
      init_messages(sub, P, ms);
      for (int c = 0; c < sub.n; ++c) pr.e[c] = hard(st0, ms, c);
    } else {
      bool f = forced_g && paths[i].id == forced_path;
      pr = run_path(sub, st0, P, paths[i], f ? forced_g : nullptr, f ? forced_v : nullptr,
                    f ? n_forced : 0);
    }
    out.stats.bp_iters += pr.iters;
    out.stats.edge_iters += pr.edge_iters;
    if (paths[i].id == 0) out.stats.steps_main = pr.steps;
    if (pr.end == END_CONTRADICTION) ++n_contra;
    if (pr.end == END_EXHAUSTED) ++n_exh;
    if (pr.end == END_CONVERGED) {
      std::vector<uint8_t> e(win.n, 0);
      for (int v = 0; v < sub.n; ++v) e[keep[v]] = (uint8_t)pr.e[v];
      double pm = path_metric(win, e, syn);
      if (pm < best) {   // ties: the lowest path id (paths are in id order)
        best = pm;
        best_i = (int)i;
      }
    }
    out.paths.push_back(std::move(pr));
  }
  int pick = best_i >= 0 ? best_i : 0;   // nothing converged: the main path's final decision
  for (int v = 0; v < sub.n; ++v) out.e[keep[v]] = (uint8_t)out.paths[pick].e[v];
  out.pm = best;
  if (best_i >= 0) {
    out.flags |= 1;
    out.stats.converged_path = paths[best_i].id;
  } else {
    if (n_contra == (int)paths.size()) out.flags |= 2;
    if (n_exh > 0) out.flags |= 4;
  }
}

// Edges shared by consecutive windows, for the warm start (Sec. V's message
// reuse, which the paper leaves as future work). Reading: an edge of `next`
// (row-major, columns ascending within a row) continues the edge of `prev`
// between the same detector row and the same DEM column; unit columns of
// merged faults, and rows or columns `prev` lacks, continue nothing (-1).
std::vector<int> warm_map(const Window& prev, const Window& next) {
  std::vector<int> pcol_of_src;
  int max_src = 0;
  for (int c : prev.src) max_src = std::max(max_src, c + 1);
  for (int c : next.src) max_src = std::max(max_src, c + 1);
  pcol_of_src.assign(max_src, -1);
  for (int c = 0; c < prev.n; ++c)
    if (prev.src[c] >= 0) pcol_of_src[prev.src[c]] = c;
  std::vector<int> prow_ptr(prev.m + 1, 0);
  for (int r = 0; r < prev.m; ++r) prow_ptr[r + 1] = prow_ptr[r] + (int)prev.row_cols[r].size();
  std::vector<int> map;
  for (int r = 0; r < next.m; ++r) {
    const int rp = r + next.row0 - prev.row0;
    for (int c : next.row_cols[r]) {
      int q = -1;
      const int sc = next.src[c];
      if (sc >= 0 && rp >= 0 && rp < prev.m && pcol_of_src[sc] >= 0) {
        const auto& rc = prev.row_cols[rp];
        auto it = std::lower_bound(rc.begin(), rc.end(), pcol_of_src[sc]);
        if (it != rc.end() && *it == pcol_of_src[sc]) q = prow_ptr[rp] + (int)(it - rc.begin());
      }
      map.push_back(q);
    }
  }
  return map;
}

// A window-shaped problem from a dense [m][n] matrix and priors (no DEM).
Window dense_window(int m, int n, const uint8_t* dense, const double* llr) {
  Window win;
  win.m = m;
  win.n = n;
  win.col_rows.assign(n, {});
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < n; ++c)
      if (dense[(size_t)r * n + c]) win.col_rows[c].push_back(r);
  win.row_cols.assign(m, {});
  for (int c = 0; c < n; ++c)
    for (int r : win.col_rows[c]) win.row_cols[r].push_back(c);
  win.llr.assign(llr, llr + n);
  win.prior.resize(n);
  win.src.resize(n);
  win.commit.assign(n, 1);
  return win;
}

// ------------------------------------------------------------------ BP+OSD
//
// BP+OSD-CS (Sec. II-A, the OSD paragraph; Sec. III): flooding min-sum BP on
// the whole window, up to n_iters iterations from fresh messages, stopping at
// the first iteration whose hard decision meets the syndrome (that decision is
// then the answer). Otherwise the columns are ranked by their last posterior
// LLR, ascending -- the most likely to be flipped first -- ties by column index,
// and the first n_keep ranked columns are kept (n_keep <= 0: all of them;
// Sec. III's shortening keeps 2w'). Gauss-Jordan elimination over GF(2)
// visits the kept columns in rank order and makes a column a pivot when it has
// a 1 in a row that is not a pivot row yet (the lowest such row); the pivots
// form the information set S. OSD-0 solves H_S e_S = s with every other column
// at zero. The combination sweep (cs) also tries every single non-pivot kept
// column and every pair among the first lambda non-pivot columns in rank
// order, each with e_S solving the rest of the syndrome. The candidate of
// least cost wins; ties go to the earlier candidate in the order OSD-0, single
// columns in rank order, pairs (a, b) with a ranked before b in lexicographic
// order. Readings (the paper and its OSD sources leave them open): the cost is
// the Eq. 5 sum of prior LLRs, added up as the swept columns first, then the
// information-set columns in ascending order of their pivot rows; the pivot
// row is the lowest eligible row. If the syndrome is not in the span of the
// kept columns the answer is the BP hard decision and no path metric.

struct OsdResult {
  std::vector<uint8_t> e;
  double pm = kInf;
  int flags = 0;
  std::vector<int> order;
  int bp_iters = 0;
};

OsdResult osd_window(const Window& win, const orc_params& P, const uint8_t* syn, int n_iters,
                     bool cs, int lambda, int n_keep, const int* forced_order) {
  OsdResult R;
  R.e.assign(win.n, 0);
  Graph g = window_graph(win);
  Status st = initial_status(g, syn);
  Messages ms;
  init_messages(g, P, ms);
  bool ok = false;
  int t = 0;
  for (t = 1; t <= n_iters; ++t) {
    bp_iteration(g, st, P, ms);
    if (syndrome_ok(g, st, ms, nullptr)) {
      ok = true;
      break;
    }
  }
  R.bp_iters = ok ? t : n_iters;
  std::vector<uint8_t> hard(win.n);
  for (int c = 0; c < win.n; ++c) hard[c] = ms.post[c] <= 0.0 ? 1 : 0;
  if (ok) {
    R.e = hard;
    R.pm = path_metric(win, R.e, syn);
    R.flags = 1;
    return R;
  }
  std::vector<int> order(win.n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return ms.post[a] < ms.post[b]; });
  if (forced_order) order.assign(forced_order, forced_order + win.n);
  R.order = order;
  const int m = win.m;
  const int nk = n_keep > 0 ? std::min(n_keep, win.n) : win.n;
  // kept columns (rank order) as dense 0/1 vectors over the rows, and the syndrome
  std::vector<std::vector<uint8_t>> col(nk, std::vector<uint8_t>(m, 0));
  for (int i = 0; i < nk; ++i)
    for (int r : win.col_rows[order[i]]) col[i][r] = 1;
  std::vector<uint8_t> sv(m);
  for (int r = 0; r < m; ++r) sv[r] = syn[r] & 1;
  std::vector<char> row_used(m, 0), is_piv(nk, 0);
  std::vector<int> pcol, prow;   // pivots in the order they were found
  std::vector<int> pcol_of_row(m, -1);
  for (int i = 0; i < nk; ++i) {
    int r = -1;
    for (int rr = 0; rr < m; ++rr)
      if (!row_used[rr] && col[i][rr]) {
        r = rr;
        break;
      }
    if (r < 0) continue;
    std::vector<int> others;
    for (int rr = 0; rr < m; ++rr)
      if (rr != r && col[i][rr]) others.push_back(rr);
    // row rr += row r for every other row rr with a 1 in column i
    for (int j = 0; j < nk; ++j)
      if (col[j][r])
        for (int rr : others) col[j][rr] ^= 1;
    if (sv[r])
      for (int rr : others) sv[rr] ^= 1;
    row_used[r] = 1;
    is_piv[i] = 1;
    pcol.push_back(i);
    prow.push_back(r);
    pcol_of_row[r] = i;
  }
  for (int r = 0; r < m; ++r)
    if (!row_used[r] && sv[r]) {   // the syndrome is not in the span of the kept columns
      R.e = hard;
      return R;
    }
  std::vector<int> free_cols;
  for (int i = 0; i < nk; ++i)
    if (!is_piv[i]) free_cols.push_back(i);
  // candidate t (kept-column indices): cost and solution
  auto evaluate = [&](const std::vector<int>& tt, std::vector<uint8_t>* e_out) {
    std::vector<uint8_t> u = sv;
    double cost = 0.0;
    for (int j : tt) {
      cost += win.llr[order[j]];
      for (int r = 0; r < m; ++r) u[r] ^= col[j][r];
    }
    for (int r = 0; r < m; ++r)
      if (row_used[r] && u[r]) cost += win.llr[order[pcol_of_row[r]]];
    if (e_out) {
      e_out->assign(win.n, 0);
      for (int j : tt) (*e_out)[order[j]] = 1;
      for (size_t q = 0; q < pcol.size(); ++q)
        if (u[prow[q]]) (*e_out)[order[pcol[q]]] = 1;
    }
    return cost;
  };
  std::vector<int> best_t;
  double best = evaluate(best_t, nullptr);
  if (cs) {
    for (int j : free_cols) {
      std::vector<int> tt{j};
      const double c = evaluate(tt, nullptr);
      if (c < best) {
        best = c;
        best_t = tt;
      }
    }
    const int L = std::min<int>(lambda, (int)free_cols.size());
    for (int a = 0; a < L; ++a)
      for (int b = a + 1; b < L; ++b) {
        std::vector<int> tt{free_cols[a], free_cols[b]};
        const double c = evaluate(tt, nullptr);
        if (c < best) {
          best = c;
          best_t = tt;
        }
      }
  }
  evaluate(best_t, &R.e);
  R.pm = path_metric(win, R.e, syn);
  R.flags = std::isfinite(R.pm) ? 1 : 0;
  return R;
}

// Commit (Eq. 7-8, Sec. III): the committed columns decided 1 are applied to the
// detector record (this updates the next window's syndrome, s_2' = s_2 + H_2 e_1)
// and to the observable accumulator (Eq. 9's L e).
void commit_window(const Dem& d, const Window& win, const uint8_t* e, uint8_t* det, uint8_t* obs) {
  for (int c = 0; c < win.n; ++c) {
    if (!win.commit[c] || !e[c]) continue;
    int col = win.src[c];
    for (int t = d.h_ptr[col]; t < d.h_ptr[col + 1]; ++t) det[d.h_idx[t]] ^= 1;
    for (int t = d.l_ptr[col]; t < d.l_ptr[col + 1]; ++t) obs[d.l_idx[t]] ^= 1;
  }
}

Dem make_dem(int n_rows, int n_cols, int n_obs, int w, int n_rounds, const int* h_ptr,
             const int* h_idx, const int* l_ptr, const int* l_idx, const double* prior) {
  Dem d;
  d.n_rows = n_rows;
  d.n_cols = n_cols;
  d.n_obs = n_obs;
  d.w = w;
  d.n_rounds = n_rounds;
  d.h_ptr.assign(h_ptr, h_ptr + n_cols + 1);
  d.h_idx.assign(h_idx, h_idx + h_ptr[n_cols]);
  d.l_ptr.assign(l_ptr, l_ptr + n_cols + 1);
  d.l_idx.assign(l_idx, l_idx + l_ptr[n_cols]);
  d.prior.assign(prior, prior + n_cols);
  return d;
}

struct OrcWindow {
  Dem dem;
  Window win;
};

}  // namespace

// ====================================================================== C API

extern "C" {

// Build window k of a (W,F) sliding window over a DEM given in CSC form.
void* orc_window_new(int n_rows, int n_cols, int n_obs, int w, int n_rounds, const int* h_ptr,
                     const int* h_idx, const int* l_ptr, const int* l_idx, const double* prior,
                     int k, int W, int F) {
  OrcWindow* ow = new OrcWindow();
  ow->dem = make_dem(n_rows, n_cols, n_obs, w, n_rounds, h_ptr, h_idx, l_ptr, l_idx, prior);
  if (!build_window(ow->dem, k, W, F, ow->win)) {
    delete ow;
    return nullptr;
  }
  return ow;
}

void orc_window_free(void* h) { delete (OrcWindow*)h; }

// dims[0..3] = m, n, edges, row0
void orc_window_dims(void* h, int* dims) {
  const Window& w = ((OrcWindow*)h)->win;
  int ne = 0;
  for (auto& c : w.col_rows) ne += (int)c.size();
  dims[0] = w.m;
  dims[1] = w.n;
  dims[2] = ne;
  dims[3] = w.row0;
}

// dense [m][n] matrix, src [n], prior [n], llr [n], commit [n]
void orc_window_export(void* h, uint8_t* dense, int* src, double* prior, double* llr,
                       uint8_t* commit) {
  const Window& w = ((OrcWindow*)h)->win;
  if (dense) {
    std::memset(dense, 0, (size_t)w.m * w.n);
    for (int c = 0; c < w.n; ++c)
      for (int r : w.col_rows[c]) dense[(size_t)r * w.n + c] = 1;
  }
  for (int c = 0; c < w.n; ++c) {
    if (src) src[c] = w.src[c];
    if (prior) prior[c] = w.prior[c];
    if (llr) llr[c] = w.llr[c];
    if (commit) commit[c] = (uint8_t)w.commit[c];
  }
}

// Plain flooding BP on the whole window with no decimation: n_iters iterations,
// posteriors after each one in post[t][n]; optionally cn_min[t][m], the smallest
// incoming |VN-to-CN message| of each CN at iteration t. Returns the first
// iteration (1-based) whose hard decision met the syndrome, or 0.
int orc_window_bp(void* h, const orc_params* P, const uint8_t* syn, int n_iters, double* post,
                  double* cn_min, const double* warm_in) {
  const Window& w = ((OrcWindow*)h)->win;
  Graph g = window_graph(w);
  Status st = initial_status(g, syn);
  Messages ms;
  init_messages(g, *P, ms);
  if (warm_in) {   // warm start as in decode_window
    for (size_t e = 0; e < ms.c2v.size(); ++e)
      if (!std::isnan(warm_in[e])) ms.c2v[e] = warm_in[e];
    vn_update(g, st, *P, ms);
  }
  int first_ok = 0;
  for (int t = 0; t < n_iters; ++t) {
    bp_iteration(g, st, *P, ms, cn_min ? cn_min + (size_t)t * w.m : nullptr);
    std::memcpy(post + (size_t)t * w.n, ms.post.data(), sizeof(double) * w.n);
    if (!first_ok && syndrome_ok(g, st, ms, nullptr)) first_ok = t + 1;
  }
  return first_ok;
}

// Decode n_shots window syndromes syn[s][m]; outputs e[s][n], pm[s], flags[s],
// stats[s]. Optional logs (pass null to skip): sel[s][sel_cap] ranked kept
// columns (-1 padded); dec[s][n_paths][log_cap][3] = (VN, value, Alg. 3 count)
// per step (-1 padded); ends[s][n_paths][2] = (end reason, steps); first_post
// [s][n_post_cap] posteriors of the main path after its first step (sub-graph
// order, -inf padded).
void orc_window_decode(void* h, const orc_params* P, int n_shots, const uint8_t* syn,
                       uint8_t* e, double* pm, int* flags, orc_stats* stats, int* sel,
                       int sel_cap, int* dec, int n_paths_cap, int log_cap, int* ends,
                       double* first_post, int n_post_cap, int n_threads,
                       const double* warm_in, double* warm_out, double* pre_lsum) {
  const Window& w = ((OrcWindow*)h)->win;
  size_t ne = 0;
  for (int r = 0; r < w.m; ++r) ne += w.row_cols[r].size();
  std::atomic<int> next(0);
  auto work = [&]() {
    for (;;) {
      int s = next.fetch_add(1);
      if (s >= n_shots) break;
      WindowResult wr;
      std::vector<double> wi, wo;
      if (warm_in) wi.assign(warm_in + s * ne, warm_in + (s + 1) * ne);
      decode_window(w, *P, syn + (size_t)s * w.m, wr, nullptr, nullptr, nullptr, 0, -1,
                    warm_in ? &wi : nullptr, warm_out ? &wo : nullptr);
      if (warm_out)
        for (size_t i = 0; i < ne; ++i) warm_out[s * ne + i] = i < wo.size() ? wo[i] : std::nan("");
      if (pre_lsum)   // the preprocessing's ranking keys (NaN without preprocessing)
        for (int c = 0; c < w.n; ++c)
          pre_lsum[(size_t)s * w.n + c] = c < (int)wr.pre_lsum.size() ? wr.pre_lsum[c] : std::nan("");
      std::memcpy(e + (size_t)s * w.n, wr.e.data(), w.n);
      pm[s] = wr.pm;
      flags[s] = wr.flags;
      if (stats) stats[s] = wr.stats;
      if (sel) {
        for (int i = 0; i < sel_cap; ++i)
          sel[(size_t)s * sel_cap + i] = i < (int)wr.selected.size() ? wr.selected[i] : -1;
      }
      for (int p = 0; p < n_paths_cap; ++p) {
        const PathResult* pr = p < (int)wr.paths.size() ? &wr.paths[p] : nullptr;
        if (dec) {
          for (int i = 0; i < log_cap; ++i) {
            int* d = dec + (((size_t)s * n_paths_cap + p) * log_cap + i) * 3;
            bool have = pr && i < (int)pr->dec_g.size();
            d[0] = have ? pr->dec_g[i] : -1;
            d[1] = have ? pr->dec_v[i] : -1;
            d[2] = pr && i < (int)pr->n_agg.size() ? pr->n_agg[i] : -1;
          }
        }
        if (ends) {
          ends[((size_t)s * n_paths_cap + p) * 2 + 0] = pr ? pr->end : 0;
          ends[((size_t)s * n_paths_cap + p) * 2 + 1] = pr ? pr->steps : 0;
        }
      }
      if (first_post) {
        for (int i = 0; i < n_post_cap; ++i) {
          double v = -kInf;
          if (!wr.paths.empty() && i < (int)wr.paths[0].first_post.size())
            v = wr.paths[0].first_post[i];
          first_post[(size_t)s * n_post_cap + i] = v;
        }
      }
    }
  };
  int nt = std::max(1, n_threads);
  std::vector<std::thread> th;
  for (int i = 1; i < nt; ++i) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
}

// BP+OSD(-CS) on n_shots window syndromes syn[s][m] (see osd_window): e[s][n],
// pm[s], flags[s] (1: satisfied), bp_iters[s] (iterations run), order[s][n] the
// column ranking used (-1 when BP met the syndrome; may be null). forced_order
// [s][n] (may be null) replaces the oracle's own ranking (replay of another
// implementation's ranking).
void orc_window_osd(void* h, const orc_params* P, int n_shots, const uint8_t* syn, int n_iters,
                    int cs, int lambda, int n_keep, const int* forced_order, uint8_t* e, double* pm,
                    int* flags, int* order, int* bp_iters, int n_threads) {
  const Window& w = ((OrcWindow*)h)->win;
  std::atomic<int> next(0);
  auto work = [&]() {
    for (;;) {
      const int s = next.fetch_add(1);
      if (s >= n_shots) break;
      OsdResult R = osd_window(w, *P, syn + (size_t)s * w.m, n_iters, cs != 0, lambda, n_keep,
                               forced_order ? forced_order + (size_t)s * w.n : nullptr);
      std::memcpy(e + (size_t)s * w.n, R.e.data(), w.n);
      pm[s] = R.pm;
      flags[s] = R.flags;
      if (bp_iters) bp_iters[s] = R.bp_iters;
      if (order)
        for (int c = 0; c < w.n; ++c)
          order[(size_t)s * w.n + c] = R.order.empty() ? -1 : R.order[c];
    }
  };
  int nt = std::max(1, n_threads);
  std::vector<std::thread> th;
  for (int i = 1; i < nt; ++i) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
}

// The warm-start edge map from window `hp` to window `hn` (warm_map); map
// holds one entry per edge of hn. Returns the number of edges.
int orc_warm_map(void* hp, void* hn, int* map) {
  std::vector<int> mp = warm_map(((OrcWindow*)hp)->win, ((OrcWindow*)hn)->win);
  if (map) std::memcpy(map, mp.data(), mp.size() * sizeof(int));
  return (int)mp.size();
}

// BP+OSD(-CS) on a dense [m][n] problem with priors llr (see osd_window).
double orc_dense_osd(int m, int n, const uint8_t* dense, const double* llr, const uint8_t* syn,
                     const orc_params* P, int n_iters, int cs, int lambda, int n_keep,
                     uint8_t* e, int* flags) {
  Window win = dense_window(m, n, dense, llr);
  OsdResult R = osd_window(win, *P, syn, n_iters, cs != 0, lambda, n_keep, nullptr);
  std::memcpy(e, R.e.data(), n);
  if (flags) *flags = R.flags;
  return R.pm;
}

// Replay one path of one shot with the given kept-column set and decision
// sequence forced (the oracle's own choice is still computed); returns the
// oracle's preprocessing ranking keys and, per step, the oracle's own choice,
// every VN's Alg. 1 key (step_lsum[step][n_act], NaN when decimated), the
// smallest |VN-to-CN message| and |posterior| seen during the step's BP run,
// and the largest of the four history posteriors of both picks.
// Used to measure how far another implementation's decisions are from the
// oracle's at the first point they differ. Outputs: own_g/own_v/own_key/
// forced_key per step (the Alg. 1 sums of the oracle's pick and of the forced
// pick, in the oracle's arithmetic), lsum[n] ranking keys.
int orc_window_replay(void* h, const orc_params* P, const uint8_t* syn, const int* forced_sel,
                      int path_id, const int* forced_g, const int* forced_v, int n_forced,
                      int* own_g, int* own_v, double* own_key, double* forced_key,
                      int* own_class, int* forced_class, double* lsum, uint8_t* e_out,
                      double* pm_out, double* step_lsum, double* step_min_msg, int max_steps,
                      double* own_hmax, double* forced_hmax, double* step_min_post,
                      int* step_nagg, double* step_agg_margin, double* first_post) {
  const Window& w = ((OrcWindow*)h)->win;
  // Re-run the path step by step with forcing, recording both choices.
  Graph full = window_graph(w);
  std::vector<int> keep(w.n);
  std::iota(keep.begin(), keep.end(), 0);
  int n_act = w.n;
  if (P->pre_iters > 0) {
    Status st = initial_status(full, syn);
    Messages ms;
    init_messages(full, *P, ms);
    std::vector<double> ls(w.n, 0.0);
    for (int t = 1; t <= P->pre_iters; ++t) {
      bp_iteration(full, st, *P, ms);
      if (t > P->pre_iters - 4)
        for (int c = 0; c < w.n; ++c) ls[c] += ms.post[c];
      if (syndrome_ok(full, st, ms, nullptr)) break;
    }
    if (lsum) std::memcpy(lsum, ls.data(), sizeof(double) * w.n);
    n_act = std::min(w.n, P->trunc_factor * w.m);
    std::stable_sort(keep.begin(), keep.end(), [&](int a, int b) { return ls[a] < ls[b]; });
    keep.resize(n_act);
    if (forced_sel)
      for (int i = 0; i < n_act; ++i) keep[i] = forced_sel[i];
  }
  Graph sub;
  sub.m = w.m;
  sub.n = n_act;
  sub.col_rows.resize(n_act);
  sub.llr.resize(n_act);
  for (int v = 0; v < n_act; ++v) {
    sub.col_rows[v] = w.col_rows[keep[v]];
    sub.llr[v] = w.llr[keep[v]];
  }
  finish_graph(sub);
  Status st = initial_status(sub, syn);
  if (!peel(sub, st)) return -1;
  auto paths = path_set(*P);
  PathSpec ps = paths[0];
  for (auto& q : paths)
    if (q.id == path_id) ps = q;
  Messages ms;
  init_messages(sub, *P, ms);
  History hh;
  std::vector<int> unsat;
  int steps = 0;
  int end = 0;
  for (int D = 1; D <= ps.dmax; ++D) {
    hh.reset(sub.n);
    bool ok = false;
    double min_msg = kInf;
    std::vector<double> cmin(sub.m);
    double min_post = kInf;
    for (int t = 1; t <= P->iters_per_step; ++t) {
      bp_iteration(sub, st, *P, ms, cmin.data());
      for (int r = 0; r < sub.m; ++r) min_msg = std::min(min_msg, cmin[r]);
      for (int c = 0; c < sub.n; ++c)
        if (st.vn[c] < 0) min_post = std::min(min_post, std::fabs(ms.post[c]));
      if (t > P->iters_per_step - 4)
        for (int c = 0; c < sub.n; ++c)
          if (st.vn[c] < 0) hh.add(c, ms.post[c]);
      if (syndrome_ok(sub, st, ms, nullptr)) {
        ok = true;
        break;
      }
    }
    steps = D;
    if (D == 1 && first_post)
      for (int c = 0; c < sub.n; ++c)
        first_post[c] = st.vn[c] < 0 ? ms.post[c] : std::numeric_limits<double>::quiet_NaN();
    if (D - 1 < max_steps) {
      if (step_min_msg) step_min_msg[D - 1] = min_msg;
      if (step_min_post) step_min_post[D - 1] = min_post;
      if (step_lsum)
        for (int c = 0; c < sub.n; ++c)
          step_lsum[(size_t)(D - 1) * sub.n + c] =
              (!ok && st.vn[c] < 0) ? hh.sum[c] : std::numeric_limits<double>::quiet_NaN();
    }
    if (ok) {
      end = END_CONVERGED;
      break;
    }
    if (D == ps.dmax) {
      end = END_EXHAUSTED;
      break;
    }
    bool on_main = path_on_main(ps, P->g, D);
    std::vector<int> n_unsat(sub.n, 0);
    if (!P->low_error) {
      syndrome_ok(sub, st, ms, &unsat);
      for (int c = 0; c < sub.n; ++c)
        for (int r : sub.col_rows[c]) n_unsat[c] += unsat[r];
    }
    std::vector<int> agg;
    int fav = 0;
    int sel = select_vn(st.vn, sub.deg, hh, P->low_error != 0, D, on_main, n_unsat, &agg, &fav);
    int nagg = 0;
    double margin = kInf;   // distance of the closest Alg. 3 comparison to its threshold
    if (!P->low_error) {
      const double PA = on_main ? -3.0 : 0.0;
      const double PB = D == 1 ? -16.0 : (on_main ? -12.0 : -10.0);
      for (int c = 0; c < sub.n; ++c) {
        if (st.vn[c] != -1 || sub.deg[c] <= 2) continue;
        margin = std::min(margin, std::min(std::fabs(hh.mx[c] - PA), std::fabs(hh.sum[c] - PB)));
        if (D <= 4) margin = std::min(margin, std::fabs(hh.mn[c] - 30.0));
        if (n_unsat[c] >= 3) margin = std::min(margin, std::fabs(hh.mn[c] - 3.0));
      }
    }
    for (int c = 0; c < sub.n; ++c)
      if (agg[c] >= 0) {
        decimate(sub, st, c, agg[c]);
        ++nagg;
      }
    if (D - 1 < max_steps) {
      if (step_nagg) step_nagg[D - 1] = nagg;
      if (step_agg_margin) step_agg_margin[D - 1] = margin;
    }
    if (sel < 0) {
      end = END_NO_CANDIDATE;
      break;
    }
    int val = path_value(ps, P->g, D, fav);
    int i = D - 1;
    own_g[i] = sel;
    own_v[i] = val;
    own_key[i] = hh.sum[sel];
    own_class[i] = hh.mx[sel] <= 0.0;
    if (own_hmax) own_hmax[i] = hh.mx[sel];
    if (i < n_forced) {
      int fg = forced_g[i];
      forced_key[i] = (fg >= 0 && fg < sub.n) ? hh.sum[fg] : kInf;
      forced_class[i] = (fg >= 0 && fg < sub.n) ? (hh.mx[fg] <= 0.0) : -1;
      if (forced_hmax) forced_hmax[i] = (fg >= 0 && fg < sub.n) ? hh.mx[fg] : kInf;
      sel = fg;
      val = forced_v[i];
    }
    decimate(sub, st, sel, val);
    if (!peel(sub, st)) {
      end = END_CONTRADICTION;
      break;
    }
  }
  if (e_out) {
    std::memset(e_out, 0, w.n);
    for (int v = 0; v < sub.n; ++v) e_out[keep[v]] = (uint8_t)hard(st, ms, v);
    if (pm_out) {
      std::vector<uint8_t> ev(e_out, e_out + w.n);
      *pm_out = end == END_CONVERGED ? path_metric(w, ev, syn) : kInf;
    }
  }
  return steps * 8 + end;
}

// Full (W,F) sliding-window decode of n_shots shots: det[s][n_rows] is copied,
// windows k = 0 .. K-1 (K = 1 + ceil((n_rounds - W) / F)) are decoded and
// committed in order. With osd_iters > 0 the last window (every window when
// osd_all is set) is decoded by BP (that many iterations) + OSD-CS(osd_lambda)
// on its first osd_keep ranked columns (<= 0: all) instead of GDG: the window
// BP+OSD comparator of Sec. III, and the last-window variant of App. E. Outputs the
// residual detectors (det_out), the observable accumulator XOR the true
// observables (obs_out, so a logical error shows as a nonzero entry),
// fail[s] = 1 unless all residual detectors are 0 (Eq. 8) and obs_out is 0
// (Eq. 9), per-window flags win_flags[s][n_windows] and the committed
// correction e_out[s][n_cols] over DEM columns (caller zeroes it). With
// max_windows >= 0 only the first max_windows windows are decoded (det_out is
// then the residual record the next window sees).
int orc_decode_shots(int n_rows, int n_cols, int n_obs, int w, int n_rounds, const int* h_ptr,
                     const int* h_idx, const int* l_ptr, const int* l_idx, const double* prior,
                     int W, const orc_params* P, int n_shots, const uint8_t* det,
                     const uint8_t* obs, uint8_t* det_out, uint8_t* obs_out, uint8_t* fail,
                     int* win_flags, uint8_t* e_out, long long* edge_iters, int n_threads,
                     int max_windows, int F, int osd_iters, int osd_lambda, int osd_keep,
                     int osd_all, int warm) {
  Dem d = make_dem(n_rows, n_cols, n_obs, w, n_rounds, h_ptr, h_idx, l_ptr, l_idx, prior);
  if (W < 1 || F < 1 || F > W) return -1;
  const int nwin = n_rounds <= W ? 1 : 1 + (n_rounds - W + F - 1) / F;
  const int run_windows = (max_windows >= 0 && max_windows < nwin) ? max_windows : nwin;
  std::vector<Window> wins(nwin);
  for (int k = 0; k < nwin; ++k)
    if (!build_window(d, k, W, F, wins[k])) return -2;
  const bool use_warm = warm && P->pre_iters > 0;
  std::vector<std::vector<int>> wmaps(nwin);
  if (use_warm)
    for (int k = 1; k < nwin; ++k) wmaps[k] = warm_map(wins[k - 1], wins[k]);
  std::atomic<int> next(0);
  std::atomic<long long> ei(0);
  auto work = [&]() {
    for (;;) {
      int s = next.fetch_add(1);
      if (s >= n_shots) break;
      std::vector<uint8_t> dd(det + (size_t)s * n_rows, det + (size_t)(s + 1) * n_rows);
      std::vector<uint8_t> oo(n_obs, 0);
      std::vector<double> carry;   // messages the previous window handed over
      for (int k = 0; k < run_windows; ++k) {
        const Window& wn = wins[k];
        WindowResult wr;
        if (osd_iters > 0 && (osd_all || wn.last)) {
          // BP+OSD-CS instead of GDG on this window (Sec. III, App. E)
          OsdResult R = osd_window(wn, *P, dd.data() + wn.row0, osd_iters, true, osd_lambda,
                                   osd_keep, nullptr);
          wr.e = R.e;
          wr.flags = R.flags;
          carry.clear();
        } else if (use_warm) {
          std::vector<double> win_in;
          if (!carry.empty()) {
            win_in.resize(wmaps[k].size());
            for (size_t e = 0; e < win_in.size(); ++e)
              win_in[e] = wmaps[k][e] >= 0 ? carry[wmaps[k][e]] : std::nan("");
          }
          std::vector<double> win_out;
          decode_window(wn, *P, dd.data() + wn.row0, wr, nullptr, nullptr, nullptr, 0, -1,
                        carry.empty() ? nullptr : &win_in, &win_out);
          carry.swap(win_out);
        } else {
          decode_window(wn, *P, dd.data() + wn.row0, wr, nullptr, nullptr, nullptr, 0, -1);
        }
        ei += wr.stats.edge_iters;
        if (win_flags) win_flags[(size_t)s * nwin + k] = wr.flags;
        commit_window(d, wn, wr.e.data(), dd.data(), oo.data());
        if (e_out)
          for (int c = 0; c < wn.n; ++c)
            if (wn.commit[c] && wr.e[c]) e_out[(size_t)s * n_cols + wn.src[c]] = 1;
      }
      bool bad = false;
      for (int r = 0; r < n_rows; ++r) bad |= dd[r] != 0;
      for (int o = 0; o < n_obs; ++o) {
        oo[o] ^= obs[(size_t)s * n_obs + o];
        bad |= oo[o] != 0;
      }
      if (det_out) std::memcpy(det_out + (size_t)s * n_rows, dd.data(), n_rows);
      if (obs_out) std::memcpy(obs_out + (size_t)s * n_obs, oo.data(), n_obs);
      fail[s] = bad;
    }
  };
  int nt = std::max(1, n_threads);
  std::vector<std::thread> th;
  for (int i = 1; i < nt; ++i) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
  if (edge_iters) *edge_iters = ei.load();
  return nwin;
}

// ------------------------------------------------------------ unit-level hooks

// Alg. 1 (+ Alg. 3) on given arrays: hist[n][4] posteriors, deg[n], status[n],
// n_unsat[n]. Returns the chosen VN (or -1), fav and agg[n].
int orc_select_vn(int n, const double* hist, const int* deg, const int* status,
                  const int* n_unsat, int low_error, int D, int on_main, int* fav, int* agg) {
  History h;
  h.reset(n);
  for (int i = 0; i < n; ++i)
    for (int t = 0; t < 4; ++t) h.add(i, hist[i * 4 + t]);
  std::vector<int> vn(status, status + n), dg(deg, deg + n), nu(n_unsat, n_unsat + n), ag;
  int f = -1;
  int g = select_vn(vn, dg, h, low_error != 0, D, on_main != 0, nu, &ag, &f);
  *fav = f;
  for (int i = 0; i < n; ++i) agg[i] = ag[i];
  return g;
}

int orc_agg_dec(const double* hist4, int D, int on_main, int n_unsat) {
  History h;
  h.reset(1);
  for (int t = 0; t < 4; ++t) h.add(0, hist4[t]);
  return agg_dec(h.sum[0], h.mn[0], h.mx[0], D, on_main != 0, n_unsat);
}

// Alg. 2 branch rule: value on path `id` at depth D for favoured f; on_main flag.
int orc_path_value(const orc_params* P, int id, int D, int f, int* on_main, int* dmax) {
  auto ps = path_set(*P);
  for (auto& q : ps)
    if (q.id == id) {
      if (on_main) *on_main = path_on_main(q, P->g, D);
      if (dmax) *dmax = q.dmax;
      return path_value(q, P->g, D, f);
    }
  return -1;
}

int orc_n_paths(const orc_params* P) { return (int)path_set(*P).size(); }

// Peeling on a dense [m][n] matrix: status[n] in/out, s[m] in/out. Returns 1 ok,
// 0 contradiction.
int orc_peel(int m, int n, const uint8_t* dense, int* status, int* s) {
  Graph g;
  g.m = m;
  g.n = n;
  g.col_rows.assign(n, {});
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < n; ++c)
      if (dense[(size_t)r * n + c]) g.col_rows[c].push_back(r);
  g.llr.assign(n, 1.0);
  finish_graph(g);
  Status st;
  st.vn.assign(status, status + n);
  st.s.assign(s, s + m);
  st.cdeg.assign(m, 0);
  for (int r = 0; r < m; ++r)
    for (int c : g.row_cols[r])
      if (st.vn[c] < 0) st.cdeg[r] += 1;
  int ok = peel(g, st) ? 1 : 0;
  for (int c = 0; c < n; ++c) status[c] = st.vn[c];
  for (int r = 0; r < m; ++r) s[r] = st.s[r];
  return ok;
}

// Plain BP on a dense [m][n] matrix (no decimation): post[t][n] per iteration.
void orc_dense_bp(int m, int n, const uint8_t* dense, const double* llr, const uint8_t* syn,
                  const orc_params* P, int n_iters, double* post) {
  Graph g;
  g.m = m;
  g.n = n;
  g.col_rows.assign(n, {});
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < n; ++c)
      if (dense[(size_t)r * n + c]) g.col_rows[c].push_back(r);
  g.llr.assign(llr, llr + n);
  finish_graph(g);
  Status st = initial_status(g, syn);
  Messages ms;
  init_messages(g, *P, ms);
  for (int t = 0; t < n_iters; ++t) {
    bp_iteration(g, st, *P, ms);
    std::memcpy(post + (size_t)t * n, ms.post.data(), sizeof(double) * n);
  }
}


// decode_window on a dense problem, preprocessing included when P->pre_iters
// > 0: e[n], the kept columns in ranked order (kept[n], -1 padded; all n in
// order without preprocessing), the ranking keys pre_lsum[n] (the sum of the
// last four preprocessing posteriors; zeros without preprocessing). Returns
// PM; *n_kept receives the number of kept columns (0 if the preprocessing met
// the syndrome).
double orc_dense_window(int m, int n, const uint8_t* dense, const double* llr, const uint8_t* syn,
                        const orc_params* P, uint8_t* e, int* flags, int* kept, int* n_kept,
                        double* pre_lsum, const double* warm_in, double* warm_out) {
  Window win = dense_window(m, n, dense, llr);
  WindowResult wr;
  size_t ne = 0;
  for (int c = 0; c < n; ++c) ne += win.col_rows[c].size();
  std::vector<double> wi, wo;
  if (warm_in) wi.assign(warm_in, warm_in + ne);
  decode_window(win, *P, syn, wr, nullptr, nullptr, nullptr, 0, -1, warm_in ? &wi : nullptr,
                warm_out ? &wo : nullptr);
  if (warm_out)
    for (size_t i = 0; i < ne; ++i) warm_out[i] = i < wo.size() ? wo[i] : std::nan("");
  std::memcpy(e, wr.e.data(), n);
  if (flags) *flags = wr.flags;
  if (n_kept) *n_kept = (int)wr.selected.size();
  if (kept)
    for (int i = 0; i < n; ++i) kept[i] = i < (int)wr.selected.size() ? wr.selected[i] : -1;
  if (pre_lsum)
    for (int c = 0; c < n; ++c) pre_lsum[c] = c < (int)wr.pre_lsum.size() ? wr.pre_lsum[c] : 0.0;
  return wr.pm;
}

// One path (id path_id of the configured tree) of GDG on a dense problem, no
// preprocessing, with the per-step diagnostics of PathProbe: arrays of
// [max_steps][n]. Returns the number of steps probed (steps that reached the
// Alg. 3 / Alg. 1 stage).
int orc_dense_path_probe(int m, int n, const uint8_t* dense, const double* llr,
                         const uint8_t* syn, const orc_params* P, int path_id, int max_steps,
                         double* post, double* hsum, double* hmin, double* hmax, int* status,
                         int* n_unsat, int* agg) {
  Window win = dense_window(m, n, dense, llr);
  Graph g = window_graph(win);
  Status st0 = initial_status(g, syn);
  if (!peel(g, st0)) return -1;
  auto paths = path_set(*P);
  PathSpec ps = paths[0];
  for (auto& q : paths)
    if (q.id == path_id) ps = q;
  PathProbe probe;
  probe.max_steps = max_steps;
  probe.post = post;
  probe.hsum = hsum;
  probe.hmin = hmin;
  probe.hmax = hmax;
  probe.status = status;
  probe.n_unsat = n_unsat;
  probe.agg = agg;
  run_path(g, st0, *P, ps, nullptr, nullptr, 0, &probe);
  return probe.steps;
}

// GDG on a dense [m][n] problem with the given priors (no windowing, no
// preprocessing): e[n], returns PM (infinity if no path met the syndrome).
double orc_dense_gdg(int m, int n, const uint8_t* dense, const double* llr, const uint8_t* syn,
                     const orc_params* P, uint8_t* e, int* flags) {
  Window win;
  win.m = m;
  win.n = n;
  win.col_rows.assign(n, {});
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < n; ++c)
      if (dense[(size_t)r * n + c]) win.col_rows[c].push_back(r);
  win.row_cols.assign(m, {});
  for (int c = 0; c < n; ++c)
    for (int r : win.col_rows[c]) win.row_cols[r].push_back(c);
  win.llr.assign(llr, llr + n);
  win.prior.resize(n);
  win.src.resize(n);
  win.commit.assign(n, 1);
  orc_params Q = *P;
  Q.pre_iters = 0;
  WindowResult wr;
  decode_window(win, Q, syn, wr, nullptr, nullptr, nullptr, 0, -1);
  std::memcpy(e, wr.e.data(), n);
  if (flags) *flags = wr.flags;
  return wr.pm;
}

}  // extern "C"
