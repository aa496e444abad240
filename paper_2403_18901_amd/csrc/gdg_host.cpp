// Host side of the GDG decoder library: window construction (Sec. III, Eq. 6,
// the H_1 -> identity merge), the device layout of the window's Tanner graph,
// the decode kernel's LDS plan, and the extern "C" entry points of gdg.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/gdg.h"
#include "gdg_kernels.h"
#include "gdg_mlp.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? GDG_ENOMEM : GDG_EDEVICE;
}

template <typename T>
int upload(const std::vector<T>& v, T** d) {
  *d = nullptr;
  size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
  hipError_t e = hipMalloc((void**)d, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  if (!v.empty()) {
    e = hipMemcpy(*d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  }
  return GDG_OK;
}

int align16(int x) { return (x + 15) & ~15; }

// Checks the DEM's CSC arrays: indices in range, rows ascending per column,
// priors in (0, 1/2], no column spanning more than two consecutive rounds.
int validate_dem(const gdg_dem* d) {
  if (!d || d->n_rows <= 0 || d->n_cols <= 0 || d->n_obs < 0 || d->w <= 0 || d->n_rounds <= 0)
    return fail(GDG_EINVAL, "dem: bad sizes");
  if ((long long)d->w * d->n_rounds != d->n_rows) return fail(GDG_EINVAL, "dem: n_rows != w*n_rounds");
  if (!d->h_ptr || !d->h_idx || !d->l_ptr || !d->priors || (d->l_ptr[d->n_cols] > 0 && !d->l_idx))
    return fail(GDG_EINVAL, "dem: null array");
  if (d->h_ptr[0] != 0 || d->l_ptr[0] != 0) return fail(GDG_EINVAL, "dem: pointers must start at 0");
  for (int c = 0; c < d->n_cols; ++c) {
    int a = d->h_ptr[c], b = d->h_ptr[c + 1];
    if (b <= a) return fail(GDG_EINVAL, "dem: empty or decreasing column");
    for (int e = a; e < b; ++e) {
      int r = d->h_idx[e];
      if (r < 0 || r >= d->n_rows) return fail(GDG_EINVAL, "dem: row index out of range");
      if (e > a && r <= d->h_idx[e - 1]) return fail(GDG_EINVAL, "dem: rows not ascending");
    }
    if (d->h_idx[b - 1] / d->w - d->h_idx[a] / d->w > 1)
      return fail(GDG_EINVAL, "dem: column spans more than two rounds");
    if (d->l_ptr[c + 1] < d->l_ptr[c]) return fail(GDG_EINVAL, "dem: bad observable pointers");
    for (int e = d->l_ptr[c]; e < d->l_ptr[c + 1]; ++e)
      if (d->l_idx[e] < 0 || d->l_idx[e] >= d->n_obs)
        return fail(GDG_EINVAL, "dem: observable index out of range");
    double p = d->priors[c];
    if (!(p > 0.0 && p <= 0.5)) return fail(GDG_EINVAL, "dem: prior outside (0, 1/2]");
  }
  return GDG_OK;
}

}  // namespace

struct gdg_window {
  gdg_window_info info{};
  gdg_params prm{};
  std::vector<int> src;
  std::vector<double> llr64;
  std::vector<uint8_t> commit;
  gdg_win_dev dev{};
  gdg_lds lds{};
  gdg_commit_dev cm{};
  int waves = 1;
  int max_sub = 0;
  int bucket = 0;
  gdg_win_dev* d_dev = nullptr;   // device copy of dev
  // host copies for linking windows (warm start): the window CSR and each
  // CSR edge's message slot in the preprocessing layout
  std::vector<int> h_row_ptr, epos;
  std::vector<uint16_t> h_row_col;
  gdg_lds* d_plans = nullptr;     // device LDS plans for 1..8 wavefronts (index waves-1)
  gdg_lds plans[8]{};
  std::vector<void*> allocs;

  ~gdg_window() {
    for (void* p : allocs) (void)hipFree(p);
  }
  template <typename T>
  int put(const std::vector<T>& v, const T** out) {
    T* d = nullptr;
    int rc = upload(v, &d);
    if (d) allocs.push_back(d);
    *out = d;
    return rc;
  }
};

struct gdg_model {
  gdg_model_dev dev{};
  std::vector<void*> allocs;
  ~gdg_model() {
    for (void* p : allocs) (void)hipFree(p);
  }
};

struct gdg_dem_dev {
  gdg_dem_dev_k k{};
  std::vector<void*> allocs;
  ~gdg_dem_dev() {
    for (void* p : allocs) (void)hipFree(p);
  }
};

namespace {

// LDS plan of the decode kernel for `waves` wavefronts per workgroup.
// LDS layout of the decode kernel for one window. max_sub_edges bounds the
// truncated graph's edges, col_slots its column slots padded to multiples of
// four, tcols the slot columns of its row groups (see the kernel). The total
// is the least allocation that decodes any shot: the preprocessing, the
// sub-graph build with the worst truncation, and one path wavefront on it.
gdg_lds plan_lds(const gdg_win_dev& w, int max_sub_edges, int col_slots, int tcols, int waves) {
  gdg_lds L{};
  const int m = w.m, n = w.n, na = w.n_act, E = max_sub_edges, P = w.n_paths;
  const int e_pad_max = E + 3 * m;   // rows padded to a multiple of 4 edges
  int off = 0;
  auto take = [&](int bytes) {
    int o = off;
    off = align16(off + bytes);
    return o;
  };
  L.pbits_words = (na + 31) / 32;
  L.obits_words = (n + 31) / 32 + 1;
  L.meta_cols = tcols;
  L.sorig = take(m);
  L.sel = take(2 * na);
  L.misc = take(64);
  L.obits = take(4 * L.obits_words);
  L.eacc = take(8);
  L.u_base = off;
  // preprocessing region
  int prep = 0;
  L.sort_n = 1;
  while (L.sort_n < n) L.sort_n <<= 1;
  if (w.pre_iters > 0) {
    int po = 0;
    auto ptake = [&](int bytes) {
      int o = po;
      po = align16(po + bytes);
      return o;
    };
    L.p_post = ptake(4 * (n + 1));   // + the padding's dummy VN
    // the ranking's radix-select scratch reuses the message array
    int sort_p = 1;   // the kept keys, padded to a power of two for the sort
    while (sort_p < na) sort_p <<= 1;
    const int rank_bytes = 4 * (256 + 4) + 8 * sort_p;
    const int c2v_bytes = std::max(std::max(4 * (w.fr_epad + 8), 8 * L.sort_n), rank_bytes);
    L.p_c2v = ptake(c2v_bytes);
    L.p_keys = L.p_c2v;   // the sort keys reuse the message array
    L.p_lsum = ptake(4 * n);
    prep = po;
  }
  // sub-graph arrays of fixed size, written after the preprocessing is dead
  int so = 0;
  auto stake = [&](int bytes) {
    int o = so;
    so = align16(so + bytes);
    return o;
  };
  L.psyn = stake(m);
  L.rptr = stake(2 * (m + 1));
  L.cptr = stake(2 * (na + 1));
  L.vdeg = stake(na);
  L.st0 = stake(na);        // VN status after the peeling at a path's start
  L.sres0 = stake(4 * 64);  // per lane, the residual syndrome bits after it
  L.ppm = stake(8 * P);
  L.pend = stake(4 * P);
  L.pbits = stake(4 * P * L.pbits_words);
  L.tq = stake(4 * 8 * P);    // path task queue: 8 ints per task
  L.tready = stake(4 * P);
  L.dyn_base = so;
  const gdg_dyn_layout worst = gdg_dyn(L.dyn_base, e_pad_max, col_slots, tcols, !w.low_error);
  // sub-graph build scratch above the largest variable part
  int bo = worst.end;
  auto btake = [&](int bytes) {
    int o = bo;
    bo = align16(bo + bytes);
    return o;
  };
  L.p_loc = btake(2 * n + 2 * m);   // column map and row order
  L.p_iscan = btake(4 * std::max(2 * m + 2, na + 1));
  L.p_llr = btake(4 * na);
  L.p_deg = btake(na);
  const int one_path = worst.end + gdg_paths(e_pad_max, na, m, L.obits_words).stride;
  L.total = L.u_base + std::max(prep, std::max(bo, one_path));
  // the preprocessing keeps up to 64 slot columns' syndrome bits per wavefront
  if (w.pre_iters > 0 && (w.fr_T + waves - 1) / waves > 64) L.total = 1 << 30;
  return L;
}

// Lane-group layout of the whole window graph (the scheme the decode kernel
// builds per shot for the truncated graph; see gdg_kernels.hip).
struct FullLayout {
  std::vector<uint32_t> meta;
  std::vector<uint16_t> rvn, cidx;
  std::vector<int> cptr;
  std::vector<int> epos;   // message slot of each CSR edge
  int T = 0, epad = 0;
};

bool full_layout(int m, int n, const std::vector<int>& row_ptr, const std::vector<uint16_t>& row_col,
                 const std::vector<uint8_t>& row_kcol, const std::vector<int>& col_ptr,
                 FullLayout& F) {
  std::vector<int> order(m);
  for (int j = 0; j < m; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return row_ptr[a + 1] - row_ptr[a] > row_ptr[b + 1] - row_ptr[b];
  });
  std::vector<int> start(m), nb(m), k(m);
  int epad = 0, slots = 0;
  for (int pj = 0; pj < m; ++pj) {
    const int j = order[pj], d = row_ptr[j + 1] - row_ptr[j];
    start[pj] = epad;
    nb[pj] = (d + 3) / 4;
    int kk = nb[pj] ? 1 : 0;
    while (kk && kk < nb[pj]) kk *= 2;
    k[pj] = kk;
    epad += 4 * nb[pj];
    slots += kk;
  }
  if (epad + 8 > 16383 || 4 * n > 65535 || m > 1023) return false;
  F.epad = epad;
  F.T = (slots + 63) / 64;
  F.cptr.assign(n + 1, 0);
  for (int c = 0; c < n; ++c) F.cptr[c + 1] = F.cptr[c] + (col_ptr[c + 1] - col_ptr[c] + 3) / 4 * 4;
  F.cidx.assign(std::max(F.cptr[n], 4), (uint16_t)(4 * epad));   // padding: the zero message
  F.rvn.assign(epad + 8, (uint16_t)(4 * n));                        // padding: the dummy VN
  // idle lanes point at the dummy batch; 3 idle columns per wavefront (up to 8)
  // past the end take the loads the CN walk issues ahead of its last slots
  F.meta.assign((size_t)(F.T + 3 * 8) * 64, (uint32_t)(epad + 4));
  F.epos.assign(row_ptr[m], 0);
  int g = 0;
  for (int pj = 0; pj < m; ++pj) {
    const int j = order[pj];
    int pos = start[pj];
    for (int e = row_ptr[j]; e < row_ptr[j + 1]; ++e, ++pos) {
      const int c = row_col[e];
      F.epos[e] = pos;
      F.rvn[pos] = (uint16_t)(4 * c);
      F.cidx[F.cptr[c] + row_kcol[e]] = (uint16_t)(4 * pos);
    }
    if (!k[pj]) continue;
    int lk = 0;
    while ((1 << lk) < k[pj]) ++lk;
    for (int i = 0; i < k[pj]; ++i, ++g) {
      const int e0 = i < nb[pj] ? start[pj] + 4 * i : epad + 4;
      F.meta[g] = (uint32_t)e0 | ((uint32_t)j << kMetaRowShift) | ((uint32_t)lk << kMetaLogKShift) |
                  (i == 0 ? kMetaLead : 0u) | kMetaValid;
    }
  }
  return true;
}

// Most slot columns any truncation can need: rows of window degree D_j hold
// d_j <= D_j kept edges, sum d_j <= max_sub; a row of d edges takes the power
// of two >= ceil(d / 4) lanes. Knapsack over the edge budget.
int slot_columns_bound(const std::vector<int>& row_deg, int max_sub) {
  std::vector<int> dp(max_sub + 1, 0), nd;
  static const int kD[] = {1, 5, 9, 17, 33, 65};
  static const int kK[] = {1, 2, 4, 8, 16, 32};
  for (int Dj : row_deg) {
    nd = dp;
    for (int c = 0; c < 6 && kD[c] <= Dj; ++c)
      for (int e = kD[c]; e <= max_sub; ++e) nd[e] = std::max(nd[e], dp[e - kD[c]] + kK[c]);
    dp.swap(nd);
  }
  int best = 0;
  for (int v : dp) best = std::max(best, v);
  return (best + 63) / 64;
}

int max_lds_per_block() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 65536;
  return v > 0 ? v : 65536;
}

int cu_count() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
  return v > 0 ? v : 1;
}

// Device scratch of the decode launches on one stream when the caller gives
// no workspace: the shot counter followed by the path checkpoints. Launches on
// one stream run in order, so they can share it; it grows on demand (after
// synchronising the stream) and is kept until gdg_release_scratch or the
// process ends.
struct StreamScratch {
  int dev = 0;
  hipStream_t st = nullptr;
  char* base = nullptr;     // [256 B counter][ckpt_bytes of checkpoints]
  size_t ckpt_bytes = 0;
};
std::mutex g_scratch_mu;
std::vector<StreamScratch> g_scratch;

int stream_scratch(hipStream_t st, size_t ckpt_bytes, StreamScratch* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  StreamScratch* s = nullptr;
  for (StreamScratch& x : g_scratch)
    if (x.dev == dev && x.st == st) s = &x;
  if (!s) {
    g_scratch.push_back(StreamScratch{});
    s = &g_scratch.back();
    s->dev = dev;
    s->st = st;
  }
  if (!s->base || ckpt_bytes > s->ckpt_bytes) {
    if (s->base) {
      e = hipStreamSynchronize(st);   // earlier launches may still use the old block
      if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
      (void)hipFree(s->base);
      s->base = nullptr;
      s->ckpt_bytes = 0;
    }
    e = hipMalloc((void**)&s->base, 256 + ckpt_bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc (decode scratch)");
    s->ckpt_bytes = ckpt_bytes;
  }
  *out = *s;
  return GDG_OK;
}

int lds_per_cu() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
      hipSuccess)
    return 65536;
  return v > 0 ? v : 65536;
}

}  // namespace

extern "C" {

const char* gdg_last_error(void) { return g_err.c_str(); }

int gdg_build_window(const gdg_dem* dem, int32_t k, int32_t W, int32_t F, const gdg_params* prm,
                     gdg_window** out) {
  if (!out || !prm) return fail(GDG_EINVAL, "null argument");
  *out = nullptr;
  int rc = validate_dem(dem);
  if (rc) return rc;
  if (W < 1 || F < 1 || F > W) return fail(GDG_EINVAL, "need 1 <= F <= W");
  if (k < 0 || (long long)k * F >= dem->n_rounds) return fail(GDG_EINVAL, "window out of range");
  if (prm->iters_per_step < 4) return fail(GDG_EINVAL, "iters_per_step must be >= 4");
  if (prm->g < 0 || prm->g > 5) return fail(GDG_EINVAL, "g must be in 0..5");
  if (prm->dmax_main < 1 || prm->extra_steps < 0 || prm->pre_iters < 0 || prm->trunc_factor < 1)
    return fail(GDG_EINVAL, "bad step limits");
  if (!(prm->clip > 0.0f) || !(prm->alpha > 0.0f)) return fail(GDG_EINVAL, "bad alpha/clip");

  const int w = dem->w;
  const int r0 = k * F;                              // first round of the window
  const int Wk = std::min(W, dem->n_rounds - r0);    // rounds in it (the last may have fewer)
  const int row0 = r0 * w, m = Wk * w, last_round = r0 + Wk - 1;
  const bool last = (r0 + W >= dem->n_rounds);
  std::unique_ptr<gdg_window> win(new gdg_window());
  win->prm = *prm;
  // window columns: DEM columns starting inside, not reaching past; then unit columns
  std::vector<std::vector<int>> col_rows;
  std::vector<double> prior;
  std::vector<double> keep(m, 1.0);
  std::vector<char> touched(m, 0);
  for (int c = 0; c < dem->n_cols; ++c) {
    const int a = dem->h_ptr[c], b = dem->h_ptr[c + 1];
    const int fr = dem->h_idx[a] / w, lr = dem->h_idx[b - 1] / w;
    if (fr < r0 || fr > last_round) continue;
    if (lr > last_round) {
      for (int e = a; e < b; ++e) {
        const int r = dem->h_idx[e];
        if (r / w != last_round) continue;
        keep[r - row0] *= (1.0 - 2.0 * dem->priors[c]);
        touched[r - row0] = 1;
      }
      continue;
    }
    std::vector<int> rows;
    for (int e = a; e < b; ++e) rows.push_back(dem->h_idx[e] - row0);
    col_rows.push_back(rows);
    prior.push_back(dem->priors[c]);
    win->src.push_back(c);
    win->commit.push_back((uint8_t)(last || fr < r0 + F));
  }
  for (int r = 0; r < m; ++r) {
    if (!touched[r]) continue;
    col_rows.push_back(std::vector<int>{r});
    prior.push_back(0.5 * (1.0 - keep[r]));
    win->src.push_back(-1 - r);
    win->commit.push_back(0);
  }
  const int n = (int)col_rows.size();
  if (n == 0) return fail(GDG_EINVAL, "empty window");
  if (n > 65535 || m > 512) return fail(GDG_ESHAPE, "window too large");
  win->llr64.resize(n);
  for (int c = 0; c < n; ++c) win->llr64[c] = std::log((1.0 - prior[c]) / prior[c]);

  // CSC and CSR
  std::vector<int> col_ptr(n + 1, 0);
  for (int c = 0; c < n; ++c) col_ptr[c + 1] = col_ptr[c] + (int)col_rows[c].size();
  const int E = col_ptr[n];
  if (E > 1 << 24) return fail(GDG_ESHAPE, "too many edges");
  std::vector<std::vector<std::pair<int, int>>> rows(m);   // (column, position in column)
  for (int c = 0; c < n; ++c)
    for (size_t t = 0; t < col_rows[c].size(); ++t) rows[col_rows[c][t]].push_back({c, (int)t});
  std::vector<int> row_ptr(m + 1, 0);
  std::vector<uint16_t> row_col;
  std::vector<uint8_t> row_kcol, deg(n);
  int max_row = 0;
  for (int r = 0; r < m; ++r) {
    row_ptr[r + 1] = row_ptr[r] + (int)rows[r].size();
    max_row = std::max(max_row, (int)rows[r].size());
    for (auto& pr : rows[r]) {
      row_col.push_back((uint16_t)pr.first);
      row_kcol.push_back((uint8_t)pr.second);
    }
  }
  if (max_row > 64) return fail(GDG_ESHAPE, "a window row has more than 64 columns");
  if (E > 65535) return fail(GDG_ESHAPE, "window has more than 65535 edges");
  std::vector<uint32_t> row_cs(E);
  for (int e = 0; e < E; ++e) row_cs[e] = (uint32_t)row_col[e] | ((uint32_t)(col_ptr[row_col[e]] + row_kcol[e]) << 16);
  int max_col = 0;
  for (int c = 0; c < n; ++c) {
    deg[c] = (uint8_t)col_rows[c].size();
    max_col = std::max(max_col, (int)col_rows[c].size());
  }
  if (max_col > 255) return fail(GDG_ESHAPE, "column degree above 255");
  std::vector<float> llr(n);
  for (int c = 0; c < n; ++c) llr[c] = (float)win->llr64[c];

  const int n_act = prm->pre_iters > 0 ? std::min(n, prm->trunc_factor * m) : n;
  std::vector<int> degs(deg.begin(), deg.end());
  std::sort(degs.begin(), degs.end(), std::greater<int>());
  int max_sub = 0, col_slots = 0;
  for (int i = 0; i < n_act; ++i) {
    max_sub += degs[i];
    col_slots += (degs[i] + 3) / 4 * 4;
  }
  // CSR positions (14-bit slot field) and byte offsets (16 bit) must fit
  if (max_sub + 3 * m + 8 > 16383 || n_act > 1024) return fail(GDG_ESHAPE, "truncated graph too large");
  std::vector<int> row_deg(m);
  for (int r = 0; r < m; ++r) row_deg[r] = row_ptr[r + 1] - row_ptr[r];
  const int tcols = slot_columns_bound(row_deg, max_sub);
  if (tcols > 32) return fail(GDG_ESHAPE, "truncated graph needs more than 32 slot columns");
  int n_paths = prm->g > 0 ? (1 << prm->g) : 1;
  if (prm->g > 0 && prm->side_max_depth > prm->g) n_paths += prm->side_max_depth - prm->g;

  gdg_win_dev& D = win->dev;
  D.m = m;
  D.n = n;
  D.n_act = n_act;
  D.e_full = E;
  D.n_paths = n_paths;
  D.g = prm->g;
  D.dmax_main = prm->dmax_main;
  D.extra = prm->extra_steps;
  D.side_max_depth = prm->side_max_depth;
  D.low_error = prm->low_error ? 1 : 0;
  D.iters = prm->iters_per_step;
  D.pre_iters = prm->pre_iters;
  D.bound_ok = 1;
  for (double x : win->llr64)
    if (!(x > 0.0)) D.bound_ok = 0;
  D.alpha = prm->alpha;
  D.clip = prm->clip;
  if ((rc = win->put(row_ptr, &D.row_ptr))) return rc;
  if ((rc = win->put(row_col, &D.row_col))) return rc;
  if ((rc = win->put(row_kcol, &D.row_kcol))) return rc;
  if ((rc = win->put(row_cs, &D.row_cs))) return rc;
  if ((rc = win->put(col_ptr, &D.col_ptr))) return rc;
  if ((rc = win->put(llr, &D.llr))) return rc;
  if ((rc = win->put(win->llr64, &D.llr64))) return rc;
  if ((rc = win->put(deg, &D.deg))) return rc;
  {
    FullLayout F;
    if (!full_layout(m, n, row_ptr, row_col, row_kcol, col_ptr, F))
      return fail(GDG_ESHAPE, "window too large for the preprocessing layout");
    D.fr_T = F.T;
    D.fr_epad = F.epad;
    win->epos = F.epos;
    win->h_row_ptr = row_ptr;
    win->h_row_col = row_col;
    if ((rc = win->put(F.meta, &D.fr_meta))) return rc;
    {
      std::vector<uint32_t> rec(4 * F.meta.size());
      for (size_t i = 0; i < F.meta.size(); ++i) {
        const uint32_t e0 = F.meta[i] & kMetaEdge;
        rec[4 * i + 0] = F.meta[i];
        rec[4 * i + 1] = F.rvn[e0] | (uint32_t)F.rvn[e0 + 1] << 16;
        rec[4 * i + 2] = F.rvn[e0 + 2] | (uint32_t)F.rvn[e0 + 3] << 16;
        rec[4 * i + 3] = 0;
      }
      const uint32_t* rp = nullptr;
      if ((rc = win->put(rec, &rp))) return rc;
      D.fr_rec = reinterpret_cast<const uint4*>(rp);
    }
    if ((rc = win->put(F.rvn, &D.fr_rvn))) return rc;
    if ((rc = win->put(F.cidx, &D.fr_cidx))) return rc;
    if ((rc = win->put(F.cptr, &D.fr_cptr))) return rc;
    std::vector<uint32_t> vrec(4 * (size_t)n);
    const uint32_t zero = (uint32_t)(4 * F.epad);
    for (int c = 0; c < n; ++c) {
      const int c0 = F.cptr[c], d = deg[c];
      auto slot = [&](int k) { return k < d ? (uint32_t)F.cidx[c0 + k] : zero; };
      vrec[4 * c + 0] = slot(0) | slot(1) << 16;
      vrec[4 * c + 1] = slot(2) | slot(3) << 16;
      vrec[4 * c + 2] = slot(4) | (uint32_t)d << 16;
      uint32_t lb;
      std::memcpy(&lb, &llr[c], 4);
      vrec[4 * c + 3] = lb;
    }
    const uint32_t* vp = nullptr;
    if ((rc = win->put(vrec, &vp))) return rc;
    D.fr_vrec = reinterpret_cast<const uint4*>(vp);
  }

  // commit tables
  std::vector<std::vector<int>> by_row(dem->n_rows);
  std::vector<std::vector<int>> by_obs(dem->n_obs);
  int n_commit = 0;
  for (int c = 0; c < n; ++c) {
    if (!win->commit[c]) continue;
    ++n_commit;
    const int dc = win->src[c];
    for (int e = dem->h_ptr[dc]; e < dem->h_ptr[dc + 1]; ++e) by_row[dem->h_idx[e]].push_back(c);
    for (int e = dem->l_ptr[dc]; e < dem->l_ptr[dc + 1]; ++e) by_obs[dem->l_idx[e]].push_back(c);
  }
  std::vector<int> rg, rp(1, 0), rc_, op(1, 0), oc;
  for (int r = 0; r < dem->n_rows; ++r) {
    if (by_row[r].empty()) continue;
    rg.push_back(r);
    rc_.insert(rc_.end(), by_row[r].begin(), by_row[r].end());
    rp.push_back((int)rc_.size());
  }
  for (int o = 0; o < dem->n_obs; ++o) {
    oc.insert(oc.end(), by_obs[o].begin(), by_obs[o].end());
    op.push_back((int)oc.size());
  }
  win->cm.n_rows = (int)rg.size();
  win->cm.n_obs = dem->n_obs;
  win->cm.n_win = n;
  if ((rc = win->put(rg, &win->cm.row_global))) return rc;
  if ((rc = win->put(rp, &win->cm.row_ptr))) return rc;
  if ((rc = win->put(rc_, &win->cm.row_col))) return rc;
  if ((rc = win->put(op, &win->cm.obs_ptr))) return rc;
  if ((rc = win->put(oc, &win->cm.obs_col))) return rc;

  // Default LDS plan: four wavefronts (as many as paths if fewer and no
  // whole-window preprocessing), within the per-workgroup LDS limit. Measured on
  // MI355X for [[144,12,12]] windows: two 4-wave workgroups per CU beat one
  // 8-wave one. gdg_decode_jobs may choose another shape per launch.
  const int limit = max_lds_per_block();
  int waves = std::min(4, n_paths);
  if (prm->pre_iters > 0) waves = 4;
  gdg_lds L = plan_lds(D, max_sub, col_slots, tcols, waves);
  while (L.total > limit && waves > 1) {
    waves /= 2;
    L = plan_lds(D, max_sub, col_slots, tcols, waves);
  }
  if (L.total > limit) return fail(GDG_ESHAPE, "window does not fit in LDS");
  win->bucket = gdg_kernel_bucket(m, n_act);
  if (win->bucket < 0) return fail(GDG_ESHAPE, "window exceeds the kernel's register tiling");
  win->lds = L;
  win->waves = waves;
  win->max_sub = max_sub;
  {
    std::vector<gdg_win_dev> one(1, D);
    const gdg_win_dev* p = nullptr;
    if ((rc = win->put(one, &p))) return rc;
    win->d_dev = const_cast<gdg_win_dev*>(p);
    std::vector<gdg_lds> plans(8);
    for (int wv = 1; wv <= 8; ++wv)
      plans[wv - 1] = win->plans[wv - 1] = plan_lds(D, max_sub, col_slots, tcols, wv);
    const gdg_lds* q = nullptr;
    if ((rc = win->put(plans, &q))) return rc;
    win->d_plans = const_cast<gdg_lds*>(q);
  }

  gdg_window_info& I = win->info;
  I.k = k;
  I.W = Wk;
  I.m = m;
  I.n = n;
  I.row0 = row0;
  I.n_act = n_act;
  I.n_paths = n_paths;
  I.n_edges = E;
  I.max_sub_edges = max_sub;
  I.n_commit = n_commit;
  I.last = last ? 1 : 0;
  I.lds_bytes = L.total;
  I.waves = waves;
  I.n_msg = D.fr_epad;
  *out = win.release();
  return GDG_OK;
}

void gdg_window_free(gdg_window* win) { delete win; }

int gdg_window_get_info(const gdg_window* win, gdg_window_info* info) {
  if (!win || !info) return fail(GDG_EINVAL, "null argument");
  *info = win->info;
  return GDG_OK;
}

int gdg_link_windows(gdg_window* next, const gdg_window* prev) {
  if (!next || !prev) return fail(GDG_EINVAL, "null window");
  if (next->dev.pre_iters <= 0)
    return fail(GDG_EINVAL, "the window has no preprocessing BP to warm-start");
  // previous window: DEM column -> window column
  std::unordered_map<int, int> pcol;
  for (int c = 0; c < prev->info.n; ++c)
    if (prev->src[c] >= 0) pcol[prev->src[c]] = c;
  std::vector<int> map(std::max(1, next->dev.fr_epad), -1);
  const int shift = next->info.row0 - prev->info.row0;
  for (int j = 0; j < next->info.m; ++j) {
    const int jp = j + shift;   // the same detector row in the previous window
    if (jp < 0 || jp >= prev->info.m) continue;
    const uint16_t* pb = prev->h_row_col.data() + prev->h_row_ptr[jp];
    const uint16_t* pe = prev->h_row_col.data() + prev->h_row_ptr[jp + 1];
    for (int e = next->h_row_ptr[j]; e < next->h_row_ptr[j + 1]; ++e) {
      const int sc = next->src[next->h_row_col[e]];
      if (sc < 0) continue;   // a unit column of merged faults
      auto it = pcol.find(sc);
      if (it == pcol.end()) continue;
      const uint16_t* f = std::lower_bound(pb, pe, (uint16_t)it->second);
      if (f == pe || *f != it->second) continue;
      map[next->epos[e]] = prev->epos[prev->h_row_ptr[jp] + (int)(f - pb)];
    }
  }
  const int* d = nullptr;
  int rc = next->put(map, &d);
  if (rc) return rc;
  next->dev.warm_map = d;
  next->dev.warm_prev_slots = prev->dev.fr_epad;
  hipError_t e = hipMemcpy(next->d_dev, &next->dev, sizeof(gdg_win_dev), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  return GDG_OK;
}

int gdg_window_edge_slots(const gdg_window* win, int32_t* slot) {
  if (!win || !slot) return fail(GDG_EINVAL, "null argument");
  for (size_t e = 0; e < win->epos.size(); ++e) slot[e] = win->epos[e];
  return GDG_OK;
}

int gdg_window_columns(const gdg_window* win, int32_t* src, double* llr, uint8_t* commit) {
  if (!win) return fail(GDG_EINVAL, "null window");
  const int n = win->info.n;
  for (int c = 0; c < n; ++c) {
    if (src) src[c] = win->src[c];
    if (llr) llr[c] = win->llr64[c];
    if (commit) commit[c] = win->commit[c];
  }
  return GDG_OK;
}

}  // extern "C"

namespace {

int g_lds_set[5] = {65536, 65536, 65536, 65536, 65536};   // dynamic-LDS limit set per kernel bucket

// Shape of one decode launch, fixed before any scratch is chosen: the LDS
// allocation, register tiling, persistent grid and checkpoint geometry.
struct LaunchGeom {
  int lds = 0, bucket = 0, grid = 0, total = 0;
  bool low = true;         // every window in low-error mode
  int slots = 0;           // checkpoint slots per workgroup (0: no tree)
  long long stride = 0;    // bytes per checkpoint slot
  long long ck_per_wg() const { return (long long)slots * stride; }
};

constexpr size_t kCounterBytes = 256;   // the persistent grid's shot counter, first in any scratch

int launch_geometry(const gdg_job* jobs, int n_jobs, int waves, int workgroups, bool learn,
                    LaunchGeom& G) {
  if (!jobs || n_jobs < 1 || n_jobs > GDG_MAX_JOBS) return fail(GDG_EINVAL, "1..8 jobs per launch");
  if (waves < 1 || waves > 8) return fail(GDG_EINVAL, "waves must be in 1..8");
  if (workgroups < 0) return fail(GDG_EINVAL, "negative workgroup count");
  G = LaunchGeom{};
  for (int j = 0; j < n_jobs; ++j) {
    const gdg_window* win = jobs[j].win;
    if (!win) return fail(GDG_EINVAL, "job without a window");
    if (jobs[j].n_shots < 0) return fail(GDG_EINVAL, "negative n_shots");
    G.total += jobs[j].n_shots;
    G.lds = std::max(G.lds, win->plans[waves - 1].total);
    G.bucket = std::max(G.bucket, win->bucket);
    G.low = G.low && win->dev.low_error;
    const int n_tree = win->dev.g > 0 ? 1 << win->dev.g : 1;
    G.slots = std::max(G.slots, n_tree - 1);
    const int e_pad_max = win->max_sub + 3 * win->dev.m;
    G.stride = std::max(G.stride, (long long)(gdg_ck(win->dev.n_act, e_pad_max).bytes + 255) / 256 * 256);
  }
  if (G.lds > max_lds_per_block()) return fail(GDG_ESHAPE, "jobs do not fit in LDS at this shape");
  // Allocate the CU's LDS share at the occupancy the kernel is built for (or
  // the plans' minimum if larger): shots with larger sub-graphs then still
  // get all their path wavefronts.
  const int wps = gdg_decode_waves_per_simd(G.bucket, learn);
  int wg_per_cu = 4 * wps / waves;
  // A launch with fewer shots than that many workgroups per CU (small
  // streaming batches) needs fewer per CU: each then gets a larger share, so
  // large sub-graphs still fit all their path wavefronts and a shot's latency
  // does not grow.
  if (workgroups <= 0) {
    const int need = (int)((G.total + (long long)cu_count() - 1) / cu_count());
    wg_per_cu = std::max(1, std::min(wg_per_cu, need));
  }
  if (wg_per_cu >= 2)   // whole 2 KiB granules, so that the shares add up within the CU
    G.lds = std::max(G.lds, std::min(lds_per_cu() / wg_per_cu / 2048 * 2048, max_lds_per_block()));
  else   // one per CU: most of the CU's LDS (the full 160 KiB is refused as a dynamic size)
    G.lds = std::max(G.lds, (max_lds_per_block() - 16384) / 2048 * 2048);
  // Persistent grid at the resident workgroup count (or the caller's count):
  // workgroups take shots from a counter, and each owns the checkpoints where
  // its paths' decision tree splits.
  const int by_lds = std::max(1, lds_per_cu() / ((G.lds + 2047) / 2048 * 2048));
  const int by_waves = std::max(1, 4 * wps / waves);
  const int resident = std::min(by_lds, by_waves) * cu_count();
  G.grid = workgroups > 0 ? std::min(workgroups, G.total) : std::min(G.total, resident);
  return GDG_OK;
}

// Warm-start buffers of one job (gdg_decode_batch_warm).
struct WarmIO {
  const float* in = nullptr;
  float* out = nullptr;
  long long in_stride = 0, out_stride = 0;
};

// Launches the decode with the given scratch: the shot counter at `scratch`
// and checkpoint slots for as many workgroups as fit in the rest (the others
// replay their paths from the root, which gives the same results). Allocates
// nothing. With `chain` the items are the experiments of a chained launch.
int launch_with_scratch(const gdg_job* jobs, int n_jobs, int waves, const LaunchGeom& G,
                        const gdg_trace_dev& tr, hipStream_t st, const gdg_learn_dev* learn,
                        void* scratch, size_t scratch_bytes, const WarmIO* warm = nullptr,
                        const gdg_chain_dev* chain = nullptr) {
  gdg_jobs_dev J{};
  for (int j = 0; j < n_jobs; ++j) {
    const gdg_job& jb = jobs[j];
    if (jb.n_shots > 0) {
      if (!jb.d_syndrome || !jb.d_ehat || !jb.d_pm || !jb.d_flags)
        return fail(GDG_EINVAL, "null buffer");
      if (jb.syn_stride < jb.win->info.m) return fail(GDG_EINVAL, "syn_stride < m");
    }
  }
  if (G.total == 0) return GDG_OK;
  if (!scratch || scratch_bytes < kCounterBytes || ((uintptr_t)scratch & 255u))
    return fail(GDG_EINVAL, "scratch must be 256-byte aligned and hold at least 256 bytes");
  int item0 = 0;
  for (int j = 0; j < n_jobs; ++j) {
    const gdg_job& jb = jobs[j];
    gdg_job_dev& d = J.job[j];
    d.w = jb.win->d_dev;
    d.L = jb.win->d_plans + (waves - 1);
    d.item0 = item0;
    d.n_shots = jb.n_shots;
    d.syn = jb.d_syndrome;
    d.syn_stride = jb.syn_stride;
    d.ehat = jb.d_ehat;
    d.pm = jb.d_pm;
    d.flags = jb.d_flags;
    item0 += jb.n_shots;
  }
  J.n_jobs = n_jobs;
  J.total = G.total;
  if (chain) J.chain = *chain;
  if (warm) {
    if (n_jobs != 1) return fail(GDG_EINVAL, "a warm start takes a one-job launch");
    J.warm_in = warm->in;
    J.warm_out = warm->out;
    J.warm_in_stride = warm->in_stride;
    J.warm_out_stride = warm->out_stride;
  }
  if (learn) J.learn = *learn;
  J.lds = G.lds;
  if (G.lds > g_lds_set[G.bucket]) {
    hipError_t e = gdg_decode_set_lds_limit(G.bucket, G.lds);
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    g_lds_set[G.bucket] = G.lds;
  }
  J.work = (int*)scratch;
  J.ckpt = nullptr;
  J.ckpt_wgs = 0;
  if (G.slots > 0) {
    const long long fit = (long long)(scratch_bytes - kCounterBytes) / G.ck_per_wg();
    J.ckpt_wgs = (int)std::min<long long>(fit, G.grid);
    if (J.ckpt_wgs > 0) J.ckpt = (char*)scratch + kCounterBytes;
  }
  J.ckpt_stride = G.stride;
  J.ckpt_slots = G.slots;
  hipError_t e = gdg_launch_zero(J.work, 1, st);
  if (e != hipSuccess) return hip_fail(e, "counter reset");
  e = chain ? gdg_launch_chain(J, G.bucket, G.low, waves, G.grid, G.lds, st)
            : gdg_launch_jobs(J, G.bucket, G.low, waves, G.grid, G.lds, tr, st);
  if (e != hipSuccess) return hip_fail(e, "decode launch");
  return GDG_OK;
}

// Decode launch on the library's per-stream scratch (allocated or grown here).
int launch_jobs(const gdg_job* jobs, int n_jobs, int waves, int workgroups,
                const gdg_trace_dev& tr, hipStream_t st, const gdg_learn_dev* learn = nullptr,
                const WarmIO* warm = nullptr, const gdg_chain_dev* chain = nullptr) {
  LaunchGeom G;
  int rc = launch_geometry(jobs, n_jobs, waves, workgroups, learn && learn->mode != 0, G);
  if (rc) return rc;
  if (G.total == 0)
    return launch_with_scratch(jobs, n_jobs, waves, G, tr, st, learn, nullptr, 0, warm, chain);
  StreamScratch sc;
  rc = stream_scratch(st, (size_t)G.grid * G.ck_per_wg(), &sc);
  if (rc) return rc;
  return launch_with_scratch(jobs, n_jobs, waves, G, tr, st, learn, sc.base,
                             kCounterBytes + sc.ckpt_bytes, warm, chain);
}

}  // namespace

extern "C" {

size_t gdg_workspace_bytes(const gdg_window* win, int32_t n_shots) {
  if (!win || n_shots <= 0) return kCounterBytes;
  gdg_job job{win, n_shots, nullptr, win->info.m, nullptr, nullptr, nullptr};
  LaunchGeom G;
  if (launch_geometry(&job, 1, win->waves, 0, false, G)) return 0;
  return kCounterBytes + (size_t)G.grid * (size_t)G.ck_per_wg();
}

}  // extern "C"

namespace {

int decode_batch_impl(const gdg_window* win, int32_t n_shots, const uint8_t* d_syndrome,
                      int64_t syn_stride, uint8_t* d_ehat, double* d_pm, int32_t* d_flags,
                      void* d_workspace, size_t workspace_bytes, const gdg_trace* trace,
                      void* hip_stream, const WarmIO* warm) {
  gdg_trace_dev tr{};
  if (trace) {
    tr.sel = trace->sel;
    tr.dec = trace->dec;
    tr.log_cap = trace->log_cap;
    tr.ends = trace->ends;
    tr.first_post = trace->first_post;
    tr.edge_iters = (long long*)trace->edge_iters;
    tr.step_lsum = trace->step_lsum;
    tr.pre_post = trace->pre_post;
    if (tr.dec && tr.log_cap <= 0) return fail(GDG_EINVAL, "trace log_cap must be positive");
  }
  gdg_job job{win, n_shots, d_syndrome, syn_stride, d_ehat, d_pm, d_flags};
  // A batch of at most one shot per CU is latency-bound: each shot's workgroup
  // gets eight wavefronts (its sixteen paths in two rounds instead of four)
  // when the eight-wavefront plan fits; the answers do not depend on it.
  const int waves = (n_shots <= cu_count() && win->plans[7].total <= max_lds_per_block())
                        ? 8
                        : win->waves;
  if (!d_workspace)
    return launch_jobs(&job, 1, waves, 0, tr, (hipStream_t)hip_stream, nullptr, warm);
  LaunchGeom G;
  int rc = launch_geometry(&job, 1, waves, 0, false, G);
  if (rc) return rc;
  return launch_with_scratch(&job, 1, waves, G, tr, (hipStream_t)hip_stream, nullptr,
                             d_workspace, workspace_bytes, warm);
}

}  // namespace

extern "C" {

int gdg_decode_batch(const gdg_window* win, int32_t n_shots, const uint8_t* d_syndrome,
                     int64_t syn_stride, uint8_t* d_ehat, double* d_pm, int32_t* d_flags,
                     void* d_workspace, size_t workspace_bytes, const gdg_trace* trace,
                     void* hip_stream) {
  if (!win) return fail(GDG_EINVAL, "null window");
  if (n_shots < 0) return fail(GDG_EINVAL, "negative n_shots");
  if (n_shots == 0) return GDG_OK;
  return decode_batch_impl(win, n_shots, d_syndrome, syn_stride, d_ehat, d_pm, d_flags,
                           d_workspace, workspace_bytes, trace, hip_stream, nullptr);
}

int gdg_decode_batch_warm(const gdg_window* win, int32_t n_shots, const uint8_t* d_syndrome,
                          int64_t syn_stride, const float* d_warm_in, int64_t warm_in_stride,
                          float* d_warm_out, int64_t warm_out_stride, uint8_t* d_ehat,
                          double* d_pm, int32_t* d_flags, void* d_workspace,
                          size_t workspace_bytes, const gdg_trace* trace, void* hip_stream) {
  if (!win) return fail(GDG_EINVAL, "null window");
  if (n_shots < 0) return fail(GDG_EINVAL, "negative n_shots");
  if (n_shots == 0) return GDG_OK;
  if ((d_warm_in || d_warm_out) && win->dev.pre_iters <= 0)
    return fail(GDG_EINVAL, "the window has no preprocessing BP to warm-start");
  if (d_warm_in && !win->dev.warm_map)
    return fail(GDG_EINVAL, "warm input for a window that gdg_link_windows has not linked");
  if (d_warm_in && warm_in_stride < win->dev.warm_prev_slots)
    return fail(GDG_EINVAL, "warm_in_stride below the previous window's message slots");
  if (d_warm_out && warm_out_stride < win->dev.fr_epad)
    return fail(GDG_EINVAL, "warm_out_stride below the window's message slots");
  WarmIO w;
  w.in = d_warm_in;
  w.out = d_warm_out;
  w.in_stride = warm_in_stride;
  w.out_stride = warm_out_stride;
  return decode_batch_impl(win, n_shots, d_syndrome, syn_stride, d_ehat, d_pm, d_flags,
                           d_workspace, workspace_bytes, trace, hip_stream, &w);
}

int gdg_decode_chain(const gdg_window* first, const gdg_window* middle, const gdg_window* last,
                     int32_t n_windows, int32_t n_items, const int32_t* d_k_begin,
                     const int32_t* d_k_end, uint8_t* d_det, const int64_t* d_det_off,
                     uint8_t* d_obs, const int64_t* d_obs_off, uint8_t* d_ehat,
                     int64_t ehat_stride, double* d_pm, int32_t* d_flags, void* hip_stream) {
  if (!first) return fail(GDG_EINVAL, "null first window");
  if (n_windows < 1 || n_items < 0) return fail(GDG_EINVAL, "bad sizes");
  if (n_items == 0) return GDG_OK;
  if (n_windows > 2 && !middle) return fail(GDG_EINVAL, "a middle window is needed");
  if (n_windows >= 2 && !last) return fail(GDG_EINVAL, "a last window is needed");
  if (n_windows == 1) last = first;
  if (!middle) middle = first;
  if (first->info.k != 0 || last->info.k != n_windows - 1 || !last->info.last ||
      (n_windows > 2 && middle->info.k != 1))
    return fail(GDG_EINVAL, "windows must be k = 0, k = 1 and the last, k = n_windows - 1");
  if (!d_k_begin || !d_k_end || !d_det || !d_det_off || !d_obs || !d_obs_off || !d_ehat ||
      !d_pm || !d_flags)
    return fail(GDG_EINVAL, "null buffer");
  const gdg_window* ws[3] = {first, middle, last};
  int n_max = 0;
  for (const gdg_window* w : ws) {
    n_max = std::max(n_max, w->info.n);
    if (w->waves != first->waves) return fail(GDG_EINVAL, "windows of different launch shapes");
  }
  if (ehat_stride < n_max) return fail(GDG_EINVAL, "ehat_stride below the largest window");
  const int row_step = n_windows >= 2 ? last->info.row0 / (n_windows - 1) : 0;
  if (n_windows > 2 && middle->info.row0 != row_step)
    return fail(GDG_EINVAL, "windows do not advance by equal steps");
  gdg_chain_dev C{};
  for (int i = 0; i < 3; ++i) {
    C.w[i] = ws[i]->d_dev;
    C.L[i] = ws[i]->d_plans + (first->waves - 1);
    C.cm[i] = ws[i]->cm;
    C.row0[i] = ws[i]->info.row0;
  }
  C.K = n_windows;
  C.row_step = row_step;
  C.ehat_stride = ehat_stride;
  C.det = d_det;
  C.obs = d_obs;
  C.det_off = (const long long*)d_det_off;
  C.obs_off = (const long long*)d_obs_off;
  C.k_begin = d_k_begin;
  C.k_end = d_k_end;
  C.ehat = d_ehat;
  C.pm = d_pm;
  C.flags = d_flags;
  // one job per shape for the launch geometry (LDS, register tiling,
  // checkpoints); the first carries the item count, the buffers are unused
  gdg_job jobs[3];
  for (int i = 0; i < 3; ++i)
    jobs[i] = gdg_job{ws[i], i == 0 ? n_items : 0, d_det, first->info.m, d_ehat, d_pm, d_flags};
  gdg_trace_dev tr{};
  return launch_jobs(jobs, 3, first->waves, 0, tr, (hipStream_t)hip_stream, nullptr, nullptr, &C);
}

int gdg_decode_batch_noalloc(const gdg_window* win, int32_t n_shots, const uint8_t* d_syndrome,
                             int64_t syn_stride, uint8_t* d_ehat, double* d_pm, int32_t* d_flags,
                             void* hip_stream) {
  if (!win) return fail(GDG_EINVAL, "null window");
  if (n_shots < 0) return fail(GDG_EINVAL, "negative n_shots");
  if (n_shots == 0) return GDG_OK;
  gdg_job job{win, n_shots, d_syndrome, syn_stride, d_ehat, d_pm, d_flags};
  LaunchGeom G;
  int rc = launch_geometry(&job, 1, win->waves, 0, false, G);
  if (rc) return rc;
  void* scratch = nullptr;
  size_t bytes = 0;
  hipError_t e = gdg_static_scratch(&scratch, &bytes);
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress (static scratch)");
  if (G.slots > 0 && (size_t)G.ck_per_wg() > bytes - kCounterBytes)
    return fail(GDG_ESHAPE, "the window's path checkpoints for one workgroup exceed the fixed "
                            "scratch of gdg_decode_batch_noalloc");
  gdg_trace_dev tr{};
  return launch_with_scratch(&job, 1, win->waves, G, tr, (hipStream_t)hip_stream, nullptr,
                             scratch, bytes);
}

int gdg_release_scratch(void* hip_stream) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  const hipStream_t st = (hipStream_t)hip_stream;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  for (size_t i = 0; i < g_scratch.size(); ++i) {
    StreamScratch& x = g_scratch[i];
    if (x.dev != dev || x.st != st) continue;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (x.base) (void)hipFree(x.base);
    g_scratch.erase(g_scratch.begin() + (long)i);
    return GDG_OK;
  }
  return GDG_OK;
}

// Persistent grid of the learned decode: three workgroups per CU on 256 CUs.
constexpr int kLearnGrid = 768;

size_t gdg_learned_work_bytes(const gdg_window* win) {
  if (!win) return 0;
  return (size_t)kLearnGrid * win->waves * 16 * win->info.n_act * sizeof(float);
}

int gdg_decode_learned(const gdg_window* win, const gdg_model* model, const gdg_learn_cfg* cfg,
                       int32_t n_shots, const uint8_t* d_syndrome, int64_t syn_stride,
                       uint8_t* d_ehat, double* d_pm, int32_t* d_flags, void* d_work,
                       size_t work_bytes, void* hip_stream) {
  if (!win || !cfg) return fail(GDG_EINVAL, "null argument");
  if (cfg->mode != 1 && cfg->mode != 2) return fail(GDG_EINVAL, "mode must be 1 or 2");
  if (cfg->mode == 1 && !model) return fail(GDG_EINVAL, "learned mode needs a model");
  if (cfg->n_cand < 1 || cfg->n_cand > 16) return fail(GDG_EINVAL, "n_cand must be in 1..16");
  if (cfg->mode == 1 && (cfg->guesses < 0 || (1 << cfg->guesses) > win->info.n_paths))
    return fail(GDG_EINVAL, "2^guesses must not exceed the window's path count");
  if (cfg->mode == 2 && (cfg->rec_steps < 1 || !cfg->d_rec_x || !cfg->d_rec_col || !cfg->d_rec_fav))
    return fail(GDG_EINVAL, "record mode needs rec_steps >= 1 and its buffers");
  if (n_shots < 0) return fail(GDG_EINVAL, "negative n_shots");
  if (n_shots == 0) return GDG_OK;
  if (!d_work || work_bytes < gdg_learned_work_bytes(win)) return fail(GDG_EINVAL, "workspace too small");
  gdg_learn_dev ld{};
  ld.mode = cfg->mode;
  ld.n_cand = cfg->n_cand;
  ld.guesses = cfg->mode == 1 ? cfg->guesses : 0;
  ld.tau = cfg->tau;
  ld.pm_fallback = cfg->pm_fallback;
  ld.tree = cfg->tree ? 1 : 0;
  if (model) ld.model = model->dev;
  ld.ring = (float*)d_work;
  ld.ring_stride = win->info.n_act;
  ld.rec_steps = cfg->rec_steps;
  ld.rec_x = cfg->d_rec_x;
  ld.rec_col = cfg->d_rec_col;
  ld.rec_fav = cfg->d_rec_fav;
  gdg_job job{win, n_shots, d_syndrome, syn_stride, d_ehat, d_pm, d_flags};
  gdg_trace_dev tr{};
  tr.edge_iters = (long long*)cfg->d_edge_iters;
  return launch_jobs(&job, 1, win->waves, std::min(n_shots, kLearnGrid), tr,
                     (hipStream_t)hip_stream, &ld);
}

int gdg_decode_jobs(const gdg_job* jobs, int32_t n_jobs, const gdg_launch_cfg* cfg,
                    void* hip_stream) {
  int waves = 4, workgroups = 0;
  if (cfg) {
    if (cfg->waves) waves = cfg->waves;
    workgroups = cfg->workgroups;
  }
  gdg_trace_dev tr{};
  return launch_jobs(jobs, n_jobs, waves, workgroups, tr, (hipStream_t)hip_stream);
}

int gdg_jobs_lds_bytes(const gdg_job* jobs, int32_t n_jobs, int32_t waves) {
  if (!jobs || n_jobs < 1 || n_jobs > GDG_MAX_JOBS || waves < 1 || waves > 8) return GDG_EINVAL;
  int lds = 0;
  for (int j = 0; j < n_jobs; ++j) {
    if (!jobs[j].win) return GDG_EINVAL;
    lds = std::max(lds, jobs[j].win->plans[waves - 1].total);
  }
  return lds;
}

int gdg_commit(const gdg_window* win, int32_t n_shots, const uint8_t* d_ehat,
               uint8_t* d_detectors, int64_t det_stride, uint8_t* d_obs, int64_t obs_stride,
               void* hip_stream) {
  if (!win) return fail(GDG_EINVAL, "null window");
  if (n_shots < 0) return fail(GDG_EINVAL, "negative n_shots");
  if (n_shots == 0) return GDG_OK;
  if (!d_ehat || !d_detectors || (!d_obs && win->cm.n_obs > 0))
    return fail(GDG_EINVAL, "null buffer");
  hipError_t e = gdg_launch_commit(win->cm, n_shots, d_ehat, d_detectors, det_stride, d_obs,
                                   obs_stride, nullptr, nullptr, 0, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "commit launch");
  return GDG_OK;
}

int gdg_commit_indexed(const gdg_window* win, int32_t n_shots, const uint8_t* d_ehat,
                       uint8_t* d_detectors, const int64_t* d_det_off, uint8_t* d_obs,
                       const int64_t* d_obs_off, void* hip_stream) {
  if (!win) return fail(GDG_EINVAL, "null window");
  if (n_shots < 0) return fail(GDG_EINVAL, "negative n_shots");
  if (n_shots == 0) return GDG_OK;
  if (!d_ehat || !d_detectors || !d_det_off || (win->cm.n_obs > 0 && (!d_obs || !d_obs_off)))
    return fail(GDG_EINVAL, "null buffer");
  static_assert(sizeof(int64_t) == sizeof(long long), "offset type");
  hipError_t e = gdg_launch_commit(win->cm, n_shots, d_ehat, d_detectors, 0, d_obs, 0,
                                   (const long long*)d_det_off, (const long long*)d_obs_off,
                                   win->info.row0, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "commit launch");
  return GDG_OK;
}

int gdg_copy_rows(int32_t n, int32_t m, const uint8_t* d_src, const int64_t* d_src_off,
                  uint8_t* d_dst, const int64_t* d_dst_off, void* hip_stream) {
  if (n < 0 || m < 0) return fail(GDG_EINVAL, "negative size");
  if (n == 0 || m == 0) return GDG_OK;
  if (!d_src || !d_src_off || !d_dst) return fail(GDG_EINVAL, "null buffer");
  hipError_t e = gdg_launch_copy_rows(n, m, d_src, (const long long*)d_src_off, d_dst,
                                      (const long long*)d_dst_off, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "copy launch");
  return GDG_OK;
}

int gdg_bp(const gdg_window* win, int32_t n_shots, const uint8_t* d_syndrome, int64_t syn_stride,
           int32_t n_iters, float* d_post, int32_t* d_first_ok, void* hip_stream) {
  if (!win) return fail(GDG_EINVAL, "null window");
  if (n_shots < 0 || n_iters < 1) return fail(GDG_EINVAL, "bad sizes");
  if (n_shots == 0) return GDG_OK;
  if (!d_syndrome || !d_post || !d_first_ok) return fail(GDG_EINVAL, "null buffer");
  if (syn_stride < win->info.m) return fail(GDG_EINVAL, "syn_stride < m");
  const size_t lds = (size_t)align16(win->dev.m) + (size_t)align16(4 * (win->dev.n + 1)) +
                     4 * (size_t)(win->dev.fr_epad + 8);
  if (lds > (size_t)max_lds_per_block()) return fail(GDG_ESHAPE, "window does not fit in LDS");
  // four wavefronts, each keeping the syndrome bits of up to 64 slot columns
  if ((win->dev.fr_T + 3) / 4 > 64) return fail(GDG_ESHAPE, "window graph too large for gdg_bp");
  hipError_t e = gdg_launch_bp(win->dev, n_shots, d_syndrome, syn_stride, n_iters, d_post,
                               d_first_ok, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "bp launch");
  return GDG_OK;
}

int gdg_decode_osd(const gdg_window* win, int32_t n_shots, const uint8_t* d_syndrome,
                   int64_t syn_stride, int32_t bp_iters, int32_t cs, int32_t lambda,
                   int32_t n_keep, uint8_t* d_ehat, double* d_pm, int32_t* d_flags,
                   int32_t* d_order, int32_t* d_bp_iters, void* hip_stream) {
  if (!win) return fail(GDG_EINVAL, "null window");
  if (n_shots < 0 || bp_iters < 1 || lambda < 0) return fail(GDG_EINVAL, "bad sizes");
  if (n_shots == 0) return GDG_OK;
  if (!d_syndrome || !d_ehat || !d_pm || !d_flags) return fail(GDG_EINVAL, "null buffer");
  if (syn_stride < win->info.m) return fail(GDG_EINVAL, "syn_stride < m");
  const gdg_win_dev& w = win->dev;
  if (w.m > 512) return fail(GDG_ESHAPE, "BP+OSD supports windows of up to 512 rows");
  if ((w.fr_T + 3) / 4 > 64) return fail(GDG_ESHAPE, "window graph too large for the window BP");
  gdg_osd_lds L{};
  L.nk = n_keep > 0 ? std::min<int>(n_keep, w.n) : w.n;
  L.mw = (w.m + 31) / 32;
  L.sort_p = 1;
  while (L.sort_p < w.n) L.sort_p <<= 1;
  if (L.sort_p > 4096) return fail(GDG_ESHAPE, "BP+OSD supports windows of up to 4096 columns");
  L.obits_words = (w.n + 31) / 32 + 1;
  int off = 0;
  auto take = [&](int bytes) {
    const int o = off;
    off = align16(off + bytes);
    return o;
  };
  L.syn = take(w.m);
  L.order = take(2 * w.n);
  L.rank_of = take(2 * w.n);
  L.obits = take(4 * L.obits_words);
  L.sv = take(4 * L.mw);
  L.pcol = take(2 * w.m);
  L.llrp = 0;
  L.isp = take(L.nk);
  L.freec = take(2 * L.nk);
  L.misc = take(8 * 4);
  L.A = off;
  L.post = L.A;
  L.c2v = L.A + align16(4 * (w.n + 1));
  L.keys = L.A;
  L.mat = L.A;
  const int a_bytes = std::max(std::max(L.c2v - L.A + 4 * (w.fr_epad + 8), 8 * L.sort_p),
                               4 * L.mw * L.nk);
  L.total = L.A + align16(a_bytes);
  if (L.total > max_lds_per_block())
    return fail(GDG_ESHAPE, "BP+OSD on this window does not fit in LDS (keep fewer columns)");
  hipError_t e = gdg_launch_osd(w, L, n_shots, d_syndrome, syn_stride, bp_iters, cs ? 1 : 0,
                                lambda, d_ehat, d_pm, d_flags, d_order, d_bp_iters,
                                (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "osd launch");
  return GDG_OK;
}

int gdg_dem_upload(const gdg_dem* dem, gdg_dem_dev** out) {
  if (!out) return fail(GDG_EINVAL, "null argument");
  *out = nullptr;
  int rc = validate_dem(dem);
  if (rc) return rc;
  std::unique_ptr<gdg_dem_dev> d(new gdg_dem_dev());
  const int nc = dem->n_cols;
  std::vector<int> hp(dem->h_ptr, dem->h_ptr + nc + 1), hi(dem->h_idx, dem->h_idx + dem->h_ptr[nc]);
  std::vector<int> lp(dem->l_ptr, dem->l_ptr + nc + 1), li(dem->l_idx, dem->l_idx + dem->l_ptr[nc]);
  std::vector<uint32_t> thr(nc);
  for (int c = 0; c < nc; ++c) {
    double t = std::floor(dem->priors[c] * 4294967296.0);
    thr[c] = t >= 4294967295.0 ? 4294967295u : (uint32_t)t;
  }
  auto put = [&](auto& v, auto** p) {
    using T = typename std::remove_reference<decltype(v)>::type::value_type;
    T* dp = nullptr;
    int r = upload(v, &dp);
    if (dp) d->allocs.push_back(dp);
    *p = dp;
    return r;
  };
  d->k.n_rows = dem->n_rows;
  d->k.n_cols = nc;
  d->k.n_obs = dem->n_obs;
  if ((rc = put(hp, &d->k.h_ptr))) return rc;
  if ((rc = put(hi, &d->k.h_idx))) return rc;
  if ((rc = put(lp, &d->k.l_ptr))) return rc;
  if ((rc = put(li, &d->k.l_idx))) return rc;
  if ((rc = put(thr, &d->k.thr))) return rc;
  *out = d.release();
  return GDG_OK;
}

void gdg_dem_free(gdg_dem_dev* d) { delete d; }

int gdg_sample(const gdg_dem_dev* d, int32_t n_shots, uint64_t seed, uint32_t stream,
               uint64_t shot0, uint8_t* d_detectors, uint8_t* d_obs, void* hip_stream) {
  if (!d) return fail(GDG_EINVAL, "null dem");
  if (n_shots < 0) return fail(GDG_EINVAL, "negative n_shots");
  if (n_shots == 0) return GDG_OK;
  if (!d_detectors || (!d_obs && d->k.n_obs > 0)) return fail(GDG_EINVAL, "null buffer");
  hipError_t e = gdg_launch_sample(d->k, n_shots, seed, stream, shot0, d_detectors, d_obs,
                                   (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "sample launch");
  return GDG_OK;
}

int gdg_sample_errors(const gdg_dem_dev* d, int32_t n_shots, uint64_t seed, uint32_t stream,
                      uint64_t shot0, uint8_t* d_err, void* hip_stream) {
  if (!d) return fail(GDG_EINVAL, "null dem");
  if (n_shots < 0) return fail(GDG_EINVAL, "negative n_shots");
  if (n_shots == 0) return GDG_OK;
  if (!d_err) return fail(GDG_EINVAL, "null buffer");
  hipError_t e = gdg_launch_sample_errors(d->k, n_shots, seed, stream, shot0, d_err,
                                          (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "sample launch");
  return GDG_OK;
}

int gdg_evaluate(int32_t n_shots, int32_t n_rows, int32_t n_obs, const uint8_t* d_detectors,
                 const uint8_t* d_obs, uint8_t* d_fail, void* hip_stream) {
  if (n_shots < 0 || n_rows < 0 || n_obs < 0) return fail(GDG_EINVAL, "bad sizes");
  if (n_shots == 0) return GDG_OK;
  if (!d_detectors || !d_fail || (!d_obs && n_obs > 0)) return fail(GDG_EINVAL, "null buffer");
  hipError_t e = gdg_launch_evaluate(n_shots, n_rows, n_obs, d_detectors, d_obs, d_fail,
                                     (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "evaluate launch");
  return GDG_OK;
}

// ------------------------------------------------------------------ learned proposer network

int gdg_mlp_forward(int32_t n, const float* d_params, const float* d_x, float* d_z,
                    void* hip_stream) {
  if (n < 0) return fail(GDG_EINVAL, "negative n");
  if (n == 0) return GDG_OK;
  if (!d_params || !d_x || !d_z) return fail(GDG_EINVAL, "null buffer");
  hipError_t e = gdg_launch_mlp_forward(n, d_params, d_x, d_z, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "mlp forward launch");
  return GDG_OK;
}

size_t gdg_mlp_grad_work_bytes(int32_t n) {
  return n > 0 ? sizeof(float) * gdg_mlp_grad_work_floats(n) : 0;
}

int gdg_mlp_grad(int32_t n, const float* d_params, const float* d_x, const float* d_y,
                 float* d_grad, float* d_loss, void* d_work, size_t work_bytes,
                 void* hip_stream) {
  if (n <= 0) return fail(GDG_EINVAL, "n must be positive");
  if (!d_params || !d_x || !d_y || !d_grad || !d_work) return fail(GDG_EINVAL, "null buffer");
  if (work_bytes < gdg_mlp_grad_work_bytes(n)) return fail(GDG_EINVAL, "workspace too small");
  hipError_t e = gdg_launch_mlp_grad(n, d_params, d_x, d_y, d_grad, d_loss, (float*)d_work,
                                     (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "mlp grad launch");
  return GDG_OK;
}

int gdg_mlp_adam(int32_t step, float lr, float beta1, float beta2, float eps, float* d_params,
                 const float* d_grad, float* d_m, float* d_v, void* hip_stream) {
  if (step < 1) return fail(GDG_EINVAL, "step must be >= 1");
  if (!d_params || !d_grad || !d_m || !d_v) return fail(GDG_EINVAL, "null buffer");
  hipError_t e = gdg_launch_mlp_adam(step, lr, beta1, beta2, eps, d_params, d_grad, d_m, d_v,
                                     (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "adam launch");
  return GDG_OK;
}

}  // extern "C"


namespace {
uint16_t bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
}  // namespace

extern "C" {

int gdg_model_create(const float* h_params, gdg_model** out) {
  if (!h_params || !out) return fail(GDG_EINVAL, "null argument");
  *out = nullptr;
  const int In = GDG_MLP_IN, H = GDG_MLP_H;
  const float* W1 = h_params;
  const float* b1 = W1 + In * H;
  const float* W2 = b1 + H;
  const float* b2 = W2 + H * H;
  const float* w3 = b2 + H;
  const float b3 = w3[H];
  // A operands: tile mt, K step s, lane l -> W^T[16 mt + l % 16][16 s + 4 (l / 16) + j]
  auto pack = [&](const float* W, int n_in, int steps, std::vector<uint32_t>& dst) {
    dst.assign((size_t)4 * steps * 64 * 2, 0u);
    for (int mt = 0; mt < 4; ++mt)
      for (int s = 0; s < steps; ++s)
        for (int l = 0; l < 64; ++l) {
          uint16_t h[4];
          for (int j = 0; j < 4; ++j) {
            const int out_u = 16 * mt + l % 16, in_u = 16 * s + 4 * (l / 16) + j;
            h[j] = in_u < n_in ? bf16_rne(W[in_u * H + out_u]) : 0;
          }
          const size_t at = (((size_t)mt * steps + s) * 64 + l) * 2;
          dst[at] = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
          dst[at + 1] = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
        }
  };
  std::vector<uint32_t> a1, a2;
  pack(W1, In, 2, a1);
  pack(W2, H, 4, a2);
  std::unique_ptr<gdg_model> m(new gdg_model());
  int rc;
  uint32_t* d = nullptr;
  if ((rc = upload(a1, &d))) return rc;
  m->allocs.push_back(d);
  m->dev.a1 = (const uint2*)d;
  if ((rc = upload(a2, &d))) return rc;
  m->allocs.push_back(d);
  m->dev.a2 = (const uint2*)d;
  float* f = nullptr;
  std::vector<float> v(b1, b1 + H);
  if ((rc = upload(v, &f))) return rc;
  m->allocs.push_back(f);
  m->dev.b1 = f;
  v.assign(b2, b2 + H);
  if ((rc = upload(v, &f))) return rc;
  m->allocs.push_back(f);
  m->dev.b2 = f;
  v.assign(w3, w3 + H);
  if ((rc = upload(v, &f))) return rc;
  m->allocs.push_back(f);
  m->dev.w3 = f;
  m->dev.b3 = b3;
  *out = m.release();
  return GDG_OK;
}

void gdg_model_free(gdg_model* m) { delete m; }

int gdg_mlp_infer(const gdg_model* m, int32_t n, const float* d_x, float* d_z, void* hip_stream) {
  if (!m) return fail(GDG_EINVAL, "null model");
  if (n < 0) return fail(GDG_EINVAL, "negative n");
  if (n == 0) return GDG_OK;
  if (!d_x || !d_z) return fail(GDG_EINVAL, "null buffer");
  hipError_t e = gdg_launch_mlp_infer(m->dev, n, d_x, d_z, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "mlp infer launch");
  return GDG_OK;
}

}  // extern "C"
