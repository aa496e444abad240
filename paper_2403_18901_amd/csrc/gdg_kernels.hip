// HIP kernels (gfx950 / CDNA4) of the sliding-window GDG decoder
// (arXiv 2403.18901): min-sum belief propagation with guided decimation,
// peeling and guessing, for many shots at once.
//
// Mapping. One workgroup decodes one shot's window. All of its wavefronts
// first run the preprocessing BP on the whole window together, rank and
// truncate the columns (Sec. III, Sec. IV-C) and build the shot's truncated
// Tanner graph in LDS. Each wavefront then runs whole decision paths of Fig. 2,
// one at a time, taking the next path id from an LDS counter, so the long main
// path starts first. A path's BP messages live in LDS and registers:
//   * check node (CN) rows are spread over lane groups, one batch of four
//     edges per lane; a CN phase gathers posteriors from LDS, forms each
//     extrinsic VN-to-CN message (Eq. 3) from the posterior and the CN's
//     previous outgoing message, clips it, combines the group's two-min
//     records and sign parities with cross-lane exchanges (Eq. 1) and writes
//     the new CN-to-VN messages next to the old ones, in CSR order;
//   * the VN phase sums each owned VN's messages through a column-order index
//     (Eq. 2);
//   * the syndrome check of the previous iteration's hard decisions (Eq. 4) is
//     folded into the CN phase;
//   * Alg. 1 is a wavefront min-reduction of 64-bit keys (order-preserving
//     float bits << 32 | VN index), Alg. 3 and peeling are lane-parallel passes
//     with wavefront ballots.
// Decimated VNs hold +infinity in the posterior array, which is how CNs skip
// their stale messages (Sec. II-A). No matrix cores: the work is sparse
// gathers.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "gdg_kernels.h"

namespace {

constexpr int kWave = 64;
constexpr float kInfF = __builtin_huge_valf();

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

__device__ __forceinline__ uint32_t ord_f32(float x) {
  if (x == 0.0f) x = 0.0f;   // -0 and +0 compare equal
  uint32_t b = __float_as_uint(x);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Cross-lane exchange inside aligned lane groups (DPP): partner at lane ^ 1,
// lane ^ 2, then the mirrored lane within 8 and within 16. After the steps
// below the group size, every lane holds the group's combined value. The
// steps run under the lane mask of the groups that need them; a partner is
// always in the same group, hence active.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xf, 0xf, true);
}
constexpr int kDppXor1 = 0xB1;       // quad_perm(1, 0, 3, 2)
constexpr int kDppXor2 = 0x4E;       // quad_perm(2, 3, 0, 1)
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long x) {
  const uint32_t lo = dpp<CTRL>((uint32_t)x), hi = dpp<CTRL>((uint32_t)(x >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long readlane64(unsigned long long x, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}

// Wavefront reductions without LDS round trips: four DPP steps leave every
// lane of a row of 16 with the row's result, then the four rows' results are
// read into scalar registers. All 64 lanes must be active.
__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
  unsigned long long u;
  u = dpp64<kDppXor1>(v);
  v = u < v ? u : v;
  u = dpp64<kDppXor2>(v);
  v = u < v ? u : v;
  u = dpp64<kDppHalfMirror>(v);
  v = u < v ? u : v;
  u = dpp64<kDppMirror>(v);
  v = u < v ? u : v;
  unsigned long long r = readlane64(v, 0);
  u = readlane64(v, 16);
  r = u < r ? u : r;
  u = readlane64(v, 32);
  r = u < r ? u : r;
  u = readlane64(v, 48);
  r = u < r ? u : r;
  return r;
}

__device__ __forceinline__ int wave_sum_i32(int v) {
  v += (int)dpp<kDppXor1>((uint32_t)v);
  v += (int)dpp<kDppXor2>((uint32_t)v);
  v += (int)dpp<kDppHalfMirror>((uint32_t)v);
  v += (int)dpp<kDppMirror>((uint32_t)v);
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
         __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}

// Sum over the wavefront (any order; every lane gets it).
__device__ __forceinline__ float wave_sum_f32(float v) {
  v += __uint_as_float(dpp<kDppXor1>(__float_as_uint(v)));
  v += __uint_as_float(dpp<kDppXor2>(__float_as_uint(v)));
  v += __uint_as_float(dpp<kDppHalfMirror>(__float_as_uint(v)));
  v += __uint_as_float(dpp<kDppMirror>(__float_as_uint(v)));
  const float a = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 0));
  const float b = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16));
  const float c = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
  const float d = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 48));
  return (a + b) + (c + d);
}

__device__ __forceinline__ long long wave_sum_i64(long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ int wave_incl_scan(int x, int lane) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  return x;
}


// Exclusive prefix sum in place over a[0..len) (int32 in LDS) by wavefront 0;
// a[len] receives the total. Caller synchronises the workgroup around it.
__device__ void wg_exclusive_scan_wave0(int* a, int len) {
  int lane = threadIdx.x & (kWave - 1);
  if ((threadIdx.x >> 6) != 0) return;
  int carry = 0;
  for (int base = 0; base < len; base += kWave) {
    int i = base + lane;
    int x = i < len ? a[i] : 0;
    int inc = wave_incl_scan(x, lane);
    if (i < len) a[i] = carry + inc - x;
    carry += __shfl(inc, kWave - 1, kWave);
  }
  if (lane == 0) a[len] = carry;
}

// Ascending bitonic sort (Batcher) of P 64-bit keys in LDS by the whole
// workgroup, P a power of two; each stage compares and exchanges P / 2
// disjoint pairs, then synchronises.
__device__ void wg_bitonic_sort(unsigned long long* a, int P) {
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P / 2; i += blockDim.x) {
        const int lo = ((i & ~(j - 1)) << 1) | (i & (j - 1));   // bit j of lo clear
        const unsigned long long x = a[lo], y = a[lo + j];
        if ((x > y) == ((lo & k) == 0)) {
          a[lo] = y;
          a[lo + j] = x;
        }
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ float clip_to(float x, float c) { return __builtin_amdgcn_fmed3f(x, -c, c); }

// ------------------------------------------------------------------ decode kernel

__device__ __forceinline__ int path_value(const gdg_win_dev& w, int pid, int split, int D, int f) {
  if (pid == 0) return f;
  if (w.g > 0 && pid < (1 << w.g)) {
    if (D > w.g) return f;
    return ((pid >> (w.g - D)) & 1) ? 1 - f : f;
  }
  return D == split ? 1 - f : f;
}

__device__ __forceinline__ bool path_on_main(const gdg_win_dev& w, int pid, int split, int D) {
  if (pid == 0) return true;
  if (w.g > 0 && pid < (1 << w.g)) {
    int taken = D - 1 < w.g ? D - 1 : w.g;
    if (taken <= 0) return true;
    return (pid >> (w.g - taken)) == 0;
  }
  return D <= split;
}

// Alg. 3 for one VN: history sum / min / max over the last four posteriors.
__device__ __forceinline__ int agg_dec(float hsum, float hmin, float hmax, int D, bool on_main,
                                       int n_unsat) {
  const float PA = on_main ? -3.0f : 0.0f;
  float PB = on_main ? -12.0f : -10.0f;
  if (D == 1) PB = -16.0f;
  if (hmax < PA && hsum < PB) return 1;
  if ((hmin > 30.0f && D <= 4) || (hmin > 3.0f && n_unsat >= 3)) return 0;
  return -1;
}

enum { END_CONVERGED = 1, END_EXHAUSTED = 2, END_CONTRADICTION = 3, END_NO_CANDIDATE = 4, END_BOUND = 5 };

// State of one decision path, held by one wavefront.
//
// Check nodes (CNs). The truncated graph's rows are stored in CSR order with
// each row padded to a multiple of four edges by a dummy VN (index n_act)
// whose posterior is +infinity and whose status is "decimated to 0": a padded
// edge then behaves exactly like an edge to a decimated VN (see set_status).
// A row of nb batches of four edges is spread over a group of k lanes, k the
// power of two >= nb, one batch per lane, inside one "slot column" of 64 lanes;
// rows sorted by decreasing degree are packed into consecutive slot columns,
// which keeps every group aligned to its size. A CN phase walks the T slot
// columns: each lane forms the VN-to-CN messages of its batch, the group
// combines its two-min records and parities with cross-lane (DPP) exchanges,
// and each lane writes the new CN-to-VN messages of its batch. Lanes of a
// group with fewer batches than lanes, and idle lanes, point at a dummy batch
// of four dummy edges: their messages clip to +clip and change nothing.
//
// Variable nodes (VNs). VN v = lane + 64 r belongs to this lane; its static
// data sit in registers. Its column slots are padded to a multiple of four;
// padded slots point at a CN-to-VN message fixed at zero.
constexpr int kPad = 4;


template <int VPL>
struct PathCtx {
  __device__ __forceinline__ int vc0(int r) const { return vinfo[r] & 0xffffu; }
  __device__ __forceinline__ int vdg(int r) const { return (vinfo[r] >> 16) & 0xffu; }
  __device__ __forceinline__ int st(int r) const { return (int)((vinfo[r] >> 24) & 3u) - 1; }
  __device__ __forceinline__ void set_st(int r, int value) {
    vinfo[r] = (vinfo[r] & 0x00ffffffu) | ((uint32_t)(value + 1) << 24);
  }
  // shared (per shot) sub-graph in LDS
  const uint16_t* rvn;    // [E_pad + 8] 4 * VN of each padded CSR edge (byte offset in post)
  const uint16_t* cidx;   // [E_col] 4 * CSR position of each column-order slot (byte offset in c2v)
  const uint16_t* crow;   // [E_col] row of each column-order slot
  const uint32_t* meta;   // [T][64] slot metadata
  const uint4* rec;       // or [T][64] records (metadata, edge offsets) in global memory
  // per wavefront, LDS
  float* post;            // [n_act + 1]; +infinity once decimated and for the dummy VN
  int8_t* status;         // [n_act + 1] -1 active, 0/1 decimated
  float* c2v;             // [E_pad + 8] CN-to-VN messages in CSR order; [E_pad, +4) zero,
                          // [E_pad + 4, +4) the dummy batch
  uint8_t* unsat;         // [m]
  uint32_t* prop;         // [ceil(n_act/4)] peeling proposals, one byte per VN
  int lane, m, n, T;
  int t0 = 0, tstride = 1;   // slot column i of this walk is table column t0 + i * tstride
  uint32_t sres;          // bit t: residual syndrome of the row in slot column t
  int act_edges;          // edges of this lane's active VNs
  // VN registers
  uint32_t vinfo[VPL];   // first column slot | degree << 16 | (status + 1) << 24
  float llr[VPL];
  float hs[VPL], hmn[VPL], hmx[VPL];           // history over the last four iterations
};

// Two-min record and parities of a set of VN-to-CN messages: n1 <= n2 the bit
// patterns of the two smallest magnitudes (non-negative floats order like
// their bits); bit 31 of sp / hp: parity of the message signs / of the hard
// decisions.
struct CnAcc {
  uint32_t n1, n2, sp, hp;
};

template <int CTRL>
__device__ __forceinline__ void cn_merge(CnAcc& a) {
  const uint32_t o1 = dpp<CTRL>(a.n1), o2 = dpp<CTRL>(a.n2);
  // second smallest of {a1 <= a2} u {o1 <= o2}: min(max(a1, o1), min(a2, o2))
  a.n2 = min(max(a.n1, o1), min(a.n2, o2));
  a.n1 = min(a.n1, o1);
  a.sp ^= dpp<CTRL>(a.sp);
  a.hp ^= dpp<CTRL>(a.hp);
}

// The steps nest: a step no lane of the wavefront needs ends the sequence.
__device__ __forceinline__ void cn_group(CnAcc& a, int lk) {
  if (lk > 0) {
    cn_merge<kDppXor1>(a);
    if (lk > 1) {
      cn_merge<kDppXor2>(a);
      if (lk > 2) {
        cn_merge<kDppHalfMirror>(a);
        if (lk > 3) cn_merge<kDppMirror>(a);
      }
    }
  }
}

__device__ __forceinline__ void hp_group(uint32_t& hp, int lk) {
  if (lk > 0) {
    hp ^= dpp<kDppXor1>(hp);
    if (lk > 1) {
      hp ^= dpp<kDppXor2>(hp);
      if (lk > 2) {
        hp ^= dpp<kDppHalfMirror>(hp);
        if (lk > 3) hp ^= dpp<kDppMirror>(hp);
      }
    }
  }
}

template <int CTRL>
__device__ __forceinline__ void cnt_merge(int& cnt, int& x, int& only) {
  cnt += (int)dpp<CTRL>((uint32_t)cnt);
  x ^= (int)dpp<CTRL>((uint32_t)x);
  only = max(only, (int)dpp<CTRL>((uint32_t)only));
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// bit 31 of a ^ b, other bits zero
__device__ __forceinline__ uint32_t xor_sign(uint32_t a, uint32_t b) {
  return __builtin_amdgcn_bitop3_b32(a, b, 0x80000000u, 0x28);
}

__device__ __forceinline__ const float& at_byte(const float* base, uint32_t off) {
  return *(const float*)((const char*)base + off);
}

// Walk over the slot columns, software-pipelined so that LDS latency overlaps
// work: while slot t is computed, slot t + 1's gathers (posteriors or
// statuses), slot t + 2's edges (and previous messages) and slot t + 3's
// metadata are in flight. Four rotating slots, unrolled by hand so that the
// rotation is a renaming; the slot table has three idle columns past its
// end (and past every wavefront's share of the whole-window table) for the
// loads issued ahead of the last slots. In the
// CN phase, reading a later slot's previous messages before slot t writes its
// own is safe: batches are disjoint except the dummy batch, whose messages
// only need to be finite. Returns the OR of the per-slot results.
struct Slot {
  uint32_t mt;   // metadata
  uint2 vo;      // VN byte offsets of the batch's edges
  float4 ov;     // previous CN-to-VN messages (CN phase)
  uint4 g;       // gathered posteriors or statuses
};

// REC: the slot table is a global array of (metadata, edge offsets) records
// (the whole-window layout of the preprocessing), one 16-byte load per slot
// instead of a metadata load and a dependent edge load.
template <int VPL, bool OV, bool REC>
__device__ __forceinline__ void slot_edges(const PathCtx<VPL>& P, Slot& s) {
  const int e0 = s.mt & kMetaEdge;
  if (!REC) s.vo = *(const uint2*)(P.rvn + e0);
  if (OV) s.ov = *(const float4*)(P.c2v + e0);
}

template <int VPL, bool REC>
__device__ __forceinline__ void slot_meta(const PathCtx<VPL>& P, Slot& s, int t) {
  const int i = (P.t0 + t * P.tstride) * kWave + P.lane;
  if (REC) {
    const uint4 r = P.rec[i];
    s.mt = r.x;
    s.vo = make_uint2(r.y, r.z);
  } else {
    s.mt = P.meta[i];
  }
}

template <int VPL, bool OV, bool REC, typename Gather, typename Compute>
__device__ __forceinline__ int slot_step(const PathCtx<VPL>& P, const Slot& a, Slot& b, Slot& c,
                                         Slot& d, int t, Gather& gather, Compute& compute) {
  gather(b);
  slot_edges<VPL, OV, REC>(P, c);
  slot_meta<VPL, REC>(P, d, t + 3);
  return compute(a, t);
}

template <int VPL, bool OV, bool REC = false, typename Gather, typename Compute>
__device__ __forceinline__ int slot_walk(const PathCtx<VPL>& P, Gather gather, Compute compute) {
  const int T = P.T;
  if (T == 0) return 0;
  int acc = 0;
  Slot A, B, C, D;
  slot_meta<VPL, REC>(P, A, 0);
  slot_meta<VPL, REC>(P, B, 1);
  slot_meta<VPL, REC>(P, C, 2);
  slot_edges<VPL, OV, REC>(P, A);
  slot_edges<VPL, OV, REC>(P, B);
  gather(A);
  for (int t = 0; t < T; t += 4) {
    acc |= slot_step<VPL, OV, REC>(P, A, B, C, D, t, gather, compute);
    if (t + 1 >= T) break;
    acc |= slot_step<VPL, OV, REC>(P, B, C, D, A, t + 1, gather, compute);
    if (t + 2 >= T) break;
    acc |= slot_step<VPL, OV, REC>(P, C, D, A, B, t + 2, gather, compute);
    if (t + 3 >= T) break;
    acc |= slot_step<VPL, OV, REC>(P, D, A, B, C, t + 3, gather, compute);
  }
  return acc;
}

// Recount every row's active degree and residual syndrome from the VN status,
// find dead CNs (no active VN, residual 1) and post peeling proposals of
// degree-one CNs (Sec. IV-D, Appendix C). Updates P.sres.
template <int VPL>
__device__ __forceinline__ void cn_recount(PathCtx<VPL>& P, bool& dead, bool& proposed) {
  bool dd = false, pp = false;
  uint32_t sres = 0u;
  slot_walk<VPL, false>(
      P,
      [&](Slot& s) {
        s.g.x = (uint32_t)(int)P.status[(s.vo.x & 0xffffu) >> 2];
        s.g.y = (uint32_t)(int)P.status[s.vo.x >> 18];
        s.g.z = (uint32_t)(int)P.status[(s.vo.y & 0xffffu) >> 2];
        s.g.w = (uint32_t)(int)P.status[s.vo.y >> 18];
      },
      [&](const Slot& s, int t) {
        const uint32_t mt = s.mt;
        const int lk = (mt >> kMetaLogKShift) & 7;
        const int v0 = (s.vo.x & 0xffffu) >> 2, v1 = s.vo.x >> 18;
        const int v2 = (s.vo.y & 0xffffu) >> 2, v3 = s.vo.y >> 18;
        const int s0 = (int)s.g.x, s1 = (int)s.g.y, s2 = (int)s.g.z, s3 = (int)s.g.w;
        int cnt = (s0 < 0) + (s1 < 0) + (s2 < 0) + (s3 < 0);
        int x = (s0 == 1) ^ (s1 == 1) ^ (s2 == 1) ^ (s3 == 1);
        int only = -1;
        only = s0 < 0 ? v0 : only;
        only = s1 < 0 ? v1 : only;
        only = s2 < 0 ? v2 : only;
        only = s3 < 0 ? v3 : only;
        if (lk > 0) {
          cnt_merge<kDppXor1>(cnt, x, only);
          if (lk > 1) {
            cnt_merge<kDppXor2>(cnt, x, only);
            if (lk > 2) {
              cnt_merge<kDppHalfMirror>(cnt, x, only);
              if (lk > 3) cnt_merge<kDppMirror>(cnt, x, only);
            }
          }
        }
        const int r = (x ^ ((mt & kMetaSyn) ? 1 : 0)) & 1;
        if (mt & kMetaValid) {
          sres |= (uint32_t)r << t;
          if (cnt == 0 && r) dd = true;
          if (cnt == 1 && (mt & kMetaLead)) {
            atomicOr(&P.prop[only >> 2], (1u << r) << ((only & 3) * 8));
            pp = true;
          }
        }
        return 0;
      });
  P.sres = sres;
  dead = dd;
  proposed = pp;
}

// Decimate owned VN v (register slot r). Its posterior becomes +infinity: every
// VN-to-CN message it would send then clips to +clip with a + sign and a 0 hard
// decision, so a CN's two-min, sign parity and syndrome check see exactly its
// active neighbours plus entries at +clip -- which reproduces the rule that a
// CN with a single active neighbour sends clip -- and its outgoing message to
// the decimated VN is never read.
template <int VPL>
__device__ __forceinline__ void set_status(PathCtx<VPL>& P, int r, int v, int value) {
  P.set_st(r, value);
  P.act_edges -= P.vdg(r);
  P.status[v] = (int8_t)value;
  P.post[v] = kInfF;
}

// set_status for a VN index v that is uniform over the wavefront (a
// decision): the stores address v directly, and only the owning lane's
// register r = v / 64 changes.
template <int VPL>
__device__ __forceinline__ void set_status_uniform(PathCtx<VPL>& P, int v, int value) {
  const bool own = P.lane == (v & (kWave - 1));
  if (own) {
    P.status[v] = (int8_t)value;
    P.post[v] = kInfF;
  }
  const int rv = v >> 6;
#pragma unroll
  for (int r = 0; r < VPL; ++r)
    if (own && r == rv) {
      P.set_st(r, value);
      P.act_edges -= P.vdg(r);
    }
}

// Whether a lower bound on the path's final Eq. 5 metric passes the stopping
// threshold *thr (+infinity until a path has converged): the priors of its
// VNs fixed to 1 (decimated or peeled; they stay 1 in its answer), plus, while
// the residual syndrome has an unsatisfied row, the least prior of its active
// VNs (an answer that meets a non-zero residual syndrome sets at least one of
// them; +infinity when none is left, and such a path cannot converge).
template <int VPL>
__device__ __forceinline__ bool over_bound(const PathCtx<VPL>& P, int* thr) {
  const float t = __int_as_float(
      __builtin_amdgcn_readfirstlane(__hip_atomic_load(thr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)));
  float lb = 0.0f, mn = kInfF;
#pragma unroll
  for (int r = 0; r < VPL; ++r) {
    lb += P.st(r) == 1 ? P.llr[r] : 0.0f;
    const bool act = P.lane + kWave * r < P.n && P.st(r) < 0;
    mn = act ? fminf(mn, P.llr[r]) : mn;
  }
  float lower = wave_sum_f32(lb);
  if (wave_any(P.sres != 0u))
    lower += __uint_as_float((uint32_t)wave_min_u64((unsigned long long)__float_as_uint(mn)));
  return t < kInfF && lower > t;
}

// Peeling closure in synchronous rounds. Returns false on a contradiction
// (a dead CN, or two different proposals for one VN; then the round is not
// applied). Leaves P.sres recounted.
template <int VPL>
__device__ __forceinline__ bool peel(PathCtx<VPL>& P) {
  for (;;) {
    bool dead, proposed;
    cn_recount(P, dead, proposed);
    const bool any_dead = wave_any(dead);
    const bool any_prop = wave_any(proposed);
    wave_sync();
    if (any_dead || !any_prop) {
      if (any_prop) {
        for (int i = P.lane; i < (P.n + 3) / 4; i += kWave) P.prop[i] = 0u;
        wave_sync();
      }
      return !any_dead;
    }
    uint32_t pr[VPL];
    bool conflict = false;
#pragma unroll
    for (int r = 0; r < VPL; ++r) {
      const int v = P.lane + kWave * r;
      pr[r] = v < P.n ? (P.prop[v >> 2] >> ((v & 3) * 8)) & 3u : 0u;
      if (pr[r] == 3u) conflict = true;
    }
    const bool any_conflict = wave_any(conflict);
    wave_sync();
    for (int i = P.lane; i < (P.n + 3) / 4; i += kWave) P.prop[i] = 0u;
    if (any_conflict) {
      wave_sync();
      return false;
    }
#pragma unroll
    for (int r = 0; r < VPL; ++r)
      if (pr[r]) set_status(P, r, P.lane + kWave * r, pr[r] == 2u ? 1 : 0);
    wave_sync();
  }
}

// One flooding CN phase: new CN-to-VN messages (Eq. 1) from the extrinsic
// VN-to-CN messages (Eq. 3, clipped), each formed from the posterior and the
// CN's previous message on that edge (kept in CSR order next to it). Returns
// this lane's OR of unsatisfied rows under the hard decisions (Eq. 4) of the
// posteriors it read: a posterior's sign bit is its hard decision (the VN
// phase stores an exact zero as -0, and Eq. 4 maps 0 to 1). Decimated VNs and
// padding hold +infinity (see set_status), so no edge needs a branch.
//
// An edge whose message magnitude equals the row's smallest one receives the
// second smallest: when two edges tie at the smallest, both minima are equal,
// so this is the usual "all but the minimising edge" rule. A message of zero
// magnitude may carry either sign; it adds zero to every posterior.
// cn_slot computes slot column t from its loaded edges, messages and gathered
// posteriors; cn_phase walks the slot columns (see slot_walk).
template <int VPL>
__device__ __forceinline__ int cn_slot(PathCtx<VPL>& P, const Slot& c, int t, float alpha,
                                       float clip) {
  constexpr uint32_t kSign = 0x80000000u;
  const uint32_t mt = c.mt;
  const int e0 = mt & kMetaEdge;
  const int lk = (mt >> kMetaLogKShift) & 7;
  const float x0 = clip_to(__uint_as_float(c.g.x) - c.ov.x, clip);
  const float x1 = clip_to(__uint_as_float(c.g.y) - c.ov.y, clip);
  const float x2 = clip_to(__uint_as_float(c.g.z) - c.ov.z, clip);
  const float x3 = clip_to(__uint_as_float(c.g.w) - c.ov.w, clip);
  const uint32_t b0 = __float_as_uint(x0), b1 = __float_as_uint(x1);
  const uint32_t b2 = __float_as_uint(x2), b3 = __float_as_uint(x3);
  const float a0 = fabsf(x0), a1 = fabsf(x1), a2 = fabsf(x2), a3 = fabsf(x3);
  // two smallest of four magnitudes: inserting a into n1 <= n2 gives min(n1, a)
  // and the median of {n1, n2, a}; as the magnitudes lie in [0, clip], min and
  // max are medians with -clip and clip (three-operand medians take the
  // absolute values as operand modifiers)
  float f1 = __builtin_amdgcn_fmed3f(a0, a1, -clip);
  float f2 = __builtin_amdgcn_fmed3f(a0, a1, clip);
  f2 = __builtin_amdgcn_fmed3f(f1, f2, a2);
  f1 = __builtin_amdgcn_fmed3f(f1, a2, -clip);
  f2 = __builtin_amdgcn_fmed3f(f1, f2, a3);
  f1 = __builtin_amdgcn_fmed3f(f1, a3, -clip);
  CnAcc a;   // non-negative floats order like their bit patterns
  a.n1 = __float_as_uint(f1);
  a.n2 = __float_as_uint(f2);
  // parities of the message signs and of the hard decisions, kept in bit 31
  a.sp = xor_sign(xor3(b0, b1, b2), b3);
  a.hp = xor_sign(xor3(c.g.x, c.g.y, c.g.z), c.g.w);
  cn_group(a, lk);
  const uint32_t srow = (P.sres >> t) << 31;   // residual syndrome bit of the row
  const uint32_t sgn = a.sp ^ srow;
  const float n1 = __uint_as_float(a.n1);
  const uint32_t s1 = __float_as_uint(alpha * n1) | sgn;
  const uint32_t s2 = __float_as_uint(alpha * __uint_as_float(a.n2)) | sgn;
  float4 nv;
  nv.x = __uint_as_float((a0 == n1 ? s2 : s1) ^ (b0 & kSign));
  nv.y = __uint_as_float((a1 == n1 ? s2 : s1) ^ (b1 & kSign));
  nv.z = __uint_as_float((a2 == n1 ? s2 : s1) ^ (b2 & kSign));
  nv.w = __uint_as_float((a3 == n1 ? s2 : s1) ^ (b3 & kSign));
  *(float4*)(P.c2v + e0) = nv;
  return (int)(srow ^ a.hp);   // bit 31: the row is unsatisfied
}

// Gather of a slot's four posteriors (hard decisions in the sign bits).
template <int VPL>
__device__ __forceinline__ void gather_post(const PathCtx<VPL>& P, Slot& s) {
  s.g.x = __float_as_uint(at_byte(P.post, s.vo.x & 0xffffu));
  s.g.y = __float_as_uint(at_byte(P.post, s.vo.x >> 16));
  s.g.z = __float_as_uint(at_byte(P.post, s.vo.y & 0xffffu));
  s.g.w = __float_as_uint(at_byte(P.post, s.vo.y >> 16));
}

// Syndrome check of one slot: bit 0 set if its row is unsatisfied by the
// gathered hard decisions; optionally records the row's flag for Alg. 3.
template <int VPL>
__device__ __forceinline__ int check_slot(const PathCtx<VPL>& P, const Slot& s, int t,
                                          bool write_unsat) {
  const uint32_t mt = s.mt;
  uint32_t hp = xor3(s.g.x, s.g.y, s.g.z) ^ s.g.w;
  hp_group(hp, (mt >> kMetaLogKShift) & 7);
  const int hx = (int)(((P.sres >> t) & 1u) ^ (hp >> 31));
  if (write_unsat && (mt & kMetaLead) && (mt & kMetaValid))
    P.unsat[(mt >> kMetaRowShift) & 0x3ff] = (uint8_t)hx;
  return hx;
}

template <int VPL, bool REC = false>
__device__ __forceinline__ int cn_phase(PathCtx<VPL>& P, float alpha, float clip) {
  return slot_walk<VPL, true, REC>(
      P, [&](Slot& s) { gather_post(P, s); },
      [&](const Slot& s, int t) { return cn_slot(P, s, t, alpha, clip); });
}

// Syndrome check of the current hard decisions; optionally records each
// row's unsatisfied flag for Alg. 3.
template <int VPL, bool REC = false>
__device__ __forceinline__ int check_pass(PathCtx<VPL>& P, bool write_unsat) {
  return slot_walk<VPL, false, REC>(
      P, [&](Slot& s) { gather_post(P, s); },
      [&](const Slot& s, int t) { return check_slot(P, s, t, write_unsat); });
}

// VN phase: posteriors of the owned active VNs (Eq. 2), summed in column slot
// order, and the history of the last four iterations of the step. The first
// five slots of every owned VN are gathered together, without a branch between
// the loads (index loads, then message loads), so that their LDS latencies
// overlap: the fifth index is read for every VN -- the column slot table keeps
// four readable entries past its end -- and its message added only to VNs of
// degree above four. VNs of degree above five take a loop. The sum is formed
// negated, t = -L - m1 - m2 - ..., in the same order: round-to-nearest is
// symmetric, so -t is the sum exactly, and an exact zero (t = +0) comes out as
// -0 -- the sign bit is then the hard decision of Eq. 4. Returns the number of
// edges of the active VNs.
template <int VPL>
__device__ __forceinline__ int vn_phase(PathCtx<VPL>& P, bool hist, float* ring_slot) {
  uint2 ix[VPL];
  uint32_t ix5[VPL];
#pragma unroll
  for (int r = 0; r < VPL; ++r) {
    ix[r] = *(const uint2*)(P.cidx + P.vc0(r));
    ix5[r] = P.cidx[P.vc0(r) + 4];
  }
  __builtin_amdgcn_sched_barrier(0);
  float g[VPL][5];
#pragma unroll
  for (int r = 0; r < VPL; ++r) {
    g[r][0] = at_byte(P.c2v, ix[r].x & 0xffffu);
    g[r][1] = at_byte(P.c2v, ix[r].x >> 16);
    g[r][2] = at_byte(P.c2v, ix[r].y & 0xffffu);
    g[r][3] = at_byte(P.c2v, ix[r].y >> 16);
    g[r][4] = at_byte(P.c2v, ix5[r]);
  }
  __builtin_amdgcn_sched_barrier(0);
  float t[VPL];
  bool deep = false;
#pragma unroll
  for (int r = 0; r < VPL; ++r) {
    const float t4 = (((-P.llr[r] - g[r][0]) - g[r][1]) - g[r][2]) - g[r][3];
    t[r] = P.vdg(r) > 4 ? t4 - g[r][4] : t4;
    deep |= P.vdg(r) > 5;
  }
  if (wave_any(deep)) {
#pragma unroll
    for (int r = 0; r < VPL; ++r)
      for (int k = 5; k < P.vdg(r); ++k) t[r] -= at_byte(P.c2v, P.cidx[P.vc0(r) + k]);
  }
#pragma unroll
  for (int r = 0; r < VPL; ++r) {
    const int v = P.lane + kWave * r;
    if (v < P.n && P.st(r) < 0) {
      const float x = __uint_as_float(__float_as_uint(t[r]) ^ 0x80000000u);   // -t, -0 for +0
      P.post[v] = x;
      if (ring_slot) ring_slot[v] = x;
      if (hist) {
        // min and max as medians with -/+FLT_MAX (the posteriors are finite;
        // a median with an infinity would be turned into a min or max that
        // quiets NaNs first)
        P.hs[r] += x;
        P.hmn[r] = __builtin_amdgcn_fmed3f(P.hmn[r], x, -__FLT_MAX__);
        P.hmx[r] = __builtin_amdgcn_fmed3f(P.hmx[r], x, __FLT_MAX__);
      }
    }
  }
  return P.act_edges;
}

// VN phase of the whole-window BP: posteriors (Eq. 2) of the workgroup's VNs,
// summed in column-slot order (padding adds the zero message), exact zeros
// stored as -0 (sign bit = hard decision; the sum is formed negated as in
// vn_phase), plus the running sum of the last iterations when lsum is given.
// Four VNs per thread per round: one 16-byte record load each (first five
// message offsets, degree, prior), then all their message loads together.
__device__ __forceinline__ void full_vn_pass(const gdg_win_dev& w, float* post, const float* c2v,
                                             float* lsum) {
  const int n = w.n, bs = blockDim.x;
  constexpr int kV = 4;   // VNs per thread and round: their record loads in flight together
  for (int v0 = threadIdx.x; v0 < n; v0 += kV * bs) {
    uint4 rc[kV];
#pragma unroll
    for (int j = 0; j < kV; ++j) rc[j] = w.fr_vrec[min(v0 + j * bs, n - 1)];
    float g[kV][5];
#pragma unroll
    for (int j = 0; j < kV; ++j) {
      g[j][0] = at_byte(c2v, rc[j].x & 0xffffu);
      g[j][1] = at_byte(c2v, rc[j].x >> 16);
      g[j][2] = at_byte(c2v, rc[j].y & 0xffffu);
      g[j][3] = at_byte(c2v, rc[j].y >> 16);
      g[j][4] = at_byte(c2v, rc[j].z & 0xffffu);
    }
    float t[kV];
    bool deep = false;
#pragma unroll
    for (int j = 0; j < kV; ++j) {
      t[j] = ((((-__uint_as_float(rc[j].w) - g[j][0]) - g[j][1]) - g[j][2]) - g[j][3]) - g[j][4];
      deep |= (rc[j].z >> 16) > 5;
    }
    if (wave_any(deep)) {
#pragma unroll
      for (int j = 0; j < kV; ++j) {
        const int v = min(v0 + j * bs, n - 1);
        const int dg = rc[j].z >> 16;
        for (int k = 5; k < dg; ++k) t[j] -= at_byte(c2v, w.fr_cidx[w.fr_cptr[v] + k]);
      }
    }
#pragma unroll
    for (int j = 0; j < kV; ++j) {
      const int v = v0 + j * bs;
      if (v >= n) continue;
      const float x = __uint_as_float(__float_as_uint(t[j]) ^ 0x80000000u);
      post[v] = x;
      if (lsum) lsum[v] += x;
    }
  }
}

// Flooding min-sum on the whole window graph, by the whole workgroup: the
// preprocessing BP of Sec. III and Sec. IV-C (Eqs. 1-4), also behind gdg_bp.
// It uses the path BP's CN code on the window graph's lane-group slot table
// (built on the host), split over the wavefronts: column i of wavefront wv is
// table column wv + i W. LDS arrays: syn [m] the window syndrome, post [n + 1]
// (entry n: the padding's dummy VN), c2v [fr_epad + 2 kPad], lsum [n] (may be
// null). From fresh messages it runs up to n_iters iterations; with `stop` it
// ends after the first iteration whose hard decisions (Eq. 4) meet the
// syndrome, otherwise it runs them all. lsum accumulates the posteriors of the
// last four iterations of n_iters. rec (global [n_iters][n], may be null)
// receives every iteration's posteriors, NaN for iterations not run. Returns
// the first iteration whose hard decisions met the syndrome (0: none) and
// sets *done to the number of iterations run. Every thread enters.
// Warm start (Sec. V's message reuse): with `warm` (the previous window's
// handed-over messages, indexed through w.warm_map) the CN-to-VN messages of
// edges the previous window also had start from those values instead of
// zero, and one VN pass forms the first posteriors and VN-to-CN messages from
// them. With `hand_over` the BP ends on a CN update of its final VN-to-CN
// messages, the messages the next window starts from: a BP that stops early
// has already made it (the CN walk that found the syndrome met), otherwise
// the closing check walk makes it.
template <int VPL>
__device__ __forceinline__ int window_bp(const gdg_win_dev& w, const uint8_t* syn, float* post,
                                         float* c2v,
                         float* lsum, const int n_iters, const bool stop, float* rec, int* done,
                         const float* warm = nullptr, const bool hand_over = false) {
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = w.n;
  for (int c = tid; c < n; c += blockDim.x) {
    post[c] = w.llr[c];
    if (lsum) lsum[c] = 0.0f;
  }
  if (tid == 0) post[n] = kInfF;   // dummy VN of the row padding
  for (int e = tid; e < w.fr_epad + 2 * kPad; e += blockDim.x) {
    float x = 0.0f;
    if (warm && e < w.fr_epad) {
      const int q = w.warm_map[e];
      if (q >= 0) x = warm[q];
    }
    c2v[e] = x;
  }
  const int nw = blockDim.x >> 6;
  const int my_T = wave < w.fr_T ? (w.fr_T - wave + nw - 1) / nw : 0;
  PathCtx<VPL> F;
  F.rvn = w.fr_rvn;
  F.meta = w.fr_meta;
  F.rec = w.fr_rec;
  F.post = post;
  F.c2v = c2v;
  F.lane = lane;
  F.m = w.m;
  F.n = n;
  F.tstride = nw;
  // syndrome bits of this wavefront's slot columns (at most 64)
  uint32_t syn0 = 0u, syn1 = 0u;
  for (int i = 0; i < my_T; ++i) {
    const uint32_t mt = w.fr_meta[(wave + i * nw) * kWave + lane];
    const uint32_t b = (mt & kMetaValid) ? (uint32_t)syn[(mt >> kMetaRowShift) & 0x3ff] : 0u;
    if (i < 32)
      syn0 |= b << i;
    else
      syn1 |= b << (i - 32);
  }
  __syncthreads();
  auto walk = [&](bool messages) {
    int bad = 0;
    for (int c = 0; c < 2; ++c) {
      if (my_T <= 32 * c) break;
      F.t0 = wave + 32 * c * nw;
      F.T = min(32, my_T - 32 * c);
      F.sres = c ? syn1 : syn0;
      bad |= messages ? cn_phase<VPL, true>(F, w.alpha, w.clip) : check_pass<VPL, true>(F, false);
    }
    return bad;
  };
  int first = 0, it = 0;
  // a warm start begins with a VN pass over the carried messages (t = 0)
  for (int t = warm ? 0 : 1; t <= n_iters; ++t) {
    if (t > 0) {
      // the CN phase also checks the hard decisions of iteration t - 1
      const int any_bad = __syncthreads_or(walk(true));
      if (t >= 2 && !any_bad && first == 0) {
        first = t - 1;
        if (stop) break;
      }
    }
    full_vn_pass(w, post, c2v, lsum && t > 0 && t > n_iters - 4 ? lsum : nullptr);
    __syncthreads();
    if (t == 0) continue;
    it = t;
    if (rec)
      for (int c = tid; c < n; c += blockDim.x) rec[(long long)(t - 1) * n + c] = post[c];
  }
  if (first == 0 && !__syncthreads_or(walk(hand_over))) first = it;
  if (rec)
    for (long long i = (long long)it * n + tid; i < (long long)n_iters * n; i += blockDim.x)
      rec[i] = __builtin_nanf("");
  *done = it;
  return first;
}

// Eq. 5 in ascending window-column order: the wavefront's lanes gather the
// priors of the columns set in `bits` into `stage` in that order (a prefix sum
// over the words), then lane 0 adds them up in that order. The sum is valid on
// lane 0; `stage` holds at least as many doubles as bits can be set.
__device__ __forceinline__ double eq5_sum(const uint32_t* bits, int words, const double* llr64,
                                          double* stage, int lane) {
  int n_set = 0;
  for (int w0 = 0; w0 < words; w0 += kWave) {
    const int wd = w0 + lane;
    uint32_t x = wd < words ? bits[wd] : 0u;
    const int cnt = __builtin_popcount(x);
    const int incl = wave_incl_scan(cnt, lane);
    int pos = n_set + incl - cnt;
    while (x) {
      const int bt = __builtin_ctz(x);
      x &= x - 1u;
      stage[pos++] = llr64[wd * 32 + bt];
    }
    n_set += __builtin_amdgcn_readlane(incl, kWave - 1);
  }
  wave_sync();
  double pm = 0.0;
  if (lane == 0)
    for (int i = 0; i < n_set; ++i) pm += stage[i];
  return pm;
}

// Path checkpoint copies between global memory (the checkpoint) and the
// LDS (the path's state), in whole 16-byte words (the regions are padded to
// 16). The address spaces are explicit so the copies are global and ds
// operations rather than flat ones.
typedef unsigned int gdg_u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) gdg_u32x4 gdg_glb_u4;
typedef __attribute__((address_space(3))) gdg_u32x4 gdg_lds_u4;

template <typename D, typename S>
__device__ __forceinline__ void ck_move(D* d, const S* s, int bytes, int lane) {
  const int n = (bytes + 15) / 16;
  for (int i = lane; i < n; i += kWave) d[i] = s[i];
}

// The restore is on the claiming wavefront's critical path: four loads in
// flight per lane rather than one.
__device__ __forceinline__ void ck_copy(void* dst, const uint4* src, int bytes, int lane) {
  gdg_lds_u4* d = (gdg_lds_u4*)dst;
  const gdg_glb_u4* q = (const gdg_glb_u4*)src;
  const int n = (bytes + 15) / 16;
  int i = lane;
  for (; i + 3 * kWave < n; i += 4 * kWave) {
    const gdg_u32x4 a = q[i], b = q[i + kWave], c = q[i + 2 * kWave], e = q[i + 3 * kWave];
    d[i] = a;
    d[i + kWave] = b;
    d[i + 2 * kWave] = c;
    d[i + 3 * kWave] = e;
  }
  for (; i < n; i += kWave) d[i] = q[i];
}

__device__ __forceinline__ void ck_save(uint4* dst, const void* src, int bytes, int lane) {
  ck_move((gdg_glb_u4*)dst, (const gdg_lds_u4*)src, bytes, lane);
}

// Decodes shot `shot` of one window with the whole workgroup. Every thread
// enters and leaves together; the caller synchronises before the LDS is reused.
// kLow: every window of the launch is in low-error mode (Alg. 3 off), which
// frees the registers only Alg. 3 reads.
template <int VPL, bool kLearn, bool kLow>
__device__ __attribute__((noinline)) void decode_shot(const gdg_win_dev& wref, const gdg_lds& L, const int shot,
                            const uint8_t* __restrict__ syn, const long long syn_stride,
                            uint8_t* __restrict__ ehat, double* __restrict__ pm_out,
                            int* __restrict__ flags_out, const gdg_trace_dev& tr,
                            const gdg_learn_dev& lrn, unsigned char* smem, const int lds_alloc,
                            char* const ck, const long long ck_stride,
                            const float* __restrict__ warm_in, float* __restrict__ warm_out) {
  const gdg_win_dev w = wref;   // uniform: kept in scalar registers, not re-read
  const bool low_err = kLow || w.low_error;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m = w.m, n = w.n, n_act = w.n_act;

  // header
  uint8_t* sorig = smem + L.sorig;
  int16_t* sel = (int16_t*)(smem + L.sel);
  int* misc = (int*)(smem + L.misc);            // [0] path counter, [2] answer path
  uint32_t* obits = (uint32_t*)(smem + L.obits);  // window bitmask of the answer
  unsigned long long* eacc = (unsigned long long*)(smem + L.eacc);
  // after the preprocessing: the sub-graph and the path regions
  unsigned char* U = smem + L.u_base;
  uint8_t* psyn = U + L.psyn;                   // syndrome in sub-graph row order
  uint16_t* rptr = (uint16_t*)(U + L.rptr);
  uint16_t* cptr = (uint16_t*)(U + L.cptr);
  int8_t* st0 = (int8_t*)(U + L.st0);
  uint32_t* sres0 = (uint32_t*)(U + L.sres0);
  uint8_t* vdeg = U + L.vdeg;                   // sub-graph VN degrees (learned proposer)
  double* ppm = (double*)(U + L.ppm);
  int* pend = (int*)(U + L.pend);
  uint32_t* pbits = (uint32_t*)(U + L.pbits);
  int* tq = (int*)(U + L.tq);                   // path tasks, 8 ints each
  int* tready = (int*)(U + L.tready);           // task pushed
  uint16_t *rvn = nullptr, *cidx = nullptr, *crow = nullptr;   // sized per shot
  uint32_t* meta = nullptr;
  int path_base = 0;                            // first path region, from u_base
  int* iscan = (int*)(U + L.p_iscan);           // sub-graph build scratch (scans)
  float* sllr = (float*)(U + L.p_llr);
  uint8_t* sdeg = U + L.p_deg;

  for (int j = tid; j < m; j += blockDim.x) sorig[j] = syn[(long long)shot * syn_stride + j] & 1;
  if (tid == 0) {
    misc[0] = 0;
    misc[1] = 0;
    *eacc = 0ull;
  }
  for (int i = tid; i < L.obits_words; i += blockDim.x) obits[i] = 0u;
  __syncthreads();

  long long my_edges = 0;

  // ---------------------------------------------------------- preprocessing
  if (w.pre_iters > 0) {
    float* const ppost = (float*)(U + L.p_post);
    float* const pc2v = (float*)(U + L.p_c2v);
    float* const lsum = (float*)(U + L.p_lsum);
    int iters_done = 0;
    const bool conv =
        window_bp<VPL>(w, sorig, ppost, pc2v, lsum, w.pre_iters, true,
                       tr.pre_post ? tr.pre_post + (long long)shot * w.pre_iters * n : nullptr,
                       &iters_done, warm_in, warm_out != nullptr) != 0;
    if (tid == 0) *eacc = (unsigned long long)iters_done * (unsigned long long)w.e_full;
    if (warm_out) {
      // the messages the next window starts from (before the array is reused)
      for (int e = tid; e < w.fr_epad; e += blockDim.x) warm_out[e] = pc2v[e];
      __syncthreads();
    }
    if (conv) {
      // the hard decision of the preprocessing BP is the answer
      for (int base = wave * kWave; base < n; base += blockDim.x) {
        const int c = base + lane;
        const bool one = c < n && ppost[c] <= 0.0f;
        const unsigned long long bal = __ballot(one);
        if (lane == 0) {
          obits[base >> 5] = (uint32_t)bal;
          if ((base >> 5) + 1 < L.obits_words) obits[(base >> 5) + 1] = (uint32_t)(bal >> 32);
        }
      }
      __syncthreads();
      if (wave == 0) {
        // the message array is dead; it holds n doubles (sort_n >= n)
        const double pm = eq5_sum(obits, L.obits_words, w.llr64, (double*)pc2v, lane);
        if (lane == 0) {
          pm_out[shot] = pm;
          flags_out[shot] = 1;
        }
      }
      for (int c = tid; c < n; c += blockDim.x)
        ehat[(long long)shot * n + c] = (uint8_t)((obits[c >> 5] >> (c & 31)) & 1u);
      if (tr.sel)
        for (int v = tid; v < n_act; v += blockDim.x) tr.sel[(long long)shot * n_act + v] = -1;
      if (tr.ends)
        for (int i = tid; i < w.n_paths * 2; i += blockDim.x)
          tr.ends[(long long)shot * w.n_paths * 2 + i] = 0;
      if (tr.dec)
        for (int i = tid; i < w.n_paths * tr.log_cap * 3; i += blockDim.x)
          tr.dec[(long long)shot * w.n_paths * tr.log_cap * 3 + i] = -1;
      if (tr.first_post)
        for (int v = tid; v < n_act; v += blockDim.x)
          tr.first_post[(long long)shot * n_act + v] = __builtin_nanf("");
      if (tr.step_lsum)
        for (long long i = tid; i < (long long)w.n_paths * tr.log_cap * n_act; i += blockDim.x)
          tr.step_lsum[(long long)shot * w.n_paths * tr.log_cap * n_act + i] = __builtin_nanf("");
      if (tr.edge_iters && tid == 0) tr.edge_iters[shot] = (long long)*eacc;
      return;
    }
    // rank: ascending sum of the last four posteriors, ties by column index;
    // keep the n_act smallest keys (order-preserving float bits, column). A
    // radix select over the key's 32 + 16 bits (up to six 8-bit passes; it
    // stops once the bucket holding the n_act-th smallest key is kept whole)
    // finds a threshold K; the kept keys (<= K) are gathered in any order and
    // sorted.
    __syncthreads();
    int* hist = (int*)(U + L.p_keys);                 // [256]
    int* ctl = hist + 256;                            // [0], [1] key prefix, [2] still needed, [3] count
    unsigned long long* ck = (unsigned long long*)(ctl + 4);   // [n_act rounded up to a power of two]
    const int bs = blockDim.x;
    if (tid == 0) {
      ctl[0] = 0;
      ctl[1] = 0;
      ctl[2] = n_act;
      ctl[3] = 0;
    }
    unsigned long long kmask = 0ull;
    for (int pass = 0; pass < 6; ++pass) {
      const int shift = 40 - 8 * pass;   // key bits 47..0: ord(sum) << 16 | column
      for (int i = tid; i < 256; i += bs) hist[i] = 0;
      __syncthreads();
      const unsigned long long prefix =
          ((unsigned long long)(uint32_t)ctl[0] << 32) | (uint32_t)ctl[1];
      for (int c = tid; c < n; c += bs) {
        const unsigned long long k = ((unsigned long long)ord_f32(lsum[c]) << 16) | (unsigned)c;
        if ((k & kmask) == prefix) atomicAdd(&hist[(k >> shift) & 255u], 1);
      }
      __syncthreads();
      if (wave == 0) {
        int h[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) h[j] = hist[4 * lane + j];
        const int tot = h[0] + h[1] + h[2] + h[3];
        int run = wave_incl_scan(tot, lane) - tot;
        const int need = ctl[2];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (run < need && run + h[j] >= need) {
            unsigned long long np = prefix | ((unsigned long long)(4 * lane + j) << shift);
            // the whole bucket is kept: every key of it is <= the prefix with
            // all lower bits set, and the select ends here
            if (run + h[j] == need) np |= (1ull << shift) - 1ull;
            ctl[0] = (int)(uint32_t)(np >> 32);
            ctl[1] = (int)(uint32_t)np;
            ctl[2] = run + h[j] == need ? 0 : need - run;
          }
          run += h[j];
        }
      }
      kmask |= 0xffull << shift;
      __syncthreads();
      if (ctl[2] == 0) break;
    }
    const unsigned long long kthr = ((unsigned long long)(uint32_t)ctl[0] << 32) | (uint32_t)ctl[1];
    // the n_act kept keys (exactly those <= the threshold: keys are distinct)
    // in any order, padded with the largest key to a power of two, then
    // sorted ascending
    int sort_p = 1;
    while (sort_p < n_act) sort_p <<= 1;
    for (int i = n_act + tid; i < sort_p; i += bs) ck[i] = ~0ull;
    for (int c = tid; c < n; c += bs) {
      const unsigned long long k = ((unsigned long long)ord_f32(lsum[c]) << 16) | (unsigned)c;
      if (k <= kthr) {
        const int pos = atomicAdd(&ctl[3], 1);
        if (pos < n_act) ck[pos] = k;
      }
    }
    __syncthreads();
    wg_bitonic_sort(ck, sort_p);
    for (int i = tid; i < n_act; i += bs) sel[i] = (int16_t)(ck[i] & 0xffffu);
  } else {
    for (int v = tid; v < n_act; v += blockDim.x) sel[v] = (int16_t)v;
  }
  __syncthreads();

  // ---------------------------------------------------------- truncated sub-graph
  {
    int16_t* loc = (int16_t*)(U + L.p_loc);   // [n] sub-graph VN of each window column, or -1
    int16_t* perm = loc + n;                  // [m] rows by decreasing sub-graph degree
    for (int c = tid; c < n; c += blockDim.x) loc[c] = -1;
    __syncthreads();
    for (int v = tid; v < n_act; v += blockDim.x) loc[sel[v]] = (int16_t)v;
    for (int v = tid; v < n_act; v += blockDim.x) {
      const int c = sel[v];
      const int d = w.col_ptr[c + 1] - w.col_ptr[c];
      iscan[v] = (d + kPad - 1) / kPad * kPad;   // column slots padded to a multiple of 4
      sllr[v] = w.llr[c];
      sdeg[v] = (uint8_t)d;
      vdeg[v] = (uint8_t)d;
    }
    __syncthreads();
    wg_exclusive_scan_wave0(iscan, n_act);
    __syncthreads();
    for (int v = tid; v <= n_act; v += blockDim.x) cptr[v] = (uint16_t)iscan[v];
    __syncthreads();
    // rows in order of decreasing sub-graph degree; a row whose columns were
    // all truncated away and whose syndrome bit is 1 can never be satisfied
    int* rdeg = iscan;
    for (int j = tid; j < m; j += blockDim.x) {
      const int e1 = w.row_ptr[j + 1];
      int cnt = 0;
      for (int e = w.row_ptr[j]; e < e1; e += 8) {   // loads issued 8 at a time
        int cc[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) cc[i] = e + i < e1 ? w.row_col[e + i] : -1;
#pragma unroll
        for (int i = 0; i < 8; ++i) cnt += cc[i] >= 0 && loc[cc[i]] >= 0;
      }
      rdeg[j] = cnt;
    }
    __syncthreads();
    // position of each row: decreasing degree, ties by row index
    int dead = 0;
    for (int j = tid; j < m; j += blockDim.x) {
      const int dj = rdeg[j];
      int r = 0;
      for (int i = 0; i < m; ++i) {
        const int di = rdeg[i];
        r += di > dj || (di == dj && i < j);
      }
      perm[r] = (int16_t)j;
      dead |= dj == 0 && sorig[j];
    }
    dead = __syncthreads_or(dead);
    if (tid == 0) misc[4] = dead;
    // padded degree in sub-graph row order
    for (int pj = tid; pj < m; pj += blockDim.x)
      iscan[m + 1 + pj] = (rdeg[perm[pj]] + kPad - 1) / kPad * kPad;
    __syncthreads();
    for (int pj = tid; pj < m; pj += blockDim.x) rdeg[pj] = iscan[m + 1 + pj];
    __syncthreads();
    wg_exclusive_scan_wave0(iscan, m);
    __syncthreads();
    for (int j = tid; j <= m; j += blockDim.x) rptr[j] = (uint16_t)iscan[j];
    __syncthreads();
    // lane-group size of each row: the power of two >= its number of batches;
    // rows come by decreasing size, so the packing keeps groups aligned
    for (int pj = tid; pj < m; pj += blockDim.x) {
      const int nb = (rptr[pj + 1] - rptr[pj]) / kPad;
      iscan[m + 1 + pj] = nb == 0 ? 0 : 1 << (32 - __builtin_clz((unsigned)(2 * nb - 1)) - 1);
    }
    __syncthreads();
    wg_exclusive_scan_wave0(iscan + m + 1, m);
    __syncthreads();
    const int e_pad = rptr[m];
    const int n_slots = iscan[2 * m + 1];
    // the window's slot table is sized for the worst truncation; a shot past it
    // is flagged instead of decoded
    const int T = min((n_slots + kWave - 1) / kWave, L.meta_cols);
    const int cap = L.meta_cols * kWave;
    {
      const gdg_dyn_layout dl = gdg_dyn(L.dyn_base, e_pad, cptr[n_act], T, !low_err);
      rvn = (uint16_t*)(U + dl.rvn);
      cidx = (uint16_t*)(U + dl.cidx);
      crow = (uint16_t*)(U + dl.crow);
      meta = (uint32_t*)(U + dl.meta);
      path_base = dl.end;
    }
    const uint32_t idle = (uint32_t)(e_pad + kPad);   // the dummy batch
    for (int i = tid; i < (T + 3) * kWave; i += blockDim.x) meta[i] = idle;   // + 3 idle columns
    for (int i = tid; i < kPad; i += blockDim.x) rvn[e_pad + kPad + i] = (uint16_t)(4 * n_act);
    __syncthreads();
    for (int pj = tid; pj < m; pj += blockDim.x) {
      const int j = perm[pj];
      psyn[pj] = sorig[j];
      int pos = rptr[pj];
      const int e1 = w.row_ptr[j + 1];
      for (int e = w.row_ptr[j]; e < e1; e += 8) {   // loads issued 8 at a time
        int cc[8], kc[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          cc[i] = e + i < e1 ? w.row_col[e + i] : 0;
          kc[i] = e + i < e1 ? w.row_kcol[e + i] : 0;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int v = e + i < e1 ? loc[cc[i]] : -1;
          if (v < 0) continue;
          const int slot = cptr[v] + kc[i];
          rvn[pos] = (uint16_t)(4 * v);
          cidx[slot] = (uint16_t)(4 * pos);
          if (!low_err) crow[slot] = (uint16_t)pj;
          ++pos;
        }
      }
      for (; pos < rptr[pj + 1]; ++pos) rvn[pos] = (uint16_t)(4 * n_act);   // padding: dummy VN
      const int nb = (rptr[pj + 1] - rptr[pj]) / kPad;
      if (nb > 0) {
        const int g0 = iscan[m + 1 + pj];
        const int k = (pj + 1 < m ? iscan[m + 2 + pj] : n_slots) - g0;
        const int lk = 31 - __builtin_clz((unsigned)k);
        for (int i = 0; i < k && g0 + i < cap; ++i) {
          const int e0 = i < nb ? rptr[pj] + kPad * i : e_pad + kPad;
          meta[g0 + i] = (uint32_t)e0 | ((uint32_t)pj << kMetaRowShift) |
                         ((uint32_t)lk << kMetaLogKShift) | (sorig[j] ? kMetaSyn : 0u) |
                         (i == 0 ? kMetaLead : 0u) | kMetaValid;
        }
      }
    }
    for (int v = tid; v < n_act; v += blockDim.x) {
      const int c0 = cptr[v] + sdeg[v];
      for (int i = c0; i < cptr[v + 1]; ++i) cidx[i] = (uint16_t)(4 * e_pad);   // zero message
    }
    // four readable entries past the last column (the VN phase reads a fifth
    // index of every VN)
    for (int i = tid; i < kPad; i += blockDim.x) cidx[cptr[n_act] + i] = (uint16_t)(4 * e_pad);
    if (tid == 0) {
      misc[3] = T;
      misc[5] = n_slots > cap;
    }
    if (tr.sel)
      for (int v = tid; v < n_act; v += blockDim.x) tr.sel[(long long)shot * n_act + v] = sel[v];
    __syncthreads();
  }

  // ---------------------------------------------------------- decision paths
  // Run 0 is the configured path set: the plain tree of Fig. 2, or the learned
  // proposer's paths; run 1 is the plain tree again, as the fallback when no
  // learned path met the syndrome.
  const int mode = kLearn ? lrn.mode : 0;
  int fallback = 0;
  {
    const int e_pad = rptr[m];
    const gdg_path_layout pl = gdg_paths(e_pad, n_act, m, L.obits_words);
    // path wavefronts that fit in this launch's allocation (the LDS plan
    // guarantees one); the others only join the workgroup's barriers
    const int nwp = max(1, min((int)(blockDim.x >> 6), (lds_alloc - L.u_base - path_base) / pl.stride));
    const bool path_wave = wave < nwp;
    unsigned char* Wb = U + path_base + (path_wave ? wave : 0) * pl.stride;
    PathCtx<VPL> P;
    P.rvn = rvn;
    P.cidx = cidx;
    P.crow = crow;
    P.meta = meta;
    P.rec = nullptr;
    P.post = (float*)(Wb + pl.post);
    P.status = (int8_t*)(Wb + pl.status);
    P.c2v = (float*)(Wb + pl.c2v);
    P.unsat = Wb + pl.unsat;
    P.prop = (uint32_t*)(Wb + pl.prop);
    uint32_t* wbits = (uint32_t*)(Wb + pl.bits);
    P.lane = lane;
    P.m = m;
    P.n = n_act;
    P.T = __builtin_amdgcn_readfirstlane(misc[3]);
    P.sres = 0u;
    const bool dead0 = misc[4] != 0;
    const int T = w.iters;
    const float alpha = w.alpha, clip = w.clip;
#pragma unroll
    for (int r = 0; r < VPL; ++r) {
      const int v = lane + kWave * r;
      const int vv = v < n_act ? v : 0;
      P.vinfo[r] = v < n_act ? (uint32_t)cptr[vv] | ((uint32_t)sdeg[vv] << 16) : 0u;
      P.llr[r] = sllr[vv];
    }
    // the sub-graph build scratch (sllr, sdeg) shares LDS with the path regions
    __syncthreads();
    if (path_wave) {
      for (int i = lane; i < (n_act + 3) / 4; i += kWave) P.prop[i] = 0u;
      if (lane == 0) {
        P.post[n_act] = kInfF;   // dummy VN of the row padding
        P.status[n_act] = 0;
      }
    }
    // this wavefront's posterior history ring (learned proposer): slot j holds
    // the posteriors of BP iteration t with (t - 1) mod 16 = j
    float* const ring = mode ? lrn.ring + ((long long)blockIdx.x * (blockDim.x >> 6) + wave) *
                                              16 * lrn.ring_stride
                             : nullptr;
    wave_sync();
    // The peeling at the start of a path (Sec. IV-D) depends only on the
    // shot's syndrome and sub-graph: wavefront 0 runs it once and every path
    // starts from its result.
    if (wave == 0) {
      P.act_edges = 0;
#pragma unroll
      for (int r = 0; r < VPL; ++r) {
        const int v = lane + kWave * r;
        P.set_st(r, -1);
        if (v < n_act) P.status[v] = -1;
      }
      wave_sync();
      const bool ok = !dead0 && peel(P);
#pragma unroll
      for (int r = 0; r < VPL; ++r) {
        const int v = lane + kWave * r;
        if (v < n_act) st0[v] = (int8_t)P.st(r);
      }
      sres0[lane] = P.sres;
      if (lane == 0) misc[7] = ok;
    }
    __syncthreads();
    const bool peel0_ok = misc[7] != 0;

    for (int run = 0; run < 2; ++run) {
      if (run == 1) {
        if (mode != 1 || misc[6]) break;
        fallback = 1;
      }
      const bool learned = run == 0 && mode == 1;
      const int n_run = learned ? (1 << lrn.guesses) : w.n_paths;
      // Path tasks. A task is a range [lo, lo + size) of paths that share one
      // state up to depth d0 - 1 (the representative, path lo, stands for all
      // of them), starting fresh (d0 = 1) or from a checkpoint that the task's
      // parent left where Fig. 2's tree split: there the paths of the parent's
      // range whose bit for that depth is 1 take the other value of the
      // pending decision (gsel, val). Replaying a path from the root gives the
      // same state, messages included, so sharing changes no result. Learned
      // paths run one per task.
      const int n_tree = w.g > 0 ? 1 << w.g : 1;
      // (every path of a range must reach the split's decision: the tree
      // paths run past depth g when extra >= 1)
      const bool share = !learned && ck != nullptr && n_tree > 1 && w.extra > 0;
      // Branch and bound over the paths: with positive priors a path's Eq. 5
      // metric is at least the sum of the priors of its VNs fixed to 1 (they
      // stay 1 in its answer), plus the least active prior while its residual
      // syndrome is non-zero (see over_bound), so a path whose bound already
      // exceeds a converged path's metric cannot be the answer and stops. The comparison is in
      // FP32 against the metric widened by 2e-5, far above the rounding of
      // either side; the answer, its metric and the flags are unchanged (a
      // stop needs a converged path; a learned answer's fallback test reads
      // only the best metric). Off in record mode and when traces of every
      // path are asked for.
      const bool bound = mode != 2 && w.bound_ok && !tr.dec && !tr.ends && !tr.step_lsum;
      if (tid == 0) {
        int nt = 0;
        auto push0 = [&](int plo, int psize) {
          int* t = tq + 8 * nt;
          t[0] = plo;
          t[1] = psize;
          t[2] = 1;
          t[3] = -1;
          t[4] = 0;
          t[5] = -1;
          t[6] = 0;
          t[7] = 0;
          tready[nt++] = 1;
        };
        if (share) {
          push0(0, n_tree);
          for (int p = n_run - 1; p >= n_tree; --p) push0(p, 1);   // side branches
        } else {
          // decreasing id: the later paths of the tree deviate more often and
          // run longer, so starting them first leaves the short ones to the end
          for (int p = n_run - 1; p >= 0; --p) push0(p, 1);
        }
        for (int t = nt; t < w.n_paths; ++t) tready[t] = 0;
        misc[0] = 0;    // tasks claimed
        misc[1] = nt;   // tasks pushed
        misc[8] = 0;    // paths finished
        misc[9] = 0;    // checkpoints taken
        misc[10] = 0x7f800000;   // stopping threshold: least converged Eq. 5 metric, widened
      }
      __syncthreads();
      while (path_wave) {
        // claim the next task; wait for it to be pushed, or for every path to
        // finish (a claim past the last task)
        int ti = 0;
        if (lane == 0) ti = atomicAdd(&misc[0], 1);
        ti = __builtin_amdgcn_readfirstlane(ti);
        bool have = false;
        for (;;) {
          int rd = 0, fin = 0;
          if (lane == 0) {
            rd = ti < w.n_paths
                     ? __hip_atomic_load(&tready[ti], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)
                     : 0;
            fin = __hip_atomic_load(&misc[8], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
          rd = __builtin_amdgcn_readfirstlane(rd);
          fin = __builtin_amdgcn_readfirstlane(fin);
          if (rd) {
            have = true;
            break;
          }
          if (fin >= n_run) break;
          __builtin_amdgcn_s_sleep(2);
        }
        if (!have) break;
        int lo = __builtin_amdgcn_readfirstlane(tq[8 * ti + 0]);
        int size = __builtin_amdgcn_readfirstlane(tq[8 * ti + 1]);
        const int d0 = __builtin_amdgcn_readfirstlane(tq[8 * ti + 2]);
        // the range's representative path and its depth limits
        int pid, dmax, split;
        auto represent = [&](int p) {
          pid = p;
          if (pid == 0 || (learned && !lrn.tree)) {
            dmax = w.dmax_main;
            split = 0;
          } else if (learned) {   // Fig. 2's tree with `guesses` levels
            dmax = lrn.guesses + w.extra;
            split = lrn.guesses;
          } else if (w.g > 0 && pid < (1 << w.g)) {
            dmax = w.g + w.extra;
            split = w.g;
          } else {
            split = w.g + 1 + (pid - (1 << w.g));
            dmax = split + w.extra;
          }
          // uniform: scalar registers
          pid = __builtin_amdgcn_readfirstlane(pid);
          dmax = __builtin_amdgcn_readfirstlane(dmax);
          split = __builtin_amdgcn_readfirstlane(split);
        };
        represent(lo);
        const bool record = run == 0 && mode == 2 && pid == 0;
        const bool use_ring = learned || record;
        int guess_used = 0;
        bool deviated = false;
        // decision log rows of the range's paths: path lo + i at dlog + i * dlog_step
        int* const dlog0 = (tr.dec && !learned) ? tr.dec + (long long)shot * w.n_paths * tr.log_cap * 3
                                                : nullptr;
        int* dlog = dlog0 ? dlog0 + (long long)pid * tr.log_cap * 3 : nullptr;
        const int dlog_step = tr.log_cap * 3;

        if (d0 == 1) {
          // fresh path: the VNs left active by the initial peeling take their
          // priors as posteriors
#pragma unroll
          for (int r = 0; r < VPL; ++r) {
            const int v = lane + kWave * r;
            const int st = v < n_act ? (int)st0[v] : -1;
            P.set_st(r, st);
            if (r == 0) P.act_edges = 0;
            if (v < n_act && st < 0) P.act_edges += P.vdg(r);
            if (v < n_act) {
              P.status[v] = (int8_t)st;
              P.post[v] = st < 0 ? P.llr[r] : kInfF;
              if (use_ring)
                for (int j = 0; j < 16; ++j) ring[j * lrn.ring_stride + v] = P.llr[r];
            }
          }
          P.sres = sres0[lane];
          // t = 0: no CN message yet; also clears the zero slot and the dummy batch
          for (int e = lane; e < e_pad + 2 * kPad; e += kWave) P.c2v[e] = 0.0f;
        } else {
          // the parent's checkpoint: posteriors, statuses, messages, residual bits
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
          const gdg_ck_layout cl = gdg_ck(n_act, e_pad);
          const char* cb = ck + (long long)__builtin_amdgcn_readfirstlane(tq[8 * ti + 5]) * ck_stride;
          ck_copy(P.post, (const uint4*)(cb + cl.post), 4 * (n_act + 1), lane);
          ck_copy(P.status, (const uint4*)(cb + cl.status), n_act + 1, lane);
          ck_copy(P.c2v, (const uint4*)(cb + cl.c2v), 4 * (e_pad + 2 * kPad), lane);
          P.sres = ((const uint32_t*)(cb + cl.sres))[lane];
          wave_sync();
          P.act_edges = 0;
#pragma unroll
          for (int r = 0; r < VPL; ++r) {
            const int v = lane + kWave * r;
            const int st = v < n_act ? (int)P.status[v] : -1;
            P.set_st(r, st);
            if (v < n_act && st < 0) P.act_edges += P.vdg(r);
          }
        }
        wave_sync();
        int end = 0, steps = d0 - 1, it = 0;
        if (d0 == 1 && !peel0_ok) end = END_CONTRADICTION;
        if (d0 > 1) {
          // the decision of depth d0 - 1 with this range's value
          const int gsel = __builtin_amdgcn_readfirstlane(tq[8 * ti + 3]);
          const int val = __builtin_amdgcn_readfirstlane(tq[8 * ti + 4]);
          const int n_agg = __builtin_amdgcn_readfirstlane(tq[8 * ti + 7]);
          set_status_uniform(P, gsel, val);
          if (dlog && lane < size && d0 - 2 < tr.log_cap) {
            int* row = dlog + lane * dlog_step + (d0 - 2) * 3;
            row[0] = gsel;
            row[1] = val;
            row[2] = n_agg;
          }
          wave_sync();
          if (!peel(P)) end = END_CONTRADICTION;
          if (end == 0 && bound && over_bound(P, misc + 10)) end = END_BOUND;
        }
        for (int D = d0; end == 0 && D <= dmax; ++D) {
#pragma unroll
          for (int r = 0; r < VPL; ++r) {
            P.hs[r] = 0.0f;
            P.hmn[r] = kInfF;
            P.hmx[r] = -kInfF;
          }
          bool conv = false;
          for (int t = 1; t <= T; ++t) {
            const int bad = cn_phase(P, alpha, clip);
            const bool any_bad = wave_any(bad != 0);
            if (t >= 2 && !any_bad) {
              conv = true;
              break;
            }
            wave_sync();
            my_edges += vn_phase(P, t > T - 4, use_ring ? ring + (it & 15) * lrn.ring_stride : nullptr);
            ++it;
            wave_sync();
          }
          if (!conv) conv = !wave_any(check_pass(P, !low_err) != 0);
          steps = D;
          if (tr.step_lsum && !learned && D - 1 < tr.log_cap) {
            for (int i = 0; i < size; ++i) {
              float* sl = tr.step_lsum +
                          (((long long)shot * w.n_paths + pid + i) * tr.log_cap + (D - 1)) * n_act;
#pragma unroll
              for (int r = 0; r < VPL; ++r) {
                const int v = lane + kWave * r;
                if (v < n_act) sl[v] = (!conv && P.st(r) < 0) ? P.hs[r] : __builtin_nanf("");
              }
            }
          }
          if (tr.first_post && pid == 0 && D == 1 && run == 0) {
#pragma unroll
            for (int r = 0; r < VPL; ++r) {
              const int v = lane + kWave * r;
              if (v < n_act)
                tr.first_post[(long long)shot * n_act + v] = P.st(r) < 0 ? P.post[v] : __builtin_nanf("");
            }
          }
          if (conv) {
            end = END_CONVERGED;
            break;
          }
          if (D == dmax) {
            end = END_EXHAUSTED;
            break;
          }
          // Alg. 1 with Alg. 3 inside it
          wave_sync();
          const bool on_main = learned && !lrn.tree ? !deviated : path_on_main(w, pid, split, D);
          unsigned long long kall = ~0ull, kneg = ~0ull;
          int n_agg = 0;
          // the proposer picks this step's candidate; Alg. 1's keys are then
          // unused, and in low-error mode (no Alg. 3) the pass is skipped
          const bool use_mlp = kLearn && (learned || (record && D <= lrn.rec_steps));
#pragma unroll
          for (int r = 0; r < VPL; ++r) {
            const int v = lane + kWave * r;
            if (!(use_mlp && low_err) && v < n_act && P.st(r) < 0 && P.vdg(r) >= 3) {
              bool taken = false;
              if (!low_err) {
                int nu = 0;
                for (int e = P.vc0(r); e < P.vc0(r) + P.vdg(r); ++e) nu += P.unsat[P.crow[e]];
                const int b = agg_dec(P.hs[r], P.hmn[r], P.hmx[r], D, on_main, nu);
                if (b >= 0) {
                  set_status(P, r, v, b);
                  ++n_agg;
                  taken = true;
                }
              }
              if (!taken) {
                const uint32_t o = ord_f32(P.hs[r]);
                const unsigned long long k = ((unsigned long long)o << 32) | (unsigned)v;
                kall = k < kall ? k : kall;
                if (P.hmx[r] <= 0.0f) kneg = k < kneg ? k : kneg;
              }
            }
          }
          int gsel, fav, val;
          if (use_mlp) {
            // the proposer's candidates: the first n_cand VNs in Alg. 1's order
            // key: all-<=0 class first, then L_sum, then index
            unsigned long long mine = ~0ull;   // lane l: candidate l % 16
            uint32_t used = 0u;                // bit r: VN lane + 64 r already taken
            int n_found = 0;
            for (int i = 0; i < lrn.n_cand; ++i) {
              unsigned long long lm = ~0ull;
#pragma unroll
              for (int r = 0; r < VPL; ++r) {
                const int v = lane + kWave * r;
                if (v < n_act && P.st(r) < 0 && P.vdg(r) >= 3 && !((used >> r) & 1u)) {
                  const unsigned long long k = ((P.hmx[r] <= 0.0f ? 0ull : 1ull) << 63) |
                                               ((unsigned long long)ord_f32(P.hs[r]) << 31) |
                                               (unsigned)v;
                  lm = k < lm ? k : lm;
                }
              }
              const unsigned long long km = wave_min_u64(lm);
              if (km == ~0ull) break;
              const int kv = (int)(km & 0x7fffffffu);
              if ((kv & (kWave - 1)) == lane) used |= 1u << (kv >> 6);
              if ((lane & 15) == i) mine = km;
              ++n_found;
            }
            if (n_found == 0) {
              end = END_NO_CANDIDATE;
              break;
            }
            const bool valid = mine != ~0ull;
            const int cv = valid ? (int)(mine & 0x7fffffffu) : 0;
            const uint32_t co = (uint32_t)(mine >> 31);
            const int cfav = (mine >> 63) == 0ull ? 1 : (co <= 0x80000000u ? 1 : 0);
            // features: posteriors of iterations it - 15 .. it (priors before the
            // first), squashed, and the degree
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            const int q = lane >> 4;
            float f[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const float pv = ring[((it + 4 * q + j) & 15) * lrn.ring_stride + cv];
              f[j] = pv / (8.0f + fabsf(pv));
            }
            const float fd = (float)vdeg[cv] * 0.125f;
            if (record) {
              const long long base = ((long long)shot * lrn.rec_steps + (D - 1)) * 16 + (lane & 15);
              if (valid) {
#pragma unroll
                for (int j = 0; j < 4; ++j) lrn.rec_x[base * 17 + 4 * q + j] = f[j];
                if (q == 0) {
                  lrn.rec_x[base * 17 + 16] = fd;
                  lrn.rec_col[base] = sel[cv];
                  lrn.rec_fav[base] = cfav;
                }
              }
              // the plain main path continues with Alg. 1's choice
              const int c0 = __builtin_amdgcn_readlane(cv, 0);
              gsel = c0;
              fav = __builtin_amdgcn_readlane(cfav, 0);
              val = fav;
            } else {
              float z = mlp_score_tile(lrn.model, f, fd);
              z = valid ? z : -kInfF;
              const unsigned long long zk = ((unsigned long long)(~ord_f32(z)) << 32) | (unsigned)(lane & 15);
              const int cbest = (int)(wave_min_u64(zk) & 0xffffffffu);
              const float zb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(z), cbest));
              // the candidate most likely in error, decimated to the network's
              // decision; a guess point when that decision is not confident
              gsel = __builtin_amdgcn_readlane(cv, cbest);
              fav = zb >= 0.0f ? 1 : 0;
              val = fav;
              if (lrn.tree) {
                // guesses at depths 1..guesses as in Fig. 2 (path bit D, MSB first)
                if (pid > 0 && D <= lrn.guesses && ((pid >> (lrn.guesses - D)) & 1)) val = 1 - fav;
              } else if (fabsf(zb) < lrn.tau && guess_used < lrn.guesses) {
                const int bit = (pid >> guess_used) & 1;
                ++guess_used;
                if (bit) {
                  val = 1 - fav;
                  deviated = true;
                }
              }
            }
          } else {
            kall = wave_min_u64(kall);
            kneg = wave_min_u64(kneg);
            if (kneg != ~0ull) {
              gsel = (int)(kneg & 0xffffffffu);
              fav = 1;
            } else if (kall != ~0ull) {
              gsel = (int)(kall & 0xffffffffu);
              fav = (uint32_t)(kall >> 32) <= 0x80000000u ? 1 : 0;   // sum <= 0 -> 1
            } else {
              gsel = -1;
              fav = 0;
            }
            val = gsel < 0 ? 0 : path_value(w, pid, split, D, fav);
          }
          if (dlog || !low_err) n_agg = wave_sum_i32(n_agg);
          if (gsel < 0) {
            if (dlog && lane < size && D - 1 < tr.log_cap) {
              int* row = dlog + lane * dlog_step + (D - 1) * 3;
              row[0] = -1;
              row[1] = -1;
              row[2] = n_agg;
            }
            end = END_NO_CANDIDATE;
            break;
          }
          if (share && size > 1 && D <= w.g) {
            // Fig. 2's tree splits the range here: its upper half (bit g - D
            // set) takes 1 - fav, its lower half fav. This wavefront goes on
            // with the upper half -- the deviating paths tend to run longer, so
            // the longest chain of steps starts first -- and leaves the lower
            // half a checkpoint of the state before this decision. (The
            // recording path stays the plain main path.)
            const int h = size >> 1;
            const bool keep_upper = !record;
            int slot = 0, tn = 0;
            if (lane == 0) slot = atomicAdd(&misc[9], 1);
            slot = __builtin_amdgcn_readfirstlane(slot);
            const gdg_ck_layout cl = gdg_ck(n_act, e_pad);
            char* cb = ck + (long long)slot * ck_stride;
            ck_save((uint4*)(cb + cl.post), P.post, 4 * (n_act + 1), lane);
            ck_save((uint4*)(cb + cl.status), P.status, n_act + 1, lane);
            ck_save((uint4*)(cb + cl.c2v), P.c2v, 4 * (e_pad + 2 * kPad), lane);
            ((uint32_t*)(cb + cl.sres))[lane] = P.sres;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            wave_sync();
            if (lane == 0) {
              tn = atomicAdd(&misc[1], 1);
              int* t = tq + 8 * tn;
              t[0] = keep_upper ? lo : lo + h;
              t[1] = h;
              t[2] = D + 1;
              t[3] = gsel;
              t[4] = keep_upper ? fav : 1 - fav;
              t[5] = slot;
              t[6] = lo;
              t[7] = n_agg;
              __hip_atomic_store(&tready[tn], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            size = h;
            val = fav;
            if (keep_upper) {
              lo += h;
              represent(lo);
              if (dlog0) dlog = dlog0 + (long long)pid * tr.log_cap * 3;
              val = 1 - fav;
            }
          }
          set_status_uniform(P, gsel, val);
          if (dlog && lane < size && D - 1 < tr.log_cap) {
            int* row = dlog + lane * dlog_step + (D - 1) * 3;
            row[0] = gsel;
            row[1] = val;
            row[2] = n_agg;
          }
          wave_sync();
          if (!peel(P)) {
            end = END_CONTRADICTION;
            break;
          }
          if (bound && over_bound(P, misc + 10)) {
            end = END_BOUND;
            break;
          }
        }
        if (end == 0) end = END_EXHAUSTED;   // dmax < 1
        // traces of every path of the range
        if (dlog) {
          // entries past the last logged step
          const int first_free =
              (end == END_CONVERGED || end == END_EXHAUSTED) ? steps - 1 : steps;
          for (int p = 0; p < size; ++p)
            for (int i = lane; i < tr.log_cap; i += kWave) {
              if (i >= first_free) {
                int* row = dlog + p * dlog_step + i * 3;
                row[0] = -1;
                row[1] = -1;
                row[2] = -1;
              }
            }
        }
        if (tr.step_lsum && !learned) {
          for (int p = 0; p < size; ++p)
            for (int i = steps; i < tr.log_cap; ++i) {
              float* sl = tr.step_lsum + (((long long)shot * w.n_paths + pid + p) * tr.log_cap + i) * n_act;
              for (int v = lane; v < n_act; v += kWave) sl[v] = __builtin_nanf("");
            }
        }
        if (tr.ends && lane < size && !learned) {
          tr.ends[((long long)shot * w.n_paths + pid + lane) * 2 + 0] = end;
          tr.ends[((long long)shot * w.n_paths + pid + lane) * 2 + 1] = steps;
        }
        // path answer: bits over the sub-graph
        uint32_t* mybits = pbits + pid * L.pbits_words;
#pragma unroll
        for (int r = 0; r < VPL; ++r) {
          const int v = lane + kWave * r;
          bool one = false;
          if (v < n_act) one = P.st(r) >= 0 ? P.st(r) == 1 : P.post[v] <= 0.0f;
          const unsigned long long bal = __ballot(one);
          if (lane == 0 && kWave * r < n_act) {
            mybits[2 * r] = (uint32_t)bal;
            if (2 * r + 1 < L.pbits_words) mybits[2 * r + 1] = (uint32_t)(bal >> 32);
          }
        }
        wave_sync();
        double pm = __builtin_inf();
        if (end == END_CONVERGED) {
          // Eq. 5 in ascending window-column order
          for (int i = lane; i < L.obits_words; i += kWave) wbits[i] = 0u;
          wave_sync();
          for (int v = lane; v < n_act; v += kWave) {
            if ((mybits[v >> 5] >> (v & 31)) & 1u) {
              const int c = sel[v];
              atomicOr(&wbits[c >> 5], 1u << (c & 31));
            }
          }
          wave_sync();
          // staged in the wavefront's message array (dead once the path has
          // ended, sized for n_act doubles)
          pm = eq5_sum(wbits, L.obits_words, w.llr64, (double*)P.c2v, lane);
        }
        // every path of the range has this answer
        for (int p = 1; p < size; ++p)
          for (int i = lane; i < L.pbits_words; i += kWave) pbits[(pid + p) * L.pbits_words + i] = mybits[i];
        if (lane < size) {
          // Eq. 5 came out on lane 0
          ppm[pid + lane] = __longlong_as_double(
              (long long)readlane64((unsigned long long)__double_as_longlong(pm), 0));
          pend[pid + lane] = end;
        }
        if (bound && end == END_CONVERGED && lane == 0) {
          // the metric widened by 2e-5 in FP32 (non-negative floats order like
          // their bit patterns)
          __hip_atomic_fetch_min(misc + 10, __float_as_int((float)(pm * (1.0 + 2e-5))), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        wave_sync();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (lane == 0) atomicAdd(&misc[8], size);
      }
      __syncthreads();
      // ---------------------------------------------------------- best path
      if (tid == 0) {
        int best = -1;
        double bpm = __builtin_inf();
        int n_contra = 0, n_exh = 0;
        for (int p = 0; p < n_run; ++p) {
          if (pend[p] == END_CONTRADICTION) ++n_contra;
          if (pend[p] == END_EXHAUSTED) ++n_exh;
          if (pend[p] == END_CONVERGED && ppm[p] < bpm) {
            bpm = ppm[p];
            best = p;
          }
        }
        int fl = 0;
        if (best >= 0) {
          fl = 1;
        } else {
          if (n_contra == n_run) fl |= 2;
          if (n_exh > 0) fl |= 4;
        }
        if (misc[5]) fl |= 16;
        if (fallback) fl |= 8;
        misc[2] = best >= 0 ? best : 0;
        // a learned answer stands if its path metric is at most pm_fallback
        misc[6] = best >= 0 && !(mode == 1 && run == 0 && bpm > (double)lrn.pm_fallback);
        pm_out[shot] = bpm;
        flags_out[shot] = fl;
      }
      __syncthreads();
    }
  }
  my_edges = wave_sum_i64(my_edges);
  if (lane == 0 && my_edges) atomicAdd(eacc, (unsigned long long)my_edges);
  __syncthreads();
  if (tid == 0 && tr.edge_iters) tr.edge_iters[shot] = (long long)*eacc;

  // ---------------------------------------------------------- output
  const uint32_t* ansbits = pbits + misc[2] * L.pbits_words;
  for (int v = tid; v < n_act; v += blockDim.x) {
    if ((ansbits[v >> 5] >> (v & 31)) & 1u) {
      const int c = sel[v];
      atomicOr(&obits[c >> 5], 1u << (c & 31));
    }
  }
  __syncthreads();
  for (int c = tid; c < n; c += blockDim.x)
    ehat[(long long)shot * n + c] = (uint8_t)((obits[c >> 5] >> (c & 31)) & 1u);
}

// Commit of one shot's window correction (Eqs. 7-9) by the whole workgroup:
// every DEM row the committed columns touch flips where their XOR is 1, and
// likewise every observable. The correction is read from its window bitmask,
// which the decode leaves in LDS (ebits); a row's column indices are loaded
// four at a time so that their global loads overlap. det_rel[row] is the
// shot's detector of DEM row `row` (the record shifted by the window object's
// own first row).
__device__ __forceinline__ void commit_shot(const gdg_commit_dev& cm, const uint32_t* ebits,
                                            uint8_t* det_rel, uint8_t* obs) {
  for (int r = threadIdx.x; r < cm.n_rows + cm.n_obs; r += blockDim.x) {
    const bool is_row = r < cm.n_rows;
    const int o = r - cm.n_rows;
    const int t0 = is_row ? cm.row_ptr[r] : cm.obs_ptr[o];
    const int t1 = is_row ? cm.row_ptr[r + 1] : cm.obs_ptr[o + 1];
    const int* cols = is_row ? cm.row_col : cm.obs_col;
    uint32_t x = 0u;
    int t = t0;
    for (; t + 4 <= t1; t += 4) {
      const int c0 = cols[t], c1 = cols[t + 1], c2 = cols[t + 2], c3 = cols[t + 3];
      x ^= (ebits[c0 >> 5] >> (c0 & 31)) ^ (ebits[c1 >> 5] >> (c1 & 31)) ^
           (ebits[c2 >> 5] >> (c2 & 31)) ^ (ebits[c3 >> 5] >> (c3 & 31));
    }
    for (; t < t1; ++t) x ^= ebits[cols[t] >> 5] >> (cols[t] & 31);
    x &= 1u;
    if (!x) continue;
    if (is_row)
      det_rel[cm.row_global[r]] ^= 1;
    else
      obs[o] ^= 1;
  }
}

// One experiment of a chained launch: its windows k_begin..k_end-1 in order,
// each decoded straight from the experiment's detector record and committed
// into it (and its observables) before the next window reads its syndrome.
template <int VPL, bool kLow>
__device__ __forceinline__ void decode_chain_item(
    const gdg_chain_dev& C, const int item, const gdg_trace_dev& tr, const gdg_learn_dev& lrn,
    unsigned char* smem, const int lds_alloc, char* const ck, const long long ck_stride) {
  const int kb = max(0, C.k_begin[item]);
  const int ke = min(C.K, C.k_end[item]);
  uint8_t* eh = C.ehat + (long long)item * C.ehat_stride;
  uint8_t* obs = C.obs + C.obs_off[item];
  for (int k = kb; k < ke; ++k) {
    // the window shape with static indices only (no dynamic indexing of the
    // kernel argument, which would copy it to private memory)
    const bool first = k == 0, last = k == C.K - 1;
    const gdg_win_dev* wp = first ? C.w[0] : (last ? C.w[2] : C.w[1]);
    const gdg_lds* lp = first ? C.L[0] : (last ? C.L[2] : C.L[1]);
    const int row0 = first ? C.row0[0] : (last ? C.row0[2] : C.row0[1]);
    const long long base = C.det_off[item] + (long long)k * C.row_step;
    decode_shot<VPL, false, kLow>(*wp, *lp, 0, C.det + base, 0, eh,
                                  C.pm + (long long)item * C.K + k,
                                  C.flags + (long long)item * C.K + k, tr, lrn, smem, lds_alloc,
                                  ck, ck_stride, nullptr, nullptr);
    __syncthreads();
    const uint32_t* ebits = (const uint32_t*)(smem + lp->obits);
    if (first)
      commit_shot(C.cm[0], ebits, C.det + base - row0, obs);
    else if (last)
      commit_shot(C.cm[2], ebits, C.det + base - row0, obs);
    else
      commit_shot(C.cm[1], ebits, C.det + base - row0, obs);
    __syncthreads();
  }
}

// Persistent decode: workgroup b takes items b, b + gridDim.x, ... of the job
// table; item i belongs to the job whose first item is the largest <= i. Jobs
// may use windows of different codes (sizes): each job carries its own LDS
// layout within the launch's allocation.
// Register budget: three wavefronts per SIMD with up to 7 VNs per lane (168
// VGPRs; the plain kernel's spills stay outside the BP loops, the learned
// kernel's reach the candidate scoring but the occupancy pays for them), two
// otherwise.
template <int VPL, bool kLearn>
constexpr int kDecodeWavesPerSimd = VPL <= 7 ? 3 : 2;

template <int VPL, bool kLearn, bool kLow>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(
    kDecodeWavesPerSimd<VPL, kLearn>, kDecodeWavesPerSimd<VPL, kLearn>))) void gdg_decode_kernel(gdg_jobs_dev J, gdg_trace_dev tr) {
  extern __shared__ __align__(16) unsigned char smem[];
  char* const ck = J.ckpt && (int)blockIdx.x < J.ckpt_wgs
                       ? J.ckpt + (long long)blockIdx.x * J.ckpt_slots * J.ckpt_stride
                       : nullptr;
  int item = blockIdx.x;
  for (;;) {
    if (J.work) {
      // the next shot from the launch's counter, passed through the first LDS
      // word (the syndrome, written only once the shot starts)
      if (threadIdx.x == 0) *(int*)smem = atomicAdd(J.work, 1);
      __syncthreads();
      item = *(volatile int*)smem;
      __syncthreads();
    }
    if (item >= J.total) break;
    // pick the job with static indices only (no dynamic indexing of kernel arguments)
    gdg_job_dev jb = J.job[0];
#pragma unroll
    for (int t = 1; t < kMaxJobs; ++t)
      if (t < J.n_jobs && item >= J.job[t].item0) jb = J.job[t];
    const long long shot = item - jb.item0;
    decode_shot<VPL, kLearn, kLow>(*jb.w, *jb.L, (int)shot, jb.syn, jb.syn_stride, jb.ehat, jb.pm,
                                   jb.flags, tr, J.learn, smem, J.lds, ck, J.ckpt_stride,
                                   J.warm_in ? J.warm_in + shot * J.warm_in_stride : nullptr,
                                   J.warm_out ? J.warm_out + shot * J.warm_out_stride : nullptr);
    __syncthreads();
    if (!J.work) item += gridDim.x;
  }
}

// The chained launch (gdg_decode_chain): the decode kernel's persistent loop
// over experiments instead of shots, each item one experiment's run of
// windows (decode_chain_item). A kernel of its own, so that the plain decode
// kernel keeps its registers and stack.
template <int VPL, bool kLow>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(
    kDecodeWavesPerSimd<VPL, false>, kDecodeWavesPerSimd<VPL, false>))) void gdg_chain_kernel(gdg_jobs_dev J, gdg_trace_dev tr) {
  extern __shared__ __align__(16) unsigned char smem[];
  char* const ck = J.ckpt && (int)blockIdx.x < J.ckpt_wgs
                       ? J.ckpt + (long long)blockIdx.x * J.ckpt_slots * J.ckpt_stride
                       : nullptr;
  int item = blockIdx.x;
  for (;;) {
    if (J.work) {
      if (threadIdx.x == 0) *(int*)smem = atomicAdd(J.work, 1);
      __syncthreads();
      item = *(volatile int*)smem;
      __syncthreads();
    }
    if (item >= J.total) break;
    decode_chain_item<VPL, kLow>(J.chain, item, tr, J.learn, smem, J.lds, ck, J.ckpt_stride);
    __syncthreads();
    if (!J.work) item += gridDim.x;
  }
}

// Scratch of gdg_decode_batch_noalloc, for callers that cannot allocate:
// the shot counter and as many workgroups' path checkpoints as fit. Each
// device holds its own copy until the process ends; calls on one device share
// it. Host code uses the address from hipGetSymbolAddress, never this name.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

__global__ void gdg_zero_kernel(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ------------------------------------------------------------------ plain BP

// gdg_bp: the decode kernel's whole-window BP (window_bp) with no early stop,
// one workgroup of four wavefronts per shot. LDS: the syndrome, then
// posteriors and messages at the host's offsets.
__global__ __launch_bounds__(256) void gdg_bp_kernel(gdg_win_dev w, int post_off, int c2v_off,
                                                     int n_shots,
                                                     const uint8_t* __restrict__ syn,
                                                     long long syn_stride, int n_iters,
                                                     float* __restrict__ post_out,
                                                     int* __restrict__ first_ok) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int shot = blockIdx.x;
  if (shot >= n_shots) return;
  uint8_t* s = smem;
  for (int j = threadIdx.x; j < w.m; j += blockDim.x) s[j] = syn[(long long)shot * syn_stride + j] & 1;
  __syncthreads();
  int done = 0;
  const int first = window_bp<1>(w, s, (float*)(smem + post_off), (float*)(smem + c2v_off), nullptr,
                                 n_iters, false, post_out + (long long)shot * n_iters * w.n, &done);
  if (threadIdx.x == 0) first_ok[shot] = first;
}

// ------------------------------------------------------------------ BP + OSD
//
// The window comparator of Sec. II-A (the OSD paragraph) and Sec. III: one
// workgroup per shot. The decode kernel's whole-window BP runs up to n_iters
// iterations and stops once its hard decision meets the syndrome (that is the
// answer). Otherwise the columns are ranked by posterior, ascending, ties by
// column (a bitonic sort of 48-bit keys); the first nk ranked columns become
// bit-columns over the rows; Gauss-Jordan elimination visits them in rank
// order and makes a column a pivot at its lowest row that is not a pivot row
// yet, adding that row to every other row where the column has a 1 (in column
// form: every column with a 1 at the pivot row gets the pivot column's other
// bits flipped). OSD-0 takes the information set's solution; the combination
// sweep also tries each single non-pivot column and each pair among the first
// lambda non-pivot columns. Costs are Eq. 5 sums in double: swept columns,
// then information-set columns by ascending pivot row. The least cost wins,
// ties to the earlier candidate (OSD-0, singles in rank order, pairs in
// lexicographic order).
constexpr int kOsdMaxWords = 16;   // rows <= 512

__global__ __launch_bounds__(256) void gdg_osd_kernel(gdg_win_dev w, gdg_osd_lds L, int n_shots,
                                                      const uint8_t* __restrict__ syn,
                                                      long long syn_stride, int n_iters, int cs,
                                                      int lambda, uint8_t* __restrict__ ehat,
                                                      double* __restrict__ pm_out,
                                                      int* __restrict__ flags_out,
                                                      int* __restrict__ order_out,
                                                      int* __restrict__ iters_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int shot = blockIdx.x;
  if (shot >= n_shots) return;
  const int tid = threadIdx.x, bs = blockDim.x, lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int m = w.m, n = w.n, nk = L.nk, MW = L.mw;
  uint8_t* s = smem + L.syn;
  uint16_t* order = (uint16_t*)(smem + L.order);
  uint16_t* rank_of = (uint16_t*)(smem + L.rank_of);
  uint32_t* obits = (uint32_t*)(smem + L.obits);
  uint32_t* sv = (uint32_t*)(smem + L.sv);
  int16_t* pcol = (int16_t*)(smem + L.pcol);      // [m] pivot (rank) column of each row, -1
  uint8_t* isp = smem + L.isp;                    // [nk] 1 = pivot column
  uint16_t* freec = (uint16_t*)(smem + L.freec);  // [nk] non-pivot kept columns in rank order
  unsigned long long* misc = (unsigned long long*)(smem + L.misc);   // [0] best cost, [1] best candidate
  float* post = (float*)(smem + L.post);
  float* c2v = (float*)(smem + L.c2v);
  unsigned long long* keys = (unsigned long long*)(smem + L.keys);
  uint32_t* mat = (uint32_t*)(smem + L.mat);
  double* stage = (double*)(smem + L.A);

  for (int j = tid; j < m; j += bs) s[j] = syn[(long long)shot * syn_stride + j] & 1;
  __syncthreads();
  int done = 0;
  const int first = window_bp<1>(w, s, post, c2v, nullptr, n_iters, true, nullptr, &done);
  if (tid == 0 && iters_out) iters_out[shot] = done;
  // the BP hard decision (the answer when BP converged or the syndrome is out of reach)
  for (int i = tid; i < L.obits_words; i += bs) obits[i] = 0u;
  __syncthreads();
  for (int base = wave * kWave; base < n; base += bs) {
    const int c = base + lane;
    const unsigned long long bal = __ballot(c < n && post[c] <= 0.0f);
    if (lane == 0) {
      obits[base >> 5] = (uint32_t)bal;
      obits[(base >> 5) + 1] = (uint32_t)(bal >> 32);
    }
  }
  __syncthreads();
  auto finish = [&](bool satisfied) {
    // Eq. 5 in ascending window-column order (wave 0), and the answer bytes
    __syncthreads();
    if (wave == 0) {
      const double pm = eq5_sum(obits, L.obits_words, w.llr64, stage, lane);
      if (lane == 0) {
        pm_out[shot] = satisfied ? pm : __builtin_inf();
        flags_out[shot] = satisfied ? 1 : 0;
      }
    }
    for (int c = tid; c < n; c += bs)
      ehat[(long long)shot * n + c] = (uint8_t)((obits[c >> 5] >> (c & 31)) & 1u);
  };
  if (first) {
    if (order_out)
      for (int c = tid; c < n; c += bs) order_out[(long long)shot * n + c] = -1;
    finish(true);
    return;
  }

  // ranking: keys ord(posterior) << 16 | column, sorted ascending (the keys
  // overwrite the posteriors: read first)
  constexpr int kKeysPerThread = 16;   // sort sizes up to 4096 with 256 threads
  const int P2 = L.sort_p;
  unsigned long long kr[kKeysPerThread];
#pragma unroll
  for (int q = 0; q < kKeysPerThread; ++q) {
    const int i = tid + q * bs;
    kr[q] = i < n ? (((unsigned long long)ord_f32(post[i]) << 16) | (unsigned)i) : ~0ull;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kKeysPerThread; ++q) {
    const int i = tid + q * bs;
    if (i < P2) keys[i] = kr[q];
  }
  __syncthreads();
  wg_bitonic_sort(keys, P2);
  for (int i = tid; i < n; i += bs) {
    const int c = (int)(keys[i] & 0xffffu);
    order[i] = (uint16_t)c;
    rank_of[c] = (uint16_t)i;
    if (order_out) order_out[(long long)shot * n + i] = c;
  }
  __syncthreads();

  // bit-columns of the kept columns (rank order) and the syndrome
  for (int i = tid; i < nk * MW; i += bs) mat[i] = 0u;
  for (int r = tid; r < m; r += bs) pcol[r] = -1;
  for (int i = tid; i < nk; i += bs) isp[i] = 0;
  if (tid < MW) {
    uint32_t x = 0u;
    for (int b = 0; b < 32 && 32 * tid + b < m; ++b) x |= (uint32_t)s[32 * tid + b] << b;
    sv[tid] = x;
  }
  __syncthreads();
  for (int r = tid; r < m; r += bs)
    for (int e = w.row_ptr[r]; e < w.row_ptr[r + 1]; ++e) {
      const int i = rank_of[w.row_col[e]];
      if (i < nk) atomicOr(&mat[i * MW + (r >> 5)], 1u << (r & 31));
    }
  __syncthreads();

  // Gauss-Jordan in rank order
  uint32_t used[kOsdMaxWords];
#pragma unroll
  for (int q = 0; q < kOsdMaxWords; ++q) used[q] = 0u;
  int np = 0;
  for (int i = 0; i < nk && np < m; ++i) {
    int r = -1;
#pragma unroll
    for (int q = 0; q < kOsdMaxWords; ++q) {
      if (q >= MW) break;
      const uint32_t x = mat[i * MW + q] & ~used[q];
      if (x && r < 0) r = 32 * q + __builtin_ctz(x);
    }
    r = __builtin_amdgcn_readfirstlane(r);
    if (r < 0) continue;
    uint32_t oth[kOsdMaxWords];
#pragma unroll
    for (int q = 0; q < kOsdMaxWords; ++q) oth[q] = q < MW ? mat[i * MW + q] : 0u;
    const int rw = r >> 5;
    const uint32_t rb = 1u << (r & 31);
#pragma unroll
    for (int q = 0; q < kOsdMaxWords; ++q)
      if (q == rw) oth[q] &= ~rb;
    __syncthreads();   // every thread has read column i
    for (int j = tid; j < nk; j += bs) {
      uint32_t* cj = mat + j * MW;
      if (cj[rw] & rb) {
#pragma unroll
        for (int q = 0; q < kOsdMaxWords; ++q)
          if (q < MW) cj[q] ^= oth[q];
      }
    }
    if (tid == 0) {
      if (sv[rw] & rb) {
#pragma unroll
        for (int q = 0; q < kOsdMaxWords; ++q)
          if (q < MW) sv[q] ^= oth[q];
      }
      pcol[r] = (int16_t)i;
      isp[i] = 1;
    }
#pragma unroll
    for (int q = 0; q < kOsdMaxWords; ++q)
      if (q == rw) used[q] |= rb;
    ++np;
    __syncthreads();
  }
  // the syndrome must lie in the span of the kept columns
  bool out_of_span = false;
#pragma unroll
  for (int q = 0; q < kOsdMaxWords; ++q)
    if (q < MW && (sv[q] & ~used[q])) out_of_span = true;
  if (out_of_span) {
    finish(false);
    return;
  }
  // non-pivot kept columns in rank order (wave 0, ballots)
  if (wave == 0) {
    int cnt = 0;
    for (int base = 0; base < nk; base += kWave) {
      const int i = base + lane;
      const bool f = i < nk && !isp[i];
      const unsigned long long bal = __ballot(f);
      if (f) freec[cnt + __builtin_popcountll(bal & ((1ull << lane) - 1ull))] = (uint16_t)i;
      cnt += __builtin_popcountll(bal);
    }
    if (lane == 0) {
      misc[0] = ~0ull;
      misc[1] = ~0ull;
      misc[2] = (unsigned long long)cnt;
    }
  }
  __syncthreads();
  const int n_free = (int)misc[2];
  const int L2 = cs ? min(lambda, n_free) : 0;
  const int n_cand = 1 + (cs ? n_free : 0) + L2 * (L2 - 1) / 2;
  auto cand_cols = [&](int cand, int& j1, int& j2) {
    j1 = -1;
    j2 = -1;
    if (cand == 0) return;
    if (cand <= n_free) {
      j1 = freec[cand - 1];
      return;
    }
    int k = cand - 1 - n_free;   // pair index, lexicographic over a < b < L2
    int a = 0;
    while (k >= L2 - 1 - a) {
      k -= L2 - 1 - a;
      ++a;
    }
    j1 = freec[a];
    j2 = freec[a + 1 + k];
  };
  auto solution = [&](int j1, int j2, uint32_t (&u)[kOsdMaxWords]) {
#pragma unroll
    for (int q = 0; q < kOsdMaxWords; ++q) {
      uint32_t x = q < MW ? sv[q] : 0u;
      if (q < MW && j1 >= 0) x ^= mat[j1 * MW + q];
      if (q < MW && j2 >= 0) x ^= mat[j2 * MW + q];
      u[q] = x & used[q];
    }
  };
  unsigned long long my_cost = ~0ull, my_cand = ~0ull;
  for (int cand = tid; cand < n_cand; cand += bs) {
    int j1, j2;
    cand_cols(cand, j1, j2);
    uint32_t u[kOsdMaxWords];
    solution(j1, j2, u);
    double cost = 0.0;
    if (j1 >= 0) cost += w.llr64[order[j1]];
    if (j2 >= 0) cost += w.llr64[order[j2]];
#pragma unroll
    for (int q = 0; q < kOsdMaxWords; ++q) {
      uint32_t x = u[q];
      while (x) {
        const int r = 32 * q + __builtin_ctz(x);
        x &= x - 1u;
        cost += w.llr64[order[pcol[r]]];
      }
    }
    const unsigned long long cb = (unsigned long long)__double_as_longlong(cost);
    if (cb < my_cost || (cb == my_cost && (unsigned long long)cand < my_cand)) {
      my_cost = cb;
      my_cand = (unsigned long long)cand;
    }
  }
  atomicMin(&misc[0], my_cost);
  __syncthreads();
  if (my_cost == misc[0]) atomicMin(&misc[1], my_cand);
  __syncthreads();
  // the winner's answer bits (one thread), then its Eq. 5 metric
  if (tid == 0) {
    for (int i = 0; i < L.obits_words; ++i) obits[i] = 0u;
    int j1, j2;
    cand_cols((int)misc[1], j1, j2);
    uint32_t u[kOsdMaxWords];
    solution(j1, j2, u);
    auto set = [&](int c) { obits[c >> 5] |= 1u << (c & 31); };
    if (j1 >= 0) set(order[j1]);
    if (j2 >= 0) set(order[j2]);
#pragma unroll
    for (int q = 0; q < kOsdMaxWords; ++q) {
      uint32_t x = u[q];
      while (x) {
        const int r = 32 * q + __builtin_ctz(x);
        x &= x - 1u;
        set(order[pcol[r]]);
      }
    }
  }
  finish(true);
}

// ------------------------------------------------------------------ commit

// Folds a window's committed correction into the later rows and the
// observables of each shot (a workgroup per few shots). Shot s's row r lives
// at det[s * det_stride + r] and observable o at obs[s * obs_stride + o]; with
// per-shot offsets (det_off non-null) at det[det_off[s] + r - row0] and
// obs[obs_off[s] + o] instead.
__global__ __launch_bounds__(256) void gdg_commit_kernel(
    gdg_commit_dev cm, int n_shots, int spw, const uint8_t* __restrict__ ehat,
    uint8_t* __restrict__ det, long long det_stride, uint8_t* __restrict__ obs,
    long long obs_stride, const long long* __restrict__ det_off,
    const long long* __restrict__ obs_off, int row0) {
  // spw <= 8 shots per workgroup: their corrections are staged in LDS
  // transposed, bit q of es[c] holding column c of shot s0 + q (coalesced
  // loads of four columns of each shot at a time), then each thread folds
  // whole rows / observables for all of them with one LDS byte per column
  // (one read of the row's column list serves every shot)
  extern __shared__ __align__(16) unsigned char es[];
  const int s0 = blockIdx.x * spw;
  const int ns = min(spw, n_shots - s0);
  if (ns <= 0) return;
  if ((cm.n_win & 3) == 0 && (((uintptr_t)ehat) & 3) == 0) {
    const int n4 = cm.n_win / 4;
    for (int c = threadIdx.x; c < n4; c += blockDim.x) {
      uint32_t x = 0u;
      for (int q = 0; q < ns; ++q)
        x |= (((const uint32_t*)(ehat + (long long)(s0 + q) * cm.n_win))[c] & 0x01010101u) << q;
      ((uint32_t*)es)[c] = x;
    }
  } else {
    for (int c = threadIdx.x; c < cm.n_win; c += blockDim.x) {
      uint32_t x = 0u;
      for (int q = 0; q < ns; ++q)
        x |= (uint32_t)(ehat[(long long)(s0 + q) * cm.n_win + c] & 1u) << q;
      es[c] = (uint8_t)x;
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < cm.n_rows + cm.n_obs; r += blockDim.x) {
    const bool is_row = r < cm.n_rows;
    const int o = r - cm.n_rows;
    const int t0 = is_row ? cm.row_ptr[r] : cm.obs_ptr[o];
    const int t1 = is_row ? cm.row_ptr[r + 1] : cm.obs_ptr[o + 1];
    const int* cols = is_row ? cm.row_col : cm.obs_col;
    uint32_t xm = 0u;   // bit q: the parity for shot s0 + q
    for (int t = t0; t < t1; ++t) xm ^= es[cols[t]];
    for (int q = 0; q < ns; ++q) {
      if (!((xm >> q) & 1u)) continue;
      const int shot = s0 + q;
      if (is_row) {
        const long long at = det_off ? det_off[shot] + (cm.row_global[r] - row0)
                                     : (long long)shot * det_stride + cm.row_global[r];
        det[at] ^= 1;
      } else {
        obs[(obs_off ? obs_off[shot] : (long long)shot * obs_stride) + o] ^= 1;
      }
    }
  }
}

// Row copies at per-row offsets: dst[dst_off[i] + j] = src[src_off[i] + j], j < m
// (dst_off null: dst[i * m + j]).
__global__ void gdg_copy_rows_kernel(int n, int m, const uint8_t* __restrict__ src,
                                     const long long* __restrict__ src_off,
                                     uint8_t* __restrict__ dst,
                                     const long long* __restrict__ dst_off) {
  const int i = blockIdx.x;
  if (i >= n) return;
  const long long s = src_off[i];
  const long long d = dst_off ? dst_off[i] : (long long)i * m;
  for (int j = threadIdx.x; j < m; j += blockDim.x) dst[d + j] = src[s + j];
}

// ------------------------------------------------------------------ sampler
//
// Philox4x32-10 (Salmon et al., SC'11): ten rounds, each two 32x32 -> 64-bit
// products with the multipliers 0xD2511F53 / 0xCD9E8D57, key bumped by the
// Weyl constants 0x9E3779B9 / 0xBB67AE85 between rounds.

__device__ __forceinline__ void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// One workgroup per shot; detector and observable bits accumulate in LDS.
__global__ __launch_bounds__(256) void gdg_sample_kernel(gdg_dem_dev_k d, int n_shots, uint64_t seed,
                                                         uint32_t stream, uint64_t shot0,
                                                         uint8_t* __restrict__ det,
                                                         uint8_t* __restrict__ obs) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int s = blockIdx.x;
  if (s >= n_shots) return;
  uint32_t* dbits = (uint32_t*)smem;
  const int dw = (d.n_rows + 31) >> 5;
  uint32_t* obits = dbits + dw;
  const int ow = (d.n_obs + 31) >> 5;
  for (int i = threadIdx.x; i < dw + ow; i += blockDim.x) dbits[i] = 0u;
  __syncthreads();
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const uint32_t sh = (uint32_t)(shot0 + (uint64_t)s);
  const int ngroups = (d.n_cols + 3) >> 2;
  for (int gq = threadIdx.x; gq < ngroups; gq += blockDim.x) {
    uint32_t c[4] = {(uint32_t)gq, sh, stream, 0xC0DEu};
    philox(c, k0, k1);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int col = gq * 4 + t;
      if (col < d.n_cols && c[t] < d.thr[col]) {
        for (int e = d.h_ptr[col]; e < d.h_ptr[col + 1]; ++e) {
          const int r = d.h_idx[e];
          atomicXor(&dbits[r >> 5], 1u << (r & 31));
        }
        for (int e = d.l_ptr[col]; e < d.l_ptr[col + 1]; ++e) {
          const int o = d.l_idx[e];
          atomicXor(&obits[o >> 5], 1u << (o & 31));
        }
      }
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < d.n_rows; r += blockDim.x)
    det[(long long)s * d.n_rows + r] = (uint8_t)((dbits[r >> 5] >> (r & 31)) & 1u);
  for (int o = threadIdx.x; o < d.n_obs; o += blockDim.x)
    obs[(long long)s * d.n_obs + o] = (uint8_t)((obits[o >> 5] >> (o & 31)) & 1u);
}

// The error vectors themselves: err[s][c] = 1 iff column c fired in shot s
// (the same Philox words as gdg_sample_kernel).
__global__ __launch_bounds__(256) void gdg_sample_err_kernel(gdg_dem_dev_k d, int n_shots,
                                                             uint64_t seed, uint32_t stream,
                                                             uint64_t shot0,
                                                             uint8_t* __restrict__ err) {
  const int s = blockIdx.x;
  if (s >= n_shots) return;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const uint32_t sh = (uint32_t)(shot0 + (uint64_t)s);
  const int ngroups = (d.n_cols + 3) >> 2;
  for (int gq = threadIdx.x; gq < ngroups; gq += blockDim.x) {
    uint32_t c[4] = {(uint32_t)gq, sh, stream, 0xC0DEu};
    philox(c, k0, k1);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int col = gq * 4 + t;
      if (col < d.n_cols) err[(long long)s * d.n_cols + col] = c[t] < d.thr[col] ? 1 : 0;
    }
  }
}

__global__ void gdg_evaluate_kernel(int n_shots, int n_rows, int n_obs,
                                    const uint8_t* __restrict__ det, const uint8_t* __restrict__ obs,
                                    uint8_t* __restrict__ fail) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_shots) return;
  int bad = 0;
  for (int r = 0; r < n_rows; ++r) bad |= det[(long long)s * n_rows + r];
  for (int o = 0; o < n_obs; ++o) bad |= obs[(long long)s * n_obs + o];
  fail[s] = (uint8_t)(bad != 0);
}

}  // namespace

// ------------------------------------------------------------------ launchers

// Register tilings of the decode kernel: VNs per lane of each bucket.
#define GDG_DECODE_TILINGS(X) X(6) X(7) X(8) X(14) X(16)
constexpr int kBuckets = 5;

hipError_t gdg_static_scratch(void** ptr, size_t* bytes) {
  static std::mutex mu;
  static std::vector<void*> addr;   // per device, looked up once with that device current
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  *bytes = kStaticScratchBytes;
  return hipSuccess;
}

hipError_t gdg_launch_zero(int* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(gdg_zero_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t gdg_launch_jobs(const gdg_jobs_dev& J, int bucket, bool low, int waves, int grid,
                           int lds, const gdg_trace_dev& tr, hipStream_t st) {
  dim3 g(grid), block(waves * kWave);
  const bool learn = J.learn.mode != 0;
  int b = 0;
#define GDG_LAUNCH(V)                                                                      \
  if (b++ == bucket) {                                                                     \
    if (learn && low)                                                                      \
      hipLaunchKernelGGL((gdg_decode_kernel<V, true, true>), g, block, lds, st, J, tr);    \
    else if (learn)                                                                        \
      hipLaunchKernelGGL((gdg_decode_kernel<V, true, false>), g, block, lds, st, J, tr);   \
    else if (low)                                                                          \
      hipLaunchKernelGGL((gdg_decode_kernel<V, false, true>), g, block, lds, st, J, tr);   \
    else                                                                                   \
      hipLaunchKernelGGL((gdg_decode_kernel<V, false, false>), g, block, lds, st, J, tr);  \
    return hipGetLastError();                                                              \
  }
  GDG_DECODE_TILINGS(GDG_LAUNCH)
#undef GDG_LAUNCH
  return hipErrorInvalidValue;
}

hipError_t gdg_launch_chain(const gdg_jobs_dev& J, int bucket, bool low, int waves, int grid,
                            int lds, hipStream_t st) {
  dim3 g(grid), block(waves * kWave);
  gdg_trace_dev tr{};
  int b = 0;
#define GDG_LAUNCH(V)                                                                    \
  if (b++ == bucket) {                                                                   \
    const void* f = low ? (const void*)gdg_chain_kernel<V, true>                         \
                        : (const void*)gdg_chain_kernel<V, false>;                       \
    if (lds > 65536) {                                                                   \
      const hipError_t e =                                                               \
          hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);       \
      if (e != hipSuccess) return e;                                                     \
    }                                                                                    \
    if (low)                                                                             \
      hipLaunchKernelGGL((gdg_chain_kernel<V, true>), g, block, lds, st, J, tr);         \
    else                                                                                 \
      hipLaunchKernelGGL((gdg_chain_kernel<V, false>), g, block, lds, st, J, tr);        \
    return hipGetLastError();                                                            \
  }
  GDG_DECODE_TILINGS(GDG_LAUNCH)
#undef GDG_LAUNCH
  return hipErrorInvalidValue;
}

int gdg_decode_waves_per_simd(int bucket, bool learn) {
  int b = 0, r = 2;
#define GDG_WPS(V) \
  if (b++ == bucket) r = learn ? kDecodeWavesPerSimd<V, true> : kDecodeWavesPerSimd<V, false>;
  GDG_DECODE_TILINGS(GDG_WPS)
#undef GDG_WPS
  return r;
}

int gdg_kernel_bucket(int m, int n_act) {
  if (m > 1023) return -1;
  if (n_act <= 384) return 0;
  if (n_act <= 448) return 1;
  if (n_act <= 512) return 2;
  if (n_act <= 896) return 3;
  if (n_act <= 1024) return 4;
  return -1;
}

hipError_t gdg_decode_set_lds_limit(int bucket, int bytes) {
  static const void* const fs[3 * kBuckets] = {
#define GDG_FN(V)                                                                           \
  (const void*)gdg_decode_kernel<V, false, false>, (const void*)gdg_decode_kernel<V, true, false>, \
      (const void*)gdg_decode_kernel<V, false, true>,
      GDG_DECODE_TILINGS(GDG_FN)
#undef GDG_FN
  };
  if (bucket < 0 || bucket >= kBuckets) return hipErrorInvalidValue;
  for (int l = 0; l < 3; ++l) {
    const hipError_t e =
        hipFuncSetAttribute(fs[bucket * 3 + l], hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t gdg_launch_bp(const gdg_win_dev& w, int n_shots, const uint8_t* syn, long long stride,
                         int n_iters, float* post, int* first_ok, hipStream_t st) {
  const int post_off = gdg_align16(w.m);
  const int c2v_off = post_off + gdg_align16(4 * (w.n + 1));
  const size_t lds = (size_t)c2v_off + 4 * (size_t)(w.fr_epad + 2 * kPad);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)gdg_bp_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(gdg_bp_kernel, dim3(n_shots), dim3(4 * kWave), lds, st, w, post_off, c2v_off,
                     n_shots, syn, stride, n_iters, post, first_ok);
  return hipGetLastError();
}

hipError_t gdg_launch_osd(const gdg_win_dev& w, const gdg_osd_lds& L, int n_shots,
                          const uint8_t* syn, long long syn_stride, int n_iters, int cs,
                          int lambda, uint8_t* ehat, double* pm, int* flags, int* order,
                          int* iters, hipStream_t st) {
  if (L.total > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)gdg_osd_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, L.total);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(gdg_osd_kernel, dim3(n_shots), dim3(4 * kWave), L.total, st, w, L, n_shots,
                     syn, syn_stride, n_iters, cs, lambda, ehat, pm, flags, order, iters);
  return hipGetLastError();
}

hipError_t gdg_launch_commit(const gdg_commit_dev& cm, int n_shots, const uint8_t* ehat,
                             uint8_t* det, long long det_stride, uint8_t* obs,
                             long long obs_stride, const long long* det_off,
                             const long long* obs_off, int row0, hipStream_t st) {
  if (n_shots <= 0 || cm.n_rows + cm.n_obs == 0) return hipSuccess;
  // 8 shots per workgroup, one staged byte per window column (a window has
  // at most 65535 columns: within the default LDS limit)
  const size_t nw = ((size_t)cm.n_win + 15) & ~(size_t)15;
  const int spw = 8;
  const unsigned nb = (unsigned)((n_shots + spw - 1) / spw);
  hipLaunchKernelGGL(gdg_commit_kernel, dim3(nb), dim3(256), nw, st, cm, n_shots,
                     spw, ehat, det, det_stride, obs, obs_stride, det_off, obs_off, row0);
  return hipGetLastError();
}

hipError_t gdg_launch_copy_rows(int n, int m, const uint8_t* src, const long long* src_off,
                                uint8_t* dst, const long long* dst_off, hipStream_t st) {
  hipLaunchKernelGGL(gdg_copy_rows_kernel, dim3((unsigned)n), dim3(m >= 256 ? 256 : 64), 0, st, n,
                     m, src, src_off, dst, dst_off);
  return hipGetLastError();
}

hipError_t gdg_launch_sample(const gdg_dem_dev_k& d, int n_shots, uint64_t seed, uint32_t stream,
                             uint64_t shot0, uint8_t* det, uint8_t* obs, hipStream_t st) {
  const size_t lds = 4 * (size_t)(((d.n_rows + 31) >> 5) + ((d.n_obs + 31) >> 5));
  hipLaunchKernelGGL(gdg_sample_kernel, dim3(n_shots), dim3(256), lds, st, d, n_shots, seed,
                     stream, shot0, det, obs);
  return hipGetLastError();
}

hipError_t gdg_launch_sample_errors(const gdg_dem_dev_k& d, int n_shots, uint64_t seed,
                                    uint32_t stream, uint64_t shot0, uint8_t* err,
                                    hipStream_t st) {
  hipLaunchKernelGGL(gdg_sample_err_kernel, dim3(n_shots), dim3(256), 0, st, d, n_shots, seed,
                     stream, shot0, err);
  return hipGetLastError();
}

hipError_t gdg_launch_evaluate(int n_shots, int n_rows, int n_obs, const uint8_t* det,
                               const uint8_t* obs, uint8_t* fail, hipStream_t st) {
  const int bs = 256;
  hipLaunchKernelGGL(gdg_evaluate_kernel, dim3((n_shots + bs - 1) / bs), dim3(bs), 0, st, n_shots,
                     n_rows, n_obs, det, obs, fail);
  return hipGetLastError();
}
