// Wave-level building blocks of the combinatorial track builders (sections
// 4.3: fixed candidate slots per seed, ranked children): lane shuffles,
// reductions over a seed's slots, the 64-bit rank key of a child, a lane's
// list of its best accepted hits in LDS, wave prefix sums, and the per-call
// preparation kernels shared by the builders (queue reset, fine phi index of
// the binned hits, packed hit copy) with the layout of their workspace.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kfhost.h"

namespace {

constexpr uint64_t kInfKey = ~0ull;
constexpr uint32_t kHoleIdx = 0xFFFFFFu;
constexpr int kMaxOrig = (1 << 24) - 2;

// Event-local hit indices are 24 bits wide (0xFFFFFF marks a hole): an event
// with more than kMaxOrig + 1 binned hits cannot be built.
__device__ inline bool event_too_large(const int32_t* offsets, int ev, int n_layers, int nb) {
  const int32_t* eo = offsets + (size_t)ev * n_layers * (nb + 1);
  return eo[(size_t)(n_layers - 1) * (nb + 1) + nb] - eo[0] > kMaxOrig + 1;
}

template <typename T> __device__ inline T shfl(T v, int src) { return __shfl(v, src, 64); }
__device__ inline uint64_t shfl_u64(uint64_t v, int src) {
  uint32_t lo = __shfl((uint32_t)v, src, 64), hi = __shfl((uint32_t)(v >> 32), src, 64);
  return ((uint64_t)hi << 32) | lo;
}
__device__ inline double shfl_d(double v, int src) {
  uint64_t b = __double_as_longlong(v);
  return __longlong_as_double((long long)shfl_u64(b, src));
}
__device__ inline float shfl_t(float v, int src) { return __shfl(v, src, 64); }
// value of lane j (j uniform across the wave)
__device__ inline float readlane_t(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}
__device__ inline double readlane_t(double v, int j) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, j);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), j);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ inline double shfl_t(double v, int src) { return shfl_d(v, src); }

// The minimum over the S lanes base .. base+S-1 of one seed (S <= 8, any
// value), doubling a rotation: after the steps 1, 2, 4 a lane
// has seen the slots slot .. slot+7 (mod S), which covers the group.  Lanes
// that hold no seed (used = false) only ever read themselves.
__device__ inline int rot_lane(int base, int slot, int d, int S, bool used) {
  const int t = slot + d;
  return used ? base + (t >= S ? t - S : t) : base + slot;
}
__device__ inline uint64_t group_min(uint64_t k, int base, int slot, int S, bool used) {
  for (int d = 1; d < S; d <<= 1) {
    const uint64_t o = shfl_u64(k, rot_lane(base, slot, d, S, used));
    k = o < k ? o : k;
  }
  return k;
}

__device__ inline uint32_t chi2_bits(float c) {
  c = c > 0.f ? c : 0.f;  // chi2 >= 0; clears a negative rounding residue and -0
  return __float_as_uint(c);
}

// rank key: nhits desc, chi2 asc, parent slot asc, hit index asc (hole last)
__device__ inline uint64_t make_key(int nhits, float chi2, int slot, uint32_t orig24) {
  return ((uint64_t)(31 - nhits) << 59) | ((uint64_t)chi2_bits(chi2) << 27) | ((uint64_t)slot << 24) | orig24;
}

__device__ inline float wrap_2pi(float p) {
  const float tp = 6.283185307179586f;
  if (p < 0.f) p += tp;
  if (p >= tp) p -= tp;
  return p;
}

// Fine phi index of a z row: key(phi) = the sub-bin of a stored phi, with
// n_phi * refine sub-bins over [0, 2 pi).  The stored phi of a row is
// non-decreasing along the sorted order (hits are sorted by bin, then phi,
// and rounding to FP32 keeps the order of the FP64 phi that set the bin), so
// key is non-decreasing too and fine[j] = first position with key >= j
// brackets every hit whose stored phi lies in an interval.
__host__ __device__ inline int fine_key(float phi, float inv, int nf) {
  const float t = floorf(phi * inv);
  const int k = t > 0.f ? (int)t : 0;  // also maps NaN to 0
  return k < nf - 1 ? k : nf - 1;
}
__host__ __device__ inline float fine_inv(int nf) { return (float)nf / 6.283185307179586f; }

// A lane's accepted hits, best first (chi2 ascending, hit index ascending),
// at most cap of them.  The entries live in LDS, [cap][64] per wave, so that
// the list costs no registers; this lane's column starts at c2 / pos / orig.
// chi2 is kept in FP32 (the hit search computes it in FP32, see coop_scan).
struct TopList {
  float* c2;
  int32_t* pos;
  uint32_t* orig;
  int n;    // entries held (<= cap)
  int tot;  // accepted hits seen
  int scanned, tested;  // work counters of the hits this lane examined
};

__device__ inline bool top_before(float c2, uint32_t orig, float oc2, uint32_t oorig) {
  return c2 < oc2 || (c2 == oc2 && orig < oorig);
}

// Lanes lo .. hi-1 of a wave as a mask (0 <= lo <= 63, hi <= 64).
__device__ inline unsigned long long run_mask(int lo, int hi) {
  const unsigned long long up = hi >= 64 ? ~0ull : ((1ull << hi) - 1ull);
  return up & ~((1ull << lo) - 1ull);
}

// Sorts the first n entries of this lane's list by (chi2, hit index): the
// entries go through registers and a sorting network for N (positions from
// n on, and from cap on, as +inf): N = 4 (5 comparators), 6 (12, depth 5)
// or 8 (Batcher's odd-even merge, 19), the smallest that holds cap.
template <int N> struct SortNet;
template <> struct SortNet<4> {
  static constexpr int len = 5;
  static constexpr int c[5][2] = {{0, 1}, {2, 3}, {0, 2}, {1, 3}, {1, 2}};
};
template <> struct SortNet<6> {
  static constexpr int len = 12;
  static constexpr int c[12][2] = {{0, 5}, {1, 3}, {2, 4}, {1, 2}, {3, 4}, {0, 3},
                                   {2, 5}, {0, 1}, {2, 3}, {4, 5}, {1, 2}, {3, 4}};
};
template <> struct SortNet<8> {
  static constexpr int len = 19;
  static constexpr int c[19][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3}, {4, 6}, {5, 7}, {1, 2}, {5, 6},
                                   {0, 4}, {1, 5}, {2, 6}, {3, 7}, {2, 4}, {3, 5}, {1, 2}, {3, 4}, {5, 6}};
};
template <int N>
__device__ inline void sort_net(TopList& tl, int cap, int n) {
  float v[N];
  uint32_t o[N];
  int32_t q[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (k < cap) {
      v[k] = tl.c2[k * 64];
      o[k] = tl.orig[k * 64];
      q[k] = tl.pos[k * 64];
    }
  }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (!(k < n && k < cap)) {
      v[k] = __builtin_inff();
      o[k] = 0xFFFFFFFFu;
      q[k] = 0;
    }
  }
#pragma unroll
  for (int t = 0; t < SortNet<N>::len; ++t) {
    const int a = SortNet<N>::c[t][0], b = SortNet<N>::c[t][1];
    const bool sw = top_before(v[b], o[b], v[a], o[a]);
    const float tv = v[a];
    const uint32_t to = o[a];
    const int32_t tq = q[a];
    v[a] = sw ? v[b] : v[a];
    o[a] = sw ? o[b] : o[a];
    q[a] = sw ? q[b] : q[a];
    v[b] = sw ? tv : v[b];
    o[b] = sw ? to : o[b];
    q[b] = sw ? tq : q[b];
  }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (k < n && k < cap) {
      tl.c2[k * 64] = v[k];
      tl.orig[k * 64] = o[k];
      tl.pos[k * 64] = q[k];
    }
  }
}
__device__ inline void sort_own(TopList& tl, int cap, int n) {
  if (cap <= 4) sort_net<4>(tl, cap, n);
  else if (cap <= 6) sort_net<6>(tl, cap, n);
  else sort_net<8>(tl, cap, n);
}

// One round's admissible hits into their candidates' lists, all at once.
//
// In a round of the cooperative hit search every lane holds one
// (candidate, hit) pair, and the pairs of a candidate occupy a run of
// consecutive lanes.  The new list of a candidate is the best cap of its
// held entries and its admissible hits of the round.
//
// Where they all fit (held + admissible <= cap) the hits are appended, each
// at held plus its index among the run's admissible lanes, and the list is
// marked unsorted; a list that fills up this way is sorted at once (its
// last entry is the admission threshold), and the caller sorts the others
// at the end of the search.  Where they do not, the hits are ranked in
// parallel against the (sorted) held entries: a hit's place is the number
// of held entries that rank before it plus the number of the round's other
// admissible hits of the candidate that rank before it (read from a
// per-wave buffer the lanes publish to); a held entry moves down by the
// number of new hits whose place among the held entries is at or before
// its own (one ballot per list position); places at or past cap drop out.
// The ranking is a total order, so the lists equal those of inserting the
// hits one at a time.
//
//   keep, c2, pos, orig   this lane's pair (keep: admissible) and its hit
//   c, rlo, rhi           the pair's candidate lane and its run [rlo, rhi)
//   s0, e0                this lane's own run as a candidate (empty if s0 >= e0)
//   m                     ballot of keep (nonzero)
//   held, unsorted        this lane's list: entries, and whether they are out of order
//   thr_c2, thr_o         its admission threshold (its last entry once full)
//   pub_c2, pub_o         the wave's publish buffer, 64 entries each
__device__ inline void round_insert(TopList& tl, int cap, int lane, unsigned long long m, bool keep, float c2,
                                    int pos, uint32_t orig, int c, int rlo, int rhi, int s0, int e0, int& held,
                                    bool& unsorted, float& thr_c2, uint32_t& thr_o, float* pub_c2, uint32_t* pub_o) {
  float* wc2 = tl.c2 - lane;
  int32_t* wpos = tl.pos - lane;
  uint32_t* wor = tl.orig - lane;
  // the pair's candidate: entries held, admissible hits in the run
  const int hc = __shfl(held, c, 64);
  const unsigned long long runm = m & run_mask(rlo, rhi);
  const bool app = keep && hc + __builtin_popcountll(runm) <= cap;
  // this lane as a candidate
  const unsigned long long own = s0 < e0 ? run_mask(s0, e0) : 0ull;
  const int na = __builtin_popcountll(m & own);
  const bool ovf = na > 0 && held + na > cap;
  if (app) {
    const int idx = hc + __builtin_popcountll(runm & ((1ull << lane) - 1ull));
    wc2[idx * 64 + c] = c2;
    wpos[idx * 64 + c] = pos;
    wor[idx * 64 + c] = orig;
  }
  if (__any(ovf)) {
    if (ovf && unsorted) {
      sort_own(tl, cap, held);
      unsorted = false;
    }
    const bool rk = keep && !app;  // hits of overflowing candidates
    if (rk) {
      pub_c2[lane] = c2;
      pub_o[lane] = orig;
    }
    asm volatile("" ::: "memory");
    // place among the candidate's held entries
    int rl = 0;
    if (rk) {
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (k < hc) rl += top_before(wc2[k * 64 + c], wor[k * 64 + c], c2, orig) ? 1 : 0;
    }
    // place among the round's admissible hits of the same candidate
    int rank = rl;
    unsigned long long M = rk ? (runm & ~(1ull << lane)) : 0ull;
    while (__any(M != 0ull)) {
      int j[4];
      bool v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        v[u] = M != 0ull;
        j[u] = v[u] ? (int)__builtin_ctzll(M) : lane;
        M &= M - 1ull;
      }
      float sc[4];
      uint32_t so[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        sc[u] = pub_c2[j[u]];
        so[u] = pub_o[j[u]];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) rank += (v[u] && top_before(sc[u], so[u], c2, orig)) ? 1 : 0;
    }
    // held entries move down past the new hits before them
    int sh[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) sh[k] = k < cap ? __builtin_popcountll(__ballot(rk && rl <= k) & own) : 0;
    if (ovf) {
      float ec[8];
      int32_t ep[8];
      uint32_t eo[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (k < held && sh[k] > 0 && k + sh[k] < cap) {
          ec[k] = tl.c2[k * 64];
          ep[k] = tl.pos[k * 64];
          eo[k] = tl.orig[k * 64];
        }
      }
#pragma unroll
      for (int k = 7; k >= 0; --k) {
        if (k < held && sh[k] > 0 && k + sh[k] < cap) {
          tl.c2[(k + sh[k]) * 64] = ec[k];
          tl.pos[(k + sh[k]) * 64] = ep[k];
          tl.orig[(k + sh[k]) * 64] = eo[k];
        }
      }
    }
    asm volatile("" ::: "memory");
    if (rk && rank < cap) {
      wc2[rank * 64 + c] = c2;
      wpos[rank * 64 + c] = pos;
      wor[rank * 64 + c] = orig;
    }
  }
  asm volatile("" ::: "memory");
  if (na > 0) {
    if (ovf) {
      held = cap;
    } else {
      held += na;
      unsorted = true;
      if (held == cap) {
        sort_own(tl, cap, held);
        unsorted = false;
      }
    }
    if (held == cap) {
      thr_c2 = tl.c2[(cap - 1) * 64];
      thr_o = tl.orig[(cap - 1) * 64];
    }
  }
}

__device__ inline void top_get(const TopList& tl, int k, float& c2, int& pos, uint32_t& orig) {
  c2 = tl.c2[k * 64];
  pos = tl.pos[k * 64];
  orig = tl.orig[k * 64];
}

// Wave-wide inclusive prefix sum; returns the exclusive prefix, total via ref.
// Wave-wide scans and reductions with DPP row operations (a lane reads a
// neighbour's register through the VALU's data-parallel primitives, a few
// cycles, where a shuffle goes through the LDS crossbar): shifts by 1, 2, 4,
// 8 inside each row of 16 lanes, then lane 15 of a row into the next row and
// lane 31 into rows 2 and 3.  A lane whose source lies outside its row keeps
// the identity (`old`).
template <int CTRL, int ROWS>
__device__ inline int dpp_or(int old, int x) {
  return __builtin_amdgcn_update_dpp(old, x, CTRL, ROWS, 0xf, false);
}
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;

// Wave-wide inclusive prefix sum; returns the exclusive prefix, total via ref.
__device__ inline int wave_excl_scan(int v, int lane, int& total) {
  (void)lane;
  int x = v;
  x += dpp_or<kRowShr1, 0xf>(0, x);
  x += dpp_or<kRowShr2, 0xf>(0, x);
  x += dpp_or<kRowShr4, 0xf>(0, x);
  x += dpp_or<kRowShr8, 0xf>(0, x);
  x += dpp_or<kRowBcast15, 0xa>(0, x);
  x += dpp_or<kRowBcast31, 0xc>(0, x);
  total = __builtin_amdgcn_readlane(x, 63);
  return x - v;
}

// Wave-wide maximum (the running maximum's last lane, read by every lane).
__device__ inline int wave_max(int v) {
  constexpr int lo = -2147483647 - 1;
  int x = v;
  int t = dpp_or<kRowShr1, 0xf>(lo, x);
  x = t > x ? t : x;
  t = dpp_or<kRowShr2, 0xf>(lo, x);
  x = t > x ? t : x;
  t = dpp_or<kRowShr4, 0xf>(lo, x);
  x = t > x ? t : x;
  t = dpp_or<kRowShr8, 0xf>(lo, x);
  x = t > x ? t : x;
  t = dpp_or<kRowBcast15, 0xa>(lo, x);
  x = t > x ? t : x;
  t = dpp_or<kRowBcast31, 0xc>(lo, x);
  x = t > x ? t : x;
  return __builtin_amdgcn_readlane(x, 63);
}

// Per-wave LDS of the cooperative hit search: per round, the candidate
// whose pairs start at each lane.
struct AccBuf {
  int32_t* start;
  float* pub_c2;     // [64] the round's admissible hits (round_insert)
  uint32_t* pub_o;   // [64]
};

__device__ inline uint32_t pack_hist(int parent, uint32_t orig24) {
  return ((uint32_t)parent << 24) | (orig24 == kHoleIdx ? 0xFFFFFFu : orig24);
}

__global__ void build_clear(int32_t* queue, int32_t* event_done, int n_events, int64_t* start_tick) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *queue = 0;
  if (i == 0 && start_tick) *start_tick = INT64_MAX;
  for (int e = i; e < n_events; e += gridDim.x * blockDim.x) event_done[e] = 0;
}

// Fine phi index: one wave per (event, layer, z row).  Entry j of the row is
// the first sorted position whose key is >= j (the row's end if none).
__global__ void __launch_bounds__(256) fine_kernel(int n_rows, int n_phi, int n_z, int nf,
                                                   const int32_t* __restrict__ offsets,
                                                   const float* __restrict__ phi, int32_t* __restrict__ fine) {
  const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n_rows) return;
  const int nb = n_phi * n_z;
  const int el = row / n_z, iz = row % n_z;
  const int32_t* off = offsets + (size_t)el * (nb + 1);
  const int rs = off[iz * n_phi], re = off[(iz + 1) * n_phi];
  int32_t* f = fine + (size_t)row * (nf + 1);
  const float inv = fine_inv(nf);
  for (int p = rs + lane; p < re; p += 64) {
    const int k = fine_key(phi[p], inv, nf);
    const int kp = p > rs ? fine_key(phi[p - 1], inv, nf) : -1;
    for (int j = kp + 1; j <= k; ++j) f[j] = p;
  }
  const int kl = re > rs ? fine_key(phi[re - 1], inv, nf) : -1;
  for (int j = kl + 1 + lane; j <= nf; j += 64) f[j] = re;
}

// Packed hits for the hit search: one thread per sorted position.
__global__ void __launch_bounds__(256) pack_kernel(int n_hits, const float* __restrict__ x, const float* __restrict__ y,
                                                   const float* __restrict__ z, const float* __restrict__ phi,
                                                   const float* __restrict__ cov, const int32_t* __restrict__ orig,
                                                   float4* __restrict__ pack) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_hits) return;
  const size_t n = (size_t)n_hits;
  float4* o = pack + (size_t)p * 3;
  o[0] = make_float4(phi[p], x[p], y[p], z[p]);
  o[1] = make_float4(cov[p], cov[n + p], cov[2 * n + p], cov[3 * n + p]);
  o[2] = make_float4(cov[4 * n + p], cov[5 * n + p], __int_as_float(orig[p]), 0.f);
}

size_t pack_bytes(int n_hits) { return (((size_t)n_hits * 48) + 255) & ~(size_t)255; }

size_t fine_bytes(int n_events, int n_layers, int n_phi, int n_z, int refine) {
  return (size_t)n_events * n_layers * n_z * ((size_t)n_phi * refine + 1) * 4;
}

// Workspace: queue head and per-event counters | fine phi index | packed
// hits (48 bytes each) | history tables of the resident waves (16 per CU of the current device: four per
// SIMD, more than the build kernels' register use allows; a grid that would
// hold more waves is clamped).
size_t ws_head_bytes(int n_events) { return 256 + (((size_t)n_events * 4 + 255) & ~(size_t)255); }
int hist_waves_of_device() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                               hipSuccess || cus < 1)
    cus = 256;
  return cus * 16;
}


}  // namespace
