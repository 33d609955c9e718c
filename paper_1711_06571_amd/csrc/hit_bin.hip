// Hit binning (the hit-selection structure of section 3.1): a counting sort
// of the hits of several events into (event, layer, z bin, phi bin), hits in
// a bin ordered by (phi, original index).  Deterministic: slots inside a bin
// are assigned by rank, never by atomic arrival order.
//
// Two paths with the same result.  The fast path sorts each (event, layer)
// in one block (LDS histogram, scan, records to their bins, ranks inside
// LDS tiles of whole bins) when the input holds each event's hits grouped by
// layer, all valid; the general path takes any order and bad hits: count ->
// three-phase exclusive scan of bin counts -> offsets -> place (arbitrary
// order inside each bin, whole hit records) -> rank (exact order inside
// each bin) and write out.  A device flag selects the path, so the sequence
// has no host decision in it and can be captured in a graph.
#include <stdlib.h>
#include <string.h>

#include <algorithm>

#include "kfhost.h"

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr int kScanBlock = 1024;  // threads; each handles 2 elements

__global__ void fill_i32(int32_t* __restrict__ a, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

__device__ inline int event_of(const int32_t* __restrict__ eoff, int E, int i) {
  int lo = 0, hi = E;  // find e with eoff[e] <= i < eoff[e+1]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (eoff[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// The row coordinate of each layer: w = z on a barrel layer, w = r =
// sqrt(x^2 + y^2) on an endcap disk, binned over [lo, hi] in n_z rows.
struct RowGeom {
  int32_t disk[32];
  double lo[32], hi[32];
};

// Bin of a hit inside its (event, layer) and its stored phi.  phi and the
// bin indices are computed in FP64 with the expression order of the
// definition, so the bin of a hit never depends on contraction or
// reassociation.
__device__ inline int bin_in_layer(double x, double y, double z, int l, const RowGeom& rg, int n_phi, int n_z,
                                   float* phf_out) {
#pragma clang fp contract(off)
  double ph = atan2(y, x);
  if (ph < 0.0) ph += kTwoPi;
  const float phf = (float)ph;
  int ip = (int)floor((double)phf * (double)n_phi / kTwoPi);
  ip = ip > n_phi - 1 ? n_phi - 1 : (ip < 0 ? 0 : ip);
  const double w = rg.disk[l] ? sqrt(x * x + y * y) : z;
  const double lo = rg.lo[l], hi = rg.hi[l];
  const double fz = floor((w - lo) * (double)n_z / (hi - lo));
  const int iz = fz < 0.0 ? 0 : (fz > (double)(n_z - 1) ? n_z - 1 : (int)fz);
  *phf_out = phf;
  return iz * n_phi + ip;
}

// The same bin, with phi from the FP32 arctangent where that decides it: the
// FP32 angle (a few ulp, below 4e-6 rad from the FP64 one after the wrap)
// more than 2e-5 rad from a bin edge puts the FP64 angle in the same bin;
// otherwise (and at the ends of [0, 2 pi)) the FP64 computation above.  z
// (or r) and the row are computed as above.  (Where the two ever disagreed,
// the placement pass, which uses the FP64 bin, would find a bin over its
// count and hand the call to the general path.)
__device__ inline int bin_in_layer_fast(float xf, float yf, float zf, int l, const RowGeom& rg, int n_phi, int n_z,
                                        double phi_scale) {
#pragma clang fp contract(off)
  float p32 = atan2f(yf, xf);
  if (p32 < 0.f) p32 += 6.2831855f;
  const double tt = (double)p32 * phi_scale, m = 2e-5 * phi_scale;
  const double fl = floor(tt), fr = tt - fl;
  if (!(fr > m && fr < 1.0 - m && fl >= 0.0 && fl <= (double)(n_phi - 1))) {
    float phf;
    return bin_in_layer((double)xf, (double)yf, (double)zf, l, rg, n_phi, n_z, &phf);
  }
  const int ip = (int)fl;
  const double x = (double)xf, y = (double)yf, z = (double)zf;
  const double w = rg.disk[l] ? sqrt(x * x + y * y) : z;
  const double lo = rg.lo[l], hi = rg.hi[l];
  const double fz = floor((w - lo) * (double)n_z / (hi - lo));
  const int iz = fz < 0.0 ? 0 : (fz > (double)(n_z - 1) ? n_z - 1 : (int)fz);
  return iz * n_phi + ip;
}

__device__ inline bool finite3(float x, float y, float z) {
  return __builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z);
}

// ---- Fast path: one block per (event, layer) -------------------------------
//
// When every event's hits come grouped by layer in ascending order, all on
// valid layers with finite coordinates (as detector readout and the
// generator deliver them), the hits of an (event, layer) are one contiguous
// input range and their sorted positions are that same range.  One block
// then sorts the range on its own: an LDS histogram of the bins, a block
// scan for the bin starts, whole hit records scattered to their bins with
// LDS cursors (arbitrary order inside a bin), and tiles of whole bins in
// LDS in which every hit counts the hits of its bin with a smaller
// (phi, input index) key and is written to its sorted position.  A block
// finds its range by binary search and checks it (range ends, every layer,
// finite coordinates, no bin above the tile size); any failure raises
// `flag`, and the general kernels below then sort the whole call again.
constexpr int kSegThreads = 512;
constexpr int kSegTile = 2048;                    // positions of a rank tile at most
constexpr int kSegPer = kSegTile / kSegThreads;   // tile positions per thread
constexpr int kSegMaxBins = 4096;                 // n_phi * n_z the fast path takes

size_t seg_lds_bytes(int nb) { return (size_t)(3 * nb + 1) * 4 + (size_t)kSegTile * 12; }
constexpr int kSegUnroll = 4;  // hits per thread in flight in the two passes over the range

// First position in [lo, hi) whose value is >= v (a sorted there), hi if
// none: 64 probes per round by one wave (a few dependent loads instead of a
// binary search's twenty).  On unsorted data it still returns a position in
// [lo, hi], which the caller's checks reject.
__device__ inline int lower_bound_wave(const int32_t* __restrict__ a, int lo, int hi, int v, int lane) {
  while (hi - lo > 64) {
    const int step = (hi - lo + 63) / 64;
    const int p = lo + lane * step;
    const bool below = p < hi && a[p] < v;
    const int c = __builtin_popcountll(__ballot(below));
    const int nlo = c >= 1 ? lo + (c - 1) * step + 1 : lo;
    const int pc = lo + c * step;
    hi = (c < 64 && pc < hi) ? pc : hi;
    lo = nlo;
  }
  const bool below = lo + lane < hi && a[lo + lane] < v;
  return lo + __builtin_popcountll(__ballot(below));
}

__global__ void __launch_bounds__(kSegThreads) seg_kernel(int n, int E, const int32_t* __restrict__ eoff, int L, int n_phi,
                                                          int n_z, RowGeom rg, const int32_t* __restrict__ layer,
                                                          const float* __restrict__ xyz, const float* __restrict__ cov,
                                                          int32_t* __restrict__ flag, float4* __restrict__ rec,
                                                          int32_t* __restrict__ offsets,
                                                          float* __restrict__ sorted_xyzphi,
                                                          float* __restrict__ sorted_cov,
                                                          int32_t* __restrict__ sorted_orig) {
  extern __shared__ __align__(16) int32_t sm[];
  const int nb = n_phi * n_z;
  int32_t* hist = sm;                       // [nb] counts
  int32_t* cursor = sm + nb;                // [nb] records placed per bin
  int32_t* start = sm + 2 * nb;             // [nb + 1] bin starts inside the range
  float* kphi = (float*)(start + nb + 1);   // [kSegTile] keys of a tile
  int32_t* kidx = (int32_t*)(kphi + kSegTile);
  int32_t* kbin = kidx + kSegTile;
  __shared__ int s_bad, s_t1, s_a, s_b;
  __shared__ int32_t s_part[kSegThreads];
  const int sg = blockIdx.x, e = sg / L, l = sg - e * L, t = threadIdx.x;
  const size_t N = (size_t)n;
  // the event's range, checked: the events must tile [0, n) in order
  const int e0 = eoff ? eoff[e] : 0, e1 = eoff ? eoff[e + 1] : n;
  const int ea = e0 < 0 ? 0 : (e0 > n ? n : e0), eb = e1 < ea ? ea : (e1 > n ? n : e1);
  const bool ev_ok = ea == e0 && eb == e1 && (e > 0 || ea == 0) && (e < E - 1 || eb == n);
  if (t < 64) {
    const int a = lower_bound_wave(layer, ea, eb, l, t), b = lower_bound_wave(layer, ea, eb, l + 1, t);
    if (t == 0) {
      s_a = a;
      s_b = b;
      s_bad = !ev_ok || (b < a) || (l == 0 && a != ea) || (l == L - 1 && b != eb);
    }
  }
  for (int k = t; k < 2 * nb; k += kSegThreads) hist[k] = 0;
  __syncthreads();
  const int a = s_a, b = s_b;
  if (s_bad) {
    if (t == 0) atomicOr(flag, 1);
    return;
  }
  // histogram of the bins; every hit of the range checked
  const double phi_scale = (double)n_phi / kTwoPi;
  for (int i0 = a + t; i0 < b; i0 += kSegThreads * kSegUnroll) {
    float xf[kSegUnroll], yf[kSegUnroll], zf[kSegUnroll];
    int ly[kSegUnroll];
#pragma unroll
    for (int u = 0; u < kSegUnroll; ++u) {
      const int i = i0 + u * kSegThreads;
      if (i < b) {
        ly[u] = layer[i];
        xf[u] = xyz[i];
        yf[u] = xyz[N + i];
        zf[u] = xyz[2 * N + i];
      }
    }
#pragma unroll
    for (int u = 0; u < kSegUnroll; ++u) {
      if (i0 + u * kSegThreads < b) {
        if (ly[u] != l || !finite3(xf[u], yf[u], zf[u])) {
          s_bad = 1;
          continue;
        }
        atomicAdd(&hist[bin_in_layer_fast(xf[u], yf[u], zf[u], l, rg, n_phi, n_z, phi_scale)], 1);
      }
    }
  }
  __syncthreads();
  // exclusive scan of the counts: each thread sums a chunk of consecutive
  // bins, the chunk sums are scanned in LDS, then each chunk is written out
  const int per = (nb + kSegThreads - 1) / kSegThreads;
  const int c0 = t * per, c1 = c0 + per < nb ? c0 + per : nb;
  int sum = 0, mx = 0;
  for (int k = c0; k < c1; ++k) {
    sum += hist[k];
    mx = hist[k] > mx ? hist[k] : mx;
  }
  if (mx > kSegTile) s_bad = 1;
  s_part[t] = sum;
  __syncthreads();
  for (int d = 1; d < kSegThreads; d <<= 1) {  // Hillis-Steele inclusive
    const int v = t >= d ? s_part[t - d] : 0;
    __syncthreads();
    s_part[t] += v;
    __syncthreads();
  }
  if (s_bad) {
    if (t == 0) atomicOr(flag, 1);
    return;
  }
  int run = s_part[t] - sum;
  for (int k = c0; k < c1; ++k) {
    start[k] = run;
    run += hist[k];
  }
  if (t == kSegThreads - 1) start[nb] = s_part[t];
  __syncthreads();
  int32_t* off = offsets + (size_t)sg * (nb + 1);
  for (int k = t; k <= nb; k += kSegThreads) off[k] = a + start[k];
  // whole records to their bins (order inside a bin from the LDS cursors;
  // a slot past its bin's count would mean the two bin computations
  // disagree: the call then goes to the general path)
  for (int i0 = a + t; i0 < b; i0 += kSegThreads * kSegUnroll) {
    float4 r0[kSegUnroll], r1[kSegUnroll], r2[kSegUnroll];
#pragma unroll
    for (int u = 0; u < kSegUnroll; ++u) {
      const int i = i0 + u * kSegThreads;
      if (i < b) {
        r0[u] = make_float4(xyz[i], xyz[N + i], xyz[2 * N + i], 0.f);
        r1[u] = make_float4(cov[i], cov[N + i], cov[2 * N + i], cov[3 * N + i]);
        r2[u] = make_float4(cov[4 * N + i], cov[5 * N + i], __int_as_float(i), 0.f);
      }
    }
#pragma unroll
    for (int u = 0; u < kSegUnroll; ++u) {
      if (i0 + u * kSegThreads < b) {
        float phf;
        const int bn = bin_in_layer((double)r0[u].x, (double)r0[u].y, (double)r0[u].z, l, rg, n_phi, n_z, &phf);
        const int p = start[bn] + atomicAdd(&cursor[bn], 1);
        if (p >= start[bn + 1]) {
          s_bad = 1;
          continue;
        }
        r0[u].w = phf;
        r2[u].w = __int_as_float(bn);
        float4* r = rec + (size_t)(a + p) * 3;
        r[0] = r0[u];
        r[1] = r1[u];
        r[2] = r2[u];
      }
    }
  }
  __syncthreads();
  if (s_bad) {
    if (t == 0) atomicOr(flag, 1);
    return;
  }
  // tiles of whole bins: rank inside each bin, write the sorted arrays
  const int cnt = b - a;
  for (int t0 = 0; t0 < cnt;) {
    if (t == 0) {
      int t1 = cnt;
      if (t0 + kSegTile < cnt) {
        // the tile ends where the bin holding position t0 + kSegTile starts
        // (after t0: no bin holds more than kSegTile hits)
        const int q = t0 + kSegTile;
        int lo = 0, hi = nb;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (start[mid] <= q) lo = mid; else hi = mid;
        }
        t1 = start[lo];
      }
      s_t1 = t1;
    }
    __syncthreads();
    const int t1 = s_t1;
    float4 r0[kSegPer], r1[kSegPer], r2[kSegPer];
#pragma unroll
    for (int u = 0; u < kSegPer; ++u) {
      const int p = t0 + u * kSegThreads + t;
      if (p < t1) {
        const float4* r = rec + (size_t)(a + p) * 3;
        r0[u] = r[0];
        r1[u] = r[1];
        r2[u] = r[2];
        kphi[p - t0] = r0[u].w;
        kidx[p - t0] = __float_as_int(r2[u].z);
        kbin[p - t0] = __float_as_int(r2[u].w);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kSegPer; ++u) {
      const int p = t0 + u * kSegThreads + t;
      if (p < t1) {
        const int bn = __float_as_int(r2[u].w), i = __float_as_int(r2[u].z);
        const float ph = r0[u].w;
        const int q0 = start[bn] - t0, q1 = start[bn + 1] - t0;
        int rank = 0;
        for (int q = q0; q < q1; ++q) {
          const float pq = kphi[q];
          const int iq = kidx[q];
          rank += (pq < ph || (pq == ph && iq < i)) ? 1 : 0;
        }
        const size_t dst = (size_t)a + start[bn] + rank;
        sorted_xyzphi[dst] = r0[u].x;
        sorted_xyzphi[N + dst] = r0[u].y;
        sorted_xyzphi[2 * N + dst] = r0[u].z;
        sorted_xyzphi[3 * N + dst] = ph;
        sorted_cov[dst] = r1[u].x;
        sorted_cov[N + dst] = r1[u].y;
        sorted_cov[2 * N + dst] = r1[u].z;
        sorted_cov[3 * N + dst] = r1[u].w;
        sorted_cov[4 * N + dst] = r2[u].x;
        sorted_cov[5 * N + dst] = r2[u].y;
        sorted_orig[dst] = i - ea;
      }
    }
    __syncthreads();
    t0 = t1;
  }
}

// ---- General path: any order, bad hits --------------------------------------
// Every kernel of this path returns at once when the fast path sorted the
// call (flag == 0).

// Bin of each hit and its arrival index among the bin's hits (the value the
// count's atomic returns; the rank pass fixes the order later).  A hit on a
// layer outside [0, L) or with a non-finite coordinate has no bin: it is
// counted in `bad` and left out.
__global__ void __launch_bounds__(256) count_kernel(int n, int E, const int32_t* __restrict__ eoff, int L,
                                                    int n_phi, int n_z, RowGeom rg,
                                                    const int32_t* __restrict__ layer,
                                                    const float* __restrict__ xyz, int32_t* __restrict__ gbin_of,
                                                    float* __restrict__ phi_of, int32_t* __restrict__ arrival,
                                                    int32_t* __restrict__ count, int32_t* __restrict__ bad,
                                                    const int32_t* __restrict__ flag) {
  if (*flag == 0) return;
  const int nb = n_phi * n_z;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int l = layer[i];
    const float xf = xyz[i], yf = xyz[(size_t)n + i], zf = xyz[2 * (size_t)n + i];
    if (l < 0 || l >= L || !finite3(xf, yf, zf)) {
      gbin_of[i] = -1;
      if (bad) atomicAdd(bad, 1);
      continue;
    }
    const int e = eoff ? event_of(eoff, E, i) : 0;
    float phf;
    const int gb = (e * L + l) * nb + bin_in_layer((double)xf, (double)yf, (double)zf, l, rg, n_phi, n_z, &phf);
    gbin_of[i] = gb;
    phi_of[i] = phf;
    arrival[i] = atomicAdd(&count[gb], 1);
  }
}

// Phase 1: exclusive scan of 2*kScanBlock elements per block (Blelloch in LDS).
__global__ void __launch_bounds__(kScanBlock) scan_blocks(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                          int32_t* __restrict__ bsum, int n,
                                                          const int32_t* __restrict__ flag) {
  if (*flag == 0) return;
  __shared__ int32_t s[2 * kScanBlock];
  const int t = threadIdx.x;
  const int base = blockIdx.x * 2 * kScanBlock;
  s[2 * t] = base + 2 * t < n ? in[base + 2 * t] : 0;
  s[2 * t + 1] = base + 2 * t + 1 < n ? in[base + 2 * t + 1] : 0;
  int off = 1;
  for (int d = kScanBlock; d > 0; d >>= 1) {
    __syncthreads();
    if (t < d) {
      int ai = off * (2 * t + 1) - 1, bi = off * (2 * t + 2) - 1;
      s[bi] += s[ai];
    }
    off <<= 1;
  }
  if (t == 0) {
    bsum[blockIdx.x] = s[2 * kScanBlock - 1];
    s[2 * kScanBlock - 1] = 0;
  }
  for (int d = 1; d <= kScanBlock; d <<= 1) {
    off >>= 1;
    __syncthreads();
    if (t < d) {
      int ai = off * (2 * t + 1) - 1, bi = off * (2 * t + 2) - 1;
      int v = s[ai];
      s[ai] = s[bi];
      s[bi] += v;
    }
  }
  __syncthreads();
  if (base + 2 * t < n) out[base + 2 * t] = s[2 * t];
  if (base + 2 * t + 1 < n) out[base + 2 * t + 1] = s[2 * t + 1];
}

// Phase 2: sequential-in-chunks exclusive scan of the block sums (one block).
__global__ void __launch_bounds__(kScanBlock) scan_sums(int32_t* __restrict__ bsum, int nb,
                                                        const int32_t* __restrict__ flag) {
  if (*flag == 0) return;
  __shared__ int32_t s[kScanBlock];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  for (int c = 0; c < nb; c += kScanBlock) {
    __syncthreads();
    const int i = c + threadIdx.x;
    const int v = i < nb ? bsum[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < kScanBlock; d <<= 1) {  // Hillis-Steele inclusive
      int a = threadIdx.x >= d ? s[threadIdx.x - d] : 0;
      __syncthreads();
      s[threadIdx.x] += a;
      __syncthreads();
    }
    if (i < nb) bsum[i] = carry + s[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == kScanBlock - 1) carry += s[kScanBlock - 1];
  }
}

__global__ void scan_add(int32_t* __restrict__ out, const int32_t* __restrict__ bsum, int n,
                         const int32_t* __restrict__ flag) {
  if (*flag == 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += bsum[i / (2 * kScanBlock)];
}

// offsets[el][b] = start of bin b of (event, layer) el; entry nb closes it.
__global__ void offsets_kernel(const int32_t* __restrict__ start, const int32_t* __restrict__ count, int EL, int nb,
                               int32_t* __restrict__ offsets, const int32_t* __restrict__ flag) {
  if (*flag == 0) return;
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= (int64_t)EL * (nb + 1)) return;
  const int el = (int)(k / (nb + 1)), b = (int)(k % (nb + 1));
  const int64_t g = (int64_t)el * nb;
  offsets[k] = b < nb ? start[g + b] : start[g + nb - 1] + count[g + nb - 1];
}

// Each hit takes the slot of its bin given by its arrival index and writes
// its whole record there: (x, y, z, phi), (cov 0..3), (cov 4, cov 5, input
// index, 0).
__global__ void __launch_bounds__(256) place_kernel(int n, const int32_t* __restrict__ gbin_of,
                                                    const float* __restrict__ phi_of,
                                                    const int32_t* __restrict__ arrival, const float* __restrict__ xyz,
                                                    const float* __restrict__ cov, const int32_t* __restrict__ start,
                                                    float4* __restrict__ rec, const int32_t* __restrict__ flag) {
  if (*flag == 0) return;
  const size_t N = (size_t)n;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int gb = gbin_of[i];
    if (gb < 0) continue;
    const float4 r0 = make_float4(xyz[i], xyz[N + i], xyz[2 * N + i], phi_of[i]);
    const float4 r1 = make_float4(cov[i], cov[N + i], cov[2 * N + i], cov[3 * N + i]);
    const float4 r2 = make_float4(cov[4 * N + i], cov[5 * N + i], __int_as_float(i), 0.f);
    const int slot = start[gb] + arrival[i];
    float4* r = rec + (size_t)slot * 3;
    r[0] = r0;
    r[1] = r1;
    r[2] = r2;
  }
}

// Exact order inside each bin: rank = number of hits of the bin with a
// smaller (phi, original index) key.  One wave per bin: each lane holds one
// hit record of the bin and compares it with every hit of the bin, whose keys
// the wave passes around by shuffles 64 at a time (bins larger than 64 hits
// loop over blocks of 64).  The hit is then written to its slot in the sorted
// arrays.
__global__ void __launch_bounds__(256) rank_kernel(int NB, int n, int L, int nb_el,
                                                   const int32_t* __restrict__ eoff,
                                                   const float4* __restrict__ rec,
                                                   const int32_t* __restrict__ start,
                                                   const int32_t* __restrict__ count,
                                                   float* __restrict__ sorted_xyzphi,
                                                   float* __restrict__ sorted_cov, int32_t* __restrict__ sorted_orig,
                                                   const int32_t* __restrict__ flag) {
  if (*flag == 0) return;
  const int lane = threadIdx.x & 63;
  const int waves = gridDim.x * (blockDim.x >> 6);
  for (int gb = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); gb < NB; gb += waves) {
    const int b0 = start[gb], cnt = count[gb];
    if (cnt == 0) continue;
    // the event of the bin: bins are numbered (event * L + layer) * nb_el + bin
    const int ev_base = eoff ? eoff[gb / (L * nb_el)] : 0;
    for (int c0 = 0; c0 < cnt; c0 += 64) {
      const bool mine = c0 + lane < cnt;
      const float4* r = rec + (size_t)(b0 + c0 + (mine ? lane : 0)) * 3;
      const float4 r0 = r[0], r1 = r[1], r2 = r[2];
      const int i = __float_as_int(r2.z);
      const float ph = r0.w;
      int rank = 0;
      for (int d0 = 0; d0 < cnt; d0 += 64) {
        const bool theirs = d0 + lane < cnt;
        const float4* o = rec + (size_t)(b0 + d0 + (theirs ? lane : 0)) * 3;
        const int oi = d0 == c0 ? i : __float_as_int(o[2].z);
        const float op = d0 == c0 ? ph : o[0].w;
        const int m = cnt - d0 < 64 ? cnt - d0 : 64;
        for (int t = 0; t < m; ++t) {
          const float pj = __shfl(op, t, 64);
          const int j = __shfl(oi, t, 64);
          rank += (pj < ph || (pj == ph && j < i)) ? 1 : 0;
        }
      }
      if (mine) {
        const int dst = b0 + rank;
        const size_t N = (size_t)n;
        sorted_xyzphi[dst] = r0.x;
        sorted_xyzphi[N + dst] = r0.y;
        sorted_xyzphi[2 * N + dst] = r0.z;
        sorted_xyzphi[3 * N + dst] = ph;
        sorted_cov[dst] = r1.x;
        sorted_cov[N + dst] = r1.y;
        sorted_cov[2 * N + dst] = r1.z;
        sorted_cov[3 * N + dst] = r1.w;
        sorted_cov[4 * N + dst] = r2.x;
        sorted_cov[5 * N + dst] = r2.y;
        sorted_orig[dst] = i - ev_base;
      }
    }
  }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct BinWs {
  int32_t *gbin_of, *arrival, *count, *start, *bsum;
  int32_t* flag;  // 0: the fast path sorted the call, else the general path runs
  float* phi_of;
  float4* rec;  // [n][3] hit records in bin slots
};

size_t bin_ws_layout(int E, int L, int n_phi, int n_z, int n, char* base, BinWs* w) {
  const size_t NB = (size_t)E * L * n_phi * n_z;
  const size_t nblk = (NB + 2 * kScanBlock - 1) / (2 * kScanBlock);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  char* a = take(sizeof(int32_t) * (size_t)n);
  char* b = take(sizeof(float4) * 3 * (size_t)n);
  char* c = take(sizeof(float) * (size_t)n);
  char* d = take(sizeof(int32_t) * NB);
  char* e = take(sizeof(int32_t) * (size_t)n);
  char* f = take(sizeof(int32_t) * NB);
  char* g = take(sizeof(int32_t) * (nblk + 1));
  char* h = take(sizeof(int32_t));
  if (w) {
    w->flag = (int32_t*)h;
    w->gbin_of = (int32_t*)a;
    w->rec = (float4*)b;
    w->phi_of = (float*)c;
    w->arrival = (int32_t*)e;
    w->count = (int32_t*)d;
    w->start = (int32_t*)f;
    w->bsum = (int32_t*)g;
  }
  return off;
}

int grid_for(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

// One block per (event, layer) pays when there are many ranges to spread
// over the device: at least six per CU (68 M hits in 3 400 ranges: 4.9 ms
// grouped against 7.7 general; 12.7 M hits of 64 uneven events in 1 088
// ranges: 3.7 against 1.8, the largest ranges' blocks finishing last).
// KFTRACK_HIT_BIN_PATH=grouped or =general overrides the choice.
bool use_grouped_path(int EL) {
  const char* v = getenv("KFTRACK_HIT_BIN_PATH");
  if (v && !strcmp(v, "grouped")) return true;
  if (v && !strcmp(v, "general")) return false;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  return EL >= 6 * cus;
}

}  // namespace

extern "C" size_t hit_bin_workspace_bytes(int32_t n_events, int32_t n_layers, int32_t n_phi, int32_t n_z,
                                          int32_t n_hits) {
  if (n_events < 1 || n_layers < 1 || n_phi < 1 || n_z < 1 || n_hits < 0) return 0;
  return bin_ws_layout(n_events, n_layers, n_phi, n_z, n_hits, nullptr, nullptr);
}

namespace {

int run_hit_bin(int L, const RowGeom& rg, int32_t n_events, const int32_t* event_offsets, int32_t n_phi,
                int32_t n_z, int32_t n_hits, const int32_t* layer, const float* xyz, const float* cov,
                int32_t* offsets, float* sorted_xyzphi, float* sorted_cov, int32_t* sorted_orig, int32_t* out_bad,
                void* ws, size_t ws_bytes, void* stream) {
  if (n_events < 1 || n_phi < 1 || n_z < 1 || n_hits < 0) return KF_E_INVALID_ARG;
  if (n_events > 1 && !event_offsets) return KF_E_INVALID_ARG;
  const int64_t NB = (int64_t)n_events * L * n_phi * n_z;
  if (NB >= (1ll << 31) - 1) return KF_E_UNSUPPORTED;
  if (!offsets) return KF_E_INVALID_ARG;
  if (n_hits > 0 && (!layer || !xyz || !cov || !sorted_xyzphi || !sorted_cov || !sorted_orig))
    return KF_E_INVALID_ARG;
  const size_t need = hit_bin_workspace_bytes(n_events, L, n_phi, n_z, n_hits);
  if (!ws || ws_bytes < need || ((uintptr_t)ws & 255)) return KF_E_WORKSPACE;
  BinWs w;
  bin_ws_layout(n_events, L, n_phi, n_z, n_hits, (char*)ws, &w);
  hipStream_t s = (hipStream_t)stream;
  const int bs = 256;
  const int nb = n_phi * n_z;
  const int EL = n_events * L;
  // clear (kernels, not memset nodes, so the sequence can be captured in a graph)
  if (out_bad) hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, out_bad, (int64_t)1, 0);
  // fast path (one block per event and layer); the flag starts raised where
  // it cannot apply or would not pay
  const bool fast = nb <= kSegMaxBins && use_grouped_path(EL);
  hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, w.flag, (int64_t)1, fast ? 0 : 1);
  if (fast)
    hipLaunchKernelGGL(seg_kernel, dim3(EL), dim3(kSegThreads), seg_lds_bytes(nb), s, n_hits, n_events, event_offsets,
                       L, n_phi, n_z, rg, layer, xyz, cov, w.flag, w.rec, offsets, sorted_xyzphi, sorted_cov, sorted_orig);
  // general path (every kernel returns at once unless the flag is raised)
  const int cap = 8192;  // blocks of the grid-stride kernels
  hipLaunchKernelGGL(fill_i32, dim3(grid_for(NB, bs) > 4096 ? 4096 : grid_for(NB, bs)), dim3(bs), 0, s, w.count,
                     NB, 0);
  if (n_hits > 0)
    hipLaunchKernelGGL(count_kernel, dim3(std::min(grid_for(n_hits, bs), cap)), dim3(bs), 0, s, n_hits, n_events,
                       event_offsets, L, n_phi, n_z, rg, layer, xyz, w.gbin_of, w.phi_of, w.arrival, w.count,
                       out_bad, w.flag);
  const int nblk = (int)((NB + 2 * kScanBlock - 1) / (2 * kScanBlock));
  hipLaunchKernelGGL(scan_blocks, dim3(nblk), dim3(kScanBlock), 0, s, w.count, w.start, w.bsum, (int)NB, w.flag);
  hipLaunchKernelGGL(scan_sums, dim3(1), dim3(kScanBlock), 0, s, w.bsum, nblk, w.flag);
  hipLaunchKernelGGL(scan_add, dim3(grid_for(NB, bs)), dim3(bs), 0, s, w.start, w.bsum, (int)NB, w.flag);
  hipLaunchKernelGGL(offsets_kernel, dim3(grid_for((int64_t)EL * (nb + 1), bs)), dim3(bs), 0, s, w.start, w.count,
                     EL, nb, offsets, w.flag);
  if (n_hits > 0) {
    hipLaunchKernelGGL(place_kernel, dim3(std::min(grid_for(n_hits, bs), cap)), dim3(bs), 0, s, n_hits, w.gbin_of,
                       w.phi_of, w.arrival, xyz, cov, w.start, w.rec, w.flag);
    hipLaunchKernelGGL(rank_kernel, dim3(std::min(grid_for(NB, bs / 64), cap)), dim3(bs), 0, s, (int)NB, n_hits, L,
                       nb, event_offsets, w.rec, w.start, w.count, sorted_xyzphi, sorted_cov, sorted_orig, w.flag);
  }
  return kf_check_launch();
}

}  // namespace

extern "C" int hit_bin(const kf_geometry* g, int32_t n_events, const int32_t* event_offsets, int32_t n_phi,
                       int32_t n_z, int32_t n_hits, const int32_t* layer, const float* xyz, const float* cov,
                       int32_t* offsets, float* sorted_xyzphi, float* sorted_cov, int32_t* sorted_orig,
                       int32_t* out_bad, void* ws, size_t ws_bytes, void* stream) {
  if (kf_check_geometry(g)) return KF_E_INVALID_ARG;
  // every layer binned in z over [-z_half, z_half]
  RowGeom rg = {};
  for (int l = 0; l < g->n_layers; ++l) {
    rg.disk[l] = 0;
    rg.lo[l] = -(double)g->z_half;
    rg.hi[l] = (double)g->z_half;
  }
  return run_hit_bin(g->n_layers, rg, n_events, event_offsets, n_phi, n_z, n_hits, layer, xyz, cov, offsets,
                     sorted_xyzphi, sorted_cov, sorted_orig, out_bad, ws, ws_bytes, stream);
}

extern "C" int hit_bin_det(const kf_detector* d, int32_t n_events, const int32_t* event_offsets, int32_t n_phi,
                           int32_t n_w, int32_t n_hits, const int32_t* layer, const float* xyz, const float* cov,
                           int32_t* offsets, float* sorted_xyzphi, float* sorted_cov, int32_t* sorted_orig,
                           int32_t* out_bad, void* ws, size_t ws_bytes, void* stream) {
  if (kf_check_detector(d)) return KF_E_INVALID_ARG;
  RowGeom rg = {};
  for (int l = 0; l < d->n_layers; ++l) {
    rg.disk[l] = d->kind[l] == KF_LAYER_DISK ? 1 : 0;
    rg.lo[l] = (double)d->lo[l];
    rg.hi[l] = (double)d->hi[l];
  }
  return run_hit_bin(d->n_layers, rg, n_events, event_offsets, n_phi, n_w, n_hits, layer, xyz, cov, offsets,
                     sorted_xyzphi, sorted_cov, sorted_orig, out_bad, ws, ws_bytes, stream);
}
