// Hit binning (the hit-selection structure of section 3.1): a counting sort
// of the hits of several events into (event, layer, z bin, phi bin), hits in
// a bin ordered by (phi, original index).  Deterministic: slots inside a bin
// are assigned by rank, never by atomic arrival order.
//
// Kernels: count -> three-phase exclusive scan of bin counts -> offsets ->
// place (arbitrary order inside each bin, whole hit records) -> rank (exact
// order inside each bin) and write out.  The hit data moves with the place
// pass, which reads the input in order, so the scattered accesses are whole
// 48-byte records rather than one word from each of ten input arrays.
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

// Bin of each hit and its arrival index among the bin's hits (the value the
// count's atomic returns; the rank pass fixes the order later).  phi and the
// bin indices are computed in FP64 with the expression order of the
// definition, so the bin of a hit never depends on contraction or
// reassociation.  A hit on a layer outside [0, L) or with a non-finite
// coordinate has no bin: it is counted in `bad` and left out.
__global__ void __launch_bounds__(256) count_kernel(int n, int E, const int32_t* __restrict__ eoff, int L,
                                                    int n_phi, int n_z, RowGeom rg,
                                                    const int32_t* __restrict__ layer,
                                                    const float* __restrict__ xyz, int32_t* __restrict__ gbin_of,
                                                    float* __restrict__ phi_of, int32_t* __restrict__ arrival,
                                                    int32_t* __restrict__ count, int32_t* __restrict__ bad) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int l = layer[i];
  const double x = (double)xyz[i], y = (double)xyz[(size_t)n + i], z = (double)xyz[2 * (size_t)n + i];
  if (l < 0 || l >= L || !__builtin_isfinite(x) || !__builtin_isfinite(y) || !__builtin_isfinite(z)) {
    gbin_of[i] = -1;
    if (bad) atomicAdd(bad, 1);
    return;
  }
  const int e = eoff ? event_of(eoff, E, i) : 0;
  double ph = atan2(y, x);
  if (ph < 0.0) ph += kTwoPi;
  const float phf = (float)ph;
  int ip = (int)floor((double)phf * (double)n_phi / kTwoPi);
  ip = ip > n_phi - 1 ? n_phi - 1 : (ip < 0 ? 0 : ip);
  const double w = rg.disk[l] ? sqrt(x * x + y * y) : z;
  const double lo = rg.lo[l], hi = rg.hi[l];
  const double fz = floor((w - lo) * (double)n_z / (hi - lo));
  const int iz = fz < 0.0 ? 0 : (fz > (double)(n_z - 1) ? n_z - 1 : (int)fz);
  const int nb = n_phi * n_z;
  const int gb = (e * L + l) * nb + iz * n_phi + ip;
  gbin_of[i] = gb;
  phi_of[i] = phf;
  arrival[i] = atomicAdd(&count[gb], 1);
}

// Phase 1: exclusive scan of 2*kScanBlock elements per block (Blelloch in LDS).
__global__ void __launch_bounds__(kScanBlock) scan_blocks(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                          int32_t* __restrict__ bsum, int n) {
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
__global__ void __launch_bounds__(kScanBlock) scan_sums(int32_t* __restrict__ bsum, int nb) {
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

__global__ void scan_add(int32_t* __restrict__ out, const int32_t* __restrict__ bsum, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += bsum[i / (2 * kScanBlock)];
}

// offsets[el][b] = start of bin b of (event, layer) el; entry nb closes it.
__global__ void offsets_kernel(const int32_t* __restrict__ start, const int32_t* __restrict__ count, int EL, int nb,
                               int32_t* __restrict__ offsets) {
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
                                                    float4* __restrict__ rec) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int gb = gbin_of[i];
  if (gb < 0) return;
  const size_t N = (size_t)n;
  const float4 r0 = make_float4(xyz[i], xyz[N + i], xyz[2 * N + i], phi_of[i]);
  const float4 r1 = make_float4(cov[i], cov[N + i], cov[2 * N + i], cov[3 * N + i]);
  const float4 r2 = make_float4(cov[4 * N + i], cov[5 * N + i], __int_as_float(i), 0.f);
  const int slot = start[gb] + arrival[i];
  float4* r = rec + (size_t)slot * 3;
  r[0] = r0;
  r[1] = r1;
  r[2] = r2;
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
                                                   float* __restrict__ sorted_cov, int32_t* __restrict__ sorted_orig) {
  const int gb = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (gb >= NB) return;
  const int b0 = start[gb], cnt = count[gb];
  if (cnt == 0) return;
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

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct BinWs {
  int32_t *gbin_of, *arrival, *count, *start, *bsum;
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
  if (w) {
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
  hipLaunchKernelGGL(fill_i32, dim3(grid_for(NB, bs) > 4096 ? 4096 : grid_for(NB, bs)), dim3(bs), 0, s, w.count,
                     NB, 0);
  if (out_bad) hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, out_bad, (int64_t)1, 0);
  if (n_hits > 0)
    hipLaunchKernelGGL(count_kernel, dim3(grid_for(n_hits, bs)), dim3(bs), 0, s, n_hits, n_events, event_offsets, L,
                       n_phi, n_z, rg, layer, xyz, w.gbin_of, w.phi_of, w.arrival, w.count, out_bad);
  const int nblk = (int)((NB + 2 * kScanBlock - 1) / (2 * kScanBlock));
  hipLaunchKernelGGL(scan_blocks, dim3(nblk), dim3(kScanBlock), 0, s, w.count, w.start, w.bsum, (int)NB);
  hipLaunchKernelGGL(scan_sums, dim3(1), dim3(kScanBlock), 0, s, w.bsum, nblk);
  hipLaunchKernelGGL(scan_add, dim3(grid_for(NB, bs)), dim3(bs), 0, s, w.start, w.bsum, (int)NB);
  hipLaunchKernelGGL(offsets_kernel, dim3(grid_for((int64_t)EL * (nb + 1), bs)), dim3(bs), 0, s, w.start, w.count,
                     EL, nb, offsets);
  if (n_hits > 0) {
    hipLaunchKernelGGL(place_kernel, dim3(grid_for(n_hits, bs)), dim3(bs), 0, s, n_hits, w.gbin_of, w.phi_of,
                       w.arrival, xyz, cov, w.start, w.rec);
    hipLaunchKernelGGL(rank_kernel, dim3(grid_for(NB, bs / 64)), dim3(bs), 0, s, (int)NB, n_hits, L, nb,
                       event_offsets, w.rec, w.start, w.count, sorted_xyzphi, sorted_cov, sorted_orig);
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
