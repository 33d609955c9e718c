// LDS plan of the build kernel (kf_build.hip): the per-wave regions of one
// block and their sizes.  Host code sizes the launch with it (two blocks of
// four waves per CU need at most 80 KB each), the kernel lays out its LDS
// with it.
#pragma once
#include <stddef.h>

#include "kfmlp.h"

// pairs per lane per round of the cooperative hit search (at most)
constexpr int NP = 2;

// LDS of one block (byte offsets), per wave:
//   stash    [27][64] f32      each slot's state before this layer's prediction
//                              (FP64: only the covariance entries not in xs)
//   record   [SEEDS][27] f32   best finished candidate of each seed
//   recfield [SEEDS][5] i32    valid, nhits, status, last layer, slot
//   toplist  [cap][64] f32 chi2, then [cap][64] i32 positions, [cap][64] u32 indices
//   starts   [64 NP] i32 run starts of the cooperative hit search
//   publish  [64] f32 chi2, [64] u32 indices of a round's admissible hits
//   mlp      activation buffer of the learned window (the network runs before
//            the hit search, so the toplists of a learned build live in it)
//   xs       [6 + NPL][64] f64 FP64 builds: the state between layers (below)
// FP64 builds keep each candidate's state between layers in LDS as
// doubles: the position and momentum and the last NPL covariance entries
// (the rest of the covariance stays in registers, its FP32 copy in the
// stash for the finished record).  Held in registers through the layer
// loop, these values were spilled to scratch memory and reloaded at every
// layer; the stash then needs only the covariance entries not held in LDS.
// NPL: what fits two blocks of four waves per CU (the learned builds' network
// buffers leave room for 2; the hybrid state, which spills more, takes all
// it can), 12 in the Cartesian state (measured best).
__host__ __device__ constexpr int xs_npl(int tsize, bool learned, bool hyb) {
  return tsize == 8 ? (learned ? 2 : hyb ? 20 : 12) : -6;
}
struct LdsPlan {
  size_t stash, rec, recf, acc, pub, tl, tl_stride, mlp, xs, total;
};
__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }
__host__ __device__ inline LdsPlan lds_plan(int LB, int nwaves, int cap, int tsize, bool learned, bool hyb) {
  const int seeds = 64 / cap;
  const int npl = xs_npl(tsize, learned, hyb);
  // FP32 values per lane in the stash: all 27 without the LDS state
  const int nst = npl < 0 ? 27 : 21 - npl;
  LdsPlan p;
  (void)LB;
  p.stash = 0;
  p.rec = align16(p.stash + (size_t)nwaves * nst * 64 * 4);
  p.recf = align16(p.rec + (size_t)nwaves * seeds * 27 * 4);
  const size_t tl_wave = (size_t)cap * 64 * 12;
  p.acc = align16(p.recf + (size_t)nwaves * seeds * 5 * 4);
  p.pub = align16(p.acc + (size_t)nwaves * 64 * NP * 4);
  p.tl = align16(p.pub + (size_t)nwaves * 64 * 8);
  if (learned) {
    const size_t per = tl_wave > KFMLP_LDS_BYTES ? tl_wave : (size_t)KFMLP_LDS_BYTES;
    p.mlp = p.tl;
    p.total = p.mlp + (size_t)nwaves * per;
    p.tl_stride = per;
  } else {
    p.mlp = p.total = align16(p.tl + (size_t)nwaves * tl_wave);
    p.tl_stride = tl_wave;
  }
  p.xs = p.total;
  if (npl >= 0) p.total = align16(p.xs + (size_t)nwaves * (6 + npl) * 64 * 8);
  return p;
}
