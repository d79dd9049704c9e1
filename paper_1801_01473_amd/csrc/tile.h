// Site traversal orders shared by the force-side kernels.
#pragma once

#include "common.h"

namespace lqcd {

// Half index of the i-th site visited when the (y, z) cross-section is cut
// into tiles of ty rows and tz slices and, inside a tile, x and y run
// fastest, then z, then t (the tiles come last).  Sites whose +-t, +-z and +-y
// neighbours are in the same tile are visited close together in time, so a
// neighbour that one site loads is still in L2 when the next one needs it.
// tz = 0: lexicographic (i itself).  A bijection on [0, Vh) when ty divides Ly
// and tz divides Lz.
__device__ __forceinline__ int tiled_half_index(const KGeom& g, int i, int ty, int tz) {
  if (tz == 0) return i;
  const int row = g.Lxh * ty;
  const int inrow = i % row;
  int r = i / row;
  const int zi = r % tz;
  r /= tz;
  const int t = r % g.Lt;
  const int tile = r / g.Lt;
  const int nty = g.Ly / ty;
  const int y0 = (tile % nty) * ty, z = (tile / nty) * tz + zi;
  return inrow + g.Lxh * y0 + g.sz * z + g.st * t;
}

// A small tile edge: the first of {6, 4, 8, 3, 2} that divides L, else 0
// (no tiling).
inline int small_tile(int L) {
  for (int e : {6, 4, 8, 3, 2})
    if (L % e == 0 && L > e) return e;
  return 0;
}

// A z-slab depth for kernels whose threads are short-lived (every site of a
// slab's t slice in flight at once): the largest of {8, 6, 4, 3, 2} that
// divides L, else 0 (no tiling).
inline int slab_tile(int L) {
  for (int e : {8, 6, 4, 3, 2})
    if (L % e == 0 && L > e) return e;
  return 0;
}

// Thread order of the per-link kernels: a segment (a direction or a side)
// outermost, then chunks of kLinkChunk half indices in which the two halves
// of a workgroup take the same half indices of parity 0 and of parity 1.
// A link's staples and neighbours alternate between the parities, so both
// parities of a region are read while they are in the same XCD's L2.  The
// grid covers link_threads_per_segment() threads per segment; threads whose
// half index i is past Vh do nothing (the return value).
constexpr int kLinkChunk = 64;  // half the per-link workgroup (128 threads)

struct LinkThread {
  int seg, par, i;
};

__host__ __device__ inline int64_t link_threads_per_segment(int Vh) {
  return int64_t(2) * ((Vh + kLinkChunk - 1) / kLinkChunk) * kLinkChunk;
}

__device__ __forceinline__ bool link_thread(const KGeom& g, int64_t idx, LinkThread& t) {
  const int64_t per = link_threads_per_segment(g.Vh);
  t.seg = int(idx / per);
  const int64_t loc = idx % per;
  t.par = int((loc / kLinkChunk) & 1);
  t.i = int((loc / (2 * kLinkChunk)) * kLinkChunk + loc % kLinkChunk);
  return t.i < g.Vh;
}

}  // namespace lqcd
