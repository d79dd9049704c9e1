// Internal definitions shared by the HIP sources of liblqcd.
//
// Packed layouts (see include/lqcd.h): spinors [rhs][3][Vh] and links
// [parity][mu][element][Vh], complex numbers stored as double2 / float2, so a
// wavefront reading one element for 64 consecutive half indices issues one
// fully coalesced 1 KiB (FP64) or 512 B (FP32) request.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/lqcd.h"

namespace lqcd {

// ----------------------------------------------------------------- complex

template <typename R> struct Cplx;
template <> struct Cplx<double> { using T = double2; };
template <> struct Cplx<float> { using T = float2; };
template <typename R> using cplx = typename Cplx<R>::T;

template <typename R>
__host__ __device__ __forceinline__ cplx<R> mk(R re, R im) {
  cplx<R> z;
  z.x = re;
  z.y = im;
  return z;
}
template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return mk<R>(a.x + b.x, a.y + b.y); }
template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return mk<R>(a.x - b.x, a.y - b.y); }
template <typename R>
__device__ __forceinline__ cplx<R> cscale(R s, cplx<R> a) { return mk<R>(s * a.x, s * a.y); }
// a * b, with the fused multiply-adds written out so that every kernel
// instantiation rounds the same way (right-hand-side batching is bitwise
// neutral)
template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return mk<R>(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
// conj(a) * b, rounded exactly as cmul(conj(a), b)
template <typename R>
__device__ __forceinline__ cplx<R> cmulc(cplx<R> a, cplx<R> b) {
  return mk<R>(fma(a.x, b.x, a.y * b.y), fma(a.x, b.y, -(a.y * b.x)));
}
// acc += a * b
template <typename R>
__device__ __forceinline__ void cfma(cplx<R>& acc, cplx<R> a, cplx<R> b) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}
// acc += conj(a) * b
template <typename R>
__device__ __forceinline__ void cfmac(cplx<R>& acc, cplx<R> a, cplx<R> b) {
  acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
}
template <typename R>
__device__ __forceinline__ double cnorm2(cplx<R> a) {
  return fma((double)a.x, (double)a.x, (double)a.y * (double)a.y);
}

// ----------------------------------------------------------------- geometry

struct KGeom {
  int Lx, Lxh, Ly, Lz, Lt;
  int Vh;        // sites per parity
  int sy, sz, st;  // half-index strides of y, z, t: Lxh, Lxh*Ly, Lxh*Ly*Lz
  int anti;      // antiperiodic time
};

KGeom make_kgeom(const lqcd_geom* g);

// Coordinates of the site with half index h and parity par.
struct Site {
  int x, y, z, t;
};

__device__ __forceinline__ Site decode_site(const KGeom& g, int h, int par) {
  Site s;
  int xh = h % g.Lxh;
  int r = h / g.Lxh;
  s.y = r % g.Ly;
  r /= g.Ly;
  s.z = r % g.Lz;
  s.t = r / g.Lz;
  s.x = 2 * xh + ((s.y + s.z + s.t + par) & 1);
  return s;
}

// Half indices of the eight neighbours x +- mu of a site with half index h.
// fwd[mu] = x + mu, bwd[mu] = x - mu, periodic wrap in every direction.
__device__ __forceinline__ void neighbours(const KGeom& g, const Site& s, int h, int fwd[4],
                                           int bwd[4]) {
  const int row = h - (s.x >> 1);  // half index of (0, y, z, t)
  const int xp = (s.x + 1 == g.Lx) ? 0 : s.x + 1;
  const int xm = (s.x == 0) ? g.Lx - 1 : s.x - 1;
  fwd[0] = row + (xp >> 1);
  bwd[0] = row + (xm >> 1);
  fwd[1] = h + ((s.y + 1 == g.Ly) ? -(g.Ly - 1) * g.sy : g.sy);
  bwd[1] = h + ((s.y == 0) ? (g.Ly - 1) * g.sy : -g.sy);
  fwd[2] = h + ((s.z + 1 == g.Lz) ? -(g.Lz - 1) * g.sz : g.sz);
  bwd[2] = h + ((s.z == 0) ? (g.Lz - 1) * g.sz : -g.sz);
  fwd[3] = h + ((s.t + 1 == g.Lt) ? -(g.Lt - 1) * g.st : g.st);
  bwd[3] = h + ((s.t == 0) ? (g.Lt - 1) * g.st : -g.st);
}

// eta_mu(x) = (-1)^(x_0 + ... + x_{mu-1})
__device__ __forceinline__ void staggered_eta(const Site& s, double eta[4]) {
  eta[0] = 1.0;
  eta[1] = (s.x & 1) ? -1.0 : 1.0;
  eta[2] = ((s.x + s.y) & 1) ? -1.0 : 1.0;
  eta[3] = ((s.x + s.y + s.z) & 1) ? -1.0 : 1.0;
}

// Blocks are handed to the 8 XCDs round robin; this maps the hardware block
// id to a logical one so that each XCD works on one contiguous slab of the
// lattice (its neighbour reads then stay mostly in its own L2).  It is a
// bijection on [0, nb) whatever the dispatch order, so correctness never
// depends on it.
__device__ __forceinline__ int xcd_block(int b, int nb, int enable) {
  if (!enable) return b;
  const int q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
  return x * q + (x < r ? x : r) + k;
}

// Deterministic block sum of one double: butterfly inside each 64-lane wave,
// then wave partials summed in order by thread 0.  The result is valid in
// thread 0 only.  All threads of the block must call it.
// This thread's share of sum_i p[i] over i = threadIdx.x + k blockDim.x < n,
// added in increasing i.  The loads of a batch of kBatch terms are issued
// before any is added, so a small workgroup reading partials that other
// XCDs just wrote waits for a few memory round trips rather than one per
// term; the order of the additions, and so the result, is the plain loop's.
__device__ __forceinline__ double strided_sum(const double* __restrict__ p, int n) {
  constexpr int kBatch = 16;
  double s = 0.0;
  for (int i0 = threadIdx.x; i0 < n; i0 += kBatch * blockDim.x) {
    double v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int i = i0 + u * int(blockDim.x);
      v[u] = i < n ? p[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (i0 + u * int(blockDim.x) < n) s += v[u];
  }
  return s;
}

// strided_sum of two arrays at once: the loads of both batches issue
// together, so the two reductions wait for one chain of memory round trips
// instead of two; each sum adds its terms in strided_sum's order (same bits).
__device__ __forceinline__ void strided_sum2(const double* __restrict__ p, int n,
                                             const double* __restrict__ q, int m, double* sp,
                                             double* sq) {
  constexpr int kBatch = 16;
  const int nm = n > m ? n : m;
  double s = 0.0, t = 0.0;
  for (int i0 = threadIdx.x; i0 < nm; i0 += kBatch * blockDim.x) {
    double v[kBatch], w[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int i = i0 + u * int(blockDim.x);
      v[u] = i < n ? p[i] : 0.0;
      w[u] = i < m ? q[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int i = i0 + u * int(blockDim.x);
      if (i < n) s += v[u];
      if (i < m) t += w[u];
    }
  }
  *sp = s;
  *sq = t;
}

__device__ __forceinline__ double block_sum(double v, double* lds) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += lds[i];
  }
  __syncthreads();
  return s;
}

// ----------------------------------------------------------------- host side

// Thread-local error detail, exposed through lqcd_last_error().
void set_error(const char* fmt, ...);
void clear_error();

struct Status {
  int code = LQCD_OK;
};

#define LQCD_HIP_TRY(expr)                                                              \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      ::lqcd::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                      \
      return LQCD_ERR_HIP;                                                              \
    }                                                                                   \
  } while (0)

#define LQCD_LAUNCH_CHECK() LQCD_HIP_TRY(hipGetLastError())

// Validation helpers (host only).  Each returns LQCD_OK or sets the error.
int check_geom(const lqcd_geom* g);
int check_prec_fmt(int prec, int fmt);
int check_ptr(const void* p, const char* name);
int check_nrhs(int32_t nrhs);

// Reals stored per link: 18, 12, 14 (rows 0-1 and the determinant) or 13
// (rows 0-1 and the U(1) angle).
inline size_t link_reals(int fmt) {
  return fmt == LQCD_LINKS12 ? 12 : fmt == LQCD_LINKS12D ? 14 : fmt == LQCD_LINKS12T ? 13 : 18;
}
inline size_t real_bytes(int prec) { return prec == LQCD_F32 ? 4 : 8; }

}  // namespace lqcd
