// 3x3 complex matrices held in registers, and the link loads of the packed
// layouts.
#pragma once

#include "common.h"

namespace lqcd {

template <typename R>
struct Su3 {
  cplx<R> e[9];  // row-major: e[3*row + col]
};

template <typename R>
__device__ __forceinline__ cplx<R> conj_of(cplx<R> a) { return mk<R>(a.x, -a.y); }

// Row 2 of an SU(3) matrix is the complex conjugate of the cross product of
// rows 0 and 1 (Sec. 4.1, gauge link compression).
template <typename R>
__device__ __forceinline__ void reconstruct_row2(Su3<R>& u) {
  u.e[6] = conj_of<R>(csub<R>(cmul<R>(u.e[1], u.e[5]), cmul<R>(u.e[2], u.e[4])));
  u.e[7] = conj_of<R>(csub<R>(cmul<R>(u.e[2], u.e[3]), cmul<R>(u.e[0], u.e[5])));
  u.e[8] = conj_of<R>(csub<R>(cmul<R>(u.e[0], u.e[4]), cmul<R>(u.e[1], u.e[3])));
}

// Row 2 of a unitary link from rows 0 and 1 and d = det U (element 6 of the
// 7-element format): for V = e^{i phi} W, W in SU(3), row 2 = d conj(row0 x
// row1); d = 1 is reconstruct_row2.  Serves links that carry U(1) phases.
template <typename R>
__device__ __forceinline__ void reconstruct_row2_det(Su3<R>& u) {
  const cplx<R> d = u.e[6];
  const cplx<R> c0 = conj_of<R>(csub<R>(cmul<R>(u.e[1], u.e[5]), cmul<R>(u.e[2], u.e[4])));
  const cplx<R> c1 = conj_of<R>(csub<R>(cmul<R>(u.e[2], u.e[3]), cmul<R>(u.e[0], u.e[5])));
  const cplx<R> c2 = conj_of<R>(csub<R>(cmul<R>(u.e[0], u.e[4]), cmul<R>(u.e[1], u.e[3])));
  u.e[6] = cmul<R>(d, c0);
  u.e[7] = cmul<R>(d, c1);
  u.e[8] = cmul<R>(d, c2);
}

// NE = 8 names the U(1)-angle format (LQCD_LINKS12T): rows 0-1 of the SU(3)
// part as six complex planes, then the angle theta as one plane of reals.
// Complex planes holding stored elements, and complex numbers in one
// [parity][mu] block of Vh links (Vh is a multiple of 8).
template <int NE>
__host__ __device__ constexpr int stored_planes() { return NE == 8 ? 6 : NE; }
template <int NE>
__host__ __device__ __forceinline__ int64_t link_block(int Vh) {
  return NE == 8 ? int64_t(13) * (Vh / 2) : int64_t(NE) * Vh;
}

// The full matrix from the stored elements (9: as is; 6: SU(3) rows 0-1;
// 7: rows 0-1 and the determinant; 8: the SU(3) part of rows 0-1, whose
// U(1) factor apply_u1 adds).
template <typename R, int NE>
__device__ __forceinline__ void complete_link(Su3<R>& u) {
  if constexpr (NE == 6 || NE == 8) reconstruct_row2<R>(u);
  if constexpr (NE == 7) reconstruct_row2_det<R>(u);
}

// u <- (cos theta + i sin theta) u: the U(1) phase recomputed from its angle
// (Sec. 4.1), with the library's sincos.
template <typename R>
__device__ __forceinline__ void apply_u1(Su3<R>& u, R theta) {
  R sn, cs;
  if constexpr (sizeof(R) == 4)
    sincosf(theta, &sn, &cs);
  else
    sincos(theta, &sn, &cs);
  const cplx<R> ph = mk<R>(cs, sn);
#pragma unroll
  for (int e = 0; e < 9; ++e) u.e[e] = cmul<R>(ph, u.e[e]);
}

// Buffer resources: a scalar 64-bit base and byte range for a whole array
// block, so that each load needs one 32-bit per-lane offset (shared by every
// element and colour) plus a scalar offset.  Reads outside [0, bytes) return
// zero instead of touching memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_res(const void* base, uint32_t bytes) {
  // dword 3 of the descriptor for untyped 32-bit access on CDNA
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, int(bytes), 0x00020000);
}

// AUX: cache policy bits of the load (2: non-temporal)
template <typename R, int AUX = 0>
__device__ __forceinline__ cplx<R> ld_buf(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(R) == 4)
    return __builtin_bit_cast(cplx<R>, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
  else
    return __builtin_bit_cast(cplx<R>, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX));
}

// One real through a buffer resource (the angle plane of LQCD_LINKS12T).
template <typename R, int AUX = 0>
__device__ __forceinline__ R ld_buf_real(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(R) == 4)
    return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
  else
    return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
}

// Two single-precision complex values stored next to each other (the same
// element of two right-hand sides kept as an interleaved pair) in one 16-byte
// buffer load: a holds the first, b the second.
template <int AUX = 0>
__device__ __forceinline__ void ld_buf_pair(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                            uint32_t soff, cplx<float>& a, cplx<float>& b) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const f4 v = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX));
  a = mk<float>(v.x, v.y);
  b = mk<float>(v.z, v.w);
}

// Streaming 16-byte access to such a pair (p 16-byte aligned); NT as below.
template <bool NT>
__device__ __forceinline__ void ld_once_pair(const cplx<float>* p, cplx<float>& a,
                                             cplx<float>& b) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const f4* q = reinterpret_cast<const f4*>(p);
  const f4 v = NT ? __builtin_nontemporal_load(q) : *q;
  a = mk<float>(v.x, v.y);
  b = mk<float>(v.z, v.w);
}

template <bool NT>
__device__ __forceinline__ void st_once_pair(cplx<float>* p, cplx<float> a, cplx<float> b) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  f4 v;
  v.x = a.x;
  v.y = a.y;
  v.z = b.x;
  v.w = b.y;
  if constexpr (NT)
    __builtin_nontemporal_store(v, reinterpret_cast<f4*>(p));
  else
    *reinterpret_cast<f4*>(p) = v;
}

// Streaming access to a complex value that is read or written once: the
// non-temporal hint lets the caches evict it first.  NT = false is a plain access.
template <typename R, bool NT>
__device__ __forceinline__ cplx<R> ld_once(const cplx<R>* p) {
  if constexpr (!NT) {
    return *p;
  } else if constexpr (sizeof(R) == 4) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    const f2 v = __builtin_nontemporal_load(reinterpret_cast<const f2*>(p));
    return mk<R>(v.x, v.y);
  } else {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 v = __builtin_nontemporal_load(reinterpret_cast<const d2*>(p));
    return mk<R>(v.x, v.y);
  }
}

template <typename R, bool NT>
__device__ __forceinline__ void st_once(cplx<R>* p, cplx<R> z) {
  if constexpr (!NT) {
    *p = z;
  } else if constexpr (sizeof(R) == 4) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    f2 v;
    v.x = z.x;
    v.y = z.y;
    __builtin_nontemporal_store(v, reinterpret_cast<f2*>(p));
  } else {
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2 v;
    v.x = z.x;
    v.y = z.y;
    __builtin_nontemporal_store(v, reinterpret_cast<d2*>(p));
  }
}

// Load the link with half index h from one packed [parity][mu] block.
template <typename R, int NE>
__device__ __forceinline__ void load_link(const cplx<R>* __restrict__ base, int h, int Vh,
                                          Su3<R>& u) {
#pragma unroll
  for (int e = 0; e < stored_planes<NE>(); ++e) u.e[e] = base[int64_t(e) * Vh + h];
  complete_link<R, NE>(u);
  if constexpr (NE == 8) apply_u1<R>(u, reinterpret_cast<const R*>(base + int64_t(6) * Vh)[h]);
}

// y = U v
template <typename R>
__device__ __forceinline__ void mat_vec(const Su3<R>& u, const cplx<R> v[3], cplx<R> y[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    y[a] = cmul<R>(u.e[3 * a], v[0]);
    cfma<R>(y[a], u.e[3 * a + 1], v[1]);
    cfma<R>(y[a], u.e[3 * a + 2], v[2]);
  }
}

// y = U^dag v
template <typename R>
__device__ __forceinline__ void adj_mat_vec(const Su3<R>& u, const cplx<R> v[3], cplx<R> y[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    y[a] = cmulc<R>(u.e[a], v[0]);
    cfmac<R>(y[a], u.e[3 + a], v[1]);
    cfmac<R>(y[a], u.e[6 + a], v[2]);
  }
}

}  // namespace lqcd
