// Conversion between the natural (lexicographic, array-of-structures) layout
// callers hold and the parity-split structure-of-arrays layout the kernels
// stream (Sec. 4.1 stores fields as one array per colour component for the
// same reason: consecutive sites are consecutive in memory).  The 12-real
// link format keeps rows 0 and 1 only; row 2 is rebuilt from them.
#include "common.h"
#include "su3.h"

namespace lqcd {

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__device__ __forceinline__ double2 det3(const Su3<double>& u) {
  const double2 m0 = csub<double>(cmul<double>(u.e[4], u.e[8]), cmul<double>(u.e[5], u.e[7]));
  const double2 m1 = csub<double>(cmul<double>(u.e[3], u.e[8]), cmul<double>(u.e[5], u.e[6]));
  const double2 m2 = csub<double>(cmul<double>(u.e[3], u.e[7]), cmul<double>(u.e[4], u.e[6]));
  double2 d = cmul<double>(u.e[0], m0);
  const double2 t1 = cmul<double>(u.e[1], m1), t2 = cmul<double>(u.e[2], m2);
  d.x += t2.x - t1.x;
  d.y += t2.y - t1.y;
  return d;
}

// Writes the stored elements of the full matrix u (link h of one [parity][mu]
// block at `block`): 9 or 6 as is, 7 = rows 0-1 and det u, 8 = rows 0-1 of
// exp(-i theta) u and theta = arg(det u) / 3 (rounded to R first, so that the
// stored rows and angle rebuild u).
template <typename R, int NE>
__device__ __forceinline__ void store_link(const Su3<double>& u, cplx<R>* block, int h, int Vh) {
  cplx<R>* dst = block + h;
  if constexpr (NE == 8) {
    const double2 d = det3(u);
    const R th = R(atan2(d.y, d.x) / 3.0);
    double sn, cs;
    sincos(double(th), &sn, &cs);
    const double2 ph = make_double2(cs, -sn);
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const double2 w = cmul<double>(ph, u.e[e]);
      dst[int64_t(e) * Vh] = mk<R>((R)w.x, (R)w.y);
    }
    reinterpret_cast<R*>(block + int64_t(6) * Vh)[h] = th;
  } else {
#pragma unroll
    for (int e = 0; e < (NE == 7 ? 6 : NE); ++e)
      dst[int64_t(e) * Vh] = mk<R>((R)u.e[e].x, (R)u.e[e].y);
    if constexpr (NE == 7) {
      const double2 d = det3(u);
      dst[int64_t(6) * Vh] = mk<R>((R)d.x, (R)d.y);
    }
  }
}

// natural complex128 [4][V][3][3] -> packed [2][4][NE][Vh] of R
template <typename R, int NE>
__global__ void __launch_bounds__(kBlock) k_pack_links(KGeom g, const double2* __restrict__ nat,
                                                       cplx<R>* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t V = int64_t(2) * g.Vh;
  if (i >= 4 * V) return;
  const int mu = int(i / V);
  const int lex = int(i % V);
  int r = lex;
  const int x = r % g.Lx;
  r /= g.Lx;
  const int y = r % g.Ly;
  r /= g.Ly;
  const int z = r % g.Lz;
  const int t = r / g.Lz;
  const int par = (x + y + z + t) & 1;
  const int h = lex >> 1;
  const double2* src = nat + i * 9;
  Su3<double> u;
#pragma unroll
  for (int e = 0; e < 9; ++e) u.e[e] = src[e];
  store_link<R, NE>(u, out + (int64_t(par) * 4 + mu) * link_block<NE>(g.Vh), h, g.Vh);
}

// packed FP64 18-real SU(3) links and natural FP64 angles [4][V] -> packed
// LQCD_LINKS12T of R (rows 0-1 of U as they are, the angle per link)
template <typename R>
__global__ void __launch_bounds__(kBlock) k_pack_links_u1(KGeom g, const double2* __restrict__ U,
                                                          const double* __restrict__ theta,
                                                          cplx<R>* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(8) * g.Vh) return;
  const int pm = int(i / g.Vh);
  const int h = int(i % g.Vh);
  const int par = pm >> 2, mu = pm & 3;
  const Site s = decode_site(g, h, par);
  const int64_t lex = int64_t(2) * h + (s.x & 1);
  const double2* src = U + int64_t(pm) * 9 * g.Vh + h;
  cplx<R>* block = out + int64_t(pm) * link_block<8>(g.Vh);
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const double2 v = src[int64_t(e) * g.Vh];
    block[int64_t(e) * g.Vh + h] = mk<R>((R)v.x, (R)v.y);
  }
  reinterpret_cast<R*>(block + int64_t(6) * g.Vh)[h] = R(theta[int64_t(mu) * 2 * g.Vh + lex]);
}

// packed F64-18 -> natural complex128
__global__ void __launch_bounds__(kBlock) k_unpack_links(KGeom g, const double2* __restrict__ in,
                                                         double2* __restrict__ nat) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t V = int64_t(2) * g.Vh;
  if (i >= 4 * V) return;
  const int mu = int(i / V);
  const int lex = int(i % V);
  int r = lex;
  const int x = r % g.Lx;
  r /= g.Lx;
  const int y = r % g.Ly;
  r /= g.Ly;
  const int z = r % g.Lz;
  const int t = r / g.Lz;
  const int par = (x + y + z + t) & 1;
  const int h = lex >> 1;
  const double2* src = in + (int64_t(par) * 4 + mu) * 9 * g.Vh + h;
  double2* dst = nat + i * 9;
#pragma unroll
  for (int e = 0; e < 9; ++e) dst[e] = src[int64_t(e) * g.Vh];
}

// packed (RS, NS) -> packed (RD, ND); one thread per (parity, mu, half index)
template <typename RS, int NS, typename RD, int ND>
__global__ void __launch_bounds__(kBlock) k_convert_links(int Vh, const cplx<RS>* __restrict__ in,
                                                          cplx<RD>* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(8) * Vh) return;
  const int64_t pm = i / Vh;  // parity*4 + mu
  const int h = int(i % Vh);
  Su3<double> u;
  const cplx<RS>* blk = in + pm * link_block<NS>(Vh);
#pragma unroll
  for (int e = 0; e < stored_planes<NS>(); ++e) {
    const cplx<RS> v = blk[int64_t(e) * Vh + h];
    u.e[e] = mk<double>((double)v.x, (double)v.y);
  }
  complete_link<double, NS>(u);
  if constexpr (NS == 8)
    apply_u1<double>(u, (double)reinterpret_cast<const RS*>(blk + int64_t(6) * Vh)[h]);
  store_link<RD, ND>(u, out + pm * link_block<ND>(Vh), h, Vh);
}

// natural complex128 [nrhs][V][3] -> packed [nrhs][3][Vh] of R, one parity
template <typename R>
__global__ void __launch_bounds__(kBlock) k_pack_spinor(KGeom g, int par, int nrhs,
                                                        const double2* __restrict__ nat,
                                                        cplx<R>* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(nrhs) * g.Vh) return;
  const int rhs = int(i / g.Vh);
  const int h = int(i % g.Vh);
  const Site s = decode_site(g, h, par);
  const int64_t lex = int64_t(2) * h + (s.x & 1);
  const double2* src = nat + (int64_t(rhs) * 2 * g.Vh + lex) * 3;
  cplx<R>* dst = out + int64_t(rhs) * 3 * g.Vh + h;
#pragma unroll
  for (int c = 0; c < 3; ++c) dst[int64_t(c) * g.Vh] = mk<R>((R)src[c].x, (R)src[c].y);
}

// packed [nrhs][3][Vh] -> natural [nrhs][V][3], other parity zero
template <typename R>
__global__ void __launch_bounds__(kBlock) k_unpack_spinor(KGeom g, int par, int nrhs,
                                                          const cplx<R>* __restrict__ in,
                                                          double2* __restrict__ nat) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t V = int64_t(2) * g.Vh;
  if (i >= int64_t(nrhs) * V) return;
  const int rhs = int(i / V);
  const int lex = int(i % V);
  int r = lex;
  const int x = r % g.Lx;
  r /= g.Lx;
  const int y = r % g.Ly;
  r /= g.Ly;
  const int z = r % g.Lz;
  const int t = r / g.Lz;
  double2* dst = nat + i * 3;
  if (((x + y + z + t) & 1) != par) {
#pragma unroll
    for (int c = 0; c < 3; ++c) dst[c] = make_double2(0.0, 0.0);
    return;
  }
  const cplx<R>* src = in + int64_t(rhs) * 3 * g.Vh + (lex >> 1);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cplx<R> v = src[int64_t(c) * g.Vh];
    dst[c] = make_double2((double)v.x, (double)v.y);
  }
}

}  // namespace

namespace {

template <typename RS, int NS, typename RD, int ND>
void conv_launch(const KGeom& k, const void* src, void* dst, hipStream_t st) {
  hipLaunchKernelGGL((k_convert_links<RS, NS, RD, ND>), dim3(grid_for(int64_t(8) * k.Vh)),
                     dim3(kBlock), 0, st, k.Vh, (const cplx<RS>*)src, (cplx<RD>*)dst);
}

// the element-count template argument of a link format (8: rows 0-1 and the angle)
inline int ne_of(int fmt) {
  return fmt == LQCD_LINKS12 ? 6 : fmt == LQCD_LINKS12D ? 7 : fmt == LQCD_LINKS12T ? 8 : 9;
}

template <typename RS, int NS, typename RD>
void conv_ne(const KGeom& k, const void* src, void* dst, int df, hipStream_t st) {
  switch (ne_of(df)) {
    case 6: conv_launch<RS, NS, RD, 6>(k, src, dst, st); break;
    case 7: conv_launch<RS, NS, RD, 7>(k, src, dst, st); break;
    case 8: conv_launch<RS, NS, RD, 8>(k, src, dst, st); break;
    default: conv_launch<RS, NS, RD, 9>(k, src, dst, st); break;
  }
}

template <typename RS, int NS>
void conv_dst(const KGeom& k, const void* src, void* dst, int dp, int df, hipStream_t st) {
  if (dp == LQCD_F64)
    conv_ne<RS, NS, double>(k, src, dst, df, st);
  else
    conv_ne<RS, NS, float>(k, src, dst, df, st);
}

template <typename RS>
void conv_src(const KGeom& k, const void* src, int sf, void* dst, int dp, int df,
              hipStream_t st) {
  switch (ne_of(sf)) {
    case 6: conv_dst<RS, 6>(k, src, dst, dp, df, st); break;
    case 7: conv_dst<RS, 7>(k, src, dst, dp, df, st); break;
    case 8: conv_dst<RS, 8>(k, src, dst, dp, df, st); break;
    default: conv_dst<RS, 9>(k, src, dst, dp, df, st); break;
  }
}

}  // namespace

int convert_links_async(const KGeom& k, const void* src, int sp, int sf, void* dst, int dp,
                        int df, hipStream_t st) {
  if (sp == LQCD_F64)
    conv_src<double>(k, src, sf, dst, dp, df, st);
  else
    conv_src<float>(k, src, sf, dst, dp, df, st);
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

}  // namespace lqcd

using namespace lqcd;

extern "C" {

int lqcd_pack_links(const lqcd_geom* g, const void* U_nat, int prec, int fmt, void* U_packed,
                    void* stream) {
  clear_error();
  int st;
  if ((st = check_geom(g)) || (st = check_prec_fmt(prec, fmt)) ||
      (st = check_ptr(U_nat, "U_nat")) || (st = check_ptr(U_packed, "U_packed")))
    return st;
  const KGeom k = make_kgeom(g);
  const unsigned grid = grid_for(int64_t(8) * k.Vh);
  hipStream_t s = (hipStream_t)stream;
  const double2* src = (const double2*)U_nat;
#define LQCD_PACK(R, NE)                                                                  \
  hipLaunchKernelGGL((k_pack_links<R, NE>), dim3(grid), dim3(kBlock), 0, s, k, src,       \
                     (cplx<R>*)U_packed)
  const int ne = ne_of(fmt);
  if (prec == LQCD_F64) {
    if (ne == 9) LQCD_PACK(double, 9);
    else if (ne == 6) LQCD_PACK(double, 6);
    else if (ne == 7) LQCD_PACK(double, 7);
    else LQCD_PACK(double, 8);
  } else {
    if (ne == 9) LQCD_PACK(float, 9);
    else if (ne == 6) LQCD_PACK(float, 6);
    else if (ne == 7) LQCD_PACK(float, 7);
    else LQCD_PACK(float, 8);
  }
#undef LQCD_PACK
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

int lqcd_pack_links_u1(const lqcd_geom* g, const void* U64, const double* theta, int prec,
                       void* out, void* stream) {
  clear_error();
  int st;
  if ((st = check_geom(g)) || (st = check_prec_fmt(prec, LQCD_LINKS12T)) ||
      (st = check_ptr(U64, "U64")) || (st = check_ptr(theta, "theta")) ||
      (st = check_ptr(out, "out")))
    return st;
  if (out == U64 || static_cast<const void*>(theta) == out) {
    set_error("lqcd_pack_links_u1: out must not alias U64 or theta");
    return LQCD_ERR_INVALID_ARG;
  }
  const KGeom k = make_kgeom(g);
  const unsigned grid = grid_for(int64_t(8) * k.Vh);
  hipStream_t s = (hipStream_t)stream;
  if (prec == LQCD_F64)
    hipLaunchKernelGGL(k_pack_links_u1<double>, dim3(grid), dim3(kBlock), 0, s, k,
                       (const double2*)U64, theta, (double2*)out);
  else
    hipLaunchKernelGGL(k_pack_links_u1<float>, dim3(grid), dim3(kBlock), 0, s, k,
                       (const double2*)U64, theta, (float2*)out);
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

int lqcd_convert_links(const lqcd_geom* g, const void* src, int src_prec, int src_fmt, void* dst,
                       int dst_prec, int dst_fmt, void* stream) {
  clear_error();
  int st;
  if ((st = check_geom(g)) || (st = check_prec_fmt(src_prec, src_fmt)) ||
      (st = check_prec_fmt(dst_prec, dst_fmt)) || (st = check_ptr(src, "src")) ||
      (st = check_ptr(dst, "dst")))
    return st;
  if (src == dst) {
    set_error("convert_links: src and dst must be different buffers");
    return LQCD_ERR_INVALID_ARG;
  }
  return convert_links_async(make_kgeom(g), src, src_prec, src_fmt, dst, dst_prec, dst_fmt,
                             (hipStream_t)stream);
}

int lqcd_unpack_links(const lqcd_geom* g, const void* U_packed, void* U_nat, void* stream) {
  clear_error();
  int st;
  if ((st = check_geom(g)) || (st = check_ptr(U_packed, "U_packed")) ||
      (st = check_ptr(U_nat, "U_nat")))
    return st;
  const KGeom k = make_kgeom(g);
  hipLaunchKernelGGL(k_unpack_links, dim3(grid_for(int64_t(8) * k.Vh)), dim3(kBlock), 0,
                     (hipStream_t)stream, k, (const double2*)U_packed, (double2*)U_nat);
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

int lqcd_pack_spinor(const lqcd_geom* g, int parity, int prec, const void* nat, void* packed,
                     int32_t nrhs, void* stream) {
  clear_error();
  int st;
  if ((st = check_geom(g)) || (st = check_prec_fmt(prec, LQCD_LINKS18)) ||
      (st = check_ptr(nat, "nat")) || (st = check_ptr(packed, "packed")) ||
      (st = check_nrhs(nrhs)))
    return st;
  if (parity != 0 && parity != 1) {
    set_error("parity must be 0 or 1, got %d", parity);
    return LQCD_ERR_INVALID_ARG;
  }
  const KGeom k = make_kgeom(g);
  const unsigned grid = grid_for(int64_t(nrhs) * k.Vh);
  hipStream_t s = (hipStream_t)stream;
  if (prec == LQCD_F64)
    hipLaunchKernelGGL(k_pack_spinor<double>, dim3(grid), dim3(kBlock), 0, s, k, parity, nrhs,
                       (const double2*)nat, (double2*)packed);
  else
    hipLaunchKernelGGL(k_pack_spinor<float>, dim3(grid), dim3(kBlock), 0, s, k, parity, nrhs,
                       (const double2*)nat, (float2*)packed);
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

int lqcd_unpack_spinor(const lqcd_geom* g, int parity, int prec, const void* packed, void* nat,
                       int32_t nrhs, void* stream) {
  clear_error();
  int st;
  if ((st = check_geom(g)) || (st = check_prec_fmt(prec, LQCD_LINKS18)) ||
      (st = check_ptr(nat, "nat")) || (st = check_ptr(packed, "packed")) ||
      (st = check_nrhs(nrhs)))
    return st;
  if (parity != 0 && parity != 1) {
    set_error("parity must be 0 or 1, got %d", parity);
    return LQCD_ERR_INVALID_ARG;
  }
  const KGeom k = make_kgeom(g);
  const unsigned grid = grid_for(int64_t(nrhs) * 2 * k.Vh);
  hipStream_t s = (hipStream_t)stream;
  if (prec == LQCD_F64)
    hipLaunchKernelGGL(k_unpack_spinor<double>, dim3(grid), dim3(kBlock), 0, s, k, parity, nrhs,
                       (const double2*)packed, (double2*)nat);
  else
    hipLaunchKernelGGL(k_unpack_spinor<float>, dim3(grid), dim3(kBlock), 0, s, k, parity, nrhs,
                       (const float2*)packed, (double2*)nat);
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

}  // extern "C"
