// D_oe / D_eo (Sec. 2) for eight right-hand sides on the matrix cores: the
// contraction of each hop, a 3x3 complex link times the 3x8 complex block of
// the eight right-hand sides' neighbour spinors, as a real 6x6 by 6x8 product
// on v_mfma_f32_4x4x1_16b_f32 (sixteen independent 4x4x1 products per wave).
//
// One quad of lanes per output site (16 sites per wave): quad block b is
// lanes 4b..4b+3, and the instruction takes A[i] from lane 4b + i, B[j] from
// lane 4b + j and accumulates D[i][j] in register i of lane 4b + j.  With
//   rows  r = 0..5 of the output: Re y_0..2, Im y_0..2 (6, 7 padding),
//   k     = 0..5 of the input:    Re v_0..2, Im v_0..2,
//   cols  = the eight right-hand sides,
// a hop adds c U v, i.e. A = c [[Re U, -Im U], [Im U, Re U]] (rows r, cols k)
// times B = v (rows k, cols RHS): two row tiles x two RHS tiles x six k steps,
// 24 instructions per hop.  Lane q of a quad feeds rows q and 4 + q of A and
// right-hand sides q and 4 + q of B, and ends with the output of those two
// right-hand sides.  The hop coefficients (staggered phase, boundary sign,
// 1/2, sign of the backward hop) are folded into A.  FP32, 12-real links,
// plain mode only: the variant exists to measure the matrix cores against the
// VALU stencil on the same work.
#include <hip/hip_runtime.h>

#include "dslash.h"
#include "su3.h"

namespace lqcd {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// Real and imaginary rows of the real form [[Re U, -Im U], [Im U, Re U]] at
// input component k (k < 3: Re v_k, else Im v_{k-3}) for the complex entry z.
template <int K>
__device__ __forceinline__ float re_row(float2 z) { return K < 3 ? z.x : -z.y; }
template <int K>
__device__ __forceinline__ float im_row(float2 z) { return K < 3 ? z.y : z.x; }

// One k step of a hop: rows q and 4 + q of c A (lane q of the quad; rows 0-2
// are the real rows of U's rows 0-2, row 3 the imaginary row of U's row 0,
// rows 4-5 the imaginary rows of U's rows 1-2, rows 6-7 zero), component K of
// right-hand sides q and 4 + q.
template <int K>
__device__ __forceinline__ void step(const Su3<float>& u, const float2 (&v)[2][3], float c,
                                     int q, f4 (&acc)[2][2]) {
  constexpr int kk = K < 3 ? K : K - 3;
  const float2 u0 = u.e[kk], u1 = u.e[3 + kk], u2 = u.e[6 + kk];
  const float r0 = q == 0 ? re_row<K>(u0)
                 : q == 1 ? re_row<K>(u1)
                 : q == 2 ? re_row<K>(u2)
                          : im_row<K>(u0);
  const float r1 = q == 0 ? im_row<K>(u1) : q == 1 ? im_row<K>(u2) : 0.f;
  const float a0 = c * r0, a1 = c * r1;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const float bv = K < 3 ? v[t][kk].x : v[t][kk].y;
    acc[0][t] = __builtin_amdgcn_mfma_f32_4x4x1f32(a0, bv, acc[0][t], 0, 0, 0);
    acc[1][t] = __builtin_amdgcn_mfma_f32_4x4x1f32(a1, bv, acc[1][t], 0, 0, 0);
  }
}

template <int B>
__global__ void __launch_bounds__(256) k_dslash_mfma(const DslashCall a, const int xcd,
                                                     const int tz, const int ty) {
  if (a.halt && *a.halt) return;
  const KGeom& g = a.g;
  const int lb = xcd_block(blockIdx.x, gridDim.x, xcd);
  const int rhs0 = blockIdx.y * B;
  const int q = threadIdx.x & 3;  // lane within the site's quad
  const int idx0 = lb * (int(blockDim.x) >> 2) + (int(threadIdx.x) >> 2);
  // every lane stays active through the matrix instructions; quads past the
  // lattice compute the last site again and store nothing
  const bool valid = idx0 < g.Vh;
  const int idx = valid ? idx0 : g.Vh - 1;
  // the site traversal of k_dslash: (y, z) tiles, t inside the tile
  int h = idx;
  if (tz) {
    const int tyy = ty ? ty : g.Ly;
    const int row = g.Lxh * tyy;
    const int inrow = idx % row;
    int r = idx / row;
    const int zi = r % tz;
    r /= tz;
    const int t = r % g.Lt;
    const int tile = r / g.Lt;
    const int nty = g.Ly / tyy;
    h = inrow + g.Lxh * ((tile % nty) * tyy) + g.sz * ((tile / nty) * tz + zi) + g.st * t;
  }
  const Site s = decode_site(g, h, a.out_par);

  const int64_t par_stride = int64_t(4) * 6 * g.Vh;
  const float2* Uout = static_cast<const float2*>(a.U) + a.out_par * par_stride;
  const float2* Uin = static_cast<const float2*>(a.U) + (1 - a.out_par) * par_stride;
  constexpr uint32_t cb = sizeof(float2);
  const uint32_t link_bytes = 6u * uint32_t(g.Vh) * cb;
  const uint32_t csoff = uint32_t(g.Vh) * cb;
  // this lane's two right-hand sides q and 4 + q of the group (rows past nrhs
  // alias the last one: loaded and computed, never stored)
  int jr[2];
  __amdgpu_buffer_rsrc_t rin[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int j = rhs0 + 4 * t + q;
    jr[t] = j < a.nrhs ? j : a.nrhs - 1;
    rin[t] = make_res(static_cast<const float2*>(a.in) + int64_t(jr[t]) * a.in_stride,
                      3u * uint32_t(g.Vh) * cb);
  }
  f4 acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) acc[m][n] = f4{0.f, 0.f, 0.f, 0.f};

#pragma unroll 1
  for (int k8 = 0; k8 < 8; ++k8) {
    const int mu = k8 >> 1;
    const bool fw = (k8 & 1) == 0;
    // neighbour and phase from the coordinates (a per-hop table would be
    // indexed dynamically and live in scratch)
    int nbr;
    if (mu == 0) {
      const int xn = fw ? (s.x + 1 == g.Lx ? 0 : s.x + 1) : (s.x == 0 ? g.Lx - 1 : s.x - 1);
      nbr = h - (s.x >> 1) + (xn >> 1);
    } else {
      const int L = mu == 1 ? g.Ly : (mu == 2 ? g.Lz : g.Lt);
      const int sd = mu == 1 ? g.sy : (mu == 2 ? g.sz : g.st);
      const int cm = mu == 1 ? s.y : (mu == 2 ? s.z : s.t);
      nbr = fw ? h + (cm + 1 == L ? -(L - 1) * sd : sd) : h + (cm == 0 ? (L - 1) * sd : -sd);
    }
    const int ep = ((mu >= 1 ? s.x : 0) + (mu >= 2 ? s.y : 0) + (mu >= 3 ? s.z : 0)) & 1;
    float c = ep ? -0.5f : 0.5f;
    if (mu == 3 && g.anti && (fw ? s.t == g.Lt - 1 : s.t == 0)) c = -c;
    if (!fw) c = -c;
    const __amdgpu_buffer_rsrc_t rl =
        make_res((fw ? Uout : Uin) + int64_t(mu) * 6 * g.Vh, link_bytes);
    const uint32_t ol = uint32_t(fw ? h : nbr) * cb, on = uint32_t(nbr) * cb;
    Su3<float> u;
#pragma unroll
    for (int e = 0; e < 6; ++e) u.e[e] = ld_buf<float, 2>(rl, ol, uint32_t(e) * csoff);
    float2 v[2][3];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) v[t][cc] = ld_buf<float>(rin[t], on, uint32_t(cc) * csoff);
    complete_link<float, 6>(u);
    if (!fw) {  // U^dag
      const Su3<float> t = u;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) u.e[3 * i + j] = conj_of<float>(t.e[3 * j + i]);
    }
    step<0>(u, v, c, q, acc);
    step<1>(u, v, c, q, acc);
    step<2>(u, v, c, q, acc);
    step<3>(u, v, c, q, acc);
    step<4>(u, v, c, q, acc);
    step<5>(u, v, c, q, acc);
  }
  // lane q holds rows 0..3 (tile 0) and 4..7 (tile 1) of right-hand sides q, 4 + q
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int j = rhs0 + 4 * t + q;
    if (!valid || j >= a.nrhs || (a.live != nullptr && a.live[j * a.live_stride] == 0)) continue;
    float2* out = static_cast<float2*>(a.out) + int64_t(j) * a.out_stride + h;
    const float re[3] = {acc[0][t][0], acc[0][t][1], acc[0][t][2]};
    const float im[3] = {acc[0][t][3], acc[1][t][0], acc[1][t][1]};
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
      st_once<float, true>(out + int64_t(cc) * g.Vh, mk<float>(re[cc], im[cc]));
  }
}

}  // namespace

bool dslash_mfma_supported(const DslashCall& c, const DslashCfg& cfg) {
  return cfg.mf == 1 && !c.pairs && c.prec == LQCD_F32 && c.fmt == LQCD_LINKS12 && c.mode == DM_PLAIN &&
         c.partials == nullptr && cfg.rhs_block == 8 && cfg.tm == 0 &&
         (cfg.block == 64 || cfg.block == 128 || cfg.block == 256) &&
         (cfg.tz == 0 || c.g.Lz % cfg.tz == 0) && (cfg.ty == 0 || c.g.Ly % cfg.ty == 0);
}

int dslash_mfma_launch(const DslashCall& c, const DslashCfg& cfg, hipStream_t st) {
  if (!dslash_mfma_supported(c, cfg)) {
    set_error("matrix-core stencil not available for this call (FP32, 12-real, plain, 8 RHS)");
    return LQCD_ERR_UNSUPPORTED;
  }
  const int sites = cfg.block / 4;
  const dim3 grid(unsigned((c.g.Vh + sites - 1) / sites), unsigned((c.nrhs + 7) / 8));
  hipLaunchKernelGGL(k_dslash_mfma<8>, grid, dim3(cfg.block), 0, st, c, cfg.xcd, cfg.tz, cfg.ty);
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

}  // namespace lqcd
