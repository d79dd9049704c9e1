// The hopping term D_oe / D_eo (Sec. 2) for a block of eight right-hand
// sides, marching along t.
//
// Each output site of the hop needs its two time neighbours x +- t, which sit
// in the same (x, y, z) column of the input parity: with half index
// h = col + t * st (col = xh + Lxh (y + Ly z)), the output at (col, t) reads
// the inputs at (col, t - 1) and (col, t + 1).  A thread that owns one column
// and walks Tc consecutive time slices therefore loads each input of its
// column once and keeps the last two in registers: the time hops never go
// back to L2, and the reuse distance of the spatial hops (x, y, z neighbours
// at the same slice, loaded by the neighbouring columns' threads) is one
// step of the march.  Links stream once, as in k_dslash.
//
// The eight right-hand sides of a column are split over P adjacent lanes of
// BL right-hand sides each (P * BL = 8): the lanes of a column load the same
// link element in one instruction, so each link still crosses HBM once per
// eight right-hand sides, while each lane holds only BL spinors per slice.
//
// The hops are accumulated in k_dslash's order (x, y, z, t; forward then
// backward) with the same products and fused multiply-adds, so the results
// are bit for bit those of every k_dslash configuration.
#include <hip/hip_runtime.h>

#include "dslash.h"
#include "su3.h"

namespace lqcd {

namespace {

template <typename R, int NE, int BL>
__device__ __forceinline__ void load_spinors(const __amdgpu_buffer_rsrc_t (&rin)[BL],
                                             uint32_t off, uint32_t csoff, cplx<R> (&v)[BL][3]) {
#pragma unroll
  for (int b = 0; b < BL; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c) v[b][c] = ld_buf<R>(rin[b], off, uint32_t(c) * csoff);
}

// acc[b] += coef * (u v[b]) for the lane's right-hand sides
template <typename R, int BL>
__device__ __forceinline__ void hop_acc(const Su3<R>& u, const cplx<R> (&v)[BL][3], R coef,
                                        cplx<R> (&acc)[BL][3]) {
#pragma unroll
  for (int b = 0; b < BL; ++b) {
    cplx<R> y[3];
    mat_vec<R>(u, v[b], y);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      acc[b][c].x = fma(coef, y[c].x, acc[b][c].x);
      acc[b][c].y = fma(coef, y[c].y, acc[b][c].y);
    }
  }
}

template <typename R, int NE>
__device__ __forceinline__ void load_link_buf(__amdgpu_buffer_rsrc_t rl, uint32_t off,
                                              uint32_t csoff, bool dagger, Su3<R>& u) {
#pragma unroll
  for (int e = 0; e < NE; ++e) u.e[e] = ld_buf<R, 2>(rl, off, uint32_t(e) * csoff);
  complete_link<R, NE>(u);
  if (dagger) {
    const Su3<R> t = u;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) u.e[3 * i + j] = conj_of<R>(t.e[3 * j + i]);
  }
}

// Grid: x = column blocks x time chunks (chunk-major), XCD remapped; y = groups
// of P * BL right-hand sides.  Thread = (column, lane of the column).
template <typename R, int NE, int P, int BL, int MODE>
__global__ void __launch_bounds__(256) k_dslash_tm(const DslashCall a, const int xcd,
                                                   const int tc, const int ncb) {
  constexpr int B = P * BL;
  __shared__ double lds[B][4];
  if (a.halt && *a.halt) return;
  const KGeom& g = a.g;
  const int lb = xcd_block(blockIdx.x, gridDim.x, xcd);
  const int cblk = lb % ncb, chunk = lb / ncb;
  const int rhs0 = blockIdx.y * B;
  const int part = int(threadIdx.x) % P;  // which BL right-hand sides of the group
  const int col = cblk * (int(blockDim.x) / P) + int(threadIdx.x) / P;
  const int ncol = g.st;  // columns = sites of one time slice of one parity

  bool lv[BL];
  bool any = false;
#pragma unroll
  for (int q = 0; q < B; ++q) {
    const int j = rhs0 + q;
    const bool l = j < a.nrhs && (a.live == nullptr || a.live[j * a.live_stride] != 0);
    any |= l;
    if (q / BL == part) lv[q % BL] = l;
  }
  if (!any) return;  // uniform over the block

  double nrm[BL];
#pragma unroll
  for (int b = 0; b < BL; ++b) nrm[b] = 0.0;

  if (col < ncol) {
    const int xh = col % g.Lxh;
    const int yz = col / g.Lxh;
    const int y = yz % g.Ly, z = yz / g.Ly;
    const int64_t par_stride = int64_t(4) * NE * g.Vh;
    const cplx<R>* Uout = static_cast<const cplx<R>*>(a.U) + a.out_par * par_stride;
    const cplx<R>* Uin = static_cast<const cplx<R>*>(a.U) + (1 - a.out_par) * par_stride;
    constexpr uint32_t cbytes = sizeof(cplx<R>);
    const uint32_t link_bytes = uint32_t(NE) * uint32_t(g.Vh) * cbytes;
    const uint32_t csoff = uint32_t(g.Vh) * cbytes;
    // this lane's right-hand sides; rows past nrhs alias the last one (loaded
    // and computed, never stored)
    int jrow[BL];
    __amdgpu_buffer_rsrc_t rin[BL];
#pragma unroll
    for (int b = 0; b < BL; ++b) {
      const int j = rhs0 + part * BL + b;
      jrow[b] = j < a.nrhs ? j : a.nrhs - 1;
      rin[b] = make_res(static_cast<const cplx<R>*>(a.in) + int64_t(jrow[b]) * a.in_stride,
                        3u * uint32_t(g.Vh) * cbytes);
    }
    // per right-hand side scalars of the fused updates
    R m2s[BL], alpha[BL];
    int slot_in[BL], slot_out[BL];
#pragma unroll
    for (int b = 0; b < BL; ++b) {
      m2s[b] = R(0);
      alpha[b] = R(0);
      slot_in[b] = slot_out[b] = jrow[b];
      if (MODE != DM_PLAIN) m2s[b] = R(a.m2s ? a.m2s[jrow[b] * a.m2s_stride] : a.m2s_c);
      if (MODE == DM_CG) {
        alpha[b] = R(a.alpha[jrow[b] * a.alpha_stride]);
        if (a.r_iter) {
          const int it = a.r_iter[jrow[b] * a.r_iter_stride];
          slot_in[b] = jrow[b] * a.r_slots + it % a.r_slots;
          slot_out[b] = jrow[b] * a.r_slots + (it + 1) % a.r_slots;
        }
      }
    }

    const int t0 = chunk * tc;
    cplx<R> prv[BL][3], cur[BL][3];
    load_spinors<R, NE, BL>(rin, uint32_t(col + (t0 == 0 ? g.Lt - 1 : t0 - 1) * g.st) * cbytes,
                            csoff, prv);
    load_spinors<R, NE, BL>(rin, uint32_t(col + t0 * g.st) * cbytes, csoff, cur);

#pragma unroll 1
    for (int k = 0; k < tc; ++k) {
      const int t = t0 + k;
      const int h = col + t * g.st;
      const int tn = t + 1 == g.Lt ? 0 : t + 1;
      const int tb = t == 0 ? g.Lt - 1 : t - 1;
      cplx<R> nxt[BL][3];
      load_spinors<R, NE, BL>(rin, uint32_t(col + tn * g.st) * cbytes, csoff, nxt);
      const int x = 2 * xh + ((y + z + t + a.out_par) & 1);

      cplx<R> acc[BL][3];
#pragma unroll
      for (int b = 0; b < BL; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[b][c] = mk<R>(0, 0);

      // x, y, z: forward then backward, one hop per iteration
#pragma unroll 1
      for (int q = 0; q < 6; ++q) {
        const int mu = q >> 1;
        const bool fw = (q & 1) == 0;
        int nbr;
        if (mu == 0) {
          const int xn = fw ? (x + 1 == g.Lx ? 0 : x + 1) : (x == 0 ? g.Lx - 1 : x - 1);
          nbr = h - xh + (xn >> 1);
        } else {
          const int L = mu == 1 ? g.Ly : g.Lz;
          const int sd = mu == 1 ? g.sy : g.sz;
          const int cm = mu == 1 ? y : z;
          nbr = fw ? h + (cm + 1 == L ? -(L - 1) * sd : sd) : h + (cm == 0 ? (L - 1) * sd : -sd);
        }
        const int ep = ((mu >= 1 ? x : 0) + (mu >= 2 ? y : 0)) & 1;
        R coef = ep ? R(-0.5) : R(0.5);
        if (!fw) coef = -coef;
        Su3<R> u;
        load_link_buf<R, NE>(make_res((fw ? Uout : Uin) + int64_t(mu) * NE * g.Vh, link_bytes),
                             uint32_t(fw ? h : nbr) * cbytes, csoff, !fw, u);
        cplx<R> v[BL][3];
        load_spinors<R, NE, BL>(rin, uint32_t(nbr) * cbytes, csoff, v);
        hop_acc<R, BL>(u, v, coef, acc);
      }
      // t: forward hop on the next slice, backward hop on the previous one
      const int ept = (x + y + z) & 1;
      {
        R coef = ept ? R(-0.5) : R(0.5);
        if (g.anti && t == g.Lt - 1) coef = -coef;
        Su3<R> u;
        load_link_buf<R, NE>(make_res(Uout + int64_t(3) * NE * g.Vh, link_bytes),
                             uint32_t(h) * cbytes, csoff, false, u);
        hop_acc<R, BL>(u, nxt, coef, acc);
      }
      {
        R coef = ept ? R(-0.5) : R(0.5);
        if (g.anti && t == 0) coef = -coef;
        coef = -coef;
        Su3<R> u;
        load_link_buf<R, NE>(make_res(Uin + int64_t(3) * NE * g.Vh, link_bytes),
                             uint32_t(col + tb * g.st) * cbytes, csoff, true, u);
        hop_acc<R, BL>(u, prv, coef, acc);
      }

      // own-site operands of the fused updates, all loaded before use
      cplx<R> dv[BL][3], rv[BL][3];
      if (MODE != DM_PLAIN) {
#pragma unroll
        for (int b = 0; b < BL; ++b) {
          const cplx<R>* d =
              static_cast<const cplx<R>*>(a.diag) + int64_t(jrow[b]) * a.diag_stride + h;
#pragma unroll
          for (int c = 0; c < 3; ++c) dv[b][c] = ld_once<R, true>(d + int64_t(c) * g.Vh);
          if (MODE == DM_CG) {
            const cplx<R>* r =
                static_cast<const cplx<R>*>(a.r) + int64_t(slot_in[b]) * a.r_stride + h;
#pragma unroll
            for (int c = 0; c < 3; ++c) rv[b][c] = ld_once<R, true>(r + int64_t(c) * g.Vh);
          }
        }
      }
#pragma unroll
      for (int b = 0; b < BL; ++b) {
        if (!lv[b]) continue;
        const int j = jrow[b];
        if (MODE == DM_PLAIN) {
          cplx<R>* out = static_cast<cplx<R>*>(a.out) + int64_t(j) * a.out_stride + h;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            st_once<R, true>(out + int64_t(c) * g.Vh, acc[b][c]);
            nrm[b] += cnorm2<R>(acc[b][c]);
          }
        } else if (MODE == DM_AXPY) {
          cplx<R>* out = static_cast<cplx<R>*>(a.out) + int64_t(j) * a.out_stride + h;
#pragma unroll
          for (int c = 0; c < 3; ++c)
            st_once<R, true>(out + int64_t(c) * g.Vh,
                             mk<R>(fma(m2s[b], dv[b][c].x, -acc[b][c].x),
                                   fma(m2s[b], dv[b][c].y, -acc[b][c].y)));
        } else {  // DM_CG
          cplx<R>* r = static_cast<cplx<R>*>(a.r) + int64_t(slot_out[b]) * a.r_stride + h;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const R wx = fma(m2s[b], dv[b][c].x, -acc[b][c].x);
            const R wy = fma(m2s[b], dv[b][c].y, -acc[b][c].y);
            cplx<R> rn = rv[b][c];
            rn.x = fma(-alpha[b], wx, rn.x);
            rn.y = fma(-alpha[b], wy, rn.y);
            st_once<R, true>(r + int64_t(c) * g.Vh, rn);
            nrm[b] += cnorm2<R>(rn);
          }
        }
      }
#pragma unroll
      for (int b = 0; b < BL; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          prv[b][c] = cur[b][c];
          cur[b][c] = nxt[b][c];
        }
    }
  }

  if (a.partials) {
    const int nblk = gridDim.x;
#pragma unroll
    for (int q = 0; q < B; ++q) {
      double v = 0.0;
#pragma unroll
      for (int b = 0; b < BL; ++b)
        if (q == part * BL + b) v = nrm[b];
      const double sum = block_sum(v, lds[q]);
      const int j = rhs0 + q;
      if (threadIdx.x == 0 && j < a.nrhs &&
          (a.live == nullptr || a.live[j * a.live_stride] != 0))
        a.partials[int64_t(j) * nblk + lb] = sum;
    }
  }
}

template <typename R, int NE, int P, int MODE>
int launch_tm(const DslashCall& c, const DslashCfg& cfg, hipStream_t st) {
  constexpr int BL = 8 / P;
  const int ngroups = (c.nrhs + 7) / 8;
  const int ncb = dslash_tm_column_blocks(c.g, cfg);
  const dim3 grid(unsigned(ncb * (c.g.Lt / cfg.tm)), unsigned(ngroups));
  const int lds = dslash_lds_bytes(cfg);
  if (lds < 0) {
    set_error("occupancy cap %d is below one workgroup of %d threads", cfg.occ, cfg.block);
    return LQCD_ERR_UNSUPPORTED;
  }
  hipLaunchKernelGGL((k_dslash_tm<R, NE, P, BL, MODE>), grid, dim3(cfg.block), lds, st, c,
                     cfg.xcd, cfg.tm, ncb);
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

template <typename R, int NE, int MODE>
int launch_tm_p(const DslashCall& c, const DslashCfg& cfg, hipStream_t st) {
  switch (cfg.tp) {
    case 2: return launch_tm<R, NE, 2, MODE>(c, cfg, st);
    case 4: return launch_tm<R, NE, 4, MODE>(c, cfg, st);
    default: break;
  }
  set_error("t-march lanes per column must be 2 or 4, got %d", cfg.tp);
  return LQCD_ERR_UNSUPPORTED;
}

}  // namespace

bool dslash_tm_supported(const DslashCall& c, const DslashCfg& cfg) {
  if (!(cfg.tm > 0 && !c.pairs && c.g.Lt % cfg.tm == 0 && cfg.rhs_block == 8 &&
        (cfg.tp == 2 || cfg.tp == 4) && c.fmt == LQCD_LINKS12 &&
        (c.mode == DM_PLAIN || c.mode == DM_AXPY || c.mode == DM_CG) && cfg.tz == 0 &&
        cfg.ty == 0 && cfg.ilv == 0 && cfg.lf == 0 && cfg.hh == 0 && cfg.nt == 1 &&
        cfg.ns == 1 && (cfg.block == 64 || cfg.block == 128 || cfg.block == 256)))
    return false;
  // the norm partials of one right-hand side must fit the solver's
  // ceil(Vh / 64) slots
  return int64_t(dslash_nblocks(c.g, cfg)) <= (int64_t(c.g.Vh) + 63) / 64;
}

int dslash_tm_launch(const DslashCall& c, const DslashCfg& cfg, hipStream_t st) {
  if (!dslash_tm_supported(c, cfg)) {
    set_error("t-march configuration (tm %d, lanes %d) not available for this call", cfg.tm,
              cfg.tp);
    return LQCD_ERR_UNSUPPORTED;
  }
  if (c.prec == LQCD_F64) {
    switch (c.mode) {
      case DM_PLAIN: return launch_tm_p<double, 6, DM_PLAIN>(c, cfg, st);
      case DM_AXPY: return launch_tm_p<double, 6, DM_AXPY>(c, cfg, st);
      default: return launch_tm_p<double, 6, DM_CG>(c, cfg, st);
    }
  }
  switch (c.mode) {
    case DM_PLAIN: return launch_tm_p<float, 6, DM_PLAIN>(c, cfg, st);
    case DM_AXPY: return launch_tm_p<float, 6, DM_AXPY>(c, cfg, st);
    default: return launch_tm_p<float, 6, DM_CG>(c, cfg, st);
  }
}

}  // namespace lqcd
