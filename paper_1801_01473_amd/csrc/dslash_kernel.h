// The k_dslash kernel family (templates), shared by the translation units
// that instantiate it: one per (precision, link format), compiled in parallel.
//
// One thread per output site; each thread
//   * decodes its coordinates and the half indices of its 8 neighbours with
//     periodic wrap, and the staggered phase / antiperiodic time sign from
//     the coordinates (Sec. 4.1 carries both in a U(1) factor; for +-1
//     factors nothing needs to be stored),
//   * loads each of its 8 links once (rebuilding row 2 for the 12-real
//     format) and applies it to up to B right-hand sides, so B spinor fields
//     share one link stream,
//   * writes the result, or folds it into the solver's vector update
//     (the paper's separate final sum kernel of Eq. (2), Sec. 5.2), and
//     accumulates FP64 block partials of the norms the solver needs.
// Links dominate the traffic (8 links per site vs 8+1 spinors): every link of
// the lattice is read exactly once per application, spinor neighbour reuse
// comes from L2 / MALL.
#pragma once

#include <hip/hip_runtime.h>

#include "dslash.h"
#include "su3.h"

namespace lqcd {

namespace {

// Half index of the i-th site visited.  tz = 0: lexicographic (i = h).
// tz > 0: the (y, z) cross-section is cut into tiles of ty rows (ty = 0: all
// Ly) and tz slices; inside a tile x and y run fastest, then z, then t, and
// the tiles come last -- consecutive workgroups sweep t through one small
// tile, so an input site is reused as a +-t neighbour (and as a y, z
// neighbour inside the tile) while still in L2.  A tile row of one (z, t) is
// a contiguous run of half indices, so loads stay coalesced.  A bijection on
// [0, Vh) when ty divides Ly and tz divides Lz.
__device__ __forceinline__ int site_of(const KGeom& g, int i, int tz, int ty) {
  if (tz == 0) return i;
  const int tyy = ty ? ty : g.Ly;
  const int row = g.Lxh * tyy;
  const int inrow = i % row;  // x and y inside the tile
  int r = i / row;
  const int zi = r % tz;
  r /= tz;
  const int t = r % g.Lt;
  const int tile = r / g.Lt;
  const int nty = g.Ly / tyy;
  const int y0 = (tile % nty) * tyy, z = (tile / nty) * tz + zi;
  return inrow + g.Lxh * y0 + g.sz * z + g.st * t;
}

// Slot index (in units of r_stride) of right-hand side j's residual of its
// current iteration + ahead (ahead = 1: the slot the update writes).
__device__ __forceinline__ int64_t r_slot(const DslashCall& a, int j, int ahead) {
  if (!a.r_iter) return j;
  const int it = a.r_iter[j * a.r_iter_stride];
  return int64_t(j) * a.r_slots + (it + ahead) % a.r_slots;
}

// V: bit 0 marks the link loads non-temporal (each link is read once; the
// hint keeps L2 for the spinors that neighbours read again), bit 1 schedules
// every load of a direction before its arithmetic (more loads in flight per
// wave, more registers held), bit 2 walks the eight hops one per iteration
// (half the loads held per iteration, so more waves fit; the backward link is
// conjugate-transposed in registers so that one product serves both), bit 4
// reads the input, the fused update's own-site direction (diag) and the plain
// mode's output as right-hand-side pairs (DslashCall::pairs; FP32, B even):
// one 16-byte access moves the same element of two right-hand sides, half the
// memory instructions of separate rows, with the same arithmetic and bits.
template <typename R, int NE, int B, int MODE, typename RO, int V>
__global__ void __launch_bounds__(256) k_dslash(const DslashCall a, const int xcd, const int tz,
                                                const int ty, const int ngroups,
                                                const int ilv) {
  constexpr int LAUX = (V & 1) ? 2 : 0;  // buffer cache policy of link loads: 2 = nt
  constexpr bool LF = (V & 2) != 0;
  constexpr bool HH = (V & 4) != 0;
  constexpr bool NS = (V & 8) != 0;  // own-site operands and outputs non-temporal
  constexpr bool PR = (V & 16) != 0;  // right-hand sides in interleaved pairs
  static_assert(!PR || (sizeof(R) == 4 && B % 2 == 0 && (MODE == DM_PLAIN || MODE == DM_CG)),
                "pairs: FP32, an even RHS block, plain or fused CG mode");
  constexpr int NRow = PR ? B / 2 : B;  // input rows loaded per element (pairs count once)
  __shared__ double lds[B][4];
  if (a.halt && *a.halt) return;
  const KGeom& g = a.g;
  // workgroup -> (site block, RHS group)
  const int nblk = ilv ? gridDim.x / ngroups : gridDim.x;
  const int lb0 = xcd_block(blockIdx.x, gridDim.x, xcd);
  const int lb = a.rev ? int(gridDim.x) - 1 - lb0 : lb0;  // reverse block order
  const int blk = ilv ? lb / ngroups : lb;
  const int rhs0 = (ilv ? lb % ngroups : blockIdx.y) * B;
  bool lv[B];
  bool any = false;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = rhs0 + b;
    lv[b] = j < a.nrhs && (a.live == nullptr || a.live[j * a.live_stride] != 0);
    any |= lv[b];
  }
  if (!any) return;  // uniform over the block

  const int idx = blk * blockDim.x + threadIdx.x;
  const int h = idx < a.g.Vh ? site_of(a.g, idx, tz, ty) : idx;
  double nrm[B];
#pragma unroll
  for (int b = 0; b < B; ++b) nrm[b] = 0.0;

  if (h < g.Vh) {
    const Site s = decode_site(g, h, a.out_par);
    int fwd[4], bwd[4];
    neighbours(g, s, h, fwd, bwd);
    double eta[4];
    staggered_eta(s, eta);

    cplx<R> acc[B][3];
#pragma unroll
    for (int b = 0; b < B; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[b][c] = mk<R>(0, 0);

    const int64_t par_stride = int64_t(4) * link_block<NE>(g.Vh);
    const cplx<R>* Uout = static_cast<const cplx<R>*>(a.U) + a.out_par * par_stride;
    const cplx<R>* Uin = static_cast<const cplx<R>*>(a.U) + (1 - a.out_par) * par_stride;
    constexpr uint32_t cb = sizeof(cplx<R>);
    const uint32_t link_bytes = uint32_t(link_block<NE>(g.Vh)) * cb;
    // Input rows of the block's right-hand sides; rows past nrhs alias the
    // last one (loaded and computed, never stored), so the loads of every
    // right-hand side issue together without a branch between them.
    // With pairs, rows 2q and 2q + 1 (nrhs even) fill the 2 in_stride values
    // from row 2q's start, element by element: the pair's resource covers
    // both, a site's element sits at 16 bytes per site, a colour 16 Vh bytes on.
    __amdgpu_buffer_rsrc_t rin[NRow];
#pragma unroll
    for (int b = 0; b < NRow; ++b) {
      const int jr = PR ? (rhs0 + 2 * b < a.nrhs ? rhs0 + 2 * b : a.nrhs - 2)
                        : (rhs0 + b < a.nrhs ? rhs0 + b : a.nrhs - 1);
      rin[b] = make_res(static_cast<const cplx<R>*>(a.in) + int64_t(jr) * a.in_stride,
                        (PR ? 6u : 3u) * uint32_t(g.Vh) * cb);
    }
    const uint32_t csoff = uint32_t(g.Vh) * cb;  // colour stride in bytes
    constexpr uint32_t pw = PR ? 2u : 1u;          // element width of the input rows

    if (HH) {
      // one hop per iteration: k = 2 mu + (0 forward, 1 backward)
#pragma unroll 1
      for (int k = 0; k < 8; ++k) {
        const int mu = k >> 1;
        const bool fw = (k & 1) == 0;
        // neighbour and phase from the coordinates (a per-k table would be
        // indexed dynamically and live in scratch)
        int nbr;
        if (mu == 0) {
          const int xn = fw ? (s.x + 1 == g.Lx ? 0 : s.x + 1) : (s.x == 0 ? g.Lx - 1 : s.x - 1);
          nbr = h - (s.x >> 1) + (xn >> 1);
        } else {
          const int L = mu == 1 ? g.Ly : (mu == 2 ? g.Lz : g.Lt);
          const int st = mu == 1 ? g.sy : (mu == 2 ? g.sz : g.st);
          const int cm = mu == 1 ? s.y : (mu == 2 ? s.z : s.t);
          nbr = fw ? h + (cm + 1 == L ? -(L - 1) * st : st) : h + (cm == 0 ? (L - 1) * st : -st);
        }
        const int ep = ((mu >= 1 ? s.x : 0) + (mu >= 2 ? s.y : 0) + (mu >= 3 ? s.z : 0)) & 1;
        R c = ep ? R(-0.5) : R(0.5);
        if (mu == 3 && g.anti && (fw ? s.t == g.Lt - 1 : s.t == 0)) c = -c;
        if (!fw) c = -c;
        Su3<R> u;
        cplx<R> v[B][3];
        const __amdgpu_buffer_rsrc_t rl =
            make_res((fw ? Uout : Uin) + int64_t(mu) * link_block<NE>(g.Vh), link_bytes);
        const uint32_t ol = uint32_t(fw ? h : nbr) * cb, on = uint32_t(nbr) * cb;
#pragma unroll
        for (int e = 0; e < stored_planes<NE>(); ++e)
          u.e[e] = ld_buf<R, LAUX>(rl, ol, uint32_t(e) * csoff);
        R th = R(0);
        if constexpr (NE == 8)
          th = ld_buf_real<R, LAUX>(rl, uint32_t(fw ? h : nbr) * uint32_t(sizeof(R)), 6u * csoff);
        if constexpr (PR) {
#pragma unroll
          for (int q = 0; q < NRow; ++q)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
              ld_buf_pair(rin[q], pw * on, uint32_t(cc) * pw * csoff, v[2 * q][cc],
                          v[2 * q + 1][cc]);
        } else {
#pragma unroll
          for (int b = 0; b < B; ++b)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) v[b][cc] = ld_buf<R>(rin[b], on, uint32_t(cc) * csoff);
        }
        complete_link<R, NE>(u);
        if constexpr (NE == 8) apply_u1<R>(u, th);
        if (!fw) {  // U^dag
          Su3<R> t = u;
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) u.e[3 * i + j] = conj_of<R>(t.e[3 * j + i]);
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
          cplx<R> y[3];
          mat_vec<R>(u, v[b], y);
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) {
            acc[b][cc].x = fma(c, y[cc].x, acc[b][cc].x);
            acc[b][cc].y = fma(c, y[cc].y, acc[b][cc].y);
          }
        }
        if (LF) {
          __builtin_amdgcn_sched_group_barrier(0x020, NE + 3 * NRow, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, 4096, 0);
        }
      }
    } else {
    // One direction per iteration (not unrolled: an unrolled body lets the
    // compiler hoist every direction's loads at once and run out of
    // registers).  Each iteration first issues all of its loads -- both links
    // and both neighbours of every right-hand side -- so one memory round
    // trip serves the whole iteration, then does the arithmetic.
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
      R cf = R(0.5 * eta[mu]), cb_ = cf;
      if (mu == 3 && g.anti) {
        if (s.t == g.Lt - 1) cf = -cf;  // link (x, t) crosses the time boundary
        if (s.t == 0) cb_ = -cb_;       // link (x - t, t) crosses it
      }
      const int nf = fwd[mu], nb = bwd[mu];
      Su3<R> uf, ub;
      cplx<R> vf[B][3], vb[B][3];
      R thf = R(0), thb = R(0);
      {
        const __amdgpu_buffer_rsrc_t rf =
            make_res(Uout + int64_t(mu) * link_block<NE>(g.Vh), link_bytes);
        const __amdgpu_buffer_rsrc_t rb =
            make_res(Uin + int64_t(mu) * link_block<NE>(g.Vh), link_bytes);
        const uint32_t of = uint32_t(h) * cb, ob = uint32_t(nb) * cb;
#pragma unroll
        for (int e = 0; e < stored_planes<NE>(); ++e) {
          uf.e[e] = ld_buf<R, LAUX>(rf, of, uint32_t(e) * csoff);
          ub.e[e] = ld_buf<R, LAUX>(rb, ob, uint32_t(e) * csoff);
        }
        if constexpr (NE == 8) {
          thf = ld_buf_real<R, LAUX>(rf, uint32_t(h) * uint32_t(sizeof(R)), 6u * csoff);
          thb = ld_buf_real<R, LAUX>(rb, uint32_t(nb) * uint32_t(sizeof(R)), 6u * csoff);
        }
      }
      {
        const uint32_t of = uint32_t(nf) * cb, ob = uint32_t(nb) * cb;
        if constexpr (PR) {
#pragma unroll
          for (int q = 0; q < NRow; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              ld_buf_pair(rin[q], pw * of, uint32_t(c) * pw * csoff, vf[2 * q][c],
                          vf[2 * q + 1][c]);
              ld_buf_pair(rin[q], pw * ob, uint32_t(c) * pw * csoff, vb[2 * q][c],
                          vb[2 * q + 1][c]);
            }
        } else {
#pragma unroll
          for (int b = 0; b < B; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              vf[b][c] = ld_buf<R>(rin[b], of, uint32_t(c) * csoff);
              vb[b][c] = ld_buf<R>(rin[b], ob, uint32_t(c) * csoff);
            }
        }
      }
      complete_link<R, NE>(uf);
      complete_link<R, NE>(ub);
      if constexpr (NE == 8) {
        apply_u1<R>(uf, thf);
        apply_u1<R>(ub, thb);
      }
#pragma unroll
      for (int b = 0; b < B; ++b) {
        cplx<R> y[3];
        mat_vec<R>(uf, vf[b], y);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          acc[b][c].x = fma(cf, y[c].x, acc[b][c].x);
          acc[b][c].y = fma(cf, y[c].y, acc[b][c].y);
        }
        adj_mat_vec<R>(ub, vb[b], y);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          acc[b][c].x = fma(-cb_, y[c].x, acc[b][c].x);
          acc[b][c].y = fma(-cb_, y[c].y, acc[b][c].y);
        }
      }
      // loads-first variant: every load of the iteration, then the arithmetic
      if (LF) {
        __builtin_amdgcn_sched_group_barrier(0x020, 2 * NE + 6 * NRow, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, 4096, 0);
      }
    }
    }

    // Own-site operands of the fused update for every right-hand side of the
    // block, loaded before any is used (rows past nrhs alias the last one),
    // so that their latencies overlap instead of adding up per RHS.
    cplx<R> dv[B][3], rv[B][3];
    double2 bv[B][3];
    if (MODE != DM_PLAIN) {
      if constexpr (PR) {  // the direction pair of rows 2q, 2q + 1 (as the input)
#pragma unroll
        for (int q = 0; q < NRow; ++q) {
          const int jp = rhs0 + 2 * q < a.nrhs ? rhs0 + 2 * q : a.nrhs - 2;
          const cplx<R>* d =
              static_cast<const cplx<R>*>(a.diag) + int64_t(jp) * a.diag_stride + 2 * h;
#pragma unroll
          for (int c = 0; c < 3; ++c)
            ld_once_pair<NS>(d + 2 * int64_t(c) * g.Vh, dv[2 * q][c], dv[2 * q + 1][c]);
        }
      }
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int jl = rhs0 + b < a.nrhs ? rhs0 + b : a.nrhs - 1;
        if constexpr (!PR) {
          const cplx<R>* d =
              static_cast<const cplx<R>*>(a.diag) + int64_t(jl) * a.diag_stride + h;
#pragma unroll
          for (int c = 0; c < 3; ++c) dv[b][c] = ld_once<R, NS>(d + int64_t(c) * g.Vh);
        }
        if (MODE == DM_CG) {
          const cplx<R>* r = static_cast<const cplx<R>*>(a.r) + r_slot(a, jl, 0) * a.r_stride + h;
#pragma unroll
          for (int c = 0; c < 3; ++c) rv[b][c] = ld_once<R, NS>(r + int64_t(c) * g.Vh);
        }
        if (MODE == DM_RES) {
          const cplx<double>* bp =
              static_cast<const cplx<double>*>(a.b) + int64_t(jl) * a.b_stride + h;
#pragma unroll
          for (int c = 0; c < 3; ++c) bv[b][c] = ld_once<double, NS>(bp + int64_t(c) * g.Vh);
        }
      }
    }

    if constexpr (PR && MODE == DM_PLAIN) {
      // a pair is written if either row is live (rows 2q, 2q + 1 < nrhs then);
      // the other row of such a pair belongs to a finished system, whose
      // output nothing reads
#pragma unroll
      for (int q = 0; q < NRow; ++q) {
        if (!lv[2 * q] && !lv[2 * q + 1]) continue;
        cplx<R>* out = static_cast<cplx<R>*>(a.out) + int64_t(rhs0 + 2 * q) * a.out_stride + 2 * h;
#pragma unroll
        for (int c = 0; c < 3; ++c)
          st_once_pair<NS>(out + 2 * int64_t(c) * g.Vh, acc[2 * q][c], acc[2 * q + 1][c]);
      }
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      if (!lv[b]) continue;
      const int j = rhs0 + b;
      if (MODE == DM_PLAIN && PR) {
#pragma unroll
        for (int c = 0; c < 3; ++c) nrm[b] += cnorm2<R>(acc[b][c]);
      } else if (MODE == DM_PLAIN) {
        cplx<R>* out = static_cast<cplx<R>*>(a.out) + int64_t(j) * a.out_stride + h;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          st_once<R, NS>(out + int64_t(c) * g.Vh, acc[b][c]);
          nrm[b] += cnorm2<R>(acc[b][c]);
        }
      } else {
        const double m2s = a.m2s ? a.m2s[j * a.m2s_stride] : a.m2s_c;
        if (MODE == DM_AXPY) {
          cplx<R>* out = static_cast<cplx<R>*>(a.out) + int64_t(j) * a.out_stride + h;
#pragma unroll
          for (int c = 0; c < 3; ++c)
            st_once<R, NS>(out + int64_t(c) * g.Vh,
                           mk<R>(fma(R(m2s), dv[b][c].x, -acc[b][c].x),
                                 fma(R(m2s), dv[b][c].y, -acc[b][c].y)));
        } else if (MODE == DM_CG) {
          const R al = R(a.alpha[j * a.alpha_stride]);
          cplx<R>* r = static_cast<cplx<R>*>(a.r) + r_slot(a, j, 1) * a.r_stride + h;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const R wx = fma(R(m2s), dv[b][c].x, -acc[b][c].x);
            const R wy = fma(R(m2s), dv[b][c].y, -acc[b][c].y);
            cplx<R> rn = rv[b][c];
            rn.x = fma(-al, wx, rn.x);
            rn.y = fma(-al, wy, rn.y);
            st_once<R, NS>(r + int64_t(c) * g.Vh, rn);
            nrm[b] += cnorm2<R>(rn);
          }
        } else {  // DM_RES, R = double
          cplx<RO>* r = a.r ? static_cast<cplx<RO>*>(a.r) + r_slot(a, j, 0) * a.r_stride + h
                            : nullptr;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double rx = bv[b][c].x - fma(m2s, (double)dv[b][c].x, -(double)acc[b][c].x);
            const double ry = bv[b][c].y - fma(m2s, (double)dv[b][c].y, -(double)acc[b][c].y);
            if (r) st_once<RO, NS>(r + int64_t(c) * g.Vh, mk<RO>(RO(rx), RO(ry)));
            nrm[b] += fma(rx, rx, ry * ry);
          }
        }
      }
    }
  }

  if (a.partials) {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const double sum = block_sum(nrm[b], lds[b]);
      if (threadIdx.x == 0 && lv[b]) a.partials[int64_t(rhs0 + b) * nblk + blk] = sum;
    }
  }
}

template <typename R, int NE, int B, int MODE, typename RO>
int launch_one(const DslashCall& c, const DslashCfg& cfg, hipStream_t st) {
  const int ngroups = (c.nrhs + B - 1) / B;
  const int nb = dslash_nblocks(c.g, cfg);
  const int ilv = (cfg.ilv && ngroups > 1) ? 1 : 0;
  const dim3 grid = ilv ? dim3(nb * ngroups, 1) : dim3(nb, ngroups);
  const int lds = dslash_lds_bytes(cfg);
  if (lds < 0) {
    set_error("occupancy cap %d is below one workgroup of %d threads", cfg.occ, cfg.block);
    return LQCD_ERR_UNSUPPORTED;
  }
#define LQCD_K(V)                                                                         \
  hipLaunchKernelGGL((k_dslash<R, NE, B, MODE, RO, V>), grid, dim3(cfg.block), lds, st, c, \
                     cfg.xcd, cfg.tz, cfg.ty, ngroups, ilv)
  if (cfg.ns && !cfg.nt) {
    set_error("non-temporal own-site streams (ns) need non-temporal link loads (nt)");
    return LQCD_ERR_UNSUPPORTED;
  }
  if (c.pairs) {  // interleaved right-hand-side pairs (FP32, 12/18-real, B even)
    if constexpr (sizeof(R) == 4 && (NE == 6 || NE == 9) && B % 2 == 0 &&
                  (MODE == DM_PLAIN || MODE == DM_CG)) {
      switch ((cfg.nt ? 1 : 0) | (cfg.lf ? 2 : 0) | (cfg.hh ? 4 : 0) | (cfg.ns ? 8 : 0)) {
        case 0: LQCD_K(16); break;
        case 1: LQCD_K(17); break;
        case 2: LQCD_K(18); break;
        case 3: LQCD_K(19); break;
        case 4: LQCD_K(20); break;
        case 5: LQCD_K(21); break;
        case 6: LQCD_K(22); break;
        case 7: LQCD_K(23); break;
        case 9: LQCD_K(25); break;
        case 11: LQCD_K(27); break;
        case 13: LQCD_K(29); break;
        default: LQCD_K(31); break;
      }
      LQCD_LAUNCH_CHECK();
      return LQCD_OK;
    } else {
      set_error("right-hand-side pairs need FP32 12- or 18-real links, an even RHS block "
                "and the plain or fused CG mode");
      return LQCD_ERR_UNSUPPORTED;
    }
  }
  if constexpr (NE == 7 || NE == 8) {
    // the phased-link formats instantiate the plain schedule only (loads
    // first is dropped): half the variants, the same results
    switch ((cfg.nt ? 1 : 0) | (cfg.hh ? 4 : 0) | (cfg.ns ? 8 : 0)) {
      case 0: LQCD_K(0); break;
      case 1: LQCD_K(1); break;
      case 4: LQCD_K(4); break;
      case 5: LQCD_K(5); break;
      case 9: LQCD_K(9); break;
      default: LQCD_K(13); break;
    }
    LQCD_LAUNCH_CHECK();
    return LQCD_OK;
  } else {
  switch ((cfg.nt ? 1 : 0) | (cfg.lf ? 2 : 0) | (cfg.hh ? 4 : 0) | (cfg.ns ? 8 : 0)) {
    case 0: LQCD_K(0); break;
    case 1: LQCD_K(1); break;
    case 2: LQCD_K(2); break;
    case 3: LQCD_K(3); break;
    case 4: LQCD_K(4); break;
    case 5: LQCD_K(5); break;
    case 6: LQCD_K(6); break;
    case 7: LQCD_K(7); break;
    case 9: LQCD_K(9); break;
    case 11: LQCD_K(11); break;
    case 13: LQCD_K(13); break;
    default: LQCD_K(15); break;
  }
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
  }
#undef LQCD_K
}

template <typename R, int NE, int MODE, typename RO>
int launch_b(const DslashCall& c, const DslashCfg& cfg, hipStream_t st) {
  switch (cfg.rhs_block) {
    case 1: return launch_one<R, NE, 1, MODE, RO>(c, cfg, st);
    case 2: return launch_one<R, NE, 2, MODE, RO>(c, cfg, st);
    case 4: return launch_one<R, NE, 4, MODE, RO>(c, cfg, st);
    case 8: return launch_one<R, NE, 8, MODE, RO>(c, cfg, st);
    default:
      set_error("unsupported right-hand-side block %d", cfg.rhs_block);
      return LQCD_ERR_UNSUPPORTED;
  }
}

template <typename R, int NE>
int launch_mode(const DslashCall& c, const DslashCfg& cfg, hipStream_t st) {
  switch (c.mode) {
    case DM_PLAIN: return launch_b<R, NE, DM_PLAIN, R>(c, cfg, st);
    case DM_AXPY: return launch_b<R, NE, DM_AXPY, R>(c, cfg, st);
    case DM_CG: return launch_b<R, NE, DM_CG, R>(c, cfg, st);
    default: break;
  }
  set_error("dslash mode %d not available for this precision/format", c.mode);
  return LQCD_ERR_UNSUPPORTED;
}

}  // namespace

// The launcher of one (precision, link format): the plain and fused modes,
// every right-hand-side block and schedule variant.
template <typename R, int NE>
int dslash_launch_fmt(const DslashCall& c, const DslashCfg& cfg, hipStream_t st) {
  return launch_mode<R, NE>(c, cfg, st);
}

}  // namespace lqcd
