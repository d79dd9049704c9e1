// CG and multi-shift CG for the shifted systems of Eq. (2),
//     ((m^2 + sigma_i) - D_eo D_oe) x_i = b,
// whose building blocks are scalar products, vector sums and D_oe / D_eo
// (Sec. 2).  Everything runs on the GPU; the host only launches and, every
// few iterations, reads one small flag word.
//
// One iteration per system of the base shift sigma_0 (smallest sigma):
//   K1  t = D_oe p                     + FP64 partials of |t|^2
//   K2  (one workgroup) a = rho / (m2s |p|^2 + |t|^2) -- equal to <p, A p>
//       because -D_eo = D_oe^dag -- and the shifted zeta_s, a_s
//   K3  r -= a (m2s p - D_eo t)        + FP64 partials of |r|^2   (fused)
//   K4  (one workgroup) beta, beta_s, zeta history, per-shift freezing,
//       convergence and iteration limits
//   K5  for every active shift: x_s += a_s p_s ; p_s = zeta_s r + beta_s p_s
//                                      + FP64 partials of |p_0|^2
// With deferred shift updates (multi-shift, window W > 1) K5 only forms the
// base direction p = r + beta p and files r in a ring of W residuals; K4 also
// advances, per shift, the coefficients that express x_s and p_s in terms of
// p_s at the window start and the ring, and every W iterations K6 applies
//       x_s += sum_q cx_sq v_q ,  p_s = sum_q cp_sq v_q   (v_0 = p_s, v_q = ring)
// reading each shifted vector once per window instead of every iteration.
// All reductions are two-stage and in fixed order, so results do not depend
// on scheduling.  Kernels skip systems (and whole launches) that are done,
// so a block of iterations can be replayed as one captured hipGraph.
//
// Mixed precision: the iteration above runs in FP32 (links FP32 18- or
// 12-real) and accumulates each shift's solution in an FP32 partial sum;
// every reliable_interval iterations (and at convergence) those sums are
// added into the FP64 solutions and the base residual is recomputed in FP64
// with FP64 links (Sec. 5.4: floating point for the molecular dynamics, double
// precision for the accept/reject step).  After the base system converges the
// FP64 true residual of every (right-hand side, shift) is computed, and the
// ones above tol are refined together as independent systems by CG started
// from their current solutions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dslash.h"
#include "solver.h"

namespace lqcd {

int convert_links_async(const KGeom& k, const void* src, int sp, int sf, void* dst, int dp,
                        int df, hipStream_t st);

namespace {

constexpr int kVecBlock = 256;

// --------------------------------------------------------------- kernels

// Deterministic sum of p[0..n) by the whole workgroup, broadcast to all threads.
__device__ double wg_sum(const double* __restrict__ p, int n, double* lds) {
  __shared__ double bc;
  double s = strided_sum(p, n);
  s = block_sum(s, lds);
  if (threadIdx.x == 0) bc = s;
  __syncthreads();
  s = bc;
  __syncthreads();
  return s;
}

// wg_sum of two arrays with their loads overlapped (strided_sum2): the same
// two results, bit for bit, in one chain of memory round trips.
__device__ void wg_sum2(const double* __restrict__ p, int n, const double* __restrict__ q, int m,
                        double* lds, double* sp, double* sq) {
  __shared__ double bc[2];
  double s, t;
  strided_sum2(p, n, q, m, &s, &t);
  s = block_sum(s, lds);
  if (threadIdx.x == 0) bc[0] = s;
  t = block_sum(t, lds);
  if (threadIdx.x == 0) bc[1] = t;
  __syncthreads();
  *sp = bc[0];
  *sq = bc[1];
  __syncthreads();
}

__device__ __forceinline__ bool finite_d(double v) { return v == v && fabs(v) <= 1.7e308; }

template <typename T>
__global__ void __launch_bounds__(kVecBlock) k_zero(T* __restrict__ p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = T{};
}

// partials[v][blk] = sum |v|^2 over the block's sites (FP64 vectors [nvec][3][Vh])
__global__ void __launch_bounds__(kVecBlock) k_norm2_f64(const double2* __restrict__ v,
                                                         int64_t stride, int Vh,
                                                         double* __restrict__ part) {
  __shared__ double lds[kVecBlock / 64];
  const int j = blockIdx.y;
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (h < Vh) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double2 z = v[int64_t(j) * stride + int64_t(c) * Vh + h];
      s += z.x * z.x + z.y * z.y;
    }
  }
  s = block_sum(s, lds);
  if (threadIdx.x == 0) part[int64_t(j) * gridDim.x + blockIdx.x] = s;
}

// r = (RI) b into slot 0 of each system's residual ring (R slots), partials of |r|^2
template <typename RI>
__global__ void __launch_bounds__(kVecBlock) k_copy_to_inner(const double2* __restrict__ b,
                                                             cplx<RI>* __restrict__ r, int R,
                                                             int Vh,
                                                             double* __restrict__ part) {
  __shared__ double lds[kVecBlock / 64];
  const int j = blockIdx.y;
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (h < Vh) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t i = (int64_t(j) * 3 + c) * Vh + h;
      const cplx<RI> z = mk<RI>(RI(b[i].x), RI(b[i].y));
      r[(int64_t(j) * R * 3 + c) * Vh + h] = z;
      s += cnorm2<RI>(z);
    }
  }
  s = block_sum(s, lds);
  if (threadIdx.x == 0) part[int64_t(j) * gridDim.x + blockIdx.x] = s;
}

// Index of complex element (system j, colour c, half site h) of a field of
// [nsys][3][Vh] values, or, with pairs, of the same field with systems 2q and
// 2q + 1 interleaved element by element in their 6 Vh values (the layout the
// FP32 stencils read and write with 16-byte accesses).
__device__ __forceinline__ int64_t sys_index(int pairs, int j, int c, int h, int Vh) {
  return pairs ? (int64_t(j & ~1) * 3 + 2 * c) * Vh + 2 * int64_t(h) + (j & 1)
               : (int64_t(j) * 3 + c) * Vh + h;
}

// p_s = r for every shift, optionally x_s = 0; partials of |r|^2 (= |p|^2)
// (pc, when given: the base direction of deferred shift updates, also = r,
// in pairs when pc_pairs)
template <typename RI, typename RX>
__global__ void __launch_bounds__(kVecBlock) k_init_dirs(const cplx<RI>* __restrict__ r, int R,
                                                         cplx<RI>* __restrict__ p,
                                                         cplx<RX>* __restrict__ x,
                                                         cplx<RI>* __restrict__ pc,
                                                         int pc_pairs, int nshift, int zero_x,
                                                         int Vh, double* __restrict__ part) {
  __shared__ double lds[kVecBlock / 64];
  const int j = blockIdx.y;
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (h < Vh) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cplx<RI> z = r[(int64_t(j) * R * 3 + c) * Vh + h];  // slot 0
      s += cnorm2<RI>(z);
      if (pc) pc[sys_index(pc_pairs, j, c, h, Vh)] = z;
      for (int k = 0; k < nshift; ++k) {
        const int64_t i = ((int64_t(j) * nshift + k) * 3 + c) * Vh + h;
        p[i] = z;
        if (zero_x) x[i] = mk<RX>(0, 0);
      }
    }
  }
  s = block_sum(s, lds);
  if (threadIdx.x == 0) part[int64_t(j) * gridDim.x + blockIdx.x] = s;
}

// params = [m2s per system][delta per (system, shift)]
__global__ void __launch_bounds__(kScalarThreads) k_sc_init(
    SysState* __restrict__ st, GlobalFlags* __restrict__ gf, int nsys, int nshift,
    const double* __restrict__ params, double tol2, double sw2, const double* part_b, int nb_b,
    const double* part_r, int nb_r, const double* part_p, int nb_p) {
  __shared__ double lds[kScalarThreads / 64];
  int all_done = 1, err = 0, phase_done = 1;
  for (int j = 0; j < nsys; ++j) {
    const double bn = wg_sum(part_b + int64_t(j) * nb_b, nb_b, lds);
    const double rr = wg_sum(part_r + int64_t(j) * nb_r, nb_r, lds);
    const double pp = wg_sum(part_p + int64_t(j) * nb_p, nb_p, lds);
    if (threadIdx.x == 0) {
      SysState& S = st[j];
      S.bnorm2 = bn;
      S.target2 = tol2 * bn;
      S.rho = rr;
      S.pp = pp;
      S.m2s = params[j];
      S.a = 0.0;
      S.a_old = 1.0;
      S.b_old = 0.0;
      S.iters = 0;
      S.nrel = 0;
      S.rel = 0;
      S.upd_any = 0;
      S.r2ref = rr;
      S.rho_iter = rr;
      S.restart = 0;
      S.iters64 = 0;
      S.wpos = 0;
      S.upd64 = 0;
      S.upd32 = 0;
      S.fsh64 = S.fsh32 = 0;
      S.fsl64 = S.fsl32 = 0;
      S.err = finite_d(rr) && finite_d(bn) ? 0 : 1;
      for (int s = 0; s < kMaxShift; ++s) {
        S.zeta[s] = S.zeta_old[s] = S.zeta_new[s] = 1.0;
        S.a_s[s] = S.b_s[s] = 0.0;
        S.delta[s] = s < nshift ? params[nsys + j * nshift + s] : 0.0;
        S.active[s] = s < nshift ? 1 : 0;
        S.upd[s] = 0;
        S.dirty[s] = 0;
        S.wdirty[s] = 0;
      }
      S.conv = rr <= S.target2 ? 1 : 0;
      S.done = (S.conv || S.err) ? 1 : 0;
      S.live = !S.done;
      S.lowres = rr <= sw2 * bn ? 1 : 0;
      all_done &= S.done;
      phase_done &= (S.done | S.lowres);
      err |= S.err;
    }
  }
  if (threadIdx.x == 0) {
    gf->all_done = all_done;
    gf->error = err;
    gf->rel_req = 0;
    gf->phase_done = phase_done;
  }
}

// K2: step length of the base system and the shifted zetas; one workgroup
// per system (blockIdx.x), each reducing its own partials in fixed order.
__global__ void __launch_bounds__(kScalarThreads) k_sc_alpha(SysState* __restrict__ st,
                                                              GlobalFlags* __restrict__ gf,
                                                              int nshift, const double* part_t,
                                                              int nb_t, const double* part_p,
                                                              int nb_p) {
  __shared__ double lds[kScalarThreads / 64];
  const int j = blockIdx.x;
  double tt, pp;
  wg_sum2(part_t + int64_t(j) * nb_t, nb_t, part_p + int64_t(j) * nb_p, nb_p, lds, &tt, &pp);
  if (threadIdx.x != 0) return;
  SysState& S = st[j];
  S.upd_any = 0;
  S.restart = 0;
  for (int s = 0; s < nshift; ++s) S.upd[s] = 0;
  if (S.done) return;
  const double pAp = S.m2s * pp + tt;  // <p, (m2s - D_eo D_oe) p>
  S.pp = pp;
  if (!(pAp > 0.0) || !finite_d(pAp)) {
    S.err = 1;
    S.done = 1;
    S.live = 0;
    gf->error = 1;
    return;
  }
  const double a = S.rho / pAp;
  S.a = a;
  for (int s = 0; s < nshift; ++s) {
    if (!S.active[s]) continue;
    const double z = S.zeta[s], zo = S.zeta_old[s];
    const double zn =
        z * zo * S.a_old / (a * S.b_old * (zo - z) + zo * S.a_old * (1.0 + S.delta[s] * a));
    S.zeta_new[s] = zn;
    S.a_s[s] = a * zn / z;
    S.upd[s] = 1;
  }
  S.upd_any = 1;
}

// K4: beta, shifted betas, freezing, convergence; one workgroup per system.
// The global flags are derived afterwards by k_sc_flags.  With deferred
// shift updates (wc != nullptr) the whole workgroup then advances the window
// coefficients of the updated shifts, one thread per coefficient:
//   x_s += a_s p_s   ->  cx_s += a_s cp_s
//   p_s  = zeta_s r + b_s p_s  ->  cp_s = b_s cp_s, cp_s[n+1] = zeta_s
// where index n+1 is the residual after this iteration (ring slot n).
__global__ void __launch_bounds__(kScalarThreads) k_sc_beta(SysState* __restrict__ st,
                                                             GlobalFlags* __restrict__ gf,
                                                             int nshift, const double* part_r,
                                                             int nb_r, int max_iter,
                                                             double rel_delta2, double sw2,
                                                             int fp64, WinCoef* __restrict__ wc,
                                                             int win) {
  __shared__ double lds[kScalarThreads / 64];
  __shared__ double sh_a[kMaxShift], sh_b[kMaxShift], sh_z[kMaxShift];
  __shared__ int sh_u[kMaxShift];
  __shared__ int sh_n;
  const int j = blockIdx.x;
  const double rr = wg_sum(part_r + int64_t(j) * nb_r, nb_r, lds);
  if (threadIdx.x == 0) {
    sh_n = -1;
    SysState& S = st[j];
    bool go = S.upd_any != 0;
    if (go && !finite_d(rr)) {
      S.err = 1;
      S.done = 1;
      S.live = 0;
      S.upd_any = 0;
      gf->error = 1;
      go = false;
    }
    if (go && wc && S.wpos >= win) {  // the window was not flushed in time
      S.err = 1;
      S.done = 1;
      S.live = 0;
      S.upd_any = 0;
      gf->error = 1;
      go = false;
    }
    if (go) {
      const double beta = rr / S.rho;
      int nupd = 0;
      for (int s = 0; s < nshift; ++s) {
        sh_u[s] = S.upd[s];
        if (!S.upd[s]) continue;
        ++nupd;
        const double ratio = S.zeta_new[s] / S.zeta[s];
        S.b_s[s] = beta * ratio * ratio;
        S.zeta_old[s] = S.zeta[s];
        S.zeta[s] = S.zeta_new[s];
        S.dirty[s] = 1;
        S.wdirty[s] |= wc ? 1 : 0;
        sh_a[s] = S.a_s[s];
        sh_b[s] = S.b_s[s];
        sh_z[s] = S.zeta[s];
        if (S.zeta_new[s] * S.zeta_new[s] * rr <= S.target2) S.active[s] = 0;
      }
      S.a_old = S.a;
      S.b_old = beta;
      S.rho = rr;
      S.iters += 1;
      if (fp64) {
        S.iters64 += 1;
        S.upd64 += nupd;
      } else {
        S.upd32 += nupd;
      }
      if (rr < rel_delta2 * S.r2ref) gf->rel_req = 1;
      if (rr <= sw2 * S.bnorm2) S.lowres = 1;
      if (rr <= S.target2 || S.iters >= max_iter) {
        S.done = 1;
        S.live = 0;
        S.conv = rr <= S.target2 ? 1 : 0;
      }
      if (wc) {
        sh_n = S.wpos;
        S.wpos += 1;
      }
    }
  }
  __syncthreads();
  const int n = sh_n;
  if (n < 0) return;
  const int s = threadIdx.x / kWinRow, q = threadIdx.x % kWinRow;
  if (s >= nshift || !sh_u[s]) return;
  WinCoef& C = wc[j];
  if (q <= n) {
    const double cp = C.cp[s][q];
    C.cx[s][q] = fma(sh_a[s], cp, C.cx[s][q]);
    C.cp[s][q] = sh_b[s] * cp;
  } else if (q == n + 1) {
    C.cp[s][q] = sh_z[s];
  }
}

// all_done / phase_done over every system
__global__ void k_sc_flags(const SysState* __restrict__ st, GlobalFlags* __restrict__ gf,
                           int nsys) {
  if (threadIdx.x != 0) return;
  int all_done = 1, phase_done = 1;
  for (int j = 0; j < nsys; ++j) {
    all_done &= st[j].done;
    phase_done &= (st[j].done | st[j].lowres);
  }
  gf->all_done = all_done;
  gf->phase_done = phase_done;
}

// K5: x_s += a_s p_s ; p_s = zeta_s r + beta_s p_s for the shifts updated this iteration
template <typename RI, typename RX>
__global__ void __launch_bounds__(kVecBlock) k_ms_update(const SysState* __restrict__ st,
                                                         const cplx<RI>* __restrict__ r,
                                                         cplx<RI>* __restrict__ p,
                                                         cplx<RX>* __restrict__ x, int nshift,
                                                         int base, int Vh,
                                                         double* __restrict__ part) {
  __shared__ double lds[kVecBlock / 64];
  const int j = blockIdx.y;
  const SysState& S = st[j];
  if (!S.upd_any) return;
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  double pn = 0.0;
  if (h < Vh) {
    cplx<RI> rv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) rv[c] = r[(int64_t(j) * 3 + c) * Vh + h];
    for (int s = 0; s < nshift; ++s) {
      if (!S.upd[s]) continue;
      const RI as = RI(S.a_s[s]), zs = RI(S.zeta[s]), bs = RI(S.b_s[s]);
      const int64_t o = (int64_t(j) * nshift + s) * 3 * Vh + h;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cplx<RI> pv = p[o + int64_t(c) * Vh];
        cplx<RX> xv = x[o + int64_t(c) * Vh];
        xv.x = fma(RX(as), RX(pv.x), xv.x);
        xv.y = fma(RX(as), RX(pv.y), xv.y);
        pv.x = fma(zs, rv[c].x, bs * pv.x);
        pv.y = fma(zs, rv[c].y, bs * pv.y);
        x[o + int64_t(c) * Vh] = xv;
        p[o + int64_t(c) * Vh] = pv;
        if (s == base) pn += cnorm2<RI>(pv);
      }
    }
  }
  pn = block_sum(pn, lds);
  if (threadIdx.x == 0) part[int64_t(j) * gridDim.x + blockIdx.x] = pn;
}

// K5 with deferred shift updates: p = zeta_0 r + beta_0 p for the base
// direction only (zeta_0 = 1); r is the new residual, which the fused D_eo
// update wrote into ring slot iters % R (R = window + 1 slots, so a window's
// residuals stay in place until it is flushed); partials of |p|^2.
template <typename RI>
__global__ void __launch_bounds__(kVecBlock) k_base_update(const SysState* __restrict__ st,
                                                           const cplx<RI>* __restrict__ r,
                                                           int R, cplx<RI>* __restrict__ pc,
                                                           int base, int Vh,
                                                           double* __restrict__ part) {
  __shared__ double lds[kVecBlock / 64];
  const int j = blockIdx.y;
  const SysState& S = st[j];
  if (!S.upd_any) return;
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rs = int64_t(j) * R + S.iters % R;
  double pn = 0.0;
  if (h < Vh) {
    const RI zs = RI(S.zeta[base]), bs = RI(S.b_s[base]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t i = (int64_t(j) * 3 + c) * Vh + h;
      const cplx<RI> rv = r[(rs * 3 + c) * Vh + h];
      cplx<RI> pv = pc[i];
      pv.x = fma(zs, rv.x, bs * pv.x);
      pv.y = fma(zs, rv.y, bs * pv.y);
      pc[i] = pv;
      pn += cnorm2<RI>(pv);
    }
  }
  pn = block_sum(pn, lds);
  if (threadIdx.x == 0) part[int64_t(j) * gridDim.x + blockIdx.x] = pn;
}

// k_base_update<float> for base directions stored in pairs (systems 2q and
// 2q + 1 interleaved, blockIdx.y = q): one thread updates a site of both with
// 16-byte accesses, the same arithmetic per system and the same partials; a
// system that does not update keeps its values bit for bit.
__global__ void __launch_bounds__(kVecBlock) k_base_update_pairs(
    const SysState* __restrict__ st, const float2* __restrict__ r, int R,
    float4* __restrict__ pc, int base, int Vh, double* __restrict__ part) {
  __shared__ double lds0[kVecBlock / 64], lds1[kVecBlock / 64];
  const int j0 = 2 * blockIdx.y, j1 = j0 + 1;
  const SysState& S0 = st[j0];
  const SysState& S1 = st[j1];
  const bool u0 = S0.upd_any != 0, u1 = S1.upd_any != 0;
  if (!u0 && !u1) return;
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rs0 = int64_t(j0) * R + S0.iters % R, rs1 = int64_t(j1) * R + S1.iters % R;
  double pn0 = 0.0, pn1 = 0.0;
  if (h < Vh) {
    const float zs0 = float(S0.zeta[base]), bs0 = float(S0.b_s[base]);
    const float zs1 = float(S1.zeta[base]), bs1 = float(S1.b_s[base]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t i = (int64_t(blockIdx.y) * 3 + c) * Vh + h;  // float4 units
      const float2 rv0 = r[(rs0 * 3 + c) * Vh + h];
      const float2 rv1 = r[(rs1 * 3 + c) * Vh + h];
      float4 pv = pc[i];
      if (u0) {
        pv.x = fma(zs0, rv0.x, bs0 * pv.x);
        pv.y = fma(zs0, rv0.y, bs0 * pv.y);
        pn0 += cnorm2<float>(make_float2(pv.x, pv.y));
      }
      if (u1) {
        pv.z = fma(zs1, rv1.x, bs1 * pv.z);
        pv.w = fma(zs1, rv1.y, bs1 * pv.w);
        pn1 += cnorm2<float>(make_float2(pv.z, pv.w));
      }
      pc[i] = pv;
    }
  }
  pn0 = block_sum(pn0, lds0);
  pn1 = block_sum(pn1, lds1);
  if (threadIdx.x == 0) {
    if (u0) part[int64_t(j0) * gridDim.x + blockIdx.x] = pn0;
    if (u1) part[int64_t(j1) * gridDim.x + blockIdx.x] = pn1;
  }
}

// K6: applies the window of every system that has one open (wpos > 0) to the
// shifts updated in it; WM >= window length bounds the unrolled ring.
// The window's residuals r(k0 + 1 .. k0 + n) are ring slots (k0 + q) % R,
// k0 = iters - wpos.
template <typename RI, typename RX, int WM>
__global__ void __launch_bounds__(kVecBlock) k_ms_flush(const SysState* __restrict__ st,
                                                        const WinCoef* __restrict__ wc,
                                                        const cplx<RI>* __restrict__ ring, int R,
                                                        cplx<RI>* __restrict__ p,
                                                        cplx<RX>* __restrict__ x, int nshift,
                                                        int win, int Vh) {
  const int j = blockIdx.y;
  const SysState& S = st[j];
  const int n = S.wpos < win ? S.wpos : win;
  if (n <= 0) return;
  const int k0 = S.iters - S.wpos;
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= Vh) return;
  const WinCoef& C = wc[j];
#pragma unroll 1
  for (int c = 0; c < 3; ++c) {
    cplx<RI> v[WM];
#pragma unroll
    for (int q = 0; q < WM; ++q)
      if (q < n) v[q] = ring[((int64_t(j) * R + (k0 + 1 + q) % R) * 3 + c) * Vh + h];
    for (int s = 0; s < nshift; ++s) {
      if (!S.wdirty[s]) continue;
      const int64_t o = ((int64_t(j) * nshift + s) * 3 + c) * Vh + h;
      const cplx<RI> p0 = p[o];
      const RX cx0 = RX(C.cx[s][0]);
      const RI cp0 = RI(C.cp[s][0]);
      RX dx = cx0 * RX(p0.x), dy = cx0 * RX(p0.y);
      RI px = cp0 * p0.x, py = cp0 * p0.y;
#pragma unroll
      for (int q = 0; q < WM; ++q) {
        if (q < n) {
          const RX a = RX(C.cx[s][q + 1]);
          const RI b = RI(C.cp[s][q + 1]);
          dx = fma(a, RX(v[q].x), dx);
          dy = fma(a, RX(v[q].y), dy);
          px = fma(b, v[q].x, px);
          py = fma(b, v[q].y, py);
        }
      }
      cplx<RX> xv = x[o];
      xv.x += dx;
      xv.y += dy;
      x[o] = xv;
      p[o] = mk<RI>(px, py);
    }
  }
}

// Closes the window of every system that has one open (init: of every
// system): coefficients back to x_s += 0, p_s = p_s; counts the flush.
__global__ void __launch_bounds__(kScalarThreads) k_sc_win_reset(SysState* __restrict__ st,
                                                                  WinCoef* __restrict__ wc,
                                                                  int nshift, int fp64,
                                                                  int init) {
  __shared__ int sh_go;
  const int j = blockIdx.x;
  SysState& S = st[j];
  if (threadIdx.x == 0) sh_go = init || S.wpos > 0;
  __syncthreads();
  if (!sh_go) return;
  const int s = threadIdx.x / kWinRow, q = threadIdx.x % kWinRow;
  wc[j].cx[s][q] = 0.0;
  wc[j].cp[s][q] = q == 0 ? 1.0 : 0.0;
  if (threadIdx.x == 0) {
    if (!init) {
      long long ns = 0;
      for (int k = 0; k < nshift; ++k) ns += S.wdirty[k];
      if (fp64) {
        S.fsh64 += ns;
        S.fsl64 += S.wpos;
      } else {
        S.fsh32 += ns;
        S.fsl32 += S.wpos;
      }
    }
    S.wpos = 0;
    for (int k = 0; k < kMaxShift; ++k) S.wdirty[k] = 0;
  }
}

__global__ void k_sc_rel_begin(SysState* __restrict__ st, GlobalFlags* __restrict__ gf, int nsys,
                               int nshift) {
  if (threadIdx.x != 0) return;
  gf->rel_req = 0;
  for (int j = 0; j < nsys; ++j) {
    int any = 0;
    for (int s = 0; s < nshift; ++s) any |= st[j].dirty[s];
    st[j].rel = any;
  }
}

// x_hi += x_lo ; x_lo = 0 for every shift changed since the last reliable update
__global__ void __launch_bounds__(kVecBlock) k_accum(const SysState* __restrict__ st,
                                                     float2* __restrict__ xlo,
                                                     double2* __restrict__ xhi, int nshift,
                                                     int Vh) {
  const int k = blockIdx.y;
  const int j = k / nshift, s = k % nshift;
  if (!st[j].rel || !st[j].dirty[s]) return;
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= Vh) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t i = (int64_t(k) * 3 + c) * Vh + h;
    const float2 lo = xlo[i];
    double2 hi = xhi[i];
    hi.x += double(lo.x);
    hi.y += double(lo.y);
    xhi[i] = hi;
    xlo[i] = make_float2(0.f, 0.f);
  }
}

__global__ void __launch_bounds__(kScalarThreads) k_sc_reliable(SysState* __restrict__ st,
                                                                 GlobalFlags* __restrict__ gf,
                                                                 int nsys, int nshift, int base,
                                                                 const double* part, int nb,
                                                                 int max_iter) {
  __shared__ double lds[kScalarThreads / 64];
  int all_done = 1;
  for (int j = 0; j < nsys; ++j) {
    const double rr = wg_sum(part + int64_t(j) * nb, nb, lds);
    if (threadIdx.x != 0) continue;
    SysState& S = st[j];
    if (S.rel) {
      S.rel = 0;
      S.nrel += 1;
      for (int s = 0; s < nshift; ++s) S.dirty[s] = 0;
      if (!finite_d(rr)) {
        S.err = 1;
        S.done = 1;
        S.live = 0;
        gf->error = 1;
      } else {
        S.rho_iter = S.rho;
        S.rho = rr;
        S.r2ref = rr;
        // The FP32 recurrence drifted far from the FP64 residual: the old
        // directions no longer fit it, so restart the (shifted) directions
        // from the recomputed residual, r_s = zeta_s r.
        if (rr > 4.0 * S.rho_iter && rr > S.target2) {
          S.restart = 1;
          S.a_old = 1.0;
          S.b_old = 0.0;
          for (int s = 0; s < nshift; ++s) S.zeta_old[s] = S.zeta[s];
        }
        if (rr <= S.target2) {
          S.conv = 1;
          S.done = 1;
          S.live = 0;
        } else {
          S.conv = 0;
          if (S.iters < max_iter) {
            S.done = 0;
            S.live = 1;
            S.active[base] = 1;
          }
        }
      }
    }
    all_done &= S.done;
  }
  if (threadIdx.x == 0) gf->all_done = all_done;
}

// p_s = zeta_s r for the shifts of restarted systems, partials of |p_base|^2
// (and the base direction pc of deferred shift updates, when given)
template <typename RI>
__global__ void __launch_bounds__(kVecBlock) k_restart_dirs(const SysState* __restrict__ st,
                                                            const cplx<RI>* __restrict__ r, int R,
                                                            cplx<RI>* __restrict__ p,
                                                            cplx<RI>* __restrict__ pc,
                                                            int pc_pairs, int nshift, int base,
                                                            int Vh, double* __restrict__ part) {
  __shared__ double lds[kVecBlock / 64];
  const int j = blockIdx.y;
  const SysState& S = st[j];
  if (!S.restart) return;
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  double pn = 0.0;
  if (h < Vh) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cplx<RI> rv = r[((int64_t(j) * R + S.iters % R) * 3 + c) * Vh + h];
      for (int s = 0; s < nshift; ++s) {
        if (!S.active[s] && s != base) continue;
        const RI z = RI(S.zeta[s]);
        const cplx<RI> pv = mk<RI>(z * rv.x, z * rv.y);
        p[((int64_t(j) * nshift + s) * 3 + c) * Vh + h] = pv;
        if (s == base) {
          pn += cnorm2<RI>(pv);
          if (pc) pc[sys_index(pc_pairs, j, c, h, Vh)] = pv;
        }
      }
    }
  }
  pn = block_sum(pn, lds);
  if (threadIdx.x == 0) part[int64_t(j) * gridDim.x + blockIdx.x] = pn;
}

// FP64 Krylov state -> FP32: r, every shift's p; x_lo = 0; partials of |p_base|^2
// (with deferred shift updates the base direction is pc64 -> pc32)
// (r: the current slot, iters % R, of each system's residual ring in both)
__global__ void __launch_bounds__(kVecBlock) k_to_fp32(const SysState* __restrict__ st, int R,
                                                       const double2* __restrict__ r64,
                                                       const double2* __restrict__ p64,
                                                       const double2* __restrict__ pc64,
                                                       float2* __restrict__ r32,
                                                       float2* __restrict__ p32,
                                                       float2* __restrict__ pc32, int pc_pairs,
                                                       float2* __restrict__ xlo, int nshift,
                                                       int base, int Vh,
                                                       double* __restrict__ part) {
  __shared__ double lds[kVecBlock / 64];
  const int j = blockIdx.y;
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  double pn = 0.0;
  if (h < Vh) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t ir = (int64_t(j) * 3 + c) * Vh + h;
      const int64_t irr = ((int64_t(j) * R + st[j].iters % R) * 3 + c) * Vh + h;
      r32[irr] = make_float2(float(r64[irr].x), float(r64[irr].y));
      if (pc64) {
        const float2 pv = make_float2(float(pc64[ir].x), float(pc64[ir].y));
        pc32[sys_index(pc_pairs, j, c, h, Vh)] = pv;
        pn += cnorm2<float>(pv);
      }
      for (int s = 0; s < nshift; ++s) {
        const int64_t i = ((int64_t(j) * nshift + s) * 3 + c) * Vh + h;
        const float2 pv = make_float2(float(p64[i].x), float(p64[i].y));
        p32[i] = pv;
        xlo[i] = make_float2(0.f, 0.f);
        if (s == base && !pc64) pn += cnorm2<float>(pv);
      }
    }
  }
  pn = block_sum(pn, lds);
  if (threadIdx.x == 0) part[int64_t(j) * gridDim.x + blockIdx.x] = pn;
}

// After the FP64 phase: the FP64 solutions are current, the next reliable
// update is measured from here.
__global__ void k_sc_phase2(SysState* __restrict__ st, int nsys, int nshift) {
  if (threadIdx.x != 0) return;
  for (int j = 0; j < nsys; ++j) {
    st[j].r2ref = st[j].rho;
    for (int s = 0; s < nshift; ++s) st[j].dirty[s] = 0;
  }
}

// out[v] = sum_b part[v][b], fixed order, one workgroup per vector
__global__ void __launch_bounds__(kVecBlock) k_reduce_vec(const double* __restrict__ part, int nb,
                                                          double* __restrict__ out) {
  __shared__ double lds[kVecBlock / 64];
  const int v = blockIdx.x;
  double s = strided_sum(part + int64_t(v) * nb, nb);
  s = block_sum(s, lds);
  if (threadIdx.x == 0) out[v] = s;
}

// --------------------------------------------------------------- host side

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t r, t, p, xlo, r64, t64, p64, thi, bb, xb, st, gf, params, pt, pr, pp, pb, pres, resn,
      links, links_pre, pc, pc64, wc, total;
  bool has_xlo, has_pre, has_links;
  int win;  // window of deferred shift updates of the main solve (1: none)
};

int poll_for(const lqcd_solver_params& p) {
  return p.poll_interval > 0 ? p.poll_interval : (p.inner_prec == LQCD_F32 ? 31 : 62);
}

// Window length of deferred shift updates: shift_window reduced to a divisor
// of the poll interval, so that every replayed block of iterations ends with
// all windows closed; 1 (no deferral) for a single shift.
int window_for(const lqcd_solver_params& p, int nshift) {
  if (nshift < 2) return 1;
  const int poll = poll_for(p);
  int w = std::max(1, std::min(p.shift_window, kMaxWin));
  while (w > 1 && poll % w != 0) --w;
  return w;
}

// Workspace layout.  Mixed precision keeps FP32 iteration vectors and FP32
// partial solutions, plus FP64 iteration vectors for the FP64 opening phase
// when mixed_switch > 0.
Layout make_layout(const KGeom& g, const lqcd_solver_params& p, int nshift, int nrhs) {
  Layout L{};
  const int iprec = p.inner_prec, ifmt = p.inner_fmt;
  const size_t ri = iprec == LQCD_F32 ? 4 : 8;
  const size_t vin = size_t(3) * g.Vh * 2 * ri;
  const size_t v64 = size_t(3) * g.Vh * 16;
  const size_t nparts = size_t(nrhs) * ((g.Vh + 63) / 64);
  size_t off = 0;
  auto take = [&](size_t n) {
    const size_t o = off;
    off = align_up(off + n);
    return o;
  };
  // residuals: a ring of W + 1 slots per system with deferred shift updates
  // (the window's residuals stay in place until the window is flushed), else
  // one slot updated in place
  L.win = window_for(p, nshift);
  const size_t R = L.win > 1 ? size_t(L.win) + 1 : 1;
  L.r = take(nrhs * R * vin);
  L.t = take(nrhs * vin);
  L.p = take(size_t(nrhs) * nshift * vin);
  L.has_xlo = iprec == LQCD_F32;
  L.xlo = L.has_xlo ? take(size_t(nrhs) * nshift * vin) : 0;
  L.has_pre = iprec == LQCD_F32 && p.mixed_switch > 0.0 && nshift > 1;
  L.r64 = L.has_pre ? take(nrhs * R * v64) : 0;
  L.t64 = L.has_pre ? take(nrhs * v64) : 0;
  L.p64 = L.has_pre ? take(size_t(nrhs) * nshift * v64) : 0;
  L.thi = take(nrhs * v64);
  L.bb = take(nrhs * v64);
  L.xb = take(nrhs * v64);
  L.st = take(size_t(nrhs) * sizeof(SysState));
  L.gf = take(sizeof(GlobalFlags));
  L.params = take(size_t(nrhs) * (1 + nshift) * sizeof(double));
  L.pt = take(nparts * 8);
  L.pr = take(nparts * 8);
  L.pp = take(nparts * 8);
  L.pb = take(nparts * 8);
  L.pres = take(nparts * 8);
  L.resn = take(size_t(nrhs) * nshift * 8);
  L.has_links = !(iprec == LQCD_F64 && ifmt == LQCD_LINKS18);
  L.links = L.has_links ? take(size_t(8) * link_reals(ifmt) * g.Vh * ri) : 0;
  // the FP64 opening phase streams FP64 links in the inner format (12-real:
  // a third fewer link bytes than the 18-real copy used for residuals;
  // 12-real + determinant for links with U(1) phases)
  L.links_pre =
      (L.has_pre && ifmt != LQCD_LINKS18) ? take(size_t(8) * link_reals(ifmt) * g.Vh * 8) : 0;
  // deferred shift updates: base directions and window coefficients
  if (L.win > 1) {
    L.pc = take(nrhs * vin);
    L.pc64 = L.has_pre ? take(nrhs * v64) : 0;
    L.wc = take(size_t(nrhs) * sizeof(WinCoef));
  }
  L.total = off;
  return L;
}

// Pinned staging: [0, kPinnedParams) receives the flag word, parameters follow.
constexpr size_t kPinnedParams = 256;

// Process-wide resources: pinned host staging, capture stream, graph cache.
struct Global {
  std::mutex mu;
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipStream_t cap = nullptr;
  std::map<std::string, hipGraphExec_t> graphs;
};
Global& G() {
  static Global g;
  return g;
}

int pinned(size_t n, void** out) {
  Global& gl = G();
  if (gl.pinned_bytes < n) {
    if (gl.pinned) (void)hipHostFree(gl.pinned);
    gl.pinned = nullptr;
    gl.pinned_bytes = 0;
    LQCD_HIP_TRY(hipHostMalloc(&gl.pinned, n, hipHostMallocDefault));
    gl.pinned_bytes = n;
  }
  *out = gl.pinned;
  return LQCD_OK;
}

void clear_graphs() {
  for (auto& kv : G().graphs) (void)hipGraphExecDestroy(kv.second);
  G().graphs.clear();
}

// Kernel timing (instrumentation): when enabled, D_oe, D_eo and multi-shift
// update launches are bracketed by HIP events on their stream and their
// durations accumulate per kernel class.  Solves then run without graphs.
struct Timing {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> pool;
  struct Pending {
    hipEvent_t a, b;
    std::string cls;
  };
  std::vector<Pending> pending;
  std::vector<std::string> order;
  std::map<std::string, std::pair<int64_t, double>> acc;  // launches, total ms
};
Timing& T() {
  static Timing t;
  return t;
}

bool timing_on() {
  std::lock_guard<std::mutex> lk(T().mu);
  return T().on;
}

hipEvent_t timing_event() {
  Timing& t = T();
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records the start event of a timed launch (nullptr when timing is off).
hipEvent_t timing_begin(hipStream_t s) {
  std::lock_guard<std::mutex> lk(T().mu);
  if (!T().on) return nullptr;
  hipEvent_t e = timing_event();
  if (e) (void)hipEventRecord(e, s);
  return e;
}

void timing_end(hipEvent_t a, hipStream_t s, const std::string& cls) {
  if (!a) return;
  std::lock_guard<std::mutex> lk(T().mu);
  hipEvent_t b = timing_event();
  if (!b) return;
  (void)hipEventRecord(b, s);
  T().pending.push_back({a, b, cls});
}

// Folds completed event pairs into the totals (the stream has been synchronised).
void timing_resolve() {
  std::lock_guard<std::mutex> lk(T().mu);
  Timing& t = T();
  for (auto& p : t.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      if (!t.acc.count(p.cls)) t.order.push_back(p.cls);
      t.acc[p.cls].first += 1;
      t.acc[p.cls].second += ms;
    }
    t.pool.push_back(p.a);
    t.pool.push_back(p.b);
  }
  t.pending.clear();
}

struct Ctx {
  KGeom g;
  lqcd_solver_params p;
  int iprec, ifmt;
  const void* U64;
  const void* Uin;
  char* ws;
  Layout L;
  hipStream_t s;
  double m2;
  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
};

// One way of running the Krylov iteration: its arithmetic, links, vectors and
// stencil configurations.
struct Phase {
  int prec = LQCD_F64, fmt = LQCD_LINKS18;
  const void* U = nullptr;
  size_t r = 0, t = 0, p = 0;  // workspace offsets of r, t (odd), p_s
  size_t pc = 0;               // base direction (deferred shift updates)
  int pairs = 0;               // pc and t hold the systems in interleaved pairs (FP32)
  void* x = nullptr;           // solution accumulator: FP64 solutions or FP32 partial sums
  DslashCfg c_oe, c_eo;
  int nb_oe = 0, nb_eo = 0;
  double rel_d2 = 0.0;  // reliable-update trigger (0: never)
  double sw2 = 0.0;     // FP64 -> FP32 switch level (0: never)
};

// One run of the iteration on nsys independent systems.
struct Core {
  int nsys, nshift, base;
  bool guess;
  const double2* b;  // [nsys][3][Vh] FP64
  double2* x;        // [nsys][nshift][3][Vh] FP64
  double tol;
  Phase main, pre;   // pre: FP64 opening phase of a mixed multi-shift solve
  bool two_phase;
  DslashCfg c64_oe, c64_eo;  // FP64 18-real: residuals and verification
  int nb64_eo, nbv;
  int poll;
  int win;  // deferred shift updates when > 1
};

bool is_mixed(const Ctx& c) { return c.iprec == LQCD_F32; }

// LQCD_RHS_PAIRS=0 keeps the FP32 base directions and t one system after the
// other (for comparisons); unset or any other value: pairs wherever they apply.
bool rhs_pairs_enabled() {
  const char* e = std::getenv("LQCD_RHS_PAIRS");
  return !(e && e[0] == '0');
}

// residual ring slots per system (1: r updated in place)
int rslots(const Core& k) { return k.win > 1 ? k.win + 1 : 1; }

int64_t vstride(const Ctx& c) { return int64_t(3) * c.g.Vh; }

size_t cbytes(int prec) { return prec == LQCD_F32 ? 8 : 16; }  // bytes per complex

char* vec_at(const Ctx& c, size_t off, int prec, int64_t index) {
  return c.ws + off + size_t(index) * vstride(c) * cbytes(prec);
}

DslashCall phase_call(const Ctx& c, const Core& k, const Phase& ph, int out_par) {
  DslashCall d;
  d.g = c.g;
  d.out_par = out_par;
  d.prec = ph.prec;
  d.fmt = ph.fmt;
  d.nrhs = k.nsys;
  d.U = ph.U;
  return d;
}

DslashCall fp64_call(const Ctx& c, const Core& k, int out_par) {
  DslashCall d;
  d.g = c.g;
  d.out_par = out_par;
  d.prec = LQCD_F64;
  d.fmt = LQCD_LINKS18;
  d.nrhs = k.nsys;
  d.U = c.U64;
  return d;
}

// K6 and the window reset: applies every open window of deferred shift updates.
int launch_flush(const Ctx& c, const Core& k, const Phase& ph, hipStream_t s) {
  SysState* st = c.at<SysState>(c.L.st);
  WinCoef* wc = c.at<WinCoef>(c.L.wc);
  const dim3 grid(k.nbv, k.nsys);
  const std::string tag = std::string(ph.prec == LQCD_F32 ? "_f32" : "_f64") + "_n" +
                          std::to_string(k.nsys);
  hipEvent_t ev = timing_begin(s);
#define LQCD_FLUSH(RI, WM)                                                                     \
  hipLaunchKernelGGL((k_ms_flush<RI, RI, WM>), grid, dim3(kVecBlock), 0, s, st, wc,            \
                     c.at<const cplx<RI>>(ph.r), rslots(k), c.at<cplx<RI>>(ph.p),              \
                     static_cast<cplx<RI>*>(ph.x), k.nshift, k.win, c.g.Vh)
  if (ph.prec == LQCD_F32) {
    if (k.win <= 8) LQCD_FLUSH(float, 8);
    else if (k.win <= 16) LQCD_FLUSH(float, 16);
    else LQCD_FLUSH(float, 32);
  } else {
    if (k.win <= 8) LQCD_FLUSH(double, 8);
    else if (k.win <= 16) LQCD_FLUSH(double, 16);
    else LQCD_FLUSH(double, 32);
  }
#undef LQCD_FLUSH
  LQCD_LAUNCH_CHECK();
  timing_end(ev, s, "ms_flush" + tag);
  hipLaunchKernelGGL(k_sc_win_reset, dim3(k.nsys), dim3(kScalarThreads), 0, s, st, wc, k.nshift,
                     ph.prec == LQCD_F64 ? 1 : 0, 0);
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

int launch_iteration(const Ctx& c, const Core& k, const Phase& ph, hipStream_t s, bool flush) {
  SysState* st = c.at<SysState>(c.L.st);
  GlobalFlags* gf = c.at<GlobalFlags>(c.L.gf);
  const int64_t vs = vstride(c);
  const bool win = k.win > 1;
  int rc;
  // K1: t = D_oe p_base
  DslashCall d1 = phase_call(c, k, ph, 1);
  d1.mode = DM_PLAIN;
  d1.in = win ? c.ws + ph.pc : vec_at(c, ph.p, ph.prec, k.base);
  d1.in_stride = win ? vs : int64_t(k.nshift) * vs;
  d1.out = c.ws + ph.t;
  d1.out_stride = vs;
  d1.pairs = ph.pairs;
  d1.live = &st->live;
  d1.live_stride = kStateStrideI;
  d1.halt = &gf->all_done;
  d1.partials = c.at<double>(c.L.pt);
  const std::string tag = std::string(ph.prec == LQCD_F32 ? "_f32" : "_f64") +
                          (k.guess ? "_refine" : "") + "_n" + std::to_string(k.nsys);
  hipEvent_t ev = timing_begin(s);
  if ((rc = dslash_launch(d1, ph.c_oe, s))) return rc;
  timing_end(ev, s, "dslash_oe" + tag);
  // K2
  hipLaunchKernelGGL(k_sc_alpha, dim3(k.nsys), dim3(kScalarThreads), 0, s, st, gf, k.nshift,
                     c.at<double>(c.L.pt), ph.nb_oe, c.at<double>(c.L.pp), k.nbv);
  LQCD_LAUNCH_CHECK();
  // K3: r -= a (m2s p - D_eo t)
  DslashCall d3 = phase_call(c, k, ph, 0);
  d3.mode = DM_CG;
  d3.in = c.ws + ph.t;
  d3.in_stride = vs;
  d3.diag = win ? c.ws + ph.pc : vec_at(c, ph.p, ph.prec, k.base);
  d3.diag_stride = win ? vs : int64_t(k.nshift) * vs;
  d3.r = c.ws + ph.r;
  d3.r_stride = vs;
  d3.pairs = ph.pairs;
  if (win) {
    d3.r_iter = &st->iters;
    d3.r_iter_stride = kStateStrideI;
    d3.r_slots = rslots(k);
  }
  d3.m2s = &st->m2s;
  d3.m2s_stride = kStateStrideD;
  d3.alpha = &st->a;
  d3.alpha_stride = kStateStrideD;
  d3.live = &st->upd_any;
  d3.live_stride = kStateStrideI;
  d3.halt = &gf->all_done;
  d3.partials = c.at<double>(c.L.pr);
  d3.rev = 1;  // against D_oe's order: the last t it wrote is read first (MALL hits)
  ev = timing_begin(s);
  if ((rc = dslash_launch(d3, ph.c_eo, s))) return rc;
  timing_end(ev, s, "dslash_eo_cg" + tag);
  // K4
  hipLaunchKernelGGL(k_sc_beta, dim3(k.nsys), dim3(kScalarThreads), 0, s, st, gf, k.nshift,
                     c.at<double>(c.L.pr), ph.nb_eo, c.p.max_iter, ph.rel_d2, ph.sw2,
                     ph.prec == LQCD_F64 ? 1 : 0, win ? c.at<WinCoef>(c.L.wc) : nullptr, k.win);
  LQCD_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sc_flags, dim3(1), dim3(64), 0, s, st, gf, k.nsys);
  LQCD_LAUNCH_CHECK();
  // K5
  const dim3 grid(k.nbv, k.nsys);
  if (win) {
    ev = timing_begin(s);
    if (ph.pairs)
      hipLaunchKernelGGL(k_base_update_pairs, dim3(k.nbv, k.nsys / 2), dim3(kVecBlock), 0, s, st,
                         c.at<const float2>(ph.r), rslots(k), c.at<float4>(ph.pc), k.base,
                         c.g.Vh, c.at<double>(c.L.pp));
    else if (ph.prec == LQCD_F32)
      hipLaunchKernelGGL(k_base_update<float>, grid, dim3(kVecBlock), 0, s, st,
                         c.at<const float2>(ph.r), rslots(k), c.at<float2>(ph.pc), k.base,
                         c.g.Vh, c.at<double>(c.L.pp));
    else
      hipLaunchKernelGGL(k_base_update<double>, grid, dim3(kVecBlock), 0, s, st,
                         c.at<const double2>(ph.r), rslots(k), c.at<double2>(ph.pc), k.base,
                         c.g.Vh, c.at<double>(c.L.pp));
    LQCD_LAUNCH_CHECK();
    timing_end(ev, s, "base_update" + tag);
    return flush ? launch_flush(c, k, ph, s) : LQCD_OK;
  }
  ev = timing_begin(s);
  if (ph.prec == LQCD_F32)
    hipLaunchKernelGGL((k_ms_update<float, float>), grid, dim3(kVecBlock), 0, s, st,
                       c.at<const float2>(ph.r), c.at<float2>(ph.p), (float2*)ph.x, k.nshift,
                       k.base, c.g.Vh, c.at<double>(c.L.pp));
  else
    hipLaunchKernelGGL((k_ms_update<double, double>), grid, dim3(kVecBlock), 0, s, st,
                       c.at<const double2>(ph.r), c.at<double2>(ph.p), (double2*)ph.x, k.nshift,
                       k.base, c.g.Vh, c.at<double>(c.L.pp));
  LQCD_LAUNCH_CHECK();
  timing_end(ev, s, "ms_update" + tag);
  return LQCD_OK;
}

// r = b - A_{sigma_0} x_base in FP64 (stored in the main phase's precision)
int launch_residual(const Ctx& c, const Core& k, const double* m2s, int m2s_stride,
                    const int* live, double* part, hipStream_t s) {
  const int64_t vs = vstride(c);
  int rc;
  DslashCall e1 = fp64_call(c, k, 1);
  e1.mode = DM_PLAIN;
  e1.in = k.x + int64_t(k.base) * vs;
  e1.in_stride = int64_t(k.nshift) * vs;
  e1.out = c.ws + c.L.thi;
  e1.out_stride = vs;
  e1.live = live;
  e1.live_stride = kStateStrideI;
  if ((rc = dslash_launch(e1, k.c64_oe, s))) return rc;
  DslashCall e2 = fp64_call(c, k, 0);
  e2.mode = DM_RES;
  e2.r_prec = k.main.prec;
  e2.in = c.ws + c.L.thi;
  e2.in_stride = vs;
  e2.diag = k.x + int64_t(k.base) * vs;
  e2.diag_stride = int64_t(k.nshift) * vs;
  e2.b = k.b;
  e2.b_stride = vs;
  e2.r = c.ws + k.main.r;
  e2.r_stride = vs;
  if (rslots(k) > 1) {  // the residual of the current iteration's ring slot
    e2.r_iter = &c.at<SysState>(c.L.st)->iters;
    e2.r_iter_stride = kStateStrideI;
    e2.r_slots = rslots(k);
  }
  e2.m2s = m2s;
  e2.m2s_stride = m2s_stride;
  e2.live = live;
  e2.live_stride = kStateStrideI;
  e2.partials = part;
  return dslash_launch(e2, k.c64_eo, s);
}

int launch_reliable(const Ctx& c, const Core& k, hipStream_t s) {
  SysState* st = c.at<SysState>(c.L.st);
  GlobalFlags* gf = c.at<GlobalFlags>(c.L.gf);
  int rc;
  // open windows are applied first, so that x_lo and every p_s are current
  if (k.win > 1 && (rc = launch_flush(c, k, k.main, s))) return rc;
  hipLaunchKernelGGL(k_sc_rel_begin, dim3(1), dim3(64), 0, s, st, gf, k.nsys, k.nshift);
  LQCD_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_accum, dim3(k.nbv, k.nsys * k.nshift), dim3(kVecBlock), 0, s, st,
                     c.at<float2>(c.L.xlo), k.x, k.nshift, c.g.Vh);
  LQCD_LAUNCH_CHECK();
  rc = launch_residual(c, k, &st->m2s, kStateStrideD, &st->rel, c.at<double>(c.L.pres), s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_sc_reliable, dim3(1), dim3(kScalarThreads), 0, s, st, gf, k.nsys,
                     k.nshift, k.base, c.at<double>(c.L.pres), k.nb64_eo, c.p.max_iter);
  LQCD_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_restart_dirs<float>, dim3(k.nbv, k.nsys), dim3(kVecBlock), 0, s, st,
                     c.at<const float2>(c.L.r), rslots(k), c.at<float2>(c.L.p),
                     k.win > 1 ? c.at<float2>(c.L.pc) : nullptr, k.main.pairs, k.nshift,
                     k.base, c.g.Vh,
                     c.at<double>(c.L.pp));
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

std::string graph_key(const Ctx& c, const Core& k, const Phase& ph) {
  std::string key;
  auto add = [&](const void* p, size_t n) { key.append(static_cast<const char*>(p), n); };
  add(&c.g, sizeof(c.g));
  add(&c.ws, sizeof(void*));
  add(&c.L.total, sizeof(size_t));
  add(&c.p.max_iter, sizeof(int));
  add(&k.nsys, sizeof(int));
  add(&k.nshift, sizeof(int));
  add(&k.base, sizeof(int));
  add(&k.nbv, sizeof(int));
  add(&k.poll, sizeof(int));
  add(&k.win, sizeof(int));
  add(&ph.prec, sizeof(int));
  add(&ph.fmt, sizeof(int));
  add(&ph.U, sizeof(void*));
  add(&ph.r, sizeof(size_t));
  add(&ph.t, sizeof(size_t));
  add(&ph.p, sizeof(size_t));
  add(&ph.pc, sizeof(size_t));
  add(&ph.pairs, sizeof(int));
  add(&ph.x, sizeof(void*));
  add(&ph.c_oe, sizeof(DslashCfg));
  add(&ph.c_eo, sizeof(DslashCfg));
  add(&ph.rel_d2, sizeof(double));
  add(&ph.sw2, sizeof(double));
  return key;
}

int iteration_graph(const Ctx& c, const Core& k, const Phase& ph, hipGraphExec_t* out) {
  Global& gl = G();
  const std::string key = graph_key(c, k, ph);
  auto it = gl.graphs.find(key);
  if (it != gl.graphs.end()) {
    *out = it->second;
    return LQCD_OK;
  }
  if (gl.graphs.size() >= 32) clear_graphs();
  if (!gl.cap) LQCD_HIP_TRY(hipStreamCreateWithFlags(&gl.cap, hipStreamNonBlocking));
  LQCD_HIP_TRY(hipStreamBeginCapture(gl.cap, hipStreamCaptureModeThreadLocal));
  int rc = LQCD_OK;
  for (int i = 0; i < k.poll && rc == LQCD_OK; ++i)
    rc = launch_iteration(c, k, ph, gl.cap, (i + 1) % k.win == 0);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(gl.cap, &graph);
  if (rc != LQCD_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) {
    set_error("graph capture failed: %s", hipGetErrorString(e));
    return LQCD_ERR_HIP;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) {
    set_error("graph instantiation failed: %s", hipGetErrorString(e2));
    return LQCD_ERR_HIP;
  }
  gl.graphs[key] = exec;
  *out = exec;
  return LQCD_OK;
}

bool debug_enabled() {
  const char* e = std::getenv("LQCD_DEBUG");
  return e && e[0] == '1';
}

// LQCD_DEBUG=1: print the scalars of every system (synchronises the stream).
void debug_dump(const Ctx& c, const Core& k, const char* where) {
  if (!debug_enabled()) return;
  std::vector<SysState> h(k.nsys);
  if (hipStreamSynchronize(c.s) != hipSuccess ||
      hipMemcpy(h.data(), c.at<SysState>(c.L.st), sizeof(SysState) * k.nsys,
                hipMemcpyDeviceToHost) != hipSuccess)
    return;
  for (int j = 0; j < k.nsys; ++j)
    fprintf(stderr,
            "[lqcd debug] %s sys %d: it=%d done=%d conv=%d err=%d lowres=%d nrel=%d rho=%.3e "
            "pp=%.3e a=%.3e target2=%.3e m2s=%.3e\n",
            where, j, h[j].iters, h[j].done, h[j].conv, h[j].err, h[j].lowres, h[j].nrel,
            h[j].rho, h[j].pp, h[j].a, h[j].target2, h[j].m2s);
}

int read_flags(const Ctx& c, GlobalFlags* host) {
  void* pin = nullptr;
  int rc = pinned(kPinnedParams, &pin);
  if (rc) return rc;
  GlobalFlags* hf = static_cast<GlobalFlags*>(pin);  // flags live in [0, kPinnedParams)
  LQCD_HIP_TRY(hipMemcpyAsync(hf, c.at<GlobalFlags>(c.L.gf), sizeof(GlobalFlags),
                              hipMemcpyDeviceToHost, c.s));
  LQCD_HIP_TRY(hipStreamSynchronize(c.s));
  *host = *hf;
  timing_resolve();
  return LQCD_OK;
}

int tune_phase(const Ctx& c, const Core& k, Phase& ph) {
  int rc;
  DslashCall t = phase_call(c, k, ph, 1);
  t.pairs = ph.pairs;
  if ((rc = dslash_tuned(t, c.p.rhs_block, c.s, &ph.c_oe))) return rc;
  t.out_par = 0;
  t.mode = DM_CG;
  if ((rc = dslash_tuned(t, c.p.rhs_block, c.s, &ph.c_eo))) return rc;
  ph.nb_oe = dslash_nblocks(c.g, ph.c_oe);
  ph.nb_eo = dslash_nblocks(c.g, ph.c_eo);
  return LQCD_OK;
}

// Fills the phases of k for this context and tunes every stencil they use.
int setup_core(const Ctx& c, Core& k) {
  int rc;
  const bool mixed = is_mixed(c);
  Phase& m = k.main;
  m.prec = c.iprec;
  m.fmt = c.ifmt;
  m.U = c.Uin;
  m.r = c.L.r;
  m.t = c.L.t;
  m.p = c.L.p;
  m.pc = c.L.pc;
  k.win = k.nshift > 1 ? c.L.win : 1;
  m.x = mixed ? static_cast<void*>(c.ws + c.L.xlo) : static_cast<void*>(k.x);
  m.rel_d2 = mixed ? c.p.reliable_delta * c.p.reliable_delta : 0.0;
  m.sw2 = 0.0;
  // The FP32 stencils read and write the base direction and t as pairs of
  // systems when there is an even number of them (16-byte accesses).
  m.pairs = mixed && k.win > 1 && k.nsys % 2 == 0 &&
            (c.ifmt == LQCD_LINKS12 || c.ifmt == LQCD_LINKS18) && c.p.rhs_block != 1 &&
            rhs_pairs_enabled();
  k.two_phase = mixed && c.L.has_pre && !k.guess && k.nshift > 1;
  if (k.two_phase) {
    Phase& q = k.pre;
    q.prec = LQCD_F64;
    q.fmt = c.ifmt;
    q.U = c.ifmt != LQCD_LINKS18 ? static_cast<const void*>(c.ws + c.L.links_pre) : c.U64;
    q.r = c.L.r64;
    q.t = c.L.t64;
    q.p = c.L.p64;
    q.pc = c.L.pc64;
    q.x = k.x;
    q.rel_d2 = 0.0;
    q.sw2 = c.p.mixed_switch * c.p.mixed_switch;
    if ((rc = tune_phase(c, k, q))) return rc;
  }
  if ((rc = tune_phase(c, k, m))) return rc;
  DslashCall f = fp64_call(c, k, 1);
  if ((rc = dslash_tuned(f, 0, c.s, &k.c64_oe))) return rc;
  f.out_par = 0;
  f.mode = DM_RES;
  if ((rc = dslash_tuned(f, 0, c.s, &k.c64_eo))) return rc;
  k.nb64_eo = dslash_nblocks(c.g, k.c64_eo);
  k.nbv = (c.g.Vh + kVecBlock - 1) / kVecBlock;
  return LQCD_OK;
}

// Replays blocks of `poll` iterations of phase ph until every system is done
// (or, for the FP64 opening phase, below the switch level).  With reliable
// updates the FP64 residual is recomputed when requested, every
// reliable_interval iterations, and before accepting convergence.
int run_phase(const Ctx& c, const Core& k, const Phase& ph, bool reliable, bool stop_on_switch,
              int* iters_run, GlobalFlags* f) {
  int rc;
  hipGraphExec_t exec = nullptr;
  if (c.p.use_graph && !timing_on() && (rc = iteration_graph(c, k, ph, &exec))) return rc;
  const int ri = std::max(1, c.p.reliable_interval);
  int since_rel = 0;
  while (!f->all_done && !f->error && !(stop_on_switch && f->phase_done)) {
    if (exec) {
      LQCD_HIP_TRY(hipGraphLaunch(exec, c.s));
    } else {
      for (int i = 0; i < k.poll; ++i)
        if ((rc = launch_iteration(c, k, ph, c.s, (i + 1) % k.win == 0))) return rc;
    }
    *iters_run += k.poll;
    since_rel += k.poll;
    if ((rc = read_flags(c, f))) return rc;
    debug_dump(c, k, ph.prec == LQCD_F32 ? "poll32" : "poll64");
    if (reliable && !f->error && (f->rel_req || f->all_done || since_rel >= ri)) {
      if ((rc = launch_reliable(c, k, c.s))) return rc;
      since_rel = 0;
      if ((rc = read_flags(c, f))) return rc;
      debug_dump(c, k, "reliable");
    }
    if (*iters_run > c.p.max_iter + 2 * k.poll) break;  // device limits iterations; host guard
  }
  return LQCD_OK;
}

// Runs the Krylov iteration to convergence (or max_iter) for k.nsys systems.
int core_solve(const Ctx& c, Core& k, const double* m2s_host, const double* delta_host,
               std::vector<SysState>* state_out) {
  int rc;
  if ((rc = setup_core(c, k))) return rc;
  const hipStream_t s = c.s;
  SysState* st = c.at<SysState>(c.L.st);
  GlobalFlags* gf = c.at<GlobalFlags>(c.L.gf);
  double* dparams = c.at<double>(c.L.params);
  const bool mixed = is_mixed(c);

  // per-system parameters
  const size_t np = size_t(k.nsys) * (1 + k.nshift);
  void* pin = nullptr;
  if ((rc = pinned(kPinnedParams + np * sizeof(double), &pin))) return rc;
  double* hp = reinterpret_cast<double*>(static_cast<char*>(pin) + kPinnedParams);
  for (int j = 0; j < k.nsys; ++j) hp[j] = m2s_host[j];
  for (size_t i = 0; i < size_t(k.nsys) * k.nshift; ++i) hp[k.nsys + i] = delta_host[i];
  LQCD_HIP_TRY(hipMemcpyAsync(dparams, hp, np * sizeof(double), hipMemcpyHostToDevice, s));

  const dim3 gv(k.nbv, k.nsys);
  hipLaunchKernelGGL(k_norm2_f64, gv, dim3(kVecBlock), 0, s, k.b, vstride(c), c.g.Vh,
                     c.at<double>(c.L.pb));
  LQCD_LAUNCH_CHECK();
  const Phase& first = k.two_phase ? k.pre : k.main;
  int nb_r = k.nbv;
  if (k.guess) {
    if ((rc = launch_residual(c, k, dparams, 1, nullptr, c.at<double>(c.L.pr), s))) return rc;
    nb_r = k.nb64_eo;
  } else if (first.prec == LQCD_F32) {
    hipLaunchKernelGGL(k_copy_to_inner<float>, gv, dim3(kVecBlock), 0, s, k.b,
                       c.at<float2>(first.r), rslots(k), c.g.Vh, c.at<double>(c.L.pr));
  } else {
    hipLaunchKernelGGL(k_copy_to_inner<double>, gv, dim3(kVecBlock), 0, s, k.b,
                       c.at<double2>(first.r), rslots(k), c.g.Vh, c.at<double>(c.L.pr));
  }
  LQCD_LAUNCH_CHECK();
  if (first.prec == LQCD_F32) {
    if (!k.guess) {
      const int64_t n = int64_t(k.nsys) * k.nshift * vstride(c);
      hipLaunchKernelGGL(k_zero<double2>, dim3(2048), dim3(kVecBlock), 0, s, k.x, n);
      LQCD_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL((k_init_dirs<float, float>), gv, dim3(kVecBlock), 0, s,
                       c.at<const float2>(first.r), rslots(k), c.at<float2>(first.p),
                       (float2*)first.x,
                       k.win > 1 ? c.at<float2>(first.pc) : nullptr, first.pairs, k.nshift, 1,
                       c.g.Vh,
                       c.at<double>(c.L.pp));
  } else {
    hipLaunchKernelGGL((k_init_dirs<double, double>), gv, dim3(kVecBlock), 0, s,
                       c.at<const double2>(first.r), rslots(k), c.at<double2>(first.p), k.x,
                       k.win > 1 ? c.at<double2>(first.pc) : nullptr, 0, k.nshift,
                       k.guess ? 0 : 1, c.g.Vh, c.at<double>(c.L.pp));
  }
  LQCD_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sc_init, dim3(1), dim3(kScalarThreads), 0, s, st, gf, k.nsys, k.nshift,
                     dparams, k.tol * k.tol, first.sw2, c.at<double>(c.L.pb), k.nbv,
                     c.at<double>(c.L.pr), nb_r, c.at<double>(c.L.pp), k.nbv);
  LQCD_LAUNCH_CHECK();
  if (k.win > 1) {
    hipLaunchKernelGGL(k_sc_win_reset, dim3(k.nsys), dim3(kScalarThreads), 0, s, st,
                       c.at<WinCoef>(c.L.wc), k.nshift, 0, 1);
    LQCD_LAUNCH_CHECK();
  }

  int iters_run = 0;
  GlobalFlags f{};
  if ((rc = read_flags(c, &f))) return rc;
  debug_dump(c, k, "init");
  if (k.two_phase) {
    // FP64 opening phase until every system's residual is below mixed_switch |b|
    if ((rc = run_phase(c, k, k.pre, false, true, &iters_run, &f))) return rc;
    if (k.win > 1 && (rc = launch_flush(c, k, k.pre, s))) return rc;
    if (!f.all_done && !f.error) {
      const bool w = k.win > 1;
      hipLaunchKernelGGL(k_to_fp32, gv, dim3(kVecBlock), 0, s, st, rslots(k),
                         c.at<const double2>(c.L.r64),
                         c.at<const double2>(c.L.p64),
                         w ? c.at<const double2>(c.L.pc64) : nullptr, c.at<float2>(c.L.r),
                         c.at<float2>(c.L.p), w ? c.at<float2>(c.L.pc) : nullptr,
                         k.main.pairs, c.at<float2>(c.L.xlo), k.nshift, k.base, c.g.Vh,
                         c.at<double>(c.L.pp));
      LQCD_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_sc_phase2, dim3(1), dim3(64), 0, s, st, k.nsys, k.nshift);
      LQCD_LAUNCH_CHECK();
      debug_dump(c, k, "switch");
    }
  }
  if ((rc = run_phase(c, k, k.main, mixed, false, &iters_run, &f))) return rc;
  // a mixed solve that stopped on the iteration limit still folds its FP32 sums in
  if (mixed && !f.error) {
    if ((rc = launch_reliable(c, k, s))) return rc;
  } else if (k.win > 1 && (rc = launch_flush(c, k, k.main, s))) {
    return rc;
  }
  state_out->resize(k.nsys);
  LQCD_HIP_TRY(hipMemcpyAsync(state_out->data(), st, sizeof(SysState) * k.nsys,
                              hipMemcpyDeviceToHost, s));
  LQCD_HIP_TRY(hipStreamSynchronize(s));
  timing_resolve();  // launches after the last flag read belong to this solve
  if (f.error) {
    set_error("solver hit a non-finite value or non-positive curvature");
    return LQCD_ERR_NUMERIC;
  }
  return LQCD_OK;
}

// |b_j - (m^2 + sigma_s) x_js + D_eo D_oe x_js|^2 for every (j, s), FP64.
int verify(const Ctx& c, Core& k, const double* sigma, std::vector<double>* res2) {
  const int64_t vs = vstride(c);
  int rc;
  double* dres = c.at<double>(c.L.resn);
  for (int s = 0; s < k.nshift; ++s) {
    DslashCall e1 = fp64_call(c, k, 1);
    e1.mode = DM_PLAIN;
    e1.in = k.x + int64_t(s) * vs;
    e1.in_stride = int64_t(k.nshift) * vs;
    e1.out = c.ws + c.L.thi;
    e1.out_stride = vs;
    if ((rc = dslash_launch(e1, k.c64_oe, c.s))) return rc;
    DslashCall e2 = fp64_call(c, k, 0);
    e2.mode = DM_RES;
    e2.r_prec = LQCD_F64;
    e2.in = c.ws + c.L.thi;
    e2.in_stride = vs;
    e2.diag = k.x + int64_t(s) * vs;
    e2.diag_stride = int64_t(k.nshift) * vs;
    e2.b = k.b;
    e2.b_stride = vs;
    e2.r = nullptr;
    e2.m2s_c = c.m2 + sigma[s];
    e2.partials = c.at<double>(c.L.pres);
    if ((rc = dslash_launch(e2, k.c64_eo, c.s))) return rc;
    hipLaunchKernelGGL(k_reduce_vec, dim3(k.nsys), dim3(kVecBlock), 0, c.s,
                       c.at<const double>(c.L.pres), k.nb64_eo, dres + int64_t(s) * k.nsys);
    LQCD_LAUNCH_CHECK();
  }
  res2->resize(size_t(k.nsys) * k.nshift);
  std::vector<double> tmp(size_t(k.nsys) * k.nshift);
  LQCD_HIP_TRY(hipMemcpyAsync(tmp.data(), dres, tmp.size() * 8, hipMemcpyDeviceToHost, c.s));
  LQCD_HIP_TRY(hipStreamSynchronize(c.s));
  for (int s = 0; s < k.nshift; ++s)
    for (int j = 0; j < k.nsys; ++j) (*res2)[size_t(j) * k.nshift + s] = tmp[size_t(s) * k.nsys + j];
  return LQCD_OK;
}

int check_params(const lqcd_solver_params* p) {
  if (!p) {
    set_error("params is NULL");
    return LQCD_ERR_INVALID_ARG;
  }
  if (!(p->mass > 0.0) || !std::isfinite(p->mass)) {
    set_error("mass = %g must be finite and > 0", p->mass);
    return LQCD_ERR_INVALID_ARG;
  }
  if (!(p->tol > 0.0 && p->tol < 1.0)) {
    set_error("tol = %g must be in (0, 1)", p->tol);
    return LQCD_ERR_INVALID_ARG;
  }
  if (p->max_iter <= 0) {
    set_error("max_iter = %d must be > 0", p->max_iter);
    return LQCD_ERR_INVALID_ARG;
  }
  int rc = check_prec_fmt(p->inner_prec, p->inner_fmt);
  if (rc) return rc;
  if (p->inner_prec == LQCD_F32 && !(p->reliable_delta > 0.0 && p->reliable_delta < 1.0)) {
    set_error("reliable_delta = %g must be in (0, 1)", p->reliable_delta);
    return LQCD_ERR_INVALID_ARG;
  }
  if (p->inner_prec == LQCD_F32 && !(p->mixed_switch >= 0.0 && p->mixed_switch < 1.0)) {
    set_error("mixed_switch = %g must be in [0, 1)", p->mixed_switch);
    return LQCD_ERR_INVALID_ARG;
  }
  if (!(p->inner_tol_factor > 0.0 && p->inner_tol_factor <= 1.0)) {
    set_error("inner_tol_factor = %g must be in (0, 1]", p->inner_tol_factor);
    return LQCD_ERR_INVALID_ARG;
  }
  if (p->inner_prec == LQCD_F32 && p->reliable_interval <= 0) {
    set_error("reliable_interval = %d must be > 0 for mixed precision", p->reliable_interval);
    return LQCD_ERR_INVALID_ARG;
  }
  if (p->use_graph != 0 && p->use_graph != 1) {
    set_error("use_graph must be 0 or 1");
    return LQCD_ERR_INVALID_ARG;
  }
  if (p->rhs_block != 0 && p->rhs_block != 1 && p->rhs_block != 2 && p->rhs_block != 4 &&
      p->rhs_block != 8) {
    set_error("rhs_block = %d must be 0, 1, 2, 4 or 8", p->rhs_block);
    return LQCD_ERR_INVALID_ARG;
  }
  if (p->shift_window < 1 || p->shift_window > kMaxWin) {
    set_error("shift_window = %d must be in [1, %d]", p->shift_window, kMaxWin);
    return LQCD_ERR_INVALID_ARG;
  }
  if (p->poll_interval < 0 || p->max_refine < 0) {
    set_error("poll_interval and max_refine must be >= 0");
    return LQCD_ERR_INVALID_ARG;
  }
  return LQCD_OK;
}

// Shared driver of lqcd_cg (nshift = 1, x holds a guess) and lqcd_cg_multishift.
int solve(const lqcd_geom* geom, const lqcd_solver_params* params, const void* U64,
          const void* Uinner, int32_t nshift, const double* sigma, const void* b, void* x,
          int32_t nrhs, bool guess, lqcd_solve_stats* stats, void* ws, size_t ws_bytes,
          void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  clear_error();
  int rc;
  if ((rc = check_geom(geom)) || (rc = check_params(params)) || (rc = check_ptr(U64, "U64")) ||
      (rc = check_ptr(b, "b")) || (rc = check_ptr(x, "x")) || (rc = check_nrhs(nrhs)))
    return rc;
  if (Uinner && (rc = check_ptr(Uinner, "Uinner"))) return rc;
  if (!stats || !sigma) {
    set_error("stats and sigma must be host arrays");
    return LQCD_ERR_INVALID_ARG;
  }
  if (nshift < 1 || nshift > kMaxShift) {
    set_error("nshift = %d must be in [1, %d]", nshift, kMaxShift);
    return LQCD_ERR_INVALID_ARG;
  }
  for (int s = 0; s < nshift; ++s)
    if (!(sigma[s] >= 0.0) || !std::isfinite(sigma[s])) {
      set_error("sigma[%d] = %g must be finite and >= 0", s, sigma[s]);
      return LQCD_ERR_INVALID_ARG;
    }
  if (b == x) {
    set_error("b and x must not alias");
    return LQCD_ERR_INVALID_ARG;
  }
  Ctx c;
  c.g = make_kgeom(geom);
  c.p = *params;
  c.iprec = params->inner_prec;
  c.ifmt = params->inner_fmt;
  c.U64 = U64;
  c.L = make_layout(c.g, *params, nshift, nrhs);
  if (!ws || ws_bytes < c.L.total) {
    set_error("workspace of %zu bytes is too small: %zu needed", ws_bytes, c.L.total);
    return LQCD_ERR_WORKSPACE;
  }
  if ((rc = check_ptr(ws, "ws"))) return rc;
  c.ws = static_cast<char*>(ws);
  c.s = (hipStream_t)stream;
  c.m2 = params->mass * params->mass;

  std::lock_guard<std::mutex> lk(G().mu);
  if (!c.L.has_links) {
    c.Uin = U64;
  } else if (Uinner) {
    c.Uin = Uinner;
  } else {
    c.Uin = c.ws + c.L.links;
    if ((rc = convert_links_async(c.g, U64, LQCD_F64, LQCD_LINKS18, c.ws + c.L.links, c.iprec,
                                  c.ifmt, c.s)))
      return rc;
  }

  if (c.L.links_pre) {
    if ((rc = convert_links_async(c.g, U64, LQCD_F64, LQCD_LINKS18, c.ws + c.L.links_pre,
                                  LQCD_F64, c.ifmt, c.s)))
      return rc;
  }

  int base = 0;
  for (int s = 1; s < nshift; ++s)
    if (sigma[s] < sigma[base]) base = s;

  Core k{};
  k.nsys = nrhs;
  k.nshift = nshift;
  k.base = base;
  k.guess = guess;
  k.b = static_cast<const double2*>(b);
  k.x = static_cast<double2*>(x);
  k.tol = params->tol * params->inner_tol_factor;
  k.poll = poll_for(c.p);
  std::vector<double> m2s(nrhs, c.m2 + sigma[base]);
  std::vector<double> delta(size_t(nrhs) * nshift);
  for (int j = 0; j < nrhs; ++j)
    for (int s = 0; s < nshift; ++s) delta[size_t(j) * nshift + s] = sigma[s] - sigma[base];
  std::vector<SysState> main_state;
  const int rc_core = core_solve(c, k, m2s.data(), delta.data(), &main_state);
  if (rc_core && rc_core != LQCD_ERR_NUMERIC) return rc_core;

  std::vector<int> refine_iters(size_t(nrhs) * nshift, 0);
  std::vector<double> res2;
  if ((rc = verify(c, k, sigma, &res2))) return rc;
  // failing (rhs, shift) systems, shift-major so that a batch holds systems
  // with the same shift, which converge at the same rate
  auto failing = [&]() {
    std::vector<int> f;
    for (int s = 0; s < nshift; ++s)
      for (int j = 0; j < nrhs; ++j) {
        const double bn = main_state[j].bnorm2;
        const double r2 = res2[size_t(j) * nshift + s];
        if (!(r2 <= params->tol * params->tol * bn)) f.push_back(j * nshift + s);
      }
    return f;
  };
  int numeric = rc_core == LQCD_ERR_NUMERIC;
  for (int round = 0; round < params->max_refine && !numeric; ++round) {
    const std::vector<int> fail = failing();
    if (fail.empty()) break;
    const int64_t vs = vstride(c);
    const size_t vbytes = size_t(vs) * 16;
    for (size_t off = 0; off < fail.size(); off += size_t(nrhs)) {
      const int nb = int(std::min(fail.size() - off, size_t(nrhs)));
      std::vector<double> rm2s(nb), rdelta(nb, 0.0);
      double2* xb = c.at<double2>(c.L.xb);
      double2* bb = c.at<double2>(c.L.bb);
      for (int q = 0; q < nb; ++q) {
        const int js = fail[off + q], j = js / nshift, s = js % nshift;
        LQCD_HIP_TRY(hipMemcpyAsync(xb + q * vs, k.x + int64_t(js) * vs, vbytes,
                                    hipMemcpyDeviceToDevice, c.s));
        LQCD_HIP_TRY(hipMemcpyAsync(bb + q * vs, k.b + int64_t(j) * vs, vbytes,
                                    hipMemcpyDeviceToDevice, c.s));
        rm2s[q] = c.m2 + sigma[s];
      }
      Core r{};
      r.nsys = nb;
      r.nshift = 1;
      r.base = 0;
      r.guess = true;
      r.b = bb;
      r.x = xb;
      r.tol = 0.5 * params->tol;
      r.poll = k.poll;
      std::vector<SysState> rstate;
      const int rc2 = core_solve(c, r, rm2s.data(), rdelta.data(), &rstate);
      if (rc2 == LQCD_ERR_NUMERIC) numeric = 1;
      else if (rc2) return rc2;
      for (int q = 0; q < nb; ++q) {
        const int js = fail[off + q];
        LQCD_HIP_TRY(hipMemcpyAsync(k.x + int64_t(js) * vs, xb + q * vs, vbytes,
                                    hipMemcpyDeviceToDevice, c.s));
        refine_iters[js] += rstate[q].iters;
      }
    }
    if ((rc = verify(c, k, sigma, &res2))) return rc;
  }
  if (debug_enabled())
    for (int j = 0; j < nrhs; ++j)
      for (int s = 0; s < nshift; ++s)
        fprintf(stderr, "[lqcd debug] final rhs %d shift %d: rel residual %.3e refine %d\n", j, s,
                std::sqrt(res2[size_t(j) * nshift + s] / main_state[j].bnorm2),
                refine_iters[size_t(j) * nshift + s]);

  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  bool all_conv = true;
  for (int j = 0; j < nrhs; ++j)
    for (int s = 0; s < nshift; ++s) {
      const size_t i = size_t(j) * nshift + s;
      const double bn = main_state[j].bnorm2;
      lqcd_solve_stats& o = stats[i];
      o.iters = main_state[j].iters;
      o.iters_fp64 = main_state[j].iters64;
      o.shift_window = nshift > 1 ? c.L.win : 1;
      o.shift_updates_fp64 = main_state[j].upd64;
      o.shift_updates_fp32 = main_state[j].upd32;
      o.flush_shifts_fp64 = main_state[j].fsh64;
      o.flush_shifts_fp32 = main_state[j].fsh32;
      o.flush_slots_fp64 = main_state[j].fsl64;
      o.flush_slots_fp32 = main_state[j].fsl32;
      o.reliable_updates = main_state[j].nrel;
      o.refine_iters = refine_iters[i];
      o.true_rel_residual = bn > 0 ? std::sqrt(res2[i] / bn) : std::sqrt(res2[i]);
      o.converged = o.true_rel_residual <= params->tol ? 1 : 0;
      o.seconds = secs;
      all_conv &= o.converged == 1;
    }
  if (numeric) {
    set_error("solver hit a non-finite value or non-positive curvature");
    return LQCD_ERR_NUMERIC;
  }
  if (!all_conv) {
    set_error("true residual above tol for at least one system after max_iter / refinement");
    return LQCD_ERR_NOT_CONVERGED;
  }
  return LQCD_OK;
}

}  // namespace

void timing_release() {
  std::lock_guard<std::mutex> lk(T().mu);
  for (auto& p : T().pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  T().pending.clear();
  for (hipEvent_t e : T().pool) (void)hipEventDestroy(e);
  T().pool.clear();
}

void solver_release() {
  timing_release();
  std::lock_guard<std::mutex> lk(G().mu);
  clear_graphs();
  if (G().pinned) (void)hipHostFree(G().pinned);
  G().pinned = nullptr;
  G().pinned_bytes = 0;
  if (G().cap) (void)hipStreamDestroy(G().cap);
  G().cap = nullptr;
}

}  // namespace lqcd

using namespace lqcd;

extern "C" {

void lqcd_solver_params_default(lqcd_solver_params* p) {
  if (!p) return;
  p->mass = 0.1;
  p->tol = 1e-10;
  p->max_iter = 10000;
  p->inner_prec = LQCD_F64;
  p->inner_fmt = LQCD_LINKS18;
  p->reliable_interval = 100;
  p->use_graph = 1;
  p->rhs_block = 0;
  p->poll_interval = 0;
  p->max_refine = 3;
  p->shift_window = 31;
  p->reliable_delta = 1e-3;
  p->mixed_switch = 1e-3;
  p->inner_tol_factor = 0.7;
}

size_t lqcd_solver_workspace_bytes(const lqcd_geom* g, const lqcd_solver_params* p,
                                   int32_t nshift, int32_t nrhs) {
  if (check_geom(g) || check_params(p) || check_nrhs(nrhs) || nshift < 1 || nshift > kMaxShift)
    return 0;
  return make_layout(make_kgeom(g), *p, nshift, nrhs).total;
}

int lqcd_cg(const lqcd_geom* g, const lqcd_solver_params* p, const void* U64, const void* Uinner,
            double sigma, const void* b, void* x, int32_t nrhs, lqcd_solve_stats* stats,
            void* ws, size_t ws_bytes, void* stream) {
  return solve(g, p, U64, Uinner, 1, &sigma, b, x, nrhs, true, stats, ws, ws_bytes, stream);
}

int lqcd_cg_multishift(const lqcd_geom* g, const lqcd_solver_params* p, const void* U64,
                       const void* Uinner, int32_t nshift, const double* sigma, const void* b,
                       void* x, int32_t nrhs, lqcd_solve_stats* stats, void* ws,
                       size_t ws_bytes, void* stream) {
  return solve(g, p, U64, Uinner, nshift, sigma, b, x, nrhs, false, stats, ws, ws_bytes,
               stream);
}

int lqcd_kernel_timing_enable(int32_t on) {
  clear_error();
  if (on != 0 && on != 1) {
    set_error("lqcd_kernel_timing_enable: on must be 0 or 1");
    return LQCD_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(T().mu);
  T().on = on == 1;
  if (on) {
    T().acc.clear();
    T().order.clear();
    for (auto& pe : T().pending) {  // unresolved launches of an earlier solve
      T().pool.push_back(pe.a);
      T().pool.push_back(pe.b);
    }
    T().pending.clear();
  }
  return LQCD_OK;
}

int lqcd_kernel_timing_get(int32_t index, char* name, size_t name_len, int64_t* launches,
                           double* total_ms) {
  clear_error();
  std::lock_guard<std::mutex> lk(T().mu);
  if (index < 0 || size_t(index) >= T().order.size()) {
    set_error("kernel timing index %d out of range (%zu classes)", index, T().order.size());
    return LQCD_ERR_INVALID_ARG;
  }
  if (!name || name_len == 0 || !launches || !total_ms) {
    set_error("kernel timing outputs must be non-null");
    return LQCD_ERR_INVALID_ARG;
  }
  const std::string& cls = T().order[index];
  std::snprintf(name, name_len, "%s", cls.c_str());
  *launches = T().acc[cls].first;
  *total_ms = T().acc[cls].second;
  return LQCD_OK;
}

int lqcd_finalize(void) {
  solver_release();
  dslash_clear_tuning();
  return LQCD_OK;
}

}  // extern "C"
