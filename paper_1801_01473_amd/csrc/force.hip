// Fermion force and rational pseudofermion action.
//
// The action of Eq. (1) with M^(-1/4) in rational form is
//   S = sum_j [ alpha_0 |phi_j|^2 + sum_i alpha_i Re <phi_j, X_ji> ],
//   X_ji = (A + sigma_i)^-1 phi_j,  A = m^2 + D_oe^dag D_oe  (D_eo = -D_oe^dag).
// Its variation is dS = -sum alpha_i <X, dA X> = -2 sum alpha_i Re <chi, dD_oe X>
// with chi = D_oe X, which, link by link, is dS = sum Re Tr[dU_mu(x) M_mu(x)] with
//   x odd : M_mu(x) = -sum alpha eta_mu(x) s_mu(x) X(x+mu) chi(x)^dag
//   x even: M_mu(x) = +sum alpha eta_mu(x) s_mu(x) chi(x+mu) X(x)^dag.
// Every link touches exactly one odd site as either its forward link (x odd)
// or the backward link of x+mu (x even), so one odd site y owns the eight
// links of its star and writes each of them once: no atomics.
//
// Work split: four lanes per odd site, lane mu owns the links (y, mu) and
// (y - mu, mu).  For each (pseudofermion, shift) pair the lane computes the
// direction-mu part of chi(y) = (D_oe X)(y) with its two links, the quad adds
// the four parts with two butterfly shuffles (same order in every lane), and
// each lane adds the two outer products into its two 3x3 accumulators.  chi is
// never written to memory.  At the end the lane projects U M to the traceless
// anti-Hermitian part (mode 0) or writes M^dag (mode 1, torch's gradient).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "common.h"
#include "solver.h"
#include "su3.h"
#include "tile.h"

namespace lqcd {

namespace {

constexpr int kForceBlock = 256;  // 64 odd sites x 4 directions
constexpr int kActionBlock = 256;
constexpr int kCombineBlock = 256;

struct Alphas {
  double a[kMaxShift];
};

// Block partials and the final sum of lqcd_action_noalloc live here instead of
// in a caller workspace: 1 MiB, i.e. ceil(Vh/256) + 32 doubles for any Vh up to
// 33.5 million, more than the largest lattice the library accepts.  Each device
// holds its own copy until the process ends.  Host code never passes this name
// to a kernel (on the host it is only a stand-in for the symbol): it uses the
// device address that hipGetSymbolAddress returns for the current device.
constexpr size_t kActionScratchDoubles = size_t(1) << 17;
static __device__ __align__(256) double scratch[kActionScratchDoubles];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxScratchDevices] = {};

// The value of lane (l ^ 1) (CTRL 0xB1: quad permutation 1,0,3,2) or of lane
// (l ^ 2) (CTRL 0x4E: 2,3,0,1) of the same quad, moved by DPP in the vector
// pipeline (no LDS round trip).
template <int CTRL>
__device__ __forceinline__ double dpp_quad(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Sum over the four lanes of a quad: v + v[l ^ 1], then + the partner pair's
// sum; every lane of the quad ends with the same bits.
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp_quad<0xB1>(v);
  v += dpp_quad<0x4E>(v);
  return v;
}

__global__ void __launch_bounds__(kForceBlock) k_force(const KGeom g,
                                                       const double2* __restrict__ U,
                                                       const double2* __restrict__ X, int npf,
                                                       int nshift, const Alphas al, int mode,
                                                       int accumulate, int ty, int tz,
                                                       double2* __restrict__ F) {
  // Every even X is read by its eight odd neighbours, for every pair, so the
  // sites sharing neighbours run close together and on one XCD (one L2):
  // consecutive blocks of an XCD take consecutive sites of a (y, z)-tiled
  // order with t inside the tile.
  const int lb = xcd_block(blockIdx.x, gridDim.x, 1);
  const int64_t tid = int64_t(lb) * blockDim.x + threadIdx.x;
  const int i = int(tid >> 2);
  const int mu = int(tid & 3);
  if (i >= g.Vh) return;  // whole quads leave together
  const int h = tiled_half_index(g, i, ty, tz);  // odd site
  const Site s = decode_site(g, h, 1);
  int fwd[4], bwd[4];
  neighbours(g, s, h, fwd, bwd);
  double eta[4];
  staggered_eta(s, eta);
  double sf = eta[mu], sb = eta[mu];  // eta_mu(y) s_mu(y), eta_mu(y-mu) s_mu(y-mu)
  if (mu == 3 && g.anti) {
    if (s.t == g.Lt - 1) sf = -sf;
    if (s.t == 0) sb = -sb;
  }
  const int hf = fwd[mu], hb = bwd[mu];
  const int64_t pstride = int64_t(4) * 9 * g.Vh;
  Su3<double> Uf, Ub;
  load_link<double, 9>(U + pstride + int64_t(mu) * 9 * g.Vh, h, g.Vh, Uf);  // (y, mu), y odd
  load_link<double, 9>(U + int64_t(mu) * 9 * g.Vh, hb, g.Vh, Ub);           // (y-mu, mu), even

  Su3<double> Mf, Mb;
#pragma unroll
  for (int e = 0; e < 9; ++e) Mf.e[e] = Mb.e[e] = mk<double>(0, 0);
  // The hop coefficients sf/2, sb/2 (a sign and a power of two, so exactly)
  // go into the links, which then give the direction-mu part of chi directly.
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    Uf.e[e] = cscale<double>(0.5 * sf, Uf.e[e]);
    Ub.e[e] = cscale<double>(0.5 * sb, Ub.e[e]);
  }

  const int64_t vs = int64_t(3) * g.Vh;
  for (int j = 0; j < npf; ++j) {
    for (int i = 0; i < nshift; ++i) {
      const double2* Xk = X + (int64_t(j) * nshift + i) * vs;
      cplx<double> xf[3], xb[3], y1[3], y2[3], chi[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        xf[c] = Xk[int64_t(c) * g.Vh + hf];
        xb[c] = Xk[int64_t(c) * g.Vh + hb];
      }
      // direction-mu part of chi(y) = 1/2 [sf U_mu(y) X(y+mu) - sb U_mu(y-mu)^dag X(y-mu)]
      mat_vec<double>(Uf, xf, y1);
      adj_mat_vec<double>(Ub, xb, y2);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        chi[c].x = quad_sum(y1[c].x - y2[c].x);
        chi[c].y = quad_sum(y1[c].y - y2[c].y);
      }
      // chi already carries the 1/2 of D_oe; the 1/2 of dD_oe and the factor 2 of
      // the variation cancel, so M takes alpha * eta * s with no further factor:
      //   M_mu(y)    += cf X(y+mu) chi(y)^dag,   cf = -alpha sf
      //   M_mu(y-mu) += cb chi(y) X(y-mu)^dag,   cb =  alpha sb
      // with the coefficients folded into chi once per pair.
      const double cf = -al.a[i] * sf;
      const double cb = al.a[i] * sb;
      cplx<double> cfc[3], cbc[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cfc[c] = mk<double>(cf * chi[c].x, -cf * chi[c].y);  // cf conj(chi)
        cbc[c] = cscale<double>(cb, chi[c]);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          cfma<double>(Mf.e[3 * a + b], xf[a], cfc[b]);
          cfmac<double>(Mb.e[3 * a + b], xb[b], cbc[a]);  // += cb chi[a] conj(xb[b])
        }
    }
  }
  // the unscaled links for the projection: U = (2 s) U', exactly
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    Uf.e[e] = cscale<double>(2.0 * sf, Uf.e[e]);
    Ub.e[e] = cscale<double>(2.0 * sb, Ub.e[e]);
  }

  // outputs: forward link at (parity 1, mu, h), backward link at (parity 0, mu, hb)
  for (int side = 0; side < 2; ++side) {
    const Su3<double>& M = side == 0 ? Mf : Mb;
    const Su3<double>& Ul = side == 0 ? Uf : Ub;
    double2* out = F + (side == 0 ? pstride : 0) + int64_t(mu) * 9 * g.Vh + (side == 0 ? h : hb);
    cplx<double> res[9];
    if (mode == 1) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) res[3 * a + b] = conj_of<double>(M.e[3 * b + a]);
    } else {
      cplx<double> W[9];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          cplx<double> w = cmul<double>(Ul.e[3 * a], M.e[b]);
          cfma<double>(w, Ul.e[3 * a + 1], M.e[3 + b]);
          cfma<double>(w, Ul.e[3 * a + 2], M.e[6 + b]);
          W[3 * a + b] = w;
        }
      // TA(W) = (W - W^dag)/2 - Tr(W - W^dag)/6; Tr(W - W^dag) = 2 i Im Tr W
      const double im_tr = (W[0].y + W[4].y + W[8].y) / 3.0;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          const cplx<double> w = W[3 * a + b], wt = W[3 * b + a];
          res[3 * a + b] = mk<double>(0.5 * (w.x - wt.x), 0.5 * (w.y + wt.y) - (a == b ? im_tr : 0.0));
        }
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      cplx<double> v = res[e];
      if (accumulate) {
        const double2 o = out[int64_t(e) * g.Vh];
        v.x += o.x;
        v.y += o.y;
      }
      out[int64_t(e) * g.Vh] = v;
    }
  }
}

// partials[blk] = sum over the block's even sites of
//   sum_j [alpha0 |phi_j|^2 + sum_i alpha_i Re <phi_j, X_ji>]
__global__ void __launch_bounds__(kActionBlock) k_action(int Vh, const double2* __restrict__ phi,
                                                         const double2* __restrict__ X, int npf,
                                                         int nshift, double alpha0,
                                                         const Alphas al,
                                                         double* __restrict__ part) {
  __shared__ double lds[kActionBlock / 64];
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (h < Vh) {
    const int64_t vs = int64_t(3) * Vh;
    for (int j = 0; j < npf; ++j) {
      double2 f[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        f[c] = phi[j * vs + int64_t(c) * Vh + h];
        s += alpha0 * (f[c].x * f[c].x + f[c].y * f[c].y);
      }
      for (int i = 0; i < nshift; ++i) {
        const double2* Xk = X + (int64_t(j) * nshift + i) * vs;
        double d = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double2 x = Xk[int64_t(c) * Vh + h];
          d += f[c].x * x.x + f[c].y * x.y;  // Re(conj(phi) X)
        }
        s += al.a[i] * d;
      }
    }
  }
  s = block_sum(s, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kActionBlock) k_sum(const double* __restrict__ part, int n,
                                                      double* __restrict__ out) {
  __shared__ double lds[kActionBlock / 64];
  double s = strided_sum(part, n);
  s = block_sum(s, lds);
  if (threadIdx.x == 0) *out = s;
}

// y_j = alpha0 b_j + sum_i alpha_i X_ji for every complex element e of the
// [3][Vh] even-site vectors (blockIdx.y = j).  The terms are added in a fixed
// order (alpha0 b first, then i = 0, 1, ...), so the result is reproducible.
// y may be b (each element is read before it is written), never X.
__global__ void __launch_bounds__(kCombineBlock) k_rational_combine(
    int64_t n, const double2* __restrict__ b, const double2* X, int nshift, double alpha0,
    Alphas al, double2* y) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int64_t j = blockIdx.y;
  const double2 bv = b[j * n + e];
  double re = alpha0 * bv.x, im = alpha0 * bv.y;
  const double2* xj = X + j * nshift * n + e;
  constexpr int kChunk = 8;  // loads issued together before their products
  for (int i0 = 0; i0 < nshift; i0 += kChunk) {
    double2 v[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u)
      if (i0 + u < nshift) v[u] = xj[int64_t(i0 + u) * n];
#pragma unroll
    for (int u = 0; u < kChunk; ++u)
      if (i0 + u < nshift) {
        re = fma(al.a[i0 + u], v[u].x, re);
        im = fma(al.a[i0 + u], v[u].y, im);
      }
  }
  y[j * n + e] = make_double2(re, im);
}

// Device address of the current device's copy of `scratch`, looked up once per
// device.  Returns NULL (error text set) if the device or the lookup fails.
double* action_scratch_ptr() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) {
    set_error("no usable current HIP device (device %d) for the action scratch array", dev);
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  return g_scratch_dev[dev];
}

int check_alpha(int32_t nshift, const double* alpha) {
  if (nshift < 1 || nshift > kMaxShift) {
    set_error("nshift = %d must be in [1, %d]", nshift, kMaxShift);
    return LQCD_ERR_INVALID_ARG;
  }
  if (!alpha) {
    set_error("alpha must be a host array of nshift doubles");
    return LQCD_ERR_INVALID_ARG;
  }
  for (int i = 0; i < nshift; ++i)
    if (!std::isfinite(alpha[i])) {
      set_error("alpha[%d] is not finite", i);
      return LQCD_ERR_INVALID_ARG;
    }
  return LQCD_OK;
}

}  // namespace

}  // namespace lqcd

using namespace lqcd;

extern "C" {

int lqcd_fermion_force(const lqcd_geom* g, const void* U64, int32_t npf, int32_t nshift,
                       const double* alpha, const void* X, int32_t mode, int32_t accumulate,
                       void* F, void* stream) {
  clear_error();
  int rc;
  if ((rc = check_geom(g)) || (rc = check_ptr(U64, "U64")) || (rc = check_ptr(X, "X")) ||
      (rc = check_ptr(F, "F")) || (rc = check_alpha(nshift, alpha)))
    return rc;
  if (npf < 1 || npf > 64) {
    set_error("npf = %d must be in [1, 64]", npf);
    return LQCD_ERR_INVALID_ARG;
  }
  if (mode != 0 && mode != 1) {
    set_error("mode must be 0 (projected) or 1 (raw), got %d", mode);
    return LQCD_ERR_INVALID_ARG;
  }
  if (accumulate != 0 && accumulate != 1) {
    set_error("accumulate must be 0 or 1");
    return LQCD_ERR_INVALID_ARG;
  }
  if (F == U64 || F == X) {
    set_error("F must not alias U64 or X");
    return LQCD_ERR_INVALID_ARG;
  }
  const KGeom k = make_kgeom(g);
  Alphas al{};
  for (int i = 0; i < nshift; ++i) al.a[i] = alpha[i];
  const int64_t threads = int64_t(4) * k.Vh;
  const unsigned grid = unsigned((threads + kForceBlock - 1) / kForceBlock);
  // small (y, z) tiles: a tile's t slice is a few dozen waves, so the +-t
  // neighbours of a site are loaded by waves at nearly the same pair (at 48^4
  // 6 x 6 tiles: 11.4 ms against 12.4 ms lexicographic, both XCD-contiguous)
  const int tz = small_tile(k.Lz), ty = small_tile(k.Ly) ? small_tile(k.Ly) : k.Ly;
  hipLaunchKernelGGL(k_force, dim3(grid), dim3(kForceBlock), 0, (hipStream_t)stream, k,
                     (const double2*)U64, (const double2*)X, npf, nshift, al, mode, accumulate,
                     ty, tz, (double2*)F);
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

size_t lqcd_action_workspace_bytes(const lqcd_geom* g) {
  if (check_geom(g)) return 0;
  const KGeom k = make_kgeom(g);
  return (size_t((k.Vh + kActionBlock - 1) / kActionBlock) + 32) * sizeof(double);
}

}  // extern "C"

namespace lqcd {
namespace {

int check_action_args(const lqcd_geom* g, int32_t npf, int32_t nshift, double alpha0,
                      const double* alpha, const void* phi, const void* X, const double* S) {
  int rc;
  if ((rc = check_geom(g)) || (rc = check_ptr(phi, "phi")) || (rc = check_ptr(X, "X")) ||
      (rc = check_alpha(nshift, alpha)))
    return rc;
  if (!S) {
    set_error("S must be a host pointer");
    return LQCD_ERR_INVALID_ARG;
  }
  if (npf < 1 || npf > 64) {
    set_error("npf = %d must be in [1, 64]", npf);
    return LQCD_ERR_INVALID_ARG;
  }
  if (!std::isfinite(alpha0)) {
    set_error("alpha0 is not finite");
    return LQCD_ERR_INVALID_ARG;
  }
  return LQCD_OK;
}

// The two reduction launches of the action into `part` (ceil(Vh/256) + 32
// doubles of device memory), then the result to the host.
int run_action(const lqcd_geom* g, int32_t npf, int32_t nshift, double alpha0,
               const double* alpha, const void* phi, const void* X, double* S, double* part,
               hipStream_t s) {
  const KGeom k = make_kgeom(g);
  Alphas al{};
  for (int i = 0; i < nshift; ++i) al.a[i] = alpha[i];
  const int nb = (k.Vh + kActionBlock - 1) / kActionBlock;
  double* out = part + nb + 16;
  hipLaunchKernelGGL(k_action, dim3(nb), dim3(kActionBlock), 0, s, k.Vh, (const double2*)phi,
                     (const double2*)X, npf, nshift, alpha0, al, part);
  LQCD_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kActionBlock), 0, s, part, nb, out);
  LQCD_LAUNCH_CHECK();
  LQCD_HIP_TRY(hipMemcpyAsync(S, out, sizeof(double), hipMemcpyDeviceToHost, s));
  LQCD_HIP_TRY(hipStreamSynchronize(s));
  return LQCD_OK;
}

}  // namespace
}  // namespace lqcd

extern "C" {

int lqcd_action(const lqcd_geom* g, int32_t npf, int32_t nshift, double alpha0,
                const double* alpha, const void* phi, const void* X, double* S, void* ws,
                size_t ws_bytes, void* stream) {
  clear_error();
  int rc;
  if ((rc = check_action_args(g, npf, nshift, alpha0, alpha, phi, X, S)) ||
      (rc = check_ptr(ws, "ws")))
    return rc;
  const size_t need = lqcd_action_workspace_bytes(g);
  if (ws_bytes < need) {
    set_error("action workspace of %zu bytes is too small: %zu needed", ws_bytes, need);
    return LQCD_ERR_WORKSPACE;
  }
  return run_action(g, npf, nshift, alpha0, alpha, phi, X, S, static_cast<double*>(ws),
                    (hipStream_t)stream);
}

int lqcd_action_noalloc(const lqcd_geom* g, int32_t npf, int32_t nshift, double alpha0,
                        const double* alpha, const void* phi, const void* X, double* S,
                        void* stream) {
  clear_error();
  int rc;
  if ((rc = check_action_args(g, npf, nshift, alpha0, alpha, phi, X, S))) return rc;
  const size_t need = lqcd_action_workspace_bytes(g);
  if (need > kActionScratchDoubles * sizeof(double)) {
    set_error("lattice needs %zu bytes of action scratch, above the fixed %zu-byte array", need,
              kActionScratchDoubles * sizeof(double));
    return LQCD_ERR_WORKSPACE;
  }
  double* part = action_scratch_ptr();
  if (!part) return LQCD_ERR_HIP;
  return run_action(g, npf, nshift, alpha0, alpha, phi, X, S, part, (hipStream_t)stream);
}

int lqcd_rational_combine(const lqcd_geom* g, int32_t nrhs, int32_t nshift, double alpha0,
                          const double* alpha, const void* b, const void* X, void* y,
                          void* stream) {
  clear_error();
  int rc;
  if ((rc = check_geom(g)) || (rc = check_ptr(b, "b")) || (rc = check_ptr(X, "X")) ||
      (rc = check_ptr(y, "y")) || (rc = check_alpha(nshift, alpha)))
    return rc;
  if (nrhs < 1 || nrhs > 64) {
    set_error("nrhs = %d must be in [1, 64]", nrhs);
    return LQCD_ERR_INVALID_ARG;
  }
  if (!std::isfinite(alpha0)) {
    set_error("alpha0 is not finite");
    return LQCD_ERR_INVALID_ARG;
  }
  const KGeom k = make_kgeom(g);
  const int64_t n = int64_t(3) * k.Vh;
  const char* xb = static_cast<const char*>(X);
  const char* yb = static_cast<const char*>(y);
  const int64_t xbytes = int64_t(nrhs) * nshift * n * int64_t(sizeof(double2));
  const int64_t ybytes = int64_t(nrhs) * n * int64_t(sizeof(double2));
  if (yb < xb + xbytes && xb < yb + ybytes) {
    set_error("y must not overlap X");
    return LQCD_ERR_INVALID_ARG;
  }
  Alphas al{};
  for (int i = 0; i < nshift; ++i) al.a[i] = alpha[i];
  const dim3 grid(unsigned((n + kCombineBlock - 1) / kCombineBlock), unsigned(nrhs));
  hipLaunchKernelGGL(k_rational_combine, grid, dim3(kCombineBlock), 0, (hipStream_t)stream, n,
                     (const double2*)b, (const double2*)X, nshift, alpha0, al, (double2*)y);
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

}  // extern "C"
