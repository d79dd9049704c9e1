// Gauge part of the molecular dynamics (Sec. 2 and Sec. 4.3): the tree-level
// Symanzik action (1x1 plaquettes and 1x2 rectangles of the links), its
// force, the momentum and link steps of the integrator and the kinetic
// energy.  FP64 throughout (the accept/reject test compares energies in
// double precision, Sec. 5.4).
//
// Links and momenta use the packed 18-real FP64 link layout
// [parity][mu][9][Vh] (complex), the layout of LQCD_LINKS18 links, so the
// fermion force can be added into the same array.  Gauge links carry no
// boundary sign or staggered phase (those belong to the fermion operator).
//
// Force convention (shared with the fermion force): with dS = sum Re Tr[dU M],
// F = TA(U M), TA(W) = (W - W^dag)/2 - Tr(W - W^dag)/6, so that dS/deps =
// sum Tr[T F] for U -> exp(eps T) U.  For S_g = beta sum_loops w (1 - Re Tr
// W / 3), M_mu(x) = -(beta / 3) A_mu(x) with A the weighted sum of the staples
// of the link (the product of the other links of each loop through it).  The
// MD equations U' = i H U, H' = -i F conserve H^2/2 + S.
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.h"
#include "tile.h"

namespace lqcd {

namespace {

constexpr int kGaugeBlock = 128;
constexpr int kMdBlock = 256;

struct M3 {
  double2 e[9];
};

__device__ __forceinline__ M3 m_zero() {
  M3 r;
#pragma unroll
  for (int i = 0; i < 9; ++i) r.e[i] = make_double2(0.0, 0.0);
  return r;
}

__device__ __forceinline__ M3 m_unit() {
  M3 r = m_zero();
  r.e[0].x = r.e[4].x = r.e[8].x = 1.0;
  return r;
}

// a b, a b^dag, a^dag b
__device__ __forceinline__ M3 m_mul(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 s = cmul<double>(a.e[3 * i], b.e[j]);
      cfma<double>(s, a.e[3 * i + 1], b.e[3 + j]);
      cfma<double>(s, a.e[3 * i + 2], b.e[6 + j]);
      r.e[3 * i + j] = s;
    }
  return r;
}

__device__ __forceinline__ M3 m_mul_dag(const M3& a, const M3& b) {
  M3 r;  // r_ij = sum_k a_ik conj(b_jk)
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 s = cmulc<double>(b.e[3 * j], a.e[3 * i]);
      cfmac<double>(s, b.e[3 * j + 1], a.e[3 * i + 1]);
      cfmac<double>(s, b.e[3 * j + 2], a.e[3 * i + 2]);
      r.e[3 * i + j] = s;
    }
  return r;
}

__device__ __forceinline__ M3 m_dag_mul(const M3& a, const M3& b) {
  M3 r;  // r_ij = sum_k conj(a_ki) b_kj
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 s = cmulc<double>(a.e[i], b.e[j]);
      cfmac<double>(s, a.e[3 + i], b.e[3 + j]);
      cfmac<double>(s, a.e[6 + i], b.e[6 + j]);
      r.e[3 * i + j] = s;
    }
  return r;
}

__device__ __forceinline__ void m_axpy(double w, const M3& a, M3& acc) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    acc.e[i].x = fma(w, a.e[i].x, acc.e[i].x);
    acc.e[i].y = fma(w, a.e[i].y, acc.e[i].y);
  }
}

__device__ __forceinline__ double re_tr(const M3& a) { return a.e[0].x + a.e[4].x + a.e[8].x; }

// Coordinates with periodic wrap (named fields: a direction index chosen at
// run time selects among them, so nothing is indexed dynamically), and the
// link U_mu at a site.
struct C4 {
  int x, y, z, t;
};

__device__ __forceinline__ int wrap(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

__device__ __forceinline__ C4 shift(const KGeom& g, C4 s, int mu, int d) {
  if (mu == 0)
    s.x = wrap(s.x + d, g.Lx);
  else if (mu == 1)
    s.y = wrap(s.y + d, g.Ly);
  else if (mu == 2)
    s.z = wrap(s.z + d, g.Lz);
  else
    s.t = wrap(s.t + d, g.Lt);
  return s;
}

__device__ __forceinline__ M3 link(const KGeom& g, const double2* __restrict__ U, const C4& s,
                                   int mu) {
  const int par = (s.x + s.y + s.z + s.t) & 1;
  const int h = (s.x >> 1) + g.Lxh * (s.y + g.Ly * (s.z + g.Lz * s.t));
  const double2* p = U + (int64_t(par) * 4 + mu) * 9 * int64_t(g.Vh) + h;
  M3 r;
#pragma unroll
  for (int e = 0; e < 9; ++e) r.e[e] = p[int64_t(e) * g.Vh];
  return r;
}

__device__ __forceinline__ C4 site_c4(const KGeom& g, int h, int par) {
  const Site s = decode_site(g, h, par);
  return C4{s.x, s.y, s.z, s.t};
}

// Weighted staple sum of the link U_mu(x): Tr[U_mu(x) A] runs over every
// plaquette (weight c0) and every 1x2 rectangle (weight c1) through the link,
// each as the loop that starts along the link.
// SEL picks the staple shapes (bits): 1 plaquettes, 2 / 4 2x1 with the link
// first / second (upper), 8 / 16 the same lower, 32 / 64 1x2 upper / lower.
// The force splits the shapes over three launches to bound the live matrices.
constexpr int kStaplePlaq = 1;
constexpr int kStaplePass1 = 1 | 2 | 4, kStaplePass2 = 8 | 16, kStaplePass3 = 32 | 64;

template <int SEL>
__device__ M3 staples(const KGeom& g, const double2* __restrict__ U, const C4& x, int mu,
                      double c0, double c1) {
  M3 A = m_zero();
#pragma unroll 1
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    const C4 xp = shift(g, x, mu, 1), xn = shift(g, x, nu, 1), xm = shift(g, x, nu, -1);
    const C4 xpm = shift(g, xp, nu, -1);
    // plaquettes: up U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag,
    //             down U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
    if (SEL & 1) {
      M3 t = m_mul_dag(link(g, U, xp, nu), link(g, U, xn, mu));
      t = m_mul_dag(t, link(g, U, x, nu));
      m_axpy(c0, t, A);
      t = m_dag_mul(link(g, U, xpm, nu), m_dag_mul(link(g, U, xm, mu), link(g, U, xm, nu)));
      m_axpy(c0, t, A);
    }
    if (c1 == 0.0 || (SEL & ~1) == 0) continue;
    const C4 xmu = shift(g, x, mu, -1);
    const C4 x2p = shift(g, xp, mu, 1);
    // 2 x 1, link first, up:
    //   U_mu(x+mu) U_nu(x+2mu) U_mu(x+mu+nu)^dag U_mu(x+nu)^dag U_nu(x)^dag
    if (SEL & 2) {
      M3 t = m_mul(link(g, U, xp, mu), link(g, U, x2p, nu));
      t = m_mul_dag(t, link(g, U, shift(g, xp, nu, 1), mu));
      t = m_mul_dag(t, link(g, U, xn, mu));
      t = m_mul_dag(t, link(g, U, x, nu));
      m_axpy(c1, t, A);
    }
    // 2 x 1, link second, up:
    //   U_nu(x+mu) U_mu(x+nu)^dag U_mu(x-mu+nu)^dag U_nu(x-mu)^dag U_mu(x-mu)
    if (SEL & 4) {
      M3 t = m_mul_dag(link(g, U, xp, nu), link(g, U, xn, mu));
      t = m_mul_dag(t, link(g, U, shift(g, xmu, nu, 1), mu));
      t = m_mul_dag(t, link(g, U, xmu, nu));
      t = m_mul(t, link(g, U, xmu, mu));
      m_axpy(c1, t, A);
    }
    // 2 x 1, link first, down:
    //   U_mu(x+mu) U_nu(x+2mu-nu)^dag U_mu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
    if (SEL & 8) {
      M3 t = m_mul_dag(link(g, U, xp, mu), link(g, U, shift(g, x2p, nu, -1), nu));
      t = m_mul_dag(t, link(g, U, xpm, mu));
      t = m_mul_dag(t, link(g, U, xm, mu));
      t = m_mul(t, link(g, U, xm, nu));
      m_axpy(c1, t, A);
    }
    // 2 x 1, link second, down:
    //   U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_mu(x-mu-nu)^dag U_nu(x-mu-nu) U_mu(x-mu)
    if (SEL & 16) {
      const C4 xmm = shift(g, xmu, nu, -1);
      M3 t = m_dag_mul(link(g, U, xpm, nu), m_dag_mul(link(g, U, xm, mu), m_unit()));
      t = m_mul_dag(t, link(g, U, xmm, mu));
      t = m_mul(t, link(g, U, xmm, nu));
      t = m_mul(t, link(g, U, xmu, mu));
      m_axpy(c1, t, A);
    }
    // 1 x 2, up: U_nu(x+mu) U_nu(x+mu+nu) U_mu(x+2nu)^dag U_nu(x+nu)^dag U_nu(x)^dag
    if (SEL & 32) {
      M3 t = m_mul(link(g, U, xp, nu), link(g, U, shift(g, xp, nu, 1), nu));
      t = m_mul_dag(t, link(g, U, shift(g, xn, nu, 1), mu));
      t = m_mul_dag(t, link(g, U, xn, nu));
      t = m_mul_dag(t, link(g, U, x, nu));
      m_axpy(c1, t, A);
    }
    // 1 x 2, down:
    //   U_nu(x+mu-nu)^dag U_nu(x+mu-2nu)^dag U_mu(x-2nu)^dag U_nu(x-2nu) U_nu(x-nu)
    if (SEL & 64) {
      const C4 xm2 = shift(g, xm, nu, -1);
      M3 t = m_dag_mul(link(g, U, xpm, nu), m_dag_mul(link(g, U, shift(g, xpm, nu, -1), nu),
                                                      m_unit()));
      t = m_mul_dag(t, link(g, U, xm2, mu));
      t = m_mul(t, link(g, U, xm2, nu));
      t = m_mul(t, link(g, U, xm, nu));
      m_axpy(c1, t, A);
    }
  }
  return A;
}

// TA(W) = (W - W^dag)/2 - Tr(W - W^dag)/6
__device__ __forceinline__ M3 traceless_antiherm(const M3& w) {
  M3 r;
  const double tr_im = (w.e[0].y + w.e[4].y + w.e[8].y) / 3.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double2 a = w.e[3 * i + j], b = w.e[3 * j + i];
      r.e[3 * i + j] = make_double2(0.5 * (a.x - b.x), 0.5 * (a.y + b.y) - (i == j ? tr_im : 0.0));
    }
  return r;
}

// One thread per link in the link_thread order (segment = mu; both parities
// of 64 half indices per workgroup, so each (parity, mu, element) plane is
// written coalesced); the blocks of one XCD take consecutive chunks, and the
// half index runs through z slabs of tz slices with t inside the slab
// (tz = 0: lexicographic), so the neighbour links one thread loads are the
// ones its neighbours load, while still in that XCD's L2.
template <int SEL>
__global__ void __launch_bounds__(kGaugeBlock) k_gauge_force(KGeom g, const double2* __restrict__ U,
                                                             double beta, double c0, double c1,
                                                             int accumulate, int tz, double2* F) {
  LinkThread lt;
  if (!link_thread(g, int64_t(xcd_block(blockIdx.x, gridDim.x, 1)) * blockDim.x + threadIdx.x,
                   lt))
    return;
  const int h = tiled_half_index(g, lt.i, g.Ly, tz);
  const int par = lt.par, mu = lt.seg;
  const int pm = par * 4 + mu;
  const C4 x = site_c4(g, h, par);
  const M3 A = staples<SEL>(g, U, x, mu, c0, c1);
  M3 W = m_mul(link(g, U, x, mu), A);
  const double s = -beta / 3.0;
#pragma unroll
  for (int e = 0; e < 9; ++e) W.e[e] = make_double2(s * W.e[e].x, s * W.e[e].y);
  const M3 f = traceless_antiherm(W);
  double2* out = F + int64_t(pm) * 9 * g.Vh + h;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    double2 v = f.e[e];
    if (accumulate) {
      const double2 o = out[int64_t(e) * g.Vh];
      v.x += o.x;
      v.y += o.y;
    }
    out[int64_t(e) * g.Vh] = v;
  }
}

// ---------------------------------------------------------------- staple fields
// The force through staple fields, one unordered direction pair {mu, nu} at a
// time.  For a link direction a and another direction b, with the plaquette
// staples of the link (x, a)
//   P+_ab(x) = U_b(x+a) U_a(x+b)^dag U_b(x)^dag,
//   P-_ab(x) = U_b(x+a-b)^dag U_a(x-b)^dag U_b(x-b),
// each 2x1 / 1x2 rectangle staple of (x, a) is two products of these fields
// and single links (inserting U U^dag = 1 along the loop):
//   2x1, link first, up:   U_a(x+a) P+_ab(x+a) P+_ab(x)
//   2x1, link second, up:  P+_ab(x) U_b(x) P-_ba(x)
//   2x1, link first, down: U_a(x+a) P-_ab(x+a) P-_ab(x)
//   2x1, link second, down: P-_ab(x) U_b(x-b)^dag P-_ba(x-b)^dag
//   1x2, up:               U_b(x+a) P+_ab(x+b) U_b(x)^dag
//   1x2, down:             U_b(x+a-b)^dag P-_ab(x-b) U_b(x-b)
// Pass 1 stores P+_mu,nu, P-_mu,nu, P+_nu,mu, P-_nu,mu for every site (fields
// 0..3, each packed like one direction of the links: [parity][9][Vh]); pass 2
// forms, for the links of both directions, A_ab = c0 (P+ + P-) + c1 (the six
// rectangles) and adds -(beta/3) TA(U_a A_ab) to F_a.  Per link that is about
// 51 SU(3) products over the six pairs, against 85 for the direct sum.

__device__ __forceinline__ M3 sfield(const KGeom& g, const double2* __restrict__ P, int f,
                                     const C4& s) {
  const int par = (s.x + s.y + s.z + s.t) & 1;
  const int h = (s.x >> 1) + g.Lxh * (s.y + g.Ly * (s.z + g.Lz * s.t));
  const double2* p = P + (int64_t(f) * 2 + par) * 9 * int64_t(g.Vh) + h;
  M3 r;
#pragma unroll
  for (int e = 0; e < 9; ++e) r.e[e] = p[int64_t(e) * g.Vh];
  return r;
}

// pass 1: one thread per site (the link_thread order with one segment; sites
// in the z-slab order of k_gauge_force, blocks XCD-contiguous)
__global__ void __launch_bounds__(kGaugeBlock) k_staple_fields(KGeom g,
                                                               const double2* __restrict__ U,
                                                               int mu, int nu, int tz,
                                                               double2* P) {
  LinkThread lt;
  if (!link_thread(g, int64_t(xcd_block(blockIdx.x, gridDim.x, 1)) * blockDim.x + threadIdx.x,
                   lt))
    return;
  const int par = lt.par, h = tiled_half_index(g, lt.i, g.Ly, tz);
  const C4 x = site_c4(g, h, par);
#pragma unroll 1
  for (int f = 0; f < 4; ++f) {
    const int a = f < 2 ? mu : nu, b = f < 2 ? nu : mu;
    M3 t;
    if ((f & 1) == 0) {  // P+_ab(x) = U_b(x+a) U_a(x+b)^dag U_b(x)^dag
      t = m_mul_dag(link(g, U, shift(g, x, a, 1), b), link(g, U, shift(g, x, b, 1), a));
      t = m_mul_dag(t, link(g, U, x, b));
    } else {  // P-_ab(x) = U_b(x+a-b)^dag U_a(x-b)^dag U_b(x-b)
      const C4 xm = shift(g, x, b, -1);
      t = m_dag_mul(link(g, U, shift(g, xm, a, 1), b),
                    m_dag_mul(link(g, U, xm, a), link(g, U, xm, b)));
    }
    double2* out = P + (int64_t(f) * 2 + par) * 9 * int64_t(g.Vh) + h;
#pragma unroll
    for (int e = 0; e < 9; ++e) out[int64_t(e) * g.Vh] = t.e[e];
  }
}

// pass 2: one thread per link of the two directions (the link_thread order,
// segment = side; side 0: a = mu, side 1: a = nu; sites in the z-slab order,
// blocks XCD-contiguous).  first_mask bit side: write F_a instead of adding
// to it.
__global__ void __launch_bounds__(kGaugeBlock) k_force_pair(KGeom g, const double2* __restrict__ U,
                                                            const double2* __restrict__ P,
                                                            int mu, int nu, double beta,
                                                            double c0, double c1, int first_mask,
                                                            int tz, double2* F) {
  LinkThread lt;
  if (!link_thread(g, int64_t(xcd_block(blockIdx.x, gridDim.x, 1)) * blockDim.x + threadIdx.x,
                   lt))
    return;
  const int h = tiled_half_index(g, lt.i, g.Ly, tz);
  const int side = lt.seg, par = lt.par;
  const int a = side ? nu : mu, b = side ? mu : nu;
  const int fp = side ? 2 : 0, fm = side ? 3 : 1, fmo = side ? 1 : 3;  // P+_ab, P-_ab, P-_ba
  const C4 x = site_c4(g, h, par);
  const C4 xa = shift(g, x, a, 1), xb = shift(g, x, b, 1), xmb = shift(g, x, b, -1);
  // Terms in an order that retires each field soon after its last use; the
  // links and fields used twice are loaded again (cache hits) rather than
  // held.  (Scheduling barriers between the terms halve the registers, 184
  // against 256 + 106 AGPRs, but serialise the terms' loads: 36.1 against
  // 33.2 ms at 48^4, so the compiler's hoisting is kept.)
  M3 A = m_zero();
  {
    const M3 pp = sfield(g, P, fp, x);
    m_axpy(c0, pp, A);
    if (c1 != 0.0) {
      m_axpy(c1, m_mul(m_mul(link(g, U, xa, a), sfield(g, P, fp, xa)), pp), A);
      m_axpy(c1, m_mul(m_mul(pp, link(g, U, x, b)), sfield(g, P, fmo, x)), A);
    }
  }
  {
    const M3 pm = sfield(g, P, fm, x);
    m_axpy(c0, pm, A);
    if (c1 != 0.0) {
      m_axpy(c1, m_mul(m_mul(link(g, U, xa, a), sfield(g, P, fm, xa)), pm), A);
      m_axpy(c1, m_mul_dag(m_mul_dag(pm, link(g, U, xmb, b)), sfield(g, P, fmo, xmb)), A);
    }
  }
  if (c1 != 0.0) {
    m_axpy(c1, m_mul_dag(m_mul(link(g, U, xa, b), sfield(g, P, fp, xb)), link(g, U, x, b)), A);
    m_axpy(c1,
           m_mul(m_dag_mul(link(g, U, shift(g, xa, b, -1), b), sfield(g, P, fm, xmb)),
                 link(g, U, xmb, b)),
           A);
  }
  M3 W = m_mul(link(g, U, x, a), A);
  const double s = -beta / 3.0;
#pragma unroll
  for (int e = 0; e < 9; ++e) W.e[e] = make_double2(s * W.e[e].x, s * W.e[e].y);
  const M3 f = traceless_antiherm(W);
  double2* out = F + (int64_t(par) * 4 + a) * 9 * g.Vh + h;
  const bool first = (first_mask >> side) & 1;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    double2 v = f.e[e];
    if (!first) {
      const double2 o = out[int64_t(e) * g.Vh];
      v.x += o.x;
      v.y += o.y;
    }
    out[int64_t(e) * g.Vh] = v;
  }
}

// Sum over the loops whose first corner is the thread's site of
// w (1 - Re Tr W / 3): plaquettes mu < nu, 2 x 1 rectangles for every mu != nu.
__global__ void __launch_bounds__(kGaugeBlock) k_gauge_action(KGeom g, const double2* __restrict__ U,
                                                              double c0, double c1,
                                                              double* __restrict__ part) {
  __shared__ double lds[kGaugeBlock / 64];
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (idx < int64_t(2) * g.Vh) {
    const int par = int(idx / g.Vh), h = int(idx % g.Vh);
    const C4 x = site_c4(g, h, par);
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
      const C4 xp = shift(g, x, mu, 1);
#pragma unroll 1
      for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        const C4 xn = shift(g, x, nu, 1);
        if (mu < nu) {  // U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
          M3 t = m_mul(link(g, U, x, mu), link(g, U, xp, nu));
          t = m_mul_dag(t, link(g, U, xn, mu));
          t = m_mul_dag(t, link(g, U, x, nu));
          s += c0 * (1.0 - re_tr(t) / 3.0);
        }
        if (c1 != 0.0) {
          // U_mu(x) U_mu(x+mu) U_nu(x+2mu) U_mu(x+mu+nu)^dag U_mu(x+nu)^dag U_nu(x)^dag
          M3 t = m_mul(link(g, U, x, mu), link(g, U, xp, mu));
          t = m_mul(t, link(g, U, shift(g, xp, mu, 1), nu));
          t = m_mul_dag(t, link(g, U, shift(g, xp, nu, 1), mu));
          t = m_mul_dag(t, link(g, U, xn, mu));
          t = m_mul_dag(t, link(g, U, x, nu));
          s += c1 * (1.0 - re_tr(t) / 3.0);
        }
      }
    }
  }
  s = block_sum(s, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kMdBlock) k_reduce_one(const double* __restrict__ part, int n,
                                                          double scale, double* __restrict__ out) {
  __shared__ double lds[kMdBlock / 64];
  double s = strided_sum(part, n);
  s = block_sum(s, lds);
  if (threadIdx.x == 0) *out = scale * s;
}

// H <- H - i eps F, element-wise over the packed arrays
__global__ void __launch_bounds__(kMdBlock) k_md_momenta(int64_t n, const double2* __restrict__ F,
                                                         double eps, double2* __restrict__ H) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 f = F[i];
  double2 h = H[i];
  h.x = fma(eps, f.y, h.x);
  h.y = fma(-eps, f.x, h.y);
  H[i] = h;
}

// exp(X) for the anti-Hermitian X = i eps H: scaling and squaring, with a
// Taylor polynomial of degree 12 on ||Y|| <= 1/4 (remainder < 3e-18).
__device__ M3 expm_su3(const M3& X) {
  double nrm2 = 0.0;
#pragma unroll
  for (int e = 0; e < 9; ++e) nrm2 += X.e[e].x * X.e[e].x + X.e[e].y * X.e[e].y;
  double nrm = sqrt(nrm2);
  int sq = 0;
  while (nrm > 0.25 && sq < 40) {
    nrm *= 0.5;
    ++sq;
  }
  const double sc = ldexp(1.0, -sq);
  M3 Y;
#pragma unroll
  for (int e = 0; e < 9; ++e) Y.e[e] = make_double2(sc * X.e[e].x, sc * X.e[e].y);
  // Horner: E = I + Y/1 (I + Y/2 (I + ... (I + Y/12)))
  M3 E = m_unit();
#pragma unroll 1
  for (int k = 12; k >= 1; --k) {
    M3 t = m_mul(Y, E);
    const double inv = 1.0 / k;
#pragma unroll
    for (int e = 0; e < 9; ++e) t.e[e] = make_double2(inv * t.e[e].x, inv * t.e[e].y);
    t.e[0].x += 1.0;
    t.e[4].x += 1.0;
    t.e[8].x += 1.0;
    E = t;
  }
#pragma unroll 1
  for (int k = 0; k < sq; ++k) E = m_mul(E, E);
  return E;
}

// Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1): the nearest
// special-unitary matrix up to rounding, applied after each link update so
// that the links stay in SU(3) over many steps.
__device__ M3 reunitarize(M3 u) {
  double n0 = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) n0 += u.e[j].x * u.e[j].x + u.e[j].y * u.e[j].y;
  n0 = 1.0 / sqrt(n0);
#pragma unroll
  for (int j = 0; j < 3; ++j) u.e[j] = make_double2(n0 * u.e[j].x, n0 * u.e[j].y);
  double2 d = make_double2(0.0, 0.0);  // <row0, row1> = sum_j conj(row0_j) row1_j
#pragma unroll
  for (int j = 0; j < 3; ++j) cfmac<double>(d, u.e[j], u.e[3 + j]);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double2 p = cmul<double>(d, u.e[j]);
    u.e[3 + j].x -= p.x;
    u.e[3 + j].y -= p.y;
  }
  double n1 = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) n1 += u.e[3 + j].x * u.e[3 + j].x + u.e[3 + j].y * u.e[3 + j].y;
  n1 = 1.0 / sqrt(n1);
#pragma unroll
  for (int j = 0; j < 3; ++j) u.e[3 + j] = make_double2(n1 * u.e[3 + j].x, n1 * u.e[3 + j].y);
  // row2 = conj(row0 x row1)
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int a = (j + 1) % 3, b = (j + 2) % 3;
    const double2 p = cmul<double>(u.e[a], u.e[3 + b]);
    const double2 q = cmul<double>(u.e[b], u.e[3 + a]);
    u.e[6 + j] = make_double2(p.x - q.x, -(p.y - q.y));
  }
  return u;
}

// U <- exp(i eps H) U, one thread per link
__global__ void __launch_bounds__(kGaugeBlock) k_md_links(KGeom g, const double2* __restrict__ H,
                                                          double eps, double2* __restrict__ U) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(8) * g.Vh) return;
  const int h = int(idx % g.Vh);
  const int64_t base = (idx / g.Vh) * 9 * int64_t(g.Vh) + h;
  M3 X, u;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    const double2 v = H[base + int64_t(e) * g.Vh];
    X.e[e] = make_double2(-eps * v.y, eps * v.x);  // i eps H
    u.e[e] = U[base + int64_t(e) * g.Vh];
  }
  const M3 r = reunitarize(m_mul(expm_su3(X), u));
#pragma unroll
  for (int e = 0; e < 9; ++e) U[base + int64_t(e) * g.Vh] = r.e[e];
}

// per link Tr H^2 = sum_ab Re(H_ab H_ba)
__global__ void __launch_bounds__(kGaugeBlock) k_kinetic(KGeom g, const double2* __restrict__ H,
                                                         double* __restrict__ part) {
  __shared__ double lds[kGaugeBlock / 64];
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (idx < int64_t(8) * g.Vh) {
    const int h = int(idx % g.Vh);
    const int64_t base = (idx / g.Vh) * 9 * int64_t(g.Vh) + h;
    M3 m;
#pragma unroll
    for (int e = 0; e < 9; ++e) m.e[e] = H[base + int64_t(e) * g.Vh];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const double2 p = cmul<double>(m.e[3 * a + b], m.e[3 * b + a]);
        s += p.x;
      }
  }
  s = block_sum(s, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// U_out = exp(i theta) U_in per link, theta natural [4][V] (lex = 2 h + bit)
__global__ void __launch_bounds__(kMdBlock) k_u1_phases(KGeom g, const double2* __restrict__ U,
                                                        const double* __restrict__ theta,
                                                        double2* __restrict__ out) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(8) * g.Vh) return;
  const int h = int(idx % g.Vh);
  const int pm = int(idx / g.Vh);
  const int par = pm >> 2, mu = pm & 3;
  const Site s = decode_site(g, h, par);
  const int64_t lex = int64_t(s.x) + int64_t(g.Lx) * (s.y + int64_t(g.Ly) * (s.z + int64_t(g.Lz) * s.t));
  const int64_t V = int64_t(2) * g.Vh;
  double sn, cs;
  sincos(theta[mu * V + lex], &sn, &cs);
  const double2 u = make_double2(cs, sn);
  const int64_t base = int64_t(pm) * 9 * g.Vh + h;
#pragma unroll
  for (int e = 0; e < 9; ++e) out[base + int64_t(e) * g.Vh] = cmul<double>(u, U[base + int64_t(e) * g.Vh]);
}

// ---- stout smearing (Sec. 2: the Dirac operator uses k-times stout-smeared
// links) and the chain rule of the force through one smearing level.
// U' = exp(X) U, X = TA(Omega), Omega = rho A^dag U^dag = rho (U A)^dag, A the
// plaquette staple sum of the link (so X = -rho TA(U A)).

__device__ __forceinline__ M3 m_dag(const M3& a) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[3 * i + j] = make_double2(a.e[3 * j + i].x, -a.e[3 * j + i].y);
  return r;
}

__device__ __forceinline__ M3 m_scale(double s, M3 a) {
#pragma unroll
  for (int e = 0; e < 9; ++e) a.e[e] = make_double2(s * a.e[e].x, s * a.e[e].y);
  return a;
}

__device__ __forceinline__ M3 m_add(M3 a, const M3& b) {
#pragma unroll
  for (int e = 0; e < 9; ++e) a.e[e] = make_double2(a.e[e].x + b.e[e].x, a.e[e].y + b.e[e].y);
  return a;
}

__device__ __forceinline__ void stout_x(const KGeom& g, const double2* __restrict__ U, const C4& x,
                                        int mu, double rho, M3& A, M3& u, M3& X) {
  A = staples<kStaplePlaq>(g, U, x, mu, 1.0, 0.0);
  u = link(g, U, x, mu);
  X = m_scale(-rho, traceless_antiherm(m_mul(u, A)));
}

// One thread per link, in the thread and site order of k_gauge_force.
__global__ void __launch_bounds__(kGaugeBlock) k_stout_smear(KGeom g, const double2* __restrict__ U,
                                                             double rho, int tz,
                                                             double2* __restrict__ out) {
  LinkThread lt;
  if (!link_thread(g, int64_t(xcd_block(blockIdx.x, gridDim.x, 1)) * blockDim.x + threadIdx.x,
                   lt))
    return;
  const int h = tiled_half_index(g, lt.i, g.Ly, tz);
  const int pm = lt.par * 4 + lt.seg;
  const C4 x = site_c4(g, h, pm >> 2);
  M3 A, u, X;
  stout_x(g, U, x, pm & 3, rho, A, u, X);
  const M3 r = m_mul(expm_su3(X), u);
  double2* o = out + int64_t(pm) * 9 * g.Vh + h;
#pragma unroll
  for (int e = 0; e < 9; ++e) o[int64_t(e) * g.Vh] = r.e[e];
}

// (exp(X), L(X, B)) with L(X, B) = sum_k 1/k! sum_j X^j B X^(k-1-j), the
// top-right block of exp([[X, B], [0, X]]): scaling and squaring of the block
// matrix, (E, G) -> (E E, E G + G E), degree-12 Taylor on ||X|| <= 1/4.
__device__ void expm_frechet(const M3& X, const M3& B, M3& E, M3& G) {
  double nrm2 = 0.0;
#pragma unroll
  for (int e = 0; e < 9; ++e) nrm2 += X.e[e].x * X.e[e].x + X.e[e].y * X.e[e].y;
  double nrm = sqrt(nrm2);
  int sq = 0;
  while (nrm > 0.25 && sq < 40) {
    nrm *= 0.5;
    ++sq;
  }
  const double sc = ldexp(1.0, -sq);
  const M3 Xs = m_scale(sc, X), Bs = m_scale(sc, B);
  E = m_unit();
  G = m_zero();
  M3 P = m_unit();  // Xs^k
  M3 D = Bs;        // D_k, k = 1
  double f = 1.0;   // 1/k!
#pragma unroll 1
  for (int k = 1; k <= 12; ++k) {
    f /= k;
    P = m_mul(Xs, P);
    E = m_add(E, m_scale(f, P));
    G = m_add(G, m_scale(f, D));
    D = m_add(m_mul(Xs, D), m_mul(Bs, P));  // D_{k+1} = X D_k + B X^k
  }
#pragma unroll 1
  for (int k = 0; k < sq; ++k) {
    const M3 G2 = m_add(m_mul(E, G), m_mul(G, E));
    E = m_mul(E, E);
    G = G2;
  }
}

// Per link, from the raw gradient G' = M'^dag with respect to the smeared
// link: K = rho Lam^dag U and the local part Mloc = M' E + rho A Lam^dag of
// M, Lam = TA(L(X, U M')).
__global__ void __launch_bounds__(kGaugeBlock) k_stout_lambda(KGeom g, const double2* __restrict__ U,
                                                              double rho, int tz,
                                                              const double2* __restrict__ Gp,
                                                              double2* __restrict__ K,
                                                              double2* __restrict__ Mloc) {
  LinkThread lt;
  if (!link_thread(g, int64_t(xcd_block(blockIdx.x, gridDim.x, 1)) * blockDim.x + threadIdx.x,
                   lt))
    return;
  const int h = tiled_half_index(g, lt.i, g.Ly, tz);
  const int pm = lt.par * 4 + lt.seg;
  const C4 x = site_c4(g, h, pm >> 2);
  M3 A, u, X;
  stout_x(g, U, x, pm & 3, rho, A, u, X);
  const int64_t base = int64_t(pm) * 9 * g.Vh + h;
  M3 gp;
#pragma unroll
  for (int e = 0; e < 9; ++e) gp.e[e] = Gp[base + int64_t(e) * g.Vh];
  const M3 Mp = m_dag(gp);
  M3 E, Gm;
  expm_frechet(X, m_mul(u, Mp), E, Gm);
  const M3 lam_dag = m_dag(traceless_antiherm(Gm));
  const M3 k = m_scale(rho, m_mul(lam_dag, u));
  const M3 ml = m_add(m_mul(Mp, E), m_scale(rho, m_mul(A, lam_dag)));
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    K[base + int64_t(e) * g.Vh] = k.e[e];
    Mloc[base + int64_t(e) * g.Vh] = ml.e[e];
  }
}

// M of link (y, a) = Mloc + the terms of Re Tr[dA_mu(x) K_mu(x)] in which the
// link appears, for every other direction m:
//   U_m(y-m+a)^dag U_a(y-m)^dag K_m(y-m)        (first link of an upper staple)
//   (K_m(y) U_a(y+m) U_m(y+a)^dag)^dag           (last link of an upper staple)
//   (U_m(y-m)^dag U_a(y-m) K_m(y-m+a))^dag       (first link of a lower staple)
//   K_m(y+a) U_a(y+m)^dag U_m(y)^dag             (last link of a lower staple)
//   (U_m(y-m)^dag K_a(y-m) U_m(y-m+a))^dag       (middle of an upper staple)
//   (U_m(y) K_a(y+m) U_m(y+a)^dag)^dag           (middle of a lower staple)
// Output: mode 0 F = TA(U M), mode 1 the raw gradient M^dag.
__global__ void __launch_bounds__(kGaugeBlock) k_stout_gather(KGeom g, const double2* __restrict__ U,
                                                              const double2* __restrict__ K,
                                                              const double2* __restrict__ Mloc,
                                                              int mode, int tz,
                                                              double2* __restrict__ out) {
  LinkThread lt;
  if (!link_thread(g, int64_t(xcd_block(blockIdx.x, gridDim.x, 1)) * blockDim.x + threadIdx.x,
                   lt))
    return;
  const int h = tiled_half_index(g, lt.i, g.Ly, tz);
  const int pm = lt.par * 4 + lt.seg;
  const int a = pm & 3;
  const C4 y = site_c4(g, h, pm >> 2);
  const int64_t base = int64_t(pm) * 9 * g.Vh + h;
  M3 M;
#pragma unroll
  for (int e = 0; e < 9; ++e) M.e[e] = Mloc[base + int64_t(e) * g.Vh];
#pragma unroll 1
  for (int m = 0; m < 4; ++m) {
    if (m == a) continue;
    const C4 ym = shift(g, y, m, -1), yp = shift(g, y, m, 1), ya = shift(g, y, a, 1);
    const C4 yma = shift(g, ym, a, 1);
    M = m_add(M, m_mul(m_dag_mul(link(g, U, yma, m), m_dag(link(g, U, ym, a))), link(g, K, ym, m)));
    M = m_add(M, m_dag(m_mul_dag(m_mul(link(g, K, y, m), link(g, U, yp, a)), link(g, U, ya, m))));
    M = m_add(M, m_dag(m_mul(m_dag_mul(link(g, U, ym, m), link(g, U, ym, a)), link(g, K, yma, m))));
    M = m_add(M, m_mul_dag(m_mul_dag(link(g, K, ya, m), link(g, U, yp, a)), link(g, U, y, m)));
    M = m_add(M, m_dag(m_mul(m_dag_mul(link(g, U, ym, m), link(g, K, ym, a)), link(g, U, yma, m))));
    M = m_add(M, m_dag(m_mul_dag(m_mul(link(g, U, y, m), link(g, K, yp, a)), link(g, U, ya, m))));
  }
  const M3 r = mode == 0 ? traceless_antiherm(m_mul(link(g, U, y, a), M)) : m_dag(M);
#pragma unroll
  for (int e = 0; e < 9; ++e) out[base + int64_t(e) * g.Vh] = r.e[e];
}

int check_c1(double beta, double c1) {
  if (!std::isfinite(beta) || !std::isfinite(c1)) {
    set_error("beta and c1 must be finite");
    return LQCD_ERR_INVALID_ARG;
  }
  return LQCD_OK;
}

int reduce_to_host(const double* part, int nb, double scale, double* out_dev, double* host,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_one, dim3(1), dim3(kMdBlock), 0, s, part, nb, scale, out_dev);
  LQCD_LAUNCH_CHECK();
  LQCD_HIP_TRY(hipMemcpyAsync(host, out_dev, sizeof(double), hipMemcpyDeviceToHost, s));
  LQCD_HIP_TRY(hipStreamSynchronize(s));
  return LQCD_OK;
}

}  // namespace

}  // namespace lqcd

using namespace lqcd;

extern "C" {

int lqcd_apply_u1_phases(const lqcd_geom* g, const void* U64, const double* theta, void* out,
                         void* stream) {
  clear_error();
  int rc;
  if ((rc = check_geom(g)) || (rc = check_ptr(U64, "U64")) || (rc = check_ptr(out, "out")))
    return rc;
  if (!theta || (reinterpret_cast<uintptr_t>(theta) & 7)) {
    set_error("theta must be an 8-byte aligned device array of 4 V doubles");
    return LQCD_ERR_INVALID_ARG;
  }
  const KGeom k = make_kgeom(g);
  const int64_t n = int64_t(8) * k.Vh;
  hipLaunchKernelGGL(k_u1_phases, dim3(unsigned((n + kMdBlock - 1) / kMdBlock)), dim3(kMdBlock),
                     0, (hipStream_t)stream, k, (const double2*)U64, theta, (double2*)out);
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

int lqcd_stout_smear(const lqcd_geom* g, const void* U64, double rho, void* out, void* stream) {
  clear_error();
  int rc;
  if ((rc = check_geom(g)) || (rc = check_ptr(U64, "U64")) || (rc = check_ptr(out, "out")))
    return rc;
  if (!std::isfinite(rho)) {
    set_error("rho must be finite");
    return LQCD_ERR_INVALID_ARG;
  }
  if (out == U64) {
    set_error("out must not alias U64 (every link reads its neighbours)");
    return LQCD_ERR_INVALID_ARG;
  }
  const KGeom k = make_kgeom(g);
  const int64_t n = 4 * link_threads_per_segment(k.Vh);
  hipLaunchKernelGGL(k_stout_smear, dim3(unsigned(n / kGaugeBlock)),
                     dim3(kGaugeBlock), 0, (hipStream_t)stream, k, (const double2*)U64, rho,
                     slab_tile(k.Lz), (double2*)out);
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

size_t lqcd_stout_workspace_bytes(const lqcd_geom* g) {
  if (check_geom(g)) return 0;
  const KGeom k = make_kgeom(g);
  return size_t(2) * 8 * 9 * size_t(k.Vh) * sizeof(double2);
}

int lqcd_stout_force(const lqcd_geom* g, const void* U64, double rho, const void* G_smeared,
                     int32_t mode, void* out, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  int rc;
  if ((rc = check_geom(g)) || (rc = check_ptr(U64, "U64")) ||
      (rc = check_ptr(G_smeared, "G_smeared")) || (rc = check_ptr(out, "out")) ||
      (rc = check_ptr(ws, "ws")))
    return rc;
  if (!std::isfinite(rho)) {
    set_error("rho must be finite");
    return LQCD_ERR_INVALID_ARG;
  }
  if (mode != 0 && mode != 1) {
    set_error("mode must be 0 (projected) or 1 (raw), got %d", mode);
    return LQCD_ERR_INVALID_ARG;
  }
  if (ws_bytes < lqcd_stout_workspace_bytes(g)) {
    set_error("stout workspace of %zu bytes is too small: %zu needed", ws_bytes,
              lqcd_stout_workspace_bytes(g));
    return LQCD_ERR_WORKSPACE;
  }
  if (out == U64 || out == G_smeared) {
    set_error("out must not alias U64 or G_smeared");
    return LQCD_ERR_INVALID_ARG;
  }
  const KGeom k = make_kgeom(g);
  const int64_t n = int64_t(8) * k.Vh;
  double2* K = static_cast<double2*>(ws);
  double2* Mloc = K + n * 9;
  const hipStream_t s = (hipStream_t)stream;
  const dim3 grid(unsigned(4 * link_threads_per_segment(k.Vh) / kGaugeBlock));
  const int tz = slab_tile(k.Lz);
  hipLaunchKernelGGL(k_stout_lambda, grid, dim3(kGaugeBlock), 0, s, k, (const double2*)U64, rho,
                     tz, (const double2*)G_smeared, K, Mloc);
  LQCD_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_stout_gather, grid, dim3(kGaugeBlock), 0, s, k, (const double2*)U64,
                     (const double2*)K, (const double2*)Mloc, mode, tz, (double2*)out);
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

size_t lqcd_gauge_workspace_bytes(const lqcd_geom* g) {
  if (check_geom(g)) return 0;
  const KGeom k = make_kgeom(g);
  return (size_t((int64_t(8) * k.Vh + kGaugeBlock - 1) / kGaugeBlock) + 32) * sizeof(double);
}

int lqcd_gauge_action(const lqcd_geom* g, const void* U64, double beta, double c1, double* S,
                      void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  int rc;
  if ((rc = check_geom(g)) || (rc = check_ptr(U64, "U64")) || (rc = check_ptr(ws, "ws")) ||
      (rc = check_c1(beta, c1)))
    return rc;
  if (!S) {
    set_error("S must be a host pointer");
    return LQCD_ERR_INVALID_ARG;
  }
  if (ws_bytes < lqcd_gauge_workspace_bytes(g)) {
    set_error("gauge workspace of %zu bytes is too small: %zu needed", ws_bytes,
              lqcd_gauge_workspace_bytes(g));
    return LQCD_ERR_WORKSPACE;
  }
  const KGeom k = make_kgeom(g);
  const int nb = int((int64_t(2) * k.Vh + kGaugeBlock - 1) / kGaugeBlock);
  double* part = static_cast<double*>(ws);
  const hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_gauge_action, dim3(nb), dim3(kGaugeBlock), 0, s, k, (const double2*)U64,
                     1.0 - 8.0 * c1, c1, part);
  LQCD_LAUNCH_CHECK();
  return reduce_to_host(part, nb, beta, part + nb + 16, S, s);
}

int lqcd_gauge_force(const lqcd_geom* g, const void* U64, double beta, double c1,
                     int32_t accumulate, void* F, void* stream) {
  clear_error();
  int rc;
  if ((rc = check_geom(g)) || (rc = check_ptr(U64, "U64")) || (rc = check_ptr(F, "F")) ||
      (rc = check_c1(beta, c1)))
    return rc;
  if (accumulate != 0 && accumulate != 1) {
    set_error("accumulate must be 0 or 1");
    return LQCD_ERR_INVALID_ARG;
  }
  if (F == U64) {
    set_error("F must not alias U64");
    return LQCD_ERR_INVALID_ARG;
  }
  const KGeom k = make_kgeom(g);
  const int64_t n = 4 * link_threads_per_segment(k.Vh);
  // F is linear in the staple sum, so the shapes split over three launches:
  // the later ones add TA(U (-beta/3) A_k) onto the first's result.
  const dim3 grid(unsigned(n / kGaugeBlock));
  const hipStream_t s = (hipStream_t)stream;
  const int tz = slab_tile(k.Lz);
  if (c1 == 0.0) {
    hipLaunchKernelGGL(k_gauge_force<kStaplePlaq>, grid, dim3(kGaugeBlock), 0, s, k,
                       (const double2*)U64, beta, 1.0, 0.0, accumulate, tz, (double2*)F);
    LQCD_LAUNCH_CHECK();
    return LQCD_OK;
  }
  hipLaunchKernelGGL(k_gauge_force<kStaplePass1>, grid, dim3(kGaugeBlock), 0, s, k,
                     (const double2*)U64, beta, 1.0 - 8.0 * c1, c1, accumulate, tz, (double2*)F);
  LQCD_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gauge_force<kStaplePass2>, grid, dim3(kGaugeBlock), 0, s, k,
                     (const double2*)U64, beta, 1.0 - 8.0 * c1, c1, 1, tz, (double2*)F);
  LQCD_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_gauge_force<kStaplePass3>, grid, dim3(kGaugeBlock), 0, s, k,
                     (const double2*)U64, beta, 1.0 - 8.0 * c1, c1, 1, tz, (double2*)F);
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

size_t lqcd_gauge_force_staples_workspace_bytes(const lqcd_geom* g) {
  if (check_geom(g)) return 0;
  const KGeom k = make_kgeom(g);
  return size_t(4) * 2 * 9 * size_t(k.Vh) * sizeof(double2);
}

int lqcd_gauge_force_staples(const lqcd_geom* g, const void* U64, double beta, double c1,
                             int32_t accumulate, void* F, void* ws, size_t ws_bytes,
                             void* stream) {
  clear_error();
  int rc;
  if ((rc = check_geom(g)) || (rc = check_ptr(U64, "U64")) || (rc = check_ptr(F, "F")) ||
      (rc = check_ptr(ws, "ws")) || (rc = check_c1(beta, c1)))
    return rc;
  if (accumulate != 0 && accumulate != 1) {
    set_error("accumulate must be 0 or 1");
    return LQCD_ERR_INVALID_ARG;
  }
  if (F == U64 || ws == U64 || ws == F) {
    set_error("F, U64 and ws must be distinct buffers");
    return LQCD_ERR_INVALID_ARG;
  }
  const size_t need = lqcd_gauge_force_staples_workspace_bytes(g);
  if (ws_bytes < need) {
    set_error("gauge force workspace of %zu bytes is too small: %zu needed", ws_bytes, need);
    return LQCD_ERR_WORKSPACE;
  }
  const KGeom k = make_kgeom(g);
  const hipStream_t s = (hipStream_t)stream;
  const dim3 g1(unsigned(link_threads_per_segment(k.Vh) / kGaugeBlock));
  const dim3 g2(unsigned(2 * link_threads_per_segment(k.Vh) / kGaugeBlock));
  const int tz = slab_tile(k.Lz);
  int seen = 0;  // directions whose F has been written
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = mu + 1; nu < 4; ++nu) {
      int first = 0;
      if (!accumulate) {
        if (!(seen & (1 << mu))) first |= 1;
        if (!(seen & (1 << nu))) first |= 2;
      }
      seen |= (1 << mu) | (1 << nu);
      hipLaunchKernelGGL(k_staple_fields, g1, dim3(kGaugeBlock), 0, s, k, (const double2*)U64,
                         mu, nu, tz, (double2*)ws);
      LQCD_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_force_pair, g2, dim3(kGaugeBlock), 0, s, k, (const double2*)U64,
                         (const double2*)ws, mu, nu, beta, 1.0 - 8.0 * c1, c1, first, tz,
                         (double2*)F);
      LQCD_LAUNCH_CHECK();
    }
  return LQCD_OK;
}

int lqcd_md_update_momenta(const lqcd_geom* g, const void* F, double eps, void* H,
                           void* stream) {
  clear_error();
  int rc;
  if ((rc = check_geom(g)) || (rc = check_ptr(F, "F")) || (rc = check_ptr(H, "H"))) return rc;
  if (!std::isfinite(eps)) {
    set_error("eps must be finite");
    return LQCD_ERR_INVALID_ARG;
  }
  if (F == H) {
    set_error("F must not alias H");
    return LQCD_ERR_INVALID_ARG;
  }
  const KGeom k = make_kgeom(g);
  const int64_t n = int64_t(8) * 9 * k.Vh;
  hipLaunchKernelGGL(k_md_momenta, dim3(unsigned((n + kMdBlock - 1) / kMdBlock)), dim3(kMdBlock),
                     0, (hipStream_t)stream, n, (const double2*)F, eps, (double2*)H);
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

int lqcd_md_update_links(const lqcd_geom* g, const void* H, double eps, void* U64,
                         void* stream) {
  clear_error();
  int rc;
  if ((rc = check_geom(g)) || (rc = check_ptr(H, "H")) || (rc = check_ptr(U64, "U64"))) return rc;
  if (!std::isfinite(eps)) {
    set_error("eps must be finite");
    return LQCD_ERR_INVALID_ARG;
  }
  if (H == U64) {
    set_error("H must not alias U64");
    return LQCD_ERR_INVALID_ARG;
  }
  const KGeom k = make_kgeom(g);
  const int64_t n = int64_t(8) * k.Vh;
  hipLaunchKernelGGL(k_md_links, dim3(unsigned((n + kGaugeBlock - 1) / kGaugeBlock)),
                     dim3(kGaugeBlock), 0, (hipStream_t)stream, k, (const double2*)H, eps,
                     (double2*)U64);
  LQCD_LAUNCH_CHECK();
  return LQCD_OK;
}

int lqcd_kinetic_energy(const lqcd_geom* g, const void* H, double* K, void* ws, size_t ws_bytes,
                        void* stream) {
  clear_error();
  int rc;
  if ((rc = check_geom(g)) || (rc = check_ptr(H, "H")) || (rc = check_ptr(ws, "ws"))) return rc;
  if (!K) {
    set_error("K must be a host pointer");
    return LQCD_ERR_INVALID_ARG;
  }
  if (ws_bytes < lqcd_gauge_workspace_bytes(g)) {
    set_error("gauge workspace of %zu bytes is too small: %zu needed", ws_bytes,
              lqcd_gauge_workspace_bytes(g));
    return LQCD_ERR_WORKSPACE;
  }
  const KGeom k = make_kgeom(g);
  const int nb = int((int64_t(8) * k.Vh + kGaugeBlock - 1) / kGaugeBlock);
  double* part = static_cast<double*>(ws);
  const hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_kinetic, dim3(nb), dim3(kGaugeBlock), 0, s, k, (const double2*)H, part);
  LQCD_LAUNCH_CHECK();
  return reduce_to_host(part, nb, 0.5, part + nb + 16, K, s);
}

}  // extern "C"
