// Internal interface of the D_oe / D_eo kernel family.
#pragma once

#include "common.h"

namespace lqcd {

// What the kernel does with acc = (D in)(x) at its output site:
enum DMode {
  DM_PLAIN = 0,  // out = acc                       (+ sum |acc|^2 if partials)
  DM_AXPY = 1,   // out = m2s * diag - acc          (operator of Eq. (2))
  DM_CG = 2,     // r -= alpha * (m2s * diag - acc) (+ sum |r|^2)
  DM_RES = 3     // res = b - (m2s * diag - acc), FP64; r = res if r (+ sum |res|^2)
};

struct DslashCall {
  KGeom g;
  int out_par = 0;        // parity of the output sites (1: D_oe, 0: D_eo)
  int prec = LQCD_F64;    // links, input and arithmetic
  int fmt = LQCD_LINKS18;
  int nrhs = 1;
  int mode = DM_PLAIN;
  int r_prec = LQCD_F64;  // DM_RES: precision of the stored residual
  const void* U = nullptr;
  const void* in = nullptr;
  int64_t in_stride = 0;  // complex elements between consecutive right-hand sides
  void* out = nullptr;
  int64_t out_stride = 0;
  const void* diag = nullptr;
  int64_t diag_stride = 0;
  void* r = nullptr;
  int64_t r_stride = 0;     // complex elements between consecutive slots (or RHS)
  // Residual ring: right-hand side j keeps r_slots slots; the residual of its
  // iteration it is slot it % r_slots (r_iter: per-RHS iteration counters).
  // DM_CG reads slot it and writes slot it + 1; DM_RES writes slot it.
  // r_iter == nullptr: one slot per RHS, updated in place.
  const int* r_iter = nullptr;
  int r_iter_stride = 0;    // in ints
  int r_slots = 1;
  const void* b = nullptr;  // DM_RES: FP64 right-hand side
  int64_t b_stride = 0;
  const double* m2s = nullptr;  // per right-hand side diagonal, or m2s_c when null
  int m2s_stride = 0;           // in doubles
  double m2s_c = 0.0;
  const double* alpha = nullptr;
  int alpha_stride = 0;
  const int* live = nullptr;  // per right-hand side work flag, null = all
  int live_stride = 0;        // in ints
  const int* halt = nullptr;  // early-exit flag checked at kernel entry
  // 1: the site blocks run in reverse order (the same blocks, sites, partials
  // and bits).  The solver runs D_eo against the direction of the D_oe before
  // it, so D_eo first reads the t that D_oe wrote last, while it is still in
  // the last-level (MALL) cache.
  int rev = 0;
  // 1: in, diag and (plain mode) out hold the right-hand sides as interleaved
  // pairs: rows 2q and 2q + 1 share the 2 * stride values from row 2q's start,
  // complex element (c, h) of row 2q + e at index 2 (c Vh + h) + e.  FP32,
  // 12- or 18-real links, plain or fused CG mode, nrhs and the RHS block even,
  // strides of at least 3 Vh.  The stencil then moves each element of two
  // right-hand sides with one 16-byte access (same arithmetic, same bits).
  int pairs = 0;
  double* partials = nullptr; // [nrhs][nblocks]
};

struct DslashCfg {
  int block = 256;  // threads per workgroup (64, 128, 256)
  int rhs_block = 1;  // right-hand sides sharing one link load (1, 2, 4, 8)
  int xcd = 1;      // XCD-contiguous block remap
  int tz = 0;       // site traversal: 0 lexicographic; n > 0 walks (y, z) tiles of ty rows
                    // and tz slices with t inside the tile loop (shorter +-t reuse distance)
  int ty = 0;       // y rows per tile (0: all of Ly); only with tz > 0
  int nt = 0;       // 1: link loads marked non-temporal (each link is used once)
  int occ = 0;      // >0: cap resident waves per SIMD (dynamic LDS reservation), which
                    // shrinks the set of sites in flight so neighbours stay in L2
  int ilv = 0;      // 1: the RHS groups of one site block are consecutive workgroups (links
                    // then come from L2 after the first group, and fewer distinct sites are
                    // in flight); 0: RHS groups along the second grid dimension
  int lf = 0;       // 1: every load of a direction is scheduled before its arithmetic (more
                    // loads in flight per wave, more registers held); buffer loads only
  int hh = 0;       // 1: one hop (forward or backward) per loop iteration instead of both
                    // of a direction: half the loads held, more waves; buffer loads only
  int ns = 0;       // 1: the own-site operands and the outputs (each touched once) are loaded
                    // and stored non-temporal as well, leaving L2 to the neighbour spinors;
                    // only with nt = 1
  int tm = 0;       // > 0: march along t, tm slices per thread (k_dslash_tm; needs
                    // rhs_block 8, 12-real links, tz = ty = ilv = lf = hh = 0, nt = ns = 1)
  int tp = 2;       // t-march: lanes per column sharing its eight right-hand sides (2 or 4)
  int mf = 0;       // 1: the matrix-core contraction (k_dslash_mfma; FP32, 12-real, plain
                    // mode, rhs_block 8, tm = 0); pinned only, never picked by the tuner
};

// Dynamic LDS a workgroup reserves so that at most occ waves per SIMD are resident.
inline int dslash_lds_bytes(const DslashCfg& c) {
  if (c.occ <= 0) return 0;
  const int waves = c.block / 64;                 // per workgroup
  const int wg_per_cu = (4 * c.occ) / waves;      // 4 SIMDs per CU
  if (wg_per_cu < 1) return -1;
  return (160 * 1024) / wg_per_cu / 1024 * 1024;  // 160 KiB of LDS per CU
}

// Workgroups covering one time slice of columns in the t-march.
inline int dslash_tm_column_blocks(const KGeom& g, const DslashCfg& c) {
  const int cols = c.block / c.tp;
  return (g.st + cols - 1) / cols;
}

// Number of workgroups along the site dimension for a configuration.
inline int dslash_nblocks(const KGeom& g, const DslashCfg& c) {
  if (c.tm > 0) return dslash_tm_column_blocks(g, c) * (g.Lt / c.tm);
  return (g.Vh + c.block - 1) / c.block;
}
// Largest partials array any configuration can need.
inline size_t dslash_partials_max(const KGeom& g, int nrhs) {
  return size_t(nrhs) * size_t((g.Vh + 63) / 64);
}

int dslash_launch(const DslashCall& c, const DslashCfg& cfg, hipStream_t st);

// k_dslash for one precision R and link format NE (6: 12-real, 7: 12-real and
// determinant, 8: 12-real and U(1) angle, 9: 18-real), instantiated in
// dslash_inst_*.hip; and the FP64 residual mode on 18-real links.
template <typename R, int NE>
int dslash_launch_fmt(const DslashCall& c, const DslashCfg& cfg, hipStream_t st);
int dslash_launch_res(const DslashCall& c, const DslashCfg& cfg, hipStream_t st);

// The t-march kernel family (dslash_tm.hip).
bool dslash_tm_supported(const DslashCall& c, const DslashCfg& cfg);
int dslash_tm_launch(const DslashCall& c, const DslashCfg& cfg, hipStream_t st);

// The matrix-core variant (dslash_mfma.hip).
bool dslash_mfma_supported(const DslashCall& c, const DslashCfg& cfg);
int dslash_mfma_launch(const DslashCall& c, const DslashCfg& cfg, hipStream_t st);

// Tuned configuration for this call's shape (times candidates on first use
// with private scratch buffers; cached per process).  `forced_rhs_block` > 0
// pins the right-hand-side block.
int dslash_tuned(const DslashCall& c, int forced_rhs_block, hipStream_t st, DslashCfg* out);
void dslash_clear_tuning();

}  // namespace lqcd
