// Host-side plumbing of the C ABI: status strings, thread-local error detail,
// geometry validation and buffer sizes.
#include <cstdarg>
#include <cstdio>

#include "common.h"

namespace lqcd {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = 0; }

KGeom make_kgeom(const lqcd_geom* g) {
  KGeom k;
  k.Lx = g->L[0];
  k.Lxh = g->L[0] / 2;
  k.Ly = g->L[1];
  k.Lz = g->L[2];
  k.Lt = g->L[3];
  k.sy = k.Lxh;
  k.sz = k.Lxh * k.Ly;
  k.st = k.Lxh * k.Ly * k.Lz;
  k.Vh = k.st * k.Lt;
  k.anti = g->antiperiodic_t ? 1 : 0;
  return k;
}

int check_geom(const lqcd_geom* g) {
  if (!g) {
    set_error("geometry pointer is NULL");
    return LQCD_ERR_INVALID_ARG;
  }
  int64_t V = 1;
  for (int mu = 0; mu < 4; ++mu) {
    const int n = g->L[mu];
    if (n < 2 || (n & 1)) {
      set_error("extent L[%d] = %d must be even and >= 2", mu, n);
      return LQCD_ERR_INVALID_ARG;
    }
    V *= n;
  }
  if ((V / 2) * 144 >= (int64_t(1) << 32)) {
    // byte offsets inside one [9][Vh] FP64 link block (the stencil's buffer
    // loads) stay in uint32
    set_error("lattice too large: V/2 = %lld must be below 2^32 / 144 = %lld", (long long)(V / 2),
              (long long)(((int64_t(1) << 32) - 1) / 144));
    return LQCD_ERR_INVALID_ARG;
  }
  if (g->antiperiodic_t != 0 && g->antiperiodic_t != 1) {
    set_error("antiperiodic_t must be 0 or 1, got %d", g->antiperiodic_t);
    return LQCD_ERR_INVALID_ARG;
  }
  return LQCD_OK;
}

int check_prec_fmt(int prec, int fmt) {
  if (prec != LQCD_F64 && prec != LQCD_F32) {
    set_error("precision must be LQCD_F64 (0) or LQCD_F32 (1), got %d", prec);
    return LQCD_ERR_INVALID_ARG;
  }
  if (fmt != LQCD_LINKS18 && fmt != LQCD_LINKS12 && fmt != LQCD_LINKS12D &&
      fmt != LQCD_LINKS12T) {
    set_error("link format must be LQCD_LINKS18 (0), LQCD_LINKS12 (1), LQCD_LINKS12D (2) or "
              "LQCD_LINKS12T (3), got %d",
              fmt);
    return LQCD_ERR_INVALID_ARG;
  }
  return LQCD_OK;
}

int check_ptr(const void* p, const char* name) {
  if (!p) {
    set_error("%s is NULL", name);
    return LQCD_ERR_INVALID_ARG;
  }
  if (reinterpret_cast<uintptr_t>(p) & 15) {
    set_error("%s = %p is not 16-byte aligned", name, p);
    return LQCD_ERR_INVALID_ARG;
  }
  return LQCD_OK;
}

int check_nrhs(int32_t nrhs) {
  if (nrhs < 1 || nrhs > 64) {
    set_error("nrhs = %d must be in [1, 64]", nrhs);
    return LQCD_ERR_INVALID_ARG;
  }
  return LQCD_OK;
}

}  // namespace lqcd

using namespace lqcd;

extern "C" {

const char* lqcd_status_string(int s) {
  switch (s) {
    case LQCD_OK: return "LQCD_OK";
    case LQCD_ERR_INVALID_ARG: return "LQCD_ERR_INVALID_ARG";
    case LQCD_ERR_UNSUPPORTED: return "LQCD_ERR_UNSUPPORTED";
    case LQCD_ERR_WORKSPACE: return "LQCD_ERR_WORKSPACE";
    case LQCD_ERR_HIP: return "LQCD_ERR_HIP";
    case LQCD_ERR_NOT_CONVERGED: return "LQCD_ERR_NOT_CONVERGED";
    case LQCD_ERR_NUMERIC: return "LQCD_ERR_NUMERIC";
    default: return "LQCD_ERR_UNKNOWN";
  }
}

const char* lqcd_last_error(void) { return g_err; }

int lqcd_version(void) { return 10000; }

size_t lqcd_links_bytes(const lqcd_geom* g, int prec, int fmt) {
  if (check_geom(g) != LQCD_OK || check_prec_fmt(prec, fmt) != LQCD_OK) return 0;
  const KGeom k = make_kgeom(g);
  return size_t(2) * 4 * link_reals(fmt) * size_t(k.Vh) * real_bytes(prec);
}

size_t lqcd_spinor_bytes(const lqcd_geom* g, int prec) {
  if (check_geom(g) != LQCD_OK || check_prec_fmt(prec, LQCD_LINKS18) != LQCD_OK) return 0;
  const KGeom k = make_kgeom(g);
  return size_t(3) * size_t(k.Vh) * 2 * real_bytes(prec);
}

}  // extern "C"
