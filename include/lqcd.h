/*
 * lqcd.h -- C ABI of the MI355X (gfx950) staggered even/odd solver library.
 *
 * The library applies the off-diagonal blocks D_oe, D_eo of the staggered
 * Dirac matrix and solves the shifted systems of Eq. (2),
 *     (m^2 I - D_eo D_oe + sigma_i) x_i = b,   i = 1..r,
 * with conjugate gradient and its multi-shift form (Sec. 2), and computes the
 * fermion force, the link derivative of the rational pseudofermion action of
 * Eq. (1) (Sec. 2, the MD force that dominates the run time).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Geometry: extents L = {Lx, Ly, Lz, Lt} (direction mu = 0..3 is x, y, z, t),
 *   each even and >= 2, with 144 * V/2 < 2^32 (byte offsets inside one FP64
 *   18-real link block fit 32 bits; e.g. 86^4 is the largest hypercube);
 *   lex = x + Lx*(y + Ly*(z + Lz*t)); parity =
 *   (x+y+z+t) mod 2 (0 even, 1 odd); V = Lx*Ly*Lz*Lt; Vh = V/2.  Within one
 *   parity a site's half index is lex >> 1 (unique because Lx is even).
 *   Boundaries are periodic in x, y, z; time is antiperiodic when
 *   antiperiodic_t != 0 (the time links leaving the last time slice carry a
 *   minus sign).  Staggered phases eta_mu(x) = (-1)^(x_0+...+x_{mu-1}).
 *
 * Hopping term (Sec. 2; the U(1) factor of Sec. 4.1 carrying the staggered
 * phases and the antiperiodic time boundary):
 *   (D psi)(x) = 1/2 sum_mu eta_mu(x) [ s_mu(x) U_mu(x) psi(x+mu)
 *                                       - s_mu(x-mu) U_mu(x-mu)^dag psi(x-mu) ]
 *   D_oe maps even sites to odd sites, D_eo odd to even; D_oe^dag = -D_eo.
 *
 * Natural layouts (what callers hold):
 *   links   complex128 [4][V][3][3]   U[mu][lex][row][col]
 *   fields  complex128 [nrhs][V][3]
 * Packed layouts (what the solver streams; all structure-of-arrays so that
 * consecutive half indices are consecutive in memory):
 *   spinor  complex  [nrhs][3][Vh]                  one parity
 *   links   complex  [2][4][NE][Vh]  parity of the site the link leaves,
 *           direction, element, half index.  NE = 9 (LQCD_LINKS18, full
 *           matrix, element = 3*row+col) or NE = 6 (LQCD_LINKS12, rows 0-1;
 *           row 2 is rebuilt as the complex conjugate of the cross product of
 *           rows 0 and 1, Sec. 4.1 -- only valid for SU(3) links) or NE = 7
 *           (LQCD_LINKS12D, rows 0-1 and the determinant d as element 6; row
 *           2 = d conj(row0 x row1), exact for every unitary link, so links
 *           carrying U(1) phases (lqcd_apply_u1_phases) stay compressed).
 *           LQCD_LINKS12T (the paper's U(1)-phase storage, Sec. 4.1): a link
 *           u U with U in SU(3) and u = exp(i theta) is stored as rows 0-1 of
 *           U and the angle theta; each [parity][mu] block holds the six
 *           complex planes of Vh followed by one plane of Vh reals (theta),
 *           i.e. 6.5 complex planes (a tensor view [2][4][13][Vh/2]); the
 *           operator rebuilds row 2 and multiplies by cos theta + i sin theta.
 *   complex = two IEEE doubles (LQCD_F64) or two floats (LQCD_F32).
 *
 * Memory and streams: every data pointer is a device pointer owned by the
 * caller, 16-byte aligned; the library never frees it.  `stream` is a
 * hipStream_t (NULL = the default stream).  Pack, unpack, D_oe/D_eo and the
 * force are asynchronous on that stream.  The solvers and the action read
 * results back to the host and synchronise the stream before returning.
 *
 * Errors: every call validates its arguments on the host before any device
 * work; on error nothing is written and a status != LQCD_OK is returned,
 * with a readable detail in lqcd_last_error() (thread-local).  No C++
 * exception crosses this boundary.
 */
#ifndef LQCD_H
#define LQCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum lqcd_status {
    LQCD_OK = 0,
    LQCD_ERR_INVALID_ARG = 1,   /* bad geometry, pointer, size or enum          */
    LQCD_ERR_UNSUPPORTED = 2,   /* valid but not implemented combination         */
    LQCD_ERR_WORKSPACE = 3,     /* workspace missing or smaller than required    */
    LQCD_ERR_HIP = 4,           /* a HIP runtime call failed (detail in message) */
    LQCD_ERR_NOT_CONVERGED = 5, /* max_iter reached; best iterate and stats kept */
    LQCD_ERR_NUMERIC = 6        /* NaN/Inf or a non-positive curvature p.Ap      */
};

enum lqcd_prec { LQCD_F64 = 0, LQCD_F32 = 1 };
enum lqcd_link_fmt { LQCD_LINKS18 = 0, LQCD_LINKS12 = 1, LQCD_LINKS12D = 2, LQCD_LINKS12T = 3 };

typedef struct {
    int32_t L[4];           /* Lx, Ly, Lz, Lt: each even and >= 2;
                               144 Vh < 2^32 (V < 5.96e7, e.g. 86^4)     */
    int32_t antiperiodic_t; /* 1: antiperiodic time boundary, 0: periodic    */
} lqcd_geom;

/* Human-readable name of a status code (static storage). */
const char *lqcd_status_string(int status);
/* Detail of the last error raised on the calling thread ("" if none). */
const char *lqcd_last_error(void);
/* Library version: major*10000 + minor*100 + patch. */
int lqcd_version(void);
/* Releases cached graphs and tuning tables; later calls rebuild them. */
int lqcd_finalize(void);

/* Bytes of one packed link field ([2][4][NE][Vh] complex), 0 on bad input. */
size_t lqcd_links_bytes(const lqcd_geom *g, int prec, int fmt);
/* Bytes of one packed single-parity spinor ([3][Vh] complex), 0 on bad input. */
size_t lqcd_spinor_bytes(const lqcd_geom *g, int prec);

/*
 * Pack natural complex128 links [4][V][3][3] into the packed layout of the
 * requested precision (round to nearest for LQCD_F32) and format.
 * LQCD_LINKS12 drops row 2, which is exact only for SU(3) links; the caller
 * must not fold phases or boundary signs into the links (the kernels apply
 * them).  U_packed must hold lqcd_links_bytes(g, prec, fmt) bytes.
 */
int lqcd_pack_links(const lqcd_geom *g, const void *U_nat, int prec, int fmt,
                    void *U_packed, void *stream);

/*
 * Convert an already packed field into another precision/format
 * (e.g. LQCD_F64/LQCD_LINKS18 -> LQCD_F32/LQCD_LINKS12 for the inner solver).
 * Every source format is first completed to the full matrix; LQCD_LINKS12D
 * destinations store its determinant; LQCD_LINKS12T destinations split it as
 * exp(i theta) U with theta = arg(det) / 3 and U = exp(-i theta) V in SU(3).
 */
int lqcd_convert_links(const lqcd_geom *g, const void *src, int src_prec, int src_fmt,
                       void *dst, int dst_prec, int dst_fmt, void *stream);

/*
 * Unpack a packed LQCD_F64/LQCD_LINKS18 field (links or force) into natural
 * complex128 [4][V][3][3].
 */
int lqcd_unpack_links(const lqcd_geom *g, const void *U_packed, void *U_nat, void *stream);

/*
 * Pack the sites of one parity of natural complex128 fields [nrhs][V][3]
 * into packed [nrhs][3][Vh] of precision prec.  Sites of the other parity
 * are not read.
 */
int lqcd_pack_spinor(const lqcd_geom *g, int parity, int prec, const void *nat,
                     void *packed, int32_t nrhs, void *stream);

/*
 * Inverse of lqcd_pack_spinor: writes every site of nat [nrhs][V][3]
 * (complex128); sites of the other parity are set to zero.
 */
int lqcd_unpack_spinor(const lqcd_geom *g, int parity, int prec, const void *packed,
                       void *nat, int32_t nrhs, void *stream);

/*
 * D_oe (Sec. 2): out_odd = D_oe in_even for nrhs packed right-hand sides
 * ([nrhs][3][Vh] each, precision prec) with links U_packed of (prec, fmt).
 * Each link is loaded once per site and reused across the right-hand sides.
 * 1 <= nrhs <= 64.  in and out must not overlap.
 * Launch configuration: tuned on the first call for each (geometry,
 * precision, format, nrhs, mode) and cached for the process; that first call
 * allocates temporary scratch and synchronises the stream.  Environment:
 * LQCD_TUNE=0 uses a fixed default instead, LQCD_TUNE_VERBOSE=1 prints the
 * timings, LQCD_DSLASH_CFG="block,rhs_block,xcd,tz[,nt,occ,ilv,lf,hh,ty,ns]"
 * pins one configuration (testing and profiling), LQCD_TUNE_CACHE=<file>
 * keeps tuned configurations across processes (one text line per shape,
 * keyed by GPU architecture and CU count; entries that are not valid for the
 * shape are ignored).
 */
int lqcd_doe(const lqcd_geom *g, int prec, int fmt, const void *U_packed,
             const void *in_even, void *out_odd, int32_t nrhs, void *stream);

/* D_eo (Sec. 2): out_even = D_eo in_odd; otherwise as lqcd_doe. */
int lqcd_deo(const lqcd_geom *g, int prec, int fmt, const void *U_packed,
             const void *in_odd, void *out_even, int32_t nrhs, void *stream);

/*
 * The operator of Eq. (2) on even sites:
 *   out_even = (mass^2 + sigma) in_even - D_eo D_oe in_even
 * computed as D_oe into tmp_odd ([nrhs][3][Vh], caller scratch) followed by
 * D_eo with the diagonal term fused into its store (the paper's separate
 * final sum kernel, Sec. 5.2, folded into D_eo).
 */
int lqcd_apply_A(const lqcd_geom *g, int prec, int fmt, const void *U_packed,
                 double mass, double sigma, const void *in_even, void *out_even,
                 void *tmp_odd, int32_t nrhs, void *stream);

typedef struct {
    double mass;               /* m > 0 (the operator uses m^2)                     */
    double tol;                /* relative true residual target, 0 < tol < 1         */
    int32_t max_iter;          /* per solve (refinement counted separately)          */
    int32_t inner_prec;        /* LQCD_F64: plain FP64; LQCD_F32: mixed, see below   */
    int32_t inner_fmt;         /* link format of the inner operator                  */
    int32_t reliable_interval; /* mixed: FP64 residual recomputation period (iters)  */
    int32_t use_graph;         /* 1: replay iteration blocks as a captured hipGraph  */
    int32_t rhs_block;         /* right-hand sides per D_oe/D_eo link load, 0 = tuned */
    int32_t poll_interval;     /* iterations between host convergence checks, 0 = auto
                                  (31 mixed, 62 FP64)                                */
    int32_t max_refine;        /* rounds of per-shift refinement allowed, >= 0       */
    int32_t shift_window;      /* multi-shift: iterations between materialisations of
                                  the shifted x_s, p_s (1..31; 1 = every iteration) */
    double reliable_delta;     /* mixed: also update when |r| fell by this factor    */
    double mixed_switch;       /* mixed multi-shift: iterate in FP64 until |r| <=
                                  mixed_switch |b|, then in FP32 (0: FP32 throughout) */
    double inner_tol_factor;   /* the main iteration stops, and freezes shifts, at
                                  inner_tol_factor * tol (0 < f <= 1); every system is
                                  still verified against tol and refined if above it */
} lqcd_solver_params;

typedef struct {
    int32_t iters;             /* Krylov iterations of the main (multi-shift) solve */
    int32_t reliable_updates;  /* FP64 residual recomputations                       */
    int32_t refine_iters;      /* iterations spent in per-shift refinement           */
    int32_t converged;         /* 1 if the true residual is <= tol                   */
    double true_rel_residual;  /* ||b - (A+sigma) x|| / ||b||, FP64, FP64-18 links   */
    double seconds;            /* wall time of the whole call                        */
    int32_t iters_fp64;        /* of iters, those run in FP64 arithmetic             */
    int32_t shift_window;      /* window length used by the main solve (1: none)     */
    int64_t shift_updates_fp64; /* main solve: sum over FP64 iterations of updated shifts */
    int64_t shift_updates_fp32; /* the same over FP32 iterations                      */
    int64_t flush_shifts_fp64; /* main solve: sum over FP64 window flushes of the
                                  shifts materialised                               */
    int64_t flush_shifts_fp32; /* the same over FP32 window flushes                  */
    int64_t flush_slots_fp64;  /* sum over FP64 window flushes of residuals combined */
    int64_t flush_slots_fp32;  /* the same over FP32 window flushes                  */
} lqcd_solve_stats;

/* Fills p with defaults: tol 1e-10, max_iter 10000, F64 inner, LINKS18,
 * reliable_interval 100, use_graph 1, rhs_block 0, poll 0, max_refine 3,
 * shift_window 31, reliable_delta 1e-3, mixed_switch 1e-3, inner_tol_factor 0.7. */
void lqcd_solver_params_default(lqcd_solver_params *p);

/* Device workspace that lqcd_cg / lqcd_cg_multishift need for these sizes. */
size_t lqcd_solver_workspace_bytes(const lqcd_geom *g, const lqcd_solver_params *p,
                                   int32_t nshift, int32_t nrhs);

/*
 * Conjugate gradient on one shifted system of Eq. (2) for nrhs independent
 * right-hand sides:  ((m^2 + sigma) - D_eo D_oe) x_j = b_j.
 *   U64_packed   LQCD_F64/LQCD_LINKS18 links (used for every FP64 residual)
 *   Uinner       links of (inner_prec, inner_fmt) or NULL (then converted
 *                from U64_packed into the workspace); ignored for F64/18
 *   b            packed even FP64 [nrhs][3][Vh]
 *   x            packed even FP64 [nrhs][3][Vh]; on entry the initial guess
 *   stats        host array [nrhs]
 * Mixed precision (inner_prec = LQCD_F32): the Krylov iteration runs in FP32;
 * whenever the iterated residual has fallen by reliable_delta since the last
 * update, or reliable_interval iterations have passed, or the iteration
 * believes it has converged, the FP32 correction is added into the FP64
 * solution and the residual is recomputed in FP64 (Sec. 5.4: the production
 * split, single precision for MD and double for the accept step).
 * Dot products, norms and the CG scalars are always FP64.  A mixed multi-shift
 * solve first iterates in FP64 until the base residual is below mixed_switch
 * |b|: FP32 rounding then only perturbs the shifted systems at that scale,
 * which keeps their final refinement short.
 * Returns LQCD_ERR_NOT_CONVERGED if any system misses tol within max_iter
 * (x holds the best iterate, stats are filled).
 */
int lqcd_cg(const lqcd_geom *g, const lqcd_solver_params *p, const void *U64_packed,
            const void *Uinner, double sigma, const void *b, void *x, int32_t nrhs,
            lqcd_solve_stats *stats, void *ws, size_t ws_bytes, void *stream);

/*
 * Multi-shift CG (Sec. 2): solves all systems of Eq. (2)
 *   ((m^2 + sigma_i) - D_eo D_oe) x_ji = b_j,  i < nshift, j < nrhs
 * from one Krylov sequence per right-hand side, built on the smallest shift.
 *   sigma   host [nshift], each >= 0, 1 <= nshift <= 32
 *   b       packed even FP64 [nrhs][3][Vh]
 *   x       packed even FP64 [nrhs][nshift][3][Vh] (output; not read)
 *   stats   host [nrhs][nshift]
 * A shift stops updating once its collinear residual is below tol.
 * Deferred shift updates: only the base direction is formed every iteration;
 * each shifted x_s, p_s is a linear combination of its value at the start of
 * a window and of the base residuals of the window (the recurrences of
 * Sec. 2 are linear in them), so the shifted vectors are read and written
 * once per window of shift_window iterations (reduced to a divisor of the
 * poll interval) instead of every iteration.  The window's residuals are kept
 * in the workspace.  After
 * the base system converges, the FP64 true residual of every (j, i) is
 * computed; systems above tol are refined together by warm-started CG on
 * their residuals, up to max_refine rounds.  All right-hand sides share each
 * link load in D_oe/D_eo.  With FP32 inner precision, 12- or 18-real inner
 * links and an even nrhs, the FP32 phase keeps the base directions and D_oe's
 * output in the workspace with right-hand sides 2q and 2q + 1 interleaved
 * element by element, so the stencils load both with one 16-byte access; with
 * the same stencil launch configurations the results are the same bits as
 * with separate rows, which the environment variable LQCD_RHS_PAIRS=0 selects
 * (comparisons).  b, x and the workspace size are unaffected.
 * 1 <= nrhs <= 64.
 */
int lqcd_cg_multishift(const lqcd_geom *g, const lqcd_solver_params *p,
                       const void *U64_packed, const void *Uinner, int32_t nshift,
                       const double *sigma, const void *b, void *x, int32_t nrhs,
                       lqcd_solve_stats *stats, void *ws, size_t ws_bytes, void *stream);

/*
 * Fermion force (Sec. 2): the derivative of
 *   S = sum_j sum_i alpha_i Re <phi_j, X_ji>,  X_ji = (A + sigma_i)^-1 phi_j,
 * with respect to the links, given the solutions X.  With M_mu(x) defined by
 * dS = sum_{x,mu} Re Tr[dU_mu(x) M_mu(x)]:
 *   mode 0: F = TA(U M), TA(W) = (W - W^dag)/2 - Tr(W - W^dag)/6, the su(3)
 *           force (dS/deps = sum Tr[T F] for U -> exp(eps T) U, T in su(3));
 *   mode 1: F = M^dag = dS/dRe U + i dS/dIm U (torch's gradient convention).
 *   U64_packed  LQCD_F64/LQCD_LINKS18 links
 *   alpha       host [nshift]
 *   X           packed even FP64 [npf][nshift][3][Vh]
 *   F           packed FP64 [2][4][9][Vh] (layout of LQCD_LINKS18 links);
 *               accumulate != 0 adds into F instead of overwriting it.
 * D_oe X is recomputed per odd site in registers, never stored; each link is
 * written by exactly one thread (no atomics).
 */
int lqcd_fermion_force(const lqcd_geom *g, const void *U64_packed, int32_t npf,
                       int32_t nshift, const double *alpha, const void *X, int32_t mode,
                       int32_t accumulate, void *F, void *stream);

/*
 * Rational pseudofermion action (Eq. (1) fermion term in rational form):
 *   S = sum_j [ alpha0 ||phi_j||^2 + sum_i alpha_i Re <phi_j, X_ji> ]
 *   phi  packed even FP64 [npf][3][Vh];  X as for lqcd_fermion_force.
 * The result (FP64, fixed-order reduction) is written to *S on the host.
 * ws must hold lqcd_action_workspace_bytes(g) bytes.
 */
size_t lqcd_action_workspace_bytes(const lqcd_geom *g);
int lqcd_action(const lqcd_geom *g, int32_t npf, int32_t nshift, double alpha0,
                const double *alpha, const void *phi, const void *X, double *S,
                void *ws, size_t ws_bytes, void *stream);

/*
 * lqcd_action without a workspace argument and without any device allocation,
 * for callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, kernels and
 * result as lqcd_action, bit for bit; the block partials live in a fixed 1 MiB
 * device array of the library (one copy per device, held until the process
 * ends), which covers every lattice the library accepts.  The first call on a
 * device looks up that copy's address.  A lattice that would need more
 * returns LQCD_ERR_WORKSPACE.  Every call on one device shares the array:
 * calls that overlap on one device (other streams or host threads) race and
 * must be serialised by the caller.  Synchronises the stream before returning.
 */
int lqcd_action_noalloc(const lqcd_geom *g, int32_t npf, int32_t nshift, double alpha0,
                        const double *alpha, const void *phi, const void *X, double *S,
                        void *stream);

/*
 * Rational function of A applied to vectors, from the multi-shift solutions
 * (Sec. 2: the shifts of Eq. (2) are the poles of the rational approximation
 * used by RHMC):
 *   y_j = alpha0 b_j + sum_i alpha_i X_ji,   X_ji = (A + sigma_i)^-1 b_j,
 * so that y_j = r(A) b_j for r(x) = alpha0 + sum_i alpha_i / (x + sigma_i).
 * With the coefficients of r ~ x^(1/8) and b = Gaussian noise this is the
 * pseudofermion heatbath.
 *   b      packed even FP64 [nrhs][3][Vh]
 *   X      packed even FP64 [nrhs][nshift][3][Vh] (the x of lqcd_cg_multishift)
 *   alpha  host [nshift]
 *   y      packed even FP64 [nrhs][3][Vh]; may be b, must not overlap X.
 * The terms are added in a fixed order (FP64 fused multiply-adds), so the
 * result is reproducible.  1 <= nrhs <= 64, 1 <= nshift <= 32.  Stream-ordered,
 * asynchronous, allocates nothing.
 */
int lqcd_rational_combine(const lqcd_geom *g, int32_t nrhs, int32_t nshift, double alpha0,
                          const double *alpha, const void *b, const void *X, void *y,
                          void *stream);

/*
 * U(1) phases on the links (Sec. 4.1): every flavour couples to a U(1) field
 * u_mu(x) = exp(i theta_mu(x)) -- imaginary chemical potential, background
 * (electro)magnetic fields -- and the Dirac operator then hops with
 * u_mu(x) U_mu(x) instead of U_mu(x).  This writes those phased links:
 *   U64    packed FP64 18-real links (in)
 *   theta  device FP64 [4][V], natural lexicographic order
 *   out    packed FP64 18-real (may be U64).
 * Every entry point then takes `out` as its FP64 links: D_oe/D_eo, the
 * solvers and the fermion force (whose TA(U M) is unchanged by the factor).
 * Phased links are not in SU(3) (det = exp(3 i theta)), so LQCD_LINKS12 --
 * which rebuilds row 2 from det = 1 -- must not be used with them; the
 * compressed formats for them are LQCD_LINKS12D (rows 0-1 and the determinant,
 * 7 complex per link) and LQCD_LINKS12T (rows 0-1 and the angle, 6.5 complex
 * per link), e.g. as the inner solver format.  Stream-ordered.
 */
int lqcd_apply_u1_phases(const lqcd_geom *g, const void *U64, const double *theta, void *out,
                         void *stream);

/*
 * LQCD_LINKS12T links from an SU(3) field and one flavour's U(1) angles
 * (Sec. 4.1: the gauge field is shared, each flavour keeps its own phases
 * theta_mu(x), and the operator recomputes cos theta + i sin theta on line):
 *   U64    packed FP64 18-real SU(3) links (rows 0-1 are stored as they are)
 *   theta  device FP64 [4][V], natural lexicographic order
 *   prec   precision of the output (the angle is stored in it too)
 *   out    packed LQCD_LINKS12T links, lqcd_links_bytes(g, prec, LQCD_LINKS12T)
 * D_oe/D_eo on `out` equal D_oe/D_eo on lqcd_apply_u1_phases(U64, theta).
 * Stream-ordered.
 */
int lqcd_pack_links_u1(const lqcd_geom *g, const void *U64, const double *theta, int prec,
                       void *out, void *stream);

/*
 * Stout smearing (Sec. 2: the Dirac operator hops with the k-times stout
 * smeared links U^(k), the MD evolves the unsmeared U^(0)).  One level:
 *   U' = exp(X) U,  X = TA(Omega),  Omega = rho C U^dag,
 * C = sum over nu != mu of the plaquette staples of the link (isotropic
 * rho).  Packed FP64 18-real in and out; out must not alias U64.
 */
int lqcd_stout_smear(const lqcd_geom *g, const void *U64, double rho, void *out, void *stream);

/*
 * Chain rule of the force through one smearing level.  G_smeared is the raw
 * gradient with respect to the smeared links, G' = M'^dag with dS = sum Re
 * Tr[dU' M'] (lqcd_fermion_force mode 1, or this function's mode 1 one level
 * up); U64 are the links before this level.  With E = exp(X) and
 * Lam = TA(L(X, U M')), L(X, B) = sum_k 1/k! sum_j X^j B X^(k-1-j) (the
 * Frechet derivative of exp, computed by scaling and squaring):
 *   M = M' E + rho A Lam^dag + (the staple terms of Re Tr[dA K], K = rho Lam^dag U),
 * A the staple sum; out = TA(U M) (mode 0, the force on U) or M^dag (mode 1,
 * for the next level down).  ws holds lqcd_stout_workspace_bytes(g) (two link
 * fields); out must not alias U64 or G_smeared.  Stream-ordered.
 */
size_t lqcd_stout_workspace_bytes(const lqcd_geom *g);
int lqcd_stout_force(const lqcd_geom *g, const void *U64, double rho, const void *G_smeared,
                     int32_t mode, void *out, void *ws, size_t ws_bytes, void *stream);

/*
 * Gauge part of the molecular dynamics (Sec. 2, Sec. 4.3).  Links U64 and
 * momenta H use the packed FP64 18-real link layout [2][4][9][Vh] (complex);
 * gauge links carry no boundary sign or staggered phase.
 *
 * Tree-level Symanzik action (Sec. 2: only 1x1 and 1x2 loops enter):
 *   S_g = beta sum_x [ c0 sum_{mu<nu} (1 - Re Tr P_mu,nu(x)/3)
 *                    + c1 sum_{mu!=nu} (1 - Re Tr R_mu,nu(x)/3) ],
 * P the plaquette, R the rectangle two links along mu and one along nu,
 * c0 = 1 - 8 c1; c1 = -1/12 is tree-level Symanzik, c1 = 0 Wilson.  The
 * result (FP64, fixed-order reduction) is written to *S on the host; ws must
 * hold lqcd_gauge_workspace_bytes(g) bytes; synchronises the stream.
 */
size_t lqcd_gauge_workspace_bytes(const lqcd_geom *g);
int lqcd_gauge_action(const lqcd_geom *g, const void *U64, double beta, double c1, double *S,
                      void *ws, size_t ws_bytes, void *stream);

/*
 * Gauge force: F = TA(U M) with dS_g = sum Re Tr[dU M] (the convention of
 * lqcd_fermion_force mode 0), i.e. F_mu(x) = -(beta/3) TA(U_mu(x) A_mu(x)),
 * A the c0/c1-weighted sum of the 6 plaquette and 18 rectangle staples of the
 * link.  accumulate != 0 adds into F (e.g. onto the fermion force).  One
 * thread per link; F must not alias U64.  Stream-ordered, asynchronous.
 */
int lqcd_gauge_force(const lqcd_geom *g, const void *U64, double beta, double c1,
                     int32_t accumulate, void *F, void *stream);

/*
 * The same force through staple fields (Sec. 4.3: the staples of 1x1 and 1x2
 * rectangles are the gauge force's building blocks).  For each pair of
 * directions the plaquette staples P+ / P- of every link are stored in the
 * workspace, and each rectangle staple is then two products of those fields
 * and single links (about 51 SU(3) products per link instead of 85).
 * ws must hold lqcd_gauge_force_staples_workspace_bytes(g) bytes (four FP64
 * 18-real link planes: 576 B per site) and not alias U64 or F.  Equal to
 * lqcd_gauge_force up to rounding.  Stream-ordered, asynchronous.
 */
size_t lqcd_gauge_force_staples_workspace_bytes(const lqcd_geom *g);
int lqcd_gauge_force_staples(const lqcd_geom *g, const void *U64, double beta, double c1,
                             int32_t accumulate, void *F, void *ws, size_t ws_bytes,
                             void *stream);

/*
 * MD steps (Sec. 4.3 and Alg. 2: "new momenta", "new configuration").  With U' = i H U,
 * H Hermitian traceless, and F the force above, H^2/2 + S is conserved by
 * H' = -i F:
 *   lqcd_md_update_momenta: H <- H - i eps F           (F must not alias H)
 *   lqcd_md_update_links:   U <- exp(i eps H) U, the exponential by scaling
 *     and squaring of a degree-12 Taylor polynomial, then the rows
 *     re-orthonormalised (row 2 = conj(row0 x row1)), so U stays in SU(3).
 * Stream-ordered, asynchronous, allocate nothing.
 */
int lqcd_md_update_momenta(const lqcd_geom *g, const void *F, double eps, void *H,
                           void *stream);
int lqcd_md_update_links(const lqcd_geom *g, const void *H, double eps, void *U64,
                         void *stream);

/*
 * Kinetic term H^2/2 of Eq. (1): half the sum over links of Tr H^2 (FP64,
 * fixed-order reduction) to *K on the host; ws as for lqcd_gauge_action.
 */
int lqcd_kinetic_energy(const lqcd_geom *g, const void *H, double *K, void *ws,
                        size_t ws_bytes, void *stream);

/*
 * Achievable HBM bandwidth of the current device: STREAM-style copy
 * (read + write) and triad (2 reads + write) over `bytes` per array, median
 * of `reps` timed launches, in GB/s (1e9 B/s).  The roofline of the
 * bandwidth-bound kernels above (the Dirac operator is ~6x below machine
 * balance, Sec. 4.1) is read against this figure and the 8 TB/s specification.
 * Allocates three temporary arrays and synchronises the device.
 */
int lqcd_stream_bandwidth(size_t bytes, int32_t reps, double *copy_gbs, double *triad_gbs);

/*
 * Kernel timing (instrumentation of the solvers; not needed to use them).
 * While enabled, lqcd_cg / lqcd_cg_multishift launch without graph replay
 * and bracket every D_oe, fused D_eo + residual update and multi-shift
 * update launch with HIP events on the caller's stream; durations accumulate
 * per kernel class, named "<kernel>_<f64|f32>[_refine]_n<systems>".
 * lqcd_kernel_timing_enable(1) clears the totals and enables, (0) disables.
 * lqcd_kernel_timing_get reads class `index` (0-based, in first-seen order);
 * it returns LQCD_ERR_INVALID_ARG past the last class.
 */
int lqcd_kernel_timing_enable(int32_t on);
int lqcd_kernel_timing_get(int32_t index, char *name, size_t name_len, int64_t *launches,
                           double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* LQCD_H */
