/*
 * Plain FP64 CPU oracle for the even/odd staggered solver.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * table or helper with the GPU library: everything below is written out
 * directly from the definitions, in natural (lexicographic, unsplit) layout,
 * with plain loops, one site at a time.  It is meant to be slow and obvious.
 *
 * Layout (natural, complex128 = two doubles re, im):
 *   links   U[mu][lex][a][b]       mu = 0..3 (x, y, z, t), 3x3 row-major
 *   fields  psi[lex][c]            c = 0..2 colour, all V sites
 *   lex = x + Lx*(y + Ly*(z + Lz*t)), parity = (x+y+z+t) mod 2 (0 = even).
 * Even-site vectors are full-lattice arrays whose odd entries are ignored on
 * input and written as zero on output.
 *
 * What each function follows:
 *   hop / doe / deo    the off-diagonal blocks D_oe, D_eo of the staggered
 *                      Dirac matrix (Sec. 2: nearest-neighbour hopping with
 *                      U_mu(x) times a U(1) factor that carries the staggered
 *                      phases and the antiperiodic time boundary, Sec. 4.1),
 *                      normalised with a factor 1/2 so that D_oe^dag = -D_eo
 *                      and the free operator has spectrum m^2 + sum sin^2 p.
 *   apply_A            the shifted normal operator (m^2 - D_eo D_oe + sigma)
 *                      of Eq. (2), on even sites.
 *   cg                 conjugate gradient on one system of Eq. (2).
 *   cg_multishift      the shifted (multi-mass) CG that solves all systems
 *                      of Eq. (2) from one Krylov sequence (Sec. 2).
 *   action             the fermion term of Eq. (1) with M^(-1/4) replaced by
 *                      its rational form alpha_0 + sum_i alpha_i/(A+sigma_i).
 *   force              the derivative of that action with respect to the
 *                      links (the fermion force driving the MD, Sec. 2 and
 *                      Sec. 4), as the exact derivative of the quadratic form.
 *   gauge_action       the tree-level Symanzik gauge action S_g of Eq. (1):
 *                      every 1x1 plaquette and every 1x2 rectangle (both
 *                      orientations) enumerated once, weights c0 = 1 - 8 c1
 *                      and c1 (Sec. 2).
 *   gauge_force        its derivative with respect to the links: for every
 *                      loop and every link on it, the product of the other
 *                      links around the loop (the exact derivative of the
 *                      loop's real trace), then the su(3) projection used by
 *                      force (Sec. 4, the MD gauge term).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* geometry                                                             */
/* ------------------------------------------------------------------ */

static long volume_of(const int L[4]) { return (long)L[0] * L[1] * L[2] * L[3]; }

static long lex_of(const int L[4], const int c[4])
{
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

static void coords_of(const int L[4], long lex, int c[4])
{
    c[0] = (int)(lex % L[0]); lex /= L[0];
    c[1] = (int)(lex % L[1]); lex /= L[1];
    c[2] = (int)(lex % L[2]); lex /= L[2];
    c[3] = (int)lex;
}

static int parity_of(const int c[4]) { return (c[0] + c[1] + c[2] + c[3]) & 1; }

/* neighbour of c one step along mu, in direction dir = +1 or -1, periodic wrap */
static void step(const int L[4], const int c[4], int mu, int dir, int out[4])
{
    for (int k = 0; k < 4; ++k) out[k] = c[k];
    out[mu] = (c[mu] + dir + L[mu]) % L[mu];
}

/* staggered phase eta_mu(x) = (-1)^(x_0 + ... + x_{mu-1}) */
static double eta(int mu, const int c[4])
{
    int s = 0;
    for (int nu = 0; nu < mu; ++nu) s += c[nu];
    return (s & 1) ? -1.0 : 1.0;
}

/* boundary sign carried by the link (c, mu): -1 on time links that cross
 * the last time slice when time is antiperiodic, +1 otherwise */
static double link_sign(const int L[4], int antiperiodic, int mu, const int c[4])
{
    return (antiperiodic && mu == 3 && c[3] == L[3] - 1) ? -1.0 : 1.0;
}

static const cplx *link_at(const cplx *U, long V, int mu, long lex)
{
    return U + ((long)mu * V + lex) * 9;
}

/* ------------------------------------------------------------------ */
/* hopping term                                                         */
/* ------------------------------------------------------------------ */

/*
 * out(x) = 1/2 sum_mu eta_mu(x) [ s_mu(x) U_mu(x) in(x+mu)
 *                                 - s_mu(x-mu) U_mu(x-mu)^dag in(x-mu) ]
 * for every site x of parity out_parity; sites of the other parity in out
 * are set to zero.  Input entries of parity out_parity are never read.
 */
void orc_hop(const int *L, int antiperiodic, const double *Ud, const double *ind,
             double *outd, int out_parity)
{
    const long V = volume_of(L);
    const cplx *U = (const cplx *)Ud;
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;

#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        int c[4];
        coords_of(L, x, c);
        cplx acc[3] = {0, 0, 0};
        if (parity_of(c) == out_parity) {
            for (int mu = 0; mu < 4; ++mu) {
                int cf[4], cb[4];
                step(L, c, mu, +1, cf);
                step(L, c, mu, -1, cb);
                const double e = eta(mu, c);
                const double sf = link_sign(L, antiperiodic, mu, c);
                const double sb = link_sign(L, antiperiodic, mu, cb);
                const cplx *Uf = link_at(U, V, mu, x);
                const cplx *Ub = link_at(U, V, mu, lex_of(L, cb));
                const cplx *pf = in + lex_of(L, cf) * 3;
                const cplx *pb = in + lex_of(L, cb) * 3;
                for (int a = 0; a < 3; ++a) {
                    cplx fwd = 0, bwd = 0;
                    for (int b = 0; b < 3; ++b) {
                        fwd += Uf[a * 3 + b] * pf[b];          /* U psi      */
                        bwd += conj(Ub[b * 3 + a]) * pb[b];    /* U^dag psi  */
                    }
                    acc[a] += e * (sf * fwd - sb * bwd);
                }
            }
        }
        for (int a = 0; a < 3; ++a) out[x * 3 + a] = 0.5 * acc[a];
    }
}

/* D_oe: even input -> odd output;  D_eo: odd input -> even output */
void orc_doe(const int *L, int anti, const double *U, const double *in, double *out)
{
    orc_hop(L, anti, U, in, out, 1);
}

void orc_deo(const int *L, int anti, const double *U, const double *in, double *out)
{
    orc_hop(L, anti, U, in, out, 0);
}

/* ------------------------------------------------------------------ */
/* even-site vector algebra (sequential, fixed order)                   */
/* ------------------------------------------------------------------ */

static int is_even(const int L[4], long x)
{
    int c[4];
    coords_of(L, x, c);
    return parity_of(c) == 0;
}

/* <a, b> = sum over even sites and colours of conj(a) b */
static cplx dot_even(const int L[4], const cplx *a, const cplx *b)
{
    const long V = volume_of(L);
    cplx s = 0;
    for (long x = 0; x < V; ++x)
        if (is_even(L, x))
            for (int c = 0; c < 3; ++c) s += conj(a[x * 3 + c]) * b[x * 3 + c];
    return s;
}

static double norm2_even(const int L[4], const cplx *a)
{
    return creal(dot_even(L, a, a));
}

/*
 * y = (m2 + sigma) x - D_eo D_oe x on even sites; tmp is an odd-site scratch
 * field of V*3 complex.
 */
void orc_apply_A(const int *L, int anti, const double *Ud, double m2,
                 double sigma, const double *xd, double *yd, double *tmpd)
{
    const long V = volume_of(L);
    const cplx *x = (const cplx *)xd;
    cplx *y = (cplx *)yd;
    orc_doe(L, anti, Ud, xd, tmpd);
    orc_deo(L, anti, Ud, tmpd, yd);
    for (long s = 0; s < V; ++s)
        for (int c = 0; c < 3; ++c)
            y[s * 3 + c] = is_even(L, s) ? (m2 + sigma) * x[s * 3 + c] - y[s * 3 + c] : 0;
}

/* ||b - (A + sigma) x|| / ||b|| on even sites */
double orc_true_residual(const int *L, int anti, const double *Ud, double m2,
                         double sigma, const double *bd, const double *xd)
{
    const long V = volume_of(L);
    cplx *Ax = calloc((size_t)V * 3, sizeof(cplx));
    cplx *tmp = calloc((size_t)V * 3, sizeof(cplx));
    const cplx *b = (const cplx *)bd;
    orc_apply_A(L, anti, Ud, m2, sigma, xd, (double *)Ax, (double *)tmp);
    for (long s = 0; s < V * 3; ++s) Ax[s] = b[s] - Ax[s];
    double rn = sqrt(norm2_even(L, Ax)), bn = sqrt(norm2_even(L, b));
    free(Ax);
    free(tmp);
    return bn > 0 ? rn / bn : rn;
}

/* ------------------------------------------------------------------ */
/* conjugate gradient on one system of Eq. (2)                          */
/* ------------------------------------------------------------------ */

/*
 * Solves ((m2 + sigma) - D_eo D_oe) x = b on even sites.  x holds the
 * initial guess on entry.  Iterates until ||r|| <= tol ||b||, then checks the
 * recomputed residual b - A x and restarts from it if it is still above tol.
 * Returns 0 on convergence, 1 otherwise; *iters is the total iteration count
 * and *true_res the final relative true residual.
 */
int orc_cg(const int *L, int anti, const double *Ud, double m2, double sigma,
           const double *bd, double *xd, double tol, int max_iter,
           int *iters, double *true_res)
{
    const long V = volume_of(L);
    const long n = V * 3;
    const cplx *b = (const cplx *)bd;
    cplx *x = (cplx *)xd;
    cplx *r = calloc((size_t)n, sizeof(cplx));
    cplx *p = calloc((size_t)n, sizeof(cplx));
    cplx *w = calloc((size_t)n, sizeof(cplx));
    cplx *tmp = calloc((size_t)n, sizeof(cplx));
    const double bnorm = sqrt(norm2_even(L, b));
    int it = 0, status = 1;

    for (long s = 0; s < V; ++s)
        if (!is_even(L, s))
            for (int c = 0; c < 3; ++c) x[s * 3 + c] = 0;

    for (int restart = 0; restart < 20 && it < max_iter; ++restart) {
        /* r = b - A x, p = r */
        orc_apply_A(L, anti, Ud, m2, sigma, xd, (double *)w, (double *)tmp);
        for (long s = 0; s < n; ++s) { r[s] = b[s] - w[s]; p[s] = r[s]; }
        double rho = norm2_even(L, r);
        if (sqrt(rho) <= tol * bnorm) { status = 0; break; }
        while (it < max_iter) {
            orc_apply_A(L, anti, Ud, m2, sigma, (const double *)p, (double *)w, (double *)tmp);
            const double pw = creal(dot_even(L, p, w));
            const double a = rho / pw;
            for (long s = 0; s < n; ++s) { x[s] += a * p[s]; r[s] -= a * w[s]; }
            const double rho_new = norm2_even(L, r);
            ++it;
            if (sqrt(rho_new) <= tol * bnorm) break;
            const double beta = rho_new / rho;
            for (long s = 0; s < n; ++s) p[s] = r[s] + beta * p[s];
            rho = rho_new;
        }
        if (orc_true_residual(L, anti, Ud, m2, sigma, bd, xd) <= tol) { status = 0; break; }
    }
    *iters = it;
    *true_res = orc_true_residual(L, anti, Ud, m2, sigma, bd, xd);
    free(r); free(p); free(w); free(tmp);
    return status;
}

/* ------------------------------------------------------------------ */
/* multi-shift CG                                                       */
/* ------------------------------------------------------------------ */

/*
 * Solves ((m2 + sigma_s) - D_eo D_oe) x_s = b for s = 0..nshift-1 with one
 * Krylov sequence built on the smallest shift sigma_0.  The solution of shift
 * s is kept collinear-residual with the base system through the scalar zeta_s
 * (r_s = zeta_s r), updated by the three-term relation that follows from the
 * Lanczos form of CG: with delta_s = sigma_s - sigma_0,
 *   zeta_s' = zeta_s zeta_s^old a^old /
 *             ( a b^old (zeta_s^old - zeta_s) + zeta_s^old a^old (1 + delta_s a) )
 *   a_s = a zeta_s'/zeta_s,   b_s = b (zeta_s'/zeta_s)^2,
 *   x_s += a_s p_s,           p_s = zeta_s' r + b_s p_s.
 * A shift stops updating once |zeta_s'| ||r|| <= tol ||b||; the iteration stops
 * when the base shift converges.  With verify != 0, any shift whose recomputed
 * residual is above tol is then finished by plain CG started from its
 * multi-shift solution; with verify == 0 that last step (and the residual
 * recomputation) is skipped and true_res is left as NaN.
 *
 * x is [nshift][V][3]; iters_out receives the multi-shift iteration count
 * (plus refinement iterations in iters_out[1]); true_res is [nshift].
 */
int orc_cg_multishift(const int *L, int anti, const double *Ud, double m2,
                      int nshift, const double *sigma, const double *bd,
                      double *xd, double tol, int max_iter, int *iters_out,
                      double *true_res, int verify)
{
    const long V = volume_of(L);
    const long n = V * 3;
    const cplx *b = (const cplx *)bd;
    cplx *x = (cplx *)xd;
    int base = 0;
    for (int s = 1; s < nshift; ++s)
        if (sigma[s] < sigma[base]) base = s;
    const double sig0 = sigma[base];

    cplx *r = calloc((size_t)n, sizeof(cplx));
    cplx *p = calloc((size_t)n, sizeof(cplx));
    cplx *w = calloc((size_t)n, sizeof(cplx));
    cplx *tmp = calloc((size_t)n, sizeof(cplx));
    cplx *ps = calloc((size_t)n * nshift, sizeof(cplx));
    double *zeta = malloc(sizeof(double) * nshift);
    double *zeta_old = malloc(sizeof(double) * nshift);
    int *active = malloc(sizeof(int) * nshift);

    for (long s = 0; s < n; ++s) {
        const int ev = is_even(L, s / 3);
        r[s] = ev ? b[s] : 0;
        p[s] = r[s];
        for (int k = 0; k < nshift; ++k) { ps[k * n + s] = r[s]; x[k * n + s] = 0; }
    }
    for (int k = 0; k < nshift; ++k) { zeta[k] = zeta_old[k] = 1.0; active[k] = 1; }

    const double bnorm = sqrt(norm2_even(L, b));
    double rho = norm2_even(L, r);
    double a_old = 1.0, b_old = 0.0;
    int it = 0;
    while (it < max_iter && sqrt(rho) > tol * bnorm) {
        orc_apply_A(L, anti, Ud, m2, sig0, (const double *)p, (double *)w, (double *)tmp);
        const double a = rho / creal(dot_even(L, p, w));
        double *zeta_new = malloc(sizeof(double) * nshift);
        for (int k = 0; k < nshift; ++k) {
            zeta_new[k] = zeta[k];
            if (!active[k]) continue;
            const double delta = sigma[k] - sig0;
            zeta_new[k] = zeta[k] * zeta_old[k] * a_old /
                          (a * b_old * (zeta_old[k] - zeta[k]) +
                           zeta_old[k] * a_old * (1.0 + delta * a));
            const double ak = a * zeta_new[k] / zeta[k];
            for (long s = 0; s < n; ++s) x[k * n + s] += ak * ps[k * n + s];
        }
        for (long s = 0; s < n; ++s) r[s] -= a * w[s];
        const double rho_new = norm2_even(L, r);
        const double beta = rho_new / rho;
        for (int k = 0; k < nshift; ++k) {
            if (!active[k]) continue;
            const double ratio = zeta_new[k] / zeta[k];
            const double bk = beta * ratio * ratio;
            for (long s = 0; s < n; ++s) ps[k * n + s] = zeta_new[k] * r[s] + bk * ps[k * n + s];
            zeta_old[k] = zeta[k];
            zeta[k] = zeta_new[k];
            if (fabs(zeta_new[k]) * sqrt(rho_new) <= tol * bnorm) active[k] = 0;
        }
        for (long s = 0; s < n; ++s) p[s] = r[s] + beta * p[s];
        a_old = a;
        b_old = beta;
        rho = rho_new;
        free(zeta_new);
        ++it;
    }
    iters_out[0] = it;
    iters_out[1] = 0;
    int status = 0;
    for (int k = 0; k < nshift && !verify; ++k) true_res[k] = NAN;
    for (int k = 0; k < nshift && verify; ++k) {
        double tr = orc_true_residual(L, anti, Ud, m2, sigma[k], bd, (const double *)(x + k * n));
        if (tr > tol) {
            int extra = 0;
            status |= orc_cg(L, anti, Ud, m2, sigma[k], bd, (double *)(x + k * n), tol,
                             max_iter, &extra, &tr);
            iters_out[1] += extra;
        }
        true_res[k] = tr;
    }
    if (it >= max_iter) status = 1;
    free(r); free(p); free(w); free(tmp); free(ps);
    free(zeta); free(zeta_old); free(active);
    return status;
}

/* ------------------------------------------------------------------ */
/* rational action and its link derivative                              */
/* ------------------------------------------------------------------ */

/*
 * S = sum_j [ alpha0 ||phi_j||^2 + sum_i alpha_i Re <phi_j, X_ij> ]
 * phi is [npf][V][3]; X is [npf][nshift][V][3] with X_ij = (A + sigma_i)^-1 phi_j.
 */
double orc_action(const int *L, int npf, int nshift, double alpha0,
                  const double *alpha, const double *phid, const double *Xd)
{
    const long n = volume_of(L) * 3;
    const cplx *phi = (const cplx *)phid;
    const cplx *X = (const cplx *)Xd;
    double S = 0.0;
    for (int j = 0; j < npf; ++j) {
        S += alpha0 * norm2_even(L, phi + j * n);
        for (int i = 0; i < nshift; ++i)
            S += alpha[i] * creal(dot_even(L, phi + j * n, X + ((long)j * nshift + i) * n));
    }
    return S;
}

/*
 * Force of S with respect to the links.  With A_i = (m2 + sigma_i) + D_oe^dag D_oe
 * and X = A_i^-1 phi, the variation is
 *   dS = -sum alpha_i <X, dA_i X> = -2 sum alpha_i Re <chi, dD_oe X>,  chi = D_oe X,
 * which, written link by link as dS = sum Re Tr[dU_mu(x) M_mu(x)], gives
 *   x odd :  M_mu(x) = - sum alpha eta_mu(x) s_mu(x) X(x+mu) chi(x)^dag
 *   x even:  M_mu(x) = + sum alpha eta_mu(x) s_mu(x) chi(x+mu) X(x)^dag
 * (the odd site x is where the link is a forward hop of D_oe, the even site x
 * is the backward hop of the odd site x+mu; eta_mu(x+mu) = eta_mu(x)).
 *
 * mode 0: F = TA(U M), TA(W) = (W - W^dag)/2 - Tr(W - W^dag)/6, so that
 *         for U -> exp(eps T) U, T in su(3): dS/deps = sum Tr[T F].
 * mode 1: F = M^dag, the derivative dS/dRe U + i dS/dIm U.
 * F is natural [4][V][3][3].  X is [npf][nshift][V][3], alpha is [nshift].
 */
void orc_force(const int *L, int anti, const double *Ud, int npf, int nshift,
               const double *alpha, const double *Xd, int mode, double *Fd)
{
    const long V = volume_of(L);
    const long n = V * 3;
    const cplx *U = (const cplx *)Ud;
    const cplx *X = (const cplx *)Xd;
    cplx *F = (cplx *)Fd;
    cplx *M = calloc((size_t)4 * V * 9, sizeof(cplx));
    cplx *chi = calloc((size_t)n, sizeof(cplx));

    for (int j = 0; j < npf; ++j) {
        for (int i = 0; i < nshift; ++i) {
            const cplx *Xk = X + ((long)j * nshift + i) * n;
            orc_doe(L, anti, Ud, (const double *)Xk, (double *)chi);
#pragma omp parallel for schedule(static)
            for (long x = 0; x < V; ++x) {
                int c[4], cf[4];
                coords_of(L, x, c);
                for (int mu = 0; mu < 4; ++mu) {
                    step(L, c, mu, +1, cf);
                    const long xf = lex_of(L, cf);
                    const double coef = alpha[i] * eta(mu, c) * link_sign(L, anti, mu, c);
                    cplx *Mx = M + ((long)mu * V + x) * 9;
                    for (int a = 0; a < 3; ++a)
                        for (int bb = 0; bb < 3; ++bb) {
                            if (parity_of(c) == 1)
                                Mx[a * 3 + bb] -= coef * Xk[xf * 3 + a] * conj(chi[x * 3 + bb]);
                            else
                                Mx[a * 3 + bb] += coef * chi[xf * 3 + a] * conj(Xk[x * 3 + bb]);
                        }
                }
            }
        }
    }

    for (long l = 0; l < 4 * V; ++l) {
        const cplx *Ul = U + l * 9;
        const cplx *Ml = M + l * 9;
        cplx *Fl = F + l * 9;
        if (mode == 1) {
            for (int a = 0; a < 3; ++a)
                for (int bb = 0; bb < 3; ++bb) Fl[a * 3 + bb] = conj(Ml[bb * 3 + a]);
        } else {
            cplx W[9];
            for (int a = 0; a < 3; ++a)
                for (int bb = 0; bb < 3; ++bb) {
                    cplx s = 0;
                    for (int k = 0; k < 3; ++k) s += Ul[a * 3 + k] * Ml[k * 3 + bb];
                    W[a * 3 + bb] = s;
                }
            cplx tr = 0;
            for (int a = 0; a < 3; ++a) tr += W[a * 3 + a] - conj(W[a * 3 + a]);
            for (int a = 0; a < 3; ++a)
                for (int bb = 0; bb < 3; ++bb)
                    Fl[a * 3 + bb] = 0.5 * (W[a * 3 + bb] - conj(W[bb * 3 + a])) -
                                     (a == bb ? tr / 6.0 : 0);
        }
    }
    free(M);
    free(chi);
}

/* ------------------------------------------------------------------ */
/* gauge action and force (tree-level Symanzik)                          */
/* ------------------------------------------------------------------ */

static void mat_mul(const cplx *A, const cplx *B, cplx *C)
{
    cplx T[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            cplx s = 0;
            for (int k = 0; k < 3; ++k) s += A[a * 3 + k] * B[k * 3 + b];
            T[a * 3 + b] = s;
        }
    memcpy(C, T, sizeof(T));
}

static void mat_dag(const cplx *A, cplx *B)
{
    cplx T[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) T[a * 3 + b] = conj(A[b * 3 + a]);
    memcpy(B, T, sizeof(T));
}

/* One closed path of n links: link k is U_{mu[k]}(site[k]), used as U (dag 0)
 * or as U^dag (dag 1). */
typedef struct {
    int n;
    long site[6];
    int mu[6];
    int dag[6];
} loop_t;

static void path_add(const int L[4], loop_t *lp, int c[4], int mu, int dir)
{
    int nb[4];
    if (dir > 0) {
        lp->site[lp->n] = lex_of(L, c);
        lp->mu[lp->n] = mu;
        lp->dag[lp->n] = 0;
        step(L, c, mu, +1, nb);
    } else {
        step(L, c, mu, -1, nb);
        lp->site[lp->n] = lex_of(L, nb);
        lp->mu[lp->n] = mu;
        lp->dag[lp->n] = 1;
    }
    lp->n++;
    for (int k = 0; k < 4; ++k) c[k] = nb[k];
}

/* matrix of link k of the loop as it enters the product */
static void loop_link(const cplx *U, long V, const loop_t *lp, int k, cplx *out)
{
    const cplx *u = link_at(U, V, lp->mu[k], lp->site[k]);
    if (lp->dag[k])
        mat_dag(u, out);
    else
        memcpy(out, u, 9 * sizeof(cplx));
}

/* the loops whose first corner is x: plaquettes mu < nu (weight c0) and the
 * 2 (along mu) x 1 (along nu) rectangles for every mu != nu (weight c1) */
static int loops_at(const int L[4], long x, loop_t lps[18], double w[18], double c0, double c1)
{
    int n = 0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = 0; nu < 4; ++nu) {
            if (nu == mu) continue;
            int c[4];
            if (mu < nu) {
                coords_of(L, x, c);
                loop_t *lp = &lps[n];
                lp->n = 0;
                path_add(L, lp, c, mu, +1);
                path_add(L, lp, c, nu, +1);
                path_add(L, lp, c, mu, -1);
                path_add(L, lp, c, nu, -1);
                w[n++] = c0;
            }
            coords_of(L, x, c);
            loop_t *lp = &lps[n];
            lp->n = 0;
            path_add(L, lp, c, mu, +1);
            path_add(L, lp, c, mu, +1);
            path_add(L, lp, c, nu, +1);
            path_add(L, lp, c, mu, -1);
            path_add(L, lp, c, mu, -1);
            path_add(L, lp, c, nu, -1);
            w[n++] = c1;
        }
    return n;
}

/* S_g = beta sum_loops w (1 - Re Tr W / 3) */
double orc_gauge_action(const int *L, const double *Ud, double beta, double c1)
{
    const long V = volume_of(L);
    const cplx *U = (const cplx *)Ud;
    const double c0 = 1.0 - 8.0 * c1;
    double S = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : S)
    for (long x = 0; x < V; ++x) {
        loop_t lps[18];
        double w[18];
        const int nl = loops_at(L, x, lps, w, c0, c1);
        for (int l = 0; l < nl; ++l) {
            cplx W[9], Lk[9];
            loop_link(U, V, &lps[l], 0, W);
            for (int k = 1; k < lps[l].n; ++k) {
                loop_link(U, V, &lps[l], k, Lk);
                mat_mul(W, Lk, W);
            }
            S += beta * w[l] * (1.0 - creal(W[0] + W[4] + W[8]) / 3.0);
        }
    }
    return S;
}

/* F = TA(U M) with dS_g = sum Re Tr[dU M]: for a loop W = L_1 ... L_n and
 * its link k, d Re Tr W = Re Tr[dL_k R_k] with R_k = L_{k+1} ... L_n L_1
 * ... L_{k-1}; for L_k = U that is Re Tr[dU R_k], for L_k = U^dag it is
 * Re Tr[dU R_k^dag].  F natural [4][V][3][3]. */
void orc_gauge_force(const int *L, const double *Ud, double beta, double c1, double *Fd)
{
    const long V = volume_of(L);
    const cplx *U = (const cplx *)Ud;
    cplx *F = (cplx *)Fd;
    const double c0 = 1.0 - 8.0 * c1;
    cplx *M = calloc((size_t)4 * V * 9, sizeof(cplx));
    for (long x = 0; x < V; ++x) {
        loop_t lps[18];
        double w[18];
        const int nl = loops_at(L, x, lps, w, c0, c1);
        for (int l = 0; l < nl; ++l) {
            const loop_t *lp = &lps[l];
            for (int k = 0; k < lp->n; ++k) {
                cplx R[9], Lk[9];
                memset(R, 0, sizeof(R));
                R[0] = R[4] = R[8] = 1.0;
                for (int q = 1; q < lp->n; ++q) {
                    loop_link(U, V, lp, (k + q) % lp->n, Lk);
                    mat_mul(R, Lk, R);
                }
                if (lp->dag[k]) mat_dag(R, R);
                cplx *Ml = M + ((long)lp->mu[k] * V + lp->site[k]) * 9;
                for (int e = 0; e < 9; ++e) Ml[e] += -beta * w[l] / 3.0 * R[e];
            }
        }
    }
    for (long l = 0; l < 4 * V; ++l) {
        cplx W[9];
        mat_mul(U + l * 9, M + l * 9, W);
        cplx tr = 0;
        for (int a = 0; a < 3; ++a) tr += W[a * 3 + a] - conj(W[a * 3 + a]);
        cplx *Fl = F + l * 9;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                Fl[a * 3 + b] = 0.5 * (W[a * 3 + b] - conj(W[b * 3 + a])) - (a == b ? tr / 6.0 : 0);
    }
    free(M);
}

/* ------------------------------------------------------------------ */
/* threads                                                              */
/* ------------------------------------------------------------------ */

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
