/*
 * Per-matrix arithmetic of the seeded input generators (synthetic SU(3)
 * links).  The random numbers themselves are drawn by numpy's PCG64 in
 * synth/__init__.py and passed in; this file only turns them into matrices.
 * It contains nothing of the solver (no hopping term, no Krylov method).
 *
 * Complex numbers are interleaved doubles; a matrix is 9 complex row-major.
 */
#include <complex.h>
#include <math.h>

typedef double complex cplx;

/* rows 0 and 1 Gram-Schmidt orthonormalised, row 2 = conj(row0 x row1) */
static void complete_su3(cplx m[9])
{
    double n0 = 0;
    for (int k = 0; k < 3; ++k) n0 += creal(m[k] * conj(m[k]));
    n0 = 1.0 / sqrt(n0);
    for (int k = 0; k < 3; ++k) m[k] *= n0;
    cplx d = 0;
    for (int k = 0; k < 3; ++k) d += conj(m[k]) * m[3 + k];
    double n1 = 0;
    for (int k = 0; k < 3; ++k) {
        m[3 + k] -= d * m[k];
        n1 += creal(m[3 + k] * conj(m[3 + k]));
    }
    n1 = 1.0 / sqrt(n1);
    for (int k = 0; k < 3; ++k) m[3 + k] *= n1;
    m[6] = conj(m[1] * m[5] - m[2] * m[4]);
    m[7] = conj(m[2] * m[3] - m[0] * m[5]);
    m[8] = conj(m[0] * m[4] - m[1] * m[3]);
}

static void matmul3(const cplx a[9], const cplx b[9], cplx c[9])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            c[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}

/* Haar SU(3) from 9 complex Gaussians per matrix */
void synth_su3_from_gauss(const double *z, double *out, long n)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        cplx m[9];
        for (int k = 0; k < 9; ++k) m[k] = z[18 * i + 2 * k] + I * z[18 * i + 2 * k + 1];
        complete_su3(m);
        for (int k = 0; k < 9; ++k) {
            out[18 * i + 2 * k] = creal(m[k]);
            out[18 * i + 2 * k + 1] = cimag(m[k]);
        }
    }
}

/*
 * exp(i beta H) with H = sum_a c_a lambda_a / 2 (Gell-Mann matrices), by
 * scaling and squaring of a degree-12 Taylor polynomial (|A| <= 1/8 after
 * scaling), then rows re-orthonormalised so the result is SU(3) to rounding.
 */
void synth_su3_expi(const double *c, double beta, double *out, long n)
{
    const double s3 = 1.0 / sqrt(3.0);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        const double *a = c + 8 * i;
        cplx H[9];
        H[0] = 0.5 * (a[2] + s3 * a[7]);
        H[4] = 0.5 * (-a[2] + s3 * a[7]);
        H[8] = 0.5 * (-2.0 * s3 * a[7]);
        H[1] = 0.5 * (a[0] - I * a[1]);
        H[3] = conj(H[1]);
        H[2] = 0.5 * (a[3] - I * a[4]);
        H[6] = conj(H[2]);
        H[5] = 0.5 * (a[5] - I * a[6]);
        H[7] = conj(H[5]);
        cplx A[9];
        double nrm = 0;
        for (int r = 0; r < 3; ++r) {
            double row = 0;
            for (int k = 0; k < 3; ++k) {
                A[3 * r + k] = I * beta * H[3 * r + k];
                row += cabs(A[3 * r + k]);
            }
            if (row > nrm) nrm = row;
        }
        int sq = 0;
        while (nrm > 0.125) {
            nrm *= 0.5;
            ++sq;
        }
        const double scale = ldexp(1.0, -sq);
        for (int k = 0; k < 9; ++k) A[k] *= scale;
        cplx E[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, T[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, tmp[9];
        for (int d = 1; d <= 12; ++d) {
            matmul3(T, A, tmp);
            for (int k = 0; k < 9; ++k) {
                T[k] = tmp[k] / d;
                E[k] += T[k];
            }
        }
        for (int s = 0; s < sq; ++s) {
            matmul3(E, E, tmp);
            for (int k = 0; k < 9; ++k) E[k] = tmp[k];
        }
        complete_su3(E);
        for (int k = 0; k < 9; ++k) {
            out[18 * i + 2 * k] = creal(E[k]);
            out[18 * i + 2 * k + 1] = cimag(E[k]);
        }
    }
}
