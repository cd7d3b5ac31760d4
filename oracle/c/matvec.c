/* Dense on-the-fly product y = A_bc x for the oracle (test infrastructure only).
 *
 * A_bc[i][j] = b_i * w * K(|x_i - x_j|) * c_j for i != j and b_i * c_i * a_self on
 * the diagonal (Section 2.1, (e:a_2d)/(e:a_3d)); K = -(1/2pi) log r (2D),
 * 1/(4 pi r) (3D) (e:k).  A plain double loop, parallel over rows only.
 *
 * pts: N x d row-major; x: N x nrhs row-major (right-hand sides fastest);
 * rows: the nrows row indices to compute (all rows when NULL);
 * y: nrows x nrhs row-major.
 */
#include <math.h>
#include <stdlib.h>

void oracle_matvec(int d, long N, const double* pts, const double* b, const double* c,
                   double w, double a_self, int nrhs, const double* x,
                   const long* rows, long nrows, double* y)
{
    const double inv2pi = 1.0 / (2.0 * M_PI);
    const double inv4pi = 1.0 / (4.0 * M_PI);
#pragma omp parallel for schedule(dynamic, 16)
    for (long ii = 0; ii < nrows; ++ii) {
        long i = rows ? rows[ii] : ii;
        double* acc = y + ii * nrhs;
        for (int k = 0; k < nrhs; ++k) acc[k] = 0.0;
        for (long j = 0; j < N; ++j) {
            double a;
            if (j == i) {
                a = c[i] * a_self;
            } else {
                double r2 = 0.0;
                for (int t = 0; t < d; ++t) {
                    double dx = pts[i * d + t] - pts[j * d + t];
                    r2 += dx * dx;
                }
                double r = sqrt(r2);
                double kv = (d == 2) ? -inv2pi * log(r) : inv4pi / r;
                a = w * kv * c[j];
            }
            const double* xj = x + j * nrhs;
            for (int k = 0; k < nrhs; ++k) acc[k] += a * xj[k];
        }
        for (int k = 0; k < nrhs; ++k) acc[k] *= b[i];
    }
}
