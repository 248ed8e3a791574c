/* Image structure function by direct differences, FP64.
 *
 * Oracle code (test infrastructure only).  For each wave vector q and lag m:
 *     D[q][m] = 1/(N-m) * sum_{n=m}^{N-1} |F[q][n] - F[q][n-m]|^2
 * which is Eq. (1) of the paper (section "The algorithm") with its indices read
 * as I_n - I_{n-m}.  A plain double loop; no FFT, no reordering of the sum.
 *
 * F: [Q][N] complex, interleaved (re, im) doubles.  D: [Q][M] doubles.
 */
#include <omp.h>

void oracle_direct_diff(const double *F, long Q, long N, long M, double *D, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (long q = 0; q < Q; ++q) {
        const double *f = F + 2 * q * N;
        double *d = D + q * M;
        for (long m = 0; m < M; ++m) {
            double acc = 0.0;
            for (long n = m; n < N; ++n) {
                double dr = f[2 * n] - f[2 * (n - m)];
                double di = f[2 * n + 1] - f[2 * (n - m) + 1];
                acc += dr * dr + di * di;
            }
            d[m] = acc / (double)(N - m);
        }
    }
}
