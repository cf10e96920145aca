/* Risbo half step for Wigner d at a fixed angle (oracle; test use only).
 *
 * Same arithmetic as the numpy form in oracle/wigner.py (the SU(2) polynomial
 * construction behind the recursion the paper names in Section 2.2):
 *
 *   D^{n+1}_{c,a} = ( q sqrt(c a)            D^n_{c-1,a-1}
 *                   + p sqrt((n+1-c) a)      D^n_{c,a-1}
 *                   - p sqrt(c (n+1-a))      D^n_{c-1,a}
 *                   + q sqrt((n+1-c)(n+1-a)) D^n_{c,a} ) / (n+1)
 *
 * D^n is (n+1) x (n+1), row-major, row index c, column index a.  Entries whose
 * magnitude falls below 1e-300 are flushed to zero.  Plain loops, rows in
 * parallel with OpenMP.
 */
#include <math.h>

void oracle_risbo_half_step(const double *D, int n, double *out, double p, double q,
                            const double *sq /* sqrt(k), k = 0 .. n+1 */)
{
    const int w0 = n + 1, w1 = n + 2;
    const double inv = 1.0 / (double)(n + 1);
#pragma omp parallel for schedule(static)
    for (int c = 0; c <= n + 1; ++c) {
        for (int a = 0; a <= n + 1; ++a) {
            double v = 0.0;
            if (c >= 1 && a >= 1) v += q * sq[c] * sq[a] * D[(c - 1) * w0 + (a - 1)];
            if (c <= n && a >= 1) v += p * sq[n + 1 - c] * sq[a] * D[c * w0 + (a - 1)];
            if (c >= 1 && a <= n) v -= p * sq[c] * sq[n + 1 - a] * D[(c - 1) * w0 + a];
            if (c <= n && a <= n) v += q * sq[n + 1 - c] * sq[n + 1 - a] * D[c * w0 + a];
            v *= inv;
            if (fabs(v) < 1e-300) v = 0.0;
            out[c * w1 + a] = v;
        }
    }
}
