/* The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_sanitizers.py): every entry point over small random problems,
 * targets equal to and apart from the sources, points on and near the wall,
 * coincident sources; the results must be finite and the sanitizers silent. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_halfspace(int kernel, const double* y, const double* s, long n_src, const double* x, long n_tgt,
                     double* u, int nthreads);
int oracle_freespace(int kernel, const double* y, const double* s, long n_src, const double* x, long n_tgt,
                     double* u, int nthreads);
void oracle_correction(int kernel, const double* y, const double* s, const double* x, double* phi, double* grad);

static double urand(unsigned long long* st)
{
    *st = *st * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(*st >> 11) / 9007199254740992.0;
}

int main(void)
{
    unsigned long long st = 7;
    int bad = 0;
    for (int kernel = 0; kernel < 3; ++kernel) {
        for (int rep = 0; rep < 20; ++rep) {
            const long n = 1 + (long)(urand(&st) * 40), t = 1 + (long)(urand(&st) * 30);
            double* y = malloc(sizeof(double) * 3 * n);
            double* s = malloc(sizeof(double) * 6 * n);
            double* x = malloc(sizeof(double) * 3 * (n + t));
            double* u = malloc(sizeof(double) * 3 * (n + t));
            for (long i = 0; i < n; ++i) {
                for (int a = 0; a < 3; ++a) y[3 * i + a] = urand(&st);
                y[3 * i + 2] = rep % 3 == 0 ? 1e-8 + 1e-3 * urand(&st) : y[3 * i + 2] + 1e-9;
                for (int a = 0; a < 6; ++a) s[6 * i + a] = urand(&st) - 0.5;
            }
            if (n > 1) for (int a = 0; a < 3; ++a) y[3 * (n - 1) + a] = y[a]; /* coincident pair */
            for (long i = 0; i < n; ++i) for (int a = 0; a < 3; ++a) x[3 * i + a] = y[3 * i + a];
            for (long i = n; i < n + t; ++i) {
                for (int a = 0; a < 3; ++a) x[3 * i + a] = urand(&st);
                if (i % 4 == 0) x[3 * i + 2] = 0.0; /* on the wall */
            }
            if (oracle_halfspace(kernel, y, s, n, x, n + t, u, 1) != 0) ++bad;
            for (long i = 0; i < 3 * (n + t); ++i) bad += !isfinite(u[i]);
            if (oracle_freespace(kernel, y, s, n, x + 3 * n, t, u, 2) != 0) ++bad;
            for (long i = 0; i < 3 * t; ++i) bad += !isfinite(u[i]);
            double phi[4], grad[12];
            oracle_correction(kernel, y, s, x + 3 * n, phi, grad);
            free(y);
            free(s);
            free(x);
            free(u);
        }
    }
    printf("oracle: %d problems with errors or non-finite values\n", bad);
    return bad ? 1 : 0;
}
