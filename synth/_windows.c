/* Window builder for the synthetic de-gridding rows.
 *
 * Data generation only (no part of the measurement operator): each row of G
 * is an S x S window made of the outer product of two 1-D vectors (the
 * Kaiser-Bessel taps convolved with a separable w-kernel, one per axis),
 * optionally convolved in 2-D with the Fourier kernel of an antenna pair's
 * direction-dependent effects (Section 3.1: a linear convolution of the
 * pair's DDE kernels with the interpolation kernel).
 *
 *   win[i][j] = sum_{a,b} D[a][b] * uy[i-a] * ux[j-b],   S = skw + sd - 1
 *
 * Built with gcc -O3 -fopenmp; loaded with ctypes from synth/windows.py.
 */
#include <stdint.h>
#include <complex.h>
#include <string.h>

#define SKW_MAX 32
#define SD_MAX 7

static void build_one(int skw, const double complex *uy, const double complex *ux,
                      int sd, const double complex *D, double complex *w /* S*S */)
{
    const int S = skw + sd - 1;
    if (sd <= 1) {
        const double complex d0 = (sd == 1 && D) ? D[0] : 1.0;
        for (int i = 0; i < skw; ++i) {
            const double complex a = d0 * uy[i];
            for (int j = 0; j < skw; ++j) w[i * S + j] = a * ux[j];
        }
        return;
    }
    double complex outer[SKW_MAX * SKW_MAX];
    for (int i = 0; i < skw; ++i)
        for (int j = 0; j < skw; ++j) outer[i * skw + j] = uy[i] * ux[j];
    for (int k = 0; k < S * S; ++k) w[k] = 0.0;
    for (int a = 0; a < sd; ++a)
        for (int b = 0; b < sd; ++b) {
            const double complex d = D[a * sd + b];
            if (d == 0.0) continue;
            for (int i = 0; i < skw; ++i)
                for (int j = 0; j < skw; ++j)
                    w[(i + a) * S + (j + b)] += d * outer[i * skw + j];
        }
}

/* uy, ux: [M][ldu] complex128; pair_id[m] < 0 means no DDE kernel.
 * pairs: [npairs][SD_MAX*SD_MAX] complex128 (row-major sd x sd), pair_sd[npairs].
 * out_off[m]: element offset of visibility m's window in out.
 * out_kind: 0 = complex128, 1 = complex64. Returns 0, or -1 on bad sizes. */
int synth_windows(int64_t M, const int32_t *skw, const double complex *uy,
                  const double complex *ux, int32_t ldu, const int32_t *pair_id,
                  const double complex *pairs, const int32_t *pair_sd,
                  const int64_t *out_off, void *out, int out_kind)
{
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t m = 0; m < M; ++m) {
        const int k = skw[m];
        const int p = pair_id ? pair_id[m] : -1;
        const int sd = p >= 0 ? pair_sd[p] : 1;
        if (k < 1 || k > SKW_MAX || k > ldu || sd < 1 || sd > SD_MAX) { bad = 1; continue; }
        const double complex *D = p >= 0 ? pairs + (int64_t)p * SD_MAX * SD_MAX : 0;
        double complex w[(SKW_MAX + SD_MAX) * (SKW_MAX + SD_MAX)];
        /* D is stored with a fixed leading dimension; repack to sd x sd. */
        double complex Dp[SD_MAX * SD_MAX];
        if (D)
            for (int a = 0; a < sd; ++a)
                for (int b = 0; b < sd; ++b) Dp[a * sd + b] = D[a * SD_MAX + b];
        build_one(k, uy + m * ldu, ux + m * ldu, D ? sd : 1, D ? Dp : 0, w);
        const int S = k + (D ? sd : 1) - 1;
        if (out_kind == 0) {
            double complex *o = (double complex *)out + out_off[m];
            memcpy(o, w, sizeof(double complex) * S * S);
        } else {
            float complex *o = (float complex *)out + out_off[m];
            for (int t = 0; t < S * S; ++t) o[t] = (float complex)w[t];
        }
    }
    return bad ? -1 : 0;
}
