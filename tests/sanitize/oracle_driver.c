/* Sanitizer driver for the FP64 oracle (test infrastructure): every decoder,
 * stopping rule, decision mode, state dump and op counter, and the unrolled
 * form, on a small random code, with AddressSanitizer and
 * UndefinedBehaviorSanitizer watching.  Exit status 0 when every call
 * returns 0 and the outputs are in range. */
#include <stdio.h>
#include <stdlib.h>

int orc_decode(int algo, int M, int N, const int *row_ptr, const int *col_idx, const float *llr,
               long long B, int max_iter, double lmax, double alpha, int hd_mode, int stop_rule,
               unsigned char *bits_out, int *iters_out, int dump_sweep, long long ndump, double *dumpQ,
               double *dumpR, double *dumpOm, double *dumpLam, long long *opcounts, int nthreads);
int orc_unrolled(int M, int N, const int *row_ptr, const int *col_idx, const int *grp, int G, int T,
                 const double *w, const double *beta, const float *llr, long long B, double lmax,
                 double *out, int nthreads);

static unsigned long long s = 88172645463325252ull;
static double uni(void) { /* xorshift64, [0, 1) */
    s ^= s << 13; s ^= s >> 7; s ^= s << 17;
    return (double)(s >> 11) / 9007199254740992.0;
}

int main(void) {
    enum { M = 24, N = 48, DC = 6, B = 64, T = 12 };
    int row_ptr[M + 1], col_idx[M * DC], grp[N];
    for (int i = 0; i <= M; ++i) row_ptr[i] = i * DC;
    for (int i = 0; i < M; ++i) {       /* DC distinct ascending columns per row */
        int used[N] = {0}, k = 0;
        while (k < DC) {
            const int v = (int)(uni() * N);
            if (!used[v]) { used[v] = 1; ++k; }
        }
        k = 0;
        for (int v = 0; v < N; ++v) if (used[v]) col_idx[i * DC + k++] = v;
    }
    for (int v = 0; v < N; ++v) grp[v] = v % 4;
    float *llr = malloc(sizeof(float) * B * N);
    for (int i = 0; i < B * N; ++i) llr[i] = (float)(4.0 * uni() - 1.0 + (i % 97 == 0 ? 1e4 : 0.0));
    unsigned char *bits = malloc((size_t)B * N);
    int *iters = malloc(sizeof(int) * B);
    double *dq = malloc(sizeof(double) * 8 * N), *dr = malloc(sizeof(double) * 8 * M * DC);
    double *dom = malloc(sizeof(double) * 8 * M), *dl = malloc(sizeof(double) * 8 * N);
    long long *ops = malloc(sizeof(long long) * T * 3);
    int bad = 0;
    for (int algo = 0; algo <= 5; ++algo)
        for (int stop = 0; stop <= 2; ++stop)
            for (int hd = 0; hd <= 1; ++hd) {
                if (stop == 1 && !(algo == 0 || algo == 5)) continue;
                const int rc = orc_decode(algo, M, N, row_ptr, col_idx, llr, B, T, 20.0, 0.75, hd, stop, bits,
                                          iters, 3, 8, dq, dr, dom, dl, algo == 0 ? ops : NULL, 2);
                bad |= rc != 0;
                for (int f = 0; f < B; ++f) bad |= iters[f] < 0 || iters[f] > T;
                for (int i = 0; i < B * N; ++i) bad |= bits[i] > 1;
            }
    /* argument checks and empty batches */
    bad |= orc_decode(0, 0, N, row_ptr, col_idx, llr, B, T, 20.0, 0.75, 0, 0, bits, iters, 0, 0, 0, 0, 0, 0, 0, 1) != -1;
    bad |= orc_decode(0, M, N, row_ptr, col_idx, llr, 0, T, 20.0, 0.75, 0, 0, bits, iters, 0, 0, 0, 0, 0, 0, 0, 1) != 0;
    double w[T * 4], beta[T * 4];
    for (int i = 0; i < T * 4; ++i) { w[i] = 0.8 + 0.4 * uni(); beta[i] = 0.1 * uni(); }
    double *out = malloc(sizeof(double) * B * N);
    bad |= orc_unrolled(M, N, row_ptr, col_idx, grp, 4, T, w, beta, llr, B, 20.0, out, 2) != 0;
    free(llr); free(bits); free(iters); free(dq); free(dr); free(dom); free(dl); free(ops); free(out);
    printf("oracle driver: %s\n", bad ? "FAILED" : "ok");
    return bad;
}
