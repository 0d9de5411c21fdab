/*
 * Progressive edge growth (PEG) construction of an LDPC parity-check matrix
 * (X.-Y. Hu, E. Eleftheriou, D. M. Arnold, "Regular and irregular progressive
 * edge-growth Tanner graphs", IEEE Trans. Inf. Theory 51(1), 2005), the
 * construction the paper uses for its simulated codes (Sec. V).
 *
 * Input generation only: this file knows nothing of the decoders.
 *
 * Variable nodes are placed one at a time in order of non-decreasing degree,
 * and each of their edges is placed before the next variable's.  An edge of
 * variable v goes to the eligible check farthest from v in the graph built so
 * far (distance measured by a breadth-first search from v; a check the
 * search never reaches is farthest of all), ties broken by lowest current
 * check degree, then by a seeded generator.  This is PEG's rule: the first
 * edge goes to a lowest-degree check, and every later one to a check that
 * closes no cycle, or the longest one possible.
 *
 * Eligible: not already a neighbour of v, and below its degree cap.  Check
 * degrees are capped at lo, except that up to n_hi checks may reach lo + 1;
 * when the variable degrees sum to lo * M + n_hi, every check ends with degree
 * lo or lo + 1 and exactly n_hi of them with lo + 1 (a regular code: n_hi = 0).
 */
#include <limits.h>
#include <stdint.h>
#include <stdlib.h>

static uint64_t rng_next(uint64_t *s) {  /* splitmix64 */
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/*
 * N variables of degrees vdeg[N] (any order), M checks.  On success the
 * checks of variable v are vedge[off(v) .. off(v) + vdeg[v]) with
 * off(v) = vdeg[0] + ... + vdeg[v-1], in placement order.
 * Returns 0; -1 on bad arguments; -2 if an edge finds no eligible check.
 */
int peg_build(int N, int M, const int *vdeg, int lo, int n_hi, uint64_t seed, int *vedge) {
    if (N <= 0 || M <= 0 || !vdeg || !vedge || lo < 1 || n_hi < 0 || n_hi > M) return -1;
    int dmax = 0;
    for (int v = 0; v < N; ++v) {
        if (vdeg[v] < 1 || vdeg[v] > M) return -1;
        if (vdeg[v] > dmax) dmax = vdeg[v];
    }
    int *voff = malloc(sizeof(int) * (N + 1));
    int *vcnt = calloc(N, sizeof(int));      /* edges placed per variable */
    int *cdeg = calloc(M, sizeof(int));      /* current check degrees */
    int *cadj = malloc(sizeof(int) * M * (size_t)(lo + 1));  /* check -> variables */
    int *order = malloc(sizeof(int) * N);
    int *clev = malloc(sizeof(int) * M);     /* BFS level of each check, INT_MAX = unreached */
    int *vseen = malloc(sizeof(int) * N);    /* BFS stamp of variables */
    int *vq = malloc(sizeof(int) * N);       /* BFS queue of variables */
    int *cq = malloc(sizeof(int) * M);       /* checks in the order reached */
    int *cand = malloc(sizeof(int) * M);
    voff[0] = 0;
    for (int v = 0; v < N; ++v) voff[v + 1] = voff[v] + vdeg[v];
    int k = 0;
    for (int d = 1; d <= dmax; ++d)
        for (int v = 0; v < N; ++v)
            if (vdeg[v] == d) order[k++] = v;
    for (int v = 0; v < N; ++v) vseen[v] = -1;
    int stamp = 0, hi_left = n_hi, rc = 0;
    uint64_t rs = seed;
    for (int oi = 0; oi < N && rc == 0; ++oi) {
        const int v = order[oi];
        for (int j = 0; j < vdeg[v]; ++j) {
            /* distances from v: level 0 = v's checks, level l + 1 = checks of the
             * variables adjacent to the checks of level l */
            for (int c = 0; c < M; ++c) clev[c] = INT_MAX;
            ++stamp;
            int vh = 0, vt = 0, ch = 0, ct = 0;
            vq[vt++] = v;
            vseen[v] = stamp;
            for (int level = 0;; ++level) {
                const int c0 = ct;
                for (; vh < vt; ++vh) {
                    const int u = vq[vh];
                    for (int i = voff[u]; i < voff[u] + vcnt[u]; ++i) {
                        const int c = vedge[i];
                        if (clev[c] == INT_MAX) {
                            clev[c] = level;
                            cq[ct++] = c;
                        }
                    }
                }
                if (ct == c0) break;
                for (; ch < ct; ++ch) {
                    const int c = cq[ch];
                    for (int i = 0; i < cdeg[c]; ++i) {
                        const int u = cadj[(size_t)c * (lo + 1) + i];
                        if (vseen[u] != stamp) {
                            vseen[u] = stamp;
                            vq[vt++] = u;
                        }
                    }
                }
            }
            /* farthest eligible check, then lowest degree, then at random */
            int blev = -1, bdeg = INT_MAX, nc = 0;
            for (int c = 0; c < M; ++c) {
                if (cdeg[c] > lo || (cdeg[c] == lo && hi_left == 0)) continue;
                int nb = 0;
                for (int i = voff[v]; i < voff[v] + vcnt[v]; ++i) nb |= vedge[i] == c;
                if (nb) continue;
                if (clev[c] > blev || (clev[c] == blev && cdeg[c] < bdeg)) {
                    blev = clev[c];
                    bdeg = cdeg[c];
                    nc = 0;
                }
                if (clev[c] == blev && cdeg[c] == bdeg) cand[nc++] = c;
            }
            if (nc == 0) {
                rc = -2;
                break;
            }
            const int c = cand[rng_next(&rs) % (uint64_t)nc];
            if (cdeg[c] == lo) --hi_left;
            vedge[voff[v] + vcnt[v]++] = c;
            cadj[(size_t)c * (lo + 1) + cdeg[c]++] = v;
        }
    }
    free(voff); free(vcnt); free(cdeg); free(cadj); free(order);
    free(clev); free(vseen); free(vq); free(cq); free(cand);
    return rc;
}
