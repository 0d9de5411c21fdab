/*
 * FP64 CPU oracle for check-belief propagation (CBP) decoding and the
 * belief-propagation schedules it is compared with.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: it is built and used by the tests, the smoke check and the
 * benchmark's CPU baseline.  It shares no code with the GPU library.
 *
 * Reference: W. Guan, L. Liang, "Check-Belief Propagation Decoding of LDPC
 * Codes", IEEE Trans. Commun. (arXiv 2305.05286).
 *
 *   phi(x)   = -log tanh(x/2)                          Sec. II-A, eq. (equ_s2e5)
 *   psi+(x,y)= sgn x sgn y phi(phi|x| + phi|y|)        Sec. IV-B, eq. (equ_s4e6)
 *   psi-(x,y)= sgn x sgn y phi(|phi|x| - phi|y||)      Sec. IV-B, eq. (equ_s4e13);
 *                                                      absolute value per App. A (equ_ae8)
 *   CBP      Sec. IV-C, Steps 1-3 (eqs. equ_s4e15 .. equ_s4e23)
 *   LBP      Sec. II-B (equ_s2e10, equ_s2e12) with the check rule of Sec. II-A (equ_s2e4)
 *   FBP      Sec. II-A (equ_s2e3, equ_s2e4, equ_s2e6, equ_s2e7)
 *   NMS      normalized min-sum check rule (alpha * sign * min), Sec. I / IV-D
 *
 * Readings of the paper that this file fixes (the paper is silent or garbled):
 *   R1  A check-node that has not been updated yet in this decode passes no
 *       message: the B2V output is 0 until the variable has been visited once
 *       (Step 1 sets Omega = +inf only as the seed of the C2B recursion).
 *   R2  The commit of Step 2(1)e stores the B2V output R_new(c_j -> v) into
 *       R(c_j -> v) (the printed index c_i is a typo), and it is stored before
 *       R(c_i -> v) is read, which matters when c_j == c_i (degree-1 column).
 *   R3  V2C magnitudes entering phi are clamped to [a, LMAX], a = phi(LMAX);
 *       check-beliefs and their differences are not clamped.  NMS: |Q| <= LMAX.
 *   R4  Stopping: by default the syndrome H x^T = 0 is tested on [L < 0]
 *       before the first sweep and after every full sweep.  The paper's own
 *       rule (M consecutive check updates with Omega > 0 and no sign flip) is
 *       stop_rule = 1 (CBP only); stop_rule = 2 runs exactly max_iter sweeps.
 *   R5  Hard decision: by default x_v = [Lambda_v < 0] from the V2C phase of
 *       v's last visit in the sweep (Step 3).  hd_mode = 1 uses the flushed
 *       posterior Q_v + psi-(Omega_last(v), Q_v) instead.
 *   R6  Rows are processed in index order, the edges of a row in ascending
 *       column order; sgn(0) = +1; Lambda = 0 decides bit 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_CBP = 0, ORC_LBP = 1, ORC_FBP = 2, ORC_LBP_NMS = 3, ORC_FBP_NMS = 4, ORC_CBP_NMS = 5 };

/* ------------------------------------------------------------------ */
/* scalar functions                                                    */
/* ------------------------------------------------------------------ */

/* phi(x) = -log(tanh(x/2)) = log1p(2/expm1(x)); phi(0) = +inf, phi(+inf) = 0. */
double orc_phi(double x) { return log1p(2.0 / expm1(x)); }

static inline double sgn(double x) { return x >= 0.0 ? 1.0 : -1.0; }

/* phi of a clamped V2C magnitude (reading R3). */
double orc_phiq(double y, double lmax) {
    double a = orc_phi(lmax);
    double m = fabs(y);
    if (m < a) m = a;
    if (m > lmax) m = lmax;
    return orc_phi(m);
}

/* psi+ of eq. (equ_s4e6); x is a check-belief (may be +inf), y a V2C message. */
double orc_psi_plus(double x, double y, double lmax) {
    return sgn(x) * sgn(y) * orc_phi(orc_phi(fabs(x)) + orc_phiq(y, lmax));
}

/* psi- of eq. (equ_s4e13) with the absolute value of App. A. */
double orc_psi_minus(double x, double y, double lmax) {
    return sgn(x) * sgn(y) * orc_phi(fabs(orc_phi(fabs(x)) - orc_phiq(y, lmax)));
}

/* ------------------------------------------------------------------ */
/* graph helpers                                                       */
/* ------------------------------------------------------------------ */

typedef struct {
    int M, N, E;
    const int *row_ptr, *col_idx;
    int *row_of;  /* E: row of each edge */
} graph_t;

static int syndrome_zero(const graph_t *g, const unsigned char *x) {
    for (int i = 0; i < g->M; ++i) {
        int p = 0;
        for (int e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) p ^= x[g->col_idx[e]];
        if (p) return 0;
    }
    return 1;
}

typedef struct {
    int dump_sweep;         /* dump state after this sweep (0 = none) */
    double *Q, *R, *Om, *Lam; /* per-frame dump rows, may be NULL */
    long long *ops;         /* [max_iter][3]: B2V, V2C, C2B per sweep (frame 0 only) */
} dump_t;

/* ------------------------------------------------------------------ */
/* CBP, Sec. IV-C (log-tanh form, and the normalized min-sum form)     */
/* ------------------------------------------------------------------ */

/*
 * Check-belief of the min-sum form (reading of eqs. equ_s4e18xx/equ_s4e21xx):
 * the two smallest clamped |Q| (unscaled) and the product of the signs.
 */
typedef struct { double m1, m2, s; } nms_belief;

static int cbp_frame(const graph_t *g, const float *L, int max_iter, double lmax,
                     double alpha, int hd_mode, int stop_rule, int nms,
                     unsigned char *x, const dump_t *d, double *Q, double *R,
                     double *Om, nms_belief *Ob, int *last) {
    const int M = g->M, N = g->N, E = g->E;
    /* Step 1: latest V2C = channel LLR (equ_s4e15), Omega = inf (equ_s4e16), R = 0 (equ_s4e17) */
    for (int v = 0; v < N; ++v) { Q[v] = (double)L[v]; last[v] = -1; x[v] = L[v] < 0.0f; }
    for (int e = 0; e < E; ++e) R[e] = 0.0;
    for (int i = 0; i < M; ++i) { Om[i] = INFINITY; Ob[i].m1 = Ob[i].m2 = INFINITY; Ob[i].s = 1.0; }
    if (stop_rule == 0 && syndrome_zero(g, x)) return 0;
    long long run = 0; /* consecutive good check updates (stop_rule 1) */
    long long rows_done = 0;
    for (int t = 1; t <= max_iter; ++t) {
        long long *ops = (d && d->ops) ? d->ops + 3 * (t - 1) : NULL;
        for (int i = 0; i < M; ++i) {           /* Step 2: check-nodes in order */
            double w = INFINITY;                 /* Omega^(-1) = inf */
            nms_belief wb = {INFINITY, INFINITY, 1.0};
            int flip = 0;
            for (int e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
                int v = g->col_idx[e];
                int ej = last[v];                /* a) latest updated neighbour c_j */
                double Rn = 0.0;
                if (ej >= 0) {                   /* b) B2V, eq. (equ_s4e18) */
                    int j = g->row_of[ej];
                    if (!nms) {
                        Rn = orc_psi_minus(Om[j], Q[v], lmax);
                    } else {
                        double aq = fabs(Q[v]);
                        if (aq > lmax) aq = lmax;
                        double mag = (aq == Ob[j].m1) ? Ob[j].m2 : Ob[j].m1;
                        Rn = Ob[j].s * sgn(Q[v]) * alpha * mag;
                    }
                    R[ej] = Rn;                  /* e) commit R(c_j -> v), reading R2 */
                    if (ops) ops[0]++;
                }
                double lam = Q[v] + Rn;          /* eq. (equ_s4e20) */
                unsigned char nx = lam < 0.0;    /* eq. (equ_s2e7) */
                if (nx != x[v]) flip = 1;
                x[v] = nx;
                double Qn = lam - R[e];          /* c) V2C, eq. (equ_s4e19) */
                if (ops) ops[1]++;
                if (!nms) {
                    w = orc_psi_plus(w, Qn, lmax); /* d) C2B, eq. (equ_s4e21) */
                } else {
                    double aq = fabs(Qn);
                    if (aq > lmax) aq = lmax;
                    if (aq < wb.m1) { wb.m2 = wb.m1; wb.m1 = aq; }
                    else if (aq < wb.m2) { wb.m2 = aq; }
                    wb.s *= sgn(Qn);
                }
                if (ops) ops[2]++;
                Q[v] = Qn;                       /* e) commit, eq. (equ_s4e22) */
                last[v] = e;
            }
            Om[i] = w;                           /* (2) eq. (equ_s4e23) */
            Ob[i] = wb;
            ++rows_done;
            if (stop_rule == 1) {
                double om = nms ? wb.s : w;
                if (om > 0.0 && !flip) ++run; else run = 0;
                if (run >= M) {
                    if (hd_mode == 1) goto flush_and_stop;
                    return (int)((rows_done + M - 1) / M);
                }
            }
        }
        if (hd_mode == 1) {
            for (int v = 0; v < N; ++v) {
                double Rn = 0.0;
                if (last[v] >= 0) {
                    int j = g->row_of[last[v]];
                    if (!nms) Rn = orc_psi_minus(Om[j], Q[v], lmax);
                    else {
                        double aq = fabs(Q[v]);
                        if (aq > lmax) aq = lmax;
                        Rn = Ob[j].s * sgn(Q[v]) * alpha * ((aq == Ob[j].m1) ? Ob[j].m2 : Ob[j].m1);
                    }
                }
                x[v] = (Q[v] + Rn) < 0.0;
            }
        }
        if (d && d->dump_sweep == t) {
            if (d->Q) memcpy(d->Q, Q, sizeof(double) * N);
            if (d->R) memcpy(d->R, R, sizeof(double) * E);
            if (d->Om) {
                if (!nms) memcpy(d->Om, Om, sizeof(double) * M);
                else for (int i = 0; i < M; ++i) d->Om[i] = Ob[i].s * alpha * Ob[i].m1;
            }
            if (d->Lam) {
                for (int v = 0; v < N; ++v) {
                    double Rn = 0.0;
                    if (last[v] >= 0) {
                        int j = g->row_of[last[v]];
                        if (!nms) Rn = orc_psi_minus(Om[j], Q[v], lmax);
                        else {
                            double aq = fabs(Q[v]);
                            if (aq > lmax) aq = lmax;
                            Rn = Ob[j].s * sgn(Q[v]) * alpha * ((aq == Ob[j].m1) ? Ob[j].m2 : Ob[j].m1);
                        }
                    }
                    d->Lam[v] = Q[v] + Rn;
                }
            }
        }
        if (stop_rule == 0 && syndrome_zero(g, x)) return t;
    }
    return max_iter;
flush_and_stop:
    for (int v = 0; v < N; ++v) {
        double Rn = 0.0;
        if (last[v] >= 0) {
            int j = g->row_of[last[v]];
            if (!nms) Rn = orc_psi_minus(Om[j], Q[v], lmax);
            else {
                double aq = fabs(Q[v]);
                if (aq > lmax) aq = lmax;
                Rn = Ob[j].s * sgn(Q[v]) * alpha * ((aq == Ob[j].m1) ? Ob[j].m2 : Ob[j].m1);
            }
        }
        x[v] = (Q[v] + Rn) < 0.0;
    }
    return (int)((rows_done + M - 1) / M);
}

/* ------------------------------------------------------------------ */
/* Check-node rule shared by the LBP/FBP references (Sec. II-A)        */
/* ------------------------------------------------------------------ */

/* C2V of eq. (equ_s2e4) for every edge of one row, computed directly from the
 * other edges (no exclusion trick), or its normalized min-sum counterpart. */
static void check_rule(int deg, const double *q, double *out, int nms, double alpha, double lmax) {
    for (int a = 0; a < deg; ++a) {
        double s = 1.0;
        if (!nms) {
            double sum = 0.0;
            for (int b = 0; b < deg; ++b) {
                if (b == a) continue;
                s *= sgn(q[b]);
                sum += orc_phiq(q[b], lmax);
            }
            out[a] = s * orc_phi(sum);
        } else {
            double mn = INFINITY;
            for (int b = 0; b < deg; ++b) {
                if (b == a) continue;
                s *= sgn(q[b]);
                double aq = fabs(q[b]);
                if (aq > lmax) aq = lmax;
                if (aq < mn) mn = aq;
            }
            out[a] = s * alpha * mn;
        }
    }
}

/* Layered BP, Sec. II-B: Q = Lambda - R (equ_s2e10), Lambda = Q + R_new (equ_s2e12). */
static int lbp_frame(const graph_t *g, const float *L, int max_iter, double lmax, double alpha,
                     int nms, int stop_rule, unsigned char *x, const dump_t *d, double *Lam, double *R,
                     double *q, double *rn) {
    const int M = g->M, N = g->N, E = g->E;
    for (int v = 0; v < N; ++v) { Lam[v] = (double)L[v]; x[v] = L[v] < 0.0f; }
    for (int e = 0; e < E; ++e) R[e] = 0.0;
    if (stop_rule != 2 && syndrome_zero(g, x)) return 0;
    for (int t = 1; t <= max_iter; ++t) {
        for (int i = 0; i < M; ++i) {
            int b0 = g->row_ptr[i], deg = g->row_ptr[i + 1] - b0;
            for (int k = 0; k < deg; ++k) q[k] = Lam[g->col_idx[b0 + k]] - R[b0 + k];
            check_rule(deg, q, rn, nms, alpha, lmax);
            for (int k = 0; k < deg; ++k) {
                Lam[g->col_idx[b0 + k]] = q[k] + rn[k];
                R[b0 + k] = rn[k];
            }
        }
        for (int v = 0; v < N; ++v) x[v] = Lam[v] < 0.0;
        if (d && d->dump_sweep == t) {
            if (d->Lam) memcpy(d->Lam, Lam, sizeof(double) * N);
            if (d->R) memcpy(d->R, R, sizeof(double) * E);
        }
        if (stop_rule != 2 && syndrome_zero(g, x)) return t;
    }
    return max_iter;
}

/* Flooding BP, Sec. II-A: all V2C (equ_s2e3), then all C2V (equ_s2e4),
 * posterior (equ_s2e6) and hard decision (equ_s2e7). */
static int fbp_frame(const graph_t *g, const float *L, int max_iter, double lmax, double alpha,
                     int nms, int stop_rule, unsigned char *x, const dump_t *d, double *Lam, double *R,
                     double *q, double *rn, double *qall) {
    const int M = g->M, N = g->N, E = g->E;
    for (int v = 0; v < N; ++v) { Lam[v] = (double)L[v]; x[v] = L[v] < 0.0f; }
    for (int e = 0; e < E; ++e) R[e] = 0.0;
    if (stop_rule != 2 && syndrome_zero(g, x)) return 0;
    for (int t = 1; t <= max_iter; ++t) {
        for (int e = 0; e < E; ++e) qall[e] = Lam[g->col_idx[e]] - R[e];
        for (int i = 0; i < M; ++i) {
            int b0 = g->row_ptr[i], deg = g->row_ptr[i + 1] - b0;
            for (int k = 0; k < deg; ++k) q[k] = qall[b0 + k];
            check_rule(deg, q, rn, nms, alpha, lmax);
            for (int k = 0; k < deg; ++k) R[b0 + k] = rn[k];
        }
        for (int v = 0; v < N; ++v) Lam[v] = (double)L[v];
        for (int e = 0; e < E; ++e) Lam[g->col_idx[e]] += R[e];
        for (int v = 0; v < N; ++v) x[v] = Lam[v] < 0.0;
        if (d && d->dump_sweep == t) {
            if (d->Lam) memcpy(d->Lam, Lam, sizeof(double) * N);
            if (d->R) memcpy(d->R, R, sizeof(double) * E);
        }
        if (stop_rule != 2 && syndrome_zero(g, x)) return t;
    }
    return max_iter;
}

/* ------------------------------------------------------------------ */
/* batch entry point                                                   */
/* ------------------------------------------------------------------ */

/*
 * Decode B frames.  llr: float32 [B][N]; bits_out: uint8 [B][N]; iters_out: int32 [B].
 * Dumps (optional, may be NULL): state after sweep `dump_sweep` of the first
 * `ndump` frames, row-major [ndump][N] (Q, Lam), [ndump][E] (R), [ndump][M] (Om).
 * Unwritten dump rows (frame stopped earlier) are left untouched.
 * opcounts (optional): [max_iter][3] per-sweep B2V/V2C/C2B counts of frame 0 (CBP only).
 * Returns 0, or -1 on bad arguments.
 */
int orc_decode(int algo, int M, int N, const int *row_ptr, const int *col_idx,
               const float *llr, long long B, int max_iter, double lmax, double alpha,
               int hd_mode, int stop_rule, unsigned char *bits_out, int *iters_out,
               int dump_sweep, long long ndump, double *dumpQ, double *dumpR, double *dumpOm,
               double *dumpLam, long long *opcounts, int nthreads) {
    if (M <= 0 || N <= 0 || !row_ptr || !col_idx || B < 0 || max_iter < 0) return -1;
    if (B == 0) return 0;
    if (!llr || !bits_out || !iters_out) return -1;
    graph_t g;
    g.M = M; g.N = N; g.E = row_ptr[M]; g.row_ptr = row_ptr; g.col_idx = col_idx;
    g.row_of = (int *)malloc(sizeof(int) * (size_t)(g.E > 0 ? g.E : 1));
    int maxdeg = 1;
    for (int i = 0; i < M; ++i) {
        int dg = row_ptr[i + 1] - row_ptr[i];
        if (dg > maxdeg) maxdeg = dg;
        for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) g.row_of[e] = i;
    }
    if (opcounts) memset(opcounts, 0, sizeof(long long) * 3 * (size_t)max_iter);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        double *A = (double *)malloc(sizeof(double) * (size_t)N);
        double *R = (double *)malloc(sizeof(double) * (size_t)g.E);
        double *Om = (double *)malloc(sizeof(double) * (size_t)M);
        nms_belief *Ob = (nms_belief *)malloc(sizeof(nms_belief) * (size_t)M);
        double *qall = (double *)malloc(sizeof(double) * (size_t)g.E);
        double *q = (double *)malloc(sizeof(double) * (size_t)maxdeg);
        double *rn = (double *)malloc(sizeof(double) * (size_t)maxdeg);
        int *last = (int *)malloc(sizeof(int) * (size_t)N);
#pragma omp for schedule(dynamic, 8)
        for (long long f = 0; f < B; ++f) {
            dump_t dd, *dp = NULL;
            if (f < ndump && dump_sweep > 0) {
                dd.dump_sweep = dump_sweep;
                dd.Q = dumpQ ? dumpQ + f * (long long)N : NULL;
                dd.R = dumpR ? dumpR + f * (long long)g.E : NULL;
                dd.Om = dumpOm ? dumpOm + f * (long long)M : NULL;
                dd.Lam = dumpLam ? dumpLam + f * (long long)N : NULL;
                dd.ops = NULL;
                dp = &dd;
            }
            if (f == 0 && opcounts) {
                if (!dp) { dd.dump_sweep = 0; dd.Q = dd.R = dd.Om = dd.Lam = NULL; dp = &dd; }
                dd.ops = opcounts;
            }
            const float *L = llr + f * (long long)N;
            unsigned char *x = bits_out + f * (long long)N;
            int it;
            switch (algo) {
            case ORC_CBP: it = cbp_frame(&g, L, max_iter, lmax, alpha, hd_mode, stop_rule, 0, x, dp, A, R, Om, Ob, last); break;
            case ORC_CBP_NMS: it = cbp_frame(&g, L, max_iter, lmax, alpha, hd_mode, stop_rule, 1, x, dp, A, R, Om, Ob, last); break;
            case ORC_LBP: it = lbp_frame(&g, L, max_iter, lmax, alpha, 0, stop_rule, x, dp, A, R, q, rn); break;
            case ORC_LBP_NMS: it = lbp_frame(&g, L, max_iter, lmax, alpha, 1, stop_rule, x, dp, A, R, q, rn); break;
            case ORC_FBP: it = fbp_frame(&g, L, max_iter, lmax, alpha, 0, stop_rule, x, dp, A, R, q, rn, qall); break;
            case ORC_FBP_NMS: it = fbp_frame(&g, L, max_iter, lmax, alpha, 1, stop_rule, x, dp, A, R, q, rn, qall); break;
            default: it = -1;
            }
            iters_out[f] = it;
        }
        free(A); free(R); free(Om); free(Ob); free(qall); free(q); free(rn); free(last);
    }
    free(g.row_of);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Unrolled CBP with learnable B2V weights                             */
/* ------------------------------------------------------------------ */

/*
 * T sweeps of CBP (Sec. IV-C, rows in order, no stopping test) in which the
 * B2V output R_new(c_j -> v) of eq. (equ_s4e18) is replaced, in sweep t, by
 *     sgn(R_new) * max(w[t][grp[v]] * |R_new| - beta[t][grp[v]], 0)
 * before it is committed (equ_s4e22) and added to Q_v (equ_s4e20); grp[v] is
 * the variable's weight group (the base block-column of a QC code).  w = 1,
 * beta = 0 is plain CBP.  Output: o_v = Q_v plus the same weighted B2V from
 * v's latest check with the weights of the last sweep, the soft value whose
 * sign is the flushed hard decision (hd_mode = 1).
 */
static void cbp_unrolled_frame(const graph_t *g, const float *L, int T, const int *grp, int G,
                               const double *w, const double *beta, double lmax, double *out,
                               double *Q, double *R, double *Om, int *last) {
    const int M = g->M, N = g->N, E = g->E;
    for (int v = 0; v < N; ++v) { Q[v] = (double)L[v]; last[v] = -1; }
    for (int e = 0; e < E; ++e) R[e] = 0.0;
    for (int i = 0; i < M; ++i) Om[i] = INFINITY;
    for (int t = 0; t < T; ++t) {
        for (int i = 0; i < M; ++i) {
            double om = INFINITY;
            for (int e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
                int v = g->col_idx[e];
                int ej = last[v];
                double Rn = 0.0;
                if (ej >= 0) {
                    double r = orc_psi_minus(Om[g->row_of[ej]], Q[v], lmax);
                    int k = t * G + grp[v];
                    double mag = w[k] * fabs(r) - beta[k];
                    Rn = sgn(r) * (mag > 0.0 ? mag : 0.0);
                    R[ej] = Rn;
                }
                double Qn = Q[v] + Rn - R[e];
                om = orc_psi_plus(om, Qn, lmax);
                Q[v] = Qn;
                last[v] = e;
            }
            Om[i] = om;
        }
    }
    for (int v = 0; v < N; ++v) {
        double Rn = 0.0;
        if (last[v] >= 0) {
            double r = orc_psi_minus(Om[g->row_of[last[v]]], Q[v], lmax);
            int k = (T - 1) * G + grp[v];
            double mag = w[k] * fabs(r) - beta[k];
            Rn = sgn(r) * (mag > 0.0 ? mag : 0.0);
        }
        out[v] = Q[v] + Rn;
    }
}

/*
 * Unrolled weighted CBP on B frames.  grp: int32 [N] in [0, G); w, beta:
 * float64 [T][G]; llr float32 [B][N]; out float64 [B][N].  Returns 0, or -1
 * on bad arguments.
 */
int orc_unrolled(int M, int N, const int *row_ptr, const int *col_idx, const int *grp, int G,
                 int T, const double *w, const double *beta, const float *llr, long long B,
                 double lmax, double *out, int nthreads) {
    if (M <= 0 || N <= 0 || !row_ptr || !col_idx || !grp || G <= 0 || T <= 0 || !w || !beta || B < 0)
        return -1;
    if (B == 0) return 0;
    if (!llr || !out) return -1;
    for (int v = 0; v < N; ++v)
        if (grp[v] < 0 || grp[v] >= G) return -1;
    graph_t g;
    g.M = M; g.N = N; g.E = row_ptr[M]; g.row_ptr = row_ptr; g.col_idx = col_idx;
    g.row_of = (int *)malloc(sizeof(int) * (size_t)(g.E > 0 ? g.E : 1));
    for (int i = 0; i < M; ++i)
        for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) g.row_of[e] = i;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        double *Q = (double *)malloc(sizeof(double) * (size_t)N);
        double *R = (double *)malloc(sizeof(double) * (size_t)(g.E > 0 ? g.E : 1));
        double *Om = (double *)malloc(sizeof(double) * (size_t)M);
        int *last = (int *)malloc(sizeof(int) * (size_t)N);
#pragma omp for schedule(dynamic, 4)
        for (long long f = 0; f < B; ++f)
            cbp_unrolled_frame(&g, llr + f * (long long)N, T, grp, G, w, beta, lmax,
                               out + f * (long long)N, Q, R, Om, last);
        free(Q); free(R); free(Om); free(last);
    }
    free(g.row_of);
    return 0;
}

/* Number of OpenMP threads a parallel region would use (1 without OpenMP). */
int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
