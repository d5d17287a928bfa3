/*
 * FP64 CPU oracle for non-disjoint group-shuffled BP (NDGSBP) decoding.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the parity authority for the HIP
 * decoder and is used by the tests, the package smoke check and the CPU
 * baseline leg of the benchmark. No product code path may call it.
 * It shares no code, header or table with the HIP library.
 *
 * What it computes (Sec. II-C, "Initialization" and Steps 2-4):
 *   - messages start as L_{m->n} = 0 and L_{n->m} = L_n (the paper is silent
 *     on message initialisation; this is the textbook start);
 *   - for every iteration l = 1..I_max, the CN groups G_1..G_G are visited
 *     in order; for each group:
 *       (a) CN update, eq. (1), for every m in G_g and n in N(m), evaluated
 *           from the VN->CN messages as they stood before the group (all
 *           CNs of a group update in parallel);
 *       (b) VN update, eq. (2), for every n in the union of N(m) over the
 *           group and every m in M(n);
 *   - after the last group: total LLR, eq. (3) (the sum runs over M(n)),
 *     hard decision d_n = 1 iff L_total < 0 (Step 4a) and the syndrome
 *     D H^T over all M checks (Step 4b); with early stop a zero syndrome
 *     ends the decode at iteration l.
 *
 * Eq. (1) is evaluated in sign-magnitude form, which equals
 * 2 atanh(prod tanh(x/2)) exactly in real arithmetic:
 *   B(x_1..x_k) = (prod_i s(x_i)) * phi(clampS(sum_i phi(clampX(|x_i|)))),
 *   s(x) = -1 iff x < 0, phi(x) = log1p(2 / expm1(x)) = -ln tanh(x/2),
 *   clampX and clampS both clamp to [phi(30), 30].
 * The exclusive sum over N(m)\n is a literal loop (no total-minus-own).
 * The clamp is this project's definition; the paper does not specify one.
 *
 * Groups are passed explicitly (CSR over CN ids); window expansion lives in
 * the Python side of the oracle.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define REF_XMAX 30.0

static double ref_phi(double x) { return log1p(2.0 / expm1(x)); }

static double ref_clamp(double a, double lo) {
    if (a < lo) return lo;
    if (a > REF_XMAX) return REF_XMAX;
    return a;
}

/* phi(x), exported for the tests */
double ref_phi_f64(double x) { return ref_phi(x); }

/* B over k inputs (eq. 1 in sign-magnitude form); exported for the tests */
double ref_boxplus(const double* x, int k) {
    const double lo = ref_phi(REF_XMAX);
    double sgn = 1.0, s = 0.0;
    for (int i = 0; i < k; ++i) {
        if (x[i] < 0.0) sgn = -sgn;
        s += ref_phi(ref_clamp(fabs(x[i]), lo));
    }
    return sgn * ref_phi(ref_clamp(s, lo));
}

typedef struct {
    int M, N, E, G;
    const int32_t* row_ptr; /* M+1 */
    const int32_t* col;     /* E   */
    const int32_t* gptr;    /* G+1 */
    const int32_t* gcn;     /* gptr[G] */
    int32_t* vptr;          /* N+1: edges of VN n are vedge[vptr[n]..vptr[n+1]) */
    int32_t* vedge;         /* E   */
    int32_t* ecn;           /* E: the CN of each edge */
    const float* llr;
    int F, max_iter, early_stop;
    double* post;
    uint8_t* hard;
    int32_t* iters;
    uint8_t* syn_ok;
    double* margin; /* F: smallest |total LLR| over VNs in the last two iterations run */
    int nthreads;
    int gper; /* groups per iteration: iteration l uses block (l-1) mod (G / gper) */
    int vertical; /* groups hold VN ids: the vertical group-shuffled schedule */
} ref_job;

typedef struct {
    ref_job* job;
    int tid;
} ref_task;

static void decode_frame(const ref_job* J, int f, double* Lch, double* Lcv, double* Lvc,
                         double* tmp, int32_t* stamp, double* P) {
    const int M = J->M, N = J->N, E = J->E;
    const float* y = J->llr + (size_t)f * N;
    for (int n = 0; n < N; ++n) Lch[n] = (double)y[n];
    for (int e = 0; e < E; ++e) {
        Lcv[e] = 0.0;
        Lvc[e] = Lch[J->col[e]];
    }
    for (int n = 0; n < N; ++n) stamp[n] = -1;
    int used = J->max_iter, ok = 0;
    int visit = 0;
    /* stop margin: the smallest change of total LLRs that could change the
       iteration at which Step 4 stops the frame (see run_job) */
    double margin = INFINITY;
    const int R = J->G / J->gper;
    for (int l = 1; l <= J->max_iter; ++l) {
        const int g0 = ((l - 1) % R) * J->gper;
        for (int g = g0; g < g0 + J->gper; ++g, ++visit) {
            if (J->vertical) {
                /* Vertical group-shuffled BP (the prior-art schedule of Sec. I,
                   VN groups): (a) for every n of the group and m in M(n), the
                   CN->VN message of eq. (1) from the VN->CN messages as they
                   stood before the group; (b) eq. (2) for every n of the
                   group and every m in M(n). */
                for (int q = J->gptr[g]; q < J->gptr[g + 1]; ++q) {
                    const int n = J->gcn[q];
                    for (int a = J->vptr[n]; a < J->vptr[n + 1]; ++a) {
                        const int e = J->vedge[a];
                        const int m = J->ecn[e];
                        const int b = J->row_ptr[m], d = J->row_ptr[m + 1] - b;
                        int k = 0;
                        for (int j = 0; j < d; ++j)
                            if (b + j != e) tmp[k++] = Lvc[b + j];
                        Lcv[e] = ref_boxplus(tmp, k);
                    }
                }
                for (int q = J->gptr[g]; q < J->gptr[g + 1]; ++q) {
                    const int n = J->gcn[q];
                    for (int a = J->vptr[n]; a < J->vptr[n + 1]; ++a) {
                        double s = Lch[n];
                        for (int c = J->vptr[n]; c < J->vptr[n + 1]; ++c)
                            if (c != a) s += Lcv[J->vedge[c]];
                        Lvc[J->vedge[a]] = s;
                    }
                }
                continue;
            }
            /* (a) CN update, eq. (1): Lvc is not written in this phase, so every
               CN of the group reads the pre-group VN->CN messages. */
            for (int q = J->gptr[g]; q < J->gptr[g + 1]; ++q) {
                const int m = J->gcn[q];
                const int b = J->row_ptr[m], d = J->row_ptr[m + 1] - b;
                for (int i = 0; i < d; ++i) {
                    int k = 0;
                    for (int j = 0; j < d; ++j)
                        if (j != i) tmp[k++] = Lvc[b + j];
                    Lcv[b + i] = ref_boxplus(tmp, k);
                }
            }
            /* (b) VN update, eq. (2): every n touched by the group, every m in M(n). */
            for (int q = J->gptr[g]; q < J->gptr[g + 1]; ++q) {
                const int m = J->gcn[q];
                for (int e = J->row_ptr[m]; e < J->row_ptr[m + 1]; ++e) {
                    const int n = J->col[e];
                    if (stamp[n] == visit) continue;
                    stamp[n] = visit;
                    for (int a = J->vptr[n]; a < J->vptr[n + 1]; ++a) {
                        double s = Lch[n];
                        for (int c = J->vptr[n]; c < J->vptr[n + 1]; ++c)
                            if (c != a) s += Lcv[J->vedge[c]];
                        Lvc[J->vedge[a]] = s;
                    }
                }
            }
        }
        /* Step 3, eq. (3): total LLR over M(n) */
        for (int n = 0; n < N; ++n) {
            double s = Lch[n];
            for (int a = J->vptr[n]; a < J->vptr[n + 1]; ++a) s += Lcv[J->vedge[a]];
            P[n] = s;
        }
        /* Step 4: hard decision and syndrome over all M checks. Beside it,
           for the stop margin: with a zero syndrome, the smallest |P| of a
           VN in some check (a flip there would fail a check); otherwise the
           largest, over failing checks, of the smallest |P| in the check (a
           zero syndrome needs a flip in every failing check). */
        ok = 1;
        double firm_fail = 0.0, weakest = INFINITY;
        for (int m = 0; m < M; ++m) {
            int par = 0;
            double low = INFINITY;
            for (int e = J->row_ptr[m]; e < J->row_ptr[m + 1]; ++e) {
                par ^= (P[J->col[e]] < 0.0);
                if (fabs(P[J->col[e]]) < low) low = fabs(P[J->col[e]]);
            }
            if (par) {
                ok = 0;
                if (low > firm_fail) firm_fail = low;
            }
            if (low < weakest) weakest = low;
        }
        const double here = ok ? weakest : firm_fail;
        if (here < margin) margin = here;
        if (J->early_stop && ok) {
            used = l;
            break;
        }
    }
    if (J->post) memcpy(J->post + (size_t)f * N, P, sizeof(double) * N);
    if (J->hard)
        for (int n = 0; n < N; ++n) J->hard[(size_t)f * N + n] = (uint8_t)(P[n] < 0.0);
    if (J->iters) J->iters[f] = used;
    if (J->syn_ok) J->syn_ok[f] = (uint8_t)ok;
    if (J->margin) J->margin[f] = margin;
}

static void* worker(void* arg) {
    ref_task* t = (ref_task*)arg;
    const ref_job* J = t->job;
    int dmax = 1;
    for (int m = 0; m < J->M; ++m) {
        int d = J->row_ptr[m + 1] - J->row_ptr[m];
        if (d > dmax) dmax = d;
    }
    double* Lch = malloc(sizeof(double) * J->N);
    double* P = malloc(sizeof(double) * J->N);
    double* Lcv = malloc(sizeof(double) * (J->E + 1));
    double* Lvc = malloc(sizeof(double) * (J->E + 1));
    double* tmp = malloc(sizeof(double) * dmax);
    int32_t* stamp = malloc(sizeof(int32_t) * J->N);
    if (Lch && P && Lcv && Lvc && tmp && stamp)
        for (int f = t->tid; f < J->F; f += J->nthreads) decode_frame(J, f, Lch, Lcv, Lvc, tmp, stamp, P);
    free(Lch);
    free(P);
    free(Lcv);
    free(Lvc);
    free(tmp);
    free(stamp);
    return NULL;
}

/*
 * Decode F frames (llr: F x N float32, row-major). groups: gptr[G+1], gcn,
 * taken gper at a time: iteration l (from 1) processes groups
 * b*gper .. b*gper + gper - 1 with b = (l - 1) mod (G / gper), i.e. a new
 * grouping every iteration, cycling through G / gper of them (Step 4 returns
 * to the grouping of Step 1); gper = 0 means all G groups every iteration.
 * Outputs (each may be NULL): post F x N doubles, hard F x N bytes,
 * iters F ints, syn_ok F bytes, margin F doubles. margin is a diagnostic
 * for the test bar: the smallest change of the total LLRs of eq. (3) that
 * could move the iteration at which Step 4 stops, i.e. the minimum over the
 * iterations run of: with a zero syndrome, the smallest |P| of a VN in some
 * check; with a nonzero one, the largest over failing checks of the
 * smallest |P| in that check. nthreads <= 0 uses every online CPU.
 * Returns the number of threads used, or a negative value on bad input.
 */
static int run_job(int M, int N, const int32_t* row_ptr, const int32_t* col, int G, const int32_t* gptr,
                   const int32_t* gcn, int gper, int vertical, const float* llr, int F, int max_iter,
                   int early_stop, double* post, uint8_t* hard, int32_t* iters, uint8_t* syn_ok, double* margin,
                   int nthreads) {
    if (M <= 0 || N <= 0 || G <= 0 || F < 0 || max_iter < 1) return -1;
    if (gper == 0) gper = G;
    if (gper < 0 || G % gper) return -1;
    const int E = row_ptr[M];
    for (int m = 0; m < M; ++m)
        if (row_ptr[m + 1] < row_ptr[m]) return -1;
    for (int e = 0; e < E; ++e)
        if (col[e] < 0 || col[e] >= N) return -1;
    for (int q = 0; q < gptr[G]; ++q)
        if (gcn[q] < 0 || gcn[q] >= (vertical ? N : M)) return -1;
    if (F == 0) return 0;
    ref_job J;
    memset(&J, 0, sizeof J);
    J.M = M; J.N = N; J.E = E; J.G = G; J.gper = gper; J.vertical = vertical;
    J.row_ptr = row_ptr; J.col = col; J.gptr = gptr; J.gcn = gcn;
    J.llr = llr; J.F = F; J.max_iter = max_iter; J.early_stop = early_stop;
    J.post = post; J.hard = hard; J.iters = iters; J.syn_ok = syn_ok; J.margin = margin;
    /* VN -> edge adjacency (M(n)), edges listed in increasing edge id */
    J.vptr = calloc((size_t)N + 1, sizeof(int32_t));
    J.vedge = malloc(sizeof(int32_t) * (E + 1));
    J.ecn = malloc(sizeof(int32_t) * (E + 1));
    int32_t* fill = calloc((size_t)N, sizeof(int32_t));
    if (!J.vptr || !J.vedge || !J.ecn || !fill) {
        free(J.vptr); free(J.vedge); free(J.ecn); free(fill);
        return -2;
    }
    for (int m = 0; m < M; ++m)
        for (int e = row_ptr[m]; e < row_ptr[m + 1]; ++e) J.ecn[e] = m;
    for (int e = 0; e < E; ++e) J.vptr[col[e] + 1]++;
    for (int n = 0; n < N; ++n) J.vptr[n + 1] += J.vptr[n];
    for (int e = 0; e < E; ++e) {
        int n = col[e];
        J.vedge[J.vptr[n] + fill[n]++] = e;
    }
    free(fill);
    int T = nthreads > 0 ? nthreads : (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (T < 1) T = 1;
    if (T > F) T = F;
    J.nthreads = T;
    pthread_t* th = malloc(sizeof(pthread_t) * T);
    ref_task* tk = malloc(sizeof(ref_task) * T);
    for (int t = 0; t < T; ++t) {
        tk[t].job = &J;
        tk[t].tid = t;
        pthread_create(&th[t], NULL, worker, &tk[t]);
    }
    for (int t = 0; t < T; ++t) pthread_join(th[t], NULL);
    free(th);
    free(tk);
    free(J.vptr);
    free(J.vedge);
    free(J.ecn);
    return T;
}

int ref_decode_schedule(int M, int N, const int32_t* row_ptr, const int32_t* col, int G, const int32_t* gptr,
                        const int32_t* gcn, int gper, const float* llr, int F, int max_iter, int early_stop,
                        double* post, uint8_t* hard, int32_t* iters, uint8_t* syn_ok, double* margin,
                        int nthreads) {
    return run_job(M, N, row_ptr, col, G, gptr, gcn, gper, 0, llr, F, max_iter, early_stop, post, hard, iters,
                   syn_ok, margin, nthreads);
}

/* Vertical group-shuffled decoding: groups gptr[G+1], gvn over VN ids (each
 * processed as in decode_frame), the same groups every iteration. */
int ref_decode_vertical(int M, int N, const int32_t* row_ptr, const int32_t* col, int G, const int32_t* gptr,
                        const int32_t* gvn, const float* llr, int F, int max_iter, int early_stop, double* post,
                        uint8_t* hard, int32_t* iters, uint8_t* syn_ok, int nthreads) {
    return run_job(M, N, row_ptr, col, G, gptr, gvn, 0, 1, llr, F, max_iter, early_stop, post, hard, iters,
                   syn_ok, NULL, nthreads);
}

/* The same with one grouping for every iteration. */
int ref_decode(int M, int N, const int32_t* row_ptr, const int32_t* col, int G, const int32_t* gptr,
               const int32_t* gcn, const float* llr, int F, int max_iter, int early_stop, double* post,
               uint8_t* hard, int32_t* iters, uint8_t* syn_ok, int nthreads) {
    return ref_decode_schedule(M, N, row_ptr, col, G, gptr, gcn, 0, llr, F, max_iter, early_stop, post, hard,
                               iters, syn_ok, NULL, nthreads);
}
