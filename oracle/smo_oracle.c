/*
 * smo_oracle.c -- plain FP64 CPU reference of the parallel adaptive-shrinking
 * SMO trainer (Narasimhan, Vishnu, Holder, Hoisie, "Fast Support Vector
 * Machines Using Parallel Adaptive Shrinking on Distributed Systems").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or constant generator with
 * the HIP library.
 *
 * Everything is double precision and written in the order of the paper's
 * equations, without blocking, fusion or reordering.  Loops over samples whose
 * iterations are independent (the f update, reconstruction, full recompute,
 * classifier) may run on several OpenMP threads: each sample's own sum is still
 * formed by one thread in the written order, so the results do not depend on
 * the thread count (orc_set_threads; 1 = the plain single-threaded program):
 *
 *   kernel          K(a,b) = exp(-gamma * sum_k (a_k - b_k)^2)       Sec. "Datasets"
 *                   (gamma = 1/(2 sigma^2)); the squared distance is the
 *                   direct difference over the union of the two rows, so
 *                   K(a,a) == 1 exactly
 *   f (gamma_i)     f_i = sum_j alpha_j y_j K_ij - y_i                eq:fcache
 *   index sets      I0..I4 from (alpha, y)                             eq:setinfo
 *   selection       b_up = min f over I0+I1+I2, b_low = max f over     eq:bminmax
 *                   I0+I3+I4, lowest sample index on ties
 *   stop test       continue while b_low - b_up > T (T = 2 eps, or     eq:kktterm
 *                   20 eps in the first shrinking phase)               Alg. 5
 *   pair update     eq:alphaup / eq:rho, clipped to the box             Alg. 2
 *   f update        eq:fup over the active set                          Alg. 2 / 4
 *   shrink rule     eq:shrink, every H iterations                       Alg. 4, Table 3
 *   reconstruction  f of every shrunk sample from the support vectors  Alg. 6
 *   threshold       beta = mean f over I0, else (b_up + b_low)/2        Sec. 3.1
 *   classifier      sum_j alpha_j y_j K(x_j, z) - beta                  eq:classi
 *
 * Readings of passages the paper leaves open (the same list is in the design
 * notes): the eq:fup sum has both terms; rho = -eta and a non-positive eta is
 * replaced by TAU (the ascent step then runs to the box end, Platt's choice
 * for a linear objective); the box ends L, H are Platt's; alpha within
 * DELTA*C of 0 or C is snapped to the bound; the shrink test uses the b_up /
 * b_low that selected the current pair, applied to the updated f; the shrink
 * counter is decremented every iteration and reset to min(|active|, H) after a
 * shrink pass; "random: k" is a fixed count k; the multi-reconstruction
 * variant reconstructs each time the active set meets the tolerance and keeps
 * shrinking at 2 eps; the first selection comes from the initial state
 * (alpha = 0, f = -y), not from the explicit initial pair of Alg. 1.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_TAU 1e-12        /* floor for eta = K_uu + K_ll - 2 K_ul */
#define ORC_DELTA 1e-12      /* snap alpha to a bound within DELTA*C */
#define ORC_PAR_MIN 4096     /* loops over fewer samples stay on one thread */

static int orc_threads = 1;

/* Threads for the per-sample loops (>= 1); returns the count in effect. */
int orc_set_threads(int t) {
    orc_threads = t < 1 ? 1 : t;
    return orc_threads;
}
int orc_get_threads(void) { return orc_threads; }
int orc_max_threads(void) { return omp_get_num_procs(); }

enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_EINVAL = -1, ORC_EONECLASS = -2, ORC_ENONFINITE = -3,
       ORC_ENOMEM = -4 };
enum { ORC_SHRINK_NONE = 0, ORC_SHRINK_SINGLE = 1, ORC_SHRINK_MULTI = 2 };
enum { ORC_KIND_FIXED = 0, ORC_KIND_FRACTION = 1 };

typedef struct {
    int32_t n, d;
    int32_t is_csr;
    const double* x;           /* dense: row-major n x d */
    const int32_t* row_ptr;    /* csr: n+1 entries */
    const int32_t* col;        /* csr: sorted, unique within a row, in [0, d) */
    const double* val;
    const int8_t* y;           /* +1 / -1 (may be NULL for query sets) */
} orc_data;

typedef struct {
    double C, gamma, eps;
    int32_t shrink_mode;       /* ORC_SHRINK_* */
    int32_t shrink_kind;       /* ORC_KIND_* */
    double shrink_param;       /* k for "random: k", fraction for "numsamples" */
    int64_t max_iter;
    int32_t dual_fresh;        /* 1: dual objective from an O(n_sv^2) recompute */
    int32_t pad;
} orc_params;

typedef struct {
    double beta, b_up, b_low, dual_obj;
    int64_t iterations;
    int32_t n_sv, n_bsv, n_recon, status;
    int64_t shrink_passes;
    int64_t shrunk_total;      /* samples removed over all shrink passes */
} orc_result;

typedef struct {
    int64_t cap, count;        /* per-iteration records written: min(iterations, cap) */
    int32_t* i_up;
    int32_t* i_low;
    double* b_up;
    double* b_low;
    double* obj;               /* dual objective from the maintained f (may be NULL) */
    int32_t* n_active;         /* active-set size after the iteration (may be NULL) */
} orc_trace;

/* ------------------------------------------------------------------ kernel */

/* Squared Euclidean distance between row i of A and row j of B, by direct
 * difference (dense) or over the union of the two sorted column lists (CSR). */
static double sqdist(const orc_data* A, int64_t i, const orc_data* B, int64_t j) {
    double s = 0.0;
    if (!A->is_csr && !B->is_csr) {
        const double* a = A->x + i * A->d;
        const double* b = B->x + j * B->d;
        for (int k = 0; k < A->d; ++k) {
            double t = a[k] - b[k];
            s += t * t;
        }
        return s;
    }
    if (A->is_csr && B->is_csr) {
        int32_t p = A->row_ptr[i], pe = A->row_ptr[i + 1];
        int32_t q = B->row_ptr[j], qe = B->row_ptr[j + 1];
        while (p < pe || q < qe) {
            double t;
            if (q >= qe || (p < pe && A->col[p] < B->col[q])) {
                t = A->val[p++];
            } else if (p >= pe || B->col[q] < A->col[p]) {
                t = -B->val[q++];
            } else {
                t = A->val[p++] - B->val[q++];
            }
            s += t * t;
        }
        return s;
    }
    /* mixed: A dense, B csr (or the reverse) */
    const orc_data* D = A->is_csr ? B : A;
    const orc_data* S = A->is_csr ? A : B;
    int64_t di = A->is_csr ? j : i, si = A->is_csr ? i : j;
    const double* a = D->x + di * D->d;
    int32_t q = S->row_ptr[si], qe = S->row_ptr[si + 1];
    for (int k = 0; k < D->d; ++k) {
        double b = 0.0;
        if (q < qe && S->col[q] == k) b = S->val[q++];
        double t = a[k] - b;
        s += t * t;
    }
    return s;
}

double orc_kernel(const orc_data* A, int64_t i, const orc_data* B, int64_t j, double gamma) {
    return exp(-gamma * sqdist(A, i, B, j));
}

/* ------------------------------------------------------------------ index sets (eq:setinfo) */

static int in_up(int8_t y, double a, double C) {   /* I0 u I1 u I2 */
    return (a > 0.0 && a < C) || (y > 0 && a == 0.0) || (y < 0 && a == C);
}
static int in_low(int8_t y, double a, double C) {  /* I0 u I3 u I4 */
    return (a > 0.0 && a < C) || (y > 0 && a == C) || (y < 0 && a == 0.0);
}

int32_t orc_set_id(int8_t y, double a, double C) { /* 0..4 as in eq:setinfo */
    if (a > 0.0 && a < C) return 0;
    if (y > 0) return a == 0.0 ? 1 : 3;
    return a == C ? 2 : 4;
}

/* ------------------------------------------------------------------ selection (eq:bminmax) */

/* S lists sample ids in increasing order; ties keep the first (lowest) id. */
void orc_select(int64_t nS, const int32_t* S, const double* f, const double* alpha, const int8_t* y,
                double C, double* b_up, int32_t* i_up, double* b_low, int32_t* i_low) {
    double bu = INFINITY, bl = -INFINITY;
    int32_t iu = -1, il = -1;
    for (int64_t t = 0; t < nS; ++t) {
        int32_t i = S[t];
        if (in_up(y[i], alpha[i], C) && f[i] < bu) { bu = f[i]; iu = i; }
        if (in_low(y[i], alpha[i], C) && f[i] > bl) { bl = f[i]; il = i; }
    }
    *b_up = bu; *i_up = iu; *b_low = bl; *i_low = il;
}

/* ------------------------------------------------------------------ pair update (eq:alphaup, eq:rho) */

static double snap(double a, double C) {
    if (a < ORC_DELTA * C) return 0.0;
    if (a > C - ORC_DELTA * C) return C;
    return a;
}

/* New (alpha_up, alpha_low) for the pair, from f_up = b_up, f_low = b_low. */
void orc_pair_update(double a_up, double a_low, int8_t y_up, int8_t y_low, double f_up, double f_low,
                     double K_uu, double K_ll, double K_ul, double C, double* new_up, double* new_low) {
    double eta = K_uu + K_ll - 2.0 * K_ul;      /* = -rho */
    if (eta < ORC_TAU) eta = ORC_TAU;
    double s = (double)y_up * (double)y_low;
    double L, H;
    if (s < 0) {
        L = fmax(0.0, a_low - a_up);
        H = fmin(C, C + a_low - a_up);
    } else {
        L = fmax(0.0, a_low + a_up - C);
        H = fmin(C, a_low + a_up);
    }
    double al = a_low + (double)y_low * (f_up - f_low) / eta;
    if (al < L) al = L;
    if (al > H) al = H;
    double au = a_up + s * (a_low - al);
    *new_low = snap(al, C);
    *new_up = snap(au, C);
}

/* ------------------------------------------------------------------ whole-set quantities */

/* f_i = sum_j alpha_j y_j K_ij - y_i for every i (eq:fcache), increasing j. */
void orc_f_full(const orc_data* X, const double* alpha, double gamma, double* f) {
#pragma omp parallel for schedule(dynamic, 64) num_threads(orc_threads) if (X->n >= 64 && orc_threads > 1)
    for (int64_t i = 0; i < X->n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < X->n; ++j)
            if (alpha[j] > 0.0) s += alpha[j] * (double)X->y[j] * orc_kernel(X, i, X, j, gamma);
        f[i] = s - (double)X->y[i];
    }
}

/* Dual objective of eq:lagdual from scratch: sum alpha - 1/2 sum_ij a_i a_j y_i y_j K_ij. */
double orc_dual(const orc_data* X, const double* alpha, double gamma) {
    int64_t m = 0;
    int32_t* sv = (int32_t*)malloc(sizeof(int32_t) * (X->n > 0 ? X->n : 1));
    double lin = 0.0;
    for (int64_t i = 0; i < X->n; ++i)
        if (alpha[i] > 0.0) { sv[m++] = (int32_t)i; lin += alpha[i]; }
    double* g = (double*)malloc(sizeof(double) * (m > 0 ? m : 1));
#pragma omp parallel for schedule(dynamic, 64) num_threads(orc_threads) if (m >= 64 && orc_threads > 1)
    for (int64_t a = 0; a < m; ++a) {
        int32_t i = sv[a];
        double s = 0.0;
        for (int64_t b = 0; b < m; ++b) {
            int32_t j = sv[b];
            s += alpha[j] * (double)X->y[j] * orc_kernel(X, i, X, j, gamma);
        }
        g[a] = s;
    }
    double quad = 0.0;
    for (int64_t a = 0; a < m; ++a) quad += alpha[sv[a]] * (double)X->y[sv[a]] * g[a];
    free(g);
    free(sv);
    return lin - 0.5 * quad;
}

/* Decision values sum_j alpha_j y_j K(x_j, z_q) - beta (eq:classi before sgn). */
void orc_decision(const orc_data* X, const double* alpha, double beta, double gamma, const orc_data* Q,
                  double* out) {
#pragma omp parallel for schedule(dynamic, 16) num_threads(orc_threads) if (Q->n >= 16 && orc_threads > 1)
    for (int64_t q = 0; q < Q->n; ++q) {
        double s = 0.0;
        for (int64_t j = 0; j < X->n; ++j)
            if (alpha[j] > 0.0) s += alpha[j] * (double)X->y[j] * orc_kernel(X, j, Q, q, gamma);
        out[q] = s - beta;
    }
}

/* ------------------------------------------------------------------ input checks */

int orc_validate(const orc_data* X, const orc_params* P) {
    if (!X || !P || X->n < 2 || X->d < 1 || !X->y) return ORC_EINVAL;
    if (!(P->C > 0.0) || !(P->gamma > 0.0) || !(P->eps > 0.0) || !isfinite(P->C) || !isfinite(P->gamma))
        return ORC_EINVAL;
    if (P->shrink_mode < 0 || P->shrink_mode > 2) return ORC_EINVAL;
    if (P->shrink_mode != ORC_SHRINK_NONE && !(P->shrink_param > 0.0)) return ORC_EINVAL;
    int pos = 0, neg = 0;
    for (int64_t i = 0; i < X->n; ++i) {
        if (X->y[i] == 1) pos = 1;
        else if (X->y[i] == -1) neg = 1;
        else return ORC_EINVAL;
    }
    if (X->is_csr) {
        if (X->row_ptr[0] != 0) return ORC_EINVAL;
        for (int64_t i = 0; i < X->n; ++i) {
            if (X->row_ptr[i + 1] < X->row_ptr[i]) return ORC_EINVAL;
            for (int32_t p = X->row_ptr[i]; p < X->row_ptr[i + 1]; ++p) {
                if (X->col[p] < 0 || X->col[p] >= X->d) return ORC_EINVAL;
                if (p > X->row_ptr[i] && X->col[p] <= X->col[p - 1]) return ORC_EINVAL;
                if (!isfinite(X->val[p])) return ORC_ENONFINITE;
            }
        }
    } else {
        for (int64_t k = 0; k < (int64_t)X->n * X->d; ++k)
            if (!isfinite(X->x[k])) return ORC_ENONFINITE;
    }
    if (!pos || !neg) return ORC_EONECLASS;
    return ORC_OK;
}

/* ------------------------------------------------------------------ training driver (Alg. 1, 2, 4, 5, 6) */

/* Alg. 6: f of every sample outside the active set, from the current support vectors. */
static void reconstruct(const orc_data* X, const double* alpha, double gamma, const uint8_t* active_mask,
                        double* f) {
#pragma omp parallel for schedule(dynamic, 64) num_threads(orc_threads) if (X->n >= 64 && orc_threads > 1)
    for (int64_t i = 0; i < X->n; ++i) {
        if (active_mask[i]) continue;
        double s = 0.0;
        for (int64_t j = 0; j < X->n; ++j)
            if (alpha[j] > 0.0) s += alpha[j] * (double)X->y[j] * orc_kernel(X, i, X, j, gamma);
        f[i] = s - (double)X->y[i];
    }
}

static int64_t heuristic_h(const orc_params* P, int64_t n) {
    double h = P->shrink_kind == ORC_KIND_FIXED ? P->shrink_param : ceil(P->shrink_param * (double)n);
    if (h < 1.0) h = 1.0;
    return (int64_t)h;
}

int orc_train(const orc_data* X, const orc_params* P, double* alpha, double* f, orc_result* R,
              orc_trace* T) {
    int rc = orc_validate(X, P);
    if (rc) return rc;
    const int64_t n = X->n;
    const double C = P->C, eps = P->eps;
    int32_t* act = (int32_t*)malloc(sizeof(int32_t) * n);
    int32_t* all = (int32_t*)malloc(sizeof(int32_t) * n);
    uint8_t* mask = (uint8_t*)malloc(n);
    if (!act || !all || !mask) { free(act); free(all); free(mask); return ORC_ENOMEM; }

    /* initial state: alpha = 0, f = -y, every sample active */
    for (int64_t i = 0; i < n; ++i) {
        alpha[i] = 0.0;
        f[i] = -(double)X->y[i];
        act[i] = all[i] = (int32_t)i;
    }
    int64_t n_act = n;
    int shrinking = P->shrink_mode != ORC_SHRINK_NONE;
    double thr = shrinking ? 20.0 * eps : 2.0 * eps;
    const int64_t H = shrinking ? heuristic_h(P, n) : 0;
    int64_t counter = H;
    int64_t iter = 0, passes = 0, shrunk_total = 0;
    int32_t n_recon = 0;
    int status = ORC_OK;
    if (T) T->count = 0;

    double bu, bl;
    int32_t iu, il;
    orc_select(n_act, act, f, alpha, X->y, C, &bu, &iu, &bl, &il);

    for (;;) {
        while (bl - bu > thr) {
            if (iter >= P->max_iter) { status = ORC_NOT_CONVERGED; break; }
            /* pair update (eq:alphaup / eq:rho) */
            double Kuu = orc_kernel(X, iu, X, iu, P->gamma);
            double Kll = orc_kernel(X, il, X, il, P->gamma);
            double Kul = orc_kernel(X, iu, X, il, P->gamma);
            double nu, nl;
            orc_pair_update(alpha[iu], alpha[il], X->y[iu], X->y[il], bu, bl, Kuu, Kll, Kul, C, &nu, &nl);
            double du = nu - alpha[iu], dl = nl - alpha[il];
            double yu = (double)X->y[iu], yl = (double)X->y[il];
            /* f update over the active set (eq:fup) */
#pragma omp parallel for schedule(static) num_threads(orc_threads) if (n_act >= ORC_PAR_MIN && orc_threads > 1)
            for (int64_t t = 0; t < n_act; ++t) {
                int32_t i = act[t];
                f[i] += yu * du * orc_kernel(X, iu, X, i, P->gamma) + yl * dl * orc_kernel(X, il, X, i, P->gamma);
            }
            alpha[iu] = nu;
            alpha[il] = nl;
            /* shrink pass (Alg. 4 with eq:shrink), using the b's that selected this pair */
            if (shrinking) {
                if (--counter == 0) {
                    int64_t m = 0;
                    for (int64_t t = 0; t < n_act; ++t) {
                        int32_t i = act[t];
                        int32_t s = orc_set_id(X->y[i], alpha[i], C);
                        int drop = ((s == 3 || s == 4) && f[i] < bu) || ((s == 1 || s == 2) && f[i] > bl);
                        if (!drop) act[m++] = i;
                    }
                    shrunk_total += n_act - m;
                    n_act = m;
                    ++passes;
                    counter = n_act < H ? n_act : H;
                    if (counter < 1) counter = 1;
                }
            }
            ++iter;
            if (T && T->count < T->cap) {
                int64_t k = T->count++;
                T->i_up[k] = iu;
                T->i_low[k] = il;
                T->b_up[k] = bu;
                T->b_low[k] = bl;
                if (T->n_active) T->n_active[k] = (int32_t)n_act;
                if (T->obj) {
                    double o = 0.0;
                    for (int64_t i = 0; i < n; ++i) o += alpha[i] - 0.5 * alpha[i] * (double)X->y[i] * (f[i] + (double)X->y[i]);
                    T->obj[k] = o;
                }
            }
            orc_select(n_act, act, f, alpha, X->y, C, &bu, &iu, &bl, &il);
        }
        if (!shrinking || status != ORC_OK) break;
        /* the active set meets the tolerance: reconstruct the shrunk samples (Alg. 6) */
        memset(mask, 0, n);
        for (int64_t t = 0; t < n_act; ++t) mask[act[t]] = 1;
        if (n_act < n) reconstruct(X, alpha, P->gamma, mask, f);
        ++n_recon;
        memcpy(act, all, sizeof(int32_t) * n);
        n_act = n;
        orc_select(n_act, act, f, alpha, X->y, C, &bu, &iu, &bl, &il);
        if (bl - bu <= 2.0 * eps) break;
        thr = 2.0 * eps;
        if (P->shrink_mode == ORC_SHRINK_SINGLE) {
            shrinking = 0;                 /* continue on every sample, no more shrinking */
        } else {
            counter = H;                   /* multi: keep shrinking at 2 eps */
        }
    }
    if (n_act < n) {                       /* iteration cap hit while samples were shrunk */
        memset(mask, 0, n);
        for (int64_t t = 0; t < n_act; ++t) mask[act[t]] = 1;
        reconstruct(X, alpha, P->gamma, mask, f);
        ++n_recon;
        n_act = n;
        memcpy(act, all, sizeof(int32_t) * n);
        orc_select(n_act, act, f, alpha, X->y, C, &bu, &iu, &bl, &il);
    }

    /* threshold beta and summary (Sec. 3.1) */
    double sum0 = 0.0;
    int64_t n0 = 0;
    int32_t nsv = 0, nbsv = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (alpha[i] > 0.0) ++nsv;
        if (alpha[i] == C) ++nbsv;
        if (alpha[i] > 0.0 && alpha[i] < C) { sum0 += f[i]; ++n0; }
    }
    if (R) {
        R->beta = n0 ? sum0 / (double)n0 : 0.5 * (bu + bl);
        R->b_up = bu;
        R->b_low = bl;
        if (P->dual_fresh) {
            R->dual_obj = orc_dual(X, alpha, P->gamma);
        } else {
            double o = 0.0;
            for (int64_t i = 0; i < n; ++i) o += alpha[i] - 0.5 * alpha[i] * (double)X->y[i] * (f[i] + (double)X->y[i]);
            R->dual_obj = o;
        }
        R->iterations = iter;
        R->n_sv = nsv;
        R->n_bsv = nbsv;
        R->n_recon = n_recon;
        R->status = status;
        R->shrink_passes = passes;
        R->shrunk_total = shrunk_total;
    }
    free(act);
    free(all);
    free(mask);
    return status;
}
