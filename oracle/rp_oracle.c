/*
 * rp_oracle.c -- plain, single-threaded FP64 CPU reference for reachability
 * probabilities of a discrete-time Markov chain (Cormie-Bowins, "A Comparison
 * of Sequential and GPU Implementations of Iterative Methods to Compute
 * Reachability Probabilities", GRAPHITE 2012).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  It shares no code, header, table or helper with the GPU
 * path and must never be linked into it.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.
 *
 * Everything here is deliberately naive: one thread, FP64 throughout, sums
 * taken left to right in storage order, no blocking or fusion beyond what the
 * paper's equations and algorithms state.
 *
 * Conventions
 *   A chain is given in compressed row storage (Section 4): rp[n+1], col[nnz],
 *   val[nnz].  Inside a row the columns are strictly ascending.
 *   Class codes: 0 = S_{=0}, 1 = S_{=1}, 2 = S_? (Section 2.2).
 *   The reduced system over S_? (Section 2.3) is kept as
 *       d[i]      = 1 - P(i,i)              (diagonal of I - A)
 *       A_off     = P restricted to S_? x S_?, diagonal removed (CSR)
 *       b[i]      = P(i, S_{=1})
 *   so that (I - A) x = b reads  d[i] x[i] - sum_{j != i} A_off(i,j) x[j] = b[i].
 *
 * Parity pins: every function below is checked in tests/ against the worked
 * example of Section 2, closed forms, brute force or LAPACK (see the test
 * files).  None is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_BAD_CHAIN 1
#define ORC_NOT_CONVERGED 2
#define ORC_BREAKDOWN 3
#define ORC_SINGULAR 4
#define ORC_NOMEM 5

/* ------------------------------------------------------------------------ */
/* Input validation (Section 2: P maps S x S to [0,1] and every row of P sums
 * to one).  Returns -1 when the chain is well formed, otherwise the first bad
 * row (or n when rp itself is malformed).  *reason receives a code:
 *   1 row_ptr not monotone / wrong ends, 2 column out of range,
 *   3 columns not strictly ascending, 4 value not finite or outside [0,1],
 *   5 row sum differs from 1 by more than tol*max(1,deg),
 *   6 column outside the row's own instance block.                          */
int64_t orc_validate(int64_t n, int64_t nnz, const int32_t *rp,
                     const int32_t *col, const double *val,
                     int64_t ninst, const int64_t *inst_off, double tol,
                     int32_t *reason)
{
    *reason = 0;
    if (rp[0] != 0 || (int64_t)rp[n] != nnz) { *reason = 1; return n; }
    int64_t inst = 0;
    for (int64_t i = 0; i < n; i++) {
        while (inst + 1 < ninst && i >= inst_off[inst + 1]) inst++;
        int64_t lo = inst_off[inst], hi = inst_off[inst + 1];
        if (rp[i + 1] < rp[i]) { *reason = 1; return i; }
        double sum = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
            if (col[k] < 0 || col[k] >= n) { *reason = 2; return i; }
            if (col[k] < lo || col[k] >= hi) { *reason = 6; return i; }
            if (k > rp[i] && col[k] <= col[k - 1]) { *reason = 3; return i; }
            if (!(val[k] >= 0.0 && val[k] <= 1.0)) { *reason = 4; return i; }
            sum += val[k];
        }
        int64_t deg = rp[i + 1] - rp[i];
        double allow = tol * (deg > 1 ? (double)deg : 1.0);
        if (!(fabs(sum - 1.0) <= allow)) { *reason = 5; return i; }
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Backward search over the underlying digraph (Section 2.2): there is an edge
 * s -> s' exactly when P(s,s') > 0.  Starting from the states flagged in
 * `seed`, mark every state that can reach a seed state.  States flagged in
 * `blocked` are never marked unless they are seeds (they stop the search).
 * Plain FIFO breadth-first search on an explicitly built reverse adjacency. */
static int backward_reach(int64_t n, const int32_t *rp, const int32_t *col,
                          const double *val, const uint8_t *seed,
                          const uint8_t *blocked, uint8_t *mark)
{
    int64_t nnz = rp[n];
    int64_t *cnt = calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *src = malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *queue = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!cnt || !src || !fill || !queue) {
        free(cnt); free(src); free(fill); free(queue);
        return ORC_NOMEM;
    }
    /* reverse adjacency: for each target t, the list of sources s with P(s,t)>0 */
    for (int64_t s = 0; s < n; s++)
        for (int64_t k = rp[s]; k < rp[s + 1]; k++)
            if (val[k] > 0.0) cnt[col[k] + 1]++;
    for (int64_t t = 0; t < n; t++) cnt[t + 1] += cnt[t];
    for (int64_t t = 0; t < n; t++) fill[t] = cnt[t];
    for (int64_t s = 0; s < n; s++)
        for (int64_t k = rp[s]; k < rp[s + 1]; k++)
            if (val[k] > 0.0) src[fill[col[k]]++] = s;

    int64_t head = 0, tail = 0;
    for (int64_t s = 0; s < n; s++) {
        mark[s] = seed[s] ? 1 : 0;
        if (seed[s]) queue[tail++] = s;
    }
    while (head < tail) {
        int64_t t = queue[head++];
        for (int64_t k = cnt[t]; k < cnt[t + 1]; k++) {
            int64_t s = src[k];
            if (!mark[s] && !(blocked && blocked[s])) {
                mark[s] = 1;
                queue[tail++] = s;
            }
        }
    }
    free(cnt); free(src); free(fill); free(queue);
    return ORC_OK;
}

/* Partition S into S_{=0}, S_{=1}, S_? (Section 2.2).
 *   S_{=0}: complement of the states that can reach GS (GS included).
 *   S_{=1}: complement of the states that can reach S_{=0}; goal states are
 *           absorbing for "eventually GS", so the second search never passes
 *           through a goal state.
 *   S_?   : the rest.
 * With prob0_only set, S_{=1} is taken to be GS itself (only the first search
 * is done); the reduced system then has b = P(s, GS), as Section 2.3 writes it. */
int orc_partition(int64_t n, const int32_t *rp, const int32_t *col,
                  const double *val, const uint8_t *goal, int prob0_only,
                  uint8_t *cls)
{
    uint8_t *reach_goal = malloc((size_t)(n > 0 ? n : 1));
    uint8_t *s0 = malloc((size_t)(n > 0 ? n : 1));
    uint8_t *reach_s0 = malloc((size_t)(n > 0 ? n : 1));
    if (!reach_goal || !s0 || !reach_s0) {
        free(reach_goal); free(s0); free(reach_s0);
        return ORC_NOMEM;
    }
    int rc = backward_reach(n, rp, col, val, goal, NULL, reach_goal);
    if (rc == ORC_OK) {
        for (int64_t s = 0; s < n; s++) s0[s] = reach_goal[s] ? 0 : 1;
        if (prob0_only) {
            for (int64_t s = 0; s < n; s++)
                cls[s] = s0[s] ? 0 : (goal[s] ? 1 : 2);
        } else {
            rc = backward_reach(n, rp, col, val, s0, goal, reach_s0);
            if (rc == ORC_OK)
                for (int64_t s = 0; s < n; s++)
                    cls[s] = s0[s] ? 0 : (reach_s0[s] ? 2 : 1);
        }
    }
    free(reach_goal); free(s0); free(reach_s0);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Reduced system over S_? (Section 2.3).  States of S_? are numbered in
 * ascending state order (map[s] = reduced index or -1).  For each reduced row,
 * walking P's row in storage order: the diagonal gives d = 1 - P(i,i); an
 * entry into S_? (other than the diagonal) is copied into A_off; an entry into
 * S_{=1} is added to b; an entry into S_{=0} is dropped.  Zero-valued stored
 * entries are not edges and are dropped.
 * Output arrays must hold n (map), n+1 (arp), nnz (acol/aval), n (d, b). */
int orc_assemble(int64_t n, const int32_t *rp, const int32_t *col,
                 const double *val, const uint8_t *cls, int64_t *map,
                 int64_t *nq_out, int64_t *arp, int64_t *acol, double *aval,
                 double *d, double *b, int64_t *z_out)
{
    int64_t nq = 0;
    for (int64_t s = 0; s < n; s++) map[s] = (cls[s] == 2) ? nq++ : -1;
    int64_t z = 0;
    arp[0] = 0;
    for (int64_t s = 0; s < n; s++) {
        if (cls[s] != 2) continue;
        int64_t i = map[s];
        double pii = 0.0, bi = 0.0;
        for (int64_t k = rp[s]; k < rp[s + 1]; k++) {
            int64_t t = col[k];
            if (t == s) { pii = val[k]; continue; }
            if (!(val[k] > 0.0)) continue;
            if (cls[t] == 2) { acol[z] = map[t]; aval[z] = val[k]; z++; }
            else if (cls[t] == 1) bi += val[k];
        }
        d[i] = 1.0 - pii;
        b[i] = bi;
        arp[i + 1] = z;
    }
    *nq_out = nq;
    *z_out = z;
    return ORC_OK;
}

/* Plain transpose of the off-diagonal part (used for the adjoint system). The
 * entries of each transposed row appear in ascending original-row order. */
int orc_transpose(int64_t nq, const int64_t *arp, const int64_t *acol,
                  const double *aval, int64_t *trp, int64_t *tcol,
                  double *tval)
{
    int64_t z = arp[nq];
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(nq > 0 ? nq : 1));
    if (!fill) return ORC_NOMEM;
    for (int64_t i = 0; i <= nq; i++) trp[i] = 0;
    for (int64_t k = 0; k < z; k++) trp[acol[k] + 1]++;
    for (int64_t i = 0; i < nq; i++) trp[i + 1] += trp[i];
    for (int64_t i = 0; i < nq; i++) fill[i] = trp[i];
    for (int64_t i = 0; i < nq; i++)
        for (int64_t k = arp[i]; k < arp[i + 1]; k++) {
            int64_t j = acol[k];
            tcol[fill[j]] = i;
            tval[fill[j]] = aval[k];
            fill[j]++;
        }
    free(fill);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* y = (I - A) u, i.e.  y_i = d_i u_i - sum_{j != i} A_off(i,j) u_j. */
static void apply_m(int64_t nq, const int64_t *arp, const int64_t *acol,
                    const double *aval, const double *d, const double *u,
                    double *y)
{
    for (int64_t i = 0; i < nq; i++) {
        double acc = 0.0;
        for (int64_t k = arp[i]; k < arp[i + 1]; k++) acc += aval[k] * u[acol[k]];
        y[i] = d[i] * u[i] - acc;
    }
}

static double dot(int64_t nq, const double *u, const double *v)
{
    double acc = 0.0;
    for (int64_t i = 0; i < nq; i++) acc += u[i] * v[i];
    return acc;
}

static double norm_inf(int64_t nq, const double *u)
{
    double m = 0.0;
    for (int64_t i = 0; i < nq; i++) {
        double a = fabs(u[i]);
        if (a > m || a != a) m = a;
    }
    return m;
}

/* r = b - (I - A) x, returned together with max_i |r_i|. */
double orc_residual(int64_t nq, const int64_t *arp, const int64_t *acol,
                    const double *aval, const double *d, const double *b,
                    const double *x, double *r)
{
    apply_m(nq, arp, acol, aval, d, x, r);
    for (int64_t i = 0; i < nq; i++) r[i] = b[i] - r[i];
    return norm_inf(nq, r);
}

/* ------------------------------------------------------------------------ */
/* Error certificate.  I - A is a nonsingular M-matrix on S_? (every state of
 * S_? leaks to S_{=0} or S_{=1}), so its inverse is entrywise non-negative and
 * for any approximation xh:  |xh - x*| = |(I-A)^{-1} r| <= ||r||_inf * T with
 * T = (I-A)^{-1} 1 (the expected number of steps spent in S_?).  An upper
 * bound on ||T||_inf follows from any approximation Th with residual
 * rT = 1 - (I-A) Th of norm below one: T <= Th + ||rT|| T, hence
 * ||T||_inf <= ||Th||_inf / (1 - ||rT||_inf).
 * Th is computed by plain Jacobi from zero (monotone increasing towards T)
 * until the residual, recomputed from scratch, is at most 1e-3.
 * Returns the bound, or a negative value when it could not be established. */
double orc_tbound(int64_t nq, const int64_t *arp, const int64_t *acol,
                  const double *aval, const double *d, int64_t max_iter)
{
    if (nq == 0) return 0.0;
    double *t = calloc((size_t)nq, sizeof(double));
    double *tn = calloc((size_t)nq, sizeof(double));
    double *r = calloc((size_t)nq, sizeof(double));
    double *one = malloc(sizeof(double) * (size_t)nq);
    if (!t || !tn || !r || !one) {
        free(t); free(tn); free(r); free(one);
        return -1.0;
    }
    for (int64_t i = 0; i < nq; i++) one[i] = 1.0;
    double bound = -1.0;
    for (int64_t it = 0; it < max_iter; it++) {
        for (int64_t i = 0; i < nq; i++) {
            double acc = one[i];
            for (int64_t k = arp[i]; k < arp[i + 1]; k++) acc += aval[k] * t[acol[k]];
            tn[i] = acc / d[i];
        }
        double *sw = t; t = tn; tn = sw;
        if ((it & 15) == 15 || it + 1 == max_iter) {
            double rn = orc_residual(nq, arp, acol, aval, d, one, t, r);
            if (rn <= 1e-3) {
                bound = norm_inf(nq, t) / (1.0 - rn);
                break;
            }
        }
    }
    free(t); free(tn); free(r); free(one);
    return bound;
}

/* ------------------------------------------------------------------------ */
/* Jacobi method (Section 3.1) on (I - A) x = b:
 *     x'_i = (b_i + sum_{j != i} A_off(i,j) x_j) / d_i
 * one full sweep from the previous iterate (double buffered), then
 * delta = max_i |x'_i - x_i|.  Starting vector: x0 if given, else zero.
 * Stopping rule:
 *   stop_mode 0 (the paper's rule): stop after the first sweep with delta < tol.
 *   stop_mode 1 (certified): stop after the first sweep whose result x
 *               satisfies tbound * ||b - (I-A) x||_inf <= tol, the residual
 *               recomputed from scratch after every sweep.
 * Returns ORC_OK or ORC_NOT_CONVERGED (x still holds the last iterate). */
int orc_jacobi(int64_t nq, const int64_t *arp, const int64_t *acol,
               const double *aval, const double *d, const double *b,
               const double *x0, double tol, int64_t max_iter, int stop_mode,
               double tbound, double *x, int64_t *iters_out,
               double *delta_out)
{
    double *xn = malloc(sizeof(double) * (size_t)(nq > 0 ? nq : 1));
    double *r = malloc(sizeof(double) * (size_t)(nq > 0 ? nq : 1));
    if (!xn || !r) { free(xn); free(r); return ORC_NOMEM; }
    for (int64_t i = 0; i < nq; i++) x[i] = x0 ? x0[i] : 0.0;
    int64_t it = 0;
    double delta = INFINITY;
    int rc = ORC_NOT_CONVERGED;
    if (nq == 0) { delta = 0.0; rc = ORC_OK; }
    while (rc != ORC_OK && it < max_iter) {
        delta = 0.0;
        for (int64_t i = 0; i < nq; i++) {
            double acc = b[i];
            for (int64_t k = arp[i]; k < arp[i + 1]; k++) acc += aval[k] * x[acol[k]];
            xn[i] = acc / d[i];
            double dl = fabs(xn[i] - x[i]);
            if (dl > delta || dl != dl) delta = dl;
        }
        memcpy(x, xn, sizeof(double) * (size_t)nq);
        it++;
        if (stop_mode == 0) {
            if (delta < tol) rc = ORC_OK;
        } else {
            double rn = orc_residual(nq, arp, acol, aval, d, b, x, r);
            if (tbound * rn <= tol) rc = ORC_OK;
        }
    }
    *iters_out = it;
    *delta_out = delta;
    free(xn); free(r);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* BiCGStab (Section 3.2; van der Vorst), un-preconditioned, on M x = b with
 * M = I - A.  Each step does one bi-conjugate-gradient update and then a
 * one-dimensional minimal-residual smoothing:
 *   - the shadow residual rhat is fixed at the first residual (rhat.r0 =
 *     |r0|^2 > 0 unless r0 = 0);
 *   - rho = rhat.r.  The new search direction p keeps p orthogonal in the BiCG
 *     sense: p = r + beta (p - omega M p_old) with
 *     beta = (rho / rho_old) (alpha / omega), where M p_old is the v of the
 *     previous step; the first step has p = v = 0, so p = r;
 *   - v = M p; alpha = rho / (rhat.v) makes s = r - alpha v the BiCG
 *     residual, orthogonal to rhat;
 *   - t = M s; omega = (t.s)/(t.t) minimises |s - omega t|_2 (omega = 0 when
 *     t = 0, i.e. s = 0);
 *   - the iterate moves along both directions, x += alpha p + omega s, and
 *     the residual follows, r = s - omega t.
 * The scalars start at rho = alpha = omega = 1.
 * Stopping rule:
 *   stop_mode 0 (the paper's GPU kernel, Section 5.2): stop once every
 *               |s_i| <= tol.
 *   stop_mode 1 (certified): after each step recompute the true residual
 *               b - M x; stop when tbound * ||b - M x||_inf <= tol.  When the
 *               recurrence residual has drifted from the true one (||r|| below
 *               1e-3 * ||b - M x||) the method restarts from the current x
 *               with r = rhat = b - M x.
 * A zero rhat.r or rhat.v is a breakdown: in certified mode the method
 * restarts from the current x (at most 64 times); otherwise ORC_BREAKDOWN is
 * returned. */
int orc_bicgstab(int64_t nq, const int64_t *arp, const int64_t *acol,
                 const double *aval, const double *d, const double *b,
                 const double *x0, double tol, int64_t max_iter,
                 int stop_mode, double tbound, double *x, int64_t *iters_out,
                 double *smax_out)
{
    size_t sz = sizeof(double) * (size_t)(nq > 0 ? nq : 1);
    double *r = malloc(sz), *rhat = malloc(sz), *p = malloc(sz), *v = malloc(sz);
    double *s = malloc(sz), *t = malloc(sz), *rtrue = malloc(sz);
    if (!r || !rhat || !p || !v || !s || !t || !rtrue) {
        free(r); free(rhat); free(p); free(v); free(s); free(t); free(rtrue);
        return ORC_NOMEM;
    }
    for (int64_t i = 0; i < nq; i++) x[i] = x0 ? x0[i] : 0.0;
    int64_t steps = 0;
    double smax = 0.0;
    int rc = ORC_NOT_CONVERGED;
    int restarts_left = 64;
    int restart = 1;
    double rho = 1.0, alpha = 1.0, omega = 1.0;

    double rnorm0 = orc_residual(nq, arp, acol, aval, d, b, x, r);
    if (nq == 0 || rnorm0 == 0.0) rc = ORC_OK;
    if (stop_mode == 1 && tbound * rnorm0 <= tol) rc = ORC_OK;
    while (rc != ORC_OK && steps < max_iter) {
        if (restart) {
            memcpy(rhat, r, sz);
            for (int64_t i = 0; i < nq; i++) { v[i] = 0.0; p[i] = 0.0; }
            rho = 1.0; alpha = 1.0; omega = 1.0;
            restart = 0;
        }
        double rho_old = rho;
        rho = dot(nq, rhat, r);
        if (rho == 0.0) {
            if (stop_mode == 1 && restarts_left-- > 0) {
                orc_residual(nq, arp, acol, aval, d, b, x, r);
                restart = 1;
                continue;
            }
            rc = ORC_BREAKDOWN;
            break;
        }
        double beta = (rho * alpha) / (rho_old * omega);
        for (int64_t i = 0; i < nq; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        apply_m(nq, arp, acol, aval, d, p, v);
        double rhat_v = dot(nq, rhat, v);
        if (rhat_v == 0.0) {
            if (stop_mode == 1 && restarts_left-- > 0) {
                orc_residual(nq, arp, acol, aval, d, b, x, r);
                restart = 1;
                continue;
            }
            rc = ORC_BREAKDOWN;
            break;
        }
        alpha = rho / rhat_v;
        for (int64_t i = 0; i < nq; i++) s[i] = r[i] - alpha * v[i];
        apply_m(nq, arp, acol, aval, d, s, t);
        double tt = dot(nq, t, t);
        omega = (tt == 0.0) ? 0.0 : dot(nq, t, s) / tt;
        smax = norm_inf(nq, s);
        for (int64_t i = 0; i < nq; i++) x[i] = x[i] + alpha * p[i] + omega * s[i];
        for (int64_t i = 0; i < nq; i++) r[i] = s[i] - omega * t[i];
        steps++;
        if (stop_mode == 0) {
            if (smax <= tol) rc = ORC_OK;
        } else {
            double rtrue_norm = orc_residual(nq, arp, acol, aval, d, b, x, rtrue);
            if (tbound * rtrue_norm <= tol) {
                rc = ORC_OK;
            } else if (norm_inf(nq, r) < 1e-3 * rtrue_norm || omega == 0.0) {
                memcpy(r, rtrue, sz);
                restart = 1;
            }
        }
    }
    *iters_out = steps;
    *smax_out = smax;
    free(r); free(rhat); free(p); free(v); free(s); free(t); free(rtrue);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Dense Gaussian elimination with partial pivoting (Section 2.3 mentions
 * direct elimination as the O(n^3) alternative).  Solves Mx = rhs for one
 * right-hand side; M (row-major nq x nq) is overwritten.                    */
int orc_dense_solve(int64_t nq, double *m, const double *rhs, double *x)
{
    double *bb = malloc(sizeof(double) * (size_t)(nq > 0 ? nq : 1));
    if (!bb) return ORC_NOMEM;
    for (int64_t i = 0; i < nq; i++) bb[i] = rhs[i];
    for (int64_t k = 0; k < nq; k++) {
        int64_t piv = k;
        double best = fabs(m[k * nq + k]);
        for (int64_t i = k + 1; i < nq; i++) {
            double c = fabs(m[i * nq + k]);
            if (c > best) { best = c; piv = i; }
        }
        if (best == 0.0) { free(bb); return ORC_SINGULAR; }
        if (piv != k) {
            for (int64_t j = 0; j < nq; j++) {
                double tmp = m[k * nq + j];
                m[k * nq + j] = m[piv * nq + j];
                m[piv * nq + j] = tmp;
            }
            double tmp = bb[k]; bb[k] = bb[piv]; bb[piv] = tmp;
        }
        for (int64_t i = k + 1; i < nq; i++) {
            double f = m[i * nq + k] / m[k * nq + k];
            if (f == 0.0) continue;
            for (int64_t j = k; j < nq; j++) m[i * nq + j] -= f * m[k * nq + j];
            bb[i] -= f * bb[k];
        }
    }
    for (int64_t i = nq - 1; i >= 0; i--) {
        double acc = bb[i];
        for (int64_t j = i + 1; j < nq; j++) acc -= m[i * nq + j] * x[j];
        x[i] = acc / m[i * nq + i];
    }
    free(bb);
    return ORC_OK;
}

/* Dense matrix of I - A from the reduced system (row-major, nq x nq). */
void orc_dense_m(int64_t nq, const int64_t *arp, const int64_t *acol,
                 const double *aval, const double *d, double *m)
{
    for (int64_t i = 0; i < nq * nq; i++) m[i] = 0.0;
    for (int64_t i = 0; i < nq; i++) {
        m[i * nq + i] = d[i];
        for (int64_t k = arp[i]; k < arp[i + 1]; k++) m[i * nq + acol[k]] -= aval[k];
    }
}

/* ------------------------------------------------------------------------ */
/* Gradient of L(x) with respect to every stored transition probability,
 * given the adjoint lam solving (I - A)^T lam = dL/dx on S_?.  Since
 * d(I - A) = -dA and db = dP(., S_{=1}), every stored entry (i, j) with i in
 * S_? gets  dL/dP(i,j) = lam_i * xfull_j  (xfull = 1 on S_{=1}, 0 on S_{=0},
 * the solution on S_?); entries of rows outside S_? get zero (their rows do
 * not enter the system, the partition is held fixed). */
void orc_gradient(int64_t n, const int32_t *rp, const int32_t *col,
                  const uint8_t *cls, const int64_t *map, const double *lam,
                  const double *xfull, double *g)
{
    for (int64_t s = 0; s < n; s++)
        for (int64_t k = rp[s]; k < rp[s + 1]; k++)
            g[k] = (cls[s] == 2) ? lam[map[s]] * xfull[col[k]] : 0.0;
}

/* ------------------------------------------------------------------------ */
/* The experiments of Section 6 solve a general system A x = b (A square,
 * random, diagonally dominant, positive integers) with the same two methods.
 * Section 3.1's Jacobi splits A into its diagonal D and the rest R:
 * x' = D^{-1} (b - R x).  In the solvers' form d[i] x[i] - sum A_off(i,j) x[j]
 * = b[i] that is d = diag(A), A_off = -R, b = rhs.  A is given in compressed
 * row storage with ascending columns; a row without a stored diagonal entry
 * makes the system unusable for Jacobi (returns ORC_SINGULAR).  Outputs:
 * arp[n+1], acol/aval (at most nnz), d[n], b[n]; *z = entries of A_off.     */
int orc_matrix_system(int64_t n, const int32_t *rp, const int32_t *col,
                      const double *val, const double *rhs, int64_t *arp,
                      int64_t *acol, double *aval, double *d, double *b,
                      int64_t *z)
{
    int64_t k = 0;
    arp[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        int have_diag = 0;
        d[i] = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; e++) {
            if (col[e] == i) {
                d[i] = val[e];
                have_diag = 1;
            } else {
                acol[k] = col[e];
                aval[k] = -val[e];
                k++;
            }
        }
        if (!have_diag || d[i] == 0.0)
            return ORC_SINGULAR;
        b[i] = rhs[i];
        arp[i + 1] = k;
    }
    *z = k;
    return ORC_OK;
}

/* Bound on ||A^{-1}||_inf for a strictly row diagonally dominant A (Varah,
 * 1975): ||A^{-1}||_inf <= 1 / min_i (|a_ii| - sum_{j != i} |a_ij|).  Then
 * max|x - x*| <= bound * ||b - A x||_inf certifies a solution, as the
 * (I - A)^{-1} 1 factor does for Markov chains.  Returns -1 when some row
 * is not strictly dominant (no bound).                                      */
double orc_dominance_bound(int64_t nq, const int64_t *arp, const double *aval,
                           const double *d)
{
    double gap = INFINITY;
    for (int64_t i = 0; i < nq; i++) {
        double off = 0.0;
        for (int64_t e = arp[i]; e < arp[i + 1]; e++)
            off += fabs(aval[e]);
        const double g = fabs(d[i]) - off;
        if (!(g > 0.0))
            return -1.0;
        if (g < gap)
            gap = g;
    }
    return nq > 0 ? 1.0 / gap : 0.0;
}

/* Strongly connected components of the graph of A_off over S_? (an edge
 * i -> j where A_off(i,j) > 0; the self-loops sit in d and join no two
 * states), for the decomposition that Section 8 proposes as future work:
 * solve the components in reverse topological order, the one-state ones by
 * substitution.  Tarjan's algorithm (depth-first search keeping a stack of
 * the states not yet assigned and the lowest discovery index reachable),
 * run from the states in ascending order, without recursion.  A component
 * is complete only after every component reachable from it, so they come
 * out sinks first; there
 *   label[i] = smallest reduced index in i's component,
 *   level[i] = 0 if no edge leaves i's component, else 1 + the largest level
 *              of a component an edge leads to,
 * and *ncomp = number of components.  Work arrays: 4 nq int64.           */
int orc_scc(int64_t nq, const int64_t *arp, const int64_t *acol,
            const double *aval, int64_t *label, int64_t *level, int64_t *ncomp)
{
    int64_t *disc = malloc(sizeof(int64_t) * (size_t)(nq > 0 ? nq : 1));
    int64_t *low = malloc(sizeof(int64_t) * (size_t)(nq > 0 ? nq : 1));
    int64_t *stk = malloc(sizeof(int64_t) * (size_t)(nq > 0 ? nq : 1));
    int64_t *call = malloc(sizeof(int64_t) * (size_t)(nq > 0 ? nq : 1));
    int64_t *edge = malloc(sizeof(int64_t) * (size_t)(nq > 0 ? nq : 1));
    char *on = calloc((size_t)(nq > 0 ? nq : 1), 1);
    if (!disc || !low || !stk || !call || !edge || !on) {
        free(disc); free(low); free(stk); free(call); free(edge); free(on);
        return ORC_NOMEM;
    }
    for (int64_t i = 0; i < nq; i++) {
        disc[i] = -1;
        label[i] = -1;
        level[i] = -1;
    }
    int64_t t = 0, sp = 0, comps = 0;
    for (int64_t s = 0; s < nq; s++) {
        if (disc[s] >= 0)
            continue;
        /* explicit depth-first search: call[] holds the path, edge[v] the
         * next entry of row v to look at */
        int64_t depth = 0;
        call[depth++] = s;
        disc[s] = low[s] = t++;
        stk[sp++] = s;
        on[s] = 1;
        edge[s] = arp[s];
        while (depth > 0) {
            const int64_t v = call[depth - 1];
            if (edge[v] < arp[v + 1]) {
                const int64_t e = edge[v]++;
                if (!(aval[e] > 0.0))
                    continue;
                const int64_t w = acol[e];
                if (disc[w] < 0) {
                    disc[w] = low[w] = t++;
                    stk[sp++] = w;
                    on[w] = 1;
                    edge[w] = arp[w];
                    call[depth++] = w;
                } else if (on[w] && disc[w] < low[v]) {
                    low[v] = disc[w];
                }
                continue;
            }
            /* v is finished */
            depth--;
            if (depth > 0) {
                const int64_t u = call[depth - 1];
                if (low[v] < low[u])
                    low[u] = low[v];
            }
            if (low[v] != disc[v])
                continue;
            /* v roots a component: pop it, find its smallest index and the
             * levels of the components its edges lead to (all complete) */
            int64_t top = sp;
            int64_t mn = v, lv = 0;
            do {
                const int64_t w = stk[--top];
                if (w < mn)
                    mn = w;
            } while (stk[top] != v);
            for (int64_t q = top; q < sp; q++) {
                const int64_t w = stk[q];
                on[w] = 0;
            }
            for (int64_t q = top; q < sp; q++) {
                const int64_t w = stk[q];
                for (int64_t e = arp[w]; e < arp[w + 1]; e++) {
                    if (!(aval[e] > 0.0))
                        continue;
                    const int64_t x = acol[e];
                    if (level[x] >= 0 && level[x] + 1 > lv)
                        lv = level[x] + 1;
                }
            }
            for (int64_t q = top; q < sp; q++) {
                label[stk[q]] = mn;
                level[stk[q]] = lv;
            }
            sp = top;
            comps++;
        }
    }
    *ncomp = comps;
    free(disc); free(low); free(stk); free(call); free(edge); free(on);
    return ORC_OK;
}
