/*
 * FP64 CPU oracle for APPGA applied to the SHOITV-regularised Poisson PET model,
 * and for FPPA / AFPPA-N / AFPPA-GN on the nonsmooth HOITV model (Section 4.3)
 * (Lin, He, Schmidtlein, Han, arXiv 2409.13344).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this code.  It shares nothing with
 * the GPU library: no headers, no helpers, no tables.  It is deliberately
 * plain and slow: every step is the paper's definition written out in double
 * precision, single-threaded, without blocking, fusion or reordering.
 *
 * Pinned by tests/test_oracle_*.py (Kronecker construction of B1 and B2,
 * adjoint identities, finite differences, the MLEM identity, identity-system
 * fixed points, count preservation, KKT at the minimiser of long runs,
 * Lemma 5 / Proposition 6 step inequalities, nonexpansiveness; for AFPPA:
 * KKT of the nonsmooth model, perturbation optimality, the MLEM and APPGA
 * reductions at lambda = 0, scaling equivariance, dual feasibility, and FPPA
 * as an averaged operator in the Condat-Vu metric).
 *
 * Readings of points the paper leaves open:
 *  - the first row of D is zero (D_11 = 0), so B annihilates constants;
 *  - image index j = r*N + c (row-major), Kronecker X (x) Y acts as X along r
 *    and Y along c; the objective is invariant under the other ordering;
 *  - the EM preconditioner uses f^k (not the extrapolated point);
 *  - y_i = (A x)_i + gamma_i is floored at tau_i = 1e-6*gamma_i (1e-30 when
 *    gamma_i = 0) before the ratio; floors are counted;
 *  - f^0 = f^1 = the initial image; ACTc = sum(g) - sum(gamma);
 *  - the field-of-view disk has radius N/2 about the image centre;
 *  - AFPPA: the prox of (lambda/rho) phi uses the plain group l2 norm (phi as
 *    defined in Section 2.1 already carries lambda), so b and c are projections
 *    onto balls of radius lambda1 and lambda2; p_max is taken over P at f^k
 *    (floored at 1e-30); b^0 = b^1 = 0 and c^0 = c^1 = 0.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_DOMAIN (-3)
#define ORC_E_OOM (-4)

/* ------------------------------------------------------------------------ */
/* System matrix products (Section 2.1: A in R+^{m x d}, CSR, FP64).        */
/* ------------------------------------------------------------------------ */

/* y = A x */
void orc_forward(int64_t m, const int64_t *row_ptr, const int32_t *col, const double *val,
                 const double *x, double *y)
{
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            s += val[k] * x[col[k]];
        y[i] = s;
    }
}

/* out = A^T r, by scattering every row of A (no stored transpose). */
void orc_back(int64_t m, int64_t d, const int64_t *row_ptr, const int32_t *col, const double *val,
              const double *r, double *out)
{
    for (int64_t j = 0; j < d; ++j)
        out[j] = 0.0;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            out[col[k]] += val[k] * r[i];
}

/* ------------------------------------------------------------------------ */
/* Difference operators (Section 2.1).  D is the N x N backward difference  */
/* matrix: D_{j,j} = 1 and D_{j,j-1} = -1 for j = 2..N (1-based), all other */
/* entries zero.  The 1-D operators below loop over exactly those entries.  */
/* ------------------------------------------------------------------------ */

typedef void (*op1d_fn)(int n, const double *x, ptrdiff_t sx, double *y, ptrdiff_t sy, double *tmp);

static void op_I(int n, const double *x, ptrdiff_t sx, double *y, ptrdiff_t sy, double *tmp)
{
    (void)tmp;
    for (int j = 0; j < n; ++j)
        y[j * sy] = x[j * sx];
}

/* y = D x: for every entry (row j, column j) = 1 and (row j, column j-1) = -1. */
static void op_D(int n, const double *x, ptrdiff_t sx, double *y, ptrdiff_t sy, double *tmp)
{
    (void)tmp;
    for (int j = 0; j < n; ++j)
        y[j * sy] = 0.0;
    for (int j = 1; j < n; ++j) {
        y[j * sy] += 1.0 * x[j * sx];
        y[j * sy] += -1.0 * x[(j - 1) * sx];
    }
}

/* y = D^T x: the same entries with row and column exchanged. */
static void op_Dt(int n, const double *x, ptrdiff_t sx, double *y, ptrdiff_t sy, double *tmp)
{
    (void)tmp;
    for (int j = 0; j < n; ++j)
        y[j * sy] = 0.0;
    for (int j = 1; j < n; ++j) {
        y[j * sy] += 1.0 * x[j * sx];
        y[(j - 1) * sy] += -1.0 * x[j * sx];
    }
}

static void op_negD(int n, const double *x, ptrdiff_t sx, double *y, ptrdiff_t sy, double *tmp)
{
    op_D(n, x, sx, y, sy, tmp);
    for (int j = 0; j < n; ++j)
        y[j * sy] = -y[j * sy];
}

static void op_negDt(int n, const double *x, ptrdiff_t sx, double *y, ptrdiff_t sy, double *tmp)
{
    op_Dt(n, x, sx, y, sy, tmp);
    for (int j = 0; j < n; ++j)
        y[j * sy] = -y[j * sy];
}

/* y = -D^T D x (tmp holds D x; n doubles). */
static void op_negDtD(int n, const double *x, ptrdiff_t sx, double *y, ptrdiff_t sy, double *tmp)
{
    op_D(n, x, sx, tmp, 1, NULL);
    op_Dt(n, tmp, 1, y, sy, NULL);
    for (int j = 0; j < n; ++j)
        y[j * sy] = -y[j * sy];
}

/* out = (X kron Y) f for an N x N image f stored row-major (index r*N + c):
 * Y acts along c within every row, then X along r within every column.
 * work: N*N + N doubles. */
static void kron_apply(int n, op1d_fn X, op1d_fn Y, const double *f, double *out, double *work)
{
    double *t = work;
    double *line = work + (size_t)n * n;
    for (int r = 0; r < n; ++r)
        Y(n, f + (size_t)r * n, 1, t + (size_t)r * n, 1, line);
    for (int c = 0; c < n; ++c)
        X(n, t + c, n, out + c, n, line);
}

static void kron_accum(int n, op1d_fn X, op1d_fn Y, const double *f, double *acc, double *work)
{
    double *o = work + (size_t)n * n + n;
    kron_apply(n, X, Y, f, o, work);
    for (size_t j = 0; j < (size_t)n * n; ++j)
        acc[j] += o[j];
}

static double *orc_work(int n)
{
    return (double *)malloc(sizeof(double) * ((size_t)2 * n * n + n));
}

/* u = B1 f = [ (I kron D) f ; (D kron I) f ]   (2d) */
int orc_b1(int n, const double *f, double *u)
{
    size_t d = (size_t)n * n;
    double *w = orc_work(n);
    if (!w) return ORC_E_OOM;
    kron_apply(n, op_I, op_D, f, u, w);
    kron_apply(n, op_D, op_I, f, u + d, w);
    free(w);
    return ORC_OK;
}

/* v = B2 f = [ (I kron -D^T D) f ; (-D^T kron D) f ; (-D^T D kron I) f ; (D kron -D^T) f ]  (4d) */
int orc_b2(int n, const double *f, double *v)
{
    size_t d = (size_t)n * n;
    double *w = orc_work(n);
    if (!w) return ORC_E_OOM;
    kron_apply(n, op_I, op_negDtD, f, v, w);
    kron_apply(n, op_negDt, op_D, f, v + d, w);
    kron_apply(n, op_negDtD, op_I, f, v + 2 * d, w);
    kron_apply(n, op_D, op_negDt, f, v + 3 * d, w);
    free(w);
    return ORC_OK;
}

/* out = B1^T p, using (X kron Y)^T = X^T kron Y^T. */
int orc_b1t(int n, const double *p, double *out)
{
    size_t d = (size_t)n * n;
    double *w = orc_work(n);
    if (!w) return ORC_E_OOM;
    memset(out, 0, sizeof(double) * d);
    kron_accum(n, op_I, op_Dt, p, out, w);
    kron_accum(n, op_Dt, op_I, p + d, out, w);
    free(w);
    return ORC_OK;
}

/* out = B2^T q; (-D^T D)^T = -D^T D, (-D^T kron D)^T = -D kron D^T,
 * (D kron -D^T)^T = D^T kron -D. */
int orc_b2t(int n, const double *q, double *out)
{
    size_t d = (size_t)n * n;
    double *w = orc_work(n);
    if (!w) return ORC_E_OOM;
    memset(out, 0, sizeof(double) * d);
    kron_accum(n, op_I, op_negDtD, q, out, w);
    kron_accum(n, op_negD, op_Dt, q + d, out, w);
    kron_accum(n, op_negDtD, op_I, q + 2 * d, out, w);
    kron_accum(n, op_Dt, op_negD, q + 3 * d, out, w);
    free(w);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Smoothed l2 norm (eq. def:smoothL2) and its gradient (eq. gradenvL2).    */
/* ------------------------------------------------------------------------ */

double orc_s_eps(const double *x, int len, double eps)
{
    double q = 0.0;
    for (int k = 0; k < len; ++k)
        q += x[k] * x[k];
    double nrm = sqrt(q);
    if (nrm > eps)
        return nrm - eps / 2.0;
    return q / (2.0 * eps);
}

/* SHOITV value lambda1*sum s_eps((B1 f)_i, (B1 f)_{d+i}) + lambda2*sum s_eps(4-vector). */
int orc_reg_value(int n, double lambda1, double lambda2, double eps, const double *f, double *value)
{
    size_t d = (size_t)n * n;
    double *u = (double *)malloc(sizeof(double) * 6 * d);
    if (!u) return ORC_E_OOM;
    double *v = u + 2 * d;
    int st = orc_b1(n, f, u);
    if (st == ORC_OK) st = orc_b2(n, f, v);
    double s1 = 0.0, s2 = 0.0;
    for (size_t i = 0; i < d && st == ORC_OK; ++i) {
        double a[2] = {u[i], u[d + i]};
        double b[4] = {v[i], v[d + i], v[2 * d + i], v[3 * d + i]};
        s1 += orc_s_eps(a, 2, eps);
        s2 += orc_s_eps(b, 4, eps);
    }
    *value = lambda1 * s1 + lambda2 * s2;
    free(u);
    return st;
}

/* out = B^T grad(phi~)(B f): per pixel the weights lambda/max(||.||, eps)
 * of the two groups (Section 2.2, gradient of phi~). */
int orc_grad_reg(int n, double lambda1, double lambda2, double eps, const double *f, double *out)
{
    size_t d = (size_t)n * n;
    double *u = (double *)malloc(sizeof(double) * 7 * d);
    if (!u) return ORC_E_OOM;
    double *v = u + 2 * d;
    double *tmp = u + 6 * d;
    int st = orc_b1(n, f, u);
    if (st == ORC_OK) st = orc_b2(n, f, v);
    for (size_t i = 0; i < d && st == ORC_OK; ++i) {
        double n1 = sqrt(u[i] * u[i] + u[d + i] * u[d + i]);
        double w1 = lambda1 / (n1 > eps ? n1 : eps);
        u[i] *= w1;
        u[d + i] *= w1;
        double q = 0.0;
        for (int c = 0; c < 4; ++c)
            q += v[c * d + i] * v[c * d + i];
        double n2 = sqrt(q);
        double w2 = lambda2 / (n2 > eps ? n2 : eps);
        for (int c = 0; c < 4; ++c)
            v[c * d + i] *= w2;
    }
    if (st == ORC_OK) st = orc_b1t(n, u, out);
    if (st == ORC_OK) st = orc_b2t(n, v, tmp);
    if (st == ORC_OK)
        for (size_t j = 0; j < d; ++j)
            out[j] += tmp[j];
    free(u);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Poisson fidelity (eq. FidelityTerm) and its gradient.                    */
/* ------------------------------------------------------------------------ */

/* Floor applied to y = A x + gamma before the ratio g / y. */
static double y_floor(double gamma_i)
{
    return gamma_i > 0.0 ? 1e-6 * gamma_i : 1e-30;
}

/* e = 1 - g / max(A x + gamma, tau); returns the number of floored bins in *clamps. */
void orc_ratio(int64_t m, const double *ax, const double *g, const double *gamma, double *e,
               int64_t *clamps)
{
    int64_t nc = 0;
    for (int64_t i = 0; i < m; ++i) {
        double y = ax[i] + gamma[i];
        double tau = y_floor(gamma[i]);
        if (y < tau) {
            y = tau;
            ++nc;
        }
        e[i] = 1.0 - g[i] / y;
    }
    if (clamps) *clamps += nc;
}

/* grad F(x) = A^T (1 - g / (A x + gamma)) (with the floor). */
int orc_grad_fidelity(int64_t m, int64_t d, const int64_t *row_ptr, const int32_t *col,
                      const double *val, const double *g, const double *gamma, const double *x,
                      double *out, int64_t *clamps)
{
    double *y = (double *)malloc(sizeof(double) * 2 * (size_t)m);
    if (!y) return ORC_E_OOM;
    double *e = y + m;
    orc_forward(m, row_ptr, col, val, x, y);
    orc_ratio(m, y, g, gamma, e, clamps);
    orc_back(m, d, row_ptr, col, val, e, out);
    free(y);
    return ORC_OK;
}

/* F(x) = <A x, 1> - <ln(A x + gamma), g>, with 0 * ln(.) := 0. */
double orc_fidelity_from_ax(int64_t m, const double *ax, const double *g, const double *gamma)
{
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        s += ax[i];
        if (g[i] != 0.0)
            s -= g[i] * log(ax[i] + gamma[i]);
    }
    return s;
}

/* Phi(x) = F(x) + phi~(B x) + iota(x) (eq. model:SHOTV2); +inf if x has a negative entry. */
int orc_objective(int n, int64_t m, const int64_t *row_ptr, const int32_t *col, const double *val,
                  const double *g, const double *gamma, double lambda1, double lambda2, double eps,
                  const double *x, double *value)
{
    size_t d = (size_t)n * n;
    for (size_t j = 0; j < d; ++j)
        if (x[j] < 0.0) {
            *value = INFINITY;
            return ORC_OK;
        }
    double *ax = (double *)malloc(sizeof(double) * (size_t)m);
    if (!ax) return ORC_E_OOM;
    orc_forward(m, row_ptr, col, val, x, ax);
    double fv = orc_fidelity_from_ax(m, ax, g, gamma);
    free(ax);
    double rv = 0.0;
    int st = orc_reg_value(n, lambda1, lambda2, eps, x, &rv);
    *value = fv + rv;
    return st;
}

/* ------------------------------------------------------------------------ */
/* EM preconditioner support (eq. EM), initial image, momentum (eq. GNtheta) */
/* ------------------------------------------------------------------------ */

/* Lambda_j = (A^T 1)_j if positive, else 1. */
int orc_em_lambda(int64_t m, int64_t d, const int64_t *row_ptr, const int32_t *col,
                  const double *val, double *lam)
{
    double *ones = (double *)malloc(sizeof(double) * (size_t)m);
    if (!ones) return ORC_E_OOM;
    for (int64_t i = 0; i < m; ++i)
        ones[i] = 1.0;
    orc_back(m, d, row_ptr, col, val, ones, lam);
    for (int64_t j = 0; j < d; ++j)
        if (!(lam[j] > 0.0))
            lam[j] = 1.0;
    free(ones);
    return ORC_OK;
}

/* Uniform disk TMC * 1_disk, TMC = ACTc / (NPFOV * NPA), ACTc = sum g - sum gamma. */
int orc_init_image(int n, int64_t m, int n_angles, const double *g, const double *gamma, double *f)
{
    double actc = 0.0;
    for (int64_t i = 0; i < m; ++i)
        actc += g[i] - gamma[i];
    if (!(actc > 0.0) || n_angles <= 0)
        return ORC_E_DOMAIN;
    double ctr = (n - 1) / 2.0, rad2 = (n / 2.0) * (n / 2.0);
    int64_t npfov = 0;
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            int in = (c - ctr) * (c - ctr) + (r - ctr) * (r - ctr) <= rad2;
            f[(size_t)r * n + c] = in ? 1.0 : 0.0;
            npfov += in;
        }
    double tmc = actc / ((double)npfov * (double)n_angles);
    for (size_t j = 0; j < (size_t)n * n; ++j)
        f[j] *= tmc;
    return ORC_OK;
}

/* theta_k = (t_{k-1} - 1) / t_k with t_k = a k^omega + b. */
double orc_theta(int k, double a, double b, double omega)
{
    double tkm1 = a * pow((double)(k - 1), omega) + b;
    double tk = a * pow((double)k, omega) + b;
    return (tkm1 - 1.0) / tk;
}

/* ------------------------------------------------------------------------ */
/* APPGA (eq. APPGAiter with the closed-form prox max(., 0)).               */
/* ------------------------------------------------------------------------ */

#define ORC_MOMENTUM_GN 0
#define ORC_MOMENTUM_NONE 1
#define ORC_PRECOND_EM 0
#define ORC_PRECOND_EM_FROZEN 1
#define ORC_PRECOND_FIXED 2

/*
 * Runs `iterations` applications of T (f^2, ..., f^{K+1}) from f^0 = f^1 =
 * f_init (or the disk image when f_init is NULL) and writes f^{K+1}.
 * obj_hist (nullable, K+1 entries): Phi(f^1), ..., Phi(f^{K+1}).
 * re_hist (nullable, K entries): ||f^{k+1} - f^k|| / ||f^{k+1}||.
 * f_hist (nullable, (K+1)*d entries): f^1, ..., f^{K+1}.
 * fixed_p: the diagonal of P in FIXED mode (d entries, or NULL for the
 * scalar fixed_p_scalar in every pixel).
 * round_f32: a diagnostic, not the method.  When nonzero, the quantities an
 * FP32 implementation stores between its steps -- f~^k, A f~^k, e, grad F,
 * grad R and f^{k+1} -- are rounded to the nearest FP32 value each iteration, so that
 * comparing the run with the exact one measures how much the problem
 * amplifies FP32-size perturbations injected at every iteration.
 */
int orc_appga(int n, int64_t m, const int64_t *row_ptr, const int32_t *col, const double *val,
              int n_angles, const double *g, const double *gamma, double lambda1, double lambda2,
              double eps, double omega, double a, double b, double beta, int iterations,
              int momentum, int precond, int precond_freeze_iter, const double *fixed_p,
              double fixed_p_scalar, const double *f_init, double *f_out, double *obj_hist,
              double *re_hist, double *f_hist, int64_t *clamps, int round_f32)
{
    if (n <= 0 || m < 0 || iterations < 0 || !row_ptr || !g || !gamma || !f_out)
        return ORC_E_ARG;
    if (!(eps > 0.0) || lambda1 < 0.0 || lambda2 < 0.0 || !(beta > 0.0) || !(omega > 0.0) ||
        omega > 1.0 || !(a > 0.0) || (omega == 1.0 && a >= 0.5))
        return ORC_E_DOMAIN;
    size_t d = (size_t)n * n;
    double *buf = (double *)malloc(sizeof(double) * (8 * d + 2 * (size_t)m));
    if (!buf) return ORC_E_OOM;
    double *f = buf, *fprev = buf + d, *ft = buf + 2 * d, *gF = buf + 3 * d, *gR = buf + 4 * d;
    double *lam = buf + 5 * d, *p = buf + 6 * d, *fn = buf + 7 * d;
    double *y = buf + 8 * d, *e = y + m;
    int st = ORC_OK;
    int64_t nclamp = 0;

    if (f_init) {
        memcpy(f, f_init, sizeof(double) * d);
    } else {
        st = orc_init_image(n, m, n_angles, g, gamma, f);
        if (st != ORC_OK) {
            free(buf);
            return st;
        }
    }
    memcpy(fprev, f, sizeof(double) * d);
    orc_em_lambda(m, (int64_t)d, row_ptr, col, val, lam);
    if (obj_hist)
        orc_objective(n, m, row_ptr, col, val, g, gamma, lambda1, lambda2, eps, f, &obj_hist[0]);
    if (f_hist)
        memcpy(f_hist, f, sizeof(double) * d);

    for (int k = 1; k <= iterations && st == ORC_OK; ++k) {
        double theta = momentum == ORC_MOMENTUM_NONE ? 0.0 : orc_theta(k, a, b, omega);
        for (size_t j = 0; j < d; ++j)
            ft[j] = f[j] + theta * (f[j] - fprev[j]);
        if (round_f32)
            for (size_t j = 0; j < d; ++j) ft[j] = (double)(float)ft[j];
        /* grad F at the extrapolated point */
        orc_forward(m, row_ptr, col, val, ft, y);
        if (round_f32)
            for (int64_t i = 0; i < m; ++i) y[i] = (double)(float)y[i];
        orc_ratio(m, y, g, gamma, e, &nclamp);
        if (round_f32)
            for (int64_t i = 0; i < m; ++i) e[i] = (double)(float)e[i];
        orc_back(m, (int64_t)d, row_ptr, col, val, e, gF);
        /* grad of the smoothed regulariser at the extrapolated point */
        st = orc_grad_reg(n, lambda1, lambda2, eps, ft, gR);
        if (round_f32)
            for (size_t j = 0; j < d; ++j) {
                gF[j] = (double)(float)gF[j];
                gR[j] = (double)(float)gR[j];
            }
        /* diagonal preconditioner */
        if (precond == ORC_PRECOND_FIXED) {
            for (size_t j = 0; j < d; ++j)
                p[j] = fixed_p ? fixed_p[j] : fixed_p_scalar;
        } else if (precond == ORC_PRECOND_EM || k == 1 || k <= precond_freeze_iter) {
            for (size_t j = 0; j < d; ++j)
                p[j] = beta * f[j] / lam[j];
        }
        /* preconditioned gradient step and the prox of the indicator */
        for (size_t j = 0; j < d; ++j) {
            double z = ft[j] - p[j] * (gF[j] + gR[j]);
            fn[j] = z > 0.0 ? z : 0.0;
            if (round_f32) fn[j] = (double)(float)fn[j];
        }
        if (re_hist) {
            double dn = 0.0, nn = 0.0;
            for (size_t j = 0; j < d; ++j) {
                dn += (fn[j] - f[j]) * (fn[j] - f[j]);
                nn += fn[j] * fn[j];
            }
            re_hist[k - 1] = nn > 0.0 ? sqrt(dn) / sqrt(nn) : 0.0;
        }
        memcpy(fprev, f, sizeof(double) * d);
        memcpy(f, fn, sizeof(double) * d);
        if (obj_hist)
            orc_objective(n, m, row_ptr, col, val, g, gamma, lambda1, lambda2, eps, f,
                          &obj_hist[k]);
        if (f_hist)
            memcpy(f_hist + (size_t)k * d, f, sizeof(double) * d);
    }
    memcpy(f_out, f, sizeof(double) * d);
    if (clamps) *clamps = nclamp;
    free(buf);
    return st;
}

/* ------------------------------------------------------------------------ */
/* AFPPA for the nonsmooth HOITV model (Section 4.3: FPPA with the momentum   */
/* of eq. GNtheta or Nesterov's, eq. AFPPAiter).                             */
/* ------------------------------------------------------------------------ */

#define ORC_MOMENTUM_NESTEROV 2

/* Nesterov's sequence (Section 4.3): t_0 = 1, t_k = (1 + sqrt(1 + 4 t_{k-1}^2)) / 2. */
double orc_t_nesterov(int k)
{
    double t = 1.0;
    for (int i = 1; i <= k; ++i)
        t = (1.0 + sqrt(1.0 + 4.0 * t * t)) / 2.0;
    return t;
}

/* theta_k = (t_{k-1} - 1) / t_k of Nesterov's sequence. */
double orc_theta_nesterov(int k)
{
    return (orc_t_nesterov(k - 1) - 1.0) / orc_t_nesterov(k);
}

/* HOITV value (model HOTV): lambda1 sum ||((B1 f)_i, (B1 f)_{d+i})|| + lambda2 sum ||4-vector||. */
int orc_hoitv_value(int n, double lambda1, double lambda2, const double *f, double *value)
{
    size_t d = (size_t)n * n;
    double *u = (double *)malloc(sizeof(double) * 6 * d);
    if (!u) return ORC_E_OOM;
    double *v = u + 2 * d;
    int st = orc_b1(n, f, u);
    if (st == ORC_OK) st = orc_b2(n, f, v);
    double s1 = 0.0, s2 = 0.0;
    for (size_t i = 0; i < d && st == ORC_OK; ++i) {
        s1 += sqrt(u[i] * u[i] + u[d + i] * u[d + i]);
        double q = 0.0;
        for (int c = 0; c < 4; ++c)
            q += v[c * d + i] * v[c * d + i];
        s2 += sqrt(q);
    }
    *value = lambda1 * s1 + lambda2 * s2;
    free(u);
    return st;
}

/* Objective of the nonsmooth model at f >= 0: fidelity + HOITV. */
int orc_objective_hoitv(int n, int64_t m, const int64_t *row_ptr, const int32_t *col, const double *val,
                        const double *g, const double *gamma, double lambda1, double lambda2, const double *f,
                        double *value)
{
    double *ax = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    if (!ax) return ORC_E_OOM;
    orc_forward(m, row_ptr, col, val, f, ax);
    double reg = 0.0;
    int st = orc_hoitv_value(n, lambda1, lambda2, f, &reg);
    *value = orc_fidelity_from_ax(m, ax, g, gamma) + reg;
    free(ax);
    return st;
}

/* (I - prox_{t ||.||_2})(z) for one group of `len` components: the projection
 * of z onto the l2 ball of radius t, z * min(1, t / ||z||). */
static void orc_ball_projection(double *z, int len, double t)
{
    double q = 0.0;
    for (int c = 0; c < len; ++c)
        q += z[c] * z[c];
    double nrm = sqrt(q);
    if (nrm > t) {
        double s = t / nrm;
        for (int c = 0; c < len; ++c)
            z[c] *= s;
    }
}

/*
 * Runs `iterations` steps of AFPPA (momentum GN, NONE = FPPA, or NESTEROV) from
 * f^0 = f^1 = f_init (or the disk image) with b^0 = b^1 = 0 (2d) and
 * c^0 = c^1 = 0 (4d), and writes f^{K+1} (and b^{K+1}, c^{K+1} when b_out /
 * c_out are given).  Each step, with theta_k from the momentum:
 *   f~ = f + theta (f - f_prev), b~ and c~ likewise;
 *   P = beta f^k / Lambda (EM) or the scalar fixed_p_scalar (FIXED);
 *   rho1 = 1 / (2 * 8 * p_max), rho2 = 1 / (2 * 64 * p_max), p_max = max_j P_jj;
 *   f^{k+1} = max(f~ - P (grad F(f~) + B1^T b~ + B2^T c~), 0);
 *   b^{k+1} = rho1 (I - prox_{(lambda1/rho1) ||.||})(b~ / rho1 + B1 (2 f^{k+1} - f~)), per pixel
 *   group of 2 components, and c^{k+1} likewise with rho2, lambda2 and 4 components.
 * The prox is read with the unweighted group l2 norm (phi_1 as defined in
 * Section 2.1 already carries lambda1), so the ball radius is lambda/rho.
 * obj_hist (K+1): the nonsmooth objective at f^1 .. f^{K+1}; re_hist (K):
 * ||f^{k+1} - f^k|| / ||f^{k+1}||; rho_hist (2K): rho1, rho2 per step.
 * round_f32: a diagnostic, not the method.  When nonzero, the quantities an
 * FP32 implementation holds between its steps -- f~, b~, c~, A f~, e, grad F,
 * B1^T b~ + B2^T c~, p_max, f^{k+1}, 2 f^{k+1} - f~, b^{k+1} and c^{k+1} -- are
 * rounded to the nearest FP32 value each iteration, so that comparing the run
 * with the exact one measures how much the run amplifies FP32-size
 * perturbations injected at every iteration.
 */
int orc_afppa(int n, int64_t m, const int64_t *row_ptr, const int32_t *col, const double *val,
              int n_angles, const double *g, const double *gamma, double lambda1, double lambda2,
              double omega, double a, double b, double beta, int iterations, int momentum, int precond,
              double fixed_p_scalar, const double *f_init, double *f_out, double *b_out, double *c_out,
              double *obj_hist, double *re_hist, double *rho_hist, int64_t *clamps, int round_f32)
{
    if (n <= 0 || m < 0 || iterations < 0 || !row_ptr || !g || !gamma || !f_out)
        return ORC_E_ARG;
    if (lambda1 < 0.0 || lambda2 < 0.0 || !(beta > 0.0) || !(omega > 0.0) || omega > 1.0 || !(a > 0.0) ||
        (omega == 1.0 && a >= 0.5) || (precond != ORC_PRECOND_EM && precond != ORC_PRECOND_FIXED) ||
        (precond == ORC_PRECOND_FIXED && !(fixed_p_scalar > 0.0)))
        return ORC_E_DOMAIN;
    size_t d = (size_t)n * n;
    double *buf = (double *)malloc(sizeof(double) * (31 * d + 2 * (size_t)m));
    if (!buf) return ORC_E_OOM;
    double *f = buf, *fprev = buf + d, *ft = buf + 2 * d, *gF = buf + 3 * d, *t1 = buf + 4 * d;
    double *t2 = buf + 5 * d, *lam = buf + 6 * d, *p = buf + 7 * d, *fn = buf + 8 * d, *w = buf + 9 * d;
    double *bq = buf + 10 * d, *bprev = buf + 12 * d, *bt = buf + 14 * d, *u = buf + 16 * d;
    double *cq = buf + 18 * d, *cprev = buf + 22 * d, *ct = buf + 26 * d;
    double *v = (double *)malloc(sizeof(double) * 4 * d);
    double *y = buf + 31 * d, *e = y + m;
    if (!v) {
        free(buf);
        return ORC_E_OOM;
    }
    int st = ORC_OK;
    int64_t nclamp = 0;
    if (f_init) {
        memcpy(f, f_init, sizeof(double) * d);
    } else {
        st = orc_init_image(n, m, n_angles, g, gamma, f);
    }
    memcpy(fprev, f, sizeof(double) * d);
    memset(bq, 0, sizeof(double) * 4 * d);      /* b and b_prev */
    memset(cq, 0, sizeof(double) * 8 * d);      /* c and c_prev */
    orc_em_lambda(m, (int64_t)d, row_ptr, col, val, lam);
    if (obj_hist && st == ORC_OK)
        st = orc_objective_hoitv(n, m, row_ptr, col, val, g, gamma, lambda1, lambda2, f, &obj_hist[0]);

    for (int k = 1; k <= iterations && st == ORC_OK; ++k) {
        /* orc_theta_nesterov rebuilds t_k from t_0 (O(k)); the runs here are short */
        double theta = momentum == ORC_MOMENTUM_NONE       ? 0.0
                       : momentum == ORC_MOMENTUM_NESTEROV ? orc_theta_nesterov(k)
                                                           : orc_theta(k, a, b, omega);
        for (size_t j = 0; j < d; ++j)
            ft[j] = f[j] + theta * (f[j] - fprev[j]);
        for (size_t j = 0; j < 2 * d; ++j)
            bt[j] = bq[j] + theta * (bq[j] - bprev[j]);
        for (size_t j = 0; j < 4 * d; ++j)
            ct[j] = cq[j] + theta * (cq[j] - cprev[j]);
        if (round_f32) {
            for (size_t j = 0; j < d; ++j) ft[j] = (double)(float)ft[j];
            for (size_t j = 0; j < 2 * d; ++j) bt[j] = (double)(float)bt[j];
            for (size_t j = 0; j < 4 * d; ++j) ct[j] = (double)(float)ct[j];
        }
        /* grad F at the extrapolated point */
        orc_forward(m, row_ptr, col, val, ft, y);
        if (round_f32)
            for (int64_t i = 0; i < m; ++i) y[i] = (double)(float)y[i];
        orc_ratio(m, y, g, gamma, e, &nclamp);
        if (round_f32)
            for (int64_t i = 0; i < m; ++i) e[i] = (double)(float)e[i];
        orc_back(m, (int64_t)d, row_ptr, col, val, e, gF);
        st = orc_b1t(n, bt, t1);
        if (st == ORC_OK) st = orc_b2t(n, ct, t2);
        if (round_f32)
            for (size_t j = 0; j < d; ++j) {
                gF[j] = (double)(float)gF[j];
                t1[j] = (double)(float)(t1[j] + t2[j]);
                t2[j] = 0.0;
            }
        /* preconditioner and the dual step sizes */
        double pmax = 0.0;
        for (size_t j = 0; j < d; ++j) {
            p[j] = precond == ORC_PRECOND_FIXED ? fixed_p_scalar : beta * f[j] / lam[j];
            if (p[j] > pmax) pmax = p[j];
        }
        if (pmax < 1e-30) pmax = 1e-30;
        if (round_f32) pmax = (double)(float)pmax;
        double rho1 = 1.0 / (2.0 * 8.0 * pmax), rho2 = 1.0 / (2.0 * 64.0 * pmax);
        if (rho_hist) {
            rho_hist[2 * (k - 1)] = rho1;
            rho_hist[2 * (k - 1) + 1] = rho2;
        }
        /* primal step */
        for (size_t j = 0; j < d; ++j) {
            double z = ft[j] - p[j] * (gF[j] + t1[j] + t2[j]);
            fn[j] = z > 0.0 ? z : 0.0;
            if (round_f32) fn[j] = (double)(float)fn[j];
            w[j] = 2.0 * fn[j] - ft[j];
            if (round_f32) w[j] = (double)(float)w[j];
        }
        /* dual steps */
        if (st == ORC_OK) st = orc_b1(n, w, u);
        if (st == ORC_OK) st = orc_b2(n, w, v);
        memcpy(bprev, bq, sizeof(double) * 2 * d);
        memcpy(cprev, cq, sizeof(double) * 4 * d);
        for (size_t i = 0; i < d && st == ORC_OK; ++i) {
            double z1[2] = {bt[i] / rho1 + u[i], bt[d + i] / rho1 + u[d + i]};
            orc_ball_projection(z1, 2, lambda1 / rho1);
            bq[i] = rho1 * z1[0];
            bq[d + i] = rho1 * z1[1];
            double z2[4];
            for (int c = 0; c < 4; ++c)
                z2[c] = ct[c * d + i] / rho2 + v[c * d + i];
            orc_ball_projection(z2, 4, lambda2 / rho2);
            for (int c = 0; c < 4; ++c)
                cq[c * d + i] = rho2 * z2[c];
            if (round_f32) {
                bq[i] = (double)(float)bq[i];
                bq[d + i] = (double)(float)bq[d + i];
                for (int c = 0; c < 4; ++c) cq[c * d + i] = (double)(float)cq[c * d + i];
            }
        }
        if (re_hist) {
            double dn = 0.0, nn = 0.0;
            for (size_t j = 0; j < d; ++j) {
                dn += (fn[j] - f[j]) * (fn[j] - f[j]);
                nn += fn[j] * fn[j];
            }
            re_hist[k - 1] = nn > 0.0 ? sqrt(dn) / sqrt(nn) : 0.0;
        }
        memcpy(fprev, f, sizeof(double) * d);
        memcpy(f, fn, sizeof(double) * d);
        if (obj_hist && st == ORC_OK)
            st = orc_objective_hoitv(n, m, row_ptr, col, val, g, gamma, lambda1, lambda2, f, &obj_hist[k]);
    }
    memcpy(f_out, f, sizeof(double) * d);
    if (b_out) memcpy(b_out, bq, sizeof(double) * 2 * d);
    if (c_out) memcpy(c_out, cq, sizeof(double) * 4 * d);
    if (clamps) *clamps = nclamp;
    free(v);
    free(buf);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Factored forward model (Section 4.1 simulation set-up): a space-invariant */
/* Gaussian PSF H in image space and per-ray attenuation factors, so that   */
/* A = diag(n) G H for a geometric projector G.                             */
/* ------------------------------------------------------------------------ */

/* Taps w[0..2R] of the 1-D Gaussian of full width at half maximum `fwhm`
 * (in pixels), sigma = fwhm / (2 sqrt(2 ln 2)), at offsets -R..R, normalised
 * to sum 1 over those 2R + 1 offsets. */
int orc_psf_taps(double fwhm, int R, double *w)
{
    if (!w || R < 0 || !(fwhm > 0.0)) return ORC_E_DOMAIN;
    double sigma = fwhm / (2.0 * sqrt(2.0 * log(2.0)));
    double s = 0.0;
    for (int t = -R; t <= R; ++t) {
        w[t + R] = exp(-(double)t * t / (2.0 * sigma * sigma));
        s += w[t + R];
    }
    for (int t = 0; t <= 2 * R; ++t)
        w[t] /= s;
    return ORC_OK;
}

/* out = H x for the n x n image x: out(r, c) = sum_{|a|,|b| <= R} w[a] w[b] x(r + a, c + b),
 * where positions outside the image contribute 0 (so H is symmetric). */
int orc_psf_apply(int n, int R, const double *w, const double *x, double *out)
{
    if (n <= 0 || R < 0 || !w || !x || !out) return ORC_E_ARG;
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            double s = 0.0;
            for (int a = -R; a <= R; ++a) {
                int rr = r + a;
                if (rr < 0 || rr >= n) continue;
                for (int b = -R; b <= R; ++b) {
                    int cc = c + b;
                    if (cc < 0 || cc >= n) continue;
                    s += w[a + R] * w[b + R] * x[(size_t)rr * n + cc];
                }
            }
            out[(size_t)r * n + c] = s;
        }
    return ORC_OK;
}

/* Attenuation factor of every ray: n_i = exp(-(G mu)_i), mu the attenuation
 * coefficient per pixel in units of the projector's path lengths. */
int orc_attenuation(int64_t m, const int64_t *row_ptr, const int32_t *col, const double *val,
                    const double *mu, double *out)
{
    if (m < 0 || !row_ptr || !mu || !out) return ORC_E_ARG;
    orc_forward(m, row_ptr, col, val, mu, out);
    for (int64_t i = 0; i < m; ++i)
        out[i] = exp(-out[i]);
    return ORC_OK;
}
