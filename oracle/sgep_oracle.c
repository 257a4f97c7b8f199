/*
 * sgep_oracle.c -- FP64 CPU oracle for the gamma-EigenGame hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code with the HIP
 * path.  Everything is plain double precision and written for a reader to
 * check against the paper line by line of the mathematics, not for speed.
 *
 * Paper: Gemp, Chen, McWilliams, "The Symmetric Generalized Eigenvalue
 * Problem as a Nash Equilibrium" (ICLR 2023, arXiv 2206.04993).
 *
 * Contents
 *   oracle_cholesky        B = L L^T                    (B must be SPD: Sec. 1)
 *   oracle_jacobi_eigh     cyclic Jacobi eigensolver    (Golub & Van Loan,
 *                          Matrix Computations, cyclic Jacobi with the stable
 *                          two-by-two symmetric Schur decomposition)
 *   oracle_gep_topk        top-k of A v = lambda B v via L^{-1} A L^{-T}
 *                          (App. A, similar-matrices proposition and the
 *                          B-orthogonality lemma)
 *   oracle_eta             step-size schedules (Sec. 3 step-size condition;
 *                          App. H neural-CCA table: warmup + harmonic decay)
 *   oracle_gamma_step      one iteration of Alg. 2 (stochastic gamma-EigenGame)
 *                          with M = 1, written per player with explicit sums
 *                          over the minibatch rows (CCA, GENERAL, LDA and the
 *                          kurtosis form of ICA of Sec. 1); with pb->smooth, Alg. 3
 *                          (App. G: the clipped denominator replaced by a
 *                          smooth log-space estimate with its own variable)
 *   oracle_gamma_step_dense  the same Alg. 2 iteration with exact A and B
 *                          (full batch; used by the fixed-point pins)
 *   oracle_alg1_step       one iteration of Alg. 1 (deterministic, exact B y_j)
 *
 * Layout conventions: square matrices are row-major n x n.  The players'
 * vectors V (and the auxiliary [Bv] called G) are d x k column-major: player
 * i occupies V[i*d .. i*d+d-1].  Minibatch views are row-major, one sample
 * per row, with an explicit leading dimension.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_KIND_CCA 0
#define OR_KIND_GENERAL 1
#define OR_KIND_LDA 2
#define OR_KIND_ICA 3

#define OR_OPT_SGD 0
#define OR_OPT_ADAM 1

#define OR_SCHED_CONST 0
#define OR_SCHED_INV 1
#define OR_SCHED_WARMUP_HARMONIC 2

/* ------------------------------------------------------------------------- */
/* Dense linear algebra                                                       */
/* ------------------------------------------------------------------------- */

/* In place Cholesky factorisation of the SPD matrix a (n x n, row-major).
 * On success the lower triangle holds L with B = L L^T, the strict upper
 * triangle is zeroed and 0 is returned.  Returns -1 (a left partially
 * overwritten) if a pivot is not strictly positive, i.e. B is not positive
 * definite, which the problem statement forbids. */
int oracle_cholesky(int n, double *a)
{
    for (int j = 0; j < n; ++j) {
        double s = a[(size_t)j * n + j];
        for (int p = 0; p < j; ++p)
            s -= a[(size_t)j * n + p] * a[(size_t)j * n + p];
        if (!(s > 0.0))
            return -1;
        double ljj = sqrt(s);
        a[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double t = a[(size_t)i * n + j];
            for (int p = 0; p < j; ++p)
                t -= a[(size_t)i * n + p] * a[(size_t)j * n + p];
            a[(size_t)i * n + j] = t / ljj;
        }
        for (int i = 0; i < j; ++i)
            a[(size_t)i * n + j] = 0.0;
    }
    return 0;
}

/* Off-diagonal Frobenius norm and full Frobenius norm of a (n x n). */
static void frob_parts(int n, const double *a, double *off, double *all)
{
    double so = 0.0, sa = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double v = a[(size_t)i * n + j] * a[(size_t)i * n + j];
            sa += v;
            if (i != j)
                so += v;
        }
    *off = sqrt(so);
    *all = sqrt(sa);
}

/* Cyclic Jacobi for a symmetric matrix.  a (n x n, row-major) is destroyed:
 * on return its diagonal holds the eigenvalues.  z (n x n, row-major) receives
 * the eigenvectors as COLUMNS (z[r*n + c] is component r of vector c); w the
 * eigenvalues (unsorted, w[c] belongs to column c).  Sweeps until
 * off(a) <= tol * ||a||_F, or until a sweep finds every off-diagonal element
 * negligible at working precision against its diagonal pair
 * (|a_pq| <= eps sqrt(|a_pp a_qq|), the relative threshold of Demmel and
 * Veselic, 1992: the off-diagonal norm of a large matrix stops shrinking at
 * a rounding floor that can lie above tol * ||a||_F), or max_sweeps is
 * reached.  Returns the number of sweeps used, or -1 if it did not
 * converge. */
int oracle_jacobi_eigh(int n, double *a, double *w, double *z, double tol, int max_sweeps)
{
    /* the eigenvectors are accumulated as ROWS of zt (contiguous updates) */
    double *zt = (double *)malloc((size_t)n * n * sizeof(double));
    if (!zt)
        return -1;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            zt[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    double off, all;
    frob_parts(n, a, &off, &all);
    int sweep = 0, rc = 0;
    while (off > tol * all) {
        if (sweep >= max_sweeps) {
            rc = -1;
            break;
        }
        int rotated = 0;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[(size_t)p * n + q];
                const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
                if (fabs(apq) <= DBL_EPSILON * sqrt(fabs(app * aqq)))
                    continue; /* negligible (zero included) */
                rotated = 1;
                /* two-by-two symmetric Schur decomposition: J = [[c, s], [-s, c]]
                 * on (p, q) with t = s / c the smaller root of
                 * t^2 + 2 tau t - 1 = 0, so that J^T a J has a zero in
                 * position (p, q) (Golub and Van Loan, Sec. 8.5) */
                const double tau = (aqq - app) / (2.0 * apq);
                double t;
                if (tau >= 0.0)
                    t = 1.0 / (tau + sqrt(1.0 + tau * tau));
                else
                    t = -1.0 / (-tau + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double sn = t * c;
                /* rows p and q of J^T a J outside the 2 x 2 block, mirrored into
                 * columns p and q (a stays symmetric) */
                for (int r = 0; r < n; ++r) {
                    if (r == p || r == q)
                        continue;
                    const double apr = a[(size_t)p * n + r], aqr = a[(size_t)q * n + r];
                    const double np = c * apr - sn * aqr, nq = sn * apr + c * aqr;
                    a[(size_t)p * n + r] = np;
                    a[(size_t)r * n + p] = np;
                    a[(size_t)q * n + r] = nq;
                    a[(size_t)r * n + q] = nq;
                }
                /* the 2 x 2 block in closed form */
                a[(size_t)p * n + p] = app - t * apq;
                a[(size_t)q * n + q] = aqq + t * apq;
                a[(size_t)p * n + q] = 0.0;
                a[(size_t)q * n + p] = 0.0;
                /* vectors: z <- z J, i.e. rows p and q of zt */
                for (int r = 0; r < n; ++r) {
                    const double zp = zt[(size_t)p * n + r], zq = zt[(size_t)q * n + r];
                    zt[(size_t)p * n + r] = c * zp - sn * zq;
                    zt[(size_t)q * n + r] = sn * zp + c * zq;
                }
            }
        }
        ++sweep;
        frob_parts(n, a, &off, &all);
        if (!rotated)
            break;
    }
    for (int i = 0; i < n; ++i) {
        w[i] = a[(size_t)i * n + i];
        for (int j = 0; j < n; ++j)
            z[(size_t)j * n + i] = zt[(size_t)i * n + j];
    }
    free(zt);
    return rc < 0 ? rc : sweep;
}

/* Forward substitution: solve L x = rhs for lower-triangular L (n x n,
 * row-major), in place on x (length n). */
static void solve_lower(int n, const double *L, double *x)
{
    for (int i = 0; i < n; ++i) {
        double s = x[i];
        for (int p = 0; p < i; ++p)
            s -= L[(size_t)i * n + p] * x[p];
        x[i] = s / L[(size_t)i * n + i];
    }
}

/* Back substitution: solve L^T x = rhs, in place on x. */
static void solve_lower_transposed(int n, const double *L, double *x)
{
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int p = i + 1; p < n; ++p)
            s -= L[(size_t)p * n + i] * x[p];
        x[i] = s / L[(size_t)i * n + i];
    }
}

/* Top-k generalized eigenpairs of A v = lambda B v (A symmetric, B SPD), the
 * problem of Sec. 1, by the reduction of App. A: with B = L L^T the matrix
 * C = L^{-1} A L^{-T} is symmetric and similar to B^{-1} A, its eigenvectors
 * w give v = L^{-T} w, and those v are B-orthonormal.
 *   A, B   : d x d row-major, not modified
 *   lam    : out, k eigenvalues in descending order
 *   V      : out, d x k column-major, B-orthonormal (V^T B V = I)
 *   canon  : if nonzero, flip each column so that its largest-magnitude
 *            component (lowest index on ties) is positive
 * Returns 0, -1 if B is not SPD, -2 if Jacobi did not converge, -3 on
 * allocation failure. */
int oracle_gep_topk(int d, const double *A, const double *B, int k, double *lam, double *V, int canon)
{
    size_t dd = (size_t)d * d;
    double *L = (double *)malloc(dd * sizeof(double));
    double *C = (double *)malloc(dd * sizeof(double));
    double *Z = (double *)malloc(dd * sizeof(double));
    double *w = (double *)malloc((size_t)d * sizeof(double));
    double *col = (double *)malloc((size_t)d * sizeof(double));
    int *order = (int *)malloc((size_t)d * sizeof(int));
    int rc = 0;
    if (!L || !C || !Z || !w || !col || !order) {
        rc = -3;
        goto done;
    }
    memcpy(L, B, dd * sizeof(double));
    if (oracle_cholesky(d, L) != 0) {
        rc = -1;
        goto done;
    }
    /* W = L^{-1} A, column by column; stored transposed in Z (row c = column c of W) */
    for (int c = 0; c < d; ++c) {
        for (int r = 0; r < d; ++r)
            col[r] = A[(size_t)r * d + c];
        solve_lower(d, L, col);
        for (int r = 0; r < d; ++r)
            Z[(size_t)c * d + r] = col[r]; /* Z = W^T */
    }
    /* C = W L^{-T} = (L^{-1} W^T)^T: solve for each column of W^T */
    for (int c = 0; c < d; ++c) {
        for (int r = 0; r < d; ++r)
            col[r] = Z[(size_t)r * d + c];
        solve_lower(d, L, col);
        for (int r = 0; r < d; ++r)
            C[(size_t)c * d + r] = col[r]; /* transpose back */
    }
    /* symmetrise away rounding */
    for (int i = 0; i < d; ++i)
        for (int j = i + 1; j < d; ++j) {
            double m = 0.5 * (C[(size_t)i * d + j] + C[(size_t)j * d + i]);
            C[(size_t)i * d + j] = m;
            C[(size_t)j * d + i] = m;
        }
    if (oracle_jacobi_eigh(d, C, w, Z, 1e-15, 100) < 0) {
        rc = -2;
        goto done;
    }
    /* stable selection sort by eigenvalue, descending */
    for (int i = 0; i < d; ++i)
        order[i] = i;
    for (int i = 0; i < d; ++i) {
        int best = i;
        for (int j = i + 1; j < d; ++j)
            if (w[order[j]] > w[order[best]])
                best = j;
        if (best != i) {
            int t = order[best];
            for (int j = best; j > i; --j)
                order[j] = order[j - 1];
            order[i] = t;
        }
    }
    for (int i = 0; i < k; ++i) {
        int c = order[i];
        lam[i] = w[c];
        for (int r = 0; r < d; ++r)
            col[r] = Z[(size_t)r * d + c];
        solve_lower_transposed(d, L, col); /* v = L^{-T} w */
        if (canon) {
            int arg = 0;
            for (int r = 1; r < d; ++r)
                if (fabs(col[r]) > fabs(col[arg]))
                    arg = r;
            if (col[arg] < 0.0)
                for (int r = 0; r < d; ++r)
                    col[r] = -col[r];
        }
        memcpy(V + (size_t)i * d, col, (size_t)d * sizeof(double));
    }
done:
    free(L);
    free(C);
    free(Z);
    free(w);
    free(col);
    free(order);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Step-size schedules                                                        */
/* ------------------------------------------------------------------------- */

/* eta_t for iteration t = 1, 2, ...
 *   CONST            : eta0
 *   INV              : eta0 / (1 + t / t0)  -- square-summable, not summable
 *                      (Sec. 3 condition of the convergence theorem)
 *   WARMUP_HARMONIC  : linear warmup to eta0 at t_c, then decay proportional
 *                      to 1/(t + Delta) reaching eta_T at t = T (App. H, the
 *                      schedule used with Adam for neural CCA). Delta solves
 *                      eta0 (t_c + Delta) / (T + Delta) = eta_T. */
double oracle_eta(int schedule, double t, double eta0, double eta_T, double t0, double t_c, double T)
{
    switch (schedule) {
    case OR_SCHED_CONST:
        return eta0;
    case OR_SCHED_INV:
        return eta0 / (1.0 + t / t0);
    case OR_SCHED_WARMUP_HARMONIC: {
        if (t < t_c)
            return eta0 * t / t_c;
        double delta = (eta_T * T - eta0 * t_c) / (eta0 - eta_T);
        return eta0 * (t_c + delta) / (t + delta);
    }
    default:
        return NAN;
    }
}

/* ------------------------------------------------------------------------- */
/* Alg. 2, one iteration                                                      */
/* ------------------------------------------------------------------------- */

typedef struct {
    int32_t kind;      /* OR_KIND_* */
    int32_t k;         /* players */
    int32_t n_classes; /* LDA */
    int32_t optimizer; /* OR_OPT_* */
    int64_t dx, dy;    /* CCA: d = dx + dy; GENERAL: dx = dy = d; LDA: dx = d */
    double eps_reg;    /* ridge added to B (GENERAL, LDA): B = E[...] + eps I */
    double rho;        /* clip of <v_j, [Bv]_j> (Alg. 2) */
    double adam_b1, adam_b2, adam_eps;
    const double *class_means;  /* LDA: n_classes x d, row-major */
    const double *class_priors; /* LDA: n_classes */
    int32_t smooth;    /* 0: Alg. 2 (clip at rho); 1: Alg. 3 (smooth estimate) */
    int32_t pad;
    double nu;         /* Alg. 3: upper bound of lambda_max(B), nu > rho > 0 */
} oracle_problem;

static int64_t problem_dim(const oracle_problem *pb)
{
    return pb->kind == OR_KIND_CCA ? pb->dx + pb->dy : pb->dx;
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += a[i] * b[i];
    return s;
}

/* Minibatch estimates A_t v and B_t v for one vector v (length d), as explicit
 * sums over the b rows of the minibatch with the 1/b mean normalisation of
 * Sec. 1 ((1/n) X^T X).  CCA: the block matrices of Sec. 1 with expectations
 * replaced by minibatch means.  GENERAL: A = E[y y^T], B = E[x x^T] + eps I.
 * LDA: B = within-class covariance E[(x - mu_l)(x - mu_l)^T] + eps I,
 * A = between-class covariance sum_c pi_c (mu_c - mu)(mu_c - mu)^T with
 * mu = sum_c pi_c mu_c (exact: class means and priors are given). */
static void minibatch_products(const oracle_problem *pb, int64_t b,
                               const double *X, int64_t ldx, const double *Y, int64_t ldy,
                               const int32_t *labels, const double *v, double *Av, double *Bv,
                               double *tmp /* length d */)
{
    int64_t d = problem_dim(pb);
    memset(Av, 0, (size_t)d * sizeof(double));
    memset(Bv, 0, (size_t)d * sizeof(double));
    if (pb->kind == OR_KIND_CCA) {
        int64_t dx = pb->dx, dy = pb->dy;
        const double *vx = v, *vy = v + dx;
        for (int64_t r = 0; r < b; ++r) {
            const double *x = X + r * ldx, *y = Y + r * ldy;
            double px = dot(dx, x, vx), py = dot(dy, y, vy);
            for (int64_t f = 0; f < dx; ++f) {
                Av[f] += x[f] * py;
                Bv[f] += x[f] * px;
            }
            for (int64_t f = 0; f < dy; ++f) {
                Av[dx + f] += y[f] * px;
                Bv[dx + f] += y[f] * py;
            }
        }
        for (int64_t f = 0; f < d; ++f) {
            Av[f] /= (double)b;
            Bv[f] /= (double)b;
        }
    } else if (pb->kind == OR_KIND_GENERAL) {
        for (int64_t r = 0; r < b; ++r) {
            const double *x = X + r * ldx, *y = Y + r * ldy;
            double px = dot(d, x, v), py = dot(d, y, v);
            for (int64_t f = 0; f < d; ++f) {
                Av[f] += y[f] * py;
                Bv[f] += x[f] * px;
            }
        }
        for (int64_t f = 0; f < d; ++f) {
            Av[f] /= (double)b;
            Bv[f] = Bv[f] / (double)b + pb->eps_reg * v[f];
        }
    } else if (pb->kind == OR_KIND_ICA) {
        /* ICA in its kurtosis form (Sec. 1): with C_t = (1/b) sum_r x_r x_r^T,
         *   A_t v = (1/b) sum_r ||x_r||^2 x_r (x_r^T v) - tr(C_t) C_t v - 2 C_t (C_t v)
         *   B_t v = C_t v + eps v
         * all from the one minibatch; C_t (C_t v) is a second pass over the rows. */
        double *Cv = tmp, tr = 0.0;
        memset(Cv, 0, (size_t)d * sizeof(double));
        for (int64_t r = 0; r < b; ++r) {
            const double *x = X + r * ldx;
            double nr = dot(d, x, x), p = dot(d, x, v);
            tr += nr;
            for (int64_t f = 0; f < d; ++f) {
                Cv[f] += x[f] * p;
                Av[f] += nr * x[f] * p;
            }
        }
        tr /= (double)b;
        for (int64_t f = 0; f < d; ++f) {
            Cv[f] /= (double)b;
            Av[f] /= (double)b;
        }
        for (int64_t r = 0; r < b; ++r) {
            const double *x = X + r * ldx;
            double q = dot(d, x, Cv);
            for (int64_t f = 0; f < d; ++f)
                Av[f] -= 2.0 * x[f] * q / (double)b;
        }
        for (int64_t f = 0; f < d; ++f) {
            Av[f] -= tr * Cv[f];
            Bv[f] = Cv[f] + pb->eps_reg * v[f];
        }
    } else { /* LDA */
        int c = pb->n_classes;
        for (int64_t r = 0; r < b; ++r) {
            const double *x = X + r * ldx;
            const double *mu = pb->class_means + (size_t)labels[r] * d;
            for (int64_t f = 0; f < d; ++f)
                tmp[f] = x[f] - mu[f];
            double pe = dot(d, tmp, v);
            for (int64_t f = 0; f < d; ++f)
                Bv[f] += tmp[f] * pe;
        }
        for (int64_t f = 0; f < d; ++f)
            Bv[f] = Bv[f] / (double)b + pb->eps_reg * v[f];
        /* overall mean */
        double *mbar = tmp;
        memset(mbar, 0, (size_t)d * sizeof(double));
        for (int cc = 0; cc < c; ++cc)
            for (int64_t f = 0; f < d; ++f)
                mbar[f] += pb->class_priors[cc] * pb->class_means[(size_t)cc * d + f];
        for (int cc = 0; cc < c; ++cc) {
            const double *mu = pb->class_means + (size_t)cc * d;
            double pm = 0.0;
            for (int64_t f = 0; f < d; ++f)
                pm += (mu[f] - mbar[f]) * v[f];
            for (int64_t f = 0; f < d; ++f)
                Av[f] += pb->class_priors[cc] * (mu[f] - mbar[f]) * pm;
        }
    }
}

/* The body of Alg. 2 once A_t v_i and B_t v_i are known for every player.
 * All players read the same V_t and G_t (the parfor over players); the
 * auxiliary update uses B_t v_i of the pre-step vector.
 *   V     : in/out, d x k column-major, unit columns on entry and exit
 *   G     : in/out, the auxiliary [Bv], d x k column-major
 *   AV,BV : A_t v_i, B_t v_i, d x k column-major
 *   m, s2 : Adam first and second moments (d x k) or NULL for SGD
 *   t     : iteration number (1-based; Adam bias correction)
 *   ema_a, ema_b : running means of v_i^T A_t v_i and v_i^T B_t v_i at rate
 *           gamma (eigenvalue readout lambda_i = ema_a / ema_b), may be NULL
 *   grad_out : optional d x k copy of the update direction (tests)
 *   z     : Alg. 3 only (pb->smooth): the k log-space variables z_j, in/out
 * Returns the number of parents whose <v_j, [Bv]_j> was clipped at rho
 * (Alg. 2; always 0 for Alg. 3). */
static int alg2_body(const oracle_problem *pb, int64_t d, double *V, double *G,
                     const double *AV, const double *BV, double eta, double gamma, double t,
                     double *m, double *s2, double *ema_a, double *ema_b, double *grad_out,
                     double *z)
{
    int k = pb->k;
    double *s = (double *)malloc((size_t)k * sizeof(double));
    double *vgs = (double *)malloc((size_t)k * sizeof(double));
    double *Vn = (double *)malloc((size_t)d * k * sizeof(double));
    int clipped = 0;
    const double lrho = log(pb->rho), lspan = log(pb->nu) - log(pb->rho);
    for (int j = 0; j < k; ++j) {
        double vg = dot(d, V + (size_t)j * d, G + (size_t)j * d);
        vgs[j] = vg;
        if (pb->smooth) {
            /* Alg. 3: [<v, B v>]_j = exp(log rho + (log nu - log rho) sigmoid(z_j)) */
            double sg = 1.0 / (1.0 + exp(-z[j]));
            s[j] = exp(lrho + lspan * sg);
        } else {
            /* Alg. 2: s_j = max(<v_j, [Bv]_j>, rho), the clipped estimate of ||v_j||_B^2 */
            if (vg < pb->rho) {
                vg = pb->rho;
                ++clipped;
            }
            s[j] = vg;
        }
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < k; ++i) {
        const double *vi = V + (size_t)i * d;
        const double *Avi = AV + (size_t)i * d, *Bvi = BV + (size_t)i * d;
        double *gi = Vn + (size_t)i * d; /* holds the direction first */
        double vBv = dot(d, vi, Bvi);
        double vAv = dot(d, vi, Avi);
        /* rewards: (v_i^T B v_i) A v_i - (v_i^T A v_i) B v_i */
        for (int64_t f = 0; f < d; ++f)
            gi[f] = vBv * Avi[f] - vAv * Bvi[f];
        /* penalties: sum over parents j < i of
         *   (v_i^T A y_j) [ <v_i, B v_i> [By]_j - <v_i, [By]_j> B v_i ]
         * with y_j = v_j / sqrt(s_j) and [By]_j = [Bv]_j / sqrt(s_j) */
        for (int j = 0; j < i; ++j) {
            double rs = 1.0 / sqrt(s[j]);
            const double *Avj = AV + (size_t)j * d; /* A_t v_j, so A_t y_j = rs * A_t v_j */
            const double *gj = G + (size_t)j * d;
            double viAyj = rs * dot(d, vi, Avj);
            double viByj = rs * dot(d, vi, gj);
            for (int64_t f = 0; f < d; ++f)
                gi[f] -= viAyj * (vBv * rs * gj[f] - viByj * Bvi[f]);
        }
        if (ema_a) {
            ema_a[i] += gamma * (vAv - ema_a[i]);
            ema_b[i] += gamma * (vBv - ema_b[i]);
        }
    }
    if (grad_out)
        memcpy(grad_out, Vn, (size_t)d * k * sizeof(double));
    /* Riemannian step: v_i' = v_i + eta * direction, then back to the sphere;
     * the Adam variant feeds the direction to Adam as an ascent gradient. */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < k; ++i) {
        double *vi = V + (size_t)i * d;
        double *gi = Vn + (size_t)i * d;
        if (pb->optimizer == OR_OPT_ADAM) {
            double *mi = m + (size_t)i * d, *si = s2 + (size_t)i * d;
            double c1 = 1.0 - pow(pb->adam_b1, t), c2 = 1.0 - pow(pb->adam_b2, t);
            for (int64_t f = 0; f < d; ++f) {
                mi[f] = pb->adam_b1 * mi[f] + (1.0 - pb->adam_b1) * gi[f];
                si[f] = pb->adam_b2 * si[f] + (1.0 - pb->adam_b2) * gi[f] * gi[f];
                gi[f] = vi[f] + eta * (mi[f] / c1) / (sqrt(si[f] / c2) + pb->adam_eps);
            }
        } else {
            for (int64_t f = 0; f < d; ++f)
                gi[f] = vi[f] + eta * gi[f];
        }
        double nrm = sqrt(dot(d, gi, gi));
        for (int64_t f = 0; f < d; ++f)
            gi[f] /= nrm;
    }
    /* auxiliary variable: [Bv]_i <- [Bv]_i + gamma (B_t v_i - [Bv]_i) */
    for (int i = 0; i < k; ++i) {
        double *gi = G + (size_t)i * d;
        const double *Bvi = BV + (size_t)i * d;
        for (int64_t f = 0; f < d; ++f)
            gi[f] += gamma * (Bvi[f] - gi[f]);
    }
    /* Alg. 3: z_i <- z_i + gamma grad_z, grad_z = (<v_i, [Bv]_i> - s_i) s_i
     * (log nu - log rho) sigmoid(z_i) (1 - sigmoid(z_i)), with v_i, [Bv]_i and
     * s_i of this iteration (before the updates above) */
    if (pb->smooth)
        for (int i = 0; i < k; ++i) {
            double sg = 1.0 / (1.0 + exp(-z[i]));
            z[i] += gamma * (vgs[i] - s[i]) * s[i] * lspan * sg * (1.0 - sg);
        }
    memcpy(V, Vn, (size_t)d * k * sizeof(double));
    free(s);
    free(vgs);
    free(Vn);
    return clipped;
}

/* One iteration of Alg. 2 (M = 1) on the minibatch (X, Y[, labels]) of b rows.
 * See alg2_body for V, G, m, s2, ema_a, ema_b, grad_out.  Returns the clip
 * count, or -1 on allocation failure. */
int oracle_gamma_step(const oracle_problem *pb, int64_t b,
                      const double *X, int64_t ldx, const double *Y, int64_t ldy,
                      const int32_t *labels, double *V, double *G, double eta, double gamma,
                      double t, double *m, double *s2, double *ema_a, double *ema_b,
                      double *grad_out, double *z)
{
    int64_t d = problem_dim(pb);
    int k = pb->k;
    double *AV = (double *)malloc((size_t)d * k * sizeof(double));
    double *BV = (double *)malloc((size_t)d * k * sizeof(double));
    if (!AV || !BV) {
        free(AV);
        free(BV);
        return -1;
    }
#pragma omp parallel
    {
        double *tmp = (double *)malloc((size_t)d * sizeof(double));
#pragma omp for schedule(static)
        for (int i = 0; i < k; ++i)
            minibatch_products(pb, b, X, ldx, Y, ldy, labels, V + (size_t)i * d,
                               AV + (size_t)i * d, BV + (size_t)i * d, tmp);
        free(tmp);
    }
    int rc = alg2_body(pb, d, V, G, AV, BV, eta, gamma, t, m, s2, ema_a, ema_b, grad_out, z);
    free(AV);
    free(BV);
    return rc;
}

/* Alg. 2 iteration with exact A and B (d x d row-major): the full-batch case,
 * A_t = A, B_t = B.  Used for the fixed-point and consistency pins. */
int oracle_gamma_step_dense(const oracle_problem *pb, int64_t d, const double *A, const double *B,
                            double *V, double *G, double eta, double gamma, double t,
                            double *m, double *s2, double *ema_a, double *ema_b, double *grad_out,
                            double *z)
{
    int k = pb->k;
    double *AV = (double *)malloc((size_t)d * k * sizeof(double));
    double *BV = (double *)malloc((size_t)d * k * sizeof(double));
    if (!AV || !BV) {
        free(AV);
        free(BV);
        return -1;
    }
    for (int i = 0; i < k; ++i)
        for (int64_t r = 0; r < d; ++r) {
            AV[(size_t)i * d + r] = dot(d, A + (size_t)r * d, V + (size_t)i * d);
            BV[(size_t)i * d + r] = dot(d, B + (size_t)r * d, V + (size_t)i * d);
        }
    int rc = alg2_body(pb, d, V, G, AV, BV, eta, gamma, t, m, s2, ema_a, ema_b, grad_out, z);
    free(AV);
    free(BV);
    return rc;
}

/* One iteration of Alg. 1 (deterministic): y_j = v_j / sqrt(v_j^T B v_j) with
 * exact B, rewards and penalties as in the update direction of Sec. 3, then
 * the retraction step.  V in/out d x k column-major with unit columns. */
int oracle_alg1_step(int64_t d, int k, const double *A, const double *B, double *V, double eta,
                     double *grad_out)
{
    double *AV = (double *)malloc((size_t)d * k * sizeof(double));
    double *BV = (double *)malloc((size_t)d * k * sizeof(double));
    double *Vn = (double *)malloc((size_t)d * k * sizeof(double));
    if (!AV || !BV || !Vn) {
        free(AV);
        free(BV);
        free(Vn);
        return -1;
    }
    for (int i = 0; i < k; ++i)
        for (int64_t r = 0; r < d; ++r) {
            AV[(size_t)i * d + r] = dot(d, A + (size_t)r * d, V + (size_t)i * d);
            BV[(size_t)i * d + r] = dot(d, B + (size_t)r * d, V + (size_t)i * d);
        }
    for (int i = 0; i < k; ++i) {
        const double *vi = V + (size_t)i * d, *Avi = AV + (size_t)i * d, *Bvi = BV + (size_t)i * d;
        double *gi = Vn + (size_t)i * d;
        double vBv = dot(d, vi, Bvi), vAv = dot(d, vi, Avi);
        for (int64_t f = 0; f < d; ++f)
            gi[f] = vBv * Avi[f] - vAv * Bvi[f];
        for (int j = 0; j < i; ++j) {
            const double *vj = V + (size_t)j * d;
            double rs = 1.0 / sqrt(dot(d, vj, BV + (size_t)j * d)); /* 1 / ||v_j||_B */
            double viAyj = rs * dot(d, vi, AV + (size_t)j * d);
            double viByj = rs * dot(d, vi, BV + (size_t)j * d);
            for (int64_t f = 0; f < d; ++f)
                gi[f] -= viAyj * (vBv * rs * BV[(size_t)j * d + f] - viByj * Bvi[f]);
        }
    }
    if (grad_out)
        memcpy(grad_out, Vn, (size_t)d * k * sizeof(double));
    for (int i = 0; i < k; ++i) {
        double *gi = Vn + (size_t)i * d;
        const double *vi = V + (size_t)i * d;
        for (int64_t f = 0; f < d; ++f)
            gi[f] = vi[f] + eta * gi[f];
        double nrm = sqrt(dot(d, gi, gi));
        for (int64_t f = 0; f < d; ++f)
            gi[f] /= nrm;
    }
    memcpy(V, Vn, (size_t)d * k * sizeof(double));
    free(AV);
    free(BV);
    free(Vn);
    return 0;
}

/* Library self-description for the Python loader. */
int oracle_abi_version(void) { return 1; }

/* Threads an OpenMP region of this library uses (for the CPU baseline). */
#ifdef _OPENMP
#include <omp.h>
#endif
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
