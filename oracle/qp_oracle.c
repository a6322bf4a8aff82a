/*
 * Reference (oracle) implementation of the projection method for
 * quasiperiodic elliptic problems  -div(a grad u) = f,  a(x) = A(P^T x).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously-correct
 * CPU reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header or table with the GPU library.
 *
 * Everything is IEEE double precision, complex numbers are C99 `double complex`
 * (interleaved re,im in memory).  Each routine cites the passage of the paper
 * it follows (Jiang, Li, Zhang, Zhang, "Projection method for quasiperiodic
 * elliptic equations and application to quasiperiodic homogenization").
 *
 * Readings taken where the paper is silent (also listed in the design notes):
 *  - k_V -_N k_U is the componentwise difference mod N; the weight W uses the
 *    representatives k_V, k_U in K_N^n (eq. n-discrete).
 *  - The zero frequency is excluded from trial and test space (Sec. 3.1.1,
 *    zero-mean space): U_0 = 0 and F_0 is ignored.
 *  - M is an approximate inverse (eq. precond), so "solve M z = r" in Alg. 2 is
 *    applied as z = M r; |q_ij|^2 is used in the column norms.
 *  - "until convergence" is ||r||_2 <= tol * ||F'||_2 with U_0 = 0, where F' is
 *    F with the zero frequency removed.
 *  - Inner products are (x, y) = y^H x; for the Hermitian positive definite Q
 *    the PCG scalars are real and their real parts are used.
 *
 * parity pins: see the oracle tests (closed forms, brute force, invariants).
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int d;                /* physical dimension                          */
    int n;                /* parent (lifted) dimension                   */
    int N;                /* points per parent dimension, D = N^n        */
    int g;                /* number of coefficient modes                 */
    const double *P;      /* d x n projection matrix, row-major          */
    const int *modes;     /* g x n integer modes m                       */
    const double *coef;   /* g complex coefficients Ahat_m (re, im)      */
    const double *coefs;  /* NULL (scalar coefficient a), or a diagonal
                             coefficient diag(a_1..a_d) (App. D): d x g
                             complex, Ahat of a_l at mode r at (l g + r)   */
} qo_problem;

/* D = N^n */
/* OpenMP threads of the routines below (timing only; no arithmetic). */
void qo_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
}

int qo_max_threads(void)
{
    return omp_get_max_threads();
}

long qo_size(int n, int N)
{
    long D = 1;
    for (int t = 0; t < n; ++t) D *= N;
    return D;
}

/* Representative in K_N^1 = {-N/2 <= k < N/2} of the class x mod N
 * (inverse conversion, Sec. 3.1.2: i_k = ibar_k if ibar_k < N/2, else ibar_k - N). */
int qo_rep(int N, long x)
{
    long r = x % N;
    if (r < 0) r += N;
    return (2 * r < N) ? (int)r : (int)(r - N);
}

/* Tensor-to-vector conversion C (Sec. 3.1.2, eq. conversion):
 * i = sum_k (i_k mod N) * N^(n-k), first index slowest. */
long qo_index(int n, int N, const int *k)
{
    long i = 0;
    for (int t = 0; t < n; ++t) {
        long b = k[t] % N;
        if (b < 0) b += N;
        i = i * N + b;
    }
    return i;
}

/* Inverse conversion C^{-1} (Sec. 3.1.2, eq. inverse_convert):
 * ibar_k = floor((i mod N^(n-k+1)) / N^(n-k)), then shift to K_N. */
void qo_multi_index(int n, int N, long i, int *k)
{
    for (int t = n - 1; t >= 0; --t) {
        long b = i % N;
        i /= N;
        k[t] = (2 * b < N) ? (int)b : (int)(b - N);
    }
}

/* P k for an integer vector k (d values). */
static void proj(const qo_problem *p, const int *k, double *out)
{
    for (int l = 0; l < p->d; ++l) {
        double s = 0.0;
        for (int t = 0; t < p->n; ++t) s += p->P[l * p->n + t] * (double)k[t];
        out[l] = s;
    }
}

static double dotd(int d, const double *a, const double *b)
{
    double s = 0.0;
    for (int l = 0; l < d; ++l) s += a[l] * b[l];
    return s;
}

static double complex coef_at(const qo_problem *p, int r)
{
    return p->coef[2 * r] + I * p->coef[2 * r + 1];
}

/* Ahat of the l-th diagonal entry a_l at mode r (the scalar a when there is
 * no diagonal coefficient). */
static double complex coef_l(const qo_problem *p, int r, int l)
{
    if (!p->coefs) return coef_at(p, r);
    const double *c = p->coefs + 2 * ((long)l * p->g + r);
    return c[0] + I * c[1];
}

/* Index of the mode congruent to `k` mod N, or -1 when no mode is. */
static int mode_of_class(const qo_problem *p, const int *k)
{
    for (int r = 0; r < p->g; ++r) {
        int same = 1;
        for (int t = 0; t < p->n; ++t)
            if (qo_rep(p->N, (long)k[t] - p->modes[r * p->n + t]) != 0) { same = 0; break; }
        if (same) return r;
    }
    return -1;
}

/* Ahat for the mode congruent to `k` mod N, or 0 when no mode is. */
static double complex coef_of_class(const qo_problem *p, const int *k)
{
    const int r = mode_of_class(p, k);
    return (r < 0) ? 0.0 : coef_at(p, r);
}

/* The same for the diagonal entry a_l. */
static double complex coef_of_class_l(const qo_problem *p, const int *k, int l)
{
    const int r = mode_of_class(p, k);
    return (r < 0) ? 0.0 : coef_l(p, r, l);
}

static int is_zero(int n, const int *k)
{
    for (int t = 0; t < n; ++t) if (k[t] != 0) return 0;
    return 1;
}

/* Stiffness product y = Q u with Q = A o W (Sec. 3.1.2, eq. linear_system):
 *   y_{k_V} = sum_{k_U in K_N^n} Ahat_{k_V -_N k_U} (P k_V).(P k_U) U_{k_U}
 * (eq. n-discrete).  Only the g nonzero Ahat contribute: for a mode m the
 * column is the k_U in K_N^n congruent to k_V - m.  Row k_V = 0 is not part of
 * the test space and is returned as 0. */
static double complex matvec_row(const qo_problem *p, const double complex *u, long i)
{
    int kv[8], ku[8];
    double pkv[8], pku[8];
    qo_multi_index(p->n, p->N, i, kv);
    if (is_zero(p->n, kv)) return 0.0;
    proj(p, kv, pkv);
    double complex acc = 0.0;
    for (int r = 0; r < p->g; ++r) {
        for (int t = 0; t < p->n; ++t)
            ku[t] = qo_rep(p->N, (long)kv[t] - p->modes[r * p->n + t]);
        proj(p, ku, pku);
        const double complex uj = u[qo_index(p->n, p->N, ku)];
        if (!p->coefs) {
            const double w = dotd(p->d, pkv, pku);
            acc += coef_at(p, r) * w * uj;
        } else {
            /* diagonal coefficient (App. D): Q = sum_l A^l o W^l with
             * W^l = (P k_V)_l (P k_U)_l */
            for (int l = 0; l < p->d; ++l) acc += coef_l(p, r, l) * (pkv[l] * pku[l]) * uj;
        }
    }
    return acc;
}

void qo_matvec(const qo_problem *p, const double *u_, double *y_)
{
    const double complex *u = (const double complex *)u_;
    double complex *y = (double complex *)y_;
    const long D = qo_size(p->n, p->N);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < D; ++i) y[i] = matvec_row(p, u, i);
}

/* The same product at the listed rows only: y[j] = (Q u)_{rows[j]}. */
void qo_matvec_rows(const qo_problem *p, const double *u_, long nrows, const long *rows,
                    double *y_)
{
    const double complex *u = (const double complex *)u_;
    double complex *y = (double complex *)y_;
    for (long j = 0; j < nrows; ++j) y[j] = matvec_row(p, u, rows[j]);
}

/* Diagonal preconditioner.
 * kind 0: the Frobenius-optimal M = argmin ||Q M - I||_F over diagonal M
 *         (eq. precond, Theorem): M_jj = q_jj / ||Q e_j||_2^2, with
 *         q_jj = Ahat_0 |P k_j|^2 and ||Q e_j||^2 = sum_rows |q_ij|^2.
 *         Column j has entries in the rows k_i congruent to k_j + m for each
 *         mode m, with value Ahat_m (P k_i).(P k_j).
 * kind 1: Jacobi, M_jj = 1 / q_jj.
 * M_00 = 0 (frequency 0 is not an unknown). */
void qo_precond(const qo_problem *p, int kind, double *M)
{
    const long D = qo_size(p->n, p->N);
    int zero[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const double a0 = creal(coef_of_class(p, zero));
    double a0l[8];  /* diagonal coefficient: q_jj = sum_l Ahat^l_0 (P k_j)_l^2 */
    for (int l = 0; l < p->d; ++l) a0l[l] = creal(coef_of_class_l(p, zero, l));
#pragma omp parallel for schedule(static)
    for (long j = 0; j < D; ++j) {
        int kj[8], ki[8];
        double pkj[8], pki[8];
        qo_multi_index(p->n, p->N, j, kj);
        if (is_zero(p->n, kj)) { M[j] = 0.0; continue; }
        proj(p, kj, pkj);
        double qjj = a0 * dotd(p->d, pkj, pkj);
        if (p->coefs) {
            qjj = 0.0;
            for (int l = 0; l < p->d; ++l) qjj += a0l[l] * pkj[l] * pkj[l];
        }
        if (kind == 1) { M[j] = (qjj != 0.0) ? 1.0 / qjj : 0.0; continue; }
        double colnorm2 = 0.0;
        for (int r = 0; r < p->g; ++r) {
            for (int t = 0; t < p->n; ++t)
                ki[t] = qo_rep(p->N, (long)kj[t] + p->modes[r * p->n + t]);
            proj(p, ki, pki);
            double complex q = coef_at(p, r) * dotd(p->d, pki, pkj);
            if (p->coefs) {
                q = 0.0;
                for (int l = 0; l < p->d; ++l) q += coef_l(p, r, l) * (pki[l] * pkj[l]);
            }
            colnorm2 += creal(q) * creal(q) + cimag(q) * cimag(q);
        }
        M[j] = (colnorm2 != 0.0) ? qjj / colnorm2 : 0.0;
    }
}

/* (x, y) = y^H x */
static double complex inner(long D, const double complex *x, const double complex *y)
{
    double re = 0.0, im = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : re, im)
    for (long i = 0; i < D; ++i) {
        const double complex v = x[i] * conj(y[i]);
        re += creal(v);
        im += cimag(v);
    }
    return re + I * im;
}

/* C-PCG, Alg. 2, started from U_0 = 0:
 *   r_0 = F', z_0 = M r_0, h_0 = z_0;
 *   alpha = (r,z)/(Qh,h); U += alpha h; r -= alpha Qh; z = M r;
 *   beta = (r+,z+)/(r,z); h = z + beta h;
 * until ||r|| <= tol ||F'||.  Returns 0 on convergence, 1 when maxit steps
 * did not converge, 2 when (Qh,h) <= 0 (Q not positive definite).
 * `iters` = number of U updates performed, `relres` = final ||r||/||F'||.
 * ab (NULL or 2 maxit doubles): the scalars of every step, alpha of step j
 * at ab[2j] and the beta that follows it at ab[2j+1] (not written after the
 * last step). */
int qo_pcg_ex(const qo_problem *p, int kind, const double *F_, double *U_,
              double tol, int maxit, int *iters, double *relres, double *ab)
{
    const long D = qo_size(p->n, p->N);
    double complex *U = (double complex *)U_;
    double complex *r = malloc(sizeof(double complex) * D);
    double complex *z = malloc(sizeof(double complex) * D);
    double complex *h = malloc(sizeof(double complex) * D);
    double complex *q = malloc(sizeof(double complex) * D);
    double *M = malloc(sizeof(double) * D);
    int status = 1, it = 0;

    qo_precond(p, kind, M);
    memcpy(r, F_, sizeof(double complex) * D);
    r[0] = 0.0;                                   /* F' : no zero frequency */
    for (long i = 0; i < D; ++i) { U[i] = 0.0; z[i] = M[i] * r[i]; h[i] = z[i]; }
    const double fnorm = sqrt(creal(inner(D, r, r)));
    double rnorm = fnorm;
    if (fnorm == 0.0) { status = 0; goto done; }
    double rz = creal(inner(D, r, z));
    while (it < maxit) {
        qo_matvec(p, (const double *)h, (double *)q);
        const double hq = creal(inner(D, q, h));   /* (Qh, h) */
        if (!(hq > 0.0)) { status = 2; break; }
        const double alpha = rz / hq;
        if (ab) ab[2 * it] = alpha;
        for (long i = 0; i < D; ++i) {
            U[i] += alpha * h[i];
            r[i] -= alpha * q[i];
            z[i] = M[i] * r[i];
        }
        ++it;
        rnorm = sqrt(creal(inner(D, r, r)));
        if (rnorm <= tol * fnorm) { status = 0; break; }
        const double rz_new = creal(inner(D, r, z));
        const double beta = rz_new / rz;
        if (ab) ab[2 * (it - 1) + 1] = beta;
        rz = rz_new;
        for (long i = 0; i < D; ++i) h[i] = z[i] + beta * h[i];
    }
done:
    if (iters) *iters = it;
    if (relres) *relres = (fnorm > 0.0) ? rnorm / fnorm : 0.0;
    free(r); free(z); free(h); free(q); free(M);
    return status;
}

int qo_pcg(const qo_problem *p, int kind, const double *F_, double *U_,
           double tol, int maxit, int *iters, double *relres)
{
    return qo_pcg_ex(p, kind, F_, U_, tol, maxit, iters, relres, NULL);
}

/* Discrete Fourier-Bohr transform on the collocation grid T_N^n (Sec. 2.3):
 * the coefficients of values f_j sampled at y_j = 2 pi j / N (j in
 * {0..N-1}^n) are  Fhat_k = (1/D) sum_j f_j exp(-i k.y_j),  and the samples
 * of a coefficient vector are  f_j = sum_k Fhat_k exp(i k.y_j).  Both vectors
 * are in the storage order of Sec. 3.1.2 (entry i holds the multi-index with
 * digits of i in base N, first axis slowest; for coefficients the digits are
 * k mod N, which gives the same exp(i k.y_j)).  The phase k.y_j is taken as
 * 2 pi ((sum_t k_t j_t) mod N) / N with the integer product reduced exactly.
 * Evaluated straight from the definition, one output at a time (O(D) per
 * output): out[r] is the transform at storage index rows[r]. */
void qo_dft_rows(int n, int N, int inverse, const double *in_, long nrows, const long *rows,
                 double *out_)
{
    const double complex *in = (const double complex *)in_;
    double complex *out = (double complex *)out_;
    const long D = qo_size(n, N);
    const double sign = inverse ? 1.0 : -1.0;
    const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(dynamic, 1)
    for (long r = 0; r < nrows; ++r) {
        int k[8], j[8];
        long i = rows[r];
        for (int t = n - 1; t >= 0; --t) { k[t] = (int)(i % N); i /= N; }
        double complex acc = 0.0;
        for (long s = 0; s < D; ++s) {
            long rest = s;
            for (int t = n - 1; t >= 0; --t) { j[t] = (int)(rest % N); rest /= N; }
            long ph = 0;
            for (int t = 0; t < n; ++t) ph = (ph + (long)k[t] * j[t]) % N;
            const double th = sign * two_pi * (double)ph / (double)N;
            acc += in[s] * (cos(th) + I * sin(th));
        }
        out[r] = inverse ? acc : acc / (double)D;
    }
}

/* Right-hand side of the corrector equation -div(a(e_j + grad chi)) = 0, i.e.
 * -div(a grad chi) = d a / d x_j (Sec. 5.2, eq. corrector; App. D, f_1 = d_x1 alpha).
 * The x_j-derivative of exp(i (P k).x) is i (P k)_j exp(i (P k).x), so
 * F_k = i (P k)_j Ahat_k on the coefficient's modes and 0 elsewhere.  For a
 * diagonal coefficient the source is d a_j / d x_j (App. D: f_1 = d_x1 alpha,
 * f_2 = d_x2 beta), so Ahat is that of a_j. */
void qo_corrector_rhs(const qo_problem *p, int j, double *F_)
{
    double complex *F = (double complex *)F_;
    const long D = qo_size(p->n, p->N);
    double pk[8];
    for (long i = 0; i < D; ++i) F[i] = 0.0;
    for (int r = 0; r < p->g; ++r) {
        const int *m = p->modes + r * p->n;
        proj(p, m, pk);
        F[qo_index(p->n, p->N, m)] += I * pk[j] * coef_l(p, r, j);
    }
}

/* Homogenized coefficient, flux form (Sec. 5.2, eq. homcoefficient):
 *   A*_ij = mean{ e_i . a (e_j + grad chi_j) }
 *         = Ahat_0 delta_ij + mean{ a d_{x_i} chi_j }.
 * With the discrete mean mean_N{g} = (1/D) sum over the collocation grid
 * (Sec. 2.3), the product of the two trigonometric polynomials keeps the
 * frequency pairs whose sum is 0 mod N:
 *   mean_N{a d_i chi} = sum_{k in K_N^n} Ahat_{class(-k)} * i (P k)_i * chi_k.
 * For a diagonal coefficient e_i . A (e_j + grad chi_j) = a_i (delta_ij +
 * d_{x_i} chi_j) (App. D, eqs. homcoefficient11-22), so Ahat is that of a_i.
 * Returns the real part; *imag receives the imaginary part (0 for real a). */
double qo_astar_flux(const qo_problem *p, int i_, int j_, const double *chi_, double *imag)
{
    const double complex *chi = (const double complex *)chi_;
    const long D = qo_size(p->n, p->N);
    int zero[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double complex acc = (i_ == j_) ? coef_of_class_l(p, zero, i_) : 0.0;
    double re = 0.0, im = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : re, im)
    for (long idx = 0; idx < D; ++idx) {
        int k[8], mk[8];
        double pk[8];
        qo_multi_index(p->n, p->N, idx, k);
        for (int t = 0; t < p->n; ++t) mk[t] = -k[t];
        const double complex am = coef_of_class_l(p, mk, i_);
        if (am == 0.0) continue;
        proj(p, k, pk);
        const double complex v = am * I * pk[i_] * chi[idx];
        re += creal(v);
        im += cimag(v);
    }
    acc += re + I * im;
    if (imag) *imag = cimag(acc);
    return creal(acc);
}

/* Homogenized coefficient, energy form: A*_ij = Ahat_0 delta_ij - chi_i^H Q chi_j
 * (equal to the flux form at the exact discrete corrector since Q chi_j = F_j
 * and Q is Hermitian; symmetric by construction).  For a diagonal coefficient
 * the first term is the mean of A, Ahat^i_0 delta_ij. */
double qo_astar_energy(const qo_problem *p, int i_, int j_, const double *chi_i_,
                       const double *chi_j_, double *imag)
{
    const long D = qo_size(p->n, p->N);
    int zero[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double complex *q = malloc(sizeof(double complex) * D);
    qo_matvec(p, chi_j_, (double *)q);
    const double complex e = inner(D, q, (const double complex *)chi_i_); /* chi_i^H Q chi_j */
    free(q);
    const double complex a = ((i_ == j_) ? coef_of_class_l(p, zero, i_) : 0.0) - e;
    if (imag) *imag = cimag(a);
    return creal(a);
}

/* Minimum and maximum of A(y) = sum_m Ahat_m exp(i m.y) over the collocation
 * grid y_j = 2 pi j / N (Sec. 2.3); used for the ellipticity check.  For a
 * diagonal coefficient: the extrema over every entry a_l. */
void qo_coef_extrema(const qo_problem *p, double *amin, double *amax)
{
    const long D = qo_size(p->n, p->N);
    double lo = INFINITY, hi = -INFINITY;
#pragma omp parallel for schedule(static) reduction(min : lo) reduction(max : hi)
    for (long idx = 0; idx < D; ++idx) {
        long rest = idx;
        double y[8];
        for (int t = p->n - 1; t >= 0; --t) {
            y[t] = 2.0 * M_PI * (double)(rest % p->N) / (double)p->N;
            rest /= p->N;
        }
        const int nl = p->coefs ? p->d : 1;
        for (int l = 0; l < nl; ++l) {
            double complex a = 0.0;
            for (int r = 0; r < p->g; ++r) {
                double ph = 0.0;
                for (int t = 0; t < p->n; ++t) ph += p->modes[r * p->n + t] * y[t];
                a += coef_l(p, r, l) * cexp(I * ph);
            }
            const double v = creal(a);
            if (v < lo) lo = v;
            if (v > hi) hi = v;
        }
    }
    *amin = lo;
    *amax = hi;
}
