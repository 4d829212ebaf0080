/*
 * nep_oracle.c -- plain FP64 CPU reference for the NEP energy / force / virial
 * evaluation and velocity-Verlet MD.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no source with the HIP library.
 *
 * What it computes (Sec. II.A of the paper, Eqs. 2-8; Sec. II.C, Eqs. 15-16):
 *   f_c(r)   = 1/2 [1 + cos(pi r / r_c)]   for r <= r_c, else 0         (Eq. 8)
 *   f_k(r)   = 1/2 [T_k(2 (r/r_c - 1)^2 - 1) + 1] f_c(r),  k = 0..N_bas   (Eq. 7)
 *   g_n(r)   = sum_k c^{t_i t_j}_{nk} f_k(r)                              (Eq. 6)
 *   q_n      = sum_{j != i} g^R_n(r_ij),  n = 0..n_max^R                  (Eq. 3)
 *   A_nlm    = sum_{j != i} g^A_n(r_ij) Y_lm(theta_ij, phi_ij)            (Eq. 5)
 *   q_nl     = sum_m (-1)^m A_nlm A_nl(-m),  l = 1..l_max                 (Eq. 4)
 *   U_i      = sum_mu w1_mu tanh(sum_nu w0_{mu nu} q_nu - b0_mu) - b1      (Eq. 2)
 *   F_i      = sum_j (dU_i/dr_ij - dU_j/dr_ji),   r_ij = r_j - r_i
 *   W_i      = sum_j r_ij (x) dU_j/dr_ji                                   (Eq. 15)
 *   W        = sum_i W_i                                                    (Eq. 16)
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes): Y_lm are the complex orthonormal spherical harmonics with the
 * Condon-Shortley phase; N_bas counts from 0 so there are N_bas+1 basis
 * functions; c is indexed by the ordered type pair (t_i, t_j); the network
 * weights w0, b0, w1 are per centre type with one shared b1; no descriptor
 * scaling; the 4-/5-body angular terms are not part of the descriptor.
 *
 * Arrays: positions (n,3) row-major double; forces (n,3); per-bead virial
 * (n,9) row-major tensor W[a][b] = sum_j (r_ij)_a (dU_j/dr_ji)_b.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_LMAX 8
#define OR_KMAX 32

typedef struct {
    int n_types, n_max_R, n_max_A, basis_R, basis_A, l_max, n_hidden;
    double rc_R[64], rc_A[64]; /* [ti*n_types + tj] */
} or_model;

/* ------------------------------------------------------------------------ */
/* Chebyshev basis with cosine cutoff (Eqs. 6-8) and d/dr                    */
/* ------------------------------------------------------------------------ */
int or_basis(int n_basis, double r, double rc, double *f, double *df)
{
    /* fills k = 0..n_basis; returns 0 when r > rc (all zero) */
    int K = n_basis + 1;
    if (K > OR_KMAX) return -1;
    if (r > rc) {
        for (int k = 0; k < K; ++k) { f[k] = 0.0; df[k] = 0.0; }
        return 0;
    }
    double fc = 0.5 * (1.0 + cos(M_PI * r / rc));
    double dfc = -0.5 * M_PI / rc * sin(M_PI * r / rc);
    double s = r / rc - 1.0;
    double x = 2.0 * s * s - 1.0;
    double dxdr = 4.0 * s / rc;
    /* Chebyshev polynomials of the first kind by their three-term recurrence,
       and their x-derivatives from differentiating that recurrence. */
    double T[OR_KMAX], dT[OR_KMAX];
    T[0] = 1.0; dT[0] = 0.0;
    if (K > 1) { T[1] = x; dT[1] = 1.0; }
    for (int k = 2; k < K; ++k) {
        T[k] = 2.0 * x * T[k - 1] - T[k - 2];
        dT[k] = 2.0 * T[k - 1] + 2.0 * x * dT[k - 1] - dT[k - 2];
    }
    for (int k = 0; k < K; ++k) {
        f[k] = 0.5 * (T[k] + 1.0) * fc;
        df[k] = 0.5 * dT[k] * dxdr * fc + 0.5 * (T[k] + 1.0) * dfc;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* complex spherical harmonics with Condon-Shortley phase                    */
/* Y_lm(u) = K_lm (-1)^m (u_x + i u_y)^m P_l^{(m)}(u_z),  m >= 0,            */
/* Y_l,-m = (-1)^m conj(Y_lm);  P_l^{(m)} is the m-th derivative of the      */
/* Legendre polynomial P_l.  Written as a polynomial in the unit vector, so   */
/* its gradient has no pole; the gradient with respect to the pair vector r  */
/* is (I - u u^T) grad_u Y / |r|.                                            */
/* ------------------------------------------------------------------------ */
static double g_leg[OR_LMAX + 2][OR_LMAX + 2]; /* g_leg[l][p]: coeff of z^p in P_l */
static int g_leg_ready = 0;

static void leg_init(void)
{
    if (g_leg_ready) return;
    memset(g_leg, 0, sizeof g_leg);
    g_leg[0][0] = 1.0;
    g_leg[1][1] = 1.0;
    /* Bonnet: (l+1) P_{l+1} = (2l+1) z P_l - l P_{l-1} */
    for (int l = 1; l <= OR_LMAX; ++l)
        for (int p = 0; p <= l + 1; ++p) {
            double a = (p > 0 ? (2.0 * l + 1.0) * g_leg[l][p - 1] : 0.0);
            double b = l * g_leg[l - 1][p];
            g_leg[l + 1][p] = (a - b) / (l + 1.0);
        }
    g_leg_ready = 1;
}

/* m-th derivative of P_l evaluated at z */
static double leg_deriv(int l, int m, double z)
{
    if (m > l) return 0.0;
    double acc = 0.0;
    for (int p = l; p >= m; --p) {
        double c = g_leg[l][p];
        for (int t = 0; t < m; ++t) c *= (double)(p - t);
        acc = acc * z + c;
    }
    return acc;
}

static double fact(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

/* Y_lm at pair vector d (|d| > 0) and its gradient with respect to d */
void or_ylm(int l, int m, const double d[3], double *re, double *im,
            double *grad_re /*[3] or NULL*/, double *grad_im /*[3] or NULL*/)
{
    leg_init();
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double u[3] = {d[0] / r, d[1] / r, d[2] / r};
    int ma = m < 0 ? -m : m;
    double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * fact(l - ma) / fact(l + ma));
    double sgn = (ma % 2) ? -1.0 : 1.0;
    double complex w = u[0] + I * u[1];
    double complex wm = 1.0, wm1 = 0.0; /* w^m and w^(m-1) by repeated products */
    for (int t = 0; t < ma; ++t) {
        wm1 = wm;
        wm *= w;
    }
    double Dm = leg_deriv(l, ma, u[2]);
    double Dm1 = leg_deriv(l, ma + 1, u[2]);
    double complex Y = K * sgn * wm * Dm;
    double complex gu[3];
    gu[0] = K * sgn * ma * wm1 * Dm;
    gu[1] = K * sgn * ma * I * wm1 * Dm;
    gu[2] = K * sgn * wm * Dm1;
    if (m < 0) {
        Y = sgn * conj(Y);
        for (int a = 0; a < 3; ++a) gu[a] = sgn * conj(gu[a]);
    }
    *re = creal(Y);
    *im = cimag(Y);
    if (grad_re) {
        double complex ug = u[0] * gu[0] + u[1] * gu[1] + u[2] * gu[2];
        for (int a = 0; a < 3; ++a) {
            double complex g = (gu[a] - ug * u[a]) / r;
            grad_re[a] = creal(g);
            grad_im[a] = cimag(g);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* pair enumeration: all (j, image) with |r_j + n L - r_i| < rc_max,         */
/* (j, n) != (i, 0).  Simple cell binning with cells no smaller than rc_max. */
/* ------------------------------------------------------------------------ */
typedef struct {
    int nc[3];
    double lo[3], cs[3];
    int m[3];
    int *head, *next; /* linked cell lists */
} or_cells;

static void cells_build(or_cells *c, int n, const double *pos, const double *box,
                        const int *pbc, double rc)
{
    for (int d = 0; d < 3; ++d) {
        double lo, ext;
        if (pbc[d]) { lo = 0.0; ext = box[d]; }
        else {
            double mn = 1e300, mx = -1e300;
            for (int i = 0; i < n; ++i) {
                double x = pos[3 * i + d];
                if (x < mn) mn = x;
                if (x > mx) mx = x;
            }
            if (n == 0) { mn = 0.0; mx = 0.0; }
            lo = mn; ext = mx - mn;
        }
        int nc = (int)floor(ext / rc);
        if (nc < 1) nc = 1;
        if (nc > 256) nc = 256;
        c->nc[d] = nc;
        c->lo[d] = lo;
        c->cs[d] = ext > 0 ? ext / nc : 1.0;
        int m = (int)ceil(rc / c->cs[d]);
        if (m < 1) m = 1;
        c->m[d] = m;
    }
    long ncell = (long)c->nc[0] * c->nc[1] * c->nc[2];
    c->head = (int *)malloc(sizeof(int) * ncell);
    c->next = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (long k = 0; k < ncell; ++k) c->head[k] = -1;
    for (int i = n - 1; i >= 0; --i) {
        int ci[3];
        for (int d = 0; d < 3; ++d) {
            int k = (int)floor((pos[3 * i + d] - c->lo[d]) / c->cs[d]);
            if (k < 0) k = 0;
            if (k >= c->nc[d]) k = c->nc[d] - 1;
            ci[d] = k;
        }
        long key = ((long)ci[2] * c->nc[1] + ci[1]) * c->nc[0] + ci[0];
        c->next[i] = c->head[key];
        c->head[key] = i;
    }
}

static void cells_free(or_cells *c)
{
    free(c->head);
    free(c->next);
}

typedef struct {
    int j;
    double d[3]; /* r_ij = r_j + n L - r_i */
    double r;
} or_pair;

/* appends bead i's pairs within rc to *out (grown as needed); returns count */
static int pairs_of(const or_cells *c, int i, const double *pos, const double *box,
                    const int *pbc, double rc, or_pair **out, int *cap)
{
    int cnt = 0;
    int ci[3];
    for (int d = 0; d < 3; ++d) {
        int k = (int)floor((pos[3 * i + d] - c->lo[d]) / c->cs[d]);
        if (k < 0) k = 0;
        if (k >= c->nc[d]) k = c->nc[d] - 1;
        ci[d] = k;
    }
    double rc2 = rc * rc;
    for (int dz = -c->m[2]; dz <= c->m[2]; ++dz)
    for (int dy = -c->m[1]; dy <= c->m[1]; ++dy)
    for (int dx = -c->m[0]; dx <= c->m[0]; ++dx) {
        int dd[3] = {dx, dy, dz};
        int cc[3];
        double sh[3];
        int skip = 0;
        for (int d = 0; d < 3; ++d) {
            int k = ci[d] + dd[d];
            if (pbc[d]) {
                int img = (int)floor((double)k / c->nc[d]);
                cc[d] = k - img * c->nc[d];
                sh[d] = img * box[d];
            } else {
                if (k < 0 || k >= c->nc[d]) { skip = 1; break; }
                cc[d] = k;
                sh[d] = 0.0;
            }
        }
        if (skip) continue;
        long key = ((long)cc[2] * c->nc[1] + cc[1]) * c->nc[0] + cc[0];
        int zero_shift = (sh[0] == 0.0 && sh[1] == 0.0 && sh[2] == 0.0);
        for (int j = c->head[key]; j >= 0; j = c->next[j]) {
            if (j == i && zero_shift) continue;
            double v[3];
            for (int d = 0; d < 3; ++d) v[d] = pos[3 * j + d] + sh[d] - pos[3 * i + d];
            double r2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            if (r2 >= rc2) continue;
            if (cnt == *cap) {
                *cap = *cap ? 2 * *cap : 64;
                *out = (or_pair *)realloc(*out, sizeof(or_pair) * (*cap));
            }
            or_pair *p = &(*out)[cnt++];
            p->j = j;
            p->d[0] = v[0]; p->d[1] = v[1]; p->d[2] = v[2];
            p->r = sqrt(r2);
        }
    }
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* per-bead evaluation: descriptor, network, pair partials dU_i/dr_ij        */
/* ------------------------------------------------------------------------ */
typedef struct {
    const double *w0, *b0, *w1, *b1, *cR, *cA;
} or_params;

static or_params split_params(const or_model *m, const double *p)
{
    int T = m->n_types, H = m->n_hidden;
    int nR = m->n_max_R + 1, nA = m->n_max_A + 1;
    int D = nR + nA * m->l_max;
    or_params q;
    q.w0 = p;
    q.b0 = q.w0 + (size_t)T * H * D;
    q.w1 = q.b0 + (size_t)T * H;
    q.b1 = q.w1 + (size_t)T * H;
    q.cR = q.b1 + 1;
    q.cA = q.cR + (size_t)T * T * nR * (m->basis_R + 1);
    return q;
}

long or_param_count(const or_model *m)
{
    int T = m->n_types, H = m->n_hidden;
    int nR = m->n_max_R + 1, nA = m->n_max_A + 1;
    int D = nR + nA * m->l_max;
    return (long)T * H * D + 2L * T * H + 1 + (long)T * T * nR * (m->basis_R + 1) +
           (long)T * T * nA * (m->basis_A + 1);
}

static double rc_max_of(const or_model *m)
{
    double r = 0.0;
    for (int a = 0; a < m->n_types * m->n_types; ++a) {
        if (m->rc_R[a] > r) r = m->rc_R[a];
        if (m->rc_A[a] > r) r = m->rc_A[a];
    }
    return r;
}

/*
 * Evaluate bead i given its pair list: returns U_i, writes the descriptor
 * (optional) and dU_i/dr_ij for every pair into f[3*np].
 */
static double bead_eval(const or_model *m, const or_params *P, const int *types, int i,
                        const or_pair *pr, int np, double *desc_out, double *f)
{
    int T = m->n_types, H = m->n_hidden;
    int nR = m->n_max_R + 1, nA = m->n_max_A + 1, L = m->l_max;
    int KR = m->basis_R + 1, KA = m->basis_A + 1;
    int D = nR + nA * L;
    int ti = types[i];
    double q[256];
    double complex A[16][OR_LMAX + 1][2 * OR_LMAX + 1];
    double fk[OR_KMAX], dfk[OR_KMAX];

    for (int v = 0; v < D; ++v) q[v] = 0.0;
    for (int n = 0; n < nA; ++n)
        for (int l = 0; l <= L; ++l)
            for (int mm = 0; mm <= 2 * L; ++mm) A[n][l][mm] = 0.0;

    /* descriptor: radial (Eq. 3) and angular sums (Eq. 5) */
    for (int p = 0; p < np; ++p) {
        int tj = types[pr[p].j];
        double rcR = m->rc_R[ti * T + tj], rcA = m->rc_A[ti * T + tj];
        double r = pr[p].r;
        if (r < rcR) {
            or_basis(m->basis_R, r, rcR, fk, dfk);
            const double *c = P->cR + (size_t)(ti * T + tj) * nR * KR;
            for (int n = 0; n < nR; ++n) {
                double g = 0.0;
                for (int k = 0; k < KR; ++k) g += c[n * KR + k] * fk[k];
                q[n] += g;
            }
        }
        if (r < rcA) {
            or_basis(m->basis_A, r, rcA, fk, dfk);
            const double *c = P->cA + (size_t)(ti * T + tj) * nA * KA;
            for (int l = 1; l <= L; ++l)
                for (int mm = -l; mm <= l; ++mm) {
                    double yr, yi;
                    or_ylm(l, mm, pr[p].d, &yr, &yi, NULL, NULL);
                    double complex Y = yr + I * yi;
                    for (int n = 0; n < nA; ++n) {
                        double g = 0.0;
                        for (int k = 0; k < KA; ++k) g += c[n * KA + k] * fk[k];
                        A[n][l][mm + L] += g * Y;
                    }
                }
        }
    }
    /* q_nl = sum_m (-1)^m A_nlm A_nl(-m)   (Eq. 4) */
    for (int l = 1; l <= L; ++l)
        for (int n = 0; n < nA; ++n) {
            double complex s = 0.0;
            for (int mm = -l; mm <= l; ++mm) {
                double sg = (mm % 2) ? -1.0 : 1.0;
                s += sg * A[n][l][mm + L] * A[n][l][-mm + L];
            }
            q[nR + (l - 1) * nA + n] = creal(s);
        }
    if (desc_out)
        for (int v = 0; v < D; ++v) desc_out[v] = q[v];

    /* network (Eq. 2) and its gradient with respect to q */
    const double *w0 = P->w0 + (size_t)ti * H * D;
    const double *b0 = P->b0 + (size_t)ti * H;
    const double *w1 = P->w1 + (size_t)ti * H;
    double U = -P->b1[0];
    double dUdq[256];
    for (int v = 0; v < D; ++v) dUdq[v] = 0.0;
    for (int mu = 0; mu < H; ++mu) {
        double z = -b0[mu];
        for (int v = 0; v < D; ++v) z += w0[mu * D + v] * q[v];
        double h = tanh(z);
        U += w1[mu] * h;
        double s = w1[mu] * (1.0 - h * h);
        for (int v = 0; v < D; ++v) dUdq[v] += s * w0[mu * D + v];
    }

    /* pair partials dU_i/dr_ij by the chain rule through q */
    for (int p = 0; p < np; ++p) {
        int tj = types[pr[p].j];
        double rcR = m->rc_R[ti * T + tj], rcA = m->rc_A[ti * T + tj];
        double r = pr[p].r;
        double u[3] = {pr[p].d[0] / r, pr[p].d[1] / r, pr[p].d[2] / r};
        double fx = 0.0, fy = 0.0, fz = 0.0;
        if (r < rcR) {
            or_basis(m->basis_R, r, rcR, fk, dfk);
            const double *c = P->cR + (size_t)(ti * T + tj) * nR * KR;
            double s = 0.0;
            for (int n = 0; n < nR; ++n) {
                double dg = 0.0;
                for (int k = 0; k < KR; ++k) dg += c[n * KR + k] * dfk[k];
                s += dUdq[n] * dg;
            }
            fx += s * u[0]; fy += s * u[1]; fz += s * u[2];
        }
        if (r < rcA) {
            or_basis(m->basis_A, r, rcA, fk, dfk);
            const double *c = P->cA + (size_t)(ti * T + tj) * nA * KA;
            double g[16], dg[16];
            for (int n = 0; n < nA; ++n) {
                g[n] = 0.0; dg[n] = 0.0;
                for (int k = 0; k < KA; ++k) {
                    g[n] += c[n * KA + k] * fk[k];
                    dg[n] += c[n * KA + k] * dfk[k];
                }
            }
            for (int l = 1; l <= L; ++l) {
                /* dA_nlm/dr_ij for this pair = dg_n u Y_lm + g_n grad Y_lm */
                double complex Y[2 * OR_LMAX + 1], GY[2 * OR_LMAX + 1][3];
                for (int mm = -l; mm <= l; ++mm) {
                    double yr, yi, gr[3], gi[3];
                    or_ylm(l, mm, pr[p].d, &yr, &yi, gr, gi);
                    Y[mm + L] = yr + I * yi;
                    for (int a = 0; a < 3; ++a) GY[mm + L][a] = gr[a] + I * gi[a];
                }
                for (int n = 0; n < nA; ++n) {
                    double w = dUdq[nR + (l - 1) * nA + n];
                    double complex acc[3] = {0.0, 0.0, 0.0};
                    for (int mm = -l; mm <= l; ++mm) {
                        double sg = (mm % 2) ? -1.0 : 1.0;
                        for (int a = 0; a < 3; ++a) {
                            double complex dA_m = dg[n] * u[a] * Y[mm + L] + g[n] * GY[mm + L][a];
                            double complex dA_mm = dg[n] * u[a] * Y[-mm + L] + g[n] * GY[-mm + L][a];
                            acc[a] += sg * (dA_m * A[n][l][-mm + L] + A[n][l][mm + L] * dA_mm);
                        }
                    }
                    fx += w * creal(acc[0]);
                    fy += w * creal(acc[1]);
                    fz += w * creal(acc[2]);
                }
            }
        }
        f[3 * p + 0] = fx;
        f[3 * p + 1] = fy;
        f[3 * p + 2] = fz;
    }
    return U;
}

/* ------------------------------------------------------------------------ */
/* public: energy / forces / virial                                         */
/* ------------------------------------------------------------------------ */
/*
 * or_efv: evaluates beads.  If n_target > 0, only the beads in target[] get
 * U, F, W filled (the others are left untouched); the routine then evaluates
 * every bead within the largest cutoff of a target, which is what their
 * forces need.  If n_target == 0 every bead is a target.
 * pos is copied and wrapped into [0, L) on periodic dimensions.
 * Returns the number of pairs evaluated, or -1 on bad input.
 */
long or_efv(const or_model *m, const double *params, int n, const double *pos_in,
            const int *types, const double *box, const int *pbc,
            int n_target, const int *target,
            double *U, double *F, double *Wb, double *E_tot, double *W_tot,
            double *desc /* (n, D) or NULL */, int n_threads)
{
    if (n < 0 || m->n_max_A + 1 > 16 || m->l_max > OR_LMAX) return -1;
    int D = (m->n_max_R + 1) + (m->n_max_A + 1) * m->l_max;
    if (D > 256) return -1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    or_params P = split_params(m, params);
    double rc = rc_max_of(m);
    double *pos = (double *)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    for (int i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            double x = pos_in[3 * i + d];
            if (pbc[d]) {
                x = fmod(x, box[d]);
                if (x < 0) x += box[d];
                if (x >= box[d]) x -= box[d];
            }
            pos[3 * i + d] = x;
        }
    or_cells cells;
    cells_build(&cells, n, pos, box, pbc, rc);

    /* which beads are evaluated, and which receive outputs */
    char *is_target = (char *)calloc(n > 0 ? n : 1, 1);
    char *is_eval = (char *)calloc(n > 0 ? n : 1, 1);
    if (n_target <= 0) {
        memset(is_target, 1, n);
        memset(is_eval, 1, n);
    } else {
        for (int t = 0; t < n_target; ++t) {
            if (target[t] < 0 || target[t] >= n) { free(pos); cells_free(&cells); free(is_target); free(is_eval); return -1; }
            is_target[target[t]] = 1;
            is_eval[target[t]] = 1;
        }
        or_pair *tmp = NULL;
        int cap = 0;
        for (int t = 0; t < n_target; ++t) {
            int c = pairs_of(&cells, target[t], pos, box, pbc, rc, &tmp, &cap);
            for (int p = 0; p < c; ++p) is_eval[tmp[p].j] = 1;
        }
        free(tmp);
    }
    int n_eval = 0;
    for (int i = 0; i < n; ++i) n_eval += is_eval[i];
    int *eval_list = (int *)malloc(sizeof(int) * (n_eval > 0 ? n_eval : 1));
    for (int i = 0, k = 0; i < n; ++i)
        if (is_eval[i]) eval_list[k++] = i;

    /* per evaluated bead: pairs, U_i, dU_i/dr_ij */
    or_pair **pairs = (or_pair **)calloc(n_eval > 0 ? n_eval : 1, sizeof(or_pair *));
    double **fij = (double **)calloc(n_eval > 0 ? n_eval : 1, sizeof(double *));
    int *npairs = (int *)calloc(n_eval > 0 ? n_eval : 1, sizeof(int));
    double *Ue = (double *)calloc(n_eval > 0 ? n_eval : 1, sizeof(double));
    leg_init();
#pragma omp parallel for schedule(dynamic, 16)
    for (int e = 0; e < n_eval; ++e) {
        int i = eval_list[e];
        or_pair *pr = NULL;
        int cap = 0;
        int np = pairs_of(&cells, i, pos, box, pbc, rc, &pr, &cap);
        double *f = (double *)malloc(sizeof(double) * 3 * (np > 0 ? np : 1));
        Ue[e] = bead_eval(m, &P, types, i, pr, np, desc ? desc + (size_t)i * D : NULL, f);
        pairs[e] = pr;
        fij[e] = f;
        npairs[e] = np;
    }

    /* serial, fixed-order assembly of F_i and W_i */
    for (int i = 0; i < n; ++i)
        if (is_target[i]) {
            for (int d = 0; d < 3; ++d) F[3 * i + d] = 0.0;
            if (Wb)
                for (int a = 0; a < 9; ++a) Wb[9 * i + a] = 0.0;
        }
    long total_pairs = 0;
    for (int e = 0; e < n_eval; ++e) {
        int i = eval_list[e];
        if (is_target[i]) U[i] = Ue[e];
        total_pairs += npairs[e];
        for (int p = 0; p < npairs[e]; ++p) {
            int j = pairs[e][p].j;
            const double *f = fij[e] + 3 * p;   /* dU_i/dr_ij */
            const double *d = pairs[e][p].d;    /* r_ij */
            if (is_target[i])
                for (int a = 0; a < 3; ++a) F[3 * i + a] += f[a];
            if (is_target[j]) {
                for (int a = 0; a < 3; ++a) F[3 * j + a] -= f[a];
                /* W_j += r_ji (x) dU_i/dr_ij  with r_ji = -r_ij   (Eq. 15) */
                if (Wb)
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) Wb[9 * j + 3 * a + b] += -d[a] * f[b];
            }
        }
    }
    if (n_target <= 0) {
        double E = 0.0, W[9] = {0};
        for (int i = 0; i < n; ++i) {
            E += U[i];
            if (Wb)
                for (int a = 0; a < 9; ++a) W[a] += Wb[9 * i + a];
        }
        if (E_tot) *E_tot = E;
        if (W_tot)
            for (int a = 0; a < 9; ++a) W_tot[a] = W[a];
    }
    for (int e = 0; e < n_eval; ++e) { free(pairs[e]); free(fij[e]); }
    free(pairs); free(fij); free(npairs); free(Ue); free(eval_list);
    free(is_target); free(is_eval); free(pos);
    cells_free(&cells);
    return total_pairs;
}

/* all pairs within the given cutoff (per type pair), for set comparisons:
 * writes up to cap entries of (i, j, nx, ny, nz); returns the total count.   */
long or_pairs_within(int n, const double *pos_in, const int *types, int n_types,
                     const double *rc_table, const double *box, const int *pbc,
                     long cap, int32_t *out)
{
    double rc = 0.0;
    for (int a = 0; a < n_types * n_types; ++a)
        if (rc_table[a] > rc) rc = rc_table[a];
    double *pos = (double *)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    memcpy(pos, pos_in, sizeof(double) * 3 * n);
    or_cells cells;
    cells_build(&cells, n, pos, box, pbc, rc);
    or_pair *pr = NULL;
    int pcap = 0;
    long cnt = 0;
    for (int i = 0; i < n; ++i) {
        int np = pairs_of(&cells, i, pos, box, pbc, rc, &pr, &pcap);
        for (int p = 0; p < np; ++p) {
            int j = pr[p].j;
            double rcp = rc_table[types[i] * n_types + types[j]];
            if (pr[p].r >= rcp) continue;
            if (cnt < cap) {
                int32_t *o = out + 5 * cnt;
                o[0] = i;
                o[1] = j;
                for (int d = 0; d < 3; ++d) {
                    double s = pr[p].d[d] - (pos[3 * j + d] - pos[3 * i + d]);
                    o[2 + d] = pbc[d] ? (int32_t)lround(s / box[d]) : 0;
                }
            }
            ++cnt;
        }
    }
    free(pr);
    free(pos);
    cells_free(&cells);
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* velocity-Verlet NVE in FP64                                              */
/*   v += dt/2 * a(F);  x += dt v;  [affine strain];  F = F(x);  v += dt/2 a */
/* with a = ACCEL * F / m.  Engineering strain: L_d(s) = L0_d (1 + rate_d s) */
/* ------------------------------------------------------------------------ */
int or_md(const or_model *m, const double *params, int n, double *pos, double *vel,
          const int *types, const double *mass_by_type, double *box, const double *box0,
          const int *pbc, double dt, int n_steps, long step0, const double *strain_rate,
          double accel, double *F, double *E_pot, double *E_kin, int n_threads)
{
    double *U = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double E;
    /* forces at the starting positions */
    if (or_efv(m, params, n, pos, types, box, pbc, 0, NULL, U, F, NULL, &E, NULL, NULL, n_threads) < 0) {
        free(U);
        return -1;
    }
    for (int s = 0; s < n_steps; ++s) {
        for (int i = 0; i < n; ++i) {
            double a = 0.5 * dt * accel / mass_by_type[types[i]];
            for (int d = 0; d < 3; ++d) {
                vel[3 * i + d] += a * F[3 * i + d];
                pos[3 * i + d] += dt * vel[3 * i + d];
            }
        }
        if (strain_rate) {
            long st = step0 + s;
            for (int d = 0; d < 3; ++d) {
                if (strain_rate[d] == 0.0) continue;
                double L_old = box0[d] * (1.0 + strain_rate[d] * (double)st);
                double L_new = box0[d] * (1.0 + strain_rate[d] * (double)(st + 1));
                double lam = L_new / L_old;
                for (int i = 0; i < n; ++i) pos[3 * i + d] *= lam;
                box[d] = L_new;
            }
        }
        if (or_efv(m, params, n, pos, types, box, pbc, 0, NULL, U, F, NULL, &E, NULL, NULL, n_threads) < 0) {
            free(U);
            return -1;
        }
        double K = 0.0;
        for (int i = 0; i < n; ++i) {
            double mi = mass_by_type[types[i]];
            double a = 0.5 * dt * accel / mi;
            for (int d = 0; d < 3; ++d) {
                vel[3 * i + d] += a * F[3 * i + d];
                K += 0.5 * mi * vel[3 * i + d] * vel[3 * i + d] / accel;
            }
        }
        if (E_pot) E_pot[s] = E;
        if (E_kin) E_kin[s] = K;
    }
    free(U);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* ensembles and the HNEMD driving force, FP64                              */
/*                                                                          */
/* The paper equilibrates in NVT/NPT (Sec. III.A.1, III.C.3) and measures   */
/* thermal conductivity by HNEMD (Sec. III.B.3) inside an external engine,  */
/* naming no algorithm beyond the HNEMD reference.  Taken here:             */
/*  - Berendsen velocity rescaling: after the second half-kick of a step,   */
/*    v *= lam, lam^2 = 1 + (dt/tau_T)(T0/T - 1), T = 2K/(N_f k_B),         */
/*    N_f = 3N - 3;                                                          */
/*  - Bussi-Donadio-Parrinello stochastic velocity rescaling (J. Chem.      */
/*    Phys. 126, 014101): the kinetic energy after the step is drawn from   */
/*    the exact solution of its stochastic equation over dt, with c =       */
/*    exp(-dt/tau_T), target Kbar = N_f k_B T0 / 2, a standard normal R and */
/*    S, a chi-square with N_f - 1 degrees of freedom (both given per step):*/
/*      K' = c K + (1 - c) Kbar (S + R^2)/N_f + 2 R sqrt(c (1-c) K Kbar/N_f)*/
/*    and v *= sqrt(K'/K) with the sign of R + sqrt(c N_f K/((1-c) Kbar));  */
/*  - a Berendsen barostat per periodic axis whose scale factor is set once */
/*    per call from a given pressure P_in (the previous call's mean):       */
/*      mu_d = cbrt(1 - beta dt/tau_P (P0_d - P_in_d)), clamped to          */
/*      [0.99, 1.01], positions and box scaled by mu_d after every drift;   */
/*    P_dd = (2 K_dd + W_dd)/V with K_dd = sum m v_d^2 / 2;                 */
/*  - HNEMD (Fan et al., Phys. Rev. B 99, 064308): driving force             */
/*      F_i^ext = W_i^T F_e - (1/N) sum_k W_k^T F_e                         */
/*    (the mean removed so that the momentum is conserved), added to the    */
/*    force of the step's second half-kick; potential heat current          */
/*      J = sum_i W_i v_i  (after the thermostat).                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int thermostat;          /* 0 none, 1 Berendsen, 2 Bussi */
    double T_target, tau_T;  /* K, fs */
    const double *noise;     /* [n_steps][2]: R, S (Bussi) */
    double kB;               /* eV/K */
    int barostat;            /* 0 none, 1 Berendsen (periodic axes) */
    double P_target[3], tau_P, beta;   /* eV/nm^3, fs, 1/(eV/nm^3) */
    double P_in[3];          /* sets this call's scale factor (non-finite: none) */
    double Fe[3];            /* 1/nm */
    /* constrained bead centres of mass (Sec. II.C.1): atoms of bead I are
       group_start[I] .. group_start[I+1]-1; n_groups 0 = no constraint */
    int n_groups;
    const int *group_start;
    double *F_sum;           /* [n_groups][3] += sum_{i in I} f_i every step (Eq. 12) */
    double *W_sum;           /* [n_groups][9] += sum_{i in I} W_i every step (Eq. 14) */
} or_md_opts;

int or_md_ens(const or_model *m, const double *params, int n, double *pos, double *vel,
              const int *types, const double *mass_by_type, double *box, const double *box0,
              const int *pbc, double dt, int n_steps, long step0, const double *strain_rate,
              double accel, const or_md_opts *o, double *F, double *E_pot, double *E_kin,
              double *W_trace /*[n_steps][9]*/, double *J_trace /*[n_steps][3]*/,
              double *P_out /*[3] mean diagonal pressure*/, int n_threads)
{
    int N = n > 0 ? n : 1;
    double *U = (double *)malloc(sizeof(double) * N);
    double *Wb = (double *)malloc(sizeof(double) * 9 * N);
    double E, Wt[9];
    int hnemd = o && (o->Fe[0] != 0.0 || o->Fe[1] != 0.0 || o->Fe[2] != 0.0);
    int con = o && o->n_groups > 0;
    double mu[3] = {1.0, 1.0, 1.0};
    if (o && o->barostat == 1) {
        for (int d = 0; d < 3; ++d) {
            if (!pbc[d] || !isfinite(o->P_in[d])) continue;
            double f = 1.0 - o->beta * dt / o->tau_P * (o->P_target[d] - o->P_in[d]);
            double md = cbrt(f);
            if (md < 0.99) md = 0.99;
            if (md > 1.01) md = 1.01;
            mu[d] = md;
        }
    }
    double Psum[3] = {0.0, 0.0, 0.0};
    /* forces at the starting positions (the plain potential force; with the
       constraint, its projection, which is not accumulated) */
    if (or_efv(m, params, n, pos, types, box, pbc, 0, NULL, U, F, NULL, &E, NULL, NULL, n_threads) < 0) {
        free(U); free(Wb);
        return -1;
    }
    if (con)
        for (int g = 0; g < o->n_groups; ++g) {
            double FI[3] = {0.0, 0.0, 0.0}, MI = 0.0;
            for (int i = o->group_start[g]; i < o->group_start[g + 1]; ++i) {
                MI += mass_by_type[types[i]];
                for (int a = 0; a < 3; ++a) FI[a] += F[3 * i + a];
            }
            for (int i = o->group_start[g]; i < o->group_start[g + 1]; ++i)
                for (int a = 0; a < 3; ++a) F[3 * i + a] -= mass_by_type[types[i]] / MI * FI[a];
        }
    for (int s = 0; s < n_steps; ++s) {
        for (int i = 0; i < n; ++i) {
            double a = 0.5 * dt * accel / mass_by_type[types[i]];
            for (int d = 0; d < 3; ++d) {
                vel[3 * i + d] += a * F[3 * i + d];
                pos[3 * i + d] += dt * vel[3 * i + d];
            }
        }
        for (int d = 0; d < 3; ++d) {
            double lam = mu[d];
            if (strain_rate && strain_rate[d] != 0.0) {
                long st = step0 + s;
                double L_old = box0[d] * (1.0 + strain_rate[d] * (double)st);
                double L_new = box0[d] * (1.0 + strain_rate[d] * (double)(st + 1));
                lam = L_new / L_old;
                box[d] = L_new;
            } else if (lam != 1.0) {
                box[d] *= lam;
            }
            if (lam != 1.0)
                for (int i = 0; i < n; ++i) pos[3 * i + d] *= lam;
        }
        if (or_efv(m, params, n, pos, types, box, pbc, 0, NULL, U, F, Wb, &E, Wt, NULL, n_threads) < 0) {
            free(U); free(Wb);
            return -1;
        }
        if (con) {
            /* the centre of mass of every bead's atoms is held fixed: the
               constraint force on atom i is -(m_i / M_I) sum_{k in I} f_k, so
               the bead's atoms feel no net force; the accumulated bead force
               and virial are the unconstrained sums (Eqs. 12, 14) */
            for (int g = 0; g < o->n_groups; ++g) {
                double FI[3] = {0.0, 0.0, 0.0}, WI[9] = {0.0}, MI = 0.0;
                for (int i = o->group_start[g]; i < o->group_start[g + 1]; ++i) {
                    MI += mass_by_type[types[i]];
                    for (int a = 0; a < 3; ++a) FI[a] += F[3 * i + a];
                    for (int a = 0; a < 9; ++a) WI[a] += Wb[9 * i + a];
                }
                for (int a = 0; a < 3; ++a) o->F_sum[3 * g + a] += FI[a];
                for (int a = 0; a < 9; ++a) o->W_sum[9 * g + a] += WI[a];
                for (int i = o->group_start[g]; i < o->group_start[g + 1]; ++i) {
                    double w = mass_by_type[types[i]] / MI;
                    for (int a = 0; a < 3; ++a) F[3 * i + a] -= w * FI[a];
                }
            }
        }
        if (hnemd) {
            double mean[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < n; ++i)
                for (int b = 0; b < 3; ++b)
                    for (int a = 0; a < 3; ++a) mean[b] += Wb[9 * i + 3 * a + b] * o->Fe[a];
            for (int b = 0; b < 3; ++b) mean[b] /= (double)n;
            for (int i = 0; i < n; ++i)
                for (int b = 0; b < 3; ++b) {
                    double fe = 0.0;
                    for (int a = 0; a < 3; ++a) fe += Wb[9 * i + 3 * a + b] * o->Fe[a];
                    F[3 * i + b] += fe - mean[b];
                }
        }
        double Kd[3] = {0.0, 0.0, 0.0}, J[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < n; ++i) {
            double mi = mass_by_type[types[i]];
            double a = 0.5 * dt * accel / mi;
            for (int d = 0; d < 3; ++d) {
                vel[3 * i + d] += a * F[3 * i + d];
                Kd[d] += 0.5 * mi * vel[3 * i + d] * vel[3 * i + d] / accel;
            }
            for (int a2 = 0; a2 < 3; ++a2)
                for (int b = 0; b < 3; ++b) J[a2] += Wb[9 * i + 3 * a2 + b] * vel[3 * i + b];
        }
        double K = Kd[0] + Kd[1] + Kd[2];
        double lam = 1.0;
        if (o && o->thermostat && n > 1 && K > 0.0) {
            double Nf = 3.0 * n - 3.0;
            double Kbar = 0.5 * Nf * o->kB * o->T_target;
            if (o->thermostat == 1) {
                double T = 2.0 * K / (Nf * o->kB);
                double l2 = 1.0 + dt / o->tau_T * (o->T_target / T - 1.0);
                lam = sqrt(l2 > 0.0 ? l2 : 0.0);
            } else {
                double R = o->noise[2 * s], S = o->noise[2 * s + 1];
                double c = exp(-dt / o->tau_T);
                double Kn = c * K + (1.0 - c) * Kbar * (S + R * R) / Nf +
                            2.0 * R * sqrt(c * (1.0 - c) * K * Kbar / Nf);
                lam = sqrt(Kn / K);
                if (R + sqrt(c * Nf * K / ((1.0 - c) * Kbar)) < 0.0) lam = -lam;
            }
            for (int i = 0; i < 3 * n; ++i) vel[i] *= lam;
        }
        double l2 = lam * lam;
        double V = box[0] * box[1] * box[2];
        for (int d = 0; d < 3; ++d) {
            Kd[d] *= l2;
            Psum[d] += (2.0 * Kd[d] + Wt[4 * d]) / V;
        }
        if (E_pot) E_pot[s] = E;
        if (E_kin) E_kin[s] = K * l2;
        if (W_trace)
            for (int a = 0; a < 9; ++a) W_trace[9 * s + a] = Wt[a];
        if (J_trace)
            for (int a = 0; a < 3; ++a) J_trace[3 * s + a] = lam * J[a];
    }
    if (P_out)
        for (int d = 0; d < 3; ++d) P_out[d] = n_steps > 0 ? Psum[d] / n_steps : NAN;
    free(U);
    free(Wb);
    return 0;
}

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
