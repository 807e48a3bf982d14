/*
 * matcha_oracle.c -- plain, slow, FP64 CPU oracle for the rotational-alignment
 * path of "Matcha: Fast Volume Alignment by Frequency-Marched Newton Method".
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the cpu_baseline
 * leg of bench.py load this library.  It shares no code, header, table or helper
 * with the HIP library; the only thing both sides see is the seeded input.
 *
 * Every function follows the passage cited in its comment and is written for
 * readability: full (l, m, n) sums, no symmetry shortcuts, no blocking.
 *
 * Conventions (paper App. A.3-A.5):
 *   g(a, b, c) = r_z(a) r_y(b) r_z(c)                         (eq. Euler)
 *   D^l_mn(a, b, c) = e^{-ima} d^l_mn(b) e^{-inc}              (eq. wigner-D)
 *   d^l_mn(b) = <l m| exp(-i b J_y) |l n>   (Condon-Shortley phase)
 *   C^l_mn = sum_r w_r f_lm(r) conj(h_ln(r))                  (eq. sigmalmm, k -> r)
 *   C_L(g) = Re sum_{l<=L} sum_{m,n} C^l_mn conj(D^l_mn(g))   (eq. cc-L; the
 *            conjugation of D is the "conjugation absorbed into the coefficients"
 *            reading, which makes C_L(g) = <f, g o h> for (g o h)_l = D^l(g) h_l)
 * Arrays:
 *   f, h : shell-major [R][(L+1)^2] complex, lm = l*l + l + m
 *   C    : packed by l, block l at l(4l^2-1)/3, (2l+1)^2 entries row-major (m, n)
 *   d    : same packing as C
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MO_PI 3.14159265358979323846

/* per-candidate / per-particle status bits */
#define MO_NONFINITE 1u
#define MO_INDEFINITE 2u
#define MO_SINGULAR 4u
#define MO_NEAR_POLE 8u
#define MO_FEW_MAXIMA 16u
#define MO_EARLY_STOP 32u

static long mo_blk(int l) { return (long)l * (4L * l * l - 1) / 3; }
static long mo_nterms(int L) { return mo_blk(L + 1); } /* (L+1)(2L+1)(2L+3)/3, App. A.5 */
static long mo_lm(int l, int m) { return (long)l * l + l + m; }
static long mo_at(int l, int m, int n) { return mo_blk(l) + (long)(m + l) * (2 * l + 1) + (n + l); }

long mo_term_count(int L) { return mo_nterms(L); }

/* Thread count of the OpenMP loops over particles and grid slices (timing plumbing only). */
void mo_set_num_threads(int n) { omp_set_num_threads(n); }
int mo_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ Wigner d
 * d^l_mn(b) on its "edge" l = max(|m|, |n|): the explicit finite sum of App. A.4
 * has a single term there,
 *   d^j_{j,k}(b) = (-1)^{j-k} sqrt(binom(2j, j+k)) cos^{j+k}(b/2) sin^{j-k}(b/2),
 * and the other three edges follow from d_mn = (-1)^{m-n} d_nm = d_{-n,-m}. */
static double mo_edge_top(int j, int k, double b)
{
    double lb = 0.5 * (lgamma(2.0 * j + 1) - lgamma(j + k + 1.0) - lgamma(j - k + 1.0));
    double v = exp(lb) * pow(cos(0.5 * b), j + k) * pow(sin(0.5 * b), j - k);
    return ((j - k) & 1) ? -v : v;
}

static double mo_edge(int l0, int m, int n, double b)
{
    if (m == l0) return mo_edge_top(l0, n, b);
    if (m == -l0) return (((n + l0) & 1) ? -1.0 : 1.0) * mo_edge_top(l0, -n, b);
    if (n == l0) return (((m - l0) & 1) ? -1.0 : 1.0) * mo_edge_top(l0, m, b);
    return mo_edge_top(l0, -m, b); /* n == -l0 */
}

/* All d^l_mn(b), l <= L, by the standard three-term recurrence in l at fixed
 * (m, n) started from the edge value (App. A.4: d admits explicit finite sums and
 * recurrences):
 *   d^{l+1} = a_l (cos b - mn / (l(l+1))) d^l - b_l d^{l-1},
 *   a_l = (l+1)(2l+1) / sqrt(((l+1)^2-m^2)((l+1)^2-n^2)),
 *   b_l = (l+1) sqrt((l^2-m^2)(l^2-n^2)) / (l sqrt(((l+1)^2-m^2)((l+1)^2-n^2))).
 * Beta derivatives use the J_y ladder (App. A.4: beta derivatives are finite
 * combinations of neighbouring d with known coefficients); with
 * cp_n = sqrt((l-n)(l+n+1)), cm_n = sqrt((l+n)(l-n+1)):
 *   d'_mn  = (cm_n d_{m,n-1} - cp_n d_{m,n+1}) / 2
 *   d''_mn = (cm_n cm_{n-1} d_{m,n-2} - 2(l(l+1)-n^2) d_mn + cp_n cp_{n+1} d_{m,n+2}) / 4
 * d1 / d2 may be NULL. */
void mo_wigner_d(int L, double b, double *d, double *d1, double *d2)
{
    const double cb = cos(b);
    for (int m = -L; m <= L; ++m) {
        for (int n = -L; n <= L; ++n) {
            int l0 = abs(m) > abs(n) ? abs(m) : abs(n);
            double dm1 = 0.0, dl = mo_edge(l0, m, n, b);
            d[mo_at(l0, m, n)] = dl;
            for (int l = l0; l < L; ++l) {
                double l1 = l + 1.0;
                double den = sqrt((l1 * l1 - (double)m * m) * (l1 * l1 - (double)n * n));
                double a = l1 * (2.0 * l + 1.0) / den;
                double bb = 0.0, c = 0.0;
                if (l > 0) {
                    bb = l1 * sqrt(((double)l * l - (double)m * m) * ((double)l * l - (double)n * n)) / (l * den);
                    c = (double)m * n / ((double)l * l1);
                }
                double dn = a * (cb - c) * dl - bb * dm1;
                dm1 = dl;
                dl = dn;
                d[mo_at(l + 1, m, n)] = dl;
            }
        }
    }
    if (!d1 && !d2) return;
    for (int l = 0; l <= L; ++l) {
        for (int m = -l; m <= l; ++m) {
            for (int n = -l; n <= l; ++n) {
                double cp = sqrt((double)(l - n) * (l + n + 1));
                double cm = sqrt((double)(l + n) * (l - n + 1));
                double dnm1 = n - 1 >= -l ? d[mo_at(l, m, n - 1)] : 0.0;
                double dnp1 = n + 1 <= l ? d[mo_at(l, m, n + 1)] : 0.0;
                if (d1) d1[mo_at(l, m, n)] = 0.5 * (cm * dnm1 - cp * dnp1);
                if (d2) {
                    double cm2 = sqrt((double)(l + n - 1) * (l - n + 2)); /* cm_{n-1} */
                    double cp2 = sqrt((double)(l - n - 1) * (l + n + 2)); /* cp_{n+1} */
                    double dnm2 = n - 2 >= -l ? d[mo_at(l, m, n - 2)] : 0.0;
                    double dnp2 = n + 2 <= l ? d[mo_at(l, m, n + 2)] : 0.0;
                    if (n - 1 < -l) cm2 = 0.0;
                    if (n + 1 > l) cp2 = 0.0;
                    d2[mo_at(l, m, n)] = 0.25 * (cm * cm2 * dnm2 - 2.0 * ((double)l * (l + 1) - (double)n * n) * d[mo_at(l, m, n)] +
                                                 cp * cp2 * dnp2);
                }
            }
        }
    }
}

/* ------------------------------------------------------- coefficient assembly
 * eq. sigmalmm with the radial index k read as the shell index r and the shell
 * quadrature weight w_r:  C^l_mn = sum_r w_r f_lm(r) conj(h_ln(r)), l <= L.
 * f: [Rf][(Lf+1)^2], h: [Rh][(Lh+1)^2]; shells 0..R-1 of both are used. */
void mo_coeff_assemble(int L, int R, const double complex *f, int Lf, const double complex *h, int Lh,
                       const double *w, double complex *C)
{
    const long sf = (long)(Lf + 1) * (Lf + 1), sh = (long)(Lh + 1) * (Lh + 1);
    for (int l = 0; l <= L; ++l)
        for (int m = -l; m <= l; ++m)
            for (int n = -l; n <= l; ++n) {
                double complex acc = 0.0;
                for (int r = 0; r < R; ++r)
                    acc += w[r] * f[r * sf + mo_lm(l, m)] * conj(h[r * sh + mo_lm(l, n)]);
                C[mo_at(l, m, n)] = acc;
            }
}

/* ----------------------------------------------------------- the objective
 * C_L(a, b, c) = Re sum C^l_mn e^{i(ma + nc)} d^l_mn(b) and its chart derivatives
 * (Sec. 2.2 and App. A.4: alpha and gamma derivatives act diagonally, -im and
 * -in on D, hence +im, +in on conj(D); beta derivatives come from d', d'').
 * out[10] = F, F_a, F_b, F_c, F_aa, F_ab, F_ac, F_bb, F_bc, F_cc. */
void mo_eval(int L, const double complex *C, double a, double b, double c, double *out)
{
    long N = mo_nterms(L);
    double *d = malloc(sizeof(double) * N), *d1 = malloc(sizeof(double) * N), *d2 = malloc(sizeof(double) * N);
    mo_wigner_d(L, b, d, d1, d2);
    double s[10] = {0};
    for (int l = 0; l <= L; ++l)
        for (int m = -l; m <= l; ++m)
            for (int n = -l; n <= l; ++n) {
                long i = mo_at(l, m, n);
                double complex z = C[i] * cexp(I * (m * a + n * c));
                double re = creal(z), im = cimag(z);
                s[0] += re * d[i];
                s[1] += -m * im * d[i];
                s[2] += re * d1[i];
                s[3] += -n * im * d[i];
                s[4] += -(double)m * m * re * d[i];
                s[5] += -m * im * d1[i];
                s[6] += -(double)m * n * re * d[i];
                s[7] += re * d2[i];
                s[8] += -n * im * d1[i];
                s[9] += -(double)n * n * re * d[i];
            }
    memcpy(out, s, sizeof s);
    free(d);
    free(d1);
    free(d2);
}

double mo_eval_F(int L, const double complex *C, double a, double b, double c)
{
    long N = mo_nterms(L);
    double *d = malloc(sizeof(double) * N);
    mo_wigner_d(L, b, d, NULL, NULL);
    double F = 0.0;
    for (int l = 0; l <= L; ++l)
        for (int m = -l; m <= l; ++m)
            for (int n = -l; n <= l; ++n) {
                long i = mo_at(l, m, n);
                F += creal(C[i] * cexp(I * (m * a + n * c))) * d[i];
            }
    free(d);
    return F;
}

/* ------------------------------------------------------------- SOFFT search
 * Sec. 2.3: C_{L0} on an equiangular grid of n^3 rotations.  The grid value at a
 * node is, by definition, C_{L0} evaluated there, so the oracle evaluates the
 * band-limited sum directly at every node: a_j = 2 pi j / n, c_k = 2 pi k / n and
 * the pole-avoiding midpoints b_i = pi (2i+1) / (2n).
 * grid[(i*n + j)*n + k] = C_B(a_j, b_i, c_k). */
void mo_soft_grid(int B, const double complex *C, int n, double *grid)
{
    long N = mo_nterms(B);
    int W = 2 * B + 1;
    double complex *ea = malloc(sizeof(double complex) * n * W);
    for (int j = 0; j < n; ++j)
        for (int m = -B; m <= B; ++m) {
            long r = ((long)m * j) % n;
            if (r < 0) r += n;
            ea[j * W + m + B] = cexp(I * 2.0 * MO_PI * (double)r / n);
        }
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < n; ++i) {
        double *d = malloc(sizeof(double) * N);
        double bi = MO_PI * (2.0 * i + 1.0) / (2.0 * n);
        mo_wigner_d(B, bi, d, NULL, NULL);
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                double F = 0.0;
                for (int l = 0; l <= B; ++l)
                    for (int m = -l; m <= l; ++m)
                        for (int q = -l; q <= l; ++q) {
                            long t = mo_at(l, m, q);
                            F += creal(C[t] * ea[j * W + m + B] * ea[k * W + q + B]) * d[t];
                        }
                grid[((long)i * n + j) * n + k] = F;
            }
        free(d);
    }
    free(ea);
}

/* Sec. 2.3 / Alg. 1: keep the P strongest local maxima of the grid.
 * A node is a local maximum when it beats each of its 26 neighbours (a and c wrap,
 * b neighbours outside [0, n) do not exist); "beats" orders by value and, among
 * equal values, the smaller linear index wins.  Maxima are ranked by (value desc,
 * index asc).  If there are fewer than Kc maxima the list is filled with the best
 * remaining nodes in the same order.  Returns the number of local maxima found. */
static int mo_beats(double v, long i, double u, long j) { return v > u || (v == u && i < j); }

typedef struct {
    double v;
    long i;
} mo_node;

static int mo_node_cmp(const void *x, const void *y)
{
    const mo_node *a = x, *b = y;
    if (a->v != b->v) return a->v > b->v ? -1 : 1;
    return a->i < b->i ? -1 : (a->i > b->i);
}

int mo_soft_select(int n, const double *grid, int Kc, int64_t *idx_out, double *val_out)
{
    long n3 = (long)n * n * n;
    mo_node *mx = malloc(sizeof(mo_node) * n3), *rest = malloc(sizeof(mo_node) * n3);
    long nmx = 0, nrest = 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                long me = ((long)i * n + j) * n + k;
                double v = grid[me];
                int is_max = 1;
                for (int di = -1; di <= 1 && is_max; ++di) {
                    int ii = i + di;
                    if (ii < 0 || ii >= n) continue;
                    for (int dj = -1; dj <= 1 && is_max; ++dj)
                        for (int dk = -1; dk <= 1 && is_max; ++dk) {
                            if (!di && !dj && !dk) continue;
                            int jj = (j + dj + n) % n, kk = (k + dk + n) % n;
                            long o = ((long)ii * n + jj) * n + kk;
                            if (!mo_beats(v, me, grid[o], o)) is_max = 0;
                        }
                }
                if (is_max) mx[nmx++] = (mo_node){v, me};
                else rest[nrest++] = (mo_node){v, me};
            }
    qsort(mx, nmx, sizeof(mo_node), mo_node_cmp);
    qsort(rest, nrest, sizeof(mo_node), mo_node_cmp);
    for (int t = 0; t < Kc; ++t) {
        mo_node q = t < nmx ? mx[t] : rest[t - nmx];
        idx_out[t] = q.i;
        val_out[t] = q.v;
    }
    free(mx);
    free(rest);
    return (int)nmx;
}

/* ---------------------------------------------------------------- Newton step
 * Sec. 2.2: theta <- theta - H^{-1} grad C_L in the wrapped ZYZ chart, with the
 * 3x3 system inverted in explicit (cofactor) form.  Readings where the paper is
 * silent: a non-negative-definite H still takes the pure Newton step and is
 * flagged; |det H| <= 1e-30 max|H|^3 (or a non-finite value) skips the step; a
 * positive max_step clips the step's largest component (off when 0); b leaving
 * [0, pi] is reflected with (a + pi, c + pi), the same rotation. */
static double mo_wrap2pi(double x)
{
    x = fmod(x, 2.0 * MO_PI);
    return x < 0.0 ? x + 2.0 * MO_PI : x;
}

/* theta += dth (largest component clipped to max_step when positive), b reflected into [0, pi] */
static void mo_apply_step(double *dth, double max_step, double *th, double *step_inf)
{
    double mx = fmax(fabs(dth[0]), fmax(fabs(dth[1]), fabs(dth[2])));
    if (max_step > 0.0 && mx > max_step) {
        for (int i = 0; i < 3; ++i) dth[i] *= max_step / mx;
        mx = max_step;
    }
    *step_inf = mx;
    double a = th[0] + dth[0], b = th[1] + dth[1], c = th[2] + dth[2];
    b = mo_wrap2pi(b);
    if (b > MO_PI) {
        b = 2.0 * MO_PI - b;
        a += MO_PI;
        c += MO_PI;
    }
    th[0] = mo_wrap2pi(a);
    th[1] = b;
    th[2] = mo_wrap2pi(c);
}

unsigned mo_newton_step(const double *e, double max_step, double *th, double *step_inf)
{
    /* e = F, Fa, Fb, Fc, Faa, Fab, Fac, Fbb, Fbc, Fcc */
    unsigned st = 0;
    for (int i = 0; i < 10; ++i)
        if (!isfinite(e[i])) return MO_NONFINITE;
    double H[3][3] = {{e[4], e[5], e[6]}, {e[5], e[7], e[8]}, {e[6], e[8], e[9]}};
    double g[3] = {e[1], e[2], e[3]};
    double A[3][3]; /* adjugate */
    A[0][0] = H[1][1] * H[2][2] - H[1][2] * H[2][1];
    A[0][1] = H[0][2] * H[2][1] - H[0][1] * H[2][2];
    A[0][2] = H[0][1] * H[1][2] - H[0][2] * H[1][1];
    A[1][0] = H[1][2] * H[2][0] - H[1][0] * H[2][2];
    A[1][1] = H[0][0] * H[2][2] - H[0][2] * H[2][0];
    A[1][2] = H[0][2] * H[1][0] - H[0][0] * H[1][2];
    A[2][0] = H[1][0] * H[2][1] - H[1][1] * H[2][0];
    A[2][1] = H[0][1] * H[2][0] - H[0][0] * H[2][1];
    A[2][2] = H[0][0] * H[1][1] - H[0][1] * H[1][0];
    double det = H[0][0] * A[0][0] + H[0][1] * A[1][0] + H[0][2] * A[2][0];
    double hmax = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) hmax = fmax(hmax, fabs(H[i][j]));
    /* negative definite <=> leading minors of -H positive */
    if (!(-H[0][0] > 0.0 && A[2][2] > 0.0 && -det > 0.0)) st |= MO_INDEFINITE;
    if (!(fabs(det) > 1e-30 * hmax * hmax * hmax)) {
        *step_inf = 0.0;
        return st | MO_SINGULAR;
    }
    double dth[3];
    for (int i = 0; i < 3; ++i) dth[i] = -(A[i][0] * g[0] + A[i][1] * g[1] + A[i][2] * g[2]) / det;
    mo_apply_step(dth, max_step, th, step_inf);
    return st;
}

/* ------------------------------------------------------ gradient ascent step
 * The first-order comparator of Sec. 4.1 (Fig. newton_v_gd): theta <- theta + t grad C_L in the
 * same chart, t = rate / ((1 + L)^2 |C_L(theta)|).  The paper gives no step rule.  This one takes
 * the Bernstein bound of App. A.7 on the Hessian, B2 (1 + L)^2 ||C_L||_inf, as the smoothness
 * constant of a 1/M step, with |C_L| at the current point standing in for the sup norm; rate plays
 * the part of 1 / B2.  Clipping, reflection and the non-finite flag as for the Newton step; the
 * Hessian is not used. */
unsigned mo_gradient_step(const double *e, double rate, int L, double max_step, double *th, double *step_inf)
{
    for (int i = 0; i < 4; ++i)
        if (!isfinite(e[i])) {
            *step_inf = 0.0;
            return MO_NONFINITE;
        }
    double t = rate / ((1.0 + L) * (1.0 + L) * fmax(fabs(e[0]), 1e-300));
    double dth[3] = {t * e[1], t * e[2], t * e[3]};
    mo_apply_step(dth, max_step, th, step_inf);
    return 0;
}

/* ------------------------------------------------------------ march + select
 * Alg. 1: from the retained candidates, M_iter Newton steps (gradient ascent steps when gd_rate > 0,
 * the first-order comparator) on C_{L_j} at every
 * cutoff of the schedule (the first cutoff is the SOFFT band L0, i.e. the
 * optional refinement at the search band), then the candidate with the largest C_{L_J} at
 * its final point.  The per-particle schedule is the global one with every
 * cutoff >= Lp dropped and Lp appended (cutoffs above L_max are skipped, Sec. 4.1).
 * Early stopping (Sec. 2.4) is optional: at a level, stop stepping once
 * |grad| <= tol_grad |F|, the last step's max component <= tol_step, or
 * |F_t - F_{t-1}| <= tol_rel |F_t|.
 * cand: [Kc][4] (a, b, c, value) in/out; on return value = C_{L_J} at the final point.
 * cand_status: [Kc] flags or NULL.  Returns the index of the selected candidate. */
typedef struct {
    int n_levels;
    const int *levels;
    int steps;
    double max_step;
    int early_stop;
    double tol_grad, tol_step, tol_rel;
} mo_march_cfg;

int mo_schedule(int Lp, const int *levels, int n_levels, int *out)
{
    int k = 0;
    for (int j = 0; j < n_levels; ++j)
        if (levels[j] < Lp) out[k++] = levels[j];
    out[k++] = Lp;
    return k;
}

int mo_march(int Lp, const double complex *C, int n_levels, const int *levels, int steps, double max_step, int early_stop,
             double tol_grad, double tol_step, double tol_rel, double gd_rate, int Kc, double *cand,
             unsigned *cand_status)
{
    int sched[64];
    int ns = mo_schedule(Lp, levels, n_levels, sched);
    int best = 0;
    for (int p = 0; p < Kc; ++p) {
        double th[3] = {cand[4 * p], cand[4 * p + 1], cand[4 * p + 2]};
        unsigned st = 0;
        for (int j = 0; j < ns; ++j) {
            double Fprev = NAN;
            for (int t = 0; t < steps; ++t) {
                double e[10], sinf = 0.0;
                mo_eval(sched[j], C, th[0], th[1], th[2], e);
                if (early_stop) {
                    double gn = sqrt(e[1] * e[1] + e[2] * e[2] + e[3] * e[3]);
                    if (gn <= tol_grad * fabs(e[0]) || (t > 0 && fabs(e[0] - Fprev) <= tol_rel * fabs(e[0]))) {
                        st |= MO_EARLY_STOP;
                        break;
                    }
                }
                Fprev = e[0];
                if (gd_rate > 0.0)
                    st |= mo_gradient_step(e, gd_rate, sched[j], max_step, th, &sinf);
                else
                    st |= mo_newton_step(e, max_step, th, &sinf);
                if (sin(th[1]) < 1e-3) st |= MO_NEAR_POLE;
                if (early_stop && sinf <= tol_step) {
                    st |= MO_EARLY_STOP;
                    break;
                }
            }
        }
        double F = mo_eval_F(sched[ns - 1], C, th[0], th[1], th[2]);
        if (!isfinite(F)) st |= MO_NONFINITE;
        cand[4 * p] = th[0];
        cand[4 * p + 1] = th[1];
        cand[4 * p + 2] = th[2];
        cand[4 * p + 3] = F;
        if (cand_status) cand_status[p] = st;
        /* ties keep the lower index; a non-finite value never wins over a finite one */
        if (p > 0 && isfinite(F) && (!isfinite(cand[4 * best + 3]) || F > cand[4 * best + 3])) best = p;
    }
    return best;
}

/* ------------------------------------------------------------- whole path
 * One particle: assemble C (l <= Lp, shells 0..Rp-1), SOFFT at B on an n^3 grid,
 * keep Kc, march, select.  best[4] = (a, b, c, C_{L_J}); returns status bits of
 * the selected candidate plus FEW_MAXIMA. */
unsigned mo_align_one(int Lp, int Rp, const double complex *f, const double complex *h, int Lh, const double *w, int B,
                      int n, int Kc, int n_levels, const int *levels, int steps, double max_step, double *cand,
                      double *best, int *best_idx)
{
    double complex *C = malloc(sizeof(double complex) * mo_nterms(Lp));
    mo_coeff_assemble(Lp, Rp, f, Lp, h, Lh, w, C);
    long n3 = (long)n * n * n;
    double *grid = malloc(sizeof(double) * n3);
    mo_soft_grid(B, C, n, grid);
    int64_t *idx = malloc(sizeof(int64_t) * Kc);
    double *val = malloc(sizeof(double) * Kc);
    int nmx = mo_soft_select(n, grid, Kc, idx, val);
    for (int p = 0; p < Kc; ++p) {
        long i = idx[p] / ((long)n * n), j = (idx[p] / n) % n, k = idx[p] % n;
        cand[4 * p] = 2.0 * MO_PI * j / n;
        cand[4 * p + 1] = MO_PI * (2.0 * i + 1.0) / (2.0 * n);
        cand[4 * p + 2] = 2.0 * MO_PI * k / n;
        cand[4 * p + 3] = val[p];
    }
    unsigned *cst = malloc(sizeof(unsigned) * Kc);
    int b = mo_march(Lp, C, n_levels, levels, steps, max_step, 0, 0, 0, 0, 0.0, Kc, cand, cst);
    memcpy(best, cand + 4 * b, 4 * sizeof(double));
    *best_idx = b;
    unsigned st = cst[b] | (nmx < Kc ? MO_FEW_MAXIMA : 0u);
    free(cst);
    free(C);
    free(grid);
    free(idx);
    free(val);
    return st;
}

/* ------------------------------------------------------------------- adjoint
 * Differentiation of sum_i g_i C_{L}(R_i*) at fixed R_i* (envelope theorem).
 * Gradients are packed as d/dRe + i d/dIm of the full complex arrays:
 *   grad_h[r][l,n] += g_i w_r sum_m f_lm(r) conj(D^l_mn(R_i*))
 *   grad_f_i[r][l,m] = g_i w_r sum_n D^l_mn(R_i*) h_ln(r)
 * One particle per call; grad_h accumulates, grad_f is overwritten. */
void mo_grad_one(int L, int R, const double complex *f, const double complex *h, int Lh, const double *w,
                 const double *euler, double g, double complex *grad_h, double complex *grad_f)
{
    const long sf = (long)(L + 1) * (L + 1), sh = (long)(Lh + 1) * (Lh + 1);
    long N = mo_nterms(L);
    double *d = malloc(sizeof(double) * N);
    mo_wigner_d(L, euler[1], d, NULL, NULL);
    for (int l = 0; l <= L; ++l)
        for (int r = 0; r < R; ++r) {
            for (int n = -l; n <= l; ++n) {
                double complex acc = 0.0;
                for (int m = -l; m <= l; ++m) {
                    double complex D = cexp(-I * (m * euler[0] + n * euler[2])) * d[mo_at(l, m, n)];
                    acc += f[r * sf + mo_lm(l, m)] * conj(D);
                }
                if (grad_h) grad_h[r * sh + mo_lm(l, n)] += g * w[r] * acc;
            }
            if (grad_f)
                for (int m = -l; m <= l; ++m) {
                    double complex acc = 0.0;
                    for (int n = -l; n <= l; ++n) {
                        double complex D = cexp(-I * (m * euler[0] + n * euler[2])) * d[mo_at(l, m, n)];
                        acc += D * h[r * sh + mo_lm(l, n)];
                    }
                    grad_f[r * sf + mo_lm(l, m)] = g * w[r] * acc;
                }
        }
    free(d);
}

/* batch driver over particles (OpenMP), used for the CPU baseline timing.
 * f_flat / f_offset: ragged particles as in the input format; outputs per particle. */
void mo_align_batch(int P, const int *Lp, const int *Rp, const int64_t *f_offset, const double complex *f_flat,
                    const double complex *h, int Lh, const double *w, int B, int n, int Kc, int n_levels,
                    const int *levels, int steps, double max_step, double *cand, double *best, int *best_idx,
                    unsigned *status)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int p = 0; p < P; ++p)
        status[p] = mo_align_one(Lp[p], Rp[p], f_flat + f_offset[p], h, Lh, w, B, n, Kc, n_levels, levels, steps,
                                 max_step, cand + (long)p * Kc * 4, best + 4L * p, best_idx + p);
}
