/*
 * lhf_oracle.c -- plain FP64 CPU oracle for the Lamb-Helmholtz vortex FMM.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * What it computes (Gumerov & Duraiswami, "Efficient FMM accelerated vortex
 * methods in three dimensions via the Lamb-Helmholtz decomposition"):
 *
 *   (A) direct sums of the Biot-Savart velocity v (eq. 1, with the smoothing
 *       kernel of eq. 2 / eq. vem1) and of the stretching term
 *       s_j = (omega_j . grad) v at x_j (eq. s1.1), self term excluded;
 *   (B) a plain FMM in the two-potential (phi, chi) form (eq. 4):
 *       P2M by Method 2 (eq. eve4) and Method 1 (eqs. eve5-eve10),
 *       M2M / M2L / L2L with the full translation matrices of eq. mr3
 *       followed by the general conversion operators of eqs. drt10 / drt11
 *       (no rotations: this is the plain definition, O(p^4) per translation),
 *       L2P of v (eq. evf3) and of grad v / s (eqs. dt3, evf5, evf6),
 *       near field by (A) over adjacent leaves.
 *
 * Storage is the plain complex one: coefficient (n, m), -n <= m <= n, at
 * index n*n + n + m; truncation number p keeps orders n = 0..p-1 (Sec. 5.1).
 * Precision: FP64 throughout; compiled with -ffp-contract=off.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - no 1/(4 pi) factor: eq. 1 is used literally (eq. 7 absorbs it);
 *   - translation vector t = new centre - old centre (eq. bas1);
 *   - M2L computes chi-hat to order p (one extra row) before the R-basis
 *     conversion, then truncates to p-1 ("reading B");
 *   - octree: cube [lo, lo+L]^3, integer coordinates
 *     q = min(floor((x-lo)*(2^21/L)), 2^21-1), level-l box = q >> (21-l),
 *     empty boxes skipped, M2L from level 2, V-list = children of the
 *     parent's neighbours that are not adjacent (adjacency is closed),
 *     U-list = adjacent leaves (incl. self);
 *   - the near field (U-list pairs) uses the smoothed kernel, the far field
 *     the singular one (eq. 2: the core only changes the near field).
 *
 * Parity pins: every routine here is checked by the CPU tests against closed
 * forms, identities, finite differences or brute force (see tests/).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define IDX(n, m) ((n) * (n) + (n) + (m))
#define QBITS 21
#define MAXLEV 21

/* ------------------------------------------------------------------------- */
/* small helpers                                                              */
/* ------------------------------------------------------------------------- */

static double fact(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; i++) f *= (double)i;
    return f;
}

/* i^k for integer k (any sign) */
static cplx ipow(int k)
{
    int r = ((k % 4) + 4) % 4;
    switch (r) {
    case 0: return 1.0;
    case 1: return I;
    case 2: return -1.0;
    default: return -I;
    }
}

static double sgn_pow(int k) { return (k & 1) ? -1.0 : 1.0; }

/* coefficient lookup with the zero extension of eq. rsbf7 */
static cplx cget(const cplx *c, int nmax, int n, int m)
{
    if (n < 0 || n >= nmax || m < -n || m > n) return 0.0;
    return c[IDX(n, m)];
}

/* ------------------------------------------------------------------------- */
/* Basis functions, eqs. rsbf1-rsbf3                                          */
/* ------------------------------------------------------------------------- */

/* Associated Legendre functions P_n^m(mu), 0<=m<=n<nmax, WITH the
 * Condon-Shortley phase (-1)^m of eq. rsbf3, by the textbook recurrences
 *   P_m^m = (-1)^m (2m-1)!! (1-mu^2)^{m/2},  P_{m+1}^m = mu (2m+1) P_m^m,
 *   (n-m) P_n^m = (2n-1) mu P_{n-1}^m - (n+m-1) P_{n-2}^m.
 * P[n*nmax+m]. */
static void legendre(int nmax, double mu, double *P)
{
    double sth = sqrt(fmax(0.0, 1.0 - mu * mu));
    double pmm = 1.0;
    for (int m = 0; m < nmax; m++) {
        if (m > 0) pmm *= -(2.0 * m - 1.0) * sth;
        P[m * nmax + m] = pmm;
        if (m + 1 < nmax) P[(m + 1) * nmax + m] = mu * (2.0 * m + 1.0) * pmm;
        for (int n = m + 2; n < nmax; n++)
            P[n * nmax + m] = ((2.0 * n - 1.0) * mu * P[(n - 1) * nmax + m] -
                               (n + m - 1.0) * P[(n - 2) * nmax + m]) / (double)(n - m);
    }
}

/* R_n^m(r) (eq. rsbf2) for n < nmax, all m. */
void lho_basis_R(int nmax, const double r[3], cplx *out)
{
    double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    memset(out, 0, sizeof(cplx) * (size_t)nmax * nmax);
    if (rr == 0.0) {
        out[0] = 1.0;
        return;
    }
    double mu = r[2] / rr, ph = atan2(r[1], r[0]);
    double *P = (double *)malloc(sizeof(double) * (size_t)nmax * nmax);
    legendre(nmax, mu, P);
    for (int n = 0; n < nmax; n++) {
        double rn = pow(rr, (double)n);
        for (int m = -n; m <= n; m++) {
            int am = abs(m);
            out[IDX(n, m)] = sgn_pow(n) * ipow(am) / fact(n + am) * rn * P[n * nmax + am] *
                             cexp(I * (double)m * ph);
        }
    }
    free(P);
}

/* S_n^m(r) (eq. rsbf2) for n < nmax, all m; r != 0. */
void lho_basis_S(int nmax, const double r[3], cplx *out)
{
    double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    double mu = r[2] / rr, ph = atan2(r[1], r[0]);
    double *P = (double *)malloc(sizeof(double) * (size_t)nmax * nmax);
    legendre(nmax, mu, P);
    for (int n = 0; n < nmax; n++) {
        double rn1 = pow(rr, -(double)(n + 1));
        for (int m = -n; m <= n; m++) {
            int am = abs(m);
            out[IDX(n, m)] = ipow(-am) * fact(n - am) * rn1 * P[n * nmax + am] *
                             cexp(I * (double)m * ph);
        }
    }
    free(P);
}

/* ------------------------------------------------------------------------- */
/* Smoothed core, eqs. 2 and vem1                                             */
/* ------------------------------------------------------------------------- */

/* f(r) = K(r;a)/r^3 and g(r) = f'(r)/r.  smooth = 0: singular kernel K = 1.
 * Gaussian core: K = erf(r/(a sqrt2)) - sqrt(2/pi)(r/a) exp(-r^2/2a^2),
 * K' = sqrt(2/pi) (r^2/a^3) exp(-r^2/2a^2).  For small u = r^2/(2a^2) the
 * closed form cancels, so the Taylor series of
 *   f = sqrt(2/pi)/a^3 * (1/r^3) int_0^r s^2 exp(-s^2/2a^2) ds
 *     = sqrt(2/pi)/a^3 * sum_k (-u)^k / (k! (2k+3))
 * and of g = (1/a^2) df/du is used there. */
void lho_kernel_fg(double r, double a, int smooth, double *f, double *g)
{
    if (!smooth) {
        double r2 = r * r;
        double ir3 = 1.0 / (r2 * r);
        *f = ir3;
        *g = -3.0 * ir3 / r2;
        return;
    }
    const double c = sqrt(2.0 / M_PI);
    double u = r * r / (2.0 * a * a);
    if (u < 0.02) {
        double fs = 0.0, gs = 0.0, term = 1.0; /* term = (-u)^k / k! */
        for (int k = 0; k < 12; k++) {
            fs += term / (2.0 * k + 3.0);
            term *= -u / (double)(k + 1);
        }
        /* g series: sum_{k>=1} (-1)^k u^{k-1} / ((k-1)! (2k+3)) */
        double t2 = -1.0; /* k=1: (-1)^1 u^0 / 0! */
        for (int k = 1; k < 13; k++) {
            gs += t2 / (2.0 * k + 3.0);
            t2 *= -u / (double)k;
        }
        *f = c / (a * a * a) * fs;
        *g = c / (a * a * a * a * a) * gs;
    } else {
        double K = erf(r / (a * sqrt(2.0))) - c * (r / a) * exp(-u);
        double r2 = r * r;
        *f = K / (r2 * r);
        *g = c * exp(-u) / (a * a * a * r2) - 3.0 * K / (r2 * r2 * r);
    }
}

/* contribution of source (xi, wi, qi) to target (xj, wj): v, grad v (row k = component,
 * column l = derivative) and s.  r = xj - xi.  The vortex part is eq. 1 with the kernel
 * f = K/r^3; the monopole (source) part qi is the term -grad(qi/r) of eq. 7, smoothed with
 * the same kernel: qi f r.  Its gradient is qi (f delta_kl + g r_k r_l) (g = f'/r). */
static void pair_accum(const double *xj, const double *wj, const double *xi, const double *wi, double qi,
                       double a, int smooth, double *v, double *s, double *gv)
{
    double r[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double rr = sqrt(r2);
    if (rr == 0.0 && !smooth) return; /* coincident distinct points, singular: defined as 0 */
    double f, g;
    lho_kernel_fg(rr, a, smooth, &f, &g);
    double wxr[3] = {wi[1] * r[2] - wi[2] * r[1], wi[2] * r[0] - wi[0] * r[2], wi[0] * r[1] - wi[1] * r[0]};
    double wxw[3] = {wi[1] * wj[2] - wi[2] * wj[1], wi[2] * wj[0] - wi[0] * wj[2], wi[0] * wj[1] - wi[1] * wj[0]};
    double wjr = wj[0] * r[0] + wj[1] * r[1] + wj[2] * r[2];
    for (int k = 0; k < 3; k++) {
        v[k] += f * wxr[k];
        s[k] += f * wxw[k] + g * wjr * wxr[k];
    }
    if (qi != 0.0)
        for (int k = 0; k < 3; k++) {
            v[k] += qi * f * r[k];
            s[k] += qi * (f * wj[k] + g * wjr * r[k]);
        }
    if (gv) {
        /* d_l (f (w x r))_k = g r_l (w x r)_k + f eps_{k a l} w_a */
        for (int k = 0; k < 3; k++)
            for (int l = 0; l < 3; l++) gv[3 * k + l] += g * r[l] * wxr[k];
        gv[3 * 0 + 1] += f * (-wi[2]); /* eps_{0 a 1}: a=2 -> eps_{021} = -1 */
        gv[3 * 0 + 2] += f * (wi[1]);  /* eps_{012} = +1 */
        gv[3 * 1 + 0] += f * (wi[2]);  /* eps_{120} = +1 */
        gv[3 * 1 + 2] += f * (-wi[0]); /* eps_{102} = -1 */
        gv[3 * 2 + 0] += f * (-wi[1]); /* eps_{210} = -1 */
        gv[3 * 2 + 1] += f * (wi[0]);  /* eps_{201} = +1 */
        if (qi != 0.0)
            for (int k = 0; k < 3; k++)
                for (int l = 0; l < 3; l++) gv[3 * k + l] += qi * (g * r[k] * r[l] + (k == l ? f : 0.0));
    }
}

/* ------------------------------------------------------------------------- */
/* Octree (uniform depth), rule stated in the header                          */
/* ------------------------------------------------------------------------- */

static uint64_t spread3(uint32_t v)
{
    uint64_t k = 0;
    for (int b = 0; b < QBITS; b++) k |= (uint64_t)((v >> b) & 1u) << (3 * b);
    return k;
}
static uint32_t gather3(uint64_t k)
{
    uint32_t v = 0;
    for (int b = 0; b < QBITS; b++) v |= (uint32_t)((k >> (3 * b)) & 1u) << b;
    return v;
}
static uint64_t morton(uint32_t ix, uint32_t iy, uint32_t iz)
{
    return spread3(ix) | (spread3(iy) << 1) | (spread3(iz) << 2);
}

/* integer coordinate of one component: min(floor((x-lo)*(2^21/L)), 2^21-1) */
static uint32_t qcoord(double x, double lo, double scale)
{
    double t = (x - lo) * scale;
    double fl = floor(t);
    if (fl < 0.0) fl = 0.0; /* callers validate the domain; clamp for safety */
    if (fl > (double)((1u << QBITS) - 1u)) fl = (double)((1u << QBITS) - 1u);
    return (uint32_t)fl;
}

typedef struct {
    int depth;
    double lo[3], L;
    int64_t n;
    uint32_t *q;     /* [n][3] integer coordinates */
    int64_t *order;  /* particle indices sorted by leaf key (stable) */
    int64_t nb[MAXLEV + 1];
    uint64_t *key[MAXLEV + 1];
    int64_t *first[MAXLEV + 1];
    int64_t *count[MAXLEV + 1];
} otree;

typedef struct {
    uint64_t k;
    int64_t i;
} kidx;

static int cmp_kidx(const void *a, const void *b)
{
    const kidx *x = (const kidx *)a, *y = (const kidx *)b;
    if (x->k < y->k) return -1;
    if (x->k > y->k) return 1;
    return (x->i < y->i) ? -1 : (x->i > y->i);
}

static void tree_build(otree *T, int64_t n, const double *x, int depth, const double lo[3], double L)
{
    memset(T, 0, sizeof(*T));
    T->depth = depth;
    T->n = n;
    T->L = L;
    for (int d = 0; d < 3; d++) T->lo[d] = lo[d];
    double scale = (double)(1u << QBITS) / L;
    T->q = (uint32_t *)malloc(sizeof(uint32_t) * 3 * (size_t)n);
    kidx *ki = (kidx *)malloc(sizeof(kidx) * (size_t)n);
    for (int64_t i = 0; i < n; i++) {
        for (int d = 0; d < 3; d++) T->q[3 * i + d] = qcoord(x[3 * i + d], lo[d], scale);
        int sh = QBITS - depth;
        ki[i].k = morton(T->q[3 * i] >> sh, T->q[3 * i + 1] >> sh, T->q[3 * i + 2] >> sh);
        ki[i].i = i;
    }
    qsort(ki, (size_t)n, sizeof(kidx), cmp_kidx);
    T->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; i++) T->order[i] = ki[i].i;
    for (int l = 0; l <= depth; l++) {
        int sh = 3 * (depth - l);
        int64_t nb = 0;
        for (int64_t i = 0; i < n; i++)
            if (i == 0 || (ki[i].k >> sh) != (ki[i - 1].k >> sh)) nb++;
        T->nb[l] = nb;
        T->key[l] = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nb + 1));
        T->first[l] = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb + 1));
        T->count[l] = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb + 1));
        int64_t b = -1;
        for (int64_t i = 0; i < n; i++) {
            if (i == 0 || (ki[i].k >> sh) != (ki[i - 1].k >> sh)) {
                b++;
                T->key[l][b] = ki[i].k >> sh;
                T->first[l][b] = i;
                T->count[l][b] = 0;
            }
            T->count[l][b]++;
        }
    }
    free(ki);
}

static void tree_free(otree *T)
{
    free(T->q);
    free(T->order);
    for (int l = 0; l <= T->depth; l++) {
        free(T->key[l]);
        free(T->first[l]);
        free(T->count[l]);
    }
}

/* index of the box with Morton key k at level l, or -1 */
static int64_t tree_find(const otree *T, int l, uint64_t k)
{
    int64_t lo = 0, hi = T->nb[l] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (T->key[l][mid] == k) return mid;
        if (T->key[l][mid] < k) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

static void box_coords(uint64_t k, int c[3])
{
    c[0] = (int)gather3(k);
    c[1] = (int)gather3(k >> 1);
    c[2] = (int)gather3(k >> 2);
}

static void box_centre(const otree *T, int l, uint64_t k, double c[3])
{
    int ic[3];
    box_coords(k, ic);
    double h = T->L / (double)(1u << l);
    for (int d = 0; d < 3; d++) c[d] = T->lo[d] + ((double)ic[d] + 0.5) * h;
}

/* ------------------------------------------------------------------------- */
/* P2M, Sec. 4.3                                                              */
/* ------------------------------------------------------------------------- */

/* Method 2 (eq. eve4): add the (phi, chi) multipole coefficients about
 * 'centre' of the vortex elements (x_l, w_l) into phi, chi (p^2 each). */
void lho_p2m_method2(int p, const double centre[3], int64_t n, const double *x, const double *w, const double *q,
                     cplx *phi, cplx *chi)
{
    cplx *g = (cplx *)malloc(sizeof(cplx) * (size_t)p * p);
    cplx *R = (cplx *)malloc(sizeof(cplx) * (size_t)p * p);
    for (int64_t l = 0; l < n; l++) {
        double mr[3] = {-(x[3 * l] - centre[0]), -(x[3 * l + 1] - centre[1]), -(x[3 * l + 2] - centre[2])};
        lho_basis_R(p, mr, R);
        /* g_n^m = R_n^{-m}(-r_l) */
        for (int nn = 0; nn < p; nn++)
            for (int m = -nn; m <= nn; m++) g[IDX(nn, m)] = R[IDX(nn, -m)];
        double wx = w[3 * l], wy = w[3 * l + 1], wz = w[3 * l + 2];
        for (int nn = 0; nn < p; nn++)
            for (int m = -nn; m <= nn; m++) {
                cplx a = (wx - I * wy) * (nn - m + 1) / 2.0 * cget(g, p, nn, m - 1) -
                         (wx + I * wy) * (nn + m + 1) / 2.0 * cget(g, p, nn, m + 1) -
                         I * wz * (double)m * cget(g, p, nn, m);
                phi[IDX(nn, m)] += a / (double)(nn + 1);
                /* monopole (eq. 7): phi gains -q_l / |y - x_l| = -q_l sum g_n^m S_n^m (eq. rsbf5) */
                if (q) phi[IDX(nn, m)] -= q[l] * cget(g, p, nn, m);
                if (nn > 0) {
                    cplx b = 0.5 * (wy + I * wx) * cget(g, p, nn - 1, m - 1) -
                             0.5 * (wy - I * wx) * cget(g, p, nn - 1, m + 1) -
                             wz * cget(g, p, nn - 1, m);
                    chi[IDX(nn, m)] += -b / (double)nn;
                }
            }
    }
    free(g);
    free(R);
}

/* Method 1 (eqs. eve5-eve10): psi and varpi are dipoles with moments
 * r_l x w_l and -w_l; the dipole expansion is obtained by differentiating
 * eq. rsbf5 with respect to the source point, using eq. dt2:
 *   psi_n^m = -1/2 (P_y + i P_x) g_{n-1}^{m-1} + 1/2 (P_y - i P_x) g_{n-1}^{m+1} + P_z g_{n-1}^m,
 * then phi_n^m = -psi_n^m/(n+1), chi_n^m = -varpi_n^m/n, chi_0^0 = 0. */
void lho_p2m_method1(int p, const double centre[3], int64_t n, const double *x, const double *w,
                     cplx *phi, cplx *chi)
{
    cplx *g = (cplx *)malloc(sizeof(cplx) * (size_t)p * p);
    cplx *R = (cplx *)malloc(sizeof(cplx) * (size_t)p * p);
    for (int64_t l = 0; l < n; l++) {
        double rl[3] = {x[3 * l] - centre[0], x[3 * l + 1] - centre[1], x[3 * l + 2] - centre[2]};
        double mr[3] = {-rl[0], -rl[1], -rl[2]};
        lho_basis_R(p, mr, R);
        for (int nn = 0; nn < p; nn++)
            for (int m = -nn; m <= nn; m++) g[IDX(nn, m)] = R[IDX(nn, -m)];
        const double *wl = &w[3 * l];
        double P[3] = {rl[1] * wl[2] - rl[2] * wl[1], rl[2] * wl[0] - rl[0] * wl[2], rl[0] * wl[1] - rl[1] * wl[0]};
        double Q[3] = {-wl[0], -wl[1], -wl[2]};
        for (int nn = 1; nn < p; nn++)
            for (int m = -nn; m <= nn; m++) {
                cplx psi = -0.5 * (P[1] + I * P[0]) * cget(g, p, nn - 1, m - 1) +
                           0.5 * (P[1] - I * P[0]) * cget(g, p, nn - 1, m + 1) + P[2] * cget(g, p, nn - 1, m);
                cplx vpi = -0.5 * (Q[1] + I * Q[0]) * cget(g, p, nn - 1, m - 1) +
                           0.5 * (Q[1] - I * Q[0]) * cget(g, p, nn - 1, m + 1) + Q[2] * cget(g, p, nn - 1, m);
                phi[IDX(nn, m)] += -psi / (double)(nn + 1);
                chi[IDX(nn, m)] += -vpi / (double)nn;
            }
    }
    free(g);
    free(R);
}

/* ------------------------------------------------------------------------- */
/* Translations: eq. mr3 (full matrices) + conversion, eqs. drt10 / drt11    */
/* ------------------------------------------------------------------------- */

/* R-basis conversion (eq. drt10) of translated (ph, ch) with general t.
 * ph has p orders, ch has pc orders (pc = p or p+1); result truncated to p. */
static void convert_R(int p, int pc, const double t[3], const cplx *ph, const cplx *ch, cplx *outph,
                      cplx *outch)
{
    cplx tp = t[0] + I * t[1], tm = t[0] - I * t[1];
    cplx sp = t[1] + I * t[0], sm = t[1] - I * t[0];
    for (int n = 0; n < p; n++)
        for (int m = -n; m <= n; m++) {
            cplx f = ph[IDX(n, m)];
            if (n > 0)
                f -= (tp * (double)(n - m) / 2.0 * cget(ch, pc, n, m + 1) -
                      tm * (double)(n + m) / 2.0 * cget(ch, pc, n, m - 1) -
                      I * t[2] * (double)m * cget(ch, pc, n, m)) / (double)n;
            cplx c = cget(ch, pc, n, m) +
                     (0.5 * sp * cget(ch, pc, n + 1, m - 1) - 0.5 * sm * cget(ch, pc, n + 1, m + 1) -
                      t[2] * cget(ch, pc, n + 1, m)) / (double)(n + 1);
            outph[IDX(n, m)] = f;
            outch[IDX(n, m)] = c;
        }
}

/* S-basis conversion (eq. drt11), p orders in and out. */
static void convert_S(int p, const double t[3], const cplx *ph, const cplx *ch, cplx *outph, cplx *outch)
{
    cplx tp = t[0] + I * t[1], tm = t[0] - I * t[1];
    cplx sp = t[1] + I * t[0], sm = t[1] - I * t[0];
    for (int n = 0; n < p; n++)
        for (int m = -n; m <= n; m++) {
            cplx f = ph[IDX(n, m)] +
                     (-tp * (double)(n + m + 1) / 2.0 * cget(ch, p, n, m + 1) +
                      tm * (double)(n - m + 1) / 2.0 * cget(ch, p, n, m - 1) -
                      I * t[2] * (double)m * cget(ch, p, n, m)) / (double)(n + 1);
            cplx c = ch[IDX(n, m)];
            if (n > 0)
                c -= (0.5 * sp * cget(ch, p, n - 1, m - 1) - 0.5 * sm * cget(ch, p, n - 1, m + 1) -
                      t[2] * cget(ch, p, n - 1, m)) / (double)n;
            outph[IDX(n, m)] = f;
            outch[IDX(n, m)] = c;
        }
}

/* M2M: multipole (phi, chi) about c_old -> about c_new, t = c_new - c_old.
 * (S|S): hat_n^m = sum_{n'<=n, m'} R_{n-n'}^{m'-m}(t) in_{n'}^{m'}; then drt11.
 * Result is ADDED into (oph, och). */
void lho_m2m(int p, const double t[3], const cplx *phi, const cplx *chi, cplx *oph, cplx *och)
{
    size_t P2 = (size_t)p * p;
    cplx *Rt = (cplx *)malloc(sizeof(cplx) * P2);
    cplx *hp = (cplx *)calloc(P2, sizeof(cplx)), *hc = (cplx *)calloc(P2, sizeof(cplx));
    cplx *tp = (cplx *)malloc(sizeof(cplx) * P2), *tc = (cplx *)malloc(sizeof(cplx) * P2);
    lho_basis_R(p, t, Rt);
    for (int n = 0; n < p; n++)
        for (int m = -n; m <= n; m++) {
            cplx ap = 0.0, ac = 0.0;
            for (int n2 = 0; n2 <= n; n2++)
                for (int m2 = -n2; m2 <= n2; m2++) {
                    cplx c = cget(Rt, p, n - n2, m2 - m);
                    ap += c * phi[IDX(n2, m2)];
                    ac += c * chi[IDX(n2, m2)];
                }
            hp[IDX(n, m)] = ap;
            hc[IDX(n, m)] = ac;
        }
    convert_S(p, t, hp, hc, tp, tc);
    for (size_t k = 0; k < P2; k++) {
        oph[k] += tp[k];
        och[k] += tc[k];
    }
    free(Rt);
    free(hp);
    free(hc);
    free(tp);
    free(tc);
}

/* M2L: multipole about c_s -> local about c_t, t = c_t - c_s.
 * (S|R): hat_n^m = sum_{n'<p, m'} S_{n+n'}^{m'-m}(t) in_{n'}^{m'}, phi-hat for
 * n<p, chi-hat for n<=p (reading B), then drt10 truncated to n<p.  ADDED. */
void lho_m2l(int p, const double t[3], const cplx *phi, const cplx *chi, cplx *oph, cplx *och)
{
    int ns = 2 * p + 1;
    size_t P2 = (size_t)p * p, P21 = (size_t)(p + 1) * (p + 1);
    cplx *St = (cplx *)malloc(sizeof(cplx) * (size_t)ns * ns);
    cplx *hp = (cplx *)calloc(P2, sizeof(cplx)), *hc = (cplx *)calloc(P21, sizeof(cplx));
    cplx *tp = (cplx *)malloc(sizeof(cplx) * P2), *tc = (cplx *)malloc(sizeof(cplx) * P2);
    lho_basis_S(ns, t, St);
    for (int n = 0; n <= p; n++)
        for (int m = -n; m <= n; m++) {
            cplx ap = 0.0, ac = 0.0;
            for (int n2 = 0; n2 < p; n2++)
                for (int m2 = -n2; m2 <= n2; m2++) {
                    cplx c = cget(St, ns, n + n2, m2 - m);
                    ap += c * phi[IDX(n2, m2)];
                    ac += c * chi[IDX(n2, m2)];
                }
            if (n < p) hp[IDX(n, m)] = ap;
            hc[IDX(n, m)] = ac;
        }
    convert_R(p, p + 1, t, hp, hc, tp, tc);
    for (size_t k = 0; k < P2; k++) {
        oph[k] += tp[k];
        och[k] += tc[k];
    }
    free(St);
    free(hp);
    free(hc);
    free(tp);
    free(tc);
}

/* L2L: local about c_old -> local about c_new, t = c_new - c_old.
 * (R|R): hat_n^m = sum_{n'>=n, m'} R_{n'-n}^{m'-m}(t) in_{n'}^{m'}; drt10. ADDED. */
void lho_l2l(int p, const double t[3], const cplx *phi, const cplx *chi, cplx *oph, cplx *och)
{
    size_t P2 = (size_t)p * p;
    cplx *Rt = (cplx *)malloc(sizeof(cplx) * P2);
    cplx *hp = (cplx *)calloc(P2, sizeof(cplx)), *hc = (cplx *)calloc(P2, sizeof(cplx));
    cplx *tp = (cplx *)malloc(sizeof(cplx) * P2), *tc = (cplx *)malloc(sizeof(cplx) * P2);
    lho_basis_R(p, t, Rt);
    for (int n = 0; n < p; n++)
        for (int m = -n; m <= n; m++) {
            cplx ap = 0.0, ac = 0.0;
            for (int n2 = n; n2 < p; n2++)
                for (int m2 = -n2; m2 <= n2; m2++) {
                    cplx c = cget(Rt, p, n2 - n, m2 - m);
                    ap += c * phi[IDX(n2, m2)];
                    ac += c * chi[IDX(n2, m2)];
                }
            hp[IDX(n, m)] = ap;
            hc[IDX(n, m)] = ac;
        }
    convert_R(p, p, t, hp, hc, tp, tc);
    for (size_t k = 0; k < P2; k++) {
        oph[k] += tp[k];
        och[k] += tc[k];
    }
    free(Rt);
    free(hp);
    free(hc);
    free(tp);
    free(tc);
}

/* ------------------------------------------------------------------------- */
/* L2P, Sec. 4.5                                                              */
/* ------------------------------------------------------------------------- */

/* velocity coefficients v_k (eq. evf3) from local (phi, chi), p orders */
static void vel_coeffs(int p, const cplx *phi, const cplx *chi, cplx *vx, cplx *vy, cplx *vz)
{
    for (int n = 0; n < p; n++)
        for (int m = -n; m <= n; m++) {
            cplx pm1 = cget(phi, p, n + 1, m - 1), pp1 = cget(phi, p, n + 1, m + 1), p0 = cget(phi, p, n + 1, m);
            cplx cm1 = cget(chi, p, n, m - 1), cp1 = cget(chi, p, n, m + 1), c0 = cget(chi, p, n, m);
            vx[IDX(n, m)] = 0.5 * (I * pm1 + I * pp1 + (double)(n - m) * cp1 - (double)(n + m) * cm1);
            vy[IDX(n, m)] = 0.5 * (pm1 - pp1 + I * (double)(n - m) * cp1 + I * (double)(n + m) * cm1);
            vz[IDX(n, m)] = -p0 - I * (double)m * c0;
        }
}

/* D_t in the R basis (eq. dt3): out_n^m = 1/2 (ty + i tx) in_{n+1}^{m-1}
 *   - 1/2 (ty - i tx) in_{n+1}^{m+1} - tz in_{n+1}^m */
static void apply_Dt_R(int p, const double t[3], const cplx *in, cplx *out)
{
    cplx sp = t[1] + I * t[0], sm = t[1] - I * t[0];
    for (int n = 0; n < p; n++)
        for (int m = -n; m <= n; m++)
            out[IDX(n, m)] = 0.5 * sp * cget(in, p, n + 1, m - 1) - 0.5 * sm * cget(in, p, n + 1, m + 1) -
                             t[2] * cget(in, p, n + 1, m);
}

/* Evaluate the local expansion (phi, chi) about 'centre' at the points x with
 * strengths w: v (3), s (3), grad v (9, row = component, col = derivative),
 * optional imaginary parts of v (3) and grad v (9) (they must vanish).  ADDED. */
void lho_l2p(int p, const double centre[3], const cplx *phi, const cplx *chi, int64_t n, const double *x,
             const double *w, double *v, double *s, double *gv, double *imv, double *imgv)
{
    size_t P2 = (size_t)p * p;
    cplx *vk[3], *u[3][3];
    for (int k = 0; k < 3; k++) {
        vk[k] = (cplx *)malloc(sizeof(cplx) * P2);
        for (int l = 0; l < 3; l++) u[l][k] = (cplx *)malloc(sizeof(cplx) * P2);
    }
    vel_coeffs(p, phi, chi, vk[0], vk[1], vk[2]);
    /* u_lk = D_{e_l} v_k (eq. evf6) */
    for (int l = 0; l < 3; l++) {
        double e[3] = {0, 0, 0};
        e[l] = 1.0;
        for (int k = 0; k < 3; k++) apply_Dt_R(p, e, vk[k], u[l][k]);
    }
    cplx *R = (cplx *)malloc(sizeof(cplx) * P2);
    for (int64_t j = 0; j < n; j++) {
        double r[3] = {x[3 * j] - centre[0], x[3 * j + 1] - centre[1], x[3 * j + 2] - centre[2]};
        lho_basis_R(p, r, R);
        cplx V[3] = {0, 0, 0}, G[3][3] = {{0}};
        for (size_t q = 0; q < P2; q++) {
            for (int k = 0; k < 3; k++) {
                V[k] += vk[k][q] * R[q];
                for (int l = 0; l < 3; l++) G[k][l] += u[l][k][q] * R[q];
            }
        }
        const double *wj = &w[3 * j];
        for (int k = 0; k < 3; k++) {
            v[3 * j + k] += creal(V[k]);
            if (imv) imv[3 * j + k] += cimag(V[k]);
            /* s_k = sum_l w_l u_lk (eq. evf6) */
            s[3 * j + k] += wj[0] * creal(G[k][0]) + wj[1] * creal(G[k][1]) + wj[2] * creal(G[k][2]);
            for (int l = 0; l < 3; l++) {
                if (gv) gv[9 * j + 3 * k + l] += creal(G[k][l]);
                if (imgv) imgv[9 * j + 3 * k + l] += cimag(G[k][l]);
            }
        }
    }
    free(R);
    for (int k = 0; k < 3; k++) {
        free(vk[k]);
        for (int l = 0; l < 3; l++) free(u[l][k]);
    }
}

/* P2L: local (R-basis) expansion about centre of the field of elements (x, w, q) lying
 * outside its ball.  Defined as the translation (M2L with the R-basis conversion, reading B)
 * of each element's own multipole expansion about its position: an element at the centre of
 * its expansion has no truncation error (orders n <= 1 only), so the local coefficients of
 * orders n <= p-1 are exact.  ADDED into (phi, chi). */
void lho_p2l(int p, const double centre[3], int64_t n, const double *x, const double *w, const double *q,
             cplx *phi, cplx *chi)
{
    size_t P2 = (size_t)p * p;
    cplx *mp = (cplx *)malloc(sizeof(cplx) * P2), *mc = (cplx *)malloc(sizeof(cplx) * P2);
    for (int64_t l = 0; l < n; l++) {
        memset(mp, 0, sizeof(cplx) * P2);
        memset(mc, 0, sizeof(cplx) * P2);
        lho_p2m_method2(p, &x[3 * l], 1, &x[3 * l], &w[3 * l], q ? &q[l] : NULL, mp, mc);
        double t[3] = {centre[0] - x[3 * l], centre[1] - x[3 * l + 1], centre[2] - x[3 * l + 2]};
        lho_m2l(p, t, mp, mc, phi, chi);
    }
    free(mp);
    free(mc);
}

/* M2P: the field of a multipole expansion (phi, chi) about centre (p orders) at target
 * points y outside its ball: v, s = (w_j . grad) v (w: strengths at the targets) and, if g is
 * not NULL, grad v (row = component, column = derivative).  Defined as the translation of the
 * expansion to a local expansion about the target itself (M2L, at least three orders so that
 * the orders n <= 2 the evaluation needs are formed) evaluated at its centre (L2P at r = 0):
 * the exact field of the truncated multipole expansion.  ADDED into v, s, g. */
void lho_m2p(int p, const double centre[3], const cplx *phi, const cplx *chi, int64_t n, const double *y,
             const double *w, double *v, double *s, double *g)
{
    int pl = p < 3 ? 3 : p;
    size_t PL2 = (size_t)pl * pl, P2 = (size_t)p * p;
    cplx *ip = (cplx *)calloc(PL2, sizeof(cplx)), *ic = (cplx *)calloc(PL2, sizeof(cplx));
    cplx *lp = (cplx *)malloc(sizeof(cplx) * PL2), *lc = (cplx *)malloc(sizeof(cplx) * PL2);
    memcpy(ip, phi, sizeof(cplx) * P2);
    memcpy(ic, chi, sizeof(cplx) * P2);
    for (int64_t j = 0; j < n; j++) {
        memset(lp, 0, sizeof(cplx) * PL2);
        memset(lc, 0, sizeof(cplx) * PL2);
        double t[3] = {y[3 * j] - centre[0], y[3 * j + 1] - centre[1], y[3 * j + 2] - centre[2]};
        lho_m2l(pl, t, ip, ic, lp, lc);
        double vv[3] = {0, 0, 0}, ss[3] = {0, 0, 0}, gg[9] = {0};
        lho_l2p(pl, &y[3 * j], lp, lc, 1, &y[3 * j], &w[3 * j], vv, ss, gg, NULL, NULL);
        for (int k = 0; k < 3; k++) {
            v[3 * j + k] += vv[k];
            s[3 * j + k] += ss[k];
        }
        if (g)
            for (int k = 0; k < 9; k++) g[9 * j + k] += gg[k];
    }
    free(ip);
    free(ic);
    free(lp);
    free(lc);
}

/* ------------------------------------------------------------------------- */
/* (A) direct sums                                                            */
/* ------------------------------------------------------------------------- */

/* mode 0: singular kernel everywhere; 1: smoothed everywhere;
 * 2: split by the uniform octree of depth 'depth' on the cube [lo, lo+L]^3:
 *    smoothed if the leaves of source and target are adjacent, else singular.
 * Targets: ntarg indices into the n elements (all if targ == NULL).
 * Outputs are indexed by target position in the list. */
void lho_direct(int64_t n, const double *x, const double *w, const double *q, double a, int mode, int depth,
                const double lo[3], double L, int64_t ntarg, const int64_t *targ, double *v, double *s,
                double *gv)
{
    uint32_t *lq = NULL;
    if (mode == 2) {
        double scale = (double)(1u << QBITS) / L;
        lq = (uint32_t *)malloc(sizeof(uint32_t) * 3 * (size_t)n);
        for (int64_t i = 0; i < n; i++)
            for (int d = 0; d < 3; d++) lq[3 * i + d] = qcoord(x[3 * i + d], lo[d], scale) >> (QBITS - depth);
    }
    int64_t nt = targ ? ntarg : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t jj = 0; jj < nt; jj++) {
        int64_t j = targ ? targ[jj] : jj;
        double vv[3] = {0, 0, 0}, ss[3] = {0, 0, 0}, gg[9] = {0};
        for (int64_t i = 0; i < n; i++) {
            if (i == j) continue;
            int smooth = (mode == 1);
            if (mode == 2) {
                int adj = 1;
                for (int d = 0; d < 3; d++) {
                    int64_t dd = (int64_t)lq[3 * i + d] - (int64_t)lq[3 * j + d];
                    if (dd < -1 || dd > 1) adj = 0;
                }
                smooth = adj;
            }
            pair_accum(&x[3 * j], &w[3 * j], &x[3 * i], &w[3 * i], q ? q[i] : 0.0, a, smooth, vv, ss,
                       gv ? gg : NULL);
        }
        for (int k = 0; k < 3; k++) {
            v[3 * jj + k] = vv[k];
            s[3 * jj + k] = ss[k];
        }
        if (gv)
            for (int k = 0; k < 9; k++) gv[9 * jj + k] = gg[k];
    }
    free(lq);
}

/* ------------------------------------------------------------------------- */
/* (B) the FMM                                                                */
/* ------------------------------------------------------------------------- */

typedef struct {
    int64_t n_m2l, n_m2m, n_l2l, n_p2p_pairs;
    double t_tree, t_up, t_down, t_near; /* wall-clock seconds of the phases */
    int64_t n_wx_pairs;                  /* adaptive: W/X pairs summed directly (singular) */
    int64_t n_leaf, n_box;               /* adaptive: leaves and boxes of the tree */
    int32_t max_level, reserved;
} lho_stats;

static double wtime(void)
{
#ifdef _OPENMP
    return omp_get_wtime();
#else
    return 0.0;
#endif
}

/* Visit the V-list (interaction list) of box (l, k): children of the parent's
 * neighbours that are not adjacent to the box and are non-empty. */
static int vlist(const otree *T, int l, uint64_t k, int64_t *out)
{
    int c[3];
    box_coords(k, c);
    int nside = 1 << l;
    int cnt = 0;
    int pc[3] = {c[0] >> 1, c[1] >> 1, c[2] >> 1};
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                int np[3] = {pc[0] + dx, pc[1] + dy, pc[2] + dz};
                for (int ch = 0; ch < 8; ch++) {
                    int cc[3] = {2 * np[0] + (ch & 1), 2 * np[1] + ((ch >> 1) & 1), 2 * np[2] + ((ch >> 2) & 1)};
                    if (cc[0] < 0 || cc[1] < 0 || cc[2] < 0 || cc[0] >= nside || cc[1] >= nside || cc[2] >= nside)
                        continue;
                    if (abs(cc[0] - c[0]) <= 1 && abs(cc[1] - c[1]) <= 1 && abs(cc[2] - c[2]) <= 1) continue;
                    int64_t b = tree_find(T, l, morton((uint32_t)cc[0], (uint32_t)cc[1], (uint32_t)cc[2]));
                    if (b >= 0) out[cnt++] = b;
                }
            }
    return cnt;
}

/* gather the elements of box (l, b) */
static void box_points(const otree *T, const double *x, const double *w, const double *q, int l, int64_t b,
                       double *bx, double *bw, double *bq)
{
    int64_t f = T->first[l][b], c = T->count[l][b];
    for (int64_t i = 0; i < c; i++) {
        int64_t e = T->order[f + i];
        for (int d = 0; d < 3; d++) {
            bx[3 * i + d] = x[3 * e + d];
            bw[3 * i + d] = w[3 * e + d];
        }
        if (q) bq[i] = q[e];
    }
}

/* Full or leaf-sampled FMM evaluation of v and s (and optionally grad v).
 *  what: bit 0 = far field (expansions), bit 1 = near field (direct, U-list).
 *  sample: list of element indices; only the leaves holding them are
 *          evaluated (their outputs written, others untouched); NULL = all.
 *  p2m_method: 1 or 2.
 * Returns 0 on success. */
int lho_fmm(int64_t n, const double *x, const double *w, const double *q, double a, int p, int depth,
            const double lo[3], double L, int what, int p2m_method, int64_t nsample, const int64_t *sample,
            double *v, double *s, double *gv, lho_stats *st)
{
    if (depth < 2 || depth > 10 || p < 1 || n < 1) return -1;
    double t0 = wtime();
    otree T;
    tree_build(&T, n, x, depth, lo, L);
    size_t P2 = (size_t)p * p;
    int smooth = a > 0.0;
    lho_stats stats;
    memset(&stats, 0, sizeof(stats));
    stats.t_tree = wtime() - t0;

    /* which leaves to evaluate */
    int64_t nleaf = T.nb[depth];
    char *want = (char *)calloc((size_t)nleaf, 1);
    if (!sample) {
        memset(want, 1, (size_t)nleaf);
    } else {
        int sh = QBITS - depth;
        for (int64_t i = 0; i < nsample; i++) {
            int64_t e = sample[i];
            uint64_t k = morton(T.q[3 * e] >> sh, T.q[3 * e + 1] >> sh, T.q[3 * e + 2] >> sh);
            int64_t b = tree_find(&T, depth, k);
            if (b >= 0) want[b] = 1;
        }
    }

    if (what & 1) {
        /* ---------- upward pass: P2M at leaves, M2M to level 2 ---------- */
        double t1 = wtime();
        cplx *M[MAXLEV + 1];
        for (int l = 2; l <= depth; l++) M[l] = (cplx *)calloc((size_t)T.nb[l] * 2 * P2, sizeof(cplx));
#pragma omp parallel
        {
            double *bx = NULL, *bw = NULL, *bq = NULL;
            int64_t cap = 0;
#pragma omp for schedule(dynamic, 4)
            for (int64_t b = 0; b < nleaf; b++) {
                int64_t c = T.count[depth][b];
                if (c > cap) {
                    free(bx);
                    free(bw);
                    free(bq);
                    cap = c;
                    bx = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                    bw = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                    bq = (double *)malloc(sizeof(double) * (size_t)cap);
                }
                box_points(&T, x, w, q, depth, b, bx, bw, bq);
                double cen[3];
                box_centre(&T, depth, T.key[depth][b], cen);
                cplx *ph = &M[depth][(size_t)b * 2 * P2], *ch = ph + P2;
                if (p2m_method == 1) lho_p2m_method1(p, cen, c, bx, bw, ph, ch);
                else lho_p2m_method2(p, cen, c, bx, bw, q ? bq : NULL, ph, ch);
            }
            free(bx);
            free(bw);
            free(bq);
        }
        for (int l = depth - 1; l >= 2; l--) {
            int sh = 3;
#pragma omp parallel for schedule(dynamic, 4)
            for (int64_t b = 0; b < T.nb[l]; b++) {
                double cp[3];
                box_centre(&T, l, T.key[l][b], cp);
                cplx *ph = &M[l][(size_t)b * 2 * P2], *ch = ph + P2;
                for (int chn = 0; chn < 8; chn++) {
                    int64_t cb = tree_find(&T, l + 1, (T.key[l][b] << sh) | (uint64_t)chn);
                    if (cb < 0) continue;
                    double cc[3];
                    box_centre(&T, l + 1, T.key[l + 1][cb], cc);
                    double t[3] = {cp[0] - cc[0], cp[1] - cc[1], cp[2] - cc[2]};
                    const cplx *iph = &M[l + 1][(size_t)cb * 2 * P2];
                    lho_m2m(p, t, iph, iph + P2, ph, ch);
                }
            }
        }

        stats.t_up = wtime() - t1;
        t1 = wtime();
        /* ---------- downward pass ---------- */
        if (!sample) {
            cplx *Lc[MAXLEV + 1];
            for (int l = 2; l <= depth; l++) Lc[l] = (cplx *)calloc((size_t)T.nb[l] * 2 * P2, sizeof(cplx));
            int64_t nm2l = 0, nl2l = 0;
            for (int l = 2; l <= depth; l++) {
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : nm2l, nl2l)
                for (int64_t b = 0; b < T.nb[l]; b++) {
                    double ct[3];
                    box_centre(&T, l, T.key[l][b], ct);
                    cplx *ph = &Lc[l][(size_t)b * 2 * P2], *ch = ph + P2;
                    if (l > 2) {
                        int64_t pb = tree_find(&T, l - 1, T.key[l][b] >> 3);
                        double cp[3];
                        box_centre(&T, l - 1, T.key[l - 1][pb], cp);
                        double t[3] = {ct[0] - cp[0], ct[1] - cp[1], ct[2] - cp[2]};
                        const cplx *iph = &Lc[l - 1][(size_t)pb * 2 * P2];
                        lho_l2l(p, t, iph, iph + P2, ph, ch);
                        nl2l++;
                    }
                    int64_t vl[189];
                    int nv = vlist(&T, l, T.key[l][b], vl);
                    for (int i = 0; i < nv; i++) {
                        double cs[3];
                        box_centre(&T, l, T.key[l][vl[i]], cs);
                        double t[3] = {ct[0] - cs[0], ct[1] - cs[1], ct[2] - cs[2]};
                        const cplx *iph = &M[l][(size_t)vl[i] * 2 * P2];
                        lho_m2l(p, t, iph, iph + P2, ph, ch);
                    }
                    nm2l += nv;
                }
            }
            stats.n_m2l = nm2l;
            stats.n_l2l = nl2l;
            /* L2P */
#pragma omp parallel
            {
                double *bx = NULL, *bw = NULL, *bv = NULL, *bs = NULL, *bg = NULL;
                int64_t cap = 0;
#pragma omp for schedule(dynamic, 4)
                for (int64_t b = 0; b < nleaf; b++) {
                    if (!want[b]) continue;
                    int64_t c = T.count[depth][b];
                    if (c > cap) {
                        free(bx); free(bw); free(bv); free(bs); free(bg);
                        cap = c;
                        bx = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                        bw = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                        bv = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                        bs = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                        bg = (double *)malloc(sizeof(double) * 9 * (size_t)cap);
                    }
                    box_points(&T, x, w, NULL, depth, b, bx, bw, NULL);
                    memset(bv, 0, sizeof(double) * 3 * (size_t)c);
                    memset(bs, 0, sizeof(double) * 3 * (size_t)c);
                    memset(bg, 0, sizeof(double) * 9 * (size_t)c);
                    double cen[3];
                    box_centre(&T, depth, T.key[depth][b], cen);
                    const cplx *ph = &Lc[depth][(size_t)b * 2 * P2];
                    lho_l2p(p, cen, ph, ph + P2, c, bx, bw, bv, bs, bg, NULL, NULL);
                    for (int64_t i = 0; i < c; i++) {
                        int64_t e = T.order[T.first[depth][b] + i];
                        for (int d = 0; d < 3; d++) {
                            v[3 * e + d] += bv[3 * i + d];
                            s[3 * e + d] += bs[3 * i + d];
                        }
                        if (gv)
                            for (int d = 0; d < 9; d++) gv[9 * e + d] += bg[9 * i + d];
                    }
                }
                free(bx); free(bw); free(bv); free(bs); free(bg);
            }
            for (int l = 2; l <= depth; l++) free(Lc[l]);
        } else {
            /* leaf-sampled: for each wanted leaf walk its ancestor chain */
            int64_t nm2l = 0;
#pragma omp parallel
            {
                cplx *chain = (cplx *)malloc(sizeof(cplx) * 2 * P2 * (size_t)(depth + 1));
                double *bx = NULL, *bw = NULL, *bv = NULL, *bs = NULL, *bg = NULL;
                int64_t cap = 0;
#pragma omp for schedule(dynamic, 1) reduction(+ : nm2l)
                for (int64_t b = 0; b < nleaf; b++) {
                    if (!want[b]) continue;
                    memset(chain, 0, sizeof(cplx) * 2 * P2 * (size_t)(depth + 1));
                    uint64_t lk = T.key[depth][b];
                    for (int l = 2; l <= depth; l++) {
                        uint64_t k = lk >> (3 * (depth - l));
                        double ct[3];
                        box_centre(&T, l, k, ct);
                        cplx *ph = &chain[(size_t)l * 2 * P2], *ch = ph + P2;
                        if (l > 2) {
                            double cp[3];
                            box_centre(&T, l - 1, k >> 3, cp);
                            double t[3] = {ct[0] - cp[0], ct[1] - cp[1], ct[2] - cp[2]};
                            const cplx *iph = &chain[(size_t)(l - 1) * 2 * P2];
                            lho_l2l(p, t, iph, iph + P2, ph, ch);
                        }
                        int64_t vl[189];
                        int nv = vlist(&T, l, k, vl);
                        for (int i = 0; i < nv; i++) {
                            double cs[3];
                            box_centre(&T, l, T.key[l][vl[i]], cs);
                            double t[3] = {ct[0] - cs[0], ct[1] - cs[1], ct[2] - cs[2]};
                            const cplx *iph = &M[l][(size_t)vl[i] * 2 * P2];
                            lho_m2l(p, t, iph, iph + P2, ph, ch);
                        }
                        nm2l += nv;
                    }
                    int64_t c = T.count[depth][b];
                    if (c > cap) {
                        free(bx); free(bw); free(bv); free(bs); free(bg);
                        cap = c;
                        bx = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                        bw = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                        bv = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                        bs = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                        bg = (double *)malloc(sizeof(double) * 9 * (size_t)cap);
                    }
                    box_points(&T, x, w, NULL, depth, b, bx, bw, NULL);
                    memset(bv, 0, sizeof(double) * 3 * (size_t)c);
                    memset(bs, 0, sizeof(double) * 3 * (size_t)c);
                    memset(bg, 0, sizeof(double) * 9 * (size_t)c);
                    double cen[3];
                    box_centre(&T, depth, lk, cen);
                    const cplx *ph = &chain[(size_t)depth * 2 * P2];
                    lho_l2p(p, cen, ph, ph + P2, c, bx, bw, bv, bs, bg, NULL, NULL);
                    for (int64_t i = 0; i < c; i++) {
                        int64_t e = T.order[T.first[depth][b] + i];
                        for (int d = 0; d < 3; d++) {
                            v[3 * e + d] += bv[3 * i + d];
                            s[3 * e + d] += bs[3 * i + d];
                        }
                        if (gv)
                            for (int d = 0; d < 9; d++) gv[9 * e + d] += bg[9 * i + d];
                    }
                }
                free(chain);
                free(bx); free(bw); free(bv); free(bs); free(bg);
            }
            stats.n_m2l = nm2l;
        }
        for (int l = 2; l <= depth; l++) free(M[l]);
        stats.t_down = wtime() - t1;
    }

    if (what & 2) {
        /* ---------- near field: adjacent leaves, smoothed kernel ---------- */
        double t2 = wtime();
        int64_t npairs = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : npairs)
        for (int64_t b = 0; b < nleaf; b++) {
            if (!want[b]) continue;
            int c[3];
            box_coords(T.key[depth][b], c);
            int nside = 1 << depth;
            int64_t nb_list[27];
            int nn = 0;
            for (int dz = -1; dz <= 1; dz++)
                for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                        int cc[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
                        if (cc[0] < 0 || cc[1] < 0 || cc[2] < 0 || cc[0] >= nside || cc[1] >= nside ||
                            cc[2] >= nside)
                            continue;
                        int64_t nbx = tree_find(&T, depth, morton((uint32_t)cc[0], (uint32_t)cc[1], (uint32_t)cc[2]));
                        if (nbx >= 0) nb_list[nn++] = nbx;
                    }
            for (int64_t it = 0; it < T.count[depth][b]; it++) {
                int64_t j = T.order[T.first[depth][b] + it];
                double vv[3] = {0, 0, 0}, ss[3] = {0, 0, 0}, gg[9] = {0};
                for (int u = 0; u < nn; u++) {
                    for (int64_t is = 0; is < T.count[depth][nb_list[u]]; is++) {
                        int64_t i = T.order[T.first[depth][nb_list[u]] + is];
                        if (i == j) continue;
                        pair_accum(&x[3 * j], &w[3 * j], &x[3 * i], &w[3 * i], q ? q[i] : 0.0, a, smooth, vv,
                                   ss, gv ? gg : NULL);
                        npairs++;
                    }
                }
                for (int d = 0; d < 3; d++) {
                    v[3 * j + d] += vv[d];
                    s[3 * j + d] += ss[d];
                }
                if (gv)
                    for (int d = 0; d < 9; d++) gv[9 * j + d] += gg[d];
            }
        }
        stats.n_p2p_pairs = npairs;
        stats.t_near = wtime() - t2;
    }
    if (st) *st = stats;
    free(want);
    tree_free(&T);
    return 0;
}

/* number of OpenMP threads the oracle uses */
int lho_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Tree summary for tests: per level the number of non-empty boxes, and the
 * total number of V-list pairs (M2L translations) and U-list pairs. */
int lho_tree_counts(int64_t n, const double *x, int depth, const double lo[3], double L, int64_t *nb,
                    int64_t *n_m2l, int64_t *n_p2p)
{
    otree T;
    tree_build(&T, n, x, depth, lo, L);
    int64_t tot = 0, pp = 0;
    for (int l = 0; l <= depth; l++) nb[l] = T.nb[l];
    for (int l = 2; l <= depth; l++)
        for (int64_t b = 0; b < T.nb[l]; b++) {
            int64_t vl[189];
            tot += vlist(&T, l, T.key[l][b], vl);
        }
    int nside = 1 << depth;
    for (int64_t b = 0; b < T.nb[depth]; b++) {
        int c[3];
        box_coords(T.key[depth][b], c);
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    int cc[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
                    if (cc[0] < 0 || cc[1] < 0 || cc[2] < 0 || cc[0] >= nside || cc[1] >= nside || cc[2] >= nside)
                        continue;
                    int64_t nbx = tree_find(&T, depth, morton((uint32_t)cc[0], (uint32_t)cc[1], (uint32_t)cc[2]));
                    if (nbx >= 0) pp += T.count[depth][b] * T.count[depth][nbx];
                }
    }
    *n_m2l = tot;
    *n_p2p = pp - n; /* self pairs excluded */
    tree_free(&T);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* (C) adaptive octree FMM                                                     */
/*                                                                            */
/* Tree: a box is split while it holds more than maxleaf elements, down to    */
/* level maxl.  Box (l, k) belongs to the tree iff l = 0 or its parent holds  */
/* more than maxleaf elements; it is a leaf iff it belongs and holds at most  */
/* maxleaf elements or l = maxl.  Lists after Carrier, Greengard & Rokhlin    */
/* (the adaptive scheme the paper builds on), with closed adjacency of boxes  */
/* of any sizes:                                                              */
/*   U(b), b leaf:  leaves adjacent to b (b included) -- direct, smoothed;    */
/*   V(B), level>=2: same-level boxes of the tree, not adjacent to B, whose   */
/*                   parents are adjacent -- M2L;                             */
/*   W(b), b leaf:  boxes of the tree below a colleague of b (same-level      */
/*                   adjacent box), whose parent is adjacent to b but which   */
/*                   are not -- here summed directly with the singular kernel;*/
/*   X(B):          leaves C with B in W(C) -- likewise direct, singular.     */
/* A target leaf b receives L2P of its local expansion (levels >= 2, built by */
/* L2L + M2L over V down its ancestor chain), U(b) smoothed, and W(b) plus    */
/* X(A) for every A from b up to the root, singular.                          */
/* ------------------------------------------------------------------------- */

typedef struct {
    otree T;
    int maxl;
    int64_t maxleaf;
    char *in[MAXLEV + 1];
    char *leaf[MAXLEV + 1];
} atree;

static void atree_build(atree *A, int64_t n, const double *x, int64_t maxleaf, int maxl, const double lo[3],
                        double L)
{
    tree_build(&A->T, n, x, maxl, lo, L);
    A->maxl = maxl;
    A->maxleaf = maxleaf;
    for (int l = 0; l <= maxl; l++) {
        A->in[l] = (char *)calloc((size_t)A->T.nb[l] + 1, 1);
        A->leaf[l] = (char *)calloc((size_t)A->T.nb[l] + 1, 1);
        for (int64_t b = 0; b < A->T.nb[l]; b++) {
            int in = 1;
            if (l > 0) {
                int64_t pb = tree_find(&A->T, l - 1, A->T.key[l][b] >> 3);
                in = A->in[l - 1][pb] && A->T.count[l - 1][pb] > maxleaf;
            }
            A->in[l][b] = (char)in;
            A->leaf[l][b] = (char)(in && (A->T.count[l][b] <= maxleaf || l == maxl));
        }
    }
}

static void atree_free(atree *A)
{
    for (int l = 0; l <= A->maxl; l++) {
        free(A->in[l]);
        free(A->leaf[l]);
    }
    tree_free(&A->T);
}

/* closed boxes (l1, k1) and (l2, k2) touch or overlap */
static int adjacent(int l1, uint64_t k1, int l2, uint64_t k2)
{
    int c1[3], c2[3];
    box_coords(k1, c1);
    box_coords(k2, c2);
    for (int d = 0; d < 3; d++) {
        int64_t lo1 = (int64_t)c1[d] << (QBITS - l1), hi1 = (int64_t)(c1[d] + 1) << (QBITS - l1);
        int64_t lo2 = (int64_t)c2[d] << (QBITS - l2), hi2 = (int64_t)(c2[d] + 1) << (QBITS - l2);
        if (lo1 > hi2 || lo2 > hi1) return 0;
    }
    return 1;
}

/* tree box at level l with key k, or -1 */
static int64_t atree_find(const atree *A, int l, uint64_t k)
{
    int64_t b = tree_find(&A->T, l, k);
    return (b >= 0 && A->in[l][b]) ? b : -1;
}

/* first index at level l whose key is >= k */
static int64_t lower_key(const otree *T, int l, uint64_t k)
{
    int64_t lo = 0, hi = T->nb[l];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (T->key[l][mid] < k) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

/* same-level neighbours (colleagues) of (l, k) that belong to the tree, self excluded */
static int colleagues(const atree *A, int l, uint64_t k, int64_t *out)
{
    int c[3];
    box_coords(k, c);
    int nside = 1 << l, cnt = 0;
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                if (!dx && !dy && !dz) continue;
                int cc[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
                if (cc[0] < 0 || cc[1] < 0 || cc[2] < 0 || cc[0] >= nside || cc[1] >= nside || cc[2] >= nside)
                    continue;
                int64_t b = atree_find(A, l, morton((uint32_t)cc[0], (uint32_t)cc[1], (uint32_t)cc[2]));
                if (b >= 0) out[cnt++] = b;
            }
    return cnt;
}

/* a growable list of (level, box) */
typedef struct {
    int *lev;
    int64_t *box;
    int64_t n, cap;
} blist;

static void blist_push(blist *L, int l, int64_t b)
{
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 64;
        L->lev = (int *)realloc(L->lev, sizeof(int) * (size_t)L->cap);
        L->box = (int64_t *)realloc(L->box, sizeof(int64_t) * (size_t)L->cap);
    }
    L->lev[L->n] = l;
    L->box[L->n] = b;
    L->n++;
}

static void blist_free(blist *L)
{
    free(L->lev);
    free(L->box);
}

/* U(b): leaves adjacent to leaf (lb, b) -- every leaf lies below some tree box at
 * level min(lb, its level); scan all leaves inside the 3x3x3 block around b at each level */
static void list_U(const atree *A, int lb, int64_t b, blist *out)
{
    const otree *T = &A->T;
    uint64_t kb = T->key[lb][b];
    for (int l = 0; l <= A->maxl; l++) {
        if (l <= lb) {
            /* coarser or same level: the candidate is the neighbour of b's ancestor */
            uint64_t ka = kb >> (3 * (lb - l));
            int c[3];
            box_coords(ka, c);
            int nside = 1 << l;
            for (int dz = -1; dz <= 1; dz++)
                for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                        int cc[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
                        if (cc[0] < 0 || cc[1] < 0 || cc[2] < 0 || cc[0] >= nside || cc[1] >= nside ||
                            cc[2] >= nside)
                            continue;
                        uint64_t kc = morton((uint32_t)cc[0], (uint32_t)cc[1], (uint32_t)cc[2]);
                        int64_t q = atree_find(A, l, kc);
                        if (q >= 0 && A->leaf[l][q] && adjacent(lb, kb, l, kc)) blist_push(out, l, q);
                    }
        } else {
            /* finer leaves: descendants of b's colleagues */
            int64_t col[26];
            int nc = colleagues(A, lb, kb, col);
            for (int i = 0; i < nc; i++) {
                uint64_t kc = T->key[lb][col[i]];
                int sh = 3 * (l - lb);
                for (int64_t q = lower_key(T, l, kc << sh); q < T->nb[l] && (T->key[l][q] >> sh) == kc; q++)
                    if (A->leaf[l][q] && adjacent(lb, kb, l, T->key[l][q])) blist_push(out, l, q);
            }
        }
    }
}

/* W(b): tree boxes below a colleague of leaf (lb, b), parent adjacent to b, itself not */
static void list_W(const atree *A, int lb, int64_t b, blist *out)
{
    const otree *T = &A->T;
    uint64_t kb = T->key[lb][b];
    int64_t col[26];
    int nc = colleagues(A, lb, kb, col);
    for (int i = 0; i < nc; i++) {
        uint64_t kc = T->key[lb][col[i]];
        for (int l = lb + 1; l <= A->maxl; l++) {
            int sh = 3 * (l - lb);
            for (int64_t q = lower_key(T, l, kc << sh); q < T->nb[l] && (T->key[l][q] >> sh) == kc; q++) {
                if (!A->in[l][q]) continue;
                uint64_t kq = T->key[l][q];
                if (adjacent(l - 1, kq >> 3, lb, kb) && !adjacent(l, kq, lb, kb)) blist_push(out, l, q);
            }
        }
    }
}

/* X(B) for tree box (la, a): leaves C (coarser than B) with B in W(C), i.e. C is a
 * colleague of B's ancestor at C's level, C is adjacent to B's parent, not to B */
static void list_X(const atree *A, int la, int64_t a, blist *out)
{
    const otree *T = &A->T;
    uint64_t ka = T->key[la][a];
    for (int lc = 0; lc < la; lc++) {
        uint64_t kanc = ka >> (3 * (la - lc));
        int64_t col[26];
        int nc = colleagues(A, lc, kanc, col);
        for (int i = 0; i < nc; i++) {
            if (!A->leaf[lc][col[i]]) continue;
            uint64_t kc = T->key[lc][col[i]];
            if (adjacent(la - 1, ka >> 3, lc, kc) && !adjacent(la, ka, lc, kc)) blist_push(out, lc, col[i]);
        }
    }
}

/* V(B) restricted to the tree (level >= 2) */
static int list_V(const atree *A, int l, uint64_t k, int64_t *out)
{
    int64_t tmp[189];
    int nv = vlist(&A->T, l, k, tmp), cnt = 0;
    for (int i = 0; i < nv; i++)
        if (A->in[l][tmp[i]]) out[cnt++] = tmp[i];
    return cnt;
}

/* add the direct sum over the elements of box (l, q) into target element j */
static int64_t box_direct(const atree *A, const double *x, const double *w, const double *qm, double a,
                          int smooth, int l, int64_t q, int64_t j, double *vv, double *ss, double *gg)
{
    const otree *T = &A->T;
    int64_t np = 0;
    for (int64_t is = 0; is < T->count[l][q]; is++) {
        int64_t i = T->order[T->first[l][q] + is];
        if (i == j) continue;
        pair_accum(&x[3 * j], &w[3 * j], &x[3 * i], &w[3 * i], qm ? qm[i] : 0.0, a, smooth, vv, ss, gg);
        np++;
    }
    return np;
}

/* Adaptive FMM of v and s (FP64, direct-mode translations), and of grad v
 * (row = component, column = derivative) when gv is not NULL.  what / sample as
 * in lho_fmm (sample: the leaves holding the sampled elements are evaluated).
 * maxleaf >= 0, 1 <= maxl <= 10.  Returns 0 on success. */
int lho_fmm_adaptive(int64_t n, const double *x, const double *w, const double *qm, double a, int p,
                     int64_t maxleaf, int maxl, const double lo[3], double L, int what, int64_t nsample,
                     const int64_t *sample, double *v, double *s, double *gv, int wx_mode, lho_stats *st)
{
    if (maxl < 1 || maxl > 10 || p < 1 || n < 1 || maxleaf < 0) return -1;
    double t0 = wtime();
    atree A;
    atree_build(&A, n, x, maxleaf, maxl, lo, L);
    const otree *T = &A.T;
    size_t P2 = (size_t)p * p;
    int smooth = a > 0.0;
    lho_stats stats;
    memset(&stats, 0, sizeof(stats));
    for (int l = 0; l <= maxl; l++)
        for (int64_t b = 0; b < T->nb[l]; b++) {
            stats.n_box += A.in[l][b];
            stats.n_leaf += A.leaf[l][b];
            if (A.in[l][b]) stats.max_level = l;
        }
    /* wanted leaves */
    char *want[MAXLEV + 1];
    for (int l = 0; l <= maxl; l++) {
        want[l] = (char *)calloc((size_t)T->nb[l] + 1, 1);
        for (int64_t b = 0; b < T->nb[l]; b++) want[l][b] = (char)(A.leaf[l][b] && !sample);
    }
    if (sample)
        for (int64_t i = 0; i < nsample; i++) {
            int64_t e = sample[i];
            for (int l = 0; l <= maxl; l++) {
                int sh = QBITS - l;
                int64_t b = atree_find(&A, l, morton(T->q[3 * e] >> sh, T->q[3 * e + 1] >> sh, T->q[3 * e + 2] >> sh));
                if (b >= 0 && A.leaf[l][b]) {
                    want[l][b] = 1;
                    break;
                }
            }
        }
    stats.t_tree = wtime() - t0;

    if (what & 1) {
        double t1 = wtime();
        /* upward: P2M at leaves of levels >= 2, M2M into the non-leaf boxes */
        cplx *M[MAXLEV + 1] = {0}, *Lc[MAXLEV + 1] = {0};
        for (int l = 2; l <= maxl; l++) {
            M[l] = (cplx *)calloc((size_t)T->nb[l] * 2 * P2 + 1, sizeof(cplx));
            Lc[l] = (cplx *)calloc((size_t)T->nb[l] * 2 * P2 + 1, sizeof(cplx));
        }
        for (int l = maxl; l >= 2; l--) {
#pragma omp parallel
            {
                double *bx = NULL, *bw = NULL, *bq = NULL;
                int64_t cap = 0;
#pragma omp for schedule(dynamic, 4)
                for (int64_t b = 0; b < T->nb[l]; b++) {
                    if (!A.in[l][b]) continue;
                    double cen[3];
                    box_centre(T, l, T->key[l][b], cen);
                    cplx *ph = &M[l][(size_t)b * 2 * P2], *ch = ph + P2;
                    if (A.leaf[l][b]) {
                        int64_t c = T->count[l][b];
                        if (c > cap) {
                            free(bx);
                            free(bw);
                            free(bq);
                            cap = c;
                            bx = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                            bw = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                            bq = (double *)malloc(sizeof(double) * (size_t)cap);
                        }
                        box_points(T, x, w, qm, l, b, bx, bw, bq);
                        lho_p2m_method2(p, cen, c, bx, bw, qm ? bq : NULL, ph, ch);
                    } else {
                        for (int chn = 0; chn < 8; chn++) {
                            int64_t cb = atree_find(&A, l + 1, (T->key[l][b] << 3) | (uint64_t)chn);
                            if (cb < 0) continue;
                            double cc[3];
                            box_centre(T, l + 1, T->key[l + 1][cb], cc);
                            double t[3] = {cen[0] - cc[0], cen[1] - cc[1], cen[2] - cc[2]};
                            const cplx *iph = &M[l + 1][(size_t)cb * 2 * P2];
                            lho_m2m(p, t, iph, iph + P2, ph, ch);
                        }
                    }
                }
                free(bx);
                free(bw);
                free(bq);
            }
        }
        stats.t_up = wtime() - t1;
        t1 = wtime();
        /* downward: every tree box of levels >= 2 (only the chains of wanted leaves when sampling) */
        char *need[MAXLEV + 1] = {0};
        for (int l = 2; l <= maxl; l++) {
            need[l] = (char *)calloc((size_t)T->nb[l] + 1, 1);
            for (int64_t b = 0; b < T->nb[l]; b++) need[l][b] = (char)(A.in[l][b] && !sample);
        }
        if (sample)
            for (int l = 2; l <= maxl; l++)
                for (int64_t b = 0; b < T->nb[l]; b++)
                    if (want[l][b])
                        for (int la = 2; la <= l; la++)
                            need[la][tree_find(T, la, T->key[l][b] >> (3 * (l - la)))] = 1;
        int64_t nm2l = 0;
        for (int l = 2; l <= maxl; l++) {
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : nm2l)
            for (int64_t b = 0; b < T->nb[l]; b++) {
                if (!need[l][b]) continue;
                double ct[3];
                box_centre(T, l, T->key[l][b], ct);
                cplx *ph = &Lc[l][(size_t)b * 2 * P2], *ch = ph + P2;
                if (l > 2) {
                    int64_t pb = tree_find(T, l - 1, T->key[l][b] >> 3);
                    double cp[3];
                    box_centre(T, l - 1, T->key[l - 1][pb], cp);
                    double t[3] = {ct[0] - cp[0], ct[1] - cp[1], ct[2] - cp[2]};
                    const cplx *iph = &Lc[l - 1][(size_t)pb * 2 * P2];
                    lho_l2l(p, t, iph, iph + P2, ph, ch);
                }
                int64_t vl[189];
                int nv = list_V(&A, l, T->key[l][b], vl);
                for (int i = 0; i < nv; i++) {
                    double cs[3];
                    box_centre(T, l, T->key[l][vl[i]], cs);
                    double t[3] = {ct[0] - cs[0], ct[1] - cs[1], ct[2] - cs[2]};
                    const cplx *iph = &M[l][(size_t)vl[i] * 2 * P2];
                    lho_m2l(p, t, iph, iph + P2, ph, ch);
                }
                nm2l += nv;
            }
        }
        stats.n_m2l = nm2l;
        /* wx_mode 1: the X interactions of a wanted leaf and of its ancestors at levels >= 2 enter
         * the leaf's local expansion by P2L (an ancestor's X source is at least as well separated
         * from the leaf as from the ancestor) */
        if (wx_mode)
            for (int l = 2; l <= maxl; l++) {
#pragma omp parallel for schedule(dynamic, 1)
                for (int64_t b = 0; b < T->nb[l]; b++) {
                    if (!want[l][b]) continue;
                    double ct[3];
                    box_centre(T, l, T->key[l][b], ct);
                    cplx *ph = &Lc[l][(size_t)b * 2 * P2], *ch = ph + P2;
                    blist X = {0};
                    for (int la = l; la >= 2; la--) {
                        int64_t ab = tree_find(T, la, T->key[l][b] >> (3 * (l - la)));
                        list_X(&A, la, ab, &X);
                    }
                    for (int64_t qq = 0; qq < X.n; qq++) {
                        int64_t c = T->count[X.lev[qq]][X.box[qq]];
                        double *bx = (double *)malloc(sizeof(double) * 3 * (size_t)c);
                        double *bw = (double *)malloc(sizeof(double) * 3 * (size_t)c);
                        double *bq = (double *)malloc(sizeof(double) * (size_t)c);
                        box_points(T, x, w, qm, X.lev[qq], X.box[qq], bx, bw, bq);
                        lho_p2l(p, ct, c, bx, bw, qm ? bq : NULL, ph, ch);
                        free(bx);
                        free(bw);
                        free(bq);
                    }
                    blist_free(&X);
                }
            }
        /* L2P at the wanted leaves of levels >= 2 */
        for (int l = 2; l <= maxl; l++) {
#pragma omp parallel
            {
                double *bx = NULL, *bw = NULL, *bv = NULL, *bs = NULL, *bg = NULL;
                int64_t cap = 0;
#pragma omp for schedule(dynamic, 4)
                for (int64_t b = 0; b < T->nb[l]; b++) {
                    if (!want[l][b]) continue;
                    int64_t c = T->count[l][b];
                    if (c > cap) {
                        free(bx); free(bw); free(bv); free(bs); free(bg);
                        cap = c;
                        bx = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                        bw = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                        bv = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                        bs = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                        bg = (double *)malloc(sizeof(double) * 9 * (size_t)cap);
                    }
                    box_points(T, x, w, NULL, l, b, bx, bw, NULL);
                    memset(bv, 0, sizeof(double) * 3 * (size_t)c);
                    memset(bs, 0, sizeof(double) * 3 * (size_t)c);
                    memset(bg, 0, sizeof(double) * 9 * (size_t)c);
                    double cen[3];
                    box_centre(T, l, T->key[l][b], cen);
                    const cplx *ph = &Lc[l][(size_t)b * 2 * P2];
                    lho_l2p(p, cen, ph, ph + P2, c, bx, bw, bv, bs, bg, NULL, NULL);
                    for (int64_t i = 0; i < c; i++) {
                        int64_t e = T->order[T->first[l][b] + i];
                        for (int d = 0; d < 3; d++) {
                            v[3 * e + d] += bv[3 * i + d];
                            s[3 * e + d] += bs[3 * i + d];
                        }
                        if (gv)
                            for (int d = 0; d < 9; d++) gv[9 * e + d] += bg[9 * i + d];
                    }
                }
                free(bx); free(bw); free(bv); free(bs); free(bg);
            }
        }
        /* wx_mode 1: the W boxes (levels >= 2) of a wanted leaf act by M2P of their multipoles */
        if (wx_mode)
            for (int l = 0; l <= maxl; l++) {
#pragma omp parallel for schedule(dynamic, 1)
                for (int64_t b = 0; b < T->nb[l]; b++) {
                    if (!want[l][b]) continue;
                    blist W = {0};
                    list_W(&A, l, b, &W);
                    int64_t c = T->count[l][b];
                    double *bx = (double *)malloc(sizeof(double) * 3 * (size_t)c);
                    double *bw = (double *)malloc(sizeof(double) * 3 * (size_t)c);
                    double *bv = (double *)calloc(3 * (size_t)c, sizeof(double));
                    double *bs = (double *)calloc(3 * (size_t)c, sizeof(double));
                    double *bg = (double *)calloc(9 * (size_t)c, sizeof(double));
                    box_points(T, x, w, NULL, l, b, bx, bw, NULL);
                    for (int64_t qq = 0; qq < W.n; qq++) {
                        if (W.lev[qq] < 2) continue;  /* no multipole: summed directly below */
                        double cs[3];
                        box_centre(T, W.lev[qq], T->key[W.lev[qq]][W.box[qq]], cs);
                        const cplx *mph = &M[W.lev[qq]][(size_t)W.box[qq] * 2 * P2];
                        lho_m2p(p, cs, mph, mph + P2, c, bx, bw, bv, bs, bg);
                    }
                    for (int64_t i = 0; i < c; i++) {
                        int64_t e = T->order[T->first[l][b] + i];
                        for (int d = 0; d < 3; d++) {
                            v[3 * e + d] += bv[3 * i + d];
                            s[3 * e + d] += bs[3 * i + d];
                        }
                        if (gv)
                            for (int d = 0; d < 9; d++) gv[9 * e + d] += bg[9 * i + d];
                    }
                    free(bx); free(bw); free(bv); free(bs); free(bg);
                    blist_free(&W);
                }
            }
        for (int l = 2; l <= maxl; l++) {
            free(M[l]);
            free(Lc[l]);
            free(need[l]);
        }
        stats.t_down = wtime() - t1;
    }

    if (what & 2) {
        /* near field: U smoothed, W and X (of the leaf and its ancestors) singular */
        double t2 = wtime();
        int64_t nu = 0, nwx = 0;
        for (int l = 0; l <= maxl; l++) {
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nu, nwx)
            for (int64_t b = 0; b < T->nb[l]; b++) {
                if (!want[l][b]) continue;
                blist U = {0}, WX = {0};
                list_U(&A, l, b, &U);
                {
                    blist Wb = {0};
                    list_W(&A, l, b, &Wb);
                    for (int64_t qq = 0; qq < Wb.n; qq++)  /* wx_mode 1: levels >= 2 by M2P */
                        if (!wx_mode || Wb.lev[qq] < 2) blist_push(&WX, Wb.lev[qq], Wb.box[qq]);
                    blist_free(&Wb);
                }
                for (int la = l; la >= 0; la--) {
                    if (wx_mode && l >= 2 && la >= 2) continue;  /* by P2L into the leaf's local expansion */
                    int64_t ab = tree_find(T, la, T->key[l][b] >> (3 * (l - la)));
                    list_X(&A, la, ab, &WX);
                }
                for (int64_t it = 0; it < T->count[l][b]; it++) {
                    int64_t j = T->order[T->first[l][b] + it];
                    double vv[3] = {0, 0, 0}, ss[3] = {0, 0, 0}, gg[9] = {0};
                    double *gp = gv ? gg : NULL;
                    for (int64_t q = 0; q < U.n; q++)
                        nu += box_direct(&A, x, w, qm, a, smooth, U.lev[q], U.box[q], j, vv, ss, gp);
                    for (int64_t q = 0; q < WX.n; q++)
                        nwx += box_direct(&A, x, w, qm, a, 0, WX.lev[q], WX.box[q], j, vv, ss, gp);
                    for (int d = 0; d < 3; d++) {
                        v[3 * j + d] += vv[d];
                        s[3 * j + d] += ss[d];
                    }
                    if (gv)
                        for (int d = 0; d < 9; d++) gv[9 * j + d] += gg[d];
                }
                blist_free(&U);
                blist_free(&WX);
            }
        }
        stats.n_p2p_pairs = nu;
        stats.n_wx_pairs = nwx;
        stats.t_near = wtime() - t2;
    }
    if (st) *st = stats;
    for (int l = 0; l <= maxl; l++) free(want[l]);
    atree_free(&A);
    return 0;
}

/* Direct sums with the adaptive split rule: the smoothed kernel between
 * elements of adjacent leaves of the adaptive tree, the singular one otherwise. */
void lho_direct_adaptive(int64_t n, const double *x, const double *w, const double *q, double a, int64_t maxleaf,
                         int maxl, const double lo[3], double L, int64_t ntarg, const int64_t *targ, double *v,
                         double *s)
{
    atree A;
    atree_build(&A, n, x, maxleaf, maxl, lo, L);
    const otree *T = &A.T;
    int *el = (int *)malloc(sizeof(int) * (size_t)n);
    uint64_t *ek = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    for (int64_t e = 0; e < n; e++)
        for (int l = 0; l <= maxl; l++) {
            int sh = QBITS - l;
            uint64_t k = morton(T->q[3 * e] >> sh, T->q[3 * e + 1] >> sh, T->q[3 * e + 2] >> sh);
            int64_t b = atree_find(&A, l, k);
            if (b >= 0 && A.leaf[l][b]) {
                el[e] = l;
                ek[e] = k;
                break;
            }
        }
    int smooth_ok = a > 0.0;
    int64_t nt = targ ? ntarg : n;
    /* closed integer extent [lo, hi] of every element's leaf, per dimension: two leaves are
     * adjacent iff their extents overlap in all three dimensions (the predicate of adjacent()) */
    int64_t *ext = (int64_t *)malloc(sizeof(int64_t) * 6 * (size_t)n);
    for (int64_t e = 0; e < n; e++) {
        int c[3];
        box_coords(ek[e], c);
        for (int d = 0; d < 3; d++) {
            ext[6 * e + d] = (int64_t)c[d] << (QBITS - el[e]);
            ext[6 * e + 3 + d] = (int64_t)(c[d] + 1) << (QBITS - el[e]);
        }
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t jj = 0; jj < nt; jj++) {
        int64_t j = targ ? targ[jj] : jj;
        double vv[3] = {0, 0, 0}, ss[3] = {0, 0, 0};
        const int64_t *ej = &ext[6 * j];
        for (int64_t i = 0; i < n; i++) {
            if (i == j) continue;
            const int64_t *ei = &ext[6 * i];
            int adj = !(ei[0] > ej[3] || ej[0] > ei[3] || ei[1] > ej[4] || ej[1] > ei[4] || ei[2] > ej[5] ||
                        ej[2] > ei[5]);
            int sm = smooth_ok && adj;
            pair_accum(&x[3 * j], &w[3 * j], &x[3 * i], &w[3 * i], q ? q[i] : 0.0, a, sm, vv, ss, NULL);
        }
        for (int k = 0; k < 3; k++) {
            v[3 * jj + k] = vv[k];
            s[3 * jj + k] = ss[k];
        }
    }
    free(ext);
    free(el);
    free(ek);
    atree_free(&A);
}

/* Test of the list definitions: for every ordered pair of leaves (target b,
 * source c) count the mechanisms that carry c's elements to b's -- c in U(b);
 * levels l >= 2 where c's ancestor is in V(b's ancestor); an ancestor-or-self of
 * c in W(b); c in X(an ancestor-or-self of b).  Each pair must be carried once.
 * Returns the minimum and maximum count and the number of leaves. */
void lho_adaptive_coverage(int64_t n, const double *x, int64_t maxleaf, int maxl, const double lo[3], double L,
                           int64_t *minc, int64_t *maxc, int64_t *nleaf)
{
    atree A;
    atree_build(&A, n, x, maxleaf, maxl, lo, L);
    const otree *T = &A.T;
    int64_t nl = 0;
    for (int l = 0; l <= maxl; l++)
        for (int64_t b = 0; b < T->nb[l]; b++) nl += A.leaf[l][b];
    int *ll = (int *)malloc(sizeof(int) * (size_t)nl);
    int64_t *lb = (int64_t *)malloc(sizeof(int64_t) * (size_t)nl);
    int64_t q = 0;
    for (int l = 0; l <= maxl; l++)
        for (int64_t b = 0; b < T->nb[l]; b++)
            if (A.leaf[l][b]) {
                ll[q] = l;
                lb[q++] = b;
            }
    int64_t mn = INT64_MAX, mx = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(min : mn) reduction(max : mx)
    for (int64_t i = 0; i < nl; i++) {
        int l1 = ll[i];
        uint64_t k1 = T->key[l1][lb[i]];
        blist U = {0}, W = {0}, X = {0};
        list_U(&A, l1, lb[i], &U);
        list_W(&A, l1, lb[i], &W);
        for (int la = l1; la >= 0; la--) {
            blist Xa = {0};
            list_X(&A, la, tree_find(T, la, k1 >> (3 * (l1 - la))), &Xa);
            for (int64_t t = 0; t < Xa.n; t++) blist_push(&X, Xa.lev[t], Xa.box[t]);
            blist_free(&Xa);
        }
        for (int64_t j = 0; j < nl; j++) {
            int l2 = ll[j];
            uint64_t k2 = T->key[l2][lb[j]];
            int64_t cnt = 0;
            for (int64_t t = 0; t < U.n; t++) cnt += (U.lev[t] == l2 && U.box[t] == lb[j]);
            for (int l = 2; l <= (l1 < l2 ? l1 : l2); l++) {
                uint64_t a1 = k1 >> (3 * (l1 - l)), a2 = k2 >> (3 * (l2 - l));
                if (!adjacent(l, a1, l, a2) && adjacent(l - 1, a1 >> 3, l - 1, a2 >> 3)) cnt++;
            }
            for (int64_t t = 0; t < W.n; t++)
                if (W.lev[t] <= l2 && (k2 >> (3 * (l2 - W.lev[t]))) == T->key[W.lev[t]][W.box[t]]) cnt++;
            for (int64_t t = 0; t < X.n; t++) cnt += (X.lev[t] == l2 && X.box[t] == lb[j]);
            if (cnt < mn) mn = cnt;
            if (cnt > mx) mx = cnt;
        }
        blist_free(&U);
        blist_free(&W);
        blist_free(&X);
    }
    *minc = mn;
    *maxc = mx;
    *nleaf = nl;
    free(ll);
    free(lb);
    atree_free(&A);
}

/* Adaptive tree summary: boxes and leaves per level (nb, nlf: [maxl + 1]) */
void lho_adaptive_counts(int64_t n, const double *x, int64_t maxleaf, int maxl, const double lo[3], double L,
                         int64_t *nb, int64_t *nlf)
{
    atree A;
    atree_build(&A, n, x, maxleaf, maxl, lo, L);
    for (int l = 0; l <= maxl; l++) {
        nb[l] = nlf[l] = 0;
        for (int64_t b = 0; b < A.T.nb[l]; b++) {
            nb[l] += A.in[l][b];
            nlf[l] += A.leaf[l][b];
        }
    }
    atree_free(&A);
}

/* ---------------------------------------------------------------------------------------------
 * Scalar harmonic FMM: the comparison workload of Sec. 5.2 (potential and gradient of sources in
 * a potential flow, run on the same tree at the same truncation number):
 *   Phi(y_j) = sum_{i != j} q_i / |y_j - x_i|,   grad Phi(y_j) = -sum_{i != j} q_i (y_j - x_i) / |y_j - x_i|^3
 * with the singular kernel everywhere.  The expansions carry the single potential phi:
 *   P2M   phi_n^m = sum q_i g_n^m(x_i - c), the expansion of eq. rsbf5 of each source (the monopole
 *         part of eq. eve4 with the opposite sign: there the monopole enters v with a minus);
 *   M2M, M2L, L2L by eq. mr3 on the pair (phi, chi = 0): the conversions of eqs. drt10 / drt11
 *         add chi terms only, so phi is translated as a scalar expansion and chi stays zero;
 *   L2P   Phi = sum_n sum_m phi_n^m R_n^m(y - c), grad Phi by eq. evf3 with chi = 0;
 *   near field over adjacent leaves.
 * ------------------------------------------------------------------------------------------- */

/* Direct sums of Phi and grad Phi at the targets (all elements when targets == NULL), the
 * target's own source excluded. */
void lho_scalar_direct(int64_t n, const double *x, const double *q, int64_t nt, const int64_t *targets, double *phi,
                       double *gphi)
{
    int64_t m = targets ? nt : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < m; k++) {
        int64_t j = targets ? targets[k] : k;
        double f = 0.0, g[3] = {0.0, 0.0, 0.0};
        for (int64_t i = 0; i < n; i++) {
            if (i == j) continue;
            double r[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
            double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            if (r2 == 0.0) continue;
            double ir = 1.0 / sqrt(r2), ir3 = ir * ir * ir;
            f += q[i] * ir;
            for (int d = 0; d < 3; d++) g[d] -= q[i] * r[d] * ir3;
        }
        phi[k] = f;
        for (int d = 0; d < 3; d++) gphi[3 * k + d] = g[d];
    }
}

/* Scalar FMM on the uniform octree of the given depth.  what / sample as in lho_fmm (outputs of
 * the elements of the sampled leaves, others untouched).  Returns 0 on success. */
int lho_fmm_scalar(int64_t n, const double *x, const double *q, int p, int depth, const double lo[3], double L,
                   int what, int64_t nsample, const int64_t *sample, double *phi, double *gphi, lho_stats *st)
{
    if (depth < 2 || depth > 8 || p < 1 || n < 1) return -1;
    otree T;
    tree_build(&T, n, x, depth, lo, L);
    size_t P2 = (size_t)p * p;
    lho_stats stats;
    memset(&stats, 0, sizeof(stats));
    int64_t nleaf = T.nb[depth];
    char *want = (char *)calloc((size_t)nleaf + 1, 1);
    if (!sample) {
        memset(want, 1, (size_t)nleaf);
    } else {
        int sh = QBITS - depth;
        for (int64_t i = 0; i < nsample; i++) {
            int64_t e = sample[i];
            int64_t b = tree_find(&T, depth, morton(T.q[3 * e] >> sh, T.q[3 * e + 1] >> sh, T.q[3 * e + 2] >> sh));
            if (b >= 0) want[b] = 1;
        }
    }
    if (what & 1) {
        /* upward: P2M at the leaves, M2M to level 2 (phi only; chi inputs zero, chi outputs discarded) */
        cplx *M[MAXLEV + 1], *Lc[MAXLEV + 1];
        for (int l = 2; l <= depth; l++) {
            M[l] = (cplx *)calloc((size_t)T.nb[l] * P2 + 1, sizeof(cplx));
            Lc[l] = (cplx *)calloc((size_t)T.nb[l] * P2 + 1, sizeof(cplx));
        }
        double *wzero = (double *)calloc(3 * (size_t)n, sizeof(double));
#pragma omp parallel
        {
            cplx *zero = (cplx *)calloc(P2, sizeof(cplx)), *sink = (cplx *)calloc(P2, sizeof(cplx));
            cplx *tmp = (cplx *)calloc(P2, sizeof(cplx));
            double *bx = NULL, *bw = NULL, *bq = NULL;
            int64_t cap = 0;
#pragma omp for schedule(dynamic, 4)
            for (int64_t b = 0; b < nleaf; b++) {
                int64_t c = T.count[depth][b];
                if (c > cap) {
                    free(bx);
                    free(bw);
                    free(bq);
                    cap = c;
                    bx = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                    bw = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
                    bq = (double *)malloc(sizeof(double) * (size_t)cap);
                }
                box_points(&T, x, wzero, q, depth, b, bx, bw, bq);  /* no vortex strengths */
                double cen[3];
                box_centre(&T, depth, T.key[depth][b], cen);
                memset(tmp, 0, sizeof(cplx) * P2);
                memset(sink, 0, sizeof(cplx) * P2);
                lho_p2m_method2(p, cen, c, bx, bw, bq, tmp, sink);  /* phi = -sum q g */
                cplx *ph = &M[depth][(size_t)b * P2];
                for (size_t k = 0; k < P2; k++) ph[k] = -tmp[k];
            }
            free(bx);
            free(bw);
            free(bq);
            free(zero);
            free(sink);
            free(tmp);
        }
        for (int l = depth - 1; l >= 2; l--) {
#pragma omp parallel
            {
                cplx *zero = (cplx *)calloc(P2, sizeof(cplx)), *sink = (cplx *)calloc(P2, sizeof(cplx));
#pragma omp for schedule(dynamic, 4)
                for (int64_t b = 0; b < T.nb[l]; b++) {
                    double cp[3];
                    box_centre(&T, l, T.key[l][b], cp);
                    for (int chn = 0; chn < 8; chn++) {
                        int64_t cb = tree_find(&T, l + 1, (T.key[l][b] << 3) | (uint64_t)chn);
                        if (cb < 0) continue;
                        double cc[3];
                        box_centre(&T, l + 1, T.key[l + 1][cb], cc);
                        double t[3] = {cp[0] - cc[0], cp[1] - cc[1], cp[2] - cc[2]};
                        lho_m2m(p, t, &M[l + 1][(size_t)cb * P2], zero, &M[l][(size_t)b * P2], sink);
                    }
                }
                free(zero);
                free(sink);
            }
        }
        /* downward: L2L from the parent and M2L over the V-list, every box of levels 2..depth (when
         * sampling: only the ancestor chains of the wanted leaves) */
        int64_t nm2l = 0;
        char *need[MAXLEV + 1] = {0};
        for (int l = 2; l <= depth; l++) {
            need[l] = (char *)calloc((size_t)T.nb[l] + 1, 1);
            for (int64_t b = 0; b < T.nb[l]; b++) need[l][b] = (char)!sample;
        }
        if (sample)
            for (int64_t b = 0; b < nleaf; b++)
                if (want[b])
                    for (int la = 2; la <= depth; la++)
                        need[la][tree_find(&T, la, T.key[depth][b] >> (3 * (depth - la)))] = 1;
        for (int l = 2; l <= depth; l++) {
#pragma omp parallel reduction(+ : nm2l)
            {
                cplx *zero = (cplx *)calloc(P2, sizeof(cplx)), *sink = (cplx *)calloc(P2, sizeof(cplx));
#pragma omp for schedule(dynamic, 4)
                for (int64_t b = 0; b < T.nb[l]; b++) {
                    if (!need[l][b]) continue;
                    double ct[3];
                    box_centre(&T, l, T.key[l][b], ct);
                    cplx *ph = &Lc[l][(size_t)b * P2];
                    if (l > 2) {
                        int64_t pb = tree_find(&T, l - 1, T.key[l][b] >> 3);
                        double cp[3];
                        box_centre(&T, l - 1, T.key[l - 1][pb], cp);
                        double t[3] = {ct[0] - cp[0], ct[1] - cp[1], ct[2] - cp[2]};
                        lho_l2l(p, t, &Lc[l - 1][(size_t)pb * P2], zero, ph, sink);
                    }
                    int64_t vl[189];
                    int nv = vlist(&T, l, T.key[l][b], vl);
                    for (int i = 0; i < nv; i++) {
                        double cs[3];
                        box_centre(&T, l, T.key[l][vl[i]], cs);
                        double t[3] = {ct[0] - cs[0], ct[1] - cs[1], ct[2] - cs[2]};
                        lho_m2l(p, t, &M[l][(size_t)vl[i] * P2], zero, ph, sink);
                    }
                    nm2l += nv;
                }
                free(zero);
                free(sink);
            }
        }
        stats.n_m2l = nm2l;
        /* L2P: Phi = sum phi_n^m R_n^m, grad Phi from eq. evf3 with chi = 0 */
#pragma omp parallel
        {
            cplx *zero = (cplx *)calloc(P2, sizeof(cplx)), *R = (cplx *)malloc(sizeof(cplx) * P2);
#pragma omp for schedule(dynamic, 4)
            for (int64_t b = 0; b < nleaf; b++) {
                if (!want[b]) continue;
                double cen[3];
                box_centre(&T, depth, T.key[depth][b], cen);
                const cplx *ph = &Lc[depth][(size_t)b * P2];
                for (int64_t i = 0; i < T.count[depth][b]; i++) {
                    int64_t e = T.order[T.first[depth][b] + i];
                    double r[3] = {x[3 * e] - cen[0], x[3 * e + 1] - cen[1], x[3 * e + 2] - cen[2]};
                    lho_basis_R(p, r, R);
                    cplx f = 0.0;
                    for (size_t k = 0; k < P2; k++) f += ph[k] * R[k];
                    phi[e] += creal(f);
                    double w0[3] = {0, 0, 0}, vv[3] = {0, 0, 0}, ss[3] = {0, 0, 0}, gg[9];
                    lho_l2p(p, cen, ph, zero, 1, &x[3 * e], w0, vv, ss, gg, NULL, NULL);
                    for (int d = 0; d < 3; d++) gphi[3 * e + d] += vv[d];
                }
            }
            free(zero);
            free(R);
        }
        for (int l = 2; l <= depth; l++) {
            free(M[l]);
            free(Lc[l]);
            free(need[l]);
        }
        free(wzero);
    }
    if (what & 2) {
        /* near field: adjacent leaves (incl. the own one), singular kernel */
        int64_t npairs = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : npairs)
        for (int64_t b = 0; b < nleaf; b++) {
            if (!want[b]) continue;
            int c[3];
            box_coords(T.key[depth][b], c);
            int nside = 1 << depth;
            for (int64_t it = 0; it < T.count[depth][b]; it++) {
                int64_t j = T.order[T.first[depth][b] + it];
                double f = 0.0, g[3] = {0.0, 0.0, 0.0};
                for (int dz = -1; dz <= 1; dz++)
                    for (int dy = -1; dy <= 1; dy++)
                        for (int dx = -1; dx <= 1; dx++) {
                            int cc[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
                            if (cc[0] < 0 || cc[1] < 0 || cc[2] < 0 || cc[0] >= nside || cc[1] >= nside ||
                                cc[2] >= nside)
                                continue;
                            int64_t nb = tree_find(&T, depth, morton((uint32_t)cc[0], (uint32_t)cc[1], (uint32_t)cc[2]));
                            if (nb < 0) continue;
                            for (int64_t k = 0; k < T.count[depth][nb]; k++) {
                                int64_t i = T.order[T.first[depth][nb] + k];
                                if (i == j) continue;
                                double r[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1],
                                               x[3 * j + 2] - x[3 * i + 2]};
                                double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                                if (r2 == 0.0) continue;
                                double ir = 1.0 / sqrt(r2), ir3 = ir * ir * ir;
                                f += q[i] * ir;
                                for (int d = 0; d < 3; d++) g[d] -= q[i] * r[d] * ir3;
                                npairs++;
                            }
                        }
                phi[j] += f;
                for (int d = 0; d < 3; d++) gphi[3 * j + d] += g[d];
            }
        }
        stats.n_p2p_pairs = npairs;
    }
    if (st) *st = stats;
    free(want);
    tree_free(&T);
    return 0;
}

/* ---------------------------------------------------------------------------------------------
 * Vortex filaments (Sec. 5.3, App. B): straight segments C_i from X[s0_i] to X[s1_i] with constant
 * circulation G_i; receivers are the vertices X.  With the library's convention (no 1/(4 pi), as
 * for the particles), the velocity of one segment at y not on it is eq. dis2 without its factor:
 *   v_i(y) = G_i (r1 x r2) / (r1 r2 + r1 . r2) (1/r1 + 1/r2),  r1 = y - x1, r2 = y - x2,
 * and v_i(y) = 0 for y on C_i (a vertex of the segment).  Far away a segment is the point vortex
 * of strength G_i l_i (l_i = x2 - x1) at its centre; its multipole is that of N_q Gauss-Legendre
 * points x_c + l xi_j / 2 with strengths G_i l_i w_j / 2 (eqs. vf5, vf6), exact for every order
 * n < p when N_q = floor((p - 1)/2) + 1 (eq. vf7).
 * ------------------------------------------------------------------------------------------- */

/* Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on P_nq (nq <= 64) */
void lho_gauss_legendre(int nq, double *xi, double *w)
{
    for (int i = 0; i < nq; i++) {
        double x = cos(M_PI * (i + 0.75) / (nq + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= nq; k++) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (nq == 1) {
                p1 = x;
                p0 = 1.0;
            }
            dp = nq * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= nq; k++) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (nq == 1) {
                p1 = x;
                p0 = 1.0;
            }
            dp = nq * (x * p1 - p0) / (x * x - 1.0);
        }
        xi[i] = x;
        w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

/* velocity of segment (x1, x2, G) at y (eq. dis2 without 1/(4 pi)); 0 on the segment's line */
static void seg_velocity(const double *y, const double *x1, const double *x2, double G, double *v)
{
    double r1[3] = {y[0] - x1[0], y[1] - x1[1], y[2] - x1[2]};
    double r2[3] = {y[0] - x2[0], y[1] - x2[1], y[2] - x2[2]};
    double a = sqrt(r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2]);
    double b = sqrt(r2[0] * r2[0] + r2[1] * r2[1] + r2[2] * r2[2]);
    double c[3] = {r1[1] * r2[2] - r1[2] * r2[1], r1[2] * r2[0] - r1[0] * r2[2], r1[0] * r2[1] - r1[1] * r2[0]};
    double den = a * b + r1[0] * r2[0] + r1[1] * r2[1] + r1[2] * r2[2];
    double c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    if (a == 0.0 || b == 0.0 || c2 == 0.0 || den == 0.0) return;
    double f = G * (1.0 / a + 1.0 / b) / den;
    for (int d = 0; d < 3; d++) v[d] += f * c[d];
}

/* direct sum at the vertices (all when targets == NULL): segments containing the receiver vertex
 * are skipped */
void lho_filament_direct(int64_t nv, const double *X, int64_t ns, const int32_t *seg, const double *G, int64_t nt,
                         const int64_t *targets, double *v)
{
    int64_t m = targets ? nt : nv;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < m; k++) {
        int64_t j = targets ? targets[k] : k;
        double vv[3] = {0, 0, 0};
        for (int64_t i = 0; i < ns; i++) {
            if (seg[2 * i] == j || seg[2 * i + 1] == j) continue;
            seg_velocity(&X[3 * j], &X[3 * seg[2 * i]], &X[3 * seg[2 * i + 1]], G[i], vv);
        }
        for (int d = 0; d < 3; d++) v[3 * k + d] = vv[d];
    }
}

/* FMM of the filament velocity at the vertices on the uniform octree of the given depth built on
 * the points {segment centres} U {vertices} (points 0..ns-1 the centres, ns..ns+nv-1 the
 * vertices).  nq quadrature points per segment in P2M (0: eq. vf7).  what: bit 0 far field
 * (expansions of the segments in non-adjacent boxes), bit 1 near field (eq. dis2 over the
 * segments whose centres lie in leaves adjacent to the vertex's).  Returns 0 on success. */
int lho_filament_fmm(int64_t nv, const double *X, int64_t ns, const int32_t *seg, const double *G, int p, int depth,
                     const double lo[3], double L, int nq, int what, double *v, lho_stats *st)
{
    if (depth < 2 || depth > 8 || p < 1 || nv < 1 || ns < 1) return -1;
    if (nq <= 0) nq = (p - 1) / 2 + 1;
    if (nq > 64) return -1;
    double xi[64], wq[64];
    lho_gauss_legendre(nq, xi, wq);
    int64_t n = ns + nv;
    double *pts = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *om = (double *)calloc(3 * (size_t)n, sizeof(double));
    for (int64_t i = 0; i < ns; i++)
        for (int d = 0; d < 3; d++) {
            double x1 = X[3 * seg[2 * i] + d], x2 = X[3 * seg[2 * i + 1] + d];
            pts[3 * i + d] = 0.5 * (x1 + x2);
            om[3 * i + d] = G[i] * (x2 - x1);  /* G l */
        }
    memcpy(pts + 3 * ns, X, sizeof(double) * 3 * (size_t)nv);
    otree T;
    tree_build(&T, n, pts, depth, lo, L);
    size_t P2 = (size_t)p * p;
    lho_stats stats;
    memset(&stats, 0, sizeof(stats));
    int64_t nleaf = T.nb[depth];
    memset(v, 0, sizeof(double) * 3 * (size_t)nv);
    if (what & 1) {
        cplx *M[MAXLEV + 1], *Lc[MAXLEV + 1];
        for (int l = 2; l <= depth; l++) {
            M[l] = (cplx *)calloc((size_t)T.nb[l] * 2 * P2 + 1, sizeof(cplx));
            Lc[l] = (cplx *)calloc((size_t)T.nb[l] * 2 * P2 + 1, sizeof(cplx));
        }
        /* P2M: the quadrature points of the leaf's segments (eq. vf6) */
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t b = 0; b < nleaf; b++) {
            int64_t c = T.count[depth][b];
            double *bx = (double *)malloc(sizeof(double) * 3 * (size_t)(c * nq + 1));
            double *bw = (double *)malloc(sizeof(double) * 3 * (size_t)(c * nq + 1));
            int64_t k = 0;
            for (int64_t it = 0; it < c; it++) {
                int64_t e = T.order[T.first[depth][b] + it];
                if (e >= ns) continue;  /* a vertex: no source */
                double l[3];
                for (int d = 0; d < 3; d++) l[d] = X[3 * seg[2 * e + 1] + d] - X[3 * seg[2 * e] + d];
                for (int j = 0; j < nq; j++, k++)
                    for (int d = 0; d < 3; d++) {
                        bx[3 * k + d] = pts[3 * e + d] + 0.5 * l[d] * xi[j];
                        bw[3 * k + d] = 0.5 * wq[j] * om[3 * e + d];
                    }
            }
            double cen[3];
            box_centre(&T, depth, T.key[depth][b], cen);
            cplx *ph = &M[depth][(size_t)b * 2 * P2];
            if (k > 0) lho_p2m_method2(p, cen, k, bx, bw, NULL, ph, ph + P2);
            free(bx);
            free(bw);
        }
        for (int l = depth - 1; l >= 2; l--) {
#pragma omp parallel for schedule(dynamic, 4)
            for (int64_t b = 0; b < T.nb[l]; b++) {
                double cp[3];
                box_centre(&T, l, T.key[l][b], cp);
                cplx *ph = &M[l][(size_t)b * 2 * P2];
                for (int chn = 0; chn < 8; chn++) {
                    int64_t cb = tree_find(&T, l + 1, (T.key[l][b] << 3) | (uint64_t)chn);
                    if (cb < 0) continue;
                    double cc[3];
                    box_centre(&T, l + 1, T.key[l + 1][cb], cc);
                    double t[3] = {cp[0] - cc[0], cp[1] - cc[1], cp[2] - cc[2]};
                    const cplx *iph = &M[l + 1][(size_t)cb * 2 * P2];
                    lho_m2m(p, t, iph, iph + P2, ph, ph + P2);
                }
            }
        }
        int64_t nm2l = 0;
        for (int l = 2; l <= depth; l++) {
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : nm2l)
            for (int64_t b = 0; b < T.nb[l]; b++) {
                double ct[3];
                box_centre(&T, l, T.key[l][b], ct);
                cplx *ph = &Lc[l][(size_t)b * 2 * P2];
                if (l > 2) {
                    int64_t pb = tree_find(&T, l - 1, T.key[l][b] >> 3);
                    double cp[3];
                    box_centre(&T, l - 1, T.key[l - 1][pb], cp);
                    double t[3] = {ct[0] - cp[0], ct[1] - cp[1], ct[2] - cp[2]};
                    const cplx *iph = &Lc[l - 1][(size_t)pb * 2 * P2];
                    lho_l2l(p, t, iph, iph + P2, ph, ph + P2);
                }
                int64_t vl[189];
                int nvl = vlist(&T, l, T.key[l][b], vl);
                for (int i = 0; i < nvl; i++) {
                    double cs[3];
                    box_centre(&T, l, T.key[l][vl[i]], cs);
                    double t[3] = {ct[0] - cs[0], ct[1] - cs[1], ct[2] - cs[2]};
                    const cplx *iph = &M[l][(size_t)vl[i] * 2 * P2];
                    lho_m2l(p, t, iph, iph + P2, ph, ph + P2);
                }
                nm2l += nvl;
            }
        }
        stats.n_m2l = nm2l;
        /* L2P at the vertices */
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t b = 0; b < nleaf; b++) {
            double cen[3];
            box_centre(&T, depth, T.key[depth][b], cen);
            const cplx *ph = &Lc[depth][(size_t)b * 2 * P2];
            for (int64_t it = 0; it < T.count[depth][b]; it++) {
                int64_t e = T.order[T.first[depth][b] + it];
                if (e < ns) continue;
                double w0[3] = {0, 0, 0}, vv[3] = {0, 0, 0}, ss[3] = {0, 0, 0}, gg[9];
                lho_l2p(p, cen, ph, ph + P2, 1, &pts[3 * e], w0, vv, ss, gg, NULL, NULL);
                for (int d = 0; d < 3; d++) v[3 * (e - ns) + d] += vv[d];
            }
        }
        for (int l = 2; l <= depth; l++) {
            free(M[l]);
            free(Lc[l]);
        }
    }
    if (what & 2) {
        int64_t npairs = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : npairs)
        for (int64_t b = 0; b < nleaf; b++) {
            int c[3];
            box_coords(T.key[depth][b], c);
            int nside = 1 << depth;
            for (int64_t it = 0; it < T.count[depth][b]; it++) {
                int64_t e = T.order[T.first[depth][b] + it];
                if (e < ns) continue;
                int64_t j = e - ns;
                double vv[3] = {0, 0, 0};
                for (int dz = -1; dz <= 1; dz++)
                    for (int dy = -1; dy <= 1; dy++)
                        for (int dx = -1; dx <= 1; dx++) {
                            int cc[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
                            if (cc[0] < 0 || cc[1] < 0 || cc[2] < 0 || cc[0] >= nside || cc[1] >= nside ||
                                cc[2] >= nside)
                                continue;
                            int64_t nb = tree_find(&T, depth, morton((uint32_t)cc[0], (uint32_t)cc[1], (uint32_t)cc[2]));
                            if (nb < 0) continue;
                            for (int64_t k = 0; k < T.count[depth][nb]; k++) {
                                int64_t i = T.order[T.first[depth][nb] + k];
                                if (i >= ns || seg[2 * i] == j || seg[2 * i + 1] == j) continue;
                                seg_velocity(&X[3 * j], &X[3 * seg[2 * i]], &X[3 * seg[2 * i + 1]], G[i], vv);
                                npairs++;
                            }
                        }
                for (int d = 0; d < 3; d++) v[3 * j + d] += vv[d];
            }
        }
        stats.n_p2p_pairs = npairs;
    }
    if (st) *st = stats;
    free(pts);
    free(om);
    tree_free(&T);
    return 0;
}
