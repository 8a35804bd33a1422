/*
 * Plain FP64 CPU oracle for periodic Ewald energies and single-particle move
 * deltas.  TEST INFRASTRUCTURE ONLY: it exists to check the HIP library and is
 * called from the tests, from the smoke check and from the CPU-baseline leg of
 * the benchmark.  The library never links or calls it, and it shares no code,
 * header, table or helper with the library.
 *
 * What it computes (paper Sec. 2.2, "Ewald summation"):
 *
 *   V_Ew = sum_{i<j} q_i q_j v_E(r_i - r_j) + 1/2 sum_j q_j^2 v_M          (Eq. 2)
 *
 * with the 3D pair potential v_E and Madelung term v_M of Eqs. (3)-(4) and the
 * strictly two-dimensional (z = 0) forms of Eqs. (5)-(6).  Writing alpha for
 * sqrt(gamma) and collecting terms, the energy is the sum of four parts:
 *
 *   real        sum_{i<j} q_i q_j sum_R erfc(alpha|r_ij - R|)/|r_ij - R|
 *               + 1/2 sum_i q_i^2 sum_{R != 0} erfc(alpha|R|)/|R|
 *   reciprocal  (2 pi/Omega) sum_{G != 0} exp(-G^2/4alpha^2)/G^2 |rho(G)|^2     (3D)
 *               (pi/A)       sum_{G != 0} erfc(G/2alpha)/G     |rho(G)|^2     (2D)
 *               rho(G) = sum_j q_j exp(i G.r_j)
 *   self        -(alpha/sqrt(pi)) sum_i q_i^2
 *   background  -(pi/(2 Omega alpha^2)) Q^2 (3D),  -(sqrt(pi)/(A alpha)) Q^2 (2D),
 *               Q = sum_i q_i.
 *
 * The real-space lattice sum is truncated at |r - R| < r_cut (a term is kept
 * iff the distance is strictly below r_cut); the reciprocal sum runs over all
 * nonzero G = n.B with |G| <= g_cut (inclusive, with a relative slack of 1e-12
 * on |G|^2 so that rounding cannot drop lattice points that lie exactly on the
 * cutoff sphere).  With large cutoffs this is the converged Ewald energy.
 *
 * Algorithm, deliberately plain:
 *   - images by brute force over every lattice vector in a box that contains
 *     the ball of radius r_cut around the displacement (no minimum image);
 *   - the full G set (both G and -G), exp(iG.r) by direct cos/sin of the
 *     Cartesian dot product (no separable phase tables);
 *   - libm erfc, exp, cos, sin, sqrt; OpenMP only across walkers.
 *
 * Single-particle moves (paper Sec. 2.1): particle k moves r_k -> r'.
 *   dE_real  = q_k sum_{j != k} q_j [phi(r' - r_j) - phi(r_k - r_j)]
 *   dE_recip = c sum_G f(G) [2 Re(conj(rho) delta) + |delta|^2],
 *              delta(G) = q_k (exp(iG.r') - exp(iG.r_k))
 * and an accepted move sets rho <- rho + delta, r_k <- r'.
 *
 * Long-range Jastrow value (paper Sec. 2.3, Eq. (9) written through the
 * structure factor): J = sum_{G in half set} a_{s(G)} |rho(G)|^2 where s(G) is
 * the index of the shell of equal |G| (ascending, 0-based) and a_s = 0 for
 * s >= n_jastrow.  Summed here over the full set with a factor 1/2.
 *
 * Its derivatives with respect to one particle's position (the values and
 * derivatives of the p term that Sec. 5.2 offloads; the kinetic energy of QMC
 * needs the gradient and the Laplacian, Sec. 2.1) are taken from the pair
 * form of the same J: with the plane-wave pair function
 *   P(r) = 1/2 sum_{G != 0} a_{s(G)} cos(G.r)          (Eq. (9), full set)
 * J = P(0) sum_i q_i^2 + 2 sum_{i<j} q_i q_j P(r_i - r_j), so
 *   grad_k J = 2 q_k sum_{j != k} q_j grad P(r_k - r_j),  grad P(r) = -1/2 sum_G a G sin(G.r)
 *   lap_k J  = 2 q_k sum_{j != k} q_j lap P(r_k - r_j),   lap P(r)  = -1/2 sum_G a |G|^2 cos(G.r)
 * evaluated by direct pair and G loops (no structure factor).
 *
 * Layered two-dimensional systems (2D cell, particles at heights z_i): the
 * energy is taken straight from the pair potential of Eq. (5) and the
 * Madelung term of Eq. (6) (gamma = alpha^2),
 *   E = sum_{i<j} q_i q_j v_E(r_i - r_j, z_i - z_j) + 1/2 sum_i q_i^2 v_M,
 *   v_E = (pi/A) sum_{G != 0} [e^{zG} erfc(G/2a + z a) + e^{-zG} erfc(G/2a - z a)]/G cos(G.r)
 *       + sum_R erfc(a d_R)/d_R  (d_R = sqrt(|r - R|^2 + z^2) < r_cut, R in the plane)
 *       - (2 pi/A) [z erf(z a) + exp(-a^2 z^2)/(a sqrt(pi))],
 * pair by pair over the full G set (no structure factors), reported in the
 * same four parts (the z-dependent constant as the background part).  Moves
 * are in the plane (a particle keeps its height); the delta is the change of
 * the pair sum over the moved particle's partners.
 *
 * Jastrow two-body polynomial term (paper Sec. 2.3, Eq. (8)), optional:
 *   u_c(r) = sum_{l=0}^{N_u} alpha_{c,l} r^l (r - L_u)^C   for r < L_u, else 0,
 * with a coefficient set c per spin channel (c = 0 for a pair of equal spin
 * labels, 1 for unequal labels: u differs for parallel and antiparallel
 * spins, Sec. 2.3).  Particles with a negative label (the fixed ions) take
 * no part.  U = sum_{i<j} u_c(|r_i - r_j - R|) summed by brute force over
 * every lattice vector R with |r_i - r_j - R| < L_u (with L_u no larger than
 * half the shortest lattice vector that is the nearest image alone).  U is
 * added to the Jastrow value, its move change to the Jastrow delta and
 *   grad_k U = sum_{j,R} u'(rho) (d - R)/rho,
 *   lap_k U  = sum_{j,R} [u''(rho) + (dim - 1) u'(rho)/rho],  d = r_k - r_j,
 * to the Jastrow gradient and Laplacian, with u' and u'' from the product
 * rule on the polynomial and the (r - L_u)^C factor.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define O_PI 3.14159265358979323846

typedef struct {
    int dim;                 /* 2 or 3 */
    double lat[9];           /* rows a_i; a 2D cell uses lat[0],lat[1],lat[3],lat[4] */
    double alpha, r_cut, g_cut;
    int n_jastrow;           /* number of shell coefficients (0: no Jastrow) */
    const double *jastrow_a; /* [n_jastrow] */
    int n_u;                 /* u-term coefficients per spin channel, N_u + 1 (0: no u term) */
    int u_c;                 /* the exponent C of (r - L_u) */
    double u_cut;            /* L_u */
    const double *u_alpha;   /* [2][n_u]: channel 0 equal spin labels, 1 unequal */
    const int *spin;         /* [n] per particle: spin label, negative = no u term */
    const double *z;         /* 2D: [n] heights of the particles (layered systems), or NULL (z = 0) */
} osys;

/* ---- small helpers (plain, written out) -------------------------------- */

static double cell_measure(const osys *s) {
    const double *a = s->lat;
    if (s->dim == 2) return fabs(a[0] * a[4] - a[1] * a[3]);
    return fabs(a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                a[2] * (a[3] * a[7] - a[4] * a[6]));
}

/* Reciprocal vectors b_i (rows of bm) with a_i . b_j = 2 pi delta_ij. */
static void recip_vectors(const osys *s, double bm[9]) {
    const double *a = s->lat;
    memset(bm, 0, 9 * sizeof(double));
    if (s->dim == 2) {
        double det = a[0] * a[4] - a[1] * a[3];
        /* inverse of [[a0,a1],[a3,a4]] transposed, times 2 pi */
        bm[0] = 2 * O_PI * a[4] / det;
        bm[1] = -2 * O_PI * a[3] / det;
        bm[3] = -2 * O_PI * a[1] / det;
        bm[4] = 2 * O_PI * a[0] / det;
        return;
    }
    double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                 a[2] * (a[3] * a[7] - a[4] * a[6]);
    /* b_1 = 2 pi (a_2 x a_3)/det, etc. */
    const double *a1 = a, *a2 = a + 3, *a3 = a + 6;
    double c23[3] = {a2[1] * a3[2] - a2[2] * a3[1], a2[2] * a3[0] - a2[0] * a3[2], a2[0] * a3[1] - a2[1] * a3[0]};
    double c31[3] = {a3[1] * a1[2] - a3[2] * a1[1], a3[2] * a1[0] - a3[0] * a1[2], a3[0] * a1[1] - a3[1] * a1[0]};
    double c12[3] = {a1[1] * a2[2] - a1[2] * a2[1], a1[2] * a2[0] - a1[0] * a2[2], a1[0] * a2[1] - a1[1] * a2[0]};
    for (int d = 0; d < 3; ++d) {
        bm[0 + d] = 2 * O_PI * c23[d] / det;
        bm[3 + d] = 2 * O_PI * c31[d] / det;
        bm[6 + d] = 2 * O_PI * c12[d] / det;
    }
}

static double vnorm(const double *v, int dim) {
    double t = 0;
    for (int d = 0; d < dim; ++d) t += v[d] * v[d];
    return sqrt(t);
}

/* ---- G vectors ----------------------------------------------------------- */

typedef struct {
    int n;           /* number of G (full set, G != 0) */
    double *g;       /* [n][3] Cartesian */
    double *g2;      /* [n] |G|^2 */
    int *shell;      /* [n] shell index, ascending |G| */
    int n_shells;
} gset;

static int cmp_double(const void *x, const void *y) {
    double a = *(const double *)x, b = *(const double *)y;
    return (a > b) - (a < b);
}

static void gset_build(const osys *s, gset *out) {
    double bm[9];
    recip_vectors(s, bm);
    int dim = s->dim;
    int nmax[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) /* the G ball spans |n_d| <= g_cut |a_d| / 2 pi */
        nmax[d] = (int)ceil(s->g_cut * vnorm(s->lat + 3 * d, dim) / (2 * O_PI)) + 1;
    double lim = s->g_cut * s->g_cut * (1.0 + 1e-12);
    int cap = (2 * nmax[0] + 1) * (2 * nmax[1] + 1) * (2 * nmax[2] + 1);
    out->g = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
    out->g2 = (double *)malloc(sizeof(double) * (size_t)cap);
    out->shell = (int *)malloc(sizeof(int) * (size_t)cap);
    int n = 0;
    for (int i = -nmax[0]; i <= nmax[0]; ++i)
        for (int j = -nmax[1]; j <= nmax[1]; ++j)
            for (int k = -nmax[2]; k <= nmax[2]; ++k) {
                if (i == 0 && j == 0 && k == 0) continue;
                double gv[3];
                for (int d = 0; d < 3; ++d) gv[d] = i * bm[d] + j * bm[3 + d] + k * bm[6 + d];
                double g2 = gv[0] * gv[0] + gv[1] * gv[1] + gv[2] * gv[2];
                if (g2 <= lim) {
                    memcpy(out->g + 3 * n, gv, sizeof gv);
                    out->g2[n] = g2;
                    ++n;
                }
            }
    out->n = n;
    /* shells: distinct |G|^2 values (relative tolerance 1e-9), ascending */
    double *sorted = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    memcpy(sorted, out->g2, sizeof(double) * (size_t)n);
    qsort(sorted, (size_t)n, sizeof(double), cmp_double);
    double *uniq = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int nu = 0;
    for (int i = 0; i < n; ++i)
        if (nu == 0 || sorted[i] > uniq[nu - 1] * (1.0 + 1e-9)) uniq[nu++] = sorted[i];
    for (int i = 0; i < n; ++i) {
        int sidx = 0;
        for (int u = 0; u < nu; ++u)
            if (fabs(out->g2[i] - uniq[u]) <= 1e-9 * uniq[u]) { sidx = u; break; }
        out->shell[i] = sidx;
    }
    out->n_shells = nu;
    free(sorted);
    free(uniq);
}

static void gset_free(gset *g) {
    free(g->g);
    free(g->g2);
    free(g->shell);
}

/* Reciprocal-space kernel f(G) per the full-set sum, including the prefactor:
 * 3D (2 pi/Omega) exp(-G^2/4a^2)/G^2, 2D (pi/A) erfc(G/2a)/G. */
static double recip_factor(const osys *s, double g2, double measure) {
    double a = s->alpha;
    if (s->dim == 3) return 2 * O_PI / measure * exp(-g2 / (4 * a * a)) / g2;
    double g = sqrt(g2);
    return O_PI / measure * erfc(g / (2 * a)) / g;
}

static double jastrow_coef(const osys *s, int shell) {
    if (s->n_jastrow <= 0 || shell >= s->n_jastrow) return 0.0;
    return s->jastrow_a[shell];
}

/* ---- real space ------------------------------------------------------------ */

/* sum over lattice vectors R of erfc(alpha|d - R|)/|d - R| for |d - R| < r_cut,
 * skipping R = 0 when skip_zero is set.  The box of lattice indices is chosen
 * so that it contains every R within r_cut of d. */
static double real_image_sum(const osys *s, const double *bm, const double *dv, int skip_zero) {
    int dim = s->dim;
    double rc = s->r_cut, a = s->alpha;
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) {
        /* fractional coordinate of dv along a_d is (dv . b_d)/(2 pi) */
        double f = 0;
        for (int e = 0; e < dim; ++e) f += dv[e] * bm[3 * d + e];
        f /= 2 * O_PI;
        /* |(dv - R).b_d| <= |dv - R| |b_d| < r_cut |b_d| bounds index d */
        double ext = rc * vnorm(bm + 3 * d, dim) / (2 * O_PI);
        lo[d] = (int)floor(f - ext);
        hi[d] = (int)ceil(f + ext);
    }
    double sum = 0;
    for (int i = lo[0]; i <= hi[0]; ++i)
        for (int j = lo[1]; j <= hi[1]; ++j)
            for (int k = lo[2]; k <= hi[2]; ++k) {
                if (skip_zero && i == 0 && j == 0 && k == 0) continue;
                double r[3] = {0, 0, 0};
                for (int e = 0; e < dim; ++e)
                    r[e] = dv[e] - (i * s->lat[e] + j * s->lat[3 + e] + k * s->lat[6 + e]);
                double d2 = 0;
                for (int e = 0; e < dim; ++e) d2 += r[e] * r[e];
                double dist = sqrt(d2);
                if (dist < rc) sum += erfc(a * dist) / dist;
            }
    return sum;
}

/* ---- layered 2D systems (Eq. (5) with z != 0) ------------------------------------ */

/* sum over in-plane lattice vectors R of erfc(a d)/d, d = sqrt(|dv - R|^2 + z^2) < r_cut */
static double real_image_sum_z(const osys *s, const double *bm, const double *dv, double z) {
    double rc = s->r_cut, a = s->alpha;
    int lo[2], hi[2];
    for (int d = 0; d < 2; ++d) {
        double f = (dv[0] * bm[3 * d] + dv[1] * bm[3 * d + 1]) / (2 * O_PI);
        double ext = rc * vnorm(bm + 3 * d, 2) / (2 * O_PI);
        lo[d] = (int)floor(f - ext);
        hi[d] = (int)ceil(f + ext);
    }
    double sum = 0;
    for (int i = lo[0]; i <= hi[0]; ++i)
        for (int j = lo[1]; j <= hi[1]; ++j) {
            double r0 = dv[0] - (i * s->lat[0] + j * s->lat[3]);
            double r1 = dv[1] - (i * s->lat[1] + j * s->lat[4]);
            double dist = sqrt(r0 * r0 + r1 * r1 + z * z);
            sum += dist < rc ? erfc(a * dist) / dist : 0.0;
        }
    return sum;
}

/* (pi/A) sum_{G != 0} [e^{zG} erfc(G/2a + za) + e^{-zG} erfc(G/2a - za)]/G cos(G.r) */
static double recip_pair_2d(const osys *s, const gset *g, const double *dv, double z, double area) {
    double a = s->alpha, sum = 0;
    for (int t = 0; t < g->n; ++t) {
        double gg = sqrt(g->g2[t]);
        double f = exp(z * gg) * erfc(gg / (2 * a) + z * a) + exp(-z * gg) * erfc(gg / (2 * a) - z * a);
        sum += f / gg * cos(g->g[3 * t] * dv[0] + g->g[3 * t + 1] * dv[1]);
    }
    return O_PI / area * sum;
}

/* the z-dependent constant of v_E: -(2 pi/A) [z erf(z a) + exp(-a^2 z^2)/(a sqrt(pi))] */
static double const_pair_2d(const osys *s, double z, double area) {
    double a = s->alpha;
    return -2 * O_PI / area * (z * erf(z * a) + exp(-a * a * z * z) / (a * sqrt(O_PI)));
}

/* Energy parts of a layered 2D configuration, pair by pair. */
static void energy_layered(const osys *s, int n, const double *pos, const double *q, double *parts) {
    double bm[9];
    recip_vectors(s, bm);
    double area = cell_measure(s), a = s->alpha;
    gset g;
    gset_build(s, &g);
    double e_real = 0, e_recip = 0, e_bg = 0, q2 = 0;
    for (int i = 0; i < n; ++i) {
        q2 += q[i] * q[i];
        for (int j = i + 1; j < n; ++j) {
            double dv[2] = {pos[2 * i] - pos[2 * j], pos[2 * i + 1] - pos[2 * j + 1]};
            double z = s->z[i] - s->z[j];
            double qq = q[i] * q[j];
            e_real += qq * real_image_sum_z(s, bm, dv, z);
            e_recip += qq * recip_pair_2d(s, &g, dv, z, area);
            e_bg += qq * const_pair_2d(s, z, area);
        }
    }
    /* 1/2 sum_i q_i^2 v_M: own images, the G sum at z = 0, and the constants */
    double zero[3] = {0, 0, 0};
    e_real += 0.5 * q2 * real_image_sum(s, bm, zero, 1);
    double vm_recip = 0;
    for (int t = 0; t < g.n; ++t) {
        double gg = sqrt(g.g2[t]);
        vm_recip += erfc(gg / (2 * a)) / gg;
    }
    e_recip += 0.5 * q2 * 2 * O_PI / area * vm_recip;
    e_bg += 0.5 * q2 * (-2 * sqrt(O_PI) / (area * a));
    gset_free(&g);
    parts[0] = e_real;
    parts[1] = e_recip;
    parts[2] = -a / sqrt(O_PI) * q2;
    parts[3] = e_bg;
    parts[4] = parts[0] + parts[1] + parts[2] + parts[3];
}

/* Change of the layered energy when particle k moves in its plane to rn:
 * q_k sum_{j != k} q_j [V(rn - r_j) - V(r_k - r_j)] (the constant cancels). */
static double delta_layered(const osys *s, const double *bm, const gset *g, int n, const double *pos,
                            const double *q, int k, const double *rn) {
    double area = cell_measure(s), sum = 0;
    for (int j = 0; j < n; ++j) {
        if (j == k) continue;
        double z = s->z[k] - s->z[j];
        double dn[2] = {rn[0] - pos[2 * j], rn[1] - pos[2 * j + 1]};
        double dold[2] = {pos[2 * k] - pos[2 * j], pos[2 * k + 1] - pos[2 * j + 1]};
        double vn = real_image_sum_z(s, bm, dn, z) + recip_pair_2d(s, g, dn, z, area);
        double vo = real_image_sum_z(s, bm, dold, z) + recip_pair_2d(s, g, dold, z, area);
        sum += q[j] * (vn - vo);
    }
    return q[k] * sum;
}

/* ---- Jastrow u term ------------------------------------------------------------ */

/* u_c(r), u_c'(r), u_c''(r) of Eq. (8), for 0 <= r < L_u. */
static void u_eval(const osys *s, int c, double r, double *u, double *du, double *d2u) {
    const double *a = s->u_alpha + (size_t)c * (size_t)s->n_u;
    double P = 0, dP = 0, d2P = 0; /* the polynomial sum_l alpha_l r^l and its derivatives */
    for (int l = 0; l < s->n_u; ++l) {
        P += a[l] * pow(r, l);
        if (l >= 1) dP += l * a[l] * pow(r, l - 1);
        if (l >= 2) d2P += l * (l - 1) * a[l] * pow(r, l - 2);
    }
    int C = s->u_c;
    double x = r - s->u_cut;
    double xc = pow(x, C), xc1 = pow(x, C - 1), xc2 = C >= 2 ? pow(x, C - 2) : 0.0;
    *u = P * xc;
    *du = dP * xc + C * P * xc1;
    *d2u = d2P * xc + 2.0 * C * dP * xc1 + (double)C * (C - 1) * P * xc2;
}

static int u_channel(const osys *s, int i, int j) {
    if (s->n_u <= 0 || !s->spin || s->spin[i] < 0 || s->spin[j] < 0) return -1;
    return s->spin[i] == s->spin[j] ? 0 : 1;
}

/* sum over lattice vectors R with |d - R| < L_u of u_c(|d - R|) (val), and of
 * its gradient with respect to d (grad) and Laplacian (lap); the index box is
 * chosen as in real_image_sum. */
static void u_image_sum(const osys *s, const double *bm, const double *dv, int c, double *val, double *grad,
                        double *lap) {
    int dim = s->dim;
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) {
        double f = 0;
        for (int e = 0; e < dim; ++e) f += dv[e] * bm[3 * d + e];
        f /= 2 * O_PI;
        double ext = s->u_cut * vnorm(bm + 3 * d, dim) / (2 * O_PI);
        lo[d] = (int)floor(f - ext);
        hi[d] = (int)ceil(f + ext);
    }
    double v = 0, g[3] = {0, 0, 0}, l = 0;
    for (int i = lo[0]; i <= hi[0]; ++i)
        for (int j = lo[1]; j <= hi[1]; ++j)
            for (int k = lo[2]; k <= hi[2]; ++k) {
                double r[3] = {0, 0, 0};
                for (int e = 0; e < dim; ++e)
                    r[e] = dv[e] - (i * s->lat[e] + j * s->lat[3 + e] + k * s->lat[6 + e]);
                double d2 = 0;
                for (int e = 0; e < dim; ++e) d2 += r[e] * r[e];
                double rho = sqrt(d2);
                if (rho >= s->u_cut) continue;
                double u, du, d2u;
                u_eval(s, c, rho, &u, &du, &d2u);
                v += u;
                for (int e = 0; e < dim; ++e) g[e] += du * r[e] / rho;
                l += d2u + (dim - 1) * du / rho;
            }
    if (val) *val = v;
    if (grad)
        for (int e = 0; e < dim; ++e) grad[e] = g[e];
    if (lap) *lap = l;
}

/* U = sum_{i<j} u(r_ij) over one configuration. */
static double u_total(const osys *s, const double *bm, int n, const double *pos) {
    int dim = s->dim;
    double tot = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            int c = u_channel(s, i, j);
            if (c < 0) continue;
            double dv[3] = {0, 0, 0}, v;
            for (int e = 0; e < dim; ++e) dv[e] = pos[dim * i + e] - pos[dim * j + e];
            u_image_sum(s, bm, dv, c, &v, NULL, NULL);
            tot += v;
        }
    return tot;
}

/* ---- public entry points --------------------------------------------------- */

int oracle_count_g(const osys *s, int *n_full, int *n_shells) {
    gset g;
    gset_build(s, &g);
    *n_full = g.n;
    *n_shells = g.n_shells;
    gset_free(&g);
    return 0;
}

/* Full set of G vectors: Cartesian [n][3], |G|^2, shell index.  Arrays must
 * hold oracle_count_g's n_full entries. */
int oracle_gvectors(const osys *s, double *g_out, double *g2_out, int *shell_out) {
    gset g;
    gset_build(s, &g);
    memcpy(g_out, g.g, sizeof(double) * 3 * (size_t)g.n);
    memcpy(g2_out, g.g2, sizeof(double) * (size_t)g.n);
    memcpy(shell_out, g.shell, sizeof(int) * (size_t)g.n);
    gset_free(&g);
    return 0;
}

/* rho(G) = sum_j q_j exp(i G.r_j) at caller-given Cartesian G vectors. */
int oracle_rho_at(const osys *s, int n, const double *pos, const double *q, int n_g,
                  const double *g, double *rho_re_im /* [n_g][2] */) {
    int dim = s->dim;
    for (int t = 0; t < n_g; ++t) {
        double re = 0, im = 0;
        for (int j = 0; j < n; ++j) {
            double ph = 0;
            for (int e = 0; e < dim; ++e) ph += g[3 * t + e] * pos[dim * j + e];
            re += q[j] * cos(ph);
            im += q[j] * sin(ph);
        }
        rho_re_im[2 * t] = re;
        rho_re_im[2 * t + 1] = im;
    }
    return 0;
}

/* Energy of one configuration.  parts[0..4] = real, reciprocal, self,
 * background, total; *jastrow = J (0 when no coefficients). */
int oracle_energy(const osys *s, int n, const double *pos, const double *q, double *parts,
                  double *jastrow) {
    int dim = s->dim;
    if (dim == 2 && s->z) { /* layered: no Jastrow terms */
        energy_layered(s, n, pos, q, parts);
        if (jastrow) *jastrow = 0.0;
        return 0;
    }
    double bm[9];
    recip_vectors(s, bm);
    double meas = cell_measure(s);
    /* real space: pairs plus each particle's own images */
    double e_real = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double dv[3] = {0, 0, 0};
            for (int e = 0; e < dim; ++e) dv[e] = pos[dim * i + e] - pos[dim * j + e];
            e_real += q[i] * q[j] * real_image_sum(s, bm, dv, 0);
        }
    {
        double zero[3] = {0, 0, 0};
        double self_img = real_image_sum(s, bm, zero, 1);
        double q2 = 0;
        for (int i = 0; i < n; ++i) q2 += q[i] * q[i];
        e_real += 0.5 * q2 * self_img;
    }
    /* reciprocal space, full set */
    gset g;
    gset_build(s, &g);
    double e_recip = 0, jas = 0;
    for (int t = 0; t < g.n; ++t) {
        double re = 0, im = 0;
        for (int j = 0; j < n; ++j) {
            double ph = 0;
            for (int e = 0; e < dim; ++e) ph += g.g[3 * t + e] * pos[dim * j + e];
            re += q[j] * cos(ph);
            im += q[j] * sin(ph);
        }
        double r2 = re * re + im * im;
        e_recip += recip_factor(s, g.g2[t], meas) * r2;
        jas += 0.5 * jastrow_coef(s, g.shell[t]) * r2;
    }
    gset_free(&g);
    double q2 = 0, qt = 0;
    for (int i = 0; i < n; ++i) {
        q2 += q[i] * q[i];
        qt += q[i];
    }
    double a = s->alpha;
    double e_self = -a / sqrt(O_PI) * q2;
    double e_bg = (dim == 3) ? -O_PI / (2 * meas * a * a) * qt * qt : -sqrt(O_PI) / (meas * a) * qt * qt;
    parts[0] = e_real;
    parts[1] = e_recip;
    parts[2] = e_self;
    parts[3] = e_bg;
    parts[4] = e_real + e_recip + e_self + e_bg;
    if (s->n_u > 0) jas += u_total(s, bm, n, pos);
    if (jastrow) *jastrow = jas;
    return 0;
}

/* Gradient (grad[0..dim)) and Laplacian (*lap) of J with respect to the
 * position of particle k, by the pair form above. */
int oracle_jastrow_derivs(const osys *s, int n, const double *pos, const double *q, int k, double *grad,
                          double *lap) {
    int dim = s->dim;
    double bm[9];
    recip_vectors(s, bm);
    gset g;
    gset_build(s, &g);
    double gr[3] = {0, 0, 0}, lp = 0;
    for (int j = 0; j < n; ++j) {
        if (j == k) continue;
        double d[3] = {0, 0, 0};
        for (int e = 0; e < dim; ++e) d[e] = pos[dim * k + e] - pos[dim * j + e];
        double pg[3] = {0, 0, 0}, pl = 0; /* grad P and lap P at d */
        for (int t = 0; t < g.n; ++t) {
            double a = jastrow_coef(s, g.shell[t]);
            if (a == 0.0) continue;
            double ph = 0;
            for (int e = 0; e < dim; ++e) ph += g.g[3 * t + e] * d[e];
            for (int e = 0; e < dim; ++e) pg[e] += -0.5 * a * g.g[3 * t + e] * sin(ph);
            pl += -0.5 * a * g.g2[t] * cos(ph);
        }
        for (int e = 0; e < dim; ++e) gr[e] += 2 * q[k] * q[j] * pg[e];
        lp += 2 * q[k] * q[j] * pl;
        int c = u_channel(s, k, j);
        if (c >= 0) {
            double ug[3] = {0, 0, 0}, ul = 0;
            u_image_sum(s, bm, d, c, NULL, ug, &ul);
            for (int e = 0; e < dim; ++e) gr[e] += ug[e];
            lp += ul;
        }
    }
    for (int e = 0; e < dim; ++e) grad[e] = gr[e];
    *lap = lp;
    gset_free(&g);
    return 0;
}

/* One walker: initial energy, then n_steps proposed moves of mobile particles
 * (indices k[m] < n_mobile; particles are ordered mobile first).  For each
 * move the incremental delta (and Jastrow delta) is written; accepted moves
 * update rho and the position.  Outputs: e0[0..4] parts of the initial energy,
 * delta[m], djas[m], *j0 initial Jastrow, final positions in pos_final, and,
 * when jgrad and jlap are not NULL, the gradient jgrad[m][dim] and Laplacian
 * jlap[m] of J with respect to the moved particle at the proposed
 * configuration (particle k[m] at its proposal, whether or not accepted).
 * Returns 0. */
int oracle_run(const osys *s, int n, int n_mobile, const double *pos0, const double *q,
               int n_steps, const int32_t *k, const double *new_pos, const uint8_t *accept,
               double *e0, double *j0, double *delta, double *djas, double *pos_final,
               double *jgrad, double *jlap) {
    (void)n_mobile;
    int dim = s->dim;
    double bm[9];
    recip_vectors(s, bm);
    double meas = cell_measure(s);
    double *pos = (double *)malloc(sizeof(double) * (size_t)dim * (size_t)(n > 0 ? n : 1));
    memcpy(pos, pos0, sizeof(double) * (size_t)dim * (size_t)n);
    oracle_energy(s, n, pos, q, e0, j0);
    gset g;
    gset_build(s, &g);
    double *rre = (double *)calloc((size_t)(g.n > 0 ? g.n : 1), sizeof(double));
    double *rim = (double *)calloc((size_t)(g.n > 0 ? g.n : 1), sizeof(double));
    double *fac = (double *)malloc(sizeof(double) * (size_t)(g.n > 0 ? g.n : 1));
    double *jc = (double *)malloc(sizeof(double) * (size_t)(g.n > 0 ? g.n : 1));
    for (int t = 0; t < g.n; ++t) {
        fac[t] = recip_factor(s, g.g2[t], meas);
        jc[t] = 0.5 * jastrow_coef(s, g.shell[t]);
        for (int j = 0; j < n; ++j) {
            double ph = 0;
            for (int e = 0; e < dim; ++e) ph += g.g[3 * t + e] * pos[dim * j + e];
            rre[t] += q[j] * cos(ph);
            rim[t] += q[j] * sin(ph);
        }
    }
    for (int m = 0; m < n_steps; ++m) {
        int kk = k[m];
        const double *rn = new_pos + (size_t)dim * (size_t)m;
        const double *ro = pos + dim * kk;
        if (dim == 2 && s->z) { /* layered: pair form */
            delta[m] = delta_layered(s, bm, &g, n, pos, q, kk, rn);
            djas[m] = 0.0;
            if (accept[m])
                for (int e = 0; e < dim; ++e) pos[dim * kk + e] = rn[e];
            continue;
        }
        /* real space */
        double dr = 0;
        for (int j = 0; j < n; ++j) {
            if (j == kk) continue;
            double dn[3] = {0, 0, 0}, dold[3] = {0, 0, 0};
            for (int e = 0; e < dim; ++e) {
                dn[e] = rn[e] - pos[dim * j + e];
                dold[e] = ro[e] - pos[dim * j + e];
            }
            dr += q[j] * (real_image_sum(s, bm, dn, 0) - real_image_sum(s, bm, dold, 0));
        }
        dr *= q[kk];
        /* reciprocal space */
        double drec = 0, dj = 0;
        for (int t = 0; t < g.n; ++t) {
            double pn = 0, po = 0;
            for (int e = 0; e < dim; ++e) {
                pn += g.g[3 * t + e] * rn[e];
                po += g.g[3 * t + e] * ro[e];
            }
            double dre = q[kk] * (cos(pn) - cos(po));
            double dim_ = q[kk] * (sin(pn) - sin(po));
            double tt = 2 * (rre[t] * dre + rim[t] * dim_) + dre * dre + dim_ * dim_;
            drec += fac[t] * tt;
            dj += jc[t] * tt;
        }
        /* Jastrow u term: pairs of particle k with every other labelled particle */
        for (int j = 0; j < n; ++j) {
            int c = j == kk ? -1 : u_channel(s, kk, j);
            if (c < 0) continue;
            double dn[3] = {0, 0, 0}, dold[3] = {0, 0, 0}, un, uo;
            for (int e = 0; e < dim; ++e) {
                dn[e] = rn[e] - pos[dim * j + e];
                dold[e] = ro[e] - pos[dim * j + e];
            }
            u_image_sum(s, bm, dn, c, &un, NULL, NULL);
            u_image_sum(s, bm, dold, c, &uo, NULL, NULL);
            dj += un - uo;
        }
        delta[m] = dr + drec;
        djas[m] = dj;
        if (jgrad && jlap) {
            double *prop = (double *)malloc(sizeof(double) * (size_t)dim * (size_t)n);
            memcpy(prop, pos, sizeof(double) * (size_t)dim * (size_t)n);
            for (int e = 0; e < dim; ++e) prop[dim * kk + e] = rn[e];
            oracle_jastrow_derivs(s, n, prop, q, kk, jgrad + (size_t)dim * (size_t)m, jlap + m);
            free(prop);
        }
        if (accept[m]) {
            for (int t = 0; t < g.n; ++t) {
                double pn = 0, po = 0;
                for (int e = 0; e < dim; ++e) {
                    pn += g.g[3 * t + e] * rn[e];
                    po += g.g[3 * t + e] * ro[e];
                }
                rre[t] += q[kk] * (cos(pn) - cos(po));
                rim[t] += q[kk] * (sin(pn) - sin(po));
            }
            for (int e = 0; e < dim; ++e) pos[dim * kk + e] = rn[e];
        }
    }
    if (pos_final) memcpy(pos_final, pos, sizeof(double) * (size_t)dim * (size_t)n);
    free(rre);
    free(rim);
    free(fac);
    free(jc);
    gset_free(&g);
    free(pos);
    return 0;
}

/* Many walkers of one system, OpenMP across walkers.  Arrays are packed per
 * walker: pos0 [W][n][dim], k [S][W], new_pos [S][W][dim], accept [S][W];
 * outputs e0 [W][5], j0 [W], delta [S][W], djas [S][W].  Returns the number of
 * threads used. */
int oracle_run_batch(const osys *s, int n_walkers, int n, int n_mobile, const double *pos0,
                     const double *q, int n_steps, const int32_t *k, const double *new_pos,
                     const uint8_t *accept, double *e0, double *j0, double *delta, double *djas,
                     int n_threads) {
    int dim = s->dim;
    int used = 1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
    }
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int w = 0; w < n_walkers; ++w) {
        int32_t *kw = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_steps > 0 ? n_steps : 1));
        double *nw = (double *)malloc(sizeof(double) * (size_t)dim * (size_t)(n_steps > 0 ? n_steps : 1));
        uint8_t *aw = (uint8_t *)malloc((size_t)(n_steps > 0 ? n_steps : 1));
        double *dw = (double *)malloc(sizeof(double) * (size_t)(n_steps > 0 ? n_steps : 1));
        double *jw = (double *)malloc(sizeof(double) * (size_t)(n_steps > 0 ? n_steps : 1));
        for (int m = 0; m < n_steps; ++m) {
            kw[m] = k[(size_t)m * n_walkers + w];
            aw[m] = accept[(size_t)m * n_walkers + w];
            for (int e = 0; e < dim; ++e) nw[dim * m + e] = new_pos[((size_t)m * n_walkers + w) * dim + e];
        }
        oracle_run(s, n, n_mobile, pos0 + (size_t)w * n * dim, q, n_steps, kw, nw, aw,
                   e0 + 5 * (size_t)w, j0 + w, dw, jw, NULL, NULL, NULL);
        for (int m = 0; m < n_steps; ++m) {
            delta[(size_t)m * n_walkers + w] = dw[m];
            djas[(size_t)m * n_walkers + w] = jw[m];
        }
        free(kw);
        free(nw);
        free(aw);
        free(dw);
        free(jw);
    }
    return used;
}

/* ---- blip (B-spline) orbitals (paper Sec. 2.4) ----------------------------------
 *
 * Orbitals re-represented on a periodic grid of n1 x n2 x n3 points along the
 * lattice vectors: with fractional coordinates s = r A^-1 and x_d = n_d s_d,
 *   psi_m(r) = sum_{i,j,k} a[i][j][k][m] Th(x_1 - i) Th(x_2 - j) Th(x_3 - k),
 * the sum over every grid point, each blip function taken at the periodic
 * image of its offset nearest to zero (the grid is periodic with the cell).
 * Th is the cubic B-spline blip function with Th(0) = 1:
 *   Th(x) = 1 - 3/2 x^2 + 3/4 |x|^3   (|x| <= 1),   1/4 (2 - |x|)^3   (1 < |x| < 2),
 * zero beyond (3/2 times the cardinal cubic B-spline).  The gradient and the
 * Laplacian with respect to r follow by the chain rule: d/dr_e = sum_d
 * Ainv[e][d] n_d d/dx_d, and the Laplacian takes the full second-derivative
 * matrix in x (the cell need not be orthogonal). */

static double blip_th(double x, int der) {
    double ax = fabs(x), sg = x < 0 ? -1.0 : 1.0;
    if (ax >= 2.0) return 0.0;
    if (ax <= 1.0) {
        if (der == 0) return 1.0 - 1.5 * x * x + 0.75 * ax * ax * ax;
        if (der == 1) return -3.0 * x + 2.25 * sg * x * x;
        return -3.0 + 4.5 * ax;
    }
    double t = 2.0 - ax;
    if (der == 0) return 0.25 * t * t * t;
    if (der == 1) return -0.75 * sg * t * t;
    return 1.5 * t;
}

/* Values val[p][m], gradients grad[p][3][m] and Laplacians lap[p][m] (either
 * of the last two may be NULL) of n_orb orbitals at n_pts Cartesian points
 * pos[p][3], for coefficients coef[n1][n2][n3][n_orb]; lat holds the rows a_i. */
int oracle_blip_eval(const double *lat, int n1, int n2, int n3, int n_orb, const double *coef, int n_pts,
                     const double *pos, double *val, double *grad, double *lap) {
    osys tmp;
    memset(&tmp, 0, sizeof tmp);
    tmp.dim = 3;
    memcpy(tmp.lat, lat, sizeof tmp.lat);
    double bm[9];
    recip_vectors(&tmp, bm);
    /* Ainv[e][d] = bm[d][e] / 2 pi */
    double ainv[9];
    for (int e = 0; e < 3; ++e)
        for (int d = 0; d < 3; ++d) ainv[3 * e + d] = bm[3 * d + e] / (2 * O_PI);
    int nn[3] = {n1, n2, n3};
    /* J[e][d] = d x_d / d r_e */
    double J[9];
    for (int e = 0; e < 3; ++e)
        for (int d = 0; d < 3; ++d) J[3 * e + d] = ainv[3 * e + d] * nn[d];
    for (int p = 0; p < n_pts; ++p) {
        double x[3];
        for (int d = 0; d < 3; ++d) {
            double s = 0;
            for (int e = 0; e < 3; ++e) s += pos[3 * p + e] * ainv[3 * e + d];
            x[d] = nn[d] * s;
        }
        double *v = val + (size_t)p * n_orb;
        double *g = grad ? grad + (size_t)p * 3 * n_orb : NULL;
        double *l = lap ? lap + (size_t)p * n_orb : NULL;
        for (int m = 0; m < n_orb; ++m) {
            v[m] = 0;
            if (g) g[m] = g[n_orb + m] = g[2 * n_orb + m] = 0;
            if (l) l[m] = 0;
        }
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n2; ++j)
                for (int k = 0; k < n3; ++k) {
                    int idx[3] = {i, j, k};
                    double off[3], th[3][3];
                    int inside = 1;
                    for (int d = 0; d < 3; ++d) {
                        off[d] = x[d] - idx[d];
                        off[d] -= nn[d] * floor(off[d] / nn[d] + 0.5); /* nearest periodic image */
                        if (fabs(off[d]) >= 2.0) inside = 0;
                        for (int q = 0; q < 3; ++q) th[d][q] = blip_th(off[d], q);
                    }
                    if (!inside) continue;
                    double b = th[0][0] * th[1][0] * th[2][0];
                    /* derivatives of the product in x */
                    double dx[3] = {th[0][1] * th[1][0] * th[2][0], th[0][0] * th[1][1] * th[2][0],
                                    th[0][0] * th[1][0] * th[2][1]};
                    double hx[9];
                    for (int d = 0; d < 3; ++d)
                        for (int d2 = 0; d2 < 3; ++d2) {
                            double prod = 1;
                            for (int c = 0; c < 3; ++c) {
                                int order = (c == d) + (c == d2);
                                prod *= th[c][order];
                            }
                            hx[3 * d + d2] = prod;
                        }
                    double gr[3] = {0, 0, 0}, lp = 0;
                    for (int e = 0; e < 3; ++e) {
                        for (int d = 0; d < 3; ++d) gr[e] += J[3 * e + d] * dx[d];
                        for (int d = 0; d < 3; ++d)
                            for (int d2 = 0; d2 < 3; ++d2) lp += J[3 * e + d] * J[3 * e + d2] * hx[3 * d + d2];
                    }
                    const double *a = coef + (((size_t)i * n2 + j) * n3 + k) * (size_t)n_orb;
                    for (int m = 0; m < n_orb; ++m) {
                        v[m] += a[m] * b;
                        if (g)
                            for (int e = 0; e < 3; ++e) g[e * n_orb + m] += a[m] * gr[e];
                        if (l) l[m] += a[m] * lp;
                    }
                }
    }
    return 0;
}
