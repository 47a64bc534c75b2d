/*
 * tlsph_oracle.c -- plain FP64 CPU oracle for one Total-Lagrangian SPH
 * timestep with ductile damage (de Vaucorbeil & Hutchinson,
 * arXiv:1901.07374).
 *
 * TEST INFRASTRUCTURE ONLY: the reference that the GPU library is checked
 * against.  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load it.  It shares no source with the GPU library.
 *
 * Written for a reader holding the paper: every function names the section,
 * equation or algorithm it follows, in the paper's order and notation, with
 * no blocking, fusion or reordering beyond what the equations state.  Pair
 * sums run over each neighbour list in ascending index order, and every
 * OpenMP loop writes only its own particle, so results do not depend on the
 * thread count.  Build with -ffp-contract=off (no fused multiply-adds).
 *
 * Where the paper is silent or ambiguous, the reading taken is stated at the
 * point of use ("Reading: ...").
 *
 * Parity unpinned: the hourglass control term (the paper cites a scheme
 * without printing its formula) is pinned only by invariants -- zero for
 * affine motion and rigid rotation, antisymmetric, restoring -- not by a
 * value from the paper.  The same holds for the follow-on pieces the paper
 * names without formulas (the velocity damping, the penalty contact): their
 * pins are invariants and closed forms of the forms read, not the paper's
 * numbers.
 */
#include "tlsph_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Small 3x3 helpers (row-major A[3a+b])                                     */
/* ------------------------------------------------------------------------ */
static double det3(const double a[9]) {
    return a[0] * (a[4] * a[8] - a[5] * a[7])
         - a[1] * (a[3] * a[8] - a[5] * a[6])
         + a[2] * (a[3] * a[7] - a[4] * a[6]);
}

/* inverse by adjugate / determinant; returns the determinant */
static double inv3(const double a[9], double out[9]) {
    double d = det3(a);
    out[0] = (a[4] * a[8] - a[5] * a[7]) / d;
    out[1] = (a[2] * a[7] - a[1] * a[8]) / d;
    out[2] = (a[1] * a[5] - a[2] * a[4]) / d;
    out[3] = (a[5] * a[6] - a[3] * a[8]) / d;
    out[4] = (a[0] * a[8] - a[2] * a[6]) / d;
    out[5] = (a[2] * a[3] - a[0] * a[5]) / d;
    out[6] = (a[3] * a[7] - a[4] * a[6]) / d;
    out[7] = (a[1] * a[6] - a[0] * a[7]) / d;
    out[8] = (a[0] * a[4] - a[1] * a[3]) / d;
    return d;
}

static void mul3(const double a[9], const double b[9], double out[9]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += a[3 * i + k] * b[3 * k + j];
            out[3 * i + j] = s;
        }
}

static void transpose3(const double a[9], double out[9]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) out[3 * j + i] = a[3 * i + j];
}

/* Voigt (xx, yy, zz, yz, xz, xy) <-> full symmetric tensor */
static void voigt_to_full(const double s[6], double a[9]) {
    a[0] = s[0]; a[4] = s[1]; a[8] = s[2];
    a[5] = a[7] = s[3];
    a[2] = a[6] = s[4];
    a[1] = a[3] = s[5];
}

static void full_to_voigt(const double a[9], double s[6]) {
    s[0] = a[0]; s[1] = a[4]; s[2] = a[8];
    s[3] = 0.5 * (a[5] + a[7]);
    s[4] = 0.5 * (a[2] + a[6]);
    s[5] = 0.5 * (a[1] + a[3]);
}

static double ddot3(const double a[9], const double b[9]) {
    double s = 0.0;
    for (int k = 0; k < 9; ++k) s += a[k] * b[k];
    return s;
}

/* von Mises equivalent of a deviator: sqrt(3/2 s:s) */
static double von_mises(const double sd[9]) { return sqrt(1.5 * ddot3(sd, sd)); }

/* ------------------------------------------------------------------------ */
/* Sec. 2.2: kernel.  Reading: the paper names no kernel; the cubic spline   */
/* with compact support of radius h (q = r/h) is used, normalised to 1 in 3D */
/* (condition of unit integral), W = 0 for r >= h.                           */
/* ------------------------------------------------------------------------ */
void orc_kernel(double r, double h, double *W, double *dWdr) {
    double q = r / h;
    double c = 8.0 / (M_PI * h * h * h);
    if (q < 0.5) {
        *W = c * (1.0 - 6.0 * q * q + 6.0 * q * q * q);
        *dWdr = c / h * (-12.0 * q + 18.0 * q * q);
    } else if (q < 1.0) {
        double a = 1.0 - q;
        *W = c * 2.0 * a * a * a;
        *dWdr = c / h * (-6.0 * a * a);
    } else {
        *W = 0.0;
        *dWdr = 0.0;
    }
}

/* Kernel gradient of eq. SPH_gradient_kernel: dW/dr (X_j - X_i) / |X_j - X_i| */
static void kernel_gradient(const double Xij[3], double h, double gradW[3], double *W) {
    double r = sqrt(Xij[0] * Xij[0] + Xij[1] * Xij[1] + Xij[2] * Xij[2]);
    double w, dw;
    orc_kernel(r, h, &w, &dw);
    for (int a = 0; a < 3; ++a) gradW[a] = dw * Xij[a] / r;
    if (W) *W = w;
}

/* ------------------------------------------------------------------------ */
/* Sec. 2 / Sec. 7: the neighbour set S_i is fixed in the reference          */
/* configuration for the whole run.  Reading: S_i = {j != i in the same      */
/* specimen with |X_j - X_i| < h}; r = h is excluded (W and W' vanish there).*/
/* Graded spacing (the paper's finest specimens refine towards the notch):  */
/* reading, each particle has its own support h_i = k V_i^(1/3) and a pair   */
/* uses h_ij = (h_i + h_j) / 2 for membership and for its kernel, so S_i is   */
/* symmetric and gradW_ji = -gradW_ij.                                      */
/* A uniform cell grid of edge max h per specimen finds the candidates.      */
/* ------------------------------------------------------------------------ */
void orc_support_radii(int64_t n, const double *V0, const int32_t *spec,
                       const orc_material *mat, double *hs) {
    for (int64_t i = 0; i < n; ++i) {
        const orc_material *m = &mat[spec[i]];
        hs[i] = m->h_per_spacing > 0.0 ? m->h_per_spacing * cbrt(V0[i]) : m->h;
    }
}

/* support radius of the pair (i, j) */
static double pair_h(const orc_problem *p, int64_t i, int64_t j) {
    return p->hs ? 0.5 * (p->hs[i] + p->hs[j]) : p->mat[p->spec[i]].h;
}
static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

typedef struct {
    double lo[3];
    int64_t dim[3];
    int64_t *start;   /* [ncell+1] */
    int32_t *items;   /* particle indices grouped by cell */
} cell_grid;

static int64_t cell_of(const cell_grid *g, const double x[3], double h, int64_t c[3]) {
    for (int a = 0; a < 3; ++a) {
        int64_t k = (int64_t)floor((x[a] - g->lo[a]) / h);
        if (k < 0) k = 0;
        if (k >= g->dim[a]) k = g->dim[a] - 1;
        c[a] = k;
    }
    return c[0] + g->dim[0] * (c[1] + g->dim[1] * c[2]);
}

static int64_t neighbours_of(int64_t i, const double *X, const cell_grid *g, double h,
                             const double *hs, int32_t *buf) {
    int64_t c[3];
    cell_of(g, &X[3 * i], h, c);
    int64_t k = 0;
    double h2 = h * h;
    for (int64_t dz = -1; dz <= 1; ++dz)
        for (int64_t dy = -1; dy <= 1; ++dy)
            for (int64_t dx = -1; dx <= 1; ++dx) {
                int64_t cx = c[0] + dx, cy = c[1] + dy, cz = c[2] + dz;
                if (cx < 0 || cy < 0 || cz < 0 || cx >= g->dim[0] || cy >= g->dim[1] ||
                    cz >= g->dim[2])
                    continue;
                int64_t id = cx + g->dim[0] * (cy + g->dim[1] * cz);
                for (int64_t t = g->start[id]; t < g->start[id + 1]; ++t) {
                    int32_t j = g->items[t];
                    if (j == i) continue;
                    double d0 = X[3 * j + 0] - X[3 * i + 0];
                    double d1 = X[3 * j + 1] - X[3 * i + 1];
                    double d2 = X[3 * j + 2] - X[3 * i + 2];
                    double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                    double lim = h2;
                    if (hs) {
                        double hij = 0.5 * (hs[i] + hs[j]);
                        lim = hij * hij;
                    }
                    if (r2 < lim) {
                        if (buf) buf[k] = j;
                        ++k;
                    }
                }
            }
    if (buf) qsort(buf, (size_t)k, sizeof(int32_t), cmp_i32);
    return k;
}

int64_t orc_build_neighbors(int64_t n, const double *X, const int32_t *spec,
                            const orc_material *mat, const double *hs, int64_t *row_ptr,
                            int32_t *col, int64_t cap) {
    int32_t n_spec = 0;
    for (int64_t i = 0; i < n; ++i)
        if (spec[i] + 1 > n_spec) n_spec = spec[i] + 1;
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    cell_grid *grids = (cell_grid *)calloc((size_t)(n_spec > 0 ? n_spec : 1), sizeof(cell_grid));
    double *edge = (double *)calloc((size_t)(n_spec > 0 ? n_spec : 1), sizeof(double));
    /* one grid per specimen, cells of edge max h_i */
    for (int32_t s = 0; s < n_spec; ++s) {
        cell_grid *g = &grids[s];
        double h = mat[s].h;
        if (hs) {
            h = 0.0;
            for (int64_t i = 0; i < n; ++i)
                if (spec[i] == s && hs[i] > h) h = hs[i];
        }
        edge[s] = h;
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        int64_t ns = 0;
        for (int64_t i = 0; i < n; ++i) {
            if (spec[i] != s) continue;
            ++ns;
            for (int a = 0; a < 3; ++a) {
                if (X[3 * i + a] < lo[a]) lo[a] = X[3 * i + a];
                if (X[3 * i + a] > hi[a]) hi[a] = X[3 * i + a];
            }
        }
        if (ns == 0) continue;
        int64_t ncell = 1;
        for (int a = 0; a < 3; ++a) {
            g->lo[a] = lo[a];
            g->dim[a] = (int64_t)floor((hi[a] - lo[a]) / h) + 1;
            ncell *= g->dim[a];
        }
        g->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
        g->items = (int32_t *)malloc((size_t)ns * sizeof(int32_t));
        int64_t c[3];
        for (int64_t i = 0; i < n; ++i)
            if (spec[i] == s) g->start[cell_of(g, &X[3 * i], h, c) + 1] += 1;
        for (int64_t k = 0; k < ncell; ++k) g->start[k + 1] += g->start[k];
        int64_t *fill = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
        memcpy(fill, g->start, (size_t)ncell * sizeof(int64_t));
        for (int64_t i = 0; i < n; ++i)
            if (spec[i] == s) g->items[fill[cell_of(g, &X[3 * i], h, c)]++] = (int32_t)i;
        free(fill);
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        cnt[i] = neighbours_of(i, X, &grids[spec[i]], edge[spec[i]], hs, NULL);
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[i];
    int64_t nnz = row_ptr[n];
    if (nnz <= cap && col) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            neighbours_of(i, X, &grids[spec[i]], edge[spec[i]], hs, &col[row_ptr[i]]);
    }
    for (int32_t s = 0; s < n_spec; ++s) {
        free(grids[s].start);
        free(grids[s].items);
    }
    free(grids);
    free(edge);
    free(cnt);
    return nnz;
}

/* ------------------------------------------------------------------------ */
/* Eq. correction_matrix: L_i = sum_j V_j (X_j - X_i) (x) gradW_i(X_ij),    */
/* over the fixed support (Reading: the same-side support of Sec. 3 is the   */
/* fixed reference list; cracks act only through the (1 - D) weights).      */
/* Inverse by adjugate; singular when |det L| <= 1e-12 |L|_F^3.             */
/* ------------------------------------------------------------------------ */
int64_t orc_shape_matrices(const orc_problem *p, double *L, double *Linv) {
    int64_t bad = -1;
    for (int64_t i = 0; i < p->n; ++i) {
        double Li[9] = {0};
        for (int64_t t = p->row_ptr[i]; t < p->row_ptr[i + 1]; ++t) {
            int32_t j = p->col[t];
            double Xij[3], g[3];
            for (int a = 0; a < 3; ++a) Xij[a] = p->X[3 * j + a] - p->X[3 * i + a];
            kernel_gradient(Xij, pair_h(p, i, j), g, NULL);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Li[3 * a + b] += p->V0[j] * Xij[a] * g[b];
        }
        double nrm = sqrt(ddot3(Li, Li));
        double d = det3(Li);
        if (L) memcpy(&L[9 * i], Li, sizeof Li);
        if (!(fabs(d) > 1e-12 * nrm * nrm * nrm)) {
            if (bad < 0) bad = i;
            memset(&Linv[9 * i], 0, 9 * sizeof(double));
            continue;
        }
        inv3(Li, &Linv[9 * i]);
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Sec. 5.4, eq. void_fraction_function.  Reading: f >= f_F gives           */
/* f* = 1/q1 (failed).                                                      */
/* ------------------------------------------------------------------------ */
double orc_fstar(const orc_material *m, double f) {
    if (f <= m->fc) return f;
    if (f < m->fF) return m->fc + (1.0 / m->q1 - m->fc) / (m->fF - m->fc) * (f - m->fc);
    return 1.0 / m->q1;
}

/* D = q1 f* (Sec. 5.4), exactly 1 once f reaches f_F */
static double gtn_damage(const orc_material *m, double f) {
    if (f >= m->fF) return 1.0;
    double D = m->q1 * orc_fstar(m, f);
    return D < 1.0 ? D : 1.0;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4, eq. pH (Mie-Grueneisen).  Returns the mean stress sigma_m of     */
/* sigma = sigma_m I + sigma_d (tension positive).                           */
/* Readings: the printed formula is the pressure p (compression positive),  */
/* so sigma_m = -p; eta = rho/rho0 = 1/J (eq. conservation1); the damaged   */
/* branch applies in tension, decided on the undamaged value, with the      */
/* prefactor rho0 (1 - D) and eta = (1 - D)/J as printed; the energy term is */
/* Gamma0 rho0 e for e per unit mass (Gamma0 = 0 in every workload).        */
/* ------------------------------------------------------------------------ */
static double mie_gruneisen(double pref, double c0, double S, double G0, double eta) {
    double mu = eta - 1.0;
    double den = eta - S * mu;
    return pref * c0 * c0 * mu * (eta - 0.5 * G0 * mu) / (den * den);
}

double orc_mean_stress_eos(const orc_material *m, double J, double D, double e,
                           int32_t damaged_branch_allowed) {
    double eta = 1.0 / J;
    double p = mie_gruneisen(m->rho0, m->c0, m->S_alpha, m->Gamma0, eta)
             + m->Gamma0 * m->rho0 * e;
    if (damaged_branch_allowed && p < 0.0) {
        double eta_d = (1.0 - D) / J;
        p = mie_gruneisen(m->rho0 * (1.0 - D), m->c0, m->S_alpha, m->Gamma0, eta_d)
          + m->Gamma0 * m->rho0 * e;
    }
    return -p;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4, eq. JC_viscoplastic_model without the (1 - D) factor, and the    */
/* other hardening laws Sec. 4 names (forms in the header, readings).       */
/* Readings: the homologous temperature T* is a constant of the specimen   */
/* (0 by default: isothermal) and its factor 1 - T*^m multiplies every law; */
/* reference rate eps_dot0 is a parameter; ln of the normalised rate is     */
/* floored at 0; the rate factor multiplies every law (C = 0: rate         */
/* independent).                                                            */
/* ------------------------------------------------------------------------ */
static double thermal_factor(const orc_material *m) {
    return m->T_star > 0.0 ? 1.0 - pow(m->T_star, m->m) : 1.0;
}

static double hardening_law(const orc_material *m, double eps) {
    switch (m->flow) {
    case ORC_FLOW_LINEAR: return m->A + m->B * eps;
    case ORC_FLOW_SWIFT: return m->B * pow(m->flow_e0 + eps, m->n);
    case ORC_FLOW_VOCE: return m->A - m->B * expm1(-m->flow_beta * eps);
    default: return m->A + m->B * pow(eps, m->n);
    }
}

static double hardening(const orc_material *m, double eps) {
    return thermal_factor(m) * hardening_law(m, eps);
}

/* dh/deps.  Reading: the Johnson-Cook slope is taken as 0 at eps = 0,      */
/* where it is unbounded for n < 1.                                         */
static double hardening_slope_law(const orc_material *m, double eps) {
    switch (m->flow) {
    case ORC_FLOW_LINEAR: return m->B;
    case ORC_FLOW_SWIFT: return m->B * m->n * pow(m->flow_e0 + eps, m->n - 1.0);
    case ORC_FLOW_VOCE: return m->B * m->flow_beta * exp(-m->flow_beta * eps);
    default: return eps > 0.0 ? m->B * m->n * pow(eps, m->n - 1.0) : 0.0;
    }
}

static double hardening_slope(const orc_material *m, double eps) {
    return thermal_factor(m) * hardening_slope_law(m, eps);
}

static double rate_factor(const orc_material *m, double eps_rate) {
    double rs = eps_rate / m->eps_dot0;
    if (rs < 1.0) rs = 1.0;
    return 1.0 + m->C * log(rs);
}

double orc_flow_stress(const orc_material *m, double eps, double eps_rate) {
    return hardening(m, eps) * rate_factor(m, eps_rate);
}

/* d sigma_f / d eps at a fixed rate */
static double flow_stress_slope(const orc_material *m, double eps, double eps_rate) {
    return hardening_slope(m, eps) * rate_factor(m, eps_rate);
}

/* ------------------------------------------------------------------------ */
/* Sec. 5.1: maximum principal stress, by cyclic Jacobi rotations.          */
/* ------------------------------------------------------------------------ */
double orc_principal_max(const double sig[6]) {
    double a[9];
    voigt_to_full(sig, a);
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = a[1] * a[1] + a[2] * a[2] + a[5] * a[5];
        double diag = a[0] * a[0] + a[4] * a[4] + a[8] * a[8];
        if (off <= 1e-36 * diag || off == 0.0) break;
        static const int P[3] = {0, 0, 1}, Qi[3] = {1, 2, 2};
        for (int r = 0; r < 3; ++r) {
            int p = P[r], q = Qi[r];
            double apq = a[3 * p + q];
            if (apq == 0.0) continue;
            double theta = (a[3 * q + q] - a[3 * p + p]) / (2.0 * apq);
            double t = (fabs(theta) > 1e150)
                           ? 0.5 / theta
                           : (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
            /* rotation J with J_pp = J_qq = c, J_pq = s, J_qp = -s: a <- J^T a J */
            double Jm[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, JT[9], tmp[9];
            Jm[3 * p + p] = c; Jm[3 * q + q] = c;
            Jm[3 * p + q] = s; Jm[3 * q + p] = -s;
            transpose3(Jm, JT);
            mul3(JT, a, tmp);
            mul3(tmp, Jm, a);
            a[3 * p + q] = a[3 * q + p] = 0.0;
        }
    }
    double mx = a[0];
    if (a[4] > mx) mx = a[4];
    if (a[8] > mx) mx = a[8];
    return mx;
}

/* Sec. 5.4, eq. omega: 1 - (27 det(sigma_d) / (2 sigma_eq^3))^2, kept in  */
/* [0, 1] as the text states.                                               */
double orc_omega(const double sig[6]) {
    double a[9];
    voigt_to_full(sig, a);
    double sm = (a[0] + a[4] + a[8]) / 3.0;
    a[0] -= sm; a[4] -= sm; a[8] -= sm;
    double seq = von_mises(a);
    if (!(seq > 0.0)) return 0.0;
    double xi = 27.0 * det3(a) / (2.0 * seq * seq * seq);
    double w = 1.0 - xi * xi;
    if (w < 0.0) w = 0.0;
    if (w > 1.0) w = 1.0;
    return w;
}

/* ------------------------------------------------------------------------ */
/* Objective rotation of the stored deviator.  Reading (the paper does not  */
/* state its stress rate): Hughes-Winget increment                           */
/* R = (I - dt/2 w)^-1 (I + dt/2 w), sd <- R sd R^T.                          */
/* ------------------------------------------------------------------------ */
void orc_hughes_winget(double dt, const double w[9], const double sd_in[9],
                       double sd_out[9]) {
    double Am[9], Bm[9], Ai[9], R[9], RT[9], tmp[9];
    for (int k = 0; k < 9; ++k) {
        double id = (k % 4 == 0) ? 1.0 : 0.0;
        Am[k] = id - 0.5 * dt * w[k];
        Bm[k] = id + 0.5 * dt * w[k];
    }
    inv3(Am, Ai);
    mul3(Ai, Bm, R);
    transpose3(R, RT);
    mul3(R, sd_in, tmp);
    mul3(tmp, RT, sd_out);
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 (Sec. 4): explicit radial return with Johnson-Cook flow.     */
/* Readings: sigma_y of the plastic-strain line is the damaged flow stress  */
/* sigma_f(eps_n, rate_n)(1 - D) of the yield test (explicit hardening);    */
/* the increment is divided by 3G(1 - D), matching the 2G(1 - D) trial.     */
/*                                                                          */
/* Implicit variant (m->implicit_return): the increment d solves the        */
/* consistency condition with the flow stress at the end of the step,       */
/*   sigma_eq,tr - 3G(1 - D) d = (1 - D) sigma_f(eps_n + d, d / dt),         */
/* yielding if sigma_eq,tr >= (1 - D) sigma_f(eps_n, 0).  The left side     */
/* falls and the right side rises with d, so the root is unique in          */
/* [0, (sigma_eq,tr - (1 - D) sigma_f(eps_n, 0)) / (3G(1 - D))]; it is found  */
/* by Newton steps kept inside a shrinking bracket (bisection when a step   */
/* leaves it), to a step of 1e-14 relative to d or to the increment        */
/* sigma_eq,tr / (3G(1 - D)) that would unload the trial stress, at most    */
/* 100 iterations.                                                          */
/* ------------------------------------------------------------------------ */
static double implicit_increment(const orc_material *m, double k3, double omD, double seq_tr,
                                 double eps_p, double dt, double d_max, int32_t *failed) {
    double lo = 0.0, hi = d_max, d = d_max;
    for (int it = 0; it < 100; ++it) {
        double rate = d / dt;
        double h = hardening(m, eps_p + d), rf = rate_factor(m, rate);
        double g = seq_tr - k3 * d - omD * h * rf;
        if (g > 0.0) lo = d; else hi = d;
        /* d/dd of the rate factor: C / d above the reference rate */
        double drf = rate / m->eps_dot0 > 1.0 ? m->C / d : 0.0;
        double dg = -k3 - omD * (hardening_slope(m, eps_p + d) * rf + h * drf);
        double nd = d - g / dg;
        if (!(nd > lo && nd < hi)) nd = 0.5 * (lo + hi);
        double step = fabs(nd - d);
        d = nd;
        if (step <= 1e-14 * d || step <= 1e-14 * seq_tr / k3 || hi - lo <= 1e-14 * hi) return d;
    }
    *failed = 1;
    return d;
}

static void alg1_return(const orc_material *m, double G, double D, double dt,
                        const double sd_n[9], const double deps_d[9], double eps_p,
                        double eps_rate, double sd_out[9], double *dep, int32_t *yielded,
                        int32_t *newton_failed) {
    double sd_tr[9];
    for (int k = 0; k < 9; ++k) sd_tr[k] = sd_n[k] + 2.0 * G * (1.0 - D) * deps_d[k];
    double seq_tr = von_mises(sd_tr);
    double sf = orc_flow_stress(m, eps_p, m->implicit_return ? 0.0 : eps_rate) * (1.0 - D);
    if (seq_tr < sf) {
        memcpy(sd_out, sd_tr, sizeof sd_tr);
        *dep = 0.0;
        *yielded = 0;
        return;
    }
    double k3 = 3.0 * G * (1.0 - D);
    double sy = sf;
    *dep = (seq_tr - sf) / k3;
    if (m->implicit_return) {
        *dep = implicit_increment(m, k3, 1.0 - D, seq_tr, eps_p, dt, *dep, newton_failed);
        sy = seq_tr - k3 * *dep;
    }
    for (int k = 0; k < 9; ++k) sd_out[k] = sy / seq_tr * sd_tr[k];
    *yielded = 1;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2 (Sec. 5.4): GTN return mapping with two Newton-Raphson      */
/* loops, always FP64.                                                      */
/* Readings: sigma_M is the undamaged matrix flow stress; f* enters the     */
/* yield function and its derivative, f the strain-increment equation, the  */
/* ratio alpha and the void update, as printed; the trial mean stress is    */
/* the undamaged Mie-Grueneisen value of the algorithm's first line;        */
/* sigma_y inside the second loop is x sigma_f(eps_M,n + d_eps_M) (the form */
/* its derivative g' assumes); the mean stress returns by                   */
/* sigma_m = sigma_m,trial - 3G(1-D) sigma* d_eps_p_eq with                 */
/* d_eps_p_eq = (sigma_eq,trial - sigma_y)/(3G(1-D)), which keeps the        */
/* triaxiality constant as the derivation assumes; nucleation is the        */
/* Chu-Needleman normal distribution (squared exponent) times d_eps_M;      */
/* Newton tolerances 1e-14 (absolute on x; on d_eps_M relative to the      */
/* increment c sigma_eq,trial that would unload the trial stress, the scale */
/* its rounding is set by: relative to d_eps_M itself a small increment    */
/* never converges), at most 50                                             */
/* iterations; a trial stress below 1e-12 sigma_M is elastic.               */
/* ------------------------------------------------------------------------ */
static void gtn_return(const orc_material *m, double G, double D, double dt,
                       const double sd_tr[9], double sm_tr, orc_point *pt,
                       double sd_out[9], double *sm_out, orc_point_info *info) {
    double f = pt->f_void;
    double fs = orc_fstar(m, f);
    double seq_tr = von_mises(sd_tr);
    double rate = pt->eps_p_rate;
    double sM = orc_flow_stress(m, pt->eps_p, rate);
    double dem = 0.0;
    int elastic = 1;
    double sstar = 0.0, Phi_tr = -1.0;
    if (seq_tr >= 1e-12 * sM) {
        sstar = sm_tr / seq_tr;
        double r = seq_tr / sM;
        Phi_tr = r * r + 2.0 * m->q1 * fs * cosh(1.5 * m->q2 * sstar * r)
               - (1.0 + m->q3 * fs * fs);
        elastic = Phi_tr < 0.0;
    }
    if (elastic) {
        memcpy(sd_out, sd_tr, 9 * sizeof(double));
        *sm_out = sm_tr;
        pt->eps_p_rate = 0.0;
        info->yielded = 0;
        return;
    }
    info->yielded = 1;
    /* first loop: x = sigma_y / sigma_M on the yield surface */
    double x = seq_tr / sM < 1.0 ? seq_tr / sM : 1.0;
    int it;
    for (it = 0; it < 50; ++it) {
        double arg = 1.5 * m->q2 * sstar * x;
        double Phi = x * x + 2.0 * m->q1 * fs * cosh(arg) - (1.0 + m->q3 * fs * fs);
        double dPhi = 2.0 * x + 3.0 * m->q1 * m->q2 * fs * sstar * sinh(arg);
        double dx = -Phi / dPhi;
        x += dx;
        if (fabs(dx) <= 1e-14) break;
    }
    info->newton_x_iters = it + 1;
    if (it == 50) info->newton_failed |= 1;
    /* second loop: matrix plastic strain increment */
    double arg = 1.5 * m->q2 * sstar * x;
    double c = (x + 1.5 * m->q1 * m->q2 * f * sstar * sinh(arg)) /
               (3.0 * G * (1.0 - D) * (1.0 - f));
    double sy = x * sM;
    dem = c * (seq_tr - sy);
    for (it = 0; it < 50; ++it) {
        double e1 = pt->eps_p + dem;
        double sf = orc_flow_stress(m, e1, rate);
        double g = dem - c * (seq_tr - x * sf);
        double dg = 1.0 + c * x * flow_stress_slope(m, e1, rate);
        double next = dem - g / dg;
        if (next < 0.0) next = 0.5 * dem; /* keep the increment non-negative */
        double step = next - dem;
        dem = next;
        if (fabs(step) <= 1e-14 * c * seq_tr) break;
    }
    info->newton_e_iters = it + 1;
    if (it == 50) info->newton_failed |= 2;
    pt->eps_p += dem;
    sM = orc_flow_stress(m, pt->eps_p, rate);
    sy = x * sM;
    for (int k = 0; k < 9; ++k) sd_out[k] = sy / seq_tr * sd_tr[k];
    double dep_eq = (seq_tr - sy) / (3.0 * G * (1.0 - D));
    *sm_out = sm_tr - 3.0 * G * (1.0 - D) * sstar * dep_eq;
    double alpha = 1.5 * (sM / sy) * m->q1 * m->q2 * f * sinh(arg);
    double s_new[6], full[9];
    for (int k = 0; k < 9; ++k) full[k] = sd_out[k];
    full[0] += *sm_out; full[4] += *sm_out; full[8] += *sm_out;
    full_to_voigt(full, s_new);
    double omega = orc_omega(s_new);
    double zN = (pt->eps_p - m->eN) / m->sN;
    double AN = m->fN / (m->sN * sqrt(2.0 * M_PI)) * exp(-0.5 * zN * zN);
    double df = AN * dem
              + (1.0 - f) / (alpha * sstar + 1.0) * (sM / sy)
                * (alpha * (1.0 - f) + f * m->k_omega * omega) * dem;
    pt->f_void = f + df;
    pt->eps_p_rate = dem / dt;
    info->dep = dem;
}

/* ------------------------------------------------------------------------ */
/* Constitutive update of one particle over one step (Secs. 4-5).           */
/* Readings: F^{n+1} = F^n + dt Fdot (the time integral of                   */
/* eq. Crack_approx_F); strain increment d dt with d = sym(Fdot Fbar^-1),    */
/* Fbar = (F^n + F^{n+1})/2; deviator rotated by Hughes-Winget; damage D^n   */
/* acts in the step, D^{n+1} = min(1, 10 max(0, D_init - 1)) at its end     */
/* (CL/JC, only when plastic strain grew); D = 1 carries no stress          */
/* (Sec. 3.1); energy e += dt J sigma:d / rho0 (eq. conservation3);          */
/* PK1 P = J sigma F^-T.                                                    */
/* ------------------------------------------------------------------------ */
void orc_point_update(const orc_material *m, double dt, const double Fdot[9],
                      orc_point *pt, double P[9], orc_point_info *info) {
    orc_point_info dummy;
    if (!info) info = &dummy;
    memset(info, 0, sizeof *info);
    double Fn[9], Fn1[9];
    memcpy(Fn, pt->F, sizeof Fn);
    for (int k = 0; k < 9; ++k) Fn1[k] = Fn[k] + dt * Fdot[k];
    memcpy(pt->F, Fn1, sizeof Fn1);
    double J = det3(Fn1);
    info->J = J;
    if (pt->D >= 1.0) {
        memset(pt->sig, 0, sizeof pt->sig);
        memset(P, 0, 9 * sizeof(double));
        return;
    }
    /* kinematics */
    double Fbar[9], Fbi[9], l[9], d[9], w[9];
    for (int k = 0; k < 9; ++k) Fbar[k] = 0.5 * (Fn[k] + Fn1[k]);
    inv3(Fbar, Fbi);
    mul3(Fdot, Fbi, l);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            d[3 * a + b] = 0.5 * (l[3 * a + b] + l[3 * b + a]);
            w[3 * a + b] = 0.5 * (l[3 * a + b] - l[3 * b + a]);
        }
    double S[9], sd_n[9];
    voigt_to_full(pt->sig, S);
    double sm_old = (S[0] + S[4] + S[8]) / 3.0;
    for (int k = 0; k < 9; ++k) sd_n[k] = S[k];
    sd_n[0] -= sm_old; sd_n[4] -= sm_old; sd_n[8] -= sm_old;
    double sd_rot[9];
    orc_hughes_winget(dt, w, sd_n, sd_rot);
    double deps_d[9];
    for (int k = 0; k < 9; ++k) deps_d[k] = d[k] * dt;
    double tr = (deps_d[0] + deps_d[4] + deps_d[8]) / 3.0;
    deps_d[0] -= tr; deps_d[4] -= tr; deps_d[8] -= tr;
    double G = m->E / (2.0 * (1.0 + m->nu));
    double D = pt->D;
    double sd_new[9], sm;

    if (m->damage == ORC_DMG_GTN) {
        double sd_tr[9];
        for (int k = 0; k < 9; ++k) sd_tr[k] = sd_rot[k] + 2.0 * G * (1.0 - D) * deps_d[k];
        double sm_tr = orc_mean_stress_eos(m, J, D, pt->e, 0);
        gtn_return(m, G, D, dt, sd_tr, sm_tr, pt, sd_new, &sm, info);
        pt->D = gtn_damage(m, pt->f_void);
    } else {
        sm = orc_mean_stress_eos(m, J, D, pt->e, 1);
        double dep;
        int32_t y;
        alg1_return(m, G, D, dt, sd_rot, deps_d, pt->eps_p, pt->eps_p_rate, sd_new, &dep, &y,
                    &info->newton_failed);
        info->yielded = y;
        info->dep = dep;
        pt->eps_p += dep;
        pt->eps_p_rate = dep / dt;
        if (dep > 0.0 && (m->damage == ORC_DMG_JC || m->damage == ORC_DMG_CL)) {
            if (m->damage == ORC_DMG_JC) {
                /* Sec. 5.2: D_init = sum d_eps / eps_f; Reading: d_eps_eq is
                 * the plastic increment, triaxiality sigma_m / sigma_eq and the
                 * rate at the end of the step, T* the specimen's constant */
                double seq = von_mises(sd_new);
                double sstar = sm / seq;
                double Tstar = m->T_star;
                double ef = (m->D1 + m->D2 * exp(m->D3 * sstar)) *
                            pow(1.0 + pt->eps_p_rate / m->eps_dot0, m->D4) *
                            (1.0 + m->D5 * Tstar);
                pt->d_init += dep / ef;
            } else {
                /* Sec. 5.1, eq. cockcroft-latham, right-endpoint quadrature */
                double full[9], s6[6];
                memcpy(full, sd_new, sizeof full);
                full[0] += sm; full[4] += sm; full[8] += sm;
                full_to_voigt(full, s6);
                double s1 = orc_principal_max(s6);
                pt->w_p += (s1 > 0.0 ? s1 : 0.0) * dep;
                pt->d_init = pt->w_p / m->Wcr;
            }
            /* Sec. 5.3 damage evolution, held in [0, 1] */
            double Dn = 10.0 * (pt->d_init - 1.0);
            if (Dn < 0.0) Dn = 0.0;
            if (Dn > 1.0) Dn = 1.0;
            pt->D = Dn;
        }
    }
    double sig[9];
    memcpy(sig, sd_new, sizeof sig);
    sig[0] += sm; sig[4] += sm; sig[8] += sm;
    if (pt->D >= 1.0) memset(sig, 0, sizeof sig);
    full_to_voigt(sig, pt->sig);
    voigt_to_full(pt->sig, sig);
    double Fi[9], FiT[9];
    inv3(Fn1, Fi);
    transpose3(Fi, FiT);
    mul3(sig, FiT, P);
    for (int k = 0; k < 9; ++k) P[k] *= J;
    /* eq. conservation3, de/dt = dF/dt : P / rho0, trapezoidal in P over the
     * step (P^n from the stress and F at the start of the step) */
    double Pn[9], Fni[9], FniT[9], Jn = det3(Fn);
    inv3(Fn, Fni);
    transpose3(Fni, FniT);
    mul3(S, FniT, Pn);
    double work = 0.0;
    for (int k = 0; k < 9; ++k) work += Fdot[k] * 0.5 * (Jn * Pn[k] + P[k]);
    pt->e += dt * work / m->rho0;
}

/* ------------------------------------------------------------------------ */
/* Initial state.                                                           */
/* ------------------------------------------------------------------------ */
void orc_init_state(const orc_problem *p, const double *v_init, orc_state *s) {
    for (int32_t k = 0; k < p->n_spec; ++k) s->t[k] = 0.0;
    for (int64_t i = 0; i < p->n; ++i) {
        const orc_material *m = &p->mat[p->spec[i]];
        for (int a = 0; a < 3; ++a) {
            s->u[3 * i + a] = 0.0;
            s->v[3 * i + a] = v_init ? v_init[3 * i + a] : 0.0;
            s->force[3 * i + a] = 0.0;
            s->fvisc[3 * i + a] = 0.0;
        }
        for (int k = 0; k < 9; ++k) {
            s->F[9 * i + k] = (k % 4 == 0) ? 1.0 : 0.0;
            s->Q[9 * i + k] = 0.0;
        }
        for (int k = 0; k < 6; ++k) s->sig[6 * i + k] = 0.0;
        s->eps_p[i] = s->eps_p_rate[i] = s->d_init[i] = s->w_p[i] = s->e[i] = 0.0;
        s->f_void[i] = m->f0;
        s->D[i] = (m->damage == ORC_DMG_GTN) ? gtn_damage(m, m->f0) : 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* One step n -> n+1.  Reading (the integrator is not described): leapfrog; */
/* forces at t^n with D^n, kick to v^{n+1/2}, prescribed velocities at      */
/* t^{n+1/2}, failed particles at rest (Sec. 3.1), drift, then dF/dt from    */
/* v^{n+1/2} and D^n and the constitutive update to t^{n+1}.                 */
/* ------------------------------------------------------------------------ */
static int is_reference_neighbour(const orc_problem *p, int64_t i, int32_t j) {
    int64_t lo = p->row_ptr[i], hi = p->row_ptr[i + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (p->col[mid] < j) lo = mid + 1; else hi = mid;
    }
    return lo < p->row_ptr[i + 1] && p->col[lo] == j;
}

static void contact_forces(const orc_problem *p, orc_state *s) {
    const int64_t n = p->n;
    int any = 0;
    for (int32_t k = 0; k < p->n_spec; ++k) any |= p->mat[k].contact_k > 0.0;
    if (!any || n == 0) return;
    /* current positions, radii; a uniform grid of edge 2 max a over all */
    double *x = (double *)malloc((size_t)n * 3 * sizeof(double));
    double *rad = (double *)malloc((size_t)n * sizeof(double));
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double amax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        rad[i] = 0.5 * cbrt(p->V0[i]);
        if (rad[i] > amax) amax = rad[i];
        for (int a = 0; a < 3; ++a) {
            x[3 * i + a] = p->X[3 * i + a] + s->u[3 * i + a];
            if (x[3 * i + a] < lo[a]) lo[a] = x[3 * i + a];
            if (x[3 * i + a] > hi[a]) hi[a] = x[3 * i + a];
        }
    }
    cell_grid g;
    const double edge = 2.0 * amax;
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = lo[a];
        g.dim[a] = (int64_t)floor((hi[a] - lo[a]) / edge) + 1;
        ncell *= g.dim[a];
    }
    g.start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    g.items = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int64_t c[3];
    for (int64_t i = 0; i < n; ++i) g.start[cell_of(&g, &x[3 * i], edge, c) + 1] += 1;
    for (int64_t k = 0; k < ncell; ++k) g.start[k + 1] += g.start[k];
    int64_t *fill = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
    memcpy(fill, g.start, (size_t)ncell * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) g.items[fill[cell_of(&g, &x[3 * i], edge, c)]++] = (int32_t)i;
    free(fill);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const orc_material *mi = &p->mat[p->spec[i]];
        int64_t ci[3];
        cell_of(&g, &x[3 * i], edge, ci);
        double f[3] = {0, 0, 0};
        for (int64_t dz = -1; dz <= 1; ++dz)
            for (int64_t dy = -1; dy <= 1; ++dy)
                for (int64_t dx = -1; dx <= 1; ++dx) {
                    int64_t cx = ci[0] + dx, cy = ci[1] + dy, cz = ci[2] + dz;
                    if (cx < 0 || cy < 0 || cz < 0 || cx >= g.dim[0] || cy >= g.dim[1] ||
                        cz >= g.dim[2])
                        continue;
                    int64_t id = cx + g.dim[0] * (cy + g.dim[1] * cz);
                    for (int64_t t = g.start[id]; t < g.start[id + 1]; ++t) {
                        int32_t j = g.items[t];
                        if (j == i) continue;
                        const orc_material *mj = &p->mat[p->spec[j]];
                        double kc = 0.5 * (mi->contact_k + mj->contact_k);
                        if (!(kc > 0.0)) continue;
                        double d[3], r2 = 0.0;
                        for (int a = 0; a < 3; ++a) {
                            d[a] = x[3 * j + a] - x[3 * i + a];
                            r2 += d[a] * d[a];
                        }
                        double rc = rad[i] + rad[j];
                        if (!(r2 < rc * rc) || !(r2 > 0.0)) continue;
                        if (p->spec[i] == p->spec[j] && s->D[i] < 1.0 && s->D[j] < 1.0 &&
                            is_reference_neighbour(p, i, j))
                            continue;
                        double r = sqrt(r2), delta = rc - r;
                        double Es = 1.0 / ((1.0 - mi->nu * mi->nu) / mi->E +
                                           (1.0 - mj->nu * mj->nu) / mj->E);
                        double F = kc * (4.0 / 3.0) * Es * sqrt(rad[i] * rad[j] / rc) *
                                   delta * sqrt(delta);
                        for (int a = 0; a < 3; ++a) f[a] -= F * d[a] / r;
                    }
                }
        for (int a = 0; a < 3; ++a) s->force[3 * i + a] += f[a];
    }
    free(g.start);
    free(g.items);
    free(x);
    free(rad);
}

void orc_step(const orc_problem *p, orc_state *s) {
    const int64_t n = p->n;

    /* 1. nodal forces: damage-modified form of eq. DSPH_nodal_forces (Sec. */
    /* 3.1) plus hourglass control.  Reading (the paper cites its hourglass  */
    /* scheme without a formula): error vector e_ij = Fbar_ij X_ij - x_ij    */
    /* with Fbar_ij = (F_i + F_j)/2, its projection delta on the current pair */
    /* direction, and the pair force                                          */
    /* -alpha E (1-D_i)(1-D_j) V_i V_j W_ij delta / |X_ij|^2 x_ij/|x_ij|.     */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const orc_material *m = &p->mat[p->spec[i]];
        double fi[3] = {0, 0, 0}, fhg[3] = {0, 0, 0};
        const double *Qi = &s->Q[9 * i], *Fi = &s->F[9 * i];
        double Di = s->D[i], Vi = p->V0[i];
        for (int64_t t = p->row_ptr[i]; t < p->row_ptr[i + 1]; ++t) {
            int32_t j = p->col[t];
            const double *Qj = &s->Q[9 * j], *Fj = &s->F[9 * j];
            double Dj = s->D[j], Vj = p->V0[j];
            double Xij[3], g[3], W;
            for (int a = 0; a < 3; ++a) Xij[a] = p->X[3 * j + a] - p->X[3 * i + a];
            kernel_gradient(Xij, pair_h(p, i, j), g, &W);
            for (int a = 0; a < 3; ++a) {
                double acc = 0.0;
                for (int b = 0; b < 3; ++b)
                    acc += ((1.0 - Dj) * Qi[3 * a + b] + (1.0 - Di) * Qj[3 * a + b]) * g[b];
                fi[a] += Vi * Vj * acc;
            }
            double xij[3], eij[3];
            for (int a = 0; a < 3; ++a)
                xij[a] = Xij[a] + s->u[3 * j + a] - s->u[3 * i + a];
            double r0 = sqrt(Xij[0] * Xij[0] + Xij[1] * Xij[1] + Xij[2] * Xij[2]);
            double r = sqrt(xij[0] * xij[0] + xij[1] * xij[1] + xij[2] * xij[2]);
            if (!(r > 0.0)) continue;
            for (int a = 0; a < 3; ++a) {
                double acc = 0.0;
                for (int b = 0; b < 3; ++b) acc += 0.5 * (Fi[3 * a + b] + Fj[3 * a + b]) * Xij[b];
                eij[a] = acc - xij[a];
            }
            double delta = (eij[0] * xij[0] + eij[1] * xij[1] + eij[2] * xij[2]) / r;
            double Ebar = 0.5 * (m->E + p->mat[p->spec[j]].E);
            double coef = -m->hg_alpha * Ebar * (1.0 - Di) * (1.0 - Dj) * Vi * Vj * W * delta /
                          (r0 * r0);
            for (int a = 0; a < 3; ++a) fhg[a] += coef * xij[a] / r;
        }
        for (int a = 0; a < 3; ++a) s->force[3 * i + a] = fi[a] + fhg[a] + s->fvisc[3 * i + a];
    }

    /* 1b. penalty contact between bodies and across cracks, beyond the      */
    /* kinematic wall (the paper has none).  Reading: particles are spheres  */
    /* of radius a_i = V_i^(1/3) / 2; two particles closer than a_i + a_j    */
    /* in the current configuration repel by the Hertz law of two such       */
    /* spheres,                                                              */
    /* F = k (4/3) E* sqrt(a_i a_j / (a_i + a_j)) delta^(3/2),               */
    /* delta = a_i + a_j - |x_ij|, 1/E* = (1-nu_i^2)/E_i + (1-nu_j^2)/E_j,     */
    /* k = (k_i + k_j)/2, along x_ij; reference neighbours that are both     */
    /* intact interact through the SPH forces only.  Positions at t^n.       */
    contact_forces(p, s);

    /* 2-3. kick, prescribed velocities, failed particles at rest, drift,   */
    /* rigid frictionless wall (projection onto the plane, inward normal    */
    /* velocity removed).                                                   */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const orc_material *m = &p->mat[p->spec[i]];
        double dt = m->dt;
        double mass = m->rho0 * p->V0[i];
        double *v = &s->v[3 * i], *u = &s->u[3 * i];
        const double *X = &p->X[3 * i];
        for (int a = 0; a < 3; ++a) v[a] += dt * s->force[3 * i + a] / mass;
        int32_t b = p->bc[i];
        if (b >= 0) {
            const orc_bc *g = &p->bcs[b];
            double th = s->t[p->spec[i]] + 0.5 * dt;
            double ramp = g->tau > 0.0 ? 1.0 - exp(-th / g->tau) : 1.0;
            for (int c = 0; c < 3; ++c)
                if (g->mask & (1 << c))
                    v[c] = g->v_max[c] * ramp
                         + (g->grad[3 * c + 0] * X[0] + g->grad[3 * c + 1] * X[1]
                            + g->grad[3 * c + 2] * X[2]);
        }
        if (s->D[i] >= 1.0) v[0] = v[1] = v[2] = 0.0;
        for (int a = 0; a < 3; ++a) u[a] += dt * v[a];
        if (m->has_wall) {
            const double *nw = m->wall_n;
            double x[3] = {X[0] + u[0], X[1] + u[1], X[2] + u[2]};
            double dn = x[0] * nw[0] + x[1] * nw[1] + x[2] * nw[2] - m->wall_d;
            if (dn < 0.0) {
                for (int a = 0; a < 3; ++a) u[a] = (x[a] - dn * nw[a]) - X[a];
                double vn = v[0] * nw[0] + v[1] * nw[1] + v[2] * nw[2];
                if (vn < 0.0)
                    for (int a = 0; a < 3; ++a) v[a] -= vn * nw[a];
            }
        }
    }

    /* 4. eq. Crack_approx_Fdot: dF/dt = sum_j V_j (1 - D_j)(v_j - v_i)     */
    /*    (x) gradW_i(X_ij) L_i^-1, with D at level n.                      */
    /*    With it, the artificial particle-velocity damping Sec. 2 says     */
    /*    TLSPH needs against rank deficiency (no formula given).  Reading: */
    /*    the Monaghan viscosity on the reference pair geometry,            */
    /*      mu_ij = h (v_ij . X_ij) / (|X_ij|^2 + 0.01 h^2),                */
    /*      Pi_ij = (-Q1 c0 mu_ij + Q2 mu_ij^2) / rho0 for v_ij . X_ij < 0  */
    /*      (else 0),                                                       */
    /*      f_i = sum_j m_i m_j (1 - D_i)(1 - D_j) Pi_ij gradW_ij,          */
    /*    with v = v^{n+1/2} and D at level n, applied in the next kick.    */
    double *Fdot = (double *)malloc((size_t)n * 9 * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const orc_material *m = &p->mat[p->spec[i]];
        const double *Li = &p->Linv[9 * i];
        double Fd[9] = {0}, fv[3] = {0, 0, 0};
        const int av = m->av_q1 != 0.0 || m->av_q2 != 0.0;
        for (int64_t t = p->row_ptr[i]; t < p->row_ptr[i + 1]; ++t) {
            int32_t j = p->col[t];
            double Xij[3], g[3], gh[3];
            const double hij = pair_h(p, i, j);
            for (int a = 0; a < 3; ++a) Xij[a] = p->X[3 * j + a] - p->X[3 * i + a];
            kernel_gradient(Xij, hij, g, NULL);
            /* corrected gradient: row vector gradW times L^-1 */
            for (int b = 0; b < 3; ++b)
                gh[b] = g[0] * Li[0 * 3 + b] + g[1] * Li[1 * 3 + b] + g[2] * Li[2 * 3 + b];
            double wgt = p->V0[j] * (1.0 - s->D[j]);
            for (int a = 0; a < 3; ++a) {
                double dv = s->v[3 * j + a] - s->v[3 * i + a];
                for (int b = 0; b < 3; ++b) Fd[3 * a + b] += wgt * dv * gh[b];
            }
            if (av) {
                double vx = 0.0, r2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    vx += (s->v[3 * j + a] - s->v[3 * i + a]) * Xij[a];
                    r2 += Xij[a] * Xij[a];
                }
                if (vx < 0.0) {
                    double mu = hij * vx / (r2 + 0.01 * hij * hij);
                    double Pi = (-m->av_q1 * m->c0 * mu + m->av_q2 * mu * mu) / m->rho0;
                    double mm = m->rho0 * p->V0[i] * m->rho0 * p->V0[j] *
                                (1.0 - s->D[i]) * (1.0 - s->D[j]);
                    for (int a = 0; a < 3; ++a) fv[a] += mm * Pi * g[a];
                }
            }
        }
        memcpy(&Fdot[9 * i], Fd, sizeof Fd);
        for (int a = 0; a < 3; ++a) s->fvisc[3 * i + a] = fv[a];
    }

    /* 5-13. constitutive update, Q_i = P_i L_i^-T */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const orc_material *m = &p->mat[p->spec[i]];
        orc_point pt;
        memcpy(pt.F, &s->F[9 * i], sizeof pt.F);
        memcpy(pt.sig, &s->sig[6 * i], sizeof pt.sig);
        pt.eps_p = s->eps_p[i];
        pt.eps_p_rate = s->eps_p_rate[i];
        pt.d_init = s->d_init[i];
        pt.w_p = s->w_p[i];
        pt.f_void = s->f_void[i];
        pt.D = s->D[i];
        pt.e = s->e[i];
        double P[9];
        orc_point_update(m, m->dt, &Fdot[9 * i], &pt, P, NULL);
        memcpy(&s->F[9 * i], pt.F, sizeof pt.F);
        memcpy(&s->sig[6 * i], pt.sig, sizeof pt.sig);
        s->eps_p[i] = pt.eps_p;
        s->eps_p_rate[i] = pt.eps_p_rate;
        s->d_init[i] = pt.d_init;
        s->w_p[i] = pt.w_p;
        s->f_void[i] = pt.f_void;
        s->D[i] = pt.D;
        s->e[i] = pt.e;
        const double *Li = &p->Linv[9 * i];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
                for (int c = 0; c < 3; ++c) acc += P[3 * a + c] * Li[3 * b + c];
                s->Q[9 * i + 3 * a + b] = (pt.D >= 1.0) ? 0.0 : acc;
            }
    }
    free(Fdot);
    for (int32_t k = 0; k < p->n_spec; ++k) s->t[k] += p->mat[k].dt;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics of a state: the quantities the runs of Sec. 6 are read by     */
/* (the force on each gripped end, i.e. minus its reaction, and the grips'   */
/* displacement) and the two energies of eq. conservation3's balance.        */
/* Per specimen: sum 1/2 m |v|^2 with m = rho0 V0 and v the stored           */
/* half-step velocity, sum m e, the number of failed particles (D >= 1),     */
/* max D, and the specimen's time.  Per prescribed-velocity group: the sum   */
/* of the members' nodal forces, their mean displacement, their count.      */
/* Plain sums in ascending particle order.                                   */
/* ------------------------------------------------------------------------ */
void orc_diagnostics(const orc_problem *p, const orc_state *s, double *spec_diag,
                     double *bc_diag) {
    for (int32_t q = 0; q < p->n_spec; ++q) {
        for (int k = 0; k < 8; ++k) spec_diag[8 * q + k] = 0.0;
        spec_diag[8 * q + 4] = s->t[q];
    }
    for (int32_t g = 0; g < p->n_bc; ++g)
        for (int k = 0; k < 8; ++k) bc_diag[8 * g + k] = 0.0;
    for (int64_t i = 0; i < p->n; ++i) {
        int32_t q = p->spec[i];
        double m = p->mat[q].rho0 * p->V0[i];
        const double *v = s->v + 3 * i;
        double *o = spec_diag + 8 * q;
        o[0] += 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        o[1] += m * s->e[i];
        if (s->D[i] >= 1.0) o[2] += 1.0;
        if (s->D[i] > o[3]) o[3] = s->D[i];
        int32_t g = p->bc[i];
        if (g >= 0 && g < p->n_bc) {
            double *b = bc_diag + 8 * g;
            for (int a = 0; a < 3; ++a) {
                b[a] += s->force[3 * i + a];
                b[3 + a] += s->u[3 * i + a];
            }
            b[6] += 1.0;
        }
    }
    for (int32_t g = 0; g < p->n_bc; ++g) {
        double *b = bc_diag + 8 * g;
        if (b[6] > 0.0)
            for (int a = 0; a < 3; ++a) b[3 + a] /= b[6];
    }
}

/* Thread count of the OpenMP loops (results do not depend on it). */
void orc_set_threads(int32_t nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int32_t orc_get_threads(void) {
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}
