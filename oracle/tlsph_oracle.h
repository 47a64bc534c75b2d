/*
 * tlsph_oracle.h -- plain FP64 CPU oracle for one Total-Lagrangian SPH
 * timestep with ductile damage (de Vaucorbeil & Hutchinson, "A damage and
 * failure implementation for the simulation of ductile solids with
 * Total-Lagrangian SPH", arXiv:1901.07374).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct reference
 * the GPU library is checked against.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it; the product path never
 * does.  It shares no source with the GPU library.
 *
 * Layout (host memory, caller order): vectors double[n][3]; tensors
 * double[n][9] row-major (A_ab at 3a+b); symmetric tensors double[n][6] in
 * Voigt order (xx, yy, zz, yz, xz, xy).  SI units.
 */
#ifndef TLSPH_ORACLE_H
#define TLSPH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_DMG_NONE = 0, ORC_DMG_CL = 1, ORC_DMG_JC = 2, ORC_DMG_GTN = 3 };
/* Strain-hardening law of the flow stress (Sec. 4 names linear plastic,
 * Johnson-Cook, Swift and Voce; the forms are readings):
 *   JC      A + B eps^n          LINEAR  A + B eps
 *   SWIFT   B (e0 + eps)^n       VOCE    A + B (1 - exp(-beta eps))
 * each times the rate factor 1 + C ln max(eps_rate / eps_dot0, 1). */
enum { ORC_FLOW_JC = 0, ORC_FLOW_LINEAR = 1, ORC_FLOW_SWIFT = 2, ORC_FLOW_VOCE = 3 };

/* Per-specimen material and run parameters. */
typedef struct {
    double rho0, E, nu, c0, S_alpha, Gamma0;   /* Mie-Grueneisen EOS, Sec. 4 */
    double A, B, n, C, eps_dot0;               /* Johnson-Cook flow, Sec. 4 */
    int32_t damage;                            /* ORC_DMG_* */
    double Wcr;                                /* Cockcroft-Latham, Sec. 5.1 */
    double D1, D2, D3, D4, D5;                 /* Johnson-Cook failure, Sec. 5.2 */
    double q1, q2, q3, f0, fN, eN, sN, fc, fF, k_omega; /* GTN, Sec. 5.4 */
    double h, dt, hg_alpha;                    /* support radius, step, hourglass */
    int32_t has_wall;
    double wall_n[3], wall_d;                  /* rigid plane x.n = d */
    int32_t flow;                              /* ORC_FLOW_* */
    int32_t implicit_return;                   /* 1: hardening at the end of the step */
    double flow_e0, flow_beta;                 /* Swift offset strain, Voce rate */
    double av_q1, av_q2;                       /* artificial viscosity (0: off) */
    double h_per_spacing;                      /* > 0: support h_i = this times   */
                                               /* V_i^(1/3) per particle (graded  */
                                               /* spacing); 0: h for all          */
    double contact_k;                          /* penalty contact factor (0: off) */
    double T_star, m;                          /* homologous temperature (held    */
                                               /* constant; 0: isothermal) and    */
                                               /* thermal exponent, Sec. 4        */
} orc_material;

/* Prescribed-velocity group: component c (bit c of mask) is set to
 * v_max[c] (1 - exp(-t/tau)) + sum_b grad[3c+b] X_b  (tau = 0: v_max[c]). */
typedef struct {
    int32_t mask;
    double v_max[3], tau, grad[9];
} orc_bc;

typedef struct {
    int64_t n;
    int32_t n_spec;
    const int32_t *spec;        /* [n] specimen of each particle            */
    const orc_material *mat;    /* [n_spec]                                 */
    const double *X;            /* [n][3] reference positions               */
    const double *V0;           /* [n] reference volumes                    */
    const int32_t *bc;          /* [n] group id, -1 = free                  */
    int32_t n_bc;
    const orc_bc *bcs;          /* [n_bc]                                   */
    const int64_t *row_ptr;     /* [n+1] neighbour list (ascending rows)    */
    const int32_t *col;         /* [nnz]                                    */
    const double *Linv;         /* [n][9] inverse correction matrices       */
    const double *hs;           /* [n] support radius of each particle      */
} orc_problem;

typedef struct {
    double *t;                  /* [n_spec] time of each specimen           */
    double *u, *v;              /* [n][3] displacement, half-step velocity  */
    double *F;                  /* [n][9] deformation gradient              */
    double *sig;                /* [n][6] Cauchy stress                     */
    double *eps_p, *eps_p_rate; /* [n] eq. plastic strain (matrix for GTN)  */
    double *d_init, *w_p;       /* [n] damage initiation, CL plastic work   */
    double *f_void, *D, *e;     /* [n] void fraction, damage, energy/mass   */
    double *Q;                  /* [n][9] P L^-T                            */
    double *force;              /* [n][3] internal + hourglass (+ viscous)  */
    double *fvisc;              /* [n][3] artificial viscous force, computed */
                                /* from v^{n+1/2} and applied in the next   */
                                /* step's kick                              */
} orc_state;

/* One material point, for the constitutive pieces on their own. */
typedef struct {
    double F[9], sig[6];
    double eps_p, eps_p_rate, d_init, w_p, f_void, D, e;
} orc_point;

typedef struct {
    double dep;          /* plastic strain increment of the step            */
    double J;            /* det F at the end of the step                    */
    int32_t yielded;
    int32_t newton_x_iters, newton_e_iters, newton_failed;
} orc_point_info;

/* Cubic-spline kernel with compact support of radius h. */
void orc_kernel(double r, double h, double *W, double *dWdr);

/* Support radius of each particle: mat.h, or h_per_spacing V_i^(1/3). */
void orc_support_radii(int64_t n, const double *V0, const int32_t *spec,
                       const orc_material *mat, double *hs);

/* Neighbour sets S_i = { j != i, same specimen, |X_j - X_i| < h_ij } with
 * h_ij = (h_i + h_j) / 2 (hs; NULL: the specimen's h).
 * Rows ascending.  Returns nnz; if nnz > cap only row_ptr is written. */
int64_t orc_build_neighbors(int64_t n, const double *X, const int32_t *spec,
                            const orc_material *mat, const double *hs, int64_t *row_ptr,
                            int32_t *col, int64_t cap);

/* Correction matrices L_i and their inverses.  Returns -1, or the index of
 * the first particle whose L is singular. */
int64_t orc_shape_matrices(const orc_problem *p, double *L, double *Linv);

/* u = 0, v = v_init, F = I, sig = 0, accumulators 0, f = f0, D = q1 f*(f0)
 * under GTN (else 0), Q = 0, t = 0. */
void orc_init_state(const orc_problem *p, const double *v_init, orc_state *s);

/* One leapfrog step of every specimen. */
void orc_step(const orc_problem *p, orc_state *s);

/* Diagnostics of the state: spec_diag double[n_spec][8] = sum 1/2 m |v|^2,
 * sum m e, failed count (D >= 1), max D, time, 0, 0, 0; bc_diag
 * double[n_bc][8] = summed nodal force (3), mean displacement (3), count, 0.
 * Plain sums in ascending particle order. */
void orc_diagnostics(const orc_problem *p, const orc_state *s, double *spec_diag,
                     double *bc_diag);

/* Constitutive update of one material point over one step, given dF/dt. */
void orc_point_update(const orc_material *m, double dt, const double Fdot[9],
                      orc_point *pt, double P[9], orc_point_info *info);

/* Pieces exposed for the pin tests. */
double orc_mean_stress_eos(const orc_material *m, double J, double D, double e,
                           int32_t damaged_branch_allowed);
double orc_flow_stress(const orc_material *m, double eps, double eps_rate);
double orc_principal_max(const double sig[6]);
double orc_omega(const double sig[6]);
double orc_fstar(const orc_material *m, double f);
void orc_hughes_winget(double dt, const double w[9], const double sd_in[9],
                       double sd_out[9]);

/* OpenMP thread count (results are identical for any count). */
void orc_set_threads(int32_t nthreads);
int32_t orc_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
