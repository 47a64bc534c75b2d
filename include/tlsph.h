/*
 * tlsph.h -- C ABI of the MI355X (gfx950) Total-Lagrangian SPH timestep with
 * ductile damage of de Vaucorbeil & Hutchinson, "A damage and failure
 * implementation for the simulation of ductile solids with Total-Lagrangian
 * Smooth Particle Hydrodynamics" (arXiv:1901.07374).
 *
 * One step, over a neighbour list fixed in the reference configuration
 * (Sec. 2), gathers the damage-weighted velocity gradient dF/dt with the
 * corrected kernel gradient (eqs. Crack_approx_Fdot, correction_matrix),
 * updates F, the Mie-Grueneisen mean stress (Sec. 4, eq. pH), the
 * Johnson-Cook radial return (Algorithm 1), the Cockcroft-Latham /
 * Johnson-Cook / GTN damage (Secs. 5.1-5.4, Algorithm 2), then the damaged
 * nodal forces (Sec. 3.1) with hourglass control and a leapfrog update.
 *
 * Conventions
 *  - Pointers marked (dev) are HIP device memory owned by the caller; the
 *    library never allocates device memory.  Pointers marked (host) are read
 *    during the call only.
 *  - Per-particle device arrays exchanged through the ABI are in the caller's
 *    particle order and component-major ("SoA"): a vector field is
 *    double[3][n], a tensor double[9][n] with A_ab at component 3a+b, a
 *    symmetric tensor double[6][n] in Voigt order (xx, yy, zz, yz, xz, xy).
 *  - Particles of specimen s are the contiguous range
 *    [spec_offsets[s], spec_offsets[s+1]); neighbours never cross specimens.
 *  - SI units (m, kg, s, Pa).
 *  - Every call returns a status; nothing throws or aborts across the ABI.
 *    Argument errors are detected before any HIP call.  Detail text of the
 *    last failure is available from tlsph_last_error().
 *  - All device work is ordered on the stream passed in, host copies
 *    included.  Only tlsph_build_neighbors, tlsph_autotune,
 *    tlsph_set_launch_shape (a new tile size) and tlsph_info synchronise with
 *    the host, on that stream.  A context is used by one host thread at a
 *    time.
 *  - Summation order is fixed per particle (no floating-point atomics): the
 *    same inputs give bitwise identical results run to run and for every
 *    launch shape the autotuner may pick.
 */
#ifndef TLSPH_H
#define TLSPH_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tlsph_ctx tlsph_ctx;

typedef enum {
    TLSPH_OK = 0,
    TLSPH_E_INVALID_ARG = 1,   /* null pointer, negative size, bad enum, ...   */
    TLSPH_E_BAD_STATE = 2,     /* call order: e.g. step before build           */
    TLSPH_E_HIP = 3,           /* a HIP runtime call failed (text in last_error) */
    TLSPH_E_SINGULAR_L = 4,    /* a correction matrix is singular (Sec. 2.2)   */
    TLSPH_E_NONFINITE = 5,     /* non-finite state found by the finite check    */
    TLSPH_E_CAPACITY = 6,      /* a particle has more than k_cap neighbours    */
    TLSPH_E_UNSUPPORTED = 7    /* outside the library's limits                 */
} tlsph_status;

typedef enum {
    TLSPH_FP64 = 0,   /* every quantity in double precision                     */
    TLSPH_MIXED = 1   /* kernel gradients, F - I, stresses, Q and pair forces in
                         float with fixed-order float sums; correction-matrix
                         inversion, the GTN return mapping, plastic-strain and
                         damage accumulators, displacement and velocity in double */
} tlsph_precision;

typedef enum {
    TLSPH_DMG_NONE = 0,   /* Johnson-Cook plasticity without damage evolution */
    TLSPH_DMG_CL = 1,     /* Cockcroft-Latham initiation (Sec. 5.1) + Sec. 5.3 */
    TLSPH_DMG_JC = 2,     /* Johnson-Cook initiation (Sec. 5.2) + Sec. 5.3     */
    TLSPH_DMG_GTN = 3     /* Gurson-Tvergaard-Needleman (Sec. 5.4, Alg. 2)     */
} tlsph_damage;

typedef enum {
    TLSPH_FLOW_JC = 0,      /* A + B eps^n (eq. JC_viscoplastic_model)             */
    TLSPH_FLOW_LINEAR = 1,  /* A + B eps                                         */
    TLSPH_FLOW_SWIFT = 2,   /* B (flow_e0 + eps)^n                               */
    TLSPH_FLOW_VOCE = 3     /* A + B (1 - exp(-flow_beta eps))                   */
} tlsph_flow;   /* strain-hardening law of the flow stress (Sec. 4 names all four; the
                   forms are readings); every law is multiplied by the rate factor
                   1 + C ln max(eps_rate / eps_dot0, 1) and by 1 - D */

/* create() flags */
#define TLSPH_STORE_FORCE   1u  /* keep the nodal force of every particle (else only
                                   of particles in a prescribed-velocity group) */
#define TLSPH_USE_GRAPHS    2u  /* tlsph_step replays a captured two-step hipGraph */
#define TLSPH_CHECK_FINITE  4u  /* latch TLSPH_E_NONFINITE if a stress turns non-finite */
#define TLSPH_NO_STAGING    8u  /* gather neighbours from global memory instead of staging
                                   each tile and its halo in LDS (same results, bitwise) */

/* One specimen: material (Sec. 4 and Tables 1-3) and run parameters. */
typedef struct {
    double rho0, E, nu, c0, S_alpha, Gamma0;  /* Mie-Grueneisen EOS (eq. pH)        */
    double A, B, n, C, eps_dot0;              /* Johnson-Cook flow                  */
    int32_t damage;                           /* tlsph_damage                       */
    double Wcr;                               /* Cockcroft-Latham critical work     */
    double D1, D2, D3, D4, D5;                /* Johnson-Cook failure strain        */
    double q1, q2, q3, f0, fN, eN, sN, fc, fF, k_omega; /* GTN                      */
    double h;                                 /* kernel support radius (> 0)        */
    double dt;                                /* time step (> 0)                    */
    double hg_alpha;                          /* hourglass control coefficient      */
    int32_t has_wall;                         /* 1: rigid frictionless plane        */
    double wall_n[3], wall_d;                 /* plane x . n = d, n unit normal     */
    int32_t flow;                             /* tlsph_flow                         */
    int32_t implicit_return;                  /* 0: Algorithm 1 with the flow stress at
                                                 the step's start (explicit hardening);
                                                 1: the plastic increment solves the
                                                 consistency condition with the flow
                                                 stress at the step's end (hardening and
                                                 rate); no effect under GTN            */
    double flow_e0;                           /* Swift offset strain (> 0)          */
    double flow_beta;                         /* Voce saturation rate (>= 0)        */
    double av_q1, av_q2;                      /* artificial particle-velocity damping
                                                 (Sec. 2; both 0: off): Monaghan
                                                 viscosity on the reference pair
                                                 geometry, mu = h v_ij.X_ij /
                                                 (|X_ij|^2 + 0.01 h^2), Pi = (-av_q1 c0
                                                 mu + av_q2 mu^2) / rho0 for approaching
                                                 pairs, f_i = sum_j m_i m_j (1 - D_i)
                                                 (1 - D_j) Pi gradW_ij, from v^{n+1/2},
                                                 applied in the next kick            */
    double h_per_spacing;                     /* > 0: graded spacing, each particle's
                                                 support h_i = h_per_spacing V_i^(1/3)
                                                 and a pair's (h_i + h_j) / 2 (membership
                                                 and kernel); the staged kernels then
                                                 carry each slot's support in LDS.
                                                 0: h for all                        */
    double contact_k;                         /* penalty contact factor (0: off): particles
                                                 are spheres of radius V_i^(1/3)/2; two
                                                 closer than a_i + a_j in the current
                                                 configuration repel by the Hertz law
                                                 F = k (4/3) E* sqrt(a_i a_j/(a_i+a_j))
                                                 delta^(3/2), k the mean of the two
                                                 factors; intact reference neighbours
                                                 interact through SPH only (see
                                                 tlsph_set_contact)                   */
    double T_star, m;                         /* homologous temperature T* in [0, 1),
                                                 held constant, and the thermal
                                                 exponent m (> 0 when T* > 0): the flow
                                                 stress carries 1 - T*^m (eq.
                                                 JC_viscoplastic_model), the JC failure
                                                 strain 1 + D5 T* (Sec. 5.2); T* = 0:
                                                 isothermal                           */
    int32_t newton_max_iter;                  /* iteration cap of the Newton loops of
                                                 Algorithm 2 and of the implicit return
                                                 (0: 50 and 100); a loop that reaches it
                                                 keeps its last iterate and raises info
                                                 flag bit 1.  Tests force that path with
                                                 a cap of 1                           */
} tlsph_specimen;

/* Prescribed-velocity group.  At mid-step time t the velocity component c of
 * every member with bit c of mask set is v_max[c] (1 - exp(-t/tau)) +
 * sum_b grad[3c+b] X_b (X the reference position; tau = 0 means v_max[c]). */
typedef struct {
    int32_t mask;
    double v_max[3];
    double tau;
    double grad[9];
} tlsph_bc_group;

/* Fields of tlsph_get_state / tlsph_set_state (components, then meaning). */
typedef enum {
    TLSPH_F_X = 0,          /* 3  reference position (get only)                    */
    TLSPH_F_U = 1,          /* 3  displacement u = x - X                           */
    TLSPH_F_V = 2,          /* 3  velocity at the last half step v^{n+1/2}          */
    TLSPH_F_DEFGRAD = 3,    /* 9  deformation gradient F                           */
    TLSPH_F_SIGMA = 4,      /* 6  Cauchy stress                                    */
    TLSPH_F_EPS_P = 5,      /* 1  equivalent plastic strain (matrix strain, GTN)   */
    TLSPH_F_EPS_P_RATE = 6, /* 1  plastic strain rate of the last step             */
    TLSPH_F_D_INIT = 7,     /* 1  damage initiation variable                       */
    TLSPH_F_W_P = 8,        /* 1  Cockcroft-Latham plastic work                    */
    TLSPH_F_VOID = 9,       /* 1  GTN void volume fraction f                       */
    TLSPH_F_D = 10,         /* 1  damage D                                         */
    TLSPH_F_E_INT = 11,     /* 1  internal energy per unit mass                    */
    TLSPH_F_FORCE = 12,     /* 3  nodal force of the last step (get only)          */
    TLSPH_F_Q = 13,         /* 9  Q = P L^-T used by the next force evaluation     */
    TLSPH_F_TIME = 14,      /* n_spec time of each specimen (not per particle)     */
    TLSPH_F_LINV = 15,      /* 9  inverse correction matrix (get only)             */
    TLSPH_F_VISC = 16,      /* 3  artificial viscous force for the next kick        */
    TLSPH_F_H = 17          /* 9  F - I as stored (exact round trip: checkpoints)   */
} tlsph_field;

#define TLSPH_N_DIAG 8
/* Per-specimen diagnostics, double[n_spec][8]:
 *   0 kinetic energy  sum 1/2 m v^2          1 internal energy sum m e
 *   2 failed particles (D = 1)              3 max D
 *   4 time                                  5-7 reserved (0)
 * Per prescribed-velocity group, double[n_bc][8]:
 *   0-2 sum of the nodal force over the group (the negative of the reaction)
 *   3-5 mean displacement of the group      6 member count    7 reserved  */

/* Bytes of device workspace for n particles in n_spec specimens with at most
 * n_bc prescribed-velocity groups and k_cap neighbours per particle.
 * Host only, no HIP call.  Errors: INVALID_ARG (n < 1, n_spec < 1,
 * n_bc < 0, k_cap < 1 or > 512, bad precision, null bytes). */
tlsph_status tlsph_workspace_bytes(int64_t n, int32_t n_spec, int32_t n_bc, int32_t k_cap,
                                   tlsph_precision precision, size_t *bytes);

/* Create a context over a caller-owned device workspace of ws_bytes >=
 * tlsph_workspace_bytes(...).  spec_offsets (host, int64[n_spec+1],
 * non-decreasing, 0 .. n), spec (host, tlsph_specimen[n_spec]) and bc (host,
 * tlsph_bc_group[n_bc], may be null when n_bc = 0) are copied.  The
 * workspace must stay allocated until tlsph_destroy and is not touched by
 * anything else.  Errors: INVALID_ARG (sizes, parameters outside their
 * domain: rho0, E, c0, h, dt <= 0, nu outside (-1, 0.5), damage enum,
 * workspace too small or not 256-byte aligned), HIP. */
tlsph_status tlsph_create(int64_t n, int32_t n_spec, const int64_t *spec_offsets,
                          const tlsph_specimen *spec, int32_t n_bc, const tlsph_bc_group *bc,
                          tlsph_precision precision, int32_t k_cap, uint32_t flags,
                          void *workspace, size_t ws_bytes, hipStream_t stream,
                          tlsph_ctx **out);

/* Reference configuration and the fixed neighbour list (Sec. 2: S_i is set
 * once in the undeformed configuration and never rebuilt).
 * X (dev, double[3][n]) reference positions, V0 (dev, double[n]) reference
 * volumes, bc_group (dev, int32[n], -1 = free, else < n_bc).  They are copied.
 * Builds S_i = { j != i in the same specimen : |X_j - X_i| < h } on the GPU
 * (particles reordered along a Hilbert curve internally), the correction
 * matrices L_i (eq. correction_matrix) and their inverses in double, and the
 * initial state: u = 0, v = 0, F = I, stress and accumulators 0, f = f0,
 * D = q1 f*(f0) under GTN (else 0), Q = 0, time 0.  Synchronises the stream
 * once.  Errors: CAPACITY (some particle has more than k_cap neighbours),
 * SINGULAR_L (|det L_i| <= 1e-12 |L_i|_F^3; index in last_error),
 * UNSUPPORTED (more than 16384 cells of size h along an axis), HIP. */
tlsph_status tlsph_build_neighbors(tlsph_ctx *ctx, const double *X, const double *V0,
                                   const int32_t *bc_group, hipStream_t stream);

/* Advance every specimen by n_steps leapfrog steps (each specimen with its
 * own dt).  One step: nodal forces at t^n with D^n (Sec. 3.1, damaged form of
 * eq. DSPH_nodal_forces, plus hourglass control), kick to v^{n+1/2},
 * prescribed velocities at t^{n+1/2}, failed particles (D = 1) at rest,
 * drift (rigid wall if set), then dF/dt from v^{n+1/2} and D^n
 * (eq. Crack_approx_Fdot), F^{n+1} = F^n + dt dF/dt (eq. Crack_approx_F) and
 * the constitutive and damage update to t^{n+1}.  Asynchronous; enqueues no
 * host synchronisation, allocation or memset, so a caller may capture it.
 * Errors: BAD_STATE (before build), INVALID_ARG (n_steps < 0), HIP. */
tlsph_status tlsph_step(tlsph_ctx *ctx, int32_t n_steps, hipStream_t stream);

/* Copy a field to dst (dev, double, layout of tlsph_field in caller order;
 * bytes must equal components * n * 8, or n_spec * 8 for TIME).  Fields held
 * in float in the mixed form are widened.  Errors: BAD_STATE, INVALID_ARG. */
tlsph_status tlsph_get_state(tlsph_ctx *ctx, tlsph_field field, double *dst, size_t bytes,
                             hipStream_t stream);

/* Overwrite a field from src (dev, same layout as get).  X, FORCE and LINV
 * are read-only.  Lets a caller inject a state for one-step checks and
 * resume from a checkpoint.  Errors: BAD_STATE, INVALID_ARG. */
tlsph_status tlsph_set_state(tlsph_ctx *ctx, tlsph_field field, const double *src, size_t bytes,
                             hipStream_t stream);

/* Number of neighbour pairs (sum of |S_i|), known after build.  Host only. */
tlsph_status tlsph_neighbor_count(const tlsph_ctx *ctx, int64_t *nnz);

/* The neighbour list in caller order as CSR with ascending rows:
 * row_ptr (dev, int64[n+1]), col (dev, int32[nnz]).  Errors: BAD_STATE. */
tlsph_status tlsph_get_neighbors(tlsph_ctx *ctx, int64_t *row_ptr, int32_t *col,
                                 hipStream_t stream);

/* Diagnostics (layout above) into spec_diag (dev, double[n_spec][8]) and,
 * if n_bc > 0 and bc_diag is not null, bc_diag (dev, double[n_bc][8]).
 * Fixed-order reductions.  Errors: BAD_STATE, INVALID_ARG. */
tlsph_status tlsph_get_diagnostics(tlsph_ctx *ctx, double *spec_diag, double *bc_diag,
                                   hipStream_t stream);

/* The same diagnostics for callers that cannot allocate device memory at
 * the call (code under graph capture, serving loops, harnesses that forbid
 * allocation): identical kernels, summation order and results, with the
 * chunk partials in a static device array of the library (1 MiB per device,
 * 16384 partials: one per 2048 particles of each specimen and each group,
 * at least one each) instead of the workspace.  Allocates nothing; the first
 * call on a device looks up that device's array.  Every call on one device
 * shares the array: calls that overlap on one device (other streams or
 * threads) race and must be ordered by the caller.  Errors: as
 * tlsph_get_diagnostics, CAPACITY when the partials would not fit. */
tlsph_status tlsph_get_diagnostics_static(tlsph_ctx *ctx, double *spec_diag, double *bc_diag,
                                          hipStream_t stream);

/* Replace the prescribed-velocity table (host, tlsph_bc_group[n_bc],
 * n_bc <= the count given at create), ordered on the stream.  Errors:
 * INVALID_ARG, HIP. */
tlsph_status tlsph_set_bc_groups(tlsph_ctx *ctx, int32_t n_bc, const tlsph_bc_group *bc,
                                 hipStream_t stream);

/* Pick the launch shape of each step kernel by timing the candidates on the
 * current state; the state is saved and restored, so results are unchanged.
 * Synchronises.  Errors: BAD_STATE, HIP. */
tlsph_status tlsph_autotune(tlsph_ctx *ctx, hipStream_t stream);

/* Per-kernel timing with HIP events recorded on the stream around both step
 * kernels of every stride-th step (stride 0 switches timing off; steps then
 * run without graphs).  tlsph_kernel_times synchronises on the last event
 * and returns the summed milliseconds and launch counts of the force pass
 * (index 0) and the deformation/constitutive pass (index 1), then clears
 * them.  Errors: INVALID_ARG (stride < 0), HIP. */
tlsph_status tlsph_enable_kernel_timing(tlsph_ctx *ctx, int32_t stride);
tlsph_status tlsph_kernel_times(tlsph_ctx *ctx, double ms[2], int64_t launches[2]);

/* Launch shape and layout facts: [0] threads per block of the force pass
 * (negative when the LDS-staged variant is in use), [1] of the deformation
 * pass (0: staged over the force pass's tiles; -T: staged over tiles of T
 * particles of its own), [2] neighbour pairs, [3] padded slots of the sliced neighbour layout,
 * [4] particles, [5] sticky device error flags (bit 0 non-finite, bit 1 GTN
 * Newton not converged, bit 2 a contact list missed a pair: a particle had
 * more than 32 contact candidates, left the list's skin, or the contact grid
 * outgrew 2^14 cells per axis), [6] lanes per particle of the force pass, [7] LDS
 * bytes per workgroup of the staged force pass (0 when unstaged), [8]
 * particles per tile of the staged force pass (0 when unstaged).  The flags
 * are read after the work already queued on the stream: synchronises it. */
tlsph_status tlsph_info(tlsph_ctx *ctx, int64_t out[9], hipStream_t stream);

/* Pin the launch shape (host int32[5]): [0] 1 = LDS-staged force pass, 0 =
 * gathers from global memory; [1] lanes per particle of the force pass (1,
 * 2 or 4); [2] threads per block of the unstaged force pass (64, 128, 192 or
 * 256; ignored when staged, which runs tile * lanes threads per block);
 * [3] threads per block of the deformation pass (64 to 256, multiple of 64),
 * or 0 = LDS-staged over the force pass's tiles, or -T = LDS-staged over
 * tiles of T particles of its own (64 to 256; their halo lists are built
 * into arrays of their own); [4] particles per tile of the staged force pass
 * (64 to 256; 0 = the size chosen at build, which fills whole rounds of
 * compute units).  A new tile size rebuilds the per-tile halo lists on the
 * stream and synchronises.  The staged deformation pass runs two tiles per
 * workgroup where a tile is not a multiple of 64 particles.  Every
 * shape gives bitwise identical results: the neighbour sums keep one
 * canonical order.  Errors: INVALID_ARG, BAD_STATE (before build),
 * UNSUPPORTED (staged requested where a tile and its halo do not fit in
 * LDS), HIP. */
tlsph_status tlsph_set_launch_shape(tlsph_ctx *ctx, const int32_t shape[5], hipStream_t stream);

/* Penalty contact (specimens with contact_k > 0): the candidate list of
 * each particle (particles within a_i + a_j + skin in the current
 * configuration, at most 32) is rebuilt on the stream every `every` steps;
 * between rebuilds it is valid while no particle moves more than skin / 2,
 * which the force pass checks (info flag bit 2 otherwise).  Default every = 1,
 * skin = 0: rebuilt every step, exact.  With graphs, steps with contact
 * replay graphs of twice the rebuild interval, each starting at a rebuild
 * (eager steps lead up to the first).  Errors: INVALID_ARG (every < 1, skin
 * < 0 or not finite). */
tlsph_status tlsph_set_contact(tlsph_ctx *ctx, int32_t every, double skin);

/* Run control of a batch: each specimen stops on its own, at a step cap or
 * once failed, while the others go on; a stopped specimen keeps its state
 * (later steps leave it alone; the LDS-staged passes launch over the list of
 * tiles that still hold a running specimen's particle, so stopped specimens
 * cost next to nothing).  Failure is read off the specimen's load, as the
 * tensile tests of Sec. 6 read the strain at failure off the decay of the
 * stress once damage sets in: the load is the reaction of one boundary group,
 * sign * (sum over the group's particles of one component of the nodal force
 * of Sec. 3.1 at t^n, as the force pass computes it before the prescribed
 * velocity replaces the kick), summed in a fixed order; the specimen has
 * failed after the first step whose reaction is below drop * (its running
 * peak), once that peak is positive and at least min_peak.  A step's stop
 * decision comes after the step, so a stopped specimen has taken exactly the
 * steps counted for it. */
typedef struct {
    int64_t step_cap;   /* stop after this many steps from the call (0: no cap) */
    int32_t group;      /* watched boundary group, -1: none (the cap alone) */
    int32_t axis;       /* force component 0, 1 or 2 */
    double sign;        /* +1 or -1 */
    double drop;        /* in (0, 1) */
    double min_peak;    /* >= 0 (newtons) */
} tlsph_stop_rule;

/* Set run control (rules: host tlsph_stop_rule[n_spec], read before the call
 * returns) or switch it off (rules = NULL: every specimen steps again, from
 * the state it kept).  Setting resets every specimen's step count, peak and
 * stop reason.  Steps with run control add two small kernels each (the
 * reaction and stop test, one block per specimen, and the tile list, one
 * block that returns at once unless a specimen stopped); graphs capture them
 * too.  Autotuning times the passes over every specimen and keeps the
 * control.  Building the neighbour list switches it off.  Synchronises the
 * stream.  Errors: BAD_STATE (before build), INVALID_ARG (a rule out of
 * range: step_cap < 0, group outside [-1, n_bc), axis, sign not +-1, drop
 * outside (0, 1), min_peak < 0 or not finite), HIP. */
tlsph_status tlsph_set_run_control(tlsph_ctx *ctx, const tlsph_stop_rule *rules,
                                   hipStream_t stream);

/* Run-control status after the work queued on the stream (synchronises it).
 * Host outputs, each may be NULL: why[n_spec] (0 running, 1 stopped at its
 * cap, 2 failed), steps[n_spec] (steps taken since the control was set),
 * peak[n_spec] (running peak of the reaction; 0 without a watched group),
 * n_running (specimens still running).  Errors: BAD_STATE (no run control),
 * HIP. */
tlsph_status tlsph_get_run_status(tlsph_ctx *ctx, int32_t *why, int64_t *steps, double *peak,
                                  int32_t *n_running, hipStream_t stream);

/* Step until every specimen has stopped or max_steps steps have run, reading
 * the running count every check_every steps (one synchronisation each; the
 * steps in between go as tlsph_step, graphs included).  steps_run (host, may
 * be NULL) receives the steps launched, a multiple of check_every unless
 * max_steps cut the last chunk.  Errors: BAD_STATE (no run control),
 * INVALID_ARG (max_steps < 0, check_every < 1), HIP. */
tlsph_status tlsph_run(tlsph_ctx *ctx, int64_t max_steps, int32_t check_every,
                       int64_t *steps_run, hipStream_t stream);

/* Free the host-side context (not the workspace).  Null is accepted. */
void tlsph_destroy(tlsph_ctx *ctx);

const char *tlsph_status_string(tlsph_status status);
const char *tlsph_last_error(const tlsph_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* TLSPH_H */
