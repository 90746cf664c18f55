/*
 * lbimb.h -- C ABI of the MI355X LB-IMB-DEM library (liblbimb.so).
 *
 * The library advances a lattice-Boltzmann fluid (D2Q9 or D3Q19, LBGK)
 * coupled to rigid particles by the Noble-Torczynski immersed moving boundary
 * and moved by a frictionless soft-sphere DEM, following Xiong et al.,
 * "Large-Scale DNS of Gas-Solid Flow on Mole-8.5" ("Numerical scheme",
 * Eqs. 1-5).  Every step runs on one GPU in hand-written HIP kernels.
 *
 * Conventions for every call
 *   - Return value: LBM_OK (0) or a negative LBM_E_* code.  No C++ exception
 *     crosses this boundary.  lbm_last_error() gives a message for the last
 *     failing call on a context.
 *   - Units are lattice units (lattice spacing h = 1, time step dt = 1).
 *   - Lattice fields are stored with x fastest: node n = x + nx*(y + ny*z).
 *     Populations are [Q][N], velocities [D][N], densities [N].
 *   - Particle arrays are [n][3] doubles (2D: z components are zero on output
 *     and ignored on input; the angular velocity uses component z only).
 *   - ptr_kind: LBM_HOST (0) means a host pointer; the call finishes the copy
 *     before returning.  LBM_DEVICE (1) means a device pointer on the
 *     context's GPU; the call is asynchronous on the context's stream.
 *   - Ownership: the caller owns the workspace and all input and output
 *     buffers; the library copies inputs and keeps no caller pointer except
 *     the workspace, which must stay allocated until lbm_destroy().
 *   - A context is bound to one HIP stream and is not thread-safe.
 */
#ifndef LBIMB_H
#define LBIMB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
enum {
    LBM_OK = 0,
    LBM_E_INVALID = -1,          /* bad argument or configuration */
    LBM_E_NOMEM = -2,            /* workspace too small */
    LBM_E_HIP = -3,              /* a HIP runtime call failed */
    LBM_E_NONFINITE = -4,        /* a non-finite value in the state, or a particle centre outside the box */
    LBM_E_SLOT_OVERFLOW = -5,    /* more than LBM_MAX_OWNERS particles cover one node */
    LBM_E_STATE = -6,            /* call out of order (e.g. step before particles) */
    LBM_E_IO = -7,               /* save/load file error */
    LBM_E_CELL_OVERFLOW = -8,    /* a DEM cell holds more than its capacity */
    LBM_E_CONTACT_OVERFLOW = -9  /* a particle has more than LBM_MAX_CONTACTS contacts */
};

enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1 };

/* Storage of the populations.  FP64 stores f_i; FP32_SHIFTED stores
 * g_i = f_i - w_i in binary32 and computes in binary32; FP16_STORE stores
 * g_i / w_i in binary16 and computes in binary32.  Particle forces, torques
 * and motion are binary64 in every mode. */
enum { LBM_FP64 = 0, LBM_FP32_SHIFTED = 1, LBM_FP16_STORE = 2 };

enum { LBM_HOST = 0, LBM_DEVICE = 1 };

/* Solid fraction eps of a node's cell ("Numerical scheme", Fig. 1).
 * SAMPLING: the count of S^D sub-cell sample points inside the particle.
 * TABLE: the paper's table lookup, eps = phi(d, theta) (Eq. 6): for the one
 * particle radius in use, a table of counts on the same S^D scale indexed by
 * rho = |r| - R (64 bins over [-sqrt(D)/2, sqrt(D)/2]) and by the direction
 * of r folded into the symmetric wedge (sorted component magnitudes
 * a >= b >= c; t1 = b/|r| and, in 3D, t2 = c/|r|, 16 bins each over
 * [0, 1/sqrt(2)] and [0, 1/sqrt(3)]); an entry is the coverage of the cell
 * centred at its bin centre measured with 16^D reference points, rounded to
 * the S^D scale.  Requires every particle to have the same radius R >= 1. */
enum { LBM_EPS_SAMPLING = 0, LBM_EPS_TABLE = 1 };

#define LBM_MAX_OWNERS 4      /* particles that may cover one node */
#define LBM_MAX_CONTACTS 32   /* contacts per particle per step */
#define LBM_MAX_PARTICLES 4194303

typedef struct lbm_config {
    int lattice;            /* LBM_D2Q9 or LBM_D3Q19 */
    int storage;            /* LBM_FP64, LBM_FP32_SHIFTED or LBM_FP16_STORE */
    int nx, ny, nz;         /* lattice size; nz = 1 for D2Q9 */
    int wall_y;             /* 0: periodic in y; 1: halfway bounce-back walls at
                               y = -1/2 and y = ny - 1/2.  x and z are periodic. */
    double tau;             /* BGK relaxation time, > 1/2 (Eq. 1) */
    double fluid_force[3];  /* body force per unit mass on the fluid; enters as
                               F_i = 3 w_i rho (c_i . g) (Eq. 1, term F_i) */
    double particle_accel[3]; /* acceleration of every free particle (gravity
                                 including buoyancy) */
    int eps_samples;        /* S: sub-cell sample points per axis for the solid
                               fraction eps (S^D samples per node, 1..8) */
    double kn;              /* DEM normal stiffness (Eq. 4) */
    double restitution;     /* DEM restitution coefficient e, 0 < e <= 1 (Eq. 5) */
    int max_particles;      /* capacity reserved in the workspace */
    double max_radius;      /* largest particle radius the workspace is sized for
                               (<= 0 selects 8 lattice units) */
    int eps_mode;           /* LBM_EPS_SAMPLING or LBM_EPS_TABLE */
} lbm_config;

typedef struct lbm_ctx lbm_ctx;

/* Device bytes the caller must provide for `cfg` (any alignment >= 256). */
int lbm_workspace_bytes(const lbm_config *cfg, size_t *bytes);

/* Validates `cfg` (tau > 1/2, sizes, samples), lays out the state inside
 * `workspace` (device memory of at least lbm_workspace_bytes), binds the
 * context to `hip_stream` (a hipStream_t; NULL means the null stream) and
 * sets the fluid to rest, f = f^eq(1, 0).  Errors: LBM_E_INVALID,
 * LBM_E_NOMEM, LBM_E_HIP. */
int lbm_create(const lbm_config *cfg, void *workspace, size_t ws_bytes,
               void *hip_stream, lbm_ctx **out);

void lbm_destroy(lbm_ctx *ctx);

/* Replaces the particle set (n may be 0: a fluid without particles; some
 * call of lbm_set_particles or lbm_load must precede the first lbm_step).
 * pos/vel/omega [n][3], radius/rho_s [n],
 * fixed [n] (1: the particle never moves; its force and torque are still
 * reported).  Clears the health flags a failed lbm_step left set.  Mass is rho_s pi R^2 (disc of unit depth) or rho_s 4/3 pi R^3,
 * moment of inertia m R^2 / 2 or 2 m R^2 / 5.  `fixed` may be NULL.  Host
 * pointers only for this call (ptr_kind must be LBM_HOST).  Errors:
 * LBM_E_INVALID (n > max_particles, radius <= 0 or > max_radius, a particle wider than the
 * periodic box, a centre outside the box, two particles overlapping by more
 * than half the smaller radius). */
int lbm_set_particles(lbm_ctx *ctx, int64_t n, const double *pos, const double *vel,
                      const double *omega, const double *radius, const double *rho_s,
                      const uint8_t *fixed, int ptr_kind);

/* Sets the pre-collision populations f(x, t), [Q][N] binary64, converting
 * them to the storage format. */
int lbm_set_distributions(lbm_ctx *ctx, const double *f, int ptr_kind);

/* Gets the pre-collision populations f(x, t), [Q][N] binary64 (for shifted
 * storage: w_i + g_i, or w_i + w_i h_i). */
int lbm_get_distributions(lbm_ctx *ctx, double *f, int ptr_kind);

/* Advances `nsteps` time steps.  One step: particle footprint and solid
 * fraction; fused pull streaming + LBGK/IMB collision (Eqs. 1-2); hydrodynamic
 * force and torque per particle (Eq. 3); DEM contacts (Eqs. 4-5); symplectic
 * Euler update of the particles.  Returns after the work is queued and the
 * health flags are read back (which synchronises the stream).  The flags
 * stay set once raised: after an error the state is not a valid step of the
 * method, and every later lbm_step reports the same error until
 * lbm_set_particles or lbm_load replaces the state.
 * Errors: LBM_E_STATE (no lbm_set_particles or lbm_load yet),
 * LBM_E_SLOT_OVERFLOW, LBM_E_CELL_OVERFLOW, LBM_E_CONTACT_OVERFLOW,
 * LBM_E_NONFINITE, LBM_E_HIP. */
int lbm_step(lbm_ctx *ctx, int64_t nsteps);

/* Hydrodynamic force and torque on each particle from the last completed
 * step, [n][3] binary64 (Eq. 3, sign: force exerted by the fluid on the
 * particle). */
int lbm_get_forces(lbm_ctx *ctx, double *F, double *T, int ptr_kind);

/* DEM contact force on each particle from the last completed step, [n][3]. */
int lbm_get_contact_forces(lbm_ctx *ctx, double *Fc, int ptr_kind);

/* Particle state at the current time, [n][3] each. */
int lbm_get_particles(lbm_ctx *ctx, double *pos, double *vel, double *omega, int ptr_kind);

/* Moments of the pre-collision populations f(x, t): rho [N] and
 * u [D][N] = sum_i f_i c_i / rho, binary64 in every storage mode. */
int lbm_get_macro(lbm_ctx *ctx, double *rho, double *u, int ptr_kind);

/* IMB momentum exchange q_n = beta_n sum_i Omega^S_i c_i of the last step,
 * [D][N] binary64; zero where no particle covers the node. */
int lbm_get_q(lbm_ctx *ctx, double *q, int ptr_kind);

/* Number of completed time steps. */
int64_t lbm_time(const lbm_ctx *ctx);

/* Number of particles currently set (after lbm_set_particles or lbm_load). */
int64_t lbm_particle_count(const lbm_ctx *ctx);

/* Per-phase kernel timing.  enable: 0 off, 1 every phase, 2 the lattice
 * phase only (least perturbation of the step).  While enabled, lbm_step
 * launches the step kernels one by one (no graph) with HIP events around the
 * timed phases on the stream each phase runs on; lbm_get_timing synchronises
 * and returns the summed milliseconds and the number of launches of each phase
 * since timing was enabled.  Phases: 0 footprint, 1 lattice
 * (stream-collide-IMB), 2 hydrodynamic force and integration, 3 cell list,
 * 4 DEM contacts, 5 unused (integration runs inside phase 2).  Errors:
 * LBM_E_INVALID for another `enable`. */
#define LBM_NPHASES 6
int lbm_set_timing(lbm_ctx *ctx, int enable);
int lbm_get_timing(lbm_ctx *ctx, double *ms, int64_t *launches);

/* Launch shape of the lattice kernel (the update of Eq. 1 with the
 * immersed-boundary terms of Eq. 2).  threads: the workgroup width along x,
 * one workgroup covering all or part of one lattice row; 0 selects the
 * built-in rule (the whole row when nx <= 256, else 256 threads), otherwise
 * 64, 128, 192 or 256 (the end of a row that the last workgroup overhangs is
 * masked).  order: LBM_ORDER_LINEAR hands tiles to workgroups in launch
 * order; LBM_ORDER_XCD renumbers workgroups so that each of the GPU's 8
 * XCDs (which the hardware feeds workgroup ids in turn) takes one contiguous
 * run of tiles, keeping neighbouring rows in one L2.  cu_groups: 0, or at
 * most 3..8 of the kernel's workgroups resident on one CU at a time (the
 * launch reserves 160 KiB / cu_groups of LDS, rounded down to 512 bytes,
 * that the kernel does not use).
 * The launch shape never changes a bit of the result.  Takes effect from the
 * next step (captured step graphs are dropped).  A new context starts with
 * width 0, linear order and no cap.  Errors: LBM_E_INVALID for another
 * width, order or cap, or for XCD order on a grid of 2^32 workgroups or
 * more.  lbm_get_lattice_block writes the width in use (the rule resolved),
 * the order and the cap; LBM_E_INVALID for a null argument. */
enum { LBM_ORDER_LINEAR = 0, LBM_ORDER_XCD = 1 };
int lbm_set_lattice_block(lbm_ctx *ctx, int threads, int order, int cu_groups);
int lbm_get_lattice_block(const lbm_ctx *ctx, int *threads, int *order, int *cu_groups);

/* DEM neighbour search ("Parallel implementation": a neighbour list rebuilt
 * about every 100th step, after Xu et al.).  every = 0 (a new context's
 * default): the cell list is rebuilt every step and the contacts gathered from
 * it.  every >= 1: each particle keeps the list of the particles within
 * R_i + R_j + skin of it (minimum image) at the last build; the list is rebuilt
 * on the device when `every` steps have passed since the build, or earlier
 * when some particle has moved 0.49 skin or more since the build (the
 * displacement guard: a pair missing from the lists cannot touch before
 * that), and at the first step after lbm_set_particles, lbm_load or this call.
 * Contacts then sum the touching listed neighbours in ascending id, as the
 * per-step search does: both modes give the same bits.  The cell edge becomes
 * 2 R_max + skin.  A list holds at most 2 LBM_MAX_CONTACTS entries
 * (LBM_E_CONTACT_OVERFLOW beyond).  Takes effect from the next step.  Errors:
 * LBM_E_INVALID (every < 0; skin outside (0, 2 max_radius] when every >= 1;
 * the cell grid would exceed the reserved budget). */
int lbm_set_neighbour_list(lbm_ctx *ctx, int every, double skin);

/* The neighbour-search mode in force and, in builds (may be NULL), the number
 * of list builds so far (synchronises). */
int lbm_get_neighbour_list(lbm_ctx *ctx, int *every, double *skin, int64_t *builds);

/* Slab pipeline (lattices with walls in y and particles).  Every step of the
 * method chains footprint -> lattice update (Eqs. 1-2) -> force and torque
 * sums (Eq. 3) -> integration -> next footprint.  With K slabs the lattice
 * update of a step runs slab by slab in y, and the particles whose footprint
 * lies in slabs g - 1 .. g (with one node of margin for the step's motion)
 * take their force sums, integration and next footprint on the side stream
 * as soon as slab g is done, while the later slabs update; the next step's
 * slab k waits only for groups k and k + 1.  Every particle and node runs the
 * same arithmetic as in the plain step, so the results are the same bits.
 * slabs: 1 off (a new context's default: on MI355X the overlapped particle
 * kernels slow the lattice kernel by more than they hide), 0 automatic (4),
 * 2..8 requested.  In use are at most as many slabs as keep every slab at
 * least 2 R_max + 5 rows high, and one (the plain step) without walls in y or
 * particles; lbm_get_pipeline gives the number in use.  Pipelined steps are
 * launched one by one (never captured as a graph).  The pipeline needs every
 * particle to move at most one node in y per step: a faster one raises
 * LBM_E_NONFINITE at the step.  Errors: LBM_E_INVALID (slabs outside 0..8). */
int lbm_set_pipeline(lbm_ctx *ctx, int slabs);
int lbm_get_pipeline(const lbm_ctx *ctx, int *slabs);

/* Chooses the lattice kernel's launch shape by measurement.  Each of the 24
 * candidates (width 64, 128, 192, 256 for k % 4 = 0..3, order (k / 4) % 2,
 * cap 0, 4, 3 workgroups per CU for k / 8 = 0..2; XCD candidates skipped
 * where the grid is too large for them) runs 1 + `steps` real time steps
 * twice, so the simulation advances by up to 48 (1 + steps) steps; the result
 * does not depend on the shape.  The lattice phase is timed as in timing
 * mode 2, and the candidate with the shortest mean lattice kernel time is
 * kept.  best_threads, best_order and best_cu_groups (each may be null)
 * receive it; ms_out (24 doubles, may be null) the mean milliseconds per
 * lattice launch of each candidate (the faster of the two passes; HUGE_VAL
 * for a skipped one).  The timing mode in force before the call is restored
 * with its counters cleared.  Errors: LBM_E_INVALID for steps outside
 * 1..100000; a failed step returns its code with the previous shape and
 * timing mode restored. */
int lbm_autotune_lattice_block(lbm_ctx *ctx, int steps, int *best_threads, int *best_order,
                               int *best_cu_groups, double *ms_out);

/* Writes / reads the full state (populations in storage format, particles,
 * forces, time) to / from a file.  The file records the configuration.
 * lbm_load reads and checks the whole file before it changes anything: a
 * file of another configuration or with particles that lbm_set_particles
 * would reject gives LBM_E_INVALID, a short, overlong or unreadable file
 * LBM_E_IO, and in both cases the context keeps its state.  A loaded state
 * rebuilds the DEM cell grid from its radii and starts with clear health
 * flags. */
int lbm_save(lbm_ctx *ctx, const char *path);
int lbm_load(lbm_ctx *ctx, const char *path);

/* Suspension-wide sums of the current state ("Simulation results": the
 * temporal evolution of the area-averaged inter-phase slip velocity and of the
 * drag, Figs. 5 and 7).  Node sums run over the pre-collision populations
 * f(x, t); eps_n is the solid fraction of the last completed step's footprint
 * (zero everywhere before the first step).  Reductions have a fixed order,
 * so a state gives the same bits every time.  Synchronises the stream. */
typedef struct lbm_stats {
    int64_t t;                      /* completed time steps */
    int64_t np;                     /* particles */
    int64_t nodes;                  /* lattice nodes N */
    double mass;                    /* sum_n rho_n */
    double fluid_momentum[3];       /* sum_n sum_i c_i f_i */
    double solid_fraction;          /* sum_n eps_n / N */
    double fluid_velocity[3];       /* fluid phase: sum_n (1 - eps_n) j_n / sum_n (1 - eps_n) rho_n */
    double particle_momentum[3];    /* sum_p m_p v_p */
    double particle_velocity[3];    /* sum_p m_p v_p / sum_p m_p */
    double mean_particle_velocity[3]; /* (1/np) sum_p v_p */
    double slip_velocity[3];        /* fluid_velocity - particle_velocity */
    double mean_drag[3];            /* (1/np) sum_p F^h_p of the last step (Eq. 3) */
} lbm_stats;

int lbm_get_stats(lbm_ctx *ctx, lbm_stats *out);

/* ------------------------------------------------ batched drag ensemble
 * Many small fully periodic cubic D3Q19 boxes, each with fixed equal spheres
 * and its own tau and fluid body force, advanced together in shifted FP32
 * storage (drag-data generation).  The per-node arithmetic is that of
 * lbm_step with LBM_FP32_SHIFTED and particles at rest, so a box gives the
 * same bits in a batch as alone.  Sphere footprints are computed once at
 * creation (sub-cell sampling with eps_samples per axis). */
typedef struct lbm_box {
    int edge;                /* box edge L (L x L x L nodes), 2R + 2 <= L */
    double tau;              /* > 1/2 */
    double fluid_force[3];   /* body force per unit mass on the fluid */
    int nspheres;            /* >= 0 */
    const double *pos;       /* [nspheres][3], centres in [0, L) */
    double radius;           /* sphere radius R */
    double init_velocity[3]; /* uniform fluid velocity of the initial state,
                                f = f^eq(1, init_velocity); |u| <= 0.2 */
} lbm_box;

typedef struct lbm_batch lbm_batch;

enum { LBM_BATCH_PER_STEP = 0, LBM_BATCH_PERSISTENT = 1 };

int lbm_batch_workspace_bytes(const lbm_box *boxes, int nbox, int eps_samples, size_t *bytes);

/* Copies the box descriptions (sphere positions included), computes the
 * footprints and sets every box to its initial state (uniform density 1 and
 * velocity init_velocity, rest when zero).  Errors: LBM_E_INVALID, LBM_E_NOMEM,
 * LBM_E_HIP, LBM_E_SLOT_OVERFLOW (a node covered by more than 4 spheres). */
int lbm_batch_create(const lbm_box *boxes, int nbox, int eps_samples, void *workspace,
                     size_t ws_bytes, void *hip_stream, lbm_batch **out);
void lbm_batch_destroy(lbm_batch *b);

/* Tile shape: lattice rows (of L nodes) per workgroup for the boxes of the
 * given edge; rows must divide L*L. */
int lbm_batch_set_tile_rows(lbm_batch *b, int edge, int rows);

/* Advances every active box by nsteps, either with one launch per step
 * (LBM_BATCH_PER_STEP) or with one persistent launch (LBM_BATCH_PERSISTENT).
 * Synchronises and checks the error flags.  Errors: LBM_E_HIP, LBM_E_STATE
 * (a persistent wait hit its bound). */
int lbm_batch_run(lbm_batch *b, int64_t nsteps, int mode);

/* Advances the active boxes until each one's drag is steady, at most
 * max_steps steps.  Every check_every steps (the last chunk may be shorter)
 * the device computes the hydrodynamic forces (Eq. 3) and, for each active box
 * with spheres, retires it when max over its spheres and components of
 * |F - F_prev| < tol * (mean over its spheres of |F|), F_prev being the force
 * at the previous check of this call (the first check only records it).
 * Boxes without spheres never retire.  The check runs on the device; the host
 * reads one integer per check (the active boxes left) and stops when it is
 * zero.  Full chunks are replayed as a captured HIP graph (check_every steps in
 * `mode`, the forces and the check).  steady[nbox] (may be NULL) receives 1 for
 * the boxes this call retired; stop_step[nbox] (may be NULL) the batch time
 * (lbm_batch_time) at which each box stopped: its retiring check, the call's
 * end for boxes still active, the call's start for boxes retired before.
 * Host pointers; synchronises.  Errors: LBM_E_INVALID (max_steps < 0,
 * check_every < 1, tol not positive and finite, another mode), LBM_E_HIP,
 * LBM_E_STATE (a persistent wait hit its bound). */
int lbm_batch_run_steady(lbm_batch *b, int64_t max_steps, double tol, int check_every, int mode,
                         uint8_t *steady, int64_t *stop_step);

/* Per-sphere drag data of the current state, spheres in box order (the
 * closure's training and evaluation rows; "Simulation results" relates the
 * drag to slip velocity and solid fraction).  F [total][3] binary64: the
 * hydrodynamic force of the last step (as lbm_batch_forces).  feat
 * [total][40] binary32, computed on the device in binary64 and rounded:
 *   0      spheres other than this one with minimum-image centre distance
 *          below 3R, over 27
 *   1      log10 max(Re, 1e-6), Re = |U| 2R / nu, U the box's superficial
 *          mean velocity (lbm_batch_mean_velocity), nu = (tau - 1/2) / 3
 *   2..4   the shell velocity (lbm_batch_shell_velocity) over |U|, in the frame
 *          e_x = U / |U|, e_y = e_x x z-hat normalised (e_x x y-hat when that
 *          is shorter than 1e-8), e_z = e_x x e_y
 *   5..36  the 16 nearest other spheres by distance (ties: lower index first),
 *          each as (offset along e_x, distance across e_x) over 2R; slots
 *          beyond the box's other spheres hold L / 2R
 *   37     box solid fraction n (4/3) pi R^3 / L^3
 *   38     2R / L
 *   39     nearest surface gap (min distance - 2R) / 2R, or L / 2R for a
 *          single sphere
 * Either output may be NULL.  Synchronises.  Errors: LBM_E_INVALID (bad
 * ptr_kind; feat requested with a box of more than 64 spheres), LBM_E_HIP. */
int lbm_batch_get_drag(lbm_batch *b, double *F, float *feat, int ptr_kind);

/* Boxes with active[b] == 0 are no longer advanced (retired). */
int lbm_batch_set_active(lbm_batch *b, const uint8_t *active);

/* Hydrodynamic force and torque on every sphere from the last step, spheres
 * numbered box by box in input order, [total][3] binary64 (Eq. 3). */
int lbm_batch_forces(lbm_batch *b, double *F, double *T, int ptr_kind);

/* Superficial mean fluid velocity (1/N) sum_n sum_i f_i c_i of every box,
 * [nbox][3] binary64. */
int lbm_batch_mean_velocity(lbm_batch *b, double *U, int ptr_kind);

/* Local flow seen by each sphere: the mean pre-collision fluid velocity
 * (sum_i c_i f_i) / (sum_i f_i) over the nodes with no sub-cell sample of any
 * sphere whose minimum-image distance to the sphere centre lies in [R + 1, 2R];
 * [nspheres][3] binary64, spheres in box order.  Errors: LBM_E_INVALID,
 * LBM_E_HIP. */
int lbm_batch_shell_velocity(lbm_batch *b, double *u, int ptr_kind);

/* Pre-collision populations f_i = w_i + g_i of one box, [19][L^3] binary64. */
int lbm_batch_get_distributions(lbm_batch *b, int box, double *f, int ptr_kind);

/* Times every tile shape (rows 1, 2, 4, 8, 16) for each edge present and
 * both run modes over `steps` steps, keeps the fastest, and returns the boxes
 * to rest at time 0.  rows_out[k] and ms_out[k] (may be NULL) receive, for the
 * k-th distinct edge in ascending order, the chosen rows and the step time. */
int lbm_batch_autotune(lbm_batch *b, int steps, int *edges_out, int *rows_out, int *mode_out,
                       double *ms_per_step_out);

int64_t lbm_batch_time(const lbm_batch *b);

const char *lbm_error_string(int code);
const char *lbm_last_error(const lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBIMB_H */
