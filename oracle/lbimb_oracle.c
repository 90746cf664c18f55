/*
 * lbimb_oracle.c -- plain, slow, FP64 CPU oracle of the LB-IMB-DEM step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP library: every formula below is written out here from the paper
 * (Xiong et al., "Large-Scale DNS of Gas-Solid Flow on Mole-8.5"):
 *
 *   - LBGK with the Noble-Torczynski immersed moving boundary, Eq. (1)
 *   - weighting function beta(eps, tau), Eq. (2)
 *   - solid collision operator Omega^S (the unnumbered line after Eq. (2))
 *   - solid fraction eps of a lattice cell ("Numerical scheme", Fig. 1 text)
 *   - hydrodynamic force and torque sums, Eq. (3)
 *   - frictionless linear spring-dashpot DEM, Eqs. (4)-(5)
 *   - D2Q9 / D3Q19 lattices ("Numerical scheme", first paragraph)
 *
 * Readings where the paper is silent or garbled (all listed in the design
 * notes of the repository):
 *   - equilibrium: standard second-order LBGK form, c_s^2 = 1/3;
 *   - body force: F_i = 3 w_i rho (c_i . g), u excludes any half-force shift;
 *   - eps by sub-cell sampling, S points per axis at offsets (k+1/2)/S - 1/2,
 *     inside test dx^2+dy^2(+dz^2) <= R^2, eps = min(count, S^D) / S^D;
 *   - eps by table lookup (Eq. 6, gamma = phi(d, theta)), the alternative the
 *     paper ran on its GPUs: for one particle radius a table holds the count
 *     on the S^D scale as a function of rho = |r| - R (r the node-minus-centre
 *     displacement) and of the direction of r folded into the symmetric wedge
 *     (sorted magnitudes a >= b >= c of its components, t1 = b/|r|,
 *     t2 = c/|r|); see eps_table_build for the bins and the reference counts;
 *   - several particles on a node: one eps from the summed count, V_S the
 *     count-weighted mean of the owners' rigid-body velocities (ascending
 *     particle id), force shares count_pn / count_n;
 *   - V_S = v_p + omega_p x (x_n - x_p), minimum image;
 *   - Eq. (3) gives the momentum the fluid gains; the force on the particle
 *     is its negative; 3D uses the same sum over i = 1..18; h = dt = 1;
 *   - Eq. (5): overlap delta = R_i + R_j - |r_ij| (the printed R_i - R_j is
 *     a typo), repulsive force (k delta - eta v_n) n_ij on i, and the printed
 *     "eta_n" expression is the contact time; the damping that gives
 *     restitution e is eta = -2 ln(e) sqrt(m_eff k) / sqrt(pi^2 + ln^2 e);
 *   - walls (y only): halfway bounce-back at y = -1/2 and y = ny - 1/2, the
 *     same contact law against the wall with m_eff = m_i;
 *   - time integration: symplectic Euler, dt = 1, forces at t from state at t;
 *   - sums of per-node force contributions use compensated summation
 *     (Ogita, Rump & Oishi 2005, "Sum2") so their rounding does not depend on
 *     summation order.
 *
 * Floating point: IEEE binary64, round to nearest even, compiled with
 * -ffp-contract=off and no fast-math.  Every expression is evaluated left to
 * right exactly as written.
 *
 * Threads (OpenMP, optional): the per-node loops (footprint, collision,
 * streaming, moments) and the per-particle loops (force sums, contacts,
 * integration) are split over threads without changing any result.  Every
 * node and every particle is still computed by exactly the same arithmetic
 * in the same order; in particular the footprint gives each thread a slab of
 * the outermost lattice axis and every thread walks the particles in
 * ascending id, so each node still accumulates its owners in ascending id.
 * orc_set_threads(1) gives the plain serial program.  Loops over fewer
 * nodes or particles than the parallel minimum (orc_set_parallel_minimum)
 * stay on the calling thread, where a parallel region would cost more than
 * the work.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.141592653589793

/* loops smaller than these run on the calling thread */
static long par_min_nodes = 32768;
static long par_min_particles = 256;

/* ---------------------------------------------------------------- lattices */
/* D2Q9: 0 rest; 1..4 axis; 5..8 diagonals. */
static const int d2q9_c[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const int d2q9_opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* D3Q19: 0 rest; 1..6 axis pairs; 7..18 face diagonals, in +/- pairs. */
static const int d3q19_c[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const int d3q19_opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9,
                                  12, 11, 14, 13, 16, 15, 18, 17};

typedef struct {
    int D, Q;
    const int (*c)[3];
    const int *opp;
    double w[19];
} orc_lattice;

static void lattice_init(orc_lattice *L, int dim) {
    if (dim == 2) {
        L->D = 2; L->Q = 9; L->c = d2q9_c; L->opp = d2q9_opp;
        L->w[0] = 4.0 / 9.0;
        for (int i = 1; i <= 4; i++) L->w[i] = 1.0 / 9.0;
        for (int i = 5; i <= 8; i++) L->w[i] = 1.0 / 36.0;
    } else {
        L->D = 3; L->Q = 19; L->c = d3q19_c; L->opp = d3q19_opp;
        L->w[0] = 1.0 / 3.0;
        for (int i = 1; i <= 6; i++) L->w[i] = 1.0 / 18.0;
        for (int i = 7; i <= 18; i++) L->w[i] = 1.0 / 36.0;
    }
}

/* ------------------------------------------------------------------ state */
typedef struct orc_sim {
    orc_lattice L;
    int nx, ny, nz;
    long N;
    int wall_y;          /* 1: halfway bounce-back walls in y; x (and z) periodic */
    double tau;
    double gf[3];        /* fluid body force per unit mass */
    double ap[3];        /* particle acceleration (gravity incl. buoyancy) */
    int S;               /* sub-samples per axis for eps */
    int eps_mode;        /* 0: sub-cell sampling, 1: table lookup (Eq. 6) */
    int *tab;            /* lookup table (eps_mode 1), for radius tab_R */
    double tab_R;
    double kn, restitution, ce; /* ce = -2 ln e / sqrt(pi^2 + ln^2 e) */
    int couple;          /* 0: hydrodynamic force on particles switched off */

    double *f;           /* pre-collision f(x,t), [Q][N] */
    double *fs;          /* post-collision scratch, [Q][N] */
    int *ctot;           /* total sub-sample count per node */
    double *vnum;        /* [3][N] count-weighted rigid velocity sums */
    double *q;           /* [3][N] q_n = beta * sum_i Omega_i c_i */

    int np;
    double *x, *v, *om;  /* [np][3] */
    double *R, *rhos, *m, *I;
    unsigned char *fixed;
    double *Fh, *Th, *Fc; /* [np][3], last completed step */
    long t;
} orc_sim;

static long node_index(const orc_sim *s, int x, int y, int z) {
    return (long)x + (long)s->nx * ((long)y + (long)s->ny * (long)z);
}

/* Minimum-image displacement along a periodic axis of length Lp. */
static double min_image(double d, double Lp) {
    if (d > 0.5 * Lp) d = d - Lp;
    else if (d < -0.5 * Lp) d = d + Lp;
    return d;
}

/* Displacement x_n - x_p along axis a, minimum image on periodic axes. */
static double node_disp(const orc_sim *s, int a, int coord, double xp) {
    double d = (double)coord - xp;
    if (a == 0) return min_image(d, (double)s->nx);
    if (a == 1) return s->wall_y ? d : min_image(d, (double)s->ny);
    return min_image(d, (double)s->nz);
}

/* ------------------------------------------------------------ equilibrium */
/* f^eq_i(rho,u) = w_i rho (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u) */
static double feq_i(const orc_lattice *L, int i, double rho, const double u[3]) {
    double cu = (double)L->c[i][0] * u[0] + (double)L->c[i][1] * u[1];
    double usq = u[0] * u[0] + u[1] * u[1];
    if (L->D == 3) {
        cu = cu + (double)L->c[i][2] * u[2];
        usq = usq + u[2] * u[2];
    }
    return L->w[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
}

/* Body-force term F_i = 3 w_i rho (c_i . g). */
static double force_i(const orc_lattice *L, int i, double rho, const double g[3]) {
    double cg = (double)L->c[i][0] * g[0] + (double)L->c[i][1] * g[1];
    if (L->D == 3) cg = cg + (double)L->c[i][2] * g[2];
    return 3.0 * L->w[i] * rho * cg;
}

/* Eq. (2). */
static double beta_of_eps(double eps, double tau) {
    return eps * (tau - 0.5) / ((1.0 - eps) + (tau - 0.5));
}

/* ------------------------------------------------------------- Sum2 (ORO) */
static void two_sum(double a, double b, double *s, double *e) {
    double x = a + b;
    double bb = x - a;
    *e = (a - (x - bb)) + (b - bb);
    *s = x;
}

typedef struct { double s, c; } orc_acc;

static void acc_add(orc_acc *A, double p) {
    double s, e;
    two_sum(A->s, p, &s, &e);
    A->s = s;
    A->c = A->c + e;
}

static double acc_value(const orc_acc *A) { return A->s + A->c; }

/* ------------------------------------------------------- particle geometry */
static void particle_bbox(const orc_sim *s, int p, int lo[3], int hi[3]) {
    for (int a = 0; a < 3; a++) {
        if (a == 2 && s->L.D == 2) { lo[a] = 0; hi[a] = 0; continue; }
        double c = s->x[3 * p + a];
        double r = s->R[p];
        lo[a] = (int)ceil(c - r - 0.5);
        hi[a] = (int)floor(c + r + 0.5);
    }
}

/* Wrap an unwrapped node coordinate into the box; returns -1 if the node
 * lies beyond a wall (such cells do not exist). */
static int wrap_coord(const orc_sim *s, int a, int c) {
    int n = a == 0 ? s->nx : (a == 1 ? s->ny : s->nz);
    if (a == 1 && s->wall_y) return (c < 0 || c >= n) ? -1 : c;
    c %= n;
    if (c < 0) c += n;
    return c;
}

/* Number of sub-sample points of node (ix,iy,iz) inside particle p. */
static int sample_count(const orc_sim *s, int p, int ix, int iy, int iz) {
    const int S = s->S;
    double R2 = s->R[p] * s->R[p];
    double d0 = node_disp(s, 0, ix, s->x[3 * p + 0]);
    double d1 = node_disp(s, 1, iy, s->x[3 * p + 1]);
    double d2 = s->L.D == 3 ? node_disp(s, 2, iz, s->x[3 * p + 2]) : 0.0;
    int count = 0;
    int kzmax = s->L.D == 3 ? S : 1;
    for (int kz = 0; kz < kzmax; kz++)
        for (int ky = 0; ky < S; ky++)
            for (int kx = 0; kx < S; kx++) {
                double ox = ((double)kx + 0.5) / (double)S - 0.5;
                double oy = ((double)ky + 0.5) / (double)S - 0.5;
                double dx = d0 + ox;
                double dy = d1 + oy;
                double r2 = dx * dx + dy * dy;
                if (s->L.D == 3) {
                    double oz = ((double)kz + 0.5) / (double)S - 0.5;
                    double dz = d2 + oz;
                    r2 = r2 + dz * dz;
                }
                if (r2 <= R2) count++;
            }
    return count;
}

/* ------------------------------------------------ eps by table lookup (Eq. 6)
 * A node's cell is the unit square/cube centred on it.  With H = sqrt(D)/2
 * (half its diagonal), the cell is wholly inside the particle when
 * rho = |r| - R <= -H and wholly outside when rho >= H.  In between,
 * rho falls in one of TAB_NRHO bins of width 2H/TAB_NRHO, t1 = b/|r| in
 * [0, 1/sqrt(2)] in one of TAB_NT bins (index floor(t1 * sqrt(2) * TAB_NT)),
 * and in 3D t2 = c/|r| in [0, 1/sqrt(3)] likewise (floor(t2 * sqrt(3) * TAB_NT)).
 * The entry of a bin is the coverage of the cell whose centre sits at the bin
 * centre (|r| = R + rho_c, components (a, b, c) = (sqrt(|r|^2 - b^2 - c^2),
 * t1_c |r|, t2_c |r|)), measured with TAB_M^D reference points at offsets
 * (k+1/2)/TAB_M - 1/2 and the inside test of the sampling rule, and put on
 * the S^D scale by integer rounding: (k_in S^D + TAB_M^D/2) / TAB_M^D. */
#define TAB_NRHO 64
#define TAB_NT 16
#define TAB_M 16

static int eps_table_len(int D) { return TAB_NRHO * TAB_NT * (D == 3 ? TAB_NT : 1); }

static void eps_table_build(int D, int S, double R, int *tab) {
    const double H = sqrt((double)D) * 0.5;
    const double wr = 2.0 * H / (double)TAB_NRHO;
    const double k1 = sqrt(2.0) * (double)TAB_NT, k2 = sqrt(3.0) * (double)TAB_NT;
    const long Smax = D == 3 ? (long)S * S * S : (long)S * S;
    const long Mtot = D == 3 ? (long)TAB_M * TAB_M * TAB_M : (long)TAB_M * TAB_M;
    const double R2 = R * R;
    const int n2 = D == 3 ? TAB_NT : 1;
    for (int ir = 0; ir < TAB_NRHO; ir++)
        for (int i1 = 0; i1 < TAB_NT; i1++)
            for (int i2 = 0; i2 < n2; i2++) {
                double rn = R + (-H + ((double)ir + 0.5) * wr);
                double b = ((double)i1 + 0.5) / k1 * rn;
                double c = D == 3 ? ((double)i2 + 0.5) / k2 * rn : 0.0;
                double a2 = rn * rn - b * b - c * c;
                double a = a2 > 0.0 ? sqrt(a2) : 0.0;
                long kin = 0;
                int mz = D == 3 ? TAB_M : 1;
                for (int kz = 0; kz < mz; kz++)
                    for (int ky = 0; ky < TAB_M; ky++)
                        for (int kx = 0; kx < TAB_M; kx++) {
                            double dx = a + (((double)kx + 0.5) / (double)TAB_M - 0.5);
                            double dy = b + (((double)ky + 0.5) / (double)TAB_M - 0.5);
                            double r2 = dx * dx + dy * dy;
                            if (D == 3) {
                                double dz = c + (((double)kz + 0.5) / (double)TAB_M - 0.5);
                                r2 = r2 + dz * dz;
                            }
                            if (r2 <= R2) kin++;
                        }
                tab[(ir * TAB_NT + i1) * n2 + i2] = (int)((kin * Smax + Mtot / 2) / Mtot);
            }
}

/* Count on the S^D scale of a node at displacement (d0, d1, d2) from the
 * centre of a particle of radius R (the table's radius). */
static int eps_table_lookup(int D, int S, double R, const int *tab, double d0, double d1, double d2) {
    const double H = sqrt((double)D) * 0.5;
    const double wr = 2.0 * H / (double)TAB_NRHO;
    const double k1 = sqrt(2.0) * (double)TAB_NT, k2 = sqrt(3.0) * (double)TAB_NT;
    const int Smax = D == 3 ? S * S * S : S * S;
    double r2 = d0 * d0 + d1 * d1;
    if (D == 3) r2 = r2 + d2 * d2;
    double r = sqrt(r2);
    double rho = r - R;
    if (rho <= -H) return Smax;
    if (rho >= H) return 0;
    int ir = (int)floor((rho + H) / wr);
    if (ir < 0) ir = 0;
    if (ir > TAB_NRHO - 1) ir = TAB_NRHO - 1;
    /* sorted magnitudes a >= b >= c */
    double a = fabs(d0), b = fabs(d1), c = D == 3 ? fabs(d2) : 0.0, t;
    if (b > a) { t = a; a = b; b = t; }
    if (c > b) { t = b; b = c; c = t; }
    if (b > a) { t = a; a = b; b = t; }
    (void)a;
    int i1 = (int)floor(b / r * k1);
    if (i1 > TAB_NT - 1) i1 = TAB_NT - 1;
    if (D == 2) return tab[ir * TAB_NT + i1];
    int i2 = (int)floor(c / r * k2);
    if (i2 > TAB_NT - 1) i2 = TAB_NT - 1;
    return tab[(ir * TAB_NT + i1) * TAB_NT + i2];
}

/* Count of particle p on node (ix,iy,iz) in the selected eps mode. */
static int node_count(const orc_sim *s, int p, int ix, int iy, int iz) {
    if (s->eps_mode == 0) return sample_count(s, p, ix, iy, iz);
    double d0 = node_disp(s, 0, ix, s->x[3 * p + 0]);
    double d1 = node_disp(s, 1, iy, s->x[3 * p + 1]);
    double d2 = s->L.D == 3 ? node_disp(s, 2, iz, s->x[3 * p + 2]) : 0.0;
    return eps_table_lookup(s->L.D, s->S, s->R[p], s->tab, d0, d1, d2);
}

/* ------------------------------------------------------------- lifecycle */
orc_sim *orc_create(int dim, int nx, int ny, int nz, int wall_y, double tau,
                    const double *gf, const double *ap, int samples,
                    double kn, double restitution) {
    if ((dim != 2 && dim != 3) || nx < 1 || ny < 1 || nz < 1 || tau <= 0.5 || samples < 1)
        return NULL;
    if (dim == 2 && nz != 1) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    lattice_init(&s->L, dim);
    s->nx = nx; s->ny = ny; s->nz = nz;
    s->N = (long)nx * ny * nz;
    s->wall_y = wall_y;
    s->tau = tau;
    for (int a = 0; a < 3; a++) { s->gf[a] = gf[a]; s->ap[a] = ap[a]; }
    s->S = samples;
    s->kn = kn;
    s->restitution = restitution;
    double le = log(restitution);
    s->ce = -2.0 * le / sqrt(ORC_PI * ORC_PI + le * le);
    s->couple = 1;
    long QN = (long)s->L.Q * s->N;
    s->f = (double *)malloc(sizeof(double) * QN);
    s->fs = (double *)malloc(sizeof(double) * QN);
    s->ctot = (int *)malloc(sizeof(int) * s->N);
    s->vnum = (double *)malloc(sizeof(double) * 3 * s->N);
    s->q = (double *)calloc(3 * s->N, sizeof(double));
    if (!s->f || !s->fs || !s->ctot || !s->vnum || !s->q) {
        free(s->f); free(s->fs); free(s->ctot); free(s->vnum); free(s->q); free(s);
        return NULL;
    }
    /* fluid at rest: f = f^eq(1, 0) */
    double u0[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < s->L.Q; i++) {
        double fe = feq_i(&s->L, i, 1.0, u0);
#pragma omp parallel for schedule(static) if (s->N >= par_min_nodes)
        for (long n = 0; n < s->N; n++) s->f[(long)i * s->N + n] = fe;
    }
    return s;
}

static void free_particles(orc_sim *s) {
    free(s->x); free(s->v); free(s->om); free(s->R); free(s->rhos);
    free(s->m); free(s->I); free(s->fixed); free(s->Fh); free(s->Th); free(s->Fc);
    s->x = s->v = s->om = s->R = s->rhos = s->m = s->I = NULL;
    s->Fh = s->Th = s->Fc = NULL;
    s->fixed = NULL;
    s->np = 0;
}

void orc_destroy(orc_sim *s) {
    if (!s) return;
    free_particles(s);
    free(s->f); free(s->fs); free(s->ctot); free(s->vnum); free(s->q); free(s->tab);
    free(s);
}

void orc_set_coupling(orc_sim *s, int couple) { s->couple = couple; }

static int nx_of(const orc_sim *s) { return s->nx; }

/* Particle arrays are [np][3]; 2D ignores z and uses omega[.][2] only.
 * Mass: rho_s pi R^2 (disc of unit depth) or rho_s (4/3) pi R^3;
 * moment of inertia: m R^2 / 2 (disc) or 2 m R^2 / 5 (sphere). */
int orc_set_eps_mode(orc_sim *s, int mode);

int orc_set_particles(orc_sim *s, int np, const double *pos, const double *vel,
                      const double *omega, const double *radius,
                      const double *rho_s, const unsigned char *fixed) {
    free_particles(s);
    if (np < 0) return -1;
    for (int p = 0; p < np; p++) {
        /* the bounding box of a particle must not wrap onto itself */
        double span = 2.0 * radius[p] + 2.0;
        if (!(radius[p] > 0.0) || span > (double)nx_of(s) ||
            (!s->wall_y && span > (double)s->ny) || (s->L.D == 3 && span > (double)s->nz))
            return -1;
    }
    s->np = np;
    size_t n3 = (size_t)(np > 0 ? np : 1) * 3;
    size_t n1 = (size_t)(np > 0 ? np : 1);
    s->x = (double *)calloc(n3, sizeof(double));
    s->v = (double *)calloc(n3, sizeof(double));
    s->om = (double *)calloc(n3, sizeof(double));
    s->Fh = (double *)calloc(n3, sizeof(double));
    s->Th = (double *)calloc(n3, sizeof(double));
    s->Fc = (double *)calloc(n3, sizeof(double));
    s->R = (double *)calloc(n1, sizeof(double));
    s->rhos = (double *)calloc(n1, sizeof(double));
    s->m = (double *)calloc(n1, sizeof(double));
    s->I = (double *)calloc(n1, sizeof(double));
    s->fixed = (unsigned char *)calloc(n1, 1);
    for (int p = 0; p < np; p++) {
        for (int a = 0; a < 3; a++) {
            s->x[3 * p + a] = pos[3 * p + a];
            s->v[3 * p + a] = vel[3 * p + a];
            s->om[3 * p + a] = omega[3 * p + a];
        }
        if (s->L.D == 2) {
            s->x[3 * p + 2] = 0.0; s->v[3 * p + 2] = 0.0;
            s->om[3 * p + 0] = 0.0; s->om[3 * p + 1] = 0.0;
        }
        double r = radius[p];
        s->R[p] = r;
        s->rhos[p] = rho_s[p];
        if (s->L.D == 2) {
            s->m[p] = rho_s[p] * (ORC_PI * r * r);
            s->I[p] = 0.5 * s->m[p] * r * r;
        } else {
            s->m[p] = rho_s[p] * (4.0 / 3.0 * ORC_PI * r * r * r);
            s->I[p] = 0.4 * s->m[p] * r * r;
        }
        s->fixed[p] = fixed ? fixed[p] : 0;
    }
    /* a lookup table belongs to the radius of the particles it was built for */
    if (s->eps_mode == 1 && orc_set_eps_mode(s, 1) != 0) return -1;
    return 0;
}

int orc_set_f(orc_sim *s, const double *f) {
    memcpy(s->f, f, sizeof(double) * (size_t)s->L.Q * (size_t)s->N);
    return 0;
}

int orc_get_f(const orc_sim *s, double *f) {
    memcpy(f, s->f, sizeof(double) * (size_t)s->L.Q * (size_t)s->N);
    return 0;
}

/* Moments of the pre-collision f(x,t): rho[N], u[D][N] = sum_i f_i c_i / rho. */
int orc_get_macro(const orc_sim *s, double *rho, double *u) {
    const orc_lattice *L = &s->L;
#pragma omp parallel for schedule(static) if (s->N >= par_min_nodes)
    for (long n = 0; n < s->N; n++) {
        double r = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < L->Q; i++) {
            double fi = s->f[(long)i * s->N + n];
            r = r + fi;
            for (int a = 0; a < L->D; a++) j[a] = j[a] + (double)L->c[i][a] * fi;
        }
        rho[n] = r;
        for (int a = 0; a < L->D; a++) u[(long)a * s->N + n] = j[a] / r;
    }
    return 0;
}

int orc_get_particles(const orc_sim *s, double *pos, double *vel, double *omega) {
    memcpy(pos, s->x, sizeof(double) * 3 * (size_t)s->np);
    memcpy(vel, s->v, sizeof(double) * 3 * (size_t)s->np);
    memcpy(omega, s->om, sizeof(double) * 3 * (size_t)s->np);
    return 0;
}

int orc_get_forces(const orc_sim *s, double *F, double *T) {
    memcpy(F, s->Fh, sizeof(double) * 3 * (size_t)s->np);
    memcpy(T, s->Th, sizeof(double) * 3 * (size_t)s->np);
    return 0;
}

int orc_get_contact_forces(const orc_sim *s, double *Fc) {
    memcpy(Fc, s->Fc, sizeof(double) * 3 * (size_t)s->np);
    return 0;
}

/* q_n of the last collision, [3][N]; zero at uncovered nodes. */
int orc_get_q(const orc_sim *s, double *q) {
    memcpy(q, s->q, sizeof(double) * 3 * (size_t)s->N);
    return 0;
}

long orc_time(const orc_sim *s) { return s->t; }

/* ------------------------------------------------------------ step pieces */

/* Footprint: total count per node and the count-weighted rigid velocity sum,
 * accumulated over particles in ascending id.  This pass covers the nodes
 * whose outermost coordinate (z in 3D, y in 2D) lies in [o0, o1); nodes
 * beyond a wall do not exist. */
static void footprint_slab(orc_sim *s, int o0, int o1) {
    const int D = s->L.D;
    for (int p = 0; p < s->np; p++) {
        int lo[3], hi[3];
        particle_bbox(s, p, lo, hi);
        const double *xp = &s->x[3 * p], *vp = &s->v[3 * p], *wp = &s->om[3 * p];
        for (int cz = lo[2]; cz <= hi[2]; cz++) {
            int iz = D == 3 ? wrap_coord(s, 2, cz) : 0;
            if (iz < 0 || (D == 3 && (iz < o0 || iz >= o1))) continue;
            for (int cy = lo[1]; cy <= hi[1]; cy++) {
                int iy = wrap_coord(s, 1, cy);
                if (iy < 0 || (D == 2 && (iy < o0 || iy >= o1))) continue;
                for (int cx = lo[0]; cx <= hi[0]; cx++) {
                    int ix = wrap_coord(s, 0, cx);
                    int cnt = node_count(s, p, ix, iy, iz);
                    if (cnt == 0) continue;
                    long n = node_index(s, ix, iy, iz);
                    double rx = node_disp(s, 0, ix, xp[0]);
                    double ry = node_disp(s, 1, iy, xp[1]);
                    double vr[3];
                    if (D == 3) {
                        double rz = node_disp(s, 2, iz, xp[2]);
                        vr[0] = vp[0] + (wp[1] * rz - wp[2] * ry);
                        vr[1] = vp[1] + (wp[2] * rx - wp[0] * rz);
                        vr[2] = vp[2] + (wp[0] * ry - wp[1] * rx);
                    } else {
                        vr[0] = vp[0] - wp[2] * ry;
                        vr[1] = vp[1] + wp[2] * rx;
                        vr[2] = 0.0;
                    }
                    double c = (double)cnt;
                    for (int a = 0; a < 3; a++)
                        s->vnum[(long)a * s->N + n] = s->vnum[(long)a * s->N + n] + c * vr[a];
                    s->ctot[n] += cnt;
                }
            }
        }
    }
}

static void footprint(orc_sim *s) {
    const long N = s->N;
#pragma omp parallel for schedule(static) if (N >= par_min_nodes)
    for (long n = 0; n < N; n++) {
        s->ctot[n] = 0;
        s->vnum[n] = 0.0;
        s->vnum[N + n] = 0.0;
        s->vnum[2 * N + n] = 0.0;
    }
    /* slabs of the outermost axis are disjoint node sets */
    const int nouter = s->L.D == 3 ? s->nz : s->ny;
    const int nslab = nouter < 64 ? nouter : 64;
#pragma omp parallel for schedule(dynamic, 1) if (N >= par_min_nodes)
    for (int k = 0; k < nslab; k++)
        footprint_slab(s, (int)((long)nouter * k / nslab), (int)((long)nouter * (k + 1) / nslab));
}

/* Collision of one node, Eq. (1).  fin[Q] are the pre-collision values,
 * count the total sub-sample count, vs the solid velocity V_S (used only if
 * count > 0).  Writes fout[Q] and q[3]. */
static void collide_node(const orc_lattice *L, double tau, const double gf[3],
                         int Smax, const double *fin, int count, const double vs[3],
                         double *fout, double q[3]) {
    const int Q = L->Q, D = L->D;
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0}, u[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; i++) {
        rho = rho + fin[i];
        for (int a = 0; a < D; a++) j[a] = j[a] + (double)L->c[i][a] * fin[i];
    }
    for (int a = 0; a < D; a++) u[a] = j[a] / rho;

    double feq[19];
    for (int i = 0; i < Q; i++) feq[i] = feq_i(L, i, rho, u);

    double beta = 0.0;
    double Om[19];
    for (int i = 0; i < Q; i++) Om[i] = 0.0;
    if (count > 0) {
        int cc = count < Smax ? count : Smax;
        double eps = (double)cc / (double)Smax;
        beta = beta_of_eps(eps, tau);
        for (int i = 0; i < Q; i++) {
            int o = L->opp[i];
            Om[i] = (fin[o] - fin[i]) + (feq_i(L, i, rho, vs) - feq[o]);
        }
    }
    double a_relax = (1.0 - beta) / tau;
    for (int i = 0; i < Q; i++)
        fout[i] = fin[i] - a_relax * (fin[i] - feq[i]) + beta * Om[i] + force_i(L, i, rho, gf);

    q[0] = q[1] = q[2] = 0.0;
    if (count > 0) {
        double mom[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; i++)
            for (int a = 0; a < D; a++) mom[a] = mom[a] + (double)L->c[i][a] * Om[i];
        for (int a = 0; a < D; a++) q[a] = beta * mom[a];
    }
}

/* Exposed for unit tests: collide one node in isolation. */
void orc_collide_node(int dim, double tau, const double *gf, int samples,
                      const double *fin, int count, const double *vs,
                      double *fout, double *q) {
    orc_lattice L;
    lattice_init(&L, dim);
    int Smax = dim == 2 ? samples * samples : samples * samples * samples;
    collide_node(&L, tau, gf, Smax, fin, count, vs, fout, q);
}

void orc_feq(int dim, double rho, const double *u, double *feq) {
    orc_lattice L;
    lattice_init(&L, dim);
    for (int i = 0; i < L.Q; i++) feq[i] = feq_i(&L, i, rho, u);
}

static void collide_all(orc_sim *s) {
    const orc_lattice *L = &s->L;
    const int Q = L->Q;
    const int Smax = L->D == 2 ? s->S * s->S : s->S * s->S * s->S;
#pragma omp parallel for schedule(static) if (s->N >= par_min_nodes)
    for (long n = 0; n < s->N; n++) {
        double fin[19], fout[19], vs[3] = {0.0, 0.0, 0.0}, q[3];
        for (int i = 0; i < Q; i++) fin[i] = s->f[(long)i * s->N + n];
        int count = s->ctot[n];
        if (count > 0) {
            double den = (double)count;
            for (int a = 0; a < 3; a++) vs[a] = s->vnum[(long)a * s->N + n] / den;
        }
        collide_node(L, s->tau, s->gf, Smax, fin, count, vs, fout, q);
        for (int i = 0; i < Q; i++) s->fs[(long)i * s->N + n] = fout[i];
        for (int a = 0; a < 3; a++) s->q[(long)a * s->N + n] = q[a];
    }
}

/* Streaming: f_i(x + c_i, t+1) = f*_i(x); beyond a wall the population is
 * reflected into the opposite direction at the same node. */
static void stream_all(orc_sim *s) {
    const orc_lattice *L = &s->L;
    /* every (direction, target node) is written by exactly one source */
#pragma omp parallel for collapse(2) schedule(static) if (s->N >= par_min_nodes)
    for (int z = 0; z < s->nz; z++)
        for (int y = 0; y < s->ny; y++)
            for (int x = 0; x < s->nx; x++) {
                long n = node_index(s, x, y, z);
                for (int i = 0; i < L->Q; i++) {
                    double val = s->fs[(long)i * s->N + n];
                    int tx = x + L->c[i][0], ty = y + L->c[i][1], tz = z + L->c[i][2];
                    int wx = wrap_coord(s, 0, tx), wy = wrap_coord(s, 1, ty), wz = wrap_coord(s, 2, tz);
                    if (wy < 0) {
                        s->f[(long)L->opp[i] * s->N + n] = val;
                    } else {
                        s->f[(long)i * s->N + node_index(s, wx, wy, wz)] = val;
                    }
                }
            }
}

/* Eq. (3) with shares: F_p = -sum_n s_pn q_n, T_p = -sum_n r_pn x (s_pn q_n). */
static void hydro_forces(orc_sim *s) {
    const int D = s->L.D;
#pragma omp parallel for schedule(dynamic, 16) if (s->np >= par_min_particles)
    for (int p = 0; p < s->np; p++) {
        orc_acc F[3] = {{0, 0}, {0, 0}, {0, 0}}, T[3] = {{0, 0}, {0, 0}, {0, 0}};
        int lo[3], hi[3];
        particle_bbox(s, p, lo, hi);
        const double *xp = &s->x[3 * p];
        for (int cz = lo[2]; cz <= hi[2]; cz++)
            for (int cy = lo[1]; cy <= hi[1]; cy++)
                for (int cx = lo[0]; cx <= hi[0]; cx++) {
                    int ix = wrap_coord(s, 0, cx), iy = wrap_coord(s, 1, cy);
                    int iz = D == 3 ? wrap_coord(s, 2, cz) : 0;
                    if (ix < 0 || iy < 0 || iz < 0) continue;
                    int cnt = node_count(s, p, ix, iy, iz);
                    if (cnt == 0) continue;
                    long n = node_index(s, ix, iy, iz);
                    double sh = (double)cnt / (double)s->ctot[n];
                    double t[3];
                    for (int a = 0; a < 3; a++) t[a] = sh * s->q[(long)a * s->N + n];
                    double rx = node_disp(s, 0, ix, xp[0]);
                    double ry = node_disp(s, 1, iy, xp[1]);
                    for (int a = 0; a < D; a++) acc_add(&F[a], t[a]);
                    if (D == 3) {
                        double rz = node_disp(s, 2, iz, xp[2]);
                        acc_add(&T[0], ry * t[2] - rz * t[1]);
                        acc_add(&T[1], rz * t[0] - rx * t[2]);
                        acc_add(&T[2], rx * t[1] - ry * t[0]);
                    } else {
                        acc_add(&T[2], rx * t[1] - ry * t[0]);
                    }
                }
        for (int a = 0; a < 3; a++) {
            s->Fh[3 * p + a] = -acc_value(&F[a]);
            s->Th[3 * p + a] = -acc_value(&T[a]);
        }
        if (D == 2) { s->Fh[3 * p + 2] = 0.0; s->Th[3 * p + 0] = 0.0; s->Th[3 * p + 1] = 0.0; }
        if (!s->couple)
            for (int a = 0; a < 3; a++) { s->Fh[3 * p + a] = 0.0; s->Th[3 * p + a] = 0.0; }
    }
}

/* Eqs. (4)-(5), all pairs (ascending j) then the walls. */
static void dem_forces_impl(int D, int np, const double *x, const double *v,
                            const double *R, const double *m, double kn, double ce,
                            const double Lbox[3], int wall_y, double *Fc) {
#pragma omp parallel for schedule(dynamic, 16) if (np >= par_min_particles)
    for (int i = 0; i < np; i++) {
        double F[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < np; j++) {
            if (j == i) continue;
            double d[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < D; a++) {
                double dd = x[3 * i + a] - x[3 * j + a];
                if (!(a == 1 && wall_y)) dd = min_image(dd, Lbox[a]);
                d[a] = dd;
            }
            double d2 = d[0] * d[0] + d[1] * d[1];
            if (D == 3) d2 = d2 + d[2] * d[2];
            double dist = sqrt(d2);
            double delta = (R[i] + R[j]) - dist;
            if (!(delta > 0.0)) continue;
            double nrm[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < D; a++) nrm[a] = d[a] / dist;
            double vn = (v[3 * i + 0] - v[3 * j + 0]) * nrm[0] + (v[3 * i + 1] - v[3 * j + 1]) * nrm[1];
            if (D == 3) vn = vn + (v[3 * i + 2] - v[3 * j + 2]) * nrm[2];
            double meff = m[i] * m[j] / (m[i] + m[j]);
            double eta = ce * sqrt(meff * kn);
            double fmag = kn * delta - eta * vn;
            for (int a = 0; a < D; a++) F[a] = F[a] + fmag * nrm[a];
        }
        if (wall_y) {
            double eta = ce * sqrt(m[i] * kn);
            /* lower wall at y = -1/2, normal +y */
            double dl = R[i] - (x[3 * i + 1] + 0.5);
            if (dl > 0.0) {
                double fmag = kn * dl - eta * v[3 * i + 1];
                F[1] = F[1] + fmag;
            }
            /* upper wall at y = Ly - 1/2, normal -y */
            double du = R[i] - ((Lbox[1] - 0.5) - x[3 * i + 1]);
            if (du > 0.0) {
                double fmag = kn * du - eta * (-v[3 * i + 1]);
                F[1] = F[1] - fmag;
            }
        }
        for (int a = 0; a < 3; a++) Fc[3 * i + a] = F[a];
    }
}

/* Exposed for unit tests: contact forces of a particle set in isolation. */
void orc_dem_forces(int dim, int np, const double *x, const double *v,
                    const double *R, const double *m, double kn, double restitution,
                    const double *Lbox, int wall_y, double *Fc) {
    double le = log(restitution);
    double ce = -2.0 * le / sqrt(ORC_PI * ORC_PI + le * le);
    dem_forces_impl(dim, np, x, v, R, m, kn, ce, Lbox, wall_y, Fc);
}

static double wrap_pos(double x, double Lp) {
    if (x < 0.0) {
        x = x + Lp;
        if (x >= Lp) x = x - Lp;
    } else if (x >= Lp) {
        x = x - Lp;
    }
    return x;
}

/* Symplectic Euler, dt = 1:  v += (F^h + F^c + m a)/m;  omega += T^h / I;
 * x += v (new);  periodic wrap. */
static void integrate(orc_sim *s) {
    const int D = s->L.D;
    double Lb[3] = {(double)s->nx, (double)s->ny, (double)s->nz};
#pragma omp parallel for schedule(static) if (s->np >= par_min_particles)
    for (int p = 0; p < s->np; p++) {
        if (s->fixed[p]) continue;
        for (int a = 0; a < D; a++) {
            double ftot = s->Fh[3 * p + a] + s->Fc[3 * p + a] + s->m[p] * s->ap[a];
            s->v[3 * p + a] = s->v[3 * p + a] + ftot / s->m[p];
        }
        if (D == 3) {
            for (int a = 0; a < 3; a++)
                s->om[3 * p + a] = s->om[3 * p + a] + s->Th[3 * p + a] / s->I[p];
        } else {
            s->om[3 * p + 2] = s->om[3 * p + 2] + s->Th[3 * p + 2] / s->I[p];
        }
        for (int a = 0; a < D; a++) {
            double xn = s->x[3 * p + a] + s->v[3 * p + a];
            if (!(a == 1 && s->wall_y)) xn = wrap_pos(xn, Lb[a]);
            s->x[3 * p + a] = xn;
        }
    }
}

int orc_step(orc_sim *s, int nsteps) {
    double Lb[3] = {(double)s->nx, (double)s->ny, (double)s->nz};
    for (int k = 0; k < nsteps; k++) {
        footprint(s);
        collide_all(s);
        stream_all(s);
        hydro_forces(s);
        dem_forces_impl(s->L.D, s->np, s->x, s->v, s->R, s->m, s->kn, s->ce, Lb, s->wall_y, s->Fc);
        integrate(s);
        s->t++;
    }
    return 0;
}

/* Exposed for unit tests: per-node total counts of the current footprint
 * (ctot[N]) and the count of one particle on one node. */
int orc_footprint_counts(orc_sim *s, int *ctot) {
    footprint(s);
    memcpy(ctot, s->ctot, sizeof(int) * (size_t)s->N);
    return 0;
}

int orc_particle_node_count(const orc_sim *s, int p, int ix, int iy, int iz) {
    return node_count(s, p, ix, iy, iz);
}

/* Selects the eps rule: 0 sub-cell sampling, 1 table lookup.  The table
 * needs every particle to have the same radius, at least 1 (so that a node
 * at the centre is wholly inside); returns -1 otherwise.  Call after
 * orc_set_particles (and again after every later orc_set_particles). */
int orc_set_eps_mode(orc_sim *s, int mode) {
    if (mode != 0 && mode != 1) return -1;
    free(s->tab);
    s->tab = NULL;
    s->eps_mode = mode;
    if (mode == 0) return 0;
    if (s->np < 1) return -1;
    double R = s->R[0];
    for (int p = 1; p < s->np; p++)
        if (s->R[p] != R) return -1;
    if (!(R >= 1.0)) return -1;
    s->tab = (int *)malloc(sizeof(int) * (size_t)eps_table_len(s->L.D));
    if (!s->tab) return -1;
    eps_table_build(s->L.D, s->S, R, s->tab);
    s->tab_R = R;
    return 0;
}

/* For tests: the table count of a displacement (d0, d1, d2) for radius R and
 * S samples per axis (the table of the last (D, S, R) asked for is kept). */
int orc_eps_table_count(int D, int S, double R, double d0, double d1, double d2) {
    static int *tab = NULL;
    static int tD = 0, tS = 0;
    static double tR = 0.0;
    if (!tab || tD != D || tS != S || tR != R) {
        free(tab);
        tab = (int *)malloc(sizeof(int) * (size_t)eps_table_len(D));
        if (!tab) return -1;
        eps_table_build(D, S, R, tab);
        tD = D; tS = S; tR = R;
    }
    return eps_table_lookup(D, S, R, tab, d0, d1, d2);
}

double orc_sum2(const double *p, long n) {
    orc_acc A = {0.0, 0.0};
    for (long i = 0; i < n; i++) acc_add(&A, p[i]);
    return acc_value(&A);
}

double orc_beta(double eps, double tau) { return beta_of_eps(eps, tau); }

/* Number of threads the oracle's parallel loops use from now on (n >= 1;
 * n <= 0 selects every core).  Returns the number in effect; 1 when built
 * without OpenMP. */
/* Smallest node loop and particle loop that run on several threads (values
 * below 1 are taken as 1).  Results do not depend on them. */
void orc_set_parallel_minimum(long nodes, long particles) {
    par_min_nodes = nodes < 1 ? 1 : nodes;
    par_min_particles = particles < 1 ? 1 : particles;
}

int orc_set_threads(int n) {
#ifdef _OPENMP
    if (n <= 0) n = omp_get_num_procs();
    omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
