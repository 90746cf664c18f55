// internal.h -- device-side data layout, lattice traits and launcher
// declarations shared by the HIP translation units of liblbimb.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbimb {

// ---------------------------------------------------------------- lattices
// D2Q9 and D3Q19 velocity sets (the paper's "Numerical scheme").  Ordering:
// rest first, then axis directions, then diagonals; opposite directions are
// adjacent so that opp() is a table lookup.  The weight class k selects
// w = {4/9, 1/9, 1/36} (D2Q9) or {1/3, 1/18, 1/36} (D3Q19).
struct D2Q9 {
    static constexpr int D = 2, Q = 9;
    static constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    static constexpr int wc[9] = {0, 1, 1, 1, 1, 2, 2, 2, 2};
    static constexpr double w[3] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0};
    static constexpr float invw[3] = {2.25f, 9.0f, 36.0f};
};

struct D3Q19 {
    static constexpr int D = 3, Q = 19;
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    static constexpr int wc[19] = {0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2};
    static constexpr double w[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};
    static constexpr float invw[3] = {3.0f, 18.0f, 36.0f};
};

enum : uint32_t {
    FLAG_SLOT_OVERFLOW = 1u,
    FLAG_CELL_OVERFLOW = 2u,
    FLAG_CONTACT_OVERFLOW = 4u,
    FLAG_NONFINITE = 8u,
    FLAG_BATCH_TIMEOUT = 16u,
    FLAG_FAST = 32u,       // a particle moved more than one node in y in a step (slab pipeline)
};

constexpr int MAX_OWNERS = 4;
constexpr int MAX_CONTACTS = 32;
constexpr int CELL_CAP = 16;
constexpr int NL_CAP = 2 * MAX_CONTACTS;  // neighbour-list entries per particle
constexpr int SLOT_COUNT_BITS = 10;  // count of sub-samples (<= 512) in the low bits

// eps lookup table (Eq. 6): bins of rho = |r| - R and of the folded direction
constexpr int EPS_TAB_NRHO = 64;
constexpr int EPS_TAB_NT = 16;
constexpr int EPS_TAB_M = 16;  // reference points per axis behind each entry

// Particle state, structure of arrays, binary64.  Vectors are [3][P].
struct Particles {
    double *x, *v, *w;     // position, velocity, angular velocity
    double *R, *m, *I;     // radius, mass, moment of inertia
    uint8_t *fixed;
    double *Fh, *Th, *Fc;  // hydrodynamic force/torque, contact force
    int *bb;               // [6][P] painted bounding box, lower and upper corner
    uint32_t *list;        // [P][list_cap] covered nodes: count | kx << 10 | ky << 17 | kz << 24
    int *list_len;         // [P]
    int list_cap;
    int np;
};

// Lattice geometry shared by every kernel.
struct Geom {
    int nx, ny, nz;
    int wall_y;
    int64_t N;
    double Lx, Ly, Lz;     // box lengths as doubles
};

// Arguments of the fused stream-collide-IMB kernel.
// Per-node IMB exchange record, written by the lattice kernel at covered
// nodes and read by the force kernel: q_n = beta sum_i Omega_i c_i (binary64,
// z component 0 in 2D) and the total sub-sample count.  32 bytes, so one
// record is one aligned pair of 16-byte stores / loads.
struct alignas(32) QRec {
    double q[3];
    int tot;
    int pad;
};

// The same record for the binary32 storage modes, whose q is computed in
// binary32: 16 bytes, one aligned 16-byte store / load.
struct alignas(16) QRec32 {
    float q[3];
    int tot;
};

// Reads q and the total count of node n from either record kind.
__device__ __forceinline__ void read_qrec(const void *qr, bool r32, int64_t n, double q[3], int &tot) {
    if (r32) {
        const QRec32 r = ((const QRec32 *)qr)[n];
        q[0] = (double)r.q[0]; q[1] = (double)r.q[1]; q[2] = (double)r.q[2];
        tot = r.tot;
    } else {
        const QRec r = ((const QRec *)qr)[n];
        q[0] = r.q[0]; q[1] = r.q[1]; q[2] = r.q[2];
        tot = r.tot;
    }
}

struct LBArgs {
    const void *A;         // post-collision populations of the previous step
    void *B;               // post-collision populations of this step
    uint8_t *nown;         // owners per node; zeroed here once read (last reader in the step)
    const uint32_t *slots; // [MAX_OWNERS][N] (pid << 10 | count)
    const double *beta_tab;   // beta(eps) for count 0..Smax
    const double *arel_tab;   // (1 - beta) / tau for count 0..Smax
    void *qr;              // [N] IMB exchange records (covered nodes): QRec (FP64) or QRec32
    const double *px, *pv, *pw;  // particle SoA
    int np;
    Geom g;
    int Smax;
    double arel0;          // 1 / tau
    double cg[19];         // c_i . g_fluid per direction
    float cgf[19];
    float arel0f;
    float tauf;
    uint32_t *flags;
    int y0, ny_run;        // rows y0 .. y0 + ny_run - 1 of every z plane (a slab; ny_run = ny: all)
};

// Slab pipeline (walls in y): the lattice update of a step runs slab by slab
// in y; the particles whose footprint can reach no higher than slab g (with a
// node of margin for the step's motion) form group g, whose force sums,
// integration and next footprint run as soon as slabs g - 1 and g are done.
constexpr int PIPE_MAX = 8;
struct Groups {
    const int *count;      // [K] particles of each group this step
    const int *list;       // [K][P] their ids
    int *ncount;           // [K] the next step's groups (filled by the integration)
    int *nlist;            // [K][P]
    int K;                 // slabs (1: no pipeline)
    int g;                 // the group a launch takes; -1: every particle, one per workgroup
    int stride;            // entries reserved per group list
    int ys[PIPE_MAX + 1];  // slab k holds rows ys[k] .. ys[k + 1] - 1
};

// Group of a particle at height y with radius R: the slab that holds the
// highest node its footprint can reach after one more step of at most one
// node, floor(y + R + 3/2).
__device__ __forceinline__ int slab_group(const Groups &G, double y, double R) {
    const int top = (int)floor(y + R + 1.5);
    int k = 0;
    while (k + 1 < G.K && G.ys[k + 1] <= top) k++;
    return k;
}

struct FootArgs {
    Particles P;
    Geom g;
    uint8_t *nown;
    uint32_t *slots;
    int S;
    uint32_t *flags;
    // table lookup of eps (null: sub-cell sampling); H = sqrt(D)/2, the rho
    // bin width and the direction scales sqrt(2) NT and sqrt(3) NT
    const uint16_t *tab;
    double tabH, tabW, tabK1, tabK2;
    Groups G;
};

struct ForceArgs {
    Particles P;
    Geom g;
    const void *qr;        // QRec (FP64 storage) or QRec32 (binary32 storage modes)
    int rec32;
    int D;
    int integrate;         // 1: the kernel also advances the particle (needs F^c of this step)
    double ap[3];          // particle acceleration (gravity with buoyancy)
    uint32_t *flags;
    Groups G;              // G.K > 1: the integration also files the particle in its next group
};

struct CellArgs {
    Particles P;
    Geom g;
    int ncx, ncy, ncz;
    int *cell_count;
    int *cell_ids;         // [ncell][CELL_CAP]
    uint32_t *flags;
    int D;
    double kn, ce;
    double ap[3];
    // neighbour-list mode: lists of the pairs within R_i + R_j + skin, rebuilt
    // after `every` steps or when a particle has moved skin / 2 since the build
    int every;
    double skin;
    int *nl;               // [P][NL_CAP] neighbour ids, ascending
    int *nl_len;           // [P]
    double *xb;            // [3][P] positions at the last build
    int *nl_state;         // [0] rebuild flag, [1] steps since the last build
    int64_t *nl_builds;    // builds so far
    int64_t ncell;         // ncx * ncy * ncz
};

// Suspension-wide sums (lbm_get_stats): node pass over the lattice rows with a
// fixed number of workgroups, one row of STATS_PK values per particle, one
// final workgroup.  tot receives 4 + STATS_PK values: mass, j (3), then the
// particle sums m v (3), v (3), F^h (3), eps-share of mass, of momentum (3),
// eps (the node's solid fraction split over its owners), m.
constexpr int STATS_NT = 256;
constexpr int STATS_NODE_GROUPS = 1024;
constexpr int STATS_PK = 15;

struct StatsArgs {
    const void *A;         // current state (pre-collision populations by pull)
    Geom g;
    Particles P;
    const void *qr;        // exchange records of the last step (node totals)
    int rec32;
    int Smax;
    double *node_part;     // [STATS_NODE_GROUPS][4]
    double *part_rows;     // [np][STATS_PK]
    double *tot;           // [4 + STATS_PK]
};

// One periodic cubic box of the batched ensemble (fixed spheres).
struct BatchBox {
    int L;                 // edge
    int rows;              // lattice rows per tile (tile shape)
    int ntiles;            // L*L / rows
    int tile0;             // first global tile index of the box
    int64_t off;           // element offset of the box's populations in A / B
    int64_t noff;          // node offset of the box in per-node arrays
    int table;             // offset of the box's beta / (1-beta)/tau tables
    int active;            // 0: retired (skipped)
    float arel0f;          // 1 / tau
    float cgf[19];         // c_i . g_fluid
    float g0[19];          // initial shifted populations f^eq_i(1, u0) - w_i
    double radius;         // sphere radius of the box
    double tau;            // relaxation time
    int sph0;              // first sphere of the box (global sphere index)
    int nsph;              // spheres in the box
};

// State of the steady-drag check of lbm_batch_run_steady.
struct BatchSteady {
    double *Fprev;         // [nsph][3] force at the previous check
    int *steady;           // [nbox] 1: retired by the check
    int64_t *stop;         // [nbox] batch time at which the box retired
    int *remaining;        // active boxes after the last check
    int *first;            // 1: the next check only records F_prev (cleared by the check)
    int64_t *tnow;         // batch time of the last check (advanced by the check)
    double tol;
};

struct BatchArgs {
    float *A, *B;              // population pool, shifted storage
    const BatchBox *boxes;
    const int *tile_box;       // [ntiles] box of each global tile
    const uint16_t *cnt;       // [total_nodes] static total sample count
    const float *beta, *arel;  // per-box tables
    float *q;                  // [3][total_nodes]
    int64_t total_nodes;
    int nbox, ntiles, Smax;
    int *queue;                // persistent work counter
    int *done;                 // [nbox] tiles finished (persistent mode)
    uint32_t *flags;
    // spheres
    int nsph;
    const int *sph_box;
    const double *sph_x;       // [nsph][3] position in its box
    const int *list_start;     // [nsph + 1]
    const uint32_t *list;      // node | count << 20
    double *F, *T;             // [nsph][3]
};

// launchers (batch.hip)
hipError_t launch_batch_step(const BatchArgs &a, int parity, hipStream_t s);
hipError_t launch_batch_persistent(const BatchArgs &a, int nsteps, int parity0, int grid, hipStream_t s);
hipError_t launch_batch_force(const BatchArgs &a, hipStream_t s);
hipError_t launch_batch_mean(const BatchArgs &a, int parity, double *U, hipStream_t s);
hipError_t launch_batch_get_f(const BatchArgs &a, int b, int L, int parity, double *f, hipStream_t s);
hipError_t launch_batch_init(const BatchArgs &a, int nbox, int maxL, hipStream_t s);
hipError_t launch_batch_shell(const BatchArgs &a, int parity, double *u, hipStream_t s);
hipError_t launch_batch_check(const BatchArgs &a, BatchBox *boxes, const BatchSteady &st, int64_t k,
                              hipStream_t s);
hipError_t launch_batch_features(const BatchArgs &a, const double *U, const double *Us, float *feat,
                                 hipStream_t s);
int batch_persistent_grid();

// launchers (lb_kernels.hip)
// width: threads per workgroup of the lattice kernel (64, 128, 192 or 256),
// 0 for the built-in rule (the whole row up to 256 threads); order: 0 linear,
// 1 XCD order (workgroups renumbered so each XCD takes a contiguous run);
// cu_groups: 0, or 3..8 workgroups per CU at most (an unused LDS reservation)
hipError_t launch_lb(int lattice, int storage, const LBArgs &a, int width, int order, int cu_groups,
                     hipStream_t s);
unsigned lds_reserve_bytes(int cu_groups);
int lattice_block_width(int nx, int width);        // the width a launch uses
bool xcd_order_fits(const Geom &g, int width);     // grid below 2^32 workgroups
hipError_t launch_fill_rest_f64(int lattice, const Geom &g, double *A, hipStream_t s);
hipError_t launch_get_f(int lattice, int storage, const Geom &g, const void *A, double *f,
                        hipStream_t s);
hipError_t launch_set_f(int lattice, int storage, const Geom &g, const double *f, void *A,
                        hipStream_t s);
hipError_t launch_macro(int lattice, int storage, const Geom &g, const void *A, double *rho,
                        double *u, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t count, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, uint64_t value, int64_t count, hipStream_t s);

// launcher (stats.hip)
hipError_t launch_stats(int lattice, int storage, const StatsArgs &a, hipStream_t s);

// launchers (particle_kernels.hip)
hipError_t launch_foot_paint(const FootArgs &a, int D, hipStream_t s);
hipError_t launch_force(const ForceArgs &a, hipStream_t s);
// files every particle in its group of the current step (G.nlist / G.ncount
// must be cleared first)
hipError_t launch_assign_groups(const ForceArgs &a, hipStream_t s);
hipError_t launch_list_q(const ForceArgs &a, double *out, hipStream_t s);
hipError_t launch_cells(const CellArgs &a, hipStream_t s);
hipError_t launch_dem(const CellArgs &a, hipStream_t s);
// neighbour-list mode: the guard, a conditional rebuild (cells and lists) and
// the contacts from the lists; phase_mid is called between the rebuild and the
// contacts (for the per-phase timing)
hipError_t launch_nl_rebuild(const CellArgs &a, hipStream_t s);
hipError_t launch_nl_contacts(const CellArgs &a, hipStream_t s);

}  // namespace lbimb
