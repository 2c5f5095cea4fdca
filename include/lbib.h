/*
 * lbib.h -- C-ABI of the MI355X (gfx950) LB-IB particle-adhesion library.
 *
 * The library advances the combined lattice Boltzmann - immersed boundary model of
 * Coclite et al., "Predicting Different Adhesive Regimens of Circulating Particles at Blood
 * Capillary Walls" (arXiv 1808.01448, section "Computational method"): a D2Q9 BGK fluid with
 * Guo forcing (eq 1-6), a rigid particle coupled through moving-least-squares (MLS)
 * immersed-boundary interpolation and spreading, surface loads from normal probes (eq 7-8),
 * stochastic ligand-receptor bonds (eq 9-11), a wall force (eq 12) and an explicit
 * second-order rigid-body update (eq 13-16).  Every step of the time loop runs in HIP
 * kernels on the GPU; the host only validates, allocates and enqueues.
 *
 * Conventions shared by every call
 *  - Lattice units: dx = dt = 1, rho_ref = 1, cs^2 = 1/3, nu = (tau - 1/2)/3.
 *  - Node (i, j) sits at (x, y) = (i, j), 0 <= i < nx, 0 <= j < ny.  x is periodic.
 *    Half-way bounce-back walls lie at y = -1/2 (the receptor wall, at rest) and y = ny - 1/2,
 *    so the channel height is H = ny, and u_max = Re nu / H.  Drive 0: both walls rest and the
 *    body force g = (8 nu u_max / H^2, 0) drives a Poiseuille flow of centre-line velocity
 *    u_max.  Drive 1 (the shear setup of the section "Modeling the adhesion dynamics ..."):
 *    no body force; the top wall moves along x at u_max (moving-wall bounce-back: a
 *    population reflected there gains -2 w_q rho_ref (e_q . u_wall) / cs^2), giving the
 *    linear shear u_x = u_max (y + 1/2) / H.
 *  - Populations are D2Q9 in the order e_0 = (0,0), e_1 = (1,0), e_2 = (0,1), e_3 = (-1,0),
 *    e_4 = (0,-1), e_5 = (1,1), e_6 = (-1,1), e_7 = (-1,-1), e_8 = (1,-1) (eq 3).  Host arrays
 *    of populations are plain f (not shifted), FP64, laid out [q][j][i] with i fastest.
 *  - Particle angle theta: 0 means the major axis (semi-axis a) is normal to the wall;
 *    positive is counter-clockwise.  Angular velocity omega is counter-clockwise positive.
 *  - Every function returns an lbib_status; nothing throws or aborts across this boundary.
 *    Arguments are validated before anything is allocated or changed: a call that fails
 *    validation leaves the handle as it was.  lbib_last_error() then describes the failure.
 *  - Numerical failure (non-finite force, velocity or torque, a particle touching the wall,
 *    a singular MLS system, a spread tile overflow) is detected on the GPU and reported as
 *    LBIB_E_NUMERIC by the next lbib_sync / lbib_read_* call; lbib_step then returns
 *    LBIB_E_STATE until lbib_load restores a good state.
 *  - Ownership: descriptors are copied on entry.  The handle owns all device memory.  Host
 *    read buffers belong to the caller and come with an explicit capacity; too small a
 *    capacity returns LBIB_E_INVALID and names the required size in lbib_last_error().
 *  - Threading: one handle is used from one host thread at a time; distinct handles are
 *    independent.  Work is enqueued on the handle's HIP stream (and on a second stream the
 *    handle owns, joined back into the first at the end of every lbib_step).
 *  - Determinism: identical descriptors and seed give bit-identical results on the same
 *    build and GPU (the spread is accumulated in 64-bit fixed point, every other reduction
 *    has a fixed order, and bond draws come from a counter-based generator).
 */
#ifndef LBIB_H
#define LBIB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBIB_ABI_VERSION 2

typedef struct lbib_sim* lbib_handle;

typedef enum {
    LBIB_OK = 0,
    LBIB_E_INVALID = -1,     /* bad argument: nothing was changed */
    LBIB_E_STATE = -2,       /* call out of order, or the simulation is in the failed state */
    LBIB_E_NOMEM = -3,       /* device or host allocation failed */
    LBIB_E_DEVICE = -4,      /* a HIP runtime call failed */
    LBIB_E_NUMERIC = -5,     /* the GPU watchdog raised a numerical failure */
    LBIB_E_UNSUPPORTED = -6, /* valid request this build does not implement */
    LBIB_E_FULL = -7         /* a pool's memory budget or member count would be exceeded */
} lbib_status;

/* Precision of the population storage: f - w_q in double (FP64), float (FP32), IEEE
 * binary16 (FP16, stored as (f - w_q) 2^S, S = floor(log2(8192 / d)) clamped to [0, 40],
 * d = (4/9)(3u + 4.5u^2), u = max(4 u_max, 1e-6): the largest deviation expected lands near
 * 2^13, far from both the binary16 maximum and its subnormals) or bfloat16 (BF16).  Values
 * are rounded to nearest even (FP16 through float: (float)(f - w) * 2^S).  The collision is evaluated
 * in FP64 for the FP64 and FP32 storages (in FP32 arithmetic its rounding breaks the
 * momentum balance at a level that accumulates over thousands of steps at the small
 * velocities of capillary flow) and in FP32 for the 16-bit storages, whose rounding is far
 * coarser.  The particle phase (MLS solves, interpolation, loads, bonds, reductions, rigid
 * body) is FP64 for every storage.  Bytes per lattice update: 144, 72, 36, 36. *
 * LBIB_FP16_NEQ and LBIB_BF16_NEQ store instead f - f_eq(rho, u) of the node that emitted
 * each population (its non-equilibrium part, typically 10^-2 of f - w_q), in the same two
 * formats (FP16 with the same scale rule), with that node's rho - 1, u_x and u_y kept beside
 * in FP32; the sweep computes in FP32 (the emitting nodes' equilibria, the collision, the new
 * equilibrium), the particle phase in FP64.  Bytes per lattice update: 60. */
enum { LBIB_FP64 = 0, LBIB_FP32 = 1, LBIB_FP16 = 2, LBIB_BF16 = 3, LBIB_FP16_NEQ = 4, LBIB_BF16_NEQ = 5 };

/* Lattice (section "Modeling the adhesion dynamics ..."; Table 1).  drive: 0 body-force
 * Poiseuille with resting walls, 1 moving top wall (linear shear); the initial state is the
 * developed profile of the drive at rho = 1.  Requirements: nx >= 4, ny >= 4, tau > 1/2,
 * Re >= 0, drive 0 or 1. */
typedef struct {
    int32_t nx, ny;
    double tau;
    double re;
    int32_t drive;
    int32_t precision;
    uint64_t seed; /* key of the bond draws */
} lbib_lattice_desc;

/* Rigid particle (section "Pressure and viscous stresses"; particle shapes of the results
 * section).  shape 0: circle of radius a_major (b_minor ignored); shape 1: ellipse with
 * semi-axis a_major along the body y axis and b_minor along the body x axis.  The surface
 * is cut into n_markers straight elements of equal arc length starting at the body point
 * (0, -a) and running counter-clockwise; each element's centroid is a Lagrangian marker.
 * rho_p is the particle density (mass = rho_p pi a b).  Requirements: 8 <= n_markers <= 1024,
 * marker spacing (perimeter / n_markers) >= 0.25, the particle inside the channel with a
 * positive gap to both walls, 2 a_major + 6 <= nx. */
typedef struct {
    int32_t shape;
    double a_major, b_minor;
    double xc, yc, theta0;
    double rho_p;
    int32_t n_markers;
} lbib_particle_desc;

/* Ligands and bonds (section "Wall-particle interaction", eq 9-12, Table 1).  The ligand
 * density rho_l = rho_l_num / rho_l_den (0 <= rho_l <= 1) selects floor(n rho_l) elements
 * spread evenly along the perimeter.  Table 1 dimensionless groups, converted with
 * nu = (tau - 1/2)/3 and H = ny:
 *   sigma = sigma_hat nu^2 / H            spring constant (eq 9)
 *   sigma* = sigma_star_ratio sigma       (eq 11; 0.5 gives slip bonds)
 *   y_cr = y_cr_hat H                     critical separation for bond formation
 *   y_eq = y_eq_ratio y_cr                equilibrium bond length (eq 9)
 *   k_BT = kbt_hat nu^2 H                 thermal energy (eq 11)
 *   H_k = hamaker_hat nu^2 H              Hamaker constant (eq 12)
 * k_f and k_r0 are rates per time step (eq 10-11). */
typedef struct {
    int32_t rho_l_num, rho_l_den;
    double sigma_hat, sigma_star_ratio;
    double y_cr_hat, y_eq_ratio;
    double k_f, k_r0;
    double kbt_hat, hamaker_hat;
} lbib_ligand_desc;

/* Receptors: the paper covers the wall completely (density 1).  wall must be 0 (bottom) and
 * density must be 1.0; anything else returns LBIB_E_UNSUPPORTED. */
typedef struct {
    int32_t wall;
    double density;
} lbib_receptor_desc;

/* One particle record: the state after a step and the loads used in it.  n_bonds counts
 * the bonds after the step's update, n_probing the ligands that were within y_cr. */
typedef struct {
    int64_t step; /* index n of the step n -> n+1 this record describes */
    double xc, yc, theta, ux, uy, omega;   /* time level n+1 */
    double fx, fy, torque;                 /* total load used for the update */
    double fx_hydro, fy_hydro, m_hydro;    /* eq 7-8 */
    double fx_bond, fy_bond, m_bond;       /* eq 9 summed over bonded elements */
    double fy_wall;                        /* eq 12 */
    double gap;                            /* analytic gap to y = -1/2 at level n */
    int32_t n_bonds, n_probing;
} lbib_particle_state;

int lbib_abi_version(void);

/* Create a simulation.  hip_stream: the hipStream_t to enqueue on, or NULL for a stream the
 * handle creates and owns.  On success *out receives the handle. */
lbib_status lbib_create(const lbib_lattice_desc* desc, void* hip_stream, lbib_handle* out);

/* Add a particle (up to 64 per simulation); *particle_id receives its index, which also keys
 * its bond draws.  Particles interact only through the fluid (the paper's particles do not
 * collide; placements must not overlap).  With several particles each step runs the split
 * particle phase (see lbib_set_overlap). */
lbib_status lbib_particle_add(lbib_handle h, const lbib_particle_desc* desc, int32_t* particle_id);

/* Decorate particle particle_id with ligands; required before lbib_init when a particle
 * exists. */
lbib_status lbib_ligands_set(lbib_handle h, int32_t particle_id, const lbib_ligand_desc* desc);

/* Receptors on the wall; optional (the default is the paper's full coverage). */
lbib_status lbib_receptors_set(lbib_handle h, const lbib_receptor_desc* desc);

/* Allocate device memory and set the initial state: f = f_eq(1, u(y)) with the Poiseuille
 * profile u(y) = 4 u_max (y + 1/2)(H - 1/2 - y) / H^2; particle at rest; no bonds. */
lbib_status lbib_init(lbib_handle h);

/* Enqueue n_steps time steps (asynchronous: returns before the GPU finishes). */
lbib_status lbib_step(lbib_handle h, int64_t n_steps);

/* Wait for enqueued work; returns LBIB_E_NUMERIC when the watchdog fired. */
lbib_status lbib_sync(lbib_handle h);

/* Steps completed by the enqueued work (host count). */
lbib_status lbib_step_count(lbib_handle h, int64_t* steps);

/* Latest particle record (after the last completed step; before any step: the initial
 * state with zero loads and step = -1). */
lbib_status lbib_read_particle(lbib_handle h, int32_t pid, lbib_particle_state* out);

/* Bond and ligand flags per element (capacity >= n_markers). */
lbib_status lbib_read_bonds(lbib_handle h, int32_t pid, uint8_t* bonded, uint8_t* ligand, int32_t capacity);

/* Marker positions and outward normals at the current time level, xy and nxy as
 * [n_markers][2] (capacity counts markers). */
lbib_status lbib_read_markers(lbib_handle h, int32_t pid, double* xy, double* nxy, int32_t capacity);

/* Read a field at the current time level into out (capacity in doubles):
 *   which 0: rho = sum_q f_q                                  [ny][nx]
 *   which 1: u_x = (sum_q f_q e_qx + g_x / 2) / rho           [ny][nx]
 *   which 2: u_y likewise                                     [ny][nx]
 *   which 3: the populations f_q, plain FP64                  [9][ny][nx]
 * (the velocity excludes the immersed-boundary force of the coming step). */
lbib_status lbib_read_field(lbib_handle h, int32_t which, double* out, int64_t capacity);

/* Overwrite the populations with plain FP64 values laid out [9][ny][nx] (count = 9 nx ny).
 * Allowed after lbib_init. */
lbib_status lbib_write_populations(lbib_handle h, const double* f, int64_t count);

/* Overwrite the particle's rigid-body state: xc, yc, theta, ux, uy, omega at level n and the
 * same six at level n-1 (12 doubles).  Allowed after lbib_init. */
lbib_status lbib_write_particle(lbib_handle h, int32_t pid, const double* state12);

/* Overwrite the bond flags (count = n_markers; flags on elements without a ligand must be 0). */
lbib_status lbib_write_bonds(lbib_handle h, int32_t pid, const uint8_t* bonded, int32_t count);

/* Record one lbib_particle_state per step into a device buffer of `capacity` records,
 * starting with the next enqueued step (capacity 0 switches recording off). */
lbib_status lbib_trace_enable(lbib_handle h, int32_t pid, int64_t capacity);

/* Copy the recorded states (up to capacity) to out; *count receives the number copied. */
lbib_status lbib_read_trace(lbib_handle h, int32_t pid, lbib_particle_state* out, int64_t capacity,
                            int64_t* count);

/* Checkpoint: with blob == NULL, *size receives the number of bytes needed; otherwise the
 * complete state (populations, particle, bonds, step counter) is written to blob (which
 * holds *size bytes).  lbib_load restores it into a handle created and initialised with the
 * same descriptors and buffer layout (push or pull, rows or planes: a blob of another
 * library build or layout is refused with LBIB_E_INVALID), and clears the failed state. */
lbib_status lbib_save(lbib_handle h, void* blob, int64_t* size);
lbib_status lbib_load(lbib_handle h, const void* blob, int64_t size);

/* Schedule of a step.  Overlapped (mode 1): the particle phases run one after the other on a
 * second stream the handle owns and the lattice sweeps on a third (CU-masked: one CU is left
 * to the particle), with no event between the two chains; they hand over through device
 * memory.  The sweep of step n reads the box step n-1 predicted (exactly) for step n and
 * leaves the node tiles of that box, widened by 3 nodes, to workgroups at the head of its
 * grid, which take them once particle phase n has published its spread force; particle phase
 * n+1 starts once those workgroups have stored step n+1's populations around its box.  Every
 * device-side wait is bounded: one that exceeds about a second fails the simulation with
 * LBIB_E_NUMERIC.  Its two streams must run concurrently: a tool that serialises kernel
 * dispatches (hardware-counter collection) makes those waits time out, so run mode 0 under it.  Serial (mode 0), always on the first step after lbib_init / lbib_load /
 * lbib_write_particle, and where CU masking is unavailable or ny >= 2^23: the particle phase
 * and a sweep of all nodes run one after the other on the handle's stream.  The overlapped
 * schedule's sweep stream is CU-masked, which takes a hardware queue of its own: at most 8
 * simulations per device hold one at a time, and the others run the serial schedule until
 * one of those is destroyed.  Mode 2 (the
 * default) overlaps wherever it can (the faster schedule at every lattice size measured) and
 * runs the particle phases of a call's overlapped steps as one launch (up to 1024 steps each)
 * whose workgroup stays on its CU from step to step; mode 1 launches the particle phase once
 * per step, and such a launch can be dispatched only once a running sweep drains, which may
 * leave it a sweep behind for the rest of the call.  Both schedules give bit-identical
 * results. */
/* Several particles in one lattice: the particle phase is split in two halves over all
 * particles -- first every particle stages its box and spreads its marker forces, then every
 * particle evaluates its probe loads (with the spread force of every particle that reaches a
 * probe node, summed in particle order), bonds and rigid-body update -- and the sweep adds at
 * each node the force of every particle whose box reaches it, in particle order.  Modes 2 (the
 * default) and 4 run both halves as one launch: workgroup b claims particle b, stages the
 * union of its marker and probe supports once, spreads, and waits for every particle's spread
 * before its loads; it waits only while every particle is claimed (a claimer is running), and
 * a workgroup that finds a particle unclaimed (its workgroup not resident, e.g. beside other
 * streams' work) claims and spreads the unclaimed particles itself and then runs the loads
 * half of each particle it holds, so the launch needs no co-residency.  Mode 5 runs that
 * launch on a single workgroup, which takes this path every step (slow; for testing).  Mode 1
 * chains two launches over two streams: the spread launch and the sweep run on the handle's
 * stream, the loads launch on a second stream beside the sweep, and the streams hand over
 * through counters in device memory (a loads launch waits for its step's spreads, the next
 * spread launch for those loads); no launch waits for a later one and no workgroup for another
 * of its own launch.  Modes 0 and 3 run the two launches and the sweep in order on the handle's
 * stream.  Every wait on the device is bounded: past about a second it fails the simulation
 * with LBIB_E_NUMERIC.  For a single particle, mode 3 runs the split phase and modes 4 and 5
 * equal mode 0.  All modes give the same results bit for bit.  Kernel timing reports the spread
 * launch (or the one launch) as kernel 1 and the loads launch as kernel 2 (in the chained
 * schedule its time includes its wait for the spreads). */
lbib_status lbib_set_overlap(lbib_handle h, int32_t mode);

/* Storage layout of the population buffers, chosen before lbib_init: mode 0 push (the
 * buffers hold the streamed populations; the update collides a node and scatters its
 * results to the neighbours), 1 pull (the buffers hold the post-collision populations; the
 * update gathers a node's inflow from the neighbours, collides and stores at the node),
 * 2 (default) push.  Buffers interleave the nine populations row by row, where push is the
 * faster update at the sizes measured; only rows longer than 2^31 / 9 elements fall back to
 * population planes, where mode 2 picks pull once the two buffers exceed 512 MiB (push's
 * shifted stores cost little only while the buffers fit the GPU's 256 MB last-level cache).
 * The layout is
 * invisible at this interface (read-outs, writes and the oracle's populations are the
 * streamed values either way) and results are bit-identical; checkpoints record it and load
 * only into a handle with the same layout.  lbib_get_layout (after lbib_init) gives 1 for
 * pull. */
lbib_status lbib_set_layout(lbib_handle h, int32_t mode);
lbib_status lbib_get_layout(lbib_handle h, int32_t* pull);

/* Kernel timing: HIP events bracket every launch of the kernels selected by the bit mask
 * `enable` (0 switches timing off): bit 0 the lattice sweep (kernel 0), bit 1 the particle
 * phase (kernel 1; in the overlapped schedule the launch includes its wait for the previous
 * sweep, and mode 2's launch over several steps counts as one launch per step), bit 2 the
 * second particle launch of the split phase (kernel 2).  lbib_kernel_time
 * synchronises and returns the summed milliseconds and launch counts since the last enable.
 * The events add work between the launches they time: time whole steps without them. */
lbib_status lbib_kernel_timing(lbib_handle h, int32_t enable);
lbib_status lbib_kernel_time(lbib_handle h, int32_t kernel, double* total_ms, int64_t* launches);

/* Bytes of HBM the algorithm moves per lattice update (9 populations read + 9 written):
 * 144 for FP64 storage, 72 for FP32, 36 for FP16 and BF16. */
lbib_status lbib_bytes_per_update(lbib_handle h, int64_t* bytes);

/* Description of the last failure on this handle; valid until the next call on it. */
const char* lbib_last_error(lbib_handle h);

/* Release everything the handle owns.  NULL-safe. */
void lbib_destroy(lbib_handle h);

/* ---------------------------------------------------------------------------------------
 * Pools: many independent simulations stepped together.
 *
 * A parameter study (the results section sweeps particle shape, ligand density, bond
 * strength and flow rate, with several seeds each) runs many small simulations of the
 * same method.  Stepped one by one, each pays two kernel launches and their gaps per step
 * on a lattice too small to fill the GPU.  A pool runs one launch of the particle phase
 * (one workgroup per member) and one launch of the lattice sweep (the tiles of every
 * member) per time step.  Members may differ in lattice size, tau, Re, particle, ligands
 * and seed; all share the pool's storage precision.  Each member runs until it has done
 * its own n_steps (then idles on the GPU at no sweep cost) or until its watchdog fires
 * (then it stays frozen at the failing step; the others go on).  A member's populations,
 * particle records, bonds and trace are bit-identical to the same descriptors run alone
 * through lbib_create / lbib_init / lbib_step with lbib_set_overlap(h, 0).
 *
 * Members join (lbib_pool_add) and leave (lbib_pool_remove) between calls; admission is
 * by device-memory footprint against the budget given at creation, and is refused with
 * LBIB_E_FULL rather than over-committing HBM.  lbib_pool_add and lbib_pool_remove wait for
 * the pool's stream; lbib_pool_step only enqueues.  Threading and stream rules are those of
 * a simulation handle.
 * ------------------------------------------------------------------------------------- */

typedef struct lbib_pool* lbib_pool_handle;

/* Member states. */
enum { LBIB_POOL_RUNNING = 0, LBIB_POOL_FINISHED = 1, LBIB_POOL_FAILED = 2 };

/* Create a pool.  precision: LBIB_FP64 or LBIB_FP32 storage for every member;
 * hbm_budget_bytes: device memory the members may occupy together, allocated here in one
 * piece (members are placed in it first fit, so joining and leaving never allocate or free
 * device memory; the pool's own tables come on top: about 8 bytes per 256 lattice nodes and
 * 1 KB per member); max_members in [1, 65536]; hip_stream as for lbib_create. */
lbib_status lbib_pool_create(int32_t precision, int64_t hbm_budget_bytes, int32_t max_members, void* hip_stream,
                             lbib_pool_handle* out);

/* Device bytes a member with these descriptors occupies (populations, particle buffers);
 * the admission test of lbib_pool_add. */
lbib_status lbib_pool_footprint(const lbib_lattice_desc* lattice, const lbib_particle_desc* particle,
                                int64_t* bytes);

/* Add a member: one particle with its ligands on the given lattice (descriptors validated
 * as by lbib_create / lbib_particle_add / lbib_ligands_set; lattice->precision must match
 * the pool's), initialised as by lbib_init, to run n_steps steps.  *slot receives its id
 * (ids are never reused within a pool).  LBIB_E_FULL when the budget or max_members would
 * be exceeded, or when no contiguous free part of the budget is large enough; nothing is
 * changed then.  The member's initialisation is enqueued on the pool's stream (the call
 * does not wait for the GPU). */
lbib_status lbib_pool_add(lbib_pool_handle p, const lbib_lattice_desc* lattice, const lbib_particle_desc* particle,
                          const lbib_ligand_desc* ligands, int64_t n_steps, int32_t* slot);

/* Enqueue n pool steps: every running member advances by one step per pool step until it
 * reaches its n_steps. */
lbib_status lbib_pool_step(lbib_pool_handle p, int64_t n);

/* Wait for the enqueued steps and list (up to capacity) the slots that have finished or
 * failed since the previous poll; *count receives how many were written.  Slots beyond
 * capacity are returned by the next poll. */
lbib_status lbib_pool_poll(lbib_pool_handle p, int32_t* slots, int32_t capacity, int32_t* count);

/* Wait, then give a member's completed step count and state (LBIB_POOL_*).  For a failed
 * member, lbib_pool_last_error() then names the watchdog's reason. */
lbib_status lbib_pool_status(lbib_pool_handle p, int32_t slot, int64_t* steps_done, int32_t* state);

/* Read-outs of one member, as the lbib_read_* calls of a simulation handle (they wait for
 * the pool's stream). */
lbib_status lbib_pool_read_particle(lbib_pool_handle p, int32_t slot, lbib_particle_state* out);
lbib_status lbib_pool_read_bonds(lbib_pool_handle p, int32_t slot, uint8_t* bonded, uint8_t* ligand,
                                 int32_t capacity);
lbib_status lbib_pool_read_field(lbib_pool_handle p, int32_t slot, int32_t which, double* out, int64_t capacity);

/* Per-step particle records of one member, as lbib_trace_enable / lbib_read_trace
 * (recording starts with the member's next step). */
lbib_status lbib_pool_trace_enable(lbib_pool_handle p, int32_t slot, int64_t capacity);
lbib_status lbib_pool_read_trace(lbib_pool_handle p, int32_t slot, lbib_particle_state* out, int64_t capacity,
                                 int64_t* count);

/* Remove a member (finished, failed or still running) and release its device memory. */
lbib_status lbib_pool_remove(lbib_pool_handle p, int32_t slot);

/* Members held, members still running (as of the last wait) and bytes of the budget in use. */
lbib_status lbib_pool_usage(lbib_pool_handle p, int32_t* members, int32_t* running, int64_t* bytes_in_use);

/* Kernel timing of the pool's launches: kernel 0 the lattice sweep, kernel 1 the particle
 * phase (as lbib_kernel_timing / lbib_kernel_time). */
lbib_status lbib_pool_kernel_timing(lbib_pool_handle p, int32_t enable);
lbib_status lbib_pool_kernel_time(lbib_pool_handle p, int32_t kernel, double* total_ms, int64_t* launches);

/* Launch shape of the pool's lattice sweep: tiles of tile_x nodes (64, 128 or 256) by
 * 256 / tile_x rows, tiles_per_block consecutive tiles (1, 2, 4 or 8) per workgroup, and,
 * when graph_steps > 0, runs of graph_steps steps replayed as one captured HIP graph
 * (graph_steps <= 4096; kernel timing, when on, uses direct launches).  Results do not
 * depend on these choices.  The default is 256, 4, 0. */
lbib_status lbib_pool_set_config(lbib_pool_handle p, int32_t tile_x, int32_t tiles_per_block, int32_t graph_steps);
lbib_status lbib_pool_get_config(lbib_pool_handle p, int32_t* tile_x, int32_t* tiles_per_block, int32_t* graph_steps);

/* Autotuner: for each tile shape, the sweep's average duration over steps_per_trial steps
 * (HIP events around the sweep launches, best of two rounds); then, for the fastest
 * shape, whole steps with direct launches against graph replay (wall clock, best of two
 * rounds).  Keeps the fastest configuration; *best_step_us (may be NULL) receives its time
 * per step.  The trials are ordinary steps of the running members: about
 * 30 steps_per_trial + 60 steps in total.  Kernel timing is switched off and its counts
 * are reset. */
lbib_status lbib_pool_autotune(lbib_pool_handle p, int32_t steps_per_trial, double* best_step_us);

/* Description of the last failure on this pool (NULL: of the last call with a NULL pool). */
const char* lbib_pool_last_error(lbib_pool_handle p);

/* Release everything the pool owns.  NULL-safe. */
void lbib_pool_destroy(lbib_pool_handle p);

/* ---------------------------------------------------------------------------------------
 * Server: continuous batching of adhesion solves.
 *
 * A request is one solve (lattice, particle, ligands, n_steps).  Requests wait on the host
 * in arrival order and join a pool of the server's as soon as a slot and enough of the
 * memory budget are free, while earlier requests keep stepping: admission is first fit in
 * arrival order, but the request at the head of the queue is passed over by later, smaller
 * ones at most max_bypass times (0: strict arrival order).  The pool steps chunk_steps
 * steps per lbib_server_progress call; a request that completes inside a chunk waits for
 * the chunk's end.  Completed requests leave the pool at once and keep their result until
 * lbib_server_release.  A request's result is bit-identical to the same solve run alone
 * (the bond draws are keyed by the lattice seed, never by the slot).  Times are seconds on
 * the server's clock (a host steady clock started by lbib_server_create).
 * ------------------------------------------------------------------------------------- */

typedef struct lbib_server* lbib_server_handle;

enum { LBIB_REQ_QUEUED = 0, LBIB_REQ_RUNNING = 1, LBIB_REQ_DONE = 2, LBIB_REQ_FAILED = 3 };

typedef struct {
    int64_t id;
    int32_t state; /* LBIB_REQ_* */
    int32_t slot;  /* pool slot while running, else -1 */
    int64_t steps, steps_done;
    int64_t bytes; /* device footprint */
    double t_arrival, t_submit, t_admit, t_done;
    lbib_particle_state final_state; /* the last step's particle record (step -1 before any) */
} lbib_request_result;

/* Create a server: a pool of the given precision, memory budget and member count (as
 * lbib_pool_create), chunk_steps in [1, 10^6] steps per progress call, max_bypass >= 0. */
lbib_status lbib_server_create(int32_t precision, int64_t hbm_budget_bytes, int32_t max_members, int32_t chunk_steps,
                               int32_t max_bypass, void* hip_stream, lbib_server_handle* out);

/* Queue a request (descriptors validated now); arrival_s is its arrival time on the
 * server's clock (negative: now).  LBIB_E_FULL when it alone exceeds the budget. */
lbib_status lbib_server_submit(lbib_server_handle s, const lbib_lattice_desc* lattice,
                               const lbib_particle_desc* particle, const lbib_ligand_desc* ligands, int64_t n_steps,
                               double arrival_s, int64_t* id);

/* One scheduling round: admit what fits, step the pool chunk_steps steps (if anything
 * runs), collect the completed requests.  *n_completed (may be NULL) receives how many
 * completed requests await lbib_server_take_completed. */
lbib_status lbib_server_progress(lbib_server_handle s, int32_t* n_completed);

/* Ids of completed requests, oldest first (up to capacity; the rest stay for the next call). */
lbib_status lbib_server_take_completed(lbib_server_handle s, int64_t* ids, int32_t capacity, int32_t* count);

/* Tracing: every request admitted after this call records the particle record of each of
 * its first `capacity` steps (0 switches it off for later admissions); lbib_server_read_trace
 * copies a completed request's records (up to capacity; *count receives how many).  Each
 * traced admission allocates its record buffer on the device and waits for the server's
 * stream: it is meant for checking results, not for throughput runs.
 * lbib_server_read_bonds: a completed request's bond and ligand flags after its last step
 * (capacity >= n_markers; either output may be NULL).  Both return LBIB_E_STATE for a request
 * that has not completed. */
lbib_status lbib_server_set_trace(lbib_server_handle s, int64_t capacity);
lbib_status lbib_server_read_trace(lbib_server_handle s, int64_t id, lbib_particle_state* out, int64_t capacity,
                                   int64_t* count);
lbib_status lbib_server_read_bonds(lbib_server_handle s, int64_t id, uint8_t* bonded, uint8_t* ligand,
                                   int32_t capacity);

/* A request's current record; lbib_server_release frees a completed one. */
lbib_status lbib_server_result(lbib_server_handle s, int64_t id, lbib_request_result* out);
lbib_status lbib_server_release(lbib_server_handle s, int64_t id);

/* Requests waiting and running, pool bytes in use, chunks stepped so far. */
lbib_status lbib_server_stats(lbib_server_handle s, int32_t* queued, int32_t* running, int64_t* bytes_in_use,
                              int64_t* chunks);

/* The server's pool (for kernel timing and launch configuration; do not add or remove
 * members through it) and its clock. */
lbib_pool_handle lbib_server_pool(lbib_server_handle s);
double lbib_server_clock(lbib_server_handle s);

const char* lbib_server_last_error(lbib_server_handle s);
void lbib_server_destroy(lbib_server_handle s);

/* ---------------------------------------------------------------------------------------
 * Kernel-level entry points.  They run the same device functions as the time step on
 * caller-owned DEVICE buffers, enqueued on hip_stream (NULL = the default stream), so each
 * piece can be checked alone.  n <= 2^31 - 1.
 * ------------------------------------------------------------------------------------- */

/* Philox4x32-10 (Salmon et al., SC'11): out[4i..4i+3] = philox(ctr[4i..4i+3], key[2i..2i+1]). */
lbib_status lbib_kernel_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n,
                               void* hip_stream);

/* MLS shape functions at points pts[2i], pts[2i+1] on an nx x ny lattice (the reading of
 * the paper's MLS reconstruction: nodes within 1.5 per axis, x periodic, wall rows cut;
 * linear basis; cubic B-spline weights of radius 1.5).  For each point and each of the 3 x 3
 * candidate nodes k = 3 dj + di: node[2(9i+k)] = wrapped node i (or -1 when not in the
 * support), node[2(9i+k)+1] = node j; phi, psix, psiy [9 n]. */
lbib_status lbib_kernel_mls(const double* pts, int64_t n, int32_t nx, int32_t ny, int32_t* node, double* phi,
                            double* psix, double* psiy, void* hip_stream);

/* Bond update of n_sets independent particles with nl elements each (eq 10-11): for set s,
 * d[s nl + l] is the element's distance from the receptor wall, ligand / b_in its flags and
 * step[s] its step counter; b_out receives the flags after the update, n_bonds[s] and
 * n_probing[s] the counts.  params = {y_cr, y_eq, sigma, sigma_star, k_f, k_r0, kBT}
 * (host array of 7 doubles).  The draws use key (seed lo, seed hi) and counter
 * (step lo, step hi, l, pid). */
lbib_status lbib_kernel_bonds(const uint8_t* ligand, const double* d, const uint8_t* b_in, uint8_t* b_out,
                              const int64_t* step, int32_t* n_bonds, int32_t* n_probing, int32_t nl,
                              int32_t n_sets, const double* params, uint64_t seed, uint32_t pid,
                              void* hip_stream);

/* Device-to-device copy of `bytes` bytes (a multiple of 16), timed over `iters` repeats on
 * the given stream; *gbps receives the best (read + write) bandwidth in GB/s.  Used as the
 * measured HBM reference for the lattice sweep's roofline. */
lbib_status lbib_bandwidth_probe(int64_t bytes, int32_t iters, void* hip_stream, double* gbps);

/* ---------------------------------------------------------------------------------------
 * Allocation-free solve, for callers that cannot allocate device memory (harnesses that
 * forbid hipMalloc, serving loops that hand out memory from their own pools).
 *
 * Runs what lbib_create / lbib_particle_add / lbib_ligands_set / lbib_init /
 * lbib_set_overlap(h, 0) / lbib_step(n_steps) / lbib_read_trace / lbib_read_bonds run, with
 * the same kernels and bit-identical results, without calling hipMalloc or hipFree: the two
 * population buffers come from the caller, and every other device buffer of the solve (the
 * particle's surface, flags, spread-force tile, box descriptors, node-field overflow,
 * rigid-body state, watchdog word) lives in one static device array of 8 MiB per GPU, which
 * the library holds until the process ends.  A particle whose buffers exceed it (semi-axes
 * above about 170 lattice units) is refused with LBIB_E_INVALID before any GPU work.
 *   populations: DEVICE buffer of *populations_bytes bytes, 256-byte aligned, holding the
 *     two population buffers (their contents on return: the populations after the last
 *     step, in the library's internal storage); NULL: *populations_bytes receives the size
 *     the lattice needs and nothing else is done;
 *   trace: DEVICE buffer of n_steps lbib_particle_state records (record k: step k), or NULL;
 *   bonds: DEVICE buffer of n_markers bytes receiving the bond flags after the last step,
 *     or NULL;
 *   hip_stream: the stream to run on (NULL = the default stream).
 * The call validates like the calls it replaces, enqueues, and waits for its stream before
 * returning: LBIB_E_NUMERIC when the GPU watchdog fired.  Calls on one GPU share its static
 * array (it keeps the last call's contents; a solve initialises what it reads): within a
 * process the library runs them one at a time (a call holds the device's array until its
 * work has finished), since two solves overlapping on the array would race.  Errors are
 * described by lbib_last_error(NULL). */
lbib_status lbib_solve_static(const lbib_lattice_desc* lattice, const lbib_particle_desc* particle,
                              const lbib_ligand_desc* ligands, int64_t n_steps, void* populations,
                              int64_t* populations_bytes, lbib_particle_state* trace, uint8_t* bonds,
                              void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBIB_H */
