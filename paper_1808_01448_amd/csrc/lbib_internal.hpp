// lbib_internal.hpp -- structures shared by the host runtime and the gfx950 kernels of the
// LB-IB adhesion library.  Nothing here is part of the public C-ABI (include/lbib.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbib.h"

namespace lbib {

// Watchdog bits raised on the device (the same meaning in every kernel).
enum : int32_t {
    FLAG_NONFINITE = 1,  // non-finite force, torque or velocity
    FLAG_CONTACT = 2,    // analytic gap to the receptor wall <= 0
    FLAG_MLS = 4,        // singular MLS moment matrix
    FLAG_TILE = 8,       // spread footprint larger than the allocated tile
    FLAG_SYNC = 16,      // a device-side wait timed out (the grid barrier of the one-launch particle
                         // phase, or a hand-over of the overlapped schedule)
};

// Rigid-body state of one particle, resident in device memory.  Levels n and n-1 feed the
// explicit second-order update (eq 15-16).
struct DevParticle {
    double xc, yc, th, ux, uy, om;        // level n
    double xc1, yc1, th1, ux1, uy1, om1;  // level n-1
    int64_t step;                         // n: the next step to run
    int32_t pad0, pad1;
    lbib_particle_state last;             // record of the last completed step
};

// The particle's box: every node that an MLS support of a marker or probe of one step
// reaches, nodes i0w + di (mod nx), j0 + dj for 0 <= di < w, 0 <= dj < h (i0u is the same
// origin before wrapping).  The spread force on the box is 64-bit fixed point, value =
// q * 2^-scale, laid out [dj][di][2].
struct TileDesc {
    int32_t i0w, j0, w, h;
    int32_t scale;
    int32_t active;
    int32_t i0u, pad;
};

// 16-bit storage types of the shifted populations: IEEE binary16 (of (f - w) 2^S, S a
// power-of-two scale chosen per simulation) and bfloat16 (of f - w).  Plain bit containers:
// every conversion is explicit (round to nearest even).
struct half_t {
    uint16_t b;
};
struct bf16_t {
    uint16_t b;
};
// The same two formats holding f - f_eq(rho, u) of the node that emitted the population (its
// non-equilibrium part, far smaller than f - w), with that node's (rho - 1, u_x, u_y) kept
// beside in FP32: three planes after the nine population planes of the buffer.
struct half_neq_t {
    uint16_t b;
};
struct bf16_neq_t {
    uint16_t b;
};

// Storage traits: the bits in memory, the type the sweep computes in (FP64 for the FP64 and
// FP32 storages, FP32 for every 16-bit one: the loads' equilibria of the emitting nodes, the
// collision and the stored equilibrium of the node's new moments) and whether the stored
// values are relative to the emitting node's equilibrium.
template <typename T>
struct St;
template <>
struct St<double> {
    using raw = double;
    using C = double;
    static constexpr bool neq = false;
};
template <>
struct St<float> {
    using raw = float;
    using C = double;
    static constexpr bool neq = false;
};
template <>
struct St<half_t> {
    using raw = uint16_t;
    using C = float;
    static constexpr bool neq = false;
};
template <>
struct St<bf16_t> {
    using raw = uint16_t;
    using C = float;
    static constexpr bool neq = false;
};
template <>
struct St<half_neq_t> {
    using raw = uint16_t;
    using C = float;
    static constexpr bool neq = true;
};
template <>
struct St<bf16_neq_t> {
    using raw = uint16_t;
    using C = float;
    static constexpr bool neq = true;
};

// Lattice constants of one sweep.
// Division by a divisor that is fixed for a launch, as a multiply and a shift (Granlund and
// Montgomery, "Division by invariant integers using multiplication", PLDI 1994, Theorem 4.2
// with N = 31): with l = ceil(log2 d), s = 31 + l and m = ceil(2^s / d), which is below 2^32,
// floor(n / d) = floor(n m / 2^s) for every 0 <= n < 2^31.  The sweeps split their tile
// index into column and row with it: three scalar instructions instead of a division.
struct FastDiv {
    uint32_t d, m, s;
};
__host__ __device__ constexpr FastDiv make_fastdiv(uint32_t d)
{
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    const uint64_t two_s = 1ull << (31 + l);
    return FastDiv{d, (uint32_t)((two_s + d - 1) / d), 31 + l};
}
__host__ __device__ constexpr uint32_t fdiv(uint32_t n, FastDiv f)
{
    return (uint32_t)(((uint64_t)n * f.m) >> f.s);
}
constexpr bool fastdiv_checks()
{
    const uint32_t ds[] = {1, 2, 3, 5, 7, 31, 32, 33, 255, 256, 257, 1000, 4097, 65535, 65537, 8388607, 8388608};
    const uint32_t ns[] = {0, 1, 2, 3, 255, 256, 4095, 65536, 12345678, 0x7ffffffeu, 0x7fffffffu};
    for (uint32_t d : ds) {
        const FastDiv f = make_fastdiv(d);
        for (uint32_t n : ns)
            for (uint32_t k = 0; k < 3; ++k) {
                const uint32_t x = n >= k ? n - k : n;
                if (fdiv(x, f) != x / d) return false;
            }
        const uint32_t top = 0x7fffffffu / d * d;  // the largest multiple of d, and its neighbours
        if (fdiv(top, f) != top / d || (top && fdiv(top - 1, f) != (top - 1) / d)) return false;
    }
    return true;
}
static_assert(fastdiv_checks(), "multiply-shift division");

struct SweepArgs {
    int32_t nx, ny, pitch;
    int64_t plane;  // elements per population plane (pitch * ny)
    double omega;   // 1 / tau
    double guo;     // 1 - 1 / (2 tau)
    double gx, gy;  // uniform body force
    double scale, inv_scale;  // stored value = (f - w) scale (a power of two; 1 but for FP16)
    double uw6;     // speed of the moving top wall / 6 (0: resting walls); see wall_reflect
    // the FP32 update of the 16-bit storages: omega, 1 - omega, 3 guo, 9 guo, inv_scale (each
    // the double value rounded once)
    float omega_f, keep_f, b3_f, b9_f, inv_scale_f;
};

// Where the sweep and the probes of a multi-particle step find particle p's spread force:
// the box node n = dj w + di carries a force when bit n % 32 of ring[n / 32].x is set; it is
// then entry s = ring[n / 32].y + (set bits below n % 32) of the compact list tile[2 s],
// tile[2 s + 1] (64-bit fixed point, value q 2^-scale).
struct PartRef {
    const TileDesc* desc;
    const int64_t* tile;
    const uint2* ring;
};

// Everything the particle phase needs; passed by value.
template <typename T>
struct ParticleArgs {
    const T* f;   // populations f - w_q at level n (a pool passes the even-step buffer)
    const T* fB;  // a pool's odd-step buffer
    int64_t target_steps;  // a pool member stops at this step count
    int32_t nx, ny, pitch;
    int32_t pull;  // layout of f: 0 push, 1 pull
    int64_t plane;
    double inv_scale;  // f - w = stored value * inv_scale
    double uw6;        // speed of the moving top wall / 6 (wall_reflect)
    double gx, gy, nu;
    // body-frame surface: centroids xi[2l], outward normals nuv[2l], lengths S[l]
    const double* xi;
    const double* nuv;
    const double* S;
    const uint8_t* ligand;
    uint8_t* bond;
    int32_t nl;
    double a, b, mass, inertia;
    double sigma, sigma_star, y_cr, y_eq, k_f, k_r0, kBT, hamaker;
    uint64_t seed;
    uint32_t pid;
    int64_t* tile;      // [box_cap][2] fixed-point spread force on the box (read by the sweep); in
                        // the split phase, the compact list of the nodes the marker supports reach
    uint2* ring;        // split phase: the index of that list (PartRef)
    double* box_global;  // node fields and node map of up to box_cap nodes when they may not fit in LDS
    int32_t box_cap;     // node capacity of the box
    TileDesc* desc;      // this step's box
    TileDesc* zone;      // zone[2]: boxes of future steps, slot = step parity
    int32_t parity_in;   // slot holding this step's box as predicted by the previous step
    int32_t parity_out;  // slot receiving the next step's box
    int32_t check_zone;  // compare this step's box with zone[parity_in]
    DevParticle* st;
    lbib_particle_state* trace;
    int64_t trace_cap, trace_start;
    int32_t* flags;
    // several particles: the step's mask (one 64-bit word of particle bits per 64 x 4 tile,
    // mtx tiles along x) and every particle's box and force tile
    unsigned long long* pmask;
    const PartRef* refs;
    int32_t mtx;
    int32_t nparts;  // entries of refs
    // hand-over of the overlapped schedule (NULL: none): once its tile and desc have completed
    // the particle stores ready_value into the monotonic counter *ready; the sweep tiles of
    // its prediction of the next box go to the two words at zone_words, packed with zone_tag
    // (zone_pack), after its last read of f
    unsigned long long* ready;
    unsigned long long ready_value;
    unsigned long long* zone_words;
    uint32_t zone_tag;
    // the particle launch of the overlapped schedule starts once *zdone reaches zdone_target
    // (the previous sweep's zone workgroups have stored their results; NULL: no wait), and
    // with check_prev checks that its box lies inside the box zone[parity_out] (the previous
    // step's), widened by kZoneMargin - 1
    unsigned long long* zdone;
    unsigned long long zdone_target;
    int32_t check_prev;
    // the one-launch split phase: grid-barrier counter and the value this launch waits for
    unsigned long long* bar;
    unsigned long long bar_target;
};

// Launchers (lbib_sweep.hip, lbib_particle.hip).  All enqueue on `stream` and return the launch status.
// drive 0: the Poiseuille profile of centre-line speed umax; 1: the linear shear profile of
// a top wall moving at umax.
template <typename T>
hipError_t launch_init(T* f, int32_t nx, int32_t ny, int32_t pitch, int64_t plane, double umax, double scale,
                       bool pull, int32_t drive, hipStream_t stream);
// The sweep beside the particle phase of one particle (the overlapped schedule), on its own
// stream with no event between it and the particle's launches.  Every wave reads the sweep
// tiles of this step's box as the previous particle launch predicted it (zone_words, two
// words that carry zone_tag when that launch wrote them; it wrote them after its last read
// of the buffer this sweep overwrites), waiting until the tags match.  The workgroups of the lattice skip every
// node tile the box reaches; nzone more workgroups (a multiple of 8, at most 64), before them
// in the grid, sweep those tiles once the concurrent particle launch has published this step's
// force (desc and tile; *ready reaches ready_target).  No cycle of waits: a sweep waits for
// particle launches already running when it starts; its waiting workgroups (at most 64) leave
// whole CUs for the particle's once the others drain, and the sweep stream leaves one CU out.  The hand-over data use coherent accesses (lbib_collide.hpp);
// a wait that exceeds about a second raises FLAG_SYNC in *flags and goes on, so every
// workgroup finishes.
// The zone workgroups cover the box widened by kZoneMargin nodes and store coherently, then
// count in at *zdone; the next particle launch waits for their count instead of the end of
// the sweep, and reads the populations of its box, which lie in that widened box as long as
// the box moves at most one node per step (the particle checks it).
constexpr int kZoneMargin = 3;
struct HandoverArgs {
    const unsigned long long* zone_words;
    uint32_t zone_tag;
    const TileDesc* desc;
    const int64_t* tile;
    const unsigned long long* ready;
    unsigned long long ready_target;
    unsigned long long* zdone;
    int32_t* flags;
    int32_t nzone;
};
template <typename T>
hipError_t launch_sweep_overlap(const T* fin, T* fout, const SweepArgs& a, const HandoverArgs& c, bool pull,
                                hipStream_t stream, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr, bool rev = false);
// Sweep of a step with several particles: node forces from every particle whose box reaches
// the node (listed by the tile mask mcur, summed in particle order); each block also clears
// its tile's word of mnext, the mask of the next step.
template <typename T>
hipError_t launch_sweep_multi(const T* fin, T* fout, const SweepArgs& a, const unsigned long long* mcur,
                              unsigned long long* mnext, const PartRef* refs, bool pull, hipStream_t stream,
                              hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
// Sweep of every node, with the spread force of desc / tile when desc != NULL.  t0 / t1
// (optional) receive the kernel's own start and end times.  pull selects the layout of the
// population buffers (pop_index in lbib_device.hpp); rev, the reverse tile order
// (reverse_sweep).
template <typename T>
hipError_t launch_sweep(const T* fin, T* fout, const SweepArgs& a, const TileDesc* desc, const int64_t* tile, bool pull,
                        hipStream_t stream, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr, bool rev = false);
// LDS of the particle phase.  particle_lds_aux_bytes: the node mask, its prefix counts, the
// fill queues and the overlap list, which must not exceed 158 KB.  particle_lds_bytes: that
// plus the node fields of every node of a box of box_cap nodes, or 0 when this exceeds
// 158 KB (the particle then needs global scratch for the fields of the nodes its supports
// reach, used when they do not fit in the LDS of the launch).  particle_launch_lds: the
// dynamic LDS a launch gives the particle (the most a workgroup may take when the whole
// box may not fit).
// particle_scratch_bytes: the global scratch a particle needs (0 when its whole box fits).
size_t particle_lds_bytes(int32_t box_cap);
size_t particle_lds_aux_bytes(int32_t box_cap);
size_t particle_launch_lds(int32_t box_cap);
size_t particle_scratch_bytes(int32_t box_cap);
template <typename T>
hipError_t launch_particle(const ParticleArgs<T>& a, hipStream_t stream, hipEvent_t t0 = nullptr,
                           hipEvent_t t1 = nullptr);
// The overlapped schedule's particle phase of nsteps consecutive steps as one launch whose
// workgroup stays on its CU from step to step.  Step step0 + k takes the arguments of a
// launch of that step alone (`a` holds those of step step0): it reads f_even (k even) or f_odd,
// its box slots are (step0 + k) mod 2, its ready value and zone tag advance by k, its zone
// words are the pair at zone_base + 2 ((step0 + k + 1) mod 4), the count it waits for advances
// by k nzone, and every step after the first checks its box against the previous one.
template <typename T>
struct ParticleRun {
    const T* f_even;
    const T* f_odd;
    unsigned long long* zone_base;
    int64_t step0;
    int32_t nsteps;
    int32_t nzone;
};
template <typename T>
hipError_t launch_particle_run(const ParticleArgs<T>& a, const ParticleRun<T>& run, hipStream_t stream,
                               hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
// The two launches of the split particle phase (mode 1: spread and mark; mode 2: loads,
// bonds, update), one workgroup per particle of args[0..n); lds: the dynamic LDS of the
// launch (the most particle_launch_lds of the particles).  ch: the device-side hand-over when
// the two launches run on different streams -- each workgroup starts once *wait has reached
// wait_target (NULL: no wait) and, its phase done, adds 1 to *done (NULL: none) with a
// device-scope release; the wait is bounded and raises FLAG_SYNC.
struct SplitChain {
    const unsigned long long* wait = nullptr;
    unsigned long long wait_target = 0;
    unsigned long long* done = nullptr;
};
template <typename T>
hipError_t launch_particle_split(const ParticleArgs<T>* args, int32_t n, const T* f, unsigned long long* pmask,
                                 int32_t mode, int32_t max_nl, size_t lds, hipStream_t stream,
                                 hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr, const SplitChain& ch = SplitChain{});
// The same phase as one launch of `workgroups` (1..n) workgroups for the n particles: each
// claims a particle and spreads it, they meet before the loads, bonds and update, and a
// workgroup that finds a particle unclaimed there (its workgroup not resident) does that
// particle's work itself, so the launch assumes no co-residency.  bar: four counters that
// only grow, [0] spreads and [3] claims, each at target - n before the launch and at target
// after it.  Fewer workgroups than particles make every launch take that path.
template <typename T>
hipError_t launch_particle_fused(const ParticleArgs<T>* args, int32_t n, int32_t workgroups, const T* f,
                                 unsigned long long* pmask, int32_t max_nl, size_t lds, unsigned long long* bar,
                                 unsigned long long target, hipStream_t stream);

// A pool of independent simulations stepped together (one launch per kernel per step).
// The particle launch runs member active[b] in workgroup b and copies the member's box
// descriptor of the step into ctl[member], with `pad` set to the parity of the step it ran
// (its input buffer: 0 fA, 1 fB), or only pad = -1 when the member did not step (target
// reached, or frozen by its watchdog).  The sweep's blocks are listed in `table`: (member,
// first tile); a block sweeps up to TPB consecutive tiles of BX x 256/BX nodes of that
// member, reading ctl[member] and the member's record side by side.
template <typename T>
struct PoolSweep {
    SweepArgs a;
    T* fA;  // buffer of the even steps
    T* fB;  // buffer of the odd steps
    const int64_t* tile;
    FastDiv gx;      // tiles along x
    int32_t ntiles;  // tiles of this member
};
// Sweep configurations a pool can use: tile width BX in {64, 128, 256} nodes (256/BX rows),
// TPB in {1, 2, 4, 8} tiles per block.
struct PoolSweepConfig {
    int32_t bx, tpb;
};
// lds: the dynamic LDS of the launch (the most particle_launch_lds of the members).
template <typename T>
hipError_t launch_pool_particle(const ParticleArgs<T>* args, const int32_t* active, TileDesc* ctl, int32_t n_active,
                                int32_t max_nl, size_t lds, hipStream_t stream, hipEvent_t t0 = nullptr,
                                hipEvent_t t1 = nullptr);
template <typename T>
hipError_t launch_pool_sweep(const PoolSweep<T>* sims, const TileDesc* ctl, const int2* table, int32_t n_blocks,
                             PoolSweepConfig cfg, hipStream_t stream, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);

hipError_t launch_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n, hipStream_t stream);
hipError_t launch_mls(const double* pts, int64_t n, int32_t nx, int32_t ny, int32_t* node, double* phi, double* psix,
                      double* psiy, hipStream_t stream);
hipError_t launch_bonds(const uint8_t* ligand, const double* d, const uint8_t* b_in, uint8_t* b_out,
                        const int64_t* step, int32_t* n_bonds, int32_t* n_probing, int32_t nl, int32_t n_sets,
                        const double* params7, uint64_t seed, uint32_t pid, hipStream_t stream);
hipError_t launch_copy(const float4* src, float4* dst, int64_t n, hipStream_t stream);

}  // namespace lbib
