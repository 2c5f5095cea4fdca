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

// Footprint of the spread force written by the particle phase and read by the sweep:
// nodes i0w + di (mod nx), j0 + dj for 0 <= di < w, 0 <= dj < h; the force components are
// 64-bit fixed point with value = q * 2^-scale.
struct TileDesc {
    int32_t i0w, j0, w, h;
    int32_t scale;
    int32_t active;
    int32_t pad0, pad1;
};

// Lattice constants of one sweep (the collision is evaluated in FP64 for both storage
// precisions).
struct SweepArgs {
    int32_t nx, ny, pitch;
    int64_t plane;  // elements per population plane (pitch * ny)
    double omega;   // 1 / tau
    double guo;     // 1 - 1 / (2 tau)
    double gx, gy;  // uniform body force
};

// Everything the particle phase needs; passed by value.
template <typename T>
struct ParticleArgs {
    const T* f;  // populations f - w_q at level n
    int32_t nx, ny, pitch;
    int64_t plane;
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
    int64_t* tile;  // [cap_h][cap_w][2] fixed-point spread force
    int32_t cap_w, cap_h;
    TileDesc* desc;
    DevParticle* st;
    lbib_particle_state* trace;
    int64_t trace_cap, trace_start;
    int32_t* flags;
};

// Launchers (lbib_kernels.hip).  All enqueue on `stream` and return the launch status.
template <typename T>
hipError_t launch_init(T* f, int32_t nx, int32_t ny, int32_t pitch, int64_t plane, double umax, hipStream_t stream);
template <typename T>
hipError_t launch_sweep(const T* fin, T* fout, const SweepArgs& a, const TileDesc* desc, const int64_t* tile,
                        hipStream_t stream);
template <typename T>
hipError_t launch_particle(const ParticleArgs<T>& a, hipStream_t stream);

hipError_t launch_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n, hipStream_t stream);
hipError_t launch_mls(const double* pts, int64_t n, int32_t nx, int32_t ny, int32_t* node, double* phi, double* psix,
                      double* psiy, hipStream_t stream);
hipError_t launch_bonds(const uint8_t* ligand, const double* d, const uint8_t* b_in, uint8_t* b_out,
                        const int64_t* step, int32_t* n_bonds, int32_t* n_probing, int32_t nl, int32_t n_sets,
                        const double* params7, uint64_t seed, uint32_t pid, hipStream_t stream);
hipError_t launch_copy(const float4* src, float4* dst, int64_t n, hipStream_t stream);

}  // namespace lbib
