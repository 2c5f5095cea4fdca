// lbib_host.hpp -- host pieces shared by the single-simulation handle and the pool:
// descriptor validation, unit conversion (Table 1 groups to lattice units), particle
// preparation, device buffers of a particle and the population download.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "lbib.h"
#include "lbib_geometry.hpp"
#include "lbib_internal.hpp"

namespace lbib {

constexpr int kMaxMarkers = 1024;

// Lattice constants derived from a descriptor.
struct LatticeGeom {
    int nx = 0, ny = 0;
    int row = 0;        // elements per row of one population (nx padded to 256 bytes)
    int pitch = 0;      // elements from a node to the one above it (9 row, or row for planes)
    int64_t plane = 0;  // elements from population q to q + 1 of a node (row, or row ny)
    int64_t mpitch = 0;  // f - f_eq storages: FP32 moment k of (i, j) at k plane + j mpitch + i
    bool interleaved = false;  // rows of nine population segments [j][q][i] (else planes)
    size_t elem = 0;    // bytes per stored population
    bool pull = false;  // buffer layout (push: streamed values; pull: post-collision values)
    int precision = LBIB_FP64;
    double scale = 1.0;  // stored value = (f - w) scale (a power of two; 1 but for FP16)
    double tau = 0, nu = 0, umax = 0, gx = 0, gy = 0;
    int drive = 0;    // 0 body-force Poiseuille, 1 moving top wall (linear shear)
    double uw = 0;    // speed of the top wall (umax for drive 1, else 0)
    bool neq = false;       // values relative to the emitting node's equilibrium, moments beside
    size_t buf_bytes = 0;   // one population buffer: 9 row ny elements (+ 3 row ny FP32 moments)
    int upd_bytes = 0;      // HBM bytes of one lattice update
};

// Host conversions of the 16-bit storages (round to nearest even).
uint16_t f32_to_f16(float f);
float f16_to_f32(uint16_t h);
uint16_t f32_to_bf16(float f);
float bf16_to_f32(uint16_t h);

// Element index of population q of node (i, j) in a buffer of this geometry (the host
// mirror of the device's pop_index).
int64_t host_pop_index(const LatticeGeom& g, int q, int i, int j);

// One particle: host description, surface, ligand layout and its device buffers.
struct Particle {
    lbib_particle_desc desc{};
    lbib_ligand_desc lig{};
    bool has_ligands = false;
    int nl = 0;
    double a = 0, b = 0, mass = 0, inertia = 0;
    Surface surf;
    std::vector<uint8_t> ligand;
    double *d_xi = nullptr, *d_nuv = nullptr, *d_S = nullptr;
    uint8_t *d_lig = nullptr, *d_bond = nullptr;
    int64_t* d_tile = nullptr;
    uint2* d_ring = nullptr;  // split phase: per 32 box nodes, the mask word and the slots before it
    double* d_box = nullptr;  // node fields and node map when they may not fit in LDS
    int box_cap = 0;
    TileDesc* d_desc = nullptr;
    TileDesc* d_zone = nullptr;  // two slots, by step parity
    // the overlapped schedule's hand-over words (0: force-ready count, 1: zone workgroups'
    // count, from 2: four slots of the packed box; ParticleArgs, HandoverArgs) and the side of
    // its widened box at most
    unsigned long long* d_count = nullptr;
    int zone_side = 0;
    DevParticle* d_st = nullptr;
    lbib_particle_state* d_trace = nullptr;
    int64_t trace_cap = 0, trace_start = 0;
    // the device buffers above (trace aside) are carved from one block: owned (freed by
    // free_particle) or provided by the caller (a pool's arena)
    char* block = nullptr;
    bool own_block = false;
    // host staging of the initial upload (kept until the stream-ordered copies have run)
    DevParticle st0{};
    TileDesc td0[2] = {};
    std::vector<uint8_t> zeros;
};

inline bool is_finite(double v) { return std::isfinite(v); }

// Support function of the ellipse along the wall normal: its lowest point is h below the
// centroid.
inline double support_h(double a, double b, double th)
{
    const double s = std::sin(th), c = std::cos(th);
    return std::sqrt(b * b * s * s + a * a * c * c);
}

template <typename T>
hipError_t dalloc(T** p, size_t count)
{
    return hipMalloc((void**)p, (count ? count : 1) * sizeof(T));
}

template <typename T>
void dfree(T*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

// Validation: LBIB_OK, or an error status with the reason in msg.
lbib_status check_lattice(const lbib_lattice_desc& d, std::string& msg);
lbib_status check_ligands(const lbib_ligand_desc& d, std::string& msg);
// Validates the particle against the lattice and fills the host part of p.
lbib_status prepare_particle(const lbib_lattice_desc& lat, const lbib_particle_desc& d, Particle& p, std::string& msg);
void set_ligands(Particle& p, const lbib_ligand_desc& d);
LatticeGeom lattice_geom(const lbib_lattice_desc& d);

// Device bytes a simulation of this lattice and particle (or none) needs.
int64_t footprint_bytes(const lbib_lattice_desc& lat, const Particle* p);

constexpr size_t kAlign = 256;
inline size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// Bytes of the particle's device block (every buffer aligned to 256 bytes).
int zone_workgroups(const Particle& p, bool pull);
size_t particle_block_bytes(const Particle& p);
// Point the particle's buffers into `block` (particle_block_bytes(p) bytes, not owned).
void carve_particle(Particle& p, char* block);
// One owned device block for the particle's buffers.
hipError_t alloc_particle(Particle& p);
void free_particle(Particle& p);
// Geometry, ligands, no bonds and the particle at rest at its initial placement, enqueued
// on `s` (stream-ordered copies from the particle's own staging).
hipError_t upload_particle(Particle& p, hipStream_t s);

template <typename T>
void fill_particle_args(ParticleArgs<T>& a, const LatticeGeom& g, uint64_t seed, const Particle& p, int32_t* flags);

// Constants of a lattice sweep (relaxation, forcing, storage scale, wall speed).
SweepArgs make_sweep_args(const LatticeGeom& g);
// Whether the lattice sweep of step `step` takes its tiles in reverse order (see lbib_host.cpp).
bool reverse_sweep(const LatticeGeom& g, int64_t step);

// The message lbib_last_error(NULL) returns on this thread (calls that fail before they
// have a handle).
void set_null_error(const std::string& msg);

// Initial populations f = f_eq(1, u_poiseuille(y)) (shifted, in the geometry's layout),
// padding zeroed.
hipError_t init_populations(void* f, const LatticeGeom& g, hipStream_t s);

// Plain FP64 populations [9][ny][nx] from a device buffer of shifted ones.
hipError_t download_populations(const void* fdev, const LatticeGeom& g, std::vector<double>& f);
// Overwrite a device buffer with plain FP64 populations [9][ny][nx].
hipError_t upload_populations(void* fdev, const LatticeGeom& g, const double* f);
// rho (which 0), u_x (1), u_y (2) or the populations (3) from plain populations.
void field_from_populations(const std::vector<double>& f, const LatticeGeom& g, int which, double* out);

}  // namespace lbib
