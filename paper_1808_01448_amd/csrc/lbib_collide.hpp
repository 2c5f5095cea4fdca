// lbib_collide.hpp -- the per-node update of the lattice sweep, shared by the sweep of one
// simulation and the sweep of a pool: BGK collision with Guo forcing (eq 1-6) evaluated in
// FP64, and streaming with half-way bounce-back at the two walls and periodic x, in the
// push or the pull layout of the population buffers.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lbib_device.hpp"
#include "lbib_internal.hpp"

namespace lbib {

using namespace dev;

// ---------------------------------------------------------------------------------------
// Lattice sweep: collide (eq 1, 2, 4 with the moments of eq 5-6) and stream.
// In the shifted variables (rho = 1 + drho) the equilibrium is
//   f_eq - w = w (drho + A + drho A),  A = 3 e.u + 9/2 (e.u)^2 - 3/2 u^2,
// and u = j' - j' drho / (1 + drho) with j' = sum g e + F/2; neither form ever adds the
// O(1) density to the O(1e-5) deviations.  Device code is compiled without FMA
// contraction and the fused operations below are explicit, so every kernel that runs this
// update (either layout, one simulation or a pool) computes the same sequence and gives
// bit-identical results.
// ---------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void collide_node(const T gs[9], const SweepArgs& a, double Fx, double Fy, T post[9])
{
    double g[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) g[q] = (double)gs[q];
    double drho, jx, jy;
    shifted_moments<double, double>(g, drho, jx, jy);
    const double r = drho / (1.0 + drho);
    const double jxF = fma(0.5, Fx, jx), jyF = fma(0.5, Fy, jy);
    const double ux = fma(-jxF, r, jxF), uy = fma(-jyF, r, jyF);
    const double uu = fma(ux, ux, uy * uy);
    const double uF = fma(ux, Fx, uy * Fy);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const double eu = kEx[q] * ux + kEy[q] * uy;
        const double eF = kEx[q] * Fx + kEy[q] * Fy;
        const double A = fma(4.5 * eu, eu, fma(-1.5, uu, 3.0 * eu));
        const double geq = kW[q] * fma(drho, A, drho + A);
        const double src = a.guo * kW[q] * fma(9.0 * eu, eF, 3.0 * (eF - uF));
        post[q] = (T)(fma(-a.omega, g[q] - geq, g[q]) + src);
    }
}

// Push layout: collide node (i, j) and scatter its populations to the neighbours, with
// half-way bounce-back at the two walls and periodic x.
template <typename T>
__device__ __forceinline__ void collide_push(const T* __restrict__ fin, T* __restrict__ fout, const SweepArgs& a,
                                             int i, int j, double Fx, double Fy)
{
    const int64_t P = a.plane;
    const size_t c = (size_t)j * a.pitch + i;
    // populations are read exactly once per step: stream them past the caches
    T gs[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) gs[q] = __builtin_nontemporal_load(fin + q * P + c);
    T post[9];
    collide_node<T>(gs, a, Fx, Fy, post);

    const int ip = (i + 1 == a.nx) ? 0 : i + 1;
    const int im = (i == 0) ? a.nx - 1 : i - 1;
    const size_t up = (size_t)(j + 1) * a.pitch, dn = (size_t)(j - 1) * a.pitch, row = (size_t)j * a.pitch;
    const bool top = (j + 1 == a.ny), bot = (j == 0);
    // shifted values reflect unchanged: w_q = w_opp(q)
    fout[0 * P + c] = post[0];
    fout[1 * P + row + ip] = post[1];
    fout[3 * P + row + im] = post[3];
    if (!top) {
        fout[2 * P + up + i] = post[2];
        fout[5 * P + up + ip] = post[5];
        fout[6 * P + up + im] = post[6];
    } else {
        fout[4 * P + c] = post[2];
        fout[7 * P + c] = post[5];
        fout[8 * P + c] = post[6];
    }
    if (!bot) {
        fout[4 * P + dn + i] = post[4];
        fout[7 * P + dn + im] = post[7];
        fout[8 * P + dn + ip] = post[8];
    } else {
        fout[2 * P + c] = post[4];
        fout[5 * P + c] = post[7];
        fout[6 * P + c] = post[8];
    }
}

// Pull layout: gather the streamed populations of (i, j) from the previous step's
// post-collision values (bounce-back across the walls), collide, and store the
// post-collision values at (i, j) itself.  Every store is aligned and each value is written
// once, so both go past the caches; the gathers hit lines neighbouring waves also read.
template <typename T>
__device__ __forceinline__ void collide_pull(const T* __restrict__ fin, T* __restrict__ fout, const SweepArgs& a,
                                             int i, int j, double Fx, double Fy)
{
    const int64_t P = a.plane;
    const size_t c = (size_t)j * a.pitch + i;
    T gs[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) gs[q] = __builtin_nontemporal_load(fin + pop_index(q, i, j, a.nx, a.ny, a.pitch, P, true));
    T post[9];
    collide_node<T>(gs, a, Fx, Fy, post);
#pragma unroll
    for (int q = 0; q < 9; ++q) __builtin_nontemporal_store(post[q], fout + q * P + c);
}

// Node update in either layout.
template <typename T, bool PULL>
__device__ __forceinline__ void collide_stream(const T* __restrict__ fin, T* __restrict__ fout, const SweepArgs& a,
                                               int i, int j, double Fx, double Fy)
{
    if (PULL)
        collide_pull<T>(fin, fout, a, i, j, Fx, Fy);
    else
        collide_push<T>(fin, fout, a, i, j, Fx, Fy);
}

__device__ __forceinline__ bool in_box(const TileDesc& d, int i, int j, int nx)
{
    int di = i - d.i0w;
    if (di < 0) di += nx;
    const int dj = j - d.j0;
    return di < d.w && dj >= 0 && dj < d.h;
}

}  // namespace lbib
