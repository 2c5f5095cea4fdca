// lbib_collide.hpp -- the per-node update of the lattice sweep, shared by the sweep of one
// simulation and the sweep of a pool: BGK collision with Guo forcing (eq 1-6) evaluated in
// FP64, and streaming with half-way bounce-back at the two walls (the top one possibly
// moving along x) and periodic x, in the push or the pull layout of the population buffers.
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
// In the shifted variables (rho = 1 + drho) the BGK update with Guo's source is
//   post_q = (1 - omega) g_q + omega (f_eq,q - w_q) + S_q,
//   f_eq,q - w_q = w_q (drho + rho A),  A = 3 e.u + 9/2 (e.u)^2 - 3/2 u^2,
//   S_q = (1 - omega/2) w_q (3 (e.F - u.F) + 9 (e.u)(e.F)),
// with u = j' - j' drho / (1 + drho), j' = sum g e + F/2; no term ever adds the O(1) density
// to the O(1e-5) deviations.  Split by parity in e_q,
//   post_q = (1 - omega) g_q + w_q (I + E_q + O_q),  post_opp(q) = (1 - omega) g_opp(q) + w_q (I + E_q - O_q),
//   I = omega drho - 3/2 omega rho u^2 - 3 (1 - omega/2) u.F,
//   E_q = (e.u) (9/2 omega rho e.u + 9 (1 - omega/2) e.F),  O_q = 3 omega rho e.u + 3 (1 - omega/2) e.F,
// so each pair of opposite directions shares its terms: about half the arithmetic of the
// direction-by-direction form, which sets the time of the FP64 update on FP32 storage.
// Device code is compiled without FMA contraction and the fused operations below are
// explicit, so every kernel that runs this update (either layout, one simulation or a pool)
// computes the same sequence and gives bit-identical results.  The compute type C is FP64
// for the FP64 and FP32 storages and FP32 for the 16-bit ones, whose storage rounding is far
// coarser than FP32 arithmetic.
// ---------------------------------------------------------------------------------------
// m (optional): the (rho - 1, u_x, u_y) the equilibrium was formed with.
template <typename C>
__device__ __forceinline__ void collide_node(const C g[9], const SweepArgs& a, C Fx, C Fy, C post[9], C* m = nullptr)
{
    C drho, jx, jy;
    shifted_moments<C, C>(g, drho, jx, jy);
    const C omega = (C)a.omega, guo = (C)a.guo, keep = (C)1 - omega;
    const C r = drho / ((C)1 + drho);
    const C jxF = fma((C)0.5, Fx, jx), jyF = fma((C)0.5, Fy, jy);
    const C ux = fma(-jxF, r, jxF), uy = fma(-jyF, r, jyF);
    const C uu = fma(ux, ux, uy * uy);
    const C uF = fma(ux, Fx, uy * Fy);
    const C orho = fma(omega, drho, omega);  // omega rho
    const C a3 = (C)3 * orho, a45 = (C)4.5 * orho, b3 = (C)3 * guo, b9 = (C)9 * guo;
    const C iso = fma(-b3, uF, fma((C)-1.5 * orho, uu, omega * drho));
    post[0] = fma(keep, g[0], (C)kW[0] * iso);
    auto pair = [&](int q, int o, C eu, C eF) {
        const C odd = fma(a3, eu, b3 * eF);
        const C even = fma(eu, fma(a45, eu, b9 * eF), iso);
        post[q] = fma(keep, g[q], (C)kW[q] * (even + odd));
        post[o] = fma(keep, g[o], (C)kW[q] * (even - odd));
    };
    pair(1, 3, ux, Fx);
    pair(2, 4, uy, Fy);
    pair(5, 7, ux + uy, Fx + Fy);
    pair(6, 8, uy - ux, Fy - Fx);
    if (m) {
        m[0] = drho;
        m[1] = ux;
        m[2] = uy;
    }
}

// Non-equilibrium storages: the post-collision values leave relative to the equilibrium of
// the moments stored for this node (rounded to FP32 first, so that every reader forms the same
// equilibrium from them), and the moments are stored at the node.
template <typename T, typename C>
__device__ __forceinline__ void neq_encode(T* fout, const SweepArgs& a, size_t c, const C m[3], C post[9], bool nt)
{
    if constexpr (St<T>::neq) {
        float* mo = neq_moments(fout, a.plane);
        const float m0 = (float)m[0], m1 = (float)m[1], m2 = (float)m[2];
        if (nt) {
            __builtin_nontemporal_store(m0, mo + c);
            __builtin_nontemporal_store(m1, mo + a.plane + c);
            __builtin_nontemporal_store(m2, mo + 2 * a.plane + c);
        } else {
            mo[c] = m0;
            mo[a.plane + c] = m1;
            mo[2 * a.plane + c] = m2;
        }
        C feq[9];
        feq_shift_all<C>((C)m0, (C)m1, (C)m2, feq);
#pragma unroll
        for (int q = 0; q < 9; ++q) post[q] -= feq[q];
    }
}

// Push layout: collide node (i, j) and scatter its populations to the neighbours, with
// half-way bounce-back at the two walls and periodic x.
template <typename T>
__device__ __forceinline__ void collide_push(const T* __restrict__ fin, T* __restrict__ fout, const SweepArgs& a,
                                             int i, int j, double Fx, double Fy)
{
    using C = typename St<T>::C;
    const int64_t P = a.plane;
    const size_t c = (size_t)j * a.pitch + i;
    // populations are read exactly once per step: stream them past the caches
    C g[9];
    load_node<T, C>(fin, i, j, a.nx, a.ny, a.pitch, P, false, a.inv_scale, a.uw6, true, g);
    C post[9], m[3];
    collide_node<C>(g, a, (C)Fx, (C)Fy, post, m);
    neq_encode<T, C>(fout, a, c, m, post, false);

    const int ip = (i + 1 == a.nx) ? 0 : i + 1;
    const int im = (i == 0) ? a.nx - 1 : i - 1;
    const size_t up = (size_t)(j + 1) * a.pitch, dn = (size_t)(j - 1) * a.pitch, row = (size_t)j * a.pitch;
    const bool top = (j + 1 == a.ny), bot = (j == 0);
    const double sc = a.scale;
    // shifted values reflect unchanged: w_q = w_opp(q)
    st_store(fout, 0 * P + c, post[0], sc, false);
    st_store(fout, 1 * P + row + ip, post[1], sc, false);
    st_store(fout, 3 * P + row + im, post[3], sc, false);
    if (!top) {
        st_store(fout, 2 * P + up + i, post[2], sc, false);
        st_store(fout, 5 * P + up + ip, post[5], sc, false);
        st_store(fout, 6 * P + up + im, post[6], sc, false);
    } else {
        st_store(fout, 4 * P + c, post[2], sc, false);
        st_store(fout, 7 * P + c, post[5], sc, false);
        st_store(fout, 8 * P + c, post[6], sc, false);
    }
    if (!bot) {
        st_store(fout, 4 * P + dn + i, post[4], sc, false);
        st_store(fout, 7 * P + dn + im, post[7], sc, false);
        st_store(fout, 8 * P + dn + ip, post[8], sc, false);
    } else {
        st_store(fout, 2 * P + c, post[4], sc, false);
        st_store(fout, 5 * P + c, post[7], sc, false);
        st_store(fout, 6 * P + c, post[8], sc, false);
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
    using C = typename St<T>::C;
    const int64_t P = a.plane;
    const size_t c = (size_t)j * a.pitch + i;
    C g[9];
    load_node<T, C>(fin, i, j, a.nx, a.ny, a.pitch, P, true, a.inv_scale, a.uw6, true, g);
    C post[9], m[3];
    collide_node<C>(g, a, (C)Fx, (C)Fy, post, m);
    neq_encode<T, C>(fout, a, c, m, post, true);
#pragma unroll
    for (int q = 0; q < 9; ++q) st_store(fout, q * P + c, post[q], a.scale, true);
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
