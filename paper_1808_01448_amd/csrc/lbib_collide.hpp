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
__device__ __forceinline__ void neq_encode(T* fout, const SweepArgs& a, int i, int j, const C m[3], C post[9], int pol)
{
    if constexpr (St<T>::neq) {
        float* mo = neq_moments(fout, a.pitch, a.plane, a.ny);
        const size_t c = (size_t)j * neq_mpitch(a.pitch, a.plane) + i;
        const float m0 = (float)m[0], m1 = (float)m[1], m2 = (float)m[2];
        put(mo + c, m0, pol);
        put(mo + a.plane + c, m1, pol);
        put(mo + 2 * a.plane + c, m2, pol);
        C feq[9];
        feq_shift_all<C>((C)m0, (C)m1, (C)m2, feq);
#pragma unroll
        for (int q = 0; q < 9; ++q) post[q] -= feq[q];
    }
}

// Push layout: collide node (i, j), whose populations g load_node presented, and scatter
// its results to the neighbours, with half-way bounce-back at the two walls and periodic x.
// COH: coherent stores (a concurrently running launch reads the results).
template <typename T, bool COH = false>
__device__ __forceinline__ void push_update(T* __restrict__ fout, const SweepArgs& a, int i, int j,
                                            const typename St<T>::C (&g)[9], double Fx, double Fy)
{
    using C = typename St<T>::C;
    const int64_t P = a.plane;
    const size_t c = (size_t)j * a.pitch + i;
    const int pol = COH ? ST_COH : ST_PLAIN;
    C post[9], m[3];
    collide_node<C>(g, a, (C)Fx, (C)Fy, post, m);
    neq_encode<T, C>(fout, a, i, j, m, post, pol);

    const int ip = (i + 1 == a.nx) ? 0 : i + 1;
    const int im = (i == 0) ? a.nx - 1 : i - 1;
    const size_t up = (size_t)(j + 1) * a.pitch, dn = (size_t)(j - 1) * a.pitch, row = (size_t)j * a.pitch;
    const bool top = (j + 1 == a.ny), bot = (j == 0);
    const double sc = a.scale;
    // shifted values reflect unchanged: w_q = w_opp(q)
    st_store(fout, 0 * P + c, post[0], sc, pol);
    st_store(fout, 1 * P + row + ip, post[1], sc, pol);
    st_store(fout, 3 * P + row + im, post[3], sc, pol);
    if (!top) {
        st_store(fout, 2 * P + up + i, post[2], sc, pol);
        st_store(fout, 5 * P + up + ip, post[5], sc, pol);
        st_store(fout, 6 * P + up + im, post[6], sc, pol);
    } else {
        st_store(fout, 4 * P + c, post[2], sc, pol);
        st_store(fout, 7 * P + c, post[5], sc, pol);
        st_store(fout, 8 * P + c, post[6], sc, pol);
    }
    if (!bot) {
        st_store(fout, 4 * P + dn + i, post[4], sc, pol);
        st_store(fout, 7 * P + dn + im, post[7], sc, pol);
        st_store(fout, 8 * P + dn + ip, post[8], sc, pol);
    } else {
        st_store(fout, 2 * P + c, post[4], sc, pol);
        st_store(fout, 5 * P + c, post[7], sc, pol);
        st_store(fout, 6 * P + c, post[8], sc, pol);
    }
}

// Pull layout: collide node (i, j), whose inflow g load_node gathered from the previous
// step's post-collision values (bounce-back across the walls), and store the post-collision
// values at (i, j) itself.  Every store is aligned and each value is written once, so both
// go past the caches; the gathers hit lines neighbouring waves also read.
template <typename T, bool COH = false>
__device__ __forceinline__ void pull_update(T* __restrict__ fout, const SweepArgs& a, int i, int j,
                                            const typename St<T>::C (&g)[9], double Fx, double Fy)
{
    using C = typename St<T>::C;
    const int64_t P = a.plane;
    const size_t c = (size_t)j * a.pitch + i;
    const int pol = COH ? ST_COH : ST_NT;
    C post[9], m[3];
    collide_node<C>(g, a, (C)Fx, (C)Fy, post, m);
    neq_encode<T, C>(fout, a, i, j, m, post, pol);
#pragma unroll
    for (int q = 0; q < 9; ++q) st_store(fout, q * P + c, post[q], a.scale, pol);
}

// The populations of node (i, j) at the start of a step in the compute type, read past the
// caches (they are read once per step).
template <typename T, bool PULL>
__device__ __forceinline__ void update_load(const T* __restrict__ fin, const SweepArgs& a, int i, int j,
                                            typename St<T>::C (&g)[9])
{
    load_node<T, typename St<T>::C>(fin, i, j, a.nx, a.ny, a.pitch, a.plane, PULL, a.inv_scale, a.uw6, true, g);
}

template <typename T, bool PULL, bool COH = false>
__device__ __forceinline__ void update_store(T* __restrict__ fout, const SweepArgs& a, int i, int j,
                                             const typename St<T>::C (&g)[9], double Fx, double Fy)
{
    if (PULL)
        pull_update<T, COH>(fout, a, i, j, g, Fx, Fy);
    else
        push_update<T, COH>(fout, a, i, j, g, Fx, Fy);
}

// Node update in either layout.
template <typename T, bool PULL>
__device__ __forceinline__ void collide_stream(const T* __restrict__ fin, T* __restrict__ fout, const SweepArgs& a,
                                               int i, int j, double Fx, double Fy)
{
    typename St<T>::C g[9];
    update_load<T, PULL>(fin, a, i, j, g);
    update_store<T, PULL>(fout, a, i, j, g, Fx, Fy);
}

// Hand-over of the particle's force tile to the concurrent sweep (HandoverArgs) without cache
// maintenance: loads and stores at agent scope are coherent across the XCDs' L2 caches, so
// the writer only has to wait for its stores to complete before it sets the ready bit.  (A
// release or acquire fence at agent scope writes back or invalidates a whole L2, which
// beside the sweep's store stream costs tens of microseconds.)
__device__ __forceinline__ void coherent_store(int64_t* p, int64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t coherent_load(const int64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void coherent_store(TileDesc* p, const TileDesc& d)
{
    const int64_t* s = (const int64_t*)&d;
#pragma unroll
    for (int k = 0; k < 4; ++k) coherent_store((int64_t*)p + k, s[k]);
}
__device__ __forceinline__ TileDesc coherent_load(const TileDesc* p)
{
    TileDesc d;
    int64_t* s = (int64_t*)&d;
#pragma unroll
    for (int k = 0; k < 4; ++k) s[k] = coherent_load((const int64_t*)p + k);
    return d;
}
// Waits until every store this lane has issued has completed (s_waitcnt vmcnt(0)).
__device__ __forceinline__ void stores_done() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Polls a monotonic hand-over counter (one lane) until it reaches target, sleeping between
// polls.  Gives up after 2^20 polls (about a second) and raises FLAG_SYNC, and returns at
// once while FLAG_SYNC is raised, so a simulation whose hand-over failed drains quickly.
__device__ __forceinline__ void wait_counter(const unsigned long long* p, unsigned long long target, int32_t* flags)
{
    for (unsigned polls = 0; __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target; ++polls) {
        if ((polls & 255u) == 0 && (__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & FLAG_SYNC))
            return;
        if (polls > (1u << 20)) {
            atomicOr(flags, FLAG_SYNC);
            return;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}
__device__ __forceinline__ void publish_counter(unsigned long long* p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A predicted box in two 64-bit words, each carrying a 16-bit tag, so that one coherent
// load of each gives a consistent box (both tags current) without a separate flag: word 0
// i0w (32 bits), j0 (16); word 1 w (16), h (16), active (1); tag in the top 16 bits of
// both.  Needs j0, w, h < 2^16.
__device__ __forceinline__ void zone_pack(const TileDesc& z, uint32_t tag, unsigned long long* p)
{
    const unsigned long long t = (unsigned long long)(tag & 0xffffu) << 48;
    const bool ok = z.active && z.j0 < 65536 && z.w < 65536 && z.h < 65536;
    coherent_store((int64_t*)p, (int64_t)(t | ((unsigned long long)(uint32_t)z.j0 << 32) | (uint32_t)z.i0w));
    coherent_store((int64_t*)p + 1, (int64_t)(t | ((unsigned long long)ok << 32) | ((unsigned long long)(uint32_t)z.h << 16) |
                                             (uint32_t)z.w));
}
// Waits (one lane) until both words of the box carry tag, then unpacks it (inactive when the
// wait times out, which raises FLAG_SYNC).  The first attempt uses plain loads: the tags
// validate whatever they return (a stale copy only carries an older tag), and once the box is
// written they mostly hit in the L2 that the first workgroup of the XCD filled.
__device__ __forceinline__ TileDesc zone_wait(const unsigned long long* p, uint32_t tag, int32_t* flags)
{
    TileDesc z{};
    const unsigned long long t = tag & 0xffffu;
    unsigned long long w0 = p[0], w1 = p[1];
    for (unsigned polls = 0;; ++polls) {
        if ((w0 >> 48) == t && (w1 >> 48) == t) {
            z.i0w = (int32_t)(uint32_t)w0;
            z.j0 = (int32_t)((w0 >> 32) & 0xffffu);
            z.w = (int32_t)(w1 & 0xffffu);
            z.h = (int32_t)((w1 >> 16) & 0xffffu);
            z.active = (int32_t)((w1 >> 32) & 1u);
            return z;
        }
        if ((polls & 255u) == 0 && (__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & FLAG_SYNC))
            return z;
        if (polls > (1u << 20)) {
            atomicOr(flags, FLAG_SYNC);
            return z;
        }
        if (polls) __builtin_amdgcn_s_sleep(1);
        w0 = (unsigned long long)coherent_load((const int64_t*)p);
        w1 = (unsigned long long)coherent_load((const int64_t*)p + 1);
    }
}

// Node tiles of a lattice sweep, one per 256-thread workgroup: 256 x 1 in both layouts (a
// wave's x-shifted stores or loads then meet a neighbouring tile's lines at one end of a
// 256-node row segment, not of a 64-node one).  Measured in row-interleaved buffers, FP32
// (median sweep times): push 1 % faster than 128 x 2 and 3 % faster than 64 x 4 at
// 4096 x 1024, about 6 % and 13 % at 8192 x 4096; pull 1-4 % faster than 128 x 2.
template <bool PULL>
struct Tile {
    static constexpr int W = 256, H = 1;
};

// The TW x TH node tiles of the sweep that a box, widened by m nodes on every side, reaches:
// columns tx0, tx0 + 1, ... (ntx of them, periodic over the gx columns; the last column may be
// narrower than TW nodes), rows ty0 .. ty0 + nty - 1.  Zone tile e is column
// (tx0 + e % ntx) mod gx of row ty0 + e / ntx.  The box is inactive, or has i0w in [0, nx),
// w <= nx and rows j0 .. j0 + h - 1 in [0, ny).
struct ZoneTiles {
    int tx0, ntx, ty0, nty;
};
template <int TW, int TH>
__device__ __forceinline__ ZoneTiles zone_tiles(const TileDesc& z, int nx, int ny, int gx, int m)
{
    ZoneTiles t{0, 0, 0, 0};
    if (!z.active || z.w <= 0 || z.h <= 0) return t;
    const int w = min(z.w + 2 * m, nx);
    int i0 = z.i0w - m;
    if (i0 < 0) i0 += nx;
    t.tx0 = i0 / TW;
    int covered = min(TW * t.tx0 + TW, nx) - i0;
    int tx = t.tx0;
    t.ntx = 1;
    while (covered < w && t.ntx < gx) {
        tx = tx + 1 == gx ? 0 : tx + 1;
        covered += min(TW * tx + TW, nx) - TW * tx;
        ++t.ntx;
    }
    t.ty0 = max(z.j0 - m, 0) / TH;
    t.nty = min(z.j0 + z.h - 1 + m, ny - 1) / TH - t.ty0 + 1;
    return t;
}
__device__ __forceinline__ bool zone_has_tile(const ZoneTiles& t, int tx, int ty, int gx)
{
    if (ty < t.ty0 || ty >= t.ty0 + t.nty) return false;
    int k = tx - t.tx0;
    if (k < 0) k += gx;
    return k < t.ntx;
}

__device__ __forceinline__ bool in_box(const TileDesc& d, int i, int j, int nx)
{
    int di = i - d.i0w;
    if (di < 0) di += nx;
    const int dj = j - d.j0;
    return di < d.w && dj >= 0 && dj < d.h;
}

}  // namespace lbib
