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
    constexpr bool f32 = sizeof(C) == 4;
    C omega, keep, b3, b9, r;
    if constexpr (f32) {
        // constants rounded once on the host; the reciprocal instruction (1 ulp) for the
        // divide, whose error sits far below the 16-bit storage's rounding
        omega = a.omega_f;
        keep = a.keep_f;
        b3 = a.b3_f;
        b9 = a.b9_f;
        r = drho * __builtin_amdgcn_rcpf((C)1 + drho);
    } else {
        omega = (C)a.omega;
        keep = (C)1 - omega;
        b3 = (C)3 * (C)a.guo;
        b9 = (C)9 * (C)a.guo;
        r = drho / ((C)1 + drho);
    }
    const C jxF = fma((C)0.5, Fx, jx), jyF = fma((C)0.5, Fy, jy);
    const C ux = fma(-jxF, r, jxF), uy = fma(-jyF, r, jyF);
    const C uu = fma(ux, ux, uy * uy);
    const C uF = fma(ux, Fx, uy * Fy);
    const C orho = fma(omega, drho, omega);  // omega rho
    const C a3 = (C)3 * orho, a45 = (C)4.5 * orho;
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

// ---------------------------------------------------------------------------------------
// Addressing of the sweeps.  Every sweep tile is at least one wave wide and exactly one row
// per wave, so the row j of a node is the same for all lanes of its wave: each (row,
// population) segment's base address is formed in scalar registers, and each lane adds the
// 32-bit byte offset of its column, which the loads and stores take as their vector operand.
// (A 64-bit address per lane and access costs two to three vector instructions; in the
// 16-bit storages that was a third of the work of a node.)  The bases are running sums, one
// 64-bit scalar addition of a plane or a row per segment, rather than a 64-bit product per
// segment: scalar instructions issue at the rate of vector ones, one per cycle per CU.  The
// update functions below take j wave-uniform and i in [0, nx).
// ---------------------------------------------------------------------------------------
// An opaque copy of a lane's 32-bit offset (no instruction): the compiler can then neither
// widen it to 64 bits nor push the base addition into the arms of a select that formed it.
__device__ __forceinline__ uint32_t opaque(uint32_t v)
{
    asm("" : "+v"(v));
    return v;
}
struct Cols {
    uint32_t o[3];  // byte offsets of the columns i - 1, i, i + 1 (periodic)
};
template <typename S>
__device__ __forceinline__ Cols cols(int i, int nx)
{
    const uint32_t im = i == 0 ? nx - 1 : i - 1, ip = i + 1 == nx ? 0 : i + 1, sz = sizeof(S);
    return Cols{{opaque(im * sz), opaque((uint32_t)i * sz), opaque(ip * sz)}};
}
// A wave-uniform pointer passed through readfirstlane (a no-op on such a value): the compiler
// keeps it whole in scalar registers, cannot fold a lane's offset into it, and cannot turn a
// chain of such bases back into products.  It is rebuilt as a global-memory pointer, so the
// accesses stay global ones.
template <typename S>
__device__ __forceinline__ S* sbase(S* p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (S*)(__attribute__((address_space(1))) S*)(((uint64_t)hi << 32) | lo);
}
template <typename S>
__device__ __forceinline__ const S* sbase(const S* p)
{
    return sbase(const_cast<S*>(p));
}
// The segment n elements on from base b.
template <typename S>
__device__ __forceinline__ S* snext(S* b, int64_t n)
{
    return sbase(b + n);
}
// The element at byte offset off from base b.
template <typename S>
__device__ __forceinline__ S* at(S* b, uint32_t off)
{
    return (S*)((__attribute__((address_space(1))) char*)(__attribute__((address_space(1))) S*)sbase(b) + off);
}
__device__ __forceinline__ int wave_row(int j) { return __builtin_amdgcn_readfirstlane(j); }

// Columns i - 1, i, i + 1 (periodic) of one row segment of a float plane, for a wave whose
// active lanes hold the consecutive columns of one row (lane L at column i0 + L; lanes past the
// row's end inactive): each lane loads its own column and takes its neighbours' values from
// the adjacent lanes by one-lane wave shifts; the two values beyond the wave's ends come from
// scalar loads and go to its first and last active lane.  One aligned load per row segment
// instead of three, two of them straddling cache lines.
struct WaveCols {
    uint32_t own;      // byte offset of the lane's column
    int left, right;   // the columns beyond the wave's two ends (wave-uniform)
    bool first, last;  // the lane is the wave's first / last active one
};
__device__ __forceinline__ WaveCols wave_cols(int i, int nx)
{
    const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    const int i0 = __builtin_amdgcn_readfirstlane(i - lane);
    const int nact = min(64, nx - i0);
    WaveCols w;
    w.own = opaque((uint32_t)i * 4u);
    w.left = i0 == 0 ? nx - 1 : i0 - 1;
    w.right = i0 + nact == nx ? 0 : i0 + nact;
    w.first = lane == 0;
    w.last = lane == nact - 1;
    return w;
}
__device__ __forceinline__ void row_trio(const float* b, const WaveCols& w, float (&v)[3])
{
    const float c = *at(b, w.own);
    const float hl = sbase(b)[w.left], hr = sbase(b)[w.right];
    const int ci = __builtin_bit_cast(int, c);
    // DPP wave_shr:1 (lane L reads lane L - 1) and wave_shl:1 (lane L reads lane L + 1)
    const float sl = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(ci, ci, 0x138, 0xf, 0xf, false));
    const float sr = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(ci, ci, 0x130, 0xf, 0xf, false));
    v[0] = w.first ? hl : sl;
    v[1] = c;
    v[2] = w.last ? hr : sr;
}

// Non-equilibrium storages: the post-collision values leave relative to the equilibrium of
// the moments stored for this node (rounded to FP32 first, so that every reader forms the same
// equilibrium from them), and the moments are stored at the node.
template <typename T, typename C>
__device__ __forceinline__ void neq_encode(T* fout, const SweepArgs& a, int i, int j, const C m[3], C post[9], int pol)
{
    if constexpr (St<T>::neq) {
        float* m0p = sbase(neq_moments(fout, a.pitch, a.plane, a.ny) + (int64_t)j * neq_mpitch(a.pitch, a.plane));
        float* m1p = snext(m0p, a.plane);
        float* m2p = snext(m1p, a.plane);
        const uint32_t o = (uint32_t)i * 4u;
        const float m0 = (float)m[0], m1 = (float)m[1], m2 = (float)m[2];
        put(at(m0p, o), m0, pol);
        put(at(m1p, o), m1, pol);
        put(at(m2p, o), m2, pol);
        const C x = (C)m1, y = (C)m2;
        const FeqNode<C> n = feq_node<C>((C)m0, x, y);
        post[0] = fma(-(C)kW[0], feq_r0<C>(n), post[0]);
#pragma unroll
        for (int q = 1; q < 9; ++q) post[q] = fma(-(C)kW[q], feq_r<C>(n, e_dot<C>(q, x, y)), post[q]);
    }
}

// Push layout: collide node (i, j), whose populations update_load presented, and scatter
// its results to the neighbours, with half-way bounce-back at the two walls and periodic x.
// COH: coherent stores (a concurrently running launch reads the results).
template <typename T, bool COH = false>
__device__ __forceinline__ void push_update(T* __restrict__ fout, const SweepArgs& a, int i, int j,
                                            const typename St<T>::C (&g)[9], double Fx, double Fy)
{
    using C = typename St<T>::C;
    j = wave_row(j);
    const int64_t P = a.plane, R = a.pitch;
    const int pol = COH ? ST_COH : ST_PLAIN;
    C post[9], m[3];
    collide_node<C>(g, a, (C)Fx, (C)Fy, post, m);
    neq_encode<T, C>(fout, a, i, j, m, post, pol);

    const Cols c = cols<T>(i, a.nx);
    const bool top = (j + 1 == a.ny), bot = (j == 0);
    const double sc = a.scale;
    auto out = [&](T* b, uint32_t o, C v) { st_store(at(b, o), 0, v, sc, pol); };
    // every value is stored once: along e_q into plane q of the neighbour in the row above
    // (q = 2, 5, 6), below (4, 7, 8) or alongside; where that link crosses a wall it reflects
    // into plane opp(q) of the node itself (shifted values reflect unchanged: w_q = w_opp(q))
    T* b[9];
    b[0] = sbase(fout + (int64_t)j * R);
#pragma unroll
    for (int q = 1; q < 9; ++q) b[q] = snext(b[q - 1], P);
    out(b[0], c.o[1], post[0]);
    out(b[1], c.o[2], post[1]);
    out(b[3], c.o[0], post[3]);
    out(top ? b[4] : snext(b[2], R), c.o[1], post[2]);
    out(top ? b[7] : snext(b[5], R), opaque(top ? c.o[1] : c.o[2]), post[5]);
    out(top ? b[8] : snext(b[6], R), opaque(top ? c.o[1] : c.o[0]), post[6]);
    out(bot ? b[2] : snext(b[4], -R), c.o[1], post[4]);
    out(bot ? b[5] : snext(b[7], -R), opaque(bot ? c.o[1] : c.o[0]), post[7]);
    out(bot ? b[6] : snext(b[8], -R), opaque(bot ? c.o[1] : c.o[2]), post[8]);
}

// Pull layout: collide node (i, j), whose inflow update_load gathered from the previous
// step's post-collision values (bounce-back across the walls), and store the post-collision
// values at (i, j) itself.  Every store is aligned and each value is written once, so both
// go past the caches; the gathers hit lines neighbouring waves also read.
template <typename T, bool COH = false>
__device__ __forceinline__ void pull_update(T* __restrict__ fout, const SweepArgs& a, int i, int j,
                                            const typename St<T>::C (&g)[9], double Fx, double Fy)
{
    using C = typename St<T>::C;
    j = wave_row(j);
    const int pol = COH ? ST_COH : ST_NT;
    C post[9], m[3];
    collide_node<C>(g, a, (C)Fx, (C)Fy, post, m);
    neq_encode<T, C>(fout, a, i, j, m, post, pol);
    T* b = sbase(fout + (int64_t)j * a.pitch);
    const uint32_t o = (uint32_t)i * (uint32_t)sizeof(T);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        st_store(at(b, o), 0, post[q], a.scale, pol);
        if (q < 8) b = snext(b, a.plane);
    }
}

// The populations of node (i, j) at the start of a step in the compute type, read past the
// caches (they are read once per step): the values load_node presents, addressed by rows.
template <typename T, bool PULL>
__device__ __forceinline__ void update_load(const T* __restrict__ fin, const SweepArgs& a, int i, int j,
                                            typename St<T>::C (&g)[9])
{
    using C = typename St<T>::C;
    j = wave_row(j);
    const int64_t P = a.plane, R = a.pitch;
    const Cols c = cols<T>(i, a.nx);
    const bool top = (j + 1 == a.ny), bot = (j == 0);
    // plane q of the node's own row
    const T* b[9];
    b[0] = sbase(fin + (int64_t)j * R);
#pragma unroll
    for (int q = 1; q < 9; ++q) b[q] = snext(b[q - 1], P);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        // push: the value at the node itself; pull: the one (i - e_x, j - e_y) emitted along
        // e_q, or the node's own along opp(q) where that link crosses a wall (pop_index)
        const T* p = b[q];
        uint32_t o = c.o[1];
        if (PULL && kEy[q] != 0) {
            const bool wall = kEy[q] > 0 ? bot : top;
            p = wall ? b[kOpp[q]] : snext(b[q], -kEy[q] * R);
            o = kEx[q] == 0 ? c.o[1] : opaque(wall ? c.o[1] : c.o[1 - kEx[q]]);
        } else if (PULL) {
            o = c.o[1 - kEx[q]];
        }
        g[q] = (C)st_load(at(p, o), 0, a.inv_scale, true);
    }
    if constexpr (St<T>::neq) {
        // plus the shifted equilibrium of the node that emitted each value (pop_source), from
        // the moments k = 0, 1, 2 of columns i - 1, i, i + 1 of rows j - 1, j, j + 1
        const int64_t mp = neq_mpitch(a.pitch, a.plane);
        const float* m1 = sbase(neq_moments(fin, a.pitch, a.plane, a.ny) + (int64_t)j * mp);
        if (!top && !bot) {
            const WaveCols wc = wave_cols(i, a.nx);
            float mv[3][3][3];  // [row j - 1 + r][moment k][column i - 1 + c]
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const float* b = r == 1 ? m1 : snext(m1, (r - 1) * mp);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    row_trio(b, wc, mv[r][k]);
                    if (k < 2) b = snext(b, P);
                }
            }
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int r = 1 - kEy[q], c = 1 - kEx[q];  // the emitter (i - e_x, j - e_y)
                const C x = (C)mv[r][1][c], y = (C)mv[r][2][c];
                const FeqNode<C> n = feq_node<C>((C)mv[r][0][c], x, y);
                g[q] = fma((C)kW[q], q == 0 ? feq_r0<C>(n) : feq_r<C>(n, e_dot<C>(q, x, y)), g[q]);
            }
        } else {
            // a wall row: a link that crosses the wall reflects, emitted by the node itself
            const float* mr[3][3];
            mr[1][0] = m1;
            mr[0][0] = bot ? m1 : snext(m1, -mp);
            mr[2][0] = top ? m1 : snext(m1, mp);
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                mr[r][1] = snext(mr[r][0], P);
                mr[r][2] = snext(mr[r][1], P);
            }
            const Cols cm = cols<float>(i, a.nx);
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const bool wall = kEy[q] > 0 ? bot : kEy[q] < 0 ? top : false;
                const int r = 1 - kEy[q];  // the emitter's row j - e_y, as an index of mr
                const float* const* rb = wall ? mr[1] : mr[r];
                const uint32_t o = kEx[q] == 0 ? cm.o[1] : opaque(wall ? cm.o[1] : cm.o[1 - kEx[q]]);
                const C x = (C)*at(rb[1], o), y = (C)*at(rb[2], o);
                const FeqNode<C> n = feq_node<C>((C)*at(rb[0], o), x, y);
                const C eu = e_dot<C>(q, x, y);  // e_dir.u = -e_q.u for a reflected population
                g[q] = fma((C)kW[q], q == 0 ? feq_r0<C>(n) : feq_r<C>(n, wall ? -eu : eu), g[q]);
            }
        }
    }
    wall_reflect<C>(g, j, a.ny, a.uw6);
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

// Node tiles of a lattice sweep, one per 256-thread workgroup: 256 x 1 in both layouts (a
// wave's x-shifted stores or loads then meet a neighbouring tile's lines at one end of a
// 256-node row segment, not of a 64-node one).  Measured in row-interleaved buffers, FP32
// (median sweep times): push 1 % faster than 128 x 2 and 3 % faster than 64 x 4 at
// 4096 x 1024, about 6 % and 13 % at 8192 x 4096; pull 1-4 % faster than 128 x 2.
template <bool PULL>
struct Tile {
    static constexpr int W = 256, H = 1;
};
static_assert(Tile<true>::W == Tile<false>::W && Tile<true>::H == Tile<false>::H,
              "the particle phase predicts the box's tiles for either layout");

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

// The sweep tiles of a predicted box (zone_tiles) in two 64-bit words, each carrying a 16-bit
// tag, so that one coherent load of each gives a consistent value (both tags current) without
// a separate flag: word 0 tx0 (24 bits), ty0 (24); word 1 ntx (24), nty (23); tag in the top
// 16 bits of both.  Needs gx < 2^24 and ny < 2^23 (no tiles otherwise).
__device__ __forceinline__ void zone_pack(const ZoneTiles& z, uint32_t tag, unsigned long long* p)
{
    const unsigned long long t = (unsigned long long)(tag & 0xffffu) << 48;
    const bool ok = z.ntx > 0 && z.nty > 0 && z.tx0 < (1 << 24) && z.ntx < (1 << 24) && z.ty0 < (1 << 24) &&
                    z.nty < (1 << 23);
    const unsigned long long w0 = ok ? ((unsigned long long)z.ty0 << 24) | (unsigned long long)z.tx0 : 0ull;
    const unsigned long long w1 = ok ? ((unsigned long long)z.nty << 24) | (unsigned long long)z.ntx : 0ull;
    coherent_store((int64_t*)p, (int64_t)(t | w0));
    coherent_store((int64_t*)p + 1, (int64_t)(t | w1));
}
__device__ __forceinline__ ZoneTiles zone_unpack(unsigned long long w0, unsigned long long w1)
{
    return ZoneTiles{(int)(w0 & 0xffffffu), (int)(w1 & 0xffffffu), (int)((w0 >> 24) & 0xffffffu),
                     (int)((w1 >> 24) & 0x7fffffu)};
}
// Waits (one lane) until both words carry tag, then unpacks them (no tiles when the wait
// times out, which raises FLAG_SYNC).  The first attempt uses plain loads: the tags validate
// whatever they return (a stale copy only carries an older tag), and once the words are
// written they mostly hit in the L2 that the first workgroup of the XCD filled.
__device__ __forceinline__ ZoneTiles zone_wait(const unsigned long long* p, uint32_t tag, int32_t* flags)
{
    const unsigned long long t = tag & 0xffffu;
    unsigned long long w0 = p[0], w1 = p[1];
    for (unsigned polls = 0;; ++polls) {
        if ((w0 >> 48) == t && (w1 >> 48) == t) return zone_unpack(w0, w1);
        if ((polls & 255u) == 0 && (__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & FLAG_SYNC))
            return ZoneTiles{0, 0, 0, 0};
        if (polls > (1u << 20)) {
            atomicOr(flags, FLAG_SYNC);
            return ZoneTiles{0, 0, 0, 0};
        }
        if (polls) __builtin_amdgcn_s_sleep(1);
        w0 = (unsigned long long)coherent_load((const int64_t*)p);
        w1 = (unsigned long long)coherent_load((const int64_t*)p + 1);
    }
}
// The same for a whole wave without a barrier: every lane reads the two words (one cache
// line) and the wave goes by the first lane's values, so the result is wave-uniform.
__device__ __forceinline__ unsigned long long first_lane(unsigned long long v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ ZoneTiles zone_wait_wave(const unsigned long long* p, uint32_t tag, int32_t* flags)
{
    const unsigned long long t = tag & 0xffffu;
    unsigned long long w0 = first_lane(p[0]), w1 = first_lane(p[1]);
    for (unsigned polls = 0;; ++polls) {
        if ((w0 >> 48) == t && (w1 >> 48) == t) return zone_unpack(w0, w1);
        if ((polls & 255u) == 0 &&
            (__builtin_amdgcn_readfirstlane(__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) &
             FLAG_SYNC))
            return ZoneTiles{0, 0, 0, 0};
        if (polls > (1u << 20)) {
            if (__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)) == 0) atomicOr(flags, FLAG_SYNC);
            return ZoneTiles{0, 0, 0, 0};
        }
        if (polls) __builtin_amdgcn_s_sleep(1);
        w0 = first_lane((unsigned long long)coherent_load((const int64_t*)p));
        w1 = first_lane((unsigned long long)coherent_load((const int64_t*)p + 1));
    }
}

__device__ __forceinline__ bool in_box(const TileDesc& d, int i, int j, int nx)
{
    int di = i - d.i0w;
    if (di < 0) di += nx;
    const int dj = j - d.j0;
    return di < d.w && dj >= 0 && dj < d.h;
}

}  // namespace lbib
