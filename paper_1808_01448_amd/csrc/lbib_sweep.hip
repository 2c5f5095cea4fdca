// lbib_sweep.hip -- gfx950 lattice kernels of the LB-IB adhesion step: the initial state and
// the lattice sweep (BGK collision with Guo forcing, eq 1-6, then push-streaming with
// half-way bounce-back at the two walls and periodic x).
//
// Populations are stored shifted, g_q = f_q - w_q, at element q plane + j pitch + i (rows of
// nine population segments, or population planes for rows too long for a 32-bit pitch), in
// the push layout (streamed values, scattered to the neighbours after the collision) or the
// pull layout (post-collision values, gathered from the neighbours before it).
// The shift keeps the FP32 storage accurate at the O(1e-4) velocities of the paper's
// capillary flows; the rest state is exactly g = 0.  The collision itself is evaluated in
// FP64 for both storage precisions: in FP32 arithmetic its rounding breaks the exact
// momentum balance of each collision at the 1e-12 level, and at these velocities the
// drift accumulates to ~3e-5 of the particle velocity within 2000 steps, while FP32
// storage alone costs ~3e-8.  The sweep stays bound by HBM traffic either way.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <math.h>
#include <stdint.h>

#include "lbib_collide.hpp"
#include "lbib_device.hpp"
#include "lbib_internal.hpp"

namespace lbib {

using namespace dev;

// ---------------------------------------------------------------------------------------
// Initial state: f = f_eq(1, (u(y), 0)) with the developed profile of a channel with walls
// at y = -1/2 and y = ny - 1/2: Poiseuille (drive 0) or the linear shear of a top wall
// moving at umax (drive 1).  Stored shifted: g_q = w_q (3 e.u + 9/2 (e.u)^2 - 3/2 u^2).
// In the pull layout each stored value is the one that streams into the node and direction
// where the initial state prescribes it.  A value that reaches the top row through a moving
// wall is stored without the wall term, which every load adds (wall_reflect).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double init_u(int j, int ny, double umax, int drive)
{
    const double H = (double)ny;
    return drive == 1 ? umax * (j + 0.5) / H : 4.0 * umax * (j + 0.5) * (H - 0.5 - j) / (H * H);
}

__device__ __forceinline__ double init_value(int q, int j, int ny, double umax, int drive)
{
    const double u = init_u(j, ny, umax, drive);
    const double eu = kEx[q] * u;
    return kW[q] * (3.0 * eu + 4.5 * eu * eu - 1.5 * u * u);
}

template <typename T, bool PULL>
__global__ __launch_bounds__(256) void init_kernel(T* f, int nx, int ny, int pitch, int64_t plane, double umax,
                                                   double scale, int drive)
{
    const double uw6 = drive == 1 ? umax / 6.0 : 0.0;
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int j = blockIdx.y * 4 + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const size_t c = (size_t)j * pitch + i;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        // push: population q of (i, j); pull: the value (i, j) emits along e_q, which arrives
        // as population q at (i + e_x, j + e_y), or reflects into population opp(q) at (i, j)
        const int dj = j + kEy[q];
        double v = !PULL ? init_value(q, j, ny, umax, drive)
                         : (dj >= 0 && dj < ny ? init_value(q, dj, ny, umax, drive)
                                               : init_value(kOpp[q], j, ny, umax, drive));
        // the slot the top row's loads of populations 7 and 8 read
        const int p = !PULL ? q : (dj >= ny ? kOpp[q] : -1);
        if (j == ny - 1 && p == 7) v += uw6;
        if (j == ny - 1 && p == 8) v -= uw6;
        if constexpr (St<T>::neq) {
            // relative to the equilibrium its reader forms from the emitting node's moments
            int si = i, sj = j, dir = q;
            if (!PULL) pop_source(q, i, j, nx, ny, si, sj, dir);
            v -= feq_shift<double>(dir, 0.0, (double)(float)init_u(sj, ny, umax, drive), 0.0);
        }
        st_store(f, q * plane + c, (typename St<T>::C)v, scale, false);
    }
    if constexpr (St<T>::neq) {
        float* m = neq_moments(f, pitch, plane, ny);
        const size_t mc = (size_t)j * neq_mpitch(pitch, plane) + i;
        m[mc] = 0.0f;
        m[plane + mc] = (float)init_u(j, ny, umax, drive);
        m[2 * plane + mc] = 0.0f;
    }
}

template <typename T>
hipError_t launch_init(T* f, int32_t nx, int32_t ny, int32_t pitch, int64_t plane, double umax, double scale,
                       bool pull, int32_t drive, hipStream_t stream)
{
    dim3 block(64, 4), grid((nx + 63) / 64, (ny + 3) / 4);
    if (pull)
        hipLaunchKernelGGL((init_kernel<T, true>), grid, block, 0, stream, f, nx, ny, pitch, plane, umax, scale,
                           (int)drive);
    else
        hipLaunchKernelGGL((init_kernel<T, false>), grid, block, 0, stream, f, nx, ny, pitch, plane, umax, scale,
                           (int)drive);
    return hipGetLastError();
}

// Tiles (Tile<PULL>; 64 x 4 for several particles) over a 1-D grid.  Workgroups are dispatched
// round-robin over the eight XCDs; the remap gives each XCD a contiguous band of tiles, so the
// x-shifted accesses at a tile's edge land in cache lines the same XCD's L2 already holds.
__device__ __forceinline__ int xcd_tile(int b, int nblocks)
{
    const int q = nblocks >> 3, r = nblocks & 7, x = b & 7, k = b >> 3;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// The force at node (i, j): the body force plus, inside the box d, the spread force of its
// dense tile (COHERENT: written by a workgroup running beside this one).
template <bool COHERENT>
__device__ __forceinline__ void box_force(const TileDesc& d, const int64_t* __restrict__ tile, int i, int j, int nx,
                                          double& Fx, double& Fy)
{
    if (d.active && in_box(d, i, j, nx)) {
        int di = i - d.i0w;
        if (di < 0) di += nx;
        const int64_t* t = tile + 2 * ((size_t)(j - d.j0) * d.w + di);
        Fx += ldexp((double)(COHERENT ? coherent_load(t) : t[0]), -d.scale);
        Fy += ldexp((double)(COHERENT ? coherent_load(t + 1) : t[1]), -d.scale);
    }
}

// Every node; the particle's spread force from desc / tile when desc != NULL.  rev: the tiles
// in reverse order (odd steps of a lattice well beyond the last-level cache, so that the first
// tiles read are the last the previous sweep wrote).
template <typename T, bool PULL>
__global__ __launch_bounds__(256) void sweep_kernel(const T* __restrict__ fin, T* __restrict__ fout, SweepArgs a,
                                                    const TileDesc* __restrict__ desc,
                                                    const int64_t* __restrict__ tile, FastDiv gx, int nblocks,
                                                    int rev)
{
    using TL = Tile<PULL>;
    static_assert(TL::W >= 64, "the sweep's addressing takes each wave's nodes from one row");
    int b = xcd_tile(blockIdx.x, nblocks);
    if (rev) b = nblocks - 1 - b;
    const int ty = (int)fdiv((uint32_t)b, gx), tx = b - ty * (int)gx.d;
    const int i = tx * TL::W + (int)threadIdx.x % TL::W;
    const int j = ty * TL::H + (int)threadIdx.x / TL::W;
    if (i >= a.nx || j >= a.ny) return;
    double Fx = a.gx, Fy = a.gy;
    if (desc) box_force<false>(*desc, tile, i, j, a.nx, Fx, Fy);
    collide_stream<T, PULL>(fin, fout, a, i, j, Fx, Fy);
}

// The sweep beside the particle phase (HandoverArgs).  The first nzone workgroups (a multiple
// of 8, so the XCD remap of the others is unchanged) sweep the tiles of the widened box: they
// are dispatched first and wait for the particle's force beside the rest of the sweep rather
// than at its end.  The others sweep the tiles outside it; each loads its populations before
// it learns the box (no launch writes fin during the sweep), so that wait overlaps the loads.
// rev: the other workgroups' tiles in reverse order, as in sweep_kernel.
// At most 64 VGPRs (eight waves per SIMD); for the f - f_eq storages, whose loads of 27
// moments are then issued in small groups with a wait after each, at most 80 (six or seven).
template <typename T, bool PULL>
__global__ __launch_bounds__(256, St<T>::neq ? 7 : 8) void sweep_overlap_kernel(const T* __restrict__ fin,
                                                                                 T* __restrict__ fout, SweepArgs a,
                                                                                 HandoverArgs c, FastDiv gxd,
                                                                                 int nblocks, int rev)
{
    using TL = Tile<PULL>;
    __shared__ ZoneTiles zs;
    __shared__ TileDesc ds;
    const int gx = (int)gxd.d;
    if ((int)blockIdx.x >= c.nzone) {
        int b = xcd_tile((int)blockIdx.x - c.nzone, nblocks);
        if (rev) b = nblocks - 1 - b;
        const int ty = (int)fdiv((uint32_t)b, gxd), tx = b - ty * gx;
        const int i = tx * TL::W + (int)threadIdx.x % TL::W, j = ty * TL::H + (int)threadIdx.x / TL::W;
        const bool in = i < a.nx && j < a.ny;
        typename St<T>::C g[9];
        if (in) update_load<T, PULL>(fin, a, i, j, g);
        // each wave learns the box's tiles by itself (no barrier)
        const ZoneTiles zt = zone_wait_wave(c.zone_words, c.zone_tag, c.flags);
        if (!in || zone_has_tile(zt, tx, ty, gx)) return;
        update_store<T, PULL>(fout, a, i, j, g, a.gx, a.gy);
        return;
    }
    if (threadIdx.x == 0) zs = zone_wait(c.zone_words, c.zone_tag, c.flags);
    __syncthreads();
    const ZoneTiles zt = zs;
    const int nt = zt.ntx * zt.nty;
    const int e0 = (int)blockIdx.x;
    if (e0 < nt) {
        if (threadIdx.x == 0) {
            wait_counter(c.ready, c.ready_target, c.flags);
            ds = coherent_load(c.desc);
        }
        __syncthreads();
        const TileDesc d = ds;
        // one iteration at a time: an unrolled copy of the update would raise the register
        // allocation of the whole kernel, whose other workgroups run the plain update
#pragma unroll 1
        for (int e = e0; e < nt; e += c.nzone) {
            int tx = zt.tx0 + e % zt.ntx;
            if (tx >= gx) tx -= gx;
            const int i = tx * TL::W + (int)threadIdx.x % TL::W;
            const int j = (zt.ty0 + e / zt.ntx) * TL::H + (int)threadIdx.x / TL::W;
            if (i >= a.nx || j >= a.ny) continue;
            typename St<T>::C g[9];
            update_load<T, PULL>(fin, a, i, j, g);
            double Fx = a.gx, Fy = a.gy;
            box_force<true>(d, c.tile, i, j, a.nx, Fx, Fy);
            update_store<T, PULL, true>(fout, a, i, j, g, Fx, Fy);
        }
    }
    // the next particle launch reads these results once every zone workgroup has counted in
    stores_done();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(c.zdone, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sweep of a step with several particles (64 x 4 tiles, a row per wave: those of the tile mask).
template <typename T, bool PULL>
__global__ __launch_bounds__(256) void sweep_multi_kernel(const T* __restrict__ fin, T* __restrict__ fout, SweepArgs a,
                                                          const unsigned long long* __restrict__ mcur,
                                                          unsigned long long* __restrict__ mnext,
                                                          const PartRef* __restrict__ refs, FastDiv gx, int nblocks)
{
    const int b = xcd_tile(blockIdx.x, nblocks);
    const unsigned long long m = mcur[b];
    if (threadIdx.x == 0) mnext[b] = 0ull;
    const int ty = (int)fdiv((uint32_t)b, gx), tx = b - ty * (int)gx.d;
    const int i = tx * 64 + (int)(threadIdx.x & 63);
    const int j = ty * 4 + (int)(threadIdx.x >> 6);
    if (i >= a.nx || j >= a.ny) return;
    double Fx = a.gx, Fy = a.gy;
    for (unsigned long long r = m; r; r &= r - 1) {
        const PartRef pr = refs[__builtin_ctzll(r)];
        const TileDesc d = *pr.desc;
        if (d.active && in_box(d, i, j, a.nx)) {
            int di = i - d.i0w;
            if (di < 0) di += a.nx;
            const int n = (j - d.j0) * d.w + di;
            const uint2 r = pr.ring[n >> 5];
            if ((r.x >> (n & 31)) & 1u) {  // a marker support reaches the node
                const int64_t* t = pr.tile + 2 * ((int)r.y + __popc(r.x & ((1u << (n & 31)) - 1u)));
                Fx += ldexp((double)t[0], -d.scale);
                Fy += ldexp((double)t[1], -d.scale);
            }
        }
    }
    collide_stream<T, PULL>(fin, fout, a, i, j, Fx, Fy);
}

template <typename T>
hipError_t launch_sweep_multi(const T* fin, T* fout, const SweepArgs& a, const unsigned long long* mcur,
                              unsigned long long* mnext, const PartRef* refs, bool pull, hipStream_t stream,
                              hipEvent_t t0, hipEvent_t t1)
{
    const int gx = (a.nx + 63) / 64, gy = (a.ny + 3) / 4, nb = gx * gy;
    if (pull)
        hipExtLaunchKernelGGL(sweep_multi_kernel<T, true>, dim3(nb), dim3(256), 0u, stream, t0, t1, 0u, fin, fout, a,
                              mcur, mnext, refs, make_fastdiv(gx), nb);
    else
        hipExtLaunchKernelGGL(sweep_multi_kernel<T, false>, dim3(nb), dim3(256), 0u, stream, t0, t1, 0u, fin, fout,
                              a, mcur, mnext, refs, make_fastdiv(gx), nb);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep(const T* fin, T* fout, const SweepArgs& a, const TileDesc* desc, const int64_t* tile, bool pull,
                        hipStream_t stream, hipEvent_t t0, hipEvent_t t1, bool rev)
{
    if (pull) {
        using TL = Tile<true>;
        const int gx = (a.nx + TL::W - 1) / TL::W, nb = gx * ((a.ny + TL::H - 1) / TL::H);
        hipExtLaunchKernelGGL(sweep_kernel<T, true>, dim3(nb), dim3(256), 0u, stream, t0, t1, 0u, fin, fout, a, desc,
                              tile, make_fastdiv(gx), nb, (int)rev);
    } else {
        using TL = Tile<false>;
        const int gx = (a.nx + TL::W - 1) / TL::W, nb = gx * ((a.ny + TL::H - 1) / TL::H);
        hipExtLaunchKernelGGL(sweep_kernel<T, false>, dim3(nb), dim3(256), 0u, stream, t0, t1, 0u, fin, fout, a, desc,
                              tile, make_fastdiv(gx), nb, (int)rev);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep_overlap(const T* fin, T* fout, const SweepArgs& a, const HandoverArgs& c, bool pull,
                                hipStream_t stream, hipEvent_t t0, hipEvent_t t1, bool rev)
{
    if (c.nzone < 8 || c.nzone > 64 || c.nzone % 8) return hipErrorInvalidValue;
    if (pull) {
        using TL = Tile<true>;
        const int gx = (a.nx + TL::W - 1) / TL::W, nb = gx * ((a.ny + TL::H - 1) / TL::H);
        hipExtLaunchKernelGGL(sweep_overlap_kernel<T, true>, dim3(nb + c.nzone), dim3(256), 0u, stream, t0, t1, 0u, fin,
                              fout, a, c, make_fastdiv(gx), nb, (int)rev);
    } else {
        using TL = Tile<false>;
        const int gx = (a.nx + TL::W - 1) / TL::W, nb = gx * ((a.ny + TL::H - 1) / TL::H);
        hipExtLaunchKernelGGL(sweep_overlap_kernel<T, false>, dim3(nb + c.nzone), dim3(256), 0u, stream, t0, t1, 0u,
                              fin, fout, a, c, make_fastdiv(gx), nb, (int)rev);
    }
    return hipGetLastError();
}

#define LBIB_SWEEP_INSTANTIATE(T)                                                                               \
    template hipError_t launch_init<T>(T*, int32_t, int32_t, int32_t, int64_t, double, double, bool, int32_t,     \
                                       hipStream_t);                                                             \
    template hipError_t launch_sweep<T>(const T*, T*, const SweepArgs&, const TileDesc*, const int64_t*, bool,     \
                                        hipStream_t, hipEvent_t, hipEvent_t, bool);                               \
    template hipError_t launch_sweep_overlap<T>(const T*, T*, const SweepArgs&, const HandoverArgs&, bool,         \
                                                hipStream_t, hipEvent_t, hipEvent_t, bool);                       \
    template hipError_t launch_sweep_multi<T>(const T*, T*, const SweepArgs&, const unsigned long long*,           \
                                              unsigned long long*, const PartRef*, bool, hipStream_t, hipEvent_t,  \
                                              hipEvent_t);
LBIB_SWEEP_INSTANTIATE(double)
LBIB_SWEEP_INSTANTIATE(float)
LBIB_SWEEP_INSTANTIATE(half_t)
LBIB_SWEEP_INSTANTIATE(bf16_t)
LBIB_SWEEP_INSTANTIATE(half_neq_t)
LBIB_SWEEP_INSTANTIATE(bf16_neq_t)
#undef LBIB_SWEEP_INSTANTIATE

}  // namespace lbib
