// lbib_sweep.hip -- gfx950 lattice kernels of the LB-IB adhesion step: the initial state and
// the lattice sweep (BGK collision with Guo forcing, eq 1-6, then push-streaming with
// half-way bounce-back at the two walls and periodic x).
//
// Populations are stored shifted, g_q = f_q - w_q, as planes [q][j][i] with a row pitch.
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

#include "lbib_device.hpp"
#include "lbib_internal.hpp"

namespace lbib {

using namespace dev;

// ---------------------------------------------------------------------------------------
// Initial state: f = f_eq(1, (u(y), 0)) with the Poiseuille profile of a channel with walls
// at y = -1/2 and y = ny - 1/2.  Stored shifted: g_q = w_q (3 e.u + 9/2 (e.u)^2 - 3/2 u^2).
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void init_kernel(T* f, int nx, int ny, int pitch, int64_t plane, double umax)
{
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int j = blockIdx.y * 4 + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const double H = (double)ny;
    const double u = 4.0 * umax * (j + 0.5) * (H - 0.5 - j) / (H * H);
    const size_t c = (size_t)j * pitch + i;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const double eu = kEx[q] * u;
        f[q * plane + c] = (T)(kW[q] * (3.0 * eu + 4.5 * eu * eu - 1.5 * u * u));
    }
}

template <typename T>
hipError_t launch_init(T* f, int32_t nx, int32_t ny, int32_t pitch, int64_t plane, double umax, hipStream_t stream)
{
    dim3 block(64, 4), grid((nx + 63) / 64, (ny + 3) / 4);
    hipLaunchKernelGGL(init_kernel<T>, grid, block, 0, stream, f, nx, ny, pitch, plane, umax);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Lattice sweep: collide (eq 1, 2, 4 with the moments of eq 5-6) and push-stream.
// In the shifted variables (rho = 1 + drho) the equilibrium is
//   f_eq - w = w (drho + A + drho A),  A = 3 e.u + 9/2 (e.u)^2 - 3/2 u^2,
// and u = j' - j' drho / (1 + drho) with j' = sum g e + F/2; neither form ever adds the
// O(1) density to the O(1e-5) deviations.
// ---------------------------------------------------------------------------------------
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

    double g[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) g[q] = (double)gs[q];
    double drho, jx, jy;
    shifted_moments<double, double>(g, drho, jx, jy);
    const double r = drho / (1.0 + drho);
    const double jxF = jx + 0.5 * Fx, jyF = jy + 0.5 * Fy;
    const double ux = jxF - jxF * r, uy = jyF - jyF * r;
    const double uu = ux * ux + uy * uy;
    const double uF = ux * Fx + uy * Fy;

    T post[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const double eu = kEx[q] * ux + kEy[q] * uy;
        const double eF = kEx[q] * Fx + kEy[q] * Fy;
        const double A = 3.0 * eu + 4.5 * eu * eu - 1.5 * uu;
        const double geq = kW[q] * (drho + A + drho * A);
        const double src = a.guo * kW[q] * (3.0 * (eF - uF) + 9.0 * eu * eF);
        post[q] = (T)(g[q] - a.omega * (g[q] - geq) + src);
    }

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

__device__ __forceinline__ bool in_box(const TileDesc& d, int i, int j, int nx)
{
    int di = i - d.i0w;
    if (di < 0) di += nx;
    const int dj = j - d.j0;
    return di < d.w && dj >= 0 && dj < d.h;
}

// 64 x 4 node tiles over a 1-D grid.  Workgroups are dispatched round-robin over the eight
// XCDs; the remap gives each XCD a contiguous band of tiles, so the x-shifted stores at a
// tile's edge land in cache lines the same XCD's L2 is already writing.
template <typename T, int MODE>
__global__ __launch_bounds__(256) void sweep_kernel(const T* __restrict__ fin, T* __restrict__ fout, SweepArgs a,
                                                    const TileDesc* __restrict__ desc,
                                                    const int64_t* __restrict__ tile, int gx, int nblocks)
{
    int b = blockIdx.x;
    {
        const int q = nblocks >> 3, r = nblocks & 7, x = b & 7, k = b >> 3;
        b = (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
    }
    const int i = (b % gx) * 64 + (int)(threadIdx.x & 63);
    const int j = (b / gx) * 4 + (int)(threadIdx.x >> 6);
    if (i >= a.nx || j >= a.ny) return;
    double Fx = a.gx, Fy = a.gy;
    if (MODE == SWEEP_OUTSIDE) {
        const TileDesc d = *desc;
        if (d.active && in_box(d, i, j, a.nx)) return;
    } else if (desc) {
        const TileDesc d = *desc;
        if (d.active && in_box(d, i, j, a.nx)) {
            int di = i - d.i0w;
            if (di < 0) di += a.nx;
            const int64_t* t = tile + 2 * ((size_t)(j - d.j0) * d.w + di);
            Fx += ldexp((double)t[0], -d.scale);
            Fy += ldexp((double)t[1], -d.scale);
        }
    }
    collide_push<T>(fin, fout, a, i, j, Fx, Fy);
}

// The nodes of the particle's box only.
template <typename T>
__global__ __launch_bounds__(256) void sweep_box_kernel(const T* __restrict__ fin, T* __restrict__ fout, SweepArgs a,
                                                        const TileDesc* __restrict__ desc,
                                                        const int64_t* __restrict__ tile)
{
    const TileDesc d = *desc;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (!d.active || k >= d.w * d.h) return;
    const int di = k % d.w, dj = k / d.w;
    int i = d.i0w + di;
    if (i >= a.nx) i -= a.nx;
    const int j = d.j0 + dj;
    const int64_t* t = tile + 2 * (size_t)k;
    collide_push<T>(fin, fout, a, i, j, a.gx + ldexp((double)t[0], -d.scale), a.gy + ldexp((double)t[1], -d.scale));
}

// Sweep of a pool of independent simulations in one launch.  Block b sweeps up to TPB
// consecutive tiles (BX x 256/BX nodes each) of member table[b].x, starting at tile
// table[b].y; the table lists each member's tiles in order, so after the XCD remap a
// member's tiles share one XCD's L2.  ctl[member] says which buffer the member's particle
// phase just read (0: fA, 1: fB) or that it did not step (-1: nothing to do).  A block pays
// its member lookups once for TPB tiles.
template <typename T, int BX, int TPB>
__global__ __launch_bounds__(256) void pool_sweep_kernel(const PoolSweep<T>* __restrict__ sims,
                                                         const int32_t* __restrict__ ctl,
                                                         const int2* __restrict__ table, int nblocks)
{
    constexpr int BY = 256 / BX;
    int b = blockIdx.x;
    {
        const int q = nblocks >> 3, r = nblocks & 7, x = b & 7, k = b >> 3;
        b = (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
    }
    const int2 e = table[b];
    const int par = ctl[e.x];
    if (par < 0) return;
    const PoolSweep<T>& ps = sims[e.x];
    const T* fin = par ? ps.fB : ps.fA;
    T* fout = par ? ps.fA : ps.fB;
    const SweepArgs a = ps.a;
    const TileDesc d = *ps.desc;
    const int tx = (int)(threadIdx.x % BX), ty = (int)(threadIdx.x / BX);
    const int tend = min(e.y + TPB, ps.ntiles);
    for (int t = e.y; t < tend; ++t) {
        const int i = (t % ps.gx) * BX + tx;
        const int j = (t / ps.gx) * BY + ty;
        if (i >= a.nx || j >= a.ny) continue;
        double Fx = a.gx, Fy = a.gy;
        if (d.active && in_box(d, i, j, a.nx)) {
            int di = i - d.i0w;
            if (di < 0) di += a.nx;
            const int64_t* tl = ps.tile + 2 * ((size_t)(j - d.j0) * d.w + di);
            Fx += ldexp((double)tl[0], -d.scale);
            Fy += ldexp((double)tl[1], -d.scale);
        }
        collide_push<T>(fin, fout, a, i, j, Fx, Fy);
    }
}

template <typename T>
hipError_t launch_pool_sweep(const PoolSweep<T>* sims, const int32_t* ctl, const int2* table, int32_t n_blocks,
                             PoolSweepConfig cfg, hipStream_t stream, hipEvent_t t0, hipEvent_t t1)
{
    if (n_blocks <= 0) return hipSuccess;
#define LBIB_POOL_SWEEP(BX_, TPB_)                                                                                     \
    if (cfg.bx == BX_ && cfg.tpb == TPB_) {                                                                            \
        if (t0 || t1)                                                                                                  \
            hipExtLaunchKernelGGL(pool_sweep_kernel<T, BX_, TPB_>, dim3(n_blocks), dim3(256), 0u, stream, t0, t1, 0u,  \
                                  sims, ctl, table, n_blocks);                                                         \
        else                                                                                                           \
            hipLaunchKernelGGL((pool_sweep_kernel<T, BX_, TPB_>), dim3(n_blocks), dim3(256), 0, stream, sims, ctl,     \
                               table, n_blocks);                                                                       \
        return hipGetLastError();                                                                                      \
    }
    LBIB_POOL_SWEEP(64, 1)
    LBIB_POOL_SWEEP(64, 2)
    LBIB_POOL_SWEEP(64, 4)
    LBIB_POOL_SWEEP(64, 8)
    LBIB_POOL_SWEEP(128, 1)
    LBIB_POOL_SWEEP(128, 2)
    LBIB_POOL_SWEEP(128, 4)
    LBIB_POOL_SWEEP(128, 8)
    LBIB_POOL_SWEEP(256, 1)
    LBIB_POOL_SWEEP(256, 2)
    LBIB_POOL_SWEEP(256, 4)
    LBIB_POOL_SWEEP(256, 8)
#undef LBIB_POOL_SWEEP
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_sweep(const T* fin, T* fout, const SweepArgs& a, int mode, const TileDesc* desc,
                        const int64_t* tile, int32_t box_cap, hipStream_t stream, hipEvent_t t0, hipEvent_t t1)
{
    if (mode == SWEEP_BOX) {
        hipExtLaunchKernelGGL(sweep_box_kernel<T>, dim3((box_cap + 255) / 256), dim3(256), 0u, stream, t0, t1, 0u, fin,
                              fout, a, desc, tile);
        return hipGetLastError();
    }
    const int gx = (a.nx + 63) / 64, gy = (a.ny + 3) / 4, nb = gx * gy;
    if (mode == SWEEP_OUTSIDE)
        hipExtLaunchKernelGGL(sweep_kernel<T, SWEEP_OUTSIDE>, dim3(nb), dim3(256), 0u, stream, t0, t1, 0u, fin, fout, a,
                              desc, tile, gx, nb);
    else
        hipExtLaunchKernelGGL(sweep_kernel<T, SWEEP_ALL>, dim3(nb), dim3(256), 0u, stream, t0, t1, 0u, fin, fout, a,
                              desc, tile, gx, nb);
    return hipGetLastError();
}

template hipError_t launch_init<float>(float*, int32_t, int32_t, int32_t, int64_t, double, hipStream_t);
template hipError_t launch_init<double>(double*, int32_t, int32_t, int32_t, int64_t, double, hipStream_t);
template hipError_t launch_sweep<float>(const float*, float*, const SweepArgs&, int, const TileDesc*, const int64_t*,
                                        int32_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_sweep<double>(const double*, double*, const SweepArgs&, int, const TileDesc*,
                                         const int64_t*, int32_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_pool_sweep<float>(const PoolSweep<float>*, const int32_t*, const int2*, int32_t,
                                             PoolSweepConfig, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_pool_sweep<double>(const PoolSweep<double>*, const int32_t*, const int2*, int32_t,
                                              PoolSweepConfig, hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace lbib
