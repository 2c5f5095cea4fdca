// lbib_pool_sweep.hip -- gfx950 lattice sweep of a pool of independent simulations (one
// launch for every member's tiles).
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <math.h>
#include <stdint.h>

#include "lbib_collide.hpp"
#include "lbib_device.hpp"
#include "lbib_internal.hpp"

namespace lbib {

// Sweep of a pool of independent simulations in one launch.  Block b sweeps up to TPB
// consecutive tiles (BX x 256/BX nodes each) of member table[b].x, starting at tile
// table[b].y; the table lists each member's tiles in order, so after the XCD remap a
// member's tiles share one XCD's L2.  ctl[member] holds the member's box of this step and,
// in pad, which buffer its particle phase just read (0: fA, 1: fB) or that it did not step
// (-1: nothing to do); it is loaded beside the member's record, so a block waits for two
// dependent loads (its table entry, then both) before its populations.  A block pays these
// lookups once for TPB tiles.  Pool buffers use the pull layout: a pool's
// working set is far larger than the MALL, where the aligned stores of the pull update
// move HBM traffic faster than the shifted stores of the push update (216 members of
// 512-2048 x 128-256 nodes, row-interleaved FP32: pull 665 us per sweep, push 764 us).
template <typename T, int BX, int TPB>
__global__ __launch_bounds__(256) void pool_sweep_kernel(const PoolSweep<T>* __restrict__ sims,
                                                         const TileDesc* __restrict__ ctl,
                                                         const int2* __restrict__ table, int nblocks)
{
    constexpr int BY = 256 / BX;
    static_assert(BX >= 64, "the sweep's addressing takes each wave's nodes from one row");
    int b = blockIdx.x;
    {
        const int q = nblocks >> 3, r = nblocks & 7, x = b & 7, k = b >> 3;
        b = (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
    }
    const int2 e = table[b];
    const TileDesc d = ctl[e.x];
    const PoolSweep<T>& ps = sims[e.x];
    if (d.pad < 0) return;
    const T* fin = d.pad ? ps.fB : ps.fA;
    T* fout = d.pad ? ps.fA : ps.fB;
    const SweepArgs a = ps.a;
    const int tx = (int)(threadIdx.x % BX), ty = (int)(threadIdx.x / BX);
    const int tend = min(e.y + TPB, ps.ntiles);
    for (int t = e.y; t < tend; ++t) {
        const int row = (int)fdiv((uint32_t)t, ps.gx);
        const int i = (t - row * (int)ps.gx.d) * BX + tx;
        const int j = row * BY + ty;
        if (i >= a.nx || j >= a.ny) continue;
        double Fx = a.gx, Fy = a.gy;
        if (d.active && in_box(d, i, j, a.nx)) {
            int di = i - d.i0w;
            if (di < 0) di += a.nx;
            const int64_t* tl = ps.tile + 2 * ((size_t)(j - d.j0) * d.w + di);
            Fx += ldexp((double)tl[0], -d.scale);
            Fy += ldexp((double)tl[1], -d.scale);
        }
        collide_stream<T, true>(fin, fout, a, i, j, Fx, Fy);
    }
}

template <typename T>
hipError_t launch_pool_sweep(const PoolSweep<T>* sims, const TileDesc* ctl, const int2* table, int32_t n_blocks,
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

#define LBIB_POOL_SWEEP_INSTANTIATE(T)                                                                      \
    template hipError_t launch_pool_sweep<T>(const PoolSweep<T>*, const TileDesc*, const int2*, int32_t,         \
                                             PoolSweepConfig, hipStream_t, hipEvent_t, hipEvent_t);
LBIB_POOL_SWEEP_INSTANTIATE(double)
LBIB_POOL_SWEEP_INSTANTIATE(float)
LBIB_POOL_SWEEP_INSTANTIATE(half_t)
LBIB_POOL_SWEEP_INSTANTIATE(bf16_t)
LBIB_POOL_SWEEP_INSTANTIATE(half_neq_t)
LBIB_POOL_SWEEP_INSTANTIATE(bf16_neq_t)
#undef LBIB_POOL_SWEEP_INSTANTIATE

}  // namespace lbib
