// lbib_particle.hip -- gfx950 particle-phase kernels of the LB-IB particle-adhesion step.
//
// The particle phase of step n runs as one workgroup per particle: it stages the node
// fields of the particle's box (every node an MLS support of a marker or probe reaches),
// interpolates the fluid velocity at the Lagrangian markers, forms the direct-forcing
// marker forces and spreads them into a 64-bit fixed-point force field on the box (read by
// the lattice sweep), evaluates the probe loads (eq 7-8), updates the stochastic bonds
// (eq 9-11), adds the wall force (eq 12), reduces force and torque in FP64 and advances the
// rigid body (eq 13-16).  It also predicts the box of step n+1, so the sweep of the nodes
// outside it may run concurrently with the next particle phase.
//
// The file also holds the kernel-level entry points (Philox, MLS, bond update) and the
// copy kernel of the bandwidth probe.
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
// Workgroup reductions: butterfly within each 64-wide wavefront, then the per-wave partials
// in wave order.  The order is fixed, so results are bit-reproducible.
// ---------------------------------------------------------------------------------------
constexpr int PB = 512;       // threads of the particle workgroup
constexpr int NW = PB / 64;   // wavefronts per workgroup

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_isum(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_ior(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_imin(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Sum of N doubles over the workgroup; every thread receives the totals.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double (*sh)[NW])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) sh[k][w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double s = sh[k][0];
#pragma unroll
        for (int u = 1; u < NW; ++u) s += sh[k][u];
        v[k] = s;
    }
    __syncthreads();
}

// Integer combination over the workgroup: op 0 sum, 1 or, 2 min.
template <int N>
__device__ __forceinline__ void block_int(int (&v)[N], const int (&op)[N], int (*sh)[NW])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = op[k] == 0 ? wave_isum(v[k]) : op[k] == 1 ? wave_ior(v[k]) : wave_imin(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) sh[k][w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        int s = sh[k][0];
#pragma unroll
        for (int u = 1; u < NW; ++u) s = op[k] == 0 ? s + sh[k][u] : op[k] == 1 ? (s | sh[k][u]) : min(s, sh[k][u]);
        v[k] = s;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------------------
// Particle phase
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ double fluid_row(double y, int ny)
{
    // transfer points between a wall and the first node row are transferred as if they sat
    // on that row (the linear fit would otherwise extrapolate and destabilise the coupling)
    return y < 0.0 ? 0.0 : (y > ny - 1.0 ? ny - 1.0 : y);
}

// Node range an MLS support at (X, Y) can reach (the candidate box of mls_shape; rows cut at
// the walls).  False for non-finite or absurd points.
__device__ __forceinline__ bool support_range(double X, double Y, int ny, int& ilo, int& ihi, int& jlo, int& jhi)
{
    if (!(fabs(X) < 1e9 && fabs(Y) < 1e9)) return false;
    ilo = (int)floor(X - 1.5) + 1;
    ihi = (int)ceil(X + 1.5) - 1;
    jlo = max((int)floor(Y - 1.5) + 1, 0);
    jhi = min((int)ceil(Y + 1.5) - 1, ny - 1);
    return jhi >= jlo;
}

// Marker l of a particle at (xc, yc, theta): position, outward normal and probe point.
struct MarkerGeo {
    double X, Y, nx, ny, px, py;
};

// (bx, by): body-frame centroid of the element, (mx, my): its body-frame outward normal.
__device__ __forceinline__ MarkerGeo marker_geo(double bx, double by, double mx, double my, double xc, double yc,
                                                double cth, double sth, int ny)
{
    MarkerGeo g;
    g.X = xc + cth * bx - sth * by;
    g.Y = yc + sth * bx + cth * by;
    g.nx = cth * mx - sth * my;
    g.ny = sth * mx + cth * my;
    g.px = g.X + 1.2 * g.nx;  // probe 1.2 dx along the outward normal (below eq 8)
    g.py = fluid_row(g.Y + 1.2 * g.ny, ny);
    return g;
}

// LDS of the particle phase (dynamic, lds_bytes bytes), in this order: the probe launch's
// list of the particles whose boxes overlap this one (kMaxParticles entries), mask[wcap]
// (one bit per box node, set where a support of this launch reaches), pre[wcap] (the
// marked nodes before each mask word) and, when they fit, the node fields and the node map
// (slot -> box node) of the marked nodes; otherwise those live in the global scratch
// box_global.  wcap = ceil(box_cap / 32).  A marked node's slot is its rank among the
// marked nodes in row-major box order, so the fields take kSlotBytes per node of the ring
// that the supports cover next to the surface, not per node of the box.
struct NodeView {
    double *rho, *ux, *uy, *inv;    // density, u* (velocity with half the uniform drive and without
                                    // the spread force), 1/rho
    unsigned long long *fx, *fy;    // this particle's fixed-point spread force; in the probe launch
                                    // of several particles, the total spread force (FP64 bits)
};

// A particle whose box of this step overlaps the box of the particle running the probe
// launch, with where its spread force lies (PartRef); pid: its index.
struct OvEntry {
    const int64_t* tile;
    const uint2* ring;
    int32_t i0w, j0, w, h, scale, pid;
};

constexpr int kMaxParticles = 64;
constexpr int kFields = 6;                      // per marked node: 4 doubles + 2 64-bit integers
constexpr size_t kSlotBytes = kFields * 8 + 4;  // the fields and the node map entry
constexpr int kFillU = 4;                       // marked nodes per lane in flight while summing forces
constexpr size_t kLdsMax = 158 * 1024;          // dynamic LDS a workgroup may take beside the static part
constexpr size_t kLdsHead = sizeof(OvEntry) * kMaxParticles;

size_t particle_lds_aux_bytes(int32_t box_cap)
{
    return kLdsHead + (size_t)((box_cap + 31) / 32) * 8;
}

size_t particle_lds_bytes(int32_t box_cap)
{
    const size_t bytes = particle_lds_aux_bytes(box_cap) + (size_t)box_cap * kSlotBytes;
    return bytes <= kLdsMax ? bytes : 0;
}

size_t particle_launch_lds(int32_t box_cap)
{
    const size_t bytes = particle_lds_bytes(box_cap);
    return bytes ? bytes : kLdsMax;
}

size_t particle_scratch_bytes(int32_t box_cap)
{
    return particle_lds_bytes(box_cap) ? 0 : (size_t)box_cap * kSlotBytes;
}

// The markers of this thread (l = threadIdx.x + k PB) at one position of the particle.
template <int MPT>
struct MarkerSet {
    double X[MPT], Y[MPT], NX[MPT], NY[MPT], PX[MPT], PY[MPT];
    bool in[MPT];
};

// Per-marker surface data of this thread's markers, read once at the start of the launch
// (so the loads overlap): body-frame centroid and normal, element length, ligand and bond
// flags at the start of the step.
template <int MPT>
struct MarkerData {
    double bx[MPT], by[MPT], mx[MPT], my[MPT], S[MPT];
    bool lig[MPT], bnd[MPT];
};

template <int MPT>
__device__ __forceinline__ void marker_set(const MarkerData<MPT>& D, int nl, int ny, double xc, double yc, double cth,
                                           double sth, MarkerSet<MPT>& G)
{
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
        const int l = threadIdx.x + k * PB;
        G.in[k] = l < nl;
        G.X[k] = G.Y[k] = G.NX[k] = G.NY[k] = G.PX[k] = G.PY[k] = 0.0;
        if (G.in[k]) {
            const MarkerGeo g = marker_geo(D.bx[k], D.by[k], D.mx[k], D.my[k], xc, yc, cth, sth, ny);
            G.X[k] = g.X;
            G.Y[k] = g.Y;
            G.NX[k] = g.nx;
            G.NY[k] = g.ny;
            G.PX[k] = g.px;
            G.PY[k] = g.py;
        }
    }
}

// Bounding box (unwrapped x) of every marker and probe support of the set: minima of
// (i_lo, -i_hi, j_lo, -j_hi) accumulated into r[4].
template <int MPT>
__device__ __forceinline__ void set_bounds(const MarkerSet<MPT>& G, int ny, int (&r)[4])
{
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
        if (!G.in[k]) continue;
#pragma unroll
        for (int pt = 0; pt < 2; ++pt) {
            int ilo, ihi, jlo, jhi;
            const bool ok = pt == 0 ? support_range(G.X[k], fluid_row(G.Y[k], ny), ny, ilo, ihi, jlo, jhi)
                                    : support_range(G.PX[k], G.PY[k], ny, ilo, ihi, jlo, jhi);
            if (ok) {
                r[0] = min(r[0], ilo);
                r[1] = min(r[1], -ihi);
                r[2] = min(r[2], jlo);
                r[3] = min(r[3], -jhi);
            }
        }
    }
}

// Set the mask bits of the support window at (X, Y) (the full window of mls_shape: nodes of
// zero weight are read too, multiplied by zero); a window row is at most 3 nodes, so one
// atomic per mask word it touches.
__device__ __forceinline__ void mark_window(double X, double Y, int ny, int x0, int y0, int w, int h, uint32_t* mask)
{
    int ilo, ihi, jlo, jhi;
    if (!support_range(X, Y, ny, ilo, ihi, jlo, jhi)) return;
    ilo = max(ilo - x0, 0);
    ihi = min(ihi - x0, w - 1);
    jlo = max(jlo - y0, 0);
    jhi = min(jhi - y0, h - 1);
    if (ihi < ilo) return;
    const uint64_t run = (1ull << (ihi - ilo + 1)) - 1ull;
    for (int j = jlo; j <= jhi; ++j) {
        const int n = j * w + ilo;
        const uint64_t bits = run << (n & 31);
        atomicOr(mask + (n >> 5), (uint32_t)bits);
        if (bits >> 32) atomicOr(mask + (n >> 5) + 1, (uint32_t)(bits >> 32));
    }
}

// which: bit 0 the marker windows, bit 1 the probe windows.
template <int MPT>
__device__ __forceinline__ void mark_windows(const MarkerSet<MPT>& G, int ny, int which, int x0, int y0, int w, int h,
                                             uint32_t* mask)
{
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
        if (!G.in[k]) continue;
        if (which & 1) mark_window(G.X[k], fluid_row(G.Y[k], ny), ny, x0, y0, w, h, mask);
        if (which & 2) mark_window(G.PX[k], G.PY[k], ny, x0, y0, w, h, mask);
    }
}

// Exclusive prefix of the popcounts of mask[0..nw) into pre; returns the total to every
// thread.  Thread t takes a run of consecutive words, so the runs are in word order.
__device__ __forceinline__ int mask_prefix(const uint32_t* mask, int* pre, int nw, int (*sh)[NW])
{
    const int per = (nw + PB - 1) / PB;
    const int w0 = min((int)threadIdx.x * per, nw), w1 = min(w0 + per, nw);
    int s = 0;
    for (int k = w0; k < w1; ++k) s += __popc(mask[k]);
    const int lane = threadIdx.x & 63;
    int incl = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int v = __shfl_up(incl, d, 64);
        if (lane >= d) incl += v;
    }
    if (lane == 63) sh[0][threadIdx.x >> 6] = incl;
    __syncthreads();
    int run = incl - s, total = 0;
#pragma unroll
    for (int u = 0; u < NW; ++u) {
        const int v = sh[0][u];
        if (u < (int)(threadIdx.x >> 6)) run += v;
        total += v;
    }
    for (int k = w0; k < w1; ++k) {
        pre[k] = run;
        run += __popc(mask[k]);
    }
    __syncthreads();
    return total;
}

// The node map: slot -> box node, for the marked nodes of mask[0..nw).  Each half-wave
// takes one word per round, one bit per lane; four rounds' words are read at once.
__device__ __forceinline__ void write_node_map(const uint32_t* mask, const int* pre, int nw, int* nodes)
{
    constexpr int kU = 4, kStep = PB / 32;
    const int b = threadIdx.x & 31;
    const uint32_t below = (1u << b) - 1u;
    for (int k0 = (int)(threadIdx.x >> 5); k0 < nw; k0 += kU * kStep) {
        uint32_t m[kU];
        int p[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int k = k0 + u * kStep;
            m[u] = k < nw ? mask[k] : 0u;
            p[u] = k < nw ? pre[k] : 0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if ((m[u] >> b) & 1u) nodes[p[u] + __popc(m[u] & below)] = 32 * (k0 + u * kStep) + b;
    }
}

// Slot of marked box node n.
__device__ __forceinline__ int node_slot(const uint32_t* mask, const int* pre, int n)
{
    const int wd = n >> 5;
    return pre[wd] + __popc(mask[wd] & ((1u << (n & 31)) - 1u));
}

// The particles (this one included) whose boxes of this step overlap this particle's box,
// in particle order (the boxes are arcs along the periodic x axis); only they can put a
// spread force on its probe nodes.
// Lane q of the first wave holds particle q's reference rq and box dq (read at the start of
// the launch, so the loads overlap the work before).
template <typename T>
__device__ __forceinline__ int overlap_list(const ParticleArgs<T>& a, const PartRef& rq, const TileDesc& dq, int x0,
                                            int y0, int w, int h, OvEntry* ov, int (*sh)[NW])
{
    if (threadIdx.x < 64) {
        const int q = threadIdx.x;
        bool take = false;
        OvEntry e{};
        if (q < a.nparts && w > 0 && h > 0) {
            const TileDesc d = dq;
            if (d.active && d.w > 0 && d.h > 0) {
                const int xw = wrap(x0, a.nx);
                int dq = d.i0w - xw;
                if (dq < 0) dq += a.nx;
                int dm = xw - d.i0w;
                if (dm < 0) dm += a.nx;
                take = (dq < w || dm < d.w) && d.j0 < y0 + h && y0 < d.j0 + d.h;
                e.tile = rq.tile;
                e.ring = rq.ring;
                e.pid = q;
                e.i0w = d.i0w;
                e.j0 = d.j0;
                e.w = d.w;
                e.h = d.h;
                e.scale = d.scale;
            }
        }
        const unsigned long long bal = __ballot(take);
        const int below =
            (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        if (take) ov[below] = e;
        if (q == 0) sh[0][0] = __popcll(bal);
    }
    __syncthreads();
    const int n = sh[0][0];
    __syncthreads();
    return n;
}

// Marked nodes per lane whose loads are in flight at once while filling: four, or two where a
// node takes 36 loads (the f - f_eq storages: nine values and the three moments of each of
// their nine sources) in a phase whose other state would then spill.
template <typename T>
constexpr int fill_nodes_per_lane(int mode)
{
    return St<T>::neq && mode != 1 ? 2 : 4;
}

// Node fields at the marked nodes: slots s0 + tid + u PB for u < U per round, so the
// loads of U nodes per lane are in flight at once and neighbouring lanes read
// neighbouring nodes of a row.  TOTAL (the probe launch of several particles): also the
// total spread force at each node, summed over the overlapping particles in particle order.
template <typename T, bool TOTAL, int U>
__device__ __forceinline__ void fill_nodes(const ParticleArgs<T>& a, const NodeView& B, const int* nodes, int nm,
                                           int x0, int y0, int w, const OvEntry* ov, int nov)
{
    for (int s0 = 0; s0 < nm; s0 += PB * U) {
        int kk[U], ii[U], jj[U];
        double v[U][9];
        // A wave loads the nodes of its slots of the round where it has any (so a small box
        // issues no loads for empty waves); a slot past the end in such a wave reads the first
        // marked node and stores nothing, so the wave's loads carry no divergent branch.
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int sl = s0 + u * PB + (int)threadIdx.x;
            const int k = nodes[sl < nm ? sl : 0];
            kk[u] = sl < nm ? k : -1;
            jj[u] = y0 + k / w;
            ii[u] = wrap(x0 + k % w, a.nx);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (s0 + u * PB + (int)(threadIdx.x & ~63u) < nm)
                load_node<T, double>(a.f, ii[u], jj[u], a.nx, a.ny, a.pitch, a.plane, a.pull != 0, a.inv_scale,
                                     a.uw6, false, v[u]);
        double fx[U], fy[U];
#pragma unroll
        for (int u = 0; u < U; ++u) fx[u] = fy[u] = 0.0;
        if (TOTAL) {
            // two overlapping particles per round, so their index and force loads overlap;
            // the sums still run in particle order
            for (int e0 = 0; e0 < nov; e0 += 2) {
                const int ne = min(2, nov - e0);
                OvEntry E[2];
                E[0] = ov[e0];
                E[1] = ov[e0 + ne - 1];
                int n[2][U];
                uint2 r[2][U];
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        int di = ii[u] - E[q].i0w;
                        if (di < 0) di += a.nx;
                        const int dj = jj[u] - E[q].j0;
                        n[q][u] = (q < ne && kk[u] >= 0 && di < E[q].w && dj >= 0 && dj < E[q].h) ? dj * E[q].w + di
                                                                                                   : -1;
                        r[q][u] = n[q][u] >= 0 ? E[q].ring[n[q][u] >> 5] : make_uint2(0u, 0u);
                    }
                int64_t tx[2][U], ty[2][U];
                bool in[2][U];
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int nn = n[q][u];
                        in[q][u] = nn >= 0 && ((r[q][u].x >> (nn & 31)) & 1u);
                        tx[q][u] = ty[q][u] = 0;
                        if (in[q][u]) {
                            const int sl = (int)r[q][u].y + __popc(r[q][u].x & ((1u << (nn & 31)) - 1u));
                            tx[q][u] = E[q].tile[2 * sl];
                            ty[q][u] = E[q].tile[2 * sl + 1];
                        }
                    }
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (!in[q][u]) continue;
                        fx[u] += ldexp((double)tx[q][u], -E[q].scale);
                        fy[u] += ldexp((double)ty[q][u], -E[q].scale);
                    }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (kk[u] < 0) continue;
            const int sl = s0 + u * PB + (int)threadIdx.x;
            double dr, jx, jy;
            shifted_moments<double, double>(v[u], dr, jx, jy);
            const double rho = 1.0 + dr;
            const double inv = 1.0 / rho;
            B.rho[sl] = rho;
            B.inv[sl] = inv;
            B.ux[sl] = (jx + 0.5 * a.gx) * inv;
            B.uy[sl] = (jy + 0.5 * a.gy) * inv;
            B.fx[sl] = TOTAL ? (unsigned long long)__double_as_longlong(fx[u]) : 0ull;
            B.fy[sl] = TOTAL ? (unsigned long long)__double_as_longlong(fy[u]) : 0ull;
        }
    }
}

template <bool LDS>
__device__ __forceinline__ void force_add(unsigned long long* p, int64_t v)
{
    if (LDS)
        atomicAdd(p, (unsigned long long)v);
    else
        __hip_atomic_fetch_add(p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool LDS>
__device__ __forceinline__ unsigned long long force_load(const unsigned long long* p)
{
    if (LDS) return *p;
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The total spread force at every marked node, summed over the overlapping particles in
// particle order, written over this particle's own fixed-point value (FP64 bits): its own
// share comes from LDS, the others' from their compact lists (the one-launch split phase,
// after its grid barrier).
template <typename T, bool LDS>
__device__ __forceinline__ void total_forces(const ParticleArgs<T>& a, const NodeView& B, const int* nodes, int nm,
                                             int x0, int y0, int w, const OvEntry* ov, int nov)
{
    for (int s0 = 0; s0 < nm; s0 += PB * kFillU) {
        int sl[kFillU], ii[kFillU], jj[kFillU];
        double fx[kFillU], fy[kFillU];
#pragma unroll
        for (int u = 0; u < kFillU; ++u) {
            sl[u] = s0 + u * PB + (int)threadIdx.x;
            fx[u] = fy[u] = 0.0;
            ii[u] = jj[u] = 0;
            if (sl[u] < nm) {
                const int k = nodes[sl[u]];
                jj[u] = y0 + k / w;
                ii[u] = wrap(x0 + k % w, a.nx);
            }
        }
        for (int e = 0; e < nov; ++e) {
            const OvEntry E = ov[e];
            const bool self = E.pid == (int)a.pid;
            int64_t tx[kFillU], ty[kFillU];
            bool in[kFillU];
#pragma unroll
            for (int u = 0; u < kFillU; ++u) {
                in[u] = false;
                tx[u] = ty[u] = 0;
                if (sl[u] >= nm) continue;
                if (self) {
                    in[u] = true;
                    tx[u] = (int64_t)force_load<LDS>(B.fx + sl[u]);
                    ty[u] = (int64_t)force_load<LDS>(B.fy + sl[u]);
                    continue;
                }
                int di = ii[u] - E.i0w;
                if (di < 0) di += a.nx;
                const int dj = jj[u] - E.j0;
                if (di >= E.w || dj < 0 || dj >= E.h) continue;
                const int n = dj * E.w + di;
                const uint2 r = E.ring[n >> 5];
                if (!((r.x >> (n & 31)) & 1u)) continue;
                const int q = (int)r.y + __popc(r.x & ((1u << (n & 31)) - 1u));
                in[u] = true;
                tx[u] = E.tile[2 * q];
                ty[u] = E.tile[2 * q + 1];
            }
#pragma unroll
            for (int u = 0; u < kFillU; ++u) {
                if (!in[u]) continue;
                fx[u] += ldexp((double)tx[u], -E.scale);
                fy[u] += ldexp((double)ty[u], -E.scale);
            }
        }
#pragma unroll
        for (int u = 0; u < kFillU; ++u) {
            if (sl[u] >= nm) continue;
            B.fx[sl[u]] = (unsigned long long)__double_as_longlong(fx[u]);
            B.fy[sl[u]] = (unsigned long long)__double_as_longlong(fy[u]);
        }
    }
}

// Meeting point of the one-launch split phase, which assumes nothing about which of its
// workgroups are resident together.  Workgroups claim particles (claim_particle), which the
// counter at ctr + kClaimWord counts; here the workgroup barrier completes every wave's stores,
// one thread releases them at device scope and counts this spread in at *ctr, then polls until
// every spread of the launch has counted in (target).  It waits only while every particle is
// claimed: a claimer is running, so its spread will count in.  While a particle is unclaimed
// (its workgroup may be waiting for a CU this one holds) it returns false at once, and the
// caller spreads the unclaimed particles itself.  Its device-scope acquire invalidates the
// CU's caches, which every wave of the workgroup shares, before the second workgroup barrier
// lets them read.  The wait gives up after kSpinLimit polls and raises FLAG_SYNC, so every
// workgroup always finishes.
constexpr unsigned kSpinLimit = 1u << 22;
constexpr int kClaimWord = 3;   // claims counted in this launch (after the chained schedule's two words)
constexpr int kClaimWords = 4;  // then one claim word per particle

__device__ __forceinline__ bool claimed_barrier(unsigned long long* ctr, unsigned long long target, int& flags)
{
    __shared__ int go;
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(ctr, 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        unsigned polls = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(ctr + kClaimWord, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                ok = 0;
                break;
            }
            if (++polls > kSpinLimit) {
                flags |= FLAG_SYNC;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        go = ok;
    }
    __syncthreads();
    return go != 0;
}

// Claims particle k for this launch: its claim word (ctr + kClaimWords + k) holds the number
// of the last launch that claimed it, so an exchange with this launch's number claims it at
// most once per launch without a reset; the one that claims it also counts it at
// ctr + kClaimWord.  Different particles' claims touch different words, so workgroups claiming
// their own particles at once do not contend.
__device__ __forceinline__ bool claim_particle(unsigned long long* ctr, int k, unsigned long long launch)
{
    const unsigned long long was =
        __hip_atomic_exchange(ctr + kClaimWords + k, launch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (was == launch) return false;
    __hip_atomic_fetch_add(ctr + kClaimWord, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Set this particle's bit in the step's mask of every 64 x 4 tile its box reaches.
template <typename T>
__device__ __forceinline__ void mark_tiles(const ParticleArgs<T>& a, int x0, int y0, int w, int h)
{
    const unsigned long long bit = 1ull << a.pid;
    const int ty0 = y0 >> 2, ty1 = (y0 + h - 1) >> 2;
    for (int c = threadIdx.x; c < w; c += PB) {
        const int i = wrap(x0 + c, a.nx);
        if (c != 0 && (i & 63) != 0) continue;  // one thread per tile column of the box
        for (int ty = ty0; ty <= ty1; ++ty) atomicOr(a.pmask + (size_t)ty * a.mtx + (i >> 6), bit);
    }
}

// A double of the particle state, stored coherently across the XCDs' L2 caches.
__device__ __forceinline__ void state_store(double* p, double v) { coherent_store((int64_t*)p, __double_as_longlong(v)); }

// What the first part of the particle phase hands to the rest.
template <int MPT>
struct PhaseCtx {
    double xc, yc, th, ux, uy, om, cth, sth;
    double xc1, yc1, th1, ux1, uy1, om1;  // level n-1
    int64_t step;
    int x0, y0, w, h, nbox, nmarked, flags;
    bool box_ok;
    const uint32_t* mask;
    const int* pre;
    const int* nodes;
    MarkerSet<MPT> G;
    MarkerData<MPT> D;
    TileDesc zin;
};

// The particle phase after the box and its marked nodes are known; LDS: the node fields are
// in LDS, else in the global scratch (plain loads and stores ordered by the workgroup
// barriers, device-scope atomics for the force).
template <typename T, int MPT, bool LDS, int MODE>
__device__ __forceinline__ bool phase_body(const ParticleArgs<T>& a, const PhaseCtx<MPT>& c, const NodeView& B,
                                           OvEntry* ov, int nov, double (*shd)[NW], int (*shi)[NW])
{
    const int tid = threadIdx.x;
    const int nl = a.nl;
    const int x0 = c.x0, y0 = c.y0, w = c.w, h = c.h, nbox = c.nbox;
    const bool box_ok = c.box_ok;
    const uint32_t* mask = c.mask;
    const int* pre = c.pre;
    const double xc = c.xc, yc = c.yc, th = c.th, ux = c.ux, uy = c.uy, om = c.om, cth = c.cth, sth = c.sth;
    const int64_t step = c.step;
    int flags = c.flags;
    DevParticle* st = a.st;

    fill_nodes<T, MODE == 2, fill_nodes_per_lane<T>(MODE)>(a, B, c.nodes, c.nmarked, x0, y0, w, ov, nov);
    __syncthreads();

    // ---- markers: MLS interpolation and direct forcing ----------------------------------
    double S[MPT], SFx[MPT], SFy[MPT], PH[MPT][9];
    int I0[MPT], J0[MPT], NXS[MPT], NYS[MPT], SR[MPT][3];
    bool OK[MPT], LIG[MPT], BND[MPT];
    double maxsf = 0.0;
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
        const int l = tid + k * PB;
        OK[k] = LIG[k] = BND[k] = false;
        NXS[k] = NYS[k] = I0[k] = J0[k] = 0;
        S[k] = SFx[k] = SFy[k] = 0.0;
        if (l < nl) {
            S[k] = c.D.S[k];
            LIG[k] = c.D.lig[k];
            BND[k] = c.D.bnd[k];
            Mls m;
            const bool ok = MODE != 2 && box_ok && mls_shape(c.G.X[k], fluid_row(c.G.Y[k], a.ny), a.ny, m, false);
            if (ok) {
                double rl = 0.0, usx = 0.0, usy = 0.0;
#pragma unroll
                for (int bb = 0; bb < 3; ++bb) {
                    // the window row is marked whole, so its nodes hold consecutive slots
                    SR[k][bb] = bb < m.nys ? node_slot(mask, pre, (m.j0 + bb - y0) * w + (m.i0 - x0)) : 0;
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) {
                        const double p = m.phi[3 * bb + cc];
                        PH[k][3 * bb + cc] = p;
                        if (bb < m.nys && cc < m.nxs) {
                            const int s = SR[k][bb] + cc;
                            rl += p * B.rho[s];
                            usx += p * B.ux[s];
                            usy += p * B.uy[s];
                        }
                    }
                }
                const double rx = c.G.X[k] - xc, ry = c.G.Y[k] - yc;
                OK[k] = true;
                SFx[k] = S[k] * (2.0 * rl * (ux - om * ry - usx));
                SFy[k] = S[k] * (2.0 * rl * (uy + om * rx - usy));
                I0[k] = m.i0;
                J0[k] = m.j0;
                NXS[k] = m.nxs;
                NYS[k] = m.nys;
                const double mag = fmax(fabs(SFx[k]), fabs(SFy[k]));
                maxsf = (mag <= 1e300) ? fmax(maxsf, mag) : INFINITY;
            } else if (MODE != 2 && box_ok) {
                flags |= FLAG_MLS;
            }
        }
    }
    bool spread_ok = false;
    int scale = 0;
    if (MODE != 2) {
        maxsf = wave_max(maxsf);
        if ((tid & 63) == 0) shd[0][tid >> 6] = maxsf;
        __syncthreads();
        maxsf = shd[0][0];
#pragma unroll
        for (int u = 1; u < NW; ++u) maxsf = fmax(maxsf, shd[0][u]);
        __syncthreads();

        // ---- spread: 64-bit fixed point, so the sum does not depend on the order --------
        // |phi| < 2 and at most 64 markers reach a node, so |sum| < 2^7 maxsf; with
        // maxsf < 2^e the scale 2^(55-e) keeps every node below 2^62.
        const bool finite_sf = maxsf <= 1e300;
        spread_ok = box_ok && finite_sf;
        if (box_ok && !finite_sf && tid == 0) flags |= FLAG_NONFINITE;
        int e2 = 0;
        frexp(finite_sf ? maxsf : 1.0, &e2);
        scale = 55 - e2;
        if (spread_ok) {
#pragma unroll
            for (int k = 0; k < MPT; ++k) {
                if (!OK[k]) continue;
#pragma unroll
                for (int bb = 0; bb < 3; ++bb)
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) {
                        if (bb >= NYS[k] || cc >= NXS[k]) continue;
                        const double p = PH[k][3 * bb + cc];
                        const int s = SR[k][bb] + cc;
                        force_add<LDS>(B.fx + s, (int64_t)llrint(ldexp(p * SFx[k], scale)));
                        force_add<LDS>(B.fy + s, (int64_t)llrint(ldexp(p * SFy[k], scale)));
                    }
            }
        }
        __syncthreads();
        if (spread_ok && (MODE == 1 || MODE == 4)) {
            // the compact list and its index for the sweep and the other particles' probes
            for (int k = tid; k < c.nmarked; k += PB) {
                longlong2 t;
                t.x = (long long)force_load<LDS>(B.fx + k);
                t.y = (long long)force_load<LDS>(B.fy + k);
                *(longlong2*)(a.tile + 2 * (size_t)k) = t;
            }
            for (int k = tid; k < (nbox + 31) / 32; k += PB) a.ring[k] = make_uint2(mask[k], (uint32_t)pre[k]);
        } else if (spread_ok) {
            // the box's tile for the sweep: zero where no marker support reaches
            for (int k = tid; k < nbox; k += PB) {
                const uint32_t mw = mask[k >> 5];
                unsigned long long qx = 0, qy = 0;
                if ((mw >> (k & 31)) & 1u) {
                    const int s = pre[k >> 5] + __popc(mw & ((1u << (k & 31)) - 1u));
                    qx = force_load<LDS>(B.fx + s);
                    qy = force_load<LDS>(B.fy + s);
                }
                // coherent stores: the concurrent sweep may read them (HandoverArgs)
                coherent_store(a.tile + 2 * (size_t)k, (int64_t)qx);
                coherent_store(a.tile + 2 * (size_t)k + 1, (int64_t)qy);
            }
        }
        if (tid == 0) {
            TileDesc d;
            d.i0w = wrap(box_ok ? x0 : 0, a.nx);
            d.j0 = box_ok ? y0 : 0;
            d.w = box_ok ? w : 0;
            d.h = box_ok ? h : 0;
            d.scale = scale;
            d.active = spread_ok ? 1 : 0;
            d.i0u = box_ok ? x0 : 0;
            d.pad = 0;
            coherent_store(a.desc, d);
            if (a.check_zone) {
                const TileDesc z = c.zin;
                // the concurrent sweep sweeps the tiles of the predicted box with this force:
                // only valid when the prediction equals this box
                if (!z.active || z.i0w != d.i0w || z.j0 != d.j0 || z.w != d.w || z.h != d.h) flags |= FLAG_TILE;
            }
        }
        if (MODE == 0 && a.ready) {
            // the concurrent sweep's zone workgroups read the tile and desc once this count
            // is published; every lane's stores have completed before it
            stores_done();
            __syncthreads();
            if (tid == 0) publish_counter(a.ready, a.ready_value);
        }
    }
    if (MODE == 1 || MODE == 4) {
        __syncthreads();
        if (box_ok) mark_tiles(a, x0, y0, w, h);
    }
    if (MODE == 1) {
        int v[1] = {flags};
        const int op[1] = {1};
        block_int<1>(v, op, shi);
        if (tid == 0 && v[0]) atomicOr(a.flags, v[0]);
        return true;
    }
    if (MODE == 4) {
        // every particle's list, index, box and tile bits of this step are written: meet,
        // then read the other boxes and sum the total spread force at the marked nodes
        if (!claimed_barrier(a.bar, a.bar_target, flags)) {
            // a particle is unclaimed: publish this spread's flags, leave the loads to the caller
            int v[1] = {flags};
            const int op[1] = {1};
            block_int<1>(v, op, shi);
            if (tid == 0 && v[0]) atomicOr(a.flags, v[0]);
            return false;
        }
        PartRef rq{};
        TileDesc dq{};
        if (tid < a.nparts) {
            rq = a.refs[tid];
            dq = *rq.desc;
        }
        const int nov4 = overlap_list(a, rq, dq, x0, y0, w, h, ov, shi);
        total_forces<T, LDS>(a, B, c.nodes, c.nmarked, x0, y0, w, ov, nov4);
        __syncthreads();
    }

    // ---- probe loads (eq 7-8) and wall distances ---------------------------------------
    double TX[MPT], TY[MPT], D[MPT];
    bool PRB[MPT];
    int nprobe = 0;
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
        const int l = tid + k * PB;
        TX[k] = TY[k] = 0.0;
        D[k] = 0.0;
        PRB[k] = false;
        if (l < nl) {
            Mls m;
            const bool ok = box_ok && mls_shape(c.G.PX[k], c.G.PY[k], a.ny, m, true);
            if (ok) {
                double rp = 0.0, gxx = 0.0, gxy = 0.0, gyx = 0.0, gyy = 0.0;
#pragma unroll
                for (int bb = 0; bb < 3; ++bb) {
                    const int sr = bb < m.nys ? node_slot(mask, pre, (m.j0 + bb - y0) * w + (m.i0 - x0)) : 0;
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) {
                        if (bb < m.nys && cc < m.nxs) {
                            const int e = 3 * bb + cc;
                            const int s = sr + cc;
                            double vx = B.ux[s], vy = B.uy[s];
                            if (MODE == 2 || MODE == 4) {
                                const double fx = __longlong_as_double((long long)B.fx[s]);
                                const double fy = __longlong_as_double((long long)B.fy[s]);
                                const double hinv = 0.5 * B.inv[s];
                                vx += fx * hinv;
                                vy += fy * hinv;
                            } else if (spread_ok) {
                                const unsigned long long qx = force_load<LDS>(B.fx + s);
                                const unsigned long long qy = force_load<LDS>(B.fy + s);
                                const double hinv = 0.5 * B.inv[s];
                                vx += ldexp((double)(int64_t)qx, -scale) * hinv;
                                vy += ldexp((double)(int64_t)qy, -scale) * hinv;
                            }
                            rp += m.phi[e] * B.rho[s];
                            gxx += m.psx[e] * vx;
                            gxy += m.psy[e] * vx;
                            gyx += m.psx[e] * vy;
                            gyy += m.psy[e] * vy;
                        }
                    }
                }
                const double p = (rp - 1.0) * (1.0 / 3.0);
                const double sxx = rp * a.nu * (2.0 * gxx), syy = rp * a.nu * (2.0 * gyy);
                const double sxy = rp * a.nu * (gxy + gyx);
                TX[k] = (-p * c.G.NX[k] + sxx * c.G.NX[k] + sxy * c.G.NY[k]) * S[k];
                TY[k] = (-p * c.G.NY[k] + sxy * c.G.NX[k] + syy * c.G.NY[k]) * S[k];
            } else if (box_ok) {
                flags |= FLAG_MLS;
            }
            D[k] = c.G.Y[k] + 0.5;
            PRB[k] = LIG[k] && D[k] < a.y_cr;
            nprobe += PRB[k] ? 1 : 0;
        }
    }
    {
        int v[1] = {nprobe};
        const int op[1] = {0};
        block_int<1>(v, op, shi);
        nprobe = v[0];
    }

    // ---- bonds (eq 9-11) and the partial sums of the loads ----------------------------
    const double Pf = -expm1(-a.k_f * ((double)nprobe / (double)nl));
    const uint64_t Tf = prob_threshold(Pf);
    const BondParams bp{a.y_cr, a.y_eq, a.sigma, a.sigma_star, a.k_f, a.k_r0, a.kBT};
    double acc[6] = {0, 0, 0, 0, 0, 0};  // hydro x, y, moment; bond x, y, moment
    int nb = 0;
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
        const int l = tid + k * PB;
        if (l < nl) {
            const double rx = c.G.X[k] - xc, ry = c.G.Y[k] - yc;
            const uint8_t b = bond_update(LIG[k], BND[k], D[k], Tf, bp, a.seed, step, (uint32_t)l, a.pid);
            // coherent: the next step's spread may run on another XCD without a release here
            __hip_atomic_store(a.bond + l, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            acc[0] += TX[k];
            acc[1] += TY[k];
            acc[2] += rx * TY[k] - ry * TX[k];
            if (b) {
                const double mag = a.sigma * (D[k] - a.y_eq);
                const double fx = mag * c.G.NX[k], fy = mag * c.G.NY[k];
                acc[3] += fx;
                acc[4] += fy;
                acc[5] += rx * fy - ry * fx;
                ++nb;
            }
        }
    }
    // per-wave partials, then thread 0 (the only user) adds them in wave order
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] = wave_sum(acc[k]);
    nb = wave_isum(nb);
    flags = wave_ior(flags);
    if ((tid & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) shd[k][tid >> 6] = acc[k];
        shi[0][tid >> 6] = nb;
        shi[1][tid >> 6] = flags;
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            double sum = shd[k][0];
#pragma unroll
            for (int u = 1; u < NW; ++u) sum += shd[k][u];
            acc[k] = sum;
        }
        nb = shi[0][0];
        flags = shi[1][0];
        for (int u = 1; u < NW; ++u) {
            nb += shi[0][u];
            flags |= shi[1][u];
        }
    }
    // ---- wall force (eq 12), totals and the rigid-body update (eq 13-16) --------------
    if (tid == 0) {
        const double hx = acc[0], hy = acc[1], hm = acc[2], bx_ = acc[3], by_ = acc[4], bm = acc[5];
        const double gap = yc + 0.5 - sqrt(a.b * a.b * sth * sth + a.a * a.a * cth * cth);
        int32_t fl = flags;
        if (!(gap > 0.0)) fl |= FLAG_CONTACT;
        const double eps = gap > 1e-3 ? gap : 1e-3;
        const double fw = a.hamaker / (8.0 * sqrt(2.0)) * sqrt(sqrt(a.a * a.b) / (eps * eps * eps * eps * eps));
        const double Fx = hx + bx_, Fy = hy + by_ + fw, M = hm + bm;
        const double nux = (2.0 / 3.0) * (2.0 * ux - 0.5 * c.ux1 + Fx / a.mass);
        const double nuy = (2.0 / 3.0) * (2.0 * uy - 0.5 * c.uy1 + Fy / a.mass);
        const double nom = (2.0 / 3.0) * (2.0 * om - 0.5 * c.om1 + M / a.inertia);
        const double nxc = (2.0 / 3.0) * (2.0 * xc - 0.5 * c.xc1 + nux);
        const double nyc = (2.0 / 3.0) * (2.0 * yc - 0.5 * c.yc1 + nuy);
        const double nth = (2.0 / 3.0) * (2.0 * th - 0.5 * c.th1 + nom);
        if (!(isfinite(Fx) && isfinite(Fy) && isfinite(M) && isfinite(nux) && isfinite(nuy) && isfinite(nom)))
            fl |= FLAG_NONFINITE;
        // the state the next step starts from, stored coherently (as the bond flags)
        state_store(&st->xc1, xc);
        state_store(&st->yc1, yc);
        state_store(&st->th1, th);
        state_store(&st->ux1, ux);
        state_store(&st->uy1, uy);
        state_store(&st->om1, om);
        state_store(&st->xc, nxc);
        state_store(&st->yc, nyc);
        state_store(&st->th, nth);
        state_store(&st->ux, nux);
        state_store(&st->uy, nuy);
        state_store(&st->om, nom);
        coherent_store(&st->step, step + 1);
        lbib_particle_state rec;
        rec.step = step;
        rec.xc = nxc;
        rec.yc = nyc;
        rec.theta = nth;
        rec.ux = nux;
        rec.uy = nuy;
        rec.omega = nom;
        rec.fx = Fx;
        rec.fy = Fy;
        rec.torque = M;
        rec.fx_hydro = hx;
        rec.fy_hydro = hy;
        rec.m_hydro = hm;
        rec.fx_bond = bx_;
        rec.fy_bond = by_;
        rec.m_bond = bm;
        rec.fy_wall = fw;
        rec.gap = gap;
        rec.n_bonds = nb;
        rec.n_probing = nprobe;
        st->last = rec;
        const int64_t kk = step - a.trace_start;
        if (a.trace && kk >= 0 && kk < a.trace_cap) a.trace[kk] = rec;
        if (fl) atomicOr(a.flags, fl);
        shd[0][0] = nxc;
        shd[1][0] = nyc;
        shd[2][0] = nth;
    }
    __syncthreads();

    // ---- the box of the next step (the sweep of the nodes outside it may then run while
    // the next particle phase does) -------------------------------------------------------
    if (MODE == 0) {
        const double nxc = shd[0][0], nyc = shd[1][0], nth = shd[2][0];
        MarkerSet<MPT> Gn;
        marker_set<MPT>(c.D, a.nl, a.ny, nxc, nyc, cos(nth), sin(nth), Gn);
        int rn[4] = {0x7fffffff, 0x7fffffff, 0x7fffffff, 0x7fffffff};
        set_bounds<MPT>(Gn, a.ny, rn);
        const int op[4] = {2, 2, 2, 2};
        block_int<4>(rn, op, shi);
        if (tid == 0) {
            const int nw = (rn[0] != 0x7fffffff) ? -rn[1] - rn[0] + 1 : 0;
            const int nh = (rn[2] != 0x7fffffff) ? -rn[3] - rn[2] + 1 : 0;
            TileDesc z;
            z.i0w = wrap(rn[0] != 0x7fffffff ? rn[0] : 0, a.nx);
            z.j0 = rn[2] != 0x7fffffff ? rn[2] : 0;
            z.w = nw;
            z.h = nh;
            z.scale = 0;
            z.active = (nw > 0 && nh > 0 && nw <= a.nx && (int64_t)nw * nh <= a.box_cap) ? 1 : 0;
            z.i0u = rn[0] != 0x7fffffff ? rn[0] : 0;
            z.pad = 0;
            a.zone[a.parity_out] = z;
            // the next sweep reads the box from these words, and overwrites f once it has
            // them: f was last read by the probes, whose results the update above used
            if (a.zone_words) {
                using TL = Tile<false>;
                const int gx = (a.nx + TL::W - 1) / TL::W;
                zone_pack(zone_tiles<TL::W, TL::H>(z, a.nx, a.ny, gx, kZoneMargin), a.zone_tag, a.zone_words);
            }
        }
    }
    return true;
}

// Lays out the node fields and the node map of the marked nodes from base (LDS: dynamic LDS,
// else the global scratch), writes the map and runs the rest of the phase.
template <typename T, int MPT, bool LDS, int MODE>
__device__ __forceinline__ bool phase_rest(const ParticleArgs<T>& a, PhaseCtx<MPT>& c, double* base, OvEntry* ov,
                                           int nov, double (*shd)[NW], int (*shi)[NW])
{
    const int m = c.nmarked;
    NodeView B;
    B.rho = base;
    B.ux = base + m;
    B.uy = base + 2 * m;
    B.inv = base + 3 * m;
    B.fx = (unsigned long long*)(base + 4 * m);
    B.fy = (unsigned long long*)(base + 5 * m);
    int* nodes = (int*)(base + 6 * m);
    c.nodes = nodes;
    write_node_map(c.mask, c.pre, (c.nbox + 31) / 32, nodes);
    __syncthreads();
    return phase_body<T, MPT, LDS, MODE>(a, c, B, ov, nov, shd, shi);
}

// One particle's phase, run by one workgroup.  MPT markers per thread (nl <= MPT * PB);
// lds: the dynamic LDS of lds_bytes bytes.
// MODE 0: the whole phase of a simulation's only particle.  With several particles the
// phase is split in two launches so that every probe sees the spread force of every
// particle: MODE 1 stages the marker supports, spreads the marker forces into the
// particle's tile and marks the step's tile mask; MODE 2 stages the probe supports with the
// total spread force there and evaluates the probe loads, the bonds, the wall force and the
// rigid-body update.
// Returns false only in MODE 4, when the phase stopped after its spread (claimed_barrier).
// shd, shi: the workgroup's reduction scratch in LDS.
template <typename T, int MPT, int MODE>
__device__ __forceinline__ bool particle_phase(const ParticleArgs<T>& a, char* lds, uint32_t lds_bytes,
                                               double (*shd)[NW], int (*shi)[NW])
{
    const int tid = threadIdx.x;
    OvEntry* ov = (OvEntry*)lds;
    const int wcap = (a.box_cap + 31) / 32;
    uint32_t* mask = (uint32_t*)(lds + kLdsHead);
    int* pre = (int*)(mask + wcap);
    double* fields = (double*)(pre + wcap);  // 8-byte aligned: kLdsHead and 8 wcap are multiples of 8
    const size_t aux = kLdsHead + (size_t)wcap * 8;
    const int lds_slots = lds_bytes > aux ? (int)((lds_bytes - aux) / kSlotBytes) : 0;

    // the probe launch's references to every particle's box and force list
    PartRef rq{};
    TileDesc dq{};
    if (MODE == 2 && tid < a.nparts) {
        rq = a.refs[tid];
        dq = *rq.desc;
    }
    PhaseCtx<MPT> c;
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
        const int l = tid + k * PB;
        c.D.bx[k] = c.D.by[k] = c.D.mx[k] = c.D.my[k] = c.D.S[k] = 0.0;
        c.D.lig[k] = c.D.bnd[k] = false;
        if (l < a.nl) {
            c.D.bx[k] = a.xi[2 * l];
            c.D.by[k] = a.xi[2 * l + 1];
            c.D.mx[k] = a.nuv[2 * l];
            c.D.my[k] = a.nuv[2 * l + 1];
            c.D.S[k] = a.S[l];
            c.D.lig[k] = a.ligand[l] != 0;
            c.D.bnd[k] = a.bond[l] != 0;
        }
    }
    TileDesc zin{};  // the box the previous step predicted for this one (thread 0)
    if (MODE == 0 && a.check_zone && tid == 0) zin = a.zone[a.parity_in];
    c.zin = zin;
    const DevParticle* st = a.st;
    c.xc = st->xc;
    c.yc = st->yc;
    c.th = st->th;
    c.ux = st->ux;
    c.uy = st->uy;
    c.om = st->om;
    c.step = st->step;
    c.xc1 = st->xc1;
    c.yc1 = st->yc1;
    c.th1 = st->th1;
    c.ux1 = st->ux1;
    c.uy1 = st->uy1;
    c.om1 = st->om1;
    c.cth = cos(c.th);
    c.sth = sin(c.th);
    c.flags = 0;
    marker_set<MPT>(c.D, a.nl, a.ny, c.xc, c.yc, c.cth, c.sth, c.G);

    // ---- the box: every node a marker or probe support reaches this step --------------
    int r[4] = {0x7fffffff, 0x7fffffff, 0x7fffffff, 0x7fffffff};
    set_bounds<MPT>(c.G, a.ny, r);
    {
        const int op[4] = {2, 2, 2, 2};
        block_int<4>(r, op, shi);
    }
    c.x0 = r[0];
    c.y0 = r[2];
    c.w = (r[0] != 0x7fffffff) ? -r[1] - r[0] + 1 : 0;
    c.h = (r[2] != 0x7fffffff) ? -r[3] - r[2] + 1 : 0;
    c.box_ok = c.w > 0 && c.h > 0 && c.w <= a.nx && (int64_t)c.w * c.h <= a.box_cap;
    if (!c.box_ok && tid == 0) c.flags |= FLAG_TILE;
    if (MODE == 0 && a.zdone) {
        // the overlapped schedule: the previous sweep's zone workgroups have stored this
        // step's populations around the box (coherently) once they have all counted in; the
        // acquire drops stale copies from this CU's caches before any of them is read
        if (tid == 0) {
            wait_counter(a.zdone, a.zdone_target, a.flags);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (a.check_prev && c.box_ok) {
                // those workgroups covered the previous box widened by kZoneMargin: this box
                // must lie in it widened by kZoneMargin - 1 (its readers' sources one further)
                const TileDesc zp = a.zone[a.parity_out];
                const int m = kZoneMargin - 1;
                int dx = ((c.x0 - zp.i0w) % a.nx + a.nx) % a.nx;
                if (dx >= a.nx / 2) dx -= a.nx;
                const bool okx = zp.w + 2 * m >= a.nx || (dx >= -m && dx + c.w <= zp.w + m);
                const bool oky = c.y0 >= zp.j0 - m && c.y0 + c.h <= zp.j0 + zp.h + m;
                if (!zp.active || !okx || !oky) c.flags |= FLAG_TILE;
            }
        }
        __syncthreads();
    }

    // ---- the nodes this launch's supports reach, and their slots ------------------------
    c.nbox = c.box_ok ? c.w * c.h : 0;
    const int nw = (c.nbox + 31) / 32;
    for (int k = tid; k < nw; k += PB) mask[k] = 0u;
    __syncthreads();
    if (c.box_ok)
        mark_windows<MPT>(c.G, a.ny, (MODE == 0 || MODE == 4) ? 3 : MODE == 1 ? 1 : 2, c.x0, c.y0, c.w, c.h, mask);
    __syncthreads();
    c.nmarked = mask_prefix(mask, pre, nw, shi);
    c.mask = mask;
    c.pre = pre;
    const int nov = MODE == 2 ? overlap_list(a, rq, dq, c.x0, c.y0, c.w, c.h, ov, shi) : 0;

    // fields and node map in LDS when they fit, else in the global scratch
    const bool fits = c.nmarked <= lds_slots;
    if (!fits && !a.box_global) {  // no scratch to hold them (a launch with too little LDS)
        c.box_ok = false;
        c.nbox = 0;
        c.nmarked = 0;
        if (tid == 0) c.flags |= FLAG_TILE;
    }
    if (fits || !a.box_global) return phase_rest<T, MPT, true, MODE>(a, c, fields, ov, nov, shd, shi);
    return phase_rest<T, MPT, false, MODE>(a, c, a.box_global, ov, nov, shd, shi);
}

template <typename T, int MPT, int MODE>
__device__ __forceinline__ void particle_phase(const ParticleArgs<T>& a, char* lds, uint32_t lds_bytes)
{
    __shared__ double shd[8][NW];
    __shared__ int shi[8][NW];
    (void)particle_phase<T, MPT, MODE>(a, lds, lds_bytes, shd, shi);
}

template <typename T, int MPT>
__global__ __launch_bounds__(PB) void particle_kernel(ParticleArgs<T> a, uint32_t lds_bytes)
{
    extern __shared__ double lds_dyn[];
    particle_phase<T, MPT, 0>(a, (char*)lds_dyn, lds_bytes);
}

// ParticleRun: one workgroup runs the particle phase of every step of the run in turn.  A
// launch per step needs about half a CU's registers before it can start; while the concurrent
// sweep is dispatching, each CU's freed slots go to further sweep workgroups, so such a launch
// that misses the previous sweep's drain starts only after the next one's, and its force comes
// after that sweep's bulk (59 instead of 46 us per step at 4096 x 1024, until the call ends).
// A workgroup that keeps its CU is never queued behind the sweep.  The step body is a call,
// not inlined: a loop around the inlined phase keeps values live across its back edge and
// spills; the call takes only the step index and reads the run's arguments from a copy in LDS.
template <typename T>
struct RunStage {
    ParticleArgs<T> a;
    ParticleRun<T> run;
    uint32_t lds_bytes;
};
constexpr size_t kRunStageBytes = 768;
static_assert(sizeof(RunStage<double>) <= kRunStageBytes && sizeof(RunStage<half_neq_t>) <= kRunStageBytes,
              "the run's arguments fit their LDS copy");
__shared__ __align__(16) unsigned char run_stage[kRunStageBytes];

template <typename T, int MPT>
__device__ __noinline__ void run_step(int32_t k_in)
{
    extern __shared__ double lds_dyn[];
    const int32_t k = __builtin_amdgcn_readfirstlane(k_in);
    // the copy's words are uniform: each goes to a scalar register as it is read
    RunStage<T> sg;
    {
        static_assert(sizeof(RunStage<T>) % 4 == 0, "whole words");
        constexpr int nw = (int)(sizeof(RunStage<T>) / 4);
        const uint32_t* src = reinterpret_cast<const uint32_t*>(run_stage);
        uint32_t w[nw];
#pragma unroll
        for (int i = 0; i < nw; ++i) w[i] = __builtin_amdgcn_readfirstlane(src[i]);
        __builtin_memcpy(&sg, w, sizeof(sg));
    }
    ParticleArgs<T> a = sg.a;
    const ParticleRun<T> run = sg.run;
    const uint32_t lds_bytes = sg.lds_bytes;
    const int64_t step = run.step0 + k;
    a.f = (k & 1) ? run.f_odd : run.f_even;
    a.parity_in = (int32_t)(step & 1);
    a.parity_out = a.parity_in ^ 1;
    a.ready_value += (unsigned long long)k;
    a.zone_words = run.zone_base + 2 * ((step + 1) & 3);
    a.zone_tag = (uint32_t)(a.ready_value & 0xffffu);
    a.zdone_target += (unsigned long long)k * (unsigned long long)run.nzone;
    if (k > 0) a.check_prev = 1;
    particle_phase<T, MPT, 0>(a, (char*)lds_dyn, lds_bytes);
}

template <typename T, int MPT>
__global__ __launch_bounds__(PB) void particle_run_kernel(ParticleArgs<T> a, ParticleRun<T> run, uint32_t lds_bytes)
{
    if (threadIdx.x == 0) {
        RunStage<T>& sg = *reinterpret_cast<RunStage<T>*>(run_stage);
        sg.a = a;
        sg.run = run;
        sg.lds_bytes = lds_bytes;
    }
    __syncthreads();
    for (int32_t k = 0; k < run.nsteps; ++k) {
        run_step<T, MPT>(k);
        __syncthreads();  // every wave is done with this step's LDS before the next step's writes
    }
}

// Hand-over between the two launches of the split phase when they run on different streams.
// chain_wait: one thread polls the monotonic counter until it reaches target (bounded: past
// about a second it raises FLAG_SYNC and goes on), then its device-scope acquire drops stale
// copies from the caches the workgroup reads through, before the barrier lets every wave read.
// chain_publish: the barrier completes every wave's stores; one thread's device-scope release
// makes them visible to every XCD and counts this workgroup in.
__device__ __forceinline__ void chain_wait(const unsigned long long* ctr, unsigned long long target, int32_t* flags)
{
    if (threadIdx.x == 0) {
        wait_counter(ctr, target, flags);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}
// COHERENT: everything the waiting launch reads was stored coherently (the loads launch's
// particle state and bond flags), so waiting for the stores to complete replaces the release,
// which would write back the XCD's whole L2 -- costly beside a concurrent sweep's stores.
template <bool COHERENT>
__device__ __forceinline__ void chain_publish(unsigned long long* ctr)
{
    if (COHERENT) stores_done();
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_fetch_add(ctr, 1ull, COHERENT ? __ATOMIC_RELAXED : __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Split particle phase of a simulation with several particles: workgroup b runs particle b
// in MODE 1 (spread) or MODE 2 (loads, bonds, update) on the populations f of this step and
// the step's tile mask.  wait (optional): start once *wait reaches wait_target; done
// (optional): count this workgroup in at *done when its phase is complete.
template <typename T, int MPT, int MODE>
__global__ __launch_bounds__(PB) void split_particle_kernel(const ParticleArgs<T>* __restrict__ args,
                                                            const T* __restrict__ f,
                                                            unsigned long long* __restrict__ pmask, uint32_t lds_bytes,
                                                            const unsigned long long* wait,
                                                            unsigned long long wait_target, unsigned long long* done)
{
    extern __shared__ double lds_dyn[];
    ParticleArgs<T> a = args[blockIdx.x];
    a.f = f;
    a.pmask = pmask;
    if (wait) chain_wait(wait, wait_target, a.flags);
    particle_phase<T, MPT, MODE>(a, (char*)lds_dyn, lds_bytes);
    if (done) chain_publish<MODE == 2>(done);
}

template <typename K>
hipError_t allow_max_lds(K kernel, bool& done)
{
    if (done) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
    if (e == hipSuccess) done = true;
    return e;
}

template <typename T, int MPT, int MODE>
hipError_t launch_split_mode(const ParticleArgs<T>* args, int32_t n, const T* f, unsigned long long* pmask, size_t lds,
                             const SplitChain& ch, hipStream_t stream, hipEvent_t t0, hipEvent_t t1)
{
    static bool attr = false;
    hipError_t e = allow_max_lds(split_particle_kernel<T, MPT, MODE>, attr);
    if (e != hipSuccess) return e;
    hipExtLaunchKernelGGL(split_particle_kernel<T, MPT, MODE>, dim3(n), dim3(PB), (uint32_t)lds, stream, t0, t1, 0u,
                          args, f, pmask, (uint32_t)lds, ch.wait, ch.wait_target, ch.done);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_particle_split(const ParticleArgs<T>* args, int32_t n, const T* f, unsigned long long* pmask,
                                 int32_t mode, int32_t max_nl, size_t lds, hipStream_t stream, hipEvent_t t0,
                                 hipEvent_t t1, const SplitChain& ch)
{
    if (n <= 0) return hipSuccess;
    if (n > kMaxParticles || lds > kLdsMax || lds < kLdsHead || (mode != 1 && mode != 2)) return hipErrorInvalidValue;
#define LBIB_SPLIT(M)                                                                                \
    return mode == 1 ? launch_split_mode<T, M, 1>(args, n, f, pmask, lds, ch, stream, t0, t1)       \
                     : launch_split_mode<T, M, 2>(args, n, f, pmask, lds, ch, stream, t0, t1)
    if (max_nl <= PB) LBIB_SPLIT(1);
    if (max_nl <= 2 * PB) LBIB_SPLIT(2);
#undef LBIB_SPLIT
    return hipErrorInvalidValue;
}

// One particle's phase (MODE 1 or 2) on the one-launch phase's fallback path, out of line so
// that its registers do not weigh on the common path.
template <typename T, int MPT, int MODE>
__device__ __noinline__ void fallback_phase(const ParticleArgs<T>* args, int k, const T* f, unsigned long long* pmask,
                                            uint32_t lds_bytes, double (*shd)[NW], int (*shi)[NW])
{
    extern __shared__ double lds_dyn[];
    ParticleArgs<T> b = args[__builtin_amdgcn_readfirstlane(k)];
    b.f = f;
    b.pmask = pmask;
    (void)particle_phase<T, MPT, MODE>(b, (char*)lds_dyn, lds_bytes, shd, shi);
}

// The split phase as one launch (MODE 4), assuming nothing about which of its workgroups are
// resident together.  Workgroup b claims particle b (claim_particle), stages the union of its
// marker and probe supports once, spreads, and meets the others at claimed_barrier before the
// loads.  One that starts after its particle was claimed by another has nothing to do.  One
// that finds a particle unclaimed at the barrier (its workgroup not started, perhaps waiting
// for a CU this one holds) claims and spreads every particle still unclaimed (MODE 1), waits
// until every spread has counted in, and runs the loads half (MODE 2) of each particle it
// holds, its own first: every wait is then on running workgroups.  A launch with fewer
// workgroups than particles takes that path.  ctr: [0] spreads counted in and [kClaimWord]
// claims counted, both at target - np before the launch and at target after it; from
// [kClaimWords], a claim word per particle (claim_particle); launch: this launch's number.
template <typename T, int MPT>
__global__ __launch_bounds__(PB) void fused_particle_kernel(const ParticleArgs<T>* __restrict__ args,
                                                            const T* __restrict__ f,
                                                            unsigned long long* __restrict__ pmask, uint32_t lds_bytes,
                                                            unsigned long long* ctr, unsigned long long target, int np,
                                                            unsigned long long launch)
{
    extern __shared__ double lds_dyn[];
    __shared__ double shd[8][NW];
    __shared__ int shi[8][NW];
    __shared__ int took;
    __shared__ int held[kMaxParticles];
    const int p = (int)blockIdx.x;
    if (threadIdx.x == 0) took = claim_particle(ctr, p, launch) ? 1 : 0;
    __syncthreads();
    if (!took) return;
    {
        ParticleArgs<T> a = args[p];
        a.f = f;
        a.pmask = pmask;
        a.bar = ctr;
        a.bar_target = target;
        if (particle_phase<T, MPT, 4>(a, (char*)lds_dyn, lds_bytes, shd, shi)) return;
    }
    int nheld = 0;
    for (int q = 0; q < np; ++q) {
        __syncthreads();
        if (threadIdx.x == 0)
            took = __hip_atomic_load(ctr + kClaimWords + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != launch &&
                   claim_particle(ctr, q, launch);
        __syncthreads();
        if (!took) continue;
        fallback_phase<T, MPT, 1>(args, q, f, pmask, lds_bytes, shd, shi);
        chain_publish<false>(ctr);
        if (threadIdx.x == 0) held[nheld] = q;
        ++nheld;
    }
    chain_wait(ctr, target, args[p].flags);
    for (int k = -1; k < nheld; ++k) {
        __syncthreads();
        fallback_phase<T, MPT, 2>(args, k < 0 ? p : held[k], f, pmask, lds_bytes, shd, shi);
    }
}

template <typename T, int MPT>
hipError_t launch_fused_mpt(const ParticleArgs<T>* args, int32_t n, int32_t wg, const T* f, unsigned long long* pmask,
                            size_t lds, unsigned long long* bar, unsigned long long target, hipStream_t stream)
{
    static bool attr = false;
    hipError_t e = allow_max_lds(fused_particle_kernel<T, MPT>, attr);
    if (e != hipSuccess) return e;
    hipExtLaunchKernelGGL(fused_particle_kernel<T, MPT>, dim3(wg), dim3(PB), (uint32_t)lds, stream, nullptr, nullptr,
                          0u, args, f, pmask, (uint32_t)lds, bar, target, (int)n, target / (unsigned long long)n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_particle_fused(const ParticleArgs<T>* args, int32_t n, int32_t workgroups, const T* f,
                                 unsigned long long* pmask, int32_t max_nl, size_t lds, unsigned long long* bar,
                                 unsigned long long target, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    if (n > kMaxParticles || workgroups < 1 || workgroups > n || lds > kLdsMax || lds < kLdsHead || !bar ||
        target < (unsigned long long)n)
        return hipErrorInvalidValue;
    if (max_nl <= PB) return launch_fused_mpt<T, 1>(args, n, workgroups, f, pmask, lds, bar, target, stream);
    if (max_nl <= 2 * PB) return launch_fused_mpt<T, 2>(args, n, workgroups, f, pmask, lds, bar, target, stream);
    return hipErrorInvalidValue;
}

// Particle phases of a pool of independent simulations: workgroup b runs member
// k = active[b].  A member whose step counter has reached its target, or whose watchdog
// has raised a flag, does nothing (ctl[k].pad = -1: its sweep does nothing either), so a
// failed member stays frozen at the step that failed.  Otherwise ctl[k] receives the box
// descriptor of step n with pad = the parity of n: the populations of step n are in f for
// even n and in fB for odd n.
template <typename T, int MPT>
__global__ __launch_bounds__(PB) void pool_particle_kernel(const ParticleArgs<T>* __restrict__ args,
                                                           const int32_t* __restrict__ active,
                                                           TileDesc* __restrict__ ctl, uint32_t lds_bytes)
{
    extern __shared__ double lds_dyn[];
    const int k = active[blockIdx.x];
    ParticleArgs<T> a = args[k];
    const int64_t n = a.st->step;
    if (n >= a.target_steps || *a.flags != 0) {
        if (threadIdx.x == 0) ctl[k].pad = -1;
        return;
    }
    a.f = (n & 1) ? a.fB : a.f;
    particle_phase<T, MPT, 0>(a, (char*)lds_dyn, lds_bytes);
    if (threadIdx.x == 0) {  // the thread that wrote *a.desc in the particle phase
        TileDesc d = coherent_load(a.desc);
        d.pad = (int32_t)(n & 1);
        ctl[k] = d;
    }
}

template <typename T, int MPT>
hipError_t launch_pool_mpt(const ParticleArgs<T>* args, const int32_t* active, TileDesc* ctl, int32_t n_active,
                           size_t lds, hipStream_t stream, hipEvent_t t0, hipEvent_t t1)
{
    static bool attr = false;
    hipError_t e = allow_max_lds(pool_particle_kernel<T, MPT>, attr);
    if (e != hipSuccess) return e;
    if (t0 || t1)
        hipExtLaunchKernelGGL((pool_particle_kernel<T, MPT>), dim3(n_active), dim3(PB), (uint32_t)lds, stream, t0, t1,
                              0u, args, active, ctl, (uint32_t)lds);
    else
        hipLaunchKernelGGL((pool_particle_kernel<T, MPT>), dim3(n_active), dim3(PB), lds, stream, args, active, ctl,
                           (uint32_t)lds);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pool_particle(const ParticleArgs<T>* args, const int32_t* active, TileDesc* ctl, int32_t n_active,
                                int32_t max_nl, size_t lds, hipStream_t stream, hipEvent_t t0, hipEvent_t t1)
{
    if (n_active <= 0) return hipSuccess;
    if (lds > kLdsMax || lds < kLdsHead) return hipErrorInvalidValue;
    if (max_nl <= PB) return launch_pool_mpt<T, 1>(args, active, ctl, n_active, lds, stream, t0, t1);
    if (max_nl <= 2 * PB) return launch_pool_mpt<T, 2>(args, active, ctl, n_active, lds, stream, t0, t1);
    return hipErrorInvalidValue;
}

template <typename T, int MPT>
hipError_t launch_particle_mpt(const ParticleArgs<T>& a, hipStream_t stream, hipEvent_t t0, hipEvent_t t1)
{
    static bool attr = false;
    hipError_t e = allow_max_lds(particle_kernel<T, MPT>, attr);
    if (e != hipSuccess) return e;
    const size_t lds = particle_launch_lds(a.box_cap);
    if (particle_lds_aux_bytes(a.box_cap) > lds) return hipErrorInvalidValue;
    hipExtLaunchKernelGGL(particle_kernel<T, MPT>, dim3(1), dim3(PB), (uint32_t)lds, stream, t0, t1, 0u, a,
                          (uint32_t)lds);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_particle(const ParticleArgs<T>& a, hipStream_t stream, hipEvent_t t0, hipEvent_t t1)
{
    if (a.nl <= PB) return launch_particle_mpt<T, 1>(a, stream, t0, t1);
    if (a.nl <= 2 * PB) return launch_particle_mpt<T, 2>(a, stream, t0, t1);
    return hipErrorInvalidValue;
}

template <typename T, int MPT>
hipError_t launch_particle_run_mpt(const ParticleArgs<T>& a, const ParticleRun<T>& run, hipStream_t stream,
                                   hipEvent_t t0, hipEvent_t t1)
{
    static bool attr = false;
    hipError_t e = allow_max_lds(particle_run_kernel<T, MPT>, attr);
    if (e != hipSuccess) return e;
    const size_t lds = particle_launch_lds(a.box_cap);
    if (particle_lds_aux_bytes(a.box_cap) > lds) return hipErrorInvalidValue;
    hipExtLaunchKernelGGL(particle_run_kernel<T, MPT>, dim3(1), dim3(PB), (uint32_t)lds, stream, t0, t1, 0u, a, run,
                          (uint32_t)lds);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_particle_run(const ParticleArgs<T>& a, const ParticleRun<T>& run, hipStream_t stream, hipEvent_t t0,
                               hipEvent_t t1)
{
    if (run.nsteps <= 0 || !run.f_even || !run.f_odd || !run.zone_base || !a.ready || !a.zdone || !a.check_zone)
        return hipErrorInvalidValue;
    if (a.nl <= PB) return launch_particle_run_mpt<T, 1>(a, run, stream, t0, t1);
    if (a.nl <= 2 * PB) return launch_particle_run_mpt<T, 2>(a, run, stream, t0, t1);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------------------
// Kernel-level entry points (same device functions as the time step)
// ---------------------------------------------------------------------------------------
__global__ void philox_kernel(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t c0 = ctr[4 * k], c1 = ctr[4 * k + 1], c2 = ctr[4 * k + 2], c3 = ctr[4 * k + 3];
    philox4x32_10(c0, c1, c2, c3, key[2 * k], key[2 * k + 1]);
    out[4 * k] = c0;
    out[4 * k + 1] = c1;
    out[4 * k + 2] = c2;
    out[4 * k + 3] = c3;
}

hipError_t launch_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(philox_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, ctr, key, out, n);
    return hipGetLastError();
}

__global__ void mls_kernel(const double* pts, int64_t n, int nx, int ny, int32_t* node, double* phi, double* psix,
                           double* psiy)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    Mls m;
    const bool ok = mls_shape(pts[2 * k], pts[2 * k + 1], ny, m, true);
    for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) {
            const int e = 3 * b + a;
            const bool in = ok && a < m.nxs && b < m.nys;
            node[2 * (9 * k + e)] = in ? wrap(m.i0 + a, nx) : -1;
            node[2 * (9 * k + e) + 1] = in ? m.j0 + b : -1;
            phi[9 * k + e] = in ? m.phi[e] : 0.0;
            psix[9 * k + e] = in ? m.psx[e] : 0.0;
            psiy[9 * k + e] = in ? m.psy[e] : 0.0;
        }
}

hipError_t launch_mls(const double* pts, int64_t n, int32_t nx, int32_t ny, int32_t* node, double* phi, double* psix,
                      double* psiy, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(mls_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, pts, n, nx, ny, node, phi,
                       psix, psiy);
    return hipGetLastError();
}

// One workgroup per set: count the probing ligands, then update every element.
__global__ __launch_bounds__(PB) void bonds_kernel(const uint8_t* ligand, const double* d, const uint8_t* b_in,
                                                   uint8_t* b_out, const int64_t* step, int32_t* n_bonds,
                                                   int32_t* n_probing, int nl, BondParams p, uint64_t seed,
                                                   uint32_t pid)
{
    __shared__ int shi[1][NW];
    const int s = blockIdx.x;
    const size_t base = (size_t)s * nl;
    int np = 0;
    for (int l = threadIdx.x; l < nl; l += PB) np += (ligand[base + l] && d[base + l] < p.y_cr) ? 1 : 0;
    {
        int v[1] = {np};
        const int op[1] = {0};
        block_int<1>(v, op, shi);
        np = v[0];
    }
    const uint64_t Tf = prob_threshold(-expm1(-p.k_f * ((double)np / (double)nl)));
    int nb = 0;
    for (int l = threadIdx.x; l < nl; l += PB) {
        const uint8_t b = bond_update(ligand[base + l] != 0, b_in[base + l] != 0, d[base + l], Tf, p, seed, step[s],
                                      (uint32_t)l, pid);
        b_out[base + l] = b;
        nb += b;
    }
    {
        int v[1] = {nb};
        const int op[1] = {0};
        block_int<1>(v, op, shi);
        nb = v[0];
    }
    if (threadIdx.x == 0) {
        n_bonds[s] = nb;
        n_probing[s] = np;
    }
}

hipError_t launch_bonds(const uint8_t* ligand, const double* d, const uint8_t* b_in, uint8_t* b_out,
                        const int64_t* step, int32_t* n_bonds, int32_t* n_probing, int32_t nl, int32_t n_sets,
                        const double* q, uint64_t seed, uint32_t pid, hipStream_t stream)
{
    if (n_sets <= 0) return hipSuccess;
    BondParams p{q[0], q[1], q[2], q[3], q[4], q[5], q[6]};
    hipLaunchKernelGGL(bonds_kernel, dim3(n_sets), dim3(PB), 0, stream, ligand, d, b_in, b_out, step, n_bonds,
                       n_probing, nl, p, seed, pid);
    return hipGetLastError();
}

// Plain streaming copy: each thread moves four 16-byte vectors, all loads issued before
// the stores, loads and stores past the caches (data touched once).
typedef float lbib_v4f __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void copy_kernel(const lbib_v4f* __restrict__ src, lbib_v4f* __restrict__ dst,
                                                   int64_t n)
{
    const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    lbib_v4f v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (base + 256 * u < n) v[u] = __builtin_nontemporal_load(src + base + 256 * u);
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (base + 256 * u < n) __builtin_nontemporal_store(v[u], dst + base + 256 * u);
}

hipError_t launch_copy(const float4* src, float4* dst, int64_t n, hipStream_t stream)
{
    const int64_t blocks = (n + 1023) / 1024;
    if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(copy_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, (const lbib_v4f*)src,
                       (lbib_v4f*)dst, n);
    return hipGetLastError();
}

#define LBIB_PARTICLE_INSTANTIATE(T)                                                                        \
    template hipError_t launch_pool_particle<T>(const ParticleArgs<T>*, const int32_t*, TileDesc*, int32_t,      \
                                                int32_t, size_t, hipStream_t, hipEvent_t, hipEvent_t);          \
    template hipError_t launch_particle<T>(const ParticleArgs<T>&, hipStream_t, hipEvent_t, hipEvent_t);        \
    template hipError_t launch_particle_run<T>(const ParticleArgs<T>&, const ParticleRun<T>&, hipStream_t,      \
                                               hipEvent_t, hipEvent_t);                                          \
    template hipError_t launch_particle_split<T>(const ParticleArgs<T>*, int32_t, const T*, unsigned long long*, \
                                                 int32_t, int32_t, size_t, hipStream_t, hipEvent_t, hipEvent_t,  \
                                                 const SplitChain&);                                               \
    template hipError_t launch_particle_fused<T>(const ParticleArgs<T>*, int32_t, int32_t, const T*,             \
                                                 unsigned long long*, int32_t, size_t, unsigned long long*,       \
                                                 unsigned long long, hipStream_t);
LBIB_PARTICLE_INSTANTIATE(double)
LBIB_PARTICLE_INSTANTIATE(float)
LBIB_PARTICLE_INSTANTIATE(half_t)
LBIB_PARTICLE_INSTANTIATE(bf16_t)
LBIB_PARTICLE_INSTANTIATE(half_neq_t)
LBIB_PARTICLE_INSTANTIATE(bf16_neq_t)
#undef LBIB_PARTICLE_INSTANTIATE

}  // namespace lbib
