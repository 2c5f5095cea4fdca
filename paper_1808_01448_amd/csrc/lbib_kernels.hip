// lbib_kernels.hip -- gfx950 kernels of the LB-IB particle-adhesion time step.
//
// One time step n -> n+1 is two launches on one stream:
//   particle phase (one workgroup per particle): markers at level n, MLS interpolation of
//     the fluid at the markers, direct-forcing marker forces, deterministic spread into a
//     fixed-point force tile, probe loads (eq 7-8), bond update (eq 9-11), wall force
//     (eq 12), FP64 force/torque reductions and the rigid-body update (eq 13-16);
//   lattice sweep (one thread per node): BGK collision with Guo forcing (eq 1-6) using the
//     uniform drive plus the tile force, then push-streaming with half-way bounce-back at
//     the two walls and periodic x.
// The sweep reads buffer A and writes buffer B; the particle phase of the next step reads B.
//
// Populations are stored shifted, g_q = f_q - w_q, as planes [q][j][i] with a row pitch.
// The shift keeps the FP32 storage accurate at the O(1e-4) velocities of the paper's
// capillary flows; the rest state is exactly g = 0.  The collision itself is evaluated in
// FP64 for both storage precisions: in FP32 arithmetic its rounding breaks the exact
// momentum balance of each collision at the 1e-12 level, and at these velocities the
// drift accumulates to ~3e-5 of the particle velocity within 2000 steps, while FP32
// storage alone costs ~3e-8.  The sweep stays bound by HBM traffic either way.
#include <hip/hip_runtime.h>
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
template <typename T, bool TILE>
__global__ __launch_bounds__(256) void sweep_kernel(const T* __restrict__ fin, T* __restrict__ fout, SweepArgs a,
                                                    const TileDesc* __restrict__ desc,
                                                    const int64_t* __restrict__ tile)
{
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int j = blockIdx.y * 4 + threadIdx.y;
    if (i >= a.nx || j >= a.ny) return;
    const int64_t P = a.plane;
    const size_t c = (size_t)j * a.pitch + i;

    T gs[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) gs[q] = fin[q * P + c];

    double Fx = a.gx, Fy = a.gy;
    if (TILE) {
        const TileDesc d = *desc;
        if (d.active) {
            int di = i - d.i0w;
            if (di < 0) di += a.nx;
            const int dj = j - d.j0;
            if (di < d.w && dj >= 0 && dj < d.h) {
                const int64_t* t = tile + 2 * ((size_t)dj * d.w + di);
                Fx += ldexp((double)t[0], -d.scale);
                Fy += ldexp((double)t[1], -d.scale);
            }
        }
    }

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

template <typename T>
hipError_t launch_sweep(const T* fin, T* fout, const SweepArgs& a, const TileDesc* desc, const int64_t* tile,
                        hipStream_t stream)
{
    dim3 block(64, 4), grid((a.nx + 63) / 64, (a.ny + 3) / 4);
    if (desc)
        hipLaunchKernelGGL((sweep_kernel<T, true>), grid, block, 0, stream, fin, fout, a, desc, tile);
    else
        hipLaunchKernelGGL((sweep_kernel<T, false>), grid, block, 0, stream, fin, fout, a, desc, tile);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Workgroup reductions: butterfly within each 64-wide wavefront, then the per-wave partials
// in wave order.  The order is fixed, so results are bit-reproducible.
// ---------------------------------------------------------------------------------------
constexpr int PB = 256;       // threads of the particle workgroup
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

// The 3 x 3 candidate nodes of an MLS support: density deviation and momentum of each,
// from 81 independent loads (addresses clamped into the lattice; candidates outside the
// support carry zero MLS weight, so their values never contribute).
template <typename T>
__device__ __forceinline__ void gather9(const T* __restrict__ f, int nx, int ny, int pitch, int64_t P, const Mls& m,
                                        double (&drho)[9], double (&jx)[9], double (&jy)[9])
{
    T v[9][9];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        int jj = m.j0 + b;
        jj = jj < 0 ? 0 : (jj > ny - 1 ? ny - 1 : jj);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t base = (size_t)jj * pitch + wrap(m.i0 + c, nx);
#pragma unroll
            for (int q = 0; q < 9; ++q) v[3 * b + c][q] = f[q * P + base];
        }
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) shifted_moments<double, T>(v[k], drho[k], jx[k], jy[k]);
}

__device__ __forceinline__ double fluid_row(double y, int ny)
{
    // transfer points between a wall and the first node row are transferred as if they sat
    // on that row (the linear fit would otherwise extrapolate and destabilise the coupling)
    return y < 0.0 ? 0.0 : (y > ny - 1.0 ? ny - 1.0 : y);
}

// MPT markers per thread (nl <= MPT * PB).  LDS_TILE: the fixed-point spread tile lives in
// dynamic LDS (capacity cap_w x cap_h x 2 x 8 bytes), else in the global tile with
// device-scope atomics.
template <typename T, int MPT, bool LDS_TILE>
__global__ __launch_bounds__(PB) void particle_kernel(ParticleArgs<T> a)
{
    extern __shared__ unsigned long long lds_tile[];
    __shared__ double shd[8][NW];
    __shared__ int shi[8][NW];
    const int tid = threadIdx.x;
    const int nl = a.nl;

    DevParticle* st = a.st;
    const double xc = st->xc, yc = st->yc, th = st->th, ux = st->ux, uy = st->uy, om = st->om;
    const int64_t step = st->step;
    const double cth = cos(th), sth = sin(th);
    int flags = 0;

    // per-marker state kept in registers across the phases
    double X[MPT], Y[MPT], NX[MPT], NY[MPT], S[MPT], SFx[MPT], SFy[MPT], PH[MPT][9];
    int I0[MPT], J0[MPT], NXS[MPT], NYS[MPT];
    bool OK[MPT], LIG[MPT], BND[MPT];

    // ---- markers, MLS interpolation, direct forcing -----------------------------------
    double maxsf = 0.0;
    int imin = 0x7fffffff, imaxn = 0x7fffffff, jmin = 0x7fffffff, jmaxn = 0x7fffffff;  // maxima as -min
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
        const int l = tid + k * PB;
        OK[k] = false;
        NXS[k] = NYS[k] = 0;
        SFx[k] = SFy[k] = 0.0;
        if (l < nl) {
            const double bx = a.xi[2 * l], by = a.xi[2 * l + 1];
            const double mx = a.nuv[2 * l], my = a.nuv[2 * l + 1];
            S[k] = a.S[l];
            LIG[k] = a.ligand[l] != 0;
            BND[k] = a.bond[l] != 0;
            X[k] = xc + cth * bx - sth * by;
            Y[k] = yc + sth * bx + cth * by;
            NX[k] = cth * mx - sth * my;
            NY[k] = sth * mx + cth * my;
            Mls m;
            const bool ok = mls_shape(X[k], fluid_row(Y[k], a.ny), a.ny, m, false);
            double dr[9], jxn[9], jyn[9];
            gather9<T>(a.f, a.nx, a.ny, a.pitch, a.plane, m, dr, jxn, jyn);
            double rl = 0.0, usx = 0.0, usy = 0.0;
#pragma unroll
            for (int e = 0; e < 9; ++e) {
                const double rho = 1.0 + dr[e];
                const double p = m.phi[e];
                rl += p * rho;
                usx += p * ((jxn[e] + 0.5 * a.gx) / rho);
                usy += p * ((jyn[e] + 0.5 * a.gy) / rho);
                PH[k][e] = p;
            }
            const double rx = X[k] - xc, ry = Y[k] - yc;
            const double Fx = 2.0 * rl * (ux - om * ry - usx);
            const double Fy = 2.0 * rl * (uy + om * rx - usy);
            if (ok) {
                OK[k] = true;
                SFx[k] = S[k] * Fx;
                SFy[k] = S[k] * Fy;
                I0[k] = m.i0;
                J0[k] = m.j0;
                NXS[k] = m.nxs;
                NYS[k] = m.nys;
                const double mag = fmax(fabs(SFx[k]), fabs(SFy[k]));
                maxsf = (mag <= 1e300) ? fmax(maxsf, mag) : INFINITY;
                imin = min(imin, m.i0);
                imaxn = min(imaxn, -(m.i0 + m.nxs - 1));
                jmin = min(jmin, m.j0);
                jmaxn = min(jmaxn, -(m.j0 + m.nys - 1));
            } else {
                flags |= FLAG_MLS;
            }
        }
    }
    maxsf = wave_max(maxsf);
    if ((tid & 63) == 0) shd[0][tid >> 6] = maxsf;
    {
        int v[4] = {imin, imaxn, jmin, jmaxn};
        const int op[4] = {2, 2, 2, 2};
        block_int<4>(v, op, shi);  // contains the barriers that publish shd[0]
        imin = v[0];
        imaxn = v[1];
        jmin = v[2];
        jmaxn = v[3];
    }
    maxsf = shd[0][0];
#pragma unroll
    for (int u = 1; u < NW; ++u) maxsf = fmax(maxsf, shd[0][u]);
    const int i0 = imin, ihi = -imaxn, j0 = jmin, jhi = -jmaxn;
    const int w = (imin != 0x7fffffff && ihi >= i0) ? ihi - i0 + 1 : 0;
    const int h = (jmin != 0x7fffffff && jhi >= j0) ? jhi - j0 + 1 : 0;

    // ---- spread: 64-bit fixed point, so the sum does not depend on the order --------
    // |phi| < 2 and at most 64 markers reach a node, so |sum| < 2^7 maxsf; with
    // maxsf < 2^e the scale 2^(55-e) keeps every node below 2^62.
    const bool finite_sf = maxsf <= 1e300;
    const bool spread_ok = finite_sf && w > 0 && h > 0 && w <= a.cap_w && h <= a.cap_h;
    if (tid == 0 && !spread_ok && (w > 0 || !finite_sf)) flags |= finite_sf ? FLAG_TILE : FLAG_NONFINITE;
    int e2 = 0;
    frexp(finite_sf ? maxsf : 1.0, &e2);
    const int scale = 55 - e2;
    const int nt = 2 * w * h;
    if (spread_ok) {
        for (int k = tid; k < nt; k += PB) {
            if (LDS_TILE)
                lds_tile[k] = 0ull;
            else
                __hip_atomic_store(a.tile + k, (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    if (spread_ok) {
#pragma unroll
        for (int k = 0; k < MPT; ++k) {
            if (!OK[k]) continue;
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (b >= NYS[k] || c >= NXS[k]) continue;
                    const double p = PH[k][3 * b + c];
                    const int idx = 2 * ((J0[k] + b - j0) * w + (I0[k] + c - i0));
                    const int64_t qx = (int64_t)llrint(ldexp(p * SFx[k], scale));
                    const int64_t qy = (int64_t)llrint(ldexp(p * SFy[k], scale));
                    if (LDS_TILE) {
                        atomicAdd(&lds_tile[idx], (unsigned long long)qx);
                        atomicAdd(&lds_tile[idx + 1], (unsigned long long)qy);
                    } else {
                        __hip_atomic_fetch_add(a.tile + idx, qx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_fetch_add(a.tile + idx + 1, qy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
        }
    }
    __syncthreads();
    if (LDS_TILE && spread_ok) {
        for (int k = tid; k < nt; k += PB) a.tile[k] = (int64_t)lds_tile[k];
    }
    if (tid == 0) {
        TileDesc d;
        d.i0w = wrap(i0 == 0x7fffffff ? 0 : i0, a.nx);
        d.j0 = j0 == 0x7fffffff ? 0 : j0;
        d.w = w;
        d.h = h;
        d.scale = scale;
        d.active = spread_ok ? 1 : 0;
        d.pad0 = d.pad1 = 0;
        *a.desc = d;
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
            const bool ok = mls_shape(X[k] + 1.2 * NX[k], fluid_row(Y[k] + 1.2 * NY[k], a.ny), a.ny, m, true);
            if (!ok) flags |= FLAG_MLS;
            double dr[9], jxn[9], jyn[9];
            gather9<T>(a.f, a.nx, a.ny, a.pitch, a.plane, m, dr, jxn, jyn);
            double rp = 0.0, gxx = 0.0, gxy = 0.0, gyx = 0.0, gyy = 0.0;
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int e = 3 * b + c;
                    double fbx = 0.0, fby = 0.0;
                    if (spread_ok && b < m.nys && c < m.nxs) {
                        int di = m.i0 + c - i0;
                        di = ((di % a.nx) + a.nx) % a.nx;  // the probe may sit on another image
                        const int dj = m.j0 + b - j0;
                        if (di < w && dj >= 0 && dj < h) {
                            const int idx = 2 * (dj * w + di);
                            int64_t qx, qy;
                            if (LDS_TILE) {
                                qx = (int64_t)lds_tile[idx];
                                qy = (int64_t)lds_tile[idx + 1];
                            } else {
                                qx = __hip_atomic_load(a.tile + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                qy = __hip_atomic_load(a.tile + idx + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            }
                            fbx = ldexp((double)qx, -scale);
                            fby = ldexp((double)qy, -scale);
                        }
                    }
                    const double rho = 1.0 + dr[e];
                    const double vx = (jxn[e] + 0.5 * (a.gx + fbx)) / rho;
                    const double vy = (jyn[e] + 0.5 * (a.gy + fby)) / rho;
                    rp += m.phi[e] * rho;
                    gxx += m.psx[e] * vx;
                    gxy += m.psy[e] * vx;
                    gyx += m.psx[e] * vy;
                    gyy += m.psy[e] * vy;
                }
            const double p = (rp - 1.0) * (1.0 / 3.0);
            const double sxx = rp * a.nu * (2.0 * gxx), syy = rp * a.nu * (2.0 * gyy);
            const double sxy = rp * a.nu * (gxy + gyx);
            if (ok) {
                TX[k] = (-p * NX[k] + sxx * NX[k] + sxy * NY[k]) * S[k];
                TY[k] = (-p * NY[k] + sxy * NX[k] + syy * NY[k]) * S[k];
            }
            D[k] = Y[k] + 0.5;
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
            const double rx = X[k] - xc, ry = Y[k] - yc;
            const uint8_t b = bond_update(LIG[k], BND[k], D[k], Tf, bp, a.seed, step, (uint32_t)l, a.pid);
            a.bond[l] = b;
            acc[0] += TX[k];
            acc[1] += TY[k];
            acc[2] += rx * TY[k] - ry * TX[k];
            if (b) {
                const double mag = a.sigma * (D[k] - a.y_eq);
                const double fx = mag * NX[k], fy = mag * NY[k];
                acc[3] += fx;
                acc[4] += fy;
                acc[5] += rx * fy - ry * fx;
                ++nb;
            }
        }
    }
    block_sum<6>(acc, shd);
    {
        int v[2] = {nb, flags};
        const int op[2] = {0, 1};
        block_int<2>(v, op, shi);
        nb = v[0];
        flags = v[1];
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
        const double nux = (2.0 / 3.0) * (2.0 * ux - 0.5 * st->ux1 + Fx / a.mass);
        const double nuy = (2.0 / 3.0) * (2.0 * uy - 0.5 * st->uy1 + Fy / a.mass);
        const double nom = (2.0 / 3.0) * (2.0 * om - 0.5 * st->om1 + M / a.inertia);
        const double nxc = (2.0 / 3.0) * (2.0 * xc - 0.5 * st->xc1 + nux);
        const double nyc = (2.0 / 3.0) * (2.0 * yc - 0.5 * st->yc1 + nuy);
        const double nth = (2.0 / 3.0) * (2.0 * th - 0.5 * st->th1 + nom);
        if (!(isfinite(Fx) && isfinite(Fy) && isfinite(M) && isfinite(nux) && isfinite(nuy) && isfinite(nom)))
            fl |= FLAG_NONFINITE;
        st->xc1 = xc;
        st->yc1 = yc;
        st->th1 = th;
        st->ux1 = ux;
        st->uy1 = uy;
        st->om1 = om;
        st->xc = nxc;
        st->yc = nyc;
        st->th = nth;
        st->ux = nux;
        st->uy = nuy;
        st->om = nom;
        st->step = step + 1;
        lbib_particle_state r;
        r.step = step;
        r.xc = nxc;
        r.yc = nyc;
        r.theta = nth;
        r.ux = nux;
        r.uy = nuy;
        r.omega = nom;
        r.fx = Fx;
        r.fy = Fy;
        r.torque = M;
        r.fx_hydro = hx;
        r.fy_hydro = hy;
        r.m_hydro = hm;
        r.fx_bond = bx_;
        r.fy_bond = by_;
        r.m_bond = bm;
        r.fy_wall = fw;
        r.gap = gap;
        r.n_bonds = nb;
        r.n_probing = nprobe;
        st->last = r;
        const int64_t kk = step - a.trace_start;
        if (a.trace && kk >= 0 && kk < a.trace_cap) a.trace[kk] = r;
        if (fl) atomicOr(a.flags, fl);
    }
}

template <typename T, int MPT>
hipError_t launch_particle_mpt(const ParticleArgs<T>& a, hipStream_t stream)
{
    const size_t tile_bytes = (size_t)a.cap_w * a.cap_h * 2 * sizeof(unsigned long long);
    if (tile_bytes <= 60 * 1024)  // leaves room for the static reduction arrays in 64 KB
        hipLaunchKernelGGL((particle_kernel<T, MPT, true>), dim3(1), dim3(PB), tile_bytes, stream, a);
    else
        hipLaunchKernelGGL((particle_kernel<T, MPT, false>), dim3(1), dim3(PB), 0, stream, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_particle(const ParticleArgs<T>& a, hipStream_t stream)
{
    if (a.nl <= PB) return launch_particle_mpt<T, 1>(a, stream);
    if (a.nl <= 2 * PB) return launch_particle_mpt<T, 2>(a, stream);
    if (a.nl <= 4 * PB) return launch_particle_mpt<T, 4>(a, stream);
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

__global__ __launch_bounds__(256) void copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) dst[k] = src[k];
}

hipError_t launch_copy(const float4* src, float4* dst, int64_t n, hipStream_t stream)
{
    hipLaunchKernelGGL(copy_kernel, dim3(256 * 64), dim3(256), 0, stream, src, dst, n);
    return hipGetLastError();
}

template hipError_t launch_init<float>(float*, int32_t, int32_t, int32_t, int64_t, double, hipStream_t);
template hipError_t launch_init<double>(double*, int32_t, int32_t, int32_t, int64_t, double, hipStream_t);
template hipError_t launch_sweep<float>(const float*, float*, const SweepArgs&, const TileDesc*, const int64_t*,
                                        hipStream_t);
template hipError_t launch_sweep<double>(const double*, double*, const SweepArgs&, const TileDesc*, const int64_t*,
                                         hipStream_t);
template hipError_t launch_particle<float>(const ParticleArgs<float>&, hipStream_t);
template hipError_t launch_particle<double>(const ParticleArgs<double>&, hipStream_t);

}  // namespace lbib
