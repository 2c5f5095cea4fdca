// lbib_device.hpp -- device functions of the LB-IB adhesion step (gfx950).
//
// Lattice constants of D2Q9 (eq 3 and the weights below it), the Philox4x32-10 counter-based
// generator used for the bond draws (Salmon et al., SC'11), the moving-least-squares shape
// functions used for interpolation, spreading and probe derivatives, and the per-element
// stochastic bond decision (eq 10-11).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbib_internal.hpp"

namespace lbib {
namespace dev {

// ---------------------------------------------------------------------------------------
// D2Q9
// ---------------------------------------------------------------------------------------
constexpr int kEx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kEy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr double kW[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                          1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

// Element index of population q of node (i, j) at the start of a step, in the two storage
// layouts of a population buffer (element q plane + j pitch + i: row-interleaved [j][q][i]
// with plane = the padded row and pitch = nine of them, or planes [q][j][i] with pitch = the
// padded row and plane = pitch ny):
//  - push: the buffer holds the streamed populations, each at its own node;
//  - pull: the buffer holds the previous step's post-collision populations at the node that
//    emitted them; population q of (i, j) is the one emitted along e_q by (i - e_x, j - e_y)
//    (x periodic), or, when that link crosses a wall, the opposite population emitted by
//    (i, j) itself (half-way bounce-back).
// Streaming is a permutation, so both layouts present the same values.
__device__ __forceinline__ int64_t pop_index(int q, int i, int j, int nx, int ny, int pitch, int64_t plane, bool pull)
{
    // selects rather than branches, so a caller's loads of several nodes can all be in flight
    const int sj = j - kEy[q];
    const bool wall = sj < 0 || sj >= ny;
    int si = i - kEx[q];
    si = si < 0 ? si + nx : (si >= nx ? si - nx : si);
    const bool moved = pull && !wall;
    const int qq = pull && wall ? kOpp[q] : q;
    return qq * plane + (int64_t)(moved ? sj : j) * pitch + (moved ? si : i);
}

// Loads and stores of one stored population (f - w, in the compute type of the storage),
// optionally past the caches (nt).
__device__ __forceinline__ double st_load(const double* p, int64_t i, double, bool nt)
{
    return nt ? __builtin_nontemporal_load(p + i) : p[i];
}
__device__ __forceinline__ double st_load(const float* p, int64_t i, double, bool nt)
{
    return (double)(nt ? __builtin_nontemporal_load(p + i) : p[i]);
}
__device__ __forceinline__ float st_load(const half_t* p, int64_t i, double inv_scale, bool nt)
{
    const uint16_t* r = (const uint16_t*)p;
    const uint16_t b = nt ? __builtin_nontemporal_load(r + i) : r[i];
    // x s as one mixed-precision fma (adding -0 leaves every product, -0 included, unchanged)
    return __builtin_fmaf((float)__builtin_bit_cast(_Float16, b), (float)inv_scale, -0.0f);
}
__device__ __forceinline__ float st_load(const bf16_t* p, int64_t i, double, bool nt)
{
    const uint16_t* r = (const uint16_t*)p;
    const uint16_t b = nt ? __builtin_nontemporal_load(r + i) : r[i];
    return __builtin_bit_cast(float, (uint32_t)b << 16);
}

__device__ __forceinline__ float st_load(const half_neq_t* p, int64_t i, double inv_scale, bool nt)
{
    return st_load((const half_t*)p, i, inv_scale, nt);
}
__device__ __forceinline__ float st_load(const bf16_neq_t* p, int64_t i, double inv_scale, bool nt)
{
    return st_load((const bf16_t*)p, i, inv_scale, nt);
}

// Store policies: plain; non-temporal (past the caches); coherent (an agent-scope store,
// visible to other XCDs without cache maintenance, for data a concurrently running launch
// reads).  A bool argument selects plain or non-temporal.
enum : int { ST_PLAIN = 0, ST_NT = 1, ST_COH = 2 };
template <typename S>
__device__ __forceinline__ void put(S* p, S v, int pol)
{
    if (pol == ST_COH)
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else if (pol == ST_NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}
__device__ __forceinline__ void st_store(double* p, int64_t i, double v, double, int pol)
{
    put(p + i, v, pol);
}
__device__ __forceinline__ void st_store(float* p, int64_t i, double v, double, int pol)
{
    put(p + i, (float)v, pol);
}
__device__ __forceinline__ void st_store(half_t* p, int64_t i, float v, double scale, int pol)
{
    put((uint16_t*)p + i, __builtin_bit_cast(uint16_t, (_Float16)(v * (float)scale)), pol);
}
__device__ __forceinline__ void st_store(bf16_t* p, int64_t i, float v, double, int pol)
{
    // the conversion instruction: round to nearest even, NaN stays a NaN
    put((uint16_t*)p + i, __builtin_bit_cast(uint16_t, (__bf16)v), pol);
}

__device__ __forceinline__ void st_store(half_neq_t* p, int64_t i, double v, double scale, int pol)
{
    st_store((half_t*)p, i, (float)v, scale, pol);
}
__device__ __forceinline__ void st_store(bf16_neq_t* p, int64_t i, double v, double scale, int pol)
{
    st_store((bf16_t*)p, i, (float)v, scale, pol);
}

// The three FP32 moments (rho - 1, u_x, u_y) of every node of a non-equilibrium buffer follow
// its nine population segments, laid out like them: moment k of node (i, j) is element
// k plane + j neq_mpitch + i from neq_moments.  Row-interleaved buffers (pitch = 9 plane, which
// population planes never satisfy: there plane = pitch ny with ny >= 4) hold rows [j][k][i];
// population planes are followed by three moment planes.
__device__ __forceinline__ int64_t neq_mpitch(int pitch, int64_t plane)
{
    return (int64_t)pitch == 9 * plane ? 3 * plane : (int64_t)pitch;
}
__device__ __forceinline__ int64_t neq_mbase(int pitch, int64_t plane, int ny)
{
    return (int64_t)pitch == 9 * plane ? (int64_t)pitch * ny : 9 * plane;
}
template <typename T>
__device__ __forceinline__ const float* neq_moments(const T* f, int pitch, int64_t plane, int ny)
{
    return (const float*)((const uint16_t*)f + neq_mbase(pitch, plane, ny));
}
template <typename T>
__device__ __forceinline__ float* neq_moments(T* f, int pitch, int64_t plane, int ny)
{
    return (float*)((uint16_t*)f + neq_mbase(pitch, plane, ny));
}

// e_q . (x, y) for the D2Q9 directions, formed so that the value for the opposite direction
// is the exact negative.
template <typename C>
__device__ __forceinline__ C e_dot(int q, C x, C y)
{
    switch (q) {
        case 1: return x;
        case 2: return y;
        case 3: return -x;
        case 4: return -y;
        case 5: return x + y;
        case 6: return y - x;
        case 7: return -(x + y);
        case 8: return x - y;
        default: return (C)0;
    }
}

// Shifted equilibrium (eq 2) f_eq,q - w_q = w_q (drho + rho A), A = 3 e.u + 9/2 (e.u)^2 -
// 3/2 u^2, as w_q r_q with r_q = drho + rho (e.u (3 + 9/2 e.u) + P) and P = -3/2 u^2 per node:
// three fused operations per direction once rho and P are known (r_0 = drho + rho P).  The
// writers (neq_encode) and the readers (load_node, update_load) of the f - f_eq storages form
// r_q from the same stored FP32 moments with this one sequence, so both sides agree bit for
// bit; e.u for the opposite direction is the exact negative (e_dot).
template <typename C>
struct FeqNode {
    C drho, rho, P;
};
template <typename C>
__device__ __forceinline__ FeqNode<C> feq_node(C drho, C ux, C uy)
{
    return FeqNode<C>{drho, (C)1 + drho, (C)-1.5 * fma(ux, ux, uy * uy)};
}
template <typename C>
__device__ __forceinline__ C feq_r(const FeqNode<C>& n, C eu)
{
    return fma(n.rho, fma(eu, fma((C)4.5, eu, (C)3), n.P), n.drho);
}
template <typename C>
__device__ __forceinline__ C feq_r0(const FeqNode<C>& n)
{
    return fma(n.rho, n.P, n.drho);
}
// f_eq,q - w_q of direction q (eu: e_q.u).
template <typename C>
__device__ __forceinline__ C feq_shift_eu(int q, const FeqNode<C>& n, C eu)
{
    return (C)kW[q] * (q == 0 ? feq_r0<C>(n) : feq_r<C>(n, eu));
}
template <typename C>
__device__ __forceinline__ C feq_shift(int q, C drho, C ux, C uy)
{
    return feq_shift_eu<C>(q, feq_node<C>(drho, ux, uy), e_dot<C>(q, ux, uy));
}

// The node that emitted population q of node (i, j) and the direction it emitted it in:
// (i - e_x, j - e_y) along q, or (i, j) itself along the opposite direction when that link
// crosses a wall.
__device__ __forceinline__ void pop_source(int q, int i, int j, int nx, int ny, int& si, int& sj, int& dir)
{
    const int jj = j - kEy[q];
    const bool wall = jj < 0 || jj >= ny;
    int ii = i - kEx[q];
    ii = ii < 0 ? ii + nx : (ii >= nx ? ii - nx : ii);
    si = wall ? i : ii;
    sj = wall ? j : jj;
    dir = wall ? kOpp[q] : q;
}

// Density and momentum of shifted populations g_q = f_q - w_q: rho = 1 + sum g (the weights
// sum to one), j = sum g e (the weights carry no momentum).
template <typename R, typename S>
__device__ __forceinline__ void shifted_moments(const S* g, R& drho, R& jx, R& jy)
{
    R g0 = (R)g[0], g1 = (R)g[1], g2 = (R)g[2], g3 = (R)g[3], g4 = (R)g[4];
    R g5 = (R)g[5], g6 = (R)g[6], g7 = (R)g[7], g8 = (R)g[8];
    drho = ((g0 + g1) + (g2 + g3)) + ((g4 + g5) + (g6 + g7)) + g8;
    jx = (g1 - g3) + (g5 - g7) + (g8 - g6);
    jy = (g2 - g4) + (g5 - g7) + (g6 - g8);
}

// ---------------------------------------------------------------------------------------
// Philox4x32-10: ten rounds of the Philox S-box on a 128-bit counter; the 64-bit key is
// advanced by the Weyl increments (0x9E3779B9, 0xBB67AE85) between rounds.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                              uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a = c0, b = c2;
        const uint32_t hi0 = __umulhi(0xD2511F53u, a), lo0 = 0xD2511F53u * a;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, b), lo1 = 0xCD9E8D57u * b;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// An event of probability P fires when a uniform 32-bit draw r satisfies r < T(P) with
// T(P) = floor(P 2^32); T(0) = 0 never fires, T(1) = 2^32 always does; NaN counts as 0.
__device__ __forceinline__ uint64_t prob_threshold(double P)
{
    if (!(P > 0.0)) return 0ull;
    if (P >= 1.0) return 4294967296ull;
    return (uint64_t)floor(P * 4294967296.0);
}

// ---------------------------------------------------------------------------------------
// Moving least squares on the lattice (reading of the MLS reconstruction the paper cites):
// support = nodes with |i - X| < 1.5 (x periodic) and |j - Y| < 1.5 inside the fluid rows
// 0..ny-1; basis [1, dx, dy] with d = node - point; weight w(|dx|/1.5) w(|dy|/1.5) with w the
// cubic B-spline.  The support is a tensor grid of nxs x nys nodes starting at (i0, j0)
// (i0 unwrapped); entry k = 3 b + a refers to node (i0 + a, j0 + b).
// ---------------------------------------------------------------------------------------
struct Mls {
    int i0, j0, nxs, nys;
    double phi[9], psx[9], psy[9];
};

__device__ __forceinline__ double bspline(double s)
{
    if (s <= 0.5) return 2.0 / 3.0 + s * s * (4.0 * s - 4.0);
    if (s < 1.0) {
        const double r = 1.0 - s;
        return (4.0 / 3.0) * r * r * r;
    }
    return 0.0;
}

// Returns false when the moment matrix is singular (empty or degenerate support).
__device__ inline bool mls_shape(double X, double Y, int ny, Mls& m, bool want_grad)
{
    if (!(fabs(X) < 1e9 && fabs(Y) < 1e9)) {  // non-finite or absurd point: empty support
        m.i0 = m.j0 = 0;
        m.nxs = m.nys = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k) m.phi[k] = m.psx[k] = m.psy[k] = 0.0;
        return false;
    }
    const int ilo = (int)floor(X - 1.5) + 1, ihi = (int)ceil(X + 1.5) - 1;
    int jlo = (int)floor(Y - 1.5) + 1, jhi = (int)ceil(Y + 1.5) - 1;
    jlo = jlo < 0 ? 0 : jlo;
    jhi = jhi > ny - 1 ? ny - 1 : jhi;
    m.i0 = ilo;
    m.j0 = jlo;
    m.nxs = ihi - ilo + 1;
    m.nys = jhi - jlo + 1;
    double wx[3], dx[3], wy[3], dy[3];
    // one-dimensional moments; the weight is a tensor product, so the 3x3 moment matrix is
    // built from products of these sums
    double x0 = 0, x1 = 0, x2 = 0, y0 = 0, y1 = 0, y2 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        dx[a] = (double)(ilo + a) - X;
        wx[a] = a < m.nxs ? bspline(fabs(dx[a]) * (1.0 / 1.5)) : 0.0;
        x0 += wx[a];
        x1 += wx[a] * dx[a];
        x2 += wx[a] * dx[a] * dx[a];
        dy[a] = (double)(jlo + a) - Y;
        wy[a] = (a < m.nys && m.nys > 0) ? bspline(fabs(dy[a]) * (1.0 / 1.5)) : 0.0;
        y0 += wy[a];
        y1 += wy[a] * dy[a];
        y2 += wy[a] * dy[a] * dy[a];
    }
    const double a00 = x0 * y0, a01 = x1 * y0, a02 = x0 * y1;
    const double a11 = x2 * y0, a12 = x1 * y1, a22 = x0 * y2;
    // symmetric inverse by cofactors
    const double c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22, c02 = a01 * a12 - a02 * a11;
    const double c11 = a00 * a22 - a02 * a02, c12 = a01 * a02 - a00 * a12, c22 = a00 * a11 - a01 * a01;
    const double det = a00 * c00 + a01 * c01 + a02 * c02;
    if (!(det > 0.0) || m.nys <= 0) {
#pragma unroll
        for (int k = 0; k < 9; ++k) m.phi[k] = m.psx[k] = m.psy[k] = 0.0;
        return false;
    }
    const double id = 1.0 / det;
    const double i00 = c00 * id, i01 = c01 * id, i02 = c02 * id, i11 = c11 * id, i12 = c12 * id, i22 = c22 * id;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double W = wx[a] * wy[b];
            m.phi[3 * b + a] = W * (i00 + i01 * dx[a] + i02 * dy[b]);
            if (want_grad) {
                m.psx[3 * b + a] = W * (i01 + i11 * dx[a] + i12 * dy[b]);
                m.psy[3 * b + a] = W * (i02 + i12 * dx[a] + i22 * dy[b]);
            }
        }
    }
    return true;
}

// Moving top wall: a population that reaches the top row through the wall (directions 7
// and 8, reflected from 5 and 6 at the same node) carries -2 w e.u_wall / cs^2, i.e.
// -u_w/6 and +u_w/6.  Buffers hold the reflected values without it and every load of level
// n adds it, in either layout, so both layouts store the same values.
template <typename C>
__device__ __forceinline__ void wall_reflect(C (&g)[9], int j, int ny, double uw6)
{
    if (j == ny - 1 && uw6 != 0.0) {
        g[7] -= (C)uw6;
        g[8] += (C)uw6;
    }
}

// The nine shifted populations g_q = f_q - w_q of node (i, j) at the start of a step, read
// from a buffer in either layout as type R: the stored value, plus, for the non-equilibrium
// storages, the shifted equilibrium of the node that emitted it (from the stored moments),
// plus the moving wall's term.
// Three consecutive FP32 values of a row, read by one load (global loads of several dwords
// need only dword alignment).
struct alignas(4) RowTriple {
    float v[3];
};

template <typename T, typename R>
__device__ __forceinline__ void load_node(const T* f, int i, int j, int nx, int ny, int pitch, int64_t plane, bool pull,
                                          double inv_scale, double uw6, bool nt, R (&g)[9])
{
#pragma unroll
    for (int q = 0; q < 9; ++q) g[q] = (R)st_load(f, pop_index(q, i, j, nx, ny, pitch, plane, pull), inv_scale, nt);
    if constexpr (St<T>::neq) {
        const float* m = neq_moments(f, pitch, plane, ny);
        const int64_t mp = neq_mpitch(pitch, plane);
        // The moments of the 3 x 3 neighbourhood, mm[r][k][c] = moment k of node
        // (i - 1 + c, j - 1 + r) (periodic in x): each row's three columns come from one load
        // of columns c0 .. c0 + 2, c0 kept inside the row (nx >= 4), and at the two edge
        // columns the column across the periodic edge from a load of its own.  Rows past a
        // wall are read clamped and never used (such links take the node's own moments).
        const int c0 = min(max(i - 1, 0), nx - 3);
        const bool wl = i == 0, wr = i == nx - 1;
        const int cw = wl ? nx - 1 : 0;
        float mm[3][3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int64_t row = (int64_t)min(max(j - 1 + r, 0), ny - 1) * mp;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const RowTriple t = *(const RowTriple*)(m + k * plane + row + c0);
                float e = 0.0f;
                if (wl || wr) e = m[k * plane + row + cw];
                mm[r][k][0] = wl ? e : (wr ? t.v[1] : t.v[0]);
                mm[r][k][1] = wl ? t.v[0] : (wr ? t.v[2] : t.v[1]);
                mm[r][k][2] = wl ? t.v[1] : (wr ? e : t.v[2]);
            }
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            // the node that emitted population q (pop_source): (i - e_x, j - e_y) along q, or
            // the node itself along opp(q) where that link crosses a wall
            const int sj = j - kEy[q];
            const bool wall = sj < 0 || sj >= ny;
            const int r = 1 - kEy[q], c = 1 - kEx[q];  // constants once the loop is unrolled
            const R d = (R)(wall ? mm[1][0][1] : mm[r][0][c]);
            const R x = (R)(wall ? mm[1][1][1] : mm[r][1][c]), y = (R)(wall ? mm[1][2][1] : mm[r][2][c]);
            const FeqNode<R> n = feq_node<R>(d, x, y);
            const R eu = e_dot<R>(q, x, y);  // e_dir.u = -e_q.u for a reflected population
            g[q] = fma((R)kW[q], q == 0 ? feq_r0<R>(n) : feq_r<R>(n, wall ? -eu : eu), g[q]);
        }
    }
    wall_reflect<R>(g, j, ny, uw6);
}

__device__ __forceinline__ int wrap(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

// ---------------------------------------------------------------------------------------
// Bonds (eq 10-11)
// ---------------------------------------------------------------------------------------
struct BondParams {
    double y_cr, y_eq, sigma, sigma_star, k_f, k_r0, kBT;
};

// Bond flag after the update of element l.  Tf = T(P_f) of the particle (eq 10).  A bond
// present at the start of the step ruptures when draw r1 < T(P_r) (eq 11, bond length d);
// otherwise a ligand within y_cr of the wall forms a bond when draw r0 < Tf.  A bond broken
// in this step does not re-form in it.  Key (seed lo, seed hi), counter (step lo, step hi,
// l, pid).
__device__ __forceinline__ uint8_t bond_update(bool ligand, bool bonded, double d, uint64_t Tf, const BondParams& p,
                                               uint64_t seed, int64_t step, uint32_t l, uint32_t pid)
{
    if (!ligand) return 0;
    uint32_t c0 = (uint32_t)(uint64_t)step, c1 = (uint32_t)((uint64_t)step >> 32), c2 = l, c3 = pid;
    philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    if (bonded) {
        const double ext = d - p.y_eq;
        const double Pr = -expm1(-p.k_r0 * exp((p.sigma - p.sigma_star) * ext * ext / (2.0 * p.kBT)));
        return (uint64_t)c1 < prob_threshold(Pr) ? 0 : 1;
    }
    if (d < p.y_cr) return (uint64_t)c0 < Tf ? 1 : 0;
    return 0;
}

}  // namespace dev
}  // namespace lbib
