/*
 * lbib_oracle.c -- plain FP64 CPU oracle of the LB-IB particle-adhesion time step
 * (Coclite et al., "Predicting Different Adhesive Regimens of Circulating Particles at
 * Blood Capillary Walls", arXiv 1808.01448).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no source with the GPU library: its own lattice
 * constants, geometry, moving-least-squares, Philox generator and rigid-body step.
 *
 * Every function cites the passage of the paper it follows.  Where the paper is silent or
 * garbled the reading taken is named in the comment.
 *
 * Units: lattice units, dx = dt = 1 (section "Fluid-structure interaction strategy").
 * Storage: plain populations f[q][j][i] (x fastest), FP64.
 * Grid: node (i, j) sits at (x, y) = (i, j); x periodic; half-way bounce-back walls at
 *       y = -1/2 and y = ny - 1/2, so the channel height is H = ny.
 *
 * Parity pins: every exported function is pinned by the CPU test-suite against closed
 * forms, invariants, library routines or brute force (see tests/test_oracle_*.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define CS2 (1.0 / 3.0) /* squared lattice speed of sound, cs = 1/sqrt(3) (below eq 1) */

/* D2Q9 velocity set, eq 3: e_0 = 0; e_1..e_4 = (cos, sin)((i-1) pi/2);
 * e_5..e_8 = sqrt(2) (cos, sin)((2i-9) pi/4).  Weights below eq 3. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WQ[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

#define IDX(q, j, i, nx, ny) ((((size_t)(q)) * (size_t)(ny) + (size_t)(j)) * (size_t)(nx) + (size_t)(i))

void orc_lattice(int32_t* ex, int32_t* ey, double* w, int32_t* opp)
{
    for (int q = 0; q < 9; ++q) {
        ex[q] = EX[q];
        ey[q] = EY[q];
        w[q] = WQ[q];
        opp[q] = OPP[q];
    }
}

/* ------------------------------------------------------------------------------------- */
/* Fluid: eq 1-6                                                                          */
/* ------------------------------------------------------------------------------------- */

/* Equilibrium, eq 2 (second-order Hermite expansion of the Maxwell-Boltzmann distribution). */
void orc_feq(double rho, double ux, double uy, double* out)
{
    double uu = ux * ux + uy * uy;
    for (int q = 0; q < 9; ++q) {
        double eu = EX[q] * ux + EY[q] * uy;
        out[q] = WQ[q] * rho * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* Forcing term, eq 4 (Guo et al.):
 *   F_i = (1 - 1/(2 tau)) w_i [ (e_i - u)/cs^2 + (e_i . u) e_i / cs^4 ] . F            */
void orc_guo(double tau, double ux, double uy, double Fx, double Fy, double* out)
{
    for (int q = 0; q < 9; ++q) {
        double eu = EX[q] * ux + EY[q] * uy;
        double cx = (EX[q] - ux) / CS2 + eu * EX[q] / (CS2 * CS2);
        double cy = (EY[q] - uy) / CS2 + eu * EY[q] / (CS2 * CS2);
        out[q] = (1.0 - 1.0 / (2.0 * tau)) * WQ[q] * (cx * Fx + cy * Fy);
    }
}

/* Moments, eq 5-6.  Eq 6 as printed is garbled; the reading taken is the Guo half-force
 * shift rho u = sum_i f_i e_i + (dt/2) F with F the total body force on the node. */
void orc_moments(const double* f9, double Fx, double Fy, double* rho, double* ux, double* uy)
{
    double r = 0.0, jx = 0.0, jy = 0.0;
    for (int q = 0; q < 9; ++q) {
        r += f9[q];
        jx += f9[q] * EX[q];
        jy += f9[q] * EY[q];
    }
    *rho = r;
    *ux = (jx + 0.5 * Fx) / r;
    *uy = (jy + 0.5 * Fy) / r;
}

/* One collide-and-stream sweep, eq 1 with the forcing term of eq 4 added on the right-hand
 * side (dt = 1):  f*_i = f_i - (f_i - f_i^eq)/tau + F_i,  then f_i(x + e_i) = f*_i(x).
 * x is periodic.  With walls != 0 a link leaving the channel through y = -1/2 or
 * y = ny - 1/2 is reflected back into the opposite direction at the same node (half-way
 * bounce-back); the top wall moves along x at speed uw, which the reflection carries as
 * f_opp(i)(x) = f*_i(x) - 2 w_i rho_w (e_i . u_wall) / cs^2 with rho_w = 1 (the reading of
 * the moving wall of the shear setup, "Modeling the adhesion dynamics" section, for
 * half-way walls; the paper's own walls are Zou-He known-velocity nodes).  With
 * walls == 0 y is periodic too (test mode).  The body force on node (i, j) is (gx, gy)
 * plus fib (two planes [c][j][i]) when given.  Rows are independent, so the OpenMP split
 * cannot change any result bit. */
void orc_collide_stream_uw(int32_t nx, int32_t ny, int32_t walls, double uw, double tau, double gx, double gy,
                           const double* fib, const double* fin, double* fout)
{
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            double f9[9], feq[9], src[9];
            for (int q = 0; q < 9; ++q) f9[q] = fin[IDX(q, j, i, nx, ny)];
            double Fx = gx, Fy = gy;
            if (fib) {
                Fx += fib[IDX(0, j, i, nx, ny)];
                Fy += fib[IDX(1, j, i, nx, ny)];
            }
            double rho, ux, uy;
            orc_moments(f9, Fx, Fy, &rho, &ux, &uy);
            orc_feq(rho, ux, uy, feq);
            orc_guo(tau, ux, uy, Fx, Fy, src);
            for (int q = 0; q < 9; ++q) {
                double post = f9[q] - (f9[q] - feq[q]) / tau + src[q];
                int id = ((i + EX[q]) % nx + nx) % nx;
                int jd = j + EY[q];
                if (walls) {
                    if (jd < 0)
                        fout[IDX(OPP[q], j, i, nx, ny)] = post;
                    else if (jd >= ny)
                        fout[IDX(OPP[q], j, i, nx, ny)] = post - 2.0 * WQ[q] * (EX[q] * uw) / CS2;
                    else
                        fout[IDX(q, jd, id, nx, ny)] = post;
                } else {
                    jd = (jd % ny + ny) % ny;
                    fout[IDX(q, jd, id, nx, ny)] = post;
                }
            }
        }
    }
}

/* The same sweep with resting walls. */
void orc_collide_stream(int32_t nx, int32_t ny, int32_t walls, double tau, double gx, double gy,
                        const double* fib, const double* fin, double* fout)
{
    orc_collide_stream_uw(nx, ny, walls, 0.0, tau, gx, gy, fib, fin, fout);
}

/* ------------------------------------------------------------------------------------- */
/* Moving least squares (the reconstruction the paper cites for interpolation, spreading  */
/* and the probe derivatives).  The paper gives neither support, basis nor weight; the    */
/* reading: support = nodes with |i - X| < 1.5 (x by minimum image) and |j - Y| < 1.5     */
/* inside 0 <= j <= ny-1; linear basis p = [1, dx, dy] with dx = node - point; weight the  */
/* tensor product of the cubic B-spline w(s), s = |d|/1.5.                                 */
/* ------------------------------------------------------------------------------------- */

#define MLS_R 1.5

/* Cubic B-spline on [0, 1]: 2/3 - 4 s^2 + 4 s^3 up to s = 1/2, (4/3)(1 - s)^3 beyond (the
 * factored form keeps the outer branch non-negative near s = 1). */
static double spline_w(double s)
{
    if (s <= 0.5) return 2.0 / 3.0 - 4.0 * s * s + 4.0 * s * s * s;
    if (s <= 1.0) {
        double r = 1.0 - s;
        return (4.0 / 3.0) * r * r * r;
    }
    return 0.0;
}

double orc_spline_w(double s) { return spline_w(s); }

/* Solve the 3x3 system A C = B (B has m columns, row-major 3 x m) in place by Gaussian
 * elimination with partial pivoting.  Returns 0, or -1 for an exactly singular pivot. */
static int solve3(double A[3][3], double* B, int m)
{
    for (int c = 0; c < 3; ++c) {
        int p = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(A[r][c]) > fabs(A[p][c])) p = r;
        if (A[p][c] == 0.0) return -1;
        if (p != c) {
            for (int k = 0; k < 3; ++k) {
                double t = A[c][k];
                A[c][k] = A[p][k];
                A[p][k] = t;
            }
            for (int k = 0; k < m; ++k) {
                double t = B[c * m + k];
                B[c * m + k] = B[p * m + k];
                B[p * m + k] = t;
            }
        }
        for (int r = c + 1; r < 3; ++r) {
            double l = A[r][c] / A[c][c];
            for (int k = c; k < 3; ++k) A[r][k] -= l * A[c][k];
            for (int k = 0; k < m; ++k) B[r * m + k] -= l * B[c * m + k];
        }
    }
    for (int c = 2; c >= 0; --c) {
        for (int k = 0; k < m; ++k) {
            double s = B[c * m + k];
            for (int r = c + 1; r < 3; ++r) s -= A[c][r] * B[r * m + k];
            B[c * m + k] = s / A[c][c];
        }
    }
    return 0;
}

/* MLS shape functions at the point (X, Y).  Writes up to 9 support nodes (wrapped i, j),
 * their offsets, phi (interpolation: u(X) ~ sum phi_k u_k) and psix/psiy (the diffuse
 * derivative: du/dx(X) ~ sum psix_k u_k).  Node order: j ascending, then i ascending.
 * Returns the node count, or -1 when the moment matrix is singular. */
int32_t orc_mls(int32_t nx, int32_t ny, double X, double Y, int32_t* ni, int32_t* nj, double* phi,
                double* psix, double* psiy)
{
    double dx[9], dy[9], W[9];
    int n = 0;
    int fx = (int)floor(X), fy = (int)floor(Y);
    for (int jc = fy - 1; jc <= fy + 2; ++jc) {
        if (jc < 0 || jc > ny - 1) continue;
        double ddy = (double)jc - Y;
        if (fabs(ddy) >= MLS_R) continue;
        for (int ic = fx - 1; ic <= fx + 2; ++ic) {
            double ddx = (double)ic - X;
            if (fabs(ddx) >= MLS_R) continue;
            ni[n] = ((ic % nx) + nx) % nx;
            nj[n] = jc;
            dx[n] = ddx;
            dy[n] = ddy;
            W[n] = spline_w(fabs(ddx) / MLS_R) * spline_w(fabs(ddy) / MLS_R);
            ++n;
        }
    }
    double A[3][3] = {{0}};
    double B[3 * 9];
    for (int k = 0; k < n; ++k) {
        double p[3] = {1.0, dx[k], dy[k]};
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) A[r][c] += W[k] * p[r] * p[c];
        B[0 * n + k] = p[0];
        B[1 * n + k] = p[1];
        B[2 * n + k] = p[2];
    }
    if (n == 0 || solve3(A, B, n) != 0) return -1;
    for (int k = 0; k < n; ++k) {
        phi[k] = W[k] * B[0 * n + k];
        psix[k] = W[k] * B[1 * n + k];
        psiy[k] = W[k] * B[2 * n + k];
    }
    return n;
}

/* ------------------------------------------------------------------------------------- */
/* Particle surface (section "Pressure and viscous stresses"): nl linear elements with     */
/* centroid, outward normal and length.  Vertices at equal arc length along the ellipse   */
/* (semi-axis a along body y, b along body x), starting at the body point (0, -a) and     */
/* running counter-clockwise.                                                             */
/* ------------------------------------------------------------------------------------- */

static double ell_speed(double a, double b, double t)
{
    double ct = cos(t), st = sin(t);
    return sqrt(b * b * ct * ct + a * a * st * st);
}

/* Arc length of the ellipse point (b sin t, -a cos t) from t = 0 to t, by composite
 * 5-point Gauss-Legendre quadrature on panels no wider than 2 pi / 2048. */
double orc_ellipse_arc(double a, double b, double t)
{
    static const double gx[5] = {-0.9061798459386640, -0.5384693101056831, 0.0, 0.5384693101056831,
                                 0.9061798459386640};
    static const double gw[5] = {0.2369268850561891, 0.4786286704993665, 0.5688888888888889,
                                 0.4786286704993665, 0.2369268850561891};
    if (t == 0.0) return 0.0;
    int panels = (int)ceil(fabs(t) / (2.0 * M_PI / 2048.0));
    if (panels < 1) panels = 1;
    double h = t / panels, s = 0.0;
    for (int p = 0; p < panels; ++p) {
        double c = (p + 0.5) * h;
        for (int k = 0; k < 5; ++k) s += gw[k] * ell_speed(a, b, c + 0.5 * h * gx[k]);
    }
    return s * 0.5 * h;
}

/* Vertices V (nl x 2), element centroids xi, outward unit normals nu and lengths S, all in
 * the body frame.  shape 0: circle of radius a (closed form); shape 1: ellipse.
 * Returns 0, or -1 on bad arguments. */
int32_t orc_geometry(int32_t shape, double a, double b, int32_t nl, double* V, double* xi, double* nu,
                     double* S)
{
    if (nl < 3 || a <= 0.0 || (shape == 1 && b <= 0.0)) return -1;
    if (shape == 0) {
        for (int k = 0; k < nl; ++k) {
            double t = 2.0 * M_PI * k / nl;
            V[2 * k] = a * sin(t);
            V[2 * k + 1] = -a * cos(t);
        }
    } else {
        double P = orc_ellipse_arc(a, b, 2.0 * M_PI);
        V[0] = 0.0;
        V[1] = -a;
        for (int k = 1; k < nl; ++k) {
            double target = P * k / nl;
            double t = 2.0 * M_PI * k / nl;
            for (int it = 0; it < 50; ++it) { /* Newton on s(t) = target */
                double dt = (orc_ellipse_arc(a, b, t) - target) / ell_speed(a, b, t);
                t -= dt;
                if (fabs(dt) < 1e-15) break;
            }
            V[2 * k] = b * sin(t);
            V[2 * k + 1] = -a * cos(t);
        }
    }
    for (int l = 0; l < nl; ++l) {
        int m = (l + 1) % nl;
        double tx = V[2 * m] - V[2 * l], ty = V[2 * m + 1] - V[2 * l + 1];
        double len = sqrt(tx * tx + ty * ty);
        S[l] = len;
        xi[2 * l] = 0.5 * (V[2 * m] + V[2 * l]);
        xi[2 * l + 1] = 0.5 * (V[2 * m + 1] + V[2 * l + 1]);
        nu[2 * l] = ty / len; /* outward for a counter-clockwise polygon */
        nu[2 * l + 1] = -tx / len;
    }
    return 0;
}

/* Ligand decoration: density rho_l = p/q ligands per element, spread evenly along the
 * perimeter (the paper: "uniformly distributed").  Element l carries a ligand iff
 * floor((l+1) p / q) - floor(l p / q) == 1, which gives floor(nl p / q) ligands. */
void orc_ligand_flags(int32_t nl, int32_t p, int32_t q, uint8_t* flags)
{
    for (int l = 0; l < nl; ++l) {
        int64_t a = ((int64_t)(l + 1) * p) / q, b = ((int64_t)l * p) / q;
        flags[l] = (uint8_t)((a - b) == 1);
    }
}

/* ------------------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,   */
/* 3", SC'11): ten rounds of the 4x32 Philox S-box, the key bumped by the Weyl constants   */
/* between rounds.                                                                        */
/* ------------------------------------------------------------------------------------- */

void orc_philox4x32_10(const uint32_t* ctr_in, const uint32_t* key_in, uint32_t* out)
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* n independent draws: out[4k..4k+3] = philox(ctr[4k..4k+3], key[2k..2k+1]). */
void orc_philox_batch(int64_t n, const uint32_t* ctr, const uint32_t* key, uint32_t* out)
{
    for (int64_t k = 0; k < n; ++k) orc_philox4x32_10(ctr + 4 * k, key + 2 * k, out + 4 * k);
}

/* Integer threshold of a probability: an event of probability P fires iff the uniform
 * 32-bit draw r satisfies r < T(P) = floor(P * 2^32); T(0) = 0 never fires, T(1) = 2^32
 * always fires.  NaN is taken as 0. */
uint64_t orc_threshold(double P)
{
    if (!(P > 0.0)) return 0;
    if (P >= 1.0) return 4294967296ull;
    return (uint64_t)floor(P * 4294967296.0);
}

/* ------------------------------------------------------------------------------------- */
/* Ligand-receptor bonds (section "Wall-particle interaction", eq 9-11).                  */
/* ------------------------------------------------------------------------------------- */

/* One stochastic bond update of one particle.
 *  d[l]   : distance of element l's centroid from the receptor wall y = -1/2;
 *  probing: ligand and d < y_cr (the critical separation for bond formation);
 *  Nl     : probing elements over all elements (eq 10), P_f = 1 - exp(-k_f Nl dt);
 *  P_r    : eq 11 with the bond length y_l = d[l] and sigma* = sigma_star;
 *  A bond present at the start of the step may rupture (draw r1 < T(P_r)); otherwise a
 *  probing ligand may form a bond (draw r0 < T(P_f)).  A bond broken in this step does not
 *  re-form in the same step.  The draws are Philox4x32-10 with key (seed lo, seed hi) and
 *  counter (step lo, step hi, l, pid).  Returns the number of bonds after the update. */
int32_t orc_bonds(int32_t nl, const uint8_t* ligand, const double* d, const uint8_t* b_in, uint8_t* b_out,
                  double y_cr, double y_eq, double sigma, double sigma_star, double k_f, double k_r0,
                  double kBT, uint64_t seed, int64_t step, uint32_t pid, int32_t* n_probing_out)
{
    int n_probing = 0;
    for (int l = 0; l < nl; ++l)
        if (ligand[l] && d[l] < y_cr) ++n_probing;
    double Nl = (double)n_probing / (double)nl;
    double Pf = -expm1(-k_f * Nl);
    uint64_t Tf = orc_threshold(Pf);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int n_bonds = 0;
    for (int l = 0; l < nl; ++l) {
        uint8_t nb = 0;
        if (ligand[l]) {
            uint32_t ctr[4] = {(uint32_t)(uint64_t)step, (uint32_t)((uint64_t)step >> 32), (uint32_t)l, pid};
            uint32_t r[4];
            orc_philox4x32_10(ctr, key, r);
            if (b_in[l]) {
                double ext = d[l] - y_eq;
                double Pr = -expm1(-k_r0 * exp((sigma - sigma_star) * ext * ext / (2.0 * kBT)));
                nb = (uint64_t)r[1] < orc_threshold(Pr) ? 0 : 1;
            } else if (d[l] < y_cr) {
                nb = (uint64_t)r[0] < Tf ? 1 : 0;
            }
        }
        b_out[l] = nb;
        n_bonds += nb;
    }
    if (n_probing_out) *n_probing_out = n_probing;
    return n_bonds;
}

/* Van der Waals-like particle-wall force, eq 12: F_w = H_k / (8 sqrt 2) sqrt(r / eps^5) along
 * the wall normal (+y, away from the bottom wall), applied at the centroid.  eps is the
 * analytic gap between the ellipse and the wall y = -1/2; r = sqrt(a b) (the radius for a
 * circle).  eps is floored at eps_min = 1e-3; eps <= 0 raises *flag. */
double orc_wall_force(double yc, double theta, double a, double b, double hamaker, double* gap,
                      int32_t* flag)
{
    double st = sin(theta), ct = cos(theta);
    double eps = yc + 0.5 - sqrt(b * b * st * st + a * a * ct * ct);
    if (gap) *gap = eps;
    if (!(eps > 0.0) && flag) *flag = 1;
    double e = eps > 1e-3 ? eps : 1e-3;
    double r = sqrt(a * b);
    return hamaker / (8.0 * sqrt(2.0)) * sqrt(r / (e * e * e * e * e));
}

/* Explicit second-order velocity update, eq 15-16:
 *   v(t) = 2/3 (2 v(t - dt) - v(t - 2 dt)/2 + vdot(t) dt). */
double orc_bdf2(double v_nm1, double v_nm2, double rate) { return (2.0 / 3.0) * (2.0 * v_nm1 - 0.5 * v_nm2 + rate); }

/* ------------------------------------------------------------------------------------- */
/* Interpolation, spreading and surface loads on node fields                              */
/* ------------------------------------------------------------------------------------- */

/* Transfer points are kept on the band of fluid node rows 0 <= y <= ny-1.  The paper does
 * not say how a marker or probe that lies between a wall and the first node row is
 * treated; the reading taken is that it is transferred as if it sat on that row.  (Left
 * where it is, the linear MLS fit extrapolates with weights 1+d and -d on the two rows it
 * sees, and the interpolate-spread loop of the direct forcing has a gain above 2: the
 * coupled step then diverges within a few tens of steps even for a fixed particle.) */
static double fluid_row_y(double y, int ny)
{
    if (y < 0.0) return 0.0;
    if (y > ny - 1.0) return ny - 1.0;
    return y;
}

/* Direct-forcing marker force (reading of the Favier et al. direct forcing the paper
 * cites): F_l = 2 rho_l (U_d - U*_l) where U*_l, rho_l are the MLS interpolants of the
 * node velocity without the IB force and the node density.  The factor 2 undoes the half
 * force shift of eq 6, so the forced velocity at the marker equals U_d. */
int32_t orc_ib_forces(int32_t nx, int32_t ny, const double* rho, const double* ux, const double* uy,
                      int32_t nl, const double* X, const double* Ud, double* F)
{
    int32_t ni[9], nj[9];
    double phi[9], psx[9], psy[9];
    for (int l = 0; l < nl; ++l) {
        int n = orc_mls(nx, ny, X[2 * l], fluid_row_y(X[2 * l + 1], ny), ni, nj, phi, psx, psy);
        if (n < 0) return -1;
        double r = 0.0, sx = 0.0, sy = 0.0;
        for (int k = 0; k < n; ++k) {
            size_t c = (size_t)nj[k] * nx + ni[k];
            r += phi[k] * rho[c];
            sx += phi[k] * ux[c];
            sy += phi[k] * uy[c];
        }
        F[2 * l] = 2.0 * r * (Ud[2 * l] - sx);
        F[2 * l + 1] = 2.0 * r * (Ud[2 * l + 1] - sy);
    }
    return 0;
}

/* Spread: fib(x_k) += phi_k(X_l) S_l F_l for l ascending (the transpose of the MLS
 * interpolation with the marker volume S_l dx).  fib holds two planes [c][j][i] and is
 * accumulated into. */
int32_t orc_spread(int32_t nx, int32_t ny, int32_t nl, const double* X, const double* S, const double* F,
                   double* fib)
{
    int32_t ni[9], nj[9];
    double phi[9], psx[9], psy[9];
    for (int l = 0; l < nl; ++l) {
        int n = orc_mls(nx, ny, X[2 * l], fluid_row_y(X[2 * l + 1], ny), ni, nj, phi, psx, psy);
        if (n < 0) return -1;
        double sfx = S[l] * F[2 * l], sfy = S[l] * F[2 * l + 1];
        for (int k = 0; k < n; ++k) {
            fib[IDX(0, nj[k], ni[k], nx, ny)] += phi[k] * sfx;
            fib[IDX(1, nj[k], ni[k], nx, ny)] += phi[k] * sfy;
        }
    }
    return 0;
}

/* Surface tractions, eq 7-8: for each element, at its probe point P_l (1.2 dx along the
 * outward normal, kept on the fluid rows like every transfer point), p_l = cs^2 (rho(P_l) - 1) and the velocity gradient G = grad u(P_l) by
 * the MLS diffuse derivative; the viscous stress is rho(P_l) nu (G + G^T) and the element
 * load t_l = (-p_l n_l + tau_l . n_l) S_l.  (Eq 8 is printed with the label F_p; it is the
 * viscous part.)  The pressure gauge 1 cancels on a closed surface. */
int32_t orc_tractions(int32_t nx, int32_t ny, double nu, const double* rho, const double* ux,
                      const double* uy, int32_t nl, const double* P, const double* n, const double* S,
                      double* t)
{
    int32_t ni[9], nj[9];
    double phi[9], psx[9], psy[9];
    for (int l = 0; l < nl; ++l) {
        int m = orc_mls(nx, ny, P[2 * l], fluid_row_y(P[2 * l + 1], ny), ni, nj, phi, psx, psy);
        if (m < 0) return -1;
        double r = 0.0, gxx = 0.0, gxy = 0.0, gyx = 0.0, gyy = 0.0;
        for (int k = 0; k < m; ++k) {
            size_t c = (size_t)nj[k] * nx + ni[k];
            r += phi[k] * rho[c];
            gxx += psx[k] * ux[c]; /* d ux / dx */
            gxy += psy[k] * ux[c]; /* d ux / dy */
            gyx += psx[k] * uy[c]; /* d uy / dx */
            gyy += psy[k] * uy[c]; /* d uy / dy */
        }
        double p = CS2 * (r - 1.0);
        double sxx = r * nu * (2.0 * gxx), syy = r * nu * (2.0 * gyy);
        double sxy = r * nu * (gxy + gyx);
        double nx_ = n[2 * l], ny_ = n[2 * l + 1];
        t[2 * l] = (-p * nx_ + sxx * nx_ + sxy * ny_) * S[l];
        t[2 * l + 1] = (-p * ny_ + sxy * nx_ + syy * ny_) * S[l];
    }
    return 0;
}

/* ------------------------------------------------------------------------------------- */
/* The whole time step                                                                    */
/* ------------------------------------------------------------------------------------- */

typedef struct {
    int32_t nx, ny;
    double tau, re;
    uint64_t seed;
    int32_t walls;     /* 1: bounce-back walls (the product's only mode); 0: periodic y (test) */
    int32_t init_rest; /* 0: start from f_eq(1, u_poiseuille(y)); 1: start from f_eq(1, 0) */
    double extra_gx, extra_gy; /* body force added to the Poiseuille drive (test hooks) */
    int32_t has_particle;      /* particle 0 from the fields below */
    int32_t shape;
    double a, b, xc, yc, theta0, rho_p;
    int32_t nl;
    int32_t rho_l_num, rho_l_den;
    double sigma_hat, sigma_star_ratio, y_cr_hat, y_eq_ratio, k_f, k_r0, kbt_hat, hamaker_hat;
    int32_t drive; /* 0: body-force Poiseuille, resting walls; 1: resting bottom wall, top wall
                      moving at u_max, no body force (linear shear) */
} orc_params;

/* One particle: shape and placement, ligands and bond constants (Table 1 groups). */
typedef struct {
    int32_t shape;
    double a, b, xc, yc, theta0, rho_p;
    int32_t nl;
    int32_t rho_l_num, rho_l_den;
    double sigma_hat, sigma_star_ratio, y_cr_hat, y_eq_ratio, k_f, k_r0, kbt_hat, hamaker_hat;
} orc_particle_params;

#define ORC_TRACE_W 20
#define ORC_MAX_PARTICLES 64

typedef struct {
    orc_particle_params q;
    double sigma, sigma_star, y_cr, y_eq, kBT, hamaker, mass, inertia;
    double xc, yc, th, ux_p, uy_p, om;   /* time level n   */
    double xc1, yc1, th1, ux1, uy1, om1; /* time level n-1 */
    double *V, *xi, *nuv, *S, *X, *nrm, *Pp, *Ud, *Fl, *tl, *dd, *fb;
    uint8_t *ligand, *bond, *bond_new;
    double rec[ORC_TRACE_W]; /* record of the last step */
} orc_particle;

typedef struct {
    orc_params p;
    double nu, umax, gx, gy;
    int64_t step;
    int32_t flags;
    double *f, *fn, *fib, *rho, *ux, *uy;
    int32_t np;
    orc_particle* P[ORC_MAX_PARTICLES];
} orc_sim;

/* Lattice-unit constants of a particle from the Table 1 groups (rho_ref = 1, H = ny). */
static void derive_particle(const orc_sim* s, orc_particle* P)
{
    const orc_particle_params* q = &P->q;
    double H = (double)s->p.ny;
    double g = s->nu * s->nu / H; /* rho_ref nu^2 / H */
    P->sigma = q->sigma_hat * g;
    P->sigma_star = q->sigma_star_ratio * P->sigma;
    P->y_cr = q->y_cr_hat * H;
    P->y_eq = q->y_eq_ratio * P->y_cr;
    P->kBT = q->kbt_hat * s->nu * s->nu * H;
    P->hamaker = q->hamaker_hat * s->nu * s->nu * H;
    P->mass = q->rho_p * M_PI * q->a * q->b;
    P->inertia = P->mass * (q->a * q->a + q->b * q->b) / 4.0;
}

/* Lattice-unit constants: nu from tau (below eq 1); Re = H u_max / nu ("Modeling the
 * adhesion dynamics" section) gives u_max, the centre-line speed of the Poiseuille drive
 * (body force 8 nu u_max / H^2) or the speed of the moving top wall of the shear drive. */
static void derive(orc_sim* s)
{
    const orc_params* p = &s->p;
    double H = (double)p->ny;
    s->nu = CS2 * (p->tau - 0.5);
    s->umax = p->re * s->nu / H;
    s->gx = (p->drive == 1 ? 0.0 : 8.0 * s->nu * s->umax / (H * H)) + p->extra_gx;
    s->gy = p->extra_gy;
}

/* Speed of the moving top wall (0 for the resting walls of the Poiseuille drive). */
static double wall_speed(const orc_sim* s) { return s->p.drive == 1 ? s->umax : 0.0; }

static void place_markers(orc_particle* P)
{
    int nl = P->q.nl;
    double c = cos(P->th), sn = sin(P->th);
    for (int l = 0; l < nl; ++l) {
        double bx = P->xi[2 * l], by = P->xi[2 * l + 1];
        P->X[2 * l] = P->xc + c * bx - sn * by;
        P->X[2 * l + 1] = P->yc + sn * bx + c * by;
        double mx = P->nuv[2 * l], my = P->nuv[2 * l + 1];
        P->nrm[2 * l] = c * mx - sn * my;
        P->nrm[2 * l + 1] = sn * mx + c * my;
    }
}

static void free_particle(orc_particle* P)
{
    if (!P) return;
    free(P->V); free(P->xi); free(P->nuv); free(P->S); free(P->X); free(P->nrm); free(P->Pp);
    free(P->Ud); free(P->Fl); free(P->tl); free(P->dd); free(P->fb);
    free(P->ligand); free(P->bond); free(P->bond_new);
    free(P);
}

/* Add a particle at rest at its placement, with no bonds; returns its index (the particle
 * index of its bond draws) or -1. */
int32_t orc_sim_add_particle(orc_sim* s, const orc_particle_params* q)
{
    if (s->np >= ORC_MAX_PARTICLES || s->step != 0 || q->nl < 3) return -1;
    orc_particle* P = (orc_particle*)calloc(1, sizeof(orc_particle));
    P->q = *q;
    if (q->shape == 0) P->q.b = q->a;
    int nl = q->nl;
    P->V = (double*)calloc(2 * nl, sizeof(double));
    P->xi = (double*)calloc(2 * nl, sizeof(double));
    P->nuv = (double*)calloc(2 * nl, sizeof(double));
    P->S = (double*)calloc(nl, sizeof(double));
    P->X = (double*)calloc(2 * nl, sizeof(double));
    P->nrm = (double*)calloc(2 * nl, sizeof(double));
    P->Pp = (double*)calloc(2 * nl, sizeof(double));
    P->Ud = (double*)calloc(2 * nl, sizeof(double));
    P->Fl = (double*)calloc(2 * nl, sizeof(double));
    P->tl = (double*)calloc(2 * nl, sizeof(double));
    P->dd = (double*)calloc(nl, sizeof(double));
    P->fb = (double*)calloc(2 * nl, sizeof(double));
    P->ligand = (uint8_t*)calloc(nl, 1);
    P->bond = (uint8_t*)calloc(nl, 1);
    P->bond_new = (uint8_t*)calloc(nl, 1);
    if (orc_geometry(P->q.shape, P->q.a, P->q.b, nl, P->V, P->xi, P->nuv, P->S) != 0) {
        free_particle(P);
        return -1;
    }
    orc_ligand_flags(nl, q->rho_l_num, q->rho_l_den, P->ligand);
    P->xc = P->xc1 = q->xc;
    P->yc = P->yc1 = q->yc;
    P->th = P->th1 = q->theta0;
    derive_particle(s, P);
    s->P[s->np] = P;
    return s->np++;
}

orc_sim* orc_sim_create(const orc_params* p)
{
    if (p->nx < 4 || p->ny < 4 || !(p->tau > 0.5) || p->drive < 0 || p->drive > 1) return NULL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    s->p = *p;
    derive(s);
    size_t N = (size_t)p->nx * p->ny;
    s->f = (double*)calloc(9 * N, sizeof(double));
    s->fn = (double*)calloc(9 * N, sizeof(double));
    s->fib = (double*)calloc(2 * N, sizeof(double));
    s->rho = (double*)calloc(N, sizeof(double));
    s->ux = (double*)calloc(N, sizeof(double));
    s->uy = (double*)calloc(N, sizeof(double));
    double H = (double)p->ny;
    for (int j = 0; j < p->ny; ++j) {
        /* the developed profile: parabolic (Poiseuille) or linear (shear), walls at -1/2, H - 1/2 */
        double u0 = p->drive == 1 ? s->umax * (j + 0.5) / H : 4.0 * s->umax * (j + 0.5) * (H - 0.5 - j) / (H * H);
        if (p->init_rest) u0 = 0.0;
        double feq[9];
        orc_feq(1.0, u0, 0.0, feq);
        for (int i = 0; i < p->nx; ++i)
            for (int q = 0; q < 9; ++q) s->f[IDX(q, j, i, p->nx, p->ny)] = feq[q];
    }
    if (p->has_particle) {
        orc_particle_params q = {p->shape, p->a, p->b, p->xc, p->yc, p->theta0, p->rho_p, p->nl,
                                 p->rho_l_num, p->rho_l_den, p->sigma_hat, p->sigma_star_ratio,
                                 p->y_cr_hat, p->y_eq_ratio, p->k_f, p->k_r0, p->kbt_hat, p->hamaker_hat};
        if (orc_sim_add_particle(s, &q) != 0) {
            free(s->f); free(s->fn); free(s->fib); free(s->rho); free(s->ux); free(s->uy);
            free(s);
            return NULL;
        }
        if (p->shape == 0) s->p.b = p->a;
    }
    return s;
}

void orc_sim_destroy(orc_sim* s)
{
    if (!s) return;
    free(s->f); free(s->fn); free(s->fib); free(s->rho); free(s->ux); free(s->uy);
    for (int k = 0; k < s->np; ++k) free_particle(s->P[k]);
    free(s);
}

/* Node fields rho and u = (sum f e + F/2) / rho with F = g (+ fib when with_fib). */
static void node_fields(orc_sim* s, int with_fib)
{
    int nx = s->p.nx, ny = s->p.ny;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double f9[9];
            for (int q = 0; q < 9; ++q) f9[q] = s->f[IDX(q, j, i, nx, ny)];
            double Fx = s->gx, Fy = s->gy;
            if (with_fib) {
                Fx += s->fib[IDX(0, j, i, nx, ny)];
                Fy += s->fib[IDX(1, j, i, nx, ny)];
            }
            size_t c = (size_t)j * nx + i;
            orc_moments(f9, Fx, Fy, &s->rho[c], &s->ux[c], &s->uy[c]);
        }
}

/* Loads, bonds and the rigid-body update of particle k (steps 8-12 below), from the forced
 * step-n node fields. */
static void particle_update(orc_sim* s, int k)
{
    const orc_params* p = &s->p;
    orc_particle* P = s->P[k];
    const orc_particle_params* q = &P->q;
    int nx = p->nx, ny = p->ny, nl = q->nl;
    double Fh[3] = {0, 0, 0}, Fb[3] = {0, 0, 0}, Fw = 0.0, gap = 0.0;
    int n_probing = 0;
    for (int l = 0; l < nl; ++l) { /* probe 1.2 dx along the outward normal (below eq 8) */
        P->Pp[2 * l] = P->X[2 * l] + 1.2 * P->nrm[2 * l];
        P->Pp[2 * l + 1] = P->X[2 * l + 1] + 1.2 * P->nrm[2 * l + 1];
    }
    if (orc_tractions(nx, ny, s->nu, s->rho, s->ux, s->uy, nl, P->Pp, P->nrm, P->S, P->tl) != 0) s->flags |= 4;
    for (int l = 0; l < nl; ++l) P->dd[l] = P->X[2 * l + 1] + 0.5;
    int n_bonds = orc_bonds(nl, P->ligand, P->dd, P->bond, P->bond_new, P->y_cr, P->y_eq, P->sigma, P->sigma_star,
                            q->k_f, q->k_r0, P->kBT, p->seed, s->step, (uint32_t)k, &n_probing);
    for (int l = 0; l < nl; ++l) {
        P->bond[l] = P->bond_new[l];
        double mag = P->bond[l] ? P->sigma * (P->dd[l] - P->y_eq) : 0.0; /* eq 9 */
        P->fb[2 * l] = mag * P->nrm[2 * l];
        P->fb[2 * l + 1] = mag * P->nrm[2 * l + 1];
    }
    int32_t wflag = 0;
    Fw = orc_wall_force(P->yc, P->th, q->a, q->b, P->hamaker, &gap, &wflag);
    if (wflag) s->flags |= 2;
    for (int l = 0; l < nl; ++l) {
        double rx = P->X[2 * l] - P->xc, ry = P->X[2 * l + 1] - P->yc;
        Fh[0] += P->tl[2 * l];
        Fh[1] += P->tl[2 * l + 1];
        Fh[2] += rx * P->tl[2 * l + 1] - ry * P->tl[2 * l];
        Fb[0] += P->fb[2 * l];
        Fb[1] += P->fb[2 * l + 1];
        Fb[2] += rx * P->fb[2 * l + 1] - ry * P->fb[2 * l];
    }
    double Fx = Fh[0] + Fb[0], Fy = Fh[1] + Fb[1] + Fw, M = Fh[2] + Fb[2];
    double ux_n = orc_bdf2(P->ux_p, P->ux1, Fx / P->mass);
    double uy_n = orc_bdf2(P->uy_p, P->uy1, Fy / P->mass);
    double om_n = orc_bdf2(P->om, P->om1, M / P->inertia);
    double xc_n = orc_bdf2(P->xc, P->xc1, ux_n);
    double yc_n = orc_bdf2(P->yc, P->yc1, uy_n);
    double th_n = orc_bdf2(P->th, P->th1, om_n);
    if (!isfinite(Fx) || !isfinite(Fy) || !isfinite(M) || !isfinite(ux_n) || !isfinite(uy_n) || !isfinite(om_n))
        s->flags |= 1;
    P->ux1 = P->ux_p; P->uy1 = P->uy_p; P->om1 = P->om;
    P->xc1 = P->xc; P->yc1 = P->yc; P->th1 = P->th;
    P->ux_p = ux_n; P->uy_p = uy_n; P->om = om_n;
    P->xc = xc_n; P->yc = yc_n; P->th = th_n;
    double rec[ORC_TRACE_W] = {(double)s->step, P->xc, P->yc, P->th, P->ux_p, P->uy_p, P->om,
                               Fx, Fy, M, Fh[0], Fh[1], Fh[2], Fb[0], Fb[1], Fb[2], Fw, gap,
                               (double)n_bonds, (double)n_probing};
    memcpy(P->rec, rec, sizeof(rec));
}

/* One time step n -> n+1 in the order:
 *  1 markers of every particle at (X_c^n, theta^n);  2 node moments without the IB force;
 *  3-4 MLS interpolation and direct-forcing marker forces;  5 spread to the lattice,
 *  particles in index order (particles meet only through the fluid);
 *  6-7 collide (eq 1, 4) and stream with the total body force g + fib;
 *  then for each particle: 8 probe loads (eq 7-8) from the forced step-n fields (the spread
 *  force of every particle included);  9 bonds (eq 9-11; the particle's index keys its
 *  draws);  10 wall force (eq 12);  11 totals F, M;  12 rigid-body update (eq 13-16).
 * trace (np x ORC_TRACE_W doubles) receives the records of this step when not NULL. */
static int step_once(orc_sim* s, double* trace)
{
    const orc_params* p = &s->p;
    int nx = p->nx, ny = p->ny;
    size_t N = (size_t)nx * ny;
    memset(s->fib, 0, 2 * N * sizeof(double));
    if (s->np > 0) {
        for (int k = 0; k < s->np; ++k) place_markers(s->P[k]);
        node_fields(s, 0);
        for (int k = 0; k < s->np; ++k) {
            orc_particle* P = s->P[k];
            int nl = P->q.nl;
            for (int l = 0; l < nl; ++l) {
                double rx = P->X[2 * l] - P->xc, ry = P->X[2 * l + 1] - P->yc;
                P->Ud[2 * l] = P->ux_p - P->om * ry;
                P->Ud[2 * l + 1] = P->uy_p + P->om * rx;
            }
            if (orc_ib_forces(nx, ny, s->rho, s->ux, s->uy, nl, P->X, P->Ud, P->Fl) != 0) s->flags |= 4;
            if (orc_spread(nx, ny, nl, P->X, P->S, P->Fl, s->fib) != 0) s->flags |= 4;
        }
    }
    orc_collide_stream_uw(nx, ny, p->walls, wall_speed(s), p->tau, s->gx, s->gy, s->np > 0 ? s->fib : NULL, s->f,
                          s->fn);
    if (s->np > 0) {
        node_fields(s, 1);
        for (int k = 0; k < s->np; ++k) {
            particle_update(s, k);
            if (trace) memcpy(trace + (size_t)k * ORC_TRACE_W, s->P[k]->rec, sizeof(s->P[k]->rec));
        }
    }
    double* t = s->f;
    s->f = s->fn;
    s->fn = t;
    s->step += 1;
    return s->flags;
}

/* nsteps steps; trace (when not NULL) receives particle 0's record of each step. */
int32_t orc_sim_step(orc_sim* s, int64_t nsteps, double* trace)
{
    double* all = s->np > 1 && trace ? (double*)malloc((size_t)s->np * ORC_TRACE_W * sizeof(double)) : NULL;
    for (int64_t n = 0; n < nsteps; ++n) {
        double* t = trace ? (all ? all : trace + n * ORC_TRACE_W) : NULL;
        step_once(s, t);
        if (all) memcpy(trace + n * ORC_TRACE_W, all, ORC_TRACE_W * sizeof(double));
    }
    free(all);
    return s->flags;
}

/* nsteps steps; trace (when not NULL) receives every particle's record: [n][k][ORC_TRACE_W]. */
int32_t orc_sim_step_all(orc_sim* s, int64_t nsteps, double* trace)
{
    for (int64_t n = 0; n < nsteps; ++n)
        step_once(s, trace ? trace + (size_t)n * s->np * ORC_TRACE_W : NULL);
    return s->flags;
}

int32_t orc_sim_num_particles(const orc_sim* s) { return s->np; }

void orc_sim_get_f(const orc_sim* s, double* out) { memcpy(out, s->f, 9 * (size_t)s->p.nx * s->p.ny * sizeof(double)); }
void orc_sim_set_f(orc_sim* s, const double* in) { memcpy(s->f, in, 9 * (size_t)s->p.nx * s->p.ny * sizeof(double)); }
void orc_sim_get_fib(const orc_sim* s, double* out) { memcpy(out, s->fib, 2 * (size_t)s->p.nx * s->p.ny * sizeof(double)); }
int64_t orc_sim_get_step(const orc_sim* s) { return s->step; }
int32_t orc_sim_get_flags(const orc_sim* s) { return s->flags; }

/* Derived lattice-unit parameters: nu, umax, gx, gy, then particle 0's sigma, sigma*, y_cr,
 * y_eq, kBT, H_k, mass, inertia (zeros without a particle). */
void orc_sim_get_derived(const orc_sim* s, double* out)
{
    const orc_particle* P = s->np > 0 ? s->P[0] : NULL;
    double v[12] = {s->nu, s->umax, s->gx, s->gy,
                    P ? P->sigma : 0.0, P ? P->sigma_star : 0.0, P ? P->y_cr : 0.0, P ? P->y_eq : 0.0,
                    P ? P->kBT : 0.0, P ? P->hamaker : 0.0, P ? P->mass : 0.0, P ? P->inertia : 0.0};
    memcpy(out, v, sizeof(v));
}

/* Particle k's state: xc, yc, theta, ux, uy, omega and the same at the previous level. */
void orc_sim_get_particle_k(const orc_sim* s, int32_t k, double* out)
{
    const orc_particle* P = s->P[k];
    double v[12] = {P->xc, P->yc, P->th, P->ux_p, P->uy_p, P->om, P->xc1, P->yc1, P->th1, P->ux1, P->uy1, P->om1};
    memcpy(out, v, sizeof(v));
}

void orc_sim_set_particle_k(orc_sim* s, int32_t k, const double* in)
{
    orc_particle* P = s->P[k];
    P->xc = in[0]; P->yc = in[1]; P->th = in[2]; P->ux_p = in[3]; P->uy_p = in[4]; P->om = in[5];
    P->xc1 = in[6]; P->yc1 = in[7]; P->th1 = in[8]; P->ux1 = in[9]; P->uy1 = in[10]; P->om1 = in[11];
}

void orc_sim_get_bonds_k(const orc_sim* s, int32_t k, uint8_t* bonded, uint8_t* ligand)
{
    memcpy(bonded, s->P[k]->bond, s->P[k]->q.nl);
    memcpy(ligand, s->P[k]->ligand, s->P[k]->q.nl);
}

void orc_sim_set_bonds_k(orc_sim* s, int32_t k, const uint8_t* bonded) { memcpy(s->P[k]->bond, bonded, s->P[k]->q.nl); }

void orc_sim_get_particle(const orc_sim* s, double* out) { orc_sim_get_particle_k(s, 0, out); }
void orc_sim_set_particle(orc_sim* s, const double* in) { orc_sim_set_particle_k(s, 0, in); }
void orc_sim_get_bonds(const orc_sim* s, uint8_t* bonded, uint8_t* ligand) { orc_sim_get_bonds_k(s, 0, bonded, ligand); }
void orc_sim_set_bonds(orc_sim* s, const uint8_t* bonded) { orc_sim_set_bonds_k(s, 0, bonded); }

/* Body-frame geometry (xi, nu, S) and the lab-frame markers / normals of particle 0. */
void orc_sim_get_geometry(const orc_sim* s, double* xi, double* nu, double* S)
{
    const orc_particle* P = s->P[0];
    memcpy(xi, P->xi, 2 * P->q.nl * sizeof(double));
    memcpy(nu, P->nuv, 2 * P->q.nl * sizeof(double));
    memcpy(S, P->S, P->q.nl * sizeof(double));
}

void orc_sim_get_markers_k(orc_sim* s, int32_t k, double* X, double* n)
{
    orc_particle* P = s->P[k];
    place_markers(P);
    memcpy(X, P->X, 2 * P->q.nl * sizeof(double));
    memcpy(n, P->nrm, 2 * P->q.nl * sizeof(double));
}

void orc_sim_get_markers(orc_sim* s, double* X, double* n) { orc_sim_get_markers_k(s, 0, X, n); }

int32_t orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
