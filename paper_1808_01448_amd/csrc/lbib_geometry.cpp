// lbib_geometry.cpp -- FP64 host construction of the particle surface (section "Pressure
// and viscous stresses": nl straight elements with centroid, outward normal and length).
//
// Vertices sit at equal arc length along the ellipse x = b sin t, y = -a cos t (semi-axis a
// along the body y axis), starting at t = 0 and running counter-clockwise.  The arc length
// is computed from the Fourier cosine series of the speed |dx/dt| = sqrt(b^2 cos^2 t +
// a^2 sin^2 t), an even pi-periodic analytic function whose coefficients decay
// geometrically; the trapezoid rule gives them to round-off, and integrating the series
// term by term gives s(t) in closed form.  Newton's method then places each vertex.
#include <cmath>
#include <vector>

#include "lbib_geometry.hpp"

namespace lbib {

namespace {

struct ArcSeries {
    double c0 = 0.0;
    std::vector<double> c;  // c[m-1] multiplies cos(2 m t)
    double a = 0.0, b = 0.0;

    double speed(double t) const
    {
        const double ct = std::cos(t), st = std::sin(t);
        return std::sqrt(b * b * ct * ct + a * a * st * st);
    }
    double arc(double t) const
    {
        double s = c0 * t;
        for (size_t m = 1; m <= c.size(); ++m) s += c[m - 1] * std::sin(2.0 * m * t) / (2.0 * m);
        return s;
    }
};

ArcSeries make_series(double a, double b)
{
    ArcSeries S;
    S.a = a;
    S.b = b;
    const int N = 4096;  // samples over one period [0, pi)
    std::vector<double> v(N);
    for (int k = 0; k < N; ++k) v[k] = S.speed(M_PI * k / N);
    double s0 = 0.0;
    for (int k = 0; k < N; ++k) s0 += v[k];
    S.c0 = s0 / N;
    const double scale = std::fabs(S.c0);
    // the coefficients fall geometrically, as ((a - b) / (a + b))^m; below ~1e-14 of the mean
    // they are the trapezoid sums' round-off, so the series stops there
    for (int m = 1; m < N / 2; ++m) {
        double cm = 0.0;
        for (int k = 0; k < N; ++k) cm += v[k] * std::cos(2.0 * m * M_PI * k / N);
        cm *= 2.0 / N;
        if (m > 8 && std::fabs(cm) < 1e-14 * scale) break;
        S.c.push_back(cm);
    }
    return S;
}

}  // namespace

double ellipse_perimeter(double a, double b)
{
    // the series has mean c0 over [0, 2 pi): the perimeter is 2 pi c0
    return 2.0 * M_PI * make_series(a, b).c0;
}

bool build_surface(int shape, double a, double b, int nl, Surface& out)
{
    if (nl < 3 || !(a > 0.0)) return false;
    if (shape == 0) b = a;
    if (!(b > 0.0)) return false;
    std::vector<double> vx(nl), vy(nl);
    if (shape == 0) {
        for (int k = 0; k < nl; ++k) {
            const double t = 2.0 * M_PI * k / nl;
            vx[k] = a * std::sin(t);
            vy[k] = -a * std::cos(t);
        }
    } else {
        const ArcSeries S = make_series(a, b);
        const double P = 2.0 * M_PI * S.c0;
        vx[0] = 0.0;
        vy[0] = -a;
        for (int k = 1; k < nl; ++k) {
            const double target = P * k / nl;
            double t = 2.0 * M_PI * k / nl;
            for (int it = 0; it < 60; ++it) {  // quadratic convergence: a few steps reach round-off
                const double dt = (S.arc(t) - target) / S.speed(t);
                t -= dt;
                if (std::fabs(dt) < 1e-15 * (1.0 + std::fabs(t))) break;
            }
            vx[k] = b * std::sin(t);
            vy[k] = -a * std::cos(t);
        }
    }
    out.xi.assign(2 * nl, 0.0);
    out.nu.assign(2 * nl, 0.0);
    out.S.assign(nl, 0.0);
    double perim = 0.0;
    for (int l = 0; l < nl; ++l) {
        const int m = (l + 1) % nl;
        const double tx = vx[m] - vx[l], ty = vy[m] - vy[l];
        const double len = std::sqrt(tx * tx + ty * ty);
        out.S[l] = len;
        out.xi[2 * l] = 0.5 * (vx[m] + vx[l]);
        out.xi[2 * l + 1] = 0.5 * (vy[m] + vy[l]);
        out.nu[2 * l] = ty / len;  // right of the travel direction = outward (counter-clockwise)
        out.nu[2 * l + 1] = -tx / len;
        perim += len;
    }
    out.perimeter = perim;
    return true;
}

}  // namespace lbib
