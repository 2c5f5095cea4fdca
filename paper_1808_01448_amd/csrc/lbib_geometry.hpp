// lbib_geometry.hpp -- host construction of the particle surface elements.
#pragma once

#include <vector>

namespace lbib {

struct Surface {
    std::vector<double> xi;  // [nl][2] element centroids (body frame)
    std::vector<double> nu;  // [nl][2] outward unit normals (body frame)
    std::vector<double> S;   // [nl] element lengths
    double perimeter = 0.0;  // polygon perimeter
};

// shape 0: circle of radius a; shape 1: ellipse with semi-axis a along body y, b along x.
bool build_surface(int shape, double a, double b, int nl, Surface& out);

// Perimeter of the smooth ellipse.
double ellipse_perimeter(double a, double b);

}  // namespace lbib
