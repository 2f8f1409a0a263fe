// Internal declarations of the IMEX-DG library (host side).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/imexdg.h"

namespace imx {

enum FaceKind : int { WALL = 0, CONF = 1, FINE = 2, COARSE = 3 };

void set_error(const std::string& msg);
// Text of the last error raised on the calling thread and a counter that every
// set_error advances, so that an entry point can tell whether it raised one.
const std::string& thread_error();
uint64_t error_generation();
// Placed at the top of an entry point that acts on an object: when the call
// raises an error, the object keeps a copy (its own last error, independent
// of other objects and threads).
struct ErrScope {
    std::string* dst;
    uint64_t gen;
    explicit ErrScope(std::string* d) : dst(d), gen(error_generation()) {}
    ~ErrScope() {
        if (dst && error_generation() != gen) *dst = thread_error();
    }
};

// 1D tables of the nodal Gauss-Legendre basis of degree r (n = r + 1 points)
// on the reference interval [0, 1].
struct Basis1D {
    int n = 0;
    std::vector<double> x, w;       // GL points and weights
    std::vector<double> D;          // D[q*n + i] = l_i'(x_q)
    std::vector<double> face;       // face[s*n + i] = l_i(s)
    std::vector<double> half;       // half[(h*n + a)*n + i] = l_i((h + x_a)/2)
    std::vector<double> gll;        // Gauss-Lobatto points (geometry support points)
    void build(int degree);
};

// Lagrange polynomials of `nodes` (and their derivatives) at t.
void lagrange(const std::vector<double>& nodes, double t, double* val, double* der);

struct Mesh {
    imx_mesh_desc desc{};
    std::vector<double> boxes;
    int r = 0, n = 0, Np = 0, Nf = 0;
    int64_t E = 0;
    int Lmax = 0;
    bool deformed = false;
    Basis1D basis;
    std::vector<int> base, level, sub;       // [E*3], [E], [E*3]
    // faces: kind, neighbour (CONF/FINE: element, COARSE: hanging index), aux
    // (FINE: subface | coarse hanging index << 2)
    std::vector<int> fkind, fnbr, faux;      // [E*6]
    std::vector<int> hang;                   // [nh*4] fine neighbours of coarse faces
    int64_t nh = 0;
    // geometry
    std::vector<double> h;                   // [E*3] element sizes (affine part)
    std::vector<double> WJ;                  // [E*Np] quadrature weight * det J
    std::vector<double> G;                   // [9][E][Np] W detJ dxi_d/dx_c, deformed only
    std::vector<double> nS;                  // [E][6][3][Nf] W2 * outward area vector, deformed only
    std::vector<double> xyz;                 // [3][E][Np]
    // terrain-following elements, compact form of the metric: J22 = dz/dxi_z at
    // the Gauss points of the element's (x, y) plane, J20 and J21 there divided
    // by phi = 1 - zeta / Lz, J22 on the x- and y-faces, and phi at the node
    // levels and the two z-faces; per element cm_stride(n) values (deformed only)
    std::vector<double> cm;
};

// entries per element of Mesh::cm: [NF] J22, [NF] J20 / phi, [NF] J21 / phi,
// [2n] J22 on the x-faces (side s, y index a: s n + a), [2n] J22 on the
// y-faces (side s, x index a), [n] phi at the node levels, [2] phi at z = 0, 1
constexpr int cm_stride(int n) { return 3 * n * n + 5 * n + 2; }

imx_status build_mesh(const imx_mesh_desc& d, Mesh& m);

}  // namespace imx

struct imx_mesh {
    imx::Mesh m;
};
