// Host-side mesh construction: leaves of the nested 2:1 refinement, face
// connectivity (conforming, periodic, wall, hanging) and the isoparametric
// geometry of every element at its Gauss-Legendre points.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <stdexcept>

#include "internal.hpp"

namespace imx {

// ---------------------------------------------------------------- 1D tables
static void legendre(int n, double x, double& p, double& dp) {
    // P_n and P_n' by the three-term recurrence
    double p0 = 1.0, p1 = x;
    if (n == 0) { p = 1.0; dp = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
    }
    p = p1;
    dp = n * (x * p1 - p0) / (x * x - 1.0);
}

void lagrange(const std::vector<double>& nodes, double t, double* val, double* der) {
    const int n = (int)nodes.size();
    for (int i = 0; i < n; ++i) {
        double v = 1.0;
        for (int m = 0; m < n; ++m)
            if (m != i) v *= (t - nodes[m]) / (nodes[i] - nodes[m]);
        if (val) val[i] = v;
        if (der) {
            double s = 0.0;
            for (int m = 0; m < n; ++m) {
                if (m == i) continue;
                double term = 1.0 / (nodes[i] - nodes[m]);
                for (int l = 0; l < n; ++l)
                    if (l != i && l != m) term *= (t - nodes[l]) / (nodes[i] - nodes[l]);
                s += term;
            }
            der[i] = s;
        }
    }
}

void Basis1D::build(int degree) {
    n = degree + 1;
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    // Gauss-Legendre: Newton on P_n from Chebyshev guesses, mapped to [0, 1]
    for (int k = 0; k < n; ++k) {
        double t = -std::cos(M_PI * (k + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(n, t, p, dp);
            double dt = p / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-17) break;
        }
        double p, dp;
        legendre(n, t, p, dp);
        x[k] = 0.5 * (t + 1.0);
        w[k] = 1.0 / ((1.0 - t * t) * dp * dp);     // 2/((1-t^2)P'^2) halved for [0,1]
    }
    // Gauss-Lobatto: endpoints and the roots of P'_{n-1} (Newton on P'_{n-1})
    gll.assign(n, 0.0);
    gll[0] = 0.0;
    gll[n - 1] = 1.0;
    for (int k = 1; k < n - 1; ++k) {
        double t = -std::cos(M_PI * k / (n - 1));
        for (int it = 0; it < 100; ++it) {
            // f = P'_{m}, f' = P''_{m} = (2 t P'_m - m(m+1) P_m) / (1 - t^2)
            const int m = n - 1;
            double p, dp;
            legendre(m, t, p, dp);
            double d2 = (2.0 * t * dp - m * (m + 1.0) * p) / (1.0 - t * t);
            double dt = dp / d2;
            t -= dt;
            if (std::fabs(dt) < 1e-17) break;
        }
        gll[k] = 0.5 * (t + 1.0);
    }
    D.assign(n * n, 0.0);
    std::vector<double> tmp(n);
    for (int q = 0; q < n; ++q) {
        lagrange(x, x[q], nullptr, tmp.data());
        for (int i = 0; i < n; ++i) D[q * n + i] = tmp[i];
    }
    face.assign(2 * n, 0.0);
    for (int s = 0; s < 2; ++s) {
        lagrange(x, (double)s, tmp.data(), nullptr);
        for (int i = 0; i < n; ++i) face[s * n + i] = tmp[i];
    }
    half.assign(2 * n * n, 0.0);
    for (int hh = 0; hh < 2; ++hh)
        for (int a = 0; a < n; ++a) {
            lagrange(x, 0.5 * (hh + x[a]), tmp.data(), nullptr);
            for (int i = 0; i < n; ++i) half[(hh * n + a) * n + i] = tmp[i];
        }
}

// ---------------------------------------------------------------- surface
static double surface(const imx_mesh_desc& d, double x, double y) {
    double dx = x - d.xc, dy = y - d.yc;
    if (d.periodic_x) dx -= d.Lx * std::nearbyint(dx / d.Lx);
    if (d.periodic_y) dy -= d.Ly * std::nearbyint(dy / d.Ly);
    double r2 = (dx * dx + dy * dy) / (d.a * d.a);
    if (d.terrain == IMX_BELL) return d.h0 / (1.0 + r2);
    if (d.terrain == IMX_GAUSS) return d.h0 * std::exp(-r2);
    return 0.0;
}

static const int TANG[3][2] = {{1, 2}, {0, 2}, {0, 1}};

// Compact metric of terrain-following element e (layout at cm_stride). The
// Gal-Chen map interpolated on the base cell is z = S (1 - zeta / Lz) + zeta,
// with S the surface interpolated on the cell's Gauss-Lobatto points and zeta
// the undeformed height, linear in the reference coordinate (the interpolant of
// a linear function is that function). So dz/dxi_x = sc S_x phi and
// dz/dxi_y = sc S_y phi with phi = 1 - zeta / Lz, and dz/dxi_z = sc h0z (1 - S / Lz)
// does not depend on zeta. Every entry of W cof(J), W det J and n dS is a
// product of these and the affine h_x, h_y; the result is checked against the
// mapped geometry of the element at 1e-12 of its largest entry (false: it
// does not reproduce it).
static bool compact_metric(Mesh& m, int64_t e, const std::vector<double>& hsv, const double h0[3]) {
    const int n = m.n, Nf = m.Nf, Np = m.Np, K = cm_stride(n);
    const int64_t E = m.E;
    const Basis1D& B = m.basis;
    const imx_mesh_desc& d = m.desc;
    const double sc = std::ldexp(1.0, -m.level[e]);
    const int* b = &m.base[3 * e];
    const int* sb = &m.sub[3 * e];
    double* cme = &m.cm[(size_t)e * K];
    auto surf = [&](double ex, double ey, double& S, double& Sx, double& Sy) {
        double lx[8], dx[8], ly[8], dy[8];
        lagrange(B.gll, ex, lx, dx);
        lagrange(B.gll, ey, ly, dy);
        S = Sx = Sy = 0.0;
        for (int a = 0; a < n; ++a)
            for (int bb = 0; bb < n; ++bb) {
                const double v = hsv[a * n + bb];
                S += lx[a] * ly[bb] * v;
                Sx += dx[a] * ly[bb] * v;
                Sy += lx[a] * dy[bb] * v;
            }
    };
    auto j22 = [&](double S) { return h0[2] * (1.0 - S / d.Lz) * sc; };
    auto phi = [&](double xi) { return 1.0 - (b[2] + (sb[2] + xi) * sc) * h0[2] / d.Lz; };
    double S, Sx, Sy;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            surf((sb[0] + B.x[i]) * sc, (sb[1] + B.x[j]) * sc, S, Sx, Sy);
            cme[i + n * j] = j22(S);
            cme[Nf + i + n * j] = Sx * sc;
            cme[2 * Nf + i + n * j] = Sy * sc;
        }
    for (int s = 0; s < 2; ++s)
        for (int a = 0; a < n; ++a) {
            surf((sb[0] + s) * sc, (sb[1] + B.x[a]) * sc, S, Sx, Sy);
            cme[3 * Nf + s * n + a] = j22(S);
            surf((sb[0] + B.x[a]) * sc, (sb[1] + s) * sc, S, Sx, Sy);
            cme[3 * Nf + 2 * n + s * n + a] = j22(S);
        }
    for (int k = 0; k < n; ++k) cme[3 * Nf + 4 * n + k] = phi(B.x[k]);
    cme[3 * Nf + 5 * n] = phi(0.0);
    cme[3 * Nf + 5 * n + 1] = phi(1.0);
    // the entries the kernels form from it, against the mapped geometry
    const double J00 = m.h[3 * e], J11 = m.h[3 * e + 1];
    const int keep[5][2] = {{0, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}};
    double gmax = 0, gdev = 0, wdev = 0, nmax = 0, ndev = 0;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const int node = i + n * (j + n * k), ij = i + n * j;
                const double W = B.w[i] * B.w[j] * B.w[k];
                const double J22 = cme[ij], ph = cme[3 * Nf + 4 * n + k];
                const double J20 = cme[Nf + ij] * ph, J21 = cme[2 * Nf + ij] * ph;
                const double g5[5] = {W * (J11 * J22), W * (J00 * J22), W * (-(J11 * J20)), W * (-(J00 * J21)),
                                      W * (J00 * J11)};
                for (int t = 0; t < 5; ++t) {
                    const double ref = m.G[((size_t)(keep[t][0] * 3 + keep[t][1]) * E + e) * Np + node];
                    gmax = std::max(gmax, std::fabs(ref));
                    gdev = std::max(gdev, std::fabs(g5[t] - ref));
                }
                const double wj = W * (J00 * (J11 * J22)), wref = m.WJ[e * Np + node];
                wdev = std::max(wdev, std::fabs(wj - wref) / wref);
            }
    for (int dd = 0; dd < 3; ++dd)
        for (int side = 0; side < 2; ++side)
            for (int bq = 0; bq < n; ++bq)
                for (int aq = 0; aq < n; ++aq) {
                    const int f = 2 * dd + side, pt = aq + n * bq;
                    const double W2 = B.w[aq] * B.w[bq] * (side ? 1.0 : -1.0);
                    double v[3] = {0, 0, 0};
                    if (dd == 0) {
                        v[0] = W2 * (J11 * cme[3 * Nf + side * n + aq]);
                    } else if (dd == 1) {
                        v[1] = W2 * (J00 * cme[3 * Nf + 2 * n + side * n + aq]);
                    } else {
                        const double ph = cme[3 * Nf + 5 * n + side];
                        v[0] = W2 * (-(J11 * (cme[Nf + pt] * ph)));
                        v[1] = W2 * (-(J00 * (cme[2 * Nf + pt] * ph)));
                        v[2] = W2 * (J00 * J11);
                    }
                    for (int c = 0; c < 3; ++c) {
                        const double ref = m.nS[((e * 6 + f) * 3 + c) * Nf + pt];
                        nmax = std::max(nmax, std::fabs(ref));
                        ndev = std::max(ndev, std::fabs(v[c] - ref));
                    }
                }
    return gdev <= 1e-12 * gmax && ndev <= 1e-12 * nmax && wdev <= 1e-12;
}

imx_status build_mesh(const imx_mesh_desc& d, Mesh& m) {
    if (d.nx < 1 || d.ny < 1 || d.nz < 1 || d.degree < 1 || d.degree > 4 || !(d.Lx > 0) ||
        !(d.Ly > 0) || !(d.Lz > 0) || d.n_ref < 0 || (d.n_ref > 0 && !d.ref_boxes) ||
        (d.terrain != IMX_FLAT && d.terrain != IMX_BELL && d.terrain != IMX_GAUSS) ||
        (d.terrain != IMX_FLAT && !(d.a > 0))) {
        set_error("imx_mesh_create: invalid mesh description");
        return IMX_EINVAL;
    }
    m.desc = d;
    m.boxes.assign(d.ref_boxes, d.ref_boxes + 6 * d.n_ref);
    m.desc.ref_boxes = m.boxes.data();
    m.r = d.degree;
    m.n = d.degree + 1;
    m.Np = m.n * m.n * m.n;
    m.Nf = m.n * m.n;
    m.deformed = d.terrain != IMX_FLAT;
    m.basis.build(d.degree);
    const double h0[3] = {d.Lx / d.nx, d.Ly / d.ny, d.Lz / d.nz};
    const int nb[3] = {d.nx, d.ny, d.nz};

    // ---- leaves, depth first in the documented order
    std::function<void(const int*, int, const int*)> visit = [&](const int* b, int L, const int* s) {
        bool refine = false;
        if (L < d.n_ref) {
            const double* box = &m.boxes[6 * L];
            refine = true;
            for (int c = 0; c < 3; ++c) {
                double lo = (b[c] + s[c] / std::ldexp(1.0, L)) * h0[c];
                double hi = (b[c] + (s[c] + 1) / std::ldexp(1.0, L)) * h0[c];
                if (!(lo < box[2 * c + 1] && box[2 * c] < hi)) refine = false;
            }
        }
        if (refine) {
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx)
                    for (int cz = 0; cz < 2; ++cz) {
                        int cs[3] = {2 * s[0] + cx, 2 * s[1] + cy, 2 * s[2] + cz};
                        visit(b, L + 1, cs);
                    }
        } else {
            m.base.insert(m.base.end(), b, b + 3);
            m.level.push_back(L);
            m.sub.insert(m.sub.end(), s, s + 3);
        }
    };
    for (int by = 0; by < d.ny; ++by)
        for (int bx = 0; bx < d.nx; ++bx)
            for (int bz = 0; bz < d.nz; ++bz) {
                int b[3] = {bx, by, bz}, s[3] = {0, 0, 0};
                visit(b, 0, s);
            }
    const int64_t E = (int64_t)m.level.size();
    m.E = E;
    int Lmax = 0;
    for (int L : m.level) Lmax = std::max(Lmax, L);
    m.Lmax = Lmax;

    // ---- owner grid at the finest level
    const int64_t nf[3] = {(int64_t)d.nx << Lmax, (int64_t)d.ny << Lmax, (int64_t)d.nz << Lmax};
    std::vector<int> owner((size_t)(nf[0] * nf[1] * nf[2]), -1);
    auto oidx = [&](int64_t X, int64_t Y, int64_t Z) { return (size_t)((X * nf[1] + Y) * nf[2] + Z); };
    std::vector<int64_t> org(E * 3), size(E);
    for (int64_t e = 0; e < E; ++e) {
        int64_t sz = (int64_t)1 << (Lmax - m.level[e]);
        size[e] = sz;
        for (int c = 0; c < 3; ++c) org[3 * e + c] = ((int64_t)m.base[3 * e + c] << Lmax) + m.sub[3 * e + c] * sz;
        for (int64_t X = 0; X < sz; ++X)
            for (int64_t Y = 0; Y < sz; ++Y)
                for (int64_t Z = 0; Z < sz; ++Z)
                    owner[oidx(org[3 * e] + X, org[3 * e + 1] + Y, org[3 * e + 2] + Z)] = (int)e;
    }

    // ---- faces
    m.fkind.assign(E * 6, WALL);
    m.fnbr.assign(E * 6, -1);
    m.faux.assign(E * 6, 0);
    std::vector<int> coarse_nb(E * 6 * 4, -1);
    const bool per[3] = {d.periodic_x != 0, d.periodic_y != 0, false};
    for (int64_t e = 0; e < E; ++e) {
        const int64_t* o = &org[3 * e];
        const int64_t s = size[e];
        const int L = m.level[e];
        for (int dd = 0; dd < 3; ++dd)
            for (int side = 0; side < 2; ++side) {
                const int f = 2 * dd + side;
                int64_t P[3] = {o[0], o[1], o[2]};
                P[dd] = side ? o[dd] + s : o[dd] - 1;
                if (P[dd] < 0 || P[dd] >= nf[dd]) {
                    if (!per[dd]) continue;  // wall
                    P[dd] = (P[dd] + nf[dd]) % nf[dd];
                }
                int nbe = owner[oidx(P[0], P[1], P[2])];
                int Lnb = m.level[nbe];
                const int t1 = TANG[dd][0], t2 = TANG[dd][1];
                if (Lnb == L) {
                    m.fkind[6 * e + f] = CONF;
                    m.fnbr[6 * e + f] = nbe;
                } else if (Lnb == L - 1) {
                    m.fkind[6 * e + f] = FINE;
                    m.fnbr[6 * e + f] = nbe;
                    int h1 = (int)((o[t1] - org[3 * nbe + t1]) / s);
                    int h2 = (int)((o[t2] - org[3 * nbe + t2]) / s);
                    m.faux[6 * e + f] = h1 + 2 * h2;
                } else if (Lnb == L + 1) {
                    m.fkind[6 * e + f] = COARSE;
                    for (int h2 = 0; h2 < 2; ++h2)
                        for (int h1 = 0; h1 < 2; ++h1) {
                            int64_t Q[3] = {P[0], P[1], P[2]};
                            Q[t1] = o[t1] + h1 * (s / 2);
                            Q[t2] = o[t2] + h2 * (s / 2);
                            int nq = owner[oidx(Q[0], Q[1], Q[2])];
                            if (m.level[nq] != L + 1) {
                                set_error("imx_mesh_create: refinement is not 2:1 balanced");
                                return IMX_EINVAL;
                            }
                            coarse_nb[(6 * e + f) * 4 + h1 + 2 * h2] = nq;
                        }
                } else {
                    set_error("imx_mesh_create: refinement is not 2:1 balanced");
                    return IMX_EINVAL;
                }
            }
    }
    // hanging indices: coarse faces in element/face order
    std::vector<int> hidx(E * 6, -1);
    m.nh = 0;
    for (int64_t ef = 0; ef < E * 6; ++ef)
        if (m.fkind[ef] == COARSE) {
            hidx[ef] = (int)m.nh;
            m.fnbr[ef] = (int)m.nh;
            for (int h = 0; h < 4; ++h) m.hang.push_back(coarse_nb[ef * 4 + h]);
            ++m.nh;
        }
    for (int64_t e = 0; e < E; ++e)
        for (int f = 0; f < 6; ++f)
            if (m.fkind[6 * e + f] == FINE) {
                int c = m.fnbr[6 * e + f];
                int fc = f ^ 1;
                m.faux[6 * e + f] |= hidx[6 * c + fc] << 2;
            }

    // ---- geometry
    const int n = m.n, Np = m.Np, Nf = m.Nf;
    const Basis1D& B = m.basis;
    m.h.assign(E * 3, 0.0);
    m.WJ.assign(E * Np, 0.0);
    m.xyz.assign(3 * E * Np, 0.0);
    if (m.deformed) {
        m.G.assign(9 * E * Np, 0.0);
        m.nS.assign(E * 6 * 3 * Nf, 0.0);
        m.cm.assign((size_t)E * cm_stride(n), 0.0);
    }
    bool inverted = false, cm_bad = false;
#pragma omp parallel for schedule(static) reduction(|| : inverted, cm_bad)
    for (int64_t e = 0; e < E; ++e) {
        const int L = m.level[e];
        const double sc = std::ldexp(1.0, -L);
        const int* b = &m.base[3 * e];
        const int* sb = &m.sub[3 * e];
        for (int c = 0; c < 3; ++c) m.h[3 * e + c] = h0[c] * sc;
        // Gal-Chen heights at the Gauss-Lobatto points of the base cell
        std::vector<double> zg, hsv;
        if (m.deformed) {
            zg.assign(n * n * n, 0.0);
            hsv.assign(n * n, 0.0);
            for (int a = 0; a < n; ++a)
                for (int bb = 0; bb < n; ++bb) {
                    double xa = (b[0] + B.gll[a]) * h0[0], yb = (b[1] + B.gll[bb]) * h0[1];
                    double hs = surface(d, xa, yb);
                    hsv[a * n + bb] = hs;
                    for (int c = 0; c < n; ++c) {
                        double zeta = (b[2] + B.gll[c]) * h0[2];
                        zg[(a * n + bb) * n + c] = hs + zeta * (d.Lz - hs) / d.Lz;
                    }
                }
        }
        // map and Jacobian at reference point xi
        auto map = [&](const double xi[3], double X[3], double J[3][3]) {
            double eta[3];
            for (int c = 0; c < 3; ++c) eta[c] = (sb[c] + xi[c]) * sc;
            X[0] = (b[0] + eta[0]) * h0[0];
            X[1] = (b[1] + eta[1]) * h0[1];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) J[r][c] = 0.0;
            J[0][0] = h0[0] * sc;
            J[1][1] = h0[1] * sc;
            if (!m.deformed) {
                X[2] = (b[2] + eta[2]) * h0[2];
                J[2][2] = h0[2] * sc;
                return;
            }
            double lv[3][8], ld[3][8];
            for (int c = 0; c < 3; ++c) lagrange(B.gll, eta[c], lv[c], ld[c]);
            double z = 0, z0 = 0, z1 = 0, z2 = 0;
            for (int a = 0; a < n; ++a)
                for (int bb = 0; bb < n; ++bb) {
                    double sv = 0, sd = 0;
                    for (int c = 0; c < n; ++c) {
                        double v = zg[(a * n + bb) * n + c];
                        sv += v * lv[2][c];
                        sd += v * ld[2][c];
                    }
                    z += lv[0][a] * lv[1][bb] * sv;
                    z0 += ld[0][a] * lv[1][bb] * sv;
                    z1 += lv[0][a] * ld[1][bb] * sv;
                    z2 += lv[0][a] * lv[1][bb] * sd;
                }
            X[2] = z;
            J[2][0] = z0 * sc;
            J[2][1] = z1 * sc;
            J[2][2] = z2 * sc;
        };
        auto cofactor = [](const double J[3][3], double C[3][3], double& det) {
            // C[d][c] = det(J) * (J^{-1})[d][c]  (adjugate)
            C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
            C[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
            C[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
            C[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
            C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
            C[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
            C[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
            C[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
            C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            det = J[0][0] * C[0][0] + J[0][1] * C[1][0] + J[0][2] * C[2][0];
        };
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    const int node = i + n * (j + n * k);
                    const double xi[3] = {B.x[i], B.x[j], B.x[k]};
                    double X[3], J[3][3], C[3][3], det;
                    map(xi, X, J);
                    cofactor(J, C, det);
                    if (!(det > 0)) inverted = true;
                    const double W = B.w[i] * B.w[j] * B.w[k];
                    m.WJ[e * Np + node] = W * det;
                    for (int c = 0; c < 3; ++c) m.xyz[(c * E + e) * Np + node] = X[c];
                    if (m.deformed)
                        for (int dd = 0; dd < 3; ++dd)
                            for (int c = 0; c < 3; ++c)
                                m.G[((size_t)(dd * 3 + c) * E + e) * Np + node] = W * C[dd][c];
                }
        if (m.deformed)
            for (int dd = 0; dd < 3; ++dd)
                for (int side = 0; side < 2; ++side)
                    for (int bq = 0; bq < n; ++bq)
                        for (int aq = 0; aq < n; ++aq) {
                            double xi[3];
                            xi[dd] = side;
                            xi[TANG[dd][0]] = B.x[aq];
                            xi[TANG[dd][1]] = B.x[bq];
                            double X[3], J[3][3], C[3][3], det;
                            map(xi, X, J);
                            cofactor(J, C, det);
                            const double W2 = B.w[aq] * B.w[bq] * (side ? 1.0 : -1.0);
                            const int f = 2 * dd + side, pt = aq + n * bq;
                            for (int c = 0; c < 3; ++c)
                                m.nS[((e * 6 + f) * 3 + c) * Nf + pt] = W2 * C[dd][c];
                        }
        if (m.deformed && !compact_metric(m, e, hsv, h0)) cm_bad = true;
    }
    if (inverted) {
        set_error("imx_mesh_create: inverted element (non-positive Jacobian)");
        return IMX_EINVAL;
    }
    if (cm_bad) {
        set_error("imx_mesh_create: the compact terrain metric does not reproduce the mapped geometry");
        return IMX_EINVAL;
    }
    return IMX_OK;
}

}  // namespace imx
