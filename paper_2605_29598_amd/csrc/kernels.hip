// HIP kernels (gfx950) of the rotating IMEX-DG hot path.
//
// Element kernels: a workgroup holds EPB elements with one lane per node; the
// nodal basis sits at the Gauss-Legendre points, so volume terms are
// pointwise plus one 1D derivative contraction per direction (staged in LDS)
// and face traces are one contraction along the face normal. Faces are
// handled element by element: conforming and periodic neighbours are read
// from global memory, slip walls use the mirror state, and a face between
// two refinement levels is integrated on the four fine subfaces (the coarse
// trace is interpolated onto them, and the coarse side integrates with the
// transposed interpolation). Both sides of a face evaluate the numerical flux
// from the same inputs with the same arithmetic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "kernels.hpp"

namespace imx {

// ------------------------------------------------------------------ tables
HostTab make_tab(const Basis1D& b) {
    HostTab t{};
    t.n = b.n;
    for (int i = 0; i < b.n * b.n; ++i) t.D[i] = b.D[i];
    for (int i = 0; i < 2 * b.n; ++i) t.f[i] = b.face[i];
    for (int i = 0; i < 2 * b.n * b.n; ++i) t.H[i] = b.half[i];
    for (int i = 0; i < b.n; ++i) t.w[i] = b.w[i];
    return t;
}

template <int N, typename R>
struct Tab {
    R D[N][N];      // D[q][i] = l_i'(x_q)
    R f[2][N];      // f[s][i] = l_i(s)
    R H[2][N][N];   // H[h][a][i] = l_i((h + x_a)/2)
    R w[N];
    R W2[N * N];        // w_a w_b at face point a + N b
    R W3[N * N * N];    // w_i w_j w_k at node i + N (j + N k)
    R iW3[N * N * N];   // 1 / W3
};

template <int N, typename R>
static Tab<N, R> to_tab(const HostTab& h) {
    Tab<N, R> t;
    for (int q = 0; q < N; ++q)
        for (int i = 0; i < N; ++i) t.D[q][i] = (R)h.D[q * N + i];
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < N; ++i) t.f[s][i] = (R)h.f[s * N + i];
    for (int hh = 0; hh < 2; ++hh)
        for (int a = 0; a < N; ++a)
            for (int i = 0; i < N; ++i) t.H[hh][a][i] = (R)h.H[(hh * N + a) * N + i];
    for (int i = 0; i < N; ++i) t.w[i] = (R)h.w[i];
    for (int b = 0; b < N; ++b)
        for (int a = 0; a < N; ++a) t.W2[a + N * b] = (R)(h.w[a] * h.w[b]);
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                const double W = h.w[i] * h.w[j] * h.w[k];   // the same product as the host's W detJ
                t.W3[i + N * (j + N * k)] = (R)W;
                t.iW3[i + N * (j + N * k)] = (R)(1.0 / W);
            }
    return t;
}

// the basis tables are indexed per lane, so every block keeps a copy in LDS
// (visible after the block's first barrier)
template <int N, typename R>
__device__ __forceinline__ void load_tab(const Tab<N, R>* __restrict__ src, Tab<N, R>* dst) {
    constexpr int NW = (int)(sizeof(Tab<N, R>) / sizeof(R));
    const R* a = (const R*)src;
    R* b = (R*)dst;
    for (int i = threadIdx.x; i < NW; i += blockDim.x) b[i] = a[i];
}

size_t fofs_count(int n) {
    const int NP = n * n * n, NF = n * n, NR = (6 * NF + NP - 1) / NP;
    return (size_t)NR * NP;
}

void fill_fofs(int n, uint64_t* out) {
    const int NP = n * n * n, NF = n * n, NR = (6 * NF + NP - 1) / NP;
    for (int r = 0; r < NR; ++r)
        for (int node = 0; node < NP; ++node) {
            const int it = node + r * NP;
            uint64_t w = 0;
            if (it < 6 * NF) {
                const int f = it / NF, pt = it % NF, d = f >> 1, a = pt % n, b = pt / n;
                for (int m = 0; m < n; ++m) {
                    const int nd = d == 0 ? m + n * (a + n * b) : (d == 1 ? a + n * (m + n * b) : a + n * (b + n * m));
                    w |= (uint64_t)nd << (8 * m);
                }
                w |= (uint64_t)f << 40;
                w |= (uint64_t)pt << 48;
            } else {
                w |= (uint64_t)6 << 40;
            }
            out[r * NP + node] = w;
        }
}

size_t tab_bytes(int n, int f32) {
    switch (n) {
        case 2: return f32 ? sizeof(Tab<2, float>) : sizeof(Tab<2, double>);
        case 3: return f32 ? sizeof(Tab<3, float>) : sizeof(Tab<3, double>);
        case 4: return f32 ? sizeof(Tab<4, float>) : sizeof(Tab<4, double>);
        default: return f32 ? sizeof(Tab<5, float>) : sizeof(Tab<5, double>);
    }
}

template <int N, typename R>
static void fill_n(const HostTab& h, void* out) {
    Tab<N, R> t = to_tab<N, R>(h);
    std::memcpy(out, &t, sizeof(t));
}

void fill_tab(const HostTab& h, int f32, void* out) {
    switch (h.n) {
        case 2: f32 ? fill_n<2, float>(h, out) : fill_n<2, double>(h, out); break;
        case 3: f32 ? fill_n<3, float>(h, out) : fill_n<3, double>(h, out); break;
        case 4: f32 ? fill_n<4, float>(h, out) : fill_n<4, double>(h, out); break;
        default: f32 ? fill_n<5, float>(h, out) : fill_n<5, double>(h, out); break;
    }
}

template <typename R>
struct Geom {
    int64_t E;
    int deformed;
    const int* kind;
    const int* nbr;
    const int* aux;
    const int* hang;
    const double* h;
    const double* hinv;   // 1 / h, per element and direction
    const R* WJ;
    const R* G;     // terrain-following meshes: W cof(J) entries (0,0), (1,1), (2,0), (2,1), (2,2) as [5][E][Np]
    const R* nS;    // terrain-following meshes: n dS as [E][10][Nf] (x, y faces: normal component; z faces: 3)
    const double* eg;     // affine elements: h[3], 1/h[3], det J, 1/det J (8 per element)
    const R* iWJ;         // 1 / WJ (deformed meshes)
    const uint64_t* fofs; // face-point words per (round, lane), see fo_node
    int gnx, gny, gnz, gpx, gpy;   // unrefined box meshes: base grid and periodicity
    const R* cm;          // compact terrain metric [E][cm_stride(N)] or null
};

template <typename R>
static Geom<R> geom(const DevMesh& m);
template <>
Geom<double> geom<double>(const DevMesh& m) {
    return {m.E, m.deformed, m.kind, m.nbr, m.aux, m.hang, m.h, m.hinv, m.WJ, m.G, m.nS, m.eg, m.iWJ, m.fofs,
            m.gnx, m.gny, m.gnz, m.gpx, m.gpy, m.cm};
}
template <>
Geom<float> geom<float>(const DevMesh& m) {
    return {m.E, m.deformed, m.kind, m.nbr, m.aux, m.hang, m.h, m.hinv, m.WJf, m.Gf, m.nSf, m.eg, m.iWJf, m.fofs,
            m.gnx, m.gny, m.gnz, m.gpx, m.gpy, m.cmf};
}

constexpr int epb_of(int N) { return N == 2 ? 16 : (N == 3 ? 9 : (N == 4 ? 4 : 2)); }
constexpr int threads_of(int N) { return ((epb_of(N) * N * N * N + 63) / 64) * 64; }
// elements per workgroup of the specialised Krylov-loop passes
constexpr int epb_mv(int N) { return epb_of(N); }
constexpr int threads_mv(int N) { return ((epb_mv(N) * N * N * N + 63) / 64) * 64; }

// Element slot of a lane within its workgroup. With Np = 64 one wavefront
// holds exactly one element: the slot is then taken from the first lane, which
// tells the compiler that it is wave-uniform, so per-element values (index,
// neighbour lists, edge lengths) live in scalar registers.
template <int NP>
__device__ __forceinline__ int elem_slot(int tid) {
    if constexpr (NP == 64) return __builtin_amdgcn_readfirstlane(tid >> 6);
    else return tid / NP;
}

// Consecutive workgroups are dispatched round-robin over the 8 XCDs; give
// every XCD a contiguous run of logical blocks so that neighbouring elements
// meet in the same L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t G) {
    const int64_t q = G >> 3, r = G & 7, x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

// Face points of the all-faces kernels: lane `node` of an element handles the
// points it = node + r NP (r < NR) of the element's 6 (r+1)^2 face points.
// Per (r, node) a host-built 64-bit word holds the offsets within the element
// of the N nodes along the face normal through that point (bytes 0..N-1), the
// face (byte 5; 6 when the lane has no point in round r) and the point (byte 6).
__device__ __forceinline__ int fo_node(uint64_t w, int m) { return (int)((w >> (8 * m)) & 0xff); }
__device__ __forceinline__ int fo_face(uint64_t w) { return (int)((w >> 40) & 0xff); }
__device__ __forceinline__ int fo_point(uint64_t w) { return (int)((w >> 48) & 0xff); }

// Neighbour across face f of element e of an unrefined box mesh (elements
// numbered bz + nz (bx + nx by)): kind CONF (also across a periodic seam) or
// WALL, computed instead of read from the face tables.
template <typename R>
__device__ __forceinline__ void grid_nbr(const Geom<R>& g, int e, int f, int& kind, int& nb) {
    // element indices are non-negative: unsigned division needs no sign handling
    const unsigned nz = (unsigned)g.gnz, nx = (unsigned)g.gnx, t = (unsigned)e / nz, u = t / nx;
    const int bz = (int)((unsigned)e - t * nz), bx = (int)(t - u * nx), by = (int)u;
    const int d = f >> 1, step = (f & 1) ? 1 : -1;
    int c[3] = {bx, by, bz};
    const int n[3] = {g.gnx, g.gny, g.gnz}, per[3] = {g.gpx, g.gpy, 0};
    int v = c[d] + step;
    bool wall = false;
    if (v < 0 || v >= n[d]) {
        if (per[d]) v = v < 0 ? v + n[d] : v - n[d];
        else wall = true;
    }
    c[d] = v;
    kind = wall ? WALL : CONF;
    nb = wall ? e : c[2] + g.gnz * (c[0] + g.gnx * c[1]);
}

template <int N>
__device__ __forceinline__ int node_of(int d, int m, int a, int b) {
    return d == 0 ? m + N * (a + N * b) : (d == 1 ? a + N * (m + N * b) : a + N * (b + N * m));
}

// The face points a lane handles in the all-faces kernels: points
// it = node + r NP (r < NR) of the element's 6 (r+1)^2 face points. With ST
// (unrefined box meshes) face, point and the node offsets along the normal
// are computed from `it`; otherwise they come from the host-built words.
template <int N, bool ST>
struct LanePoints {
    static constexpr int NP = N * N * N, NF = N * N, NR = (6 * NF + NP - 1) / NP;
    uint64_t fo[ST ? 1 : NR];
    int node;
    __device__ __forceinline__ void init(const uint64_t* __restrict__ fofs, int nd) {
        node = nd;
        if constexpr (!ST) {
#pragma unroll
            for (int r = 0; r < NR; ++r) fo[r] = fofs[r * NP + nd];
        }
    }
    // face of point r (6: the lane has no point in round r)
    __device__ __forceinline__ int face(int r) const {
        if constexpr (ST) {
            const int it = node + r * NP;
            return it < 6 * NF ? it / NF : 6;
        } else {
            return fo_face(fo[r]);
        }
    }
    __device__ __forceinline__ int point(int r) const {
        if constexpr (ST) {
            const int it = node + r * NP;
            return it < 6 * NF ? it % NF : 0;
        } else {
            return fo_point(fo[r]);
        }
    }
    // node offset within the element of the m-th node along the normal through point r
    __device__ __forceinline__ int off(int r, int m) const {
        if constexpr (ST) {
            const int pt = point(r);
            return node_of<N>(face(r) >> 1, m, pt % N, pt / N);
        } else {
            return fo_node(fo[r], m);
        }
    }
};

template <int N>
__device__ __forceinline__ void split_node(int d, int node, int& m, int& pt) {
    const int i = node % N, j = (node / N) % N, k = node / (N * N);
    if (d == 0) { m = i; pt = j + N * k; }
    else if (d == 1) { m = j; pt = i + N * k; }
    else { m = k; pt = i + N * j; }
}

// products and sums with one rounding each (no contraction into fma)
__device__ __forceinline__ double mul_rn(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ float mul_rn(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ double add_rn(double a, double b) { return __dadd_rn(a, b); }
__device__ __forceinline__ float add_rn(float a, float b) { return __fadd_rn(a, b); }
__device__ __forceinline__ double fma_rn(double a, double b, double c) { return __fma_rn(a, b, c); }
__device__ __forceinline__ float fma_rn(float a, float b, float c) { return __fmaf_rn(a, b, c); }
__device__ __forceinline__ double div_rn(double a, double b) { return __ddiv_rn(a, b); }
__device__ __forceinline__ float div_rn(float a, float b) { return __fdiv_rn(a, b); }

// (rho, u, p) of a node from its conserved (rho, m, E). Face values are
// traces of these primitives; each operation is rounded on its own, so the
// lane that stages its own node and a lane that gathers it as a neighbour
// value get the same bits (both sides of a face then trace the same values).
template <typename R>
__device__ __forceinline__ void prim_of(const R* c, R* P, R gm1) {
    const R r = c[0], ir = div_rn((R)1, r);
    const R u0 = mul_rn(c[1], ir), u1 = mul_rn(c[2], ir), u2 = mul_rn(c[3], ir);
    const R kin = mul_rn((R)0.5, add_rn(add_rn(mul_rn(u0, u0), mul_rn(u1, u1)), mul_rn(u2, u2)));
    P[0] = r;
    P[1] = u0;
    P[2] = u1;
    P[3] = u2;
    P[4] = mul_rn(gm1, add_rn(c[4], -mul_rn(r, kin)));
}

// Trace of a Q_r field along the normal: sum over m (in order) of
// l_m(s) v_m as one product and a chain of fused multiply-adds. Every trace
// of the library, whether its values come from LDS, registers or global
// memory, is formed by this chain, so both sides of a face see the same
// bits.
template <int N, typename R>
__device__ __forceinline__ R trace_chain(const R* fv, const R* v) {
    R acc = mul_rn(fv[0], v[0]);
#pragma unroll
    for (int m = 1; m < N; ++m) acc = fma_rn(fv[m], v[m], acc);
    return acc;
}

// value of a Q_r field (nodal array f of one element) at face point pt
template <int N, typename R, typename P>
__device__ __forceinline__ R face_value(const P* f, const R* fv, int d, int pt) {
    const int a = pt % N, b = pt / N;
    R v[N];
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = (R)f[node_of<N>(d, m, a, b)];
    return trace_chain<N, R>(fv, v);
}

// traces of (rho, u, p) of one element (conserved fields at q + t * fs + base)
// at face point pt: each node along the normal converted by prim_of, then the
// chain of trace_chain per field
template <int N, typename R>
__device__ __forceinline__ void face_value_prim(const R* q, size_t fs, size_t base, const R* fv, int d, int pt,
                                                R gm1, R* P) {
    const int a = pt % N, b = pt / N;
    R acc[5];
#pragma unroll
    for (int m = 0; m < N; ++m) {
        const size_t nd = base + node_of<N>(d, m, a, b);
        R c[5], v[5];
#pragma unroll
        for (int t = 0; t < 5; ++t) c[t] = q[t * fs + nd];
        prim_of<R>(c, v, gm1);
#pragma unroll
        for (int t = 0; t < 5; ++t) acc[t] = m == 0 ? mul_rn(fv[0], v[t]) : fma_rn(fv[m], v[t], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < 5; ++t) P[t] = acc[t];
}

// face polynomial with GL values fv (LDS) at GL point pt of quarter h
template <int N, typename R>
__device__ __forceinline__ R sub_interp(const R* fv, const Tab<N, R>& T, int h, int pt) {
    const int a = pt % N, b = pt / N, h1 = h & 1, h2 = h >> 1;
    R acc = 0;
#pragma unroll
    for (int bb = 0; bb < N; ++bb) {
        R s = 0;
#pragma unroll
        for (int aa = 0; aa < N; ++aa) s += T.H[h1][a][aa] * fv[aa + N * bb];
        acc += T.H[h2][b][bb] * s;
    }
    return acc;
}

// transpose: contribution of subface values sv (quarter h) to coarse point pt
template <int N, typename R>
__device__ __forceinline__ R sub_interp_T(const R* sv, const Tab<N, R>& T, int h, int pt) {
    const int a = pt % N, b = pt / N, h1 = h & 1, h2 = h >> 1;
    R acc = 0;
#pragma unroll
    for (int bb = 0; bb < N; ++bb) {
        R s = 0;
#pragma unroll
        for (int aa = 0; aa < N; ++aa) s += T.H[h1][aa][a] * sv[aa + N * bb];
        acc += T.H[h2][bb][b] * s;
    }
    return acc;
}

// The terrain-following (Gal-Chen) map keeps x and y affine in the reference
// coordinates, so W cof(J) vanishes at (0,1), (0,2), (1,0), (1,2) and the n dS
// of the x- and y-faces has only its normal component: only the other
// entries are stored (the host checks that the dropped ones are zero).
template <int N, typename R>
__device__ __forceinline__ void nS_gc(const Geom<R>& g, int64_t e, int f, int pt, R nS[3]) {
    constexpr int NF = N * N;
    const R* b = g.nS + (size_t)e * 10 * NF;
    if (f < 4) {
        nS[0] = nS[1] = nS[2] = 0;
        nS[f >> 1] = b[f * NF + pt];
    } else {
        const int s0 = 4 + 3 * (f - 4);
#pragma unroll
        for (int c = 0; c < 3; ++c) nS[c] = b[(s0 + c) * NF + pt];
    }
}
// W cof(J)[dd][c] at entry o = e Np + node of a field of E Np values
template <typename R>
__device__ __forceinline__ R G_gc(const Geom<R>& g, size_t fsz, int dd, int c, size_t o) {
    if (dd == 0) return c == 0 ? g.G[o] : (R)0;
    if (dd == 1) return c == 1 ? g.G[fsz + o] : (R)0;
    return g.G[(size_t)(2 + c) * fsz + o];
}

// The same entries from the compact metric (meshes without hanging faces):
// J20 = (J20 / phi) phi, J21 likewise, J22 from the element's (x, y) plane,
// J00 = h_x, J11 = h_y, multiplied in the host geometry's order; the weights
// come from the global copy of the tables (read before the first barrier).
template <int N, typename R>
__device__ __forceinline__ void cm_node(const Geom<R>& g, const Tab<N, R>* __restrict__ Tg, int64_t e, int node,
                                        R J00, R J11, R gv[5], R& iwj) {
    constexpr int NF = N * N;
    const R* c = g.cm + (size_t)e * cm_stride(N);
    const int ij = node % NF, k = node / NF;
    const R W = Tg->W3[node];
    const R J22 = c[ij], ph = c[3 * NF + 4 * N + k];
    const R J20 = c[NF + ij] * ph, J21 = c[2 * NF + ij] * ph;
    gv[0] = W * (J11 * J22);
    gv[1] = W * (J00 * J22);
    gv[2] = W * (-(J11 * J20));
    gv[3] = W * (-(J00 * J21));
    gv[4] = W * (J00 * J11);
    iwj = (R)1 / (W * (J00 * (J11 * J22)));
}
// W detJ at a node from the compact metric
template <int N, typename R>
__device__ __forceinline__ R cm_wj(const Geom<R>& g, const Tab<N, R>* __restrict__ Tg, int64_t e, int node) {
    const R J22 = g.cm[(size_t)e * cm_stride(N) + node % (N * N)];
    return Tg->W3[node] * ((R)g.h[3 * e] * ((R)g.h[3 * e + 1] * J22));
}
// n dS of face f at point pt (a + N b) from the compact metric: on x-faces
// J11 J22, on y-faces J00 J22 (J22 at the face), on z-faces the third row of
// cof(J) with phi at the face
template <int N, typename R>
__device__ __forceinline__ void cm_area(const Geom<R>& g, const Tab<N, R>* __restrict__ Tg, int64_t e, R J00, R J11,
                                        int f, int pt, R nS[3]) {
    constexpr int NF = N * N;
    const R* c = g.cm + (size_t)e * cm_stride(N);
    const int d = f >> 1, s = f & 1, a = pt % N;
    const R w2 = Tg->W2[pt], W2 = s ? w2 : -w2;
    nS[0] = nS[1] = nS[2] = 0;
    if (d == 0) {
        nS[0] = W2 * (J11 * c[3 * NF + s * N + a]);
    } else if (d == 1) {
        nS[1] = W2 * (J00 * c[3 * NF + 2 * N + s * N + a]);
    } else {
        const R ph = c[3 * NF + 5 * N + s];
        nS[0] = W2 * (-(J11 * (c[NF + pt] * ph)));
        nS[1] = W2 * (-(J00 * (c[2 * NF + pt] * ph)));
        nS[2] = W2 * (J00 * J11);
    }
}

// W2-weighted outward area vector of face f of element e at point pt
template <int N, typename R>
__device__ __forceinline__ void area(const Geom<R>& g, const Tab<N, R>& T, int64_t e, int f, int pt, R nS[3]) {
    constexpr int NF = N * N;
    if (g.deformed) {
        nS_gc<N, R>(g, e, f, pt, nS);
        return;
    }
    const int d = f >> 1, s = f & 1;
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const R A = T.w[pt % N] * T.w[pt / N] * (R)(g.h[3 * e + t1] * g.h[3 * e + t2]);
    nS[0] = nS[1] = nS[2] = 0;
    nS[d] = s ? A : -A;
}

// the same with the geometry class known at compile time
template <int N, typename R, bool AFF>
__device__ __forceinline__ void area_t(const Geom<R>& g, const Tab<N, R>& T, int64_t e, int f, int pt, R nS[3]) {
    constexpr int NF = N * N;
    if constexpr (!AFF) {
        nS_gc<N, R>(g, e, f, pt, nS);
    } else {
        const int d = f >> 1, s = f & 1;
        const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
        const R A = T.w[pt % N] * T.w[pt / N] * (R)(g.h[3 * e + t1] * g.h[3 * e + t2]);
        nS[0] = nS[1] = nS[2] = 0;
        nS[d] = s ? A : -A;
    }
}

// W detJ (d xi_d / d x_c) at a node
template <int N, typename R>
__device__ __forceinline__ R metric(const Geom<R>& g, int64_t e, int node, int d, int c, R wj) {
    constexpr int NP = N * N * N;
    if (g.deformed) return G_gc<R>(g, (size_t)g.E * NP, d, c, (size_t)e * NP + node);
    return d == c ? wj * (R)g.hinv[3 * e + d] : (R)0;
}

// sum_d (D_d^T G_d) at node, G in LDS [3][NP]
template <int N, typename R>
__device__ __forceinline__ R div_T(const R* G, const Tab<N, R>& T, int node) {
    const int i = node % N, j = (node / N) % N, k = node / (N * N);
    R acc = 0;
#pragma unroll
    for (int q = 0; q < N; ++q) acc += T.D[q][i] * G[q + N * (j + N * k)];
#pragma unroll
    for (int q = 0; q < N; ++q) acc += T.D[q][j] * G[N * N * N + i + N * (q + N * k)];
#pragma unroll
    for (int q = 0; q < N; ++q) acc += T.D[q][k] * G[2 * N * N * N + i + N * (j + N * q)];
    return acc;
}

// ---------------------------------------------------------- Euler fluxes
// Normal fluxes seen from side A (area vector nS of side A) from the face
// values (rho, u, p) of both sides: 0..4 non-stiff (rho, m, E with Rusanov
// dissipation on rho, m, rho kappa; m = rho u, kappa = |u|^2 / 2), 5..7
// stiff pressure {p} nS, 8 stiff enthalpy {rho h u}.nS + Rusanov on rho e.
// A slip wall mirrors u.
template <typename R>
__device__ __forceinline__ void euler_flux(const R* pa, const R* pbin, const R* nS, bool wall, R igm1, R hfac,
                                           R* fl) {
    const R dS = sqrt(nS[0] * nS[0] + nS[1] * nS[1] + nS[2] * nS[2]);
    const R idS = (R)1 / dS;
    const R nh[3] = {nS[0] * idS, nS[1] * idS, nS[2] * idS};
    R pb[5];
    if (wall) {
        const R un = pa[1] * nh[0] + pa[2] * nh[1] + pa[3] * nh[2];
        pb[0] = pa[0];
        pb[4] = pa[4];
        for (int c = 0; c < 3; ++c) pb[1 + c] = pa[1 + c] - (R)2 * un * nh[c];
    } else {
        for (int t = 0; t < 5; ++t) pb[t] = pbin[t];
    }
    const R rA = pa[0], rB = pb[0];
    const R uA[3] = {pa[1], pa[2], pa[3]}, uB[3] = {pb[1], pb[2], pb[3]};
    R mA[3], mB[3];
    for (int c = 0; c < 3; ++c) {
        mA[c] = rA * uA[c];
        mB[c] = rB * uB[c];
    }
    const R kA = (R)0.5 * (uA[0] * uA[0] + uA[1] * uA[1] + uA[2] * uA[2]);
    const R kB = (R)0.5 * (uB[0] * uB[0] + uB[1] * uB[1] + uB[2] * uB[2]);
    const R pA = pa[4], pB = pb[4];
    const R unSA = uA[0] * nS[0] + uA[1] * nS[1] + uA[2] * nS[2];
    const R unSB = uB[0] * nS[0] + uB[1] * nS[1] + uB[2] * nS[2];
    // lambda dS = max(|u_A . n|, |u_B . n|) dS = max(|u_A . nS|, |u_B . nS|)
    const R hl = (R)0.5 * fmax(fabs(unSA), fabs(unSB));
    const R mnA = mA[0] * nS[0] + mA[1] * nS[1] + mA[2] * nS[2];
    const R mnB = mB[0] * nS[0] + mB[1] * nS[1] + mB[2] * nS[2];
    fl[0] = (R)0.5 * (mnA + mnB) + hl * (rA - rB);
    for (int c = 0; c < 3; ++c) fl[1 + c] = (R)0.5 * (mA[c] * unSA + mB[c] * unSB) + hl * (mA[c] - mB[c]);
    fl[4] = (R)0.5 * (kA * mnA + kB * mnB) + hl * (rA * kA - rB * kB);
    const R pavg = (R)0.5 * (pA + pB);
    for (int c = 0; c < 3; ++c) fl[5 + c] = pavg * nS[c];
    const R hA = hfac * pA, hB = hfac * pB;
    fl[8] = (R)0.5 * (hA * unSA + hB * unSB) + hl * (pA - pB) * igm1;
}

// (rho h)^k (w . nS) at a face point, rounded the same way wherever formed
template <typename R>
__device__ __forceinline__ R fb_value(R hfac, R hk, R w0, R w1, R w2, const R* nS) {
    const R wn = add_rn(add_rn(mul_rn(w0, nS[0]), mul_rn(w1, nS[1])), mul_rn(w2, nS[2]));
    return mul_rn(mul_rn(hfac, hk), wn);
}

// value of the coarse neighbour's face polynomial (face (d, side) of the
// element at f) at point pt of quarter sub; the same arithmetic as taking
// the coarse face values first and then sub_interp
template <int N, typename R, typename P>
__device__ __forceinline__ R coarse_point(const P* f, const R* fv, const Tab<N, R>& T, int d, int sub, int pt) {
    const int a = pt % N, b = pt / N, h1 = sub & 1, h2 = sub >> 1;
    R acc = 0;
#pragma unroll 1
    for (int bb = 0; bb < N; ++bb) {
        R s = 0;
#pragma unroll 1
        for (int aa = 0; aa < N; ++aa) s += T.H[h1][a][aa] * face_value<N>(f, fv, d, aa + N * bb);
        acc += T.H[h2][b][bb] * s;
    }
    return acc;
}

// coarse_point for the five primitives (rho, u, p) of the coarse neighbour
// (conserved fields at q + t * fs + base)
template <int N, typename R>
__device__ __forceinline__ void coarse_point_prim(const R* q, size_t fs, size_t base, const R* fv, const Tab<N, R>& T,
                                                  int d, int sub, int pt, R gm1, R* P) {
    const int a = pt % N, b = pt / N, h1 = sub & 1, h2 = sub >> 1;
    R acc[5] = {0, 0, 0, 0, 0};
#pragma unroll 1
    for (int bb = 0; bb < N; ++bb) {
        R s[5] = {0, 0, 0, 0, 0};
#pragma unroll 1
        for (int aa = 0; aa < N; ++aa) {
            R v[5];
            face_value_prim<N, R>(q, fs, base, fv, d, aa + N * bb, gm1, v);
#pragma unroll
            for (int t = 0; t < 5; ++t) s[t] += T.H[h1][a][aa] * v[t];
        }
#pragma unroll
        for (int t = 0; t < 5; ++t) acc[t] += T.H[h2][b][bb] * s[t];
    }
#pragma unroll
    for (int t = 0; t < 5; ++t) P[t] = acc[t];
}

// =====================================================================
// Explicit residual: fNS = M^{-1} T_NS, fS = M^{-1} T_S (momentum, energy)
// =====================================================================
// HANG = false compiles out the coarse-neighbour interpolation, for meshes
// without hanging faces (it sets the register count of the all-faces path).
template <int N, typename R, bool SLOW, bool AFF, bool HANG = true>
__global__ void __launch_bounds__(threads_of(N))
k_explicit(const int* __restrict__ elist, int64_t nel, const R* __restrict__ q, R* __restrict__ fNS, R* __restrict__ fS, Geom<R> g, const Tab<N, R>* __restrict__ Tg,
           PhysK ph, const double* __restrict__ sponge) {
    constexpr int NP = N * N * N, NF = N * N, EPB = epb_of(N);
    constexpr int L_FAST = 6 * 9 * NF, L_SLOW = 5 * NF + 5 * NF + 9 * NF + 4 * 9 * NF, L_VOL = 9 * NP;
    constexpr int UN = (L_FAST > L_SLOW ? L_FAST : L_SLOW) > L_VOL ? (L_FAST > L_SLOW ? L_FAST : L_SLOW) : L_VOL;
    __shared__ R s_q[EPB][5][NP];
    __shared__ R s_u[EPB][UN];
    const int tid = threadIdx.x, le = elem_slot<NP>(tid), node = tid - le * NP;
    __shared__ Tab<N, R> T;
    load_tab<N, R>(Tg, &T);
    const int64_t slot = xcd_block(blockIdx.x, gridDim.x) * EPB + le;
    const bool act = le < EPB && slot < nel;
    const int64_t e = act ? (elist ? (int64_t)elist[slot] : slot) : 0;
    const size_t fs = (size_t)g.E * NP;
    const R gm1 = (R)ph.gm1, igm1 = (R)ph.igm1, hfac = (R)ph.hfac;
    // the element's own nodes as (rho, u, p): face values are their traces
    if (act) {
        R c[5], P[5];
        for (int t = 0; t < 5; ++t) c[t] = q[t * fs + e * NP + node];
        prim_of<R>(c, P, gm1);
        for (int t = 0; t < 5; ++t) s_q[le][t][node] = P[t];
    }
    constexpr bool slow = SLOW;
    __syncthreads();
    R acc[9];
    for (int o = 0; o < 9; ++o) acc[o] = 0;
    R* U = &s_u[le][0];

    if (!slow) {
        // all faces at once: U[(f*9 + o)*NF + pt]
        if (act)
            for (int it = node; it < 6 * NF; it += NP) {
                const int f = it / NF, pt = it - f * NF, d = f >> 1, s = f & 1;
                const int kind = g.kind[e * 6 + f], nbr = g.nbr[e * 6 + f];
                R qa[5], qb[5], nS[3], fl[9];
                for (int t = 0; t < 5; ++t) qa[t] = face_value<N>(&s_q[le][t][0], T.f[s], d, pt);
                if (kind == CONF)
                    face_value_prim<N, R>(q, fs, (size_t)nbr * NP, T.f[1 - s], d, pt, gm1, qb);
                else if (HANG && kind == FINE) {
                    if constexpr (HANG)
                        coarse_point_prim<N, R>(q, fs, (size_t)nbr * NP, T.f[1 - s], T, d, g.aux[e * 6 + f] & 3, pt,
                                                gm1, qb);
                }
                area_t<N, R, AFF>(g, T, e, f, pt, nS);
                euler_flux<R>(qa, qb, nS, kind == WALL, igm1, hfac, fl);
                for (int o = 0; o < 9; ++o) U[(f * 9 + o) * NF + pt] = fl[o];
            }
        __syncthreads();
        if (act)
            for (int f = 0; f < 6; ++f) {
                int m, pt;
                split_node<N>(f >> 1, node, m, pt);
                const R lf = T.f[f & 1][m];
                for (int o = 0; o < 9; ++o) acc[o] -= lf * U[(f * 9 + o) * NF + pt];
            }
    } else {
        R* s_own = U;                 // [5][NF]
        R* s_nb = U + 5 * NF;         // [5][NF]
        R* s_fl = U + 10 * NF;        // [9][NF]
        R* s_sub = U + 19 * NF;       // [4][9][NF]
        for (int f = 0; f < 6; ++f) {
            const int d = f >> 1, s = f & 1;
            const int kind = act ? g.kind[e * 6 + f] : -1;
            const int nbr = act ? g.nbr[e * 6 + f] : 0;
            const int aux = act ? g.aux[e * 6 + f] : 0;
            if (act && node < NF) {
                for (int t = 0; t < 5; ++t) s_own[t * NF + node] = face_value<N>(&s_q[le][t][0], T.f[s], d, node);
                if (kind == CONF || kind == FINE) {
                    R P[5];
                    face_value_prim<N, R>(q, fs, (size_t)nbr * NP, T.f[1 - s], d, node, gm1, P);
                    for (int t = 0; t < 5; ++t) s_nb[t * NF + node] = P[t];
                }
            }
            __syncthreads();
            if (act) {
                const int nit = kind == COARSE ? 4 * NF : NF;
                for (int it = node; it < nit; it += NP) {
                    const int hs = it / NF, pt = it - hs * NF;
                    R qa[5], qb[5], nS[3], fl[9];
                    bool wall = false;
                    if (kind == COARSE) {
                        const int fn = g.hang[nbr * 4 + hs];
                        for (int t = 0; t < 5; ++t) qa[t] = sub_interp<N>(s_own + t * NF, T, hs, pt);
                        face_value_prim<N, R>(q, fs, (size_t)fn * NP, T.f[1 - s], d, pt, gm1, qb);
                        area_t<N, R, AFF>(g, T, fn, f ^ 1, pt, nS);
                        for (int c = 0; c < 3; ++c) nS[c] = -nS[c];
                    } else {
                        for (int t = 0; t < 5; ++t) qa[t] = s_own[t * NF + pt];
                        if (kind == CONF)
                            for (int t = 0; t < 5; ++t) qb[t] = s_nb[t * NF + pt];
                        else if (kind == FINE)
                            for (int t = 0; t < 5; ++t) qb[t] = sub_interp<N>(s_nb + t * NF, T, aux & 3, pt);
                        else
                            wall = true;
                        area_t<N, R, AFF>(g, T, e, f, pt, nS);
                    }
                    euler_flux<R>(qa, qb, nS, wall, igm1, hfac, fl);
                    if (kind == COARSE)
                        for (int o = 0; o < 9; ++o) s_sub[(hs * 9 + o) * NF + pt] = fl[o];
                    else
                        for (int o = 0; o < 9; ++o) s_fl[o * NF + pt] = fl[o];
                }
            }
            __syncthreads();
            if (act && kind == COARSE && node < NF)
                for (int o = 0; o < 9; ++o) {
                    R v = 0;
                    for (int h = 0; h < 4; ++h) v += sub_interp_T<N>(s_sub + (h * 9 + o) * NF, T, h, node);
                    s_fl[o * NF + node] = v;
                }
            __syncthreads();
            if (act) {
                int m, pt;
                split_node<N>(d, node, m, pt);
                const R lf = T.f[s][m];
                for (int o = 0; o < 9; ++o) acc[o] -= lf * s_fl[o * NF + pt];
            }
            __syncthreads();
        }
    }
    __syncthreads();   // the volume staging reuses the face buffers

    // volume terms, three outputs per round: U[(o3*3 + d)*NP + node]
    R rho = 1, u[3] = {0, 0, 0}, mom[3] = {0, 0, 0}, kin = 0, p = 0, wj = 1;
    if (act) {
        rho = s_q[le][0][node];
        for (int c = 0; c < 3; ++c) {
            u[c] = s_q[le][1 + c][node];
            mom[c] = rho * u[c];
        }
        kin = (R)0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        p = s_q[le][4][node];
        wj = AFF ? T.W3[node] * (R)g.eg[e * 8 + 6] : g.WJ[e * NP + node];
    }
    for (int r3 = 0; r3 < 3; ++r3) {
        if (act)
            for (int o3 = 0; o3 < 3; ++o3) {
                const int o = 3 * r3 + o3;
                R F[3];
                if (o == 0) {
                    for (int c = 0; c < 3; ++c) F[c] = mom[c];
                } else if (o < 4) {
                    const R mo = mom[o - 1];
                    for (int c = 0; c < 3; ++c) F[c] = mo * u[c];
                } else if (o == 4) {
                    for (int c = 0; c < 3; ++c) F[c] = kin * mom[c];
                } else if (o < 8) {
                    for (int c = 0; c < 3; ++c) F[c] = (c == o - 5) ? p : (R)0;
                } else {
                    const R rh = hfac * p;
                    for (int c = 0; c < 3; ++c) F[c] = rh * u[c];
                }
                if constexpr (AFF) {
#pragma unroll
                    for (int dd = 0; dd < 3; ++dd) U[(o3 * 3 + dd) * NP + node] = (wj * (R)g.hinv[3 * e + dd]) * F[dd];
                } else {
#pragma unroll
                    for (int dd = 0; dd < 3; ++dd) {
                        R v = 0;
#pragma unroll
                        for (int c = 0; c < 3; ++c) v += G_gc<R>(g, fs, dd, c, (size_t)e * NP + node) * F[c];
                        U[(o3 * 3 + dd) * NP + node] = v;
                    }
                }
            }
        __syncthreads();
        if (act)
            for (int o3 = 0; o3 < 3; ++o3) acc[3 * r3 + o3] += div_T<N>(U + o3 * 3 * NP, T, node);
        __syncthreads();
    }
    if (!act) return;
    acc[5] += wj * rho * (R)ph.f * u[1];
    acc[6] -= wj * rho * (R)ph.f * u[0];
    acc[7] -= wj * rho * (R)ph.g;
    acc[8] -= wj * rho * (R)ph.g * u[2];
    if (ph.sponge) {
        const R lam = (R)sponge[e * NP + node];
        for (int c = 0; c < 3; ++c) acc[1 + c] -= wj * lam * (mom[c] - rho * (R)ph.su[c]);
    }
    const R iwj = AFF ? T.iW3[node] * (R)g.eg[e * 8 + 7] : g.iWJ[e * NP + node];
    for (int t = 0; t < 5; ++t) fNS[t * fs + e * NP + node] = acc[t] * iwj;
    for (int t = 0; t < 4; ++t) fS[t * fs + e * NP + node] = acc[5 + t] * iwj;
}

// Explicit residual on terrain-following (Gal-Chen) elements without a
// coarse hanging face. Same weak forms as k_explicit, organised for few
// synchronisation points and few LDS round trips:
//  - every global load that does not depend on another (own fields, the five
//    stored entries of W cof(J), 1 / W detJ, the sponge coefficient, this
//    lane's face table entries, kinds, neighbours and n dS) is issued before
//    the first barrier; the neighbour values along the normal are gathered
//    face point by face point after it (holding them all would halve the
//    occupancy);
//  - the volume term uses the sparsity of W cof(J): a flux vector F has the
//    contravariant components (G00 F0, G11 F1, G20 F0 + G21 F1 + G22 F2), and
//    the pressure terms need five staged arrays instead of nine, so the nine
//    outputs take 23 contractions in three rounds;
//  - the sources (gravity, Coriolis, sponge) are added after the division by
//    W detJ, which they carry as a factor, so W detJ itself is not read.
template <int N, typename R, bool HANG = true>
__global__ void __launch_bounds__(threads_of(N))
k_explicit_gc(const int* __restrict__ elist, int64_t nel, const R* __restrict__ q, R* __restrict__ fNS,
              R* __restrict__ fS, Geom<R> g, const Tab<N, R>* __restrict__ Tg, PhysK ph,
              const double* __restrict__ sponge) {
    constexpr int NP = N * N * N, NF = N * N, EPB = epb_of(N);
    constexpr int NR = (6 * NF + NP - 1) / NP;   // face points per lane
    constexpr int LU = 54 * NF > 9 * NP ? 54 * NF : 9 * NP;
    __shared__ R s_q[EPB][5][NP];
    __shared__ R s_u[EPB][LU];
    __shared__ Tab<N, R> T;
    load_tab<N, R>(Tg, &T);
    const int tid = threadIdx.x, le = elem_slot<NP>(tid), node = tid - le * NP;
    const int64_t slot = xcd_block(blockIdx.x, gridDim.x) * EPB + le;
    const bool act = le < EPB && slot < nel;
    const int64_t e = act ? (elist ? (int64_t)elist[slot] : slot) : 0;
    const size_t fs = (size_t)g.E * NP, o = (size_t)e * NP + node;
    const R gm1 = (R)ph.gm1, igm1 = (R)ph.igm1, hfac = (R)ph.hfac;
    R* U = &s_u[le][0];
    R qv[5] = {1, 0, 0, 0, 1}, gv[5] = {0, 0, 0, 0, 0}, iwj = 0, lam = 0;
    R nsv[NR][3];
    int kf[NR], nf[NR];
    uint64_t fo[NR];
    if (act) {
        // the own node as (rho, u, p): face values are traces of these
        R c[5], P[5];
#pragma unroll
        for (int t = 0; t < 5; ++t) c[t] = q[t * fs + o];
        prim_of<R>(c, P, gm1);
#pragma unroll
        for (int t = 0; t < 5; ++t) s_q[le][t][node] = P[t];
#pragma unroll
        for (int t = 0; t < 5; ++t) gv[t] = g.G[t * fs + o];
        iwj = g.iWJ[o];
        if (ph.sponge) lam = (R)sponge[o];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            fo[r] = g.fofs[r * NP + node];
            const bool full = (r + 1) * NP <= 6 * NF;
            const int f = fo_face(fo[r]);
            const bool has = full || f < 6;
            const int fc = has ? f : 5;
            kf[r] = has ? g.kind[e * 6 + fc] : WALL;
            nf[r] = g.nbr[e * 6 + fc];
            nS_gc<N, R>(g, e, fc, fo_point(fo[r]), nsv[r]);
        }
    }
    __syncthreads();
    R acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = 0;
    // numerical fluxes at every face point: U[(f*9 + o)*NF + pt]
    if (act)
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int f = fo_face(fo[r]);
            if ((r + 1) * NP > 6 * NF && f >= 6) continue;
            const int pt = fo_point(fo[r]), d = f >> 1, s = f & 1;
            R qa[5], qb[5], fl[9];
#pragma unroll
            for (int t = 0; t < 5; ++t) {
                R v[N];
#pragma unroll
                for (int m = 0; m < N; ++m) v[m] = s_q[le][t][fo_node(fo[r], m)];
                qa[t] = trace_chain<N, R>(T.f[s], v);
            }
            if (HANG && kf[r] == FINE) {
                if constexpr (HANG)
                    coarse_point_prim<N, R>(q, fs, (size_t)nf[r] * NP, T.f[1 - s], T, d, g.aux[e * 6 + f] & 3, pt,
                                            gm1, qb);
            } else if (kf[r] == CONF) {
                // the neighbour's nodes along the normal (conforming and periodic
                // faces), each converted to (rho, u, p), traced by the same chain
                const size_t nb = (size_t)nf[r] * NP;
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    R c[5], v[5];
#pragma unroll
                    for (int t = 0; t < 5; ++t) c[t] = q[t * fs + nb + fo_node(fo[r], m)];
                    prim_of<R>(c, v, gm1);
#pragma unroll
                    for (int t = 0; t < 5; ++t) qb[t] = m == 0 ? mul_rn(T.f[1 - s][0], v[t]) : fma_rn(T.f[1 - s][m], v[t], qb[t]);
                }
            } else {
#pragma unroll
                for (int t = 0; t < 5; ++t) qb[t] = qa[t];   // wall: mirrored inside the flux
            }
            euler_flux<R>(qa, qb, nsv[r], kf[r] == WALL, igm1, hfac, fl);
#pragma unroll
            for (int k = 0; k < 9; ++k) U[(f * 9 + k) * NF + pt] = fl[k];
            // one face point at a time: keeps the next point's gathers from
            // being hoisted above this one's flux (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
    __syncthreads();
    if (act)
        for (int f = 0; f < 6; ++f) {
            int m, pt;
            split_node<N>(f >> 1, node, m, pt);
            const R lf = T.f[f & 1][m];
#pragma unroll
            for (int k = 0; k < 9; ++k) acc[k] -= lf * U[(f * 9 + k) * NF + pt];
        }
    __syncthreads();   // the volume staging reuses U
    // own values again from LDS (not kept in registers across the face phase)
    if (act)
#pragma unroll
        for (int t = 0; t < 5; ++t) qv[t] = s_q[le][t][node];
    const R rho = qv[0];
    const R u[3] = {qv[1], qv[2], qv[3]};
    const R mom[3] = {rho * u[0], rho * u[1], rho * u[2]};
    const R kin = (R)0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const R p = qv[4];
    const int ix = node % N, jy = (node / N) % N, kz = node / (N * N);
    // contravariant components of a flux vector F into U[3*a .. 3*a+2]
    auto stage3 = [&](int a, R F0, R F1, R F2) {
        U[(3 * a) * NP + node] = gv[0] * F0;
        U[(3 * a + 1) * NP + node] = gv[1] * F1;
        U[(3 * a + 2) * NP + node] = gv[2] * F0 + gv[3] * F1 + gv[4] * F2;
    };
    auto div3 = [&](int a) -> R {
        const R* A0 = U + (3 * a) * NP;
        const R* A1 = U + (3 * a + 1) * NP;
        const R* A2 = U + (3 * a + 2) * NP;
        R v = 0;
#pragma unroll
        for (int qq = 0; qq < N; ++qq) v += T.D[qq][ix] * A0[qq + N * (jy + N * kz)];
#pragma unroll
        for (int qq = 0; qq < N; ++qq) v += T.D[qq][jy] * A1[ix + N * (qq + N * kz)];
#pragma unroll
        for (int qq = 0; qq < N; ++qq) v += T.D[qq][kz] * A2[ix + N * (jy + N * qq)];
        return v;
    };
    // round 1: mass flux and the x and y momentum fluxes
    if (act) {
        stage3(0, mom[0], mom[1], mom[2]);
        stage3(1, mom[0] * u[0], mom[0] * u[1], mom[0] * u[2]);
        stage3(2, mom[1] * u[0], mom[1] * u[1], mom[1] * u[2]);
    }
    __syncthreads();
    if (act) {
        acc[0] += div3(0);
        acc[1] += div3(1);
        acc[2] += div3(2);
    }
    __syncthreads();
    // round 2: z momentum, kinetic energy and enthalpy fluxes
    if (act) {
        stage3(0, mom[2] * u[0], mom[2] * u[1], mom[2] * u[2]);
        stage3(1, kin * mom[0], kin * mom[1], kin * mom[2]);
        const R rh = hfac * p;
        stage3(2, rh * u[0], rh * u[1], rh * u[2]);
    }
    __syncthreads();
    if (act) {
        acc[3] += div3(0);
        acc[4] += div3(1);
        acc[8] += div3(2);
    }
    __syncthreads();
    // round 3: the pressure, (G00 p, G11 p, G20 p, G21 p, G22 p)
    if (act)
#pragma unroll
        for (int t = 0; t < 5; ++t) U[t * NP + node] = gv[t] * p;
    __syncthreads();
    if (!act) return;
    {
        R x0 = 0, y1 = 0, z0 = 0, z1 = 0, z2 = 0;
#pragma unroll
        for (int qq = 0; qq < N; ++qq) {
            x0 += T.D[qq][ix] * U[qq + N * (jy + N * kz)];
            y1 += T.D[qq][jy] * U[NP + ix + N * (qq + N * kz)];
            const int zq = ix + N * (jy + N * qq);
            z0 += T.D[qq][kz] * U[2 * NP + zq];
            z1 += T.D[qq][kz] * U[3 * NP + zq];
            z2 += T.D[qq][kz] * U[4 * NP + zq];
        }
        acc[5] += x0 + z0;
        acc[6] += y1 + z1;
        acc[7] += z2;
    }
    const R fc = (R)ph.f, gg = (R)ph.g;
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        R v = acc[t] * iwj;
        if (t >= 1 && t <= 3 && ph.sponge) v -= lam * (mom[t - 1] - rho * (R)ph.su[t - 1]);
        fNS[t * fs + o] = v;
    }
    fS[o] = acc[5] * iwj + rho * fc * u[1];
    fS[fs + o] = acc[6] * iwj - rho * fc * u[0];
    fS[2 * fs + o] = acc[7] * iwj - rho * gg;
    fS[3 * fs + o] = acc[8] * iwj - rho * gg * u[2];
}

// =====================================================================
// Schur pass 1: w = P (Fh/rho - M^{-1} B p / rho) (+ R1 lag), face buffers
// =====================================================================
template <int N, typename R, bool SLOW>
__global__ void __launch_bounds__(threads_of(N))
k_pass1(const int* __restrict__ elist, int64_t nel, const R* __restrict__ p, const R* __restrict__ pscale, const R* __restrict__ Fh,
        const R* __restrict__ rho, const R* __restrict__ pk, const R* __restrict__ uk, R* __restrict__ w,
        R* __restrict__ FB, R* __restrict__ FBh, Geom<R> g, const Tab<N, R>* __restrict__ Tg, StageK sk,
        const int* __restrict__ ctrl) {
    if (ctrl && *ctrl != 0) return;
    constexpr int NP = N * N * N, NF = N * N, EPB = epb_of(N);
    constexpr int L_FAST = 6 * 3 * NF, L_SLOW = 4 * NF + NF + 3 * NF + 4 * 3 * NF, L_VOL = 3 * NP;
    constexpr int NR = (6 * NF + NP - 1) / NP;   // face points per lane
    constexpr int UN = (L_FAST > L_SLOW ? L_FAST : L_SLOW) > L_VOL ? (L_FAST > L_SLOW ? L_FAST : L_SLOW) : L_VOL;
    __shared__ R s_p[EPB][NP];
    __shared__ R s_pk[EPB][NP];
    __shared__ R s_w[EPB][3][NP];
    __shared__ R s_u[EPB][UN];
    __shared__ int s_kind[EPB][6], s_nbr[EPB][6];
    const int tid = threadIdx.x, le = elem_slot<NP>(tid), node = tid - le * NP;
    __shared__ Tab<N, R> T;
    load_tab<N, R>(Tg, &T);
    const int64_t slot = xcd_block(blockIdx.x, gridDim.x) * EPB + le;
    const bool act = le < EPB && slot < nel;
    const int64_t e = act ? (elist ? (int64_t)elist[slot] : slot) : 0;
    const size_t fs = (size_t)g.E * NP;
    const R gam = (R)sk.gamma;
    const R sc = pscale ? pscale[0] : (R)1;
    R* U = &s_u[le][0];
    // every global load of the kernel is issued here, before the first barrier:
    // own fields, the face table and (fast path) the neighbour gathers
    R* FL = U;                 // fast path: {p} nS at FL[(f*3 + c)*NF + pt]
    R nbv[NR][N];              // fast path: the neighbour's values along the normal at this lane's points
    R wj = (R)1, rl = (R)1, fh[3] = {0, 0, 0}, ukv[2] = {0, 0};
    if (act) {
        s_p[le][node] = p ? p[e * NP + node] : (R)0;
        s_pk[le][node] = pk[e * NP + node];
        wj = g.WJ[e * NP + node];
        rl = rho[e * NP + node];
        if (Fh)
            for (int c = 0; c < 3; ++c) fh[c] = Fh[c * fs + e * NP + node];
        if (uk && Fh && sk.scheme == 1) {
            ukv[0] = uk[0 * fs + e * NP + node];
            ukv[1] = uk[1 * fs + e * NP + node];
        }
        int kf[6], nf[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            kf[f] = g.kind[e * 6 + f];
            nf[f] = g.nbr[e * 6 + f];
        }
        if (node < 6) {
            s_kind[le][node] = kf[node];
            s_nbr[le][node] = nf[node];
        }
        if (!SLOW && p) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const int it = node + r * NP;
                int f = it / NF;
                f = f < 6 ? f : 5;
                const int pt = it - f * NF, d = f >> 1, a = pt % N, b = pt / N;
                const bool ld = it < 6 * NF && kf[f] == CONF;
                const R* src = p + (size_t)(ld ? nf[f] : 0) * NP;
#pragma unroll
                for (int m = 0; m < N; ++m) nbv[r][m] = ld ? src[node_of<N>(d, m, a, b)] : (R)0;
            }
        }
    }
    constexpr bool slow = SLOW;
    __syncthreads();
    R acc[3] = {0, 0, 0};
    if (p) {
        if (!slow) {
            if (act)
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const int it = node + r * NP;
                    if (it >= 6 * NF) break;
                    const int f = it / NF, pt = it - f * NF, d = f >> 1, s = f & 1;
                    const int kind = s_kind[le][f];
                    const R pa = sc * face_value<N>(&s_p[le][0], T.f[s], d, pt);
                    R pb = pa;
                    if (kind == CONF) {
                        pb = sc * trace_chain<N, R>(T.f[1 - s], nbv[r]);
                    } else if (kind == FINE) {
                        pb = sc * coarse_point<N>(p + (size_t)s_nbr[le][f] * NP, T.f[1 - s], T, d,
                                                  g.aux[e * 6 + f] & 3, pt);
                    }
                    R nS[3];
                    area<N>(g, T, e, f, pt, nS);
                    const R avg = (R)0.5 * (pa + pb);
                    for (int c = 0; c < 3; ++c) FL[(f * 3 + c) * NF + pt] = avg * nS[c];
                }
            __syncthreads();
            if (act)
                for (int f = 0; f < 6; ++f) {
                    int m, pt;
                    split_node<N>(f >> 1, node, m, pt);
                    const R lf = T.f[f & 1][m];
                    for (int c = 0; c < 3; ++c) acc[c] += lf * FL[(f * 3 + c) * NF + pt];
                }
        } else {
            R* s_own = U;               // [NF]
            R* s_nb = U + NF;           // [NF]
            R* s_fl = U + 2 * NF;       // [3][NF]
            R* s_sub = U + 5 * NF;      // [4][3][NF]
            for (int f = 0; f < 6; ++f) {
                const int d = f >> 1, s = f & 1;
                const int kind = act ? g.kind[e * 6 + f] : -1;
                const int nbr = act ? g.nbr[e * 6 + f] : 0;
                const int aux = act ? g.aux[e * 6 + f] : 0;
                if (act && node < NF) {
                    s_own[node] = sc * face_value<N>(&s_p[le][0], T.f[s], d, node);
                    if (kind == CONF || kind == FINE)
                        s_nb[node] = sc * face_value<N>(p + (size_t)nbr * NP, T.f[1 - s], d, node);
                }
                __syncthreads();
                if (act) {
                    const int nit = kind == COARSE ? 4 * NF : NF;
                    for (int it = node; it < nit; it += NP) {
                        const int hs = it / NF, pt = it - hs * NF;
                        R pa, pb, nS[3];
                        if (kind == COARSE) {
                            const int fn = g.hang[nbr * 4 + hs];
                            pa = sub_interp<N>(s_own, T, hs, pt);
                            pb = sc * face_value<N>(p + (size_t)fn * NP, T.f[1 - s], d, pt);
                            area<N>(g, T, fn, f ^ 1, pt, nS);
                            for (int c = 0; c < 3; ++c) nS[c] = -nS[c];
                        } else {
                            pa = s_own[pt];
                            pb = kind == CONF ? s_nb[pt] : (kind == FINE ? sub_interp<N>(s_nb, T, aux & 3, pt) : pa);
                            area<N>(g, T, e, f, pt, nS);
                        }
                        const R avg = (R)0.5 * (pa + pb);
                        for (int c = 0; c < 3; ++c) {
                            if (kind == COARSE) s_sub[(hs * 3 + c) * NF + pt] = avg * nS[c];
                            else s_fl[c * NF + pt] = avg * nS[c];
                        }
                    }
                }
                __syncthreads();
                if (act && kind == COARSE && node < NF)
                    for (int c = 0; c < 3; ++c) {
                        R v = 0;
                        for (int h = 0; h < 4; ++h) v += sub_interp_T<N>(s_sub + (h * 3 + c) * NF, T, h, node);
                        s_fl[c * NF + node] = v;
                    }
                __syncthreads();
                if (act) {
                    int m, pt;
                    split_node<N>(d, node, m, pt);
                    const R lf = T.f[s][m];
                    for (int c = 0; c < 3; ++c) acc[c] += lf * s_fl[c * NF + pt];
                }
                __syncthreads();
            }
        }
        __syncthreads();
        // volume: -int p div(phi_c)
        const R pv = act ? sc * s_p[le][node] : (R)0;
        if (!g.deformed) {
            if (act) U[node] = wj * pv;
            __syncthreads();
            if (act) {
                const int i = node % N, j = (node / N) % N, k = node / (N * N);
                R d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
                for (int qq = 0; qq < N; ++qq) {
                    d0 += T.D[qq][i] * U[qq + N * (j + N * k)];
                    d1 += T.D[qq][j] * U[i + N * (qq + N * k)];
                    d2 += T.D[qq][k] * U[i + N * (j + N * qq)];
                }
                acc[0] -= d0 * (R)g.hinv[3 * e + 0];
                acc[1] -= d1 * (R)g.hinv[3 * e + 1];
                acc[2] -= d2 * (R)g.hinv[3 * e + 2];
            }
        } else {
            for (int c = 0; c < 3; ++c) {
                if (act)
                    for (int dd = 0; dd < 3; ++dd) U[dd * NP + node] = metric<N>(g, e, node, dd, c, wj) * pv;
                __syncthreads();
                if (act) acc[c] -= div_T<N>(U, T, node);
                __syncthreads();
            }
        }
    }
    R wv[3] = {0, 0, 0};
    if (act) {
        const R r = rl;
        const R cdt = (R)sk.c_dt, beta = (R)sk.beta;
        R v[3];
        const R iwj = (R)1 / wj, ir = (R)1 / r;
        for (int c = 0; c < 3; ++c) v[c] = (fh[c] - cdt * acc[c] * iwj) * ir;
        if (sk.scheme == 1) {
            // the lagged rotation -A^{-1} R u^k = -beta J u^k belongs to the
            // right-hand side F - R u^k, so it comes with Fh only
            if (uk && Fh) {
                v[0] += beta * ukv[1];
                v[1] -= beta * ukv[0];
            }
            wv[0] = v[0];
            wv[1] = v[1];
            wv[2] = v[2];
        } else {
            const R si = (R)sk.rot_si;
            wv[0] = si * (v[0] + beta * v[1]);
            wv[1] = si * (-beta * v[0] + v[1]);
            wv[2] = v[2];
        }
        for (int c = 0; c < 3; ++c) {
            w[c * fs + e * NP + node] = wv[c];
            s_w[le][c][node] = wv[c];
        }
    }
    if (!FB) return;
    __syncthreads();
    // face buffers: (rho h)^k (w . nS) on this element's side of every face
    const R hfac = (R)sk.hfac;
    if (!slow) {
        if (act)
            for (int it = node; it < 6 * NF; it += NP) {
                const int f = it / NF, pt = it - f * NF, d = f >> 1, s = f & 1;
                if (g.kind[e * 6 + f] == WALL) continue;
                R nS[3];
                area<N>(g, T, e, f, pt, nS);
                const R hk = face_value<N>(&s_pk[le][0], T.f[s], d, pt);
                const R w0 = face_value<N>(&s_w[le][0][0], T.f[s], d, pt);
                const R w1 = face_value<N>(&s_w[le][1][0], T.f[s], d, pt);
                const R w2 = face_value<N>(&s_w[le][2][0], T.f[s], d, pt);
                FB[((size_t)e * 6 + f) * NF + pt] = fb_value<R>(hfac, hk, w0, w1, w2, nS);
            }
        return;
    }
    R* s_own = U;   // [4][NF]
    for (int f = 0; f < 6; ++f) {
        const int d = f >> 1, s = f & 1;
        const int kind = act ? g.kind[e * 6 + f] : -1;
        const int nbr = act ? g.nbr[e * 6 + f] : 0;
        if (act && node < NF) {
            s_own[node] = face_value<N>(&s_pk[le][0], T.f[s], d, node);
            for (int c = 0; c < 3; ++c) s_own[(1 + c) * NF + node] = face_value<N>(&s_w[le][c][0], T.f[s], d, node);
        }
        __syncthreads();
        if (act && kind != WALL) {
            const int nit = kind == COARSE ? 4 * NF : NF;
            for (int it = node; it < nit; it += NP) {
                const int hs = it / NF, pt = it - hs * NF;
                R nS[3], vals[4];
                if (kind == COARSE) {
                    const int fn = g.hang[nbr * 4 + hs];
                    for (int t = 0; t < 4; ++t) vals[t] = sub_interp<N>(s_own + t * NF, T, hs, pt);
                    area<N>(g, T, fn, f ^ 1, pt, nS);
                    for (int c = 0; c < 3; ++c) nS[c] = -nS[c];
                    FBh[((size_t)nbr * 4 + hs) * NF + pt] = fb_value<R>(hfac, vals[0], vals[1], vals[2], vals[3], nS);
                } else {
                    for (int t = 0; t < 4; ++t) vals[t] = s_own[t * NF + pt];
                    area<N>(g, T, e, f, pt, nS);
                    FB[((size_t)e * 6 + f) * NF + pt] = fb_value<R>(hfac, vals[0], vals[1], vals[2], vals[3], nS);
                }
            }
        }
        __syncthreads();
    }
}

// =====================================================================
// Schur pass 2: out = alpha (Gp - p/(gamma-1) - M^{-1} C^k w - [R2] M^{-1} M_g w)
// =====================================================================
template <int N, typename R, bool SLOW>
__global__ void __launch_bounds__(threads_of(N))
k_pass2(const int* __restrict__ elist, int64_t nel, const R* __restrict__ Gp, const R* __restrict__ p,
        const R* __restrict__ pscale, const R* __restrict__ w, const R* __restrict__ pk, const R* __restrict__ rho,
        const R* __restrict__ FB, const R* __restrict__ FBh, R* __restrict__ out, R alpha, int dual, Geom<R> g,
        const Tab<N, R>* __restrict__ Tg, StageK sk, const R* __restrict__ V, int nv, int64_t ldv,
        double* __restrict__ partial, const int* __restrict__ ctrl) {
    if (ctrl && *ctrl != 0) return;
    constexpr int NP = N * N * N, NF = N * N, EPB = epb_of(N);
    constexpr int L_FACE = SLOW ? 5 * NF : 6 * NF;
    __shared__ R s_face[EPB][L_FACE];
    __shared__ R s_vol[EPB][3][NP];
    const int tid = threadIdx.x, le = elem_slot<NP>(tid), node = tid - le * NP;
    __shared__ Tab<N, R> T;
    load_tab<N, R>(Tg, &T);
    const int64_t slot = xcd_block(blockIdx.x, gridDim.x) * EPB + le;
    const bool act = le < EPB && slot < nel;
    const int64_t e = act ? (elist ? (int64_t)elist[slot] : slot) : 0;
    const size_t fs = (size_t)g.E * NP;
    const R gam = (R)sk.gamma;
    R* U = &s_face[le][0];
    // all global loads first: own fields, and (fast path) both sides' face fluxes
    R wv[3] = {0, 0, 0}, wj = 1, rh = 0, rl = 0, gp = 0, pv = 0;
    if (act) {
        wj = g.WJ[e * NP + node];
        for (int c = 0; c < 3; ++c) wv[c] = w[c * fs + e * NP + node];
        rh = (R)sk.hfac * pk[e * NP + node];
        if (sk.scheme == 2) rl = rho[e * NP + node];
        if (Gp) gp = Gp[e * NP + node];
        if (p) pv = (pscale ? pscale[0] : (R)1) * p[e * NP + node];
        if (!SLOW)
            for (int it = node; it < 6 * NF; it += NP) {
                const int f = it / NF, pt = it - f * NF;
                const int kind = g.kind[e * 6 + f];
                R v = 0;
                if (kind == CONF) {
                    const int nbr = g.nbr[e * 6 + f];
                    v = (R)0.5 * (FB[((size_t)e * 6 + f) * NF + pt] - FB[((size_t)nbr * 6 + (f ^ 1)) * NF + pt]);
                } else if (kind == FINE) {
                    const int aux = g.aux[e * 6 + f];
                    v = (R)0.5 * (FB[((size_t)e * 6 + f) * NF + pt] -
                                  FBh[((size_t)(aux >> 2) * 4 + (aux & 3)) * NF + pt]);
                }
                U[f * NF + pt] = v;
            }
        // contravariant (rho h)^k w for the volume term
        for (int dd = 0; dd < 3; ++dd) {
            R v = 0;
            for (int c = 0; c < 3; ++c) v += metric<N>(g, e, node, dd, c, wj) * wv[c];
            s_vol[le][dd][node] = rh * v;
        }
    }
    __syncthreads();
    R acc = 0;
    if (!SLOW) {
        if (act)
            for (int f = 0; f < 6; ++f) {
                int m, pt;
                split_node<N>(f >> 1, node, m, pt);
                acc += T.f[f & 1][m] * U[f * NF + pt];
            }
    } else {
        R* s_fl = U;          // [NF]
        R* s_sub = U + NF;    // [4][NF]
        for (int f = 0; f < 6; ++f) {
            const int d = f >> 1, s = f & 1;
            const int kind = act ? g.kind[e * 6 + f] : -1;
            const int nbr = act ? g.nbr[e * 6 + f] : 0;
            const int aux = act ? g.aux[e * 6 + f] : 0;
            if (act) {
                const int nit = kind == COARSE ? 4 * NF : NF;
                for (int it = node; it < nit; it += NP) {
                    const int hs = it / NF, pt = it - hs * NF;
                    if (kind == COARSE) {
                        const int fn = g.hang[nbr * 4 + hs];
                        s_sub[hs * NF + pt] = (R)0.5 * (FBh[((size_t)nbr * 4 + hs) * NF + pt] -
                                                        FB[((size_t)fn * 6 + (f ^ 1)) * NF + pt]);
                    } else if (kind == CONF) {
                        s_fl[pt] = (R)0.5 * (FB[((size_t)e * 6 + f) * NF + pt] - FB[((size_t)nbr * 6 + (f ^ 1)) * NF + pt]);
                    } else if (kind == FINE) {
                        s_fl[pt] = (R)0.5 * (FB[((size_t)e * 6 + f) * NF + pt] -
                                             FBh[((size_t)(aux >> 2) * 4 + (aux & 3)) * NF + pt]);
                    } else {
                        s_fl[pt] = 0;
                    }
                }
            }
            __syncthreads();
            if (act && kind == COARSE && node < NF) {
                R v = 0;
                for (int h = 0; h < 4; ++h) v += sub_interp_T<N>(s_sub + h * NF, T, h, node);
                s_fl[node] = v;
            }
            __syncthreads();
            if (act) {
                int m, pt;
                split_node<N>(d, node, m, pt);
                acc += T.f[s][m] * s_fl[pt];
            }
            __syncthreads();
        }
    }
    R res = 0;
    if (act) {
        acc -= div_T<N>(&s_vol[le][0][0], T, node);
        const R cdt = (R)sk.c_dt;
        res = gp;
        if (p) res -= pv * (R)sk.igm1;
        res -= cdt * acc / wj;
        if (sk.scheme == 2) res -= cdt * (R)sk.g * rl * wv[2];
        res *= alpha;
        out[e * NP + node] = dual ? res * wj : res;
    }
    if (!V) return;
    // fused Gram-Schmidt projections: partial sums of <V_i, out>_M (i < nv)
    // and <out, out>_M for this workgroup, in a fixed order
    __shared__ double s_red[threads_of(N) / 64][33];
    const double wz = act ? (double)wj * (double)res : 0.0;
    const int lane = tid & 63, wid = tid >> 6;
    for (int i0 = 0; i0 <= nv; i0 += 8) {
        double v[8];   // eight projections per batch so that their loads overlap
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = i0 + k;
            v[k] = i < nv ? (act ? wz * (double)V[(int64_t)i * ldv + e * NP + node] : 0.0)
                          : (i == nv ? wz * (double)res : 0.0);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
        if (lane == 0)
            for (int k = 0; k < 8; ++k)
                if (i0 + k <= nv) s_red[wid][i0 + k] = v[k];
    }
    __syncthreads();
    if (tid <= nv) {
        double t = 0;
        for (int k = 0; k < threads_of(N) / 64; ++k) t += s_red[k][tid];
        partial[(size_t)blockIdx.x * (nv + 1) + tid] = t;
    }
}

// =====================================================================
// Schur complement inside the Krylov loop: z = M^{-1} S (sc x). Specialised
// instances of passes 1 and 2 for the elements without a coarse hanging face:
// no right-hand side, the scheme and the geometry class (affine or
// isoparametric) fixed at compile time, one coefficient cr = 1/(W detJ rho_l)
// per node instead of W detJ and rho_l with two divisions, and on affine
// elements W detJ, the face areas and the metric formed from the tensor
// weights and the element's edge lengths instead of read per node.
// =====================================================================
template <int N, typename R, bool AFF>
struct ElemGeo {
    // scalar members (an array here would be indexed through scratch memory)
    R hi0 = 0, hi1 = 0, hi2 = 0, dJ = 0, idJ = 0, A0 = 0, A1 = 0, A2 = 0;
    __device__ __forceinline__ void load(const double* __restrict__ eg, int e) {
        if constexpr (AFF) {
            const double* q = eg + (size_t)e * 8;
            const double h0 = q[0], h1 = q[1], h2 = q[2];
            hi0 = (R)q[3];
            hi1 = (R)q[4];
            hi2 = (R)q[5];
            dJ = (R)q[6];
            idJ = (R)q[7];
            A0 = (R)(h1 * h2);   // area factor h_t1 h_t2 of the faces normal to x, y, z
            A1 = (R)(h0 * h2);
            A2 = (R)(h0 * h1);
        }
    }
    __device__ __forceinline__ R hi(int d) const { return d == 0 ? hi0 : (d == 1 ? hi1 : hi2); }
};

// Schur pass 1 inside the Krylov loop. From w it writes the face buffer
// (rho h)^k w . n dS and, in w[0], the element's own part of pass 2: its
// volume term c_dt (W detJ)^{-1} sum_d D_d^T (contravariant (rho h)^k w)_d
// minus, for R2, the gravity term c_dt g rho_l w_z; pass 2 then adds the
// pressure and face terms. rho (rho_l) is read only for R2 on
// terrain-following meshes.
template <int N, typename R, bool AFF, int SCH>
__global__ void __launch_bounds__(threads_mv(N))
k_mv1(const int* __restrict__ elist, int nel, const R* __restrict__ p, const R* __restrict__ pscale,
      const R* __restrict__ cr, const R* __restrict__ pk, const R* __restrict__ rho, R* __restrict__ w,
      R* __restrict__ FB, Geom<R> g, const Tab<N, R>* __restrict__ Tg, StageK sk, const int* __restrict__ ctrl) {
    if (ctrl && *ctrl != 0) return;   // the Krylov cycle has stopped
    constexpr int NP = N * N * N, NF = N * N, EPB = epb_mv(N);
    constexpr int NR = (6 * NF + NP - 1) / NP;   // face points per lane
    constexpr int LF = AFF ? 6 * NF : 18 * NF, LV = AFF ? NP : 3 * NP;
    __shared__ R s_p[EPB][NP];
    __shared__ R s_pk[EPB][NP];
    __shared__ R s_w[EPB][3][NP];
    __shared__ R s_u[EPB][LF > LV ? LF : LV];
    __shared__ R s_A[EPB][3];   // affine: face area factor h_t1 h_t2 per direction
    __shared__ R s_v[AFF ? EPB : 1][NP];   // affine: W detJ sc p for the volume term
    __shared__ Tab<N, R> T;
    load_tab<N, R>(Tg, &T);
    const int tid = threadIdx.x, le = elem_slot<NP>(tid), node = tid - le * NP;
    const int slot = (int)xcd_block(blockIdx.x, gridDim.x) * EPB + le;
    const bool act = le < EPB && slot < nel;
    const int e = act ? (elist ? elist[slot] : slot) : 0;
    const unsigned fs = (unsigned)g.E * NP, o = (unsigned)e * NP + node;
    const R sc = pscale ? pscale[0] : (R)1;
    R* U = &s_u[le][0];
    // all global loads before the first barrier: own values, the lane's face
    // table entries and the neighbour values along the normal
    R crv = 0, nbv[NR][N];
    int kf[NR], nf[NR];
    uint64_t fo[NR];   // this lane's face points: node offsets along the normal, face, point
    ElemGeo<N, R, AFF> eg;
    if (act) {
        s_p[le][node] = p[o];
        s_pk[le][node] = pk[o];
        crv = cr[o];
        eg.load(g.eg, e);
        if constexpr (AFF) {
            if (node < 3) s_A[le][node] = node == 0 ? eg.A0 : (node == 1 ? eg.A1 : eg.A2);
            // (the LDS copy of the tables is not visible before the first barrier)
            s_v[le][node] = (Tg->W3[node] * eg.dJ) * (sc * p[o]);
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            fo[r] = g.fofs[r * NP + node];
            const bool full = (r + 1) * NP <= 6 * NF;   // every lane has a point in this round
            const int f = fo_face(fo[r]);
            kf[r] = (full || f < 6) ? g.kind[e * 6 + f] : WALL;
            nf[r] = g.nbr[e * 6 + ((full || f < 6) ? f : 5)];
            const bool ld = kf[r] == CONF;
            const R* src = p + (size_t)(unsigned)(ld ? nf[r] : 0) * NP;
#pragma unroll
            for (int m = 0; m < N; ++m) nbv[r][m] = ld ? src[fo_node(fo[r], m)] : (R)0;
        }
    }
    __syncthreads();
    // {p} n dS at every face point
    if (act)
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int f = fo_face(fo[r]);
            if ((r + 1) * NP > 6 * NF && f >= 6) continue;
            const int pt = fo_point(fo[r]), d = f >> 1, s = f & 1;
            R vals[N];
#pragma unroll
            for (int m = 0; m < N; ++m) vals[m] = s_p[le][fo_node(fo[r], m)];
            const R pa = sc * trace_chain<N, R>(T.f[s], vals);
            R pb = pa;
            if (kf[r] == CONF) pb = sc * trace_chain<N, R>(T.f[1 - s], nbv[r]);
            else if (kf[r] == FINE)
                pb = sc * coarse_point<N>(p + (size_t)(unsigned)nf[r] * NP, T.f[1 - s], T, d, g.aux[e * 6 + f] & 3, pt);
            const R avg = (R)0.5 * (pa + pb);
            if constexpr (AFF) {
                const R Af = T.W2[pt] * s_A[le][d];
                U[f * NF + pt] = avg * (s ? Af : -Af);
            } else {
                {
                    R nS[3];
                    nS_gc<N, R>(g, e, f, pt, nS);
#pragma unroll
                    for (int c = 0; c < 3; ++c) U[(f * 3 + c) * NF + pt] = avg * nS[c];
                }
            }
        }
    // affine volume term (after the face points: their registers are free) -int (sc p) div(phi_c), from s_v
    R vol[3] = {0, 0, 0};
    if constexpr (AFF) {
        if (act) {
            const int i = node % N, j = (node / N) % N, k = node / (N * N);
            const R* Uv = &s_v[le][0];
#pragma unroll
            for (int q = 0; q < N; ++q) {
                vol[0] += T.D[q][i] * Uv[q + N * (j + N * k)];
                vol[1] += T.D[q][j] * Uv[i + N * (q + N * k)];
                vol[2] += T.D[q][k] * Uv[i + N * (j + N * q)];
            }
        }
    }
    __syncthreads();
    R acc[3] = {0, 0, 0};
    if (act) {
        if constexpr (AFF) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                int m, pt;
                split_node<N>(d, node, m, pt);
                acc[d] += T.f[0][m] * U[(2 * d) * NF + pt];
                acc[d] += T.f[1][m] * U[(2 * d + 1) * NF + pt];
            }
        } else {
            for (int f = 0; f < 6; ++f) {
                int m, pt;
                split_node<N>(f >> 1, node, m, pt);
                const R lf = T.f[f & 1][m];
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[c] += lf * U[(f * 3 + c) * NF + pt];
            }
        }
    }
    if constexpr (AFF) {
        if (act) {
            acc[0] -= vol[0] * eg.hi0;
            acc[1] -= vol[1] * eg.hi1;
            acc[2] -= vol[2] * eg.hi2;
        }
    } else {
        // volume: -int (sc p) div(phi_c), one metric row at a time through U
        __syncthreads();
        const R pv = act ? sc * s_p[le][node] : (R)0;
        for (int c = 0; c < 3; ++c) {
            if (act)
#pragma unroll
                for (int dd = 0; dd < 3; ++dd) U[dd * NP + node] = G_gc<R>(g, fs, dd, c, o) * pv;
            __syncthreads();
            if (act) acc[c] -= div_T<N>(U, T, node);
            __syncthreads();
        }
    }
    // w = (I + beta J)^{-1} A^{-1} (-B p) [R2] or A^{-1}(-B p) [R1]: (rho h)^k w
    // in registers for the own part of pass 2, w plain in LDS for this
    // element's face traces
    R hq[3] = {0, 0, 0}, wz = 0;   // (rho h)^k w, w_z
    if (act) {
        const R cdt = (R)sk.c_dt, beta = (R)sk.beta;
        R v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = -(cdt * acc[c]) * crv;
        R wv[3];
        if constexpr (SCH == 2) {
            const R si = (R)sk.rot_si;
            wv[0] = si * (v[0] + beta * v[1]);
            wv[1] = si * (-beta * v[0] + v[1]);
            wv[2] = v[2];
        } else {
            wv[0] = v[0];
            wv[1] = v[1];
            wv[2] = v[2];
        }
        const R rh = (R)sk.hfac * s_pk[le][node];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            hq[c] = rh * wv[c];
            s_w[le][c][node] = wv[c];
        }
        wz = wv[2];
    }
    __syncthreads();
    // face buffer: (rho h)^k (w . n dS) on this element's side of each face
    if (act) {
        const R hfac = (R)sk.hfac;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int f = fo_face(fo[r]);
            if (((r + 1) * NP > 6 * NF && f >= 6) || kf[r] == WALL) continue;
            const int pt = fo_point(fo[r]), d = f >> 1, s = f & 1;
            R vk[N];
#pragma unroll
            for (int m = 0; m < N; ++m) vk[m] = s_pk[le][fo_node(fo[r], m)];
            const R hk = hfac * trace_chain<N, R>(T.f[s], vk);
            R fbv;
            if constexpr (AFF) {
                R vw[N];
#pragma unroll
                for (int m = 0; m < N; ++m) vw[m] = s_w[le][d][fo_node(fo[r], m)];
                const R Af = T.W2[pt] * s_A[le][d];
                fbv = hk * (trace_chain<N, R>(T.f[s], vw) * (s ? Af : -Af));
            } else {
                R wn = 0, nS[3];
                nS_gc<N, R>(g, e, f, pt, nS);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    R vw[N];
#pragma unroll
                    for (int m = 0; m < N; ++m) vw[m] = s_w[le][c][fo_node(fo[r], m)];
                    wn += trace_chain<N, R>(T.f[s], vw) * nS[c];
                }
                fbv = hk * wn;
            }
            FB[(size_t)(unsigned)(e * 6 + f) * NF + pt] = fbv;
        }
    }
    {
        // the own-element part of pass 2 from the contravariant (rho h)^k w in
        // LDS (s_w is free once every lane has read its traces)
        __syncthreads();
        if (act) {
            if constexpr (AFF) {
                const R wj = T.W3[node] * eg.dJ;
                s_w[le][0][node] = (wj * eg.hi0) * hq[0];
                s_w[le][1][node] = (wj * eg.hi1) * hq[1];
                s_w[le][2][node] = (wj * eg.hi2) * hq[2];
            } else {
#pragma unroll
                for (int dd = 0; dd < 3; ++dd) {
                    R v = 0;
#pragma unroll
                    for (int c = 0; c < 3; ++c) v += G_gc<R>(g, fs, dd, c, o) * hq[c];
                    s_w[le][dd][node] = v;
                }
            }
        }
        __syncthreads();
        if (act) {
            const R dv = div_T<N>(&s_w[le][0][0], T, node);
            const R cdt = (R)sk.c_dt;
            R qv;
            if constexpr (AFF) {
                qv = cdt * dv * (T.iW3[node] * eg.idJ);
                if constexpr (SCH == 2) {
                    const R rho_l = (R)1 / (crv * (T.W3[node] * eg.dJ));   // cr = 1 / (W detJ rho_l)
                    qv -= cdt * (R)sk.g * (rho_l * wz);
                }
            } else {
                qv = cdt * dv * g.iWJ[o];
                if constexpr (SCH == 2) qv -= cdt * (R)sk.g * (rho[o] * wz);
            }
            w[o] = qv;
        }
    }
}

// Schur pass 1 inside the Krylov loop on terrain-following (Gal-Chen)
// elements. Same result as k_mv1 with AFF = false, organised for few
// synchronisation points: every global load (own fields, the five stored
// entries of W cof(J), 1 / W detJ, rho_l, this lane's face table entries, n dS
// of its face points and the neighbour values along the normal) is issued
// before the first barrier and kept in registers, and the volume pressure
// term uses the sparsity of W cof(J): -int p div(phi_c) is
// D_x^T(G00 p) + D_z^T(G20 p), D_y^T(G11 p) + D_z^T(G21 p) and D_z^T(G22 p),
// five 1D contractions staged together, instead of nine in three rounds.
// Four barriers in all.
template <int N, typename R, int SCH, bool CM>
__global__ void __launch_bounds__(threads_mv(N))
k_mv1_gc(const int* __restrict__ elist, int nel, const R* __restrict__ p, const R* __restrict__ pscale,
         const R* __restrict__ cr, const R* __restrict__ pk, const R* __restrict__ rho, R* __restrict__ w,
         R* __restrict__ FB, Geom<R> g, const Tab<N, R>* __restrict__ Tg, StageK sk, const int* __restrict__ ctrl) {
    if (ctrl && *ctrl != 0) return;   // the Krylov cycle has stopped
    constexpr int NP = N * N * N, NF = N * N, EPB = epb_mv(N);
    constexpr int NR = (6 * NF + NP - 1) / NP;   // face points per lane
    constexpr int LU = 18 * NF > 3 * NP ? 18 * NF : 3 * NP;
    __shared__ R s_p[EPB][NP];
    __shared__ R s_pk[EPB][NP];
    __shared__ R s_a[EPB][5][NP];   // G p (five entries), then w (three components)
    __shared__ R s_u[EPB][LU];      // {p} n dS per face point, then the contravariant (rho h)^k w
    __shared__ Tab<N, R> T;
    load_tab<N, R>(Tg, &T);
    const int tid = threadIdx.x, le = elem_slot<NP>(tid), node = tid - le * NP;
    const int slot = (int)xcd_block(blockIdx.x, gridDim.x) * EPB + le;
    const bool act = le < EPB && slot < nel;
    const int e = act ? (elist ? elist[slot] : slot) : 0;
    const unsigned fs = (unsigned)g.E * NP, o = (unsigned)e * NP + node;
    const R sc = pscale ? pscale[0] : (R)1;
    R* U = &s_u[le][0];
    R crv = 0, iwj = 0, rl = 0, gv[5] = {0, 0, 0, 0, 0}, nbv[NR][N], nsv[NR][3];
    int kf[NR], nf[NR];
    LanePoints<N, false> lp;
    if (act) {
        const R pv = p[o];
        s_p[le][node] = pv;
        s_pk[le][node] = pk[o];
        crv = cr[o];
        if constexpr (SCH == 2) rl = rho[o];
        R J00 = 0, J11 = 0;
        if constexpr (CM) {
            J00 = (R)g.h[3 * e];
            J11 = (R)g.h[3 * e + 1];
            cm_node<N, R>(g, Tg, e, node, J00, J11, gv, iwj);
        } else {
            iwj = g.iWJ[o];
#pragma unroll
            for (int t = 0; t < 5; ++t) gv[t] = g.G[t * fs + o];
        }
        lp.init(g.fofs, node);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const bool full = (r + 1) * NP <= 6 * NF;   // every lane has a point in this round
            const int f = lp.face(r);
            const bool has = full || f < 6;
            const int fc = has ? f : 5;
            kf[r] = has ? g.kind[e * 6 + fc] : WALL;
            nf[r] = g.nbr[e * 6 + fc];
            if constexpr (CM) cm_area<N, R>(g, Tg, e, J00, J11, fc, lp.point(r), nsv[r]);
            else nS_gc<N, R>(g, e, fc, lp.point(r), nsv[r]);
            const bool ld = kf[r] == CONF;
            const R* src = p + (size_t)(unsigned)(ld ? nf[r] : 0) * NP;
#pragma unroll
            for (int m = 0; m < N; ++m) nbv[r][m] = ld ? src[lp.off(r, m)] : (R)0;
        }
        const R pvs = sc * pv;
#pragma unroll
        for (int t = 0; t < 5; ++t) s_a[le][t][node] = gv[t] * pvs;
    }
    __syncthreads();
    // {p} n dS at every face point of the element
    if (act)
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int f = lp.face(r);
            if ((r + 1) * NP > 6 * NF && f >= 6) continue;
            const int pt = lp.point(r), d = f >> 1, s = f & 1;
            R vals[N];
#pragma unroll
            for (int m = 0; m < N; ++m) vals[m] = s_p[le][lp.off(r, m)];
            const R pa = sc * trace_chain<N, R>(T.f[s], vals);
            R pb = pa;
            if (kf[r] == CONF) pb = sc * trace_chain<N, R>(T.f[1 - s], nbv[r]);
            else if (kf[r] == FINE)
                pb = sc * coarse_point<N>(p + (size_t)(unsigned)nf[r] * NP, T.f[1 - s], T, d, g.aux[e * 6 + f] & 3, pt);
            const R avg = (R)0.5 * (pa + pb);
            // the n dS of an x- or y-face has only its own component (terrain-following
            // map; the other two are exactly zero, so the sum of the first two is that
            // component): one value there, three on the z-faces (lanes with f >= 4 only)
            const int c0 = f < 4 ? d : 0;
            U[(f * 3 + c0) * NF + pt] = avg * (f < 4 ? nsv[r][0] + nsv[r][1] : nsv[r][0]);
            if (f >= 4) {
                U[(f * 3 + 1) * NF + pt] = avg * nsv[r][1];
                U[(f * 3 + 2) * NF + pt] = avg * nsv[r][2];
            }
        }
    // volume: -int (sc p) div(phi_c) from the five metric-weighted pressures
    R vol[3] = {0, 0, 0};
    if (act) {
        const int i = node % N, j = (node / N) % N, k = node / (N * N);
        const R* A0 = &s_a[le][0][0];
        const R* A1 = &s_a[le][1][0];
        const R* A20 = &s_a[le][2][0];
        const R* A21 = &s_a[le][3][0];
        const R* A22 = &s_a[le][4][0];
        R x0 = 0, x1 = 0, z0 = 0, z1 = 0, z2 = 0;
#pragma unroll
        for (int q = 0; q < N; ++q) {
            x0 += T.D[q][i] * A0[q + N * (j + N * k)];
            x1 += T.D[q][j] * A1[i + N * (q + N * k)];
            const int zq = i + N * (j + N * q);
            z0 += T.D[q][k] * A20[zq];
            z1 += T.D[q][k] * A21[zq];
            z2 += T.D[q][k] * A22[zq];
        }
        vol[0] = x0 + z0;
        vol[1] = x1 + z1;
        vol[2] = z2;
    }
    __syncthreads();
    // w = (I + beta J)^{-1} A^{-1} (-B p) [R2] or A^{-1}(-B p) [R1]
    R hq[3] = {0, 0, 0}, wz = 0;
    if (act) {
        R acc[3] = {0, 0, 0};
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            int m, pt;
            split_node<N>(f >> 1, node, m, pt);
            const R lf = T.f[f & 1][m];
            if (f < 4) {
                acc[f >> 1] += lf * U[(f * 3 + (f >> 1)) * NF + pt];
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[c] += lf * U[(f * 3 + c) * NF + pt];
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] -= vol[c];
        const R cdt = (R)sk.c_dt, beta = (R)sk.beta;
        R v[3], wv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = -(cdt * acc[c]) * crv;
        if constexpr (SCH == 2) {
            const R si = (R)sk.rot_si;
            wv[0] = si * (v[0] + beta * v[1]);
            wv[1] = si * (-beta * v[0] + v[1]);
            wv[2] = v[2];
        } else {
            wv[0] = v[0];
            wv[1] = v[1];
            wv[2] = v[2];
        }
        const R rh = (R)sk.hfac * s_pk[le][node];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            hq[c] = rh * wv[c];
            s_a[le][c][node] = wv[c];
        }
        wz = wv[2];
    }
    __syncthreads();
    if (act) {
        // face buffer: (rho h)^k (w . n dS) on this element's side of each face
        const R hfac = (R)sk.hfac;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int f = lp.face(r);
            if (((r + 1) * NP > 6 * NF && f >= 6) || kf[r] == WALL) continue;
            const int pt = lp.point(r), s = f & 1;
            R vk[N];
#pragma unroll
            for (int m = 0; m < N; ++m) vk[m] = s_pk[le][lp.off(r, m)];
            const R hk = hfac * trace_chain<N, R>(T.f[s], vk);
            // x- and y-faces: the normal component of w only (as for {p} n dS above)
            const int c0 = f < 4 ? f >> 1 : 0;
            R vw[N];
#pragma unroll
            for (int m = 0; m < N; ++m) vw[m] = s_a[le][c0][lp.off(r, m)];
            R wn = trace_chain<N, R>(T.f[s], vw) * (f < 4 ? nsv[r][0] + nsv[r][1] : nsv[r][0]);
            if (f >= 4) {
#pragma unroll
                for (int c = 1; c < 3; ++c) {
#pragma unroll
                    for (int m = 0; m < N; ++m) vw[m] = s_a[le][c][lp.off(r, m)];
                    wn += trace_chain<N, R>(T.f[s], vw) * nsv[r][c];
                }
            }
            FB[(size_t)(unsigned)(e * 6 + f) * NF + pt] = hk * wn;
        }
        // contravariant (rho h)^k w for the own part of pass 2 (U is free:
        // every lane has lifted its face values before the last barrier)
        U[node] = gv[0] * hq[0];
        U[NP + node] = gv[1] * hq[1];
        U[2 * NP + node] = gv[2] * hq[0] + gv[3] * hq[1] + gv[4] * hq[2];
    }
    __syncthreads();
    if (act) {
        const R dv = div_T<N>(U, T, node);
        const R cdt = (R)sk.c_dt;
        R qv = cdt * dv * iwj;
        if constexpr (SCH == 2) qv -= cdt * (R)sk.g * (rl * wz);
        w[o] = qv;
    }
}

// Schur pass 2 inside the Krylov loop: qw[0] holds the element's own volume
// and gravity part formed by pass 1; the pressure and face terms are added.
// With ST (unrefined box meshes) the neighbour of each face comes from the
// element index instead of the face tables, which takes two dependent loads
// off the path to the neighbour's face buffer (orography box: 166 -> 127 us;
// the same change made Schur pass 1 slower, 400 -> 560 us, and is not used
// there).
template <int N, typename R, bool AFF, bool ST, bool CM>
__global__ void __launch_bounds__(threads_mv(N))
k_mv2(const int* __restrict__ elist, int nel, const R* __restrict__ p, const R* __restrict__ pscale,
      const R* __restrict__ qw, const R* __restrict__ FB,
      const R* __restrict__ FBh, R* __restrict__ out, int dual, Geom<R> g, const Tab<N, R>* __restrict__ Tg,
      StageK sk, const int* __restrict__ ctrl) {
    if (ctrl && *ctrl != 0) return;
    constexpr int NP = N * N * N, NF = N * N, EPB = epb_mv(N);
    constexpr int NR = (6 * NF + NP - 1) / NP;
    __shared__ R s_face[EPB][6 * NF];
    __shared__ Tab<N, R> T;
    load_tab<N, R>(Tg, &T);
    const int tid = threadIdx.x, le = elem_slot<NP>(tid), node = tid - le * NP;
    const int slot = (int)xcd_block(blockIdx.x, gridDim.x) * EPB + le;
    const bool act = le < EPB && slot < nel;
    const int e = act ? (elist ? elist[slot] : slot) : 0;
    const unsigned o = (unsigned)e * NP + node;
    R* U = &s_face[le][0];
    R pv = 0, qv = 0;   // scaled x, own part from pass 1
    R iwj = 0, wjd = 0;  // terrain-following: 1 / W detJ (and W detJ for the dual form), loaded up front
    ElemGeo<N, R, AFF> eg;
    if (act) {
        eg.load(g.eg, e);
        qv = qw[o];
        pv = (pscale ? pscale[0] : (R)1) * p[o];
        if constexpr (CM) {
            wjd = cm_wj<N, R>(g, Tg, e, node);
            iwj = (R)1 / wjd;
        } else if constexpr (!AFF) {
            iwj = g.iWJ[o];
            if (dual) wjd = g.WJ[o];
        }
        // {(rho h)^k w} . n dS from the two sides' face buffers
        LanePoints<N, ST> lp;
        lp.init(g.fofs, node);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int f = lp.face(r);
            if ((r + 1) * NP > 6 * NF && f >= 6) continue;
            const int pt = lp.point(r);
            int kind, nb;
            if constexpr (ST) {
                grid_nbr<R>(g, e, f, kind, nb);
            } else {
                kind = g.kind[e * 6 + f];
                nb = g.nbr[e * 6 + f];
            }
            R v = 0;
            if (kind == CONF) {
                v = (R)0.5 * (FB[(size_t)(unsigned)(e * 6 + f) * NF + pt] - FB[(size_t)(unsigned)(nb * 6 + (f ^ 1)) * NF + pt]);
            } else if (kind == FINE) {
                const int aux = g.aux[e * 6 + f];
                v = (R)0.5 * (FB[(size_t)(unsigned)(e * 6 + f) * NF + pt] -
                              FBh[(size_t)(unsigned)((aux >> 2) * 4 + (aux & 3)) * NF + pt]);
            }
            U[f * NF + pt] = v;
        }
    }
    __syncthreads();
    if (!act) return;
    R acc = 0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        int m, pt;
        split_node<N>(f >> 1, node, m, pt);
        acc += T.f[f & 1][m] * U[f * NF + pt];
    }
    if constexpr (AFF) iwj = T.iW3[node] * eg.idJ;
    const R cdt = (R)sk.c_dt;
    R res = -(pv * (R)sk.igm1);
    res -= cdt * acc * iwj;
    res += qv;
    // z = -res = M^{-1} S (sc x); the dual form is S (sc x) = -res W detJ
    if (dual) {
        const R wj = AFF ? T.W3[node] * eg.dJ : wjd;
        out[o] = -res * wj;
    } else {
        out[o] = -res;
    }
}

// =====================================================================
// Pass 2 for r = 3 on affine meshes without hanging faces: one wavefront per
// element (64 lanes = 4^3 nodes). Pass 1 has formed the element's own volume
// and gravity part, so this pass adds the pressure term and the face terms
// from the two sides' face buffers; the only LDS use is the basis tables and
// the only barrier the one after loading them. (Pass 1 in a wavefront form,
// with its traces taken through cross-lane permutes, measured slower than the
// LDS form above: 87 against 69 us on the 48,000-element channel.)
// =====================================================================
template <typename R>
struct Wave4 {
    int lane, ind[3];   // node index along x, y, z
    __device__ __forceinline__ explicit Wave4(int l) : lane(l) {
        ind[0] = l & 3;
        ind[1] = (l >> 2) & 3;
        ind[2] = l >> 4;
    }
    // face point (a + 4 b) of this lane's line in direction d
    __device__ __forceinline__ int point(int d) const {
        return d == 0 ? ind[1] + 4 * ind[2] : (d == 1 ? ind[0] + 4 * ind[2] : ind[0] + 4 * ind[1]);
    }
};

template <typename R>
__global__ void __launch_bounds__(256)
k_mv2w(int nel, const R* __restrict__ p, const R* __restrict__ pscale, const R* __restrict__ qw,
       const R* __restrict__ FB, R* __restrict__ out, int dual,
       Geom<R> g, const Tab<4, R>* __restrict__ Tg, StageK sk, const int* __restrict__ ctrl) {
    if (ctrl && *ctrl != 0) return;
    constexpr int NP = 64, NF = 16;
    __shared__ Tab<4, R> T;
    load_tab<4, R>(Tg, &T);
    __syncthreads();
    const int e = __builtin_amdgcn_readfirstlane((int)xcd_block(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    if (e >= nel) return;
    const Wave4<R> W(threadIdx.x & 63);
    const unsigned o = (unsigned)e * NP + W.lane;
    const R qv = qw[o];   // own volume and gravity part, from pass 1
    const R pv = (pscale ? pscale[0] : (R)1) * p[o];
    const double* q8 = g.eg + (size_t)e * 8;
    const R dJ = (R)q8[6], idJ = (R)q8[7];
    R uf[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int kind = g.kind[e * 6 + f], nb = g.nbr[e * 6 + f];
        const int pt = W.point(f >> 1);
        uf[f] = kind == CONF ? (R)0.5 * (FB[(size_t)(unsigned)(e * 6 + f) * NF + pt] -
                                         FB[(size_t)(unsigned)(nb * 6 + (f ^ 1)) * NF + pt])
                             : (R)0;
    }
    R acc = 0;
#pragma unroll
    for (int f = 0; f < 6; ++f) acc += T.f[f & 1][W.ind[f >> 1]] * uf[f];
    const R wj = T.W3[W.lane] * dJ;
    const R iwj = T.iW3[W.lane] * idJ;
    const R cdt = (R)sk.c_dt;
    R res = -(pv * (R)sk.igm1);
    res -= cdt * acc * iwj;
    res += qv;
    out[o] = dual ? -res * wj : -res;
}

// =====================================================================
// Picard refresh: Gp = G0h - M^{-1} Lambda^k - rho kappa^k [- R1 gravity lag]
// =====================================================================
// lambda/2 ((rho e)_A - (rho e)_B) dS with lambda = max(|u_A . n|, |u_B . n|):
// the unit normal's 1/dS cancels against dS
template <int N>
__device__ __forceinline__ double lambda_flux(const double* a, const double* b, const double* nS, double igm1) {
    const double unA = a[0] * nS[0] + a[1] * nS[1] + a[2] * nS[2];
    const double unB = b[0] * nS[0] + b[1] * nS[1] + b[2] * nS[2];
    const double lam = fmax(fabs(unA), fabs(unB));
    return 0.5 * lam * (a[3] - b[3]) * igm1;
}

template <int N, bool SLOW>
__global__ void __launch_bounds__(threads_of(N))
k_lambda(const int* __restrict__ elist, int64_t nel, const double* __restrict__ pk, const double* __restrict__ uk, const double* __restrict__ rho,
         const double* __restrict__ G0h, double* __restrict__ Gp, Geom<double> g,
         const Tab<N, double>* __restrict__ Tg, StageK sk) {
    using R = double;
    constexpr int NP = N * N * N, NF = N * N, EPB = epb_of(N);
    constexpr int L_FAST = 6 * NF, L_SLOW = 4 * NF + 4 * NF + NF + 4 * NF;
    constexpr int UN = L_FAST > L_SLOW ? L_FAST : L_SLOW;
    __shared__ R s_q[EPB][4][NP];
    __shared__ R s_u[EPB][UN];
    const int tid = threadIdx.x, le = elem_slot<NP>(tid), node = tid - le * NP;
    __shared__ Tab<N, R> T;
    load_tab<N, R>(Tg, &T);
    const int64_t slot = xcd_block(blockIdx.x, gridDim.x) * EPB + le;
    const bool act = le < EPB && slot < nel;
    const int64_t e = act ? (elist ? (int64_t)elist[slot] : slot) : 0;
    const size_t fs = (size_t)g.E * NP;
    const R igm1 = sk.igm1;
    R* U = &s_u[le][0];
    // fields 0..2: u^k, 3: p^k
    auto src = [&](int t) -> const R* { return t < 3 ? uk + t * fs : pk; };
    if (act)
        for (int t = 0; t < 4; ++t) s_q[le][t][node] = src(t)[e * NP + node];
    constexpr bool slow = SLOW;
    __syncthreads();
    R acc = 0;
    if (!slow) {
        if (act)
            for (int it = node; it < 6 * NF; it += NP) {
                const int f = it / NF, pt = it - f * NF, d = f >> 1, s = f & 1;
                const int kind = g.kind[e * 6 + f], nbr = g.nbr[e * 6 + f];
                R v = 0;
                if (kind != WALL) {
                    R a[4], b[4], nS[3];
                    for (int t = 0; t < 4; ++t) {
                        a[t] = face_value<N>(&s_q[le][t][0], T.f[s], d, pt);
                        b[t] = kind == CONF ? face_value<N>(src(t) + (size_t)nbr * NP, T.f[1 - s], d, pt)
                                            : coarse_point<N>(src(t) + (size_t)nbr * NP, T.f[1 - s], T, d,
                                                              g.aux[e * 6 + f] & 3, pt);
                    }
                    area<N>(g, T, e, f, pt, nS);
                    v = lambda_flux<N>(a, b, nS, igm1);
                }
                U[f * NF + pt] = v;
            }
        __syncthreads();
        if (act)
            for (int f = 0; f < 6; ++f) {
                int m, pt;
                split_node<N>(f >> 1, node, m, pt);
                acc += T.f[f & 1][m] * U[f * NF + pt];
            }
    } else {
        R* s_own = U;              // [4][NF]
        R* s_nb = U + 4 * NF;      // [4][NF]
        R* s_fl = U + 8 * NF;      // [NF]
        R* s_sub = U + 9 * NF;     // [4][NF]
        for (int f = 0; f < 6; ++f) {
            const int d = f >> 1, s = f & 1;
            const int kind = act ? g.kind[e * 6 + f] : -1;
            const int nbr = act ? g.nbr[e * 6 + f] : 0;
            const int aux = act ? g.aux[e * 6 + f] : 0;
            if (act && node < NF) {
                for (int t = 0; t < 4; ++t) s_own[t * NF + node] = face_value<N>(&s_q[le][t][0], T.f[s], d, node);
                if (kind == CONF || kind == FINE)
                    for (int t = 0; t < 4; ++t)
                        s_nb[t * NF + node] = face_value<N>(src(t) + (size_t)nbr * NP, T.f[1 - s], d, node);
            }
            __syncthreads();
            if (act) {
                const int nit = kind == COARSE ? 4 * NF : NF;
                for (int it = node; it < nit; it += NP) {
                    const int hs = it / NF, pt = it - hs * NF;
                    R a[4], b[4], nS[3];
                    if (kind == WALL) {
                        s_fl[pt] = 0;
                        continue;
                    }
                    if (kind == COARSE) {
                        const int fn = g.hang[nbr * 4 + hs];
                        for (int t = 0; t < 4; ++t) {
                            a[t] = sub_interp<N>(s_own + t * NF, T, hs, pt);
                            b[t] = face_value<N>(src(t) + (size_t)fn * NP, T.f[1 - s], d, pt);
                        }
                        area<N>(g, T, fn, f ^ 1, pt, nS);
                        for (int c = 0; c < 3; ++c) nS[c] = -nS[c];
                    } else {
                        for (int t = 0; t < 4; ++t) {
                            a[t] = s_own[t * NF + pt];
                            b[t] = kind == CONF ? s_nb[t * NF + pt] : sub_interp<N>(s_nb + t * NF, T, aux & 3, pt);
                        }
                        area<N>(g, T, e, f, pt, nS);
                    }
                    const R v = lambda_flux<N>(a, b, nS, igm1);
                    if (kind == COARSE) s_sub[hs * NF + pt] = v;
                    else s_fl[pt] = v;
                }
            }
            __syncthreads();
            if (act && kind == COARSE && node < NF) {
                R v = 0;
                for (int h = 0; h < 4; ++h) v += sub_interp_T<N>(s_sub + h * NF, T, h, node);
                s_fl[node] = v;
            }
            __syncthreads();
            if (act) {
                int m, pt;
                split_node<N>(d, node, m, pt);
                acc += T.f[s][m] * s_fl[pt];
            }
            __syncthreads();
        }
    }
    if (!act) return;
    const R iwj = g.deformed ? g.iWJ[e * NP + node] : T.iW3[node] * g.eg[e * 8 + 7];
    const R r = rho[e * NP + node];
    const R u0 = s_q[le][0][node], u1 = s_q[le][1][node], u2 = s_q[le][2][node];
    R res = G0h[e * NP + node] - sk.c_dt * acc * iwj - r * 0.5 * (u0 * u0 + u1 * u1 + u2 * u2);
    if (sk.scheme == 1) res -= sk.c_dt * sk.g * r * u2;
    Gp[e * NP + node] = res;
}

// ------------------------------------------------------------ launchers
template <typename R>
static const void* tab_ptr(const DevMesh& m);
template <>
const void* tab_ptr<double>(const DevMesh& m) { return m.tab; }
template <>
const void* tab_ptr<float>(const DevMesh& m) { return m.tabf; }

// =====================================================================
// Geostrophic imbalance of the x momentum (planetary-scale wave test,
// Sec. 4.2): per workgroup, sum of W detJ |(1/rho) dp/dx - f v| and of
// W detJ; dp/dx is the derivative of the element's own pressure polynomial
// at its nodes, sum_d (d xi_d / d x) sum_m l_m'(xi_i) p_m.
// =====================================================================
template <int N>
__global__ void __launch_bounds__(threads_of(N))
k_geo(int64_t nel, const double* __restrict__ q, Geom<double> g, const Tab<N, double>* __restrict__ Tg,
      double gm1, double fcor, double* __restrict__ partial) {
    using R = double;
    constexpr int NP = N * N * N, EPB = epb_of(N), NW = threads_of(N) / 64;
    __shared__ R s_p[EPB][NP];
    __shared__ R s_red[NW][2];
    __shared__ Tab<N, R> T;
    load_tab<N, R>(Tg, &T);
    const int tid = threadIdx.x, le = elem_slot<NP>(tid), node = tid - le * NP;
    const size_t fs = (size_t)g.E * NP;
    const int i = node % N, j = (node / N) % N, k = node / (N * N);
    R acc0 = 0, acc1 = 0;
    for (int64_t base = (int64_t)blockIdx.x * EPB; base < nel; base += (int64_t)gridDim.x * EPB) {
        const int64_t e = base + le;
        const bool act = le < EPB && e < nel;
        R rho = 1, v = 0, wj = 0;
        __syncthreads();   // the previous group's pressure has been read
        if (act) {
            const size_t o = (size_t)e * NP + node;
            rho = q[o];
            const R m0 = q[fs + o], m1 = q[2 * fs + o], m2 = q[3 * fs + o];
            s_p[le][node] = gm1 * (q[4 * fs + o] - (R)0.5 * (m0 * m0 + m1 * m1 + m2 * m2) / rho);
            v = m1 / rho;
            wj = g.WJ[o];
        }
        __syncthreads();
        if (act) {
            const R* P = &s_p[le][0];
            R dxi[3] = {0, 0, 0};
#pragma unroll
            for (int m = 0; m < N; ++m) {
                dxi[0] += T.D[i][m] * P[m + N * (j + N * k)];
                dxi[1] += T.D[j][m] * P[i + N * (m + N * k)];
                dxi[2] += T.D[k][m] * P[i + N * (j + N * m)];
            }
            R dpdx = 0;
#pragma unroll
            for (int d = 0; d < 3; ++d) dpdx += metric<N, R>(g, e, node, d, 0, wj) * dxi[d];
            dpdx /= wj;
            acc0 += wj * fabs(dpdx / rho - (R)fcor * v);
            acc1 += wj;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        acc0 += __shfl_xor(acc0, off, 64);
        acc1 += __shfl_xor(acc1, off, 64);
    }
    if ((tid & 63) == 0) {
        s_red[tid >> 6][0] = acc0;
        s_red[tid >> 6][1] = acc1;
    }
    __syncthreads();
    if (tid < 2) {
        R t = 0;
        for (int w = 0; w < NW; ++w) t += s_red[w][tid];
        partial[(size_t)blockIdx.x * 2 + tid] = t;
    }
}

// =====================================================================
// Vertical-slice model (Sec. 2, eq. vertical_slice): L2 projection onto
// fields constant in y within each element. One lane per y-line of nodes
// (field, element, k, i): the line becomes sum_j w_j f_j / sum_j w_j, the
// exact element mean in y of the degree-r polynomial.
// =====================================================================
template <int N>
__global__ void __launch_bounds__(256)
k_slice_project(int64_t nlines, double* __restrict__ q, const Tab<N, double>* __restrict__ Tg) {
    constexpr int NP = N * N * N;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < nlines; t += (int64_t)gridDim.x * 256) {
        const int64_t fe = t / (N * N);          // field * E + element
        const int ki = (int)(t - fe * (N * N)), k = ki / N, i = ki - k * N;
        double* base = q + fe * NP + i + N * N * k;
        double s = 0, ws = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            s += Tg->w[j] * base[N * j];
            ws += Tg->w[j];
        }
        const double m = s / ws;
#pragma unroll
        for (int j = 0; j < N; ++j) base[N * j] = m;
    }
}

// The two element sets of a mesh with hanging faces write disjoint outputs:
// the face-by-face launch over the elements owning a coarse hanging face runs
// on the side stream, forked from and joined back into `st`, beside the
// all-faces launch over the others. Measured worth it for the explicit
// residual and the Picard refresh (face-by-face part of 70 us and more on the
// refined orography box), not for the Schur passes (12 to 32 us, less than
// the fork and join cost), which keep one stream (fork = false).
template <typename FF, typename SF>
static void fork_join(const DevMesh& m, hipStream_t st, FF&& fast, SF&& slow, bool fork = true) {
    if (fork && m.ncoarse && m.side) {
        (void)hipEventRecord(m.fork, st);
        (void)hipStreamWaitEvent(m.side, m.fork, 0);
        slow(m.side);
        fast(st);
        (void)hipEventRecord(m.join, m.side);
        (void)hipStreamWaitEvent(st, m.join, 0);
    } else {
        fast(st);
        if (m.ncoarse) slow(st);
    }
}

// Launches kern over all elements, or (meshes with hanging faces) the
// face-by-face instance over the elements owning a coarse hanging face and
// the all-faces instance over the others.
template <int N, bool FORK, typename KF, typename KS, typename... Args>
static void launch_split(const DevMesh& m, KF fast, KS slow, hipStream_t st, Args... args) {
    constexpr int EPB = epb_of(N);
    auto go = [&](auto kern, const int* list, int64_t n, hipStream_t s) {
        if (n <= 0) return;
        const int64_t nb = (n + EPB - 1) / EPB;
        hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(threads_of(N)), 0, s, list, n, args...);
    };
    fork_join(
        m, st, [&](hipStream_t s) { go(fast, m.ncoarse ? m.reg_list : nullptr, m.E - m.ncoarse, s); },
        [&](hipStream_t s) { go(slow, m.crs_list, m.ncoarse, s); }, FORK);
}

#define IMX_DISPATCH_N(n, CALL) \
    switch (n) {                 \
        case 2: CALL(2); break;  \
        case 3: CALL(3); break;  \
        case 4: CALL(4); break;  \
        case 5: CALL(5); break;  \
    }

template <typename R>
void launch_explicit(const DevMesh& m, const HostTab&, const PhysK& ph, const R* q, R* fNS, R* fS,
                     hipStream_t st) {
#define CALL(NN)                                                                                               \
    do {                                                                                                       \
        const Tab<NN, R>* tb = (const Tab<NN, R>*)tab_ptr<R>(m);                                                \
        if (m.deformed && m.ncoarse)                                                                           \
            launch_split<NN, true>(m, k_explicit_gc<NN, R, true>, k_explicit<NN, R, true, false>, st, q, fNS, fS, \
                                   geom<R>(m), tb, ph, m.sponge);                                              \
        else if (m.deformed)                                                                                   \
            launch_split<NN, true>(m, k_explicit_gc<NN, R, false>, k_explicit<NN, R, true, false>, st, q, fNS, fS, \
                                   geom<R>(m), tb, ph, m.sponge);                                              \
        else if (m.ncoarse)                                                                                    \
            launch_split<NN, true>(m, k_explicit<NN, R, false, true, true>, k_explicit<NN, R, true, true>, st, q, \
                                   fNS, fS, geom<R>(m), tb, ph, m.sponge);                                     \
        else                                                                                                   \
            launch_split<NN, true>(m, k_explicit<NN, R, false, true, false>, k_explicit<NN, R, true, true>, st, q, \
                                   fNS, fS, geom<R>(m), tb, ph, m.sponge);                                     \
    } while (0)
    IMX_DISPATCH_N(m.n, CALL)
#undef CALL
}
template void launch_explicit<double>(const DevMesh&, const HostTab&, const PhysK&, const double*, double*,
                                      double*, hipStream_t);

template <typename R>
void launch_pass1(const DevMesh& m, const HostTab&, const StageK& sk, const R* p, const R* pscale,
                  const R* Fh, const R* rho, const R* pk, const R* uk, R* w, R* FB, R* FBh, hipStream_t st) {
#define CALL(NN)                                                                                         \
    launch_split<NN, false>(m, k_pass1<NN, R, false>, k_pass1<NN, R, true>, st, p, pscale, Fh, rho, pk, uk, w, FB, \
                     FBh, geom<R>(m), (const Tab<NN, R>*)tab_ptr<R>(m), sk, (const int*)nullptr)
    IMX_DISPATCH_N(m.n, CALL)
#undef CALL
}
template void launch_pass1<double>(const DevMesh&, const HostTab&, const StageK&, const double*, const double*,
                                   const double*, const double*, const double*, const double*, double*, double*,
                                   double*, hipStream_t);
template void launch_pass1<float>(const DevMesh&, const HostTab&, const StageK&, const float*, const float*,
                                  const float*, const float*, const float*, const float*, float*, float*, float*,
                                  hipStream_t);

template <typename R, int N>
static void pass2_n(const DevMesh& m, const StageK& sk, const R* Gp, const R* p, const R* pscale, const R* w,
                    const R* pk, const R* rho, const R* FB, const R* FBh, R* out, double alpha, int dual,
                    const R* V, int nv, double* partial, double* dots, hipStream_t st) {
    constexpr int EPB = epb_of(N);
    const Tab<N, R>* T = (const Tab<N, R>*)tab_ptr<R>(m);
    const int64_t L = m.Lp;
    const int64_t nf = m.ncoarse ? m.E - m.ncoarse : m.E, ns = m.ncoarse;
    const int64_t bf = (nf + EPB - 1) / EPB, bs = (ns + EPB - 1) / EPB;
    fork_join(
        m, st,
        [&](hipStream_t s) {
            if (bf > 0)
                hipLaunchKernelGGL((k_pass2<N, R, false>), dim3((unsigned)bf), dim3(threads_of(N)), 0, s,
                                   m.ncoarse ? m.reg_list : nullptr, nf, Gp, p, pscale, w, pk, rho, FB, FBh, out,
                                   (R)alpha, dual, geom<R>(m), T, sk, V, nv, L, partial, (const int*)nullptr);
        },
        [&](hipStream_t s) {
            if (bs > 0)
                hipLaunchKernelGGL((k_pass2<N, R, true>), dim3((unsigned)bs), dim3(threads_of(N)), 0, s, m.crs_list,
                                   ns, Gp, p, pscale, w, pk, rho, FB, FBh, out, (R)alpha, dual, geom<R>(m), T, sk, V,
                                   nv, L, partial ? partial + (size_t)bf * (nv + 1) : nullptr, (const int*)nullptr);
        },
        false);
    if (V) launch_final_sum(partial, (int)(bf + bs), nv + 1, dots, st);
}

template <typename R>
void launch_pass2(const DevMesh& m, const HostTab&, const StageK& sk, const R* Gp, const R* p,
                  const R* pscale, const R* w, const R* pk, const R* rho, const R* FB, const R* FBh, R* out,
                  double alpha, int dual, hipStream_t st, const R* V, int nv, double* partial, double* dots) {
#define CALL(NN) pass2_n<R, NN>(m, sk, Gp, p, pscale, w, pk, rho, FB, FBh, out, alpha, dual, V, nv, partial, dots, st)
    IMX_DISPATCH_N(m.n, CALL)
#undef CALL
}
template void launch_pass2<double>(const DevMesh&, const HostTab&, const StageK&, const double*, const double*,
                                   const double*, const double*, const double*, const double*, const double*,
                                   const double*, double*, double, int, hipStream_t, const double*, int, double*,
                                   double*);
template void launch_pass2<float>(const DevMesh&, const HostTab&, const StageK&, const float*, const float*,
                                  const float*, const float*, const float*, const float*, const float*,
                                  const float*, float*, double, int, hipStream_t, const float*, int, double*,
                                  double*);

template <typename R, int N, bool AFF, int SCH, bool CM>
static void mv_n(const DevMesh& m, const StageK& sk, const R* x, const R* xs, const R* cr, const R* rho,
                 const R* pk, R* w, R* FB, R* FBh, R* out, int dual, hipStream_t st, const int* ctrl) {
    constexpr int EPB = epb_of(N), EPBM = epb_mv(N);
    const Tab<N, R>* T = (const Tab<N, R>*)tab_ptr<R>(m);
    const int64_t nf = m.ncoarse ? m.E - m.ncoarse : m.E, ns = m.ncoarse;
    const int64_t bf = (nf + EPBM - 1) / EPBM, bs = (ns + EPB - 1) / EPB;
    const int* fl = m.ncoarse ? m.reg_list : nullptr;
    if (!out) {
        fork_join(
            m, st,
            [&](hipStream_t s) {
                if (bf > 0) {
                    if constexpr (AFF)
                        hipLaunchKernelGGL((k_mv1<N, R, AFF, SCH>), dim3((unsigned)bf), dim3(threads_mv(N)), 0, s,
                                           fl, (int)nf, x, xs, cr, pk, rho, w, FB, geom<R>(m), T, sk, ctrl);
                    else
                        hipLaunchKernelGGL((k_mv1_gc<N, R, SCH, CM>), dim3((unsigned)bf), dim3(threads_mv(N)), 0, s, fl,
                                           (int)nf, x, xs, cr, pk, rho, w, FB, geom<R>(m), T, sk, ctrl);
                }
            },
            [&](hipStream_t s) {
                if (bs > 0)
                    hipLaunchKernelGGL((k_pass1<N, R, true>), dim3((unsigned)bs), dim3(threads_of(N)), 0, s,
                                       m.crs_list, ns, x, xs, (const R*)nullptr, rho, pk, (const R*)nullptr, w, FB,
                                       FBh, geom<R>(m), T, sk, ctrl);
            },
            false);
    } else {
        fork_join(
            m, st,
            [&](hipStream_t s) {
                if (bf > 0) {
                    if (m.structured)
                        hipLaunchKernelGGL((k_mv2<N, R, AFF, true, CM>), dim3((unsigned)bf), dim3(threads_mv(N)), 0, s,
                                           fl, (int)nf, x, xs, (const R*)w, (const R*)FB, (const R*)FBh, out, dual,
                                           geom<R>(m), T, sk, ctrl);
                    else
                        hipLaunchKernelGGL((k_mv2<N, R, AFF, false, CM>), dim3((unsigned)bf), dim3(threads_mv(N)), 0, s,
                                           fl, (int)nf, x, xs, (const R*)w, (const R*)FB, (const R*)FBh, out, dual,
                                           geom<R>(m), T, sk, ctrl);
                }
            },
            [&](hipStream_t s) {
                if (bs > 0)
                    hipLaunchKernelGGL((k_pass2<N, R, true>), dim3((unsigned)bs), dim3(threads_of(N)), 0, s,
                                       m.crs_list, ns, (const R*)nullptr, x, xs, (const R*)w, pk, rho, (const R*)FB,
                                       (const R*)FBh, out, (R)-1.0, dual, geom<R>(m), T, sk, (const R*)nullptr, 0,
                                       (int64_t)0, (double*)nullptr, ctrl);
            },
            false);
    }
}

template <typename R>
static void mv2w(const DevMesh& m, const StageK& sk, const R* x, const R* xs, const R* qw, const R* FB, R* out,
                 int dual, hipStream_t st, const int* ctrl) {
    const Tab<4, R>* T = (const Tab<4, R>*)tab_ptr<R>(m);
    const unsigned nb = (unsigned)((m.E + 3) / 4);
    hipLaunchKernelGGL((k_mv2w<R>), dim3(nb), dim3(256), 0, st, (int)m.E, x, xs, qw, FB, out, dual, geom<R>(m),
                       T, sk, ctrl);
}

template <typename R>
static void mv_dispatch(const DevMesh& m, const StageK& sk, const R* x, const R* xs, const R* cr, const R* rho,
                        const R* pk, R* w, R* FB, R* FBh, R* out, int dual, hipStream_t st, const int* ctrl) {
    // r = 3, affine, no hanging faces: pass 2 runs one element per wavefront
    if (out && m.n == 4 && !m.deformed && m.nh == 0) {
        mv2w<R>(m, sk, x, xs, w, FB, out, dual, st, ctrl);
        return;
    }
    // terrain-following meshes without hanging faces form their metric from the compact form
    const bool cm = geom<R>(m).cm != nullptr;
#define MV(NN)                                                                                            \
    do {                                                                                                  \
        if (!m.deformed) {                                                                                \
            if (sk.scheme == 2) mv_n<R, NN, true, 2, false>(m, sk, x, xs, cr, rho, pk, w, FB, FBh, out, dual, st, ctrl); \
            else mv_n<R, NN, true, 1, false>(m, sk, x, xs, cr, rho, pk, w, FB, FBh, out, dual, st, ctrl);       \
        } else if (cm) {                                                                                  \
            if (sk.scheme == 2) mv_n<R, NN, false, 2, true>(m, sk, x, xs, cr, rho, pk, w, FB, FBh, out, dual, st, ctrl); \
            else mv_n<R, NN, false, 1, true>(m, sk, x, xs, cr, rho, pk, w, FB, FBh, out, dual, st, ctrl);       \
        } else {                                                                                          \
            if (sk.scheme == 2) mv_n<R, NN, false, 2, false>(m, sk, x, xs, cr, rho, pk, w, FB, FBh, out, dual, st, ctrl); \
            else mv_n<R, NN, false, 1, false>(m, sk, x, xs, cr, rho, pk, w, FB, FBh, out, dual, st, ctrl);      \
        }                                                                                                 \
    } while (0)
    IMX_DISPATCH_N(m.n, MV)
#undef MV
}

template <typename R>
void launch_mv1(const DevMesh& m, const StageK& sk, const R* x, const R* xs, const R* cr, const R* rho,
                const R* pk, R* w, R* FB, R* FBh, hipStream_t st, const int* ctrl) {
    mv_dispatch<R>(m, sk, x, xs, cr, rho, pk, w, FB, FBh, nullptr, 0, st, ctrl);
}
template <typename R>
void launch_mv2(const DevMesh& m, const StageK& sk, const R* x, const R* xs, const R* w, const R* pk,
                const R* rho, const R* FB, const R* FBh, R* out, int dual, hipStream_t st, const int* ctrl) {
    mv_dispatch<R>(m, sk, x, xs, (const R*)nullptr, rho, pk, (R*)w, (R*)FB, (R*)FBh, out, dual, st, ctrl);
}
template void launch_mv1<double>(const DevMesh&, const StageK&, const double*, const double*, const double*,
                                 const double*, const double*, double*, double*, double*, hipStream_t, const int*);
template void launch_mv1<float>(const DevMesh&, const StageK&, const float*, const float*, const float*,
                                const float*, const float*, float*, float*, float*, hipStream_t, const int*);
template void launch_mv2<double>(const DevMesh&, const StageK&, const double*, const double*, const double*,
                                 const double*, const double*, const double*, const double*, double*, int,
                                 hipStream_t, const int*);
template void launch_mv2<float>(const DevMesh&, const StageK&, const float*, const float*, const float*,
                                const float*, const float*, const float*, const float*, float*, int, hipStream_t,
                                const int*);

size_t pass2_partial_count(const DevMesh& m) {
    const int e = m.n == 2 ? 16 : (m.n == 3 ? 9 : (m.n == 4 ? 4 : 2));
    const int64_t nf = m.ncoarse ? m.E - m.ncoarse : m.E;
    return (size_t)((nf + e - 1) / e + (m.ncoarse + e - 1) / e) * 33;
}

void launch_lambda(const DevMesh& m, const HostTab&, const StageK& sk, const double* pk, const double* uk,
                   const double* rho, const double* G0h, double* Gp, hipStream_t st) {
#define CALL(NN)                                                                                    \
    launch_split<NN, true>(m, k_lambda<NN, false>, k_lambda<NN, true>, st, pk, uk, rho, G0h, Gp, geom<double>(m), \
                     (const Tab<NN, double>*)m.tab, sk)
    IMX_DISPATCH_N(m.n, CALL)
#undef CALL
}

void launch_slice_project(const DevMesh& m, double* q, hipStream_t st) {
#define CALL(NN)                                                                                         \
    do {                                                                                                 \
        const int64_t nl = 5 * m.E * NN * NN;                                                            \
        int64_t g = (nl + 255) / 256;                                                                    \
        if (g > 8192) g = 8192;                                                                          \
        hipLaunchKernelGGL(k_slice_project<NN>, dim3((unsigned)g), dim3(256), 0, st, nl, q,               \
                           (const Tab<NN, double>*)m.tab);                                              \
    } while (0)
    IMX_DISPATCH_N(m.n, CALL)
#undef CALL
}

int launch_geo(const DevMesh& m, const double* q, double gm1, double fcor, double* partial, int max_blocks,
               hipStream_t st) {
    int nb = 0;
#define CALL(NN)                                                                                          \
    do {                                                                                                  \
        const int64_t groups = (m.E + epb_of(NN) - 1) / epb_of(NN);                                      \
        nb = (int)(groups < max_blocks ? groups : max_blocks);                                            \
        if (nb < 1) nb = 1;                                                                               \
        hipLaunchKernelGGL(k_geo<NN>, dim3((unsigned)nb), dim3(threads_of(NN)), 0, st, (int64_t)m.E, q,  \
                           geom<double>(m), (const Tab<NN, double>*)m.tab, gm1, fcor, partial);          \
    } while (0)
    IMX_DISPATCH_N(m.n, CALL)
#undef CALL
    return nb;
}

}  // namespace imx
