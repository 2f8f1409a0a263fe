// Solution transfer between two refinements of one base grid (dynamic
// adaptivity of the statically refined meshes of Sec. 4.3): leaves present
// in both meshes are copied, a new leaf inside an old coarser leaf takes the
// old polynomial at its nodes (exact), a new leaf covering old finer leaves
// takes the L2 projection of the old solution with the mass-matrix
// quadrature (W detJ at the nodes), which keeps the integral of every field.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "internal.hpp"

namespace imx {

// Source of a new leaf: an old leaf and how it relates to the new one.
// code bits: 0-1 kind (0 same, 1 old is coarser: evaluate, 2 old is finer:
// project), 2-3 level difference k (1 or 2), 4-5 / 6-7 / 8-9 position of the
// finer leaf inside the coarser along x / y / z (0 .. 2^k - 1).
enum { SRC_SAME = 0, SRC_COARSER = 1, SRC_FINER = 2 };

struct TransferPlan {
    std::vector<int> off;    // [E_to + 1] into elem / code
    std::vector<int> elem;   // old leaf
    std::vector<int> code;
};

using LeafKey = std::tuple<int, int, int, int, int, int, int>;   // base xyz, level, sub xyz

static LeafKey key_of(const Mesh& m, int64_t e) {
    return LeafKey(m.base[3 * e], m.base[3 * e + 1], m.base[3 * e + 2], m.level[e], m.sub[3 * e],
                   m.sub[3 * e + 1], m.sub[3 * e + 2]);
}

static bool same_grid(const Mesh& a, const Mesh& b) {
    const imx_mesh_desc &da = a.desc, &db = b.desc;
    return da.Lx == db.Lx && da.Ly == db.Ly && da.Lz == db.Lz && da.nx == db.nx && da.ny == db.ny &&
           da.nz == db.nz && da.degree == db.degree && da.periodic_x == db.periodic_x &&
           da.periodic_y == db.periodic_y && da.terrain == db.terrain && da.h0 == db.h0 && da.a == db.a &&
           da.xc == db.xc && da.yc == db.yc;
}

static imx_status build_plan(const Mesh& from, const Mesh& to, TransferPlan& p) {
    std::map<LeafKey, int> index;
    for (int64_t e = 0; e < from.E; ++e) index[key_of(from, e)] = (int)e;
    // old leaves per base cell, for the coarsening search
    std::map<std::tuple<int, int, int>, std::vector<int>> by_base;
    for (int64_t e = 0; e < from.E; ++e)
        by_base[std::make_tuple(from.base[3 * e], from.base[3 * e + 1], from.base[3 * e + 2])].push_back((int)e);
    p.off.assign(to.E + 1, 0);
    p.elem.clear();
    p.code.clear();
    for (int64_t t = 0; t < to.E; ++t) {
        const int* b = &to.base[3 * t];
        const int lt = to.level[t];
        const int* st = &to.sub[3 * t];
        bool done = false;
        for (int lf = lt; lf >= 0 && !done; --lf) {
            const int k = lt - lf;
            const int sf[3] = {st[0] >> k, st[1] >> k, st[2] >> k};
            auto it = index.find(LeafKey(b[0], b[1], b[2], lf, sf[0], sf[1], sf[2]));
            if (it == index.end()) continue;
            if (k > 2) return IMX_EINVAL;
            int code = k == 0 ? SRC_SAME : SRC_COARSER | (k << 2);
            for (int c = 0; c < 3; ++c) code |= (st[c] - (sf[c] << k)) << (4 + 2 * c);
            p.elem.push_back(it->second);
            p.code.push_back(code);
            done = true;
        }
        if (!done) {
            int found = 0;
            for (int e : by_base[std::make_tuple(b[0], b[1], b[2])]) {
                const int lf = from.level[e];
                if (lf <= lt) continue;
                const int k = lf - lt;
                const int* sf = &from.sub[3 * e];
                if ((sf[0] >> k) != st[0] || (sf[1] >> k) != st[1] || (sf[2] >> k) != st[2]) continue;
                if (k > 2) return IMX_EINVAL;
                int code = SRC_FINER | (k << 2);
                for (int c = 0; c < 3; ++c) code |= (sf[c] - (st[c] << k)) << (4 + 2 * c);
                p.elem.push_back(e);
                p.code.push_back(code);
                ++found;
            }
            if (!found) return IMX_EINVAL;
        }
        p.off[t + 1] = (int)p.elem.size();
    }
    return IMX_OK;
}

// T[(k - 1) * 4 + pos][i][a] = l_a((pos + x_i) / 2^k), k = 1, 2, pos < 2^k:
// the Lagrange polynomials of a coarser leaf at the nodes of the finer leaf
// at position pos, k levels down (8 tables of n x n).
static void fill_tables(const Basis1D& b, std::vector<double>& T) {
    const int n = b.n;
    T.assign((size_t)8 * n * n, 0.0);
    std::vector<double> val(n), der(n);
    for (int k = 1; k <= 2; ++k)
        for (int pos = 0; pos < (1 << k); ++pos)
            for (int i = 0; i < n; ++i) {
                lagrange(b.x, (pos + b.x[i]) / double(1 << k), val.data(), der.data());
                for (int a = 0; a < n; ++a) T[(((size_t)(k - 1) * 4 + pos) * n + i) * n + a] = val[a];
            }
}

// workspace layout (256-byte aligned parts)
struct TransferLayout {
    size_t off_off, elem_off, code_off, wjf_off, wjt_off, tab_off, total;
};
static TransferLayout transfer_layout(const Mesh& from, const Mesh& to, size_t nsrc) {
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    TransferLayout L{};
    size_t o = 0;
    L.off_off = o;
    o += al((to.E + 1) * sizeof(int));
    L.elem_off = o;
    o += al(nsrc * sizeof(int));
    L.code_off = o;
    o += al(nsrc * sizeof(int));
    L.wjf_off = o;
    o += al((size_t)from.E * from.Np * sizeof(double));
    L.wjt_off = o;
    o += al((size_t)to.E * to.Np * sizeof(double));
    L.tab_off = o;
    o += al((size_t)8 * from.n * from.n * sizeof(double));
    L.total = o;
    return L;
}

// One workgroup per new leaf, one lane per node.
template <int N>
__global__ void __launch_bounds__(128)
k_transfer(int64_t Eto, int64_t Efrom, int nfields, const int* __restrict__ off, const int* __restrict__ elem,
           const int* __restrict__ code, const double* __restrict__ wjf, const double* __restrict__ wjt,
           const double* __restrict__ tab, const double* __restrict__ qf, double* __restrict__ qt) {
    constexpr int NP = N * N * N;
    __shared__ double s_t[8 * N * N];
    __shared__ double s_u[NP];
    const int64_t t = blockIdx.x;
    const int lane = threadIdx.x;
    for (int i = lane; i < 8 * N * N; i += blockDim.x) s_t[i] = tab[i];
    const bool act = lane < NP;
    const int ix = lane % N, iy = (lane / N) % N, iz = lane / (N * N);
    const int s0 = off[t], s1 = off[t + 1];
    for (int f = 0; f < nfields; ++f) {
        const double* src = qf + (size_t)f * Efrom * NP;
        double acc = 0.0;
        bool proj = false;
        for (int s = s0; s < s1; ++s) {
            const int e = elem[s], c = code[s];
            const int kind = c & 3, k = (c >> 2) & 3;
            __syncthreads();   // the previous source's values are no longer read
            if (act) s_u[lane] = kind == SRC_FINER ? wjf[(size_t)e * NP + lane] * src[(size_t)e * NP + lane]
                                                   : src[(size_t)e * NP + lane];
            __syncthreads();
            if (!act) continue;
            if (kind == SRC_SAME) {
                acc = s_u[lane];
            } else {
                const double* Tx = s_t + ((k - 1) * 4 + ((c >> 4) & 3)) * N * N;
                const double* Ty = s_t + ((k - 1) * 4 + ((c >> 6) & 3)) * N * N;
                const double* Tz = s_t + ((k - 1) * 4 + ((c >> 8) & 3)) * N * N;
                if (kind == SRC_COARSER) {
                    // the old polynomial at this node: sum_abc u_abc l_a(x') l_b(y') l_c(z')
                    double v = 0.0;
                    for (int cc = 0; cc < N; ++cc) {
                        double vy = 0.0;
                        for (int bb = 0; bb < N; ++bb) {
                            double vx = 0.0;
#pragma unroll
                            for (int aa = 0; aa < N; ++aa) vx += Tx[ix * N + aa] * s_u[aa + N * (bb + N * cc)];
                            vy += Ty[iy * N + bb] * vx;
                        }
                        v += Tz[iz * N + cc] * vy;
                    }
                    acc = v;
                } else {
                    // projection: sum over the old nodes q of W detJ u(q) l_i(x_q)
                    proj = true;
                    double v = 0.0;
                    for (int cc = 0; cc < N; ++cc) {
                        double vy = 0.0;
                        for (int bb = 0; bb < N; ++bb) {
                            double vx = 0.0;
#pragma unroll
                            for (int aa = 0; aa < N; ++aa) vx += Tx[aa * N + ix] * s_u[aa + N * (bb + N * cc)];
                            vy += Ty[bb * N + iy] * vx;
                        }
                        v += Tz[cc * N + iz] * vy;
                    }
                    acc += v;
                }
            }
        }
        if (act) qt[(size_t)f * Eto * NP + (size_t)t * NP + lane] = proj ? acc / wjt[(size_t)t * NP + lane] : acc;
    }
}

}  // namespace imx

using namespace imx;

extern "C" {

imx_status imx_transfer_workspace_bytes(const imx_mesh* from, const imx_mesh* to, size_t* bytes) {
    if (!from || !to || !bytes) {
        set_error("imx_transfer_workspace_bytes: null argument");
        return IMX_EINVAL;
    }
    if (!same_grid(from->m, to->m)) {
        set_error("imx_transfer_workspace_bytes: meshes differ in box, base grid, degree or terrain");
        return IMX_EINVAL;
    }
    TransferPlan p;
    if (build_plan(from->m, to->m, p) != IMX_OK) {
        set_error("imx_transfer_workspace_bytes: refinement levels differ by more than 2");
        return IMX_EINVAL;
    }
    *bytes = transfer_layout(from->m, to->m, p.elem.size()).total;
    return IMX_OK;
}

imx_status imx_transfer_state(const imx_mesh* from, const imx_mesh* to, void* ws_dev, size_t ws_bytes,
                              const double* q_from_dev, double* q_to_dev, int nfields, void* hip_stream) {
    if (!from || !to || !ws_dev || !q_from_dev || !q_to_dev || nfields < 1) {
        set_error("imx_transfer_state: null argument or nfields < 1");
        return IMX_EINVAL;
    }
    if (((uintptr_t)ws_dev & 255) != 0) {
        set_error("imx_transfer_state: workspace must be 256-byte aligned");
        return IMX_EINVAL;
    }
    const Mesh &mf = from->m, &mt = to->m;
    if (!same_grid(mf, mt)) {
        set_error("imx_transfer_state: meshes differ in box, base grid, degree or terrain");
        return IMX_EINVAL;
    }
    TransferPlan p;
    if (build_plan(mf, mt, p) != IMX_OK) {
        set_error("imx_transfer_state: refinement levels differ by more than 2");
        return IMX_EINVAL;
    }
    const TransferLayout L = transfer_layout(mf, mt, p.elem.size());
    if (ws_bytes < L.total) {
        set_error("imx_transfer_state: workspace smaller than imx_transfer_workspace_bytes");
        return IMX_ENOMEM;
    }
    std::vector<double> tab;
    fill_tables(mf.basis, tab);
    hipStream_t st = (hipStream_t)hip_stream;
    char* ws = (char*)ws_dev;
    struct Up { size_t off; const void* src; size_t n; } ups[] = {
        {L.off_off, p.off.data(), p.off.size() * sizeof(int)},
        {L.elem_off, p.elem.data(), p.elem.size() * sizeof(int)},
        {L.code_off, p.code.data(), p.code.size() * sizeof(int)},
        {L.wjf_off, mf.WJ.data(), mf.WJ.size() * sizeof(double)},
        {L.wjt_off, mt.WJ.data(), mt.WJ.size() * sizeof(double)},
        {L.tab_off, tab.data(), tab.size() * sizeof(double)},
    };
    for (const Up& u : ups) {
        // synchronous with respect to the host buffers, which die with this call
        const hipError_t e = hipMemcpyAsync(ws + u.off, u.src, u.n, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) {
            set_error(std::string("imx_transfer_state: upload: ") + hipGetErrorString(e));
            return IMX_EHIP;
        }
    }
    if (hipStreamSynchronize(st) != hipSuccess) {
        set_error("imx_transfer_state: upload synchronisation failed");
        return IMX_EHIP;
    }
    const dim3 grid((unsigned)mt.E), block(128);
    auto* off = (const int*)(ws + L.off_off);
    auto* el = (const int*)(ws + L.elem_off);
    auto* co = (const int*)(ws + L.code_off);
    auto* wjf = (const double*)(ws + L.wjf_off);
    auto* wjt = (const double*)(ws + L.wjt_off);
    auto* tb = (const double*)(ws + L.tab_off);
    switch (mf.n) {
        case 2: hipLaunchKernelGGL(k_transfer<2>, grid, block, 0, st, mt.E, mf.E, nfields, off, el, co, wjf, wjt, tb, q_from_dev, q_to_dev); break;
        case 3: hipLaunchKernelGGL(k_transfer<3>, grid, block, 0, st, mt.E, mf.E, nfields, off, el, co, wjf, wjt, tb, q_from_dev, q_to_dev); break;
        case 4: hipLaunchKernelGGL(k_transfer<4>, grid, block, 0, st, mt.E, mf.E, nfields, off, el, co, wjf, wjt, tb, q_from_dev, q_to_dev); break;
        default: hipLaunchKernelGGL(k_transfer<5>, grid, block, 0, st, mt.E, mf.E, nfields, off, el, co, wjf, wjt, tb, q_from_dev, q_to_dev); break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("imx_transfer_state: launch: ") + hipGetErrorString(e));
        return IMX_EHIP;
    }
    return IMX_OK;
}

}  // extern "C"
