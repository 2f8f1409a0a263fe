// Streaming kernels: stage combinations of the ARK2 scheme and the Krylov
// vector work of GMRES (M-weighted multi-dot products, Gram-Schmidt updates,
// norms). Reductions write one partial per workgroup and are summed by a
// single workgroup in a fixed order, so every result is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"

namespace imx {

constexpr int TPB = 256;

static unsigned grid_for(int64_t L, int64_t per_block = TPB * 4) {
    int64_t g = (L + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (unsigned)g;
}

// block reduction of NV values held per thread; result in red[v] for thread 0 use
template <int NV>
__device__ __forceinline__ void block_sum(double* v, double* red) {
    // wavefront (64 lanes) butterfly, then across the 4 wavefronts of the block
#pragma unroll
    for (int i = 0; i < NV; ++i)
        for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
        for (int i = 0; i < NV; ++i) red[wid * NV + i] = v[i];
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0;
        for (int k = 0; k < TPB / 64; ++k) s += red[k * NV + threadIdx.x];
        red[TPB / 64 * NV + threadIdx.x] = s;
    }
    __syncthreads();
}

// final fixed-order sum of partials[nb][nv] -> out[nv], one workgroup per value
__global__ void k_final_sum(const double* __restrict__ partial, int nb, int nv, double* __restrict__ out,
                            const int* __restrict__ ctrl) {
    if (ctrl && *ctrl != 0) return;
    __shared__ double red[TPB];
    const int v = blockIdx.x;
    double s = 0;
    for (int b = threadIdx.x; b < nb; b += TPB) s += partial[(size_t)b * nv + v];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = TPB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[v] = red[0];
}

// p[b] summed over b = t, t + TPB, ... < nb in that order, with eight loads in
// flight (a plain loop waits for each load before the next)
__device__ __forceinline__ double strided_sum(const double* __restrict__ p, int t, int nb) {
    double sum = 0;
    int b = t;
    for (; b + 7 * TPB < nb; b += 8 * TPB) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = p[b + k * TPB];
#pragma unroll
        for (int k = 0; k < 8; ++k) sum += v[k];
    }
    for (; b + TPB < nb; b += 2 * TPB) {
        const double v0 = p[b], v1 = p[b + TPB];
        sum += v0;
        sum += v1;
    }
    if (b < nb) sum += p[b];
    return sum;
}

// the same sums over partials stored [nv][nb] (contiguous per value)
__global__ void k_final_sum_t(const double* __restrict__ partial, int nb, double* __restrict__ out,
                              const int* __restrict__ ctrl) {
    if (ctrl && *ctrl != 0) return;
    __shared__ double red[TPB];
    const int v = blockIdx.x;
    red[threadIdx.x] = strided_sum(partial + (size_t)v * nb, threadIdx.x, nb);
    __syncthreads();
    for (int off = TPB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[v] = red[0];
}

static void final_sum(const double* partial, int nb, int nv, double* out, hipStream_t st,
                      const int* ctrl = nullptr) {
    hipLaunchKernelGGL(k_final_sum, dim3(nv), dim3(TPB), 0, st, partial, nb, nv, out, ctrl);
}
void launch_final_sum(const double* partial, int nb, int nv, double* out, hipStream_t st) {
    final_sum(partial, nb, nv, out, st);
}

// 16-byte lanes: two binary64 or four binary32 values per load
template <typename R>
struct Vec16;
template <>
struct Vec16<double> {
    using T = double2;
    static constexpr int W = 2;
};
template <>
struct Vec16<float> {
    using T = float4;
    static constexpr int W = 4;
};
template <typename T, typename R>
__device__ __forceinline__ R lane(const T& v, int k) {
    return ((const R*)&v)[k];
}
template <typename T, typename R>
__device__ __forceinline__ void set_lane(T& v, int k, R x) {
    ((R*)&v)[k] = x;
}

static unsigned stream_grid(int64_t L) {
    int64_t g = (L + TPB * 2 - 1) / (TPB * 2);
    if (g > RED_BLOCKS) g = RED_BLOCKS;
    if (g < 1) g = 1;
    return (unsigned)g;
}

// W detJ from the tables (affine meshes, or terrain-following ones with the
// compact metric) for the entries a lane visits: the
// element e and node n of its first entry are advanced by the grid stride
// (de elements and dn nodes) instead of dividing every index by Np. The
// binary32 weights are the rounded binary64 products, as in the stored array.
struct TabWalk {
    int e, n, de, dn;
    __device__ __forceinline__ TabWalk(const WSrc& ws, int64_t idx0, int64_t stride) {
        e = (int)(idx0 / ws.np);
        n = (int)(idx0 - (int64_t)e * ws.np);
        de = (int)(stride / ws.np);
        dn = (int)(stride - (int64_t)de * ws.np);
    }
    __device__ __forceinline__ void advance(int np) {
        n += dn;
        e += de;
        if (n >= np) {
            n -= np;
            ++e;
        }
    }
};

// the W lanes' weights of 16-byte lane x (TABW 0: the stored array; 1: from
// the tables, affine; 2: from the tables and the compact terrain metric)
template <typename R, typename VT, int W, int TABW>
__device__ __forceinline__ void lane_weights(const R* WJ, const WSrc& ws, const TabWalk& tw, int64_t x, double* wv) {
    if constexpr (TABW) {
#pragma unroll
        for (int k = 0; k < W; ++k) {
            int e = tw.e, n = tw.n + k;
            if (n >= ws.np) {   // Np > W: at most one wrap
                n -= ws.np;
                ++e;
            }
            const int ec = e < ws.E ? e : ws.E - 1;   // padding entries: load in bounds, weigh 0
            const double* q = ws.eg + 8 * (int64_t)ec;
            double dj;
            if constexpr (TABW == 2) dj = q[0] * (q[1] * ws.cm[(int64_t)ec * ws.K + n % ws.nf]);
            else dj = q[6];
            const double v = (double)(R)(ws.W3[n] * dj);
            wv[k] = e < ws.E ? v : 0.0;
        }
    } else {
        const VT ww = ((const VT*)WJ)[x];
#pragma unroll
        for (int k = 0; k < W; ++k) wv[k] = (double)lane<VT, R>(ww, k);
    }
}

// The lane's byte offset from a wave-uniform address, made opaque in every
// iteration of a walk (an empty statement that emits no instruction): the
// compiler cannot then hoist "vector + lane" out of the loop as a 64-bit
// per-lane address per vector, and every load takes the scalar-base form
// (one 32-bit offset register shared by all the vectors a lane reads).
__device__ __forceinline__ uint32_t lane_offset(uint32_t off) {
    asm volatile("" : "+v"(off));
    return off;
}

// ------------------------------------------------------- multi-dot products
// partial[v][b] = sum over workgroup b's entries of WJ * V_v * z. The vectors
// split into NG chunks over the wavefronts of one workgroup (4 / NG wavefronts
// per chunk, at most CH running sums per lane, so the lanes keep full
// occupancy): every chunk walks the same entries at the same time, so z and the
// weights come from HBM once and from the compute unit's caches for the other
// chunks.
template <typename R, int NG, int CH, int TABW>
__global__ void __launch_bounds__(TPB)
k_dots(int64_t L, const R* __restrict__ V, int64_t ldv, const R* __restrict__ z, const R* __restrict__ WJ,
       double* __restrict__ partial, int nvtot, const int* __restrict__ ctrl, WSrc ws) {
    if (ctrl && *ctrl != 0) return;
    constexpr int WPG = TPB / 64 / NG;   // wavefronts per chunk
    using VT = typename Vec16<R>::T;
    constexpr int W = Vec16<R>::W;
    __shared__ double red[TPB / 64][CH];
    // the wavefront index is uniform: the chunk, its vectors and the walk's
    // base offset live in scalar registers
    const int ln = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gi = wid % NG, sub = wid / NG;
    const int per = (nvtot + NG - 1) / NG, v0 = gi * per;
    const int nv = nvtot - v0 < per ? nvtot - v0 : per;
    double acc[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) acc[i] = 0;
    // every running sum loads unconditionally (a guarded load would wait for
    // each vector in turn); sums past the chunk's last vector repeat that
    // vector's address and are never written out
    const char* vp[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) {
        int vi = v0 + (i < nv ? i : nv - 1);
        vi = vi < nvtot ? (vi < 0 ? 0 : vi) : nvtot - 1;
        vp[i] = (const char*)(V + (int64_t)vi * ldv);
    }
    const int64_t nvec = L / W;   // ldv and L are multiples of W
    // a wavefront walks 64 consecutive 16-byte lanes from a uniform base b:
    // each address is a scalar base plus the lane's 32-bit offset
    const int64_t b0 = (blockIdx.x * (int64_t)WPG + sub) * 64, xs = (int64_t)gridDim.x * WPG * 64;
    const uint32_t lo0 = (uint32_t)ln * (uint32_t)sizeof(VT);
    TabWalk tw(ws, TABW ? (b0 + ln) * W : 0, TABW ? xs * W : 0);
    for (int64_t b = b0; b < nvec; b += xs) {
        const int64_t x = b + ln;
        if (x < nvec) {
            const int64_t bo = b * (int64_t)sizeof(VT);
            const uint32_t lo = lane_offset(lo0);
            VT v[CH];
#pragma unroll
            for (int i = 0; i < CH; ++i) v[i] = *(const VT*)(vp[i] + bo + lo);
            const VT zz = *(const VT*)((const char*)z + bo + lo);
            double wz[W];
            lane_weights<R, VT, W, TABW>(WJ, ws, tw, x, wz);
#pragma unroll
            for (int k = 0; k < W; ++k) wz[k] *= (double)lane<VT, R>(zz, k);
#pragma unroll
            for (int i = 0; i < CH; ++i)
#pragma unroll
                for (int k = 0; k < W; ++k) acc[i] += wz[k] * (double)lane<VT, R>(v[i], k);
        }
        if constexpr (TABW) tw.advance(ws.np);
    }
#pragma unroll
    for (int i = 0; i < CH; ++i)
        for (int off = 32; off > 0; off >>= 1) acc[i] += __shfl_xor(acc[i], off, 64);
    if (ln == 0)
#pragma unroll
        for (int i = 0; i < CH; ++i) red[wid][i] = acc[i];
    __syncthreads();
    if (threadIdx.x < nvtot) {
        const int g = threadIdx.x / per, i = threadIdx.x - g * per;
        double sum = 0;
        for (int k = 0; k < WPG; ++k) sum += red[k * NG + g][i];
        partial[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = sum;   // [vector][workgroup]
    }
}

// one running sum per vector of a chunk: the chunk length (nv / NG rounded up)
// is the template's CH, so that no load repeats an address except in the
// last chunk
template <typename R, int TABW>
static void dots_launch(unsigned g, int nv, int64_t L, const R* V, int64_t ldv, const R* z, const R* WJ,
                        double* partial, hipStream_t st, const int* ctrl, const WSrc& ws) {
#define IMX_DOTS(NG, CH) \
    hipLaunchKernelGGL((k_dots<R, NG, CH, TABW>), dim3(g), dim3(TPB), 0, st, L, V, ldv, z, WJ, partial, nv, ctrl, ws)
    if (nv <= 2)
        IMX_DOTS(1, 2);
    else if (nv <= 4)
        IMX_DOTS(1, 4);
    else if (nv <= 8)
        IMX_DOTS(1, 8);
    else if (nv <= 10)
        IMX_DOTS(2, 5);
    else if (nv <= 12)
        IMX_DOTS(2, 6);
    else if (nv <= 14)
        IMX_DOTS(2, 7);
    else if (nv <= 16)
        IMX_DOTS(2, 8);
    else if (nv <= 20)
        IMX_DOTS(4, 5);
    else if (nv <= 24)
        IMX_DOTS(4, 6);
    else if (nv <= 28)
        IMX_DOTS(4, 7);
    else if (nv <= 32)
        IMX_DOTS(4, 8);
    else   // nv <= MAXV = 33
        IMX_DOTS(4, 9);
#undef IMX_DOTS
}

template <typename R>
void launch_dots(int64_t L, int nv, const R* V, int64_t ldv, const R* z, const R* WJ, double* partial,
                 double* out, hipStream_t st, const int* ctrl, WSrc ws) {
    // grid measured on the 3 M-entry channel basis: 512 workgroups (two per
    // compute unit) for every vector count; 256, 384, 1024 and 2048 were slower
    const unsigned gmax = 512;
    const unsigned g = stream_grid(L) > gmax ? gmax : stream_grid(L);
    // binary32 vectors read their stored weights on terrain-following meshes:
    // for them the 4-byte weight costs less than forming it from the metric
    constexpr int TCM = sizeof(R) == 8 ? 2 : 0;
    if (ws.cm)
        dots_launch<R, TCM>(g, nv, L, V, ldv, z, WJ, partial, st, ctrl, ws);
    else if (ws.W3)
        dots_launch<R, 1>(g, nv, L, V, ldv, z, WJ, partial, st, ctrl, ws);
    else
        dots_launch<R, 0>(g, nv, L, V, ldv, z, WJ, partial, st, ctrl, ws);
    hipLaunchKernelGGL(k_final_sum_t, dim3(nv), dim3(TPB), 0, st, partial, (int)g, out, ctrl);
}
template void launch_dots<double>(int64_t, int, const double*, int64_t, const double*, const double*, double*,
                                  double*, hipStream_t, const int*, WSrc);
template void launch_dots<float>(int64_t, int, const float*, int64_t, const float*, const float*, double*, double*,
                                 hipStream_t, const int*, WSrc);

// --------------------------------------------------- Gram-Schmidt update
// z1 = z - sum_i raw[i] s[i]^2 V_i and its squared M-norm (no basis vector
// kept live: one running value per lane)
template <typename R, int CH, int TABW>
__global__ void __launch_bounds__(TPB)
k_axpy_norm(int64_t L, int nv, const R* __restrict__ V, int64_t ldv, const double* __restrict__ raw,
            const double* __restrict__ s, const R* z, R* z1, const R* __restrict__ WJ, double* __restrict__ partial,
            const int* __restrict__ ctrl, WSrc ws) {
    if (ctrl && *ctrl != 0) return;
    using VT = typename Vec16<R>::T;
    constexpr int W = Vec16<R>::W;
    __shared__ double red[(TPB / 64 + 1)];
    __shared__ double cf[CH];
    if (threadIdx.x < CH) cf[threadIdx.x] = threadIdx.x < nv ? raw[threadIdx.x] * s[threadIdx.x] * s[threadIdx.x] : 0.0;
    __syncthreads();
    double acc[1] = {0.0};
    const int64_t nvec = L / W;
    const int64_t x0 = blockIdx.x * (int64_t)TPB + threadIdx.x, xs = (int64_t)gridDim.x * TPB;
    TabWalk tw(ws, TABW ? x0 * W : 0, TABW ? xs * W : 0);
    for (int64_t x = x0; x < nvec; x += xs) {
        const VT zin = ((const VT*)z)[x];
        double zz[W];
#pragma unroll
        for (int k = 0; k < W; ++k) zz[k] = (double)lane<VT, R>(zin, k);
#pragma unroll
        for (int i = 0; i < CH; ++i)
            if (i < nv) {
                const VT v = ((const VT*)(V + (int64_t)i * ldv))[x];
                const double c = cf[i];
#pragma unroll
                for (int k = 0; k < W; ++k) zz[k] -= c * (double)lane<VT, R>(v, k);
            }
        VT zo;
#pragma unroll
        for (int k = 0; k < W; ++k) set_lane<VT, R>(zo, k, (R)zz[k]);
        ((VT*)z1)[x] = zo;
        double wv[W];
        lane_weights<R, VT, W, TABW>(WJ, ws, tw, x, wv);
        if constexpr (TABW) tw.advance(ws.np);
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const double zr = (double)lane<VT, R>(zo, k);
            acc[0] += wv[k] * zr * zr;
        }
    }
    block_sum<1>(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = red[TPB / 64];
}

int axpy_norm_blocks(int64_t L) { return (int)stream_grid(L); }

template <typename R, int TABW>
static void axpy_norm_launch(unsigned g, int64_t L, int nv, const R* V, int64_t ldv, const double* raw,
                             const double* s, const R* z, R* z1, const R* WJ, double* partial, hipStream_t st,
                             const int* ctrl, const WSrc& ws) {
    if (nv <= 8)
        hipLaunchKernelGGL((k_axpy_norm<R, 8, TABW>), dim3(g), dim3(TPB), 0, st, L, nv, V, ldv, raw, s, z, z1, WJ,
                           partial, ctrl, ws);
    else if (nv <= 16)
        hipLaunchKernelGGL((k_axpy_norm<R, 16, TABW>), dim3(g), dim3(TPB), 0, st, L, nv, V, ldv, raw, s, z, z1, WJ,
                           partial, ctrl, ws);
    else
        hipLaunchKernelGGL((k_axpy_norm<R, 32, TABW>), dim3(g), dim3(TPB), 0, st, L, nv, V, ldv, raw, s, z, z1, WJ,
                           partial, ctrl, ws);
}

template <typename R>
void launch_axpy_norm(int64_t L, int nv, const R* V, int64_t ldv, const double* raw, const double* s, const R* z,
                      R* z1, const R* WJ, double* partial, hipStream_t st, const int* ctrl, WSrc ws) {
    const unsigned g = stream_grid(L);
    constexpr int TCM = sizeof(R) == 8 ? 2 : 0;   // binary32: the stored weights, as for the dots
    if (ws.cm)
        axpy_norm_launch<R, TCM>(g, L, nv, V, ldv, raw, s, z, z1, WJ, partial, st, ctrl, ws);
    else if (ws.W3)
        axpy_norm_launch<R, 1>(g, L, nv, V, ldv, raw, s, z, z1, WJ, partial, st, ctrl, ws);
    else
        axpy_norm_launch<R, 0>(g, L, nv, V, ldv, raw, s, z, z1, WJ, partial, st, ctrl, ws);
}
template void launch_axpy_norm<double>(int64_t, int, const double*, int64_t, const double*, const double*,
                                       const double*, double*, const double*, double*, hipStream_t, const int*, WSrc);
template void launch_axpy_norm<float>(int64_t, int, const float*, int64_t, const double*, const double*,
                                      const float*, float*, const float*, double*, hipStream_t, const int*, WSrc);

// ------------------------------------------------- Arnoldi step on the device
// Column j of the Hessenberg matrix from the Gram-Schmidt projections, the
// Givens rotations and the residual estimate (Saad, Alg. 6.9): the Krylov loop
// then needs no host round trip per iteration. One workgroup: it sums the
// update's partial norms (same fixed order as the final sums), loads the
// column and the earlier rotations into LDS in parallel, one lane applies the
// recurrence, and the column is written back in parallel.
__global__ void __launch_bounds__(TPB)
k_givens(GState* __restrict__ G, int j, const double* __restrict__ raw, const double* __restrict__ raw2,
         const double* __restrict__ npart, int nb) {
    const int t = threadIdx.x;
    const int st0 = G->status;
    if (raw2 == nullptr ? st0 != 0 : st0 != 2) return;
    __shared__ double red[TPB];
    __shared__ double col[GM + 1], cs[GM], sn[GM];
    __shared__ int keep;
    // every global load is issued before the first LDS write and before any
    // sum needs its value: the column, the earlier rotations, the scalars lane
    // 0 needs after the reduction, and the partial norms eight at a time (the
    // additions keep the order b = t, t + TPB, ...)
    double h = 0, csv = 0, snv = 0;
    if (t <= j) {
        h = G->sv[t] * raw[t];
        if (raw2) h += G->sv[t] * raw2[t];
    }
    if (t < j) {
        csv = G->cs[t];
        snv = G->sn[t];
    }
    double gj = 0, tolb = 0, zz = 0;
    int its0 = 0, maxit = 0, fixed = 0;
    if (t == 0) {
        gj = G->g[j];
        tolb = G->tolb;
        its0 = G->its;
        maxit = G->maxit;
        fixed = G->fixed;
        if (raw2 == nullptr) zz = raw[j + 1];
    }
    red[t] = strided_sum(npart, t, nb);
    if (t <= j) col[t] = h;
    if (t < j) {
        cs[t] = csv;
        sn[t] = snv;
    }
    __syncthreads();
    for (int off = TPB / 2; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    if (t == 0) {
        const double nrm = red[0];
        // severe cancellation in the single classical Gram-Schmidt pass: the
        // host runs a second pass and finishes the column
        if (raw2 == nullptr && nrm < 1e-6 * zz) {
            G->status = 2;
            keep = 0;
        } else {
            keep = 1;
            if (raw2) G->status = 0;
            const double hnext = sqrt(nrm);
            // earlier rotations applied down the column; the entry below the
            // current one stays in a register from one rotation to the next
            double cur = col[0];
            for (int i = 0; i < j; ++i) {
                const double a = cur, b = col[i + 1];
                col[i] = cs[i] * a + sn[i] * b;
                cur = -sn[i] * a + cs[i] * b;
            }
            const double hj = j > 0 ? cur : col[0];
            const double den = hypot(hj, hnext);
            const double c = hj / den, s = hnext / den;
            G->cs[j] = c;
            G->sn[j] = s;
            col[j] = den;
            col[j + 1] = 0.0;
            G->g[j + 1] = -s * gj;
            G->g[j] = c * gj;
            G->k = j + 1;
            const int its = its0 + 1;
            G->its = its;
            if (!isfinite(hnext)) {
                G->status = 3;
            } else if (hnext == 0.0 || its >= maxit || (!fixed && fabs(-s * gj) <= tolb)) {
                G->status = 1;
            } else {
                G->sv[j + 1] = 1.0 / hnext;
                G->svf[j + 1] = (float)(1.0 / hnext);
            }
        }
    }
    __syncthreads();
    if (keep && t <= j + 1) G->H[t * GM + j] = col[t];
}
void launch_givens(GState* G, int j, const double* raw, const double* raw2, const double* npart, int nb,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_givens, dim3(1), dim3(TPB), 0, st, G, j, raw, raw2, npart, nb);
}

// ----------------------------------------------------------- linear combination
template <typename R>
__global__ void k_lincomb(int64_t L, int nv, const R* __restrict__ V, int64_t ldv, const double* __restrict__ coef,
                          R* __restrict__ x) {
    using VT = typename Vec16<R>::T;
    constexpr int W = Vec16<R>::W;
    const int64_t nvec = L / W;
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < nvec; i += (int64_t)gridDim.x * TPB) {
        const VT xin = ((const VT*)x)[i];
        double acc[W];
#pragma unroll
        for (int k = 0; k < W; ++k) acc[k] = (double)lane<VT, R>(xin, k);
        for (int j = 0; j < nv; ++j) {
            const VT v = ((const VT*)(V + (int64_t)j * ldv))[i];
#pragma unroll
            for (int k = 0; k < W; ++k) acc[k] += coef[j] * (double)lane<VT, R>(v, k);
        }
        VT o;
#pragma unroll
        for (int k = 0; k < W; ++k) set_lane<VT, R>(o, k, (R)acc[k]);
        ((VT*)x)[i] = o;
    }
}
template <typename R>
void launch_lincomb(int64_t L, int nv, const R* V, int64_t ldv, const double* coef, R* x, hipStream_t st) {
    hipLaunchKernelGGL((k_lincomb<R>), dim3(stream_grid(L)), dim3(TPB), 0, st, L, nv, V, ldv, coef, x);
}
template void launch_lincomb<double>(int64_t, int, const double*, int64_t, const double*, double*, hipStream_t);
template void launch_lincomb<float>(int64_t, int, const float*, int64_t, const double*, float*, hipStream_t);

// ------------------------------------------------------------ weighted dots
__global__ void __launch_bounds__(TPB)
k_wdot(int64_t L, const double* __restrict__ a, const double* __restrict__ b, const double* __restrict__ WJ,
       double* __restrict__ partial) {
    __shared__ double red[(TPB / 64 + 1)];
    double acc[1] = {0};
    for (int64_t x = blockIdx.x * (int64_t)TPB + threadIdx.x; x < L; x += (int64_t)gridDim.x * TPB)
        acc[0] += WJ[x] * a[x] * b[x];
    block_sum<1>(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = red[TPB / 64];
}
void launch_wdot(int64_t L, const double* a, const double* b, const double* WJ, double* partial, double* out,
                 hipStream_t st) {
    const unsigned g = grid_for(L, TPB * 8) > RED_BLOCKS ? RED_BLOCKS : grid_for(L, TPB * 8);
    hipLaunchKernelGGL(k_wdot, dim3(g), dim3(TPB), 0, st, L, a, b ? b : a, WJ, partial);
    final_sum(partial, (int)g, 1, out, st);
}

__global__ void __launch_bounds__(TPB)
k_picard_var(int64_t L, const double* __restrict__ p0, const double* __restrict__ u0, const double* __restrict__ p1,
             const double* __restrict__ u1, const double* __restrict__ rho, const double* __restrict__ WJ,
             double gamma, double* __restrict__ partial) {
    __shared__ double red[(TPB / 64 + 1) * 2];
    double acc[2] = {0, 0};
    for (int64_t x = blockIdx.x * (int64_t)TPB + threadIdx.x; x < L; x += (int64_t)gridDim.x * TPB) {
        const double dp = p1[x] - p0[x];
        double du2 = 0;
        for (int c = 0; c < 3; ++c) {
            const double du = u1[c * L + x] - u0[c * L + x];
            du2 += du * du;
        }
        acc[0] += WJ[x] * (dp * dp + gamma * p1[x] * rho[x] * du2);
        acc[1] += WJ[x] * p1[x] * p1[x];
    }
    block_sum<2>(acc, red);
    if (threadIdx.x < 2) partial[blockIdx.x * 2 + threadIdx.x] = red[TPB / 64 * 2 + threadIdx.x];
}
void launch_picard_var(int64_t L, const double* p0, const double* u0, const double* p1, const double* u1,
                       const double* rho, const double* WJ, double gamma, double* partial, double* out,
                       hipStream_t st) {
    const unsigned g = grid_for(L, TPB * 8) > RED_BLOCKS ? RED_BLOCKS : grid_for(L, TPB * 8);
    hipLaunchKernelGGL(k_picard_var, dim3(g), dim3(TPB), 0, st, L, p0, u0, p1, u1, rho, WJ, gamma, partial);
    final_sum(partial, (int)g, 2, out, st);
}

__global__ void __launch_bounds__(TPB)
k_mass(int64_t L, const double* __restrict__ q, const double* __restrict__ WJ, double* __restrict__ partial) {
    __shared__ double red[(TPB / 64 + 1) * 2];
    double acc[2] = {0, 0};
    for (int64_t x = blockIdx.x * (int64_t)TPB + threadIdx.x; x < L; x += (int64_t)gridDim.x * TPB) {
        acc[0] += WJ[x] * q[x];
        for (int t = 0; t < 5; ++t)
            if (!isfinite(q[t * L + x])) acc[1] += 1.0;
    }
    block_sum<2>(acc, red);
    if (threadIdx.x < 2) partial[blockIdx.x * 2 + threadIdx.x] = red[TPB / 64 * 2 + threadIdx.x];
}
int mass_blocks(int64_t L) {
    return (int)(grid_for(L, TPB * 8) > RED_BLOCKS ? RED_BLOCKS : grid_for(L, TPB * 8));
}
void launch_mass(int64_t L, const double* q, const double* WJ, double* partial, double* out, hipStream_t st) {
    const unsigned g = (unsigned)mass_blocks(L);
    hipLaunchKernelGGL(k_mass, dim3(g), dim3(TPB), 0, st, L, q, WJ, partial);
    final_sum(partial, (int)g, 2, out, st);
}

// ---------------------------------------------------------- stage combines
__global__ void k_stage_prepare(int64_t L, const double* __restrict__ y, const double* __restrict__ fN0,
                                const double* __restrict__ fN1, const double* __restrict__ fS0,
                                const double* __restrict__ fS1, const double* __restrict__ yp, StageCoef c,
                                double* __restrict__ rho, double* __restrict__ Fh, double* __restrict__ G0h,
                                double* __restrict__ p0, double* __restrict__ u0) {
    for (int64_t x = blockIdx.x * (int64_t)TPB + threadIdx.x; x < L; x += (int64_t)gridDim.x * TPB) {
        const double* fN[2] = {fN0, fN1};
        const double* fS[2] = {fS0, fS1};
        double r = 0, F[3] = {0, 0, 0}, G = 0;
        for (int m = 0; m < c.l; ++m) {
            r += c.a[m] * fN[m][x];
            for (int k = 0; k < 3; ++k) F[k] += c.a[m] * fN[m][(1 + k) * L + x] + c.at[m] * fS[m][k * L + x];
            G += c.a[m] * fN[m][4 * L + x] + c.at[m] * fS[m][3 * L + x];
        }
        const double rl = y[x] + c.dt * r;
        rho[x] = rl;
        for (int k = 0; k < 3; ++k) Fh[k * L + x] = y[(1 + k) * L + x] + c.dt * F[k];
        Fh[2 * L + x] -= c.c_dt * c.g * rl;
        G0h[x] = y[4 * L + x] + c.dt * G;
        const double rp = yp[x];
        double k2 = 0;
        for (int k = 0; k < 3; ++k) {
            const double uu = yp[(1 + k) * L + x] / rp;
            u0[k * L + x] = uu;
            k2 += uu * uu;
        }
        p0[x] = (c.gamma - 1.0) * (yp[4 * L + x] - rp * 0.5 * k2);
    }
}
void launch_stage_prepare(int64_t L, const double* y, const double* const* fNS, const double* const* fS,
                          const double* yprev, const StageCoef& c, double* rho, double* Fh, double* G0h,
                          double* p0, double* u0, hipStream_t st) {
    hipLaunchKernelGGL(k_stage_prepare, dim3(grid_for(L)), dim3(TPB), 0, st, L, y, fNS[0], c.l > 1 ? fNS[1] : fNS[0],
                       fS[0], c.l > 1 ? fS[1] : fS[0], yprev, c, rho, Fh, G0h, p0, u0);
}

__global__ void k_finalize(int64_t L, const double* __restrict__ rho, const double* __restrict__ p,
                           const double* __restrict__ u, double gamma, double* __restrict__ Y) {
    for (int64_t x = blockIdx.x * (int64_t)TPB + threadIdx.x; x < L; x += (int64_t)gridDim.x * TPB) {
        const double r = rho[x];
        double k2 = 0;
        Y[x] = r;
        for (int k = 0; k < 3; ++k) {
            const double uu = u[k * L + x];
            Y[(1 + k) * L + x] = r * uu;
            k2 += uu * uu;
        }
        Y[4 * L + x] = p[x] / (gamma - 1.0) + 0.5 * r * k2;
    }
}
void launch_finalize(int64_t L, const double* rho, const double* p, const double* u, double gamma, double* Y,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(grid_for(L)), dim3(TPB), 0, st, L, rho, p, u, gamma, Y);
}

struct FinalArgs {
    const double* fN[3];
    const double* fS[3];
    double b[3];
};
__global__ void k_final_update(int64_t L, const double* __restrict__ y, FinalArgs a, double dt,
                               double* __restrict__ yn) {
    for (int64_t x = blockIdx.x * (int64_t)TPB + threadIdx.x; x < L; x += (int64_t)gridDim.x * TPB) {
        for (int t = 0; t < 5; ++t) {
            double s = 0;
            for (int l = 0; l < 3; ++l) {
                double v = a.fN[l][t * L + x];
                if (t > 0) v += a.fS[l][(t - 1) * L + x];
                s += a.b[l] * v;
            }
            yn[t * L + x] = y[t * L + x] + dt * s;
        }
    }
}
void launch_final_update(int64_t L, const double* y, const double* const* fNS, const double* const* fS,
                         const double* b, double dt, double* ynew, hipStream_t st) {
    FinalArgs a;
    for (int l = 0; l < 3; ++l) {
        a.fN[l] = fNS[l];
        a.fS[l] = fS[l];
        a.b[l] = b[l];
    }
    hipLaunchKernelGGL(k_final_update, dim3(grid_for(L)), dim3(TPB), 0, st, L, y, a, dt, ynew);
}

__global__ void k_scale_div(int64_t L, int nf, const double* __restrict__ in, const double* __restrict__ WJ,
                            double* __restrict__ out) {
    for (int64_t x = blockIdx.x * (int64_t)TPB + threadIdx.x; x < L; x += (int64_t)gridDim.x * TPB)
        for (int t = 0; t < nf; ++t) out[t * L + x] = in[t * L + x] / WJ[x];
}
void launch_scale_div(int64_t L, int nf, const double* in, const double* WJ, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_div, dim3(grid_for(L)), dim3(TPB), 0, st, L, nf, in, WJ, out);
}

// Rayleigh relaxation of the whole conserved state towards a target, added
// to the non-stiff tendencies M^{-1} T_NS (the layer coefficient per node)
__global__ void k_sponge_relax(int64_t L, const double* __restrict__ q, const double* __restrict__ target,
                               const double* __restrict__ lam, double* __restrict__ fNS) {
    for (int64_t x = blockIdx.x * (int64_t)TPB + threadIdx.x; x < L; x += (int64_t)gridDim.x * TPB) {
        const double l = lam[x];
        if (l == 0.0) continue;
#pragma unroll
        for (int t = 0; t < 5; ++t) fNS[t * L + x] -= l * (q[t * L + x] - target[t * L + x]);
    }
}

void launch_sponge_relax(int64_t L, const double* q, const double* target, const double* lam, double* fNS,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_sponge_relax, dim3(grid_for(L)), dim3(TPB), 0, st, L, q, target, lam, fNS);
}

__global__ void k_stage_coef(int64_t L, const double* __restrict__ rho, const double* __restrict__ WJ,
                             double* __restrict__ cr, float* __restrict__ crf) {
    for (int64_t x = blockIdx.x * (int64_t)TPB + threadIdx.x; x < L; x += (int64_t)gridDim.x * TPB) {
        const double c = 1.0 / (WJ[x] * rho[x]);
        cr[x] = c;
        if (crf) crf[x] = (float)c;
    }
}
void launch_stage_coef(int64_t L, const double* rho, const double* WJ, double* cr, float* crf, hipStream_t st) {
    hipLaunchKernelGGL(k_stage_coef, dim3(grid_for(L)), dim3(TPB), 0, st, L, rho, WJ, cr, crf);
}

__global__ void k_d2f(int64_t L, const double* __restrict__ in, float* __restrict__ out) {
    for (int64_t x = blockIdx.x * (int64_t)TPB + threadIdx.x; x < L; x += (int64_t)gridDim.x * TPB) out[x] = (float)in[x];
}
void launch_d2f(int64_t L, const double* in, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_d2f, dim3(grid_for(L)), dim3(TPB), 0, st, L, in, out);
}

__global__ void k_f2d_add(int64_t L, const float* __restrict__ in, const double* __restrict__ s,
                          double* __restrict__ x) {
    const double sc = s ? s[0] : 1.0;
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < L; i += (int64_t)gridDim.x * TPB)
        x[i] += sc * (double)in[i];
}
void launch_f2d_add(int64_t L, const float* in, const double* scale, double* x, hipStream_t st) {
    hipLaunchKernelGGL(k_f2d_add, dim3(grid_for(L)), dim3(TPB), 0, st, L, in, scale, x);
}

__global__ void k_axpby(int64_t L, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                        double* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < L; i += (int64_t)gridDim.x * TPB)
        out[i] = a * x[i] + (y ? b * y[i] : 0.0);
}
void launch_axpby(int64_t L, double a, const double* x, double b, const double* y, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(L)), dim3(TPB), 0, st, L, a, x, b, y, out);
}

// out = in * s (s from device: s[0], or 1/sqrt(s[0]) when invert_sqrt)
__global__ void k_scale_store(int64_t L, const double* __restrict__ in, const double* __restrict__ s, int inv,
                              double* __restrict__ out) {
    const double sc = inv ? 1.0 / sqrt(s[0]) : s[0];
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < L; i += (int64_t)gridDim.x * TPB) out[i] = sc * in[i];
}
void launch_scale_store(int64_t L, const double* in, const double* s_ptr, int invert_sqrt, double* out,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_scale_store, dim3(grid_for(L)), dim3(TPB), 0, st, L, in, s_ptr, invert_sqrt, out);
}
__global__ void k_scale_store_f(int64_t L, const double* __restrict__ in, const double* __restrict__ s,
                                float* __restrict__ out) {
    const double sc = s[0];
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < L; i += (int64_t)gridDim.x * TPB)
        out[i] = (float)(sc * in[i]);
}
void launch_scale_store_f(int64_t L, const double* in, const double* s_ptr, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_store_f, dim3(grid_for(L)), dim3(TPB), 0, st, L, in, s_ptr, out);
}

}  // namespace imx
