// Device data views and kernel launchers of the IMEX-DG hot path.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "internal.hpp"

namespace imx {

// Geometry and connectivity on the device, in binary64 and (for the mixed
// precision inner loop) binary32 shadows.
struct DevMesh {
    int64_t E = 0, nh = 0;
    int64_t Lp = 0;                 // E*Np rounded up to a multiple of 4 (Krylov vector stride)
    int n = 0, Np = 0, Nf = 0;
    int deformed = 0;
    const int* kind = nullptr;      // [E*6]
    const int* nbr = nullptr;       // [E*6]
    const int* aux = nullptr;       // [E*6]
    const int* hang = nullptr;      // [nh*4]
    const double* h = nullptr;      // [E*3]
    const double* hinv = nullptr;   // [E*3] 1 / h
    const double* WJ = nullptr;     // [E*Np]
    const double* G = nullptr;      // [5][E][Np] terrain-following meshes: W cof(J) (0,0) (1,1) (2,0) (2,1) (2,2)
    const double* nS = nullptr;     // [E][10][Nf] terrain-following meshes: n dS, normal component on x/y faces
    const double* sponge = nullptr; // [E*Np] or null
    const float* WJf = nullptr;
    const float* Gf = nullptr;
    const float* nSf = nullptr;
    const double* eg = nullptr;     // [E*8] affine elements: h[3], 1/h[3], det J, 1/det J
    const double* iWJ = nullptr;    // [E*Np] 1 / WJ (deformed meshes)
    const float* iWJf = nullptr;
    // terrain-following meshes without hanging faces: the compact metric
    // ([E][cm_stride(n)], Mesh::cm) from which the Krylov passes form W cof(J),
    // 1 / W detJ and n dS instead of reading them
    const double* cm = nullptr;
    const float* cmf = nullptr;
    const uint64_t* fofs = nullptr; // [fofs_count(n)] face-point words of the all-faces kernels
    // unrefined box meshes: element e = bz + nz (bx + nx by), so neighbours and
    // face kinds follow from the index (structured != 0 once the host has
    // checked this against the face tables)
    int structured = 0, gnx = 0, gny = 0, gnz = 0, gpx = 0, gpy = 0;
    int64_t ncoarse = 0;            // elements owning a coarse hanging face
    const int* reg_list = nullptr;  // [E - ncoarse] the other elements
    const int* crs_list = nullptr;  // [ncoarse]
    const void* tab = nullptr;      // basis tables (binary64), device
    const void* tabf = nullptr;     // basis tables (binary32), device
    // meshes with hanging faces: the face-by-face kernels of crs_list run on
    // `side` beside the all-faces kernels of reg_list (fork and join events)
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

struct PhysK {
    double gamma, g, f;
    double gm1, igm1, hfac;   // gamma - 1, 1 / (gamma - 1), gamma / (gamma - 1)
    double su[3];
    int sponge;
};

struct StageK {
    double c_dt;    // a_ll * dt
    double beta;    // a_ll * dt * f
    double gamma, g;
    double hfac;    // gamma / (gamma - 1): (rho h) = hfac p
    double igm1;    // 1 / (gamma - 1)
    double rot_si;  // 1 / (1 + beta^2), the scale of (I + beta J)^{-1} on the horizontal block
    int scheme;     // 1: R1, 2: R2
};

// Tables of the 1D basis (host copy, converted per launch).
struct HostTab {
    int n;
    double D[64], f[16], H[2 * 64], w[8];
};
HostTab make_tab(const Basis1D& b);
// device layout of the basis tables of degree n-1: size and host-side image
size_t tab_bytes(int n, int f32);
// per-lane face-point words (node offsets along the normal, face, point)
size_t fofs_count(int n);
void fill_fofs(int n, uint64_t* out);
void fill_tab(const HostTab& h, int f32, void* out);

// --- element kernels (templated on the floating type R = double / float)
template <typename R>
void launch_explicit(const DevMesh& m, const HostTab& t, const PhysK& ph, const R* q, R* fNS, R* fS,
                     hipStream_t st);

// w = P(Fh/rho - M^{-1}B(sc*p)/rho [+R1 lag]); writes w [3] and the face flux
// buffers FB [E*6*Nf], FBh [nh*4*Nf] used by pass 2.
template <typename R>
void launch_pass1(const DevMesh& m, const HostTab& t, const StageK& sk, const R* p, const R* pscale,
                  const R* Fh, const R* rho, const R* pk, const R* uk, R* w, R* FB, R* FBh,
                  hipStream_t st);

// out = alpha * (Gp - sc*p/(gamma-1) - M^{-1}C^k w - [R2] c g rho w_z) [* WJ if dual]
// With V != null also dots[i] = <V_i, out>_M (i < nv) and dots[nv] = <out, out>_M
// (partial: pass2_partial_count(m) doubles of scratch).
template <typename R>
void launch_pass2(const DevMesh& m, const HostTab& t, const StageK& sk, const R* Gp, const R* p,
                  const R* pscale, const R* w, const R* pk, const R* rho, const R* FB, const R* FBh,
                  R* out, double alpha, int dual, hipStream_t st, const R* V = nullptr, int nv = 0,
                  double* partial = nullptr, double* dots = nullptr);
size_t pass2_partial_count(const DevMesh& m);

// Schur complement inside the Krylov loop (no right-hand side):
// launch_mv1: face buffers of x scaled by *xs (xs may be null), cr = 1 / (WJ rho_l);
// w[0] receives each element's own volume and gravity part of pass 2 (the
// elements owning a coarse hanging face store (rho h)^k w, three fields);
// launch_mv2: out = M^{-1} S (xs x) (dual = 0) or S (xs x) (dual = 1), after
// launch_mv1.
// With ctrl != null every workgroup returns at once while *ctrl != 0 (a
// Krylov cycle that has stopped on the device).
template <typename R>
void launch_mv1(const DevMesh& m, const StageK& sk, const R* x, const R* xs, const R* cr, const R* rho,
                const R* pk, R* w, R* FB, R* FBh, hipStream_t st, const int* ctrl = nullptr);
template <typename R>
void launch_mv2(const DevMesh& m, const StageK& sk, const R* x, const R* xs, const R* w, const R* pk,
                const R* rho, const R* FB, const R* FBh, R* out, int dual, hipStream_t st,
                const int* ctrl = nullptr);
// cr = 1 / (WJ rho), and its binary32 copy when crf != null
void launch_stage_coef(int64_t L, const double* rho, const double* WJ, double* cr, float* crf, hipStream_t st);
void launch_final_sum(const double* partial, int nb, int nv, double* out, hipStream_t st);

// Gp = G0h - M^{-1}Lambda^k - rho kappa^k [R1: - c g rho uk_z]
void launch_lambda(const DevMesh& m, const HostTab& t, const StageK& sk, const double* pk, const double* uk,
                   const double* rho, const double* G0h, double* Gp, hipStream_t st);

// --- streaming kernels (binary64 state arithmetic)
struct StageCoef {
    double a[3], at[3];   // a_lm, a~_lm for m < l
    int l;                // number of previous stages
    double dt, c_dt, g, gamma;
};
void launch_stage_prepare(int64_t L, const double* y, const double* const* fNS, const double* const* fS,
                          const double* yprev, const StageCoef& c, double* rho, double* Fh, double* G0h,
                          double* p0, double* u0, hipStream_t st);
void launch_finalize(int64_t L, const double* rho, const double* p, const double* u, double gamma, double* Y,
                     hipStream_t st);
void launch_final_update(int64_t L, const double* y, const double* const* fNS, const double* const* fS,
                         const double* b, double dt, double* ynew, hipStream_t st);
void launch_scale_div(int64_t L, int nf, const double* in, const double* WJ, double* out, hipStream_t st);
// damping layers relaxing the whole state: fNS[t] -= lam (q[t] - target[t]), t = 0..4 ([5][L] fields)
void launch_sponge_relax(int64_t L, const double* q, const double* target, const double* lam, double* fNS,
                         hipStream_t st);

// --- reductions: partial sums per block then a fixed-order final sum
constexpr int RED_BLOCKS = 4096;
constexpr int MAXV = 33;   // restart length <= 32
// Krylov vectors are stored with L rounded up to a multiple of 4 (padding is
// zero and carries zero weight), so the streaming kernels use 16-byte lanes.
// Source of the weights W detJ of the Krylov inner products: the stored
// array WJ, or on affine meshes the tensor weight of the node times the
// element's det J (per-element constants, 8 per element, det J at index 6),
// which saves one vector read per launch; on terrain-following meshes with
// the compact metric, the tensor weight times h_x (h_y J22). Entries at and beyond nreal (the
// padding of the basis) weigh 0.
struct WSrc {
    const double* W3 = nullptr;   // null: read the stored array
    const double* eg = nullptr;
    int E = 0, np = 0;
    // terrain-following meshes with the compact metric: det J = h_x (h_y J22),
    // J22 from the element's (x, y) plane (entry n % nf of its K values)
    const double* cm = nullptr;
    int nf = 0, K = 0;
};
// out[i] = sum WJ * V_i * z  (i < nv), V_i = V + i*ldv, all length L (R = double or float)
template <typename R>
void launch_dots(int64_t L, int nv, const R* V, int64_t ldv, const R* z, const R* WJ, double* partial,
                 double* out, hipStream_t st, const int* ctrl = nullptr, WSrc ws = WSrc());
// z1 = z - sum_i c_i V_i with c_i = raw[i]*s[i]^2 (z and z1 may be the same
// array); the partial sums of the squared M-norm sum WJ z1^2 are left in
// partial[0 .. axpy_norm_blocks(L)) for launch_givens
template <typename R>
void launch_axpy_norm(int64_t L, int nv, const R* V, int64_t ldv, const double* raw, const double* s, const R* z,
                      R* z1, const R* WJ, double* partial, hipStream_t st, const int* ctrl = nullptr,
                      WSrc ws = WSrc());

// State of one restarted-GMRES cycle kept on the device (restart length <= GM).
constexpr int GM = 32;
struct GState {
    double H[(GM + 1) * GM];   // Hessenberg matrix, row i column j at H[i * GM + j], rotated in place
    double g[GM + 1];          // rotated right-hand side |r0| e_1
    double cs[GM], sn[GM];     // Givens rotations
    double sv[GM + 1];         // basis scales: V_i / |V_i| = sv_i V_i
    double tolb;               // stop when |g_{j+1}| <= tolb (unless fixed)
    int status;                // 0 running, 1 stopped, 2 second Gram-Schmidt pass needed, 3 non-finite
    int k;                     // columns completed in this cycle
    int its;                   // matrix-vector products of the whole solve
    int maxit, fixed;
    float svf[GM + 1];         // binary32 copies of sv
};
// Column j: raw = first-pass projections <V_i, z> (i <= j) and raw[j+1] = |z|^2;
// |z1|^2 after the update is the sum of npart[0..nb) (the partials of
// launch_axpy_norm, nb = axpy_norm_blocks(L)).
// raw2 == null: first pass (may set status 2); raw2 != null: finishes a column
// after the host's second pass.
void launch_givens(GState* G, int j, const double* raw, const double* raw2, const double* npart, int nb,
                   hipStream_t st);
int axpy_norm_blocks(int64_t L);
// x += sum_i coef[i] V_i
template <typename R>
void launch_lincomb(int64_t L, int nv, const R* V, int64_t ldv, const double* coef, R* x, hipStream_t st);
// out[0] = sum WJ a^2 ; (a may be null -> uses b) generic weighted dot of two vectors
void launch_wdot(int64_t L, const double* a, const double* b, const double* WJ, double* partial, double* out,
                 hipStream_t st);
// Picard variation: out[0] = sum WJ (dp^2 + gamma p rho |du|^2), out[1] = sum WJ p^2
void launch_picard_var(int64_t L, const double* p0, const double* u0, const double* p1, const double* u1,
                       const double* rho, const double* WJ, double gamma, double* partial, double* out,
                       hipStream_t st);
// sum WJ rho (out[0]) and a non-finite flag over the state (out[1] = count);
// partial holds mass_blocks(L) x 2 doubles
void launch_mass(int64_t L, const double* q, const double* WJ, double* partial, double* out, hipStream_t st);
int mass_blocks(int64_t L);
// Geostrophic imbalance partial sums: partial[b][0] = sum W detJ |(1/rho) dp/dx - f v|,
// partial[b][1] = sum W detJ over the elements of workgroup b; returns the
// number of workgroups (at most max_blocks).
int launch_geo(const DevMesh& m, const double* q, double gm1, double fcor, double* partial, int max_blocks,
               hipStream_t st);
// Vertical-slice model: each y-line of nodes of the 5 fields of q [5][E][Np]
// replaced by its Gauss-weighted mean (in place)
void launch_slice_project(const DevMesh& m, double* q, hipStream_t st);

// conversions / vector helpers
void launch_d2f(int64_t L, const double* in, float* out, hipStream_t st);
void launch_f2d_add(int64_t L, const float* in, const double* scale, double* x, hipStream_t st);
void launch_axpby(int64_t L, double a, const double* x, double b, const double* y, double* out, hipStream_t st);
void launch_scale_store(int64_t L, const double* in, const double* s_ptr, int invert_sqrt, double* out,
                        hipStream_t st);
void launch_scale_store_f(int64_t L, const double* in, const double* s_ptr, float* out, hipStream_t st);

}  // namespace imx
