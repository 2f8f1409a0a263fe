// Host runtime of the IMEX-DG library: solver objects over a caller-owned
// device workspace, the GMRES and Picard drivers of the implicit stages, the
// IMEX-ARK2 step (Sec. 3) and the C-ABI entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

namespace imx {

static thread_local std::string g_err;
static thread_local uint64_t g_err_gen = 0;
void set_error(const std::string& msg) {
    g_err = msg;
    ++g_err_gen;
}
const std::string& thread_error() { return g_err; }
uint64_t error_generation() { return g_err_gen; }

#define HIPCHK(call)                                                        \
    do {                                                                    \
        hipError_t e_ = (call);                                             \
        if (e_ != hipSuccess) {                                             \
            set_error(std::string(#call) + ": " + hipGetErrorString(e_));   \
            return IMX_EHIP;                                                \
        }                                                                   \
    } while (0)

#define CHK(call)                         \
    do {                                  \
        imx_status s_ = (call);           \
        if (s_ != IMX_OK) return s_;      \
    } while (0)

// Key of a captured chunk of Krylov columns: everything its launches take by
// value or point at, zero-filled first so that two keys compare bytewise.
struct ChunkKey {
    int prec;                  // 0: binary64 Krylov loop, 1: binary32 inner loop
    int j0, jend, scheme;
    const void *V, *WJ, *a, *b, *c;   // basis, weights, matvec stage buffers
    double c_dt, beta, gamma, g, hfac, igm1, rot_si;
};
static ChunkKey chunk_key(int prec, const void* V, const void* WJ, const void* a, const void* b, const void* c,
                          const StageK& k) {
    ChunkKey key;
    std::memset(&key, 0, sizeof(key));
    key.prec = prec;
    key.scheme = k.scheme;
    key.V = V;
    key.WJ = WJ;
    key.a = a;
    key.b = b;
    key.c = c;
    key.c_dt = k.c_dt;
    key.beta = k.beta;
    key.gamma = k.gamma;
    key.g = k.g;
    key.hfac = k.hfac;
    key.igm1 = k.igm1;
    key.rot_si = k.rot_si;
    return key;
}

// Scratch of the allocation-free entry point imx_total_mass_noalloc: the
// mass reduction's per-workgroup partial sums (at most RED_BLOCKS workgroups
// of 2 values, whatever the mesh size). Each GPU holds its own copy until the
// process ends. Host code never uses the array's name as a device address:
// its address on each device is taken once with hipGetSymbolAddress (with that
// device current) and kept in g_scratch_dev.
constexpr size_t NOALLOC_SCRATCH_DOUBLES = (size_t)RED_BLOCKS * 2;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on `device`, which must be the current device;
// looked up on the first call per device.
static imx_status noalloc_scratch(int device, double** out) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) {
        set_error("allocation-free scratch: device index out of range");
        return IMX_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error(std::string("allocation-free scratch: hipGetSymbolAddress: ") + hipGetErrorString(e));
            return IMX_EHIP;
        }
        g_scratch_dev[device] = (double*)ptr;
    }
    *out = g_scratch_dev[device];
    return IMX_OK;
}

// Butcher tableaux of Sec. 3 (explicit / implicit), chi = 2 - sqrt(2), a32 = 1/2.
struct Tableau {
    double a[3][3], at[3][3], b[3];
    Tableau() {
        const double chi = 2.0 - std::sqrt(2.0);
        std::memset(this, 0, sizeof(*this));
        a[1][0] = chi;
        a[2][0] = 0.5;
        a[2][1] = 0.5;
        at[1][0] = at[1][1] = chi / 2;
        at[2][0] = at[2][1] = 0.5 - chi / 4;
        at[2][2] = chi / 2;
        b[0] = b[1] = 0.5 - chi / 4;
        b[2] = chi / 2;
    }
};
static const Tableau TAB;

}  // namespace imx

using namespace imx;

struct imx_solver {
    const double* starget = nullptr;   // caller's state the damping layers relax towards (null: momentum only)
    const Mesh* mesh = nullptr;
    imx_phys phys{};
    imx_numerics num{};
    hipStream_t st = nullptr;
    int device = 0;
    int64_t E = 0, L = 0, Lp = 0;
    int Np = 0, Nf = 0, m = 30;   // m: GMRES restart length in use
    int m_cap = 30;               // restart length the workspace was laid out for
    bool bound = false, mixed = false;
    mutable std::string err;      // last error raised by a call on this solver
    size_t ws_bytes = 0;
    char* ws = nullptr;
    DevMesh dm;
    HostTab tab{};
    // binary64 buffers
    double *y = nullptr, *ybak = nullptr, *Y = nullptr;
    double *fN[3] = {}, *fS[3] = {};
    double *rho = nullptr, *Fh = nullptr, *G0h = nullptr, *Gp = nullptr;
    double *p = nullptr, *pn = nullptr, *u = nullptr, *un = nullptr, *w = nullptr;
    double *FB = nullptr, *FBh = nullptr;
    double *V = nullptr, *z = nullptr, *z1 = nullptr, *b = nullptr;
    double *partial = nullptr, *partial2 = nullptr, *dsc = nullptr;   // reduction scratch, device scalars
    // binary32 shadows for the mixed inner loop
    float *Vf = nullptr, *zf = nullptr, *z1f = nullptr, *wf = nullptr, *FBf = nullptr, *FBhf = nullptr;
    float *rhof = nullptr, *pkf = nullptr, *WJf = nullptr, *Gf = nullptr, *nSf = nullptr, *xf = nullptr;
    double* cr = nullptr;    // 1 / (WJ rho_l) of the current stage
    float* crf = nullptr;
    double* w3 = nullptr;    // tensor weights w_i w_j w_k of the nodes (Np)
    WSrc wsrc;               // affine meshes: Krylov weights from w3 and det J instead of WJ
    GState* gst = nullptr;   // device state of the running Krylov cycle
    GState* hgs = nullptr;   // pinned host copies: [0] upload, [1] download
    // pinned host scalars
    double* hsc = nullptr;
    // captured Krylov chunks (imx_solver_set_graphs): replayed on st, captured on cst
    bool graphs = false;
    hipStream_t cst = nullptr;
    hipStream_t side = nullptr;           // meshes with hanging faces: see DevMesh::side
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::vector<std::pair<ChunkKey, hipGraphExec_t>> chunk_graphs;
    // kernel timing (imx_solver_timing)
    bool timing = false;
    struct TRec { int kind; hipEvent_t a, b; double bytes; };
    std::vector<TRec> trec;
    std::vector<hipEvent_t> tpool;
    double t_ms[IMX_K_COUNT] = {}, t_bytes[IMX_K_COUNT] = {};
    int64_t t_count[IMX_K_COUNT] = {};
    // device scalar slots (offsets into dsc)
    enum { S_RAW1 = 0, S_RAW2 = 64, S_COEF = 256, S_MISC = 320, S_N = 384 };
};

namespace imx {

struct Layout {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    }
};

// Computes (and with base != null, assigns) the workspace layout.
static size_t layout(imx_solver* s, char* base) {
    Layout Lo;
    const int64_t L = s->L, E = s->E;
    const int Np = s->Np, Nf = s->Nf;
    const Mesh& m = *s->mesh;
    auto D = [&](size_t n) -> double* { size_t o = Lo.take(n * sizeof(double)); return base ? (double*)(base + o) : nullptr; };
    auto F = [&](size_t n) -> float* { size_t o = Lo.take(n * sizeof(float)); return base ? (float*)(base + o) : nullptr; };
    auto I = [&](size_t n) -> int* { size_t o = Lo.take(n * sizeof(int)); return base ? (int*)(base + o) : nullptr; };
    DevMesh& dm = s->dm;
    dm.kind = I(E * 6);
    dm.nbr = I(E * 6);
    dm.aux = I(E * 6);
    dm.hang = I(std::max<int64_t>(m.nh, 1) * 4);
    {
        int64_t nc = 0;
        for (int64_t e = 0; e < E; ++e) {
            bool c = false;
            for (int f = 0; f < 6; ++f) c |= m.fkind[6 * e + f] == COARSE;
            nc += c;
        }
        dm.ncoarse = nc;
        if (nc) {
            dm.reg_list = I(E - nc + 1);
            dm.crs_list = I(nc);
        }
    }
    dm.h = D(E * 3);
    dm.hinv = D(E * 3);
    dm.tab = D(tab_bytes(m.n, 0) / 8 + 1);
    dm.fofs = (const uint64_t*)D(fofs_count(m.n));
    dm.tabf = D(tab_bytes(m.n, 1) / 8 + 1);
    dm.WJ = D(s->Lp);
    dm.eg = D(E * 8);
    s->w3 = D(Np);
    if (m.deformed) {
        dm.G = D(5 * L);
        dm.nS = D((size_t)E * 10 * Nf);
        dm.iWJ = D(L);
        if (m.nh == 0) dm.cm = D((size_t)E * cm_stride(m.n));
    }
    s->cr = D(L);
    if (s->phys.sponge_lambda != 0.0) dm.sponge = D(L);
    s->y = D(5 * L);
    s->ybak = D(5 * L);
    s->Y = D(5 * L);
    for (int l = 0; l < 3; ++l) {
        s->fN[l] = D(5 * L);
        s->fS[l] = D(4 * L);
    }
    s->rho = D(L);
    s->Fh = D(3 * L);
    s->G0h = D(L);
    s->Gp = D(L);
    s->p = D(s->Lp);
    s->pn = D(s->Lp);
    s->u = D(3 * L);
    s->un = D(3 * L);
    s->w = D(3 * L);
    s->FB = D((size_t)E * 6 * Nf);
    s->FBh = D(std::max<int64_t>(m.nh, 1) * 4 * Nf);
    s->V = D((size_t)(s->m_cap + 1) * s->Lp);
    s->z = D(s->Lp);
    s->z1 = D(s->Lp);
    s->b = D(L);
    s->partial = D((size_t)RED_BLOCKS * MAXV + (size_t)RED_BLOCKS * 34);
    s->partial2 = D(pass2_partial_count(s->dm));
    s->dsc = D(imx_solver::S_N);
    {
        size_t o = Lo.take(sizeof(GState));
        s->gst = base ? (GState*)(base + o) : nullptr;
    }
    if (s->mixed) {
        s->Vf = F((size_t)(s->m_cap + 1) * s->Lp);
        s->zf = F(L);
        s->z1f = F(L);
        s->wf = F(3 * L);
        s->FBf = F((size_t)E * 6 * Nf);
        s->FBhf = F(std::max<int64_t>(m.nh, 1) * 4 * Nf);
        s->rhof = F(L);
        s->pkf = F(L);
        s->xf = F(s->Lp);
        s->WJf = F(s->Lp);
        s->crf = F(L);
        dm.WJf = s->WJf;
        if (m.deformed) {
            s->Gf = F(5 * L);
            s->nSf = F((size_t)E * 10 * Nf);
            dm.Gf = s->Gf;
            dm.nSf = s->nSf;
            dm.iWJf = F(L);
            if (m.nh == 0) dm.cmf = F((size_t)E * cm_stride(m.n));
        }
    }
    return Lo.off;
}

static imx_status validate_num(const imx_numerics& n) {
    if (!(n.dt > 0) || (n.scheme != IMX_R1 && n.scheme != IMX_R2) ||
        (n.precision != IMX_FP64 && n.precision != IMX_MIXED) || n.picard_max < 1 || n.gmres_max < 1 ||
        n.gmres_restart < 1 || n.gmres_restart > MAXV - 1 || !(n.gmres_tol >= 0) || !(n.picard_tol >= 0)) {
        set_error("invalid numerics (dt > 0, scheme R1/R2, 1 <= gmres_restart <= 32, positive caps)");
        return IMX_EINVAL;
    }
    if (n.precision == IMX_MIXED && !(n.inner_tol > 0 && n.inner_tol < 1)) {
        set_error("IMX_MIXED needs 0 < inner_tol < 1");
        return IMX_EINVAL;
    }
    return IMX_OK;
}

static StageK stage_k(const imx_solver* s, double a_ll) {
    StageK k;
    k.c_dt = a_ll * s->num.dt;
    k.beta = a_ll * s->num.dt * s->phys.f;
    k.gamma = s->phys.gamma;
    k.g = s->phys.g;
    k.hfac = s->phys.gamma / (s->phys.gamma - 1.0);
    k.igm1 = 1.0 / (s->phys.gamma - 1.0);
    k.rot_si = 1.0 / (1.0 + k.beta * k.beta);
    k.scheme = s->num.scheme;
    return k;
}

static imx_status sync_read(imx_solver* s, const double* dev, int n) {
    HIPCHK(hipMemcpyAsync(s->hsc, dev, n * sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return IMX_OK;
}

static imx_status put_scalars(imx_solver* s, double* dev, const double* vals, int n, int slot) {
    // each slot of the pinned buffer is written once before its copy is queued
    double* h = s->hsc + 512 + slot;
    std::memcpy(h, vals, n * sizeof(double));
    HIPCHK(hipMemcpyAsync(dev, h, n * sizeof(double), hipMemcpyHostToDevice, s->st));
    return IMX_OK;
}

// ----------------------------------------------------------- kernel timing
static void timing_flush(imx_solver* s) {
    if (s->trec.empty()) return;
    (void)hipStreamSynchronize(s->st);
    for (auto& r : s->trec) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, r.a, r.b);
        s->t_ms[r.kind] += ms;
        s->t_bytes[r.kind] += r.bytes;
        s->t_count[r.kind] += 1;
        s->tpool.push_back(r.a);
        s->tpool.push_back(r.b);
    }
    s->trec.clear();
}

static hipEvent_t timing_event(imx_solver* s) {
    if (s->tpool.empty()) {
        if (s->trec.size() > 4096) timing_flush(s);
        if (s->tpool.empty()) {
            hipEvent_t e;
            // no system-scope fences: these events only time kernels on the device
            (void)hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
            return e;
        }
    }
    hipEvent_t e = s->tpool.back();
    s->tpool.pop_back();
    return e;
}

// Runs `launch` (a kernel launch on s->st), bracketed by events when timing.
template <typename Fn>
static void timed(imx_solver* s, int kind, double bytes, Fn&& launch) {
    if (!s->timing) {
        launch();
        return;
    }
    imx_solver::TRec r{kind, timing_event(s), timing_event(s), bytes};
    (void)hipEventRecord(r.a, s->st);
    launch();
    (void)hipEventRecord(r.b, s->st);
    s->trec.push_back(r);
}

// algorithmic bytes of one launch: nfields nodal fields of the element kernels
// plus the stored geometry of terrain-following elements
static double field_bytes(const imx_solver* s, double nfields, bool geometry) {
    double b = nfields * (double)s->L * 8.0;
    // stored geometry of a terrain-following element: W detJ (or its inverse),
    // 5 entries of W cof(J) per node, 10 n dS values per face point
    if (geometry && s->mesh->deformed) b += (double)s->E * (6.0 * s->Np + 10.0 * s->Nf) * 8.0;
    return b;
}

// algorithmic bytes of the matrix-vector product's two passes. Pass 1 reads
// x, rho_l (as cr) and p^k (and rho_l itself for R2 on terrain-following
// meshes) and the geometry, and writes the element's own part of pass 2
// (1 field: volume divergence of (rho h)^k w and the R2 gravity term); pass 2
// reads x and that field (and W detJ^{-1} on terrain-following meshes) and
// writes S x. The face buffers are not counted. Where the mesh has the
// compact terrain metric, pass 1 reads it (cm_stride(n) values and h_x, h_y per
// element) in place of the stored geometry, and pass 2 forms W detJ^{-1} from
// its J22 values (Nf and h_x, h_y per element).
static double mv1_bytes(const imx_solver* s, int scheme) {
    const double nf = 4.0 + (s->mesh->deformed && scheme == 2 ? 1.0 : 0.0);
    if (s->dm.cm) return nf * (double)s->L * 8.0 + (double)s->E * (cm_stride(s->mesh->n) + 2.0) * 8.0;
    return field_bytes(s, nf, true);
}
static double mv2_bytes(const imx_solver* s) {
    if (s->dm.cm) return 3.0 * (double)s->L * 8.0 + (double)s->E * (s->Nf + 2.0) * 8.0;
    return field_bytes(s, 3.0 + (s->mesh->deformed ? 1.0 : 0.0), false);
}

// ------------------------------------------------------------ stage context
struct StageCtx {
    StageK k;
    const double* Fh;   // primal momentum right-hand side (M^{-1}(f - f_g))
    const double* Gp;   // primal energy right-hand side (M^{-1}(g - Lambda - k ...))
    const double* pk;   // lagged pressure
    const double* uk;   // lagged velocity (R1)
    const double* rho;
};

// r = M^{-1}(RHS - S x) with x scaled by *xs (device) if xs != null
static void residual(imx_solver* s, const StageCtx& c, const double* x, const double* xs, double* out) {
    const double n1 = (x ? 1 : 0) + 3 + 1 + 3 + (c.k.scheme == 1 ? 3 : 0);   // x, Fh, rho, w (, uk)
    timed(s, IMX_K_PASS1, field_bytes(s, n1, true), [&] {
        launch_pass1<double>(s->dm, s->tab, c.k, x, xs, c.Fh, c.rho, c.pk, c.uk, s->w, s->FB, s->FBh, s->st);
    });
    const double n2 = 1 + (x ? 1 : 0) + 3 + 1 + (c.k.scheme == 2 ? 1 : 0) + 1;   // Gp, x, w, pk, rho, out
    timed(s, IMX_K_PASS2, field_bytes(s, n2, true), [&] {
        launch_pass2<double>(s->dm, s->tab, c.k, c.Gp, x, xs, s->w, c.pk, c.rho, s->FB, s->FBh, out, 1.0, 0, s->st);
    });
}

// r = M^{-1}(RHS - S x) as b - M^{-1} S x, with b = M^{-1} RHS formed once per
// solve (s->b): the Krylov loop's own matrix-vector kernels and one axpby
// instead of the right-hand-side passes
static void residual_b(imx_solver* s, const StageCtx& c, const double* x, double* out) {
    timed(s, IMX_K_PASS1, mv1_bytes(s, c.k.scheme), [&] {
        launch_mv1<double>(s->dm, c.k, x, nullptr, s->cr, c.rho, c.pk, s->w, s->FB, s->FBh, s->st);
    });
    timed(s, IMX_K_PASS2, mv2_bytes(s), [&] {
        launch_mv2<double>(s->dm, c.k, x, nullptr, s->w, c.pk, c.rho, s->FB, s->FBh, out, 0, s->st);
    });
    timed(s, IMX_K_STAGE, 3 * (double)s->L * 8.0, [&] { launch_axpby(s->L, 1.0, s->b, -1.0, out, out, s->st); });
}

struct GmresOut {
    int its = 0;
    double relres = 0.0;
};

static void drop_chunk_graphs(imx_solver* s) {
    for (auto& e : s->chunk_graphs) (void)hipGraphExecDestroy(e.second);
    s->chunk_graphs.clear();
}

// The replayable graph of one chunk of Krylov columns: looked up by key, else
// captured from `body` on the solver's capture stream (thread-local capture, so
// other solvers' threads are not affected) and instantiated.
template <typename F>
static imx_status chunk_graph(imx_solver* s, const ChunkKey& key, F&& body, hipGraphExec_t& ex) {
    for (auto& e : s->chunk_graphs)
        if (std::memcmp(&e.first, &key, sizeof(ChunkKey)) == 0) {
            ex = e.second;
            return IMX_OK;
        }
    if (s->chunk_graphs.size() >= 128) drop_chunk_graphs(s);
    if (!s->cst) HIPCHK(hipStreamCreateWithFlags(&s->cst, hipStreamNonBlocking));
    hipStream_t run = s->st;
    s->st = s->cst;
    hipError_t e = hipStreamBeginCapture(s->cst, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) body();
    hipGraph_t g = nullptr;
    const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(s->cst, &g) : e;
    s->st = run;
    if (e2 != hipSuccess) {
        set_error(std::string("Krylov chunk capture: ") + hipGetErrorString(e2));
        return IMX_EHIP;
    }
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        set_error(std::string("Krylov chunk instantiation: ") + hipGetErrorString(e));
        return IMX_EHIP;
    }
    s->chunk_graphs.emplace_back(key, ex);
    return IMX_OK;
}

// One cycle of GMRES(m) on the device (Saad, Alg. 6.9) from V_0 = r0 (unscaled,
// |r0|_M = beta): for each column the matrix-vector product, one classical
// Gram-Schmidt pass (projections and |z|^2 in one read of the basis, then the
// update and |z1|^2), and the Givens step in one workgroup. The host queues
// the columns in chunks and reads the cycle state once per chunk; kernels of
// a cycle that has stopped return at once. A column with severe cancellation
// (|z1|^2 < 1e-6 |z|^2) stops the chunk and gets a second pass from the host.
// `mv(j, x, xs_d, xs_f, out, ctrl)` queues out = A (xs x). With `key` (and
// graphs on, kernel timing off) each chunk's launches are captured once into
// a HIP graph and replayed: the chunk is a fixed launch sequence whose
// arguments the key lists, and its kernels read the stop flag on the device.
template <typename R, typename MV>
static imx_status arnoldi_cycle(imx_solver* s, R* V, const R* WJ, int m, double beta, double tolb, int its0,
                                int maxit, bool fixed, MV&& mv, const GState*& out, const ChunkKey* key = nullptr) {
    const int64_t L = s->Lp;
    GState* G = s->gst;
    GState* up = s->hgs;
    GState* dn = s->hgs + 1;
    double* raw1 = s->dsc + imx_solver::S_RAW1;
    double* raw2 = s->dsc + imx_solver::S_RAW2;
    std::memset(up, 0, sizeof(GState));
    up->g[0] = beta;
    up->sv[0] = 1.0 / beta;
    up->svf[0] = (float)up->sv[0];
    up->tolb = tolb;
    up->its = its0;
    up->maxit = maxit;
    up->fixed = fixed ? 1 : 0;
    HIPCHK(hipMemcpyAsync(G, up, sizeof(GState), hipMemcpyHostToDevice, s->st));
    const int* ctrl = &G->status;
    const double vb = (double)L * sizeof(R);
    auto column = [&](int j, const double* raw2p, const int* c) {
        R* Vn = V + (size_t)(j + 1) * L;
        double* raw = raw2p ? raw2 : raw1;
        const int nd = raw2p ? j + 1 : j + 2;   // the second pass needs no |z|^2
        // the weight vector, unless taken from the tables (with the compact
        // metric, binary64 only: the J22 plane of each element)
        const double wb = s->wsrc.cm ? (sizeof(R) == 8 ? (double)s->E * s->Nf * 8.0 : vb) : (s->wsrc.W3 ? 0.0 : vb);
        timed(s, IMX_K_DOTS, nd * vb + wb,
              [&] { launch_dots<R>(L, nd, V, L, Vn, WJ, s->partial, raw, s->st, c, s->wsrc); });
        timed(s, IMX_K_ORTHO, (j + 3) * vb + wb, [&] {
            launch_axpy_norm<R>(L, j + 1, V, L, raw, G->sv, Vn, Vn, WJ, s->partial, s->st, c, s->wsrc);
        });
        launch_givens(G, j, raw1, raw2p, s->partial, axpy_norm_blocks(L), s->st);
    };
    constexpr int CHUNK = 8;
    int j = 0;
    while (j < m) {
        const int jend = std::min(m, j + CHUNK);
        auto chunk = [&] {
            for (int jj = j; jj < jend; ++jj) {
                mv(jj, V + (size_t)jj * L, &G->sv[jj], &G->svf[jj], V + (size_t)(jj + 1) * L, ctrl);
                column(jj, nullptr, ctrl);
            }
        };
        if (key && s->graphs && !s->timing) {
            ChunkKey k = *key;
            k.j0 = j;
            k.jend = jend;
            hipGraphExec_t ex = nullptr;
            CHK(chunk_graph(s, k, chunk, ex));
            HIPCHK(hipGraphLaunch(ex, s->st));
        } else {
            chunk();
        }
        HIPCHK(hipMemcpyAsync(dn, G, sizeof(GState), hipMemcpyDeviceToHost, s->st));
        HIPCHK(hipStreamSynchronize(s->st));
        if (dn->status == 2) {
            const int jc = dn->k;
            column(jc, raw2, nullptr);
            HIPCHK(hipMemcpyAsync(dn, G, sizeof(GState), hipMemcpyDeviceToHost, s->st));
            HIPCHK(hipStreamSynchronize(s->st));
            j = jc + 1;
            if (dn->status != 0) break;
            continue;
        }
        if (dn->status != 0) break;
        j = jend;
    }
    out = dn;
    if (dn->status == 3) {
        set_error("GMRES: non-finite Krylov vector");
        return IMX_ENONFINITE;
    }
    return IMX_OK;
}

// y = H^{-1} g (upper triangular k x k of a finished cycle), coefficients y_i sv_i
static void cycle_coefficients(const GState& G, int k, double* cf) {
    double yv[GM];
    for (int i = k - 1; i >= 0; --i) {
        double t = G.g[i];
        for (int l = i + 1; l < k; ++l) t -= G.H[i * GM + l] * yv[l];
        yv[i] = t / G.H[i * GM + i];
    }
    for (int i = 0; i < k; ++i) cf[i] = yv[i] * G.sv[i];
}

// Restarted GMRES(m) for A x = b, A = M^{-1} S, in the M inner product. x:
// initial guess in, solution out. Stops when the Givens residual estimate
// reaches tol*|b| (unless `fixed`), after maxit products, or on breakdown;
// every restart recomputes the true residual.
static imx_status gmres(imx_solver* s, const StageCtx& c, double* x, double bnorm, double tol, int maxit,
                        bool fixed, GmresOut& out) {
    const int64_t L = s->Lp;   // Krylov vector stride (element kernels touch the first E*Np)
    double* V = s->V;
    double* coef = s->dsc + imx_solver::S_COEF;
    double* bb = s->dsc + imx_solver::S_MISC;
    residual_b(s, c, x, V);
    timed(s, IMX_K_REDUCE, 2 * (double)L * 8.0,
          [&] { launch_wdot(L, V, nullptr, s->dm.WJ, s->partial, bb, s->st); });
    CHK(sync_read(s, bb, 1));
    double beta = std::sqrt(s->hsc[0]);
    int its = 0;
    auto mv = [&](int, const double* xj, const double* xs, const float*, double* o, const int* ctrl) {
        timed(s, IMX_K_PASS1, mv1_bytes(s, c.k.scheme), [&] {
            launch_mv1<double>(s->dm, c.k, xj, xs, s->cr, c.rho, c.pk, s->w, s->FB, s->FBh, s->st, ctrl);
        });
        timed(s, IMX_K_PASS2, mv2_bytes(s), [&] {
            launch_mv2<double>(s->dm, c.k, xj, xs, s->w, c.pk, c.rho, s->FB, s->FBh, o, 0, s->st, ctrl);
        });
    };
    while (true) {
        if (!std::isfinite(beta)) {
            set_error("GMRES: non-finite residual");
            return IMX_ENONFINITE;
        }
        if (beta == 0.0 || its >= maxit || (!fixed && beta <= tol * bnorm)) break;
        const GState* G = nullptr;
        const ChunkKey key = chunk_key(0, V, s->dm.WJ, s->cr, c.rho, c.pk, c.k);
        CHK(arnoldi_cycle<double>(s, V, s->dm.WJ, s->m, beta, tol * bnorm, its, maxit, fixed, mv, G, &key));
        const int k = G->k;
        its = G->its;
        double cf[GM];
        cycle_coefficients(*G, k, cf);
        CHK(put_scalars(s, coef, cf, k, 100));
        timed(s, IMX_K_LINCOMB, (k + 2) * (double)L * 8.0,
              [&] { launch_lincomb<double>(L, k, V, L, coef, x, s->st); });
        residual_b(s, c, x, V);
        timed(s, IMX_K_REDUCE, 2 * (double)L * 8.0,
              [&] { launch_wdot(L, V, nullptr, s->dm.WJ, s->partial, bb, s->st); });
        CHK(sync_read(s, bb, 1));
        beta = std::sqrt(s->hsc[0]);
    }
    out.its = its;
    out.relres = bnorm > 0 ? beta / bnorm : 0.0;
    return IMX_OK;
}

// Solves the pressure system of the current stage context for x (initial
// guess in, solution out) to gmres_tol.

// One binary32 Arnoldi cycle (at most `maxit` steps) of GMRES for the
// correction equation A d = r / |r|, started from d = 0 with Vf[0] holding
// r / |r| (M-norm ~ 1). Accumulates d into s->xf. Returns the step count.
static imx_status inner_cycle_f32(imx_solver* s, const StageK& k, double beta, double tol, int maxit, int& steps) {
    const int64_t L = s->Lp;
    const int m = std::min(s->m, maxit);
    double* coef = s->dsc + imx_solver::S_COEF;
    auto mv = [&](int, const float* xj, const double*, const float* xs, float* o, const int* ctrl) {
        timed(s, IMX_K_PASS1, mv1_bytes(s, k.scheme) / 2, [&] {
            launch_mv1<float>(s->dm, k, xj, xs, s->crf, s->rhof, s->pkf, s->wf, s->FBf, s->FBhf, s->st, ctrl);
        });
        timed(s, IMX_K_PASS2, mv2_bytes(s) / 2, [&] {
            launch_mv2<float>(s->dm, k, xj, xs, s->wf, s->pkf, s->rhof, s->FBf, s->FBhf, o, 0, s->st, ctrl);
        });
    };
    const GState* G = nullptr;
    const ChunkKey key = chunk_key(1, s->Vf, s->WJf, s->crf, s->rhof, s->pkf, k);
    CHK(arnoldi_cycle<float>(s, s->Vf, s->WJf, m, beta, tol * beta, 0, m, false, mv, G, &key));
    const int kk = G->k;
    double cf[GM];
    cycle_coefficients(*G, kk, cf);
    CHK(put_scalars(s, coef, cf, kk, 100));
    timed(s, IMX_K_LINCOMB, (kk + 2) * (double)L * 4.0,
          [&] { launch_lincomb<float>(L, kk, s->Vf, L, coef, s->xf, s->st); });
    steps = kk;
    return IMX_OK;
}

// Mixed precision: binary64 defect correction x += |r| d, r = b - A x formed
// in binary64, d from one binary32 GMRES cycle on A d = r/|r| to the relative
// reduction inner_tol; stops on the same binary64 criterion as the plain path.
static imx_status pressure_solve_mixed(imx_solver* s, const StageCtx& c, double* x, double bnorm, GmresOut& out) {
    const int64_t L = s->L;
    double* bb = s->dsc + imx_solver::S_MISC;
    timed(s, IMX_K_STAGE, 4 * (double)L * 12.0, [&] {
        launch_d2f(L, c.rho, s->rhof, s->st);
        launch_d2f(L, c.pk, s->pkf, s->st);
    });
    const bool fixed = s->num.fixed_iterations != 0;
    int total = 0;
    double rel = 0.0;
    for (int outer = 0;; ++outer) {
        residual_b(s, c, x, s->z1);
        timed(s, IMX_K_REDUCE, 2 * (double)L * 8.0,
              [&] { launch_wdot(L, s->z1, nullptr, s->dm.WJ, s->partial, bb, s->st); });
        CHK(sync_read(s, bb, 1));
        const double rn = std::sqrt(s->hsc[0]);
        rel = bnorm > 0 ? rn / bnorm : 0.0;
        if (!std::isfinite(rn)) {
            set_error("mixed GMRES: non-finite residual");
            return IMX_ENONFINITE;
        }
        if (rn == 0.0 || total >= s->num.gmres_max || (!fixed && rn <= s->num.gmres_tol * bnorm)) break;
        // Vf[0] = r / |r| in binary32, d = 0
        const double inv = 1.0 / rn;
        CHK(put_scalars(s, bb + 1, &inv, 1, 300));
        timed(s, IMX_K_STAGE, (double)L * 12.0, [&] {
            launch_scale_store_f(L, s->z1, bb + 1, s->Vf, s->st);
            (void)hipMemsetAsync(s->xf, 0, s->Lp * sizeof(float), s->st);
        });
        int steps = 0;
        CHK(inner_cycle_f32(s, c.k, 1.0, s->num.inner_tol, s->num.gmres_max - total, steps));
        total += steps;
        CHK(put_scalars(s, bb + 2, &rn, 1, 301));
        timed(s, IMX_K_STAGE, (double)L * 20.0, [&] { launch_f2d_add(L, s->xf, bb + 2, x, s->st); });
        if (steps == 0) break;
    }
    out.its = total;
    out.relres = rel;
    return IMX_OK;
}

static imx_status pressure_solve(imx_solver* s, const StageCtx& c, double* x, GmresOut& out) {
    const int64_t L = s->L;
    double* bb = s->dsc + imx_solver::S_MISC;
    // |b|_M with b = M^{-1} RHS: the residual at x = 0
    residual(s, c, nullptr, nullptr, s->b);
    timed(s, IMX_K_REDUCE, 2 * (double)L * 8.0,
          [&] { launch_wdot(L, s->b, nullptr, s->dm.WJ, s->partial, bb, s->st); });
    CHK(sync_read(s, bb, 1));
    const double bnorm = std::sqrt(s->hsc[0]);
    if (s->num.precision == IMX_MIXED) return pressure_solve_mixed(s, c, x, bnorm, out);
    return gmres(s, c, x, bnorm, s->num.gmres_tol, s->num.gmres_max, s->num.fixed_iterations != 0, out);
}

// Picard iteration on the stage system; p, u: initial iterate in, result out.
static imx_status stage_solve(imx_solver* s, double a_ll, const double* rho, const double* Fh, const double* G0h,
                              double*& p, double*& u, double*& pn, double*& un, imx_solve_stats* st) {
    const int64_t L = s->L;
    const bool fixed = s->num.fixed_iterations != 0;
    StageK k = stage_k(s, a_ll);
    imx_solve_stats stats{};
    timed(s, IMX_K_STAGE, (double)L * (s->mixed ? 28.0 : 24.0),
          [&] { launch_stage_coef(L, rho, s->dm.WJ, s->cr, s->mixed ? s->crf : nullptr, s->st); });
    bool converged = false;
    double* bb = s->dsc + imx_solver::S_MISC;
    for (int it = 0; it < s->num.picard_max; ++it) {
        timed(s, IMX_K_LAMBDA, field_bytes(s, 8, true),
              [&] { launch_lambda(s->dm, s->tab, k, p, u, rho, G0h, s->Gp, s->st); });
        StageCtx c{k, Fh, s->Gp, p, u, rho};
        HIPCHK(hipMemcpyAsync(pn, p, L * sizeof(double), hipMemcpyDeviceToDevice, s->st));
        GmresOut go;
        CHK(pressure_solve(s, c, pn, go));
        // velocity recovery from the momentum equation
        timed(s, IMX_K_PASS1, field_bytes(s, 1 + 3 + 1 + 3 + (k.scheme == 1 ? 3 : 0), true), [&] {
            launch_pass1<double>(s->dm, s->tab, k, pn, nullptr, Fh, rho, p, u, un, nullptr, nullptr, s->st);
        });
        timed(s, IMX_K_REDUCE, 10 * (double)L * 8.0, [&] {
            launch_picard_var(L, p, u, pn, un, rho, s->dm.WJ, s->phys.gamma, s->partial, bb, s->st);
        });
        CHK(sync_read(s, bb, 2));
        const double var = std::sqrt(s->hsc[0] / s->hsc[1]);
        std::swap(p, pn);
        std::swap(u, un);
        stats.picard_iters++;
        stats.gmres_iters += go.its;
        stats.gmres_relres = go.relres;
        stats.picard_variation = var;
        if (!std::isfinite(var)) {
            if (st) *st = stats;
            set_error("Picard: non-finite iterate");
            return IMX_ENONFINITE;
        }
        if (!fixed && var <= s->num.picard_tol) {
            converged = true;
            break;
        }
    }
    if (st) *st = stats;
    if (!fixed && !converged) {
        set_error("Picard iteration did not converge within picard_max");
        return IMX_ENOCONV;
    }
    return IMX_OK;
}

static PhysK phys_k(const imx_solver* s) {
    PhysK k;
    k.gamma = s->phys.gamma;
    k.g = s->phys.g;
    k.f = s->phys.f;
    k.gm1 = s->phys.gamma - 1.0;
    k.igm1 = 1.0 / (s->phys.gamma - 1.0);
    k.hfac = s->phys.gamma / (s->phys.gamma - 1.0);
    for (int c = 0; c < 3; ++c) k.su[c] = s->phys.sponge_u[c];
    // with a target state the element kernels leave the layers out and the
    // relaxation of the whole state follows them (explicit_eval)
    k.sponge = s->phys.sponge_lambda != 0.0 && !s->starget;
    return k;
}

// T_NS and T_S of Sec. 3 at q as nodal tendencies; the damping layers relax
// the momentum inside the element kernels, or the whole state afterwards
static void explicit_eval(imx_solver* s, const PhysK& ph, const double* q, double* fN, double* fS) {
    launch_explicit<double>(s->dm, s->tab, ph, q, fN, fS, s->st);
    if (s->starget && s->dm.sponge) launch_sponge_relax(s->L, q, s->starget, s->dm.sponge, fN, s->st);
}

static imx_status one_step(imx_solver* s, imx_step_stats* acc) {
    const int64_t L = s->L;
    const double dt = s->num.dt;
    const PhysK ph = phys_k(s);
    HIPCHK(hipMemcpyAsync(s->ybak, s->y, 5 * L * sizeof(double), hipMemcpyDeviceToDevice, s->st));
    timed(s, IMX_K_EXPLICIT, field_bytes(s, 14 + (ph.sponge ? 1 : 0), true),
          [&] { explicit_eval(s, ph, s->y, s->fN[0], s->fS[0]); });
    for (int l = 1; l <= 2; ++l) {
        StageCoef c{};
        for (int mm = 0; mm < l; ++mm) {
            c.a[mm] = TAB.a[l][mm];
            c.at[mm] = TAB.at[l][mm];
        }
        c.l = l;
        c.dt = dt;
        c.c_dt = TAB.at[l][l] * dt;
        c.g = s->phys.g;
        c.gamma = s->phys.gamma;
        const double* yprev = l == 1 ? s->y : s->Y;
        timed(s, IMX_K_STAGE, (5 + 9 * l + 5 + 1 + 3 + 1 + 1 + 3) * (double)L * 8.0, [&] {
            launch_stage_prepare(L, s->y, s->fN, s->fS, yprev, c, s->rho, s->Fh, s->G0h, s->p, s->u, s->st);
        });
        imx_solve_stats ss{};
        imx_status rc = stage_solve(s, TAB.at[l][l], s->rho, s->Fh, s->G0h, s->p, s->u, s->pn, s->un, &ss);
        acc->picard_iters += ss.picard_iters;
        acc->gmres_iters += ss.gmres_iters;
        if (rc != IMX_OK) {
            (void)hipMemcpyAsync(s->y, s->ybak, 5 * L * sizeof(double), hipMemcpyDeviceToDevice, s->st);
            return rc;
        }
        timed(s, IMX_K_STAGE, 10 * (double)L * 8.0,
              [&] { launch_finalize(L, s->rho, s->p, s->u, s->phys.gamma, s->Y, s->st); });
        timed(s, IMX_K_EXPLICIT, field_bytes(s, 14 + (ph.sponge ? 1 : 0), true),
              [&] { explicit_eval(s, ph, s->Y, s->fN[l], s->fS[l]); });
    }
    timed(s, IMX_K_STAGE, (5 + 27 + 5) * (double)L * 8.0,
          [&] { launch_final_update(L, s->y, s->fN, s->fS, TAB.b, dt, s->y, s->st); });
    if (s->phys.slice)
        timed(s, IMX_K_STAGE, 10 * (double)L * 8.0, [&] { launch_slice_project(s->dm, s->y, s->st); });
    double* bb = s->dsc + imx_solver::S_MISC;
    timed(s, IMX_K_REDUCE, 6 * (double)L * 8.0, [&] { launch_mass(L, s->y, s->dm.WJ, s->partial, bb, s->st); });
    CHK(sync_read(s, bb, 2));
    if (s->hsc[1] != 0.0 || !std::isfinite(s->hsc[0])) {
        HIPCHK(hipMemcpyAsync(s->y, s->ybak, 5 * L * sizeof(double), hipMemcpyDeviceToDevice, s->st));
        HIPCHK(hipStreamSynchronize(s->st));
        set_error("non-finite state after step");
        return IMX_ENONFINITE;
    }
    acc->mass = s->hsc[0];
    acc->steps++;
    return IMX_OK;
}

}  // namespace imx

// =================================================================== C-ABI
extern "C" {

const char* imx_last_error(void) { return imx::g_err.c_str(); }

const char* imx_solver_last_error(const imx_solver* s) { return s ? s->err.c_str() : ""; }

imx_status imx_mesh_create(const imx_mesh_desc* desc, imx_mesh** out) {
    if (!desc || !out) {
        set_error("imx_mesh_create: null argument");
        return IMX_EINVAL;
    }
    imx_mesh* m = new (std::nothrow) imx_mesh;
    if (!m) return IMX_ENOMEM;
    try {
        imx_status rc = build_mesh(*desc, m->m);
        if (rc != IMX_OK) {
            delete m;
            return rc;
        }
    } catch (const std::bad_alloc&) {
        delete m;
        set_error("imx_mesh_create: out of host memory");
        return IMX_ENOMEM;
    }
    *out = m;
    return IMX_OK;
}

imx_status imx_mesh_create_box(const imx_mesh_desc* desc, imx_mesh** out) { return imx_mesh_create(desc, out); }

imx_status imx_mesh_info(const imx_mesh* mesh, int64_t* n_elem, int* nodes_per_elem, int64_t* n_hanging,
                         int* deformed) {
    if (!mesh) return IMX_EINVAL;
    if (n_elem) *n_elem = mesh->m.E;
    if (nodes_per_elem) *nodes_per_elem = mesh->m.Np;
    if (n_hanging) *n_hanging = mesh->m.nh;
    if (deformed) *deformed = mesh->m.deformed ? 1 : 0;
    return IMX_OK;
}

imx_status imx_mesh_node_coords(const imx_mesh* mesh, double* xyz) {
    if (!mesh || !xyz) return IMX_EINVAL;
    std::memcpy(xyz, mesh->m.xyz.data(), mesh->m.xyz.size() * sizeof(double));
    return IMX_OK;
}

imx_status imx_mesh_mass_diag(const imx_mesh* mesh, double* mh) {
    if (!mesh || !mh) return IMX_EINVAL;
    std::memcpy(mh, mesh->m.WJ.data(), mesh->m.WJ.size() * sizeof(double));
    return IMX_OK;
}

void imx_mesh_destroy(imx_mesh* mesh) { delete mesh; }

imx_status imx_solver_create(const imx_mesh* mesh, const imx_phys* phys, const imx_numerics* num, void* stream,
                             imx_solver** out) {
    if (!mesh || !phys || !num || !out) {
        set_error("imx_solver_create: null argument");
        return IMX_EINVAL;
    }
    CHK(validate_num(*num));
    {
        const imx_mesh_desc& d = mesh->m.desc;
        if (!(phys->sponge_xw >= 0.0) || !(phys->sponge_yw >= 0.0) || 2.0 * phys->sponge_xw > d.Lx ||
            2.0 * phys->sponge_yw > d.Ly) {
            set_error("imx_solver_create: lateral sponge widths must be >= 0 and at most half the domain");
            return IMX_EINVAL;
        }
        if (phys->sponge_lambda != 0.0 &&
            (!(phys->sponge_lambda > 0.0) || !std::isfinite(phys->sponge_lambda) || !(phys->sponge_zT > phys->sponge_zB))) {
            set_error("imx_solver_create: sponge needs a finite sponge_lambda > 0 and sponge_zT > sponge_zB");
            return IMX_EINVAL;
        }
    }
    if (phys->slice) {
        const imx_mesh_desc& d = mesh->m.desc;
        if (d.ny != 1 || !d.periodic_y || mesh->m.nh != 0 || mesh->m.deformed) {
            set_error("imx_solver_create: the slice model needs one periodic element in y, no refinement and flat "
                      "ground");
            return IMX_EINVAL;
        }
    }
    imx_solver* s = new (std::nothrow) imx_solver;
    if (!s) return IMX_ENOMEM;
    s->mesh = &mesh->m;
    s->phys = *phys;
    s->num = *num;
    s->st = (hipStream_t)stream;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        set_error("imx_solver_create: no HIP device");
        return IMX_EHIP;
    }
    {
        // the allocation-free entry point's scratch address on this device
        double* scr = nullptr;
        const imx_status rs = noalloc_scratch(s->device, &scr);
        if (rs != IMX_OK) {
            delete s;
            return rs;
        }
    }
    s->E = mesh->m.E;
    s->Np = mesh->m.Np;
    s->Nf = mesh->m.Nf;
    s->L = s->E * s->Np;
    s->Lp = (s->L + 3) & ~int64_t(3);
    if (9 * s->L >= (int64_t(1) << 31) || s->E * 6 * s->Nf >= (int64_t(1) << 31)) {
        delete s;
        set_error("imx_solver_create: mesh too large (9 E Np and 6 E Nf must stay below 2^31)");
        return IMX_EINVAL;
    }
    s->m = s->m_cap = num->gmres_restart;
    s->mixed = num->precision == IMX_MIXED;
    s->dm.E = s->E;
    s->dm.Lp = s->Lp;
    s->dm.nh = mesh->m.nh;
    s->dm.n = mesh->m.n;
    s->dm.Np = s->Np;
    s->dm.Nf = s->Nf;
    s->dm.deformed = mesh->m.deformed;
    s->tab = make_tab(mesh->m.basis);
    s->ws_bytes = layout(s, nullptr);
    if (hipHostMalloc((void**)&s->hsc, 2048 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        delete s;
        set_error("imx_solver_create: pinned host buffer");
        return IMX_ENOMEM;
    }
    if (hipHostMalloc((void**)&s->hgs, 2 * sizeof(GState), hipHostMallocDefault) != hipSuccess) {
        (void)hipHostFree(s->hsc);
        delete s;
        set_error("imx_solver_create: pinned host buffer");
        return IMX_ENOMEM;
    }
    *out = s;
    return IMX_OK;
}

imx_status imx_solver_workspace_bytes(const imx_solver* s, size_t* bytes) {
    ErrScope es_(s ? &s->err : nullptr);
    if (!s || !bytes) return IMX_EINVAL;
    *bytes = s->ws_bytes;
    return IMX_OK;
}

imx_status imx_solver_bind_workspace(imx_solver* s, void* dev, size_t bytes) {
    ErrScope es_(s ? &s->err : nullptr);
    if (!s || !dev) return IMX_EINVAL;
    drop_chunk_graphs(s);   // captured against the previous workspace
    if (bytes < s->ws_bytes) {
        set_error("imx_solver_bind_workspace: workspace too small");
        return IMX_ENOMEM;
    }
    if (((uintptr_t)dev & 255) != 0) {
        set_error("imx_solver_bind_workspace: workspace must be 256-byte aligned");
        return IMX_EINVAL;
    }
    s->ws = (char*)dev;
    layout(s, s->ws);
    if (s->dm.ncoarse) {
        // side stream for the elements owning a coarse hanging face (default priority)
        if (!s->side) {
            HIPCHK(hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming));
        }
        s->dm.side = s->side;
        s->dm.fork = s->ev_fork;
        s->dm.join = s->ev_join;
    }
    // zero first: the padding of the Krylov-stride vectors (and WJ) stays zero
    HIPCHK(hipMemsetAsync(s->ws, 0, s->ws_bytes, s->st));
    const Mesh& m = *s->mesh;
    // host staging vectors are reused and go out of scope: each upload completes before the next
    auto up = [&](const void* dst, const void* src, size_t n) -> imx_status {
        HIPCHK(hipMemcpyAsync((void*)dst, src, n, hipMemcpyHostToDevice, s->st));
        HIPCHK(hipStreamSynchronize(s->st));
        return IMX_OK;
    };
    {
        // unrefined box: neighbours and face kinds follow from the element
        // index; use that in the all-faces kernels only if it reproduces the
        // face tables exactly
        const imx_mesh_desc& d = m.desc;
        DevMesh& dm = s->dm;
        dm.structured = 0;
        dm.gnx = d.nx;
        dm.gny = d.ny;
        dm.gnz = d.nz;
        dm.gpx = d.periodic_x ? 1 : 0;
        dm.gpy = d.periodic_y ? 1 : 0;
        if (m.nh == 0 && m.E == (int64_t)d.nx * d.ny * d.nz) {
            bool ok = true;
            for (int64_t e = 0; e < m.E && ok; ++e) {
                const int bz = (int)(e % d.nz), t = (int)(e / d.nz), bx = t % d.nx, by = t / d.nx;
                for (int f = 0; f < 6 && ok; ++f) {
                    const int dir = f >> 1, step = (f & 1) ? 1 : -1;
                    int c[3] = {bx, by, bz};
                    const int n[3] = {d.nx, d.ny, d.nz}, per[3] = {dm.gpx, dm.gpy, 0};
                    int v = c[dir] + step;
                    bool wall = false;
                    if (v < 0 || v >= n[dir]) {
                        if (per[dir]) v = v < 0 ? v + n[dir] : v - n[dir];
                        else wall = true;
                    }
                    c[dir] = v;
                    const int kind = wall ? WALL : CONF;
                    const int nb = c[2] + d.nz * (c[0] + d.nx * c[1]);
                    ok = m.fkind[6 * e + f] == kind && (wall || m.fnbr[6 * e + f] == nb);
                }
            }
            dm.structured = ok ? 1 : 0;
        }
    }
    CHK(up(s->dm.kind, m.fkind.data(), m.fkind.size() * sizeof(int)));
    CHK(up(s->dm.nbr, m.fnbr.data(), m.fnbr.size() * sizeof(int)));
    CHK(up(s->dm.aux, m.faux.data(), m.faux.size() * sizeof(int)));
    if (m.nh) CHK(up(s->dm.hang, m.hang.data(), m.hang.size() * sizeof(int)));
    // element lists of the all-faces kernels (elements without a coarse face)
    // and of the face-by-face kernels, on meshes with hanging faces; the first
    // is ordered tile by tile over 8 x 8 base columns so that face neighbours
    // are processed close together in time and meet in the same L2. (On
    // meshes without them the kernels take the natural order: the list's
    // dependent load per element cost more than the saved re-reads.)
    std::vector<int> reg, crs;
    if (s->dm.ncoarse) {
        for (int64_t e = 0; e < s->E; ++e) {
            bool c = false;
            for (int f = 0; f < 6; ++f) c |= m.fkind[6 * e + f] == COARSE;
            (c ? crs : reg).push_back((int)e);
        }
        constexpr int TILE = 8;
        auto key = [&](int e) {
            const int bx = m.base[3 * e], by = m.base[3 * e + 1];
            return std::make_tuple(by / TILE, bx / TILE, by, bx);
        };
        std::stable_sort(reg.begin(), reg.end(), [&](int a, int b) { return key(a) < key(b); });
        CHK(up(s->dm.reg_list, reg.data(), reg.size() * sizeof(int)));
    }
    if (!crs.empty()) CHK(up(s->dm.crs_list, crs.data(), crs.size() * sizeof(int)));
    CHK(up(s->dm.h, m.h.data(), m.h.size() * sizeof(double)));
    std::vector<double> hinv(m.h.size());
    for (size_t i = 0; i < hinv.size(); ++i) hinv[i] = 1.0 / m.h[i];
    CHK(up(s->dm.hinv, hinv.data(), hinv.size() * sizeof(double)));
    // per element: h[3], 1/h[3], det J = h0 (h1 h2) (the host geometry's product), 1 / det J
    std::vector<double> eg((size_t)s->E * 8);
    for (int64_t e = 0; e < s->E; ++e) {
        const double* h = &m.h[3 * e];
        double* q = &eg[8 * e];
        for (int c = 0; c < 3; ++c) {
            q[c] = h[c];
            q[3 + c] = hinv[3 * e + c];
        }
        q[6] = h[0] * (h[1] * h[2]);
        q[7] = 1.0 / q[6];
    }
    CHK(up(s->dm.eg, eg.data(), eg.size() * sizeof(double)));
    {
        // the same products as the host geometry's W detJ = (w_i w_j w_k) det J
        const int n = m.n;
        std::vector<double> w3((size_t)s->Np);
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) w3[i + n * (j + n * k)] = s->tab.w[i] * s->tab.w[j] * s->tab.w[k];
        CHK(up(s->w3, w3.data(), w3.size() * sizeof(double)));
        s->wsrc = WSrc();
        if (!m.deformed || s->dm.cm) {
            s->wsrc.W3 = s->w3;
            s->wsrc.eg = s->dm.eg;
            s->wsrc.E = (int)s->E;
            s->wsrc.np = s->Np;
            s->wsrc.cm = s->dm.cm;
            s->wsrc.nf = s->Nf;
            s->wsrc.K = cm_stride(m.n);
        }
    }
    std::vector<char> tabimg(tab_bytes(m.n, 0)), tabimgf(tab_bytes(m.n, 1));
    fill_tab(s->tab, 0, tabimg.data());
    fill_tab(s->tab, 1, tabimgf.data());
    CHK(up(s->dm.tab, tabimg.data(), tabimg.size()));
    std::vector<uint64_t> fo(fofs_count(m.n));
    fill_fofs(m.n, fo.data());
    CHK(up(s->dm.fofs, fo.data(), fo.size() * sizeof(uint64_t)));
    CHK(up(s->dm.tabf, tabimgf.data(), tabimgf.size()));
    CHK(up(s->dm.WJ, m.WJ.data(), m.WJ.size() * sizeof(double)));
    std::vector<double> iwj, g5, n10;
    if (m.deformed) {
        // terrain-following geometry: x and y are affine in the reference
        // coordinates, so only 5 entries of W cof(J) and, on x- and y-faces,
        // only the normal component of n dS can be nonzero; keep those
        const size_t Lz = (size_t)s->L, NF = (size_t)s->Nf;
        const int keep[5][2] = {{0, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}};
        g5.resize(5 * Lz);
        for (int k = 0; k < 5; ++k)
            std::memcpy(&g5[k * Lz], &m.G[(keep[k][0] * 3 + keep[k][1]) * Lz], Lz * sizeof(double));
        bool ok = true;
        for (int dd = 0; dd < 2; ++dd)
            for (int c = 0; c < 3; ++c)
                if (c != dd)
                    for (size_t i = 0; i < Lz; ++i) ok &= m.G[(dd * 3 + c) * Lz + i] == 0.0;
        n10.resize((size_t)s->E * 10 * NF);
        for (int64_t e = 0; e < s->E; ++e) {
            const double* src = &m.nS[(size_t)e * 18 * NF];
            double* dst = &n10[(size_t)e * 10 * NF];
            for (int f = 0; f < 6; ++f)
                for (int c = 0; c < 3; ++c)
                    for (size_t pt = 0; pt < NF; ++pt) {
                        const double v = src[(f * 3 + c) * NF + pt];
                        if (f < 4) {
                            if (c == f / 2) dst[f * NF + pt] = v;
                            else ok &= v == 0.0;
                        } else {
                            dst[(4 + 3 * (f - 4) + c) * NF + pt] = v;
                        }
                    }
        }
        if (!ok) {
            set_error("imx_solver_bind_workspace: geometry is not of terrain-following form");
            return IMX_EINVAL;
        }
        CHK(up(s->dm.G, g5.data(), g5.size() * sizeof(double)));
        CHK(up(s->dm.nS, n10.data(), n10.size() * sizeof(double)));
        iwj.resize(s->L);
        for (int64_t i = 0; i < s->L; ++i) iwj[i] = 1.0 / m.WJ[i];
        CHK(up(s->dm.iWJ, iwj.data(), iwj.size() * sizeof(double)));
        if (s->dm.cm) CHK(up(s->dm.cm, m.cm.data(), m.cm.size() * sizeof(double)));
    }
    std::vector<double> spl;
    if (s->dm.sponge) {
        // Rayleigh sponge coefficient at every node: the largest of the top
        // layer's and the lateral layers' sin^2 profiles
        spl.resize(s->L);
        const double zB = s->phys.sponge_zB, zT = s->phys.sponge_zT, lam = s->phys.sponge_lambda;
        const double ext[2] = {m.desc.Lx, m.desc.Ly}, wid[2] = {s->phys.sponge_xw, s->phys.sponge_yw};
        auto profile = [lam](double t) {   // t in [0, 1]: depth into the layer
            const double sn = std::sin(0.5 * M_PI * t);
            return lam * sn * sn;
        };
        for (int64_t i = 0; i < s->L; ++i) {
            const double zz = m.xyz[2 * s->L + i];
            double v = zz >= zB ? profile((zz - zB) / (zT - zB)) : 0.0;
            for (int d = 0; d < 2; ++d) {
                if (wid[d] <= 0.0) continue;
                const double x = m.xyz[d * s->L + i];
                double t = 0.0;
                if (x < wid[d]) t = (wid[d] - x) / wid[d];
                else if (x > ext[d] - wid[d]) t = (x - (ext[d] - wid[d])) / wid[d];
                if (t > 0.0) v = std::max(v, profile(t));
            }
            spl[i] = v;
        }
        CHK(up(s->dm.sponge, spl.data(), spl.size() * sizeof(double)));
    }
    std::vector<float> tmp;
    if (s->mixed) {
        tmp.assign(m.WJ.begin(), m.WJ.end());
        CHK(up(s->WJf, tmp.data(), tmp.size() * sizeof(float)));
        if (m.deformed) {
            tmp.assign(g5.begin(), g5.end());
            CHK(up(s->Gf, tmp.data(), tmp.size() * sizeof(float)));
            tmp.assign(n10.begin(), n10.end());
            CHK(up(s->nSf, tmp.data(), tmp.size() * sizeof(float)));
            std::vector<float> iwf(iwj.begin(), iwj.end());
            CHK(up(s->dm.iWJf, iwf.data(), iwf.size() * sizeof(float)));
            if (s->dm.cmf) {
                tmp.assign(m.cm.begin(), m.cm.end());
                CHK(up(s->dm.cmf, tmp.data(), tmp.size() * sizeof(float)));
            }
        }
    }
    HIPCHK(hipMemsetAsync(s->dsc, 0, imx_solver::S_N * sizeof(double), s->st));
    HIPCHK(hipStreamSynchronize(s->st));   // host staging vectors go out of scope
    s->bound = true;
    return IMX_OK;
}

imx_status imx_solver_set_numerics(imx_solver* s, const imx_numerics* num) {
    ErrScope es_(s ? &s->err : nullptr);
    if (!s || !num) return IMX_EINVAL;
    CHK(validate_num(*num));
    if (num->gmres_restart > s->m_cap || (num->precision == IMX_MIXED && !s->mixed)) {
        set_error("imx_solver_set_numerics: restart length / precision exceed the bound workspace");
        return IMX_EINVAL;
    }
    s->num = *num;
    s->m = num->gmres_restart;
    drop_chunk_graphs(s);   // captured for the previous cycle length and coefficients
    return IMX_OK;
}

#define NEED_BOUND(s)                                      \
    do {                                                   \
        if (!(s)) return IMX_EINVAL;                       \
        if (!(s)->bound) {                                 \
            set_error("solver has no workspace bound");    \
            return IMX_ESTATE;                             \
        }                                                  \
    } while (0)

imx_status imx_set_state(imx_solver* s, const double* q) {
    ErrScope es_(s ? &s->err : nullptr);
    NEED_BOUND(s);
    HIPCHK(hipMemcpyAsync(s->y, q, 5 * s->L * sizeof(double), hipMemcpyDeviceToDevice, s->st));
    return IMX_OK;
}

imx_status imx_get_state(const imx_solver* s, double* q) {
    ErrScope es_(s ? &s->err : nullptr);
    NEED_BOUND(s);
    HIPCHK(hipMemcpyAsync(q, s->y, 5 * s->L * sizeof(double), hipMemcpyDeviceToDevice, s->st));
    return IMX_OK;
}

imx_status imx_explicit_residual(imx_solver* s, const double* q, double* fNS, double* fS) {
    ErrScope es_(s ? &s->err : nullptr);
    NEED_BOUND(s);
    if (!q || !fNS || !fS) return IMX_EINVAL;
    const PhysK ph = phys_k(s);
    timed(s, IMX_K_EXPLICIT, field_bytes(s, 14 + (ph.sponge ? 1 : 0), true),
          [&] { explicit_eval(s, ph, q, fNS, fS); });
    HIPCHK(hipGetLastError());
    return IMX_OK;
}

imx_status imx_implicit_setup(imx_solver* s, const double* rho_l, const double* p_lag, const double* u_lag) {
    ErrScope es_(s ? &s->err : nullptr);
    NEED_BOUND(s);
    if (!rho_l || !p_lag || !u_lag) return IMX_EINVAL;
    const size_t L = s->L * sizeof(double);
    HIPCHK(hipMemcpyAsync(s->rho, rho_l, L, hipMemcpyDeviceToDevice, s->st));
    launch_stage_coef(s->L, s->rho, s->dm.WJ, s->cr, s->mixed ? s->crf : nullptr, s->st);
    HIPCHK(hipMemcpyAsync(s->p, p_lag, L, hipMemcpyDeviceToDevice, s->st));
    HIPCHK(hipMemcpyAsync(s->u, u_lag, 3 * L, hipMemcpyDeviceToDevice, s->st));
    return IMX_OK;
}

imx_status imx_schur_apply(imx_solver* s, const double* pin, double* out) {
    ErrScope es_(s ? &s->err : nullptr);
    NEED_BOUND(s);
    if (!pin || !out) return IMX_EINVAL;
    const double a_ll = TAB.at[1][1];
    StageK k = stage_k(s, a_ll);
    timed(s, IMX_K_PASS1, mv1_bytes(s, k.scheme), [&] {
        launch_mv1<double>(s->dm, k, pin, nullptr, s->cr, s->rho, s->p, s->w, s->FB, s->FBh, s->st);
    });
    timed(s, IMX_K_PASS2, mv2_bytes(s), [&] {
        launch_mv2<double>(s->dm, k, pin, nullptr, s->w, s->p, s->rho, s->FB, s->FBh, out, 1, s->st);
    });
    HIPCHK(hipGetLastError());
    return IMX_OK;
}

imx_status imx_implicit_solve(imx_solver* s, const double* rho_l, const double* F, const double* G0,
                              const double* p0, const double* u0, double* pout, double* uout,
                              imx_solve_stats* stats) {
    ErrScope es_(s ? &s->err : nullptr);
    NEED_BOUND(s);
    if (!rho_l || !F || !G0 || !p0 || !u0 || !pout || !uout) return IMX_EINVAL;
    const int64_t L = s->L;
    const size_t B = L * sizeof(double);
    HIPCHK(hipMemcpyAsync(s->rho, rho_l, B, hipMemcpyDeviceToDevice, s->st));
    launch_scale_div(L, 3, F, s->dm.WJ, s->Fh, s->st);
    launch_scale_div(L, 1, G0, s->dm.WJ, s->G0h, s->st);
    HIPCHK(hipMemcpyAsync(s->p, p0, B, hipMemcpyDeviceToDevice, s->st));
    HIPCHK(hipMemcpyAsync(s->u, u0, 3 * B, hipMemcpyDeviceToDevice, s->st));
    imx_status rc = stage_solve(s, TAB.at[1][1], s->rho, s->Fh, s->G0h, s->p, s->u, s->pn, s->un, stats);
    HIPCHK(hipMemcpyAsync(pout, s->p, B, hipMemcpyDeviceToDevice, s->st));
    HIPCHK(hipMemcpyAsync(uout, s->u, 3 * B, hipMemcpyDeviceToDevice, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return rc;
}

imx_status imx_step(imx_solver* s, int nsteps, imx_step_stats* stats) {
    ErrScope es_(s ? &s->err : nullptr);
    NEED_BOUND(s);
    if (nsteps < 0) return IMX_EINVAL;
    imx_step_stats acc{};
    for (int i = 0; i < nsteps; ++i) {
        imx_status rc = one_step(s, &acc);
        if (rc != IMX_OK) {
            if (stats) *stats = acc;
            return rc;
        }
    }
    if (stats) *stats = acc;
    return IMX_OK;
}

imx_status imx_total_mass(imx_solver* s, double* mass) {
    ErrScope es_(s ? &s->err : nullptr);
    NEED_BOUND(s);
    if (!mass) return IMX_EINVAL;
    double* bb = s->dsc + imx_solver::S_MISC;
    launch_mass(s->L, s->y, s->dm.WJ, s->partial, bb, s->st);
    CHK(sync_read(s, bb, 2));
    *mass = s->hsc[0];
    return IMX_OK;
}

imx_status imx_total_mass_noalloc(const imx_solver* s, const double* q_dev, double* out_dev) {
    ErrScope es_(s ? &s->err : nullptr);
    NEED_BOUND(s);
    if (!q_dev || !out_dev) {
        set_error("imx_total_mass_noalloc: null pointer");
        return IMX_EINVAL;
    }
    // the reduction uses at most RED_BLOCKS workgroups of 2 partial sums
    if ((size_t)mass_blocks(s->L) * 2 > NOALLOC_SCRATCH_DOUBLES) {
        set_error("imx_total_mass_noalloc: reduction grid exceeds the static scratch");
        return IMX_EINVAL;
    }
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != s->device) {
        set_error("imx_total_mass_noalloc: the solver's device is not the current device");
        return IMX_EINVAL;
    }
    double* scr = nullptr;
    CHK(noalloc_scratch(s->device, &scr));
    launch_mass(s->L, q_dev, s->dm.WJ, scr, out_dev, s->st);
    HIPCHK(hipGetLastError());
    return IMX_OK;
}

imx_status imx_geo_imbalance(imx_solver* s, double* egeo) {
    ErrScope es_(s ? &s->err : nullptr);
    NEED_BOUND(s);
    if (!egeo) return IMX_EINVAL;
    double* bb = s->dsc + imx_solver::S_MISC;
    const int nb = launch_geo(s->dm, s->y, s->phys.gamma - 1.0, s->phys.f, s->partial, RED_BLOCKS, s->st);
    launch_final_sum(s->partial, nb, 2, bb, s->st);
    CHK(sync_read(s, bb, 2));
    *egeo = s->hsc[0] / s->hsc[1];
    return IMX_OK;
}

imx_status imx_solver_set_sponge_target(imx_solver* s, const double* q_target_dev) {
    imx::ErrScope es_(s ? &s->err : nullptr);
    if (!s) return IMX_EINVAL;
    s->starget = q_target_dev;
    return IMX_OK;
}

imx_status imx_solver_set_graphs(imx_solver* s, int enable) {
    ErrScope es_(s ? &s->err : nullptr);
    if (!s) return IMX_EINVAL;
    s->graphs = enable != 0;
    if (!s->graphs) drop_chunk_graphs(s);
    return IMX_OK;
}

imx_status imx_solver_timing(imx_solver* s, int enable) {
    ErrScope es_(s ? &s->err : nullptr);
    NEED_BOUND(s);
    timing_flush(s);
    if (enable) {
        for (int k = 0; k < IMX_K_COUNT; ++k) {
            s->t_ms[k] = 0.0;
            s->t_bytes[k] = 0.0;
            s->t_count[k] = 0;
        }
    }
    s->timing = enable != 0;
    return IMX_OK;
}

imx_status imx_solver_timing_report(imx_solver* s, int kind, double* ms, double* bytes, int64_t* launches) {
    ErrScope es_(s ? &s->err : nullptr);
    NEED_BOUND(s);
    if (kind < 0 || kind >= IMX_K_COUNT) return IMX_EINVAL;
    timing_flush(s);
    if (ms) *ms = s->t_ms[kind];
    if (bytes) *bytes = s->t_bytes[kind];
    if (launches) *launches = s->t_count[kind];
    return IMX_OK;
}

void imx_solver_destroy(imx_solver* s) {
    if (!s) return;
    timing_flush(s);
    for (auto e : s->tpool) (void)hipEventDestroy(e);
    drop_chunk_graphs(s);
    if (s->cst) (void)hipStreamDestroy(s->cst);
    if (s->side) {
        (void)hipStreamSynchronize(s->side);
        (void)hipStreamDestroy(s->side);
        (void)hipEventDestroy(s->ev_fork);
        (void)hipEventDestroy(s->ev_join);
    }
    if (s->hsc) (void)hipHostFree(s->hsc);
    if (s->hgs) (void)hipHostFree(s->hgs);
    delete s;
}

}  // extern "C"
