// Ensemble server: continuous admission of IMEX-DG integrations into a shared
// device memory pool, one stream and one host worker per running member.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// First-fit allocator over [0, size) with coalescing free list.
class Pool {
   public:
    explicit Pool(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t size() const { return size_; }

   private:
    size_t size_, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

enum MemberState { WAITING, RUNNING, DONE };

struct Member {
    uint64_t id = 0;
    imx_mesh_desc desc{};
    std::vector<double> boxes;
    imx_phys phys{};
    imx_numerics num{};
    int nsteps = 0;
    imx_mesh* mesh = nullptr;
    imx_solver* solver = nullptr;
    hipStream_t stream = nullptr;
    size_t ws_bytes = 0, ws_off = 0;
    size_t pool_bytes = 0;            // workspace + device copy of the state
    std::vector<double> state;        // q0 on submit, final state when done
    std::vector<double> step_ms;
    std::atomic<int> state_flag{WAITING};
    int status = IMX_OK;
    std::string err;
    bool reaped = false;
    int64_t gmres = 0;
    double dofs = 0;
    Clock::time_point t_submit, t_admit, t_done;
    std::thread worker;
};

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (v.size() - 1);
    const size_t lo = (size_t)pos;
    const size_t hi = std::min(lo + 1, v.size() - 1);
    return v[lo] + (pos - lo) * (v[hi] - v[lo]);
}

}  // namespace

struct imx_server {
    char* pool_base = nullptr;
    std::unique_ptr<Pool> pool;
    int max_running = 1;
    int device = 0;
    uint64_t next_id = 1;
    std::mutex mu;
    std::map<uint64_t, std::unique_ptr<Member>> members;
    std::deque<uint64_t> waiting;
    int64_t submitted = 0, admitted = 0, completed = 0, rejected = 0;
    bool any_admit = false;
    Clock::time_point t_first_admit, t_last_done;
    std::vector<double> all_step_ms;
    double dof_updates = 0.0;
    int graphs = 0;    // members admitted from now on replay their Krylov chunks from HIP graphs
    std::string err;   // last error raised by a call on this server
};

using imx::set_error;

extern "C" {

imx_status imx_server_create(void* pool_dev, size_t pool_bytes, int max_running, imx_server** out) {
    if (!pool_dev || pool_bytes < 4096 || max_running < 1 || !out) {
        set_error("imx_server_create: invalid argument");
        return IMX_EINVAL;
    }
    if (((uintptr_t)pool_dev & 255) != 0) {
        set_error("imx_server_create: pool must be 256-byte aligned");
        return IMX_EINVAL;
    }
    imx_server* sv = new (std::nothrow) imx_server;
    if (!sv) return IMX_ENOMEM;
    sv->pool_base = (char*)pool_dev;
    sv->pool.reset(new Pool(pool_bytes));
    sv->max_running = max_running;
    (void)hipGetDevice(&sv->device);
    *out = sv;
    return IMX_OK;
}

imx_status imx_server_submit(imx_server* sv, const imx_mesh_desc* desc, const imx_phys* phys,
                             const imx_numerics* num, const double* q0, int nsteps, uint64_t* id) {
    imx::ErrScope es_(sv ? &sv->err : nullptr);
    if (!sv || !desc || !phys || !num || !q0 || nsteps < 0 || !id) return IMX_EINVAL;
    std::unique_ptr<Member> m(new (std::nothrow) Member);
    if (!m) return IMX_ENOMEM;
    m->boxes.assign(desc->ref_boxes, desc->ref_boxes + 6 * std::max(desc->n_ref, 0));
    m->desc = *desc;
    m->desc.ref_boxes = m->boxes.data();
    m->phys = *phys;
    m->num = *num;
    m->nsteps = nsteps;
    imx_status rc = imx_mesh_create(&m->desc, &m->mesh);
    if (rc != IMX_OK) return rc;
    rc = imx_solver_create(m->mesh, &m->phys, &m->num, nullptr, &m->solver);
    if (rc != IMX_OK) {
        imx_mesh_destroy(m->mesh);
        return rc;
    }
    (void)imx_solver_workspace_bytes(m->solver, &m->ws_bytes);
    imx_solver_destroy(m->solver);   // the running solver is made on admission, on the member's stream
    m->solver = nullptr;
    int64_t E = 0;
    int Np = 0;
    (void)imx_mesh_info(m->mesh, &E, &Np, nullptr, nullptr);
    const size_t state_doubles = (size_t)5 * E * Np;
    const size_t need = m->ws_bytes + ((state_doubles * 8 + 255) & ~size_t(255));
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->submitted++;
    if (need > sv->pool->size()) {
        sv->rejected++;
        imx_mesh_destroy(m->mesh);
        set_error("imx_server_submit: request can never fit the memory pool");
        return IMX_EREJECT;
    }
    m->pool_bytes = need;
    m->state.assign(q0, q0 + state_doubles);
    m->dofs = (double)state_doubles;
    m->id = sv->next_id++;
    m->t_submit = Clock::now();
    *id = m->id;
    sv->waiting.push_back(m->id);
    sv->members[m->id] = std::move(m);
    return IMX_OK;
}

}  // extern "C"

// Worker: uploads q0, runs the steps, downloads the final state.
static void member_main(imx_server* sv, Member* m, double* state_dev) {
    (void)hipSetDevice(sv->device);
    (void)hipMemcpyAsync(state_dev, m->state.data(), m->state.size() * 8, hipMemcpyHostToDevice, m->stream);
    imx_status rc = imx_set_state(m->solver, state_dev);
    for (int k = 0; rc == IMX_OK && k < m->nsteps; ++k) {
        const auto t0 = Clock::now();
        imx_step_stats st{};
        rc = imx_step(m->solver, 1, &st);
        const auto t1 = Clock::now();
        if (rc != IMX_OK) break;
        m->gmres += st.gmres_iters;
        m->step_ms.push_back(ms_since(t0, t1));
    }
    m->status = rc;
    if (rc != IMX_OK) m->err = imx_solver_last_error(m->solver);
    (void)imx_get_state(m->solver, state_dev);
    (void)hipMemcpyAsync(m->state.data(), state_dev, m->state.size() * 8, hipMemcpyDeviceToHost, m->stream);
    (void)hipStreamSynchronize(m->stream);
    m->t_done = Clock::now();
    m->state_flag.store(DONE);
}

extern "C" {

imx_status imx_server_tick(imx_server* sv, int* n_running, int* n_waiting) {
    imx::ErrScope es_(sv ? &sv->err : nullptr);
    if (!sv) return IMX_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    (void)hipSetDevice(sv->device);
    int running = 0;
    // reap finished members: their pool slice and stream go back
    for (auto& kv : sv->members) {
        Member* m = kv.second.get();
        const int f = m->state_flag.load();
        if (f == DONE && !m->reaped) {
            if (m->worker.joinable()) m->worker.join();
            imx_solver_destroy(m->solver);
            m->solver = nullptr;
            (void)hipStreamDestroy(m->stream);
            m->stream = nullptr;
            sv->pool->release(m->ws_off, m->pool_bytes);
            m->reaped = true;
            sv->completed++;
            sv->t_last_done = std::max(sv->t_last_done, m->t_done);
            sv->all_step_ms.insert(sv->all_step_ms.end(), m->step_ms.begin(), m->step_ms.end());
            sv->dof_updates += m->dofs * (double)m->step_ms.size();
        } else if (f == RUNNING) {
            ++running;
        }
    }
    // admit in arrival order every waiting member that fits (later, smaller
    // requests may pass one that does not fit yet)
    for (auto it = sv->waiting.begin(); it != sv->waiting.end() && running < sv->max_running;) {
        Member* m = sv->members[*it].get();
        size_t off = 0;
        if (!sv->pool->alloc(m->pool_bytes, &off)) {
            ++it;
            continue;
        }
        m->ws_off = off;
        imx_status rc = IMX_OK;
        if (hipStreamCreate(&m->stream) != hipSuccess) {
            set_error("imx_server_tick: hipStreamCreate failed");
            rc = IMX_EHIP;
        }
        if (rc == IMX_OK) rc = imx_solver_create(m->mesh, &m->phys, &m->num, m->stream, &m->solver);
        if (rc == IMX_OK) rc = imx_solver_bind_workspace(m->solver, sv->pool_base + off, m->ws_bytes);
        if (rc == IMX_OK && sv->graphs) rc = imx_solver_set_graphs(m->solver, 1);
        m->t_admit = Clock::now();
        it = sv->waiting.erase(it);
        if (rc != IMX_OK) {
            // the member ends here with the error; nothing of it stays on the device
            if (m->solver) imx_solver_destroy(m->solver);
            m->solver = nullptr;
            if (m->stream) (void)hipStreamSynchronize(m->stream), (void)hipStreamDestroy(m->stream);
            m->stream = nullptr;
            sv->pool->release(off, m->pool_bytes);
            m->status = rc;
            m->err = imx_last_error();
            m->t_done = m->t_admit;
            m->state.clear();
            m->state_flag.store(DONE);
            m->reaped = true;
            sv->completed++;
            continue;
        }
        double* state_dev = (double*)(sv->pool_base + off + m->ws_bytes);
        if (!sv->any_admit) {
            sv->any_admit = true;
            sv->t_first_admit = m->t_admit;
        }
        m->state_flag.store(RUNNING);
        m->worker = std::thread(member_main, sv, m, state_dev);
        sv->admitted++;
        ++running;
    }
    if (n_running) *n_running = running;
    if (n_waiting) *n_waiting = (int)sv->waiting.size();
    return IMX_OK;
}

imx_status imx_server_result(imx_server* sv, uint64_t id, double* q_host, imx_member_stats* stats) {
    imx::ErrScope es_(sv ? &sv->err : nullptr);
    if (!sv) return IMX_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->members.find(id);
    if (it == sv->members.end()) {
        set_error("imx_server_result: unknown id");
        return IMX_EINVAL;
    }
    Member* m = it->second.get();
    if (!m->reaped) {
        set_error("imx_server_result: member has not finished (call imx_server_tick)");
        return IMX_ESTATE;
    }
    if (q_host && !m->state.empty()) std::memcpy(q_host, m->state.data(), m->state.size() * 8);
    if (m->status != IMX_OK) set_error("member failed: " + m->err);
    if (stats) {
        stats->steps_done = (int)m->step_ms.size();
        stats->status = m->status;
        stats->p50_step_ms = percentile(m->step_ms, 0.5);
        stats->p99_step_ms = percentile(m->step_ms, 0.99);
        double s = 0;
        for (double v : m->step_ms) s += v;
        stats->mean_step_ms = m->step_ms.empty() ? 0.0 : s / m->step_ms.size();
        stats->queue_ms = ms_since(m->t_submit, m->t_admit);
        stats->run_ms = ms_since(m->t_admit, m->t_done);
        stats->gmres_iters = m->gmres;
    }
    return IMX_OK;
}

imx_status imx_server_query(imx_server* sv, imx_server_stats* st) {
    imx::ErrScope es_(sv ? &sv->err : nullptr);
    if (!sv || !st) return IMX_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    int64_t running = 0;
    for (auto& kv : sv->members)
        if (kv.second->state_flag.load() != WAITING && !kv.second->reaped) ++running;
    st->submitted = sv->submitted;
    st->admitted = sv->admitted;
    st->completed = sv->completed;
    st->rejected = sv->rejected;
    st->running = running;
    st->waiting = (int64_t)sv->waiting.size();
    st->pool_bytes = sv->pool->size();
    st->pool_bytes_in_use = sv->pool->used();
    st->pool_bytes_peak = sv->pool->peak();
    st->p50_step_ms = percentile(sv->all_step_ms, 0.5);
    st->p99_step_ms = percentile(sv->all_step_ms, 0.99);
    st->dof_updates = sv->dof_updates;
    st->busy_seconds = sv->any_admit && sv->completed ? ms_since(sv->t_first_admit, sv->t_last_done) * 1e-3 : 0.0;
    return IMX_OK;
}

imx_status imx_server_set_graphs(imx_server* sv, int enable) {
    imx::ErrScope es_(sv ? &sv->err : nullptr);
    if (!sv) return IMX_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->graphs = enable ? 1 : 0;
    return IMX_OK;
}

const char* imx_server_last_error(const imx_server* sv) { return sv ? sv->err.c_str() : ""; }

void imx_server_destroy(imx_server* sv) {
    if (!sv) return;
    for (auto& kv : sv->members) {
        Member* m = kv.second.get();
        if (m->worker.joinable()) m->worker.join();
        if (m->solver) imx_solver_destroy(m->solver);
        if (m->stream) (void)hipStreamDestroy(m->stream);
        if (m->mesh) imx_mesh_destroy(m->mesh);
    }
    delete sv;
}

}  // extern "C"
