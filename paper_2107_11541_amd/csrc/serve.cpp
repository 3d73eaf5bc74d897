// serve.cpp -- continuous batching of assemble + solve requests on one GPU.
//
// One request is the per-time-step work of the paper's Algorithm 1 on its own
// mesh: the momentum operator M/dt + C + K with its right-hand sides and the
// pressure (Poisson) system assembled into CSR (Section 4.2), the Dirichlet
// elimination, then the PCG solve (Section 5.2).  Many small meshes give
// kernels far too small to fill 256 compute units, so the runtime
//   * plans meshes on host threads while the GPU works (the planner is the
//     fe_mesh_upload preprocessing, on one to four threads per mesh);
//   * places every admitted request in one pre-allocated device arena
//     (admission by footprint; no hipMalloc per request);
//   * assembles the requests admitted in one pass together: one launch per
//     (colour, type) launch index and element type over all of them;
//   * advances all admitted requests' PCG iterations together, three
//     launches per iteration whatever the number of requests, and polls
//     their device-side stop flags asynchronously (one small copy per poll);
//   * finishes a request (true residual, copies to the host) behind an
//     event and frees its arena space as soon as the copies have landed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host.h"

using namespace feasm;

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

enum Phase { kQueued, kPlanned, kRunning, kFinishing, kDone };

struct Job {
    int64_t ticket = 0;
    fe_job desc{};
    Phase phase = kQueued;
    Clock::time_point t_submit, t_planned, t_admitted, t_done;
    // planner output
    std::unique_ptr<MeshImage> img;
    std::vector<double> fields;   // mesh numbering: u [3][N], rho [N], mu [N]
    size_t bytes = 0;             // arena bytes this request needs
    int skipped = 0;              // admissions that passed it by
    // device state
    fe_mesh_s *mesh = nullptr;
    int slot = -1;
    double *vals_m = nullptr, *rhs_m = nullptr, *vals_p = nullptr, *rhs_p = nullptr, *fields_d = nullptr,
           *x_d = nullptr;
    int k = 0;                    // batched iterations launched
    int it = 0;                   // iterations done (device count)
    int32_t dev_status = FE_OK;
    hipEvent_t done_ev = nullptr;
    fe_job_result res{};
};

void set_message(fe_job_result &r, const std::string &m)
{
    snprintf(r.message, sizeof r.message, "%s", m.c_str());
}

// Per-slot host read-back area (pinned): [0] true rr, [1] true bb,
// [2] recursive rr, [3] b.b, [4..5] assembly status word.
constexpr int kResDoubles = 8;

}  // namespace

struct fe_server_s {
    fe_ctx_s *ctx = nullptr;
    fe_ctx_s sctx;                // the dispatcher's own context (its error text, its stream)
    hipStream_t stream = nullptr;
    char *arena_base = nullptr;
    std::unique_ptr<DevArena> arena;
    int max_slots = 0;
    BatchJob *jobs_d = nullptr, *jobs_h = nullptr;   // per-slot system descriptions
    char *kargs_d = nullptr, *kargs_h = nullptr;     // per-slot assembly arguments (momentum, Poisson)
    int32_t *flags_d = nullptr, *flags_h = nullptr;  // per-slot PCG flag words (4 ints)
    double *res_d = nullptr, *res_h = nullptr;       // per-slot read-back area
    std::vector<double *> stage;                     // per-slot pinned staging for x and mom_rhs
    std::vector<size_t> stage_cap;
    hipEvent_t poll_ev = nullptr;

    std::mutex mu;
    std::condition_variable cv_plan, cv_work, cv_done;
    std::deque<Job *> submit_q;
    std::vector<Job *> ready, active, finishing;
    std::unordered_map<int64_t, std::unique_ptr<Job>> jobs;
    std::vector<int> free_slots;
    std::vector<std::thread> planners;
    std::thread dispatcher;
    bool stop = false;
    int planners_busy = 0;
    // Planned images of finished requests, kept (at most one per planner
    // thread) so that the next plan reuses their host arrays instead of
    // faulting hundreds of MB of fresh pages in (96^3: ~15 % of a plan).
    std::mutex pool_mu;
    std::vector<std::unique_ptr<MeshImage>> img_pool;
    size_t pool_cap = 0;
    int64_t next_ticket = 1;
    int64_t completed = 0, batches = 0, batched_requests = 0;
    std::string err;
};

namespace {

// ---- planning (host threads) -----------------------------------------------

std::unique_ptr<MeshImage> take_image(fe_server_s *S)
{
    {
        std::lock_guard<std::mutex> lk(S->pool_mu);
        if (!S->img_pool.empty()) {
            std::unique_ptr<MeshImage> img = std::move(S->img_pool.back());
            S->img_pool.pop_back();
            return img;
        }
    }
    return std::make_unique<MeshImage>();
}

void give_image(fe_server_s *S, std::unique_ptr<MeshImage> &img)
{
    if (!img) return;
    std::unique_ptr<MeshImage> mine = std::move(img);
    std::lock_guard<std::mutex> lk(S->pool_mu);
    if (S->img_pool.size() < S->pool_cap) S->img_pool.push_back(std::move(mine));
}

// idle: no other request waits to be planned (see planner_main)
void plan_job(fe_server_s *S, Job *j, bool idle)
{
    RoctxRange rr("serve: plan");
    const fe_job &q = j->desc;
    // one thread per mesh keeps every planner busy; large meshes get a few
    // more so that they do not set the latency tail alone, and more again
    // when nothing else waits for the planners
    const int64_t threads = idle ? std::min<int64_t>(8, q.n_elems / 100000) : std::min<int64_t>(4, q.n_elems / 200000);
    set_thread_budget((int)std::max<int64_t>(1, threads));
    j->img = take_image(S);
    std::string err;
    int st = FE_OK;
    if (!(q.dt > 0.0) || !(q.rtol > 0.0) || q.max_iter < 0 || !q.u || !q.rho || !q.mu || !q.x) {
        st = FE_EINVAL;
        err = "request needs dt > 0, rtol > 0, max_iter >= 0 and u, rho, mu, x";
    } else {
        st = mesh_prepare(q.elem_types ? 8 : (int)q.type, q.elem_types, q.n_nodes, q.coords, q.n_elems, q.conn,
                          q.n_dirichlet,
                          q.dirichlet_nodes, true, *j->img, err, false);
    }
    if (st != FE_OK) {
        j->res.status = (fe_status)st;
        set_message(j->res, err);
        give_image(S, j->img);
        return;
    }
    const DevMesh &d = j->img->d;
    const int64_t N = d.N;
    const std::vector<int32_t> &perm = j->img->P.node_perm;   // mesh index -> user id
    j->fields.resize((size_t)5 * N);
    double *f = j->fields.data();
    for (int c = 0; c < 3; ++c)
        for (int64_t i = 0; i < N; ++i) f[c * N + i] = q.u[c * N + perm[i]];
    for (int64_t i = 0; i < N; ++i) {
        f[3 * N + i] = q.rho[perm[i]];
        f[4 * N + i] = q.mu[perm[i]];
    }
    const size_t vb = DevArena::round((size_t)d.nnz * 8), nb = DevArena::round((size_t)N * 8);
    j->bytes = j->img->device_bytes() + cg_bytes(N, q.max_iter) + 2 * vb + 3 * nb + nb + 5 * nb + nb;
}

void planner_main(fe_server_s *S)
{
    for (;;) {
        Job *j;
        bool idle = false;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_plan.wait(lk, [&] { return S->stop || !S->submit_q.empty(); });
            if (S->submit_q.empty()) return;   // stop requested and nothing left
            j = S->submit_q.front();
            S->submit_q.pop_front();
            ++S->planners_busy;
            idle = S->submit_q.empty() && S->planners_busy == 1;
        }
        try {
            plan_job(S, j, idle);
        } catch (const std::bad_alloc &) {
            j->img.reset();
            j->fields = std::vector<double>();
            j->res.status = FE_ENOMEM;
            set_message(j->res, "host memory exhausted while planning the mesh");
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            --S->planners_busy;
            j->t_planned = Clock::now();
            if (j->res.status == FE_OK && j->bytes > S->arena->capacity()) {
                j->res.status = FE_ENOMEM;
                set_message(j->res, "request footprint exceeds the server's HBM budget");
                give_image(S, j->img);
            }
            if (j->res.status != FE_OK) {
                j->phase = kDone;
                j->t_done = j->t_planned;
                ++S->completed;
                S->cv_done.notify_all();
            } else {
                j->phase = kPlanned;
                auto it = std::lower_bound(S->ready.begin(), S->ready.end(), j,
                                           [](const Job *a, const Job *b) { return a->ticket < b->ticket; });
                S->ready.insert(it, j);
            }
            S->cv_work.notify_all();
        }
    }
}

// ---- device stages (dispatcher thread, server lock NOT held) ----------------

fe_status ensure_stage(fe_server_s *S, int slot, size_t doubles)
{
    if (S->stage_cap[slot] >= doubles) return FE_OK;
    if (S->stage[slot]) (void)hipHostFree(S->stage[slot]);
    S->stage[slot] = nullptr;
    S->stage_cap[slot] = 0;
    size_t cap = std::max(doubles, (size_t)1 << 16);
    if (hipHostMalloc((void **)&S->stage[slot], cap * sizeof(double), hipHostMallocDefault) != hipSuccess)
        return FE_ENOMEM;
    S->stage_cap[slot] = cap;
    return FE_OK;
}

// The assembly arguments of an admitted request (FP64, coloured plan).
AsmArgs job_asm_args(Job *j, int op)
{
    fe_mesh_s *m = j->mesh;
    const int64_t N = m->dm.N;
    AsmArgs a{};
    a.m = &m->dm;
    a.op = op;
    a.dt = j->desc.dt;
    a.u = j->fields_d;
    a.rho = j->fields_d + 3 * N;
    a.mu = j->fields_d + 4 * N;
    a.status = m->status;
    a.values = op == FE_OP_MOMENTUM ? j->vals_m : j->vals_p;
    a.rhs = op == FE_OP_MOMENTUM ? j->rhs_m : j->rhs_p;
    return a;
}

// Allocates an admitted request's device memory, uploads its mesh and
// fields and writes its assembly arguments; the assemblies, the Dirichlet
// elimination and the PCG set-up follow with the other admissions of the
// pass (assemble_admitted, admit_finish).  On failure every allocation is
// returned and the status says why (FE_ENOMEM: try again later).
fe_status admit(fe_server_s *S, Job *j)
{
    RoctxRange rr("serve: admit");
    fe_ctx_s *c = &S->sctx;
    const fe_job &q = j->desc;
    auto *m = new fe_mesh_s();
    m->ctx = c;   // the server's private context
    m->arena = S->arena.get();
    m->listed = false;
    j->mesh = m;
    const DevMesh &d = j->img->d;
    const int64_t N = d.N, nnz = d.nnz;
    // pinned staging for the results first: its failure is not a lack of
    // arena space and must fail the request rather than defer it
    if (ensure_stage(S, j->slot, (size_t)4 * N) != FE_OK) {
        delete m;
        j->mesh = nullptr;
        fail(c, FE_EDEVICE, "could not allocate pinned host staging for the results");
        return FE_EDEVICE;
    }
    fe_status s = mesh_commit(m, *j->img, S->stream);
    if (s == FE_OK) s = ensure_cg(m, q.max_iter, false);
    double **bufs[] = {&j->vals_m, &j->rhs_m, &j->vals_p, &j->rhs_p, &j->fields_d, &j->x_d};
    const size_t sizes[] = {(size_t)nnz, (size_t)3 * N, (size_t)nnz, (size_t)N, (size_t)5 * N, (size_t)N};
    for (int b = 0; b < 6 && s == FE_OK; ++b) s = mesh_alloc(m, (void **)bufs[b], sizes[b] * sizeof(double));
    if (s != FE_OK) {
        mesh_release(m);
        delete m;
        j->mesh = nullptr;
        return s;
    }
    CGWork &w = m->cg;
    w.flags = S->flags_d + 4 * j->slot;   // polled with every other slot's flags in one copy
    HIPCALL(c, hipMemcpyAsync(j->fields_d, j->fields.data(), j->fields.size() * sizeof(double), hipMemcpyHostToDevice,
                              S->stream));
    // the two assemblies run batched with the other admissions of this pass
    // (assemble_admitted); their kernel arguments go to this slot's entries
    char *kh = S->kargs_h + (size_t)2 * j->slot * kKArgsBytes;
    fill_kargs(job_asm_args(j, FE_OP_MOMENTUM), kh);
    fill_kargs(job_asm_args(j, FE_OP_POISSON), kh + kKArgsBytes);
    HIPCALL(c, hipMemcpyAsync(S->kargs_d + (size_t)2 * j->slot * kKArgsBytes, kh, 2 * kKArgsBytes,
                              hipMemcpyHostToDevice, S->stream));
    return FE_OK;
}

// The momentum and Poisson assemblies of the requests admitted in one
// dispatcher pass: one launch per (colour, type) launch index and element
// type over all of them, each request's blocks running the code of its own
// coloured launch (its results do not depend on the batch).
fe_status assemble_admitted(fe_server_s *S, const std::vector<Job *> &js)
{
    fe_ctx_s *c = &S->sctx;
    AsmArgs a[kMaxBatch];
    int slot[kMaxBatch];
    const int n = (int)js.size();
    if (n < 1 || n > kMaxBatch) return fail(c, FE_EINVAL, "internal: %d admissions in one pass", n);
    for (int o = 0; o < 2; ++o) {
        for (int i = 0; i < n; ++i) {
            a[i] = job_asm_args(js[i], o == 0 ? FE_OP_MOMENTUM : FE_OP_POISSON);
            slot[i] = 2 * js[i]->slot + o;
        }
        HIPCALL(c, launch_assemble_batch(a, slot, n, S->kargs_d, S->stream));
    }
    return FE_OK;
}

// After the assemblies: the Dirichlet elimination, the PCG set-up and the
// request's entry in the batched PCG's table.
fe_status admit_finish(fe_server_s *S, Job *j)
{
    fe_ctx_s *c = &S->sctx;
    const fe_job &q = j->desc;
    fe_mesh_s *m = j->mesh;
    const int64_t N = m->dm.N, nnz = m->dm.nnz;
    CGWork &w = m->cg;
    HIPCALL(c, launch_dirichlet(m->dm, j->vals_p, j->rhs_p, nullptr, S->stream));
    HIPCALL(c, cg_setup<double>(m->dm, j->vals_p, j->rhs_p, j->x_d, w, q.rtol, S->stream, true));
    BatchJob &b = S->jobs_h[j->slot];
    b.sm = spmv_map(m->dm);
    b.vals = j->vals_p;
    b.n = N;
    b.vec = spmv_vec_capable(j->vals_p, nnz) ? 1 : 0;
    if (!b.vec) return fail(c, FE_EINVAL, "internal: arena value array not 16-byte aligned");
    b.x = j->x_d;
    b.r = w.r;
    b.z = w.z;
    b.p = w.p;
    b.q = w.q;
    b.dinv = w.dinv;
    b.part = w.part;
    b.hist = w.hist;
    b.scal = w.hist + 4 * w.hist_cap;
    b.flags = w.flags;
    b.nb_spmv = cg_spmv_groups(m->dm);
    b.nb_vec = w.nb;
    HIPCALL(c, hipMemcpyAsync(S->jobs_d + j->slot, &b, sizeof(BatchJob), hipMemcpyHostToDevice, S->stream));
    return FE_OK;
}

// Queues the true residual and the copies back; records done_ev.
fe_status finish_queue(fe_server_s *S, Job *j)
{
    fe_ctx_s *c = &S->sctx;
    fe_mesh_s *m = j->mesh;
    CGWork &w = m->cg;
    const int64_t N = m->dm.N;
    double *rd = S->res_d + kResDoubles * j->slot, *rh = S->res_h + kResDoubles * j->slot;
    HIPCALL(c, residual_f64(m->dm, j->vals_p, j->rhs_p, j->x_d, w.d64, w.part, rd, S->stream));
    HIPCALL(c, hipMemcpyAsync(rd + 2, w.hist + 4 * (size_t)j->it + 1, sizeof(double), hipMemcpyDeviceToDevice,
                              S->stream));
    HIPCALL(c, hipMemcpyAsync(rd + 3, w.hist + 4 * (size_t)w.hist_cap, sizeof(double), hipMemcpyDeviceToDevice,
                              S->stream));
    HIPCALL(c, hipMemcpyAsync(rd + 4, m->status, sizeof(AsmStatus), hipMemcpyDeviceToDevice, S->stream));
    HIPCALL(c, hipMemcpyAsync(rh, rd, kResDoubles * sizeof(double), hipMemcpyDeviceToHost, S->stream));
    double *st = S->stage[j->slot];
    HIPCALL(c, hipMemcpyAsync(st, j->x_d, N * sizeof(double), hipMemcpyDeviceToHost, S->stream));
    if (j->desc.mom_rhs)
        HIPCALL(c, hipMemcpyAsync(st + N, j->rhs_m, 3 * N * sizeof(double), hipMemcpyDeviceToHost, S->stream));
    if (!j->done_ev) HIPCALL(c, hipEventCreateWithFlags(&j->done_ev, hipEventDisableTiming));
    HIPCALL(c, hipEventRecord(j->done_ev, S->stream));
    return FE_OK;
}

// Results to the caller's buffers (user numbering); arena space returned.
void finish_host(fe_server_s *S, Job *j)
{
    RoctxRange rr("serve: finish");
    fe_mesh_s *m = j->mesh;
    const int64_t N = m->dm.N;
    const double *rh = S->res_h + kResDoubles * j->slot, *st = S->stage[j->slot];
    const std::vector<int32_t> &perm = j->img->P.node_perm;
    for (int64_t i = 0; i < N; ++i) j->desc.x[perm[i]] = st[i];
    if (j->desc.mom_rhs)
        for (int c = 0; c < 3; ++c)
            for (int64_t i = 0; i < N; ++i) j->desc.mom_rhs[c * N + perm[i]] = st[N + c * N + i];
    fe_job_result &r = j->res;
    r.iterations = j->it;
    r.true_rel_residual = rh[1] > 0 ? std::sqrt(rh[0] / rh[1]) : std::sqrt(rh[0]);
    r.rel_residual = rh[3] > 0 ? std::sqrt(rh[2] / rh[3]) : std::sqrt(rh[2]);
    AsmStatus as;
    memcpy(&as, rh + 4, sizeof as);
    double md;
    memcpy(&md, &as.min_det_key, 8);
    r.min_detJ = md;
    const bool bad_ok = as.first_bad < (long long)j->img->P.elem_perm.size();
    r.first_bad_elem = as.first_bad >= 0 && bad_ok ? j->img->P.elem_perm[as.first_bad] : -1;
    if (!bad_ok) {
        r.status = FE_EDEVICE;
        set_message(r, "assembly status names an element out of range");
    }
    if (r.first_bad_elem >= 0) {
        r.status = FE_EBADELEM;
        set_message(r, "det J <= 0 in element " + std::to_string(r.first_bad_elem) + " (user id)");
    } else if (j->dev_status == FE_EBREAKDOWN) {
        r.status = FE_EBREAKDOWN;
        set_message(r, "CG breakdown (p.Ap <= 0 or non-finite)");
    } else if (j->dev_status == FE_ENOCONV) {
        r.status = FE_ENOCONV;
        set_message(r, "CG did not reach rtol in max_iter iterations");
    }
    mesh_release(m);
    delete m;
    j->mesh = nullptr;
    if (j->done_ev) (void)hipEventDestroy(j->done_ev);
    j->done_ev = nullptr;
    give_image(S, j->img);
    j->fields = std::vector<double>();
}

void fail_job(fe_server_s *S, Job *j, fe_status s, const std::string &msg)
{
    j->res.status = s;
    set_message(j->res, msg);
    if (j->mesh) {
        (void)hipStreamSynchronize(S->stream);
        mesh_release(j->mesh);
        delete j->mesh;
        j->mesh = nullptr;
    }
}

// ---- dispatcher ----------------------------------------------------------------

constexpr int kPollEvery = 4;      // batched iterations between flag copies
constexpr int kMaxBypass = 8;      // admissions that may pass a request that does not fit
constexpr int kMaxRunAhead = 24;   // iterations launched past an unread poll

void dispatcher_main(fe_server_s *S)
{
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    bool poll_inflight = false;
    int since_poll = 0;
    std::vector<std::pair<Job *, int>> snap;   // (request, iterations launched) at the poll
    auto complete = [&](Job *j) {
        j->phase = kDone;
        j->t_done = Clock::now();
        if (j->slot >= 0) S->free_slots.push_back(j->slot);
        j->slot = -1;
        ++S->completed;
        S->cv_done.notify_all();
    };
    for (;;) {
        // 1. requests whose copies have landed
        for (size_t i = 0; i < S->finishing.size();) {
            Job *j = S->finishing[i];
            if (hipEventQuery(j->done_ev) == hipSuccess) {
                S->finishing.erase(S->finishing.begin() + (long)i);
                lk.unlock();
                finish_host(S, j);
                lk.lock();
                complete(j);
            } else {
                ++i;
            }
        }
        // 2. admissions, in ticket order; a request that does not fit may be
        // passed by later ones: each admission past it counts, and after
        // kMaxBypass of them nothing behind it is admitted until it fits
        std::vector<Job *> passed;   // requests of this pass that did not fit
        std::vector<Job *> fresh;    // admitted in this pass: assembled together below
        for (size_t i = 0; i < S->ready.size() && !S->free_slots.empty();) {
            Job *j = S->ready[i];
            if (j->bytes > S->arena->free_bytes()) {
                if (j->skipped >= kMaxBypass) break;
                passed.push_back(j);
                ++i;
                continue;
            }
            S->ready.erase(S->ready.begin() + (long)i);
            j->slot = S->free_slots.back();
            S->free_slots.pop_back();
            lk.unlock();
            fe_status s = admit(S, j);
            lk.lock();
            if (s == FE_ENOMEM && !j->mesh) {   // fragmentation: retry later
                S->free_slots.push_back(j->slot);
                j->slot = -1;
                S->ready.insert(S->ready.begin() + (long)i, j);
                break;
            }
            if (s != FE_OK) {
                lk.unlock();
                fail_job(S, j, s, S->sctx.err);
                lk.lock();
                complete(j);
                continue;
            }
            j->t_admitted = Clock::now();
            fresh.push_back(j);
            for (Job *p : passed) ++p->skipped;   // j was admitted ahead of them
        }
        if (!fresh.empty()) {
            lk.unlock();
            std::vector<fe_status> st(fresh.size(), assemble_admitted(S, fresh));
            for (size_t i = 0; i < fresh.size(); ++i)
                if (st[i] == FE_OK) st[i] = admit_finish(S, fresh[i]);
            lk.lock();
            for (size_t i = 0; i < fresh.size(); ++i) {
                Job *j = fresh[i];
                if (st[i] != FE_OK) {
                    lk.unlock();
                    fail_job(S, j, st[i], S->sctx.err);
                    lk.lock();
                    complete(j);
                    continue;
                }
                j->phase = kRunning;
                j->k = 0;
                S->active.push_back(j);
            }
        }
        // 3. idle?
        if (S->active.empty()) {
            if (!S->finishing.empty()) {
                hipEvent_t e = S->finishing.front()->done_ev;
                lk.unlock();
                (void)hipEventSynchronize(e);
                lk.lock();
                continue;
            }
            if (S->stop && S->submit_q.empty() && S->ready.empty() && S->planners_busy == 0) break;
            S->cv_work.wait_for(lk, std::chrono::milliseconds(2));
            continue;
        }
        // 4. one batched iteration over the requests still iterating
        BatchList L{};
        L.wgs[0] = L.wgv[0] = 0;
        bool any_at_max = false;
        std::vector<Job *> carried;
        for (Job *j : S->active) {
            if (j->k >= j->desc.max_iter) {
                any_at_max = true;
                continue;
            }
            const BatchJob &b = S->jobs_h[j->slot];
            L.slot[L.n] = j->slot;
            L.k[L.n] = j->k;
            L.wgs[L.n + 1] = L.wgs[L.n] + b.nb_spmv;
            L.wgv[L.n + 1] = L.wgv[L.n] + b.nb_vec;
            ++L.n;
            carried.push_back(j);
        }
        if (L.n > 0) {
            lk.unlock();
            hipError_t e = batch_iteration(S->jobs_d, L, S->stream);
            lk.lock();
            if (e != hipSuccess) S->err = hipGetErrorString(e);
            for (Job *j : carried) ++j->k;
            ++S->batches;
            S->batched_requests += L.n;
            ++since_poll;
        }
        // 5. poll the stop flags without blocking the launches
        if (!poll_inflight && (since_poll >= kPollEvery || any_at_max || L.n == 0)) {
            snap.clear();
            for (Job *j : S->active) snap.push_back({j, j->k});
            lk.unlock();
            (void)hipMemcpyAsync(S->flags_h, S->flags_d, (size_t)kMaxBatch * 4 * sizeof(int32_t),
                                 hipMemcpyDeviceToHost, S->stream);
            (void)hipEventRecord(S->poll_ev, S->stream);
            lk.lock();
            poll_inflight = true;
            since_poll = 0;
        }
        if (poll_inflight) {
            hipError_t q = hipEventQuery(S->poll_ev);
            if (q == hipErrorNotReady && (since_poll >= kMaxRunAhead || L.n == 0)) {
                lk.unlock();
                (void)hipEventSynchronize(S->poll_ev);
                lk.lock();
                q = hipSuccess;
            }
            if (q == hipSuccess) {
                poll_inflight = false;
                for (auto &pr : snap) {
                    Job *j = pr.first;
                    const int32_t *f = S->flags_h + 4 * j->slot;
                    const bool done = f[0] != 0, at_max = pr.second >= j->desc.max_iter;
                    if (!done && !at_max) continue;
                    j->it = f[2];
                    j->dev_status = done ? f[1] : FE_ENOCONV;
                    S->active.erase(std::find(S->active.begin(), S->active.end(), j));
                    lk.unlock();
                    fe_status s = finish_queue(S, j);
                    lk.lock();
                    if (s != FE_OK) {
                        lk.unlock();
                        fail_job(S, j, s, S->sctx.err);
                        lk.lock();
                        complete(j);
                        continue;
                    }
                    j->phase = kFinishing;
                    S->finishing.push_back(j);
                }
            }
        }
    }
}

void fill_result(Job *j, fe_job_result *r)
{
    j->res.plan_ms = ms_between(j->t_submit, j->t_planned);
    const bool admitted = j->t_admitted.time_since_epoch().count() != 0;
    j->res.wait_ms = admitted ? ms_between(j->t_planned, j->t_admitted) : 0.0;
    j->res.run_ms = admitted ? ms_between(j->t_admitted, j->t_done) : 0.0;
    j->res.total_ms = ms_between(j->t_submit, j->t_done);
    if (r) *r = j->res;
}

}  // namespace

extern "C" {

fe_status fe_serve_create(fe_ctx c, size_t hbm_budget, int32_t max_slots, int32_t host_threads, fe_server *out)
{
    if (!c || !out) return FE_EINVAL;
    *out = nullptr;
    if (max_slots < 1 || max_slots > kMaxBatch || host_threads < 1 || host_threads > 64 || hbm_budget < (1u << 20))
        return fail(c, FE_EINVAL, "serve: max_slots 1..%d, host_threads 1..64, hbm_budget >= 1 MiB", kMaxBatch);
    HIPCALL(c, hipSetDevice(c->device));
    auto S = std::make_unique<fe_server_s>();
    S->ctx = c;
    S->max_slots = max_slots;
    auto cleanup = [&]() {
        if (S->arena_base) (void)hipFree(S->arena_base);
        if (S->jobs_d) (void)hipFree(S->jobs_d);
        if (S->flags_d) (void)hipFree(S->flags_d);
        if (S->res_d) (void)hipFree(S->res_d);
        if (S->jobs_h) (void)hipHostFree(S->jobs_h);
        if (S->kargs_d) (void)hipFree(S->kargs_d);
        if (S->kargs_h) (void)hipHostFree(S->kargs_h);
        if (S->flags_h) (void)hipHostFree(S->flags_h);
        if (S->res_h) (void)hipHostFree(S->res_h);
        if (S->poll_ev) (void)hipEventDestroy(S->poll_ev);
        if (S->stream) (void)hipStreamDestroy(S->stream);
    };
    bool ok = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&S->poll_ev, hipEventDisableTiming) == hipSuccess &&
              hipMalloc((void **)&S->arena_base, hbm_budget) == hipSuccess &&
              hipMalloc((void **)&S->jobs_d, kMaxBatch * sizeof(BatchJob)) == hipSuccess &&
              hipMalloc((void **)&S->flags_d, kMaxBatch * 4 * sizeof(int32_t)) == hipSuccess &&
              hipMalloc((void **)&S->res_d, kMaxBatch * kResDoubles * sizeof(double)) == hipSuccess &&
              hipHostMalloc((void **)&S->jobs_h, kMaxBatch * sizeof(BatchJob), hipHostMallocDefault) == hipSuccess &&
              hipMalloc((void **)&S->kargs_d, 2 * kMaxBatch * kKArgsBytes) == hipSuccess &&
              hipHostMalloc((void **)&S->kargs_h, 2 * kMaxBatch * kKArgsBytes, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void **)&S->flags_h, kMaxBatch * 4 * sizeof(int32_t), hipHostMallocDefault) ==
                  hipSuccess &&
              hipHostMalloc((void **)&S->res_h, kMaxBatch * kResDoubles * sizeof(double), hipHostMallocDefault) ==
                  hipSuccess;
    if (!ok) {
        cleanup();
        return fail(c, FE_ENOMEM, "serve: could not allocate the arena (%zu bytes) or its tables", hbm_budget);
    }
    memset(S->jobs_h, 0, kMaxBatch * sizeof(BatchJob));
    memset(S->kargs_h, 0, 2 * kMaxBatch * kKArgsBytes);
    S->sctx.device = c->device;
    S->sctx.stream = S->stream;
    memset(S->flags_h, 0, kMaxBatch * 4 * sizeof(int32_t));
    S->arena = std::make_unique<DevArena>(S->arena_base, hbm_budget);
    S->stage.assign(kMaxBatch, nullptr);
    S->stage_cap.assign(kMaxBatch, 0);
    for (int s = max_slots - 1; s >= 0; --s) S->free_slots.push_back(s);
    S->pool_cap = (size_t)host_threads;
    fe_server_s *raw = S.release();
    for (int t = 0; t < host_threads; ++t) raw->planners.emplace_back(planner_main, raw);
    raw->dispatcher = std::thread(dispatcher_main, raw);
    *out = raw;
    return FE_OK;
}

fe_status fe_serve_submit(fe_server S, const fe_job *job, int64_t *ticket)
{
    if (!S || !job || !ticket) return FE_EINVAL;
    auto j = std::make_unique<Job>();
    j->desc = *job;
    j->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return FE_EINVAL;
    j->ticket = S->next_ticket++;
    *ticket = j->ticket;
    S->submit_q.push_back(j.get());
    S->jobs.emplace(j->ticket, std::move(j));
    S->cv_plan.notify_one();
    return FE_OK;
}

fe_status fe_serve_poll(fe_server S, int64_t ticket, int32_t *done, fe_job_result *result)
{
    if (!S || !done) return FE_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return FE_EINVAL;
    Job *j = it->second.get();
    *done = j->phase == kDone ? 1 : 0;
    if (*done) {
        fill_result(j, result);
        S->jobs.erase(it);
    }
    return FE_OK;
}

fe_status fe_serve_wait(fe_server S, int64_t ticket, fe_job_result *result)
{
    if (!S) return FE_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return FE_EINVAL;
    Job *j = it->second.get();
    S->cv_done.wait(lk, [&] { return j->phase == kDone; });
    fill_result(j, result);
    S->jobs.erase(ticket);
    return FE_OK;
}

fe_status fe_serve_stats(fe_server S, int64_t *completed, int64_t *batches, int64_t *batched_requests)
{
    if (!S) return FE_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (completed) *completed = S->completed;
    if (batches) *batches = S->batches;
    if (batched_requests) *batched_requests = S->batched_requests;
    return FE_OK;
}

void fe_serve_destroy(fe_server S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_plan.notify_all();
    S->cv_work.notify_all();
    for (auto &t : S->planners) t.join();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->cv_work.notify_all();
    }
    S->dispatcher.join();
    (void)hipSetDevice(S->ctx->device);
    (void)hipStreamSynchronize(S->stream);
    for (double *p : S->stage)
        if (p) (void)hipHostFree(p);
    (void)hipFree(S->arena_base);
    (void)hipFree(S->jobs_d);
    (void)hipFree(S->flags_d);
    (void)hipFree(S->res_d);
    (void)hipHostFree(S->jobs_h);
    (void)hipFree(S->kargs_d);
    (void)hipHostFree(S->kargs_h);
    (void)hipHostFree(S->flags_h);
    (void)hipHostFree(S->res_h);
    (void)hipEventDestroy(S->poll_ev);
    (void)hipStreamDestroy(S->stream);
    delete S;
}

}  // extern "C"
