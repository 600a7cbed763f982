// Serving loop: a queue of PDEP jobs (setup + pdep_eigs) run by a pool of worker
// threads, admitted in submission order under an HBM budget.  Each worker owns a HIP
// stream (non-blocking, default priority) and a rocBLAS handle; a job's device memory
// comes from stream-ordered allocations on that stream, so admitting a job never
// synchronises the device and the kernels of concurrently running jobs overlap.
//
// Resident systems: a context set up once and kept, with one batcher thread and its
// own stream, serving chi0 requests.  The batcher takes the requests queued on its
// system in order (up to max_batch_pert perturbations), runs them as one chi0_apply on
// their concatenated perturbations and hands each request its rows of the result.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "pdep_internal.h"

namespace {

using Clock = std::chrono::steady_clock;
double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

thread_local std::string t_err;

struct JobRec {
    uint64_t ticket = 0;
    pdep_job job{};
    std::vector<double> vloc;
    int state = PDEP_JOB_QUEUED;
    int status = PDEP_OK;
    std::string msg;
    std::vector<double> eps;
    size_t est = 0, chi0_budget = 0;
    int eig_iterations = 0;
    double gap = 0.0;
    Clock::time_point t_submit, t_start, t_end;
};

}  // namespace

struct Chi0Req {
    uint64_t ticket = 0, sys = 0;
    bool eigs = false;              // a PDEP Davidson (pdep_submit_eigs) instead of a chi0 block
    int n_pdep = 0;                 // eigs: dielectric eigenvalues wanted
    uint64_t seed = 0;              // eigs: start block of the library generator
    pdep_eig_opts eo{};             // eigs: options
    std::vector<double> eps;        // eigs: result (descending)
    int eig_iterations = 0;
    int n_pert = 0;
    std::vector<double> phi, out;   // n_pert rows of N_pw - 1 complex (interleaved)
    int state = PDEP_JOB_QUEUED;
    int status = PDEP_OK;
    std::string msg;
    int batch_requests = 0, batch_pert = 0;
    bool delivered = false;         // out was copied to the caller and released
    pdep_apply_stats st{};
    Clock::time_point t_submit, t_start, t_end;
};

struct SysRec {
    uint64_t id = 0;
    pdep_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    rocblas_handle blas = nullptr;
    int max_batch = 0;        // perturbations per batch (0: no limit)
    int npw = 0;              // N_pw of the system (rows of N_pw - 1 complex on S')
    size_t est = 0;           // committed against the server budget while resident
    double gap = 0.0;         // HOMO-LUMO gap of its ground state
    pdep_info info{};         // sizes and ground-state figures, fixed once it is set up
    bool stop = false;
    std::deque<Chi0Req*> queue;
    std::condition_variable cv;   // waits on the server mutex
    std::thread batcher;
};

struct pdep_server {
    pdep_server_opts opts{};
    int device = 0;
    size_t budget = 0;
    std::mutex mu;
    std::condition_variable cv;      // wakes workers (new job, capacity freed, stop)
    std::condition_variable done_cv; // wakes pdep_server_wait
    std::deque<JobRec*> queue;
    std::map<uint64_t, std::unique_ptr<JobRec>> jobs;
    uint64_t next_ticket = 1;
    bool stop = false;
    int running = 0, peak_running = 0, n_done = 0, n_failed = 0;
    size_t committed = 0, peak_committed = 0;
    std::vector<std::thread> workers;
    std::map<uint64_t, std::unique_ptr<SysRec>> systems;
    std::map<uint64_t, std::unique_ptr<Chi0Req>> reqs;
    uint64_t next_system = 1;
};

namespace {

void* stream_alloc(size_t bytes, void* ctx) {
    void* p = nullptr;
    if (hipMallocAsync(&p, bytes, static_cast<hipStream_t>(ctx)) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}
void stream_free(void* p, void* ctx) { (void)hipFreeAsync(p, static_cast<hipStream_t>(ctx)); }

bool admissible(pdep_server* S) {
    if (S->queue.empty() || S->running >= S->opts.max_running) return false;
    const JobRec* j = S->queue.front();
    // a job that does not fit starts only on an otherwise empty device (no running job and
    // no resident system holds memory), so that a job larger than the free budget cannot
    // wait forever behind smaller ones
    return S->committed + j->est <= S->budget || (S->running == 0 && S->committed == 0);
}

void run_fake(pdep_server* S, JobRec* j) {
    const double ms = S->opts.fake_ms_per_gb * (double)j->est / 1e9;
    std::this_thread::sleep_for(std::chrono::microseconds((long long)(ms * 1000.0)));
    if (j->job.opts.cg_maxit == 1) {          // forced failure for isolation tests
        j->status = PDEP_ENOTCONV;
        j->msg = "forced failure (cg_maxit = 1)";
        return;
    }
    j->eps.resize(j->job.n_pdep);
    for (int i = 0; i < j->job.n_pdep; ++i) j->eps[i] = 1.0 + (double)(j->job.seed % 97 + 1) / (i + 1);
    j->status = PDEP_OK;
}

void run_gpu(JobRec* j, hipStream_t stream, rocblas_handle blas) {
    pdep_opts o = j->job.opts;
    o.stream = stream;
    o.alloc.alloc = stream_alloc;
    o.alloc.free = stream_free;
    o.alloc.ctx = stream;
    o.flags = 0;
    o.hbm_budget = j->chi0_budget;
    pdep_ctx* ctx = nullptr;
    int rc = pdep::setup_context(&j->job.cell, j->vloc.data(), &o, nullptr, nullptr, blas, &ctx);
    if (rc != PDEP_OK) {
        j->status = rc;
        j->msg = pdep_last_error();
        return;
    }
    pdep_info info{};
    pdep_get_info(ctx, &info);
    j->gap = info.gap;
    j->eps.assign(j->job.n_pdep, 0.0);
    pdep_eig_stats st{};
    rc = pdep_eigs(ctx, j->job.n_pdep, j->job.seed, nullptr, &j->job.eig, j->eps.data(), nullptr, &st);
    if (rc != PDEP_OK) j->msg = pdep_last_error();
    j->status = rc;
    j->eig_iterations = st.iterations;
    pdep_destroy(ctx);
    (void)hipStreamSynchronize(stream);
}

void worker_main(pdep_server* S) {
    const bool fake = (S->opts.flags & PDEP_SERVER_FAKE) != 0;
    hipStream_t stream = nullptr;
    rocblas_handle blas = nullptr;
    if (!fake) {
        (void)hipSetDevice(S->device);
        if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
        if (rocblas_create_handle(&blas) != rocblas_status_success) blas = nullptr;
        if (blas) rocblas_set_stream(blas, stream);
    }
    for (;;) {
        JobRec* j = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->stop || admissible(S); });
            if (S->stop) break;
            j = S->queue.front();
            S->queue.pop_front();
            j->state = PDEP_JOB_RUNNING;
            j->t_start = Clock::now();
            S->committed += j->est;
            S->running += 1;
            S->peak_committed = std::max(S->peak_committed, S->committed);
            S->peak_running = std::max(S->peak_running, S->running);
        }
        if (fake) {
            run_fake(S, j);
        } else if (!stream || !blas) {
            j->status = PDEP_EDEVICE;
            j->msg = "worker could not create its stream / rocBLAS handle";
        } else {
            run_gpu(j, stream, blas);
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            j->t_end = Clock::now();
            j->state = j->status == PDEP_OK ? PDEP_JOB_DONE : PDEP_JOB_FAILED;
            (j->status == PDEP_OK ? S->n_done : S->n_failed) += 1;
            S->committed -= j->est;
            S->running -= 1;
        }
        S->cv.notify_all();
        S->done_cv.notify_all();
    }
    if (blas) rocblas_destroy_handle(blas);
    if (stream) (void)hipStreamDestroy(stream);
}

// One batch at a time for system y: the queued requests in order, up to y->max_batch
// perturbations (at least one request), as one chi0_apply.
void batcher_main(pdep_server* S, SysRec* y) {
    const bool fake = (S->opts.flags & PDEP_SERVER_FAKE) != 0;
    if (!fake) (void)hipSetDevice(S->device);
    const size_t row = 2 * (size_t)(y->npw - 1);   // doubles per perturbation
    std::vector<double> phi, out;
    for (;;) {
        std::vector<Chi0Req*> batch;
        int np = 0;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            y->cv.wait(lk, [&] { return y->stop || !y->queue.empty(); });
            if (y->stop) break;
            while (!y->queue.empty()) {
                Chi0Req* r = y->queue.front();
                // a PDEP Davidson runs alone; chi0 blocks batch up to max_batch perturbations
                if (!batch.empty() && (r->eigs || batch[0]->eigs)) break;
                if (!batch.empty() && y->max_batch > 0 && np + r->n_pert > y->max_batch) break;
                y->queue.pop_front();
                batch.push_back(r);
                np += r->n_pert;
            }
            const auto now = Clock::now();
            for (Chi0Req* r : batch) {
                r->state = PDEP_JOB_RUNNING;
                r->t_start = now;
                r->batch_requests = (int)batch.size();
                r->batch_pert = np;
            }
        }
        if (batch[0]->eigs) {
            Chi0Req* r = batch[0];
            std::vector<double> eps(r->n_pdep, 0.0);
            int rc = PDEP_OK, iters = 0;
            std::string msg;
            if (fake) {
                std::this_thread::sleep_for(std::chrono::microseconds((long long)(S->opts.fake_ms_per_gb * 1000.0)));
                for (int i = 0; i < r->n_pdep; ++i) eps[i] = 1.0 + (double)(r->seed % 97 + 1) / (i + 1);
            } else {
                pdep_eig_stats est{};
                rc = pdep_eigs(y->ctx, r->n_pdep, r->seed, nullptr, &r->eo, eps.data(), nullptr, &est);
                if (rc != PDEP_OK) msg = pdep_last_error();
                iters = est.iterations;
            }
            {
                std::lock_guard<std::mutex> lk(S->mu);
                r->t_end = Clock::now();
                r->status = rc;
                r->eig_iterations = iters;
                r->state = rc == PDEP_OK ? PDEP_JOB_DONE : PDEP_JOB_FAILED;
                if (rc == PDEP_OK) r->eps.swap(eps);
                else r->msg = msg;
            }
            S->done_cv.notify_all();
            continue;
        }
        int rc = PDEP_OK;
        std::string msg;
        pdep_apply_stats st{};
        size_t off = 0;
        try {
            phi.resize((size_t)np * row);
            out.assign((size_t)np * row, 0.0);
        } catch (const std::bad_alloc&) {
            rc = PDEP_ENOMEM;
            msg = "no host memory for the batch";
        }
        if (rc == PDEP_OK)
            for (Chi0Req* r : batch) {
                std::copy(r->phi.begin(), r->phi.end(), phi.begin() + off);
                off += r->phi.size();
            }
        if (rc == PDEP_OK && fake) {
            const double ms = S->opts.fake_ms_per_gb + np;
            std::this_thread::sleep_for(std::chrono::microseconds((long long)(ms * 1000.0)));
            for (size_t i = 0; i < phi.size(); ++i) out[i] = -0.5 * phi[i];
        } else if (rc == PDEP_OK) {
            rc = chi0_apply(y->ctx, np, phi.data(), out.data(), &st);
            if (rc != PDEP_OK) msg = pdep_last_error();
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            const auto now = Clock::now();
            off = 0;
            for (Chi0Req* r : batch) {
                r->t_end = now;
                r->status = rc;
                r->st = st;
                if (rc == PDEP_OK) {
                    try {
                        r->out.assign(out.begin() + off, out.begin() + off + (size_t)r->n_pert * row);
                    } catch (const std::bad_alloc&) {
                        r->status = PDEP_ENOMEM;
                        r->msg = "no host memory for the request's result";
                    }
                } else {
                    r->msg = msg;
                }
                r->state = r->status == PDEP_OK ? PDEP_JOB_DONE : PDEP_JOB_FAILED;
                off += (size_t)r->n_pert * row;
                std::vector<double>().swap(r->phi);
            }
        }
        S->done_cv.notify_all();
    }
}

// Stop a system's batcher (its queued requests fail) and free it; y is out of the map.
void close_system(pdep_server* S, std::unique_ptr<SysRec> y) {
    {
        std::lock_guard<std::mutex> lk(S->mu);
        y->stop = true;
        const auto now = Clock::now();
        for (Chi0Req* r : y->queue) {
            r->state = PDEP_JOB_FAILED;
            r->status = PDEP_EINVAL;
            r->msg = "system removed before the request ran";
            r->t_start = r->t_end = now;
        }
        y->queue.clear();
    }
    y->cv.notify_all();
    S->done_cv.notify_all();
    if (y->batcher.joinable()) y->batcher.join();
    int dev_prev = -1;   // the caller's current device, restored after the frees
    if (y->stream && hipGetDevice(&dev_prev) != hipSuccess) {
        (void)hipGetLastError();
        dev_prev = -1;
    }
    if (y->stream) (void)hipSetDevice(S->device);
    if (y->ctx) pdep_destroy(y->ctx);
    if (y->stream) (void)hipStreamSynchronize(y->stream);
    if (y->blas) rocblas_destroy_handle(y->blas);
    if (y->stream) (void)hipStreamDestroy(y->stream);
    if (dev_prev >= 0 && dev_prev != S->device) (void)hipSetDevice(dev_prev);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->committed -= y->est;
    }
    S->cv.notify_all();   // a queued job may fit in the memory the system held
}

int fail(int code, const std::string& m) {
    t_err = m;
    pdep_set_error_message(m.c_str());
    return code;
}

}  // namespace

namespace pdep {

size_t job_hbm_estimate(const pdep_cell& cell, const pdep_opts& o, int n_pdep, const pdep_eig_opts& eo,
                        size_t* chi0_budget) {
    Basis b;
    build_basis(cell, b);
    const size_t nv = (size_t)std::max(1, o.n_v), npw = b.npw, ng = b.ng;
    const size_t ld = (npw + 63) / 64 * 64;
    const size_t sticks_row = (size_t)b.dims.nz * b.dims.sld * 16;
    const size_t fixed = ng * 12 + nv * npw * 48 + (nv + 1) / 2 * ng * 16 + npw * 64 + ((size_t)64 << 20);
    // ground state (Davidson on N_v + 1 states)
    const size_t want = nv + 1, nbg = want + std::max<size_t>(4, want / 8);
    const size_t mg = std::min(npw, std::max(3 * nbg, nbg + 32));
    const size_t gs = 2 * mg * ld * 16 + 3 * nbg * ld * 16 + mg * sticks_row + mg * mg * 16 * 2;
    // PDEP Davidson and one chi0 tile
    const size_t nb = (size_t)n_pdep + (size_t)std::max(0, eo.n_buffer);
    const size_t mp = (size_t)pdep_subspace_max(b.npw, n_pdep, eo);
    const size_t dav = 2 * mp * ld * 16 + 4 * nb * ld * 16 + mp * mp * 16 * 2 + ((size_t)64 << 20);
    const size_t inner = o.precision != PDEP_FP64 ? 8 : 16;
    const size_t row = ld * 16 * 5 + ld * inner * 11 + sticks_row + nv * 16 + 256;
    const size_t per_pert = nv * row + 2 * ng * 8;
    const size_t tile = std::min<size_t>(nb, 16);
    const size_t chi0 = tile * per_pert + (size_t)(8 << 20) * 16;
    if (chi0_budget) *chi0_budget = tile * per_pert;
    return fixed + std::max(gs, dav + chi0);
}

}  // namespace pdep

extern "C" {

int pdep_server_create(const pdep_server_opts* o, pdep_server** out) {
    if (out) *out = nullptr;
    if (!o || !out) return fail(PDEP_EINVAL, "null argument");
    if (o->max_running < 1) return fail(PDEP_EINVAL, "max_running must be >= 1");
    auto S = std::make_unique<pdep_server>();
    S->opts = *o;
    if (S->opts.queue_capacity <= 0) S->opts.queue_capacity = 1024;
    const bool fake = (o->flags & PDEP_SERVER_FAKE) != 0;
    if (!fake) {
        if (hipGetDevice(&S->device) != hipSuccess) {
            (void)hipGetLastError();
            return fail(PDEP_EDEVICE, "no HIP device");
        }
    }
    S->budget = o->hbm_budget;
    if (S->budget == 0) {
        size_t fr = 0, tot = 0;
        if (fake || hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            fr = (size_t)64 << 30;
        }
        S->budget = (size_t)(0.8 * (double)fr);
    }
    for (int w = 0; w < o->max_running; ++w) S->workers.emplace_back(worker_main, S.get());
    *out = S.release();
    return PDEP_OK;
}

int pdep_submit(pdep_server* S, const pdep_job* job, uint64_t* ticket) {
    if (!S || !job || !ticket) return fail(PDEP_EINVAL, "null argument");
    auto j = std::make_unique<JobRec>();
    j->job = *job;
    try {
        PDEP_REQUIRE(job->vloc != nullptr, PDEP_EINVAL, "null vloc");
        PDEP_REQUIRE(job->opts.n_v >= 1, PDEP_EINVAL, "n_v must be >= 1");
        PDEP_REQUIRE(job->n_pdep >= 1, PDEP_EINVAL, "n_pdep must be >= 1");
        PDEP_REQUIRE(job->eig.tol > 0 && job->eig.maxit >= 1 && job->eig.n_buffer >= 0 && job->eig.scr_tol >= 0 &&
                         job->eig.scr_maxit >= 0 && (job->eig.reducible == 0 || job->eig.reducible == 1),
                     PDEP_EINVAL, "bad eig options");
        PDEP_REQUIRE(job->eig.max_subspace <= 0 || job->eig.max_subspace >= 2 * (job->n_pdep + job->eig.n_buffer),
                     PDEP_EINVAL, "max_subspace must be 0 or at least 2 (n_pdep + n_buffer)");
        j->est = pdep::job_hbm_estimate(job->cell, job->opts, job->n_pdep, job->eig, &j->chi0_budget);
        const size_t ng = (size_t)job->cell.n[0] * job->cell.n[1] * job->cell.n[2];
        j->vloc.assign(job->vloc, job->vloc + ng);
        for (double v : j->vloc) PDEP_REQUIRE(std::isfinite(v), PDEP_EINVAL, "V_loc contains NaN or Inf");
    } catch (const pdep::Error& e) {
        return fail(e.code, e.what());
    } catch (const std::exception& e) {
        return fail(PDEP_EINVAL, e.what());
    }
    j->job.vloc = nullptr;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(PDEP_EINVAL, "server is shutting down");
    if (j->est > S->budget)
        return fail(PDEP_ENOMEM, "job needs " + std::to_string(j->est >> 20) + " MiB, budget is " +
                                     std::to_string(S->budget >> 20) + " MiB");
    if ((int)S->queue.size() >= S->opts.queue_capacity) return fail(PDEP_EBUSY, "queue full");
    j->ticket = S->next_ticket++;
    j->t_submit = Clock::now();
    *ticket = j->ticket;
    S->queue.push_back(j.get());
    S->jobs[j->ticket] = std::move(j);
    S->cv.notify_all();
    return PDEP_OK;
}

int pdep_poll(pdep_server* S, uint64_t ticket, int* state, pdep_job_result* res, double* eps_out, int eps_cap) {
    if (!S || !state) return fail(PDEP_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return fail(PDEP_ENOTFOUND, "unknown ticket");
    JobRec* j = it->second.get();
    *state = j->state;
    if (res) {
        std::memset(res, 0, sizeof(*res));
        res->n_pdep = j->job.n_pdep;
        res->hbm_estimate = j->est;
        if (j->state == PDEP_JOB_DONE || j->state == PDEP_JOB_FAILED) {
            res->status = j->status;
            res->eig_iterations = j->eig_iterations;
            res->gap = j->gap;
            res->queue_ms = ms_between(j->t_submit, j->t_start);
            res->run_ms = ms_between(j->t_start, j->t_end);
            res->latency_ms = ms_between(j->t_submit, j->t_end);
        }
    }
    if (j->state == PDEP_JOB_DONE && eps_out)
        for (int i = 0; i < std::min(eps_cap, (int)j->eps.size()); ++i) eps_out[i] = j->eps[i];
    if (j->state == PDEP_JOB_FAILED) pdep_set_error_message(j->msg.c_str());
    return PDEP_OK;
}

int pdep_server_wait(pdep_server* S, uint64_t ticket, double timeout_ms, int* state) {
    if (!S || !state) return fail(PDEP_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(S->mu);
    int* st = nullptr;   // state of the job or chi0 request (records are never erased)
    if (auto it = S->jobs.find(ticket); it != S->jobs.end()) st = &it->second->state;
    else if (auto ir = S->reqs.find(ticket); ir != S->reqs.end()) st = &ir->second->state;
    if (!st) return fail(PDEP_ENOTFOUND, "unknown ticket");
    auto finished = [&] { return *st == PDEP_JOB_DONE || *st == PDEP_JOB_FAILED; };
    if (timeout_ms < 0)
        S->done_cv.wait(lk, finished);
    else
        S->done_cv.wait_for(lk, std::chrono::microseconds((long long)(timeout_ms * 1000.0)), finished);
    *state = *st;
    return PDEP_OK;
}

int pdep_server_stats_get(pdep_server* S, pdep_server_stats* st) {
    if (!S || !st) return fail(PDEP_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    st->queued = (int)S->queue.size();
    st->running = S->running;
    st->done = S->n_done;
    st->failed = S->n_failed;
    st->committed_bytes = S->committed;
    st->peak_committed_bytes = S->peak_committed;
    st->peak_running = S->peak_running;
    return PDEP_OK;
}

int pdep_server_add_system(pdep_server* S, const pdep_cell* cell, const double* vloc, const pdep_opts* opts,
                           int max_batch_pert, uint64_t* system_id) {
    if (!S || !cell || !vloc || !opts || !system_id) return fail(PDEP_EINVAL, "null argument");
    if (max_batch_pert < 0) return fail(PDEP_EINVAL, "max_batch_pert must be >= 0");
    const bool fake = (S->opts.flags & PDEP_SERVER_FAKE) != 0;
    auto y = std::make_unique<SysRec>();
    y->max_batch = max_batch_pert;
    try {
        PDEP_REQUIRE(opts->n_v >= 1, PDEP_EINVAL, "n_v must be >= 1");
        pdep_eig_opts eo{};
        eo.tol = 1e-6;
        eo.maxit = 1;
        y->est = pdep::job_hbm_estimate(*cell, *opts, max_batch_pert > 0 ? max_batch_pert : 16, eo, nullptr);
        pdep::Basis b;
        pdep::build_basis(*cell, b);
        y->npw = b.npw;
        const size_t ng = (size_t)cell->n[0] * cell->n[1] * cell->n[2];
        for (size_t i = 0; i < ng; ++i) PDEP_REQUIRE(std::isfinite(vloc[i]), PDEP_EINVAL, "V_loc contains NaN or Inf");
    } catch (const pdep::Error& e) {
        return fail(e.code, e.what());
    } catch (const std::exception& e) {
        return fail(PDEP_EINVAL, e.what());
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) return fail(PDEP_EINVAL, "server is shutting down");
        if (S->committed + y->est > S->budget)
            return fail(PDEP_ENOMEM, "system needs " + std::to_string(y->est >> 20) + " MiB, " +
                                         std::to_string((S->budget - std::min(S->budget, S->committed)) >> 20) +
                                         " MiB of the budget are free");
        S->committed += y->est;   // reserved while the system is set up and resident
        S->peak_committed = std::max(S->peak_committed, S->committed);
    }
    // the system lives on the server's device; the caller's current device is restored
    int dev_prev = -1;
    if (!fake && hipGetDevice(&dev_prev) != hipSuccess) {
        (void)hipGetLastError();
        dev_prev = -1;
    }
    auto restore_device = [&] {
        if (dev_prev >= 0 && dev_prev != S->device) (void)hipSetDevice(dev_prev);
    };
    auto release = [&](int code, const std::string& m) {
        if (y->blas) rocblas_destroy_handle(y->blas);
        if (y->stream) (void)hipStreamDestroy(y->stream);
        restore_device();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->committed -= y->est;
        }
        S->cv.notify_all();   // a queued job may fit in the memory reserved here
        return fail(code, m);
    };
    if (!fake) {
        if (hipSetDevice(S->device) != hipSuccess) {
            (void)hipGetLastError();
            return release(PDEP_EDEVICE, "could not select the server's device");
        }
        if (hipStreamCreateWithFlags(&y->stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            y->stream = nullptr;
            return release(PDEP_EDEVICE, "could not create the system's stream");
        }
        if (rocblas_create_handle(&y->blas) != rocblas_status_success) {
            y->blas = nullptr;
            return release(PDEP_EDEVICE, "could not create the system's rocBLAS handle");
        }
        rocblas_set_stream(y->blas, y->stream);
        pdep_opts o = *opts;
        o.stream = y->stream;
        o.alloc.alloc = stream_alloc;
        o.alloc.free = stream_free;
        o.alloc.ctx = y->stream;
        o.flags = 0;   // host arrays: requests hold host copies
        const int rc = pdep::setup_context(cell, vloc, &o, nullptr, nullptr, y->blas, &y->ctx);
        if (rc != PDEP_OK) return release(rc, pdep_last_error());
        pdep_get_info(y->ctx, &y->info);
        y->npw = y->info.n_pw;
        y->gap = y->info.gap;
        restore_device();
    } else {
        y->info.n_pw = y->npw;
        y->info.n_v = opts->n_v;
        y->info.n_grid = cell->n[0] * cell->n[1] * cell->n[2];
        y->info.volume = cell->L[0] * cell->L[1] * cell->L[2];
    }
    SysRec* yp = y.get();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        y->id = S->next_system++;
        *system_id = y->id;
        S->systems[y->id] = std::move(y);
        yp->batcher = std::thread(batcher_main, S, yp);
    }
    return PDEP_OK;
}

int pdep_server_system_info(pdep_server* S, uint64_t system_id, pdep_info* info) {
    if (!S || !info) return fail(PDEP_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->systems.find(system_id);
    if (it == S->systems.end()) return fail(PDEP_ENOTFOUND, "unknown system");
    *info = it->second->info;
    return PDEP_OK;
}

int pdep_server_remove_system(pdep_server* S, uint64_t system_id) {
    if (!S) return fail(PDEP_EINVAL, "null argument");
    std::unique_ptr<SysRec> y;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->systems.find(system_id);
        if (it == S->systems.end()) return fail(PDEP_ENOTFOUND, "unknown system");
        y = std::move(it->second);
        S->systems.erase(it);
    }
    close_system(S, std::move(y));
    return PDEP_OK;
}

int pdep_submit_chi0(pdep_server* S, uint64_t system_id, int n_pert, const double* phi, uint64_t* ticket) {
    if (!S || !phi || !ticket) return fail(PDEP_EINVAL, "null argument");
    if (n_pert < 1) return fail(PDEP_EINVAL, "n_pert must be >= 1");
    int npw = 0;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->systems.find(system_id);
        if (it == S->systems.end()) return fail(PDEP_ENOTFOUND, "unknown system");
        npw = it->second->npw;
    }
    std::unique_ptr<Chi0Req> r;
    try {
        r = std::make_unique<Chi0Req>();
        r->phi.assign(phi, phi + (size_t)n_pert * 2 * (size_t)(npw - 1));
    } catch (const std::bad_alloc&) {
        return fail(PDEP_ENOMEM, "no host memory for the request's copy of phi");
    }
    r->sys = system_id;
    r->n_pert = n_pert;
    for (double v : r->phi)
        if (!std::isfinite(v)) return fail(PDEP_EINVAL, "phi contains NaN or Inf");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(PDEP_EINVAL, "server is shutting down");
    auto it = S->systems.find(system_id);
    if (it == S->systems.end()) return fail(PDEP_ENOTFOUND, "system removed");
    SysRec* y = it->second.get();
    if ((int)y->queue.size() >= S->opts.queue_capacity) return fail(PDEP_EBUSY, "queue full");
    r->ticket = S->next_ticket++;
    r->t_submit = Clock::now();
    *ticket = r->ticket;
    y->queue.push_back(r.get());
    S->reqs[r->ticket] = std::move(r);
    y->cv.notify_all();
    return PDEP_OK;
}

int pdep_submit_eigs(pdep_server* S, uint64_t system_id, int n_pdep, uint64_t seed, const pdep_eig_opts* eo,
                     uint64_t* ticket) {
    if (!S || !eo || !ticket) return fail(PDEP_EINVAL, "null argument");
    if (n_pdep < 1) return fail(PDEP_EINVAL, "n_pdep must be >= 1");
    if (!(eo->tol > 0 && eo->maxit >= 1 && eo->n_buffer >= 0 && eo->scr_tol >= 0 && eo->scr_maxit >= 0 &&
          (eo->reducible == 0 || eo->reducible == 1)))
        return fail(PDEP_EINVAL, "bad eig options");
    if (eo->max_subspace > 0 && eo->max_subspace < 2 * (n_pdep + eo->n_buffer))
        return fail(PDEP_EINVAL, "max_subspace must be 0 or at least 2 (n_pdep + n_buffer)");
    auto r = std::make_unique<Chi0Req>();
    r->sys = system_id;
    r->eigs = true;
    r->n_pdep = n_pdep;
    r->seed = seed;
    r->eo = *eo;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return fail(PDEP_EINVAL, "server is shutting down");
    auto it = S->systems.find(system_id);
    if (it == S->systems.end()) return fail(PDEP_ENOTFOUND, "unknown system");
    SysRec* y = it->second.get();
    if (n_pdep >= y->npw - 1) return fail(PDEP_EINVAL, "n_pdep must be below the number of plane waves");
    if ((int)y->queue.size() >= S->opts.queue_capacity) return fail(PDEP_EBUSY, "queue full");
    r->ticket = S->next_ticket++;
    r->t_submit = Clock::now();
    *ticket = r->ticket;
    y->queue.push_back(r.get());
    S->reqs[r->ticket] = std::move(r);
    y->cv.notify_all();
    return PDEP_OK;
}

int pdep_poll_eigs(pdep_server* S, uint64_t ticket, int* state, pdep_job_result* res, double* eps_out, int eps_cap) {
    if (!S || !state) return fail(PDEP_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end() || !it->second->eigs) return fail(PDEP_ENOTFOUND, "unknown ticket");
    const Chi0Req* r = it->second.get();
    *state = r->state;
    if (res) {
        std::memset(res, 0, sizeof(*res));
        res->n_pdep = r->n_pdep;
        if (auto sy = S->systems.find(r->sys); sy != S->systems.end()) {
            res->hbm_estimate = sy->second->est;
            res->gap = sy->second->gap;
        }
        if (r->state == PDEP_JOB_DONE || r->state == PDEP_JOB_FAILED) {
            res->status = r->status;
            res->eig_iterations = r->eig_iterations;
            res->queue_ms = ms_between(r->t_submit, r->t_start);
            res->run_ms = ms_between(r->t_start, r->t_end);
            res->latency_ms = ms_between(r->t_submit, r->t_end);
        }
    }
    if (r->state == PDEP_JOB_DONE && eps_out)
        for (int i = 0; i < std::min(eps_cap, (int)r->eps.size()); ++i) eps_out[i] = r->eps[i];
    if (r->state == PDEP_JOB_FAILED) pdep_set_error_message(r->msg.c_str());
    return PDEP_OK;
}

int pdep_poll_chi0(pdep_server* S, uint64_t ticket, int* state, pdep_chi0_result* res, double* out,
                   int out_cap_pert) {
    if (!S || !state) return fail(PDEP_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end() || it->second->eigs) return fail(PDEP_ENOTFOUND, "unknown ticket");
    Chi0Req* r = it->second.get();
    *state = r->state;
    if (res) {
        std::memset(res, 0, sizeof(*res));
        res->n_pert = r->n_pert;
        if (r->state != PDEP_JOB_QUEUED) {
            res->batch_requests = r->batch_requests;
            res->batch_pert = r->batch_pert;
        }
        if (r->state == PDEP_JOB_DONE || r->state == PDEP_JOB_FAILED) {
            res->status = r->status;
            res->queue_ms = ms_between(r->t_submit, r->t_start);
            res->run_ms = ms_between(r->t_start, r->t_end);
            res->latency_ms = ms_between(r->t_submit, r->t_end);
            res->stats = r->st;
        }
    }
    if (r->state == PDEP_JOB_DONE && out && out_cap_pert >= r->n_pert) {
        if (r->delivered) return fail(PDEP_EINVAL, "the request's result was already delivered");
        std::copy(r->out.begin(), r->out.end(), out);
        std::vector<double>().swap(r->out);
        r->delivered = true;
    }
    if (r->state == PDEP_JOB_FAILED) pdep_set_error_message(r->msg.c_str());
    return PDEP_OK;
}

int pdep_server_destroy(pdep_server* S) {
    if (!S) return PDEP_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (JobRec* j : S->queue) {
            j->state = PDEP_JOB_FAILED;
            j->status = PDEP_EINVAL;
            j->msg = "server destroyed before the job started";
        }
        S->queue.clear();
    }
    S->cv.notify_all();
    S->done_cv.notify_all();
    for (auto& t : S->workers) t.join();
    std::vector<std::unique_ptr<SysRec>> sys;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto& kv : S->systems) sys.push_back(std::move(kv.second));
        S->systems.clear();
    }
    for (auto& y : sys) close_system(S, std::move(y));
    delete S;
    return PDEP_OK;
}

}  // extern "C"
