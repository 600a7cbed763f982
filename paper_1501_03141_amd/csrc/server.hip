// Serving loop: a queue of PDEP jobs (setup + pdep_eigs) run by a pool of worker
// threads, admitted in submission order under an HBM budget.  Each worker owns a HIP
// stream (non-blocking, default priority) and a rocBLAS handle; a job's device memory
// comes from stream-ordered allocations on that stream, so admitting a job never
// synchronises the device and the kernels of concurrently running jobs overlap.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
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
    return S->committed + j->est <= S->budget || S->running == 0;
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
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return fail(PDEP_ENOTFOUND, "unknown ticket");
    JobRec* j = it->second.get();
    auto finished = [&] { return j->state == PDEP_JOB_DONE || j->state == PDEP_JOB_FAILED; };
    if (timeout_ms < 0)
        S->done_cv.wait(lk, finished);
    else
        S->done_cv.wait_for(lk, std::chrono::microseconds((long long)(timeout_ms * 1000.0)), finished);
    *state = j->state;
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
    delete S;
    return PDEP_OK;
}

}  // extern "C"
