// C ABI entry points (declared in include/pdep.h): argument checks, host/device
// marshalling, S <-> S' conversion, timing and error reporting.  All numerical work is
// in the kernels of fft.hip / linalg.hip driven by solver.hip and davidson.hip.
#include <chrono>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "pdep_internal.h"

using pdep::Ctx;
using pdep::Error;

struct pdep_ctx {
    Ctx c;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

bool all_finite(const double* p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit Timer(hipStream_t st) : s(st) {
        PDEP_HIP(hipEventCreate(&a));
        PDEP_HIP(hipEventCreate(&b));
        PDEP_HIP(hipEventRecord(a, s));
    }
    double stop() {
        float ms = 0.f;
        PDEP_HIP(hipEventRecord(b, s));
        PDEP_HIP(hipEventSynchronize(b));
        PDEP_HIP(hipEventElapsedTime(&ms, a, b));
        return ms;
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

enum CapiSlot { C_IN = pdep::WS_CAPI_IN, C_OUT = pdep::WS_CAPI_OUT, C_STAGE = pdep::WS_CAPI_STAGE };

}  // namespace

// ------------------------------------------------------- no-allocation scratch ---
// Fixed device memory of chi0_apply_noalloc: every device the library runs on holds
// its own copy for the life of the process.  In host code `scratch` only names the
// variable; its device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_addr[kMaxDevices] = {};
std::mutex g_scratch_call_mu[kMaxDevices];   // one no-allocation call per device at a time

// Device address of device dev's copy of `scratch` (dev must be the current device the
// first time).
char* scratch_address(int dev) {
    PDEP_REQUIRE(dev >= 0 && dev < kMaxDevices, PDEP_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        PDEP_REQUIRE(e == hipSuccess && p != nullptr, PDEP_EDEVICE,
                     std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_addr[dev] = static_cast<char*>(p);
    }
    return g_scratch_addr[dev];
}

void check_ctx(pdep_ctx* ctx) { PDEP_REQUIRE(ctx != nullptr, PDEP_EINVAL, "null context"); }

// Build the resident packed orbital grids u_2j(r) + i u_2j+1(r) (the orbitals are real
// in r, so one complex grid holds two of them; the last one alone for odd N_v) and the
// FP32 copies of Psi and V.
void finish_setup(Ctx& c) {
    const pdep::Basis& b = c.basis;
    const int nv = c.nv, npw = b.npw;
    hipStream_t s = c.stream;
    const int nvp = pdep::pair_count(nv, nv);
    c.upair.ensure(&c.al, (size_t)nvp * b.ng * sizeof(double2));
    double2* sticks = static_cast<double2*>(c.ws(pdep::WS_SETUP_STICKS, (size_t)nv * b.dims.nz * b.dims.sld *
                                                                           sizeof(double2)));
    pdep::launch_sphere_to_sticks_pair<double>(b.dims, b.tables, c.psi64.as<double2>(), npw, nv, sticks, s, nv);
    pdep::launch_slab_inv_store<double>(b.dims, b.tables, sticks, nvp, c.upair.as<double2>(), nullptr, s);
    // FP32 copy with the padded sphere row stride (zero padding): 16-byte aligned rows
    const long ld32 = pdep::sphere_ld(npw);
    c.psi32.ensure(&c.al, (size_t)nv * ld32 * sizeof(float2));
    pdep::launch_fill_zero(c.psi32.get(), (size_t)nv * ld32 * sizeof(float2), s);
    pdep::launch_convert_rows<double, float>(nv, npw, c.psi64.as<double2>(), npw, nullptr, nullptr,
                                             c.psi32.as<float2>(), ld32, s);
    // weighted half-sphere copy for the projection coefficients of half-sphere rows
    c.psi32w.ensure(&c.al, (size_t)nv * ld32 * sizeof(float2));
    pdep::launch_fill_zero(c.psi32w.get(), (size_t)nv * ld32 * sizeof(float2), s);
    pdep::launch_half_weights<float>(nv, pdep::half_len(npw), c.psi32.as<float2>(), ld32, c.psi32w.as<float2>(), ld32,
                                     s);
    c.psi64w.ensure(&c.al, (size_t)nv * npw * sizeof(double2));
    pdep::launch_fill_zero(c.psi64w.get(), (size_t)nv * npw * sizeof(double2), s);
    pdep::launch_half_weights<double>(nv, pdep::half_len(npw), c.psi64.as<double2>(), npw, c.psi64w.as<double2>(),
                                      npw, s);
    c.eps_dev.ensure(&c.al, (size_t)nv * sizeof(double));
    PDEP_HIP(hipMemcpyAsync(c.eps_dev.get(), c.eps.data(), nv * sizeof(double), hipMemcpyHostToDevice, s));
    // residual of the orbitals in use
    const long ld = npw;
    double2* hx = static_cast<double2*>(c.ws(C_OUT, (size_t)nv * ld * sizeof(double2)));
    pdep::apply_h64(c, c.psi64.as<double2>(), ld, nv, c.eps_dev.as<double>(), nv, hx, ld, sticks);
    double* dots = static_cast<double*>(c.ws(C_STAGE, (size_t)nv * sizeof(double)));
    pdep::launch_row_dots<double>(nv, npw, hx, ld, hx, ld, dots, nullptr, s);
    std::vector<double> r2(nv);
    PDEP_HIP(hipMemcpyAsync(r2.data(), dots, nv * sizeof(double), hipMemcpyDeviceToHost, s));
    PDEP_HIP(hipStreamSynchronize(s));
    double mx = 0.0;
    for (double x : r2) mx = std::max(mx, std::sqrt(std::max(x, 0.0)));
    c.gs_residual = mx;
    pdep::tune_cache_load(c);
}

}  // namespace

#define API_BEGIN try {
#define API_END                                                                  \
    }                                                                            \
    catch (const Error& e) { return fail(e.code, e.what()); }                    \
    catch (const std::bad_alloc&) { return fail(PDEP_ENOMEM, "host allocation failed"); } \
    catch (const std::exception& e) { return fail(PDEP_EDEVICE, e.what()); }     \
    g_err.clear();                                                               \
    return PDEP_OK;

extern "C" {

void pdep_default_opts(pdep_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->n_v = 1;
    o->precision = PDEP_FP64;
    o->cg_tol = 1e-10;
    o->cg_maxit = 2000;
    o->inner_tol = 1e-5;
    o->refine_maxit = 8;
    o->precond = 1;
    o->gap_min = 1e-3;
    o->gs_tol = 1e-10;
    o->gs_maxit = 400;
}

const char* pdep_last_error(void) { return g_err.c_str(); }

void pdep_set_error_message(const char* m) { g_err = m ? m : ""; }

int pdep_setup(const pdep_cell* cell, const double* vloc, const pdep_opts* opts, const double* psi_in,
               const double* eps_in, pdep_ctx** out) {
    return pdep::setup_context(cell, vloc, opts, psi_in, eps_in, nullptr, out);
}

}  // extern "C"

int pdep::setup_context(const pdep_cell* cell, const double* vloc, const pdep_opts* opts, const double* psi_in,
                        const double* eps_in, void* blas, pdep_ctx** out) {
    if (out) *out = nullptr;
    pdep_ctx* ctx = nullptr;
    API_BEGIN
    PDEP_REQUIRE(cell && vloc && opts && out, PDEP_EINVAL, "null argument");
    PDEP_REQUIRE(opts->n_v >= 1, PDEP_EINVAL, "n_v must be >= 1");
    PDEP_REQUIRE(opts->precision == PDEP_FP64 || opts->precision == PDEP_MIXED_FP32 ||
                     opts->precision == PDEP_MIXED_BF16X3,
                 PDEP_EINVAL, "bad precision");
    PDEP_REQUIRE(opts->cg_tol > 0 && opts->cg_tol < 1 && opts->cg_maxit >= 1, PDEP_EINVAL, "bad CG tolerance/cap");
    PDEP_REQUIRE(opts->precision == PDEP_FP64 || (opts->inner_tol > 0 && opts->inner_tol < 1), PDEP_EINVAL,
                 "bad inner tolerance");
    PDEP_REQUIRE((psi_in == nullptr) == (eps_in == nullptr), PDEP_EINVAL, "psi_in and eps_in go together");
    ctx = new pdep_ctx();
    Ctx& c = ctx->c;
    c.blas = blas;
    c.own_blas = false;
    c.opts = *opts;
    c.al.a = opts->alloc;
    c.stream = static_cast<hipStream_t>(opts->stream);
    pdep::build_basis(*cell, c.basis);
    const pdep::Basis& b = c.basis;
    PDEP_REQUIRE(all_finite(vloc, b.ng), PDEP_EINVAL, "V_loc contains NaN or Inf");
    PDEP_REQUIRE(opts->n_v + 1 < b.npw, PDEP_EINVAL, "n_v too large for the basis");
    PDEP_HIP(hipGetDevice(&c.device));
    (void)scratch_address(c.device);   // resolved once per device, with it current
    pdep::upload_basis(c.basis, &c.al, c.stream);
    c.nv = opts->n_v;
    // the slab passes read V in z-major order [iz][ix][iy]
    std::vector<double> vz((size_t)b.ng);
    for (int ix = 0; ix < b.n[0]; ++ix)
        for (int iy = 0; iy < b.n[1]; ++iy)
            for (int iz = 0; iz < b.n[2]; ++iz)
                vz[((size_t)iz * b.n[0] + ix) * b.n[1] + iy] = vloc[((size_t)ix * b.n[1] + iy) * b.n[2] + iz];
    c.vloc64.ensure(&c.al, (size_t)b.ng * sizeof(double));
    PDEP_HIP(hipMemcpyAsync(c.vloc64.get(), vz.data(), (size_t)b.ng * sizeof(double), hipMemcpyHostToDevice, c.stream));
    std::vector<float> v32(vz.begin(), vz.end());
    c.vloc32.ensure(&c.al, (size_t)b.ng * sizeof(float));
    PDEP_HIP(hipMemcpyAsync(c.vloc32.get(), v32.data(), (size_t)b.ng * sizeof(float), hipMemcpyHostToDevice, c.stream));
    PDEP_HIP(hipStreamSynchronize(c.stream));
    if (psi_in) {
        PDEP_REQUIRE(all_finite(psi_in, (size_t)2 * c.nv * b.npw) && all_finite(eps_in, c.nv), PDEP_EINVAL,
                     "psi_in / eps_in contain NaN or Inf");
        c.eps.assign(eps_in, eps_in + c.nv);
        c.psi64.ensure(&c.al, (size_t)c.nv * b.npw * sizeof(double2));
        PDEP_HIP(hipMemcpyAsync(c.psi64.get(), psi_in, (size_t)c.nv * b.npw * sizeof(double2), hipMemcpyHostToDevice,
                                c.stream));
        c.gap = 0.0;
        c.gs_iterations = 0;
    } else {
        pdep::ground_state(c);
        if (c.gap < opts->gap_min) {
            const std::string m = "HOMO-LUMO gap " + std::to_string(c.gap) + " Ha below gap_min";
            delete ctx;
            ctx = nullptr;
            return fail(PDEP_EGAP, m);
        }
    }
    pdep::realify_orbitals(c);
    finish_setup(c);
    *out = ctx;
    ctx = nullptr;
    }
    catch (const Error& e) { delete ctx; return fail(e.code, e.what()); }
    catch (const std::bad_alloc&) { delete ctx; return fail(PDEP_ENOMEM, "host allocation failed"); }
    catch (const std::exception& e) { delete ctx; return fail(PDEP_EDEVICE, e.what()); }
    g_err.clear();
    return PDEP_OK;
}

extern "C" {

int pdep_get_info(pdep_ctx* ctx, pdep_info* info) {
    API_BEGIN
    check_ctx(ctx);
    PDEP_REQUIRE(info != nullptr, PDEP_EINVAL, "null info");
    const Ctx& c = ctx->c;
    info->n_pw = c.basis.npw;
    info->n_v = c.nv;
    info->n_grid = c.basis.ng;
    info->gap = c.gap;
    info->volume = c.basis.omega;
    info->gs_iterations = c.gs_iterations;
    info->gs_residual = c.gs_residual;
    API_END
}

int pdep_get_gvectors(pdep_ctx* ctx, int* n_pw, int32_t* miller) {
    API_BEGIN
    check_ctx(ctx);
    PDEP_REQUIRE(n_pw != nullptr || miller != nullptr, PDEP_EINVAL, "null n_pw and miller");
    if (n_pw) *n_pw = ctx->c.basis.npw;
    if (miller) std::memcpy(miller, ctx->c.basis.miller.data(), ctx->c.basis.miller.size() * sizeof(int32_t));
    API_END
}

int pdep_get_orbitals(pdep_ctx* ctx, double* eps, double* psi) {
    API_BEGIN
    check_ctx(ctx);
    Ctx& c = ctx->c;
    if (eps) std::memcpy(eps, c.eps.data(), c.nv * sizeof(double));
    if (psi) {
        PDEP_HIP(hipMemcpyAsync(psi, c.psi64.get(), (size_t)c.nv * c.basis.npw * sizeof(double2), hipMemcpyDeviceToHost,
                                c.stream));
        PDEP_HIP(hipStreamSynchronize(c.stream));
    }
    API_END
}

}  // extern "C"

namespace {

void fill_apply_stats(const Ctx& c, const pdep::ApplyStats& as, double ms, pdep_apply_stats* st) {
    if (!st) return;
    st->n_rhs = as.n_rhs;
    st->cg_iter_max = as.cg_iter_max;
    st->cg_iter_total = as.cg_iter_total;
    st->op_applications = as.op_applications;
    st->refine_steps = as.refine_steps;
    st->n_notconv = as.n_notconv;
    st->max_rel_residual = as.max_rel_residual;
    st->ms = ms;
    st->fft_chunk = c.opts.precision == PDEP_FP64 ? c.fft_chunk64 : c.fft_chunk32;
    st->n_fp32_fallback_rows = as.n_fp32_fallback;
    st->graph_launches = as.graph_launches;
    st->graph_captures = as.graph_captures;
    st->graph_updates = as.graph_updates;
}

// Context state that a no-allocation call changes, restored on every exit.
struct NoallocGuard {
    Ctx& c;
    int rhs_tile;
    size_t split;
    NoallocGuard(Ctx& cc, pdep::Arena* a, size_t split_elems) : c(cc), rhs_tile(cc.opts.rhs_tile), split(cc.split_elems) {
        c.arena = a;
        c.split_elems = split_elems;
    }
    ~NoallocGuard() {
        c.arena = nullptr;
        c.opts.rhs_tile = rhs_tile;
        c.split_elems = split;
    }
};

}  // namespace

extern "C" {

int chi0_apply_noalloc(pdep_ctx* ctx, int n_pert, const double* phi, double* out, pdep_apply_stats* st) {
    API_BEGIN
    check_ctx(ctx);
    Ctx& c = ctx->c;
    PDEP_REQUIRE(n_pert >= 0, PDEP_EINVAL, "n_pert must be >= 0");
    if (st) std::memset(st, 0, sizeof(*st));
    if (n_pert == 0) { g_err.clear(); return PDEP_OK; }
    PDEP_REQUIRE(phi && out, PDEP_EINVAL, "null phi/out");
    const int npw = c.basis.npw, n1 = npw - 1, g0 = c.basis.g0;
    const long ld = pdep::sphere_ld(npw);
    const bool dev = (c.opts.flags & PDEP_DEVICE_PTRS) != 0;
    hipStream_t s = c.stream;
    if (!dev) PDEP_REQUIRE(all_finite(phi, (size_t)2 * n_pert * n1), PDEP_EINVAL, "phi contains NaN or Inf");
    char* base = scratch_address(c.device);
    std::lock_guard<std::mutex> call_lk(g_scratch_call_mu[c.device]);
    pdep::ProfSuspend no_events;
    const auto t0 = std::chrono::steady_clock::now();
    pdep::Arena arena;
    arena.base = base;
    arena.cap = kScratchBytes;
    NoallocGuard guard(c, &arena, (size_t)1 << 20);
    // perturbations per pass: staging rows (in and out, plus host staging) and the chi0
    // work of one tile must fit the scratch
    const size_t stage_pp = (size_t)2 * ld * sizeof(double2) + (dev ? 0 : (size_t)n1 * sizeof(double2)) + 1024;
    int chunk = 0;
    for (int p = n_pert; p >= 1; p = p > 8 ? p - (p + 7) / 8 : p - 1)
        if ((size_t)p * stage_pp + pdep::chi0_work_bytes(c, p) <= kScratchBytes) {
            chunk = p;
            break;
        }
    PDEP_REQUIRE(chunk >= 1, PDEP_ENOMEM,
                 "one perturbation needs " + std::to_string((stage_pp + pdep::chi0_work_bytes(c, 1)) >> 20) +
                     " MiB of work space, beyond the " + std::to_string(kScratchBytes >> 20) +
                     " MiB no-allocation scratch (N_v = " + std::to_string(c.nv) + ", N_pw = " +
                     std::to_string(npw) + "): use chi0_apply");
    c.opts.rhs_tile = chunk * c.nv;   // each pass is a single tile
    pdep::ApplyStats as;
    for (int p0 = 0; p0 < n_pert; p0 += chunk) {
        const int np = std::min(chunk, n_pert - p0);
        arena.reset();
        double2* in_s = static_cast<double2*>(c.ws(C_IN, (size_t)np * ld * sizeof(double2)));
        double2* out_s = static_cast<double2*>(c.ws(C_OUT, (size_t)np * ld * sizeof(double2)));
        const double2* src = reinterpret_cast<const double2*>(phi) + (size_t)p0 * n1;
        double2* dst = reinterpret_cast<double2*>(out) + (size_t)p0 * n1;
        if (dev) {
            pdep::launch_expand_s1(np, npw, g0, src, n1, in_s, ld, s);
        } else {
            double2* stage = static_cast<double2*>(c.ws(C_STAGE, (size_t)np * n1 * sizeof(double2)));
            PDEP_HIP(hipMemcpyAsync(stage, src, (size_t)np * n1 * sizeof(double2), hipMemcpyHostToDevice, s));
            pdep::launch_expand_s1(np, npw, g0, stage, n1, in_s, ld, s);
        }
        pdep::chi0bar_sphere(c, np, in_s, out_s, as);
        if (dev) {
            pdep::launch_compact_s1(np, npw, g0, out_s, ld, dst, n1, s);
        } else {
            double2* stage = static_cast<double2*>(c.ws(C_STAGE, (size_t)np * n1 * sizeof(double2)));
            pdep::launch_compact_s1(np, npw, g0, out_s, ld, stage, n1, s);
            PDEP_HIP(hipMemcpyAsync(dst, stage, (size_t)np * n1 * sizeof(double2), hipMemcpyDeviceToHost, s));
        }
        PDEP_HIP(hipStreamSynchronize(s));   // the next pass reuses the scratch
    }
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    fill_apply_stats(c, as, ms, st);
    if (as.n_notconv > 0)
        return fail(PDEP_ENOTCONV, std::to_string(as.n_notconv) + " Sternheimer systems missed cg_tol");
    API_END
}

int chi0_apply(pdep_ctx* ctx, int n_pert, const double* phi, double* out, pdep_apply_stats* st) {
    API_BEGIN
    check_ctx(ctx);
    Ctx& c = ctx->c;
    PDEP_REQUIRE(n_pert >= 0, PDEP_EINVAL, "n_pert must be >= 0");
    if (st) std::memset(st, 0, sizeof(*st));
    if (n_pert == 0) { g_err.clear(); return PDEP_OK; }
    PDEP_REQUIRE(phi && out, PDEP_EINVAL, "null phi/out");
    const int npw = c.basis.npw, n1 = npw - 1, g0 = c.basis.g0;
    const long ld = pdep::sphere_ld(npw);
    const bool dev = (c.opts.flags & PDEP_DEVICE_PTRS) != 0;
    hipStream_t s = c.stream;
    Timer tm(s);
    double2* in_s = static_cast<double2*>(c.ws(C_IN, (size_t)n_pert * ld * sizeof(double2)));
    double2* out_s = static_cast<double2*>(c.ws(C_OUT, (size_t)n_pert * ld * sizeof(double2)));
    if (dev) {
        pdep::launch_expand_s1(n_pert, npw, g0, reinterpret_cast<const double2*>(phi), n1, in_s, ld, s);
    } else {
        PDEP_REQUIRE(all_finite(phi, (size_t)2 * n_pert * n1), PDEP_EINVAL, "phi contains NaN or Inf");
        double2* stage = static_cast<double2*>(c.ws(C_STAGE, (size_t)n_pert * n1 * sizeof(double2)));
        PDEP_HIP(hipMemcpyAsync(stage, phi, (size_t)n_pert * n1 * sizeof(double2), hipMemcpyHostToDevice, s));
        pdep::launch_expand_s1(n_pert, npw, g0, stage, n1, in_s, ld, s);
    }
    pdep::ApplyStats as;
    pdep::chi0bar_sphere(c, n_pert, in_s, out_s, as);
    if (dev) {
        pdep::launch_compact_s1(n_pert, npw, g0, out_s, ld, reinterpret_cast<double2*>(out), n1, s);
    } else {
        double2* stage = static_cast<double2*>(c.ws(C_STAGE, (size_t)n_pert * n1 * sizeof(double2)));
        pdep::launch_compact_s1(n_pert, npw, g0, out_s, ld, stage, n1, s);
        PDEP_HIP(hipMemcpyAsync(out, stage, (size_t)n_pert * n1 * sizeof(double2), hipMemcpyDeviceToHost, s));
    }
    const double ms = tm.stop();
    fill_apply_stats(c, as, ms, st);
    if (as.n_notconv > 0)
        return fail(PDEP_ENOTCONV, std::to_string(as.n_notconv) + " Sternheimer systems missed cg_tol");
    API_END
}

int chi0_apply_raw(pdep_ctx* ctx, int n_pert, const double* dv_r, double* dn_r, pdep_apply_stats* st) {
    API_BEGIN
    check_ctx(ctx);
    Ctx& c = ctx->c;
    PDEP_REQUIRE(n_pert >= 0, PDEP_EINVAL, "n_pert must be >= 0");
    if (st) std::memset(st, 0, sizeof(*st));
    if (n_pert == 0) { g_err.clear(); return PDEP_OK; }
    PDEP_REQUIRE(dv_r && dn_r, PDEP_EINVAL, "null dv/dn");
    const size_t ng = c.basis.ng;
    const bool dev = (c.opts.flags & PDEP_DEVICE_PTRS) != 0;
    hipStream_t s = c.stream;
    Timer tm(s);
    const pdep::Basis& b = c.basis;
    const size_t bytes = (size_t)n_pert * ng * sizeof(double);
    // grids cross the ABI in C order and are z-major inside
    double* stage = static_cast<double*>(c.ws(C_STAGE, bytes));
    double* dvz = static_cast<double*>(c.ws(C_IN, bytes));
    double* dnz = static_cast<double*>(c.ws(C_OUT, bytes));
    const double* dv_dev = dv_r;
    if (!dev) {
        PDEP_REQUIRE(all_finite(dv_r, (size_t)n_pert * ng), PDEP_EINVAL, "dv contains NaN or Inf");
        PDEP_HIP(hipMemcpyAsync(stage, dv_r, bytes, hipMemcpyHostToDevice, s));
        dv_dev = stage;
    }
    pdep::launch_transpose_grid(b.n[0], b.n[1], b.n[2], n_pert, dv_dev, dvz, true, s);
    pdep::ApplyStats as;
    pdep::chi0_grid(c, n_pert, dvz, dnz, as);
    if (dev) {
        pdep::launch_transpose_grid(b.n[0], b.n[1], b.n[2], n_pert, dnz, dn_r, false, s);
    } else {
        pdep::launch_transpose_grid(b.n[0], b.n[1], b.n[2], n_pert, dnz, stage, false, s);
        PDEP_HIP(hipMemcpyAsync(dn_r, stage, bytes, hipMemcpyDeviceToHost, s));
    }
    const double ms = tm.stop();
    fill_apply_stats(c, as, ms, st);
    if (as.n_notconv > 0)
        return fail(PDEP_ENOTCONV, std::to_string(as.n_notconv) + " Sternheimer systems missed cg_tol");
    API_END
}

int chibar_apply(pdep_ctx* ctx, int n_pert, const double* phi, double* out, double tol, int maxit,
                 pdep_chibar_stats* st) {
    API_BEGIN
    check_ctx(ctx);
    Ctx& c = ctx->c;
    PDEP_REQUIRE(n_pert >= 0, PDEP_EINVAL, "n_pert must be >= 0");
    PDEP_REQUIRE(tol > 0 && tol < 1 && maxit >= 1, PDEP_EINVAL, "bad self-consistency tolerance / cap");
    if (st) std::memset(st, 0, sizeof(*st));
    if (n_pert == 0) { g_err.clear(); return PDEP_OK; }
    PDEP_REQUIRE(phi && out, PDEP_EINVAL, "null phi/out");
    const int npw = c.basis.npw, n1 = npw - 1, g0 = c.basis.g0;
    const long ld = pdep::sphere_ld(npw);
    const bool dev = (c.opts.flags & PDEP_DEVICE_PTRS) != 0;
    hipStream_t s = c.stream;
    Timer tm(s);
    double2* in_s = static_cast<double2*>(c.ws(C_IN, (size_t)n_pert * ld * sizeof(double2)));
    double2* out_s = static_cast<double2*>(c.ws(C_OUT, (size_t)n_pert * ld * sizeof(double2)));
    if (dev) {
        pdep::launch_expand_s1(n_pert, npw, g0, reinterpret_cast<const double2*>(phi), n1, in_s, ld, s);
    } else {
        PDEP_REQUIRE(all_finite(phi, (size_t)2 * n_pert * n1), PDEP_EINVAL, "phi contains NaN or Inf");
        double2* stage = static_cast<double2*>(c.ws(C_STAGE, (size_t)n_pert * n1 * sizeof(double2)));
        PDEP_HIP(hipMemcpyAsync(stage, phi, (size_t)n_pert * n1 * sizeof(double2), hipMemcpyHostToDevice, s));
        pdep::launch_expand_s1(n_pert, npw, g0, stage, n1, in_s, ld, s);
    }
    pdep::ApplyStats as;
    const pdep::ScreenResult r = pdep::chibar_sphere(c, n_pert, in_s, out_s, tol, maxit, as);
    if (dev) {
        pdep::launch_compact_s1(n_pert, npw, g0, out_s, ld, reinterpret_cast<double2*>(out), n1, s);
    } else {
        double2* stage = static_cast<double2*>(c.ws(C_STAGE, (size_t)n_pert * n1 * sizeof(double2)));
        pdep::launch_compact_s1(n_pert, npw, g0, out_s, ld, stage, n1, s);
        PDEP_HIP(hipMemcpyAsync(out, stage, (size_t)n_pert * n1 * sizeof(double2), hipMemcpyDeviceToHost, s));
    }
    const double ms = tm.stop();
    if (st) {
        st->passes = r.passes;
        st->chi0_columns = r.chi0_columns;
        st->n_notconv = r.n_notconv;
        st->max_rel_residual = r.max_rel_residual;
        st->cg_iter_total = as.cg_iter_total;
        st->cg_notconv = as.n_notconv;
        st->ms = ms;
    }
    if (r.n_notconv > 0)
        return fail(PDEP_ENOTCONV, std::to_string(r.n_notconv) + " columns missed the self-consistency tolerance");
    if (as.n_notconv > 0)
        return fail(PDEP_ENOTCONV, std::to_string(as.n_notconv) + " Sternheimer systems missed cg_tol");
    API_END
}

int pdep_body_lanczos(pdep_ctx* ctx, int n_pert, const double* phi, int n_lanczos, int n_freq, const double* freq,
                      double* body, pdep_lanczos_stats* st) {
    API_BEGIN
    check_ctx(ctx);
    Ctx& c = ctx->c;
    if (st) std::memset(st, 0, sizeof(*st));
    PDEP_REQUIRE(n_pert >= 1 && n_lanczos >= 1 && n_freq >= 1, PDEP_EINVAL, "n_pert, n_lanczos and n_freq must be >= 1");
    PDEP_REQUIRE(phi && freq && body, PDEP_EINVAL, "null phi/freq/body");
    for (int f = 0; f < n_freq; ++f)
        PDEP_REQUIRE(std::isfinite(freq[f]) && freq[f] >= 0.0, PDEP_EINVAL, "frequencies must be finite and >= 0");
    PDEP_REQUIRE((long)n_pert * c.nv <= 65535L * 64, PDEP_EINVAL, "too many chains for one block");
    const int npw = c.basis.npw, n1 = npw - 1, g0 = c.basis.g0;
    const long ld = pdep::sphere_ld(npw);
    const bool dev = (c.opts.flags & PDEP_DEVICE_PTRS) != 0;
    hipStream_t s = c.stream;
    Timer tm(s);
    double2* in_s = static_cast<double2*>(c.ws(C_IN, (size_t)n_pert * ld * sizeof(double2)));
    if (dev) {
        pdep::launch_expand_s1(n_pert, npw, g0, reinterpret_cast<const double2*>(phi), n1, in_s, ld, s);
    } else {
        PDEP_REQUIRE(all_finite(phi, (size_t)2 * n_pert * n1), PDEP_EINVAL, "phi contains NaN or Inf");
        double2* stage = static_cast<double2*>(c.ws(C_STAGE, (size_t)n_pert * n1 * sizeof(double2)));
        PDEP_HIP(hipMemcpyAsync(stage, phi, (size_t)n_pert * n1 * sizeof(double2), hipMemcpyHostToDevice, s));
        pdep::launch_expand_s1(n_pert, npw, g0, stage, n1, in_s, ld, s);
    }
    const pdep::LanczosResult r = pdep::body_lanczos(c, n_pert, in_s, 0, n_lanczos, n_freq, freq, body);
    const double ms = tm.stop();
    if (st) {
        st->chains = r.chains;
        st->max_length = r.max_length;
        st->h_applications = r.h_applications;
        st->ms = ms;
    }
    API_END
}

int pdep_head_wings(pdep_ctx* ctx, int n_pert, const double* phi, int n_lanczos, int n_freq, const double* freq,
                    double* F, double* U, double* B, double* Lambda, double* Xi, pdep_lanczos_stats* st) {
    API_BEGIN
    check_ctx(ctx);
    Ctx& c = ctx->c;
    if (st) std::memset(st, 0, sizeof(*st));
    PDEP_REQUIRE(n_pert >= 1 && n_lanczos >= 1 && n_freq >= 1, PDEP_EINVAL, "n_pert, n_lanczos and n_freq must be >= 1");
    PDEP_REQUIRE(phi && freq, PDEP_EINVAL, "null phi/freq");
    for (int f = 0; f < n_freq; ++f)
        PDEP_REQUIRE(std::isfinite(freq[f]) && freq[f] >= 0.0, PDEP_EINVAL, "frequencies must be finite and >= 0");
    PDEP_REQUIRE((long)(n_pert + 3) * c.nv <= 65535L * 64, PDEP_EINVAL, "too many chains for one block");
    const int npw = c.basis.npw, n1 = npw - 1, g0 = c.basis.g0;
    const long ld = pdep::sphere_ld(npw);
    const bool dev = (c.opts.flags & PDEP_DEVICE_PTRS) != 0;
    hipStream_t s = c.stream;
    Timer tm(s);
    double2* in_s = static_cast<double2*>(c.ws(C_IN, (size_t)n_pert * ld * sizeof(double2)));
    if (dev) {
        pdep::launch_expand_s1(n_pert, npw, g0, reinterpret_cast<const double2*>(phi), n1, in_s, ld, s);
    } else {
        PDEP_REQUIRE(all_finite(phi, (size_t)2 * n_pert * n1), PDEP_EINVAL, "phi contains NaN or Inf");
        double2* stage = static_cast<double2*>(c.ws(C_STAGE, (size_t)n_pert * n1 * sizeof(double2)));
        PDEP_HIP(hipMemcpyAsync(stage, phi, (size_t)n_pert * n1 * sizeof(double2), hipMemcpyHostToDevice, s));
        pdep::launch_expand_s1(n_pert, npw, g0, stage, n1, in_s, ld, s);
    }
    const size_t nb = (size_t)n_pert + 3, np = (size_t)n_pert;
    std::vector<double> E((size_t)n_freq * nb * nb);
    pdep::ApplyStats ds;
    const pdep::LanczosResult r = pdep::body_lanczos(c, n_pert, in_s, 3, n_lanczos, n_freq, freq, E.data(), &ds);
    for (int f = 0; f < n_freq; ++f)
        pdep::bfinal(n_pert, E.data() + (size_t)f * nb * nb, c.basis.L, F ? F + 9 * (size_t)f : nullptr,
                     U ? U + 3 * np * f : nullptr, B ? B + np * np * f : nullptr, Lambda ? Lambda + np * np * f : nullptr,
                     Xi ? Xi + f : nullptr);
    const double ms = tm.stop();
    if (st) {
        st->chains = r.chains;
        st->max_length = r.max_length;
        st->h_applications = r.h_applications;
        st->ms = ms;
    }
    if (ds.n_notconv > 0)
        return fail(PDEP_ENOTCONV, std::to_string(ds.n_notconv) + " dipole-vector solves missed cg_tol");
    API_END
}

int pdep_qp_energies(pdep_ctx* ctx, int n_pdep, const double* phi, int n_states, const int* states,
                     const double* vxc, const pdep_qp_opts* opts, pdep_qp_result* out, int n_e,
                     const double* energies, double* sigma_c_e, pdep_qp_stats* st) {
    API_BEGIN
    check_ctx(ctx);
    Ctx& c = ctx->c;
    if (st) std::memset(st, 0, sizeof(*st));
    const int npw = c.basis.npw, n1 = npw - 1, g0 = c.basis.g0;
    PDEP_REQUIRE(phi && states && out, PDEP_EINVAL, "null phi/states/out");
    PDEP_REQUIRE(n_pdep >= 1 && n_pdep < n1, PDEP_EINVAL, "n_pdep out of range");
    PDEP_REQUIRE(n_states >= 1 && n_states <= 64, PDEP_EINVAL, "n_states must be 1 .. 64");
    for (int k = 0; k < n_states; ++k)
        PDEP_REQUIRE(states[k] >= 0 && states[k] < c.nv, PDEP_EINVAL, "states must be occupied band indices");
    PDEP_REQUIRE(n_e >= 0 && (n_e == 0 || (energies && sigma_c_e)), PDEP_EINVAL,
                 "energies and sigma_c_e are needed for n_e > 0");
    pdep_qp_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (o.n_lanczos == 0) o.n_lanczos = 40;
    if (o.n_freq == 0) o.n_freq = 64;
    if (o.omega0 == 0.0) o.omega0 = 0.5;
    if (o.eta == 0.0) o.eta = 1e-3;
    if (o.secant_tol == 0.0) o.secant_tol = 1e-8;
    if (o.secant_maxit == 0) o.secant_maxit = 40;
    if (o.dE == 0.0) o.dE = 1e-3;
    PDEP_REQUIRE(o.n_lanczos >= 1 && o.n_freq >= 1 && o.n_freq <= 4096 && o.omega0 > 0.0 && o.eta > 0.0 &&
                     o.secant_tol > 0.0 && o.secant_maxit >= 1 && o.dE > 0.0 && std::isfinite(o.e_fermi),
                 PDEP_EINVAL, "bad qp options");
    if (o.e_fermi == 0.0) {
        PDEP_REQUIRE(c.gap > 0.0, PDEP_EINVAL,
                     "e_fermi is required: the gap is unknown for orbitals given by the caller");
        o.e_fermi = c.eps[c.nv - 1] + 0.5 * c.gap;
    }
    PDEP_REQUIRE(o.e_fermi > c.eps[c.nv - 1], PDEP_EINVAL, "e_fermi must lie above the highest occupied energy");
    if (vxc)
        for (int k = 0; k < n_states; ++k) PDEP_REQUIRE(std::isfinite(vxc[k]), PDEP_EINVAL, "vxc is not finite");
    for (int k = 0; k < n_states * n_e; ++k)
        PDEP_REQUIRE(std::isfinite(energies[k]), PDEP_EINVAL, "energies are not finite");
    PDEP_REQUIRE((long)(n_pdep + 3) * c.nv <= 65535L * 64, PDEP_EINVAL, "too many chains for one block");
    const long ld = pdep::sphere_ld(npw);
    const bool dev = (c.opts.flags & PDEP_DEVICE_PTRS) != 0;
    hipStream_t s = c.stream;
    Timer tm(s);
    double2* in_s = static_cast<double2*>(c.ws(C_IN, (size_t)n_pdep * ld * sizeof(double2)));
    if (dev) {
        pdep::launch_expand_s1(n_pdep, npw, g0, reinterpret_cast<const double2*>(phi), n1, in_s, ld, s);
    } else {
        PDEP_REQUIRE(all_finite(phi, (size_t)2 * n_pdep * n1), PDEP_EINVAL, "phi contains NaN or Inf");
        double2* stage = static_cast<double2*>(c.ws(C_STAGE, (size_t)n_pdep * n1 * sizeof(double2)));
        PDEP_HIP(hipMemcpyAsync(stage, phi, (size_t)n_pdep * n1 * sizeof(double2), hipMemcpyHostToDevice, s));
        pdep::launch_expand_s1(n_pdep, npw, g0, stage, n1, in_s, ld, s);
    }
    pdep::ApplyStats ds;
    const pdep::QpStats q =
        pdep::qp_energies(c, n_pdep, in_s, n_states, states, vxc, o, out, n_e, energies, sigma_c_e, &ds);
    const double ms = tm.stop();
    int notconv = 0;
    for (int k = 0; k < n_states; ++k) notconv += out[k].converged ? 0 : 1;
    if (st) {
        st->chains = q.chains;
        st->max_length = q.max_length;
        st->h_applications = q.h_applications;
        st->secant_iterations = q.secant_iterations;
        st->residue_points = q.residue_points;
        st->ms = ms;
    }
    if (ds.n_notconv > 0)
        return fail(PDEP_ENOTCONV, std::to_string(ds.n_notconv) + " dipole-vector solves missed cg_tol");
    if (notconv > 0)
        return fail(PDEP_ENOTCONV, std::to_string(notconv) + " quasiparticle equations did not converge");
    API_END
}

int pdep_eigs(pdep_ctx* ctx, int n_pdep, uint64_t seed, const double* phi0, const pdep_eig_opts* eo_in,
              double* eps_out, double* basis_out, pdep_eig_stats* st) {
    API_BEGIN
    check_ctx(ctx);
    Ctx& c = ctx->c;
    PDEP_REQUIRE(eps_out != nullptr, PDEP_EINVAL, "null eps_out");
    const int npw = c.basis.npw, n1 = npw - 1, g0 = c.basis.g0;
    PDEP_REQUIRE(n_pdep >= 1 && n_pdep < n1, PDEP_EINVAL, "n_pdep out of range");
    pdep_eig_opts eo;
    std::memset(&eo, 0, sizeof(eo));
    eo.tol = 1e-9;
    eo.maxit = 60;
    if (eo_in) eo = *eo_in;
    PDEP_REQUIRE(eo.tol > 0 && eo.maxit >= 1 && eo.n_buffer >= 0 && eo.scr_tol >= 0 && eo.scr_maxit >= 0 &&
                     (eo.reducible == 0 || eo.reducible == 1),
                 PDEP_EINVAL, "bad eig options");
    if (st) std::memset(st, 0, sizeof(*st));
    const long ld = pdep::sphere_ld(npw);
    const bool dev = (c.opts.flags & PDEP_DEVICE_PTRS) != 0;
    hipStream_t s = c.stream;
    Timer tm(s);
    // C_IN / C_OUT are used by chi0 inside the Davidson loop: keep own buffers here
    pdep::Buf phi0_s, basis_s, stage;
    if (phi0) {
        phi0_s.ensure(&c.al, (size_t)n_pdep * ld * sizeof(double2));
        if (dev) {
            pdep::launch_expand_s1(n_pdep, npw, g0, reinterpret_cast<const double2*>(phi0), n1, phi0_s.as<double2>(),
                                   ld, s);
        } else {
            PDEP_REQUIRE(all_finite(phi0, (size_t)2 * n_pdep * n1), PDEP_EINVAL, "phi0 contains NaN or Inf");
            stage.ensure(&c.al, (size_t)n_pdep * n1 * sizeof(double2));
            PDEP_HIP(hipMemcpyAsync(stage.get(), phi0, (size_t)n_pdep * n1 * sizeof(double2), hipMemcpyHostToDevice, s));
            pdep::launch_expand_s1(n_pdep, npw, g0, stage.as<double2>(), n1, phi0_s.as<double2>(), ld, s);
        }
    }
    if (basis_out) basis_s.ensure(&c.al, (size_t)n_pdep * ld * sizeof(double2));
    std::vector<double> lam(n_pdep);
    pdep::EigResult r = pdep::pdep_davidson(c, n_pdep, seed, phi0 ? phi0_s.as<double2>() : nullptr, eo, lam.data(),
                                            basis_out ? basis_s.as<double2>() : nullptr);
    // chi0bar: eps = 1 - lambda; chibar: eps^-1 = 1 + mu
    for (int i = 0; i < n_pdep; ++i) eps_out[i] = eo.reducible ? 1.0 / (1.0 + lam[i]) : 1.0 - lam[i];
    if (basis_out) {
        if (dev) {
            pdep::launch_compact_s1(n_pdep, npw, g0, basis_s.as<double2>(), ld, reinterpret_cast<double2*>(basis_out),
                                    n1, s);
        } else {
            stage.ensure(&c.al, (size_t)n_pdep * n1 * sizeof(double2));
            pdep::launch_compact_s1(n_pdep, npw, g0, basis_s.as<double2>(), ld, stage.as<double2>(), n1, s);
            PDEP_HIP(hipMemcpyAsync(basis_out, stage.get(), (size_t)n_pdep * n1 * sizeof(double2),
                                    hipMemcpyDeviceToHost, s));
        }
    }
    const double ms = tm.stop();
    if (st) {
        st->iterations = r.iterations;
        st->chi0_columns = r.columns;
        st->max_residual = r.max_residual;
        st->cg_iter_total = r.cg_iter_total;
        st->ms = ms;
        st->n_notconv = r.n_notconv + r.scr_notconv;
        st->scr_passes = r.scr_passes;
    }
    if (!r.converged) return fail(PDEP_ENOTCONV, "PDEP Davidson did not reach tol");
    if (r.n_notconv > 0)
        return fail(PDEP_ENOTCONV, std::to_string(r.n_notconv) +
                                       " Sternheimer systems of the chi0bar applications missed cg_tol");
    if (r.scr_notconv > 0)
        return fail(PDEP_ENOTCONV, std::to_string(r.scr_notconv) +
                                       " chibar applications missed the self-consistency tolerance");
    API_END
}

int pdep_destroy(pdep_ctx* ctx) {
    API_BEGIN
    if (!ctx) { g_err.clear(); return PDEP_OK; }
    (void)hipStreamSynchronize(ctx->c.stream);
    delete ctx;
    API_END
}

}  // extern "C"
