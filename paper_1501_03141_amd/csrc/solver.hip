// Batched Sternheimer solves and the chi0 chain on the device.
//
// For a block of real potentials dV_i(r) and every occupied band v (one "row" per
// pair (i, v), row = i * N_v + v):
//   b_iv  = -P_c Fwd(dV_i u_v)                               (right-hand side, FP64)
//   solve   P_c (H - e_v) P_c dc_iv = b_iv  on range(P_c)    (Sec. 2.3, Eq. stern)
//   dn_i  = (4/Omega) Re sum_v conj(u_v) Inv(dc_iv)           (Eq. deltani, Gamma, 2 spins)
//   out_i = sqrt(4 pi)/|G| Fwd(dn_i) on S'                    (Eq. chiisamatrixinpdep)
//
// The solve is a preconditioned conjugate gradient (the paper's suggestion after
// Eq. stern) batched over all rows of a tile, wrapped in an FP64 iterative refinement:
//   x = 0, r = b;  repeat:  d ~ A^-1 r by CG in precision T (FP64 or FP32),
//                           x += d,  r = b - A x in FP64,
// until ||r|| <= cg_tol ||b|| per row.  In FP64 mode the inner CG already aims at the
// final tolerance, so one step normally suffices and the second FP64 residual only
// confirms it.  In mixed mode the inner FP32 CG reduces the residual by inner_tol per
// step.  Converged rows drop out of later steps (the row list is compacted on the host).
//
// Inner CG (rows independent, per-row scalars in FP64):
//   r = b, z = P_c K r, p = z
//   q = A p;  alpha = <r,z>/<p,q>;  x += alpha p;  r -= alpha q;  z = P_c K r;
//   beta = <r,z>_new/<r,z>;  p = z + beta p;  stop when ||r||^2 <= thr2
// with A = P_c (H - e_v) applied as stick pass -> slab pass (V_loc) -> stick pass with
// the kinetic/shift epilogue -> P_c GEMM pair, and K the diagonal kinetic preconditioner
// 1/max(1/2|G|^2 - e_v, kPrecondFloor) with a floor of 0.1 Ha (the paper does not fix K;
// it only changes iteration counts).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <string>
#include <unistd.h>
#include <utility>
#include <vector>
#include "pdep_internal.h"

namespace pdep {

namespace {

enum Slot {
    W_B64 = 0, W_X64, W_R64, W_XA, W_QA, W_RHS, W_CX, W_CR, W_CZ, W_CP, W_CQ, W_STICKS, W_S, W_SCAL,
    W_ROWS, W_VR, W_DN, W_REF2, W_XOUT, W_MAP, W_SPLIT, W_PQP, W_LAST
};
static_assert(W_LAST <= WS_SOLVER_END, "solver work-space slots overlap the others");

template <typename T> const cplx<T>* psi_of(Ctx& c);
template <> const double2* psi_of<double>(Ctx& c) { return c.psi64.as<double2>(); }
template <> const float2* psi_of<float>(Ctx& c) { return c.psi32.as<float2>(); }
// row strides of the two copies of Psi
template <typename T> long psi_ld(Ctx& c) { return sizeof(T) == sizeof(float) ? sphere_ld(c.basis.npw) : c.basis.npw; }
template <typename T> const T* vloc_of(Ctx& c);
template <> const double* vloc_of<double>(Ctx& c) { return c.vloc64.as<double>(); }
template <> const float* vloc_of<float>(Ctx& c) { return c.vloc32.as<float>(); }
template <typename T> const T* kin_of(Ctx& c);
template <> const double* kin_of<double>(Ctx& c) { return c.basis.d_kin64.as<double>(); }
template <> const float* kin_of<float>(Ctx& c) { return c.basis.d_kin32.as<float>(); }

// bytes of one row of the sticks buffer (sized for FP64, also used for FP32)
size_t sticks_row_bytes(const Ctx& c) {
    const FftDims& d = c.basis.dims;
    return (size_t)d.nz * d.sld * sizeof(double2);
}

}  // namespace

long sphere_ld(int npw) { return ((long)npw + 63) / 64 * 64; }
int half_len(int npw) { return (npw + 1) / 2; }

// Row stride of the projection coefficients S[row][band] (16-byte aligned FP32 rows)
// and the work space for nrows rows (either precision).
long coef_ld(int nv) { return ((long)nv + 3) / 4 * 4; }
size_t coef_bytes(int nv, int nrows) { return (size_t)nrows * coef_ld(nv) * sizeof(double2); }

// Y <- P_c Y = Y - Psi (Psi^H Y) for nrows half-sphere rows (entries k <= c of vectors
// real in r, the centre last).  With Psi real in r as well, Psi^H Y is real and equals
// Re sum_{k <= c} w_k conj(Psi_k) Y_k with w = 2 off the centre (the weights sit in the
// copies psi32w / psi64w), and the update touches the half sphere only.  S: work space
// of coef_bytes(nv, nrows).  In the BF16x3 mode the FP32 pair runs on the bf16 matrix
// cores (three products, real coefficients).
// Rows from which a first application tunes launch shapes by timing them on its data.
constexpr int kTuneRows = 1024;

namespace {

// Device time (ms) of f() on stream s: run twice, the second run timed.
template <class F> float time_twice(hipStream_t s, F&& f) {
    hipEvent_t e0, e1;
    PDEP_HIP(hipEventCreate(&e0));
    PDEP_HIP(hipEventCreate(&e1));
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {
        PDEP_HIP(hipEventRecord(e0, s));
        f();
        PDEP_HIP(hipEventRecord(e1, s));
        PDEP_HIP(hipEventSynchronize(e1));
        PDEP_HIP(hipEventElapsedTime(&ms, e0, e1));
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
}

std::string tune_key(const Ctx& c) {
    const char* prec = c.opts.precision == PDEP_FP64 ? "fp64" : (c.opts.precision == PDEP_MIXED_FP32 ? "fp32" : "bf16x3");
    return std::to_string(c.basis.n[0]) + "x" + std::to_string(c.basis.n[1]) + "x" + std::to_string(c.basis.n[2]) +
           " npw " + std::to_string(c.basis.npw) + " nv " + std::to_string(c.nv) + " " + prec;
}

// The cache file: one line per problem, {"<key>": {"<name>": <int>, ...}}, inside one
// JSON object.
using TuneMap = std::map<std::string, std::map<std::string, long>>;
std::mutex g_tune_mu;

TuneMap tune_read(const char* path) {
    TuneMap m;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t a = line.find('"');
        if (a == std::string::npos) continue;
        const size_t b = line.find('"', a + 1);
        const size_t brace = line.find('{', b == std::string::npos ? 0 : b);
        if (b == std::string::npos || brace == std::string::npos) continue;
        auto& entry = m[line.substr(a + 1, b - a - 1)];
        size_t q = brace;
        while ((q = line.find('"', q + 1)) != std::string::npos) {
            const size_t q2 = line.find('"', q + 1);
            const size_t colon = q2 == std::string::npos ? q2 : line.find(':', q2);
            if (colon == std::string::npos) break;
            entry[line.substr(q + 1, q2 - q - 1)] = std::strtol(line.c_str() + colon + 1, nullptr, 10);
            q = line.find_first_of(",}", colon);
            if (q == std::string::npos || line[q] == '}') break;
        }
    }
    return m;
}

}  // namespace

void tune_cache_load(Ctx& c) {
    const char* path = std::getenv("PDEP_TUNE_CACHE");
    if (!path || !*path) return;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const TuneMap m = tune_read(path);
    const auto it = m.find(tune_key(c));
    if (it == m.end()) return;
    auto get = [&](const char* k) {
        const auto f = it->second.find(k);
        return f == it->second.end() ? 0 : (int)f->second;
    };
    c.fft_chunk32 = get("chain_rows_fp32");
    c.fft_chunk64 = get("chain_rows_fp64");
    c.step_shape.splitk_target = get("step_splitk_target");
    c.ahb_shape.splitk_target = get("coef_splitk_target");
    c.ahb_shape.col_tiles = get("coef_col_tiles");
    if (verbose()) fprintf(stderr, "[pdep] tuned shapes of %s read from %s\n", tune_key(c).c_str(), path);
}

void tune_cache_store(const Ctx& c) {
    const char* path = std::getenv("PDEP_TUNE_CACHE");
    if (!path || !*path) return;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    TuneMap m = tune_read(path);
    auto& e = m[tune_key(c)];
    auto put = [&](const char* k, int v) {
        if (v > 0) e[k] = v;
    };
    put("chain_rows_fp32", c.fft_chunk32);
    put("chain_rows_fp64", c.fft_chunk64);
    put("step_splitk_target", c.step_shape.splitk_target);
    put("coef_splitk_target", c.ahb_shape.splitk_target);
    put("coef_col_tiles", c.ahb_shape.col_tiles);
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    {
        std::ofstream f(tmp);
        f << "{\n";
        size_t i = 0;
        for (const auto& kv : m) {
            f << "  \"" << kv.first << "\": {";
            size_t j = 0;
            for (const auto& nv : kv.second) f << (j++ ? ", " : "") << "\"" << nv.first << "\": " << nv.second;
            f << "}" << (++i < m.size() ? "," : "") << "\n";
        }
        f << "}\n";
    }
    if (std::rename(tmp.c_str(), path) != 0) std::remove(tmp.c_str());
}

template <typename T>
void project_c(Ctx& c, cplx<T>* Y, long ld, int nrows, double2* S) {
    const int npw = c.basis.npw, nv = c.nv, nh = half_len(npw);
    const long lds = coef_ld(nv);
    cplx<T>* St = reinterpret_cast<cplx<T>*>(S);
    const size_t split_elems = c.split_elems;    // split-K partial products (complex elements)
    cplx<T>* work = static_cast<cplx<T>*>(c.ws(W_SPLIT, split_elems * sizeof(cplx<T>)));
    if constexpr (sizeof(T) == sizeof(double)) {
        // Real coefficients over half spheres.  S = Re(Psi_w^H Y) by the split-K MFMA GEMM
        // (real parts written as complex with zero imaginary parts); with the rows read as
        // real vectors of 2 nh doubles, Y -= S Psi is a real GEMM on the FP64 matrix cores.
        if (nrows <= 0) return;
        launch_gemm_ahb<T>(nv, nrows, nh, c.psi64w.as<double2>(), npw, Y, ld, St, lds, work, split_elems, c.stream,
                           true);
        // (the split-K buffer is free once the coefficient GEMM is done)
        launch_dgemm_sub(nv, nrows, nh, c.psi64.as<double2>(), npw, St, lds, Y, ld, reinterpret_cast<double*>(work),
                         2 * split_elems, c.stream);
    } else {
        const long lp = sphere_ld(npw);
        const float2* pw = c.psi32w.as<float2>();
        if (c.pc_x3) {
            float* Sr = reinterpret_cast<float*>(S);
            float* wr = reinterpret_cast<float*>(work);
            if (c.ahb_shape.splitk_target == 0 && nrows >= kTuneRows && !c.arena && !c.capturing) {
                // the coefficient GEMM only reads Y: time its launch shapes on the live rows
                float best = 0.f;
                for (const GemmShape g : {GemmShape{512, 8}, GemmShape{1024, 8}, GemmShape{256, 8}, GemmShape{512, 4},
                                          GemmShape{1024, 4}}) {
                    const float ms = time_twice(c.stream, [&] {
                        launch_gemm_ahb_x3_real(nv, nrows, nh, pw, lp, Y, ld, Sr, lds, wr, 2 * split_elems, c.stream,
                                                nullptr, nullptr, 0.0, g);
                    });
                    if (verbose())
                        fprintf(stderr, "[pdep] coefficient GEMM, %d rows, split-K target %d, %d column tiles: %.3f ms\n",
                                nrows, g.splitk_target, g.col_tiles, ms);
                    if (c.ahb_shape.splitk_target == 0 || ms < best) {
                        best = ms;
                        c.ahb_shape = g;
                    }
                }
                tune_cache_store(c);
            }
            launch_gemm_ahb_x3_real(nv, nrows, nh, pw, lp, Y, ld, Sr, lds, wr, 2 * split_elems, c.stream, nullptr,
                                    nullptr, 0.0, c.ahb_shape);
            launch_gemm_update_x3_real(nv, nrows, nh, psi_of<T>(c), lp, Sr, lds, -1.0, 1.0, Y, ld, c.stream);
        } else {
            launch_gemm_ahb<T>(nv, nrows, nh, pw, lp, Y, ld, St, lds, work, split_elems, c.stream, true);
            launch_gemm_update<T>(nv, nrows, nh, psi_of<T>(c), lp, St, lds, -1.0, 1.0, Y, ld, c.stream, true);
        }
    }
}

// Rows per launch of the transform chain (sticks pass, slab pass, sticks pass).  With
// blocks of rows whose sticks fit in the on-die cache, each pass reads what the previous
// one wrote from that cache instead of HBM.  The block size is chosen by timing: on the
// first application with at least kTuneRows rows, the chain runs for candidate sizes
// around the cache rule (and for all rows at once) on the actual data and the fastest
// is kept for the context (per precision).  Every row is independent, so the results do
// not depend on the choice.  PDEP_FFT_CHUNK=<fp32 rows>[:<fp64 rows>] in the environment
// fixes the sizes instead (for profiling runs that must launch the shapes of a tuned run).
constexpr double kChunkCacheBytes = 150e6;   // about half of the 256 MB last-level cache

int fft_chunk_env(bool fp64) {
    static const std::pair<int, int> v = [] {
        int a = 0, b = 0;
        if (const char* e = std::getenv("PDEP_FFT_CHUNK")) {
            a = std::atoi(e);
            const char* colon = std::strchr(e, ':');
            b = colon ? std::atoi(colon + 1) : 0;
        }
        return std::make_pair(std::max(a, 0), std::max(b, 0));
    }();
    return fp64 ? v.second : v.first;
}

template <typename T> int& fft_chunk_of(Ctx& c) { return sizeof(T) == sizeof(float) ? c.fft_chunk32 : c.fft_chunk64; }



template <typename T> int fft_chunk_rule(const Ctx& c) {
    const FftDims& d = c.basis.dims;
    // rows are paired: two rows per sticks row
    const double row = (double)d.nz * d.sld * sizeof(cplx<T>) / 2.0;
    return std::max(32, (int)(kChunkCacheBytes / row));
}

// Partial dot products per row written by the epilogue of apply_op<T> on half-sphere rows.
template <typename T> int op_dot_groups(const FftDims& d) { return sticks_to_sphere_pair_groups<T>(d); }

// q = [P_c] (H - shift) p: stick pass, slab pass with V_loc, stick pass with the
// kinetic/shift epilogue, then (optionally) the P_c GEMM pair.  pq_part (may be null,
// only without the projection): per-row partial sums of Re<p, q> from the epilogue,
// op_dot_groups of them per row.  half: the rows are half spheres of vectors real in r,
// transformed two rows per complex transform (the block size of the chain is tuned);
// otherwise full spheres, one transform per row, all rows in one block.
template <typename T>
void apply_op(Ctx& c, const cplx<T>* p, cplx<T>* q, long ld, int nrows, const double* shift, int nshift,
              bool project, bool half, void* sticks_buf, double2* S, double* pq_part = nullptr) {
    const Basis& b = c.basis;
    PDEP_REQUIRE(!(project && pq_part), PDEP_EINVAL, "apply_op: partial dots are of the unprojected q");
    PDEP_REQUIRE(half || !(project || pq_part), PDEP_EINVAL, "apply_op: projection and dots need half-sphere rows");
    cplx<T>* sk = static_cast<cplx<T>*>(sticks_buf);
    const bool paired = half;
    const int npq = op_dot_groups<T>(b.dims);
    auto chain = [&](int chunk) {
        if (paired) chunk += chunk & 1;   // pairs never straddle two blocks
        for (int r0 = 0; r0 < nrows; r0 += chunk) {
            const int nr = std::min(chunk, nrows - r0);
            const cplx<T>* pc = p + (long)r0 * ld;
            const bool per_row = nshift == nrows;
            const double* shc = per_row ? shift + r0 : shift;
            const int nsh = per_row ? nr : nshift;
            double* pqc = pq_part ? pq_part + (long)r0 * npq : nullptr;
            if (paired) {
                launch_sphere_to_sticks_pair<T>(b.dims, b.tables, pc, ld, nr, sk, c.stream);
                launch_slab_hv<T>(b.dims, b.tables, sk, (nr + 1) / 2, vloc_of<T>(c), c.stream);
                launch_sticks_to_sphere_pair<T>(b.dims, b.tables, sk, nr, q + (long)r0 * ld, ld, EPI_SHIFTED_H, 0.0, pc,
                                                ld, kin_of<T>(c), shc, nsh, c.stream, pqc);
            } else {
                launch_sphere_to_sticks<T>(b.dims, b.tables, pc, ld, nr, nullptr, sk, c.stream);
                launch_slab_hv<T>(b.dims, b.tables, sk, nr, vloc_of<T>(c), c.stream);
                launch_sticks_to_sphere<T>(b.dims, b.tables, sk, nr, q + (long)r0 * ld, ld, EPI_SHIFTED_H, 0.0, pc, ld,
                                           kin_of<T>(c), shc, nsh, nullptr, c.stream, pqc);
            }
        }
    };
    if (!half) {
        chain(nrows);
        return;
    }
    int& tuned = fft_chunk_of<T>(c);
    if (tuned == 0) tuned = fft_chunk_env(sizeof(T) == sizeof(double));
    if (tuned == 0 && nrows >= kTuneRows && !c.arena) {   // timing needs events (no-allocation calls skip it)
        const int rule = fft_chunk_rule<T>(c);
        std::vector<int> cand;
        for (int v : {rule / 2, (3 * rule) / 4, rule, (3 * rule) / 2, 2 * rule, nrows}) {
            v = std::min(std::max(v, 32), nrows);
            if (std::find(cand.begin(), cand.end(), v) == cand.end()) cand.push_back(v);
        }
        hipEvent_t e0, e1;
        PDEP_HIP(hipEventCreate(&e0));
        PDEP_HIP(hipEventCreate(&e1));
        float best = 0.f;
        for (int v : cand) {
            float ms = 0.f;
            for (int rep = 0; rep < 2; ++rep) {   // the second run is timed
                PDEP_HIP(hipEventRecord(e0, c.stream));
                chain(v);
                PDEP_HIP(hipEventRecord(e1, c.stream));
                PDEP_HIP(hipEventSynchronize(e1));
                PDEP_HIP(hipEventElapsedTime(&ms, e0, e1));
            }
            if (verbose()) fprintf(stderr, "[pdep] transform chain, %d rows in blocks of %d: %.3f ms\n", nrows, v, ms);
            if (tuned == 0 || ms < best) {
                best = ms;
                tuned = v;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (verbose()) fprintf(stderr, "[pdep] transform chain block size %d rows\n", tuned), fflush(stderr);
        tune_cache_store(c);
    }
    chain(tuned > 0 ? tuned : nrows);
    if (project) project_c<T>(c, q, ld, nrows, S);
}

void apply_h64(Ctx& c, const double2* x, long ldx, int nrows, const double* shift, int nshift, double2* out,
               long ldo, double2* sticks_buf) {
    PDEP_REQUIRE(ldx == ldo, PDEP_EINVAL, "apply_h64: ld mismatch");
    apply_op<double>(c, x, out, ldx, nrows, shift, nshift, false, false, sticks_buf, nullptr);
}

namespace {

// Per-row inputs/outputs of the inner solver (original row order) and shared scratch.
struct CgScalars {
    double *rz_new, *pq, *rr, *thr2, *shift;   // thr2 / shift: inputs per original row
    int *active, *iters, *n_active;            // iters: output per original row
    // per-slot state of the compacted active set, two sets for ping-pong gathers
    double *s_rz[2], *s_shift[2], *s_thr2[2];
    int *s_iters[2], *s_id[2];
};

CgScalars cg_scalars(Ctx& c, int n) {
    const size_t nd = 5 * (size_t)n + 6 * (size_t)n, ni = 3 * (size_t)n + 4 * (size_t)n + 64;
    char* base = static_cast<char*>(c.ws(W_SCAL, nd * sizeof(double) + ni * sizeof(int)));
    CgScalars s;
    double* d = reinterpret_cast<double*>(base);
    s.rz_new = d; s.pq = d + n; s.rr = d + 2 * n; s.thr2 = d + 3 * n; s.shift = d + 4 * n;
    for (int k = 0; k < 2; ++k) {
        s.s_rz[k] = d + (5 + 3 * k) * (size_t)n;
        s.s_shift[k] = d + (6 + 3 * k) * (size_t)n;
        s.s_thr2[k] = d + (7 + 3 * k) * (size_t)n;
    }
    int* i = reinterpret_cast<int*>(base + nd * sizeof(double));
    s.active = i; s.iters = i + n; s.n_active = i + 2 * n;
    for (int k = 0; k < 2; ++k) {
        s.s_iters[k] = i + 2 * n + 64 + 2 * k * (size_t)n;
        s.s_id[k] = i + 2 * n + 64 + (2 * k + 1) * (size_t)n;
    }
    return s;
}

// Compaction kernels.  map[j] = old slot of new slot j.
// Compaction in place: live slot src[j] (at or beyond the new count) moves into the
// retired slot dst[j] (below it); the two sets are disjoint, so no slot is both read and
// written.
template <typename T>
__global__ void k_move_state(int K, long ld, const int* __restrict__ dst, const int* __restrict__ src,
                             cplx<T>* x, cplx<T>* r, cplx<T>* z, cplx<T>* p) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (k >= K) return;
    const long o = (long)src[j] * ld + k, n = (long)dst[j] * ld + k;
    if (x) x[n] = x[o];
    r[n] = r[o];
    if (z) z[n] = z[o];
    p[n] = p[o];
}

__global__ void k_move_slots(int nm, const int* __restrict__ dst, const int* __restrict__ src, double* rz,
                             double* sh, double* th, int* it, int* id, int* active) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nm) return;
    const int d = dst[j], o = src[j];
    rz[d] = rz[o];
    sh[d] = sh[o];
    th[d] = th[o];
    it[d] = it[o];
    id[d] = id[o];
    active[d] = 1;
}

// Retire slots: Xout[id[o]] = x[o], iters_out[id[o]] = iters[o] for o in list.
template <typename T>
__global__ void k_retire(int K, long ld, const int* __restrict__ list, const int* __restrict__ id,
                         const cplx<T>* __restrict__ x, cplx<T>* __restrict__ xout) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (k >= K) return;
    const int o = list[j];
    xout[(long)id[o] * ld + k] = x[(long)o * ld + k];
}

__global__ void k_retire_iters(int n, const int* __restrict__ list, const int* __restrict__ id,
                               const int* __restrict__ it, int* __restrict__ iters_out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int o = list[j];
    iters_out[id[o]] = it[o];
}

__global__ void k_iota_copy(int n, const double* __restrict__ sh, const double* __restrict__ th,
                            double* __restrict__ sh1, double* __restrict__ th1, int* __restrict__ id,
                            int* __restrict__ it) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    sh1[j] = sh[j];
    th1[j] = th[j];
    id[j] = j;
    it[j] = 0;
}

// Inner batched PCG in precision T on n rows: solves P_c (H - shift) x = b with x0 = 0.
// sc.shift / sc.thr2 (per row) must be filled by the caller.  The solution of row i is
// left in the W_XOUT buffer at row i and its iteration count in sc.iters[i].
// Rows that converge drop out: whenever fewer than 9/10 of the current slots are still
// active, converged slots retire their solution and the live CG state is gathered
// into a compact set of slots, so every kernel runs on active rows only.
template <typename T>
int cg_inner(Ctx& c, int n, const cplx<T>* b, long ld, CgScalars& sc, int maxit, ApplyStats& st) {
    // half-sphere rows (entries k <= c of vectors real in r)
    constexpr bool half = true;
    const int npw = half_len(c.basis.npw), nv = c.nv;
    // Graph mode runs the solve on the context's own capture stream (a stream that is not
    // the legacy default stream can be captured), ordered after the caller's stream by an
    // event at entry and before it at exit.
    const bool use_graph = (c.opts.flags & PDEP_CG_GRAPHS) != 0 && !c.arena;   // instantiation may allocate
    struct StreamSwitch {
        Ctx& c;
        hipStream_t orig = nullptr;
        bool on = false;
        StreamSwitch(Ctx& cc, bool enable) : c(cc) {
            if (!enable) return;
            if (!c.graph_stream) {
                PDEP_HIP(hipStreamCreateWithFlags(&c.graph_stream, hipStreamNonBlocking));
                PDEP_HIP(hipEventCreateWithFlags(&c.graph_event, hipEventDisableTiming));
            }
            orig = c.stream;
            PDEP_HIP(hipEventRecord(c.graph_event, orig));
            PDEP_HIP(hipStreamWaitEvent(c.graph_stream, c.graph_event, 0));
            c.stream = c.graph_stream;
            on = true;
        }
        ~StreamSwitch() {
            if (!on) return;
            (void)hipEventRecord(c.graph_event, c.graph_stream);
            (void)hipStreamWaitEvent(orig, c.graph_event, 0);
            c.stream = orig;
        }
    } stream_switch(c, use_graph);
    hipStream_t s = c.stream;
    const size_t vbytes = (size_t)n * ld * sizeof(cplx<T>);
    cplx<T>* x = static_cast<cplx<T>*>(c.ws(W_CX, vbytes));
    cplx<T>* r = static_cast<cplx<T>*>(c.ws(W_CR, vbytes));
    cplx<T>* z = static_cast<cplx<T>*>(c.ws(W_CZ, vbytes));
    cplx<T>* p = static_cast<cplx<T>*>(c.ws(W_CP, vbytes));
    cplx<T>* q = static_cast<cplx<T>*>(c.ws(W_CQ, vbytes));
    cplx<T>* xout = static_cast<cplx<T>*>(c.ws(W_XOUT, vbytes));
    int* dmap = static_cast<int*>(c.ws(W_MAP, (size_t)2 * n * sizeof(int) + 64));
    void* sticks = c.ws(W_STICKS, (size_t)n * sticks_row_bytes(c));
    double2* S = static_cast<double2*>(c.ws(W_S, coef_bytes(nv, n)));
    const int pre = c.opts.precond;
    // per-row partial sums: <p, q> (stick groups of the H epilogue), <r, K r> and ||r||^2
    // (blocks of the CG step)
    const int npq = op_dot_groups<T>(c.basis.dims), nblk = (npw + 255) / 256;
    double* pq_part = static_cast<double*>(c.ws(W_PQP, (size_t)n * (npq + 2 * nblk) * sizeof(double) + 64));
    double* rz_part = pq_part + (size_t)n * npq;
    double* rr_part = rz_part + (size_t)n * nblk;
    const T* kin = kin_of<T>(c);
    // BF16x3 with the preconditioner: fused direction update (no z pass)
    const bool fused = pre && sizeof(T) == sizeof(float) && c.pc_x3;
    // BF16x3 products: a row whose residual grows 100-fold (or is not a number) has
    // diverged and stops; the refinement solves it again with FP32 products
    const double rr_max = (sizeof(T) == sizeof(float) && c.pc_x3) ? 1e4 : 0.0;
    int ncur = n;

    hipLaunchKernelGGL(k_iota_copy, dim3((n + 255) / 256), dim3(256), 0, s, n, sc.shift, sc.thr2, sc.s_shift[0],
                       sc.s_thr2[0], sc.s_id[0], sc.s_iters[0]);
    PDEP_HIP(hipGetLastError());
    // fused path: x lives in xout at the caller's row (slot ids start as the identity)
    launch_cg_init<T>(n, npw, b, ld, fused ? xout : x, r, z, kin, sc.s_shift[0], n, pre, s);
    if (pre) project_c<T>(c, z, ld, n, S);
    PDEP_HIP(hipMemcpyAsync(p, z, vbytes, hipMemcpyDeviceToDevice, s));
    launch_row_dots<T>(n, npw, r, ld, z, ld, sc.s_rz[0], sc.rr, s, half);
    launch_fill_i32(sc.active, n, 1, s);
    launch_fill_zero(sc.n_active, sizeof(int), s);
    launch_cg_check(n, sc.rr, sc.s_thr2[0], sc.active, sc.s_iters[0], sc.s_rz[0], nullptr, sc.n_active, 0, s);
    int h_active = 0;
    PDEP_HIP(hipMemcpyAsync(&h_active, sc.n_active, sizeof(int), hipMemcpyDeviceToHost, s));
    PDEP_HIP(hipStreamSynchronize(s));
    std::vector<int> flags, keep, ret, mv;
    // retire the slots in `list` (host)
    auto retire = [&](const std::vector<int>& list) {
        if (list.empty()) return;
        const int nr = (int)list.size();
        PDEP_HIP(hipMemcpyAsync(dmap + n, list.data(), nr * sizeof(int), hipMemcpyHostToDevice, s));
        {
            ProfScope prof_(K_MISC, s, fused ? 0.0 : 2.0 * nr * npw * sizeof(cplx<T>));
            if (!fused)   // the fused path accumulates x in place (row s_id of xout)
                hipLaunchKernelGGL(k_retire<T>, dim3((npw + 255) / 256, nr), dim3(256), 0, s, npw, ld, dmap + n,
                                   sc.s_id[0], x, xout);
            hipLaunchKernelGGL(k_retire_iters, dim3((nr + 255) / 256), dim3(256), 0, s, nr, dmap + n, sc.s_id[0],
                               sc.s_iters[0], sc.iters);
        }
        PDEP_HIP(hipGetLastError());
    };
    int it = 0;
    // the host reads the active count every `poll` iterations (compaction, exit): 2 beats 4
    // on the medium block (fewer iterations on rows that have converged, 278 -> 272 ms)
    const int poll = 2;
    // graph mode: one executable graph per phase of the 8-iteration re-projection cycle,
    // for the current slot count (destroyed when compaction changes it, and at exit)
    int graph_ncur = -1;
    hipGraphExec_t graph_exec[8 / poll] = {};
    bool graph_valid[8 / poll] = {};
    struct GraphsGuard {
        hipGraphExec_t* e;
        int n;
        ~GraphsGuard() {
            for (int i = 0; i < n; ++i)
                if (e[i]) (void)hipGraphExecDestroy(e[i]);
        }
    } graphs_guard{graph_exec, 8 / poll};
    while (h_active > 0 && it < maxit) {
        if (h_active < ncur && (10 * h_active < 9 * ncur)) {
            // compact: retire converged slots, then fill the holes they leave below the new
            // count with the live slots above it (state is moved only for those)
            flags.resize(ncur);
            PDEP_HIP(hipMemcpyAsync(flags.data(), sc.active, ncur * sizeof(int), hipMemcpyDeviceToHost, s));
            PDEP_HIP(hipStreamSynchronize(s));
            keep.clear();
            ret.clear();
            for (int j = 0; j < ncur; ++j) (flags[j] ? keep : ret).push_back(j);
            retire(ret);
            // move the live slots at or beyond nk into the retired slots below it
            const int nk = (int)keep.size();
            mv.clear();
            for (int j : ret)
                if (j < nk) mv.push_back(j);
            const int nm = (int)mv.size();
            for (int j : keep)
                if (j >= nk) mv.push_back(j);
            if (nm > 0) {
                PDEP_HIP(hipMemcpyAsync(dmap, mv.data(), 2 * nm * sizeof(int), hipMemcpyHostToDevice, s));
                ProfScope prof_(K_MISC, s, ((fused ? 4.0 : 8.0) * nm) * npw * sizeof(cplx<T>));
                hipLaunchKernelGGL(k_move_state<T>, dim3((npw + 255) / 256, nm), dim3(256), 0, s, npw, ld, dmap,
                                   dmap + nm, fused ? nullptr : x, r, fused ? nullptr : z, p);
                hipLaunchKernelGGL(k_move_slots, dim3((nm + 255) / 256), dim3(256), 0, s, nm, dmap, dmap + nm,
                                   sc.s_rz[0], sc.s_shift[0], sc.s_thr2[0], sc.s_iters[0], sc.s_id[0], sc.active);
                PDEP_HIP(hipGetLastError());
            }
            PDEP_HIP(hipStreamSynchronize(s));   // keep / ret / mv host vectors are reused
            ncur = nk;
        }
        const int nstep = std::min(poll, maxit - it);
        double* rz = sc.s_rz[0];
        double* sh = sc.s_shift[0];
        // one CG iteration on the ncur live slots (reproject: r is projected again after
        // it; last: the final iteration of the block)
        auto iteration = [&](bool reproject, bool last) {

            // With the preconditioner z = P_c K r is projected every iteration, so p stays in
            // range(P_c) and q = (H - shift) p needs no projection: <p, q> and the update of
            // x are unchanged by it.  What q adds to r outside range(P_c) is rounding (the
            // orbitals are eigenvectors of H); it is removed from r once per group of
            // iterations, so it stays far below the inner tolerance.  The inner products
            // come from the kernels that produce their operands: <p, q> from the epilogue
            // of H (partial sums per stick group), <r, z> = <r, K r> (r in range(P_c)) and
            // ||r||^2 from the step that updates r.  Without the preconditioner z = r, q
            // is projected every time and the products are separate passes.
            if (pre && fused) {
                // z = P_c K r is never stored: the coefficient GEMM applies K to r on the
                // fly and the update GEMM writes p = K r - Psi S + beta p directly
                apply_op<T>(c, p, q, ld, ncur, sh, ncur, false, true, sticks, S, pq_part);
                st.op_applications++;
                // x += alpha p happens in the direction GEMM (which reads the old p anyway)
                float* beta = reinterpret_cast<float*>(sc.pq);   // sc.pq is not used on this path
                float* alpha = beta + n;
                if constexpr (sizeof(T) == sizeof(float)) {
                    float* Sr = reinterpret_cast<float*>(S);
                    float* wr = static_cast<float*>(c.ws(W_SPLIT, c.split_elems * sizeof(float2)));
                    const long lp = sphere_ld(c.basis.npw), lds = coef_ld(nv);
                    if (nv <= 128) {
                        // r -= alpha q and its inner products inside the coefficient GEMM
                        CgStepFuse cs;
                        cs.q = q;
                        cs.rz = rz;
                        cs.pq = pq_part;
                        cs.npq = npq;
                        cs.active = sc.active;
                        cs.alpha_out = alpha;
                        cs.rz_part = rz_part;
                        cs.rr_part = rr_part;
                        cs.rz_new = sc.rz_new;
                        cs.rr = sc.rr;
                        cs.beta = beta;
                        cs.count = sc.n_active;   // cleared here for the check below
                        auto step = [&](float2* rr_in, GemmShape g) {
                            launch_gemm_ahb_x3_step(nv, ncur, npw, c.psi32w.as<float2>(), lp, rr_in, ld, Sr, lds, wr,
                                                    2 * c.split_elems, s, kin, sh, kPrecondFloor, cs, nblk, g);
                        };
                        if (c.step_shape.splitk_target == 0 && ncur >= kTuneRows && !c.arena && !c.capturing) {
                            // time the split-K targets on a copy of r (z is not used in this mode);
                            // every other output of the trial runs is written again by the real step
                            PDEP_HIP(hipMemcpyAsync(z, r, (size_t)ncur * ld * sizeof(cplx<T>), hipMemcpyDeviceToDevice,
                                                    s));
                            float best = 0.f;
                            for (int t : {512, 1024, 2048}) {
                                const float ms = time_twice(s, [&] { step(z, GemmShape{t, 0}); });
                                if (verbose())
                                    fprintf(stderr, "[pdep] fused CG step, %d rows, split-K target %d: %.3f ms\n",
                                            ncur, t, ms);
                                if (c.step_shape.splitk_target == 0 || ms < best) {
                                    best = ms;
                                    c.step_shape.splitk_target = t;
                                }
                            }
                            tune_cache_store(c);
                        }
                        step(r, c.step_shape);
                    } else {
                        launch_cg_step1<T>(ncur, npw, nullptr, r, nullptr, p, q, ld, rz, pq_part, npq, sc.active,
                                           kin, sh, ncur, pre, s, rz_part, rr_part, sc.rz_new, sc.rr, half, beta,
                                           alpha);
                        launch_gemm_ahb_x3_real(nv, ncur, npw, c.psi32w.as<float2>(), lp, r, ld, Sr, lds, wr,
                                                2 * c.split_elems, s, kin, sh, kPrecondFloor);
                    }
                    launch_cg_direction_x3(nv, ncur, npw, psi_of<T>(c), lp, Sr, lds, r, ld, kin, sh, kPrecondFloor,
                                           beta, alpha, xout, sc.s_id[0], sc.active, p, ld, s);
                }
                // r is re-projected every 8 iterations
                if (reproject) project_c<T>(c, r, ld, ncur, S);
            } else if (pre) {
                apply_op<T>(c, p, q, ld, ncur, sh, ncur, false, true, sticks, S, pq_part);
                st.op_applications++;
                launch_cg_step1<T>(ncur, npw, x, r, z, p, q, ld, rz, pq_part, npq, sc.active, kin, sh, ncur, pre, s,
                                   rz_part, rr_part, sc.rz_new, sc.rr, half);
                project_c<T>(c, z, ld, ncur, S);
                if (last) project_c<T>(c, r, ld, ncur, S);
            } else {
                apply_op<T>(c, p, q, ld, ncur, sh, ncur, true, true, sticks, S);
                st.op_applications++;
                launch_row_dots<T>(ncur, npw, p, ld, q, ld, sc.pq, nullptr, s, half);
                launch_cg_step1<T>(ncur, npw, x, r, z, p, q, ld, rz, sc.pq, 1, sc.active, kin, sh, ncur, pre, s);
                launch_row_dots<T>(ncur, npw, r, ld, z, ld, sc.rz_new, sc.rr, s, half);
            }
            if (!(pre && fused)) launch_cg_step2<T>(ncur, npw, p, z, ld, sc.rz_new, rz, sc.active, s);
            if (!(pre && fused && nv <= 128)) launch_fill_zero(sc.n_active, sizeof(int), s);
            launch_cg_check(ncur, sc.rr, sc.s_thr2[0], sc.active, sc.s_iters[0], rz, sc.rz_new, sc.n_active, 1,
                            s, rr_max);
        };
        auto block = [&](int it0, int n) {
            for (int k = 0; k < n; ++k) iteration((it0 + k + 1) % 8 == 0, k == n - 1);
        };
        // The kernels of a block of `poll` iterations can be captured once per slot count
        // and replayed as a HIP graph (the host still reads the active count after each
        // block).  The first block of a solve runs eagerly: it sizes every work buffer and
        // tunes the transform chain, which must not happen under capture.  The graph holds
        // kernels only (the counter is cleared by a kernel, not a memset).
        const bool graph_ok = use_graph && nstep == poll && it > 0 && !profiling_on();
        if (graph_ok) {
            const int variant = (it % 8) / poll;   // which iteration of the 8 re-projects r
            if (graph_ncur != ncur) {
                for (auto& v : graph_valid) v = false;   // kept for an in-place update
                graph_ncur = ncur;
            }
            hipGraphExec_t& ex = graph_exec[variant];
            if (!graph_valid[variant]) {
                hipGraph_t g = nullptr;
                const long long ops = st.op_applications;   // counted at launch, not at capture
                PDEP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                try {
                    c.capturing = true;
                    block(it, nstep);
                    c.capturing = false;
                    st.op_applications = ops;
                } catch (...) {
                    c.capturing = false;
                    hipGraph_t dead = nullptr;
                    (void)hipStreamEndCapture(s, &dead);
                    if (dead) (void)hipGraphDestroy(dead);
                    throw;
                }
                PDEP_HIP(hipStreamEndCapture(s, &g));
                // a graph of the same shape (another row count) is updated in place; a new
                // shape (the chain's block count changed) is instantiated
                bool updated = false;
                if (ex) {
                    hipGraphNode_t bad = nullptr;
                    hipGraphExecUpdateResult why;
                    updated = hipGraphExecUpdate(ex, g, &bad, &why) == hipSuccess;
                    if (!updated) {
                        (void)hipGetLastError();
                        (void)hipGraphExecDestroy(ex);
                        ex = nullptr;
                    }
                }
                hipError_t e = hipSuccess;
                if (!updated) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                PDEP_HIP(e);
                graph_valid[variant] = true;
                ++st.graph_captures;
                if (updated) ++st.graph_updates;
            }
            PDEP_HIP(hipGraphLaunch(ex, s));
            ++st.graph_launches;
            st.op_applications += nstep;
        } else {
            block(it, nstep);
        }
        it += nstep;
        PDEP_HIP(hipMemcpyAsync(&h_active, sc.n_active, sizeof(int), hipMemcpyDeviceToHost, s));
        PDEP_HIP(hipStreamSynchronize(s));
    }
    // retire everything that is left (converged or at the iteration cap)
    std::vector<int> all(ncur);
    for (int j = 0; j < ncur; ++j) all[j] = j;
    retire(all);
    PDEP_HIP(hipStreamSynchronize(s));
    return it;
}

template <typename T> cplx<T>* cg_solution(Ctx& c) { return static_cast<cplx<T>*>(c.ws_current(W_XOUT)); }

}  // namespace

// Solve all n rows of b64 to opts.cg_tol; x64 receives dc (not yet re-projected).  The
// rows are half spheres (entries k <= c of vectors real in r, row stride ld).
// ref2 (may be null): per-row squared norm of the right-hand side before P_c.  A row
// whose projected norm is below 1e-13 of it carries only rounding noise (the
// perturbation acts inside the occupied space, e.g. a constant dV) and is solved as
// b = 0, x = 0.
void solve_rows(Ctx& c, int n, const double2* b64, double2* x64, long ld, ApplyStats& st,
                const double* ref2) {
    const int npw = half_len(c.basis.npw), nv = c.nv;
    hipStream_t s = c.stream;
    const double tol = c.opts.cg_tol;
    const bool mixed = c.opts.precision != PDEP_FP64;
    const size_t vb64 = (size_t)n * ld * sizeof(double2);
    double2* r64 = static_cast<double2*>(c.ws(W_R64, vb64));
    double2* xa = static_cast<double2*>(c.ws(W_XA, vb64));
    double2* qa = static_cast<double2*>(c.ws(W_QA, vb64));
    // packed host->device row data: rows (int), scale, invscale (double)
    char* rowbuf = static_cast<char*>(c.ws(W_ROWS, (size_t)n * (sizeof(int) + 2 * sizeof(double)) + 64));
    double* d_scale = reinterpret_cast<double*>(rowbuf);
    double* d_invscale = d_scale + n;
    int* d_rows = reinterpret_cast<int*>(d_invscale + n);
    CgScalars sc = cg_scalars(c, n);

    std::vector<double> bb(n), rr(n), dots(n);
    launch_row_dots<double>(n, npw, b64, ld, b64, ld, sc.rr, nullptr, s, true);
    PDEP_HIP(hipMemcpyAsync(bb.data(), sc.rr, n * sizeof(double), hipMemcpyDeviceToHost, s));
    PDEP_HIP(hipStreamSynchronize(s));
    // x starts at zero and r at b: the first step reads b itself, and when it updates
    // every row it writes x = its correction (zeros elsewhere) instead of adding it to a
    // zero-filled x, so neither the fill nor the copy of b is made then
    for (int i = 0; i < n; ++i) PDEP_REQUIRE(std::isfinite(bb[i]), PDEP_EINVAL, "non-finite right-hand side");
    if (ref2) {
        std::vector<double> w2(n);
        PDEP_HIP(hipMemcpyAsync(w2.data(), ref2, n * sizeof(double), hipMemcpyDeviceToHost, s));
        PDEP_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < n; ++i)
            if (bb[i] <= 1e-26 * w2[i]) bb[i] = 0.0;
    }
    rr = bb;
    std::vector<int> it_row(n, 0);
    std::vector<int> rows;
    // BF16x3 projection products in the inner solves until a row diverges with them
    bool x3 = c.opts.precision == PDEP_MIXED_BF16X3;
    // rows that ran an inner solve with FP32 products after such a divergence
    std::vector<char> fp32_row(c.opts.precision == PDEP_MIXED_BF16X3 ? n : 0, 0);
    for (int step = 0;; ++step) {
        rows.clear();
        for (int i = 0; i < n; ++i)
            if (bb[i] > 0.0 && rr[i] > tol * tol * bb[i]) rows.push_back(i);
        const int na = (int)rows.size();
        const bool set_x = step == 0 && na == n;   // the first update writes every row of x
        if (step == 0 && !set_x) launch_fill_zero(x64, vb64, s);
        if (rows.empty()) break;
        if (step >= std::max(1, c.opts.refine_maxit)) {
            st.n_notconv += (int)rows.size();
            break;
        }
        const double2* rsrc = step == 0 ? b64 : r64;   // r = b before the first update
        std::vector<double> scale(na), invscale(na), shift(na), thr2(na);
        for (int j = 0; j < na; ++j) {
            const int i = rows[j];
            const double rn = std::sqrt(rr[i]);
            scale[j] = 1.0 / rn;
            invscale[j] = rn;
            shift[j] = c.eps[i % nv];
            if (mixed) {
                // reduce by inner_tol per step, but no further than the final target needs
                // (with a 0.8 margin: the FP64 residual after an inner solve stays within
                // 1% of the FP32 estimate, so the last step lands at <= 0.81 cg_tol and a
                // row that misses is refined again)
                const double t = std::max(c.opts.inner_tol, 0.8 * tol * std::sqrt(bb[i]) / rn);
                thr2[j] = t * t;
            } else {
                const double t = 0.5 * tol * std::sqrt(bb[i]) / rn;
                thr2[j] = std::max(t * t, 1e-30);
            }
        }
        PDEP_HIP(hipMemcpyAsync(d_scale, scale.data(), na * sizeof(double), hipMemcpyHostToDevice, s));
        PDEP_HIP(hipMemcpyAsync(d_invscale, invscale.data(), na * sizeof(double), hipMemcpyHostToDevice, s));
        PDEP_HIP(hipMemcpyAsync(d_rows, rows.data(), na * sizeof(int), hipMemcpyHostToDevice, s));
        PDEP_HIP(hipMemcpyAsync(sc.shift, shift.data(), na * sizeof(double), hipMemcpyHostToDevice, s));
        PDEP_HIP(hipMemcpyAsync(sc.thr2, thr2.data(), na * sizeof(double), hipMemcpyHostToDevice, s));
        const long ldh = sphere_ld(npw);
        if (mixed) {
            float2* rhs = static_cast<float2*>(c.ws(W_RHS, (size_t)na * ldh * sizeof(float2)));
            launch_convert_rows<double, float>(na, npw, rsrc, ld, d_rows, d_scale, rhs, ldh, s);
            c.pc_x3 = x3;
            if (!fp32_row.empty() && !x3)
                for (int i : rows) fp32_row[i] = 1;
            cg_inner<float>(c, na, rhs, ldh, sc, c.opts.cg_maxit, st);
            // a diverged row (iterations reported negative) keeps its x: its solution is
            // dropped, and the remaining steps use FP32 products
            std::vector<int> itd(na);
            PDEP_HIP(hipMemcpyAsync(itd.data(), sc.iters, na * sizeof(int), hipMemcpyDeviceToHost, s));
            PDEP_HIP(hipStreamSynchronize(s));
            bool dropped = false;
            for (int j = 0; j < na; ++j)
                if (itd[j] < 0) {
                    invscale[j] = 0.0;
                    dropped = true;
                }
            if (dropped) {
                PDEP_HIP(hipMemcpyAsync(d_invscale, invscale.data(), na * sizeof(double), hipMemcpyHostToDevice, s));
                if (verbose())
                    fprintf(stderr, "[pdep] refinement step %d: BF16x3 inner solves diverged, FP32 products from here\n",
                            step + 1), fflush(stderr);
                x3 = false;
            }
            launch_axpy_rows<float>(na, npw, cg_solution<float>(c), ldh, d_rows, d_invscale, x64, ld, s, set_x);
        } else {
            double2* rhs = static_cast<double2*>(c.ws(W_RHS, (size_t)na * ldh * sizeof(double2)));
            launch_convert_rows<double, double>(na, npw, rsrc, ld, d_rows, d_scale, rhs, ldh, s);
            cg_inner<double>(c, na, rhs, ldh, sc, c.opts.cg_maxit, st);
            launch_axpy_rows<double>(na, npw, cg_solution<double>(c), ldh, d_rows, d_invscale, x64, ld, s, set_x);
        }
        std::vector<int> its(na);
        PDEP_HIP(hipMemcpyAsync(its.data(), sc.iters, na * sizeof(int), hipMemcpyDeviceToHost, s));
        // true FP64 residual of the rows just updated (all rows: no gather needed)
        const double2* xin = x64;
        if (na < n) {
            launch_convert_rows<double, double>(na, npw, x64, ld, d_rows, nullptr, xa, ld, s);
            xin = xa;
        }
        apply_op<double>(c, xin, qa, ld, na, sc.shift, na, true, true,
                         c.ws(W_STICKS, (size_t)na * sticks_row_bytes(c)),
                         static_cast<double2*>(c.ws(W_S, coef_bytes(nv, na))));
        st.op_applications++;
        launch_residual_rows(na, npw, b64, ld, d_rows, qa, ld, r64, ld, sc.rr, true, s);
        PDEP_HIP(hipMemcpyAsync(dots.data(), sc.rr, na * sizeof(double), hipMemcpyDeviceToHost, s));
        PDEP_HIP(hipStreamSynchronize(s));
        int itmax = 0;
        double worst = 0.0;
        for (int j = 0; j < na; ++j) {
            const int itj = its[j] < 0 ? -its[j] - 1 : its[j];
            rr[rows[j]] = dots[j];
            it_row[rows[j]] += itj;
            itmax = std::max(itmax, itj);
            worst = std::max(worst, std::sqrt(dots[j] / bb[rows[j]]));
        }
        st.refine_steps = std::max(st.refine_steps, step + 1);
        if (verbose())
            fprintf(stderr, "[pdep] refinement step %d: %d systems, inner CG %d iterations, worst FP64 residual %.2e\n",
                    step + 1, na, itmax, worst), fflush(stderr);
    }
    for (char f : fp32_row) st.n_fp32_fallback += f;
    for (int i = 0; i < n; ++i) {
        st.cg_iter_total += it_row[i];
        st.cg_iter_max = std::max(st.cg_iter_max, it_row[i]);
        if (bb[i] > 0.0) st.max_rel_residual = std::max(st.max_rel_residual, std::sqrt(rr[i] / bb[i]));
    }
    st.n_rhs += n;
}

namespace {

size_t row_bytes(const Ctx& c, long ld) {
    const size_t inner = c.opts.precision != PDEP_FP64 ? sizeof(float2) : sizeof(double2);
    return (size_t)ld * sizeof(double2) * 5 + (size_t)ld * inner * 6 + sticks_row_bytes(c) +
           (size_t)c.nv * sizeof(double2) + 128;
}

}  // namespace

// Device work space of chi0bar_sphere on npert perturbations run as one tile (an upper
// bound): the per-row bound above for every Sternheimer system, the potential and
// density grids, the split-K buffer and the smaller sticks block of the perturbation
// preparation that precedes the tile's.
size_t chi0_work_bytes(const Ctx& c, int npert) {
    const long ld = sphere_ld(c.basis.npw);
    const size_t per_pert = (size_t)c.nv * (row_bytes(c, ld) + 1024) + 2 * (size_t)c.basis.ng * sizeof(double);
    return (size_t)npert * per_pert + c.split_elems * sizeof(double2) +
           (size_t)std::min(npert, 256) * sticks_row_bytes(c) + ((size_t)1 << 20);
}

namespace {

int perturbation_tile(Ctx& c, int npert, long ld) {
    if (c.opts.rhs_tile > 0)
        return std::max(1, std::min({npert, c.opts.rhs_tile / std::max(1, c.nv), 65535 / std::max(1, c.nv)}));
    size_t budget = c.opts.hbm_budget;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            fr = (size_t)32 << 30;
        }
        budget = std::min((size_t)(fr * 0.6), (size_t)96 << 30);
    }
    const size_t per_pert = (size_t)c.nv * row_bytes(c, ld) + 2 * (size_t)c.basis.ng * sizeof(double);
    size_t tp = budget / std::max<size_t>(per_pert, 1);
    PDEP_REQUIRE(tp >= 1, PDEP_ENOMEM, "HBM budget below the work space of one perturbation");
    tp = std::min<size_t>(tp, (size_t)(65535 / std::max(1, c.nv)));   // launch grid limit on rows
    return (int)std::min<size_t>((size_t)npert, std::max<size_t>(tp, 1));
}

// Core chain for real z-major grid potentials Vr [npert][ng] (device).  Writes dn
// [npert][ng] z-major (if non-null) and/or the projected result out [npert][ld_out] in
// S order (if non-null).
void chi0_core(Ctx& c, int npert, const double* Vr, double* dn_out, double2* out, long ld_out, ApplyStats& st) {
    const Basis& b = c.basis;
    const int nv = c.nv, npw = b.npw;
    const long ld = sphere_ld(npw);
    const long ng = b.ng;
    hipStream_t s = c.stream;
    const int tile = perturbation_tile(c, npert, ld);
    for (int p0 = 0; p0 < npert; p0 += tile) {
        const int tp = std::min(tile, npert - p0);
        const int nrow = tp * nv;
        double2* sticks = static_cast<double2*>(c.ws(W_STICKS, (size_t)nrow * sticks_row_bytes(c)));
        double2* b64 = static_cast<double2*>(c.ws(W_B64, (size_t)nrow * ld * sizeof(double2)));
        double2* x64 = static_cast<double2*>(c.ws(W_X64, (size_t)nrow * ld * sizeof(double2)));
        double2* S = static_cast<double2*>(c.ws(W_S, coef_bytes(nv, nrow)));
        // right-hand sides b = -P_c Fwd(dV_i u_v), two bands per transform: the packed
        // orbital grids u_2j + i u_2j+1 times the real dV_i give the two products as the
        // real and imaginary parts.  The rows are half spheres (the first half_len(npw)
        // entries of each row) from here on.
        const int nvp = pair_count(nv, nv);
        launch_slab_fwd_product<double>(b.dims, b.tables, Vr + (long)p0 * ng, c.upair.as<double2>(), nvp, tp * nvp,
                                        sticks, s);
        launch_sticks_to_sphere_pair<double>(b.dims, b.tables, sticks, nrow, b64, ld, EPI_SCALE, -1.0, nullptr, 0,
                                             nullptr, nullptr, 0, s, nullptr, nv);
        double* ref2 = static_cast<double*>(c.ws(W_REF2, (size_t)nrow * sizeof(double)));
        launch_row_dots<double>(nrow, half_len(npw), b64, ld, b64, ld, ref2, nullptr, s, true);
        project_c<double>(c, b64, ld, nrow, S);
        PDEP_HIP(hipStreamSynchronize(s));
        solve_rows(c, nrow, b64, x64, ld, st, ref2);
        S = static_cast<double2*>(c.ws(W_S, coef_bytes(nv, nrow)));
        project_c<double>(c, x64, ld, nrow, S);
        // density response, two bands per transform: Inv(dc_2j + i dc_2j+1) against the
        // packed orbitals, Re(conj(u_2j + i u_2j+1) (f + i g)) = u_2j f + u_2j+1 g
        sticks = static_cast<double2*>(c.ws(W_STICKS, (size_t)nrow * sticks_row_bytes(c)));
        launch_sphere_to_sticks_pair<double>(b.dims, b.tables, x64, ld, nrow, sticks, s, nv);
        double* dn = dn_out ? dn_out + (long)p0 * ng
                            : static_cast<double*>(c.ws(W_DN, (size_t)tp * ng * sizeof(double)));
        launch_slab_density(b.dims, b.tables, sticks, tp, nvp, c.upair.as<double2>(), 4.0 / b.omega, dn, s);
        if (out) {
            launch_slab_fwd_product<double>(b.dims, b.tables, dn, nullptr, 1, tp, sticks, s);
            launch_sticks_to_sphere<double>(b.dims, b.tables, sticks, tp, out + (long)p0 * ld_out, ld_out, EPI_GSCALE,
                                            0.0, nullptr, 0, nullptr, nullptr, 0, b.d_coul.as<double>(), s);
        }
        PDEP_HIP(hipStreamSynchronize(s));
    }
}

}  // namespace

void chi0_grid(Ctx& c, int npert, const double* dv, double* dn, ApplyStats& st) {
    chi0_core(c, npert, dv, dn, nullptr, 0, st);
}

void rhs_half_rows(Ctx& c, int npert, const double2* phi, double2* W, long ld) {
    const Basis& b = c.basis;
    const int nv = c.nv, nrow = npert * nv;
    hipStream_t s = c.stream;
    double* Vr = static_cast<double*>(c.ws(W_VR, (size_t)npert * b.ng * sizeof(double)));
    double2* sticks = static_cast<double2*>(c.ws(W_STICKS, (size_t)std::max(npert, nrow) * sticks_row_bytes(c)));
    // V_i = Re Inv(sqrt(4 pi)/|G| phi_i), then P_c Fwd(V_i u_v) for the band pairs
    launch_sphere_to_sticks<double>(b.dims, b.tables, phi, sphere_ld(b.npw), npert, b.d_coul.as<double>(), sticks, s);
    launch_slab_inv_store<double>(b.dims, b.tables, sticks, npert, nullptr, Vr, s);
    const int nvp = pair_count(nv, nv);
    launch_slab_fwd_product<double>(b.dims, b.tables, Vr, c.upair.as<double2>(), nvp, npert * nvp, sticks, s);
    launch_sticks_to_sphere_pair<double>(b.dims, b.tables, sticks, nrow, W, ld, EPI_SCALE, 1.0, nullptr, 0, nullptr,
                                         nullptr, 0, s, nullptr, nv);
    project_c<double>(c, W, ld, nrow, static_cast<double2*>(c.ws(W_S, coef_bytes(nv, nrow))));
}

const double2* rhs_coefficients(Ctx& c) { return static_cast<const double2*>(c.ws_current(W_S)); }

void apply_deflated_h64(Ctx& c, const double2* q, double2* z, long ld, int nrows, const double* zero_shift) {
    apply_op<double>(c, q, z, ld, nrows, zero_shift, 1, true, true,
                     c.ws(W_STICKS, (size_t)nrows * sticks_row_bytes(c)),
                     static_cast<double2*>(c.ws(W_S, coef_bytes(c.nv, nrows))));
}

void chi0bar_sphere(Ctx& c, int npert, const double2* phi, double2* out, ApplyStats& st) {
    const Basis& b = c.basis;
    const long ld = sphere_ld(b.npw);
    double* Vr = static_cast<double*>(c.ws(W_VR, (size_t)npert * b.ng * sizeof(double)));
    // dV_i = Re Inv(sqrt(4 pi)/|G| phi_i), processed in chunks to bound the plane buffer
    const int chunk = 256;
    for (int p0 = 0; p0 < npert; p0 += chunk) {
        const int np = std::min(chunk, npert - p0);
        double2* sticks = static_cast<double2*>(c.ws(W_STICKS, (size_t)np * sticks_row_bytes(c)));
        launch_sphere_to_sticks<double>(b.dims, b.tables, phi + (long)p0 * ld, ld, np, b.d_coul.as<double>(), sticks,
                                        c.stream);
        launch_slab_inv_store<double>(b.dims, b.tables, sticks, np, nullptr, Vr + (long)p0 * b.ng, c.stream);
    }
    chi0_core(c, npert, Vr, nullptr, out, ld, st);
}

template void project_c<double>(Ctx&, double2*, long, int, double2*);
template void project_c<float>(Ctx&, float2*, long, int, double2*);

}  // namespace pdep
