// Block Davidson eigensolvers (FP64):
//  - ground state: the N_v + 1 lowest eigenpairs of the Kohn-Sham H (to get the
//    occupied orbitals and the HOMO-LUMO gap);
//  - PDEP: the n_pdep lowest (most screened) eigenpairs of chi0bar (Sec. 2.3: an
//    orthonormal random start, chi0bar applied to the block through the Sternheimer
//    chain, diagonalisation of the projected matrix, iterate; the paper names the
//    Davidson algorithm for this iteration).
// Both follow the same scheme: Rayleigh-Ritz on the search space V (orthonormal
// columns), residuals r_i = A x_i - theta_i x_i of the wanted Ritz pairs, expansion by
// the (preconditioned, for H) residuals of the unconverged pairs orthogonalised twice
// against V and orthonormalised among themselves, restart from the Ritz vectors when
// V would exceed its maximum size.  Small dense eigenproblems go to rocSOLVER.
//
// For PDEP every vector is Hermitian-symmetric (real in r) and all combination
// coefficients are kept real, so the projected matrices are real symmetric.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "pdep_internal.h"

namespace pdep {

namespace {

// r = a - theta[row] * b
__global__ void k_ritz_residual(int K, const double2* __restrict__ a, const double2* __restrict__ b, long ld,
                                const double* __restrict__ theta, double2* __restrict__ r) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (k >= K) return;
    const long o = (long)row * ld + k;
    const double t = theta[row];
    r[o] = make_double2(a[o].x - t * b[o].x, a[o].y - t * b[o].y);
}

// t = r / (1 + max(0, 1/2|G|^2 - theta))
__global__ void k_precond_h(int K, double2* __restrict__ r, long ld, const double* __restrict__ kin,
                            const double* __restrict__ theta) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (k >= K) return;
    const double d = kin[k] - theta[row];
    const double f = 1.0 / (1.0 + (d > 0.0 ? d : 0.0));
    const long o = (long)row * ld + k;
    r[o].x *= f;
    r[o].y *= f;
}

void ritz_residual(int nrows, int K, const double2* a, const double2* b, long ld, const double* theta, double2* r,
                   hipStream_t s) {
    if (nrows <= 0) return;
    hipLaunchKernelGGL(k_ritz_residual, dim3((K + 255) / 256, nrows), dim3(256), 0, s, K, a, b, ld, theta, r);
    PDEP_HIP(hipGetLastError());
}

void precond_h(int nrows, int K, double2* r, long ld, const double* kin, const double* theta, hipStream_t s) {
    if (nrows <= 0) return;
    hipLaunchKernelGGL(k_precond_h, dim3((K + 255) / 256, nrows), dim3(256), 0, s, K, r, ld, kin, theta);
    PDEP_HIP(hipGetLastError());
}

// SplitMix64 (Steele, Lea & Flood 2014) and Box-Muller normals for the library's own
// random starting vectors.
struct SplitMix64 {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    void normal2(double& a, double& b) {
        const double u1 = uniform(), u2 = uniform();
        const double rad = std::sqrt(-2.0 * std::log(u1));
        a = rad * std::cos(2.0 * M_PI * u2);
        b = rad * std::sin(2.0 * M_PI * u2);
    }
};

// rocBLAS handle for rocSOLVER calls: the context's (created on first use and kept for
// the context's lifetime, or supplied by the server worker), bound to the context stream.
// The device work space of each call comes from the context allocator: the call is made
// once as a size query, the context's work-space buffer grows to that size and is handed
// to the handle, and then the call runs.
struct Solver {
    Ctx& c;
    rocblas_handle h = nullptr;
    explicit Solver(Ctx& cc) : c(cc) {
        if (!c.blas) {
            rocblas_handle nh = nullptr;
            if (rocblas_create_handle(&nh) != rocblas_status_success)
                throw Error(PDEP_EDEVICE, "rocblas_create_handle failed");
            c.blas = nh;
            c.own_blas = true;
        }
        h = static_cast<rocblas_handle>(c.blas);
        rocblas_set_stream(h, c.stream);
    }
    template <typename F>
    rocblas_status run(F&& call) {
        size_t need = 0;
        PDEP_REQUIRE(rocblas_start_device_memory_size_query(h) == rocblas_status_success, PDEP_EDEVICE,
                     "rocblas size query failed");
        call();
        PDEP_REQUIRE(rocblas_stop_device_memory_size_query(h, &need) == rocblas_status_success, PDEP_EDEVICE,
                     "rocblas size query failed");
        c.blas_ws.ensure(&c.al, std::max<size_t>(need, 256));
        PDEP_REQUIRE(rocblas_set_workspace(h, c.blas_ws.get(), c.blas_ws.bytes()) == rocblas_status_success,
                     PDEP_EDEVICE, "rocblas_set_workspace failed");
        return call();
    }
};

enum DSlot { D_V = 0, D_AV, D_X, D_AX, D_R, D_T, D_T2, D_M, D_W, D_TH, D_INFO, D_ROWS, D_SPLIT, D_COUNT };

struct Workspace {
    Ctx& c;
    Buf b[D_COUNT];
    explicit Workspace(Ctx& cc) : c(cc) {}
    void* get(int i, size_t bytes) { b[i].ensure(&c.al, bytes); return b[i].get(); }
    // split-K partial products for the projected-matrix GEMMs
    static constexpr size_t kSplitElems = (size_t)4 << 20;
    double2* split() { return static_cast<double2*>(get(D_SPLIT, kSplitElems * sizeof(double2))); }
};

// Host copy of S[n][m] (double2, N x M, ld lds) -> complex vector.
std::vector<double2> d2h(const double2* d, size_t n, hipStream_t s) {
    std::vector<double2> h(n);
    PDEP_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(double2), hipMemcpyDeviceToHost, s));
    PDEP_HIP(hipStreamSynchronize(s));
    return h;
}

// Dense eigensolve of an m x m matrix on the device.  Hermitian complex (real_sym =
// false) or real symmetric (true; the input is the real part of the complex buffer).
// On return `vec` holds eigenvectors as columns (column-major, ld m) in complex form
// (imaginary parts zero for real_sym) and `w` the ascending eigenvalues (host).
//
// Divide and conquer (syevd/heevd) first.  rocSOLVER's complex divide and conquer can
// return non-finite eigenvectors with info = 0 for a (numerically) diagonal input of
// order above 64, which is exactly what the Gram matrix of an already orthonormal
// block is; every result is therefore checked and a non-finite one is recomputed by
// QR iteration (syev/heev) from the kept host copy of the matrix.
void dense_eig(Workspace& ws, Solver& sv, std::vector<double2>& A, int m, bool real_sym, std::vector<double>& w,
               std::vector<double2>& vec) {
    hipStream_t s = ws.c.stream;
    // symmetrise: A[n][k] holds <V_k, A V_n>; column-major element (k, n) = A[n*m + k]
    for (int n = 0; n < m; ++n)
        for (int k = 0; k <= n; ++k) {
            double2 a = A[(size_t)n * m + k], b = A[(size_t)k * m + n];
            double re = 0.5 * (a.x + b.x), im = 0.5 * (a.y - b.y);
            if (real_sym) im = 0.0;
            A[(size_t)n * m + k] = make_double2(re, im);
            A[(size_t)k * m + n] = make_double2(re, -im);
        }
    double* dW = static_cast<double*>(ws.get(D_TH, 2 * (size_t)m * sizeof(double) + 64));
    double* dE = dW + m;
    int* dinfo = static_cast<int*>(ws.get(D_INFO, 64));
    auto solve = [&](bool divide_conquer) -> int {
        w.assign(m, 0.0);
        vec.assign((size_t)m * m, make_double2(0, 0));
        rocblas_status st;
        if (real_sym) {
            std::vector<double> Ar((size_t)m * m);
            for (size_t i = 0; i < Ar.size(); ++i) Ar[i] = A[i].x;
            double* dA = static_cast<double*>(ws.get(D_M, (size_t)m * m * sizeof(double2)));
            PDEP_HIP(hipMemcpyAsync(dA, Ar.data(), Ar.size() * sizeof(double), hipMemcpyHostToDevice, s));
            st = sv.run([&] {
                return divide_conquer
                           ? rocsolver_dsyevd(sv.h, rocblas_evect_original, rocblas_fill_lower, m, dA, m, dW, dE, dinfo)
                           : rocsolver_dsyev(sv.h, rocblas_evect_original, rocblas_fill_lower, m, dA, m, dW, dE, dinfo);
            });
            PDEP_REQUIRE(st == rocblas_status_success, PDEP_EDEVICE, "rocsolver_dsyev(d) failed");
            PDEP_HIP(hipMemcpyAsync(Ar.data(), dA, Ar.size() * sizeof(double), hipMemcpyDeviceToHost, s));
            PDEP_HIP(hipMemcpyAsync(w.data(), dW, m * sizeof(double), hipMemcpyDeviceToHost, s));
            PDEP_HIP(hipStreamSynchronize(s));
            for (size_t i = 0; i < Ar.size(); ++i) vec[i] = make_double2(Ar[i], 0.0);
        } else {
            double2* dA = static_cast<double2*>(ws.get(D_M, (size_t)m * m * sizeof(double2)));
            auto* zA = reinterpret_cast<rocblas_double_complex*>(dA);
            PDEP_HIP(hipMemcpyAsync(dA, A.data(), A.size() * sizeof(double2), hipMemcpyHostToDevice, s));
            st = sv.run([&] {
                return divide_conquer
                           ? rocsolver_zheevd(sv.h, rocblas_evect_original, rocblas_fill_lower, m, zA, m, dW, dE, dinfo)
                           : rocsolver_zheev(sv.h, rocblas_evect_original, rocblas_fill_lower, m, zA, m, dW, dE, dinfo);
            });
            PDEP_REQUIRE(st == rocblas_status_success, PDEP_EDEVICE, "rocsolver_zheev(d) failed");
            PDEP_HIP(hipMemcpyAsync(vec.data(), dA, vec.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
            PDEP_HIP(hipMemcpyAsync(w.data(), dW, m * sizeof(double), hipMemcpyDeviceToHost, s));
            PDEP_HIP(hipStreamSynchronize(s));
        }
        int info = 0;
        PDEP_HIP(hipMemcpyAsync(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost, s));
        PDEP_HIP(hipStreamSynchronize(s));
        return info;
    };
    auto finite = [&]() {
        for (double x : w)
            if (!std::isfinite(x)) return false;
        for (const double2& v : vec)
            if (!std::isfinite(v.x) || !std::isfinite(v.y)) return false;
        return true;
    };
    int info = solve(true);
    if (info != 0 || !finite()) info = solve(false);
    if (info != 0 || !finite()) {
        double amax = 0.0, herm = 0.0;
        bool fin = true;
        for (int n = 0; n < m; ++n)
            for (int k = 0; k < m; ++k) {
                const double2 a = A[(size_t)n * m + k], b = A[(size_t)k * m + n];
                fin = fin && std::isfinite(a.x) && std::isfinite(a.y);
                amax = std::max(amax, std::hypot(a.x, a.y));
                herm = std::max(herm, std::hypot(a.x - b.x, a.y + b.y));
            }
        throw Error(PDEP_EDEVICE, "dense eigensolver failed (info " + std::to_string(info) + ", n " +
                                      std::to_string(m) + (real_sym ? ", real" : ", complex") +
                                      (fin ? ", finite input" : ", NON-FINITE input") + ", max " +
                                      std::to_string(amax) + ", hermitian defect " + std::to_string(herm) + ")");
    }
}

// Y[j] = sum_i X[i] * C[j][i]  (C host, N x M complex, row j = coefficients of output j)
void combine(Ctx& c, const double2* X, int M, int N, long ld, const std::vector<double2>& C, double2* Y,
             double2* Cdev) {
    const int npw = c.basis.npw;
    PDEP_HIP(hipMemcpyAsync(Cdev, C.data(), (size_t)N * M * sizeof(double2), hipMemcpyHostToDevice, c.stream));
    launch_gemm_update<double>(M, N, npw, X, ld, Cdev, M, 1.0, 0.0, Y, ld, c.stream);
    PDEP_HIP(hipStreamSynchronize(c.stream));   // C is pageable host memory owned by the caller
}

// Scale every row of T to unit norm and drop rows whose norm is below `drop` (relative
// to their norm before the last projection, i.e. rows that were already in span(V)).
// Returns the number of rows kept (compacted to the front of T).
int normalise_rows(Ctx& c, Workspace& ws, double2* T, int nt, long ld, const std::vector<double>& ref, double drop,
                   std::vector<double>& norms_out) {
    const int npw = c.basis.npw;
    hipStream_t s = c.stream;
    double* dn = static_cast<double*>(ws.get(D_TH, 2 * (size_t)std::max(nt, 1) * sizeof(double) + 64));
    launch_row_dots<double>(nt, npw, T, ld, T, ld, dn, nullptr, s);
    std::vector<double> n2(nt);
    PDEP_HIP(hipMemcpyAsync(n2.data(), dn, nt * sizeof(double), hipMemcpyDeviceToHost, s));
    PDEP_HIP(hipStreamSynchronize(s));
    std::vector<int> keep;
    std::vector<double> scale;
    norms_out.clear();
    for (int j = 0; j < nt; ++j) {
        const double nj = std::sqrt(std::max(n2[j], 0.0));
        const double r = ref.empty() ? 1.0 : ref[j];
        if (nj > drop * r && nj > 1e-300) {
            keep.push_back(j);
            scale.push_back(1.0 / nj);
            norms_out.push_back(1.0);
        }
    }
    const int nk = (int)keep.size();
    if (nk == 0) return 0;
    char* rb = static_cast<char*>(ws.get(D_ROWS, (size_t)nk * (sizeof(double) + sizeof(int)) + 64));
    double* dscale = reinterpret_cast<double*>(rb);
    int* drows = reinterpret_cast<int*>(dscale + nk);
    double2* T2 = static_cast<double2*>(ws.get(D_T2, (size_t)nk * ld * sizeof(double2)));
    PDEP_HIP(hipMemcpyAsync(dscale, scale.data(), nk * sizeof(double), hipMemcpyHostToDevice, s));
    PDEP_HIP(hipMemcpyAsync(drows, keep.data(), nk * sizeof(int), hipMemcpyHostToDevice, s));
    launch_convert_rows<double, double>(nk, npw, T, ld, drows, dscale, T2, ld, s);
    PDEP_HIP(hipMemcpyAsync(T, T2, (size_t)nk * ld * sizeof(double2), hipMemcpyDeviceToDevice, s));
    PDEP_HIP(hipStreamSynchronize(s));
    return nk;
}

// Orthonormalise the nt rows of T (in place) against the m orthonormal rows of V and
// among themselves.  Each of two rounds: unit-normalise the rows, project out V twice
// (classical Gram-Schmidt, twice), drop rows that lost all but 1e-8 of their norm
// (already in span(V)), renormalise, and orthonormalise the block through the
// eigen-decomposition of its Gram matrix (directions with relative weight below
// 1e-12 dropped).  real_coef keeps every combination coefficient real (Hermitian-
// symmetric vectors stay Hermitian-symmetric).  Returns the number of rows kept.
int orthonormalise(Ctx& c, Workspace& ws, Solver& sv, const double2* V, int m, double2* T, int nt, long ld,
                   bool real_coef) {
    const int npw = c.basis.npw;
    hipStream_t s = c.stream;
    std::vector<double> unit, unit2;
    for (int round = 0; round < 2 && nt > 0; ++round) {
        nt = normalise_rows(c, ws, T, nt, ld, {}, 1e-300, unit);
        if (nt == 0) break;
        if (m > 0) {
            double2* Cdev = static_cast<double2*>(ws.get(D_W, (size_t)std::max(m, nt) * nt * sizeof(double2) + 64));
            for (int pass = 0; pass < 2; ++pass) {
                launch_gemm_ahb<double>(m, nt, npw, V, ld, T, ld, Cdev, m, ws.split(), Workspace::kSplitElems, s);   // C[j][i] = <V_i, T_j>
                if (real_coef) {
                    std::vector<double2> C = d2h(Cdev, (size_t)nt * m, s);
                    for (auto& x : C) x.y = 0.0;
                    PDEP_HIP(hipMemcpyAsync(Cdev, C.data(), C.size() * sizeof(double2), hipMemcpyHostToDevice, s));
                    PDEP_HIP(hipStreamSynchronize(s));
                }
                launch_gemm_update<double>(m, nt, npw, V, ld, Cdev, m, -1.0, 1.0, T, ld, s);
            }
            nt = normalise_rows(c, ws, T, nt, ld, unit, 1e-8, unit2);
            if (nt == 0) break;
        }
        double2* Cdev = static_cast<double2*>(ws.get(D_W, (size_t)std::max(m, nt) * nt * sizeof(double2) + 64));
        launch_gemm_ahb<double>(nt, nt, npw, T, ld, T, ld, Cdev, nt, ws.split(), Workspace::kSplitElems, s);
        std::vector<double2> G = d2h(Cdev, (size_t)nt * nt, s);
        std::vector<double> w;
        std::vector<double2> Q;
        dense_eig(ws, sv, G, nt, real_coef, w, Q);
        const double wmax = std::max(w.empty() ? 0.0 : w.back(), 1e-300);
        std::vector<double2> C;
        int kept = 0;
        for (int j = nt - 1; j >= 0; --j) {
            if (w[j] <= 1e-12 * wmax) continue;
            const double f = 1.0 / std::sqrt(w[j]);
            for (int i = 0; i < nt; ++i) {
                const double2 q = Q[(size_t)j * nt + i];   // column j, row i
                C.push_back(make_double2(q.x * f, real_coef ? 0.0 : q.y * f));
            }
            ++kept;
        }
        if (kept == 0) return 0;
        double2* T2 = static_cast<double2*>(ws.get(D_T2, (size_t)kept * ld * sizeof(double2)));
        combine(c, T, nt, kept, ld, C, T2, Cdev);
        PDEP_HIP(hipMemcpyAsync(T, T2, (size_t)kept * ld * sizeof(double2), hipMemcpyDeviceToDevice, s));
        nt = kept;
    }
    PDEP_HIP(hipStreamSynchronize(s));
    return nt;
}

// Throws PDEP_EDEVICE naming `what` if any of the nrows rows holds a non-finite value.
void check_finite_rows(Ctx& c, Workspace& ws, const double2* X, int nrows, long ld, const char* what) {
    if (nrows <= 0) return;
    double* dn = static_cast<double*>(ws.get(D_TH, 2 * (size_t)nrows * sizeof(double) + 64));
    launch_row_dots<double>(nrows, c.basis.npw, X, ld, X, ld, dn, nullptr, c.stream);
    std::vector<double> n2(nrows);
    PDEP_HIP(hipMemcpyAsync(n2.data(), dn, nrows * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    PDEP_HIP(hipStreamSynchronize(c.stream));
    for (int i = 0; i < nrows; ++i)
        if (!std::isfinite(n2[i]))
            throw Error(PDEP_EDEVICE, std::string("non-finite values in ") + what + " (row " + std::to_string(i) +
                                          " of " + std::to_string(nrows) + ")");
}

}  // namespace

Ctx::~Ctx() {
    if (own_blas && blas) rocblas_destroy_handle(static_cast<rocblas_handle>(blas));
    if (graph_stream) {
        (void)hipStreamSynchronize(graph_stream);
        (void)hipStreamDestroy(graph_stream);
    }
    if (graph_event) (void)hipEventDestroy(graph_event);
}

// ------------------------------------------------------------------ ground state ---
void ground_state(Ctx& c) {
    const Basis& b = c.basis;
    const int npw = b.npw, nv = c.nv;
    const long ld = sphere_ld(npw);
    hipStream_t s = c.stream;
    Solver sv(c);
    Workspace ws(c);
    const int want = nv + 1;                       // the LUMO gives the gap
    const int nb = std::min(npw - 1, want + std::max(4, want / 8));
    PDEP_REQUIRE(want < npw, PDEP_EINVAL, "n_v must be smaller than the number of plane waves");
    const int mmax = std::min(npw, std::max(3 * nb, nb + 32));
    double2* V = static_cast<double2*>(ws.get(D_V, (size_t)mmax * ld * sizeof(double2)));
    double2* AV = static_cast<double2*>(ws.get(D_AV, (size_t)mmax * ld * sizeof(double2)));
    double2* X = static_cast<double2*>(ws.get(D_X, (size_t)nb * ld * sizeof(double2)));
    double2* AX = static_cast<double2*>(ws.get(D_AX, (size_t)nb * ld * sizeof(double2)));
    double2* R = static_cast<double2*>(ws.get(D_R, (size_t)nb * ld * sizeof(double2)));
    double2* sticks = static_cast<double2*>(c.ws(WS_SETUP_STICKS, (size_t)mmax * b.dims.nz * b.dims.sld * sizeof(double2)));
    double* dtheta = static_cast<double*>(c.ws(WS_DAV_THETA, (size_t)mmax * sizeof(double) * 2 + 64));
    double* dzero = dtheta + mmax;
    launch_fill_zero(dzero, (size_t)mmax * sizeof(double), s);
    double2* Cdev = static_cast<double2*>(c.ws(WS_DAV_C, (size_t)mmax * mmax * sizeof(double2)));
    double* dots = static_cast<double*>(c.ws(WS_DAV_DOTS, (size_t)mmax * sizeof(double) + 64));

    // random start weighted towards low kinetic energy
    std::vector<double2> h0((size_t)nb * ld, make_double2(0, 0));
    SplitMix64 rng{0x5eedull + (uint64_t)npw * 1315423911ull};
    for (int j = 0; j < nb; ++j)
        for (int k = 0; k < npw; ++k) {
            double a, bb;
            rng.normal2(a, bb);
            const double wgt = 1.0 / ((1.0 + b.kin[k]) * (1.0 + b.kin[k]));
            h0[(size_t)j * ld + k] = make_double2(a * wgt, bb * wgt);
        }
    PDEP_HIP(hipMemcpyAsync(V, h0.data(), h0.size() * sizeof(double2), hipMemcpyHostToDevice, s));
    int m = orthonormalise(c, ws, sv, nullptr, 0, V, nb, ld, false);
    check_finite_rows(c, ws, V, m, ld, "the orthonormalised start block");
    apply_h64(c, V, ld, m, dzero, 1, AV, ld, sticks);
    check_finite_rows(c, ws, AV, m, ld, "H applied to the start block");
    const double tol = c.opts.gs_tol;
    std::vector<double> theta, rn(nb);
    int it = 0;
    bool conv = false;
    double maxres = 0.0;
    for (it = 1; it <= c.opts.gs_maxit; ++it) {
        launch_gemm_ahb<double>(m, m, npw, V, ld, AV, ld, Cdev, m, ws.split(), Workspace::kSplitElems, s);
        std::vector<double2> M = d2h(Cdev, (size_t)m * m, s);
        std::vector<double2> Y;
        dense_eig(ws, sv, M, m, false, theta, Y);
        const int k = std::min(nb, m);
        // Ritz vectors: X_j = sum_i V_i Y[i][j]  -> coefficient rows = columns of Y
        std::vector<double2> C(Y.begin(), Y.begin() + (size_t)k * m);
        combine(c, V, m, k, ld, C, X, Cdev);
        combine(c, AV, m, k, ld, C, AX, Cdev);
        PDEP_HIP(hipMemcpyAsync(dtheta, theta.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
        ritz_residual(k, npw, AX, X, ld, dtheta, R, s);
        launch_row_dots<double>(k, npw, R, ld, R, ld, dots, nullptr, s);
        std::vector<double> r2(k);
        PDEP_HIP(hipMemcpyAsync(r2.data(), dots, k * sizeof(double), hipMemcpyDeviceToHost, s));
        PDEP_HIP(hipStreamSynchronize(s));
        maxres = 0.0;
        std::vector<int> unconv;
        for (int j = 0; j < k; ++j) {
            rn[j] = std::sqrt(std::max(r2[j], 0.0));
            if (j < want) maxres = std::max(maxres, rn[j]);
            if (rn[j] > tol) unconv.push_back(j);
        }
        if (verbose() && (it % 10 == 1))
            fprintf(stderr, "[pdep] ground state it %d: subspace %d, max residual %.2e\n", it, m, maxres), fflush(stderr);
        if (maxres <= tol) { conv = true; break; }
        // expansion vectors: preconditioned residuals of unconverged pairs
        int nt = (int)unconv.size();
        if (m + nt > mmax) {          // restart from the Ritz vectors
            PDEP_HIP(hipMemcpyAsync(V, X, (size_t)k * ld * sizeof(double2), hipMemcpyDeviceToDevice, s));
            PDEP_HIP(hipMemcpyAsync(AV, AX, (size_t)k * ld * sizeof(double2), hipMemcpyDeviceToDevice, s));
            m = k;
        }
        nt = std::min(nt, mmax - m);  // V and AV hold mmax columns
        if (nt <= 0) break;
        double2* T = static_cast<double2*>(ws.get(D_T, (size_t)nt * ld * sizeof(double2)));
        std::vector<double> th_sel(nt);
        for (int j = 0; j < nt; ++j) {
            PDEP_HIP(hipMemcpyAsync(T + (size_t)j * ld, R + (size_t)unconv[j] * ld, ld * sizeof(double2),
                                    hipMemcpyDeviceToDevice, s));
            th_sel[j] = theta[unconv[j]];
        }
        PDEP_HIP(hipMemcpyAsync(dtheta, th_sel.data(), nt * sizeof(double), hipMemcpyHostToDevice, s));
        precond_h(nt, npw, T, ld, b.d_kin64.as<double>(), dtheta, s);
        const int kept = orthonormalise(c, ws, sv, V, m, T, nt, ld, false);
        if (kept == 0) break;
        PDEP_HIP(hipMemcpyAsync(V + (size_t)m * ld, T, (size_t)kept * ld * sizeof(double2), hipMemcpyDeviceToDevice, s));
        check_finite_rows(c, ws, V + (size_t)m * ld, kept, ld, "the ground-state expansion vectors");
        apply_h64(c, V + (size_t)m * ld, ld, kept, dzero, 1, AV + (size_t)m * ld, ld, sticks);
        check_finite_rows(c, ws, AV + (size_t)m * ld, kept, ld, "H applied to the expansion vectors");
        m += kept;
    }
    PDEP_REQUIRE(conv, PDEP_ENOTCONV,
                 "ground-state Davidson did not reach gs_tol (residual " + std::to_string(maxres) + ")");
    c.eps.assign(theta.begin(), theta.begin() + nv);
    c.gap = theta[nv] - theta[nv - 1];
    c.gs_iterations = it;
    c.gs_residual = maxres;
    c.psi64.ensure(&c.al, (size_t)nv * npw * sizeof(double2));
    PDEP_HIP(hipMemcpy2DAsync(c.psi64.get(), npw * sizeof(double2), X, ld * sizeof(double2), npw * sizeof(double2),
                              nv, hipMemcpyDeviceToDevice, s));
    PDEP_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------ orbitals real in r ---
namespace {

// Row j of psi -> rows j (A) and nv + j (B) of v: A = (psi + conj psi(-G)) / 2 and
// B = (psi - conj psi(-G)) / 2i, the coefficients of Re psi(r) and Im psi(r).  The
// sphere order puts -G_k at npw - 1 - k.
__global__ void k_sym_split(int npw, int nv, const double2* __restrict__ psi, long ldp, double2* __restrict__ v,
                            long ldv) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (k >= npw) return;
    const double2 p = psi[(long)j * ldp + k], q = psi[(long)j * ldp + npw - 1 - k];
    // q* = (q.x, -q.y)
    v[(long)j * ldv + k] = make_double2(0.5 * (p.x + q.x), 0.5 * (p.y - q.y));
    v[(long)(nv + j) * ldv + k] = make_double2(0.5 * (p.y + q.y), -0.5 * (p.x - q.x));
}

}  // namespace

// The orbitals are replaced by an orthonormal basis of the same occupied subspace made
// of functions that are real in r (Hermitian-symmetric coefficients), each a Ritz
// vector of H in that subspace.  H is real in r, so conjugation in r maps eigenvectors
// to eigenvectors of the same energy: the occupied subspace of a gapped system is
// closed under it and the real and imaginary parts (in r) of the orbitals span it.  The
// 2 N_v parts have a Gram matrix with N_v eigenvalues 1 and N_v eigenvalues 0; the
// eigenvectors of the first N_v give an orthonormal real basis, and Rayleigh-Ritz with
// H (real symmetric) rotates it into Ritz vectors.
void realify_orbitals(Ctx& c) {
    const Basis& b = c.basis;
    const int npw = b.npw, nv = c.nv, m = 2 * nv;
    const long ld = sphere_ld(npw);
    hipStream_t s = c.stream;
    Solver sv(c);
    Workspace ws(c);
    double2* V = static_cast<double2*>(ws.get(D_V, (size_t)m * ld * sizeof(double2)));
    double2* X = static_cast<double2*>(ws.get(D_X, (size_t)nv * ld * sizeof(double2)));
    double2* AX = static_cast<double2*>(ws.get(D_AX, (size_t)nv * ld * sizeof(double2)));
    double2* sticks = static_cast<double2*>(c.ws(WS_SETUP_STICKS, (size_t)nv * b.dims.nz * b.dims.sld * sizeof(double2)));
    double* dtheta = static_cast<double*>(c.ws(WS_DAV_THETA, (size_t)m * sizeof(double) * 2 + 64));
    double2* Cdev = static_cast<double2*>(c.ws(WS_DAV_C, (size_t)m * m * sizeof(double2)));
    launch_fill_zero(V, (size_t)m * ld * sizeof(double2), s);
    hipLaunchKernelGGL(k_sym_split, dim3((npw + 255) / 256, nv), dim3(256), 0, s, npw, nv, c.psi64.as<double2>(),
                       (long)npw, V, ld);
    PDEP_HIP(hipGetLastError());
    launch_gemm_ahb<double>(m, m, npw, V, ld, V, ld, Cdev, m, ws.split(), Workspace::kSplitElems, s);
    std::vector<double2> G = d2h(Cdev, (size_t)m * m, s);
    std::vector<double> w;
    std::vector<double2> Q;
    dense_eig(ws, sv, G, m, true, w, Q);
    const double wmax = std::max(w[m - 1], 1e-300);
    PDEP_REQUIRE(w[nv - 1] <= 1e-6 * wmax && w[nv] >= 0.5 * wmax, PDEP_EINVAL,
                 "the orbitals do not span a subspace closed under complex conjugation in r (Gram eigenvalues " +
                     std::to_string(w[nv - 1]) + " and " + std::to_string(w[nv]) +
                     "): they are not the complete occupied eigenspace of H");
    std::vector<double2> C((size_t)nv * m);
    for (int j = 0; j < nv; ++j) {
        const int col = m - 1 - j;
        const double f = 1.0 / std::sqrt(w[col]);
        for (int i = 0; i < m; ++i) C[(size_t)j * m + i] = make_double2(Q[(size_t)col * m + i].x * f, 0.0);
    }
    combine(c, V, m, nv, ld, C, X, Cdev);
    launch_sym_fix(nv, npw, X, ld, s);
    // Rayleigh-Ritz with H in the real basis
    double* dzero = dtheta + m;
    launch_fill_zero(dzero, sizeof(double), s);
    apply_h64(c, X, ld, nv, dzero, 1, AX, ld, sticks);
    launch_gemm_ahb<double>(nv, nv, npw, X, ld, AX, ld, Cdev, nv, ws.split(), Workspace::kSplitElems, s);
    std::vector<double2> Hm = d2h(Cdev, (size_t)nv * nv, s);
    std::vector<double> theta;
    std::vector<double2> Y;
    dense_eig(ws, sv, Hm, nv, true, theta, Y);
    std::vector<double2> C2(Y.begin(), Y.begin() + (size_t)nv * nv);
    for (auto& x : C2) x.y = 0.0;
    combine(c, X, nv, nv, ld, C2, V, Cdev);
    launch_sym_fix(nv, npw, V, ld, s);
    PDEP_HIP(hipMemcpy2DAsync(c.psi64.get(), npw * sizeof(double2), V, ld * sizeof(double2), npw * sizeof(double2),
                              nv, hipMemcpyDeviceToDevice, s));
    PDEP_HIP(hipStreamSynchronize(s));
    double dmax = 0.0;
    for (int j = 0; j < nv; ++j) dmax = std::max(dmax, std::abs(theta[j] - c.eps[j]));
    if (verbose())
        fprintf(stderr, "[pdep] orbitals made real in r: Gram split %.2e / %.2e, max |d eps| %.2e\n", w[nv - 1],
                w[nv], dmax), fflush(stderr);
    c.eps.assign(theta.begin(), theta.begin() + nv);
}

// --------------------------------------------------------------------------- PDEP --
EigResult pdep_davidson(Ctx& c, int npdep, uint64_t seed, const double2* phi0_dev, const pdep_eig_opts& eo,
                        double* lam_out, double2* basis_out_dev) {
    const Basis& b = c.basis;
    const int npw = b.npw;
    const long ld = sphere_ld(npw);
    hipStream_t s = c.stream;
    Solver sv(c);
    Workspace ws(c);
    EigResult res;
    PDEP_REQUIRE(npdep >= 1 && npdep < npw - 1, PDEP_EINVAL, "n_pdep must be between 1 and N_pw' - 1");
    const int nb = std::min(npw - 1, npdep + std::max(0, eo.n_buffer));
    // After a restart the search space holds the nb Ritz vectors and grows by at most nb
    // residuals, so it needs room for 2 nb columns.
    PDEP_REQUIRE(eo.max_subspace <= 0 || eo.max_subspace >= 2 * nb, PDEP_EINVAL,
                 "max_subspace must be 0 or at least 2 (n_pdep + n_buffer)");
    const int mmax = pdep_subspace_max(npw, npdep, eo);
    double2* V = static_cast<double2*>(ws.get(D_V, (size_t)mmax * ld * sizeof(double2)));
    double2* AV = static_cast<double2*>(ws.get(D_AV, (size_t)mmax * ld * sizeof(double2)));
    double2* X = static_cast<double2*>(ws.get(D_X, (size_t)nb * ld * sizeof(double2)));
    double2* AX = static_cast<double2*>(ws.get(D_AX, (size_t)nb * ld * sizeof(double2)));
    double2* R = static_cast<double2*>(ws.get(D_R, (size_t)nb * ld * sizeof(double2)));
    double* dtheta = static_cast<double*>(c.ws(WS_DAV_THETA, (size_t)mmax * sizeof(double) * 2 + 64));
    double2* Cdev = static_cast<double2*>(c.ws(WS_DAV_C, (size_t)mmax * mmax * sizeof(double2)));
    double* dots = static_cast<double*>(c.ws(WS_DAV_DOTS, (size_t)mmax * sizeof(double) + 64));

    // start block: caller's vectors, or the library's own random Hermitian-symmetric ones
    if (phi0_dev)
        PDEP_HIP(hipMemcpyAsync(V, phi0_dev, (size_t)npdep * ld * sizeof(double2), hipMemcpyDeviceToDevice, s));
    {
        const int first = phi0_dev ? npdep : 0;
        if (nb > first) {
            std::vector<double2> h((size_t)(nb - first) * ld, make_double2(0, 0));
            SplitMix64 rng{seed};
            // pair index of -G for every G
            // the sphere is listed lexicographically and is closed under G -> -G, so the
            // partner -G of entry k is entry npw - 1 - k
            std::vector<int> neg(npw);
            for (int k = 0; k < npw; ++k) neg[k] = npw - 1 - k;
            for (int j = 0; j < nb - first; ++j)
                for (int k = 0; k < npw; ++k) {
                    if (k == b.g0) continue;
                    const int kn = neg[k];
                    if (kn < k) continue;         // fill each +-G pair once
                    double a, bb;
                    rng.normal2(a, bb);
                    a *= M_SQRT1_2;
                    bb *= M_SQRT1_2;
                    h[(size_t)j * ld + k] = make_double2(a, bb);
                    h[(size_t)j * ld + kn] = make_double2(a, -bb);
                }
            PDEP_HIP(hipMemcpyAsync(V + (size_t)first * ld, h.data(), h.size() * sizeof(double2),
                                    hipMemcpyHostToDevice, s));
            PDEP_HIP(hipStreamSynchronize(s));
        }
    }
    int m = orthonormalise(c, ws, sv, nullptr, 0, V, nb, ld, true);
    PDEP_REQUIRE(m == nb, PDEP_EINVAL, "start vectors are linearly dependent");
    ApplyStats st;
    // the operator: chi0bar, or the reducible chibar made self-consistent per application
    const double scr_tol = eo.scr_tol > 0.0 ? eo.scr_tol : 0.1 * eo.tol;
    const int scr_maxit = eo.scr_maxit > 0 ? eo.scr_maxit : 200;
    auto apply = [&](int n, const double2* X, double2* AX) {
        if (eo.reducible) {
            const ScreenResult r = chibar_sphere(c, n, X, AX, scr_tol, scr_maxit, st);
            res.scr_passes += r.passes;
            res.scr_notconv += r.n_notconv;
            return (int)r.chi0_columns;
        }
        chi0bar_sphere(c, n, X, AX, st);
        return n;
    };
    res.columns += apply(m, V, AV);
    check_finite_rows(c, ws, AV, m, ld, "chi0bar applied to the start block");
    std::vector<double> theta;
    double maxres = 0.0;
    int it;
    for (it = 1; it <= eo.maxit; ++it) {
        launch_gemm_ahb<double>(m, m, npw, V, ld, AV, ld, Cdev, m, ws.split(), Workspace::kSplitElems, s);
        std::vector<double2> M = d2h(Cdev, (size_t)m * m, s);
        std::vector<double2> Y;
        dense_eig(ws, sv, M, m, true, theta, Y);
        const int k = std::min(nb, m);
        std::vector<double2> C(Y.begin(), Y.begin() + (size_t)k * m);
        combine(c, V, m, k, ld, C, X, Cdev);
        combine(c, AV, m, k, ld, C, AX, Cdev);
        PDEP_HIP(hipMemcpyAsync(dtheta, theta.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
        ritz_residual(k, npw, AX, X, ld, dtheta, R, s);
        launch_row_dots<double>(k, npw, R, ld, R, ld, dots, nullptr, s);
        std::vector<double> r2(k);
        PDEP_HIP(hipMemcpyAsync(r2.data(), dots, k * sizeof(double), hipMemcpyDeviceToHost, s));
        PDEP_HIP(hipStreamSynchronize(s));
        maxres = 0.0;
        std::vector<int> unconv;
        for (int j = 0; j < k; ++j) {
            const double rj = std::sqrt(std::max(r2[j], 0.0));
            if (j < npdep) maxres = std::max(maxres, rj);
            if (rj > eo.tol) unconv.push_back(j);
        }
        if (verbose())
            fprintf(stderr, "[pdep] PDEP it %d: subspace %d, max residual %.2e, lambda_0 %.10f\n", it, m, maxres,
                    theta[0]), fflush(stderr);
        if (maxres <= eo.tol) { res.converged = true; break; }
        if (it == eo.maxit) break;
        int nt = (int)unconv.size();
        if (m + nt > mmax) {
            PDEP_HIP(hipMemcpyAsync(V, X, (size_t)k * ld * sizeof(double2), hipMemcpyDeviceToDevice, s));
            PDEP_HIP(hipMemcpyAsync(AV, AX, (size_t)k * ld * sizeof(double2), hipMemcpyDeviceToDevice, s));
            m = k;
        }
        // never more columns than V and AV hold (only short of 2 nb when N_pw' caps mmax)
        nt = std::min(nt, mmax - m);
        if (nt <= 0) break;
        double2* T = static_cast<double2*>(ws.get(D_T, (size_t)nt * ld * sizeof(double2)));
        for (int j = 0; j < nt; ++j)
            PDEP_HIP(hipMemcpyAsync(T + (size_t)j * ld, R + (size_t)unconv[j] * ld, ld * sizeof(double2),
                                    hipMemcpyDeviceToDevice, s));
        const int kept = orthonormalise(c, ws, sv, V, m, T, nt, ld, true);
        if (kept == 0) break;
        PDEP_HIP(hipMemcpyAsync(V + (size_t)m * ld, T, (size_t)kept * ld * sizeof(double2), hipMemcpyDeviceToDevice, s));
        res.columns += apply(kept, V + (size_t)m * ld, AV + (size_t)m * ld);
        check_finite_rows(c, ws, AV + (size_t)m * ld, kept, ld, "chi0bar applied to the expansion vectors");
        m += kept;
    }
    res.iterations = std::min(it, eo.maxit);
    res.max_residual = maxres;
    res.cg_iter_total = st.cg_iter_total;
    res.n_notconv = st.n_notconv;
    for (int j = 0; j < npdep; ++j) lam_out[j] = theta[j];
    if (basis_out_dev)
        PDEP_HIP(hipMemcpyAsync(basis_out_dev, X, (size_t)npdep * ld * sizeof(double2), hipMemcpyDeviceToDevice, s));
    PDEP_HIP(hipStreamSynchronize(s));
    return res;
}

}  // namespace pdep
