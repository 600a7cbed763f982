// The reducible polarizability in the RPA: chibar = (1 - chi0bar)^-1 chi0bar
// (Eq. linearalgebrachichi0), applied to blocks of potentials on S' by making the
// Sternheimer response self-consistent with the Hartree potential of the density it
// induces (the Hartree term of Eq. LF, Eq. LFHartree; Fig. pdepscheme, right panel).
//
// In the symmetrised variables of the chi0bar chain (phi~ = sqrt(4 pi)/|G| phi, the
// output sqrt(4 pi)/|G| dn), the Hartree potential of the response dn to the total
// perturbation is dV_H(G) = 4 pi dn(G)/|G|^2 = sqrt(4 pi)/|G| x(G) with x the chain's
// output, so the self-consistent response x satisfies x = chi0bar (phi + x), i.e.
// (1 - chi0bar) y = phi with x = y - phi.  1 - chi0bar is Hermitian with eigenvalues
// 1 - lambda_i >= 1 (chi0bar is negative semidefinite), so the self-consistency is
// reached by conjugate gradients on y: every pass applies chi0bar (all Sternheimer
// solves of the block for the current direction) and the passes are Krylov-mixed
// instead of linearly mixed, which converges in about sqrt(eps_max) times fewer passes
// to the same fixed point.  Columns whose residual reaches tol ||phi|| leave the block.
#include <algorithm>
#include <cmath>
#include <vector>

#include "pdep_internal.h"

namespace pdep {

namespace {

enum ScrSlot { S_Y = WS_SCR_Y, S_R, S_P, S_C, S_T, S_ROWS, S_DOTS };

// Ra -= alpha (Pa - Ca)   (the residual update with (1 - chi0bar) Pa = Pa - Ca)
__global__ void k_scr_residual(int K, long ld, const double* __restrict__ alpha, const double2* __restrict__ p,
                               const double2* __restrict__ cp, double2* __restrict__ r) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (k >= K) return;
    const long o = (long)j * ld + k;
    const double a = alpha[j];
    r[o].x -= a * (p[o].x - cp[o].x);
    r[o].y -= a * (p[o].y - cp[o].y);
}

// Pa = Ra + beta Pa
__global__ void k_scr_direction(int K, long ld, const double* __restrict__ beta, const double2* __restrict__ r,
                                double2* __restrict__ p) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (k >= K) return;
    const long o = (long)j * ld + k;
    const double b = beta[j];
    p[o] = make_double2(r[o].x + b * p[o].x, r[o].y + b * p[o].y);
}

// out = y - phi
__global__ void k_scr_finish(int K, long ld, const double2* __restrict__ y, const double2* __restrict__ phi,
                             double2* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (k >= K) return;
    const long o = (long)j * ld + k;
    out[o] = make_double2(y[o].x - phi[o].x, y[o].y - phi[o].y);
}

dim3 grid_rows(int K, int n) { return dim3((unsigned)((K + 255) / 256), (unsigned)n); }

}  // namespace

ScreenResult chibar_sphere(Ctx& c, int n, const double2* phi, double2* out, double tol, int maxit,
                           ApplyStats& st) {
    ScreenResult res;
    if (n <= 0) return res;
    const int npw = c.basis.npw;
    const long ld = sphere_ld(npw);
    hipStream_t s = c.stream;
    const size_t vb = (size_t)n * ld * sizeof(double2);
    double2* Y = static_cast<double2*>(c.ws(S_Y, vb));
    double2* Ra = static_cast<double2*>(c.ws(S_R, vb));
    double2* Pa = static_cast<double2*>(c.ws(S_P, vb));
    double2* Ca = static_cast<double2*>(c.ws(S_C, vb));
    double2* T = static_cast<double2*>(c.ws(S_T, vb));
    char* rb = static_cast<char*>(c.ws(S_ROWS, (size_t)n * (sizeof(int) + 2 * sizeof(double)) + 64));
    double* d_coef = reinterpret_cast<double*>(rb);
    int* d_rows = reinterpret_cast<int*>(d_coef + n);
    double* dots = static_cast<double*>(c.ws(S_DOTS, (size_t)2 * n * sizeof(double) + 64));

    // y = 0, r = phi, p = r
    launch_fill_zero(Y, vb, s);
    PDEP_HIP(hipMemcpyAsync(Ra, phi, vb, hipMemcpyDeviceToDevice, s));
    PDEP_HIP(hipMemcpyAsync(Pa, phi, vb, hipMemcpyDeviceToDevice, s));
    launch_row_dots<double>(n, npw, phi, ld, phi, ld, dots, nullptr, s);
    std::vector<double> bb(n), rr(n), pcp(n), pp(n), coef(n);
    PDEP_HIP(hipMemcpyAsync(bb.data(), dots, n * sizeof(double), hipMemcpyDeviceToHost, s));
    PDEP_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < n; ++j) PDEP_REQUIRE(std::isfinite(bb[j]), PDEP_EINVAL, "non-finite potential");
    std::vector<int> act;                      // original column of each active slot
    for (int j = 0; j < n; ++j) {
        rr[j] = bb[j];
        if (bb[j] > 0.0) act.push_back(j);
    }
    // active slots are kept compact: slot k of Ra / Pa belongs to column act[k]
    if ((int)act.size() < n && !act.empty()) {
        PDEP_HIP(hipMemcpyAsync(d_rows, act.data(), act.size() * sizeof(int), hipMemcpyHostToDevice, s));
        launch_convert_rows<double, double>((int)act.size(), npw, phi, ld, d_rows, nullptr, Ra, ld, s);
        PDEP_HIP(hipMemcpyAsync(Pa, Ra, act.size() * ld * sizeof(double2), hipMemcpyDeviceToDevice, s));
    }
    std::vector<double> rs;                    // ||r||^2 per active slot
    for (int j : act) rs.push_back(bb[j]);
    int pass = 0;
    while (!act.empty() && pass < maxit) {
        ++pass;
        const int na = (int)act.size();
        // C = chi0bar P: the Sternheimer solves of every active column for its direction
        chi0bar_sphere(c, na, Pa, Ca, st);
        res.chi0_columns += na;
        launch_row_dots<double>(na, npw, Pa, ld, Ca, ld, dots, dots + n, s);
        PDEP_HIP(hipMemcpyAsync(pcp.data(), dots, na * sizeof(double), hipMemcpyDeviceToHost, s));
        PDEP_HIP(hipMemcpyAsync(pp.data(), dots + n, na * sizeof(double), hipMemcpyDeviceToHost, s));
        PDEP_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < na; ++k) {
            const double pap = pp[k] - pcp[k];           // <p, (1 - chi0bar) p> >= ||p||^2
            PDEP_REQUIRE(pap > 0.0 && std::isfinite(pap), PDEP_EDEVICE,
                         "chibar: <p, (1 - chi0bar) p> is not positive (column " + std::to_string(act[k]) + ")");
            coef[k] = rs[k] / pap;
        }
        PDEP_HIP(hipMemcpyAsync(d_coef, coef.data(), na * sizeof(double), hipMemcpyHostToDevice, s));
        PDEP_HIP(hipMemcpyAsync(d_rows, act.data(), na * sizeof(int), hipMemcpyHostToDevice, s));
        launch_axpy_rows<double>(na, npw, Pa, ld, d_rows, d_coef, Y, ld, s);   // y += alpha p
        hipLaunchKernelGGL(k_scr_residual, grid_rows(npw, na), dim3(256), 0, s, npw, ld, d_coef, Pa, Ca, Ra);
        PDEP_HIP(hipGetLastError());
        launch_row_dots<double>(na, npw, Ra, ld, Ra, ld, dots, nullptr, s);
        std::vector<double> rn(na);
        PDEP_HIP(hipMemcpyAsync(rn.data(), dots, na * sizeof(double), hipMemcpyDeviceToHost, s));
        PDEP_HIP(hipStreamSynchronize(s));
        // beta and the columns that stay
        std::vector<int> keep, keep_col;
        std::vector<double> beta, rs_next;
        for (int k = 0; k < na; ++k) {
            const int j = act[k];
            rr[j] = rn[k];
            if (rn[k] > tol * tol * bb[j]) {
                keep.push_back(k);
                keep_col.push_back(j);
                beta.push_back(rn[k] / rs[k]);
                rs_next.push_back(rn[k]);
            }
        }
        const int nk = (int)keep.size();
        if (nk == 0) { act.clear(); break; }
        PDEP_HIP(hipMemcpyAsync(d_coef, beta.data(), nk * sizeof(double), hipMemcpyHostToDevice, s));
        if (nk < na) {
            // compact the slots of the columns that stay (gather through T)
            PDEP_HIP(hipMemcpyAsync(d_rows, keep.data(), nk * sizeof(int), hipMemcpyHostToDevice, s));
            launch_convert_rows<double, double>(nk, npw, Ra, ld, d_rows, nullptr, T, ld, s);
            PDEP_HIP(hipMemcpyAsync(Ra, T, nk * ld * sizeof(double2), hipMemcpyDeviceToDevice, s));
            launch_convert_rows<double, double>(nk, npw, Pa, ld, d_rows, nullptr, T, ld, s);
            PDEP_HIP(hipMemcpyAsync(Pa, T, nk * ld * sizeof(double2), hipMemcpyDeviceToDevice, s));
        }
        hipLaunchKernelGGL(k_scr_direction, grid_rows(npw, nk), dim3(256), 0, s, npw, ld, d_coef, Ra, Pa);
        PDEP_HIP(hipGetLastError());
        PDEP_HIP(hipStreamSynchronize(s));   // host vectors above are reused next pass
        act = keep_col;
        rs = rs_next;
    }
    hipLaunchKernelGGL(k_scr_finish, grid_rows(npw, n), dim3(256), 0, s, npw, ld, Y, phi, out);
    PDEP_HIP(hipGetLastError());
    PDEP_HIP(hipStreamSynchronize(s));
    res.passes = pass;
    res.n_notconv = (int)act.size();
    for (int j = 0; j < n; ++j)
        if (bb[j] > 0.0) res.max_rel_residual = std::max(res.max_rel_residual, std::sqrt(rr[j] / bb[j]));
    return res;
}

}  // namespace pdep
