// The body of chi0bar at imaginary and real frequencies in a basis of potentials by
// deflated Lanczos chains (Sec. 2.4: Eqs. MCdef, MCfinal; the body of Eq. finalB, the
// Adler-Wiser form of Eq. AdlerWiser).
//
// With w_jv = P_c Fwd(V_j u_v) (V_j = Re Inv(phi~_j), the Sternheimer right-hand side up
// to sign) and A_v = P_c (H - e_v) P_c on range(P_c):
//   B_ij = -(4/Omega) sum_v <w_iv| g(A_v) |w_jv>,
// g(D) = D / (D^2 + u^2) at the imaginary frequency i u (at u = 0 the static chi0bar of
// the Sternheimer chain) and [1/(D + w - i eta) + 1/(D - w - i eta)] / 2 at the real
// frequency w.  For every (j, v) one Lanczos chain of the deflated Hamiltonian P_c H P_c
// starts at q_1 = w_jv / ||w_jv||; all chains advance together as one block of
// half-sphere FP64 rows (one batched application of H per step, the stick/slab
// transforms and the P_c GEMM pair of the solver).  At every step the overlaps
// <w_iv|q_n> with all basis potentials i of the same band are one GEMM per band and stay
// on the device.  The chain coefficients (T, the overlaps) do not depend on the
// frequency, so every frequency is a sum over the chain (Eq. MCfinal):
//   <w_iv| g(A_v) |w_jv> = ||w_jv|| sum_n <w_iv|q_n> [g(T - e_v)]_n1.
// The paper diagonalises T; here the column [g(T - e_v)]_n1, a combination of
// [(T - s)^-1]_n1 at two complex shifts s, comes from tridiagonal eliminations, one
// thread per chain and frequency (the same numbers, in O(n) instead of O(n^3), and
// without an iterative eigensolver on the nearly degenerate "ghost" eigenvalues that long
// chains in floating point develop), and the sums over (v, n) are one contraction kernel
// per block of frequencies.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "pdep_internal.h"

namespace pdep {

namespace {

enum LzSlot { L_W = WS_LZ_W, L_WW, L_Q, L_QP, L_Z, L_O, L_SC, L_WORK, L_G, L_COEF, L_COL, L_CP, L_DP, L_TRI, L_OUT };

// z -= alpha q + beta qp (rows)
__global__ void k_lz_orth(int K, long ld, const double* __restrict__ alpha, const double* __restrict__ beta,
                          const double2* __restrict__ q, const double2* __restrict__ qp, double2* __restrict__ z) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (k >= K) return;
    const long o = (long)j * ld + k;
    const double a = alpha[j], b = beta[j];
    z[o].x -= a * q[o].x + b * qp[o].x;
    z[o].y -= a * q[o].y + b * qp[o].y;
}

// qp = q; q = z * inv (inv 0 closes the chain: q = 0 from here on)
__global__ void k_lz_next(int K, long ld, const double* __restrict__ inv, const double2* __restrict__ z,
                          double2* __restrict__ q, double2* __restrict__ qp) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (k >= K) return;
    const long o = (long)j * ld + k;
    const double f = inv[j];
    qp[o] = q[o];
    q[o] = make_double2(f * z[o].x, f * z[o].y);
}

dim3 grid_rows(int K, int n) { return dim3((unsigned)((K + 255) / 256), (unsigned)n); }

// g[a * nv + v][k] = [H, r_a] psi_v = -i G_a(k) c_v(k) on the half sphere (a local
// potential: the commutator is -d/dr_a); G: [3][K] Cartesian components
__global__ void k_commutator_rows(int K, int nv, const double* __restrict__ G, const double2* __restrict__ psi,
                                  long ldp, double2* __restrict__ g, long ld) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y, a = row / nv, v = row - a * nv;
    if (k >= K) return;
    const double ga = G[(long)a * K + k];
    const double2 c = psi[(long)v * ldp + k];
    g[(long)row * ld + k] = make_double2(ga * c.y, -ga * c.x);
}

// x[r] *= s
__global__ void k_scale_rows(int K, long ld, double sc, double2* __restrict__ x) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const long o = (long)blockIdx.y * ld + k;
    x[o].x *= sc;
    x[o].y *= sc;
}

__device__ __forceinline__ double2 cmul(double2 p, double2 q) {
    return make_double2(p.x * q.x - p.y * q.y, p.x * q.y + p.y * q.x);
}
__device__ __forceinline__ double2 cdiv(double2 p, double2 q) {
    const double den = q.x * q.x + q.y * q.y;
    return make_double2((p.x * q.x + p.y * q.y) / den, (p.y * q.x - p.x * q.y) / den);
}

// First column y of (T - s)^-1 for a chain's symmetric tridiagonal T (diagonal
// alpha[n * nrow + r], off-diagonal beta[n * nrow + r], length L) and a complex shift s:
// tridiagonal elimination without pivoting, then back substitution.  y, cp: [L] with
// stride nz.  With Im s != 0 every pivot keeps an imaginary part at least |Im s| in
// size (the recursion only adds to it), and with s real below the spectrum of T the
// pivots are positive, so the elimination never divides by zero.
__device__ void tri_column(int L, int nrow, int r, const double* __restrict__ alpha, const double* __restrict__ beta,
                           double2 sh, double2* y, double2* cp, int nz) {
    double2 piv = make_double2(alpha[r] - sh.x, -sh.y);
    cp[0] = L > 1 ? cdiv(make_double2(beta[r], 0.0), piv) : make_double2(0.0, 0.0);
    y[0] = cdiv(make_double2(1.0, 0.0), piv);
    for (int i = 1; i < L; ++i) {
        const double bi = beta[(long)(i - 1) * nrow + r];
        const double2 c1 = cp[(long)(i - 1) * nz];
        piv = make_double2(alpha[(long)i * nrow + r] - sh.x - bi * c1.x, -sh.y - bi * c1.y);
        cp[(long)i * nz] = i + 1 < L ? cdiv(make_double2(beta[(long)i * nrow + r], 0.0), piv) : make_double2(0.0, 0.0);
        const double2 d1 = y[(long)(i - 1) * nz];
        y[(long)i * nz] = cdiv(make_double2(-bi * d1.x, -bi * d1.y), piv);
    }
    for (int i = L - 2; i >= 0; --i) {
        const double2 t = cmul(cp[(long)i * nz], y[(long)(i + 1) * nz]);
        y[(long)i * nz] = make_double2(y[(long)i * nz].x - t.x, y[(long)i * nz].y - t.y);
    }
}

// col[r][n][z] = [ (T_r - e_r - a_z)^-1 + (T_r - e_r - b_z)^-1 ]_{n1} / 2 for every chain
// r (block) and point z (thread); zeros beyond the chain's length.  e_r: the band energy
// of the chain.  For b = conj(a) (imaginary frequencies) the two terms are conjugate and
// the real part of the first is taken.  cp, dp: scratch of the size of col.
__global__ void k_lz_columns(int nrow, int nl, int nz, const double* __restrict__ alpha,
                             const double* __restrict__ beta, const int* __restrict__ len,
                             const double* __restrict__ e_row, const double2* __restrict__ za,
                             const double2* __restrict__ zb, double2* __restrict__ col, double2* __restrict__ cp,
                             double2* __restrict__ dp) {
    const int r = blockIdx.x, z = threadIdx.x;
    if (z >= nz) return;
    const int L = len[r];
    const long base = (long)r * nl * nz + z;
    double2* y = col + base;
    for (int n = L; n < nl; ++n) y[(long)n * nz] = make_double2(0.0, 0.0);
    if (L == 0) return;
    const double2 a = za[z], b = zb[z];
    const bool conj_pair = (b.x == a.x && b.y == -a.y);
    tri_column(L, nrow, r, alpha, beta, make_double2(e_row[r] + a.x, a.y), y, cp + base, nz);
    if (conj_pair) {
        for (int n = 0; n < L; ++n) y[(long)n * nz].y = 0.0;
        return;
    }
    double2* y2 = dp + base;
    tri_column(L, nrow, r, alpha, beta, make_double2(e_row[r] + b.x, b.y), y2, cp + base, nz);
    for (int n = 0; n < L; ++n) {
        const long o = (long)n * nz;
        y[o] = make_double2(0.5 * (y[o].x + y2[o].x), 0.5 * (y[o].y + y2[o].y));
    }
}

constexpr int kZC = 16;   // frequency points per contraction pass

// out[z][i][j] = pref sum_v ||w_jv|| sum_n O[n][v][j][i] col[jv][n][z] for the nz <= kZC
// points of one pass: block (j, 64 values of i), thread i.
__global__ void __launch_bounds__(64) k_lz_contract(int npert, int nv, int nl, int nz, const double2* __restrict__ O,
                                                    const double* __restrict__ wn, const int* __restrict__ len,
                                                    const double2* __restrict__ col, double pref,
                                                    double2* __restrict__ out) {
    const int j = blockIdx.x;
    const int i = blockIdx.y * 64 + threadIdx.x;
    double2 acc[kZC];
#pragma unroll
    for (int z = 0; z < kZC; ++z) acc[z] = make_double2(0.0, 0.0);
    if (i < npert) {
        const size_t oblk = (size_t)npert * npert;
        for (int v = 0; v < nv; ++v) {
            const int r = j * nv + v;
            const int L = len[r];
            const double w = wn[r];
            const double2* cr = col + (size_t)r * nl * nz;
            for (int n = 0; n < L; ++n) {
                const double o = w * O[((size_t)n * nv + v) * oblk + (size_t)j * npert + i].x;
#pragma unroll
                for (int z = 0; z < kZC; ++z)
                    if (z < nz) {
                        const double2 c = cr[(size_t)n * nz + z];
                        acc[z].x += o * c.x;
                        acc[z].y += o * c.y;
                    }
            }
        }
#pragma unroll
        for (int z = 0; z < kZC; ++z)
            if (z < nz)
                out[((size_t)z * npert + i) * npert + j] = make_double2(pref * acc[z].x, pref * acc[z].y);
    }
}

}  // namespace

void run_chains(Ctx& c, int npert_in, const double2* phi, int ndir, int nl, Chains& ch, ApplyStats* dir_st,
                std::vector<double>* coef) {
    const Basis& b = c.basis;
    // start vectors: the npert_in potentials, then ndir (0 or 3) Cartesian directions
    const int npert = npert_in + ndir;
    const int nv = c.nv, nh = half_len(b.npw), nrow = npert * nv;
    const long ld = sphere_ld(b.npw);
    hipStream_t s = c.stream;
    ch = Chains();
    ch.npert = npert;
    ch.nv = nv;
    ch.nl = nl;
    ch.nrow = nrow;
    const size_t vb = (size_t)nrow * ld * sizeof(double2);
    double2* W = static_cast<double2*>(c.ws(L_W, vb));
    double2* Ww = static_cast<double2*>(c.ws(L_WW, vb));
    double2* Q = static_cast<double2*>(c.ws(L_Q, vb));
    double2* Qp = static_cast<double2*>(c.ws(L_QP, vb));
    double2* Z = static_cast<double2*>(c.ws(L_Z, vb));
    const size_t oblk = (size_t)npert * npert;                    // overlaps of one (step, band)
    double2* O = static_cast<double2*>(c.ws(L_O, (size_t)nl * nv * oblk * sizeof(double2)));
    double* sc = static_cast<double*>(c.ws(L_SC, (size_t)4 * nrow * sizeof(double) + 64));
    double *d_a = sc, *d_b = sc + nrow, *d_inv = sc + 2 * nrow, *d_zero = sc + 3 * nrow;
    const size_t split_elems = (size_t)1 << 20;
    double2* work = static_cast<double2*>(c.ws(L_WORK, split_elems * sizeof(double2)));

    rhs_half_rows(c, npert_in, phi, W, ld);
    if (coef) {
        // the coefficients of the projection just done, still in its coefficient buffer
        const long lds = coef_ld(nv);
        const int nr = npert_in * nv;
        std::vector<double2> S((size_t)nr * lds);
        PDEP_HIP(hipMemcpyAsync(S.data(), rhs_coefficients(c), S.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
        PDEP_HIP(hipStreamSynchronize(s));
        coef->assign((size_t)nr * nv, 0.0);
        for (int r = 0; r < nr; ++r)
            for (int m = 0; m < nv; ++m) (*coef)[(size_t)r * nv + m] = S[(size_t)r * lds + m].x;
    }
    if (ndir > 0) {
        // the dipole vectors xi^a_v = P_c r_a psi_v: (H - e_v) xi = P_c [H, r_a] psi_v
        // (Eq. commu), solved like the Sternheimer systems, scaled by sqrt(4 pi) (the
        // Coulomb factor of the head potential) and appended as extra start vectors
        const int nd = ndir * nv;
        std::vector<double> G((size_t)3 * nh);
        for (int k = 0; k < nh; ++k)
            for (int a = 0; a < 3; ++a) G[(size_t)a * nh + k] = 2.0 * M_PI * b.miller[3 * (size_t)k + a] / b.L[a];
        double* d_G = static_cast<double*>(c.ws(L_G, (size_t)3 * nh * sizeof(double) + 64));
        PDEP_HIP(hipMemcpyAsync(d_G, G.data(), G.size() * sizeof(double), hipMemcpyHostToDevice, s));
        double2* gb = Z;                                     // free until the chains start
        double2* xd = W + (size_t)npert_in * nv * ld;
        hipLaunchKernelGGL(k_commutator_rows, grid_rows(nh, nd), dim3(256), 0, s, nh, nv, d_G, c.psi64.as<double2>(),
                           (long)b.npw, gb, ld);
        PDEP_HIP(hipGetLastError());
        project_c<double>(c, gb, ld, nd, static_cast<double2*>(c.ws(L_COEF, coef_bytes(nv, nd) + 64)));
        PDEP_HIP(hipStreamSynchronize(s));
        ApplyStats ds;
        solve_rows(c, nd, gb, xd, ld, ds, nullptr);
        project_c<double>(c, xd, ld, nd, static_cast<double2*>(c.ws(L_COEF, coef_bytes(nv, nd) + 64)));
        hipLaunchKernelGGL(k_scale_rows, grid_rows(nh, nd), dim3(256), 0, s, nh, ld, std::sqrt(4.0 * M_PI), xd);
        PDEP_HIP(hipGetLastError());
        if (dir_st) *dir_st = ds;
    }
    launch_fill_zero(d_zero, sizeof(double), s);
    launch_fill_zero(Qp, vb, s);
    launch_half_weights<double>(nrow, nh, W, ld, Ww, ld, s);
    launch_row_dots<double>(nrow, nh, W, ld, W, ld, d_a, nullptr, s, true);
    std::vector<double> inv(nrow);
    ch.wn.assign(nrow, 0.0);
    ch.alpha.assign((size_t)nl * nrow, 0.0);
    ch.beta.assign((size_t)nl * nrow, 0.0);
    PDEP_HIP(hipMemcpyAsync(ch.wn.data(), d_a, nrow * sizeof(double), hipMemcpyDeviceToHost, s));
    PDEP_HIP(hipStreamSynchronize(s));
    ch.len.assign(nrow, 0);                  // chain length (0: the start vector is zero)
    for (int r = 0; r < nrow; ++r) {
        ch.wn[r] = std::sqrt(std::max(ch.wn[r], 0.0));
        inv[r] = ch.wn[r] > 0.0 ? 1.0 / ch.wn[r] : 0.0;
        ch.len[r] = ch.wn[r] > 0.0 ? nl : 0;
    }
    PDEP_HIP(hipMemcpyAsync(d_inv, inv.data(), nrow * sizeof(double), hipMemcpyHostToDevice, s));
    launch_convert_rows<double, double>(nrow, nh, W, ld, nullptr, d_inv, Q, ld, s);   // q_1 = w / ||w||
    std::vector<double> bprev(nrow, 0.0);
    for (int n = 0; n < nl; ++n) {
        apply_deflated_h64(c, Q, Z, ld, nrow, d_zero);
        ++ch.h_applications;
        for (int v = 0; v < nv; ++v)      // <w_iv | q_jv> for every i, j of band v
            launch_gemm_ahb<double>(npert, npert, nh, Ww + (long)v * ld, (long)nv * ld, Q + (long)v * ld,
                                    (long)nv * ld, O + ((size_t)n * nv + v) * oblk, npert, work, split_elems, s, true);
        launch_row_dots<double>(nrow, nh, Q, ld, Z, ld, d_a, nullptr, s, true);   // alpha_n = <q_n, H~ q_n>
        PDEP_HIP(hipMemcpyAsync(ch.alpha.data() + (size_t)n * nrow, d_a, nrow * sizeof(double), hipMemcpyDeviceToHost,
                                s));
        if (n == nl - 1) break;
        PDEP_HIP(hipMemcpyAsync(d_b, bprev.data(), nrow * sizeof(double), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_lz_orth, grid_rows(nh, nrow), dim3(256), 0, s, nh, ld, d_a, d_b, Q, Qp, Z);
        PDEP_HIP(hipGetLastError());
        launch_row_dots<double>(nrow, nh, Z, ld, Z, ld, d_b, nullptr, s, true);  // beta_{n+1}^2
        std::vector<double> b2(nrow);
        PDEP_HIP(hipMemcpyAsync(b2.data(), d_b, nrow * sizeof(double), hipMemcpyDeviceToHost, s));
        PDEP_HIP(hipStreamSynchronize(s));
        for (int r = 0; r < nrow; ++r) {
            const double bn = std::sqrt(std::max(b2[r], 0.0));
            const double an = ch.alpha[(size_t)n * nrow + r];
            if (ch.len[r] > n + 1 && bn > 1e-14 * std::abs(an) + 1e-300) {
                ch.beta[(size_t)n * nrow + r] = bn;
                bprev[r] = bn;
                inv[r] = 1.0 / bn;
            } else {                          // the chain closed: an invariant subspace
                ch.len[r] = std::min(ch.len[r], n + 1);
                bprev[r] = 0.0;
                inv[r] = 0.0;
            }
        }
        PDEP_HIP(hipMemcpyAsync(d_inv, inv.data(), nrow * sizeof(double), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_lz_next, grid_rows(nh, nrow), dim3(256), 0, s, nh, ld, d_inv, Z, Q, Qp);
        PDEP_HIP(hipGetLastError());
    }
    PDEP_HIP(hipStreamSynchronize(s));
    for (int r = 0; r < nrow; ++r)
        if (ch.len[r] > 0) {
            ++ch.chains;
            ch.max_length = std::max(ch.max_length, ch.len[r]);
        }
    ch.O = O;
}

void chain_body(Ctx& c, const Chains& ch, int nz, const FreqPoint* zp, double2* out) {
    if (nz <= 0) return;
    hipStream_t s = c.stream;
    const int nrow = ch.nrow, nl = ch.nl, np = ch.npert, nv = ch.nv;
    PDEP_REQUIRE(np <= 65535, PDEP_EINVAL, "too many basis potentials for one contraction");
    const int zc = std::min(nz, kZC);
    const size_t colb = (size_t)nrow * nl * zc * sizeof(double2);
    double2* col = static_cast<double2*>(c.ws(L_COL, colb));
    double2* cp = static_cast<double2*>(c.ws(L_CP, colb));
    double2* dp = static_cast<double2*>(c.ws(L_DP, colb));
    const size_t oblk = (size_t)np * np;
    double2* d_out = static_cast<double2*>(c.ws(L_OUT, (size_t)zc * oblk * sizeof(double2)));
    // chain tables: alpha, beta [nl][nrow], length, norm and band energy per row, points
    const size_t tri_b = (size_t)2 * nl * nrow * sizeof(double) + (size_t)nrow * (sizeof(int) + 2 * sizeof(double)) +
                         (size_t)2 * kZC * sizeof(double2) + 256;
    char* tri = static_cast<char*>(c.ws(L_TRI, tri_b));
    double* d_alpha = reinterpret_cast<double*>(tri);
    double* d_beta = d_alpha + (size_t)nl * nrow;
    double* d_wn = d_beta + (size_t)nl * nrow;
    double* d_e = d_wn + nrow;
    double2* d_za = reinterpret_cast<double2*>(d_e + nrow);
    double2* d_zb = d_za + kZC;
    int* d_len = reinterpret_cast<int*>(d_zb + kZC);
    std::vector<double> e_row(nrow);
    for (int r = 0; r < nrow; ++r) e_row[r] = c.eps[r % nv];
    PDEP_HIP(hipMemcpyAsync(d_alpha, ch.alpha.data(), ch.alpha.size() * sizeof(double), hipMemcpyHostToDevice, s));
    PDEP_HIP(hipMemcpyAsync(d_beta, ch.beta.data(), ch.beta.size() * sizeof(double), hipMemcpyHostToDevice, s));
    PDEP_HIP(hipMemcpyAsync(d_wn, ch.wn.data(), nrow * sizeof(double), hipMemcpyHostToDevice, s));
    PDEP_HIP(hipMemcpyAsync(d_e, e_row.data(), nrow * sizeof(double), hipMemcpyHostToDevice, s));
    PDEP_HIP(hipMemcpyAsync(d_len, ch.len.data(), nrow * sizeof(int), hipMemcpyHostToDevice, s));
    const double pref = -4.0 / c.basis.omega;
    for (int z0 = 0; z0 < nz; z0 += kZC) {
        const int n = std::min(kZC, nz - z0);
        std::vector<double2> a(n), bb(n);
        for (int k = 0; k < n; ++k) {
            a[k] = zp[z0 + k].a;
            bb[k] = zp[z0 + k].b;
        }
        PDEP_HIP(hipMemcpyAsync(d_za, a.data(), n * sizeof(double2), hipMemcpyHostToDevice, s));
        PDEP_HIP(hipMemcpyAsync(d_zb, bb.data(), n * sizeof(double2), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_lz_columns, dim3((unsigned)nrow), dim3(64), 0, s, nrow, nl, n, d_alpha, d_beta, d_len,
                           d_e, d_za, d_zb, col, cp, dp);
        PDEP_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_lz_contract, dim3((unsigned)np, (unsigned)((np + 63) / 64)), dim3(64), 0, s, np, nv, nl, n,
                           ch.O, d_wn, d_len, col, pref, d_out);
        PDEP_HIP(hipGetLastError());
        PDEP_HIP(hipMemcpyAsync(out + (size_t)z0 * oblk, d_out, (size_t)n * oblk * sizeof(double2),
                                hipMemcpyDeviceToHost, s));
    }
    PDEP_HIP(hipStreamSynchronize(s));
}

LanczosResult body_lanczos(Ctx& c, int npert_in, const double2* phi, int ndir, int nl, int nfreq, const double* u,
                           double* body, ApplyStats* dir_st) {
    Chains ch;
    run_chains(c, npert_in, phi, ndir, nl, ch, dir_st, nullptr);
    std::vector<FreqPoint> zp(nfreq);
    for (int f = 0; f < nfreq; ++f) zp[f] = FreqPoint{make_double2(0.0, u[f]), make_double2(0.0, -u[f])};
    const size_t oblk = (size_t)ch.npert * ch.npert;
    std::vector<double2> out((size_t)nfreq * oblk);
    chain_body(c, ch, nfreq, zp.data(), out.data());
    for (size_t k = 0; k < out.size(); ++k) body[k] = out[k].x;
    LanczosResult res;
    res.chains = ch.chains;
    res.max_length = ch.max_length;
    res.h_applications = ch.h_applications;
    return res;
}

// Gauss-Legendre nodes and weights on [-1, 1]: Newton iteration on the roots of P_n
// from the Chebyshev guesses, P_n by its three-term recurrence.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::abs(dz) < 1e-16) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

namespace {

// In-place inverse of the n x n row-major matrix A (Gauss-Jordan, partial pivoting);
// S is double or std::complex<double>.
template <typename S>
void invert(int n, std::vector<S>& A) {
    std::vector<S> I((size_t)n * n, S(0.0));
    for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = S(1.0);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::abs(A[(size_t)r * n + col]) > std::abs(A[(size_t)piv * n + col])) piv = r;
        PDEP_REQUIRE(std::abs(A[(size_t)piv * n + col]) != 0.0, PDEP_EDEVICE, "1 - B is singular");
        if (piv != col)
            for (int j = 0; j < n; ++j) {
                std::swap(A[(size_t)piv * n + j], A[(size_t)col * n + j]);
                std::swap(I[(size_t)piv * n + j], I[(size_t)col * n + j]);
            }
        const S d = S(1.0) / A[(size_t)col * n + col];
        for (int j = 0; j < n; ++j) {
            A[(size_t)col * n + j] *= d;
            I[(size_t)col * n + j] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const S f = A[(size_t)r * n + col];
            if (f == S(0.0)) continue;
            for (int j = 0; j < n; ++j) {
                A[(size_t)r * n + j] -= f * A[(size_t)col * n + j];
                I[(size_t)r * n + j] -= f * I[(size_t)col * n + j];
            }
        }
    }
    A.swap(I);
}

// Eq. Bfinal from the extended matrix e(i, j) of the np potentials and three directions
// (directions last).  The products keep the order of the formula, so the complex
// symmetric case (real frequencies) needs no conjugation: mu_ij = 1/3 sum_a U_ia U_aj.
template <typename S, typename Get>
void bfinal_t(int np, Get e, const double L[3], S* Lam, S* Xi) {
    // M = (1 - B)^-1, mu_ij = 1/3 sum_a U_ia U_aj (U_ia from the chains of the
    // directions, U_aj from those of the potentials), f = Tr F / 3
    std::vector<S> M((size_t)np * np), mu((size_t)np * np, S(0.0));
    for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) {
            M[(size_t)i * np + j] = (i == j ? S(1.0) : S(0.0)) - e(i, j);
            S acc(0.0);
            for (int a = 0; a < 3; ++a) acc += e(i, np + a) * e(np + a, j);
            mu[(size_t)i * np + j] = acc / 3.0;
        }
    invert(np, M);
    const S f = (e(np, np) + e(np + 1, np + 1) + e(np + 2, np + 2)) / 3.0;
    S tr(0.0);
    for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) tr += mu[(size_t)i * np + j] * M[(size_t)j * np + i];
    const S k = S(1.0) - f - tr;
    if (Xi) *Xi = (S(1.0) - k) / k * bz_coulomb_integral(L);
    if (!Lam) return;
    // Lambda = M B + M mu M / k
    std::vector<S> MB((size_t)np * np, S(0.0)), Mmu((size_t)np * np, S(0.0));
    for (int i = 0; i < np; ++i)
        for (int l = 0; l < np; ++l) {
            const S m = M[(size_t)i * np + l];
            for (int j = 0; j < np; ++j) {
                MB[(size_t)i * np + j] += m * e(l, j);
                Mmu[(size_t)i * np + j] += m * mu[(size_t)l * np + j];
            }
        }
    for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) {
            S acc(0.0);
            for (int l = 0; l < np; ++l) acc += Mmu[(size_t)i * np + l] * M[(size_t)l * np + j];
            Lam[(size_t)i * np + j] = MB[(size_t)i * np + j] + acc / k;
        }
}

}  // namespace

double bz_coulomb_integral(const double L[3]) {
    // the box |q_a| <= h_a is six pyramids over its faces; on the face q_a = h_a the
    // radial integral of q^2 / q^2 leaves h_a times the integral of 1 / (1 + s^2 + t^2)
    // over |s| <= h_b / h_a, |t| <= h_c / h_a, whose t integral is closed:
    // 2 atan(t_max / sqrt(1 + s^2)) / sqrt(1 + s^2)
    std::vector<double> x, w;
    gauss_legendre(64, x, w);
    const double h[3] = {M_PI / L[0], M_PI / L[1], M_PI / L[2]};
    double total = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double sb = h[(a + 1) % 3] / h[a], sc = h[(a + 2) % 3] / h[a];
        double val = 0.0;
        for (int i = 0; i < 64; ++i) {
            const double s = sb * x[i], r = std::sqrt(1.0 + s * s);
            val += sb * w[i] * 2.0 * std::atan(sc / r) / r;
        }
        total += 2.0 * h[a] * val;
    }
    return total * 4.0 * M_PI / (8.0 * M_PI * M_PI * M_PI);
}

void bfinal(int np, const double* E, const double L[3], double* F, double* U, double* B, double* Lam, double* Xi) {
    const int nb = np + 3;
    auto e = [&](int i, int j) { return E[(size_t)i * nb + j]; };
    if (F)
        for (int a = 0; a < 3; ++a)
            for (int bb = 0; bb < 3; ++bb) F[a * 3 + bb] = e(np + a, np + bb);
    if (U)
        for (int a = 0; a < 3; ++a)
            for (int j = 0; j < np; ++j) U[(size_t)a * np + j] = e(np + a, j);
    if (B)
        for (int i = 0; i < np; ++i)
            for (int j = 0; j < np; ++j) B[(size_t)i * np + j] = e(i, j);
    if (!Lam && !Xi) return;
    bfinal_t<double>(np, e, L, Lam, Xi);
}

void bfinal_complex(int np, const double2* E, const double L[3], double2* Lam, double2* Xi) {
    using C = std::complex<double>;
    const int nb = np + 3;
    auto e = [&](int i, int j) {
        const double2 v = E[(size_t)i * nb + j];
        return C(v.x, v.y);
    };
    std::vector<C> lam(Lam ? (size_t)np * np : 0);
    C xi;
    bfinal_t<C>(np, e, L, Lam ? lam.data() : nullptr, Xi ? &xi : nullptr);
    if (Xi) *Xi = make_double2(xi.real(), xi.imag());
    if (Lam)
        for (size_t k = 0; k < lam.size(); ++k) Lam[k] = make_double2(lam[k].real(), lam[k].imag());
}

}  // namespace pdep
