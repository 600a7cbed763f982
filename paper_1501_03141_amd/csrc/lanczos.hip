// The body of chi0bar at imaginary frequencies in a basis of potentials by deflated
// Lanczos chains (Sec. 2.4: Eqs. MCdef, MCfinal; the body of Eq. finalB, the
// Adler-Wiser form of Eq. AdlerWiser at omega = i u).
//
// With w_jv = P_c Fwd(V_j u_v) (V_j = Re Inv(phi~_j), the Sternheimer right-hand side up
// to sign) and A_v = P_c (H - e_v) P_c on range(P_c):
//   B_ij(iu) = -(4/Omega) sum_v Re <w_iv| A_v (A_v^2 + u^2)^-1 |w_jv>,
// which at u = 0 is the static chi0bar of the Sternheimer chain.  For every (j, v) one
// Lanczos chain of the deflated Hamiltonian P_c H P_c starts at q_1 = w_jv / ||w_jv||;
// all chains advance together as one block of half-sphere FP64 rows (one batched
// application of H per step, the stick/slab transforms and the P_c GEMM pair of the
// solver).  At every step the overlaps <w_iv|q_n> with all basis potentials i of the
// same band are one GEMM per band.  The chain coefficients (T, the overlaps) do not
// depend on u, so every frequency is a sum over the chain (Eq. MCfinal):
//   <w_iv| f(A_v) |w_jv> = ||w_jv|| sum_{n,k} <w_iv|q_n> U_nk f(d_k - e_v) U_1k,
// f(x) = x / (x^2 + u^2), T = U D U^t.  The paper diagonalises T; here the column
// sum_k U_nk f(d_k - e_v) U_1k = Re [(T - e_v - i u)^-1]_n1 comes from one tridiagonal
// elimination per chain and frequency (the same number, in O(n) instead of O(n^3), and
// without an iterative eigensolver on the nearly degenerate "ghost" eigenvalues that
// long chains in floating point develop).
#include <algorithm>
#include <cmath>
#include <vector>

#include "pdep_internal.h"

namespace pdep {

namespace {

enum LzSlot { L_W = WS_LZ_W, L_WW, L_Q, L_QP, L_Z, L_O, L_SC, L_WORK, L_G, L_COEF };

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

// x = Re y with (T - z) y = e_1 for the symmetric tridiagonal T (diagonal a[0..n),
// off-diagonal b[0..n-1)) and z = e + i u: the first column of
// (T - e) ((T - e)^2 + u^2)^-1, i.e. sum_k U_nk f(d_k - e) U_1k for T = U diag(d) U^t.
// Tridiagonal elimination without pivoting: T - e is positive definite for e below the
// spectrum of the deflated Hamiltonian (an occupied energy), so T - e - i u has a positive
// definite Hermitian part and the elimination is stable.
void resolvent_column(int n, const double* a, const double* b, double e, double u, std::vector<double2>& w,
                      double* x) {
    w.resize(2 * (size_t)n);
    double2* cp = w.data();          // modified super-diagonal
    double2* dp = w.data() + n;      // modified right-hand side
    auto cdiv = [](double2 p, double2 q) {
        const double den = q.x * q.x + q.y * q.y;
        return make_double2((p.x * q.x + p.y * q.y) / den, (p.y * q.x - p.x * q.y) / den);
    };
    double2 piv = make_double2(a[0] - e, -u);
    cp[0] = n > 1 ? cdiv(make_double2(b[0], 0.0), piv) : make_double2(0.0, 0.0);
    dp[0] = cdiv(make_double2(1.0, 0.0), piv);
    for (int i = 1; i < n; ++i) {
        const double bi = b[i - 1];
        piv = make_double2(a[i] - e - bi * cp[i - 1].x, -u - bi * cp[i - 1].y);
        cp[i] = i + 1 < n ? cdiv(make_double2(b[i], 0.0), piv) : make_double2(0.0, 0.0);
        dp[i] = cdiv(make_double2(-bi * dp[i - 1].x, -bi * dp[i - 1].y), piv);
    }
    double2 y = dp[n - 1];
    x[n - 1] = y.x;
    for (int i = n - 2; i >= 0; --i) {
        y = make_double2(dp[i].x - (cp[i].x * y.x - cp[i].y * y.y), dp[i].y - (cp[i].x * y.y + cp[i].y * y.x));
        x[i] = y.x;
    }
}

}  // namespace

LanczosResult body_lanczos(Ctx& c, int npert_in, const double2* phi, int ndir, int nl, int nfreq, const double* u,
                           double* body, ApplyStats* dir_st) {
    LanczosResult res;
    const Basis& b = c.basis;
    // start vectors: the npert_in potentials, then ndir (0 or 3) Cartesian directions
    const int npert = npert_in + ndir;
    const int nv = c.nv, nh = half_len(b.npw), nrow = npert * nv;
    const long ld = sphere_ld(b.npw);
    hipStream_t s = c.stream;
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
    std::vector<double> wn(nrow), inv(nrow), alpha((size_t)nl * nrow, 0.0), beta((size_t)nl * nrow, 0.0);
    PDEP_HIP(hipMemcpyAsync(wn.data(), d_a, nrow * sizeof(double), hipMemcpyDeviceToHost, s));
    PDEP_HIP(hipStreamSynchronize(s));
    std::vector<int> len(nrow, 0);           // chain length (0: the start vector is zero)
    for (int r = 0; r < nrow; ++r) {
        wn[r] = std::sqrt(std::max(wn[r], 0.0));
        inv[r] = wn[r] > 0.0 ? 1.0 / wn[r] : 0.0;
        len[r] = wn[r] > 0.0 ? nl : 0;
    }
    PDEP_HIP(hipMemcpyAsync(d_inv, inv.data(), nrow * sizeof(double), hipMemcpyHostToDevice, s));
    launch_convert_rows<double, double>(nrow, nh, W, ld, nullptr, d_inv, Q, ld, s);   // q_1 = w / ||w||
    std::vector<double> bprev(nrow, 0.0);
    for (int n = 0; n < nl; ++n) {
        apply_deflated_h64(c, Q, Z, ld, nrow, d_zero);
        ++res.h_applications;
        for (int v = 0; v < nv; ++v)      // <w_iv | q_jv> for every i, j of band v
            launch_gemm_ahb<double>(npert, npert, nh, Ww + (long)v * ld, (long)nv * ld, Q + (long)v * ld,
                                    (long)nv * ld, O + ((size_t)n * nv + v) * oblk, npert, work, split_elems, s, true);
        launch_row_dots<double>(nrow, nh, Q, ld, Z, ld, d_a, nullptr, s, true);   // alpha_n = <q_n, H~ q_n>
        PDEP_HIP(hipMemcpyAsync(alpha.data() + (size_t)n * nrow, d_a, nrow * sizeof(double), hipMemcpyDeviceToHost, s));
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
            const double an = alpha[(size_t)n * nrow + r];
            if (len[r] > n + 1 && bn > 1e-14 * std::abs(an) + 1e-300) {
                beta[(size_t)n * nrow + r] = bn;
                bprev[r] = bn;
                inv[r] = 1.0 / bn;
            } else {                          // the chain closed: an invariant subspace
                len[r] = std::min(len[r], n + 1);
                bprev[r] = 0.0;
                inv[r] = 0.0;
            }
        }
        PDEP_HIP(hipMemcpyAsync(d_inv, inv.data(), nrow * sizeof(double), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_lz_next, grid_rows(nh, nrow), dim3(256), 0, s, nh, ld, d_inv, Z, Q, Qp);
        PDEP_HIP(hipGetLastError());
    }
    std::vector<double2> Oh((size_t)nl * nv * oblk);
    PDEP_HIP(hipMemcpyAsync(Oh.data(), O, Oh.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
    PDEP_HIP(hipStreamSynchronize(s));

    // every frequency from the chains: B[f][i][j] = -(4/Omega) sum_v ||w_jv|| sum_n <w_iv|q_n> c_n
    std::fill(body, body + (size_t)nfreq * oblk, 0.0);
    const double pref = -4.0 / b.omega;
    std::vector<double> cf((size_t)nfreq * nl), xcol(nl), ta(nl), tb(nl);
    std::vector<double2> wsp;
    for (int v = 0; v < nv; ++v)
        for (int j = 0; j < npert; ++j) {
            const int r = j * nv + v, L = len[r];
            if (L == 0) continue;
            ++res.chains;
            res.max_length = std::max(res.max_length, L);
            for (int n = 0; n < L; ++n) {
                ta[n] = alpha[(size_t)n * nrow + r];
                tb[n] = n + 1 < L ? beta[(size_t)n * nrow + r] : 0.0;
            }
            for (int f = 0; f < nfreq; ++f) {
                resolvent_column(L, ta.data(), tb.data(), c.eps[v], u[f], wsp, xcol.data());
                for (int n = 0; n < L; ++n) cf[(size_t)f * nl + n] = pref * wn[r] * xcol[n];
            }
            for (int n = 0; n < L; ++n) {
                const double2* ov = Oh.data() + ((size_t)n * nv + v) * oblk + (size_t)j * npert;   // <w_iv|q_jv>
                for (int f = 0; f < nfreq; ++f) {
                    const double cn = cf[(size_t)f * nl + n];
                    double* bf = body + (size_t)f * oblk;
                    for (int i = 0; i < npert; ++i) bf[(size_t)i * npert + j] += ov[i].x * cn;
                }
            }
        }
    return res;
}

namespace {

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

// In-place inverse of the n x n row-major matrix A (Gauss-Jordan, partial pivoting).
void invert(int n, std::vector<double>& A) {
    std::vector<double> I((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::abs(A[(size_t)r * n + col]) > std::abs(A[(size_t)piv * n + col])) piv = r;
        PDEP_REQUIRE(A[(size_t)piv * n + col] != 0.0, PDEP_EDEVICE, "1 - B is singular");
        if (piv != col)
            for (int j = 0; j < n; ++j) {
                std::swap(A[(size_t)piv * n + j], A[(size_t)col * n + j]);
                std::swap(I[(size_t)piv * n + j], I[(size_t)col * n + j]);
            }
        const double d = 1.0 / A[(size_t)col * n + col];
        for (int j = 0; j < n; ++j) {
            A[(size_t)col * n + j] *= d;
            I[(size_t)col * n + j] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const double f = A[(size_t)r * n + col];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) {
                A[(size_t)r * n + j] -= f * A[(size_t)col * n + j];
                I[(size_t)r * n + j] -= f * I[(size_t)col * n + j];
            }
        }
    }
    A.swap(I);
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
    // M = (1 - B)^-1, mu_ij = 1/3 sum_a U_ia U_aj (U_ia from the chains of the
    // directions, U_aj from those of the potentials), f = Tr F / 3
    std::vector<double> M((size_t)np * np), mu((size_t)np * np, 0.0);
    for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) {
            M[(size_t)i * np + j] = (i == j ? 1.0 : 0.0) - e(i, j);
            double acc = 0.0;
            for (int a = 0; a < 3; ++a) acc += e(i, np + a) * e(np + a, j);
            mu[(size_t)i * np + j] = acc / 3.0;
        }
    invert(np, M);
    const double f = (e(np, np) + e(np + 1, np + 1) + e(np + 2, np + 2)) / 3.0;
    double tr = 0.0;
    for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) tr += mu[(size_t)i * np + j] * M[(size_t)j * np + i];
    const double k = 1.0 - f - tr;
    if (Xi) *Xi = (1.0 - k) / k * bz_coulomb_integral(L);
    if (!Lam) return;
    // Lambda = M B + M mu M / k
    std::vector<double> MB((size_t)np * np, 0.0), Mmu((size_t)np * np, 0.0);
    for (int i = 0; i < np; ++i)
        for (int l = 0; l < np; ++l) {
            const double m = M[(size_t)i * np + l];
            for (int j = 0; j < np; ++j) {
                MB[(size_t)i * np + j] += m * e(l, j);
                Mmu[(size_t)i * np + j] += m * mu[(size_t)l * np + j];
            }
        }
    for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) {
            double acc = 0.0;
            for (int l = 0; l < np; ++l) acc += Mmu[(size_t)i * np + l] * M[(size_t)l * np + j];
            Lam[(size_t)i * np + j] = MB[(size_t)i * np + j] + acc / k;
        }
}

}  // namespace pdep
