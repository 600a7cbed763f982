// G0W0 quasiparticle energies of occupied states (Sec. 2.2 self-energy in the PDEP basis,
// Sec. 2.5 contour deformation, Eqs. QPenergies and QPconZ).
//
// W_p(w) = Xi(w) + (1/Omega) sum_ij V_i Lambda_ij(w) V_j (Eq. Wchihb) with Lambda, Xi from
// the head, wings and body of the Lanczos chains (Eq. Bfinal).  For the state n,
//   <n m| W_p |m n> = Xi delta_mn + (1/Omega) sum_ij b_mi Lambda_ij b_mj,
// b_mi = <c_m| Fwd(V_i u_n)>, and G_KS(z) = sum_m |m><m| / (z - e_m) (Eq. Glehmann) is split
// by P_v and P_c: the occupied part is the sum over the N_v orbitals, whose b_mi are the
// projection coefficients of the right-hand sides (Eq. MVfinal); the empty part
// <w_in| (z - P_c H P_c)^-1 |w_jn> comes from the chains started at w_jn = P_c Fwd(V_j u_n),
// the body's chains of band n, with each chain's T = U diag(d) U^t diagonalised (Eq.
// MCfinal): poles d_k with residues ||w_jn|| U_1k sum_l <w_in|q_l> U_lk.  Every pole p
// (position e_p) then carries a weight T_p(w) = <n|..|n> contraction with W_p(w), and
//   Sigma_C(E) = sum_p [ -sgn(E - e_p) T_p(0) / 2
//                        - (1/pi) int_0^inf (T_p(iu) - T_p(0)) (E - e_p) / ((E - e_p)^2 + u^2) du
//                        + f_p T_p(e_p - E) ]                     (Eqs. contourdeformationfinal, fcontour)
// (the imaginary-axis integral of each pole's Lorentzian with T_p(0) is exact, the smooth
// rest takes Gauss-Legendre nodes of u = omega0 t / (1 - t); f_p = +1 for e_F < e_p < E, -1
// for E < e_p < e_F).  W_p at the residues' real frequencies carries a broadening eta.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "pdep_internal.h"
#include "tridiag_eigen.h"

namespace pdep {

namespace {

enum GwSlot { G_VR = WS_GW, G_STICKS, G_ROWS, G_NORM };

// out[s][r] = the component (n_s mod 2) of the packed orbital pair n_s / 2: u_{n_s}(r)
__global__ void k_band_grids(long ng, int nst, const int* __restrict__ states, const double2* __restrict__ upair,
                             double* __restrict__ out) {
    const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int st = blockIdx.y;
    if (r >= ng) return;
    const int n = states[st];
    const double2 u = upair[(long)(n >> 1) * ng + r];
    out[(long)st * ng + r] = (n & 1) ? u.y : u.x;
}

// norm[row] = sum_{G in S'} (4 pi / |G|^2) |x_G|^2 over the full sphere, from the half row
// (entries k < nh - 1 stand for G and -G; the centre G = 0 is last and has coul = 0)
__global__ void __launch_bounds__(256) k_coulomb_norms(int nh, const double2* __restrict__ x, long ld,
                                                       const double* __restrict__ coul, double* __restrict__ norm) {
    __shared__ double red[256];
    const double2* xr = x + (long)blockIdx.x * ld;
    double acc = 0.0;
    for (int k = threadIdx.x; k < nh; k += 256) {
        const double c = coul[k];
        const double2 v = xr[k];
        acc += (k + 1 < nh ? 2.0 : 1.0) * c * c * (v.x * v.x + v.y * v.y);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) norm[blockIdx.x] = red[0];
}

using C = std::complex<double>;

// The poles of one state's G_KS and their residue vectors over the basis potentials.
struct Poles {
    int np = 0;
    std::vector<double> e;         // positions
    std::vector<int> occ;          // 1 for the occupied orbitals (explicit sum)
    std::vector<int> self;         // 1 for the state itself (carries Xi)
    // residue of pole p: occupied m: the vector b_m (rank one, r_ij = b_i b_j); chain
    // pole (j, k): the column c_ijk (only column j nonzero)
    std::vector<double> vec;       // [p][np]
    std::vector<int> col;          // chain poles: j; occupied: -1
};

// T_p = (1/Omega) sum_ij Lambda_ij r_ij (+ Xi for the state itself) for one frequency
template <typename S>
S pole_weight(const Poles& P, int p, const S* lam, S xi, double omega) {
    const int np = P.np;
    const double* v = P.vec.data() + (size_t)p * np;
    S acc(0.0);
    if (P.col[p] < 0) {
        for (int i = 0; i < np; ++i) {
            S row(0.0);
            for (int j = 0; j < np; ++j) row += lam[(size_t)i * np + j] * v[j];
            acc += v[i] * row;
        }
    } else {
        const int j = P.col[p];
        for (int i = 0; i < np; ++i) acc += lam[(size_t)i * np + j] * v[i];
    }
    acc /= omega;
    if (P.self[p]) acc += xi;
    return acc;
}

}  // namespace

QpStats qp_energies(Ctx& c, int np, const double2* phi, int nst, const int* states, const double* vxc,
                    const pdep_qp_opts& o, pdep_qp_result* out, int ne, const double* energies, double* sig_e,
                    ApplyStats* dir_st) {
    QpStats qs;
    const Basis& b = c.basis;
    const int nv = c.nv, nl = o.n_lanczos, nf = o.n_freq;
    const double omega = b.omega, ef = o.e_fermi, eta = o.eta;
    hipStream_t s = c.stream;

    // chains of the potentials and the three directions; occupied pair coefficients
    Chains ch;
    std::vector<double> coef;
    run_chains(c, np, phi, 3, nl, ch, dir_st, &coef);
    qs.chains = ch.chains;
    qs.max_length = ch.max_length;
    qs.h_applications = ch.h_applications;
    const int npe = ch.npert;                     // np + 3
    const size_t oblk = (size_t)npe * npe;

    // imaginary-axis nodes: u_0 = 0, then Gauss-Legendre on t in (0, 1), u = omega0 t / (1 - t)
    std::vector<double> gx, gw;
    gauss_legendre(nf, gx, gw);
    std::vector<double> u(nf + 1, 0.0), wu(nf + 1, 0.0);
    for (int f = 0; f < nf; ++f) {
        const double t = 0.5 * (gx[f] + 1.0);
        u[f + 1] = o.omega0 * t / (1.0 - t);
        wu[f + 1] = 0.5 * gw[f] * o.omega0 / ((1.0 - t) * (1.0 - t));
    }
    const int nz = nf + 1;
    std::vector<FreqPoint> zp(nz);
    for (int f = 0; f < nz; ++f) zp[f] = FreqPoint{make_double2(0.0, u[f]), make_double2(0.0, -u[f])};
    std::vector<double2> Ez((size_t)nz * oblk);
    chain_body(c, ch, nz, zp.data(), Ez.data());
    std::vector<double> lam_im((size_t)nz * np * np), xi_im(nz), Er(oblk);
    for (int f = 0; f < nz; ++f) {
        for (size_t k = 0; k < oblk; ++k) Er[k] = Ez[(size_t)f * oblk + k].x;
        bfinal(np, Er.data(), b.L, nullptr, nullptr, nullptr, lam_im.data() + (size_t)f * np * np, &xi_im[f]);
    }

    // Sigma_X: rows Fwd(u_n u_m) on S for every state n and occupied m, their Coulomb norms
    std::vector<double> sx(nst, 0.0);
    {
        const long ng = b.ng, ld = sphere_ld(b.npw);
        const int nh = half_len(b.npw), nvp = pair_count(nv, nv), nrow = nst * nv;
        double* Vr = static_cast<double*>(c.ws(G_VR, (size_t)nst * ng * sizeof(double) + 64 * sizeof(int)));
        int* d_states = reinterpret_cast<int*>(Vr + (size_t)nst * ng);
        double2* sticks = static_cast<double2*>(
            c.ws(G_STICKS, (size_t)std::max(nrow, nst * nvp) * b.dims.nz * b.dims.sld * sizeof(double2)));
        double2* X = static_cast<double2*>(c.ws(G_ROWS, (size_t)nrow * ld * sizeof(double2)));
        double* d_norm = static_cast<double*>(c.ws(G_NORM, (size_t)nrow * sizeof(double)));
        PDEP_REQUIRE(nst <= 64, PDEP_EINVAL, "at most 64 states per call");
        PDEP_HIP(hipMemcpyAsync(d_states, states, nst * sizeof(int), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_band_grids, dim3((unsigned)((ng + 255) / 256), (unsigned)nst), dim3(256), 0, s, ng, nst,
                           d_states, c.upair.as<double2>(), Vr);
        PDEP_HIP(hipGetLastError());
        launch_slab_fwd_product<double>(b.dims, b.tables, Vr, c.upair.as<double2>(), nvp, nst * nvp, sticks, s);
        launch_sticks_to_sphere_pair<double>(b.dims, b.tables, sticks, nrow, X, ld, EPI_SCALE, 1.0, nullptr, 0, nullptr,
                                             nullptr, 0, s, nullptr, nv);
        hipLaunchKernelGGL(k_coulomb_norms, dim3((unsigned)nrow), dim3(256), 0, s, nh, X, ld, b.d_coul.as<double>(),
                           d_norm);
        PDEP_HIP(hipGetLastError());
        std::vector<double> nrm(nrow);
        PDEP_HIP(hipMemcpyAsync(nrm.data(), d_norm, nrow * sizeof(double), hipMemcpyDeviceToHost, s));
        PDEP_HIP(hipStreamSynchronize(s));
        const double ibz = bz_coulomb_integral(b.L);
        for (int st = 0; st < nst; ++st) {
            double acc = 0.0;
            for (int m = 0; m < nv; ++m) acc += nrm[(size_t)st * nv + m];
            sx[st] = -acc / omega - ibz;
        }
    }

    std::vector<double2> Oh((size_t)nl * oblk);
    for (int st = 0; st < nst; ++st) {
        const int n = states[st];
        // poles: the occupied orbitals, then the Ritz values of the chains (j, n)
        Poles P;
        P.np = np;
        for (int m = 0; m < nv; ++m) {
            P.e.push_back(c.eps[m]);
            P.occ.push_back(1);
            P.self.push_back(m == n ? 1 : 0);
            P.col.push_back(-1);
            for (int i = 0; i < np; ++i) P.vec.push_back(coef[((size_t)i * nv + n) * nv + m]);
        }
        for (int l = 0; l < nl; ++l)
            PDEP_HIP(hipMemcpyAsync(Oh.data() + (size_t)l * oblk, ch.O + ((size_t)l * nv + n) * oblk,
                                    oblk * sizeof(double2), hipMemcpyDeviceToHost, s));
        PDEP_HIP(hipStreamSynchronize(s));
        for (int j = 0; j < np; ++j) {
            const int r = j * nv + n, L = ch.len[r];
            if (L == 0) continue;
            std::vector<double> d(L), e(L > 1 ? L - 1 : 0), U;
            for (int l = 0; l < L; ++l) {
                d[l] = ch.alpha[(size_t)l * ch.nrow + r];
                if (l + 1 < L) e[l] = ch.beta[(size_t)l * ch.nrow + r];
            }
            PDEP_REQUIRE(tridiag_eigen(L, d, e, U), PDEP_EDEVICE, "tridiagonal eigensolver did not converge");
            for (int k = 0; k < L; ++k) {
                P.e.push_back(d[k]);
                P.occ.push_back(0);
                P.self.push_back(0);
                P.col.push_back(j);
                const double u1 = ch.wn[r] * U[k];           // ||w_jn|| U_1k
                for (int i = 0; i < np; ++i) {
                    double acc = 0.0;
                    for (int l = 0; l < L; ++l) acc += Oh[(size_t)l * oblk + (size_t)j * npe + i].x * U[(size_t)l * L + k];
                    P.vec.push_back(u1 * acc);
                }
            }
        }
        const int npol = (int)P.e.size();
        // weights on the imaginary axis
        std::vector<double> Wt((size_t)npol * nz);
        for (int p = 0; p < npol; ++p)
            for (int f = 0; f < nz; ++f)
                Wt[(size_t)p * nz + f] = pole_weight<double>(P, p, lam_im.data() + (size_t)f * np * np, xi_im[f], omega);

        auto sigma_c = [&](double E) -> C {
            double integ = 0.0;
            std::vector<int> rp;
            std::vector<double> rf;
            for (int p = 0; p < npol; ++p) {
                const double dd = E - P.e[p];
                const double* wt = Wt.data() + (size_t)p * nz;
                double rem = 0.0;
                for (int f = 1; f < nz; ++f) rem += wu[f] * (wt[f] - wt[0]) * dd / (dd * dd + u[f] * u[f]);
                integ += -(dd >= 0.0 ? 0.5 : -0.5) * wt[0] - rem / M_PI;
                if (ef < P.e[p] && P.e[p] < E) {
                    rp.push_back(p);
                    rf.push_back(1.0);
                } else if (E < P.e[p] && P.e[p] < ef) {
                    rp.push_back(p);
                    rf.push_back(-1.0);
                }
            }
            C res(0.0);
            if (!rp.empty()) {
                // W_p at the real frequencies |e_p - E| (even in the frequency)
                const int nr = (int)rp.size();
                std::vector<FreqPoint> zr(nr);
                for (int k = 0; k < nr; ++k) {
                    const double w = std::abs(P.e[rp[k]] - E);
                    zr[k] = FreqPoint{make_double2(-w, eta), make_double2(w, eta)};
                }
                std::vector<double2> Er2((size_t)nr * oblk), lam2((size_t)np * np);
                chain_body(c, ch, nr, zr.data(), Er2.data());
                qs.residue_points += nr;
                std::vector<C> lamc((size_t)np * np);
                for (int k = 0; k < nr; ++k) {
                    double2 xi2;
                    bfinal_complex(np, Er2.data() + (size_t)k * oblk, b.L, lam2.data(), &xi2);
                    for (size_t q = 0; q < lamc.size(); ++q) lamc[q] = C(lam2[q].x, lam2[q].y);
                    res += rf[k] * pole_weight<C>(P, rp[k], lamc.data(), C(xi2.x, xi2.y), omega);
                }
            }
            return C(integ, 0.0) + res;
        };

        pdep_qp_result& R = out[st];
        std::memset(&R, 0, sizeof(R));
        const double en = c.eps[n], vx = vxc ? vxc[st] : 0.0;
        R.eps_ks = en;
        R.sigma_x = sx[st];
        const C s0 = sigma_c(en);
        R.sigma_c_ks[0] = s0.real();
        R.sigma_c_ks[1] = s0.imag();
        const double h = o.dE;
        const double dsig = (sigma_c(en + h).real() - sigma_c(en - h).real()) / (2.0 * h);
        R.z = 1.0 / (1.0 - dsig);
        const double g0v = sx[st] + s0.real() - vx;        // g(e_n) of g(E) = e_n + Sigma(E) - vxc - E
        R.e_lin = en + R.z * g0v;
        // secant through (e_n, g(e_n)) and (e_lin, g(e_lin))
        double x0 = en, g0 = g0v, x1 = R.e_lin;
        C s1 = sigma_c(x1);
        double g1 = en + sx[st] + s1.real() - vx - x1;
        int it = 0;
        bool conv = false;
        for (it = 1; it <= o.secant_maxit; ++it) {
            if (g1 == 0.0) { conv = true; break; }
            if (g1 == g0) break;
            const double x2 = x1 - g1 * (x1 - x0) / (g1 - g0);
            x0 = x1;
            g0 = g1;
            x1 = x2;
            s1 = sigma_c(x1);
            g1 = en + sx[st] + s1.real() - vx - x1;
            if (std::abs(x1 - x0) <= o.secant_tol) { conv = true; break; }
        }
        R.e_qp = x1;
        R.sigma_c_qp[0] = s1.real();
        R.sigma_c_qp[1] = s1.imag();
        R.iterations = std::min(it, o.secant_maxit);
        R.converged = conv ? 1 : 0;
        qs.secant_iterations += R.iterations;
        if (energies && sig_e)
            for (int k = 0; k < ne; ++k) {
                const C v = sigma_c(energies[(size_t)st * ne + k]);
                sig_e[((size_t)st * ne + k) * 2] = v.real();
                sig_e[((size_t)st * ne + k) * 2 + 1] = v.imag();
            }
    }
    return qs;
}

}  // namespace pdep
