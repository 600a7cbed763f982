// Plane-wave sphere, grid tables, twiddle tables and the device allocator.
//
// The basis is every G = 2 pi (mx/Lx, my/Ly, mz/Lz) with 1/2 |G|^2 <= ecut (the
// plane-wave expansion of Sec. 2.1), enumerated lexicographically in (mx, my, mz).
// Because mz is the fastest index, every (mx, my) z-stick of the sphere is a
// contiguous run, which is what the stick passes of the transforms read and write.
#include <algorithm>
#include <cmath>

#include "pdep_internal.h"

namespace pdep {

void* Allocator::get(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 256;
    if (a.alloc) {
        p = a.alloc(bytes, a.ctx);
    } else {
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
    }
    PDEP_REQUIRE(p != nullptr, PDEP_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    return p;
}

void Allocator::put(void* p) {
    if (!p) return;
    if (a.alloc) {
        if (a.free) a.free(p, a.ctx);
    } else {
        (void)hipFree(p);
    }
}

void Buf::ensure(Allocator* al, size_t bytes) {
    if (p_ && bytes_ >= bytes && al_ == al) return;
    release();
    p_ = al->get(bytes);
    bytes_ = bytes;
    al_ = al;
}

void Buf::release() {
    if (p_ && al_) al_->put(p_);
    p_ = nullptr;
    bytes_ = 0;
}

namespace {

bool grid_ok(int n) {
    if (n < 4 || n > 128) return false;
    while (n % 3 == 0) n /= 3;
    while (n % 2 == 0) n /= 2;
    return n == 1;
}

// exp(-2 pi i m / n), m = 0..n-1, in extended precision and rounded once.
void twiddles(int n, std::vector<double>& out) {
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int m = 0; m < n; ++m) {
        const long double a = two_pi * (long double)m / (long double)n;
        out.push_back((double)cosl(a));
        out.push_back((double)-sinl(a));
    }
}

}  // namespace

void build_basis(const pdep_cell& cell, Basis& b) {
    for (int d = 0; d < 3; ++d) {
        PDEP_REQUIRE(std::isfinite(cell.L[d]) && cell.L[d] > 0.0, PDEP_EINVAL, "cell lengths must be positive");
        PDEP_REQUIRE(grid_ok(cell.n[d]), PDEP_EINVAL,
                     "grid sizes must be products of 2s and 3s between 4 and 128");
        b.L[d] = cell.L[d];
        b.n[d] = cell.n[d];
    }
    PDEP_REQUIRE(std::isfinite(cell.ecut) && cell.ecut > 0.0, PDEP_EINVAL, "ecut must be positive");
    b.ecut = cell.ecut;
    b.omega = cell.L[0] * cell.L[1] * cell.L[2];
    b.ng = cell.n[0] * cell.n[1] * cell.n[2];
    const double two_pi = 2.0 * M_PI;
    int nmax[3];
    for (int d = 0; d < 3; ++d) nmax[d] = (int)std::floor(std::sqrt(2.0 * cell.ecut) * cell.L[d] / two_pi) + 1;
    b.miller.clear();
    b.kin.clear();
    b.coul.clear();
    int mabs[3] = {0, 0, 0};
    for (int mx = -nmax[0]; mx <= nmax[0]; ++mx)
        for (int my = -nmax[1]; my <= nmax[1]; ++my)
            for (int mz = -nmax[2]; mz <= nmax[2]; ++mz) {
                const double gx = two_pi * mx / cell.L[0];
                const double gy = two_pi * my / cell.L[1];
                const double gz = two_pi * mz / cell.L[2];
                const double g2 = gx * gx + gy * gy + gz * gz;
                if (0.5 * g2 <= cell.ecut) {
                    b.miller.push_back(mx);
                    b.miller.push_back(my);
                    b.miller.push_back(mz);
                    b.kin.push_back(0.5 * g2);
                    b.coul.push_back(g2 > 0.0 ? std::sqrt(4.0 * M_PI) / std::sqrt(g2) : 0.0);
                    mabs[0] = std::max(mabs[0], std::abs(mx));
                    mabs[1] = std::max(mabs[1], std::abs(my));
                    mabs[2] = std::max(mabs[2], std::abs(mz));
                }
            }
    b.npw = (int)b.kin.size();
    for (int d = 0; d < 3; ++d)
        PDEP_REQUIRE(2 * mabs[d] + 1 <= cell.n[d], PDEP_EINVAL,
                     "the wavefunction sphere does not fit the FFT grid (increase n or lower ecut)");
    b.g0 = -1;
    for (int k = 0; k < b.npw; ++k)
        if (b.miller[3 * k] == 0 && b.miller[3 * k + 1] == 0 && b.miller[3 * k + 2] == 0) b.g0 = k;
    PDEP_REQUIRE(b.g0 >= 0 && b.npw >= 2, PDEP_EINVAL, "cutoff too small");
    b.mxmax = mabs[0];
    b.ax = 2 * b.mxmax + 1;
    // z-sticks: maximal runs of equal (mx, my) in the lexicographic order
    b.stick_start.clear();
    b.slab_pos.clear();
    b.stick_pos.resize(b.npw);
    for (int k = 0; k < b.npw; ++k) {
        const int mx = b.miller[3 * k], my = b.miller[3 * k + 1], mz = b.miller[3 * k + 2];
        if (k == 0 || mx != b.miller[3 * (k - 1)] || my != b.miller[3 * (k - 1) + 1]) {
            b.stick_start.push_back(k);
            const int ix = ((mx % b.n[0]) + b.n[0]) % b.n[0];
            const int iy = ((my % b.n[1]) + b.n[1]) % b.n[1];
            b.slab_pos.push_back(ix * b.n[1] + iy);
        }
        const int s = (int)b.stick_start.size() - 1;
        const int iz = ((mz % b.n[2]) + b.n[2]) % b.n[2];
        b.stick_pos[k] = s * b.n[2] + iz;
    }
    b.stick_start.push_back(b.npw);
    // x columns: for each mx in -mxmax..mxmax the sticks with that mx are consecutive and
    // cover my = -ymax(mx)..ymax(mx) (the sphere is convex and symmetric)
    b.col_start.assign(b.ax + 1, -1);
    b.col_my0.assign(b.ax, 0);
    const int nsticks = (int)b.stick_start.size() - 1;
    for (int s = 0; s < nsticks; ++s) {
        const int k = b.stick_start[s];
        const int c = b.miller[3 * k] + b.mxmax;
        if (b.col_start[c] < 0) {
            b.col_start[c] = s;
            b.col_my0[c] = b.miller[3 * k + 1];
        }
    }
    b.col_start[b.ax] = nsticks;
    for (int c = 0; c < b.ax; ++c) {
        PDEP_REQUIRE(b.col_start[c] >= 0, PDEP_EINVAL, "internal: empty x column in the sphere");
        const int cnt = (c + 1 < b.ax ? b.col_start[c + 1] : nsticks) - b.col_start[c];
        PDEP_REQUIRE(b.col_my0[c] <= 0 && cnt == 1 - 2 * b.col_my0[c], PDEP_EINVAL,
                     "internal: x column of the sphere is not a symmetric my range");
    }
    FftDims& d = b.dims;
    d.nx = b.n[0];
    d.ny = b.n[1];
    d.nz = b.n[2];
    d.ax = b.ax;
    d.mxmax = b.mxmax;
    d.mymax = 0;
    for (int c = 0; c < b.ax; ++c) d.mymax = std::max(d.mymax, -b.col_my0[c]);
    d.npw = b.npw;
    d.ns = (int)b.slab_pos.size();
    d.sld = (d.ns + 31) / 32 * 32;
    d.sg_max = 0;
    for (int s0 = 0; s0 < d.ns; s0 += kRegStickGroup) {
        const int s1 = std::min(d.ns, s0 + kRegStickGroup);
        d.sg_max = std::max(d.sg_max, b.stick_start[s1] - b.stick_start[s0]);
    }
    d.sgp_max = 0;
    for (int s0 = 0; s0 < (d.ns + 1) / 2; s0 += kPairStickGroup) {
        const int s1 = std::min((d.ns + 1) / 2, s0 + kPairStickGroup);
        d.sgp_max = std::max(d.sgp_max, b.stick_start[s1] - b.stick_start[s0]);
    }
    // every stick covers a symmetric mz range (convex, inversion-symmetric sphere)
    for (int s = 0; s < d.ns; ++s) {
        const int k0 = b.stick_start[s], cnt = b.stick_start[s + 1] - k0;
        PDEP_REQUIRE(cnt % 2 == 1 && b.miller[3 * k0 + 2] == -(cnt - 1) / 2, PDEP_EINVAL,
                     "internal: z stick of the sphere is not a symmetric mz range");
    }
    // inversion: the lexicographic order of an inversion-symmetric set is reversed by
    // G -> -G, so -G_k is entry npw - 1 - k, G = 0 the centre (npw - 1) / 2, and stick
    // ns - 1 - s the mirror of stick s (vectors real in r are stored as half spheres)
    PDEP_REQUIRE(b.npw % 2 == 1 && b.g0 == (b.npw - 1) / 2 && d.ns % 2 == 1, PDEP_EINVAL,
                 "internal: the sphere is not inversion symmetric");
    for (int k = 0; k < b.npw; ++k)
        for (int a = 0; a < 3; ++a)
            PDEP_REQUIRE(b.miller[3 * (b.npw - 1 - k) + a] == -b.miller[3 * k + a], PDEP_EINVAL,
                         "internal: the sphere order does not pair G with -G");
    for (int s = 0; s < d.ns; ++s)
        PDEP_REQUIRE(b.stick_start[d.ns - 1 - s] == b.npw - b.stick_start[s + 1], PDEP_EINVAL,
                     "internal: the stick order does not pair mirror sticks");
    d.px = make_axis_plan(d.nx);
    d.py = make_axis_plan(d.ny);
    d.pz = make_axis_plan(d.nz);
}

void upload_basis(Basis& b, Allocator* al, hipStream_t s) {
    auto up = [&](Buf& dst, const void* src, size_t bytes) {
        dst.ensure(al, bytes);
        PDEP_HIP(hipMemcpyAsync(dst.get(), src, bytes, hipMemcpyHostToDevice, s));
    };
    up(b.d_stick_start, b.stick_start.data(), b.stick_start.size() * sizeof(int));
    up(b.d_stick_pos, b.stick_pos.data(), b.stick_pos.size() * sizeof(int));
    up(b.d_slab_pos, b.slab_pos.data(), b.slab_pos.size() * sizeof(int));
    std::vector<int> cols(b.col_start);
    cols.insert(cols.end(), b.col_my0.begin(), b.col_my0.end());
    up(b.d_cols, cols.data(), cols.size() * sizeof(int));
    up(b.d_kin64, b.kin.data(), b.kin.size() * sizeof(double));
    std::vector<float> k32(b.kin.begin(), b.kin.end());
    up(b.d_kin32, k32.data(), k32.size() * sizeof(float));
    up(b.d_coul, b.coul.data(), b.coul.size() * sizeof(double));
    std::vector<double> tw;
    twiddles(b.n[0], tw);
    twiddles(b.n[1], tw);
    twiddles(b.n[2], tw);
    std::vector<float> tw32(tw.begin(), tw.end());
    up(b.d_tw64, tw.data(), tw.size() * sizeof(double));
    up(b.d_tw32, tw32.data(), tw32.size() * sizeof(float));
    PDEP_HIP(hipStreamSynchronize(s));
    BasisTables& t = b.tables;
    t.stick_start = b.d_stick_start.as<int>();
    t.stick_pos = b.d_stick_pos.as<int>();
    t.slab_pos = b.d_slab_pos.as<int>();
    t.col_start = b.d_cols.as<int>();
    t.col_my0 = b.d_cols.as<int>() + b.ax + 1;
    const double* t64 = b.d_tw64.as<double>();
    const float* t32 = b.d_tw32.as<float>();
    t.twx64 = t64;
    t.twy64 = t64 + 2 * b.n[0];
    t.twz64 = t64 + 2 * (b.n[0] + b.n[1]);
    t.twx32 = t32;
    t.twy32 = t32 + 2 * b.n[0];
    t.twz32 = t32 + 2 * (b.n[0] + b.n[1]);
}

}  // namespace pdep
