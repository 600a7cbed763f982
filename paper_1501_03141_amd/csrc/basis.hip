// Plane-wave sphere, grid tables, twiddle tables and the device allocator.
//
// The basis is every G = 2 pi (mx/Lx, my/Ly, mz/Lz) with 1/2 |G|^2 <= ecut (the
// plane-wave expansion of Sec. 2.1), enumerated lexicographically in (mx, my, mz).
// Because mx is the slowest index, the sphere is naturally stored plane by plane,
// which is what the plane passes of the transforms read and write.
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
    b.plane_start.assign(b.ax + 1, 0);
    b.stick_k.assign(b.ax, 0);
    b.lds_idx.resize(b.npw);
    for (int k = 0; k < b.npw; ++k) {
        const int a = b.miller[3 * k] + b.mxmax;
        b.plane_start[a + 1] = k + 1;
        b.stick_k[a] = std::max(b.stick_k[a], std::abs(b.miller[3 * k + 1]));
        const int iy = ((b.miller[3 * k + 1] % b.n[1]) + b.n[1]) % b.n[1];
        const int iz = ((b.miller[3 * k + 2] % b.n[2]) + b.n[2]) % b.n[2];
        b.lds_idx[k] = iy * b.n[2] + iz;
    }
    for (int a = 1; a <= b.ax; ++a) b.plane_start[a] = std::max(b.plane_start[a], b.plane_start[a - 1]);
    FftDims& d = b.dims;
    d.nx = b.n[0];
    d.ny = b.n[1];
    d.nz = b.n[2];
    d.ax = b.ax;
    d.mxmax = b.mxmax;
    d.npw = b.npw;
    d.px = make_axis_plan(d.nx);
    d.py = make_axis_plan(d.ny);
    d.pz = make_axis_plan(d.nz);
    // z chunk of the pencil kernels: the largest divisor of nz whose FP64 tile stays <= 40 KB
    d.zc = 1;
    for (int zc = d.nz; zc >= 1; --zc)
        if (d.nz % zc == 0 && (size_t)d.nx * zc * 16 <= 40 * 1024 && d.nx * zc <= 256 * 24) {
            d.zc = zc;
            break;
        }
}

void upload_basis(Basis& b, Allocator* al, hipStream_t s) {
    auto up = [&](Buf& dst, const void* src, size_t bytes) {
        dst.ensure(al, bytes);
        PDEP_HIP(hipMemcpyAsync(dst.get(), src, bytes, hipMemcpyHostToDevice, s));
    };
    up(b.d_plane_start, b.plane_start.data(), b.plane_start.size() * sizeof(int));
    up(b.d_stick_k, b.stick_k.data(), b.stick_k.size() * sizeof(int));
    up(b.d_lds_idx, b.lds_idx.data(), b.lds_idx.size() * sizeof(int));
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
    t.plane_start = b.d_plane_start.as<int>();
    t.stick_k = b.d_stick_k.as<int>();
    t.lds_idx = b.d_lds_idx.as<int>();
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
