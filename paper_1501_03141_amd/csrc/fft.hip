// Batched pruned 3D FFTs between the wavefunction sphere and the real-space grid.
//
// A sphere vector (coefficients c_G, G in S) and a grid function are related by
//   Inv(c)(r) = sum_G c_G exp(iG.r),   Fwd(f)(G) = N_g^-1 sum_r f(r) exp(-iG.r).
// The 3D transform is split into three passes so that each pass keeps one 2D slab
// or one set of pencils in LDS:
//   plane pass  (one workgroup per (row, active x-plane)): z transforms of the
//               non-empty sticks and y transforms of every z column, in LDS;
//   pencil pass (one workgroup per (row, y, z-chunk)): x transforms of pencils, with
//               the real-space work (multiply by V, density accumulation, products)
//               fused between the inverse and the forward transform;
//   plane pass back to the sphere with a fused epilogue (kinetic term and shift,
//               scaling).
// Only the 2 mx_max + 1 x-planes that intersect the sphere travel through HBM
// between passes ("planes" buffer, layout [row][a][iy][iz]).  Each 1D transform is a
// mixed-radix (2, 3, 4, 8) Stockham FFT executed by the whole workgroup: every stage
// loads its butterfly inputs into registers, synchronises, and writes the outputs
// back in place.  Twiddles come from a table exp(-2 pi i m / n) built in double
// precision on the host and staged in LDS.
#include "pdep_internal.h"

namespace pdep {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxElems = 24;   // register budget of one stage: items * radix <= 24

template <typename T> __device__ __forceinline__ cplx<T> mk(T a, T b) { cplx<T> r; r.x = a; r.y = b; return r; }
// (generic over the vector type: cplx<T> is not deducible)
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
// multiply by SIGN * i
template <typename T, int SIGN> __device__ __forceinline__ cplx<T> mul_si(cplx<T> a) {
    return SIGN > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}

// In-register DFT of length R, y_k = sum_n v_n exp(SIGN 2 pi i n k / R).
template <typename T, int R, int SIGN> struct Dft;
template <typename T, int SIGN> struct Dft<T, 2, SIGN> {
    static __device__ __forceinline__ void run(cplx<T>* v) {
        cplx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};
template <typename T, int SIGN> struct Dft<T, 3, SIGN> {
    static __device__ __forceinline__ void run(cplx<T>* v) {
        const T h = T(0.86602540378443864676);   // sqrt(3)/2
        cplx<T> s = cadd(v[1], v[2]);
        cplx<T> d = csub(v[1], v[2]);
        cplx<T> m = mk<T>(v[0].x - T(0.5) * s.x, v[0].y - T(0.5) * s.y);
        cplx<T> t = mul_si<T, SIGN>(mk<T>(h * d.x, h * d.y));
        v[0] = cadd(v[0], s);
        v[1] = cadd(m, t);
        v[2] = csub(m, t);
    }
};
template <typename T, int SIGN> struct Dft<T, 4, SIGN> {
    static __device__ __forceinline__ void run(cplx<T>* v) {
        cplx<T> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        cplx<T> s13 = cadd(v[1], v[3]), d13 = mul_si<T, SIGN>(csub(v[1], v[3]));
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, d13);
        v[3] = csub(d02, d13);
    }
};
template <typename T, int SIGN> struct Dft<T, 8, SIGN> {
    static __device__ __forceinline__ void run(cplx<T>* v) {
        cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
        cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
        Dft<T, 4, SIGN>::run(e);
        Dft<T, 4, SIGN>::run(o);
        const T r = T(0.70710678118654752440);
        // w8^k = exp(SIGN 2 pi i k / 8)
        cplx<T> o1 = cmul(o[1], mk<T>(r, SIGN * r));
        cplx<T> o2 = mul_si<T, SIGN>(o[2]);
        cplx<T> o3 = cmul(o[3], mk<T>(-r, SIGN * r));
        v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);   v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);   v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);   v[7] = csub(e[3], o3);
    }
};

// Line l of a transform starts at LDS offset ((lo + l) mod m) * ls.
struct LineMap {
    int lo, m, ls;
    __device__ __forceinline__ int base(int l) const {
        int q = lo + l;
        if (q >= m) q -= m;
        return q * ls;
    }
};

// One Stockham stage over `nlines` lines of length N in LDS (element stride es).
// Ns = product of the radices of the previous stages.
template <typename T, int R, int SIGN>
__device__ __forceinline__ void fft_stage(cplx<T>* buf, int N, int Ns, int nlines, LineMap lm, int es,
                                          const cplx<T>* tw, bool line_fast) {
    constexpr int MAXI = kMaxElems / R;
    const int nb = N / R;
    const int total = nlines * nb;
    const int stride = N / (Ns * R);
    const int tid = threadIdx.x;
    cplx<T> v[MAXI][R];
    int ob[MAXI];
#pragma unroll
    for (int it = 0; it < MAXI; ++it) {
        const int item = tid + it * kThreads;
        ob[it] = -1;
        if (item < total) {
            int line, j;
            if (line_fast) { line = item % nlines; j = item / nlines; }
            else { j = item % nb; line = item / nb; }
            const int base = lm.base(line);
            const int jm = j % Ns;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                cplx<T> x = buf[base + (j + k * nb) * es];
                if (k > 0) {
                    cplx<T> w = tw[k * jm * stride];
                    if (SIGN > 0) w.y = -w.y;
                    x = cmul(x, w);
                }
                v[it][k] = x;
            }
            Dft<T, R, SIGN>::run(v[it]);
            ob[it] = base + ((j / Ns) * Ns * R + jm) * es;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < MAXI; ++it) {
        if (ob[it] >= 0) {
#pragma unroll
            for (int k = 0; k < R; ++k) buf[ob[it] + k * Ns * es] = v[it][k];
        }
    }
    __syncthreads();
}

template <typename T, int SIGN>
__device__ void fft_lines(cplx<T>* buf, const AxisPlan& p, int nlines, LineMap lm, int es,
                          const cplx<T>* tw, bool line_fast) {
    int Ns = 1;
    for (int s = 0; s < p.nst; ++s) {
        const int R = p.rad[s];
        if (R == 4) fft_stage<T, 4, SIGN>(buf, p.n, Ns, nlines, lm, es, tw, line_fast);
        else if (R == 8) fft_stage<T, 8, SIGN>(buf, p.n, Ns, nlines, lm, es, tw, line_fast);
        else if (R == 3) fft_stage<T, 3, SIGN>(buf, p.n, Ns, nlines, lm, es, tw, line_fast);
        else fft_stage<T, 2, SIGN>(buf, p.n, Ns, nlines, lm, es, tw, line_fast);
        Ns *= R;
    }
}

template <typename T> __device__ __forceinline__ const T* tw_of(const BasisTables& t, int axis);
template <> __device__ __forceinline__ const double* tw_of<double>(const BasisTables& t, int axis) {
    return axis == 0 ? t.twx64 : (axis == 1 ? t.twy64 : t.twz64);
}
template <> __device__ __forceinline__ const float* tw_of<float>(const BasisTables& t, int axis) {
    return axis == 0 ? t.twx32 : (axis == 1 ? t.twy32 : t.twz32);
}

template <typename T>
__device__ __forceinline__ void load_tw(cplx<T>* dst, const BasisTables& t, int axis, int n) {
    const T* src = tw_of<T>(t, axis);
    for (int e = threadIdx.x; e < n; e += kThreads) dst[e] = mk<T>(src[2 * e], src[2 * e + 1]);
}

// ------------------------------------------------------------------ plane passes ---

template <typename T>
__global__ __launch_bounds__(kThreads) void k_sphere_to_planes(FftDims d, BasisTables t,
                                                               const cplx<T>* __restrict__ in, long ld_in,
                                                               const int* __restrict__ rows,
                                                               const double* __restrict__ gscale,
                                                               cplx<T>* __restrict__ planes) {
    extern __shared__ __align__(16) unsigned char smem[];
    using C = cplx<T>;
    const int psz = d.ny * d.nz;
    C* buf = reinterpret_cast<C*>(smem);
    C* twy = buf + psz;
    C* twz = twy + d.ny;
    const int a = blockIdx.x;
    const int row = blockIdx.y;
    const int src_row = rows ? rows[row] : row;
    for (int e = threadIdx.x; e < psz; e += kThreads) buf[e] = mk<T>(0, 0);
    load_tw<T>(twy, t, 1, d.ny);
    load_tw<T>(twz, t, 2, d.nz);
    __syncthreads();
    const int k0 = t.plane_start[a], k1 = t.plane_start[a + 1];
    const C* src = in + (long)src_row * ld_in;
    for (int k = k0 + threadIdx.x; k < k1; k += kThreads) {
        C v = src[k];
        if (gscale) {
            const T g = (T)gscale[k];
            v.x *= g;
            v.y *= g;
        }
        buf[t.lds_idx[k]] = v;
    }
    __syncthreads();
    const int kk = t.stick_k[a];
    fft_lines<T, +1>(buf, d.pz, 2 * kk + 1, LineMap{(d.ny - kk) % d.ny, d.ny, d.nz}, 1, twz, false);
    fft_lines<T, +1>(buf, d.py, d.nz, LineMap{0, d.nz, 1}, d.nz, twy, true);
    C* dst = planes + ((long)row * d.ax + a) * psz;
    for (int e = threadIdx.x; e < psz; e += kThreads) dst[e] = buf[e];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_planes_to_sphere(
    FftDims d, BasisTables t, const cplx<T>* __restrict__ planes, const int* __restrict__ rows,
    cplx<T>* __restrict__ out, long ld_out, int epi, double alpha, const cplx<T>* __restrict__ x, long ld_x,
    const T* __restrict__ kin, const double* __restrict__ shift, int nshift, const double* __restrict__ gscale) {
    extern __shared__ __align__(16) unsigned char smem[];
    using C = cplx<T>;
    const int psz = d.ny * d.nz;
    C* buf = reinterpret_cast<C*>(smem);
    C* twy = buf + psz;
    C* twz = twy + d.ny;
    const int a = blockIdx.x;
    const int row = blockIdx.y;
    const C* src = planes + ((long)row * d.ax + a) * psz;
    for (int e = threadIdx.x; e < psz; e += kThreads) buf[e] = src[e];
    load_tw<T>(twy, t, 1, d.ny);
    load_tw<T>(twz, t, 2, d.nz);
    __syncthreads();
    fft_lines<T, -1>(buf, d.py, d.nz, LineMap{0, d.nz, 1}, d.nz, twy, true);
    const int kk = t.stick_k[a];
    fft_lines<T, -1>(buf, d.pz, 2 * kk + 1, LineMap{(d.ny - kk) % d.ny, d.ny, d.nz}, 1, twz, false);
    const int orow = rows ? rows[row] : row;
    const int k0 = t.plane_start[a], k1 = t.plane_start[a + 1];
    const T inv_ng = T(1.0 / ((double)d.nx * d.ny * d.nz));
    C* o = out + (long)orow * ld_out;
    if (epi == EPI_SHIFTED_H) {
        const T sh = (T)shift[orow % nshift];
        const C* xr = x + (long)orow * ld_x;
        for (int k = k0 + threadIdx.x; k < k1; k += kThreads) {
            const C f = buf[t.lds_idx[k]];
            const C xv = xr[k];
            const T dk = kin[k] - sh;
            o[k] = mk<T>(f.x * inv_ng + dk * xv.x, f.y * inv_ng + dk * xv.y);
        }
    } else if (epi == EPI_GSCALE) {
        for (int k = k0 + threadIdx.x; k < k1; k += kThreads) {
            const C f = buf[t.lds_idx[k]];
            const T g = (T)gscale[k] * inv_ng;
            o[k] = mk<T>(f.x * g, f.y * g);
        }
    } else {
        const T s = (T)alpha * inv_ng;
        for (int k = k0 + threadIdx.x; k < k1; k += kThreads) {
            const C f = buf[t.lds_idx[k]];
            o[k] = mk<T>(f.x * s, f.y * s);
        }
    }
}

// ------------------------------------------------------------------ pencil passes --
// A workgroup owns the x pencils of one (row, iy, z-chunk): an nx x zc tile in LDS with
// element (ix, z) at ix * zc + z.

template <typename T>
__device__ __forceinline__ void load_active_rows(cplx<T>* buf, const FftDims& d, const cplx<T>* planes_row,
                                                 int iy, int z0) {
    const int zc = d.zc;
    for (int e = threadIdx.x; e < d.nx * zc; e += kThreads) buf[e] = mk<T>(0, 0);
    __syncthreads();
    for (int e = threadIdx.x; e < d.ax * zc; e += kThreads) {
        const int a = e / zc, z = e - (e / zc) * zc;
        int ix = a - d.mxmax;
        if (ix < 0) ix += d.nx;
        buf[ix * zc + z] = planes_row[((long)a * d.ny + iy) * d.nz + z0 + z];
    }
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ void store_active_rows(const cplx<T>* buf, const FftDims& d, cplx<T>* planes_row,
                                                  int iy, int z0) {
    const int zc = d.zc;
    for (int e = threadIdx.x; e < d.ax * zc; e += kThreads) {
        const int a = e / zc, z = e - (e / zc) * zc;
        int ix = a - d.mxmax;
        if (ix < 0) ix += d.nx;
        planes_row[((long)a * d.ny + iy) * d.nz + z0 + z] = buf[ix * zc + z];
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_pencil_hv(FftDims d, BasisTables t, cplx<T>* __restrict__ planes,
                                                        const T* __restrict__ V, long v_stride,
                                                        const int* __restrict__ vsel) {
    extern __shared__ __align__(16) unsigned char smem[];
    using C = cplx<T>;
    C* buf = reinterpret_cast<C*>(smem);
    C* twx = buf + d.nx * d.zc;
    const int nzc = d.nz / d.zc;
    const int iy = blockIdx.x / nzc, z0 = (blockIdx.x - iy * nzc) * d.zc;
    const int row = blockIdx.y;
    load_tw<T>(twx, t, 0, d.nx);
    C* prow = planes + (long)row * d.ax * d.ny * d.nz;
    load_active_rows<T>(buf, d, prow, iy, z0);
    fft_lines<T, +1>(buf, d.px, d.zc, LineMap{0, d.zc, 1}, d.zc, twx, true);
    const T* Vr = V + (vsel ? (long)vsel[row] * v_stride : 0);
    for (int e = threadIdx.x; e < d.nx * d.zc; e += kThreads) {
        const int ix = e / d.zc, z = e - (e / d.zc) * d.zc;
        const T vv = Vr[((long)ix * d.ny + iy) * d.nz + z0 + z];
        buf[e].x *= vv;
        buf[e].y *= vv;
    }
    __syncthreads();
    fft_lines<T, -1>(buf, d.px, d.zc, LineMap{0, d.zc, 1}, d.zc, twx, true);
    store_active_rows<T>(buf, d, prow, iy, z0);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_pencil_inv_store(FftDims d, BasisTables t,
                                                               const cplx<T>* __restrict__ planes,
                                                               cplx<T>* __restrict__ grid_c, T* __restrict__ grid_r) {
    extern __shared__ __align__(16) unsigned char smem[];
    using C = cplx<T>;
    C* buf = reinterpret_cast<C*>(smem);
    C* twx = buf + d.nx * d.zc;
    const int nzc = d.nz / d.zc;
    const int iy = blockIdx.x / nzc, z0 = (blockIdx.x - iy * nzc) * d.zc;
    const int row = blockIdx.y;
    const long ng = (long)d.nx * d.ny * d.nz;
    load_tw<T>(twx, t, 0, d.nx);
    load_active_rows<T>(buf, d, planes + (long)row * d.ax * d.ny * d.nz, iy, z0);
    fft_lines<T, +1>(buf, d.px, d.zc, LineMap{0, d.zc, 1}, d.zc, twx, true);
    for (int e = threadIdx.x; e < d.nx * d.zc; e += kThreads) {
        const int ix = e / d.zc, z = e - (e / d.zc) * d.zc;
        const long g = ((long)ix * d.ny + iy) * d.nz + z0 + z;
        if (grid_c) grid_c[row * ng + g] = buf[e];
        else grid_r[row * ng + g] = buf[e].x;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_pencil_fwd_product(FftDims d, BasisTables t, const T* __restrict__ Vr,
                                                                 const cplx<T>* __restrict__ u, int nv,
                                                                 cplx<T>* __restrict__ planes) {
    extern __shared__ __align__(16) unsigned char smem[];
    using C = cplx<T>;
    C* buf = reinterpret_cast<C*>(smem);
    C* twx = buf + d.nx * d.zc;
    const int nzc = d.nz / d.zc;
    const int iy = blockIdx.x / nzc, z0 = (blockIdx.x - iy * nzc) * d.zc;
    const int row = blockIdx.y;
    const long ng = (long)d.nx * d.ny * d.nz;
    load_tw<T>(twx, t, 0, d.nx);
    const T* vrow = Vr + (u ? (long)(row / nv) : (long)row) * ng;
    const C* urow = u ? u + (long)(row % nv) * ng : nullptr;
    for (int e = threadIdx.x; e < d.nx * d.zc; e += kThreads) {
        const int ix = e / d.zc, z = e - (e / d.zc) * d.zc;
        const long g = ((long)ix * d.ny + iy) * d.nz + z0 + z;
        const T vv = vrow[g];
        if (urow) {
            const C uu = urow[g];
            buf[e] = mk<T>(vv * uu.x, vv * uu.y);
        } else {
            buf[e] = mk<T>(vv, 0);
        }
    }
    __syncthreads();
    fft_lines<T, -1>(buf, d.px, d.zc, LineMap{0, d.zc, 1}, d.zc, twx, true);
    store_active_rows<T>(buf, d, planes + (long)row * d.ax * d.ny * d.nz, iy, z0);
}

constexpr int kMaxAcc = 24;

__global__ __launch_bounds__(kThreads) void k_pencil_density(FftDims d, BasisTables t,
                                                             const double2* __restrict__ planes, int nv,
                                                             const double2* __restrict__ u, double scale,
                                                             double* __restrict__ dn) {
    extern __shared__ __align__(16) unsigned char smem[];
    double2* buf = reinterpret_cast<double2*>(smem);
    double2* twx = buf + d.nx * d.zc;
    const int nzc = d.nz / d.zc;
    const int iy = blockIdx.x / nzc, z0 = (blockIdx.x - iy * nzc) * d.zc;
    const int pert = blockIdx.y;
    const long ng = (long)d.nx * d.ny * d.nz;
    const long plane_row = (long)d.ax * d.ny * d.nz;
    load_tw<double>(twx, t, 0, d.nx);
    double acc[kMaxAcc];
#pragma unroll
    for (int j = 0; j < kMaxAcc; ++j) acc[j] = 0.0;
    const int nel = d.nx * d.zc;
    for (int v = 0; v < nv; ++v) {
        load_active_rows<double>(buf, d, planes + ((long)pert * nv + v) * plane_row, iy, z0);
        fft_lines<double, +1>(buf, d.px, d.zc, LineMap{0, d.zc, 1}, d.zc, twx, true);
        const double2* uv = u + (long)v * ng;
#pragma unroll
        for (int j = 0; j < kMaxAcc; ++j) {
            const int e = threadIdx.x + j * kThreads;
            if (e < nel) {
                const int ix = e / d.zc, z = e - (e / d.zc) * d.zc;
                const double2 uu = uv[((long)ix * d.ny + iy) * d.nz + z0 + z];
                const double2 f = buf[e];
                acc[j] += uu.x * f.x + uu.y * f.y;     // Re(conj(u) f)
            }
        }
        __syncthreads();
    }
    double* out = dn + (long)pert * ng;
#pragma unroll
    for (int j = 0; j < kMaxAcc; ++j) {
        const int e = threadIdx.x + j * kThreads;
        if (e < nel) {
            const int ix = e / d.zc, z = e - (e / d.zc) * d.zc;
            out[((long)ix * d.ny + iy) * d.nz + z0 + z] = scale * acc[j];
        }
    }
}

// ------------------------------------------------------------------ host checks ----

void check_stages(const AxisPlan& p, int nlines, const char* what) {
    int Ns = 1;
    for (int s = 0; s < p.nst; ++s) {
        const int R = p.rad[s];
        const long items = (long)nlines * (p.n / R);
        PDEP_REQUIRE(items <= (long)kThreads * (kMaxElems / R), PDEP_EINVAL,
                     std::string("FFT stage too large for one workgroup: ") + what);
        Ns *= R;
    }
    PDEP_REQUIRE(Ns == p.n, PDEP_EINVAL, "bad radix plan");
}

template <typename T> size_t plane_lds(const FftDims& d) {
    return sizeof(cplx<T>) * ((size_t)d.ny * d.nz + d.ny + d.nz);
}
template <typename T> size_t pencil_lds(const FftDims& d) {
    return sizeof(cplx<T>) * ((size_t)d.nx * d.zc + d.nx);
}

void check_plane(const FftDims& d, const BasisTables&) {
    check_stages(d.pz, d.ny, "z sticks");
    check_stages(d.py, d.nz, "y columns");
}
void check_pencil(const FftDims& d) { check_stages(d.px, d.zc, "x pencils"); }
void check_rows(int nrows) { PDEP_REQUIRE(nrows <= 65535, PDEP_EINVAL, "too many rows for one transform launch"); }

}  // namespace

AxisPlan make_axis_plan(int n) {
    AxisPlan p;
    p.n = n;
    int m = n;
    while (m % 3 == 0) { p.rad[p.nst++] = 3; m /= 3; }
    int twos = 0;
    while (m % 2 == 0) { ++twos; m /= 2; }
    PDEP_REQUIRE(m == 1, PDEP_EINVAL, "grid sizes must be products of 2s and 3s");
    if (twos % 2 == 1 && twos >= 3) { p.rad[p.nst++] = 8; twos -= 3; }
    while (twos >= 2) { p.rad[p.nst++] = 4; twos -= 2; }
    if (twos == 1) p.rad[p.nst++] = 2;
    PDEP_REQUIRE(p.nst <= 8, PDEP_EINVAL, "radix plan too long");
    return p;
}

template <typename T>
void launch_sphere_to_planes(const FftDims& d, const BasisTables& t, const cplx<T>* in, long ld_in,
                             const int* rows, int nrows, const double* gscale, cplx<T>* planes, hipStream_t s) {
    if (nrows <= 0) return;
    check_plane(d, t);
    check_rows(nrows);
    dim3 grid(d.ax, nrows);
    const double pl_ = (double)d.ax * d.ny * d.nz * sizeof(cplx<T>);   // one row of planes
    const double sp_ = (double)d.npw * sizeof(cplx<T>);                 // one sphere vector
    ProfScope prof_(K_SPHERE_TO_PLANES, s, (double)nrows * (sp_ + pl_));
    hipLaunchKernelGGL(k_sphere_to_planes<T>, grid, dim3(kThreads), plane_lds<T>(d), s, d, t, in, ld_in, rows,
                       gscale, planes);
    PDEP_HIP(hipGetLastError());
}

template <typename T>
void launch_planes_to_sphere(const FftDims& d, const BasisTables& t, const cplx<T>* planes, int nrows,
                             const int* rows, cplx<T>* out, long ld_out, int epi, double alpha, const cplx<T>* x,
                             long ld_x, const T* kin, const double* shift, int nshift, const double* gscale,
                             hipStream_t s) {
    if (nrows <= 0) return;
    check_plane(d, t);
    check_rows(nrows);
    dim3 grid(d.ax, nrows);
    const double pl_ = (double)d.ax * d.ny * d.nz * sizeof(cplx<T>);   // one row of planes
    const double sp_ = (double)d.npw * sizeof(cplx<T>);                 // one sphere vector
    ProfScope prof_(K_PLANES_TO_SPHERE, s, (double)nrows * (pl_ + sp_ + (epi == EPI_SHIFTED_H ? sp_ : 0.0)));
    hipLaunchKernelGGL(k_planes_to_sphere<T>, grid, dim3(kThreads), plane_lds<T>(d), s, d, t, planes, rows, out,
                       ld_out, epi, alpha, x, ld_x, kin, shift, nshift > 0 ? nshift : 1, gscale);
    PDEP_HIP(hipGetLastError());
}

template <typename T>
void launch_pencil_hv(const FftDims& d, const BasisTables& t, cplx<T>* planes, int nrows, const T* V,
                      long v_stride, const int* vsel, hipStream_t s) {
    if (nrows <= 0) return;
    check_pencil(d);
    check_rows(nrows);
    dim3 grid(d.ny * (d.nz / d.zc), nrows);
    const double pl_ = (double)d.ax * d.ny * d.nz * sizeof(cplx<T>);   // one row of planes
    const double sp_ = (double)d.npw * sizeof(cplx<T>);                 // one sphere vector
    ProfScope prof_(K_PENCIL_HV, s, (double)nrows * 2.0 * pl_ + (double)d.nx * d.ny * d.nz * sizeof(T));
    hipLaunchKernelGGL(k_pencil_hv<T>, grid, dim3(kThreads), pencil_lds<T>(d), s, d, t, planes, V, v_stride, vsel);
    PDEP_HIP(hipGetLastError());
}

template <typename T>
void launch_pencil_inv_store(const FftDims& d, const BasisTables& t, const cplx<T>* planes, int nrows,
                             cplx<T>* grid_c, T* grid_r, hipStream_t s) {
    if (nrows <= 0) return;
    check_pencil(d);
    check_rows(nrows);
    dim3 grid(d.ny * (d.nz / d.zc), nrows);
    const double pl_ = (double)d.ax * d.ny * d.nz * sizeof(cplx<T>);   // one row of planes
    const double sp_ = (double)d.npw * sizeof(cplx<T>);                 // one sphere vector
    ProfScope prof_(K_PENCIL_INV_STORE, s,
                    (double)nrows * (pl_ + (double)d.nx * d.ny * d.nz * (grid_c ? sizeof(cplx<T>) : sizeof(T))));
    hipLaunchKernelGGL(k_pencil_inv_store<T>, grid, dim3(kThreads), pencil_lds<T>(d), s, d, t, planes, grid_c,
                       grid_r);
    PDEP_HIP(hipGetLastError());
}

template <typename T>
void launch_pencil_fwd_product(const FftDims& d, const BasisTables& t, const T* Vr, const cplx<T>* u, int nv,
                               int nrows, cplx<T>* planes, hipStream_t s) {
    if (nrows <= 0) return;
    check_pencil(d);
    check_rows(nrows);
    dim3 grid(d.ny * (d.nz / d.zc), nrows);
    const double pl_ = (double)d.ax * d.ny * d.nz * sizeof(cplx<T>);   // one row of planes
    const double sp_ = (double)d.npw * sizeof(cplx<T>);                 // one sphere vector
    const double g_ = (double)d.nx * d.ny * d.nz;
    ProfScope prof_(K_PENCIL_FWD_PRODUCT, s,
                    (double)nrows * (pl_ + g_ * (u ? sizeof(cplx<T>) : 0)) + g_ * sizeof(T) * (u ? nrows / nv : nrows));
    hipLaunchKernelGGL(k_pencil_fwd_product<T>, grid, dim3(kThreads), pencil_lds<T>(d), s, d, t, Vr, u,
                       nv > 0 ? nv : 1, planes);
    PDEP_HIP(hipGetLastError());
}

void launch_pencil_density(const FftDims& d, const BasisTables& t, const double2* planes, int npert, int nv,
                           const double2* u, double scale, double* dn, hipStream_t s) {
    if (npert <= 0) return;
    check_pencil(d);
    PDEP_REQUIRE(d.nx * d.zc <= kThreads * kMaxAcc, PDEP_EINVAL, "density tile too large");
    check_rows(npert);
    dim3 grid(d.ny * (d.nz / d.zc), npert);
    const double g_ = (double)d.nx * d.ny * d.nz;
    ProfScope prof_(K_PENCIL_DENSITY, s,
                    (double)npert * nv * ((double)d.ax * d.ny * d.nz * 16.0 + g_ * 16.0) + (double)npert * g_ * 8.0);
    hipLaunchKernelGGL(k_pencil_density, grid, dim3(kThreads), pencil_lds<double>(d), s, d, t, planes, nv, u, scale,
                       dn);
    PDEP_HIP(hipGetLastError());
}

#define PDEP_INST_FFT(T)                                                                                       \
    template void launch_sphere_to_planes<T>(const FftDims&, const BasisTables&, const cplx<T>*, long,         \
                                             const int*, int, const double*, cplx<T>*, hipStream_t);           \
    template void launch_planes_to_sphere<T>(const FftDims&, const BasisTables&, const cplx<T>*, int,          \
                                             const int*, cplx<T>*, long, int, double, const cplx<T>*, long,     \
                                             const T*, const double*, int, const double*, hipStream_t);         \
    template void launch_pencil_hv<T>(const FftDims&, const BasisTables&, cplx<T>*, int, const T*, long,       \
                                      const int*, hipStream_t);                                                \
    template void launch_pencil_inv_store<T>(const FftDims&, const BasisTables&, const cplx<T>*, int,          \
                                             cplx<T>*, T*, hipStream_t);                                        \
    template void launch_pencil_fwd_product<T>(const FftDims&, const BasisTables&, const T*, const cplx<T>*,   \
                                               int, int, cplx<T>*, hipStream_t);

PDEP_INST_FFT(double)
PDEP_INST_FFT(float)

}  // namespace pdep
