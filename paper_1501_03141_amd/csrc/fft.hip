// Batched pruned 3D FFTs between the wavefunction sphere and the real-space grid.
//
// A sphere vector (coefficients c_G, G in S) and a grid function are related by
//   Inv(c)(r) = sum_G c_G exp(iG.r),   Fwd(f)(G) = N_g^-1 sum_r f(r) exp(-iG.r).
// The sphere is a union of z-sticks: for each (mx, my) with at least one G in S, the
// entries with that (mx, my) are contiguous in the lexicographic sphere order and
// cover mz = -k..k.  The 3D transform is done in two kinds of passes:
//   stick pass (one workgroup per (row, group of sticks)): the length-nz transforms
//               of the non-empty sticks only, read from / written to the sphere with
//               a fused epilogue on the way back (kinetic term and shift, scaling);
//   slab pass  (one workgroup per (row, z)): the 2D (x, y) transform of one z slab in
//               LDS -- y transforms of the non-empty x columns only, x transforms of
//               every y row -- with the real-space work (multiply by V, products,
//               density accumulation) fused between the inverse and forward halves.
// Between passes only the stick values travel through HBM ("sticks" buffer, layout
// [row][iz][stick], stick index fastest so that both passes move contiguous runs).
// Real-space grids handed to or produced by the slab pass are z-major ([iz][ix][iy]).
//
// Each 1D transform is a mixed-radix (2, 3, 4, 8) Stockham FFT run by the whole
// workgroup on lines held in LDS: every stage loads its butterfly inputs into
// registers, synchronises, and writes the outputs back in place.  The common grid
// sizes are compile-time template parameters (all index arithmetic is then by
// constants); other sizes use the same code with run-time sizes.  Twiddles come from
// tables exp(-2 pi i m / n) built in extended precision on the host.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "pdep_internal.h"

namespace pdep {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxElems = 24;   // register budget of one stage: items * radix <= 24

// Sticks per stick-pass workgroup for a given nz: about 1.5k elements per workgroup
// (0.75k for FP64 at nz = 48, measured 10% faster there).
template <typename T> __host__ __device__ constexpr int sticks_per_group(int nz) {
    return nz >= 96 ? 16 : (nz >= 48 ? (sizeof(T) > sizeof(float) ? 16 : 32) : (nz >= 24 ? 48 : 64));
}

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

// ------------------------------------------------------- register-resident DFTs ---
// A whole line of length N held by one thread, transformed with every index and every
// twiddle a compile-time constant (mixed radix 2/3/4/8, decimation in time).  The
// twiddles exp(+-2 pi i e / N) are evaluated at compile time: the angle is reduced to
// the first octant with integer arithmetic and sin / cos come from their Taylor
// series (Horner form, 13 terms; |x| <= pi/4, error below one unit in the last place
// of a double).

template <int B, int E, typename F> __device__ __forceinline__ void sfor(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

struct TwCS { double c, s; };
constexpr double sin_small(double x) {
    const double x2 = x * x;
    double r = 1.0;
    for (int k = 13; k >= 1; --k) r = 1.0 - x2 / ((2.0 * k) * (2.0 * k + 1.0)) * r;
    return x * r;
}
constexpr double cos_small(double x) {
    const double x2 = x * x;
    double r = 1.0;
    for (int k = 13; k >= 1; --k) r = 1.0 - x2 / ((2.0 * k - 1.0) * (2.0 * k)) * r;
    return r;
}
// exp(2 pi i e / N)
constexpr TwCS unit_root(int e, int N) {
    e = ((e % N) + N) % N;
    const int q = (4 * e) / N, r = (4 * e) % N;   // angle = (pi/2) (q + r / N)
    const double half_pi = 1.5707963267948966192;
    double c = 0.0, sn = 0.0;
    if (2 * r <= N) {
        const double x = half_pi * r / N;
        c = cos_small(x);
        sn = sin_small(x);
    } else {
        const double x = half_pi * (N - r) / N;
        c = sin_small(x);
        sn = cos_small(x);
    }
    for (int i = 0; i < q; ++i) {
        const double t = c;
        c = -sn;
        sn = t;
    }
    return TwCS{c, sn};
}

constexpr int reg_radix(int n) { return (n % 4 == 0 && n > 8) ? 4 : (n % 3 == 0 ? 3 : 2); }
constexpr bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
// inverse of a modulo m (gcd(a, m) = 1)
constexpr int inv_mod(int a, int m) {
    for (int x = 1; x < m; ++x)
        if ((a * x) % m == 1) return x;
    return 1;
}

template <typename T, int SIGN, int N, int IS> __device__ __forceinline__ void dft_reg(const cplx<T>* x, cplx<T>* X);

// Good-Thomas split N = N1 N2 with gcd(N1, N2) = 1: input n = (N2 n1 + N1 n2) mod N and
// output k = (N2 a k1 + N1 b k2) mod N, a = N2^-1 mod N1, b = N1^-1 mod N2, turn the
// length-N DFT into an N1 x N2 two-dimensional DFT with no twiddle factors.
template <typename T, int SIGN, int N1, int N2>
__device__ __forceinline__ void dft_pfa(const cplx<T>* x, cplx<T>* X) {
    constexpr int N = N1 * N2;
    constexpr int a = inv_mod(N2 % N1, N1), b = inv_mod(N1 % N2, N2);
    cplx<T> Z[N];   // Z[k1 * N2 + n2]: length-N1 DFTs over n1
    sfor<0, N2>([&](auto n2c) {
        constexpr int n2 = decltype(n2c)::value;
        cplx<T> v[N1];
        sfor<0, N1>([&](auto n1c) {
            constexpr int n1 = decltype(n1c)::value;
            v[n1] = x[(N2 * n1 + N1 * n2) % N];
        });
        Dft<T, N1, SIGN>::run(v);
        sfor<0, N1>([&](auto k1c) {
            constexpr int k1 = decltype(k1c)::value;
            Z[k1 * N2 + n2] = v[k1];
        });
    });
    sfor<0, N1>([&](auto k1c) {
        constexpr int k1 = decltype(k1c)::value;
        cplx<T> Y[N2];
        dft_reg<T, SIGN, N2, 1>(Z + k1 * N2, Y);
        sfor<0, N2>([&](auto k2c) {
            constexpr int k2 = decltype(k2c)::value;
            X[(N2 * a * k1 + N1 * b * k2) % N] = Y[k2];
        });
    });
}

// X[k] = sum_n x[n * IS] exp(SIGN 2 pi i n k / N), k = 0..N-1.
template <typename T, int SIGN, int N, int IS>
__device__ __forceinline__ void dft_reg(const cplx<T>* x, cplx<T>* X) {
    if constexpr (IS == 1 && N % 3 == 0 && N > 3 && pow2(N / 3)) {
        dft_pfa<T, SIGN, 3, N / 3>(x, X);
    } else if constexpr (N == 1) {
        X[0] = x[0];
    } else if constexpr (N == 2 || N == 3 || N == 4 || N == 8) {
        cplx<T> v[N];
        sfor<0, N>([&](auto n) { v[decltype(n)::value] = x[decltype(n)::value * IS]; });
        Dft<T, N, SIGN>::run(v);
        sfor<0, N>([&](auto k) { X[decltype(k)::value] = v[decltype(k)::value]; });
    } else {
        constexpr int R = reg_radix(N);
        constexpr int M = N / R;
        // n = n1 + R n2: length-M transforms of the R decimated sequences, then
        // twiddles exp(SIGN 2 pi i n1 k1 / N) and radix-R butterflies.
        cplx<T> Y[N];
        sfor<0, R>([&](auto n1c) {
            constexpr int n1 = decltype(n1c)::value;
            dft_reg<T, SIGN, M, IS * R>(x + n1 * IS, Y + n1 * M);
        });
        sfor<0, M>([&](auto k1c) {
            constexpr int k1 = decltype(k1c)::value;
            cplx<T> v[R];
            sfor<0, R>([&](auto n1c) {
                constexpr int n1 = decltype(n1c)::value;
                if constexpr ((n1 * k1) % N == 0) {
                    v[n1] = Y[n1 * M + k1];
                } else {
                    constexpr TwCS w = unit_root(SIGN * n1 * k1, N);
                    v[n1] = cmul(Y[n1 * M + k1], mk<T>((T)w.c, (T)w.s));
                }
            });
            Dft<T, R, SIGN>::run(v);
            sfor<0, R>([&](auto k2c) {
                constexpr int k2 = decltype(k2c)::value;
                X[k1 + M * k2] = v[k2];
            });
        });
    }
}

// Line l of a transform starts at LDS offset ((lo + l) mod m) * ls.
struct LineMap {
    int lo, m, ls;
    __device__ __forceinline__ int base(int l) const {
        int q = lo + l;
        if (q >= m) q -= m;
        return q * ls;
    }
};

// Radix plan as a compile-time value (make_axis_plan uses the same factorisation).
struct CPlan {
    int nst;
    int rad[8];
};
constexpr CPlan cplan(int n) {
    CPlan p{0, {0, 0, 0, 0, 0, 0, 0, 0}};
    int m = n;
    while (m % 3 == 0 && m > 1) { p.rad[p.nst++] = 3; m /= 3; }
    int twos = 0;
    while (m % 2 == 0 && m > 1) { ++twos; m /= 2; }
    if (twos % 2 == 1 && twos >= 3) { p.rad[p.nst++] = 8; twos -= 3; }
    while (twos >= 2) { p.rad[p.nst++] = 4; twos -= 2; }
    if (twos == 1) p.rad[p.nst++] = 2;
    return p;
}

// One Stockham stage over `nlines` lines of length N in LDS (element stride es).
// Ns = product of the radices of the previous stages.  Template arguments that are 0
// are taken from the run-time arguments.  LF: consecutive threads take consecutive
// lines (for lines that are adjacent in LDS) instead of consecutive butterflies.
template <typename T, int R, int SIGN, int N_, int NS_, int NL_, bool LF>
__device__ __forceinline__ void fft_stage(cplx<T>* buf, int n_rt, int ns_rt, int nl_rt, LineMap lm, int es,
                                          const cplx<T>* tw) {
    constexpr int MAXI_CT = (N_ > 0 && NL_ > 0) ? (NL_ * (N_ / R) + kThreads - 1) / kThreads : kMaxElems / R;
    constexpr int MAXI = MAXI_CT < kMaxElems / R ? MAXI_CT : kMaxElems / R;
    const int N = N_ ? N_ : n_rt;
    const int Ns = N_ ? NS_ : ns_rt;
    const int nlines = NL_ ? NL_ : nl_rt;
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
            if (LF) { line = item % nlines; j = item / nlines; }
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

template <typename T, int SIGN, int N, int NL, bool LF, int S, int NS>
__device__ __forceinline__ void fft_ct(cplx<T>* buf, int nl_rt, LineMap lm, int es, const cplx<T>* tw) {
    constexpr CPlan P = cplan(N);
    if constexpr (S < P.nst) {
        constexpr int R = P.rad[S];
        fft_stage<T, R, SIGN, N, NS, NL, LF>(buf, N, NS, nl_rt, lm, es, tw);
        fft_ct<T, SIGN, N, NL, LF, S + 1, NS * R>(buf, nl_rt, lm, es, tw);
    }
}

// All stages of a length-N transform over nlines lines.  N == 0: run-time plan p.
template <typename T, int SIGN, int N, int NL, bool LF>
__device__ __forceinline__ void fft_lines(cplx<T>* buf, const AxisPlan& p, int nlines, LineMap lm, int es,
                                          const cplx<T>* tw) {
    if constexpr (N > 0) {
        fft_ct<T, SIGN, N, NL, LF, 0, 1>(buf, nlines, lm, es, tw);
    } else {
        int Ns = 1;
        for (int s = 0; s < p.nst; ++s) {
            const int R = p.rad[s];
            if (R == 4) fft_stage<T, 4, SIGN, 0, 0, NL, LF>(buf, p.n, Ns, nlines, lm, es, tw);
            else if (R == 8) fft_stage<T, 8, SIGN, 0, 0, NL, LF>(buf, p.n, Ns, nlines, lm, es, tw);
            else if (R == 3) fft_stage<T, 3, SIGN, 0, 0, NL, LF>(buf, p.n, Ns, nlines, lm, es, tw);
            else fft_stage<T, 2, SIGN, 0, 0, NL, LF>(buf, p.n, Ns, nlines, lm, es, tw);
            Ns *= R;
        }
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

// ------------------------------------------------------------------ stick passes ---

// sphere rows -> sticks (inverse z transforms).  gscale (per G, may be null)
// multiplies the coefficients while scattering.
template <typename T, int NZ_>
__global__ __launch_bounds__(kThreads) void k_sphere_to_sticks(FftDims d, BasisTables t,
                                                               const cplx<T>* __restrict__ in, long ld_in,
                                                               const double* __restrict__ gscale,
                                                               cplx<T>* __restrict__ sticks) {
    extern __shared__ __align__(16) unsigned char smem[];
    using C = cplx<T>;
    const int NZ = NZ_ ? NZ_ : d.nz;
    const int SG = sticks_per_group<T>(NZ);
    C* buf = reinterpret_cast<C*>(smem);
    C* twz = buf + SG * NZ;
    const int s0 = blockIdx.x * SG;
    const int ns_here = min(SG, d.ns - s0);
    const int row = blockIdx.y;
    for (int e = threadIdx.x; e < SG * NZ; e += kThreads) buf[e] = mk<T>(0, 0);
    load_tw<T>(twz, t, 2, NZ);
    __syncthreads();
    const int k0 = t.stick_start[s0], k1 = t.stick_start[s0 + ns_here];
    const C* src = in + (long)row * ld_in;
    const int off = s0 * NZ;
    for (int k = k0 + threadIdx.x; k < k1; k += kThreads) {
        C v = src[k];
        if (gscale) {
            const T g = (T)gscale[k];
            v.x *= g;
            v.y *= g;
        }
        buf[t.stick_pos[k] - off] = v;
    }
    __syncthreads();
    fft_lines<T, +1, NZ_, 0, false>(buf, d.pz, ns_here, LineMap{0, SG, NZ}, 1, twz);
    C* dst = sticks + (long)row * NZ * d.sld + s0;
    for (int e = threadIdx.x; e < SG * NZ; e += kThreads) {
        const int sl = e % SG, z = e / SG;
        if (sl < ns_here) dst[(long)z * d.sld + sl] = buf[sl * NZ + z];
    }
}

// Sum of v over the NT threads of a workgroup (fixed order), result in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

// sticks -> sphere rows (forward z transforms, 1/N_g) with an epilogue.
template <typename T, int NZ_>
__global__ __launch_bounds__(kThreads) void k_sticks_to_sphere(
    FftDims d, BasisTables t, const cplx<T>* __restrict__ sticks, cplx<T>* __restrict__ out, long ld_out, int epi,
    double alpha, const cplx<T>* __restrict__ x, long ld_x, const T* __restrict__ kin,
    const double* __restrict__ shift, int nshift, const double* __restrict__ gscale, double* __restrict__ dot_part) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kThreads];
    using C = cplx<T>;
    const int NZ = NZ_ ? NZ_ : d.nz;
    const int SG = sticks_per_group<T>(NZ);
    C* buf = reinterpret_cast<C*>(smem);
    C* twz = buf + SG * NZ;
    const int s0 = blockIdx.x * SG;
    const int ns_here = min(SG, d.ns - s0);
    const int row = blockIdx.y;
    const C* src = sticks + (long)row * NZ * d.sld + s0;
    for (int e = threadIdx.x; e < SG * NZ; e += kThreads) {
        const int sl = e % SG, z = e / SG;
        if (sl < ns_here) buf[sl * NZ + z] = src[(long)z * d.sld + sl];
    }
    load_tw<T>(twz, t, 2, NZ);
    __syncthreads();
    fft_lines<T, -1, NZ_, 0, false>(buf, d.pz, ns_here, LineMap{0, SG, NZ}, 1, twz);
    const int k0 = t.stick_start[s0], k1 = t.stick_start[s0 + ns_here];
    const int off = s0 * NZ;
    const T inv_ng = T(1.0 / ((double)d.nx * d.ny * d.nz));
    C* o = out + (long)row * ld_out;
    if (epi == EPI_SHIFTED_H) {
        const T sh = (T)shift[row % nshift];
        const C* xr = x + (long)row * ld_x;
        double acc = 0.0;
        for (int k = k0 + threadIdx.x; k < k1; k += kThreads) {
            const C f = buf[t.stick_pos[k] - off];
            const C xv = xr[k];
            const T dk = kin[k] - sh;
            const C ov = mk<T>(f.x * inv_ng + dk * xv.x, f.y * inv_ng + dk * xv.y);
            o[k] = ov;
            acc += (double)xv.x * (double)ov.x + (double)xv.y * (double)ov.y;
        }
        if (dot_part) {
            const double tot = block_sum<kThreads>(acc, red);
            if (threadIdx.x == 0) dot_part[(long)row * gridDim.x + blockIdx.x] = tot;
        }
    } else if (epi == EPI_GSCALE) {
        for (int k = k0 + threadIdx.x; k < k1; k += kThreads) {
            const C f = buf[t.stick_pos[k] - off];
            const T g = (T)gscale[k] * inv_ng;
            o[k] = mk<T>(f.x * g, f.y * g);
        }
    } else {
        const T sc = (T)alpha * inv_ng;
        for (int k = k0 + threadIdx.x; k < k1; k += kThreads) {
            const C f = buf[t.stick_pos[k] - off];
            o[k] = mk<T>(f.x * sc, f.y * sc);
        }
    }
}

// Register-resident sticks -> sphere pass (FP32): one thread per z stick of a group
// of kRegStickGroup sticks, the whole length-NZ line in registers.  A stick's sphere
// entries are contiguous and cover mz = -kz..kz, so line index iz holds mz = iz or
// iz - NZ and the stick needs no position table.  The group's sphere entries pass
// through LDS so that the sphere side (with the epilogue) is written coalesced; the
// sticks side ([row][iz][stick]) is read coalesced across the threads of a group.
// (The same structure for the sphere -> sticks direction measured slower than the
// LDS-staged kernel, which is kept for it.)
template <int NZ>
__global__ __launch_bounds__(kRegStickGroup) void k_sticks_to_sphere_reg(
    FftDims d, BasisTables t, const float2* __restrict__ sticks, float2* __restrict__ out, long ld_out, int epi,
    double alpha, const float2* __restrict__ x, long ld_x, const float* __restrict__ kin,
    const double* __restrict__ shift, int nshift, const double* __restrict__ gscale, double* __restrict__ dot_part) {
    constexpr int HALF = (NZ + 1) / 2;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kRegStickGroup];
    float2* buf = reinterpret_cast<float2*>(smem);
    const int s0 = blockIdx.x * kRegStickGroup, row = blockIdx.y;
    const int nsh = min(kRegStickGroup, d.ns - s0);
    const int kb = t.stick_start[s0], ke = t.stick_start[s0 + nsh];
    const int sl = threadIdx.x;
    if (sl < nsh) {
        const float2* srcs = sticks + (long)row * NZ * d.sld + s0 + sl;
        float2 v[NZ], X[NZ];
        sfor<0, NZ>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            v[i] = srcs[(long)i * d.sld];
        });
        dft_reg<float, -1, NZ, 1>(v, X);
        const int ks = t.stick_start[s0 + sl] - kb, kz = (t.stick_start[s0 + sl + 1] - kb - ks - 1) / 2;
        float2* line = buf + ks + kz;
        sfor<0, NZ>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int mz = i < HALF ? i : i - NZ;
            if (mz >= -kz && mz <= kz) line[mz] = X[i];
        });
    }
    __syncthreads();
    const float inv_ng = 1.0f / (float)((double)d.nx * d.ny * d.nz);
    float2* o = out + (long)row * ld_out;
    if (epi == EPI_SHIFTED_H) {
        const float sh = (float)shift[row % nshift];
        const float2* xr = x + (long)row * ld_x;
        double acc = 0.0;
        for (int k = kb + threadIdx.x; k < ke; k += kRegStickGroup) {
            const float2 f = buf[k - kb], xv = xr[k];
            const float dk = kin[k] - sh;
            const float2 ov = make_float2(f.x * inv_ng + dk * xv.x, f.y * inv_ng + dk * xv.y);
            o[k] = ov;
            acc += (double)xv.x * (double)ov.x + (double)xv.y * (double)ov.y;
        }
        if (dot_part) {
            const double tot = block_sum<kRegStickGroup>(acc, red);
            if (threadIdx.x == 0) dot_part[(long)row * gridDim.x + blockIdx.x] = tot;
        }
    } else if (epi == EPI_GSCALE) {
        for (int k = kb + threadIdx.x; k < ke; k += kRegStickGroup) {
            const float2 f = buf[k - kb];
            const float g = (float)gscale[k] * inv_ng;
            o[k] = make_float2(f.x * g, f.y * g);
        }
    } else {
        const float sc = (float)alpha * inv_ng;
        for (int k = kb + threadIdx.x; k < ke; k += kRegStickGroup) {
            const float2 f = buf[k - kb];
            o[k] = make_float2(f.x * sc, f.y * sc);
        }
    }
}

// ------------------------------------------------------- paired half-sphere rows ---
// Rows that are real in r (Hermitian-symmetric coefficients, c_{-G} = conj c_G) are kept
// as half spheres: entries k <= c = (npw - 1) / 2 of the sphere order, where -G_k is
// entry npw - 1 - k and the centre c is G = 0.  Two such rows a, b travel through one
// complex transform: Inv(a + i b) = a(r) + i b(r) with both parts real, so a real
// potential acts on each part separately, and after the forward transform W of the
// product a_G = (W_G + conj W_-G) / 2, b_G = (W_G - conj W_-G) / 2i.

// Rows come in groups of `group` consecutive rows (all rows: one group); packed row j is
// pair j' of group g (j = g * ceil(group / 2) + j'), i.e. rows g * group + 2 j' and the
// next one, which is absent (zero) when it falls outside the group or past nrows.
struct PairRows {
    int a;
    bool has_b;
};
__device__ __forceinline__ PairRows pair_rows(int pr, int group, int nrows) {
    const int hp = (group + 1) / 2;
    const int g = pr / hp, j = pr - g * hp;
    const int a = g * group + 2 * j;
    return PairRows{a, 2 * j + 1 < group && a + 1 < nrows};
}

// Half-sphere rows a, b of packed row j -> its sticks (inverse z transforms).  The
// entries k > c come from the mirrors npw - 1 - k (conjugated); the centre is taken
// real.
template <typename T, int NZ_>
__global__ __launch_bounds__(kThreads) void k_sphere_to_sticks_pair(FftDims d, BasisTables t,
                                                                    const cplx<T>* __restrict__ in, long ld_in,
                                                                    int nrows, int group,
                                                                    cplx<T>* __restrict__ sticks) {
    extern __shared__ __align__(16) unsigned char smem[];
    using C = cplx<T>;
    const int NZ = NZ_ ? NZ_ : d.nz;
    const int SG = sticks_per_group<T>(NZ);
    C* buf = reinterpret_cast<C*>(smem);
    C* twz = buf + SG * NZ;
    const int s0 = blockIdx.x * SG;
    const int ns_here = min(SG, d.ns - s0);
    const int pr = blockIdx.y;
    const PairRows rw = pair_rows(pr, group, nrows);
    const bool has_b = rw.has_b;
    for (int e = threadIdx.x; e < SG * NZ; e += kThreads) buf[e] = mk<T>(0, 0);
    load_tw<T>(twz, t, 2, NZ);
    __syncthreads();
    const int k0 = t.stick_start[s0], k1 = t.stick_start[s0 + ns_here];
    const int npw = d.npw, c = (npw - 1) / 2;
    const C* a = in + (long)rw.a * ld_in;
    const C* b = a + ld_in;
    const int off = s0 * NZ;
    for (int k = k0 + threadIdx.x; k < k1; k += kThreads) {
        const int src = k <= c ? k : npw - 1 - k;
        C va = a[src];
        C vb = has_b ? b[src] : mk<T>(0, 0);
        if (k == c) {
            va.y = 0;
            vb.y = 0;
        } else if (k > c) {
            va.y = -va.y;
            vb.y = -vb.y;
        }
        buf[t.stick_pos[k] - off] = mk<T>(va.x - vb.y, va.y + vb.x);
    }
    __syncthreads();
    fft_lines<T, +1, NZ_, 0, false>(buf, d.pz, ns_here, LineMap{0, SG, NZ}, 1, twz);
    C* dst = sticks + (long)pr * NZ * d.sld + s0;
    for (int e = threadIdx.x; e < SG * NZ; e += kThreads) {
        const int sl = e % SG, z = e / SG;
        if (sl < ns_here) dst[(long)z * d.sld + sl] = buf[sl * NZ + z];
    }
}

// Register-resident form of the paired sphere-to-sticks pass (FP32): 128 threads, one z
// stick each with its line in registers; threads 0..63 take kPairStickGroup front sticks,
// threads 64..127 their mirrors.  The half-sphere entries of the group (every entry of
// the front sticks up to the centre c) are read once, with all loads of a thread in
// flight, into LDS for both rows: a front stick takes a_k + i b_k at its mz, its mirror
// conj(a_k) + i conj(b_k) at -mz (the coefficients of functions real in r at -G).  The
// middle stick (its own mirror, handled by its front thread) takes its entries k > c from
// their mirrors npw - 1 - k, conjugated, and the centre real.
template <int NZ>
__global__ __launch_bounds__(2 * kPairStickGroup) void k_sphere_to_sticks_pair_reg(
    FftDims d, BasisTables t, const float2* __restrict__ in, long ld_in, int nrows, int group,
    float2* __restrict__ sticks) {
    constexpr int HALF = (NZ + 1) / 2;
    constexpr int GS = kPairStickGroup, NT = 2 * kPairStickGroup, LQ = 8;
    extern __shared__ __align__(16) unsigned char smem[];
    float2* la = reinterpret_cast<float2*>(smem);
    float2* lb = la + d.sgp_max;
    const int nfront = (d.ns + 1) / 2;
    const int s0 = blockIdx.x * GS, pr = blockIdx.y;
    const int nf = min(GS, nfront - s0);
    const int c = (d.npw - 1) / 2;
    const int kb = t.stick_start[s0], ne = min(t.stick_start[s0 + nf], c + 1) - kb;
    const PairRows rw = pair_rows(pr, group, nrows);
    const bool has_b = rw.has_b;
    const float2* a = in + (long)rw.a * ld_in + kb;
    // an absent second row reads the first again (finite values) and is scaled to zero:
    // a select or a branch around its load would wait for each load inside the branch
    const float2* b = has_b ? a + ld_in : a;
    const float bscale = has_b ? 1.f : 0.f;
    const int tid = threadIdx.x;
    for (int e0 = 0; e0 < ne; e0 += LQ * NT) {
        float2 ra[LQ], rb[LQ];
        sfor<0, LQ>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const int e = min(e0 + tid + q * NT, ne - 1);
            ra[q] = a[e];
            const float2 vb = b[e];
            rb[q] = make_float2(bscale * vb.x, bscale * vb.y);
        });
        sfor<0, LQ>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const int e = min(e0 + tid + q * NT, ne - 1);   // unguarded: see stage_rows_in
            la[e] = ra[q];
            lb[e] = rb[q];
        });
    }
    __syncthreads();
    const bool mir = tid >= GS;                 // wave-uniform
    const int j = mir ? tid - GS : tid;
    if (j >= nf) return;
    const int sf = s0 + j, sk = mir ? d.ns - 1 - sf : sf;
    if (mir && sk == sf) return;                // the middle stick: its front thread writes it
    const int ks = t.stick_start[sf], kz = (t.stick_start[sf + 1] - ks - 1) / 2;
    const int k0 = ks + kz;                     // front entry of mz = 0
    float2 v[NZ], X[NZ];
    sfor<0, NZ>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int mz = i < HALF ? i : i - NZ;
        float2 w = make_float2(0.f, 0.f);
        if (mz >= -kz && mz <= kz) {
            const int k = k0 + (mir ? -mz : mz);   // front entry (of -G for the mirror)
            const bool back = k > c;               // the upper half of the middle stick
            const int e = (back ? d.npw - 1 - k : k) - kb;
            float2 va = la[e], vb = lb[e];
            if (k == c) {
                va.y = 0.f;
                vb.y = 0.f;
            } else if (back != mir) {
                va.y = -va.y;
                vb.y = -vb.y;
            }
            w = make_float2(va.x - vb.y, va.y + vb.x);
        }
        v[i] = w;
    });
    dft_reg<float, +1, NZ, 1>(v, X);
    float2* dst = sticks + (long)pr * NZ * d.sld + sk;
    sfor<0, NZ>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        dst[(long)i * d.sld] = X[i];
    });
}

// Sticks of packed row j -> half-sphere rows a, b (pair_rows) with the epilogue
// EPI_SHIFTED_H, out = F + (kin - shift[row % nshift]) x and, when dot_part is non-null,
// the partial sums of Re<x, out> over the full sphere (weight 2 off the centre) per
// workgroup; or EPI_SCALE, out = alpha F.  A workgroup transforms SG / 2 sticks of the
// front half (s <= (ns - 1) / 2, which hold every entry k <= c) and their mirrors
// ns - 1 - s.
template <typename T, int NZ_>
__global__ __launch_bounds__(kThreads) void k_sticks_to_sphere_pair(
    FftDims d, BasisTables t, const cplx<T>* __restrict__ sticks, int nrows, int group, cplx<T>* __restrict__ out,
    long ld_out, int epi, double alpha, const cplx<T>* __restrict__ x, long ld_x, const T* __restrict__ kin,
    const double* __restrict__ shift, int nshift, double* __restrict__ dot_part) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[2][kThreads];
    using C = cplx<T>;
    const int NZ = NZ_ ? NZ_ : d.nz;
    const int SG = sticks_per_group<T>(NZ), SGH = SG / 2;
    C* buf = reinterpret_cast<C*>(smem);
    C* twz = buf + SG * NZ;
    const int nfront = (d.ns + 1) / 2;
    const int s0 = blockIdx.x * SGH;
    const int nf = min(SGH, nfront - s0);
    const int pr = blockIdx.y;
    const C* src = sticks + (long)pr * NZ * d.sld;
    // line j < SGH: front stick s0 + j; line SGH + j: its mirror
    for (int e = threadIdx.x; e < SG * NZ; e += kThreads) {
        const int sl = e % SG, z = e / SG;
        const int j = sl < SGH ? sl : sl - SGH;
        C v = mk<T>(0, 0);
        if (j < nf) v = src[(long)z * d.sld + (sl < SGH ? s0 + j : d.ns - 1 - s0 - j)];
        buf[sl * NZ + z] = v;
    }
    load_tw<T>(twz, t, 2, NZ);
    __syncthreads();
    fft_lines<T, -1, NZ_, 0, false>(buf, d.pz, SG, LineMap{0, SG, NZ}, 1, twz);
    const int c = (d.npw - 1) / 2;
    const int k0 = t.stick_start[s0], k1 = min(t.stick_start[s0 + nf], c + 1);
    const T inv_ng = T(1.0 / ((double)d.nx * d.ny * d.nz));
    const PairRows rw = pair_rows(pr, group, nrows);
    const int ra = rw.a, rb = ra + 1;
    const bool has_b = rw.has_b;
    C* oa = out + (long)ra * ld_out;
    C* ob = oa + ld_out;
    if (epi == EPI_SCALE) {
        const T half = T(0.5 * alpha) * inv_ng;
        for (int k = k0 + threadIdx.x; k < k1; k += kThreads) {
            const int pos = t.stick_pos[k];
            const int st = pos / NZ, iz = pos - st * NZ;
            const int j = st - s0;
            const C W = buf[j * NZ + iz];
            const C Wm = buf[(SGH + j) * NZ + (iz == 0 ? 0 : NZ - iz)];
            oa[k] = mk<T>(half * (W.x + Wm.x), half * (W.y - Wm.y));
            if (has_b) ob[k] = mk<T>(half * (W.y + Wm.y), half * (Wm.x - W.x));
        }
        return;
    }
    const T half = T(0.5) * inv_ng;
    const T sha = (T)shift[ra % nshift], shb = has_b ? (T)shift[rb % nshift] : T(0);
    const C* xa = x + (long)ra * ld_x;
    const C* xb = xa + ld_x;
    double acca = 0.0, accb = 0.0;
    for (int k = k0 + threadIdx.x; k < k1; k += kThreads) {
        const int pos = t.stick_pos[k];
        const int st = pos / NZ, iz = pos - st * NZ;
        const int j = st - s0;
        const C W = buf[j * NZ + iz];
        const C Wm = buf[(SGH + j) * NZ + (iz == 0 ? 0 : NZ - iz)];
        const double w = k == c ? 1.0 : 2.0;
        const T kk = kin[k];
        {
            const C xv = xa[k];
            const T dk = kk - sha;
            const C ov = mk<T>(half * (W.x + Wm.x) + dk * xv.x, half * (W.y - Wm.y) + dk * xv.y);
            oa[k] = ov;
            acca += w * ((double)xv.x * (double)ov.x + (double)xv.y * (double)ov.y);
        }
        if (has_b) {
            const C xv = xb[k];
            const T dk = kk - shb;
            const C ov = mk<T>(half * (W.y + Wm.y) + dk * xv.x, half * (Wm.x - W.x) + dk * xv.y);
            ob[k] = ov;
            accb += w * ((double)xv.x * (double)ov.x + (double)xv.y * (double)ov.y);
        }
    }
    if (dot_part) {
        red[0][threadIdx.x] = acca;
        red[1][threadIdx.x] = accb;
        __syncthreads();
        for (int s = kThreads / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) {
                red[0][threadIdx.x] += red[0][threadIdx.x + s];
                red[1][threadIdx.x] += red[1][threadIdx.x + s];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            dot_part[(long)ra * gridDim.x + blockIdx.x] = red[0][0];
            if (has_b) dot_part[(long)rb * gridDim.x + blockIdx.x] = red[1][0];
        }
    }
}

// Register-resident form of the paired sticks-to-sphere pass (FP32, EPI_SHIFTED_H): 128
// threads, one z stick each with the whole line in registers; threads 0..63 take
// kPairStickGroup front sticks, threads 64..127 their mirrors.  The transforms land in
// two LDS arrays indexed by the front entry k (the mirror one holding W at -G_k), from
// which the epilogue separates the two rows as in k_sticks_to_sphere_pair.
template <int NZ>
__global__ __launch_bounds__(2 * kPairStickGroup) void k_sticks_to_sphere_pair_reg(
    FftDims d, BasisTables t, const float2* __restrict__ sticks, int nrows, int group, float2* __restrict__ out,
    long ld_out, const float2* __restrict__ x, long ld_x, const float* __restrict__ kin,
    const double* __restrict__ shift, int nshift, double* __restrict__ dot_part) {
    constexpr int HALF = (NZ + 1) / 2;
    constexpr int GS = kPairStickGroup, NT = 2 * kPairStickGroup;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[2][NT];
    float2* bufF = reinterpret_cast<float2*>(smem);
    float2* bufM = bufF + d.sgp_max;
    const int nfront = (d.ns + 1) / 2;
    const int s0 = blockIdx.x * GS, pr = blockIdx.y;
    const int nf = min(GS, nfront - s0);
    const int kb = t.stick_start[s0], ke = t.stick_start[s0 + nf];
    const int tid = threadIdx.x;
    const bool mir = tid >= GS;                 // wave-uniform
    const int j = mir ? tid - GS : tid;
    if (j < nf) {
        const int sf = s0 + j;
        const int sk = mir ? d.ns - 1 - sf : sf;
        const float2* src = sticks + (long)pr * NZ * d.sld + sk;
        float2 v[NZ], X[NZ];
        sfor<0, NZ>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            v[i] = src[(long)i * d.sld];
        });
        dft_reg<float, -1, NZ, 1>(v, X);
        const int ks = t.stick_start[sf] - kb, kz = (t.stick_start[sf + 1] - t.stick_start[sf] - 1) / 2;
        float2* line = (mir ? bufM : bufF) + ks + kz;
        const int sgn = mir ? -1 : 1;           // the mirror stick's mz lands at the front entry of -mz
        sfor<0, NZ>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int mz = i < HALF ? i : i - NZ;
            if (mz >= -kz && mz <= kz) line[sgn * mz] = X[i];
        });
    }
    __syncthreads();
    const int c = (d.npw - 1) / 2;
    const int k1 = min(ke, c + 1);
    const float inv_ng = 1.0f / (float)((double)d.nx * d.ny * d.nz);
    const float half = 0.5f * inv_ng;
    const PairRows rw = pair_rows(pr, group, nrows);
    const int ra = rw.a, rb = ra + 1;
    const bool has_b = rw.has_b;
    const float sha = (float)shift[ra % nshift], shb = has_b ? (float)shift[rb % nshift] : 0.f;
    float2* oa = out + (long)ra * ld_out;
    float2* ob = oa + ld_out;
    const float2* xa = x + (long)ra * ld_x;
    const float2* xb = xa + ld_x;
    double acca = 0.0, accb = 0.0;
    // LQ entries per thread at a time: their kinetic energies and x values are loaded
    // before the first is used (clamped indices, so every load is in bounds)
    constexpr int LQ = 8;
    for (int e0 = kb + tid; e0 < k1; e0 += LQ * NT) {
        float kk[LQ];
        float2 xva[LQ], xvb[LQ];
        sfor<0, LQ>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const int k = min(e0 + q * NT, k1 - 1);
            kk[q] = kin[k];
            xva[q] = xa[k];
            xvb[q] = has_b ? xb[k] : make_float2(0.f, 0.f);
        });
        sfor<0, LQ>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const int k = e0 + q * NT;
            if (k < k1) {
                const float2 W = bufF[k - kb], Wm = bufM[k - kb];
                const double w = k == c ? 1.0 : 2.0;
                {
                    const float2 xv = xva[q];
                    const float dk = kk[q] - sha;
                    const float2 ov = make_float2(half * (W.x + Wm.x) + dk * xv.x, half * (W.y - Wm.y) + dk * xv.y);
                    oa[k] = ov;
                    acca += w * ((double)xv.x * (double)ov.x + (double)xv.y * (double)ov.y);
                }
                if (has_b) {
                    const float2 xv = xvb[q];
                    const float dk = kk[q] - shb;
                    const float2 ov = make_float2(half * (W.y + Wm.y) + dk * xv.x, half * (Wm.x - W.x) + dk * xv.y);
                    ob[k] = ov;
                    accb += w * ((double)xv.x * (double)ov.x + (double)xv.y * (double)ov.y);
                }
            }
        });
    }
    if (dot_part) {
        red[0][tid] = acca;
        red[1][tid] = accb;
        __syncthreads();
        for (int s = NT / 2; s > 0; s >>= 1) {
            if (tid < s) {
                red[0][tid] += red[0][tid + s];
                red[1][tid] += red[1][tid + s];
            }
            __syncthreads();
        }
        if (tid == 0) {
            dot_part[(long)ra * gridDim.x + blockIdx.x] = red[0][0];
            if (has_b) dot_part[(long)rb * gridDim.x + blockIdx.x] = red[1][0];
        }
    }
}

// ------------------------------------------------------------------- slab passes ---
// A workgroup owns one z slab of one row: an nx x ny tile in LDS, element (ix, iy) at
// ix * ny + iy.  The non-empty x columns are ix = mx mod nx for |mx| <= mxmax.

template <typename T, int NX_, int NY_>
__device__ __forceinline__ void slab_inverse(cplx<T>* buf, const FftDims& d, const cplx<T>* twx, const cplx<T>* twy) {
    const int NX = NX_ ? NX_ : d.nx;
    const int NY = NY_ ? NY_ : d.ny;
    // y transforms of the non-empty columns (contiguous lines of length NY)
    fft_lines<T, +1, NY_, 0, false>(buf, d.py, d.ax, LineMap{(NX - d.mxmax) % NX, NX, NY}, 1, twy);
    // x transforms of every row iy (lines adjacent in LDS, element stride NY)
    fft_lines<T, +1, NX_, NY_, true>(buf, d.px, NY, LineMap{0, NY, 1}, NY, twx);
}

template <typename T, int NX_, int NY_>
__device__ __forceinline__ void slab_forward(cplx<T>* buf, const FftDims& d, const cplx<T>* twx, const cplx<T>* twy) {
    const int NX = NX_ ? NX_ : d.nx;
    const int NY = NY_ ? NY_ : d.ny;
    fft_lines<T, -1, NX_, NY_, true>(buf, d.px, NY, LineMap{0, NY, 1}, NY, twx);
    fft_lines<T, -1, NY_, 0, false>(buf, d.py, d.ax, LineMap{(NX - d.mxmax) % NX, NX, NY}, 1, twy);
}

template <typename T>
__device__ __forceinline__ void slab_scatter(cplx<T>* buf, int nxy, const BasisTables& t, int ns,
                                             const cplx<T>* src) {
    for (int e = threadIdx.x; e < nxy; e += kThreads) buf[e] = mk<T>(0, 0);
    __syncthreads();
    for (int s = threadIdx.x; s < ns; s += kThreads) buf[t.slab_pos[s]] = src[s];
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ void slab_gather(const cplx<T>* buf, const BasisTables& t, int ns, cplx<T>* dst) {
    for (int s = threadIdx.x; s < ns; s += kThreads) dst[s] = buf[t.slab_pos[s]];
}

enum SlabMode : int { SLAB_HV = 0, SLAB_INV_C, SLAB_INV_R, SLAB_FWD_PRODUCT, SLAB_FWD_REAL };

// One kernel for the slab work of every operation (MODE is a template argument):
//   SLAB_HV          sticks -> inverse -> * V(z, x, y) -> forward -> sticks (in place)
//   SLAB_INV_C / _R  sticks -> inverse -> complex / real grid [row][z][x][y]
//   SLAB_FWD_PRODUCT grid Vr[row / nv] * u[row % nv] -> forward -> sticks
//   SLAB_FWD_REAL    real grid Vr[row] -> forward -> sticks
template <typename T, int NX_, int NY_, int MODE>
__global__ __launch_bounds__(kThreads) void k_slab(FftDims d, BasisTables t, cplx<T>* __restrict__ sticks,
                                                   const T* __restrict__ Vr, const cplx<T>* __restrict__ u,
                                                   int nv, cplx<T>* __restrict__ grid_c, T* __restrict__ grid_r) {
    extern __shared__ __align__(16) unsigned char smem[];
    using C = cplx<T>;
    const int NX = NX_ ? NX_ : d.nx;
    const int NY = NY_ ? NY_ : d.ny;
    const int nxy = NX * NY;
    C* buf = reinterpret_cast<C*>(smem);
    C* twx = buf + nxy;
    C* twy = twx + NX;
    const int z = blockIdx.x;
    const int row = blockIdx.y;
    const long ng = (long)nxy * d.nz;
    load_tw<T>(twx, t, 0, NX);
    load_tw<T>(twy, t, 1, NY);
    C* srow = sticks + ((long)row * d.nz + z) * d.sld;
    if constexpr (MODE == SLAB_HV || MODE == SLAB_INV_C || MODE == SLAB_INV_R) {
        slab_scatter<T>(buf, nxy, t, d.ns, srow);
        slab_inverse<T, NX_, NY_>(buf, d, twx, twy);
        if constexpr (MODE == SLAB_HV) {
            const T* vz = Vr + (long)z * nxy;
            for (int e = threadIdx.x; e < nxy; e += kThreads) {
                const T vv = vz[e];
                buf[e].x *= vv;
                buf[e].y *= vv;
            }
            __syncthreads();
            slab_forward<T, NX_, NY_>(buf, d, twx, twy);
            slab_gather<T>(buf, t, d.ns, srow);
        } else if constexpr (MODE == SLAB_INV_C) {
            C* g = grid_c + row * ng + (long)z * nxy;
            for (int e = threadIdx.x; e < nxy; e += kThreads) g[e] = buf[e];
        } else {
            T* g = grid_r + row * ng + (long)z * nxy;
            for (int e = threadIdx.x; e < nxy; e += kThreads) g[e] = buf[e].x;
        }
    } else {
        const T* vz = Vr + (MODE == SLAB_FWD_PRODUCT ? (long)(row / nv) : (long)row) * ng + (long)z * nxy;
        if constexpr (MODE == SLAB_FWD_PRODUCT) {
            const C* uz = u + (long)(row % nv) * ng + (long)z * nxy;
            for (int e = threadIdx.x; e < nxy; e += kThreads) {
                const T vv = vz[e];
                const C uu = uz[e];
                buf[e] = mk<T>(vv * uu.x, vv * uu.y);
            }
        } else {
            for (int e = threadIdx.x; e < nxy; e += kThreads) buf[e] = mk<T>(vz[e], 0);
        }
        __syncthreads();
        slab_forward<T, NX_, NY_>(buf, d, twx, twy);
        slab_gather<T>(buf, t, d.ns, srow);
    }
}

// Stick rows of nzh consecutive z slabs (nzh * sld elements, contiguous in the sticks
// buffer) to LDS and back, in 16-byte pieces with up to K loads in flight per thread
// before the first LDS write: a loop that waited for each load before its LDS write
// would pay the memory latency once per piece.  The copy back writes only the sphere's
// sticks (index < ns within each slab row), so the padding of the rows is left as it is.
template <typename E, int NT, int K = 8>
__device__ __forceinline__ void stage_rows_in(E* lds, const E* g, int nzh, int sld) {
    static_assert(sizeof(E) == 8 || sizeof(E) == 16, "8- or 16-byte elements");
    constexpr int PER = 16 / sizeof(E);   // elements per piece (sld is a multiple of 32)
    const int n = nzh * sld / PER;
    const float4* src = reinterpret_cast<const float4*>(g);
    float4* dst = reinterpret_cast<float4*>(lds);
    for (int b = 0; b < n; b += K * NT) {
        float4 r[K];
        sfor<0, K>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            r[k] = src[min(b + (int)threadIdx.x + k * NT, n - 1)];
        });
        // every lane writes (the lanes past the end write the last piece again, with its
        // own value): a guarded store would let the compiler sink each load into its
        // guard and wait for it there, one load at a time
        sfor<0, K>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            dst[min(b + (int)threadIdx.x + k * NT, n - 1)] = r[k];
        });
    }
}
template <typename E, int NT, int K = 8>
__device__ __forceinline__ void stage_rows_out(E* g, const E* lds, int nzh, int sld, int ns) {
    constexpr int PER = 16 / sizeof(E);
    const int n = nzh * sld / PER;
    const float4* src = reinterpret_cast<const float4*>(lds);
    float4* dst = reinterpret_cast<float4*>(g);
    for (int b = 0; b < n; b += K * NT) {
        float4 r[K];
        sfor<0, K>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            r[k] = src[min(b + (int)threadIdx.x + k * NT, n - 1)];
        });
        sfor<0, K>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const int i = b + (int)threadIdx.x + k * NT;
            if (i < n) {
                const int e = i * PER;
                const int ein = e - (e / sld) * sld;   // index within the slab row
                if (ein + PER <= ns) {
                    dst[i] = r[k];
                } else if (PER == 2 && ein < ns) {
                    reinterpret_cast<float2*>(dst + i)[0] = make_float2(r[k].x, r[k].y);
                }
            }
        });
    }
}

// Slab pass of H (V multiply), FP32, NX = NY = NL, with every line in registers: a
// workgroup of 256 threads (four waves) takes ZG = 256 / NL consecutive z slabs of one
// row.  Lines are read at clamped indices and masked afterwards, so the loads of a
// line issue back to back.
//   1. the ZG stick rows are copied to LDS (stage_rows_in);
//   2. one thread per (slab, non-empty x column), packed into the first ZG * ax
//      threads: its y line from the stick row (zeros outside the column's my range),
//      inverse y DFT, written to the transpose plane [slab][iy][column];
//   3. one thread per (slab, iy): its x line (zeros at empty columns), inverse x DFT,
//      times V(z, x, y), forward x DFT, non-empty columns written back;
//   4. one thread per (slab, column): forward y DFT, the column's my range written to
//      the stick row;
//   5. stick rows copied back.
// The stick rows and the transpose plane share LDS: every thread holds its line in
// registers across the barrier that separates reading one from writing the other.
// MX >= 0: the sphere's largest |mx| and |my| are at most MX, and |mx| reaches it (the
// launcher checks both), so the x lines read their non-empty columns and write back
// the needed outputs at fixed indices, and the y lines hold zeros at the frequencies
// |my| > MX as compile-time constants: the DFT stages that only see those zeros, and the
// outputs of the forward transforms that are never stored, are not computed.
// (A zero-padded (column, my) square for the y lines as well measured no faster.)
template <int NL, int MX>
__global__ __launch_bounds__(256) void k_slab_hv_reg(FftDims d, BasisTables t, float2* __restrict__ sticks,
                                                     const float* __restrict__ Vr) {
    constexpr int ZG = 256 / NL;
    constexpr int HALF = (NL + 1) / 2;   // index i holds frequency i (i < HALF) or i - NL
    // frequency my of index i lies outside the compiled y range (a zero of every y line)
    constexpr auto y_out = [](int my) { return MX >= 0 && (my < -MX || my > MX); };
    extern __shared__ __align__(16) unsigned char smem[];
    float2* lds = reinterpret_cast<float2*>(smem);
    const int mxmax = MX >= 0 ? MX : d.mxmax, sld = d.sld, nz = d.nz;
    const int ax = 2 * mxmax + 1;
    const int axp = ax | 1;
    const int z0 = blockIdx.x * ZG, row = blockIdx.y;
    const int tid = threadIdx.x;
    const int zl = tid / NL, li = tid - zl * NL;   // x passes: (slab, iy)
    const int zc = tid / ax, lc = tid - zc * ax;   // y passes: (slab, column)
    const int nzh = min(ZG, nz - z0);
    const bool zact = zl < nzh && zl < ZG;
    const bool col = zc < nzh;
    float2* g = sticks + ((long)row * nz + z0) * sld;
    stage_rows_in<float2, 256>(lds, g, nzh, sld);
    __syncthreads();

    int s0 = 0, my0 = 0;
    float2 v[NL], X[NL];
    if (col) {
        s0 = t.col_start[lc];
        my0 = t.col_my0[lc];
        const float2* sr = lds + zc * sld + s0 - my0;
        sfor<0, NL>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int my = i < HALF ? i : i - NL;
            if constexpr (y_out(my)) {
                v[i] = make_float2(0.f, 0.f);
            } else {
                const float2 val = sr[min(max(my, my0), -my0)];
                v[i] = (my >= my0 && my <= -my0) ? val : make_float2(0.f, 0.f);
            }
        });
    }
    __syncthreads();
    float2* tp = lds + (long)zl * NL * axp;     // transpose plane of the x-pass slab: [iy][column]
    float2* tc = lds + (long)zc * NL * axp;     // transpose plane of the y-pass slab
    if (col) {
        dft_reg<float, +1, NL, 1>(v, X);
        sfor<0, NL>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            tc[i * axp + lc] = X[i];
        });
    }
    __syncthreads();
    if (zact) {
        const float2* tr = tp + li * axp + mxmax;
        sfor<0, NL>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int mx = i < HALF ? i : i - NL;
            const float2 val = tr[min(max(mx, -mxmax), mxmax)];
            v[i] = (mx >= -mxmax && mx <= mxmax) ? val : make_float2(0.f, 0.f);
        });
        dft_reg<float, +1, NL, 1>(v, X);
        const float* vz = Vr + (long)(z0 + zl) * NL * NL + li;
        sfor<0, NL>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const float vv = vz[i * NL];
            X[i].x *= vv;
            X[i].y *= vv;
        });
        dft_reg<float, -1, NL, 1>(X, v);
        float2* tw = tp + li * axp + mxmax;
        sfor<0, NL>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int mx = i < HALF ? i : i - NL;
            if (mx >= -mxmax && mx <= mxmax) tw[mx] = v[i];
        });
    }
    __syncthreads();
    if (col) {
        sfor<0, NL>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            v[i] = tc[i * axp + lc];
        });
    }
    __syncthreads();
    if (col) {
        dft_reg<float, -1, NL, 1>(v, X);
        float2* sw = lds + zc * sld + s0 - my0;
        sfor<0, NL>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int my = i < HALF ? i : i - NL;
            if constexpr (!y_out(my)) {
                if (my >= my0 && my <= -my0) sw[my] = X[i];
            }
        });
    }
    __syncthreads();
    stage_rows_out<float2, 256>(g, lds, nzh, sld, d.ns);
}

// ---------------------------------------------- FP64 slab pass, lines on lane quads ---
// A double line of length NL does not fit one lane's registers, so each line is held by
// the four lanes of a DPP quad (lanes 4u .. 4u + 3; lane t = 0..3 of the quad), NL / 4
// values each, and split by one radix-4 step whose butterflies combine values across the
// quad in two radix-2 exchanges (quad_perm [1, 0, 3, 2] and [2, 3, 0, 1]).  All lanes of
// a quad always take the same branch.

template <int CTRL> __device__ __forceinline__ double quad_swap(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}
// v of lane t ^ 1 (CTRL 0xB1) or t ^ 2 (CTRL 0x4E)
template <int CTRL> __device__ __forceinline__ double2 quad_swap(double2 v) {
    return make_double2(quad_swap<CTRL>(v.x), quad_swap<CTRL>(v.y));
}
constexpr int kSwap1 = 0xB1, kSwap2 = 0x4E;

// Per-lane constants of the quad transforms: sign factors of the two exchanges and the
// quarter-turn factor of lane 3, so that every butterfly is branch-free multiply-adds.
struct QuadLane {
    int t;          // lane in the quad
    double s1, s2;  // -1 for the lanes that take (other - mine) in the t^1 / t^2 exchange
    double qc, qs;  // exp(SIGN 2 pi i / 4) for lane 3 (SIGN +1: (0, 1)), 1 otherwise
};
template <int SIGN> __device__ __forceinline__ QuadLane quad_lane(int t) {
    QuadLane L;
    L.t = t;
    L.s1 = (t & 1) ? -1.0 : 1.0;
    L.s2 = (t >> 1) ? -1.0 : 1.0;
    L.qc = t == 3 ? 0.0 : 1.0;
    L.qs = t == 3 ? (double)SIGN : 0.0;
    return L;
}
// mine * sign + other
__device__ __forceinline__ double2 quad_bfly(double2 mine, double2 other, double sg) {
    return make_double2(fma(sg, mine.x, other.x), fma(sg, mine.y, other.y));
}
__device__ __forceinline__ double2 cmul_d(double2 a, double c, double s) {
    return make_double2(fma(a.x, c, -a.y * s), fma(a.x, s, a.y * c));
}

// Position of the lane's block in the output of quad_dft_dit (and in the input of
// quad_dft_dif): lane t holds indices k + (N / 4) quad_block(t).
__device__ __forceinline__ int quad_block(int t) { return (t >> 1) + 2 * (t & 1); }

// Length-N DFT (exponent sign SIGN) of a line on a quad, decimation in time: lane t
// holds x[4j + t] in v[j]; on return it holds X[k + (N / 4) quad_block(t)] in v[k].
// With t = t0 + 2 t1 and y_t = w^(t k) E_t[k] (E_t the length-N/4 DFT of the lane's
// values): the exchange across t1 forms B_t0(t1) = y_t0 + (-1)^t1 y_(t0+2), the one
// across t0 forms X[k + (N/4)(t1 + 2 t0)] = B_0(t1) + (-1)^t0 w4^t1 B_1(t1).
// tw[e] = exp(2 pi i e / N), e < N (conjugated for SIGN -1).
template <int SIGN, int N>
__device__ __forceinline__ void quad_dft_dit(double2 (&v)[N / 4], const QuadLane& L, const double2* tw) {
    constexpr int Q = N / 4;
    double2 E[Q];
    dft_reg<double, SIGN, Q, 1>(v, E);
    sfor<0, Q>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        double2 y = E[k];
        if constexpr (k > 0) {
            const double2 w = tw[(L.t * k) % N];
            y = cmul_d(y, w.x, SIGN * w.y);
        }
        const double2 bq = cmul_d(quad_bfly(y, quad_swap<kSwap2>(y), L.s2), L.qc, L.qs);
        v[k] = quad_bfly(bq, quad_swap<kSwap1>(bq), L.s1);
    });
}

// Decimation in frequency: lane t holds x[n + (N / 4) quad_block(t)] in v[n]; on return
// it holds X[4k + t] in v[k].  With s = quad_block(t) = s0 + 2 s1 (s0 = t >> 1,
// s1 = t & 1): the exchange across s1 forms C_s0(s1) = x_s0 + (-1)^s1 x_(s0+2), the one
// across s0 forms Z_t = C_0(s1) + (-1)^s0 w4^s1 C_1(s1), and lane t finishes with the
// length-N/4 DFT of w^(t n) Z_t[n].
template <int SIGN, int N>
__device__ __forceinline__ void quad_dft_dif(double2 (&v)[N / 4], const QuadLane& L, const double2* tw) {
    constexpr int Q = N / 4;
    double2 a[Q];
    sfor<0, Q>([&](auto nc) {
        constexpr int n = decltype(nc)::value;
        const double2 x = v[n];
        const double2 c = cmul_d(quad_bfly(x, quad_swap<kSwap1>(x), L.s1), L.qc, L.qs);
        double2 z = quad_bfly(c, quad_swap<kSwap2>(c), L.s2);
        if constexpr (n > 0) {
            const double2 w = tw[(L.t * n) % N];
            z = cmul_d(z, w.x, SIGN * w.y);
        }
        a[n] = z;
    });
    dft_reg<double, SIGN, Q, 1>(a, v);
}

// Slab data elements (double2) of the lane-quad kernel: ZG = 64 / nl stick rows or
// transpose planes, whichever is larger (they share LDS).
__host__ __device__ inline int quad64_data_elems(const FftDims& d, int nl) {
    const int zg = 64 / nl, axp = (2 * d.mxmax + 1) | 1;
    const int a = zg * d.sld, b = zg * nl * axp;
    return a > b ? a : b;
}

// Threads of the lane-quad slab passes of H and of the forward transform: one quad per
// (slab, iy) line of the x pass, ZG = 64 / NL slabs (192 threads for NL = 24 and 48: no
// wave without an x line).  The density pass keeps 256 threads: it is held to two waves
// per SIMD by its accumulators, and three-wave workgroups would leave SIMD slots empty.
constexpr int quad64_threads(int nl) { return 4 * (64 / nl) * nl; }

// Slab pass of H (V multiply), FP64, NX = NY = NL (a multiple of 4): the register slab
// pass with every line on a lane quad.  A workgroup of quad64_threads(NL) threads takes
// ZG = 64 / NL consecutive z slabs of one row: stick rows to LDS; one quad per (slab,
// non-empty column): inverse y DFT into the transpose plane [slab][iy][column]; one
// quad per (slab, iy): inverse x DFT (decimation in time), times V(z, x, y), forward x
// DFT (decimation in frequency, which takes the input in the order the inverse left
// it), non-empty columns written back; one quad per (slab, column): forward y DFT into
// the stick row; stick rows back.  Stick rows and transpose planes share LDS (every
// quad holds its line in registers across the barrier between).
template <int NL>
__global__ __launch_bounds__(quad64_threads(NL)) void k_slab_hv_quad64(FftDims d, BasisTables t,
                                                                       double2* __restrict__ sticks,
                                                                       const double* __restrict__ Vr) {
    static_assert(NL % 4 == 0 && NL <= 64, "lines split over a lane quad");
    constexpr int Q = NL / 4, H = NL / 2;
    constexpr int ZG = 64 / NL, NT = quad64_threads(NL);
    extern __shared__ __align__(16) unsigned char smem[];
    double2* lds = reinterpret_cast<double2*>(smem);
    const int mxmax = d.mxmax, sld = d.sld, nz = d.nz;
    const int ax = 2 * mxmax + 1;
    const int axp = ax | 1;
    const int z0 = blockIdx.x * ZG, row = blockIdx.y;
    const int tid = threadIdx.x, u = tid >> 2, tl = tid & 3;
    const int blk = Q * quad_block(tl);
    const int zl = u / NL, li = u - zl * NL;   // x passes: (slab, iy)
    const int zc = u / ax, lc = u - zc * ax;   // y passes: (slab, column)
    const int nzh = min(ZG, nz - z0);
    const bool xact = zl < nzh;
    const bool col = zc < nzh;
    double2* g = sticks + ((long)row * nz + z0) * sld;
    const int ns = d.ns;
    // twiddles exp(2 pi i e / NL) behind the slab data
    double2* tw = lds + quad64_data_elems(d, NL);
    if (tid < NL) {
        const double ang = 6.283185307179586476925 * tid / NL;
        tw[tid] = make_double2(cos(ang), sin(ang));
    }
    stage_rows_in<double2, NT, 4>(lds, g, nzh, sld);
    __syncthreads();
    const QuadLane Lp = quad_lane<+1>(tl), Lm = quad_lane<-1>(tl);

    int s0 = 0, my0 = 0;
    double2 v[Q];
    if (col) {
        s0 = t.col_start[lc];
        my0 = t.col_my0[lc];
        const double2* sr = lds + zc * sld + s0 - my0;
        sfor<0, Q>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const int iy = 4 * j + tl;
            const int my = iy < H ? iy : iy - NL;
            const double2 val = sr[min(max(my, my0), -my0)];
            v[j] = (my >= my0 && my <= -my0) ? val : make_double2(0.0, 0.0);
        });
    }
    __syncthreads();
    double2* tp = lds + (long)zl * NL * axp;   // transpose plane of the x-pass slab: [iy][column]
    double2* tc = lds + (long)zc * NL * axp;   // transpose plane of the y-pass slab
    if (col) {
        quad_dft_dit<+1, NL>(v, Lp, tw);
        sfor<0, Q>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            tc[(k + blk) * axp + lc] = v[k];
        });
    }
    __syncthreads();
    if (xact) {
        const double2* tr = tp + li * axp + mxmax;
        sfor<0, Q>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            const int ix = 4 * j + tl;
            const int mx = ix < H ? ix : ix - NL;
            const double2 val = tr[min(max(mx, -mxmax), mxmax)];
            v[j] = (mx >= -mxmax && mx <= mxmax) ? val : make_double2(0.0, 0.0);
        });
        quad_dft_dit<+1, NL>(v, Lp, tw);
        const double* vz = Vr + (long)(z0 + zl) * NL * NL + li;
        sfor<0, Q>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const double vv = vz[(k + blk) * NL];
            v[k].x *= vv;
            v[k].y *= vv;
        });
        quad_dft_dif<-1, NL>(v, Lm, tw);
        double2* tw2 = tp + li * axp + mxmax;
        sfor<0, Q>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const int ix = 4 * k + tl;
            const int mx = ix < H ? ix : ix - NL;
            if (mx >= -mxmax && mx <= mxmax) tw2[mx] = v[k];
        });
    }
    __syncthreads();
    if (col) {
        sfor<0, Q>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            v[j] = tc[(4 * j + tl) * axp + lc];
        });
    }
    __syncthreads();
    if (col) {
        quad_dft_dit<-1, NL>(v, Lm, tw);
        double2* sw = lds + zc * sld + s0 - my0;
        sfor<0, Q>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const int iy = k + blk;
            const int my = iy < H ? iy : iy - NL;
            if (my >= my0 && my <= -my0) sw[my] = v[k];
        });
    }
    __syncthreads();
    for (int zz = 0; zz < nzh; ++zz)
        for (int e = tid; e < ns; e += NT) g[(long)zz * sld + e] = lds[zz * sld + e];
}

// Density on lane quads (FP64, NX = NY = NL): for ZG = 64 / NL slabs of PB consecutive
// perturbations, loop over the nv stick rows of their bands: inverse y into the transpose
// plane, inverse x (decimation in time: the lane holds x = k + (NL/4) quad_block(t) of
// line iy), accumulate Re(conj(u_v) f) in registers; scaled sums written at the end.
// The perturbations of a workgroup share each u_v (read once from memory, then from
// cache).
template <int NL, int PB>
__global__ __launch_bounds__(256) void k_slab_density_quad64(FftDims d, BasisTables t,
                                                             const double2* __restrict__ sticks, int npert, int nv,
                                                             const double2* __restrict__ u, double scale,
                                                             double* __restrict__ dn) {
    constexpr int Q = NL / 4, H = NL / 2;
    constexpr int ZG = 64 / NL;
    extern __shared__ __align__(16) unsigned char smem[];
    double2* lds = reinterpret_cast<double2*>(smem);
    const int mxmax = d.mxmax, sld = d.sld, nz = d.nz;
    const int ax = 2 * mxmax + 1;
    const int axp = ax | 1;
    const int z0 = blockIdx.x * ZG, p0 = blockIdx.y * PB;
    const int np = min(PB, npert - p0);
    const int tid = threadIdx.x, uq = tid >> 2, tl = tid & 3;
    const int blk = Q * quad_block(tl);
    const int zl = uq / NL, li = uq - zl * NL;   // x passes: (slab, iy)
    const int zc = uq / ax, lc = uq - zc * ax;   // y passes: (slab, column)
    const int nzh = min(ZG, nz - z0);
    const bool xact = zl < nzh;
    const bool col = zc < nzh;
    const long ng = (long)NL * NL * nz;
    double2* tw = lds + quad64_data_elems(d, NL);
    if (tid < NL) {
        const double ang = 6.283185307179586476925 * tid / NL;
        tw[tid] = make_double2(cos(ang), sin(ang));
    }
    const QuadLane Lp = quad_lane<+1>(tl);
    const int s0 = col ? t.col_start[lc] : 0, my0 = col ? t.col_my0[lc] : 0;
    double2* tp = lds + (long)zl * NL * axp;
    double2* tc = lds + (long)zc * NL * axp;
    double acc[PB][Q];
#pragma unroll
    for (int q = 0; q < PB; ++q)
#pragma unroll
        for (int k = 0; k < Q; ++k) acc[q][k] = 0.0;
    for (int v = 0; v < nv; ++v) {
#pragma unroll
        for (int q = 0; q < PB; ++q) {
            if (q >= np) break;   // uniform over the workgroup
            const double2* g = sticks + (((long)(p0 + q) * nv + v) * nz + z0) * sld;
            __syncthreads();   // the previous row's transpose planes are read
            stage_rows_in<double2, 256, 4>(lds, g, nzh, sld);
            __syncthreads();
            double2 w[Q];
            if (col) {
                const double2* sr = lds + zc * sld + s0 - my0;
                sfor<0, Q>([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    const int iy = 4 * j + tl;
                    const int my = iy < H ? iy : iy - NL;
                    const double2 val = sr[min(max(my, my0), -my0)];
                    w[j] = (my >= my0 && my <= -my0) ? val : make_double2(0.0, 0.0);
                });
            }
            __syncthreads();
            if (col) {
                quad_dft_dit<+1, NL>(w, Lp, tw);
                sfor<0, Q>([&](auto kc) {
                    constexpr int k = decltype(kc)::value;
                    tc[(k + blk) * axp + lc] = w[k];
                });
            }
            __syncthreads();
            if (xact) {
                const double2* tr = tp + li * axp + mxmax;
                sfor<0, Q>([&](auto jc) {
                    constexpr int j = decltype(jc)::value;
                    const int ix = 4 * j + tl;
                    const int mx = ix < H ? ix : ix - NL;
                    const double2 val = tr[min(max(mx, -mxmax), mxmax)];
                    w[j] = (mx >= -mxmax && mx <= mxmax) ? val : make_double2(0.0, 0.0);
                });
                quad_dft_dit<+1, NL>(w, Lp, tw);
                const double2* uz = u + (long)v * ng + (long)(z0 + zl) * NL * NL + li;
                sfor<0, Q>([&](auto kc) {
                    constexpr int k = decltype(kc)::value;
                    const double2 uu = uz[(k + blk) * NL];
                    acc[q][k] += uu.x * w[k].x + uu.y * w[k].y;
                });
            }
        }
    }
    if (xact) {
#pragma unroll
        for (int q = 0; q < PB; ++q) {
            if (q >= np) break;
            double* out = dn + (long)(p0 + q) * ng + (long)(z0 + zl) * NL * NL + li;
#pragma unroll
            for (int k = 0; k < Q; ++k) out[(k + blk) * NL] = scale * acc[q][k];
        }
    }
}

// Forward slab pass on lane quads (FP64, NX = NY = NL): grid V_r[row / nv] u[row % nv]
// (PRODUCT) or V_r[row] (real) -> forward x (decimation in frequency on the lane's
// contiguous x block) into the transpose plane -> forward y (decimation in time) -> the
// row's sticks.
template <int NL, bool PRODUCT>
__global__ __launch_bounds__(quad64_threads(NL)) void k_slab_fwd_quad64(FftDims d, BasisTables t,
                                                                        double2* __restrict__ sticks,
                                                                        const double* __restrict__ Vr,
                                                                        const double2* __restrict__ u, int nv) {
    constexpr int Q = NL / 4, H = NL / 2;
    constexpr int ZG = 64 / NL, NT = quad64_threads(NL);
    extern __shared__ __align__(16) unsigned char smem[];
    double2* lds = reinterpret_cast<double2*>(smem);
    const int mxmax = d.mxmax, sld = d.sld, nz = d.nz;
    const int ax = 2 * mxmax + 1;
    const int axp = ax | 1;
    const int z0 = blockIdx.x * ZG, row = blockIdx.y;
    const int tid = threadIdx.x, uq = tid >> 2, tl = tid & 3;
    const int blk = Q * quad_block(tl);
    const int zl = uq / NL, li = uq - zl * NL;
    const int zc = uq / ax, lc = uq - zc * ax;
    const int nzh = min(ZG, nz - z0);
    const bool xact = zl < nzh;
    const bool col = zc < nzh;
    const long ng = (long)NL * NL * nz;
    double2* tw = lds + quad64_data_elems(d, NL);
    if (tid < NL) {
        const double ang = 6.283185307179586476925 * tid / NL;
        tw[tid] = make_double2(cos(ang), sin(ang));
    }
    __syncthreads();
    const QuadLane Lm = quad_lane<-1>(tl);
    double2 w[Q];
    double2* tp = lds + (long)zl * NL * axp;
    double2* tc = lds + (long)zc * NL * axp;
    if (xact) {
        const long zo = (long)(z0 + zl) * NL * NL + li;
        const double* vz = Vr + (PRODUCT ? (long)(row / nv) : (long)row) * ng + zo;
        sfor<0, Q>([&](auto nc) {
            constexpr int n = decltype(nc)::value;
            const double vv = vz[(n + blk) * NL];
            if constexpr (PRODUCT) {
                const double2 uu = u[(long)(row % nv) * ng + zo + (n + blk) * NL];
                w[n] = make_double2(vv * uu.x, vv * uu.y);
            } else {
                w[n] = make_double2(vv, 0.0);
            }
        });
        quad_dft_dif<-1, NL>(w, Lm, tw);
        double2* tw2 = tp + li * axp + mxmax;
        sfor<0, Q>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const int ix = 4 * k + tl;
            const int mx = ix < H ? ix : ix - NL;
            if (mx >= -mxmax && mx <= mxmax) tw2[mx] = w[k];
        });
    }
    __syncthreads();
    int s0 = 0, my0 = 0;
    if (col) {
        s0 = t.col_start[lc];
        my0 = t.col_my0[lc];
        sfor<0, Q>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            w[j] = tc[(4 * j + tl) * axp + lc];
        });
    }
    __syncthreads();
    if (col) {
        quad_dft_dit<-1, NL>(w, Lm, tw);
        double2* sw = lds + zc * sld + s0 - my0;
        sfor<0, Q>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const int iy = k + blk;
            const int my = iy < H ? iy : iy - NL;
            if (my >= my0 && my <= -my0) sw[my] = w[k];
        });
    }
    __syncthreads();
    double2* g = sticks + ((long)row * nz + z0) * sld;
    const int ns = d.ns;
    stage_rows_out<double2, NT, 4>(g, lds, nzh, sld, ns);
}

constexpr int kMaxAcc = 24;

// Density: dn_i(z, x, y) = scale * Re sum_v conj(u_v(z, x, y)) Inv(sticks[i * nv + v])(z, x, y).
template <int NX_, int NY_>
__global__ __launch_bounds__(kThreads) void k_slab_density(FftDims d, BasisTables t,
                                                           const double2* __restrict__ sticks, int nv,
                                                           const double2* __restrict__ u, double scale,
                                                           double* __restrict__ dn) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int NX = NX_ ? NX_ : d.nx;
    const int NY = NY_ ? NY_ : d.ny;
    const int nxy = NX * NY;
    double2* buf = reinterpret_cast<double2*>(smem);
    double2* twx = buf + nxy;
    double2* twy = twx + NX;
    const int z = blockIdx.x;
    const int pert = blockIdx.y;
    const long ng = (long)nxy * d.nz;
    load_tw<double>(twx, t, 0, NX);
    load_tw<double>(twy, t, 1, NY);
    double acc[kMaxAcc];
#pragma unroll
    for (int j = 0; j < kMaxAcc; ++j) acc[j] = 0.0;
    for (int v = 0; v < nv; ++v) {
        const double2* srow = sticks + (((long)pert * nv + v) * d.nz + z) * d.sld;
        slab_scatter<double>(buf, nxy, t, d.ns, srow);
        slab_inverse<double, NX_, NY_>(buf, d, twx, twy);
        const double2* uz = u + (long)v * ng + (long)z * nxy;
#pragma unroll
        for (int j = 0; j < kMaxAcc; ++j) {
            const int e = threadIdx.x + j * kThreads;
            if (e < nxy) {
                const double2 uu = uz[e];
                const double2 f = buf[e];
                acc[j] += uu.x * f.x + uu.y * f.y;     // Re(conj(u) f)
            }
        }
        __syncthreads();
    }
    double* out = dn + (long)pert * ng + (long)z * nxy;
#pragma unroll
    for (int j = 0; j < kMaxAcc; ++j) {
        const int e = threadIdx.x + j * kThreads;
        if (e < nxy) out[e] = scale * acc[j];
    }
}

// Grid layout change between C order [ix][iy][iz] and z-major [iz][ix][iy]; g indexes
// the output.
__global__ void k_transpose_grid(int nx, int ny, int nz, const double* __restrict__ in, double* __restrict__ out,
                                 int to_zmajor) {
    const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long ng = (long)nx * ny * nz;
    if (g >= ng) return;
    const int row = blockIdx.y;
    long src;
    if (to_zmajor) {
        const int iz = (int)(g / ((long)nx * ny));
        const int rem = (int)(g - (long)iz * nx * ny);
        const int ix = rem / ny, iy = rem - (rem / ny) * ny;
        src = ((long)ix * ny + iy) * nz + iz;
    } else {
        const int ix = (int)(g / ((long)ny * nz));
        const int rem = (int)(g - (long)ix * ny * nz);
        const int iy = rem / nz, iz = rem - (rem / nz) * nz;
        src = ((long)iz * nx + ix) * ny + iy;
    }
    out[(long)row * ng + g] = in[(long)row * ng + src];
}

// ------------------------------------ FP64 paired sticks-to-sphere pass on lane quads ---
// The FP64 form of the register sticks-to-sphere pass: a z stick of NZ doubles is held
// by the four lanes of a DPP quad (NZ / 4 values each) and transformed with the lane-quad
// DFT of the slab pass.  A workgroup of 256 threads takes kQuadStickGroup front sticks
// (quads 0 .. 31, waves 0 and 1) and their mirrors ns - 1 - s (quads 32 .. 63, waves 2
// and 3); the two half-sphere rows are separated as in k_sticks_to_sphere_pair_reg.
// (The sphere-to-sticks direction on lane quads measured slower than the LDS form, with
// and without an LDS tile for whole-row stores, and is not used.)
constexpr int kQuadStickGroup = 32;

// Sticks of packed row pr -> half-sphere rows a, b with the epilogue EPI_SHIFTED_H of
// k_sticks_to_sphere_pair (out = F + (kin - shift) x, optional partial sums of
// Re<x, out> per row and workgroup), FP64.
template <int NZ>
__global__ __launch_bounds__(256) void k_sticks_to_sphere_pair_quad64(
    FftDims d, BasisTables t, const double2* __restrict__ sticks, int nrows, int group, double2* __restrict__ out,
    long ld_out, const double2* __restrict__ x, long ld_x, const double* __restrict__ kin,
    const double* __restrict__ shift, int nshift, double* __restrict__ dot_part) {
    static_assert(NZ % 4 == 0 && NZ <= 64, "sticks split over a lane quad");
    constexpr int Q = NZ / 4, HALF = (NZ + 1) / 2;
    constexpr int GS = kQuadStickGroup, NT = 256, LQ = 4;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[2][NT];
    double2* bufF = reinterpret_cast<double2*>(smem);
    double2* bufM = bufF + d.sgp_max;
    double2* tw = bufM + d.sgp_max;   // exp(2 pi i e / NZ), e < NZ
    const int nfront = (d.ns + 1) / 2;
    const int s0 = blockIdx.x * GS, pr = blockIdx.y;
    const int nf = min(GS, nfront - s0);
    const int kb = t.stick_start[s0], ke = t.stick_start[s0 + nf];
    const int tid = threadIdx.x;
    if (tid < NZ) {
        const double ang = 6.283185307179586476925 * tid / NZ;
        tw[tid] = make_double2(cos(ang), sin(ang));
    }
    const int u = tid >> 2, tl = tid & 3;
    const bool mir = u >= GS;                   // wave-uniform
    const int j = mir ? u - GS : u;
    const int sf = s0 + j;
    double2 v[Q];
    if (j < nf) {
        const int sk = mir ? d.ns - 1 - sf : sf;
        const double2* src = sticks + (long)pr * NZ * d.sld + sk;
        sfor<0, Q>([&](auto jc) {
            constexpr int jj = decltype(jc)::value;
            v[jj] = src[(long)(4 * jj + tl) * d.sld];
        });
    }
    __syncthreads();   // the twiddle table is complete
    if (j < nf) {
        const QuadLane L = quad_lane<-1>(tl);
        quad_dft_dit<-1, NZ>(v, L, tw);
        const int blk = Q * quad_block(tl);
        const int ks = t.stick_start[sf] - kb, kz = (t.stick_start[sf + 1] - t.stick_start[sf] - 1) / 2;
        double2* line = (mir ? bufM : bufF) + ks + kz;
        const int sgn = mir ? -1 : 1;           // the mirror stick's mz lands at the front entry of -mz
        sfor<0, Q>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const int i = k + blk;
            const int mz = i < HALF ? i : i - NZ;
            if (mz >= -kz && mz <= kz) line[sgn * mz] = v[k];
        });
    }
    __syncthreads();
    const int c = (d.npw - 1) / 2;
    const int k1 = min(ke, c + 1);
    const double half = 0.5 / ((double)d.nx * d.ny * d.nz);
    const PairRows rw = pair_rows(pr, group, nrows);
    const int ra = rw.a, rb = ra + 1;
    const bool has_b = rw.has_b;
    const double sha = shift[ra % nshift], shb = has_b ? shift[rb % nshift] : 0.0;
    double2* oa = out + (long)ra * ld_out;
    double2* ob = oa + ld_out;
    const double2* xa = x + (long)ra * ld_x;
    const double2* xb = xa + ld_x;
    double acca = 0.0, accb = 0.0;
    // LQ entries per thread at a time, their kinetic energies and x values loaded before
    // the first is used (clamped indices, so every load is in bounds)
    for (int e0 = kb + tid; e0 < k1; e0 += LQ * NT) {
        double kk[LQ];
        double2 xva[LQ], xvb[LQ];
        sfor<0, LQ>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const int k = min(e0 + q * NT, k1 - 1);
            kk[q] = kin[k];
            xva[q] = xa[k];
            xvb[q] = has_b ? xb[k] : make_double2(0.0, 0.0);
        });
        sfor<0, LQ>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const int k = e0 + q * NT;
            if (k < k1) {
                const double2 W = bufF[k - kb], Wm = bufM[k - kb];
                const double w = k == c ? 1.0 : 2.0;
                {
                    const double2 xv = xva[q];
                    const double dk = kk[q] - sha;
                    const double2 ov = make_double2(half * (W.x + Wm.x) + dk * xv.x, half * (W.y - Wm.y) + dk * xv.y);
                    oa[k] = ov;
                    acca += w * (xv.x * ov.x + xv.y * ov.y);
                }
                if (has_b) {
                    const double2 xv = xvb[q];
                    const double dk = kk[q] - shb;
                    const double2 ov = make_double2(half * (W.y + Wm.y) + dk * xv.x, half * (Wm.x - W.x) + dk * xv.y);
                    ob[k] = ov;
                    accb += w * (xv.x * ov.x + xv.y * ov.y);
                }
            }
        });
    }
    if (dot_part) {
        red[0][tid] = acca;
        red[1][tid] = accb;
        __syncthreads();
        for (int s = NT / 2; s > 0; s >>= 1) {
            if (tid < s) {
                red[0][tid] += red[0][tid + s];
                red[1][tid] += red[1][tid + s];
            }
            __syncthreads();
        }
        if (tid == 0) {
            dot_part[(long)ra * gridDim.x + blockIdx.x] = red[0][0];
            if (has_b) dot_part[(long)rb * gridDim.x + blockIdx.x] = red[1][0];
        }
    }
}

// ------------------------------------------------------------------ host side ------

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
void check_rows(int nrows) { PDEP_REQUIRE(nrows <= 65535, PDEP_EINVAL, "too many rows for one transform launch"); }
void check_sticks(const FftDims& d) { check_stages(d.pz, sticks_per_group<float>(d.nz), "z sticks"); }
void check_slab(const FftDims& d) {
    check_stages(d.py, d.ax, "y columns");
    check_stages(d.px, d.ny, "x rows");
}

template <typename T> size_t stick_lds(const FftDims& d) {
    return sizeof(cplx<T>) * ((size_t)sticks_per_group<T>(d.nz) * d.nz + d.nz);
}
template <typename T> size_t slab_lds(const FftDims& d) {
    return sizeof(cplx<T>) * ((size_t)d.nx * d.ny + d.nx + d.ny);
}
// The register stick passes apply to FP32 lines of a compiled length up to 48 whose
// group staging fits the 64 KB of LDS one workgroup may use.
bool stick_reg_ok(const FftDims& d) {
    const bool len = d.nz == 16 || d.nz == 24 || d.nz == 32 || d.nz == 48;
    return len && d.sg_max > 0 && (size_t)d.sg_max * sizeof(float2) <= 65536;
}
template <typename T> dim3 stick_grid(const FftDims& d, int nrows) {
    return dim3((d.ns + sticks_per_group<T>(d.nz) - 1) / sticks_per_group<T>(d.nz), nrows);
}

// Compile-time size dispatch: f.template operator()<N>() for the supported constant
// sizes, N = 0 (run-time sizes) otherwise.
template <typename F> void with_n(int n, F&& f) {
    switch (n) {
        case 16: f.template operator()<16>(); break;
        case 24: f.template operator()<24>(); break;
        case 32: f.template operator()<32>(); break;
        case 48: f.template operator()<48>(); break;
        case 64: f.template operator()<64>(); break;
        case 96: f.template operator()<96>(); break;
        default: f.template operator()<0>(); break;
    }
}
template <typename F> void with_nxy(int nx, int ny, F&& f) {
    if (nx != ny) { f.template operator()<0>(); return; }
    with_n(nx, f);
}

}  // namespace

AxisPlan make_axis_plan(int n) {
    AxisPlan p;
    p.n = n;
    const CPlan c = cplan(n);
    int prod = 1;
    for (int s = 0; s < c.nst; ++s) { p.rad[p.nst++] = c.rad[s]; prod *= c.rad[s]; }
    PDEP_REQUIRE(prod == n && n > 1, PDEP_EINVAL, "grid sizes must be products of 2s and 3s");
    return p;
}

template <typename T>
void launch_sphere_to_sticks(const FftDims& d, const BasisTables& t, const cplx<T>* in, long ld_in, int nrows,
                             const double* gscale, cplx<T>* sticks, hipStream_t s) {
    if (nrows <= 0) return;
    check_sticks(d);
    check_rows(nrows);
    const double sp = (double)d.npw * sizeof(cplx<T>), sk = (double)d.nz * d.ns * sizeof(cplx<T>);
    ProfScope prof_(sizeof(T) == sizeof(double) ? K_SPHERE_TO_STICKS64 : K_SPHERE_TO_STICKS, s, (double)nrows * (sp + sk));
    with_n(d.nz, [&]<int NZ>() {
        hipLaunchKernelGGL((k_sphere_to_sticks<T, NZ>), stick_grid<T>(d, nrows), dim3(kThreads), stick_lds<T>(d), s, d, t,
                           in, ld_in, gscale, sticks);
    });
    PDEP_HIP(hipGetLastError());
}

template <typename T>
void launch_sticks_to_sphere(const FftDims& d, const BasisTables& t, const cplx<T>* sticks, int nrows, cplx<T>* out,
                             long ld_out, int epi, double alpha, const cplx<T>* x, long ld_x, const T* kin,
                             const double* shift, int nshift, const double* gscale, hipStream_t s,
                             double* dot_part) {
    if (nrows <= 0) return;
    PDEP_REQUIRE(!dot_part || epi == EPI_SHIFTED_H, PDEP_EINVAL, "sticks_to_sphere: dot products need EPI_SHIFTED_H");
    check_sticks(d);
    check_rows(nrows);
    const double sp = (double)d.npw * sizeof(cplx<T>), sk = (double)d.nz * d.ns * sizeof(cplx<T>);
    ProfScope prof_(sizeof(T) == sizeof(double) ? K_STICKS_TO_SPHERE64 : K_STICKS_TO_SPHERE, s,
                    (double)nrows * (sk + sp + (epi == EPI_SHIFTED_H ? sp : 0.0)));
    if constexpr (sizeof(T) == sizeof(float)) {
        if (stick_reg_ok(d)) {
            const dim3 grid((d.ns + kRegStickGroup - 1) / kRegStickGroup, nrows);
            const size_t lds = (size_t)d.sg_max * sizeof(float2);
            with_n(d.nz, [&]<int NZ>() {
                if constexpr (NZ > 0 && NZ <= 48)
                    hipLaunchKernelGGL((k_sticks_to_sphere_reg<NZ>), grid, dim3(kRegStickGroup), lds, s, d, t,
                                       sticks, out, ld_out, epi, alpha, x, ld_x, kin, shift, nshift > 0 ? nshift : 1,
                                       gscale, dot_part);
            });
            PDEP_HIP(hipGetLastError());
            return;
        }
    }
    with_n(d.nz, [&]<int NZ>() {
        hipLaunchKernelGGL((k_sticks_to_sphere<T, NZ>), stick_grid<T>(d, nrows), dim3(kThreads), stick_lds<T>(d), s, d,
                           t, sticks, out, ld_out, epi, alpha, x, ld_x, kin, shift, nshift > 0 ? nshift : 1, gscale,
                           dot_part);
    });
    PDEP_HIP(hipGetLastError());
}

// The register paired pass applies to FP32 lines of a compiled length up to 48 whose two
// staging arrays fit 64 KB of LDS.
bool pair_reg_ok(const FftDims& d) {
    const bool len = d.nz == 16 || d.nz == 24 || d.nz == 32 || d.nz == 48;
    return len && d.sgp_max > 0 && 2 * (size_t)d.sgp_max * sizeof(float2) <= 65536;
}

// The FP64 lane-quad sticks-to-sphere pass: z lengths that are multiples of 4 up to 48,
// its staging arrays, twiddles and reduction space within 64 KB of LDS.
bool pair_quad64_ok(const FftDims& d) {
    const bool len = d.nz == 16 || d.nz == 24 || d.nz == 32 || d.nz == 48;
    return len && d.sgp_max > 0 &&
           (2 * (size_t)d.sgp_max + d.nz) * sizeof(double2) + 2 * 256 * sizeof(double) <= 65536;
}
size_t pair_quad64_lds(const FftDims& d) { return (2 * (size_t)d.sgp_max + d.nz) * sizeof(double2); }

template <typename T> int sticks_to_sphere_pair_groups(const FftDims& d) {
    if (sizeof(T) == sizeof(float) && pair_reg_ok(d)) return ((d.ns + 1) / 2 + kPairStickGroup - 1) / kPairStickGroup;
    if (sizeof(T) == sizeof(double) && pair_quad64_ok(d))
        return ((d.ns + 1) / 2 + kQuadStickGroup - 1) / kQuadStickGroup;
    const int sgh = sticks_per_group<T>(d.nz) / 2;
    return ((d.ns + 1) / 2 + sgh - 1) / sgh;
}

int pair_count(int nrows, int group) {
    const int g = group > 0 ? group : nrows;
    return (nrows / g) * ((g + 1) / 2) + ((nrows % g) + 1) / 2;
}

template <typename T>
void launch_sphere_to_sticks_pair(const FftDims& d, const BasisTables& t, const cplx<T>* in, long ld_in, int nrows,
                                  cplx<T>* sticks, hipStream_t s, int group) {
    if (nrows <= 0) return;
    check_sticks(d);
    const int npair = pair_count(nrows, group);
    check_rows(npair);
    const double hp = (double)((d.npw + 1) / 2) * sizeof(cplx<T>), sk = (double)d.nz * d.ns * sizeof(cplx<T>);
    ProfScope prof_(sizeof(T) == sizeof(double) ? K_SPHERE_TO_STICKS64 : K_SPHERE_TO_STICKS, s,
                    (double)nrows * hp + (double)npair * sk);
    if constexpr (sizeof(T) == sizeof(float)) {
        if (pair_reg_ok(d)) {
            const dim3 grid(((d.ns + 1) / 2 + kPairStickGroup - 1) / kPairStickGroup, npair);
            const size_t lds = 2 * (size_t)d.sgp_max * sizeof(float2);
            with_n(d.nz, [&]<int NZ>() {
                if constexpr (NZ > 0 && NZ <= 48)
                    hipLaunchKernelGGL((k_sphere_to_sticks_pair_reg<NZ>), grid, dim3(2 * kPairStickGroup), lds, s, d,
                                       t, in, ld_in, nrows, group > 0 ? group : nrows, sticks);
            });
            PDEP_HIP(hipGetLastError());
            return;
        }
    }
    with_n(d.nz, [&]<int NZ>() {
        hipLaunchKernelGGL((k_sphere_to_sticks_pair<T, NZ>), stick_grid<T>(d, npair), dim3(kThreads), stick_lds<T>(d), s,
                           d, t, in, ld_in, nrows, group > 0 ? group : nrows, sticks);
    });
    PDEP_HIP(hipGetLastError());
}

template <typename T>
void launch_sticks_to_sphere_pair(const FftDims& d, const BasisTables& t, const cplx<T>* sticks, int nrows,
                                  cplx<T>* out, long ld_out, int epi, double alpha, const cplx<T>* x, long ld_x,
                                  const T* kin, const double* shift, int nshift, hipStream_t s, double* dot_part,
                                  int group) {
    if (nrows <= 0) return;
    PDEP_REQUIRE(epi == EPI_SHIFTED_H || (epi == EPI_SCALE && !dot_part), PDEP_EINVAL,
                 "sticks_to_sphere_pair: EPI_SHIFTED_H, or EPI_SCALE without dot products");
    check_sticks(d);
    const int npair = pair_count(nrows, group);
    check_rows(npair);
    const double hp = (double)((d.npw + 1) / 2) * sizeof(cplx<T>), sk = (double)d.nz * d.ns * sizeof(cplx<T>);
    ProfScope prof_(sizeof(T) == sizeof(double) ? K_STICKS_TO_SPHERE64 : K_STICKS_TO_SPHERE, s,
                    (double)npair * sk + 2.0 * nrows * hp);
    // dot_part holds one partial sum per row and group of the kernel that takes
    // EPI_SHIFTED_H (sticks_to_sphere_pair_groups)
    PDEP_REQUIRE(!dot_part || epi == EPI_SHIFTED_H, PDEP_EINVAL, "sticks_to_sphere_pair: dot products need EPI_SHIFTED_H");
    if constexpr (sizeof(T) == sizeof(float)) {
        if (epi == EPI_SHIFTED_H && pair_reg_ok(d)) {
            const dim3 grid(((d.ns + 1) / 2 + kPairStickGroup - 1) / kPairStickGroup, npair);
            const size_t lds = 2 * (size_t)d.sgp_max * sizeof(float2);
            with_n(d.nz, [&]<int NZ>() {
                if constexpr (NZ > 0 && NZ <= 48)
                    hipLaunchKernelGGL((k_sticks_to_sphere_pair_reg<NZ>), grid, dim3(2 * kPairStickGroup), lds, s, d,
                                       t, sticks, nrows, group > 0 ? group : nrows, out, ld_out, x, ld_x, kin, shift,
                                       nshift > 0 ? nshift : 1, dot_part);
            });
            PDEP_HIP(hipGetLastError());
            return;
        }
    } else {
        if (epi == EPI_SHIFTED_H && pair_quad64_ok(d)) {
            const dim3 grid(((d.ns + 1) / 2 + kQuadStickGroup - 1) / kQuadStickGroup, npair);
            with_n(d.nz, [&]<int NZ>() {
                if constexpr (NZ > 0 && NZ % 4 == 0 && NZ <= 48)
                    hipLaunchKernelGGL((k_sticks_to_sphere_pair_quad64<NZ>), grid, dim3(256), pair_quad64_lds(d), s,
                                       d, t, sticks, nrows, group > 0 ? group : nrows, out, ld_out, x, ld_x, kin,
                                       shift, nshift > 0 ? nshift : 1, dot_part);
            });
            PDEP_HIP(hipGetLastError());
            return;
        }
    }
    const int sgh = sticks_per_group<T>(d.nz) / 2;
    const dim3 grid(((d.ns + 1) / 2 + sgh - 1) / sgh, npair);
    with_n(d.nz, [&]<int NZ>() {
        hipLaunchKernelGGL((k_sticks_to_sphere_pair<T, NZ>), grid, dim3(kThreads), stick_lds<T>(d), s, d, t, sticks,
                           nrows, group > 0 ? group : nrows, out, ld_out, epi, alpha, x, ld_x, kin, shift,
                           nshift > 0 ? nshift : 1, dot_part);
    });
    PDEP_HIP(hipGetLastError());
}

namespace {

template <typename T, int MODE>
void launch_slab(const FftDims& d, const BasisTables& t, int nrows, cplx<T>* sticks, const T* Vr, const cplx<T>* u,
                 int nv, cplx<T>* grid_c, T* grid_r, hipStream_t s, int kid, double bytes, double flops = 0.0) {
    if (nrows <= 0) return;
    check_slab(d);
    check_rows(nrows);
    ProfScope prof_(kid, s, bytes, flops);
    with_nxy(d.nx, d.ny, [&]<int N>() {
        hipLaunchKernelGGL((k_slab<T, N, N, MODE>), dim3(d.nz, nrows), dim3(kThreads), slab_lds<T>(d), s, d, t,
                           sticks, Vr, u, nv > 0 ? nv : 1, grid_c, grid_r);
    });
    PDEP_HIP(hipGetLastError());
}

}  // namespace

// Compiled sphere radius of the register slab kernel per line length: the largest |mx|
// of a 12 Ha sphere on the grids of the workloads (n = 16, 24, 32, 48 with L = 20 n / 48
// bohr; also 10 Ha at 32^3 and 15 bohr).  Other radii use the run-time form.
constexpr int slab_mx_const(int n) { return n == 16 ? 5 : n == 24 ? 7 : n == 32 ? 10 : n == 48 ? 15 : -1; }

// LDS of the register slab kernel for line length nl (0 if it does not apply).
size_t slab_reg_lds(const FftDims& d, int nl) {
    if (d.nx != d.ny || d.nx != nl) return 0;
    const int zg = 256 / nl;
    const size_t elems = std::max((size_t)zg * d.sld, (size_t)zg * nl * (size_t)(d.ax | 1));
    const size_t bytes = elems * sizeof(float2);
    return bytes <= 65536 ? bytes : 0;
}

// LDS of the FP64 lane-quad slab kernel for line length nl (0 if it does not apply):
// the slab data and nl twiddles.
size_t slab_quad64_lds(const FftDims& d, int nl) {
    if (d.nx != d.ny || d.nx != nl || nl % 4 != 0 || nl > 64 || 2 * d.mxmax + 1 > nl) return 0;
    const size_t bytes = ((size_t)quad64_data_elems(d, nl) + nl) * sizeof(double2);
    return bytes <= 65536 ? bytes : 0;
}

template <typename T>
void launch_slab_hv(const FftDims& d, const BasisTables& t, cplx<T>* sticks, int nrows, const T* Vz, hipStream_t s) {
    const double sk = (double)d.nz * d.ns * sizeof(cplx<T>);
    const double bytes = (double)nrows * 2.0 * sk + (double)d.nx * d.ny * d.nz * sizeof(T);
    // algorithmic flops: 5 n log2 n per length-n complex line (inverse and forward y on the
    // non-empty columns, inverse and forward x on every row) plus the real multiply by V
    const double lines_y = 2.0 * d.ax * d.nz, lines_x = 2.0 * d.ny * d.nz;
    const double flops = (double)nrows * (lines_y * 5.0 * d.ny * std::log2((double)d.ny) +
                                          lines_x * 5.0 * d.nx * std::log2((double)d.nx) +
                                          2.0 * d.nx * d.ny * d.nz);
    if constexpr (sizeof(T) == sizeof(double)) {
        bool done = false;
        with_n(d.nx, [&]<int N>() {
            if constexpr (N > 0 && N <= 64 && N % 4 == 0) {
                const size_t lds = slab_quad64_lds(d, N);
                if (lds > 0 && nrows > 0) {
                    check_rows(nrows);
                    constexpr int ZG = 64 / N;
                    ProfScope prof_(K_SLAB_HV64, s, bytes, flops);
                    const dim3 grid((d.nz + ZG - 1) / ZG, nrows);
                    hipLaunchKernelGGL((k_slab_hv_quad64<N>), grid, dim3(quad64_threads(N)), lds, s, d, t, sticks,
                                       Vz);
                    PDEP_HIP(hipGetLastError());
                    done = true;
                }
            }
        });
        if (done || nrows <= 0) return;
    }
    if constexpr (sizeof(T) == sizeof(float)) {
        bool done = false;
        with_n(d.nx, [&]<int N>() {
            if constexpr (N > 0 && N <= 48) {
                const size_t lds = slab_reg_lds(d, N);
                if (lds > 0 && nrows > 0) {
                    check_rows(nrows);
                    constexpr int ZG = 256 / N;
                    ProfScope prof_(K_SLAB_HV, s, bytes, flops);
                    const dim3 grid((d.nz + ZG - 1) / ZG, nrows);
                    if (d.mxmax == slab_mx_const(N) && d.mymax <= slab_mx_const(N))
                        hipLaunchKernelGGL((k_slab_hv_reg<N, slab_mx_const(N)>), grid, dim3(256), lds, s, d, t,
                                           sticks, Vz);
                    else
                        hipLaunchKernelGGL((k_slab_hv_reg<N, -1>), grid, dim3(256), lds, s, d, t, sticks, Vz);
                    PDEP_HIP(hipGetLastError());
                    done = true;
                }
            }
        });
        if (done || nrows <= 0) return;
    }
    launch_slab<T, SLAB_HV>(d, t, nrows, sticks, Vz, nullptr, 1, nullptr, nullptr, s,
                            sizeof(T) == sizeof(double) ? K_SLAB_HV64 : K_SLAB_HV, bytes, flops);
}

template <typename T>
void launch_slab_inv_store(const FftDims& d, const BasisTables& t, cplx<T>* sticks, int nrows, cplx<T>* grid_c,
                           T* grid_r, hipStream_t s) {
    const double sk = (double)d.nz * d.ns * sizeof(cplx<T>);
    const double g = (double)d.nx * d.ny * d.nz * (grid_c ? sizeof(cplx<T>) : sizeof(T));
    if (grid_c)
        launch_slab<T, SLAB_INV_C>(d, t, nrows, sticks, nullptr, nullptr, 1, grid_c, nullptr, s, K_SLAB_INV_STORE,
                                   (double)nrows * (sk + g));
    else
        launch_slab<T, SLAB_INV_R>(d, t, nrows, sticks, nullptr, nullptr, 1, nullptr, grid_r, s, K_SLAB_INV_STORE,
                                   (double)nrows * (sk + g));
}

template <typename T>
void launch_slab_fwd_product(const FftDims& d, const BasisTables& t, const T* Vr, const cplx<T>* u, int nv, int nrows,
                             cplx<T>* sticks, hipStream_t s) {
    const double sk = (double)d.nz * d.ns * sizeof(cplx<T>);
    const double g = (double)d.nx * d.ny * d.nz;
    if constexpr (sizeof(T) == sizeof(double)) {
        bool done = false;
        with_n(d.nx, [&]<int N>() {
            if constexpr (N > 0 && N <= 64 && N % 4 == 0) {
                const size_t lds = slab_quad64_lds(d, N);
                if (lds > 0 && nrows > 0) {
                    check_rows(nrows);
                    constexpr int ZG = 64 / N;
                    const dim3 grid((d.nz + ZG - 1) / ZG, nrows);
                    if (u) {
                        ProfScope prof_(K_SLAB_FWD_PRODUCT, s,
                                        (double)nrows * (sk + g * sizeof(cplx<T>)) + g * sizeof(T) * (nrows / nv));
                        hipLaunchKernelGGL((k_slab_fwd_quad64<N, true>), grid, dim3(quad64_threads(N)), lds, s, d, t,
                                           sticks, Vr, u, nv);
                    } else {
                        ProfScope prof_(K_SLAB_FWD_PRODUCT, s, (double)nrows * (sk + g * sizeof(T)));
                        hipLaunchKernelGGL((k_slab_fwd_quad64<N, false>), grid, dim3(quad64_threads(N)), lds, s, d, t,
                                           sticks, Vr, nullptr, 1);
                    }
                    PDEP_HIP(hipGetLastError());
                    done = true;
                }
            }
        });
        if (done || nrows <= 0) return;
    }
    if (u)
        launch_slab<T, SLAB_FWD_PRODUCT>(d, t, nrows, sticks, Vr, u, nv, nullptr, nullptr, s, K_SLAB_FWD_PRODUCT,
                                         (double)nrows * (sk + g * sizeof(cplx<T>)) + g * sizeof(T) * (nrows / nv));
    else
        launch_slab<T, SLAB_FWD_REAL>(d, t, nrows, sticks, Vr, nullptr, 1, nullptr, nullptr, s, K_SLAB_FWD_PRODUCT,
                                      (double)nrows * (sk + g * sizeof(T)));
}

void launch_slab_density(const FftDims& d, const BasisTables& t, const double2* sticks, int npert, int nv,
                         const double2* u, double scale, double* dn, hipStream_t s) {
    if (npert <= 0) return;
    check_slab(d);
    check_rows(npert);
    PDEP_REQUIRE(d.nx * d.ny <= kThreads * kMaxAcc, PDEP_EINVAL, "density slab too large");
    const double g = (double)d.nx * d.ny * d.nz;
    ProfScope prof_(K_SLAB_DENSITY, s,
                    (double)npert * nv * ((double)d.nz * d.ns * 16.0 + g * 16.0) + (double)npert * g * 8.0);
    bool done = false;
    with_n(d.nx, [&]<int N>() {
        if constexpr (N > 0 && N <= 64 && N % 4 == 0) {
            const size_t lds = slab_quad64_lds(d, N);
            if (lds > 0) {
                constexpr int ZG = 64 / N, PB = 2;
                hipLaunchKernelGGL((k_slab_density_quad64<N, PB>), dim3((d.nz + ZG - 1) / ZG, (npert + PB - 1) / PB),
                                   dim3(256), lds, s, d, t, sticks, npert, nv, u, scale, dn);
                done = true;
            }
        }
    });
    if (done) {
        PDEP_HIP(hipGetLastError());
        return;
    }
    with_nxy(d.nx, d.ny, [&]<int N>() {
        hipLaunchKernelGGL((k_slab_density<N, N>), dim3(d.nz, npert), dim3(kThreads), slab_lds<double>(d), s, d, t,
                           sticks, nv, u, scale, dn);
    });
    PDEP_HIP(hipGetLastError());
}

void launch_transpose_grid(int nx, int ny, int nz, int nrows, const double* in, double* out, bool to_zmajor,
                           hipStream_t s) {
    if (nrows <= 0) return;
    check_rows(nrows);
    const long ng = (long)nx * ny * nz;
    ProfScope prof_(K_MISC, s, 16.0 * ng * nrows);
    hipLaunchKernelGGL(k_transpose_grid, dim3((unsigned)((ng + 255) / 256), nrows), dim3(256), 0, s, nx, ny, nz, in,
                       out, to_zmajor ? 1 : 0);
    PDEP_HIP(hipGetLastError());
}

template <typename T> int sticks_to_sphere_groups(const FftDims& d) {
    if (sizeof(T) == sizeof(float) && stick_reg_ok(d)) return (d.ns + kRegStickGroup - 1) / kRegStickGroup;
    return (int)stick_grid<T>(d, 1).x;
}

#define PDEP_INST_FFT(T)                                                                                          \
    template void launch_sphere_to_sticks<T>(const FftDims&, const BasisTables&, const cplx<T>*, long, int,       \
                                             const double*, cplx<T>*, hipStream_t);                               \
    template void launch_sticks_to_sphere<T>(const FftDims&, const BasisTables&, const cplx<T>*, int, cplx<T>*,   \
                                             long, int, double, const cplx<T>*, long, const T*, const double*,     \
                                             int, const double*, hipStream_t, double*);                           \
    template int sticks_to_sphere_groups<T>(const FftDims&);                                                      \
    template int sticks_to_sphere_pair_groups<T>(const FftDims&);                                                 \
    template void launch_sphere_to_sticks_pair<T>(const FftDims&, const BasisTables&, const cplx<T>*, long, int,  \
                                                  cplx<T>*, hipStream_t, int);                                    \
    template void launch_sticks_to_sphere_pair<T>(const FftDims&, const BasisTables&, const cplx<T>*, int,        \
                                                  cplx<T>*, long, int, double, const cplx<T>*, long, const T*,    \
                                                  const double*, int, hipStream_t, double*, int);                 \
    template void launch_slab_hv<T>(const FftDims&, const BasisTables&, cplx<T>*, int, const T*, hipStream_t);    \
    template void launch_slab_inv_store<T>(const FftDims&, const BasisTables&, cplx<T>*, int, cplx<T>*, T*,       \
                                           hipStream_t);                                                          \
    template void launch_slab_fwd_product<T>(const FftDims&, const BasisTables&, const T*, const cplx<T>*, int,   \
                                             int, cplx<T>*, hipStream_t);

PDEP_INST_FFT(double)
PDEP_INST_FFT(float)

}  // namespace pdep
