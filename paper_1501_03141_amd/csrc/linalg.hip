// Dense kernels on blocks of sphere vectors (rows of length K, row stride ld):
//  - the occupied-space projection P_c x = x - Psi (Psi^H x) as a GEMM pair,
//  - per-row inner products and norms (accumulated in FP64),
//  - the element-wise parts of the batched preconditioned CG,
//  - precision conversion, row gathers and updates used by the refinement loop.
#include <algorithm>

#include "pdep_internal.h"

namespace pdep {

namespace {

template <typename T> __device__ __forceinline__ cplx<T> mk(T a, T b) { cplx<T> r; r.x = a; r.y = b; return r; }

// ------------------------------------------------------------------------ GEMMs ---
// Complex GEMMs on the matrix cores.  A complex product is written as a real one of
// twice the size: with interleaved storage (re, im), the pair of real rows
// (a_re, a_im) and (-a_im, a_re) dotted with an interleaved vector y give Re and Im of
// conj(a) . y, and the real 2x2 block [[a_re, a_im], [-a_im, a_re]] applied to an
// interleaved coefficient (s_re, s_im) gives the interleaved a * s.  The expansion is
// done while staging tiles in LDS, so memory holds only the complex data.
//
// Matrix-core instruction: 16x16x4 (f32 or f64), one wave, A[m][k] from lane
// (m + 16 k), B[k][n] from lane (n + 16 k); result slot i of lane l is row
// 4*(l/16) + i (f32) or 4*i + l/16 (f64) of column l % 16.
typedef float mfma_f4 __attribute__((ext_vector_type(4)));
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<float> {
    using acc = mfma_f4;
    static __device__ __forceinline__ acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};
template <> struct Mfma<double> {
    using acc = mfma_d4;
    static __device__ __forceinline__ acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int i) { return 4 * i + (lane >> 4); }
};

constexpr int kPad = 4;

// S[n][m] = sum_k conj(A[m][k]) B[n][k].  Real form C[m'][n] = sum_k' A'[m'][k'] B'[n][k']
// with m' = 2m + s.  Workgroup tile: 32 complex rows of A (64 real) x 64 rows of B,
// K staged 16 complex (32 real) at a time; 4 waves in a 2 x 2 arrangement, each 32 x 32.
// Split-K: workgroup z covers k in [z * kchunk, (z + 1) * kchunk) and writes its
// partial product to S + z * N * lds (reduced afterwards in a fixed order).
// REAL: only Re S (imaginary parts stored as zero): the A tile holds only the (re, im)
// rows, 64 complex rows per workgroup, half the matrix-core work.
template <typename T, bool REAL>
__global__ __launch_bounds__(256) void k_gemm_ahb(int M, int N, int K, const cplx<T>* __restrict__ A, long lda,
                                                  const cplx<T>* __restrict__ B, long ldb, cplx<T>* __restrict__ S,
                                                  long lds, int kchunk, int real_out) {
    constexpr int BMC = REAL ? 64 : 32, BN = 64, BKC = 16;
    constexpr int BMR = 64, BKR = 2 * BKC;
    __shared__ T As[BKR][BMR + kPad];
    __shared__ T Bs[BKR][BN + kPad];
    using Op = Mfma<T>;
    const int m0 = blockIdx.x * BMC, n0 = blockIdx.y * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    typename Op::acc acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = typename Op::acc{0, 0, 0, 0};
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(K, kbeg + kchunk);
    S += (long)blockIdx.z * N * lds;
    // the next step's tiles are loaded into registers while the current one is multiplied
    constexpr int NA = BMC * BKC / 256;
    cplx<T> pa[NA], pb[4];
    auto fetch = [&](int kc) {
#pragma unroll
        for (int j = 0; j < NA; ++j) {
            const int e = tid + 256 * j;
            const int r = e / BKC, g = e % BKC;
            pa[j].x = 0; pa[j].y = 0;
            if (m0 + r < M && kc + g < kend) pa[j] = A[(long)(m0 + r) * lda + kc + g];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = tid + 256 * j;
            const int r = e / BKC, g = e % BKC;
            pb[j].x = 0; pb[j].y = 0;
            if (n0 + r < N && kc + g < kend) pb[j] = B[(long)(n0 + r) * ldb + kc + g];
        }
    };
    if (kbeg < kend) fetch(kbeg);
    for (int kc = kbeg; kc < kend; kc += BKC) {
#pragma unroll
        for (int j = 0; j < NA; ++j) {
            const int e = tid + 256 * j;
            const int r = e / BKC, g = e % BKC;
            const cplx<T> v = pa[j];
            if constexpr (REAL) {
                As[2 * g][r] = v.x;
                As[2 * g + 1][r] = v.y;
            } else {
                As[2 * g][2 * r] = v.x;
                As[2 * g + 1][2 * r] = v.y;
                As[2 * g][2 * r + 1] = -v.y;
                As[2 * g + 1][2 * r + 1] = v.x;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = tid + 256 * j;
            const int r = e / BKC, g = e % BKC;
            Bs[2 * g][r] = pb[j].x;
            Bs[2 * g + 1][r] = pb[j].y;
        }
        __syncthreads();
        if (kc + BKC < kend) fetch(kc + BKC);
#pragma unroll
        for (int kk = 0; kk < BKR; kk += 4) {
            const int kr = kk + (lane >> 4), c = lane & 15;
            const T a0 = As[kr][wm + c], a1 = As[kr][wm + 16 + c];
            const T b0 = Bs[kr][wn + c], b1 = Bs[kr][wn + 16 + c];
            acc[0][0] = Op::mma(a0, b0, acc[0][0]);
            acc[0][1] = Op::mma(a0, b1, acc[0][1]);
            acc[1][0] = Op::mma(a1, b0, acc[1][0]);
            acc[1][1] = Op::mma(a1, b1, acc[1][1]);
        }
        __syncthreads();
    }
    T* So = reinterpret_cast<T*>(S);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int mr = wm + 16 * a + Op::row(lane, i);       // real row in the tile
                const int n = n0 + wn + 16 * b + (lane & 15);
                if constexpr (REAL) {
                    const int m = m0 + mr;
                    if (m < M && n < N) {
                        So[((long)n * lds + m) * 2] = acc[a][b][i];
                        So[((long)n * lds + m) * 2 + 1] = T(0);
                    }
                } else {
                    const int m = m0 + (mr >> 1), part = mr & 1;
                    if (m < M && n < N) So[((long)n * lds + m) * 2 + part] = (real_out && part) ? T(0) : acc[a][b][i];
                }
            }
}

// S[n][m] = sum_z P[z][n][m] in the order z = 0, 1, ... (deterministic split-K sum).
template <typename T>
__global__ void k_splitk_reduce(int M, int N, long lds, int splits, const cplx<T>* __restrict__ P,
                                cplx<T>* __restrict__ S, int real_out) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)N * M) return;
    const long n = e / M, m = e - (e / M) * M;
    const long stride = (long)N * lds;
    T re = 0, im = 0;
    for (int z = 0; z < splits; ++z) {
        const cplx<T> v = P[z * stride + n * lds + m];
        re += v.x;
        im += v.y;
    }
    cplx<T> o;
    o.x = re;
    o.y = real_out ? T(0) : im;
    S[n * lds + m] = o;
}

// Y[n][k] = beta Y[n][k] + alpha sum_m A[m][k] S[n][m].  Real form over k' = 2k + c
// (columns) and m' = 2m + s (contraction).  Workgroup tile: 64 rows n x 64 complex
// columns (128 real), contraction staged 16 complex (32 real) at a time; 4 waves in a
// 2 x 2 arrangement, each 32 rows x 64 real columns.
// REAL: the imaginary parts of S are taken as zero; the contraction then runs over m
// directly (32 m per step, half the matrix-core work).
template <typename T, bool REAL>
__global__ __launch_bounds__(256) void k_gemm_update(int M, int N, int K, const cplx<T>* __restrict__ A, long lda,
                                                     const cplx<T>* __restrict__ S, long lds, double alpha,
                                                     double beta, cplx<T>* __restrict__ Y, long ldy) {
    constexpr int BN = 64, BKC = 64, BMC = REAL ? 32 : 16;
    constexpr int BKR = 2 * BKC, BMR = 32;
    __shared__ T Ss[BMR][BN + kPad];    // [m'][n]
    __shared__ T Bs[BMR][BKR + kPad];   // [m'][k']
    using Op = Mfma<T>;
    const int k0 = blockIdx.x * BKC, n0 = blockIdx.y * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wn = (wave & 1) * 32, wk = (wave >> 1) * 64;
    typename Op::acc acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = typename Op::acc{0, 0, 0, 0};
    // the next step's tiles are loaded into registers while the current one is multiplied
    constexpr int NS = BN * BMC / 256, NA = BMC * BKC / 256;
    T psr[NS], psi[REAL ? 1 : NS];   // S tile (real parts; imaginary parts unless REAL)
    cplx<T> pa[NA];
    auto fetch = [&](int mc) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {        // S: 64 rows x BMC complex
            const int e = tid + 256 * j;
            const int r = e / BMC, mm = e % BMC;
            const bool in = n0 + r < N && mc + mm < M;
            const T* sp = reinterpret_cast<const T*>(S + (long)(in ? n0 + r : 0) * lds + (in ? mc + mm : 0));
            psr[j] = in ? sp[0] : T(0);
            if constexpr (!REAL) psi[j] = in ? sp[1] : T(0);
        }
#pragma unroll
        for (int j = 0; j < NA; ++j) {        // A: BMC complex rows x 64 complex columns
            const int e = tid + 256 * j;
            const int mm = e / BKC, g = e % BKC;
            pa[j].x = 0; pa[j].y = 0;
            if (mc + mm < M && k0 + g < K) pa[j] = A[(long)(mc + mm) * lda + k0 + g];
        }
    };
    fetch(0);
    for (int mc = 0; mc < M; mc += BMC) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int e = tid + 256 * j;
            const int r = e / BMC, mm = e % BMC;
            if constexpr (REAL) {
                Ss[mm][r] = psr[j];
            } else {
                Ss[2 * mm][r] = psr[j];
                Ss[2 * mm + 1][r] = psi[j];
            }
        }
#pragma unroll
        for (int j = 0; j < NA; ++j) {
            const int e = tid + 256 * j;
            const int mm = e / BKC, g = e % BKC;
            const cplx<T> v = pa[j];
            if constexpr (REAL) {
                Bs[mm][2 * g] = v.x;
                Bs[mm][2 * g + 1] = v.y;
            } else {
                Bs[2 * mm][2 * g] = v.x;
                Bs[2 * mm][2 * g + 1] = v.y;
                Bs[2 * mm + 1][2 * g] = -v.y;
                Bs[2 * mm + 1][2 * g + 1] = v.x;
            }
        }
        __syncthreads();
        if (mc + BMC < M) fetch(mc + BMC);
#pragma unroll
        for (int kk = 0; kk < BMR; kk += 4) {
            const int kr = kk + (lane >> 4), c = lane & 15;
            const T a0 = Ss[kr][wn + c], a1 = Ss[kr][wn + 16 + c];
            T b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) b[q] = Bs[kr][wk + 16 * q + c];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                acc[0][q] = Op::mma(a0, b[q], acc[0][q]);
                acc[1][q] = Op::mma(a1, b[q], acc[1][q]);
            }
        }
        __syncthreads();
    }
    T* Yo = reinterpret_cast<T*>(Y);
    const T al = (T)alpha, be = (T)beta;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int n = n0 + wn + 16 * a + Op::row(lane, i);
                const int kr = k0 * 2 + wk + 16 * q + (lane & 15);   // real column
                if (n < N && (kr >> 1) < K) {
                    T* y = Yo + (long)n * ldy * 2 + kr;
                    const T old = beta != 0.0 ? *y : T(0);
                    *y = be * old + al * acc[a][q][i];
                }
            }
}

// Y[n][kr] -= sum_m S[n][m] A[m][kr] in real arithmetic: the projection update of FP64
// half-sphere rows with real coefficients (rows read as real vectors of 2 K doubles; S
// real, row stride lds).  Four waves (2 x 2), each WR x WC blocks of 16 x 16 outputs on
// the FP64 matrix cores (16 x 16 x 4 steps): workgroup tile 32 WR rows x 32 WC real
// columns.  The Y tile is loaded first, so that its latency hides behind the product;
// m is staged 16 at a time through LDS while the next stage's tiles are loaded into
// registers.
constexpr int kDgM = 16, kDgPad = 2, kDgWR = 4, kDgWC = 2;
template <int WR, int WC>
__global__ __launch_bounds__(256, 2) void k_dgemm_sub(int M, int N, int K2, const double* __restrict__ A, long lda2,
                                                      const double* __restrict__ S, long lds,
                                                      double* __restrict__ Y, long ldy2) {
    constexpr int TN = 32 * WR, TK = 32 * WC;
    constexpr int SJ = TN * kDgM / 256, AJ = TK * kDgM / 512;   // per-thread loads (S doubles, A double2s)
    static_assert(SJ >= 1 && AJ >= 1, "tile too small for the loaders");
    __shared__ double Ss[kDgM][TN + kDgPad];   // [m][n]
    __shared__ double As[kDgM][TK + kDgPad];   // [m][kr]
    using Op = Mfma<double>;
    const int k0 = blockIdx.x * TK, n0 = blockIdx.y * TN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wn = (wave & 1) * 16 * WR, wk = (wave >> 1) * 16 * WC;
    const int nb = n0 + wn + (lane >> 4), kb = k0 + wk + (lane & 15);
    double yv[WR][WC][4];
#pragma unroll
    for (int q = 0; q < WR; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int n = nb + 16 * q + 4 * i;   // Op::row(lane, i) = 4 i + lane / 16
#pragma unroll
            for (int r = 0; r < WC; ++r) {
                const int kr = kb + 16 * r;
                yv[q][r][i] = (n < N && kr < K2) ? Y[(long)n * ldy2 + kr] : 0.0;
            }
        }
    Op::acc acc[WR][WC];
#pragma unroll
    for (int a = 0; a < WR; ++a)
#pragma unroll
        for (int b = 0; b < WC; ++b) acc[a][b] = Op::acc{0, 0, 0, 0};
    // S: thread -> (m = tid % 16, n = tid / 16 + 16 j); A: thread -> (m, kr pair) with the
    // TK / 2 pairs of a row of A fastest
    constexpr int AP = TK / 2;
    const int sm = tid & 15, sn = tid >> 4;
    double ps[SJ];
    double2 pa[AJ];
    auto fetch = [&](int mc) {
#pragma unroll
        for (int j = 0; j < SJ; ++j) {
            const int n = n0 + sn + 16 * j, m = mc + sm;
            ps[j] = (n < N && m < M) ? S[(long)n * lds + m] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < AJ; ++j) {
            const int e = tid + 256 * j;
            const int m = mc + e / AP, kr = k0 + 2 * (e % AP);
            if (m < M && kr + 1 < K2) {
                pa[j] = *reinterpret_cast<const double2*>(A + (long)m * lda2 + kr);
            } else {
                pa[j].x = (m < M && kr < K2) ? A[(long)m * lda2 + kr] : 0.0;
                pa[j].y = 0.0;
            }
        }
    };
    fetch(0);
    for (int mc = 0; mc < M; mc += kDgM) {
#pragma unroll
        for (int j = 0; j < SJ; ++j) Ss[sm][sn + 16 * j] = ps[j];
#pragma unroll
        for (int j = 0; j < AJ; ++j) {
            const int e = tid + 256 * j;
            As[e / AP][2 * (e % AP)] = pa[j].x;
            As[e / AP][2 * (e % AP) + 1] = pa[j].y;
        }
        __syncthreads();
        if (mc + kDgM < M) fetch(mc + kDgM);
#pragma unroll
        for (int kk = 0; kk < kDgM; kk += 4) {
            const int mr = kk + (lane >> 4), c = lane & 15;
            double a[WR], b[WC];
#pragma unroll
            for (int q = 0; q < WR; ++q) a[q] = Ss[mr][wn + 16 * q + c];
#pragma unroll
            for (int r = 0; r < WC; ++r) b[r] = As[mr][wk + 16 * r + c];
#pragma unroll
            for (int q = 0; q < WR; ++q)
#pragma unroll
                for (int r = 0; r < WC; ++r) acc[q][r] = Op::mma(a[q], b[r], acc[q][r]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < WR; ++q)
#pragma unroll
        for (int r = 0; r < WC; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int n = nb + 16 * q + 4 * i, kr = kb + 16 * r;
                if (n < N && kr < K2) Y[(long)n * ldy2 + kr] = yv[q][r][i] - acc[q][r][i];
            }
}

// out[r][m] = Re S[r][m] for nrows rows of lds entries
__global__ void k_real_coefs(long n, const double2* __restrict__ in, double* __restrict__ out) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i].x;
}

// ------------------------------------------------------------------- reductions ---
// Half-sphere rows (half != 0) hold the entries k <= c of a Hermitian-symmetric vector,
// the centre G = 0 last (k = K - 1); every other entry stands for itself and its mirror
// -G, so it counts twice in an inner product.
__device__ __forceinline__ double half_weight(int half, int k, int K) { return (half && k != K - 1) ? 2.0 : 1.0; }

template <typename T>
__global__ __launch_bounds__(256) void k_row_dots(int K, const cplx<T>* __restrict__ a, long lda,
                                                  const cplx<T>* __restrict__ b, long ldb, double* __restrict__ out,
                                                  double* __restrict__ out2, int half) {
    __shared__ double red[2][256];
    const int row = blockIdx.x;
    const cplx<T>* ar = a + (long)row * lda;
    const cplx<T>* br = b + (long)row * ldb;
    double s = 0.0, s2 = 0.0;
    for (int k = threadIdx.x; k < K; k += 256) {
        const cplx<T> x = ar[k], y = br[k];
        const double w = half_weight(half, k, K);
        s += w * ((double)x.x * (double)y.x + (double)x.y * (double)y.y);
        s2 += w * ((double)x.x * (double)x.x + (double)x.y * (double)x.y);
    }
    red[0][threadIdx.x] = s;
    red[1][threadIdx.x] = s2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[row] = red[0][0];
        if (out2) out2[row] = red[1][0];
    }
}

// ------------------------------------------------------------------- CG pieces ---
// K_G = 1 / max(1/2|G|^2 - shift, kPrecondFloor): the kinetic diagonal of H - e_v,
// floored (in Hartree) where it is small or negative.
template <typename T>
__device__ __forceinline__ T precond_factor(const T* kin, int k, double shift) {
    if constexpr (sizeof(T) == sizeof(float)) {
        // FP32 rows: the single-instruction reciprocal, as in the BF16x3 GEMMs that apply K
        const float d = kin[k] - (float)shift, fl = (float)kPrecondFloor;
        return __builtin_amdgcn_rcpf(d > fl ? d : fl);
    } else {
        const double d = (double)kin[k] - shift;
        return (T)(1.0 / (d > kPrecondFloor ? d : kPrecondFloor));
    }
}

template <typename T>
__global__ void k_cg_init(int K, const cplx<T>* __restrict__ b, long ld, cplx<T>* __restrict__ x,
                          cplx<T>* __restrict__ r, cplx<T>* __restrict__ z, const T* __restrict__ kin,
                          const double* __restrict__ shift, int nshift, int precond) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (k >= K) return;
    const long o = (long)row * ld + k;
    const cplx<T> bv = b[o];
    x[o] = mk<T>(0, 0);
    r[o] = bv;
    const T f = precond ? precond_factor(kin, k, shift[row % nshift]) : T(1);
    z[o] = mk<T>(f * bv.x, f * bv.y);
}

// Rows of the CG step per workgroup column: each thread takes kStep1Elems entries of a
// row (stride 256), so the per-row scalars (alpha from the <p, q> partials) are formed
// once per kStep1Elems entries.
constexpr int kStep1Elems = 4;

template <typename T>
__global__ __launch_bounds__(256) void k_cg_step1(int K, cplx<T>* __restrict__ x, cplx<T>* __restrict__ r,
                                                  cplx<T>* __restrict__ z, const cplx<T>* __restrict__ p,
                                                  const cplx<T>* __restrict__ q, long ld,
                                                  const double* __restrict__ rz, const double* __restrict__ pq,
                                                  int npq, const int* __restrict__ active, const T* __restrict__ kin,
                                                  const double* __restrict__ shift, int nshift, int precond,
                                                  double* __restrict__ rz_part, double* __restrict__ rr_part, int half,
                                                  float* __restrict__ alpha_out) {
    __shared__ double red[2][256];
    const int row = blockIdx.y;
    if (!active[row]) return;                         // whole block: one row
    double den = 0.0;
    for (int g = 0; g < npq; ++g) den += pq[(long)row * npq + g];
    const T alpha = (T)(den > 0.0 ? rz[row] / den : 0.0);
    if (alpha_out && blockIdx.x == 0 && threadIdx.x == 0) alpha_out[row] = (float)alpha;
    const double sh = shift[row % nshift];
    double srz = 0.0, srr = 0.0;
#pragma unroll
    for (int e = 0; e < kStep1Elems; ++e) {
        const int k = (blockIdx.x * kStep1Elems + e) * 256 + threadIdx.x;
        if (k < K) {
            const long o = (long)row * ld + k;
            const cplx<T> qv = q[o];
            cplx<T> rv = r[o];
            if (x) {   // null: x is updated later (with alpha_out) by the caller
                const cplx<T> pv = p[o];
                cplx<T> xv = x[o];
                xv.x += alpha * pv.x; xv.y += alpha * pv.y;
                x[o] = xv;
            }
            rv.x -= alpha * qv.x; rv.y -= alpha * qv.y;
            r[o] = rv;
            const T f = precond ? precond_factor(kin, k, sh) : T(1);
            if (z) z[o] = mk<T>(f * rv.x, f * rv.y);
            const double n2 = half_weight(half, k, K) * ((double)rv.x * (double)rv.x + (double)rv.y * (double)rv.y);
            srr += n2;
            srz += (double)f * n2;
        }
    }
    if (rz_part) {   // <r, K r> and ||r||^2 over this block (fixed-order tree)
        red[0][threadIdx.x] = srz;
        red[1][threadIdx.x] = srr;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                red[0][threadIdx.x] += red[0][threadIdx.x + w];
                red[1][threadIdx.x] += red[1][threadIdx.x + w];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            rz_part[(long)row * gridDim.x + blockIdx.x] = red[0][0];
            rr_part[(long)row * gridDim.x + blockIdx.x] = red[1][0];
        }
    }
}

// rz[row] = sum_g rz_part[row][g], rr[row] likewise (g in order); inactive rows skipped.
// beta (may be null): rz[row] / rz_old[row] (0 when rz_old[row] = 0), the CG direction factor.
__global__ void k_sum_parts(int nrows, int nparts, const double* __restrict__ rz_part,
                            const double* __restrict__ rr_part, const int* __restrict__ active,
                            double* __restrict__ rz, double* __restrict__ rr, const double* __restrict__ rz_old,
                            float* __restrict__ beta) {
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= nrows || !active[row]) return;
    double a = 0.0, b = 0.0;
    for (int g = 0; g < nparts; ++g) {
        a += rz_part[(long)row * nparts + g];
        b += rr_part[(long)row * nparts + g];
    }
    rz[row] = a;
    rr[row] = b;
    if (beta) {
        const double d = rz_old[row];
        beta[row] = (float)(d != 0.0 ? a / d : 0.0);
    }
}

template <typename T>
__global__ void k_cg_step2(int K, cplx<T>* __restrict__ p, const cplx<T>* __restrict__ z, long ld,
                           const double* __restrict__ rz_new, const double* __restrict__ rz,
                           const int* __restrict__ active) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (k >= K || !active[row]) return;
    const double den = rz[row];
    const T beta = (T)(den != 0.0 ? rz_new[row] / den : 0.0);
    const long o = (long)row * ld + k;
    const cplx<T> zv = z[o];
    cplx<T> pv = p[o];
    pv.x = zv.x + beta * pv.x;
    pv.y = zv.y + beta * pv.y;
    p[o] = pv;
}

__global__ void k_cg_check(int nrows, const double* __restrict__ rr, const double* __restrict__ thr2,
                           int* __restrict__ active, int* __restrict__ iters, double* __restrict__ rz,
                           const double* __restrict__ rz_new, int* __restrict__ n_active, int count_iter,
                           double rr_max) {
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= nrows) return;
    if (active[row]) {
        if (count_iter) iters[row] += 1;
        if (rz_new) rz[row] = rz_new[row];
        const bool diverged = rr_max > 0.0 && !(rr[row] <= rr_max);
        const int still = !diverged && rr[row] > thr2[row];
        active[row] = still;
        if (diverged) iters[row] = -iters[row] - 1;   // reported as -(iterations) - 1
        if (still) atomicAdd(n_active, 1);
    }
}

template <typename Tin, typename Tout>
__global__ void k_convert_scaled(int K, const cplx<Tin>* __restrict__ in, long ldi, const int* __restrict__ rows,
                                 const double* __restrict__ rowscale, cplx<Tout>* __restrict__ out, long ldo) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (k >= K) return;
    const long ir = rows ? rows[row] : row;
    const double s = rowscale ? rowscale[row] : 1.0;
    const cplx<Tin> v = in[ir * ldi + k];
    out[(long)row * ldo + k] = mk<Tout>((Tout)(s * (double)v.x), (Tout)(s * (double)v.y));
}

template <typename T>
__global__ void k_axpy_rows(int K, const cplx<T>* __restrict__ d, long ldd, const int* __restrict__ rows,
                            const double* __restrict__ rowscale, double2* __restrict__ x, long ldx, int set) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (k >= (set ? (int)ldx : K)) return;
    const double s = rowscale[row];
    if (set) {
        double2 xv = make_double2(0.0, 0.0);
        if (k < K && s != 0.0) {
            const cplx<T> v = d[(long)row * ldd + k];
            xv = make_double2(s * (double)v.x, s * (double)v.y);
        }
        x[(rows ? rows[row] : row) * ldx + k] = xv;
        return;
    }
    if (s == 0.0) return;   // a dropped solution (it may hold non-finite values)
    const cplx<T> v = d[(long)row * ldd + k];
    const long xr = rows ? rows[row] : row;
    double2 xv = x[xr * ldx + k];
    xv.x += s * (double)v.x;
    xv.y += s * (double)v.y;
    x[xr * ldx + k] = xv;
}

// r[rows[row]] = b[rows[row]] - q[row] and out[row] = ||r||^2 (half-sphere weights when
// half), one workgroup per row.
__global__ __launch_bounds__(256) void k_residual_rows(int K, const double2* __restrict__ b, long ldb,
                                                       const int* __restrict__ rows, const double2* __restrict__ q,
                                                       long ldq, double2* __restrict__ r, long ldr,
                                                       double* __restrict__ out, int half) {
    __shared__ double red[256];
    const int row = blockIdx.x;
    const long ir = rows[row];
    const double2* br = b + ir * ldb;
    const double2* qr = q + (long)row * ldq;
    double2* rr = r + ir * ldr;
    double acc = 0.0;
    for (int k = threadIdx.x; k < K; k += 256) {
        const double2 bv = br[k], qv = qr[k];
        const double2 v = make_double2(bv.x - qv.x, bv.y - qv.y);
        rr[k] = v;
        acc += half_weight(half, k, K) * (v.x * v.x + v.y * v.y);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[row] = red[0];
}

__global__ void k_fill_zero(uint32_t* p, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0u;
}

__global__ void k_fill_i32(int* p, int n, int value) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

__global__ void k_expand_s1(int npw, int g0, const double2* __restrict__ in, long ldi, double2* __restrict__ out,
                            long ldo) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (k >= npw) return;
    double2 v = make_double2(0.0, 0.0);
    if (k < g0) v = in[(long)row * ldi + k];
    else if (k > g0) v = in[(long)row * ldi + k - 1];
    out[(long)row * ldo + k] = v;
}

__global__ void k_compact_s1(int npw, int g0, const double2* __restrict__ in, long ldi, double2* __restrict__ out,
                             long ldo) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (k >= npw - 1) return;
    out[(long)row * ldo + k] = in[(long)row * ldi + (k < g0 ? k : k + 1)];
}

// out[r][k] = w_k in[r][k] for k < K: weight 2 except for the last entry (the centre of a
// half-sphere row), so that Re sum_k conj(out) y over the half sphere is the full inner product.
template <typename T>
__global__ void k_half_weights(int K, const cplx<T>* __restrict__ in, long ldi, cplx<T>* __restrict__ out, long ldo) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (k >= K) return;
    const T w = k == K - 1 ? T(1) : T(2);
    const cplx<T> v = in[(long)row * ldi + k];
    out[(long)row * ldo + k] = mk<T>(w * v.x, w * v.y);
}

// Make rows exactly Hermitian-symmetric: c_k and c_{npw-1-k} (the coefficients of G and
// -G in the sphere order) <- the symmetric part; the centre (G = 0) becomes real.  One
// thread per pair k <= npw - 1 - k.
__global__ void k_sym_fix(int npw, double2* __restrict__ x, long ld) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    const int m = npw - 1 - k;
    if (k > m) return;
    double2* r = x + (long)j * ld;
    const double2 a = r[k], b = r[m];
    const double2 v = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    r[k] = v;
    r[m] = make_double2(v.x, -v.y);
}

inline dim3 rows_grid(int K, int nrows) {
    PDEP_REQUIRE(nrows <= 65535, PDEP_EINVAL, "too many rows for one launch (max 65535)");
    return dim3((K + 255) / 256, nrows);
}

}  // namespace

template <typename T>
void launch_gemm_ahb(int M, int N, int K, const cplx<T>* A, long lda, const cplx<T>* B, long ldb, cplx<T>* S,
                     long lds, cplx<T>* work, size_t work_elems, hipStream_t s, bool real_out) {
    if (M <= 0 || N <= 0) return;
    PDEP_REQUIRE((N + 63) / 64 <= 65535, PDEP_EINVAL, "gemm_ahb: N too large");
    const int bmc = real_out ? 64 : 32;
    dim3 grid((M + bmc - 1) / bmc, (N + 63) / 64);
    // split K when the output tiles alone cannot fill the chip (about 1k workgroups)
    int splits = 1;
    const long tiles = (long)grid.x * grid.y;
    if (work && tiles < 512) {
        splits = (int)std::min<long>((1024 + tiles - 1) / tiles, std::max(1, K / 256));
        while (splits > 1 && (size_t)splits * N * lds > work_elems) --splits;
    }
    const int kchunk = splits > 1 ? ((K + splits - 1) / splits + 15) / 16 * 16 : K;
    if (splits > 1) splits = (K + kchunk - 1) / kchunk;
    grid.z = splits;
    // algorithmic flops: complex products (8 real flops) or, for real_out, their real parts (4)
    ProfScope prof_(sizeof(T) == sizeof(double) ? K_GEMM_AHB64 : K_GEMM_AHB, s,
                    ((double)M + N) * K * sizeof(cplx<T>) + (double)M * N * sizeof(cplx<T>),
                    (real_out ? 4.0 : 8.0) * (double)M * N * K);
    if (real_out)
        hipLaunchKernelGGL((k_gemm_ahb<T, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb,
                           splits > 1 ? work : S, lds, kchunk, 1);
    else
        hipLaunchKernelGGL((k_gemm_ahb<T, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb,
                           splits > 1 ? work : S, lds, kchunk, 0);
    PDEP_HIP(hipGetLastError());
    if (splits > 1) {
        const long tot = (long)N * M;
        hipLaunchKernelGGL(k_splitk_reduce<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, M, N, lds, splits,
                           work, S, real_out ? 1 : 0);
        PDEP_HIP(hipGetLastError());
    }
}

void launch_splitk_reduce_f32(int M, int N, long lds, int splits, const float2* P, float2* S, hipStream_t s,
                              bool real_out) {
    const long tot = (long)N * M;
    if (tot <= 0) return;
    hipLaunchKernelGGL(k_splitk_reduce<float>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, M, N, lds, splits,
                       P, S, real_out ? 1 : 0);
    PDEP_HIP(hipGetLastError());
}

template <typename T>
void launch_gemm_update(int M, int N, int K, const cplx<T>* A, long lda, const cplx<T>* S, long lds, double alpha,
                        double beta, cplx<T>* Y, long ldy, hipStream_t s, bool real_s) {
    if (N <= 0 || K <= 0) return;
    PDEP_REQUIRE((N + 63) / 64 <= 65535, PDEP_EINVAL, "gemm_update: N too large");
    dim3 grid((K + 63) / 64, (N + 63) / 64);
    ProfScope prof_(sizeof(T) == sizeof(double) ? K_GEMM_UPDATE64 : K_GEMM_UPDATE, s,
                    (double)M * K * sizeof(cplx<T>) + (double)N * M * sizeof(cplx<T>) +
                    (double)N * K * sizeof(cplx<T>) * (beta != 0.0 ? 2.0 : 1.0), (real_s ? 4.0 : 8.0) * (double)M * N * K);
    if (real_s)
        hipLaunchKernelGGL((k_gemm_update<T, true>), grid, dim3(256), 0, s, M, N, K, A, lda, S, lds, alpha, beta, Y,
                           ldy);
    else
        hipLaunchKernelGGL((k_gemm_update<T, false>), grid, dim3(256), 0, s, M, N, K, A, lda, S, lds, alpha, beta, Y,
                           ldy);
    PDEP_HIP(hipGetLastError());
}

void launch_dgemm_sub(int M, int N, int K, const double2* A, long lda, const double2* S, long lds, double2* Y,
                      long ldy, double* sr, size_t sr_elems, hipStream_t s) {
    if (N <= 0 || K <= 0 || M <= 0) return;
    constexpr int TN = 32 * kDgWR, TK = 32 * kDgWC;
    // the real parts of the coefficients, contiguous, in blocks of rows that fit sr
    const int rblk = (int)std::min<long>(N, (long)(sr_elems / (size_t)lds) / TN * TN);
    PDEP_REQUIRE(rblk >= 1, PDEP_EINVAL, "dgemm_sub: coefficient buffer too small");
    for (int r0 = 0; r0 < N; r0 += rblk) {
        const int nr = std::min(rblk, N - r0);
        const long ne = (long)nr * lds;
        hipLaunchKernelGGL(k_real_coefs, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, ne, S + (long)r0 * lds, sr);
        PDEP_HIP(hipGetLastError());
        PDEP_REQUIRE((nr + TN - 1) / TN <= 65535, PDEP_EINVAL, "dgemm_sub: too many rows");
        dim3 grid((2 * K + TK - 1) / TK, (nr + TN - 1) / TN);
        ProfScope prof_(K_GEMM_UPDATE64, s, 16.0 * M * K + 8.0 * nr * M + 32.0 * nr * K, 4.0 * (double)M * nr * K);
        hipLaunchKernelGGL((k_dgemm_sub<kDgWR, kDgWC>), grid, dim3(256), 0, s, M, nr, 2 * K,
                           reinterpret_cast<const double*>(A), 2 * lda, sr, lds,
                           reinterpret_cast<double*>(Y + (long)r0 * ldy), 2 * ldy);
        PDEP_HIP(hipGetLastError());
    }
}

template <typename T>
void launch_row_dots(int nrows, int K, const cplx<T>* a, long lda, const cplx<T>* b, long ldb, double* out,
                     double* out2, hipStream_t s, bool half) {
    if (nrows <= 0) return;
    ProfScope prof_(K_ROW_DOTS, s, 2.0 * nrows * (double)K * sizeof(cplx<T>));
    hipLaunchKernelGGL(k_row_dots<T>, dim3(nrows), dim3(256), 0, s, K, a, lda, b, ldb, out, out2, half ? 1 : 0);
    PDEP_HIP(hipGetLastError());
}

template <typename T>
void launch_cg_init(int nrows, int K, const cplx<T>* b, long ld, cplx<T>* x, cplx<T>* r, cplx<T>* z, const T* kin,
                    const double* shift, int nshift, int precond, hipStream_t s) {
    if (nrows <= 0) return;
    ProfScope prof_(K_CG_UPDATE, s, 4.0 * nrows * (double)K * sizeof(cplx<T>));
    hipLaunchKernelGGL(k_cg_init<T>, rows_grid(K, nrows), dim3(256), 0, s, K, b, ld, x, r, z, kin, shift,
                       nshift > 0 ? nshift : 1, precond);
    PDEP_HIP(hipGetLastError());
}

template <typename T>
void launch_cg_step1(int nrows, int K, cplx<T>* x, cplx<T>* r, cplx<T>* z, const cplx<T>* p, const cplx<T>* q,
                     long ld, const double* rz, const double* pq, int npq, const int* active, const T* kin,
                     const double* shift, int nshift, int precond, hipStream_t s, double* rz_part,
                     double* rr_part, double* rz_new, double* rr, bool half, float* beta, float* alpha_out) {
    if (nrows <= 0) return;
    ProfScope prof_(K_CG_UPDATE, s, (x ? 6.0 : 3.0) * nrows * (double)K * sizeof(cplx<T>));
    const dim3 grid = rows_grid((K + kStep1Elems - 1) / kStep1Elems, nrows);
    hipLaunchKernelGGL(k_cg_step1<T>, grid, dim3(256), 0, s, K, x, r, z, p, q, ld, rz, pq, npq > 0 ? npq : 1,
                       active, kin, shift, nshift > 0 ? nshift : 1, precond, rz_part, rr_part, half ? 1 : 0,
                       alpha_out);
    PDEP_HIP(hipGetLastError());
    if (rz_part) {
        hipLaunchKernelGGL(k_sum_parts, dim3((nrows + 255) / 256), dim3(256), 0, s, nrows, (int)grid.x, rz_part,
                           rr_part, active, rz_new, rr, rz, beta);
        PDEP_HIP(hipGetLastError());
    }
}

template <typename T>
void launch_cg_step2(int nrows, int K, cplx<T>* p, const cplx<T>* z, long ld, const double* rz_new, double* rz,
                     const int* active, hipStream_t s) {
    if (nrows <= 0) return;
    ProfScope prof_(K_CG_UPDATE, s, 3.0 * nrows * (double)K * sizeof(cplx<T>));
    hipLaunchKernelGGL(k_cg_step2<T>, rows_grid(K, nrows), dim3(256), 0, s, K, p, z, ld, rz_new, rz, active);
    PDEP_HIP(hipGetLastError());
}

void launch_cg_check(int nrows, const double* rr, const double* thr2, int* active, int* iters, double* rz,
                     const double* rz_new, int* n_active, int count_iter, hipStream_t s, double rr_max) {
    if (nrows <= 0) return;
    ProfScope prof_(K_CG_UPDATE, s);
    hipLaunchKernelGGL(k_cg_check, dim3((nrows + 255) / 256), dim3(256), 0, s, nrows, rr, thr2, active, iters, rz,
                       rz_new, n_active, count_iter, rr_max);
    PDEP_HIP(hipGetLastError());
}

template <typename Tin, typename Tout>
void launch_convert_rows(int nrows, int K, const cplx<Tin>* in, long ldi, const int* rows, const double* rowscale,
                         cplx<Tout>* out, long ldo, hipStream_t s) {
    if (nrows <= 0) return;
    ProfScope prof_(K_MISC, s);
    hipLaunchKernelGGL((k_convert_scaled<Tin, Tout>), rows_grid(K, nrows), dim3(256), 0, s, K, in, ldi, rows,
                       rowscale, out, ldo);
    PDEP_HIP(hipGetLastError());
}

template <typename T>
void launch_axpy_rows(int nrows, int K, const cplx<T>* d, long ldd, const int* rows, const double* rowscale,
                      double2* x, long ldx, hipStream_t s, bool set) {
    if (nrows <= 0) return;
    PDEP_REQUIRE(ldx >= K && ldx <= (1L << 30), PDEP_EINVAL, "axpy_rows: bad row stride");
    ProfScope prof_(K_MISC, s);
    hipLaunchKernelGGL(k_axpy_rows<T>, rows_grid(set ? (int)ldx : K, nrows), dim3(256), 0, s, K, d, ldd, rows,
                       rowscale, x, ldx, set ? 1 : 0);
    PDEP_HIP(hipGetLastError());
}

template <typename T>
void launch_half_weights(int nrows, int K, const cplx<T>* in, long ldi, cplx<T>* out, long ldo, hipStream_t s) {
    if (nrows <= 0) return;
    hipLaunchKernelGGL(k_half_weights<T>, rows_grid(K, nrows), dim3(256), 0, s, K, in, ldi, out, ldo);
    PDEP_HIP(hipGetLastError());
}
template void launch_half_weights<float>(int, int, const float2*, long, float2*, long, hipStream_t);
template void launch_half_weights<double>(int, int, const double2*, long, double2*, long, hipStream_t);

void launch_residual_rows(int nrows, int K, const double2* b, long ldb, const int* rows, const double2* q, long ldq,
                          double2* r, long ldr, double* out, bool half, hipStream_t s) {
    if (nrows <= 0) return;
    ProfScope prof_(K_MISC, s, 3.0 * nrows * (double)K * sizeof(double2));
    hipLaunchKernelGGL(k_residual_rows, dim3(nrows), dim3(256), 0, s, K, b, ldb, rows, q, ldq, r, ldr, out,
                       half ? 1 : 0);
    PDEP_HIP(hipGetLastError());
}


void launch_sym_fix(int nrows, int npw, double2* x, long ld, hipStream_t s) {
    if (nrows <= 0) return;
    ProfScope prof_(K_MISC, s, 32.0 * nrows * npw);
    hipLaunchKernelGGL(k_sym_fix, rows_grid(npw / 2 + 1, nrows), dim3(256), 0, s, npw, x, ld);
    PDEP_HIP(hipGetLastError());
}

void launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return;
    PDEP_REQUIRE(bytes % 4 == 0, PDEP_EINVAL, "fill_zero: size must be a multiple of 4");
    const size_t n = bytes / 4;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    ProfScope prof_(K_MISC, s);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<uint32_t*>(p), n);
    PDEP_HIP(hipGetLastError());
}

void launch_fill_i32(int* p, int n, int value, hipStream_t s) {
    if (n <= 0) return;
    ProfScope prof_(K_MISC, s);
    hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, value);
    PDEP_HIP(hipGetLastError());
}

void launch_expand_s1(int nrows, int npw, int g0, const double2* in, long ldi, double2* out, long ldo,
                      hipStream_t s) {
    if (nrows <= 0) return;
    ProfScope prof_(K_MISC, s);
    hipLaunchKernelGGL(k_expand_s1, rows_grid(npw, nrows), dim3(256), 0, s, npw, g0, in, ldi, out, ldo);
    PDEP_HIP(hipGetLastError());
}

void launch_compact_s1(int nrows, int npw, int g0, const double2* in, long ldi, double2* out, long ldo,
                       hipStream_t s) {
    if (nrows <= 0) return;
    ProfScope prof_(K_MISC, s);
    hipLaunchKernelGGL(k_compact_s1, rows_grid(npw, nrows), dim3(256), 0, s, npw, g0, in, ldi, out, ldo);
    PDEP_HIP(hipGetLastError());
}

#define PDEP_INST_LA(T)                                                                                         \
    template void launch_gemm_ahb<T>(int, int, int, const cplx<T>*, long, const cplx<T>*, long, cplx<T>*,      \
                                     long, cplx<T>*, size_t, hipStream_t, bool);                              \
    template void launch_gemm_update<T>(int, int, int, const cplx<T>*, long, const cplx<T>*, long, double,     \
                                        double, cplx<T>*, long, hipStream_t, bool);                           \
    template void launch_row_dots<T>(int, int, const cplx<T>*, long, const cplx<T>*, long, double*, double*,   \
                                     hipStream_t, bool);                                                      \
    template void launch_cg_init<T>(int, int, const cplx<T>*, long, cplx<T>*, cplx<T>*, cplx<T>*, const T*,    \
                                    const double*, int, int, hipStream_t);                                    \
    template void launch_cg_step1<T>(int, int, cplx<T>*, cplx<T>*, cplx<T>*, const cplx<T>*, const cplx<T>*,   \
                                     long, const double*, const double*, int, const int*, const T*,            \
                                     const double*, int, int, hipStream_t, double*, double*, double*,          \
                                     double*, bool, float*, float*);                                          \
    template void launch_cg_step2<T>(int, int, cplx<T>*, const cplx<T>*, long, const double*, double*,         \
                                     const int*, hipStream_t);                                                \
    template void launch_axpy_rows<T>(int, int, const cplx<T>*, long, const int*, const double*, double2*,     \
                                      long, hipStream_t, bool);

PDEP_INST_LA(double)
PDEP_INST_LA(float)

template void launch_convert_rows<double, float>(int, int, const double2*, long, const int*, const double*, float2*,
                                                 long, hipStream_t);
template void launch_convert_rows<double, double>(int, int, const double2*, long, const int*, const double*,
                                                  double2*, long, hipStream_t);
template void launch_convert_rows<float, double>(int, int, const float2*, long, const int*, const double*, double2*,
                                                 long, hipStream_t);

}  // namespace pdep
