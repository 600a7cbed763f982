// Dense kernels on blocks of sphere vectors (rows of length K, row stride ld):
//  - the occupied-space projection P_c x = x - Psi (Psi^H x) as a GEMM pair,
//  - per-row inner products and norms (accumulated in FP64),
//  - the element-wise parts of the batched preconditioned CG,
//  - precision conversion, row gathers and updates used by the refinement loop.
#include "pdep_internal.h"

namespace pdep {

namespace {

template <typename T> __device__ __forceinline__ cplx<T> mk(T a, T b) { cplx<T> r; r.x = a; r.y = b; return r; }

// ------------------------------------------------------------------------ GEMMs ---
// S[n][m] = sum_k conj(A[m][k]) B[n][k]; 32 x 32 output tile per workgroup, each thread
// a 2 x 2 sub-tile, K staged through LDS 16 columns at a time.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_ahb(int M, int N, int K, const cplx<T>* __restrict__ A, long lda,
                                                  const cplx<T>* __restrict__ B, long ldb,
                                                  const int* __restrict__ brows, double2* __restrict__ S, long lds) {
    constexpr int TM = 32, TN = 32, TK = 16;
    __shared__ cplx<T> As[TK][TM + 1];
    __shared__ cplx<T> Bs[TK][TN + 1];
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;
    T ar[2][2] = {{0, 0}, {0, 0}}, ai[2][2] = {{0, 0}, {0, 0}};
    for (int k0 = 0; k0 < K; k0 += TK) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int e = tid + 256 * j;
            const int rr = e / TK, kk = e % TK;
            const int gk = k0 + kk;
            const int gm = m0 + rr;
            As[kk][rr] = (gm < M && gk < K) ? A[(long)gm * lda + gk] : mk<T>(0, 0);
            const int gn = n0 + rr;
            cplx<T> bv = mk<T>(0, 0);
            if (gn < N && gk < K) {
                const long brow = brows ? brows[gn] : gn;
                bv = B[brow * ldb + gk];
            }
            Bs[kk][rr] = bv;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < TK; ++kk) {
            const cplx<T> a0 = As[kk][tx], a1 = As[kk][tx + 16];
            const cplx<T> b0 = Bs[kk][ty], b1 = Bs[kk][ty + 16];
            // conj(a) * b
            ar[0][0] += a0.x * b0.x + a0.y * b0.y; ai[0][0] += a0.x * b0.y - a0.y * b0.x;
            ar[0][1] += a0.x * b1.x + a0.y * b1.y; ai[0][1] += a0.x * b1.y - a0.y * b1.x;
            ar[1][0] += a1.x * b0.x + a1.y * b0.y; ai[1][0] += a1.x * b0.y - a1.y * b0.x;
            ar[1][1] += a1.x * b1.x + a1.y * b1.y; ai[1][1] += a1.x * b1.y - a1.y * b1.x;
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int m = m0 + tx + 16 * i, n = n0 + ty + 16 * j;
            if (m < M && n < N) S[(long)n * lds + m] = make_double2((double)ar[i][j], (double)ai[i][j]);
        }
}

// Y[n][k] = beta Y[n][k] + alpha sum_m A[m][k] S[n][m]; tile 16 rows x 128 columns.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_update(int M, int N, int K, const cplx<T>* __restrict__ A, long lda,
                                                     const double2* __restrict__ S, long lds, double alpha,
                                                     double beta, cplx<T>* __restrict__ Y, long ldy,
                                                     const int* __restrict__ yrows) {
    constexpr int TN = 16, TK = 128, TMc = 16;
    __shared__ cplx<T> As[TMc][TK];
    __shared__ cplx<T> Ss[TN][TMc + 1];
    const int k0 = blockIdx.x * TK, n0 = blockIdx.y * TN;
    const int tid = threadIdx.x;
    const int nl = tid / 16, kl = tid % 16;
    T accr[8], acci[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) { accr[j] = 0; acci[j] = 0; }
    for (int m0 = 0; m0 < M; m0 += TMc) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = tid + 256 * j;
            const int mm = e / TK, kk = e % TK;
            const int gm = m0 + mm, gk = k0 + kk;
            As[mm][kk] = (gm < M && gk < K) ? A[(long)gm * lda + gk] : mk<T>(0, 0);
        }
        {
            const int nn = tid / 16, mm = tid % 16;
            const int gn = n0 + nn, gm = m0 + mm;
            double2 sv = make_double2(0.0, 0.0);
            if (gn < N && gm < M) sv = S[(long)gn * lds + gm];
            Ss[nn][mm] = mk<T>((T)sv.x, (T)sv.y);
        }
        __syncthreads();
#pragma unroll 4
        for (int mm = 0; mm < TMc; ++mm) {
            const cplx<T> s = Ss[nl][mm];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const cplx<T> a = As[mm][kl + 16 * j];
                accr[j] += a.x * s.x - a.y * s.y;
                acci[j] += a.x * s.y + a.y * s.x;
            }
        }
        __syncthreads();
    }
    const int n = n0 + nl;
    if (n >= N) return;
    const long yr = yrows ? yrows[n] : n;
    cplx<T>* y = Y + yr * ldy;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = k0 + kl + 16 * j;
        if (k < K) {
            cplx<T> old = beta != 0.0 ? y[k] : mk<T>(0, 0);
            y[k] = mk<T>((T)(beta * old.x + alpha * accr[j]), (T)(beta * old.y + alpha * acci[j]));
        }
    }
}

// ------------------------------------------------------------------- reductions ---
template <typename T>
__global__ __launch_bounds__(256) void k_row_dots(int K, const cplx<T>* __restrict__ a, long lda,
                                                  const cplx<T>* __restrict__ b, long ldb, double* __restrict__ out,
                                                  double* __restrict__ out2) {
    __shared__ double red[2][256];
    const int row = blockIdx.x;
    const cplx<T>* ar = a + (long)row * lda;
    const cplx<T>* br = b + (long)row * ldb;
    double s = 0.0, s2 = 0.0;
    for (int k = threadIdx.x; k < K; k += 256) {
        const cplx<T> x = ar[k], y = br[k];
        s += (double)x.x * (double)y.x + (double)x.y * (double)y.y;
        s2 += (double)x.x * (double)x.x + (double)x.y * (double)x.y;
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
template <typename T>
__device__ __forceinline__ T precond_factor(const T* kin, int k, double shift) {
    const double d = (double)kin[k] - shift;
    return (T)(1.0 / (d > 1.0 ? d : 1.0));
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

template <typename T>
__global__ void k_cg_step1(int K, cplx<T>* __restrict__ x, cplx<T>* __restrict__ r, cplx<T>* __restrict__ z,
                           const cplx<T>* __restrict__ p, const cplx<T>* __restrict__ q, long ld,
                           const double* __restrict__ rz, const double* __restrict__ pq,
                           const int* __restrict__ active, const T* __restrict__ kin,
                           const double* __restrict__ shift, int nshift, int precond) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (k >= K || !active[row]) return;
    const double den = pq[row];
    const T alpha = (T)(den > 0.0 ? rz[row] / den : 0.0);
    const long o = (long)row * ld + k;
    const cplx<T> pv = p[o], qv = q[o];
    cplx<T> xv = x[o], rv = r[o];
    xv.x += alpha * pv.x; xv.y += alpha * pv.y;
    rv.x -= alpha * qv.x; rv.y -= alpha * qv.y;
    x[o] = xv;
    r[o] = rv;
    const T f = precond ? precond_factor(kin, k, shift[row % nshift]) : T(1);
    z[o] = mk<T>(f * rv.x, f * rv.y);
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
                           const double* __restrict__ rz_new, int* __restrict__ n_active, int count_iter) {
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= nrows) return;
    if (active[row]) {
        if (count_iter) iters[row] += 1;
        if (rz_new) rz[row] = rz_new[row];
        const int still = rr[row] > thr2[row];
        active[row] = still;
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
                            const double* __restrict__ rowscale, double2* __restrict__ x, long ldx) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (k >= K) return;
    const double s = rowscale[row];
    const cplx<T> v = d[(long)row * ldd + k];
    const long xr = rows ? rows[row] : row;
    double2 xv = x[xr * ldx + k];
    xv.x += s * (double)v.x;
    xv.y += s * (double)v.y;
    x[xr * ldx + k] = xv;
}

// out[row] = a[rows[row]] - b[row]
__global__ void k_sub_rows(int K, const double2* __restrict__ a, long lda, const int* __restrict__ rows,
                           const double2* __restrict__ b, long ldb, double2* __restrict__ out, long ldo) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (k >= K) return;
    const long ar = rows ? rows[row] : row;
    const double2 x = a[ar * lda + k], y = b[(long)row * ldb + k];
    out[(long)row * ldo + k] = make_double2(x.x - y.x, x.y - y.y);
}

__global__ void k_scatter_rows(int K, const double2* __restrict__ src, long lds, const int* __restrict__ rows,
                               double2* __restrict__ dst, long ldd) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (k >= K) return;
    dst[(long)rows[row] * ldd + k] = src[(long)row * lds + k];
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

inline dim3 rows_grid(int K, int nrows) {
    PDEP_REQUIRE(nrows <= 65535, PDEP_EINVAL, "too many rows for one launch (max 65535)");
    return dim3((K + 255) / 256, nrows);
}

}  // namespace

template <typename T>
void launch_gemm_ahb(int M, int N, int K, const cplx<T>* A, long lda, const cplx<T>* B, long ldb, const int* brows,
                     double2* S, long lds, hipStream_t s) {
    if (M <= 0 || N <= 0) return;
    PDEP_REQUIRE((N + 31) / 32 <= 65535, PDEP_EINVAL, "gemm_ahb: N too large");
    dim3 grid((M + 31) / 32, (N + 31) / 32);
    ProfScope prof_(K_GEMM_AHB, s, ((double)M + N) * K * sizeof(cplx<T>) + (double)M * N * 16.0,
                    8.0 * (double)M * N * K);
    hipLaunchKernelGGL(k_gemm_ahb<T>, grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, brows, S, lds);
    PDEP_HIP(hipGetLastError());
}

template <typename T>
void launch_gemm_update(int M, int N, int K, const cplx<T>* A, long lda, const double2* S, long lds, double alpha,
                        double beta, cplx<T>* Y, long ldy, const int* yrows, hipStream_t s) {
    if (N <= 0 || K <= 0) return;
    PDEP_REQUIRE((N + 15) / 16 <= 65535, PDEP_EINVAL, "gemm_update: N too large");
    dim3 grid((K + 127) / 128, (N + 15) / 16);
    ProfScope prof_(K_GEMM_UPDATE, s, (double)M * K * sizeof(cplx<T>) + (double)N * M * 16.0 +
                    (double)N * K * sizeof(cplx<T>) * (beta != 0.0 ? 2.0 : 1.0), 8.0 * (double)M * N * K);
    hipLaunchKernelGGL(k_gemm_update<T>, grid, dim3(256), 0, s, M, N, K, A, lda, S, lds, alpha, beta, Y, ldy, yrows);
    PDEP_HIP(hipGetLastError());
}

template <typename T>
void launch_row_dots(int nrows, int K, const cplx<T>* a, long lda, const cplx<T>* b, long ldb, double* out,
                     double* out2, hipStream_t s) {
    if (nrows <= 0) return;
    ProfScope prof_(K_ROW_DOTS, s, 2.0 * nrows * (double)K * sizeof(cplx<T>));
    hipLaunchKernelGGL(k_row_dots<T>, dim3(nrows), dim3(256), 0, s, K, a, lda, b, ldb, out, out2);
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
                     long ld, const double* rz, const double* pq, const int* active, const T* kin,
                     const double* shift, int nshift, int precond, hipStream_t s) {
    if (nrows <= 0) return;
    ProfScope prof_(K_CG_UPDATE, s, 7.0 * nrows * (double)K * sizeof(cplx<T>));
    hipLaunchKernelGGL(k_cg_step1<T>, rows_grid(K, nrows), dim3(256), 0, s, K, x, r, z, p, q, ld, rz, pq, active,
                       kin, shift, nshift > 0 ? nshift : 1, precond);
    PDEP_HIP(hipGetLastError());
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
                     const double* rz_new, int* n_active, int count_iter, hipStream_t s) {
    if (nrows <= 0) return;
    ProfScope prof_(K_CG_UPDATE, s);
    hipLaunchKernelGGL(k_cg_check, dim3((nrows + 255) / 256), dim3(256), 0, s, nrows, rr, thr2, active, iters, rz,
                       rz_new, n_active, count_iter);
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
                      double2* x, long ldx, hipStream_t s) {
    if (nrows <= 0) return;
    ProfScope prof_(K_MISC, s);
    hipLaunchKernelGGL(k_axpy_rows<T>, rows_grid(K, nrows), dim3(256), 0, s, K, d, ldd, rows, rowscale, x, ldx);
    PDEP_HIP(hipGetLastError());
}

void launch_sub_rows(int nrows, int K, const double2* a, long lda, const int* rows, const double2* b, long ldb,
                     double2* out, long ldo, hipStream_t s) {
    if (nrows <= 0) return;
    ProfScope prof_(K_MISC, s);
    hipLaunchKernelGGL(k_sub_rows, rows_grid(K, nrows), dim3(256), 0, s, K, a, lda, rows, b, ldb, out, ldo);
    PDEP_HIP(hipGetLastError());
}

void launch_scatter_rows(int nrows, int K, const double2* src, long lds, const int* rows, double2* dst, long ldd,
                         hipStream_t s) {
    if (nrows <= 0) return;
    ProfScope prof_(K_MISC, s);
    hipLaunchKernelGGL(k_scatter_rows, rows_grid(K, nrows), dim3(256), 0, s, K, src, lds, rows, dst, ldd);
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
    template void launch_gemm_ahb<T>(int, int, int, const cplx<T>*, long, const cplx<T>*, long, const int*,    \
                                     double2*, long, hipStream_t);                                            \
    template void launch_gemm_update<T>(int, int, int, const cplx<T>*, long, const double2*, long, double,     \
                                        double, cplx<T>*, long, const int*, hipStream_t);                     \
    template void launch_row_dots<T>(int, int, const cplx<T>*, long, const cplx<T>*, long, double*, double*,   \
                                     hipStream_t);                                                            \
    template void launch_cg_init<T>(int, int, const cplx<T>*, long, cplx<T>*, cplx<T>*, cplx<T>*, const T*,    \
                                    const double*, int, int, hipStream_t);                                    \
    template void launch_cg_step1<T>(int, int, cplx<T>*, cplx<T>*, cplx<T>*, const cplx<T>*, const cplx<T>*,   \
                                     long, const double*, const double*, const int*, const T*, const double*,  \
                                     int, int, hipStream_t);                                                  \
    template void launch_cg_step2<T>(int, int, cplx<T>*, const cplx<T>*, long, const double*, double*,         \
                                     const int*, hipStream_t);                                                \
    template void launch_axpy_rows<T>(int, int, const cplx<T>*, long, const int*, const double*, double2*,     \
                                      long, hipStream_t);

PDEP_INST_LA(double)
PDEP_INST_LA(float)

template void launch_convert_rows<double, float>(int, int, const double2*, long, const int*, const double*, float2*,
                                                 long, hipStream_t);
template void launch_convert_rows<double, double>(int, int, const double2*, long, const int*, const double*,
                                                  double2*, long, hipStream_t);
template void launch_convert_rows<float, double>(int, int, const float2*, long, const int*, const double*, double2*,
                                                 long, hipStream_t);

}  // namespace pdep
