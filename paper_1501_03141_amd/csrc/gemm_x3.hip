// The occupied-space projection GEMM pair in the BF16x3 precision mode: FP32 complex
// operands, each split into a high and a low bfloat16 part (x = hi + lo + O(2^-17 x)),
// and every product taken as lo*hi + hi*lo + hi*hi on the bf16 matrix cores with FP32
// accumulation.  The dropped lo*lo term and the residual of the split leave about
// 16 significant bits per product, so this mode is used only inside the inner solve,
// whose result is corrected by the FP64 residual refinement.
//
// Matrix-core instruction: v_mfma_f32_16x16x32_bf16, one wave.  Lane l supplies
// A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16] (j = 0..7, eight bf16 in
// four dwords, element j in the low half of dword j / 2 when j is even); result slot
// i of lane l is D[4 (l / 16) + i][l % 16].
//
// Complex products are taken as real ones with interleaved (re, im) storage:
//   gemm_ahb    S[n][m] = sum_k conj(A[m][k]) B[n][k]: the real row tile of A uses
//               (a_re, a_im) pairs, the imaginary row tile (-a_im, a_re) pairs, both
//               dotted with the interleaved B row; both tiles are formed from one load.
//   gemm_update Y[n][k] += sum_m S[n][m] A[m][k]: the interleaved S row is the left
//               operand; the right operand has the column tile of Re (pairs
//               (a_re, -a_im) down the contraction) and of Im (pairs (a_im, a_re)).
// Real coefficients (rows real in r, kept as half spheres) need half the products:
//   gemm_ahb_real     S[n][m] = Re sum_k conj(A[m][k]) B[n][k] = the real dot product
//                     of the interleaved rows (only the real row tile of A);
//   gemm_update_real  Y[n][k] += sum_m S[n][m] A[m][k] with S real: a real GEMM over the
//                     interleaved columns k' = 2k + c of Y and A.
#include <cstdint>
#include <type_traits>

#include "pdep_internal.h"

namespace pdep {

namespace {

typedef float x3_f4 __attribute__((ext_vector_type(4)));
typedef __bf16 x3_bf8 __attribute__((ext_vector_type(8)));
typedef uint32_t x3_u4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (operands are finite)
__device__ __forceinline__ uint32_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t h) { return __uint_as_float(h << 16); }

// Split a pair (x0, x1) into a hi dword (.x) and a lo dword (.y), element 0 in the
// low half of each.
__device__ __forceinline__ uint2 split2(float x0, float x1) {
    const uint32_t h0 = bf16_bits(x0), h1 = bf16_bits(x1);
    const uint32_t l0 = bf16_bits(x0 - bf16_value(h0)), l1 = bf16_bits(x1 - bf16_value(h1));
    return make_uint2(h0 | (h1 << 16), l0 | (l1 << 16));
}

// (a, b) -> (-b, a) on a dword of two bf16
__device__ __forceinline__ uint32_t rot_neg_first(uint32_t w) { return ((w >> 16) | (w << 16)) ^ 0x00008000u; }
// (a, b) -> (a, -b)
__device__ __forceinline__ uint32_t neg_second(uint32_t w) { return w ^ 0x80000000u; }
// (a, b) -> (b, a)
__device__ __forceinline__ uint32_t swap_halves(uint32_t w) { return (w >> 16) | (w << 16); }

__device__ __forceinline__ x3_f4 mma3(const x3_u4& ah, const x3_u4& al, const x3_u4& bh, const x3_u4& bl,
                                      x3_f4 c) {
    const x3_bf8 Ah = __builtin_bit_cast(x3_bf8, ah), Al = __builtin_bit_cast(x3_bf8, al);
    const x3_bf8 Bh = __builtin_bit_cast(x3_bf8, bh), Bl = __builtin_bit_cast(x3_bf8, bl);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, Bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bh, c, 0, 0, 0);
    return c;
}

// Four consecutive complex values p[0..3]; entries at or beyond `avail` read as zero.
__device__ __forceinline__ void load4(const float2* p, int avail, float (&v)[8]) {
    if (avail >= 4) {
        const float4 a = *reinterpret_cast<const float4*>(p);
        const float4 b = *reinterpret_cast<const float4*>(p + 2);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float2 c = q < avail ? p[q] : make_float2(0.f, 0.f);
            v[2 * q] = c.x;
            v[2 * q + 1] = c.y;
        }
    }
}

// Store v to p[0..3], entries at or beyond `avail` left untouched.
__device__ __forceinline__ void store4(float2* p, int avail, const float (&v)[8]) {
    if (avail >= 4) {
        *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
        *reinterpret_cast<float4*>(p + 2) = make_float4(v[4], v[5], v[6], v[7]);
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q < avail) p[q] = make_float2(v[2 * q], v[2 * q + 1]);
    }
}

constexpr int kRowB = 80;   // LDS bytes per staged row: 64 B of bf16 + 16 B pad (conflict-free b128 reads)

// S[n][m] = sum_{k in chunk z} conj(A[m][k]) B[n][k].
// WM waves along m (32 complex rows each), 4 / WM waves along n (16 CT rows each).
// k advances 16 complex (32 real) per step; the B tile goes through LDS (shared by
// the waves of one n range), the A fragments are loaded by each wave directly.
// Requires lda, ldb, K-chunk starts multiple of 4 complex (16-byte aligned loads).
// REAL: only the real parts, written as floats (Sv: float [N][lds]); otherwise complex
// (Sv: float2 [N][lds], imaginary parts stored as zero when real_out is set).  With kin
// non-null, B[n][k] is taken times the CG preconditioner 1 / max(kin[k] - shift[n], floor).
//
// STEP (REAL, kin set, a single m tile): B is the CG residual r before the step of this
// iteration; every workgroup first forms alpha = <r, K r> / <p, q> of its rows from the
// previous <r, K r> and the partial sums of <p, q>, stages r - alpha q in place of r,
// writes it back to B (each entry of B is staged by exactly one workgroup), and adds its
// half-sphere weighted |r|^2 and K |r|^2 in FP64; the four lanes of a row combine them
// and the workgroup's sums go to rz_part / rr_part [n][blockIdx.z].  Inactive rows are
// left as they are.  (B is then written through, so it is not declared restrict.)
// The real four-tile variants with four waves along m are held to three waves per SIMD
// (168 registers; they fit without spills).
template <int WM, int CT, bool REAL, bool STEP>
__global__ __launch_bounds__(256, (WM == 4 && CT == 4 && REAL) ? 3 : 1) void k_gemm_ahb_x3(int M, int N, int K, const float2* __restrict__ A, long lda,
                                                     const float2* B, long ldb, void* __restrict__ Sv,
                                                     long lds, int kchunk, int real_out, const float* __restrict__ kin,
                                                     const double* __restrict__ shift, float kfloor,
                                                     CgStepFuse cs) {
    constexpr int NSUB = REAL ? 1 : 2;   // row tiles of A: real part, imaginary part
    constexpr int WN = 4 / WM;
    constexpr int BMC = 32 * WM, BN = 16 * CT * WN;
    constexpr int IT = BN / 64;   // B staging items per thread (4 complex each)
    static_assert(!STEP || REAL, "the fused CG step works on real coefficients");
    __shared__ __align__(16) unsigned char Bs[2][BN * kRowB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int m0 = blockIdx.x * BMC, n0 = blockIdx.y * BN;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(K, kbeg + kchunk);
    const long zoff = (long)blockIdx.z * N * lds;
    const int lr = lane & 15, lq = lane >> 4;

    float alp[IT], qb[IT][8];
    bool act[IT];
    double srz[IT], srr[IT];
    if constexpr (STEP) {
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            const int n = n0 + ((tid + 256 * j) >> 2);
            act[j] = n < N && cs.active[n];
            double a = 0.0;
            if (act[j]) {
                double den = 0.0;
                for (int g = 0; g < cs.npq; ++g) den += cs.pq[(long)n * cs.npq + g];
                a = den > 0.0 ? cs.rz[n] / den : 0.0;
                if (blockIdx.z == 0 && (tid & 3) == 0) cs.alpha_out[n] = (float)a;
            }
            alp[j] = (float)a;
            srz[j] = 0.0;
            srr[j] = 0.0;
        }
    }

    x3_f4 acc[2][NSUB][CT];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int s = 0; s < NSUB; ++s)
#pragma unroll
            for (int c = 0; c < CT; ++c) acc[g][s][c] = x3_f4{0.f, 0.f, 0.f, 0.f};

    float ra[2][8], rb[IT][8], kb[IT][4];
    auto fetch = [&](int kc) {
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const int m = m0 + 32 * wm + 16 * g + lr;
            const int k = kc + 4 * lq;
            const int avail = m < M ? kend - k : 0;
            load4(A + (long)(m < M ? m : 0) * lda + k, avail, ra[g]);
        }
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            const int e = tid + 256 * j;
            const int n = n0 + (e >> 2), k = kc + 4 * (e & 3);
            const int avail = n < N ? kend - k : 0;
            load4(B + (long)(n < N ? n : 0) * ldb + k, avail, rb[j]);
            if constexpr (STEP) load4(cs.q + (long)(n < N ? n : 0) * ldb + k, act[j] ? avail : 0, qb[j]);
            if (kin) {
#pragma unroll
                for (int q = 0; q < 4; ++q) kb[j][q] = q < avail ? kin[k + q] : 0.f;
            }
        }
    };

    if (kbeg < kend) fetch(kbeg);
    for (int kc = kbeg; kc < kend; kc += 16) {
        // stage B (split) in LDS, A fragments in registers
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            const int e = tid + 256 * j;
            if constexpr (STEP) {
                const int n = n0 + (e >> 2), k = kc + 4 * (e & 3);
                if (act[j]) {
#pragma unroll
                    for (int q = 0; q < 8; ++q) rb[j][q] -= alp[j] * qb[j][q];
                    store4(const_cast<float2*>(B) + (long)n * ldb + k, kend - k, rb[j]);
                }
                const float sh = n < N ? (float)shift[n] : 0.f;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float d = kb[j][q] - sh;
                    const float f = __builtin_amdgcn_rcpf(d > kfloor ? d : kfloor);
                    // entries past the chunk were read as zero and add nothing
                    const double w = k + q == K - 1 ? 1.0 : 2.0;
                    const double n2 = w * ((double)rb[j][2 * q] * (double)rb[j][2 * q] +
                                           (double)rb[j][2 * q + 1] * (double)rb[j][2 * q + 1]);
                    srr[j] += n2;
                    srz[j] += (double)f * n2;
                    rb[j][2 * q] *= f;
                    rb[j][2 * q + 1] *= f;
                }
            } else if (kin) {
                const int n = n0 + (e >> 2);
                const float sh = n < N ? (float)shift[n] : 0.f;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float d = kb[j][q] - sh;
                    const float f = __builtin_amdgcn_rcpf(d > kfloor ? d : kfloor);
                    rb[j][2 * q] *= f;
                    rb[j][2 * q + 1] *= f;
                }
            }
            x3_u4 h, l;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint2 w = split2(rb[j][2 * q], rb[j][2 * q + 1]);
                h[q] = w.x;
                l[q] = w.y;
            }
            const int off = (e >> 2) * kRowB + (e & 3) * 16;
            *reinterpret_cast<x3_u4*>(&Bs[0][off]) = h;
            *reinterpret_cast<x3_u4*>(&Bs[1][off]) = l;
        }
        x3_u4 ah[2][NSUB], al[2][NSUB];   // [g][s]
#pragma unroll
        for (int g = 0; g < 2; ++g) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint2 w = split2(ra[g][2 * q], ra[g][2 * q + 1]);
                ah[g][0][q] = w.x;
                al[g][0][q] = w.y;
            }
            if constexpr (!REAL) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    ah[g][NSUB - 1][q] = rot_neg_first(ah[g][0][q]);
                    al[g][NSUB - 1][q] = rot_neg_first(al[g][0][q]);
                }
            }
        }
        __syncthreads();
        if (kc + 16 < kend) fetch(kc + 16);
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int off = (16 * CT * wn + 16 * c + lr) * kRowB + lq * 16;
            const x3_u4 bh = *reinterpret_cast<const x3_u4*>(&Bs[0][off]);
            const x3_u4 bl = *reinterpret_cast<const x3_u4*>(&Bs[1][off]);
#pragma unroll
            for (int g = 0; g < 2; ++g)
#pragma unroll
                for (int s = 0; s < NSUB; ++s) acc[g][s][c] = mma3(ah[g][s], al[g][s], bh, bl, acc[g][s][c]);
        }
        __syncthreads();
    }
    if constexpr (STEP) {
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            double a = srz[j], b = srr[j];
            a += __shfl_xor(a, 1);
            b += __shfl_xor(b, 1);
            a += __shfl_xor(a, 2);
            b += __shfl_xor(b, 2);
            const int n = n0 + ((tid + 256 * j) >> 2);
            if ((tid & 3) == 0 && act[j]) {
                cs.rz_part[(long)n * gridDim.z + blockIdx.z] = a;
                cs.rr_part[(long)n * gridDim.z + blockIdx.z] = b;
            }
        }
    }
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = m0 + 32 * wm + 16 * g + 4 * lq + i;
                const int n = n0 + 16 * CT * wn + 16 * c + lr;
                if (m < M && n < N) {
                    if constexpr (REAL) {
                        static_cast<float*>(Sv)[zoff + (long)n * lds + m] = acc[g][0][c][i];
                    } else {
                        static_cast<float2*>(Sv)[zoff + (long)n * lds + m] =
                            make_float2(acc[g][0][c][i], real_out ? 0.f : acc[g][NSUB - 1][c][i]);
                    }
                }
            }
}

// S[n][m] = sum_z P[z][n][m] over real partial products (z in order).
__global__ void k_splitk_reduce_real(int M, int N, long lds, int splits, const float* __restrict__ P,
                                     float* __restrict__ S) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)N * M) return;
    const long n = e / M, m = e - n * M;
    const long stride = (long)N * lds;
    float v = 0.f;
    for (int z = 0; z < splits; ++z) v += P[z * stride + n * lds + m];
    S[n * lds + m] = v;
}

// The fused CG step's reductions in one launch: threads e < N M reduce the split-K partial
// products as k_splitk_reduce_real (when splits > 1); the next N threads form, for the
// active rows, rz_new = sum of the <r, K r> parts, rr = sum of the ||r||^2 parts (parts
// in order) and beta = rz_new / rz_old (0 when rz_old = 0); thread 0 clears cs.count.
__global__ void k_reduce_step(int M, int N, long lds, int splits, const float* __restrict__ P, float* __restrict__ S,
                              CgStepFuse cs) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0 && cs.count) *cs.count = 0;
    const long nm = splits > 1 ? (long)N * M : 0;
    if (e < nm) {
        const long n = e / M, m = e - n * M;
        const long stride = (long)N * lds;
        float v = 0.f;
        for (int z = 0; z < splits; ++z) v += P[z * stride + n * lds + m];
        S[n * lds + m] = v;
        return;
    }
    const long row = e - nm;
    if (row >= N || !cs.active[row]) return;
    double a = 0.0, b = 0.0;
    for (int g = 0; g < splits; ++g) {
        a += cs.rz_part[row * splits + g];
        b += cs.rr_part[row * splits + g];
    }
    cs.rz_new[row] = a;
    cs.rr[row] = b;
    const double d = cs.rz[row];
    cs.beta[row] = (float)(d != 0.0 ? a / d : 0.0);
}

// Eight consecutive floats p[0..7] (16-byte aligned); entries at or beyond `avail` read as zero.
__device__ __forceinline__ void load8f(const float* p, int avail, float (&v)[8]) {
    if (avail >= 8) {
        const float4 a = *reinterpret_cast<const float4*>(p);
        const float4 b = *reinterpret_cast<const float4*>(p + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = q < avail ? p[q] : 0.f;
    }
}

// Y[n][k] = beta Y[n][k] + alpha sum_m S[n][m] A[m][k], S real (float [N][lds]).
// Real GEMM over the real and imaginary parts of Y and A.  Workgroup tile: 128 rows n
// (32 per wave) x 64 complex columns k; the contraction advances 32 m per step.  The A
// tile (32 m x 64 k) is split into LDS as [column][m] (bf16 pairs of adjacent m per
// dword, hi and lo planes), column 32 t + 16 c + j holding part c of k = 16 t + j, so
// that output tiles 2t and 2t + 1 give a lane the real and imaginary part of the same
// k (stored as one float2).  Each wave loads its own S fragments (8 consecutive m).
// Requires lda and lds multiples of 4 (16-byte aligned loads).
// FUSED (the CG direction update): Y = p and, for active rows n only,
//   p <- K r - sum_m S[n][m] A[m][k] + beta_n p,  K = 1 / max(kin[k] - shift[n], floor),
//   beta_n from the array beta; alpha and beta are unused.  Before that, x[n] += a_n p[n]
//   (the old p) with a_n from the array xalpha (x has the stride of p).
struct DirUpdate {
    const float2* r;
    long ldr;
    const float* kin;
    const double* shift;
    const float* beta;
    const float* xalpha;
    float2* x;
    const int* xrow;   // row of x that slot n updates (null: row n)
    const int* active;
    float kfloor;
};
template <bool FUSED, int AR = 2>
__global__ __launch_bounds__(256, 4) void k_gemm_update_x3r(int M, int N, int K, const float2* __restrict__ A,
                                                         long lda, const float* __restrict__ S, long lds,
                                                         float alpha, float beta, float2* __restrict__ Y, long ldy,
                                                         DirUpdate du) {
    constexpr int BK = 64, BNR = 64 * AR;   // AR 16-row halves per wave
    __shared__ __align__(16) unsigned char As[2][2 * BK * kRowB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int k0 = blockIdx.x * BK, n0 = blockIdx.y * BNR;
    const int lr = lane & 15, lq = lane >> 4;

    x3_f4 acc[AR][8];   // [a: 16-row part of the wave's rows][b: 16 real columns]
#pragma unroll
    for (int a = 0; a < AR; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = x3_f4{0.f, 0.f, 0.f, 0.f};

    // A staging: thread -> (rows 2 mp and 2 mp + 1, 4 consecutive k from kg)
    const int mp = tid & 15, kg = 4 * (tid >> 4);
    float rs[AR][8], ra[2][8];
    auto fetch = [&](int mc) {
#pragma unroll
        for (int a = 0; a < AR; ++a) {
            const int n = n0 + 16 * AR * wave + 16 * a + lr;
            const int m = mc + 8 * lq;
            const int avail = n < N ? M - m : 0;
            load8f(S + (long)(n < N ? n : 0) * lds + m, avail, rs[a]);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int m = mc + 2 * mp + h, k = k0 + kg;
            const int avail = m < M ? K - k : 0;
            load4(A + (long)(m < M ? m : 0) * lda + k, avail, ra[h]);
        }
    };

    fetch(0);
    for (int mc = 0; mc < M; mc += 32) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const uint2 w = split2(ra[0][2 * q + c], ra[1][2 * q + c]);
                const int kl = kg + q;
                const int off = (32 * (kl >> 4) + 16 * c + (kl & 15)) * kRowB + mp * 4;
                *reinterpret_cast<uint32_t*>(&As[0][off]) = w.x;
                *reinterpret_cast<uint32_t*>(&As[1][off]) = w.y;
            }
        x3_u4 sh[AR], sl[AR];
#pragma unroll
        for (int a = 0; a < AR; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint2 w = split2(rs[a][2 * q], rs[a][2 * q + 1]);
                sh[a][q] = w.x;
                sl[a][q] = w.y;
            }
        __syncthreads();
        if (mc + 32 < M) fetch(mc + 32);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int off = (16 * b + lr) * kRowB + lq * 16;
            const x3_u4 bh = *reinterpret_cast<const x3_u4*>(&As[0][off]);
            const x3_u4 bl = *reinterpret_cast<const x3_u4*>(&As[1][off]);
#pragma unroll
            for (int a = 0; a < AR; ++a) acc[a][b] = mma3(sh[a], sl[a], bh, bl, acc[a][b]);
        }
        __syncthreads();
    }
    if constexpr (FUSED) {
        // The lane's rows are updated EB at a time, every load of a batch (r, p, x and the
        // kinetic energies of its columns) issued before the first store: stores to x and
        // p may alias the next entry's loads as far as the compiler knows, so an entry-by-
        // entry loop waits for memory once per entry.  One row per batch measured best
        // (more rows hold more registers and lower the occupancy).
        constexpr int EB = 1;
        float kk[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = k0 + 16 * t + lr;
            kk[t] = du.kin[k < K ? k : K - 1];
        }
        // the active flags and x rows of all the lane's rows, loaded together up front, so
        // that a row's loads below depend on registers only (loaded per row, each row waited
        // for its flag and then for its x row before its data loads)
        bool lv[AR][4];
        int xr[AR][4];
#pragma unroll
        for (int a = 0; a < AR; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int n = n0 + 16 * AR * wave + 16 * a + 4 * lq + i;
                const int nn = n < N ? n : 0;
                lv[a][i] = (n < N) & (du.active[nn] != 0);
                xr[a][i] = du.xrow ? du.xrow[nn] : nn;
            }
#pragma unroll
        for (int a = 0; a < AR; ++a)
#pragma unroll
            for (int i0 = 0; i0 < 4; i0 += EB) {
                bool live[EB];
                float bn[EB], an[EB], sh[EB];
                long xo[EB];
                float2 rv[EB][4], pv[EB][4], xv[EB][4];
#pragma unroll
                for (int e = 0; e < EB; ++e) {
                    const int n = n0 + 16 * AR * wave + 16 * a + 4 * lq + i0 + e;
                    live[e] = lv[a][i0 + e];
                    const int nn = n < N ? n : 0;
                    bn[e] = du.beta[nn];
                    an[e] = du.xalpha[nn];
                    sh[e] = (float)du.shift[nn];
                    xo[e] = (long)xr[a][i0 + e] * ldy;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        int k = k0 + 16 * t + lr;
                        k = k < K ? k : K - 1;
                        rv[e][t] = du.r[(long)nn * du.ldr + k];
                        pv[e][t] = Y[(long)nn * ldy + k];
                        xv[e][t] = du.x[xo[e] + k];
                    }
                }
#pragma unroll
                for (int e = 0; e < EB; ++e) {
                    if (!live[e]) continue;
                    const int n = n0 + 16 * AR * wave + 16 * a + 4 * lq + i0 + e;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int k = k0 + 16 * t + lr;
                        if (k < K) {
                            const float d = kk[t] - sh[e];
                            const float f = __builtin_amdgcn_rcpf(d > du.kfloor ? d : du.kfloor);
                            float2 x = xv[e][t];
                            x.x += an[e] * pv[e][t].x;
                            x.y += an[e] * pv[e][t].y;
                            du.x[xo[e] + k] = x;
                            Y[(long)n * ldy + k] =
                                make_float2(f * rv[e][t].x - acc[a][2 * t][i0 + e] + bn[e] * pv[e][t].x,
                                            f * rv[e][t].y - acc[a][2 * t + 1][i0 + e] + bn[e] * pv[e][t].y);
                        }
                    }
                }
            }
    } else {
#pragma unroll
        for (int a = 0; a < AR; ++a) {
            // the row group's old values are loaded together (clamped indices) and held
            // before the guarded stores: loaded inside the guard, each would be waited for
            // on its own
            float2 old[4][4];
            if (beta != 0.f) {
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int n = min(n0 + 16 * AR * wave + 16 * a + 4 * lq + i, N - 1);
                        const int k = min(k0 + 16 * t + lr, K - 1);
                        old[t][i] = Y[(long)n * ldy + k];
                    }
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int i = 0; i < 4; ++i) asm volatile("" ::"v"(old[t][i].x), "v"(old[t][i].y));
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int n = n0 + 16 * AR * wave + 16 * a + 4 * lq + i;
                    const int k = k0 + 16 * t + lr;
                    if (n < N && k < K) {
                        float2 o = make_float2(alpha * acc[a][2 * t][i], alpha * acc[a][2 * t + 1][i]);
                        if (beta != 0.f) {
                            o.x += beta * old[t][i].x;
                            o.y += beta * old[t][i].y;
                        }
                        Y[(long)n * ldy + k] = o;
                    }
                }
        }
    }
}

// Y[n][k] = beta Y[n][k] + alpha sum_m S[n][m] A[m][k].
// Workgroup tile: 128 rows n (32 per wave) x 64 complex columns k; the contraction
// advances 16 complex m (32 real) per step.  The A tile (16 m x 64 k) is split into
// LDS as [k][m] dwords (hi: (hi(re), hi(im)), lo likewise); each wave loads its own
// S fragments.  Requires lds multiple of 4 complex (16-byte aligned S loads).
__global__ __launch_bounds__(256) void k_gemm_update_x3(int M, int N, int K, const float2* __restrict__ A,
                                                        long lda, const float2* __restrict__ S, long lds,
                                                        float alpha, float beta, float2* __restrict__ Y, long ldy) {
    constexpr int BK = 64, BNR = 128;
    __shared__ __align__(16) unsigned char As[2][BK * kRowB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int k0 = blockIdx.x * BK, n0 = blockIdx.y * BNR;
    const int lr = lane & 15, lq = lane >> 4;

    x3_f4 acc[2][4][2];   // [a][b][d]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int d = 0; d < 2; ++d) acc[a][b][d] = x3_f4{0.f, 0.f, 0.f, 0.f};

    // A staging: thread -> (m row, 4 consecutive k)
    const int sm = tid >> 4, sk = 4 * (tid & 15);
    float rs[2][8], ra[8];
    auto fetch = [&](int mc) {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int n = n0 + 32 * wave + 16 * a + lr;
            const int m = mc + 4 * lq;
            const int avail = n < N ? M - m : 0;
            load4(S + (long)(n < N ? n : 0) * lds + m, avail, rs[a]);
        }
        const int m = mc + sm, k = k0 + sk;
        const int avail = m < M ? K - k : 0;
        load4(A + (long)(m < M ? m : 0) * lda + k, avail, ra);
    };

    fetch(0);
    for (int mc = 0; mc < M; mc += 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint2 w = split2(ra[2 * q], ra[2 * q + 1]);
            const int off = (sk + q) * kRowB + sm * 4;
            *reinterpret_cast<uint32_t*>(&As[0][off]) = w.x;
            *reinterpret_cast<uint32_t*>(&As[1][off]) = w.y;
        }
        x3_u4 sh[2], sl[2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint2 w = split2(rs[a][2 * q], rs[a][2 * q + 1]);
                sh[a][q] = w.x;
                sl[a][q] = w.y;
            }
        __syncthreads();
        if (mc + 16 < M) fetch(mc + 16);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int off = (16 * b + lr) * kRowB + lq * 16;
            const x3_u4 wh = *reinterpret_cast<const x3_u4*>(&As[0][off]);
            const x3_u4 wl = *reinterpret_cast<const x3_u4*>(&As[1][off]);
            x3_u4 bh[2], bl[2];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                bh[0][q] = neg_second(wh[q]);     // (re, -im): real output column
                bl[0][q] = neg_second(wl[q]);
                bh[1][q] = swap_halves(wh[q]);    // (im, re): imaginary output column
                bl[1][q] = swap_halves(wl[q]);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int d = 0; d < 2; ++d) acc[a][b][d] = mma3(sh[a], sl[a], bh[d], bl[d], acc[a][b][d]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int n = n0 + 32 * wave + 16 * a + 4 * lq + i;
                const int k = k0 + 16 * b + lr;
                if (n < N && k < K) {
                    float2* y = Y + (long)n * ldy + k;
                    float2 o = make_float2(alpha * acc[a][b][0][i], alpha * acc[a][b][1][i]);
                    if (beta != 0.f) {
                        const float2 old = *y;
                        o.x += beta * old.x;
                        o.y += beta * old.y;
                    }
                    *y = o;
                }
            }
}

}  // namespace

namespace {

// REAL: S and work are float arrays (real parts only).
template <bool REAL>
int gemm_ahb_x3(int M, int N, int K, const float2* A, long lda, const float2* B, long ldb, void* S, long lds,
                void* work, size_t work_elems, hipStream_t s, bool real_out, const float* kin = nullptr,
                const double* shift = nullptr, float kfloor = 0.f, const CgStepFuse* cs = nullptr,
                int max_parts = 0, GemmShape shape = {}) {
    if (M <= 0 || N <= 0) return 0;
    PDEP_REQUIRE(lda % 4 == 0 && ldb % 4 == 0, PDEP_EINVAL, "gemm_ahb_x3: leading dimensions must be multiples of 4");
    const int WM = M <= 32 ? 1 : (M <= 64 ? 2 : 4);
    // eight column tiles per wave when all four waves run along m and are mostly full;
    // the fused CG step keeps four (three waves per SIMD instead of two: its extra r and
    // q traffic needs the latency hiding more than the shared B tile; 5-12% faster)
    const int CT = (M > 96 && !cs) ? (shape.col_tiles == 4 ? 4 : 8) : 4;
    const int BMC = 32 * WM, BN = 16 * CT * (4 / WM);
    PDEP_REQUIRE((N + BN - 1) / BN <= 65535, PDEP_EINVAL, "gemm_ahb_x3: N too large");
    dim3 grid((M + BMC - 1) / BMC, (N + BN - 1) / BN);
    if (cs) {
        PDEP_REQUIRE(REAL && kin && grid.x == 1 && max_parts > 0, PDEP_EINVAL,
                     "gemm_ahb_x3: the fused CG step needs real output, the preconditioner and one m tile");
    }
    // split K until about 512 workgroups (two per CU; more splits only add partial-sum
    // traffic: measured best at 512 for N_v = 128 and 512); 1024 for the fused step
    int splits = 1;
    const long tiles = (long)grid.x * grid.y;
    const long target = shape.splitk_target > 0 ? shape.splitk_target : (cs ? 1024 : 512);
    if (work && tiles < target) {
        splits = (int)std::min<long>((target + tiles - 1) / tiles, std::max(1, K / 256));
        if (cs) splits = std::min(splits, max_parts);
        while (splits > 1 && (size_t)splits * N * lds > work_elems) --splits;
    }
    const int kchunk = splits > 1 ? ((K + splits - 1) / splits + 15) / 16 * 16 : K;
    if (splits > 1) splits = (K + kchunk - 1) / kchunk;
    grid.z = splits;
    // algorithmic: complex products (8 real flops) or their real parts (4); the fused
    // step also reads q and writes r back
    const double esz = REAL ? sizeof(float) : sizeof(float2);
    ProfScope prof_(K_GEMM_AHB, s,
                    ((double)M + N * (cs ? 3.0 : 1.0)) * K * sizeof(float2) + (double)M * N * esz,
                    (REAL ? 4.0 : 8.0) * (double)M * N * K);
    void* out = splits > 1 ? work : S;
    const int ro = (real_out && splits == 1) ? 1 : 0;
    const CgStepFuse none{};
    auto launch = [&](auto step) {
        constexpr bool ST = decltype(step)::value;
        const CgStepFuse& c = cs ? *cs : none;
        if (WM == 1)
            hipLaunchKernelGGL((k_gemm_ahb_x3<1, 4, REAL, ST>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, out,
                               lds, kchunk, ro, kin, shift, kfloor, c);
        else if (WM == 2)
            hipLaunchKernelGGL((k_gemm_ahb_x3<2, 4, REAL, ST>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, out,
                               lds, kchunk, ro, kin, shift, kfloor, c);
        else if (CT == 8)
            hipLaunchKernelGGL((k_gemm_ahb_x3<4, 8, REAL, ST>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, out,
                               lds, kchunk, ro, kin, shift, kfloor, c);
        else
            hipLaunchKernelGGL((k_gemm_ahb_x3<4, 4, REAL, ST>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, out,
                               lds, kchunk, ro, kin, shift, kfloor, c);
    };
    if constexpr (REAL) {
        if (cs)
            launch(std::true_type{});
        else
            launch(std::false_type{});
    } else {
        launch(std::false_type{});
    }
    PDEP_HIP(hipGetLastError());
    if (cs) {
        if constexpr (REAL) {
            const long tot = (splits > 1 ? (long)N * M : 0) + N;
            hipLaunchKernelGGL(k_reduce_step, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, M, N, lds, splits,
                               static_cast<const float*>(work), static_cast<float*>(S), *cs);
            PDEP_HIP(hipGetLastError());
        }
    } else if (splits > 1) {
        if constexpr (REAL) {
            const long tot = (long)N * M;
            hipLaunchKernelGGL(k_splitk_reduce_real, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, M, N, lds,
                               splits, static_cast<const float*>(work), static_cast<float*>(S));
            PDEP_HIP(hipGetLastError());
        } else {
            launch_splitk_reduce_f32(M, N, lds, splits, static_cast<const float2*>(work), static_cast<float2*>(S), s,
                                     real_out);
        }
    }
    return splits;
}

}  // namespace

void launch_gemm_ahb_x3(int M, int N, int K, const float2* A, long lda, const float2* B, long ldb, float2* S,
                        long lds, float2* work, size_t work_elems, hipStream_t s, bool real_out) {
    gemm_ahb_x3<false>(M, N, K, A, lda, B, ldb, S, lds, work, work_elems, s, real_out);
}

void launch_gemm_ahb_x3_real(int M, int N, int K, const float2* A, long lda, const float2* B, long ldb, float* S,
                             long lds, float* work, size_t work_elems, hipStream_t s, const float* kin,
                             const double* shift, double kfloor, GemmShape shape) {
    PDEP_REQUIRE(lds % 4 == 0, PDEP_EINVAL, "gemm_ahb_x3_real: lds must be a multiple of 4");
    PDEP_REQUIRE(!kin || (shift && kfloor > 0), PDEP_EINVAL, "gemm_ahb_x3_real: preconditioner needs shifts");
    gemm_ahb_x3<true>(M, N, K, A, lda, B, ldb, S, lds, work, work_elems, s, true, kin, shift, (float)kfloor, nullptr,
                      0, shape);
}

int launch_gemm_ahb_x3_step(int M, int N, int K, const float2* A, long lda, float2* r, long ldr, float* S, long lds,
                            float* work, size_t work_elems, hipStream_t s, const float* kin, const double* shift,
                            double kfloor, const CgStepFuse& cs, int max_parts, GemmShape shape) {
    PDEP_REQUIRE(lds % 4 == 0, PDEP_EINVAL, "gemm_ahb_x3_step: lds must be a multiple of 4");
    PDEP_REQUIRE(kin && shift && kfloor > 0, PDEP_EINVAL, "gemm_ahb_x3_step: the step needs the preconditioner");
    PDEP_REQUIRE(M <= 128, PDEP_EINVAL, "gemm_ahb_x3_step: at most 128 coefficient rows");
    return gemm_ahb_x3<true>(M, N, K, A, lda, r, ldr, S, lds, work, work_elems, s, true, kin, shift, (float)kfloor,
                             &cs, max_parts, shape);
}

void launch_gemm_update_x3_real(int M, int N, int K, const float2* A, long lda, const float* S, long lds,
                                double alpha, double beta, float2* Y, long ldy, hipStream_t s) {
    if (N <= 0 || K <= 0) return;
    PDEP_REQUIRE(lda % 4 == 0 && lds % 4 == 0, PDEP_EINVAL,
                 "gemm_update_x3_real: leading dimensions must be multiples of 4");
    PDEP_REQUIRE((N + 63) / 64 <= 65535, PDEP_EINVAL, "gemm_update_x3_real: N too large");
    dim3 grid((K + 63) / 64, (N + 63) / 64);
    ProfScope prof_(K_GEMM_UPDATE, s, (double)M * K * sizeof(float2) + (double)N * M * sizeof(float) +
                    (double)N * K * sizeof(float2) * (beta != 0.0 ? 2.0 : 1.0), 4.0 * (double)M * N * K);
    hipLaunchKernelGGL((k_gemm_update_x3r<false, 1>), grid, dim3(256), 0, s, M, N, K, A, lda, S, lds, (float)alpha,
                       (float)beta, Y, ldy, DirUpdate{});
    PDEP_HIP(hipGetLastError());
}

void launch_cg_direction_x3(int M, int N, int K, const float2* A, long lda, const float* S, long lds, const float2* r,
                            long ldr, const float* kin, const double* shift, double kfloor, const float* beta,
                            const float* alpha, float2* x, const int* xrow, const int* active, float2* p, long ldp,
                            hipStream_t s) {
    if (N <= 0 || K <= 0) return;
    PDEP_REQUIRE(lda % 4 == 0 && lds % 4 == 0, PDEP_EINVAL,
                 "cg_direction_x3: leading dimensions must be multiples of 4");
    // 16 rows per wave (64 per workgroup): the epilogue-heavy fused form runs 6-10% faster
    // than with 32 at N_v = 128 (equal at 512)
    PDEP_REQUIRE((N + 63) / 64 <= 65535, PDEP_EINVAL, "cg_direction_x3: N too large");
    dim3 grid((K + 63) / 64, (N + 63) / 64);
    ProfScope prof_(K_GEMM_UPDATE, s, (double)M * K * sizeof(float2) + (double)N * M * sizeof(float) +
                    (double)N * K * sizeof(float2) * 5.0, 4.0 * (double)M * N * K);
    const DirUpdate du{r, ldr, kin, shift, beta, alpha, x, xrow, active, (float)kfloor};
    hipLaunchKernelGGL((k_gemm_update_x3r<true, 1>), grid, dim3(256), 0, s, M, N, K, A, lda, S, lds, -1.f, 0.f, p,
                       ldp, du);
    PDEP_HIP(hipGetLastError());
}

void launch_gemm_update_x3(int M, int N, int K, const float2* A, long lda, const float2* S, long lds, double alpha,
                           double beta, float2* Y, long ldy, hipStream_t s) {
    if (N <= 0 || K <= 0) return;
    PDEP_REQUIRE(lda % 4 == 0 && lds % 4 == 0, PDEP_EINVAL,
                 "gemm_update_x3: leading dimensions must be multiples of 4");
    PDEP_REQUIRE((N + 127) / 128 <= 65535, PDEP_EINVAL, "gemm_update_x3: N too large");
    dim3 grid((K + 63) / 64, (N + 127) / 128);
    ProfScope prof_(K_GEMM_UPDATE, s, (double)M * K * sizeof(float2) + (double)N * M * sizeof(float2) +
                    (double)N * K * sizeof(float2) * (beta != 0.0 ? 2.0 : 1.0), 8.0 * (double)M * N * K);
    hipLaunchKernelGGL(k_gemm_update_x3, grid, dim3(256), 0, s, M, N, K, A, lda, S, lds, (float)alpha, (float)beta, Y,
                       ldy);
    PDEP_HIP(hipGetLastError());
}

}  // namespace pdep
