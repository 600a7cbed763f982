// Internal declarations of the PDEP chi0 library: device types, basis tables,
// kernel launchers and the context.  Not part of the public ABI (include/pdep.h).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pdep.h"

// capi.hip: sets the calling thread's pdep_last_error() message (internal)
extern "C" void pdep_set_error_message(const char* m);

namespace pdep {

// ---------------------------------------------------------------- errors --------
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define PDEP_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            throw ::pdep::Error(PDEP_EDEVICE, std::string(#call) + ": " +                \
                                                  hipGetErrorString(e_));                \
    } while (0)

#define PDEP_REQUIRE(cond, code, msg)                                                    \
    do {                                                                                 \
        if (!(cond)) throw ::pdep::Error((code), (msg));                                 \
    } while (0)

// ---------------------------------------------------------------- complex --------
template <typename T> struct V2;
template <> struct V2<double> { using type = double2; };
template <> struct V2<float> { using type = float2; };
template <typename T> using cplx = typename V2<T>::type;

// ---------------------------------------------------------------- memory ---------
struct Allocator {
    pdep_allocator a{};
    void* get(size_t bytes);
    void put(void* p);
};

// Device buffer owned through the context allocator; move-only.
class Buf {
  public:
    Buf() = default;
    Buf(const Buf&) = delete;
    Buf& operator=(const Buf&) = delete;
    Buf(Buf&& o) noexcept { swap(o); }
    Buf& operator=(Buf&& o) noexcept { release(); swap(o); return *this; }
    ~Buf() { release(); }
    void ensure(Allocator* al, size_t bytes);     // grows (contents not kept)
    void release();
    template <typename T> T* as() const { return static_cast<T*>(p_); }
    size_t bytes() const { return bytes_; }
    void* get() const { return p_; }
  private:
    void swap(Buf& o) noexcept { std::swap(p_, o.p_); std::swap(bytes_, o.bytes_); std::swap(al_, o.al_); }
    void* p_ = nullptr;
    size_t bytes_ = 0;
    Allocator* al_ = nullptr;
};

// ---------------------------------------------------------------- logging --------
// Progress lines on stderr when the environment variable PDEP_VERBOSE is set (long
// solves report each refinement step / eigensolver iteration).
bool verbose();

// ---------------------------------------------------------------- profiling ------
// Kernel classes timed by the opt-in profiler (prof.hip; see pdep_profile_enable).
enum KernelId : int {
    K_SPHERE_TO_STICKS = 0, K_SLAB_HV, K_STICKS_TO_SPHERE, K_SLAB_INV_STORE, K_SLAB_FWD_PRODUCT,
    K_SLAB_DENSITY, K_GEMM_AHB, K_GEMM_UPDATE, K_ROW_DOTS, K_CG_UPDATE, K_MISC, K_SLAB_HV64,
    K_SPHERE_TO_STICKS64, K_STICKS_TO_SPHERE64, K_GEMM_AHB64, K_GEMM_UPDATE64, K_COUNT
};
// Records HIP events around the launch made during its lifetime (when profiling is on),
// with the launch's algorithmic HBM bytes and flops.
class ProfScope {
  public:
    ProfScope(int kid, hipStream_t s, double bytes = 0.0, double flops = 0.0);
    ~ProfScope();
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;
  private:
    int kid_;
    hipStream_t s_;
    double bytes_, flops_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
    bool active_ = false;
};

// True while launches of this thread are being timed (pdep_profile_enable).
bool profiling_on();
// While one exists on a thread, the launches of that thread are not timed (the
// no-allocation entry point creates no events).
struct ProfSuspend {
    ProfSuspend();
    ~ProfSuspend();
    ProfSuspend(const ProfSuspend&) = delete;
    ProfSuspend& operator=(const ProfSuspend&) = delete;
};

// ---------------------------------------------------------------- FFT geometry ---
// Radix plan of one axis: n = prod(rad[0..nst)), radices in {2,3,4,8}.
struct AxisPlan {
    int n = 0;
    int nst = 0;
    int rad[8] = {0};
};

// Everything a transform kernel needs to know about the grid and the sphere, passed
// by value.  The sphere is a union of ns z-sticks (one per (mx, my) that has a G in S),
// each a contiguous run of the lexicographic sphere order.  The x columns that can be
// non-empty in a z slab are mx = -mxmax..mxmax (ax of them).
struct FftDims {
    int nx, ny, nz;
    int ax, mxmax;
    int mymax;                // largest |my| of the sphere's sticks
    int npw;
    int ns;                   // number of sticks
    int sld;                  // stick leading dimension of the sticks buffer (>= ns)
    int sg_max;               // most sphere entries in one group of kRegStickGroup sticks
    int sgp_max;              // most sphere entries in one group of kPairStickGroup front sticks
    AxisPlan px, py, pz;
};

// Sticks per workgroup of the register stick passes.
constexpr int kRegStickGroup = 128;
// Front sticks per workgroup of the register paired sticks-to-sphere pass (each with its mirror).
constexpr int kPairStickGroup = 64;

// Device tables of the sphere / grid (one set per context).
struct BasisTables {
    const int* stick_start;   // [ns + 1] first sphere index of each stick
    const int* stick_pos;     // [npw]    stick * nz + (mz mod nz)
    const int* slab_pos;      // [ns]     (mx mod nx) * ny + (my mod ny)
    const int* col_start;     // [ax + 1] first stick of each non-empty x column c = mx + mxmax
    const int* col_my0;       // [ax]     my of that stick (the column spans my0 .. -my0)
    const double* twx64; const double* twy64; const double* twz64;  // n complex each: exp(-2 pi i m / n)
    const float* twx32; const float* twy32; const float* twz32;
};

// ------------------------------------------------------------- launchers (fft.hip)
// Buffers: "sticks" rows of nz * sld complex ([row][iz][stick]); real-space grids are
// z-major ([row][iz][ix][iy]).
// sphere rows (stride ld_in) -> sticks (inverse z transforms); gscale (per G, may be
// null) multiplies the coefficients on the way in.
template <typename T>
void launch_sphere_to_sticks(const FftDims& d, const BasisTables& t, const cplx<T>* in, long ld_in, int nrows,
                             const double* gscale, cplx<T>* sticks, hipStream_t s);
enum SphereEpilogue : int {
    EPI_SCALE = 0,            // out = alpha * F
    EPI_SHIFTED_H = 1,        // out = F + (kin - shift[row % nshift]) * x
    EPI_GSCALE = 2,           // out = F * gscale
};
// sticks -> sphere rows (forward z transforms, 1/N_g) with an epilogue.  With
// EPI_SHIFTED_H and dot_part non-null, each workgroup also writes Re<x, out> over its
// part of the row (FP64 sum) to dot_part[row * G + group], G = sticks_to_sphere_groups.
template <typename T>
void launch_sticks_to_sphere(const FftDims& d, const BasisTables& t, const cplx<T>* sticks, int nrows, cplx<T>* out,
                             long ld_out, int epi, double alpha, const cplx<T>* x, long ld_x, const T* kin,
                             const double* shift, int nshift, const double* gscale, hipStream_t s,
                             double* dot_part = nullptr);
// number of partial dot products per row that launch_sticks_to_sphere<T> writes
template <typename T> int sticks_to_sphere_groups(const FftDims& d);
// Paired half-sphere rows (rows real in r, entries k <= c = (npw - 1) / 2 of the sphere
// order, the rest implied by c_{npw-1-k} = conj c_k): two rows share one packed sticks
// row (the transform of a + i b).  The rows form groups of `group` consecutive rows (0:
// one group) and pairs stay inside a group: packed row g * ceil(group / 2) + j holds
// rows g * group + 2j and g * group + 2j + 1 (absent past the group or nrows).
int pair_count(int nrows, int group);
template <typename T>
void launch_sphere_to_sticks_pair(const FftDims& d, const BasisTables& t, const cplx<T>* in, long ld_in, int nrows,
                                  cplx<T>* sticks, hipStream_t s, int group = 0);
// packed sticks -> half-sphere rows with EPI_SHIFTED_H (dot_part may be null: Re<x, out>
// of the full vectors, sticks_to_sphere_pair_groups partials per row) or EPI_SCALE
template <typename T>
void launch_sticks_to_sphere_pair(const FftDims& d, const BasisTables& t, const cplx<T>* sticks, int nrows,
                                  cplx<T>* out, long ld_out, int epi, double alpha, const cplx<T>* x, long ld_x,
                                  const T* kin, const double* shift, int nshift, hipStream_t s, double* dot_part,
                                  int group = 0);
template <typename T> int sticks_to_sphere_pair_groups(const FftDims& d);
// sticks -> inverse (y, x) -> * V(z, x, y) (z-major real grid) -> forward -> sticks, in place.
template <typename T>
void launch_slab_hv(const FftDims& d, const BasisTables& t, cplx<T>* sticks, int nrows, const T* Vz, hipStream_t s);
// sticks -> inverse (y, x) -> complex grid (grid_c) or its real part (grid_r).
template <typename T>
void launch_slab_inv_store(const FftDims& d, const BasisTables& t, cplx<T>* sticks, int nrows, cplx<T>* grid_c,
                           T* grid_r, hipStream_t s);
// grids -> forward (x, y) -> sticks: f = Vr[row / nv] * u[row % nv], or f = Vr[row] (real) when u is null.
template <typename T>
void launch_slab_fwd_product(const FftDims& d, const BasisTables& t, const T* Vr, const cplx<T>* u, int nv, int nrows,
                             cplx<T>* sticks, hipStream_t s);
// dn_i = scale * Re sum_v conj(u_v) Inv(sticks[i * nv + v]), z-major real grids.
void launch_slab_density(const FftDims& d, const BasisTables& t, const double2* sticks, int npert, int nv,
                         const double2* u, double scale, double* dn, hipStream_t s);
// C-order [ix][iy][iz] <-> z-major [iz][ix][iy] for nrows real grids.
void launch_transpose_grid(int nx, int ny, int nz, int nrows, const double* in, double* out, bool to_zmajor,
                           hipStream_t s);

// --------------------------------------------------------- launchers (linalg.hip)
// S[n][m] = sum_k conj(A[m][k]) * B[n][k]   (complex, matrix cores; A: M x K, B: N x K,
// S: N x M, leading dimensions in complex elements).  work (work_elems complex, may be
// null) holds split-K partial products when the output alone is too small to fill the
// GPU; the partials are summed in a fixed order.
// real_out: S gets only the real parts (imaginary parts stored as zero).
template <typename T>
void launch_gemm_ahb(int M, int N, int K, const cplx<T>* A, long lda, const cplx<T>* B, long ldb, cplx<T>* S,
                     long lds, cplx<T>* work, size_t work_elems, hipStream_t s, bool real_out = false);
// Y[n][k] = beta*Y + alpha * sum_m A[m][k] * S[n][m]   (S: N x M; Y must not alias A or S);
// real_s: the imaginary parts of S are zero (and not read)
// Y -= S A for FP64 half-sphere rows with real coefficients (the imaginary parts of the
// complex coefficient buffer S are ignored): N rows of K complex entries (2 K reals), A:
// M rows (stride lda complex), S: N rows of M (stride lds complex), on the FP64 matrix
// cores.  sr: work space of sr_elems doubles for the contiguous real coefficients (rows
// are processed in blocks that fit it).
void launch_dgemm_sub(int M, int N, int K, const double2* A, long lda, const double2* S, long lds, double2* Y,
                      long ldy, double* sr, size_t sr_elems, hipStream_t s);
template <typename T>
void launch_gemm_update(int M, int N, int K, const cplx<T>* A, long lda, const cplx<T>* S, long lds,
                        double alpha, double beta, cplx<T>* Y, long ldy, hipStream_t s, bool real_s = false);
// BF16x3 variants of the two GEMMs above for FP32 operands (16 significant bits per
// product; for the inner solve of the refinement only).  lda/ldb/lds multiples of 4.
void launch_gemm_ahb_x3(int M, int N, int K, const float2* A, long lda, const float2* B, long ldb, float2* S,
                        long lds, float2* work, size_t work_elems, hipStream_t s, bool real_out = false);
void launch_gemm_update_x3(int M, int N, int K, const float2* A, long lda, const float2* S, long lds, double alpha,
                           double beta, float2* Y, long ldy, hipStream_t s);
// Launch shape of the BF16x3 coefficient GEMMs (0 = the built-in rule): split K until
// about splitk_target workgroups; col_tiles 4 or 8 column tiles per wave (plain GEMM with
// more than 96 coefficient rows only).
struct GemmShape {
    int splitk_target = 0;
    int col_tiles = 0;
};
// Real-coefficient BF16x3 pair (S real, float [N][lds], lds multiple of 4):
//   S[n][m] = Re sum_k conj(A[m][k]) B[n][k];   Y[n][k] = beta Y + alpha sum_m S[n][m] A[m][k]
// kin non-null: B[n][k] is taken times the CG preconditioner 1 / max(kin[k] - shift[n], kfloor)
void launch_gemm_ahb_x3_real(int M, int N, int K, const float2* A, long lda, const float2* B, long ldb, float* S,
                             long lds, float* work, size_t work_elems, hipStream_t s, const float* kin = nullptr,
                             const double* shift = nullptr, double kfloor = 0.0, GemmShape shape = {});
void launch_gemm_update_x3_real(int M, int N, int K, const float2* A, long lda, const float* S, long lds,
                                double alpha, double beta, float2* Y, long ldy, hipStream_t s);
// The residual update of a preconditioned CG step, for the rows of launch_gemm_ahb_x3_step.
struct CgStepFuse {
    const float2* q = nullptr;     // q = (H - shift) p of this iteration, stride as r
    const double* rz = nullptr;    // <r, K r> before the step
    const double* pq = nullptr;    // partial sums of <p, q>, npq per row
    int npq = 0;
    const int* active = nullptr;   // rows not active are left unchanged
    float* alpha_out = nullptr;    // alpha = <r, K r> / <p, q> of the active rows
    double* rz_part = nullptr;     // [row][part] partial sums of the new <r, K r> ...
    double* rr_part = nullptr;     // ... and of the new ||r||^2 (half-sphere weights)
    double* rz_new = nullptr;      // the sums: new <r, K r> ...
    double* rr = nullptr;          // ... new ||r||^2 ...
    float* beta = nullptr;         // ... and beta = new <r, K r> / rz (active rows)
    int* count = nullptr;          // set to zero (the active-row counter of this iteration)
};
// launch_gemm_ahb_x3_real (with the preconditioner) on r after the step: for the active
// rows r <- r - alpha q, written back in place, and <r, K r>, ||r||^2 of the new r and
// the CG factor beta (M <= 128).  Returns the number of partial sums per row
// (<= max_parts).
int launch_gemm_ahb_x3_step(int M, int N, int K, const float2* A, long lda, float2* r, long ldr, float* S, long lds,
                            float* work, size_t work_elems, hipStream_t s, const float* kin, const double* shift,
                            double kfloor, const CgStepFuse& cs, int max_parts, GemmShape shape = {});
// CG direction update with the projected preconditioned residual formed in the GEMM:
// for active rows n, x[xrow[n]] += alpha[n] p[n] (the old p; xrow null: row n) and
// p[n] <- K r[n] - sum_m S[n][m] A[m] + beta[n] p[n], where S = Re(A^H K r) comes from
// launch_gemm_ahb_x3_real with the same kin / shift / kfloor; x and p share the stride.
void launch_cg_direction_x3(int M, int N, int K, const float2* A, long lda, const float* S, long lds, const float2* r,
                            long ldr, const float* kin, const double* shift, double kfloor, const float* beta,
                            const float* alpha, float2* x, const int* xrow, const int* active, float2* p, long ldp,
                            hipStream_t s);
// floor of the CG preconditioner 1 / max(1/2|G|^2 - e_v, floor) (Hartree)
constexpr double kPrecondFloor = 0.1;
// S[n][m] = sum_z P[z][n][m], z = 0, 1, ... in order (split-K partial products)
void launch_splitk_reduce_f32(int M, int N, long lds, int splits, const float2* P, float2* S, hipStream_t s,
                              bool real_out = false);
// per-row dot products: out[r] = Re <a_r, b_r>, out2[r] = ||a_r||^2 (out2 may be null).
// half: the rows are half spheres of Hermitian-symmetric vectors (entries k <= c of the
// sphere order, the centre G = 0 last) and the products are those of the full vectors.
template <typename T>
void launch_row_dots(int nrows, int K, const cplx<T>* a, long lda, const cplx<T>* b, long ldb,
                     double* out, double* out2, hipStream_t s, bool half = false);
// Batched preconditioned CG, element-wise parts (the algorithm is in solver.hip).
template <typename T>
void launch_cg_init(int nrows, int K, const cplx<T>* b, long ld, cplx<T>* x, cplx<T>* r, cplx<T>* z,
                    const T* kin, const double* shift, int nshift, int precond, hipStream_t s);
// pq: npq partial sums of <p, q> per row (row-major), added in order.  With rz_part
// non-null (work space of nrows * ceil(K / 256) doubles each, as rr_part), the step also
// forms <r, K r> and ||r||^2 of the updated r and writes their row sums to rz_new, rr
// (active rows only): for r in range(P_c), <r, P_c K r> = <r, K r>.
template <typename T>
void launch_cg_step1(int nrows, int K, cplx<T>* x, cplx<T>* r, cplx<T>* z, const cplx<T>* p,
                     const cplx<T>* q, long ld, const double* rz, const double* pq, int npq, const int* active,
                     const T* kin, const double* shift, int nshift, int precond, hipStream_t s,
                     double* rz_part = nullptr, double* rr_part = nullptr, double* rz_new = nullptr,
                     double* rr = nullptr, bool half = false, float* beta = nullptr, float* alpha_out = nullptr);
template <typename T>
void launch_cg_step2(int nrows, int K, cplx<T>* p, const cplx<T>* z, long ld, const double* rz_new,
                     double* rz, const int* active, hipStream_t s);
// active[r] &= rr[r] > thr2[r]; iters[r] += count_iter for rows active on entry; rz <- rz_new;
// n_active += number of rows still active.  rr_max > 0: a row whose rr exceeds it (or is
// not a number) stops as diverged, its iteration count stored as -(count) - 1.
void launch_cg_check(int nrows, const double* rr, const double* thr2, int* active, int* iters,
                     double* rz, const double* rz_new, int* n_active, int count_iter, hipStream_t s,
                     double rr_max = 0.0);
// out[r] = rowscale[r] * in[rows[r]] with precision conversion (rows, rowscale may be null)
template <typename Tin, typename Tout>
void launch_convert_rows(int nrows, int K, const cplx<Tin>* in, long ldi, const int* rows,
                         const double* rowscale, cplx<Tout>* out, long ldo, hipStream_t s);
// x[rows[r]] += rowscale[r] * d[r] (rows with rowscale 0 are left untouched); with set,
// x[rows[r]] = rowscale[r] * d[r] instead, zeros for rowscale 0 and in the padding
// entries K .. ldx - 1 (the state of a zero-filled x after the update)
template <typename T>
void launch_axpy_rows(int nrows, int K, const cplx<T>* d, long ldd, const int* rows,
                      const double* rowscale, double2* x, long ldx, hipStream_t s, bool set = false);
// out[r][k] = 2 in[r][k] for k < K - 1, in[r][K - 1] at k = K - 1 (half-sphere weights)
template <typename T>
void launch_half_weights(int nrows, int K, const cplx<T>* in, long ldi, cplx<T>* out, long ldo, hipStream_t s);
// res[rows[r]] = b[rows[r]] - q[r] and out[r] = ||res[rows[r]]||^2 (half-sphere weights when half)
void launch_residual_rows(int nrows, int K, const double2* b, long ldb, const int* rows, const double2* q, long ldq,
                          double2* res, long ldr, double* out, bool half, hipStream_t s);
// rows <- their Hermitian-symmetric part (c_{-G} = conj c_G; -G_k sits at npw - 1 - k)
void launch_sym_fix(int nrows, int npw, double2* x, long ld, hipStream_t s);
void launch_fill_zero(void* p, size_t bytes, hipStream_t s);
void launch_fill_i32(int* p, int n, int value, hipStream_t s);
// S' <-> S: expand inserts a zero at G = 0 (index g0); compact drops it.  Rows of length
// npw - 1 (ld_in) and npw (ld_out), or the reverse.
void launch_expand_s1(int nrows, int npw, int g0, const double2* in, long ldi, double2* out, long ldo,
                      hipStream_t s);
void launch_compact_s1(int nrows, int npw, int g0, const double2* in, long ldi, double2* out, long ldo,
                       hipStream_t s);

// ------------------------------------------------------------------ context ------
struct Basis {
    double L[3];
    int n[3];
    double ecut;
    double omega;
    int ng;
    int npw;
    int g0;                               // index of G = 0 in S
    int ax, mxmax;
    std::vector<int32_t> miller;          // 3 * npw
    std::vector<int> stick_start, stick_pos, slab_pos, col_start, col_my0;
    std::vector<double> kin, coul;        // coul[g0] = 0
    FftDims dims{};
    Buf d_stick_start, d_stick_pos, d_slab_pos, d_cols, d_kin64, d_kin32, d_coul, d_tw64, d_tw32;
    BasisTables tables{};
};

void build_basis(const pdep_cell& cell, Basis& b);
void upload_basis(Basis& b, Allocator* al, hipStream_t s);
AxisPlan make_axis_plan(int n);

// Context work-space slots (Ctx::ws): solver.hip owns [0, WS_SOLVER_END); the others
// stay alive across solver calls and must not overlap it.
enum WsSlot : int {
    WS_SOLVER_END = 28,
    WS_CAPI_IN = 28, WS_CAPI_OUT = 29, WS_CAPI_STAGE = 30,
    WS_SETUP_STICKS = 31, WS_DAV_THETA = 32, WS_DAV_C = 33, WS_DAV_DOTS = 34,
    WS_SCR_Y = 35,            // screening.hip: 35 .. 41
    WS_LZ_W = 42,             // lanczos.hip: 42 .. 56
    WS_GW = 57,               // gw.hip: 57 .. 61
    WS_COUNT = 62
};

// Work space carved from a fixed device region instead of the allocator (the
// no-allocation entry point): each work-space slot keeps its region while requests fit
// it and otherwise takes a new one behind the last; exhausting the region throws
// PDEP_ENOMEM.  Contents are not kept when a slot moves (as with Buf::ensure).
struct Arena {
    char* base = nullptr;
    size_t cap = 0, used = 0;
    char* p[WS_COUNT] = {};
    size_t n[WS_COUNT] = {};
    void reset() {
        used = 0;
        for (int i = 0; i < WS_COUNT; ++i) { p[i] = nullptr; n[i] = 0; }
    }
    void* get(int i, size_t bytes) {
        if (p[i] && n[i] >= bytes) return p[i];
        const size_t off = (used + 255) / 256 * 256;
        if (off > cap || bytes > cap - off)
            throw Error(PDEP_ENOMEM, "no-allocation scratch of " + std::to_string(cap >> 20) +
                                         " MiB exhausted (work-space slot " + std::to_string(i) + " needs " +
                                         std::to_string(bytes) + " bytes, " + std::to_string(cap - std::min(off, cap)) +
                                         " left)");
        p[i] = base + off;
        n[i] = bytes;
        used = off + bytes;
        return p[i];
    }
};

struct Ctx {
    Ctx() = default;
    Ctx(const Ctx&) = delete;
    Ctx& operator=(const Ctx&) = delete;
    ~Ctx();
    pdep_opts opts{};
    Allocator al;
    hipStream_t stream = nullptr;
    int device = 0;
    Basis basis;
    int nv = 0;
    std::vector<double> eps;              // [nv]
    double gap = 0.0;
    int gs_iterations = 0;
    double gs_residual = 0.0;
    Buf vloc64, vloc32;                   // [ng] z-major
    Buf psi64, psi32;                     // [nv][npw] complex FP64; [nv][sphere_ld(npw)] FP32
    Buf psi32w, psi64w;                   // psi32 / psi64 with the half-sphere weights (2 off the centre)
    Buf upair;                            // [ceil(nv/2)][ng] complex grids u_2j + i u_2j+1, z-major
    Buf eps_dev;                          // [nv] double
    Buf kin32;                            // float kinetic
    // solver work space (grown on demand)
    void* blas = nullptr;                 // rocblas_handle for rocSOLVER calls
    bool own_blas = false;
    Buf blas_ws;                          // rocSOLVER work space, from the context allocator
    // the inner FP32 solves of the mixed mode use the BF16x3 projection products (set per
    // refinement step: rows that diverge with them are solved again with FP32 products)
    bool pc_x3 = false;
    Buf w[WS_COUNT];
    // set for the duration of a no-allocation call: work space comes from it, the
    // projection update avoids library GEMMs, and the chain block is not timed
    Arena* arena = nullptr;
    // complex elements of the split-K partial-product buffers of the projection GEMMs
    size_t split_elems = (size_t)8 << 20;
    void* ws(int i, size_t bytes) {
        if (arena) return arena->get(i, bytes);
        w[i].ensure(&al, bytes);
        return w[i].get();
    }
    // the current region of work-space slot i (as last returned by ws)
    void* ws_current(int i) const { return arena ? static_cast<void*>(arena->p[i]) : w[i].get(); }
    // rows per launch of the transform chain for FP32 / FP64 rows (0: not tuned yet)
    int fft_chunk32 = 0, fft_chunk64 = 0;
    // launch shapes of the BF16x3 coefficient GEMMs: the fused CG step and the plain one
    // (splitk_target 0: not tuned yet)
    GemmShape step_shape, ahb_shape;
    bool capturing = false;               // a HIP graph is being captured (no tuning runs)
    // PDEP_CG_GRAPHS: the stream the inner CG is captured on, and the event that orders it
    hipStream_t graph_stream = nullptr;
    hipEvent_t graph_event = nullptr;
};

// solver.hip
// Tuned launch parameters shared across processes: with PDEP_TUNE_CACHE=<file> set, the
// values tuned for a problem (grid, N_pw, N_v, precision) are read at set-up and written
// back (one JSON object per problem) when a tuning run picks new ones.
void tune_cache_load(Ctx& c);
void tune_cache_store(const Ctx& c);
// Leading dimension (elements) of stored sphere vectors.
long sphere_ld(int npw);
// bytes of the projection coefficients of nrows rows (either precision), coef_ld(nv) per row
size_t coef_bytes(int nv, int nrows);
long coef_ld(int nv);
// entries of a half-sphere row (k <= (npw - 1) / 2, the centre G = 0 last)
int half_len(int npw);
template <typename T> void project_c(Ctx& c, cplx<T>* Y, long ld, int nrows, double2* S);
struct ApplyStats {
    int n_rhs = 0, cg_iter_max = 0, refine_steps = 0, n_notconv = 0;
    int n_fp32_fallback = 0;              // BF16x3 mode: systems re-solved with FP32 projection products
    long long graph_captures = 0, graph_launches = 0;   // PDEP_CG_GRAPHS: CG blocks captured / replayed
    long long graph_updates = 0;          // captures that updated an executable graph in place
    long long cg_iter_total = 0, op_applications = 0;
    double max_rel_residual = 0.0;
};
// Apply H (shift per row) to `nrows` FP64 sphere vectors: out = (H - shift) x.
void apply_h64(Ctx& c, const double2* x, long ldx, int nrows, const double* shift, int nshift,
               double2* out, long ldo, double2* sticks_buf);
void solve_rows(Ctx& c, int n, const double2* b64, double2* x64, long ld, ApplyStats& st, const double* ref2);
// chi0 on real z-major grid potentials (device): dv [npert][ng] -> dn [npert][ng] (FP64)
void chi0_grid(Ctx& c, int npert, const double* dv, double* dn, ApplyStats& st);
// chi0bar on S (device, FP64, G0 entry ignored/zero): phi [npert][npw] -> out [npert][npw]
void chi0bar_sphere(Ctx& c, int npert, const double2* phi, double2* out, ApplyStats& st);
// W [npert * N_v half-sphere FP64 rows, stride ld, row = i * N_v + v] <- P_c Fwd(V_i u_v)
// with V_i = Re Inv(sqrt(4 pi)/|G| phi_i) (the Sternheimer right-hand sides up to sign);
// phi: npert rows on S (stride sphere_ld(npw), G = 0 entry zero)
void rhs_half_rows(Ctx& c, int npert, const double2* phi, double2* W, long ld);
// The projection coefficients <c_m| Fwd(V_i u_v)> of the last rhs_half_rows call (device,
// row i * nv + v, coef_ld(nv) complex entries per row with zero imaginary parts), valid
// until the next projection through the solver's coefficient buffer.
const double2* rhs_coefficients(Ctx& c);
// z = P_c H P_c q on FP64 half-sphere rows (zero_shift: one device double 0.0)
void apply_deflated_h64(Ctx& c, const double2* q, double2* z, long ld, int nrows, const double* zero_shift);
// upper bound of the device work space chi0bar_sphere takes for npert perturbations in
// one tile (opts.rhs_tile >= npert * N_v)
size_t chi0_work_bytes(const Ctx& c, int npert);

// capi.hip: pdep_setup with an optional caller-owned rocblas_handle (server workers)
int setup_context(const pdep_cell* cell, const double* vloc, const pdep_opts* opts, const double* psi_in,
                  const double* eps_in, void* blas, pdep_ctx** out);
// bytes a job needs on the device (setup + Davidson + one chi0 tile); chi0_budget
// receives the part reserved for the chi0 work space (the job's opts.hbm_budget)
size_t job_hbm_estimate(const pdep_cell& cell, const pdep_opts& o, int n_pdep, const pdep_eig_opts& eo,
                        size_t* chi0_budget);

// screening.hip: chibar = (1 - chi0bar)^-1 chi0bar on n potentials on S (device, FP64,
// rows of stride sphere_ld(npw), G = 0 entry zero), self-consistent to tol ||phi||
struct ScreenResult {
    int passes = 0;               // chi0bar applications to the block (self-consistency passes)
    long long chi0_columns = 0;   // chi0bar columns computed
    int n_notconv = 0;            // columns that missed tol within maxit passes
    double max_rel_residual = 0.0;
};
ScreenResult chibar_sphere(Ctx& c, int n, const double2* phi, double2* out, double tol, int maxit,
                           ApplyStats& st);

// lanczos.hip: deflated Lanczos chains of P_c H P_c (Sec. 2.4) from the start vectors
// w_jv = P_c Fwd(V_j u_v) of the basis potentials phi (npert rows on S, device) and,
// with ndir = 3, the dipole vectors xi^a_v of Eq. commu scaled by sqrt(4 pi) (rows
// npert .. npert + 2).  Row r = j * nv + v; chains advance together as one block.
struct Chains {
    int npert = 0, nv = 0, nl = 0, nrow = 0;   // npert counts the directions
    std::vector<double> alpha, beta;            // [nl][nrow]: T's diagonal, off-diagonal
    std::vector<int> len;                       // chain length (0: zero start vector)
    std::vector<double> wn;                     // ||w_r||
    const double2* O = nullptr;                 // device [nl][nv][j][i]: Re <w_iv|q_n of chain jv>
    long long h_applications = 0;
    int chains = 0, max_length = 0;
};
// coef (may be null) receives <c_m| Fwd(V_i u_v)> before P_c, [npert_in * nv][nv] (row
// i * nv + v, column m): the occupied-state pair coefficients.  Ch.O stays valid until
// the next call that uses the Lanczos work space.
void run_chains(Ctx& c, int npert_in, const double2* phi, int ndir, int nl, Chains& ch, ApplyStats* dir_st,
                std::vector<double>* coef);
// A frequency point: every transition of energy D enters as [1/(D - a) + 1/(D - b)] / 2.
// Imaginary frequency i u: a = i u, b = -i u (D / (D^2 + u^2)); real frequency w with
// broadening eta: a = -w + i eta, b = w + i eta.
struct FreqPoint {
    double2 a, b;
};
// The matrix of -(4/Omega) sum_v <w_iv| g(A_v) |w_jv> over all start vectors at nz
// points (g as above, A_v = P_c (H - e_v) P_c), host [nz][npert][npert] complex.
void chain_body(Ctx& c, const Chains& ch, int nz, const FreqPoint* z, double2* out);

struct LanczosResult {
    int chains = 0, max_length = 0;
    long long h_applications = 0;
};
// The body of chi0bar at imaginary frequencies u (host array) in the basis phi, body
// (host) [nfreq][npert][npert].  With ndir = 3 the directions join (after the npert
// potentials): body is then [nfreq][npert + 3][npert + 3] with the head F in the last
// 3 x 3 block and the wings in the last rows / columns; dir_st (may be null) receives
// the statistics of their Sternheimer solves.
LanczosResult body_lanczos(Ctx& c, int npert, const double2* phi, int ndir, int n_lanczos, int nfreq,
                           const double* u, double* body, ApplyStats* dir_st = nullptr);

// Gauss-Legendre nodes and weights of order n on [-1, 1].
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
// The integral of 4 pi / q^2 over the Brillouin zone of a Gamma-only orthorhombic cell,
// |q_a| <= pi / L_a, divided by (2 pi)^3.
double bz_coulomb_integral(const double L[3]);
// Eq. Bfinal at one frequency from the extended matrix E [(np + 3) x (np + 3)] of
// body_lanczos with the three directions: F (3 x 3), U (U_aj, 3 x np), B (np x np),
// Lambda (np x np) and Xi (a scalar), each output may be null.
void bfinal(int np, const double* E, const double L[3], double* F, double* U, double* B, double* Lam, double* Xi);
// The same at a real frequency, where E is complex symmetric.
void bfinal_complex(int np, const double2* E, const double L[3], double2* Lam, double2* Xi);

// gw.hip: G0W0 quasiparticle energies of occupied states (pdep_qp_energies)
struct QpStats {
    int chains = 0, max_length = 0, secant_iterations = 0, residue_points = 0;
    long long h_applications = 0;
};
QpStats qp_energies(Ctx& c, int np, const double2* phi, int nst, const int* states, const double* vxc,
                    const pdep_qp_opts& o, pdep_qp_result* out, int ne, const double* energies, double* sig_e,
                    ApplyStats* dir_st);

// davidson.hip
void ground_state(Ctx& c);
// orbitals -> Hermitian-symmetric (real in r) Ritz vectors of the same subspace
void realify_orbitals(Ctx& c);
struct EigResult {
    int iterations = 0, columns = 0;
    int n_notconv = 0;                    // Sternheimer systems that missed cg_tol (all chi0 applications)
    int scr_passes = 0, scr_notconv = 0;  // reducible: self-consistency passes, columns that missed scr_tol
    double max_residual = 0.0;
    long long cg_iter_total = 0;
    bool converged = false;
};
// Columns of the PDEP Davidson search space: max_subspace (default 4 n_pdep), but never
// fewer than twice the block (n_pdep + n_buffer), which a restart needs, nor more than
// N_pw - 1.
inline int pdep_subspace_max(int npw, int npdep, const pdep_eig_opts& eo) {
    const int nb = std::min(npw - 1, npdep + std::max(0, eo.n_buffer));
    const int want = eo.max_subspace > 0 ? eo.max_subspace : 4 * npdep;
    return std::min(npw - 1, std::max(want, 2 * nb));
}
EigResult pdep_davidson(Ctx& c, int npdep, uint64_t seed, const double2* phi0_dev, const pdep_eig_opts& eo,
                        double* lam_out, double2* basis_out_dev);

}  // namespace pdep
