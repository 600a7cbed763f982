// Internal declarations of the PDEP chi0 library: device types, basis tables,
// kernel launchers and the context.  Not part of the public ABI (include/pdep.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pdep.h"

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
    K_SPHERE_TO_PLANES = 0, K_PENCIL_HV, K_PLANES_TO_SPHERE, K_PENCIL_INV_STORE, K_PENCIL_FWD_PRODUCT,
    K_PENCIL_DENSITY, K_GEMM_AHB, K_GEMM_UPDATE, K_ROW_DOTS, K_CG_UPDATE, K_MISC, K_COUNT
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

// ---------------------------------------------------------------- FFT geometry ---
// Radix plan of one axis: n = prod(rad[0..nst)), radices in {2,3,4,8}.
struct AxisPlan {
    int n = 0;
    int nst = 0;
    int rad[8] = {0};
};

// Everything a transform kernel needs to know about the grid and the sphere, passed
// by value.  The sphere is stored plane by plane: plane a (0 <= a < ax) holds the G
// with mx = a - mxmax, at offsets [plane_start[a], plane_start[a+1]); within a plane
// the G with my = -k..k (k = stick_k[a]) form the z-sticks that can be non-zero.
struct FftDims {
    int nx, ny, nz;
    int ax, mxmax;
    int npw;
    int zc;                   // z chunk of the x-pencil kernels (divides nz)
    AxisPlan px, py, pz;
};

// Device tables of the sphere / grid (one set per context).
struct BasisTables {
    const int* plane_start;   // [ax + 1]
    const int* stick_k;       // [ax]
    const int* lds_idx;       // [npw]  iy*nz + iz inside a plane
    const double* twx64; const double* twy64; const double* twz64;  // n complex each: exp(-2 pi i m / n)
    const float* twx32; const float* twy32; const float* twz32;
};

// ------------------------------------------------------------- launchers (fft.hip)
// sphere vectors -> planes (inverse z then y transforms); rows of `in` have stride ld_in;
// rows selected through rows[] when non-null.  gscale (per G, may be null) multiplies
// the coefficients while scattering.
template <typename T>
void launch_sphere_to_planes(const FftDims& d, const BasisTables& t, const cplx<T>* in, long ld_in,
                             const int* rows, int nrows, const double* gscale, cplx<T>* planes,
                             hipStream_t s);
// planes -> x pencils: inverse x-FFT, * V, forward x-FFT (in place in planes).
template <typename T>
void launch_pencil_hv(const FftDims& d, const BasisTables& t, cplx<T>* planes, int nrows,
                      const T* V, long v_stride, const int* vsel, hipStream_t s);
// planes -> full complex grid (inverse x-FFT), optional real part only.
template <typename T>
void launch_pencil_inv_store(const FftDims& d, const BasisTables& t, const cplx<T>* planes, int nrows,
                             cplx<T>* grid_c, T* grid_r, hipStream_t s);
// full grids -> planes: f(r) = Vr(r) * u(r) (Vr row = row / nv, u row = row % nv), or, with u
// null, f(r) = Vr(r) (real data).  Forward x-FFT, active planes kept.
template <typename T>
void launch_pencil_fwd_product(const FftDims& d, const BasisTables& t, const T* Vr, const cplx<T>* u,
                               int nv, int nrows, cplx<T>* planes, hipStream_t s);
// density: for each perturbation i, dn_i(r) = scale * Re sum_v conj(u_v(r)) Inv-x(planes[i*nv+v]).
void launch_pencil_density(const FftDims& d, const BasisTables& t, const double2* planes, int npert,
                           int nv, const double2* u, double scale, double* dn, hipStream_t s);

enum SphereEpilogue : int {
    EPI_SCALE = 0,            // out = alpha * F
    EPI_SHIFTED_H = 1,        // out = F + (kin - shift[row % nshift]) * x
    EPI_GSCALE = 2,           // out = F * gscale
};
// planes -> sphere (forward y then z transforms, 1/N_g), with an epilogue.
template <typename T>
void launch_planes_to_sphere(const FftDims& d, const BasisTables& t, const cplx<T>* planes, int nrows,
                             const int* rows, cplx<T>* out, long ld_out, int epi, double alpha,
                             const cplx<T>* x, long ld_x, const T* kin, const double* shift, int nshift,
                             const double* gscale, hipStream_t s);

// --------------------------------------------------------- launchers (linalg.hip)
// S[n][m] = sum_k conj(A[m][k]) * B[brows[n]][k]   (complex; A: M x K, B rows of length K,
// S: N x M, leading dimensions in elements); brows may be null (identity).
template <typename T>
void launch_gemm_ahb(int M, int N, int K, const cplx<T>* A, long lda, const cplx<T>* B, long ldb,
                     const int* brows, double2* S, long lds, hipStream_t s);
// Y[yrows[n]][k] = beta*Y + alpha * sum_m A[m][k] * S[n][m]   (S double2, N x M)
template <typename T>
void launch_gemm_update(int M, int N, int K, const cplx<T>* A, long lda, const double2* S, long lds,
                        double alpha, double beta, cplx<T>* Y, long ldy, const int* yrows, hipStream_t s);
// per-row dot products: out[r] = Re <a_r, b_r>, out2[r] = ||a_r||^2 (out2 may be null)
template <typename T>
void launch_row_dots(int nrows, int K, const cplx<T>* a, long lda, const cplx<T>* b, long ldb,
                     double* out, double* out2, hipStream_t s);
// Batched preconditioned CG, element-wise parts (the algorithm is in solver.hip).
template <typename T>
void launch_cg_init(int nrows, int K, const cplx<T>* b, long ld, cplx<T>* x, cplx<T>* r, cplx<T>* z,
                    const T* kin, const double* shift, int nshift, int precond, hipStream_t s);
template <typename T>
void launch_cg_step1(int nrows, int K, cplx<T>* x, cplx<T>* r, cplx<T>* z, const cplx<T>* p,
                     const cplx<T>* q, long ld, const double* rz, const double* pq, const int* active,
                     const T* kin, const double* shift, int nshift, int precond, hipStream_t s);
template <typename T>
void launch_cg_step2(int nrows, int K, cplx<T>* p, const cplx<T>* z, long ld, const double* rz_new,
                     double* rz, const int* active, hipStream_t s);
// active[r] &= rr[r] > thr2[r]; iters[r] += count_iter for rows active on entry; rz <- rz_new;
// n_active += number of rows still active.
void launch_cg_check(int nrows, const double* rr, const double* thr2, int* active, int* iters,
                     double* rz, const double* rz_new, int* n_active, int count_iter, hipStream_t s);
// out[r] = rowscale[r] * in[rows[r]] with precision conversion (rows, rowscale may be null)
template <typename Tin, typename Tout>
void launch_convert_rows(int nrows, int K, const cplx<Tin>* in, long ldi, const int* rows,
                         const double* rowscale, cplx<Tout>* out, long ldo, hipStream_t s);
// x[rows[r]] += rowscale[r] * d[r]
template <typename T>
void launch_axpy_rows(int nrows, int K, const cplx<T>* d, long ldd, const int* rows,
                      const double* rowscale, double2* x, long ldx, hipStream_t s);
// out[r] = a[rows[r]] - b[r]
void launch_sub_rows(int nrows, int K, const double2* a, long lda, const int* rows, const double2* b,
                     long ldb, double2* out, long ldo, hipStream_t s);
// dst[rows[r]] = src[r]
void launch_scatter_rows(int nrows, int K, const double2* src, long lds, const int* rows, double2* dst,
                         long ldd, hipStream_t s);
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
    std::vector<int> plane_start, stick_k, lds_idx;
    std::vector<double> kin, coul;        // coul[g0] = 0
    FftDims dims{};
    Buf d_plane_start, d_stick_k, d_lds_idx, d_kin64, d_kin32, d_coul, d_tw64, d_tw32;
    BasisTables tables{};
};

void build_basis(const pdep_cell& cell, Basis& b);
void upload_basis(Basis& b, Allocator* al, hipStream_t s);
AxisPlan make_axis_plan(int n);

struct Ctx {
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
    Buf vloc64, vloc32;                   // [ng]
    Buf psi64, psi32;                     // [nv][npw] complex
    Buf u64;                              // [nv][ng] complex grids
    Buf eps_dev;                          // [nv] double
    Buf kin32;                            // float kinetic
    // solver work space (grown on demand)
    Buf w[24];
    void* ws(int i, size_t bytes) { w[i].ensure(&al, bytes); return w[i].get(); }
};

// solver.hip
// Leading dimension (elements) of stored sphere vectors.
long sphere_ld(int npw);
// Workspace slot used for the plane buffer of one-off transforms at setup.
constexpr int W_STAGE_PLANES = 20;
template <typename T> void project_c(Ctx& c, cplx<T>* Y, long ld, int nrows, double2* S);
struct ApplyStats {
    int n_rhs = 0, cg_iter_max = 0, refine_steps = 0, n_notconv = 0;
    long long cg_iter_total = 0, op_applications = 0;
    double max_rel_residual = 0.0;
};
// Apply H (shift per row) to `nrows` FP64 sphere vectors: out = (H - shift) x.
void apply_h64(Ctx& c, const double2* x, long ldx, int nrows, const double* shift, int nshift,
               double2* out, long ldo, double2* planes);
void solve_rows(Ctx& c, int n, const double2* b64, double2* x64, long ld, ApplyStats& st, const double* ref2);
// chi0 on real grid potentials (device): dv [npert][ng] -> dn [npert][ng] (FP64)
void chi0_grid(Ctx& c, int npert, const double* dv, double* dn, ApplyStats& st);
// chi0bar on S (device, FP64, G0 entry ignored/zero): phi [npert][npw] -> out [npert][npw]
void chi0bar_sphere(Ctx& c, int npert, const double2* phi, double2* out, ApplyStats& st);

// davidson.hip
void ground_state(Ctx& c);
struct EigResult {
    int iterations = 0, columns = 0;
    double max_residual = 0.0;
    long long cg_iter_total = 0;
    bool converged = false;
};
EigResult pdep_davidson(Ctx& c, int npdep, uint64_t seed, const double2* phi0_dev, const pdep_eig_opts& eo,
                        double* lam_out, double2* basis_out_dev);

}  // namespace pdep
