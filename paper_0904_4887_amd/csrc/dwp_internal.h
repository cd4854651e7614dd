// Internal declarations of libdwp: device buffers, multigrid levels, the
// context, and the host-side launchers of every kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dwp.h"

namespace dwp {

// ----------------------------------------------------------------------------
// Error handling: every HIP call is checked; a failure becomes a C++ exception
// inside the library and a dwp_status at the ABI boundary.
struct Error {
    int status;
    std::string msg;
};

[[noreturn]] void fail(int status, const std::string &msg);

#define DWP_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            ::dwp::fail(DWP_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define DWP_LAUNCH_CHECK() DWP_HIP(hipGetLastError())

// Device buffer owned by the context (RAII).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void alloc(size_t n_bytes);
    void release();
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// ----------------------------------------------------------------------------
// One level of the wet-slab hierarchy.  Arrays of the unknowns and of eps hold
// nw + 2 planes: plane 0 and plane nw + 1 are the Dirichlet planes next to the
// slab (zero for the correction, the neighbouring node eps for eps); plane
// p = k + 1 holds slab plane k.  x and y are periodic.
struct Level {
    int nx = 0, ny = 0, nw = 0;   // slab dimensions of this level
    double h[3] = {0, 0, 0};
    bool zc = false;              // coarsened in z from the previous level
    size_t plane = 0;             // nx * ny
    DevBuf eps;                   // (nw + 2) planes, T
    DevBuf u;                     // (nw + 2) planes, T, ghost planes zero
    DevBuf u2;                    // second copy for out-of-place sweeps
    DevBuf f;                     // nw planes, T
    DevBuf r;                     // nw planes, T (residual scratch)
    size_t n_interior() const { return plane * (size_t)nw; }
    size_t n_ghosted() const { return plane * (size_t)(nw + 2); }
};

struct Plan {
    int nx = 0, ny = 0, nz = 0;
    double L[3] = {0, 0, 0};
    double h[3] = {0, 0, 0};
    size_t N = 0;
    int nkx = 0;                  // nx / 2 + 1
    int ldc = 0;                  // row stride of the half spectrum: nkx rounded up to 8
    int k_w0 = 0, k_w1 = 0;       // wet planes [k_w0, k_w1) mod nz
    int nw = 0;                   // k_w1 - k_w0
    std::vector<Level *> levels;  // levels[0] is the fine slab
    size_t bottom = 0;            // first level handled by the single-workgroup kernel
};

// Radix plan of one FFT axis.
struct FFTAxis {
    int n = 0;
    std::vector<int> radices;     // product = n
    DevBuf tw;                    // n complex twiddles exp(-2 pi i t / n), double2
    DevBuf lam;                   // n (or nkx for x) discrete symbol values
    DevBuf tw32, lam32;           // the same in float32 (float32 dry-update variant)
};

// Kernel groups timed when profiling is on.
enum ProfGroup {
    PG_FFT_X = 0,      // x passes of the dry update (R2C / C2R of two rows at once)
    PG_FFT_Y,          // y passes
    PG_FFT_Z,          // z pass with the Green's-function multiply
    PG_RBGS_FINE,      // one colour pass of red-black Gauss-Seidel on the fine slab
    PG_RBGS_COARSE,    // colour passes on the coarser levels
    PG_MG_OTHER,       // residuals and transfers of the large levels
    PG_MG_BOTTOM,      // the single-workgroup bottom of the V-cycle
    PG_APPLY,          // full-box operator / residual
    PG_WET,            // wet-slab residual extraction and combination
    PG_MULTIDOT,       // Gram-Schmidt projections (V^T w, with ||w||^2)
    PG_AXPY,           // Gram-Schmidt updates w -= V h and x += Z y
    PG_VEC,            // other vector kernels (scaling, norms)
    PG_BUILD,          // eps and rho builders
    PG_FORCES,         // adjoint and forces
    PG_COUNT
};

struct Profiler {
    bool on = false;
    int only = -1;                // >= 0: time only this group
    double ms[PG_COUNT] = {0};
    double bytes[PG_COUNT] = {0};
    long launches[PG_COUNT] = {0};
    std::vector<hipEvent_t> pool;
    struct Pending {
        int group, ev;
        double bytes;
    };
    std::vector<Pending> pending;
    size_t next = 0;
    int begin(hipStream_t s, int group = -1);                 // -1 when off
    void end(hipStream_t s, int ev, int group, double bytes);
    // An event pair for a launch that records them itself at the kernel's
    // start and end (hipExtLaunchKernel): reserve, launch, then done.
    int reserve(int group);                                   // -1 when off
    hipEvent_t event(int ev, int k) const { return ev < 0 ? nullptr : pool[ev + k]; }
    void done(int ev, int group, double bytes);
    void collect();                                           // after a stream sync
    void reset();
    ~Profiler();
};

const char *prof_group_name(int g);

// Phase timers of a solve: an event is recorded on the stream where a phase
// begins; the time from one mark to the next is charged to the earlier mark's
// phase.
enum SolvePhase { PH_FFT = 0, PH_MG, PH_KRYLOV, PH_COUNT };

struct PhaseTimer {
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<int> phase;       // phase of each recorded mark
    size_t used = 0;
    void start();
    void mark(hipStream_t s, int ph);
    // after a stream sync: ms[PH_COUNT] from the recorded marks; stops
    void finish(double *ms);
    ~PhaseTimer();
};

}  // namespace dwp

struct dwp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    dwp_opts opts{};
    dwp::Plan plan;
    bool have_grid = false, have_eps = false, have_solution = false;
    int precision_built = -1;     // precision of the current level buffers

    // full-box float64 arrays
    dwp::DevBuf eps, sinv, S, b, r, w, phi_last, gbuf;
    dwp::DevBuf V, Z;             // Krylov bases, (restart + 1) N and restart N
    dwp::DevBuf V32;              // float32 Arnoldi basis, (restart + 1) N (opts.krylov_fp32)
    dwp::DevBuf eps32;            // eps rounded to float32, N (opts.krylov_fp32: the Krylov operator's copy)
    dwp::DevBuf G632;             // D1 eps rounded to float32, 3 N (krylov_fp32 with order 6)
    dwp::DevBuf cbuf;             // FFT workspace, nkx * ny * nz double2
    dwp::DevBuf Hz;               // per-plane height factor (exclusion)
    dwp::DevBuf partial;          // reduction partials
    dwp::DevBuf coef;             // small device vectors (Krylov coefficients)
    dwp::DevBuf atoms;            // packed atom data
    dwp::DevBuf fpart;            // force partials
    dwp::FFTAxis fx, fy, fz;
    double *host = nullptr;       // pinned host staging (small)
    size_t host_len = 0;
    dwp::Profiler prof;
    double mean_rho = 0.0;
    // atom bookkeeping of the last build_epsilon
    int eps_natoms = -1;
    bool eps_exclusion = false;
    std::vector<double> atom_rec;      // host copy of the last atom upload
    std::vector<double> eps_geometry;  // switch geometry of the last build_epsilon
    bool eps_density = false;          // eps built from a density grid; S holds d eps / d rho
    // sixth-order operator
    dwp::DevBuf G6;               // D1_d eps, 3N
    dwp::DevBuf lam, adj_rhs;     // adjoint solution and its right-hand side
    bool have_adjoint = false;
    bool transposed = false;      // the Krylov solve in progress is the adjoint one
    int fft_order = 0;            // order the FFT symbol tables were built for
    double background = 0.0;      // uniform background of the last order-6 solve
    double first_cycle_red = -1.0;  // residual reduction of the last solve's first cycle (< 0: none yet)
    dwp::PhaseTimer phases;       // phase timers of the solve in progress
    dwp::DevBuf bw_rhs, bw_lam;   // adjoint right-hand side and solution of dwp_backward
};

namespace dwp {

constexpr int RED_BLOCKS = 1024;      // blocks of every partial-sum kernel
constexpr int RED_THREADS = 256;

// ----------------------------------------------------------------------------
// Launchers (defined in the kernel translation units).

// kern_grid.hip: full-box stencils
void launch_apply_full(hipStream_t s, const Plan &p, const double *phi, const double *eps,
                       const double *b, double *out, bool residual);
void launch_eps_gradient(hipStream_t s, const Plan &p, const double *phi, double *g);
// out = V_eps = -(1/8 pi) G deps (Eq. 6; G as in the eps gradient), plus phi if add_phi (Eq. 5)
void launch_v_eps(hipStream_t s, const Plan &p, const double *phi, const double *deps, bool add_phi, double *out);
// eps and d eps/d rho from a density grid (Eqs. 7 and 8)
void launch_eps_density(hipStream_t s, const double *rho, double *eps, double *deps, size_t n, double eps_inf,
                        double rho0, double beta);
void launch_eps_pair(hipStream_t s, const Plan &p, const double *a, const double *b, double scale, double *g);
void launch_fill(hipStream_t s, double *x, double v, size_t n);
void launch_scale_dev(hipStream_t s, double *x, const double *num, const double *den_sq,
                      size_t n, int mode);
void launch_rhs(hipStream_t s, const double *rho, const double *sum, double inv_n, double *b, size_t n);
void launch_sub_mean(hipStream_t s, double *x, const double *sum, double inv_n, size_t n);
void launch_mul(hipStream_t s, double *y, const double *a, const double *x, size_t n);
// out = a x + b y (y == nullptr: out = a x)
void launch_axpby(hipStream_t s, double *out, double a, const double *x, double b, const double *y, size_t n);
void launch_rsqrt(hipStream_t s, const double *eps, double *sinv, size_t n);
void launch_check_eps(hipStream_t s, const double *eps, size_t n, int *flags);
void launch_check_finite(hipStream_t s, const double *x, size_t n, int *flags);

// wet slab <-> full box
template <class T>
void launch_wet_residual(hipStream_t s, const Plan &p, const double *v, const double *dD,
                         const double *eps, T *fW);
// the wet residual of a float32 Krylov vector v with the float32 dry update dD
// and eps rounded to float32 (the arithmetic stays float64)
template <class T>
void launch_wet_residual_v32(hipStream_t s, const Plan &p, const float *v, const float *dD, const float *eps,
                             T *fW);
// the same for a float16 Krylov basis vector v
template <class T>
void launch_wet_residual_v16(hipStream_t s, const Plan &p, const _Float16 *v, const float *dD, const float *eps,
                             T *fW);
// out = A phi rounded to float32 for float32 phi and eps (a float32 Krylov
// basis vector; float64 arithmetic)
void launch_apply_full_f32(hipStream_t s, const Plan &p, const float *phi, const float *eps, float *out);
void launch_to_f32(hipStream_t s, const double *x, float *y, size_t n);
template <class T>
void launch_wet_add(hipStream_t s, const Plan &p, const T *uW, double *z);
template <class T>
void launch_wet_add(hipStream_t s, const Plan &p, const T *uW, float *z);
template <class T>
void launch_wet_eps(hipStream_t s, const Plan &p, const double *eps, T *epsW);

// level operations
template <class T>
void launch_level_residual(hipStream_t s, const Level &L, T *r);  // r = f - A u
template <class T>
void launch_level_smooth(hipStream_t s, const Level &L, int color);
// fc = full weighting of the fine residual rf; also zeroes C.u
template <class T>
void launch_restrict(hipStream_t s, const Level &F, const Level &C, const T *rf, T *fc);
// fc = full weighting of the fine residual f - A u (never stored), coarse u zeroed
template <class T>
void launch_resid_restrict(hipStream_t s, const Level &F, const Level &C);
template <class T>
void launch_prolong_add(hipStream_t s, const Level &F, const Level &C);

template <class T>
void launch_coarsen_eps(hipStream_t s, const Level &F, const Level &C);
template <class T>
void launch_zero(hipStream_t s, T *x, size_t n);
// One red-black sweep (first_color, then the other) from uin to uout in a
// single pass; uin, uout: ghosted arrays of level L (ghost planes zero).
// With zadd (a box array of nzb planes), the row-band kernel adds the result
// into zadd at box planes (kw0 + k) mod nzb instead of writing uout, and the
// call returns true; the tiled kernel ignores zadd and returns false.
template <class T>
bool sweep_band_fits(const Level &L);  // the row-band fused sweep takes this level
template <class T>
bool launch_sweep_fused(hipStream_t s, const Level &L, const T *uin, T *uout, int first_color, bool zero_in,
                        bool tiles_only, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr,
                        T *zadd = nullptr, int nzb = 0, int kw0 = 0);
// The rest of a V-cycle from level l0 down, in one single-workgroup kernel.
template <class T>
void launch_vcycle_bottom(hipStream_t s, const std::vector<Level *> &levels, size_t l0, int pre, int post,
                          int coarse_sweeps);
constexpr size_t BOTTOM_MAX_POINTS = 8192;     // levels this small (and below) go to the bottom kernel
constexpr size_t BOTTOM_LDS_BYTES = 160 * 1024;  // the bottom set runs out of LDS when it fits this
constexpr size_t FUSED_MIN_POINTS = 1u << 20;  // levels this large use the fused sweep
constexpr size_t BAND_MIN_POINTS = 1u << 14;   // the row-band fused sweep from this size where it fits

// kern_sixth.hip: the sixth-order operator (order = 6)
void launch_d1eps(hipStream_t s, const Plan &p, const double *eps, double *G);    // G: 3N
// out = A6 x (or A6^T x), or b - that when residual
void launch_apply6(hipStream_t s, const Plan &p, const double *x, const double *eps, const double *G,
                   const double *b, double *out, bool residual, bool trans);
// A6 (A6^T) applied to a float32 Krylov vector with eps and D1 eps rounded to
// float32; float64 arithmetic, float32 out, no removal of the mean
void launch_apply6_f32(hipStream_t s, const Plan &p, const float *x, const float *eps, const float *G, float *out,
                       bool trans);
template <class T>
void launch_wet_residual6(hipStream_t s, const Plan &p, const double *v, const double *dD, const double *eps,
                          const double *G, T *fW, bool trans);
// finest wet level, sixth-order operator (slab unknowns zero outside W):
// smooth: one weighted-Jacobi sweep u -> out (ghosted); else out = f - A6 u
template <class T>
void launch_wet6(hipStream_t s, const Plan &p, const Level &L, const T *u, T *out, const double *eps, const double *G,
                 bool smooth, double omega);
void launch_grad6(hipStream_t s, const Plan &p, const double *phi, const double *lam, double *g);
void launch_charge_potential(hipStream_t s, const Plan &p, const double *phi, const double *lam, double *psi);
// out = gr * m / h^3 (+ add)
void launch_scaled_product(hipStream_t s, const Plan &p, const double *gr, const double *m, const double *add,
                           double *out);

// kern_fft.hip
// symbol of the operator of the given order (2: 7-point, 6: Eq. 18) along one axis
void fft_plan_axis(FFTAxis &ax, int n, double h, bool half, int order);
// out = s .* L^{-1} (s .* r) (s == nullptr: unscaled), zero mean; fp32: the
// spectrum (cbuf, sized for float64) and the transforms in float32
void launch_vacuum_solve(hipStream_t st, const Plan &p, const FFTAxis &ax, const FFTAxis &ay,
                         const FFTAxis &az, const double *r, const double *sinv, void *cbuf,
                         double *out, Profiler *prof, bool fp32);
// the same from a float32 Krylov basis vector to a float32 preconditioned one
void launch_vacuum_solve(hipStream_t st, const Plan &p, const FFTAxis &ax, const FFTAxis &ay,
                         const FFTAxis &az, const float *r, const double *sinv, void *cbuf,
                         float *out, Profiler *prof, bool fp32);
// and from a float16 one
void launch_vacuum_solve(hipStream_t st, const Plan &p, const FFTAxis &ax, const FFTAxis &ay,
                         const FFTAxis &az, const _Float16 *r, const double *sinv, void *cbuf,
                         float *out, Profiler *prof, bool fp32);

// kern_blas.hip: deterministic reductions
void launch_dot(hipStream_t s, const double *x, const double *y, size_t n, double *partial,
                double *out);
void launch_sum(hipStream_t s, const double *x, size_t n, double *partial, double *out);
// out[i] = V_i . w (i < nv); if norm_out: *norm_out = w . w (same pass)
void launch_multidot(hipStream_t s, const double *V, size_t ldv, int nv, const double *w,
                     size_t n, double *partial, double *out, double *norm_out);
// w -= sum_i c[i] V_i ; if norm_out: *norm_out = ||w||^2
void launch_axpy_multi(hipStream_t s, double *w, const double *V, size_t ldv, int nv,
                       const double *c, size_t n, double sign, double *partial, double *norm_out);
bool orth_update_supported(const double *V, size_t ldv, int nv, size_t n);
// mean_free: w is an operator output whose mean must go too (its sum at hc[67]
// from launch_multidot_sum); the constant direction is removed in the same pass
void launch_orth_update(hipStream_t s, double *w, const double *V, size_t ldv, int nv, double *hc, size_t n,
                        double *partial, bool mean_free = false);
// the projection of launch_multidot (nv <= 16, 16-byte aligned) with the sum of
// w's elements into *sum_out as well
void launch_multidot_sum(hipStream_t s, const double *V, size_t ldv, int nv, const double *w, size_t n,
                         double *partial, double *out, double *norm_out, double *sum_out);
// float32 Krylov basis (mixed precision): projections and update in float64
// arithmetic on float32 vectors (n and ldv multiples of 4, 16-byte aligned)
bool krylov32_supported(const float *V, size_t ldv, size_t n);
// the float32 orth update rescales its result to unit norm only when that norm
// is off 1 by more than this (float64 vectors: 1e-8)
constexpr double RESCALE_TOL_F32 = 1e-6;
// Hessenberg column slot of the float16 basis' Gram row (see launch_multidot16)
constexpr int GRAM_SLOT = 20;
void launch_multidot32(hipStream_t s, const float *V, size_t ldv, int nv, const float *w, size_t n, double *partial,
                       double *out, double *norm_out);
void launch_orth_update32(hipStream_t s, float *w, const float *V, size_t ldv, int nv, double *hc, size_t n,
                          double *partial, bool mean_free = false);
// the float32 projection with the sum of w as well (mean-free Arnoldi step)
void launch_multidot32_sum(hipStream_t s, const float *V, size_t ldv, int nv, const float *w, size_t n,
                           double *partial, double *out, double *norm_out, double *sum_out);
// x -= mean(x) for a float32 vector (the sum lands at *sum_out)
void launch_sub_mean32(hipStream_t s, float *x, size_t n, double *partial, double *sum_out);
void launch_scale_to32(hipStream_t s, float *x32, const double *r, const double *den_sq, size_t n);
// float16 Krylov basis (mixed precision, second order): the basis V in
// float16, the current vector also in float32 (w, the preconditioner's
// input); projections and update in float64 arithmetic (n and ldv multiples
// of 8, 16-byte aligned)
bool krylov16_supported(const void *V, size_t ldv, size_t n);
// (nv <= 16; with gram_out, also the last vector's products with V_0..V_{nv-1}
// into gram_out[0..nv), the row of the basis' Gram matrix that the update of
// a float16 basis divides by)
void launch_multidot16(hipStream_t s, const _Float16 *V, size_t ldv, int nv, const float *w, size_t n,
                       double *partial, double *out, double *norm_out, double *gram_out);
// vn <- (w - sum_q h_q V_q) / beta in float16 (w read in float32, not written),
// beta the exact norm of w - V h through the basis' Gram matrix, whose row q
// the projection pass of step q left in Hessenberg column q (hd0 + q hstride)
void launch_orth_update16(hipStream_t s, const float *w, _Float16 *vn, const _Float16 *V, size_t ldv, int nv,
                          double *hc, const double *hd0, int hstride, size_t n);
// xh = r / sqrt(*den_sq) in float16 (and in float32 into x32 unless null)
void launch_scale_to16(hipStream_t s, float *x32, _Float16 *xh, const double *r, const double *den_sq, size_t n);
// x += sum_q c[q] Z_q with float32 Z_q (nv <= 16), float64 x and sums
void launch_axpy_multi32(hipStream_t s, double *x, const float *Z, size_t ldz, int nv, const double *c, size_t n);
// energy sums: out[0] = sum rho phi (compensated), out[1] = sum_faces eps_f (D_f phi)^2
void launch_energy(hipStream_t s, const Plan &p, const double *rho, const double *phi,
                   const double *eps, double *partial, double *out);

// kern_atoms.hip
struct AtomParams {
    double eps_inf, delta, delta_z, z_lim;
    int exclusion;
    int model;                    // 0: product of switches; 1: dummy density (Eqs. 9, 10, 19)
    double beta, decay;           // model 1
};
constexpr int GAMMA_MAX_ATOMS = 4096;
// S: N doubles (model 0: the switch product) or 2N (model 1: log gamma, then
// d eps / d log gamma)
void launch_build_eps(hipStream_t s, const Plan &p, int n, const double *atoms_dev,
                      const AtomParams &ap, double *Hz, double *eps, double *S);
void launch_build_rho(hipStream_t s, const Plan &p, int n, const double *atoms_dev,
                      double *rho);
void launch_forces(hipStream_t s, const Plan &p, int n, const double *atoms_dev,
                   const AtomParams *ap, const double *phi, const double *g, const double *S,
                   const double *Hz, double *fpart, double *out);
size_t forces_partial_len(const Plan &p, int n, int model);

}  // namespace dwp
