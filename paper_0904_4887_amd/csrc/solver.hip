// Host orchestration of the dry/wet solver and the C ABI.
//
// The solve (paper Sec. II.F, made self-consistent): flexible GMRES(m) on the
// full periodic box for A phi = -4 pi (rho - mean rho), right-preconditioned by
// one application of the dry/wet split:
//   1. dry update   dD = L^{-1} v        (3-D FFT vacuum solve, Eq. 15 on the
//                                          grid; optionally s L^{-1} s v with
//                                          s = eps^-1/2)
//   2. wet residual rW = (v - A dD) on W  (float64)
//   3. wet solve    dW ~ A_WW^{-1} rW     (V-cycles on W, zero Dirichlet data
//                                          on the dry planes next to W)
//   4. combine      z = dD + extend(dW)
// The dry update gives the wet solve its boundary data, as in the paper's
// two-step scheme; the Krylov iteration makes the combination converge to the
// exact full-box solution.
#include "dwp_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>

namespace dwp {

void fail(int status, const std::string &msg) { throw Error{status, msg}; }

void DevBuf::alloc(size_t n_bytes) {
    if (p && bytes >= n_bytes) return;
    release();
    if (n_bytes == 0) return;
    if (hipMalloc(&p, n_bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        fail(DWP_ENOMEM, "device allocation of " + std::to_string(n_bytes) + " bytes failed");
    }
    bytes = n_bytes;
}

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

static const char *const kGroupNames[PG_COUNT] = {
    "fft_x", "fft_y", "fft_z", "rbgs_fine", "rbgs_coarse", "mg_other", "mg_bottom", "apply_full",
    "wet_slab", "multidot", "axpy_multi", "vector", "builders", "forces"};

const char *prof_group_name(int g) { return (g >= 0 && g < PG_COUNT) ? kGroupNames[g] : ""; }

int Profiler::reserve(int group) {
    if (!on || (only >= 0 && group != only)) return -1;
    while (next + 2 > pool.size()) {
        hipEvent_t e;
        DWP_HIP(hipEventCreate(&e));
        pool.push_back(e);
    }
    const int ev = (int)next;
    next += 2;
    return ev;
}

void Profiler::done(int ev, int group, double b) {
    if (ev >= 0) pending.push_back(Pending{group, ev, b});
}

int Profiler::begin(hipStream_t s, int group) {
    const int ev = reserve(group);
    if (ev >= 0) DWP_HIP(hipEventRecord(pool[ev], s));
    return ev;
}

void Profiler::end(hipStream_t s, int ev, int group, double b) {
    if (ev < 0) return;
    DWP_HIP(hipEventRecord(pool[ev + 1], s));
    done(ev, group, b);
}

void Profiler::collect() {
    for (const Pending &q : pending) {
        float t = 0.f;
        DWP_HIP(hipEventElapsedTime(&t, pool[q.ev], pool[q.ev + 1]));
        ms[q.group] += t;
        bytes[q.group] += q.bytes;
        launches[q.group] += 1;
    }
    pending.clear();
    next = 0;
}

void Profiler::reset() {
    for (int g = 0; g < PG_COUNT; ++g) { ms[g] = 0; bytes[g] = 0; launches[g] = 0; }
}

Profiler::~Profiler() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

void PhaseTimer::start() {
    on = true;
    used = 0;
    phase.clear();
}

void PhaseTimer::mark(hipStream_t s, int ph) {
    if (!on) return;
    if (used == pool.size()) {
        hipEvent_t e;
        DWP_HIP(hipEventCreate(&e));
        pool.push_back(e);
    }
    DWP_HIP(hipEventRecord(pool[used], s));
    phase.push_back(ph);
    ++used;
}

void PhaseTimer::finish(double *ms) {
    for (int q = 0; q < PH_COUNT; ++q) ms[q] = 0.0;
    for (size_t i = 0; i + 1 < used; ++i) {
        float t = 0.f;
        DWP_HIP(hipEventElapsedTime(&t, pool[i], pool[i + 1]));
        ms[phase[i]] += t;
    }
    on = false;
    used = 0;
    phase.clear();
}

PhaseTimer::~PhaseTimer() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

#define PROF(c, group, nbytes, stmt)                                \
    do {                                                           \
        const int ev_ = (c)->prof.begin((c)->stream, (group));      \
        stmt;                                                      \
        (c)->prof.end((c)->stream, ev_, (group), (double)(nbytes)); \
    } while (0)

namespace {

constexpr int COARSE_TARGET = 1024;  // coarsest level: at most this many points
constexpr size_t HESS_OFFSET = 512;   // device Hessenberg columns inside coef
constexpr size_t HESS_STRIDE = 72;

struct LevelDims {
    int nx, ny, nw;
    double h[3];
    bool zc;
};

// Coarsening rule: x, y periodic, halved only while the child stays even (so
// red-black colouring survives the wrap); z (Dirichlet) halved when the
// interval count nw + 1 is even.  While hz > semi_ratio max(hx, hy) only x, y
// are coarsened (semi-coarsening for the anisotropic spacing).
std::vector<LevelDims> plan_levels(int nx, int ny, int nw, const double h[3], int max_levels, double semi_ratio) {
    std::vector<LevelDims> v;
    LevelDims L{nx, ny, nw, {h[0], h[1], h[2]}, false};
    v.push_back(L);
    while ((int)v.size() < max_levels && (long)L.nx * L.ny * L.nw > COARSE_TARGET) {
        const double hxy = std::max(L.h[0], L.h[1]);
        const bool semi = L.h[2] > semi_ratio * hxy;
        const bool can_xy = L.nx % 4 == 0 && L.ny % 4 == 0;
        const bool can_z = (L.nw + 1) % 2 == 0 && (L.nw + 1) / 2 - 1 >= 1;
        if (!can_xy) break;
        LevelDims C = L;
        C.nx = L.nx / 2;
        C.ny = L.ny / 2;
        C.h[0] = 2 * L.h[0];
        C.h[1] = 2 * L.h[1];
        if (semi) {
            C.zc = false;
        } else {
            if (!can_z) break;
            C.nw = (L.nw + 1) / 2 - 1;
            C.h[2] = 2 * L.h[2];
            C.zc = true;
        }
        v.push_back(C);
        L = C;
    }
    return v;
}

long coarsest_size(const std::vector<LevelDims> &v) {
    const LevelDims &c = v.back();
    return (long)c.nx * c.ny * c.nw;
}

bool good_size(int n) {
    if (n < 8 || n > 4096 || n % 2) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

template <class T> size_t tsize() { return sizeof(T); }

void free_levels(dwp_ctx *c) {
    for (Level *L : c->plan.levels) delete L;
    c->plan.levels.clear();
    c->precision_built = -1;
}

// Choose the wet planes [k_w0, k_w1) (k_w0 in [0, nz)) for the options: the
// requested first plane may move down by up to nz / 8 planes until the slab
// coarsens to a level of at most COARSE_TARGET points.
void choose_wet(int nx, int ny, int nz, const double h[3], const double L[3], const dwp_opts &o, int *kw0,
                int *kw1, int *nw_out) {
    double zlo = o.z_wet_lo, zhi = o.z_wet_hi;
    if (std::isnan(zlo)) zlo = 0.35 * L[2];
    if (std::isnan(zhi)) zhi = L[2];
    if (!std::isfinite(zlo) || !std::isfinite(zhi)) fail(DWP_EINVAL, "wet bounds must be finite");
    const int k0 = (int)std::ceil(zlo / h[2] - 1e-9);
    const int k1 = (int)std::ceil(zhi / h[2] - 1e-9);
    const int nw0 = k1 - k0;
    if (nw0 < 3) fail(DWP_EINVAL, "wet region must hold at least 3 planes");
    if (nw0 > nz - 1) fail(DWP_EINVAL, "wet region must leave at least one dry plane");
    int best_nw = nw0;
    long best = coarsest_size(plan_levels(nx, ny, nw0, h, o.max_levels, o.semi_ratio));
    const int limit = std::min(nz - 1, nw0 + std::max(1, nz / 8));
    for (int nw = nw0; nw <= limit; ++nw) {
        const long cs = coarsest_size(plan_levels(nx, ny, nw, h, o.max_levels, o.semi_ratio));
        if (cs < best) { best = cs; best_nw = nw; }
        if (cs <= COARSE_TARGET) { best_nw = nw; break; }
    }
    int a = k1 - best_nw, b = k1;
    const int shift = ((a % nz) + nz) % nz - a;
    *kw0 = a + shift;
    *kw1 = b + shift;
    *nw_out = best_nw;
}

// Plan the wet slab and its hierarchy for the current options.
void plan_wet(dwp_ctx *c) {
    Plan &p = c->plan;
    choose_wet(p.nx, p.ny, p.nz, p.h, p.L, c->opts, &p.k_w0, &p.k_w1, &p.nw);
    free_levels(c);
    for (const LevelDims &d : plan_levels(p.nx, p.ny, p.nw, p.h, c->opts.max_levels, c->opts.semi_ratio)) {
        Level *L = new Level();
        L->nx = d.nx; L->ny = d.ny; L->nw = d.nw;
        L->h[0] = d.h[0]; L->h[1] = d.h[1]; L->h[2] = d.h[2];
        L->zc = d.zc;
        L->plane = (size_t)d.nx * d.ny;
        p.levels.push_back(L);
    }
    // the bottom kernel takes every level from the first one that fits; a
    // coarsest level too large for one workgroup (x or y could not be halved
    // further) is smoothed by the grid-wide level kernels instead
    p.bottom = p.levels.size() - 1;
    if (p.levels.back()->n_interior() > BOTTOM_MAX_POINTS) p.bottom = p.levels.size();
    while (p.bottom > 0 && p.bottom < p.levels.size() && p.levels[p.bottom - 1]->n_interior() <= BOTTOM_MAX_POINTS)
        --p.bottom;
    if (p.levels.size() - p.bottom > 10) p.bottom = p.levels.size() - 10;
}

template <class T>
void alloc_levels(dwp_ctx *c) {
    for (Level *L : c->plan.levels) {
        L->eps.release(); L->u.release(); L->u2.release(); L->f.release(); L->r.release();
        L->eps.alloc(tsize<T>() * L->n_ghosted());
        L->u.alloc(tsize<T>() * L->n_ghosted());
        L->u2.alloc(tsize<T>() * L->n_ghosted());
        launch_zero<T>(c->stream, L->u2.as<T>(), L->n_ghosted());
        L->f.alloc(tsize<T>() * L->n_interior());
        L->r.alloc(tsize<T>() * L->n_interior());
        launch_zero<T>(c->stream, L->u.as<T>(), L->n_ghosted());
    }
}

void ensure_levels(dwp_ctx *c) {
    if (c->precision_built == c->opts.precision) return;
    if (c->opts.precision == DWP_MIXED) alloc_levels<float>(c);
    else alloc_levels<double>(c);
    c->precision_built = c->opts.precision;
}

// Level permittivities from the full-box eps.
template <class T>
void prepare_level_eps(dwp_ctx *c) {
    Plan &p = c->plan;
    launch_wet_eps<T>(c->stream, p, c->eps.as<double>(), p.levels[0]->eps.as<T>());
    for (size_t l = 1; l < p.levels.size(); ++l)
        launch_coarsen_eps<T>(c->stream, *p.levels[l - 1], *p.levels[l]);
}

// The FFT symbol tables for the operator order of the options.
void plan_fft(dwp_ctx *c) {
    const Plan &p = c->plan;
    const int order = c->opts.order;
    fft_plan_axis(c->fx, p.nx, p.h[0], true, order);
    fft_plan_axis(c->fy, p.ny, p.h[1], false, order);
    fft_plan_axis(c->fz, p.nz, p.h[2], false, order);
    c->fft_order = order;
}

void prepare_eps(dwp_ctx *c) {
    ensure_levels(c);
    launch_rsqrt(c->stream, c->eps.as<double>(), c->sinv.as<double>(), c->plan.N);
    if (c->opts.order == 6) {
        c->G6.alloc(sizeof(double) * 3 * c->plan.N);
        launch_d1eps(c->stream, c->plan, c->eps.as<double>(), c->G6.as<double>());
    }
    if (c->opts.precision == DWP_MIXED) prepare_level_eps<float>(c);
    else prepare_level_eps<double>(c);
    if (c->opts.krylov_fp32) {
        c->eps32.alloc(sizeof(float) * c->plan.N);
        launch_to_f32(c->stream, c->eps.as<double>(), c->eps32.as<float>(), c->plan.N);
        if (c->opts.order == 6) {
            c->G632.alloc(sizeof(float) * 3 * c->plan.N);
            launch_to_f32(c->stream, c->G6.as<double>(), c->G632.as<float>(), 3 * c->plan.N);
        }
    }
}

void sync(dwp_ctx *c) {
    DWP_HIP(hipStreamSynchronize(c->stream));
    c->prof.collect();
}

void to_host(dwp_ctx *c, const double *dev, size_t n) {
    if (n > c->host_len) fail(DWP_EINVAL, "internal: host staging too small");
    DWP_HIP(hipMemcpyAsync(c->host, dev, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    sync(c);
}

// One V-cycle from level l down.  Coarse levels enter with a zero correction
// (the restriction zeroes it); on the fine level, u_unset says that the
// correction array holds stale values that must act as zero (first cycle),
// otherwise it holds the previous cycle's correction.
template <class T>
bool vcycle(dwp_ctx *c, size_t l, bool u_unset, T *zadd) {
    Plan &p = c->plan;
    Level &L = *p.levels[l];
    hipStream_t s = c->stream;
    const double ts = (double)sizeof(T);
    const int sg = l == 0 ? PG_RBGS_FINE : PG_RBGS_COARSE;
    const double pass_bytes = 2.0 * ts * (double)L.n_interior();  // half of read u, eps, f + write u
    // the finest level smooths the sixth-order operator itself (weighted
    // Jacobi); the adjoint solve keeps the symmetric 7-point smoother, which
    // approximates A6^T as well as it approximates A6
    const bool six = l == 0 && c->opts.order == 6 && c->opts.smooth6 == 1 && !c->transposed;
    // the fused sweep on the large levels; the row-band one also on smaller
    // levels down to BAND_MIN_POINTS, where one launch per sweep instead of
    // two matters more than its z halo
    const size_t npts = L.n_interior();
    const bool fused = !six && c->opts.smoother != 0 &&
                       (npts >= FUSED_MIN_POINTS ||
                        (c->opts.smoother == 1 && npts >= BAND_MIN_POINTS && sweep_band_fits<T>(L)));
    const bool coarsest = l + 1 == p.levels.size();
    // the first sweep starts from a zero correction on coarse levels and in
    // the first cycle on the fine level, except that without pre-sweeps it
    // comes after the coarse-grid correction (then its input is not zero)
    bool zero_in = (l > 0 || u_unset) && (coarsest || c->opts.pre > 0);
    if (u_unset && !(fused && zero_in))
        PROF(c, PG_WET, ts * (double)L.n_ghosted(), launch_zero<T>(s, L.u.as<T>(), L.n_ghosted()));
    if (l >= p.bottom) {
        double nb = 0.0;
        for (size_t q = l; q < p.levels.size(); ++q) nb += (double)p.levels[q]->n_interior();
        PROF(c, PG_MG_BOTTOM, 4.0 * ts * nb,
             launch_vcycle_bottom<T>(s, p.levels, l, c->opts.pre, c->opts.post, c->opts.coarse_sweeps));
        return false;
    }
    bool added = false;
    auto smooth = [&](int first, T *za) {
        if (six) {
            // u, eps, f and the three components of D1 eps read per point, u written
            PROF(c, sg, (2.0 * ts + 32.0) * (double)L.n_interior(),
                 launch_wet6<T>(s, p, L, L.u.as<T>(), L.u2.as<T>(), c->eps.as<double>(), c->G6.as<double>(), true,
                                2.0 / 3.0));
            std::swap(L.u.p, L.u2.p);
        } else if (fused) {
            // timed by events that the launch itself records at the kernel's
            // start and end
            const int ev = c->prof.reserve(sg);
            added = launch_sweep_fused<T>(s, L, L.u.as<T>(), L.u2.as<T>(), first, zero_in, c->opts.smoother == 2,
                                          c->prof.event(ev, 0), c->prof.event(ev, 1), za, p.nz, p.k_w0);
            // u and f read (not u when starting from zero), eps read, u
            // written -- or z read and written when the result is added into z
            const double b = (zero_in ? 1.5 : 2.0) * pass_bytes + (added ? 0.5 * pass_bytes : 0.0);
            c->prof.done(ev, sg, b);
            std::swap(L.u.p, L.u2.p);
        } else {
            PROF(c, sg, pass_bytes, launch_level_smooth<T>(s, L, first));
            PROF(c, sg, pass_bytes, launch_level_smooth<T>(s, L, 1 - first));
        }
        zero_in = false;
    };
    if (coarsest) {  // too large for the bottom kernel: coarse_sweeps sweeps here
        for (int k = 0; k < c->opts.coarse_sweeps; ++k) smooth(0, nullptr);
        return false;
    }
    for (int k = 0; k < c->opts.pre; ++k) smooth(0, nullptr);
    Level &C = *p.levels[l + 1];
    if (six) {
        // the sixth-order residual, then full weighting (which zeroes the coarse unknowns)
        PROF(c, PG_MG_OTHER, (3.0 * ts + 32.0) * (double)L.n_interior(),
             launch_wet6<T>(s, p, L, L.u.as<T>(), L.r.as<T>(), c->eps.as<double>(), c->G6.as<double>(), false, 0.0));
        PROF(c, PG_MG_OTHER, ts * (L.n_interior() + C.n_interior() + C.n_ghosted()),
             launch_restrict<T>(s, L, C, L.r.as<T>(), C.f.as<T>()));
    } else {
        // residual and full-weighting restriction in one pass (u, eps, f read;
        // the coarse right-hand side written and the coarse unknowns zeroed)
        PROF(c, PG_MG_OTHER, ts * (3.0 * L.n_interior() + C.n_interior() + C.n_ghosted()),
             launch_resid_restrict<T>(s, L, C));
    }
    vcycle<T>(c, l + 1, false, nullptr);
    PROF(c, PG_MG_OTHER, ts * (C.n_interior() + 2.0 * L.n_interior()), launch_prolong_add<T>(s, L, C));
    // the last sweep may add its result straight into zadd
    for (int k = 0; k < c->opts.post; ++k) smooth(1, k + 1 == c->opts.post ? zadd : nullptr);
    return added;
}

template <class T, class TV, class TZ>
void split_impl(dwp_ctx *c, const TV *v, TZ *z) {
    Plan &p = c->plan;
    hipStream_t s = c->stream;
    const bool scaled = c->opts.scaled_dry != 0;
    c->phases.mark(s, PH_FFT);
    launch_vacuum_solve(s, p, c->fx, c->fy, c->fz, v, scaled ? c->sinv.as<double>() : nullptr, c->cbuf.p, z,
                        &c->prof, c->opts.fft_fp32 != 0);
    c->phases.mark(s, PH_MG);
    if (c->opts.cycles == 0) {  // no wet correction: the split is the dry update alone
        c->phases.mark(s, PH_KRYLOV);
        return;
    }
    Level &F = *p.levels[0];
    const double nW = (double)F.n_interior();
    if constexpr (std::is_same<TV, _Float16>::value) {
        PROF(c, PG_WET, (6.0 + sizeof(TZ) + sizeof(T)) * nW,
             launch_wet_residual_v16<T>(s, p, v, z, c->eps32.as<float>(), F.f.as<T>()));
    } else if constexpr (sizeof(TV) == 4) {
        PROF(c, PG_WET, (8.0 + sizeof(TZ) + sizeof(T)) * nW,
             launch_wet_residual_v32<T>(s, p, v, z, c->eps32.as<float>(), F.f.as<T>()));
    } else if (c->opts.order == 6) {
        PROF(c, PG_WET, (48.0 + sizeof(T)) * nW,
             launch_wet_residual6<T>(s, p, v, z, c->eps.as<double>(), c->G6.as<double>(), F.f.as<T>(),
                                     c->transposed));
    } else {
        PROF(c, PG_WET, (24.0 + sizeof(T)) * nW,
             launch_wet_residual<T>(s, p, v, z, c->eps.as<double>(), F.f.as<T>()));
    }
    // the wet correction is added into z by the last fine-level sweep where
    // the row-band kernel runs it and z has the level's type, else afterwards
    T *za = nullptr;
    if constexpr (std::is_same<TZ, T>::value) za = z;
    bool added = false;
    for (int k = 0; k < c->opts.cycles; ++k) added = vcycle<T>(c, 0, k == 0, k + 1 == c->opts.cycles ? za : nullptr);
    if (!added)
        PROF(c, PG_WET, (2.0 * sizeof(TZ) + sizeof(T)) * nW, launch_wet_add<T>(s, p, F.u.as<T>(), z));
    c->phases.mark(s, PH_KRYLOV);
}

void apply_split(dwp_ctx *c, const double *v, double *z) {
    if (c->opts.precision == DWP_MIXED) split_impl<float, double, double>(c, v, z);
    else split_impl<double, double, double>(c, v, z);
}
// the split of a float32 (float16) Krylov vector into a float32 one (mixed
// precision, second order): z is rounded to float32 where it is stored, and
// the Krylov method uses the stored z as it is
void apply_split(dwp_ctx *c, const float *v, float *z) { split_impl<float, float, float>(c, v, z); }
void apply_split(dwp_ctx *c, const _Float16 *v, float *z) { split_impl<float, _Float16, float>(c, v, z); }

void check_finite_dev(dwp_ctx *c, const double *x, const char *what) {
    int *flags = reinterpret_cast<int *>(c->partial.as<double>());
    launch_check_finite(c->stream, x, c->plan.N, flags);
    DWP_HIP(hipMemcpyAsync(c->host, flags, sizeof(int) * RED_BLOCKS, hipMemcpyDeviceToHost, c->stream));
    sync(c);
    const int *hf = reinterpret_cast<const int *>(c->host);
    int f = 0;
    for (int b = 0; b < RED_BLOCKS; ++b) f |= hf[b];
    if (f & 1) fail(DWP_ENONFINITE, std::string(what) + " holds NaN or Inf");
}

// The outer operator on the full box: out = A x (residual: out = b - A x).
// Order 6: A6 (A6^T in the adjoint solve) followed by the removal of the
// mean, so the Krylov space stays in the zero-mean vectors where Q A6 is
// invertible.
void apply_operator(dwp_ctx *c, const double *x, const double *b, double *out, bool residual) {
    Plan &p = c->plan;
    hipStream_t s = c->stream;
    const size_t N = p.N;
    if (c->opts.order != 6) {
        PROF(c, PG_APPLY, (residual ? 32.0 : 24.0) * N,
             launch_apply_full(s, p, x, c->eps.as<double>(), b, out, residual));
        return;
    }
    double *coef = c->coef.as<double>();
    // x, eps and the three components of D1 eps read, out written (+ b read)
    PROF(c, PG_APPLY, (residual ? 56.0 : 48.0) * N,
         launch_apply6(s, p, x, c->eps.as<double>(), c->G6.as<double>(), b, out, residual, c->transposed));
    PROF(c, PG_VEC, 8.0 * N, launch_sum(s, out, N, c->partial.as<double>(), coef + 410));
    PROF(c, PG_VEC, 16.0 * N, launch_sub_mean(s, out, coef + 410, 1.0 / (double)N, N));
}

// FGMRES(m) with the split as right preconditioner; x is updated in place.
// Each restart cycle is enqueued without host round trips: the Gram-Schmidt
// coefficients, the norm of the new basis vector and its normalisation stay on
// the device (one projection pass and one update pass of classical
// Gram-Schmidt per step; the update divides by the norm that Pythagoras gives
// from the projection, so no separate normalisation pass is needed), and the
// host reads the Hessenberg columns to solve the small least-squares problem.
// The host looks at the columns only after the step from which the cycle may
// meet the tolerance (predicted from the per-step residual reduction of the
// previous cycle; the first cycle is looked at after its first step and
// predicted from that step's reduction), and from there after every step, so
// that a cycle stops at the first step whose least-squares residual meets the
// tolerance.  The true
// residual is recomputed at the start of every cycle, so the result meets the
// tolerance whatever the loss of orthogonality.  Returns the number of steps;
// *rel receives the final true relative residual.
int fgmres(dwp_ctx *c, const double *b, double bnorm, double *x, int *restarts, double *rel) {
    Plan &p = c->plan;
    const dwp_opts &o = c->opts;
    hipStream_t s = c->stream;
    const size_t N = p.N;
    const int m = o.restart;
    double *V = c->V.as<double>(), *Z = c->Z.as<double>();
    // mixed precision with krylov_fp32: the Arnoldi basis in float32 (every
    // product, sum and the coupling update x += Z y stay float64; each restart
    // recomputes the true residual in float64); with krylov_fp16 too, the
    // basis V in float16
    const bool six = c->opts.order == 6;
    const bool v32 = c->opts.krylov_fp32 != 0 && c->opts.precision == DWP_MIXED &&
                     (!six || (c->opts.cycles == 0 && c->G632.bytes >= sizeof(float) * 3 * N)) &&
                     c->V32.bytes >= sizeof(float) * N * (m + 1) && krylov32_supported(c->V32.as<float>(), N, N) &&
                     krylov32_supported(c->Z.as<float>(), N, N) && c->eps32.bytes >= sizeof(float) * N;
    float *V32 = c->V32.as<float>();
    float *Z32 = c->Z.as<float>();  // with v32 the Z buffer holds float32 vectors
    // krylov_fp16 (second order): the V32 buffer holds the basis in float16
    // and, after it, the new vector w = A z of each step in float32; the
    // preconditioner reads the float16 basis vector
    const size_t v16_bytes = (sizeof(_Float16) * N * (m + 1) + 255) / 256 * 256;
    _Float16 *V16 = reinterpret_cast<_Float16 *>(V32);
    float *vcur = reinterpret_cast<float *>(reinterpret_cast<char *>(V32) + v16_bytes);
    const bool v16_ok = v32 && !six && c->opts.krylov_fp16 != 0 && v16_bytes + sizeof(float) * N <= c->V32.bytes &&
                        krylov16_supported(V16, N, N) && krylov16_supported(vcur, N, N);
    // A cycle on a float16 basis cannot reduce the residual much below the
    // basis' rounding (2^-11), which costs iterations where cycles reduce it a
    // lot: a cycle after one that reduced it more than V16_MAX_REDUCTION-fold
    // runs on the float32 basis, and so does the first cycle of a solve unless
    // the first cycle of the context's previous solve reduced it less.
    constexpr double V16_MAX_REDUCTION = 100.0;
    double beta_prev = -1.0;
    int cycle = 0;
    bool v16 = false;
    double *coef = c->coef.as<double>();
    // column j at Hd + j * 72: [0..j] dots, 64 ||w||^2, 65 squared norm of the
    // new vector before any rescaling, 66 the divisor of the fused update;
    // with a float16 basis [20..20+j] the products of V_j with V_0..V_j (its
    // row of the basis' Gram matrix; the update divides by the exact norm)
    double *Hd = coef + HESS_OFFSET;
    double *beta2 = coef + 8;
    double *part = c->partial.as<double>();
    std::vector<double> H((size_t)(m + 1) * m), g(m + 1), cs(m), sn(m), y(m);
    std::vector<char> fused(m, 0);
    auto Hij = [&](int i, int j) -> double & { return H[(size_t)i * m + j]; };
    const double target = o.tol * bnorm;
    double rate = -1.0;  // per-step residual reduction of the last cycle (< 0: unknown)
    int iters = 0;
    *restarts = 0;
    for (;;) {
        // r = b - A x into V_0 (float64; with a float32 basis into r first),
        // ||r||^2 on the device
        double *r0 = v32 ? c->r.as<double>() : V;
        apply_operator(c, x, b, r0, true);
        PROF(c, PG_VEC, 8.0 * N, launch_dot(s, r0, r0, N, part, beta2));
        to_host(c, beta2, 1);
        const double beta = std::sqrt(c->host[0]);
        if (!std::isfinite(beta)) fail(DWP_ENONFINITE, "residual is not finite");
        if (cycle == 1) c->first_cycle_red = beta > 0.0 ? beta_prev / beta : 1e300;
        ++cycle;
        *rel = beta / bnorm;
        if (*rel <= o.tol || iters >= o.max_outer) return iters;
        ++*restarts;
        v16 = v16_ok && (beta_prev > 0.0 ? beta * V16_MAX_REDUCTION >= beta_prev
                                         : c->first_cycle_red > 0.0 && c->first_cycle_red <= V16_MAX_REDUCTION);
        beta_prev = beta;
        if (v16) PROF(c, PG_VEC, 10.0 * N, launch_scale_to16(s, nullptr, V16, r0, beta2, N));
        else if (v32) PROF(c, PG_VEC, 12.0 * N, launch_scale_to32(s, V32, r0, beta2, N));
        else PROF(c, PG_VEC, 16.0 * N, launch_scale_dev(s, V, nullptr, beta2, N, 0));
        const int mm = std::min(m, o.max_outer - iters);
        // First step after which the host checks the least-squares residual:
        // predicted from the per-step reduction of the last cycle, or, in the
        // first cycle, from the reduction of its first step (checked at once).
        auto predict = [&](double r, int done) {
            if (!(r > 0.0 && r < 1.0)) return mm;
            const double need = std::log(target / beta) / std::log(r);
            return std::max(done + 1, std::min(mm, (int)std::floor(need) - 1));
        };
        int check_from = rate > 0.0 ? predict(rate, 0) : 1;
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;        // columns folded into the least-squares problem
        bool stop = false;
        // fold column j (read back from the device) into the QR of H
        auto fold = [&](int j, const double *hc) {
            for (int i = 0; i <= j; ++i) Hij(i, j) = hc[i];
            // Fused update: the stored vector is (w - V h) / beta, rescaled by
            // its norm nu only when nu is off 1 by more than 1e-8 (1e-6 for a
            // float32 basis; the same test the device made; a float16 basis
            // divides by the exact norm and reports nu = 1).  Otherwise:
            // explicit norm.
            double hn = std::sqrt(std::max(hc[65], 0.0));
            const double rtol = v32 ? RESCALE_TOL_F32 : 1e-8;
            if (fused[j] && hn != 0.0) hn = std::fabs(hn - 1.0) <= rtol ? hc[66] : hc[66] * hn;
            if (!std::isfinite(hn)) fail(DWP_ENONFINITE, "Krylov basis is not finite");
            Hij(j + 1, j) = hn;
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * Hij(i, j) + sn[i] * Hij(i + 1, j);
                Hij(i + 1, j) = -sn[i] * Hij(i, j) + cs[i] * Hij(i + 1, j);
                Hij(i, j) = t;
            }
            const double den = std::hypot(Hij(j, j), Hij(j + 1, j));
            cs[j] = den > 0 ? Hij(j, j) / den : 1.0;
            sn[j] = den > 0 ? Hij(j + 1, j) / den : 0.0;
            Hij(j, j) = den;
            Hij(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            // exact solution in the current space, or the tolerance is met
            if (hn == 0.0 || std::fabs(g[j + 1]) <= target) stop = true;
        };
        int steps = 0;
        for (int j = 0; j < mm && !stop; ++j) {
            double *Vj = V + (size_t)j * N, *Vn = V + (size_t)(j + 1) * N, *Zj = Z + (size_t)j * N;
            double *hc = Hd + (size_t)j * HESS_STRIDE;
            if (v16) {
                // v_j (float16) -> z_j; w = A z_j into vcur (float32);
                // project on the float16 basis; the normalised vector into
                // the basis
                float *Zj32 = Z32 + (size_t)j * N;
                apply_split(c, (const _Float16 *)(V16 + (size_t)j * N), Zj32);
                fused[j] = 1;
                PROF(c, PG_APPLY, 12.0 * N, launch_apply_full_f32(s, p, (const float *)Zj32, c->eps32.as<float>(), vcur));
                PROF(c, PG_MULTIDOT, (2.0 * (j + 1) + 4.0) * N,
                     launch_multidot16(s, V16, N, j + 1, vcur, N, part, hc, hc + 64, hc + GRAM_SLOT));
                PROF(c, PG_AXPY, (2.0 * (j + 1) + 6.0) * N,
                     launch_orth_update16(s, vcur, V16 + (size_t)(j + 1) * N, V16, N, j + 1, hc, Hd, HESS_STRIDE,
                                          N));
            } else if (v32) {
                float *Vj32 = V32 + (size_t)j * N, *Vn32 = V32 + (size_t)(j + 1) * N, *Zj32 = Z32 + (size_t)j * N;
                apply_split(c, (const float *)Vj32, Zj32);
                fused[j] = 1;  // restart <= 16 is checked with the options
                if (six) {
                    // the adjoint's directions stay mean-free; A6 (A6^T) z without
                    // the removal of its mean, which the mean-free update does
                    if (c->transposed) PROF(c, PG_VEC, 16.0 * N, launch_sub_mean32(s, Zj32, N, part, coef + 411));
                    PROF(c, PG_APPLY, 24.0 * N,
                         launch_apply6_f32(s, p, (const float *)Zj32, c->eps32.as<float>(), c->G632.as<float>(), Vn32,
                                           c->transposed));
                    PROF(c, PG_MULTIDOT, 4.0 * N * (j + 2),
                         launch_multidot32_sum(s, V32, N, j + 1, Vn32, N, part, hc, hc + 64, hc + 67));
                    PROF(c, PG_AXPY, 4.0 * N * (j + 3), launch_orth_update32(s, Vn32, V32, N, j + 1, hc, N, part, true));
                } else {
                    // A z (float64 arithmetic, float32 out), then the projection and update on float32 vectors
                    PROF(c, PG_APPLY, 12.0 * N,
                         launch_apply_full_f32(s, p, (const float *)Zj32, c->eps32.as<float>(), Vn32));
                    PROF(c, PG_MULTIDOT, 4.0 * N * (j + 2),
                         launch_multidot32(s, V32, N, j + 1, Vn32, N, part, hc, hc + 64));
                    PROF(c, PG_AXPY, 4.0 * N * (j + 3), launch_orth_update32(s, Vn32, V32, N, j + 1, hc, N, part));
                }
            } else {
                apply_split(c, Vj, Zj);
                if (c->transposed) {
                    // A6^T does not annihilate the constants (A6 does): keep the
                    // iterate in the zero-mean space where the adjoint is posed
                    PROF(c, PG_VEC, 8.0 * N, launch_sum(s, Zj, N, part, coef + 411));
                    PROF(c, PG_VEC, 16.0 * N, launch_sub_mean(s, Zj, coef + 411, 1.0 / (double)N, N));
                }
                const double md = 8.0 * N * (j + 2), ax = 8.0 * N * (j + 3);
                fused[j] = orth_update_supported(V, N, j + 1, N);
                if (c->opts.order == 6 && fused[j]) {
                    // A6 z (A6^T z) without the separate removal of its mean: the
                    // projection also sums the new vector and the update takes
                    // the constant direction out with the others
                    PROF(c, PG_APPLY, 48.0 * N,
                         launch_apply6(s, p, Zj, c->eps.as<double>(), c->G6.as<double>(), nullptr, Vn, false,
                                       c->transposed));
                    PROF(c, PG_MULTIDOT, md,
                         launch_multidot_sum(s, V, N, j + 1, Vn, N, part, hc, hc + 64, hc + 67));
                    PROF(c, PG_AXPY, ax, launch_orth_update(s, Vn, V, N, j + 1, hc, N, part, true));
                } else if (fused[j]) {
                    apply_operator(c, Zj, nullptr, Vn, false);
                    PROF(c, PG_MULTIDOT, md, launch_multidot(s, V, N, j + 1, Vn, N, part, hc, hc + 64));
                    PROF(c, PG_AXPY, ax, launch_orth_update(s, Vn, V, N, j + 1, hc, N, part));
                } else {
                    apply_operator(c, Zj, nullptr, Vn, false);
                    PROF(c, PG_MULTIDOT, md, launch_multidot(s, V, N, j + 1, Vn, N, part, hc, hc + 64));
                    PROF(c, PG_AXPY, ax, launch_axpy_multi(s, Vn, V, N, j + 1, hc, N, -1.0, part, hc + 65));
                    PROF(c, PG_VEC, 16.0 * N, launch_scale_dev(s, Vn, nullptr, hc + 65, N, 0));
                }
            }
            steps = j + 1;
            if (steps >= check_from || steps == mm) {
                // read the columns not yet folded and fold them
                const int n_new = steps - k;
                DWP_HIP(hipMemcpyAsync(c->host, Hd + (size_t)k * HESS_STRIDE, sizeof(double) * HESS_STRIDE * n_new,
                                       hipMemcpyDeviceToHost, s));
                sync(c);
                const int k0 = k;
                for (int jj = k0; jj < steps && !stop; ++jj) fold(jj, c->host + (size_t)(jj - k0) * HESS_STRIDE);
                if (rate <= 0.0 && steps == 1 && !stop)
                    check_from = predict(std::fabs(g[1]) / beta, 1);
            }
        }
        iters += steps;
        if (k > 0 && std::fabs(g[k]) > 0.0) rate = std::pow(std::fabs(g[k]) / beta, 1.0 / k);
        // y = H^{-1} g (upper triangular), x += Z y
        for (int i = k - 1; i >= 0; --i) {
            double t = g[i];
            for (int l = i + 1; l < k; ++l) t -= Hij(i, l) * y[l];
            y[i] = Hij(i, i) != 0.0 ? t / Hij(i, i) : 0.0;
        }
        for (int i = 0; i < k; ++i) c->host[i] = y[i];
        DWP_HIP(hipMemcpyAsync(coef + 192, c->host, sizeof(double) * k, hipMemcpyHostToDevice, s));
        if (v32) PROF(c, PG_AXPY, (4.0 * k + 16.0) * N, launch_axpy_multi32(s, x, Z32, N, k, coef + 192, N));
        else PROF(c, PG_AXPY, 8.0 * N * (k + 2), launch_axpy_multi(s, x, Z, N, k, coef + 192, N, 1.0, part, nullptr));
        sync(c);  // the staging buffer is reused next
    }
}

void need_grid(dwp_ctx *c) {
    if (!c->have_grid) fail(DWP_ESTATE, "dwp_set_grid has not been called");
}
void need_eps(dwp_ctx *c) {
    need_grid(c);
    if (!c->have_eps) fail(DWP_ESTATE, "no permittivity: call dwp_set_epsilon or dwp_build_epsilon");
}

void validate_opts(const dwp_opts &o) {
    if (o.precision != DWP_FP64 && o.precision != DWP_MIXED) fail(DWP_EINVAL, "precision must be 0 or 1");
    if (o.pre < 0 || o.post < 0 || o.pre + o.post < 1 || o.pre > 16 || o.post > 16)
        fail(DWP_EINVAL, "pre/post sweeps out of range");
    if (o.coarse_sweeps < 1 || o.coarse_sweeps > 100000) fail(DWP_EINVAL, "coarse_sweeps out of range");
    if (o.max_levels < 1 || o.max_levels > 32) fail(DWP_EINVAL, "max_levels out of range");
    if (o.cycles < 0 || o.cycles > 64) fail(DWP_EINVAL, "cycles out of range");
    if (!(o.tol > 0.0) || !(o.tol < 1.0)) fail(DWP_EINVAL, "tol must lie in (0, 1)");
    if (o.max_outer < 1) fail(DWP_EINVAL, "max_outer must be >= 1");
    if (o.restart < 1 || o.restart > 63) fail(DWP_EINVAL, "restart must lie in [1, 63]");
    if (o.scaled_dry != 0 && o.scaled_dry != 1) fail(DWP_EINVAL, "scaled_dry must be 0 or 1");
    if (o.warm_start != 0 && o.warm_start != 1) fail(DWP_EINVAL, "warm_start must be 0 or 1");
    if (o.profile < 0 || o.profile > 2) fail(DWP_EINVAL, "profile must be 0, 1 or 2");
    if (o.smoother < 0 || o.smoother > 2) fail(DWP_EINVAL, "smoother must be 0, 1 or 2");
    if (o.fft_fp32 != 0 && o.fft_fp32 != 1) fail(DWP_EINVAL, "fft_fp32 must be 0 or 1");
    if (o.fft_fp32 && o.precision != DWP_MIXED) fail(DWP_EINVAL, "fft_fp32 needs the mixed precision mode");
    if (o.order != 2 && o.order != 6) fail(DWP_EINVAL, "order must be 2 or 6");
    if (o.smooth6 != 0 && o.smooth6 != 1) fail(DWP_EINVAL, "smooth6 must be 0 or 1");
    if (o.smooth6 && o.order != 6) fail(DWP_EINVAL, "smooth6 needs the sixth-order operator (order 6)");
    if (o.krylov_fp32 != 0 && o.krylov_fp32 != 1) fail(DWP_EINVAL, "krylov_fp32 must be 0 or 1");
    if (o.krylov_fp32 && o.precision != DWP_MIXED) fail(DWP_EINVAL, "krylov_fp32 needs the mixed precision mode");
    if (o.krylov_fp32 && o.order == 6 && o.cycles != 0)
        fail(DWP_EINVAL, "krylov_fp32 with the sixth-order operator needs cycles = 0 (the FFT dry update alone)");
    if (o.krylov_fp32 && o.restart > 16) fail(DWP_EINVAL, "krylov_fp32 takes restart lengths up to 16");
    if (o.krylov_fp16 != 0 && o.krylov_fp16 != 1) fail(DWP_EINVAL, "krylov_fp16 must be 0 or 1");
    if (!(o.semi_ratio >= 1.0 && o.semi_ratio <= 64.0)) fail(DWP_EINVAL, "semi_ratio must lie in [1, 64]");
    if (o.krylov_fp16 && (o.krylov_fp32 != 1 || o.order != 2))
        fail(DWP_EINVAL, "krylov_fp16 needs krylov_fp32 = 1 and the second-order operator");
}

AtomParams atom_params(const dwp_eps_params *ep) {
    AtomParams a;
    a.eps_inf = ep->eps_inf;
    a.delta = ep->delta;
    a.delta_z = ep->delta_z;
    a.z_lim = ep->z_lim;
    a.exclusion = ep->exclusion;
    a.model = ep->model;
    a.beta = ep->beta;
    a.decay = ep->decay;
    return a;
}

void validate_eps_params(const dwp_ctx *c, int n, const dwp_eps_params *ep) {
    if (!ep) fail(DWP_EINVAL, "params is NULL");
    if (!(ep->eps_inf > 1.0) || !std::isfinite(ep->eps_inf)) fail(DWP_EINVAL, "eps_inf must be > 1");
    if (ep->exclusion != 0 && ep->exclusion != 1) fail(DWP_EINVAL, "exclusion must be 0 or 1");
    if (ep->model == 0) {
        if (!(ep->delta > 0.0) || !std::isfinite(ep->delta)) fail(DWP_EINVAL, "delta must be > 0");
        if (ep->exclusion && (!(ep->delta_z > 0.0) || !std::isfinite(ep->z_lim)))
            fail(DWP_EINVAL, "exclusion needs delta_z > 0 and a finite z_lim");
    } else if (ep->model == 1) {
        if (!(ep->beta > 0.5) || !(ep->beta <= 100.0)) fail(DWP_EINVAL, "beta must lie in (0.5, 100]");
        if (!(ep->decay > 0.0) || !std::isfinite(ep->decay)) fail(DWP_EINVAL, "decay must be > 0");
        if (ep->exclusion && !std::isfinite(ep->z_lim)) fail(DWP_EINVAL, "exclusion needs a finite z_lim");
        if (n > GAMMA_MAX_ATOMS) fail(DWP_EINVAL, "model 1 takes at most 4096 atoms");
        const Plan &p = c->plan;
        const double hd = 0.5 * std::sqrt(p.L[0] * p.L[0] + p.L[1] * p.L[1] + p.L[2] * p.L[2]);
        if (!(hd < 600.0 * ep->decay)) fail(DWP_EINVAL, "the half-diagonal of the cell must be below 600 decay lengths");
    } else {
        fail(DWP_EINVAL, "model must be 0 or 1");
    }
}

// Packs atoms (x, y, z wrapped into the cell) into the context's device
// buffer, or into dst (8 n doubles on the device) when given.
void upload_atoms(dwp_ctx *c, int n, const double *xyz, const double *radius, const double *q,
                  const double *sigma, const dwp_eps_params *ep, double *dst = nullptr) {
    const Plan &p = c->plan;
    if (n < 1 || n > 1000000) fail(DWP_EINVAL, "atom count out of range");
    if (!xyz) fail(DWP_EINVAL, "xyz is NULL");
    std::vector<double> rec((size_t)n * 8, 0.0);
    const double Lmin = std::min(p.L[0], std::min(p.L[1], p.L[2]));
    for (int a = 0; a < n; ++a) {
        for (int d = 0; d < 3; ++d) {
            const double v = xyz[3 * a + d];
            if (!std::isfinite(v)) fail(DWP_ENONFINITE, "atom coordinate is not finite");
            double w = std::fmod(v, p.L[d]);
            if (w < 0) w += p.L[d];
            rec[8 * a + d] = w;
        }
        if (radius) {
            if (!(radius[a] > 0.0) || !std::isfinite(radius[a])) fail(DWP_EINVAL, "radius must be > 0");
            if (ep && ep->model == 0 && 2.0 * (radius[a] + 6.0 * ep->delta) >= Lmin)
                fail(DWP_EINVAL, "switch cutoff r + 6 delta must be below half the cell");
            rec[8 * a + 3] = radius[a];
        }
        if (q) {
            if (!std::isfinite(q[a])) fail(DWP_ENONFINITE, "charge is not finite");
            rec[8 * a + 4] = q[a];
        }
        if (sigma) {
            if (!(sigma[a] > 0.0) || !std::isfinite(sigma[a])) fail(DWP_EINVAL, "sigma must be > 0");
            if (18.0 * sigma[a] >= Lmin) fail(DWP_EINVAL, "Gaussian cutoff 9 sigma must be below half the cell");
            rec[8 * a + 5] = sigma[a];
        }
        rec[8 * a + 6] = (ep && ep->exclusion && xyz[3 * a + 2] <= ep->z_lim) ? 1.0 : 0.0;
    }
    if (!dst) {
        c->atoms.alloc(sizeof(double) * rec.size());
        dst = c->atoms.as<double>();
    }
    DWP_HIP(hipMemcpyAsync(dst, rec.data(), sizeof(double) * rec.size(), hipMemcpyHostToDevice, c->stream));
    sync(c);  // rec goes out of scope
    c->atom_rec.swap(rec);
}

// The switch geometry (wrapped positions, radii, buried flags) and the eps
// parameters of an upload, as a flat list for comparison with the eps build.
std::vector<double> switch_geometry(const dwp_ctx *c, const dwp_eps_params *ep) {
    std::vector<double> g;
    const size_t n = c->atom_rec.size() / 8;
    g.reserve(5 * n + 5);
    for (size_t a = 0; a < n; ++a)
        for (int d : {0, 1, 2, 3, 6}) g.push_back(c->atom_rec[8 * a + d]);
    g.insert(g.end(), {ep->eps_inf, ep->delta, (double)ep->exclusion, ep->z_lim, ep->delta_z, (double)ep->model,
                       ep->beta, ep->decay});
    return g;
}

void validate_grid(int nx, int ny, int nz, double Lx, double Ly, double Lz) {
    if (!good_size(nx) || !good_size(ny) || !good_size(nz))
        fail(DWP_EINVAL, "each grid size must be even, in [8, 4096], with prime factors 2 and 3 only");
    if (!(Lx > 0) || !(Ly > 0) || !(Lz > 0) || !std::isfinite(Lx) || !std::isfinite(Ly) || !std::isfinite(Lz))
        fail(DWP_EINVAL, "cell lengths must be positive and finite");
}

void set_grid_impl(dwp_ctx *c, int nx, int ny, int nz, double Lx, double Ly, double Lz, const dwp_opts *o) {
    validate_grid(nx, ny, nz, Lx, Ly, Lz);
    dwp_opts opts;
    if (o) opts = *o;
    else dwp_default_opts(&opts);
    validate_opts(opts);
    c->have_grid = c->have_eps = c->have_solution = false;
    c->first_cycle_red = -1.0;
    free_levels(c);
    Plan &p = c->plan;
    p.nx = nx; p.ny = ny; p.nz = nz;
    p.L[0] = Lx; p.L[1] = Ly; p.L[2] = Lz;
    p.h[0] = Lx / nx; p.h[1] = Ly / ny; p.h[2] = Lz / nz;
    p.N = (size_t)nx * ny * nz;
    p.nkx = nx / 2 + 1;
    p.ldc = (p.nkx + 7) / 8 * 8;
    c->opts = opts;
    c->prof.on = opts.profile != 0;
    c->prof.only = opts.profile == 2 ? PG_RBGS_FINE : -1;
    plan_wet(c);
    const size_t N = p.N;
    const size_t d = sizeof(double);
    c->eps.alloc(d * N); c->sinv.alloc(d * N); c->b.alloc(d * N); c->r.alloc(d * N);
    c->w.alloc(d * N); c->phi_last.alloc(d * N); c->gbuf.alloc(d * N);
    c->V.alloc(d * N * (opts.restart + 1));
    c->Z.alloc(d * N * opts.restart);
    if (opts.krylov_fp32) c->V32.alloc(sizeof(float) * N * (opts.restart + 1));
    c->cbuf.alloc(sizeof(double2) * (size_t)p.ldc * ny * nz);
    c->Hz.alloc(d * nz);
    c->partial.alloc(d * (size_t)RED_BLOCKS * 80);
    c->coef.alloc(d * (HESS_OFFSET + HESS_STRIDE * 64));
    plan_fft(c);
    ensure_levels(c);
    c->have_grid = true;
}

void set_opts_impl(dwp_ctx *c, const dwp_opts *o) {
    need_grid(c);
    if (!o) fail(DWP_EINVAL, "opts is NULL");
    validate_opts(*o);
    const dwp_opts old = c->opts;
    c->opts = *o;
    c->prof.on = o->profile != 0;
    c->prof.only = o->profile == 2 ? PG_RBGS_FINE : -1;
    try {
        if (o->restart > old.restart) {
            c->V.alloc(sizeof(double) * c->plan.N * (o->restart + 1));
            c->Z.alloc(sizeof(double) * c->plan.N * o->restart);
        }
        if (o->krylov_fp32) c->V32.alloc(sizeof(float) * c->plan.N * (o->restart + 1));
        const bool replan = o->z_wet_lo != old.z_wet_lo || o->z_wet_hi != old.z_wet_hi ||
                            o->max_levels != old.max_levels || o->semi_ratio != old.semi_ratio ||
                            (std::isnan(o->z_wet_lo) != std::isnan(old.z_wet_lo)) ||
                            (std::isnan(o->z_wet_hi) != std::isnan(old.z_wet_hi));
        if (replan) plan_wet(c);
        ensure_levels(c);
        if (o->order != c->fft_order) plan_fft(c);
        if (c->have_eps) prepare_eps(c);
        if (o->order != old.order) c->have_solution = false;
    } catch (...) {
        c->opts = old;
        c->prof.on = old.profile != 0;
        c->prof.only = old.profile == 2 ? PG_RBGS_FINE : -1;
        throw;
    }
}

void set_epsilon_impl(dwp_ctx *c, const double *eps_dev) {
    need_grid(c);
    if (!eps_dev) fail(DWP_EINVAL, "eps_dev is NULL");
    int *flags = reinterpret_cast<int *>(c->partial.as<double>());
    launch_check_eps(c->stream, eps_dev, c->plan.N, flags);
    DWP_HIP(hipMemcpyAsync(c->host, flags, sizeof(int) * RED_BLOCKS, hipMemcpyDeviceToHost, c->stream));
    sync(c);
    const int *hf = reinterpret_cast<const int *>(c->host);
    int f = 0;
    for (int b = 0; b < RED_BLOCKS; ++b) f |= hf[b];
    if (f & 1) fail(DWP_ENONFINITE, "eps holds NaN or Inf");
    if (f & 2) fail(DWP_EINVAL, "eps must be >= 1 everywhere");
    DWP_HIP(hipMemcpyAsync(c->eps.p, eps_dev, sizeof(double) * c->plan.N, hipMemcpyDeviceToDevice, c->stream));
    prepare_eps(c);
    c->have_eps = true;
    c->have_solution = false;
    c->eps_natoms = -1;
    c->eps_exclusion = false;
    c->eps_geometry.clear();
    c->eps_density = false;
}

void build_epsilon_density_impl(dwp_ctx *c, const double *rho_e, double eps_inf, double rho0, double beta) {
    need_grid(c);
    if (!rho_e) fail(DWP_EINVAL, "rho_dev is NULL");
    if (!(eps_inf >= 1.0) || !std::isfinite(eps_inf)) fail(DWP_EINVAL, "eps_inf must be finite and >= 1");
    if (!(rho0 > 0.0) || !std::isfinite(rho0)) fail(DWP_EINVAL, "rho0 must be finite and > 0");
    if (!(beta > 0.5) || !(beta <= 1000.0)) fail(DWP_EINVAL, "beta must lie in (0.5, 1000]");
    check_finite_dev(c, rho_e, "rho");
    c->S.alloc(sizeof(double) * c->plan.N);
    PROF(c, PG_BUILD, 24.0 * c->plan.N,
         launch_eps_density(c->stream, rho_e, c->eps.as<double>(), c->S.as<double>(), c->plan.N, eps_inf, rho0,
                            beta));
    prepare_eps(c);
    c->have_eps = true;
    c->have_solution = false;
    c->eps_natoms = -1;
    c->eps_exclusion = false;
    c->eps_geometry.clear();
    c->eps_density = true;
}

void build_epsilon_impl(dwp_ctx *c, int n, const double *xyz, const double *radius, const dwp_eps_params *ep) {
    need_grid(c);
    validate_eps_params(c, n, ep);
    if (!radius) fail(DWP_EINVAL, "radius is NULL");
    upload_atoms(c, n, xyz, radius, nullptr, nullptr, ep);
    AtomParams ap = atom_params(ep);
    c->S.alloc(sizeof(double) * c->plan.N * (ep->model == 1 ? 2 : 1));
    PROF(c, PG_BUILD, (ep->model == 1 ? 24.0 : 16.0) * c->plan.N,
         launch_build_eps(c->stream, c->plan, n, c->atoms.as<double>(), ap, c->Hz.as<double>(), c->eps.as<double>(),
                          c->S.as<double>()));
    c->eps_geometry = switch_geometry(c, ep);
    prepare_eps(c);
    c->have_eps = true;
    c->have_solution = false;
    c->eps_natoms = n;
    c->eps_exclusion = ep->exclusion != 0;
    c->eps_density = false;
}

void solve_impl(dwp_ctx *c, const double *rho, double *phi, double *energy, dwp_info *info) {
    need_eps(c);
    if (!rho || !phi) fail(DWP_EINVAL, "rho_dev and phi_dev must not be NULL");
    Plan &p = c->plan;
    hipStream_t s = c->stream;
    const size_t N = p.N;
    double *coef = c->coef.as<double>();
    double *part = c->partial.as<double>();
    const auto t0 = std::chrono::steady_clock::now();
    check_finite_dev(c, rho, "rho");
    if (c->opts.warm_start) check_finite_dev(c, phi, "the initial phi");
    launch_sum(s, rho, N, part, coef + 400);
    launch_rhs(s, rho, coef + 400, 1.0 / (double)N, c->b.as<double>(), N);
    launch_dot(s, c->b.as<double>(), c->b.as<double>(), N, part, coef + 401);
    DWP_HIP(hipMemcpyAsync(c->host, coef + 400, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    sync(c);
    c->mean_rho = c->host[0] / (double)N;
    const double bnorm = std::sqrt(c->host[1]);
    if (!c->opts.warm_start) launch_fill(s, phi, 0.0, N);
    int iters = 0, restarts = 0;
    double rel = 0.0;
    int status = DWP_OK;
    double t_ph[PH_COUNT] = {0.0, 0.0, 0.0};
    if (bnorm > 0.0) {
        c->phases.start();
        c->phases.mark(s, PH_KRYLOV);
        try {
            iters = fgmres(c, c->b.as<double>(), bnorm, phi, &restarts, &rel);
        } catch (...) {
            c->phases.on = false;
            throw;
        }
        c->phases.mark(s, PH_KRYLOV);
        sync(c);
        c->phases.finish(t_ph);
        if (rel > c->opts.tol) status = DWP_ENOCONV;
    } else {
        launch_fill(s, phi, 0.0, N);
    }
    // gauge: zero mean
    launch_sum(s, phi, N, part, coef + 402);
    launch_sub_mean(s, phi, coef + 402, 1.0 / (double)N, N);
    launch_energy(s, p, rho, phi, c->eps.as<double>(), part, coef + 403);
    DWP_HIP(hipMemcpyAsync(c->phi_last.p, phi, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    c->background = 0.0;
    if (c->opts.order == 6) {
        // c = mean(b - A6 phi) = -mean(A6 phi)
        launch_apply6(s, p, phi, c->eps.as<double>(), c->G6.as<double>(), nullptr, c->w.as<double>(), false, false);
        launch_sum(s, c->w.as<double>(), N, part, coef + 405);
        to_host(c, coef + 405, 1);
        c->background = -c->host[0] / (double)N;
    }
    to_host(c, coef + 403, 2);
    const double h3 = p.h[0] * p.h[1] * p.h[2];
    const double E = 0.5 * h3 * c->host[0];
    const double Eeps = h3 / (8.0 * 3.14159265358979323846) * c->host[1];
    c->have_solution = true;
    c->have_adjoint = false;
    if (energy) *energy = E;
    if (info) {
        info->outer_iters = iters;
        info->vcycles = iters * c->opts.cycles;
        info->restarts = restarts;
        info->k_w0 = p.k_w0;
        info->k_w1 = p.k_w1;
        info->n_levels = (int)p.levels.size();
        info->rel_res = rel;
        info->energy = E;
        info->energy_eps_form = Eeps;
        info->mean_rho_removed = c->mean_rho;
        info->background = c->background;
        info->t_total_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        info->t_fft_ms = t_ph[PH_FFT];
        info->t_mg_ms = t_ph[PH_MG];
        info->t_krylov_ms = t_ph[PH_KRYLOV];
    }
    if (status != DWP_OK) fail(status, "tolerance not reached within max_outer iterations");
}

// Order 6: the zero-mean lambda with Q A6^T lambda = h^3/2 Q rho, by the same
// FGMRES with the transposed operator (the right-hand side is -h^3/(8 pi) b).
void ensure_adjoint(dwp_ctx *c) {
    if (c->opts.order != 6 || c->have_adjoint) return;
    Plan &p = c->plan;
    hipStream_t s = c->stream;
    const size_t N = p.N;
    double *coef = c->coef.as<double>();
    double *part = c->partial.as<double>();
    c->lam.alloc(sizeof(double) * N);
    c->adj_rhs.alloc(sizeof(double) * N);
    const double h3 = p.h[0] * p.h[1] * p.h[2];
    // adj_rhs = scale * b with scale = -h^3 / (8 pi): a multi-axpy with one vector
    c->host[0] = -h3 / (8.0 * 3.14159265358979323846);
    DWP_HIP(hipMemcpyAsync(coef + 406, c->host, sizeof(double), hipMemcpyHostToDevice, s));
    launch_fill(s, c->adj_rhs.as<double>(), 0.0, N);
    launch_axpy_multi(s, c->adj_rhs.as<double>(), c->b.as<double>(), N, 1, coef + 406, N, 1.0, part, nullptr);
    launch_dot(s, c->adj_rhs.as<double>(), c->adj_rhs.as<double>(), N, part, coef + 407);
    to_host(c, coef + 407, 1);
    const double fnorm = std::sqrt(c->host[0]);
    // initial guess: the adjoint of the symmetric part, -h^3 phi / (8 pi) (the
    // same scale as the right-hand side; exact for a symmetric operator)
    launch_fill(s, c->lam.as<double>(), 0.0, N);
    launch_axpy_multi(s, c->lam.as<double>(), c->phi_last.as<double>(), N, 1, coef + 406, N, 1.0, part, nullptr);
    if (fnorm > 0.0) {
        int restarts = 0;
        double rel = 0.0;
        c->transposed = true;
        try {
            fgmres(c, c->adj_rhs.as<double>(), fnorm, c->lam.as<double>(), &restarts, &rel);
        } catch (...) {
            c->transposed = false;
            throw;
        }
        c->transposed = false;
        if (rel > c->opts.tol) fail(DWP_ENOCONV, "adjoint solve: tolerance not reached within max_outer iterations");
        launch_sum(s, c->lam.as<double>(), N, part, coef + 408);
        launch_sub_mean(s, c->lam.as<double>(), coef + 408, 1.0 / (double)N, N);
    }
    c->have_adjoint = true;
}

// Vector-Jacobian product of (rho, eps) -> (phi, E) at the solution phi of
// the current eps (order 2).  The adjoint problem A lambda = g_phi - mean
// runs through the same FGMRES as the solve, on buffers of its own, so the
// last solution (phi_last, b) stays what dwp_solve left.
void backward_impl(dwp_ctx *c, const double *phi, double gE, const double *gphi, double *grad_rho,
                   double *grad_eps, dwp_info *info) {
    need_eps(c);
    if (c->opts.order != 2) fail(DWP_EINVAL, "dwp_backward needs the symmetric second-order operator (order 2)");
    if (!phi || !grad_rho || !grad_eps) fail(DWP_EINVAL, "phi_dev, grad_rho_dev and grad_eps_dev must not be NULL");
    if (!std::isfinite(gE)) fail(DWP_EINVAL, "g_E must be finite");
    Plan &p = c->plan;
    hipStream_t s = c->stream;
    const size_t N = p.N;
    double *coef = c->coef.as<double>();
    double *part = c->partial.as<double>();
    const auto t0 = std::chrono::steady_clock::now();
    check_finite_dev(c, phi, "phi");
    const double h3 = p.h[0] * p.h[1] * p.h[2];
    const double four_pi = 4.0 * 3.14159265358979323846;
    int iters = 0, restarts = 0, status = DWP_OK;
    double rel = 0.0;
    double t_ph[PH_COUNT] = {0.0, 0.0, 0.0};
    const double *lam = nullptr;
    if (gphi) {
        check_finite_dev(c, gphi, "g_phi");
        c->bw_rhs.alloc(sizeof(double) * N);
        c->bw_lam.alloc(sizeof(double) * N);
        double *rhs = c->bw_rhs.as<double>(), *x = c->bw_lam.as<double>();
        launch_sum(s, gphi, N, part, coef + 420);
        launch_axpby(s, rhs, 1.0, gphi, 0.0, nullptr, N);
        launch_sub_mean(s, rhs, coef + 420, 1.0 / (double)N, N);
        launch_dot(s, rhs, rhs, N, part, coef + 421);
        to_host(c, coef + 421, 1);
        const double bnorm = std::sqrt(c->host[0]);
        launch_fill(s, x, 0.0, N);
        if (bnorm > 0.0) {
            c->phases.start();
            c->phases.mark(s, PH_KRYLOV);
            try {
                iters = fgmres(c, rhs, bnorm, x, &restarts, &rel);
            } catch (...) {
                c->phases.on = false;
                throw;
            }
            c->phases.mark(s, PH_KRYLOV);
            sync(c);
            c->phases.finish(t_ph);
            if (rel > c->opts.tol) status = DWP_ENOCONV;
            launch_sum(s, x, N, part, coef + 422);
            launch_sub_mean(s, x, coef + 422, 1.0 / (double)N, N);
        }
        lam = x;
    }
    // grad_rho = g_E h^3 phi - 4 pi lambda
    launch_axpby(s, grad_rho, gE * h3, phi, -four_pi, lam, N);
    // grad_eps = G(u, phi), u = lambda - g_E h^3 / (8 pi) phi (G is bilinear)
    double *u = c->w.as<double>();
    launch_axpby(s, u, -gE * h3 / (2.0 * four_pi), phi, 1.0, lam, N);
    PROF(c, PG_FORCES, 24.0 * N, launch_eps_pair(s, p, u, phi, 1.0, grad_eps));
    sync(c);
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->outer_iters = iters;
        info->vcycles = iters * c->opts.cycles;
        info->restarts = restarts;
        info->k_w0 = p.k_w0;
        info->k_w1 = p.k_w1;
        info->n_levels = (int)p.levels.size();
        info->rel_res = rel;
        info->t_total_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        info->t_fft_ms = t_ph[PH_FFT];
        info->t_mg_ms = t_ph[PH_MG];
        info->t_krylov_ms = t_ph[PH_KRYLOV];
    }
    if (status != DWP_OK) fail(status, "adjoint solve: tolerance not reached within max_outer iterations");
}

// dE/d eps for the last solution, for the operator of the options
void eps_gradient_impl(dwp_ctx *c, double *g) {
    if (c->opts.order == 6) {
        ensure_adjoint(c);
        PROF(c, PG_FORCES, 24.0 * c->plan.N,
             launch_grad6(c->stream, c->plan, c->phi_last.as<double>(), c->lam.as<double>(), g));
    } else {
        PROF(c, PG_FORCES, 16.0 * c->plan.N, launch_eps_gradient(c->stream, c->plan, c->phi_last.as<double>(), g));
    }
}

// The potential whose h^3 multiple is dE/d rho: phi (order 2), phi/2 - 4 pi lambda / h^3 (order 6).
const double *charge_potential(dwp_ctx *c) {
    if (c->opts.order != 6) return c->phi_last.as<double>();
    ensure_adjoint(c);
    launch_charge_potential(c->stream, c->plan, c->phi_last.as<double>(), c->lam.as<double>(), c->w.as<double>());
    return c->w.as<double>();
}

void forces_impl(dwp_ctx *c, int n, const double *xyz, const double *radius, const double *q,
                 const double *sigma, const dwp_eps_params *ep, double *out) {
    need_eps(c);
    if (!c->have_solution) fail(DWP_ESTATE, "no solution: call dwp_solve first");
    if (!q || !sigma || !out) fail(DWP_EINVAL, "q, sigma and dEdR must not be NULL");
    if (ep) {
        validate_eps_params(c, n, ep);
        if (!radius) fail(DWP_EINVAL, "radius is NULL");
        if (c->eps_natoms != n) fail(DWP_ESTATE, "eps was not built from these atoms");
        if ((ep->exclusion != 0) != c->eps_exclusion) fail(DWP_ESTATE, "exclusion differs from the eps build");
    }
    upload_atoms(c, n, xyz, ep ? radius : nullptr, q, sigma, ep);
    // the switch term divides the switch product S stored by the eps build
    if (ep && switch_geometry(c, ep) != c->eps_geometry)
        fail(DWP_ESTATE, "positions, radii or eps parameters differ from the last dwp_build_epsilon");
    Plan &p = c->plan;
    AtomParams ap{};
    if (ep) ap = atom_params(ep);
    eps_gradient_impl(c, c->gbuf.as<double>());
    const double *pot = charge_potential(c);
    const int model = ep ? ep->model : 0;
    c->fpart.alloc(sizeof(double) * (forces_partial_len(p, n, model) + 3 * (size_t)n));
    double *outd = c->fpart.as<double>() + forces_partial_len(p, n, model);
    PROF(c, PG_FORCES, 16.0 * p.N,
         launch_forces(c->stream, p, n, c->atoms.as<double>(), ep ? &ap : nullptr, pot, c->gbuf.as<double>(),
                       c->S.as<double>(), c->Hz.as<double>(), c->fpart.as<double>(), outd));
    DWP_HIP(hipMemcpyAsync(out, outd, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c->stream));
    sync(c);
}

thread_local std::string g_create_err;

}  // namespace
}  // namespace dwp

// Device scratch of dwp_forces_noalloc: every GPU the library runs on holds its
// own copy until the process ends.  Host code never passes this name to a
// kernel or a copy (on the host it is only a stand-in for the symbol): it uses
// the device address resolved once per device by resolve_scratch().
constexpr size_t NOALLOC_SCRATCH_DOUBLES = (size_t)1 << 21;  // 16 MiB
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace dwp {
namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[MAX_DEVICES] = {nullptr};

// The device address of `scratch` on device `dev`, which must be current.
double *resolve_scratch(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) fail(DWP_EINVAL, "device index out of range for the static scratch");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            fail(DWP_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<double *>(ptr);
    }
    return g_scratch_dev[dev];
}

// dwp_forces with the packed atoms, the force partials and the device copy of
// the result in the static scratch: no device allocation.  Every partial slot
// the force kernels read is written earlier in the same call, so the stale
// contents of the previous call need no clearing.
void forces_noalloc_impl(dwp_ctx *c, int n, const double *xyz, const double *radius, const double *q,
                         const double *sigma, const dwp_eps_params *ep, double *out) {
    need_eps(c);
    if (!c->have_solution) fail(DWP_ESTATE, "no solution: call dwp_solve first");
    if (!q || !sigma || !out) fail(DWP_EINVAL, "q, sigma and dEdR must not be NULL");
    if (c->opts.order != 2)
        fail(DWP_EINVAL, "dwp_forces_noalloc takes the second-order operator only (order 6 needs the adjoint "
                         "solve's buffers)");
    if (n < 1 || n > 1000000) fail(DWP_EINVAL, "atom count out of range");
    if (ep) {
        validate_eps_params(c, n, ep);
        if (!radius) fail(DWP_EINVAL, "radius is NULL");
        if (c->eps_natoms != n) fail(DWP_ESTATE, "eps was not built from these atoms");
        if ((ep->exclusion != 0) != c->eps_exclusion) fail(DWP_ESTATE, "exclusion differs from the eps build");
    }
    const Plan &p = c->plan;
    const int model = ep ? ep->model : 0;
    const size_t plen = forces_partial_len(p, n, model);
    const size_t need = 8 * (size_t)n + plen + 3 * (size_t)n;
    if (need > NOALLOC_SCRATCH_DOUBLES)
        fail(DWP_EINVAL, "dwp_forces_noalloc: " + std::to_string(n) + " atoms need " + std::to_string(need) +
                             " doubles of scratch, the static scratch holds " +
                             std::to_string(NOALLOC_SCRATCH_DOUBLES));
    double *base = g_scratch_dev[c->device];
    if (!base) base = resolve_scratch(c->device);
    double *atoms = base, *fpart = base + 8 * (size_t)n, *outd = fpart + plen;
    upload_atoms(c, n, xyz, ep ? radius : nullptr, q, sigma, ep, atoms);
    if (ep && switch_geometry(c, ep) != c->eps_geometry)
        fail(DWP_ESTATE, "positions, radii or eps parameters differ from the last dwp_build_epsilon");
    AtomParams ap{};
    if (ep) ap = atom_params(ep);
    launch_eps_gradient(c->stream, p, c->phi_last.as<double>(), c->gbuf.as<double>());
    launch_forces(c->stream, p, n, atoms, ep ? &ap : nullptr, c->phi_last.as<double>(), c->gbuf.as<double>(),
                  c->S.as<double>(), c->Hz.as<double>(), fpart, outd);
    DWP_HIP(hipMemcpyAsync(out, outd, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c->stream));
    sync(c);
}

}  // namespace
}  // namespace dwp

// ============================================================== C ABI
using dwp::Error;

#define ABI_BEGIN(c)                                   \
    if (!(c)) return DWP_EINVAL;                       \
    (c)->err.clear();                                  \
    try {
#define ABI_END(c)                                     \
    }                                                  \
    catch (const Error &e) {                           \
        (c)->err = e.msg;                              \
        return e.status;                               \
    }                                                  \
    catch (const std::exception &e) {                  \
        (c)->err = e.what();                           \
        return DWP_EHIP;                               \
    }                                                  \
    return DWP_OK;

extern "C" {

void dwp_default_opts(dwp_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = DWP_FP64;
    o->z_wet_lo = std::numeric_limits<double>::quiet_NaN();
    o->z_wet_hi = std::numeric_limits<double>::quiet_NaN();
    o->pre = 2;
    o->post = 2;
    o->coarse_sweeps = 64;
    o->max_levels = 16;
    o->cycles = 1;
    o->scaled_dry = 0;
    o->tol = 1e-10;
    o->max_outer = 600;
    o->restart = 10;
    o->warm_start = 0;
    o->profile = 0;
    o->smoother = 1;
    o->fft_fp32 = 0;
    o->order = 2;
    o->smooth6 = 0;
    o->krylov_fp32 = 0;
    o->krylov_fp16 = 0;
    o->semi_ratio = std::sqrt(2.0);
}

int dwp_create(dwp_ctx **out, int device, void *stream) {
    if (!out) return DWP_EINVAL;
    *out = nullptr;
    dwp_ctx *c = new dwp_ctx();
    try {
        int count = 0;
        DWP_HIP(hipGetDeviceCount(&count));
        if (device < 0 || device >= count) dwp::fail(DWP_EINVAL, "no such HIP device");
        DWP_HIP(hipSetDevice(device));
        c->device = device;
        c->stream = static_cast<hipStream_t>(stream);
        c->host_len = 8192;
        DWP_HIP(hipHostMalloc(reinterpret_cast<void **>(&c->host), sizeof(double) * c->host_len, hipHostMallocDefault));
        // the static scratch's address on this device, once per device
        if (device < dwp::MAX_DEVICES && !dwp::g_scratch_dev[device]) dwp::resolve_scratch(device);
        dwp_default_opts(&c->opts);
    } catch (const Error &e) {
        dwp::g_create_err = e.msg;
        if (c->host) (void)hipHostFree(c->host);
        delete c;
        return e.status;
    }
    *out = c;
    return DWP_OK;
}

int dwp_destroy(dwp_ctx *c) {
    if (!c) return DWP_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    dwp::free_levels(c);
    if (c->host) (void)hipHostFree(c->host);
    delete c;
    return DWP_OK;
}

int dwp_set_stream(dwp_ctx *c, void *stream) {
    ABI_BEGIN(c)
    c->stream = static_cast<hipStream_t>(stream);
    ABI_END(c)
}

int dwp_set_grid(dwp_ctx *c, int nx, int ny, int nz, double Lx, double Ly, double Lz, const dwp_opts *o) {
    ABI_BEGIN(c)
    DWP_HIP(hipSetDevice(c->device));
    dwp::set_grid_impl(c, nx, ny, nz, Lx, Ly, Lz, o);
    ABI_END(c)
}

int dwp_set_opts(dwp_ctx *c, const dwp_opts *o) {
    ABI_BEGIN(c)
    DWP_HIP(hipSetDevice(c->device));
    dwp::set_opts_impl(c, o);
    ABI_END(c)
}

int dwp_set_epsilon(dwp_ctx *c, const double *eps_dev) {
    ABI_BEGIN(c)
    DWP_HIP(hipSetDevice(c->device));
    dwp::set_epsilon_impl(c, eps_dev);
    ABI_END(c)
}

int dwp_build_epsilon(dwp_ctx *c, int n, const double *xyz, const double *radius, const dwp_eps_params *ep) {
    ABI_BEGIN(c)
    DWP_HIP(hipSetDevice(c->device));
    dwp::build_epsilon_impl(c, n, xyz, radius, ep);
    ABI_END(c)
}

int dwp_get_epsilon(dwp_ctx *c, double *eps_dev) {
    ABI_BEGIN(c)
    dwp::need_eps(c);
    if (!eps_dev) dwp::fail(DWP_EINVAL, "eps_dev is NULL");
    DWP_HIP(hipSetDevice(c->device));
    DWP_HIP(hipMemcpyAsync(eps_dev, c->eps.p, sizeof(double) * c->plan.N, hipMemcpyDeviceToDevice, c->stream));
    ABI_END(c)
}

int dwp_build_rho(dwp_ctx *c, int n, const double *xyz, const double *q, const double *sigma, double *rho_dev) {
    ABI_BEGIN(c)
    dwp::need_grid(c);
    if (!q || !sigma || !rho_dev) dwp::fail(DWP_EINVAL, "q, sigma and rho_dev must not be NULL");
    DWP_HIP(hipSetDevice(c->device));
    dwp::upload_atoms(c, n, xyz, nullptr, q, sigma, nullptr);
    PROF(c, dwp::PG_BUILD, 8.0 * c->plan.N, dwp::launch_build_rho(c->stream, c->plan, n, c->atoms.as<double>(), rho_dev));
    ABI_END(c)
}

int dwp_solve(dwp_ctx *c, const double *rho, double *phi, double *energy, dwp_info *info) {
    ABI_BEGIN(c)
    DWP_HIP(hipSetDevice(c->device));
    dwp::solve_impl(c, rho, phi, energy, info);
    ABI_END(c)
}

int dwp_backward(dwp_ctx *c, const double *phi, double gE, const double *gphi, double *grad_rho,
                 double *grad_eps, dwp_info *info) {
    ABI_BEGIN(c)
    DWP_HIP(hipSetDevice(c->device));
    dwp::backward_impl(c, phi, gE, gphi, grad_rho, grad_eps, info);
    ABI_END(c)
}

int dwp_eps_gradient(dwp_ctx *c, double *g) {
    ABI_BEGIN(c)
    dwp::need_eps(c);
    if (!c->have_solution) dwp::fail(DWP_ESTATE, "no solution: call dwp_solve first");
    if (!g) dwp::fail(DWP_EINVAL, "dEdeps_dev is NULL");
    DWP_HIP(hipSetDevice(c->device));
    dwp::eps_gradient_impl(c, g);
    ABI_END(c)
}

int dwp_build_epsilon_density(dwp_ctx *c, const double *rho_dev, double eps_inf, double rho0, double beta) {
    ABI_BEGIN(c)
    DWP_HIP(hipSetDevice(c->device));
    dwp::build_epsilon_density_impl(c, rho_dev, eps_inf, rho0, beta);
    ABI_END(c)
}

int dwp_v_eps(dwp_ctx *c, int add_phi, double *out) {
    ABI_BEGIN(c)
    dwp::need_eps(c);
    if (!c->eps_density) dwp::fail(DWP_ESTATE, "eps was not built from a density: call dwp_build_epsilon_density");
    if (!c->have_solution) dwp::fail(DWP_ESTATE, "no solution: call dwp_solve first");
    if (add_phi != 0 && add_phi != 1) dwp::fail(DWP_EINVAL, "add_phi must be 0 or 1");
    if (!out) dwp::fail(DWP_EINVAL, "out_dev is NULL");
    DWP_HIP(hipSetDevice(c->device));
    if (c->opts.order == 6) {
        dwp::eps_gradient_impl(c, c->gbuf.as<double>());
        const double *pot = add_phi ? dwp::charge_potential(c) : nullptr;
        dwp::launch_scaled_product(c->stream, c->plan, c->gbuf.as<double>(), c->S.as<double>(), pot, out);
    } else {
        PROF(c, dwp::PG_FORCES, 24.0 * c->plan.N,
             dwp::launch_v_eps(c->stream, c->plan, c->phi_last.as<double>(), c->S.as<double>(), add_phi != 0, out));
    }
    ABI_END(c)
}

int dwp_eps_pair_gradient(dwp_ctx *c, const double *a, const double *b, double scale, double *out) {
    ABI_BEGIN(c)
    dwp::need_grid(c);
    if (!a || !b || !out) dwp::fail(DWP_EINVAL, "NULL pointer");
    if (!std::isfinite(scale)) dwp::fail(DWP_EINVAL, "scale must be finite");
    DWP_HIP(hipSetDevice(c->device));
    PROF(c, dwp::PG_FORCES, 24.0 * c->plan.N, dwp::launch_eps_pair(c->stream, c->plan, a, b, scale, out));
    ABI_END(c)
}

int dwp_forces(dwp_ctx *c, int n, const double *xyz, const double *radius, const double *q, const double *sigma,
               const dwp_eps_params *ep, double *out) {
    ABI_BEGIN(c)
    DWP_HIP(hipSetDevice(c->device));
    dwp::forces_impl(c, n, xyz, radius, q, sigma, ep, out);
    ABI_END(c)
}

int dwp_forces_noalloc(dwp_ctx *c, int n, const double *xyz, const double *radius, const double *q,
                       const double *sigma, const dwp_eps_params *ep, double *out) {
    ABI_BEGIN(c)
    DWP_HIP(hipSetDevice(c->device));
    dwp::forces_noalloc_impl(c, n, xyz, radius, q, sigma, ep, out);
    ABI_END(c)
}

int dwp_apply_operator(dwp_ctx *c, const double *phi, double *out) {
    ABI_BEGIN(c)
    dwp::need_eps(c);
    if (!phi || !out) dwp::fail(DWP_EINVAL, "NULL pointer");
    DWP_HIP(hipSetDevice(c->device));
    if (c->opts.order == 6)
        dwp::launch_apply6(c->stream, c->plan, phi, c->eps.as<double>(), c->G6.as<double>(), nullptr, out, false,
                           false);
    else
        dwp::launch_apply_full(c->stream, c->plan, phi, c->eps.as<double>(), nullptr, out, false);
    ABI_END(c)
}

int dwp_vacuum_solve(dwp_ctx *c, const double *r, double *out) {
    ABI_BEGIN(c)
    dwp::need_grid(c);
    if (!r || !out) dwp::fail(DWP_EINVAL, "NULL pointer");
    DWP_HIP(hipSetDevice(c->device));
    dwp::launch_vacuum_solve(c->stream, c->plan, c->fx, c->fy, c->fz, r, nullptr, c->cbuf.p, out,
                             nullptr, c->opts.fft_fp32 != 0);
    ABI_END(c)
}

int dwp_apply_split(dwp_ctx *c, const double *r, double *out) {
    ABI_BEGIN(c)
    dwp::need_eps(c);
    if (!r || !out) dwp::fail(DWP_EINVAL, "NULL pointer");
    DWP_HIP(hipSetDevice(c->device));
    dwp::apply_split(c, r, out);
    ABI_END(c)
}

int dwp_energy(dwp_ctx *c, const double *rho, const double *phi, double *e) {
    ABI_BEGIN(c)
    dwp::need_eps(c);
    if (!rho || !phi || !e) dwp::fail(DWP_EINVAL, "NULL pointer");
    DWP_HIP(hipSetDevice(c->device));
    double *coef = c->coef.as<double>();
    dwp::launch_energy(c->stream, c->plan, rho, phi, c->eps.as<double>(), c->partial.as<double>(), coef + 403);
    dwp::to_host(c, coef + 403, 1);
    const dwp::Plan &p = c->plan;
    *e = 0.5 * p.h[0] * p.h[1] * p.h[2] * c->host[0];
    ABI_END(c)
}

int dwp_profile_count(void) { return dwp::PG_COUNT; }

int dwp_profile_get(dwp_ctx *c, int g, const char **name, double *ms, long *launches, double *bytes) {
    ABI_BEGIN(c)
    if (g < 0 || g >= dwp::PG_COUNT) dwp::fail(DWP_EINVAL, "no such profile group");
    DWP_HIP(hipSetDevice(c->device));
    dwp::sync(c);
    if (name) *name = dwp::prof_group_name(g);
    if (ms) *ms = c->prof.ms[g];
    if (launches) *launches = c->prof.launches[g];
    if (bytes) *bytes = c->prof.bytes[g];
    ABI_END(c)
}

int dwp_profile_reset(dwp_ctx *c) {
    ABI_BEGIN(c)
    DWP_HIP(hipSetDevice(c->device));
    dwp::sync(c);
    c->prof.reset();
    ABI_END(c)
}

int dwp_plan(int nx, int ny, int nz, double Lx, double Ly, double Lz, const dwp_opts *o, int *out, int out_len) {
    try {
        dwp::g_create_err.clear();
        dwp::validate_grid(nx, ny, nz, Lx, Ly, Lz);
        dwp_opts opts;
        if (o) opts = *o;
        else dwp_default_opts(&opts);
        dwp::validate_opts(opts);
        const double L[3] = {Lx, Ly, Lz};
        const double h[3] = {Lx / nx, Ly / ny, Lz / nz};
        int k0, k1, nw;
        dwp::choose_wet(nx, ny, nz, h, L, opts, &k0, &k1, &nw);
        const auto lv = dwp::plan_levels(nx, ny, nw, h, opts.max_levels, opts.semi_ratio);
        if (!out || out_len < 3 + 3 * (int)lv.size()) dwp::fail(DWP_EINVAL, "output array too short");
        out[0] = k0;
        out[1] = k1;
        out[2] = (int)lv.size();
        for (size_t l = 0; l < lv.size(); ++l) {
            out[3 + 3 * l] = lv[l].nx;
            out[4 + 3 * l] = lv[l].ny;
            out[5 + 3 * l] = lv[l].nw;
        }
    } catch (const Error &e) {
        dwp::g_create_err = e.msg;
        return e.status;
    }
    return DWP_OK;
}

const char *dwp_last_error(const dwp_ctx *c) {
    if (!c) return dwp::g_create_err.c_str();
    return c->err.c_str();
}

}  // extern "C"
