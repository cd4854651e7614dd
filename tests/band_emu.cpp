// Host stepping of the row-band red-black sweep: every thread of every block
// runs the kernel's own per-thread code (band_sweep.h) in plain C++, each
// global and LDS access is checked against its buffer, and the output is
// compared with two in-place colour passes.  Threads of a step run in both
// orders, which must agree: no thread may read, within one step, a value
// another thread writes in it (the kernel has one barrier per step).
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <vector>
#include <random>
#include <algorithm>
#define __host__
#define __device__
#define __forceinline__ inline
#include <limits>
#define BAND_CHECK(i, n) do { if (!((size_t)(i) < (size_t)(n))) { fprintf(stderr, "OOB %s:%d %zu >= %zu\n", __FILE__, __LINE__, (size_t)(i), (size_t)(n)); abort(); } } while (0)
// the device divides by the hardware reciprocal; here plain division (the
// comparison below is with colour passes that use the same function)
namespace dwp {
inline float gs_value(float off, float f, float diag) { return (off - f) / diag; }
inline double gs_value(double off, double f, double diag) { return (off - f) / diag; }
}
#include "band_sweep.h"
#include "band_apply.h"
#include "band_restrict.h"
using namespace dwp;

// one block: every thread's prologue, then the steps with a barrier between
// them (threads of a step in order, or in reverse)
template <class T, int W, bool ZIN, bool DOWN, int PD>
void march(const BandArgs<T> &a, T *lds, int band, int chunk, int nt, bool reverse) {
    std::vector<BandSweep<T, W, ZIN, DOWN, PD>> th(nt);
    for (int t = 0; t < nt; ++t) { th[t].init(a, lds, band, chunk, t); th[t].prologue(); }
    const int m0 = th[0].first(), n = th[0].nsteps(), D = DOWN ? -1 : 1;
    for (int st = 0; st < n; st += 2) {
        for (int q = 0; q < nt; ++q) th[reverse ? nt - 1 - q : q].template step<0>(m0 + D * st);
        for (int q = 0; q < nt; ++q) th[reverse ? nt - 1 - q : q].template step<1>(m0 + D * (st + 1));
    }
}

template <class T, int W, bool ZIN>
int run(int nx, int ny, int nw, int ty, int kc, int c0, bool reverse, unsigned seed, int nzb = 0, int kw0 = 0) {
    const size_t plane = (size_t)nx * ny;
    // nzb > 0: the sweep adds its output into a box array z of nzb planes at
    // box planes (kw0 + k) mod nzb instead of writing out
    std::vector<T> z((size_t)nzb * plane), z0;
    for (size_t i = 0; i < z.size(); ++i) z[i] = (T)(0.25 * (double)(i % 7) - 0.5);
    z0 = z;
    std::vector<T> u((nw + 2) * plane, T(0)), e((nw + 2) * plane), f(nw * plane), out((nw + 2) * plane, T(0));
    std::mt19937 g(seed);
    std::uniform_real_distribution<double> U(0, 1);
    for (auto &x : e) x = (T)(1.0 + 77.0 * U(g));
    if (!ZIN) for (size_t i = plane; i < (nw + 1) * plane; ++i) u[i] = (T)(U(g) - 0.5);
    for (auto &x : f) x = (T)(10.0 * (U(g) - 0.5));
    const T cx = (T)1.3, cy = (T)0.7, cz = (T)0.4;
    // reference: two colour passes in place on a copy of u
    std::vector<T> ref = u;
    auto at = [&](int i, int j, int k) -> size_t { return (size_t)(k + 1) * plane + (size_t)((j + ny) % ny) * nx + (i + nx) % nx; };
    for (int col = 0; col < 2; ++col) {
        const int cc = col == 0 ? c0 : 1 - c0;
        for (int k = 0; k < nw; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    if (((i + j + k) & 1) != cc) continue;
                    const T e0 = e[at(i, j, k)];
                    ref[at(i, j, k)] = band_point<T>(cx, cy, cz, e0, e[at(i + 1, j, k)], e[at(i - 1, j, k)], e[at(i, j + 1, k)],
                                                     e[at(i, j - 1, k)], e[at(i, j, k + 1)], e[at(i, j, k - 1)],
                                                     ref[at(i + 1, j, k)], ref[at(i - 1, j, k)], ref[at(i, j + 1, k)],
                                                     ref[at(i, j - 1, k)], ref[at(i, j, k + 1)], ref[at(i, j, k - 1)],
                                                     f[(size_t)k * plane + (size_t)j * nx + i]);
                }
    }
    const int bands = ny / ty, nchunks = (nw + kc - 1) / kc, nb = bands * nchunks, nt = (ty + 4) * (nx / W);
    const int gb = bands % 4 == 0 ? 4 : (bands % 2 == 0 ? 2 : 1);
    BandArgs<T> a{u.data(), out.data(), e.data(), f.data(), nx, ny, nw, ty, bands, kc, c0, cx, cy, cz,
                  nzb ? z.data() : nullptr, nzb, kw0};
    std::vector<int> seen(nb, 0);
    for (int t = 0; t < nb; ++t) {
        // the kernel's tile -> (band, chunk) decoding; odd chunks march down
        const int g = t / (gb * nchunks), q = t - g * gb * nchunks;
        const int chunk = q / gb, band = g * gb + (q - (q / gb) * gb);
        BAND_CHECK(band, bands);
        BAND_CHECK(chunk, nchunks);
        ++seen[chunk * bands + band];
        std::vector<T> lds(band_lds_elems(nx, ty), std::numeric_limits<T>::quiet_NaN());
        // both prefetch depths the kernel may use, alternating over the tiles
        if (chunk & 1) {
            if (t & 1) march<T, W, ZIN, true, 1>(a, lds.data(), band, chunk, nt, reverse);
            else march<T, W, ZIN, true, 2>(a, lds.data(), band, chunk, nt, reverse);
        } else {
            if (t & 1) march<T, W, ZIN, false, 2>(a, lds.data(), band, chunk, nt, reverse);
            else march<T, W, ZIN, false, 1>(a, lds.data(), band, chunk, nt, reverse);
        }
    }
    for (int v : seen)
        if (v != 1) { printf("tile mapping is not a bijection\n"); return 1; }
    double md = 0, mref = 0;
    size_t bad = 0;
    if (nzb) {
        // z at the wet planes gained exactly the sweep's result, other box
        // planes and out's interior are untouched, out's zero plane stays zero
        size_t zbad = 0;
        for (int kb = 0; kb < nzb; ++kb)
            for (size_t q = 0; q < plane; ++q) {
                const int k = ((kb - kw0) % nzb + nzb) % nzb;
                const size_t i = (size_t)kb * plane + q;
                const T want = k < nw ? (T)(z0[i] + ref[(size_t)(k + 1) * plane + q]) : z0[i];
                if (!(z[i] == want)) ++zbad;
            }
        for (size_t i = 0; i < out.size(); ++i)
            if (out[i] != T(0)) ++zbad;
        printf("%s W=%d ZIN=%d %dx%dx%d ty=%d kc=%d c0=%d rev=%d added into %d box planes from %d: mismatches %zu\n",
               sizeof(T) == 4 ? "f32" : "f64", W, (int)ZIN, nx, ny, nw, ty, kc, c0, (int)reverse, nzb, kw0, zbad);
        return zbad != 0;
    }
    for (size_t i = 0; i < out.size(); ++i) {
        const bool ghost = i < plane || i >= (nw + 1) * plane;
        const double want = ghost ? 0.0 : (double)ref[i];
        const double d = std::fabs((double)out[i] - want);
        if (!(d <= 0.0)) ++bad;
        if (std::isnan(d)) md = INFINITY; else md = std::max(md, d);
        mref = std::max(mref, std::fabs(want));
    }
    printf("%s W=%d ZIN=%d %dx%dx%d ty=%d kc=%d c0=%d rev=%d: blocks %d threads %d  maxdiff %.3g (max %.3g) mismatches %zu\n",
           sizeof(T) == 4 ? "f32" : "f64", W, (int)ZIN, nx, ny, nw, ty, kc, c0, (int)reverse, nb, nt, md, mref, bad);
    return bad != 0;
}

// The row-band operator (band_apply.h) against the 7-point operator written
// out point by point in float64, on the box (MODE 0, 1) or on wet planes that
// wrap around the periodic z (MODE 2).
template <int MODE, class TS>
int run_apply(int nx, int ny, int nz, int nplanes, int k_w0, int ty, int kc, bool reverse, unsigned seed) {
    const size_t plane = (size_t)nx * ny;
    std::vector<TS> phi(nz * plane), eps(nz * plane), b(nz * plane), out((MODE == 2 ? nplanes : nz) * plane, TS(-7));
    std::mt19937 g(seed);
    std::uniform_real_distribution<double> U(0, 1);
    for (auto &x : phi) x = (TS)(U(g) - 0.5);
    for (auto &x : eps) x = (TS)(1.0 + 77.0 * U(g));
    for (auto &x : b) x = (TS)(U(g) - 0.5);
    const double cx = 1.7, cy = 0.9, cz = 0.35;
    const int bands = ny / ty, nchunks = (nplanes + kc - 1) / kc, nb = bands * nchunks;
    const int W = ApplyVec<TS>::W, nt = (ty + 2) * (nx / W);
    const int gb = bands % 4 == 0 ? 4 : (bands % 2 == 0 ? 2 : 1);
    ApplyArgs<TS, TS> a{phi.data(), eps.data(), b.data(), out.data(), nx, ny, nz, k_w0, nplanes, ty, bands, kc,
                        cx, cy, cz};
    std::vector<int> seen(nb, 0);
    for (int t = 0; t < nb; ++t) {
        const int gg = t / (gb * nchunks), q = t - gg * gb * nchunks;
        const int chunk = q / gb, band = gg * gb + (q - (q / gb) * gb);
        BAND_CHECK(band, bands);
        BAND_CHECK(chunk, nchunks);
        ++seen[chunk * bands + band];
        std::vector<TS> lds(apply_lds_elems(nx, ty), std::numeric_limits<TS>::quiet_NaN());
        std::vector<BandApply<MODE, TS, TS>> th(nt);
        for (int i = 0; i < nt; ++i) { th[i].init(a, lds.data(), band, chunk, i); th[i].prologue(); }
        for (int kk = th[0].kk0; kk < th[0].kk1; ++kk)
            for (int i = 0; i < nt; ++i) th[reverse ? nt - 1 - i : i].step(kk);
    }
    for (int v : seen)
        if (v != 1) { printf("tile mapping is not a bijection\n"); return 1; }
    auto at = [&](int i, int j, int k) -> size_t {
        return (size_t)((k % nz + nz) % nz) * plane + (size_t)((j + ny) % ny) * nx + (i + nx) % nx;
    };
    size_t bad = 0;
    double md = 0;
    for (int kk = 0; kk < (MODE == 2 ? nplanes : nz); ++kk)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int k = MODE == 2 ? k_w0 + kk : kk;
                const double p0 = phi[at(i, j, k)], e0 = eps[at(i, j, k)];
                auto t = [&](int di, int dj, int dk) {
                    return ((double)e0 + (double)eps[at(i + di, j + dj, k + dk)]) * ((double)phi[at(i + di, j + dj, k + dk)] - p0);
                };
                double v = cx * (t(1, 0, 0) + t(-1, 0, 0)) + cy * (t(0, 1, 0) + t(0, -1, 0)) + cz * (t(0, 0, 1) + t(0, 0, -1));
                v *= 0.5;
                const TS want = MODE == 0 ? (TS)v : (TS)((double)b[at(i, j, k)] - v);
                const TS got = out[(size_t)kk * plane + (size_t)j * nx + i];
                if (got != want) ++bad;
                md = std::max(md, std::fabs((double)got - (double)want));
            }
    printf("apply MODE %d %s %dx%dx%d planes %d from %d ty=%d kc=%d rev=%d: blocks %d threads %d maxdiff %.3g mismatches %zu\n",
           MODE, sizeof(TS) == 4 ? "f32" : "f64", nx, ny, nz, nplanes, k_w0, ty, kc, (int)reverse, nb, nt, md, bad);
    return bad != 0;
}

// The row-band residual + full-weighting restriction (band_restrict.h)
// against the residual and the weighting written out point by point, with z
// coarsened or kept.
template <class T, int W, bool ZC>
int run_restrict(int nx, int ny, int nw, int tyc, int kcc, bool reverse, unsigned seed) {
    const size_t plane = (size_t)nx * ny;
    const int nxc = nx / 2, nyc = ny / 2, nwc = ZC ? (nw - 1) / 2 : nw;
    const size_t planec = (size_t)nxc * nyc;
    std::vector<T> u((nw + 2) * plane, T(0)), e((nw + 2) * plane), f(nw * plane);
    std::vector<T> fc(nwc * planec, T(7)), uc((nwc + 2) * planec, T(7));
    std::mt19937 g(seed);
    std::uniform_real_distribution<double> U(0, 1);
    for (size_t i = plane; i < (nw + 1) * plane; ++i) u[i] = (T)(U(g) - 0.5);
    for (auto &x : e) x = (T)(1.0 + 77.0 * U(g));
    for (auto &x : f) x = (T)(10.0 * (U(g) - 0.5));
    const T cx = (T)1.3, cy = (T)0.7, cz = (T)0.4;
    const int bands = nyc / tyc, nchunks = (nwc + kcc - 1) / kcc, nb = bands * nchunks, nt = (2 * tyc + 3) * (nx / W);
    const int gb = bands % 4 == 0 ? 4 : (bands % 2 == 0 ? 2 : 1);
    RestrictArgs<T> a{u.data(), e.data(), f.data(), fc.data(), uc.data(), nx, ny, nw, nxc, nyc, nwc, tyc, bands, kcc,
                      cx, cy, cz};
    std::vector<int> seen(nb, 0);
    for (int t = 0; t < nb; ++t) {
        const int gg = t / (gb * nchunks), q = t - gg * gb * nchunks;
        const int chunk = q / gb, band = gg * gb + (q - (q / gb) * gb);
        BAND_CHECK(band, bands);
        BAND_CHECK(chunk, nchunks);
        ++seen[chunk * bands + band];
        std::vector<T> lds(restrict_lds_elems(nx, tyc), std::numeric_limits<T>::quiet_NaN());
        std::vector<BandRestrict<T, W, ZC>> th(nt);
        for (int i = 0; i < nt; ++i) { th[i].init(a, lds.data(), band, chunk, i); th[i].prologue(); }
        for (int k = th[0].k0; k <= th[0].k1; ++k)
            for (int i = 0; i < nt; ++i) th[reverse ? nt - 1 - i : i].step(k);
    }
    for (int v : seen)
        if (v != 1) { printf("tile mapping is not a bijection\n"); return 1; }
    auto at = [&](int i, int j, int k) -> size_t { return (size_t)(k + 1) * plane + (size_t)((j + ny) % ny) * nx + (i + nx) % nx; };
    std::vector<T> res(nw * plane);
    for (int k = 0; k < nw; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const T e0 = e[at(i, j, k)], u0 = u[at(i, j, k)];
                const T wxp = cx * (e0 + e[at(i + 1, j, k)]), wxm = cx * (e0 + e[at(i - 1, j, k)]);
                const T wyp = cy * (e0 + e[at(i, j + 1, k)]), wym = cy * (e0 + e[at(i, j - 1, k)]);
                const T wzp = cz * (e0 + e[at(i, j, k + 1)]), wzm = cz * (e0 + e[at(i, j, k - 1)]);
                const T off = T(0.5) * (wxp * u[at(i + 1, j, k)] + wxm * u[at(i - 1, j, k)] + wyp * u[at(i, j + 1, k)] +
                                        wym * u[at(i, j - 1, k)] + wzp * u[at(i, j, k + 1)] + wzm * u[at(i, j, k - 1)]);
                const T dg = T(0.5) * (wxp + wxm + wyp + wym + wzp + wzm);
                res[(size_t)k * plane + (size_t)j * nx + i] = f[(size_t)k * plane + (size_t)j * nx + i] - (off - dg * u0);
            }
    auto rat = [&](int i, int j, int k) { return res[(size_t)k * plane + (size_t)((j + ny) % ny) * nx + (i + nx) % nx]; };
    auto Rin = [&](int ic, int jc, int k) {
        T sx[3];
        for (int d = 0; d < 3; ++d) {
            const int j = 2 * jc - 1 + d;
            sx[d] = T(0.25) * rat(2 * ic - 1, j, k) + T(0.5) * rat(2 * ic, j, k) + T(0.25) * rat(2 * ic + 1, j, k);
        }
        return T(0.25) * sx[0] + T(0.5) * sx[1] + T(0.25) * sx[2];
    };
    size_t bad = 0;
    double md = 0;
    for (int kc = 0; kc < nwc; ++kc)
        for (int jc = 0; jc < nyc; ++jc)
            for (int ic = 0; ic < nxc; ++ic) {
                T want;
                if (!ZC) want = Rin(ic, jc, kc);
                else {
                    T acc = T(0.25) * Rin(ic, jc, 2 * kc);
                    acc += T(0.5) * Rin(ic, jc, 2 * kc + 1);
                    want = acc + T(0.25) * Rin(ic, jc, 2 * kc + 2);
                }
                const T got = fc[(size_t)kc * planec + (size_t)jc * nxc + ic];
                if (got != want) ++bad;
                md = std::max(md, std::fabs((double)got - (double)want));
            }
    for (T v : uc)
        if (v != T(0)) ++bad;
    printf("restrict %s W=%d ZC=%d %dx%dx%d tyc=%d kcc=%d rev=%d: blocks %d threads %d maxdiff %.3g mismatches %zu\n",
           sizeof(T) == 4 ? "f32" : "f64", W, (int)ZC, nx, ny, nw, tyc, kcc, (int)reverse, nb, nt, md, bad);
    return bad != 0;
}

int main() {
    int fails = 0;
    for (int rev = 0; rev < 2; ++rev)
        for (int c0 = 0; c0 < 2; ++c0) {
            fails += run<float, 4, false>(24, 24, 13, 4, 4, c0, rev, 1);
            fails += run<float, 4, false>(32, 16, 9, 8, 2, c0, rev, 2);
            fails += run<float, 4, true>(24, 24, 13, 4, 6, c0, rev, 3);
            fails += run<float, 2, false>(18, 12, 11, 6, 4, c0, rev, 4);
            fails += run<float, 2, true>(18, 12, 11, 6, 4, c0, rev, 5);
            fails += run<double, 2, false>(20, 24, 10, 12, 8, c0, rev, 6);
            fails += run<double, 2, true>(20, 24, 10, 12, 8, c0, rev, 7);
            fails += run<float, 4, false>(192, 24, 21, 12, 6, c0, rev, 8);
            fails += run<float, 4, false>(16, 8, 5, 4, 64, c0, rev, 9);
            fails += run<float, 4, false>(8, 8, 1, 4, 2, c0, rev, 10);
            fails += run<float, 4, false>(24, 32, 23, 8, 3, c0, rev, 11);
            fails += run<double, 2, true>(12, 16, 17, 4, 5, c0, rev, 12);
            fails += run<float, 4, false>(24, 24, 13, 4, 4, c0, rev, 21, 20, 15);  // wraps the box
            fails += run<float, 2, false>(18, 12, 11, 6, 4, c0, rev, 22, 16, 3);
            fails += run<double, 2, false>(20, 24, 10, 12, 8, c0, rev, 23, 10, 0);  // every box plane wet
            fails += run<float, 2, false>(10, 36, 9, 6, 1, c0, rev, 13);
        }
    for (int rev = 0; rev < 2; ++rev) {
        fails += run_apply<0, float>(24, 32, 20, 20, 0, 8, 6, rev, 21);
        fails += run_apply<0, double>(16, 12, 9, 9, 0, 4, 4, rev, 22);
        fails += run_apply<1, double>(12, 12, 10, 10, 0, 6, 3, rev, 23);
        fails += run_apply<2, float>(32, 16, 24, 11, 17, 16, 4, rev, 24);  // wet planes 17 .. 27 wrap past 24
        fails += run_apply<2, double>(8, 24, 12, 12, 0, 12, 5, rev, 25);
        fails += run_apply<2, float>(192, 12, 10, 7, 2, 4, 64, rev, 26);
    }
    for (int rev = 0; rev < 2; ++rev) {
        fails += run_restrict<float, 4, true>(16, 24, 15, 6, 2, rev, 31);
        fails += run_restrict<float, 4, false>(24, 16, 9, 4, 3, rev, 32);
        fails += run_restrict<double, 2, true>(12, 16, 11, 2, 1, rev, 33);
        fails += run_restrict<double, 2, false>(8, 24, 7, 6, 4, rev, 34);
        fails += run_restrict<float, 4, true>(48, 32, 21, 8, 64, rev, 35);
        fails += run_restrict<float, 2, true>(12, 8, 5, 2, 1, rev, 36);
    }
    printf("%s (%d failing cases)\n", fails ? "FAIL" : "OK", fails);
    return fails != 0;
}
