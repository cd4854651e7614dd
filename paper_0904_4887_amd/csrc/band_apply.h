// The 7-point operator on full-width row bands: the per-thread state and
// plane step of k_apply_band (kern_grid.hip).
//
// (A phi)_n = 1/2 sum over the six faces f of n of c_d (eps_n + eps_nb) (phi_nb - phi_n),
// c_d = 1 / h_d^2, on the periodic box (MODE 0: out = A phi; MODE 1: out =
// b - A phi) or on the wet planes kk = 0 .. nplanes - 1 at box planes
// (k_w0 + kk) mod nz (MODE 2: out[kk] = b - A phi, b read at the box plane).
// The arithmetic is float64 whatever the storage type TS of phi and eps.
//
// A block owns TY whole rows of every plane of a chunk [kk0, kk1) of planes.
// Thread t owns one W-wide vector (16 bytes of TS) of band row r (grid row
// j0 - 1 + r, r = 0 .. TY + 1): it loads that vector of phi and eps (and of b)
// for every plane, keeps planes kk - 1 .. kk + 1 in registers (the z
// neighbours), stashes plane kk + 1 in LDS for the others' in-plane
// neighbours, and, on rows 1 .. TY, writes plane kk of out as one vector.
// One barrier per plane step (plane kk + 1 is stashed while plane kk is read:
// two ring slots).  Same conventions as band_sweep.h: plain arithmetic and
// addressing on pointers, BAND_CHECK(i, n) a bounds hook for a host build.
#pragma once

#include <type_traits>

#ifndef BAND_CHECK
#define BAND_CHECK(i, n) ((void)0)
#endif

namespace dwp {

template <class TS> struct ApplyVec;
template <> struct ApplyVec<float> {
    static constexpr int W = 4;
    typedef float V __attribute__((ext_vector_type(4)));
};
template <> struct ApplyVec<double> {
    static constexpr int W = 2;
    typedef double V __attribute__((ext_vector_type(2)));
};

template <class T, int W> struct ApplyVecOf {
    typedef T V __attribute__((ext_vector_type(W)));
};

template <class TS, class TB> struct ApplyArgs {
    const TS *phi, *eps;  // box arrays, nz planes of nx * ny
    const TB *b;          // MODE 1, 2: box array (float16 under a float32 phi)
    TS *out;              // MODE 0, 1: box array; MODE 2: nplanes planes
    int nx, ny, nz, k_w0, nplanes;
    int ty, bands, kc;
    double cx, cy, cz;
};

// Elements of TS in one block's LDS: phi and eps, 2 slots of TY + 2 rows.
__host__ __device__ inline int apply_lds_elems(int nx, int ty) { return 4 * (ty + 2) * nx; }

template <int MODE, class TS, class TB>
struct BandApply {
    typedef typename ApplyVec<TS>::V V;
    static constexpr int W = ApplyVec<TS>::W;
    typedef typename ApplyVecOf<TB, W>::V VB;  // W values of b

    ApplyArgs<TS, TB> a;
    int j0, kk0, kk1, base;
    TS *sp, *se;
    size_t plane;
    int r, x0;
    bool out_row;
    unsigned ou;  // element offset of the thread's vector in a plane
    // planes kk - 1, kk, kk + 1 of phi and eps; b of plane kk; set kk + 2 in flight
    V P0, P1, P2, E0, E1, E2, QP, QE;
    VB NB, QB;

    __host__ __device__ __forceinline__ void init(const ApplyArgs<TS, TB> &args, TS *lds, int band, int chunk,
                                                  int tid) {
        a = args;
        plane = (size_t)a.nx * a.ny;
        j0 = band * a.ty;
        kk0 = chunk * a.kc;
        kk1 = kk0 + a.kc < a.nplanes ? kk0 + a.kc : a.nplanes;
        base = MODE == 2 ? a.k_w0 : 0;
        sp = lds;
        se = sp + 2 * (a.ty + 2) * a.nx;
        const int vr = a.nx / W;
        r = tid / vr;
        x0 = (tid - r * vr) * W;
        out_row = r >= 1 && r <= a.ty;
        const int j = (j0 - 1 + r + a.ny) % a.ny;
        ou = (unsigned)(j * a.nx + x0);
    }
    // box plane of wet (or box) plane q, periodic
    __host__ __device__ __forceinline__ size_t boxp(int q) const {
        int k = (base + q) % a.nz;
        if (k < 0) k += a.nz;
        return (size_t)k * plane;
    }
    __host__ __device__ __forceinline__ V ld(const TS *f, int q) const {
        const size_t o = boxp(q) + ou;
        BAND_CHECK(o + W - 1, (size_t)a.nz * plane);
        return *(const V *)(f + o);
    }
    // set q = {phi(q), eps(q), b(q - 1)}; loads past the chunk's planes
    // (kk0 - 1 .. kk1) re-read its last one, which is cached
    __host__ __device__ __forceinline__ void fetch(int q) {
        const int qc = q > kk1 ? kk1 : q;
        QP = ld(a.phi, qc);
        QE = ld(a.eps, qc);
        if constexpr (MODE != 0) {
            const int qb = q - 1 > kk1 - 1 ? kk1 - 1 : q - 1;
            const size_t o = boxp(qb) + ou;
            BAND_CHECK(o + W - 1, (size_t)a.nz * plane);
            static_assert(std::is_same<TB, TS>::value || sizeof(TB) < sizeof(TS), "b is stored like phi or narrower");
            QB = *(const VB *)(a.b + o);
        }
    }
    __host__ __device__ __forceinline__ void stash(int q, const V &p, const V &e) {
        const int s = (q - kk0 + 2) & 1;
        const int o = s * (a.ty + 2) * a.nx + r * a.nx + x0;
        BAND_CHECK((size_t)o + W - 1, (size_t)2 * (a.ty + 2) * a.nx);
        *(V *)(sp + o) = p;
        *(V *)(se + o) = e;
    }
    // registers as after step kk0 - 1, LDS for step kk0, set kk0 + 1 in flight
    __host__ __device__ __forceinline__ void prologue() {
        P1 = ld(a.phi, kk0 - 1);
        E1 = ld(a.eps, kk0 - 1);
        P2 = ld(a.phi, kk0);
        E2 = ld(a.eps, kk0);
        stash(kk0, P2, E2);
        fetch(kk0 + 1);
    }
    __host__ __device__ __forceinline__ void step(int kk) {
        P0 = P1; P1 = P2; P2 = QP;
        E0 = E1; E1 = E2; E2 = QE;
        if constexpr (MODE != 0) NB = QB;
        stash(kk + 1, P2, E2);
        fetch(kk + 2);
        if (!out_row) return;
        const int s = (kk - kk0 + 2) & 1;
        const TS *lp = sp + s * (a.ty + 2) * a.nx, *le = se + s * (a.ty + 2) * a.nx;
        const int xl = (x0 - 1 + a.nx) % a.nx, xr = (x0 + W) % a.nx;
        BAND_CHECK((size_t)(r + 1) * a.nx + x0 + W - 1, (size_t)(a.ty + 2) * a.nx);
        const double pl = lp[r * a.nx + xl], pr = lp[r * a.nx + xr];
        const double el = le[r * a.nx + xl], er = le[r * a.nx + xr];
        const V pu = *(const V *)(lp + (r + 1) * a.nx + x0), pd = *(const V *)(lp + (r - 1) * a.nx + x0);
        const V eu = *(const V *)(le + (r + 1) * a.nx + x0), ed = *(const V *)(le + (r - 1) * a.nx + x0);
        V o;
        for (int e = 0; e < W; ++e) {
            const double p0 = P1[e], e0 = E1[e];
            const double pxr = e + 1 < W ? (double)P1[e + 1] : pr, exr = e + 1 < W ? (double)E1[e + 1] : er;
            const double pxl = e > 0 ? (double)P1[e - 1] : pl, exl = e > 0 ? (double)E1[e - 1] : el;
            double v = a.cx * ((e0 + exr) * (pxr - p0) + (e0 + exl) * (pxl - p0)) +
                       a.cy * ((e0 + (double)eu[e]) * ((double)pu[e] - p0) + (e0 + (double)ed[e]) * ((double)pd[e] - p0)) +
                       a.cz * ((e0 + (double)E2[e]) * ((double)P2[e] - p0) + (e0 + (double)E0[e]) * ((double)P0[e] - p0));
            v *= 0.5;
            if constexpr (MODE == 0) o[e] = (TS)v;
            else o[e] = (TS)((double)NB[e] - v);
        }
        const size_t dst = (MODE == 2 ? (size_t)kk * plane : boxp(kk)) + ou;
        BAND_CHECK(dst + W - 1, (size_t)(MODE == 2 ? a.nplanes : a.nz) * plane);
        *(V *)(a.out + dst) = o;
    }
};

}  // namespace dwp
