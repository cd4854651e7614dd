// Fused red-black Gauss-Seidel sweep on full-width row bands: the per-thread
// state and plane step of k_sweep_band (kern_grid.hip).
//
// Same sweep as the tiled fused kernel (u_out = one red-black sweep of u_in,
// first colour c0 from u_in, second colour from the new first-colour values),
// on a different block shape.  A block owns TY whole rows of every plane of a
// z chunk [k0, k1): the x direction wraps inside the block, so there is no x
// halo, and each plane of u, eps and f is read as a few contiguous runs of
// whole rows (the y halo: 2 rows of u and eps on each side).  Thread t owns
// one W-wide vector of one band row, r = t / (nx / W) in 0 .. TY + 3 (band row
// r is grid row j0 - 2 + r), for every purpose: it loads that vector of each
// plane, keeps the planes around the current one in registers (so all z
// neighbours are its own registers), computes the first colour at plane m
// (rows 1 .. TY + 2) and the second colour at plane m - 1 (rows 2 .. TY + 1)
// at the same W / 2 columns -- the colour of a column flips from plane to
// plane -- and writes plane m - 1 of the output as one vector.
//
// A block marches up (plane m, then m + 1) or down; the result is the same
// either way (each colour depends only on the other), so neighbouring chunks
// march in opposite directions and reach the planes they share -- the 2-plane
// z halo each reads of the other -- at the same time, while those planes are
// still in L2.  Below, "m + 1" is the next plane of the march (m - 1 when
// marching down), "m - 1" the previous one, and so on.
//
// LDS holds only what other threads read, the in-plane neighbours: u_in of
// plane m at the second-colour points (the only ones the first colour reads;
// one value per pair of columns), eps of planes m - 1 and m, and the new
// first-colour values of plane m - 1 (one per pair of columns).  One barrier
// per plane step: step m stashes plane m + 1 and the first colour of plane m,
// which are read only after the barrier, so the rings need 2 slots of u, 3 of
// eps (plane m + 1 is written while planes m - 1 and m are read) and 2 of the
// first colour.
//
// The code is plain arithmetic and addressing on pointers so that a host
// build can step it thread by thread; BAND_CHECK(i, n) is a bounds hook that
// such a build defines.  It needs gs_value(off, f, diag) declared before it.
#pragma once

#ifndef BAND_CHECK
#define BAND_CHECK(i, n) ((void)0)
#endif

namespace dwp {

template <class T, int W> struct BandVec;
template <> struct BandVec<float, 4> { typedef float V __attribute__((ext_vector_type(4))); };
template <> struct BandVec<float, 2> { typedef float V __attribute__((ext_vector_type(2))); };
template <> struct BandVec<double, 2> { typedef double V __attribute__((ext_vector_type(2))); };

// Launch-wide parameters.
template <class T> struct BandArgs {
    const T *uin;  // ghosted: plane k (-1 .. nw) at (k + 1) * nx * ny
    T *uout;       // ghosted like uin; its plane -1 holds zeros
    const T *e;    // ghosted like uin
    const T *f;    // planes 0 .. nw - 1
    int nx, ny, nw;
    int ty, bands, kc;
    int c0;
    T cx, cy, cz;
    // when set, the output planes are added into this box array (nzb planes
    // of nx * ny; output plane k at box plane (kw0 + k) mod nzb) instead of
    // being stored in uout
    T *zadd;
    int nzb, kw0;
};

// Elements of one block's LDS: u (2 slots), eps (3), first colour (2).
__host__ __device__ inline int band_lds_elems(int nx, int ty) {
    return 2 * (ty + 4) * (nx / 2) + 3 * (ty + 4) * nx + 2 * (ty + 2) * (nx / 2);
}

template <class T>
__host__ __device__ __forceinline__ T band_point(T cx, T cy, T cz, T e0, T exp, T exm, T eyp, T eym, T ezp, T ezm,
                                                 T uxp, T uxm, T uyp, T uym, T uzp, T uzm, T fv) {
    const T wxp = cx * (e0 + exp), wxm = cx * (e0 + exm);
    const T wyp = cy * (e0 + eyp), wym = cy * (e0 + eym);
    const T wzp = cz * (e0 + ezp), wzm = cz * (e0 + ezm);
    const T off = T(0.5) * (wxp * uxp + wxm * uxm + wyp * uyp + wym * uym + wzp * uzp + wzm * uzm);
    const T dg = T(0.5) * (wxp + wxm + wyp + wym + wzp + wzm);
    return gs_value(off, fv, dg);
}

// PD: planes loaded ahead (1 or 2; each costs 3 W-vectors of registers).
template <class T, int W, bool ZIN, bool DOWN, int PD>
struct BandSweep {
    typedef typename BandVec<T, W>::V V;
    static constexpr int H = W / 2;         // points of each colour in a vector
    static constexpr int D = DOWN ? -1 : 1;  // direction of the march

    BandArgs<T> a;
    int j0, k0, k1;
    int qlo, qhi, flo, fhi;  // planes the block reads: u, eps in [qlo, qhi], f in [flo, fhi]
    T *su, *se, *sr;  // LDS rings
    int nh;           // nx / 2
    size_t plane;
    // this thread
    int r, x0;
    bool red_row, blk_row;
    unsigned ou, of;  // element offsets in a plane: the u / eps vector, the f vector
    int par;          // (c0 - j) & 1: first-colour points of plane m sit at x0 + p + 2i, p = (par - m) & 1
    // Registers at step m, with p = (par - m) & 1 (first-colour columns of
    // plane m at x0 + p + 2i, those of planes m - 1 and m + 1 at x0 + 1 - p + 2i):
    //   U0, U1, U2  u of planes m-1, m, m+1 at their second-colour columns (the
    //               only u_in values a sweep reads): x0 + p + 2i, x0 + 1-p + 2i, x0 + p + 2i
    //   E1, E2, E3  eps of planes m-1, m, m+1;  E0  eps of plane m-2 at x0 + p + 2i
    //   F1          f of plane m;  F0  f of plane m-1 at x0 + p + 2i
    //   R0, R1, R2  first colour of planes m-2, m-1, m at their columns
    V E1, E2, E3, F1;
    T U0[H], U1[H], U2[H], E0[H], F0[H], R0[H], R1[H], R2[H];
    V PU[PD], PE[PD], PF[PD];  // loads in flight: set q = {u(q), eps(q), f(q - D)}, slot = step index % PD

    // ring position of plane q: >= 0 for every plane used (k0 - 4 .. k1 + 3)
    __host__ __device__ __forceinline__ int lp(int q) const { return q - k0 + 4; }

    __host__ __device__ __forceinline__ void init(const BandArgs<T> &args, T *lds, int band, int chunk, int tid) {
        a = args;
        nh = a.nx / 2;
        plane = (size_t)a.nx * a.ny;
        j0 = band * a.ty;
        k0 = chunk * a.kc;
        k1 = k0 + a.kc < a.nw ? k0 + a.kc : a.nw;
        // the first colour at k0 - 1 .. k1 reads u, eps of k0 - 2 .. k1 + 1 and
        // f of its own planes, clipped to the stored ones; loads of planes
        // beyond (the prefetches of the last steps, the unused start of the
        // prologue) re-read the nearest plane of the range, which is cached
        qlo = k0 - 2 > -1 ? k0 - 2 : -1;
        qhi = k1 + 1 < a.nw ? k1 + 1 : a.nw;
        flo = k0 - 1 > 0 ? k0 - 1 : 0;
        fhi = k1 < a.nw - 1 ? k1 : a.nw - 1;
        su = lds;
        se = su + 2 * (a.ty + 4) * nh;
        sr = se + 3 * (a.ty + 4) * a.nx;
        // threads of the even band rows first, then those of the odd rows, so
        // that a wavefront whose threads share the row parity (all of them when
        // (ty + 4) / 2 * nx / W is a multiple of 64) shares the column parity p
        // of every step and runs one branch of it
        const int vr = a.nx / W, half_nt = (a.ty + 4) / 2 * vr;
        const int g = tid >= half_nt ? 1 : 0, q = tid - g * half_nt;
        r = 2 * (q / vr) + g;
        x0 = (q % vr) * W;
        red_row = r >= 1 && r <= a.ty + 2;
        blk_row = r >= 2 && r <= a.ty + 1;
        const int j = (j0 - 2 + r + 2 * a.ny) % a.ny;
        const int rf = r < 1 ? 1 : (r > a.ty + 2 ? a.ty + 2 : r);  // f rows beyond the first colour repeat a used one
        const int jf = (j0 - 2 + rf + 2 * a.ny) % a.ny;
        ou = (unsigned)(j * a.nx + x0);
        of = (unsigned)(jf * a.nx + x0);
        par = (a.c0 - j) & 1;
        for (int i = 0; i < H; ++i) R0[i] = R1[i] = R2[i] = T(0);
    }

    // second-colour columns of plane q: x0 + s + 2i
    __host__ __device__ __forceinline__ int scol(int q) const { return (par + 1 - q) & 1; }
    __host__ __device__ __forceinline__ static void half(T *d, const V &v, int s) {
        for (int i = 0; i < H; ++i) d[i] = s ? v[2 * i + 1] : v[2 * i];
    }

    __host__ __device__ __forceinline__ V ld_u(int q) const {
        const int k = q < qlo ? qlo : (q > qhi ? qhi : q);
        BAND_CHECK((size_t)(k + 1) * plane + ou + W - 1, (size_t)(a.nw + 2) * plane);
        return *(const V *)(a.uin + (size_t)(k + 1) * plane + ou);
    }
    __host__ __device__ __forceinline__ V ld_e(int q) const {
        const int k = q < qlo ? qlo : (q > qhi ? qhi : q);
        BAND_CHECK((size_t)(k + 1) * plane + ou + W - 1, (size_t)(a.nw + 2) * plane);
        return *(const V *)(a.e + (size_t)(k + 1) * plane + ou);
    }
    __host__ __device__ __forceinline__ V ld_f(int q) const {
        const int k = q < flo ? flo : (q > fhi ? fhi : q);
        BAND_CHECK((size_t)k * plane + of + W - 1, (size_t)a.nw * plane);
        return *(const V *)(a.f + (size_t)k * plane + of);
    }
    // set q into prefetch slot s
    __host__ __device__ __forceinline__ void fetch(int q, int s) {
        if constexpr (ZIN) PU[s] = V(0);
        else PU[s] = ld_u(q);
        PE[s] = ld_e(q);
        PF[s] = ld_f(q - D);
    }

    // u ring: second-colour values of plane q (uc, as kept in registers), one
    // per column pair
    __host__ __device__ __forceinline__ void stash_u(int q, const T *uc) {
        if constexpr (!ZIN) {
            T *d = su + (lp(q) & 1) * (a.ty + 4) * nh + r * nh + x0 / 2;
            BAND_CHECK((size_t)(d - su) + H - 1, (size_t)2 * (a.ty + 4) * nh);
            for (int i = 0; i < H; ++i) d[i] = uc[i];
        }
    }
    __host__ __device__ __forceinline__ void stash_e(int q, const V &e) {
        T *d = se + (lp(q) % 3) * (a.ty + 4) * a.nx + r * a.nx + x0;
        BAND_CHECK((size_t)(d - se) + W - 1, (size_t)3 * (a.ty + 4) * a.nx);
        *(V *)d = e;
    }

    // The march: steps i = 0 .. nsteps() - 1 at planes m = first() + D i.  The
    // first colour is computed at every m (k0 - 1 .. k1, the chunk and the
    // planes beside it), the second at m - D when that lies in the chunk.
    __host__ __device__ __forceinline__ int first() const { return DOWN ? k1 : k0 - 1; }
    __host__ __device__ __forceinline__ int nsteps() const { return k1 - k0 + 2; }

    // Prologue: registers as after step -1, LDS for step 0, the sets of the
    // first PD steps in flight.
    __host__ __device__ __forceinline__ void prologue() {
        const int m0 = first();
        if constexpr (ZIN) {
            for (int i = 0; i < H; ++i) U0[i] = U1[i] = U2[i] = T(0);
        } else {
            half(U1, ld_u(m0 - D), scol(m0 - D));
            half(U2, ld_u(m0), scol(m0));
        }
        E1 = ld_e(m0 - 2 * D);
        E2 = ld_e(m0 - D);
        E3 = ld_e(m0);
        F1 = ld_f(m0 - D);
        stash_u(m0, U2);
        stash_e(m0 - D, E2);
        stash_e(m0, E3);
        for (int d = 0; d < PD; ++d) fetch(m0 + (d + 1) * D, d);
    }

    // One plane step (S = the step index, of which S % PD is the prefetch slot
    // consumed and refilled), specialised on the column parity p of its first
    // colour.
    template <int S>
    __host__ __device__ __forceinline__ void step(int m) {
        if ((par - m) & 1) run<S % PD, 1>(m);
        else run<S % PD, 0>(m);
    }
    template <int B, int p>
    __host__ __device__ __forceinline__ void run(int m) {
        // rotate to planes m-1 .. m+1 of u, m-2 .. m+1 of eps, m-1, m of f (in
        // the direction of the march)
        if constexpr (!ZIN)
            for (int i = 0; i < H; ++i) { U0[i] = U1[i]; U1[i] = U2[i]; }
        half(E0, E1, p);
        half(F0, F1, p);
        for (int i = 0; i < H; ++i) { R0[i] = R1[i]; R1[i] = R2[i]; }
        if constexpr (!ZIN) half(U2, PU[B], p);
        E1 = E2; E2 = E3; E3 = PE[B];
        F1 = PF[B];
        stash_u(m + D, U2);
        stash_e(m + D, E3);
        fetch(m + (PD + 1) * D, B);
        const int xe = p ? (x0 + W) % a.nx : (x0 - W + a.nx) % a.nx;  // vector holding the one outside neighbour
        const int ue = p ? 0 : H - 1, ee = p ? 0 : W - 1;               // its element
        // first colour at plane m, columns x0 + p + 2i
        if (red_row) {
            const T *sul = su + (lp(m) & 1) * (a.ty + 4) * nh;
            const T *sel = se + (lp(m) % 3) * (a.ty + 4) * a.nx;
            BAND_CHECK((size_t)(r + 1) * nh + x0 / 2 + H - 1, (size_t)(a.ty + 4) * nh);
            BAND_CHECK((size_t)(r + 1) * a.nx + x0 + W - 1, (size_t)(a.ty + 4) * a.nx);
            T uedge = T(0), uym[H], uyp[H];  // u_in of plane m at its second-colour columns
            if constexpr (!ZIN) {
                uedge = sul[r * nh + xe / 2 + ue];
                for (int i = 0; i < H; ++i) {
                    uym[i] = sul[(r - 1) * nh + x0 / 2 + i];
                    uyp[i] = sul[(r + 1) * nh + x0 / 2 + i];
                }
            } else {
                for (int i = 0; i < H; ++i) uym[i] = uyp[i] = T(0);
            }
            const T eedge = sel[r * a.nx + xe + ee];
            const T *eym = sel + (r - 1) * a.nx + x0 + p, *eyp = sel + (r + 1) * a.nx + x0 + p;
            for (int i = 0; i < H; ++i) {
                const int c = 2 * i;  // the point is element c + p
                const T uxm = p ? U1[i] : (i ? U1[i - 1] : uedge);
                const T uxp = p ? (i < H - 1 ? U1[i + 1] : uedge) : U1[i];
                const T exm = p ? E2[c] : (i ? E2[c - 1] : eedge);
                const T exp = p ? (i < H - 1 ? E2[c + 2] : eedge) : E2[c + 1];
                const T e0 = p ? E2[c + 1] : E2[c];
                const T en = p ? E3[c + 1] : E3[c], ep = p ? E1[c + 1] : E1[c];  // next, previous plane
                const T v = band_point<T>(a.cx, a.cy, a.cz, e0, exp, exm, eyp[c], eym[c], DOWN ? ep : en,
                                          DOWN ? en : ep, uxp, uxm, uyp[i],
                                          uym[i], DOWN ? U0[i] : U2[i], DOWN ? U2[i] : U0[i], p ? F1[c + 1] : F1[c]);
                R2[i] = (m >= 0 && m < a.nw) ? v : T(0);  // planes -1 and nw are the zero boundary
            }
            T *d = sr + (lp(m) & 1) * (a.ty + 2) * nh + (r - 1) * nh + x0 / 2;
            BAND_CHECK((size_t)(d - sr) + H - 1, (size_t)2 * (a.ty + 2) * nh);
            for (int i = 0; i < H; ++i) d[i] = R2[i];
        }
        // second colour at plane k = m - 1, the same columns; output plane k
        if (blk_row) {
            const int k = m - D;
            const T *srl = sr + (lp(k) & 1) * (a.ty + 2) * nh;
            const T *sel = se + (lp(k) % 3) * (a.ty + 4) * a.nx;
            BAND_CHECK((size_t)r * nh + x0 / 2 + H - 1, (size_t)(a.ty + 2) * nh);
            const T redge = srl[(r - 1) * nh + xe / 2 + ue];
            const T eedge = sel[r * a.nx + xe + ee];
            const T *eym = sel + (r - 1) * a.nx + x0 + p, *eyp = sel + (r + 1) * a.nx + x0 + p;
            V o;
            for (int i = 0; i < H; ++i) {
                const int c = 2 * i;
                const T rxm = p ? R1[i] : (i ? R1[i - 1] : redge);
                const T rxp = p ? (i < H - 1 ? R1[i + 1] : redge) : R1[i];
                const T exm = p ? E1[c] : (i ? E1[c - 1] : eedge);
                const T exp = p ? (i < H - 1 ? E1[c + 2] : eedge) : E1[c + 1];
                const T e0 = p ? E1[c + 1] : E1[c];
                const T en = p ? E2[c + 1] : E2[c];  // eps of the next plane (m); E0: the previous
                const T v = band_point<T>(a.cx, a.cy, a.cz, e0, exp, exm, eyp[c], eym[c], DOWN ? E0[i] : en,
                                          DOWN ? en : E0[i], rxp, rxm,
                                          srl[r * nh + x0 / 2 + i], srl[(r - 2) * nh + x0 / 2 + i],
                                          DOWN ? R0[i] : R2[i], DOWN ? R2[i] : R0[i], F0[i]);
                o[c] = p ? R1[i] : v;
                o[c + 1] = p ? v : R1[i];
            }
            // one store per thread and step; steps outside the chunk write
            // zeros into the zero plane -1 of the output
            const bool valid = k >= k0 && k < k1;
            if (a.zadd && valid) {
                T *zd = a.zadd + (size_t)((a.kw0 + k) % a.nzb) * plane + ou;
                BAND_CHECK((size_t)(zd - a.zadd) + W - 1, (size_t)a.nzb * plane);
                *(V *)zd = *(const V *)zd + o;
            } else {
                T *dst = a.uout + (valid ? (size_t)(k + 1) * plane : 0) + ou;
                BAND_CHECK((size_t)(dst - a.uout) + W - 1, (size_t)(a.nw + 2) * plane);
                *(V *)dst = valid ? o : V(0);
            }
        }
    }
};

}  // namespace dwp
