// Level residual and full-weighting restriction in one pass, on full-width
// row bands: the per-thread state and plane step of k_resid_restrict_band
// (kern_grid.hip).
//
// fc = R (f - A u) on the coarse level, R the full weighting (1/4, 1/2, 1/4
// along x and y, and along z when z is coarsened: coarse plane kc from fine
// planes 2 kc .. 2 kc + 2; otherwise coarse plane kc is fine plane kc), with
// the coarse unknowns uc zeroed (the coarse level starts from a zero
// correction).  A u is the 7-point operator of the level in the level's
// precision T, the same arithmetic as the sweeps.
//
// A block owns TYC coarse rows of a chunk of coarse planes: fine rows
// 2 jc0 - 2 .. 2 jc0 + 2 TYC (band rows r = 0 .. 2 TYC + 2; the residual is
// needed on rows 1 .. 2 TYC + 1, the 3 x 3 stencils of the coarse rows, which
// sit on the even band rows 2 .. 2 TYC).  Thread t owns one W-wide vector of
// one band row: it loads that vector of u, eps and f for each fine plane,
// keeps planes k - 1 .. k + 1 of u and eps in registers, stashes plane k + 1
// in LDS for the others' in-plane neighbours, computes the residual of its
// vector at plane k into an LDS ring, and -- one step later, once the ring
// holds the whole band -- a thread of an even row forms the in-plane
// restriction of its W / 2 coarse columns from the rows around it, adding it
// with its z weight into registers that close a coarse plane.  One barrier
// per plane step.  Same conventions as band_sweep.h.
#pragma once

#ifndef BAND_CHECK
#define BAND_CHECK(i, n) ((void)0)
#endif

namespace dwp {

template <class T> struct RestrictArgs {
    const T *u, *e;  // fine level, ghosted: plane k (-1 .. nw) at (k + 1) nx ny
    const T *f;      // fine level, planes 0 .. nw - 1
    T *fc;           // coarse right-hand side, planes 0 .. nwc - 1
    T *uc;           // coarse unknowns, ghosted
    int nx, ny, nw, nxc, nyc, nwc;
    int tyc, bands, kcc;  // coarse rows per band, bands, coarse planes per chunk
    T cx, cy, cz;
};

// Elements of T in one block's LDS: u and eps (2 slots of 2 TYC + 3 rows),
// the residual (2 slots of 2 TYC + 1 rows).
__host__ __device__ inline int restrict_lds_elems(int nx, int tyc) {
    return 4 * (2 * tyc + 3) * nx + 2 * (2 * tyc + 1) * nx;
}

template <class T, int W, bool ZC>
struct BandRestrict {
    typedef typename BandVec<T, W>::V V;
    static constexpr int H = W / 2;  // coarse columns of a vector: x0 / 2 .. x0 / 2 + H - 1

    RestrictArgs<T> a;
    int jc0, c0, c1, k0, k1, nr;
    T *su, *se, *sr;
    size_t plane, planec;
    int r, x0;
    bool res_row, out_row;
    unsigned ou, of, oc;  // the thread's vector in a fine plane (u, eps; f) and its coarse columns
    // planes k - 1, k, k + 1 of u and eps, f of plane k; set k + 2 in flight
    V U0, U1, U2, E0, E1, E2, F1, PU, PE, PF;
    T acc[H];  // the coarse plane being summed (z coarsening)

    __host__ __device__ __forceinline__ void init(const RestrictArgs<T> &args, T *lds, int band, int chunk, int tid) {
        a = args;
        plane = (size_t)a.nx * a.ny;
        planec = (size_t)a.nxc * a.nyc;
        nr = 2 * a.tyc + 3;
        jc0 = band * a.tyc;
        c0 = chunk * a.kcc;
        c1 = c0 + a.kcc < a.nwc ? c0 + a.kcc : a.nwc;
        k0 = ZC ? 2 * c0 : c0;
        k1 = ZC ? 2 * c1 + 1 : c1;  // residual planes [k0, k1)
        su = lds;
        se = su + 2 * nr * a.nx;
        sr = se + 2 * nr * a.nx;
        const int vr = a.nx / W;
        r = tid / vr;
        x0 = (tid - r * vr) * W;
        res_row = r >= 1 && r <= 2 * a.tyc + 1;
        out_row = r >= 2 && r <= 2 * a.tyc && (r & 1) == 0;
        const int jf = (2 * jc0 - 2 + r + 2 * a.ny) % a.ny;
        const int rf = r < 1 ? 1 : (r > 2 * a.tyc + 1 ? 2 * a.tyc + 1 : r);  // f rows beyond the residual repeat one
        const int jff = (2 * jc0 - 2 + rf + 2 * a.ny) % a.ny;
        ou = (unsigned)(jf * a.nx + x0);
        of = (unsigned)(jff * a.nx + x0);
        const int jc = out_row ? jc0 + (r - 2) / 2 : jc0;
        oc = (unsigned)(jc * a.nxc + x0 / 2);
        for (int i = 0; i < H; ++i) acc[i] = T(0);
    }
    // u, eps of plane q (k0 - 1 .. k1, inside the ghosted range); f of plane q
    // (k0 .. k1 - 1); loads past the block's planes re-read the last one
    __host__ __device__ __forceinline__ V ld_g(const T *p, int q) const {
        const int k = q > k1 ? k1 : q;
        BAND_CHECK((size_t)(k + 1) * plane + ou + W - 1, (size_t)(a.nw + 2) * plane);
        return *(const V *)(p + (size_t)(k + 1) * plane + ou);
    }
    __host__ __device__ __forceinline__ V ld_f(int q) const {
        const int k = q > k1 - 1 ? k1 - 1 : q;
        BAND_CHECK((size_t)k * plane + of + W - 1, (size_t)a.nw * plane);
        return *(const V *)(a.f + (size_t)k * plane + of);
    }
    __host__ __device__ __forceinline__ void stash(int q, const V &uu, const V &ee) {
        const int o = ((q - k0 + 2) & 1) * nr * a.nx + r * a.nx + x0;
        BAND_CHECK((size_t)o + W - 1, (size_t)2 * nr * a.nx);
        *(V *)(su + o) = uu;
        *(V *)(se + o) = ee;
    }
    // registers as after step k0 - 1, LDS for step k0, set k0 + 1 in flight
    __host__ __device__ __forceinline__ void prologue() {
        U1 = ld_g(a.u, k0 - 1);
        E1 = ld_g(a.e, k0 - 1);
        U2 = ld_g(a.u, k0);
        E2 = ld_g(a.e, k0);
        stash(k0, U2, E2);
        PU = ld_g(a.u, k0 + 1);
        PE = ld_g(a.e, k0 + 1);
        PF = ld_f(k0);
    }
    // Step k (k0 .. k1): the residual of plane k (k < k1) and the
    // restriction of plane k - 1 (k > k0).
    __host__ __device__ __forceinline__ void step(int k) {
        U0 = U1; U1 = U2; U2 = PU;
        E0 = E1; E1 = E2; E2 = PE;
        F1 = PF;
        stash(k + 1, U2, E2);
        PU = ld_g(a.u, k + 2);
        PE = ld_g(a.e, k + 2);
        PF = ld_f(k + 1);
        if (res_row && k < k1) {
            const int s = (k - k0 + 2) & 1;
            const T *lu = su + s * nr * a.nx, *le = se + s * nr * a.nx;
            const int xl = (x0 - 1 + a.nx) % a.nx, xr = (x0 + W) % a.nx;
            BAND_CHECK((size_t)(r + 1) * a.nx + x0 + W - 1, (size_t)nr * a.nx);
            const T ul = lu[r * a.nx + xl], ur = lu[r * a.nx + xr], el = le[r * a.nx + xl], er = le[r * a.nx + xr];
            const V uu = *(const V *)(lu + (r + 1) * a.nx + x0), ud = *(const V *)(lu + (r - 1) * a.nx + x0);
            const V eu = *(const V *)(le + (r + 1) * a.nx + x0), ed = *(const V *)(le + (r - 1) * a.nx + x0);
            V res;
            for (int i = 0; i < W; ++i) {
                const T e0 = E1[i], u0 = U1[i];
                const T exp = i + 1 < W ? E1[i + 1] : er, exm = i > 0 ? E1[i - 1] : el;
                const T uxp = i + 1 < W ? U1[i + 1] : ur, uxm = i > 0 ? U1[i - 1] : ul;
                const T wxp = a.cx * (e0 + exp), wxm = a.cx * (e0 + exm);
                const T wyp = a.cy * (e0 + eu[i]), wym = a.cy * (e0 + ed[i]);
                const T wzp = a.cz * (e0 + E2[i]), wzm = a.cz * (e0 + E0[i]);
                const T off = T(0.5) * (wxp * uxp + wxm * uxm + wyp * uu[i] + wym * ud[i] + wzp * U2[i] + wzm * U0[i]);
                const T dg = T(0.5) * (wxp + wxm + wyp + wym + wzp + wzm);
                res[i] = F1[i] - (off - dg * u0);
            }
            const int o = s * (nr - 2) * a.nx + (r - 1) * a.nx + x0;
            BAND_CHECK((size_t)o + W - 1, (size_t)2 * (nr - 2) * a.nx);
            *(V *)(sr + o) = res;
        }
        const int kf = k - 1;  // fine plane whose residual the ring holds complete
        if (out_row && kf >= k0) {
            const T *lr = sr + ((kf - k0 + 2) & 1) * (nr - 2) * a.nx;
            const int xe = (x0 - W + a.nx) % a.nx;
            T sx[3][H];
            for (int d = 0; d < 3; ++d) {
                const int row = r - 2 + d;  // band rows r - 1 .. r + 1
                BAND_CHECK((size_t)row * a.nx + x0 + W - 1, (size_t)(nr - 2) * a.nx);
                const V v = *(const V *)(lr + row * a.nx + x0);
                const T left = lr[row * a.nx + xe + W - 1];
                for (int i = 0; i < H; ++i)
                    sx[d][i] = T(0.25) * (i ? v[2 * i - 1] : left) + T(0.5) * v[2 * i] + T(0.25) * v[2 * i + 1];
            }
            int kc = -1;
            T out[H];
            for (int i = 0; i < H; ++i) {
                const T R = T(0.25) * sx[0][i] + T(0.5) * sx[1][i] + T(0.25) * sx[2][i];
                if (!ZC) {
                    kc = kf;
                    out[i] = R;
                } else if ((kf & 1) == 0) {
                    if (kf > k0) {
                        kc = kf / 2 - 1;
                        out[i] = acc[i] + T(0.25) * R;
                    }
                    acc[i] = T(0.25) * R;
                } else {
                    acc[i] += T(0.5) * R;
                }
            }
            if (kc >= 0) {
                BAND_CHECK((size_t)kc * planec + oc + H - 1, (size_t)a.nwc * planec);
                for (int i = 0; i < H; ++i) {
                    a.fc[(size_t)kc * planec + oc + i] = out[i];
                    a.uc[(size_t)(kc + 1) * planec + oc + i] = T(0);
                    if (kc == 0) a.uc[oc + i] = T(0);
                    if (kc == a.nwc - 1) a.uc[(size_t)(a.nwc + 1) * planec + oc + i] = T(0);
                }
            }
        }
    }
};

}  // namespace dwp
