// The paper's sixth-order operator (Sec. II.F, Eqs. 16-18) on the full
// periodic box, its transpose, and the gradient kernels its adjoint needs.
//
//   A6 x   = sum_d G_d D1_d x + eps D2_d x,        G_d = D1_d eps,
//   A6^T y = sum_d -D1_d(G_d y) + D2_d(eps y),
// with the seven-point central stencils
//   D1 f_i = (1/h) sum_{n=1..3} a_n (f_{i+n} - f_{i-n}),   a = (3/4, -3/20, 1/60),
//   D2 f_i = (1/h^2) [b_0 f_i + sum_{n=1..3} b_n (f_{i+n} + f_{i-n})],
//   b = (-49/18, 3/2, -3/20, 1/90).
// G is computed once per permittivity.  One thread per node, neighbours read
// through the caches (the 19-point star of x and, for the transpose, of eps
// and G); every axis is periodic and at least 8 long, so a shift of up to 3
// wraps at most once.
#include "dwp_internal.h"

namespace dwp {

namespace {

constexpr int SX = 64, SY = 4;
constexpr double A1 = 0.75, A2 = -0.15, A3 = 1.0 / 60.0;
constexpr double B0 = -49.0 / 18.0, B1 = 1.5, B2 = -0.15, B3 = 1.0 / 90.0;
constexpr double FOUR_PI = 4.0 * 3.14159265358979323846;

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

struct Grid6 {
    int nx, ny, nz;
    size_t plane, N;
    double ihx, ihy, ihz;        // 1/h
    double ihx2, ihy2, ihz2;     // 1/h^2
};

Grid6 make_grid6(const Plan &p) {
    Grid6 g;
    g.nx = p.nx; g.ny = p.ny; g.nz = p.nz;
    g.plane = (size_t)p.nx * p.ny;
    g.N = p.N;
    g.ihx = 1.0 / p.h[0]; g.ihy = 1.0 / p.h[1]; g.ihz = 1.0 / p.h[2];
    g.ihx2 = g.ihx * g.ihx; g.ihy2 = g.ihy * g.ihy; g.ihz2 = g.ihz * g.ihz;
    return g;
}

// Offsets of the six neighbours at distance 1..3 along each axis, as flat
// index differences (periodic).
struct Star {
    long long xp[3], xm[3], yp[3], ym[3], zp[3], zm[3];
};

__device__ __forceinline__ Star star(const Grid6 &g, int i, int j, int k) {
    Star s;
#pragma unroll
    for (int n = 1; n <= 3; ++n) {
        s.xp[n - 1] = wrap(i + n, g.nx) - i;
        s.xm[n - 1] = wrap(i - n, g.nx) - i;
        s.yp[n - 1] = (long long)(wrap(j + n, g.ny) - j) * g.nx;
        s.ym[n - 1] = (long long)(wrap(j - n, g.ny) - j) * g.nx;
        s.zp[n - 1] = (long long)(wrap(k + n, g.nz) - k) * (long long)g.plane;
        s.zm[n - 1] = (long long)(wrap(k - n, g.nz) - k) * (long long)g.plane;
    }
    return s;
}

__device__ __forceinline__ double d1(const double *f, size_t c, const long long *p, const long long *m, double ih) {
    return ih * (A1 * (f[c + p[0]] - f[c + m[0]]) + A2 * (f[c + p[1]] - f[c + m[1]]) + A3 * (f[c + p[2]] - f[c + m[2]]));
}

__device__ __forceinline__ double d2(const double *f, size_t c, const long long *p, const long long *m, double ih2) {
    return ih2 * (B0 * f[c] + B1 * (f[c + p[0]] + f[c + m[0]]) + B2 * (f[c + p[1]] + f[c + m[1]]) +
                  B3 * (f[c + p[2]] + f[c + m[2]]));
}

// products f g at offsets, for the transpose
__device__ __forceinline__ double d1p(const double *f, const double *w, size_t c, const long long *p,
                                      const long long *m, double ih) {
    double s = 0.0;
    const double a[3] = {A1, A2, A3};
#pragma unroll
    for (int n = 0; n < 3; ++n) s += a[n] * (f[c + p[n]] * w[c + p[n]] - f[c + m[n]] * w[c + m[n]]);
    return ih * s;
}

__device__ __forceinline__ double d2p(const double *f, const double *w, size_t c, const long long *p,
                                      const long long *m, double ih2) {
    double s = B0 * f[c] * w[c];
    const double b[3] = {B1, B2, B3};
#pragma unroll
    for (int n = 0; n < 3; ++n) s += b[n] * (f[c + p[n]] * w[c + p[n]] + f[c + m[n]] * w[c + m[n]]);
    return ih2 * s;
}

template <bool TRANS>
__device__ __forceinline__ double op6(const Grid6 &g, const double *__restrict__ x, const double *__restrict__ eps,
                                      const double *__restrict__ G, size_t c, const Star &s) {
    const double *Gx = G, *Gy = G + g.N, *Gz = G + 2 * g.N;
    if (!TRANS) {
        const double e = eps[c];
        return Gx[c] * d1(x, c, s.xp, s.xm, g.ihx) + Gy[c] * d1(x, c, s.yp, s.ym, g.ihy) +
               Gz[c] * d1(x, c, s.zp, s.zm, g.ihz) +
               e * (d2(x, c, s.xp, s.xm, g.ihx2) + d2(x, c, s.yp, s.ym, g.ihy2) + d2(x, c, s.zp, s.zm, g.ihz2));
    }
    return -d1p(Gx, x, c, s.xp, s.xm, g.ihx) - d1p(Gy, x, c, s.yp, s.ym, g.ihy) - d1p(Gz, x, c, s.zp, s.zm, g.ihz) +
           d2p(eps, x, c, s.xp, s.xm, g.ihx2) + d2p(eps, x, c, s.yp, s.ym, g.ihy2) +
           d2p(eps, x, c, s.zp, s.zm, g.ihz2);
}

// G_d = D1_d eps for the three directions
__global__ void __launch_bounds__(SX *SY) k_d1eps(Grid6 g, const double *__restrict__ eps, double *__restrict__ G) {
    const int i = blockIdx.x * SX + threadIdx.x, j = blockIdx.y * SY + threadIdx.y, k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const size_t c = (size_t)k * g.plane + (size_t)j * g.nx + i;
    const Star s = star(g, i, j, k);
    G[c] = d1(eps, c, s.xp, s.xm, g.ihx);
    G[g.N + c] = d1(eps, c, s.yp, s.ym, g.ihy);
    G[2 * g.N + c] = d1(eps, c, s.zp, s.zm, g.ihz);
}

// MODE 0: out = op x;  MODE 1: out = b - op x
template <int MODE, bool TRANS>
__global__ void __launch_bounds__(SX *SY)
k_apply6(Grid6 g, const double *__restrict__ x, const double *__restrict__ eps, const double *__restrict__ G,
         const double *__restrict__ b, double *__restrict__ out) {
    const int i = blockIdx.x * SX + threadIdx.x, j = blockIdx.y * SY + threadIdx.y, k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const size_t c = (size_t)k * g.plane + (size_t)j * g.nx + i;
    const double v = op6<TRANS>(g, x, eps, G, c, star(g, i, j, k));
    out[c] = MODE == 0 ? v : b[c] - v;
}

// Wet residual: fW (slab plane q = box plane (k_w0 + q) mod nz) = v - op dD
template <class T, bool TRANS>
__global__ void __launch_bounds__(SX *SY)
k_wet_residual6(Grid6 g, int k_w0, const double *__restrict__ v, const double *__restrict__ dD,
                const double *__restrict__ eps, const double *__restrict__ G, T *__restrict__ fW) {
    const int i = blockIdx.x * SX + threadIdx.x, j = blockIdx.y * SY + threadIdx.y, q = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const int k = wrap(k_w0 + q, g.nz);
    const size_t c = (size_t)k * g.plane + (size_t)j * g.nx + i;
    const double r = v[c] - op6<TRANS>(g, dD, eps, G, c, star(g, i, j, k));
    fW[(size_t)q * g.plane + (size_t)j * g.nx + i] = (T)r;
}

// dE/d eps_n = sum_d D1_d(lam D1_d phi)_n - lam_n (sum_d D2_d phi)_n; the inner D1
// at a shifted node uses that node's own (wrapped) offsets.
__global__ void __launch_bounds__(SX *SY)
k_grad6(Grid6 g, const double *__restrict__ phi, const double *__restrict__ lam, double *__restrict__ out) {
    const int i = blockIdx.x * SX + threadIdx.x, j = blockIdx.y * SY + threadIdx.y, k = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const size_t c = (size_t)k * g.plane + (size_t)j * g.nx + i;
    const double lc = lam[c];
    double s = 0.0;
    {
        // x
        const Star s0 = star(g, i, j, k);
        const double a[3] = {A1, A2, A3};
        double acc = 0.0;
#pragma unroll
        for (int n = 0; n < 3; ++n) {
            const Star sp = star(g, wrap(i + n + 1, g.nx), j, k), sm = star(g, wrap(i - n - 1, g.nx), j, k);
            const size_t cp = c + s0.xp[n], cm = c + s0.xm[n];
            double dp = 0.0, dm = 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                dp += a[q] * (phi[cp + sp.xp[q]] - phi[cp + sp.xm[q]]);
                dm += a[q] * (phi[cm + sm.xp[q]] - phi[cm + sm.xm[q]]);
            }
            acc += a[n] * (lam[cp] * dp - lam[cm] * dm);
        }
        s += g.ihx * g.ihx * acc - lc * d2(phi, c, s0.xp, s0.xm, g.ihx2);
        // y
        acc = 0.0;
#pragma unroll
        for (int n = 0; n < 3; ++n) {
            const Star sp = star(g, i, wrap(j + n + 1, g.ny), k), sm = star(g, i, wrap(j - n - 1, g.ny), k);
            const size_t cp = c + s0.yp[n], cm = c + s0.ym[n];
            double dp = 0.0, dm = 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                dp += a[q] * (phi[cp + sp.yp[q]] - phi[cp + sp.ym[q]]);
                dm += a[q] * (phi[cm + sm.yp[q]] - phi[cm + sm.ym[q]]);
            }
            acc += a[n] * (lam[cp] * dp - lam[cm] * dm);
        }
        s += g.ihy * g.ihy * acc - lc * d2(phi, c, s0.yp, s0.ym, g.ihy2);
        // z
        acc = 0.0;
#pragma unroll
        for (int n = 0; n < 3; ++n) {
            const Star sp = star(g, i, j, wrap(k + n + 1, g.nz)), sm = star(g, i, j, wrap(k - n - 1, g.nz));
            const size_t cp = c + s0.zp[n], cm = c + s0.zm[n];
            double dp = 0.0, dm = 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                dp += a[q] * (phi[cp + sp.zp[q]] - phi[cp + sp.zm[q]]);
                dm += a[q] * (phi[cm + sm.zp[q]] - phi[cm + sm.zm[q]]);
            }
            acc += a[n] * (lam[cp] * dp - lam[cm] * dm);
        }
        s += g.ihz * g.ihz * acc - lc * d2(phi, c, s0.zp, s0.zm, g.ihz2);
    }
    out[c] = s;
}

// psi = phi / 2 - 4 pi lam / h^3 (h^3 psi = dE/d rho);  mode 1: out = g m / h^3 (+ psi if add)
__global__ void k_charge_potential(const double *__restrict__ phi, const double *__restrict__ lam, double s4pi_h3,
                                   double *__restrict__ psi, size_t n) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        psi[t] = 0.5 * phi[t] - s4pi_h3 * lam[t];
}

__global__ void k_scaled_product(const double *__restrict__ gr, const double *__restrict__ m, double inv_h3,
                                 const double *__restrict__ add, double *__restrict__ out, size_t n) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        out[t] = gr[t] * m[t] * inv_h3 + (add ? add[t] : 0.0);
}

int grid1d6(size_t n) {
    size_t b = (n + 255) / 256;
    return (int)(b > 4096 ? 4096 : b);
}

}  // namespace

void launch_d1eps(hipStream_t s, const Plan &p, const double *eps, double *G) {
    const Grid6 g = make_grid6(p);
    dim3 gr((p.nx + SX - 1) / SX, (p.ny + SY - 1) / SY, p.nz), blk(SX, SY);
    k_d1eps<<<gr, blk, 0, s>>>(g, eps, G);
    DWP_LAUNCH_CHECK();
}

void launch_apply6(hipStream_t s, const Plan &p, const double *x, const double *eps, const double *G,
                   const double *b, double *out, bool residual, bool trans) {
    const Grid6 g = make_grid6(p);
    dim3 gr((p.nx + SX - 1) / SX, (p.ny + SY - 1) / SY, p.nz), blk(SX, SY);
    if (residual) {
        if (trans) k_apply6<1, true><<<gr, blk, 0, s>>>(g, x, eps, G, b, out);
        else k_apply6<1, false><<<gr, blk, 0, s>>>(g, x, eps, G, b, out);
    } else {
        if (trans) k_apply6<0, true><<<gr, blk, 0, s>>>(g, x, eps, G, b, out);
        else k_apply6<0, false><<<gr, blk, 0, s>>>(g, x, eps, G, b, out);
    }
    DWP_LAUNCH_CHECK();
}

template <class T>
void launch_wet_residual6(hipStream_t s, const Plan &p, const double *v, const double *dD, const double *eps,
                          const double *G, T *fW, bool trans) {
    const Grid6 g = make_grid6(p);
    dim3 gr((p.nx + SX - 1) / SX, (p.ny + SY - 1) / SY, p.nw), blk(SX, SY);
    if (trans) k_wet_residual6<T, true><<<gr, blk, 0, s>>>(g, p.k_w0, v, dD, eps, G, fW);
    else k_wet_residual6<T, false><<<gr, blk, 0, s>>>(g, p.k_w0, v, dD, eps, G, fW);
    DWP_LAUNCH_CHECK();
}
template void launch_wet_residual6<float>(hipStream_t, const Plan &, const double *, const double *, const double *,
                                          const double *, float *, bool);
template void launch_wet_residual6<double>(hipStream_t, const Plan &, const double *, const double *,
                                           const double *, const double *, double *, bool);

void launch_grad6(hipStream_t s, const Plan &p, const double *phi, const double *lam, double *g_out) {
    const Grid6 g = make_grid6(p);
    dim3 gr((p.nx + SX - 1) / SX, (p.ny + SY - 1) / SY, p.nz), blk(SX, SY);
    k_grad6<<<gr, blk, 0, s>>>(g, phi, lam, g_out);
    DWP_LAUNCH_CHECK();
}

void launch_charge_potential(hipStream_t s, const Plan &p, const double *phi, const double *lam, double *psi) {
    const double h3 = p.h[0] * p.h[1] * p.h[2];
    k_charge_potential<<<grid1d6(p.N), 256, 0, s>>>(phi, lam, FOUR_PI / h3, psi, p.N);
    DWP_LAUNCH_CHECK();
}

void launch_scaled_product(hipStream_t s, const Plan &p, const double *gr, const double *m, const double *add,
                           double *out) {
    const double h3 = p.h[0] * p.h[1] * p.h[2];
    k_scaled_product<<<grid1d6(p.N), 256, 0, s>>>(gr, m, 1.0 / h3, add, out, p.N);
    DWP_LAUNCH_CHECK();
}

}  // namespace dwp
