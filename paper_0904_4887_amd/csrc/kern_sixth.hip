// The paper's sixth-order operator (Sec. II.F, Eqs. 16-18) on the full
// periodic box, its transpose, and the gradient kernels its adjoint needs.
//
//   A6 x   = sum_d G_d D1_d x + eps D2_d x,        G_d = D1_d eps,
//   A6^T y = sum_d -D1_d(G_d y) + D2_d(eps y),
// with the seven-point central stencils
//   D1 f_i = (1/h) sum_{n=1..3} a_n (f_{i+n} - f_{i-n}),   a = (3/4, -3/20, 1/60),
//   D2 f_i = (1/h^2) [b_0 f_i + sum_{n=1..3} b_n (f_{i+n} + f_{i-n})],
//   b = (-49/18, 3/2, -3/20, 1/90).
// G is computed once per permittivity.  The operators are LDS-tiled (below);
// the gradient kernel reads its wider stencil through the caches.  Every axis
// is periodic and at least 8 long, so a shift of up to 3 wraps at most once.
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

// LDS-tiled form of the operator, its transpose and their residual forms.  A
// block owns a 64 x 4 column tile and marches up a chunk of Z6 planes; at each
// plane it stages the tile plus a 3-cell halo in x and y in LDS and keeps the
// z neighbours (k-3 .. k+3) of its own column in registers, so that every
// input element is read from memory about once per plane instead of once per
// stencil point.
//   forward:    LDS holds x;              registers hold x at k-3..k+3.
//   transposed: LDS holds eps y, Gx y, Gy y (the products the transpose
//               differentiates);         registers hold eps y and Gz y.
// MODE 0: out = op x;  1: out = b - op x;  2: out (wet slab plane q, type T) =
// b - op x at box plane (k_w0 + q) mod nz.
constexpr int T6X = 64, T6Y = 4, H6 = 3;
constexpr int L6X = T6X + 2 * H6, L6Y = T6Y + 2 * H6, L6N = L6X * L6Y;
constexpr int T6N = T6X * T6Y;
constexpr int T6L = (L6N + T6N - 1) / T6N;  // tile loads per thread
constexpr int Z6 = 16;                      // planes per block

// TX, TE: storage of x and of eps, G (float32 for a float32 Krylov vector); the
// arithmetic is float64 either way
template <int MODE, bool TRANS, class T, class TX = double, class TE = double>
__global__ void __launch_bounds__(T6N)
k_op6_tile(Grid6 g, int k_w0, int nplanes, int tiles_x, int tiles_y, const TX *__restrict__ x,
           const TE *__restrict__ eps, const TE *__restrict__ G, const double *__restrict__ b,
           T *__restrict__ out) {
    __shared__ double s0[L6N], s1[TRANS ? L6N : 1], s2[TRANS ? L6N : 1];
    const int tid = threadIdx.x;
    const int tile = blockIdx.x;
    const int i0 = (tile % tiles_x) * T6X, j0 = ((tile / tiles_x) % tiles_y) * T6Y;
    const int q0 = (tile / (tiles_x * tiles_y)) * Z6, q1 = min(nplanes, q0 + Z6);
    const int lx = tid % T6X, ly = tid / T6X;
    const int i = i0 + lx, j = j0 + ly;
    const bool own = i < g.nx && j < g.ny;
    const size_t cc = own ? (size_t)j * g.nx + i : 0;  // in-plane offset of this thread's node
    const TE *Gx = G, *Gy = G + g.N, *Gz = G + 2 * g.N;
    // in-plane offsets of this thread's tile loads (periodic, any tile overhang)
    size_t lo[T6L];
#pragma unroll
    for (int m = 0; m < T6L; ++m) {
        const int q = min(tid + T6N * m, L6N - 1);
        const int xr = q % L6X, yr = q / L6X;
        const int gx = ((i0 - H6 + xr) % g.nx + g.nx) % g.nx, gy = ((j0 - H6 + yr) % g.ny + g.ny) % g.ny;
        lo[m] = (size_t)gy * g.nx + gx;
    }
    auto zplane = [&](int k) { return (size_t)(((k % g.nz) + g.nz) % g.nz) * g.plane; };
    const int kb = MODE == 2 ? k_w0 : 0;
    // z queues: a[d] and c[d] for plane k - 3 + d
    double a[7], c[7];
    auto zload = [&](int k, double &av, double &cv) {
        const size_t o = zplane(k) + cc;
        if (TRANS) {
            const double y = (double)x[o];
            av = (double)eps[o] * y;
            cv = (double)Gz[o] * y;
        } else {
            av = (double)x[o];
            cv = 0.0;
        }
    };
    const int kfirst = kb + q0;
#pragma unroll
    for (int d = 0; d < 6; ++d) zload(kfirst - 3 + d, a[d], c[d]);
    const int lc = (ly + H6) * L6X + lx + H6;
    const double ihx = g.ihx, ihy = g.ihy, ihz = g.ihz, ihx2 = g.ihx2, ihy2 = g.ihy2, ihz2 = g.ihz2;
    for (int q = q0; q < q1; ++q) {
        const int k = kb + q;
        zload(k + 3, a[6], c[6]);
        const size_t zp = zplane(k);
        __syncthreads();  // the previous plane's LDS reads are done
#pragma unroll
        for (int m = 0; m < T6L; ++m) {
            const int t = tid + T6N * m;
            if (t < L6N) {
                const size_t o = zp + lo[m];
                if (TRANS) {
                    const double y = (double)x[o];
                    s0[t] = (double)eps[o] * y;
                    s1[t] = (double)Gx[o] * y;
                    s2[t] = (double)Gy[o] * y;
                } else {
                    s0[t] = (double)x[o];
                }
            }
        }
        __syncthreads();
        if (own) {
            const size_t o = zp + cc;
            double v;
            if (!TRANS) {
                const double d1x = ihx * (A1 * (s0[lc + 1] - s0[lc - 1]) + A2 * (s0[lc + 2] - s0[lc - 2]) +
                                          A3 * (s0[lc + 3] - s0[lc - 3]));
                const double d1y = ihy * (A1 * (s0[lc + L6X] - s0[lc - L6X]) + A2 * (s0[lc + 2 * L6X] - s0[lc - 2 * L6X]) +
                                          A3 * (s0[lc + 3 * L6X] - s0[lc - 3 * L6X]));
                const double d1z = ihz * (A1 * (a[4] - a[2]) + A2 * (a[5] - a[1]) + A3 * (a[6] - a[0]));
                const double xc = a[3];
                const double d2 = ihx2 * (B0 * xc + B1 * (s0[lc + 1] + s0[lc - 1]) + B2 * (s0[lc + 2] + s0[lc - 2]) +
                                          B3 * (s0[lc + 3] + s0[lc - 3])) +
                                  ihy2 * (B0 * xc + B1 * (s0[lc + L6X] + s0[lc - L6X]) +
                                          B2 * (s0[lc + 2 * L6X] + s0[lc - 2 * L6X]) +
                                          B3 * (s0[lc + 3 * L6X] + s0[lc - 3 * L6X])) +
                                  ihz2 * (B0 * xc + B1 * (a[4] + a[2]) + B2 * (a[5] + a[1]) + B3 * (a[6] + a[0]));
                v = (double)Gx[o] * d1x + (double)Gy[o] * d1y + (double)Gz[o] * d1z + (double)eps[o] * d2;
            } else {
                const double d1x = ihx * (A1 * (s1[lc + 1] - s1[lc - 1]) + A2 * (s1[lc + 2] - s1[lc - 2]) +
                                          A3 * (s1[lc + 3] - s1[lc - 3]));
                const double d1y = ihy * (A1 * (s2[lc + L6X] - s2[lc - L6X]) + A2 * (s2[lc + 2 * L6X] - s2[lc - 2 * L6X]) +
                                          A3 * (s2[lc + 3 * L6X] - s2[lc - 3 * L6X]));
                const double d1z = ihz * (A1 * (c[4] - c[2]) + A2 * (c[5] - c[1]) + A3 * (c[6] - c[0]));
                const double pc = a[3];
                const double d2 = ihx2 * (B0 * pc + B1 * (s0[lc + 1] + s0[lc - 1]) + B2 * (s0[lc + 2] + s0[lc - 2]) +
                                          B3 * (s0[lc + 3] + s0[lc - 3])) +
                                  ihy2 * (B0 * pc + B1 * (s0[lc + L6X] + s0[lc - L6X]) +
                                          B2 * (s0[lc + 2 * L6X] + s0[lc - 2 * L6X]) +
                                          B3 * (s0[lc + 3 * L6X] + s0[lc - 3 * L6X])) +
                                  ihz2 * (B0 * pc + B1 * (a[4] + a[2]) + B2 * (a[5] + a[1]) + B3 * (a[6] + a[0]));
                v = -(d1x + d1y + d1z) + d2;
            }
            if (MODE == 0) out[o] = (T)v;
            else if (MODE == 1) out[o] = (T)(b[o] - v);
            else out[(size_t)q * g.plane + cc] = (T)(b[o] - v);
        }
#pragma unroll
        for (int d = 0; d < 6; ++d) { a[d] = a[d + 1]; c[d] = c[d + 1]; }
    }
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

// The sixth-order operator on the finest level of the wet multigrid: the
// slab's unknowns u (a ghosted level array, slab plane q at plane q + 1) are
// taken as zero on every plane outside the slab -- the Dirichlet data of the
// wet solve, reaching the three planes the seven-point stencils span beyond
// it -- and eps, G = D1 eps are the full-box arrays, slab plane q being box
// plane (k_w0 + q) mod nz.  MODE 0: one weighted-Jacobi sweep of A6_WW u = f,
// uout = u + omega (f - A6 u) / d, d = B0 eps sum_d 1/h_d^2 the diagonal of A6
// (the seven-point stencils couple points of equal red-black colour, so the
// colour ordering of the second-order smoother does not carry over); MODE 1:
// out = f - A6 u (slab planes, not ghosted).  Sums in float64.
template <class T, int MODE>
__global__ void __launch_bounds__(SX *SY)
k_wet6(const T *__restrict__ u, T *__restrict__ out, const T *__restrict__ f, const double *__restrict__ eps,
       const double *__restrict__ G, Grid6 g, int k_w0, int nw, double omega) {
    const int i = blockIdx.x * SX + threadIdx.x, j = blockIdx.y * SY + threadIdx.y, q = blockIdx.z;
    if (i >= g.nx || j >= g.ny) return;
    const size_t pl = g.plane;
    const size_t c = (size_t)j * g.nx + i;
    const size_t cb = (size_t)((k_w0 + q) % g.nz) * pl + c;
    auto U = [&](int qq, size_t off) -> double {
        return (qq < 0 || qq >= nw) ? 0.0 : (double)u[(size_t)(qq + 1) * pl + off];
    };
    const size_t row = (size_t)j * g.nx;
    const double u0 = U(q, c);
    double xs[3], ys[3], zs[3], xd[3], yd[3], zd[3];
#pragma unroll
    for (int n = 1; n <= 3; ++n) {
        const double xp = U(q, row + wrap(i + n, g.nx)), xm = U(q, row + wrap(i - n, g.nx));
        const double yp = U(q, (size_t)wrap(j + n, g.ny) * g.nx + i), ym = U(q, (size_t)wrap(j - n, g.ny) * g.nx + i);
        const double zp = U(q + n, c), zm = U(q - n, c);
        xs[n - 1] = xp + xm; xd[n - 1] = xp - xm;
        ys[n - 1] = yp + ym; yd[n - 1] = yp - ym;
        zs[n - 1] = zp + zm; zd[n - 1] = zp - zm;
    }
    const double d1x = g.ihx * (A1 * xd[0] + A2 * xd[1] + A3 * xd[2]);
    const double d1y = g.ihy * (A1 * yd[0] + A2 * yd[1] + A3 * yd[2]);
    const double d1z = g.ihz * (A1 * zd[0] + A2 * zd[1] + A3 * zd[2]);
    const double d2x = g.ihx2 * (B0 * u0 + B1 * xs[0] + B2 * xs[1] + B3 * xs[2]);
    const double d2y = g.ihy2 * (B0 * u0 + B1 * ys[0] + B2 * ys[1] + B3 * ys[2]);
    const double d2z = g.ihz2 * (B0 * u0 + B1 * zs[0] + B2 * zs[1] + B3 * zs[2]);
    const double e = eps[cb];
    const double a6 = G[cb] * d1x + G[g.N + cb] * d1y + G[2 * g.N + cb] * d1z + e * (d2x + d2y + d2z);
    const double fv = (double)f[(size_t)q * pl + c];
    if (MODE == 0) {
        const double d = e * B0 * (g.ihx2 + g.ihy2 + g.ihz2);
        out[(size_t)(q + 1) * pl + c] = (T)(u0 + omega * (fv - a6) / d);
    } else {
        out[(size_t)q * pl + c] = (T)(fv - a6);
    }
}

}  // namespace

void launch_d1eps(hipStream_t s, const Plan &p, const double *eps, double *G) {
    const Grid6 g = make_grid6(p);
    dim3 gr((p.nx + SX - 1) / SX, (p.ny + SY - 1) / SY, p.nz), blk(SX, SY);
    k_d1eps<<<gr, blk, 0, s>>>(g, eps, G);
    DWP_LAUNCH_CHECK();
}

template <int MODE, bool TRANS, class T, class TX = double, class TE = double>
static void launch_op6_tile(hipStream_t s, const Plan &p, int k_w0, int nplanes, const TX *x, const TE *eps,
                            const TE *G, const double *b, T *out) {
    const Grid6 g = make_grid6(p);
    const int tx = (p.nx + T6X - 1) / T6X, ty = (p.ny + T6Y - 1) / T6Y, tz = (nplanes + Z6 - 1) / Z6;
    k_op6_tile<MODE, TRANS, T, TX, TE><<<tx * ty * tz, T6N, 0, s>>>(g, k_w0, nplanes, tx, ty, x, eps, G, b, out);
    DWP_LAUNCH_CHECK();
}

void launch_apply6_f32(hipStream_t s, const Plan &p, const float *x, const float *eps, const float *G, float *out,
                       bool trans) {
    if (trans) launch_op6_tile<0, true, float, float, float>(s, p, 0, p.nz, x, eps, G, nullptr, out);
    else launch_op6_tile<0, false, float, float, float>(s, p, 0, p.nz, x, eps, G, nullptr, out);
}

void launch_apply6(hipStream_t s, const Plan &p, const double *x, const double *eps, const double *G,
                   const double *b, double *out, bool residual, bool trans) {
    if (residual) {
        if (trans) launch_op6_tile<1, true, double>(s, p, 0, p.nz, x, eps, G, b, out);
        else launch_op6_tile<1, false, double>(s, p, 0, p.nz, x, eps, G, b, out);
    } else {
        if (trans) launch_op6_tile<0, true, double>(s, p, 0, p.nz, x, eps, G, b, out);
        else launch_op6_tile<0, false, double>(s, p, 0, p.nz, x, eps, G, b, out);
    }
}

template <class T>
void launch_wet_residual6(hipStream_t s, const Plan &p, const double *v, const double *dD, const double *eps,
                          const double *G, T *fW, bool trans) {
    if (trans) launch_op6_tile<2, true, T>(s, p, p.k_w0, p.nw, dD, eps, G, v, fW);
    else launch_op6_tile<2, false, T>(s, p, p.k_w0, p.nw, dD, eps, G, v, fW);
}
template <class T>
void launch_wet6(hipStream_t s, const Plan &p, const Level &L, const T *u, T *out, const double *eps, const double *G,
                 bool smooth, double omega) {
    if (L.nx != p.nx || L.ny != p.ny || L.nw != p.nw) fail(DWP_EINVAL, "internal: not the finest wet level");
    dim3 gr((p.nx + SX - 1) / SX, (p.ny + SY - 1) / SY, L.nw), blk(SX, SY);
    if (smooth) k_wet6<T, 0><<<gr, blk, 0, s>>>(u, out, L.f.as<T>(), eps, G, make_grid6(p), p.k_w0, L.nw, omega);
    else k_wet6<T, 1><<<gr, blk, 0, s>>>(u, out, L.f.as<T>(), eps, G, make_grid6(p), p.k_w0, L.nw, omega);
    DWP_LAUNCH_CHECK();
}
template void launch_wet6<float>(hipStream_t, const Plan &, const Level &, const float *, float *, const double *,
                                 const double *, bool, double);
template void launch_wet6<double>(hipStream_t, const Plan &, const Level &, const double *, double *, const double *,
                                  const double *, bool, double);

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
