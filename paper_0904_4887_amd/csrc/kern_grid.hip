// Grid kernels: the 7-point conservative operator on the periodic box, the
// permittivity adjoint, the wet-slab extraction and combination, and the
// multigrid level kernels (red-black Gauss-Seidel, residual, full-weighting
// restriction, trilinear prolongation, coefficient coarsening).
//
// Operator (paper Eq. 3 in conservative form, face eps = mean of its nodes):
//   (A u)_n = sum over the 6 neighbours m of n of
//             1/2 (eps_n + eps_m) (u_m - u_n) / h_d^2.
#include <algorithm>
#include <mutex>

#include "dwp_internal.h"

namespace dwp {

namespace {

constexpr int BX = 64, BY = 4;

__device__ __forceinline__ int wrap_p(int i, int n) { return (i + 1 == n) ? 0 : i + 1; }
__device__ __forceinline__ int wrap_m(int i, int n) { return (i == 0) ? n - 1 : i - 1; }

// ---------------------------------------------------------------- full box

// The operator on arrays that are not all 16-byte aligned (the tiled kernel
// further down handles the aligned case): a thread owns one (i, j) column for
// ZM consecutive planes and keeps phi and eps of planes k-1, k, k+1 in
// registers, so each point loads its centre values once and its four in-plane
// neighbours through the cache.  Blocks are renumbered so that each of the 8
// XCDs (the hardware deals blocks round-robin over them) works on a
// contiguous range of tiles, i.e. of planes, keeping neighbour planes in its
// own L2.  mode 0: out = A phi; 1: out = b - A phi; 2: outW[kk] = b - A phi at
// box plane (k_w0 + kk) mod nz for kk < nplanes (b = v, output of type T).
constexpr int ZM = 8;

__device__ __forceinline__ int xcd_tile(int nb_real) {
    const int per = gridDim.x / 8;  // the grid is padded to a multiple of 8
    return (blockIdx.x % 8) * per + blockIdx.x / 8;
}

template <class T>
__device__ __forceinline__ T ld_at(const T *base, unsigned byte_off) {
    return *(const T *)((const char *)base + byte_off);
}

template <class T, int MODE, class TB, class TP, class TE>
__global__ void __launch_bounds__(BX *BY)
k_apply_zmarch(const TP *__restrict__ phi, const TE *__restrict__ eps, const TB *__restrict__ b,
               T *__restrict__ out, int nx, int ny, int nz, double cx, double cy, double cz, int k_w0,
               int nplanes, int tiles_x, int tiles_y, int nb_real) {
    const int t = xcd_tile(nb_real);
    if (t >= nb_real) return;
    const int tx = t % tiles_x, ty = (t / tiles_x) % tiles_y, tz = t / (tiles_x * tiles_y);
    const int i = tx * BX + threadIdx.x, j = ty * BY + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const size_t plane = (size_t)nx * ny;
    // byte offsets inside a plane (the plane base pointers are uniform)
    const int col = j * nx + i;
    // element offsets inside a plane (phi and eps are read at the same ones)
    const unsigned oc = (unsigned)col;
    const unsigned oxp = (unsigned)(j * nx + wrap_p(i, nx)), oxm = (unsigned)(j * nx + wrap_m(i, nx));
    const unsigned oyp = (unsigned)(wrap_p(j, ny) * nx + i), oym = (unsigned)(wrap_m(j, ny) * nx + i);
    const int kk0 = tz * ZM, kk1 = min(nplanes, kk0 + ZM);
    auto boxk = [&](int kk) { return MODE == 2 ? (k_w0 + kk) % nz : kk; };
    auto P = [&](int k) { return phi + (size_t)k * plane; };
    auto E = [&](int k) { return eps + (size_t)k * plane; };
    auto lp = [](const TP *base, unsigned o) { return (double)base[o]; };
    // Software pipeline: the centre values of plane k+1 and the in-plane
    // neighbours of plane k are loaded one plane ahead of their use.
    int k = boxk(kk0);
    const int km = wrap_m(k, nz);
    double pm = lp(P(km), oc), em = E(km)[oc], p0 = lp(P(k), oc), e0 = E(k)[oc];
    double nb[8];
    auto load_nb = [&](int kq, double *o) {
        const TP *pq = P(kq);
        const TE *ee = E(kq);
        o[0] = lp(pq, oxp); o[1] = ee[oxp]; o[2] = lp(pq, oxm); o[3] = ee[oxm];
        o[4] = lp(pq, oyp); o[5] = ee[oyp]; o[6] = lp(pq, oym); o[7] = ee[oym];
    };
    load_nb(k, nb);
    int kp = wrap_p(k, nz);
    double pp = lp(P(kp), oc), ep = E(kp)[oc];
    for (int kk = kk0; kk < kk1; ++kk) {
        // prefetch for plane kk + 1 (clamped inside the chunk: always a valid address)
        const bool more = kk + 1 < kk1;
        const int kn = wrap_p(kp, nz);
        const int kq = more ? kn : kp;
        double nb2[8];
        load_nb(kp, nb2);
        const double pq = lp(P(kq), oc), eq = E(kq)[oc];
        double acc = cx * ((e0 + nb[1]) * (nb[0] - p0) + (e0 + nb[3]) * (nb[2] - p0)) +
                     cy * ((e0 + nb[5]) * (nb[4] - p0) + (e0 + nb[7]) * (nb[6] - p0)) +
                     cz * ((e0 + ep) * (pp - p0) + (e0 + em) * (pm - p0));
        acc *= 0.5;
        if (MODE == 0) out[(size_t)k * plane + col] = (T)acc;
        else if (MODE == 1) out[(size_t)k * plane + col] = (T)((double)b[(size_t)k * plane + col] - acc);
        else out[(size_t)kk * plane + col] = (T)((double)b[(size_t)k * plane + col] - acc);
        pm = p0; em = e0; p0 = pp; e0 = ep; pp = pq; ep = eq;
#pragma unroll
        for (int q = 0; q < 8; ++q) nb[q] = nb2[q];
        k = kp; kp = kn;
    }
}

// The same operator with the plane tile staged in LDS.  A block owns a tile
// of 64 x 8 points for a chunk of apply_zch planes; each thread owns two adjacent x
// points.  Per plane step the block loads the next plane's tile (phi and eps,
// 1-cell halo in y, 2 in x to keep 16-byte alignment) with 16-byte loads into
// a two-slot LDS ring, each thread loads its own two centre values three
// planes ahead, and the in-plane neighbours come from LDS while the z
// neighbours stay in registers.  One barrier per step: the slot written at
// step k was last read at step k-1.  Needs nx even and every array 16-byte
// aligned (the launcher checks).
constexpr int ATX = 64, ATY = 8;            // points per tile
constexpr int AHX2 = (ATX + 4) / 2;         // double2 per LDS row (x halo 2)
constexpr int AHY = ATY + 2;                // rows (y halo 1)
constexpr int AQ = AHX2 * AHY;              // double2 items per field per plane
constexpr int AQT = (AQ + 255) / 256;       // per thread
// planes per block: 16 for the full-box operator, 12 for the wet residual
// (measured best at 192 x 192 x 384 among 8, 12, 16, 24 and 32)
template <int MODE> constexpr int apply_zch() { return MODE == 2 ? 12 : 16; }

// two consecutive values of a float64 or float32 field at element offset o, as double2
__device__ __forceinline__ double2 ld2(const double *base, unsigned o) { return ld_at((const double2 *)base, o * 8u); }
__device__ __forceinline__ double2 ld2(const float *base, unsigned o) {
    const float2 v = ld_at((const float2 *)base, o * 4u);
    return make_double2(v.x, v.y);
}
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld2(const _Float16 *base, unsigned o) {
    const half2v v = ld_at((const half2v *)base, o * 2u);
    return make_double2((double)v[0], (double)v[1]);
}

template <class T, int MODE, class TB, class TP, class TE>
__global__ void __launch_bounds__(256)
k_apply_tile(const TP *__restrict__ phi, const TE *__restrict__ eps, const TB *__restrict__ b,
             T *__restrict__ out, int nx, int ny, int nz, double cx, double cy, double cz, int k_w0, int nplanes,
             int tiles_x, int tiles_y, int nb_real) {
    __shared__ double2 sp[2][AQT * 256], se[2][AQT * 256];
    const int t = xcd_tile(nb_real);
    if (t >= nb_real) return;
    const int i0 = (t % tiles_x) * ATX, j0 = ((t / tiles_x) % tiles_y) * ATY;
    constexpr int ZCH = apply_zch<MODE>();
    const int kk0 = (t / (tiles_x * tiles_y)) * ZCH, kk1 = min(nplanes, kk0 + ZCH);
    const int tid = threadIdx.x + 32 * threadIdx.y;
    const size_t plane = (size_t)nx * ny;
    unsigned oq[AQT];
#pragma unroll
    for (int m = 0; m < AQT; ++m) {
        const int q = min(tid + 256 * m, AQ - 1);  // padding lanes repeat the last item
        const int xr = q % AHX2, yr = q / AHX2;
        const int x = ((i0 - 2 + 2 * xr) % nx + nx) % nx, y = ((j0 - 1 + yr) % ny + ny) % ny;
        oq[m] = (unsigned)(y * nx + x);  // element offset
    }
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int gi = i0 + 2 * lx, gj = j0 + ly;
    const bool own = gi < nx && gj < ny;
    const unsigned oc = own ? (unsigned)(gj * nx + gi) : 0u;  // element offset
    auto wrapk = [&](int k) { return k < 0 ? k + nz : (k >= nz ? k - nz : k); };
    auto P = [&](int k) { return phi + (size_t)wrapk(k) * plane; };
    auto E = [&](int k) { return eps + (size_t)wrapk(k) * plane; };
    const int kb0 = MODE == 2 ? (k_w0 + kk0) % nz : kk0;  // box plane of the first step
    double2 tp[AQT], te[AQT];
    auto fetch_tile = [&](int k) {
        const TP *pp = P(k);
        const TE *ee = E(k);
#pragma unroll
        for (int m = 0; m < AQT; ++m) {
            tp[m] = ld2(pp, oq[m]);
            te[m] = ld2(ee, oq[m]);
        }
    };
    auto stash = [&](int slot) {
#pragma unroll
        for (int m = 0; m < AQT; ++m) {
            sp[slot][tid + 256 * m] = tp[m];
            se[slot][tid + 256 * m] = te[m];
        }
    };
    double2 pm = ld2(P(kb0 - 1), oc), em = ld2(E(kb0 - 1), oc);
    double2 p0 = ld2(P(kb0), oc), e0 = ld2(E(kb0), oc);
    double2 pp = ld2(P(kb0 + 1), oc), ep = ld2(E(kb0 + 1), oc);
    fetch_tile(kb0);
    stash(0);
    fetch_tile(kb0 + 1);
    double2 pn = ld2(P(kb0 + 2), oc), en = ld2(E(kb0 + 2), oc);
    const int r = ly + 1, c2 = lx + 1;
    for (int kk = kk0; kk < kk1; ++kk) {
        const int s = (kk - kk0) & 1;
        const int k = wrapk(kb0 + (kk - kk0));  // box plane of this step
        __syncthreads();
        stash(s ^ 1);  // plane k + 1
        fetch_tile(k + 2);
        const double2 pq = ld2(P(k + 3), oc), eq = ld2(E(k + 3), oc);
        const double2 *lp = sp[s], *le = se[s];
        const double2 xl_p = lp[r * AHX2 + c2 - 1], xl_e = le[r * AHX2 + c2 - 1];
        const double2 xr_p = lp[r * AHX2 + c2 + 1], xr_e = le[r * AHX2 + c2 + 1];
        const double2 yu_p = lp[(r + 1) * AHX2 + c2], yu_e = le[(r + 1) * AHX2 + c2];
        const double2 yd_p = lp[(r - 1) * AHX2 + c2], yd_e = le[(r - 1) * AHX2 + c2];
        double a0 = cx * ((e0.x + e0.y) * (p0.y - p0.x) + (e0.x + xl_e.y) * (xl_p.y - p0.x)) +
                    cy * ((e0.x + yu_e.x) * (yu_p.x - p0.x) + (e0.x + yd_e.x) * (yd_p.x - p0.x)) +
                    cz * ((e0.x + ep.x) * (pp.x - p0.x) + (e0.x + em.x) * (pm.x - p0.x));
        double a1 = cx * ((e0.y + xr_e.x) * (xr_p.x - p0.y) + (e0.y + e0.x) * (p0.x - p0.y)) +
                    cy * ((e0.y + yu_e.y) * (yu_p.y - p0.y) + (e0.y + yd_e.y) * (yd_p.y - p0.y)) +
                    cz * ((e0.y + ep.y) * (pp.y - p0.y) + (e0.y + em.y) * (pm.y - p0.y));
        a0 *= 0.5;
        a1 *= 0.5;
        if (own) {
            const size_t dst = (size_t)(MODE == 2 ? kk : k) * plane + (size_t)(gj * nx + gi);
            if (MODE == 0) {
                if constexpr (sizeof(T) == 8) {
                    *(double2 *)(out + dst) = make_double2(a0, a1);
                } else {
                    *(float2 *)(out + dst) = make_float2((float)a0, (float)a1);
                }
            } else {
                const double2 bv = ld2(b + (size_t)k * plane, oc);
                const double bx = bv.x, by = bv.y;
                out[dst] = (T)(bx - a0);
                out[dst + 1] = (T)(by - a1);
            }
        }
        pm = p0; em = e0; p0 = pp; e0 = ep; pp = pn; ep = en; pn = pq; en = eq;
    }
}

// G_n = sum_d 1/2 [(D+ phi)^2 + (D- phi)^2] at node n (the faces around n carry
// half of eps_n each).  MODE 0: g = scale G (scale = -h^3 / 8 pi: dE/d eps_n,
// Eq. 11); MODE 1: g = scale G m_n (scale = -1 / 8 pi, m = d eps / d rho: V_eps
// of Eq. 6 on the grid); MODE 2: g = phi_n + that (the density derivative of the
// energy, Eq. 5).
template <int MODE>
__global__ void __launch_bounds__(BX *BY)
k_eps_gradient(const double *__restrict__ phi, const double *__restrict__ m, double *__restrict__ g, int nx,
               int ny, int nz, double ihx, double ihy, double ihz, double scale) {
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= nx || j >= ny) return;
    const size_t plane = (size_t)nx * ny;
    const size_t row = (size_t)k * plane + (size_t)j * nx;
    const size_t c = row + i;
    const double p0 = phi[c];
    double dxp = (phi[row + wrap_p(i, nx)] - p0) * ihx, dxm = (p0 - phi[row + wrap_m(i, nx)]) * ihx;
    double dyp = (phi[(size_t)k * plane + (size_t)wrap_p(j, ny) * nx + i] - p0) * ihy;
    double dym = (p0 - phi[(size_t)k * plane + (size_t)wrap_m(j, ny) * nx + i]) * ihy;
    double dzp = (phi[(size_t)wrap_p(k, nz) * plane + (size_t)j * nx + i] - p0) * ihz;
    double dzm = (p0 - phi[(size_t)wrap_m(k, nz) * plane + (size_t)j * nx + i]) * ihz;
    double v = scale * 0.5 * (dxp * dxp + dxm * dxm + dyp * dyp + dym * dym + dzp * dzp + dzm * dzm);
    if (MODE >= 1) v *= m[c];
    if (MODE == 2) v += p0;
    g[c] = v;
}

// Eq. 7 and its derivative Eq. 8 at every node, with the density read as
// max(rho, 0): 1 + (eps_inf - 1)/2 (1 + (1 - p)/(1 + p)) = 1 + (eps_inf - 1)/(1 + p)
// with p = (rho/rho_0)^(2 beta), and d eps/d rho = -(eps_inf - 1) 2 beta p / (rho (1 + p)^2).
// Requires 2 beta > 1, so that the derivative is 0 at zero density.
__global__ void k_eps_density(const double *__restrict__ rho, double *__restrict__ eps, double *__restrict__ deps,
                              size_t n, double eps_inf, double inv_rho0, double two_beta) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const double r = fmax(rho[t], 0.0);
        double e = eps_inf, d = 0.0;
        if (r > 0.0) {
            const double p = pow(r * inv_rho0, two_beta);
            const double q = 1.0 / (1.0 + p);
            e = 1.0 + (eps_inf - 1.0) * q;
            d = (1.0 - eps_inf) * two_beta * (p / r) * q * q;
        }
        eps[t] = e;
        deps[t] = d;
    }
}

// out_n = scale * sum_d 1/2 [(D+_d a)(D+_d b) + (D-_d a)(D-_d b)]: the derivative
// of the bilinear form a.A b with respect to the node permittivity eps_n
// (times -scale), used for gradients through phi.
__global__ void __launch_bounds__(BX *BY)
k_eps_pair(const double *__restrict__ pa, const double *__restrict__ pb, double *__restrict__ g, int nx, int ny,
           int nz, double ihx, double ihy, double ihz, double scale) {
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= nx || j >= ny) return;
    const size_t plane = (size_t)nx * ny;
    const size_t row = (size_t)k * plane + (size_t)j * nx;
    const size_t c = row + i;
    const size_t nbr[6] = {row + wrap_p(i, nx), row + wrap_m(i, nx),
                           (size_t)k * plane + (size_t)wrap_p(j, ny) * nx + i,
                           (size_t)k * plane + (size_t)wrap_m(j, ny) * nx + i,
                           (size_t)wrap_p(k, nz) * plane + (size_t)j * nx + i,
                           (size_t)wrap_m(k, nz) * plane + (size_t)j * nx + i};
    const double ih[3] = {ihx, ihy, ihz};
    double acc = 0.0;
    for (int q = 0; q < 6; ++q) {
        const double da = (pa[nbr[q]] - pa[c]) * ih[q / 2], db = (pb[nbr[q]] - pb[c]) * ih[q / 2];
        acc += da * db;
    }
    g[c] = scale * 0.5 * acc;
}

// ---------------------------------------------------------------- vectors
__global__ void k_fill(double *x, double v, size_t n) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        x[t] = v;
}
template <class T>
__global__ void k_zero(T *x, size_t n) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        x[t] = T(0);
}
// mode 0: x *= 1/sqrt(*den_sq) (0 when *den_sq is 0: a breakdown leaves a zero
// vector); mode 1: x *= *num
__global__ void k_scale_dev(double *x, const double *num, const double *den_sq, size_t n, int mode) {
    const double s = mode == 0 ? (*den_sq > 0.0 ? 1.0 / sqrt(*den_sq) : 0.0) : *num;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        x[t] *= s;
}
// b = -4 pi (rho - mean), mean = (*sum) * inv_n
__global__ void k_rhs(const double *rho, const double *sum, double inv_n, double *b, size_t n) {
    const double m = *sum * inv_n;
    const double fpi = -4.0 * 3.14159265358979323846;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        b[t] = fpi * (rho[t] - m);
}
__global__ void k_sub_mean(double *x, const double *sum, double inv_n, size_t n) {
    const double m = *sum * inv_n;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        x[t] -= m;
}
__global__ void k_mul(double *y, const double *a, const double *x, size_t n) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        y[t] = a[t] * x[t];
}
__global__ void k_axpby(double *out, double a, const double *x, double b, const double *y, size_t n) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        out[t] = y ? a * x[t] + b * y[t] : a * x[t];
}
__global__ void k_rsqrt(const double *eps, double *s, size_t n) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        s[t] = 1.0 / sqrt(eps[t]);
}
// flags[blockIdx.x]: bit 0 non-finite, bit 1 below one (each block writes its own word)
__global__ void k_check(const double *x, size_t n, int *flags, int check_ge1) {
    __shared__ int sflag[256];
    int f = 0;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const double v = x[t];
        if (!isfinite(v)) f |= 1;
        else if (check_ge1 && v < 1.0) f |= 2;
    }
    sflag[threadIdx.x] = f;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sflag[threadIdx.x] |= sflag[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) flags[blockIdx.x] = sflag[0];
}

// ---------------------------------------------------------------- wet slab <-> box

// z at box plane (k_w0 + kk) mod nz += uW (ghosted plane kk + 1).  Grid:
// (plane chunks, kk); PAIRS: two consecutive points per thread (plane even,
// z 16-byte aligned); QUADS (float32 both): four, 16-byte accesses (plane a
// multiple of 4).
template <class T, bool PAIRS, class TZ, bool QUADS = false>
__global__ void k_wet_add(const T *__restrict__ uW, TZ *__restrict__ z, int plane, int nz, int k_w0) {
    const int kk = blockIdx.y;
    const int k = (k_w0 + kk) % nz;
    const T *src = uW + (size_t)(kk + 1) * plane;
    TZ *dst = z + (size_t)k * plane;
    const int q = (QUADS ? 4 : PAIRS ? 2 : 1) * (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= plane) return;
    if constexpr (QUADS) {
        static_assert(sizeof(T) == 4 && sizeof(TZ) == 4, "float32 quads");
        float4 v = *reinterpret_cast<float4 *>(dst + q);
        const float4 u = *reinterpret_cast<const float4 *>(src + q);
        v.x = (float)((double)v.x + (double)u.x);
        v.y = (float)((double)v.y + (double)u.y);
        v.z = (float)((double)v.z + (double)u.z);
        v.w = (float)((double)v.w + (double)u.w);
        *reinterpret_cast<float4 *>(dst + q) = v;
    } else if constexpr (PAIRS && sizeof(TZ) == 8) {
        double2 v = *reinterpret_cast<double2 *>(dst + q);
        v.x += (double)src[q];
        v.y += (double)src[q + 1];
        *reinterpret_cast<double2 *>(dst + q) = v;
    } else if constexpr (PAIRS) {
        float2 v = *reinterpret_cast<float2 *>(dst + q);
        v.x = (float)((double)v.x + (double)src[q]);
        v.y = (float)((double)v.y + (double)src[q + 1]);
        *reinterpret_cast<float2 *>(dst + q) = v;
    } else {
        dst[q] = (TZ)((double)dst[q] + (double)src[q]);
    }
}

// epsW ghosted plane p <- eps at box plane (k_w0 - 1 + p) mod nz, p in [0, nw + 2)
template <class T>
__global__ void k_wet_eps(const double *__restrict__ eps, T *__restrict__ epsW, int nx, int ny, int nz,
                          int k_w0, int nw) {
    const size_t plane = (size_t)nx * ny;
    const size_t total = plane * (nw + 2);
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        const int p = (int)(t / plane);
        const size_t rem = t - (size_t)p * plane;
        const int k = ((k_w0 - 1 + p) % nz + nz) % nz;
        epsW[t] = (T)eps[(size_t)k * plane + rem];
    }
}

// ---------------------------------------------------------------- levels
struct LevelArgs {
    int nx, ny, nw;
    float cxf, cyf, czf;
    double cx, cy, cz;
};

template <class T> __device__ __forceinline__ T cxv(const LevelArgs &a, int d);
template <> __device__ __forceinline__ float cxv<float>(const LevelArgs &a, int d) {
    return d == 0 ? a.cxf : (d == 1 ? a.cyf : a.czf);
}
template <> __device__ __forceinline__ double cxv<double>(const LevelArgs &a, int d) {
    return d == 0 ? a.cx : (d == 1 ? a.cy : a.cz);
}

// Gauss-Seidel value (off - f) / diag through the hardware reciprocal.  The
// smoother only shapes the preconditioner, so the last bit of the quotient
// does not matter; in FP64 two Newton steps bring the estimate to full
// precision.
__device__ __forceinline__ float gs_value(float off, float f, float diag) {
    return (off - f) * __builtin_amdgcn_rcpf(diag);
}
__device__ __forceinline__ double gs_value(double off, double f, double diag) {
    double r = __builtin_amdgcn_rcp(diag);
    double e = __builtin_fma(-diag, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-diag, r, 1.0);
    r = __builtin_fma(r, e, r);
    return (off - f) * r;
}
}  // namespace
}  // namespace dwp
#include "band_sweep.h"
#include "band_apply.h"
#include "band_restrict.h"
namespace dwp {
namespace {

// Row-band variant of k_apply_tile (per-thread code in band_apply.h):
// (ty + 2) * nx / W threads, the tile -> (band, chunk) order of k_sweep_band.
template <int MODE, class TS, class TB>
__global__ void __launch_bounds__(1024) k_apply_band(ApplyArgs<TS, TB> a, int nb_real, int gb) {
    extern __shared__ __align__(16) unsigned char apply_lds[];
    const int t = xcd_tile(nb_real);
    if (t >= nb_real) return;
    const int nchunks = (a.nplanes + a.kc - 1) / a.kc;
    const int g = t / (gb * nchunks), q = t - g * gb * nchunks;
    const int chunk = q / gb, band = g * gb + (q - (q / gb) * gb);
    BandApply<MODE, TS, TB> b;
    b.init(a, reinterpret_cast<TS *>(apply_lds), band, chunk, threadIdx.x);
    b.prologue();
    __syncthreads();
    for (int kk = b.kk0; kk < b.kk1; ++kk) {
        b.step(kk);
        __syncthreads();
    }
}

// Row-band variant of k_resid_restrict (per-thread code in band_restrict.h):
// (2 tyc + 3) * nx / W threads, the tile -> (band, chunk) order of k_sweep_band.
template <class T, int W, bool ZC>
__global__ void __launch_bounds__(1024) k_resid_restrict_band(RestrictArgs<T> a, int nb_real, int gb) {
    extern __shared__ __align__(16) unsigned char restrict_lds[];
    const int t = xcd_tile(nb_real);
    if (t >= nb_real) return;
    const int nchunks = (a.nwc + a.kcc - 1) / a.kcc;
    const int g = t / (gb * nchunks), q = t - g * gb * nchunks;
    const int chunk = q / gb, band = g * gb + (q - (q / gb) * gb);
    BandRestrict<T, W, ZC> b;
    b.init(a, reinterpret_cast<T *>(restrict_lds), band, chunk, threadIdx.x);
    b.prologue();
    __syncthreads();
    for (int k = b.k0; k <= b.k1; ++k) {
        b.step(k);
        __syncthreads();
    }
}



// Neighbour sums at ghosted index g of slab point (i, j): returns the
// off-diagonal sum  sum_m w_m u_m  and the diagonal  sum_m w_m,
// w_m = 1/2 (eps_n + eps_m) / h_d^2.
template <class T>
__device__ __forceinline__ void level_sums(const T *__restrict__ u, const T *__restrict__ e,
                                           const LevelArgs &a, int i, int j, int g, T &off,
                                           T &diag) {
    // 32-bit offsets: the levels that use this (the bottom of the V-cycle)
    // hold a few thousand points
    const int plane = a.nx * a.ny;
    const int rowbase = g - i;
    const int xp = rowbase + wrap_p(i, a.nx), xm = rowbase + wrap_m(i, a.nx);
    const int pbase = g - j * a.nx;  // start of (plane, row 0) + i
    const int yp = pbase + wrap_p(j, a.ny) * a.nx;
    const int ym = pbase + wrap_m(j, a.ny) * a.nx;
    const int zp = g + plane, zm = g - plane;
    const T e0 = e[g];
    const T cx = cxv<T>(a, 0), cy = cxv<T>(a, 1), cz = cxv<T>(a, 2);
    const T wxp = cx * (e0 + e[xp]), wxm = cx * (e0 + e[xm]);
    const T wyp = cy * (e0 + e[yp]), wym = cy * (e0 + e[ym]);
    const T wzp = cz * (e0 + e[zp]), wzm = cz * (e0 + e[zm]);
    off = T(0.5) * (wxp * u[xp] + wxm * u[xm] + wyp * u[yp] + wym * u[ym] + wzp * u[zp] + wzm * u[zm]);
    diag = T(0.5) * (wxp + wxm + wyp + wym + wzp + wzm);
}

// The same sums for kernels whose block lies in one plane: u0 and e0 point
// at the ghosted plane BELOW the point (uniform over the block), so every
// neighbour sits at a non-negative 32-bit offset from them.
template <class T>
__device__ __forceinline__ void level_sums_u(const T *__restrict__ u0, const T *__restrict__ e0p,
                                             const LevelArgs &a, int i, int j, T &off, T &diag, T &uc) {
    const int plane = a.nx * a.ny;
    const int c = plane + j * a.nx + i;
    const int rowb = c - i;
    const int xp = rowb + wrap_p(i, a.nx), xm = rowb + wrap_m(i, a.nx);
    const int yp = c + (wrap_p(j, a.ny) - j) * a.nx, ym = c + (wrap_m(j, a.ny) - j) * a.nx;
    const T e0 = e0p[c];
    const T cx = cxv<T>(a, 0), cy = cxv<T>(a, 1), cz = cxv<T>(a, 2);
    const T wxp = cx * (e0 + e0p[xp]), wxm = cx * (e0 + e0p[xm]);
    const T wyp = cy * (e0 + e0p[yp]), wym = cy * (e0 + e0p[ym]);
    const T wzp = cz * (e0 + e0p[c + plane]), wzm = cz * (e0 + e0p[c - plane]);
    off = T(0.5) * (wxp * u0[xp] + wxm * u0[xm] + wyp * u0[yp] + wym * u0[ym] + wzp * u0[c + plane] +
                    wzm * u0[c - plane]);
    diag = T(0.5) * (wxp + wxm + wyp + wym + wzp + wzm);
    uc = u0[c];
}

// r = f - A u at every slab point (r, f not ghosted)
template <class T>
__global__ void __launch_bounds__(BX *BY)
k_level_residual(const T *__restrict__ u, const T *__restrict__ e, const T *__restrict__ f,
                 T *__restrict__ r, LevelArgs a) {
    const int i = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int kk = blockIdx.z;
    if (i >= a.nx || j >= a.ny) return;
    const size_t plane = (size_t)a.nx * a.ny;
    const T *u0 = u + (size_t)kk * plane, *e0 = e + (size_t)kk * plane;
    const T *fk = f + (size_t)kk * plane;
    T *rk = r + (size_t)kk * plane;
    T off, diag, uc;
    level_sums_u(u0, e0, a, i, j, off, diag, uc);
    const int li = j * a.nx + i;
    rk[li] = fk[li] - (off - diag * uc);
}

// One colour of red-black Gauss-Seidel: points with (i + j + kk) % 2 == color
// take u = (off - f) / diag.  nx is even, so the colouring is consistent
// across the periodic wrap and no two points of one colour are neighbours.
template <class T>
__global__ void __launch_bounds__(BX *BY)
k_level_smooth(T *__restrict__ u, const T *__restrict__ e, const T *__restrict__ f, LevelArgs a,
               int color) {
    const int t = blockIdx.x * BX + threadIdx.x;
    const int j = blockIdx.y * BY + threadIdx.y;
    const int kk = blockIdx.z;
    const int i = 2 * t + ((j + kk + color) & 1);
    if (i >= a.nx || j >= a.ny) return;
    const size_t plane = (size_t)a.nx * a.ny;
    T *u0 = u + (size_t)kk * plane;
    const T *e0 = e + (size_t)kk * plane;
    T off, diag, uc;
    level_sums_u<T>(u0, e0, a, i, j, off, diag, uc);
    const int li = j * a.nx + i;
    u0[a.nx * a.ny + li] = gs_value(off, f[(size_t)kk * plane + li], diag);
}


// Full weighting: 1/4, 1/2, 1/4 along every coarsened direction (periodic in
// x, y; in z the three fine planes 2kc, 2kc+1, 2kc+2 all lie inside the slab).
// The coarse unknowns (ghosted array uc) are zeroed in the same launch.
// Grid: (x tiles, y tiles, coarse plane kc).
template <class T>
__global__ void __launch_bounds__(BX *BY)
k_restrict(const T *__restrict__ rf, T *__restrict__ fc, T *__restrict__ uc, int nxf, int nyf, int nxc, int nyc,
           int nwc, int zc) {
    const int ic = blockIdx.x * BX + threadIdx.x, jc = blockIdx.y * BY + threadIdx.y, kc = blockIdx.z;
    if (ic >= nxc || jc >= nyc) return;
    const size_t planec = (size_t)nxc * nyc, planef = (size_t)nxf * nyf;
    const int cidx = jc * nxc + ic;
    uc[(size_t)(kc + 1) * planec + cidx] = T(0);
    if (kc == 0) uc[cidx] = T(0);
    if (kc == nwc - 1) uc[(size_t)(nwc + 1) * planec + cidx] = T(0);
    const T w3[3] = {T(0.25), T(0.5), T(0.25)};
    const int i0 = 2 * ic;
    const int im = i0 == 0 ? nxf - 1 : i0 - 1, ip = i0 + 1 == nxf ? 0 : i0 + 1;
    T acc = T(0);
    const int nzt = zc ? 3 : 1;
    for (int dz = 0; dz < nzt; ++dz) {
        const int kf = zc ? 2 * kc + dz : kc;
        const T wz = zc ? w3[dz] : T(1);
        const T *pf = rf + (size_t)kf * planef;
        for (int dy = -1; dy <= 1; ++dy) {
            const int jf = (2 * jc + dy + nyf) % nyf;
            const T *row = pf + jf * nxf;
            const T sx = T(0.25) * row[im] + T(0.5) * row[i0] + T(0.25) * row[ip];
            acc += wz * w3[dy + 1] * sx;
        }
    }
    fc[(size_t)kc * planec + cidx] = acc;
}

// Trilinear interpolation of the coarse correction, added to the fine
// unknowns.  x and y are always coarsened by 2, z when zc.  One thread per
// fine x pair (2 ic, 2 ic + 1): the even point takes the coarse value at ic,
// the odd one the mean of ic and ic + 1, so both come from the same two coarse
// values per contributing coarse row and nothing diverges inside a wave (one
// wave spans a single fine row j; a block a single fine plane).  Grid: (pair
// tiles, rows, fine plane kf).
template <class T>
__global__ void __launch_bounds__(BX *BY)
k_prolong_add(T *__restrict__ uf, const T *__restrict__ uc, int nxf, int nyf, int nxc, int nyc, int zc) {
    const int ic = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, kf = blockIdx.z;
    if (ic >= nxc || j >= nyf) return;
    const size_t planef = (size_t)nxf * nyf, planec = (size_t)nxc * nyc;
    const int icp = ic + 1 == nxc ? 0 : ic + 1;
    // coarse rows (y) and planes (z, ghosted index) with their weights
    const int jc0 = j >> 1, jc1 = (j & 1) ? (jc0 + 1 == nyc ? 0 : jc0 + 1) : jc0;
    const T wy1 = (j & 1) ? T(0.5) : T(0), wy0 = T(1) - wy1;
    int pz0, pz1;
    T wz1;
    if (zc) {
        if (kf & 1) { pz0 = pz1 = (kf - 1) / 2 + 1; wz1 = T(0); }
        else { pz0 = kf / 2; pz1 = kf / 2 + 1; wz1 = T(0.5); }
    } else {
        pz0 = pz1 = kf + 1;
        wz1 = T(0);
    }
    const T wz0 = T(1) - wz1;
    T ev = T(0), od = T(0);
    auto row = [&](int pz, int jc, T w) {
        const T *r = uc + (size_t)pz * planec + (size_t)jc * nxc;
        const T a = r[ic], b = r[icp];
        ev += w * a;
        od += w * (T(0.5) * (a + b));
    };
    row(pz0, jc0, wz0 * wy0);
    if (wy1 != T(0)) row(pz0, jc1, wz0 * wy1);
    if (wz1 != T(0)) {
        row(pz1, jc0, wz1 * wy0);
        if (wy1 != T(0)) row(pz1, jc1, wz1 * wy1);
    }
    T *f = uf + (size_t)(kf + 1) * planef + (size_t)j * nxf + 2 * ic;
    f[0] += ev;
    f[1] += od;
}

// The same interpolation with CP coarse columns (2 CP fine points, 16 bytes
// of T) per thread: the fine points are read and written as one vector, and
// the CP + 1 coarse values of each contributing coarse row are loaded once.
// Same arithmetic, in the same order, as k_prolong_add.  Needs nxc a
// multiple of CP (the launcher checks).
template <class T, int CP>
__global__ void __launch_bounds__(BX *BY)
k_prolong_add_v(T *__restrict__ uf, const T *__restrict__ uc, int nxf, int nyf, int nxc, int nyc, int zc) {
    typedef typename BandVec<T, 2 * CP>::V V;
    const int q = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y, kf = blockIdx.z;
    const int ic0 = q * CP;
    if (ic0 >= nxc || j >= nyf) return;
    const size_t planef = (size_t)nxf * nyf, planec = (size_t)nxc * nyc;
    const int jc0 = j >> 1, jc1 = (j & 1) ? (jc0 + 1 == nyc ? 0 : jc0 + 1) : jc0;
    const T wy1 = (j & 1) ? T(0.5) : T(0), wy0 = T(1) - wy1;
    int pz0, pz1;
    T wz1;
    if (zc) {
        if (kf & 1) { pz0 = pz1 = (kf - 1) / 2 + 1; wz1 = T(0); }
        else { pz0 = kf / 2; pz1 = kf / 2 + 1; wz1 = T(0.5); }
    } else {
        pz0 = pz1 = kf + 1;
        wz1 = T(0);
    }
    const T wz0 = T(1) - wz1;
    const int icl = ic0 + CP == nxc ? 0 : ic0 + CP;  // the coarse column after the thread's last
    T ev[CP], od[CP];
    for (int c = 0; c < CP; ++c) ev[c] = od[c] = T(0);
    auto row = [&](int pz, int jc, T w) {
        const T *r = uc + (size_t)pz * planec + (size_t)jc * nxc;
        T v[CP + 1];
        for (int c = 0; c < CP; ++c) v[c] = r[ic0 + c];
        v[CP] = r[icl];
        for (int c = 0; c < CP; ++c) {
            ev[c] += w * v[c];
            od[c] += w * (T(0.5) * (v[c] + v[c + 1]));
        }
    };
    row(pz0, jc0, wz0 * wy0);
    if (wy1 != T(0)) row(pz0, jc1, wz0 * wy1);
    if (wz1 != T(0)) {
        row(pz1, jc0, wz1 * wy0);
        if (wy1 != T(0)) row(pz1, jc1, wz1 * wy1);
    }
    V *f = (V *)(uf + (size_t)(kf + 1) * planef + (size_t)j * nxf + 2 * ic0);
    V x = *f;
    for (int c = 0; c < CP; ++c) {
        x[2 * c] += ev[c];
        x[2 * c + 1] += od[c];
    }
    *f = x;
}

// Coarse node eps by full weighting of the fine node eps (ghost planes map to
// ghost planes).
template <class T>
__global__ void k_coarsen_eps(const T *__restrict__ ef, T *__restrict__ ec, int nxf, int nyf,
                              int nxc, int nyc, int nwc, int zc) {
    const size_t planec = (size_t)nxc * nyc, planef = (size_t)nxf * nyf;
    const size_t total = planec * (nwc + 2);
    const T w3[3] = {T(0.25), T(0.5), T(0.25)};
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < total; q += (size_t)gridDim.x * blockDim.x) {
        const int ic = (int)(q % nxc);
        const int jc = (int)((q / nxc) % nyc);
        const int pc = (int)(q / planec);
        int pf[3];
        T wz[3];
        int nzt;
        if (!zc) { pf[0] = pc; wz[0] = T(1); nzt = 1; }
        else if (pc == 0) { pf[0] = 0; wz[0] = T(1); nzt = 1; }
        else if (pc == nwc + 1) { pf[0] = 2 * nwc + 2; wz[0] = T(1); nzt = 1; }
        else { pf[0] = 2 * pc - 1; pf[1] = 2 * pc; pf[2] = 2 * pc + 1; wz[0] = w3[0]; wz[1] = w3[1]; wz[2] = w3[2]; nzt = 3; }
        T acc = T(0);
        for (int a = 0; a < nzt; ++a)
            for (int dy = -1; dy <= 1; ++dy) {
                const int jf = (2 * jc + dy + nyf) % nyf;
                const size_t rb = (size_t)pf[a] * planef + (size_t)jf * nxf;
                const int i0 = 2 * ic;
                const T sx = T(0.25) * ef[rb + (i0 == 0 ? nxf - 1 : i0 - 1)] + T(0.5) * ef[rb + i0] +
                             T(0.25) * ef[rb + (i0 + 1 == nxf ? 0 : i0 + 1)];
                acc += wz[a] * w3[dy + 1] * sx;
            }
        ec[q] = acc;
    }
}

// ---------------------------------------------------------------- fused sweep
// One full red-black sweep in a single pass over HBM, out of place:
// u_out = sweep(u_in).  The first colour c0 is updated from u_in (its
// neighbours all have the other colour), the second colour from the new
// first-colour values.  A block owns a TX x TY tile of (x, y) for a chunk of
// kc planes and marches up in z with LDS rings: at step m it stashes plane
// m+1 of u_in, eps and f (tile plus a 2-cell halo, loaded FPD steps
// earlier) and starts loading plane m+1+FPD, computes first-colour values at plane m on
// the tile plus a 1-cell halo, then second-colour values at plane m-1 on the
// tile, and writes plane m-1 of u_out.  Halo values are recomputed by each
// block that needs them (from u_in, which nobody writes), so the result does
// not depend on block order.  Equals two colour passes in place.
//
// Two barriers per step: one after the stash (first colour may read plane
// m+1), one after the first colour (second colour reads it).  A ring slot is
// rewritten only when every thread is known to be past its last read: a
// thread that stashes at step m has only passed the second barrier of step
// m-1, so a slot read by the second colour of step m-1 must not be reused at
// step m.  That needs 4 planes of u, f and first-colour values and 5 of eps
// (read by the second colour one step later than by the first; 8 are kept).
// The step loop is unrolled by 8 so that every ring slot is a constant.
constexpr int FTX = 32, FTY = 16;
constexpr int FRX = FTX + 2, FRY = FTY + 2;  // first-colour values: tile + 1-cell halo
constexpr int FNT = FTX * FTY;               // threads
constexpr int FUNROLL = 8;
constexpr int FPD = 2;  // prefetch distance in plane steps (divides FUNROLL)

template <class T>
__device__ __forceinline__ T ld_off(const T *base, unsigned byte_off) {
    return *(const T *)((const char *)base + byte_off);
}

// W-wide vector of T (16 or 8 bytes) for the tile loads: clang's native
// vector types, which stay in registers (the HIP float4 / double2 structs held
// in arrays can end up in scratch memory).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <class T, int W> struct FVec;
template <> struct FVec<float, 4> { using V = f32x4; };
template <> struct FVec<float, 2> { using V = f32x2; };
template <> struct FVec<double, 2> { using V = f64x2; };

// Tiles are loaded as W-wide vectors: the x range starts HL = W cells left of
// the tile (a multiple of W, at least the 2-cell halo) and rows are
// LW = FTX + 2 HL cells long.  u and eps carry a 2-cell halo in y, f a 1-cell
// halo.  nx must be a multiple of W so that no vector straddles the wrap.
template <int W> struct FLayout {
    static constexpr int HL = W < 2 ? 2 : W;
    static constexpr int LW = FTX + 2 * HL;
    static constexpr int VR = LW / W;               // vectors per row
    static constexpr int NVU = VR * (FTY + 4);      // u / eps vectors per plane
    static constexpr int NVF = VR * (FTY + 2);      // f vectors per plane
    static_assert(NVU <= FNT && NVF <= FNT, "one vector per thread");
};

// ZIN: u_in is known to be zero (the first sweep of a V-cycle on a level
// whose correction starts from zero): its loads are skipped.
template <class T, int W, bool ZIN>
__global__ void __launch_bounds__(FNT)
k_sweep_fused(const T *__restrict__ uin, T *__restrict__ uout, const T *__restrict__ e, const T *__restrict__ f,
              LevelArgs a, int c0, int tiles_x, int tiles_y, int kc, int nb_real) {
    using L = FLayout<W>;
    using V = typename FVec<T, W>::V;
    constexpr int LW = L::LW, HL = L::HL;
    __shared__ __align__(16) T su[4][L::NVU * W];
    __shared__ __align__(16) T se[8][L::NVU * W];
    __shared__ __align__(16) T sf[4][L::NVF * W];
    __shared__ T sr[4][FRY * FRX];
    // XCD-aware order: each XCD gets a contiguous run of tiles (x fastest,
    // then y, then z chunk), so neighbouring tiles share its L2.
    const int tile = xcd_tile(nb_real);
    if (tile >= nb_real) return;
    const int nx = a.nx, ny = a.ny, nw = a.nw;
    const size_t plane = (size_t)nx * ny;
    const int i0 = (tile % tiles_x) * FTX, j0 = ((tile / tiles_x) % tiles_y) * FTY;
    const int k0 = (tile / (tiles_x * tiles_y)) * kc, k1 = min(nw, k0 + kc);
    const T cx = cxv<T>(a, 0), cy = cxv<T>(a, 1), cz = cxv<T>(a, 2);
    const int tid = threadIdx.x;
    const int base_par = (i0 + j0) & 1;  // colour of local (x, y, m) = (base_par + x + y + m) & 1
    // This thread's vector of the u / eps tile and of the f tile: byte offset
    // inside a plane (periodic wrap) and LDS element index.  Threads past the
    // last vector repeat it and skip the LDS store.
    const bool su_on = tid < L::NVU, sf_on = tid < L::NVF;
    unsigned ohu, ohf;
    int lhu, lhf;
    {
        const int q = min(tid, L::NVU - 1), xr = q % L::VR, yr = q / L::VR;
        const int i = ((i0 - HL + W * xr) % nx + nx) % nx, j = ((j0 - 2 + yr) % ny + ny) % ny;
        ohu = (unsigned)((j * nx + i) * sizeof(T));
        lhu = yr * LW + W * xr;
    }
    {
        const int q = min(tid, L::NVF - 1), xr = q % L::VR, yr = q / L::VR;
        const int i = ((i0 - HL + W * xr) % nx + nx) % nx, j = ((j0 - 1 + yr) % ny + ny) % ny;
        ohf = (unsigned)((j * nx + i) * sizeof(T));
        lhf = yr * LW + W * xr;
    }
    // first-colour work: thread tid < FRX*FRY/2 takes the tid-th first-colour
    // point of the tile + 1-cell halo (rows of FRX = 34 hold 17 of each colour)
    const bool red_on = tid < FRX * FRY / 2;
    const int ry = tid / (FRX / 2) - 1, rt = tid % (FRX / 2);
    // second-colour work: threads < FTX*FTY/2 compute, the others copy the
    // first-colour values of the tile to the output
    const bool blk_on = tid < FTX * FTY / 2;
    const int q2 = blk_on ? tid : tid - FTX * FTY / 2;
    const int by = q2 / (FTX / 2), bt = q2 % (FTX / 2);
    const int c1 = blk_on ? 1 - c0 : c0;
    const int j_out = j0 + by;

    V pu[FPD], pe[FPD], pf[FPD];
    // Loads are unconditional: plane indices are clamped into the ghosted
    // range, which is harmless because values of planes outside [-1, nw] (f:
    // outside [0, nw)) are never used.  Keeping the loads free of branches and
    // selects lets them stay in flight for FPD steps.
    auto fetch = [&](int k, V &du, V &de, V &df) {
        const int kk = min(max(k, -1), nw), kf = min(max(k, 0), nw - 1);
        const T *bu = uin + (size_t)(kk + 1) * plane, *be = e + (size_t)(kk + 1) * plane;
        const T *bf = f + (size_t)kf * plane;
        if constexpr (ZIN) du = V(0);
        else du = *(const V *)((const char *)bu + ohu);
        de = *(const V *)((const char *)be + ohu);
        df = *(const V *)((const char *)bf + ohf);
    };
    // Ring slot of plane p: its local index p - k0 + 2 modulo the ring depth.
    // Step ls works on m = k0 - 1 + ls, so plane m + d has local index
    // ls + 1 + d; ls is passed modulo 8 (a compile-time constant below).
    auto stash = [&](int lp, const V &du, const V &de, const V &df) {
        if (su_on) {
            *(V *)&su[lp & 3][lhu] = du;
            *(V *)&se[lp & 7][lhu] = de;
        }
        if (sf_on) *(V *)&sf[lp & 3][lhf] = df;
    };
    auto update = [&](const T *el, const T *ep, const T *en, int h, T uxp, T uxm, T uyp, T uym, T uzp, T uzm,
                      T fv) {
        const T e0 = el[h];
        const T wxp = cx * (e0 + el[h + 1]), wxm = cx * (e0 + el[h - 1]);
        const T wyp = cy * (e0 + el[h + LW]), wym = cy * (e0 + el[h - LW]);
        const T wzp = cz * (e0 + ep[h]), wzm = cz * (e0 + en[h]);
        const T off = T(0.5) * (wxp * uxp + wxm * uxm + wyp * uyp + wym * uym + wzp * uzp + wzm * uzm);
        const T dg = T(0.5) * (wxp + wxm + wyp + wym + wzp + wzm);
        return gs_value(off, fv, dg);
    };
    auto step = [&](int ls, int m, V &du, V &de, V &df) {
        const int l0 = ls + 1;     // local index of plane m
        stash(l0 + 1, du, de, df);  // plane m + 1, fetched FPD steps ago
        fetch(m + 1 + FPD, du, de, df);  // in flight for the next FPD steps
        __syncthreads();
        if (red_on) {  // first colour at plane m on the tile + 1-cell halo
            const int off = (c0 - base_par - ry - m + 1) & 1;
            const int x = -1 + 2 * rt + off;
            const int q = (ry + 1) * FRX + (x + 1);
            const int h = (ry + 2) * LW + (x + HL), hf = (ry + 1) * LW + (x + HL);
            T v = T(0);
            if (m >= 0 && m < nw) {
                const T *um = su[l0 & 3];
                v = update(se[l0 & 7], se[(l0 + 1) & 7], se[(l0 + 7) & 7], h, um[h + 1], um[h - 1], um[h + LW],
                           um[h - LW], su[(l0 + 1) & 3][h], su[(l0 + 3) & 3][h], sf[l0 & 3][hf]);
            }
            sr[l0 & 3][q] = v;
        }
        __syncthreads();
        const int k = m - 1;  // second colour at plane k on the tile, write plane k
        {
            const int lk = l0 + 7;  // local index of plane k, kept non-negative
            const int off = (c1 - base_par - by - k) & 1;
            const int x = 2 * bt + off;
            const int i = i0 + x;
            const int r = (by + 1) * FRX + (x + 1);
            const T *rm = sr[lk & 3];
            T v = rm[r];
            if (blk_on) {
                const int h = (by + 2) * LW + (x + HL), hf = (by + 1) * LW + (x + HL);
                v = update(se[lk & 7], se[(lk + 1) & 7], se[(lk + 7) & 7], h, rm[r + 1], rm[r - 1], rm[r + FRX],
                           rm[r - FRX], sr[(lk + 1) & 3][r], sr[(lk + 3) & 3][r], sf[lk & 3][hf]);
            }
            // Every thread stores once per step, so the compiler can count the
            // outstanding memory operations exactly (a conditional store would
            // make it wait for all prefetched loads).  Steps or positions that
            // own no point store a zero into the ghost plane 0 of uout, which
            // already holds zeros and is never written otherwise.
            const bool ij_ok = i < nx && j_out < ny;
            const bool valid = ij_ok && k >= k0 && k < k1;
            T *dst = uout + (valid ? (size_t)(k + 1) * plane : 0) + (ij_ok ? (size_t)j_out * nx + i : 0);
            *dst = valid ? v : T(0);
        }
    };
    // Prologue: planes k0 - 2 and k0 - 1 go straight to their ring slots
    // (local indices 0 and 1), planes k0 .. k0 + FPD - 1 are put in flight.
    fetch(k0 - 2, pu[0], pe[0], pf[0]);
    stash(0, pu[0], pe[0], pf[0]);
    fetch(k0 - 1, pu[1], pe[1], pf[1]);
    stash(1, pu[1], pe[1], pf[1]);
#pragma unroll
    for (int d = 0; d < FPD; ++d) fetch(k0 + d, pu[d], pe[d], pf[d]);
    // Steps m = k0-1 .. k0+kc, kc + 2 of them, a multiple of FUNROLL (the
    // launcher picks kc that way): no step is conditional, so the prefetched
    // registers rotate without copies (a copy would wait for the loads).  In a
    // chunk cut short by the top of the slab the extra steps write nothing.
    const int nsteps = kc + 2;
    for (int base = 0; base < nsteps; base += FUNROLL) {
#pragma unroll
        for (int s = 0; s < FUNROLL; ++s) step(s, k0 - 1 + base + s, pu[s % FPD], pe[s % FPD], pf[s % FPD]);
    }
}

// Row-band variant of the fused sweep (per-thread code in band_sweep.h): one
// W-wide vector of one band row per thread, (ty + 4) * nx / W threads.
// Planes loaded ahead: one for the general float32 variant with 4-wide
// vectors (measured in the slab solve: 2 % faster than two, whose registers
// it does not need), two otherwise.  One block of (ty + 4) * nx / W threads
// per CU is the measured optimum at 192 x 192: capping registers for two
// (six wavefronts per SIMD) spills and shortens the z chunks, 40 % slower.
template <class T, int W, bool ZIN> constexpr int band_pd() { return ZIN || W == 2 ? 2 : 1; }
template <class T, int W, bool ZIN, bool DOWN>
__device__ __forceinline__ void band_march(const BandArgs<T> &a, T *lds, int band, int chunk) {
    BandSweep<T, W, ZIN, DOWN, band_pd<T, W, ZIN>()> b;
    b.init(a, lds, band, chunk, threadIdx.x);
    b.prologue();
    __syncthreads();
    // an even number of steps (one past the chunk writes nothing), so that
    // the prefetch slot of each step is a constant
    const int m0 = b.first(), n = b.nsteps();
    for (int st = 0; st < n; st += 2) {
        b.template step<0>(m0 + b.D * st);
        __syncthreads();
        b.template step<1>(m0 + b.D * (st + 1));
        __syncthreads();
    }
}
// Tile t -> (band, chunk): groups of gb consecutive bands (gb divides the band
// count), chunks in order inside a group, so that the contiguous run of tiles
// each XCD receives covers a few neighbouring bands over a run of neighbouring
// chunks, whose shared halo rows and planes then meet in that XCD's L2.  Odd
// chunks march down, even ones up.
template <class T, int W, bool ZIN>
__global__ void __launch_bounds__(1024) k_sweep_band(BandArgs<T> a, int nb_real, int gb) {
    extern __shared__ __align__(16) unsigned char band_lds[];
    const int t = xcd_tile(nb_real);
    if (t >= nb_real) return;
    const int nchunks = (a.nw + a.kc - 1) / a.kc;
    const int g = t / (gb * nchunks), q = t - g * gb * nchunks;
    const int chunk = q / gb, band = g * gb + (q - (q / gb) * gb);
    T *lds = reinterpret_cast<T *>(band_lds);
    if (chunk & 1) band_march<T, W, ZIN, true>(a, lds, band, chunk);
    else band_march<T, W, ZIN, false>(a, lds, band, chunk);
}

// ---------------------------------------------------------------- residual + restriction
// fc = full weighting of the fine residual r = f - A u, in one pass, with the
// coarse unknowns zeroed (the coarse level starts its cycle from a zero
// correction); r itself is never written.  A block owns a tile of RCX x RCY
// coarse columns (one thread each) and marches up a chunk of fine planes.
// Each plane step stages u and eps of the plane above (tile + 2-cell halo,
// vector loads issued one step ahead) and f of the current plane in LDS rings,
// computes the fine residual of the current plane at the (2 RCX + 1) x
// (2 RCY + 1) points the 3 x 3 stencils of the tile cover, and each thread
// then forms its coarse column's in-plane weighted sum R.  Without z
// coarsening R is the coarse value of the same plane; with z coarsening fine
// plane 2 kc + dz adds R with weight 1/4, 1/2, 1/4 to coarse plane kc, so an
// even fine plane closes one coarse plane and opens the next.
constexpr int RCX = 16, RCY = 16;            // coarse columns per tile (threads)
constexpr int RNT = RCX * RCY;               // 256
constexpr int RFX = 2 * RCX, RFY = 2 * RCY;  // fine points per tile
constexpr int RRX = RFX + 1, RRY = RFY + 1;  // fine residual points the stencils cover
template <int W> struct RLay {
    static constexpr int HL = W < 2 ? 2 : W;  // x halo of the staged rows (>= 2, a multiple of W)
    static constexpr int LW = RFX + 2 * HL;   // staged row length
    static constexpr int VR = LW / W;
    static constexpr int NU = RFY + 4, NF = RFY + 2;  // staged rows of u / eps and of f
    static constexpr int NVU = VR * NU, NVF = VR * NF;
    static constexpr int MU = (NVU + RNT - 1) / RNT, MF = (NVF + RNT - 1) / RNT;
};

template <class T, int W, bool ZC>
__global__ void __launch_bounds__(RNT)
k_resid_restrict(const T *__restrict__ u, const T *__restrict__ e, const T *__restrict__ f, T *__restrict__ fc,
                 T *__restrict__ uc, LevelArgs a, int nxc, int nyc, int nwc, int tiles_x, int tiles_y, int kcc,
                 int nb_real) {
    using Ly = RLay<W>;
    using V = typename FVec<T, W>::V;
    constexpr int LW = Ly::LW, HL = Ly::HL;
    __shared__ __align__(16) T su[3][Ly::NVU * W];
    __shared__ __align__(16) T se[3][Ly::NVU * W];
    __shared__ __align__(16) T sf[Ly::NVF * W];
    __shared__ T rr[RRY * RRX];
    const int tile = xcd_tile(nb_real);
    if (tile >= nb_real) return;
    const int nx = a.nx, ny = a.ny, nw = a.nw;
    const size_t plane = (size_t)nx * ny, planec = (size_t)nxc * nyc;
    const int x0 = (tile % tiles_x) * RFX, y0 = ((tile / tiles_x) % tiles_y) * RFY;
    const int c0 = (tile / (tiles_x * tiles_y)) * kcc, c1 = min(nwc, c0 + kcc);  // coarse planes
    const int k0 = ZC ? 2 * c0 : c0, k1 = ZC ? 2 * c1 + 1 : c1;                   // fine planes [k0, k1)
    const T cx = cxv<T>(a, 0), cy = cxv<T>(a, 1), cz = cxv<T>(a, 2);
    const int tid = threadIdx.x;
    // staged vectors of this thread: byte offset in a plane, LDS index (-1: none)
    unsigned ou[Ly::MU], of[Ly::MF];
    int lu[Ly::MU], lf[Ly::MF];
#pragma unroll
    for (int m = 0; m < Ly::MU; ++m) {
        const int q = tid + RNT * m, qq = min(q, Ly::NVU - 1);
        const int row = qq / Ly::VR, col = qq % Ly::VR;
        const int x = ((x0 - HL + W * col) % nx + nx) % nx, y = ((y0 - 2 + row) % ny + ny) % ny;
        ou[m] = (unsigned)((y * nx + x) * sizeof(T));
        lu[m] = q < Ly::NVU ? row * LW + W * col : -1;
    }
#pragma unroll
    for (int m = 0; m < Ly::MF; ++m) {
        const int q = tid + RNT * m, qq = min(q, Ly::NVF - 1);
        const int row = qq / Ly::VR, col = qq % Ly::VR;
        const int x = ((x0 - HL + W * col) % nx + nx) % nx, y = ((y0 - 1 + row) % ny + ny) % ny;
        of[m] = (unsigned)((y * nx + x) * sizeof(T));
        lf[m] = q < Ly::NVF ? row * LW + W * col : -1;
    }
    V pu[Ly::MU], pe[Ly::MU], pf[Ly::MF];
    // loads are unconditional, planes clamped into the arrays
    auto fetch = [&](int k) {
        const int kk = min(max(k, -1), nw), kf = min(max(k - 1, 0), nw - 1);  // u, eps of k; f of k - 1
        const T *bu = u + (size_t)(kk + 1) * plane, *be = e + (size_t)(kk + 1) * plane, *bf = f + (size_t)kf * plane;
#pragma unroll
        for (int m = 0; m < Ly::MU; ++m) {
            pu[m] = *(const V *)((const char *)bu + ou[m]);
            pe[m] = *(const V *)((const char *)be + ou[m]);
        }
#pragma unroll
        for (int m = 0; m < Ly::MF; ++m) pf[m] = *(const V *)((const char *)bf + of[m]);
    };
    auto slot = [](int k) { return ((k % 3) + 3) % 3; };
    auto stash_ue = [&](int k) {
#pragma unroll
        for (int m = 0; m < Ly::MU; ++m)
            if (lu[m] >= 0) {
                *(V *)&su[slot(k)][lu[m]] = pu[m];
                *(V *)&se[slot(k)][lu[m]] = pe[m];
            }
    };
    auto stash_f = [&]() {
#pragma unroll
        for (int m = 0; m < Ly::MF; ++m)
            if (lf[m] >= 0) *(V *)&sf[lf[m]] = pf[m];
    };
    // restriction weights of this thread's coarse column
    const int tx = tid % RCX, ty = tid / RCX;
    const int ic = x0 / 2 + tx, jc = y0 / 2 + ty;
    const bool own = ic < nxc && jc < nyc;
    const size_t cidx = own ? (size_t)jc * nxc + ic : 0;
    const int rc = (2 * ty + 1) * RRX + (2 * tx + 1);  // centre of its 3 x 3 stencil in rr
    // prologue: planes k0 - 1 and k0 into the ring, k0 + 1 (and f of k0) in flight
    fetch(k0 - 1);
    stash_ue(k0 - 1);
    fetch(k0);
    stash_ue(k0);
    fetch(k0 + 1);
    T acc = T(0);
    for (int k = k0; k < k1; ++k) {
        stash_ue(k + 1);
        stash_f();  // f of plane k
        fetch(k + 2);
        __syncthreads();
        {
            const T *U0 = su[slot(k)], *Um = su[slot(k - 1)], *Up = su[slot(k + 1)];
            const T *E0 = se[slot(k)], *Em = se[slot(k - 1)], *Ep = se[slot(k + 1)];
            for (int q = tid; q < RRX * RRY; q += RNT) {
                const int rx = q % RRX, ry = q / RRX;
                const int h = (ry + 1) * LW + rx - 1 + HL, hf = ry * LW + rx - 1 + HL;
                const T e0 = E0[h], u0 = U0[h];
                const T wxp = cx * (e0 + E0[h + 1]), wxm = cx * (e0 + E0[h - 1]);
                const T wyp = cy * (e0 + E0[h + LW]), wym = cy * (e0 + E0[h - LW]);
                const T wzp = cz * (e0 + Ep[h]), wzm = cz * (e0 + Em[h]);
                const T off = T(0.5) * (wxp * U0[h + 1] + wxm * U0[h - 1] + wyp * U0[h + LW] + wym * U0[h - LW] +
                                        wzp * Up[h] + wzm * Um[h]);
                const T dg = T(0.5) * (wxp + wxm + wyp + wym + wzp + wzm);
                rr[q] = sf[hf] - (off - dg * u0);
            }
        }
        __syncthreads();
        const T sx0 = T(0.25) * rr[rc - RRX - 1] + T(0.5) * rr[rc - RRX] + T(0.25) * rr[rc - RRX + 1];
        const T sx1 = T(0.25) * rr[rc - 1] + T(0.5) * rr[rc] + T(0.25) * rr[rc + 1];
        const T sx2 = T(0.25) * rr[rc + RRX - 1] + T(0.5) * rr[rc + RRX] + T(0.25) * rr[rc + RRX + 1];
        const T R = T(0.25) * sx0 + T(0.5) * sx1 + T(0.25) * sx2;
        int kc_done = -1;
        T out = T(0);
        if (!ZC) {
            kc_done = k;
            out = R;
        } else if ((k & 1) == 0) {
            if (k > k0) {
                kc_done = k / 2 - 1;
                out = acc + T(0.25) * R;
            }
            acc = T(0.25) * R;
        } else {
            acc += T(0.5) * R;
        }
        if (own && kc_done >= 0) {
            fc[(size_t)kc_done * planec + cidx] = out;
            uc[(size_t)(kc_done + 1) * planec + cidx] = T(0);
            if (kc_done == 0) uc[cidx] = T(0);
            if (kc_done == nwc - 1) uc[(size_t)(nwc + 1) * planec + cidx] = T(0);
        }
    }
}

// ---------------------------------------------------------------- V-cycle bottom
// Levels small enough for one workgroup run the rest of the V-cycle inside a
// single kernel (one CU), phases separated by barriers: this replaces a few
// dozen tiny launches per cycle.
template <class T>
struct LevelDesc {
    T *u, *f, *r;
    const T *e;
    LevelArgs a;
    int zc;
    unsigned mh, mx, my;  // bt_div multipliers for nx / 2, nx, ny
};
// q / d through one multiply-high with m = floor((2^32 - 1) / d) + 1 (m = 0
// for d = 1): exact whenever q d < 2^32, which holds on these levels.
__device__ __forceinline__ int bt_div(int q, unsigned m) { return m ? (int)__umulhi((unsigned)q, m) : q; }
inline unsigned bt_magic(int d) { return d > 1 ? 0xFFFFFFFFu / (unsigned)d + 1u : 0u; }
constexpr int MAX_BOTTOM = 10;
template <class T>
struct Bottom {
    LevelDesc<T> L[MAX_BOTTOM];
    int nl, pre, post, coarse;
};

template <class T>
__device__ void bt_smooth(const LevelDesc<T> &d, int color) {
    const int half = d.a.nx / 2;
    const int per = half * d.a.ny * d.a.nw;
    const int plane = d.a.nx * d.a.ny;
    for (int q = threadIdx.x; q < per; q += blockDim.x) {
        const int qh = bt_div(q, d.mh), t = q - qh * half;
        const int kk = bt_div(qh, d.my), j = qh - kk * d.a.ny;
        const int i = 2 * t + ((j + kk + color) & 1);
        const int li = kk * plane + j * d.a.nx + i;
        T off, diag;
        level_sums(d.u, d.e, d.a, i, j, li + plane, off, diag);
        d.u[li + plane] = gs_value(off, d.f[li], diag);
    }
    __syncthreads();
}

template <class T>
__device__ void bt_residual(const LevelDesc<T> &d) {
    const int plane = d.a.nx * d.a.ny;
    const int n = plane * d.a.nw;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        const int qx = bt_div(q, d.mx), i = q - qx * d.a.nx;
        const int j = qx - bt_div(qx, d.my) * d.a.ny;
        T off, diag;
        level_sums(d.u, d.e, d.a, i, j, q + plane, off, diag);
        d.r[q] = d.f[q] - (off - diag * d.u[q + plane]);
    }
    __syncthreads();
}

template <class T>
__device__ void bt_restrict_zero(const LevelDesc<T> &F, const LevelDesc<T> &C) {
    const T w3[3] = {T(0.25), T(0.5), T(0.25)};
    const int nxf = F.a.nx, nyf = F.a.ny, nxc = C.a.nx, nyc = C.a.ny;
    const int planef = nxf * nyf, planec = nxc * nyc;
    const int n = planec * C.a.nw;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        const int qx = bt_div(q, C.mx), ic = q - qx * nxc;
        const int kc = bt_div(qx, C.my), jc = qx - kc * nyc;
        T acc = T(0);
        const int nzt = C.zc ? 3 : 1;
        for (int dz = 0; dz < nzt; ++dz) {
            const int kf = C.zc ? 2 * kc + dz : kc;
            const T wz = C.zc ? w3[dz] : T(1);
            for (int dy = -1; dy <= 1; ++dy) {
                const int jy = 2 * jc + dy;
                const int jf = jy < 0 ? jy + nyf : (jy >= nyf ? jy - nyf : jy);
                const int rb = kf * planef + jf * nxf;
                const int i0 = 2 * ic;
                const T sx = T(0.25) * F.r[rb + (i0 == 0 ? nxf - 1 : i0 - 1)] + T(0.5) * F.r[rb + i0] +
                             T(0.25) * F.r[rb + (i0 + 1 == nxf ? 0 : i0 + 1)];
                acc += wz * w3[dy + 1] * sx;
            }
        }
        C.f[q] = acc;
    }
    const int ng = planec * (C.a.nw + 2);
    for (int q = threadIdx.x; q < ng; q += blockDim.x) C.u[q] = T(0);
    __syncthreads();
}

template <class T>
__device__ void bt_prolong(const LevelDesc<T> &F, const LevelDesc<T> &C) {
    const int nxf = F.a.nx, nyf = F.a.ny, nxc = C.a.nx, nyc = C.a.ny;
    const int planef = nxf * nyf, planec = nxc * nyc;
    const int n = planef * F.a.nw;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        const int qx = bt_div(q, F.mx), i = q - qx * nxf;
        const int kf = bt_div(qx, F.my), j = qx - kf * nyf;
        int ix[2], jy[2], pz[2];
        T wx[2], wyv[2], wz[2];
        int nxs, nys, nzs;
        if (i & 1) { ix[0] = i >> 1; ix[1] = (ix[0] + 1 == nxc) ? 0 : ix[0] + 1; wx[0] = wx[1] = T(0.5); nxs = 2; }
        else { ix[0] = i >> 1; wx[0] = T(1); nxs = 1; }
        if (j & 1) { jy[0] = j >> 1; jy[1] = (jy[0] + 1 == nyc) ? 0 : jy[0] + 1; wyv[0] = wyv[1] = T(0.5); nys = 2; }
        else { jy[0] = j >> 1; wyv[0] = T(1); nys = 1; }
        if (C.zc) {
            if (kf & 1) { pz[0] = (kf - 1) / 2 + 1; wz[0] = T(1); nzs = 1; }
            else { pz[0] = kf / 2; pz[1] = kf / 2 + 1; wz[0] = wz[1] = T(0.5); nzs = 2; }
        } else { pz[0] = kf + 1; wz[0] = T(1); nzs = 1; }
        T acc = T(0);
        for (int a = 0; a < nzs; ++a)
            for (int b = 0; b < nys; ++b)
                for (int c = 0; c < nxs; ++c)
                    acc += wz[a] * wyv[b] * wx[c] * C.u[pz[a] * planec + jy[b] * nxc + ix[c]];
        F.u[q + planef] += acc;
    }
    __syncthreads();
}

constexpr int BOTTOM_LDS = 2048;  // coarsest level staged in LDS when its ghosted size fits

// V-cycle over levels L[0..nl-1] of the bottom set; L[0].f is given and
// L[0].u holds the initial guess.  The coarsest level's sweeps run out of LDS
// when it is small enough.
template <class T>
__global__ void __launch_bounds__(1024) k_vcycle_bottom(Bottom<T> B) {
    __shared__ T lu[BOTTOM_LDS], lf[BOTTOM_LDS], le[BOTTOM_LDS];
    for (int l = 0; l + 1 < B.nl; ++l) {
        for (int k = 0; k < B.pre; ++k) { bt_smooth(B.L[l], 0); bt_smooth(B.L[l], 1); }
        bt_residual(B.L[l]);
        bt_restrict_zero(B.L[l], B.L[l + 1]);
    }
    {
        const LevelDesc<T> &c = B.L[B.nl - 1];
        const int plane = c.a.nx * c.a.ny;
        const int ng = plane * (c.a.nw + 2), ni = plane * c.a.nw;
        if (ng <= BOTTOM_LDS) {
            for (int q = threadIdx.x; q < ng; q += blockDim.x) { lu[q] = c.u[q]; le[q] = c.e[q]; }
            for (int q = threadIdx.x; q < ni; q += blockDim.x) lf[q] = c.f[q];
            __syncthreads();
            LevelDesc<T> d = c;
            d.u = lu;
            d.f = lf;
            d.e = le;
            for (int k = 0; k < B.coarse; ++k) { bt_smooth(d, 0); bt_smooth(d, 1); }
            for (int q = threadIdx.x; q < ng; q += blockDim.x) c.u[q] = lu[q];
            __syncthreads();
        } else {
            for (int k = 0; k < B.coarse; ++k) { bt_smooth(c, 0); bt_smooth(c, 1); }
        }
    }
    for (int l = B.nl - 2; l >= 0; --l) {
        bt_prolong(B.L[l], B.L[l + 1]);
        for (int k = 0; k < B.post; ++k) { bt_smooth(B.L[l], 1); bt_smooth(B.L[l], 0); }
    }
}

// The same V-cycle with every array of the bottom set in LDS (up to 160 KB
// per workgroup on gfx950): the first level's u and f and every level's eps
// are staged in once, u is written back at the end, and every phase between
// reads and writes LDS only.  off[4 l + {0,1,2,3}] are the element offsets of
// level l's u (ghosted), f, r (interior) and eps (ghosted) in LDS.
struct BottomLds {
    int off[4 * MAX_BOTTOM];
};
template <class T>
__global__ void __launch_bounds__(1024) k_vcycle_bottom_lds(Bottom<T> B, BottomLds O) {
    extern __shared__ __align__(16) unsigned char bl_raw[];
    T *lds = reinterpret_cast<T *>(bl_raw);
    auto D = [&](int l) {
        LevelDesc<T> d = B.L[l];
        d.u = lds + O.off[4 * l];
        d.f = lds + O.off[4 * l + 1];
        d.r = lds + O.off[4 * l + 2];
        d.e = lds + O.off[4 * l + 3];
        return d;
    };
    for (int l = 0; l < B.nl; ++l) {
        const LevelArgs &a = B.L[l].a;
        const int ng = a.nx * a.ny * (a.nw + 2);
        T *e = lds + O.off[4 * l + 3];
        for (int q = threadIdx.x; q < ng; q += blockDim.x) e[q] = B.L[l].e[q];
    }
    {
        const LevelArgs &a = B.L[0].a;
        const int ni = a.nx * a.ny * a.nw, ng = ni + 2 * a.nx * a.ny;
        T *u = lds + O.off[0], *f = lds + O.off[1];
        for (int q = threadIdx.x; q < ng; q += blockDim.x) u[q] = B.L[0].u[q];
        for (int q = threadIdx.x; q < ni; q += blockDim.x) f[q] = B.L[0].f[q];
    }
    __syncthreads();
    for (int l = 0; l + 1 < B.nl; ++l) {
        const LevelDesc<T> d = D(l);
        for (int k = 0; k < B.pre; ++k) { bt_smooth(d, 0); bt_smooth(d, 1); }
        bt_residual(d);
        bt_restrict_zero(d, D(l + 1));
    }
    {
        const LevelDesc<T> c = D(B.nl - 1);
        for (int k = 0; k < B.coarse; ++k) { bt_smooth(c, 0); bt_smooth(c, 1); }
    }
    for (int l = B.nl - 2; l >= 0; --l) {
        const LevelDesc<T> d = D(l);
        bt_prolong(d, D(l + 1));
        for (int k = 0; k < B.post; ++k) { bt_smooth(d, 1); bt_smooth(d, 0); }
    }
    {
        const LevelArgs &a = B.L[0].a;
        const int ng = a.nx * a.ny * (a.nw + 2);
        const T *u = lds + O.off[0];
        for (int q = threadIdx.x; q < ng; q += blockDim.x) B.L[0].u[q] = u[q];
    }
}

inline int grid1d(size_t n, int threads = 256) {
    size_t b = (n + threads - 1) / threads;
    if (b > 16384) b = 16384;
    if (b < 1) b = 1;
    return (int)b;
}

LevelArgs level_args(const Level &L) {
    LevelArgs a;
    a.nx = L.nx; a.ny = L.ny; a.nw = L.nw;
    a.cx = 1.0 / (L.h[0] * L.h[0]);
    a.cy = 1.0 / (L.h[1] * L.h[1]);
    a.cz = 1.0 / (L.h[2] * L.h[2]);
    a.cxf = (float)a.cx; a.cyf = (float)a.cy; a.czf = (float)a.cz;
    return a;
}

}  // namespace

// ============================================================== launchers
static bool al16(const void *q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; }

// Resident blocks per CU of a kernel at a block shape (threads, dynamic LDS
// bytes), cached per device: the occupancy query is a host call per launch
// otherwise.  The raised dynamic-LDS limit is set the first time a kernel is
// seen on a device.
struct OccKey {
    const void *fn;
    int dev, nt;
    size_t bytes;
    int per;
};
static int occupancy(const void *fn, int nt, size_t bytes) {
    static OccKey cache[64];
    static int used = 0;
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
    int dev = 0;
    DWP_HIP(hipGetDevice(&dev));
    bool seen = false;
    for (int i = 0; i < used; ++i) {
        const OccKey &k = cache[i];
        if (k.fn == fn && k.dev == dev) {
            seen = true;
            if (k.nt == nt && k.bytes == bytes) return k.per;
        }
    }
    if (!seen) DWP_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)BOTTOM_LDS_BYTES));
    int per = 0;
    DWP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, nt, bytes));
    if (used < 64) cache[used++] = OccKey{fn, dev, nt, bytes, per};
    return per;
}
static int cu_count() {
    static int cus[64] = {0};
    int dev = 0;
    DWP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) fail(DWP_EINVAL, "internal: device index out of range");
    if (!cus[dev]) DWP_HIP(hipDeviceGetAttribute(&cus[dev], hipDeviceAttributeMultiprocessorCount, dev));
    return cus[dev];
}

// The operator on row bands: false (nothing launched) where the shape does
// not fit -- nx not a multiple of the vector width, more than 1024 threads,
// no band height in APPLY_ROWS dividing ny.  The chunk length fills whole
// rounds of resident blocks.
constexpr int APPLY_ROWS[] = {16, 12, 8, 6, 4};
template <int MODE, class TS, class TB>
static bool apply_band(hipStream_t s, const Plan &p, const TS *phi, const TS *eps, const TB *b, TS *out,
                       int nplanes) {
    constexpr int W = ApplyVec<TS>::W;
    if (p.nx % W || !al16(phi) || !al16(eps) || !al16(out) || (MODE != 0 && !al16(b))) return false;
    int ty = 0;
    for (int t : APPLY_ROWS)
        if (p.ny % t == 0 && p.ny >= t + 2 && (t + 2) * (p.nx / W) <= 1024 &&
            sizeof(TS) * (size_t)apply_lds_elems(p.nx, t) <= BOTTOM_LDS_BYTES) {
            ty = t;
            break;
        }
    if (!ty) return false;
    const int nt = (ty + 2) * (p.nx / W);
    const size_t bytes = sizeof(TS) * (size_t)apply_lds_elems(p.nx, ty);
    const int per = occupancy(reinterpret_cast<const void *>(&k_apply_band<MODE, TS, TB>), nt, bytes);
    if (per < 1) return false;
    const int bands = p.ny / ty;
    const long slots = (long)cu_count() * per;
    int kc = 1;
    long best = -1;
    for (int c = 1; c <= 64; ++c) {
        const long blocks = (long)bands * ((nplanes + c - 1) / c);
        const long cost = (blocks + slots - 1) / slots * (c + 2);
        if (best < 0 || cost < best) { best = cost; kc = c; }
    }
    const int nb = bands * ((nplanes + kc - 1) / kc), padded = (nb + 7) / 8 * 8;
    const int gb = bands % 4 == 0 ? 4 : (bands % 2 == 0 ? 2 : 1);
    ApplyArgs<TS, TB> a{phi, eps, b, out, p.nx, p.ny, p.nz, p.k_w0, nplanes, ty, bands, kc,
                        1.0 / (p.h[0] * p.h[0]), 1.0 / (p.h[1] * p.h[1]), 1.0 / (p.h[2] * p.h[2])};
    k_apply_band<MODE, TS, TB><<<padded, nt, bytes, s>>>(a, nb, gb);
    DWP_LAUNCH_CHECK();
    return true;
}

template <class T, int MODE, class TB = double, class TP = double, class TE = double>
void launch_zmarch(hipStream_t s, const Plan &p, const TP *phi, const TE *eps, const TB *b, T *out,
                   int nplanes) {
    // row bands where phi, eps and out share one storage type (and b too)
    if constexpr (std::is_same<TP, TE>::value && std::is_same<T, TP>::value &&
                  (MODE == 0 || std::is_same<TB, TP>::value || sizeof(TB) < sizeof(TP))) {
        if (apply_band<MODE, T, TB>(s, p, phi, eps, b, out, nplanes)) return;
    }
    const bool tile_ok = p.nx % 2 == 0 && al16(phi) && al16(eps) && (MODE == 0 || al16(b)) && al16(out);
    if (tile_ok) {
        constexpr int ZCH = apply_zch<MODE>();
        const int tx = (p.nx + ATX - 1) / ATX, ty = (p.ny + ATY - 1) / ATY, tz = (nplanes + ZCH - 1) / ZCH;
        const int nb = tx * ty * tz, padded = (nb + 7) / 8 * 8;
        k_apply_tile<T, MODE, TB, TP, TE><<<padded, dim3(32, 8), 0, s>>>(phi, eps, b, out, p.nx, p.ny, p.nz,
                                                             1.0 / (p.h[0] * p.h[0]), 1.0 / (p.h[1] * p.h[1]),
                                                             1.0 / (p.h[2] * p.h[2]), p.k_w0, nplanes, tx, ty, nb);
        DWP_LAUNCH_CHECK();
        return;
    }
    const int tx = (p.nx + BX - 1) / BX, ty = (p.ny + BY - 1) / BY, tz = (nplanes + ZM - 1) / ZM;
    const int nb = tx * ty * tz;
    const int padded = (nb + 7) / 8 * 8;
    k_apply_zmarch<T, MODE, TB, TP, TE><<<padded, dim3(BX, BY), 0, s>>>(phi, eps, b, out, p.nx, p.ny, p.nz, 1.0 / (p.h[0] * p.h[0]),
                                                            1.0 / (p.h[1] * p.h[1]), 1.0 / (p.h[2] * p.h[2]), p.k_w0,
                                                            nplanes, tx, ty, nb);
    DWP_LAUNCH_CHECK();
}

void launch_apply_full(hipStream_t s, const Plan &p, const double *phi, const double *eps,
                       const double *b, double *out, bool residual) {
    if (residual) launch_zmarch<double, 1>(s, p, phi, eps, b, out, p.nz);
    else launch_zmarch<double, 0>(s, p, phi, eps, b, out, p.nz);
}

void launch_eps_gradient(hipStream_t s, const Plan &p, const double *phi, double *g) {
    const double h3 = p.h[0] * p.h[1] * p.h[2];
    const double scale = -h3 / (8.0 * 3.14159265358979323846);
    dim3 gr((p.nx + BX - 1) / BX, (p.ny + BY - 1) / BY, p.nz), blk(BX, BY);
    k_eps_gradient<0><<<gr, blk, 0, s>>>(phi, nullptr, g, p.nx, p.ny, p.nz, 1.0 / p.h[0], 1.0 / p.h[1],
                                         1.0 / p.h[2], scale);
    DWP_LAUNCH_CHECK();
}

void launch_v_eps(hipStream_t s, const Plan &p, const double *phi, const double *deps, bool add_phi, double *out) {
    const double scale = -1.0 / (8.0 * 3.14159265358979323846);
    dim3 gr((p.nx + BX - 1) / BX, (p.ny + BY - 1) / BY, p.nz), blk(BX, BY);
    if (add_phi)
        k_eps_gradient<2><<<gr, blk, 0, s>>>(phi, deps, out, p.nx, p.ny, p.nz, 1.0 / p.h[0], 1.0 / p.h[1],
                                             1.0 / p.h[2], scale);
    else
        k_eps_gradient<1><<<gr, blk, 0, s>>>(phi, deps, out, p.nx, p.ny, p.nz, 1.0 / p.h[0], 1.0 / p.h[1],
                                             1.0 / p.h[2], scale);
    DWP_LAUNCH_CHECK();
}

void launch_eps_density(hipStream_t s, const double *rho, double *eps, double *deps, size_t n, double eps_inf,
                        double rho0, double beta) {
    k_eps_density<<<grid1d(n), 256, 0, s>>>(rho, eps, deps, n, eps_inf, 1.0 / rho0, 2.0 * beta);
    DWP_LAUNCH_CHECK();
}

void launch_eps_pair(hipStream_t s, const Plan &p, const double *a, const double *b, double scale, double *g) {
    dim3 gr((p.nx + BX - 1) / BX, (p.ny + BY - 1) / BY, p.nz), blk(BX, BY);
    k_eps_pair<<<gr, blk, 0, s>>>(a, b, g, p.nx, p.ny, p.nz, 1.0 / p.h[0], 1.0 / p.h[1], 1.0 / p.h[2], scale);
    DWP_LAUNCH_CHECK();
}

void launch_fill(hipStream_t s, double *x, double v, size_t n) {
    k_fill<<<grid1d(n), 256, 0, s>>>(x, v, n);
    DWP_LAUNCH_CHECK();
}
void launch_scale_dev(hipStream_t s, double *x, const double *num, const double *den_sq, size_t n, int mode) {
    k_scale_dev<<<grid1d(n), 256, 0, s>>>(x, num, den_sq, n, mode);
    DWP_LAUNCH_CHECK();
}
void launch_rhs(hipStream_t s, const double *rho, const double *sum, double inv_n, double *b, size_t n) {
    k_rhs<<<grid1d(n), 256, 0, s>>>(rho, sum, inv_n, b, n);
    DWP_LAUNCH_CHECK();
}
void launch_sub_mean(hipStream_t s, double *x, const double *sum, double inv_n, size_t n) {
    k_sub_mean<<<grid1d(n), 256, 0, s>>>(x, sum, inv_n, n);
    DWP_LAUNCH_CHECK();
}
void launch_mul(hipStream_t s, double *y, const double *a, const double *x, size_t n) {
    k_mul<<<grid1d(n), 256, 0, s>>>(y, a, x, n);
    DWP_LAUNCH_CHECK();
}
void launch_axpby(hipStream_t s, double *out, double a, const double *x, double b, const double *y, size_t n) {
    k_axpby<<<grid1d(n), 256, 0, s>>>(out, a, x, b, y, n);
    DWP_LAUNCH_CHECK();
}
void launch_rsqrt(hipStream_t s, const double *eps, double *sinv, size_t n) {
    k_rsqrt<<<grid1d(n), 256, 0, s>>>(eps, sinv, n);
    DWP_LAUNCH_CHECK();
}
void launch_check_eps(hipStream_t s, const double *eps, size_t n, int *flags) {
    k_check<<<RED_BLOCKS, 256, 0, s>>>(eps, n, flags, 1);
    DWP_LAUNCH_CHECK();
}
void launch_check_finite(hipStream_t s, const double *x, size_t n, int *flags) {
    k_check<<<RED_BLOCKS, 256, 0, s>>>(x, n, flags, 0);
    DWP_LAUNCH_CHECK();
}

template <class T>
void launch_wet_residual(hipStream_t s, const Plan &p, const double *v, const double *dD,
                         const double *eps, T *fW) {
    launch_zmarch<T, 2>(s, p, dD, eps, v, fW, p.nw);
}
template <class T>
void launch_wet_residual_v32(hipStream_t s, const Plan &p, const float *v, const float *dD, const float *eps,
                             T *fW) {
    launch_zmarch<T, 2, float, float, float>(s, p, dD, eps, v, fW, p.nw);
}
template <class T>
void launch_wet_residual_v16(hipStream_t s, const Plan &p, const _Float16 *v, const float *dD, const float *eps,
                             T *fW) {
    launch_zmarch<T, 2, _Float16, float, float>(s, p, dD, eps, v, fW, p.nw);
}
void launch_apply_full_f32(hipStream_t s, const Plan &p, const float *phi, const float *eps, float *out) {
    launch_zmarch<float, 0, double, float, float>(s, p, phi, eps, (const double *)nullptr, out, p.nz);
}
__global__ void k_to_f32(const double *__restrict__ x, float *__restrict__ y, size_t n) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        y[t] = (float)x[t];
}
void launch_to_f32(hipStream_t s, const double *x, float *y, size_t n) {
    k_to_f32<<<grid1d(n), 256, 0, s>>>(x, y, n);
    DWP_LAUNCH_CHECK();
}
template <class T, class TZ>
static void wet_add_t(hipStream_t s, const Plan &p, const T *uW, TZ *z) {
    const int plane = p.nx * p.ny;
    const bool pairs = plane % 2 == 0 && (reinterpret_cast<uintptr_t>(z) & 15) == 0;
    const bool quads = sizeof(T) == 4 && sizeof(TZ) == 4 && plane % 4 == 0 &&
                       (reinterpret_cast<uintptr_t>(z) & 15) == 0 && (reinterpret_cast<uintptr_t>(uW) & 15) == 0;
    if constexpr (sizeof(T) == 4 && sizeof(TZ) == 4) {
        if (quads) {
            dim3 g((plane / 4 + 255) / 256, p.nw);
            k_wet_add<T, false, TZ, true><<<g, 256, 0, s>>>(uW, z, plane, p.nz, p.k_w0);
            DWP_LAUNCH_CHECK();
            return;
        }
    }
    const int per = pairs ? plane / 2 : plane;
    dim3 g((per + 255) / 256, p.nw);
    if (pairs) k_wet_add<T, true, TZ><<<g, 256, 0, s>>>(uW, z, plane, p.nz, p.k_w0);
    else k_wet_add<T, false, TZ><<<g, 256, 0, s>>>(uW, z, plane, p.nz, p.k_w0);
    DWP_LAUNCH_CHECK();
}
template <class T>
void launch_wet_add(hipStream_t s, const Plan &p, const T *uW, double *z) { wet_add_t<T, double>(s, p, uW, z); }
template <class T>
void launch_wet_add(hipStream_t s, const Plan &p, const T *uW, float *z) { wet_add_t<T, float>(s, p, uW, z); }
template <class T>
void launch_wet_eps(hipStream_t s, const Plan &p, const double *eps, T *epsW) {
    const size_t n = (size_t)p.nx * p.ny * (p.nw + 2);
    k_wet_eps<T><<<grid1d(n), 256, 0, s>>>(eps, epsW, p.nx, p.ny, p.nz, p.k_w0, p.nw);
    DWP_LAUNCH_CHECK();
}

template <class T>
void launch_level_residual(hipStream_t s, const Level &L, T *r) {
    LevelArgs a = level_args(L);
    dim3 g((L.nx + BX - 1) / BX, (L.ny + BY - 1) / BY, L.nw), blk(BX, BY);
    k_level_residual<T><<<g, blk, 0, s>>>(L.u.as<T>(), L.eps.as<T>(), L.f.as<T>(), r, a);
    DWP_LAUNCH_CHECK();
}
template <class T>
void launch_level_smooth(hipStream_t s, const Level &L, int color) {
    LevelArgs a = level_args(L);
    const int half = L.nx / 2;
    dim3 g((half + BX - 1) / BX, (L.ny + BY - 1) / BY, L.nw), blk(BX, BY);
    k_level_smooth<T><<<g, blk, 0, s>>>(L.u.as<T>(), L.eps.as<T>(), L.f.as<T>(), a, color);
    DWP_LAUNCH_CHECK();
}
template <class T>
void launch_restrict(hipStream_t s, const Level &F, const Level &C, const T *rf, T *fc) {
    dim3 g((C.nx + BX - 1) / BX, (C.ny + BY - 1) / BY, C.nw), blk(BX, BY);
    k_restrict<T><<<g, blk, 0, s>>>(rf, fc, C.u.as<T>(), F.nx, F.ny, C.nx, C.ny, C.nw, C.zc ? 1 : 0);
    DWP_LAUNCH_CHECK();
}
template <class T, int W, bool ZC>
static void resid_restrict_w(hipStream_t s, const Level &F, const Level &C) {
    LevelArgs a = level_args(F);
    const int tx = (F.nx + RFX - 1) / RFX, ty = (F.ny + RFY - 1) / RFY;
    // coarse planes per block: blocks run in ceil(blocks / slots) rounds of
    // (fine planes + 2) serial plane steps; pick the chunk with the fewest
    // steps in all (ties: the longer chunk, fewer halo planes re-read)
    static int slots[64] = {0};
    int dev = 0;
    DWP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) fail(DWP_EINVAL, "internal: device index out of range");
    if (!slots[dev]) {
        int cus = 0, per = 0;
        DWP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        DWP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_resid_restrict<T, W, ZC>, RNT, 0));
        slots[dev] = std::max(1, cus * per);
    }
    int kcc = 1;
    long best = -1;
    for (int kq = 1; kq <= C.nw; ++kq) {
        const long blocks = (long)tx * ty * ((C.nw + kq - 1) / kq);
        const long cost = (blocks + slots[dev] - 1) / slots[dev] * ((ZC ? 2 * kq + 1 : kq) + 2);
        if (best < 0 || cost <= best) { best = cost; kcc = kq; }
    }
    const int tz = (C.nw + kcc - 1) / kcc;
    const int nb = tx * ty * tz, padded = (nb + 7) / 8 * 8;
    k_resid_restrict<T, W, ZC><<<padded, RNT, 0, s>>>(F.u.as<T>(), F.eps.as<T>(), F.f.as<T>(), C.f.as<T>(),
                                                      C.u.as<T>(), a, C.nx, C.ny, C.nw, tx, ty, kcc, nb);
    DWP_LAUNCH_CHECK();
}

// Vector width of the staged rows: 16-byte loads need nx to be a multiple
// of the vector (always true for a level that has a coarser one: x is halved
// only when nx is a multiple of 4).
// Row bands of tyc coarse rows (RESTRICT_ROWS, the first that divides nyc
// within 1024 threads and the LDS); false where none fits.
constexpr int RESTRICT_ROWS[] = {6, 8, 4, 12, 2};
template <class T, int W, bool ZC>
static bool resid_restrict_band(hipStream_t s, const Level &F, const Level &C) {
    int tyc = 0;
    for (int t : RESTRICT_ROWS)
        if (C.ny % t == 0 && (2 * t + 3) * (F.nx / W) <= 1024 && F.ny >= 2 * t + 3 &&
            sizeof(T) * (size_t)restrict_lds_elems(F.nx, t) <= BOTTOM_LDS_BYTES) {
            tyc = t;
            break;
        }
    if (!tyc) return false;
    const int nt = (2 * tyc + 3) * (F.nx / W);
    const size_t bytes = sizeof(T) * (size_t)restrict_lds_elems(F.nx, tyc);
    const int per = occupancy(reinterpret_cast<const void *>(&k_resid_restrict_band<T, W, ZC>), nt, bytes);
    if (per < 1) return false;
    const int bands = C.ny / tyc;
    const long slots = (long)cu_count() * per;
    int kcc = 1;
    long best = -1;
    for (int c = 1; c <= 64; ++c) {
        const long blocks = (long)bands * ((C.nw + c - 1) / c);
        const long cost = (blocks + slots - 1) / slots * ((ZC ? 2 * c + 1 : c) + 2);
        if (best < 0 || cost < best) { best = cost; kcc = c; }
    }
    const int nb = bands * ((C.nw + kcc - 1) / kcc), padded = (nb + 7) / 8 * 8;
    const int gb = bands % 4 == 0 ? 4 : (bands % 2 == 0 ? 2 : 1);
    const LevelArgs la = level_args(F);
    const bool f32 = sizeof(T) == 4;
    RestrictArgs<T> a{F.u.as<T>(), F.eps.as<T>(), F.f.as<T>(), C.f.as<T>(), C.u.as<T>(), F.nx, F.ny, F.nw,
                      C.nx, C.ny, C.nw, tyc, bands, kcc,
                      (T)(f32 ? la.cxf : la.cx), (T)(f32 ? la.cyf : la.cy), (T)(f32 ? la.czf : la.cz)};
    k_resid_restrict_band<T, W, ZC><<<padded, nt, bytes, s>>>(a, nb, gb);
    DWP_LAUNCH_CHECK();
    return true;
}

template <class T>
void launch_resid_restrict(hipStream_t s, const Level &F, const Level &C) {
    if (F.nx != 2 * C.nx || F.ny != 2 * C.ny || F.nx % 4 != 0 || (C.zc ? F.nw != 2 * C.nw + 1 : F.nw != C.nw))
        fail(DWP_EINVAL, "internal: residual-restriction needs x and y halved (z halved or kept)");
    constexpr int W = sizeof(T) == 4 ? 4 : 2;
    if (C.zc) {
        if (!resid_restrict_band<T, W, true>(s, F, C)) resid_restrict_w<T, W, true>(s, F, C);
    } else if (!resid_restrict_band<T, W, false>(s, F, C)) {
        resid_restrict_w<T, W, false>(s, F, C);
    }
}

template <class T>
void launch_prolong_add(hipStream_t s, const Level &F, const Level &C) {
    if (F.nx != 2 * C.nx || F.ny != 2 * C.ny) fail(DWP_EINVAL, "internal: prolongation needs x and y coarsened by 2");
    // 16-byte vectors of fine points where the coarse columns split into
    // whole vectors (float: 2 coarse columns, double: 1)
    constexpr int CP = sizeof(T) == 4 ? 2 : 1;
    if (C.nx % CP == 0) {
        dim3 g((C.nx / CP + BX - 1) / BX, (F.ny + BY - 1) / BY, F.nw), blk(BX, BY);
        k_prolong_add_v<T, CP><<<g, blk, 0, s>>>(F.u.as<T>(), C.u.as<T>(), F.nx, F.ny, C.nx, C.ny, C.zc ? 1 : 0);
    } else {
        dim3 g((C.nx + BX - 1) / BX, (F.ny + BY - 1) / BY, F.nw), blk(BX, BY);
        k_prolong_add<T><<<g, blk, 0, s>>>(F.u.as<T>(), C.u.as<T>(), F.nx, F.ny, C.nx, C.ny, C.zc ? 1 : 0);
    }
    DWP_LAUNCH_CHECK();
}
template <class T>
void launch_coarsen_eps(hipStream_t s, const Level &F, const Level &C) {
    const size_t n = C.n_ghosted();
    k_coarsen_eps<T><<<grid1d(n), 256, 0, s>>>(F.eps.as<T>(), C.eps.as<T>(), F.nx, F.ny, C.nx, C.ny, C.nw, C.zc ? 1 : 0);
    DWP_LAUNCH_CHECK();
}
// Chunk length (planes per block) of the fused sweep: kc + 2 plane steps, a
// multiple of FUNROLL.  Blocks run in ceil(blocks / slots) rounds, where
// slots = resident blocks on the whole device; the cost model
// rounds * (kc + 2) picks the chunk that fills the last round best.
static int fused_chunk(int tiles, int nw, int slots) {
    int best = FUNROLL - 2;
    long best_cost = -1;
    for (int kc = FUNROLL - 2; kc <= 8 * FUNROLL - 2; kc += FUNROLL) {
        const long blocks = (long)tiles * ((nw + kc - 1) / kc);
        const long rounds = (blocks + slots - 1) / slots;
        const long cost = rounds * (kc + 2);
        if (best_cost < 0 || cost < best_cost) { best_cost = cost; best = kc; }
    }
    return best;
}

template <class T, int W, bool ZIN>
static int fused_slots() {
    static int slots[64] = {0};
    int dev = 0;
    DWP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) fail(DWP_EINVAL, "internal: device index out of range");
    if (!slots[dev]) {
        int cus = 0, per = 0;
        DWP_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        DWP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sweep_fused<T, W, ZIN>, FNT, 0));
        slots[dev] = std::max(1, cus * per);
    }
    return slots[dev];
}

template <class T, int W, bool ZIN>
static void sweep_fused_w(hipStream_t s, const Level &L, const T *uin, T *uout, int first_color,
                          hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    LevelArgs a = level_args(L);
    const int tx = (L.nx + FTX - 1) / FTX, ty = (L.ny + FTY - 1) / FTY;
    const int kc = fused_chunk(tx * ty, L.nw, fused_slots<T, W, ZIN>());
    const int tz = (L.nw + kc - 1) / kc;
    const int nb = tx * ty * tz, padded = (nb + 7) / 8 * 8;
    hipExtLaunchKernelGGL(k_sweep_fused<T, W, ZIN>, dim3(padded), dim3(FNT), 0, s, e0, e1, 0, uin, uout,
                          L.eps.as<T>(), L.f.as<T>(), a, first_color, tx, ty, kc, nb);
    DWP_LAUNCH_CHECK();
}
template <class T, int W>
static void sweep_fused_z(hipStream_t s, const Level &L, const T *uin, T *uout, int first_color, bool zero_in,
                          hipEvent_t e0, hipEvent_t e1) {
    if (zero_in) sweep_fused_w<T, W, true>(s, L, uin, uout, first_color, e0, e1);
    else sweep_fused_w<T, W, false>(s, L, uin, uout, first_color, e0, e1);
}

// Row-band sweep: returns false (and launches nothing) where the band shape
// does not fit -- nx not a multiple of W, more than 1024 threads per block,
// or no band height ty in BAND_ROWS that divides ny.  ty = 0 picks the first
// height that fits; the chunk kc is chosen by the same round-filling cost
// model as the tiled kernel's.
constexpr int BAND_ROWS[] = {12, 8, 16, 6, 4};
template <class T, int W>
static bool band_rows_fit(const Level &L, int t) {
    const long nt = (long)(t + 4) * (L.nx / W);
    const size_t bytes = sizeof(T) * (size_t)band_lds_elems(L.nx, t);
    return L.nx % W == 0 && L.nx >= 2 * W && t >= 2 && t % 2 == 0 && L.ny % t == 0 && L.ny >= t + 4 && nt <= 1024 &&
           bytes <= BOTTOM_LDS_BYTES;
}
template <class T, int W>
static int band_rows(const Level &L) {
    for (int t : BAND_ROWS)
        if (band_rows_fit<T, W>(L, t)) return t;
    return 0;
}
template <class T, int W, bool ZIN>
static bool sweep_band_w(hipStream_t s, const Level &L, const T *uin, T *uout, int first_color, int ty,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr, T *zadd = nullptr, int nzb = 0,
                         int kw0 = 0) {
    if (ty == 0) ty = band_rows<T, W>(L);
    if (ty == 0 || !band_rows_fit<T, W>(L, ty)) return false;
    const int nt = (ty + 4) * (L.nx / W);
    const size_t bytes = sizeof(T) * (size_t)band_lds_elems(L.nx, ty);
    const int per = occupancy(reinterpret_cast<const void *>(&k_sweep_band<T, W, ZIN>), nt, bytes);
    if (per < 1) return false;
    const int bands = L.ny / ty;
    const long slots = (long)cu_count() * per;
    int kc = 1;
    long best = -1;
    for (int c = 1; c <= 64; ++c) {
        const long blocks = (long)bands * ((L.nw + c - 1) / c);
        const long cost = (blocks + slots - 1) / slots * (c + 2);
        if (best < 0 || cost < best) { best = cost; kc = c; }
    }
    const int nb = bands * ((L.nw + kc - 1) / kc), padded = (nb + 7) / 8 * 8;
    const int gb = bands % 4 == 0 ? 4 : (bands % 2 == 0 ? 2 : 1);
    const LevelArgs la = level_args(L);
    const bool f32 = sizeof(T) == 4;
    BandArgs<T> a{uin, uout, L.eps.as<T>(), L.f.as<T>(), L.nx, L.ny, L.nw, ty, bands, kc, first_color,
                  (T)(f32 ? la.cxf : la.cx), (T)(f32 ? la.cyf : la.cy), (T)(f32 ? la.czf : la.cz),
                  zadd, nzb, kw0};
    hipExtLaunchKernelGGL(k_sweep_band<T, W, ZIN>, dim3(padded), dim3(nt), (uint32_t)bytes, s, e0, e1, 0, a, nb, gb);
    DWP_LAUNCH_CHECK();
    return true;
}

// 16-byte tile loads when nx allows (float: nx % 4 == 0), else 8-byte ones;
// the level arrays come from hipMalloc and planes are whole vectors.
template <>
bool sweep_band_fits<float>(const Level &L) {
    return L.nx % 4 == 0 ? band_rows<float, 4>(L) != 0 : band_rows<float, 2>(L) != 0;
}
template <>
bool sweep_band_fits<double>(const Level &L) {
    return band_rows<double, 2>(L) != 0;
}
// The row-band kernel where its shape fits (unless tiles_only), else the
// tiled one.
template <class T, int W>
static bool sweep_band_z(hipStream_t s, const Level &L, const T *uin, T *uout, int first_color, bool zero_in,
                         hipEvent_t e0, hipEvent_t e1, T *zadd, int nzb, int kw0) {
    return zero_in ? sweep_band_w<T, W, true>(s, L, uin, uout, first_color, 0, e0, e1, zadd, nzb, kw0)
                   : sweep_band_w<T, W, false>(s, L, uin, uout, first_color, 0, e0, e1, zadd, nzb, kw0);
}
// Returns whether the sweep added its output into zadd (the row-band kernel
// did); otherwise it is in uout.
template <>
bool launch_sweep_fused<float>(hipStream_t s, const Level &L, const float *uin, float *uout, int first_color,
                               bool zero_in, bool tiles_only, hipEvent_t e0, hipEvent_t e1, float *zadd, int nzb,
                               int kw0) {
    const bool w4 = L.nx % 4 == 0;
    if (!tiles_only && (w4 ? sweep_band_z<float, 4>(s, L, uin, uout, first_color, zero_in, e0, e1, zadd, nzb, kw0)
                           : sweep_band_z<float, 2>(s, L, uin, uout, first_color, zero_in, e0, e1, zadd, nzb, kw0)))
        return zadd != nullptr;
    if (w4) sweep_fused_z<float, 4>(s, L, uin, uout, first_color, zero_in, e0, e1);
    else sweep_fused_z<float, 2>(s, L, uin, uout, first_color, zero_in, e0, e1);
    return false;
}
template <>
bool launch_sweep_fused<double>(hipStream_t s, const Level &L, const double *uin, double *uout, int first_color,
                                bool zero_in, bool tiles_only, hipEvent_t e0, hipEvent_t e1, double *zadd, int nzb,
                                int kw0) {
    if (!tiles_only && sweep_band_z<double, 2>(s, L, uin, uout, first_color, zero_in, e0, e1, zadd, nzb, kw0))
        return zadd != nullptr;
    sweep_fused_z<double, 2>(s, L, uin, uout, first_color, zero_in, e0, e1);
    return false;
}

template <class T>
void launch_vcycle_bottom(hipStream_t s, const std::vector<Level *> &levels, size_t l0, int pre, int post,
                          int coarse_sweeps) {
    Bottom<T> B{};
    B.nl = (int)(levels.size() - l0);
    if (B.nl < 1 || B.nl > MAX_BOTTOM) fail(DWP_EINVAL, "internal: bad bottom level count");
    for (int l = 0; l < B.nl; ++l) {
        const Level &L = *levels[l0 + l];
        B.L[l].u = L.u.as<T>();
        B.L[l].f = L.f.as<T>();
        B.L[l].r = L.r.as<T>();
        B.L[l].e = L.eps.as<T>();
        B.L[l].a = level_args(L);
        B.L[l].zc = L.zc ? 1 : 0;
        B.L[l].mh = bt_magic(L.nx / 2);
        B.L[l].mx = bt_magic(L.nx);
        B.L[l].my = bt_magic(L.ny);
    }
    B.pre = pre;
    B.post = post;
    B.coarse = coarse_sweeps;
    // LDS layout of the whole bottom set, if it fits one workgroup's LDS
    BottomLds O{};
    size_t at = 0;
    for (int l = 0; l < B.nl; ++l) {
        const Level &L = *levels[l0 + l];
        const size_t ng = L.n_ghosted(), ni = L.n_interior();
        O.off[4 * l] = (int)at; at += ng;
        O.off[4 * l + 1] = (int)at; at += ni;
        O.off[4 * l + 2] = (int)at; at += ni;
        O.off[4 * l + 3] = (int)at; at += ng;
        at = (at + 3) / 4 * 4;  // keep every array 16-byte aligned
    }
    const size_t bytes = at * sizeof(T);
    if (bytes <= BOTTOM_LDS_BYTES) {
        // the dynamic-LDS limit is raised once per device (the contexts of one
        // process may sit on several)
        static bool attr_set[64] = {false};
        int dev = 0;
        DWP_HIP(hipGetDevice(&dev));
        if (dev < 0 || dev >= 64) fail(DWP_EINVAL, "internal: device index out of range");
        if (!attr_set[dev]) {
            DWP_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_vcycle_bottom_lds<T>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)BOTTOM_LDS_BYTES));
            attr_set[dev] = true;
        }
        k_vcycle_bottom_lds<T><<<1, 1024, bytes, s>>>(B, O);
    } else {
        k_vcycle_bottom<T><<<1, 1024, 0, s>>>(B);
    }
    DWP_LAUNCH_CHECK();
}

template <class T>
void launch_zero(hipStream_t s, T *x, size_t n) {
    k_zero<T><<<grid1d(n), 256, 0, s>>>(x, n);
    DWP_LAUNCH_CHECK();
}

#define DWP_INST(T)                                                                                  \
    template void launch_wet_residual<T>(hipStream_t, const Plan &, const double *, const double *,  \
                                         const double *, T *);                                      \
    template void launch_wet_residual_v32<T>(hipStream_t, const Plan &, const float *, const float *,   \
                                             const float *, T *);                                        \
    template void launch_wet_residual_v16<T>(hipStream_t, const Plan &, const _Float16 *, const float *, \
                                             const float *, T *);                                        \
    template void launch_wet_add<T>(hipStream_t, const Plan &, const T *, double *);                  \
    template void launch_wet_add<T>(hipStream_t, const Plan &, const T *, float *);                   \
    template void launch_wet_eps<T>(hipStream_t, const Plan &, const double *, T *);                  \
    template void launch_level_residual<T>(hipStream_t, const Level &, T *);                          \
    template void launch_level_smooth<T>(hipStream_t, const Level &, int);                            \
    template void launch_restrict<T>(hipStream_t, const Level &, const Level &, const T *, T *);      \
    template void launch_resid_restrict<T>(hipStream_t, const Level &, const Level &);                \
    template void launch_prolong_add<T>(hipStream_t, const Level &, const Level &);                   \
    template void launch_coarsen_eps<T>(hipStream_t, const Level &, const Level &);                   \
    template void launch_zero<T>(hipStream_t, T *, size_t);                                          \
    template void launch_vcycle_bottom<T>(hipStream_t, const std::vector<Level *> &, size_t, int, int, int);
DWP_INST(float)
DWP_INST(double)

}  // namespace dwp
