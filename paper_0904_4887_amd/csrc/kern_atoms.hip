// Atom-dependent kernels: the permittivity built from the atoms, the Gaussian
// charge density, and the atomic forces dE/dR (paper Eq. 11, App. B).  Two
// permittivity models: the product of switches described next, and the
// paper's dummy density (Eqs. 9, 10, 19) further down.
//
// Permittivity: eps_n = 1 + (eps_inf - 1) prod_i s_i(d_in) H(z_n) with
// s_i(d) = 1/2 [1 + erf((d - r_i)/delta)] (exactly 0 below r_i - 6 delta and 1
// beyond r_i + 6 delta) and, when the exclusion rule is on, the height factor
// H(z) = prod_{z_i <= z_lim} 1/2 [1 + erf((z - z_i)/delta_z)] of the buried
// atoms (the smooth counterpart of the paper's Eq. 19).
//
// Forces: dE/dR_I = sum_n g_n d eps_n/dR_I + h^3 sum_n phi_n d rho_n/dR_I with
// g = dE/d eps.  The switch part needs the product of the OTHER switches at
// each node; it is S_n / s_I(n) with S_n = prod_i s_i(n) kept from the eps
// build (s_I > 0 wherever its derivative is non-zero).  The height-factor part
// of buried atoms depends on z only and is reduced per plane first.  All sums
// are per block, then per atom in a fixed order.
//
// Packed atom record (8 doubles): x, y, z, radius, q, sigma, buried, 0.
#include "dwp_internal.h"

namespace dwp {

namespace {

constexpr int AT_THREADS = 256;
constexpr int FU = 4;  // nodes of a z column whose loads k_forces issues together
constexpr int AREC = 8;
constexpr double PI = 3.14159265358979323846;
constexpr double SQRT_PI = 1.77245385090551602730;

__device__ __forceinline__ double min_image(double d, double L, double invL) { return d - L * rint(d * invL); }

struct Box {
    int nx, ny, nz;
    double hx, hy, hz, Lx, Ly, Lz, iLx, iLy, iLz;
};

Box make_box(const Plan &p) {
    Box b;
    b.nx = p.nx; b.ny = p.ny; b.nz = p.nz;
    b.hx = p.h[0]; b.hy = p.h[1]; b.hz = p.h[2];
    b.Lx = p.L[0]; b.Ly = p.L[1]; b.Lz = p.L[2];
    b.iLx = 1.0 / p.L[0]; b.iLy = 1.0 / p.L[1]; b.iLz = 1.0 / p.L[2];
    return b;
}

// Block-wide exclusive scan of 0/1 flags (AT_THREADS entries); returns this
// thread's slot and writes the total to *total.  Deterministic order.
__device__ int block_compact(int flag, int *scan, int *total) {
    scan[threadIdx.x] = flag;
    __syncthreads();
    for (int off = 1; off < AT_THREADS; off <<= 1) {
        const int v = (int)threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
    }
    const int incl = scan[threadIdx.x];
    *total = scan[AT_THREADS - 1];
    __syncthreads();
    return incl - flag;
}

// Tile of the grid handled by one block of the builders: 32 x 4 x 2 nodes.
constexpr int TX = 32, TY = 4, TZ = 2;

// Minimum-image distance (squared) from point a to the axis-aligned tile
// [lo, hi] (lengths well below L / 2).
__device__ __forceinline__ double dist2_to_tile(const Box &b, double ax, double ay, double az, double x0, double x1,
                                                double y0, double y1, double z0, double z1) {
    const double cx = 0.5 * (x0 + x1), cy = 0.5 * (y0 + y1), cz = 0.5 * (z0 + z1);
    const double dx = fmax(0.0, fabs(min_image(ax - cx, b.Lx, b.iLx)) - 0.5 * (x1 - x0));
    const double dy = fmax(0.0, fabs(min_image(ay - cy, b.Ly, b.iLy)) - 0.5 * (y1 - y0));
    const double dz = fmax(0.0, fabs(min_image(az - cz, b.Lz, b.iLz)) - 0.5 * (z1 - z0));
    return dx * dx + dy * dy + dz * dz;
}

// mode 0: permittivity switches (cutoff r + 6 delta); mode 1: Gaussians (9 sigma)
template <int MODE>
__global__ void __launch_bounds__(AT_THREADS)
k_build(const double *__restrict__ atoms, int natoms, Box b, double eps_inf, double delta,
        const double *__restrict__ Hz, double *__restrict__ out, double *__restrict__ S) {
    __shared__ double ax[AT_THREADS], ay[AT_THREADS], az[AT_THREADS], ar[AT_THREADS], aq[AT_THREADS];
    __shared__ int scan[AT_THREADS];
    __shared__ int cnt;
    const int tx = threadIdx.x % TX, ty = (threadIdx.x / TX) % TY, tz = threadIdx.x / (TX * TY);
    const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY, k0 = blockIdx.z * TZ;
    const int i = i0 + tx, j = j0 + ty, k = k0 + tz;
    const bool live = i < b.nx && j < b.ny && k < b.nz;
    const double x = i * b.hx, y = j * b.hy, z = k * b.hz;
    const double x0 = i0 * b.hx, x1 = min(i0 + TX - 1, b.nx - 1) * b.hx;
    const double y0 = j0 * b.hy, y1 = min(j0 + TY - 1, b.ny - 1) * b.hy;
    const double z0 = k0 * b.hz, z1 = min(k0 + TZ - 1, b.nz - 1) * b.hz;
    double acc = MODE == 0 ? 1.0 : 0.0;
    bool zero = false;
    for (int base = 0; base < natoms; base += AT_THREADS) {
        const int a = base + threadIdx.x;
        int keep = 0;
        double px = 0, py = 0, pz = 0, pr = 0, pq = 0;
        if (a < natoms) {
            const double *r = atoms + (size_t)a * AREC;
            px = r[0]; py = r[1]; pz = r[2];
            const double cut = MODE == 0 ? r[3] + 6.0 * delta : 9.0 * r[5];
            pr = MODE == 0 ? r[3] : r[5];
            // a Gaussian's amplitude q (2 pi sigma^2)^(-3/2), once per atom
            pq = MODE == 0 ? r[4] : r[4] * pow(2.0 * PI * r[5] * r[5], -1.5);
            keep = dist2_to_tile(b, px, py, pz, x0, x1, y0, y1, z0, z1) < cut * cut;
        }
        int total;
        const int slot = block_compact(keep, scan, &total);
        if (keep) { ax[slot] = px; ay[slot] = py; az[slot] = pz; ar[slot] = pr; aq[slot] = pq; }
        if (threadIdx.x == 0) cnt = total;
        __syncthreads();
        const int m = cnt;
        if (live && !zero) {
            for (int q = 0; q < m; ++q) {
                const double dx = min_image(x - ax[q], b.Lx, b.iLx);
                const double dy = min_image(y - ay[q], b.Ly, b.iLy);
                const double dz = min_image(z - az[q], b.Lz, b.iLz);
                const double d2 = dx * dx + dy * dy + dz * dz;
                if (MODE == 0) {
                    const double d = sqrt(d2);
                    const double t = (d - ar[q]) / delta;
                    if (t <= -6.0) { zero = true; break; }
                    if (t < 6.0) acc *= 0.5 * (1.0 + erf(t));
                } else {
                    const double s2 = ar[q] * ar[q];
                    if (d2 < 81.0 * s2) acc += aq[q] * exp(-d2 / (2.0 * s2));
                }
            }
        }
        __syncthreads();
    }
    if (!live) return;
    const size_t c = ((size_t)k * b.ny + j) * b.nx + i;
    if (MODE == 0) {
        const double Sv = zero ? 0.0 : acc;
        const double H = Hz ? Hz[k] : 1.0;
        out[c] = 1.0 + (eps_inf - 1.0) * Sv * H;
        if (S) S[c] = Sv;
    } else {
        out[c] = acc;
    }
}

// H(z_k) = prod over buried atoms of 1/2 [1 + erf((z_k - z_i)/delta_z)]
__global__ void k_height(const double *__restrict__ atoms, int natoms, int nz, double hz, double delta_z,
                         double *__restrict__ Hz) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nz) return;
    const double z = k * hz;
    double H = 1.0;
    for (int a = 0; a < natoms; ++a) {
        const double *r = atoms + (size_t)a * AREC;
        if (r[6] == 0.0) continue;
        const double t = (z - r[2]) / delta_z;
        if (t <= -6.0) { H = 0.0; break; }
        if (t < 6.0) H *= 0.5 * (1.0 + erf(t));
    }
    Hz[k] = H;
}

// ------------------------------------------------------ dummy-density model
// gamma_n = sum_a exp(t_an), t_an = -s_an (d_an - R_a) / decay (Eq. 9), with
// s_an = -1 for a buried atom a above the node (Eq. 19), else +1; then
// eps = 1 + (eps_inf - 1) q, q = 1 / (1 + gamma^(2 beta)) (Eq. 10), and the
// force kernel's inputs log gamma and K = d eps / d log gamma = -(eps_inf - 1)
// 2 beta q (1 - q).  Every atom contributes at every node (minimum image, no
// cut-off); the cell size check on the host keeps |t| < 600, so gamma neither
// overflows nor underflows.
__device__ __forceinline__ double gamma_exponent(double d, double R, double sgn, double inv_decay) {
    return -sgn * (d - R) * inv_decay;
}

__global__ void __launch_bounds__(AT_THREADS)
k_build_gamma(const double *__restrict__ atoms, int natoms, Box b, double eps_inf, double two_beta,
              double inv_decay, double *__restrict__ eps, double *__restrict__ S) {
    __shared__ double ax[AT_THREADS], ay[AT_THREADS], az[AT_THREADS], ar[AT_THREADS], ab[AT_THREADS];
    const int tx = threadIdx.x % TX, ty = (threadIdx.x / TX) % TY, tz = threadIdx.x / (TX * TY);
    const int i = blockIdx.x * TX + tx, j = blockIdx.y * TY + ty, k = blockIdx.z * TZ + tz;
    const bool live = i < b.nx && j < b.ny && k < b.nz;
    const double x = i * b.hx, y = j * b.hy, z = k * b.hz;
    double acc = 0.0;
    for (int base = 0; base < natoms; base += AT_THREADS) {
        const int a = base + threadIdx.x;
        if (a < natoms) {
            const double *r = atoms + (size_t)a * AREC;
            ax[threadIdx.x] = r[0]; ay[threadIdx.x] = r[1]; az[threadIdx.x] = r[2];
            ar[threadIdx.x] = r[3]; ab[threadIdx.x] = r[6];
        }
        __syncthreads();
        const int m = min(AT_THREADS, natoms - base);
        if (live) {
            for (int q = 0; q < m; ++q) {
                const double dx = min_image(x - ax[q], b.Lx, b.iLx);
                const double dy = min_image(y - ay[q], b.Ly, b.iLy);
                const double dz = min_image(z - az[q], b.Lz, b.iLz);
                const double d = sqrt(dx * dx + dy * dy + dz * dz);
                const double sgn = (ab[q] != 0.0 && z < az[q]) ? -1.0 : 1.0;
                acc += exp(gamma_exponent(d, ar[q], sgn, inv_decay));
            }
        }
        __syncthreads();
    }
    if (!live) return;
    const size_t c = ((size_t)k * b.ny + j) * b.nx + i;
    const size_t N = (size_t)b.nx * b.ny * b.nz;
    const double lg = log(acc);
    const double q = 1.0 / (1.0 + exp(two_beta * lg));   // exp overflows to inf: q = 0, eps = 1
    eps[c] = 1.0 + (eps_inf - 1.0) * q;
    S[c] = lg;
    S[N + c] = -(eps_inf - 1.0) * two_beta * q * (1.0 - q);
}

// Permittivity term of dE/dR for the dummy-density model:
//   dE/dR_a = sum_n g_n K_n exp(t_an - log gamma_n) s_an (r_n - R_a) / (decay d_an).
// Atoms are taken GA at a time with their sums in registers; each block walks
// its share of the nodes (one node per thread per step, grid-stride), so the
// node data (g, K, log gamma) is read once per group of GA atoms.  At the end
// of a group the block reduces its GA x 3 sums (waves, then the four waves in a
// fixed order) and writes them as its partial.  Nodes with g K = 0 add nothing.
constexpr int GA = 8;
constexpr int GAMMA_FORCE_BLOCKS = 2048;

__global__ void __launch_bounds__(AT_THREADS)
k_forces_gamma(const double *__restrict__ atoms, int natoms, Box b, double inv_decay,
               const double *__restrict__ g, const double *__restrict__ S, double *__restrict__ gpart) {
    __shared__ double red[AT_THREADS / 64][GA * 3];
    const size_t N = (size_t)b.nx * b.ny * b.nz;
    const size_t plane = (size_t)b.nx * b.ny;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int g0 = 0; g0 < natoms; g0 += GA) {
        double px[GA], py[GA], pz[GA], pr[GA], pb[GA];
#pragma unroll
        for (int q = 0; q < GA; ++q) {
            const int a = min(g0 + q, natoms - 1);
            const double *r = atoms + (size_t)a * AREC;
            px[q] = r[0]; py[q] = r[1]; pz[q] = r[2]; pr[q] = r[3]; pb[q] = r[6];
        }
        double f[GA][3];
#pragma unroll
        for (int q = 0; q < GA; ++q) f[q][0] = f[q][1] = f[q][2] = 0.0;
        // node index c and its (i, j, k), advanced by the grid stride without divisions
        const size_t stride = (size_t)gridDim.x * AT_THREADS;
        const size_t sk = stride / plane, sr = stride - sk * plane;
        const int sj = (int)(sr / b.nx), si = (int)(sr - (size_t)sj * b.nx);
        size_t c = (size_t)blockIdx.x * AT_THREADS + threadIdx.x;
        size_t k = c / plane;
        int j = (int)((c - k * plane) / b.nx), i = (int)(c - k * plane - (size_t)j * b.nx);
        for (; c < N; c += stride) {
            const double w = g[c] * S[N + c] * inv_decay;
            const double lg = S[c];
            const double x = i * b.hx, y = j * b.hy, z = k * b.hz;
            i += si; j += sj; k += sk;
            if (i >= b.nx) { i -= b.nx; ++j; }
            if (j >= b.ny) { j -= b.ny; ++k; }
            if (w == 0.0) continue;
#pragma unroll
            for (int q = 0; q < GA; ++q) {
                const double dx = min_image(x - px[q], b.Lx, b.iLx);
                const double dy = min_image(y - py[q], b.Ly, b.iLy);
                const double dz = min_image(z - pz[q], b.Lz, b.iLz);
                const double d = sqrt(dx * dx + dy * dy + dz * dz);
                const double sgn = (pb[q] != 0.0 && z < pz[q]) ? -1.0 : 1.0;
                const double e = w * exp(gamma_exponent(d, pr[q], sgn, inv_decay) - lg) * sgn;
                const double v = d > 0.0 ? e / d : 0.0;
                f[q][0] += v * dx; f[q][1] += v * dy; f[q][2] += v * dz;
            }
        }
#pragma unroll
        for (int q = 0; q < GA; ++q)
#pragma unroll
            for (int comp = 0; comp < 3; ++comp) {
                double v = f[q][comp];
                for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
                if (lane == 0) red[wid][q * 3 + comp] = v;
            }
        __syncthreads();
        if ((int)threadIdx.x < GA * 3) {
            const int q = threadIdx.x / 3;
            if (g0 + q < natoms) {
                double v = 0.0;
                for (int w2 = 0; w2 < AT_THREADS / 64; ++w2) v += red[w2][threadIdx.x];
                gpart[((size_t)blockIdx.x * natoms + g0) * 3 + threadIdx.x] = v;
            }
        }
        __syncthreads();
    }
}

// out[a][c] = charge term (sum over its chunks) + permittivity term (sum over
// the node blocks); one block per (atom, component), fixed-order reductions.
__global__ void __launch_bounds__(AT_THREADS)
k_forces_gamma_final(const double *__restrict__ fpart, int natoms, int nchunk,
                     const double *__restrict__ gpart, int nblocks, double *__restrict__ out) {
    __shared__ double red[AT_THREADS / 64];
    const int t = blockIdx.x;
    const int a = t / 3, c = t % 3;
    double e = 0.0;
    for (int q = threadIdx.x; q < nblocks; q += AT_THREADS) e += gpart[((size_t)q * natoms + a) * 3 + c];
    for (int o = 32; o > 0; o >>= 1) e += __shfl_down(e, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < nchunk; ++q) s += fpart[((size_t)a * nchunk + q) * 3 + c];
        double v = 0.0;
        for (int w = 0; w < AT_THREADS / 64; ++w) v += red[w];
        out[t] = s + v;
    }
}

int gamma_force_blocks(const Plan &p) {
    const size_t tiles = (p.N + AT_THREADS - 1) / AT_THREADS;
    return (int)std::min<size_t>(tiles, GAMMA_FORCE_BLOCKS);
}

// ---------------------------------------------------------------- forces
// Block = (atom a, chunk of the (x, y) columns of the cube around atom a).
// A thread walks one column in z over the chord inside the cut-off ball.
// The product of the OTHER switches at a node is S_n / s_a(n), with S_n the
// product of all switches stored when eps was built: on the shell where
// atom a's switch varies (|t| < 6), s_a >= erfc(6)/2 > 0, and S_n = 0
// exactly where any other switch vanishes, so the quotient is the product
// itself up to rounding.
__global__ void __launch_bounds__(AT_THREADS)
k_forces(const double *__restrict__ atoms, Box b, int eps_mode, double eps_inf, double delta,
         const double *__restrict__ phi, const double *__restrict__ g, const double *__restrict__ S,
         const double *__restrict__ Hz, int nchunk, double *__restrict__ fpart) {
    __shared__ double red[3][AT_THREADS / 64];
    const int a = blockIdx.x / nchunk, chunk = blockIdx.x % nchunk;
    const double *ra = atoms + (size_t)a * AREC;
    const double X = ra[0], Y = ra[1], Z = ra[2], Ra = ra[3], Q = ra[4], Sg = ra[5];
    const double ceps = eps_mode ? Ra + 6.0 * delta : 0.0;
    const double crho = 9.0 * Sg;
    const double Rc = fmax(ceps, crho);
    const double h3 = b.hx * b.hy * b.hz;
    const double gnorm = h3 * Q * pow(2.0 * PI * Sg * Sg, -1.5) / (Sg * Sg);
    const double inv2s2 = 1.0 / (2.0 * Sg * Sg);
    const double wz_eps = -(eps_inf - 1.0) / (delta * SQRT_PI);
    // node ranges (unwrapped indices)
    const int ilo = (int)ceil((X - Rc) / b.hx), ihi = (int)floor((X + Rc) / b.hx);
    const int jlo = (int)ceil((Y - Rc) / b.hy), jhi = (int)floor((Y + Rc) / b.hy);
    const int klo = (int)ceil((Z - Rc) / b.hz), khi = (int)floor((Z + Rc) / b.hz);
    const int cx = ihi - ilo + 1, cy = jhi - jlo + 1;
    const int ncol = cx * cy;
    const int per = (ncol + nchunk - 1) / nchunk;
    const int c0 = chunk * per, c1 = min(ncol, c0 + per);
    const size_t plane = (size_t)b.nx * b.ny;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int col = c0 + (int)threadIdx.x; col < c1; col += AT_THREADS) {
        const int iu = ilo + col % cx, ju = jlo + col / cx;
        const int i = ((iu % b.nx) + b.nx) % b.nx, j = ((ju % b.ny) + b.ny) % b.ny;
        const double dx = min_image(i * b.hx - X, b.Lx, b.iLx), dy = min_image(j * b.hy - Y, b.Ly, b.iLy);
        const double dxy2 = dx * dx + dy * dy;
        if (dxy2 >= Rc * Rc) continue;
        const double dzm = sqrt(Rc * Rc - dxy2);
        const int kl = max(klo, (int)ceil((Z - dzm) / b.hz)), kh = min(khi, (int)floor((Z + dzm) / b.hz));
        const size_t colbase = (size_t)j * b.nx + i;
        int k = ((kl % b.nz) + b.nz) % b.nz;
        // FU nodes of the column at a time: their loads are issued together,
        // then used in order (the sums' order is that of the nodes)
        for (int ku0 = kl; ku0 <= kh; ku0 += FU) {
            int kk[FU];
            double ph[FU], sv[FU], gv[FU], hv[FU];
#pragma unroll
            for (int u = 0; u < FU; ++u) {
                kk[u] = k;
                k = (k + 1 == b.nz) ? 0 : k + 1;
                ph[u] = sv[u] = gv[u] = 0.0;
                hv[u] = 1.0;
                if (ku0 + u > kh) continue;
                const double dz = min_image(kk[u] * b.hz - Z, b.Lz, b.iLz);
                const double d2 = dxy2 + dz * dz;
                const size_t c = (size_t)kk[u] * plane + colbase;
                if (d2 < crho * crho) ph[u] = phi[c];
                if (eps_mode) {
                    const double t = (sqrt(d2) - Ra) / delta;
                    if (t > -6.0 && t < 6.0) {
                        sv[u] = S[c];
                        gv[u] = g[c];
                        if (Hz) hv[u] = Hz[kk[u]];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < FU; ++u) {
                if (ku0 + u > kh) break;
                const double dz = min_image(kk[u] * b.hz - Z, b.Lz, b.iLz);
                const double d2 = dx * dx + dy * dy + dz * dz;
                // charge term: d rho_n / dR_a = q G(d) (r_n - R_a) / sigma^2
                if (d2 < crho * crho) {
                    const double w = gnorm * ph[u] * exp(-d2 * inv2s2);
                    fx += w * dx; fy += w * dy; fz += w * dz;
                }
                if (eps_mode) {
                    const double d = sqrt(d2);
                    const double t = (d - Ra) / delta;
                    if (t > -6.0 && t < 6.0 && d > 0.0) {
                        const double Sv = sv[u];
                        if (Sv != 0.0) {
                            const double H = hv[u];
                            const double sa = 0.5 * (1.0 + erf(t));
                            // d eps / dR_a = (eps_inf - 1) H (S / s_a) s_a'(t) (-(r - R_a) / (d delta))
                            const double w = wz_eps * gv[u] * H * (Sv / sa) * exp(-t * t) / d;
                            fx += w * dx; fy += w * dy; fz += w * dz;
                        }
                    }
                }
            }
        }
    }
    // block reduction of (fx, fy, fz)
    double v[3] = {fx, fy, fz};
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int c = 0; c < 3; ++c) {
        double s = v[c];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
        if (lane == 0) red[c][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int w = 0; w < AT_THREADS / 64; ++w) s += red[threadIdx.x][w];
        fpart[(size_t)blockIdx.x * 3 + threadIdx.x] = s;
    }
}

// Plane sums Q_k = sum_{i,j} g_ijk S_ijk (one block per plane).
__global__ void __launch_bounds__(AT_THREADS)
k_plane_gs(const double *__restrict__ g, const double *__restrict__ S, int nx, int ny, double *__restrict__ Q) {
    __shared__ double red[AT_THREADS / 64];
    const size_t plane = (size_t)nx * ny;
    const size_t base = (size_t)blockIdx.x * plane;
    double s = 0.0;
    for (size_t t = threadIdx.x; t < plane; t += AT_THREADS) s += g[base + t] * S[base + t];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int w = 0; w < AT_THREADS / 64; ++w) r += red[w];
        Q[blockIdx.x] = r;
    }
}

// Height-factor force on buried atom a (one block per atom):
// dE/dz_a += (eps_inf - 1) sum_k Q_k prod_{K buried != a} h_K(z_k) (-h_a'(z_k)).
__global__ void __launch_bounds__(AT_THREADS)
k_height_forces(const double *__restrict__ atoms, int natoms, int nz, double hz, double delta_z, double eps_inf,
                const double *__restrict__ Q, double *__restrict__ out) {
    __shared__ double red[AT_THREADS / 64];
    const int a = blockIdx.x;
    const double *ra = atoms + (size_t)a * AREC;
    if (ra[6] == 0.0) {
        if (threadIdx.x == 0) out[a] = 0.0;
        return;
    }
    const double za = ra[2];
    double s = 0.0;
    for (int k = threadIdx.x; k < nz; k += AT_THREADS) {
        const double z = k * hz;
        const double ta = (z - za) / delta_z;
        if (ta <= -6.0 || ta >= 6.0) continue;
        double P = 1.0;
        for (int K = 0; K < natoms; ++K) {
            if (K == a) continue;
            const double *r = atoms + (size_t)K * AREC;
            if (r[6] == 0.0) continue;
            const double t = (z - r[2]) / delta_z;
            if (t <= -6.0) { P = 0.0; break; }
            if (t < 6.0) P *= 0.5 * (1.0 + erf(t));
        }
        const double dh = exp(-ta * ta) / (delta_z * SQRT_PI);  // d h_a / dz; d h_a / dz_a = -dh
        s += Q[k] * P * (-dh);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int w = 0; w < AT_THREADS / 64; ++w) r += red[w];
        out[a] = (eps_inf - 1.0) * r;
    }
}

// out[a][c] = sum over chunks (fixed order) [+ height term on z]
__global__ void k_forces_final(const double *__restrict__ fpart, int natoms, int nchunk,
                               const double *__restrict__ hforce, double *__restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= natoms * 3) return;
    const int a = t / 3, c = t % 3;
    double s = 0.0;
    for (int q = 0; q < nchunk; ++q) s += fpart[((size_t)a * nchunk + q) * 3 + c];
    if (hforce && c == 2) s += hforce[a];
    out[t] = s;
}

int chunks_for(int natoms) {
    int nch = 8192 / (natoms > 0 ? natoms : 1);
    if (nch < 1) nch = 1;
    if (nch > 512) nch = 512;
    return nch;
}

}  // namespace

void launch_build_eps(hipStream_t s, const Plan &p, int n, const double *atoms_dev, const AtomParams &ap,
                      double *Hz, double *eps, double *S) {
    Box b = make_box(p);
    if (ap.model == 1) {
        dim3 g((p.nx + TX - 1) / TX, (p.ny + TY - 1) / TY, (p.nz + TZ - 1) / TZ);
        k_build_gamma<<<g, AT_THREADS, 0, s>>>(atoms_dev, n, b, ap.eps_inf, 2.0 * ap.beta, 1.0 / ap.decay, eps, S);
        DWP_LAUNCH_CHECK();
        return;
    }
    if (ap.exclusion) {
        k_height<<<(p.nz + 127) / 128, 128, 0, s>>>(atoms_dev, n, p.nz, p.h[2], ap.delta_z, Hz);
        DWP_LAUNCH_CHECK();
    }
    dim3 g((p.nx + TX - 1) / TX, (p.ny + TY - 1) / TY, (p.nz + TZ - 1) / TZ);
    k_build<0><<<g, AT_THREADS, 0, s>>>(atoms_dev, n, b, ap.eps_inf, ap.delta, ap.exclusion ? Hz : nullptr, eps,
                                        S);
    DWP_LAUNCH_CHECK();
}

void launch_build_rho(hipStream_t s, const Plan &p, int n, const double *atoms_dev, double *rho) {
    Box b = make_box(p);
    dim3 g((p.nx + TX - 1) / TX, (p.ny + TY - 1) / TY, (p.nz + TZ - 1) / TZ);
    k_build<1><<<g, AT_THREADS, 0, s>>>(atoms_dev, n, b, 0.0, 0.0, nullptr, rho, nullptr);
    DWP_LAUNCH_CHECK();
}

size_t forces_partial_len(const Plan &p, int n, int model) {
    const size_t gamma = model == 1 ? (size_t)gamma_force_blocks(p) * n * 3 : 0;
    return (size_t)n * chunks_for(n) * 3 + (size_t)p.nz + (size_t)n + 64 + gamma;
}

// fpart: forces_partial_len doubles; out: 3n doubles (device)
void launch_forces(hipStream_t s, const Plan &p, int n, const double *atoms_dev, const AtomParams *ap,
                   const double *phi, const double *g, const double *S, const double *Hz, double *fpart,
                   double *out) {
    Box b = make_box(p);
    const int nch = chunks_for(n);
    if (ap && ap->model == 1) {
        // charge term by the atom-centred kernel, permittivity term by node blocks
        k_forces<<<n * nch, AT_THREADS, 0, s>>>(atoms_dev, b, 0, 1.0, 1.0, phi, nullptr, nullptr, nullptr, nch, fpart);
        DWP_LAUNCH_CHECK();
        const int nb = gamma_force_blocks(p);
        double *gpart = fpart + (size_t)n * nch * 3 + (size_t)p.nz + (size_t)n + 64;
        k_forces_gamma<<<nb, AT_THREADS, 0, s>>>(atoms_dev, n, b, 1.0 / ap->decay, g, S, gpart);
        DWP_LAUNCH_CHECK();
        k_forces_gamma_final<<<3 * n, AT_THREADS, 0, s>>>(fpart, n, nch, gpart, nb, out);
        DWP_LAUNCH_CHECK();
        return;
    }
    const bool excl = ap && ap->exclusion;
    k_forces<<<n * nch, AT_THREADS, 0, s>>>(atoms_dev, b, ap ? 1 : 0, ap ? ap->eps_inf : 1.0,
                                            ap ? ap->delta : 1.0, phi, g, S, excl ? Hz : nullptr, nch, fpart);
    DWP_LAUNCH_CHECK();
    double *Q = fpart + (size_t)n * nch * 3;
    double *hf = Q + p.nz;
    if (excl) {
        k_plane_gs<<<p.nz, AT_THREADS, 0, s>>>(g, S, p.nx, p.ny, Q);
        DWP_LAUNCH_CHECK();
        k_height_forces<<<n, AT_THREADS, 0, s>>>(atoms_dev, n, p.nz, p.h[2], ap->delta_z, ap->eps_inf, Q, hf);
        DWP_LAUNCH_CHECK();
    }
    k_forces_final<<<(3 * n + 127) / 128, 128, 0, s>>>(fpart, n, nch, excl ? hf : nullptr, out);
    DWP_LAUNCH_CHECK();
}

}  // namespace dwp
