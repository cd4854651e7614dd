// Deterministic reductions and the Krylov vector kernels.
//
// Every reduction runs on a fixed grid of RED_BLOCKS blocks: each block
// reduces its grid-stride share with wave64 shuffles and LDS and writes one
// partial per output; a second kernel adds the partials of each output in a
// fixed tree order.  Results are therefore bitwise reproducible.  The energy
// sums use compensated (two-sum) accumulation throughout.
#include "dwp_internal.h"

namespace dwp {

namespace {

constexpr int MD_GROUP = 8;   // dot products per pass of multidot
constexpr int MD_STRIDE = 72; // partial slots per block: 64 dots + the norm
constexpr int NORM_SLOT = 64;
constexpr int SUM_SLOT = 65;   // partial column of the sum of w's elements (mean-free Arnoldi step)
constexpr int HC_SUM = 67;     // where that sum lands in the Hessenberg column

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Sum of v over the block; valid in thread 0.  `sh` holds one double per wave.
__device__ __forceinline__ double block_sum(double v, double *sh) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int q = 0; q < nw; ++q) r += sh[q];
    }
    return r;
}

// two-sum accumulator
struct DD {
    double s, c;
};
__device__ __forceinline__ DD dd_add(DD a, double b) {
    const double s = a.s + b;
    const double bp = s - a.s;
    const double e = (a.s - (s - bp)) + (b - bp);
    return DD{s, a.c + e};
}
__device__ __forceinline__ DD dd_merge(DD a, DD b) {
    const double s = a.s + b.s;
    const double bp = s - a.s;
    const double e = (a.s - (s - bp)) + (b.s - bp);
    return DD{s, a.c + b.c + e};
}
__device__ __forceinline__ DD wave_dd(DD v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        DD w{__shfl_down(v.s, o, 64), __shfl_down(v.c, o, 64)};
        v = dd_merge(v, w);
    }
    return v;
}

// partial[b * stride + v0 + q] = sum over block b of V_{v0+q} . w  (q < nv);
// with_norm: partial[b * stride + NORM_SLOT] = sum over block b of w . w
__global__ void __launch_bounds__(RED_THREADS)
k_multidot(const double *__restrict__ V, size_t ldv, int v0, int nv, const double *__restrict__ w, size_t n,
           double *__restrict__ partial, int stride, int with_norm) {
    __shared__ double sh[RED_THREADS / 64];
    double acc[MD_GROUP];
    double accn = 0.0;
#pragma unroll
    for (int q = 0; q < MD_GROUP; ++q) acc[q] = 0.0;
    for (size_t t = blockIdx.x * (size_t)RED_THREADS + threadIdx.x; t < n; t += (size_t)gridDim.x * RED_THREADS) {
        const double wt = w[t];
        accn += wt * wt;
#pragma unroll
        for (int q = 0; q < MD_GROUP; ++q)
            if (q < nv) acc[q] += V[(size_t)(v0 + q) * ldv + t] * wt;
    }
#pragma unroll
    for (int q = 0; q < MD_GROUP; ++q) {
        if (q < nv) {
            const double r = block_sum(acc[q], sh);
            if (threadIdx.x == 0) partial[(size_t)blockIdx.x * stride + v0 + q] = r;
        }
    }
    if (with_norm) {
        const double r = block_sum(accn, sh);
        if (threadIdx.x == 0) partial[(size_t)blockIdx.x * stride + NORM_SLOT] = r;
    }
}

// Sums over the block of NV per-thread values: out[q] valid in thread q.
template <int NV>
__device__ __forceinline__ void block_sums(const double (&v)[NV], double (*sh)[RED_THREADS / 64], double *out) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const double r = wave_sum(v[q]);
        if (lane == 0) sh[q][wid] = r;
    }
    __syncthreads();
    if ((int)threadIdx.x < NV) {
        double r = 0.0;
        for (int w = 0; w < RED_THREADS / 64; ++w) r += sh[threadIdx.x][w];
        out[threadIdx.x] = r;
    }
}

// Pair-vectorised projection: NV dot products V_{v0+q} . w and (with_norm)
// w . w over n2 element pairs (16-byte loads; every vector 16-byte aligned).
template <int NV, bool SUM = false>
__global__ void __launch_bounds__(RED_THREADS)
k_multidot2(const double *__restrict__ V, size_t ldv, int v0, const double *__restrict__ w, size_t n2,
            double *__restrict__ partial, int stride, int with_norm) {
    constexpr int NA = NV + 1 + (SUM ? 1 : 0);  // dots, ||w||^2 [, sum of w]
    __shared__ double sh[NA][RED_THREADS / 64];
    __shared__ double res[NA];
    const double2 *w2 = reinterpret_cast<const double2 *>(w);
    double acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = 0.0;
    for (size_t t = blockIdx.x * (size_t)RED_THREADS + threadIdx.x; t < n2; t += (size_t)gridDim.x * RED_THREADS) {
        const double2 wt = w2[t];
        double2 vq[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) vq[q] = reinterpret_cast<const double2 *>(V + (size_t)(v0 + q) * ldv)[t];
        acc[NV] += wt.x * wt.x + wt.y * wt.y;
        if constexpr (SUM) acc[NV + 1] += wt.x + wt.y;
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] += vq[q].x * wt.x + vq[q].y * wt.y;
    }
    block_sums<NA>(acc, sh, res);
    if ((int)threadIdx.x < NV) partial[(size_t)blockIdx.x * stride + v0 + threadIdx.x] = res[threadIdx.x];
    if (with_norm && threadIdx.x == NV) partial[(size_t)blockIdx.x * stride + NORM_SLOT] = res[NV];
    if (SUM && with_norm && (int)threadIdx.x == NV + 1) partial[(size_t)blockIdx.x * stride + SUM_SLOT] = res[NV + 1];
}

// New Arnoldi vector in one pass: w <- (w - sum_q h_q V_q) / beta with
// beta^2 = ||w||^2 - sum_q h_q^2 (Pythagoras on the projection just computed;
// h at hc[0..NV), ||w||^2 at hc[NORM_SLOT]).  When cancellation leaves no
// reliable beta (beta^2 <= 1e-20 ||w||^2) the divisor is 1.  Block 0 stores
// the divisor at *beta_out; partial[b] receives block b's share of the new
// squared norm, which the caller uses to rescale when it is not 1.
// SUM: w is not yet mean-free (the operator's output before the removal of its
// mean); the constant direction is taken out in the same pass: with mu the
// mean of w (hc[SUM_SLOT] / n), w <- (w - sum_q h_q V_q - mu) / beta and
// beta^2 = ||w||^2 - sum_q h_q^2 - n mu^2, which holds because every V_q is
// mean-free.
template <int NV, bool SUM = false>
__global__ void __launch_bounds__(RED_THREADS)
k_orth_update2(double *__restrict__ w, const double *__restrict__ V, size_t ldv, const double *__restrict__ hc,
               size_t n2, double *__restrict__ partial, double *__restrict__ beta_out) {
    __shared__ double sh[1][RED_THREADS / 64];
    __shared__ double cs[NV + 2];
    __shared__ double res[1];
    if (threadIdx.x == 0) {
        double h2 = 0.0;
        for (int q = 0; q < NV; ++q) h2 += hc[q] * hc[q];
        double mu = 0.0;
        if constexpr (SUM) {
            mu = hc[HC_SUM] / (2.0 * (double)n2);
            h2 += mu * hc[HC_SUM];
        }
        const double w2n = hc[NORM_SLOT], b2 = w2n - h2;
        const double beta = (b2 > 1e-20 * w2n) ? sqrt(b2) : 1.0;
        cs[NV] = 1.0 / beta;
        cs[NV + 1] = -mu;
        if (blockIdx.x == 0) *beta_out = beta;
    }
    if ((int)threadIdx.x < NV) cs[threadIdx.x] = -hc[threadIdx.x];
    __syncthreads();
    const double sc = cs[NV];
    double2 *w2 = reinterpret_cast<double2 *>(w);
    double nrm[1] = {0.0};
    for (size_t t = blockIdx.x * (size_t)RED_THREADS + threadIdx.x; t < n2; t += (size_t)gridDim.x * RED_THREADS) {
        double2 acc = w2[t];
        if constexpr (SUM) {
            acc.x += cs[NV + 1];
            acc.y += cs[NV + 1];
        }
        double2 vq[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) vq[q] = reinterpret_cast<const double2 *>(V + (size_t)q * ldv)[t];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            acc.x += cs[q] * vq[q].x;
            acc.y += cs[q] * vq[q].y;
        }
        acc.x *= sc;
        acc.y *= sc;
        w2[t] = acc;
        nrm[0] += acc.x * acc.x + acc.y * acc.y;
    }
    block_sums<1>(nrm, sh, res);
    if (threadIdx.x == 0) partial[blockIdx.x] = res[0];
}

// The same projection and update for a float32 Krylov basis (V and w in
// float32, four per 16-byte load; every product and sum in float64).
template <int NV, bool SUM = false>
__global__ void __launch_bounds__(RED_THREADS)
k_multidot4f(const float *__restrict__ V, size_t ldv, int v0, const float *__restrict__ w, size_t n4,
             double *__restrict__ partial, int stride, int with_norm) {
    constexpr int NA = NV + 1 + (SUM ? 1 : 0);  // dots, ||w||^2 [, sum of w]
    __shared__ double sh[NA][RED_THREADS / 64];
    __shared__ double res[NA];
    const float4 *w4 = reinterpret_cast<const float4 *>(w);
    double acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = 0.0;
    for (size_t t = blockIdx.x * (size_t)RED_THREADS + threadIdx.x; t < n4; t += (size_t)gridDim.x * RED_THREADS) {
        const float4 wt = w4[t];
        float4 vq[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) vq[q] = reinterpret_cast<const float4 *>(V + (size_t)(v0 + q) * ldv)[t];
        const double a = wt.x, b = wt.y, c = wt.z, d = wt.w;
        acc[NV] += a * a + b * b + c * c + d * d;
        if constexpr (SUM) acc[NV + 1] += (a + b) + (c + d);
#pragma unroll
        for (int q = 0; q < NV; ++q)
            acc[q] += (double)vq[q].x * a + (double)vq[q].y * b + (double)vq[q].z * c + (double)vq[q].w * d;
    }
    block_sums<NA>(acc, sh, res);
    if ((int)threadIdx.x < NV) partial[(size_t)blockIdx.x * stride + v0 + threadIdx.x] = res[threadIdx.x];
    if (with_norm && threadIdx.x == NV) partial[(size_t)blockIdx.x * stride + NORM_SLOT] = res[NV];
    if (SUM && with_norm && (int)threadIdx.x == NV + 1) partial[(size_t)blockIdx.x * stride + SUM_SLOT] = res[NV + 1];
}

template <int NV, bool SUM = false>
__global__ void __launch_bounds__(RED_THREADS)
k_orth_update4f(float *__restrict__ w, const float *__restrict__ V, size_t ldv, const double *__restrict__ hc,
                size_t n4, double *__restrict__ partial, double *__restrict__ beta_out) {
    __shared__ double sh[1][RED_THREADS / 64];
    __shared__ double cs[NV + 2];
    __shared__ double res[1];
    if (threadIdx.x == 0) {
        double h2 = 0.0;
        for (int q = 0; q < NV; ++q) h2 += hc[q] * hc[q];
        double mu = 0.0;
        if constexpr (SUM) {  // the mean of w goes too (see k_orth_update2)
            mu = hc[HC_SUM] / (4.0 * (double)n4);
            h2 += mu * hc[HC_SUM];
        }
        const double w2n = hc[NORM_SLOT], b2 = w2n - h2;
        const double beta = (b2 > 1e-20 * w2n) ? sqrt(b2) : 1.0;
        cs[NV] = 1.0 / beta;
        cs[NV + 1] = -mu;
        if (blockIdx.x == 0) *beta_out = beta;
    }
    if ((int)threadIdx.x < NV) cs[threadIdx.x] = -hc[threadIdx.x];
    __syncthreads();
    const double sc = cs[NV];
    float4 *w4 = reinterpret_cast<float4 *>(w);
    double nrm[1] = {0.0};
    for (size_t t = blockIdx.x * (size_t)RED_THREADS + threadIdx.x; t < n4; t += (size_t)gridDim.x * RED_THREADS) {
        const float4 wv = w4[t];
        double a = wv.x, b = wv.y, c = wv.z, d = wv.w;
        if constexpr (SUM) {
            a += cs[NV + 1];
            b += cs[NV + 1];
            c += cs[NV + 1];
            d += cs[NV + 1];
        }
        float4 vq[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) vq[q] = reinterpret_cast<const float4 *>(V + (size_t)q * ldv)[t];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            a += cs[q] * (double)vq[q].x;
            b += cs[q] * (double)vq[q].y;
            c += cs[q] * (double)vq[q].z;
            d += cs[q] * (double)vq[q].w;
        }
        const float4 o = make_float4((float)(a * sc), (float)(b * sc), (float)(c * sc), (float)(d * sc));
        w4[t] = o;
        nrm[0] += (double)o.x * o.x + (double)o.y * o.y + (double)o.z * o.z + (double)o.w * o.w;
    }
    block_sums<1>(nrm, sh, res);
    if (threadIdx.x == 0) partial[blockIdx.x] = res[0];
}

// The projection and update for a float16 Krylov basis: V in float16 (eight
// per 16-byte load), the new vector w = A z in float32.  The products and a
// thread's sums are float32 (a float16 value times a float32 one rounds at
// 2^-24 relative, far below the basis' own 2^-11; ||w||^2 is float64), the
// block and grid sums float64.  The update writes the normalised vector into
// the basis only: the preconditioner reads it from there.
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef float f8 __attribute__((ext_vector_type(8)));

// The float16 basis is orthonormal only to float16 rounding, so the update
// divides by the exact norm of w - V h through the basis' Gram matrix,
// ||w||^2 - 2 h.h + h^T G h (h = V^T w), and its vector comes out unit to
// float32 rounding: no rescaling pass.  G_qr = V_q . V_r of the stored values;
// row q (r <= q) is summed by the projection pass of step q, which reads
// V_0..V_q anyway, into Hessenberg column q (hd0 + q hstride) at GRAM_SLOT + r.
__device__ __forceinline__ double gram(const double *__restrict__ hd0, int hstride, int q, int r) {
    return q >= r ? hd0[(size_t)q * hstride + GRAM_SLOT + r] : hd0[(size_t)r * hstride + GRAM_SLOT + q];
}

// With gram_row, also the products of the last vector V_{v0+NV-1} with each
// V_{v0+q} (its Gram row; products of float16 values, exact in float32 and
// summed in float32 per thread) into partial[b stride + GRAM_SLOT + q].
template <int NV>
__global__ void __launch_bounds__(RED_THREADS)
k_multidot8h(const _Float16 *__restrict__ V, size_t ldv, int v0, const float *__restrict__ w, size_t n8,
             double *__restrict__ partial, int stride, int with_norm, int gram_row) {
    constexpr int NA = NV + 1;  // dots, ||w||^2 (then the Gram row)
    __shared__ double sh[NA][RED_THREADS / 64];
    __shared__ double res[NA];
    const f8 *w8 = reinterpret_cast<const f8 *>(w);
    // per thread: the dots and the Gram row in float32, ||w||^2 in float64
    double wn = 0.0;
    float acc[NV], gacc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = gacc[q] = 0.0f;
    for (size_t t = blockIdx.x * (size_t)RED_THREADS + threadIdx.x; t < n8; t += (size_t)gridDim.x * RED_THREADS) {
        const f8 wt = w8[t];
        h8 vq[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) vq[q] = reinterpret_cast<const h8 *>(V + (size_t)(v0 + q) * ldv)[t];
        double wd[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) wd[e] = wt[e];
        wn += ((wd[0] * wd[0] + wd[1] * wd[1]) + (wd[2] * wd[2] + wd[3] * wd[3])) +
              ((wd[4] * wd[4] + wd[5] * wd[5]) + (wd[6] * wd[6] + wd[7] * wd[7]));
#pragma unroll
        for (int q = 0; q < NV; ++q) {
#pragma unroll
            for (int e = 0; e < 8; ++e) acc[q] = __builtin_fmaf((float)vq[q][e], wt[e], acc[q]);
        }
        if (gram_row) {
#pragma unroll
            for (int q = 0; q < NV; ++q)
#pragma unroll
                for (int e = 0; e < 8; e += 2)
                    gacc[q] = __builtin_amdgcn_fdot2(h2{vq[q][e], vq[q][e + 1]}, h2{vq[NV - 1][e], vq[NV - 1][e + 1]},
                                                     gacc[q], false);
        }
    }
    double a[NV + 1];
#pragma unroll
    for (int q = 0; q < NV; ++q) a[q] = (double)acc[q];
    a[NV] = wn;
    block_sums<NV + 1>(a, sh, res);
    if ((int)threadIdx.x < NV) partial[(size_t)blockIdx.x * stride + v0 + threadIdx.x] = res[threadIdx.x];
    if (with_norm && threadIdx.x == NV) partial[(size_t)blockIdx.x * stride + NORM_SLOT] = res[NV];
    if (gram_row) {
        double g[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) g[q] = (double)gacc[q];
        __syncthreads();  // sh is reused
        block_sums<NV>(g, sh, res);
        if ((int)threadIdx.x < NV) partial[(size_t)blockIdx.x * stride + GRAM_SLOT + threadIdx.x] = res[threadIdx.x];
    }
}


// The update on a float16 basis with the exact divisor (see gram); block 0
// also sets the column's squared-norm slot to 1, the vector being unit.
template <int NV>
__global__ void __launch_bounds__(RED_THREADS)
k_orth_update8h(const float *__restrict__ w, _Float16 *__restrict__ vn, const _Float16 *__restrict__ V, size_t ldv,
                double *__restrict__ hc, const double *__restrict__ hd0, int hstride, size_t n8,
                double *__restrict__ beta_out) {
    __shared__ double cs[NV + 1];
    if (threadIdx.x == 0) {
        double h2 = 0.0, hgh = 0.0;
        for (int q = 0; q < NV; ++q) {
            h2 += hc[q] * hc[q];
            double row = 0.0;
            for (int r = 0; r < NV; ++r) row += gram(hd0, hstride, q, r) * hc[r];
            hgh += hc[q] * row;
        }
        const double w2n = hc[NORM_SLOT], b2 = w2n - 2.0 * h2 + hgh;
        const double beta = (b2 > 1e-20 * w2n) ? sqrt(b2) : 1.0;
        cs[NV] = 1.0 / beta;
        if (blockIdx.x == 0) {
            *beta_out = beta;
            hc[65] = 1.0;
        }
    }
    if ((int)threadIdx.x < NV) cs[threadIdx.x] = -hc[threadIdx.x];
    __syncthreads();
    const double sc = cs[NV];
    float csf[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) csf[q] = (float)cs[q];
    const f8 *w8 = reinterpret_cast<const f8 *>(w);
    h8 *vn8 = reinterpret_cast<h8 *>(vn);
    for (size_t t = blockIdx.x * (size_t)RED_THREADS + threadIdx.x; t < n8; t += (size_t)gridDim.x * RED_THREADS) {
        const f8 wv = w8[t];
        h8 vq[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) vq[q] = reinterpret_cast<const h8 *>(V + (size_t)q * ldv)[t];
        // the projection sum_q h_q V_q per point in float32, subtracted from w in float64
        float pr[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) pr[e] = 0.0f;
#pragma unroll
        for (int q = 0; q < NV; ++q)
#pragma unroll
            for (int e = 0; e < 8; ++e) pr[e] = __builtin_fmaf(csf[q], (float)vq[q][e], pr[e]);
        h8 oh;
#pragma unroll
        for (int e = 0; e < 8; ++e) oh[e] = (_Float16)(float)(((double)wv[e] + (double)pr[e]) * sc);
        vn8[t] = oh;
    }
}

// xh = r / sqrt(*den_sq) rounded to float32 and on to float16 (0 when
// *den_sq is 0), and the float32 value into x32 unless it is null
__global__ void k_scale_to_fh(float *__restrict__ x32, _Float16 *__restrict__ xh, const double *__restrict__ r,
                              const double *__restrict__ den_sq, size_t n) {
    const double s = *den_sq > 0.0 ? 1.0 / sqrt(*den_sq) : 0.0;
    for (size_t t = blockIdx.x * (size_t)RED_THREADS + threadIdx.x; t < n; t += (size_t)gridDim.x * RED_THREADS) {
        const float y = (float)(r[t] * s);
        if (x32) x32[t] = y;
        xh[t] = (_Float16)y;
    }
}

__global__ void __launch_bounds__(RED_THREADS)
k_rescale_if_f(float *__restrict__ x, const double *__restrict__ partial, int nparts, double *__restrict__ nu2,
               size_t n) {
    __shared__ double sh[RED_THREADS / 64];
    __shared__ double tot;
    double v = 0.0;
    for (int b = threadIdx.x; b < nparts; b += RED_THREADS) v += partial[b];
    const double r = block_sum(v, sh);
    if (threadIdx.x == 0) {
        tot = r;
        if (blockIdx.x == 0) *nu2 = r;
    }
    __syncthreads();
    // float32 storage leaves |nu - 1| near 1e-7 even when beta is exact, so
    // the stored vector is taken as it is unless it is off by more than 1e-6
    const double nu = sqrt(tot);
    if (nu == 0.0 || fabs(nu - 1.0) <= RESCALE_TOL_F32) return;
    const double s = 1.0 / nu;
    for (size_t t = blockIdx.x * (size_t)RED_THREADS + threadIdx.x; t < n; t += (size_t)gridDim.x * RED_THREADS)
        x[t] = (float)((double)x[t] * s);
}

// x32 = r / sqrt(*den_sq) rounded to float32 (0 when *den_sq is 0)
__global__ void k_scale_to_f(float *__restrict__ x32, const double *__restrict__ r, const double *__restrict__ den_sq,
                             size_t n) {
    const double s = *den_sq > 0.0 ? 1.0 / sqrt(*den_sq) : 0.0;
    for (size_t t = blockIdx.x * (size_t)RED_THREADS + threadIdx.x; t < n; t += (size_t)gridDim.x * RED_THREADS)
        x32[t] = (float)(r[t] * s);
}

// nu^2 = sum of the nparts block partials (every block adds them in the same
// fixed order, so all agree bitwise; block 0 stores it at *nu2); then
// x <- x / nu unless nu is 0 or within 1e-8 of 1.
__global__ void __launch_bounds__(RED_THREADS)
k_rescale_if(double *__restrict__ x, const double *__restrict__ partial, int nparts, double *__restrict__ nu2,
             size_t n) {
    __shared__ double sh[RED_THREADS / 64];
    __shared__ double tot;
    double v = 0.0;
    for (int b = threadIdx.x; b < nparts; b += RED_THREADS) v += partial[b];
    const double r = block_sum(v, sh);
    if (threadIdx.x == 0) {
        tot = r;
        if (blockIdx.x == 0) *nu2 = r;
    }
    __syncthreads();
    const double nu = sqrt(tot);
    if (nu == 0.0 || fabs(nu - 1.0) <= 1e-8) return;
    const double s = 1.0 / nu;
    for (size_t t = blockIdx.x * (size_t)RED_THREADS + threadIdx.x; t < n; t += (size_t)gridDim.x * RED_THREADS)
        x[t] *= s;
}

// Pair-vectorised w += sign * sum_q c[q] V_q (no norm).
template <int NV>
__global__ void __launch_bounds__(RED_THREADS)
k_axpy2(double *__restrict__ w, const double *__restrict__ V, size_t ldv, const double *__restrict__ c, size_t n2,
        double sign) {
    __shared__ double cs[NV];
    if ((int)threadIdx.x < NV) cs[threadIdx.x] = sign * c[threadIdx.x];
    __syncthreads();
    double2 *w2 = reinterpret_cast<double2 *>(w);
    for (size_t t = blockIdx.x * (size_t)RED_THREADS + threadIdx.x; t < n2; t += (size_t)gridDim.x * RED_THREADS) {
        double2 acc = w2[t];
        double2 vq[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) vq[q] = reinterpret_cast<const double2 *>(V + (size_t)q * ldv)[t];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            acc.x += cs[q] * vq[q].x;
            acc.y += cs[q] * vq[q].y;
        }
        w2[t] = acc;
    }
}

// x += sum_q c[q] Z_q with float32 Z_q: four points per thread (16-byte loads
// of Z, two 16-byte loads and stores of x), float64 sums.
template <int NV>
__global__ void __launch_bounds__(RED_THREADS)
k_axpy4f(double *__restrict__ x, const float *__restrict__ Z, size_t ldz, const double *__restrict__ c, size_t n4) {
    __shared__ double cs[NV];
    if ((int)threadIdx.x < NV) cs[threadIdx.x] = c[threadIdx.x];
    __syncthreads();
    double2 *x2 = reinterpret_cast<double2 *>(x);
    for (size_t t = blockIdx.x * (size_t)RED_THREADS + threadIdx.x; t < n4; t += (size_t)gridDim.x * RED_THREADS) {
        double2 a = x2[2 * t], b = x2[2 * t + 1];
        float4 zq[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) zq[q] = reinterpret_cast<const float4 *>(Z + (size_t)q * ldz)[t];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            a.x += cs[q] * (double)zq[q].x;
            a.y += cs[q] * (double)zq[q].y;
            b.x += cs[q] * (double)zq[q].z;
            b.y += cs[q] * (double)zq[q].w;
        }
        x2[2 * t] = a;
        x2[2 * t + 1] = b;
    }
}

// out[idx] = sum_b partial[b * stride + idx], one block per idx, fixed order;
// with norm_out, one more block adds column NORM_SLOT into *norm_out; the
// last ngram blocks add columns GRAM_SLOT + q into gram_out[q]
__global__ void __launch_bounds__(RED_THREADS)
k_reduce_partials(const double *__restrict__ partial, int nblocks, int stride, double *__restrict__ out,
                  int nout, double *__restrict__ norm_out, double *__restrict__ sum_out = nullptr,
                  double *__restrict__ gram_out = nullptr, int ngram = 0) {
    __shared__ double sh[RED_THREADS / 64];
    const int b0 = (int)blockIdx.x, g0 = (int)gridDim.x - ngram;
    const int idx = b0 >= g0 ? GRAM_SLOT + b0 - g0 : (b0 < nout ? b0 : (b0 == nout ? NORM_SLOT : SUM_SLOT));
    double v = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += RED_THREADS) v += partial[(size_t)b * stride + idx];
    const double r = block_sum(v, sh);
    if (threadIdx.x == 0) {
        if (b0 >= g0) gram_out[b0 - g0] = r;
        else if (b0 < nout) out[idx] = r;
        else if (b0 == nout) *norm_out = r;
        else *sum_out = r;
    }
}

__global__ void __launch_bounds__(RED_THREADS)
k_sum(const double *__restrict__ x, size_t n, double *__restrict__ partial) {
    __shared__ double sh[RED_THREADS / 64];
    double acc = 0.0;
    for (size_t t = blockIdx.x * (size_t)RED_THREADS + threadIdx.x; t < n; t += (size_t)gridDim.x * RED_THREADS)
        acc += x[t];
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// w += sign * sum_q c[q] V_q ; optionally partial[blockIdx] = sum w_new^2
__global__ void __launch_bounds__(RED_THREADS)
k_axpy_multi(double *__restrict__ w, const double *__restrict__ V, size_t ldv, int nv,
             const double *__restrict__ c, size_t n, double sign, double *__restrict__ partial) {
    __shared__ double sh[RED_THREADS / 64];
    __shared__ double cs[64];
    for (int q = threadIdx.x; q < nv && q < 64; q += RED_THREADS) cs[q] = sign * c[q];
    __syncthreads();
    double nrm = 0.0;
    for (size_t t = blockIdx.x * (size_t)RED_THREADS + threadIdx.x; t < n; t += (size_t)gridDim.x * RED_THREADS) {
        double acc = w[t];
        for (int q = 0; q < nv; ++q) acc += cs[q] * V[(size_t)q * ldv + t];
        w[t] = acc;
        nrm += acc * acc;
    }
    if (partial) {
        const double r = block_sum(nrm, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = r;
    }
}

// Energy sums with two-sum accumulation: [0] sum rho phi, [1] sum over the
// three forward faces of every node of eps_f (D_f phi)^2.
__global__ void __launch_bounds__(RED_THREADS)
k_energy(const double *__restrict__ rho, const double *__restrict__ phi, const double *__restrict__ eps,
         int nx, int ny, int nz, double cx, double cy, double cz, double *__restrict__ partial) {
    __shared__ double shs[2][RED_THREADS / 64], shc[2][RED_THREADS / 64];
    DD a{0.0, 0.0}, f{0.0, 0.0};
    const size_t plane = (size_t)nx * ny, n = plane * nz;
    for (size_t t = blockIdx.x * (size_t)RED_THREADS + threadIdx.x; t < n; t += (size_t)gridDim.x * RED_THREADS) {
        const int i = (int)(t % nx);
        const int j = (int)((t / nx) % ny);
        const int k = (int)(t / plane);
        const double p0 = phi[t], e0 = eps[t];
        a = dd_add(a, rho[t] * p0);
        const size_t xp = t - i + (i + 1 == nx ? 0 : i + 1);
        const size_t yp = t + (size_t)((j + 1 == ny ? 0 : j + 1) - j) * nx;
        const size_t zp = t + (size_t)((k + 1 == nz ? 0 : k + 1) - k) * plane;
        const double dx = phi[xp] - p0, dy = phi[yp] - p0, dz = phi[zp] - p0;
        const double fx = 0.5 * (e0 + eps[xp]) * dx * dx * cx;
        const double fy = 0.5 * (e0 + eps[yp]) * dy * dy * cy;
        const double fz = 0.5 * (e0 + eps[zp]) * dz * dz * cz;
        f = dd_add(dd_add(dd_add(f, fx), fy), fz);
    }
    a = wave_dd(a);
    f = wave_dd(f);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        shs[0][wid] = a.s; shc[0][wid] = a.c;
        shs[1][wid] = f.s; shc[1][wid] = f.c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        DD ra{0.0, 0.0}, rf{0.0, 0.0};
        for (int q = 0; q < RED_THREADS / 64; ++q) {
            ra = dd_merge(ra, DD{shs[0][q], shc[0][q]});
            rf = dd_merge(rf, DD{shs[1][q], shc[1][q]});
        }
        partial[(size_t)blockIdx.x * 4 + 0] = ra.s;
        partial[(size_t)blockIdx.x * 4 + 1] = ra.c;
        partial[(size_t)blockIdx.x * 4 + 2] = rf.s;
        partial[(size_t)blockIdx.x * 4 + 3] = rf.c;
    }
}

__global__ void __launch_bounds__(64)
k_energy_final(const double *__restrict__ partial, int nblocks, double *__restrict__ out) {
    // one wave; lane q merges blocks q, q + 64, ... then a fixed shuffle tree
    DD a{0.0, 0.0}, f{0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += 64) {
        a = dd_merge(a, DD{partial[(size_t)b * 4 + 0], partial[(size_t)b * 4 + 1]});
        f = dd_merge(f, DD{partial[(size_t)b * 4 + 2], partial[(size_t)b * 4 + 3]});
    }
    a = wave_dd(a);
    f = wave_dd(f);
    if (threadIdx.x == 0) {
        out[0] = a.s + a.c;
        out[1] = f.s + f.c;
    }
}

}  // namespace

constexpr int MD2_GROUP = 16;  // dot products per pass of the pair-vectorised multidot

bool pair_ok(const void *a, size_t ldv, size_t n) {
    return n % 2 == 0 && ldv % 2 == 0 && (reinterpret_cast<uintptr_t>(a) & 15) == 0;
}

#define DWP_NV_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

// With the sum of w as well (into *sum_out), for the mean-free Arnoldi step:
// 16-byte-aligned vectors and at most MD2_GROUP vectors only.
void launch_multidot_sum(hipStream_t s, const double *V, size_t ldv, int nv, const double *w, size_t n,
                         double *partial, double *out, double *norm_out, double *sum_out) {
    if (nv < 1 || nv > MD2_GROUP || !pair_ok(V, ldv, n) || !pair_ok(w, 0, n))
        fail(DWP_EINVAL, "internal: mean-free multidot layout");
    switch (nv) {
#define DWP_MDS_CASE(K)                                                                                      \
    case K:                                                                                                  \
        k_multidot2<K, true><<<RED_BLOCKS, RED_THREADS, 0, s>>>(V, ldv, 0, w, n / 2, partial, MD_STRIDE, 1); \
        break;
        DWP_NV_CASES(DWP_MDS_CASE)
#undef DWP_MDS_CASE
    }
    DWP_LAUNCH_CHECK();
    k_reduce_partials<<<nv + 2, RED_THREADS, 0, s>>>(partial, RED_BLOCKS, MD_STRIDE, out, nv, norm_out, sum_out);
    DWP_LAUNCH_CHECK();
}

void launch_multidot(hipStream_t s, const double *V, size_t ldv, int nv, const double *w, size_t n,
                     double *partial, double *out, double *norm_out) {
    if (nv > 64) fail(DWP_EINVAL, "multidot: at most 64 vectors");
    if (pair_ok(V, ldv, n) && pair_ok(w, 0, n)) {
        for (int v0 = 0; v0 < nv; v0 += MD2_GROUP) {
            const int g = nv - v0 < MD2_GROUP ? nv - v0 : MD2_GROUP;
            const int wn = (v0 == 0 && norm_out) ? 1 : 0;
            switch (g) {
#define DWP_MD_CASE(K)                                                                                       \
    case K:                                                                                                  \
        k_multidot2<K><<<RED_BLOCKS, RED_THREADS, 0, s>>>(V, ldv, v0, w, n / 2, partial, MD_STRIDE, wn);     \
        break;
                DWP_NV_CASES(DWP_MD_CASE)
#undef DWP_MD_CASE
            }
            DWP_LAUNCH_CHECK();
        }
    } else {
        for (int v0 = 0; v0 < nv; v0 += MD_GROUP) {
            const int g = nv - v0 < MD_GROUP ? nv - v0 : MD_GROUP;
            k_multidot<<<RED_BLOCKS, RED_THREADS, 0, s>>>(V, ldv, v0, g, w, n, partial, MD_STRIDE,
                                                          (v0 == 0 && norm_out) ? 1 : 0);
            DWP_LAUNCH_CHECK();
        }
    }
    k_reduce_partials<<<nv + (norm_out ? 1 : 0), RED_THREADS, 0, s>>>(partial, RED_BLOCKS, MD_STRIDE, out, nv,
                                                                     norm_out);
    DWP_LAUNCH_CHECK();
}

void launch_dot(hipStream_t s, const double *x, const double *y, size_t n, double *partial, double *out) {
    launch_multidot(s, x, n, 1, y, n, partial, out, nullptr);
}

void launch_sum(hipStream_t s, const double *x, size_t n, double *partial, double *out) {
    k_sum<<<RED_BLOCKS, RED_THREADS, 0, s>>>(x, n, partial);
    DWP_LAUNCH_CHECK();
    k_reduce_partials<<<1, RED_THREADS, 0, s>>>(partial, RED_BLOCKS, 1, out, 1, nullptr);
    DWP_LAUNCH_CHECK();
}

void launch_axpy_multi(hipStream_t s, double *w, const double *V, size_t ldv, int nv, const double *c, size_t n,
                       double sign, double *partial, double *norm_out) {
    if (nv > 64) fail(DWP_EINVAL, "axpy_multi: at most 64 vectors");
    if (!norm_out && nv <= 16 && pair_ok(V, ldv, n) && pair_ok(w, 0, n)) {
        switch (nv) {
#define DWP_AX_CASE(K)                                                                     \
    case K: k_axpy2<K><<<RED_BLOCKS, RED_THREADS, 0, s>>>(w, V, ldv, c, n / 2, sign); break;
            DWP_NV_CASES(DWP_AX_CASE)
#undef DWP_AX_CASE
        }
        DWP_LAUNCH_CHECK();
        return;
    }
    k_axpy_multi<<<RED_BLOCKS, RED_THREADS, 0, s>>>(w, V, ldv, nv, c, n, sign, norm_out ? partial : nullptr);
    DWP_LAUNCH_CHECK();
    if (norm_out) {
        k_reduce_partials<<<1, RED_THREADS, 0, s>>>(partial, RED_BLOCKS, 1, norm_out, 1, nullptr);
        DWP_LAUNCH_CHECK();
    }
}

bool orth_update_supported(const double *V, size_t ldv, int nv, size_t n) {
    return nv >= 1 && nv <= 16 && pair_ok(V, ldv, n);
}

// w <- (w - sum_q hc[q] V_q) / beta (see k_orth_update2); hc[65] receives the
// squared norm of the result and hc[66] the divisor beta; the result is then
// rescaled to unit norm unless that norm is 0 or within 1e-8 of 1.
void launch_orth_update(hipStream_t s, double *w, const double *V, size_t ldv, int nv, double *hc, size_t n,
                        double *partial, bool mean_free) {
    if (!orth_update_supported(V, ldv, nv, n) || !pair_ok(w, 0, n)) fail(DWP_EINVAL, "internal: orth update layout");
    if (mean_free) {
        switch (nv) {
#define DWP_OUS_CASE(K)                                                                                         \
    case K: k_orth_update2<K, true><<<RED_BLOCKS, RED_THREADS, 0, s>>>(w, V, ldv, hc, n / 2, partial, hc + 66); \
        break;
            DWP_NV_CASES(DWP_OUS_CASE)
#undef DWP_OUS_CASE
        }
    } else {
        switch (nv) {
#define DWP_OU_CASE(K)                                                                                     \
    case K: k_orth_update2<K><<<RED_BLOCKS, RED_THREADS, 0, s>>>(w, V, ldv, hc, n / 2, partial, hc + 66); break;
            DWP_NV_CASES(DWP_OU_CASE)
#undef DWP_OU_CASE
        }
    }
    DWP_LAUNCH_CHECK();
    k_rescale_if<<<RED_BLOCKS, RED_THREADS, 0, s>>>(w, partial, RED_BLOCKS, hc + 65, n);
    DWP_LAUNCH_CHECK();
}

static bool quad_ok(const void *a, size_t ldv, size_t n) {
    return n % 4 == 0 && ldv % 4 == 0 && (reinterpret_cast<uintptr_t>(a) & 15) == 0;
}

bool krylov32_supported(const float *V, size_t ldv, size_t n) { return quad_ok(V, ldv, n); }

void launch_axpy_multi32(hipStream_t s, double *x, const float *Z, size_t ldz, int nv, const double *c, size_t n) {
    if (nv < 1 || nv > 16 || !quad_ok(Z, ldz, n) || !quad_ok(x, 0, n)) fail(DWP_EINVAL, "internal: float32 axpy layout");
    switch (nv) {
#define DWP_AX4_CASE(K)                                                                     \
    case K: k_axpy4f<K><<<RED_BLOCKS, RED_THREADS, 0, s>>>(x, Z, ldz, c, n / 4); break;
        DWP_NV_CASES(DWP_AX4_CASE)
#undef DWP_AX4_CASE
    }
    DWP_LAUNCH_CHECK();
}

void launch_multidot32(hipStream_t s, const float *V, size_t ldv, int nv, const float *w, size_t n, double *partial,
                       double *out, double *norm_out) {
    if (nv > 64 || !quad_ok(V, ldv, n) || !quad_ok(w, 0, n)) fail(DWP_EINVAL, "internal: float32 multidot layout");
    for (int v0 = 0; v0 < nv; v0 += MD2_GROUP) {
        const int g = nv - v0 < MD2_GROUP ? nv - v0 : MD2_GROUP;
        const int wn = (v0 == 0 && norm_out) ? 1 : 0;
        switch (g) {
#define DWP_MD4_CASE(K)                                                                                      \
    case K:                                                                                                  \
        k_multidot4f<K><<<RED_BLOCKS, RED_THREADS, 0, s>>>(V, ldv, v0, w, n / 4, partial, MD_STRIDE, wn);    \
        break;
            DWP_NV_CASES(DWP_MD4_CASE)
#undef DWP_MD4_CASE
        }
        DWP_LAUNCH_CHECK();
    }
    k_reduce_partials<<<nv + (norm_out ? 1 : 0), RED_THREADS, 0, s>>>(partial, RED_BLOCKS, MD_STRIDE, out, nv,
                                                                     norm_out);
    DWP_LAUNCH_CHECK();
}

void launch_multidot32_sum(hipStream_t s, const float *V, size_t ldv, int nv, const float *w, size_t n,
                           double *partial, double *out, double *norm_out, double *sum_out) {
    if (nv < 1 || nv > MD2_GROUP || !quad_ok(V, ldv, n) || !quad_ok(w, 0, n))
        fail(DWP_EINVAL, "internal: float32 mean-free multidot layout");
    switch (nv) {
#define DWP_MD4S_CASE(K)                                                                                       \
    case K:                                                                                                    \
        k_multidot4f<K, true><<<RED_BLOCKS, RED_THREADS, 0, s>>>(V, ldv, 0, w, n / 4, partial, MD_STRIDE, 1);  \
        break;
        DWP_NV_CASES(DWP_MD4S_CASE)
#undef DWP_MD4S_CASE
    }
    DWP_LAUNCH_CHECK();
    k_reduce_partials<<<nv + 2, RED_THREADS, 0, s>>>(partial, RED_BLOCKS, MD_STRIDE, out, nv, norm_out, sum_out);
    DWP_LAUNCH_CHECK();
}

void launch_orth_update32(hipStream_t s, float *w, const float *V, size_t ldv, int nv, double *hc, size_t n,
                          double *partial, bool mean_free) {
    if (nv < 1 || nv > 16 || !quad_ok(V, ldv, n) || !quad_ok(w, 0, n))
        fail(DWP_EINVAL, "internal: float32 orth update layout");
    if (mean_free) {
        switch (nv) {
#define DWP_OU4S_CASE(K)                                                                                           \
    case K: k_orth_update4f<K, true><<<RED_BLOCKS, RED_THREADS, 0, s>>>(w, V, ldv, hc, n / 4, partial, hc + 66); \
        break;
            DWP_NV_CASES(DWP_OU4S_CASE)
#undef DWP_OU4S_CASE
        }
    } else {
        switch (nv) {
#define DWP_OU4_CASE(K)                                                                                     \
    case K: k_orth_update4f<K><<<RED_BLOCKS, RED_THREADS, 0, s>>>(w, V, ldv, hc, n / 4, partial, hc + 66); break;
            DWP_NV_CASES(DWP_OU4_CASE)
#undef DWP_OU4_CASE
        }
    }
    DWP_LAUNCH_CHECK();
    k_rescale_if_f<<<RED_BLOCKS, RED_THREADS, 0, s>>>(w, partial, RED_BLOCKS, hc + 65, n);
    DWP_LAUNCH_CHECK();
}

static bool oct_ok(const void *a, size_t ldv, size_t n) {
    return n % 8 == 0 && ldv % 8 == 0 && (reinterpret_cast<uintptr_t>(a) & 15) == 0;
}

bool krylov16_supported(const void *V, size_t ldv, size_t n) { return oct_ok(V, ldv, n); }

void launch_multidot16(hipStream_t s, const _Float16 *V, size_t ldv, int nv, const float *w, size_t n,
                       double *partial, double *out, double *norm_out, double *gram_out) {
    if (nv < 1 || nv > MD2_GROUP || !oct_ok(V, ldv, n) || !oct_ok(w, 0, n) || GRAM_SLOT + nv > NORM_SLOT)
        fail(DWP_EINVAL, "internal: float16 multidot layout");
    const int wn = norm_out ? 1 : 0, gr = gram_out ? 1 : 0;
    switch (nv) {
#define DWP_MD8_CASE(K)                                                                                         \
    case K:                                                                                                     \
        k_multidot8h<K><<<RED_BLOCKS, RED_THREADS, 0, s>>>(V, ldv, 0, w, n / 8, partial, MD_STRIDE, wn, gr);    \
        break;
        DWP_NV_CASES(DWP_MD8_CASE)
#undef DWP_MD8_CASE
    }
    DWP_LAUNCH_CHECK();
    const int ng = gram_out ? nv : 0;
    k_reduce_partials<<<nv + (norm_out ? 1 : 0) + ng, RED_THREADS, 0, s>>>(partial, RED_BLOCKS, MD_STRIDE, out, nv,
                                                                          norm_out, nullptr, gram_out, ng);
    DWP_LAUNCH_CHECK();
}

void launch_orth_update16(hipStream_t s, const float *w, _Float16 *vn, const _Float16 *V, size_t ldv, int nv,
                          double *hc, const double *hd0, int hstride, size_t n) {
    if (nv < 1 || nv > 16 || !oct_ok(V, ldv, n) || !oct_ok(vn, 0, n) || !oct_ok(w, 0, n) ||
        GRAM_SLOT + nv > NORM_SLOT || hstride < NORM_SLOT + 3)
        fail(DWP_EINVAL, "internal: float16 orth update layout");
    switch (nv) {
#define DWP_OU8_CASE(K)                                                                                         \
    case K:                                                                                                     \
        k_orth_update8h<K><<<RED_BLOCKS, RED_THREADS, 0, s>>>(w, vn, V, ldv, hc, hd0, hstride, n / 8, hc + 66); \
        break;
        DWP_NV_CASES(DWP_OU8_CASE)
#undef DWP_OU8_CASE
    }
    DWP_LAUNCH_CHECK();
}

void launch_scale_to16(hipStream_t s, float *x32, _Float16 *xh, const double *r, const double *den_sq, size_t n) {
    k_scale_to_fh<<<RED_BLOCKS, RED_THREADS, 0, s>>>(x32, xh, r, den_sq, n);
    DWP_LAUNCH_CHECK();
}

__global__ void __launch_bounds__(RED_THREADS) k_sum_f(const float *__restrict__ x, size_t n, double *partial) {
    __shared__ double sh[RED_THREADS / 64];
    double v = 0.0;
    for (size_t t = blockIdx.x * (size_t)RED_THREADS + threadIdx.x; t < n; t += (size_t)gridDim.x * RED_THREADS)
        v += (double)x[t];
    const double r = block_sum(v, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}
__global__ void k_sub_mean_f(float *x, const double *sum, double inv_n, size_t n) {
    const double m = *sum * inv_n;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        x[t] = (float)((double)x[t] - m);
}
void launch_sub_mean32(hipStream_t s, float *x, size_t n, double *partial, double *sum_out) {
    k_sum_f<<<RED_BLOCKS, RED_THREADS, 0, s>>>(x, n, partial);
    DWP_LAUNCH_CHECK();
    k_reduce_partials<<<1, RED_THREADS, 0, s>>>(partial, RED_BLOCKS, 1, sum_out, 1, nullptr);
    DWP_LAUNCH_CHECK();
    k_sub_mean_f<<<RED_BLOCKS, RED_THREADS, 0, s>>>(x, sum_out, 1.0 / (double)n, n);
    DWP_LAUNCH_CHECK();
}

void launch_scale_to32(hipStream_t s, float *x32, const double *r, const double *den_sq, size_t n) {
    k_scale_to_f<<<RED_BLOCKS, RED_THREADS, 0, s>>>(x32, r, den_sq, n);
    DWP_LAUNCH_CHECK();
}

void launch_energy(hipStream_t s, const Plan &p, const double *rho, const double *phi, const double *eps,
                   double *partial, double *out) {
    k_energy<<<RED_BLOCKS, RED_THREADS, 0, s>>>(rho, phi, eps, p.nx, p.ny, p.nz, 1.0 / (p.h[0] * p.h[0]),
                                                1.0 / (p.h[1] * p.h[1]), 1.0 / (p.h[2] * p.h[2]), partial);
    DWP_LAUNCH_CHECK();
    k_energy_final<<<1, 64, 0, s>>>(partial, RED_BLOCKS, out);
    DWP_LAUNCH_CHECK();
}

}  // namespace dwp
