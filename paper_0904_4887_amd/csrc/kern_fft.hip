// Periodic vacuum Poisson solve by a hand-written mixed-radix 3-D FFT.
//
// psi = L^{-1} r with L the 7-point vacuum Laplacian: in Fourier space
// psi~(m) = -r~(m) / lambda(m), lambda(m) = sum_d 4 sin^2(pi m_d / n_d) / h_d^2,
// psi~(0) = 0 -- the grid counterpart of the paper's Eq. 15, with the discrete
// symbol in place of G^2 so that the dry update inverts exactly the operator
// the wet multigrid discretises.
//
// Five passes over HBM, each a batch of 1-D transforms staged in LDS:
//   x  : two real rows packed as one complex row, forward, split (R2C)
//   y  : forward along y on tiles of consecutive kx
//   z  : forward along z, multiply by -1/(N lambda), inverse along z
//   y  : inverse
//   x  : inverse of two rows at once (C2R)
// Each 1-D transform is a Stockham autosort FFT with radix-8, -6, -4, -3 and -2
// stages; a stage reads its inputs into registers, synchronises, and writes
// its outputs back in place.  The spectrum and the transforms run in float64,
// or in float32 (S = float) for the mixed-precision variant; the real input
// and output grids are float64 either way.
#include "dwp_internal.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <type_traits>

namespace dwp {

namespace {

constexpr int FFT_THREADS = 512;
constexpr int FFT_MAXE = 4096;   // complex values per block (lines x length) at most
// Lines per block: B * n within the budget (see tile_log2), never above the
// per-block maximum, with the lines of a block within 64 KB of LDS (the n
// twiddles of the axis follow them, up to 64 KB more for n = 4096 in float64,
// where the kernel's LDS limit is raised).  The float32 x
// passes take 16 lines of 192 (measured: 0.5 ms per step less than 8).  A
// float32 z pass of 16 lines of 384 (a per-block maximum of 8192 for that
// kernel alone: 124 VGPRs, half the waves) measured 40 % slower than 8.
constexpr int FFT_BUDGET_X = 2048, FFT_BUDGET_X32 = 4096, FFT_BUDGET_Y = 4096;
// z pass: threads, lines x length per block (16 lines of 384 with 1024
// threads measured 10 % slower than 8 lines with 512)
constexpr int FFT_Z_THREADS = 512, FFT_Z_MAXE = 4096;
static_assert(FFT_Z_THREADS >= FFT_THREADS, "a radix-6 line fits every pass");
constexpr int MAX_STAGES = 12;

// Division by a small positive d through one multiply-high: with
// m = floor(2^32 / d) + 1, floor(i * m / 2^32) = floor(i / d) whenever
// i * d < 2^32, which holds for every index here (i, d < 2^16).  d = 1 is
// handled by the callers.
struct Div {
    unsigned m;
    int d;
};
Div make_div(int d) { return Div{d > 1 ? (unsigned)(0xFFFFFFFFu / (unsigned)d + 1u) : 0u, d}; }
__device__ __forceinline__ int udiv(int i, Div q) { return q.d == 1 ? i : (int)__umulhi((unsigned)i, q.m); }

// Radix plan of one axis with the per-stage constants: radix r, product p of
// the earlier radices (and its divider), and the twiddle stride n / (p r).
struct Radices {
    int n;
    int nst;
    int r[MAX_STAGES];
    int p[MAX_STAGES];
    unsigned pm[MAX_STAGES];
    int tstride[MAX_STAGES];
};

// Complex arithmetic on double2 / float2.
template <class S> struct CT;
template <> struct CT<double> { using T = double2; };
template <> struct CT<float> { using T = float2; };
template <class S> using cplx = typename CT<S>::T;
template <class C> __device__ __forceinline__ C mk(decltype(C::x) a, decltype(C::x) b) { C r; r.x = a; r.y = b; return r; }

template <class C> __device__ __forceinline__ C cmul(C a, C b) {
    return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <class C> __device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <class C> __device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
// multiply by -i (forward) or +i (inverse)
template <class C> __device__ __forceinline__ C rot(C a, bool inv) {
    return inv ? mk<C>(-a.y, a.x) : mk<C>(a.y, -a.x);
}

template <int R, class C> struct DFT;

template <class C> struct DFT<2, C> {
    static __device__ __forceinline__ void run(C *x, bool) {
        const C a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    }
};
template <class C> struct DFT<4, C> {
    static __device__ __forceinline__ void run(C *x, bool inv) {
        const C a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
        const C c = cadd(x[1], x[3]), d = csub(x[1], x[3]);
        x[0] = cadd(a, c);
        x[2] = csub(a, c);
        const C rd = rot(d, inv);  // -i d (forward)
        x[1] = cadd(b, rd);
        x[3] = csub(b, rd);
    }
};
template <class C> struct DFT<3, C> {
    static __device__ __forceinline__ void run(C *x, bool inv) {
        using S = decltype(C::x);
        // w = exp(-2 pi i / 3) = -1/2 - i sqrt(3)/2
        const S s3 = (S)0.86602540378443864676;
        const C t1 = cadd(x[1], x[2]);
        const C t2 = mk<C>(x[0].x - (S)0.5 * t1.x, x[0].y - (S)0.5 * t1.y);
        const C d = csub(x[1], x[2]);
        const C rd = rot(mk<C>(s3 * d.x, s3 * d.y), inv);  // -i s3 d (forward)
        x[0] = cadd(x[0], t1);
        x[1] = cadd(t2, rd);
        x[2] = csub(t2, rd);
    }
};
template <class C> struct DFT<6, C> {
    static __device__ __forceinline__ void run(C *x, bool inv) {
        using S = decltype(C::x);
        // two radix-3 transforms of the even and odd inputs, then one radix-2
        // layer with the sixth roots of unity w6^k = exp(-+i pi k / 3):
        // X[k] = E[k] + w6^k O[k], X[k + 3] = E[k] - w6^k O[k]
        C ev[3] = {x[0], x[2], x[4]}, od[3] = {x[1], x[3], x[5]};
        DFT<3, C>::run(ev, inv);
        DFT<3, C>::run(od, inv);
        const S h = (S)0.5, sg = inv ? (S)0.86602540378443864676 : (S)-0.86602540378443864676;
        const C t1 = mk<C>(h * od[1].x - sg * od[1].y, h * od[1].y + sg * od[1].x);    // w6 = 1/2 + i sg
        const C t2 = mk<C>(-h * od[2].x - sg * od[2].y, sg * od[2].x - h * od[2].y);   // w6^2 = -1/2 + i sg
        x[0] = cadd(ev[0], od[0]);
        x[3] = csub(ev[0], od[0]);
        x[1] = cadd(ev[1], t1);
        x[4] = csub(ev[1], t1);
        x[2] = cadd(ev[2], t2);
        x[5] = csub(ev[2], t2);
    }
};
template <class C> struct DFT<8, C> {
    static __device__ __forceinline__ void run(C *x, bool inv) {
        using S = decltype(C::x);
        // two radix-4 transforms of the even and odd inputs, then one radix-2
        // layer with the eighth roots of unity w8^k = exp(-+i pi k / 4)
        C ev[4] = {x[0], x[2], x[4], x[6]}, od[4] = {x[1], x[3], x[5], x[7]};
        DFT<4, C>::run(ev, inv);
        DFT<4, C>::run(od, inv);
        const S c = (S)0.70710678118654752440;
        const C t1 = inv ? mk<C>(c * (od[1].x - od[1].y), c * (od[1].x + od[1].y))
                         : mk<C>(c * (od[1].x + od[1].y), c * (od[1].y - od[1].x));
        const C t2 = rot(od[2], inv);
        const C t3 = inv ? mk<C>(-c * (od[3].x + od[3].y), c * (od[3].x - od[3].y))
                         : mk<C>(c * (od[3].y - od[3].x), -c * (od[3].x + od[3].y));
        x[0] = cadd(ev[0], od[0]);
        x[4] = csub(ev[0], od[0]);
        x[1] = cadd(ev[1], t1);
        x[5] = csub(ev[1], t1);
        x[2] = cadd(ev[2], t2);
        x[6] = csub(ev[2], t2);
        x[3] = cadd(ev[3], t3);
        x[7] = csub(ev[3], t3);
    }
};

// One Stockham stage of radix R on B = 2^lb lines of length n held in LDS;
// element t of line l sits at buf[l * ls + t * es].  p = product of the
// radices of the earlier stages.  Butterfly i of a line reads
// x_q = buf[i + q n/R], twiddles x_q by exp(-+2 pi i q (i mod p) / (p R)),
// and writes output r to (i - i mod p) R + i mod p + r p.
// IL: the lines are interleaved (es = B, ls = 1: element t of line l at
// t B + l), so that work item w = i B + l reads x_q at w + q T B and writes
// output r at ((i - k) R + k) B + l + r p B without per-element multiplies.
template <int R, class C, int MAXE, int NT, bool IL>
__device__ void stage(C *buf, int n, int p, unsigned pm, int tstride, int lb, int es, int ls,
                      const C *__restrict__ tw, bool inv) {
    // a block whose plan holds a radix-6 stage has at most 6 NT values (the
    // host's tile budget), so that the radix-6 stage is one butterfly per thread
    constexpr int E = R == 6 && MAXE > 6 * NT ? 6 * NT : MAXE;
    constexpr int K = (E / R + NT - 1) / NT;
    const int T = n / R;
    const int items = T << lb;
    const int bmask = (1 << lb) - 1;
    C x[K][R];
#pragma unroll
    for (int m = 0; m < K; ++m) {
        const int w = threadIdx.x + m * NT;
        if (w < items) {
            const int l = w & bmask, i = w >> lb;
#pragma unroll
            for (int q = 0; q < R; ++q) x[m][q] = IL ? buf[w + q * items] : buf[l * ls + (i + q * T) * es];
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < K; ++m) {
        const int w = threadIdx.x + m * NT;
        if (w < items) {
            const int l = w & bmask, i = w >> lb;
            const int k = p > 1 ? i - p * (int)__umulhi((unsigned)i, pm) : 0;
            if (p > 1) {
                const int kt = k * tstride;
#pragma unroll
                for (int q = 1; q < R; ++q) {
                    C t = tw[q * kt];
                    if (inv) t.y = -t.y;
                    x[m][q] = cmul(x[m][q], t);
                }
            }
            DFT<R, C>::run(x[m], inv);
            const int j = (i - k) * R + k;
            const int jb = (j << lb) + l, pb = p << lb;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (IL) buf[jb + r * pb] = x[m][r];
                else buf[l * ls + (j + r * p) * es] = x[m][r];
            }
        }
    }
    __syncthreads();
}

// R6: the plan may hold a radix-6 stage (a kernel built without it keeps the
// registers the radix-6 stage would need)
template <bool R6, bool IL, class C, int MAXE = FFT_MAXE, int NT = FFT_THREADS>
__device__ void fft_lines(C *buf, const Radices &rd, int lb, int es, int ls, const C *__restrict__ tw, bool inv) {
    for (int s = 0; s < rd.nst; ++s) {
        const int R = rd.r[s];
        if (R == 8) stage<8, C, MAXE, NT, IL>(buf, rd.n, rd.p[s], rd.pm[s], rd.tstride[s], lb, es, ls, tw, inv);
        else if (R6 && R == 6) stage<6, C, MAXE, NT, IL>(buf, rd.n, rd.p[s], rd.pm[s], rd.tstride[s], lb, es, ls, tw, inv);
        else if (R == 4) stage<4, C, MAXE, NT, IL>(buf, rd.n, rd.p[s], rd.pm[s], rd.tstride[s], lb, es, ls, tw, inv);
        else if (R == 3) stage<3, C, MAXE, NT, IL>(buf, rd.n, rd.p[s], rd.pm[s], rd.tstride[s], lb, es, ls, tw, inv);
        else stage<2, C, MAXE, NT, IL>(buf, rd.n, rd.p[s], rd.pm[s], rd.tstride[s], lb, es, ls, tw, inv);
    }
}

// A block's loads of n_el values from global memory: KL per thread issued
// together, then stored (ld(e) gives value e, st(e, v) puts it in LDS), so a
// thread waits once per KL values instead of once per value.  With ntw > 0
// the ntw twiddles tw_g[] come along into tw_l[] (LDS), so that the stages
// read them from LDS.
template <int KL, int NT, class V, class Ld, class St>
__device__ __forceinline__ void load_batched(int n_el, Ld ld, St st, const V *__restrict__ tw_g = nullptr,
                                             V *tw_l = nullptr, int ntw = 0) {
    const int tot = n_el + ntw;
    for (int e0 = 0; e0 < tot; e0 += KL * NT) {
        V v[KL];
#pragma unroll
        for (int m = 0; m < KL; ++m) {
            const int e = e0 + threadIdx.x + m * NT;
            if (e < n_el) v[m] = ld(e);
            else if (e < tot) v[m] = tw_g[e - n_el];
        }
#pragma unroll
        for (int m = 0; m < KL; ++m) {
            const int e = e0 + threadIdx.x + m * NT;
            if (e < n_el) st(e, v[m]);
            else if (e < tot) tw_l[e - n_el] = v[m];
        }
    }
}
constexpr int FFT_KL = FFT_MAXE / FFT_THREADS;  // one batch covers a block of the separate passes

// ---------------------------------------------------------------- x passes
// Rows are the nx-long x lines of the [nz][ny][nx] grid; B = 2^lb complex
// lines per block carry 2B real rows.  LDS lines are padded to n + 1 elements.
template <class S, class TI, bool R6>
__global__ void __launch_bounds__(FFT_THREADS)
k_fft_x_fwd(const TI *__restrict__ in, const double *__restrict__ sinv, cplx<S> *__restrict__ out,
            Radices rd, const cplx<S> *__restrict__ tw, int lb, int nrows, int nkx, int ldc, Div dn, Div dk, Div dn4,
            Div dk2) {
    using C = cplx<S>;
    typedef TI TI4 __attribute__((ext_vector_type(4)));
    extern __shared__ __align__(16) unsigned char lds_raw[];
    C *lds = reinterpret_cast<C *>(lds_raw);
    const int n = rd.n, ls = n + 1, B = 1 << lb;
    const int r0 = blockIdx.x * 2 * B;
    C *twl = lds + B * ls;
    if (!sinv && (n & 3) == 0) {
        // unscaled rows of a multiple of 4: four values of each row per load
        // (dn4 divides by n / 4)
        const int n4 = n >> 2;
        for (int e = threadIdx.x; e < n; e += FFT_THREADS) twl[e] = tw[e];
        constexpr int KV = (FFT_MAXE / 4 + FFT_THREADS - 1) / FFT_THREADS;
        for (int e0 = 0; e0 < B * n4; e0 += KV * FFT_THREADS) {
            TI4 va[KV], vb[KV];
#pragma unroll
            for (int m = 0; m < KV; ++m) {
                const int e = e0 + threadIdx.x + m * FFT_THREADS;
                if (e < B * n4) {
                    const int l = udiv(e, dn4), t4 = e - l * n4;
                    const int ra = r0 + 2 * l;
                    if (ra + 1 < nrows) {
                        const size_t ia = (size_t)ra * n + 4 * t4;
                        va[m] = *reinterpret_cast<const TI4 *>(in + ia);
                        vb[m] = *reinterpret_cast<const TI4 *>(in + ia + n);
                    } else {
                        va[m] = vb[m] = TI4(0);
                    }
                }
            }
#pragma unroll
            for (int m = 0; m < KV; ++m) {
                const int e = e0 + threadIdx.x + m * FFT_THREADS;
                if (e < B * n4) {
                    const int l = udiv(e, dn4), t4 = e - l * n4;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        lds[l * ls + 4 * t4 + q] = mk<C>((S)(double)va[m][q], (S)(double)vb[m][q]);
                }
            }
        }
    } else load_batched<FFT_KL, FFT_THREADS, C>(
        B * n,
        [&](int e) {
            const int l = udiv(e, dn), t = e - l * n;
            const int ra = r0 + 2 * l, rb = ra + 1;
            double a = 0.0, b = 0.0;
            if (rb < nrows) {
                const size_t ia = (size_t)ra * n + t, ib = ia + n;
                a = (double)in[ia];
                b = (double)in[ib];
                if (sinv) { a *= sinv[ia]; b *= sinv[ib]; }
            }
            return mk<C>((S)a, (S)b);
        },
        [&](int e, C v) {
            const int l = udiv(e, dn), t = e - l * n;
            lds[l * ls + t] = v;
        },
        tw, twl, n);
    __syncthreads();
    fft_lines<R6, false>(lds, rd, lb, 1, ls, twl, false);
    if constexpr (sizeof(S) == 4) {
        // two neighbouring kx per thread, stored as 16-byte pairs (ldc even)
        const int nk2 = (nkx + 1) >> 1;
        const S h = (S)0.5;
        for (int e = threadIdx.x; e < B * nk2; e += FFT_THREADS) {
            const int l = udiv(e, dk2), k = 2 * (e - l * nk2);
            const int ra = r0 + 2 * l, rb = ra + 1;
            if (rb >= nrows) continue;
            float4 A, Bq;
            {
                const C z = lds[l * ls + k], zc = lds[l * ls + (k == 0 ? 0 : n - k)];  // Z[k], Z[-k]
                A.x = h * (z.x + zc.x); A.y = h * (z.y - zc.y);
                Bq.x = h * (z.y + zc.y); Bq.y = -h * (z.x - zc.x);
            }
            if (k + 1 < nkx) {
                const C z = lds[l * ls + k + 1], zc = lds[l * ls + n - k - 1];
                A.z = h * (z.x + zc.x); A.w = h * (z.y - zc.y);
                Bq.z = h * (z.y + zc.y); Bq.w = -h * (z.x - zc.x);
                *reinterpret_cast<float4 *>(out + (size_t)ra * ldc + k) = A;
                *reinterpret_cast<float4 *>(out + (size_t)rb * ldc + k) = Bq;
            } else {
                out[(size_t)ra * ldc + k] = mk<C>(A.x, A.y);
                out[(size_t)rb * ldc + k] = mk<C>(Bq.x, Bq.y);
            }
        }
        return;
    }
    for (int e = threadIdx.x; e < B * nkx; e += FFT_THREADS) {
        const int l = udiv(e, dk), k = e - l * nkx;
        const int ra = r0 + 2 * l, rb = ra + 1;
        if (rb >= nrows) continue;
        const C z = lds[l * ls + k];
        const C zc = lds[l * ls + (k == 0 ? 0 : n - k)];  // Z[-k]
        // A = (Z + conj Z[-k]) / 2, B = (Z - conj Z[-k]) / (2 i)
        const S h = (S)0.5;
        out[(size_t)ra * ldc + k] = mk<C>(h * (z.x + zc.x), h * (z.y - zc.y));
        out[(size_t)rb * ldc + k] = mk<C>(h * (z.y + zc.y), -h * (z.x - zc.x));
    }
}

template <class S, class TO, bool R6>
__global__ void __launch_bounds__(FFT_THREADS)
k_fft_x_inv(const cplx<S> *__restrict__ in, const double *__restrict__ sinv, TO *__restrict__ out,
            Radices rd, const cplx<S> *__restrict__ tw, int lb, int nrows, int nkx, int ldc, Div dn, Div dn4) {
    using C = cplx<S>;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    C *lds = reinterpret_cast<C *>(lds_raw);
    const int n = rd.n, ls = n + 1, B = 1 << lb;
    const int r0 = blockIdx.x * 2 * B;
    C *twl = lds + B * ls;
    load_batched<FFT_KL, FFT_THREADS, C>(
        B * n,
        [&](int e) {
            const int l = udiv(e, dn), k = e - l * n;
            const int ra = r0 + 2 * l, rb = ra + 1;
            C z = mk<C>(0, 0);
            if (rb < nrows) {
                const int kk = (k < nkx) ? k : n - k;
                C A = in[(size_t)ra * ldc + kk], Bv = in[(size_t)rb * ldc + kk];
                if (kk == 0 || 2 * kk == n) { A.y = 0; Bv.y = 0; }
                if (k >= nkx) { A.y = -A.y; Bv.y = -Bv.y; }  // Hermitian extension
                z = mk<C>(A.x - Bv.y, A.y + Bv.x);           // A + i B
            }
            return z;
        },
        [&](int e, C v) {
            const int l = udiv(e, dn), k = e - l * n;
            lds[l * ls + k] = v;
        },
        tw, twl, n);
    __syncthreads();
    fft_lines<R6, false>(lds, rd, lb, 1, ls, twl, true);
    if (!sinv && (n & 3) == 0) {
        // unscaled rows of a multiple of 4: four values of each row per store
        typedef TO TO4 __attribute__((ext_vector_type(4)));
        const int n4 = n >> 2;
        for (int e = threadIdx.x; e < B * n4; e += FFT_THREADS) {
            const int l = udiv(e, dn4), t4 = e - l * n4;
            const int ra = r0 + 2 * l;
            if (ra + 1 >= nrows) continue;
            TO4 a, b;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const C z = lds[l * ls + 4 * t4 + q];
                a[q] = (TO)z.x;
                b[q] = (TO)z.y;
            }
            const size_t ia = (size_t)ra * n + 4 * t4;
            *reinterpret_cast<TO4 *>(out + ia) = a;
            *reinterpret_cast<TO4 *>(out + ia + n) = b;
        }
        return;
    }
    for (int e = threadIdx.x; e < B * n; e += FFT_THREADS) {
        const int l = udiv(e, dn), t = e - l * n;
        const int ra = r0 + 2 * l, rb = ra + 1;
        if (rb >= nrows) continue;
        const C z = lds[l * ls + t];
        const size_t ia = (size_t)ra * n + t, ib = ia + n;
        if (sinv) {
            out[ia] = (TO)((double)z.x * sinv[ia]);
            out[ib] = (TO)((double)z.y * sinv[ib]);
        } else {
            out[ia] = (TO)z.x;
            out[ib] = (TO)z.y;
        }
    }
}

// Block -> (line tile, row) of the y and z passes, XCD-aware: the grid is
// one-dimensional and padded to a multiple of 8; hardware block b runs on XCD
// b mod 8, which gets the contiguous run of tiles [xcd * per, (xcd + 1) * per),
// so the line tiles of one row (which share the 128-byte cache lines at their
// edges) run side by side on one XCD and its L2 serves the shared lines once.
// Returns false for the padding blocks.  (Tiles that leave out the columns
// beyond the last full group of B, with those columns' lines grouped along
// the rows instead, measured slower: their scattered accesses form a tail.)
__device__ __forceinline__ bool xcd_tile2(int ntx, int nty, int &tx, int &ty) {
    const int per = gridDim.x / 8;
    const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (t >= ntx * nty) return false;
    ty = t / ntx;
    tx = t - ty * ntx;
    return true;
}
inline int xcd_grid(int n) { return (n + 7) / 8 * 8; }

// Float32 spectrum, lines interleaved in LDS (element t of line l at t B + l,
// B = 2^lb >= 2): the block's B n values move between the spectrum (element
// t of line l at base + t stride + l) and LDS two neighbouring lines per
// 16-byte access; lines from bw on are zero in LDS and are not written back.
// pair_load also brings the n twiddles into twl.
__device__ __forceinline__ void pair_load(float2 *lds, const float2 *__restrict__ c, size_t base, size_t stride,
                                          int lb, int n, int bw, const float2 *__restrict__ tw, float2 *twl) {
    for (int e = threadIdx.x; e < n; e += FFT_THREADS) twl[e] = tw[e];
    constexpr int KP = FFT_MAXE / 2 / FFT_THREADS;
    const int np = (n << lb) >> 1, hmask = (1 << (lb - 1)) - 1;
    for (int e0 = 0; e0 < np; e0 += KP * FFT_THREADS) {
        float4 v[KP];
#pragma unroll
        for (int m = 0; m < KP; ++m) {
            const int e = e0 + threadIdx.x + m * FFT_THREADS;
            if (e < np) {
                const int t = e >> (lb - 1), l = (e & hmask) << 1;
                const float2 *src = c + base + (size_t)t * stride + l;
                if (l + 1 < bw) v[m] = *reinterpret_cast<const float4 *>(src);
                else if (l < bw) v[m] = make_float4(src->x, src->y, 0.0f, 0.0f);
                else v[m] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
        }
#pragma unroll
        for (int m = 0; m < KP; ++m) {
            const int e = e0 + threadIdx.x + m * FFT_THREADS;
            if (e < np) reinterpret_cast<float4 *>(lds)[e] = v[m];
        }
    }
}
__device__ __forceinline__ void pair_store(const float2 *lds, float2 *__restrict__ c, size_t base, size_t stride,
                                           int lb, int n, int bw) {
    const int np = (n << lb) >> 1, hmask = (1 << (lb - 1)) - 1;
    for (int e = threadIdx.x; e < np; e += FFT_THREADS) {
        const int t = e >> (lb - 1), l = (e & hmask) << 1;
        float2 *dst = c + base + (size_t)t * stride + l;
        const float4 v = reinterpret_cast<const float4 *>(lds)[e];
        if (l + 1 < bw) *reinterpret_cast<float4 *>(dst) = v;
        else if (l < bw) *dst = make_float2(v.x, v.y);
    }
}

// ---------------------------------------------------------------- y pass
// Block (tile of B = 2^lb consecutive kx, plane z): lines along y, LDS
// element (y, l) at y * B + l.
// INV: the inverse transform (a template argument, so that the butterflies'
// direction is fixed at compile time).
template <class S, bool R6, bool INV>
__global__ void __launch_bounds__(FFT_THREADS)
k_fft_y(cplx<S> *__restrict__ c, Radices rd, const cplx<S> *__restrict__ tw, int lb, int nkx, int ldc, int nz) {
    using C = cplx<S>;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    C *lds = reinterpret_cast<C *>(lds_raw);
    const int ny = rd.n, B = 1 << lb, bmask = B - 1;
    int bt, z;
    if (!xcd_tile2((nkx + B - 1) / B, nz, bt, z)) return;
    const int kx0 = bt * B;
    const int bw = min(B, nkx - kx0);
    const size_t base = (size_t)z * ny * ldc + kx0;
    C *twl = lds + B * ny;
    constexpr bool PAIRS = sizeof(S) == 4;
    if (PAIRS && lb >= 1) {
        pair_load(reinterpret_cast<float2 *>(lds), reinterpret_cast<const float2 *>(c), base, ldc, lb, ny, bw,
                  reinterpret_cast<const float2 *>(tw), reinterpret_cast<float2 *>(twl));
    } else {
        load_batched<FFT_KL, FFT_THREADS, C>(
            B * ny,
            [&](int e) {
                const int y = e >> lb, l = e & bmask;
                return (l < bw) ? c[base + (size_t)y * ldc + l] : mk<C>(0, 0);
            },
            [&](int e, C v) { lds[e] = v; }, tw, twl, ny);
    }
    __syncthreads();
    fft_lines<R6, true>(lds, rd, lb, B, 1, twl, INV);
    if (PAIRS && lb >= 1) {
        pair_store(reinterpret_cast<const float2 *>(lds), reinterpret_cast<float2 *>(c), base, ldc, lb, ny, bw);
        return;
    }
    for (int e = threadIdx.x; e < B * ny; e += FFT_THREADS) {
        const int y = e >> lb, l = e & bmask;
        if (l < bw) c[base + (size_t)y * ldc + l] = lds[e];
    }
}

// ---------------------------------------------------------------- z pass + Green
// -1 / lambda through the hardware reciprocal (two Newton steps in float64).
__device__ __forceinline__ double neg_recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    return -r;
}
__device__ __forceinline__ float neg_recip(float d) { return -__builtin_amdgcn_rcpf(d); }

// Block (tile of B = 2^lb consecutive kx, row y): lines along z, LDS element
// (z, l) at z * B + l.
template <class S, bool R6, int MAXE = FFT_MAXE, int NT = FFT_THREADS>
__global__ void __launch_bounds__(NT)
k_fft_z_green(cplx<S> *__restrict__ c, Radices rd, const cplx<S> *__restrict__ tw, int lb, int nkx, int ldc, int ny,
              const S *__restrict__ lamx, const S *__restrict__ lamy, const S *__restrict__ lamz, S inv_n,
              int lam_lds) {
    using C = cplx<S>;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    C *lds = reinterpret_cast<C *>(lds_raw);
    const int nz = rd.n, B = 1 << lb, bmask = B - 1;
    int bt, y;
    if (!xcd_tile2((nkx + B - 1) / B, ny, bt, y)) return;
    const int kx0 = bt * B;
    const int bw = min(B, nkx - kx0);
    const size_t zstride = (size_t)ny * ldc;
    const size_t base = (size_t)y * ldc + kx0;
    C *twl = lds + B * nz;
    // with lam_lds the symbol's z values and the block's kx values follow
    // the twiddles, loaded with the lines (the Green step then reads LDS only)
    S *lz = reinterpret_cast<S *>(twl + nz), *lx = lz + nz;
    if (lam_lds) {
        for (int e = threadIdx.x; e < nz + B; e += NT) {
            if (e < nz) lz[e] = lamz[e];
            else if (kx0 + e - nz < nkx) lx[e - nz] = lamx[kx0 + e - nz];
        }
    }
    constexpr bool PAIRS = sizeof(S) == 4 && NT == FFT_THREADS && MAXE == FFT_MAXE;
    if (PAIRS && lb >= 1) {
        pair_load(reinterpret_cast<float2 *>(lds), reinterpret_cast<const float2 *>(c), base, zstride, lb, nz, bw,
                  reinterpret_cast<const float2 *>(tw), reinterpret_cast<float2 *>(twl));
    } else {
        load_batched<(MAXE + NT - 1) / NT, NT, C>(
            B * nz,
            [&](int e) {
                const int z = e >> lb, l = e & bmask;
                return (l < bw) ? c[base + (size_t)z * zstride + l] : mk<C>(0, 0);
            },
            [&](int e, C v) { lds[e] = v; }, tw, twl, nz);
    }
    __syncthreads();
    fft_lines<R6, true, C, MAXE, NT>(lds, rd, lb, B, 1, twl, false);
    const S ly = lamy[y];
    for (int e = threadIdx.x; e < B * nz; e += NT) {
        const int z = e >> lb, l = e & bmask;
        const int kx = kx0 + l;
        S g = 0;
        if (l < bw && (kx | y | z) != 0)
            g = inv_n * neg_recip((lam_lds ? lx[l] : lamx[kx]) + ly + (lam_lds ? lz[z] : lamz[z]));
        const C v = lds[e];
        lds[e] = mk<C>(v.x * g, v.y * g);
    }
    __syncthreads();
    fft_lines<R6, true, C, MAXE, NT>(lds, rd, lb, B, 1, twl, true);
    if (PAIRS && lb >= 1) {
        pair_store(reinterpret_cast<const float2 *>(lds), reinterpret_cast<float2 *>(c), base, zstride, lb, nz, bw);
        return;
    }
    for (int e = threadIdx.x; e < B * nz; e += NT) {
        const int z = e >> lb, l = e & bmask;
        if (l < bw) c[base + (size_t)z * zstride + l] = lds[e];
    }
}

// Raise a kernel's dynamic LDS limit to 160 KB, once per device (bit d of
// `done`), when a launch asks for more than the default 64 KB.
void lds_attr(const void *fn, std::atomic<unsigned> &done, size_t bytes) {
    if (bytes <= 64 * 1024) return;
    int dev = 0;
    DWP_HIP(hipGetDevice(&dev));
    const unsigned bit = 1u << (dev & 31);
    if (done.load() & bit) return;
    DWP_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    done.fetch_or(bit);
}
template <class F> const void *fptr(F *f) { return reinterpret_cast<const void *>(f); }

Radices radices_of(const FFTAxis &ax) {
    Radices r{};
    r.n = ax.n;
    r.nst = (int)ax.radices.size();
    int p = 1;
    for (int s = 0; s < r.nst; ++s) {
        r.r[s] = ax.radices[s];
        r.p[s] = p;
        r.pm[s] = make_div(p).m;
        r.tstride[s] = ax.n / (p * ax.radices[s]);
        p *= ax.radices[s];
    }
    return r;
}

// Lines per block: the largest power of two with B * n <= budget, capped at
// 16 (16 lines of the padded spectrum are 256 contiguous bytes).
int tile_log2(int n, int budget) {
    int lb = 0;
    while (lb < 4 && (2 << lb) * n <= budget) ++lb;
    return lb;
}

}  // namespace

// Radix plan, twiddles and the discrete symbol 4 sin^2(pi m / n) / h^2 of one
// axis (m < n / 2 + 1 when `half`).  Twiddles and symbol are evaluated in long
// double on the host.
void fft_plan_axis(FFTAxis &ax, int n, double h, bool half, int order) {
    ax.n = n;
    ax.radices.clear();
    int m = n, a = 0, b = 0;
    while (m % 3 == 0) { ++a; m /= 3; }
    while (m % 2 == 0) { ++b; m /= 2; }
    // radix 8 for the power of two as far as it goes; a lone factor 2 left
    // over pairs with a factor 3 into one radix-6 stage (384 = 6 8 8: three
    // stages instead of four) on lines short enough for one radix-6
    // butterfly per thread of a block
    const bool six = a > 0 && b % 3 == 1 && n <= 6 * FFT_THREADS;
    for (int i = 0; i < a - (six ? 1 : 0); ++i) ax.radices.push_back(3);
    if (six) ax.radices.push_back(6);
    for (int i = 0; i < b / 3; ++i) ax.radices.push_back(8);
    if (b % 3 == 2) ax.radices.push_back(4);
    if (b % 3 == 1 && !six) ax.radices.push_back(2);
    if (m != 1 || (int)ax.radices.size() > MAX_STAGES) fail(DWP_EINVAL, "grid size must be 2^a 3^b");
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<double2> tw(n);
    std::vector<float2> tw32(n);
    for (int t = 0; t < n; ++t) {
        const long double a = -2.0L * pi * (long double)t / (long double)n;
        tw[t] = make_double2((double)cosl(a), (double)sinl(a));
        tw32[t] = make_float2((float)cosl(a), (float)sinl(a));
    }
    const int nl = half ? n / 2 + 1 : n;
    std::vector<double> lam(nl);
    std::vector<float> lam32(nl);
    for (int k = 0; k < nl; ++k) {
        if (order == 6) {
            // minus the eigenvalue of the seven-point second derivative (Eq. 18)
            const long double th = 2.0L * pi * (long double)k / (long double)n;
            const long double v = -(-49.0L / 18.0L) - 2.0L * (1.5L * cosl(th) - 0.15L * cosl(2.0L * th) +
                                                                 cosl(3.0L * th) / 90.0L);
            lam[k] = (double)(v / ((long double)h * (long double)h));
        } else {
            const long double s = sinl(pi * (long double)k / (long double)n);
            lam[k] = (double)(4.0L * s * s / ((long double)h * (long double)h));
        }
        lam32[k] = (float)lam[k];
    }
    ax.tw.alloc(sizeof(double2) * n);
    ax.lam.alloc(sizeof(double) * nl);
    ax.tw32.alloc(sizeof(float2) * n);
    ax.lam32.alloc(sizeof(float) * nl);
    DWP_HIP(hipMemcpy(ax.tw.p, tw.data(), sizeof(double2) * n, hipMemcpyHostToDevice));
    DWP_HIP(hipMemcpy(ax.lam.p, lam.data(), sizeof(double) * nl, hipMemcpyHostToDevice));
    DWP_HIP(hipMemcpy(ax.tw32.p, tw32.data(), sizeof(float2) * n, hipMemcpyHostToDevice));
    DWP_HIP(hipMemcpy(ax.lam32.p, lam32.data(), sizeof(float) * nl, hipMemcpyHostToDevice));
}

template <class S, class TI, class TO>
static void vacuum_solve_t(hipStream_t st, const Plan &p, const FFTAxis &ax, const FFTAxis &ay, const FFTAxis &az,
                           const TI *r, const double *sinv, void *cbuf_v, TO *out, Profiler *prof) {
    using C = cplx<S>;
    C *cbuf = static_cast<C *>(cbuf_v);
    auto TW = [](const FFTAxis &a) { return sizeof(S) == 8 ? a.tw.as<C>() : a.tw32.as<C>(); };
    auto LAM = [](const FFTAxis &a) { return sizeof(S) == 8 ? a.lam.as<S>() : a.lam32.as<S>(); };
    // algorithmic bytes of each pass: the real grid (8 B / point, twice when
    // scaled) and the half-spectrum (one complex value) read and written once
    const double Cn = (double)p.nkx * p.ny * p.nz, cb = (double)sizeof(C);
    const double bx = (sinv ? 8.0 + sizeof(TI) : (double)sizeof(TI)) * p.N + cb * Cn;
    const double bxi = (sinv ? 8.0 + sizeof(TO) : (double)sizeof(TO)) * p.N + cb * Cn;
    auto pb = [&](int g) { return prof ? prof->begin(st, g) : -1; };
    auto pe = [&](int ev, int g, double b) { if (prof) prof->end(st, ev, g, b); };
    int ev;
    // each pass in the variant with or without a radix-6 stage, as its axis'
    // plan needs (the radix-6 code costs registers where it is not used)
    auto has6 = [](const FFTAxis &a) { return std::find(a.radices.begin(), a.radices.end(), 6) != a.radices.end(); };
    auto RD = [](const FFTAxis &a) { return radices_of(a); };
    // a pass with a radix-6 stage takes at most 6 values per thread in a block
    auto budget = [&](const FFTAxis &a, int b, int nt) { return has6(a) ? std::min(b, 6 * nt) : b; };
    auto with6 = [](bool six, auto &&f) {
        if (six) f(std::true_type{});
        else f(std::false_type{});
    };
    const int nrows = p.ny * p.nz;
    const int lbx = tile_log2(p.nx, budget(ax, sizeof(S) == 4 ? FFT_BUDGET_X32 : FFT_BUDGET_X, FFT_THREADS));
    const int Bx = 1 << lbx;
    const int gx = (nrows + 2 * Bx - 1) / (2 * Bx);
    const size_t ldsx = sizeof(C) * ((size_t)Bx * (p.nx + 1) + p.nx);
    const Div dn = make_div(p.nx), dk = make_div(p.nkx), dn4 = make_div(p.nx / 4 > 0 ? p.nx / 4 : 1),
              dk2 = make_div((p.nkx + 1) / 2);
    const int lby = tile_log2(p.ny, budget(ay, FFT_BUDGET_Y, FFT_THREADS)), By = 1 << lby;
    const int gy = xcd_grid((p.nkx + By - 1) / By * p.nz);
    const size_t ldsy = sizeof(C) * ((size_t)By * p.ny + p.ny);
    auto y_pass = [&](auto inv) {
        constexpr bool INV = decltype(inv)::value;
        with6(has6(ay), [&](auto r6) {
            constexpr bool R6 = decltype(r6)::value;
            static std::atomic<unsigned> attr{0};
            lds_attr(fptr(&k_fft_y<S, R6, INV>), attr, ldsy);
            k_fft_y<S, R6, INV><<<gy, FFT_THREADS, ldsy, st>>>(cbuf, RD(ay), TW(ay), lby, p.nkx, p.ldc, p.nz);
            DWP_LAUNCH_CHECK();
        });
    };
    ev = pb(PG_FFT_X);
    with6(has6(ax), [&](auto r6) {
        constexpr bool R6 = decltype(r6)::value;
        static std::atomic<unsigned> attr{0};
        lds_attr(fptr(&k_fft_x_fwd<S, TI, R6>), attr, ldsx);
        k_fft_x_fwd<S, TI, R6><<<gx, FFT_THREADS, ldsx, st>>>(r, sinv, cbuf, RD(ax), TW(ax), lbx, nrows, p.nkx,
                                                             p.ldc, dn, dk, dn4, dk2);
        DWP_LAUNCH_CHECK();
    });
    pe(ev, PG_FFT_X, bx);
    ev = pb(PG_FFT_Y);
    y_pass(std::false_type{});
    pe(ev, PG_FFT_Y, 2.0 * cb * Cn);
    // z pass with the Green's function (lines of 8 kx; the twiddles follow
    // the lines in LDS)
    ev = pb(PG_FFT_Z);
    with6(has6(az), [&](auto r6) {
        constexpr bool R6 = decltype(r6)::value;
        const int lbz = tile_log2(p.nz, budget(az, FFT_Z_MAXE, FFT_Z_THREADS)), Bz = 1 << lbz;
        const int gz = xcd_grid((p.nkx + Bz - 1) / Bz * p.ny);
        // the symbol staged in LDS too where it fits
        const size_t base_bytes = sizeof(C) * ((size_t)Bz * p.nz + p.nz);
        const size_t lam_bytes = sizeof(S) * ((size_t)p.nz + Bz);
        const int lam_lds = base_bytes + lam_bytes <= 160 * 1024 ? 1 : 0;
        const size_t bytes = base_bytes + (lam_lds ? lam_bytes : 0);
        static std::atomic<unsigned> attr{0};
        lds_attr(fptr(&k_fft_z_green<S, R6, FFT_Z_MAXE, FFT_Z_THREADS>), attr, bytes);
        k_fft_z_green<S, R6, FFT_Z_MAXE, FFT_Z_THREADS><<<gz, FFT_Z_THREADS, bytes, st>>>(
            cbuf, RD(az), TW(az), lbz, p.nkx, p.ldc, p.ny, LAM(ax), LAM(ay), LAM(az), (S)(1.0 / (double)p.N), lam_lds);
        DWP_LAUNCH_CHECK();
    });
    pe(ev, PG_FFT_Z, 2.0 * cb * Cn);
    ev = pb(PG_FFT_Y);
    y_pass(std::true_type{});
    pe(ev, PG_FFT_Y, 2.0 * cb * Cn);
    ev = pb(PG_FFT_X);
    with6(has6(ax), [&](auto r6) {
        constexpr bool R6 = decltype(r6)::value;
        static std::atomic<unsigned> attr{0};
        lds_attr(fptr(&k_fft_x_inv<S, TO, R6>), attr, ldsx);
        k_fft_x_inv<S, TO, R6><<<gx, FFT_THREADS, ldsx, st>>>(cbuf, sinv, out, RD(ax), TW(ax), lbx, nrows,
                                                             p.nkx, p.ldc, dn, dn4);
        DWP_LAUNCH_CHECK();
    });
    pe(ev, PG_FFT_X, bxi);
}

void launch_vacuum_solve(hipStream_t st, const Plan &p, const FFTAxis &ax, const FFTAxis &ay, const FFTAxis &az,
                         const double *r, const double *sinv, void *cbuf, double *out, Profiler *prof, bool fp32) {
    if (fp32) vacuum_solve_t<float, double, double>(st, p, ax, ay, az, r, sinv, cbuf, out, prof);
    else vacuum_solve_t<double, double, double>(st, p, ax, ay, az, r, sinv, cbuf, out, prof);
}
void launch_vacuum_solve(hipStream_t st, const Plan &p, const FFTAxis &ax, const FFTAxis &ay, const FFTAxis &az,
                         const float *r, const double *sinv, void *cbuf, float *out, Profiler *prof, bool fp32) {
    if (fp32) vacuum_solve_t<float, float, float>(st, p, ax, ay, az, r, sinv, cbuf, out, prof);
    else vacuum_solve_t<double, float, float>(st, p, ax, ay, az, r, sinv, cbuf, out, prof);
}
void launch_vacuum_solve(hipStream_t st, const Plan &p, const FFTAxis &ax, const FFTAxis &ay, const FFTAxis &az,
                         const _Float16 *r, const double *sinv, void *cbuf, float *out, Profiler *prof, bool fp32) {
    if (fp32) vacuum_solve_t<float, _Float16, float>(st, p, ax, ay, az, r, sinv, cbuf, out, prof);
    else vacuum_solve_t<double, _Float16, float>(st, p, ax, ay, az, r, sinv, cbuf, out, prof);
}

}  // namespace dwp
