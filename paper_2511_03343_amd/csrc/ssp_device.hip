// ssp_device.hip - gfx950 kernels of the spectral split-step Pade range march.
//
// Transform (Sec. 3.1): the orthonormal DST-I of length N on the interior Dirichlet grid
// is evaluated as a chirp-z transform.  With M = N+1 and c_d = exp(i pi d^2/(2M)),
//   DST(x)_k = (i/2) sqrt(2/M) conj(c_k) sum_{n=1..N} conj(c_n) x_n (c_{k-n} - c_{k+n}),
// i.e. a Toeplitz term (kernel window d in [1-N, N-1]) minus a Hankel term (window
// d in [2, 2N]).  Both are cyclic convolutions of length P >= 2N-1 (a power of two), and the
// Hankel term is the Toeplitz form of the index-reversed input, whose spectrum is the
// reflected spectrum Y_{-q}.  One DST therefore costs one forward FFT of length P, a
// pointwise combine Z_q = Y_q K1_q - Y_{-q} K2_q, and one inverse FFT.
//
// Range step (Sec. 3 eq. neumannseries; Alg. 1): the state is kept in the sine basis
// multiplied by conj(c_l) (the "modulated" representation), so that the chirp factors of
// consecutive transforms fold into single pointwise tables:
//   Neumann term m:   a_m = B_j (.) IFFT(comb(FFT( A (.) IFFT(comb(FFT(a_{m-1}))) )))
// with A = v (.) conj(c)^2 (i/2) sqrt(2/M)/P and B_j = -b_j/(1 + b_j x) (.) the same factor.
// Pade factors are applied in product form u <- g_j u + (1 - g_j) w_j (the same
// approximant as the paper's sum form; better conditioned in FP32).
//
// One workgroup owns one solve for a whole launch: its field, all Pade factors and all
// Neumann terms of every step stay on chip (registers + LDS).  Precision: complex FP32
// data; FFT twiddles and the sine-space multipliers are double-float (hi + lo) products so
// that no fixed rounding of a table enters every step; residual norms in FP64; carrier
// phase in FP64.
#include "ssp_device.h"

#include <math.h>

namespace ssp {
namespace {

constexpr int kOK = 0, kNotConverged = 1, kDiverged = -4;

// ----------------------------------------------------------------------------- complex
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// x * (w.hi + w.lo) with w = (hi.re, hi.im, lo.re, lo.im): the small products first, so the
// result carries only the rounding of the arithmetic, not the rounding of the table.
__device__ __forceinline__ float2 cmul_df(float2 x, float4 w) {
    float re = fmaf(-x.y, w.w, x.x * w.z);
    re = fmaf(x.x, w.x, re);
    re = fmaf(-x.y, w.y, re);
    float im = fmaf(x.y, w.z, x.x * w.w);
    im = fmaf(x.x, w.y, im);
    im = fmaf(x.y, w.x, im);
    return make_float2(re, im);
}
// x * conj(w.hi + w.lo)
__device__ __forceinline__ float2 cmul_df_conj(float2 x, float4 w) {
    float re = fmaf(x.y, w.w, x.x * w.z);
    re = fmaf(x.x, w.x, re);
    re = fmaf(x.y, w.y, re);
    float im = fmaf(-x.x, w.w, x.y * w.z);
    im = fmaf(-x.x, w.y, im);
    im = fmaf(x.y, w.x, im);
    return make_float2(re, im);
}

// ----------------------------------------------------------------------------- memory
// Global memory is accessed through buffer resources: the base address stays in scalar
// registers and each access carries a 32-bit byte offset, which keeps loop-invariant
// 64-bit addresses out of the vector register file.  Every array addressed this way is
// smaller than 2 GiB (tables, one solve's field, one output row).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ float2 ld2(const float2 *p, int i) {
    auto v = __builtin_amdgcn_raw_buffer_load_b64(rsrc(p), i * 8, 0, 0);
    return make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
}
__device__ __forceinline__ float4 ld4(const float4 *p, int i) {
    auto v = __builtin_amdgcn_raw_buffer_load_b128(rsrc(p), i * 16, 0, 0);
    return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]),
                       __uint_as_float(v[3]));
}
__device__ __forceinline__ float ldf(const float *p, int i) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsrc(p), i * 4, 0, 0));
}
__device__ __forceinline__ void st2(float2 *p, int i, float2 v) {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    u2 x = {__float_as_uint(v.x), __float_as_uint(v.y)};
    __builtin_amdgcn_raw_buffer_store_b64(x, rsrc(p), i * 8, 0, 0);
}
__device__ __forceinline__ void stf(float *p, int i, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rsrc(p), i * 4, 0, 0);
}

// ----------------------------------------------------------------------------- radix-R DFT
// cos(2 pi i/16), i = 0..15
__device__ constexpr double kCos16[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};

// x * exp(-+ 2 pi i k / R) (minus for the forward transform), R <= 16
template <int R, bool INV>
__device__ __forceinline__ float2 mulw(float2 x, int k) {
    const int i16 = (k * (16 / R)) & 15;
    if (i16 == 0) return x;
    if (i16 == 8) return make_float2(-x.x, -x.y);
    if (i16 == 4) return INV ? make_float2(-x.y, x.x) : make_float2(x.y, -x.x);
    if (i16 == 12) return INV ? make_float2(x.y, -x.x) : make_float2(-x.y, x.x);
    const double c = kCos16[i16], s = kCos16[(i16 + 12) & 15];
    const float ch = static_cast<float>(c), cl = static_cast<float>(c - static_cast<double>(ch));
    const float sh = static_cast<float>(s), sl = static_cast<float>(s - static_cast<double>(sh));
    // forward: x (c - i s); inverse: x (c + i s)
    const float sg = INV ? -1.0f : 1.0f;
    float re = fmaf(sg * x.y, sl, x.x * cl);
    re = fmaf(x.x, ch, re);
    re = fmaf(sg * x.y, sh, re);
    float im = fmaf(-sg * x.x, sl, x.y * cl);
    im = fmaf(x.y, ch, im);
    im = fmaf(-sg * x.x, sh, im);
    return make_float2(re, im);
}

template <int R, bool INV>
struct Dft {
    // in-place DFT of x[0..R) (natural order in and out), decimation in time
    __device__ __forceinline__ static void run(float2 *x) {
        float2 e[R / 2], o[R / 2];
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
            e[k] = x[2 * k];
            o[k] = x[2 * k + 1];
        }
        Dft<R / 2, INV>::run(e);
        Dft<R / 2, INV>::run(o);
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
            float2 t = mulw<R, INV>(o[k], k);
            x[k] = cadd(e[k], t);
            x[k + R / 2] = csub(e[k], t);
        }
    }
};
template <bool INV>
struct Dft<2, INV> {
    __device__ __forceinline__ static void run(float2 *x) {
        float2 a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    }
};
template <bool INV>
struct Dft<1, INV> {
    __device__ __forceinline__ static void run(float2 *) {}
};

// ----------------------------------------------------------------------------- FFT in LDS
// LDS index map.  Kept linear so that the per-radix element offsets fold into the
// instructions' immediate offsets instead of occupying address registers.
__device__ __forceinline__ int pad(int i) { return i; }
constexpr int lds_len(int P) { return P; }

// One self-sorting (Stockham) radix-R pass over the P-point sequence in LDS:
// butterfly j (k = j mod Ns) reads x_r = buf[j + r P/R], applies w_{Ns R}^{r k}, takes the
// R-point DFT and writes buf[(j - k) R + k + r Ns].  All reads complete before any write.
template <int P, int T, int R, bool INV>
__device__ __forceinline__ void stockham_pass(float2 *buf, int Ns, const float4 *__restrict__ tw) {
    constexpr int NB = P / R;
    constexpr int PER = (NB + T - 1) / T;
    const int tid = threadIdx.x;
    float2 x[PER][R];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int j = tid + i * T;
        if (NB % T == 0 || j < NB) {
#pragma unroll
            for (int r = 0; r < R; ++r) x[i][r] = buf[pad(j + r * NB)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int j = tid + i * T;
        if (NB % T == 0 || j < NB) {
            const int k = j & (Ns - 1);
            if (Ns > 1) {
                const int stride = P / (Ns * R);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const float4 w = ld4(tw, r * k * stride);
                    x[i][r] = INV ? cmul_df_conj(x[i][r], w) : cmul_df(x[i][r], w);
                }
            }
            Dft<R, INV>::run(x[i]);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[pad(base + r * Ns)] = x[i][r];
        }
    }
    __syncthreads();
}

// largest radix <= 16 that keeps every thread busy (P/R butterflies >= T threads)
constexpr int pick_radix(int rem, int maxr) {
    int r = maxr >= 16 ? 16 : (maxr >= 8 ? 8 : (maxr >= 4 ? 4 : 2));
    return rem >= r ? r : rem;
}

template <int P, int T, bool INV, int Ns>
__device__ __forceinline__ void fft_passes(float2 *buf, const float4 *__restrict__ tw) {
    if constexpr (Ns < P) {
        constexpr int R = pick_radix(P / Ns, P / T);
        stockham_pass<P, T, R, INV>(buf, Ns, tw);
        fft_passes<P, T, INV, Ns * R>(buf, tw);
    }
}

// Z_q = Y_q K1_q - Y_{-q} K2_q in place; each thread owns the pair (q, P-q).
template <int P, int T>
__device__ __forceinline__ void chirp_combine(float2 *buf, const float2 *__restrict__ k1,
                                              const float2 *__restrict__ k2) {
    for (int q = threadIdx.x; q <= P / 2; q += T) {
        if (q == 0 || q == P / 2) {
            const float2 y = buf[pad(q)];
            buf[pad(q)] = cmul(y, csub(ld2(k1, q), ld2(k2, q)));
        } else {
            const float2 yq = buf[pad(q)], yr = buf[pad(P - q)];
            buf[pad(q)] = csub(cmul(yq, ld2(k1, q)), cmul(yr, ld2(k2, q)));
            buf[pad(P - q)] = csub(cmul(yr, ld2(k1, P - q)), cmul(yq, ld2(k2, P - q)));
        }
    }
    __syncthreads();
}

// The chirp-z core: z = IFFT(comb(FFT(x placed at positions 1..N))) at positions 1..N.
// x and z are distributed as element i of thread t <-> index m = t + i T (position m+1).
template <int P, int T>
__device__ __forceinline__ void chirp_core(float2 *buf, const SolveDesc &d, int N, const float2 *x,
                                           float2 *z) {
    constexpr int EPT = (P / 2 + T - 1) / T;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < P; idx += T)
        if (idx == 0 || idx > N) buf[pad(idx)] = make_float2(0.f, 0.f);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int m = tid + i * T;
        if (m < N) buf[pad(m + 1)] = x[i];
    }
    __syncthreads();
    fft_passes<P, T, false, 1>(buf, d.tw);
    chirp_combine<P, T>(buf, d.k1, d.k2);
    fft_passes<P, T, true, 1>(buf, d.tw);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int m = tid + i * T;
        z[i] = (m < N) ? buf[pad(m + 1)] : make_float2(0.f, 0.f);
    }
    __syncthreads();
}

// Sum two doubles over the workgroup in a fixed order (wave butterfly, then waves in
// index order); every thread returns the same values.
template <int T>
__device__ __forceinline__ void block_sum2(double &a, double &b, double *red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        red[2 * wave] = a;
        red[2 * wave + 1] = b;
    }
    __syncthreads();
    a = 0.0;
    b = 0.0;
#pragma unroll
    for (int w = 0; w < T / 64; ++w) {
        a += red[2 * w];
        b += red[2 * w + 1];
    }
    __syncthreads();
}

__device__ __forceinline__ double cnorm2(float2 v) {
    return static_cast<double>(v.x) * v.x + static_cast<double>(v.y) * v.y;
}

// exp(i sigma n) for the carrier of step n, in FP64: Cody-Waite reduction by pi/2 (two-part
// constant) and Taylor series of sin and cos on [-pi/4, pi/4] (truncation < 1e-17).
__device__ __forceinline__ float2 carrier(double sigma, long long n) {
    const double x = sigma * static_cast<double>(n);
    const double k = rint(x * 0.63661977236758134308);  // 2/pi
    const double r = fma(-k, 6.12323399573676603587e-17, fma(-k, 1.57079632679489655800, x));
    const double r2 = r * r;
    // sin r = r (1 - r^2/3! + r^4/5! - ...),  cos r = 1 - r^2/2! + r^4/4! - ...
    double sn = 1.0 / 6227020800.0, cs = 1.0 / 87178291200.0;
    sn = fma(sn, -r2, 1.0 / 39916800.0);
    sn = fma(sn, -r2, 1.0 / 362880.0);
    sn = fma(sn, -r2, 1.0 / 5040.0);
    sn = fma(sn, -r2, 1.0 / 120.0);
    sn = fma(sn, -r2, 1.0 / 6.0);
    sn = fma(sn, -r2, 1.0);
    sn *= r;
    cs = fma(cs, -r2, 1.0 / 479001600.0);
    cs = fma(cs, -r2, 1.0 / 3628800.0);
    cs = fma(cs, -r2, 1.0 / 40320.0);
    cs = fma(cs, -r2, 1.0 / 720.0);
    cs = fma(cs, -r2, 1.0 / 24.0);
    cs = fma(cs, -r2, 0.5);
    cs = fma(cs, -r2, 1.0);
    const long long q = static_cast<long long>(k) & 3;
    double c, s;
    if (q == 0) { c = cs; s = sn; }
    else if (q == 1) { c = -sn; s = cs; }
    else if (q == 2) { c = -cs; s = -sn; }
    else { c = sn; s = -cs; }
    return make_float2(static_cast<float>(c), static_cast<float>(s));
}

// v(z) = (c0/c)^2 - 1 for the analytic Munk + Gaussian-eddy environment, in FP64.
__device__ __forceinline__ float analytic_v(const SolveDesc &d, double z, double r) {
    const double eta = 2.0 * (z - d.env[2]) / d.env[2];
    double c = d.env[0] * (1.0 + d.env[1] * (eta + exp(-eta) - 1.0));
    if (d.env[3] != 0.0) {
        const double xr = (r - d.env[4]) / d.env[5], xz = (z - d.env[6]) / d.env[7];
        c -= d.env[3] * exp(-(xr * xr) - (xz * xz));
    }
    const double q = d.c0 / c;
    return static_cast<float>(q * q - 1.0);
}

template <int P, int T>
__device__ __forceinline__ void load_potential(const SolveDesc &d, long long n, float2 *A) {
    constexpr int EPT = (P / 2 + T - 1) / T;
    const int N = d.N;
    long long row = 0;
    if (d.prof_mode == PROF_TABLE_STEPS) {
        row = n - d.v_step0 - 1;
        row = row < 0 ? 0 : (row >= d.v_rows ? d.v_rows - 1 : row);
    }
    const double r = (static_cast<double>(n) - 0.5) * d.dr;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int m = threadIdx.x + i * T;
        if (m < N) {
            const float v = (d.prof_mode == PROF_ANALYTIC)
                                ? analytic_v(d, (m + 1) * d.dz, r)
                                : ldf(d.v + row * N, m);
            const float2 dm = ld2(d.dmod, m);
            A[i] = make_float2(v * dm.x, v * dm.y);
        } else {
            A[i] = make_float2(0.f, 0.f);
        }
    }
}

// ----------------------------------------------------------------------------- march
template <int P, int T>
__global__ __launch_bounds__(T) void k_march(const SolveDesc *__restrict__ descs, int nsteps) {
    __shared__ float2 buf[lds_len(P)];
    __shared__ double red[2 * (T / 64)];
    constexpr int EPT = (P / 2 + T - 1) / T;
    // large fields keep the Neumann multiplier in L2 instead of registers
    constexpr bool kBInRegs = (EPT <= 4);
    constexpr int EB = kBInRegs ? EPT : 1;
    const SolveDesc &d = descs[blockIdx.x];
    const int tid = threadIdx.x;
    const int N = d.N, p = d.p, nmax = d.nmax;

    // The state u is not held in registers: d.field holds the state at the start of the
    // step (the recovery point if the step diverges) and d.work the state between Pade
    // factors.  Every thread reads and writes only its own elements m = tid + i T, so these
    // global accesses need no barriers.
    float2 w[EPT], a[EPT], A[EPT];
    float4 Bm[EB];
    long long n = *d.step;
    if (d.prof_mode == PROF_TABLE_FIXED) load_potential<P, T>(d, n + 1, A);

    long long terms = 0, done = 0;
    int max_used = 0, notconv = 0, status = kOK;
    double max_res = 0.0;

    for (int s = 0; s < nsteps; ++s) {
        const long long nn = n + 1;
        if (d.prof_mode != PROF_TABLE_FIXED) load_potential<P, T>(d, nn, A);
        bool bad = false;
        for (int j = 0; j < p; ++j) {
            const float2 *cur = (j == 0) ? d.field : d.work;
            double t0 = 0.0, dummy = 0.0;
#pragma unroll
            for (int i = 0; i < EPT; ++i) {
                const int m = tid + i * T;
                if (m < N) {
                    a[i] = cmul_df(ld2(cur, m), ld4(d.s, j * N + m));
                    if constexpr (kBInRegs) Bm[i] = ld4(d.bmul, j * N + m);
                } else {
                    a[i] = make_float2(0.f, 0.f);
                    if constexpr (kBInRegs) Bm[i] = make_float4(0.f, 0.f, 0.f, 0.f);
                }
                w[i] = a[i];
                t0 += cnorm2(a[i]);
            }
            block_sum2<T>(t0, dummy, red);
            double tn = 0.0, wn = 0.0;
            int used = 0;
            bool conv = (nmax == 0);
            for (int it = 1; it <= nmax; ++it) {
                chirp_core<P, T>(buf, d, N, a, a);
#pragma unroll
                for (int i = 0; i < EPT; ++i) a[i] = cmul(A[i], a[i]);
                chirp_core<P, T>(buf, d, N, a, a);
                tn = 0.0;
                wn = 0.0;
#pragma unroll
                for (int i = 0; i < EPT; ++i) {
                    const int m = tid + i * T;
                    float4 bm;
                    if constexpr (kBInRegs) bm = Bm[i];
                    else bm = (m < N) ? ld4(d.bmul, j * N + m) : make_float4(0.f, 0.f, 0.f, 0.f);
                    a[i] = cmul_df(a[i], bm);
                    w[i] = cadd(w[i], a[i]);
                    tn += cnorm2(a[i]);
                    wn += cnorm2(w[i]);
                }
                block_sum2<T>(tn, wn, red);
                used = it;
                if (!(isfinite(tn) && isfinite(wn))) {
                    bad = true;
                    break;
                }
                if (tn <= d.tol2 * wn) {
                    conv = true;
                    break;
                }
            }
            if (bad) break;
            if (!conv) {
                if (tn >= t0) {  // the series' terms did not decrease: divergence
                    bad = true;
                    break;
                }
                ++notconv;
            }
            if (nmax > 0) {
                const double res = wn > 0.0 ? sqrt(tn / wn) : 0.0;
                max_res = res > max_res ? res : max_res;
            }
            terms += used;
            max_used = used > max_used ? used : max_used;
            // product-form factor: u <- g_j u + (1 - g_j) w_j  (alpha, beta double-float)
            const float4 al = ld4(d.alpha, j), be = ld4(d.beta, j);
#pragma unroll
            for (int i = 0; i < EPT; ++i) {
                const int m = tid + i * T;
                if (m < N) st2(d.work, m, cadd(cmul_df(ld2(cur, m), al), cmul_df(w[i], be)));
            }
        }
        if (bad) {
            status = kDiverged;
            break;
        }
        // commit the step
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int m = tid + i * T;
            if (m < N) st2(d.field, m, ld2(d.work, m));
        }
        n = nn;
        ++done;
        if (d.out_every > 0 && (n % d.out_every) == 0 && (d.tl_out || d.fld_out)) {
            float2 *z = w;  // w is free between steps
#pragma unroll
            for (int i = 0; i < EPT; ++i) {
                const int m = tid + i * T;
                z[i] = (m < N) ? ld2(d.field, m) : make_float2(0.f, 0.f);
            }
            chirp_core<P, T>(buf, d, N, z, z);
            const float2 car = carrier(d.sigma, n);
            const long long slot = (n - d.out_base) / d.out_every;
            const bool in_range = (n >= d.out_base) && (slot < d.nout);
            const float lr = log10f(static_cast<float>(static_cast<double>(n) * d.dr));
#pragma unroll
            for (int i = 0; i < EPT; ++i) {
                const int m = tid + i * T;
                if (m < N && in_range) {
                    const float2 ph = cmul(cmul(ld2(d.post, m), z[i]), car);
                    if (d.fld_out) st2(d.fld_out + slot * N, m, ph);
                    if (d.tl_out) stf(d.tl_out + slot * N, m, -10.0f * (log10f(ph.x * ph.x + ph.y * ph.y) - lr));
                }
            }
        }
    }
    if (tid == 0) {
        *d.step = n;
        if (status == kOK && notconv > 0) status = kNotConverged;
        DevStats st;
        st.steps_done = done;
        st.step_index = n;
        st.neumann_terms = terms;
        st.neumann_max_used = max_used;
        st.not_converged = notconv;
        st.max_residual = max_res;
        st.status = status;
        st.pad_ = 0;
        if (d.stats) *d.stats = st;
    }
}

// ----------------------------------------------------------------------------- transforms
template <int P, int T>
__global__ __launch_bounds__(T) void k_transform(const SolveDesc *__restrict__ desc, int mode,
                                                 const float2 *__restrict__ in, float2 *out,
                                                 const long long *__restrict__ step) {
    __shared__ float2 buf[lds_len(P)];
    constexpr int EPT = (P / 2 + T - 1) / T;
    const SolveDesc &d = *desc;
    const int N = d.N, tid = threadIdx.x;
    const size_t off = static_cast<size_t>(blockIdx.x) * N;
    float2 x[EPT], z[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int m = tid + i * T;
        float2 v = (m < N) ? ld2(in + off, m) : make_float2(0.f, 0.f);
        if (mode != 2 && m < N) v = cmul(v, ld2(d.pre, m));
        x[i] = v;
    }
    chirp_core<P, T>(buf, d, N, x, z);
    float2 car = make_float2(1.f, 0.f);
    if (mode == 2) {
        car = carrier(d.sigma, step[blockIdx.x]);
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int m = tid + i * T;
        if (m < N) {
            float2 v = cmul(z[i], mode == 1 ? ld2(d.dmod, m) : ld2(d.post, m));
            if (mode == 2) v = cmul(v, car);
            st2(out + off, m, v);
        }
    }
}

// workgroup size per FFT length: enough waves to hide LDS latency, <= 1024 threads
template <int P>
constexpr int threads_for() {
    return P <= 256 ? 64 : (P <= 1024 ? 128 : (P <= 4096 ? 256 : 1024));
}

template <int P>
hipError_t launch_march_P(const SolveDesc *d_descs, int nsolves, int nsteps, hipStream_t stream) {
    constexpr int T = threads_for<P>();
    hipLaunchKernelGGL((k_march<P, T>), dim3(nsolves), dim3(T), 0, stream, d_descs, nsteps);
    return hipGetLastError();
}

template <int P>
hipError_t launch_transform_P(int mode, const SolveDesc *d_desc, int B, const float2 *in,
                              float2 *out, const long long *step, hipStream_t stream) {
    constexpr int T = threads_for<P>();
    hipLaunchKernelGGL((k_transform<P, T>), dim3(B), dim3(T), 0, stream, d_desc, mode, in, out, step);
    return hipGetLastError();
}

}  // namespace

bool fft_length_supported(int P) {
    return P == 8 || P == 16 || P == 32 || P == 64 || P == 128 || P == 256 || P == 512 ||
           P == 1024 || P == 2048 || P == 4096 || P == 8192 || P == 16384;
}

#define SSP_DISPATCH_P(P, CALL) \
    switch (P) {                \
        case 8: return CALL(8);         \
        case 16: return CALL(16);       \
        case 32: return CALL(32);       \
        case 64: return CALL(64);       \
        case 128: return CALL(128);     \
        case 256: return CALL(256);     \
        case 512: return CALL(512);     \
        case 1024: return CALL(1024);   \
        case 2048: return CALL(2048);   \
        case 4096: return CALL(4096);   \
        case 8192: return CALL(8192);   \
        case 16384: return CALL(16384); \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_march(int P, const SolveDesc *d_descs, int nsolves, int nsteps, hipStream_t stream) {
    if (nsolves <= 0 || nsteps <= 0) return hipSuccess;
#define CALL_M(PP) launch_march_P<PP>(d_descs, nsolves, nsteps, stream)
    SSP_DISPATCH_P(P, CALL_M)
#undef CALL_M
}

hipError_t launch_transform(int P, int mode, const SolveDesc *d_desc, int B, const float2 *in,
                            float2 *out, const long long *step, hipStream_t stream) {
    if (B <= 0) return hipSuccess;
#define CALL_T(PP) launch_transform_P<PP>(mode, d_desc, B, in, out, step, stream)
    SSP_DISPATCH_P(P, CALL_T)
#undef CALL_T
}

}  // namespace ssp
