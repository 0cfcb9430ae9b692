// ssp_device.hip - gfx950 kernels of the spectral split-step Pade range march.
//
// Transform (Sec. 3.1): the orthonormal DST-I of length N on the interior Dirichlet grid
// is evaluated as a chirp-z transform.  With M = N+1 and c_d = exp(i pi d^2/(2M)),
//   DST(x)_k = (i/2) sqrt(2/M) conj(c_k) sum_{n=1..N} conj(c_n) x_n (c_{k-n} - c_{k+n}).
// Element n of a vector sits at chirp position n-1 (0 .. N-1), so the sum is a Toeplitz
// term (kernel window d in [1-N, N-1]) minus a Hankel term (c_{d+2}, d in [0, 2N-2]).  Both
// are cyclic convolutions of length P >= 2N-1 (a power of two), and the Hankel term is the
// Toeplitz form of the index-reversed input, whose spectrum is the reflected spectrum
// Y_{-q}.  One DST therefore costs one forward FFT of length P, a pointwise combine
// Z_q = Y_q K1_q - Y_{-q} K2_q, and one inverse FFT.
//
// Lengths above the largest FFT one workgroup holds in LDS (P = 2H, H = 16384): the input
// occupies positions below H, so the even-frequency half of FFT_P(y) is FFT_H(y) and the
// odd half is FFT_H(y (.) w_P^n).  The reflection q -> -q maps each half onto itself (even:
// k -> -k mod H; odd: k -> H-1-k), so the combine never mixes them, and the inverse is
// z_n = IFFT_H(Z_even)_n + w_P^{-n} IFFT_H(Z_odd)_n.  One DST is then two independent
// H-point chirp cores.
//
// Range step (Sec. 3 eq. neumannseries; Alg. 1): the state is kept in the sine basis
// multiplied by conj(c_l) (the "modulated" representation), so that the chirp factors of
// consecutive transforms fold into single pointwise tables:
//   Neumann term m:   a_m = B_j (.) IFFT(comb(FFT( A (.) IFFT(comb(FFT(a_{m-1}))) )))
// with A = v (.) conj(c)^2 (i/2) sqrt(2/M)/P and B_j = -b_j/(1 + b_j x) (.) the same factor.
// Pade factors are applied in product form u <- g_j u + (1 - g_j) w_j (the same
// approximant as the paper's sum form; better conditioned in FP32), written as the
// increment u <- u + (q_j u + beta_j w'_j) with q_j = r_j - 1 (r_j = g_j + (1 - g_j) s_j the
// factor's isovelocity multiplier) and w'_j the Neumann terms beyond the first.  The state
// then takes one rounding per factor: for the propagating modes r_j is within ~1e-6 of 1,
// the state changes by a few units in the last place per step, and the roundings of the
// large products g_j u and (1 - g_j) w_j would repeat from step to step and grow linearly
// with range.
//
// One workgroup owns one solve for a whole launch: the Neumann series of every Pade factor
// runs on chip (transforms in registers + LDS); the state between factors stays in
// registers where the layout has room, else in the solve's work array, and the field is
// written once per step (the recovery point if the next step diverges).  Tables the
// kernels read every term (multipliers, potential, chirp spectra) come from L2 where they
// do not fit the registers.  Precision: complex FP32
// data; FFT twiddles and the sine-space multipliers are double-float (hi + lo) products so
// that no fixed rounding of a table enters every step on the isovelocity path; residual
// norms in FP64; carrier phase in FP64.
#include "ssp_device.h"
#include "ssp_df.h"
#include "ssp_tuned.h"

#include <math.h>

#include <mutex>

namespace ssp {
namespace {

constexpr int kOK = 0, kNotConverged = 1, kDiverged = -4;


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
// element v + s with s uniform over the workgroup (the constant or uniform part goes to the
// scalar offset of the access)
__device__ __forceinline__ float2 ld2s(const float2 *p, int v, int s) {
    auto r = __builtin_amdgcn_raw_buffer_load_b64(rsrc(p), v * 8, s * 8, 0);
    return make_float2(__uint_as_float(r[0]), __uint_as_float(r[1]));
}
__device__ __forceinline__ float4 ld4(const float4 *p, int i) {
    auto v = __builtin_amdgcn_raw_buffer_load_b128(rsrc(p), i * 16, 0, 0);
    return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]),
                       __uint_as_float(v[3]));
}
__device__ __forceinline__ uint32_t ldu(const uint32_t *p, int i) {
    return __builtin_amdgcn_raw_buffer_load_b32(rsrc(p), i * 4, 0, 0);
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
// cos(2 pi i/32), i = 0..31
__device__ constexpr double kCos32[32] = {
    1.0, 9.80785280403230449126e-1, 9.23879532511286756128e-1, 8.31469612302545237079e-1,
    7.07106781186547524401e-1, 5.55570233019602224743e-1, 3.82683432365089771728e-1, 1.95090322016128267848e-1,
    0.0, -1.95090322016128267848e-1, -3.82683432365089771728e-1, -5.55570233019602224743e-1,
    -7.07106781186547524401e-1, -8.31469612302545237079e-1, -9.23879532511286756128e-1, -9.80785280403230449126e-1,
    -1.0, -9.80785280403230449126e-1, -9.23879532511286756128e-1, -8.31469612302545237079e-1,
    -7.07106781186547524401e-1, -5.55570233019602224743e-1, -3.82683432365089771728e-1, -1.95090322016128267848e-1,
    0.0, 1.95090322016128267848e-1, 3.82683432365089771728e-1, 5.55570233019602224743e-1,
    7.07106781186547524401e-1, 8.31469612302545237079e-1, 9.23879532511286756128e-1, 9.80785280403230449126e-1};

// x * exp(-+ 2 pi i k / R) (minus for the forward transform), R <= 32
template <int R, bool INV>
__device__ __forceinline__ float2 mulw(float2 x, int k) {
    static_assert(R <= 32 && 32 % R == 0, "radix must divide 32");
    const int i32 = (k * (32 / R)) & 31;
    if (i32 == 0) return x;
    if (i32 == 16) return make_float2(-x.x, -x.y);
    if (i32 == 8) return INV ? make_float2(-x.y, x.x) : make_float2(x.y, -x.x);
    if (i32 == 24) return INV ? make_float2(x.y, -x.x) : make_float2(-x.y, x.x);
    const double c = kCos32[i32], s = kCos32[(i32 + 24) & 31];
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

// DFT of x[0..R) whose upper half x[R/2..R) is zero (never read): decimation in frequency,
// X_{2k} = DFT_{R/2}(x)_k and X_{2k+1} = DFT_{R/2}(x_i w_R^i)_k, natural order out.
template <int R, bool INV>
struct DftHalfIn {
    __device__ __forceinline__ static void run(float2 *x) {
        float2 e[R / 2], o[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            e[i] = x[i];
            o[i] = mulw<R, INV>(x[i], i);
        }
        Dft<R / 2, INV>::run(e);
        Dft<R / 2, INV>::run(o);
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
            x[2 * k] = e[k];
            x[2 * k + 1] = o[k];
        }
    }
};

// DFT of x[0..R) of which only X[0..R/2) is needed (the upper half is set to zero):
// decimation in time without the subtraction half of the last stage.
template <int R, bool INV>
struct DftHalfOut {
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
            x[k] = cadd(e[k], mulw<R, INV>(o[k], k));
            x[k + R / 2] = make_float2(0.f, 0.f);
        }
    }
};

// Thread index laundered through an empty asm: index arithmetic derived from it is
// recomputed where it is used instead of being hoisted out of the range-step loops, which
// would keep dozens of loop-invariant addresses alive in vector registers.
__device__ __forceinline__ int opaque_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// ----------------------------------------------------------------------------- FFT engine
// One workgroup computes a P-point complex FFT (P a power of two).  Thread t owns the RT =
// P/T elements at positions t + i T (i < RT) in registers.  The first pass (radix RT, no
// twiddles) reads exactly those positions and the last pass (radix RT, stride T) produces
// exactly those positions, so a transform goes registers -> LDS -> ... -> registers; the
// middle passes are self-sorting (Stockham) radix passes through LDS:
//   butterfly j (k = j mod Ns) reads positions j + r P/R, multiplies by w_{Ns R}^{r k},
//   takes the R-point DFT and writes positions (j - k) R + k + r Ns.
// Because T is a multiple of every middle stride Ns, a thread's k is t mod Ns in every
// pass, so its twiddles are the same in every transform of a launch: they are computed
// once per launch and held in registers (double-float: FP32 value + bf16 pair remainder).
// LDS: each exchange has its own padding (see lps); two data buffers when they fit (one
// barrier per exchange), else one.  Every padded index of a pass is a per-thread base plus
// a compile-time offset (the offsets that are added are multiples of the padding period,
// or keep within one period), so exchanges cost no index arithmetic beyond one base per
// pass.
// Engine configurations.  A template argument K names one: the FFT length (low bits) and a
// variant (high bits) that selects the thread count, i.e. the radix of the first and last
// passes (elements per thread).  Variant 0 is the default layout; variant 1 exists where a
// second layout fits the register and LDS budgets, and the autotuner picks per length.
constexpr int kVarShift = 20;
constexpr int kSplitKey = 1 << 28;  // the engine serves a split transform (two halves)
constexpr int key_len(int K) { return K & ((1 << kVarShift) - 1); }
constexpr int key_var(int K) { return (K >> kVarShift) & 0xff; }
constexpr bool key_split(int K) { return (K & kSplitKey) != 0; }
constexpr int threads_v0(int P) { return P <= 512 ? 64 : (P == 1024 ? 128 : (P <= 4096 ? 256 : 1024)); }
constexpr int threads_v1(int P) {
    return P == 1024 ? 64 : (P == 2048 ? 128 : (P == 4096 ? 512 : (P == 8192 ? 512 : threads_v0(P))));
}
// variant 2: 32 elements per thread with a single LDS buffer, so that two workgroups share
// a compute unit and cover each other's barriers (at 16384 one workgroup of 512 threads,
// one FFT pass fewer than variant 0)
constexpr int threads_v2(int P) {
    return P == 4096 ? 128 : (P == 8192 ? 256 : (P == 16384 ? 512 : threads_v0(P)));
}
constexpr int threads_for(int P, int V) {
    return V == 2 ? threads_v2(P) : (V == 1 ? threads_v1(P) : threads_v0(P));
}
constexpr bool variant_exists(int P, int V) {
    return V == 0 || (V == 1 && threads_v1(P) != threads_v0(P)) || (V == 2 && threads_v2(P) != threads_v0(P));
}
constexpr bool has_variant(int P) { return variant_exists(P, 1) || variant_exists(P, 2); }

template <int K>
struct Cfg {
    static constexpr int P = key_len(K);
    static constexpr int T = threads_for(P, key_var(K));
    static constexpr int RT = P / T;
    static constexpr int DLEN = P + (P >> 4);  // room for the densest padding (1 per 16)
    static constexpr int O = P / 8;
    static constexpr int LOG2O = __builtin_ctz(P / 8);
    static constexpr bool SINGLE = key_var(K) == 2;  // one data buffer, two workgroups per CU
    static constexpr bool PINGPONG = !SINGLE && (2 * DLEN * 8 + 16 * T + 1024) <= 160 * 1024;
    static constexpr int MINW = SINGLE ? 2 : 1;       // waves per SIMD the kernel must allow
};

// Padded LDS index with one slot per 2^SH elements (SH = 0: none), and the same at compile
// time.  Each exchange (a pass's writes and the next pass's reads) has its own padding,
// chosen by the writer so that both access patterns spread over the 64 banks: the first
// pass writes RT consecutive elements per thread (one slot per 32), a middle pass at stride
// Ns < 16 writes R-strided groups (one per 16); later middle passes and the combine write
// unit-stride runs, which padding would only shift across the bank boundary (none).
template <int SH>
__device__ __forceinline__ int lps(int i) { return SH ? i + (i >> SH) : i; }
constexpr int lpcs(int SH, int v) { return SH ? v + (v >> SH) : v; }
constexpr int kShFirst = 5;
constexpr int mid_shift(int Ns) { return Ns < 16 ? 4 : 0; }

// radix of the middle pass at stride Ns
template <int P, int Ns>
constexpr int mid_radix() {
    return (Cfg<P>::T / Ns) < Cfg<P>::RT ? (Cfg<P>::T / Ns) : Cfg<P>::RT;
}
template <int P, int Ns>
constexpr int mid_count_from() {
    if constexpr (Ns >= Cfg<P>::T) {
        return 0;
    } else {
        return 1 + mid_count_from<P, Ns * mid_radix<P, Ns>()>();
    }
}
template <int P>
constexpr int fft_phases() { return 1 + mid_count_from<P, Cfg<P>::RT>(); }

// entries of the middle-pass twiddle table from stride Ns on: Ns (R - 1) per pass
template <int P, int Ns>
constexpr int mid_tab_from() {
    if constexpr (Ns >= Cfg<P>::T) {
        return 0;
    } else {
        constexpr int R = mid_radix<P, Ns>();
        return Ns * (R - 1) + mid_tab_from<P, Ns * R>();
    }
}
template <int P>
constexpr int mid_tab_len() { return mid_tab_from<P, Cfg<P>::RT>(); }
template <int P, int Ns>
constexpr int mid_tab_offset() { return mid_tab_len<P>() - mid_tab_from<P, Ns>(); }

// Twiddles of the last pass (w_P^{r t}, r = 1..RT-1): per thread, held in registers, except
// where registers are short: the engine of split transforms (1024 threads, 128 registers
// per lane, which the second half's state leaves short) and the layout-2 engines (31
// twiddles per thread, 93 registers) read them from a device table ([r-1][t], coalesced,
// shared by every workgroup, so it stays in L2).  The split engine loads them before the
// barrier that precedes their use in layout 0; layout 2 (also of split transforms) at their
// use (the other workgroup on the compute unit covers the latency).  (The unsplit
// 1024-thread engines measured faster with register twiddles and a few spills.)
template <int P>
struct Twiddles {
    static constexpr bool kRegs = !key_split(P) && key_var(P) != 2;
    static constexpr bool kPrefetch = key_split(P) && key_var(P) != 2;  // table twiddles loaded ahead of the barrier
    static constexpr int NTW = kRegs ? Cfg<P>::RT - 1 : 1;
    float2 h[NTW];   // FP32 nearest value
    uint32_t l[NTW]; // remainder as two bf16 (re high, im low)
    const float4 *tab;
};

// w_P^e (forward sign), e in [0, P), from the first-octant table in global memory:
// entry e' = e mod P/8 (mirrored for odd octants), rotated by (-i)^q.
template <int P>
__device__ __forceinline__ void fetch_twiddle(const uint32_t *tab, int e, float2 &h, uint32_t &l) {
    constexpr int O = Cfg<P>::O;
    const int o = e >> Cfg<P>::LOG2O, r = e & (O - 1);
    const bool odd = o & 1;
    const int idx = odd ? O - r : r;
    float hr = __uint_as_float(ldu(tab, 3 * idx)), hi = __uint_as_float(ldu(tab, 3 * idx + 1));
    const uint32_t pk = ldu(tab, 3 * idx + 2);
    float lr = __uint_as_float(pk & 0xffff0000u), li = __uint_as_float(pk << 16);
    if (odd) {
        hi = -hi;
        li = -li;
    }
    const int q = ((o + (odd ? 1 : 0)) >> 1) & 3;
    float a = hr, b = hi, c = lr, dd = li;
    if (q == 1) { a = hi; b = -hr; c = li; dd = -lr; }
    else if (q == 2) { a = -hr; b = -hi; c = -lr; dd = -li; }
    else if (q == 3) { a = -hi; b = hr; c = -li; dd = lr; }
    h = make_float2(a, b);
    // c and dd are exact bfloat16 values: repack them
    l = (__float_as_uint(c) & 0xffff0000u) | (__float_as_uint(dd) >> 16);
}

// Middle-pass table in LDS: pass at stride Ns holds w_{Ns R}^{r k} at
// offset(Ns) + (r - 1) Ns + k, so lanes with consecutive k read consecutive entries.
template <int P, int Ns>
__device__ __forceinline__ void init_mid_table(float4 *t4, const uint32_t *tab) {
    if constexpr (Ns < Cfg<P>::T) {
        constexpr int R = mid_radix<P, Ns>();
        constexpr int OFF = mid_tab_offset<P, Ns>();
        constexpr int STRIDE = Cfg<P>::P / (Ns * R);
        for (int idx = threadIdx.x; idx < Ns * (R - 1); idx += Cfg<P>::T) {
            const int r = idx / Ns + 1, k = idx & (Ns - 1);
            float2 h;
            uint32_t l;
            fetch_twiddle<P>(tab, r * k * STRIDE, h, l);
            t4[OFF + idx] = make_float4(h.x, h.y, __uint_as_float(l & 0xffff0000u), __uint_as_float(l << 16));
        }
        init_mid_table<P, Ns * R>(t4, tab);
    }
}

// All twiddles of a launch: the middle-pass table (LDS, ends with a barrier) and the
// thread's last-pass twiddles (registers).
template <int P>
__device__ __forceinline__ void init_twiddles(Twiddles<P> &tw, float4 *t4, const uint32_t *tab,
                                              const float4 *last) {
    const int tid = threadIdx.x;
    if constexpr (Twiddles<P>::kRegs) {
#pragma unroll
        for (int r = 1; r < Cfg<P>::RT; ++r) fetch_twiddle<P>(tab, r * tid, tw.h[r - 1], tw.l[r - 1]);
        tw.tab = nullptr;
    } else {
        tw.tab = last;
    }
    init_mid_table<P, Cfg<P>::RT>(t4, tab);
    __syncthreads();
}

template <bool INV>
__device__ __forceinline__ float2 twmul(float2 x, float2 h, uint32_t l) {
    const float4 w = make_float4(h.x, h.y, __uint_as_float(l & 0xffff0000u), __uint_as_float(l << 16));
    return INV ? cmul_df_conj(x, w) : cmul_df(x, w);
}

// LDS data buffers of one transform.  Exchange phase k (a write, a barrier, then reads)
// uses buffer k mod 2 (buffer 0 only when two do not fit), chosen at compile time.
struct LdsBufs {
    float2 *b0, *b1;
    float4 *tw4;  // middle-pass twiddle table: hi.re, hi.im, lo.re, lo.im
};

template <int P, int PH>
__device__ __forceinline__ float2 *phase_buf(const LdsBufs &L) {
    return (Cfg<P>::PINGPONG && (PH & 1)) ? L.b1 : L.b0;
}
// with a single buffer every thread must be done reading before anyone writes
template <int P>
__device__ __forceinline__ void before_write() {
    if constexpr (!Cfg<P>::PINGPONG) __syncthreads();
}

// middle passes: read phase PH (padding SHR), write phase PH + 1 (padding mid_shift(Ns));
// Ns = current stride until it reaches T
template <int P>
constexpr int last_tab_regs() { return Twiddles<P>::kPrefetch ? Cfg<P>::RT - 1 : 1; }
template <int P, bool INV, int Ns, int PH, int SHR>
__device__ __forceinline__ void mid_passes(float2 (&x)[Cfg<P>::RT], const LdsBufs &L,
                                           const Twiddles<P> &tw, float4 (&wl)[last_tab_regs<P>()]) {
    constexpr int T = Cfg<P>::T, RT = Cfg<P>::RT;
    if constexpr (Ns < T) {
        constexpr int R = mid_radix<P, Ns>();
        constexpr int PER = RT / R;
        constexpr int NB = Cfg<P>::P / R;
        constexpr int OFF = mid_tab_offset<P, Ns>();
        constexpr int SHW = mid_shift(Ns);
        constexpr int QR = 1 << SHR, QW = 1 << SHW;
        // constant-offset addressing applies when every added offset keeps the padding
        // count exact (see the engine notes); otherwise the index is padded per access
        constexpr bool FAST_R = SHR == 0 || ((T % QR == 0) && (NB % QR == 0));
        constexpr bool FAST_W = SHW == 0 || (((T * R) % QW == 0) &&
                                             ((Ns % QW == 0) || (QW % Ns == 0 && (Ns * R) % QW == 0)));
        const int tid = opaque_tid();
        const float2 *in = phase_buf<P, PH>(L);
        if constexpr (FAST_R) {
            const float2 *rb = in + lps<SHR>(tid);
#pragma unroll
            for (int i = 0; i < PER; ++i)
#pragma unroll
                for (int r = 0; r < R; ++r) x[i * R + r] = rb[i * lpcs(SHR, T) + r * lpcs(SHR, NB)];
        } else {
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int j = tid + i * T;
#pragma unroll
                for (int r = 0; r < R; ++r) x[i * R + r] = in[lps<SHR>(j + r * NB)];
            }
        }
        before_write<P>();
        float2 *out = phase_buf<P, PH + 1>(L);
        const int t2 = opaque_tid();
        const int k = t2 & (Ns - 1);  // T is a multiple of Ns: the same k for every i
        const float4 *wt = L.tw4 + OFF + k;
        float2 *wb = out + lps<SHW>((t2 - k) * R + k);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            float2 *v = &x[i * R];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const float4 w = wt[(r - 1) * Ns];
                v[r] = INV ? cmul_df_conj(v[r], w) : cmul_df(v[r], w);
            }
            Dft<R, INV>::run(v);
            if constexpr (FAST_W) {
#pragma unroll
                for (int r = 0; r < R; ++r) wb[i * lpcs(SHW, T * R) + lpcs(SHW, r * Ns)] = v[r];
            } else {
                const int base = (t2 + i * T - k) * R + k;
#pragma unroll
                for (int r = 0; r < R; ++r) out[lps<SHW>(base + r * Ns)] = v[r];
            }
        }
        if constexpr (Twiddles<P>::kPrefetch && Ns * R >= T) {
            // the last pass's table twiddles, loaded before its barrier so that their latency
            // overlaps the wait
            const int t3 = opaque_tid();
#pragma unroll
            for (int r = 1; r < RT; ++r) wl[r - 1] = ld4(tw.tab, (r - 1) * T + t3);
        }
        __syncthreads();
        mid_passes<P, INV, Ns * R, PH + 1, SHW>(x, L, tw, wl);
    }
}

// padding of the exchange the last pass reads (written by the last middle pass, or by the
// first pass when there is none)
template <int P, int Ns, int SH>
constexpr int last_shift_from() {
    if constexpr (Ns >= Cfg<P>::T) {
        return SH;
    } else {
        return last_shift_from<P, Ns * mid_radix<P, Ns>(), mid_shift(Ns)>();
    }
}

// Full FFT of the distributed vector x (registers in, registers out); its first exchange
// uses phase PH.  HALF_IN: positions >= P/2 of the input are zero (the thread's upper half);
// HALF_OUT: only positions < P/2 of the output are needed (the upper half is returned zero).
template <int P, bool INV, int PH, bool HALF_IN = false, bool HALF_OUT = false>
__device__ __forceinline__ void fft(float2 (&x)[Cfg<P>::RT], const LdsBufs &L, const Twiddles<P> &tw) {
    constexpr int T = Cfg<P>::T, RT = Cfg<P>::RT;
    const int tid = opaque_tid();
    // first pass: Ns = 1, butterfly j = t on positions t + r T
    if constexpr (HALF_IN && RT >= 2) DftHalfIn<RT, INV>::run(x);
    else Dft<RT, INV>::run(x);
    before_write<P>();
    {
        // tid RT + r stays within one 32-block of the padded index (RT divides 32)
        static_assert(32 % RT == 0, "first-pass radix must divide 32");
        float2 *out = phase_buf<P, PH>(L) + lps<kShFirst>(tid * RT);
#pragma unroll
        for (int r = 0; r < RT; ++r) out[r] = x[r];
    }
    __syncthreads();
    static_assert(Twiddles<P>::kRegs || RT < T, "table twiddles are loaded by the last middle pass");
    float4 wl[last_tab_regs<P>()];
    mid_passes<P, INV, RT, PH, kShFirst>(x, L, tw, wl);
    // last pass: Ns = T, butterfly j = t, twiddles w_P^{r t}, outputs at t + r T
    {
        constexpr int SHL = last_shift_from<P, RT, kShFirst>();
        const float2 *in = phase_buf<P, PH + fft_phases<P>() - 1>(L) + lps<SHL>(opaque_tid());
#pragma unroll
        for (int r = 0; r < RT; ++r) x[r] = in[r * lpcs(SHL, T)];
        if constexpr (Twiddles<P>::kRegs) {
#pragma unroll
            for (int r = 1; r < RT; ++r) x[r] = twmul<INV>(x[r], tw.h[r - 1], tw.l[r - 1]);
        } else if constexpr (Twiddles<P>::kPrefetch) {
#pragma unroll
            for (int r = 1; r < RT; ++r) x[r] = INV ? cmul_df_conj(x[r], wl[r - 1]) : cmul_df(x[r], wl[r - 1]);
        } else {
            const int t3 = opaque_tid();
#pragma unroll
            for (int r = 1; r < RT; ++r) {
                const float4 w = ld4(tw.tab, (r - 1) * T + t3);
                x[r] = INV ? cmul_df_conj(x[r], w) : cmul_df(x[r], w);
            }
        }
        if constexpr (HALF_OUT && RT >= 2) DftHalfOut<RT, INV>::run(x);
        else Dft<RT, INV>::run(x);
    }
}

// Z_q = Y_q K1_q - Y_{-q} K2_q for the distributed spectrum (one LDS exchange, phase PH).
// ODD: the odd-frequency half of a split transform, whose reflection is q -> P-1-q.
// Unsplit lengths read both spectra.  A split half derives K2 from K1 (the Hankel spectra of
// the many plans of a batch do not stay in the L2, and every spectrum value read there costs
// fabric traffic): K2_q = phi w^{s q} K1_{q + L/2} (L the convolution length, w = exp(-2 pi
// i/L); see KWin), and spectrum position q + L/2 (same parity as q) is the thread's own
// element i + RT/2, so each K1 value read serves two elements.  The phase of element i is the
// thread's base phase (the product of two double-float entries of the phase table, rounded
// once) times the double-float step w^{s 2T i} from the descriptor; element i + RT/2 takes
// sign (-1)^s times that phase.  No FP32 rounding is shared by many spectrum positions.
template <int P, int PH, bool ODD>
__device__ __forceinline__ void chirp_combine(float2 (&x)[Cfg<P>::RT], const LdsBufs &L, KWin k) {
    constexpr int T = Cfg<P>::T, RT = Cfg<P>::RT, H2 = RT / 2;
    constexpr bool SPLIT = key_split(P);
    static_assert(!SPLIT || (RT % 2 == 0 && H2 <= 16 && (2 * T) % 64 == 0), "element pairs, phase steps");
    const int tid = opaque_tid();
    float2 base = make_float2(0.f, 0.f);
    if constexpr (SPLIT) {
        // phase of element 0 (frequency 2 tid + ODD), read before the exchange
        const int q0 = 2 * tid + (ODD ? 1 : 0);
        const float4 a = ld4(k.kph, q0 & 63), b = ld4(k.kph, 64 + (q0 >> 6));
        // (a.hi + a.lo)(b.hi + b.lo) without the lo * lo term
        base = cadd(cmul_df(make_float2(a.x, a.y), b), cmul(make_float2(a.z, a.w), make_float2(b.x, b.y)));
    }
    // split halves: the K1 values of the first NPRE element pairs are requested before the
    // exchange, so that their latency (the spectra of many plans come from beyond the L2)
    // overlaps it (4 pairs measured 2% faster than none and than 8)
    constexpr int NPRE = SPLIT ? 4 : 0;
    float2 kpre[2 * NPRE + 1];
#pragma unroll
    for (int i = 0; i < NPRE; ++i) {
        kpre[2 * i] = ld2s(k.k1, tid, i * T);
        kpre[2 * i + 1] = ld2s(k.k1, tid, (i + H2) * T);
    }
    before_write<P>();
    float2 *buf = phase_buf<P, PH>(L);
    // unit-stride exchange: no padding
    {
        float2 *wb = buf + tid;
#pragma unroll
        for (int i = 0; i < RT; ++i) wb[i * T] = x[i];
    }
    __syncthreads();
    const int t2 = opaque_tid();
    // reflected position of q = t2 + i T:  even: -q mod P = u + (RT - 1 - i + c) T with
    // u = -t2 mod T, c = (t2 == 0) (position 0 itself for i = 0, c = 1);
    // odd: P - 1 - q = (T - 1 - t2) + (RT - 1 - i) T
    const int u = ODD ? (T - 1 - t2) : ((T - t2) & (T - 1));
    const int c = ODD ? 0 : (t2 == 0 ? 1 : 0);
    const float2 *rb = buf + u + c * T;
    auto refl = [&](int i) -> float2 {
        if (!ODD && i == 0) return c ? buf[0] : rb[(RT - 1) * T];
        return rb[(RT - 1 - i) * T];
    };
    if constexpr (SPLIT) {
#pragma unroll
        for (int i = 0; i < H2; ++i) {
            const float2 ph = i == 0 ? base : cmul_df(base, k.hs[i]);
            const float2 phb = make_float2(k.sg * ph.x, k.sg * ph.y);
            const float2 ka = i < NPRE ? kpre[2 * i] : ld2s(k.k1, t2, i * T);
            const float2 kb = i < NPRE ? kpre[2 * i + 1] : ld2s(k.k1, t2, (i + H2) * T);
            const float2 ya = refl(i), yb = refl(i + H2);
            x[i] = csub(cmul(x[i], ka), cmul(ya, cmul(ph, kb)));
            x[i + H2] = csub(cmul(x[i + H2], kb), cmul(yb, cmul(phb, ka)));
        }
    } else {
#pragma unroll
        for (int i = 0; i < RT; ++i)
            x[i] = csub(cmul(x[i], ld2s(k.k1, t2, i * T)), cmul(refl(i), ld2s(k.k2, t2, i * T)));
    }
}

// The chirp-z core of one DST on P positions: x <- IFFT(comb(FFT(x))) (unnormalised), x
// distributed by position; positions >= N must hold zeros on entry.  Phases 0 .. 2F
// (F = passes - 1); the opening barrier separates them from the previous core's last reads.
// HALF: the vector length N is at most P/2 (every unsplit length), so the input's upper
// half is zero and the output's upper half is not needed; it is returned zero.
template <int P, bool ODD, bool HALF = false>
__device__ __forceinline__ void chirp_core(float2 (&x)[Cfg<P>::RT], const LdsBufs &L,
                                           const Twiddles<P> &tw, KWin k) {
    constexpr int F = fft_phases<P>();
    __syncthreads();
    fft<P, false, 0, HALF, false>(x, L, tw);
    chirp_combine<P, F, ODD>(x, L, k);
    fft<P, true, F + 1, false, HALF>(x, L, tw);
}

// Largest FFT held by one workgroup, and the engine (length and variant) of a convolution
// length P.
constexpr int kMaxEngine = 16384;
template <int P>
constexpr int eng_len() { return P > kMaxEngine ? P / 2 : P; }
template <int P, int V>
constexpr int eng_key() {
    return eng_len<P>() | ((variant_exists(eng_len<P>(), V) ? V : 0) << kVarShift) |
           (P > kMaxEngine ? kSplitKey : 0);
}
template <int P, int V>
using ECfg = Cfg<eng_key<P, V>()>;

// Elements i of a thread that can hold data of a vector of length N <= P/2: all for split
// lengths, the lower half otherwise (positions t + i T >= P/2 are always beyond N).
template <int P, int V>
constexpr int live_elems() { return eng_len<P>() == P ? ECfg<P, V>::RT / 2 : ECfg<P, V>::RT; }
// ... and for the direct transform of a periodic grid of P points, all of them.  DK is the
// plan's transform kind: 0 chirp-z, 1 direct Fourier (periodic Nz = P), 2 direct sine
// (Dirichlet Nz = P/2 - 1, lower half live as for chirp-z).
constexpr int kDkChirp = 0, kDkFourier = 1, kDkSine = 2;
template <int P, int V, int DK>
constexpr int live_of() { return DK == kDkFourier ? ECfg<P, V>::RT : live_elems<P, V>(); }

// The transform of a periodic plan whose grid length is itself an engine length: the
// forward FFT (grid -> coefficients) or the unnormalised inverse FFT of the P points in
// registers, natural order in and out; the 1/sqrt(P) factors sit in the plan's modulation
// tables.  The opening barrier separates it from the previous transform's LDS reads.
template <int EK>
__device__ __forceinline__ void direct_core(float2 (&x)[Cfg<EK>::RT], const LdsBufs &L,
                                            const Twiddles<EK> &tw, bool fwd) {
    __syncthreads();
    if (fwd) fft<EK, false, 0>(x, L, tw);
    else fft<EK, true, 0>(x, L, tw);
}

// The orthonormal DST-I of a Dirichlet grid of N = P/2 - 1 points as the FFT of its odd
// extension of length P (its own inverse).  On entry the thread holds the pre-modulated
// values at its positions below P/2 (element n at position n - 1, zeros from position N
// on); their odd images, times the plan's mirror factors, go through LDS to positions
// P - 2 - m, position P - 1 is zero, and the full FFT returns the lower half of its output
// (the upper half returned zero).  The opening barrier separates the image writes from the
// previous transform's LDS reads; with two buffers the images use the one the FFT's first
// exchange does not, with one the FFT's own write barrier follows the image reads.
template <int EK>
__device__ __forceinline__ void sine_core(float2 (&x)[Cfg<EK>::RT], const LdsBufs &L,
                                          const Twiddles<EK> &tw, const float4 *mirror, int N) {
    constexpr int P = Cfg<EK>::P, T = Cfg<EK>::T, RT = Cfg<EK>::RT;
    __syncthreads();
    float2 *mb = phase_buf<EK, 1>(L);
    const int tid = opaque_tid();
#pragma unroll
    for (int i = 0; i < RT / 2; ++i) {
        const int pos = tid + i * T;
        if (pos < N) mb[P - 2 - pos] = cmul_df(x[i], ld4(mirror, pos));
    }
    if (tid == T - 1) mb[P - 1] = make_float2(0.f, 0.f);
    __syncthreads();
#pragma unroll
    for (int i = RT / 2; i < RT; ++i) x[i] = mb[tid + i * T];
    fft<EK, false, 0, false, true>(x, L, tw);
}

// One transform core for convolution length P (positions 0 .. eng_len-1 distributed as in
// the engine), with the chirp-window spectra k of the direction it runs in.  For P above
// kMaxEngine the odd-frequency half needs the input again after the even half has
// overwritten x: KEEP_GLOBAL keeps it (and the even result) in the solve's scratch
// keep[0 .. 2H) (H = P/2 positions per half), else in registers.  Both give identical
// results.  Positions >= N of the input must be zero.  Output: split lengths return zero at
// positions >= N; unsplit lengths return zero at positions >= P/2 and values without meaning
// in [N, P/2).
template <int P, int V, bool KEEP_GLOBAL, int EKEY = eng_key<P, V>()>
__device__ __forceinline__ void dst_core(float2 (&x)[Cfg<EKEY>::RT], const LdsBufs &L,
                                         const Twiddles<EKEY> &tw, const SolveDesc &d, float2 *keep,
                                         KWin k) {
    constexpr int H = eng_len<P>();
    constexpr int EK = eng_key<P, V>();
    k.hs = V == 0 ? d.hstep0 : d.hstep;  // (split lengths)
    if constexpr (H == P) {
        chirp_core<EK, false, true>(x, L, tw, k);
    } else {
        constexpr int T = Cfg<EK>::T, RT = Cfg<EK>::RT;
        // odd-frequency input y = x (.) w_P^n: for n = t + i T, w_P^n = w_P^{t + (i mod NW) T}
        // w_Q^{i / NW} with Q = P/(NW T) <= 32: NW table values per thread (the table holds
        // w_P^n for n < P/2) and a double-float radix-Q constant
        constexpr int NW = (P / T) > 32 ? (P / T) / 32 : 1, Q = P / (NW * T);
        static_assert(Q <= 32 && 32 % Q == 0 && NW * T <= P / 2, "twist factor w_Q^i is a radix constant");
        const int N = d.N;
        float2 y[KEEP_GLOBAL ? 1 : RT];
        float4 wt[NW];
#pragma unroll
        for (int k2 = 0; k2 < NW; ++k2) wt[k2] = ld4(d.twist, opaque_tid() + k2 * T);
        // (the keep scratch is two halves of H positions, one per thread position t + i T:
        // its accesses need no bounds test, and positions >= N carry zeros or unused values)
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            const int pos = opaque_tid() + i * T;
            const float2 tv = mulw<Q, false>(cmul_df(x[i], wt[i % NW]), i / NW);
            const float2 v = pos < N ? tv : make_float2(0.f, 0.f);
            if constexpr (KEEP_GLOBAL) {
                st2(keep, pos, v);
            } else {
                y[i] = v;
            }
        }
        chirp_core<EK, false>(x, L, tw, k);
        if constexpr (KEEP_GLOBAL) {
#pragma unroll
            for (int i = 0; i < RT; ++i) {
                const int pos = opaque_tid() + i * T;
                st2(keep + H, pos, x[i]);
                x[i] = ld2(keep, pos);  // zero at positions >= N
            }
            chirp_core<EK, true>(x, L, tw, KWin{k.k1 + H, nullptr, k.kph, k.sg, k.hs});
#pragma unroll
            for (int i = 0; i < RT; ++i) {
                const int pos = opaque_tid() + i * T;
                const float2 e = ld2(keep + H, pos);
                const float2 z = cadd(e, mulw<Q, true>(cmul_df_conj(x[i], wt[i % NW]), i / NW));
                x[i] = pos < N ? z : make_float2(0.f, 0.f);
            }
        } else {
            chirp_core<EK, true>(y, L, tw, KWin{k.k1 + H, nullptr, k.kph, k.sg, k.hs});
#pragma unroll
            for (int i = 0; i < RT; ++i) {
                const int pos = opaque_tid() + i * T;
                x[i] = pos < N ? cadd(x[i], mulw<Q, true>(cmul_df_conj(y[i], wt[i % NW]), i / NW))
                               : make_float2(0.f, 0.f);
            }
        }
    }
}

// LDS of one workgroup for engine length PE, carved from one array: the data buffer(s),
// then the middle-pass twiddle table (FP32 values, then the bf16 remainders).
template <int PE>
constexpr int lds_words() {  // in float4 units (16-byte aligned storage)
    return ((Cfg<PE>::PINGPONG ? 2 : 1) * Cfg<PE>::DLEN + 1) / 2 + mid_tab_len<PE>() + 1;
}
template <int PE>
__device__ __forceinline__ LdsBufs carve_lds(float4 *raw4) {
    float2 *raw = reinterpret_cast<float2 *>(raw4);
    constexpr int NB = (Cfg<PE>::PINGPONG ? 2 : 1) * Cfg<PE>::DLEN;
    return LdsBufs{raw, Cfg<PE>::PINGPONG ? raw + Cfg<PE>::DLEN : raw, raw4 + (NB + 1) / 2};
}
#define SSP_LDS_DECL(PE)                          \
    __shared__ float4 lds_raw[lds_words<PE>()];   \
    const LdsBufs L = carve_lds<PE>(lds_raw)

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

// Eddy correction of the potential in the analytic environment.  The range-independent
// Munk part v_m = (c0/c_m)^2 - 1 comes from the FP64 host table (row 0 of d.v); with
// e = dc/c_m the full potential is v = (c0/(c_m + dc))^2 - 1 = v_m + (1 + v_m) (-e (2 + e)/(1 + e)^2),
// a small correction that FP32 evaluates to the precision of the stored table.
__device__ __forceinline__ float eddy_correction(const SolveDesc &d, float vm, float z, float r) {
    if (d.env[3] == 0.0) return 0.f;
    const float xr = (r - static_cast<float>(d.env[4])) / static_cast<float>(d.env[5]);
    const float xz = (z - static_cast<float>(d.env[6])) / static_cast<float>(d.env[7]);
    const float dc = -static_cast<float>(d.env[3]) * expf(-(xr * xr) - (xz * xz));
    const float q = 1.0f + vm;                                // (c0/c_m)^2
    const float cm = static_cast<float>(d.c0) * rsqrtf(q);    // c_m
    const float e = dc / cm;
    return q * (-e * (2.0f + e) / ((1.0f + e) * (1.0f + e)));
}

// A = v (.) dmod at the thread's positions (zero at positions >= N); v of global step n,
// plus i eta when the plan has an absorbing layer (complex absorbing potential).
// Written to registers (A) when the kernel keeps it there, else to the solve's pot array.
template <int P, int V, bool IN_REGS, int DK = kDkChirp>
__device__ __forceinline__ void load_potential(const SolveDesc &d, long long n, float2 *A) {
    constexpr int T = ECfg<P, V>::T, RL = live_of<P, V, DK>();
    const int N = d.N;
    long long row = 0;
    if (d.prof_mode == PROF_TABLE_STEPS) {
        row = n - d.v_step0 - 1;
        row = row < 0 ? 0 : (row >= d.v_rows ? d.v_rows - 1 : row);
    }
    const float *vrow = d.v + row * N;
    const float r = static_cast<float>((static_cast<double>(n) - 0.5) * d.dr);
#pragma unroll
    for (int i = 0; i < RL; ++i) {
        const int pos = opaque_tid() + i * T, m = pos;
        float2 val = make_float2(0.f, 0.f);
        if (pos < N) {
            float v = ldf(vrow, m);
            if (d.prof_mode == PROF_ANALYTIC)
                v += eddy_correction(d, v, static_cast<float>((pos + d.zoff) * d.dz), r);
            const float2 dm = ld2(d.dmod, m);
            if (d.vi) val = cmul(make_float2(v, ldf(d.vi, m)), dm);
            else val = make_float2(v * dm.x, v * dm.y);
            if constexpr (!IN_REGS) st2(d.pot, m, val);
        }
        if constexpr (IN_REGS) A[i] = val;
    }
}

// ----------------------------------------------------------------------------- march
// One workgroup marches one solve through nsteps range steps.
template <int P, int V, int DK = kDkChirp>
__device__ __forceinline__ void march_body(const SolveDesc &d, int nsteps, float4 *lds_raw, double *red) {
    constexpr int T = ECfg<P, V>::T, RT = ECfg<P, V>::RT;
    constexpr int EK = eng_key<P, V>();
    // elements that can hold data (the lower half for unsplit chirp-z lengths, all for the
    // direct transform); the others stay zero
    constexpr int RL = live_of<P, V, DK>();
    // the Neumann multiplier stays in registers for up to 8 live elements per thread below
    // 1024 threads (those layouts run two waves per SIMD, so 256 registers per lane)
    constexpr bool kBInRegs = (RL <= 8) && (T < 1024);
    constexpr int EB = kBInRegs ? RL : 1;
    // ... and so does the potential A = v (.) dmod, also in the layouts of two workgroups
    // per compute unit (16 live elements, registers to spare once their twiddles come from a
    // table); otherwise it comes from L2
    constexpr bool kAInRegs = kBInRegs || (ECfg<P, V>::SINGLE && RL <= 16);
    constexpr int EA = kAInRegs ? RL : 1;
    // the series sum beyond the first term (w') stays in registers up to 8 elements per
    // thread, or 16 below 1024 threads (else in d.wacc)
    constexpr bool kWInRegs = RT <= 8 || (T < 1024 && RL <= 16);
    constexpr int EW = kWInRegs ? RL : 1;
    // the state between Pade factors stays in registers where the layout has room (one load
    // and one store of the field per step); otherwise it goes through the solve's work
    // array (a load and a store per factor).  Room: up to 8 live elements per thread below
    // 1024 threads, and 16 in the single-buffer layouts of up to 256 threads (their register
    // cap keeps two waves per SIMD; a few spills outside the term loop); elsewhere 16 more
    // would push the kernel past 256 registers and halve its occupancy
    constexpr bool kUInRegs = (T < 1024) && (RL <= 8 || (RL <= 16 && T <= 256 && ECfg<P, V>::SINGLE));
    constexpr int EU = kUInRegs ? RL : 1;
    // split transforms keep their second input in the solve's scratch (fewer spills)
    constexpr bool kKeepGlobal = true;
    const LdsBufs L = carve_lds<EK>(lds_raw);
    const int tid = threadIdx.x;
    const int N = d.N, p = d.p, nmax = d.nmax;
    Twiddles<EK> tw;
    init_twiddles<EK>(tw, L.tw4, d.tw, (key_split(EK) && key_var(EK) == 2) ? d.twl2 : d.twl);

    // d.field holds the state at the start of the step (the recovery point if the step
    // diverges); the state between Pade factors is in registers (kUInRegs) or in d.work.
    // Every thread reads and writes only its own positions, so these global accesses need
    // no barriers.
    float2 w[EW], a[RT], A[EA], u[EU];
    float4 Bm[EB];
    long long n = *d.step;
    // outputs of this launch: steps out_base, out_base + out_every, ... (row = slot)
    const long long out_base = d.out_every > 0 ? (n / d.out_every + 1) * d.out_every : 0;
    if (d.prof_mode == PROF_TABLE_FIXED) load_potential<P, V, kAInRegs, DK>(d, n + 1, A);

    long long terms = 0, done = 0;
    int max_used = 0, notconv = 0, status = kOK;
    double max_res = 0.0;

    for (int s = 0; s < nsteps; ++s) {
        const long long nn = n + 1;
        if (d.prof_mode == PROF_TABLE_STEPS && (nn - d.v_step0 - 1 < 0 || nn - d.v_step0 - 1 >= d.v_rows)) {
            status = kStatusProfileRange;  // no profile row for this step (uniform)
            break;
        }
        if (d.prof_mode != PROF_TABLE_FIXED) load_potential<P, V, kAInRegs, DK>(d, nn, A);
        if constexpr (kUInRegs) {
#pragma unroll
            for (int i = 0; i < RL; ++i) {
                const int pos = opaque_tid() + i * T;
                u[i] = pos < N ? ld2(d.field, pos) : make_float2(0.f, 0.f);
            }
        }
        bool bad = false;
        for (int j = 0; j < p; ++j) {
            const float2 *cur = (j == 0) ? d.field : d.work;
            // per-thread partial sums of |.|^2 in FP32 (a handful of terms), workgroup sums
            // in FP64
            float t0f = 0.f;
#pragma unroll
            for (int i = RL; i < RT; ++i) a[i] = make_float2(0.f, 0.f);
#pragma unroll
            for (int i = 0; i < RL; ++i) {
                const int pos = opaque_tid() + i * T, m = pos;
                if constexpr (kUInRegs) {
                    // no stores in this loop: tables at a clamped position, values selected,
                    // so that the loads overlap
                    const int pc = pos < N ? pos : N - 1;
                    const float2 av = cmul_df(u[i], ld4(d.s, j * N + pc));
                    a[i] = pos < N ? av : make_float2(0.f, 0.f);
                    if constexpr (kBInRegs) {
                        const float4 bv = ld4(d.bmul, j * N + pc);
                        Bm[i] = pos < N ? bv : make_float4(0.f, 0.f, 0.f, 0.f);
                    }
                } else if (pos < N) {
                    a[i] = cmul_df(ld2(cur, m), ld4(d.s, j * N + m));
                    if constexpr (kBInRegs) Bm[i] = ld4(d.bmul, j * N + m);
                } else {
                    a[i] = make_float2(0.f, 0.f);
                    if constexpr (kBInRegs) Bm[i] = make_float4(0.f, 0.f, 0.f, 0.f);
                }
                if constexpr (kWInRegs) w[i] = make_float2(0.f, 0.f);
                t0f += cnorm2(a[i]);
            }
            double t0 = t0f, dummy = 0.0;
            block_sum2<T>(t0, dummy, red);
            double tn = 0.0, wn = 0.0;
            int used = 0;
            bool conv = (nmax == 0);
            // half-iteration h: even -> a = A (.) S a (multiply by v); odd -> a = B_j (.) S a
            // (diagonal solve) and the term is accumulated; one transform site per loop
            for (int h = 0; h < 2 * nmax; ++h) {
                // even h: coefficients -> grid (inverse direction); odd h: grid -> coefficients
                const bool fwd = (h & 1) != 0;
                if constexpr (DK == kDkFourier) direct_core<EK>(a, L, tw, fwd);
                else if constexpr (DK == kDkSine) sine_core<EK>(a, L, tw, d.mirror, d.N);
                else dst_core<P, V, kKeepGlobal>(a, L, tw, d, d.xs, fwd ? d.kf : d.ki);
                if ((h & 1) == 0) {
#pragma unroll
                    for (int i = 0; i < RL; ++i) {
                        if constexpr (kAInRegs) {
                            a[i] = cmul(A[i], a[i]);
                        } else {
                            // pot spans the work stride: no bounds test on the load
                            const int pos = opaque_tid() + i * T;
                            const float2 pv = ld2(d.pot, pos);
                            a[i] = (pos < N) ? cmul(pv, a[i]) : make_float2(0.f, 0.f);
                        }
                    }
                    continue;
                }
                float tnf = 0.f, wpf = 0.f;
                if constexpr (kWInRegs) {
#pragma unroll
                    for (int i = 0; i < RL; ++i) {
                        const int pos = opaque_tid() + i * T;
                        if constexpr (kBInRegs) {
                            a[i] = cmul_df(a[i], Bm[i]);  // zero beyond N
                        } else {
                            // clamped position, product selected: no branch around the load
                            const float4 bm = ld4(d.bmul, j * N + (pos < N ? pos : N - 1));
                            const float2 ab = cmul_df(a[i], bm);
                            a[i] = pos < N ? ab : make_float2(0.f, 0.f);
                        }
                        tnf += cnorm2(a[i]);
                        // w' += a_m (the first term m = 1 starts it)
                        w[i] = h == 1 ? a[i] : cadd(w[i], a[i]);
                        wpf += cnorm2(w[i]);
                    }
                } else {
                    // the series sum goes through wacc, which spans the work stride: groups of
                    // G positions without a bounds test on wacc, whose loads are issued before
                    // the group's stores so that they overlap (a load cannot move above a store
                    // to a buffer that the compiler cannot tell apart from the one it reads);
                    // the multiplier row has N entries: a clamped position, the product selected
                    constexpr int G = RL < 4 ? RL : 4;
#pragma unroll
                    for (int g = 0; g < RL; g += G) {
                        float4 bm[G];
                        float2 wo[G];
#pragma unroll
                        for (int k2 = 0; k2 < G; ++k2) {
                            const int pos = opaque_tid() + (g + k2) * T;
                            if constexpr (!kBInRegs) bm[k2] = ld4(d.bmul, j * N + (pos < N ? pos : N - 1));
                            wo[k2] = h == 1 ? make_float2(0.f, 0.f) : ld2(d.wacc, pos);
                        }
#pragma unroll
                        for (int k2 = 0; k2 < G; ++k2) {
                            const int i = g + k2, pos = opaque_tid() + i * T;
                            if constexpr (kBInRegs) {
                                a[i] = cmul_df(a[i], Bm[i]);  // zero beyond N
                            } else {
                                const float2 ab = cmul_df(a[i], bm[k2]);
                                a[i] = pos < N ? ab : make_float2(0.f, 0.f);
                            }
                            tnf += cnorm2(a[i]);
                            // w' += a_m (the first term m = 1 starts it; beyond N it sums zeros)
                            const float2 ws = cadd(wo[k2], a[i]);
                            st2(d.wacc, pos, ws);
                            wpf += cnorm2(ws);
                        }
                    }
                }
                tn = tnf;
                double wp = wpf;
                block_sum2<T>(tn, wp, red);
                used = (h >> 1) + 1;
                if (!(isfinite(tn) && isfinite(wp))) {
                    bad = true;
                    break;
                }
                // The stopping rule compares |a_m|^2 with tol^2 |w|^2, w = a0 + w'.  By the
                // triangle inequality |w| <= |a0| + |w'|: while |a_m|^2 exceeds tol^2 times that
                // bound (with a margin well above the rounding of the sums) the exact test
                // cannot pass, and the exact norm (which needs a0) is formed only when it can,
                // and at the last term (whose norm the residual statistic reports).  Decisions
                // and reported norms are those of evaluating it every term.
                const double ub = sqrt(t0) + sqrt(wp);
                if (h + 1 < 2 * nmax && tn > d.tol2 * ub * ub * (1.0 + 1e-4)) continue;
                float wnf = 0.f;
                if constexpr (kWInRegs) {
#pragma unroll
                    for (int i = 0; i < RL; ++i) {
                        const int pos = opaque_tid() + i * T;
                        if (pos < N) {
                            // a0 = s_j (.) u again, from the factor's input state
                            const float2 a0v = cmul_df(kUInRegs ? u[i] : ld2(cur, pos), ld4(d.s, j * N + pos));
                            wnf += cnorm2(cadd(a0v, w[i]));
                        }
                    }
                } else {
                    // a0 = s_j (.) u again, from the factor's input state; loads at clamped
                    // positions (the state and the table have N entries) in pairs, terms
                    // selected
                    constexpr int G2 = RL < 2 ? RL : 2;
#pragma unroll
                    for (int g = 0; g < RL; g += G2) {
                        float2 uc[G2], wv[G2];
                        float4 sv[G2];
#pragma unroll
                        for (int k2 = 0; k2 < G2; ++k2) {
                            const int i = g + k2, pos = opaque_tid() + i * T, pc = pos < N ? pos : N - 1;
                            if constexpr (kUInRegs) uc[k2] = u[i];
                            else uc[k2] = ld2(cur, pc);
                            sv[k2] = ld4(d.s, j * N + pc);
                            wv[k2] = ld2(d.wacc, pos);
                        }
#pragma unroll
                        for (int k2 = 0; k2 < G2; ++k2) {
                            const int pos = opaque_tid() + (g + k2) * T;
                            const float e = cnorm2(cadd(cmul_df(uc[k2], sv[k2]), wv[k2]));
                            wnf += pos < N ? e : 0.f;
                        }
                    }
                }
                wn = wnf;
                double dummy = 0.0;
                block_sum2<T>(wn, dummy, red);
                if (!isfinite(wn)) {
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
            // product-form factor as an increment: u <- u + (q_j u + beta_j w')  (q_j, beta_j
            // double-float; w' = 0 without Neumann terms)
            const float4 be = ld4(d.beta, j);
#pragma unroll
            for (int i = 0; i < RL; ++i) {
                const int pos = opaque_tid() + i * T, m = pos;
                if constexpr (kUInRegs && kWInRegs) {
                    // registers only besides the table: clamped position, value selected
                    const float2 uc = u[i];
                    const float4 q = ld4(d.qmul, j * N + (pos < N ? pos : N - 1));
                    const float2 un = cadd(uc, cadd(cmul_df(uc, q), cmul_df(w[i], be)));
                    u[i] = pos < N ? un : uc;
                } else if (pos < N) {
                    const float2 ws = kWInRegs ? w[i] : (used > 0 ? ld2(d.wacc, m) : make_float2(0.f, 0.f));
                    const float2 uc = kUInRegs ? u[i] : ld2(cur, m);
                    const float2 un = cadd(uc, cadd(cmul_df(uc, ld4(d.qmul, j * N + m)), cmul_df(ws, be)));
                    if constexpr (kUInRegs) u[i] = un;
                    else st2(d.work, m, un);
                }
            }
        }
        if (bad) {
            status = kDiverged;
            break;
        }
        // commit the step (until here the field held the step-start state: the recovery point)
#pragma unroll
        for (int i = 0; i < RL; ++i) {
            const int pos = opaque_tid() + i * T, m = pos;
            if constexpr (kUInRegs) {
                if (pos < N) st2(d.field, m, u[i]);
            } else {
                if (pos < N) st2(d.field, m, ld2(d.work, m));
            }
        }
        n = nn;
        ++done;
        // output step: keep a snapshot of the sine-basis state; k_output turns it into the
        // physical field and TL after the march
        if (d.out_every > 0 && (n % d.out_every) == 0 && d.snap) {
            const long long slot = (n - out_base) / d.out_every;
            if (n >= out_base && slot < d.nout) {
#pragma unroll
                for (int i = 0; i < RL; ++i) {
                    const int pos = opaque_tid() + i * T, m = pos;
                    if constexpr (kUInRegs) {
                        if (pos < N) st2(d.snap + slot * N, m, u[i]);
                    } else {
                        if (pos < N) st2(d.snap + slot * N, m, ld2(d.field, m));
                    }
                }
            }
        }
    }
    if (tid == 0) {
        *d.step = n;
        if (status == kOK && notconv > 0) status = kNotConverged;
        DevStats st;  // (a solve stopped for a missing profile row keeps its steps so far)
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

// One solve per workgroup (descriptor blockIdx.x, its own step count), all with
// convolution length P.  The launch argument is the largest step count.
template <int P, int V>
__global__ __launch_bounds__((ECfg<P, V>::T), (ECfg<P, V>::MINW)) void k_march(const SolveDesc *__restrict__ descs,
                                                                               int nsteps) {
    __shared__ float4 lds_raw[lds_words<eng_key<P, V>()>()];
    __shared__ double red[2 * (ECfg<P, V>::T / 64)];
    march_body<P, V>(descs[blockIdx.x], descs[blockIdx.x].nsteps, lds_raw, red);
}

// The same march with direct transforms instead of chirp-z cores (DK: periodic plans with
// P = Nz, or Dirichlet plans with P = 2 (Nz + 1)).
template <int P, int V, int DK>
__global__ __launch_bounds__((ECfg<P, V>::T), (ECfg<P, V>::MINW)) void k_march_direct(
    const SolveDesc *__restrict__ descs, int nsteps) {
    __shared__ float4 lds_raw[lds_words<eng_key<P, V>()>()];
    __shared__ double red[2 * (ECfg<P, V>::T / 64)];
    march_body<P, V, DK>(descs[blockIdx.x], descs[blockIdx.x].nsteps, lds_raw, red);
}

// Solves of uneven length in one launch: every length that runs with 1024-thread workgroups
// (P = 8192, 16384, 32768); each workgroup takes the code path of its own descriptor's P.
constexpr int kFamilyT = 1024;
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kFamilyLds = cmax(lds_words<eng_key<8192, 0>()>(), lds_words<eng_key<16384, 0>()>());
static_assert(ECfg<8192, 0>::T == kFamilyT && ECfg<16384, 0>::T == kFamilyT &&
              ECfg<32768, 0>::T == kFamilyT, "family thread count");
__global__ __launch_bounds__(kFamilyT) void k_march_family(const SolveDesc *__restrict__ descs, int nsteps) {
    __shared__ float4 lds_raw[kFamilyLds];
    __shared__ double red[2 * (kFamilyT / 64)];
    const SolveDesc &d = descs[blockIdx.x];
    switch (d.P) {  // uniform over the workgroup
        case 8192: march_body<8192, 0>(d, d.nsteps, lds_raw, red); break;
        case 16384: march_body<16384, 0>(d, d.nsteps, lds_raw, red); break;
        case 32768: march_body<32768, 0>(d, d.nsteps, lds_raw, red); break;
        default: break;
    }
}

// ----------------------------------------------------------------------------- transforms
// Persistent over the batch: workgroup g transforms vectors g, g + G, g + 2G, ... (G =
// gridDim.x <= B, the workgroups that can be resident at once), so the twiddles are set up
// once per workgroup, and the next vector's input is loaded while the current one is
// transformed.  Each vector's in and out may be the same memory: vector v's output is
// stored after its input was read, and no other vector's input lies there.  Layout 0 (the
// most threads per workgroup) is used for every length: it measured faster for stand-alone
// transforms than the march's tuned layouts.
template <int P, int DK>
__global__ __launch_bounds__((ECfg<P, 0>::T)) void k_transform(const SolveDesc *__restrict__ desc, int mode,
                                                         const float2 *in, float2 *out,
                                                         const long long *__restrict__ step, int B) {
    constexpr int T = ECfg<P, 0>::T, RT = ECfg<P, 0>::RT;
    SSP_LDS_DECL((eng_key<P, 0>()));
    const SolveDesc &d = *desc;
    const int N = d.N;
    Twiddles<eng_key<P, 0>()> tw;
    init_twiddles<eng_key<P, 0>()>(tw, L.tw4, d.tw, d.twl);
    float2 xn[RT];
    auto load = [&](int v) {
        const float2 *vin = in + static_cast<size_t>(v) * N;
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            const int pos = opaque_tid() + i * T;
            xn[i] = pos < N ? ld2(vin, pos) : make_float2(0.f, 0.f);
        }
    };
    load(blockIdx.x);
    for (int v = blockIdx.x; v < B; v += gridDim.x) {  // uniform over the workgroup
        float2 x[RT];
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            const int pos = opaque_tid() + i * T;
            x[i] = (mode != 2 && pos < N) ? cmul(xn[i], ld2(d.pre, pos)) : xn[i];
        }
        if (v + static_cast<int>(gridDim.x) < B) load(v + gridDim.x);
        __syncthreads();  // the previous vector's last LDS reads are done
        if constexpr (DK == kDkFourier) direct_core<eng_key<P, 0>()>(x, L, tw, mode != 2);
        else if constexpr (DK == kDkSine) sine_core<eng_key<P, 0>()>(x, L, tw, d.mirror, N);
        else dst_core<P, 0, false>(x, L, tw, d, nullptr, mode == 2 ? d.ki : d.kf);
        float2 car = make_float2(1.f, 0.f);
        if (mode == 2) car = carrier(d.sigma, step[v]);
        float2 *vout = out + static_cast<size_t>(v) * N;
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            const int pos = opaque_tid() + i * T;
            if (pos < N) {
                float2 y = cmul(x[i], mode == 1 ? ld2(d.dmod, pos) : ld2(mode == 0 ? d.postf : d.post, pos));
                if (mode == 2) y = cmul(y, car);
                st2(vout, pos, y);
            }
        }
    }
}

// Output rows: blockIdx.x = solve * nout + row.  Snapshot (sine basis) -> physical field
// with the carrier of its step -> field row (complex64, in place over the snapshot when
// fld_out == snap) and TL row.
template <int P, int DK>
__global__ __launch_bounds__((ECfg<P, 0>::T)) void k_output(const SolveDesc *__restrict__ descs, int nout) {
    constexpr int T = ECfg<P, 0>::T, RT = ECfg<P, 0>::RT;
    SSP_LDS_DECL((eng_key<P, 0>()));
    const int b = blockIdx.x / nout, row = blockIdx.x % nout;
    const SolveDesc &d = descs[b];
    if (row >= d.nout || !d.snap || !d.stats || d.out_every <= 0) return;  // uniform
    const int N = d.N, tid = threadIdx.x;
    Twiddles<eng_key<P, 0>()> tw;
    init_twiddles<eng_key<P, 0>()>(tw, L.tw4, d.tw, d.twl);
    // the march that wrote the snapshots started at step step_index - steps_done
    const long long n0 = d.stats->step_index - d.stats->steps_done;
    const long long n = (n0 / d.out_every + 1) * d.out_every + static_cast<long long>(row) * d.out_every;
    if (n > d.stats->step_index) return;  // output step not reached in this launch: row untouched
    const float2 *src = d.snap + static_cast<size_t>(row) * N;
    float2 x[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        const int pos = tid + i * T;
        x[i] = (pos < N) ? ld2(src, pos) : make_float2(0.f, 0.f);
    }
    if constexpr (DK == kDkFourier) direct_core<eng_key<P, 0>()>(x, L, tw, false);
    else if constexpr (DK == kDkSine) sine_core<eng_key<P, 0>()>(x, L, tw, d.mirror, N);
    else dst_core<P, 0, false>(x, L, tw, d, nullptr, d.ki);
    const float2 car = carrier(d.sigma, n);
    const float lr = log10f(static_cast<float>(static_cast<double>(n) * d.dr));
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        const int pos = tid + i * T, m = pos;
        if (pos < N) {
            const float2 ph = cmul(cmul(ld2(d.post, m), x[i]), car);
            if (d.fld_out) st2(d.fld_out + static_cast<size_t>(row) * N, m, ph);
            if (d.tl_out) stf(d.tl_out + static_cast<size_t>(row) * N, m, -10.0f * (log10f(ph.x * ph.x + ph.y * ph.y) - lr));
        }
    }
}

// ----------------------------------------------------------------------------- plain form
// The same method as k_march, one kernel per stage and one solve per launch: the host loops
// over steps, Pade factors and Neumann half-terms; every kernel reads the series state from
// global memory and skips its work once the series has stopped (device-side flag), so the
// host never waits on the device inside a march.  Arithmetic and reduction order are those
// of k_march, so both forms give identical results.
struct PlainState {
    double t0, tn, wn;
    int done, used, bad, halt;
};

template <int P>
__global__ __launch_bounds__((ECfg<P, 0>::T)) void k_plain_start(const SolveDesc *__restrict__ desc, float2 *a, float2 *w,
                                                             PlainState *ps, int j) {
    constexpr int T = ECfg<P, 0>::T, RT = ECfg<P, 0>::RT;
    __shared__ double red[2 * (T / 64)];
    const SolveDesc &d = *desc;
    if (ps->halt) return;
    const int N = d.N;
    const float2 *cur = (j == 0) ? d.field : d.work;
    float part = 0.f;
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        const int pos = opaque_tid() + i * T, m = pos;
        if (pos < N) {
            const float2 v = cmul_df(ld2(cur, m), ld4(d.s, j * N + m));
            st2(a, m, v);
            part += cnorm2(v);
        }
    }
    double t0 = part, dummy = 0.0;
    block_sum2<T>(t0, dummy, red);
    if (threadIdx.x == 0) {
        ps->t0 = t0;
        ps->tn = 0.0;
        ps->wn = 0.0;
        ps->done = (d.nmax == 0);
        ps->used = 0;
        ps->bad = 0;
    }
}

template <int P>
__global__ __launch_bounds__((ECfg<P, 0>::T)) void k_plain_half(const SolveDesc *__restrict__ desc, float2 *a, float2 *w,
                                                            PlainState *ps, int j, int h, long long n) {
    constexpr int T = ECfg<P, 0>::T, RT = ECfg<P, 0>::RT;
    SSP_LDS_DECL((eng_key<P, 0>()));
    __shared__ double red[2 * (T / 64)];
    const SolveDesc &d = *desc;
    if (ps->halt || ps->done) return;  // uniform: the series has stopped
    Twiddles<eng_key<P, 0>()> tw;
    init_twiddles<eng_key<P, 0>()>(tw, L.tw4, d.tw, d.twl);
    const int N = d.N;
    float2 x[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        const int pos = opaque_tid() + i * T;
        x[i] = (pos < N) ? ld2(a, pos) : make_float2(0.f, 0.f);
    }
    dst_core<P, 0, false>(x, L, tw, d, nullptr, (h & 1) ? d.kf : d.ki);
    if ((h & 1) == 0) {
        float2 A[RT];
        load_potential<P, 0, true>(d, n, A);
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            const int pos = opaque_tid() + i * T;
            if (pos < N) st2(a, pos, cmul(A[i], x[i]));
        }
        return;
    }
    const float2 *cur = (j == 0) ? d.field : d.work;  // the factor's input state
    float tnf = 0.f, wnf = 0.f;
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        const int pos = opaque_tid() + i * T, m = pos;
        if (pos < N) {
            const float2 v = cmul_df(x[i], ld4(d.bmul, j * N + m));
            const float2 ww = h == 1 ? v : cadd(ld2(w, m), v);
            st2(a, m, v);
            st2(w, m, ww);
            tnf += cnorm2(v);
            wnf += cnorm2(cadd(cmul_df(ld2(cur, m), ld4(d.s, j * N + m)), ww));
        }
    }
    double tn = tnf, wn = wnf;
    block_sum2<T>(tn, wn, red);
    if (threadIdx.x == 0) {
        ps->tn = tn;
        ps->wn = wn;
        ps->used = (h >> 1) + 1;
        if (!(isfinite(tn) && isfinite(wn))) {
            ps->bad = 1;
            ps->done = 1;
        } else if (tn <= d.tol2 * wn) {
            ps->done = 1;
        }
    }
}

// End of a Pade factor: statistics, divergence test, product-form combine into d.work.
template <int P>
__global__ __launch_bounds__((ECfg<P, 0>::T)) void k_plain_finish(const SolveDesc *__restrict__ desc, const float2 *w,
                                                              PlainState *ps, int j) {
    constexpr int T = ECfg<P, 0>::T, RT = ECfg<P, 0>::RT;
    const SolveDesc &d = *desc;
    if (ps->halt) return;
    const bool conv = ps->done && !ps->bad;
    const bool diverged = ps->bad || (!conv && ps->tn >= ps->t0);
    const bool any = ps->used > 0;  // Neumann terms were added (w holds their sum)
    __syncthreads();  // every thread has read ps before thread 0 updates it
    if (diverged) {
        if (threadIdx.x == 0) {
            ps->halt = 1;
            d.stats->status = kDiverged;
        }
        return;
    }
    if (threadIdx.x == 0) {
        DevStats *st = d.stats;
        st->neumann_terms += ps->used;
        if (ps->used > st->neumann_max_used) st->neumann_max_used = ps->used;
        if (!conv && d.nmax > 0) st->not_converged += 1;
        if (d.nmax > 0) {
            const double res = ps->wn > 0.0 ? sqrt(ps->tn / ps->wn) : 0.0;
            if (res > st->max_residual) st->max_residual = res;
        }
    }
    const int N = d.N;
    const float2 *cur = (j == 0) ? d.field : d.work;
    const float4 be = ld4(d.beta, j);
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        const int pos = opaque_tid() + i * T, m = pos;
        if (pos < N) {
            const float2 uc = ld2(cur, m), ws = any ? ld2(w, m) : make_float2(0.f, 0.f);
            st2(d.work, m, cadd(uc, cadd(cmul_df(uc, ld4(d.qmul, j * N + m)), cmul_df(ws, be))));
        }
    }
}

// End of a step: commit, counters, output snapshot.
template <int P>
__global__ __launch_bounds__((ECfg<P, 0>::T)) void k_plain_commit(const SolveDesc *__restrict__ desc, PlainState *ps) {
    constexpr int T = ECfg<P, 0>::T, RT = ECfg<P, 0>::RT;
    const SolveDesc &d = *desc;
    if (ps->halt) return;
    const int N = d.N;
    const long long n = *d.step + 1;
    const long long n0 = d.stats->step_index - d.stats->steps_done;  // step at the call's start
    const long long out_base = d.out_every > 0 ? (n0 / d.out_every + 1) * d.out_every : 0;
    const long long slot = d.out_every > 0 ? (n - out_base) / d.out_every : -1;
    const bool snap = d.snap && d.out_every > 0 && (n % d.out_every) == 0 && n >= out_base && slot < d.nout;
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        const int pos = opaque_tid() + i * T, m = pos;
        if (pos < N) {
            const float2 v = ld2(d.work, m);
            st2(d.field, m, v);
            if (snap) st2(d.snap + slot * N, m, v);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        *d.step = n;
        d.stats->steps_done += 1;
        d.stats->step_index = n;
    }
}

template <int P>
hipError_t plain_march_P(const SolveDesc &hd, const SolveDesc *dd, int nsteps, float2 *work,
                         void *state, hipStream_t stream) {
    constexpr int T = ECfg<P, 0>::T;
    float2 *a = work, *w = work + hd.N;
    PlainState *ps = static_cast<PlainState *>(state);
    long long n0 = 0;
    hipError_t e = hipMemcpyAsync(&n0, hd.step, sizeof(n0), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return e;
    for (int s = 0; s < nsteps; ++s) {
        const long long n = n0 + s + 1;
        for (int j = 0; j < hd.p; ++j) {
            hipLaunchKernelGGL((k_plain_start<P>), dim3(1), dim3(T), 0, stream, dd, a, w, ps, j);
            for (int h = 0; h < 2 * hd.nmax; ++h)
                hipLaunchKernelGGL((k_plain_half<P>), dim3(1), dim3(T), 0, stream, dd, a, w, ps, j, h, n);
            hipLaunchKernelGGL((k_plain_finish<P>), dim3(1), dim3(T), 0, stream, dd, w, ps, j);
        }
        hipLaunchKernelGGL((k_plain_commit<P>), dim3(1), dim3(T), 0, stream, dd, ps);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int P>
hipError_t launch_output_P(int direct, const SolveDesc *d_descs, int nsolves, int nout, hipStream_t stream) {
    if constexpr (P <= kMaxEngine) {
        if (direct == kDkFourier) {
            hipLaunchKernelGGL((k_output<P, kDkFourier>), dim3(nsolves * nout), dim3(ECfg<P, 0>::T), 0, stream,
                               d_descs, nout);
            return hipGetLastError();
        }
        if (direct == kDkSine) {
            hipLaunchKernelGGL((k_output<P, kDkSine>), dim3(nsolves * nout), dim3(ECfg<P, 0>::T), 0, stream,
                               d_descs, nout);
            return hipGetLastError();
        }
    }
    if (direct != kDkChirp) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_output<P, kDkChirp>), dim3(nsolves * nout), dim3(ECfg<P, 0>::T), 0, stream, d_descs,
                       nout);
    return hipGetLastError();
}

template <int P, int V>
hipError_t launch_march_P(const SolveDesc *d_descs, int nsolves, int nsteps, hipStream_t stream) {
    hipLaunchKernelGGL((k_march<P, V>), dim3(nsolves), dim3(ECfg<P, V>::T), 0, stream, d_descs, nsteps);
    return hipGetLastError();
}

// variants 1 and 2 only where they differ from variant 0 (no duplicate instantiations)
template <int P>
hipError_t launch_march_PV(int v, const SolveDesc *d_descs, int nsolves, int nsteps, hipStream_t stream) {
    if constexpr (variant_exists(eng_len<P>(), 1)) {
        if (v == 1) return launch_march_P<P, 1>(d_descs, nsolves, nsteps, stream);
    }
    if constexpr (variant_exists(eng_len<P>(), 2)) {
        if (v == 2) return launch_march_P<P, 2>(d_descs, nsolves, nsteps, stream);
    }
    return launch_march_P<P, 0>(d_descs, nsolves, nsteps, stream);
}

// Grid of a persistent launch over B items: as many workgroups as can be resident at once
// (compute units x the kernel's occupancy per compute unit), at most B.
template <typename K>
hipError_t persistent_grid(K kernel, int threads, int B, int *grid) {
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0);
    if (e != hipSuccess) return e;
    const long long g = static_cast<long long>(cus > 0 ? cus : 1) * (per > 0 ? per : 1);
    *grid = B < g ? B : static_cast<int>(g);
    return hipSuccess;
}

template <int P, int DK>
hipError_t launch_transform_PK(int mode, const SolveDesc *d_desc, int B, const float2 *in, float2 *out,
                               const long long *step, hipStream_t stream) {
    constexpr int T = ECfg<P, 0>::T;
    int G = 0;
    const hipError_t e = persistent_grid(k_transform<P, DK>, T, B, &G);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_transform<P, DK>), dim3(G), dim3(T), 0, stream, d_desc, mode, in, out, step, B);
    return hipGetLastError();
}

template <int P>
hipError_t launch_transform_P(int direct, int mode, const SolveDesc *d_desc, int B, const float2 *in,
                              float2 *out, const long long *step, hipStream_t stream) {
    if constexpr (P <= kMaxEngine) {
        if (direct == kDkFourier) return launch_transform_PK<P, kDkFourier>(mode, d_desc, B, in, out, step, stream);
        if (direct == kDkSine) return launch_transform_PK<P, kDkSine>(mode, d_desc, B, in, out, step, stream);
    }
    if (direct != kDkChirp) return hipErrorInvalidValue;
    return launch_transform_PK<P, kDkChirp>(mode, d_desc, B, in, out, step, stream);
}

// Last-pass twiddle tables of the engines that read them (the split-transform engine and
// the layout-2 engines of 4096 and 8192; one per engine and device) and the kernel that
// fills one from the first-octant table: block r-1 holds w^{r t}.
constexpr int kSplitEK = eng_key<2 * kMaxEngine, 0>();
constexpr int kV2EK4096 = eng_key<4096, 2>(), kV2EK8192 = eng_key<8192, 2>(), kV2EK16384 = eng_key<16384, 2>();
template <int EK>
constexpr int twl_len() { return (Cfg<EK>::RT - 1) * Cfg<EK>::T; }
static_assert(!Twiddles<kSplitEK>::kRegs && !Twiddles<kV2EK4096>::kRegs && !Twiddles<kV2EK8192>::kRegs &&
                  !Twiddles<kV2EK16384>::kRegs,
              "engines that read a table");
__device__ float4 g_twl_split[twl_len<kSplitEK>()];
__device__ float4 g_twl_v2_4096[twl_len<kV2EK4096>()];
__device__ float4 g_twl_v2_8192[twl_len<kV2EK8192>()];
__device__ float4 g_twl_v2_16384[twl_len<kV2EK16384>()];

template <int EK>
__global__ __launch_bounds__(Cfg<EK>::T) void k_last_twiddles(const uint32_t *__restrict__ tab,
                                                              float4 *__restrict__ out) {
    constexpr int T = Cfg<EK>::T;
    const int t = threadIdx.x, r = blockIdx.x + 1;
    float2 h;
    uint32_t l;
    fetch_twiddle<EK>(tab, r * t, h, l);
    out[blockIdx.x * T + t] = make_float4(h.x, h.y, __uint_as_float(l & 0xffff0000u), __uint_as_float(l << 16));
}

// direct marches: every layout of the length (the plan picks one; see direct_variant)
template <int P, int V>
hipError_t launch_march_direct_PV(int kind, const SolveDesc *d_descs, int nsolves, int nsteps, hipStream_t stream) {
    if (kind == kDkFourier)
        hipLaunchKernelGGL((k_march_direct<P, V, kDkFourier>), dim3(nsolves), dim3(ECfg<P, V>::T), 0, stream,
                           d_descs, nsteps);
    else if (kind == kDkSine)
        hipLaunchKernelGGL((k_march_direct<P, V, kDkSine>), dim3(nsolves), dim3(ECfg<P, V>::T), 0, stream,
                           d_descs, nsteps);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}
template <int P>
hipError_t launch_march_direct_P(int kind, int v, const SolveDesc *d_descs, int nsolves, int nsteps,
                                 hipStream_t stream) {
    if constexpr (P <= kMaxEngine) {
        if constexpr (variant_exists(P, 1)) {
            if (v == 1) return launch_march_direct_PV<P, 1>(kind, d_descs, nsolves, nsteps, stream);
        }
        if constexpr (variant_exists(P, 2)) {
            if (v == 2) return launch_march_direct_PV<P, 2>(kind, d_descs, nsolves, nsteps, stream);
        }
        return launch_march_direct_PV<P, 0>(kind, d_descs, nsolves, nsteps, stream);
    } else {
        return hipErrorInvalidValue;
    }
}

}  // namespace

bool march_family_member(int P) { return P == 8192 || P == 16384 || P == 32768; }

bool engine_variant_exists(int P, int variant) {
    if (P > kMaxEngine) return variant == 0 || variant == 2;  // the split engine: layouts 0 and 2
    return variant >= 0 && variant <= 2 && variant_exists(P, variant);
}

int engine_threads(int P, int variant) {
    const int PE = P > kMaxEngine ? P / 2 : P;
    return threads_for(PE, engine_variant_exists(P, variant) ? variant : 0);
}

hipError_t launch_march_family(const SolveDesc *d_descs, int nsolves, int nsteps, hipStream_t stream) {
    if (nsolves <= 0 || nsteps <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_march_family, dim3(nsolves), dim3(kFamilyT), 0, stream, d_descs, nsteps);
    return hipGetLastError();
}

bool fft_length_supported(int P) {
    return P == 128 || P == 256 || P == 512 || P == 1024 || P == 2048 || P == 4096 || P == 8192 ||
           P == 16384 || P == 32768;
}

hipError_t last_twiddles(int P, const uint32_t *d_tw, const float4 **out) {
    *out = nullptr;
    const int which = P > kMaxEngine ? 0 : P == 8192 ? 1 : P == 4096 ? 2 : P == 16384 ? 3 : -1;
    if (which < 0) return hipSuccess;
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static const float4 *tables[kMaxDevices][4] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!tables[dev][which]) {
        // the symbol's device address on this device (the host-side name is not one)
        void *addr = nullptr;
        e = which == 0   ? hipGetSymbolAddress(&addr, HIP_SYMBOL(g_twl_split))
            : which == 1 ? hipGetSymbolAddress(&addr, HIP_SYMBOL(g_twl_v2_8192))
            : which == 2 ? hipGetSymbolAddress(&addr, HIP_SYMBOL(g_twl_v2_4096))
                         : hipGetSymbolAddress(&addr, HIP_SYMBOL(g_twl_v2_16384));
        if (e != hipSuccess) return e;
        float4 *dst = static_cast<float4 *>(addr);
        if (which == 0)
            hipLaunchKernelGGL((k_last_twiddles<kSplitEK>), dim3(Cfg<kSplitEK>::RT - 1), dim3(Cfg<kSplitEK>::T), 0,
                               nullptr, d_tw, dst);
        else if (which == 1)
            hipLaunchKernelGGL((k_last_twiddles<kV2EK8192>), dim3(Cfg<kV2EK8192>::RT - 1), dim3(Cfg<kV2EK8192>::T),
                               0, nullptr, d_tw, dst);
        else if (which == 2)
            hipLaunchKernelGGL((k_last_twiddles<kV2EK4096>), dim3(Cfg<kV2EK4096>::RT - 1), dim3(Cfg<kV2EK4096>::T),
                               0, nullptr, d_tw, dst);
        else
            hipLaunchKernelGGL((k_last_twiddles<kV2EK16384>), dim3(Cfg<kV2EK16384>::RT - 1),
                               dim3(Cfg<kV2EK16384>::T), 0, nullptr, d_tw, dst);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) return e;
        tables[dev][which] = dst;
    }
    *out = tables[dev][which];
    return hipSuccess;
}

#define SSP_DISPATCH_P(P, CALL) \
    switch (P) {                \
        case 128: return CALL(128);     \
        case 256: return CALL(256);     \
        case 512: return CALL(512);     \
        case 1024: return CALL(1024);   \
        case 2048: return CALL(2048);   \
        case 4096: return CALL(4096);   \
        case 8192: return CALL(8192);   \
        case 16384: return CALL(16384); \
        case 32768: return CALL(32768); \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_march(int P, int variant, int direct, const SolveDesc *d_descs, int nsolves, int nsteps,
                        hipStream_t stream) {
    if (nsolves <= 0 || nsteps <= 0) return hipSuccess;
    const int v = engine_variant_exists(P, variant) ? variant : 0;
    if (direct != kDkChirp) {
#define CALL_D(PP) launch_march_direct_P<PP>(direct, v, d_descs, nsolves, nsteps, stream)
        SSP_DISPATCH_P(P, CALL_D)
#undef CALL_D
    }
#define CALL_M(PP) launch_march_PV<PP>(v, d_descs, nsolves, nsteps, stream)
    SSP_DISPATCH_P(P, CALL_M)
#undef CALL_M
}

int direct_variant(int P, int kind) {
    if (P < 128 || P > kMaxEngine || (kind != kDkFourier && kind != kDkSine)) return 0;
    const int v = kTunedDirect[kind - 1][__builtin_ctz(P) - 7];
    return variant_exists(P, v) ? v : 0;
}

hipError_t launch_output(int P, int direct, const SolveDesc *d_descs, int nsolves, int nout, hipStream_t stream) {
    if (nsolves <= 0 || nout <= 0) return hipSuccess;
#define CALL_O(PP) launch_output_P<PP>(direct, d_descs, nsolves, nout, stream)
    SSP_DISPATCH_P(P, CALL_O)
#undef CALL_O
}

hipError_t plain_march(const SolveDesc &h_desc, const SolveDesc *d_desc, int nsteps, float2 *d_work,
                       void *d_state, hipStream_t stream) {
    if (nsteps <= 0) return hipSuccess;
#define CALL_PL(PP) plain_march_P<PP>(h_desc, d_desc, nsteps, d_work, d_state, stream)
    SSP_DISPATCH_P(h_desc.P, CALL_PL)
#undef CALL_PL
}

size_t plain_state_bytes() { return sizeof(PlainState); }

hipError_t launch_transform(int P, int direct, int mode, const SolveDesc *d_desc, int B, const float2 *in,
                            float2 *out, const long long *step, hipStream_t stream) {
    if (B <= 0) return hipSuccess;
#define CALL_T(PP) launch_transform_P<PP>(direct, mode, d_desc, B, in, out, step, stream)
    SSP_DISPATCH_P(P, CALL_T)
#undef CALL_T
}

}  // namespace ssp
