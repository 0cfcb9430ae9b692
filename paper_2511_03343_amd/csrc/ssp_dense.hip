// ssp_dense.hip - the orthonormal DST-I of a batch of vectors as a dense matrix product on
// the gfx950 matrix cores.
//
// Y = S X with S_kn = sqrt(2/(N+1)) sin(pi k n/(N+1)) (Sec. 3.1, the sine basis of the
// Dirichlet problem) and X the batch, each complex vector contributing two real columns.
// The product runs in fp16 MFMA (v_mfma_f32_16x16x32_f16, FP32 accumulation) with every
// operand split into a high and a low fp16 part, keeping three of the four partial
// products:  S X ~ Sh Xh + Sh Xl + Sl Xh.  fp16 keeps 11 significant bits per part, so the
// dropped Sl Xl term and the split remainders are ~2^-22 of the result, but its exponent
// range is narrow: S is stored scaled by 2^12 and every column of X by its own power of two
// (largest element in [2^13, 2^14)), and the result is scaled back exactly.
//
// Kernels: k_dense_split (one workgroup per vector: scales and fp16 planes of its two
// columns) and k_dense_gemm (128 x 128 output tile per workgroup, 4 waves of 64 x 64, K in
// chunks of 32 through double-buffered LDS (one barrier per chunk), epilogue staged through
// LDS so that stores are coalesced).
#include "ssp_dense.h"

namespace ssp {
namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 128;       // output rows and columns per workgroup
constexpr int kKc = 32;          // K per chunk (one MFMA)
constexpr int kLdsRow = kKc + 8; // padded fp16 row of an operand tile
constexpr int kThreads = 256;
constexpr int kSplitThreads = 256;

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

// Exponent e with max |x| 2^e in [2^13, 2^14) (0 for a zero column).
__device__ __forceinline__ int column_exponent(float m) {
    if (!(m > 0.f)) return 0;
    int E;
    frexpf(m, &E);  // m = f 2^E, f in [0.5, 1)
    return 14 - E;
}

// One workgroup per vector b: exponents of its columns 2b (real part) and 2b+1 (imaginary
// part), and their fp16 high/low planes over kpad rows (zero beyond n).
__global__ __launch_bounds__(kSplitThreads) void k_dense_split(const float2 *__restrict__ in, int n, int kpad,
                                                             _Float16 *__restrict__ xh, _Float16 *__restrict__ xl,
                                                             int *__restrict__ expo) {
    __shared__ float red[2 * (kSplitThreads / 64)];
    const int b = blockIdx.x, tid = threadIdx.x;
    const float2 *x = in + static_cast<size_t>(b) * n;
    float mr = 0.f, mi = 0.f;
    for (int k = tid; k < n; k += kSplitThreads) {
        const float2 v = x[k];
        mr = fmaxf(mr, fabsf(v.x));
        mi = fmaxf(mi, fabsf(v.y));
    }
    mr = wave_max(mr);
    mi = wave_max(mi);
    if ((tid & 63) == 0) {
        red[2 * (tid >> 6)] = mr;
        red[2 * (tid >> 6) + 1] = mi;
    }
    __syncthreads();
    mr = 0.f;
    mi = 0.f;
#pragma unroll
    for (int w = 0; w < kSplitThreads / 64; ++w) {
        mr = fmaxf(mr, red[2 * w]);
        mi = fmaxf(mi, red[2 * w + 1]);
    }
    const int er = column_exponent(mr), ei = column_exponent(mi);
    if (tid == 0) {
        expo[2 * b] = er;
        expo[2 * b + 1] = ei;
    }
    _Float16 *hr = xh + static_cast<size_t>(2 * b) * kpad, *hi = hr + kpad;
    _Float16 *lr = xl + static_cast<size_t>(2 * b) * kpad, *li = lr + kpad;
    for (int k = tid; k < kpad; k += kSplitThreads) {
        float vr = 0.f, vi = 0.f;
        if (k < n) {
            const float2 v = x[k];
            vr = ldexpf(v.x, er);
            vi = ldexpf(v.y, ei);
        }
        const _Float16 a = static_cast<_Float16>(vr), c = static_cast<_Float16>(vi);
        hr[k] = a;
        hi[k] = c;
        lr[k] = static_cast<_Float16>(vr - static_cast<float>(a));
        li[k] = static_cast<_Float16>(vi - static_cast<float>(c));
    }
}

struct alignas(16) GemmLds {
    union {
        struct {
            _Float16 ah[kTile][kLdsRow], al[kTile][kLdsRow];  // S rows x K chunk
            _Float16 bh[kTile][kLdsRow], bl[kTile][kLdsRow];  // X columns x K chunk
        } op[2];                                              // double buffer
        float out[kTile][kTile + 1];                          // result tile [column][row]
    };
};

// Y (complex [ncols/2][n]) = 2^-(12 + e_c) (Sh Xh + Sh Xl + Sl Xh); tile (blockIdx.y rows,
// blockIdx.x columns).  sh/sl are [kpad][kpad] row-major (zero-padded), xh/xl [cols][kpad].
__global__ __launch_bounds__(kThreads) void k_dense_gemm(const _Float16 *__restrict__ sh,
                                                       const _Float16 *__restrict__ sl,
                                                       const _Float16 *__restrict__ xh,
                                                       const _Float16 *__restrict__ xl,
                                                       const int *__restrict__ expo, int n, int kpad,
                                                       int ncols, float2 *__restrict__ out) {
    __shared__ GemmLds L;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;  // 64 x 64 sub-tile of the wave
    const int r0 = blockIdx.y * kTile, c0 = blockIdx.x * kTile;

    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // global -> LDS: per operand plane 128 rows x 32 halves = 512 segments of 8 halves;
    // thread t moves segments t and t + 256
    const int sg0 = tid, sg1 = tid + kThreads;
    const int ra = sg0 >> 2, ka = (sg0 & 3) * 8, rb = sg1 >> 2, kb = (sg1 & 3) * 8;
    const int cmax = ncols - 1;
    auto colrow = [&](int r) { return min(c0 + r, cmax); };  // columns beyond the batch: any valid data
    half8 pa[2][2], pb[2][2];  // prefetch [plane][segment]
    auto fetch = [&](int k0) {
        pa[0][0] = *reinterpret_cast<const half8 *>(sh + static_cast<size_t>(r0 + ra) * kpad + k0 + ka);
        pa[0][1] = *reinterpret_cast<const half8 *>(sh + static_cast<size_t>(r0 + rb) * kpad + k0 + kb);
        pa[1][0] = *reinterpret_cast<const half8 *>(sl + static_cast<size_t>(r0 + ra) * kpad + k0 + ka);
        pa[1][1] = *reinterpret_cast<const half8 *>(sl + static_cast<size_t>(r0 + rb) * kpad + k0 + kb);
        pb[0][0] = *reinterpret_cast<const half8 *>(xh + static_cast<size_t>(colrow(ra)) * kpad + k0 + ka);
        pb[0][1] = *reinterpret_cast<const half8 *>(xh + static_cast<size_t>(colrow(rb)) * kpad + k0 + kb);
        pb[1][0] = *reinterpret_cast<const half8 *>(xl + static_cast<size_t>(colrow(ra)) * kpad + k0 + ka);
        pb[1][1] = *reinterpret_cast<const half8 *>(xl + static_cast<size_t>(colrow(rb)) * kpad + k0 + kb);
    };
    auto store = [&](int buf) {
        auto &o = L.op[buf];
        *reinterpret_cast<half8 *>(&o.ah[ra][ka]) = pa[0][0];
        *reinterpret_cast<half8 *>(&o.ah[rb][kb]) = pa[0][1];
        *reinterpret_cast<half8 *>(&o.al[ra][ka]) = pa[1][0];
        *reinterpret_cast<half8 *>(&o.al[rb][kb]) = pa[1][1];
        *reinterpret_cast<half8 *>(&o.bh[ra][ka]) = pb[0][0];
        *reinterpret_cast<half8 *>(&o.bh[rb][kb]) = pb[0][1];
        *reinterpret_cast<half8 *>(&o.bl[ra][ka]) = pb[1][0];
        *reinterpret_cast<half8 *>(&o.bl[rb][kb]) = pb[1][1];
    };
    // double-buffered K loop: chunk k is read from buffer k mod 2 while chunk k+1 goes from
    // registers (loaded during chunk k's products) into the other buffer; one barrier per
    // chunk separates the two
    fetch(0);
    store(0);
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < kpad; k0 += kKc, cur ^= 1) {
        const bool more = k0 + kKc < kpad;
        if (more) fetch(k0 + kKc);
        const auto &o = L.op[cur];
        // MFMA operands: row (column) = lane mod 16, 8 consecutive k from 8 (lane / 16)
        const int rr = lane & 15, kk = (lane >> 4) * 8;
        half8 bh[4], bl[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            bh[j] = *reinterpret_cast<const half8 *>(&o.bh[wn * 64 + j * 16 + rr][kk]);
            bl[j] = *reinterpret_cast<const half8 *>(&o.bl[wn * 64 + j * 16 + rr][kk]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const half8 ah = *reinterpret_cast<const half8 *>(&o.ah[wm * 64 + i * 16 + rr][kk]);
            const half8 al = *reinterpret_cast<const half8 *>(&o.al[wm * 64 + i * 16 + rr][kk]);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[j], acc[i][j], 0, 0, 0);
            }
        }
        if (more) store(cur ^ 1);
        __syncthreads();
    }
    // (the loop's last barrier: operand tiles no longer read, the LDS becomes the result tile)
    // accumulator layout: lane holds rows 4 (lane / 16) + q of column lane mod 16
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                L.out[wn * 64 + j * 16 + (lane & 15)][wm * 64 + i * 16 + (lane >> 4) * 4 + q] = acc[i][j][q];
    __syncthreads();
    // coalesced stores: thread -> row of one vector (real and imaginary column together)
    const int row = tid & (kTile - 1), vb0 = tid >> 7;
    const int grow = r0 + row;
#pragma unroll 4
    for (int v = vb0; v < kTile / 2; v += kThreads / kTile) {
        const int c = c0 + 2 * v;
        if (c >= ncols || grow >= n) continue;
        const float re = ldexpf(L.out[2 * v][row], -(12 + expo[c]));
        const float im = ldexpf(L.out[2 * v + 1][row], -(12 + expo[c + 1]));
        out[static_cast<size_t>(c / 2) * n + grow] = make_float2(re, im);
    }
}

}  // namespace

hipError_t launch_dense_dst(const DenseTables &t, int B, const float2 *in, float2 *out,
                            _Float16 *xh, _Float16 *xl, int *expo, hipStream_t stream) {
    if (B <= 0) return hipSuccess;
    const int ncols = 2 * B;
    hipLaunchKernelGGL(k_dense_split, dim3(B), dim3(kSplitThreads), 0, stream, in, t.n, t.kpad, xh, xl, expo);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((ncols + kTile - 1) / kTile, t.kpad / kTile);
    hipLaunchKernelGGL(k_dense_gemm, grid, dim3(kThreads), 0, stream, t.sh, t.sl, xh, xl, expo, t.n, t.kpad,
                       ncols, out);
    return hipGetLastError();
}

hipError_t launch_dense_gemm_only(const DenseTables &t, int B, const _Float16 *xh, const _Float16 *xl,
                                  const int *expo, float2 *out, hipStream_t stream) {
    const int ncols = 2 * B;
    const dim3 grid((ncols + kTile - 1) / kTile, t.kpad / kTile);
    hipLaunchKernelGGL(k_dense_gemm, grid, dim3(kThreads), 0, stream, t.sh, t.sl, xh, xl, expo, t.n, t.kpad,
                       ncols, out);
    return hipGetLastError();
}

}  // namespace ssp
