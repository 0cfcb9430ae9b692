// ssp_dense_march.hip - the range march with every transform of the Neumann series as a
// dense product on the matrix cores (the dense engine, Dirichlet plans with N <= 2048).
//
// Sec. 3.1: on the interior Dirichlet grid the isovelocity inverse is diagonal in the basis
// of the orthonormal DST-I matrix S (symmetric, S S = I), so every term of the Neumann
// series (Sec. 3 eq. neumannseries) in the sine basis is
//     a_m = t_j (.) S (v (.) S a_{m-1}),   a_0 = s_j (.) u,   t_j = -b_j s_j,
//     s_j = 1/(1 + b_j x_l),
// and the Pade factors are applied in product form u <- g_j u + (1 - g_j) sum_m a_m.  Here
// the two products with S run over the whole batch at once: the batch of B solves of one
// grid size is the column dimension of Y = S X (each complex vector two real columns), in
// fp16 MFMA with high/low operand parts (ssp_dense.hip), so one launch computes a
// transform for every solve.  The pointwise stages and the fp16 split of the next operand
// run in one workgroup per solve; a solve whose series has stopped (tolerance met, cap
// reached, divergence) leaves zero operand columns behind and is skipped until the next
// factor.  The host drives the loop over steps, factors and terms and stops issuing terms
// once no series of the batch is active.
//
// State: u in the plain sine basis (FP32 complex) for the whole launch; the plan's stored
// representation m (.) u is converted on entry and exit and at output steps (|m| = 1).
// Precision as in the FFT engine: double-float s_j, t_j, g_j and m, FP64 residual norms in a
// fixed reduction order, FP32 data.
#include "ssp_dense.h"
#include "ssp_df.h"
#include "ssp_device.h"

#include <math.h>

namespace ssp {
namespace {

constexpr int kCT = 256;                    // threads of the per-solve kernels
constexpr int kPer = kMaxDenseNz / kCT;     // elements per thread (N <= 2048)
constexpr int kDiverged = -4, kNotConverged = 1;

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
    for (int w = 0; w < kCT / 64; ++w) {
        a += red[2 * w];
        b += red[2 * w + 1];
    }
    __syncthreads();
}

__device__ __forceinline__ void block_max2(float &a, float &b, float *red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        a = fmaxf(a, __shfl_xor(a, off, 64));
        b = fmaxf(b, __shfl_xor(b, off, 64));
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        red[2 * wave] = a;
        red[2 * wave + 1] = b;
    }
    __syncthreads();
    a = 0.f;
    b = 0.f;
#pragma unroll
    for (int w = 0; w < kCT / 64; ++w) {
        a = fmaxf(a, red[2 * w]);
        b = fmaxf(b, red[2 * w + 1]);
    }
    __syncthreads();
}

// Exponent e with max |x| 2^e in [2^13, 2^14) (0 for a zero column): the scaling the
// product kernel undoes.
__device__ __forceinline__ int column_exponent(float m) {
    if (!(m > 0.f)) return 0;
    int E;
    frexpf(m, &E);
    return 14 - E;
}

// fp16 high/low planes of the two real columns of solve b from the thread's elements x
// (positions tid + i kCT; zeros up to kpad), or zero planes.
__device__ __forceinline__ void split_planes(const float2 (&x)[kPer], int n, int kpad, int b, bool zero,
                                             _Float16 *xh, _Float16 *xl, int *expo, float *redf) {
    const int tid = threadIdx.x;
    float mr = 0.f, mi = 0.f;
    if (!zero) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            mr = fmaxf(mr, fabsf(x[i].x));
            mi = fmaxf(mi, fabsf(x[i].y));
        }
    }
    block_max2(mr, mi, redf);
    const int er = column_exponent(mr), ei = column_exponent(mi);
    if (tid == 0) {
        expo[2 * b] = er;
        expo[2 * b + 1] = ei;
    }
    _Float16 *hr = xh + static_cast<size_t>(2 * b) * kpad, *hi = hr + kpad;
    _Float16 *lr = xl + static_cast<size_t>(2 * b) * kpad, *li = lr + kpad;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int k = tid + i * kCT;
        if (k >= kpad) break;
        float vr = 0.f, vi = 0.f;
        if (!zero && k < n) {
            vr = ldexpf(x[i].x, er);
            vi = ldexpf(x[i].y, ei);
        }
        const _Float16 a = static_cast<_Float16>(vr), c = static_cast<_Float16>(vi);
        hr[k] = a;
        hi[k] = c;
        lr[k] = static_cast<_Float16>(vr - static_cast<float>(a));
        li[k] = static_cast<_Float16>(vi - static_cast<float>(c));
    }
}

// Potential v (+ i eta) of global step n on the grid (the FFT engine's load_potential
// without the chirp modulation).
__device__ __forceinline__ float2 potential_at(const SolveDesc &d, const float *vrow, int k, float r) {
    float v = vrow[k];
    if (d.prof_mode == PROF_ANALYTIC && d.env[3] != 0.0) {
        const float z = static_cast<float>((k + d.zoff) * d.dz);
        const float xr = (r - static_cast<float>(d.env[4])) / static_cast<float>(d.env[5]);
        const float xz = (z - static_cast<float>(d.env[6])) / static_cast<float>(d.env[7]);
        const float dc = -static_cast<float>(d.env[3]) * expf(-(xr * xr) - (xz * xz));
        const float q = 1.0f + v;
        const float cm = static_cast<float>(d.c0) * rsqrtf(q);
        const float e = dc / cm;
        v += q * (-e * (2.0f + e) / ((1.0f + e) * (1.0f + e)));
    }
    return make_float2(v, d.vi ? d.vi[k] : 0.f);
}

__device__ __forceinline__ long long out_base(const SolveDesc &d, long long n0) {
    return d.out_every > 0 ? (n0 / d.out_every + 1) * d.out_every : 0;
}

// ---------------------------------------------------------------------------- kernels
// entry: u = conj(m) (.) stored representation; per-solve state from the step counter
__global__ __launch_bounds__(kCT) void k_dm_enter(const SolveDesc *__restrict__ descs, DenseCol *cols, float2 *U,
                                                 int *active) {
    const int b = blockIdx.x;
    const SolveDesc &d = descs[b];
    const int n = d.N;
    if (threadIdx.x == 0) {
        DenseCol c{};
        c.n0 = *d.step;
        cols[b] = c;
        if (b == 0) *active = 0;
    }
    float2 *u = U + static_cast<size_t>(b) * n;
    for (int k = threadIdx.x; k < n; k += kCT) u[k] = cmul_df_conj(d.field[k], d.mmod[k]);
}

// start of step s of the launch: the step-start state (recovery point) and the potential
__global__ __launch_bounds__(kCT) void k_dm_step_begin(const SolveDesc *__restrict__ descs, DenseCol *cols,
                                                      const float2 *U, float2 *U0, float2 *Vb, int s) {
    const int b = blockIdx.x;
    const SolveDesc &d = descs[b];
    DenseCol &c = cols[b];
    const int n = d.N;
    const long long nn = c.n0 + c.steps_done + 1;
    const bool run = c.status >= 0 && s < d.nsteps;
    bool range_ok = true;
    long long row = 0;
    if (d.prof_mode == PROF_TABLE_STEPS) {
        row = nn - d.v_step0 - 1;
        range_ok = row >= 0 && row < d.v_rows;
    }
    __syncthreads();  // every thread has read c before thread 0 writes it
    if (threadIdx.x == 0) {
        c.step_active = run && range_ok;
        if (run && !range_ok) c.status = kStatusProfileRange;
    }
    if (!(run && range_ok)) return;
    const float *vrow = d.v + row * n;
    const float r = static_cast<float>((static_cast<double>(nn) - 0.5) * d.dr);
    const float2 *u = U + static_cast<size_t>(b) * n;
    float2 *u0 = U0 + static_cast<size_t>(b) * n, *vb = Vb + static_cast<size_t>(b) * n;
    for (int k = threadIdx.x; k < n; k += kCT) {
        u0[k] = u[k];
        vb[k] = potential_at(d, vrow, k, r);
    }
}

// start of Pade factor j: a_0 = s_j (.) u (kept in A0), its norm, the sum of the later terms
// w' = 0; the operand of the first product (zero planes where no series runs)
__global__ __launch_bounds__(kCT) void k_dm_factor_begin(const SolveDesc *__restrict__ descs, DenseCol *cols,
                                                        const float2 *U, float2 *W, float2 *A0, _Float16 *xh,
                                                        _Float16 *xl, int *expo, int kpad, int *active, int j) {
    __shared__ double red[2 * (kCT / 64)];
    __shared__ float redf[2 * (kCT / 64)];
    const int b = blockIdx.x;
    const SolveDesc &d = descs[b];
    DenseCol &c = cols[b];
    const int n = d.N;
    const bool run = c.step_active && j < d.p;
    float2 a[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) a[i] = make_float2(0.f, 0.f);
    if (run) {
        const float2 *u = U + static_cast<size_t>(b) * n;
        float2 *w = W + static_cast<size_t>(b) * n, *a0 = A0 + static_cast<size_t>(b) * n;
        float part = 0.f;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int k = threadIdx.x + i * kCT;
            if (k < n) {
                a[i] = cmul_df(u[k], d.s[static_cast<size_t>(j) * n + k]);
                a0[k] = a[i];
                w[k] = make_float2(0.f, 0.f);
                part += cnorm2(a[i]);
            }
        }
        double t0 = part, dummy = 0.0;
        block_sum2(t0, dummy, red);
        if (threadIdx.x == 0) {
            c.t0 = t0;
            c.tn = 0.0;
            c.wn = 0.0;
            c.used = 0;
            c.bad = 0;
            c.series_active = d.nmax > 0;
            if (d.nmax > 0) atomicAdd(active, 1);
        }
    } else if (threadIdx.x == 0) {
        c.series_active = 0;
    }
    split_planes(a, n, kpad, b, !(run && d.nmax > 0), xh, xl, expo, redf);
}

// after the product into grid space: y = (v + i eta) (.) S a, the operand of the next product
__global__ __launch_bounds__(kCT) void k_dm_grid(const SolveDesc *__restrict__ descs, const DenseCol *cols,
                                                const float2 *G, const float2 *Vb, _Float16 *xh, _Float16 *xl,
                                                int *expo, int kpad) {
    __shared__ float redf[2 * (kCT / 64)];
    const int b = blockIdx.x;
    if (!cols[b].series_active) return;  // uniform: its operand planes are zero
    const SolveDesc &d = descs[b];
    const int n = d.N;
    const float2 *g = G + static_cast<size_t>(b) * n, *vb = Vb + static_cast<size_t>(b) * n;
    float2 y[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int k = threadIdx.x + i * kCT;
        y[i] = k < n ? cmul(g[k], vb[k]) : make_float2(0.f, 0.f);
    }
    split_planes(y, n, kpad, b, false, xh, xl, expo, redf);
}

// after the product back into the sine basis: term m = t_j (.) S y, the series sum, the
// residual and the stopping rule; the operand of the next term (zero planes once stopped)
__global__ __launch_bounds__(kCT) void k_dm_sine(const SolveDesc *__restrict__ descs, DenseCol *cols,
                                                const float2 *G, float2 *W, const float2 *A0, _Float16 *xh,
                                                _Float16 *xl, int *expo, int kpad, int *active, int j, int m) {
    __shared__ double red[2 * (kCT / 64)];
    __shared__ float redf[2 * (kCT / 64)];
    const int b = blockIdx.x;
    DenseCol &c = cols[b];
    if (!c.series_active) return;  // uniform
    const SolveDesc &d = descs[b];
    const int n = d.N;
    const float2 *g = G + static_cast<size_t>(b) * n;
    float2 *w = W + static_cast<size_t>(b) * n;
    const float2 *a0 = A0 + static_cast<size_t>(b) * n;
    float2 a[kPer];
    float tnf = 0.f, wnf = 0.f;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int k = threadIdx.x + i * kCT;
        a[i] = make_float2(0.f, 0.f);
        if (k < n) {
            a[i] = cmul_df(g[k], d.tmul[static_cast<size_t>(j) * n + k]);
            const float2 ws = cadd(w[k], a[i]);  // w' (the norm is that of w = a0 + w')
            w[k] = ws;
            tnf += cnorm2(a[i]);
            wnf += cnorm2(cadd(a0[k], ws));
        }
    }
    double tn = tnf, wn = wnf;
    block_sum2(tn, wn, red);
    bool stop = false, bad = false, nc = false;
    if (!(isfinite(tn) && isfinite(wn))) {
        bad = true;
        stop = true;
    } else if (tn <= d.tol2 * wn) {
        stop = true;
    } else if (m >= d.nmax) {
        stop = true;
        if (tn >= c.t0) bad = true;
        else nc = true;
    }
    __syncthreads();  // every thread has read c before thread 0 writes it
    if (threadIdx.x == 0) {
        c.tn = tn;
        c.wn = wn;
        c.used = m;
        if (stop) {
            c.series_active = 0;
            c.bad = bad;
            if (nc) c.notconv += 1;
            atomicSub(active, 1);
        }
    }
    split_planes(a, n, kpad, b, stop, xh, xl, expo, redf);
}

// end of Pade factor j: divergence (back to the step-start state, the solve stops) or
// statistics and the product-form update as the increment u <- u + (q_j u + beta_j w')
__global__ __launch_bounds__(kCT) void k_dm_factor_end(const SolveDesc *__restrict__ descs, DenseCol *cols,
                                                      float2 *U, const float2 *U0, const float2 *W, int j) {
    const int b = blockIdx.x;
    DenseCol &c = cols[b];
    const SolveDesc &d = descs[b];
    if (!c.step_active || j >= d.p) return;  // uniform
    const int n = d.N;
    float2 *u = U + static_cast<size_t>(b) * n;
    const bool bad = c.bad;
    __syncthreads();
    if (bad) {
        const float2 *u0 = U0 + static_cast<size_t>(b) * n;
        for (int k = threadIdx.x; k < n; k += kCT) u[k] = u0[k];
        if (threadIdx.x == 0) {
            c.status = kDiverged;
            c.step_active = 0;
        }
        return;
    }
    const float4 be = d.beta[j];
    const float2 *w = W + static_cast<size_t>(b) * n;
    const float4 *q = d.qmul + static_cast<size_t>(j) * n;
    for (int k = threadIdx.x; k < n; k += kCT) u[k] = cadd(u[k], cadd(cmul_df(u[k], q[k]), cmul_df(w[k], be)));
    if (threadIdx.x == 0) {
        c.terms += c.used;
        c.max_used = c.used > c.max_used ? c.used : c.max_used;
        if (d.nmax > 0) {
            const double res = c.wn > 0.0 ? sqrt(c.tn / c.wn) : 0.0;
            c.max_res = res > c.max_res ? res : c.max_res;
        }
    }
}

// end of step s: counters and the snapshot of an output step (stored representation)
__global__ __launch_bounds__(kCT) void k_dm_step_end(const SolveDesc *__restrict__ descs, DenseCol *cols,
                                                    const float2 *U) {
    const int b = blockIdx.x;
    DenseCol &c = cols[b];
    const SolveDesc &d = descs[b];
    if (!c.step_active) return;  // uniform
    const long long nn = c.n0 + c.steps_done + 1;
    __syncthreads();
    if (threadIdx.x == 0) c.steps_done += 1;
    if (d.out_every > 0 && (nn % d.out_every) == 0 && d.snap) {
        const long long base = out_base(d, c.n0);
        const long long slot = (nn - base) / d.out_every;
        if (nn >= base && slot < d.nout) {
            const int n = d.N;
            const float2 *u = U + static_cast<size_t>(b) * n;
            float2 *dst = d.snap + slot * n;
            for (int k = threadIdx.x; k < n; k += kCT) dst[k] = cmul_df(u[k], d.mmod[k]);
        }
    }
}

// exit: stored representation m (.) u, step counter and statistics
__global__ __launch_bounds__(kCT) void k_dm_exit(const SolveDesc *__restrict__ descs, const DenseCol *cols,
                                                const float2 *U) {
    const int b = blockIdx.x;
    const SolveDesc &d = descs[b];
    const DenseCol &c = cols[b];
    const int n = d.N;
    const float2 *u = U + static_cast<size_t>(b) * n;
    for (int k = threadIdx.x; k < n; k += kCT) d.field[k] = cmul_df(u[k], d.mmod[k]);
    if (threadIdx.x == 0) {
        *d.step = c.n0 + c.steps_done;
        int status = c.status;
        if (status == 0 && c.notconv > 0) status = kNotConverged;
        DevStats st;
        st.steps_done = c.steps_done;
        st.step_index = c.n0 + c.steps_done;
        st.neumann_terms = c.terms;
        st.neumann_max_used = c.max_used;
        st.not_converged = c.notconv;
        st.max_residual = c.max_res;
        st.status = status;
        st.pad_ = 0;
        if (d.stats) *d.stats = st;
    }
}

}  // namespace

namespace {
constexpr size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }
}  // namespace

// Sub-arrays of the dense engine's scratch, each 256-byte aligned: U, U0, W, G, V [B][n]
// complex; xh, xl [2B][kpad] fp16; expo [2B]; cols [B]; the active-series counter.
size_t dense_work_bytes(int B, int n) {
    const size_t kpad = (static_cast<size_t>(n) + 127) / 128 * 128, bb = static_cast<size_t>(B);
    return 6 * align256(sizeof(float2) * bb * n) + 2 * align256(sizeof(_Float16) * 2 * bb * kpad) +
           align256(sizeof(int) * 2 * bb) + align256(sizeof(DenseCol) * bb) + 256;
}

DenseWork carve_dense_work(void *base, int B, int n) {
    const size_t kpad = (static_cast<size_t>(n) + 127) / 128 * 128, bb = static_cast<size_t>(B);
    char *p = static_cast<char *>(base);
    auto take = [&p](size_t bytes) {
        char *q = p;
        p += align256(bytes);
        return q;
    };
    DenseWork w;
    w.U = reinterpret_cast<float2 *>(take(sizeof(float2) * bb * n));
    w.U0 = reinterpret_cast<float2 *>(take(sizeof(float2) * bb * n));
    w.W = reinterpret_cast<float2 *>(take(sizeof(float2) * bb * n));
    w.G = reinterpret_cast<float2 *>(take(sizeof(float2) * bb * n));
    w.V = reinterpret_cast<float2 *>(take(sizeof(float2) * bb * n));
    w.A0 = reinterpret_cast<float2 *>(take(sizeof(float2) * bb * n));
    w.xh = reinterpret_cast<_Float16 *>(take(sizeof(_Float16) * 2 * bb * kpad));
    w.xl = reinterpret_cast<_Float16 *>(take(sizeof(_Float16) * 2 * bb * kpad));
    w.expo = reinterpret_cast<int *>(take(sizeof(int) * 2 * bb));
    w.cols = reinterpret_cast<DenseCol *>(take(sizeof(DenseCol) * bb));
    w.active = reinterpret_cast<int *>(take(sizeof(int)));
    return w;
}

hipError_t dense_march(const DenseTables &t, const SolveDesc *d_descs, int B, int nsteps, int pmax, int nmax_max,
                       const DenseWork &w, int *h_active, hipStream_t stream) {
    if (B <= 0 || nsteps <= 0) return hipSuccess;
    const int kpad = t.kpad;
    hipError_t e = hipSuccess;
#define DM_LAUNCH(...)                                   \
    do {                                                 \
        hipLaunchKernelGGL(__VA_ARGS__);                 \
        e = hipGetLastError();                           \
        if (e != hipSuccess) return e;                   \
    } while (0)
    DM_LAUNCH(k_dm_enter, dim3(B), dim3(kCT), 0, stream, d_descs, w.cols, w.U, w.active);
    // terms between polls of the active-series count (each poll waits for the stream)
    constexpr int kPoll = 2;
    for (int s = 0; s < nsteps; ++s) {
        DM_LAUNCH(k_dm_step_begin, dim3(B), dim3(kCT), 0, stream, d_descs, w.cols, w.U, w.U0, w.V, s);
        for (int j = 0; j < pmax; ++j) {
            DM_LAUNCH(k_dm_factor_begin, dim3(B), dim3(kCT), 0, stream, d_descs, w.cols, w.U, w.W, w.A0, w.xh,
                      w.xl, w.expo, kpad, w.active, j);
            for (int m = 1; m <= nmax_max; ++m) {
                e = launch_dense_gemm_only(t, B, w.xh, w.xl, w.expo, w.G, stream);
                if (e != hipSuccess) return e;
                DM_LAUNCH(k_dm_grid, dim3(B), dim3(kCT), 0, stream, d_descs, w.cols, w.G, w.V, w.xh, w.xl, w.expo,
                          kpad);
                e = launch_dense_gemm_only(t, B, w.xh, w.xl, w.expo, w.G, stream);
                if (e != hipSuccess) return e;
                DM_LAUNCH(k_dm_sine, dim3(B), dim3(kCT), 0, stream, d_descs, w.cols, w.G, w.W, w.A0, w.xh, w.xl,
                          w.expo, kpad, w.active, j, m);
                if (m % kPoll == 0 && m < nmax_max) {
                    e = hipMemcpyAsync(h_active, w.active, sizeof(int), hipMemcpyDeviceToHost, stream);
                    if (e == hipSuccess) e = hipStreamSynchronize(stream);
                    if (e != hipSuccess) return e;
                    if (*h_active == 0) break;
                }
            }
            DM_LAUNCH(k_dm_factor_end, dim3(B), dim3(kCT), 0, stream, d_descs, w.cols, w.U, w.U0, w.W, j);
        }
        DM_LAUNCH(k_dm_step_end, dim3(B), dim3(kCT), 0, stream, d_descs, w.cols, w.U);
    }
    DM_LAUNCH(k_dm_exit, dim3(B), dim3(kCT), 0, stream, d_descs, w.cols, w.U);
#undef DM_LAUNCH
    return hipSuccess;
}

}  // namespace ssp
