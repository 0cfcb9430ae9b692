// ssp_device.h - interface between the C ABI (host) and the HIP kernels of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace ssp {

// Per-solve statistics as kept on the device (layout identical to ssp_stats).
struct DevStats {
    int64_t steps_done;
    int64_t step_index;
    int64_t neumann_terms;
    int32_t neumann_max_used;
    int32_t not_converged;
    double max_residual;
    int32_t status;
    int32_t pad_;
};

enum ProfileMode : int { PROF_TABLE_FIXED = 0, PROF_TABLE_STEPS = 1, PROF_ANALYTIC = 2 };

// Everything one workgroup needs to march one solve.  Table pointers are shared by all
// solves of a plan; state pointers are per solve.
// The chirp-window spectra of one transform direction: K1, the Toeplitz spectrum ([P] complex
// FP32), and for unsplit lengths K2, the Hankel spectrum ([P]).  Split lengths derive K2 from
// K1 (see DeviceTables::kph): K2_q = phi w^{s q} K1_{q + P/2} (w = exp(-2 pi i/P), s = Nz - 1),
// with kph[k] = phi w^{s k} for k < 64, then kph[64 + m] = w^{64 s m} for m < P/64 (double-
// float; zero for the Fourier transform: no Hankel window), sg = (-1)^s and hs the
// double-float phase steps of the engine layout that runs the transform (SolveDesc::hstep,
// set on the device).
struct KWin {
    const float2 *k1, *k2;
    const float4 *kph;
    float sg;
    const float4 *hs;
};

struct SolveDesc {
    KWin kf;                    // [P] chirp-window spectra, forward direction (grid -> basis)
    KWin ki;                    // [P] the same for the inverse direction (== kf for the sine
                                //     and cosine transforms, their own inverses)
    const uint32_t *tw;         // first-octant twiddle table (see DeviceTables::twiddle)
    const float4 *twl;          // last-pass twiddles of the split-transform engine,
                                //     [RT-1][1024] (see last_twiddles), else null
    const float4 *twl2;         // the same for the layout-2 split engine ([31][512]: the
                                //     table of the layout-2 16384-point engine), else null
    const float2 *dmod, *post;  // [N] folded modulation; inverse post-modulation
    const float2 *pre;          // [N] forward pre-modulation (grid values -> chirp-z input)
    const float2 *postf;        // [N] forward post-modulation (stand-alone transform)
    const float4 *s, *bmul;     // [p][N] double-float
    const float4 *qmul;         // [p][N] double-float q_j = C_j r_j - 1 (see DeviceTables::qmul)
    const float4 *beta;         // [p] double-float C_j (1 - g_j)
    const float4 *twist;        // [P/2] double-float w_P^n (split transforms, P > 16384), else null
    int N, P, p, nmax;
    double tol2;                // tol^2 (squared-norm test)
    double sigma;               // k0 dr (carrier phase per step)
    double dz, dr, c0;
    int zoff;                   // depth of position m is (m + zoff) dz
    int prof_mode, v_rows;
    long long v_step0;
    const float *v;             // [v_rows][N] FP32 potential (table modes)
    const float *vi;            // [N] imaginary part of the potential (absorbing layer) or null
    double env[8];              // analytic environment (ssp_env order)
    float2 *field;              // [N] sine-basis state (modulated representation)
    float2 *work;               // [N] scratch state between Pade factors
    float2 *pot;                // [N] scratch potential A = v (.) dmod of the current step
    float2 *wacc;               // [N] scratch Neumann sum beyond the first term (kernels that do
                                //     not hold it in registers)
    float2 *xs;                 // [2][work_stride] scratch of split transforms
    long long *step;            // global step counter
    DevStats *stats;
    float2 *snap;               // [nout][N] sine-basis snapshots at output steps, or null
    float *tl_out;              // [nout][N] or null
    float2 *fld_out;            // [nout][N] or null (complex64, carrier included)
    int out_every;
    int nout;                   // output rows available in snap / tl_out / fld_out
    int nsteps;                 // range steps of this solve in the launch
    int variant;                // engine layout of the march (host-side grouping only)
    int direct;                 // direct transform kind (0 chirp-z, 1 Fourier, 2 sine; host grouping)
    const float4 *mirror;       // [N] double-float odd-extension image factors (direct sine)
    // dense engine (Dirichlet plans with N <= kMaxDenseNz), else null:
    const float4 *tmul;         // [p][N] double-float -b_j/(1 + b_j x_l) in the plain sine basis
    const float4 *mmod;         // [N] double-float m with (stored representation) = m (.) (sine
                                //     coefficients), |m| = 1
    int engine;                 // 0 FFT engine, 1 dense engine (host grouping only)
    // split lengths: Hankel phase steps w^{s D i} (i < 16, w = exp(-2 pi i/P), s = N - 1; see
    // KWin; double-float) between the elements of one thread of a split half, D = twice the
    // thread count of an engine layout: hstep for the march's layout, hstep0 for layout 0
    // (the transform, output and plain-form kernels).  Read through the descriptor, they are
    // scalar loads.
    float4 hstep[16], hstep0[16];
};

// Device statuses besides the ssp_status codes they share: a march step whose tabulated
// profile row is missing stops that solve with kStatusProfileRange (SSP_E_INVAL).
constexpr int kStatusProfileRange = -1;

// Launch the fused persistent march: one workgroup per descriptor, all with the same FFT
// length P, each marching its own descriptor's nsteps (nsteps here: the largest, 0 = no
// launch).  direct: the plans' direct transform kind (0: chirp-z cores; 1: periodic grid of
// length P, FFTs; 2: Dirichlet grid of length P/2 - 1, the FFT of the odd extension;
// P <= 16384 for both).  Returns hipSuccess or the launch error.
// Scratch per solve behind SolveDesc::work: work, pot, wacc and the two halves of xs, each
// work_stride elements (complex) long: the positions t + iT (i < live elements) that the
// threads of every layout touch, P/2 for chirp-z and direct sine plans, P (= Nz) for direct
// periodic ones; at least Nz.  The per-position loops of the Neumann terms then access this
// scratch without a bounds test (positions >= Nz hold values that are never used), which
// keeps them free of branches, so that their memory accesses overlap.
constexpr int kWorkPerSolve = 5;
__host__ __device__ inline size_t work_stride(int P, int direct) {
    return direct == 1 ? static_cast<size_t>(P) : static_cast<size_t>(P) / 2;
}
inline void set_work(SolveDesc &d, float2 *base) {
    const size_t S = work_stride(d.P, d.direct);
    d.work = base;
    d.pot = base + S;
    d.wacc = base + 2 * S;
    d.xs = base + 3 * S;
}

hipError_t launch_march(int P, int variant, int direct, const SolveDesc *d_descs, int nsolves, int nsteps,
                        hipStream_t stream);
// Autotuned layout of the direct-transform march of length P and kind (1 Fourier, 2 sine).
int direct_variant(int P, int kind);

// Engine layouts of the march kernel: variant 0 is the default; variants 1 and 2 (where they
// exist) use other thread counts, i.e. other radices for the first and last FFT passes
// (variant 2 with one LDS buffer, two workgroups per compute unit).  Results differ in
// rounding only.
bool engine_variant_exists(int P, int variant);
int engine_threads(int P, int variant);

// One launch for solves of different FFT lengths, all members of the 1024-thread family
// (march_family_member, variant 0): each workgroup runs the code of its own descriptor's P.
bool march_family_member(int P);
hipError_t launch_march_family(const SolveDesc *d_descs, int nsolves, int nsteps, hipStream_t stream);

// Convert the snapshots of the preceding march into field / TL rows: one workgroup per
// (solve, output row); rows beyond a solve's nout are skipped.  Output rows of a launch that
// starts at step n0 are the steps (n0/out_every + 1) out_every + row out_every; the step at
// the start is recovered from the solve's statistics (step_index - steps_done), so stats
// must be present whenever snapshots are.
hipError_t launch_output(int P, int direct, const SolveDesc *d_descs, int nsolves, int nout, hipStream_t stream);

// Batched transforms over B vectors of a plan's grid (tables from desc, one desc on the
// device shared by the whole batch).
//   mode 0: the forward transform of the plan's basis, grid values -> coefficients
//           (orthonormal DST-I for Dirichlet boundaries)
//   mode 1: physical -> modulated coefficient representation
//   mode 2: modulated coefficient representation -> physical field with carrier at step[b]
hipError_t launch_transform(int P, int direct, int mode, const SolveDesc *d_desc, int B, const float2 *in,
                            float2 *out, const long long *step, hipStream_t stream);

// Plain form: one kernel per stage (start, Neumann half-term, finish, commit) for the single
// solve of h_desc / d_desc, host loop over steps, factors and half-terms.  d_work holds 2N
// complex values, d_state plain_state_bytes().  d_desc->stats must be zeroed by the caller.
hipError_t plain_march(const SolveDesc &h_desc, const SolveDesc *d_desc, int nsteps, float2 *d_work,
                       void *d_state, hipStream_t stream);
size_t plain_state_bytes();

bool fft_length_supported(int P);

// Last-pass twiddles w^{r t} (r = 1 .. RT-1, thread t) of the engine that serves split
// transforms (P above the largest single-workgroup FFT: two halves of 16384 points, 1024
// threads per workgroup), as double-float float4 (hi.re, hi.im, lo.re, lo.im).  That engine
// reads them from this table instead of holding them in registers.  The table lives in
// device memory of the current device for the life of the process; the first call per
// device fills it from the first-octant table d_tw of the engine length (a kernel on the
// null stream, waited for), later calls return it.  *out is null for unsplit lengths.
// Thread-safe.
hipError_t last_twiddles(int P, const uint32_t *d_tw, const float4 **out);

}  // namespace ssp
