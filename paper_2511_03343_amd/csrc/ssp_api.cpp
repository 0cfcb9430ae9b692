// ssp_api.cpp - the C ABI (include/ssp.h): argument checks, plan and device-memory
// ownership, host<->device copies and kernel launches.
#include "../../include/ssp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "ssp_device.h"
#include "ssp_plan.h"
#include "ssp_dense.h"
#include "ssp_modal.h"
#include "ssp_tuned.h"

namespace {

thread_local std::string g_last_error;

ssp_status fail(ssp_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? SSP_E_NOMEM : SSP_E_DEVICE,           \
                        std::string(#expr) + ": " + hipGetErrorString(e_));               \
    } while (0)

// Largest supported convolution length of the chirp-z transform: two halves of the largest
// FFT one workgroup holds in LDS.
constexpr int kMaxP = 2 * ssp::kMaxEngineFFT;

template <typename T>
hipError_t dev_alloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) return hipSuccess;
    return hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
}
template <typename T>
void dev_free(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

}  // namespace

static_assert(SSP_BC_DIRICHLET == ssp::kBcDirichlet && SSP_BC_NEUMANN == ssp::kBcNeumann &&
                  SSP_BC_PERIODIC == ssp::kBcPeriodic,
              "boundary-condition codes of the ABI and the tables agree");

struct ssp_plan {
    int N = 0, P = 0, p = 0, nmax = 0;
    double H = 0, f = 0, c0 = 0, dr = 0, tol = 0, k0 = 0, sigma = 0, alpha = 0;
    int out_every = 1;
    int engine = SSP_ENGINE_AUTO;       // SSP_OPT_ENGINE
    int plain = 0;                      // SSP_OPT_PLAIN: one kernel per stage
    double gain_limit = 1e-6;           // SSP_OPT_GAIN_LIMIT
    bool contraction_check = false;     // SSP_OPT_CONTRACTION_CHECK
    int bc = ssp::kBcDirichlet;         // boundary condition (Sec. 3.1)
    int variant_opt = -1;               // SSP_OPT_VARIANT
    hipStream_t stream = nullptr;
    ssp::PadeSet ps;
    ssp::DeviceTables tab;
    // device tables
    float4 *d_kph = nullptr;  // split lengths: the phase table of the derived Hankel spectrum
    float2 *d_k1 = nullptr, *d_k2 = nullptr, *d_dmod = nullptr, *d_post = nullptr, *d_pre = nullptr;
    float2 *d_k1i = nullptr, *d_postf = nullptr;  // only where they differ
    float4 *d_mirror = nullptr;         // odd-extension image factors (direct sine transform)
    const float4 *d_twl = nullptr;      // shared last-pass twiddles of 1024-thread engines (not owned)
    const float4 *d_twl2 = nullptr;     // ... of the layout-2 split engine (split plans; not owned)
    uint32_t *d_tw = nullptr;
    float4 *d_s = nullptr, *d_bmul = nullptr, *d_qmul = nullptr, *d_beta = nullptr;
    float4 *d_twist = nullptr;
    // environment
    int prof_mode = ssp::PROF_TABLE_FIXED, v_rows = 0;
    long long v_step0 = 0;
    float *d_v = nullptr;
    size_t v_cap = 0;
    float *d_vi = nullptr;              // absorbing layer: imaginary part of v [N], or null
    double env[8] = {0};
    // state of the plan's own solve
    float2 *d_field = nullptr, *d_work = nullptr;
    long long *d_step = nullptr;
    ssp::DevStats *d_stats = nullptr;
    ssp::SolveDesc *d_desc = nullptr;   // one descriptor for the plan's own solve
    bool has_field = false;
    long long step_index = 0;
    // batched descriptors (device-resident march)
    ssp::SolveDesc *d_descs = nullptr;
    int descs_cap = 0;
    float2 *d_bwork = nullptr;          // scratch of a device batch [cap][solve_work_elems]
    int bwork_cap = 0;
    float2 *d_snap = nullptr;           // output snapshots of a device batch
    size_t snap_cap = 0;
    ssp::DevStats *d_bstats = nullptr;  // statistics of a device batch when the caller passes none
    int bstats_cap = 0;
    // recorded launches of ssp_march_device (SSP_OPT_GRAPH)
    bool use_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    struct GraphKey {
        int B, nsteps;
        void *psi, *step, *tl, *stats;
        hipStream_t stream;
        bool operator==(const GraphKey &o) const {
            return B == o.B && nsteps == o.nsteps && psi == o.psi && step == o.step && tl == o.tl &&
                   stats == o.stats && stream == o.stream;
        }
    } graph_key{};
    // output staging
    float2 *d_out_fld = nullptr;
    float *d_out_tl = nullptr;
    size_t out_cap = 0;
    // dense DST (matrix cores): split-operand scratch of the stand-alone transform (S itself
    // is shared by the plans of one grid size, see dense_tables)
    _Float16 *d_dense_xh = nullptr, *d_dense_xl = nullptr;
    // dense engine: per-plan tables and, on the first plan of a batch, the launch scratch
    float4 *d_tmul = nullptr, *d_mmod = nullptr;
    void *d_dense_work = nullptr;
    size_t dense_work_cap = 0;
    int *h_active = nullptr;            // pinned: series still running in a dense launch
    // ssp_march_batch_async: the host step counter is stale until the statistics are read
    // after the stream the batch ran on
    bool async_pending = false;
    hipStream_t pending_stream = nullptr;
    // recorded launches of ssp_march_batch_async on its first plan (SSP_OPT_GRAPH)
    hipGraph_t bgraph = nullptr;
    hipGraphExec_t bgraph_exec = nullptr;
    std::vector<const ssp_plan *> bkey_plans;
    std::vector<int> bkey_steps;
    std::vector<void *> bkey_tl;
    hipStream_t bkey_stream = nullptr;
    // contraction estimate (ssp_plan_contraction): potential rows sampled from the current
    // profile in FP64 (v + i eta), and the cached estimate for SSP_OPT_CONTRACTION_CHECK
    std::vector<std::complex<double>> vs;
    int vs_rows = 0;
    std::vector<double> h_eta;          // absorber (host copy), empty without one
    std::vector<double> rho_est;
    bool rho_valid = false;
    int *d_dense_expo = nullptr;
    int dense_cols_cap = 0;
    // side streams of a batch whose launch groups run concurrently (default priority)
    hipStream_t side[3] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr, join[3] = {nullptr, nullptr, nullptr};
    // plain-form work buffers
    float2 *d_plain = nullptr;
    void *d_plain_flags = nullptr;      // plain-form series state
};

namespace {

void drop_graph(ssp_plan *pl) {
    if (pl->graph_exec) (void)hipGraphExecDestroy(pl->graph_exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    pl->graph_exec = nullptr;
    pl->graph = nullptr;
    if (pl->bgraph_exec) (void)hipGraphExecDestroy(pl->bgraph_exec);
    if (pl->bgraph) (void)hipGraphDestroy(pl->bgraph);
    pl->bgraph_exec = nullptr;
    pl->bgraph = nullptr;
    pl->bkey_plans.clear();
}

bool dense_capable(const ssp_plan *pl) { return pl->bc == ssp::kBcDirichlet && pl->N <= ssp::kMaxDenseNz; }

ssp_status sync_pending(ssp_plan *pl);
std::vector<std::complex<double>> estimate_rows(const ssp_plan *pl);

// Engine of the plan's march: the option, or for SSP_ENGINE_AUTO the autotuner's choice for
// the plan's (Nz, p) class (dense only where the plan can run it).
int effective_engine(const ssp_plan *pl) {
    if (!dense_capable(pl) || pl->engine == SSP_ENGINE_FFT) return SSP_ENGINE_FFT;
    if (pl->engine == SSP_ENGINE_DENSE) return SSP_ENGINE_DENSE;
    return ssp::tuned_engine(pl->N, pl->p) == 1 ? SSP_ENGINE_DENSE : SSP_ENGINE_FFT;
}

// S of the dense transform for grid size n on the current device: built once per (device,
// n) and shared by every plan of that size for the life of the process.
ssp_status dense_tables(int n, ssp::DenseTables &out) {
    static std::mutex mu;
    static std::map<std::pair<int, int>, ssp::DenseTables> cache;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find({dev, n});
    if (it == cache.end()) {
        std::vector<uint16_t> sh, sl;
        int kpad = 0;
        ssp::build_dense_tables(n, kpad, sh, sl);
        _Float16 *dsh = nullptr, *dsl = nullptr;
        HIP_TRY(dev_alloc(&dsh, sh.size()));
        hipError_t e = dev_alloc(&dsl, sl.size());
        if (e == hipSuccess) e = hipMemcpy(dsh, sh.data(), sh.size() * 2, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(dsl, sl.data(), sl.size() * 2, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            dev_free(dsh);
            dev_free(dsl);
            return fail(e == hipErrorOutOfMemory ? SSP_E_NOMEM : SSP_E_DEVICE, hipGetErrorString(e));
        }
        ssp::DenseTables t;
        t.sh = dsh;
        t.sl = dsl;
        t.n = n;
        t.kpad = kpad;
        it = cache.emplace(std::make_pair(dev, n), t).first;
    }
    out = it->second;
    return SSP_OK;
}

constexpr int kSideStreams = 3;

hipError_t ensure_side_streams(ssp_plan *pl) {
    if (pl->fork) return hipSuccess;
    hipError_t e = hipSuccess;
    for (int j = 0; j < kSideStreams && e == hipSuccess; ++j) {
        e = hipStreamCreateWithFlags(&pl->side[j], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->join[j], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming);
    return e;
}

void free_side_streams(ssp_plan *pl) {
    for (int j = 0; j < kSideStreams; ++j) {
        if (pl->side[j]) (void)hipStreamDestroy(pl->side[j]);
        if (pl->join[j]) (void)hipEventDestroy(pl->join[j]);
        pl->side[j] = nullptr;
        pl->join[j] = nullptr;
    }
    if (pl->fork) (void)hipEventDestroy(pl->fork);
    pl->fork = nullptr;
}

void free_tables(ssp_plan *pl) {
    dev_free(pl->d_k1);
    dev_free(pl->d_k2);
    dev_free(pl->d_kph);
    dev_free(pl->d_k1i);
    dev_free(pl->d_postf);
    dev_free(pl->d_mirror);
    dev_free(pl->d_dmod);
    dev_free(pl->d_post);
    dev_free(pl->d_pre);
    dev_free(pl->d_tw);
    dev_free(pl->d_s);
    dev_free(pl->d_bmul);
    dev_free(pl->d_qmul);
    dev_free(pl->d_beta);
    dev_free(pl->d_twist);
    dev_free(pl->d_tmul);
    dev_free(pl->d_mmod);
}

template <typename D, typename S>
hipError_t upload(D *dst, const std::vector<S> &src) {
    return hipMemcpy(dst, src.data(), src.size() * sizeof(S), hipMemcpyHostToDevice);
}

// (Re)compute Pade coefficients and all tables for the current (N, H, f, c0, dr, p, alpha).
ssp_status build_plan_tables(ssp_plan *pl) {
    std::string err;
    ssp::PadeSet ps;
    if (!ssp::pade_coefficients(pl->sigma, pl->p, pl->alpha, ps, err)) return fail(SSP_E_INVAL, err);
    ssp::DeviceTables tab;
    ssp::build_tables(pl->N, pl->H, pl->k0, ps, pl->bc, tab);
    if (!(tab.max_gain <= 1.0 + pl->gain_limit))
        return fail(SSP_E_UNSTABLE, "max |e^{i sigma} R(x_l)| - 1 = " + std::to_string(tab.max_gain - 1.0) +
                                        " exceeds the gain limit " + std::to_string(pl->gain_limit));
    if (!ssp::fft_length_supported(tab.P)) return fail(SSP_E_UNIMPL, "unsupported FFT length");
    free_tables(pl);
    const int N = pl->N, P = tab.P, p = ps.p;
    HIP_TRY(dev_alloc(&pl->d_k1, tab.k1.size() / 2));   // [P], none for direct transforms
    HIP_TRY(dev_alloc(&pl->d_k2, tab.k2.size() / 2));    // unsplit lengths
    HIP_TRY(dev_alloc(&pl->d_kph, tab.kph.size() / 4));  // split lengths
    HIP_TRY(dev_alloc(&pl->d_tw, tab.twiddle.size()));
    HIP_TRY(dev_alloc(&pl->d_dmod, N));
    HIP_TRY(dev_alloc(&pl->d_post, N));
    HIP_TRY(dev_alloc(&pl->d_pre, N));
    HIP_TRY(dev_alloc(&pl->d_s, static_cast<size_t>(p) * N));
    HIP_TRY(dev_alloc(&pl->d_bmul, static_cast<size_t>(p) * N));
    HIP_TRY(dev_alloc(&pl->d_qmul, static_cast<size_t>(p) * N));
    HIP_TRY(dev_alloc(&pl->d_beta, p));
    HIP_TRY(dev_alloc(&pl->d_twist, tab.twist.size() / 4));
    HIP_TRY(dev_alloc(&pl->d_k1i, tab.k1i.size() / 2));
    HIP_TRY(dev_alloc(&pl->d_postf, tab.postf.size() / 2));
    if (!tab.k1i.empty()) HIP_TRY(upload(pl->d_k1i, tab.k1i));
    if (!tab.postf.empty()) HIP_TRY(upload(pl->d_postf, tab.postf));
    HIP_TRY(dev_alloc(&pl->d_mirror, tab.mirror.size() / 4));
    if (!tab.mirror.empty()) HIP_TRY(upload(pl->d_mirror, tab.mirror));
    if (!tab.k1.empty()) HIP_TRY(upload(pl->d_k1, tab.k1));
    if (!tab.k2.empty()) HIP_TRY(upload(pl->d_k2, tab.k2));
    if (!tab.kph.empty()) HIP_TRY(upload(pl->d_kph, tab.kph));
    HIP_TRY(upload(pl->d_tw, tab.twiddle));
    HIP_TRY(ssp::last_twiddles(P, pl->d_tw, &pl->d_twl));
    // split plans: their octant table is that of the 16384-point engine, whose layout-2 table
    // serves the layout-2 split engine
    if (P > 16384) HIP_TRY(ssp::last_twiddles(P / 2, pl->d_tw, &pl->d_twl2));
    HIP_TRY(upload(pl->d_dmod, tab.dmod));
    HIP_TRY(upload(pl->d_post, tab.post));
    HIP_TRY(upload(pl->d_pre, tab.pre));
    HIP_TRY(upload(pl->d_s, tab.s));
    HIP_TRY(upload(pl->d_bmul, tab.bmul));
    HIP_TRY(upload(pl->d_qmul, tab.qmul));
    HIP_TRY(upload(pl->d_beta, tab.beta));
    if (!tab.twist.empty()) HIP_TRY(upload(pl->d_twist, tab.twist));
    HIP_TRY(dev_alloc(&pl->d_tmul, tab.tmul.size() / 4));
    HIP_TRY(dev_alloc(&pl->d_mmod, tab.mmod.size() / 4));
    if (!tab.tmul.empty()) HIP_TRY(upload(pl->d_tmul, tab.tmul));
    if (!tab.mmod.empty()) HIP_TRY(upload(pl->d_mmod, tab.mmod));
    pl->ps = ps;
    pl->rho_valid = false;
    pl->P = P;
    pl->tab = std::move(tab);
    return SSP_OK;
}

// Engine layout of the plan's march: the option if set, else the autotuned choice (per
// transform kind).
int effective_variant(const ssp_plan *pl) {
    int v = pl->variant_opt;
    if (v < 0 && pl->tab.direct) {
        v = ssp::direct_variant(pl->P, pl->tab.direct);
    } else if (v < 0) {
        int lg = 0;
        while ((1 << lg) < pl->P) ++lg;
        const int idx = lg - 7;
        const int *table = v == -2 ? ssp::kTunedMixed : ssp::kTunedVariant;
        v = (idx >= 0 && idx < 9) ? table[idx] : 0;
    }
    return ssp::engine_variant_exists(pl->P, v) ? v : 0;
}

// Complex scratch elements of one solve's march (see ssp::set_work).
size_t solve_work_elems(const ssp_plan *pl) {
    return ssp::kWorkPerSolve * ssp::work_stride(pl->P, pl->tab.direct);
}

ssp::SolveDesc base_desc(const ssp_plan *pl) {
    ssp::SolveDesc d{};
    const float sg = static_cast<float>(pl->tab.ksign);
    d.kf = ssp::KWin{pl->d_k1, pl->d_k2, pl->d_kph, sg, nullptr};
    d.ki = ssp::KWin{pl->d_k1i ? pl->d_k1i : pl->d_k1, pl->d_k2, pl->d_kph, sg, nullptr};
    d.tw = pl->d_tw;
    d.twl = pl->d_twl;
    d.twl2 = pl->d_twl2;
    d.dmod = pl->d_dmod;
    d.post = pl->d_post;
    d.pre = pl->d_pre;
    d.postf = pl->d_postf ? pl->d_postf : pl->d_post;
    d.s = pl->d_s;
    d.bmul = pl->d_bmul;
    d.qmul = pl->d_qmul;
    d.beta = pl->d_beta;
    d.twist = pl->d_twist;
    d.N = pl->N;
    d.P = pl->P;
    d.p = pl->p;
    d.nmax = pl->nmax;
    d.tol2 = pl->tol * pl->tol;
    d.sigma = pl->sigma;
    const ssp::GridSpec g = ssp::grid_spec(pl->bc, pl->N, pl->H);
    d.dz = g.dz;
    d.zoff = g.zoff;
    d.dr = pl->dr;
    d.c0 = pl->c0;
    d.prof_mode = pl->prof_mode;
    d.v_rows = pl->v_rows;
    d.v_step0 = pl->v_step0;
    d.v = pl->d_v;
    d.vi = pl->d_vi;
    for (int i = 0; i < 8; ++i) d.env[i] = pl->env[i];
    d.out_every = pl->out_every;
    d.variant = effective_variant(pl);
    d.direct = pl->tab.direct;
    d.mirror = pl->d_mirror;
    d.tmul = pl->d_tmul;
    d.mmod = pl->d_mmod;
    d.engine = effective_engine(pl);
    // split lengths: Hankel phase steps w^{s D i} of the march's layout and of layout 0
    // (D = twice the layout's thread count; see SolveDesc)
    auto phase_steps = [&](float4 *h, int variant) {
        const long long P = pl->P, s = pl->N - 1, D = 2LL * ssp::engine_threads(pl->P, variant);
        for (int i = 0; i < 16; ++i) {
            const long long r = (((s % P) + P) % P) * ((D * i) % P) % P;
            const double ang = -2.0 * M_PI * static_cast<double>(r) / static_cast<double>(P);
            float f[4];
            ssp::split_df(std::cos(ang), f[0], f[2]);
            ssp::split_df(std::sin(ang), f[1], f[3]);
            h[i] = make_float4(f[0], f[1], f[2], f[3]);
        }
    };
    if (pl->P > ssp::kMaxEngineFFT && !pl->tab.direct) {
        phase_steps(d.hstep, d.variant);
        phase_steps(d.hstep0, 0);
    }
    return d;
}

long long first_output_step(long long n0, int out_every) {
    return (n0 / out_every + 1) * out_every;
}

int count_outputs(long long n0, int nsteps, int out_every) {
    if (out_every <= 0 || nsteps <= 0) return 0;
    long long first = first_output_step(n0, out_every);
    long long last = n0 + nsteps;
    if (first > last) return 0;
    return static_cast<int>((last - first) / out_every + 1);
}

ssp_status check_profile_range(const ssp_plan *pl, long long n0, int nsteps) {
    if (pl->prof_mode != ssp::PROF_TABLE_STEPS) return SSP_OK;
    if (n0 + 1 < pl->v_step0 + 1 || n0 + nsteps > pl->v_step0 + pl->v_rows)
        return fail(SSP_E_INVAL, "profile table does not cover the requested steps");
    return SSP_OK;
}

ssp_status ensure_out(ssp_plan *pl, size_t elems) {
    if (elems <= pl->out_cap) return SSP_OK;
    dev_free(pl->d_out_fld);
    dev_free(pl->d_out_tl);
    pl->out_cap = 0;
    HIP_TRY(dev_alloc(&pl->d_out_fld, elems));
    HIP_TRY(dev_alloc(&pl->d_out_tl, elems));
    pl->out_cap = elems;
    return SSP_OK;
}

ssp_status set_field_internal(ssp_plan *pl, const double *psi0) {
    std::vector<float> h(2 * static_cast<size_t>(pl->N));
    for (int i = 0; i < 2 * pl->N; ++i) {
        if (!std::isfinite(psi0[i])) return fail(SSP_E_INVAL, "non-finite starter value");
        h[i] = static_cast<float>(psi0[i]);
    }
    HIP_TRY(hipMemcpyAsync(pl->d_field, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice,
                           pl->stream));
    ssp::SolveDesc d = base_desc(pl);
    HIP_TRY(hipMemcpyAsync(pl->d_desc, &d, sizeof(d), hipMemcpyHostToDevice, pl->stream));
    HIP_TRY(ssp::launch_transform(pl->P, pl->tab.direct, 1, pl->d_desc, 1, pl->d_field, pl->d_field, nullptr,
                                  pl->stream));
    long long zero = 0;
    HIP_TRY(hipMemcpyAsync(pl->d_step, &zero, sizeof(zero), hipMemcpyHostToDevice, pl->stream));
    HIP_TRY(hipStreamSynchronize(pl->stream));
    pl->step_index = 0;
    pl->has_field = true;
    return SSP_OK;
}

}  // namespace

extern "C" {

const char *ssp_status_string(ssp_status s) {
    switch (s) {
        case SSP_OK: return "ok";
        case SSP_W_NOT_CONVERGED: return "warning: Neumann series not converged to tol";
        case SSP_E_INVAL: return "invalid argument";
        case SSP_E_NOMEM: return "out of memory";
        case SSP_E_DEVICE: return "HIP device error";
        case SSP_E_DIVERGED: return "Neumann series diverged";
        case SSP_E_UNSTABLE: return "unstable Pade coefficients";
        case SSP_E_STATE: return "invalid call order";
        case SSP_E_UNIMPL: return "not supported by this build";
    }
    return "unknown status";
}

const char *ssp_last_error(void) { return g_last_error.c_str(); }

int ssp_max_nz(void) { return kMaxP / 2; }

ssp_status ssp_plan_engine(const ssp_plan *pl, int *variant, int *threads, int *fft_length) {
    if (!pl) return fail(SSP_E_INVAL, "plan is NULL");
    const int v = effective_variant(pl);
    if (variant) *variant = v;
    if (threads) *threads = ssp::engine_threads(pl->P, v);
    if (fft_length) *fft_length = pl->P;
    return SSP_OK;
}

ssp_status ssp_pade_coefficients(double sigma, int pade_order, double alpha, double *b, double *g,
                                 double *C, double *d0, double *d) {
    if (!std::isfinite(sigma) || !(sigma > 0) || !std::isfinite(alpha))
        return fail(SSP_E_INVAL, "sigma must be finite and > 0, alpha finite");
    ssp::PadeSet ps;
    std::string err;
    if (!ssp::pade_coefficients(sigma, pade_order, alpha, ps, err)) return fail(SSP_E_INVAL, err);
    for (int j = 0; j < ps.p; ++j) {
        if (b) {
            b[2 * j] = ps.b[j].real();
            b[2 * j + 1] = ps.b[j].imag();
        }
        if (g) {
            std::complex<double> gj = ps.a[j] / ps.b[j];
            g[2 * j] = gj.real();
            g[2 * j + 1] = gj.imag();
        }
        if (d) {
            d[2 * j] = ps.d[j].real();
            d[2 * j + 1] = ps.d[j].imag();
        }
    }
    if (C) {
        C[0] = ps.C.real();
        C[1] = ps.C.imag();
    }
    if (d0) {
        d0[0] = ps.d0.real();
        d0[1] = ps.d0.imag();
    }
    return SSP_OK;
}

ssp_status ssp_plan_create(int Nz, double H, double f, double c0, double dr, int pade_order,
                           int neumann_max, double tol, ssp_plan **out) {
    return ssp_plan_create_bc(Nz, H, f, c0, dr, pade_order, neumann_max, tol, SSP_BC_DIRICHLET, out);
}

ssp_status ssp_plan_create_bc(int Nz, double H, double f, double c0, double dr, int pade_order,
                              int neumann_max, double tol, int bc, ssp_plan **out) {
    if (!out) return fail(SSP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (bc != SSP_BC_DIRICHLET && bc != SSP_BC_NEUMANN && bc != SSP_BC_PERIODIC)
        return fail(SSP_E_INVAL, "bc must be SSP_BC_DIRICHLET, SSP_BC_NEUMANN or SSP_BC_PERIODIC");
    if (Nz < 2) return fail(SSP_E_INVAL, "Nz must be >= 2");
    if (Nz > ssp_max_nz()) return fail(SSP_E_UNIMPL, "Nz above ssp_max_nz()");
    if (!(H > 0) || !(f > 0) || !(c0 > 0) || !(dr > 0) || !std::isfinite(H) || !std::isfinite(f) ||
        !std::isfinite(c0) || !std::isfinite(dr))
        return fail(SSP_E_INVAL, "H, f, c0 and dr must be finite and > 0");
    if (pade_order < 1 || pade_order > 12) return fail(SSP_E_INVAL, "pade_order must be in [1, 12]");
    if (neumann_max < 0) return fail(SSP_E_INVAL, "neumann_max must be >= 0");
    if (!(tol > 0) || !std::isfinite(tol)) return fail(SSP_E_INVAL, "tol must be finite and > 0");
    ssp_plan *pl = new (std::nothrow) ssp_plan;
    if (!pl) return fail(SSP_E_NOMEM, "host allocation failed");
    pl->N = Nz;
    pl->bc = bc;
    pl->H = H;
    pl->f = f;
    pl->c0 = c0;
    pl->dr = dr;
    pl->p = pade_order;
    pl->nmax = neumann_max;
    pl->tol = tol;
    pl->k0 = 2.0 * M_PI * f / c0;
    pl->sigma = pl->k0 * dr;
    ssp_status st = build_plan_tables(pl);
    if (st == SSP_OK) {
        hipError_t e = hipSuccess;
        if (e == hipSuccess) e = dev_alloc(&pl->d_field, Nz);
        if (e == hipSuccess) e = dev_alloc(&pl->d_work, solve_work_elems(pl));
        if (e == hipSuccess) e = dev_alloc(&pl->d_step, 1);
        if (e == hipSuccess) e = dev_alloc(&pl->d_stats, 1);
        if (e == hipSuccess) e = dev_alloc(&pl->d_desc, 1);
        if (e == hipSuccess) e = dev_alloc(&pl->d_v, Nz);
        pl->v_cap = Nz;
        if (e != hipSuccess) st = fail(SSP_E_NOMEM, hipGetErrorString(e));
    }
    if (st == SSP_OK) {
        // default environment: c = c0 everywhere, v = 0
        pl->vs.assign(Nz, 0.0);
        pl->vs_rows = 1;
        pl->v_rows = 1;
        pl->prof_mode = ssp::PROF_TABLE_FIXED;
        hipError_t e = hipMemset(pl->d_v, 0, sizeof(float) * Nz);
        if (e != hipSuccess) st = fail(SSP_E_DEVICE, hipGetErrorString(e));
    }
    if (st != SSP_OK) {
        ssp_plan_destroy(pl);
        return st;
    }
    *out = pl;
    return SSP_OK;
}

void ssp_plan_destroy(ssp_plan *pl) {
    if (!pl) return;
    if (pl->stream) (void)hipStreamSynchronize(pl->stream);
    else (void)hipDeviceSynchronize();
    drop_graph(pl);
    free_side_streams(pl);
    free_tables(pl);
    dev_free(pl->d_v);
    dev_free(pl->d_vi);
    dev_free(pl->d_field);
    dev_free(pl->d_work);
    dev_free(pl->d_bwork);
    dev_free(pl->d_snap);
    dev_free(pl->d_bstats);
    dev_free(pl->d_step);
    dev_free(pl->d_stats);
    dev_free(pl->d_desc);
    dev_free(pl->d_descs);
    dev_free(pl->d_out_fld);
    dev_free(pl->d_out_tl);
    dev_free(pl->d_plain);
    if (pl->d_dense_work) (void)hipFree(pl->d_dense_work);
    if (pl->h_active) (void)hipHostFree(pl->h_active);
    dev_free(pl->d_dense_xh);
    dev_free(pl->d_dense_xl);
    dev_free(pl->d_dense_expo);
    if (pl->d_plain_flags) (void)hipFree(pl->d_plain_flags);
    delete pl;
}

ssp_status ssp_plan_set_stream(ssp_plan *pl, void *hip_stream) {
    if (!pl) return fail(SSP_E_INVAL, "plan is NULL");
    drop_graph(pl);
    pl->stream = static_cast<hipStream_t>(hip_stream);
    return SSP_OK;
}

ssp_status ssp_plan_set_option(ssp_plan *pl, int key, double value) {
    if (!pl) return fail(SSP_E_INVAL, "plan is NULL");
    { const ssp_status sp_ = sync_pending(pl); if (sp_ != SSP_OK) return sp_; }
    drop_graph(pl);
    switch (key) {
        case SSP_OPT_ROTATION: {
            if (!std::isfinite(value) || std::fabs(value) > M_PI / 2)
                return fail(SSP_E_INVAL, "rotation must be finite with |alpha| <= pi/2");
            double old = pl->alpha;
            pl->alpha = value;
            ssp_status st = build_plan_tables(pl);
            if (st != SSP_OK) {
                std::string msg = g_last_error;
                pl->alpha = old;
                (void)build_plan_tables(pl);
                return fail(st, msg);
            }
            return SSP_OK;
        }
        case SSP_OPT_OUT_EVERY:
            if (!(value >= 1) || value != std::floor(value) || value > 1e9)
                return fail(SSP_E_INVAL, "out_every must be an integer >= 1");
            pl->out_every = static_cast<int>(value);
            return SSP_OK;
        case SSP_OPT_STREAM:
            pl->stream = reinterpret_cast<hipStream_t>(static_cast<uintptr_t>(value));
            return SSP_OK;
        case SSP_OPT_GRAPH:
            if (value != 0 && value != 1) return fail(SSP_E_INVAL, "graph must be 0 or 1");
            pl->use_graph = value == 1;
            drop_graph(pl);
            return SSP_OK;
        case SSP_OPT_ENGINE:
            if (value != SSP_ENGINE_FFT && value != SSP_ENGINE_DENSE && value != SSP_ENGINE_AUTO)
                return fail(SSP_E_INVAL, "engine must be SSP_ENGINE_FFT, SSP_ENGINE_DENSE or SSP_ENGINE_AUTO");
            if (value == SSP_ENGINE_DENSE && !dense_capable(pl))
                return fail(SSP_E_UNIMPL, "the dense engine runs Dirichlet plans with Nz <= ssp_max_dense_nz()");
            pl->engine = static_cast<int>(value);
            return SSP_OK;
        case SSP_OPT_PLAIN:
            if (value != 0 && value != 1) return fail(SSP_E_INVAL, "plain must be 0 or 1");
            pl->plain = static_cast<int>(value);
            return SSP_OK;
        case SSP_OPT_FORM:
            if (value == SSP_FORM_PRODUCT) return SSP_OK;
            if (value == SSP_FORM_SUM)
                return fail(SSP_E_UNIMPL, "the sum form is not built: its FP32 cancellation (sum |d_j| up to "
                                          "4e3) costs up to 12 bits per step; the product form evaluates the "
                                          "same approximant");
            return fail(SSP_E_INVAL, "form must be SSP_FORM_PRODUCT or SSP_FORM_SUM");
        case SSP_OPT_GAIN_LIMIT: {
            if (!(value >= 0) || !std::isfinite(value)) return fail(SSP_E_INVAL, "gain limit must be finite and >= 0");
            if (!(pl->tab.max_gain <= 1.0 + value))
                return fail(SSP_E_UNSTABLE, "max |e^{i sigma} R(x_l)| - 1 = " + std::to_string(pl->tab.max_gain - 1.0) +
                                                " exceeds the requested gain limit");
            pl->gain_limit = value;
            return SSP_OK;
        }
        case SSP_OPT_CONTRACTION_CHECK:
            if (value != 0 && value != 1) return fail(SSP_E_INVAL, "contraction check must be 0 or 1");
            pl->contraction_check = value == 1;
            return SSP_OK;
        case SSP_OPT_VARIANT:
            if (value != -2 && value != -1 && value != 0 && value != 1 && value != 2)
                return fail(SSP_E_INVAL, "variant must be -2, -1, 0, 1 or 2");
            pl->variant_opt = static_cast<int>(value);
            return SSP_OK;
        default:
            return fail(SSP_E_INVAL, "unknown option key");
    }
}

ssp_status ssp_plan_info(const ssp_plan *pl, double *sigma, double *k0, double *b, double *g,
                         double *C, double *d0, double *d) {
    if (!pl) return fail(SSP_E_INVAL, "plan is NULL");
    if (sigma) *sigma = pl->sigma;
    if (k0) *k0 = pl->k0;
    for (int j = 0; j < pl->p; ++j) {
        if (b) {
            b[2 * j] = pl->ps.b[j].real();
            b[2 * j + 1] = pl->ps.b[j].imag();
        }
        if (g) {
            std::complex<double> gj = pl->ps.a[j] / pl->ps.b[j];
            g[2 * j] = gj.real();
            g[2 * j + 1] = gj.imag();
        }
        if (d) {
            d[2 * j] = pl->ps.d[j].real();
            d[2 * j + 1] = pl->ps.d[j].imag();
        }
    }
    if (C) {
        C[0] = pl->ps.C.real();
        C[1] = pl->ps.C.imag();
    }
    if (d0) {
        d0[0] = pl->ps.d0.real();
        d0[1] = pl->ps.d0.imag();
    }
    return SSP_OK;
}

ssp_status ssp_plan_contraction(ssp_plan *pl, int iterations, double *bound, double *estimate) {
    if (!pl || iterations < 0 || iterations > 100000) return fail(SSP_E_INVAL, "plan is NULL or bad iteration count");
    std::vector<double> bd, est;
    ssp::neumann_contraction(pl->N, pl->H, pl->k0, pl->ps, pl->bc, estimate_rows(pl), pl->vs_rows, iterations, bd,
                             est);
    for (int j = 0; j < pl->p; ++j) {
        if (bound) bound[j] = bd[j];
        if (estimate) estimate[j] = est[j];
    }
    return SSP_OK;
}

ssp_status ssp_modal_starter(ssp_plan *pl, const double *c, int nsrc, const double *zs, int max_modes,
                             double *psi0, double *kappa, int *n_modes) {
    if (!pl || !c || !zs || !psi0 || nsrc < 1) return fail(SSP_E_INVAL, "NULL argument or nsrc < 1");
    if (pl->bc != ssp::kBcDirichlet) return fail(SSP_E_UNIMPL, "the modal starter is built for Dirichlet plans");
    if (pl->N > ssp::kMaxModalNz) return fail(SSP_E_UNIMPL, "Nz above the modal starter's limit (16384)");
    for (int q = 0; q < nsrc; ++q)
        if (!(zs[q] > 0) || !(zs[q] < pl->H)) return fail(SSP_E_INVAL, "every zs must lie inside (0, H)");
    const int N = pl->N;
    std::vector<double> v(N);
    for (int m = 0; m < N; ++m) {
        if (!std::isfinite(c[m]) || !(c[m] > 0)) return fail(SSP_E_INVAL, "sound speed must be finite and > 0");
        const double q = pl->c0 / c[m];
        v[m] = q * q - 1.0;
    }
    std::vector<double> u, kap;
    std::string err;
    const hipError_t e = ssp::modal_starter(N, pl->H, pl->k0, v, nsrc, zs, max_modes, pl->stream, u, kap, err);
    if (e != hipSuccess) {
        if (e == hipErrorOutOfMemory) return fail(SSP_E_NOMEM, err);
        return fail(SSP_E_DEVICE, err);
    }
    for (size_t i = 0; i < u.size(); ++i) {
        psi0[2 * i] = u[i];
        psi0[2 * i + 1] = 0.0;
    }
    if (kappa)
        for (size_t k = 0; k < kap.size(); ++k) kappa[k] = kap[k];
    if (n_modes) *n_modes = static_cast<int>(kap.size());
    return SSP_OK;
}

ssp_status ssp_set_absorber(ssp_plan *pl, const double *eta) {
    if (!pl) return fail(SSP_E_INVAL, "NULL plan");
    { const ssp_status sp_ = sync_pending(pl); if (sp_ != SSP_OK) return sp_; }
    drop_graph(pl);
    if (!eta) {
        if (pl->stream) HIP_TRY(hipStreamSynchronize(pl->stream));
        else HIP_TRY(hipDeviceSynchronize());
        dev_free(pl->d_vi);
        pl->h_eta.clear();
        pl->rho_valid = false;
        return SSP_OK;
    }
    std::vector<float> v(pl->N);
    for (int m = 0; m < pl->N; ++m) {
        if (!std::isfinite(eta[m])) return fail(SSP_E_INVAL, "non-finite absorber value");
        v[m] = static_cast<float>(eta[m]);
    }
    pl->h_eta.assign(eta, eta + pl->N);
    pl->rho_valid = false;
    if (!pl->d_vi) HIP_TRY(dev_alloc(&pl->d_vi, pl->N));
    HIP_TRY(hipMemcpyAsync(pl->d_vi, v.data(), pl->N * sizeof(float), hipMemcpyHostToDevice, pl->stream));
    HIP_TRY(hipStreamSynchronize(pl->stream));
    return SSP_OK;
}

ssp_status ssp_set_profile(ssp_plan *pl, int step0, int nsteps, const double *c) {
    if (!pl || !c) return fail(SSP_E_INVAL, "NULL argument");
    { const ssp_status sp_ = sync_pending(pl); if (sp_ != SSP_OK) return sp_; }
    drop_graph(pl);
    if (step0 < 0 || nsteps == 0 || nsteps < -1) return fail(SSP_E_INVAL, "bad step range");
    const int rows = nsteps == -1 ? 1 : nsteps;
    const size_t count = static_cast<size_t>(rows) * pl->N;
    std::vector<float> v(count);
    for (size_t i = 0; i < count; ++i) {
        if (!std::isfinite(c[i]) || !(c[i] > 0)) return fail(SSP_E_INVAL, "sound speed must be finite and > 0");
        const double q = pl->c0 / c[i];
        v[i] = static_cast<float>(q * q - 1.0);
    }
    if (count > pl->v_cap) {
        dev_free(pl->d_v);
        pl->v_cap = 0;
        HIP_TRY(dev_alloc(&pl->d_v, count));
        pl->v_cap = count;
    }
    HIP_TRY(hipMemcpyAsync(pl->d_v, v.data(), count * sizeof(float), hipMemcpyHostToDevice, pl->stream));
    HIP_TRY(hipStreamSynchronize(pl->stream));
    pl->v_rows = rows;
    pl->v_step0 = step0;
    pl->prof_mode = nsteps == -1 ? ssp::PROF_TABLE_FIXED : ssp::PROF_TABLE_STEPS;
    // rows kept in FP64 for the contraction estimate: the first, the middle and the last
    std::vector<int> pick = {0, rows / 2, rows - 1};
    pick.erase(std::unique(pick.begin(), pick.end()), pick.end());
    pl->vs.assign(pick.size() * static_cast<size_t>(pl->N), 0.0);
    for (size_t r = 0; r < pick.size(); ++r)
        for (int m = 0; m < pl->N; ++m) {
            const double q = pl->c0 / c[static_cast<size_t>(pick[r]) * pl->N + m];
            pl->vs[r * pl->N + m] = q * q - 1.0;
        }
    pl->vs_rows = static_cast<int>(pick.size());
    pl->rho_valid = false;
    return SSP_OK;
}

ssp_status ssp_set_profile_analytic(ssp_plan *pl, const ssp_env *env) {
    if (!pl || !env) return fail(SSP_E_INVAL, "NULL argument");
    { const ssp_status sp_ = sync_pending(pl); if (sp_ != SSP_OK) return sp_; }
    drop_graph(pl);
    const double e[8] = {env->munk_c1, env->munk_eps, env->munk_z1, env->eddy_amp,
                         env->eddy_r0, env->eddy_rr, env->eddy_z0, env->eddy_rz};
    for (double x : e)
        if (!std::isfinite(x)) return fail(SSP_E_INVAL, "non-finite environment parameter");
    if (!(env->munk_c1 > 0) || !(env->munk_z1 > 0)) return fail(SSP_E_INVAL, "bad Munk parameters");
    if (env->eddy_amp != 0 && (!(env->eddy_rr > 0) || !(env->eddy_rz > 0)))
        return fail(SSP_E_INVAL, "bad eddy widths");
    // the profile must stay positive: c >= munk_c1 (1 + eps (eta + e^-eta - 1)) - |amp|
    if (env->munk_c1 * (1 + std::min(0.0, env->munk_eps) * 10) - std::fabs(env->eddy_amp) <= 0)
        return fail(SSP_E_INVAL, "environment may give c <= 0");
    // range-independent part: the Munk potential on the grid, in FP64, stored as row 0 of
    // the profile table; the device adds the eddy term each step
    const int N = pl->N;
    const ssp::GridSpec g = ssp::grid_spec(pl->bc, N, pl->H);
    std::vector<float> v(N);
    for (int m = 0; m < N; ++m) {
        const double z = (m + g.zoff) * g.dz, eta = 2.0 * (z - e[2]) / e[2];
        const double c = e[0] * (1.0 + e[1] * (eta + std::exp(-eta) - 1.0));
        if (!(c > 0)) return fail(SSP_E_INVAL, "Munk profile gives c <= 0 on the grid");
        const double q = pl->c0 / c;
        v[m] = static_cast<float>(q * q - 1.0);
    }
    if (static_cast<size_t>(N) > pl->v_cap) {
        dev_free(pl->d_v);
        pl->v_cap = 0;
        HIP_TRY(dev_alloc(&pl->d_v, N));
        pl->v_cap = N;
    }
    HIP_TRY(hipMemcpyAsync(pl->d_v, v.data(), N * sizeof(float), hipMemcpyHostToDevice, pl->stream));
    HIP_TRY(hipStreamSynchronize(pl->stream));
    pl->v_rows = 1;
    pl->v_step0 = 0;
    for (int i = 0; i < 8; ++i) pl->env[i] = e[i];
    pl->prof_mode = ssp::PROF_ANALYTIC;
    // rows kept in FP64 for the contraction estimate: the Munk profile alone and with the
    // eddy at its centre range (its strongest)
    pl->vs_rows = e[3] != 0.0 ? 2 : 1;
    pl->vs.assign(static_cast<size_t>(pl->vs_rows) * N, 0.0);
    for (int r = 0; r < pl->vs_rows; ++r)
        for (int m = 0; m < N; ++m) {
            const double z = (m + g.zoff) * g.dz, eta = 2.0 * (z - e[2]) / e[2];
            double c = e[0] * (1.0 + e[1] * (eta + std::exp(-eta) - 1.0));
            if (r == 1) c -= e[3] * std::exp(-((z - e[6]) / e[7]) * ((z - e[6]) / e[7]));
            const double q = pl->c0 / c;
            pl->vs[static_cast<size_t>(r) * N + m] = q * q - 1.0;
        }
    pl->rho_valid = false;
    return SSP_OK;
}

ssp_status ssp_set_field(ssp_plan *pl, const double *psi0) {
    if (!pl || !psi0) return fail(SSP_E_INVAL, "NULL argument");
    { const ssp_status sp_ = sync_pending(pl); if (sp_ != SSP_OK) return sp_; }
    return set_field_internal(pl, psi0);
}

ssp_status ssp_get_field(const ssp_plan *cpl, double *psi) {
    ssp_plan *pl = const_cast<ssp_plan *>(cpl);
    if (!pl || !psi) return fail(SSP_E_INVAL, "NULL argument");
    { const ssp_status sp_ = sync_pending(pl); if (sp_ != SSP_OK) return sp_; }
    if (!pl->has_field) return fail(SSP_E_STATE, "no field set");
    ssp_status st = ensure_out(pl, pl->N);
    if (st != SSP_OK) return st;
    ssp::SolveDesc d = base_desc(pl);
    HIP_TRY(hipMemcpyAsync(pl->d_desc, &d, sizeof(d), hipMemcpyHostToDevice, pl->stream));
    HIP_TRY(ssp::launch_transform(pl->P, pl->tab.direct, 2, pl->d_desc, 1, pl->d_field, pl->d_out_fld, pl->d_step,
                                  pl->stream));
    std::vector<float> h(2 * static_cast<size_t>(pl->N));
    HIP_TRY(hipMemcpyAsync(h.data(), pl->d_out_fld, h.size() * sizeof(float), hipMemcpyDeviceToHost,
                           pl->stream));
    HIP_TRY(hipStreamSynchronize(pl->stream));
    for (size_t i = 0; i < h.size(); ++i) psi[i] = h[i];
    return SSP_OK;
}

int ssp_count_outputs(const ssp_plan *cpl, int nsteps) {
    ssp_plan *pl = const_cast<ssp_plan *>(cpl);
    if (!pl || sync_pending(pl) != SSP_OK) return 0;
    return count_outputs(pl->step_index, nsteps, pl->out_every);
}

ssp_status ssp_march(ssp_plan *pl, const double *psi0, int nsteps, double *field_out, float *tl_out,
                     ssp_stats *stats) {
    if (!pl) return fail(SSP_E_INVAL, "plan is NULL");
    if (nsteps < 0) return fail(SSP_E_INVAL, "nsteps must be >= 0");
    if (psi0) {
        ssp_status st = set_field_internal(pl, psi0);
        if (st != SSP_OK) return st;
    }
    if (!pl->has_field) return fail(SSP_E_STATE, "no field: pass psi0 or call ssp_set_field");
    ssp_plan *plans[1] = {pl};
    double *fo[1] = {field_out};
    float *to[1] = {tl_out};
    return ssp_march_batch(plans, 1, nsteps, fo, to, stats);
}

}  // extern "C"

namespace {

// ----------------------------------------------------------------------------- batches
// A batch prepared for launch: descriptors sorted into launch groups.  Groups: the
// uneven-length family of 1024-thread kernels (one launch), then one group per (FFT length,
// transform kind, layout), then the dense-engine groups, one per grid size (last, because
// their host-driven loop waits on its own stream while the FFT groups already run).
struct Group {
    int start, end;
    bool family, dense;
};
struct Prepared {
    std::vector<ssp::SolveDesc> sorted;
    std::vector<int> order;  // sorted position -> caller's index
    std::vector<Group> groups;
    size_t dense_bytes = 0;  // scratch of all dense groups together
};

bool in_family(const ssp::SolveDesc &d) {
    return d.engine == SSP_ENGINE_FFT && ssp::march_family_member(d.P) && d.variant == 0 && !d.direct;
}

void prepare_groups(const std::vector<ssp::SolveDesc> &descs, Prepared &b) {
    const int n = static_cast<int>(descs.size());
    b.order.resize(n);
    for (int i = 0; i < n; ++i) b.order[i] = i;
    auto rank = [](const ssp::SolveDesc &d) { return d.engine == SSP_ENGINE_DENSE ? 2 : (in_family(d) ? 0 : 1); };
    std::stable_sort(b.order.begin(), b.order.end(), [&](int x, int y) {
        const ssp::SolveDesc &p = descs[x], &q = descs[y];
        if (rank(p) != rank(q)) return rank(p) < rank(q);
        if (rank(p) == 2) {
            if (p.N != q.N) return p.N > q.N;
            return p.nsteps > q.nsteps;
        }
        if (p.P != q.P) return p.P > q.P;
        if (p.direct != q.direct) return p.direct < q.direct;
        if (p.variant != q.variant) return p.variant < q.variant;
        return p.nsteps > q.nsteps;
    });
    b.sorted.resize(n);
    for (int i = 0; i < n; ++i) b.sorted[i] = descs[b.order[i]];
    b.groups.clear();
    b.dense_bytes = 0;
    int nf = 0;
    while (nf < n && in_family(b.sorted[nf])) ++nf;
    if (nf > 0 && b.sorted[0].P != b.sorted[nf - 1].P) b.groups.push_back({0, nf, true, false});
    else nf = 0;
    for (int start = nf; start < n;) {
        const ssp::SolveDesc &h = b.sorted[start];
        const bool dense = h.engine == SSP_ENGINE_DENSE;
        int end = start;
        while (end < n) {
            const ssp::SolveDesc &d = b.sorted[end];
            const bool same = dense ? (d.engine == SSP_ENGINE_DENSE && d.N == h.N)
                                    : (d.engine != SSP_ENGINE_DENSE && d.P == h.P && d.variant == h.variant &&
                                       d.direct == h.direct);
            if (!same) break;
            ++end;
        }
        b.groups.push_back({start, end, false, dense});
        if (dense) b.dense_bytes += ssp::dense_work_bytes(end - start, h.N);
        start = end;
    }
}

bool has_dense(const Prepared &b) {
    for (const Group &g : b.groups)
        if (g.dense) return true;
    return false;
}

ssp_status ensure_dense_scratch(ssp_plan *owner, size_t bytes) {
    if (!owner->h_active) HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&owner->h_active), 64 * sizeof(int)));
    if (bytes <= owner->dense_work_cap) return SSP_OK;
    if (owner->d_dense_work) (void)hipFree(owner->d_dense_work);
    owner->d_dense_work = nullptr;
    owner->dense_work_cap = 0;
    HIP_TRY(hipMalloc(&owner->d_dense_work, bytes));
    owner->dense_work_cap = bytes;
    return SSP_OK;
}

// Issue a prepared batch whose sorted descriptors are on the device at d_descs.  Groups run
// concurrently: the first on `stream`, the others on the owner's side streams, forked from
// and joined back into `stream`.  Each group's march is followed by its output launches.
ssp_status launch_groups(ssp_plan *owner, const Prepared &b, const ssp::SolveDesc *d_descs, hipStream_t stream) {
    const int ng = static_cast<int>(b.groups.size());
    if (ng == 0) return SSP_OK;
    if (has_dense(b)) {
        ssp_status st = ensure_dense_scratch(owner, b.dense_bytes);
        if (st != SSP_OK) return st;
    }
    if (ng > 1) {
        HIP_TRY(ensure_side_streams(owner));
        HIP_TRY(hipEventRecord(owner->fork, stream));
    }
    size_t dense_off = 0;
    int dense_slot = 0;
    for (int g = 0; g < ng; ++g) {
        hipStream_t gs = g == 0 ? stream : owner->side[(g - 1) % kSideStreams];
        if (g > 0 && g <= kSideStreams) HIP_TRY(hipStreamWaitEvent(gs, owner->fork, 0));
        const Group &G = b.groups[g];
        int gmax = 0, pmax = 0, nmax_max = 0;
        for (int k = G.start; k < G.end; ++k) {
            gmax = std::max(gmax, b.sorted[k].nsteps);
            pmax = std::max(pmax, b.sorted[k].p);
            nmax_max = std::max(nmax_max, b.sorted[k].nmax);
        }
        const ssp::SolveDesc &h = b.sorted[G.start];
        if (G.dense) {
            ssp::DenseTables t;
            ssp_status st = dense_tables(h.N, t);
            if (st != SSP_OK) return st;
            const int B = G.end - G.start;
            const ssp::DenseWork w =
                ssp::carve_dense_work(static_cast<char *>(owner->d_dense_work) + dense_off, B, h.N);
            dense_off += ssp::dense_work_bytes(B, h.N);
            HIP_TRY(ssp::dense_march(t, d_descs + G.start, B, gmax, pmax, nmax_max, w,
                                     owner->h_active + (dense_slot++ % 64), gs));
        } else if (G.family) {
            HIP_TRY(ssp::launch_march_family(d_descs + G.start, G.end - G.start, gmax, gs));
        } else {
            HIP_TRY(ssp::launch_march(h.P, h.variant, h.direct, d_descs + G.start, G.end - G.start, gmax, gs));
        }
        for (int start = G.start; start < G.end;) {
            int end = start;
            while (end < G.end && b.sorted[end].P == b.sorted[start].P && b.sorted[end].direct == b.sorted[start].direct)
                ++end;
            int rows = 0;
            for (int k = start; k < end; ++k) rows = std::max(rows, b.sorted[k].snap ? b.sorted[k].nout : 0);
            HIP_TRY(ssp::launch_output(b.sorted[start].P, b.sorted[start].direct, d_descs + start, end - start, rows,
                                       gs));
            start = end;
        }
    }
    for (int j = 0; j < std::min(ng - 1, kSideStreams); ++j) {
        HIP_TRY(hipEventRecord(owner->join[j], owner->side[j]));
        HIP_TRY(hipStreamWaitEvent(stream, owner->join[j], 0));
    }
    return SSP_OK;
}

ssp_status upload_descs(ssp_plan *owner, const std::vector<ssp::SolveDesc> &sorted, hipStream_t stream) {
    const int n = static_cast<int>(sorted.size());
    if (owner->descs_cap < n) {
        drop_graph(owner);
        dev_free(owner->d_descs);
        owner->descs_cap = 0;
        HIP_TRY(dev_alloc(&owner->d_descs, n));
        owner->descs_cap = n;
    }
    HIP_TRY(hipMemcpyAsync(owner->d_descs, sorted.data(), n * sizeof(ssp::SolveDesc), hipMemcpyHostToDevice,
                           stream));
    return SSP_OK;
}

// Bring the host step counter of a plan marched by ssp_march_batch_async up to date.
ssp_status sync_pending(ssp_plan *pl) {
    if (!pl->async_pending) return SSP_OK;
    ssp::DevStats st{};
    HIP_TRY(hipStreamSynchronize(pl->pending_stream));
    HIP_TRY(hipMemcpy(&st, pl->d_stats, sizeof(st), hipMemcpyDeviceToHost));
    pl->step_index = st.step_index;
    pl->async_pending = false;
    return SSP_OK;
}

// Potential rows of the contraction estimate: the sampled profile rows plus i eta.
std::vector<std::complex<double>> estimate_rows(const ssp_plan *pl) {
    std::vector<std::complex<double>> v = pl->vs;
    if (!pl->h_eta.empty())
        for (int r = 0; r < pl->vs_rows; ++r)
            for (int m = 0; m < pl->N; ++m) v[static_cast<size_t>(r) * pl->N + m] += std::complex<double>(0, pl->h_eta[m]);
    return v;
}

constexpr int kGateIterations = 40;

// SSP_OPT_CONTRACTION_CHECK: the cached spectral-radius estimate of every factor's
// Neumann operator (Dirichlet plans); SSP_E_DIVERGED if one is >= 1.
ssp_status contraction_gate(ssp_plan *pl) {
    if (!pl->contraction_check || pl->nmax == 0 || pl->bc != ssp::kBcDirichlet) return SSP_OK;
    if (!pl->rho_valid) {
        std::vector<double> bound;
        ssp::neumann_contraction(pl->N, pl->H, pl->k0, pl->ps, pl->bc, estimate_rows(pl), pl->vs_rows,
                                 kGateIterations, bound, pl->rho_est);
        pl->rho_valid = true;
    }
    for (int j = 0; j < pl->p; ++j)
        if (!(pl->rho_est[j] < 1.0))
            return fail(SSP_E_DIVERGED, "Neumann operator of Pade factor " + std::to_string(j) +
                                            " has spectral radius ~" + std::to_string(pl->rho_est[j]) +
                                            " >= 1: the series cannot converge (contraction check)");
    return SSP_OK;
}

// Shared body of ssp_march_batch and ssp_march_batch_steps: plan i marches steps[i] steps.
ssp_status march_batch_impl(ssp_plan *const *plans, int n, const int *steps, double *const *field_out,
                            float *const *tl_out, ssp_stats *stats) {
    if (!plans || n <= 0) return fail(SSP_E_INVAL, "no plans");
    int nsteps = 0;  // the largest step count
    for (int i = 0; i < n; ++i) {
        if (steps[i] < 0) return fail(SSP_E_INVAL, "nsteps must be >= 0");
        nsteps = std::max(nsteps, steps[i]);
        if (!plans[i]) return fail(SSP_E_INVAL, "NULL plan in batch");
        if (!plans[i]->has_field) return fail(SSP_E_STATE, "plan without a field in batch");
        for (int k = 0; k < i; ++k)
            if (plans[k] == plans[i]) return fail(SSP_E_INVAL, "plan repeated in batch");
    }
    for (int i = 0; i < n; ++i) {
        ssp_status st = sync_pending(plans[i]);
        if (st == SSP_OK) st = check_profile_range(plans[i], plans[i]->step_index, steps[i]);
        if (st == SSP_OK && steps[i] > 0) st = contraction_gate(plans[i]);
        if (st != SSP_OK) return st;
    }
    hipStream_t stream = plans[0]->stream;
    std::vector<int> nout(n);
    std::vector<ssp::SolveDesc> descs(n);
    for (int i = 0; i < n; ++i) {
        ssp_plan *pl = plans[i];
        nout[i] = count_outputs(pl->step_index, steps[i], pl->out_every);
        ssp_status st = ensure_out(pl, static_cast<size_t>(nout[i]) * pl->N);
        if (st != SSP_OK) return st;
        ssp::SolveDesc d = base_desc(pl);
        d.field = pl->d_field;
        ssp::set_work(d, pl->d_work);
        d.step = pl->d_step;
        d.nout = nout[i];
        d.nsteps = steps[i];
        d.stats = pl->d_stats;
        // snapshots go to the field staging rows and are converted there in place
        d.fld_out = (field_out && field_out[i] && nout[i] > 0) ? pl->d_out_fld : nullptr;
        d.tl_out = (tl_out && tl_out[i] && nout[i] > 0) ? pl->d_out_tl : nullptr;
        d.snap = (d.fld_out || d.tl_out) ? pl->d_out_fld : nullptr;
        descs[i] = d;
    }
    ssp_plan *owner = plans[0];
    drop_graph(owner);  // d_descs is rewritten below
    Prepared b;
    prepare_groups(descs, b);
    ssp_status st0 = upload_descs(owner, b.sorted, stream);
    if (st0 != SSP_OK) return st0;
    const bool plain = n == 1 && owner->plain == 1;
    if (nsteps > 0) {
        if (plain) {
            // plain form: one kernel per stage, one solve
            ssp_plan *pl = owner;
            if (pl->tab.direct || b.sorted[0].engine != SSP_ENGINE_FFT)
                return fail(SSP_E_UNIMPL, "the plain form runs chirp-z transforms of the FFT engine only; plans with "
                                          "direct transforms (periodic Nz or Dirichlet Nz + 1 a power of two) or the "
                                          "dense engine run the fused march");
            if (!pl->d_plain) {
                HIP_TRY(dev_alloc(&pl->d_plain, 2 * static_cast<size_t>(pl->N)));
                HIP_TRY(hipMalloc(reinterpret_cast<void **>(&pl->d_plain_flags), ssp::plain_state_bytes()));
            }
            HIP_TRY(hipMemsetAsync(pl->d_plain_flags, 0, ssp::plain_state_bytes(), stream));
            ssp::DevStats z{};
            z.step_index = pl->step_index;
            HIP_TRY(hipMemcpyAsync(pl->d_stats, &z, sizeof(z), hipMemcpyHostToDevice, stream));
            HIP_TRY(ssp::plain_march(b.sorted[0], owner->d_descs, nsteps, pl->d_plain, pl->d_plain_flags, stream));
            if (b.sorted[0].snap)
                HIP_TRY(ssp::launch_output(b.sorted[0].P, false, owner->d_descs, 1, b.sorted[0].nout, stream));
        } else {
            ssp_status st = launch_groups(owner, b, owner->d_descs, stream);
            if (st != SSP_OK) return st;
        }
    }
    ssp_status worst = SSP_OK;
    std::vector<ssp::DevStats> hs(n);
    for (int i = 0; i < n; ++i)
        HIP_TRY(hipMemcpyAsync(&hs[i], plans[i]->d_stats, sizeof(ssp::DevStats), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    for (int i = 0; i < n; ++i) {
        ssp_plan *pl = plans[i];
        ssp::DevStats st = hs[i];
        if (steps[i] == 0) {
            st = ssp::DevStats{};
            st.step_index = pl->step_index;
        }
        if (plain && st.status == SSP_OK && st.not_converged > 0) st.status = SSP_W_NOT_CONVERGED;
        pl->step_index = st.step_index;
        const size_t cnt = static_cast<size_t>(nout[i]) * pl->N;
        if (field_out && field_out[i] && cnt) {
            std::vector<float> h(2 * cnt);
            HIP_TRY(hipMemcpy(h.data(), pl->d_out_fld, h.size() * sizeof(float), hipMemcpyDeviceToHost));
            for (size_t k = 0; k < h.size(); ++k) field_out[i][k] = h[k];
        }
        if (tl_out && tl_out[i] && cnt)
            HIP_TRY(hipMemcpy(tl_out[i], pl->d_out_tl, cnt * sizeof(float), hipMemcpyDeviceToHost));
        if (stats) std::memcpy(&stats[i], &st, sizeof(ssp_stats));
        ssp_status s = static_cast<ssp_status>(st.status);
        if (s < 0 && (worst >= 0 || s == SSP_E_DIVERGED)) worst = s;
        else if (s == SSP_W_NOT_CONVERGED && worst == SSP_OK) worst = SSP_W_NOT_CONVERGED;
    }
    if (worst == SSP_E_DIVERGED) g_last_error = "Neumann series diverged (per-plan statuses in the statistics)";
    else if (worst == SSP_E_INVAL) g_last_error = "a tabulated profile has no row for a step (per-plan statuses in the statistics)";
    return worst;
}

// Descriptors of a device-resident batch of B solves of one plan (ssp_march_device and its
// no-allocation variant): scratch base (solve_work_elems per solve), stats (d_stats or
// stats_base), snapshots (snap_base, nout rows per solve) and TL rows (d_tl).
std::vector<ssp::SolveDesc> device_descs(const ssp_plan *pl, int B, void *d_psi, void *d_step, int nsteps, int nout,
                                         void *d_tl, void *d_stats, float2 *work_base, ssp::DevStats *stats_base,
                                         float2 *snap_base) {
    std::vector<ssp::SolveDesc> descs(B);
    for (int b = 0; b < B; ++b) {
        ssp::SolveDesc d = base_desc(pl);
        d.field = static_cast<float2 *>(d_psi) + static_cast<size_t>(b) * pl->N;
        ssp::set_work(d, work_base + solve_work_elems(pl) * static_cast<size_t>(b));
        d.nout = nout;
        d.nsteps = nsteps;
        d.step = static_cast<long long *>(d_step) + b;
        d.stats = (d_stats ? static_cast<ssp::DevStats *>(d_stats) : stats_base) + b;
        d.tl_out = d_tl ? static_cast<float *>(d_tl) + static_cast<size_t>(b) * nout * pl->N : nullptr;
        d.fld_out = nullptr;
        if (nout == 0) d.tl_out = nullptr;
        d.snap = d.tl_out ? snap_base + static_cast<size_t>(b) * nout * pl->N : nullptr;
        descs[b] = d;
    }
    return descs;
}

// Launches of a device batch of one plan (descriptors already on the device).
ssp_status device_launch(ssp_plan *pl, const ssp::SolveDesc &h, const ssp::SolveDesc *d_descs, int B, int nsteps,
                         int nout, bool outputs) {
    if (h.engine == SSP_ENGINE_DENSE) {
        ssp::DenseTables t;
        ssp_status st = dense_tables(pl->N, t);
        if (st == SSP_OK) st = ensure_dense_scratch(pl, ssp::dense_work_bytes(B, pl->N));
        if (st != SSP_OK) return st;
        HIP_TRY(ssp::dense_march(t, d_descs, B, nsteps, pl->p, pl->nmax, ssp::carve_dense_work(pl->d_dense_work, B, pl->N),
                                 pl->h_active, pl->stream));
    } else {
        HIP_TRY(ssp::launch_march(pl->P, effective_variant(pl), pl->tab.direct, d_descs, B, nsteps, pl->stream));
    }
    if (outputs) HIP_TRY(ssp::launch_output(pl->P, pl->tab.direct, d_descs, B, nout, pl->stream));
    return SSP_OK;
}

}  // namespace

extern "C" {

ssp_status ssp_march_batch(ssp_plan *const *plans, int n, int nsteps, double *const *field_out,
                           float *const *tl_out, ssp_stats *stats) {
    if (n <= 0 || n > (1 << 24)) return fail(SSP_E_INVAL, "no plans");
    std::vector<int> steps(n, nsteps);
    return march_batch_impl(plans, n, steps.data(), field_out, tl_out, stats);
}

ssp_status ssp_march_batch_steps(ssp_plan *const *plans, int n, const int *nsteps, double *const *field_out,
                                 float *const *tl_out, ssp_stats *stats) {
    if (!nsteps) return fail(SSP_E_INVAL, "nsteps is NULL");
    return march_batch_impl(plans, n, nsteps, field_out, tl_out, stats);
}

ssp_status ssp_march_batch_async(ssp_plan *const *plans, int n, const int *nsteps, float *const *d_tl_out) {
    if (!plans || !nsteps || n <= 0 || n > (1 << 24)) return fail(SSP_E_INVAL, "bad argument");
    for (int i = 0; i < n; ++i) {
        if (!plans[i]) return fail(SSP_E_INVAL, "NULL plan in batch");
        if (nsteps[i] < 0) return fail(SSP_E_INVAL, "nsteps must be >= 0");
        if (!plans[i]->has_field) return fail(SSP_E_STATE, "plan without a field in batch");
        for (int k = 0; k < i; ++k)
            if (plans[k] == plans[i]) return fail(SSP_E_INVAL, "plan repeated in batch");
        if (plans[i]->async_pending && plans[i]->pending_stream != plans[0]->stream) {
            ssp_status st = sync_pending(plans[i]);
            if (st != SSP_OK) return st;
        }
    }
    ssp_plan *owner = plans[0];
    hipStream_t stream = owner->stream;
    // the recorded launches replay when the batch, its step counts, its output arrays and the
    // stream are those of the recording
    bool same = owner->use_graph && owner->bgraph_exec && owner->bkey_stream == stream &&
                static_cast<int>(owner->bkey_plans.size()) == n;
    for (int i = 0; same && i < n; ++i)
        same = owner->bkey_plans[i] == plans[i] && owner->bkey_steps[i] == nsteps[i] &&
               owner->bkey_tl[i] == static_cast<void *>(d_tl_out ? d_tl_out[i] : nullptr);
    if (same) {
        HIP_TRY(hipGraphLaunch(owner->bgraph_exec, stream));
    } else {
        std::vector<ssp::SolveDesc> descs(n);
        for (int i = 0; i < n; ++i) {
            ssp_plan *pl = plans[i];
            ssp_status st = contraction_gate(pl);
            if (st != SSP_OK) return st;
            // rows available: the largest number of output steps in nsteps steps (the kernels
            // place each row by the device step counter)
            const int nout = (pl->out_every > 0 && d_tl_out && d_tl_out[i]) ? nsteps[i] / pl->out_every + 1 : 0;
            st = ensure_out(pl, static_cast<size_t>(nout) * pl->N);
            if (st != SSP_OK) return st;
            ssp::SolveDesc d = base_desc(pl);
            d.field = pl->d_field;
            ssp::set_work(d, pl->d_work);
            d.step = pl->d_step;
            d.nout = nout;
            d.nsteps = nsteps[i];
            d.stats = pl->d_stats;
            d.fld_out = nullptr;
            d.tl_out = nout > 0 ? d_tl_out[i] : nullptr;
            d.snap = nout > 0 ? pl->d_out_fld : nullptr;
            descs[i] = d;
        }
        drop_graph(owner);
        Prepared b;
        prepare_groups(descs, b);
        ssp_status st = upload_descs(owner, b.sorted, stream);
        if (st != SSP_OK) return st;
        if (owner->use_graph && stream && !has_dense(b)) {
            // record the launches once (fork/join across the side streams becomes branches
            // of the graph); the descriptors above stay valid for later replays
            if (b.groups.size() > 1) HIP_TRY(ensure_side_streams(owner));
            HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
            st = launch_groups(owner, b, owner->d_descs, stream);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(stream, &g);
            if (st != SSP_OK || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                if (st != SSP_OK) return st;
                return fail(SSP_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e2));
            }
            owner->bgraph = g;
            HIP_TRY(hipGraphInstantiate(&owner->bgraph_exec, g, nullptr, nullptr, 0));
            owner->bkey_plans.assign(plans, plans + n);
            owner->bkey_steps.assign(nsteps, nsteps + n);
            owner->bkey_tl.assign(n, nullptr);
            for (int i = 0; i < n; ++i) owner->bkey_tl[i] = d_tl_out ? d_tl_out[i] : nullptr;
            owner->bkey_stream = stream;
            HIP_TRY(hipGraphLaunch(owner->bgraph_exec, stream));
        } else {
            st = launch_groups(owner, b, owner->d_descs, stream);
            if (st != SSP_OK) return st;
        }
    }
    for (int i = 0; i < n; ++i) {
        plans[i]->async_pending = true;
        plans[i]->pending_stream = stream;
    }
    return SSP_OK;
}

ssp_status ssp_batch_stats(ssp_plan *const *plans, int n, ssp_stats *stats) {
    if (!plans || n <= 0) return fail(SSP_E_INVAL, "bad argument");
    ssp_status worst = SSP_OK;
    for (int i = 0; i < n; ++i) {
        ssp_plan *pl = plans[i];
        if (!pl) return fail(SSP_E_INVAL, "NULL plan");
        ssp::DevStats st{};
        HIP_TRY(hipStreamSynchronize(pl->async_pending ? pl->pending_stream : pl->stream));
        HIP_TRY(hipMemcpy(&st, pl->d_stats, sizeof(st), hipMemcpyDeviceToHost));
        pl->step_index = st.step_index;
        pl->async_pending = false;
        if (stats) std::memcpy(&stats[i], &st, sizeof(ssp_stats));
        const ssp_status s = static_cast<ssp_status>(st.status);
        if (s < 0 && (worst >= 0 || s == SSP_E_DIVERGED)) worst = s;
        else if (s == SSP_W_NOT_CONVERGED && worst == SSP_OK) worst = SSP_W_NOT_CONVERGED;
    }
    return worst;
}

ssp_status ssp_march_device(ssp_plan *pl, int B, void *d_psi, void *d_step, int nsteps, void *d_tl,
                            void *d_stats) {
    if (!pl || B <= 0 || !d_psi || !d_step || nsteps < 0) return fail(SSP_E_INVAL, "bad argument");
    const bool dense = effective_engine(pl) == SSP_ENGINE_DENSE;
    const ssp_plan::GraphKey key{B, nsteps, d_psi, d_step, d_tl, d_stats, pl->stream};
    if (pl->use_graph && !dense && pl->graph_exec && pl->graph_key == key) {
        HIP_TRY(hipGraphLaunch(pl->graph_exec, pl->stream));
        return SSP_OK;
    }
    if (pl->use_graph && !pl->stream) return fail(SSP_E_INVAL, "graph replay needs a non-null stream");
    ssp_status st = contraction_gate(pl);
    if (st != SSP_OK) return st;
    if (pl->descs_cap < B) {
        drop_graph(pl);
        dev_free(pl->d_descs);
        pl->descs_cap = 0;
        HIP_TRY(dev_alloc(&pl->d_descs, B));
        pl->descs_cap = B;
    }
    // step counters live on the device and may differ between solves: each solve's output
    // rows are the output steps after its own counter (computed in the kernels); a
    // tabulated profile is checked against them in the kernels (a missing row stops that
    // solve with SSP_E_INVAL in its statistics)
    if (pl->bwork_cap < B) {
        dev_free(pl->d_bwork);
        pl->bwork_cap = 0;
        HIP_TRY(dev_alloc(&pl->d_bwork, solve_work_elems(pl) * static_cast<size_t>(B)));
        pl->bwork_cap = B;
    }
    if (!d_stats && pl->bstats_cap < B) {
        dev_free(pl->d_bstats);
        pl->bstats_cap = 0;
        HIP_TRY(dev_alloc(&pl->d_bstats, B));
        pl->bstats_cap = B;
    }
    // rows available per solve: the largest number of output steps in nsteps steps
    const int nout = pl->out_every > 0 ? nsteps / pl->out_every + 1 : 0;
    const size_t snap_elems = d_tl ? static_cast<size_t>(B) * nout * pl->N : 0;
    if (snap_elems > pl->snap_cap) {
        dev_free(pl->d_snap);
        pl->snap_cap = 0;
        HIP_TRY(dev_alloc(&pl->d_snap, snap_elems));
        pl->snap_cap = snap_elems;
    }
    const std::vector<ssp::SolveDesc> descs =
        device_descs(pl, B, d_psi, d_step, nsteps, nout, d_tl, d_stats, pl->d_bwork, pl->d_bstats, pl->d_snap);
    HIP_TRY(hipMemcpyAsync(pl->d_descs, descs.data(), B * sizeof(ssp::SolveDesc), hipMemcpyHostToDevice,
                           pl->stream));
    const bool outputs = d_tl && nout > 0;
    if (pl->use_graph && !dense) {
        // record the launches once; the descriptors above stay valid for later replays
        drop_graph(pl);
        HIP_TRY(hipStreamBeginCapture(pl->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = ssp::launch_march(pl->P, effective_variant(pl), pl->tab.direct, pl->d_descs, B, nsteps,
                                         pl->stream);
        if (e == hipSuccess && outputs) e = ssp::launch_output(pl->P, pl->tab.direct, pl->d_descs, B, nout, pl->stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(pl->stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(SSP_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
        }
        pl->graph = g;
        HIP_TRY(hipGraphInstantiate(&pl->graph_exec, g, nullptr, nullptr, 0));
        pl->graph_key = key;
        HIP_TRY(hipGraphLaunch(pl->graph_exec, pl->stream));
    } else {
        st = device_launch(pl, descs[0], pl->d_descs, B, nsteps, nout, outputs);
        if (st != SSP_OK) return st;
    }
    return SSP_OK;
}

}  // extern "C"

// ------------------------------------------------------------- no-allocation device march
// Scratch of ssp_march_device_noalloc: one array per device, held until the process ends.
// Host code never passes `scratch` itself to a kernel (its host-side name is not a device
// address); it passes the address hipGetSymbolAddress returns for the current device.
namespace {
constexpr size_t kNoAllocScratchBytes = static_cast<size_t>(SSP_NOALLOC_SCRATCH_MIB) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

ssp_status noalloc_scratch(unsigned char **out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static unsigned char *ptr[kMaxDevices] = {};
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SSP_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *addr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch)));
        if (!addr) return fail(SSP_E_DEVICE, "no device address for the scratch array");
        ptr[dev] = static_cast<unsigned char *>(addr);
    }
    *out = ptr[dev];
    return SSP_OK;
}

constexpr size_t round256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

// The descriptors of a device batch, written on the device from the plan's template (the
// same values device_descs builds on the host): no host buffer, no host-to-device copy.
__global__ void k_fill_descs(ssp::SolveDesc tmpl, int B, float2 *psi, long long *step, float *tl,
                             ssp::DevStats *stats, float2 *work, float2 *snap, ssp::SolveDesc *out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const size_t N = static_cast<size_t>(tmpl.N), bb = static_cast<size_t>(b);
    ssp::SolveDesc d = tmpl;
    d.field = psi + bb * N;
    const size_t S = ssp::work_stride(tmpl.P, tmpl.direct);
    d.work = work + ssp::kWorkPerSolve * bb * S;
    d.pot = d.work + S;
    d.wacc = d.work + 2 * S;
    d.xs = d.work + 3 * S;
    d.step = step + b;
    d.stats = stats + b;
    d.fld_out = nullptr;
    d.tl_out = tl ? tl + bb * tmpl.nout * N : nullptr;
    d.snap = tl ? snap + bb * tmpl.nout * N : nullptr;
    out[b] = d;
}
}  // namespace

extern "C" {

ssp_status ssp_march_device_noalloc(ssp_plan *pl, int B, void *d_psi, void *d_step, int nsteps, void *d_tl,
                                    void *d_stats) {
    if (!pl || B <= 0 || !d_psi || !d_step || nsteps < 0) return fail(SSP_E_INVAL, "bad argument");
    if (effective_engine(pl) != SSP_ENGINE_FFT)
        return fail(SSP_E_UNIMPL, "the no-allocation march runs the FFT engine (set SSP_OPT_ENGINE to SSP_ENGINE_FFT)");
    const int nout = pl->out_every > 0 ? nsteps / pl->out_every + 1 : 0;
    const bool outputs = d_tl && nout > 0;
    // scratch layout: descriptors, per-solve work, statistics (when the caller passes none),
    // output snapshots
    const size_t desc_bytes = round256(sizeof(ssp::SolveDesc) * static_cast<size_t>(B));
    const size_t work_bytes = round256(sizeof(float2) * solve_work_elems(pl) * static_cast<size_t>(B));
    const size_t stats_bytes = d_stats ? 0 : round256(sizeof(ssp::DevStats) * static_cast<size_t>(B));
    const size_t snap_bytes = outputs ? round256(sizeof(float2) * static_cast<size_t>(B) * nout * pl->N) : 0;
    const size_t need = desc_bytes + work_bytes + stats_bytes + snap_bytes;
    if (need > kNoAllocScratchBytes)
        return fail(SSP_E_INVAL, "batch needs more scratch than the fixed " +
                                     std::to_string(SSP_NOALLOC_SCRATCH_MIB) + " MiB of the no-allocation march");
    unsigned char *base = nullptr;
    ssp_status st = noalloc_scratch(&base);
    if (st != SSP_OK) return st;
    auto *d_descs = reinterpret_cast<ssp::SolveDesc *>(base);
    auto *work = reinterpret_cast<float2 *>(base + desc_bytes);
    auto *stats = reinterpret_cast<ssp::DevStats *>(base + desc_bytes + work_bytes);
    auto *snap = reinterpret_cast<float2 *>(base + desc_bytes + work_bytes + stats_bytes);
    ssp::SolveDesc tmpl = base_desc(pl);
    tmpl.nout = nout;
    tmpl.nsteps = nsteps;
    hipLaunchKernelGGL(k_fill_descs, dim3((B + 255) / 256), dim3(256), 0, pl->stream, tmpl, B,
                       static_cast<float2 *>(d_psi), static_cast<long long *>(d_step),
                       outputs ? static_cast<float *>(d_tl) : nullptr,
                       d_stats ? static_cast<ssp::DevStats *>(d_stats) : stats, work, snap, d_descs);
    HIP_TRY(hipGetLastError());
    HIP_TRY(ssp::launch_march(pl->P, effective_variant(pl), pl->tab.direct, d_descs, B, nsteps, pl->stream));
    if (outputs) HIP_TRY(ssp::launch_output(pl->P, pl->tab.direct, d_descs, B, nout, pl->stream));
    return SSP_OK;
}

ssp_status ssp_to_sine(ssp_plan *pl, int B, const void *d_phys, void *d_sine) {
    if (!pl || B <= 0 || !d_phys || !d_sine) return fail(SSP_E_INVAL, "bad argument");
    ssp::SolveDesc d = base_desc(pl);
    HIP_TRY(hipMemcpyAsync(pl->d_desc, &d, sizeof(d), hipMemcpyHostToDevice, pl->stream));
    HIP_TRY(ssp::launch_transform(pl->P, pl->tab.direct, 1, pl->d_desc, B, static_cast<const float2 *>(d_phys),
                                  static_cast<float2 *>(d_sine), nullptr, pl->stream));
    return SSP_OK;
}

ssp_status ssp_from_sine(ssp_plan *pl, int B, const void *d_sine, const void *d_step, void *d_phys) {
    if (!pl || B <= 0 || !d_sine || !d_step || !d_phys) return fail(SSP_E_INVAL, "bad argument");
    ssp::SolveDesc d = base_desc(pl);
    HIP_TRY(hipMemcpyAsync(pl->d_desc, &d, sizeof(d), hipMemcpyHostToDevice, pl->stream));
    HIP_TRY(ssp::launch_transform(pl->P, pl->tab.direct, 2, pl->d_desc, B, static_cast<const float2 *>(d_sine),
                                  static_cast<float2 *>(d_phys), static_cast<const long long *>(d_step),
                                  pl->stream));
    return SSP_OK;
}

ssp_status ssp_dst_device(ssp_plan *pl, int B, const void *d_in, void *d_out) {
    if (!pl || B <= 0 || !d_in || !d_out) return fail(SSP_E_INVAL, "bad argument");
    ssp::SolveDesc d = base_desc(pl);
    HIP_TRY(hipMemcpyAsync(pl->d_desc, &d, sizeof(d), hipMemcpyHostToDevice, pl->stream));
    HIP_TRY(ssp::launch_transform(pl->P, pl->tab.direct, 0, pl->d_desc, B, static_cast<const float2 *>(d_in),
                                  static_cast<float2 *>(d_out), nullptr, pl->stream));
    return SSP_OK;
}

int ssp_max_dense_nz(void) { return ssp::kMaxDenseNz; }

ssp_status ssp_dst_dense_device(ssp_plan *pl, int B, const void *d_in, void *d_out) {
    if (!pl || B <= 0 || !d_in || !d_out) return fail(SSP_E_INVAL, "bad argument");
    if (pl->N > ssp::kMaxDenseNz) return fail(SSP_E_UNIMPL, "Nz above ssp_max_dense_nz()");
    if (pl->bc != ssp::kBcDirichlet) return fail(SSP_E_UNIMPL, "the dense transform is the DST-I (Dirichlet plans)");
    if (B > (1 << 20)) return fail(SSP_E_INVAL, "B too large");
    ssp::DenseTables t;
    ssp_status st = dense_tables(pl->N, t);
    if (st != SSP_OK) return st;
    if (pl->dense_cols_cap < 2 * B) {
        dev_free(pl->d_dense_xh);
        dev_free(pl->d_dense_xl);
        dev_free(pl->d_dense_expo);
        pl->dense_cols_cap = 0;
        HIP_TRY(dev_alloc(&pl->d_dense_xh, static_cast<size_t>(2 * B) * t.kpad));
        HIP_TRY(dev_alloc(&pl->d_dense_xl, static_cast<size_t>(2 * B) * t.kpad));
        HIP_TRY(dev_alloc(&pl->d_dense_expo, static_cast<size_t>(2 * B)));
        pl->dense_cols_cap = 2 * B;
    }
    HIP_TRY(ssp::launch_dense_dst(t, B, static_cast<const float2 *>(d_in), static_cast<float2 *>(d_out),
                                  pl->d_dense_xh, pl->d_dense_xl, pl->d_dense_expo, pl->stream));
    return SSP_OK;
}

}  // extern "C"
