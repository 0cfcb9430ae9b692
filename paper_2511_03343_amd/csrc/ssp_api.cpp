// ssp_api.cpp - the C ABI (include/ssp.h): argument checks, plan and device-memory
// ownership, host<->device copies and kernel launches.
#include "../../include/ssp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
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
    int out_every = 1, engine = 0;
    int bc = ssp::kBcDirichlet;         // boundary condition (Sec. 3.1)
    int variant_opt = -1;               // SSP_OPT_VARIANT
    hipStream_t stream = nullptr;
    ssp::PadeSet ps;
    ssp::DeviceTables tab;
    // device tables
    float2 *d_k1 = nullptr, *d_k2 = nullptr, *d_dmod = nullptr, *d_post = nullptr, *d_pre = nullptr;
    float2 *d_k1i = nullptr, *d_k2i = nullptr, *d_postf = nullptr;  // only where they differ
    float4 *d_mirror = nullptr;         // odd-extension image factors (direct sine transform)
    const float4 *d_twl = nullptr;      // shared last-pass twiddles of 1024-thread engines (not owned)
    uint32_t *d_tw = nullptr;
    float4 *d_s = nullptr, *d_bmul = nullptr, *d_alpha = nullptr, *d_beta = nullptr;
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
    float2 *d_bwork = nullptr;          // scratch of a device batch [cap][kWorkPerSolve N]
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
    // dense DST (matrix cores): S parts and split-operand scratch
    _Float16 *d_dense_sh = nullptr, *d_dense_sl = nullptr;
    int dense_kpad = 0;
    _Float16 *d_dense_xh = nullptr, *d_dense_xl = nullptr;
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
    dev_free(pl->d_k1i);
    dev_free(pl->d_k2i);
    dev_free(pl->d_postf);
    dev_free(pl->d_mirror);
    dev_free(pl->d_dmod);
    dev_free(pl->d_post);
    dev_free(pl->d_pre);
    dev_free(pl->d_tw);
    dev_free(pl->d_s);
    dev_free(pl->d_bmul);
    dev_free(pl->d_alpha);
    dev_free(pl->d_beta);
    dev_free(pl->d_twist);
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
    if (!(tab.max_gain <= 1.0 + 1e-6))
        return fail(SSP_E_UNSTABLE, "max |e^{i sigma} R(x_l)| = " + std::to_string(tab.max_gain) +
                                        " exceeds 1 + 1e-6");
    if (!ssp::fft_length_supported(tab.P)) return fail(SSP_E_UNIMPL, "unsupported FFT length");
    free_tables(pl);
    const int N = pl->N, P = tab.P, p = ps.p;
    HIP_TRY(dev_alloc(&pl->d_k1, tab.k1.size() / 2));   // [P], none for direct transforms
    HIP_TRY(dev_alloc(&pl->d_k2, tab.k2.size() / 2));
    HIP_TRY(dev_alloc(&pl->d_tw, tab.twiddle.size()));
    HIP_TRY(dev_alloc(&pl->d_dmod, N));
    HIP_TRY(dev_alloc(&pl->d_post, N));
    HIP_TRY(dev_alloc(&pl->d_pre, N));
    HIP_TRY(dev_alloc(&pl->d_s, static_cast<size_t>(p) * N));
    HIP_TRY(dev_alloc(&pl->d_bmul, static_cast<size_t>(p) * N));
    HIP_TRY(dev_alloc(&pl->d_alpha, p));
    HIP_TRY(dev_alloc(&pl->d_beta, p));
    HIP_TRY(dev_alloc(&pl->d_twist, tab.twist.size() / 4));
    HIP_TRY(dev_alloc(&pl->d_k1i, tab.k1i.size() / 2));
    HIP_TRY(dev_alloc(&pl->d_k2i, tab.k2i.size() / 2));
    HIP_TRY(dev_alloc(&pl->d_postf, tab.postf.size() / 2));
    if (!tab.k1i.empty()) HIP_TRY(upload(pl->d_k1i, tab.k1i));
    if (!tab.k2i.empty()) HIP_TRY(upload(pl->d_k2i, tab.k2i));
    if (!tab.postf.empty()) HIP_TRY(upload(pl->d_postf, tab.postf));
    HIP_TRY(dev_alloc(&pl->d_mirror, tab.mirror.size() / 4));
    if (!tab.mirror.empty()) HIP_TRY(upload(pl->d_mirror, tab.mirror));
    if (!tab.k1.empty()) HIP_TRY(upload(pl->d_k1, tab.k1));
    if (!tab.k2.empty()) HIP_TRY(upload(pl->d_k2, tab.k2));
    HIP_TRY(upload(pl->d_tw, tab.twiddle));
    HIP_TRY(ssp::last_twiddles(P, pl->d_tw, &pl->d_twl));
    HIP_TRY(upload(pl->d_dmod, tab.dmod));
    HIP_TRY(upload(pl->d_post, tab.post));
    HIP_TRY(upload(pl->d_pre, tab.pre));
    HIP_TRY(upload(pl->d_s, tab.s));
    HIP_TRY(upload(pl->d_bmul, tab.bmul));
    HIP_TRY(upload(pl->d_alpha, tab.alpha));
    HIP_TRY(upload(pl->d_beta, tab.beta));
    if (!tab.twist.empty()) HIP_TRY(upload(pl->d_twist, tab.twist));
    pl->ps = ps;
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
        v = (idx >= 0 && idx < 9) ? ssp::kTunedVariant[idx] : 0;
    }
    return ssp::engine_variant_exists(pl->P, v) ? v : 0;
}

ssp::SolveDesc base_desc(const ssp_plan *pl) {
    ssp::SolveDesc d{};
    d.k1 = pl->d_k1;
    d.k2 = pl->d_k2;
    d.k1i = pl->d_k1i ? pl->d_k1i : pl->d_k1;
    d.k2i = pl->d_k2i ? pl->d_k2i : pl->d_k2;
    d.tw = pl->d_tw;
    d.twl = pl->d_twl;
    d.dmod = pl->d_dmod;
    d.post = pl->d_post;
    d.pre = pl->d_pre;
    d.postf = pl->d_postf ? pl->d_postf : pl->d_post;
    d.s = pl->d_s;
    d.bmul = pl->d_bmul;
    d.alpha = pl->d_alpha;
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
        if (e == hipSuccess) e = dev_alloc(&pl->d_work, ssp::kWorkPerSolve * static_cast<size_t>(Nz));
        if (e == hipSuccess) e = dev_alloc(&pl->d_step, 1);
        if (e == hipSuccess) e = dev_alloc(&pl->d_stats, 1);
        if (e == hipSuccess) e = dev_alloc(&pl->d_desc, 1);
        if (e == hipSuccess) e = dev_alloc(&pl->d_v, Nz);
        pl->v_cap = Nz;
        if (e != hipSuccess) st = fail(SSP_E_NOMEM, hipGetErrorString(e));
    }
    if (st == SSP_OK) {
        // default environment: c = c0 everywhere, v = 0
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
    dev_free(pl->d_dense_sh);
    dev_free(pl->d_dense_sl);
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
            if (value != 0 && value != 1) return fail(SSP_E_INVAL, "engine must be 0 or 1");
            pl->engine = static_cast<int>(value);
            return SSP_OK;
        case SSP_OPT_VARIANT:
            if (value != -1 && value != 0 && value != 1 && value != 2)
                return fail(SSP_E_INVAL, "variant must be -1, 0, 1 or 2");
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
    drop_graph(pl);
    if (!eta) {
        if (pl->stream) HIP_TRY(hipStreamSynchronize(pl->stream));
        else HIP_TRY(hipDeviceSynchronize());
        dev_free(pl->d_vi);
        return SSP_OK;
    }
    std::vector<float> v(pl->N);
    for (int m = 0; m < pl->N; ++m) {
        if (!std::isfinite(eta[m])) return fail(SSP_E_INVAL, "non-finite absorber value");
        v[m] = static_cast<float>(eta[m]);
    }
    if (!pl->d_vi) HIP_TRY(dev_alloc(&pl->d_vi, pl->N));
    HIP_TRY(hipMemcpyAsync(pl->d_vi, v.data(), pl->N * sizeof(float), hipMemcpyHostToDevice, pl->stream));
    HIP_TRY(hipStreamSynchronize(pl->stream));
    return SSP_OK;
}

ssp_status ssp_set_profile(ssp_plan *pl, int step0, int nsteps, const double *c) {
    if (!pl || !c) return fail(SSP_E_INVAL, "NULL argument");
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
    return SSP_OK;
}

ssp_status ssp_set_profile_analytic(ssp_plan *pl, const ssp_env *env) {
    if (!pl || !env) return fail(SSP_E_INVAL, "NULL argument");
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
    return SSP_OK;
}

ssp_status ssp_set_field(ssp_plan *pl, const double *psi0) {
    if (!pl || !psi0) return fail(SSP_E_INVAL, "NULL argument");
    return set_field_internal(pl, psi0);
}

ssp_status ssp_get_field(const ssp_plan *cpl, double *psi) {
    ssp_plan *pl = const_cast<ssp_plan *>(cpl);
    if (!pl || !psi) return fail(SSP_E_INVAL, "NULL argument");
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

int ssp_count_outputs(const ssp_plan *pl, int nsteps) {
    if (!pl) return 0;
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
        ssp_status st = check_profile_range(plans[i], plans[i]->step_index, steps[i]);
        if (st != SSP_OK) return st;
    }
    hipStream_t stream = plans[0]->stream;
    // descriptors, grouped by FFT length
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
    if (owner->descs_cap < n) {
        dev_free(owner->d_descs);
        owner->descs_cap = 0;
        HIP_TRY(dev_alloc(&owner->d_descs, n));
        owner->descs_cap = n;
    }
    // order by FFT length, longest first: each length is a contiguous range, the lengths that
    // share the 1024-thread kernel come first (one launch), and the longest solves are
    // dispatched first
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    // (the family: lengths of the 1024-thread kernel in their default layout)
    auto fam = [](const ssp::SolveDesc &d) {
        return ssp::march_family_member(d.P) && d.variant == 0 && !d.direct;
    };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const ssp::SolveDesc &a = descs[x], &b = descs[y];
        if (fam(a) != fam(b)) return fam(a);
        if (a.P != b.P) return a.P > b.P;
        if (a.direct != b.direct) return a.direct < b.direct;
        if (a.variant != b.variant) return a.variant < b.variant;
        return a.nsteps > b.nsteps;
    });
    std::vector<ssp::SolveDesc> sorted(n);
    for (int i = 0; i < n; ++i) sorted[i] = descs[order[i]];
    HIP_TRY(hipMemcpyAsync(owner->d_descs, sorted.data(), n * sizeof(ssp::SolveDesc),
                           hipMemcpyHostToDevice, stream));
    if (nsteps > 0) {
        if (n == 1 && owner->engine == 1) {
            // plain form: one kernel per stage, one solve
            ssp_plan *pl = owner;
            if (pl->tab.direct)
                return fail(SSP_E_UNIMPL, "the plain form runs chirp-z transforms only; plans with direct "
                                          "transforms (periodic Nz or Dirichlet Nz + 1 a power of two) run "
                                          "the fused kernel");
            if (!pl->d_plain) {
                HIP_TRY(dev_alloc(&pl->d_plain, 2 * static_cast<size_t>(pl->N)));
                HIP_TRY(hipMalloc(reinterpret_cast<void **>(&pl->d_plain_flags), ssp::plain_state_bytes()));
            }
            HIP_TRY(hipMemsetAsync(pl->d_plain_flags, 0, ssp::plain_state_bytes(), stream));
            long long idx = pl->step_index;
            ssp::DevStats z{};
            z.step_index = idx;
            HIP_TRY(hipMemcpyAsync(pl->d_stats, &z, sizeof(z), hipMemcpyHostToDevice, stream));
            HIP_TRY(ssp::plain_march(sorted[0], owner->d_descs, nsteps, pl->d_plain, pl->d_plain_flags, stream));
            if (sorted[0].snap) HIP_TRY(ssp::launch_output(sorted[0].P, false, owner->d_descs, 1, sorted[0].nout, stream));
        } else {
            // launch groups: the 1024-thread lengths together (one launch), then one per other
            // length; each group's march is followed by its output launches (one per length)
            struct Group { int start, end; bool family; };
            std::vector<Group> groups;
            int nf = 0;
            while (nf < n && fam(sorted[nf])) ++nf;
            if (nf > 0 && sorted[0].P != sorted[nf - 1].P) groups.push_back({0, nf, true});
            else nf = 0;
            for (int start = nf; start < n;) {
                int end = start;
                while (end < n && sorted[end].P == sorted[start].P && sorted[end].variant == sorted[start].variant &&
                       sorted[end].direct == sorted[start].direct)
                    ++end;
                groups.push_back({start, end, false});
                start = end;
            }
            // groups run concurrently: the first on the caller's stream, the others on the
            // plan's side streams, forked from and joined back into the caller's stream
            const int ng = static_cast<int>(groups.size());
            if (ng > 1) {
                HIP_TRY(ensure_side_streams(owner));
                HIP_TRY(hipEventRecord(owner->fork, stream));
            }
            for (int g = 0; g < ng; ++g) {
                hipStream_t gs = g == 0 ? stream : owner->side[(g - 1) % kSideStreams];
                if (g > 0) HIP_TRY(hipStreamWaitEvent(gs, owner->fork, 0));
                const Group &G = groups[g];
                int gmax = 0;
                for (int k = G.start; k < G.end; ++k) gmax = std::max(gmax, sorted[k].nsteps);
                if (G.family)
                    HIP_TRY(ssp::launch_march_family(owner->d_descs + G.start, G.end - G.start, gmax, gs));
                else
                    HIP_TRY(ssp::launch_march(sorted[G.start].P, sorted[G.start].variant, sorted[G.start].direct,
                                              owner->d_descs + G.start, G.end - G.start, gmax, gs));
                for (int start = G.start; start < G.end;) {
                    int end = start;
                    while (end < G.end && sorted[end].P == sorted[start].P && sorted[end].direct == sorted[start].direct)
                        ++end;
                    int rows = 0;
                    for (int k = start; k < end; ++k) rows = std::max(rows, sorted[k].snap ? sorted[k].nout : 0);
                    HIP_TRY(ssp::launch_output(sorted[start].P, sorted[start].direct, owner->d_descs + start,
                                               end - start, rows, gs));
                    start = end;
                }
            }
            for (int j = 0; j < std::min(ng - 1, kSideStreams); ++j) {
                HIP_TRY(hipEventRecord(owner->join[j], owner->side[j]));
                HIP_TRY(hipStreamWaitEvent(stream, owner->join[j], 0));
            }
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
        if (pl->engine == 1 && n == 1 && st.status == SSP_OK && st.not_converged > 0)
            st.status = SSP_W_NOT_CONVERGED;
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
        if (s == SSP_E_DIVERGED) worst = SSP_E_DIVERGED;
        else if (s == SSP_W_NOT_CONVERGED && worst == SSP_OK) worst = SSP_W_NOT_CONVERGED;
    }
    if (worst == SSP_E_DIVERGED) g_last_error = "Neumann series diverged";
    return worst;
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

ssp_status ssp_march_device(ssp_plan *pl, int B, void *d_psi, void *d_step, int nsteps, void *d_tl,
                            void *d_stats) {
    if (!pl || B <= 0 || !d_psi || !d_step || nsteps < 0) return fail(SSP_E_INVAL, "bad argument");
    const ssp_plan::GraphKey key{B, nsteps, d_psi, d_step, d_tl, d_stats, pl->stream};
    if (pl->use_graph && pl->graph_exec && pl->graph_key == key) {
        HIP_TRY(hipGraphLaunch(pl->graph_exec, pl->stream));
        return SSP_OK;
    }
    if (pl->use_graph && !pl->stream) return fail(SSP_E_INVAL, "graph replay needs a non-null stream");
    ssp_status st = check_profile_range(pl, 0, 0);
    if (st != SSP_OK) return st;
    if (pl->descs_cap < B) {
        dev_free(pl->d_descs);
        pl->descs_cap = 0;
        HIP_TRY(dev_alloc(&pl->d_descs, B));
        pl->descs_cap = B;
    }
    // step counters live on the device and may differ between solves: each solve's output
    // rows are the output steps after its own counter (computed in the kernels)
    if (pl->bwork_cap < B) {
        dev_free(pl->d_bwork);
        pl->bwork_cap = 0;
        HIP_TRY(dev_alloc(&pl->d_bwork, ssp::kWorkPerSolve * static_cast<size_t>(B) * pl->N));
        pl->bwork_cap = B;
    }
    if (!d_stats && pl->bstats_cap < B) {
        dev_free(pl->d_bstats);
        pl->bstats_cap = 0;
        HIP_TRY(dev_alloc(&pl->d_bstats, B));
        pl->bstats_cap = B;
    }
    std::vector<ssp::SolveDesc> descs(B);
    // rows available per solve: the largest number of output steps in nsteps steps
    const int nout = pl->out_every > 0 ? nsteps / pl->out_every + 1 : 0;
    const size_t snap_elems = d_tl ? static_cast<size_t>(B) * nout * pl->N : 0;
    if (snap_elems > pl->snap_cap) {
        dev_free(pl->d_snap);
        pl->snap_cap = 0;
        HIP_TRY(dev_alloc(&pl->d_snap, snap_elems));
        pl->snap_cap = snap_elems;
    }
    for (int b = 0; b < B; ++b) {
        ssp::SolveDesc d = base_desc(pl);
        d.field = static_cast<float2 *>(d_psi) + static_cast<size_t>(b) * pl->N;
        ssp::set_work(d, pl->d_bwork + ssp::kWorkPerSolve * static_cast<size_t>(b) * pl->N);
        d.nout = nout;
        d.nsteps = nsteps;
        d.step = static_cast<long long *>(d_step) + b;
        d.stats = (d_stats ? static_cast<ssp::DevStats *>(d_stats) : pl->d_bstats) + b;
        d.tl_out = d_tl ? static_cast<float *>(d_tl) + static_cast<size_t>(b) * nout * pl->N : nullptr;
        d.fld_out = nullptr;
        if (nout == 0) d.tl_out = nullptr;
        d.snap = d.tl_out ? pl->d_snap + static_cast<size_t>(b) * nout * pl->N : nullptr;
        descs[b] = d;
    }
    HIP_TRY(hipMemcpyAsync(pl->d_descs, descs.data(), B * sizeof(ssp::SolveDesc), hipMemcpyHostToDevice,
                           pl->stream));
    if (pl->use_graph) {
        // record the launches once; the descriptors above stay valid for later replays
        drop_graph(pl);
        HIP_TRY(hipStreamBeginCapture(pl->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = ssp::launch_march(pl->P, effective_variant(pl), pl->tab.direct, pl->d_descs, B, nsteps,
                                         pl->stream);
        if (e == hipSuccess && d_tl && nout > 0)
            e = ssp::launch_output(pl->P, pl->tab.direct, pl->d_descs, B, nout, pl->stream);
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
        HIP_TRY(ssp::launch_march(pl->P, effective_variant(pl), pl->tab.direct, pl->d_descs, B, nsteps, pl->stream));
        if (d_tl && nout > 0) HIP_TRY(ssp::launch_output(pl->P, pl->tab.direct, pl->d_descs, B, nout, pl->stream));
    }
    pl->step_index += nsteps;
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
    if (!pl->d_dense_sh) {
        std::vector<uint16_t> sh, sl;
        int kpad = 0;
        ssp::build_dense_tables(pl->N, kpad, sh, sl);
        HIP_TRY(dev_alloc(&pl->d_dense_sh, sh.size()));
        HIP_TRY(dev_alloc(&pl->d_dense_sl, sl.size()));
        HIP_TRY(hipMemcpy(pl->d_dense_sh, sh.data(), sh.size() * 2, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(pl->d_dense_sl, sl.data(), sl.size() * 2, hipMemcpyHostToDevice));
        pl->dense_kpad = kpad;
    }
    if (pl->dense_cols_cap < 2 * B) {
        dev_free(pl->d_dense_xh);
        dev_free(pl->d_dense_xl);
        dev_free(pl->d_dense_expo);
        pl->dense_cols_cap = 0;
        HIP_TRY(dev_alloc(&pl->d_dense_xh, static_cast<size_t>(2 * B) * pl->dense_kpad));
        HIP_TRY(dev_alloc(&pl->d_dense_xl, static_cast<size_t>(2 * B) * pl->dense_kpad));
        HIP_TRY(dev_alloc(&pl->d_dense_expo, static_cast<size_t>(2 * B)));
        pl->dense_cols_cap = 2 * B;
    }
    ssp::DenseTables t;
    t.sh = pl->d_dense_sh;
    t.sl = pl->d_dense_sl;
    t.n = pl->N;
    t.kpad = pl->dense_kpad;
    HIP_TRY(ssp::launch_dense_dst(t, B, static_cast<const float2 *>(d_in), static_cast<float2 *>(d_out),
                                  pl->d_dense_xh, pl->d_dense_xl, pl->d_dense_expo, pl->stream));
    return SSP_OK;
}

}  // extern "C"
