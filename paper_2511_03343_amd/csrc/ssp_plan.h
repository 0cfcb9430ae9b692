// ssp_plan.h - host-side plan mathematics of the SSSP library (no HIP dependencies).
//
// Pade coefficients (Sec. 2, the [p/p] approximant of exp(i sigma (sqrt(1+x) - 1)); Alg. 1
// first step), the eigenvalues of the vertical operator in the sine, cosine or Fourier
// basis (Sec. 3 and 3.1), and the tables that the device kernels consume.  Everything here is computed in FP64 or
// extended precision on the host and rounded once when stored.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace ssp {

using cld = std::complex<long double>;
using cd = std::complex<double>;

struct PadeSet {
    int p = 0;
    double sigma = 0, alpha = 0;
    std::vector<cd> b;  // denominator factors 1 + b_j x, application order
    std::vector<cd> a;  // numerator factors 1 + a_j x paired with b_j
    cd C{1, 0};         // product-form constant
    cd d0{1, 0};        // sum-form constant
    std::vector<cd> d;  // sum-form residues paired with b_j
};

// [p/p] Pade approximant of F(Z) = exp(i sigma (e^{i alpha/2} sqrt(1+Z) - 1)) mapped back to
// x with Z = e^{-i alpha}(1+x) - 1 (alpha = 0: the standard approximant).  Returns false
// (with a message) if the construction fails.
bool pade_coefficients(double sigma, int p, double alpha, PadeSet &out, std::string &err);

// R(x) = C prod (1 + a_j x)/(1 + b_j x)
cd pade_eval(const PadeSet &ps, cd x);

// In-place complex FFT of length n (a power of two), sign -1 forward.
void host_fft(std::vector<cd> &x, int sign);

// Smallest FFT length accepted by the device engine that is >= n_min.
int chirp_fft_length(int n_min);

// Largest FFT one workgroup computes in LDS; longer convolutions are split in two.
constexpr int kMaxEngineFFT = 16384;

// Boundary conditions at z = 0 and z = H (Sec. 3.1) and their transforms.
enum Boundary : int { kBcDirichlet = 0, kBcNeumann = 1, kBcPeriodic = 2 };

// Kinds of direct transform (see DeviceTables::direct).
enum DirectKind : int { kDirectNone = 0, kDirectFourier = 1, kDirectSine = 2 };

// Grid of a boundary condition: z of position m (0-based) is (m + zoff) dz.
struct GridSpec {
    int zoff;
    double dz;
};
GridSpec grid_spec(int bc, int nz, double depth);

struct DeviceTables {
    int nz = 0, P = 0, bc = kBcDirichlet;
    // direct transforms (no chirp windows), where the grid allows them:
    //   kDirectFourier: periodic grid whose length is an engine FFT length (a power of two,
    //     128 .. 16384): FFTs of length P = nz; pre = 1 and the modulations are 1/sqrt(nz)
    //   kDirectSine: Dirichlet grid with nz + 1 a power of two (P = 2(nz+1) in 128 .. 16384):
    //     the DST-I as the FFT of the odd extension of length P, built in LDS with the
    //     mirror multipliers below
    int direct = kDirectNone;
    // chirp-z transform of length nz through a cyclic convolution of length P, with the
    // chirp c_d = exp(i pi d^2 / D) (D = 2(nz+1) sine, 2(nz-1) cosine, nz Fourier):
    // [P] complex FP32 spectra of the two chirp windows, Toeplitz c_d (d in [1-nz, nz-1])
    // and Hankel (d in [0, 2nz-2]: c_{d+2} for the sine transform, whose element n sits at
    // position n-1, and -c_d for the cosine transform; zero for the Fourier transform).
    // k1/k2 serve the forward direction (grid values -> coefficients); k1i, when not empty,
    // the inverse direction (the Fourier transform only, whose Hankel window is zero both
    // ways; the sine and cosine transforms are their own inverses).  For P > kMaxEngineFFT
    // k1 is stored as the even frequencies followed by the odd ones (the two halves of a split
    // transform), and k2 is not stored: the chirp is even about M = D/2 up to a sign pattern,
    // c_{M+e} = e^{i pi M/2} (-1)^e c_e, so the Hankel window is the Toeplitz window moved by
    // s = nz - 1 positions and modulated by (-1)^e, and K2_q = phi w^{s q} K1_{q + P/2} with
    // w = exp(-2 pi i/P) and phi = e^{i pi M/2} (sine) or -e^{i pi M/2} (cosine).  kph holds
    // that phase as [64 + P/64] double-float complex: phi w^{s k} for k < 64, then w^{64 s m}
    // for m < P/64 (the device multiplies one of each; all zero for the Fourier transform);
    // ksign = (-1)^s.  Double-float, because every entry is shared by many spectrum
    // positions: an FP32 rounding there is a common relative error of a structured set of
    // K2 values, and the march accumulates it coherently (in FP32 the broadband 300 Hz
    // field drifted 3x faster).  The FP32 roundings of K1, K2 themselves are independent per
    // position, a fixed perturbation of every transform that stays below the other
    // roundings (the transforms only carry the Neumann terms; the isovelocity part of each
    // factor is a double-float product in the sine basis).
    std::vector<float> k1, k2, k1i, kph;
    int ksign = 1;
    std::vector<float> pre;           // [nz] complex FP32 forward pre-modulation
    std::vector<float> post;          // [nz] complex FP32 inverse post-modulation (incl. 1/P)
    std::vector<float> postf;         // [nz] forward post-modulation, when it differs from post
    std::vector<float> dmod;          // [nz] complex FP32 post-modulation of one direction
                                      // times pre-modulation of the other (the same both ways)
    // kDirectSine only: [nz] double-float complex -exp(4 pi i (m+1)/P), the factor between
    // the stored value at position m and its odd-extension image at position P - 2 - m
    std::vector<float> mirror;
    // exp(-2 pi i e / PE) for e = 0..PE/8, PE = the engine FFT length (P, or P/2 when split;
    // the first octant, the device rebuilds the other octants by symmetry): per entry
    // hi.re, hi.im (FP32 bit patterns) and the rounding remainders lo.re, lo.im packed as two
    // bfloat16 (re in the high half)
    std::vector<uint32_t> twiddle;
    // split transforms only: [P/2] double-float complex exp(-2 pi i n / P)
    std::vector<float> twist;
    // Pade factors in the chirp-modulated sine basis:
    std::vector<float> s;             // [p][nz] double-float complex 1/(1 + b_j x_l)
    std::vector<float> bmul;          // [p][nz] double-float complex -b_j s_jl * dmod_l (FP64 product)
    // The product-form factor u <- C_j (g_j u + (1 - g_j) w_j), w_j = s_j u + w'_j (w'_j the
    // Neumann terms beyond the first; C_j = C for the last factor, else 1) applied as the
    // increment u <- u + (q_j u + beta_j w'_j): for the propagating modes r_j = g_j + (1 -
    // g_j) s_j is within ~1e-6 of 1, and the increment keeps the FP32 roundings of the
    // large intermediate products g_j u and (1 - g_j) w_j, which repeat from step to step
    // while the mode barely changes, out of the state.
    std::vector<float> qmul;          // [p][nz] double-float complex C_j r_j - 1
    std::vector<float> beta;          // [p] double-float complex C_j (1 - g_j)
    double max_gain = 0;              // max_l |e^{i sigma} R(x_l)|
    // dense engine (Dirichlet grids with nz <= kMaxDenseGrid), else empty:
    std::vector<float> tmul;          // [p][nz] double-float complex -b_j/(1 + b_j x_l), plain sine basis
    std::vector<float> mmod;          // [nz] double-float complex m, representation = m (.) coefficients
};

// Largest grid of the dense engine (its S matrix is kpad^2 fp16 values per part).
constexpr int kMaxDenseGrid = 2048;

// Build all device tables for a grid (nz, H, k0, boundary condition) and a coefficient set.
void build_tables(int nz, double depth, double k0, const PadeSet &ps, int bc, DeviceTables &t);

// Convergence of the Neumann series of every Pade factor (Sec. 3: the series for
// (1 + b_j X)^{-1} converges when the operator K_j = b_j L_j^{-1} V is a contraction), for the
// potential rows v [rows][nz] (v + i eta, FP64) of a grid with boundary condition bc:
//   bound[j]    = max_l |b_j/(1 + b_j x_l)| max |v|, a norm bound of K_j (>= its spectral radius;
//                 below 1 the series converges geometrically for any input)
//   estimate[j] = the spectral radius of K_j by power iteration over `iterations` products
//                 (growth rate over the second half of the iteration, largest over the rows),
//                 Dirichlet grids only (NaN otherwise or for iterations <= 0); a series whose
//                 operator has spectral radius >= 1 diverges for generic inputs.
void neumann_contraction(int nz, double depth, double k0, const PadeSet &ps, int bc, const std::vector<cd> &v,
                         int rows, int iterations, std::vector<double> &bound, std::vector<double> &estimate);

// Orthonormal DST-I of complex FP64 vectors of length n, in place, through one FFT pair of a
// power-of-two length >= 2n - 1 (the host transform of the contraction estimate).
struct HostDst1 {
    explicit HostDst1(int n);
    void apply(std::vector<cd> &x) const;
    int N = 0, P = 0;
    std::vector<cd> ch, k1, k2;
};

// Split a double into hi + lo floats (hi = nearest float, lo = nearest float of the rest).
inline void split_df(double v, float &hi, float &lo) {
    hi = static_cast<float>(v);
    lo = static_cast<float>(v - static_cast<double>(hi));
}

}  // namespace ssp
