// ssp_plan.cpp - Pade coefficients and device tables, computed on the host.
//
// Pade construction (Sec. 2; Alg. 1 first step), written from the textbook definition of
// the [p/p] approximant: Taylor series of the target, the p linear matching conditions for
// the denominator, the numerator by truncated convolution, then the factor roots.  All of
// it runs in x87 extended precision (64-bit mantissa); the roots are found with the
// Aberth-Ehrlich simultaneous iteration and polished by Newton steps.
#include "ssp_plan.h"
#include "ssp_dense.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

namespace ssp {

namespace {

uint32_t float_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}
// nearest bfloat16 (round half to even) of a finite float, as its 16-bit pattern
uint16_t bf16_round(float f) {
    uint32_t u = float_bits(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

const long double kPi = 3.141592653589793238462643383279502884L;
const double kPiD = 3.141592653589793238462643383279502884;

cld expj(long double t) { return cld(std::cos(t), std::sin(t)); }

// Taylor coefficients F_0..F_n of F(Z) = exp(h(Z)), h(Z) = i s (e^{i alpha/2} sqrt(1+Z) - 1):
// F' = h' F gives n F_n = sum_{k=1..n} k h_k F_{n-k}.
std::vector<cld> taylor(long double s, long double alpha, int n) {
    const cld I(0, 1);
    const cld rot = expj(alpha / 2);
    std::vector<cld> h(n + 1), F(n + 1);
    h[0] = I * s * (rot - cld(1));
    long double binom = 1;  // binom(1/2, k)
    for (int k = 1; k <= n; ++k) {
        binom *= (0.5L - (k - 1)) / k;
        h[k] = I * s * rot * binom;
    }
    F[0] = std::exp(h[0]);
    for (int m = 1; m <= n; ++m) {
        cld acc(0);
        for (int k = 1; k <= m; ++k) acc += static_cast<long double>(k) * h[k] * F[m - k];
        F[m] = acc / static_cast<long double>(m);
    }
    return F;
}

// Gaussian elimination with partial pivoting, A is n x n row-major.
bool solve(std::vector<cld> A, std::vector<cld> b, int n, std::vector<cld> &x) {
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::abs(A[r * n + c]) > std::abs(A[piv * n + c])) piv = r;
        if (std::abs(A[piv * n + c]) == 0) return false;
        if (piv != c) {
            for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < n; ++r) {
            cld f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    x.assign(n, cld(0));
    for (int r = n - 1; r >= 0; --r) {
        cld acc = b[r];
        for (int k = r + 1; k < n; ++k) acc -= A[r * n + k] * x[k];
        x[r] = acc / A[r * n + r];
    }
    return true;
}

// polynomial c[0] + c[1] x + ... + c[n] x^n and its derivative at x
void polyval(const std::vector<cld> &c, cld x, cld &v, cld &dv) {
    v = 0;
    dv = 0;
    for (int k = static_cast<int>(c.size()) - 1; k >= 0; --k) {
        dv = dv * x + v;
        v = v * x + c[k];
    }
}

// Roots of c[0] + ... + c[n] x^n (c[n] != 0) by Aberth-Ehrlich + Newton polish.
bool roots(const std::vector<cld> &c, std::vector<cld> &z) {
    const int n = static_cast<int>(c.size()) - 1;
    z.resize(n);
    // initial guesses on a circle of the Cauchy-bound radius
    long double rad = 0;
    for (int k = 0; k < n; ++k) rad = std::max(rad, std::pow(std::abs(c[k] / c[n]), 1.0L / (n - k)));
    rad = std::max(rad, 1e-3L);
    for (int k = 0; k < n; ++k) z[k] = rad * expj(2 * kPi * (k + 0.25L) / n + 0.4L);
    for (int it = 0; it < 500; ++it) {
        long double worst = 0;
        for (int k = 0; k < n; ++k) {
            cld v, dv;
            polyval(c, z[k], v, dv);
            if (v == cld(0)) continue;
            cld ratio = v / dv;
            cld sum(0);
            for (int j = 0; j < n; ++j)
                if (j != k) sum += cld(1) / (z[k] - z[j]);
            cld step = ratio / (cld(1) - ratio * sum);
            z[k] -= step;
            worst = std::max(worst, std::abs(step) / std::max(std::abs(z[k]), 1e-30L));
        }
        if (worst < 1e-18L) break;
    }
    for (int k = 0; k < n; ++k) {
        for (int it = 0; it < 4; ++it) {
            cld v, dv;
            polyval(c, z[k], v, dv);
            if (dv == cld(0)) break;
            z[k] -= v / dv;
        }
        if (!std::isfinite(z[k].real()) || !std::isfinite(z[k].imag())) return false;
    }
    return true;
}

bool arg_less(const cld &x, const cld &y) {
    long double ax = std::arg(x), ay = std::arg(y);
    if (ax != ay) return ax < ay;
    return std::abs(x) < std::abs(y);
}

}  // namespace

bool pade_coefficients(double sigma_d, int p, double alpha_d, PadeSet &out, std::string &err) {
    if (p < 1 || p > 12) {
        err = "pade_order must be in [1, 12]";
        return false;
    }
    const long double s = sigma_d, alpha = alpha_d;
    std::vector<cld> F = taylor(s, alpha, 2 * p);
    // denominator: sum_{i=0..p} q_i F_{n-i} = 0 for n = p+1..2p, q_0 = 1
    std::vector<cld> A(p * p), rhs(p), q1;
    for (int r = 0; r < p; ++r) {
        int n = p + 1 + r;
        for (int i = 1; i <= p; ++i) A[r * p + (i - 1)] = F[n - i];
        rhs[r] = -F[n];
    }
    if (!solve(A, rhs, p, q1)) {
        err = "singular Pade system";
        return false;
    }
    std::vector<cld> q(p + 1), P(p + 1);
    q[0] = 1;
    for (int i = 0; i < p; ++i) q[i + 1] = q1[i];
    for (int n = 0; n <= p; ++n) {
        cld acc(0);
        for (int i = 0; i <= n; ++i) acc += q[i] * F[n - i];
        P[n] = acc;
    }
    std::vector<cld> rq, rp;
    if (!roots(q, rq) || !roots(P, rp)) {
        err = "Pade root finding failed";
        return false;
    }
    // Q(Z) = prod (1 + bt_j Z), P(Z) = P_0 prod (1 + at_j Z)
    std::vector<cld> bt(p), at(p);
    for (int j = 0; j < p; ++j) {
        bt[j] = cld(-1) / rq[j];
        at[j] = cld(-1) / rp[j];
    }
    std::sort(bt.begin(), bt.end(), arg_less);
    // pair each numerator factor with the denominator factor whose conjugate it is closest to
    std::vector<cld> pool = at, paired;
    for (int j = 0; j < p; ++j) {
        size_t best = 0;
        for (size_t k = 1; k < pool.size(); ++k)
            if (std::abs(pool[k] - std::conj(bt[j])) < std::abs(pool[best] - std::conj(bt[j]))) best = k;
        paired.push_back(pool[best]);
        pool.erase(pool.begin() + best);
    }
    cld C = P[0];
    std::vector<cld> b(p), a(p);
    if (alpha != 0) {
        const cld gam = expj(-alpha), beta = gam - cld(1);
        for (int j = 0; j < p; ++j) {
            C = C * (cld(1) + paired[j] * beta) / (cld(1) + bt[j] * beta);
            b[j] = bt[j] * gam / (cld(1) + bt[j] * beta);
            a[j] = paired[j] * gam / (cld(1) + paired[j] * beta);
        }
    } else {
        b = bt;
        a = paired;
    }
    std::vector<int> idx(p);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return arg_less(b[x], b[y]); });
    out.p = p;
    out.sigma = sigma_d;
    out.alpha = alpha_d;
    out.b.resize(p);
    out.a.resize(p);
    out.d.resize(p);
    cld d0 = C;
    for (int k = 0; k < p; ++k) d0 *= a[k] / b[k];
    for (int k = 0; k < p; ++k) {
        int j = idx[k];
        cld num = C, den(1);
        for (int i = 0; i < p; ++i) {
            num *= cld(1) - a[i] / b[j];
            if (i != j) den *= cld(1) - b[i] / b[j];
        }
        out.b[k] = cd(b[j]);
        out.a[k] = cd(a[j]);
        out.d[k] = cd(num / den);
    }
    out.C = cd(C);
    out.d0 = cd(d0);
    for (int k = 0; k < p; ++k)
        if (!std::isfinite(out.b[k].real()) || !std::isfinite(out.d[k].real())) {
            err = "non-finite Pade coefficient";
            return false;
        }
    return true;
}

cd pade_eval(const PadeSet &ps, cd x) {
    cd r = ps.C;
    for (int j = 0; j < ps.p; ++j) r *= (1.0 + ps.a[j] * x) / (1.0 + ps.b[j] * x);
    return r;
}

// ------------------------------------------------------------------------------ host FFT
void host_fft(std::vector<cd> &x, int sign) {
    // iterative radix-2 (the chirp lengths are powers of two): bit reversal, then log2 n
    // passes of butterflies with twiddles from a table computed once
    const int n = static_cast<int>(x.size());
    std::vector<cd> w(n / 2 > 0 ? n / 2 : 1);
    for (int j = 0; j < n / 2; ++j) {
        const double ang = sign * 2 * kPiD * static_cast<double>(j) / n;
        w[j] = cd(std::cos(ang), std::sin(ang));
    }
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(x[i], x[j]);
    }
    for (int len = 2; len <= n; len <<= 1) {
        const int half = len / 2, step = n / len;
        for (int i = 0; i < n; i += len)
            for (int k = 0; k < half; ++k) {
                const cd t = w[static_cast<size_t>(k) * step] * x[i + k + half];
                x[i + k + half] = x[i + k] - t;
                x[i + k] += t;
            }
    }
}

int chirp_fft_length(int n_min) {
    int P = 128;  // smallest length of the device FFT (two waves of butterflies)
    while (P < n_min) P *= 2;
    return P;
}

// ------------------------------------------------------------------------------ tables
GridSpec grid_spec(int bc, int nz, double depth) {
    if (bc == kBcNeumann) return {0, depth / (nz - 1)};   // n H/(Nz-1), n = 0..Nz-1
    if (bc == kBcPeriodic) return {0, depth / nz};        // n H/Nz, n = 0..Nz-1
    return {1, depth / (nz + 1)};                         // n H/(Nz+1), n = 1..Nz
}

namespace {

void put_c(std::vector<float> &v, size_t i, cd z) {
    v[2 * i] = static_cast<float>(z.real());
    v[2 * i + 1] = static_cast<float>(z.imag());
}

// FFT of a window given on positions 0..P-1, in the engine's slot order (FP64).
std::vector<cd> window_spectrum(std::vector<cd> w, int P, bool split) {
    host_fft(w, -1);
    const int PE = split ? P / 2 : P;
    std::vector<cd> out(P);
    for (int q = 0; q < P; ++q) {
        const int slot = split ? ((q & 1) ? PE + q / 2 : q / 2) : q;
        out[slot] = w[q];
    }
    return out;
}

// A spectrum as interleaved complex FP32.
std::vector<float> to_f32(const std::vector<cd> &k) {
    std::vector<float> out(2 * k.size());
    for (size_t q = 0; q < k.size(); ++q) put_c(out, static_cast<int>(q), k[q]);
    return out;
}

}  // namespace

void build_tables(int nz, double depth, double k0, const PadeSet &ps, int bc, DeviceTables &t) {
    const int N = nz;
    auto pow2 = [](long long v) { return v > 0 && (v & (v - 1)) == 0; };
    int direct = kDirectNone;
    if (bc == kBcPeriodic && N >= 128 && N <= kMaxEngineFFT && pow2(N)) direct = kDirectFourier;
    if (bc == kBcDirichlet && 2 * (N + 1) >= 128 && 2 * (N + 1) <= kMaxEngineFFT && pow2(N + 1))
        direct = kDirectSine;
    const int P = direct == kDirectFourier ? N : direct == kDirectSine ? 2 * (N + 1) : chirp_fft_length(2 * nz - 1);
    t.nz = N;
    t.P = P;
    t.bc = bc;
    t.direct = direct;
    // Every transform kernel is a sum over n of x_n times exp(+-i theta k n) terms, and
    // k n = (k^2 + n^2 - (k-n)^2)/2 = ((k+n)^2 - k^2 - n^2)/2 turns each into a chirp
    // pre-modulation, a convolution (Toeplitz window, k - n) or correlation (Hankel window,
    // k + n) with the chirp, and a chirp post-modulation:
    //   sine    sin(pi k n/M), M = Nz+1:  (i conj(c_k)/2)(conv - corr), y_n = conj(c_n) x_n
    //   cosine  cos(pi k n/M), M = Nz-1:  (conj(c_k)/2)(conv + corr),  y_n = conj(c_n) x_n
    //   Fourier exp(-2 pi i k n/Nz):      conj(c_k) conv, y_n = conj(c_n) x_n; the inverse
    //           exp(+2 pi i k n/Nz):      c_k conv', y_n = c_n x_n, window conj(c_d)
    // with c_d = exp(i pi d^2 / D), D = 2M (sine, cosine) or Nz (Fourier).
    const long long D = bc == kBcDirichlet ? 2LL * (N + 1) : (bc == kBcNeumann ? 2LL * (N - 1) : N);
    // c_d for d = 0..2N (even in d), the argument reduced exactly with d^2 mod 2D
    std::vector<cd> ch(2 * static_cast<size_t>(N) + 1);
    for (long long d = 0; d <= 2LL * N; ++d) {
        const long long r = (d * d) % (2 * D);
        const double ang = kPiD * static_cast<double>(r) / static_cast<double>(D);
        ch[d] = cd(std::cos(ang), std::sin(ang));
    }
    auto chirp = [&](long long d) { return ch[d < 0 ? -d : d]; };
    const bool split = P > kMaxEngineFFT;
    const int PE = split ? P / 2 : P;
    t.k1.clear();
    t.k2.clear();
    t.k1i.clear();
    t.kph.clear();
    t.ksign = 1;
    if (direct == kDirectNone) {
        std::vector<cd> K1(P, 0.0), K2(P, 0.0);
        for (long long d = 1 - N; d <= N - 1; ++d) K1[((d % P) + P) % P] = chirp(d);
        if (bc == kBcDirichlet) {
            // element n (1..N) at position n-1: Hankel window c_{(k-1)+(n-1)+2}
            for (long long d = 0; d <= 2LL * N - 2; ++d) K2[d % P] = chirp(d + 2);
        } else if (bc == kBcNeumann) {
            // the sum conv + corr as conv - (-corr)
            for (long long d = 0; d <= 2LL * N - 2; ++d) K2[d % P] = -chirp(d);
        }
        t.k1 = to_f32(window_spectrum(K1, P, split));
        if (!split) {
            t.k2 = to_f32(window_spectrum(K2, P, false));
        } else {
            // split lengths: the phase that derives K2 from K1 (zero: no Hankel window)
            t.kph.assign(4 * (64 + static_cast<size_t>(P) / 64), 0.f);
            if (bc != kBcPeriodic) {
                const long long M = D / 2, s = N - 1;
                static const cd quarter[4] = {cd(1, 0), cd(0, 1), cd(-1, 0), cd(0, -1)};
                const cd phi = (bc == kBcNeumann ? -1.0 : 1.0) * quarter[M % 4];  // e^{i pi M/2}
                auto wp = [&](long long j) {  // exp(-2 pi i j / P), j reduced exactly
                    const long long r = ((j % P) + P) % P;
                    const double ang = -2.0 * kPiD * static_cast<double>(r) / P;
                    return cd(std::cos(ang), std::sin(ang));
                };
                auto put = [&](int e, cd z) {  // double-float complex entry e
                    split_df(z.real(), t.kph[4 * e], t.kph[4 * e + 2]);
                    split_df(z.imag(), t.kph[4 * e + 1], t.kph[4 * e + 3]);
                };
                for (int k = 0; k < 64; ++k) put(k, phi * wp(s * k));
                for (int m = 0; m < P / 64; ++m) put(64 + m, wp(64 * s * m));
                t.ksign = (s % 2 == 0) ? 1 : -1;
            }
        }
        if (bc == kBcPeriodic) {
            for (long long d = 1 - N; d <= N - 1; ++d) K1[((d % P) + P) % P] = std::conj(chirp(d));
            t.k1i = to_f32(window_spectrum(K1, P, split));
        }
    }
    t.twist.clear();
    if (split) {
        t.twist.resize(4 * static_cast<size_t>(PE));
        for (int n = 0; n < PE; ++n) {
            const double ang = -2 * kPiD * static_cast<double>(n) / P;
            split_df(std::cos(ang), t.twist[4 * n], t.twist[4 * n + 2]);
            split_df(std::sin(ang), t.twist[4 * n + 1], t.twist[4 * n + 3]);
        }
    }
    // Modulations per position m = 0..N-1 (index n = m + 1 for the sine transform, n = m
    // otherwise).  The coefficient-space representation kept on the device is the inverse
    // transform's pre-modulated input, so that every transform of the march runs without
    // its pre- and post-modulations: they are folded into dmod (post of one direction times
    // pre of the other), which is the same in both directions.
    //   sine:    pre = conj(c_n), post = i conj(c_k) sqrt(2/M)/(2P) (orthonormal DST-I)
    //   cosine:  forward C e on grid values, inverse C/e (C the orthonormal DCT-I,
    //            e = 1/sqrt(2) at both ends): pre_f = conj(c_n) e_n^2,
    //            post_f = conj(c_k) e_k sqrt(2/M)/(2P); pre_i = conj(c_n) e_n,
    //            post_i = conj(c_k) sqrt(2/M)/(2P)
    //   Fourier: pre_f = conj(c_n), post_f = conj(c_k)/(sqrt(N) P); pre_i = c_n,
    //            post_i = c_k/(sqrt(N) P); dmod = 1/(sqrt(N) P)
    //   Fourier, direct (N an engine length): pre = 1, post = 1/sqrt(N) both ways
    //   sine, direct (P = 2(N+1)): with w^j = exp(-2 pi i j/P) and element n = m+1 at
    //            position m, DST(x)_{q+1} = sqrt(2/(N+1)) (i/2) w^q FFT_P(z)_q where z holds
    //            x_n w^n at position n-1 and its odd image -x_n w^{-n} at position P-1-n
    //            (zeros at positions N and P-1): pre = w^{m+1}, post = sqrt(2/(N+1)) (i/2) w^m,
    //            the image factor -w^{-2(m+1)} in the mirror table; the transform is its own
    //            inverse
    const cd I(0, 1);
    auto wpow = [&](long long j) {  // exp(-2 pi i j / P), j reduced exactly
        const long long r = ((j % P) + P) % P;
        const double ang = -2.0 * kPiD * static_cast<double>(r) / P;
        return cd(std::cos(ang), std::sin(ang));
    };
    std::vector<cd> dmod(N);
    const bool dense = bc == kBcDirichlet && N <= kMaxDenseGrid;
    t.mmod.clear();
    if (dense) t.mmod.assign(4 * static_cast<size_t>(N), 0.f);
    t.pre.assign(2 * N, 0.f);
    t.post.assign(2 * N, 0.f);
    t.dmod.assign(2 * N, 0.f);
    t.postf.clear();
    if (bc != kBcDirichlet) t.postf.assign(2 * N, 0.f);
    t.mirror.clear();
    if (direct == kDirectSine) t.mirror.assign(4 * static_cast<size_t>(N), 0.f);
    for (int m = 0; m < N; ++m) {
        cd pre_f, post_i, post_f, pre_i;
        if (direct == kDirectSine) {
            pre_f = pre_i = wpow(m + 1);
            post_f = post_i = std::sqrt(2.0 / (N + 1)) * 0.5 * I * wpow(m);
            const cd img = -std::conj(wpow(2LL * (m + 1)));
            split_df(img.real(), t.mirror[4 * m], t.mirror[4 * m + 2]);
            split_df(img.imag(), t.mirror[4 * m + 1], t.mirror[4 * m + 3]);
        } else if (bc == kBcDirichlet) {
            const double scale = 0.5 * std::sqrt(2.0 / (N + 1)) / P;
            const cd cb = std::conj(chirp(m + 1));
            pre_f = pre_i = cb;
            post_i = post_f = cb * I * scale;
        } else if (bc == kBcNeumann) {
            const double scale = 0.5 * std::sqrt(2.0 / (N - 1)) / P;
            const double e = (m == 0 || m == N - 1) ? std::sqrt(0.5) : 1.0;
            const cd cb = std::conj(chirp(m));
            pre_f = cb * (e * e);
            post_f = cb * (e * scale);
            pre_i = cb * e;
            post_i = cb * scale;
        } else if (direct == kDirectNone) {
            const double scale = 1.0 / (std::sqrt(static_cast<double>(N)) * P);
            const cd c = chirp(m);
            pre_f = std::conj(c);
            post_f = std::conj(c) * scale;
            pre_i = c;
            post_i = c * scale;
        } else {
            // forward FFT(x)/sqrt(N), inverse unnormalised IFFT(a)/sqrt(N)
            const double scale = 1.0 / std::sqrt(static_cast<double>(N));
            pre_f = pre_i = 1.0;
            post_f = post_i = scale;
        }
        // (the sine transform's product in the order of its original derivation)
        dmod[m] = (bc == kBcDirichlet && direct == kDirectNone)
                      ? std::conj(chirp(m + 1)) * std::conj(chirp(m + 1)) * I * (0.5 * std::sqrt(2.0 / (N + 1)) / P)
                      : post_f * pre_i;
        if (dense) {
            // stored representation = (inverse pre-modulation) (.) coefficients: the
            // stand-alone forward transform ends with dmod, the plain DST-I with post, and
            // dmod / post = pre_i for both Dirichlet transform kinds
            split_df(pre_i.real(), t.mmod[4 * m], t.mmod[4 * m + 2]);
            split_df(pre_i.imag(), t.mmod[4 * m + 1], t.mmod[4 * m + 3]);
        }
        put_c(t.pre, m, pre_f);
        put_c(t.post, m, post_i);
        put_c(t.dmod, m, dmod[m]);
        if (bc != kBcDirichlet) put_c(t.postf, m, post_f);
    }
    const int O = PE / 8;
    t.twiddle.resize(3 * static_cast<size_t>(O + 1));
    for (int e = 0; e <= O; ++e) {
        const double ang = -2 * kPiD * static_cast<double>(e) / PE;
        const double re = std::cos(ang), im = std::sin(ang);
        float hr, lr, hi, li;
        split_df(re, hr, lr);
        split_df(im, hi, li);
        t.twiddle[3 * e] = float_bits(hr);
        t.twiddle[3 * e + 1] = float_bits(hi);
        t.twiddle[3 * e + 2] = (static_cast<uint32_t>(bf16_round(lr)) << 16) | bf16_round(li);
    }
    const int p = ps.p;
    t.s.resize(static_cast<size_t>(4) * p * N);
    t.bmul.resize(static_cast<size_t>(4) * p * N);
    t.qmul.resize(static_cast<size_t>(4) * p * N);
    t.beta.resize(4 * p);
    t.tmul.clear();
    if (dense) t.tmul.resize(static_cast<size_t>(4) * p * N);
    double gain = 0;
    for (int m = 0; m < N; ++m) {
        // eigenvalue of d_z^2 / k0^2 of basis function m: -(l pi/(H k0))^2 with l = m+1
        // (sine), m (cosine) or 2 l' (Fourier, l' = m, or m - N above N/2)
        double l;
        if (bc == kBcDirichlet) l = m + 1;
        else if (bc == kBcNeumann) l = m;
        else l = 2.0 * static_cast<double>(2 * m <= N ? m : m - N);
        const double x = -std::pow(l * kPiD / (depth * k0), 2);
        cd G = std::exp(cd(0, ps.sigma)) * pade_eval(ps, cd(x, 0));
        gain = std::max(gain, std::abs(G));
        for (int j = 0; j < p; ++j) {
            cd sj = 1.0 / (1.0 + ps.b[j] * x);
            cd bj = -ps.b[j] * sj * dmod[m];
            // C_j r_j - 1 = C_j (1 - g_j)(s_j - 1) + (C_j - 1), with s_j - 1 = -b_j x s_j
            // (no cancellation for x near 0)
            const cd g = ps.a[j] / ps.b[j], Cj = j == p - 1 ? ps.C : cd(1.0, 0.0);
            const cd qj = Cj * (1.0 - g) * (-ps.b[j] * x * sj) + (Cj - 1.0);
            size_t o = (static_cast<size_t>(j) * N + m) * 4;
            split_df(sj.real(), t.s[o], t.s[o + 2]);
            split_df(sj.imag(), t.s[o + 1], t.s[o + 3]);
            split_df(qj.real(), t.qmul[o], t.qmul[o + 2]);
            split_df(qj.imag(), t.qmul[o + 1], t.qmul[o + 3]);
            split_df(bj.real(), t.bmul[o], t.bmul[o + 2]);
            split_df(bj.imag(), t.bmul[o + 1], t.bmul[o + 3]);
            if (dense) {
                const cd tj = -ps.b[j] * sj;
                split_df(tj.real(), t.tmul[o], t.tmul[o + 2]);
                split_df(tj.imag(), t.tmul[o + 1], t.tmul[o + 3]);
            }
        }
    }
    t.max_gain = gain;
    for (int j = 0; j < p; ++j) {
        cd g = ps.a[j] / ps.b[j];
        cd be = 1.0 - g;
        if (j == p - 1) be *= ps.C;
        split_df(be.real(), t.beta[4 * j], t.beta[4 * j + 2]);
        split_df(be.imag(), t.beta[4 * j + 1], t.beta[4 * j + 3]);
    }
}

}  // namespace ssp

// ------------------------------------------------------------------------------ dense DST
namespace ssp {

void build_dense_tables(int n, int &kpad, std::vector<uint16_t> &sh, std::vector<uint16_t> &sl) {
    kpad = (n + 127) / 128 * 128;
    sh.assign(static_cast<size_t>(kpad) * kpad, 0);
    sl.assign(static_cast<size_t>(kpad) * kpad, 0);
    const long long M = n + 1;
    const long double amp = std::sqrt(2.0L / M) * 4096.0L;  // S scaled by 2^12
    for (int k = 1; k <= n; ++k) {
        for (int j = 1; j <= n; ++j) {
            // sin(pi k j / M) with the argument reduced exactly: k j mod 2M
            const long long r = (static_cast<long long>(k) * j) % (2 * M);
            const double v = static_cast<double>(amp * std::sin(kPi * static_cast<long double>(r) / M));
            const _Float16 h = static_cast<_Float16>(v);
            const _Float16 l = static_cast<_Float16>(v - static_cast<double>(h));
            uint16_t hb, lb;
            std::memcpy(&hb, &h, 2);
            std::memcpy(&lb, &l, 2);
            sh[static_cast<size_t>(k - 1) * kpad + (j - 1)] = hb;
            sl[static_cast<size_t>(k - 1) * kpad + (j - 1)] = lb;
        }
    }
}

}  // namespace ssp

// ------------------------------------------------------------------ Neumann contraction
namespace ssp {

HostDst1::HostDst1(int n) : N(n) {
    // DST(x)_k = (i/2) sqrt(2/M) conj(c_k) sum_n conj(c_n) x_n (c_{k-n} - c_{k+n}),
    // c_d = exp(i pi d^2/(2M)), M = N + 1: a Toeplitz minus a Hankel sum over positions
    // n - 1, both cyclic convolutions of a power-of-two length P >= 2N - 1 (the Hankel one
    // through the reflected spectrum), as in the device's chirp-z transform
    const long long M = N + 1;
    P = 1;
    while (P < 2 * N - 1) P *= 2;
    ch.resize(2 * static_cast<size_t>(N) + 1);
    for (long long d = 0; d <= 2LL * N; ++d) {
        const long long r = (d * d) % (4 * M);
        const double ang = kPiD * static_cast<double>(r) / static_cast<double>(2 * M);
        ch[d] = cd(std::cos(ang), std::sin(ang));
    }
    k1.assign(P, 0.0);
    k2.assign(P, 0.0);
    for (long long d = 1 - N; d <= N - 1; ++d) k1[((d % P) + P) % P] = ch[d < 0 ? -d : d];
    for (long long d = 0; d <= 2LL * N - 2; ++d) k2[d % P] = ch[d + 2];
    host_fft(k1, -1);
    host_fft(k2, -1);
}

void HostDst1::apply(std::vector<cd> &x) const {
    std::vector<cd> y(P, 0.0), z(P);
    for (int n = 1; n <= N; ++n) y[n - 1] = std::conj(ch[n]) * x[n - 1];
    host_fft(y, -1);
    for (int q = 0; q < P; ++q) z[q] = y[q] * k1[q] - y[(P - q) % P] * k2[q];
    host_fft(z, +1);
    const cd scale = cd(0, 0.5) * std::sqrt(2.0 / static_cast<double>(N + 1)) / static_cast<double>(P);
    for (int k = 1; k <= N; ++k) x[k - 1] = scale * std::conj(ch[k]) * z[k - 1];
}

void neumann_contraction(int nz, double depth, double k0, const PadeSet &ps, int bc, const std::vector<cd> &v,
                         int rows, int iterations, std::vector<double> &bound, std::vector<double> &estimate) {
    const int N = nz, p = ps.p;
    std::vector<double> x(N);
    for (int m = 0; m < N; ++m) {
        double l;
        if (bc == kBcDirichlet) l = m + 1;
        else if (bc == kBcNeumann) l = m;
        else l = 2.0 * static_cast<double>(2 * m <= N ? m : m - N);
        x[m] = -std::pow(l * kPiD / (depth * k0), 2);
    }
    double vmax = 0;
    for (const cd &a : v) vmax = std::max(vmax, std::abs(a));
    bound.assign(p, 0.0);
    estimate.assign(p, std::nan(""));
    for (int j = 0; j < p; ++j) {
        double g = 0;
        for (int m = 0; m < N; ++m) g = std::max(g, std::abs(ps.b[j] / (1.0 + ps.b[j] * x[m])));
        bound[j] = g * vmax;
    }
    if (bc != kBcDirichlet || iterations <= 0 || rows <= 0) return;
    const int half = iterations / 2;
    const HostDst1 S(N);
    for (int j = 0; j < p; ++j) {
        double best = 0;
        for (int r = 0; r < rows; ++r) {
            // a fixed pseudo-random start in the sine basis (64-bit LCG)
            std::vector<cd> u(N);
            unsigned long long st = 0x9E3779B97F4A7C15ULL + 7919ULL * static_cast<unsigned long long>(j * 131 + r);
            auto rnd = [&st]() {
                st = st * 6364136223846793005ULL + 1442695040888963407ULL;
                return static_cast<double>(st >> 11) * (1.0 / 9007199254740992.0) - 0.5;
            };
            for (int m = 0; m < N; ++m) u[m] = cd(rnd(), rnd());
            double lg = 0, lg_half = 0;
            for (int it = 1; it <= iterations; ++it) {
                // u <- b_j D_j S (v (.) S u), then normalised; the log-norms accumulate
                S.apply(u);
                for (int m = 0; m < N; ++m) u[m] *= v[static_cast<size_t>(r) * N + m];
                S.apply(u);
                double nrm = 0;
                for (int m = 0; m < N; ++m) {
                    u[m] *= ps.b[j] / (1.0 + ps.b[j] * x[m]);
                    nrm += std::norm(u[m]);
                }
                nrm = std::sqrt(nrm);
                if (!(nrm > 0) || !std::isfinite(nrm)) break;
                for (int m = 0; m < N; ++m) u[m] /= nrm;
                lg += std::log(nrm);
                if (it == half) lg_half = lg;
            }
            const double rate = std::exp((lg - lg_half) / static_cast<double>(iterations - half));
            best = std::max(best, rate);
        }
        estimate[j] = best;
    }
}

}  // namespace ssp
