// ssp_tuned.h - engine layout of the fused march kernel per FFT length, chosen by
// paper_2511_03343_amd/autotune.py (written by that script; do not edit by hand).
#pragma once

namespace ssp {
// kTunedVariant[log2(P) - 7] for P = 128 ... 32768
constexpr int kTunedVariant[9] = {0, 0, 0, 0, 1, 2, 2, 2, 0};
// kTunedDirect[kind - 1][log2(P) - 7]: direct Fourier (periodic Nz = P), direct sine
// (Dirichlet Nz = P/2 - 1)
constexpr int kTunedDirect[2][9] = {{0, 0, 0, 0, 1, 0, 1, 2, 0}, {0, 0, 0, 0, 1, 2, 2, 2, 0}};
}  // namespace ssp
