// ssp_tuned.h - engine layout of the fused march kernel per FFT length, chosen by
// paper_2511_03343_amd/autotune.py (written by that script; do not edit by hand).
#pragma once

namespace ssp {
// kTunedVariant[log2(P) - 7] for P = 128 ... 32768
constexpr int kTunedVariant[9] = {0, 0, 0, 0, 1, 2, 2, 2, 0};
// kTunedDirect[kind - 1][log2(P) - 7]: direct Fourier (periodic Nz = P), direct sine
// (Dirichlet Nz = P/2 - 1)
constexpr int kTunedDirect[2][9] = {{0, 0, 0, 0, 1, 0, 0, 0, 0}, {0, 0, 0, 0, 1, 2, 2, 2, 0}};
// kTunedMixed[log2(P) - 7]: chirp-z layouts for batches that mix FFT lengths
// (SSP_OPT_VARIANT = -2), measured on a mixed-length batch
constexpr int kTunedMixed[9] = {0, 0, 0, 0, 1, 1, 1, 2, 0};
// kTunedEngine[Nz class][p class]: 1 = dense engine, 0 = FFT engine, for SSP_ENGINE_AUTO;
// Nz classes <= 256, <= 512, <= 1024, <= 2048; p classes <= 4, 5-6, 7-8, >= 9
constexpr int kTunedEngine[4][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};

inline int tuned_engine(int nz, int p) {
    const int nc = nz <= 256 ? 0 : nz <= 512 ? 1 : nz <= 1024 ? 2 : 3;
    const int pc = p <= 4 ? 0 : p <= 6 ? 1 : p <= 8 ? 2 : 3;
    return nz <= 2048 ? kTunedEngine[nc][pc] : 0;
}
}  // namespace ssp
