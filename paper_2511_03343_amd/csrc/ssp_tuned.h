// ssp_tuned.h - engine layout of the fused march kernel per FFT length, chosen by
// paper_2511_03343_amd/autotune.py (written by that script; do not edit by hand).
#pragma once

namespace ssp {
// kTunedVariant[log2(P) - 7] for P = 128 ... 32768
constexpr int kTunedVariant[9] = {0, 0, 0, 0, 1, 2, 2, 2, 0};
}  // namespace ssp
