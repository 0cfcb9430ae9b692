// ssp_dense.h - dense DST-I on the matrix cores (interface between the C ABI and the kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace ssp {

// Largest grid of the dense path (S is kpad^2 fp16 values per part: 16 MiB at 2048).
constexpr int kMaxDenseNz = 2048;

// Device copy of 2^12 S split into fp16 high and low parts, [kpad][kpad] row-major, zero
// outside the n x n block (kpad = n rounded up to 128).
struct DenseTables {
    const _Float16 *sh = nullptr, *sl = nullptr;
    int n = 0, kpad = 0;
};

// Host tables of the same layout (fp16 bit patterns).
void build_dense_tables(int n, int &kpad, std::vector<uint16_t> &sh, std::vector<uint16_t> &sl);

// Y = S X for B complex vectors (in/out [B][n] complex64, may alias: the split kernel reads
// all of in before the product kernel writes out).  Scratch:
// xh, xl [2B][kpad] fp16 and expo [2B].
hipError_t launch_dense_dst(const DenseTables &t, int B, const float2 *in, float2 *out, _Float16 *xh,
                            _Float16 *xl, int *expo, hipStream_t stream);

// The product kernel alone on operands already split by a preceding launch_dense_dst.
hipError_t launch_dense_gemm_only(const DenseTables &t, int B, const _Float16 *xh, const _Float16 *xl,
                                  const int *expo, float2 *out, hipStream_t stream);

}  // namespace ssp
