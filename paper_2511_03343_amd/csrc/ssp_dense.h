// ssp_dense.h - dense DST-I on the matrix cores (interface between the C ABI and the kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "ssp_device.h"

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

// ---------------------------------------------------------------- dense-engine march
// Per-solve state of a dense-engine launch (device; initialised by the launch itself).
struct DenseCol {
    long long n0;              // step counter at the launch's start
    long long terms;           // Neumann terms of the launch
    double t0, tn, wn, max_res;
    int steps_done, status, step_active, series_active, bad, used, max_used, notconv;
};

// Device scratch of a dense-engine launch of B solves of grid size n.
struct DenseWork {
    float2 *U, *U0, *W, *G, *V;  // [B][n]: state, step-start state, series sum beyond the first
                                 // term, product, potential
    float2 *A0;                  // [B][n]: first series term
    _Float16 *xh, *xl;           // [2B][kpad] operand planes
    int *expo;                   // [2B] operand column exponents
    DenseCol *cols;              // [B]
    int *active;                 // series still running in the batch
};
size_t dense_work_bytes(int B, int n);
DenseWork carve_dense_work(void *base, int B, int n);

// March B solves of one grid size (descriptors d_descs, each with its own plan tables, step
// count, step counter and outputs; t.n == every descriptor's N) with the dense engine: a
// host loop over the launch's steps, the Pade factors (pmax = the largest p) and the terms
// (up to nmax_max), each term two batched products with S and two per-solve pointwise
// launches.  Every kPoll terms the host reads the number of series still running (into
// the pinned h_active, waiting for the stream) and stops issuing terms when it is zero.
// Writes each solve's field, step counter, statistics and output snapshots as the fused
// march does (launch_output then converts the snapshots).
hipError_t dense_march(const DenseTables &t, const SolveDesc *d_descs, int B, int nsteps, int pmax, int nmax_max,
                       const DenseWork &w, int *h_active, hipStream_t stream);

}  // namespace ssp
