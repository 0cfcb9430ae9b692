// ssp_modal.h - normal-mode starter (Sec. 3.2) computed on the device.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

namespace ssp {

// Largest grid for which the dense depth eigenproblem is solved (three N x N FP64 matrices).
constexpr int kMaxModalNz = 16384;

// Normal-mode starters of a Dirichlet waveguide for nsrc source depths zs[s]: the dense
// vertical operator X = T diag(x) T + diag(v) in the sine basis (T the orthonormal DST-I,
// FP64), its eigendecomposition (rocSOLVER dsyevd, once for all sources), and the modal
// sums u_s(z_n) = sqrt(2 pi) sum_m Psi_m(zs_s) Psi_m(z_n) / sqrt(kappa_m) over the
// propagating modes (kappa_m^2 = k0^2 (1 + lambda_m) > 0, at most max_modes of them, lowest
// first; max_modes <= 0: all).  v [N] is the potential (c0/c)^2 - 1 on the grid.  Outputs:
// u [nsrc][N] (real), kappa [modes] in decreasing order.  Returns hipSuccess, else the HIP
// error (hipErrorUnknown for a failed rocBLAS / rocSOLVER call) with err filled in.
hipError_t modal_starter(int N, double depth, double k0, const std::vector<double> &v, int nsrc,
                         const double *zs, int max_modes, hipStream_t stream, std::vector<double> &u,
                         std::vector<double> &kappa, std::string &err);

}  // namespace ssp
