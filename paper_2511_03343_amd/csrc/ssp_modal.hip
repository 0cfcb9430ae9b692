// ssp_modal.hip - normal-mode starter (Sec. 3.2): the depth eigenproblem of the vertical
// operator in the sine basis, solved on the device in FP64.
//
// With T the orthonormal DST-I and x_l = -(l pi/(H k0))^2, the operator of the range step
// is X = T diag(x) T + diag(v); the mode functions of the Sturm-Liouville problem
// d_z^2 Psi + (k^2 - kappa^2) Psi = 0 are its eigenvectors and kappa^2 = k0^2 (1 + lambda).
// Built as two steps of dense algebra: T (a kernel), T diag(x) (a kernel), the product with
// T (rocBLAS dgemm), v on the diagonal (a kernel), then rocSOLVER dsyevd.  The unit
// eigenvectors y_m give Psi_m(z_n) = y_m[n]/sqrt(dz); Psi_m(zs) comes from the sine-basis
// coefficients a = T y_m (dgemm over the selected modes) dotted with the basis functions
// sqrt(2/H) sin(l pi zs/H) at zs (dgemm over the sources), so a source need not sit on a
// grid point.  One eigendecomposition serves every source depth of the call.
#include "ssp_modal.h"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cmath>

namespace ssp {
namespace {

constexpr double kPiM = 3.141592653589793238462643383279502884;

// T(i, j) = sqrt(2/M) sin(pi (i+1)(j+1)/M), M = N + 1, argument reduced exactly mod 2M
// (symmetric, so row- and column-major agree)
__global__ void k_sine_matrix(double *T, int N) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= N) return;
    const long long M = N + 1;
    const long long r = (static_cast<long long>(i + 1) * (j + 1)) % (2 * M);
    T[static_cast<size_t>(j) * N + i] = sqrt(2.0 / static_cast<double>(M)) *
                                        sin(kPiM * static_cast<double>(r) / static_cast<double>(M));
}

// D = T diag(x): column j scaled by x_j (column-major)
__global__ void k_scale_columns(const double *T, const double *x, double *D, int N) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= N) return;
    const size_t o = static_cast<size_t>(j) * N + i;
    D[o] = T[o] * x[j];
}

__global__ void k_add_diagonal(double *X, const double *v, int N) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) X[static_cast<size_t>(i) * N + i] += v[i];
}

struct Handle {
    rocblas_handle h = nullptr;
    ~Handle() {
        if (h) (void)rocblas_destroy_handle(h);
    }
};

struct DevBuf {
    double *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t n) { return hipMalloc(reinterpret_cast<void **>(&p), n * sizeof(double)); }
};

}  // namespace

hipError_t modal_starter(int N, double depth, double k0, const std::vector<double> &v, int nsrc,
                         const double *zs, int max_modes, hipStream_t stream, std::vector<double> &u,
                         std::vector<double> &kappa, std::string &err) {
#define MODAL_HIP(x)                                              \
    do {                                                          \
        hipError_t e_ = (x);                                      \
        if (e_ != hipSuccess) {                                   \
            err = std::string(#x ": ") + hipGetErrorString(e_);   \
            return e_;                                            \
        }                                                         \
    } while (0)
#define MODAL_LIB(x)                                              \
    do {                                                          \
        rocblas_status s_ = (x);                                  \
        if (s_ != rocblas_status_success) {                       \
            err = std::string(#x ": ") + rocblas_status_to_string(s_); \
            return hipErrorUnknown;                               \
        }                                                         \
    } while (0)
    const size_t NN = static_cast<size_t>(N) * N;
    DevBuf T, D, X, x, dv, w, eig, off, phi, psz, ud;
    rocblas_int *d_info = nullptr;
    MODAL_HIP(T.alloc(NN));
    MODAL_HIP(D.alloc(NN));
    MODAL_HIP(X.alloc(NN));
    MODAL_HIP(x.alloc(N));
    MODAL_HIP(dv.alloc(N));
    MODAL_HIP(eig.alloc(N));
    MODAL_HIP(off.alloc(N));
    const size_t NS = static_cast<size_t>(N) * nsrc;
    MODAL_HIP(phi.alloc(NS));
    MODAL_HIP(psz.alloc(NS));
    MODAL_HIP(w.alloc(NS));
    MODAL_HIP(ud.alloc(NS));
    MODAL_HIP(hipMalloc(reinterpret_cast<void **>(&d_info), sizeof(rocblas_int)));
    struct InfoFree {
        rocblas_int *&p;
        ~InfoFree() {
            if (p) (void)hipFree(p);
        }
    } info_free{d_info};

    // x_l, and the basis functions at the sources, [nsrc] columns of [N]
    std::vector<double> hx(N), hphi(NS);
    for (int l = 1; l <= N; ++l) {
        hx[l - 1] = -std::pow(l * kPiM / (depth * k0), 2);
        for (int q = 0; q < nsrc; ++q)
            hphi[static_cast<size_t>(q) * N + (l - 1)] = std::sqrt(2.0 / depth) * std::sin(l * kPiM * zs[q] / depth);
    }
    MODAL_HIP(hipMemcpyAsync(x.p, hx.data(), N * sizeof(double), hipMemcpyHostToDevice, stream));
    MODAL_HIP(hipMemcpyAsync(dv.p, v.data(), N * sizeof(double), hipMemcpyHostToDevice, stream));
    MODAL_HIP(hipMemcpyAsync(phi.p, hphi.data(), NS * sizeof(double), hipMemcpyHostToDevice, stream));

    const dim3 blk(256), grid2((N + 255) / 256, N);
    hipLaunchKernelGGL(k_sine_matrix, grid2, blk, 0, stream, T.p, N);
    MODAL_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_scale_columns, grid2, blk, 0, stream, T.p, x.p, D.p, N);
    MODAL_HIP(hipGetLastError());

    Handle handle;
    if (rocblas_create_handle(&handle.h) != rocblas_status_success) {
        err = "rocblas_create_handle failed";
        return hipErrorUnknown;
    }
    rocblas_handle h = handle.h;
    MODAL_LIB(rocblas_set_stream(h, stream));
    const double one = 1.0, zero = 0.0;
    // X = (T diag(x)) T
    MODAL_LIB(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, N, N, N, &one, D.p, N,
                            T.p, N, &zero, X.p, N));
    hipLaunchKernelGGL(k_add_diagonal, dim3((N + 255) / 256), blk, 0, stream, X.p, dv.p, N);
    MODAL_HIP(hipGetLastError());
    // eigenvalues ascending, eigenvectors over X
    MODAL_LIB(rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, N, X.p, N, eig.p, off.p,
                               d_info));
    std::vector<double> lam(N);
    rocblas_int info = 0;
    MODAL_HIP(hipMemcpyAsync(lam.data(), eig.p, N * sizeof(double), hipMemcpyDeviceToHost, stream));
    MODAL_HIP(hipMemcpyAsync(&info, d_info, sizeof(info), hipMemcpyDeviceToHost, stream));
    MODAL_HIP(hipStreamSynchronize(stream));
    if (info != 0) {
        err = "the depth eigenproblem did not converge (dsyevd info " + std::to_string(info) + ")";
        return hipErrorUnknown;
    }
    // propagating modes: the largest eigenvalues with lambda > -1, at most max_modes
    int m = 0;
    while (m < N && lam[N - 1 - m] > -1.0 && (max_modes <= 0 || m < max_modes)) ++m;
    kappa.resize(m);
    for (int k = 0; k < m; ++k) kappa[k] = k0 * std::sqrt(1.0 + lam[N - 1 - k]);
    u.assign(NS, 0.0);
    if (m > 0) {
        const double *Y = X.p + static_cast<size_t>(N - m) * N;  // columns N-m .. N-1
        // sine coefficients of the selected modes, A = T Y (into D), and
        // Psi_m(zs_q) = (A^T Phi)[m][q]
        MODAL_LIB(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, N, m, N, &one, T.p, N,
                                Y, N, &zero, D.p, N));
        MODAL_LIB(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, m, nsrc, N, &one,
                                D.p, N, phi.p, N, &zero, psz.p, m));
        const size_t MS = static_cast<size_t>(m) * nsrc;
        std::vector<double> ps(MS), wt(MS);
        MODAL_HIP(hipMemcpyAsync(ps.data(), psz.p, MS * sizeof(double), hipMemcpyDeviceToHost, stream));
        MODAL_HIP(hipStreamSynchronize(stream));
        const double dz = depth / (N + 1);
        for (int q = 0; q < nsrc; ++q)
            for (int c = 0; c < m; ++c) {
                // column c of the block is mode m-1-c (ascending eigenvalues)
                const double kap = kappa[m - 1 - c];
                const size_t o = static_cast<size_t>(q) * m + c;
                wt[o] = std::sqrt(2.0 * kPiM) * ps[o] / (std::sqrt(dz) * std::sqrt(kap));
            }
        MODAL_HIP(hipMemcpyAsync(w.p, wt.data(), MS * sizeof(double), hipMemcpyHostToDevice, stream));
        // U = Y W: [N][nsrc]
        MODAL_LIB(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, N, nsrc, m, &one, Y, N,
                                w.p, m, &zero, ud.p, N));
        MODAL_HIP(hipMemcpyAsync(u.data(), ud.p, NS * sizeof(double), hipMemcpyDeviceToHost, stream));
        MODAL_HIP(hipStreamSynchronize(stream));
    }
    return hipSuccess;
#undef MODAL_HIP
#undef MODAL_LIB
}

}  // namespace ssp
