// KL basis of the isotropic Matern field by the Nystrom method (Section 5:
// eq. matern, the collocation of the covariance eigenproblem, its symmetric
// reformulation and the Nystrom interpolation formula), built once per
// context on the device:
//   1. B = W^1/2 Sigma W^1/2 on the Q x Q midpoint nodes (w = 1/Q^2),
//   2. its eigenpairs by rocSOLVER's symmetric divide-and-conquer solver,
//   3. G^T[m][q] = sigma sqrt(w) Psi*_{m,q} / sqrt(theta_m) for the s largest,
//   4. basis[m][c] = sum_q G^T[m][q] C(x_c, x_q) at every cell centre of every
//      level: the covariance block of a chunk of cells is formed on the fly
//      and multiplied on the FP64 matrix cores by the field product kernel.
#include "internal.hpp"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>

namespace mlmc {
namespace {

struct MaternParams {
    double nu;       // smoothness
    double inv_lam;  // 1 / lambda_c
    double sq2nu;    // sqrt(2 nu)
    double norm;     // 2^(1-nu) / Gamma(nu)
};

// eq. matern at distance r.  With x = sqrt(2 nu) r / lambda_c,
// x^nu K_nu(x) = int_0^inf exp(nu (ln x + t) - x cosh t) (1 + e^(-2 nu t)) / 2 dt
// (the integral representation of K_nu times x^nu, written so that no factor
// overflows for small x), by the trapezoidal rule with step 1/8: the integrand
// is analytic in the strip |Im t| < pi/2 and decays double exponentially, so
// the rule's error is of order exp(-pi^2 / h) = e^-79, and every term is
// positive.  nu = 1/2 is the exponential itself.
__device__ double matern_cov(double r, const MaternParams &p)
{
    if (r == 0.0) return 1.0;
    if (p.nu == 0.5) return exp(-r * p.inv_lam);
    const double x = p.sq2nu * r * p.inv_lam;
    const double lx = log(x);
    constexpr double h = 0.125;
    double sum = 0.5 * exp(p.nu * lx - x);                 // t = 0, half weight
    for (int k = 1; k < 16384; ++k) {
        const double t = h * k;
        const double term = exp(p.nu * (lx + t) - x * cosh(t)) * 0.5 * (1.0 + exp(-2.0 * p.nu * t));
        sum += term;
        if (term <= 1e-18 * sum && x * sinh(t) > p.nu) break;   // past the peak, negligible
    }
    return p.norm * h * sum;
}

__device__ __forceinline__ void node_xy(int64_t q, int Q, double &x, double &y)
{
    x = ((double)(q % Q) + 0.5) / Q;
    y = ((double)(q / Q) + 0.5) / Q;
}

// B[k + n q] = w C(|x_k - x_q|), n = Q^2 (symmetric: the same in either order)
__global__ void k_nystrom_matrix(int Q, double w, MaternParams p, double *__restrict__ B)
{
    const int64_t n = (int64_t)Q * Q;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n * n) return;
    const int64_t k = id % n, q = id / n;
    double xk, yk, xq, yq;
    node_xy(k, Q, xk, yk);
    node_xy(q, Q, xq, yq);
    const double dx = xk - xq, dy = yk - yq;
    B[id] = w * matern_cov(sqrt(dx * dx + dy * dy), p);
}

// GT[m][q] = c Psi*_{j,q} / sqrt(theta_j) for j = n - 1 - m (eigenvalues come
// ascending, eigenvector j in column j of V)
__global__ void k_nystrom_gt(const double *__restrict__ V, const double *__restrict__ D, int64_t n,
                             int s, double c, double *__restrict__ GT)
{
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)s * n) return;
    const int64_t m = id / n, q = id % n, j = n - 1 - m;
    GT[id] = c * V[q + j * n] / sqrt(D[j]);
}

// Ct[q][c] = C(|x_q - x_{c0+c}|) for the mc cells c0 .. c0+mc-1 of the
// level-major hierarchy (cell p = i + n_g j of level g at ((i+1/2)/n_g, (j+1/2)/n_g))
__global__ void k_nystrom_cells(int Q, MaternParams p, int64_t c0, int64_t mc,
                                double *__restrict__ Ct)
{
    const int64_t n = (int64_t)Q * Q;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n * mc) return;
    const int64_t q = id / mc, cell = c0 + id % mc;
    int g = 0;
    while (g < kMaxMgLevels - 1 && level_offset(g + 1) <= cell) ++g;
    const int64_t pc = cell - level_offset(g);
    const int ng = 2 << g;
    const double xc = ((double)(pc % ng) + 0.5) / ng, yc = ((double)(pc / ng) + 0.5) / ng;
    double xq, yq;
    node_xy(q, Q, xq, yq);
    const double dx = xc - xq, dy = yc - yq;
    Ct[id] = matern_cov(sqrt(dx * dx + dy * dy), p);
}

unsigned grid_of(int64_t n) { return (unsigned)((n + 255) / 256); }

struct DevBuf {
    double *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

std::string matern_basis(int Q, double nu, double lam, double sigma, int s, int G, double *basis,
                         int64_t ld, std::vector<double> &theta)
{
    const int64_t n = (int64_t)Q * Q;
    const double w = 1.0 / (double)n;
    const MaternParams p{nu, 1.0 / lam, std::sqrt(2.0 * nu), std::pow(2.0, 1.0 - nu) / std::tgamma(nu)};
    auto hip_err = [](const char *what, hipError_t e) {
        return std::string(what) + ": " + hipGetErrorString(e);
    };
    DevBuf B, D, E, GT, Ct, tmp;
    int *info = nullptr;
    hipError_t e = hipMalloc((void **)&B.p, sizeof(double) * n * n);
    if (e == hipSuccess) e = hipMalloc((void **)&D.p, sizeof(double) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&E.p, sizeof(double) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&info, sizeof(int));
    if (e != hipSuccess) {
        if (info) (void)hipFree(info);
        return hip_err("Nystrom matrix allocation", e);
    }
    hipLaunchKernelGGL(k_nystrom_matrix, dim3(grid_of(n * n)), dim3(256), 0, nullptr, Q, w, p, B.p);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(info);
        return hip_err("Nystrom matrix", e);
    }
    rocblas_handle handle = nullptr;
    if (rocblas_create_handle(&handle) != rocblas_status_success) {
        (void)hipFree(info);
        return "rocblas_create_handle failed";
    }
    const rocblas_status rs = rocsolver_dsyevd(handle, rocblas_evect_original, rocblas_fill_upper,
                                               (rocblas_int)n, B.p, (rocblas_int)n, D.p, E.p, info);
    e = hipDeviceSynchronize();
    (void)rocblas_destroy_handle(handle);
    int hinfo = -1;
    if (e == hipSuccess) e = hipMemcpy(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost);
    (void)hipFree(info);
    if (e != hipSuccess) return hip_err("Nystrom eigensolve", e);
    if (rs != rocblas_status_success || hinfo != 0) return "Nystrom eigensolve did not converge";
    std::vector<double> Dh(n);
    e = hipMemcpy(Dh.data(), D.p, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_err("Nystrom eigenvalues", e);
    theta.resize(s);
    for (int m = 0; m < s; ++m) {
        theta[m] = Dh[n - 1 - m];
        if (!(theta[m] > 0.0)) return "s exceeds the positive Nystrom eigenvalues: raise nystrom_q";
    }
    e = hipMalloc((void **)&GT.p, sizeof(double) * s * n);
    if (e != hipSuccess) return hip_err("Nystrom allocation", e);
    hipLaunchKernelGGL(k_nystrom_gt, dim3(grid_of((int64_t)s * n)), dim3(256), 0, nullptr, B.p, D.p,
                       n, s, sigma * std::sqrt(w), GT.p);
    // covariance blocks of up to 2^27 entries (1 GiB), 128-cell aligned
    const int64_t M = level_offset(G + 1);
    const int64_t mc = std::max<int64_t>(128, ((int64_t)1 << 27) / n / 128 * 128);
    e = hipMalloc((void **)&Ct.p, sizeof(double) * n * std::min(mc, M));
    if (e == hipSuccess) e = hipMalloc((void **)&tmp.p, sizeof(double) * s * std::min(mc, M));
    if (e != hipSuccess) return hip_err("Nystrom allocation", e);
    for (int64_t c0 = 0; c0 < M; c0 += mc) {
        const int64_t cnt = std::min(mc, M - c0);
        hipLaunchKernelGGL(k_nystrom_cells, dim3(grid_of(n * cnt)), dim3(256), 0, nullptr, Q, p, c0,
                           cnt, Ct.p);
        // tmp[m][c] = sum_q GT[m][q] Ct[q][c]: the field product with K = n
        launch_field_gemm(nullptr, GT.p, (int)n, Ct.p, cnt, cnt, s, tmp.p, 0);
        e = hipMemcpy2DAsync(basis + c0, sizeof(double) * ld, tmp.p, sizeof(double) * cnt,
                             sizeof(double) * cnt, s, hipMemcpyDeviceToDevice, nullptr);
        if (e != hipSuccess) return hip_err("Nystrom basis copy", e);
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_err("Nystrom basis", e);
    return std::string();
}

}  // namespace mlmc
