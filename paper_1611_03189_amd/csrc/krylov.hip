// Kernels of the batched outer loop (several right-hand sides advanced together, each with
// its own scalars): SpMV on a block of vectors, per-column dot products, and the masked
// vector updates of PCG. Column c of a block is at offset c * ld.
#include "hs_device.h"

namespace hs {

constexpr int SPMV_RC = 8;     // right-hand sides per SpMV pass

// Y(:, c) = A X(:, c) for the columns [c0, c0 + SPMV_RC) of blockIdx.y
__global__ __launch_bounds__(NT) void k_spmv_multi(const int64_t* row_ptr, const int32_t* col_idx,
                                                   const double* vals, const double* X, int64_t ldx,
                                                   double* Y, int64_t ldy, int n, int nrhs) {
    const int i = blockIdx.x * NT + threadIdx.x;
    const int c0 = blockIdx.y * SPMV_RC;
    if (i >= n) return;
    double acc[SPMV_RC];
#pragma unroll
    for (int c = 0; c < SPMV_RC; ++c) acc[c] = 0.0;
    for (int64_t t = row_ptr[i]; t < row_ptr[i + 1]; ++t) {
        const double v = vals[t];
        const double* xc = X + col_idx[t] + c0 * ldx;
#pragma unroll
        for (int c = 0; c < SPMV_RC; ++c)
            if (c0 + c < nrhs) acc[c] += v * xc[c * ldx];
    }
#pragma unroll
    for (int c = 0; c < SPMV_RC; ++c)
        if (c0 + c < nrhs) Y[i + (c0 + c) * ldy] = acc[c];
}

void launch_spmv_multi(const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
                       const double* X, int64_t ldx, double* Y, int64_t ldy, int n, int nrhs,
                       int64_t nnz, hipStream_t s) {
    ProfScope ps("k_spmv", (12.0 * nnz + 8.0 * (n + 1)) * ((nrhs + SPMV_RC - 1) / SPMV_RC) + 16.0 * n * nrhs, s);
    hipLaunchKernelGGL(k_spmv_multi, dim3((n + NT - 1) / NT, (nrhs + SPMV_RC - 1) / SPMV_RC), dim3(NT), 0, s,
                       row_ptr, col_idx, vals, X, ldx, Y, ldy, n, nrhs);
    check_launch("k_spmv_multi");
}

// out[c] = A(:, c) . B(:, c); partial sums of DOTM_BLOCKS-strided slices, then one block per
// column adds them in a fixed order (the result does not depend on the other columns)


__global__ __launch_bounds__(NT) void k_dots_part(const double* A, const double* B, int64_t ld, int n,
                                                  double* part) {
    __shared__ double red[NT / WAVE];
    const int c = blockIdx.y;
    const double* a = A + c * ld;
    const double* b = B + c * ld;
    double s0 = 0.0;
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) s0 += a[i] * b[i];
    s0 = block_sum(s0, red);
    if (threadIdx.x == 0) part[c * DOTM_BLOCKS + blockIdx.x] = s0;
}

__global__ __launch_bounds__(NT) void k_dots_final(const double* part, int nb, double* out) {
    __shared__ double red[NT / WAVE];
    const int c = blockIdx.x;
    double s0 = 0.0;
    for (int i = threadIdx.x; i < nb; i += NT) s0 += part[c * DOTM_BLOCKS + i];
    s0 = block_sum(s0, red);
    if (threadIdx.x == 0) out[c] = s0;
}

void launch_dots(const double* A, const double* B, int64_t ld, int n, int nrhs, double* part, double* out,
                 hipStream_t s) {
    int nb = (n + NT - 1) / NT;
    nb = nb < 1 ? 1 : (nb > DOTM_BLOCKS ? DOTM_BLOCKS : nb);
    hipLaunchKernelGGL(k_dots_part, dim3(nb, nrhs), dim3(NT), 0, s, A, B, ld, n, part);
    check_launch("k_dots_part");
    hipLaunchKernelGGL(k_dots_final, dim3(nrhs), dim3(NT), 0, s, part, nb, out);
    check_launch("k_dots_final");
}

// X(:, c) += a_c P(:, c), R(:, c) -= a_c Q(:, c) with a_c = num[c] / den[c], active columns only
__global__ void k_axpy2_multi(double* X, const double* P, double* R, const double* Q, int64_t ld, int n,
                              const double* num, const double* den, const int* active) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= n || !active[c]) return;
    const double a = num[c] / den[c];
    X[i + c * ld] += a * P[i + c * ld];
    R[i + c * ld] -= a * Q[i + c * ld];
}

void launch_axpy2_multi(double* X, const double* P, double* R, const double* Q, int64_t ld, int n, int nrhs,
                        const double* num, const double* den, const int* active, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy2_multi, dim3((n + NT - 1) / NT, nrhs), dim3(NT), 0, s, X, P, R, Q, ld, n, num,
                       den, active);
    check_launch("k_axpy2_multi");
}

// P(:, c) = Z(:, c) + beta_c P(:, c), active columns only, with beta_c = num[c] / den[c], or
// (num[c] - sub[c]) / den[c] when sub is given (the flexible form of beta)
__global__ void k_xpby_multi(double* P, const double* Z, int64_t ld, int n, const double* num,
                             const double* sub, const double* den, const int* active) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= n || !active[c]) return;
    const double beta = sub ? (num[c] - sub[c]) / den[c] : num[c] / den[c];
    P[i + c * ld] = Z[i + c * ld] + beta * P[i + c * ld];
}

void launch_xpby_multi(double* P, const double* Z, int64_t ld, int n, int nrhs, const double* num,
                       const double* sub, const double* den, const int* active, hipStream_t s) {
    hipLaunchKernelGGL(k_xpby_multi, dim3((n + NT - 1) / NT, nrhs), dim3(NT), 0, s, P, Z, ld, n, num, sub, den,
                       active);
    check_launch("k_xpby_multi");
}

// active[c] stays set while sqrt(rr[c]) > tol * nb[c]; dst[c] = src[c] for the active columns
__global__ void k_pcg_flags(const double* rr, const double* nb, double tol, int* active, double* dst,
                            const double* src, int nrhs) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nrhs) return;
    if (active[c] && !(sqrt(rr[c]) > tol * nb[c])) active[c] = 0;
    if (dst && active[c]) dst[c] = src[c];
}

void launch_pcg_flags(const double* rr, const double* nb, double tol, int* active, double* dst,
                      const double* src, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_flags, dim3((nrhs + NT - 1) / NT), dim3(NT), 0, s, rr, nb, tol, active, dst, src,
                       nrhs);
    check_launch("k_pcg_flags");
}

// dst[c] = src[c] (scalar copies on the device)
__global__ void k_copy_scalars(double* dst, const double* src, int n) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) dst[c] = src[c];
}

void launch_copy_scalars(double* dst, const double* src, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_scalars, dim3((n + NT - 1) / NT), dim3(NT), 0, s, dst, src, n);
    check_launch("k_copy_scalars");
}

// X(:, c) += Z(:, c), active columns only (stationary iteration)
__global__ void k_add_multi(double* X, const double* Z, int64_t ld, int n, const int* active) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i < n && active[c]) X[i + c * ld] += Z[i + c * ld];
}

void launch_add_multi(double* X, const double* Z, int64_t ld, int n, int nrhs, const int* active, hipStream_t s) {
    hipLaunchKernelGGL(k_add_multi, dim3((n + NT - 1) / NT, nrhs), dim3(NT), 0, s, X, Z, ld, n, active);
    check_launch("k_add_multi");
}

// R(:, c) = B(:, c) - Q(:, c), active columns only
__global__ void k_sub_multi(double* R, const double* B, int64_t ldb, const double* Q, int64_t ld, int n,
                            const int* active) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i < n && active[c]) R[i + c * ld] = B[i + c * ldb] - Q[i + c * ld];
}

void launch_sub_multi(double* R, const double* B, int64_t ldb, const double* Q, int64_t ld, int n, int nrhs,
                      const int* active, hipStream_t s) {
    hipLaunchKernelGGL(k_sub_multi, dim3((n + NT - 1) / NT, nrhs), dim3(NT), 0, s, R, B, ldb, Q, ld, n, active);
    check_launch("k_sub_multi");
}

// ---------------------------------------------------------------------------------
// Restarted GMRES (one column): Arnoldi vector updates with coefficients on the device
// ---------------------------------------------------------------------------------
// y += sign * (*a) * x
__global__ void k_axpy_dev(double* y, const double* x, const double* a, double sign, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += (sign * a[0]) * x[i];
}

void launch_axpy_dev(double* y, const double* x, const double* a, double sign, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy_dev, dim3((n + NT - 1) / NT), dim3(NT), 0, s, y, x, a, sign, n);
    check_launch("k_axpy_dev");
}

// y = sc * x
__global__ void k_scale(double* y, const double* x, double sc, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = sc * x[i];
}

void launch_scale(double* y, const double* x, double sc, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale, dim3((n + NT - 1) / NT), dim3(NT), 0, s, y, x, sc, n);
    check_launch("k_scale");
}

// r = b - w
__global__ void k_sub(double* r, const double* b, const double* w, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) r[i] = b[i] - w[i];
}

void launch_sub(double* r, const double* b, const double* w, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_sub, dim3((n + NT - 1) / NT), dim3(NT), 0, s, r, b, w, n);
    check_launch("k_sub");
}

// x += Z y, Z: n x k (ld ldz), y: k entries on the device; the terms are added in column order
__global__ void k_gemv_acc(double* x, const double* Z, int64_t ldz, const double* y, int k, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int j = 0; j < k; ++j) acc += Z[i + j * ldz] * y[j];
    x[i] += acc;
}

void launch_gemv_acc(double* x, const double* Z, int64_t ldz, const double* y, int k, int n, hipStream_t s) {
    if (k <= 0) return;
    hipLaunchKernelGGL(k_gemv_acc, dim3((n + NT - 1) / NT), dim3(NT), 0, s, x, Z, ldz, y, k, n);
    check_launch("k_gemv_acc");
}

}  // namespace hs
