// Pivot blocks: Cholesky A = L L^T and the explicit inverse A^{-1} = L^{-T} L^{-1}, one
// workgroup per block. Used for A_ss^{-1} and S^{-1} (§3.2 elimination; Appendix A).
//
// Blocks up to PIV_LDS_MAX rows are factored in LDS with leading dimension m+1 (odd
// stride: the column walks of the inverse and of the product hit distinct banks);
// larger blocks use a global work matrix. Steps, all threads cooperating:
//   right-looking Cholesky (column scale + rank-1 trailing update per step),
//   in-place lower-triangular inverse (column j = -(L22^{-1} l_j) / l_jj, right to left),
//   A^{-1}(i,j) = sum_{k >= max(i,j)} X(k,i) X(k,j) with X = L^{-1}, both triangles written.
#include "hs_device.h"

namespace hs {

constexpr int PIV_LDS_MAX = 128;
constexpr int PIV_MAX = 1024;          // rows per thread <= PIV_MAX / NT in the inverse

template <bool LDS>
__global__ __launch_bounds__(NT) void k_chol_inv(const CholTask* tasks, int* fail) {
    extern __shared__ double lds[];
    __shared__ int bad;
    const CholTask T = tasks[blockIdx.x];
    const int m = T.m, tid = threadIdx.x;
    double* W = LDS ? lds : T.work;
    const int ldw = LDS ? m + 1 : m;
    for (int e = tid; e < m * m; e += NT) {
        const int i = e % m, j = e / m;
        W[i + j * ldw] = T.A[i + size_t(j) * T.lda];
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < m; ++j) {
        if (tid == 0) {
            const double d = W[j + j * ldw];
            if (!(d > 0.0) || !isfinite(d)) bad = 1;
            else W[j + j * ldw] = sqrt(d);
        }
        __syncthreads();
        if (bad) break;
        const double piv = W[j + j * ldw];
        for (int i = j + 1 + tid; i < m; i += NT) W[i + j * ldw] /= piv;
        __syncthreads();
        // trailing update, rows over threads (the column-j entry of a row stays in a register)
        for (int i = j + 1 + tid; i < m; i += NT) {
            const double lij = W[i + j * ldw];
            int k = j + 1;
            for (; k + 4 <= i + 1; k += 4) {
                double t[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) t[u] = W[(k + u) + j * ldw];
#pragma unroll
                for (int u = 0; u < 4; ++u) W[i + (k + u) * ldw] -= lij * t[u];
            }
            for (; k <= i; ++k) W[i + k * ldw] -= lij * W[k + j * ldw];
        }
        __syncthreads();
    }
    if (bad) {
        if (tid == 0) fail[T.id] = 1;
        return;
    }
    // X = L^{-1} in place, columns right to left
    for (int j = m - 1; j >= 0; --j) {
        if (tid == 0) W[j + j * ldw] = 1.0 / W[j + j * ldw];
        __syncthreads();
        const double ajj = -W[j + j * ldw];
        double y[PIV_MAX / NT];
        int cnt = 0;
        for (int i = j + 1 + tid; i < m; i += NT) {
            double a[4] = {0, 0, 0, 0};
            int l = j + 1;
            for (; l + 4 <= i + 1; l += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) a[u] += W[i + (l + u) * ldw] * W[(l + u) + j * ldw];
            }
            for (; l <= i; ++l) a[0] += W[i + l * ldw] * W[l + j * ldw];
            y[cnt++] = (a[0] + a[1]) + (a[2] + a[3]);
        }
        __syncthreads();
        cnt = 0;
        for (int i = j + 1 + tid; i < m; i += NT) W[i + j * ldw] = ajj * y[cnt++];
        __syncthreads();
    }
    if (!LDS) {
        // large block: X = L^{-1} stays in the work matrix (upper part zeroed); the caller
        // forms A^{-1} = X^T X with the grouped GEMM over many workgroups
        for (int e = tid; e < m * m; e += NT) {
            const int i = e % m, j = e / m;
            if (i < j) W[i + j * ldw] = 0.0;
        }
        return;
    }
    // A^{-1} = X^T X
    for (int e = tid; e < m * m; e += NT) {
        const int i = e % m, j = e / m;
        if (i < j) continue;
        double s = 0.0;
        for (int k = i; k < m; ++k) s += W[k + i * ldw] * W[k + j * ldw];
        T.Ainv[i + size_t(j) * T.ldi] = s;
        T.Ainv[j + size_t(i) * T.ldi] = s;
    }
}

void launch_chol_inv(const CholTask* d_tasks, int ntasks, int* d_fail, double flops, bool lds,
                     int max_m, hipStream_t s) {
    if (ntasks <= 0) return;
    if (max_m > PIV_MAX) throw Error{HSOLVE_ERR_INVALID, "pivot block larger than 1024"};
    ProfScope ps("k_chol_inv", flops, s);
    if (lds) {
        if (max_m > PIV_LDS_MAX) throw Error{HSOLVE_ERR_INVALID, "internal: LDS pivot too large"};
        const size_t bytes = size_t(max_m) * (max_m + 1) * sizeof(double);
        static bool attr = false;
        if (!attr) {
            HS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_chol_inv<true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       int(size_t(PIV_LDS_MAX) * (PIV_LDS_MAX + 1) * sizeof(double))));
            attr = true;
        }
        hipLaunchKernelGGL(k_chol_inv<true>, dim3(ntasks), dim3(NT), bytes, s, d_tasks, d_fail);
        check_launch("k_chol_inv<lds>");
    } else {
        hipLaunchKernelGGL(k_chol_inv<false>, dim3(ntasks), dim3(NT), 0, s, d_tasks, d_fail);
        check_launch("k_chol_inv<global>");
    }
}

}  // namespace hs
