// Pivot blocks: Cholesky A = L L^T and the explicit inverse A^{-1} = L^{-T} L^{-1}, one
// workgroup per block. Used for A_ss^{-1} and S^{-1} (§3.2 elimination; Appendix A).
//
// k_chol_inv     blocks up to PIV_LDS_MAX rows, held in LDS with leading dimension m+1
//                (odd stride: the column walks of the inverse and of the product hit
//                distinct banks): right-looking Cholesky, in-place lower-triangular
//                inverse X = L^{-1} (column j = -(X22 l_j) / l_jj, right to left), then
//                A^{-1} = X^T X written to both triangles.
// k_chol_inv_blk larger blocks (up to PIV_MAX rows) in a global work matrix, blocked by
//                PIV_NB columns: the current panel is factored in LDS, the trailing
//                matrix is updated with 4x4 register tiles; the inverse is blocked the
//                same way (X21 = -X22 L21 X11, right to left). X = L^{-1} is left in the
//                work matrix (upper triangle zeroed) for the product A^{-1} = X^T X, which
//                the caller forms with the grouped GEMM over many workgroups.
#include "hs_device.h"

namespace hs {

constexpr int PIV_LDS_MAX = 128;
constexpr int PIV_MAX = 512;
constexpr int PIV_NB = 32;
constexpr int PIV_PANEL = PIV_MAX * PIV_NB;     // doubles of the LDS panel buffer

__global__ __launch_bounds__(NT) void k_chol_inv(const CholTask* tasks, int* fail) {
    extern __shared__ double lds[];
    __shared__ int bad;
    const CholTask T = tasks[blockIdx.x];
    const int m = T.m, tid = threadIdx.x;
    double* W = lds;
    const int ldw = m + 1;
    const HS_G double* A = gp(T.A);
    HS_G double* Ainv = gp(T.Ainv);
    for (int e = tid; e < m * m; e += NT) {
        const int i = e % m, j = e / m;
        W[i + j * ldw] = A[i + size_t(j) * T.lda];
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
        double y = 0.0;
        const int i = j + 1 + tid;         // m <= PIV_LDS_MAX < NT: at most one row per thread
        if (i < m) {
            double a[4] = {0, 0, 0, 0};
            int l = j + 1;
            for (; l + 4 <= i + 1; l += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) a[u] += W[i + (l + u) * ldw] * W[(l + u) + j * ldw];
            }
            for (; l <= i; ++l) a[0] += W[i + l * ldw] * W[l + j * ldw];
            y = (a[0] + a[1]) + (a[2] + a[3]);
        }
        __syncthreads();
        if (i < m) W[i + j * ldw] = ajj * y;
        __syncthreads();
    }
    // A^{-1} = X^T X
    for (int e = tid; e < m * m; e += NT) {
        const int i = e % m, j = e / m;
        if (i < j) continue;
        double s = 0.0;
        for (int k = i; k < m; ++k) s += W[k + i * ldw] * W[k + j * ldw];
        Ainv[i + size_t(j) * T.ldi] = s;
        Ainv[j + size_t(i) * T.ldi] = s;
    }
}

// advance (I, J) by `step` positions in the column-major order of the lower tiles of a
// T x T tile grid (column J holds rows J..T-1); J == T marks the end
__device__ inline void next_lower_tile(int& I, int& J, int step, int T) {
    I += step;
    while (J < T && I >= T) {
        I -= T - (J + 1);
        ++J;
    }
}

__global__ __launch_bounds__(NT) void k_chol_inv_blk(const CholTask* tasks, int* fail) {
    extern __shared__ double Pn[];                  // panel / Y buffer, PIV_PANEL doubles
    __shared__ double X11[PIV_NB * (PIV_NB + 1)];
    __shared__ double yv[PIV_NB];
    __shared__ int bad;
    const CholTask T = tasks[blockIdx.x];
    const int m = T.m, tid = threadIdx.x;
    HS_G double* W = gp(T.work);                   // m x m, ld m
    const HS_G double* A = gp(T.A);
    const size_t ld = size_t(m);
    for (size_t e = tid; e < ld * m; e += NT) {
        const size_t i = e % ld, j = e / ld;
        W[e] = A[i + j * T.lda];
    }
    if (tid == 0) bad = 0;
    __syncthreads();

    // ---- blocked right-looking Cholesky ----
    for (int jb = 0; jb < m; jb += PIV_NB) {
        const int nb = min(PIV_NB, m - jb);
        const int r = m - jb;                        // panel rows (diagonal block first)
        for (int e = tid; e < r * nb; e += NT) {
            const int i = e % r, c = e / r;
            Pn[i + c * r] = W[(jb + i) + (jb + c) * ld];
        }
        __syncthreads();
        for (int j = 0; j < nb; ++j) {
            if (tid == 0) {
                const double d = Pn[j + j * r];
                if (!(d > 0.0) || !isfinite(d)) bad = 1;
                else Pn[j + j * r] = sqrt(d);
            }
            __syncthreads();
            if (bad) break;
            const double piv = Pn[j + j * r];
            for (int i = j + 1 + tid; i < r; i += NT) Pn[i + j * r] /= piv;
            __syncthreads();
            for (int i = j + 1 + tid; i < r; i += NT) {
                const double lij = Pn[i + j * r];
                const int cend = min(i, nb - 1);
                for (int c = j + 1; c <= cend; ++c) Pn[i + c * r] -= lij * Pn[c + j * r];
            }
            __syncthreads();
        }
        if (bad) break;
        for (int e = tid; e < r * nb; e += NT) {
            const int i = e % r, c = e / r;
            W[(jb + i) + (jb + c) * ld] = Pn[i + c * r];
        }
        // trailing update W22 -= L21 L21^T on the lower 4x4 tiles, L21 = Pn(nb.., :)
        const int t = r - nb;
        const int Tt = (t + 3) / 4;
        int I = tid, J = 0;
        next_lower_tile(I, J, 0, Tt);
        for (; J < Tt; next_lower_tile(I, J, NT, Tt)) {
            const int pi = nb + 4 * I, pj = nb + 4 * J;      // panel rows of the tile
            double acc[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    acc[u][v] = (pi + u < r && pj + v < r) ? W[(jb + pi + u) + (jb + pj + v) * ld] : 0.0;
#pragma unroll 2
            for (int k = 0; k < nb; ++k) {
                double a[4], b[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a[u] = (pi + u < r) ? Pn[pi + u + k * r] : 0.0;
                    b[u] = (pj + u < r) ? Pn[pj + u + k * r] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[u][v] -= a[u] * b[v];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (pi + u < r && pj + v < r) W[(jb + pi + u) + (jb + pj + v) * ld] = acc[u][v];
        }
        __syncthreads();
    }
    if (bad) {
        if (tid == 0) fail[T.id] = 1;
        return;
    }

    // ---- blocked inverse X = L^{-1}, panels right to left ----
    const int last = ((m - 1) / PIV_NB) * PIV_NB;
    for (int jb = last; jb >= 0; jb -= PIV_NB) {
        const int nb = min(PIV_NB, m - jb);
        const int t = m - jb - nb;
        const int l11 = PIV_NB + 1;
        for (int e = tid; e < nb * nb; e += NT) {
            const int i = e % nb, c = e / nb;
            X11[i + c * l11] = W[(jb + i) + (jb + c) * ld];
        }
        __syncthreads();
        // X11 = L11^{-1} in place, columns right to left
        for (int j = nb - 1; j >= 0; --j) {
            if (tid == 0) X11[j + j * l11] = 1.0 / X11[j + j * l11];
            __syncthreads();
            const int i = j + 1 + tid;
            if (i < nb) {
                double s = 0.0;
                for (int l = j + 1; l <= i; ++l) s += X11[i + l * l11] * X11[l + j * l11];
                yv[i] = -X11[j + j * l11] * s;
            }
            __syncthreads();
            if (i < nb) X11[i + j * l11] = yv[i];
            __syncthreads();
        }
        for (int e = tid; e < nb * nb; e += NT) {
            const int i = e % nb, c = e / nb;
            if (i >= c) W[(jb + i) + (jb + c) * ld] = X11[i + c * l11];
        }
        if (t > 0) {
            // Y = L21 X11 (t x nb) into LDS; items of one row and 4 columns
            for (int idx = tid; idx < t * (PIV_NB / 4); idx += NT) {
                const int i = idx % t, c0 = 4 * (idx / t);
                if (c0 >= nb) continue;
                double acc[4] = {0.0, 0.0, 0.0, 0.0};
                for (int l = c0; l < nb; ++l) {
                    const double rl = W[(jb + nb + i) + (jb + l) * ld];
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (c0 + v <= l) acc[v] += rl * X11[l + (c0 + v) * l11];
                }
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (c0 + v < nb) Pn[i + (c0 + v) * t] = acc[v];
            }
            __syncthreads();
            // X21 = -X22 Y, X22 = the lower-triangular inverse already in W; tiles of 4 rows x 8 cols
            const int Tr = (t + 3) / 4, Tc = (nb + 7) / 8;
            for (int idx = tid; idx < Tr * Tc; idx += NT) {
                const int i0 = 4 * (idx % Tr), c0 = 8 * (idx / Tr);
                double acc[4][8];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 8; ++v) acc[u][v] = 0.0;
                const HS_G double* X22 = W + (jb + nb) + (jb + nb) * ld;
                // columns l <= i0: every row of the tile takes part (rows beyond t read 0)
#pragma unroll 1
                for (int l = 0; l <= i0 && l < t; ++l) {
                    double x[4], y[8];
#pragma unroll
                    for (int u = 0; u < 4; ++u) x[u] = (i0 + u < t) ? X22[(i0 + u) + l * ld] : 0.0;
#pragma unroll
                    for (int v = 0; v < 8; ++v) y[v] = (c0 + v < nb) ? Pn[l + (c0 + v) * t] : 0.0;
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int v = 0; v < 8; ++v) acc[u][v] += x[u] * y[v];
                }
                // columns i0 < l <= i0 + 3: only rows u with l <= i0 + u
#pragma unroll 1
                for (int l = i0 + 1; l <= i0 + 3 && l < t; ++l) {
                    double x[4], y[8];
#pragma unroll
                    for (int u = 0; u < 4; ++u) x[u] = (i0 + u < t && l <= i0 + u) ? X22[(i0 + u) + l * ld] : 0.0;
#pragma unroll
                    for (int v = 0; v < 8; ++v) y[v] = (c0 + v < nb) ? Pn[l + (c0 + v) * t] : 0.0;
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int v = 0; v < 8; ++v) acc[u][v] += x[u] * y[v];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 8; ++v)
                        if (i0 + u < t && c0 + v < nb) W[(jb + nb + i0 + u) + (jb + c0 + v) * ld] = -acc[u][v];
            }
        }
        __syncthreads();
    }
    // upper triangle of X is zero for the product X^T X
    for (size_t e = tid; e < ld * m; e += NT) {
        const size_t i = e % ld, j = e / ld;
        if (i < j) W[e] = 0.0;
    }
}

void launch_chol_inv(const CholTask* d_tasks, int ntasks, int* d_fail, double flops, bool lds,
                     int max_m, hipStream_t s) {
    if (ntasks <= 0) return;
    if (max_m > PIV_MAX) throw Error{HSOLVE_ERR_INVALID, "pivot block larger than 512"};
    ProfScope ps(lds ? "k_chol_inv" : "k_chol_inv_blk", flops, s);
    if (lds) {
        if (max_m > PIV_LDS_MAX) throw Error{HSOLVE_ERR_INVALID, "internal: LDS pivot too large"};
        const size_t bytes = size_t(max_m) * (max_m + 1) * sizeof(double);
        static bool attr = false;
        if (!attr) {
            HS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_chol_inv),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       int(size_t(PIV_LDS_MAX) * (PIV_LDS_MAX + 1) * sizeof(double))));
            attr = true;
        }
        hipLaunchKernelGGL(k_chol_inv, dim3(ntasks), dim3(NT), bytes, s, d_tasks, d_fail);
        check_launch("k_chol_inv");
    } else {
        const size_t bytes = size_t(PIV_PANEL) * sizeof(double);
        static bool attr = false;
        if (!attr) {
            HS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_chol_inv_blk),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
            attr = true;
        }
        hipLaunchKernelGGL(k_chol_inv_blk, dim3(ntasks), dim3(NT), bytes, s, d_tasks, d_fail);
        check_launch("k_chol_inv_blk");
    }
}

}  // namespace hs
